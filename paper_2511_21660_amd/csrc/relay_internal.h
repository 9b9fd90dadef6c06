// relay_internal.h -- declarations shared by the host ABI (relay_api.cpp) and
// the gfx950 kernels (relay_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rb {

// Shape of one kernel configuration ("tile"): G lanes of a wave cooperate on
// one syndrome; lane g owns checks i = g + G*c (c < CPT) and faults
// j = g + G*v (v < VPT); DC and DV bound the row and column degrees.
struct TileShape {
    int G, CPT, DC, VPT, DV;
    int waves;  // waves per SIMD the kernel's register budget targets
};

// Arguments of the group kernel (passed by value).
struct CodeStatic;

// Work queues of the group kernels: kQueueSplit counters, kQueueStride
// unsigned long longs (256 bytes) apart; slot s claims positions
// s % kQueueSplit + kQueueSplit * n from counter s % kQueueSplit, which spreads
// the claims of thousands of slots over many addresses: device-scope atomics
// on one address serialise (with 8 counters the claims alone took ~1 ms per
// 4 x 10^5 syndromes; 64 counters cut that 4-fold, more gain little).  The
// block kernel uses counter 0 alone.  A queue occupies kQueueWords words.
constexpr int kQueueSplit = 64;
// Floats of zero padding after a code's w [N] and memory-strength table
// [R][N]: a group-kernel lane reads entries gl + G*v (v < VPT) of a row
// without clamping to N - 1, so reads past the last row stay in bounds
// (G * VPT <= kGroupReadPad for every tile); lanes past N never use them.
constexpr int kGroupReadPad = 512;
constexpr int kQueueStride = 32;
constexpr int kQueueWords = kQueueSplit * kQueueStride;

// a ^ b ^ c as one three-input logic op (the compiler emits two-input XORs
// for a chain of them)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Bit-packed I/O (RB_IO_BITS32): syndromes and corrections as uint32 words,
// entry k in bit k % 32 of word k / 32.  The kernels read a syndrome bit
// with syn_bit and the strides below count elements of the layout in use
// (bytes, or words when io_bits is set).
__device__ __forceinline__ bool syn_bit(const void *syn, size_t row, int32_t stride, int i, bool bits) {
    if (bits) return (static_cast<const uint32_t *>(syn)[row * stride + (i >> 5)] >> (i & 31)) & 1u;
    return static_cast<const uint8_t *>(syn)[row * stride + i] != 0;
}

struct GroupArgs {
    int32_t M, N;
    int32_t syn_stride, corr_stride;  // elements (bytes or words) per syndrome / correction row
    int32_t llr_stride;               // floats per marginal row
    int32_t io_bits;                  // 1: bit-packed syndromes and corrections
    int64_t B;
    int64_t count;        // queue positions to decode
    const int32_t *list;  // [count] shot of queue position k, or null (shot = k)
    const uint8_t *syn;   // [B][syn_stride]
    uint8_t *corr;        // [B][corr_stride]
    uint8_t *conv;        // [B]
    int32_t *legs;        // [B]
    int32_t *iters;       // [B]
    double *weight;       // [B] or null
    float *final_llr;     // [B][N] or null
    const float *w;       // [N] channel LLRs
    const float *gamma;   // [R][N] memory strengths, row r-1 = leg r
    int32_t w_uniform;    // 1: every w_j of the code (of every family member) is equal
    float w0;             // w_0 of the code (of member 0)
    // codes sharing one graph (mixed launch): when list_cid is set, queue
    // position k belongs to family member list_cid[k], whose w and gamma
    // follow member 0's at w + list_cid[k] * N and gamma + list_cid[k] * R * N
    const int32_t *list_cid;
    // per-lane gather tables, two 16-bit slot-relative LDS byte offsets per
    // word: lane g's entries e = c*DC + k (Lambda of check edge) and
    // e = v*DV + k (mu of fault edge) at word g*ceil(n/2) + e/2, half e%2
    const uint32_t *lam_off;  // [G][ceil(CPT*DC/2)]
    const uint32_t *mu_off;   // [G][ceil(VPT*DV/2)]
    unsigned long long *queue;  // work queue (kQueueWords counters, see below)
    int32_t num_legs, iters_first, iters_leg, num_solutions, max_total_iters;
    float L;
    // LDS byte offsets within a slot's region (slot word w -> byte 4 * SPH * w
    // with SPH = max(1, 32 / G) slots per half-wave; the kernel adds the slot
    // base 4 * (slot % SPH) + half_off * (slot / SPH))
    uint32_t lampad_off;   // +inf cell: Lambda of padded check edges
    uint32_t mupad_off;    // -0 cell: mu of padded fault edges
    uint32_t mu0_off;      // start of the check-message rows
    uint32_t half_off;     // bytes between the regions of the two half-waves
    // trace mode (rb_trace): per-column gamma, LLR scale, iteration count, output
    const float *trace_gamma;
    float scale;
    int32_t trace_T;
    float *trace;          // [B][T+1][N]
};

// Shape of a block-kernel configuration: TPB threads decode one syndrome;
// thread t owns one check (degree <= DCMAX) and faults t + TPB*v, v < VPT
// (degree <= DV).
//
// Faults are assigned to slots s = t + TPB*v in the order of decreasing
// column degree, so band v (slots TPB*v .. TPB*(v+1)-1) holds faults of
// nearly equal degree; `prof` caps the degree of each band (4 bits per band,
// band 0 in the low bits) and sizes the thread's fault-side gather table.
struct BlockShape {
    int TPB, DCMAX, VPT;
    uint64_t prof;
    int waves;
};

__host__ __device__ constexpr int prof_dv(uint64_t prof, int v) { return (int)((prof >> (4 * v)) & 15u); }

// gather-table entries of bands 0 .. v-1
__host__ __device__ constexpr int prof_pre(uint64_t prof, int v) {
    int s = 0;
    for (int u = 0; u < v; ++u) s += prof_dv(prof, u);
    return s;
}

__host__ __device__ constexpr int prof_max(uint64_t prof, int vpt) {
    int m = 0;
    for (int u = 0; u < vpt; ++u) m = prof_dv(prof, u) > m ? prof_dv(prof, u) : m;
    return m;
}

// The block kernel reads check rows in chunks of this many edges; reads past
// a wave's last row land in the next wave's rows or in the zeroed slack words
// after the message region ((kBlockChunk - 1) rows of 64 words).
constexpr int kBlockChunk = 8;

struct BlockArgs {
    int32_t M, N;
    int32_t syn_stride, corr_stride;  // elements (bytes or words) per syndrome / correction row
    int32_t io_bits;                  // 1: bit-packed syndromes and corrections
    int64_t B;
    const uint8_t *syn;
    uint8_t *corr;
    uint8_t *conv;
    int32_t *legs;
    int32_t *iters;
    double *weight;
    float *final_llr;
    const float *w;
    const float *gamma;
    const uint32_t *chk_col;   // [DCMAX/8 + 1][TPB][4] 16-bit Lambda byte addresses, 8 per chunk (last: padding)
    const uint32_t *col_mu;    // [ceil(prof_pre(VPT)/2)][TPB] two 16-bit message word indices
    const int32_t *slot_col;   // [TPB*VPT] fault held by slot s, or -1 (slots >= N)
    const float *w_slot;       // [TPB*VPT] channel LLR by slot (0 for spare slots)
    const float *gamma_slot;   // [R][TPB*VPT] memory strengths by slot
    const int32_t *chk_row;    // [TPB] check whose syndrome bit thread t adds, or -1
    const int32_t *chk_split;  // [TPB] 1: thread t holds part of a check shared with thread t ^ 1
    const int32_t *wave_deg;   // [TPB/64] row length (max degree) of wave w
    const int32_t *wave_base;  // [TPB/64] first message word of wave w (relative to mu0)
    unsigned long long *queue;
    int32_t num_legs, iters_first, iters_leg, num_solutions, max_total_iters;
    float L;
    uint32_t lampad_off, mupad_off, red_off, mu0_off;  // LDS byte offsets
    uint32_t slack_off;  // first of the (kBlockChunk - 1) * 64 slack words
    const float *trace_gamma;
    float scale;
    int32_t trace_T;
    float *trace;
    // binary16 mode (relay_block16_kernel): w and Gamma by slot as binary16
    // bits, the clip L as binary16 bits, and an LDS region of ceil(TPB*VPT/32)
    // words where packed corrections are assembled
    const uint16_t *w16_slot;      // [TPB*VPT]
    const uint16_t *gamma16_slot;  // [R][TPB*VPT]
    uint32_t L16;
    uint32_t stage_off;
};

// Largest static LDS of a variant's kernels.  The kernels address LDS by
// absolute offsets from 0, which is only valid without static LDS; the host
// refuses to plan a variant for which this is nonzero.
hipError_t block_static_lds(int v, size_t *bytes);
hipError_t variant_static_lds(int v, size_t *bytes);

int num_block_variants();
BlockShape block_variant_shape(int v);
hipError_t block_variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks);
// Allows `lds` bytes of dynamic LDS for every instantiation of variant v.
hipError_t block_prepare(int v, size_t lds);
// dst[r][s] = src[r][slot_col[s]] (0 for spare slots), r < rows
hipError_t launch_gather_slots(const float *src, int64_t src_stride, const int32_t *slot_col, int npad,
                               int rows, float *dst, hipStream_t s);
hipError_t launch_block(int v, bool prior_anchor, bool trace, const BlockArgs &a, int grid,
                        size_t lds, hipStream_t s);

// The binary16 block kernel (two syndromes per workgroup, one in each half of
// every LDS word and register): configuration v has the shape of block
// variant v.
int num_block16_variants();
BlockShape block16_variant_shape(int v);
hipError_t block16_static_lds(int v, size_t *bytes);
hipError_t block16_variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks);
hipError_t block16_prepare(int v, size_t lds);
hipError_t launch_block16(int v, bool prior_anchor, bool trace, const BlockArgs &a, int grid, size_t lds,
                          hipStream_t s);
// dst[k] = binary16 bits of src[k] (round to nearest even), k < n
hipError_t launch_to_half(const float *src, int64_t n, uint16_t *dst, hipStream_t s);

// Shape of a large-graph configuration: TPB threads decode one syndrome;
// thread t owns the fault slots t + TPB*v (v < VR) and up to kLargeRounds
// checks.
struct LargeShape {
    int TPB, VR;
};
constexpr int kLargeRounds = 4;       // checks per thread at most (M <= 4 * TPB)
constexpr int kLargeEdgeBits = 20;    // fault-side entry codes: record << 20 | sign-bit shift
constexpr int kLargeMaxRecords = 4096;  // 16-byte check records (record << 4 fits 16 bits)
constexpr int kLargeGather = 8;       // row chunk length (one byte of sign bits)
constexpr int kLargeRec = 4;          // entry codes per fault record (one 16-byte load)
constexpr int kLargeAhead = 2;        // fault-pass rounds whose slot loads are in flight ahead of use

struct LargeArgs {
    int32_t M, N;
    int32_t syn_stride, corr_stride;  // elements (bytes or words) per syndrome / correction row
    int32_t io_bits;                  // 1: bit-packed syndromes and corrections
    int64_t B;
    const uint8_t *syn;
    uint8_t *corr;
    uint8_t *conv;
    int32_t *legs;
    int32_t *iters;
    double *weight;
    float *final_llr;
    // fault slots: faults in order of decreasing column degree, slot p holds
    // fault slot_col[p] (-1 for the TPB*VR - N spare slots)
    const int32_t *slot_col;   // [TPB*VR]
    const float *w_slot;       // [TPB*VR] w by slot (0 for spare slots)
    const float *gamma_slot;   // [R][TPB*VR] gamma by slot
    float *lambda0;            // [grid][N] workspace: lambda(0) of the current chained leg per workgroup, by slot
    const int32_t *rowptr;     // [M+1] CSR
    const uint16_t *ctab;      // row i's fault slots from entry 8 * rbase[i], padded with N to a
                               // multiple of kLargeGather (16-byte aligned chunks), + one zero chunk
    const int32_t *rbase;      // [M] first chunk of row i in ctab
    const int32_t *rrec;       // [M] first LDS record of row i (one per 32 row positions)
    const int2 *fcol;          // [TPB*VR] (first entry in fedge, column degree) of each slot
    const uint32_t *frec;      // [TPB*VR][kLargeRec] the first entry codes of each slot (padding: 0)
    const uint32_t *fedge;     // [E] entry codes by slot, each column's in ascending check order
    const int32_t *chk_of;     // [kLargeRounds][TPB] check of thread t in round c, or -1
    int32_t rounds;            // check rounds in use (<= kLargeRounds)
    int32_t nrec;              // 16-byte check records
    unsigned long long *queue;
    int32_t num_legs, iters_first, iters_leg, num_solutions, max_total_iters;
    float L;
    uint32_t chk_off, red_off;  // LDS byte offsets: check records, scratch
    const float *trace_gamma;  // [N] by fault (trace runs)
    float scale;
    int32_t trace_T;
    float *trace;
};

int num_large_variants();
LargeShape large_variant_shape(int v);
hipError_t large_static_lds(int v, size_t *bytes);
hipError_t large_variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks);
hipError_t large_prepare(int v, size_t lds);
hipError_t launch_large(int v, bool prior_anchor, bool trace, const LargeArgs &a, int grid, size_t lds,
                        hipStream_t s);

// Per-code data of the mixed launch (device array).
struct CodeStatic {
    int32_t M, N;
    int32_t tile;  // index into the mixed tile switch
    // w [N] and gamma [R][N]; the members of a family are stored one after
    // another in member order, so member i's follow member 0's by i * N and
    // i * R * N floats
    const float *w;
    const float *gamma;
    int32_t w_uniform;  // 1: every w_j of every member of the code's family is equal
    float w0;           // w_0 of the code
    const uint32_t *lam_off;
    const uint32_t *mu_off;
    uint32_t lampad_off, mupad_off, mu0_off, half_off;
};

struct MixedArgs {
    GroupArgs run;  // outputs, strides (M_max, N_max), relay parameters
    const CodeStatic *codes;
    int32_t ncodes;
    // families: codes with the same graph and tile share one shot list and
    // queue; fam_rep[f] is a member whose tables the family uses, fam_size[f]
    // its number of members
    int32_t nfam;
    const int32_t *fam_rep;
    const int32_t *fam_size;
    const int32_t *list;       // shot lists, all codes
    const int32_t *list_cid;   // family member of each list position
    const int32_t *seg_start;  // [nfam] (device, written by the list kernels)
    const int32_t *seg_count;  // [nfam]
    const int32_t *order;      // [nfam] family visiting order (device, written by the list kernels)
    unsigned long long *queues;  // [nfam]
};

int num_variants();
TileShape variant_shape(int v);
// Position of group variant v in the mixed launch's tile switch, or -1.
int mixed_tile_of_variant(int v);
hipError_t mixed_occupancy(bool prior_anchor, size_t lds, int *blocks);
hipError_t launch_mixed(bool prior_anchor, const MixedArgs &m, int grid, size_t lds, hipStream_t s);
// Blocks of the variant's kernel that fit on one CU with `lds` bytes of LDS per block.
hipError_t variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks);
hipError_t launch_group(int v, bool prior_anchor, bool trace, const GroupArgs &a, int grid,
                        size_t lds, hipStream_t s);
hipError_t launch_gamma_table(float *tab, int R, int N, uint64_t seed, float g_first, float lo,
                              float hi, hipStream_t s);
hipError_t launch_reset_queue(unsigned long long *q, hipStream_t s);
// syn_out[b][i] = (syn_in ? syn_in[b][i] : 0) XOR parity of corr[b][j] over row i (CSR rowptr / colidx)
// (bits: corr, syn_in and syn_out bit-packed, ceil(N/32) and ceil(M/32) words per shot)
hipError_t launch_syndrome(int64_t B, int32_t M, int32_t N, const int32_t *rowptr, const int32_t *colidx,
                           const uint8_t *corr, const uint8_t *syn_in, uint8_t *syn_out, bool bits,
                           hipStream_t s);
// Builds per-code shot lists in `workspace` (shot_list_bytes(B, ncodes) bytes):
// positions sorted by (family, decreasing syndrome weight), the family of
// code c being code_fam[c] (identity when code_fam is null); the list of
// family f starts at list + seg_start[f] and holds seg_count[f] shots.  Also
// zeroes the per-family queue counters.  With code_member (member index of
// each code within its family), list_cid[p] = code_member[code_id[list[p]]].
// Layout (sized for ncodes >= nfam): hist[ncodes*256], seg_start[ncodes],
// seg_count[ncodes], order[ncodes], key[B], list[B], list_cid[B] (int32).
// (syn_stride in elements of the layout: bytes, or words when bits is set)
hipError_t launch_shot_lists(int64_t B, const uint8_t *syn, int32_t syn_stride, bool bits, const int32_t *code_id,
                             const int32_t *code_m, int ncodes, const int32_t *code_fam, int nfam,
                             const int32_t *code_member, void *workspace, unsigned long long *queues,
                             hipStream_t s);
size_t shot_list_bytes(int64_t B, int ncodes);
// Static scratch of the no-allocation mixed decode (queue counters of every
// code, then the shot lists): its size, and its device address on `device`,
// which must be the current device (looked up once per device, then cached).
constexpr size_t kNoAllocScratchBytes = size_t(12) << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, void **ptr);
constexpr int kWeightBinsHost = 256;              // weight bins of the shot-list sort
constexpr int kListHeader = kWeightBinsHost + 3;  // int32 words before key[] for one code

// Unrolled one-leg DMem-BP with learnable gamma_j and LLR scale, and its adjoint.
struct TrainArgs {
    int32_t M, N, E;
    int64_t B;
    const uint8_t *syn;     // [B][M]
    const float *w;         // [N] channel LLRs
    const float *gamma;     // [N] learnable memory strengths (device)
    const float *scale;     // [1] learnable LLR scale s (device)
    int32_t T, C;           // iterations, checkpoint interval
    float L;
    const int32_t *rowptr, *colidx, *colptr, *cedge;  // CSR / CSC (cedge: CSR edge id)
    float *llr_out;         // [B][N] Lambda(T)
    float *tape;            // [B][shot_floats]: w', checkpoints, segment tape
    int64_t shot_floats;
    const float *dllr;      // [B][N] dL/dLambda(T)
    float *gamma_part;      // [B][N] per-shot dL/dgamma
    float *scale_part;      // [B]
    float *dgamma;          // [N] out
    float *dscale;          // [1] out
};

size_t train_lds_bytes(int N, int E);
hipError_t launch_train_forward(const TrainArgs &a, hipStream_t s);
hipError_t launch_train_backward(const TrainArgs &a, hipStream_t s);

}  // namespace rb
