// relay_block.hip -- Relay-BP block kernel for large Tanner graphs (gfx950).
//
// Same decoder as relay_group_kernel (paper Sec. 2.3: DMem-BP legs, Relay
// chaining, S solutions), for graphs whose per-shot state does not fit a few
// lanes of a wave, such as detector-error-model matrices with thousands of
// faults and rows of degree up to 64.  One workgroup of TPB threads decodes
// one syndrome at a time and pulls the next one from a global queue.
//
// Roles.  Thread t owns a check, or half of a long check shared with thread
// t ^ 1, placed so that the 64 rows a wave handles have nearly the same length
// and the four SIMDs get about the same work; and thread t owns the fault
// slots s = t + TPB*v, v < VPT; slot s holds the fault of rank s in the order
// of decreasing column degree (slot_col), so each band v of slots has a
// small fixed degree cap and the thread gathers only that many messages.
//
// LDS.  Lambda[N_pad] by slot (N_pad = TPB*VPT; slots >= N are spare), a +inf
// cell and a -0 cell, reduction scratch, then the check-to-fault messages in
// "wave-ELL" order: wave w owns maxdeg(w) rows of 64 words, word (k, lane)
// holding edge k of the lane's check, so a thread's k-th message is at a
// fixed stride from its base and the 64 lanes of a wave access 64
// consecutive words (conflict-free).  Fault-side gathers read messages
// through per-thread 16-bit word indices.
//
// Check pass.  Edges are read in chunks of kBlockChunk: all loads of a chunk
// are issued before the first is used, so one LDS round trip is exposed per
// chunk rather than per edge.  Reads past the end of a wave's rows (the last
// chunk) return finite messages of other rows or zeroed slack words, paired
// with the +inf Lambda of a padded edge, so they change nothing.  The signs
// of nu and the position of the minimum stay in registers, so the second
// pass over the row only writes messages.
//
// The syndrome test is fused into the check pass (parity of F(t) over each
// row) and reduced with one barrier; leg and shot events are block-uniform,
// so the scheduler never diverges.

#include <algorithm>
#include <type_traits>

#include "relay_device.h"
#include "relay_internal.h"

namespace rb {
namespace {

__device__ __forceinline__ float clipb(float x, float L) { return __builtin_amdgcn_fmed3f(x, -L, L); }

__device__ __forceinline__ void opaque_b(uint32_t &x) { asm volatile("" : "+v"(x)); }

// (x & 0xffff) << 2 as one VALU instruction (an SDWA shift of the low half
// word), where the compiler would emit a shift and a mask
__device__ __forceinline__ uint32_t lo_half_x4(uint32_t x) {
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(r)
        : "v"(2u), "v"(x));
    return r;
}

// value of lane l ^ 1 (DPP quad permutation 1,0,3,2; the whole wave is active)
__device__ __forceinline__ int swap_pair(int x) { return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false); }

template <int TPB, int DCMAX, int VPT, uint64_t PROF, int WAVES, bool PRIOR, bool TRACE>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(WAVES)))
void relay_block_kernel(BlockArgs a) {
    constexpr int CH = kBlockChunk;
    constexpr int NMU = prof_pre(PROF, VPT);  // fault-side gather entries per thread
    constexpr int DV = prof_max(PROF, VPT);
    static_assert(TPB % 128 == 0 && CH == 8 && DCMAX % CH == 0 && DCMAX <= 64 && DV >= 1, "shape");
    const uint32_t red = a.red_off;                       // TPB/64 doubles (block sums)
    const uint32_t flags = a.red_off + 8u * (TPB / 64);   // TPB/64 bytes (block OR), 16-byte aligned
    const uint32_t shot_sh = flags + 4u * (TPB / 64);     // claimed shot index
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const float L = a.L;
    uint32_t tl = (uint32_t)t;  // thread index, opaque inside the loop

    // check side: Lambda byte addresses (16-bit, Lambda region < 64 KiB) of
    // the row's edges, kBlockChunk per uint4.  Chunk 0 stays in registers; the
    // others stream from the (L2-resident) table one chunk ahead of use.
    const uint4 *ctab = reinterpret_cast<const uint4 *>(a.chk_col);  // [DCMAX/CH + 1][TPB]
    uint4 col0 = ctab[t];
    // fault side: message word indices (16-bit)
    uint32_t mu_pk[(NMU + 1) / 2];
#pragma unroll
    for (int e = 0; e < (NMU + 1) / 2; ++e) mu_pk[e] = a.col_mu[(size_t)e * TPB + t];
    const int myrow = a.chk_row[t];           // check whose syndrome bit this thread adds, or -1
    const bool split = a.chk_split[t] != 0;   // shares its check with thread t ^ 1
    const bool first_half = (t & 1) == 0;
    // row length of this wave (uniform: read back as a scalar; made opaque
    // at the top of every iteration so that the chunk conditions derived from
    // it are recomputed by scalar compares rather than kept live in SGPRs)
    int wdeg = __builtin_amdgcn_readfirstlane(a.wave_deg[wave]);
    const uint32_t mrow = a.mu0_off + 4u * ((uint32_t)a.wave_base[wave] + (uint32_t)(t & 63));

    if (t == 0) {
        lds_b<float>(a.lampad_off) = __int_as_float(0x7f800000);
        lds_b<float>(a.mupad_off) = __int_as_float(0x80000000);
    }
    if (t < TPB / 256) lds_b<uint32_t>(flags + 4u * (uint32_t)t) = 0u;
    for (int q = t; q < (CH - 1) * 64; q += TPB) lds_b<float>(a.slack_off + 4u * q) = 0.0f;

    // Lambda of the thread's faults lives only in LDS (word j); it is read back
    // where needed, which keeps the register budget for the gather tables.
    // xl = (1 - gamma) * lambda(0) is constant within a leg and kept as such
    float xl[VPT], gm[VPT];
    bool sig = false;
    uint32_t best_mask = 0;
    double best_w = 0.0;
    long long shot = -1;
    int r = 0, tt = 0, total = 0, count = 0;

    auto zero_row = [&]() {
        for (int k = 0; k < wdeg; ++k) lds_b<float>(mrow + 256u * k) = 0.0f;
    };

    auto fetch = [&]() -> bool {
        if (t == 0) lds_b<unsigned long long>(shot_sh) = atomicAdd(a.queue, 1ull);
        __syncthreads();
        const unsigned long long nxt = lds_b<unsigned long long>(shot_sh);
        __syncthreads();
        if (nxt >= (unsigned long long)a.B) return false;
        shot = (long long)nxt;
        r = 1;
        tt = 0;
        total = 0;
        count = 0;
        best_w = __longlong_as_double(0x7ff0000000000000ll);
        best_mask = 0;
        sig = myrow >= 0 && syn_bit(a.syn, (size_t)shot, a.syn_stride, myrow, a.io_bits);
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const uint32_t sl = tl + TPB * v;
            const float wj = a.scale * a.w_slot[sl] + 0.0f;  // 0 for spare slots; -0 enters as +0
            float gj = a.gamma_slot[sl];
            if (TRACE) {
                const int j = a.slot_col[sl];
                gj = j >= 0 ? a.trace_gamma[j] : 0.0f;
                if (j >= 0) a.trace[(size_t)shot * (a.trace_T + 1) * a.N + j] = wj;
            }
            xl[v] = (1.0f - gj) * wj;
            gm[v] = gj;
            lds_b<float>(4u * sl) = wj;
        }
        zero_row();
        return true;
    };

    bool active = fetch();
    __syncthreads();

    while (active) {
        opaque_b(col0.x);
        opaque_b(col0.y);
        opaque_b(col0.z);
        opaque_b(col0.w);
#pragma unroll
        for (int e = 0; e < (NMU + 1) / 2; ++e) opaque_b(mu_pk[e]);
        opaque_b(tl);
        asm volatile("" : "+s"(wdeg));

        // ---------------- check pass
        // pass 1: nu = clip(Lambda - mu_old) per edge; min1, min2 and the
        // first position of the minimum, the signs of nu (bit k of sg) and
        // their parity; parity of F over the row.  Pass 2 only writes.
        // parities as sign bits: Lambda and nu are never -0 (channel LLRs
        // enter as s * w + 0 and no update turns a nonzero or +0 value into
        // -0), so a sign bit is the test x < 0; padding entries read
        // Lambda = +inf and give nu = L, both with a clear sign bit
        uint32_t fpar_u = sig ? 0x80000000u : 0u;
        float m1 = L, m2 = L;
        int amin = 0;
        uint32_t sg_lo = 0, sg_hi = 0;  // bit k: nu_k < 0
        // one chunk of W edges (W = CH, or 4 for a short last chunk)
        auto chunk = [&](auto w_tag, int c, const uint4 &tb) {
            constexpr int W = decltype(w_tag)::value;
            const uint32_t pk[4] = {tb.x, tb.y, tb.z, tb.w};
            float lv[W], mo[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const uint32_t ca = (q & 1) ? (pk[q >> 1] >> 16) : (pk[q >> 1] & 0xffffu);
                lv[q] = lds_b<float>(ca);
                mo[q] = lds_b<float>(mrow + 256u * (c + q));
            }
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int k = c + q;
                if (q & 1) fpar_u = xor3(fpar_u, __float_as_uint(lv[q - 1]), __float_as_uint(lv[q]));
                const float nu = clipb(lv[q] - mo[q], L);
                // shift the sign bit in at the bottom (one funnel shift): after
                // P processed steps, edge k sits at bit min(P,32)-1-k of sg_lo
                // (k < 32) or P-1-k of sg_hi
                if (k < 32)
                    sg_lo = __builtin_amdgcn_alignbit(sg_lo, __float_as_uint(nu), 31);
                else
                    sg_hi = __builtin_amdgcn_alignbit(sg_hi, __float_as_uint(nu), 31);
                const float av = fabsf(nu);
                amin = av < m1 ? k : amin;
                m2 = __builtin_amdgcn_fmed3f(m1, av, m2);
                m1 = __builtin_amdgcn_fmed3f(m1, av, -1.0f);  // = min(m1, av): both are >= +0
            }
        };
        // The next table entry is loaded unconditionally (the table holds one
        // padding entry past the last chunk), so the unrolled chunks rename
        // the two entries instead of copying them at branch merges.
        uint4 cur = col0;
#pragma unroll
        for (int c = 0; c < DCMAX; c += CH) {
            if (c >= wdeg) break;  // wave-uniform row length
            const uint4 nxt = ctab[(size_t)(c / CH + 1) * TPB + tl];
            if (c + CH / 2 >= wdeg)
                chunk(std::integral_constant<int, CH / 2>{}, c, cur);
            else
                chunk(std::integral_constant<int, CH>{}, c, cur);
            cur = nxt;
        }
        // the row's parities: F over the row, and sigma with the signs of nu
        // (a popcount of the collected sign bits)
        bool fpar = (fpar_u >> 31) != 0u;
        bool neg = sig != ((__popc(sg_lo ^ sg_hi) & 1) != 0);
        // a check split over threads t and t ^ 1: combine the two halves'
        // minima and parities (the first half holds the earlier edges, so it
        // keeps the minimum's position on a tie)
        bool owns_min = true;
        {
            const float m1o = __int_as_float(swap_pair(__float_as_int(m1)));
            const float m2o = __int_as_float(swap_pair(__float_as_int(m2)));
            const int bo = swap_pair((neg ? 1 : 0) | (fpar ? 2 : 0));
            if (split) {
                owns_min = first_half ? (m1 <= m1o) : (m1 < m1o);
                m2 = fminf(fmaxf(m1, m1o), fminf(m2, m2o));
                m1 = fminf(m1, m1o);
                neg ^= (bo & 1) != 0;
                fpar ^= (bo & 2) != 0;
            }
        }
        // pass 2: mu = +-m1 on every edge (sign of nu times the row parity),
        // then +-m2 at the minimum's position (m1, m2 >= +0)
        {
            const uint32_t flip = neg ? 0xffffffffu : 0u;
            const uint32_t s_lo = sg_lo ^ flip, s_hi = sg_hi ^ flip;
            const uint32_t b1 = __float_as_uint(m1);
            const int P = (wdeg + 3) & ~3;  // steps pass 1 processed
            const int P32 = P < 32 ? P : 32;
            auto pass2 = [&](auto full_tag, int c) {
                constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const int k = c + q;
                    const uint32_t sb = k < 32 ? (s_lo << (32 - P32 + k)) : (s_hi << (32 - P + k));
                    if (FULL || k < wdeg) lds_b<uint32_t>(mrow + 256u * k) = (sb & 0x80000000u) | b1;
                }
            };
#pragma unroll
            for (int c = 0; c < DCMAX; c += CH) {
                if (c >= wdeg) break;
                if (c + CH <= wdeg)
                    pass2(std::true_type{}, c);
                else
                    pass2(std::false_type{}, c);
            }
            if (wdeg > 0 && owns_min) {
                const uint32_t sa = amin < 32 ? (s_lo >> (P32 - 1 - amin)) : (s_hi >> (P - 1 - amin));
                lds_b<uint32_t>(mrow + 256u * (uint32_t)amin) = (sa << 31) | __float_as_uint(m2);
            }
        }
        const bool unsat = block_or<TPB>(fpar, flags);

        // ---------------- leg scheduler (block-uniform)
        const bool cut = a.max_total_iters > 0 && total >= a.max_total_iters;
        const bool conv_ev = !TRACE && tt >= 1 && !unsat;
        const int T_r = TRACE ? a.trace_T : (r == 1 ? a.iters_first : a.iters_leg);
        const bool leg_ev = !conv_ev && (tt >= T_r || (!TRACE && cut));
        if (conv_ev || leg_ev) {
            bool done = true;
            if (!TRACE) {
                // (loads first, so their latencies overlap: the per-slot tables
                // are padded to TPB * VPT entries)
                float wv[VPT];
#pragma unroll
                for (int v = 0; v < VPT; ++v) wv[v] = a.w_slot[tl + TPB * v];
                uint32_t fm = 0;
                double part = 0.0;
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    const uint32_t sl = tl + TPB * v;
                    const bool f = sl < (uint32_t)a.N && lds_b<float>(4u * sl) < 0.0f;
                    fm |= f ? 1u << v : 0u;
                    part += (double)(f ? wv[v] : 0.0f);  // + 0 leaves the sum's bits unchanged
                }
                const double W = block_sum<TPB>(part, red);
                if (conv_ev) {
                    ++count;
                    if (W < best_w) {
                        best_w = W;
                        best_mask = fm;
                    }
                    done = count >= a.num_solutions || r >= a.num_legs || cut;
                } else {
                    done = r >= a.num_legs || cut;
                }
                if (done) {
                    const uint32_t out = count > 0 ? best_mask : fm;
                    int jv[VPT];
#pragma unroll
                    for (int v = 0; v < VPT; ++v) jv[v] = a.slot_col[tl + TPB * v];
#pragma unroll
                    for (int v = 0; v < VPT; ++v) {
                        const uint32_t sl = tl + TPB * v;
                        const int j = jv[v];
                        if (j >= 0) {
                            if (!a.io_bits) a.corr[(size_t)shot * a.corr_stride + j] = (uint8_t)((out >> v) & 1u);
                            if (a.final_llr)
                                a.final_llr[(size_t)shot * a.N + j] = lds_b<float>(4u * sl);
                        }
                    }
                    if (a.io_bits) {
                        // slots hold faults in degree order, so the packed words are
                        // assembled in LDS: the first ceil(N/32) words of the Lambda
                        // region (read above for the marginals; the next fetch
                        // rewrites every Lambda word) are cleared, each fault ORs its
                        // bit into word j / 32, and the words go out coalesced
                        const int nw = (a.N + 31) >> 5;
                        __syncthreads();
                        for (int q = t; q < nw; q += TPB) lds_b<uint32_t>(4u * (uint32_t)q) = 0u;
                        __syncthreads();
#pragma unroll
                        for (int v = 0; v < VPT; ++v) {
                            const int j = jv[v];
                            if (j >= 0 && ((out >> v) & 1u))
                                __hip_atomic_fetch_or(&lds_b<uint32_t>(4u * (uint32_t)(j >> 5)), 1u << (j & 31),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        __syncthreads();
                        uint32_t *c32 = reinterpret_cast<uint32_t *>(a.corr) + (size_t)shot * a.corr_stride;
                        for (int q = t; q < nw; q += TPB) c32[q] = lds_b<uint32_t>(4u * (uint32_t)q);
                    }
                    if (t == 0) {
                        a.conv[shot] = count > 0 ? 1 : 0;
                        a.legs[shot] = r;
                        a.iters[shot] = total;
                        if (a.weight) a.weight[shot] = count > 0 ? best_w : W;
                    }
                }
            }
            if (!done) {
                ++r;
                tt = 0;
                // every slot, spare ones included (their gamma and w are 0 and
                // their Lambda stays 0), so the loads are issued together
                const float *gr = a.gamma_slot + (size_t)(r - 1) * (TPB * VPT);
                float gv[VPT], w0[VPT];
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    gv[v] = gr[tl + TPB * v];
                    w0[v] = PRIOR ? a.w_slot[tl + TPB * v] : 0.0f;
                }
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    const uint32_t sl = tl + TPB * v;
                    const float l0 = PRIOR ? a.scale * w0[v] + 0.0f : clipb(lds_b<float>(4u * sl), L);
                    gm[v] = gv[v];
                    xl[v] = (1.0f - gv[v]) * l0;
                }
                zero_row();
            } else {
                active = fetch();
            }
            __syncthreads();
            continue;
        }

        // ---------------- fault pass
        // Software-pipelined FD faults deep: the gathers of slot v+FD are
        // issued before slot v's sum is stored (the stores go to the Lambda
        // words of earlier slots, which no later load reads).  Band v gathers
        // prof_dv(PROF, v) messages; a fault of smaller degree reads the -0
        // cell for the rest.
        constexpr int FD = 2;
        auto mu_word = [&](int e) -> uint32_t {
            if (e & 1) return (mu_pk[e >> 1] >> 16) << 2;  // the compiler emits one SDWA shift
            return lo_half_x4(mu_pk[e >> 1]);
        };
        float gv[FD + 1][DV], gl[FD + 1];
        auto load_slot = [&](int v, float(&m)[DV], float &l) {
#pragma unroll
            for (int k = 0; k < prof_dv(PROF, v); ++k) m[k] = lds_b<float>(mu_word(prof_pre(PROF, v) + k));
            l = lds_b<float>(4u * (tl + TPB * v));
        };
#pragma unroll
        for (int v = 0; v < FD && v < VPT; ++v) load_slot(v, gv[v], gl[v]);
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            if (v + FD < VPT) load_slot(v + FD, gv[(v + FD) % (FD + 1)], gl[(v + FD) % (FD + 1)]);
            const float(&mv)[DV] = gv[v % (FD + 1)];
            const float y = gm[v] * clipb(gl[v % (FD + 1)], L);
            float acc = clipb(xl[v] + y, L);
#pragma unroll
            for (int k = 0; k < prof_dv(PROF, v); ++k) acc += mv[k];
            lds_b<float>(4u * (tl + TPB * v)) = acc;
            if (TRACE) {
                const int j = a.slot_col[tl + TPB * v];
                if (j >= 0) a.trace[((size_t)shot * (a.trace_T + 1) + tt + 1) * a.N + j] = acc;
            }
        }
        ++tt;
        ++total;
        __syncthreads();
    }
}

__global__ void gather_slots_kernel(const float *src, int64_t src_stride, const int32_t *slot_col,
                                    int npad, int rows, float *dst) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * npad) return;
    const int64_t r = idx / npad;
    const int j = slot_col[idx % npad];
    dst[idx] = j >= 0 ? src[r * src_stride + j] : 0.0f;
}

struct BlockVariant {
    BlockShape shape;
    const void *fn[2][2];
};

#define RB_BVARIANT(TPB, DCMAX, VPT, PROF, W)                                                 \
    {{TPB, DCMAX, VPT, PROF, W},                                                              \
     {{(const void *)relay_block_kernel<TPB, DCMAX, VPT, PROF, W, false, false>,              \
       (const void *)relay_block_kernel<TPB, DCMAX, VPT, PROF, W, false, true>},              \
      {(const void *)relay_block_kernel<TPB, DCMAX, VPT, PROF, W, true, false>,               \
       (const void *)relay_block_kernel<TPB, DCMAX, VPT, PROF, W, true, true>}}}

// (threads, max row degree, fault slots per thread, column-degree caps of the
// slot bands (band 0 in the low nibble), waves/SIMD); the planner takes the
// first that fits.
const BlockVariant kBlockVariants[] = {
    // M <= 512, N <= 4608 with the DEM's band caps: half-size workgroups, so
    // that two shots share a CU (windows of a few detector rounds of a DEM)
    RB_BVARIANT(512, 64, 9, 0x222333456ull, 4),
    // M <= 1024, N <= 9216, degrees sorted like a circuit-level DEM (weights
    // 2..6, mostly 2 and 3): band caps 6,5,4,3,3,3,2,2,2 (exactly those of the
    // 936 x 8785 matrix), then a looser profile 6,6,5,4,3,3,3,2,2
    RB_BVARIANT(1024, 64, 9, 0x222333456ull, 4),
    RB_BVARIANT(1024, 64, 9, 0x223334566ull, 4),
    RB_BVARIANT(1024, 64, 9, 0x666666666ull, 4),  // M <= 1024, N <= 9216, degree <= 6
    RB_BVARIANT(1024, 32, 4, 0x8888ull, 4),       // M <= 1024, N <= 4096, degree <= 8
    RB_BVARIANT(512, 32, 4, 0x8888ull, 2),        // M <= 512,  N <= 2048, degree <= 8
};

}  // namespace

int num_block_variants() { return (int)(sizeof(kBlockVariants) / sizeof(kBlockVariants[0])); }

BlockShape block_variant_shape(int v) { return kBlockVariants[v].shape; }

hipError_t block_variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, kBlockVariants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0],
        kBlockVariants[v].shape.TPB, lds);
}

hipError_t block_static_lds(int v, size_t *bytes) {
    size_t mx = 0;
    for (int p = 0; p < 2; ++p)
        for (int tr = 0; tr < 2; ++tr) {
            hipFuncAttributes attr;
            const hipError_t e = hipFuncGetAttributes(&attr, kBlockVariants[v].fn[p][tr]);
            if (e != hipSuccess) return e;
            mx = std::max(mx, (size_t)attr.sharedSizeBytes);
        }
    *bytes = mx;
    return hipSuccess;
}

hipError_t block_prepare(int v, size_t lds) {
    for (int p = 0; p < 2; ++p)
        for (int tr = 0; tr < 2; ++tr) {
            hipError_t e = hipFuncSetAttribute(kBlockVariants[v].fn[p][tr],
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

hipError_t launch_gather_slots(const float *src, int64_t src_stride, const int32_t *slot_col, int npad,
                               int rows, float *dst, hipStream_t s) {
    const int64_t n = (int64_t)rows * npad;
    if (n == 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(gather_slots_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                       s, src, src_stride, slot_col, npad, rows, dst);
    return hipGetLastError();
}

hipError_t launch_block(int v, bool prior_anchor, bool trace, const BlockArgs &a, int grid,
                        size_t lds, hipStream_t s) {
    const void *fn = kBlockVariants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0];
    BlockArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlockVariants[v].shape.TPB), args, lds, s);
}

}  // namespace rb
