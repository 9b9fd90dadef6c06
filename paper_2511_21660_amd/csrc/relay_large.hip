// relay_large.hip -- Relay-BP for Tanner graphs whose check-to-fault messages
// do not fit in LDS (gfx950), such as detector-error-model matrices with a few
// thousand checks and tens of thousands of faults.
//
// Same decoder as the group and block kernels (paper Sec. 2.3: DMem-BP legs,
// Relay chaining, S solutions).  One workgroup of TPB threads decodes one
// syndrome at a time and pulls the next one from a global queue.
//
// Compressed messages.  The min-sum update gives every edge of check i the
// magnitude m1 (the smallest |nu| over the check) except the edge holding that
// minimum (its first position), which gets m2 (the second smallest), and the
// sign sign(nu_e) XOR neg_i, where neg_i is the parity of sigma_i and of the
// signs of all nu of the check.  A check's messages are therefore fixed by
// the state (m1, m2, position of the minimum, neg) plus one sign bit per edge.
// LDS holds Lambda by fault slot and one more entry, Lambda[N] = +inf, that
// row padding reads, and 16-byte check records: a row has one record per 32
// positions, each holding the state -- m1 and m2 carrying neg as their sign
// bit, the position of the minimum as the code of its edge's fault-side
// entry -- and, in its last word, the sign bits of nu at its 32 positions
// (one byte per chunk of eight).  A fault rebuilds each message it sums from
// one 16-byte read of the record holding its edge, bit for bit the message
// the other kernels store.  A 2736 x 26208 matrix with 82.6K edges takes
// about 158 KiB.
//
// Fault slots.  Faults are renumbered in order of decreasing column degree
// (slot p holds fault slot_col[p]); thread t owns the slots t + TPB*v
// (v < VR), so the 64 faults a wave handles in one round nearly always share
// their degree and the fault pass runs no entries past it.  Lambda, w, gamma
// and the chained lambda(0) are all kept by slot; corrections and marginals
// go out by fault.
//
// Roles.  Thread t owns its slots and the checks chk_of[c][t] (c < rounds):
// checks sorted by degree form groups of 64 rows of nearly the same length,
// and the groups are dealt to the waves' rounds so that every wave has about
// the same number of row chunks to run.  The graph tables stay in
// global memory, shared by all workgroups and L2-resident: each row's fault
// slots padded to a multiple of 8 (one aligned 16-byte load per 8 edges), and
// per slot (first entry, degree) and a 16-byte record of its first 4 entry
// codes (the rest come from the entry table).  An entry code (record << 20 | ((k & 31) ^ 24) for row position k)
// names the record (bits 20..31) and, in its low five bits, the left shift
// that moves the edge's sign bit to bit 31 (chunk entry q's bit is bit 7 - q
// of the chunk's byte).
//
// Iteration (as in the block kernel): the check pass of iteration t+1 reads
// Lambda(t) for every edge, so the parity of F(t) per check is folded into it
// and reduced with one barrier; leg and shot events are block-uniform.
// Lambda, nu and every lambda(0) are never -0 (channel LLRs enter as
// s * w + 0), so sign bits are the signs the min-sum update tests with x < 0.

#include <algorithm>

#include "relay_device.h"
#include "relay_internal.h"

namespace rb {
namespace {

__device__ __forceinline__ float clipl(float x, float L) { return __builtin_amdgcn_fmed3f(x, -L, L); }

// three or four words in one LDS access (plain vector types: the LDS helpers
// take no class types)
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));

// a global-memory float (kept as a global load where the pointer is chosen at
// run time between two tables)
__device__ __forceinline__ float ld_global(const void *base, uint32_t byte_off) {
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) float gfloat;
    return *(gfloat *)((gchar *)base + byte_off);
}

__device__ __forceinline__ void lds_or(uint32_t byte_addr, uint32_t v) {
    __hip_atomic_fetch_or((__attribute__((address_space(3))) uint32_t *)(size_t)byte_addr, v, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
}

// what the fault pass loads for one slot
struct SlotLoads {
    i32x2 fc;   // first entry in fedge, degree
    u32x4 ra;   // first four entry codes
    float gv;   // gamma
    float w0;   // w (lambda(0) = s * w + 0) or the chained anchor
    float lam;  // Lambda
};

// 4 * (x & 0xffff) as one instruction (a 16 x 16-bit multiply-add)
__device__ __forceinline__ uint32_t lo16_x4(uint32_t x) {
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, 4, 0" : "=v"(r) : "v"(x));
    return r;
}

template <int TPB, int VR, bool PRIOR, bool TRACE>
__global__ __launch_bounds__(TPB) void relay_large_kernel(LargeArgs a) {
    static_assert(VR <= 32 && TPB % 256 == 0, "shape");
    static_assert(kLargeGather == 8, "a row chunk is one byte of sign bits");
    constexpr int NP = TPB * VR;                          // slots (row stride of gamma_slot)
    const uint32_t red = a.red_off;                       // TPB/64 doubles (block sums)
    const uint32_t flags = a.red_off + 8u * (TPB / 64);   // TPB/64 bytes (block OR), 16-byte aligned
    const uint32_t shot_sh = flags + 4u * (TPB / 64);     // claimed shot index
    const uint32_t chk = a.chk_off;
    const int t = threadIdx.x;
    const float L = a.L;
    const int N = a.N;
    // thread index made opaque at the top of every iteration, so that the
    // per-slot addresses are recomputed where used instead of being hoisted
    // out of the persistent loop
    uint32_t tl = (uint32_t)t;

    // this thread's checks, their degrees, first row chunks and first records
    int ci[kLargeRounds], cd[kLargeRounds], crb[kLargeRounds], crec[kLargeRounds];
#pragma unroll
    for (int c = 0; c < kLargeRounds; ++c) {
        const int i = c < a.rounds ? a.chk_of[c * TPB + t] : -1;
        ci[c] = i;
        cd[c] = i >= 0 ? a.rowptr[i + 1] - a.rowptr[i] : 0;
        crb[c] = i >= 0 ? a.rbase[i] : 0;
        crec[c] = i >= 0 ? a.rrec[i] : 0;
    }
    if (t < TPB / 256) lds_b<uint32_t>(flags + 4u * (uint32_t)t) = 0u;
    if (t == 0) lds_b<float>(4u * (uint32_t)N) = __builtin_inff();  // target of row padding entries

    // lambda(0) is s * w in leg 1 and under the prior anchor (from the shared,
    // L2-resident w by slot), else (chained legs) this workgroup's slice of
    // global memory, written at each leg change
    float *l0w = a.lambda0 + (size_t)blockIdx.x * N;
    const float *gcur = a.gamma_slot;
    uint32_t sig = 0;  // bit c: syndrome bit of check ci[c]
    uint32_t best_mask = 0;
    double best_w = 0.0;
    long long shot = -1;
    int r = 0, tt = 0, total = 0, count = 0;

    // messages restart at zero: records of zeros (states (+0, +0, 0), sign
    // bits clear) rebuild +0 on every edge
    auto zero_messages = [&]() {
        for (int q = t; q < a.nrec; q += TPB) lds_b<u32x4>(chk + 16u * (uint32_t)q) = u32x4{0u, 0u, 0u, 0u};
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
        sig = 0;
#pragma unroll
        for (int c = 0; c < kLargeRounds; ++c)
            if (ci[c] >= 0 && syn_bit(a.syn, (size_t)shot, a.syn_stride, ci[c], a.io_bits)) sig |= 1u << c;
#pragma unroll
        for (int v = 0; v < VR; ++v) {
            const int p = (int)tl + TPB * v;
            if (p < N) {
                const float wj = a.scale * a.w_slot[p] + 0.0f;  // -0 enters as +0
                lds_b<float>(4u * (uint32_t)p) = wj;
                if (TRACE) a.trace[(size_t)shot * (a.trace_T + 1) * N + a.slot_col[p]] = wj;
            }
        }
        gcur = a.gamma_slot;
        zero_messages();
        return true;
    };

    bool active = fetch();
    __syncthreads();

    while (active) {
        asm volatile("" : "+v"(tl));
        // ---------------- check pass: new states from Lambda(t) and the old
        // messages; parity of F(t) per check
        uint32_t unsat_bits = 0;
        // the first chunk of each row is loaded while the previous row runs
        // (a round without a check loads chunk 0; rounds without a check may
        // precede rounds with one)
        const uint4 *ctab4 = reinterpret_cast<const uint4 *>(a.ctab);
        uint4 first = ctab4[crb[0]];
#pragma unroll
        for (int c = 0; c < kLargeRounds; ++c) {
            const int i = ci[c];
            const uint4 first_c = first;
            if (c + 1 < kLargeRounds) first = ctab4[crb[c + 1]];
            if (i < 0) continue;
            const uint32_t ra0 = chk + 16u * (uint32_t)crec[c];  // the row's first record
            const u32x3 sto = lds_b<u32x3>(ra0);
            const uint32_t m1o = sto.x, m2o = sto.y;  // old magnitudes, signed with the old neg
            // position of the old minimum (of another row, for a record of
            // zeros: out of this row, or position 24 of row 0 whose m1 and m2
            // are both +0)
            const int amo = 32 * ((int)(sto.z >> kLargeEdgeBits) - crec[c]) + (int)((sto.z & 31u) ^ 24u);
            const uint32_t sc = ((sig >> c) & 1u) << 31;
            uint32_t fpar = sc;  // bit 31: sigma_i XOR the signs of Lambda over the row
            uint32_t negp = 0;   // XOR of the row's bytes of nu signs (neg from its popcount)
            float m1 = L, m2 = L;
            // a chunk of 8 positions is one byte of sign bits, read (old
            // signs) and written (new signs) whole
            const int deg = cd[c];
            int amin = 0;
            // eight edges per step from one aligned 16-byte load of the row's
            // padded fault slots; the Lambda gathers are issued together and
            // the next chunk is loaded one step ahead (the table ends with a
            // zero chunk, so the load past a row's last chunk stays inside it).
            // Padding entries of a row's last chunk address Lambda[N] = +inf:
            // their nu is clip(inf - mu) = L, which leaves m1 <= m2 <= L, the
            // position of the minimum, both parities and the sign bits as
            // they are, so all eight entries run without a per-edge test.
            const uint4 *rt = ctab4 + crb[c];
            uint4 cur = first_c;
            for (int k = 0; k < deg; k += kLargeGather) {
                const uint4 pk = cur;
                cur = rt[k / kLargeGather + 1];
                const uint32_t pw[4] = {pk.x, pk.y, pk.z, pk.w};
                // byte (k / 8) & 3 of word 3 of record k / 32: old signs of nu,
                // entry q in bit 7 - q
                const uint32_t ba = ra0 + 16u * (uint32_t)(k >> 5) + 12u + (uint32_t)((k >> 3) & 3);
                const uint32_t ob = lds_b<uint8_t>(ba);
                float lv[kLargeGather];
#pragma unroll
                for (int q = 0; q < kLargeGather; ++q)
                    lv[q] = lds_b<float>((q & 1) ? 4u * (pw[q >> 1] >> 16) : lo16_x4(pw[q >> 1]));
                int am = amo - k;  // entry of the old minimum, if in 0..7
                asm volatile("" : "+v"(am));  // compared with each entry's constant
                int aq = -1;                  // entry of a new minimum in this chunk
                uint32_t nb = 0u;
#pragma unroll
                for (int q = 0; q < kLargeGather; ++q) {
                    const uint32_t mag = am == q ? m2o : m1o;
                    const float mo = __uint_as_float(((ob << (24 + q)) & 0x80000000u) ^ mag);
                    if (q & 1) fpar = xor3(fpar, __float_as_uint(lv[q - 1]), __float_as_uint(lv[q]));
                    const float nu = clipl(lv[q] - mo, L);
                    nb = __builtin_amdgcn_alignbit(nb, __float_as_uint(nu), 31);  // sign of nu -> bit 7 - q
                    const float av = fabsf(nu);
                    aq = av < m1 ? q : aq;
                    m2 = __builtin_amdgcn_fmed3f(m1, av, m2);
                    m1 = __builtin_amdgcn_fmed3f(m1, av, -1.0f);  // = min(m1, av): both are >= +0
                }
                amin = aq >= 0 ? k + aq : amin;
                negp ^= nb;
                lds_b<uint8_t>(ba) = (uint8_t)nb;
            }
            const uint32_t neg = sc ^ ((uint32_t)__popc(negp) << 31);
            // the state goes to every record of the row (three-word writes
            // leave the sign bits)
            const u32x3 st = u32x3{__float_as_uint(m1) | neg, __float_as_uint(m2) | neg,
                                   ((uint32_t)(crec[c] + (amin >> 5)) << kLargeEdgeBits) | ((uint32_t)(amin & 31) ^ 24u)};
            for (int rr = 0; rr == 0 || 32 * rr < deg; ++rr) lds_b<u32x3>(ra0 + 16u * (uint32_t)rr) = st;
            unsat_bits |= fpar;
        }
        // the fault pass's first kLargeAhead slot loads go out before the
        // barrier (they read no state the check pass writes; after a leg or
        // shot event they are dropped)
        const bool from_w = PRIOR || r == 1;
        const float *l0src = from_w ? a.w_slot : l0w;
        const float l0mul = from_w ? a.scale : 1.0f;
        // (the leg's gamma row is block-uniform: kept in scalar registers)
        const uint64_t gaddr = reinterpret_cast<uint64_t>(gcur);
        const char *gsrc = reinterpret_cast<const char *>(
            ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(gaddr >> 32)) << 32) |
            (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)gaddr));
        // slot loads: (first entry, degree), the first kLargeRec entry codes,
        // gamma, lambda(0) (s * w + 0 in leg 1 and under the prior anchor,
        // else the chained anchor: x * 1 + 0 = x, a chained anchor is never
        // -0) and Lambda, for round v (slot clamped so every load is in bounds)
        auto issue = [&](int v) -> SlotLoads {
            SlotLoads o;
            const uint32_t p = (uint32_t)min((int)tl + TPB * v, N - 1);
            const uint32_t o4 = 4u * p;  // byte offsets from 32-bit products (tables < 4 GiB)
            o.fc = *reinterpret_cast<const i32x2 *>(reinterpret_cast<const char *>(a.fcol) + 2u * o4);
            o.ra = *reinterpret_cast<const u32x4 *>(reinterpret_cast<const char *>(a.frec) + 4u * o4);
            o.gv = TRACE ? a.trace_gamma[a.slot_col[p]] : ld_global(gsrc, o4);
            o.w0 = ld_global(l0src, o4);
            o.lam = lds_b<float>(o4);
            // the whole record in four consecutive registers: the compiler
            // would otherwise split it into loads issued where its entries
            // are used, or into registers the next load cannot reuse
            asm volatile("" : "+v"(o.ra));
            return o;
        };
        SlotLoads ring[kLargeAhead + 1];
#pragma unroll
        for (int v = 0; v < kLargeAhead && v < VR; ++v) ring[v] = issue(v);

        const bool unsat = block_or<TPB>((unsat_bits >> 31) != 0u, flags);

        // ---------------- leg scheduler (block-uniform)
        const bool cut = a.max_total_iters > 0 && total >= a.max_total_iters;
        const bool conv_ev = !TRACE && tt >= 1 && !unsat;
        const int T_r = TRACE ? a.trace_T : (r == 1 ? a.iters_first : a.iters_leg);
        const bool leg_ev = !conv_ev && (tt >= T_r || (!TRACE && cut));
        if (conv_ev || leg_ev) {
            bool done = true;
            if (!TRACE) {
                uint32_t fm = 0;
                double part = 0.0;
#pragma unroll
                for (int v = 0; v < VR; ++v) {
                    const int p = (int)tl + TPB * v;
                    if (p < N) {
                        const bool f = lds_b<float>(4u * (uint32_t)p) < 0.0f;
                        fm |= f ? 1u << v : 0u;
                        part += (double)(f ? a.w_slot[p] : 0.0f);  // + 0 leaves the sum's bits unchanged
                    }
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
#pragma unroll
                    for (int v = 0; v < VR; ++v) {
                        const int p = (int)tl + TPB * v;
                        if (p < N) {
                            const int j = a.slot_col[p];
                            if (!a.io_bits) a.corr[(size_t)shot * a.corr_stride + j] = (uint8_t)((out >> v) & 1u);
                            if (a.final_llr) a.final_llr[(size_t)shot * N + j] = lds_b<float>(4u * (uint32_t)p);
                        }
                    }
                    if (a.io_bits) {
                        // slots hold faults in degree order, so the packed words are
                        // assembled in LDS: the first ceil(N/32) words of the Lambda
                        // region (read above; the next fetch rewrites every Lambda
                        // word below N) are cleared, each set fault ORs its bit into
                        // word j / 32, and the words go out coalesced
                        const int nw = (N + 31) >> 5;
                        __syncthreads();
                        for (int q = t; q < nw; q += TPB) lds_b<uint32_t>(4u * (uint32_t)q) = 0u;
                        __syncthreads();
#pragma unroll
                        for (int v = 0; v < VR; ++v) {
                            const int p = (int)tl + TPB * v;
                            if (p < N && ((out >> v) & 1u)) {
                                const int j = a.slot_col[p];
                                lds_or(4u * (uint32_t)(j >> 5), 1u << (j & 31));
                            }
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
                gcur = a.gamma_slot + (size_t)(r - 1) * NP;
#pragma unroll
                for (int v = 0; v < VR; ++v) {
                    const int p = (int)tl + TPB * v;
                    if (!PRIOR && p < N) l0w[p] = clipl(lds_b<float>(4u * (uint32_t)p), L);
                }
                zero_messages();
            } else {
                active = fetch();
            }
            __syncthreads();
            continue;
        }

        // ---------------- fault pass: memory term, then the messages of the
        // slot's checks in ascending check order, each rebuilt from its
        // check's state and its edge's sign bit (one read of the record that
        // holds both).  Slot loads run kLargeAhead rounds ahead of their use.
        // The first two entries are read whatever the degree (a record's
        // padding entries name record 0, a valid address; the sum skips them
        // with a select, not an added 0, which would turn -0 into +0), the
        // next two where the degree exceeds 2 (the lanes of a wave nearly
        // always share it, so the branch drops out for the whole wave), any
        // further ones one by one from fedge (slots of such degrees are dealt
        // to different rounds in different waves, so few waves wait on them
        // at a time).
        auto st_of = [&](uint32_t pk) -> u32x4 { return lds_b<u32x4>(chk + ((pk >> 16) & 0xfff0u)); };
        auto msg = [&](uint32_t pk, const u32x4 &st) -> float {
            const uint32_t mag = pk == st.z ? st.y : st.x;  // signed with the check's neg
            return __uint_as_float(((st.w << (pk & 31u)) & 0x80000000u) ^ mag);
        };
        auto one = [&](float acc, uint32_t c0) -> float { return acc + msg(c0, st_of(c0)); };
        // round v: the slot's sum from loads `o`; the loads of round
        // v + kLargeAhead go out into `ahead` (a set whose round is done)
        // unconditionally (clamped), so the count of loads in flight is the
        // same on every path and each round waits only for its own
        const int wbase = __builtin_amdgcn_readfirstlane(t & ~63);  // the wave's first thread
        auto step = [&](int v, const SlotLoads &o, SlotLoads &ahead) {
            const int p = (int)tl + TPB * v;
            // everything taken from `o` first, so its waits come before the
            // next loads go out: the empty asm takes the values as inputs and
            // keeps the loads after it
            const float y = o.gv * clipl(o.lam, L);
            const float x = (1.0f - o.gv) * (l0mul * o.w0 + 0.0f);  // (1 - gamma) lambda(0)
            float acc = clipl(x + y, L);
            i32x2 fc = o.fc;
            u32x4 ra = o.ra;
            asm volatile("" : "+v"(acc), "+v"(fc), "+v"(ra) : : "memory");
            const int deg = fc.y, q0 = fc.x;
            const uint32_t e0 = ra.x, e1 = ra.y, e2 = ra.z, e3 = ra.w;
            const u32x4 s0 = st_of(e0), s1 = st_of(e1);
            if (v + kLargeAhead < VR) ahead = issue(v + kLargeAhead);
            if (p >= N) return;
            const float m0 = msg(e0, s0), m1 = msg(e1, s1);
            if (deg >= 2) {  // every column of the DEM-shaped matrices: no selects
                acc = (acc + m0) + m1;
            } else {
                acc = deg > 0 ? acc + m0 : acc;
            }
            if (deg > 2) {  // both loads issue together; the fourth entry is read even at degree 3
                const u32x4 s2 = st_of(e2), s3 = st_of(e3);
                const float m2 = msg(e2, s2), m3 = msg(e3, s3);
                acc += m2;
                acc = deg > 3 ? acc + m3 : acc;
            }
            for (int q = q0 + kLargeRec; q < q0 + deg; ++q) acc = one(acc, a.fedge[q]);
            lds_b<float>(4u * (uint32_t)p) = acc;
            if (TRACE) a.trace[((size_t)shot * (a.trace_T + 1) + tt + 1) * N + a.slot_col[p]] = acc;
        };
#pragma unroll
        for (int v = 0; v < VR; ++v) {
            // wave-uniform exit (lane-varying exits would nest the rounds'
            // exec masks): no slot of this wave in this or a later round
            if (wbase + TPB * v >= N) break;
            step(v, ring[v % (kLargeAhead + 1)], ring[(v + kLargeAhead) % (kLargeAhead + 1)]);
        }
        ++tt;
        ++total;
        __syncthreads();
    }
}

struct LargeVariant {
    LargeShape shape;
    const void *fn[2][2];
};

#define RB_LVARIANT(TPB, VR)                                                                   \
    {{TPB, VR},                                                                                \
     {{(const void *)relay_large_kernel<TPB, VR, false, false>,                                \
       (const void *)relay_large_kernel<TPB, VR, false, true>},                                \
      {(const void *)relay_large_kernel<TPB, VR, true, false>,                                 \
       (const void *)relay_large_kernel<TPB, VR, true, true>}}}

// (threads, fault rounds per thread): N <= TPB * VR, M <= kLargeRounds * TPB;
// the planner takes the first that fits
const LargeVariant kLargeVariants[] = {
    RB_LVARIANT(1024, 16),  // N <= 16384
    RB_LVARIANT(1024, 32),  // N <= 32768
};

}  // namespace

int num_large_variants() { return (int)(sizeof(kLargeVariants) / sizeof(kLargeVariants[0])); }

LargeShape large_variant_shape(int v) { return kLargeVariants[v].shape; }

hipError_t large_variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, kLargeVariants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0], kLargeVariants[v].shape.TPB, lds);
}

hipError_t large_static_lds(int v, size_t *bytes) {
    size_t mx = 0;
    for (int p = 0; p < 2; ++p)
        for (int tr = 0; tr < 2; ++tr) {
            hipFuncAttributes attr;
            const hipError_t e = hipFuncGetAttributes(&attr, kLargeVariants[v].fn[p][tr]);
            if (e != hipSuccess) return e;
            mx = std::max(mx, (size_t)attr.sharedSizeBytes);
        }
    *bytes = mx;
    return hipSuccess;
}

hipError_t large_prepare(int v, size_t lds) {
    for (int p = 0; p < 2; ++p)
        for (int tr = 0; tr < 2; ++tr) {
            hipError_t e = hipFuncSetAttribute(kLargeVariants[v].fn[p][tr],
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

hipError_t launch_large(int v, bool prior_anchor, bool trace, const LargeArgs &a, int grid, size_t lds,
                        hipStream_t s) {
    const void *fn = kLargeVariants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0];
    LargeArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(kLargeVariants[v].shape.TPB), args, lds, s);
}

}  // namespace rb
