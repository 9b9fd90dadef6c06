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
// LDS holds Lambda[0..N-1] and one more entry, Lambda[N] = +inf, that row
// padding reads; one 16-byte state per check; the sign bits of nu, one per
// slot of the padded row table.  A fault rebuilds each message it sums
// from the state of its check, bit for bit the message the other kernels
// store.  A 2736 x 26208 matrix with 82.6K edges takes about 156 KiB.
//
// Roles.  Thread t owns the faults j = t + TPB*v (v < VR) and the checks
// chk_of[c][t] (c < rounds): checks sorted by degree and dealt round by round,
// so the 64 rows a wave handles in one round have nearly the same length.
// The graph tables stay in global memory, shared by all workgroups and
// L2-resident: each row's fault indices padded to a multiple of 8 (one
// aligned 16-byte load per 8 edges) and one 32-byte record per fault with its
// first 8 (check, slot) entries (the records of a wave's lanes contiguous),
// the slot being the edge's position in the padded row table.
// A 32-bit word of sign bits can hold edges of two checks owned by different
// threads, so a check writes its bits of a shared word with two LDS atomics
// (clear, then set its own bits).
//
// Iteration (as in the block kernel): the check pass of iteration t+1 reads
// Lambda(t) for every edge, so the parity of F(t) per check is folded into it
// and reduced with one barrier; leg and shot events are block-uniform.

#include <algorithm>

#include "relay_device.h"
#include "relay_internal.h"

namespace rb {
namespace {

__device__ __forceinline__ float clipl(float x, float L) { return __builtin_amdgcn_fmed3f(x, -L, L); }

// four words in one LDS access (a plain vector type: the LDS helpers take no
// class types)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void lds_and(uint32_t byte_addr, uint32_t v) {
    __hip_atomic_fetch_and((__attribute__((address_space(3))) uint32_t *)(size_t)byte_addr, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_or(uint32_t byte_addr, uint32_t v) {
    __hip_atomic_fetch_or((__attribute__((address_space(3))) uint32_t *)(size_t)byte_addr, v, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int TPB, int VR, bool PRIOR, bool TRACE>
__global__ __launch_bounds__(TPB) void relay_large_kernel(LargeArgs a) {
    static_assert(VR <= 32 && VR % kLargeBatch == 0 && TPB % 256 == 0, "shape");
    static_assert(32 % kLargeGather == 0, "a row chunk lies in one sign word");
    const uint32_t red = a.red_off;                       // TPB/64 doubles (block sums)
    const uint32_t flags = a.red_off + 8u * (TPB / 64);   // TPB/64 bytes (block OR), 16-byte aligned
    const uint32_t shot_sh = flags + 4u * (TPB / 64);     // claimed shot index
    const uint32_t chk = a.chk_off, sgn = a.sgn_off;
    const int t = threadIdx.x;
    const float L = a.L;
    const int N = a.N;
    // thread index made opaque at the top of every iteration, so that the
    // per-fault addresses are recomputed where used instead of being hoisted
    // out of the persistent loop (2 * VR 64-bit pointers would spill)
    uint32_t tl = (uint32_t)t;

    // this thread's checks, their degrees and first row chunks
    int ci[kLargeRounds], cd[kLargeRounds], crb[kLargeRounds];
#pragma unroll
    for (int c = 0; c < kLargeRounds; ++c) {
        const int i = c < a.rounds ? a.chk_of[c * TPB + t] : -1;
        ci[c] = i;
        cd[c] = i >= 0 ? a.rowptr[i + 1] - a.rowptr[i] : 0;
        crb[c] = i >= 0 ? a.rbase[i] : 0;
    }
    if (t < TPB / 256) lds_b<uint32_t>(flags + 4u * (uint32_t)t) = 0u;
    if (t == 0) lds_b<float>(4u * (uint32_t)N) = __builtin_inff();  // target of row padding entries

    // (1 - gamma) * lambda(0) is formed each iteration from two values per
    // fault, read each iteration (coalesced: a wave's lanes own
    // consecutive faults), which keeps the registers for the loads in flight:
    // gamma of the current leg from the table; lambda(0) from w in leg 1 and
    // under the prior anchor, else (chained legs) from this workgroup's slice
    // of global memory, written at each leg change
    float *l0w = a.lambda0 + (size_t)blockIdx.x * N;
    const float *gcur = a.gamma;
    uint32_t sig = 0;  // bit c: syndrome bit of check ci[c]
    uint32_t best_mask = 0;
    double best_w = 0.0;
    long long shot = -1;
    int r = 0, tt = 0, total = 0, count = 0;

    // messages restart at zero: states (0, 0, 0, 0) and all sign bits clear
    // rebuild +0 on every edge
    auto zero_messages = [&]() {
#pragma unroll
        for (int c = 0; c < kLargeRounds; ++c)
            if (ci[c] >= 0) {
                const uint32_t sa = chk + 16u * (uint32_t)ci[c];
                lds_b<uint32_t>(sa) = 0u;
                lds_b<uint32_t>(sa + 4u) = 0u;
                lds_b<uint32_t>(sa + 8u) = 0u;
                lds_b<uint32_t>(sa + 12u) = 0u;
            }
        for (int q = t; q < a.nsw; q += TPB) lds_b<uint32_t>(sgn + 4u * (uint32_t)q) = 0u;
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
            const int j = (int)tl + TPB * v;
            if (j < N) {
                const float wj = a.scale * a.w[j];
                lds_b<float>(4u * (uint32_t)j) = wj;
                if (TRACE) a.trace[(size_t)shot * (a.trace_T + 1) * N + j] = wj;
            }
        }
        gcur = TRACE ? a.trace_gamma : a.gamma;
        zero_messages();
        return true;
    };

    bool active = fetch();
    __syncthreads();

    while (active) {
        asm volatile("" : "+v"(tl));
        // ---------------- check pass: new states from Lambda(t) and the old
        // messages; parity of F(t) per check
        bool unsat_local = false;
#pragma unroll
        for (int c = 0; c < kLargeRounds; ++c) {
            const int i = ci[c];
            if (i < 0) continue;
            const uint32_t sa = chk + 16u * (uint32_t)i;
            const u32x4 sto = lds_b<u32x4>(sa);
            const float m1o = __uint_as_float(sto.x);
            const float m2o = __uint_as_float(sto.y);
            const int amo = (int)sto.z;
            const uint32_t flipo = sto.w ? 0xffffffffu : 0u;
            const bool sc = (sig >> c) & 1u;
            bool fpar = sc, neg = sc;
            float m1 = L, m2 = L;
            // edge k of the row has the sign-bit slot e0 + k, its position in
            // the padded row table: rows start on multiples of kLargeGather,
            // so a chunk of kLargeGather edges never straddles a sign word
            const int e0 = crb[c] * kLargeGather, deg = cd[c];
            int amin = e0;
            // sign bits of the word being filled: old message signs, new nu
            // signs and the row's bits in it; a word shared with another
            // check is written with two atomics
            int cw = e0 >> 5;
            uint32_t osg = lds_b<uint32_t>(sgn + 4u * (uint32_t)cw) ^ flipo, nb = 0u, mask = 0u;
            auto flush = [&]() {
                const uint32_t wa = sgn + 4u * (uint32_t)cw;
                if (mask == 0xffffffffu) {
                    lds_b<uint32_t>(wa) = nb;
                } else if (mask != 0u) {
                    lds_and(wa, ~mask);
                    lds_or(wa, nb);
                }
            };
            // eight edges per step from one aligned 16-byte load of the row's
            // padded fault indices; the Lambda gathers are issued together
            // the next chunk is loaded one step ahead (the table ends with a
            // zero chunk, so the load past a row's last chunk stays inside it).
            // Padding entries of a row's last chunk address Lambda[N] = +inf:
            // their nu is clip(inf - mu) = L, which leaves m1 <= m2 <= L, the
            // position of the minimum, both parities and the sign bits as
            // they are, so all eight entries run without a per-edge test.
            // A chunk is one byte of a sign word (its slot is a multiple of
            // 8): old signs are read and new ones collected per byte.
            const uint4 *rt = reinterpret_cast<const uint4 *>(a.ctab) + crb[c];
            uint4 cur = rt[0];
            for (int k = 0; k < deg; k += kLargeGather) {
                const uint4 pk = cur;
                cur = rt[k / kLargeGather + 1];
                const uint32_t pw[4] = {pk.x, pk.y, pk.z, pk.w};
                float lv[kLargeGather];
#pragma unroll
                for (int q = 0; q < kLargeGather; ++q)
                    lv[q] = lds_b<float>(4u * ((q & 1) ? (pw[q >> 1] >> 16) : (pw[q >> 1] & 0xffffu)));
                const int ec = e0 + k;  // slot of the chunk's first entry
                if ((ec >> 5) != cw) {  // the row enters the next word of sign bits
                    flush();
                    cw = ec >> 5;
                    osg = lds_b<uint32_t>(sgn + 4u * (uint32_t)cw) ^ flipo;
                    nb = 0u;
                    mask = 0u;
                }
                const uint32_t sh = (uint32_t)ec & 31u;
                const uint32_t ob = osg >> sh;  // old message signs, entry q in bit q
                const int am = amo - ec;        // entry of the old minimum, if in 0..7
                uint32_t nb8 = 0u;
#pragma unroll
                for (int q = 0; q < kLargeGather; ++q) {
                    const float mag = am == q ? m2o : m1o;
                    const float mo = __uint_as_float(((ob << (31 - q)) & 0x80000000u) | __float_as_uint(mag));
                    fpar ^= lv[q] < 0.0f;
                    const float nu = clipl(lv[q] - mo, L);
                    const bool sn = nu < 0.0f;
                    neg ^= sn;
                    nb8 |= sn ? 1u << q : 0u;
                    const float av = fabsf(nu);
                    amin = av < m1 ? ec + q : amin;
                    m2 = __builtin_amdgcn_fmed3f(m1, av, m2);
                    m1 = __builtin_amdgcn_fmed3f(m1, av, -1.0f);  // = min(m1, av): both are >= +0
                }
                nb |= nb8 << sh;
                mask |= 0xffu << sh;  // padding slots belong to this row alone
            }
            flush();
            lds_b<float>(sa) = m1;
            lds_b<float>(sa + 4u) = m2;
            lds_b<int>(sa + 8u) = amin;
            lds_b<uint32_t>(sa + 12u) = neg ? 1u : 0u;
            unsat_local |= fpar;
        }
        const bool unsat = block_or<TPB>(unsat_local, flags);

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
                    const int j = (int)tl + TPB * v;
                    if (j < N) {
                        const bool f = lds_b<float>(4u * (uint32_t)j) < 0.0f;
                        fm |= f ? 1u << v : 0u;
                        part += (double)(f ? a.w[j] : 0.0f);  // + 0 leaves the sum's bits unchanged
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
                        const int j = (int)tl + TPB * v;
                        if (j < N) {
                            if (!a.io_bits) a.corr[(size_t)shot * a.corr_stride + j] = (uint8_t)((out >> v) & 1u);
                            if (a.final_llr) a.final_llr[(size_t)shot * N + j] = lds_b<float>(4u * (uint32_t)j);
                        }
                    }
                    if (a.io_bits) {
                        // fault j = t + TPB*v: the 64 faults of a wave in round v
                        // are words (TPB*v + 64*wave) / 32 and the next one, taken
                        // from one ballot (bits of faults >= N are 0)
                        uint32_t *c32 = reinterpret_cast<uint32_t *>(a.corr) + (size_t)shot * a.corr_stride;
                        const int lane = t & 63;
#pragma unroll
                        for (int v = 0; v < VR; ++v) {
                            const unsigned long long bal = __ballot((out >> v) & 1u);
                            const int j0 = TPB * v + (t & ~63) + (lane & 32);  // first fault of this lane's word
                            if ((lane & 31) == 0 && j0 < N)
                                c32[j0 >> 5] = (uint32_t)(lane & 32 ? bal >> 32 : bal);
                        }
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
                const float *gr = a.gamma + (size_t)(r - 1) * N;
                gcur = gr;
#pragma unroll
                for (int v = 0; v < VR; ++v) {
                    const int j = (int)tl + TPB * v;
                    if (!PRIOR && j < N) l0w[j] = clipl(lds_b<float>(4u * (uint32_t)j), L);
                }
                zero_messages();
            } else {
                active = fetch();
            }
            __syncthreads();
            continue;
        }

        // ---------------- fault pass: memory term, then the messages of the
        // fault's checks in ascending check order, each rebuilt from its
        // check's state and its edge's sign bit.  Faults go in batches of
        // kLargeBatch whose loads (column range, the 32-byte record of its
        // first kLargeGather entries, gamma, Lambda) are all issued first;
        // indices are clamped so every load is in bounds.
        // message of one (check, edge) entry, from the check's 16-byte state
        // (one LDS load) and the edge's sign word
        auto msg_of = [&](uint32_t pk) -> float {
            const uint32_t e = pk & ((1u << kLargeEdgeBits) - 1u);
            const u32x4 st = lds_b<u32x4>(chk + 16u * (pk >> kLargeEdgeBits));
            const uint32_t sw = lds_b<uint32_t>(sgn + 4u * (e >> 5));
            const uint32_t mag = e == st.z ? st.y : st.x;
            const uint32_t sb = ((sw >> (e & 31u)) ^ st.w) & 1u;
            return __uint_as_float((sb << 31) | mag);
        };
#pragma unroll
        for (int vb = 0; vb < VR; vb += kLargeBatch) {
            // this thread's faults of this and every later batch lie past N
            if ((int)tl + TPB * vb >= N) break;
            int qa[kLargeBatch], qb[kLargeBatch];
            uint4 ra[kLargeBatch], rc[kLargeBatch];
            float gv[kLargeBatch], l0[kLargeBatch], lam[kLargeBatch];
#pragma unroll
            for (int f = 0; f < kLargeBatch; ++f) {
                const int j = min((int)tl + TPB * (vb + f), N - 1);
                qa[f] = a.colptr[j];
                qb[f] = a.colptr[j + 1];
                const uint4 *fr = reinterpret_cast<const uint4 *>(a.frec) + 2 * (size_t)j;
                ra[f] = fr[0];
                rc[f] = fr[1];
                gv[f] = gcur[j];
                // lambda(0) is s * w in leg 1 and under the prior anchor (read
                // from the shared, L2-resident w), else the chained anchor
                l0[f] = (PRIOR || r == 1) ? a.scale * a.w[j] : l0w[j];
                lam[f] = lds_b<float>(4u * (uint32_t)j);
            }
#pragma unroll
            for (int f = 0; f < kLargeBatch; ++f) {
                const int j = (int)tl + TPB * (vb + f);
                if (j >= N) continue;
                const float y = gv[f] * clipl(lam[f], L);
                const float x = (1.0f - gv[f]) * l0[f];  // (1 - gamma) lambda(0)
                float acc = clipl(x + y, L);
                const uint32_t pk[kLargeGather] = {ra[f].x, ra[f].y, ra[f].z, ra[f].w,
                                                   rc[f].x, rc[f].y, rc[f].z, rc[f].w};
                // the first kLargeSure entries are read whatever the degree
                // (padding entries address check 0 and sign word 0), so their
                // loads issue together; the sum skips the padding (a select,
                // not an added 0, which would turn -0 into +0)
                const int deg = qb[f] - qa[f];
                float mv[kLargeSure];
#pragma unroll
                for (int k = 0; k < kLargeSure; ++k) mv[k] = msg_of(pk[k]);
#pragma unroll
                for (int k = 0; k < kLargeSure; ++k) acc = k < deg ? acc + mv[k] : acc;
#pragma unroll
                for (int k = kLargeSure; k < kLargeGather; ++k) {
                    if (k >= deg) break;
                    acc += msg_of(pk[k]);
                }
                for (int q = qa[f] + kLargeGather; q < qb[f]; ++q) acc += msg_of(a.fedge[q]);
                lds_b<float>(4u * (uint32_t)j) = acc;
                if (TRACE) a.trace[((size_t)shot * (a.trace_T + 1) + tt + 1) * N + j] = acc;
            }
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
