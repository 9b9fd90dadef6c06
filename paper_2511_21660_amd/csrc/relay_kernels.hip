// relay_kernels.hip -- Relay-BP decoding kernels for MI355X (gfx950).
//
// Relay (paper Sec. 2.3): legs of DMem-BP on the Tanner graph of H.  Per
// iteration t of a leg, for every check i and fault j:
//   nu_{j->i}(t-1) = Lambda_j(t-1) - mu_{i->j}(t-1)                 (clipped)
//   mu_{i->j}(t)   = (-1)^sigma_i prod_{j'!=j} sgn(nu_{j'->i}) min_{j'!=j} |nu_{j'->i}|
//   lambda_j(t)    = (1 - gamma_j) lambda_j(0) + gamma_j Lambda_j(t-1)
//   Lambda_j(t)    = lambda_j(t) + sum_i mu_{i->j}(t)       (ascending i)
//   F_j            = [Lambda_j(t) < 0];   converged iff H F = sigma.
// Leg r >= 2 restarts the check messages at zero from Lambda^{(r-1)}; the
// memory anchor is clip(Lambda^{(r-1)}) (chain) or w (prior).
//
// Execution model.  One block is one wave64.  A wave holds 64/G shot slots;
// the G lanes of a slot decode one syndrome together and pull the next one
// from a global queue when it finishes, so the long tail of hard syndromes
// never stalls the other slots of the wave.  Per-shot state lives in LDS
// (marginals Lambda[N] and one row of DC check messages per check) and in
// registers (the lane's faults: Lambda, lambda(0), gamma; its checks'
// syndrome bits).  The graph is precompiled into per-lane LDS byte offsets
// held in registers, so a gather is a single ds_read with no index load.
//
// Check update (min1 / min2 / sign parity): for one check the two smallest
// |nu| are tracked with min/max only; edge k then receives m2 if |nu_k| == m1
// else m1, which equals the minimum over the other edges exactly (on a tie
// m1 == m2).  Magnitudes are selected, never rounded, so the result is
// bit-identical to the per-edge definition.  Padded edges gather +inf, which
// clips to +L and leaves min, parity and sign untouched; padded fault edges
// gather -0, the exact identity of FP32 addition.
//
// Fused syndrome test: the check pass of iteration t+1 gathers Lambda_j(t)
// for every edge anyway, so the parity of F(t) per check is folded into it
// and the group reduces "any check unsatisfied" with one wave ballot.  When a
// slot ends a leg or a shot, that speculative check pass is discarded and
// redone from the restarted state.
//
// FP order is the canonical one (no contraction: built with
// -ffp-contract=off): nu = clip(Lambda - mu); lambda = clip(a + b) with
// a = (1 - gamma) * lambda(0), b = gamma * clip(Lambda); sums in ascending i.

#include "relay_internal.h"

namespace rb {
namespace {

__device__ __forceinline__ float clipf(float x, float L) { return fminf(fmaxf(x, -L), L); }

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) for the memory strengths
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t philox_word(uint64_t seed, uint32_t c0, uint32_t c1,
                                                uint32_t pick) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t x0 = c0, x1 = c1, x2 = 0u, x3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
        const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
        const uint32_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
    }
    return pick == 0 ? x0 : pick == 1 ? x1 : pick == 2 ? x2 : x3;
}

// gamma table [R][N]: leg 1 uses g_first; leg r >= 2 uses lo + (hi - lo) u,
// u = (x >> 8) 2^-24, x = Philox(seed; floor(j/4), r, 0, 0)[j mod 4].
__global__ void gamma_table_kernel(float *tab, int R, int N, uint64_t seed, float g_first,
                                   float lo, float hi) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)R * N) return;
    const int r = (int)(idx / N) + 1;
    const int j = (int)(idx % N);
    float g;
    if (r == 1) {
        g = g_first;
    } else {
        const uint32_t x = philox_word(seed, (uint32_t)(j >> 2), (uint32_t)r, (uint32_t)(j & 3));
        const float u = (float)(x >> 8) * 0x1p-24f;
        const float span = hi - lo;
        const float prod = span * u;
        g = lo + prod;
    }
    tab[idx] = g;
}

__global__ void reset_queue_kernel(unsigned long long *q) { *q = 0ull; }

template <typename T>
__device__ __forceinline__ T &lds_at(char *lds, uint32_t byte_addr) {
    return *reinterpret_cast<T *>(lds + byte_addr);
}

// Sum over the G lanes of a slot (xor butterfly; every lane gets the total).
template <int G>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, G);
    return x;
}

// ------------------------------------------------------------------------
// The group kernel
// ------------------------------------------------------------------------
template <int G, int CPT, int DC, int VPT, int DV, bool PRIOR, bool TRACE>
__global__ __launch_bounds__(64) void relay_group_kernel(GroupArgs a) {
    static_assert(64 % G == 0, "G must divide the wave");
    static_assert(CPT <= 32 && VPT <= 32, "per-lane bit masks are 32 bits");
    extern __shared__ __align__(16) char lds[];

    const int lane = threadIdx.x;
    const int g = lane % G;
    const int slot = lane / G;
    const uint32_t base = (uint32_t)slot * a.slot_bytes;
    const uint32_t mu_row0 = base + a.mu0_off + (uint32_t)g * DC * 4u;  // row of check g
    constexpr uint32_t ROW_STRIDE = (uint32_t)G * DC * 4u;               // bytes between c, c+1
    const unsigned long long gmask =
        (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (uint32_t)(slot * G));
    const float L = a.L;

    // ---- per-lane gather tables (absolute LDS byte addresses)
    uint32_t lam_addr[CPT][DC];
    uint32_t mu_addr[VPT][DV];
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int k = 0; k < DC; ++k) lam_addr[c][k] = base + a.lam_off[(g * CPT + c) * DC + k];
#pragma unroll
    for (int v = 0; v < VPT; ++v)
#pragma unroll
        for (int k = 0; k < DV; ++k) mu_addr[v][k] = base + a.mu_off[(g * VPT + v) * DV + k];

    if (g == 0) {
        lds_at<float>(lds, base + a.lampad_off) = __int_as_float(0x7f800000);  // +inf
        lds_at<float>(lds, base + a.mupad_off) = __int_as_float(0x80000000);   // -0
    }

    // ---- per-slot state (identical in the G lanes of a slot)
    float Lr[VPT];  // Lambda_j of the lane's faults (unclipped)
    float l0[VPT];  // lambda_j(0)
    float gm[VPT];  // gamma_j of the current leg
    uint32_t sig = 0;        // sigma bits of the lane's checks
    uint32_t best_mask = 0;  // best solution bits of the lane's faults
    double best_w = 0.0;
    long long shot = -1;
    int r = 0, t = 0, total = 0, count = 0;
    bool active = false;

    auto zero_rows = [&]() {
#pragma unroll
        for (int c = 0; c < CPT; ++c)
#pragma unroll
            for (int k = 0; k < DC; ++k) lds_at<float>(lds, mu_row0 + c * ROW_STRIDE + 4u * k) = 0.0f;
    };

    // claim the next syndrome for this slot and initialise leg 1
    auto fetch = [&]() {
        unsigned long long nxt = 0;
        if (g == 0) nxt = atomicAdd(a.queue, 1ull);
        nxt = __shfl(nxt, 0, G);
        if (nxt >= (unsigned long long)a.B) {
            active = false;
            return;
        }
        active = true;
        shot = (long long)nxt;
        r = 1;
        t = 0;
        total = 0;
        count = 0;
        best_w = __longlong_as_double(0x7ff0000000000000ll);  // +inf
        best_mask = 0;
        sig = 0;
        const uint8_t *s = a.syn + (size_t)shot * a.M;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int i = g + G * c;
            if (i < a.M && s[i]) sig |= 1u << c;
        }
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int j = g + G * v;
            float wj = 0.0f, gj = 0.0f;
            if (j < a.N) {
                wj = a.scale * a.w[j];
                gj = TRACE ? a.trace_gamma[j] : a.gamma[j];
                lds_at<float>(lds, base + 4u * j) = wj;
                if (TRACE) a.trace[(size_t)shot * (a.trace_T + 1) * a.N + j] = wj;
            }
            Lr[v] = wj;
            l0[v] = wj;
            gm[v] = gj;
        }
        zero_rows();
    };

    fetch();
    __syncthreads();

    while (__any(active)) {
        // ---------------- check pass: mu(t+1) from Lambda(t), mu(t); parity of F(t)
        bool mism = false;
        if (active) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const uint32_t row = mu_row0 + c * ROW_STRIDE;
                float mo[DC], lv[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) mo[k] = lds_at<float>(lds, row + 4u * k);
#pragma unroll
                for (int k = 0; k < DC; ++k) lv[k] = lds_at<float>(lds, lam_addr[c][k]);
                const uint32_t sc = (sig >> c) & 1u;
                uint32_t par = sc;
#pragma unroll
                for (int k = 0; k < DC; ++k) par ^= (lv[k] < 0.0f) ? 1u : 0u;
                mism |= (par != 0u);
                float nu[DC];
                uint32_t sg = sc;
                float m1 = L, m2 = L;
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    nu[k] = clipf(lv[k] - mo[k], L);
                    sg ^= (nu[k] < 0.0f) ? 1u : 0u;
                    const float av = fabsf(nu[k]);
                    m2 = fminf(m2, fmaxf(m1, av));
                    m1 = fminf(m1, av);
                }
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    const float av = fabsf(nu[k]);
                    const float mag = (av == m1) ? m2 : m1;
                    const uint32_t s = sg ^ ((nu[k] < 0.0f) ? 1u : 0u);
                    lds_at<float>(lds, row + 4u * k) = s ? -mag : mag;
                }
            }
        }
        const unsigned long long bal = __ballot(mism);

        // ---------------- leg scheduler (per slot)
        const bool cut = a.max_total_iters > 0 && total >= a.max_total_iters;
        const bool conv_ev = !TRACE && active && t >= 1 && (bal & gmask) == 0ull;
        const int T_r = TRACE ? a.trace_T : (r == 1 ? a.iters_first : a.iters_leg);
        const bool leg_ev = active && !conv_ev && (t >= T_r || (!TRACE && cut));
        const bool event = conv_ev || leg_ev;
        if (event) {
            bool done = true;
            if (!TRACE) {
                if (conv_ev) {
                    ++count;
                    double part = 0.0;
                    uint32_t fm = 0;
#pragma unroll
                    for (int v = 0; v < VPT; ++v) {
                        const int j = g + G * v;
                        if (j < a.N && Lr[v] < 0.0f) {
                            part += (double)a.w[j];
                            fm |= 1u << v;
                        }
                    }
                    const double W = group_sum<G>(part);
                    if (W < best_w) {
                        best_w = W;
                        best_mask = fm;
                    }
                    done = count >= a.num_solutions || r >= a.num_legs || cut;
                } else {
                    done = r >= a.num_legs || cut;
                }
            }
            if (!done) {
                // chain to leg r+1: restart check messages, new Gamma, new anchor
                ++r;
                t = 0;
                const float *gr = a.gamma + (size_t)(r - 1) * a.N;
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    const int j = g + G * v;
                    if (j < a.N) {
                        gm[v] = gr[j];
                        l0[v] = PRIOR ? a.w[j] : clipf(Lr[v], L);
                    }
                }
                zero_rows();
            } else {
                if (!TRACE) {
                    uint32_t fm = 0;
                    double part = 0.0;
#pragma unroll
                    for (int v = 0; v < VPT; ++v) {
                        const int j = g + G * v;
                        if (j < a.N && Lr[v] < 0.0f) {
                            fm |= 1u << v;
                            part += (double)a.w[j];
                        }
                    }
                    const double Wlast = group_sum<G>(part);
                    const uint32_t out = count > 0 ? best_mask : fm;
#pragma unroll
                    for (int v = 0; v < VPT; ++v) {
                        const int j = g + G * v;
                        if (j < a.N) {
                            a.corr[(size_t)shot * a.N + j] = (uint8_t)((out >> v) & 1u);
                            if (a.final_llr) a.final_llr[(size_t)shot * a.N + j] = Lr[v];
                        }
                    }
                    if (g == 0) {
                        a.conv[shot] = count > 0 ? 1 : 0;
                        a.legs[shot] = r;
                        a.iters[shot] = total;
                        if (a.weight) a.weight[shot] = count > 0 ? best_w : Wlast;
                    }
                }
                fetch();
            }
        }
        __syncthreads();

        // ---------------- fault pass: memory term, marginals, Lambda(t+1)
        if (active && !event) {
#pragma unroll
            for (int v = 0; v < VPT; ++v) {
                const float om = 1.0f - gm[v];
                const float x = om * l0[v];
                const float y = gm[v] * clipf(Lr[v], L);
                float acc = clipf(x + y, L);
#pragma unroll
                for (int k = 0; k < DV; ++k) acc += lds_at<float>(lds, mu_addr[v][k]);
                Lr[v] = acc;
                const int j = g + G * v;
                if (j < a.N) {
                    lds_at<float>(lds, base + 4u * j) = acc;
                    if (TRACE) a.trace[((size_t)shot * (a.trace_T + 1) + t + 1) * a.N + j] = acc;
                }
            }
            ++t;
            ++total;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// Configuration table
// ------------------------------------------------------------------------
struct Variant {
    TileShape shape;
    const void *fn[2][2];  // [prior][trace]
};

#define RB_VARIANT(G, CPT, DC, VPT, DV)                                                     \
    {{G, CPT, DC, VPT, DV},                                                                 \
     {{(const void *)relay_group_kernel<G, CPT, DC, VPT, DV, false, false>,                 \
       (const void *)relay_group_kernel<G, CPT, DC, VPT, DV, false, true>},                 \
      {(const void *)relay_group_kernel<G, CPT, DC, VPT, DV, true, false>,                  \
       (const void *)relay_group_kernel<G, CPT, DC, VPT, DV, true, true>}}}

const Variant kVariants[] = {
    // regular degree-(6, 3) graphs: bivariate-bicycle check matrices
    RB_VARIANT(4, 9, 6, 18, 3),    // M <= 36,  N <= 72
    RB_VARIANT(8, 6, 6, 12, 3),    // M <= 48,  N <= 96
    RB_VARIANT(8, 9, 6, 18, 3),    // M <= 72,  N <= 144
    RB_VARIANT(16, 5, 6, 9, 3),    // M <= 80,  N <= 144
    RB_VARIANT(16, 9, 6, 18, 3),   // M <= 144, N <= 288
    RB_VARIANT(32, 5, 6, 9, 3),    // M <= 160, N <= 288
    // irregular small graphs
    RB_VARIANT(16, 4, 16, 8, 8),   // M <= 64,  N <= 128
    RB_VARIANT(64, 4, 16, 8, 8),   // M <= 256, N <= 512
};

}  // namespace

int num_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

TileShape variant_shape(int v) { return kVariants[v].shape; }

hipError_t variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, kVariants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0], 64, lds);
}

hipError_t launch_group(int v, bool prior_anchor, bool trace, const GroupArgs &a, int grid,
                        size_t lds, hipStream_t s) {
    const void *fn = kVariants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0];
    GroupArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(64), args, lds, s);
}

hipError_t launch_gamma_table(float *tab, int R, int N, uint64_t seed, float g_first, float lo,
                              float hi, hipStream_t s) {
    const int64_t total = (int64_t)R * N;
    const int threads = 256;
    const int blocks = (int)((total + threads - 1) / threads);
    hipLaunchKernelGGL(gamma_table_kernel, dim3(blocks), dim3(threads), 0, s, tab, R, N, seed,
                       g_first, lo, hi);
    return hipGetLastError();
}

hipError_t launch_reset_queue(unsigned long long *q, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, s, q);
    return hipGetLastError();
}

}  // namespace rb
