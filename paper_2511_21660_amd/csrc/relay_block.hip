// relay_block.hip -- Relay-BP block kernel for large Tanner graphs (gfx950).
//
// Same decoder as relay_group_kernel (paper Sec. 2.3: DMem-BP legs, Relay
// chaining, S solutions), for graphs whose per-shot state does not fit a few
// lanes of a wave, such as detector-error-model matrices with thousands of
// faults and rows of degree up to 64.  One workgroup of TPB threads decodes
// one syndrome at a time and pulls the next one from a global queue.
//
// Roles.  Thread t owns the check of rank t in the order of decreasing degree
// (so the 64 rows a wave handles have nearly the same length) and the faults
// j = t + TPB*v, v < VPT.
//
// LDS.  Lambda[N_pad] (N_pad = TPB*VPT; faults >= N are spare words), a +inf
// cell and a -0 cell, then the check-to-fault messages in "wave-ELL" order:
// wave w owns maxdeg(w) rows of 64 words, word (k, lane) holding edge k of the
// lane's check, so a thread's k-th message is at a fixed stride from its base
// and the 64 lanes of a wave access 64 consecutive words (conflict-free).
// Between the two passes over a row the thread parks nu in its message words.
// Fault-side gathers read messages through per-thread 16-bit word indices.
//
// The syndrome test is fused into the check pass (parity of F(t) over each
// row) and reduced with one __syncthreads_or; leg and shot events are
// block-uniform, so the scheduler never diverges.

#include <algorithm>

#include "relay_internal.h"

namespace rb {
namespace {

__device__ __forceinline__ float clipb(float x, float L) { return __builtin_amdgcn_fmed3f(x, -L, L); }

__device__ __forceinline__ void opaque_b(uint32_t &x) { asm volatile("" : "+v"(x)); }

template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) T &lds_b(uint32_t byte_addr) {
    return *(__attribute__((address_space(3))) T *)(size_t)byte_addr;
}

// Sum over the block (every thread gets the total); `red` is the byte address
// of TPB/64 doubles of LDS scratch.
template <int TPB>
__device__ __forceinline__ double block_sum(double x, uint32_t red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds_b<double>(red + 8u * wave) = x;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) tot += lds_b<double>(red + 8u * w);
    __syncthreads();
    return tot;
}

// OR of a predicate over the block (every thread gets the result); `flags` is
// the byte address of TPB/64 words of LDS scratch.  (The library's kernels
// address LDS absolutely from 0 and must not use static LDS, so the runtime's
// __syncthreads_or, which keeps its scratch in static LDS, is not used.)
template <int TPB>
__device__ __forceinline__ bool block_or(bool pred, uint32_t flags) {
    const bool any = __any(pred);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds_b<uint32_t>(flags + 4u * wave) = any ? 1u : 0u;
    __syncthreads();
    uint32_t acc = 0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) acc |= lds_b<uint32_t>(flags + 4u * w);
    __syncthreads();
    return acc != 0;
}

template <int TPB, int DCMAX, int VPT, int DV, int WAVES, bool PRIOR, bool TRACE>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(WAVES)))
void relay_block_kernel(BlockArgs a) {
    static_assert(TPB % 64 == 0 && DCMAX % 2 == 0 && (VPT * DV) % 2 == 0, "shape");
    const uint32_t red = a.red_off;                 // TPB/64 doubles of scratch
    const uint32_t shot_sh = a.red_off + 8u * (TPB / 64);  // claimed shot index
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const float L = a.L;
    uint32_t tl = (uint32_t)t;  // thread index, opaque inside the loop

    // check side: column byte addresses (16-bit, Lambda region < 64 KiB)
    uint32_t col_pk[DCMAX / 2];
    // fault side: message word indices (16-bit)
    uint32_t mu_pk[VPT * DV / 2];
#pragma unroll
    for (int e = 0; e < DCMAX / 2; ++e) col_pk[e] = a.chk_col[(size_t)e * TPB + t];
#pragma unroll
    for (int e = 0; e < VPT * DV / 2; ++e) mu_pk[e] = a.col_mu[(size_t)e * TPB + t];
    const int myrow = a.chk_row[t];           // check index or -1
    // row length of this wave (uniform: read back as a scalar)
    const int wdeg = __builtin_amdgcn_readfirstlane(a.wave_deg[wave]);
    const uint32_t mrow = a.mu0_off + 4u * ((uint32_t)a.wave_base[wave] + (uint32_t)(t & 63));

    if (t == 0) {
        lds_b<float>(a.lampad_off) = __int_as_float(0x7f800000);
        lds_b<float>(a.mupad_off) = __int_as_float(0x80000000);
    }

    float Lr[VPT], l0[VPT], gm[VPT];
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
        sig = myrow >= 0 && a.syn[(size_t)shot * a.M + myrow] != 0;
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int j = (int)tl + TPB * v;
            float wj = 0.0f, gj = 0.0f;
            if (j < a.N) {
                wj = a.scale * a.w[j];
                gj = TRACE ? a.trace_gamma[j] : a.gamma[j];
                if (TRACE) a.trace[(size_t)shot * (a.trace_T + 1) * a.N + j] = wj;
            }
            Lr[v] = wj;
            l0[v] = wj;
            gm[v] = gj;
            lds_b<float>(4u * (uint32_t)j) = wj;
        }
        zero_row();
        return true;
    };

    bool active = fetch();
    __syncthreads();

    while (active) {
#pragma unroll
        for (int e = 0; e < DCMAX / 2; ++e) opaque_b(col_pk[e]);
#pragma unroll
        for (int e = 0; e < VPT * DV / 2; ++e) opaque_b(mu_pk[e]);
        opaque_b(tl);

        // ---------------- check pass (two passes over the thread's row)
        bool fpar = sig, neg = sig;
        float m1 = L, m2 = L;
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            if (k >= wdeg) break;  // wave-uniform row length
            const uint32_t ca = (k & 1) ? (col_pk[k >> 1] >> 16) : (col_pk[k >> 1] & 0xffffu);
            const float lv = lds_b<float>(ca);
            const float mo = lds_b<float>(mrow + 256u * k);
            fpar ^= lv < 0.0f;
            const float nu = clipb(lv - mo, L);
            neg ^= nu < 0.0f;
            const float av = fabsf(nu);
            m2 = __builtin_amdgcn_fmed3f(m1, av, m2);
            m1 = fminf(m1, av);
            lds_b<float>(mrow + 256u * k) = nu;  // park nu
        }
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            if (k >= wdeg) break;
            const float nu = lds_b<float>(mrow + 256u * k);
            const float mag = (fabsf(nu) == m1) ? m2 : m1;
            lds_b<float>(mrow + 256u * k) = (neg ^ (nu < 0.0f)) ? -mag : mag;
        }
        const bool unsat = block_or<TPB>(fpar, red);

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
                for (int v = 0; v < VPT; ++v) {
                    const int j = (int)tl + TPB * v;
                    if (j < a.N && Lr[v] < 0.0f) {
                        fm |= 1u << v;
                        part += (double)a.w[j];
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
                    for (int v = 0; v < VPT; ++v) {
                        const int j = (int)tl + TPB * v;
                        if (j < a.N) {
                            a.corr[(size_t)shot * a.N + j] = (uint8_t)((out >> v) & 1u);
                            if (a.final_llr) a.final_llr[(size_t)shot * a.N + j] = Lr[v];
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
                const float *gr = a.gamma + (size_t)(r - 1) * a.N;
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    const int j = (int)tl + TPB * v;
                    if (j < a.N) {
                        gm[v] = gr[j];
                        l0[v] = PRIOR ? a.w[j] : clipb(Lr[v], L);
                    }
                }
                zero_row();
            } else {
                active = fetch();
            }
            __syncthreads();
            continue;
        }

        // ---------------- fault pass
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const float om = 1.0f - gm[v];
            const float x = om * l0[v];
            const float y = gm[v] * clipb(Lr[v], L);
            float acc = clipb(x + y, L);
#pragma unroll
            for (int k = 0; k < DV; ++k) {
                const int e = v * DV + k;
                const uint32_t wi = (e & 1) ? (mu_pk[e >> 1] >> 16) : (mu_pk[e >> 1] & 0xffffu);
                acc += lds_b<float>(wi << 2);
            }
            Lr[v] = acc;
            lds_b<float>(4u * (tl + TPB * v)) = acc;
            if (TRACE) {
                const int j = (int)tl + TPB * v;
                if (j < a.N) a.trace[((size_t)shot * (a.trace_T + 1) + tt + 1) * a.N + j] = acc;
            }
        }
        ++tt;
        ++total;
        __syncthreads();
    }
}

struct BlockVariant {
    BlockShape shape;
    const void *fn[2][2];
};

#define RB_BVARIANT(TPB, DCMAX, VPT, DV, W)                                                   \
    {{TPB, DCMAX, VPT, DV, W},                                                                \
     {{(const void *)relay_block_kernel<TPB, DCMAX, VPT, DV, W, false, false>,                \
       (const void *)relay_block_kernel<TPB, DCMAX, VPT, DV, W, false, true>},                \
      {(const void *)relay_block_kernel<TPB, DCMAX, VPT, DV, W, true, false>,                 \
       (const void *)relay_block_kernel<TPB, DCMAX, VPT, DV, W, true, true>}}}

// (threads, max row degree, faults per thread, max column degree, waves/SIMD)
const BlockVariant kBlockVariants[] = {
    RB_BVARIANT(1024, 64, 9, 6, 4),   // M <= 1024, N <= 9216 (DEM-shaped 936 x 8785)
    RB_BVARIANT(1024, 32, 4, 8, 4),   // M <= 1024, N <= 4096
    RB_BVARIANT(512, 32, 4, 8, 2),    // M <= 512,  N <= 2048
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

hipError_t launch_block(int v, bool prior_anchor, bool trace, const BlockArgs &a, int grid,
                        size_t lds, hipStream_t s) {
    const void *fn = kBlockVariants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0];
    BlockArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlockVariants[v].shape.TPB), args, lds, s);
}

}  // namespace rb
