// relay_train.hip -- differentiable unrolled DMem-BP (one leg) and its adjoint.
//
// Forward (paper Sec. 2.3, one Relay leg from the leg-1 initialisation):
// channel LLRs w'_j = s w_j with a learnable scale s, learnable per-column
// memory strengths gamma_j, T iterations without the convergence stop:
//   nu_e(t-1)  = clip(Lambda_j(t-1) - mu_e(t-1))                e = (i, j)
//   mu_e(t)    = S_e(t) * min_{e' in N(i)\e} |nu_e'(t-1)|      (clipped at L)
//   lambda_j(t)= clip((1 - gamma_j) w'_j + gamma_j clip(Lambda_j(t-1)))
//   Lambda_j(t)= lambda_j(t) + sum_{e in N(j)} mu_e(t)            (ascending i)
// with the same FP32 operation order as the decoder, so Lambda(T) is
// bit-identical to rb_trace.  The state (Lambda, mu) is checkpointed every C
// iterations.
//
// Adjoint.  mu_e(t) depends on one nu only: the minimum over the other edges
// of its check sits at the check's argmin k1 (for e != k1) or at the second
// argmin k2 (for e == k1).  Its sign S_e is piecewise constant, so the
// gradient flows as d mu_e / d nu_src = S_e sgn(nu_src), and not at all
// through S_e, through a saturated clip, or out of a degree-1 check.  The
// memory term gives d lambda / d gamma = clip(Lambda(t-1)) - w', d lambda /
// d w' = 1 - gamma and d lambda / d Lambda(t-1) = gamma (inside the clips);
// w' = s w gives d / d s = w for both lambda(0) and Lambda(0).  The reverse
// sweep runs segment by segment: it recomputes the C states of a segment from
// its checkpoint into a tape, then walks the iterations backwards.
//
// One wave decodes one shot: lanes stride over checks and faults; the shot's
// state and adjoint live in LDS.  Per-shot gradient partials are reduced over
// the batch in a fixed order, so the gradients are deterministic.

#include "relay_internal.h"

namespace rb {
namespace {

__device__ __forceinline__ float clipt(float x, float L) { return __builtin_amdgcn_fmed3f(x, -L, L); }

template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) T &ldst(uint32_t byte_addr) {
    return *(__attribute__((address_space(3))) T *)(size_t)byte_addr;
}

// LDS of one wave (bytes): Lam[N], mu[E], nu[E], then (backward) dLam[N],
// dmu[E], dlam0[N], dgam[N].
struct TrainLds {
    uint32_t lam, mu, nu, dlam, dmu, dlam0, dgam;
};

__device__ __forceinline__ TrainLds train_lds(int N, int E) {
    TrainLds l;
    l.lam = 0;
    l.mu = l.lam + 4u * N;
    l.nu = l.mu + 4u * E;
    l.dlam = l.nu + 4u * E;
    l.dmu = l.dlam + 4u * N;
    l.dlam0 = l.dmu + 4u * E;
    l.dgam = l.dlam0 + 4u * N;
    return l;
}

// One forward iteration on the LDS state (same arithmetic as the decoder).
__device__ void train_iteration(const TrainArgs &a, const TrainLds &l, const uint8_t *sig,
                                const float *wp) {
    const int lane = threadIdx.x;
    const float L = a.L;
    for (int i = lane; i < a.M; i += 64) {
        const int b = a.rowptr[i], e1 = a.rowptr[i + 1];
        bool neg = sig[i] != 0;
        float m1 = L, m2 = L;
        for (int e = b; e < e1; ++e) {
            const float nu = clipt(ldst<float>(l.lam + 4u * a.colidx[e]) - ldst<float>(l.mu + 4u * e), L);
            ldst<float>(l.nu + 4u * e) = nu;
            neg ^= nu < 0.0f;
            const float av = fabsf(nu);
            m2 = __builtin_amdgcn_fmed3f(m1, av, m2);
            m1 = fminf(m1, av);
        }
        for (int e = b; e < e1; ++e) {
            const float nu = ldst<float>(l.nu + 4u * e);
            const float mag = (fabsf(nu) == m1) ? m2 : m1;
            ldst<float>(l.mu + 4u * e) = (neg ^ (nu < 0.0f)) ? -mag : mag;
        }
    }
    __syncthreads();
    for (int j = lane; j < a.N; j += 64) {
        const float g = a.gamma[j];
        const float om = 1.0f - g;
        const float x = om * wp[j];
        const float y = g * clipt(ldst<float>(l.lam + 4u * j), L);
        float acc = clipt(x + y, L);
        for (int c = a.colptr[j]; c < a.colptr[j + 1]; ++c) acc += ldst<float>(l.mu + 4u * a.cedge[c]);
        ldst<float>(l.lam + 4u * j) = acc;
    }
    __syncthreads();
}

__device__ __forceinline__ void save_state(const TrainArgs &a, const TrainLds &l, float *dst) {
    for (int j = threadIdx.x; j < a.N; j += 64) dst[j] = ldst<float>(l.lam + 4u * j);
    for (int e = threadIdx.x; e < a.E; e += 64) dst[a.N + e] = ldst<float>(l.mu + 4u * e);
}

__device__ __forceinline__ void load_state(const TrainArgs &a, const TrainLds &l, const float *src) {
    for (int j = threadIdx.x; j < a.N; j += 64) ldst<float>(l.lam + 4u * j) = src[j];
    for (int e = threadIdx.x; e < a.E; e += 64) ldst<float>(l.mu + 4u * e) = src[a.N + e];
    __syncthreads();
}

// shot b's scaled LLRs w' (one row of the shot scratch)
__device__ __forceinline__ float *shot_wp(const TrainArgs &a, int64_t b) {
    return a.tape + (size_t)b * a.shot_floats;
}

__global__ __launch_bounds__(64) void train_forward_kernel(TrainArgs a) {
    const int64_t b = blockIdx.x;
    if (b >= a.B) return;
    const TrainLds l = train_lds(a.N, a.E);
    const uint8_t *sig = a.syn + (size_t)b * a.M;
    float *wp = shot_wp(a, b);
    float *ckpt = wp + a.N;  // (T/C + 1) checkpoints of N + E floats
    const float s = *a.scale;
    for (int j = threadIdx.x; j < a.N; j += 64) {
        const float v = s * a.w[j];
        wp[j] = v;
        ldst<float>(l.lam + 4u * j) = v;
    }
    for (int e = threadIdx.x; e < a.E; e += 64) ldst<float>(l.mu + 4u * e) = 0.0f;
    __syncthreads();
    save_state(a, l, ckpt);
    __syncthreads();
    for (int t = 1; t <= a.T; ++t) {
        train_iteration(a, l, sig, wp);
        if (t % a.C == 0 && t < a.T) {
            save_state(a, l, ckpt + (size_t)(t / a.C) * (a.N + a.E));
            __syncthreads();
        }
    }
    for (int j = threadIdx.x; j < a.N; j += 64) a.llr_out[(size_t)b * a.N + j] = ldst<float>(l.lam + 4u * j);
}

__global__ __launch_bounds__(64) void train_backward_kernel(TrainArgs a) {
    const int64_t b = blockIdx.x;
    if (b >= a.B) return;
    const TrainLds l = train_lds(a.N, a.E);
    const float L = a.L;
    const uint8_t *sig = a.syn + (size_t)b * a.M;
    float *wp = shot_wp(a, b);
    float *ckpt = wp + a.N;
    const int nck = (a.T + a.C - 1) / a.C;  // checkpoints at t = 0, C, 2C, ... < T
    float *seg = ckpt + (size_t)nck * (a.N + a.E);  // C states of N + E floats
    float *gpart = a.gamma_part + (size_t)b * a.N;

    for (int j = threadIdx.x; j < a.N; j += 64) {
        ldst<float>(l.dlam + 4u * j) = a.dllr[(size_t)b * a.N + j];
        ldst<float>(l.dlam0 + 4u * j) = 0.0f;
        ldst<float>(l.dgam + 4u * j) = 0.0f;
    }
    for (int e = threadIdx.x; e < a.E; e += 64) ldst<float>(l.dmu + 4u * e) = 0.0f;
    __syncthreads();

    for (int k = nck - 1; k >= 0; --k) {
        const int t0 = k * a.C;
        const int t1 = min(a.T, t0 + a.C);  // segment covers iterations t0+1 .. t1
        // recompute states t0 .. t1-1 into the segment tape
        load_state(a, l, ckpt + (size_t)k * (a.N + a.E));
        save_state(a, l, seg);
        __syncthreads();
        for (int t = t0 + 1; t < t1; ++t) {
            train_iteration(a, l, sig, wp);
            save_state(a, l, seg + (size_t)(t - t0) * (a.N + a.E));
            __syncthreads();
        }
        // reverse sweep over iterations t1 .. t0+1
        for (int t = t1; t > t0; --t) {
            const float *st = seg + (size_t)(t - 1 - t0) * (a.N + a.E);  // state t-1
            // fault side of iteration t: Lambda(t) = lambda(t) + sum mu(t)
            for (int j = threadIdx.x; j < a.N; j += 64) {
                const float gl = ldst<float>(l.dlam + 4u * j);  // dLambda_j(t)
                for (int c = a.colptr[j]; c < a.colptr[j + 1]; ++c) {
                    const uint32_t e = (uint32_t)a.cedge[c];
                    ldst<float>(l.dmu + 4u * e) = ldst<float>(l.dmu + 4u * e) + gl;
                }
                const float g = a.gamma[j];
                const float lp = st[j];  // Lambda_j(t-1)
                const float om = 1.0f - g;
                const float x = om * wp[j];
                const float cl = clipt(lp, L);
                const float y = g * cl;
                const float pre = x + y;
                float dprev = 0.0f;
                if (pre > -L && pre < L) {
                    ldst<float>(l.dgam + 4u * j) = ldst<float>(l.dgam + 4u * j) + gl * (cl - wp[j]);
                    ldst<float>(l.dlam0 + 4u * j) = ldst<float>(l.dlam0 + 4u * j) + gl * om;
                    if (lp > -L && lp < L) dprev = gl * g;
                }
                ldst<float>(l.dlam + 4u * j) = dprev;  // now accumulates dLambda_j(t-1)
            }
            __syncthreads();
            // check side of iteration t: mu(t) from nu(t-1); nu(t-1) = Lambda(t-1) - mu(t-1)
            for (int i = threadIdx.x; i < a.M; i += 64) {
                const int e0 = a.rowptr[i], e1 = a.rowptr[i + 1];
                bool neg = sig[i] != 0;
                int k1 = -1, k2 = -1;
                float m1 = 0.0f, m2 = 0.0f;
                for (int e = e0; e < e1; ++e) {
                    const float nu = clipt(st[a.colidx[e]] - st[a.N + e], L);
                    ldst<float>(l.nu + 4u * e) = nu;
                    neg ^= nu < 0.0f;
                    const float av = fabsf(nu);
                    if (k1 < 0 || av < m1) {
                        k2 = k1;
                        m2 = m1;
                        k1 = e;
                        m1 = av;
                    } else if (k2 < 0 || av < m2) {
                        k2 = e;
                        m2 = av;
                    }
                }
                // dnu accumulated in place of dmu(t) after it is read
                float dnu1 = 0.0f, dnu2 = 0.0f;
                for (int e = e0; e < e1; ++e) {
                    const float dm = ldst<float>(l.dmu + 4u * e);  // dmu_e(t)
                    const int src = (e == k1) ? k2 : k1;
                    if (src < 0) continue;  // degree-1 check: constant message
                    const float nus = ldst<float>(l.nu + 4u * src);
                    if (!(fabsf(nus) < L)) continue;  // saturated minimum
                    const bool se = neg ^ (ldst<float>(l.nu + 4u * e) < 0.0f);  // sign of mu_e
                    const float sg = (nus > 0.0f) ? 1.0f : (nus < 0.0f ? -1.0f : 0.0f);
                    const float contrib = (se ? -dm : dm) * sg;
                    if (src == k1) dnu1 += contrib;
                    else dnu2 += contrib;
                }
                for (int e = e0; e < e1; ++e) {
                    const float dnu = (e == k1) ? dnu1 : (e == k2 ? dnu2 : 0.0f);
                    const float pre = st[a.colidx[e]] - st[a.N + e];
                    const bool live = pre > -L && pre < L;
                    ldst<float>(l.dmu + 4u * e) = live ? -dnu : 0.0f;  // dmu_e(t-1), nu part
                    ldst<float>(l.nu + 4u * e) = live ? dnu : 0.0f;    // dnu_e, gathered below
                }
            }
            __syncthreads();
            // dLambda_j(t-1) += sum of dnu over the column, in ascending check order
            for (int j = threadIdx.x; j < a.N; j += 64) {
                float acc = ldst<float>(l.dlam + 4u * j);
                for (int c = a.colptr[j]; c < a.colptr[j + 1]; ++c) acc += ldst<float>(l.nu + 4u * a.cedge[c]);
                ldst<float>(l.dlam + 4u * j) = acc;
            }
            __syncthreads();
        }
    }
    // dLambda(0) and dlambda(0) both flow into s through w' = s w
    float ds = 0.0f;
    for (int j = threadIdx.x; j < a.N; j += 64) {
        const float d0 = ldst<float>(l.dlam + 4u * j) + ldst<float>(l.dlam0 + 4u * j);
        ds += d0 * a.w[j];
        gpart[j] = ldst<float>(l.dgam + 4u * j);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ds += __shfl_xor(ds, off, 64);
    if (threadIdx.x == 0) a.scale_part[b] = ds;
}

// deterministic reduction over the batch: column j sums shots in order
__global__ void train_reduce_kernel(int64_t B, int N, const float *gamma_part, const float *scale_part,
                                    float *dgamma, float *dscale) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < N) {
        float acc = 0.0f;
        for (int64_t b = 0; b < B; ++b) acc += gamma_part[(size_t)b * N + j];
        dgamma[j] = acc;
    }
    if (j == N) {
        float acc = 0.0f;
        for (int64_t b = 0; b < B; ++b) acc += scale_part[b];
        *dscale = acc;
    }
}

}  // namespace

size_t train_lds_bytes(int N, int E) { return 4u * (size_t)(4 * N + 3 * E); }

hipError_t launch_train_forward(const TrainArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(train_forward_kernel, dim3((unsigned)a.B), dim3(64), train_lds_bytes(a.N, a.E), s, a);
    return hipGetLastError();
}

hipError_t launch_train_backward(const TrainArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(train_backward_kernel, dim3((unsigned)a.B), dim3(64), train_lds_bytes(a.N, a.E), s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(train_reduce_kernel, dim3((a.N + 1 + 127) / 128), dim3(128), 0, s, a.B, a.N, a.gamma_part,
                       a.scale_part, a.dgamma, a.dscale);
    return hipGetLastError();
}

}  // namespace rb
