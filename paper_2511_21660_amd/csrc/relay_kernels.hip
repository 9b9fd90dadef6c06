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
// Execution model.  One block is one wave64.  A wave holds NS = 64/G shot
// slots; the G lanes of a slot decode one syndrome together and pull the next
// one from a global queue when it finishes, so the long tail of hard
// syndromes never stalls the other slots of the wave.  Per-shot state lives in
// LDS (marginals Lambda[N] and one row of check messages per check) and in
// registers (the lane's faults: Lambda, lambda(0), gamma; its checks'
// syndrome bits).  The graph is precompiled into per-lane LDS byte offsets
// held in registers, so a gather is a single ds_read with no index load.
//
// LDS layout.  The LDS serves a wave's access in two halves of 32 lanes, each
// costing the largest number of distinct words on one of the 32 banks.  The
// SPH = 32/G slots of a half-wave (1 for G >= 32) are interleaved word by word
// in a region of their own: word w of slot s sits at word w*SPH + s % SPH of
// region s / SPH.  The slots of a half then occupy disjoint banks and each
// slot's G lanes can reach G banks (32 for G = 64).  Check messages are
// stored step-major (message k of check position q at word mu0 + k*G*CPT + q),
// so the lanes' own accesses (Lambda of fault g + G*v, the messages of checks
// g + G*c) touch consecutive words and are conflict-free, and a gather is
// conflict-free when its words are distinct modulo G; the host orders every
// check's edges towards that.
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

#include <mutex>

#include "relay_internal.h"

namespace rb {
namespace {

// clip(x) = min(max(x, -L), L) as one median-of-three (exact; no NaNs occur).
__device__ __forceinline__ float clipf(float x, float L) { return __builtin_amdgcn_fmed3f(x, -L, L); }

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

__global__ void reset_queue_kernel(unsigned long long *q) {
    if (threadIdx.x < kQueueSplit) q[threadIdx.x * kQueueStride] = 0ull;
}

// Makes `x` opaque to the optimiser for one loop trip (no instruction is
// emitted).  Used on loop-invariant registers so that values derived from
// them (unpacked gather addresses, per-column global pointers) are recomputed
// where used instead of being hoisted out of the persistent loop and spilled.
__device__ __forceinline__ void opaque(uint32_t &x) { asm volatile("" : "+v"(x)); }

// Orders the LDS accesses of one wave before and after this point for the
// compiler.  The group kernels run one wave per block, whose LDS instructions
// execute in issue order, so no hardware barrier and no wait for outstanding
// global loads is needed (unlike __syncthreads).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// LDS word at a byte address (the kernels use no static LDS, so the dynamic
// LDS window starts at address 0).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) T &lds_at(char *, uint32_t byte_addr) {
    return *(__attribute__((address_space(3))) T *)(size_t)byte_addr;
}

// Sum over the G lanes of a slot (xor butterfly; every lane gets the total).
template <int G>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, G);
    return x;
}

template <int G>
__device__ __forceinline__ int group_isum(int x) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, G);
    return x;
}

// ------------------------------------------------------------------------
// The group kernel
// ------------------------------------------------------------------------
// Decodes the syndromes of one code: slots claim queue positions k < a.count
// (shot = a.list[k], or k without a list) until the queue is exhausted, and
// the function returns once every slot of the wave is idle.
template <int G, int CPT, int DC, int VPT, int DV, bool PRIOR, bool TRACE, bool MULTI = false>
__device__ __forceinline__ void group_loop(const GroupArgs a) {
    static_assert(64 % G == 0, "G must divide the wave");
    static_assert(CPT <= 32 && VPT <= 32, "per-lane bit masks are 32 bits");
    static_assert(G * VPT <= kGroupReadPad, "unclamped w / gamma reads stay inside the padded tables");
    char *lds = nullptr;  // LDS is addressed by absolute byte offsets
    constexpr int NS = 64 / G;                     // slots per wave
    constexpr int SPH = G >= 32 ? 1 : 32 / G;      // slots per half-wave region
    constexpr uint32_t WORD = 4u * SPH;            // bytes between consecutive words of a slot
    constexpr uint32_t ROW_STRIDE = WORD * G;      // bytes between the messages of checks c, c+1
    constexpr uint32_t KSTRIDE = WORD * G * CPT;   // bytes between the messages of steps k, k+1
    // checks / faults per batch of the two passes: whole passes when their
    // gathered operands fit in a few dozen registers, else one check and three
    // faults at a time
    constexpr int CB = 2 * CPT * DC <= 40 ? CPT : 1;
    constexpr int FB = VPT * DV <= 16 ? VPT : 3;

    uint32_t lane_rt = threadIdx.x;
    opaque(lane_rt);  // keeps lane-derived constants inside this tile's code path
    const int lane = (int)lane_rt;
    const int g = lane % G;
    const int slot = lane / G;
    uint32_t gl = (uint32_t)g;  // lane in slot, made opaque inside the loop
    const uint32_t base = 4u * (uint32_t)(slot % SPH) + a.half_off * (uint32_t)(slot / SPH);  // word 0 of this slot
    // row of check g; made opaque inside the loop like the tables, so that its
    // constant row offsets fold into the LDS instructions instead of being
    // hoisted into registers of their own
    uint32_t mu_row0 = base + a.mu0_off + WORD * (uint32_t)g;
    const uint32_t lam_w0 = base + WORD * (uint32_t)g;                    // Lambda of fault g
    const unsigned long long gmask =
        (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (uint32_t)(slot * G));
    const float L = a.L;

    // ---- per-lane gather tables: two 16-bit slot-relative LDS byte offsets
    // per register; address = offset + slot base.
    constexpr int NLP = (CPT * DC + 1) / 2;
    constexpr int NMP = (VPT * DV + 1) / 2;
    uint32_t lam_pk[NLP];
    uint32_t mu_pk[NMP];
    {
        const uint32_t *lt = a.lam_off + (size_t)g * NLP;
        const uint32_t *mt = a.mu_off + (size_t)g * NMP;
#pragma unroll
        for (int e = 0; e < NLP; ++e) lam_pk[e] = lt[e];
#pragma unroll
        for (int e = 0; e < NMP; ++e) mu_pk[e] = mt[e];
    }
    auto lam_addr = [&](int c, int k) -> uint32_t {
        const int e = c * DC + k;
        return ((e & 1) ? (lam_pk[e >> 1] >> 16) : (lam_pk[e >> 1] & 0xffffu)) + base;
    };
    auto mu_addr = [&](int v, int k) -> uint32_t {
        const int e = v * DV + k;
        return ((e & 1) ? (mu_pk[e >> 1] >> 16) : (mu_pk[e >> 1] & 0xffffu)) + base;
    };

    if (g == 0) {
        lds_at<float>(lds, base + a.lampad_off) = __int_as_float(0x7f800000);  // +inf
        lds_at<float>(lds, base + a.mupad_off) = __int_as_float(0x80000000);   // -0
    }

    // ---- per-slot state (identical in the G lanes of a slot)
    float Lr[VPT];  // Lambda_j of the lane's faults (unclipped)
    float xl[VPT];  // (1 - gamma_j) lambda_j(0), fixed within a leg
    float gm[VPT];  // gamma_j of the current leg
    uint32_t sig = 0;        // sigma bits of the lane's checks
    uint32_t best_mask = 0;  // best solution bits of the lane's faults
    double best_w = 0.0;
    int shot = -1;  // shots are indexed in 32 bits (B < 2^31)
    int r = 0, t = 0, total = 0, count = 0;
    bool active = false;

    auto zero_rows = [&]() {
#pragma unroll
        for (int c = 0; c < CPT; ++c)
#pragma unroll
            for (int k = 0; k < DC; ++k) lds_at<float>(lds, mu_row0 + c * ROW_STRIDE + KSTRIDE * k) = 0.0f;
    };

    // w and gamma of a code: the launch's own, or (MULTI, codes sharing one
    // graph) those of family member cid, stored contiguously after member 0
    // (w at a.w + cid * N, memory strengths at a.gamma + cid * R * N)
    int cid = 0;
    auto code_w = [&](int c) -> const float * { return (MULTI && a.list_cid) ? a.w + (size_t)c * a.N : a.w; };
    auto code_gamma = [&](int c) -> const float * {
        return (MULTI && a.list_cid) ? a.gamma + (size_t)c * a.num_legs * a.N : a.gamma;
    };

    // Uniform priors (every w_j of a code equal, as under code-capacity
    // noise): w0 is the w of the current syndrome's code, and a solution's
    // weight is (number of faults set) x w0 -- exactly the FP64 sum, which
    // adds at most 2^9 copies of one 24-bit value -- so the event paths load
    // no w at all.
    const bool wu = a.w_uniform != 0;
    float w0 = a.w0;
    uint32_t in_n = 0;
#pragma unroll
    for (int v = 0; v < VPT; ++v) in_n |= (int)gl + G * v < a.N ? 1u << v : 0u;

    // Decision bits and weight of the current marginals: bit v of fm is
    // F = [Lambda < 0] of fault gl + G*v, i.e. the marginal's sign bit
    // (Lambda is never -0), shifted in from the top fault down and masked to
    // faults < N by in_n; the weight is the FP64 sum of w_j over the faults
    // set, over the slot's G lanes (adding +0 for the others leaves the sum's
    // bits unchanged), or the count times w0 under uniform priors.
    auto weight_of = [&](const float (&wv)[VPT], uint32_t &fm) -> double {
        fm = 0;
#pragma unroll
        for (int v = VPT - 1; v >= 0; --v) fm = __builtin_amdgcn_alignbit(fm, __float_as_uint(Lr[v]), 31);
        fm &= in_n;
        if (wu) return (double)group_isum<G>(__popc(fm)) * (double)w0;
        double part = 0.0;
#pragma unroll
        for (int v = 0; v < VPT; ++v) part += (double)(((fm >> v) & 1u) ? wv[v] : 0.0f);
        return group_sum<G>(part);
    };

    // The queue.  The slot draws positions sq + kQueueSplit * n from
    // sub-counter sq and works one position ahead: nx_shot / nx_cid hold the
    // shot (or -1: the queue is exhausted) and family member at the position
    // it will take next, loaded when the previous syndrome started, and lane 0
    // holds the n claimed for the position after that, so starting a syndrome
    // waits on neither the queue atomic nor the list.
    const unsigned sq = (blockIdx.x * (unsigned)NS + (unsigned)slot) % (unsigned)kQueueSplit;
    unsigned long long *const qk = a.queue + (size_t)sq * kQueueStride;
    unsigned claim = 0;
    int nx_shot = -1;
    int nx_cid = 0;
    auto prefetch = [&]() {
        const unsigned long long p = (unsigned long long)sq + kQueueSplit * (unsigned long long)__shfl(claim, 0, G);
        nx_shot = -1;
        if (p < (unsigned long long)a.count) {
            nx_shot = a.list ? a.list[p] : (int)p;
            if (MULTI && a.list_cid) nx_cid = a.list_cid[p];
            if (g == 0) claim = (unsigned)atomicAdd(qk, 1ull);
        }
    };

    // Loads that start the prefetched syndrome, all unconditional so they
    // issue together: the leg-1 memory strengths of its code into gm and,
    // when the code is not the launch's own, its w into xl (both arrays are
    // dead once a syndrome is done) or, under uniform priors, its w0; then its
    // syndrome bits, folded into a mask (the first use: one wait covers every
    // load).  The library's padded tables are read at gl + G*v from one base
    // address; the caller's trace gamma and syndromes have exactly N and M
    // entries, so those indices are clamped.
    auto load_start = [&](bool own_w, float &w0n) -> uint32_t {
        if (TRACE) {
#pragma unroll
            for (int v = 0; v < VPT; ++v) gm[v] = a.trace_gamma[min((int)gl + G * v, a.N - 1)];
        } else {
            const float *cg = code_gamma(nx_cid) + gl;
#pragma unroll
            for (int v = 0; v < VPT; ++v) gm[v] = cg[G * v];
        }
        w0n = a.w0;
        if (wu) {
            if (!own_w) w0n = code_w(nx_cid)[0];
        } else if (!own_w) {
            const float *cw = code_w(nx_cid) + gl;
#pragma unroll
            for (int v = 0; v < VPT; ++v) xl[v] = cw[G * v];
        }
        // (the layout test is uniform over the launch: taken once, outside the
        // loads)
        uint32_t raw[CPT];
        if (a.io_bits) {
            const uint32_t *sw = static_cast<const uint32_t *>(static_cast<const void *>(a.syn)) +
                                 (size_t)nx_shot * a.syn_stride;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int i = min((int)gl + G * c, a.M - 1);
                raw[c] = (sw[i >> 5] >> (i & 31)) & 1u;
            }
        } else {
            const uint8_t *sb = a.syn + (size_t)nx_shot * a.syn_stride;
#pragma unroll
            for (int c = 0; c < CPT; ++c) raw[c] = sb[min((int)gl + G * c, a.M - 1)];
        }
        uint32_t m = 0;
#pragma unroll
        for (int c = 0; c < CPT; ++c)
            if ((int)gl + G * c < a.M && raw[c] != 0u) m |= 1u << c;
        return m;
    };
    // leg 1 of the prefetched syndrome (channel LLRs wn, gm as loaded), then
    // the prefetch of the next position
    auto begin = [&](const float (&wn)[VPT], uint32_t nsig, float w0n) {
        shot = nx_shot;
        cid = nx_cid;
        w0 = w0n;
        active = true;
        r = 1;
        t = 0;
        total = 0;
        count = 0;
        best_w = __longlong_as_double(0x7ff0000000000000ll);  // +inf
        best_mask = 0;
        sig = nsig;
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int j = (int)gl + G * v;
            const bool in = j < a.N;
            // (+ 0 turns a -0 channel LLR, s * w with s or w zero, into +0)
            const float wj = in ? a.scale * (wu ? w0n : wn[v]) + 0.0f : 0.0f;
            const float gj = in ? gm[v] : 0.0f;
            // columns j >= N own spare words of the padded Lambda region
            lds_at<float>(lds, base + WORD * j) = wj;
            if (TRACE && in) a.trace[(size_t)shot * (a.trace_T + 1) * a.N + j] = wj;
            Lr[v] = wj;
            xl[v] = (1.0f - gj) * wj;
            gm[v] = gj;
        }
        zero_rows();
        prefetch();
    };

    if (g == 0) claim = (unsigned)atomicAdd(qk, 1ull);
    prefetch();
    if (nx_shot >= 0) {
        float w0n;
        const uint32_t nsig = load_start(false, w0n);
        begin(xl, nsig, w0n);
    }
    wave_sync();

    while (__any(active)) {
#pragma unroll
        for (int e = 0; e < NLP; ++e) opaque(lam_pk[e]);
#pragma unroll
        for (int e = 0; e < NMP; ++e) opaque(mu_pk[e]);
        opaque(gl);
        opaque(mu_row0);
        // ---------------- check pass: mu(t+1) from Lambda(t), mu(t); parity of F(t)
        // Checks are processed in batches of CB: every gather of a batch is
        // issued before its first message store (a store might alias a later
        // gather as far as the compiler knows, so an interleaved order would
        // serialise the LDS round trips); batches are fenced from each other
        // to keep live ranges inside the register budget.
        bool mism = false;
        if (active) {
#pragma unroll
            for (int c0 = 0; c0 < CPT; c0 += CB) {
                float mo[CB][DC], lv[CB][DC];
#pragma unroll
                for (int c = c0; c < c0 + CB && c < CPT; ++c) {
                    const uint32_t row = mu_row0 + c * ROW_STRIDE;
#pragma unroll
                    for (int k = 0; k < DC; ++k) mo[c - c0][k] = lds_at<float>(lds, row + KSTRIDE * k);
#pragma unroll
                    for (int k = 0; k < DC; ++k) lv[c - c0][k] = lds_at<float>(lds, lam_addr(c, k));
                }
#pragma unroll
                for (int c = c0; c < c0 + CB && c < CPT; ++c) {
                    const uint32_t row = mu_row0 + c * ROW_STRIDE;
                    // Signs as bit 31 of the words: sgn(x) = -1 iff x < 0 is the
                    // sign bit because no marginal is ever -0 (channel LLRs are
                    // taken +0 for -0 when a syndrome starts; a memory term is -0
                    // only from two -0 operands; a sum with a nonzero or a +0 term
                    // is not -0), hence no nu = clip(Lambda - mu) is -0 either.
                    // The parities are XORs of whole words (bit 31 is read); a
                    // message is its magnitude with the sign bit set by a mask:
                    // no lane masks pass through scalar registers, which shortens
                    // one syndrome's iteration by about a fifth.
                    const uint32_t sc = ((sig >> c) & 1u) << 31;
                    uint32_t fpar = sc;  // bit 31: sigma_i + parity of F(t) over the check
                    uint32_t neg = sc;   // bit 31: sigma_i + parity of the signs of nu
                    uint32_t nb[DC];
                    float av[DC];
                    float m1 = L, m2 = L;
#pragma unroll
                    for (int k = 0; k < DC; ++k) {
                        // (the parities fold two edges per three-input XOR)
                        if (k & 1)
                            fpar = xor3(fpar, __float_as_uint(lv[c - c0][k - 1]), __float_as_uint(lv[c - c0][k]));
                        else if (k == DC - 1)
                            fpar ^= __float_as_uint(lv[c - c0][k]);
                        const float nu = clipf(lv[c - c0][k] - mo[c - c0][k], L);
                        nb[k] = __float_as_uint(nu);
                        if (k & 1)
                            neg = xor3(neg, nb[k - 1], nb[k]);
                        else if (k == DC - 1)
                            neg ^= nb[k];
                        av[k] = fabsf(nu);
                        // two smallest magnitudes: with m1 <= m2, min(m2, max(m1, av)) is the
                        // median of (m1, av, m2)
                        m2 = __builtin_amdgcn_fmed3f(m1, av[k], m2);
                        // min(m1, av) as med3(m1, av, -1) (both are >= +0): one VOP3 op
                        // taking |nu| as a source modifier (a -inf bound would be
                        // rewritten into a VOP2 min that needs |nu| in a register)
                        m1 = __builtin_amdgcn_fmed3f(m1, av[k], -1.0f);
                    }
                    mism |= (fpar >> 31) != 0u;
#pragma unroll
                    for (int k = 0; k < DC; ++k) {
                        const float mag = (av[k] == m1) ? m2 : m1;  // >= +0: bit 31 clear
                        lds_at<uint32_t>(lds, row + KSTRIDE * k) =
                            ((neg ^ nb[k]) & 0x80000000u) | __float_as_uint(mag);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
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
            if (!TRACE) done = (conv_ev && count + 1 >= a.num_solutions) || r >= a.num_legs || cut;
            const bool start = done && nx_shot >= 0;
            // One round of loads for the whole event, issued before any store:
            // w of the shot's code (solution weights, the prior anchor); the
            // memory strengths of leg r+1 into gm, or those of leg 1 of the
            // prefetched syndrome with its bits and (codes sharing a graph) w.
            float wv[VPT];
            uint32_t nsig = 0;
            float w0n = w0;
            if (wu) {
#pragma unroll
                for (int v = 0; v < VPT; ++v) wv[v] = w0;
            } else {
                const float *cw = code_w(cid) + gl;
#pragma unroll
                for (int v = 0; v < VPT; ++v) wv[v] = cw[G * v];
            }
            if (!done) {
                // lanes past N load the next row's or the padding: their words
                // are never read
                const float *gr = code_gamma(cid) + (size_t)r * a.N + gl;
#pragma unroll
                for (int v = 0; v < VPT; ++v) gm[v] = gr[G * v];
            } else if (start) {
                nsig = load_start(!(MULTI && a.list_cid), w0n);
            }
            if (!TRACE && conv_ev) {
                ++count;
                uint32_t fm_conv = 0;
                const double W = weight_of(wv, fm_conv);
                if (W < best_w) {
                    best_w = W;
                    best_mask = fm_conv;
                }
            }
            if (!done) {
                // chain to leg r+1: restart check messages, new Gamma (in gm),
                // new anchor
                ++r;
                t = 0;
#pragma unroll
                for (int v = 0; v < VPT; ++v)
                    xl[v] = (1.0f - gm[v]) * (PRIOR ? a.scale * wv[v] + 0.0f : clipf(Lr[v], L));
                zero_rows();
            } else {
                // the last decision and its weight are the output only when no
                // leg converged; the outputs are stored after the next syndrome
                // has started, so its loads are consumed first
                uint32_t out = 0;
                double w_out = 0.0;
                if (!TRACE) {
                    uint32_t fm = 0;
                    const double Wlast = count > 0 ? best_w : weight_of(wv, fm);
                    out = count > 0 ? best_mask : fm;
                    w_out = count > 0 ? best_w : Wlast;
                    if (a.final_llr) {
#pragma unroll
                        for (int v = 0; v < VPT; ++v) {
                            const int j = (int)gl + G * v;
                            if (j < a.N) a.final_llr[(size_t)shot * a.llr_stride + j] = Lr[v];
                        }
                    }
                }
                const int o_shot = shot;
                const int o_legs = r, o_iters = total;
                const bool o_conv = count > 0;
                if (start) {
                    if (MULTI && a.list_cid)
                        begin(xl, nsig, w0n);
                    else
                        begin(wv, nsig, w0n);
                } else {
                    active = false;
                }
                if (!TRACE) {
                    if (a.io_bits) {
                        // word q of the packed correction holds faults 32q .. 32q+31;
                        // lane g of the slot assembles word g (ceil(N/32) <= G words,
                        // as N <= G * VPT and VPT <= 32) from one ballot per fault
                        // round v, whose slot bits are faults G*v .. G*v+G-1
                        uint32_t word = 0;
#pragma unroll
                        for (int v = 0; v < VPT; ++v) {
                            const unsigned long long bal = __ballot((out >> v) & 1u);
                            const unsigned long long sbits = G == 64 ? bal : (bal >> (slot * G)) & ((1ull << (G % 64)) - 1ull);
                            const int d = G * v - 32 * (int)gl;  // bit of word gl where fault G*v lands
                            if (d > -64 && d < 32) word |= (uint32_t)(d >= 0 ? sbits << d : sbits >> -d);
                        }
                        if ((int)gl * 32 < a.N) reinterpret_cast<uint32_t *>(a.corr)[(size_t)o_shot * a.corr_stride + gl] = word;
                    } else {
#pragma unroll
                        for (int v = 0; v < VPT; ++v) {
                            const int j = (int)gl + G * v;
                            if (j < a.N) a.corr[(size_t)o_shot * a.corr_stride + j] = (uint8_t)((out >> v) & 1u);
                        }
                    }
                    if (g == 0) {
                        a.conv[o_shot] = o_conv ? 1 : 0;
                        a.legs[o_shot] = o_legs;
                        a.iters[o_shot] = o_iters;
                        if (a.weight) a.weight[o_shot] = w_out;
                    }
                }
            }
        }
        wave_sync();

        // ---------------- fault pass: memory term, marginals, Lambda(t+1)
        // (faults in batches of FB, gathers before stores, as in the check pass)
        if (active && !event) {
#pragma unroll
            for (int v0 = 0; v0 < VPT; v0 += FB) {
                float mv[FB][DV];
#pragma unroll
                for (int v = v0; v < v0 + FB && v < VPT; ++v)
#pragma unroll
                    for (int k = 0; k < DV; ++k) mv[v - v0][k] = lds_at<float>(lds, mu_addr(v, k));
#pragma unroll
                for (int v = v0; v < v0 + FB && v < VPT; ++v) {
                    const float y = gm[v] * clipf(Lr[v], L);
                    float acc = clipf(xl[v] + y, L);
#pragma unroll
                    for (int k = 0; k < DV; ++k) acc += mv[v - v0][k];
                    Lr[v] = acc;
                    // columns j >= N of the last row of lanes own spare words of the
                    // padded Lambda region, so the write needs no bound check
                    lds_at<float>(lds, lam_w0 + WORD * G * v) = acc;
                    if (TRACE) {
                        const int j = (int)gl + G * v;
                        if (j < a.N) a.trace[((size_t)shot * (a.trace_T + 1) + t + 1) * a.N + j] = acc;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            ++t;
            ++total;
        }
        wave_sync();
    }
}

template <int G, int CPT, int DC, int VPT, int DV, int WAVES, bool PRIOR, bool TRACE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WAVES)))
void relay_group_kernel(GroupArgs a) {
    group_loop<G, CPT, DC, VPT, DV, PRIOR, TRACE>(a);
}

// ------------------------------------------------------------------------
// Mixed-code launch: each wave decodes one family at a time (the codes that
// share a graph and a tile, e.g. one code at several noise rates) with the
// family's compiled tile, drains the family's queue (one longest-first list
// over all its codes; every slot takes w and gamma from its shot's own code,
// the member index of each list position standing beside the list),
// then moves on to the next family in the order the list kernels set.
// Only tiles within a 128-VGPR budget take part, so mixing never lowers
// occupancy below what the largest code needs on its own.
// ------------------------------------------------------------------------
template <bool PRIOR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
void relay_mixed_kernel(MixedArgs m) {
    for (int q = 0; q < m.nfam; ++q) {
        const int f = m.order[q];
        const CodeStatic cs = m.codes[m.fam_rep[f]];
        GroupArgs a = m.run;
        a.M = cs.M;
        a.N = cs.N;
        a.w = cs.w;
        a.gamma = cs.gamma;
        a.w_uniform = cs.w_uniform;
        a.w0 = cs.w0;
        a.lam_off = cs.lam_off;
        a.mu_off = cs.mu_off;
        a.lampad_off = cs.lampad_off;
        a.mupad_off = cs.mupad_off;
        a.mu0_off = cs.mu0_off;
        a.half_off = cs.half_off;
        a.list = m.list + m.seg_start[f];
        a.list_cid = m.fam_size[f] > 1 ? m.list_cid + m.seg_start[f] : nullptr;
        a.count = m.seg_count[f];
        a.queue = m.queues + (size_t)f * kQueueWords;
        switch (cs.tile) {
            case 0: group_loop<8, 5, 6, 9, 3, PRIOR, false, true>(a); break;
            case 1: group_loop<16, 3, 6, 6, 3, PRIOR, false, true>(a); break;
            case 2: group_loop<16, 5, 6, 9, 3, PRIOR, false, true>(a); break;
            case 3: group_loop<32, 5, 6, 9, 3, PRIOR, false, true>(a); break;
            case 4: group_loop<64, 1, 6, 2, 3, PRIOR, false, true>(a); break;
            case 5: group_loop<64, 2, 6, 3, 3, PRIOR, false, true>(a); break;
            case 6: group_loop<64, 3, 6, 5, 3, PRIOR, false, true>(a); break;
            default: break;
        }
    }
}

// ------------------------------------------------------------------------
// Shot lists: per code, positions sorted by decreasing syndrome weight (a
// longest-first order, so the long-tailed hard syndromes start early and the
// queue ends with short ones).  Counting sort over (code, weight bin).
// ------------------------------------------------------------------------
constexpr int kWeightBins = 256;

__global__ void list_zero_kernel(int32_t *p, int n, unsigned long long *queues, int nq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
    if (i < nq * kQueueSplit) queues[(size_t)(i / kQueueSplit) * kQueueWords + (i % kQueueSplit) * kQueueStride] = 0ull;
}

constexpr int kListThreads = 256;

// Key of shot b: family-major, then decreasing syndrome weight (bin), or -1.
__device__ __forceinline__ int shot_key(int64_t b, const uint8_t *syn, int32_t syn_stride, bool bits,
                                        const int32_t *code_id, const int32_t *code_m, int ncodes,
                                        const int32_t *code_fam) {
    const int c = code_id ? code_id[b] : 0;
    if (c < 0 || c >= ncodes) return -1;  // invalid code id: shot skipped, outputs untouched
    const int m = code_m[c];
    int wgt = 0;
    if (bits) {
        const uint32_t *s = reinterpret_cast<const uint32_t *>(syn) + (size_t)b * syn_stride;
        for (int q = 0; q * 32 < m; ++q) {
            const int left = m - 32 * q;  // bits of word q inside the code's M
            wgt += __popc(left >= 32 ? s[q] : s[q] & ((1u << left) - 1u));
        }
    } else {
        const uint8_t *s = syn + (size_t)b * syn_stride;
        for (int i = 0; i < m; ++i) wgt += s[i] != 0;
    }
    const int f = code_fam ? code_fam[c] : c;
    return f * kWeightBins + (kWeightBins - 1 - min(wgt, kWeightBins - 1));
}

// Block-local histogram in LDS (dynamic LDS: nbins words), then one global
// atomic per nonzero (block, bin).
__global__ __launch_bounds__(kListThreads) void list_key_kernel(
        int64_t B, const uint8_t *syn, int32_t syn_stride, bool bits, const int32_t *code_id,
        const int32_t *code_m, int ncodes, const int32_t *code_fam, int nfam, int32_t *key, int32_t *hist) {
    const int nb = nfam * kWeightBins;
    for (int k = threadIdx.x; k < nb; k += kListThreads) *(__attribute__((address_space(3))) int32_t *)(size_t)(4u * k) = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * kListThreads + threadIdx.x;
    if (b < B) {
        const int k = shot_key(b, syn, syn_stride, bits, code_id, code_m, ncodes, code_fam);
        key[b] = k;
        if (k >= 0)
            __hip_atomic_fetch_add((__attribute__((address_space(3))) int32_t *)(size_t)(4u * k), 1,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += kListThreads) {
        const int n = *(__attribute__((address_space(3))) int32_t *)(size_t)(4u * k);
        if (n) atomicAdd(&hist[k], n);
    }
}

// single thread: exclusive scan of the histogram into positions; per-code
// segment start and length; the order in which every block visits the codes:
// decreasing mean syndrome weight, so the heaviest code's long-running shots
// start first and the launch ends on the lightest code's shortest shots.
__global__ void list_scan_kernel(int ncodes, int32_t *hist, int32_t *seg_start, int32_t *seg_count,
                                 int32_t *order) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int32_t run = 0;
    for (int c = 0; c < ncodes; ++c) {
        seg_start[c] = run;
        double wsum = 0.0;
        for (int k = 0; k < kWeightBins; ++k) {
            const int32_t n = hist[c * kWeightBins + k];
            hist[c * kWeightBins + k] = run;
            run += n;
            wsum += (double)n * (double)(kWeightBins - 1 - k);
        }
        seg_count[c] = run - seg_start[c];
        // 256 x mean weight, held in order[c] until the sort below replaces it
        order[c] = seg_count[c] > 0 ? (int32_t)(256.0 * wsum / seg_count[c]) : -1;
    }
    // stable selection by decreasing mean weight (ncodes is small)
    int32_t key[64], idx[64];
    const int n = ncodes < 64 ? ncodes : 64;
    for (int c = 0; c < n; ++c) {
        key[c] = order[c];
        idx[c] = c;
    }
    for (int a = 0; a < n; ++a) {
        int best = a;
        for (int b = a + 1; b < n; ++b)
            if (key[b] > key[best]) best = b;
        const int32_t tk = key[best], ti = idx[best];
        for (int b = best; b > a; --b) {
            key[b] = key[b - 1];
            idx[b] = idx[b - 1];
        }
        key[a] = tk;
        idx[a] = ti;
    }
    for (int c = 0; c < ncodes; ++c) order[c] = c < n ? idx[c] : c;
}

// Each block reserves one contiguous range per nonzero (block, bin) and
// places its shots inside it (order within a bin is irrelevant: every shot's
// result depends on its own syndrome only); with code_member, also the
// family member of each placed shot's code.
__global__ __launch_bounds__(kListThreads) void list_scatter_kernel(int64_t B, int nb, const int32_t *key,
                                                                    int32_t *pos, int32_t *list,
                                                                    const int32_t *code_id,
                                                                    const int32_t *code_member,
                                                                    int32_t *list_cid) {
    // LDS: count[nb], then base[nb]
    const uint32_t cnt0 = 0u, base0 = 4u * (uint32_t)nb;
    for (int k = threadIdx.x; k < nb; k += kListThreads) *(__attribute__((address_space(3))) int32_t *)(size_t)(cnt0 + 4u * k) = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * kListThreads + threadIdx.x;
    int k = -1, local = 0;
    if (b < B) {
        k = key[b];
        if (k >= 0)
            local = __hip_atomic_fetch_add((__attribute__((address_space(3))) int32_t *)(size_t)(cnt0 + 4u * k), 1,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nb; q += kListThreads) {
        const int n = *(__attribute__((address_space(3))) int32_t *)(size_t)(cnt0 + 4u * q);
        *(__attribute__((address_space(3))) int32_t *)(size_t)(base0 + 4u * q) = n ? atomicAdd(&pos[q], n) : 0;
    }
    __syncthreads();
    if (k >= 0) {
        const int32_t p = *(__attribute__((address_space(3))) int32_t *)(size_t)(base0 + 4u * k) + local;
        list[p] = (int32_t)b;
        if (list_cid) list_cid[p] = code_member[code_id[b]];
    }
}

// ------------------------------------------------------------------------
// Configuration table
// ------------------------------------------------------------------------
struct Variant {
    TileShape shape;
    const void *fn[2][2];  // [prior][trace]
};

#define RB_VARIANT(G, CPT, DC, VPT, DV, W)                                                  \
    {{G, CPT, DC, VPT, DV, W},                                                              \
     {{(const void *)relay_group_kernel<G, CPT, DC, VPT, DV, W, false, false>,              \
       (const void *)relay_group_kernel<G, CPT, DC, VPT, DV, W, false, true>},              \
      {(const void *)relay_group_kernel<G, CPT, DC, VPT, DV, W, true, false>,               \
       (const void *)relay_group_kernel<G, CPT, DC, VPT, DV, W, true, true>}}}

// (G, CPT, DC, VPT, DV, waves per SIMD the register budget targets)
const Variant kVariants[] = {
    // regular degree-(6, 3) graphs: bivariate-bicycle check matrices
    RB_VARIANT(4, 9, 6, 18, 3, 2),    // M <= 36,  N <= 72
    RB_VARIANT(8, 5, 6, 9, 3, 4),     // M <= 40,  N <= 72
    RB_VARIANT(8, 6, 6, 12, 3, 3),    // M <= 48,  N <= 96
    RB_VARIANT(16, 3, 6, 6, 3, 4),    // M <= 48,  N <= 96
    RB_VARIANT(8, 9, 6, 18, 3, 2),    // M <= 72,  N <= 144
    RB_VARIANT(16, 5, 6, 9, 3, 4),    // M <= 80,  N <= 144
    RB_VARIANT(16, 5, 6, 9, 3, 3),    // M <= 80,  N <= 144
    RB_VARIANT(16, 9, 6, 18, 3, 2),   // M <= 144, N <= 288
    RB_VARIANT(32, 5, 6, 9, 3, 4),    // M <= 160, N <= 288
    // irregular small graphs
    RB_VARIANT(16, 4, 16, 8, 8, 2),   // M <= 64,  N <= 128
    RB_VARIANT(64, 4, 16, 8, 8, 2),   // M <= 256, N <= 512
    // degree-(6, 3) graphs, one syndrome per wave: the shortest iteration for
    // a single syndrome (fewest checks and faults per lane), at more
    // lane-operations per edge than the tiles above; the choice for codes
    // whose launch time is set by a few long-running syndromes
    RB_VARIANT(64, 1, 6, 2, 3, 4),    // M <= 64,  N <= 128
    RB_VARIANT(64, 2, 6, 3, 3, 4),    // M <= 128, N <= 192
    RB_VARIANT(64, 3, 6, 5, 3, 4),    // M <= 192, N <= 320
};

// ------------------------------------------------------------------------
// Syndrome of a batch of corrections (decoding problem of Sec. 2.1: sigma =
// H F over F_2), optionally XORed into a given syndrome: out[b][i] = in[b][i]
// XOR parity of corr[b][j] over the row of check i.  One thread per (shot,
// check); a wave's lanes take consecutive checks of one shot.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void syndrome_kernel(int64_t B, int32_t M, int32_t N, const int32_t *rowptr,
                                                       const int32_t *colidx, const uint8_t *corr,
                                                       const uint8_t *syn_in, uint8_t *syn_out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * (int64_t)M) return;
    const int64_t b = idx / M;
    const int i = (int)(idx % M);
    const uint8_t *f = corr + (size_t)b * N;
    uint32_t par = syn_in ? (syn_in[idx] != 0 ? 1u : 0u) : 0u;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) par ^= f[colidx[e]] != 0 ? 1u : 0u;
    syn_out[idx] = (uint8_t)par;
}

// The same on bit-packed rows: one thread per (shot, syndrome word), the 32
// checks of word q (bits past M are written as 0).
__global__ __launch_bounds__(256) void syndrome_bits_kernel(int64_t B, int32_t M, int32_t N, const int32_t *rowptr,
                                                            const int32_t *colidx, const uint32_t *corr,
                                                            const uint32_t *syn_in, uint32_t *syn_out) {
    const int32_t WM = (M + 31) / 32, WN = (N + 31) / 32;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * (int64_t)WM) return;
    const int64_t b = idx / WM;
    const int q = (int)(idx % WM);
    const uint32_t *f = corr + (size_t)b * WN;
    uint32_t word = 0;
    for (int k = 0; k < 32 && 32 * q + k < M; ++k) {
        const int i = 32 * q + k;
        uint32_t par = 0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) par ^= (f[colidx[e] >> 5] >> (colidx[e] & 31)) & 1u;
        word |= par << k;
    }
    if (syn_in) word ^= syn_in[idx] & (32 * q + 32 <= M ? 0xffffffffu : (1u << (M - 32 * q)) - 1u);
    syn_out[idx] = word;
}

}  // namespace

int num_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

// group variants usable in the mixed launch, in the order of its tile switch
const int kMixedVariants[] = {1, 3, 5, 8, 11, 12, 13};

int mixed_tile_of_variant(int v) {
    for (int t = 0; t < (int)(sizeof(kMixedVariants) / sizeof(kMixedVariants[0])); ++t)
        if (kMixedVariants[t] == v) return t;
    return -1;
}

hipError_t mixed_occupancy(bool prior_anchor, size_t lds, int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, prior_anchor ? (const void *)relay_mixed_kernel<true> : (const void *)relay_mixed_kernel<false>,
        64, lds);
}

hipError_t launch_mixed(bool prior_anchor, const MixedArgs &m, int grid, size_t lds, hipStream_t s) {
    const void *fn = prior_anchor ? (const void *)relay_mixed_kernel<true> : (const void *)relay_mixed_kernel<false>;
    MixedArgs copy = m;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(64), args, lds, s);
}

TileShape variant_shape(int v) { return kVariants[v].shape; }

hipError_t variant_static_lds(int v, size_t *bytes) {
    size_t mx = 0;
    for (int p = 0; p < 2; ++p)
        for (int tr = 0; tr < 2; ++tr) {
            hipFuncAttributes attr;
            const hipError_t e = hipFuncGetAttributes(&attr, kVariants[v].fn[p][tr]);
            if (e != hipSuccess) return e;
            if ((size_t)attr.sharedSizeBytes > mx) mx = (size_t)attr.sharedSizeBytes;
        }
    for (int p = 0; p < 2; ++p) {
        hipFuncAttributes attr;
        const hipError_t e = hipFuncGetAttributes(
            &attr, p ? (const void *)relay_mixed_kernel<true> : (const void *)relay_mixed_kernel<false>);
        if (e != hipSuccess) return e;
        if ((size_t)attr.sharedSizeBytes > mx) mx = (size_t)attr.sharedSizeBytes;
    }
    *bytes = mx;
    return hipSuccess;
}

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

hipError_t launch_shot_lists(int64_t B, const uint8_t *syn, int32_t syn_stride, bool bits, const int32_t *code_id,
                             const int32_t *code_m, int ncodes, const int32_t *code_fam, int nfam,
                             const int32_t *code_member, void *workspace, unsigned long long *queues,
                             hipStream_t s) {
    int32_t *hist = (int32_t *)workspace;                       // ncodes * bins
    int32_t *seg_start = hist + (size_t)ncodes * kWeightBins;   // ncodes
    int32_t *seg_count = seg_start + ncodes;                    // ncodes
    int32_t *order = seg_count + ncodes;                        // ncodes
    int32_t *key = order + ncodes;                              // B
    int32_t *list = key + B;                                    // B
    int32_t *list_cid = list + B;                               // B (written with code_member)
    const int nh = nfam * kWeightBins;
    hipLaunchKernelGGL(list_zero_kernel, dim3((nh + 255) / 256), dim3(256), 0, s, hist, nh, queues, nfam);
    const int blocks = (int)((B + kListThreads - 1) / kListThreads);
    hipLaunchKernelGGL(list_key_kernel, dim3(blocks), dim3(kListThreads), 4u * (size_t)nh, s, B, syn, syn_stride,
                       bits, code_id, code_m, ncodes, code_fam, nfam, key, hist);
    hipLaunchKernelGGL(list_scan_kernel, dim3(1), dim3(64), 0, s, nfam, hist, seg_start, seg_count, order);
    hipLaunchKernelGGL(list_scatter_kernel, dim3(blocks), dim3(kListThreads), 8u * (size_t)nh, s, B, nh, key, hist,
                       list, code_id, code_member, code_member ? list_cid : nullptr);
    return hipGetLastError();
}

size_t shot_list_bytes(int64_t B, int ncodes) {
    return sizeof(int32_t) * ((size_t)ncodes * (kWeightBins + 3) + 3 * (size_t)B);
}

hipError_t launch_syndrome(int64_t B, int32_t M, int32_t N, const int32_t *rowptr, const int32_t *colidx,
                           const uint8_t *corr, const uint8_t *syn_in, uint8_t *syn_out, bool bits,
                           hipStream_t s) {
    if (bits) {
        const int64_t n = B * (int64_t)((M + 31) / 32);
        if (n == 0) return hipSuccess;
        hipLaunchKernelGGL(syndrome_bits_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, M, N, rowptr,
                           colidx, reinterpret_cast<const uint32_t *>(corr),
                           reinterpret_cast<const uint32_t *>(syn_in), reinterpret_cast<uint32_t *>(syn_out));
        return hipGetLastError();
    }
    const int64_t n = B * (int64_t)M;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(syndrome_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, M, N, rowptr, colidx,
                       corr, syn_in, syn_out);
    return hipGetLastError();
}

hipError_t launch_reset_queue(unsigned long long *q, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(kQueueSplit), 0, s, q);
    return hipGetLastError();
}

}  // namespace rb

// ------------------------------------------------------------------------
// Static scratch of rb_decode_multi_noalloc: the mixed launch's queue
// counters and shot lists, for callers that cannot allocate.  Every GPU the
// library runs on holds its own copy for the life of the process; all calls
// on one GPU share it.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol): it uses the device
// address looked up below, once per device.
// ------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[rb::kNoAllocScratchBytes];

namespace rb {

hipError_t noalloc_scratch(int device, void **ptr) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace rb
