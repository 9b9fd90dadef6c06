// relay_block16.hip -- Relay-BP with binary16 messages, two syndromes per
// workgroup (gfx950).
//
// The decoder of relay_block.hip (paper Sec. 2.3: DMem-BP legs, Relay
// chaining, S solutions) with every per-shot quantity -- Lambda, lambda(0),
// the memory term, nu and mu -- held as IEEE binary16 and every arithmetic
// result rounded to binary16 (nearest even).  The paper leaves the precision
// of Relay's messages open; on this GPU a 16-bit message pays only if one
// instruction serves two of them, so a workgroup decodes two syndromes at
// once, shot slot 0 in the low half and slot 1 in the high half of every LDS
// word and of every register that holds a message, a marginal or a memory
// term.  Each packed instruction (v_pk_add_f16, v_pk_mul_f16, v_pk_min_u16,
// ...) then advances both syndromes, and each LDS access moves both.
//
// Same graph tables, roles and LDS plan as the FP32 block kernel (one check
// row segment and VPT fault slots per thread, wave-ELL message rows), with
// these differences:
//  - Check pass: pass 1 forms d = Lambda - mu (one packed subtraction), keeps
//    the two smallest |nu| = min(|d|, L) per half with packed unsigned 16-bit
//    min / max (non-negative binary16 values order like their bit patterns),
//    XORs the words for the sign parity (bits 15 and 31) and stores nu = sign
//    | |nu| in the edge's message word.  Pass 2 reads nu back and writes
//    mu = (sign(nu) xor P) | (|nu| == m1 ? m2 : m1), the min over the other
//    edges: when the minimum is tied, m2 = m1, so no position is tracked.
//  - The parity of F over a row XORs the marginal words: F_j = 1 iff
//    Lambda_j < 0, and Lambda is never -0 (lambda starts at w >= +0, and a
//    sum of a value and its negation rounds to +0), so the sign bit is F.
//  - The two halves run their own legs and shots; a convergence or leg event
//    of one half restarts only that half (its message halves are cleared
//    with 16-bit stores, its marginal half reset or kept) while the other
//    half's fault pass proceeds, with the event half's marginals held by a
//    per-half select.
//  - Packed corrections (RB_IO_BITS32) are assembled in an LDS region of
//    their own, as the marginal words still hold the other half's shot.

#include <algorithm>
#include <type_traits>

#include "relay_device.h"
#include "relay_internal.h"

namespace rb {
namespace {

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef unsigned short u2_t __attribute__((ext_vector_type(2)));

constexpr uint32_t kSign = 0x80008000u;
constexpr uint32_t kMag = 0x7FFF7FFFu;

__device__ __forceinline__ h2_t as_h2(uint32_t x) { return __builtin_bit_cast(h2_t, x); }
__device__ __forceinline__ u2_t as_u2(uint32_t x) { return __builtin_bit_cast(u2_t, x); }
__device__ __forceinline__ uint32_t bits(h2_t x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t bits(u2_t x) { return __builtin_bit_cast(uint32_t, x); }

// packed unsigned 16-bit min / max (v_pk_min_u16, v_pk_max_u16)
__device__ __forceinline__ uint32_t umin2(uint32_t a, uint32_t b) {
    return bits(__builtin_elementwise_min(as_u2(a), as_u2(b)));
}
__device__ __forceinline__ uint32_t umax2(uint32_t a, uint32_t b) {
    return bits(__builtin_elementwise_max(as_u2(a), as_u2(b)));
}

// clip to [-L, L] of a packed binary16 word, by magnitude: min(|x|, L) with
// the sign of x (exact; infinities clip to L)
__device__ __forceinline__ uint32_t clip_bits(uint32_t x, uint32_t L2) { return (x & kSign) | umin2(x & kMag, L2); }

__device__ __forceinline__ void opaque16(uint32_t &x) { asm volatile("" : "+v"(x)); }

// A 64-bit value that is the same in every lane, moved to scalar registers
// (readfirstlane of each half; its result is a signed int, so each half is
// widened as unsigned)
__device__ __forceinline__ unsigned long long uniform64(unsigned long long x) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    return ((unsigned long long)hi << 32) | (unsigned long long)lo;
}

// Message magnitude of pass 2 for both halves, (|nu| == m1 ? m2 : m1), as
// e = min(|nu| - m1, 1) (0 iff equal, as |nu| >= m1) and e * (m1 - m2) + m2
// (mod 2^16): three packed integer instructions, written out so that the
// compiler does not turn them into per-half compares and selects.
__device__ __forceinline__ uint32_t pass2_mag(uint32_t anu, uint32_t m1, uint32_t m2, uint32_t dm) {
    uint32_t e, r;
    asm("v_pk_sub_u16 %0, %2, %3\n\t"
        "v_pk_min_u16 %0, %0, %6\n\t"
        "v_pk_mad_u16 %1, %0, %4, %5"
        : "=&v"(e), "=&v"(r)
        : "v"(anu), "v"(m1), "v"(dm), "v"(m2), "s"(0x00010001u));
    return r;
}

__device__ __forceinline__ uint32_t lo_half_x4_16(uint32_t x) {
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(r)
        : "v"(2u), "v"(x));
    return r;
}

__device__ __forceinline__ int swap_pair16(int x) { return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false); }

// OR over the block of two predicates (bit 0 and bit 1 of the result); one
// barrier, the caller guarantees another before the next call (as block_or)
template <int TPB>
__device__ __forceinline__ uint32_t block_or2(bool p0, bool p1, uint32_t flags) {
    const bool a0 = __any(p0), a1 = __any(p1);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds_b<uint8_t>(flags + (uint32_t)wave) = (a0 ? 1 : 0) | (a1 ? 2 : 0);
    __syncthreads();
    uint32_t acc = 0;
#pragma unroll
    for (int q = 0; q < TPB / 256; ++q) acc |= lds_b<uint32_t>(flags + 4u * (uint32_t)q);
    return ((acc & 0x01010101u) ? 1u : 0u) | ((acc & 0x02020202u) ? 2u : 0u);
}

template <int TPB, int DCMAX, int VPT, uint64_t PROF, int WAVES, bool PRIOR, bool TRACE>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(WAVES)))
void relay_block16_kernel(BlockArgs a) {
    constexpr int CH = kBlockChunk;
    constexpr int NMU = prof_pre(PROF, VPT);
    constexpr int DV = prof_max(PROF, VPT);
    constexpr int NPAD = TPB * VPT;
    static_assert(TPB % 128 == 0 && CH == 8 && DCMAX % CH == 0 && DCMAX <= 64 && DV >= 1, "shape");
    const uint32_t red = a.red_off;
    const uint32_t flags = a.red_off + 8u * (TPB / 64);
    const uint32_t shot_sh = flags + 4u * (TPB / 64);  // claimed shot index (8 bytes)
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const uint32_t L2 = a.L16 | (a.L16 << 16);
    const h2_t Lh = as_h2(L2);
    uint32_t tl = (uint32_t)t;

    const uint4 *ctab = reinterpret_cast<const uint4 *>(a.chk_col);
    uint4 col0 = ctab[t];
    uint32_t mu_pk[(NMU + 1) / 2];
#pragma unroll
    for (int e = 0; e < (NMU + 1) / 2; ++e) mu_pk[e] = a.col_mu[(size_t)e * TPB + t];
    const int myrow = a.chk_row[t];
    const bool split = a.chk_split[t] != 0;
    int wdeg = __builtin_amdgcn_readfirstlane(a.wave_deg[wave]);
    const uint32_t mrow = a.mu0_off + 4u * ((uint32_t)a.wave_base[wave] + (uint32_t)(t & 63));

    if (t == 0) {
        lds_b<uint32_t>(a.lampad_off) = 0x7C007C00u;  // (+inf, +inf)
        lds_b<uint32_t>(a.mupad_off) = 0x80008000u;   // (-0, -0)
    }
    if (t < TPB / 256) lds_b<uint32_t>(flags + 4u * (uint32_t)t) = 0u;
    for (int q = t; q < (CH - 1) * 64; q += TPB) lds_b<uint32_t>(a.slack_off + 4u * q) = 0u;

    // per-thread fault state, both halves packed: xl = (1 - gamma) lambda(0)
    // (fixed within a leg) and gamma
    uint32_t xl[VPT], gm[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) xl[v] = gm[v] = 0u;
    uint32_t sigw = 0;     // syndrome bit of myrow of each half at bit 15 / 31
    uint32_t bm[2] = {0u, 0u};
    double best_w[2] = {0.0, 0.0};
    long long shot[2] = {-1, -1};
    int r[2] = {0, 0}, tt[2] = {0, 0}, total[2] = {0, 0}, count[2] = {0, 0};
    bool act[2] = {false, false};

    auto half_mask = [](int h) -> uint32_t { return h ? 0xFFFF0000u : 0x0000FFFFu; };

    // clear half h of this thread's message words (16-bit stores)
    auto zero_row_half = [&](int h) {
        for (int k = 0; k < wdeg; ++k) lds_b<uint16_t>(mrow + 256u * k + 2u * (uint32_t)h) = (uint16_t)0;
    };

    // xl of half h from its anchor lambda(0) (packed words, half h used)
    auto set_leg = [&](int h, int v, uint32_t g16w, uint32_t lam0w) {
        const uint32_t hm = half_mask(h);
        const h2_t om = as_h2(0x3C003C00u) - as_h2(g16w);  // 1 - gamma
        const uint32_t x = bits(om * as_h2(lam0w));
        xl[v] = (xl[v] & ~hm) | (x & hm);
        gm[v] = (gm[v] & ~hm) | (g16w & hm);
    };

    // claim the next syndrome for half h and start its leg 1
    auto fetch = [&](int h) -> bool {
        if (t == 0) lds_b<unsigned long long>(shot_sh) = atomicAdd(a.queue, 1ull);
        __syncthreads();
        const unsigned long long nxt = lds_b<unsigned long long>(shot_sh);
        __syncthreads();
        if (nxt >= (unsigned long long)a.B) {
            act[h] = false;
            return false;
        }
        act[h] = true;
        shot[h] = (long long)uniform64(nxt);
        r[h] = 1;
        tt[h] = 0;
        total[h] = 0;
        count[h] = 0;
        best_w[h] = __longlong_as_double(0x7ff0000000000000ll);
        bm[h] = 0;
        const bool sb = myrow >= 0 && syn_bit(a.syn, (size_t)shot[h], a.syn_stride, myrow, a.io_bits);
        sigw = (sigw & ~(0x8000u << (16 * h))) | ((sb ? 0x8000u : 0u) << (16 * h));
        uint32_t w16[VPT], g16[VPT];
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const uint32_t sl = tl + TPB * v;
            w16[v] = a.w16_slot[sl];
            if (TRACE) {
                const int j = a.slot_col[sl];
                const _Float16 gh = (_Float16)(j >= 0 ? a.trace_gamma[j] : 0.0f);
                g16[v] = __builtin_bit_cast(uint16_t, gh);
            } else {
                g16[v] = a.gamma16_slot[sl];
            }
        }
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const uint32_t sl = tl + TPB * v;
            lds_b<uint16_t>(4u * sl + 2u * (uint32_t)h) = (uint16_t)w16[v];
            set_leg(h, v, g16[v] * 0x10001u, w16[v] * 0x10001u);
            if (TRACE) {
                const int j = a.slot_col[sl];
                if (j >= 0)
                    a.trace[(size_t)shot[h] * (a.trace_T + 1) * a.N + j] =
                        (float)__builtin_bit_cast(_Float16, (uint16_t)w16[v]);
            }
        }
        zero_row_half(h);
        return true;
    };

#pragma unroll
    for (int v = 0; v < VPT; ++v) lds_b<uint32_t>(4u * (tl + TPB * v)) = 0u;
    for (int k = 0; k < wdeg; ++k) lds_b<uint32_t>(mrow + 256u * k) = 0u;
    fetch(0);
    fetch(1);
    __syncthreads();

    while (act[0] || act[1]) {
        opaque16(col0.x);
        opaque16(col0.y);
        opaque16(col0.z);
        opaque16(col0.w);
#pragma unroll
        for (int e = 0; e < (NMU + 1) / 2; ++e) opaque16(mu_pk[e]);
        opaque16(tl);
        asm volatile("" : "+s"(wdeg));

        // ---------------- check pass, both halves
        uint32_t fparw = sigw, negw = sigw;
        uint32_t m1 = L2, m2 = L2;
        auto chunk = [&](auto w_tag, int c, const uint4 &tb) {
            constexpr int W = decltype(w_tag)::value;
            const uint32_t pk[4] = {tb.x, tb.y, tb.z, tb.w};
            uint32_t lv[W], mo[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const uint32_t ca = (q & 1) ? (pk[q >> 1] >> 16) : (pk[q >> 1] & 0xffffu);
                lv[q] = lds_b<uint32_t>(ca);
                mo[q] = lds_b<uint32_t>(mrow + 256u * (c + q));
            }
            uint32_t dprev = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int k = c + q;
                // parities two edges per three-input XOR (W is even)
                if (q & 1) fparw = xor3(fparw, lv[q - 1], lv[q]);
                const uint32_t d = bits(as_h2(lv[q]) - as_h2(mo[q]));
                if (q & 1) negw = xor3(negw, dprev, d);
                dprev = d;
                const uint32_t av = umin2(d & kMag, L2);
                m2 = umin2(m2, umax2(m1, av));
                m1 = umin2(m1, av);
                if (k < wdeg) lds_b<uint32_t>(mrow + 256u * k) = (d & kSign) | av;  // nu, for pass 2
            }
        };
        uint4 cur = col0;
#pragma unroll
        for (int c = 0; c < DCMAX; c += CH) {
            if (c >= wdeg) break;
            const uint4 nxt = ctab[(size_t)(c / CH + 1) * TPB + tl];
            if (c + CH / 2 >= wdeg)
                chunk(std::integral_constant<int, CH / 2>{}, c, cur);
            else
                chunk(std::integral_constant<int, CH>{}, c, cur);
            cur = nxt;
        }
        {
            const uint32_t m1o = (uint32_t)swap_pair16((int)m1);
            const uint32_t m2o = (uint32_t)swap_pair16((int)m2);
            const uint32_t no = (uint32_t)swap_pair16((int)negw);
            const uint32_t fo = (uint32_t)swap_pair16((int)fparw);
            if (split) {
                m2 = umin2(umax2(m1, m1o), umin2(m2, m2o));
                m1 = umin2(m1, m1o);
                negw ^= no;
                fparw ^= fo;
            }
        }
        // pass 2: mu = (sign(nu) xor P) | (|nu| == m1 ? m2 : m1) with
        // e = min(|nu| - m1, 1) (0 iff equal) and mag = e * (m1 - m2) + m2
        {
            const uint32_t P = negw & kSign;
            const u2_t dm = as_u2(m1) - as_u2(m2);
            for (int k = 0; k < wdeg; ++k) {
                const uint32_t nw = lds_b<uint32_t>(mrow + 256u * k);
                const uint32_t mag = pass2_mag(nw & kMag, m1, m2, bits(dm));
                lds_b<uint32_t>(mrow + 256u * k) = ((nw ^ P) & kSign) | mag;
            }
        }
        const uint32_t uns = block_or2<TPB>((fparw & 0x8000u) != 0, (fparw & 0x80000000u) != 0, flags);

        // ---------------- leg scheduler, per half (block-uniform)
        bool ev[2] = {false, false};
        bool conv_ev[2] = {false, false};
        bool cut[2] = {false, false};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!act[h]) continue;
            cut[h] = a.max_total_iters > 0 && total[h] >= a.max_total_iters;
            conv_ev[h] = !TRACE && tt[h] >= 1 && !((uns >> h) & 1u);
            const int T_r = TRACE ? a.trace_T : (r[h] == 1 ? a.iters_first : a.iters_leg);
            ev[h] = conv_ev[h] || tt[h] >= T_r || (!TRACE && cut[h]);
        }
        // halves whose fault pass runs this trip (decided before the events)
        const bool upd[2] = {act[0] && !ev[0], act[1] && !ev[1]};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!ev[h]) continue;
            bool done = true;
            if (!TRACE) {
                float wv[VPT];
#pragma unroll
                for (int v = 0; v < VPT; ++v) wv[v] = a.w_slot[tl + TPB * v];
                uint32_t fm = 0;
                double part = 0.0;
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    const uint32_t sl = tl + TPB * v;
                    const bool f = sl < (uint32_t)a.N && ((lds_b<uint32_t>(4u * sl) >> (15 + 16 * h)) & 1u);
                    fm |= f ? 1u << v : 0u;
                    part += (double)(f ? wv[v] : 0.0f);
                }
                const double Wv = block_sum<TPB>(part, red);
                // block-uniform: kept in scalar registers
                const double W = __longlong_as_double((long long)uniform64((unsigned long long)__double_as_longlong(Wv)));
                if (conv_ev[h]) {
                    ++count[h];
                    if (W < best_w[h]) {
                        best_w[h] = W;
                        bm[h] = fm;
                    }
                    done = count[h] >= a.num_solutions || r[h] >= a.num_legs || cut[h];
                } else {
                    done = r[h] >= a.num_legs || cut[h];
                }
                if (done) {
                    const long long s = shot[h];
                    const uint32_t out = count[h] > 0 ? bm[h] : fm;
                    int jv[VPT];
#pragma unroll
                    for (int v = 0; v < VPT; ++v) jv[v] = a.slot_col[tl + TPB * v];
#pragma unroll
                    for (int v = 0; v < VPT; ++v) {
                        const int j = jv[v];
                        if (j >= 0) {
                            if (!a.io_bits) a.corr[(size_t)s * a.corr_stride + j] = (uint8_t)((out >> v) & 1u);
                            if (a.final_llr) {
                                const uint32_t wl = lds_b<uint32_t>(4u * (tl + TPB * v));
                                a.final_llr[(size_t)s * a.N + j] =
                                    (float)__builtin_bit_cast(_Float16, (uint16_t)(wl >> (16 * h)));
                            }
                        }
                    }
                    if (a.io_bits) {
                        const int nw = (a.N + 31) >> 5;
                        for (int q = t; q < nw; q += TPB) lds_b<uint32_t>(a.stage_off + 4u * (uint32_t)q) = 0u;
                        __syncthreads();
#pragma unroll
                        for (int v = 0; v < VPT; ++v) {
                            const int j = jv[v];
                            if (j >= 0 && ((out >> v) & 1u))
                                __hip_atomic_fetch_or(&lds_b<uint32_t>(a.stage_off + 4u * (uint32_t)(j >> 5)),
                                                      1u << (j & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        __syncthreads();
                        uint32_t *c32 = reinterpret_cast<uint32_t *>(a.corr) + (size_t)s * a.corr_stride;
                        for (int q = t; q < nw; q += TPB) c32[q] = lds_b<uint32_t>(a.stage_off + 4u * (uint32_t)q);
                    }
                    if (t == 0) {
                        a.conv[s] = count[h] > 0 ? 1 : 0;
                        a.legs[s] = r[h];
                        a.iters[s] = total[h];
                        if (a.weight) a.weight[s] = count[h] > 0 ? best_w[h] : W;
                    }
                }
            }
            if (!done) {
                ++r[h];
                tt[h] = 0;
                const uint16_t *gr = a.gamma16_slot + (size_t)(r[h] - 1) * NPAD;
                uint32_t gv[VPT], w0[VPT];
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    gv[v] = gr[tl + TPB * v];
                    w0[v] = PRIOR ? a.w16_slot[tl + TPB * v] : 0u;
                }
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    const uint32_t sl = tl + TPB * v;
                    const uint32_t l0 = PRIOR ? w0[v] * 0x10001u : clip_bits(lds_b<uint32_t>(4u * sl), L2);
                    set_leg(h, v, gv[v] * 0x10001u, PRIOR ? l0 : ((l0 >> (16 * h)) & 0xFFFFu) * 0x10001u);
                }
                zero_row_half(h);
            } else {
                fetch(h);
            }
        }
        if (!upd[0] && !upd[1]) {
            __syncthreads();
            continue;
        }

        // ---------------- fault pass for the halves without an event
        const uint32_t keep = (upd[0] ? 0u : 0x0000FFFFu) | (upd[1] ? 0u : 0xFFFF0000u);
        constexpr int FD = 1;
        auto mu_word = [&](int e) -> uint32_t {
            if (e & 1) return (mu_pk[e >> 1] >> 16) << 2;
            return lo_half_x4_16(mu_pk[e >> 1]);
        };
        uint32_t gvv[FD + 1][DV], glv[FD + 1];
        auto load_slot = [&](int v, uint32_t(&m)[DV], uint32_t &l) {
#pragma unroll
            for (int k = 0; k < prof_dv(PROF, v); ++k) m[k] = lds_b<uint32_t>(mu_word(prof_pre(PROF, v) + k));
            l = lds_b<uint32_t>(4u * (tl + TPB * v));
        };
#pragma unroll
        for (int v = 0; v < FD && v < VPT; ++v) load_slot(v, gvv[v], glv[v]);
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            if (v + FD < VPT) load_slot(v + FD, gvv[(v + FD) % (FD + 1)], glv[(v + FD) % (FD + 1)]);
            const uint32_t(&mv)[DV] = gvv[v % (FD + 1)];
            const uint32_t lold = glv[v % (FD + 1)];
            const h2_t y = as_h2(gm[v]) * as_h2(clip_bits(lold, L2));
            const h2_t s = as_h2(xl[v]) + y;
            h2_t acc = __builtin_elementwise_min(__builtin_elementwise_max(s, -Lh), Lh);
#pragma unroll
            for (int k = 0; k < prof_dv(PROF, v); ++k) acc = acc + as_h2(mv[k]);
            const uint32_t nw = (bits(acc) & ~keep) | (lold & keep);
            lds_b<uint32_t>(4u * (tl + TPB * v)) = nw;
            if (TRACE) {
                const int j = a.slot_col[tl + TPB * v];
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (j >= 0 && upd[h])
                        a.trace[((size_t)shot[h] * (a.trace_T + 1) + tt[h] + 1) * a.N + j] =
                            (float)__builtin_bit_cast(_Float16, (uint16_t)(nw >> (16 * h)));
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (upd[h]) {
                ++tt[h];
                ++total[h];
            }
        __syncthreads();
    }
}

__global__ void to_half_kernel(const float *src, int64_t n, uint16_t *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = __builtin_bit_cast(uint16_t, (_Float16)src[i]);  // v_cvt_f16_f32: nearest even
}

struct Block16Variant {
    BlockShape shape;
    const void *fn[2][2];
};

#define RB_B16VARIANT(TPB, DCMAX, VPT, PROF, W)                                                  \
    {{TPB, DCMAX, VPT, PROF, W},                                                                 \
     {{(const void *)relay_block16_kernel<TPB, DCMAX, VPT, PROF, W, false, false>,               \
       (const void *)relay_block16_kernel<TPB, DCMAX, VPT, PROF, W, false, true>},               \
      {(const void *)relay_block16_kernel<TPB, DCMAX, VPT, PROF, W, true, false>,                \
       (const void *)relay_block16_kernel<TPB, DCMAX, VPT, PROF, W, true, true>}}}

// the shapes of the FP32 block variants, in the same order (checked by the host)
const Block16Variant kBlock16Variants[] = {
    RB_B16VARIANT(512, 64, 9, 0x222333456ull, 4),
    RB_B16VARIANT(1024, 64, 9, 0x222333456ull, 4),
    RB_B16VARIANT(1024, 64, 9, 0x223334566ull, 4),
    RB_B16VARIANT(1024, 64, 9, 0x666666666ull, 4),
    RB_B16VARIANT(1024, 32, 4, 0x8888ull, 4),
    RB_B16VARIANT(512, 32, 4, 0x8888ull, 2),
};

}  // namespace

int num_block16_variants() { return (int)(sizeof(kBlock16Variants) / sizeof(kBlock16Variants[0])); }

BlockShape block16_variant_shape(int v) { return kBlock16Variants[v].shape; }

hipError_t block16_variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, kBlock16Variants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0], kBlock16Variants[v].shape.TPB, lds);
}

hipError_t block16_static_lds(int v, size_t *bytes) {
    size_t mx = 0;
    for (int p = 0; p < 2; ++p)
        for (int tr = 0; tr < 2; ++tr) {
            hipFuncAttributes attr;
            const hipError_t e = hipFuncGetAttributes(&attr, kBlock16Variants[v].fn[p][tr]);
            if (e != hipSuccess) return e;
            mx = std::max(mx, (size_t)attr.sharedSizeBytes);
        }
    *bytes = mx;
    return hipSuccess;
}

hipError_t block16_prepare(int v, size_t lds) {
    for (int p = 0; p < 2; ++p)
        for (int tr = 0; tr < 2; ++tr) {
            hipError_t e = hipFuncSetAttribute(kBlock16Variants[v].fn[p][tr],
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

hipError_t launch_block16(int v, bool prior_anchor, bool trace, const BlockArgs &a, int grid, size_t lds,
                          hipStream_t s) {
    const void *fn = kBlock16Variants[v].fn[prior_anchor ? 1 : 0][trace ? 1 : 0];
    BlockArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock16Variants[v].shape.TPB), args, lds, s);
}

hipError_t launch_to_half(const float *src, int64_t n, uint16_t *dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(to_half_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, n, dst);
    return hipGetLastError();
}

}  // namespace rb
