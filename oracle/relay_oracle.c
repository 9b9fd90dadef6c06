/*
 * relay_oracle.c -- plain, slow CPU oracle for Relay-BP decoding.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the reference the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or table with the GPU
 * library, and it includes nothing from it.
 *
 * What it computes (paper Sec. 2.3, "Message passing decoding"):
 *   - Relay decoding: legs of Disordered-Memory BP (DMem-BP).  Initialisation
 *     nu(0) = lambda(0) = Lambda(0) = log((1-p)/p); check-to-fault messages
 *     mu_{i->j}(t) = (-1)^sigma_i * prod_{j' in N(i)\j} sgn(nu_{j'->i}(t-1))
 *                    * min_{j' in N(i)\j} |nu_{j'->i}(t-1)|;
 *     fault-to-check messages nu_{j->i}(t) = lambda_j(t) + sum_{i' in N(j)\i}
 *     mu_{i'->j}(t); marginal Lambda_j(t) = lambda_j(t) + sum_{i in N(j)}
 *     mu_{i->j}(t); decision F_j = 1 iff Lambda_j(t) < 0; convergence when
 *     H F = sigma; memory lambda_j(t) = (1-gamma_j) lambda_j(0)
 *     + gamma_j Lambda_j(t-1); chaining: leg r >= 2 starts from the previous
 *     leg's final marginals (Relay-chaining paragraph); up to R legs, leg r
 *     running at most T_r iterations; optional continuation to S solutions.
 *   - Plain min-sum BP (same section, "Belief propagation decoding"), written
 *     separately with explicit leave-one-out sums (ro_minsum_trace_*).
 *   - Sum-product BP in FP64 (textbook tanh rule) for exactness checks on
 *     trees (ro_sumproduct_trace).
 *   - The Philox4x32-10 counter-based generator (Salmon et al., SC'11) for
 *     the per-leg memory strengths.
 *
 * Readings taken where the paper is silent or inconsistent (each one is also
 * listed in the design notes of the repository):
 *   R1 nu_{j->i}(t-1) is formed as Lambda_j(t-1) - mu_{i->j}(t-1); this equals
 *      the leave-one-out sum in exact arithmetic and fixes the FP rounding.
 *   R2 every message, lambda and the memory operand are clipped to
 *      [-L, L] (L = 2^64 by default) at the points marked CLIP below; the
 *      minimum over an empty set is +inf, clipped to L.
 *   R3 sgn(x) = -1 iff x < 0 (both zeros are positive); decision F_j = 1 iff
 *      Lambda_j < 0 (the BP paragraph's "> 0" contradicts its own positive
 *      priors for unlikely faults and is read as a typo).
 *   R4 anchor: leg r >= 2 sets lambda(0) = clip(Lambda^{(r-1)}(T)) (the
 *      paper's literal chaining) or, with anchor = 1, keeps lambda(0) = w.
 *      Check messages restart at mu = 0, so nu(0) = Lambda(0).
 *   R5 R counts all legs, leg 1 included; leg 1 uses gamma_first for every
 *      column; leg r >= 2 uses gamma_{r,j} = lo + (hi - lo) * u with
 *      u = (x >> 8) * 2^-24 and x = word (j mod 4) of
 *      Philox4x32-10(key = seed, ctr = (floor(j/4), r, 0, 0)).  The same
 *      Gamma_r is used for every shot.
 *   R6 convergence is tested after every iteration t >= 1, not at t = 0.
 *   R7 S > 1: every convergence event counts; a converged leg ends and the
 *      next leg starts from the marginals of that iteration; the output is the
 *      lowest-weight solution, weight W = sum_j F_j w_j summed in FP64 in
 *      ascending j, ties kept by the earliest.
 *   R8 the memory update is computed as a = (1 - gamma) * lambda(0),
 *      b = gamma * clip(Lambda(t-1)), lambda = clip(a + b), each operation
 *      rounded separately (no fused multiply-add); Lambda_j(t) is summed
 *      starting from lambda_j(t) and adding mu_{i->j}(t) in ascending i.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw; SC'11)                         */
/* ------------------------------------------------------------------------ */

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void ro_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]) {
    uint32_t k[2] = {key[0], key[1]};
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

static uint32_t gamma_word(uint64_t seed, int leg, int j) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)(j / 4), (uint32_t)leg, 0u, 0u};
    uint32_t out[4];
    ro_philox4x32_10(key, ctr, out);
    return out[j % 4];
}

/* Memory strength of column j in leg `leg` (>= 2), FP32 (reading R5). */
float ro_gamma_f32(uint64_t seed, int leg, int j, float lo, float hi) {
    uint32_t x = gamma_word(seed, leg, j);
    float u = (float)(x >> 8) * 0x1p-24f;
    float span = hi - lo;
    float prod = span * u;
    return lo + prod;
}

double ro_gamma_f64(uint64_t seed, int leg, int j, double lo, double hi) {
    uint32_t x = gamma_word(seed, leg, j);
    double u = (double)(x >> 8) * 0x1p-24;
    double span = hi - lo;
    double prod = span * u;
    return lo + prod;
}

/* ------------------------------------------------------------------------ */
/* Tanner graph (paper Sec. 2.1): checks i, faults j, edge iff H_ij = 1      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int M, N, E;
    int *rowptr, *col;   /* edges of check i: rowptr[i]..rowptr[i+1], columns ascending */
    int *colptr, *cedge; /* edges of fault j: colptr[j]..colptr[j+1], CSR edge ids, checks ascending */
    int *row;            /* row of CSR edge e */
} graph;

static void graph_free(graph *g) {
    free(g->rowptr); free(g->col); free(g->colptr); free(g->cedge); free(g->row);
    memset(g, 0, sizeof(*g));
}

/* Returns 0, or -1 bad shape, -2 index out of range, -3 duplicate entry, -4 OOM. */
static int graph_build(graph *g, int M, int N, long nnz, const int *rows, const int *cols) {
    memset(g, 0, sizeof(*g));
    if (M < 1 || N < 1 || nnz < 0) return -1;
    for (long k = 0; k < nnz; ++k)
        if (rows[k] < 0 || rows[k] >= M || cols[k] < 0 || cols[k] >= N) return -2;
    g->M = M; g->N = N; g->E = (int)nnz;
    g->rowptr = calloc((size_t)M + 1, sizeof(int));
    g->colptr = calloc((size_t)N + 1, sizeof(int));
    g->col = malloc(sizeof(int) * (size_t)(nnz ? nnz : 1));
    g->row = malloc(sizeof(int) * (size_t)(nnz ? nnz : 1));
    g->cedge = malloc(sizeof(int) * (size_t)(nnz ? nnz : 1));
    if (!g->rowptr || !g->colptr || !g->col || !g->row || !g->cedge) { graph_free(g); return -4; }
    /* dense 0/1 matrix scan keeps the ordering obvious: rows ascending, then columns */
    unsigned char *dense = calloc((size_t)M * (size_t)N, 1);
    if (!dense) { graph_free(g); return -4; }
    for (long k = 0; k < nnz; ++k) {
        unsigned char *cell = &dense[(size_t)rows[k] * N + cols[k]];
        if (*cell) { free(dense); graph_free(g); return -3; }
        *cell = 1;
    }
    int e = 0;
    for (int i = 0; i < M; ++i) {
        g->rowptr[i] = e;
        for (int j = 0; j < N; ++j)
            if (dense[(size_t)i * N + j]) { g->col[e] = j; g->row[e] = i; ++e; }
    }
    g->rowptr[M] = e;
    int c = 0;
    for (int j = 0; j < N; ++j) {
        g->colptr[j] = c;
        for (int i = 0; i < M; ++i) {
            if (!dense[(size_t)i * N + j]) continue;
            /* locate the CSR edge (i, j) */
            for (int ee = g->rowptr[i]; ee < g->rowptr[i + 1]; ++ee)
                if (g->col[ee] == j) { g->cedge[c++] = ee; break; }
        }
    }
    g->colptr[N] = c;
    free(dense);
    return 0;
}

/* Decoder parameters (oracle's own definition). */
typedef struct {
    int32_t num_legs;        /* R, total legs including leg 1 */
    int32_t iters_first;     /* T_1 */
    int32_t iters_leg;       /* T_r, r >= 2 */
    int32_t num_solutions;   /* S */
    float gamma_first;       /* gamma for every column in leg 1 */
    float gamma_lo, gamma_hi;/* gamma_{r,j} ~ U[lo, hi) for r >= 2 */
    double llr_clip;         /* L */
    uint64_t seed;           /* Philox key for gamma */
    int32_t anchor;          /* 0: lambda(0) = clip(Lambda) per leg; 1: lambda(0) = w */
    int32_t max_total_iters; /* 0 = no cutoff */
} ro_params;

/* ------------------------------------------------------------------------ */
/* Precision-generic bodies: instantiated once for float, once for double.   */
/* ------------------------------------------------------------------------ */

#define REAL float
#define SFX(name) name##_f32
#define RFABS fabsf
#define RINF INFINITY
#include "relay_oracle_body.inc"
#undef REAL
#undef SFX
#undef RFABS
#undef RINF

#define REAL double
#define SFX(name) name##_f64
#define RFABS fabs
#define RINF ((double)INFINITY)
#include "relay_oracle_body.inc"
#undef REAL
#undef SFX
#undef RFABS
#undef RINF

/* ------------------------------------------------------------------------ */
/* Reduced-precision mode: IEEE binary16 messages and marginals.             */
/*                                                                          */
/* The paper leaves the precision of Relay's messages open (its FPGA         */
/* estimates state none).  This mode runs the same algorithm, in the same    */
/* order, with every quantity of a shot (Lambda, lambda(0), the memory term, */
/* nu, mu) held as a binary16 value and every arithmetic result rounded to   */
/* binary16, nearest-even, with IEEE overflow to infinity:                   */
/*   w16_j   = h16(log((1 - p_j) / p_j))       (rounded once from FP64)      */
/*   g16_rj  = h16(gamma_rj) of the FP32 gamma of reading R5                 */
/*   L16     = h16(min(L, 4096))               (the clip; 4096 keeps sums of */
/*             up to 15 clipped terms finite)                                */
/*   nu      = clip(h16(Lambda - mu))                                        */
/*   mu      = sgn * min |nu| over the others  (selection only, no rounding) */
/*   a       = h16(h16(1 - g16) * lambda(0)),  b = h16(g16 * clip(Lambda))   */
/*   lambda  = clip(h16(a + b)),  Lambda = h16(... h16(lambda + mu_1) ...)   */
/* in ascending check order.  The decision, the convergence test, the legs   */
/* and the S-solution rule are those of the FP32 decoder; a solution's       */
/* weight W sums the FP32 channel LLRs in FP64, as there.  Values are kept   */
/* in doubles (every binary16 value is one), and a sum, difference or        */
/* product of two binary16 values is exact in FP64, so rounding the FP64     */
/* result once gives the correctly rounded binary16 operation.               */
/* ------------------------------------------------------------------------ */

/* Nearest binary16 value to x, ties to even (IEEE 754 roundTiesToEven), as
 * a double: 11 significant bits for |x| >= 2^-14, a fixed quantum of 2^-24
 * below (subnormals), infinity from 65520 = 65504 + half a unit up. */
double ro_round_h16(double x) {
    if (isnan(x)) return x;
    double a = fabs(x);
    if (a >= 65520.0) return copysign(INFINITY, x);
    if (a == 0.0) return x;
    int e;
    frexp(a, &e);            /* a = m 2^e, m in [0.5, 1) */
    int q = e - 11;          /* quantum of the binade [2^(e-1), 2^e) */
    if (q < -24) q = -24;
    double r = nearbyint(ldexp(a, -q));  /* default rounding mode: nearest, ties to even */
    return copysign(ldexp(r, q), x);
}

static double clip_h(double x, double L) {
    if (x > L) return L;
    if (x < -L) return -L;
    return x;
}

/* One DMem-BP iteration in binary16 (same steps as the FP32 iteration). */
static void dmem_iteration_h16(const graph *g, const unsigned char *sigma, const double *gamma,
                               const double *lam0, double *Lam, double *mu, double *nu,
                               unsigned char *F, double L) {
    for (int i = 0; i < g->M; ++i) {
        for (int e = g->rowptr[i]; e < g->rowptr[i + 1]; ++e)
            nu[e] = clip_h(ro_round_h16(Lam[g->col[e]] - mu[e]), L);
        for (int e = g->rowptr[i]; e < g->rowptr[i + 1]; ++e) {
            int negative = sigma[i] ? 1 : 0;
            double mag = INFINITY;
            for (int e2 = g->rowptr[i]; e2 < g->rowptr[i + 1]; ++e2) {
                if (e2 == e) continue;
                if (nu[e2] < 0) negative ^= 1;
                if (fabs(nu[e2]) < mag) mag = fabs(nu[e2]);
            }
            mu[e] = clip_h(negative ? -mag : mag, L);
        }
    }
    for (int j = 0; j < g->N; ++j) {
        double one_minus = ro_round_h16(1.0 - gamma[j]);
        double a = ro_round_h16(one_minus * lam0[j]);
        double b = ro_round_h16(gamma[j] * clip_h(Lam[j], L));
        double acc = clip_h(ro_round_h16(a + b), L);
        for (int c = g->colptr[j]; c < g->colptr[j + 1]; ++c) acc = ro_round_h16(acc + mu[g->cedge[c]]);
        Lam[j] = acc;
        F[j] = acc < 0 ? 1 : 0;
    }
}

/* Relay decoding in the binary16 mode; arguments as ro_decode_f32 (gamma1
 * float [N] or NULL, rounded to binary16; final_llr as float, exact). */
int ro_decode_h16(int M, int N, long nnz, const int *rows, const int *cols, const double *prior,
                  const ro_params *prm, const float *gamma1, long B, const unsigned char *syn,
                  unsigned char *corr, unsigned char *conv, int *legs, int *iters, double *weight,
                  float *final_llr) {
    if (prm->num_legs < 1 || prm->iters_first < 1 || prm->iters_leg < 1 || prm->num_solutions < 1)
        return -5;
    graph g;
    int rc = graph_build(&g, M, N, nnz, rows, cols);
    if (rc) return rc;
    const double L = ro_round_h16(fmin(prm->llr_clip, 4096.0));
    float *w32 = malloc(sizeof(float) * (size_t)N);
    double *w16 = malloc(sizeof(double) * (size_t)N);
    double *lam0 = malloc(sizeof(double) * (size_t)N);
    double *Lam = malloc(sizeof(double) * (size_t)N);
    double *mu = malloc(sizeof(double) * (size_t)(g.E ? g.E : 1));
    double *nu = malloc(sizeof(double) * (size_t)(g.E ? g.E : 1));
    double *gam = malloc(sizeof(double) * (size_t)N * (size_t)prm->num_legs);
    unsigned char *F = malloc((size_t)N);
    unsigned char *best = malloc((size_t)N);
    for (int j = 0; j < N; ++j) {
        double wd = log((1.0 - prior[j]) / prior[j]);
        w32[j] = (float)wd;
        w16[j] = ro_round_h16(wd);
    }
    for (int r = 1; r <= prm->num_legs; ++r)
        for (int j = 0; j < N; ++j) {
            float g32 = r == 1 ? (gamma1 ? gamma1[j] : prm->gamma_first)
                               : ro_gamma_f32(prm->seed, r, j, prm->gamma_lo, prm->gamma_hi);
            gam[(size_t)(r - 1) * N + j] = ro_round_h16((double)g32);
        }
    for (long b = 0; b < B; ++b) {
        const unsigned char *sigma = syn + (size_t)b * M;
        for (int j = 0; j < N; ++j) { Lam[j] = w16[j]; lam0[j] = w16[j]; }
        for (int e = 0; e < g.E; ++e) mu[e] = 0;
        int count = 0, total = 0, last_leg = 0, stop = 0;
        double best_w = INFINITY;
        for (int r = 1; r <= prm->num_legs && !stop; ++r) {
            int T = (r == 1) ? prm->iters_first : prm->iters_leg;
            if (r >= 2) {
                for (int e = 0; e < g.E; ++e) mu[e] = 0;
                for (int j = 0; j < N; ++j) lam0[j] = (prm->anchor == 0) ? clip_h(Lam[j], L) : w16[j];
            }
            const double *gr = gam + (size_t)(r - 1) * N;
            for (int t = 1; t <= T; ++t) {
                if (prm->max_total_iters > 0 && total >= prm->max_total_iters) { stop = 1; break; }
                last_leg = r;
                dmem_iteration_h16(&g, sigma, gr, lam0, Lam, mu, nu, F, L);
                ++total;
                if (syndrome_ok_f32(&g, sigma, F)) {
                    ++count;
                    double W = 0.0;
                    for (int j = 0; j < N; ++j) if (F[j]) W += (double)w32[j];
                    if (W < best_w) { best_w = W; memcpy(best, F, (size_t)N); }
                    if (count >= prm->num_solutions) stop = 1;
                    break;
                }
            }
        }
        unsigned char *out = corr + (size_t)b * N;
        double W = best_w;
        if (count > 0) {
            memcpy(out, best, (size_t)N);
        } else {
            memcpy(out, F, (size_t)N);
            W = 0.0;
            for (int j = 0; j < N; ++j) if (F[j]) W += (double)w32[j];
        }
        conv[b] = count > 0 ? 1 : 0;
        legs[b] = last_leg;
        iters[b] = total;
        if (weight) weight[b] = W;
        if (final_llr)
            for (int j = 0; j < N; ++j) final_llr[(size_t)b * N + j] = (float)Lam[j];
    }
    free(w32); free(w16); free(lam0); free(Lam); free(mu); free(nu); free(gam); free(F); free(best);
    graph_free(&g);
    return 0;
}

/* One leg in binary16 from the leg-1 initialisation for exactly T
 * iterations with per-column gamma (float [N], rounded to binary16):
 * trace[b][t][j] = Lambda_j(t) as float, t = 0..T. */
int ro_trace_h16(int M, int N, long nnz, const int *rows, const int *cols, const double *prior,
                 const float *gamma, int T, double llr_clip, long B, const unsigned char *syn,
                 float *trace) {
    graph g;
    int rc = graph_build(&g, M, N, nnz, rows, cols);
    if (rc) return rc;
    const double L = ro_round_h16(fmin(llr_clip, 4096.0));
    double *w = malloc(sizeof(double) * (size_t)N);
    double *gm = malloc(sizeof(double) * (size_t)N);
    double *Lam = malloc(sizeof(double) * (size_t)N);
    double *mu = malloc(sizeof(double) * (size_t)(g.E ? g.E : 1));
    double *nu = malloc(sizeof(double) * (size_t)(g.E ? g.E : 1));
    unsigned char *F = malloc((size_t)N);
    for (int j = 0; j < N; ++j) {
        w[j] = ro_round_h16(log((1.0 - prior[j]) / prior[j]));
        gm[j] = ro_round_h16((double)gamma[j]);
    }
    for (long b = 0; b < B; ++b) {
        const unsigned char *sigma = syn + (size_t)b * M;
        float *tr = trace + (size_t)b * (size_t)(T + 1) * N;
        for (int j = 0; j < N; ++j) { Lam[j] = w[j]; tr[j] = (float)w[j]; }
        for (int e = 0; e < g.E; ++e) mu[e] = 0;
        for (int t = 1; t <= T; ++t) {
            dmem_iteration_h16(&g, sigma, gm, w, Lam, mu, nu, F, L);
            for (int j = 0; j < N; ++j) tr[(size_t)t * N + j] = (float)Lam[j];
        }
    }
    free(w); free(gm); free(Lam); free(mu); free(nu); free(F);
    graph_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sum-product BP (FP64), for exactness checks on trees.                     */
/* Messages in the log-likelihood-ratio domain:                              */
/*   check -> fault: mu = (-1)^sigma * 2 atanh(prod_{j'!=j} tanh(nu/2))      */
/*   fault -> check: nu = w + sum_{i'!=i} mu; marginal Lambda = w + sum mu.  */
/* Returns the marginal LLR trace [T+1][N] per shot.                         */
/* ------------------------------------------------------------------------ */

int ro_sumproduct_trace(int M, int N, long nnz, const int *rows, const int *cols,
                        const double *llr, int T, long B, const unsigned char *syn,
                        double *trace) {
    graph g;
    int rc = graph_build(&g, M, N, nnz, rows, cols);
    if (rc) return rc;
    double *mu = calloc((size_t)(g.E ? g.E : 1), sizeof(double));
    double *nu = calloc((size_t)(g.E ? g.E : 1), sizeof(double));
    double *newmu = calloc((size_t)(g.E ? g.E : 1), sizeof(double));
    for (long b = 0; b < B; ++b) {
        const unsigned char *s = syn + (size_t)b * M;
        double *tr = trace + (size_t)b * (T + 1) * N;
        for (int e = 0; e < g.E; ++e) { mu[e] = 0.0; nu[e] = llr[g.col[e]]; }
        for (int j = 0; j < N; ++j) tr[j] = llr[j];
        for (int t = 1; t <= T; ++t) {
            for (int i = 0; i < M; ++i) {
                for (int e = g.rowptr[i]; e < g.rowptr[i + 1]; ++e) {
                    double prod = 1.0;
                    for (int e2 = g.rowptr[i]; e2 < g.rowptr[i + 1]; ++e2)
                        if (e2 != e) prod *= tanh(nu[e2] / 2.0);
                    double m = 2.0 * atanh(prod);
                    newmu[e] = s[i] ? -m : m;
                }
            }
            memcpy(mu, newmu, sizeof(double) * (size_t)g.E);
            for (int j = 0; j < N; ++j) {
                double tot = llr[j];
                for (int c = g.colptr[j]; c < g.colptr[j + 1]; ++c) tot += mu[g.cedge[c]];
                tr[(size_t)t * N + j] = tot;
                for (int c = g.colptr[j]; c < g.colptr[j + 1]; ++c) {
                    int e = g.cedge[c];
                    double v = llr[j];
                    for (int c2 = g.colptr[j]; c2 < g.colptr[j + 1]; ++c2)
                        if (c2 != c) v += mu[g.cedge[c2]];
                    nu[e] = v;
                }
            }
        }
    }
    free(mu); free(nu); free(newmu);
    graph_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Tangent (forward-mode derivative) of one leg, along its FP32 trajectory.  */
/*                                                                           */
/* The FP32 values follow ro_trace_f32 operation for operation (same         */
/* readings R1-R3, R8), so Lambda(T) is that function's last row.  Beside    */
/* them, FP64 tangents d(.) of every quantity in a direction (dgamma, dscale)*/
/* of the memory strengths and the channel-LLR scale (plus, optionally, a    */
/* direction dwprime [N] of the scaled LLRs w' themselves), by the chain rule on */
/* the update equations of paper Sec. 2.3 with the trajectory's discrete     */
/* choices held fixed:                                                       */
/*   w'       = s w                      dw'     = ds w                      */
/*   nu_e     = clip(Lambda_j - mu_e)    dnu_e   = dLambda_j - dmu_e inside  */
/*                                                 (-L, L), else 0           */
/*   mu_e     = S_e min_{e' != e} |nu_e'|  dmu_e = S_e sgn(nu_k) dnu_k, k the */
/*              first edge of the check (ascending) attaining that minimum;  */
/*              0 if the minimum is clipped (>= L) or the set is empty       */
/*   lambda_j = clip((1-g) w' + g clip(Lambda_j))                            */
/*            dlambda = (1-g) dw' + dg (clip(Lambda_j) - w')                 */
/*                      + g dLambda_j [Lambda_j inside]  inside (-L, L)      */
/*   Lambda_j = lambda_j + sum mu_e       dLambda = dlambda + sum dmu_e      */
/* sgn(0) = 0 (|x| has no slope there).  The sign product S_e is piecewise   */
/* constant and carries no tangent.  Writes Lambda(T) [B][N] (float) and     */
/* dLambda(T) [B][N] (double).                                               */
/* ------------------------------------------------------------------------ */

int ro_tangent_f32(int M, int N, long nnz, const int *rows, const int *cols, const double *prior,
                   float scale, const float *gamma, int T, double llr_clip, long B,
                   const unsigned char *syn, const double *dgamma, double dscale,
                   const double *dwprime, float *lam_out, double *dlam_out) {
    graph g;
    int rc = graph_build(&g, M, N, nnz, rows, cols);
    if (rc) return rc;
    const float L = (float)llr_clip;
    const size_t ne = (size_t)(g.E ? g.E : 1);
    float *w = malloc(sizeof(float) * (size_t)N), *wp = malloc(sizeof(float) * (size_t)N);
    float *Lam = malloc(sizeof(float) * (size_t)N), *mu = malloc(sizeof(float) * ne);
    float *nu = malloc(sizeof(float) * ne);
    double *dwp = malloc(sizeof(double) * (size_t)N), *dLam = malloc(sizeof(double) * (size_t)N);
    double *dmu = malloc(sizeof(double) * ne), *dnu = malloc(sizeof(double) * ne);
    for (int j = 0; j < N; ++j) {
        w[j] = (float)log((1.0 - prior[j]) / prior[j]);
        wp[j] = scale * w[j];
        dwp[j] = dscale * (double)w[j] + (dwprime ? dwprime[j] : 0.0);
    }
    for (long b = 0; b < B; ++b) {
        const unsigned char *sigma = syn + (size_t)b * M;
        for (int j = 0; j < N; ++j) { Lam[j] = wp[j]; dLam[j] = dwp[j]; }
        for (int e = 0; e < g.E; ++e) { mu[e] = 0.0f; dmu[e] = 0.0; }
        for (int t = 1; t <= T; ++t) {
            for (int i = 0; i < M; ++i) {
                for (int e = g.rowptr[i]; e < g.rowptr[i + 1]; ++e) {
                    const float pre = Lam[g.col[e]] - mu[e];
                    nu[e] = pre > L ? L : (pre < -L ? -L : pre);
                    dnu[e] = (pre > -L && pre < L) ? dLam[g.col[e]] - dmu[e] : 0.0;
                }
                for (int e = g.rowptr[i]; e < g.rowptr[i + 1]; ++e) {
                    int negative = sigma[i] ? 1 : 0, k = -1;
                    float mag = INFINITY;
                    for (int e2 = g.rowptr[i]; e2 < g.rowptr[i + 1]; ++e2) {
                        if (e2 == e) continue;
                        if (nu[e2] < 0) negative ^= 1;
                        if (fabsf(nu[e2]) < mag) { mag = fabsf(nu[e2]); k = e2; }
                    }
                    const float m = negative ? -mag : mag;
                    mu[e] = m > L ? L : (m < -L ? -L : m);
                    if (k < 0 || !(mag < L)) {
                        dmu[e] = 0.0;
                    } else {
                        const double sg = nu[k] > 0 ? 1.0 : (nu[k] < 0 ? -1.0 : 0.0);
                        dmu[e] = (negative ? -1.0 : 1.0) * sg * dnu[k];
                    }
                }
            }
            for (int j = 0; j < N; ++j) {
                const float gj = gamma[j];
                const float cl = Lam[j] > L ? L : (Lam[j] < -L ? -L : Lam[j]);
                const float a = (1.0f - gj) * wp[j];
                const float bb = gj * cl;
                const float pre = a + bb;
                float acc = pre > L ? L : (pre < -L ? -L : pre);
                double dacc = 0.0;
                if (pre > -L && pre < L) {
                    dacc = (1.0 - (double)gj) * dwp[j] + dgamma[j] * ((double)cl - (double)wp[j]);
                    if (Lam[j] > -L && Lam[j] < L) dacc += (double)gj * dLam[j];
                }
                for (int c = g.colptr[j]; c < g.colptr[j + 1]; ++c) {
                    acc += mu[g.cedge[c]];
                    dacc += dmu[g.cedge[c]];
                }
                Lam[j] = acc;
                dLam[j] = dacc;
            }
        }
        for (int j = 0; j < N; ++j) {
            lam_out[(size_t)b * N + j] = Lam[j];
            dlam_out[(size_t)b * N + j] = dLam[j];
        }
    }
    free(w); free(wp); free(Lam); free(mu); free(nu); free(dwp); free(dLam); free(dmu); free(dnu);
    graph_free(&g);
    return 0;
}
