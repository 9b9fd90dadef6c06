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
