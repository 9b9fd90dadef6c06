/*
 * sanitize_oracle_main.c -- runs every entry point of the CPU oracle on
 * generated problems (random loopy graphs with empty rows and columns and
 * degree-1 checks; trees; all three precisions, both anchors, S > 1, an
 * iteration cutoff, traces, min-sum and sum-product) for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  The oracle's source is
 * included whole, so its static helpers are built the same way.
 * Exit status 0 iff every call returns 0.
 */
#include "../oracle/relay_oracle.c"

#include <stdio.h>

static unsigned rng_state = 12345u;
static unsigned rnd(void) {
    rng_state = rng_state * 1664525u + 1013904223u;
    return rng_state >> 8;
}

int main(void) {
    int bad = 0, calls = 0;
    for (int trial = 0; trial < 12; ++trial) {
        const int M = 3 + (int)(rnd() % 20), N = 4 + (int)(rnd() % 40);
        int *rows = malloc(sizeof(int) * (size_t)M * N), *cols = malloc(sizeof(int) * (size_t)M * N);
        long nnz = 0;
        for (int i = 0; i < M; ++i) {
            if (i == M / 2) continue; /* an empty row */
            for (int j = 0; j < N - 1; ++j) /* the last column stays empty */
                if (rnd() % 100 < 18) { rows[nnz] = i; cols[nnz] = j; ++nnz; }
        }
        double *prior = malloc(sizeof(double) * (size_t)N);
        for (int j = 0; j < N; ++j) prior[j] = j % 7 == 0 ? 0.5 : 0.01 + 0.3 * (double)(rnd() % 1000) / 1000.0;
        const long B = 7;
        unsigned char *syn = malloc((size_t)B * M);
        for (long k = 0; k < B * M; ++k) syn[k] = (unsigned char)(rnd() & 1);
        unsigned char *corr = malloc((size_t)B * N), *conv = malloc((size_t)B);
        int *legs = malloc(sizeof(int) * (size_t)B), *iters = malloc(sizeof(int) * (size_t)B);
        double *weight = malloc(sizeof(double) * (size_t)B), *llr64 = malloc(sizeof(double) * (size_t)B * N);
        float *llr32 = malloc(sizeof(float) * (size_t)B * N), *g1 = malloc(sizeof(float) * (size_t)N);
        double *g64 = malloc(sizeof(double) * (size_t)N);
        for (int j = 0; j < N; ++j) { g1[j] = 0.1f * (float)(j % 5); g64[j] = g1[j]; }
        ro_params p = {.num_legs = 6, .iters_first = 12, .iters_leg = 9, .num_solutions = 1 + trial % 3,
                       .gamma_first = 0.125f, .gamma_lo = -0.24f, .gamma_hi = 0.66f,
                       .llr_clip = trial % 2 ? 1e19 : 64.0, .seed = 0x52454C4159ull,
                       .anchor = trial % 2, .max_total_iters = trial % 4 == 3 ? 25 : 0};
        const int T = 6;
        float *tr32 = malloc(sizeof(float) * (size_t)B * (T + 1) * N);
        double *tr64 = malloc(sizeof(double) * (size_t)B * (T + 1) * N);
        double *llrin = malloc(sizeof(double) * (size_t)N);
        float *llrin32 = malloc(sizeof(float) * (size_t)N);
        for (int j = 0; j < N; ++j) { llrin[j] = 1.0 + (double)(j % 4); llrin32[j] = (float)llrin[j]; }
        int rc[9];
        rc[0] = ro_decode_f32(M, N, nnz, rows, cols, prior, &p, trial % 3 ? g1 : NULL, 1.0, B, syn, corr, conv, legs,
                              iters, weight, llr32);
        rc[1] = ro_decode_f64(M, N, nnz, rows, cols, prior, &p, trial % 3 ? g64 : NULL, 0.5, B, syn, corr, conv,
                              legs, iters, weight, llr64);
        rc[2] = ro_decode_h16(M, N, nnz, rows, cols, prior, &p, trial % 3 ? g1 : NULL, B, syn, corr, conv, legs,
                              iters, weight, llr32);
        rc[3] = ro_trace_f32(M, N, nnz, rows, cols, prior, 1.0, g1, T, p.llr_clip, B, syn, tr32);
        rc[4] = ro_trace_f64(M, N, nnz, rows, cols, prior, 1.0, g64, T, p.llr_clip, B, syn, tr64);
        rc[5] = ro_trace_h16(M, N, nnz, rows, cols, prior, g1, T, p.llr_clip, B, syn, tr32);
        rc[6] = ro_minsum_trace_f32(M, N, nnz, rows, cols, llrin32, T, B, syn, tr32);
        rc[7] = ro_minsum_trace_f64(M, N, nnz, rows, cols, llrin, T, B, syn, tr64);
        rc[8] = ro_sumproduct_trace(M, N, nnz, rows, cols, llrin, T, B, syn, tr64);
        for (int k = 0; k < 9; ++k) {
            ++calls;
            if (rc[k] != 0) { printf("trial %d call %d returned %d\n", trial, k, rc[k]); ++bad; }
        }
        free(rows); free(cols); free(prior); free(syn); free(corr); free(conv); free(legs); free(iters);
        free(weight); free(llr64); free(llr32); free(g1); free(g64); free(tr32); free(tr64); free(llrin);
        free(llrin32);
    }
    uint32_t key[2] = {1u, 2u}, ctr[4] = {3u, 4u, 5u, 6u}, out[4];
    ro_philox4x32_10(key, ctr, out);
    (void)ro_gamma_f32(7, 3, 5, -0.24f, 0.66f);
    (void)ro_gamma_f64(7, 3, 5, -0.24, 0.66);
    (void)ro_round_h16(1.0 / 3.0);
    printf("oracle calls: %d, failures: %d\n", calls, bad);
    return bad ? 1 : 0;
}
