/*
 * relaybp.h -- C ABI of the MI355X (gfx950) Relay-BP decoding library.
 *
 * The library decodes large batches of independent syndromes with Relay-BP:
 * successive legs of memory-augmented min-sum belief propagation (DMem-BP)
 * over the Tanner graph of a binary check / detector-error-model matrix H.
 *
 * Decoding problem (paper Sec. 2.1, circuit-decoding-problem paragraph): a
 * matrix H in F_2^{M x N}, independent fault probabilities p_j; a fault set F
 * produces the syndrome sigma = H F over F_2; the decoder returns a
 * correction F_hat.  Relay (paper Sec. 2.3, Relay decoding) runs up to R legs;
 * leg r runs at most T_r iterations of DMem-BP with memory strengths
 * Gamma_r = (gamma_{r,1..N}); leg r >= 2 starts from the final marginals of
 * leg r-1; a leg stops at the first iteration whose hard decision satisfies
 * H F_hat = sigma; decoding stops after S such solutions (lowest weight kept).
 *
 * Conventions shared by every call:
 *  - Plain C types only.  Pointers named d_* are device pointers (memory on
 *    the context's GPU, e.g. a torch tensor's data_ptr()); all others are
 *    host pointers.  `stream` is a hipStream_t passed as void* (NULL means
 *    the device's null stream).
 *  - Ownership: the caller owns every buffer it passes and must keep device
 *    buffers alive until the enqueued work completes.  A context owns its
 *    device copies of the graph, priors, parameters and workspace and frees
 *    them in rb_destroy.
 *  - Asynchrony: rb_decode and rb_trace only validate their arguments and
 *    enqueue kernels on `stream`; they return before the GPU work finishes
 *    and never synchronise or allocate.  A context is used by one stream at
 *    a time (calls on one context must not overlap on different streams).
 *  - Errors: every call returns an rb_status.  Argument and shape errors are
 *    detected on the host before any GPU work is enqueued; the call then has
 *    no effect.  rb_last_error_message() returns a thread-local description
 *    of the last failure on the calling thread.
 *  - Layouts: matrices are row-major and dense in their last dimension;
 *    batches are indexed by shot first ([B][...]).
 */
#ifndef RELAYBP_H
#define RELAYBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rb_ctx rb_ctx;

typedef enum {
    RB_OK = 0,
    RB_E_INVALID_ARG = 1,     /* null pointer, negative count, bad parameter value */
    RB_E_SHAPE = 2,           /* M, N, index or batch size out of range */
    RB_E_DUPLICATE_ENTRY = 3, /* a (row, col) pair listed twice (would cancel over F_2) */
    RB_E_PRIOR_RANGE = 4,     /* a prior outside (0, 1) or not finite */
    RB_E_DEVICE = 5,          /* HIP runtime failure or no usable device */
    RB_E_OOM = 6,             /* device or host allocation failed */
    RB_E_WORKSPACE = 7,       /* caller-provided buffer too small */
    RB_E_UNSUPPORTED = 8,     /* graph exceeds every kernel configuration built in */
    RB_E_NONFINITE = 9,       /* non-finite value where a finite one is required */
    RB_E_INTERNAL = 10        /* the library's own tables failed a consistency check */
} rb_status;

/* Layout of syndromes and corrections in device memory (rb_params.io_layout).
 * BYTES: one uint8 per check / fault, nonzero = 1 (syndromes; corrections are
 * written as 0 / 1).  BITS32: bit-packed uint32 words, W_M = ceil(M / 32) per
 * syndrome and W_N = ceil(N / 32) per correction, entry k in bit (k mod 32) of
 * word floor(k / 32); input bits past M in the last word are ignored, output
 * bits past N are written as 0.  Per-shot flags, counts, weights and
 * marginals keep their layouts. */
enum { RB_IO_BYTES = 0, RB_IO_BITS32 = 1 };

/* Arithmetic of the messages (rb_params.precision).  F32: IEEE binary32, the
 * decoder of paper Sec. 2.3 in canonical FP32 order.  F16: every per-shot
 * quantity (marginals Lambda, lambda(0), the memory term, nu and mu) held in
 * IEEE binary16 and every arithmetic result rounded to binary16 (nearest
 * even), in the same order: w16_j = binary16(log((1-p_j)/p_j)) rounded once
 * from FP64, gamma16 = binary16 of the FP32 memory strength, clip L16 =
 * binary16(min(llr_clip, 4096)) (so sums of up to 15 clipped terms stay
 * finite).  The paper does not state the precision of Relay's messages (its
 * FPGA resource estimates in the appendix on Relay resources give none).
 * Decisions, the convergence test, legs, S solutions and the weight W (FP64
 * sum of the FP32 w_j) are those of F32; final marginals are returned as
 * float.  F16 contexts run graphs that fit a block shape (two syndromes per
 * workgroup), no prior scale, no training calls and no mixed launch
 * (RB_E_UNSUPPORTED). */
enum { RB_PREC_F32 = 0, RB_PREC_F16 = 1 };

/* Anchor of the memory term in legs r >= 2 (leg 1 always uses w_j). */
enum { RB_ANCHOR_CHAIN = 0, /* lambda^{(r)}(0) = clip(Lambda^{(r-1)}(T_{r-1})), paper Sec. 2.3 */
       RB_ANCHOR_PRIOR = 1  /* lambda^{(r)}(0) = w_j = log((1-p_j)/p_j) in every leg */ };

/*
 * Decoder parameters (paper Sec. 2.3 Relay chaining; values used by the paper
 * in its appendix on Relay resources: S = 1, T_1 = 80, T_r = 60, 300 legs after
 * the first, gamma_0 = 0.125, gamma ~ U[-0.24, 0.66]).
 *   num_legs        R, the total number of legs including leg 1 (>= 1)
 *   iters_first     T_1, iteration cap of leg 1 (>= 1)
 *   iters_leg       T_r, iteration cap of every leg r >= 2 (>= 1)
 *   num_solutions   S, stop after this many converged legs (>= 1)
 *   gamma_first     memory strength of every column in leg 1
 *   gamma_lo/hi     gamma_{r,j} = lo + (hi - lo) u for r >= 2, u in [0, 1) drawn by
 *                   Philox4x32-10 (key = seed, counter = (floor(j/4), r, 0, 0), word j mod 4,
 *                   u = (word >> 8) 2^-24); the same Gamma_r for every shot
 *   llr_clip        L > 0: messages, marginals and the memory term saturate to [-L, L]
 *                   (an FP32 value, like the messages)
 *   seed            64-bit Philox key for the memory strengths
 *   anchor          RB_ANCHOR_CHAIN or RB_ANCHOR_PRIOR
 *   max_total_iters total iteration cutoff per shot across legs (0 = none); a shot
 *                   that reaches it without S solutions stops (paper Sec. 7: runs
 *                   past the cycle cutoff count as failures)
 *   io_layout       RB_IO_BYTES or RB_IO_BITS32: layout of the syndromes and
 *                   corrections that rb_decode, rb_decode_multi(_noalloc),
 *                   rb_autotune(_multi) and rb_syndrome take and return (rb_trace
 *                   and the training calls always take uint8 syndromes)
 *   precision       RB_PREC_F32 or RB_PREC_F16 (see above)
 */
typedef struct {
    int32_t num_legs;
    int32_t iters_first;
    int32_t iters_leg;
    int32_t num_solutions;
    float gamma_first;
    float gamma_lo;
    float gamma_hi;
    float llr_clip;
    uint64_t seed;
    int32_t anchor;
    int32_t max_total_iters;
    int32_t io_layout;
    int32_t precision;
} rb_params;

/* Kernel configuration chosen for a context (read-only diagnostics). */
typedef struct {
    int32_t M, N;
    int64_t num_edges;      /* E = nnz(H) */
    int32_t max_row_degree, max_col_degree;
    int32_t variant;        /* index into the built-in configuration table */
    int32_t lanes_per_shot; /* G: lanes cooperating on one syndrome */
    int32_t checks_per_lane, row_slots, cols_per_lane, col_slots;
    int32_t shots_per_block, threads_per_block;
    int32_t waves_per_simd_target; /* occupancy the kernel's register budget aims at */
    int32_t lds_bytes_per_block;
    int32_t blocks_per_cu, grid_blocks;
    int32_t num_variants;   /* size of the configuration table */
} rb_info;

/* Fills *out with the paper's parameters (R = 301 legs in total, T_1 = 80,
 * T_r = 60, S = 1, gamma_0 = 0.125, gamma in [-0.24, 0.66], L = 2^64,
 * anchor CHAIN, no cutoff, seed 0x52454C4159, RB_IO_BYTES, RB_PREC_F32).
 * RB_E_INVALID_ARG if out is NULL. */
rb_status rb_params_default(rb_params *out);

/*
 * Builds a decoder for H (COO) and priors on `device`.
 *   M, N          rows (checks / detectors) and columns (faults), both >= 1
 *   nnz           number of ones in H (>= 0); rows[k], cols[k] for k < nnz are
 *                 host int32 arrays with 0 <= rows[k] < M, 0 <= cols[k] < N, in
 *                 any order, without duplicates; empty rows and columns are allowed
 *   prior_p       host double[N], each in (0, 1); w_j = log((1-p_j)/p_j) is
 *                 evaluated in FP64 and rounded to FP32 (p_j = 1/2 gives w_j = 0)
 *   params        host pointer, copied
 * On success *out receives a new context (release with rb_destroy).  Builds
 * the check-major (CSR) and fault-major (CSC) edge layouts, the per-lane
 * gather tables of the chosen kernel configuration and the table of memory
 * strengths Gamma_1..Gamma_R on the device.  This call allocates and
 * synchronises the device.  Configurations, tried in this order: group tiles
 * (a few lanes per syndrome; small and medium codes), block shapes (one
 * 1024-thread workgroup per syndrome, M <= 1024, N <= 9216, row degree <= 64
 * after splitting rows over lane pairs), large-graph shapes (one workgroup
 * per syndrome with compressed messages, M <= 4096, N <= 32768, at most 4096
 * check records of 16 bytes with one record per 32 edges of a row and at
 * least one per row, 4N + 16 x records bytes of LDS within 160 KiB).
 * RB_E_UNSUPPORTED beyond.
 */
rb_status rb_create(rb_ctx **out, int32_t M, int32_t N, int64_t nnz, const int32_t *rows,
                    const int32_t *cols, const double *prior_p, const rb_params *params,
                    int32_t device);

/* Releases a context (NULL is a no-op).  Synchronises the context's device. */
void rb_destroy(rb_ctx *ctx);

/*
 * Relay-decodes B syndromes (paper Sec. 2.3: Relay decoding, convergence
 * criterion, Relay chaining).
 *   d_syndromes  uint8 [B][M], nonzero = 1 (RB_IO_BITS32: uint32 [B][W_M])
 *   d_corr       uint8 [B][N] out (RB_IO_BITS32: uint32 [B][W_N]): the lowest-weight
 *                converged solution, or the last hard decision (F_hat_j = 1 iff
 *                Lambda_j < 0) if no leg converged
 *   d_conv       uint8 [B] out: 1 iff at least one leg converged (H F_hat = sigma)
 *   d_legs       int32 [B] out: index (1-based) of the last leg started
 *   d_iters      int32 [B] out: iterations executed over all legs
 *   d_weight     double [B] out or NULL: sum_j F_hat_j w_j of d_corr
 *   d_final_llr  float [B][N] out or NULL: marginals Lambda after the last iteration
 * B == 0 is a no-op.  Returns RB_E_INVALID_ARG for null required pointers or
 * B < 0, RB_E_SHAPE for B >= 2^31 (shots are indexed in 32 bits).  Enqueues
 * on `stream`; no allocation, no synchronisation.
 */
rb_status rb_decode(rb_ctx *ctx, int64_t B, const uint8_t *d_syndromes, uint8_t *d_corr,
                    uint8_t *d_conv, int32_t *d_legs, int32_t *d_iters, double *d_weight,
                    float *d_final_llr, void *stream);

/*
 * Runs exactly T iterations of one DMem-BP leg from the leg-1 initialisation
 * (paper Sec. 2.3: nu(0) = lambda(0) = Lambda(0) = w) with per-column memory
 * strengths and scaled channel LLRs w'_j = scale * w_j, without the
 * convergence stop, and records the marginals.
 *   d_syndromes  uint8 [B][M]
 *   d_gamma      float [N] memory strengths gamma_j (device)
 *   T            >= 0 iterations
 *   d_trace      float [B][T+1][N] out: Lambda_j(t) for t = 0..T
 * Same kernels as rb_decode (message-level parity hook).  Enqueues on `stream`.
 * RB_E_SHAPE for B >= 2^31.
 */
rb_status rb_trace(rb_ctx *ctx, int64_t B, const uint8_t *d_syndromes, const float *d_gamma,
                   float scale, int32_t T, float *d_trace, void *stream);

/*
 * Syndrome of a batch of corrections over F_2 (the decoding problem of paper
 * Sec. 2.1: sigma = H F), optionally added to a given syndrome:
 *   d_corr      uint8 [B][N], nonzero = 1 (device; RB_IO_BITS32: uint32 [B][W_N])
 *   d_syn_in    uint8 [B][M] or NULL (device; RB_IO_BITS32: uint32 [B][W_M]); NULL
 *               reads as all zero
 *   d_syn_out   out (device), layout of d_syn_in: d_syn_in XOR (H d_corr mod 2); may
 *               alias d_syn_in
 * Windowed decoding uses it to pass the residual syndrome of committed faults
 * to the next window; it also checks corrections.  Enqueues on `stream`; no
 * allocation.  RB_E_INVALID_ARG for null required pointers, B < 0 or a
 * mixed-code context.
 */
rb_status rb_syndrome(const rb_ctx *ctx, int64_t B, const uint8_t *d_corr, const uint8_t *d_syn_in,
                      uint8_t *d_syn_out, void *stream);

/* Copies the FP32 channel LLRs w_j (host float[N]) -- test hook. */
rb_status rb_get_llr(const rb_ctx *ctx, float *host_w);

/* Copies the device table of memory strengths (host float[R][N], row r-1 =
 * Gamma_r) -- test hook for the counter-based generator. */
rb_status rb_get_gamma_table(const rb_ctx *ctx, float *host_gamma);

/* Learned first leg (the differentiable decoder's output, not part of the
 * paper's decoder): rb_set_leg_gamma replaces row `leg` - 1 of the memory
 * strength table (leg 1 = the first leg; host float[N], copied) for every
 * later decode on this context, so a first leg trained with rb_forward_train /
 * rb_backward can be run inside Relay.  rb_set_prior_scale sets s in
 * Lambda(0) = lambda(0) = s * w_j (and lambda(0) = s * w_j under the prior
 * anchor) for later decodes; the solution weight W keeps the unscaled w_j.
 * Defaults: the generated table and s = 1 (the paper's decoder).  Both copy
 * and synchronise the device; single-code contexts only (RB_E_INVALID_ARG for
 * a mixed-code context); RB_E_NONFINITE for a non-finite value,
 * RB_E_INVALID_ARG for a leg outside 1..R. */
rb_status rb_set_leg_gamma(rb_ctx *ctx, int32_t leg, const float *host_gamma);
rb_status rb_set_prior_scale(rb_ctx *ctx, float scale);

/* Fills *info with the context's kernel configuration. */
rb_status rb_get_info(const rb_ctx *ctx, rb_info *info);

/* Selects kernel configuration `variant` (index into the built-in table) for
 * later decodes; RB_E_UNSUPPORTED if the graph does not fit it.  Rebuilds the
 * gather tables (allocates and synchronises). */
rb_status rb_set_variant(rb_ctx *ctx, int32_t variant);

/* Report of rb_plan_check.  LDS cost model: 32 banks of 4-byte words; a
 * wave-wide gather costs the largest number of distinct words on one bank, so
 * a gather of 64 distinct words costs at least 2 (conflict-free). */
typedef struct {
    int32_t variant;            /* configuration checked (index as in rb_info) */
    int32_t block_kernel;       /* 0: group-kernel tile, 1: block kernel, 2: large-graph kernel (no tables costed) */
    int32_t lds_bytes;          /* LDS image of one block (block kernel) or one wave (tile) */
    int64_t check_gathers;      /* table-driven Lambda gathers of one iteration (wave-wide) */
    int64_t check_bank_cycles;  /* their summed modelled cost */
    int64_t fault_gathers;      /* table-driven message gathers of one iteration (wave-wide) */
    int64_t fault_bank_cycles;  /* their summed modelled cost */
} rb_plan_report;

/*
 * Host-only diagnostics (no device use, no context): builds the per-lane LDS
 * gather tables that rb_create would upload for H (M, N, nnz, rows, cols as in
 * rb_create) and configuration `variant` (-1: the one rb_create chooses), then
 * reads them back the way the kernels do and checks them against H: every
 * edge (i, j) is gathered exactly once on the check side, at the marginal of
 * fault j, by a lane working on check i; fault j gathers the messages of its
 * checks in ascending i (the summation order of the marginal, paper Sec. 2.3
 * DMem-BP), each at the word where check i writes the message of edge (i, j);
 * every other entry addresses the pad cell; addresses fit their 16-bit fields
 * and the LDS image.  On success *out holds the modelled bank cost of the
 * gathers.  RB_E_SHAPE / RB_E_INVALID_ARG / RB_E_DUPLICATE_ENTRY as in
 * rb_create; RB_E_UNSUPPORTED if the graph does not fit the configuration;
 * RB_E_INTERNAL if a table breaks a rule (rb_last_error_message names it).
 */
rb_status rb_plan_check(int32_t M, int32_t N, int64_t nnz, const int32_t *rows, const int32_t *cols,
                        int32_t variant, rb_plan_report *out);

/*
 * Measures every built-in kernel configuration the graph fits on B syndromes
 * (d_syndromes on the device, in the context's io_layout), `reps` timed launches each after
 * one warm-up, and keeps the fastest for later decodes.  Results do not
 * depend on the configuration (only speed does).  Allocates scratch outputs,
 * uses the null stream and synchronises the device: call it once after
 * rb_create, not inside a captured or latency-critical region.
 *   chosen_variant  out (nullable): index of the configuration kept
 *   best_ms         out (nullable): its mean time per decode, milliseconds
 */
rb_status rb_autotune(rb_ctx *ctx, int64_t B, const uint8_t *d_syndromes, int32_t reps,
                      int32_t *chosen_variant, float *best_ms);

/*
 * Longest-first scheduling for rb_decode: allocates (once, synchronising the
 * device) a workspace for batches of up to B syndromes.  Decodes of at most B
 * syndromes then first sort their shots by decreasing syndrome weight on the
 * device, so that hard syndromes start early and the persistent queue ends
 * with short ones; results are identical, only the order of work changes.
 * Block-kernel (large-graph) contexts ignore it.  Not for mixed contexts.
 */
rb_status rb_reserve(rb_ctx *ctx, int64_t B);

/* Bytes of device workspace rb_decode_multi needs for B syndromes (also the
 * size rb_reserve allocates for a single-code context). */
size_t rb_workspace_size(const rb_ctx *ctx, int64_t B);

/* One code of a mixed batch (same meaning as the arguments of rb_create). */
typedef struct {
    int32_t M, N;
    int64_t nnz;
    const int32_t *rows;
    const int32_t *cols;
    const double *prior_p;
} rb_code_desc;

/*
 * Builds one decoder for several codes (1..64) whose syndromes are decoded
 * together by rb_decode_multi in one persistent launch.  Every code is planned
 * on a tile of the mixed kernel (small and medium graphs; RB_E_UNSUPPORTED
 * otherwise) and shares `params`.  Allocates and synchronises the device.
 */
rb_status rb_create_multi(rb_ctx **out, int32_t n_codes, const rb_code_desc *codes,
                          const rb_params *params, int32_t device);

/*
 * Relay-decodes B syndromes of mixed codes in one launch (paper Sec. 2.3
 * per syndrome; the batching is this library's).  Let M_max / N_max be the
 * largest M / N over the codes.
 *   d_code_id    int32 [B]: code of each syndrome (index into the rb_create_multi
 *                list); a shot with an id outside [0, n_codes) is skipped and its
 *                outputs are left untouched
 *   d_syndromes  uint8 [B][M_max]: row b holds the code's M syndrome bits first
 *                (RB_IO_BITS32: uint32 [B][ceil(M_max / 32)], the code's bits first)
 *   d_corr       uint8 [B][N_max] out (first N entries of row b are meaningful;
 *                RB_IO_BITS32: uint32 [B][ceil(N_max / 32)], the first N bits);
 *   d_conv, d_legs, d_iters, d_weight, d_final_llr ([B][N_max]) as in rb_decode
 *   d_workspace  device buffer of at least rb_workspace_size(ctx, B) bytes, owned
 *                by the caller, not used concurrently by another call
 * Codes with the same graph and tile (for instance one code at several noise
 * rates) form a family whose shots share one list, ordered by decreasing
 * syndrome weight; each shot is decoded with its own code's priors and
 * memory strengths.  Each wave of the launch decodes one family at a time
 * with the family's tile.  Enqueues on
 * `stream` only (no allocation, no synchronisation, no memset): the call can
 * be captured in a hipGraph and replayed.  Results equal per-code rb_decode.
 */
rb_status rb_decode_multi(rb_ctx *ctx, int64_t B, const int32_t *d_code_id,
                          const uint8_t *d_syndromes, uint8_t *d_corr, uint8_t *d_conv,
                          int32_t *d_legs, int32_t *d_iters, double *d_weight, float *d_final_llr,
                          void *d_workspace, size_t workspace_bytes, void *stream);

/*
 * rb_decode_multi without a workspace argument, for callers that cannot
 * allocate device memory: code being captured into a hipGraph, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments (minus d_workspace
 * and workspace_bytes), same results as rb_decode_multi.  The shot lists and
 * queue counters live in a static device array of 12 MiB that the library
 * holds on every GPU it runs on until the process ends; the call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine), clears what
 * must start at zero with small kernels (no memset), and only enqueues on
 * `stream`.  The first call on a device looks up the array's address there.
 * Every call on one GPU, from any context, uses that GPU's one array: calls
 * that overlap on one GPU (concurrent streams, threads) race and give wrong
 * results; serialise them.
 *   returns RB_E_WORKSPACE if B > rb_noalloc_max_batch(ctx) (about 10^6
 *   syndromes), before any GPU work; otherwise as rb_decode_multi.
 */
rb_status rb_decode_multi_noalloc(rb_ctx *ctx, int64_t B, const int32_t *d_code_id,
                                  const uint8_t *d_syndromes, uint8_t *d_corr, uint8_t *d_conv,
                                  int32_t *d_legs, int32_t *d_iters, double *d_weight,
                                  float *d_final_llr, void *stream);

/* Largest batch rb_decode_multi_noalloc accepts for a mixed context (0 for
 * NULL or a single-code context); host-only. */
int64_t rb_noalloc_max_batch(const rb_ctx *ctx);

/*
 * Autotunes a mixed context: for every code k with sample_b[k] > 0, times each
 * tile of the mixed kernel that fits the code on d_samples[k] (uint8
 * [sample_b[k]][M_k], or uint32 [sample_b[k]][ceil(M_k / 32)] under
 * RB_IO_BITS32; device) and keeps the fastest.  chosen_variants
 * (nullable, int32 [n_codes]) receives the configuration kept per code.
 * Allocates scratch and synchronises the device.
 */
rb_status rb_autotune_multi(rb_ctx *ctx, const int64_t *sample_b, const uint8_t *const *d_samples,
                            int32_t reps, int32_t *chosen_variants);

/*
 * Sets the tile code k of a mixed context decodes with (a configuration index
 * as in rb_info).  RB_E_INVALID_ARG for a single-code context or k outside
 * [0, n_codes); RB_E_UNSUPPORTED if the configuration is not a tile of the
 * mixed kernel or the code does not fit it.  Codes with the same graph share
 * one shot list and queue while they also share a tile.  Rebuilds the gather
 * tables (allocates and synchronises).
 */
rb_status rb_set_code_variant(rb_ctx *ctx, int32_t k, int32_t variant);

/*
 * Differentiable decoding (learned memory strengths).  The forward pass is one
 * DMem-BP leg from the leg-1 initialisation (paper Sec. 2.3) run for exactly T
 * iterations with learnable per-column memory strengths gamma_j and channel
 * LLRs w'_j = s * w_j with a learnable scale s, in the decoder's FP32
 * arithmetic (Lambda(T) equals rb_trace's last row); it checkpoints the
 * messages every `ckpt_every` iterations into a caller-owned tape.  The
 * backward pass is the hand-written adjoint of that unrolled min-sum: it
 * recomputes each segment from its checkpoint and sweeps it in reverse,
 * routing gradients through the check minima (argmin / second argmin) and not
 * through signs or saturated clips.
 *
 * rb_train_tape_size: bytes of tape for (B, T, ckpt_every); 0 on bad input.
 */
size_t rb_train_tape_size(const rb_ctx *ctx, int64_t B, int32_t T, int32_t ckpt_every);

/*
 * Forward pass.  d_syndromes uint8 [B][M]; d_gamma float [N] and d_scale
 * float [1] on the device (read when the kernel runs, so a training loop never
 * synchronises); d_llr_out float [B][N] out: Lambda(T); d_tape at least
 * rb_train_tape_size bytes, caller-owned, kept until rb_backward has run.
 * RB_E_UNSUPPORTED for graphs whose training state exceeds 64 KiB of LDS.
 */
rb_status rb_forward_train(rb_ctx *ctx, int64_t B, const uint8_t *d_syndromes, const float *d_gamma,
                           const float *d_scale, int32_t T, int32_t ckpt_every, float *d_llr_out,
                           void *d_tape, size_t tape_bytes, void *stream);

/*
 * Backward pass for the same (B, syndromes, gamma, scale, T, ckpt_every, tape)
 * as the preceding rb_forward_train.  d_dllr float [B][N]: dLoss/dLambda(T).
 * d_dgamma float [N] and d_dscale float [1] are overwritten with dLoss/dgamma
 * and dLoss/ds summed over the batch in a fixed order (deterministic).
 */
rb_status rb_backward(rb_ctx *ctx, int64_t B, const uint8_t *d_syndromes, const float *d_gamma,
                      const float *d_scale, int32_t T, int32_t ckpt_every, void *d_tape,
                      size_t tape_bytes, const float *d_dllr, float *d_dgamma, float *d_dscale,
                      void *stream);

/* Synchronises the context's device and reports asynchronous HIP errors. */
rb_status rb_sync_status(rb_ctx *ctx);

/* Static description of a status code (never NULL). */
const char *rb_status_string(rb_status status);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *rb_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* RELAYBP_H */
