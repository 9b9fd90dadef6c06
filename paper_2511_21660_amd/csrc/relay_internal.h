// relay_internal.h -- declarations shared by the host ABI (relay_api.cpp) and
// the gfx950 kernels (relay_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rb {

// Shape of one kernel configuration ("tile"): G lanes of a wave cooperate on
// one syndrome; lane g owns checks i = g + G*c (c < CPT) and faults
// j = g + G*v (v < VPT); DC and DV bound the row and column degrees.
struct TileShape {
    int G, CPT, DC, VPT, DV;
};

// Arguments of the group kernel (passed by value).
struct GroupArgs {
    int32_t M, N;
    int64_t B;
    const uint8_t *syn;   // [B][M]
    uint8_t *corr;        // [B][N]
    uint8_t *conv;        // [B]
    int32_t *legs;        // [B]
    int32_t *iters;       // [B]
    double *weight;       // [B] or null
    float *final_llr;     // [B][N] or null
    const float *w;       // [N] channel LLRs
    const float *gamma;   // [R][N] memory strengths, row r-1 = leg r
    const uint32_t *lam_off;  // [G][CPT][DC] slot-relative byte offsets of Lambda gathers
    const uint32_t *mu_off;   // [G][VPT][DV] slot-relative byte offsets of mu gathers
    unsigned long long *queue;  // next unclaimed shot
    int32_t num_legs, iters_first, iters_leg, num_solutions, max_total_iters;
    float L;
    uint32_t slot_bytes;   // LDS bytes per shot slot
    uint32_t lampad_off;   // +inf cell: Lambda of padded check edges
    uint32_t mupad_off;    // -0 cell: mu of padded fault edges
    uint32_t mu0_off;      // start of the check-message rows
    // trace mode (rb_trace): per-column gamma, LLR scale, iteration count, output
    const float *trace_gamma;
    float scale;
    int32_t trace_T;
    float *trace;          // [B][T+1][N]
};

int num_variants();
TileShape variant_shape(int v);
// Blocks of the variant's kernel that fit on one CU with `lds` bytes of LDS per block.
hipError_t variant_occupancy(int v, bool prior_anchor, bool trace, size_t lds, int *blocks);
hipError_t launch_group(int v, bool prior_anchor, bool trace, const GroupArgs &a, int grid,
                        size_t lds, hipStream_t s);
hipError_t launch_gamma_table(float *tab, int R, int N, uint64_t seed, float g_first, float lo,
                              float hi, hipStream_t s);
hipError_t launch_reset_queue(unsigned long long *q, hipStream_t s);

}  // namespace rb
