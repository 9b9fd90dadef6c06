// relay_api.cpp -- host side of the Relay-BP C ABI (include/relaybp.h).
//
// rb_create validates the decoding problem (paper Sec. 2.1: H, p), builds the
// check-major (CSR) and fault-major (CSC) edge layouts on the host, chooses a
// kernel configuration, precompiles the per-lane LDS gather offsets of that
// configuration, and uploads them with the channel LLRs and the table of
// memory strengths Gamma_1..Gamma_R (drawn on the device by Philox4x32-10).
// rb_decode / rb_trace validate their arguments and enqueue kernels only.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/relaybp.h"
#include "relay_internal.h"

namespace {

thread_local std::string g_last_error;

rb_status fail(rb_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

rb_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return RB_E_DEVICE;
}

#define RB_HIP(call, what)                          \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

}  // namespace

struct rb_ctx {
    int device = 0;
    int32_t M = 0, N = 0;
    int64_t E = 0;
    int32_t max_row = 0, max_col = 0;
    rb_params params{};
    // host graph
    std::vector<int64_t> rowptr;  // [M+1]
    std::vector<int32_t> colidx;  // [E], ascending within a row
    std::vector<int64_t> colptr;  // [N+1]
    std::vector<int32_t> rowidx;  // [E], ascending within a column
    std::vector<int32_t> cpos;    // [E] position of edge (rowidx, j) inside its CSR row
    std::vector<float> w;         // [N]
    // device
    float *d_w = nullptr;
    float *d_gamma = nullptr;        // [R][N]
    uint32_t *d_lam_off = nullptr;
    uint32_t *d_mu_off = nullptr;
    unsigned long long *d_queue = nullptr;
    // plan
    int variant = -1;
    rb::TileShape shape{};
    uint32_t slot_bytes = 0, lampad_off = 0, mupad_off = 0, mu0_off = 0;
    int lds_bytes = 0;
    int blocks_per_cu[2] = {0, 0};  // [trace]
    int num_cu = 0;
};

namespace {

int ceil_div(int a, int b) { return (a + b - 1) / b; }

struct Layout {
    uint32_t slot_bytes, lampad_off, mupad_off, mu0_off;
    int lds_bytes;
};

Layout slot_layout(const rb::TileShape &s, int N) {
    Layout l{};
    l.lampad_off = 4u * (uint32_t)N;
    l.mupad_off = l.lampad_off + 4u;
    l.mu0_off = (l.mupad_off + 4u + 7u) & ~7u;
    uint32_t words = (l.mu0_off + 4u * (uint32_t)(s.G * s.CPT * s.DC)) / 4u;
    words = (words + 1u) & ~1u;
    while (words % 32u != 2u) words += 2u;  // spread slots over LDS banks
    l.slot_bytes = 4u * words;
    l.lds_bytes = (int)(l.slot_bytes * (uint32_t)(64 / s.G));
    return l;
}

bool variant_fits(const rb_ctx *c, const rb::TileShape &s) {
    if (ceil_div(c->M, s.G) > s.CPT || ceil_div(c->N, s.G) > s.VPT) return false;
    if (c->max_row > s.DC || c->max_col > s.DV) return false;
    return slot_layout(s, c->N).lds_bytes <= 64 * 1024;
}

// Estimated lane-operations per shot-iteration (lockstep: a slot pays for all
// of its padded rows and columns): about 10 per check edge, 2 per fault edge,
// 6 per fault.
double variant_cost(const rb::TileShape &s) {
    return (double)s.G * (10.0 * s.CPT * s.DC + 2.0 * s.VPT * s.DV + 6.0 * s.VPT);
}

rb_status build_plan(rb_ctx *c, int v) {
    const rb::TileShape s = rb::variant_shape(v);
    const Layout lay = slot_layout(s, c->N);
    std::vector<uint32_t> lam((size_t)s.G * s.CPT * s.DC, lay.lampad_off);
    std::vector<uint32_t> mu((size_t)s.G * s.VPT * s.DV, lay.mupad_off);
    for (int g = 0; g < s.G; ++g) {
        for (int cc = 0; cc < s.CPT; ++cc) {
            const int i = g + s.G * cc;
            if (i >= c->M) continue;
            const int64_t b = c->rowptr[i], e = c->rowptr[i + 1];
            for (int64_t k = 0; k < e - b; ++k)
                lam[((size_t)g * s.CPT + cc) * s.DC + k] = 4u * (uint32_t)c->colidx[b + k];
        }
        for (int vv = 0; vv < s.VPT; ++vv) {
            const int j = g + s.G * vv;
            if (j >= c->N) continue;
            const int64_t b = c->colptr[j], e = c->colptr[j + 1];
            for (int64_t k = 0; k < e - b; ++k) {
                const int i = c->rowidx[b + k];
                const uint32_t word = (uint32_t)i * s.DC + (uint32_t)c->cpos[b + k];
                mu[((size_t)g * s.VPT + vv) * s.DV + k] = lay.mu0_off + 4u * word;
            }
        }
    }
    (void)hipFree(c->d_lam_off);
    (void)hipFree(c->d_mu_off);
    c->d_lam_off = nullptr;
    c->d_mu_off = nullptr;
    RB_HIP(hipMalloc(&c->d_lam_off, lam.size() * 4), "hipMalloc(lam_off)");
    RB_HIP(hipMalloc(&c->d_mu_off, mu.size() * 4), "hipMalloc(mu_off)");
    RB_HIP(hipMemcpy(c->d_lam_off, lam.data(), lam.size() * 4, hipMemcpyHostToDevice), "copy lam_off");
    RB_HIP(hipMemcpy(c->d_mu_off, mu.data(), mu.size() * 4, hipMemcpyHostToDevice), "copy mu_off");
    c->variant = v;
    c->shape = s;
    c->slot_bytes = lay.slot_bytes;
    c->lampad_off = lay.lampad_off;
    c->mupad_off = lay.mupad_off;
    c->mu0_off = lay.mu0_off;
    c->lds_bytes = lay.lds_bytes;
    const bool prior = c->params.anchor == RB_ANCHOR_PRIOR;
    for (int tr = 0; tr < 2; ++tr) {
        int blocks = 0;
        RB_HIP(rb::variant_occupancy(v, prior, tr != 0, (size_t)lay.lds_bytes, &blocks),
               "occupancy query");
        if (blocks < 1) return fail(RB_E_UNSUPPORTED, "kernel configuration does not fit on a CU");
        c->blocks_per_cu[tr] = blocks;
    }
    return RB_OK;
}

rb_status check_params(const rb_params *p) {
    if (!p) return fail(RB_E_INVALID_ARG, "params is NULL");
    if (p->num_legs < 1 || p->iters_first < 1 || p->iters_leg < 1 || p->num_solutions < 1)
        return fail(RB_E_INVALID_ARG, "num_legs, iters_first, iters_leg, num_solutions must be >= 1");
    if (p->max_total_iters < 0) return fail(RB_E_INVALID_ARG, "max_total_iters must be >= 0");
    if (p->anchor != RB_ANCHOR_CHAIN && p->anchor != RB_ANCHOR_PRIOR)
        return fail(RB_E_INVALID_ARG, "anchor must be RB_ANCHOR_CHAIN or RB_ANCHOR_PRIOR");
    if (!std::isfinite(p->gamma_first) || !std::isfinite(p->gamma_lo) || !std::isfinite(p->gamma_hi))
        return fail(RB_E_NONFINITE, "memory strengths must be finite");
    if (p->gamma_lo > p->gamma_hi) return fail(RB_E_INVALID_ARG, "gamma_lo > gamma_hi");
    if (!std::isfinite(p->llr_clip) || !(p->llr_clip > 0.0f))
        return fail(RB_E_INVALID_ARG, "llr_clip must be finite and > 0");
    return RB_OK;
}

}  // namespace

extern "C" {

const char *rb_status_string(rb_status s) {
    switch (s) {
        case RB_OK: return "ok";
        case RB_E_INVALID_ARG: return "invalid argument";
        case RB_E_SHAPE: return "shape or index out of range";
        case RB_E_DUPLICATE_ENTRY: return "duplicate (row, col) entry";
        case RB_E_PRIOR_RANGE: return "prior outside (0, 1)";
        case RB_E_DEVICE: return "device error";
        case RB_E_OOM: return "out of memory";
        case RB_E_WORKSPACE: return "workspace too small";
        case RB_E_UNSUPPORTED: return "unsupported graph or configuration";
        case RB_E_NONFINITE: return "non-finite value";
    }
    return "unknown status";
}

const char *rb_last_error_message(void) { return g_last_error.c_str(); }

rb_status rb_params_default(rb_params *out) {
    if (!out) return fail(RB_E_INVALID_ARG, "out is NULL");
    std::memset(out, 0, sizeof(*out));
    out->num_legs = 301;
    out->iters_first = 80;
    out->iters_leg = 60;
    out->num_solutions = 1;
    out->gamma_first = 0.125f;
    out->gamma_lo = -0.24f;
    out->gamma_hi = 0.66f;
    out->llr_clip = 18446744073709551616.0f;  // 2^64
    out->seed = 0x52454C4159ull;
    out->anchor = RB_ANCHOR_CHAIN;
    out->max_total_iters = 0;
    return RB_OK;
}

rb_status rb_create(rb_ctx **out, int32_t M, int32_t N, int64_t nnz, const int32_t *rows,
                    const int32_t *cols, const double *prior_p, const rb_params *params,
                    int32_t device) {
    g_last_error.clear();
    if (!out) return fail(RB_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (M < 1 || N < 1) return fail(RB_E_SHAPE, "M and N must be >= 1");
    if (nnz < 0) return fail(RB_E_INVALID_ARG, "nnz must be >= 0");
    if (nnz > 0 && (!rows || !cols)) return fail(RB_E_INVALID_ARG, "rows/cols is NULL");
    if (!prior_p) return fail(RB_E_INVALID_ARG, "prior_p is NULL");
    if (device < 0) return fail(RB_E_INVALID_ARG, "device must be >= 0");
    if (nnz > (int64_t)M * (int64_t)N) return fail(RB_E_SHAPE, "nnz exceeds M*N");
    rb_status st = check_params(params);
    if (st != RB_OK) return st;
    for (int64_t k = 0; k < nnz; ++k)
        if (rows[k] < 0 || rows[k] >= M || cols[k] < 0 || cols[k] >= N)
            return fail(RB_E_SHAPE, "entry " + std::to_string(k) + " out of range");
    for (int32_t j = 0; j < N; ++j) {
        const double p = prior_p[j];
        if (!std::isfinite(p)) return fail(RB_E_PRIOR_RANGE, "prior " + std::to_string(j) + " not finite");
        if (!(p > 0.0 && p < 1.0)) return fail(RB_E_PRIOR_RANGE, "prior " + std::to_string(j) + " outside (0, 1)");
    }
    // sort (row, col) pairs; duplicates would silently cancel over F_2
    std::vector<std::pair<int32_t, int32_t>> rc((size_t)nnz);
    for (int64_t k = 0; k < nnz; ++k) rc[k] = {rows[k], cols[k]};
    std::sort(rc.begin(), rc.end());
    for (int64_t k = 1; k < nnz; ++k)
        if (rc[k] == rc[k - 1])
            return fail(RB_E_DUPLICATE_ENTRY, "duplicate entry (" + std::to_string(rc[k].first) + ", " +
                                                  std::to_string(rc[k].second) + ")");

    rb_ctx *c = new (std::nothrow) rb_ctx();
    if (!c) return fail(RB_E_OOM, "host allocation failed");
    c->device = device;
    c->M = M;
    c->N = N;
    c->E = nnz;
    c->params = *params;
    c->rowptr.assign((size_t)M + 1, 0);
    c->colidx.resize((size_t)nnz);
    for (int64_t k = 0; k < nnz; ++k) {
        c->rowptr[rc[k].first + 1]++;
        c->colidx[k] = rc[k].second;
    }
    for (int32_t i = 0; i < M; ++i) c->rowptr[i + 1] += c->rowptr[i];
    c->colptr.assign((size_t)N + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) c->colptr[rc[k].second + 1]++;
    for (int32_t j = 0; j < N; ++j) c->colptr[j + 1] += c->colptr[j];
    c->rowidx.resize((size_t)nnz);
    c->cpos.resize((size_t)nnz);
    {
        std::vector<int64_t> fill(c->colptr.begin(), c->colptr.end() - 1);
        for (int32_t i = 0; i < M; ++i)  // rows ascending => column lists ascending in i
            for (int64_t e = c->rowptr[i]; e < c->rowptr[i + 1]; ++e) {
                const int32_t j = c->colidx[e];
                c->rowidx[fill[j]] = i;
                c->cpos[fill[j]] = (int32_t)(e - c->rowptr[i]);
                ++fill[j];
            }
    }
    for (int32_t i = 0; i < M; ++i) c->max_row = std::max<int32_t>(c->max_row, (int32_t)(c->rowptr[i + 1] - c->rowptr[i]));
    for (int32_t j = 0; j < N; ++j) c->max_col = std::max<int32_t>(c->max_col, (int32_t)(c->colptr[j + 1] - c->colptr[j]));
    c->w.resize((size_t)N);
    for (int32_t j = 0; j < N; ++j) c->w[j] = (float)std::log((1.0 - prior_p[j]) / prior_p[j]);

    // pick the cheapest built-in configuration the graph fits
    int best = -1;
    double best_cost = 0.0;
    for (int v = 0; v < rb::num_variants(); ++v) {
        const rb::TileShape s = rb::variant_shape(v);
        if (!variant_fits(c, s)) continue;
        const double cost = variant_cost(s);
        if (best < 0 || cost < best_cost) {
            best = v;
            best_cost = cost;
        }
    }
    if (best < 0) {
        const std::string msg = "graph exceeds every built-in kernel configuration (M=" +
                                std::to_string(M) + ", N=" + std::to_string(N) +
                                ", max row degree " + std::to_string(c->max_row) +
                                ", max column degree " + std::to_string(c->max_col) + ")";
        delete c;
        return fail(RB_E_UNSUPPORTED, msg);
    }

    auto bail = [&](rb_status s2) {
        rb_destroy(c);
        return s2;
    };
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return bail(hip_fail(e, "hipSetDevice"));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return bail(hip_fail(e, "hipGetDeviceProperties"));
    c->num_cu = prop.multiProcessorCount;
    const int R = params->num_legs;
    if ((e = hipMalloc(&c->d_w, sizeof(float) * (size_t)N)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(w)"));
    if ((e = hipMalloc(&c->d_gamma, sizeof(float) * (size_t)N * (size_t)R)) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc(gamma)"));
    if ((e = hipMalloc(&c->d_queue, sizeof(unsigned long long))) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc(queue)"));
    if ((e = hipMemcpy(c->d_w, c->w.data(), sizeof(float) * (size_t)N, hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(e, "copy w"));
    if ((e = rb::launch_gamma_table(c->d_gamma, R, N, params->seed, params->gamma_first, params->gamma_lo,
                                    params->gamma_hi, nullptr)) != hipSuccess)
        return bail(hip_fail(e, "gamma table kernel"));
    if ((e = hipDeviceSynchronize()) != hipSuccess) return bail(hip_fail(e, "gamma table sync"));
    st = build_plan(c, best);
    if (st != RB_OK) return bail(st);
    *out = c;
    return RB_OK;
}

void rb_destroy(rb_ctx *c) {
    if (!c) return;
    if (c->d_w || c->d_gamma || c->d_queue || c->d_lam_off || c->d_mu_off) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(c->d_w);
        (void)hipFree(c->d_gamma);
        (void)hipFree(c->d_queue);
        (void)hipFree(c->d_lam_off);
        (void)hipFree(c->d_mu_off);
    }
    delete c;
}

static rb::GroupArgs base_args(const rb_ctx *c, int64_t B, const uint8_t *syn) {
    rb::GroupArgs a{};
    a.M = c->M;
    a.N = c->N;
    a.B = B;
    a.syn = syn;
    a.w = c->d_w;
    a.gamma = c->d_gamma;
    a.lam_off = c->d_lam_off;
    a.mu_off = c->d_mu_off;
    a.queue = c->d_queue;
    a.num_legs = c->params.num_legs;
    a.iters_first = c->params.iters_first;
    a.iters_leg = c->params.iters_leg;
    a.num_solutions = c->params.num_solutions;
    a.max_total_iters = c->params.max_total_iters;
    a.L = c->params.llr_clip;
    a.slot_bytes = c->slot_bytes;
    a.lampad_off = c->lampad_off;
    a.mupad_off = c->mupad_off;
    a.mu0_off = c->mu0_off;
    a.scale = 1.0f;
    return a;
}

static int grid_for(const rb_ctx *c, int64_t B, int trace) {
    const int shots_per_block = 64 / c->shape.G;
    const int64_t need = (B + shots_per_block - 1) / shots_per_block;
    const int64_t full = (int64_t)c->blocks_per_cu[trace] * c->num_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, full));
}

rb_status rb_decode(rb_ctx *c, int64_t B, const uint8_t *d_syn, uint8_t *d_corr, uint8_t *d_conv,
                    int32_t *d_legs, int32_t *d_iters, double *d_weight, float *d_final_llr,
                    void *stream) {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (B < 0) return fail(RB_E_INVALID_ARG, "B must be >= 0");
    if (B == 0) return RB_OK;
    if (!d_syn || !d_corr || !d_conv || !d_legs || !d_iters)
        return fail(RB_E_INVALID_ARG, "a required device pointer is NULL");
    rb::GroupArgs a = base_args(c, B, d_syn);
    a.corr = d_corr;
    a.conv = d_conv;
    a.legs = d_legs;
    a.iters = d_iters;
    a.weight = d_weight;
    a.final_llr = d_final_llr;
    hipStream_t s = (hipStream_t)stream;
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(rb::launch_reset_queue(c->d_queue, s), "queue reset");
    RB_HIP(rb::launch_group(c->variant, c->params.anchor == RB_ANCHOR_PRIOR, false, a,
                            grid_for(c, B, 0), (size_t)c->lds_bytes, s),
           "relay kernel launch");
    return RB_OK;
}

rb_status rb_trace(rb_ctx *c, int64_t B, const uint8_t *d_syn, const float *d_gamma, float scale,
                   int32_t T, float *d_trace, void *stream) {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (B < 0 || T < 0) return fail(RB_E_INVALID_ARG, "B and T must be >= 0");
    if (!std::isfinite(scale)) return fail(RB_E_NONFINITE, "scale must be finite");
    if (B == 0) return RB_OK;
    if (!d_syn || !d_gamma || !d_trace) return fail(RB_E_INVALID_ARG, "a required device pointer is NULL");
    rb::GroupArgs a = base_args(c, B, d_syn);
    a.trace_gamma = d_gamma;
    a.scale = scale;
    a.trace_T = T;
    a.trace = d_trace;
    hipStream_t s = (hipStream_t)stream;
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(rb::launch_reset_queue(c->d_queue, s), "queue reset");
    RB_HIP(rb::launch_group(c->variant, false, true, a, grid_for(c, B, 1), (size_t)c->lds_bytes, s),
           "relay trace launch");
    return RB_OK;
}

rb_status rb_get_llr(const rb_ctx *c, float *host_w) {
    if (!c || !host_w) return fail(RB_E_INVALID_ARG, "NULL argument");
    std::memcpy(host_w, c->w.data(), sizeof(float) * (size_t)c->N);
    return RB_OK;
}

rb_status rb_get_gamma_table(const rb_ctx *c, float *host_gamma) {
    if (!c || !host_gamma) return fail(RB_E_INVALID_ARG, "NULL argument");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipMemcpy(host_gamma, c->d_gamma, sizeof(float) * (size_t)c->N * (size_t)c->params.num_legs,
                     hipMemcpyDeviceToHost),
           "copy gamma table");
    return RB_OK;
}

rb_status rb_get_info(const rb_ctx *c, rb_info *info) {
    if (!c || !info) return fail(RB_E_INVALID_ARG, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->M = c->M;
    info->N = c->N;
    info->num_edges = c->E;
    info->max_row_degree = c->max_row;
    info->max_col_degree = c->max_col;
    info->variant = c->variant;
    info->lanes_per_shot = c->shape.G;
    info->checks_per_lane = c->shape.CPT;
    info->row_slots = c->shape.DC;
    info->cols_per_lane = c->shape.VPT;
    info->col_slots = c->shape.DV;
    info->shots_per_block = 64 / c->shape.G;
    info->threads_per_block = 64;
    info->lds_bytes_per_block = c->lds_bytes;
    info->blocks_per_cu = c->blocks_per_cu[0];
    info->grid_blocks = c->blocks_per_cu[0] * c->num_cu;
    info->num_variants = rb::num_variants();
    return RB_OK;
}

rb_status rb_set_variant(rb_ctx *c, int32_t v) {
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (v < 0 || v >= rb::num_variants()) return fail(RB_E_INVALID_ARG, "variant out of range");
    if (!variant_fits(c, rb::variant_shape(v))) return fail(RB_E_UNSUPPORTED, "graph does not fit the variant");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipDeviceSynchronize(), "sync before re-plan");
    return build_plan(c, v);
}

rb_status rb_sync_status(rb_ctx *c) {
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipDeviceSynchronize(), "device synchronize");
    RB_HIP(hipGetLastError(), "asynchronous error");
    return RB_OK;
}

}  // extern "C"
