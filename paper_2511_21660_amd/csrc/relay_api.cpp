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
#include <array>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <memory>
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

// No C++ exception leaves the C ABI: every entry point that returns an
// rb_status is a function-try-block whose handler calls host_exception(),
// which turns a host allocation failure (std::bad_alloc from a table, a plan
// or a message) into RB_E_OOM and any other exception into RB_E_INTERNAL.
// Contexts under construction are held by owning pointers, so nothing leaks
// on the way out.
rb_status host_exception() noexcept {
    const char *msg = "host exception";
    rb_status st = RB_E_INTERNAL;
    try {
        throw;
    } catch (const std::bad_alloc &) {
        msg = "host allocation failed";
        st = RB_E_OOM;
    } catch (const std::exception &ex) {
        try {
            g_last_error = std::string("host exception: ") + ex.what();
            return st;
        } catch (...) {
        }
    } catch (...) {
    }
    try {
        g_last_error = msg;
    } catch (...) {
    }
    return st;
}

struct CtxDeleter {
    void operator()(rb_ctx *c) const { rb_destroy(c); }
};
using CtxPtr = std::unique_ptr<rb_ctx, CtxDeleter>;

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
    std::vector<double> w64;      // [N] log((1-p)/p) in FP64 (the binary16 mode rounds it once)
    // device
    float *d_w = nullptr;
    float *d_gamma = nullptr;        // [R][N]
    uint32_t *d_lam_off = nullptr;
    uint32_t *d_mu_off = nullptr;
    unsigned long long *d_queue = nullptr;
    // plan: variants [0, num_variants) are group-kernel tiles, then block-kernel shapes
    int variant = -1;
    bool block = false;
    rb::TileShape shape{};
    rb::BlockShape bshape{};
    uint32_t red_off = 0, slack_off = 0;
    int32_t *d_chk_row = nullptr, *d_wave_deg = nullptr, *d_wave_base = nullptr;
    int32_t *d_slot_col = nullptr, *d_chk_split = nullptr;
    float *d_w_slot = nullptr;      // [TPB*VPT] w by fault slot (block and large-graph kernels)
    float *d_gamma_slot = nullptr;  // [R][TPB*VPT] gamma by fault slot (block and large-graph kernels)
    // binary16 mode (rb_params.precision = RB_PREC_F16): binary16 block kernel
    bool h16 = false;
    uint16_t *d_w16_slot = nullptr;      // [TPB*VPT] w by slot, binary16 bits
    uint16_t *d_gamma16_slot = nullptr;  // [R][TPB*VPT] gamma by slot, binary16 bits
    uint32_t L16 = 0, stage_off = 0;
    float prior_scale = 1.0f;       // s in Lambda(0) = s * w (rb_set_prior_scale)
    // longest-first shot lists for single-code decodes (rb_reserve)
    void *d_ws = nullptr;
    int64_t ws_capacity = 0;
    int32_t *d_code_m = nullptr;  // [ncodes] rows per code (1 entry for a single code)
    // mixed-code context (rb_create_multi)
    bool multi = false;
    std::vector<rb_ctx *> subs;
    rb::CodeStatic *d_codes = nullptr;
    unsigned long long *d_queues = nullptr;
    // families: codes with the same graph and tile (one shot list each)
    int32_t nfam = 0;
    int32_t *d_code_fam = nullptr, *d_fam_rep = nullptr, *d_fam_size = nullptr;
    // w and gamma of every code, the members of each family stored contiguously,
    // and each code's member index within its family
    float *d_wcat = nullptr, *d_gcat = nullptr;
    int32_t *d_code_member = nullptr;
    int32_t m_max = 0, n_max = 0;
    // large-graph kernel (compressed messages): CSR / CSC copies and tables
    bool large = false;
    rb::LargeShape lshape{};
    int32_t lrounds = 0, nrec = 0;
    uint32_t chk_off = 0;
    int32_t *d_lrowptr = nullptr, *d_chk_of = nullptr;
    int2 *d_fcol = nullptr;      // [TPB*VR] (first entry, degree) per fault slot
    float *d_lambda0 = nullptr;  // [blocks_per_cu * num_cu][N] large-graph kernel workspace
    uint16_t *d_col16 = nullptr;            // row chunks of fault slots
    int32_t *d_rbase = nullptr, *d_rrec = nullptr;
    uint32_t *d_fedge = nullptr, *d_frec = nullptr;
    // CSR / CSC on the device (training kernels)
    int32_t *d_rowptr = nullptr, *d_colidx = nullptr, *d_colptr = nullptr, *d_cedge = nullptr;
    uint32_t lampad_off = 0, mupad_off = 0, mu0_off = 0, half_off = 0;
    int lds_bytes = 0;
    int blocks_per_cu[2] = {0, 0};  // [trace]
    int num_cu = 0;
};

namespace {

int ceil_div(int a, int b) { return (a + b - 1) / b; }

struct Layout {
    uint32_t lampad_off, mupad_off, mu0_off;  // byte offsets within a slot's region (word w -> 4 * SPH * w)
    uint32_t word;                            // bytes between consecutive words of a slot (4 * SPH)
    uint32_t half_off;                        // bytes between the two half-wave regions
    int sph;                                  // slots per half-wave region
    int ks;                                   // words between the messages of steps k, k+1 (G * CPT)
    int lds_bytes;
};

// Slot layout in words: Lambda[0..G*VPT) (faults j >= N are spare words the
// padded lanes write), +inf pad, -0 pad, then the check messages step-major:
// message k of check position q (= check index) at word k * G*CPT + q.  The SPH = 32/G slots of a half-wave (1 for G >= 32) are
// interleaved word by word in one region; the wave's NS = 64/G slots fill
// NS/SPH regions.
Layout slot_layout(const rb::TileShape &s, int N) {
    Layout l{};
    const uint32_t ns = (uint32_t)(64 / s.G);
    const uint32_t sph = s.G >= 32 ? 1u : 32u / (uint32_t)s.G;
    const uint32_t nl = (uint32_t)std::max(N, s.G * s.VPT);
    l.sph = (int)sph;
    l.word = 4u * sph;
    l.ks = s.G * s.CPT;
    l.lampad_off = l.word * nl;
    l.mupad_off = l.word * (nl + 1);
    l.mu0_off = l.word * (nl + 2);
    const uint64_t words = (uint64_t)(nl + 2) + (uint64_t)s.G * s.CPT * s.DC;
    const uint64_t region = words * l.word;
    l.half_off = region > (1u << 30) ? (1u << 30) : (uint32_t)region;
    const uint64_t bytes = region * (ns / sph);
    l.lds_bytes = bytes > (1u << 30) ? (1 << 30) : (int)bytes;
    return l;
}

bool variant_fits(const rb_ctx *c, const rb::TileShape &s) {
    if (ceil_div(c->M, s.G) > s.CPT || ceil_div(c->N, s.G) > s.VPT) return false;
    if (c->max_row > s.DC || c->max_col > s.DV) return false;
    return slot_layout(s, c->N).lds_bytes <= 64 * 1024;
}

// Initial choice before any measurement: estimated lane-operations per
// shot-iteration (a slot pays for all of its padded rows and columns: about
// 10 per check edge, 2 per fault edge, 6 per fault), discounted by the
// occupancy the register budget allows.  rb_autotune replaces this guess by
// measurement.
double variant_cost(const rb::TileShape &s) {
    const double work = (double)s.G * (10.0 * s.CPT * s.DC + 2.0 * s.VPT * s.DV + 6.0 * s.VPT);
    const double occ = s.waves >= 4 ? 1.0 : s.waves == 3 ? 1.1 : s.waves == 2 ? 1.3 : 1.8;
    return work * occ;
}

// Deterministic generator for the plan's local search (splitmix64).
struct PlanRng {
    uint64_t x;
    uint32_t below(uint32_t n) {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (uint32_t)(z % n);
    }
};

// Edge order within each check for a group-kernel tile (free: the check
// update does not depend on it).  A wave's access is served in two halves of
// 32 lanes, each costing the largest number of distinct words on one LDS
// bank.  The slots of a half are interleaved word by word, so each slot owns
// ncls = min(G, 32) banks (its "classes", word index mod ncls) and a gather
// costs, per half, the largest number of the slot's lanes on one class (all
// slots of a wave run the same tables; for G = 64 the slot spans both
// halves).  Step k of check row c gathers Lambda of the fault at step k of
// each of the G checks g + G*c (class: fault index mod ncls; steps without an
// edge gather the pad cell).  The fault side does not depend on the order:
// messages are stored step-major with a step stride that is a multiple of
// ncls, so a message's class is its check's position mod ncls.  Random swaps
// of two steps of one check (edges or pads), accepted by a simulated-annealing
// rule, lower the summed cost.  Returns the step of every CSR edge.
std::vector<int32_t> group_edge_order(const rb_ctx *c, const rb::TileShape &s, const Layout &lay) {
    const int ncls = std::min(s.G, 32), DC = s.DC;
    std::vector<int32_t> pos((size_t)c->E), at((size_t)c->M * DC, -1);  // edge -> step; (check, step) -> edge
    for (int32_t i = 0; i < c->M; ++i)
        for (int64_t e = c->rowptr[i]; e < c->rowptr[i + 1]; ++e) {
            pos[(size_t)e] = (int32_t)(e - c->rowptr[i]);
            at[(size_t)i * DC + pos[(size_t)e]] = (int32_t)e;
        }
    if (c->E == 0) return pos;
    const int lampad_cls = (int)((lay.lampad_off / lay.word) % (uint32_t)ncls);
    const int nh = s.G == 64 ? 2 : 1;  // halves a slot spans
    int h[2][32];
    auto ccost = [&](int cc, int k) {
        bool padh[2] = {false, false};
        for (int x = 0; x < nh; ++x)
            for (int q = 0; q < ncls; ++q) h[x][q] = 0;
        for (int g = 0; g < s.G; ++g) {
            const int x = g >> 5, i = g + s.G * cc;
            const int e = i < c->M ? at[(size_t)i * DC + k] : -1;
            if (e < 0)
                padh[x] = true;
            else
                ++h[x][c->colidx[(size_t)e] % ncls];
        }
        int m = 0;
        for (int x = 0; x < nh; ++x) {
            if (padh[x]) ++h[x][lampad_cls];
            int mx = 0;
            for (int q = 0; q < ncls; ++q) mx = std::max(mx, h[x][q]);
            m += mx;
        }
        return m;
    };
    std::vector<int> C((size_t)s.CPT * DC);
    for (int cc = 0; cc < s.CPT; ++cc)
        for (int k = 0; k < DC; ++k) C[(size_t)cc * DC + k] = ccost(cc, k);
    PlanRng rng{0xBA4C5EEDull};
    const int64_t iters = std::min<int64_t>(4000000, 3000 * c->E);
    for (int64_t it = 0; it < iters; ++it) {
        const int i = (int)rng.below((uint32_t)c->M);
        const int a = (int)rng.below((uint32_t)DC), b = (int)rng.below((uint32_t)DC);
        int32_t &ea = at[(size_t)i * DC + a], &eb = at[(size_t)i * DC + b];
        if (a == b || (ea < 0 && eb < 0)) continue;
        const int cc = i / s.G;
        const size_t c1 = (size_t)cc * DC + a, c2 = (size_t)cc * DC + b;
        const int before = C[c1] + C[c2];
        std::swap(ea, eb);
        const int nc1 = ccost(cc, a), nc2 = ccost(cc, b);
        const int after = nc1 + nc2;
        const double temp = 1.0 * (1.0 - (double)it / (double)iters);
        bool take = after <= before;
        if (!take && temp > 0.0) take = (double)rng.below(1u << 20) < std::exp((before - after) / temp) * (double)(1u << 20);
        if (take) {
            C[c1] = nc1;
            C[c2] = nc2;
        } else {
            std::swap(ea, eb);
        }
    }
    for (int32_t i = 0; i < c->M; ++i)
        for (int k = 0; k < DC; ++k)
            if (at[(size_t)i * DC + k] >= 0) pos[(size_t)at[(size_t)i * DC + k]] = k;
    return pos;
}

// Host tables of a group-kernel tile: per lane, two 16-bit slot-relative LDS
// byte offsets per word (entry 2q in the low half, 2q+1 in the high half).
// lam: [G][ceil(CPT*DC/2)], the Lambda gathers of each check step (pad: the
// +inf cell); mu: [G][ceil(VPT*DV/2)], the message gathers of each fault in
// ascending check order (pad: the -0 cell).
struct GroupTables {
    Layout lay{};
    std::vector<uint32_t> lam, mu;
};

GroupTables group_tables(const rb_ctx *c, const rb::TileShape &s) {
    GroupTables T;
    T.lay = slot_layout(s, c->N);
    const Layout &lay = T.lay;
    const int nl = s.CPT * s.DC, nm = s.VPT * s.DV;
    const int nlp = (nl + 1) / 2, nmp = (nm + 1) / 2;
    std::vector<uint16_t> lam16((size_t)s.G * nlp * 2, (uint16_t)lay.lampad_off);
    std::vector<uint16_t> mu16((size_t)s.G * nmp * 2, (uint16_t)lay.mupad_off);
    const std::vector<int32_t> pos = group_edge_order(c, s, lay);  // CSR edge -> step in its check
    for (int g = 0; g < s.G; ++g) {
        for (int cc = 0; cc < s.CPT; ++cc) {
            const int i = g + s.G * cc;
            if (i >= c->M) continue;
            for (int64_t e = c->rowptr[i]; e < c->rowptr[i + 1]; ++e)
                lam16[(size_t)g * nlp * 2 + cc * s.DC + pos[(size_t)e]] =
                    (uint16_t)(lay.word * (uint32_t)c->colidx[e]);
        }
        for (int vv = 0; vv < s.VPT; ++vv) {
            const int j = g + s.G * vv;
            if (j >= c->N) continue;
            const int64_t b = c->colptr[j], e = c->colptr[j + 1];
            for (int64_t k = 0; k < e - b; ++k) {
                const int i = c->rowidx[b + k];
                const int p = pos[(size_t)(c->rowptr[i] + c->cpos[b + k])];
                const uint32_t word = (uint32_t)p * (uint32_t)lay.ks + (uint32_t)i;
                mu16[(size_t)g * nmp * 2 + vv * s.DV + k] = (uint16_t)(lay.mu0_off + lay.word * word);
            }
        }
    }
    T.lam.resize((size_t)s.G * nlp);
    T.mu.resize((size_t)s.G * nmp);
    for (size_t q = 0; q < T.lam.size(); ++q) T.lam[q] = (uint32_t)lam16[2 * q] | ((uint32_t)lam16[2 * q + 1] << 16);
    for (size_t q = 0; q < T.mu.size(); ++q) T.mu[q] = (uint32_t)mu16[2 * q] | ((uint32_t)mu16[2 * q + 1] << 16);
    return T;
}

rb_status build_plan(rb_ctx *c, int v) {
    const rb::TileShape s = rb::variant_shape(v);
    const GroupTables T = group_tables(c, s);
    const Layout &lay = T.lay;
    const std::vector<uint32_t> &lam = T.lam, &mu = T.mu;
    (void)hipFree(c->d_lam_off);
    (void)hipFree(c->d_mu_off);
    c->d_lam_off = nullptr;
    c->d_mu_off = nullptr;
    RB_HIP(hipMalloc(&c->d_lam_off, lam.size() * 4), "hipMalloc(lam_off)");
    RB_HIP(hipMalloc(&c->d_mu_off, mu.size() * 4), "hipMalloc(mu_off)");
    RB_HIP(hipMemcpy(c->d_lam_off, lam.data(), lam.size() * 4, hipMemcpyHostToDevice), "copy lam_off");
    RB_HIP(hipMemcpy(c->d_mu_off, mu.data(), mu.size() * 4, hipMemcpyHostToDevice), "copy mu_off");
    {
        size_t st_lds = 0;
        RB_HIP(rb::variant_static_lds(v, &st_lds), "kernel attributes");
        if (st_lds != 0) return fail(RB_E_DEVICE, "internal: group kernel uses static LDS");
    }
    c->variant = v;
    c->shape = s;
    c->lampad_off = lay.lampad_off;
    c->mupad_off = lay.mupad_off;
    c->mu0_off = lay.mu0_off;
    c->half_off = lay.half_off;
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

int total_variants() { return rb::num_variants() + rb::num_block_variants() + rb::num_large_variants(); }

struct BlockLayout {
    uint32_t lampad_off, mupad_off, red_off, mu0_off, slack_off;
    int lds_bytes;
    int npad;
};

// Block-kernel LDS: Lambda[TPB*VPT], +inf cell, -0 cell, reduction scratch,
// then the wave-ELL message rows (wave w: wave_deg[w] rows of 64 words).
BlockLayout block_layout(const rb::BlockShape &s, int64_t msg_words) {
    BlockLayout l{};
    l.npad = s.TPB * s.VPT;
    l.lampad_off = 4u * (uint32_t)l.npad;
    l.mupad_off = l.lampad_off + 4u;
    l.red_off = (l.mupad_off + 4u + 15u) & ~15u;  // block-OR flags (red_off + 8 * TPB/64) 16-byte aligned
    // scratch: TPB/64 doubles (block sums), TPB/64 words (block OR), shot index
    l.mu0_off = (l.red_off + 12u * (uint32_t)(s.TPB / 64) + 8u + 15u) & ~15u;
    l.slack_off = l.mu0_off + 4u * (uint32_t)msg_words;
    const int64_t bytes = (int64_t)l.mu0_off + 4 * (msg_words + (rb::kBlockChunk - 1) * 64);
    l.lds_bytes = bytes > (1 << 30) ? (1 << 30) : (int)bytes;
    return l;
}

// One thread's share of a check: edges rowptr[row] + b .. rowptr[row] + e.
// A long check may be split over two adjacent lanes (2p, 2p+1) of a wave,
// which combine their partial minima and parities.
struct LaneSeg {
    int32_t row = -1, b = 0, e = 0;
    bool split = false, first = true;
};

// Rows longer than this are split in two while spare lanes remain (longest
// first), so that no wave is held up by a few very long rows.
constexpr int kSplitRowDegree = 32;

// Check placement: segments sorted by decreasing length (stable) form groups
// of 64 lanes of nearly equal length; the groups are placed on waves so that
// the four SIMDs of a CU (wave w runs on SIMD w % 4) get about the same number
// of row chunks (kBlockChunk edges each), largest group first onto the least
// loaded SIMD.  lanes[t] is thread t's segment (row -1: none); wave-ELL row
// counts and first message words per wave.
void block_order(const rb_ctx *c, const rb::BlockShape &s, std::vector<LaneSeg> &lanes,
                 std::vector<int32_t> &wdeg, std::vector<int32_t> &wbase, int64_t &words) {
    auto deg = [&](int32_t i) { return (int32_t)(c->rowptr[i + 1] - c->rowptr[i]); };
    std::vector<int32_t> sorted((size_t)c->M);
    for (int32_t i = 0; i < c->M; ++i) sorted[i] = i;
    std::stable_sort(sorted.begin(), sorted.end(), [&](int32_t x, int32_t y) { return deg(x) > deg(y); });
    int spare = s.TPB - c->M - 1;  // one lane kept free for pair alignment
    std::vector<LaneSeg> pairs, singles;  // pairs: first half of each split row
    for (int32_t i : sorted) {
        const int32_t d = deg(i);
        if (spare > 0 && d > kSplitRowDegree) {
            --spare;
            pairs.push_back({i, 0, (d + 1) / 2, true, true});
        } else {
            singles.push_back({i, 0, d, false, true});
        }
    }
    // merge by decreasing length; a pair starts on an even lane
    std::vector<LaneSeg> seq;
    size_t pi = 0, si = 0;
    while (pi < pairs.size() || si < singles.size()) {
        const bool take_pair = pi < pairs.size() &&
                               (si >= singles.size() || pairs[pi].e >= singles[si].e - singles[si].b);
        if (take_pair && (seq.size() % 2 == 0 || si >= singles.size())) {
            if (seq.size() % 2 == 1) seq.push_back(LaneSeg{});  // idle lane keeps pairs aligned
            const LaneSeg f = pairs[pi++];
            seq.push_back(f);
            seq.push_back({f.row, f.e, deg(f.row), true, false});
        } else {
            seq.push_back(singles[si++]);
        }
    }
    const int nw = s.TPB / 64;
    const int ng = ceil_div((int)seq.size(), 64);
    std::vector<int32_t> gdeg((size_t)ng, 0);
    for (size_t q = 0; q < seq.size(); ++q) gdeg[q / 64] = std::max(gdeg[q / 64], seq[q].e - seq[q].b);
    // Steps the check pass runs for a group of row length d: chunks of
    // kBlockChunk edges, the last one half as wide when at most half remains.
    auto steps = [](int d) {
        int n = 0;
        for (int c = 0; c < d; c += rb::kBlockChunk) n += (c + rb::kBlockChunk / 2 >= d) ? rb::kBlockChunk / 2 : rb::kBlockChunk;
        return n;
    };
    // Groups onto SIMDs: largest first onto the least loaded SIMD, then
    // pairwise swaps between SIMDs while they lower the largest load (then
    // the sum of squared loads).  Within a SIMD the longest group takes the
    // lowest wave index (the wave that the hardware favours when issuing).
    std::vector<int> gorder((size_t)ng);
    for (int g = 0; g < ng; ++g) gorder[g] = g;
    std::stable_sort(gorder.begin(), gorder.end(), [&](int x, int y) { return gdeg[x] > gdeg[y]; });
    std::vector<std::vector<int>> on((size_t)4);
    int64_t load[4] = {0, 0, 0, 0};
    for (int g : gorder) {
        int best = -1;
        for (int q = 0; q < 4; ++q)
            if ((int)on[q].size() < nw / 4 && (best < 0 || load[q] < load[best])) best = q;
        if (best < 0) break;  // more groups than waves: caller rejects (words stays small)
        on[best].push_back(g);
        load[best] += steps(gdeg[g]);
    }
    auto score = [&](const int64_t *l) {
        int64_t mx = 0, sq = 0;
        for (int q = 0; q < 4; ++q) {
            mx = std::max(mx, l[q]);
            sq += l[q] * l[q];
        }
        return mx * (int64_t)1000000 + sq;
    };
    for (bool improved = true; improved;) {
        improved = false;
        for (int q1 = 0; q1 < 4; ++q1)
            for (int q2 = q1 + 1; q2 < 4; ++q2)
                for (size_t a1 = 0; a1 < on[q1].size(); ++a1)
                    for (size_t a2 = 0; a2 < on[q2].size(); ++a2) {
                        const int64_t d = steps(gdeg[on[q1][a1]]) - steps(gdeg[on[q2][a2]]);
                        if (d == 0) continue;
                        int64_t l2[4] = {load[0], load[1], load[2], load[3]};
                        l2[q1] -= d;
                        l2[q2] += d;
                        if (score(l2) < score(load)) {
                            std::swap(on[q1][a1], on[q2][a2]);
                            for (int q = 0; q < 4; ++q) load[q] = l2[q];
                            improved = true;
                        }
                    }
    }
    std::vector<int> group_of_wave((size_t)nw, -1);
    for (int q = 0; q < 4; ++q) {
        std::stable_sort(on[q].begin(), on[q].end(), [&](int x, int y) { return gdeg[x] > gdeg[y]; });
        for (size_t u = 0; u < on[q].size(); ++u) group_of_wave[(size_t)q + 4 * u] = on[q][u];
    }
    lanes.assign((size_t)s.TPB, LaneSeg{});
    wdeg.assign((size_t)nw, 0);
    wbase.assign((size_t)nw, 0);
    for (int w = 0; w < nw; ++w) {
        const int g = group_of_wave[w];
        if (g < 0) continue;
        wdeg[w] = gdeg[g];
        for (int l = 0; l < 64 && (size_t)(64 * g + l) < seq.size(); ++l)
            lanes[(size_t)(64 * w + l)] = seq[(size_t)(64 * g + l)];
    }
    words = 0;
    for (int w = 0; w < nw; ++w) {
        wbase[w] = (int32_t)words;
        words += (int64_t)wdeg[w] * 64;
    }
}

// faults in the order of decreasing column degree (stable): slot s holds order[s]
std::vector<int32_t> fault_order(const rb_ctx *c) {
    std::vector<int32_t> order((size_t)c->N);
    for (int32_t j = 0; j < c->N; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return (c->colptr[x + 1] - c->colptr[x]) > (c->colptr[y + 1] - c->colptr[y]);
    });
    return order;
}

bool block_fits(const rb_ctx *c, const rb::BlockShape &s) {
    if (c->M > s.TPB || ceil_div(c->N, s.TPB) > s.VPT || s.VPT > 16) return false;
    {
        // the first (largest-degree) fault of every band within the band's cap
        const std::vector<int32_t> fo = fault_order(c);
        for (int v = 0; v < s.VPT && (int64_t)v * s.TPB < c->N; ++v) {
            const int32_t j = fo[(size_t)v * s.TPB];
            if (c->colptr[j + 1] - c->colptr[j] > rb::prof_dv(s.prof, v)) return false;
        }
    }
    std::vector<LaneSeg> lanes;
    std::vector<int32_t> wdeg, wbase;
    int64_t words = 0;
    block_order(c, s, lanes, wdeg, wbase, words);
    for (const LaneSeg &g : lanes)
        if (g.e - g.b > s.DCMAX) return false;
    {
        // every segment placed
        int64_t placed = 0;
        for (const LaneSeg &g : lanes)
            if (g.row >= 0) placed += g.e - g.b;
        if (placed != c->E) return false;
    }
    const BlockLayout l = block_layout(s, words);
    if (l.lampad_off + 8u > 65535u) return false;                   // 16-bit Lambda addresses
    if ((int64_t)(l.mu0_off / 4u) + words > 65535) return false;    // 16-bit message indices
    return l.lds_bytes <= 160 * 1024;
}

// 16-byte check records of the large-graph kernel: one per 32 positions of a
// row (at least one per row), each holding the check's state and the sign
// bits of its 32 positions.
int64_t large_records(const rb_ctx *c) {
    int64_t n = 0;
    for (int32_t i = 0; i < c->M; ++i) n += std::max<int64_t>(1, (c->rowptr[i + 1] - c->rowptr[i] + 31) / 32);
    return n;
}

// Large-graph kernel LDS: Lambda[N + 1] (entry N = +inf is the target of row
// padding), the check records, reduction scratch.
struct LargeLayout {
    uint32_t chk_off, red_off;
    int32_t nrec;
    int64_t lds_bytes;
};

LargeLayout large_layout(const rb_ctx *c, const rb::LargeShape &s) {
    LargeLayout l{};
    l.nrec = (int32_t)std::min<int64_t>(large_records(c), INT32_MAX);
    l.chk_off = ((4u * (uint32_t)c->N + 4u) + 15u) & ~15u;
    l.red_off = l.chk_off + 16u * (uint32_t)std::min(l.nrec, rb::kLargeMaxRecords);
    l.lds_bytes = (int64_t)l.red_off + 12 * (s.TPB / 64) + 8;
    return l;
}

bool large_fits(const rb_ctx *c, const rb::LargeShape &s) {
    if (c->M > rb::kLargeRounds * s.TPB || c->N > s.TPB * s.VR) return false;
    if (c->N > 65535 || large_records(c) > rb::kLargeMaxRecords) return false;
    return large_layout(c, s).lds_bytes <= 160 * 1024;
}

// Staging words of the binary16 kernel's packed corrections, after the
// block layout (16-byte aligned).
uint32_t block16_stage_off(int lds_bytes) { return ((uint32_t)lds_bytes + 15u) & ~15u; }
int block16_lds_bytes(const rb::BlockShape &s, int lds_bytes) {
    return (int)block16_stage_off(lds_bytes) + 4 * ((s.TPB * s.VPT + 31) / 32);
}

bool block16_fits(const rb_ctx *c, const rb::BlockShape &s) {
    if (!block_fits(c, s)) return false;
    std::vector<LaneSeg> lanes;
    std::vector<int32_t> wdeg, wbase;
    int64_t words = 0;
    block_order(c, s, lanes, wdeg, wbase, words);
    return block16_lds_bytes(s, block_layout(s, words).lds_bytes) <= 160 * 1024;
}

bool any_fits(const rb_ctx *c, int v) {
    if (c->params.precision == RB_PREC_F16) {
        v -= rb::num_variants();
        return v >= 0 && v < rb::num_block_variants() && block16_fits(c, rb::block_variant_shape(v));
    }
    if (v < rb::num_variants()) return variant_fits(c, rb::variant_shape(v));
    v -= rb::num_variants();
    if (v < rb::num_block_variants()) return block_fits(c, rb::block_variant_shape(v));
    return large_fits(c, rb::large_variant_shape(v - rb::num_block_variants()));
}

template <typename T>
rb_status upload(T **dst, const std::vector<T> &src, const char *what) {
    (void)hipFree(*dst);
    *dst = nullptr;
    RB_HIP(hipMalloc(dst, std::max<size_t>(1, src.size()) * sizeof(T)), what);
    RB_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return RB_OK;
}


// Check lanes within each wave (free: a wave's rows may sit on any of its
// lanes, a split check on an aligned lane pair).  The fault pass's k-th
// gather of band v reads, for every fault of the band, the message of its k-th
// check, whose LDS bank is the owning lane mod 32; lanes are swapped within
// waves (pairs with pairs, single lanes with single lanes) so that, for every
// (band, k), the banks of these messages are as evenly spread as possible,
// which is what place_faults needs to give each half-wave of faults 32
// distinct banks per gather.
void spread_check_lanes(const rb_ctx *c, const rb::BlockShape &s, std::vector<LaneSeg> &lanes) {
    const int TPB = s.TPB, nw = TPB / 64, D = rb::prof_max(s.prof, s.VPT);
    const std::vector<int32_t> fo = fault_order(c);
    std::vector<int32_t> band((size_t)c->N);
    for (int64_t q = 0; q < c->N; ++q) band[(size_t)fo[(size_t)q]] = (int32_t)(q / TPB);
    // per CSR edge: histogram row (band * D + k) of the fault-side gather
    std::vector<int32_t> hrow((size_t)c->E, -1);
    for (int32_t j = 0; j < c->N; ++j)
        for (int64_t q = c->colptr[j]; q < c->colptr[j + 1] && q - c->colptr[j] < D; ++q)
            hrow[(size_t)(c->rowptr[c->rowidx[q]] + c->cpos[q])] = band[j] * D + (int32_t)(q - c->colptr[j]);
    std::vector<int64_t> hist((size_t)s.VPT * D * 32, 0);
    auto apply = [&](const LaneSeg &g, int lane, int d) {
        if (g.row < 0) return;
        for (int32_t q = g.b; q < g.e; ++q) {
            const int32_t h = hrow[(size_t)(c->rowptr[g.row] + q)];
            if (h >= 0) hist[(size_t)h * 32 + (lane & 31)] += d;
        }
    };
    // change of sum(hist^2) if segment g moves from lane a to lane b
    auto delta = [&](const LaneSeg &g, int a, int b) {
        int64_t dd = 0;
        if (g.row < 0 || (a & 31) == (b & 31)) return dd;
        for (int32_t q = g.b; q < g.e; ++q) {
            const int32_t h = hrow[(size_t)(c->rowptr[g.row] + q)];
            if (h < 0) continue;
            int64_t &x = hist[(size_t)h * 32 + (a & 31)], &y = hist[(size_t)h * 32 + (b & 31)];
            dd += (x - 1) * (x - 1) - x * x + (y + 1) * (y + 1) - y * y;
            --x;
            ++y;
        }
        for (int32_t q = g.b; q < g.e; ++q) {  // undo
            const int32_t h = hrow[(size_t)(c->rowptr[g.row] + q)];
            if (h < 0) continue;
            ++hist[(size_t)h * 32 + (a & 31)];
            --hist[(size_t)h * 32 + (b & 31)];
        }
        return dd;
    };
    for (int t = 0; t < TPB; ++t) apply(lanes[(size_t)t], t, 1);
    PlanRng rng{0xC0FFEEull};
    const int64_t iters = 64ll * TPB;
    for (int64_t it = 0; it < iters; ++it) {
        const int w = (int)rng.below((uint32_t)nw);
        int a = (int)rng.below(64), b = (int)rng.below(64);
        const LaneSeg &ga = lanes[(size_t)(64 * w + a)], &gb = lanes[(size_t)(64 * w + b)];
        if (ga.split != gb.split || a == b) continue;
        if (ga.split) {  // move whole pairs
            a &= ~1;
            b &= ~1;
            if (a == b) continue;
        }
        const int width = ga.split ? 2 : 1;
        int64_t dd = 0;
        for (int u = 0; u < width; ++u) {
            // apply each half's move before scoring the next (halves share no edge)
            const LaneSeg &x = lanes[(size_t)(64 * w + a + u)], &y = lanes[(size_t)(64 * w + b + u)];
            const int64_t d1 = delta(x, 64 * w + a + u, 64 * w + b + u);
            apply(x, 64 * w + a + u, -1);
            apply(x, 64 * w + b + u, 1);
            const int64_t d2 = delta(y, 64 * w + b + u, 64 * w + a + u);
            apply(y, 64 * w + b + u, -1);
            apply(y, 64 * w + a + u, 1);
            dd += d1 + d2;
        }
        if (dd <= 0) {
            for (int u = 0; u < width; ++u) std::swap(lanes[(size_t)(64 * w + a + u)], lanes[(size_t)(64 * w + b + u)]);
        } else {
            for (int u = 0; u < width; ++u) {
                const LaneSeg &x = lanes[(size_t)(64 * w + a + u)], &y = lanes[(size_t)(64 * w + b + u)];
                apply(y, 64 * w + a + u, -1);
                apply(y, 64 * w + b + u, 1);
                apply(x, 64 * w + b + u, -1);
                apply(x, 64 * w + a + u, 1);
            }
        }
    }
}

// Fault slots.  Band v holds the faults of degree rank [v*TPB, (v+1)*TPB)
// (fault_order), so slots below N are exactly the real ones.  Within a band
// the faults are placed with the LDS banks in mind: 32 banks (word address
// mod 32), and a wave's access is served in two halves of 32 lanes, each
// costing the largest number of distinct words on one bank:
//  * half-wave of the slot: the fault pass's k-th gather reads the message of
//    each lane's k-th check, whose bank is fixed by the lane that owns that
//    check; faults are grouped 32 to a half-wave so these banks are as
//    distinct as possible (greedy, then a local search over swaps);
//  * lane of the slot within its half: a fault's Lambda word (= its slot)
//    lies in bank slot mod 32; lanes are chosen so that, for every check wave
//    and half, no bank carries more of its edges than the wave has steps,
//    which lets the check-side edge order (order_rows) read one word per bank
//    and half in each step.
std::vector<int32_t> place_faults(const rb_ctx *c, const rb::BlockShape &s, const std::vector<int32_t> &lane_of_edge,
                                  const std::vector<int32_t> &wdeg, const BlockLayout &lay) {
    const int TPB = s.TPB, nw = TPB / 64, ng = 2 * nw;
    const std::vector<int32_t> fo = fault_order(c);
    std::vector<int32_t> slot_col((size_t)TPB * s.VPT, -1);
    const int mu0w = (int)(lay.mu0_off / 4u), padb = (int)((lay.mupad_off / 4u) % 32u);
    // check wave x half x bank: Lambda gathers
    std::vector<int32_t> load((size_t)nw * 64, 0);
    auto load_at = [&](int64_t e, int b) -> int32_t & {
        const int32_t t = lane_of_edge[(size_t)e];
        return load[(size_t)(t / 64) * 64 + (size_t)((t % 64) / 32) * 32 + (size_t)b];
    };
    PlanRng rng{0x5EED5EEDull};
    for (int v = 0; v < s.VPT && (int64_t)v * TPB < c->N; ++v) {
        const int64_t base = (int64_t)v * TPB;
        const int nf = (int)std::min<int64_t>(TPB, c->N - base);
        const int D = rb::prof_dv(s.prof, v);
        // bank of each fault's k-th message (-1: the fault has fewer edges)
        std::vector<int8_t> sig((size_t)nf * D, -1);
        for (int f = 0; f < nf; ++f) {
            const int32_t j = fo[(size_t)(base + f)];
            for (int64_t k = 0; k < c->colptr[j + 1] - c->colptr[j] && k < D; ++k) {
                const int32_t i = c->rowidx[c->colptr[j] + k];
                const int32_t t = lane_of_edge[(size_t)(c->rowptr[i] + c->cpos[c->colptr[j] + k])];
                sig[(size_t)f * D + k] = (int8_t)((mu0w + t) % 32);
            }
        }
        std::vector<int> capg((size_t)ng), member((size_t)ng * 32, -1), fill((size_t)ng, 0);
        for (int g = 0; g < ng; ++g) capg[g] = std::max(0, std::min(32, nf - 32 * g));
        // cnt[(g*D + k)*33 + b]: lanes of half-wave g whose k-th gather hits bank b; b = 32: pads
        std::vector<int> cnt((size_t)ng * D * 33, 0);
        auto cost_gk = [&](int g, int k) {
            const int *q = &cnt[((size_t)g * D + k) * 33];
            int m = q[32] > 0 ? 1 : 0;
            for (int b = 0; b < 32; ++b) m = std::max(m, q[b] + ((b == padb && q[32] > 0) ? 1 : 0));
            return m;
        };
        auto add = [&](int g, int f, int d) {
            for (int k = 0; k < D; ++k) {
                const int b = sig[(size_t)f * D + k];
                cnt[((size_t)g * D + k) * 33 + (b < 0 ? 32 : b)] += d;
            }
        };
        // cost of a group: its gathers' bank cycles, then (to steer the
        // search) the lanes beyond one on any bank
        auto cost_g = [&](int g) {
            int tot = 0;
            for (int k = 0; k < D; ++k) {
                const int *q = &cnt[((size_t)g * D + k) * 33];
                int ex = 0;
                for (int b = 0; b < 32; ++b) ex += std::max(0, q[b] + ((b == padb && q[32] > 0) ? 1 : 0) - 1);
                tot += 256 * cost_gk(g, k) + ex;
            }
            return tot;
        };
        // greedy: each fault to the group where it adds least
        for (int f = 0; f < nf; ++f) {
            int best = -1;
            long long bkey = 0;
            for (int g = 0; g < ng; ++g) {
                if (fill[g] >= capg[g]) continue;
                const int before = cost_g(g);
                add(g, f, 1);
                const int after = cost_g(g);
                add(g, f, -1);
                const long long key = (long long)(after - before) * 4096 + fill[g];
                if (best < 0 || key < bkey) {
                    best = g;
                    bkey = key;
                }
            }
            member[(size_t)best * 32 + fill[best]++] = f;
            add(best, f, 1);
        }
        // local search over swaps of two faults of different groups.  Cost of
        // a group's k-th gather: the largest number of its faults on one bank
        // (pads: one word); objective 64 x the summed costs plus the number of
        // same-bank pairs, so that unavoidable doubles gather in few gathers.
        // Faults that share a bank with another fault of their group are
        // moved, each to the best of a few random partners.
        std::vector<int> gof((size_t)nf), pos_in((size_t)nf);
        for (int g = 0; g < ng; ++g)
            for (int q = 0; q < fill[g]; ++q) {
                gof[(size_t)member[(size_t)g * 32 + q]] = g;
                pos_in[(size_t)member[(size_t)g * 32 + q]] = q;
            }
        auto bin = [&](int f, int k) { const int b = sig[(size_t)f * D + k]; return b < 0 ? 32 : b; };
        auto n_at = [&](int g, int k, int b) { return cnt[((size_t)g * D + k) * 33 + b]; };
        // per gather (g, k): how many banks hold n faults, and the largest n
        std::vector<int> nc((size_t)ng * D * 34, 0), mx((size_t)ng * D, 0);
        for (int g = 0; g < ng; ++g)
            for (int k = 0; k < D; ++k) {
                const size_t cell = (size_t)g * D + k;
                for (int b2 = 0; b2 < 32; ++b2) {
                    const int n = n_at(g, k, b2);
                    ++nc[cell * 34 + (size_t)n];
                    mx[cell] = std::max(mx[cell], n);
                }
            }
        auto cell_cost = [&](size_t cell) { return std::max(mx[cell], cnt[cell * 33 + 32] > 0 ? 1 : 0); };
        auto move = [&](int g, int k, int b2, int d) {  // one fault into (d = 1) or out of (d = -1) bank b2
            const size_t cell = (size_t)g * D + k;
            int &n = cnt[cell * 33 + (size_t)b2];
            if (b2 < 32) {
                --nc[cell * 34 + (size_t)n];
                ++nc[cell * 34 + (size_t)(n + d)];
                if (d > 0 && n + 1 > mx[cell]) mx[cell] = n + 1;
                if (d < 0 && n == mx[cell] && nc[cell * 34 + (size_t)n] == 0) mx[cell] = n - 1;
            }
            n += d;
        };
        auto clash = [&](int f) {  // other faults of f's group in f's banks
            int x = 0;
            for (int k = 0; k < D; ++k) {
                const int b2 = bin(f, k);
                if (b2 < 32) x += n_at(gof[(size_t)f], k, b2) - 1;
            }
            return x;
        };
        auto do_swap = [&](int f1, int f2) {
            const int g1 = gof[(size_t)f1], g2 = gof[(size_t)f2];
            for (int k = 0; k < D; ++k) {
                const int b1 = bin(f1, k), b2 = bin(f2, k);
                if (b1 == b2) continue;
                move(g1, k, b1, -1);
                move(g2, k, b2, -1);
                move(g1, k, b2, 1);
                move(g2, k, b1, 1);
            }
            std::swap(member[(size_t)g1 * 32 + pos_in[(size_t)f1]], member[(size_t)g2 * 32 + pos_in[(size_t)f2]]);
            std::swap(pos_in[(size_t)f1], pos_in[(size_t)f2]);
            gof[(size_t)f1] = g2;
            gof[(size_t)f2] = g1;
        };
        auto objective_delta = [&](int f1, int f2) {
            const int g1 = gof[(size_t)f1], g2 = gof[(size_t)f2];
            int before = 0, pd = 0;
            for (int k = 0; k < D; ++k) {
                const int b1 = bin(f1, k), b2 = bin(f2, k);
                if (b1 == b2) continue;
                before += cell_cost((size_t)g1 * D + k) + cell_cost((size_t)g2 * D + k);
                if (b1 < 32) pd += n_at(g2, k, b1) - (n_at(g1, k, b1) - 1);
                if (b2 < 32) pd += n_at(g1, k, b2) - (n_at(g2, k, b2) - 1);
            }
            do_swap(f1, f2);
            int after = 0;
            for (int k = 0; k < D; ++k)
                if (bin(f1, k) != bin(f2, k)) after += cell_cost((size_t)g1 * D + k) + cell_cost((size_t)g2 * D + k);
            do_swap(f1, f2);  // undo
            return 64 * (after - before) + pd;
        };
        const long long iters = 400ll * nf;
        for (long long it = 0; it < iters && nf > 32; ++it) {
            const int f1 = (int)rng.below((uint32_t)nf);
            if (clash(f1) == 0) continue;
            int best = -1, bd = 1;
            for (int tr = 0; tr < 8; ++tr) {
                const int f2 = (int)rng.below((uint32_t)nf);
                if (gof[(size_t)f2] == gof[(size_t)f1]) continue;
                const int d = objective_delta(f1, f2);
                if (d < bd || (d == bd && rng.below(2))) {
                    best = f2;
                    bd = d;
                }
            }
            if (best >= 0 && bd <= 0) do_swap(f1, best);
        }
        // lanes within each half-wave: bank = lane, balancing the check side
        for (int g = 0; g < ng; ++g) {
            std::vector<int> fs(member.begin() + (ptrdiff_t)g * 32, member.begin() + (ptrdiff_t)g * 32 + fill[g]);
            auto degf = [&](int f) { const int32_t j = fo[(size_t)(base + f)]; return c->colptr[j + 1] - c->colptr[j]; };
            std::stable_sort(fs.begin(), fs.end(), [&](int x, int y) { return degf(x) > degf(y); });
            std::vector<char> used((size_t)capg[g], 0);
            for (int f : fs) {
                const int32_t j = fo[(size_t)(base + f)];
                int best = -1;
                long long bkey = 0;
                for (int l = 0; l < capg[g]; ++l) {
                    if (used[l]) continue;
                    long long over = LLONG_MIN, sum = 0;
                    for (int64_t q = c->colptr[j]; q < c->colptr[j + 1]; ++q) {
                        const int64_t e = c->rowptr[c->rowidx[q]] + c->cpos[q];
                        const long long ld = load_at(e, l);
                        over = std::max(over, ld + 1 - (long long)wdeg[lane_of_edge[(size_t)e] / 64]);
                        sum += ld;
                    }
                    if (c->colptr[j] == c->colptr[j + 1]) over = 0;  // an empty column loads no bank
                    const long long key = over * (1ll << 32) + sum;
                    if (best < 0 || key < bkey) {
                        best = l;
                        bkey = key;
                    }
                }
                used[best] = 1;
                slot_col[(size_t)(base + 32 * g + best)] = j;
                for (int64_t q = c->colptr[j]; q < c->colptr[j + 1]; ++q)
                    ++load_at(c->rowptr[c->rowidx[q]] + c->cpos[q], best);
            }
        }
    }
    return slot_col;
}

// Edge order within the rows of each wave (free: the check update does not
// depend on it).  Step k of a wave gathers Lambda of edge k of its 64 rows.
// The order is a proper edge colouring, with wdeg colours (= steps), of the
// bipartite multigraph lanes x (bank, half), where half is the lane's half of
// the wave: every step then reads at most one word per bank in each half, the
// conflict-free rate.  Such a colouring exists when no (bank, half) carries
// more than wdeg of the wave's edges (Koenig's edge-colouring theorem); it is
// built edge by edge, swapping the two colours along an alternating path when
// the colours free at the two ends differ.  An edge whose (bank, half) is full
// takes the free step of its lane with the fewest such extra edges.
// epos[e] = step of CSR edge e; col16 = Lambda byte address per (thread, step).
void order_rows(const rb_ctx *c, const rb::BlockShape &s, const std::vector<LaneSeg> &lanes,
                const std::vector<int32_t> &wdeg, const std::vector<int32_t> &slot_of,
                std::vector<int32_t> &epos, std::vector<uint16_t> &col16) {
    const int nw = s.TPB / 64;
    for (int w = 0; w < nw; ++w) {
        const int D = wdeg[w];
        if (D == 0) continue;
        struct Ed {
            int u, v;
            int64_t e;
        };
        std::vector<Ed> ed;
        for (int l = 0; l < 64; ++l) {
            const LaneSeg &g = lanes[(size_t)(64 * w + l)];
            if (g.row < 0) continue;
            for (int32_t q = g.b; q < g.e; ++q) {
                const int64_t e = c->rowptr[g.row] + q;
                const int b = slot_of[c->colidx[e]] & 31;
                ed.push_back({l, 64 + 2 * b + (l >> 5), e});
            }
        }
        std::vector<int> at((size_t)128 * D, -1), col(ed.size(), -1);
        auto free_at = [&](int x) {
            for (int k = 0; k < D; ++k)
                if (at[(size_t)x * D + k] < 0) return k;
            return -1;
        };
        std::vector<int> path;
        for (size_t q = 0; q < ed.size(); ++q) {
            int u = ed[q].u, v = ed[q].v;
            const int a = free_at(u);
            const int b = free_at(v);
            if (b < 0) continue;  // (bank, half) full: placed below
            int k = a;
            if (at[(size_t)v * D + a] >= 0) {
                if (at[(size_t)u * D + b] < 0) {
                    k = b;
                } else {
                    // swap colours a and b along the alternating path from v
                    path.clear();
                    int x = v, cc = a;
                    while (at[(size_t)x * D + cc] >= 0) {
                        const int ej = at[(size_t)x * D + cc];
                        path.push_back(ej);
                        x = ed[ej].u == x ? ed[ej].v : ed[ej].u;
                        cc = cc == a ? b : a;
                    }
                    for (int ej : path) {
                        at[(size_t)ed[ej].u * D + col[ej]] = -1;
                        at[(size_t)ed[ej].v * D + col[ej]] = -1;
                    }
                    for (int ej : path) {
                        col[ej] = col[ej] == a ? b : a;
                        at[(size_t)ed[ej].u * D + col[ej]] = ej;
                        at[(size_t)ed[ej].v * D + col[ej]] = ej;
                    }
                }
            }
            col[q] = k;
            at[(size_t)u * D + k] = (int)q;
            at[(size_t)v * D + k] = (int)q;
        }
        std::vector<int> extra((size_t)128 * D, 0);  // (bank, half) x step: edges beyond one
        for (size_t q = 0; q < ed.size(); ++q) {
            if (col[q] >= 0) continue;
            int k = -1;
            for (int x = 0; x < D; ++x)
                if (at[(size_t)ed[q].u * D + x] < 0 &&
                    (k < 0 || extra[(size_t)ed[q].v * D + x] < extra[(size_t)ed[q].v * D + k]))
                    k = x;
            col[q] = k;
            at[(size_t)ed[q].u * D + k] = (int)q;
            ++extra[(size_t)ed[q].v * D + k];
        }
        for (size_t q = 0; q < ed.size(); ++q) {
            const int64_t e = ed[q].e;
            epos[(size_t)e] = col[q];
            col16[(size_t)(64 * w + ed[q].u) * s.DCMAX + col[q]] = (uint16_t)(4u * (uint32_t)slot_of[c->colidx[e]]);
        }
    }
}

// Host tables of the block kernel for one shape (no device work).
struct BlockTables {
    std::vector<LaneSeg> lanes;
    std::vector<int32_t> wdeg, wbase;
    BlockLayout lay{};
    std::vector<int32_t> chk_row, chk_split, slot_col;
    std::vector<uint16_t> col16, mu16;     // per thread: Lambda byte address per step; message words
    std::vector<uint32_t> col_pk, mu_pk;  // the same, packed as the kernel reads them
};

BlockTables block_tables(const rb_ctx *c, const rb::BlockShape &s) {
    BlockTables T;
    std::vector<LaneSeg> &lanes = T.lanes;
    std::vector<int32_t> &wdeg = T.wdeg, &wbase = T.wbase;
    int64_t words = 0;
    block_order(c, s, lanes, wdeg, wbase, words);
    spread_check_lanes(c, s, lanes);
    T.lay = block_layout(s, words);
    const BlockLayout &lay = T.lay;
    // chk_row: the check whose syndrome bit thread t adds (first segment only);
    // chk_split: thread t shares its check with thread t ^ 1
    std::vector<int32_t> &chk_row = T.chk_row, &chk_split = T.chk_split;
    chk_row.assign((size_t)s.TPB, -1);
    chk_split.assign((size_t)s.TPB, 0);
    std::vector<int32_t> lane_of_edge((size_t)c->E, -1);
    for (int32_t t = 0; t < s.TPB; ++t) {
        const LaneSeg &g = lanes[(size_t)t];
        if (g.row < 0) continue;
        if (g.first) chk_row[t] = g.row;
        chk_split[t] = g.split ? 1 : 0;
        for (int32_t q = g.b; q < g.e; ++q) lane_of_edge[(size_t)(c->rowptr[g.row] + q)] = t;
    }
    T.slot_col = place_faults(c, s, lane_of_edge, wdeg, lay);
    const std::vector<int32_t> &slot_col = T.slot_col;
    std::vector<int32_t> slot_of((size_t)c->N, -1);
    for (size_t q = 0; q < slot_col.size(); ++q)
        if (slot_col[q] >= 0) slot_of[(size_t)slot_col[q]] = (int32_t)q;
    const int nmu = rb::prof_pre(s.prof, s.VPT);
    const int ncp = s.DCMAX / 2, nmp = (nmu + 1) / 2;
    std::vector<uint16_t> &col16 = T.col16, &mu16 = T.mu16;
    col16.assign((size_t)s.TPB * s.DCMAX, (uint16_t)lay.lampad_off);
    mu16.assign((size_t)s.TPB * nmp * 2, (uint16_t)(lay.mupad_off / 4u));
    std::vector<int32_t> epos((size_t)c->E, 0);  // CSR edge -> message row k
    order_rows(c, s, lanes, wdeg, slot_of, epos, col16);
    for (int32_t t = 0; t < s.TPB; ++t)
        for (int v = 0; v < s.VPT; ++v) {
            const int32_t j = slot_col[(size_t)t + (size_t)s.TPB * v];
            if (j < 0) continue;
            for (int64_t k = 0; k < c->colptr[j + 1] - c->colptr[j]; ++k) {
                const int32_t i = c->rowidx[c->colptr[j] + k];
                const size_t e = (size_t)(c->rowptr[i] + c->cpos[c->colptr[j] + k]);
                const int32_t ti = lane_of_edge[e];
                const int64_t word = (int64_t)(lay.mu0_off / 4u) + wbase[ti / 64] + (int64_t)epos[e] * 64 + (ti % 64);
                mu16[(size_t)t * nmp * 2 + rb::prof_pre(s.prof, v) + k] = (uint16_t)word;
            }
        }
    // check table as [chunk][thread][4 words] (one 16-byte load per thread and
    // chunk of 8 edges, coalesced over a wave); fault table as [pair][thread]
    std::vector<uint32_t> &col_pk = T.col_pk, &mu_pk = T.mu_pk;
    col_pk.assign((size_t)(ncp + 4) * s.TPB, (uint32_t)lay.lampad_off * 0x10001u);  // + one padding chunk
    mu_pk.assign((size_t)nmp * s.TPB, 0u);
    for (int32_t t = 0; t < s.TPB; ++t) {
        for (int e = 0; e < ncp; ++e) {
            const int ch = e / 4, d = e % 4;
            col_pk[((size_t)ch * s.TPB + t) * 4 + d] =
                (uint32_t)col16[(size_t)t * s.DCMAX + 2 * e] |
                ((uint32_t)col16[(size_t)t * s.DCMAX + 2 * e + 1] << 16);
        }
        for (int e = 0; e < nmp; ++e)
            mu_pk[(size_t)e * s.TPB + t] = (uint32_t)mu16[(size_t)t * nmp * 2 + 2 * e] |
                                          ((uint32_t)mu16[(size_t)t * nmp * 2 + 2 * e + 1] << 16);
    }
    return T;
}

// ---- independent reading of the gather tables (rb_plan_check) ----
//
// The tables are decoded exactly as the kernels read them and compared with
// the graph itself, not with the planner's intermediate maps.  LDS cost model
// (measured on gfx950): 32 banks of 4-byte words (bank = word address mod 32);
// a wave-wide read is served in two halves (lanes 0-31, then 32-63), each
// costing the largest number of distinct words on one bank (a word read by
// several lanes counts once), so a gather costs at least 2 cycles.

int half_cost(std::vector<uint32_t> &words) {
    std::sort(words.begin(), words.end());
    words.erase(std::unique(words.begin(), words.end()), words.end());
    int per_bank[32] = {0}, m = 0;
    for (uint32_t w : words) m = std::max(m, ++per_bank[w % 32u]);
    return m;
}

// cost of one wave-wide gather: words[l] is lane l's word address
int gather_cost(const std::vector<uint32_t> &words) {
    std::vector<uint32_t> lo(words.begin(), words.begin() + 32), hi(words.begin() + 32, words.end());
    return half_cost(lo) + half_cost(hi);
}

// CSR edge of (i, j), or -1
int64_t find_edge(const rb_ctx *c, int32_t i, int32_t j) {
    const auto b = c->colidx.begin() + c->rowptr[i], e = c->colidx.begin() + c->rowptr[i + 1];
    const auto it = std::lower_bound(b, e, j);
    return (it != e && *it == j) ? (int64_t)(it - c->colidx.begin()) : -1;
}

std::string check_group_tables(const rb_ctx *c, const rb::TileShape &s, const GroupTables &T, rb_plan_report *r) {
    const Layout &lay = T.lay;
    const int NS = 64 / s.G, nl = s.CPT * s.DC, nm = s.VPT * s.DV;
    if (lay.sph * s.G != 32 && !(s.G >= 32 && lay.sph == 1)) return "slots per half-wave";
    const int nlp = (nl + 1) / 2, nmp = (nm + 1) / 2;
    if (T.lam.size() != (size_t)s.G * nlp || T.mu.size() != (size_t)s.G * nmp) return "table sizes";
    if (lay.half_off > 65536 || lay.lds_bytes > 65536) return "LDS image exceeds the 16-bit offsets";
    auto entry = [](const std::vector<uint32_t> &t, size_t row, int idx) {
        const uint32_t w = t[row + (size_t)(idx / 2)];
        return (idx & 1) ? (w >> 16) : (w & 0xffffu);
    };
    // offsets address words of slot 0 of a region: multiples of word
    for (uint32_t w : T.lam)
        if ((w & 0xffffu) % lay.word || (w >> 16) % lay.word) return "Lambda offset not slot-aligned";
    for (uint32_t w : T.mu)
        if ((w & 0xffffu) % lay.word || (w >> 16) % lay.word) return "message offset not slot-aligned";
    std::vector<int32_t> step((size_t)c->E, -1);
    for (int g = 0; g < s.G; ++g)
        for (int cc = 0; cc < s.CPT; ++cc) {
            const int i = g + s.G * cc;
            for (int k = 0; k < s.DC; ++k) {
                const uint32_t a = entry(T.lam, (size_t)g * nlp, cc * s.DC + k);
                if (a == lay.lampad_off) continue;
                const std::string at = "check " + std::to_string(i) + " step " + std::to_string(k);
                if (i >= c->M) return at + ": gather on a spare check row";
                const uint32_t j = a / lay.word;
                if (j >= (uint32_t)c->N) return at + ": Lambda offset outside the marginals";
                const int64_t e = find_edge(c, i, (int32_t)j);
                if (e < 0) return at + ": fault " + std::to_string(j) + " is not in the check";
                if (step[(size_t)e] >= 0) return at + ": edge gathered twice";
                step[(size_t)e] = k;
            }
        }
    for (int64_t e = 0; e < c->E; ++e)
        if (step[(size_t)e] < 0) return "CSR edge " + std::to_string(e) + " never gathered by its check";
    for (int g = 0; g < s.G; ++g)
        for (int vv = 0; vv < s.VPT; ++vv) {
            const int j = g + s.G * vv;
            const int64_t d = j < c->N ? c->colptr[j + 1] - c->colptr[j] : 0;
            for (int k = 0; k < s.DV; ++k) {
                const uint32_t a = entry(T.mu, (size_t)g * nmp, vv * s.DV + k);
                uint32_t want = lay.mupad_off;
                if (k < d) {  // k-th check of the fault in ascending order
                    const int32_t i = c->rowidx[(size_t)(c->colptr[j] + k)];
                    const int64_t e = find_edge(c, i, j);
                    want = lay.mu0_off + lay.word * ((uint32_t)step[(size_t)e] * (uint32_t)lay.ks + (uint32_t)i);
                }
                if (a != want)
                    return "fault " + std::to_string(j) + " gather " + std::to_string(k) + ": offset " +
                           std::to_string(a) + ", the message word is " + std::to_string(want);
            }
        }
    // bank model over the wave's 64 lanes (slot-major: lane = slot * G + g),
    // each half of 32 lanes costed on its own
    std::vector<uint32_t> words;
    auto wave = [&](const std::vector<uint32_t> &t, int nrow, int idx) {
        words.clear();
        for (int sl = 0; sl < NS; ++sl) {  // lane = slot * G + g
            const uint32_t base = 4u * (uint32_t)(sl % lay.sph) + lay.half_off * (uint32_t)(sl / lay.sph);
            for (int g = 0; g < s.G; ++g) words.push_back((entry(t, (size_t)g * nrow, idx) + base) / 4u);
        }
        return gather_cost(words);
    };
    for (int q = 0; q < nl; ++q) {
        r->check_gathers += 1;
        r->check_bank_cycles += wave(T.lam, nlp, q);
    }
    for (int q = 0; q < nm; ++q) {
        r->fault_gathers += 1;
        r->fault_bank_cycles += wave(T.mu, nmp, q);
    }
    r->lds_bytes = lay.lds_bytes;
    return "";
}

std::string check_block_tables(const rb_ctx *c, const rb::BlockShape &s, const BlockTables &T, rb_plan_report *r) {
    const BlockLayout &lay = T.lay;
    const int TPB = s.TPB, nw = TPB / 64;
    const int nmu = rb::prof_pre(s.prof, s.VPT), nmp = (nmu + 1) / 2, ncp = s.DCMAX / 2;
    if (T.col_pk.size() != (size_t)(ncp + 4) * TPB || T.mu_pk.size() != (size_t)nmp * TPB) return "table sizes";
    if (T.chk_row.size() != (size_t)TPB || T.chk_split.size() != (size_t)TPB ||
        T.slot_col.size() != (size_t)TPB * s.VPT || T.wdeg.size() != (size_t)nw || T.wbase.size() != (size_t)nw)
        return "map sizes";
    if (lay.lds_bytes > 160 * 1024) return "LDS image exceeds a CU";
    // slots: a permutation of the faults on slots 0..N-1, band caps respected
    std::vector<int32_t> slot_of((size_t)c->N, -1);
    for (int64_t q = 0; q < (int64_t)TPB * s.VPT; ++q) {
        const int32_t j = T.slot_col[(size_t)q];
        if ((q < c->N) != (j >= 0)) return "slot " + std::to_string(q) + ": real slots must be exactly 0..N-1";
        if (j < 0) continue;
        if (j >= c->N || slot_of[(size_t)j] >= 0) return "slot " + std::to_string(q) + ": fault repeated or out of range";
        slot_of[(size_t)j] = (int32_t)q;
        if (c->colptr[j + 1] - c->colptr[j] > rb::prof_dv(s.prof, (int)(q / TPB)))
            return "fault " + std::to_string(j) + " exceeds its band's gather count";
    }
    if (lay.lampad_off < 4u * (uint32_t)c->N || lay.lampad_off + 4u > 65536u) return "Lambda pad cell";
    // message rows: wave w owns words [wbase[w], wbase[w] + 64 wdeg[w]) after mu0
    int64_t words_end = 0;
    for (int w = 0; w < nw; ++w) {
        if (T.wdeg[w] < 0 || T.wdeg[w] > s.DCMAX) return "wave " + std::to_string(w) + ": row count";
        if (T.wbase[w] != words_end) return "wave " + std::to_string(w) + ": message rows not contiguous";
        words_end += 64ll * T.wdeg[w];
    }
    const int64_t mu0w = lay.mu0_off / 4u;
    if (mu0w + words_end > 65535) return "message words exceed the 16-bit indices";
    if (4 * (mu0w + words_end + (rb::kBlockChunk - 1) * 64) > (int64_t)lay.lds_bytes)
        return "message rows and slack exceed the LDS image";
    // checks: chk_row names each check once; a split check sits on lanes 2p, 2p+1
    std::vector<int32_t> row_of((size_t)TPB, -1), seen((size_t)c->M, 0);
    for (int t = 0; t < TPB; ++t) {
        const int32_t i = T.chk_row[t];
        if (i < -1 || i >= c->M) return "thread " + std::to_string(t) + ": check index";
        if (i >= 0 && seen[(size_t)i]++) return "check " + std::to_string(i) + " on two threads";
    }
    for (int32_t i = 0; i < c->M; ++i)
        if (!seen[(size_t)i]) return "check " + std::to_string(i) + " has no thread";
    for (int t = 0; t < TPB; ++t) {
        if (T.chk_split[t]) {
            if (!T.chk_split[t ^ 1]) return "thread " + std::to_string(t) + ": split partner";
            if ((T.chk_row[t] >= 0) == (T.chk_row[t ^ 1] >= 0)) return "thread " + std::to_string(t) + ": split owner";
            row_of[t] = T.chk_row[t] >= 0 ? T.chk_row[t] : T.chk_row[t ^ 1];
        } else {
            row_of[t] = T.chk_row[t];
        }
    }
    auto col_entry = [&](int t, int k) {  // [chunk of 8][thread][4 words of two halves]
        const uint32_t w = T.col_pk[((size_t)(k / 8) * TPB + t) * 4 + (size_t)((k / 2) % 4)];
        return (k & 1) ? (w >> 16) : (w & 0xffffu);
    };
    for (int k = 0; k < (ncp + 4) * 2; ++k)  // the padding chunk included
        for (int t = 0; t < TPB; ++t)
            if (k >= T.wdeg[t / 64] && col_entry(t, k) != lay.lampad_off)
                return "thread " + std::to_string(t) + " step " + std::to_string(k) + ": gather past the wave's rows";
    std::vector<int64_t> word_of((size_t)c->E, -1);  // message word each edge's check writes
    for (int t = 0; t < TPB; ++t)
        for (int k = 0; k < T.wdeg[t / 64]; ++k) {
            const uint32_t a = col_entry(t, k);
            if (a == lay.lampad_off) continue;
            const std::string at = "thread " + std::to_string(t) + " step " + std::to_string(k);
            if (row_of[t] < 0) return at + ": gather on an idle thread";
            if (a % 4u || a / 4u >= (uint32_t)c->N) return at + ": Lambda address outside the marginals";
            const int32_t j = T.slot_col[a / 4u];
            const int64_t e = find_edge(c, row_of[t], j);
            if (e < 0) return at + ": fault " + std::to_string(j) + " is not in check " + std::to_string(row_of[t]);
            if (word_of[(size_t)e] >= 0) return at + ": edge gathered twice";
            word_of[(size_t)e] = mu0w + T.wbase[t / 64] + 64ll * k + (t % 64);
        }
    for (int64_t e = 0; e < c->E; ++e)
        if (word_of[(size_t)e] < 0) return "CSR edge " + std::to_string(e) + " never gathered by its check";
    auto mu_entry = [&](int t, int idx) {
        const uint32_t w = T.mu_pk[(size_t)(idx / 2) * TPB + t];
        return (idx & 1) ? (w >> 16) : (w & 0xffffu);
    };
    for (int t = 0; t < TPB; ++t)
        for (int v = 0; v < s.VPT; ++v) {
            const int32_t j = T.slot_col[(size_t)t + (size_t)TPB * v];
            const int64_t d = j >= 0 ? c->colptr[j + 1] - c->colptr[j] : 0;
            for (int k = 0; k < rb::prof_dv(s.prof, v); ++k) {
                const uint32_t a = mu_entry(t, rb::prof_pre(s.prof, v) + k);
                int64_t want = lay.mupad_off / 4u;
                if (k < d) {  // k-th check of the fault in ascending order
                    const int32_t i = c->rowidx[(size_t)(c->colptr[j] + k)];
                    want = word_of[(size_t)find_edge(c, i, j)];
                }
                if ((int64_t)a != want)
                    return "fault " + std::to_string(j) + " gather " + std::to_string(k) + ": word " + std::to_string(a) +
                           ", the message word is " + std::to_string(want);
            }
        }
    std::vector<uint32_t> words;
    for (int w = 0; w < nw; ++w)
        for (int k = 0; k < T.wdeg[w]; ++k) {
            words.clear();
            for (int l = 0; l < 64; ++l) words.push_back(col_entry(64 * w + l, k) / 4u);
            r->check_gathers += 1;
            r->check_bank_cycles += gather_cost(words);
        }
    for (int w = 0; w < nw; ++w)
        for (int v = 0; v < s.VPT; ++v)
            for (int k = 0; k < rb::prof_dv(s.prof, v); ++k) {
                words.clear();
                for (int l = 0; l < 64; ++l) words.push_back(mu_entry(64 * w + l, rb::prof_pre(s.prof, v) + k));
                r->fault_gathers += 1;
                r->fault_bank_cycles += gather_cost(words);
            }
    r->lds_bytes = lay.lds_bytes;
    return "";
}

rb_status build_block_plan(rb_ctx *c, int bv) {
    const rb::BlockShape s = rb::block_variant_shape(bv);
    const BlockTables T = block_tables(c, s);
    const BlockLayout &lay = T.lay;
    const std::vector<int32_t> &slot_col = T.slot_col;
    rb_status st;
    if ((st = upload(&c->d_lam_off, T.col_pk, "upload check table")) != RB_OK) return st;
    if ((st = upload(&c->d_mu_off, T.mu_pk, "upload fault table")) != RB_OK) return st;
    if ((st = upload(&c->d_chk_row, T.chk_row, "upload row map")) != RB_OK) return st;
    if ((st = upload(&c->d_chk_split, T.chk_split, "upload split map")) != RB_OK) return st;
    if ((st = upload(&c->d_slot_col, slot_col, "upload slot map")) != RB_OK) return st;
    {
        const int npad = s.TPB * s.VPT, R = c->params.num_legs;
        std::vector<float> w_slot((size_t)npad, 0.0f);
        for (int32_t q = 0; q < c->N; ++q) w_slot[q] = c->w[(size_t)slot_col[q]];
        if ((st = upload(&c->d_w_slot, w_slot, "upload w by slot")) != RB_OK) return st;
        (void)hipFree(c->d_gamma_slot);
        c->d_gamma_slot = nullptr;
        RB_HIP(hipMalloc(&c->d_gamma_slot, sizeof(float) * (size_t)npad * (size_t)R), "hipMalloc(gamma by slot)");
        RB_HIP(rb::launch_gather_slots(c->d_gamma, c->N, c->d_slot_col, npad, R, c->d_gamma_slot, nullptr),
               "gamma by slot");
        RB_HIP(hipDeviceSynchronize(), "gamma by slot");
    }
    if ((st = upload(&c->d_wave_deg, T.wdeg, "upload wave degrees")) != RB_OK) return st;
    if ((st = upload(&c->d_wave_base, T.wbase, "upload wave bases")) != RB_OK) return st;
    {
        size_t st_lds = 0;
        RB_HIP(rb::block_static_lds(bv, &st_lds), "kernel attributes");
        if (st_lds != 0) return fail(RB_E_DEVICE, "internal: block kernel uses static LDS");
    }
    RB_HIP(rb::block_prepare(bv, (size_t)lay.lds_bytes), "allow dynamic LDS");
    c->variant = rb::num_variants() + bv;
    c->block = true;
    c->bshape = s;
    c->lampad_off = lay.lampad_off;
    c->mupad_off = lay.mupad_off;
    c->red_off = lay.red_off;
    c->slack_off = lay.slack_off;
    c->mu0_off = lay.mu0_off;
    c->lds_bytes = lay.lds_bytes;
    const bool prior = c->params.anchor == RB_ANCHOR_PRIOR;
    for (int tr = 0; tr < 2; ++tr) {
        int blocks = 0;
        RB_HIP(rb::block_variant_occupancy(bv, prior, tr != 0, (size_t)lay.lds_bytes, &blocks),
               "occupancy query");
        if (blocks < 1) return fail(RB_E_UNSUPPORTED, "block configuration does not fit on a CU");
        c->blocks_per_cu[tr] = blocks;
    }
    return RB_OK;
}

// Host tables of the large-graph kernel (no device work).  Checks sorted by
// decreasing degree form groups of 64 of nearly the same length, dealt to the
// waves' rounds so the waves' row work is balanced (below).  Faults are renumbered into slots by decreasing
// column degree (ties by index), so the 64 slots of a wave in one round
// nearly always share a degree (the dealing of degree groups to rounds is
// below).  Row chunks (8 entries, rows padded with N)
// hold fault slots.  Row i owns records rrec[i] .. rrec[i] + ceil(deg/32) - 1;
// position k of the row is bit (k & 31) ^ 7 of word 3 of record
// rrec[i] + k / 32 (a chunk of 8 positions is one byte, entry q in bit
// 7 - q).  Each fault-side entry is the code of its edge: record << 20 |
// ((k & 31) ^ 24), the low five bits being the left shift that moves the
// edge's sign bit to bit 31.
struct LargeTables {
    LargeLayout lay{};
    int32_t rounds = 0;
    std::vector<int32_t> chk_of, rowptr, rbase, rrec, slot_col;
    std::vector<int2> fcol;      // per slot: first entry in fedge, column degree
    std::vector<uint16_t> ctab;  // rows padded to multiples of kLargeGather entries, + one zero chunk
    std::vector<uint32_t> frec, fedge;
};

uint32_t large_code(int32_t rec0, int64_t k) {
    return ((uint32_t)(rec0 + k / 32) << rb::kLargeEdgeBits) | ((uint32_t)(k & 31) ^ 24u);
}

LargeTables large_tables(const rb_ctx *c, const rb::LargeShape &s) {
    constexpr int G = rb::kLargeGather;
    const int npad = s.TPB * s.VR;
    LargeTables T;
    T.lay = large_layout(c, s);
    std::vector<int32_t> order((size_t)c->M);
    for (int32_t i = 0; i < c->M; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return c->rowptr[x + 1] - c->rowptr[x] > c->rowptr[y + 1] - c->rowptr[y];
    });
    // groups of 64 checks in that order, largest cost first, each to the wave
    // with the least cost so far that has a round left (cost: three per
    // chunk of the group's longest row, one per row for its state); a
    // wave's groups take its rounds 0, 1, ...
    const int nwv = s.TPB / 64;
    const int ngr = (c->M + 63) / 64;
    std::vector<std::pair<int64_t, int>> gcost((size_t)ngr);
    for (int g = 0; g < ngr; ++g) {
        const int32_t i0 = order[(size_t)64 * g];  // the group's longest row
        gcost[(size_t)g] = {-(3 * ((c->rowptr[i0 + 1] - c->rowptr[i0] + rb::kLargeGather - 1) / rb::kLargeGather) + 1), g};
    }
    std::sort(gcost.begin(), gcost.end());
    std::vector<int64_t> wload((size_t)nwv, 0);
    std::vector<int> wrounds((size_t)nwv, 0);
    T.chk_of.assign((size_t)rb::kLargeRounds * s.TPB, -1);
    T.rounds = 0;
    for (const auto &gc : gcost) {
        int best = -1;
        for (int w = 0; w < nwv; ++w)
            if (wrounds[(size_t)w] < rb::kLargeRounds && (best < 0 || wload[(size_t)w] < wload[(size_t)best])) best = w;
        if (best < 0) break;  // more groups than rounds (the planner rejects such graphs first)
        const int rnd = wrounds[(size_t)best]++;
        wload[(size_t)best] += -gc.first;
        T.rounds = std::max(T.rounds, rnd + 1);
        for (int lane = 0; lane < 64 && 64 * gc.second + lane < c->M; ++lane)
            T.chk_of[(size_t)rnd * s.TPB + 64 * best + lane] = order[(size_t)(64 * gc.second + lane)];
    }
    std::vector<int32_t> fo((size_t)c->N);
    for (int32_t j = 0; j < c->N; ++j) fo[(size_t)j] = j;
    std::stable_sort(fo.begin(), fo.end(), [&](int32_t x, int32_t y) {
        return c->colptr[x + 1] - c->colptr[x] > c->colptr[y + 1] - c->colptr[y];
    });
    // groups of 64 faults in that order are dealt to (round v, wave w) slot
    // groups, each wave's rounds taken from a different starting round, so
    // the waves reach the highest degrees (the entries read one by one) at
    // different times
    const int nw = s.TPB / 64, nv = (c->N + s.TPB - 1) / s.TPB;
    std::vector<std::array<int, 3>> groups;  // (rotated round, wave, round)
    for (int v = 0; v < nv; ++v)
        for (int w = 0; w < nw; ++w)
            if ((int64_t)s.TPB * v + 64 * w < c->N) groups.push_back({(v - w * nv / nw + nv) % nv, w, v});
    std::sort(groups.begin(), groups.end());
    T.slot_col.assign((size_t)npad, -1);
    std::vector<int32_t> slot_of((size_t)c->N);
    int32_t next = 0;
    for (const auto &g : groups)
        for (int lane = 0; lane < 64; ++lane) {
            const int64_t p = (int64_t)s.TPB * g[2] + 64 * g[1] + lane;
            if (p >= c->N) break;
            T.slot_col[(size_t)p] = fo[(size_t)next];
            slot_of[(size_t)fo[(size_t)next++]] = (int32_t)p;
        }
    T.rowptr.assign(c->rowptr.begin(), c->rowptr.end());
    T.rbase.resize((size_t)c->M);
    T.rrec.resize((size_t)c->M);
    int64_t chunks = 0, recs = 0;
    for (int32_t i = 0; i < c->M; ++i) {
        const int64_t d = c->rowptr[i + 1] - c->rowptr[i];
        T.rbase[(size_t)i] = (int32_t)chunks;
        T.rrec[(size_t)i] = (int32_t)recs;
        chunks += (d + G - 1) / G;
        recs += std::max<int64_t>(1, (d + 31) / 32);
    }
    // padding entries of a row's last chunk hold N (the +inf entry of Lambda);
    // the closing chunk, only ever prefetched, holds zeros
    T.ctab.assign((size_t)(chunks + 1) * G, 0);
    for (int32_t i = 0; i < c->M; ++i) {
        const int64_t d = c->rowptr[i + 1] - c->rowptr[i];
        for (int64_t k = d; k < (d + G - 1) / G * G; ++k) T.ctab[(size_t)T.rbase[(size_t)i] * G + (size_t)k] = (uint16_t)c->N;
        for (int64_t e = c->rowptr[i]; e < c->rowptr[i + 1]; ++e)
            T.ctab[(size_t)T.rbase[(size_t)i] * G + (size_t)(e - c->rowptr[i])] =
                (uint16_t)slot_of[(size_t)c->colidx[(size_t)e]];
    }
    T.fedge.assign((size_t)std::max<int64_t>(1, c->E), 0u);
    T.fcol.assign((size_t)npad, int2{0, 0});
    constexpr int RC = rb::kLargeRec;
    T.frec.assign((size_t)npad * RC, 0u);
    int64_t q = 0;
    for (int32_t p = 0; p < c->N; ++p) {
        const int32_t j = T.slot_col[(size_t)p];
        T.fcol[(size_t)p] = int2{(int)q, (int)(c->colptr[j + 1] - c->colptr[j])};
        for (int64_t e = c->colptr[j]; e < c->colptr[j + 1]; ++e, ++q) {
            const int32_t i = c->rowidx[(size_t)e];
            const uint32_t code = large_code(T.rrec[(size_t)i], c->cpos[(size_t)e]);
            T.fedge[(size_t)q] = code;
            if (e - c->colptr[j] < RC) T.frec[(size_t)p * RC + (size_t)(e - c->colptr[j])] = code;
        }
    }
    return T;
}

// Independent reading of the large-graph tables: every check on exactly one
// (round, thread); rounds in use hold the checks (kernel reads rounds <
// ceil(M/TPB)); the slots a permutation of the faults; each CSR edge's row
// entry the slot of its fault; rows' records disjoint and inside the LDS
// record region; each slot's entries, decoded (record -> its row, position
// from the record and the bit), exactly its column's edges in ascending
// check order, so every message is rebuilt from its own check's state and
// sign bit; the LDS image fits.
std::string check_large_tables(const rb_ctx *c, const rb::LargeShape &s, const LargeTables &T, rb_plan_report *r) {
    if (T.lay.lds_bytes > 160 * 1024) return "LDS image exceeds a CU";
    if (T.rounds < 1 || T.rounds > rb::kLargeRounds || (int64_t)T.rounds * s.TPB < c->M) return "check rounds";
    // the kernel loads whole chunks of kLargeGather entries: a row's chunk
    // past its last edge holds N (the +inf entry of Lambda, which must not
    // overlap the check records), a record past a slot's last entry holds
    // zeros (valid addresses), and every chunk lies inside the table
    if (T.lay.chk_off < 4u * (uint32_t)c->N + 4u) return "Lambda[N] overlaps the check records";
    if (T.lay.nrec > rb::kLargeMaxRecords || T.lay.red_off < T.lay.chk_off + 16u * (uint32_t)T.lay.nrec)
        return "check records past their region";
    constexpr int G = rb::kLargeGather;
    const int npad = s.TPB * s.VR;
    constexpr int RC = rb::kLargeRec;
    if (T.frec.size() != (size_t)npad * RC || T.fcol.size() != (size_t)npad || T.slot_col.size() != (size_t)npad)
        return "slot tables";
    std::vector<int32_t> slot_of((size_t)c->N, -1);
    for (int p = 0; p < npad; ++p) {
        const int32_t j = T.slot_col[(size_t)p];
        if (p >= c->N) {
            if (j != -1) return "spare slot " + std::to_string(p) + " holds a fault";
            continue;
        }
        if (j < 0 || j >= c->N || slot_of[(size_t)j] >= 0) return "slot " + std::to_string(p) + ": not a permutation";
        slot_of[(size_t)j] = p;
    }
    std::vector<int32_t> row_of_rec((size_t)T.lay.nrec, -1);
    for (int32_t i = 0; i < c->M; ++i) {
        const int64_t d = T.rowptr[(size_t)i + 1] - T.rowptr[(size_t)i];
        const int64_t nr = std::max<int64_t>(1, (d + 31) / 32);
        for (int64_t k = 0; k < nr; ++k) {
            const int64_t rec = (int64_t)T.rrec[(size_t)i] + k;
            if (rec < 0 || rec >= T.lay.nrec || row_of_rec[(size_t)rec] >= 0) return "row " + std::to_string(i) + ": records";
            row_of_rec[(size_t)rec] = i;
        }
        if ((size_t)(T.rbase[(size_t)i] + (d + G - 1) / G) * G > T.ctab.size()) return "row chunks past the table";
        for (int64_t k = d; k < (d + G - 1) / G * G; ++k)
            if (T.ctab[(size_t)T.rbase[(size_t)i] * G + (size_t)k] != (uint32_t)c->N) return "row padding values";
        for (int64_t e = T.rowptr[(size_t)i]; e < T.rowptr[(size_t)i + 1]; ++e) {
            const uint32_t sl = T.ctab[(size_t)T.rbase[(size_t)i] * G + (size_t)(e - T.rowptr[(size_t)i])];
            if (sl >= (uint32_t)c->N || T.slot_col[sl] != c->colidx[(size_t)e])
                return "edge " + std::to_string(e) + ": wrong fault slot";
        }
    }
    for (int p = 0; p < c->N; ++p) {
        const int32_t j = T.slot_col[(size_t)p];
        const int64_t d = c->colptr[j + 1] - c->colptr[j];
        const int2 fc = T.fcol[(size_t)p];
        if (fc.y != d || fc.x < 0 || (int64_t)fc.x + d > (int64_t)T.fedge.size())
            return "slot " + std::to_string(p) + ": entry range";
        int32_t prev = -1;
        for (int64_t k = 0; k < d; ++k) {
            const uint32_t code = T.fedge[(size_t)(fc.x + k)];
            const int64_t rec = code >> rb::kLargeEdgeBits;
            if ((code & ((1u << rb::kLargeEdgeBits) - 32u)) != 0u || rec >= T.lay.nrec)
                return "slot " + std::to_string(p) + ": entry " + std::to_string(k) + " malformed";
            const int32_t i = row_of_rec[(size_t)rec];
            if (i <= prev) return "slot " + std::to_string(p) + ": checks not ascending";
            const int64_t pos = 32 * (rec - T.rrec[(size_t)i]) + (int64_t)((code & 31u) ^ 24u);  // position in the row
            const int64_t di = T.rowptr[(size_t)i + 1] - T.rowptr[(size_t)i];
            if (pos >= di || T.ctab[(size_t)T.rbase[(size_t)i] * G + (size_t)pos] != (uint32_t)p)
                return "slot " + std::to_string(p) + ": entry " + std::to_string(k) + " is not its edge";
            prev = i;
        }
        for (int k = 0; k < RC; ++k) {
            const uint32_t want = k < d ? T.fedge[(size_t)(fc.x + k)] : 0u;
            if (T.frec[(size_t)p * RC + k] != want) return "slot " + std::to_string(p) + ": record entry " + std::to_string(k);
        }
    }
    std::vector<int> seen((size_t)c->M, 0);
    for (size_t q = 0; q < T.chk_of.size(); ++q) {
        const int32_t i = T.chk_of[q];
        if (i < -1 || i >= c->M) return "placement entry " + std::to_string(q) + " out of range";
        if (i < 0) continue;
        if ((int64_t)(q / (size_t)s.TPB) >= T.rounds) return "check placed in an unused round";
        if (seen[(size_t)i]++) return "check " + std::to_string(i) + " placed twice";
    }
    for (int32_t i = 0; i < c->M; ++i)
        if (!seen[(size_t)i]) return "check " + std::to_string(i) + " not placed";
    r->lds_bytes = (int32_t)T.lay.lds_bytes;
    return "";
}

rb_status build_large_plan(rb_ctx *c, int lv) {
    const rb::LargeShape s = rb::large_variant_shape(lv);
    const LargeTables T = large_tables(c, s);
    rb_status st;
    if ((st = upload(&c->d_chk_of, T.chk_of, "upload check placement")) != RB_OK) return st;
    if ((st = upload(&c->d_lrowptr, T.rowptr, "upload rowptr")) != RB_OK) return st;
    if ((st = upload(&c->d_fcol, T.fcol, "upload slot entry ranges")) != RB_OK) return st;
    if ((st = upload(&c->d_slot_col, T.slot_col, "upload slot map")) != RB_OK) return st;
    {
        const int npad = s.TPB * s.VR, R = c->params.num_legs;
        std::vector<float> w_slot((size_t)npad, 0.0f);
        for (int32_t p = 0; p < c->N; ++p) w_slot[(size_t)p] = c->w[(size_t)T.slot_col[(size_t)p]];
        if ((st = upload(&c->d_w_slot, w_slot, "upload w by slot")) != RB_OK) return st;
        (void)hipFree(c->d_gamma_slot);
        c->d_gamma_slot = nullptr;
        RB_HIP(hipMalloc(&c->d_gamma_slot, sizeof(float) * (size_t)npad * (size_t)R), "hipMalloc(gamma by slot)");
        RB_HIP(rb::launch_gather_slots(c->d_gamma, c->N, c->d_slot_col, npad, R, c->d_gamma_slot, nullptr),
               "gamma by slot");
        RB_HIP(hipDeviceSynchronize(), "gamma by slot");
    }
    if ((st = upload(&c->d_col16, T.ctab, "upload row chunks")) != RB_OK) return st;
    if ((st = upload(&c->d_rbase, T.rbase, "upload row bases")) != RB_OK) return st;
    if ((st = upload(&c->d_rrec, T.rrec, "upload row records")) != RB_OK) return st;
    if ((st = upload(&c->d_frec, T.frec, "upload fault records")) != RB_OK) return st;
    if ((st = upload(&c->d_fedge, T.fedge, "upload fault entries")) != RB_OK) return st;
    {
        size_t st_lds = 0;
        RB_HIP(rb::large_static_lds(lv, &st_lds), "kernel attributes");
        if (st_lds != 0) return fail(RB_E_DEVICE, "internal: large-graph kernel uses static LDS");
    }
    RB_HIP(rb::large_prepare(lv, (size_t)T.lay.lds_bytes), "allow dynamic LDS");
    c->variant = rb::num_variants() + rb::num_block_variants() + lv;
    c->block = false;
    c->large = true;
    c->lshape = s;
    c->lrounds = T.rounds;
    c->nrec = T.lay.nrec;
    c->chk_off = T.lay.chk_off;
    c->red_off = T.lay.red_off;
    c->lds_bytes = (int)T.lay.lds_bytes;
    const bool prior = c->params.anchor == RB_ANCHOR_PRIOR;
    for (int tr = 0; tr < 2; ++tr) {
        int blocks = 0;
        RB_HIP(rb::large_variant_occupancy(lv, prior, tr != 0, (size_t)T.lay.lds_bytes, &blocks),
               "occupancy query");
        if (blocks < 1) return fail(RB_E_UNSUPPORTED, "large-graph configuration does not fit on a CU");
        c->blocks_per_cu[tr] = blocks;
    }
    // lambda(0) slices for the largest grid a launch uses
    (void)hipFree(c->d_lambda0);
    c->d_lambda0 = nullptr;
    const size_t grid_max = (size_t)std::max(c->blocks_per_cu[0], c->blocks_per_cu[1]) * (size_t)c->num_cu;
    RB_HIP(hipMalloc(&c->d_lambda0, sizeof(float) * grid_max * (size_t)c->N), "hipMalloc(lambda0 workspace)");
    return RB_OK;
}

// The binary16 kernel on block shape bv (after build_block_plan(c, bv)):
// w and Gamma by slot as binary16 (w rounded once from FP64, Gamma from its
// FP32 value), the clip L16 = min(L, 4096), the staging words, and the
// kernel's LDS allowance and occupancy.
rb_status build_block16_extras(rb_ctx *c, int bv) {
    if (bv >= rb::num_block16_variants()) return fail(RB_E_INTERNAL, "no binary16 kernel for this block shape");
    const rb::BlockShape s = rb::block_variant_shape(bv), s16 = rb::block16_variant_shape(bv);
    if (s.TPB != s16.TPB || s.DCMAX != s16.DCMAX || s.VPT != s16.VPT || s.prof != s16.prof || s.waves != s16.waves)
        return fail(RB_E_INTERNAL, "binary16 block shape differs from the FP32 one");
    const int npad = s.TPB * s.VPT, R = c->params.num_legs;
    std::vector<int32_t> slot_col((size_t)npad);
    RB_HIP(hipMemcpy(slot_col.data(), c->d_slot_col, sizeof(int32_t) * (size_t)npad, hipMemcpyDeviceToHost),
           "read slot map");
    std::vector<uint16_t> w16((size_t)npad, 0);
    for (int q = 0; q < npad; ++q)
        if (slot_col[q] >= 0) {
            const _Float16 h = (_Float16)c->w64[(size_t)slot_col[q]];  // one rounding, nearest even
            std::memcpy(&w16[q], &h, 2);
        }
    rb_status st;
    if ((st = upload(&c->d_w16_slot, w16, "upload binary16 w by slot")) != RB_OK) return st;
    (void)hipFree(c->d_gamma16_slot);
    c->d_gamma16_slot = nullptr;
    RB_HIP(hipMalloc(&c->d_gamma16_slot, sizeof(uint16_t) * (size_t)npad * (size_t)R), "hipMalloc(binary16 gamma)");
    RB_HIP(rb::launch_to_half(c->d_gamma_slot, (int64_t)npad * R, c->d_gamma16_slot, nullptr), "binary16 gamma");
    RB_HIP(hipDeviceSynchronize(), "binary16 gamma");
    const _Float16 lh = (_Float16)std::min(c->params.llr_clip, 4096.0f);
    uint16_t lb;
    std::memcpy(&lb, &lh, 2);
    c->L16 = lb;
    c->stage_off = block16_stage_off(c->lds_bytes);
    c->lds_bytes = block16_lds_bytes(s, c->lds_bytes);
    if (c->lds_bytes > 160 * 1024) return fail(RB_E_UNSUPPORTED, "binary16 LDS image exceeds a CU");
    {
        size_t st_lds = 0;
        RB_HIP(rb::block16_static_lds(bv, &st_lds), "kernel attributes");
        if (st_lds != 0) return fail(RB_E_DEVICE, "internal: binary16 block kernel uses static LDS");
    }
    RB_HIP(rb::block16_prepare(bv, (size_t)c->lds_bytes), "allow dynamic LDS");
    const bool prior = c->params.anchor == RB_ANCHOR_PRIOR;
    for (int tr = 0; tr < 2; ++tr) {
        int blocks = 0;
        RB_HIP(rb::block16_variant_occupancy(bv, prior, tr != 0, (size_t)c->lds_bytes, &blocks), "occupancy query");
        if (blocks < 1) return fail(RB_E_UNSUPPORTED, "binary16 block configuration does not fit on a CU");
        c->blocks_per_cu[tr] = blocks;
    }
    c->h16 = true;
    return RB_OK;
}

rb_status plan(rb_ctx *c, int v) {
    c->large = false;
    if (v < rb::num_variants()) {
        c->block = false;
        return build_plan(c, v);
    }
    v -= rb::num_variants();
    if (v < rb::num_block_variants()) {
        rb_status st = build_block_plan(c, v);
        if (st == RB_OK && c->params.precision == RB_PREC_F16) st = build_block16_extras(c, v);
        return st;
    }
    return build_large_plan(c, v - rb::num_block_variants());
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
    if (p->io_layout != RB_IO_BYTES && p->io_layout != RB_IO_BITS32)
        return fail(RB_E_INVALID_ARG, "io_layout must be RB_IO_BYTES or RB_IO_BITS32");
    if (p->precision != RB_PREC_F32 && p->precision != RB_PREC_F16)
        return fail(RB_E_INVALID_ARG, "precision must be RB_PREC_F32 or RB_PREC_F16");
    return RB_OK;
}

// Validates H (COO) and the priors and builds the host part of a context: the
// CSR / CSC edge layouts, the degrees and the FP32 channel LLRs (no device
// work).  prior_p may be NULL (plan diagnostics only: w = 0).
rb_status host_graph(rb_ctx **out, int32_t M, int32_t N, int64_t nnz, const int32_t *rows, const int32_t *cols,
                     const double *prior_p) {
    *out = nullptr;
    if (M < 1 || N < 1) return fail(RB_E_SHAPE, "M and N must be >= 1");
    if (nnz < 0) return fail(RB_E_INVALID_ARG, "nnz must be >= 0");
    if (nnz > 0 && (!rows || !cols)) return fail(RB_E_INVALID_ARG, "rows/cols is NULL");
    if (nnz > (int64_t)M * (int64_t)N) return fail(RB_E_SHAPE, "nnz exceeds M*N");
    for (int64_t k = 0; k < nnz; ++k)
        if (rows[k] < 0 || rows[k] >= M || cols[k] < 0 || cols[k] >= N)
            return fail(RB_E_SHAPE, "entry " + std::to_string(k) + " out of range");
    for (int32_t j = 0; prior_p && j < N; ++j) {
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
    CtxPtr own(new (std::nothrow) rb_ctx());
    rb_ctx *c = own.get();
    if (!c) return fail(RB_E_OOM, "host allocation failed");
    c->M = M;
    c->N = N;
    c->E = nnz;
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
    c->w.assign((size_t)N, 0.0f);
    c->w64.assign((size_t)N, 0.0);
    for (int32_t j = 0; prior_p && j < N; ++j) {
        c->w64[j] = std::log((1.0 - prior_p[j]) / prior_p[j]);
        c->w[j] = (float)c->w64[j];
    }
    *out = own.release();
    return RB_OK;
}

// The cheapest built-in group-kernel tile the graph fits; for larger graphs
// the first block-kernel shape that fits; -1 if none.
int choose_variant(const rb_ctx *c) {
    if (c->params.precision == RB_PREC_F16) {
        for (int bv = 0; bv < rb::num_block_variants(); ++bv)
            if (any_fits(c, rb::num_variants() + bv)) return rb::num_variants() + bv;
        return -1;
    }
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
    for (int bv = 0; bv < rb::num_block_variants() && best < 0; ++bv)
        if (block_fits(c, rb::block_variant_shape(bv))) best = rb::num_variants() + bv;
    for (int lv = 0; lv < rb::num_large_variants() && best < 0; ++lv)
        if (large_fits(c, rb::large_variant_shape(lv))) best = rb::num_variants() + rb::num_block_variants() + lv;
    return best;
}

std::string unsupported_message(const rb_ctx *c) {
    return "graph exceeds every built-in kernel configuration (M=" + std::to_string(c->M) + ", N=" +
           std::to_string(c->N) + ", max row degree " + std::to_string(c->max_row) + ", max column degree " +
           std::to_string(c->max_col) + ")";
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
        case RB_E_INTERNAL: return "internal consistency check failed";
    }
    return "unknown status";
}

const char *rb_last_error_message(void) { return g_last_error.c_str(); }

rb_status rb_params_default(rb_params *out) try {
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
    out->io_layout = RB_IO_BYTES;
    out->precision = RB_PREC_F32;
    return RB_OK;
} catch (...) {
    return host_exception();
}

rb_status rb_create(rb_ctx **out, int32_t M, int32_t N, int64_t nnz, const int32_t *rows,
                    const int32_t *cols, const double *prior_p, const rb_params *params,
                    int32_t device) try {
    g_last_error.clear();
    if (!out) return fail(RB_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!prior_p) return fail(RB_E_INVALID_ARG, "prior_p is NULL");
    if (device < 0) return fail(RB_E_INVALID_ARG, "device must be >= 0");
    rb_status st = check_params(params);
    if (st != RB_OK) return st;
    rb_ctx *c = nullptr;
    if ((st = host_graph(&c, M, N, nnz, rows, cols, prior_p)) != RB_OK) return st;
    CtxPtr own(c);
    c->device = device;
    c->params = *params;
    const int best = choose_variant(c);
    if (best < 0) return fail(RB_E_UNSUPPORTED, unsupported_message(c));

    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    c->num_cu = prop.multiProcessorCount;
    const int R = params->num_legs;
    // (both tables end in kGroupReadPad floats of zeros: see relay_internal.h)
    if ((e = hipMalloc(&c->d_w, sizeof(float) * ((size_t)N + rb::kGroupReadPad))) != hipSuccess)
        return hip_fail(e, "hipMalloc(w)");
    if ((e = hipMalloc(&c->d_gamma, sizeof(float) * ((size_t)N * (size_t)R + rb::kGroupReadPad))) != hipSuccess)
        return hip_fail(e, "hipMalloc(gamma)");
    if ((e = hipMemset(c->d_w + N, 0, sizeof(float) * rb::kGroupReadPad)) != hipSuccess ||
        (e = hipMemset(c->d_gamma + (size_t)N * R, 0, sizeof(float) * rb::kGroupReadPad)) != hipSuccess)
        return hip_fail(e, "clear table padding");
    if ((e = hipMalloc(&c->d_queue, sizeof(unsigned long long) * rb::kQueueWords)) != hipSuccess)
        return hip_fail(e, "hipMalloc(queue)");
    if ((e = hipMemcpy(c->d_w, c->w.data(), sizeof(float) * (size_t)N, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "copy w");
    if ((e = rb::launch_gamma_table(c->d_gamma, R, N, params->seed, params->gamma_first, params->gamma_lo,
                                    params->gamma_hi, nullptr)) != hipSuccess)
        return hip_fail(e, "gamma table kernel");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "gamma table sync");
    st = plan(c, best);
    if (st != RB_OK) return st;
    {
        std::vector<int32_t> rp(c->rowptr.begin(), c->rowptr.end()), cp(c->colptr.begin(), c->colptr.end());
        std::vector<int32_t> ce((size_t)nnz);
        for (int64_t k = 0; k < nnz; ++k) ce[k] = (int32_t)(c->rowptr[c->rowidx[k]] + c->cpos[k]);
        if ((st = upload(&c->d_rowptr, rp, "upload rowptr")) != RB_OK ||
            (st = upload(&c->d_colidx, c->colidx, "upload colidx")) != RB_OK ||
            (st = upload(&c->d_colptr, cp, "upload colptr")) != RB_OK ||
            (st = upload(&c->d_cedge, ce, "upload edge map")) != RB_OK)
            return st;
    }
    *out = own.release();
    return RB_OK;
} catch (...) {
    return host_exception();
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
        (void)hipFree(c->d_chk_row);
        (void)hipFree(c->d_wave_deg);
        (void)hipFree(c->d_wave_base);
        (void)hipFree(c->d_slot_col);
        (void)hipFree(c->d_chk_split);
        (void)hipFree(c->d_w_slot);
        (void)hipFree(c->d_gamma_slot);
        (void)hipFree(c->d_w16_slot);
        (void)hipFree(c->d_gamma16_slot);
        (void)hipFree(c->d_chk_of);
        (void)hipFree(c->d_lrowptr);
        (void)hipFree(c->d_fcol);
        (void)hipFree(c->d_col16);
        (void)hipFree(c->d_rbase);
        (void)hipFree(c->d_rrec);
        (void)hipFree(c->d_fedge);
        (void)hipFree(c->d_frec);
        (void)hipFree(c->d_lambda0);
    }
    if (c->d_rowptr || c->d_colidx || c->d_colptr || c->d_cedge) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(c->d_rowptr);
        (void)hipFree(c->d_colidx);
        (void)hipFree(c->d_colptr);
        (void)hipFree(c->d_cedge);
    }
    if (c->d_ws || c->d_code_m || c->d_codes || c->d_queues || c->d_code_fam || c->d_fam_rep || c->d_fam_size) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(c->d_ws);
        (void)hipFree(c->d_code_m);
        (void)hipFree(c->d_codes);
        (void)hipFree(c->d_queues);
        (void)hipFree(c->d_code_fam);
        (void)hipFree(c->d_fam_rep);
        (void)hipFree(c->d_fam_size);
    }
    if (c->d_wcat || c->d_gcat || c->d_code_member) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(c->d_wcat);
        (void)hipFree(c->d_gcat);
        (void)hipFree(c->d_code_member);
    }
    for (rb_ctx *s : c->subs) rb_destroy(s);
    delete c;
}

// Every w_j bit-identical (uniform priors): the group kernel then takes a
// solution's weight as a count times w_0.
static bool w_is_uniform(const rb_ctx *c) {
    for (size_t j = 1; j < c->w.size(); ++j)
        if (std::memcmp(&c->w[j], &c->w[0], sizeof(float)) != 0) return false;
    return true;
}

static rb::GroupArgs base_args(const rb_ctx *c, int64_t B, const uint8_t *syn) {
    rb::GroupArgs a{};
    a.M = c->M;
    a.N = c->N;
    a.io_bits = c->params.io_layout == RB_IO_BITS32 ? 1 : 0;
    a.syn_stride = a.io_bits ? (c->M + 31) / 32 : c->M;
    a.corr_stride = a.io_bits ? (c->N + 31) / 32 : c->N;
    a.llr_stride = c->N;
    a.B = B;
    a.count = B;
    a.list = nullptr;
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
    a.lampad_off = c->lampad_off;
    a.mupad_off = c->mupad_off;
    a.mu0_off = c->mu0_off;
    a.half_off = c->half_off;
    a.scale = c->prior_scale;
    a.w_uniform = w_is_uniform(c) ? 1 : 0;
    a.w0 = c->w.empty() ? 0.0f : c->w[0];
    return a;
}

static rb::BlockArgs block_args(const rb::GroupArgs &g, const rb_ctx *c) {
    rb::BlockArgs b{};
    b.M = g.M;
    b.N = g.N;
    b.syn_stride = g.syn_stride;
    b.corr_stride = g.corr_stride;
    b.io_bits = g.io_bits;
    b.B = g.B;
    b.syn = g.syn;
    b.corr = g.corr;
    b.conv = g.conv;
    b.legs = g.legs;
    b.iters = g.iters;
    b.weight = g.weight;
    b.final_llr = g.final_llr;
    b.w = g.w;
    b.gamma = g.gamma;
    b.chk_col = c->d_lam_off;
    b.col_mu = c->d_mu_off;
    b.chk_row = c->d_chk_row;
    b.chk_split = c->d_chk_split;
    b.w_slot = c->d_w_slot;
    b.gamma_slot = c->d_gamma_slot;
    b.slot_col = c->d_slot_col;
    b.wave_deg = c->d_wave_deg;
    b.wave_base = c->d_wave_base;
    b.queue = g.queue;
    b.num_legs = g.num_legs;
    b.iters_first = g.iters_first;
    b.iters_leg = g.iters_leg;
    b.num_solutions = g.num_solutions;
    b.max_total_iters = g.max_total_iters;
    b.L = g.L;
    b.lampad_off = c->lampad_off;
    b.mupad_off = c->mupad_off;
    b.red_off = c->red_off;
    b.mu0_off = c->mu0_off;
    b.slack_off = c->slack_off;
    b.trace_gamma = g.trace_gamma;
    b.scale = g.scale;
    b.trace_T = g.trace_T;
    b.trace = g.trace;
    b.w16_slot = c->d_w16_slot;
    b.gamma16_slot = c->d_gamma16_slot;
    b.L16 = c->L16;
    b.stage_off = c->stage_off;
    return b;
}

static rb::LargeArgs large_args(const rb::GroupArgs &g, const rb_ctx *c) {
    rb::LargeArgs b{};
    b.M = g.M;
    b.N = g.N;
    b.syn_stride = g.syn_stride;
    b.corr_stride = g.corr_stride;
    b.io_bits = g.io_bits;
    b.B = g.B;
    b.syn = g.syn;
    b.corr = g.corr;
    b.conv = g.conv;
    b.legs = g.legs;
    b.iters = g.iters;
    b.weight = g.weight;
    b.final_llr = g.final_llr;
    b.slot_col = c->d_slot_col;
    b.w_slot = c->d_w_slot;
    b.gamma_slot = c->d_gamma_slot;
    b.lambda0 = c->d_lambda0;
    b.rowptr = c->d_lrowptr;
    b.ctab = c->d_col16;
    b.rbase = c->d_rbase;
    b.fcol = c->d_fcol;
    b.frec = c->d_frec;
    b.fedge = c->d_fedge;
    b.chk_of = c->d_chk_of;
    b.rounds = c->lrounds;
    b.nrec = c->nrec;
    b.rrec = c->d_rrec;
    b.queue = g.queue;
    b.num_legs = g.num_legs;
    b.iters_first = g.iters_first;
    b.iters_leg = g.iters_leg;
    b.num_solutions = g.num_solutions;
    b.max_total_iters = g.max_total_iters;
    b.L = g.L;
    b.chk_off = c->chk_off;
    b.red_off = c->red_off;
    b.trace_gamma = g.trace_gamma;
    b.scale = g.scale;
    b.trace_T = g.trace_T;
    b.trace = g.trace;
    return b;
}

static int shots_per_block(const rb_ctx *c) {
    if (c->h16) return 2;  // one syndrome in each half of the binary16 words
    return (c->block || c->large) ? 1 : 64 / c->shape.G;
}

static int grid_for(const rb_ctx *c, int64_t B, int trace) {
    const int spb = shots_per_block(c);
    const int64_t need = (B + spb - 1) / spb;
    const int64_t full = (int64_t)c->blocks_per_cu[trace] * c->num_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, full));
}

static rb_status launch(rb_ctx *c, const rb::GroupArgs &a, bool trace, hipStream_t s) {
    const bool prior = !trace && c->params.anchor == RB_ANCHOR_PRIOR;
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(rb::launch_reset_queue(c->d_queue, s), "queue reset");
    const int grid = grid_for(c, a.B, trace ? 1 : 0);
    if (c->large) {
        RB_HIP(rb::launch_large(c->variant - rb::num_variants() - rb::num_block_variants(), prior, trace,
                                large_args(a, c), grid, (size_t)c->lds_bytes, s),
               "relay large-graph kernel launch");
    } else if (c->h16) {
        RB_HIP(rb::launch_block16(c->variant - rb::num_variants(), prior, trace, block_args(a, c), grid,
                                  (size_t)c->lds_bytes, s),
               "relay binary16 block kernel launch");
    } else if (c->block) {
        RB_HIP(rb::launch_block(c->variant - rb::num_variants(), prior, trace, block_args(a, c), grid,
                                (size_t)c->lds_bytes, s),
               "relay block kernel launch");
    } else {
        RB_HIP(rb::launch_group(c->variant, prior, trace, a, grid, (size_t)c->lds_bytes, s),
               "relay kernel launch");
    }
    return RB_OK;
}

rb_status rb_decode(rb_ctx *c, int64_t B, const uint8_t *d_syn, uint8_t *d_corr, uint8_t *d_conv,
                    int32_t *d_legs, int32_t *d_iters, double *d_weight, float *d_final_llr,
                    void *stream) try {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (B < 0) return fail(RB_E_INVALID_ARG, "B must be >= 0");
    if (B == 0) return RB_OK;
    if (B > INT32_MAX) return fail(RB_E_SHAPE, "B exceeds 2^31 - 1");
    if (!d_syn || !d_corr || !d_conv || !d_legs || !d_iters)
        return fail(RB_E_INVALID_ARG, "a required device pointer is NULL");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context: use rb_decode_multi");
    rb::GroupArgs a = base_args(c, B, d_syn);
    a.corr = d_corr;
    a.conv = d_conv;
    a.legs = d_legs;
    a.iters = d_iters;
    a.weight = d_weight;
    a.final_llr = d_final_llr;
    if (!c->block && !c->large && c->d_ws && B <= c->ws_capacity) {
        // longest-first order: shot list sorted by decreasing syndrome weight
        hipStream_t s = (hipStream_t)stream;
        RB_HIP(hipSetDevice(c->device), "hipSetDevice");
        RB_HIP(rb::launch_shot_lists(B, d_syn, a.syn_stride, a.io_bits != 0, nullptr, c->d_code_m, 1, nullptr, 1,
                                     nullptr, c->d_ws, c->d_queue, s),
               "shot list kernels");
        a.list = (const int32_t *)c->d_ws + (size_t)(rb::kListHeader + B);
        RB_HIP(rb::launch_group(c->variant, c->params.anchor == RB_ANCHOR_PRIOR, false, a,
                                grid_for(c, B, 0), (size_t)c->lds_bytes, s),
               "relay kernel launch");
        return RB_OK;
    }
    return launch(c, a, false, (hipStream_t)stream);
} catch (...) {
    return host_exception();
}

rb_status rb_syndrome(const rb_ctx *c, int64_t B, const uint8_t *d_corr, const uint8_t *d_syn_in,
                      uint8_t *d_syn_out, void *stream) try {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context: use a single code's context");
    if (B < 0) return fail(RB_E_INVALID_ARG, "B must be >= 0");
    if (B == 0) return RB_OK;
    if (!d_corr || !d_syn_out) return fail(RB_E_INVALID_ARG, "a required device pointer is NULL");
    if (B > INT64_MAX / ((int64_t)c->M + 1)) return fail(RB_E_SHAPE, "B * M overflows");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(rb::launch_syndrome(B, c->M, c->N, c->d_rowptr, c->d_colidx, d_corr, d_syn_in, d_syn_out,
                               c->params.io_layout == RB_IO_BITS32, (hipStream_t)stream),
           "syndrome kernel launch");
    return RB_OK;
} catch (...) {
    return host_exception();
}

rb_status rb_trace(rb_ctx *c, int64_t B, const uint8_t *d_syn, const float *d_gamma, float scale,
                   int32_t T, float *d_trace, void *stream) try {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context: trace one code's own context");
    if (B < 0 || T < 0) return fail(RB_E_INVALID_ARG, "B and T must be >= 0");
    if (B > INT32_MAX) return fail(RB_E_SHAPE, "B exceeds 2^31 - 1");
    if (!std::isfinite(scale)) return fail(RB_E_NONFINITE, "scale must be finite");
    if (c->h16 && scale != 1.0f) return fail(RB_E_UNSUPPORTED, "the binary16 mode has no prior scale");
    if (B == 0) return RB_OK;
    if (!d_syn || !d_gamma || !d_trace) return fail(RB_E_INVALID_ARG, "a required device pointer is NULL");
    rb::GroupArgs a = base_args(c, B, d_syn);
    a.io_bits = 0;  // the trace hook takes uint8 syndromes in either layout
    a.syn_stride = c->M;
    a.corr_stride = c->N;
    a.trace_gamma = d_gamma;
    a.scale = scale;
    a.trace_T = T;
    a.trace = d_trace;
    return launch(c, a, true, (hipStream_t)stream);
} catch (...) {
    return host_exception();
}

rb_status rb_set_leg_gamma(rb_ctx *c, int32_t leg, const float *host_gamma) try {
    g_last_error.clear();
    if (!c || !host_gamma) return fail(RB_E_INVALID_ARG, "NULL argument");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context: set the gamma of a single-code context");
    if (leg < 1 || leg > c->params.num_legs) return fail(RB_E_INVALID_ARG, "leg must be in 1..R");
    for (int32_t j = 0; j < c->N; ++j)
        if (!std::isfinite(host_gamma[j])) return fail(RB_E_NONFINITE, "gamma must be finite");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipDeviceSynchronize(), "synchronise before gamma update");
    RB_HIP(hipMemcpy(c->d_gamma + (size_t)(leg - 1) * c->N, host_gamma, sizeof(float) * (size_t)c->N,
                     hipMemcpyHostToDevice),
           "copy gamma row");
    if (c->block || c->large) {
        const int npad = c->block ? c->bshape.TPB * c->bshape.VPT : c->lshape.TPB * c->lshape.VR;
        RB_HIP(rb::launch_gather_slots(c->d_gamma + (size_t)(leg - 1) * c->N, c->N, c->d_slot_col, npad, 1,
                                       c->d_gamma_slot + (size_t)(leg - 1) * npad, nullptr),
               "gamma by slot");
        if (c->h16)
            RB_HIP(rb::launch_to_half(c->d_gamma_slot + (size_t)(leg - 1) * npad, npad,
                                      c->d_gamma16_slot + (size_t)(leg - 1) * npad, nullptr),
                   "binary16 gamma");
        RB_HIP(hipDeviceSynchronize(), "gamma by slot");
    }
    return RB_OK;
} catch (...) {
    return host_exception();
}

rb_status rb_set_prior_scale(rb_ctx *c, float scale) try {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context: set the scale of a single-code context");
    if (!std::isfinite(scale)) return fail(RB_E_NONFINITE, "scale must be finite");
    if (c->h16 && scale != 1.0f) return fail(RB_E_UNSUPPORTED, "the binary16 mode has no prior scale");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipDeviceSynchronize(), "synchronise before scale update");
    c->prior_scale = scale;
    return RB_OK;
} catch (...) {
    return host_exception();
}

rb_status rb_get_llr(const rb_ctx *c, float *host_w) try {
    if (!c || !host_w) return fail(RB_E_INVALID_ARG, "NULL argument");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context");
    std::memcpy(host_w, c->w.data(), sizeof(float) * (size_t)c->N);
    return RB_OK;
} catch (...) {
    return host_exception();
}

rb_status rb_get_gamma_table(const rb_ctx *c, float *host_gamma) try {
    if (!c || !host_gamma) return fail(RB_E_INVALID_ARG, "NULL argument");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipMemcpy(host_gamma, c->d_gamma, sizeof(float) * (size_t)c->N * (size_t)c->params.num_legs,
                     hipMemcpyDeviceToHost),
           "copy gamma table");
    return RB_OK;
} catch (...) {
    return host_exception();
}

rb_status rb_get_info(const rb_ctx *c, rb_info *info) try {
    if (!c || !info) return fail(RB_E_INVALID_ARG, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->M = c->M;
    info->N = c->N;
    info->num_edges = c->E;
    info->max_row_degree = c->max_row;
    info->max_col_degree = c->max_col;
    info->variant = c->variant;
    if (c->large) {
        info->lanes_per_shot = c->lshape.TPB;
        info->checks_per_lane = c->lrounds;
        info->row_slots = c->max_row;
        info->cols_per_lane = c->lshape.VR;
        info->col_slots = c->max_col;
        info->shots_per_block = 1;
        info->threads_per_block = c->lshape.TPB;
        info->waves_per_simd_target = c->lshape.TPB / 256;
    } else if (c->block) {
        info->lanes_per_shot = c->bshape.TPB;
        info->checks_per_lane = 1;
        info->row_slots = c->bshape.DCMAX;
        info->cols_per_lane = c->bshape.VPT;
        info->col_slots = rb::prof_max(c->bshape.prof, c->bshape.VPT);
        info->shots_per_block = 1;
        info->threads_per_block = c->bshape.TPB;
        info->waves_per_simd_target = c->bshape.waves;
    } else {
        info->lanes_per_shot = c->shape.G;
        info->checks_per_lane = c->shape.CPT;
        info->row_slots = c->shape.DC;
        info->cols_per_lane = c->shape.VPT;
        info->col_slots = c->shape.DV;
        info->shots_per_block = 64 / c->shape.G;
        info->threads_per_block = 64;
        info->waves_per_simd_target = c->shape.waves;
    }
    info->lds_bytes_per_block = c->lds_bytes;
    info->blocks_per_cu = c->blocks_per_cu[0];
    info->grid_blocks = c->blocks_per_cu[0] * c->num_cu;
    info->num_variants = total_variants();
    return RB_OK;
} catch (...) {
    return host_exception();
}

rb_status rb_set_variant(rb_ctx *c, int32_t v) try {
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context: use rb_autotune_multi");
    if (v < 0 || v >= total_variants()) return fail(RB_E_INVALID_ARG, "variant out of range");
    if (!any_fits(c, v)) return fail(RB_E_UNSUPPORTED, "graph does not fit the variant");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipDeviceSynchronize(), "sync before re-plan");
    return plan(c, v);
} catch (...) {
    return host_exception();
}

rb_status rb_plan_check(int32_t M, int32_t N, int64_t nnz, const int32_t *rows, const int32_t *cols,
                        int32_t variant, rb_plan_report *out) try {
    g_last_error.clear();
    if (!out) return fail(RB_E_INVALID_ARG, "out is NULL");
    std::memset(out, 0, sizeof(*out));
    if (variant < -1 || variant >= total_variants()) return fail(RB_E_INVALID_ARG, "variant out of range");
    rb_ctx *c = nullptr;
    rb_status st = host_graph(&c, M, N, nnz, rows, cols, nullptr);
    if (st != RB_OK) return st;
    CtxPtr own(c);
    const int v = variant < 0 ? choose_variant(c) : variant;
    if (v < 0 || !any_fits(c, v))
        return fail(RB_E_UNSUPPORTED, v < 0 ? unsupported_message(c) : "graph does not fit the variant");
    out->variant = v;
    std::string err;
    if (v < rb::num_variants()) {
        const rb::TileShape s = rb::variant_shape(v);
        err = check_group_tables(c, s, group_tables(c, s), out);
    } else if (v < rb::num_variants() + rb::num_block_variants()) {
        const rb::BlockShape s = rb::block_variant_shape(v - rb::num_variants());
        out->block_kernel = 1;
        err = check_block_tables(c, s, block_tables(c, s), out);
    } else {
        const rb::LargeShape s = rb::large_variant_shape(v - rb::num_variants() - rb::num_block_variants());
        out->block_kernel = 2;
        err = check_large_tables(c, s, large_tables(c, s), out);
    }
    if (!err.empty()) return fail(RB_E_INTERNAL, "gather tables of variant " + std::to_string(v) + ": " + err);
    return RB_OK;
} catch (...) {
    return host_exception();
}

// mean time of one decode of B syndromes with the context's current plan
static rb_status time_variant(rb_ctx *c, int64_t B, const uint8_t *d_syn, int32_t reps, float *ms_out) {
    uint8_t *corr = nullptr, *conv = nullptr;
    int32_t *legs = nullptr, *iters = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(corr);
        (void)hipFree(conv);
        (void)hipFree(legs);
        (void)hipFree(iters);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e;
    const size_t corr_row = std::max<size_t>((size_t)c->N, 4 * (((size_t)c->N + 31) / 32));  // either layout
    if ((e = hipMalloc(&corr, (size_t)B * corr_row)) != hipSuccess || (e = hipMalloc(&conv, (size_t)B)) != hipSuccess ||
        (e = hipMalloc(&legs, (size_t)B * 4)) != hipSuccess || (e = hipMalloc(&iters, (size_t)B * 4)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "timing allocation");
    }
    rb_status st = rb_decode(c, B, d_syn, corr, conv, legs, iters, nullptr, nullptr, nullptr);
    if (st == RB_OK) {
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps && st == RB_OK; ++r)
            st = rb_decode(c, B, d_syn, corr, conv, legs, iters, nullptr, nullptr, nullptr);
        (void)hipEventRecord(e1, nullptr);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) {
            cleanup();
            return hip_fail(e, "timing");
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        *ms_out = ms / (float)reps;
    }
    cleanup();
    return st;
}

rb_status rb_autotune(rb_ctx *c, int64_t B, const uint8_t *d_syn, int32_t reps,
                      int32_t *chosen_variant, float *best_ms) try {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context: use rb_autotune_multi");
    if (B < 1 || !d_syn || reps < 1) return fail(RB_E_INVALID_ARG, "need B >= 1, syndromes, reps >= 1");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipDeviceSynchronize(), "sync before autotune");
    uint8_t *corr = nullptr, *conv = nullptr;
    int32_t *legs = nullptr, *iters = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(corr);
        (void)hipFree(conv);
        (void)hipFree(legs);
        (void)hipFree(iters);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e;
    const size_t corr_row = std::max<size_t>((size_t)c->N, 4 * (((size_t)c->N + 31) / 32));  // either layout
    if ((e = hipMalloc(&corr, (size_t)B * corr_row)) != hipSuccess || (e = hipMalloc(&conv, (size_t)B)) != hipSuccess ||
        (e = hipMalloc(&legs, (size_t)B * 4)) != hipSuccess || (e = hipMalloc(&iters, (size_t)B * 4)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "autotune allocation");
    }
    int best = -1;
    float best_t = 0.0f;
    for (int v = 0; v < total_variants(); ++v) {
        if (!any_fits(c, v)) continue;
        rb_status st = plan(c, v);
        if (st != RB_OK) continue;
        st = rb_decode(c, B, d_syn, corr, conv, legs, iters, nullptr, nullptr, nullptr);  // warm-up
        if (st != RB_OK) {
            cleanup();
            return st;
        }
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps; ++r) (void)rb_decode(c, B, d_syn, corr, conv, legs, iters, nullptr, nullptr, nullptr);
        (void)hipEventRecord(e1, nullptr);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) {
            cleanup();
            return hip_fail(e, "autotune timing");
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)reps;
        if (best < 0 || ms < best_t) {
            best = v;
            best_t = ms;
        }
    }
    cleanup();
    if (best < 0) return fail(RB_E_UNSUPPORTED, "no kernel configuration fits");
    rb_status st = plan(c, best);
    if (st != RB_OK) return st;
    if (chosen_variant) *chosen_variant = best;
    if (best_ms) *best_ms = best_t;
    return RB_OK;
} catch (...) {
    return host_exception();
}

static int64_t train_shot_floats(const rb_ctx *c, int32_t T, int32_t C) {
    const int64_t nck = (T + C - 1) / C;
    return (int64_t)c->N + (nck + C) * ((int64_t)c->N + c->E);
}

size_t rb_train_tape_size(const rb_ctx *c, int64_t B, int32_t T, int32_t ckpt_every) {
    if (!c || c->multi || B < 0 || T < 0 || ckpt_every < 1) return 0;
    return sizeof(float) * (size_t)B * ((size_t)train_shot_floats(c, T, ckpt_every) + (size_t)c->N + 1);
}

static rb_status train_args(const rb_ctx *c, int64_t B, const uint8_t *d_syn, const float *d_gamma,
                            const float *d_scale, int32_t T, int32_t C, void *d_tape, size_t tape_bytes,
                            rb::TrainArgs *a) {
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code context");
    if (B < 0 || T < 0 || C < 1) return fail(RB_E_INVALID_ARG, "need B >= 0, T >= 0, ckpt_every >= 1");
    if (B > INT32_MAX) return fail(RB_E_SHAPE, "B exceeds 2^31 - 1");
    if (B > 0 && (!d_syn || !d_gamma || !d_scale || !d_tape)) return fail(RB_E_INVALID_ARG, "NULL device pointer");
    if (tape_bytes < rb_train_tape_size(c, B, T, C)) return fail(RB_E_WORKSPACE, "tape too small");
    if (rb::train_lds_bytes(c->N, (int)c->E) > 64 * 1024) return fail(RB_E_UNSUPPORTED, "graph too large for training");
    rb::TrainArgs t{};
    t.M = c->M;
    t.N = c->N;
    t.E = (int32_t)c->E;
    t.B = B;
    t.syn = d_syn;
    t.w = c->d_w;
    t.gamma = d_gamma;
    t.scale = d_scale;
    t.T = T;
    t.C = C;
    t.L = c->params.llr_clip;
    t.rowptr = c->d_rowptr;
    t.colidx = c->d_colidx;
    t.colptr = c->d_colptr;
    t.cedge = c->d_cedge;
    t.tape = (float *)d_tape;
    t.shot_floats = train_shot_floats(c, T, C);
    t.gamma_part = t.tape + (size_t)B * (size_t)t.shot_floats;
    t.scale_part = t.gamma_part + (size_t)B * c->N;
    *a = t;
    return RB_OK;
}

rb_status rb_forward_train(rb_ctx *c, int64_t B, const uint8_t *d_syn, const float *d_gamma, const float *d_scale,
                           int32_t T, int32_t ckpt_every, float *d_llr_out, void *d_tape, size_t tape_bytes,
                           void *stream) try {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (c->h16) return fail(RB_E_UNSUPPORTED, "training runs in FP32: create the context with RB_PREC_F32");
    rb::TrainArgs a{};
    rb_status st = train_args(c, B, d_syn, d_gamma, d_scale, T, ckpt_every, d_tape, tape_bytes, &a);
    if (st != RB_OK) return st;
    if (B == 0) return RB_OK;
    if (!d_llr_out) return fail(RB_E_INVALID_ARG, "d_llr_out is NULL");
    a.llr_out = d_llr_out;
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(rb::launch_train_forward(a, (hipStream_t)stream), "training forward launch");
    return RB_OK;
} catch (...) {
    return host_exception();
}

rb_status rb_backward(rb_ctx *c, int64_t B, const uint8_t *d_syn, const float *d_gamma, const float *d_scale,
                      int32_t T, int32_t ckpt_every, void *d_tape, size_t tape_bytes, const float *d_dllr,
                      float *d_dgamma, float *d_dscale, void *stream) try {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (c->h16) return fail(RB_E_UNSUPPORTED, "training runs in FP32: create the context with RB_PREC_F32");
    rb::TrainArgs a{};
    rb_status st = train_args(c, B, d_syn, d_gamma, d_scale, T, ckpt_every, d_tape, tape_bytes, &a);
    if (st != RB_OK) return st;
    if (!d_dgamma || !d_dscale || (B > 0 && !d_dllr)) return fail(RB_E_INVALID_ARG, "NULL gradient pointer");
    a.dllr = d_dllr;
    a.dgamma = d_dgamma;
    a.dscale = d_dscale;
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(rb::launch_train_backward(a, (hipStream_t)stream), "training backward launch");
    return RB_OK;
} catch (...) {
    return host_exception();
}

size_t rb_workspace_size(const rb_ctx *c, int64_t B) {
    if (!c || B < 0) return 0;
    return rb::shot_list_bytes(B, c->multi ? (int)c->subs.size() : 1);
}

rb_status rb_reserve(rb_ctx *c, int64_t B) try {
    g_last_error.clear();
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (B < 0 || B > INT32_MAX) return fail(RB_E_INVALID_ARG, "B must be in [0, 2^31)");
    if (c->multi) return fail(RB_E_INVALID_ARG, "mixed-code contexts take a caller workspace");
    if (B <= c->ws_capacity) return RB_OK;
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipDeviceSynchronize(), "sync before reserve");
    (void)hipFree(c->d_ws);
    c->d_ws = nullptr;
    c->ws_capacity = 0;
    RB_HIP(hipMalloc(&c->d_ws, rb::shot_list_bytes(B, 1)), "hipMalloc(workspace)");
    if (!c->d_code_m) {
        std::vector<int32_t> m1(1, c->M);
        rb_status st = upload(&c->d_code_m, m1, "upload code rows");
        if (st != RB_OK) return st;
    }
    c->ws_capacity = B;
    return RB_OK;
} catch (...) {
    return host_exception();
}

namespace {

// per-code data the mixed kernel reads
rb_status upload_codes(rb_ctx *m) {
    const size_t nc = m->subs.size();
    std::vector<rb::CodeStatic> cs(nc);
    int lds = 0;
    for (size_t k = 0; k < nc; ++k) {
        const rb_ctx *s = m->subs[k];
        cs[k].M = s->M;
        cs[k].N = s->N;
        cs[k].tile = rb::mixed_tile_of_variant(s->variant);
        cs[k].lam_off = s->d_lam_off;
        cs[k].mu_off = s->d_mu_off;
        cs[k].lampad_off = s->lampad_off;
        cs[k].mupad_off = s->mupad_off;
        cs[k].mu0_off = s->mu0_off;
        cs[k].half_off = s->half_off;
        lds = std::max(lds, s->lds_bytes);
        if (cs[k].tile < 0) return fail(RB_E_UNSUPPORTED, "code planned outside the mixed tile set");
    }
    // families: same tile and the same graph (identical CSR), hence identical
    // gather tables and LDS layout; members differ only in w and gamma
    std::vector<int32_t> fam(nc, -1), member(nc, 0), rep, size;
    for (size_t k = 0; k < nc; ++k) {
        const rb_ctx *a = m->subs[k];
        for (size_t f = 0; f < rep.size() && fam[k] < 0; ++f) {
            const rb_ctx *b = m->subs[(size_t)rep[f]];
            if (cs[k].tile == cs[(size_t)rep[f]].tile && a->M == b->M && a->N == b->N && a->rowptr == b->rowptr &&
                a->colidx == b->colidx) {
                fam[k] = (int32_t)f;
                member[k] = size[f]++;
            }
        }
        if (fam[k] < 0) {
            fam[k] = (int32_t)rep.size();
            rep.push_back((int32_t)k);
            size.push_back(1);
        }
    }
    // w and gamma of all codes, family by family, members in order
    const int R = m->params.num_legs;
    std::vector<size_t> woff(nc), goff(nc);
    size_t wtot = 0, gtot = 0;
    for (size_t f = 0; f < rep.size(); ++f)
        for (size_t k = 0; k < nc; ++k)
            if (fam[k] == (int32_t)f) {
                woff[k] = wtot;
                goff[k] = gtot;
                wtot += (size_t)m->subs[k]->N;
                gtot += (size_t)R * m->subs[k]->N;
            }
    std::vector<float> wcat(wtot + rb::kGroupReadPad, 0.0f), gcat(gtot + rb::kGroupReadPad, 0.0f);
    for (size_t k = 0; k < nc; ++k) {
        const rb_ctx *s = m->subs[k];
        RB_HIP(hipMemcpy(wcat.data() + woff[k], s->d_w, sizeof(float) * (size_t)s->N, hipMemcpyDeviceToHost),
               "read code w");
        RB_HIP(hipMemcpy(gcat.data() + goff[k], s->d_gamma, sizeof(float) * (size_t)R * s->N,
                         hipMemcpyDeviceToHost),
               "read code gamma");
    }
    rb_status st = upload(&m->d_wcat, wcat, "upload code w");
    if (st != RB_OK) return st;
    if ((st = upload(&m->d_gcat, gcat, "upload code gamma")) != RB_OK) return st;
    std::vector<int32_t> fam_uniform(rep.size(), 1);
    for (size_t k = 0; k < nc; ++k)
        if (!w_is_uniform(m->subs[k])) fam_uniform[(size_t)fam[k]] = 0;
    for (size_t k = 0; k < nc; ++k) {
        cs[k].w = m->d_wcat + woff[k];
        cs[k].gamma = m->d_gcat + goff[k];
        cs[k].w_uniform = fam_uniform[(size_t)fam[k]];
        cs[k].w0 = m->subs[k]->w.empty() ? 0.0f : m->subs[k]->w[0];
    }
    if ((st = upload(&m->d_codes, cs, "upload code table")) != RB_OK) return st;
    if ((st = upload(&m->d_code_member, member, "upload code members")) != RB_OK) return st;
    m->nfam = (int32_t)rep.size();
    if ((st = upload(&m->d_code_fam, fam, "upload code families")) != RB_OK) return st;
    if ((st = upload(&m->d_fam_rep, rep, "upload family members")) != RB_OK) return st;
    if ((st = upload(&m->d_fam_size, size, "upload family sizes")) != RB_OK) return st;
    m->lds_bytes = lds;
    int blocks = 0;
    RB_HIP(rb::mixed_occupancy(m->params.anchor == RB_ANCHOR_PRIOR, (size_t)lds, &blocks), "occupancy query");
    if (blocks < 1) return fail(RB_E_UNSUPPORTED, "mixed kernel does not fit on a CU");
    m->blocks_per_cu[0] = m->blocks_per_cu[1] = blocks;
    return RB_OK;
}

}  // namespace

rb_status rb_create_multi(rb_ctx **out, int32_t n_codes, const rb_code_desc *codes, const rb_params *params,
                          int32_t device) try {
    g_last_error.clear();
    if (!out) return fail(RB_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_codes < 1 || n_codes > 64 || !codes) return fail(RB_E_INVALID_ARG, "need 1..64 code descriptors");
    rb_status st = check_params(params);
    if (st != RB_OK) return st;
    if (params->precision != RB_PREC_F32)
        return fail(RB_E_UNSUPPORTED, "the mixed launch decodes in FP32 (RB_PREC_F32)");
    CtxPtr own(new (std::nothrow) rb_ctx());
    rb_ctx *m = own.get();
    if (!m) return fail(RB_E_OOM, "host allocation failed");
    m->subs.reserve((size_t)n_codes);  // so that adding a created code cannot throw
    m->multi = true;
    m->device = device;
    m->params = *params;
    for (int32_t k = 0; k < n_codes; ++k) {
        rb_ctx *s = nullptr;
        st = rb_create(&s, codes[k].M, codes[k].N, codes[k].nnz, codes[k].rows, codes[k].cols, codes[k].prior_p,
                       params, device);
        if (st != RB_OK) {
            const std::string msg = "code " + std::to_string(k) + ": " + g_last_error;
            return fail(st, msg);
        }
        m->subs.push_back(s);
        // cheapest tile of the mixed set that fits this code
        int best = -1;
        double best_cost = 0.0;
        for (int v = 0; v < rb::num_variants(); ++v) {
            if (rb::mixed_tile_of_variant(v) < 0 || !variant_fits(s, rb::variant_shape(v))) continue;
            const double cost = variant_cost(rb::variant_shape(v));
            if (best < 0 || cost < best_cost) {
                best = v;
                best_cost = cost;
            }
        }
        if (best < 0) return fail(RB_E_UNSUPPORTED, "code " + std::to_string(k) + " fits no tile of the mixed launch");
        if ((st = plan(s, best)) != RB_OK) return st;
        m->m_max = std::max(m->m_max, s->M);
        m->n_max = std::max(m->n_max, s->N);
    }
    m->num_cu = m->subs[0]->num_cu;
    m->M = m->m_max;
    m->N = m->n_max;
    std::vector<int32_t> ms;
    for (rb_ctx *s : m->subs) ms.push_back(s->M);
    if ((st = upload(&m->d_code_m, ms, "upload code rows")) != RB_OK || (st = upload_codes(m)) != RB_OK) return st;
    hipError_t e = hipMalloc(&m->d_queues, sizeof(unsigned long long) * rb::kQueueWords * (size_t)n_codes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(queues)");
    *out = own.release();
    return RB_OK;
} catch (...) {
    return host_exception();
}

// The mixed launch of rb_decode_multi: shot lists in `ws` (at least
// shot_list_bytes(B, n_codes) bytes), one queue of kQueueWords counters per
// code at `queues`.  Arguments are validated by the callers.
static rb_status launch_decode_multi(rb_ctx *c, int64_t B, const int32_t *d_code_id, const uint8_t *d_syn,
                                     uint8_t *d_corr, uint8_t *d_conv, int32_t *d_legs, int32_t *d_iters,
                                     double *d_weight, float *d_final_llr, void *ws_bytes,
                                     unsigned long long *queues, hipStream_t s) {
    const int nc = (int)c->subs.size();
    const bool bits = c->params.io_layout == RB_IO_BITS32;
    const int32_t syn_stride = bits ? (c->m_max + 31) / 32 : c->m_max;
    RB_HIP(rb::launch_shot_lists(B, d_syn, syn_stride, bits, d_code_id, c->d_code_m, nc, c->d_code_fam, c->nfam,
                                 c->d_code_member, ws_bytes, queues, s),
           "shot list kernels");
    rb::MixedArgs m{};
    m.run = base_args(c->subs[0], B, d_syn);
    m.run.syn_stride = syn_stride;
    m.run.corr_stride = bits ? (c->n_max + 31) / 32 : c->n_max;
    m.run.llr_stride = c->n_max;
    m.run.corr = d_corr;
    m.run.conv = d_conv;
    m.run.legs = d_legs;
    m.run.iters = d_iters;
    m.run.weight = d_weight;
    m.run.final_llr = d_final_llr;
    m.codes = c->d_codes;
    m.ncodes = nc;
    m.nfam = c->nfam;
    m.fam_rep = c->d_fam_rep;
    m.fam_size = c->d_fam_size;
    const int32_t *ws = (const int32_t *)ws_bytes;
    m.seg_start = ws + (size_t)nc * rb::kWeightBinsHost;
    m.seg_count = m.seg_start + nc;
    m.order = m.seg_count + nc;
    m.list = ws + (size_t)nc * (rb::kWeightBinsHost + 3) + (size_t)B;
    m.list_cid = m.list + B;
    m.queues = queues;
    const int64_t full = (int64_t)c->blocks_per_cu[0] * c->num_cu;
    const int grid = (int)std::max<int64_t>(1, full);
    RB_HIP(rb::launch_mixed(c->params.anchor == RB_ANCHOR_PRIOR, m, grid, (size_t)c->lds_bytes, s),
           "mixed kernel launch");
    return RB_OK;
}

static rb_status check_multi_args(const rb_ctx *c, int64_t B, const int32_t *d_code_id, const uint8_t *d_syn,
                                  const uint8_t *d_corr, const uint8_t *d_conv, const int32_t *d_legs,
                                  const int32_t *d_iters) {
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    if (!c->multi) return fail(RB_E_INVALID_ARG, "not a mixed-code context");
    if (B < 0) return fail(RB_E_INVALID_ARG, "B must be >= 0");
    if (B > INT32_MAX) return fail(RB_E_SHAPE, "B exceeds 2^31 - 1");
    if (B > 0 && (!d_code_id || !d_syn || !d_corr || !d_conv || !d_legs || !d_iters))
        return fail(RB_E_INVALID_ARG, "a required device pointer is NULL");
    return RB_OK;
}

rb_status rb_decode_multi(rb_ctx *c, int64_t B, const int32_t *d_code_id, const uint8_t *d_syn, uint8_t *d_corr,
                          uint8_t *d_conv, int32_t *d_legs, int32_t *d_iters, double *d_weight,
                          float *d_final_llr, void *d_workspace, size_t workspace_bytes, void *stream) try {
    g_last_error.clear();
    rb_status st = check_multi_args(c, B, d_code_id, d_syn, d_corr, d_conv, d_legs, d_iters);
    if (st != RB_OK || B == 0) return st;
    if (!d_workspace) return fail(RB_E_INVALID_ARG, "a required device pointer is NULL");
    const int nc = (int)c->subs.size();
    if (workspace_bytes < rb::shot_list_bytes(B, nc)) return fail(RB_E_WORKSPACE, "workspace too small");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    return launch_decode_multi(c, B, d_code_id, d_syn, d_corr, d_conv, d_legs, d_iters, d_weight, d_final_llr,
                               d_workspace, c->d_queues, (hipStream_t)stream);
} catch (...) {
    return host_exception();
}

// Layout of the static scratch for a context of nc codes: nc queues, then
// the shot lists at the next 256-byte boundary.
static size_t noalloc_list_offset(int nc) {
    const size_t q = sizeof(unsigned long long) * rb::kQueueWords * (size_t)nc;
    return (q + 255) / 256 * 256;
}

int64_t rb_noalloc_max_batch(const rb_ctx *c) {
    if (!c || !c->multi) return 0;
    const int nc = (int)c->subs.size();
    const size_t off = noalloc_list_offset(nc);
    const size_t head = rb::shot_list_bytes(0, nc);
    if (off + head > rb::kNoAllocScratchBytes) return 0;
    return (int64_t)((rb::kNoAllocScratchBytes - off - head) / (3 * sizeof(int32_t)));
}

rb_status rb_decode_multi_noalloc(rb_ctx *c, int64_t B, const int32_t *d_code_id, const uint8_t *d_syn,
                                  uint8_t *d_corr, uint8_t *d_conv, int32_t *d_legs, int32_t *d_iters,
                                  double *d_weight, float *d_final_llr, void *stream) try {
    g_last_error.clear();
    rb_status st = check_multi_args(c, B, d_code_id, d_syn, d_corr, d_conv, d_legs, d_iters);
    if (st != RB_OK || B == 0) return st;
    const int64_t bmax = rb_noalloc_max_batch(c);
    if (B > bmax)
        return fail(RB_E_WORKSPACE, "B = " + std::to_string(B) + " exceeds the static scratch of " +
                                        std::to_string(rb::kNoAllocScratchBytes) + " bytes (at most " +
                                        std::to_string(bmax) + " syndromes for this context)");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    void *base = nullptr;
    RB_HIP(rb::noalloc_scratch(c->device, &base), "static scratch address");
    const int nc = (int)c->subs.size();
    return launch_decode_multi(c, B, d_code_id, d_syn, d_corr, d_conv, d_legs, d_iters, d_weight, d_final_llr,
                               (unsigned char *)base + noalloc_list_offset(nc), (unsigned long long *)base,
                               (hipStream_t)stream);
} catch (...) {
    return host_exception();
}

rb_status rb_autotune_multi(rb_ctx *c, const int64_t *sample_b, const uint8_t *const *d_samples, int32_t reps,
                            int32_t *chosen_variants) try {
    g_last_error.clear();
    if (!c || !c->multi) return fail(RB_E_INVALID_ARG, "not a mixed-code context");
    if (!sample_b || !d_samples || reps < 1) return fail(RB_E_INVALID_ARG, "bad samples");
    for (size_t k = 0; k < c->subs.size(); ++k) {
        rb_ctx *s = c->subs[k];
        if (sample_b[k] >= 1 && d_samples[k]) {
            int best = -1;
            float best_t = 0.0f;
            for (int v = 0; v < rb::num_variants(); ++v) {
                if (rb::mixed_tile_of_variant(v) < 0 || !variant_fits(s, rb::variant_shape(v))) continue;
                rb_status st = rb_set_variant(s, v);
                if (st != RB_OK) return st;
                float ms = 0.0f;
                st = time_variant(s, sample_b[k], d_samples[k], reps, &ms);
                if (st != RB_OK) return st;
                if (best < 0 || ms < best_t) {
                    best = v;
                    best_t = ms;
                }
            }
            if (best >= 0) {
                rb_status st = rb_set_variant(s, best);
                if (st != RB_OK) return st;
            }
        }
        if (chosen_variants) chosen_variants[k] = s->variant;
    }
    return upload_codes(c);
} catch (...) {
    return host_exception();
}

rb_status rb_set_code_variant(rb_ctx *c, int32_t k, int32_t variant) try {
    g_last_error.clear();
    if (!c || !c->multi) return fail(RB_E_INVALID_ARG, "not a mixed-code context");
    if (k < 0 || k >= (int32_t)c->subs.size()) return fail(RB_E_INVALID_ARG, "code index out of range");
    if (variant < 0 || variant >= rb::num_variants() || rb::mixed_tile_of_variant(variant) < 0)
        return fail(RB_E_UNSUPPORTED, "not a tile of the mixed kernel");
    if (!variant_fits(c->subs[(size_t)k], rb::variant_shape(variant)))
        return fail(RB_E_UNSUPPORTED, "the code does not fit the tile");
    rb_status st = rb_set_variant(c->subs[(size_t)k], variant);
    if (st != RB_OK) return st;
    return upload_codes(c);
} catch (...) {
    return host_exception();
}

rb_status rb_sync_status(rb_ctx *c) try {
    if (!c) return fail(RB_E_INVALID_ARG, "ctx is NULL");
    RB_HIP(hipSetDevice(c->device), "hipSetDevice");
    RB_HIP(hipDeviceSynchronize(), "device synchronize");
    RB_HIP(hipGetLastError(), "asynchronous error");
    return RB_OK;
} catch (...) {
    return host_exception();
}

}  // extern "C"
