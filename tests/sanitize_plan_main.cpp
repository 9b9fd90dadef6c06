// sanitize_plan_main.cpp -- drives the host-side planner of librelaybp
// (rb_plan_check: CSR / CSC layouts, gather tables of every kernel
// configuration, the bank-aware plans, the large-graph tables and their
// consistency checks) on generated graphs, for a build with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host code.  No GPU is used.
// Exit status 0 iff every call returns RB_OK or RB_E_UNSUPPORTED.
#include <cstdint>
#include <cstdio>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "../include/relaybp.h"

struct Graph {
    const char *name;
    int m, n;
    std::vector<int32_t> rows, cols;
};

// HX = [A | B] of a bivariate-bicycle code: A, B sums of x^a y^b monomials
// with x = S_l (x) I_m, y = I_l (x) S_m acting on index u * m + v.
static Graph bb(const char *name, int l, int m, std::vector<std::pair<int, int>> a, std::vector<std::pair<int, int>> b) {
    Graph g{name, l * m, 2 * l * m, {}, {}};
    for (int half = 0; half < 2; ++half)
        for (auto [px, py] : half ? b : a)
            for (int u = 0; u < l; ++u)
                for (int v = 0; v < m; ++v) {
                    g.rows.push_back(u * m + v);
                    g.cols.push_back(half * l * m + ((u + px) % l) * m + (v + py) % m);
                }
    return g;
}

static Graph random_graph(const char *name, int m, int n, double p, unsigned seed, int max_col) {
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    Graph g{name, m, n, {}, {}};
    std::vector<int> deg(n, 0);
    for (int i = 0; i < m; ++i) {
        if (i == m / 3) continue;  // an empty row
        for (int j = 0; j < n; ++j)
            if (j != n / 2 && deg[j] < max_col && u(rng) < p) {  // column n/2 stays empty
                g.rows.push_back(i);
                g.cols.push_back(j);
                ++deg[j];
            }
    }
    return g;
}

// banded detector-error-model-like matrix: columns of weight 2..6 in a band
static Graph banded(const char *name, int m, int n, int band, unsigned seed) {
    std::mt19937 rng(seed);
    Graph g{name, m, n, {}, {}};
    const int w[10] = {2, 2, 2, 3, 3, 3, 4, 4, 5, 6};
    for (int j = 0; j < n; ++j) {
        const int k = w[rng() % 10];
        const int s = (int)(rng() % (unsigned)(m - band + 1));
        std::set<int> rs;
        while ((int)rs.size() < k) rs.insert(s + (int)(rng() % (unsigned)band));
        for (int r : rs) {
            g.rows.push_back(r);
            g.cols.push_back(j);
        }
    }
    return g;
}

int main() {
    std::vector<Graph> gs;
    gs.push_back(bb("bb72", 6, 6, {{3, 0}, {0, 1}, {0, 2}}, {{0, 3}, {1, 0}, {2, 0}}));
    gs.push_back(bb("bb90", 15, 3, {{9, 0}, {0, 1}, {0, 2}}, {{0, 0}, {2, 0}, {7, 0}}));
    gs.push_back(bb("bb144", 12, 6, {{3, 0}, {0, 1}, {0, 2}}, {{0, 3}, {1, 0}, {2, 0}}));
    gs.push_back(random_graph("irregular40x90", 40, 90, 0.06, 1, 8));
    gs.push_back(random_graph("irregular200x500", 200, 500, 0.02, 2, 6));
    gs.push_back(random_graph("longrows60x700", 60, 700, 0.07, 3, 6));
    gs.push_back(banded("banded216x1800", 216, 1800, 72, 4));
    int bad = 0, checked = 0;
    for (const Graph &g : gs) {
        rb_plan_report rep;
        for (int v = -1; v < 19; ++v) {
            const rb_status st = rb_plan_check(g.m, g.n, (int64_t)g.rows.size(), g.rows.data(), g.cols.data(), v, &rep);
            if (st == RB_E_INVALID_ARG && v >= 0) break;  // past the configuration table
            if (st != RB_OK && st != RB_E_UNSUPPORTED) {
                std::printf("%s variant %d: %s (%s)\n", g.name, v, rb_status_string(st), rb_last_error_message());
                ++bad;
            }
            checked += st == RB_OK;
        }
    }
    rb_params p;
    if (rb_params_default(&p) != RB_OK) ++bad;
    std::printf("plan checks passed: %d, failures: %d\n", checked, bad);
    return bad ? 1 : 0;
}
