// CPU check of the library's host planning (paper_2105_08798_amd/csrc/plan.cpp), built with
// the address and undefined-behaviour sanitizers by tests/test_plan_sanitized.py.
// Input file: int32 n_cells, then per cell n_i, n_b, cols_i[n_i][2], cols_b[n_b][2].
// Checks, for every cell set in the file:
//  * offsets: every (pad, interface) pair maps through the lookup to an offset holding its
//    difference; offsets distinct and numbered row-major; their count is the number of
//    distinct differences;
//  * windows (dense and offset-table tiling, several cut-off radii): every (tile, chunk)
//    with a pair within the cut-off lies inside its window; ranges valid;
//  * cluster trees and partition (several b_min, gamma): every pair covered by exactly one
//    block; leaves within b_min; a node's columns are its children's; low-rank blocks
//    admissible, dense blocks pairs of leaves.
// Prints "ok" and returns 0, or the first failure and 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <utility>
#include <vector>

#include "plan.h"

static int fails = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            if (++fails > 20) std::exit(1);               \
        }                                                 \
    } while (0)

struct Cell {
    int n_i, n_b;
    std::vector<int32_t> ci, cb;
};

static void check_offsets(const std::vector<Cell>& cells) {
    std::vector<PlanGeom> g;
    for (const Cell& c : cells) g.push_back(PlanGeom{c.n_i, c.n_b, c.ci.data(), c.cb.data()});
    const PlanOffsets o = plan_offsets(g);
    std::set<std::pair<int, int>> diffs;
    for (const Cell& c : cells)
        for (int b = 0; b < c.n_b; ++b)
            for (int i = 0; i < c.n_i; ++i) {
                const int d1 = c.cb[2 * b] - c.ci[2 * i], d2 = c.cb[2 * b + 1] - c.ci[2 * i + 1];
                diffs.insert({d1, d2});
                const int x = d1 - o.d1min, y = d2 - o.d2min;
                CHECK(x >= 0 && x < o.w1 && y >= 0 && y < o.w2, "offset outside the box");
                const int32_t e = o.lut[(size_t)x * o.w2 + y];
                CHECK(e >= 0 && e < (int32_t)o.d1.size(), "pair without an offset");
                if (e >= 0 && e < (int32_t)o.d1.size()) CHECK(o.d1[e] == d1 && o.d2[e] == d2, "wrong offset");
            }
    CHECK(diffs.size() == o.d1.size(), "offset count %zu vs %zu", o.d1.size(), diffs.size());
    for (size_t k = 1; k < o.d1.size(); ++k)
        CHECK(o.d1[k - 1] < o.d1[k] || (o.d1[k - 1] == o.d1[k] && o.d2[k - 1] < o.d2[k]), "not row-major");
}

static void check_windows(const Cell& c) {
    const int nm = 9;
    for (int dt = 0; dt < 2; ++dt) {
        const int rows_tile = 128;
        const int mp = dt ? ((3 * c.n_b + 95) / 96) * 96 : ((3 * c.n_b + rows_tile - 1) / rows_tile) * rows_tile;
        const int kp = ((6 * c.n_i + 63) / 64) * 64;
        for (double base : {0.0, 1.0, 3.5, 8.0, 1e9}) {
            std::vector<double> cut(nm);
            for (int m = 0; m < nm; ++m) cut[m] = (m == 0) ? INFINITY : base * (1.0 + 0.3 * m);
            PlanWindows w;
            plan_windows(PlanGeom{c.n_i, c.n_b, c.ci.data(), c.cb.data()}, nm, mp, kp, dt != 0, rows_tile, 1, cut, w);
            const int NT = w.n_tiles, NC = w.n_chunks;
            CHECK((int)w.win_start.size() == nm * NT && (int)w.win_len.size() == nm * NT, "window sizes");
            for (int m = 0; m < nm; ++m)
                for (int tl = 0; tl < NT; ++tl) {
                    const int s = w.win_start[(size_t)m * NT + tl], len = w.win_len[(size_t)m * NT + tl];
                    CHECK(s >= 0 && (s < NC || NC == 0) && len >= 0 && len <= NC, "window range");
                    const int b0 = dt ? 32 * tl : (tl * rows_tile) / 3;
                    const int b1 = dt ? std::min(c.n_b, b0 + 32) : std::min(c.n_b, ((tl + 1) * rows_tile + 2) / 3);
                    for (int ch = 0; ch < NC; ++ch) {
                        const int i0 = dt ? 8 * ch : (32 * ch) / 3;
                        const int i1 = dt ? std::min(c.n_i, i0 + 8) : std::min(c.n_i, (32 * (ch + 1) + 2) / 3);
                        double rmin = INFINITY;
                        for (int b = b0; b < b1; ++b)
                            for (int i = i0; i < i1; ++i) {
                                const int d1 = c.cb[2 * b] - c.ci[2 * i], d2 = c.cb[2 * b + 1] - c.ci[2 * i + 1];
                                const double x = 0.5 * d1, y = (d1 + 2.0 * d2) * (0.5 * M_SQRT1_2);
                                rmin = std::min(rmin, std::sqrt(x * x + y * y));
                            }
                        if (rmin <= cut[m]) {
                            const bool in = ((ch - s + NC) % NC) < len;
                            CHECK(in, "chunk %d of tile %d (mode %d) within the cut-off but outside its window", ch,
                                  tl, m);
                        }
                    }
                }
        }
    }
}

static void check_tree_node(const std::vector<PlanNode>& t, int n, int b_min) {
    const PlanNode& x = t[n];
    if (x.child[0] < 0) {
        CHECK((int)x.idx.size() <= b_min, "leaf of %zu columns", x.idx.size());
        return;
    }
    std::vector<int> cat = t[x.child[0]].idx;
    cat.insert(cat.end(), t[x.child[1]].idx.begin(), t[x.child[1]].idx.end());
    CHECK(cat == x.idx, "node columns differ from its children's");
    check_tree_node(t, x.child[0], b_min);
    check_tree_node(t, x.child[1], b_min);
}

static void check_partition(const Cell& c) {
    for (int b_min : {1, 7, 20})
        for (int gamma : {1, 2, 4}) {
            std::vector<PlanNode> tb, ti;
            std::vector<int> all_b(c.n_b), all_i(c.n_i);
            for (int k = 0; k < c.n_b; ++k) all_b[k] = k;
            for (int k = 0; k < c.n_i; ++k) all_i[k] = k;
            plan_tree(tb, c.cb, all_b, b_min);
            plan_tree(ti, c.ci, all_i, b_min);
            check_tree_node(tb, 0, b_min);
            check_tree_node(ti, 0, b_min);
            std::vector<PlanBlock> part;
            plan_partition(tb, ti, 0, 0, gamma, part);
            std::vector<int> cover((size_t)c.n_b * c.n_i, 0);
            for (const PlanBlock& q : part) {
                if (q.kind == 1) CHECK(plan_admissible(tb[q.t], ti[q.s], gamma), "low-rank block not admissible");
                else CHECK(tb[q.t].child[0] < 0 && ti[q.s].child[0] < 0, "dense block of a non-leaf");
                for (int b : tb[q.t].idx)
                    for (int i : ti[q.s].idx) ++cover[(size_t)b * c.n_i + i];
            }
            for (size_t k = 0; k < cover.size(); ++k)
                if (cover[k] != 1) {
                    CHECK(false, "pair %zu covered %d times (b_min %d, gamma %d)", k, cover[k], b_min, gamma);
                    break;
                }
        }
}

int main(int argc, char** argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: plan_check <geometry file>\n");
        return 2;
    }
    FILE* fp = std::fopen(argv[1], "rb");
    if (!fp) return 2;
    auto rd = [&](int32_t* p, size_t n) { return std::fread(p, 4, n, fp) == n; };
    int32_t n_sets = 0;
    if (!rd(&n_sets, 1)) return 2;
    for (int s = 0; s < n_sets; ++s) {
        int32_t n_cells = 0;
        if (!rd(&n_cells, 1)) return 2;
        std::vector<Cell> cells(n_cells);
        for (Cell& c : cells) {
            int32_t hdr[2];
            if (!rd(hdr, 2)) return 2;
            c.n_i = hdr[0];
            c.n_b = hdr[1];
            c.ci.resize(2 * (size_t)c.n_i);
            c.cb.resize(2 * (size_t)c.n_b);
            if (!rd(c.ci.data(), c.ci.size()) || !rd(c.cb.data(), c.cb.size())) return 2;
        }
        check_offsets(cells);
        for (const Cell& c : cells) {
            check_windows(c);
            check_partition(c);
        }
    }
    std::fclose(fp);
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
