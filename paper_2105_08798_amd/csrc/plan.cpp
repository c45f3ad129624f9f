// Host planning (see plan.h).
#include "plan.h"

#include <algorithm>
#include <climits>
#include <cmath>

PlanOffsets plan_offsets(const std::vector<PlanGeom>& cells) {
    PlanOffsets o;
    int lo1 = INT_MAX, hi1 = INT_MIN, lo2 = INT_MAX, hi2 = INT_MIN;
    for (const PlanGeom& p : cells) {
        int b1lo = INT_MAX, b1hi = INT_MIN, b2lo = INT_MAX, b2hi = INT_MIN;
        int i1lo = INT_MAX, i1hi = INT_MIN, i2lo = INT_MAX, i2hi = INT_MIN;
        for (int b = 0; b < p.n_b; ++b) {
            b1lo = std::min(b1lo, p.cols_b[2 * b]);
            b1hi = std::max(b1hi, p.cols_b[2 * b]);
            b2lo = std::min(b2lo, p.cols_b[2 * b + 1]);
            b2hi = std::max(b2hi, p.cols_b[2 * b + 1]);
        }
        for (int i = 0; i < p.n_i; ++i) {
            i1lo = std::min(i1lo, p.cols_i[2 * i]);
            i1hi = std::max(i1hi, p.cols_i[2 * i]);
            i2lo = std::min(i2lo, p.cols_i[2 * i + 1]);
            i2hi = std::max(i2hi, p.cols_i[2 * i + 1]);
        }
        lo1 = std::min(lo1, b1lo - i1hi);
        hi1 = std::max(hi1, b1hi - i1lo);
        lo2 = std::min(lo2, b2lo - i2hi);
        hi2 = std::max(hi2, b2hi - i2lo);
    }
    o.d1min = lo1;
    o.d2min = lo2;
    o.w1 = hi1 - lo1 + 1;
    o.w2 = hi2 - lo2 + 1;
    o.lut.assign((size_t)o.w1 * o.w2, -1);
    for (const PlanGeom& p : cells)
        for (int b = 0; b < p.n_b; ++b)
            for (int i = 0; i < p.n_i; ++i) {
                const int x = p.cols_b[2 * b] - p.cols_i[2 * i] - o.d1min;
                const int y = p.cols_b[2 * b + 1] - p.cols_i[2 * i + 1] - o.d2min;
                o.lut[(size_t)x * o.w2 + y] = 0;
            }
    int32_t n = 0;
    for (int x = 0; x < o.w1; ++x)
        for (int y = 0; y < o.w2; ++y) {
            int32_t& e = o.lut[(size_t)x * o.w2 + y];
            if (e == 0) {
                e = n++;
                o.d1.push_back(x + o.d1min);
                o.d2.push_back(y + o.d2min);
            }
        }
    return o;
}

double plan_pair_rho(int32_t a1, int32_t a2, int32_t b1, int32_t b2) {
    const int d1 = a1 - b1, d2 = a2 - b2;
    const double x = 0.5 * d1, y = (d1 + 2.0 * d2) * (0.5 * M_SQRT1_2);
    return std::sqrt(x * x + y * y);
}

void plan_windows(const PlanGeom& p, int nm, int mp, int kp, bool dt, int rows_tile, int mult,
                  const std::vector<double>& rho_cut, PlanWindows& out) {
    out.n_tiles = dt ? mp / 96 : mp / rows_tile;
    out.n_chunks = dt ? (p.n_i + 7) / 8 : kp / 64;
    const int NT_ = out.n_tiles, NC = out.n_chunks;
    // pad columns of a tile and interface columns of a chunk
    auto tile_cols = [&](int tl, int& b0, int& b1) {
        if (dt) {
            b0 = 32 * tl;
            b1 = std::min(p.n_b, b0 + 32);
        } else {
            b0 = (tl * rows_tile) / 3;
            b1 = std::min(p.n_b, ((tl + 1) * rows_tile + 2) / 3);
        }
    };
    auto chunk_cols = [&](int ch, int& i0, int& i1) {
        if (dt) {
            i0 = 8 * ch;
            i1 = std::min(p.n_i, i0 + 8);
        } else {
            i0 = (32 * ch) / 3;
            i1 = std::min(p.n_i, (32 * (ch + 1) + 2) / 3);
        }
    };
    std::vector<float> rmin((size_t)NT_ * NC, INFINITY);
    std::vector<uint8_t> real_chunk(NC, 0);
    for (int ch = 0; ch < NC; ++ch) {
        int i0, i1;
        chunk_cols(ch, i0, i1);
        real_chunk[ch] = i0 < i1;
    }
    for (int tl = 0; tl < NT_; ++tl) {
        int b0, b1;
        tile_cols(tl, b0, b1);
        for (int b = b0; b < b1; ++b) {
            const int32_t a1 = p.cols_b[2 * b], a2 = p.cols_b[2 * b + 1];
            for (int ch = 0; ch < NC; ++ch) {
                int i0, i1;
                chunk_cols(ch, i0, i1);
                float& r = rmin[(size_t)tl * NC + ch];
                for (int i = i0; i < i1; ++i)
                    r = std::min(r, (float)plan_pair_rho(a1, a2, p.cols_i[2 * i], p.cols_i[2 * i + 1]));
            }
        }
    }
    out.win_start.assign((size_t)nm * NT_, 0);
    out.win_len.assign((size_t)nm * NT_, NC);
    out.mode_skips.assign(nm, 0);
    std::vector<uint8_t> neg(NC);
    for (int m = 0; m < nm; ++m) {
        const double rc = rho_cut[(size_t)m * mult];
        for (int tl = 0; tl < NT_; ++tl) {
            int b0, b1;
            tile_cols(tl, b0, b1);
            int nneg = 0;
            for (int ch = 0; ch < NC; ++ch) {
                // (float) rmin rounds; a 1e-6 relative margin keeps the test on the safe side
                neg[ch] = (double)rmin[(size_t)tl * NC + ch] > rc * (1.0 + 1e-6) + 1e-6;
                nneg += neg[ch];
            }
            int start = 0, len = NC;
            if (nneg == NC) {
                len = 0;
            } else if (nneg > 0) {
                // longest cyclic run of negligible chunks
                int best = 0, best_end = 0, run = 0;
                for (int q = 0; q < 2 * NC; ++q) {
                    if (neg[q % NC]) {
                        ++run;
                        if (run > best && run <= NC) {
                            best = run;
                            best_end = q;
                        }
                    } else {
                        run = 0;
                    }
                }
                start = (best_end + 1) % NC;
                len = NC - best;
            }
            out.win_start[(size_t)m * NT_ + tl] = start;
            out.win_len[(size_t)m * NT_ + tl] = len;
            if (b0 < b1 && len < NC)
                for (int ch = 0; ch < NC; ++ch) {
                    const bool in = ((ch - start + NC) % NC) < len;
                    if (!in && real_chunk[ch]) out.mode_skips[m] = 1;
                }
        }
    }
}

int plan_tree(std::vector<PlanNode>& nodes, const std::vector<int32_t>& cols, std::vector<int> idx, int b_min) {
    PlanNode h;
    h.n = (long long)idx.size();
    h.xlo = h.ylo = (1LL << 40);
    h.xhi = h.yhi = -(1LL << 40);
    h.sx = h.sy = 0;
    for (int c : idx) {
        const long long X = cols[2 * c], Y = (long long)cols[2 * c] + 2LL * cols[2 * c + 1];
        h.xlo = std::min(h.xlo, X);
        h.xhi = std::max(h.xhi, X);
        h.ylo = std::min(h.ylo, Y);
        h.yhi = std::max(h.yhi, Y);
        h.sx += X;
        h.sy += Y;
    }
    const long long dx = h.xhi - h.xlo, dy = h.yhi - h.ylo;
    h.diam8 = 2 * dx * dx + dy * dy;
    const int me = (int)nodes.size();
    nodes.push_back(h);
    if ((int)idx.size() > b_min) {
        const bool on_x = 2 * dx * dx >= dy * dy;      // longer side of the bounding box
        auto key = [&](int c) -> long long {
            return on_x ? (long long)cols[2 * c] : (long long)cols[2 * c] + 2LL * cols[2 * c + 1];
        };
        std::sort(idx.begin(), idx.end(), [&](int a, int b) {
            const long long ka = key(a), kb = key(b);
            return ka != kb ? ka < kb : a < b;
        });
        const size_t half = idx.size() / 2;
        std::vector<int> lo(idx.begin(), idx.begin() + half), hi(idx.begin() + half, idx.end());
        const int c0 = plan_tree(nodes, cols, lo, b_min);
        const int c1 = plan_tree(nodes, cols, hi, b_min);
        nodes[me].child[0] = c0;
        nodes[me].child[1] = c1;
        nodes[me].idx.clear();
        nodes[me].idx.insert(nodes[me].idx.end(), nodes[c0].idx.begin(), nodes[c0].idx.end());
        nodes[me].idx.insert(nodes[me].idx.end(), nodes[c1].idx.begin(), nodes[c1].idx.end());
    } else {
        nodes[me].idx = idx;
    }
    return me;
}

// 8 diam^2 = 2 dX^2 + dY^2 and 8 dist^2 = 2 gX^2 + gY^2 (gX, gY: gaps between the boxes).
bool plan_admissible(const PlanNode& t, const PlanNode& s, int gamma) {
    const long long gx = std::max(0LL, std::max(s.xlo - t.xhi, t.xlo - s.xhi));
    const long long gy = std::max(0LL, std::max(s.ylo - t.yhi, t.ylo - s.yhi));
    return std::min(t.diam8, s.diam8) <= (long long)gamma * gamma * (2 * gx * gx + gy * gy);
}

void plan_partition(const std::vector<PlanNode>& tb, const std::vector<PlanNode>& ti, int t, int s, int gamma,
                    std::vector<PlanBlock>& out) {
    if (plan_admissible(tb[t], ti[s], gamma)) {
        out.push_back({1, t, s});
        return;
    }
    const bool tl = tb[t].child[0] < 0, sl = ti[s].child[0] < 0;
    if (tl && sl) {
        out.push_back({0, t, s});
        return;
    }
    const int tc[2] = {tl ? t : tb[t].child[0], tl ? -1 : tb[t].child[1]};
    const int sc[2] = {sl ? s : ti[s].child[0], sl ? -1 : ti[s].child[1]};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            if (tc[a] >= 0 && sc[b] >= 0) plan_partition(tb, ti, tc[a], sc[b], gamma, out);
}
