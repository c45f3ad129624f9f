// Host planning of the FBC library: plain C++ on geometry and integers only (no HIP types),
// so that the same code builds into the library and, with the address and
// undefined-behaviour sanitizers, into a CPU check program.
//  * distinct column offsets n_b - n_i and their dense lookup (Section 3.2: the Green
//    blocks depend on the offset only);
//  * negligible-block windows of the dense and offset-table products;
//  * cluster trees and the block partition of the H-matrix form (Appendix C).
#pragma once
#include <cstdint>
#include <vector>

// One cell's columns: lattice indices (n1, n2) per column, [n][2].
struct PlanGeom {
    int n_i, n_b;
    const int32_t* cols_i;
    const int32_t* cols_b;
};

// Distinct offsets (d1, d2) = col_b - col_i over every cell, numbered row-major over their
// bounding box [d1min, d1min + w1) x [d2min, d2min + w2); lut[(d1 - d1min) w2 + d2 - d2min]
// is the offset's number, -1 for none.
struct PlanOffsets {
    int d1min = 0, d2min = 0, w1 = 0, w2 = 0;
    std::vector<int32_t> lut, d1, d2;
};
PlanOffsets plan_offsets(const std::vector<PlanGeom>& cells);

// In-plane distance of column a from column b (a = 1, c = a / sqrt 2).
double plan_pair_rho(int32_t a1, int32_t a2, int32_t b1, int32_t b2);

// Negligible-block windows of one cell.  Row tiles of the product: table_form ? 32 pad
// columns : rows_tile rows (mp / tile rows of them); K chunks: table_form ? 8 interface
// columns : 64 of the kp padded reals.  At cell mode m (table mode m * mult, rho_cut
// indexed by table mode) a chunk is negligible for a tile when every (pad, interface)
// pair of the two lies farther than rho_cut; per (mode, tile) the window is the cyclic
// run [win_start, win_start + win_len) of chunks left after removing the longest cyclic
// run of negligible chunks.  mode_skips[m] = 1 when some real chunk of some non-empty
// tile lies outside its window.
struct PlanWindows {
    int n_tiles = 0, n_chunks = 0;
    std::vector<int32_t> win_start, win_len;   // [nm][n_tiles]
    std::vector<uint8_t> mode_skips;           // [nm]
};
void plan_windows(const PlanGeom& g, int nm, int mp, int kp, bool table_form, int rows_tile, int mult,
                  const std::vector<double>& rho_cut, PlanWindows& out);

// Cluster tree node: columns in tree order and the bounding box in the integer coordinates
// X = n1, Y = n1 + 2 n2 (in-plane x = X / 2, y = Y / (2 sqrt 2)).
struct PlanNode {
    std::vector<int> idx;
    long long xlo, xhi, ylo, yhi, sx, sy;
    long long n, diam8;               // 8 diam^2 = 2 dX^2 + dY^2
    int child[2] = {-1, -1};
};
// Binary space partitioning of the columns idx: each cluster is cut along the longer side
// of its bounding box at the median (ties by column index) until it holds at most b_min
// columns.  Appends the nodes (root first, children after their parent) and returns the
// index of the subtree's root.
int plan_tree(std::vector<PlanNode>& nodes, const std::vector<int32_t>& cols, std::vector<int> idx, int b_min);
// min(diam t, diam s) <= gamma dist(t, s) on the bounding boxes, in exact integers.
bool plan_admissible(const PlanNode& t, const PlanNode& s, int gamma);

struct PlanBlock {
    int kind;      // 1 low rank, 0 dense
    int t, s;      // tree nodes
};
// Block partition of t x s: admissible blocks low rank, pairs of leaves dense, every other
// block subdivided (a leaf side kept whole).
void plan_partition(const std::vector<PlanNode>& tb, const std::vector<PlanNode>& ti, int t, int s, int gamma,
                    std::vector<PlanBlock>& out);
