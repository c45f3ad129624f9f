// Shared definitions of the FBC library (host plan + device kernels), gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <cstdint>
#include <vector>

#include "../../include/fbc.h"

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

// Split-FP16 form: power-of-two scale exponent of a line mode's blocks from the largest
// table magnitude of that mode (bit pattern of a non-negative double).  |G - row mean|
// <= 2 max, so 2^e |G - row mean| < 2^14, inside the FP16 range with headroom.
__host__ __device__ inline int split16_exp_a(unsigned long long maxbits) {
    const double m = __longlong_as_double((long long)maxbits);
    return m > 0.0 ? 12 - ilogb(m) : 0;
}
typedef unsigned short us8_t __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------------
// MFMA fragment orders.  A real matrix X[rows][K'] (or the GEMM B operand, indexed
// [col][K'] the same way) is stored as 16-row blocks; inside a block the 64 lanes of a
// wave hold one MFMA operand each, so a wave-wide 16-byte load is 1 KiB contiguous.
//   FP64 16x16x4 : lane l holds X[16 blk + l%16][4 t + l/16]; two k-steps per 16 B.
//   FP32 16x16x4 : same lane map; four k-steps per 16 B.
//   BF16 16x16x32: lane l holds X[16 blk + l%16][32 t + 8 (l/16) + j], j = 0..7;
//                  hi and lo halves of the split are stored as consecutive 1 KiB runs.
// Output of the 16x16 MFMAs: FP64 c[j] = C[4 j + l/16][l%16];
//                            FP32 c[j] = C[4 (l/16) + j][l%16].
// K' is padded to a multiple of 64 for every form (zeros).
// The B operand (the transformed forces, one column per RHS and real/imaginary part)
// keeps each column's four 16-byte units of a block together: lane l's unit sits at
// position bpos(l) = 4 (l % 16) + l / 16 of its 1 KiB block, so the forward transform,
// which produces one column at a time, writes 64-byte runs; a wave still reads the
// whole block (lane order permuted).
// ---------------------------------------------------------------------------------
__host__ __device__ inline int bpos(int lane) { return ((lane & 15) << 2) | (lane >> 4); }

// Round-to-nearest FP64 -> FP16 through FP32.  The result equals direct rounding (FP32
// carries more than twice FP16's precision plus two bits, so the double rounding is
// innocuous).  The empty asm keeps the compiler from merging the two hardware
// conversions into one FP64 -> FP16 conversion, which it expands into a long integer
// sequence.
__device__ inline _Float16 f64_to_f16(double x) {
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return (_Float16)f;
}
__host__ __device__ inline int64_t frag_off_f64(int64_t r, int64_t k, int64_t kp) {
    int64_t blk = r >> 4, rr = r & 15;
    int64_t lane = ((k & 3) << 4) | rr;
    return (((blk * (kp >> 3) + (k >> 3)) * 64 + bpos((int)lane)) << 1) + ((k >> 2) & 1);
}
__host__ __device__ inline int64_t frag_off_f32(int64_t r, int64_t k, int64_t kp) {
    int64_t blk = r >> 4, rr = r & 15;
    int64_t lane = ((k & 3) << 4) | rr;
    return (((blk * (kp >> 4) + (k >> 4)) * 64 + bpos((int)lane)) << 2) + ((k >> 2) & 3);
}
// element offset (in bf16 units) of the hi part; the lo part is at +512
__host__ __device__ inline int64_t frag_off_bf16(int64_t r, int64_t k, int64_t kp) {
    int64_t blk = r >> 4, rr = r & 15;
    int64_t kk = k & 31;
    int64_t lane = ((kk >> 3) << 4) | rr;
    return ((((blk * (kp >> 5) + (k >> 5)) * 2) * 64 + bpos((int)lane)) << 3) + (kk & 7);
}

// The dense G^ stores use the same lane map but are K-major across row blocks,
// [k step][row block][lane], so the work groups of one mode, which advance through K at
// about the same rate, read neighbouring addresses at any moment.
__host__ __device__ inline int64_t frag_off_f64_km(int64_t r, int64_t k, int64_t mp) {
    int64_t blk = r >> 4, rr = r & 15;
    int64_t lane = ((k & 3) << 4) | rr;
    return ((((k >> 3) * (mp >> 4) + blk) * 64 + lane) << 1) + ((k >> 2) & 1);
}

// Symmetric 3x3 component index: xx yy zz xy xz yz
__host__ __device__ inline int sym_idx(int c, int d) {
    if (c == d) return c;
    int lo = c < d ? c : d, hi = c < d ? d : c;
    return (lo == 0) ? (hi == 1 ? 3 : 4) : 5;
}

// One work item of the per-mode complex product: a tile of 4*RB row blocks of one mode
// of one cell over one slice of K (the K split keeps enough work items to fill the chip
// evenly; the partial products of the slices are summed in fixed order by the inverse
// line transform).  Offsets are in elements of the respective arrays.
struct GemmJob {
    int64_t a_off;   // A store (dense forms) or table mode base (offset form)
    int64_t b_off;   // B fragments of this mode
    int64_t c_off;   // output [ct][mp][nm][16] doubles: this mode's record, K slice
    int32_t mb;      // row blocks of the mode (mp / 16)
    int32_t kp;      // padded K' (row stride of the fragment arrays)
    int32_t rb0;     // first row block of this tile
    int32_t ct;      // column tiles (8 RHS each)
    int32_t cell;    // cell index (offset form)
    // K' range [k0, k1) (dense forms) or interface columns [k0, k1) (offset forms); the
    // range is cyclic: indices at or beyond the padded K wrap to its start (windows around
    // the non-negligible blocks of a tile may straddle the end); k0 == k1: empty (zeros)
    int32_t k0, k1;
    int32_t ct_active;  // column tiles holding RHS of this cell (offset form skips the rest)
    int32_t crs;        // output row stride (doubles): the modes of a row are adjacent
    int32_t prec;       // offset forms: 1 = this job on FP32 MFMA (options.table_fp32), 0 = FP64
};

// Work lists of a persistent product launch: one list consumed by every work group (the
// jobs longest first), or one list per XCD (nl = 8: work group b takes jobs from list
// b mod 8 -- the XCD it runs on under round-robin dispatch -- and, once that list is
// exhausted, from the others in turn).  ctr: device counters, [l] the next job of list
// l, [8] the work groups that have left; all zero between launches.
struct PqLists {
    int* ctr;
    int nl;
    int start[9];      // list l holds the jobs [start[l], start[l + 1])
};

// Physical index of a step of a cyclic K range (idx < 2 n).
__host__ __device__ inline int wrap_k(int idx, int n) { return idx >= n ? idx - n : idx; }

// Per-cell device view used by the offset-table product kernel.
struct CellDev {
    const int32_t* cols_b;   // [n_b][2]
    const int32_t* cols_i;   // [n_i][2]
    int32_t n_b, n_i;
};

// Device-side status latch bits
enum { ST_NETFORCE = 1, ST_NONFINITE = 2 };

struct CellPlan {
    int nz, nm, n_i, n_b, R;
    int K, M;            // complex K = 3 n_i, rows M = 3 n_b
    int kp;              // padded real K' = roundup(6 n_i, 64)
    int mp;              // padded rows = roundup(3 n_b, 64 * RB), a whole work-group tile
    int ct;              // column tiles of the B / output layouts (same for every cell)
    int ctr;             // column tiles holding RHS of this cell = ceil(R / 8)
    int64_t f_off, u_off;        // offsets (doubles) into caller's f and u
    int64_t a_off;               // dense store offset (elements of the store type) of mode 0
    int64_t b_off;               // B fragments offset (elements) of mode 0
    int64_t c_off;               // GEMM output offset (doubles) of mode 0, K slice 0
    int64_t c_split;             // doubles per K slice of the GEMM output (nm*ct*mp*16)
    int64_t w_off;               // w scratch offset (doubles)
    int64_t t_off;               // f transpose scratch offset (doubles)
    int64_t red_off;             // reduction scratch offset (doubles)
    int rhs0;                    // first global RHS index
    int tw_n;                    // line length of the twiddle table used (== nz)
    int64_t tw_off;              // twiddle table offset (double2) for nz
    int32_t *cols_i_d, *cols_b_d;
    std::vector<int32_t> cols_i, cols_b;
    // Negligible-block windows: per (mode, row tile) the cyclic range of K chunks that
    // holds every block above the skip tolerance [win_start, win_start + win_len).
    int n_tiles = 0, n_chunks = 0;
    std::vector<int32_t> win_start, win_len;   // [nm][n_tiles]
    std::vector<uint8_t> mode_skips;           // [nm]: some chunk of this mode is skipped
    // Compact dense store: region r = m n_tiles + tl holds the win_len[r] chunk-tiles of
    // that window from chunk-tile reg_pre[r] on (cell-local); n_ct = reg_pre[nm n_tiles].
    std::vector<int64_t> reg_pre;
    int64_t n_ct = 0;
};
