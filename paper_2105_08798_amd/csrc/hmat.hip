// H-matrix form of the per-mode Green blocks (Appendix C): for every line mode m the
// complex matrix G^(m) (3 n_b x 3 n_i, its entries read from the FP64 offset table of a
// context -- they depend on the column offset n_b - n_i only, Section 3.2 -- so no dense
// store is needed) is split
// by the block partition of two cluster trees (binary space partitioning of the in-plane
// column positions, down to b_min columns; a block t x s is low rank when
// min(diam t, diam s) <= gamma dist(t, s), eq. geom_adm, on the clusters' bounding boxes,
// decided in exact integers), the
// admissible blocks are compressed by adaptive cross approximation with partial pivoting
// (eq. aca), and the H-matrix product y = H x replaces the dense product.  The line
// direction is diagonalised by the line transform, so the admissibility is evaluated in
// the plane (the periodic images s+ and s- share the in-plane position of s).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"
#include "plan.h"

#define NTH 256

static thread_local std::string g_herr;

static fbc_status hfail(fbc_status s, const std::string& m) {
    g_herr = m;
    return s;
}

// ---------------------------------------------------------------------------------------
// Host planning: cluster trees and block partition (geometry only, exact integers)
// ---------------------------------------------------------------------------------------
using HNode = PlanNode;
using HPart = PlanBlock;

// Device block description.
struct HBlk {
    int kind;            // 1 low rank, 0 dense
    int t_off, nt;       // pad columns: tcols[t_off .. t_off + nt)
    int s_off, ns;       // interface columns: scols[s_off .. s_off + ns)
    int cap;             // rank capacity (low rank)
    int64_t u_off, v_off;   // factor offsets within a mode (double2)
    int lr;              // index among the low-rank blocks (T workspace)
    int64_t d_off;       // dense leaves: offset of the entries within a mode (double2)
};

// Entries of G^(m): the offset table [mode][offset][6] of a one-cell FP64 offset-table
// context, through its lookup over the bounding box of the column offsets.
struct HStore {
    const double2* tab;
    const int32_t* lut;
    const int32_t* cols_b;   // [n_b][2]
    const int32_t* cols_i;   // [n_i][2]
    int64_t n_off;
    int d1min, d2min, w2;
};

__device__ inline double2 entry(const HStore& st, int m, int row, int col) {
    const int b = row / 3, c = row - 3 * b, i = col / 3, d = col - 3 * i;
    const int x = st.cols_b[2 * b] - st.cols_i[2 * i] - st.d1min;
    const int y = st.cols_b[2 * b + 1] - st.cols_i[2 * i + 1] - st.d2min;
    const int64_t o = st.lut[(int64_t)x * st.w2 + y];
    return st.tab[((int64_t)m * st.n_off + o) * 6 + sym_idx(c, d)];
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Operands of the product: either the plain layouts of fbc_hmat_apply (x [mode][3 n_i][R],
// y [mode][3 n_b][R], complex) or, inside a context's apply pipeline, the context's own
// ones: x read from the forward transform's FP64 B fragments (RHS r = 8 tile + j: column
// 16 tile + j holds Re f^ at K' = 2k, column 16 tile + j + 8 holds Im f^ there) and y
// written as the product records the inverse transform reads ([tile][row][mode][16]:
// Re of the tile's 8 RHS, then Im), every RHS slot of the tiles written (zeros past R).
struct HIo {
    const double2* x;      // plain input (NULL: fragments)
    double2* y;            // plain output (NULL: records)
    const double* bf;      // fragments of mode 0; mode m at + m * bf_mode
    int64_t bf_mode;
    int kp;
    double* rec;           // records of the cell
    int mp, nm;
    int r_out;             // RHS slots written per row: R (plain) or 8 x tiles (records)
};

template <bool PIPE>
__device__ inline double2 xval(const HIo& io, int m, int col, int r, int n_i, int R) {
    return io.x[((int64_t)m * 3 * n_i + col) * R + r];
}

// The pipeline's input in the plain layout x [mode][3 n_i][R] (one pass over the
// fragments; the products then read x with unit stride over the right-hand sides).
__global__ void __launch_bounds__(NTH) k_hmat_x(HIo io, int n_i, int R, double2* __restrict__ x) {
    const int m = blockIdx.y;
    const double* b = io.bf + (int64_t)m * io.bf_mode;
    for (int e = blockIdx.x * NTH + threadIdx.x; e < 3 * n_i * R; e += gridDim.x * NTH) {
        const int col = e / R, r = e - col * R;
        const int tile = r >> 3, j = r & 7;
        x[(int64_t)m * 3 * n_i * R + e] = make_double2(b[frag_off_f64(16 * tile + j, 2 * col, io.kp)],
                                                       b[frag_off_f64(16 * tile + j + 8, 2 * col, io.kp)]);
    }
}

template <bool PIPE>
__device__ inline void yput(const HIo& io, int m, int row, int r, int n_b, int R, double2 v) {
    if constexpr (!PIPE) {
        io.y[((int64_t)m * 3 * n_b + row) * R + r] = v;
    } else {
        double* rec = io.rec + (((int64_t)(r >> 3) * io.mp + row) * io.nm + m) * 16;
        rec[r & 7] = v.x;
        rec[8 + (r & 7)] = v.y;
    }
}

// Fixed-order reductions over the work group.
__device__ inline double block_sum_d(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = NTH / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// argmax with the smallest index among equal values; val < 0 marks "none".
__device__ inline void block_argmax(double& val, int& idx, double* redv, int* redi) {
    redv[threadIdx.x] = val;
    redi[threadIdx.x] = idx;
    __syncthreads();
    for (int s = NTH / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double v2 = redv[threadIdx.x + s];
            const int i2 = redi[threadIdx.x + s];
            if (v2 > redv[threadIdx.x] || (v2 == redv[threadIdx.x] && i2 < redi[threadIdx.x] && v2 >= 0)) {
                redv[threadIdx.x] = v2;
                redi[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    val = redv[0];
    idx = redi[0];
    __syncthreads();
}

__device__ inline int gcol(const int32_t* __restrict__ cols, int off, int j) { return 3 * cols[off + j / 3] + j % 3; }

// Adaptive cross approximation of one (low-rank block, mode): one work group.
__global__ void __launch_bounds__(NTH) k_hmat_aca(const HBlk* __restrict__ blks, const int* __restrict__ lr_ids,
                                                  const int32_t* __restrict__ tcols,
                                                  const int32_t* __restrict__ scols, HStore st,
                                                  double eps, int max_rank, int64_t u_mode, int64_t v_mode,
                                                  double2* __restrict__ U, double2* __restrict__ V,
                                                  int* __restrict__ rank, int n_lr) {
    __shared__ double redv[NTH];
    __shared__ int redi[NTH];
    extern __shared__ unsigned char used[];
    const int li = blockIdx.x, m = blockIdx.y;
    const HBlk b = blks[lr_ids[li]];
    const int nr = 3 * b.nt, nc = 3 * b.ns;
    double2* Ub = U + (int64_t)m * u_mode + b.u_off;     // U[l * nr + r]
    double2* Vb = V + (int64_t)m * v_mode + b.v_off;     // V[l * nc + j]
    for (int r = threadIdx.x; r < nr; r += NTH) used[r] = 0;
    __syncthreads();
    int i = 0, k = 0, result = 0, small = 0;
    double norm2 = 0.0;
    for (;;) {
        if (k >= max_rank) {             // another term would exceed the rank bound
            result = -1;
            break;
        }
        // residual row i into V[k]
        double bestv = -1.0;
        int bestj = 0x7fffffff;
        double2* vk = Vb + (int64_t)k * nc;
        const int grow = gcol(tcols, b.t_off, i);
        for (int j = threadIdx.x; j < nc; j += NTH) {
            double2 a = entry(st, m, grow, gcol(scols, b.s_off, j));
            for (int l = 0; l < k; ++l) {
                const double2 p = cmul(Ub[(int64_t)l * nr + i], Vb[(int64_t)l * nc + j]);
                a.x -= p.x;
                a.y -= p.y;
            }
            vk[j] = a;
            const double mag = hypot(a.x, a.y);
            if (mag > bestv) { bestv = mag; bestj = j; }
        }
        if (threadIdx.x == 0) used[i] = 1;
        block_argmax(bestv, bestj, redv, redi);
        __syncthreads();
        if (bestv <= 0.0) {
            // vanishing residual row: the next unused row, or stop
            int cand = 0x7fffffff;
            for (int r = threadIdx.x; r < nr; r += NTH)
                if (!used[r]) { cand = r; break; }
            double cv = (cand == 0x7fffffff) ? -1.0 : 1.0;
            int ci = cand;
            block_argmax(cv, ci, redv, redi);
            if (cv < 0.0) break;
            i = ci;
            continue;
        }
        const double2 piv = vk[bestj];
        __syncthreads();
        const double den = piv.x * piv.x + piv.y * piv.y;
        const double2 pinv = make_double2(piv.x / den, -piv.y / den);
        double nv2 = 0.0;
        for (int j = threadIdx.x; j < nc; j += NTH) {
            const double2 v = cmul(vk[j], pinv);
            vk[j] = v;
            nv2 += v.x * v.x + v.y * v.y;
        }
        __syncthreads();
        // residual column bestj into U[k]
        double2* uk = Ub + (int64_t)k * nr;
        const int gc = gcol(scols, b.s_off, bestj);
        double nu2 = 0.0;
        for (int r = threadIdx.x; r < nr; r += NTH) {
            double2 a = entry(st, m, gcol(tcols, b.t_off, r), gc);
            for (int l = 0; l < k; ++l) {
                const double2 p = cmul(Vb[(int64_t)l * nc + bestj], Ub[(int64_t)l * nr + r]);
                a.x -= p.x;
                a.y -= p.y;
            }
            uk[r] = a;
            nu2 += a.x * a.x + a.y * a.y;
        }
        __syncthreads();
        nu2 = block_sum_d(nu2, redv);
        nv2 = block_sum_d(nv2, redv);
        // cross terms 2 Re sum_l (u_l^H u_k)(v_l^H v_k)
        double cross = 0.0;
        for (int l = 0; l < k; ++l) {
            double ur = 0, ui = 0, vr = 0, vi = 0;
            for (int r = threadIdx.x; r < nr; r += NTH) {
                const double2 a = Ub[(int64_t)l * nr + r], c = uk[r];
                ur += a.x * c.x + a.y * c.y;
                ui += a.x * c.y - a.y * c.x;
            }
            for (int j = threadIdx.x; j < nc; j += NTH) {
                const double2 a = Vb[(int64_t)l * nc + j], c = vk[j];
                vr += a.x * c.x + a.y * c.y;
                vi += a.x * c.y - a.y * c.x;
            }
            ur = block_sum_d(ur, redv);
            ui = block_sum_d(ui, redv);
            vr = block_sum_d(vr, redv);
            vi = block_sum_d(vi, redv);
            cross += 2.0 * (ur * vr - ui * vi);
        }
        norm2 = norm2 + cross + nu2 * nv2;
        ++k;
        // stop after two consecutive terms below the bound (one small term can come from
        // a row that misses the block's large entries)
        small = (sqrt(nu2 * nv2) <= eps * sqrt(fmax(norm2, 0.0))) ? small + 1 : 0;
        if (small == 2) break;
        // next pivot row: the unused row of largest |u_k|
        double bu = -1.0;
        int bi = 0x7fffffff;
        for (int r = threadIdx.x; r < nr; r += NTH) {
            if (used[r]) continue;
            const double mag = hypot(uk[r].x, uk[r].y);
            if (mag > bu) { bu = mag; bi = r; }
        }
        block_argmax(bu, bi, redv, redi);
        if (bu < 0.0) break;
        i = bi;
    }
    if (threadIdx.x == 0) rank[(int64_t)m * n_lr + li] = (result < 0) ? -1 : k;
}

// T[lr][l][r] = sum_j V[l][j] x[col_j][r] for the low-rank blocks, Rp columns per l (the
// columns from R on zero, so the y kernel runs whole groups of HR right-hand sides).
template <bool PIPE>
__global__ void __launch_bounds__(NTH) k_hmat_vt(const HBlk* __restrict__ blks, const int* __restrict__ lr_ids,
                                                 const int32_t* __restrict__ scols, const double2* __restrict__ V,
                                                 int64_t v_mode, const int* __restrict__ rank, int n_lr,
                                                 int max_rank, HIo io, int n_i, int R, int Rp,
                                                 double2* __restrict__ T) {
    const int li = blockIdx.x, m = blockIdx.y;
    const int k = rank[(int64_t)m * n_lr + li];
    if (k <= 0) return;
    const HBlk b = blks[lr_ids[li]];
    const int nc = 3 * b.ns;
    const double2* Vb = V + (int64_t)m * v_mode + b.v_off;
    double2* Tb = T + ((int64_t)m * n_lr + li) * max_rank * Rp;
    for (int e = threadIdx.x; e < k * Rp; e += NTH) {
        const int l = e / Rp, r = e - l * Rp;
        double2 acc = make_double2(0, 0);
        if (r < R)
            for (int j = 0; j < nc; ++j) {
                const double2 p = cmul(Vb[(int64_t)l * nc + j], xval<PIPE>(io, m, gcol(scols, b.s_off, j), r, n_i, R));
                acc.x += p.x;
                acc.y += p.y;
            }
        Tb[(int64_t)l * Rp + r] = acc;
    }
}

struct HContrib {
    int blk;           // block index
    int row0;          // first row of this leaf within the block's rows
};

// Entries of the dense leaves, per mode, column-major per block (entry (row i, column j)
// at d_off + j * 3 nt + i), so that the rows of a leaf read consecutive addresses.
__global__ void __launch_bounds__(NTH) k_hmat_dense(const HBlk* __restrict__ blks, const int* __restrict__ d_ids,
                                                    const int32_t* __restrict__ tcols,
                                                    const int32_t* __restrict__ scols, HStore st,
                                                    double2* __restrict__ D, int64_t d_mode) {
    const HBlk b = blks[d_ids[blockIdx.x]];
    const int m = blockIdx.y;
    const int nr = 3 * b.nt, n = nr * 3 * b.ns;
    double2* Db = D + (int64_t)m * d_mode + b.d_off;
    for (int e = threadIdx.x; e < n; e += NTH) {
        const int j = e / nr, i = e - j * nr;
        Db[e] = entry(st, m, gcol(tcols, b.t_off, i), gcol(scols, b.s_off, j));
    }
}

// y rows of one pad leaf: sum over the blocks that cover it (low rank: U rows times T;
// dense leaves: their stored entries times x; low-rank blocks over the rank bound: the
// offset table's entries times x).  One wave per (leaf, mode), four modes per work group;
// a lane owns one row of the leaf (rows past 64 in further passes) and HR right-hand sides
// at a time, so each factor or stored entry is read once per HR of them, and the lanes
// read consecutive rows of U and of the dense entries.  The RHS slots from R to
// io.r_out are written as zeros.
#define HR 8
template <bool PIPE>
__global__ void __launch_bounds__(NTH) k_hmat_y(const HBlk* __restrict__ blks, const int32_t* __restrict__ scols,
                                                const int32_t* __restrict__ leaf_cols,
                                                const int* __restrict__ leaf_off,
                                                const HContrib* __restrict__ contrib,
                                                const int* __restrict__ contrib_off, HStore st,
                                                const double2* __restrict__ U, int64_t u_mode,
                                                const double2* __restrict__ D, int64_t d_mode,
                                                const double2* __restrict__ T, const int* __restrict__ rank,
                                                int n_lr, int max_rank, HIo io, int n_i,
                                                int n_b, int R, int Rp, int nm) {
    const int leaf = blockIdx.x, lane = threadIdx.x & 63;
    const int m = __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (threadIdx.x >> 6));
    if (m >= nm) return;
    const int c0 = leaf_off[leaf], nrow = 3 * (leaf_off[leaf + 1] - c0);
    for (int rl = lane; rl - lane < nrow; rl += 64) {          // every lane runs every pass
        const bool live = rl < nrow;
        const int grow = live ? 3 * leaf_cols[c0 + rl / 3] + rl % 3 : 0;
        for (int r0 = 0; r0 < io.r_out; r0 += HR) {
            const int nr_here = min(HR, R - r0);                  // <= 0: zero slots only
            double2 acc[HR];
#pragma unroll
            for (int q = 0; q < HR; ++q) acc[q] = make_double2(0, 0);
            for (int q2 = contrib_off[leaf]; q2 < contrib_off[leaf + 1] && nr_here > 0 && live; ++q2) {
                const HContrib cb = contrib[q2];
                const HBlk b = blks[cb.blk];
                const int br = cb.row0 + rl;                 // row within the block
                const int nr = 3 * b.nt;
                const int k = (b.kind == 1) ? rank[(int64_t)m * n_lr + b.lr] : -1;
                if (k >= 0) {
                    // T holds Rp >= r0 + HR columns, zeros past R: no per-RHS test
                    const double2* Ub = U + (int64_t)m * u_mode + b.u_off + br;
                    const double2* Tb = T + ((int64_t)m * n_lr + b.lr) * max_rank * Rp + r0;
                    for (int l = 0; l < k; ++l) {
                        const double2 u = Ub[(int64_t)l * nr];
#pragma unroll
                        for (int q = 0; q < HR; ++q) {
                            const double2 t = Tb[(int64_t)l * Rp + q];
                            acc[q].x += u.x * t.x - u.y * t.y;
                            acc[q].y += u.x * t.y + u.y * t.x;
                        }
                    }
                } else {
                    const double2* Db = (b.kind == 0) ? D + (int64_t)m * d_mode + b.d_off + br : nullptr;
                    if (nr_here == HR) {
                        for (int j = 0; j < 3 * b.ns; ++j) {
                            const int gc = gcol(scols, b.s_off, j);
                            const double2 a = Db ? Db[(int64_t)j * nr] : entry(st, m, grow, gc);
#pragma unroll
                            for (int q = 0; q < HR; ++q) {
                                const double2 x = xval<PIPE>(io, m, gc, r0 + q, n_i, R);
                                acc[q].x += a.x * x.x - a.y * x.y;
                                acc[q].y += a.x * x.y + a.y * x.x;
                            }
                        }
                    } else {
                        for (int j = 0; j < 3 * b.ns; ++j) {
                            const int gc = gcol(scols, b.s_off, j);
                            const double2 a = Db ? Db[(int64_t)j * nr] : entry(st, m, grow, gc);
                            for (int q = 0; q < nr_here; ++q) {
                                const double2 x = xval<PIPE>(io, m, gc, r0 + q, n_i, R);
                                acc[q].x += a.x * x.x - a.y * x.y;
                                acc[q].y += a.x * x.y + a.y * x.x;
                            }
                        }
                    }
                }
            }
            if (live) {
#pragma unroll
                for (int q = 0; q < HR; ++q)
                    if (r0 + q < io.r_out) yput<PIPE>(io, m, grow, r0 + q, n_b, R, acc[q]);
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------
struct fbc_hmat {
    const fbc_ctx* ctx = nullptr;
    int nm = 0, n_i = 0, n_b = 0, R = 0, max_rank = 0;
    int n_lr = 0, n_dense = 0, n_leaves = 0;
    int64_t u_mode = 0, v_mode = 0;
    HStore st{};
    std::vector<HBlk> blk;
    std::vector<int32_t> part_stream;     // kind, nt, ns, t cols, s cols per block
    std::vector<int> rank_h;              // [nm][n_lr]
    std::vector<void*> allocs;
    HBlk* blk_d = nullptr;
    int* lr_ids = nullptr;
    int* d_ids_d = nullptr;
    int32_t *tcols = nullptr, *scols = nullptr, *leaf_cols = nullptr;
    int *leaf_off = nullptr, *contrib_off = nullptr;
    HContrib* contrib = nullptr;
    double2 *U = nullptr, *V = nullptr, *T = nullptr, *D = nullptr;
    double2* xbuf = nullptr;              // pipeline input in the plain layout
    int64_t d_mode = 0;
    int* rank = nullptr;
    double stored = 0, dense_total = 0;
    int max_rank_used = 0, n_overflow = 0;
};

static void hmat_free(fbc_hmat* h) {
    if (!h) return;
    for (void* a : h->allocs) (void)hipFree(a);
    delete h;
}

template <class T>
static fbc_status halloc(fbc_hmat* h, T** p, int64_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, (size_t)std::max<int64_t>(bytes, 16));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return hfail(FBC_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + " B)");
    }
    h->allocs.push_back(*p);
    return FBC_OK;
}

extern "C" const char* fbc_hmat_last_error(void) { return g_herr.c_str(); }

extern "C" fbc_status fbc_hmat_create(const fbc_ctx* ctx, const fbc_hmat_opts* o, void* stream, fbc_hmat** out) {
    if (!out) return hfail(FBC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx || !o) return hfail(FBC_E_ARG, "context and options must not be NULL");
    if (ctx->opt.form != FBC_FORM_DTABLE_FP64 || ctx->cells.size() != 1)
        return hfail(FBC_E_UNSUPPORTED, "needs an FBC_FORM_DTABLE_FP64 context of one cell");
    if (o->b_min < 1 || o->gamma < 1 || o->gamma > 64 || !(o->eps > 0) || o->max_rank < 1 || o->max_rank > 512)
        return hfail(FBC_E_ARG, "need b_min >= 1, gamma in [1, 64], eps > 0, max_rank in [1, 512]");
    const CellPlan& p = ctx->cells[0];
    hipStream_t sm = (hipStream_t)stream;
    fbc_hmat* h = new (std::nothrow) fbc_hmat();
    if (!h) return hfail(FBC_E_NOMEM, "host allocation");
    h->ctx = ctx;
    h->nm = p.nm;
    h->n_i = p.n_i;
    h->n_b = p.n_b;
    h->R = p.R;
    h->max_rank = o->max_rank;
    h->st.tab = ctx->tab;
    h->st.lut = ctx->lut;
    h->st.cols_b = p.cols_b_d;
    h->st.cols_i = p.cols_i_d;
    h->st.n_off = ctx->n_offsets;
    h->st.d1min = ctx->d1min;
    h->st.d2min = ctx->d2min;
    h->st.w2 = ctx->w2;
    // Steps 1 and 2 on the host
    std::vector<HNode> tb, ti;
    std::vector<int> all_b(p.n_b), all_i(p.n_i);
    for (int c = 0; c < p.n_b; ++c) all_b[c] = c;
    for (int c = 0; c < p.n_i; ++c) all_i[c] = c;
    plan_tree(tb, p.cols_b, all_b, o->b_min);
    plan_tree(ti, p.cols_i, all_i, o->b_min);
    std::vector<HPart> part;
    plan_partition(tb, ti, 0, 0, o->gamma, part);
    std::vector<int32_t> tcols, scols;
    std::vector<int> lr_ids, d_ids;
    int64_t u_mode = 0, v_mode = 0, d_mode = 0;
    for (const HPart& q : part) {
        HBlk b{};
        b.kind = q.kind;
        b.t_off = (int)tcols.size();
        b.nt = (int)tb[q.t].idx.size();
        b.s_off = (int)scols.size();
        b.ns = (int)ti[q.s].idx.size();
        tcols.insert(tcols.end(), tb[q.t].idx.begin(), tb[q.t].idx.end());
        scols.insert(scols.end(), ti[q.s].idx.begin(), ti[q.s].idx.end());
        h->part_stream.push_back(q.kind);
        h->part_stream.push_back(b.nt);
        h->part_stream.push_back(b.ns);
        h->part_stream.insert(h->part_stream.end(), tb[q.t].idx.begin(), tb[q.t].idx.end());
        h->part_stream.insert(h->part_stream.end(), ti[q.s].idx.begin(), ti[q.s].idx.end());
        b.lr = -1;
        if (q.kind == 1) {
            b.cap = o->max_rank;
            b.u_off = u_mode;
            b.v_off = v_mode;
            u_mode += (int64_t)3 * b.nt * b.cap;
            v_mode += (int64_t)3 * b.ns * b.cap;
            b.lr = (int)lr_ids.size();
            lr_ids.push_back((int)h->blk.size());
        } else {
            b.d_off = d_mode;
            d_mode += (int64_t)9 * b.nt * b.ns;
            d_ids.push_back((int)h->blk.size());
        }
        h->blk.push_back(b);
    }
    h->n_lr = (int)lr_ids.size();
    h->n_dense = (int)h->blk.size() - h->n_lr;
    h->u_mode = u_mode;
    h->v_mode = v_mode;
    h->d_mode = d_mode;
    // pad leaves and the blocks covering them: a leaf's columns are a contiguous run of the
    // columns of every ancestor, in tree order
    std::vector<int> leaf_node;
    for (int n = 0; n < (int)tb.size(); ++n)
        if (tb[n].child[0] < 0) leaf_node.push_back(n);
    h->n_leaves = (int)leaf_node.size();
    std::vector<int32_t> leaf_cols;
    std::vector<int> leaf_off(1, 0);
    std::vector<int> pos_in_tree(p.n_b);           // position of a column in the root's order
    for (size_t k = 0; k < tb[0].idx.size(); ++k) pos_in_tree[tb[0].idx[k]] = (int)k;
    for (int n : leaf_node) {
        leaf_cols.insert(leaf_cols.end(), tb[n].idx.begin(), tb[n].idx.end());
        leaf_off.push_back((int)leaf_cols.size());
    }
    std::vector<HContrib> contrib;
    std::vector<int> contrib_off(1, 0);
    for (int L = 0; L < h->n_leaves; ++L) {
        const int first = pos_in_tree[tb[leaf_node[L]].idx[0]];
        for (int bi = 0; bi < (int)h->blk.size(); ++bi) {
            const HBlk& b = h->blk[bi];
            const int tfirst = pos_in_tree[tcols[b.t_off]];
            if (first >= tfirst && first < tfirst + b.nt) contrib.push_back({bi, 3 * (first - tfirst)});
        }
        contrib_off.push_back((int)contrib.size());
    }
    // device data
    fbc_status s;
    // T workspace: the right-hand sides padded to whole groups of HR (zeros)
    const int64_t t_elems = (int64_t)p.nm * std::max(h->n_lr, 1) * o->max_rank * (HR * ((p.R + HR - 1) / HR));
    if ((s = halloc(h, &h->blk_d, (int64_t)h->blk.size() * sizeof(HBlk))) != FBC_OK ||
        (s = halloc(h, &h->lr_ids, (int64_t)lr_ids.size() * 4)) != FBC_OK ||
        (s = halloc(h, &h->tcols, (int64_t)tcols.size() * 4)) != FBC_OK ||
        (s = halloc(h, &h->scols, (int64_t)scols.size() * 4)) != FBC_OK ||
        (s = halloc(h, &h->leaf_cols, (int64_t)leaf_cols.size() * 4)) != FBC_OK ||
        (s = halloc(h, &h->leaf_off, (int64_t)leaf_off.size() * 4)) != FBC_OK ||
        (s = halloc(h, &h->contrib, (int64_t)contrib.size() * sizeof(HContrib))) != FBC_OK ||
        (s = halloc(h, &h->contrib_off, (int64_t)contrib_off.size() * 4)) != FBC_OK ||
        (s = halloc(h, &h->U, (int64_t)p.nm * u_mode * 16)) != FBC_OK ||
        (s = halloc(h, &h->V, (int64_t)p.nm * v_mode * 16)) != FBC_OK ||
        (s = halloc(h, &h->T, t_elems * 16)) != FBC_OK ||
        (s = halloc(h, &h->xbuf, (int64_t)p.nm * 3 * p.n_i * p.R * 16)) != FBC_OK ||
        (s = halloc(h, &h->D, (int64_t)p.nm * d_mode * 16)) != FBC_OK ||
        (s = halloc(h, &h->d_ids_d, (int64_t)d_ids.size() * 4)) != FBC_OK ||
        (s = halloc(h, &h->rank, (int64_t)p.nm * std::max(h->n_lr, 1) * 4)) != FBC_OK) {
        hmat_free(h);
        return s;
    }
    hipError_t e = hipSuccess;
    auto up = [&](void* d, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, sm);
    };
    up(h->blk_d, h->blk.data(), h->blk.size() * sizeof(HBlk));
    up(h->lr_ids, lr_ids.data(), lr_ids.size() * 4);
    up(h->d_ids_d, d_ids.data(), d_ids.size() * 4);
    up(h->tcols, tcols.data(), tcols.size() * 4);
    up(h->scols, scols.data(), scols.size() * 4);
    up(h->leaf_cols, leaf_cols.data(), leaf_cols.size() * 4);
    up(h->leaf_off, leaf_off.data(), leaf_off.size() * 4);
    up(h->contrib, contrib.data(), contrib.size() * sizeof(HContrib));
    up(h->contrib_off, contrib_off.data(), contrib_off.size() * 4);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(sm);
        hmat_free(h);
        return hfail(FBC_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    // the dense leaves' entries, then step 3 on the device
    if (!d_ids.empty())
        hipLaunchKernelGGL(k_hmat_dense, dim3((unsigned)d_ids.size(), p.nm), dim3(NTH), 0, sm, h->blk_d, h->d_ids_d,
                           h->tcols, h->scols, h->st, h->D, d_mode);
    if (h->n_lr > 0) {
        int max_rows = 1;
        for (int li : lr_ids) max_rows = std::max(max_rows, 3 * h->blk[li].nt);
        hipLaunchKernelGGL(k_hmat_aca, dim3(h->n_lr, p.nm), dim3(NTH), (size_t)max_rows, sm, h->blk_d, h->lr_ids,
                           h->tcols, h->scols, h->st, o->eps, o->max_rank, u_mode, v_mode, h->U, h->V, h->rank,
                           h->n_lr);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    if (e == hipSuccess && h->n_lr > 0) {
        h->rank_h.resize((size_t)p.nm * h->n_lr);
        e = hipMemcpy(h->rank_h.data(), h->rank, h->rank_h.size() * 4, hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) {
        hmat_free(h);
        return hfail(FBC_E_DEVICE, std::string("cross approximation: ") + hipGetErrorString(e));
    }
    for (int m = 0; m < p.nm; ++m)
        for (const HBlk& b : h->blk) {
            const double dense = 9.0 * b.nt * b.ns;
            h->dense_total += dense;
            if (b.kind == 1) {
                const int k = h->rank_h[(size_t)m * h->n_lr + b.lr];
                if (k < 0) {
                    ++h->n_overflow;
                    h->stored += dense;
                } else {
                    h->stored += (double)k * 3.0 * (b.nt + b.ns);
                    h->max_rank_used = std::max(h->max_rank_used, k);
                }
            } else {
                h->stored += dense;
            }
        }
    *out = h;
    return FBC_OK;
}

extern "C" void fbc_hmat_destroy(fbc_hmat* h) {
    // an object attached to its context is detached first (the context's applies then
    // go back to the offset-table product)
    if (h && h->ctx && h->ctx->hmat == h) (void)fbc_set_hmat(const_cast<fbc_ctx*>(h->ctx), nullptr, nullptr);
    hmat_free(h);
}

extern "C" fbc_status fbc_hmat_get_info(const fbc_hmat* h, fbc_hmat_info* info) {
    if (!h || !info) return hfail(FBC_E_ARG, "null argument");
    info->n_blocks = (int)h->blk.size();
    info->n_low_rank = h->n_lr;
    info->n_dense = h->n_dense;
    info->max_rank_used = h->max_rank_used;
    info->n_over_rank = h->n_overflow;
    info->stored_entries = h->stored;
    info->dense_entries = h->dense_total;
    return FBC_OK;
}

extern "C" fbc_status fbc_hmat_partition(const fbc_hmat* h, int32_t* out, int64_t cap, int64_t* n_out) {
    if (!h || !n_out) return hfail(FBC_E_ARG, "null argument");
    *n_out = (int64_t)h->part_stream.size();
    if (out) {
        if (cap < *n_out) return hfail(FBC_E_ARG, "out too small");
        std::memcpy(out, h->part_stream.data(), h->part_stream.size() * 4);
    }
    return FBC_OK;
}

extern "C" fbc_status fbc_hmat_ranks(const fbc_hmat* h, int32_t* out) {
    if (!h || !out) return hfail(FBC_E_ARG, "null argument");
    if (!h->rank_h.empty()) std::memcpy(out, h->rank_h.data(), h->rank_h.size() * 4);
    return FBC_OK;
}

template <bool PIPE>
static void hmat_launch_t(fbc_hmat* h, const HIo& io, hipStream_t sm) {
    const int Rp = HR * ((h->R + HR - 1) / HR);
    if (h->n_lr > 0)
        hipLaunchKernelGGL(k_hmat_vt<PIPE>, dim3(h->n_lr, h->nm), dim3(NTH), 0, sm, h->blk_d, h->lr_ids, h->scols,
                           h->V, h->v_mode, h->rank, h->n_lr, h->max_rank, io, h->n_i, h->R, Rp, h->T);
    hipLaunchKernelGGL(k_hmat_y<PIPE>, dim3(h->n_leaves, (h->nm + 3) / 4), dim3(NTH), 0, sm, h->blk_d, h->scols,
                       h->leaf_cols, h->leaf_off, h->contrib, h->contrib_off, h->st, h->U, h->u_mode, h->D,
                       h->d_mode, h->T, h->rank, h->n_lr, h->max_rank, io, h->n_i, h->n_b, h->R, Rp, h->nm);
}

static void hmat_launch(fbc_hmat* h, const HIo& io, hipStream_t sm) {
    if (io.x) {
        hmat_launch_t<false>(h, io, sm);
        return;
    }
    HIo pio = io;
    pio.x = h->xbuf;
    const int n = 3 * h->n_i * h->R;
    hipLaunchKernelGGL(k_hmat_x, dim3((unsigned)std::min(1024, (n + NTH - 1) / NTH), h->nm), dim3(NTH), 0, sm, io,
                       h->n_i, h->R, h->xbuf);
    hmat_launch_t<true>(h, pio, sm);
}

extern "C" fbc_status fbc_hmat_apply(fbc_hmat* h, const double* fhat, double* what, void* stream) {
    if (!h) return hfail(FBC_E_ARG, "object is NULL");
    if (!fhat || !what) return hfail(FBC_E_ARG, "fhat and what must be device pointers");
    HIo io{};
    io.x = (const double2*)fhat;
    io.y = (double2*)what;
    io.r_out = h->R;
    hmat_launch(h, io, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hfail(FBC_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return FBC_OK;
}

// The product step of a context's apply pipeline (fbc_set_hmat): B fragments in, product
// records out (one K slice).
void hmat_enqueue_pipeline(fbc_hmat* h, const double* bfrag, int64_t bf_mode, int kp, double* rec, int mp, int nm,
                           int ct, hipStream_t st) {
    HIo io{};
    io.bf = bfrag;
    io.bf_mode = bf_mode;
    io.kp = kp;
    io.rec = rec;
    io.mp = mp;
    io.nm = nm;
    io.r_out = 8 * ct;
    hmat_launch(h, io, st);
}

const fbc_ctx* hmat_context(const fbc_hmat* h) { return h->ctx; }
