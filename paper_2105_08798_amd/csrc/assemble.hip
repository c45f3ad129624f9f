// Device assembly of the line-mode Green blocks (Appendix B: inverse lattice Fourier
// transform of the inverted force-constant symbol, here a discrete Brillouin-zone sum
// over an M1 x M2 in-plane torus for every line mode m; Section 3.2: blocks depend only
// on the column offset, so one table over distinct offsets feeds every store form).
#include <algorithm>

#include "fft_lds.h"
#include "kernels.h"

// ----------------------------------------------------------------------------------
// D(theta)^{-1} for theta = (m/Nz, m1/M1, m2/M2).  Phases are exact integers modulo
// L = max(Nz, M1, M2) (all powers of two), and 1 - cos(2 pi p / L) is taken as
// 2 sin^2(pi p / L) from a host table, so there is no cancellation near q = 0.
// The six symmetric components are packed two per complex array for the 2-D inverse
// FFTs: (xx + i yy), (zz + i xy), (xz + i yz).  The q = 0 term is zero (pseudo-inverse).
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_dinv(double2* __restrict__ pk, int m0, int nmc, int nz,
                                              int m1, int m2, int logL,
                                              const double* __restrict__ sn, BondTable bt) {
    const int64_t plane = (int64_t)m1 * m2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= plane * nmc) return;
    const int mloc = (int)(idx / plane);
    const int64_t rem = idx - (int64_t)mloc * plane;
    const int i1 = (int)(rem / m2);
    const int i2 = (int)(rem - (int64_t)i1 * m2);
    const int m = m0 + mloc;
    const int L = 1 << logL;
    const int s0 = L / nz, s1 = L / m1, s2 = L / m2;
    double d[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < 12; ++b) {
        const int64_t ph = (int64_t)m * bt.n[b][0] * s0 + (int64_t)i1 * bt.n[b][1] * s1 +
                           (int64_t)i2 * bt.n[b][2] * s2;
        const double s = sn[ph & (L - 1)];
        const double w = 2.0 * s * s;
#pragma unroll
        for (int c = 0; c < 6; ++c) d[c] += w * bt.p[b][c];
    }
    double2 o0 = make_double2(0, 0), o1 = o0, o2 = o0;
    if (!((m % nz) == 0 && i1 == 0 && i2 == 0)) {
        const double a = d[0], bb = d[1], c = d[2], xy = d[3], xz = d[4], yz = d[5];
        const double cxx = bb * c - yz * yz;
        const double cyy = a * c - xz * xz;
        const double czz = a * bb - xy * xy;
        const double cxy = xz * yz - xy * c;
        const double cxz = xy * yz - bb * xz;
        const double cyz = xy * xz - a * yz;
        const double inv = 1.0 / (a * cxx + xy * cxy + xz * cxz);
        o0 = make_double2(cxx * inv, cyy * inv);
        o1 = make_double2(czz * inv, cxy * inv);
        o2 = make_double2(cxz * inv, cyz * inv);
    }
    double2* base = pk + (int64_t)mloc * 3 * plane + rem;
    base[0] = o0;
    base[plane] = o1;
    base[2 * plane] = o2;
}

void launch_dinv(hipStream_t st, double2* pk, int m0, int nmc, int nz, int m1, int m2, int logL,
                 const double* sn, const BondTable& bt) {
    const int64_t total = (int64_t)nmc * m1 * m2;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_dinv, dim3((unsigned)blocks), dim3(256), 0, st, pk, m0, nmc, nz, m1, m2,
                       logL, sn, bt);
}

// ----------------------------------------------------------------------------------
// In-place batched FFT of contiguous rows (length 2^logn) through LDS (64 KiB per block).
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fft_rows(double2* __restrict__ data, int64_t nrows,
                                                  int logn, const double2* __restrict__ tw,
                                                  int inverse, int nb) {
    extern __shared__ double2 lds[];
    const int n = 1 << logn;
    const int64_t row0 = (int64_t)blockIdx.x * nb;
    const int nbh = (int)((nrows - row0) < nb ? (nrows - row0) : nb);
    for (int t = threadIdx.x; t < nbh * n; t += blockDim.x) {
        const int r = t >> logn, j = t & (n - 1);
        lds[r * n + bitrev(j, logn)] = data[(row0 + r) * n + j];
    }
    __syncthreads();
    lds_fft(lds, nbh, logn, tw, inverse != 0);
    for (int t = threadIdx.x; t < nbh * n; t += blockDim.x) data[row0 * n + t] = lds[t];
}

void launch_fft_rows(hipStream_t st, double2* data, int64_t nrows, int logn, const double2* tw,
                     bool inverse) {
    const int n = 1 << logn;
    int nb = 4096 / n;
    if (nb < 1) nb = 1;
    const int64_t blocks = (nrows + nb - 1) / nb;
    hipLaunchKernelGGL(k_fft_rows, dim3((unsigned)blocks), dim3(256),
                       (size_t)nb * n * sizeof(double2), st, data, nrows, logn, tw,
                       inverse ? 1 : 0, nb);
}

// ----------------------------------------------------------------------------------
// Tiled transpose of complex matrices: in[b][rows][cols] -> out[b][cols][rows].
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_transpose_c(const double2* __restrict__ in,
                                                     double2* __restrict__ out, int rows,
                                                     int cols) {
    __shared__ double2 tile[32][33];
    const int b = blockIdx.z;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const double2* src = in + (int64_t)b * rows * cols;
    double2* dst = out + (int64_t)b * rows * cols;
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y, c = c0 + tx;
        if (r < rows && c < cols) tile[y][tx] = src[(int64_t)r * cols + c];
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int c = c0 + y, r = r0 + tx;
        if (r < rows && c < cols) dst[(int64_t)c * rows + r] = tile[tx][y];
    }
}

void launch_transpose_c(hipStream_t st, const double2* in, double2* out, int batches, int rows,
                        int cols) {
    dim3 grid((cols + 31) / 32, (rows + 31) / 32, batches);
    hipLaunchKernelGGL(k_transpose_c, grid, dim3(256), 0, st, in, out, rows, cols);
}

// ----------------------------------------------------------------------------------
// Unpack the three complex 2-D transforms into the six symmetric components at every
// distinct column offset.  After the transposed 2-D FFT the array index is
// t[comp][d2][d1].  For packed real inputs x + i y with transforms X, Y:
// X(d) = (Z(d) + conj Z(-d)) / 2,  Y(d) = (Z(d) - conj Z(-d)) / (2 i).
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gather_table(const double2* __restrict__ t,
                                                      double2* __restrict__ tab, int nmc, int m1,
                                                      int m2, int64_t n_off,
                                                      const int32_t* __restrict__ off_d1,
                                                      const int32_t* __restrict__ off_d2,
                                                      int64_t tab_mode_stride, double scale) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_off * nmc) return;
    const int mloc = (int)(idx / n_off);
    const int64_t o = idx - (int64_t)mloc * n_off;
    const int a1 = off_d1[o] & (m1 - 1), a2 = off_d2[o] & (m2 - 1);
    const int b1 = (-off_d1[o]) & (m1 - 1), b2 = (-off_d2[o]) & (m2 - 1);
    const int64_t plane = (int64_t)m1 * m2;
    const double2* base = t + (int64_t)mloc * 3 * plane;
    double2 outv[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double2 z = base[c * plane + (int64_t)a2 * m1 + a1];
        const double2 zn = base[c * plane + (int64_t)b2 * m1 + b1];
        const double2 x = make_double2(0.5 * (z.x + zn.x) * scale, 0.5 * (z.y - zn.y) * scale);
        const double2 y = make_double2(0.5 * (z.y + zn.y) * scale, 0.5 * (zn.x - z.x) * scale);
        // packing: c=0 -> (xx, yy), c=1 -> (zz, xy), c=2 -> (xz, yz)
        const int ix = (c == 0) ? 0 : (c == 1 ? 2 : 4);
        const int iy = (c == 0) ? 1 : (c == 1 ? 3 : 5);
        outv[ix] = x;
        outv[iy] = y;
    }
    double2* dst = tab + (int64_t)mloc * tab_mode_stride + o * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) dst[c] = outv[c];
}

void launch_gather_table(hipStream_t st, const double2* t, double2* tab, int nmc, int m1, int m2,
                         int64_t n_off, const int32_t* off_d1, const int32_t* off_d2,
                         int64_t tab_mode_stride, double scale) {
    const int64_t total = n_off * nmc;
    hipLaunchKernelGGL(k_gather_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, t,
                       tab, nmc, m1, m2, n_off, off_d1, off_d2, tab_mode_stride, scale);
}

__device__ inline int64_t lut_index(const int32_t* __restrict__ cols_b,
                                    const int32_t* __restrict__ cols_i, int b, int i,
                                    const int32_t* __restrict__ lut, int d1min, int d2min,
                                    int w2) {
    const int d1 = cols_b[2 * b] - cols_i[2 * i] - d1min;
    const int d2 = cols_b[2 * b + 1] - cols_i[2 * i + 1] - d2min;
    return lut[(int64_t)d1 * w2 + d2];
}

// Mean over interface columns of each block row, per mode (the row gauge of the
// reduced-precision forms).  One thread per (mode, pad column).
__global__ void __launch_bounds__(256) k_rowmean(const double2* __restrict__ tab,
                                                 double2* __restrict__ rowmean, int nm,
                                                 int mode_mult, int64_t n_off, int n_b, int n_i,
                                                 const int32_t* __restrict__ cols_b,
                                                 const int32_t* __restrict__ cols_i,
                                                 const int32_t* __restrict__ lut, int d1min,
                                                 int d2min, int w2) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nm * n_b) return;
    const int m = (int)(idx / n_b);
    const int b = (int)(idx - (int64_t)m * n_b);
    double2 acc[6];
    for (int c = 0; c < 6; ++c) acc[c] = make_double2(0, 0);
    const double2* tm = tab + (int64_t)m * mode_mult * n_off * 6;
    for (int i = 0; i < n_i; ++i) {
        const int64_t o = lut_index(cols_b, cols_i, b, i, lut, d1min, d2min, w2);
        for (int c = 0; c < 6; ++c) {
            const double2 v = tm[o * 6 + c];
            acc[c].x += v.x;
            acc[c].y += v.y;
        }
    }
    const double s = 1.0 / n_i;
    for (int c = 0; c < 6; ++c) rowmean[idx * 6 + c] = make_double2(acc[c].x * s, acc[c].y * s);
}

void launch_rowmean(hipStream_t st, const double2* tab, double2* rowmean, int nm, int mode_mult,
                    int64_t n_off, int n_b, int n_i, const int32_t* cols_b, const int32_t* cols_i,
                    const int32_t* lut, int d1min, int d2min, int w2) {
    const int64_t total = (int64_t)nm * n_b;
    hipLaunchKernelGGL(k_rowmean, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, tab,
                       rowmean, nm, mode_mult, n_off, n_b, n_i, cols_b, cols_i, lut, d1min, d2min,
                       w2);
}

// ----------------------------------------------------------------------------------
// Dense store in MFMA fragment order.  Real matrix A[row][k'] with row = 3b + c and
// k' = 2(3i + d) + part: A = Re G^ for part 0, Im G^ for part 1 (the complex product is
// applied as one real product against [Re f, -Im f ; Im f, Re f] columns).
// ----------------------------------------------------------------------------------
__device__ inline unsigned short f32_to_bf16_rne(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline double dense_value(int row, int kq, int m, int mode_mult,
                                     const double2* __restrict__ tab,
                                     const double2* __restrict__ rowmean, int64_t n_off, int n_b,
                                     int n_i, const int32_t* __restrict__ cols_b,
                                     const int32_t* __restrict__ cols_i,
                                     const int32_t* __restrict__ lut, int d1min, int d2min,
                                     int w2) {
    if (row >= 3 * n_b || kq >= 6 * n_i) return 0.0;
    const int b = row / 3, c = row - 3 * b;
    const int kc = kq >> 1, part = kq & 1;
    const int i = kc / 3, d = kc - 3 * i;
    const int s = sym_idx(c, d);
    const int64_t o = lut_index(cols_b, cols_i, b, i, lut, d1min, d2min, w2);
    double2 v = tab[((int64_t)m * mode_mult * n_off + o) * 6 + s];
    if (rowmean) {
        const double2 r = rowmean[((int64_t)m * n_b + b) * 6 + s];
        v.x -= r.x;
        v.y -= r.y;
    }
    return part ? v.y : v.x;
}

// Compact dense store of one cell: only the K chunks inside the negligible-block window
// of each (mode, row tile) are stored.  The store is a sequence of chunk-tiles (64 K' x
// tile_rows rows each) in (mode, tile, window position) order: region r = m n_tiles + tl
// holds win_len[r] chunk-tiles from reg_pre[r] on, the window position j holding the
// cyclic chunk (win_start[r] + j) mod n_chunks.  Inside a chunk-tile the MFMA fragment
// order of the product kernels, K-major across the tile's row blocks:
//   FP64  [8 steps of 8 k'][row block][lane][2]
//   FP32  [4 steps of 16 k'][row block][lane][4]
//   split [2 steps of 32 k'][row block][hi, lo][lane][8]
// One work group per chunk-tile.
__global__ void __launch_bounds__(256) k_build_dense(int form, void* __restrict__ store,
                                                     const double2* __restrict__ tab,
                                                     const double2* __restrict__ rowmean,
                                                     const int64_t* __restrict__ reg_pre,
                                                     const int32_t* __restrict__ win_start, int n_reg,
                                                     int n_tiles, int n_chunks, int tile_rows,
                                                     int64_t n_ct, int mode_mult, int64_t n_off, int n_b,
                                                     int n_i, const int32_t* __restrict__ cols_b,
                                                     const int32_t* __restrict__ cols_i,
                                                     const int32_t* __restrict__ lut, int d1min,
                                                     int d2min, int w2,
                                                     const unsigned long long* __restrict__ amax) {
    const int trb = tile_rows >> 4;               // row blocks of a tile
    const int64_t ce = (int64_t)tile_rows * 64;   // real entries of a chunk-tile
    for (int64_t g = blockIdx.x; g < n_ct; g += gridDim.x) {
        // region of chunk-tile g: the last r with reg_pre[r] <= g (regions may be empty)
        int lo = 0, hi = n_reg;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (reg_pre[mid] <= g) lo = mid; else hi = mid;
        }
        const int r = lo;
        const int m = r / n_tiles, tl = r - m * n_tiles;
        int ch = win_start[r] + (int)(g - reg_pre[r]);
        if (ch >= n_chunks) ch -= n_chunks;
        const int row0 = tl * tile_rows, k0 = 64 * ch;
        for (int64_t x = threadIdx.x; x < ce; x += blockDim.x) {
            if (form == FBC_FORM_FP64) {
                const int sub = (int)(x & 1), lane = (int)((x >> 1) & 63);
                const int rest = (int)(x >> 7);
                const int blk = rest % trb, st = rest / trb;
                const int row = row0 + 16 * blk + (lane & 15), kq = k0 + 8 * st + 4 * sub + (lane >> 4);
                ((double*)store)[g * ce + x] = dense_value(row, kq, m, mode_mult, tab, rowmean, n_off, n_b, n_i,
                                                           cols_b, cols_i, lut, d1min, d2min, w2);
            } else if (form == FBC_FORM_FP32) {
                const int sub = (int)(x & 3), lane = (int)((x >> 2) & 63);
                const int rest = (int)(x >> 8);
                const int blk = rest % trb, st = rest / trb;
                const int row = row0 + 16 * blk + (lane & 15), kq = k0 + 16 * st + 4 * sub + (lane >> 4);
                ((float*)store)[g * ce + x] = (float)dense_value(row, kq, m, mode_mult, tab, rowmean, n_off,
                                                                 n_b, n_i, cols_b, cols_i, lut, d1min, d2min, w2);
            } else {   // split: x indexes the hi parts; the lo part of a unit is 512 later
                const int j = (int)(x & 7), lane = (int)((x >> 3) & 63);
                const int rest = (int)(x >> 9);
                const int blk = rest % trb, st = rest / trb;
                const int row = row0 + 16 * blk + (lane & 15), kq = k0 + 32 * st + 8 * (lane >> 4) + j;
                const double v = dense_value(row, kq, m, mode_mult, tab, rowmean, n_off, n_b, n_i, cols_b,
                                             cols_i, lut, d1min, d2min, w2);
                unsigned short* out = (unsigned short*)store + g * 2 * ce;
                const int64_t base = ((((int64_t)st * trb + blk) * 2) * 64 + lane) * 8 + j;
                if (form == FBC_FORM_SPLIT_FP16) {   // scaled by 2^e(m)
                    const double vs = ldexp(v, split16_exp_a(amax[m]));
                    const _Float16 h = f64_to_f16(vs);
                    const _Float16 l = f64_to_f16(vs - (double)h);
                    out[base] = __builtin_bit_cast(unsigned short, h);
                    out[base + 512] = __builtin_bit_cast(unsigned short, l);
                } else {
                    const unsigned short h = f32_to_bf16_rne((float)v);
                    out[base] = h;
                    out[base + 512] = f32_to_bf16_rne((float)(v - (double)bf16_to_f32(h)));
                }
            }
        }
    }
}

// Largest magnitude of each table mode a cell reads (superset of its blocks), as the bit
// pattern of a non-negative double: amax[m] = max over offsets, components, re/im.
__global__ void __launch_bounds__(256) k_tab_absmax(const double2* __restrict__ tab, int mode_mult,
                                                    int64_t n_off, unsigned long long* __restrict__ amax) {
    __shared__ double red[256];
    const int m = blockIdx.y;
    const double2* tm = tab + (int64_t)m * mode_mult * n_off * 6;
    double mx = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_off * 6; e += (int64_t)gridDim.x * 256)
        mx = fmax(mx, fmax(fabs(tm[e].x), fabs(tm[e].y)));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(amax + m, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Per table mode t: the largest in-plane distance of an offset whose block reaches
// tau * amax[t] (bit pattern of a non-negative double, atomic max).  Blocks of offsets
// farther than that are below the tolerance in this mode.
__global__ void __launch_bounds__(256) k_tab_rhocut(const double2* __restrict__ tab, int64_t n_off,
                                                    const int32_t* __restrict__ d1,
                                                    const int32_t* __restrict__ d2, double tau,
                                                    const unsigned long long* __restrict__ amax,
                                                    unsigned long long* __restrict__ rhocut) {
    __shared__ double red[256];
    const int t = blockIdx.y;
    const double thr = tau * __longlong_as_double((long long)amax[t]);
    const double2* tm = tab + (int64_t)t * n_off * 6;
    double mx = 0.0;
    for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < n_off; o += (int64_t)gridDim.x * 256) {
        double g = 0.0;
        for (int c = 0; c < 6; ++c) g = fmax(g, fmax(fabs(tm[o * 6 + c].x), fabs(tm[o * 6 + c].y)));
        if (g >= thr) {
            const double x = 0.5 * d1[o], y = (d1[o] + 2.0 * d2[o]) * (0.5 * M_SQRT1_2);
            mx = fmax(mx, sqrt(x * x + y * y));
        }
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(rhocut + t, (unsigned long long)__double_as_longlong(red[0]));
}

void launch_tab_rhocut(hipStream_t st, const double2* tab, int T, int64_t n_off, const int32_t* d1,
                       const int32_t* d2, double tau, unsigned long long* amax,
                       unsigned long long* rhocut) {
    hipLaunchKernelGGL(k_zero_u64, dim3((T + 255) / 256), dim3(256), 0, st, amax, T);
    hipLaunchKernelGGL(k_zero_u64, dim3((T + 255) / 256), dim3(256), 0, st, rhocut, T);
    const int sl = (int)std::min<int64_t>(64, (n_off * 6 + 255) / 256);
    hipLaunchKernelGGL(k_tab_absmax, dim3(sl, T), dim3(256), 0, st, tab, 1, n_off, amax);
    const int sl2 = (int)std::min<int64_t>(64, (n_off + 255) / 256);
    hipLaunchKernelGGL(k_tab_rhocut, dim3(sl2, T), dim3(256), 0, st, tab, n_off, d1, d2, tau, amax, rhocut);
}



void launch_build_dense(hipStream_t st, int form, void* store, const double2* tab,
                        const double2* rowmean, const int64_t* reg_pre, const int32_t* win_start,
                        int nm, int n_tiles, int n_chunks, int tile_rows, int64_t n_ct, int mode_mult,
                        int64_t n_off, int n_b, int n_i, const int32_t* cols_b, const int32_t* cols_i,
                        const int32_t* lut, int d1min, int d2min, int w2, unsigned long long* amax) {
    if (form == FBC_FORM_SPLIT_FP16) {
        hipLaunchKernelGGL(k_zero_u64, dim3((nm + 255) / 256), dim3(256), 0, st, amax, nm);
        const int sl = (int)std::min<int64_t>(64, (n_off * 6 + 255) / 256);
        hipLaunchKernelGGL(k_tab_absmax, dim3(sl, nm), dim3(256), 0, st, tab, mode_mult, n_off, amax);
    }
    if (n_ct <= 0) return;
    const int64_t blocks = std::min<int64_t>(n_ct, 1 << 20);
    hipLaunchKernelGGL(k_build_dense, dim3((unsigned)blocks), dim3(256), 0, st, form, store, tab, rowmean,
                       reg_pre, win_start, nm * n_tiles, n_tiles, n_chunks, tile_rows, n_ct, mode_mult, n_off,
                       n_b, n_i, cols_b, cols_i, lut, d1min, d2min, w2, amax);
}
