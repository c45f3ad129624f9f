// Line transforms, update and reductions of the FBC pad update (Section 2.3.2,
// eq. flexbc.up=Gpipl*fipl with eq. mean(u^p)=0; Algorithm 1 lines 7-8), and the
// residual-based relaxation (Section 2.3.3, eq. alpha, Algorithm 2).
// All reductions use a fixed partition and a fixed-order tree, so results are bitwise
// reproducible from run to run (no floating-point atomics).
#include "fft_lds.h"
#include <algorithm>

#include "kernels.h"

#define NT 256

// Blocks of an elementwise grid-stride launch (a launch holds at most 2^32 work-items).
static inline int64_t grid_blocks(int64_t n) {
    const int64_t b = (n + NT - 1) / NT;
    return b < (1 << 20) ? (b > 0 ? b : 1) : (1 << 20);
}

// Block-wide sum of `nv` doubles per thread (in place in v), fixed order.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* red) {
    for (int c = 0; c < NV; ++c) red[c * NT + threadIdx.x] = v[c];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < NV; ++c) red[c * NT + threadIdx.x] += red[c * NT + threadIdx.x + s];
        __syncthreads();
    }
    for (int c = 0; c < NV; ++c) v[c] = red[c * NT];
    __syncthreads();
}
template <int NV>
__device__ inline void block_max(double (&v)[NV], double* red) {
    for (int c = 0; c < NV; ++c) red[c * NT + threadIdx.x] = v[c];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < NV; ++c)
                red[c * NT + threadIdx.x] = fmax(red[c * NT + threadIdx.x], red[c * NT + threadIdx.x + s]);
        __syncthreads();
    }
    for (int c = 0; c < NV; ++c) v[c] = red[c * NT];
    __syncthreads();
}

// Per-layer record of the force statistics: net force (3), absolute force (3), max |f|,
// non-finite flag.
#define NF_STRIDE 8

// ----------------------------------------------------------------------------------
// Net force per layer and component, and the finiteness check of the forces.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_netforce(const double* __restrict__ f,
                                                 double* __restrict__ sums, int nz, int n_i,
                                                 int check, int* __restrict__ status) {
    __shared__ double red[7 * NT];
    const int n0 = blockIdx.x, r = blockIdx.y;
    const double* row = f + ((int64_t)r * nz + n0) * n_i * 3;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    double mx[1] = {0.0};
    for (int i = threadIdx.x; i < n_i; i += NT) {
        for (int c = 0; c < 3; ++c) {
            const double x = row[3 * i + c];
            v[c] += x;
            v[3 + c] += fabs(x);
            mx[0] = fmax(mx[0], fabs(x));
            if (!isfinite(x)) v[6] = 1.0;
        }
    }
    block_sum<7>(v, red);
    block_max<1>(mx, red);
    if (threadIdx.x == 0) {
        double* o = sums + ((int64_t)r * nz + n0) * NF_STRIDE;
        for (int c = 0; c < 6; ++c) o[c] = v[c];
        o[6] = mx[0];
        o[7] = v[6];
        if (check && (v[6] != 0.0 || !isfinite(v[3] + v[4] + v[5]))) atomicOr(status, ST_NONFINITE);
    }
}

// Split-FP16 form: scale exponent of the force operand of a cell, from a bound on the
// transformed forces, |f^(m)| <= sum_n0 |f(n0)| <= Nz max|f| (twice that after the
// projection), so that the scaled values stay below 2^14.
__global__ void __launch_bounds__(NT) k_bexp(const double* __restrict__ sums, int n_layers, int nz,
                                             int* __restrict__ bexp) {
    __shared__ double red[NT];
    double mx[1] = {0.0};
    for (int e = threadIdx.x; e < n_layers; e += NT) mx[0] = fmax(mx[0], sums[(int64_t)e * NF_STRIDE + 6]);
    block_max<1>(mx, red);
    if (threadIdx.x == 0) {
        const double bound = 2.0 * nz * mx[0];
        *bexp = (bound > 0.0 && isfinite(bound)) ? 13 - ilogb(bound) : 0;
    }
}

// Net force of the whole cell per RHS and component (sum over layers in fixed order):
// tot[r][c].  Only this total enters the gauge (line mode 0); the check compares it with
// the total absolute force.
__global__ void __launch_bounds__(NT) k_netforce_total(const double* __restrict__ sums, int nz,
                                                       double tol, int check, int project,
                                                       double* __restrict__ tot,
                                                       int* __restrict__ status) {
    __shared__ double red[6 * NT];
    const int r = blockIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int n0 = threadIdx.x; n0 < nz; n0 += NT)
        for (int c = 0; c < 6; ++c) v[c] += sums[((int64_t)r * nz + n0) * NF_STRIDE + c];
    block_sum<6>(v, red);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) tot[r * 3 + c] = v[c];
        if (check && !project) {
            int bits = 0;
            for (int c = 0; c < 3; ++c)
                if (fabs(v[c]) > tol * v[3 + c]) bits |= ST_NETFORCE;
            if (bits) atomicOr(status, bits);
        }
    }
}

// Line transform of the per-layer net force (after the projection, if any):
// shat[r][m][c] = sum_n0 (s_c(n0) - tot_c / Nz) e^{-2 pi i m n0 / Nz}, m = 0..Nz/2.
// It multiplies the subtracted row means in the inverse transform.
__global__ void __launch_bounds__(NT) k_netforce_fft(const double* __restrict__ sums,
                                                     const double* __restrict__ tot, int project,
                                                     int nz, int logn,
                                                     const double2* __restrict__ tw,
                                                     double2* __restrict__ shat) {
    extern __shared__ double2 lds[];
    const int c = blockIdx.x, r = blockIdx.y;
    const double sub = project ? tot[r * 3 + c] / nz : 0.0;
    for (int n0 = threadIdx.x; n0 < nz; n0 += NT)
        lds[bitrev(n0, logn)] = make_double2(sums[((int64_t)r * nz + n0) * NF_STRIDE + c] - sub, 0.0);
    __syncthreads();
    lds_fft(lds, 1, logn, tw, false);
    const int nm = (nz >> 1) + 1;
    for (int m = threadIdx.x; m < nm; m += NT) {
        double2 z = lds[m];
        if (project && m == 0) z = make_double2(0.0, 0.0);
        shat[((int64_t)r * nm + m) * 3 + c] = z;
    }
}

void launch_netforce(hipStream_t st, const double* f, double* sums, double* tot, double2* shat, int R,
                     int nz, int n_i, double tol, int check, int project, const double2* tw,
                     int* bexp, int* status) {
    hipLaunchKernelGGL(k_netforce, dim3(nz, R), dim3(NT), 0, st, f, sums, nz, n_i, check, status);
    hipLaunchKernelGGL(k_netforce_total, dim3(R), dim3(NT), 0, st, sums, nz, tol, check, project, tot,
                       status);
    if (bexp) hipLaunchKernelGGL(k_bexp, dim3(1), dim3(NT), 0, st, sums, R * nz, nz, bexp);
    if (shat) {
        int logn = 0;
        while ((1 << logn) < nz) ++logn;
        hipLaunchKernelGGL(k_netforce_fft, dim3(3, R), dim3(NT), (size_t)nz * sizeof(double2), st, sums,
                           tot, project, nz, logn, tw, shat);
    }
}

// ----------------------------------------------------------------------------------
// rFFT along the line for every (RHS, column component), written straight into the
// GEMM B operand in MFMA fragment order.  Two real columns are packed into one complex
// sequence; F_a(m) = (Z(m) + conj Z(-m))/2, F_b(m) = (Z(m) - conj Z(-m))/(2i).
// B columns per 8-RHS tile: n = 16 ct + j carries (Re f, -Im f) against A's (Re, Im)
// rows -> real part of the product; n + 8 carries (Im f, Re f) -> imaginary part.
// ----------------------------------------------------------------------------------
__device__ inline unsigned short f2bf(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

template <int FORM>
__device__ inline void put_b(void* bm, int n, int kq, int kp, double v) {
    if (FORM == FBC_FORM_FP64 || FORM == FBC_FORM_DTABLE_FP64) {
        ((double*)bm)[frag_off_f64(n, kq, kp)] = v;
    } else if (FORM == FBC_FORM_FP32) {
        ((float*)bm)[frag_off_f32(n, kq, kp)] = (float)v;
    } else if (FORM == FBC_FORM_SPLIT_FP16) {        // v already scaled by 2^e
        const _Float16 hi = (_Float16)(float)v;
        const _Float16 lo = (_Float16)(float)(v - (double)(float)hi);
        unsigned short* p = (unsigned short*)bm + frag_off_bf16(n, kq, kp);
        p[0] = __builtin_bit_cast(unsigned short, hi);
        p[512] = __builtin_bit_cast(unsigned short, lo);
    } else {
        const unsigned short hi = f2bf((float)v);
        const unsigned short lo = f2bf((float)(v - (double)bf2f(hi)));
        unsigned short* p = (unsigned short*)bm + frag_off_bf16(n, kq, kp);
        p[0] = hi;
        p[512] = lo;
    }
}

// Whole 16-byte fragment units of one B column n for the 2G consecutive K' entries
// kq0 .. kq0 + 2G - 1 (kq0 a multiple of 2G): FP64 units hold (kq, kq + 4), FP32 units
// (kq, kq + 4, kq + 8, kq + 12), split units 8 consecutive kq (hi run, lo run 1 KiB on).
template <int FORM, int NV>
__device__ inline void put_b_units(void* bm, int n, int kq0, int kp, const double (&v)[NV]) {
    if constexpr (FORM == FBC_FORM_FP64 || FORM == FBC_FORM_DTABLE_FP64) {
        static_assert(NV == 8, "FP64 units cover 8 K' entries");
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *(double2*)((double*)bm + frag_off_f64(n, kq0 + j, kp)) = make_double2(v[j], v[j + 4]);
    } else if constexpr (FORM == FBC_FORM_FP32) {
        static_assert(NV == 16, "FP32 units cover 16 K' entries");
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *(float4*)((float*)bm + frag_off_f32(n, kq0 + j, kp)) =
                make_float4((float)v[j], (float)v[j + 4], (float)v[j + 8], (float)v[j + 12]);
    } else {
        static_assert(NV == 8, "split units cover 8 K' entries");
        us8_t hi, lo;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if constexpr (FORM == FBC_FORM_SPLIT_FP16) {
                const _Float16 h = (_Float16)(float)v[j];
                hi[j] = __builtin_bit_cast(unsigned short, h);
                lo[j] = __builtin_bit_cast(unsigned short, (_Float16)(float)(v[j] - (double)(float)h));
            } else {
                const unsigned short h = f2bf((float)v[j]);
                hi[j] = h;
                lo[j] = f2bf((float)(v[j] - (double)bf2f(h)));
            }
        }
        unsigned short* p = (unsigned short*)bm + frag_off_bf16(n, kq0, kp);
        *(us8_t*)p = hi;
        *(us8_t*)(p + 512) = lo;
    }
}

template <int FORM>
__global__ void __launch_bounds__(NT) k_line_rfft(const double* __restrict__ f,
                                                  const double* __restrict__ tot, int project,
                                                  void* __restrict__ bfrag, int nz, int logn,
                                                  int n_i, int kp, int ct, int tc,
                                                  const double2* __restrict__ tw, double inv_cnt,
                                                  const int* __restrict__ bexp) {
    extern __shared__ double2 lds[];
    const int esc = (FORM == FBC_FORM_SPLIT_FP16) ? *bexp : 0;   // power-of-two operand scale
    // RHS fastest across blocks: the 8 RHS of a column tile, whose B fragments share
    // 256-byte lines, are written by neighbouring blocks close in time
    const int r = blockIdx.x;
    const int K = 3 * n_i;
    const int nseq = tc >> 1;
    const int nchunk = (K + tc - 1) / tc;
    double* ldsd = (double*)lds;
    for (int cy = blockIdx.y; cy < nchunk; cy += gridDim.y) {     // column chunks (grid-stride)
    const int k0 = cy * tc;
    // loads issued in batches of 8 per thread before their LDS stores (latency hiding)
    constexpr int LU = 8;
    for (int t0 = threadIdx.x; t0 < nz * tc; t0 += NT * LU) {
        double v[LU];
#pragma unroll
        for (int q = 0; q < LU; ++q) {
            const int t = t0 + q * NT;
            const int n0 = t / tc, c = t - n0 * tc, k = k0 + c;
            v[q] = (t < nz * tc && k < K) ? f[((int64_t)r * nz + n0) * K + k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < LU; ++q) {
            const int t = t0 + q * NT;
            if (t >= nz * tc) break;
            const int n0 = t / tc, c = t - n0 * tc, k = k0 + c;
            double x = v[q];
            if (k < K) {
                if (project) x -= tot[r * 3 + (k % 3)] * inv_cnt;     // mean over the cell's atoms
                if (FORM == FBC_FORM_SPLIT_FP16) x = ldexp(x, esc);
            }
            ldsd[2 * ((c >> 1) * nz + (int)bitrev(n0, logn)) + (c & 1)] = x;
        }
    }
    __syncthreads();
    lds_fft(lds, nseq, logn, tw, false);
    const int nm = (nz >> 1) + 1;
    // per mode: B elements of one mode occupy 16*ct*kp values (x2 for the bf16 split)
    const int64_t mode_elems =
        (int64_t)16 * ct * kp * ((FORM == FBC_FORM_SPLIT_BF16 || FORM == FBC_FORM_SPLIT_FP16) ? 2 : 1);
    const int tile = r >> 3, j = r & 7;
    const int nre = 16 * tile + j, nim = nre + 8;
    // G consecutive complex columns per thread, written as whole 16-byte units
    constexpr int G = (FORM == FBC_FORM_FP32) ? 8 : 4;
    if (tc % G == 0) {
        const int ng = tc / G;
        for (int t = threadIdx.x; t < nm * ng; t += NT) {
            const int m = t / ng, g = t - m * ng;
            const int kb = k0 + g * G;
            if (kb >= K) continue;
            double vre[2 * G], vim[2 * G];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const int c = g * G + q;
                double fr = 0.0, fi = 0.0;
                if (kb + q < K) {
                    const double2 z = lds[(c >> 1) * nz + m];
                    const double2 zn = lds[(c >> 1) * nz + ((nz - m) & (nz - 1))];
                    if ((c & 1) == 0) {
                        fr = 0.5 * (z.x + zn.x);
                        fi = 0.5 * (z.y - zn.y);
                    } else {
                        fr = 0.5 * (z.y + zn.y);
                        fi = 0.5 * (zn.x - z.x);
                    }
                    if (m == 0 || 2 * m == nz) fi = 0.0;
                }
                vre[2 * q] = fr;
                vre[2 * q + 1] = -fi;
                vim[2 * q] = fi;
                vim[2 * q + 1] = fr;
            }
            void* bm;
            if (FORM == FBC_FORM_FP64 || FORM == FBC_FORM_DTABLE_FP64)
                bm = (double*)bfrag + m * mode_elems;
            else if (FORM == FBC_FORM_FP32)
                bm = (float*)bfrag + m * mode_elems;
            else
                bm = (unsigned short*)bfrag + m * mode_elems;
            put_b_units<FORM>(bm, nre, 2 * kb, kp, vre);
            put_b_units<FORM>(bm, nim, 2 * kb, kp, vim);
        }
        __syncthreads();        // the next chunk overwrites the LDS sequences
        continue;
    }
    for (int t = threadIdx.x; t < nm * tc; t += NT) {
        const int m = t / tc, c = t - m * tc, k = k0 + c;
        if (k >= K) continue;
        const double2 z = lds[(c >> 1) * nz + m];
        const double2 zn = lds[(c >> 1) * nz + ((nz - m) & (nz - 1))];
        double fr, fi;
        if ((c & 1) == 0) {
            fr = 0.5 * (z.x + zn.x);
            fi = 0.5 * (z.y - zn.y);
        } else {
            fr = 0.5 * (z.y + zn.y);
            fi = 0.5 * (zn.x - z.x);
        }
        if (m == 0 || 2 * m == nz) fi = 0.0;
        void* bm;
        if (FORM == FBC_FORM_FP64 || FORM == FBC_FORM_DTABLE_FP64)
            bm = (double*)bfrag + m * mode_elems;
        else if (FORM == FBC_FORM_FP32)
            bm = (float*)bfrag + m * mode_elems;
        else
            bm = (unsigned short*)bfrag + m * mode_elems;
        put_b<FORM>(bm, nre, 2 * k, kp, fr);
        put_b<FORM>(bm, nre, 2 * k + 1, kp, -fi);
        put_b<FORM>(bm, nim, 2 * k, kp, fi);
        put_b<FORM>(bm, nim, 2 * k + 1, kp, fr);
    }
    __syncthreads();        // the next chunk overwrites the LDS sequences
    }
}

void launch_line_rfft(hipStream_t st, int form, const double* f, const double* tot, int project,
                      void* bfrag, int R, int nz, int n_i, int kp, int ct, const double2* tw,
                      const int* bexp) {
    int logn = 0;
    while ((1 << logn) < nz) ++logn;
    const int K = 3 * n_i;
    int tc = 8192 / nz;                  // nz * tc doubles = 64 KiB of LDS
    if (tc > 256) tc = 256;
    if (tc < 2) tc = 2;
    const int kk = (K + 1) & ~1;
    if (tc > kk) tc = kk;
    tc &= ~1;
    dim3 grid(R, (unsigned)std::min((K + tc - 1) / tc, 65535));
    const size_t lds = (size_t)nz * tc * sizeof(double);
    const double inv_cnt = 1.0 / ((double)n_i * nz);
    switch (form) {
        case FBC_FORM_FP32:
            hipLaunchKernelGGL(k_line_rfft<FBC_FORM_FP32>, grid, dim3(NT), lds, st, f, tot, project,
                               bfrag, nz, logn, n_i, kp, ct, tc, tw, inv_cnt, bexp);
            break;
        case FBC_FORM_SPLIT_FP16:
            hipLaunchKernelGGL(k_line_rfft<FBC_FORM_SPLIT_FP16>, grid, dim3(NT), lds, st, f, tot,
                               project, bfrag, nz, logn, n_i, kp, ct, tc, tw, inv_cnt, bexp);
            break;
        case FBC_FORM_SPLIT_BF16:
            hipLaunchKernelGGL(k_line_rfft<FBC_FORM_SPLIT_BF16>, grid, dim3(NT), lds, st, f, tot,
                               project, bfrag, nz, logn, n_i, kp, ct, tc, tw, inv_cnt, bexp);
            break;
        default:
            hipLaunchKernelGGL(k_line_rfft<FBC_FORM_FP64>, grid, dim3(NT), lds, st, f, tot, project,
                               bfrag, nz, logn, n_i, kp, ct, tc, tw, inv_cnt, bexp);
            break;
    }
}

// ----------------------------------------------------------------------------------
// Inverse rFFT along the line of the per-mode products, two RHS per complex sequence
// (Z = U_a + i U_b; U(-m) = conj U(m); the imaginary parts of modes 0 and Nz/2 are
// dropped as a real inverse transform does).  Output w[r][row][n0] scaled by 1/Nz, and
// per block and RHS the maximum |w| (for the step bound of Algorithm 2).
// Input layout c[ct][mp][m][16]: columns 0..7 real parts, 8..15 imaginary parts.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_line_irfft(const double* __restrict__ c,
                                                   double* __restrict__ w,
                                                   double* __restrict__ wmax_part, int R, int nz,
                                                   int logn, int mp, int M, int ct, int tr, int pp,
                                                   const double2* __restrict__ tw, int nsplit,
                                                   int64_t split_stride,
                                                   const double2* __restrict__ rowmean,
                                                   const double2* __restrict__ shat,
                                                   const unsigned long long* __restrict__ amax,
                                                   const int* __restrict__ bexp) {
    extern __shared__ double2 lds[];
    const int eb = bexp ? *bexp : 0;
    const int row0 = blockIdx.x * tr;
    const int tile = blockIdx.y;
    const int pair0 = blockIdx.z * pp;          // first RHS pair inside the 8-RHS tile
    const int nseq = tr * pp;
    const int nm = (nz >> 1) + 1;
    (void)ct;                                   // output layout [ct][mp][nm][16]
    // Each (mode, row, RHS pair) of the product output is read once, pair fastest, then
    // mode, then row: the modes of a row are adjacent in the output, so a wave reads one
    // contiguous run; the mirrored half of the spectrum (m > Nz/2) is written from the
    // same values.
    // The first K slice's loads are issued for LU iterations before any is used.
    constexpr int LU = 4;
    const int nload = nm * tr * pp;
    for (int t0 = threadIdx.x; t0 < nload; t0 += NT * LU) {
    double2 pv0[LU], pv1[LU];
#pragma unroll
    for (int q = 0; q < LU; ++q) {
        const int t = t0 + q * NT;
        const int pj = t % pp;
        const int rest = t / pp;
        const int mm = rest % nm, trr = rest / nm;
        const int row = row0 + trr;
        const int ja = 2 * (pair0 + pj);
        pv0[q] = pv1[q] = make_double2(0, 0);
        if (t < nload && row < M) {
            const double* src = c + (((int64_t)tile * mp + row) * nm + mm) * 16;
            pv0[q] = *(const double2*)(src + ja);
            pv1[q] = *(const double2*)(src + ja + 8);
        }
    }
#pragma unroll
    for (int q = 0; q < LU; ++q) {
        const int t = t0 + q * NT;
        if (t >= nload) break;
        const int pj = t % pp;
        const int rest = t / pp;
        const int mm = rest % nm, trr = rest / nm;
        const int s = trr * pp + pj;
        const int row = row0 + trr;
        const int ja = 2 * (pair0 + pj);
        double2 z = make_double2(0, 0), zc = make_double2(0, 0);
        if (row < M) {
            const double* src = c + (((int64_t)tile * mp + row) * nm + mm) * 16;
            const double2 v0 = pv0[q], v1 = pv1[q];
            double ar = v0.x, br = v0.y, ai = v1.x, bi = v1.y;
            for (int ks = 1; ks < nsplit; ++ks) {      // K slices, summed in fixed order
                const double* q = src + ks * split_stride;
                const double2 q0 = *(const double2*)(q + ja), q1 = *(const double2*)(q + ja + 8);
                ar += q0.x;
                br += q0.y;
                ai += q1.x;
                bi += q1.y;
            }
            if (amax) {     // split FP16: the product carries 2^(e_A(m) + e_B)
                const double sc = ldexp(1.0, -(split16_exp_a(amax[mm]) + eb));
                ar *= sc;
                ai *= sc;
                br *= sc;
                bi *= sc;
            }
            if (rowmean) {
                // exact FP64 compensation of the row gauge: + R_b(m) . sum_i f^_i(m)
                const int b = row / 3, cc = row - 3 * b;
                const double2* rm = rowmean + ((int64_t)mm * (M / 3) + b) * 6;
                for (int d = 0; d < 3; ++d) {
                    const double2 g = rm[sym_idx(cc, d)];
                    if (8 * tile + ja < R) {
                        const double2 sv = shat[((int64_t)(8 * tile + ja) * nm + mm) * 3 + d];
                        ar += g.x * sv.x - g.y * sv.y;
                        ai += g.x * sv.y + g.y * sv.x;
                    }
                    if (8 * tile + ja + 1 < R) {
                        const double2 sv = shat[((int64_t)(8 * tile + ja + 1) * nm + mm) * 3 + d];
                        br += g.x * sv.x - g.y * sv.y;
                        bi += g.x * sv.y + g.y * sv.x;
                    }
                }
            }
            if (mm == 0 || 2 * mm == nz) { ai = 0.0; bi = 0.0; }
            z = make_double2(ar - bi, ai + br);     // U_a + i U_b at m
            zc = make_double2(ar + bi, br - ai);    // conj U_a + i conj U_b at Nz - m
        }
        lds[s * nz + bitrev(mm, logn)] = z;
        if (mm > 0 && 2 * mm < nz) lds[s * nz + bitrev(nz - mm, logn)] = zc;
    }
    }
    __syncthreads();
    lds_fft(lds, nseq, logn, tw, true);
    const double scale = 1.0 / nz;
    double mx[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // per RHS inside the tile
    for (int t = threadIdx.x; t < nseq * nz; t += NT) {
        const int s = t / nz, n0 = t - s * nz;
        const int trr = s / pp, pj = s - trr * pp;
        const int row = row0 + trr;
        const int ja = 2 * (pair0 + pj);
        const int ra = 8 * tile + ja;
        if (row >= M) continue;
        const double2 z = lds[s * nz + n0];
        const double wa = z.x * scale, wb = z.y * scale;
        if (ra < R) w[((int64_t)ra * M + row) * nz + n0] = wa;
        if (ra + 1 < R) w[((int64_t)(ra + 1) * M + row) * nz + n0] = wb;
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
            if (q == ja) {
                mx[q] = fmax(mx[q], fabs(wa));
                mx[q + 1] = fmax(mx[q + 1], fabs(wb));
            }
        }
    }
    __syncthreads();
    block_max<8>(mx, (double*)lds);      // the FFT buffer is free again
    if (threadIdx.x < 8) {
        const int rr = 8 * tile + threadIdx.x;
        const int jj = threadIdx.x;
        // each RHS is covered by exactly one pair group (blockIdx.z)
        if (rr < R && jj >= 2 * pair0 && jj < 2 * (pair0 + pp))
            wmax_part[(int64_t)rr * gridDim.x + blockIdx.x] = mx[jj];
    }
}

// Rows and RHS pairs per work group of the inverse transform: 2048 complex values
// (32 KiB of LDS) per group where the line allows it.  The host sizes the per-group
// partial maxima with the same shape.
void irfft_shape(int nz, int* tr, int* pp) {
    if (4 * nz <= 2048) {
        *pp = 4;
        *tr = std::min(64, 2048 / (4 * nz));
    } else {
        *pp = std::max(1, 2048 / nz);
        *tr = 1;
    }
}

void launch_line_irfft(hipStream_t st, const double* c, double* w, double* wmax_part, int R,
                       int nz, int mp, int M, int ct, int ct_grid, const double2* tw, int nsplit,
                       int64_t split_stride, const double2* rowmean, const double2* shat,
                       const unsigned long long* amax, const int* bexp, int* n_part_out) {
    int logn = 0;
    while ((1 << logn) < nz) ++logn;
    int pp, tr;
    irfft_shape(nz, &tr, &pp);
    dim3 grid((M + tr - 1) / tr, ct_grid, 4 / pp);
    size_t lds = (size_t)tr * pp * nz * sizeof(double2);
    if (lds < 8 * NT * sizeof(double)) lds = 8 * NT * sizeof(double);   // reused by the max
    hipLaunchKernelGGL(k_line_irfft, grid, dim3(NT), lds, st, c, w, wmax_part, R, nz, logn, mp, M,
                       ct, tr, pp, tw, nsplit, split_stride, rowmean, shat, amax, bexp);
    if (n_part_out) *n_part_out = (int)grid.x;
}

// ----------------------------------------------------------------------------------
// u[r][n0][row] -= alpha_r * w[r][row][n0] (tiled transpose through LDS), with per
// block partial sums of the updated u per Cartesian component (row % 3).
// Skipped entirely when a data check has latched an error.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_axpy(const double* __restrict__ w, double* __restrict__ u,
                                             double* __restrict__ sum_part, int nz, int M,
                                             double alpha, const double* __restrict__ alpha_d,
                                             const int* __restrict__ status) {
    __shared__ double tile[32][33];
    __shared__ double red[3 * NT];
    if (status && *status) return;
    const int r = blockIdx.z;
    const int row0 = blockIdx.x * 32, n00 = blockIdx.y * 32;
    const double a = alpha_d ? alpha_d[r] : alpha;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const double* wr = w + (int64_t)r * M * nz;
    for (int y = ty; y < 32; y += 8) {
        const int row = row0 + y, n0 = n00 + tx;
        if (row < M && n0 < nz) tile[y][tx] = wr[(int64_t)row * nz + n0];
    }
    __syncthreads();
    double v[3] = {0, 0, 0};
    double* ur = u + (int64_t)r * nz * M;
    for (int y = ty; y < 32; y += 8) {
        const int n0 = n00 + y, row = row0 + tx;
        if (row < M && n0 < nz) {
            const int64_t idx = (int64_t)n0 * M + row;
            const double x = ur[idx] - a * tile[tx][y];
            ur[idx] = x;
            v[row % 3] += x;
        }
    }
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
        const int64_t nb = (int64_t)gridDim.x * gridDim.y;
        const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        for (int c = 0; c < 3; ++c) sum_part[((int64_t)r * nb + b) * 3 + c] = v[c];
    }
}

void launch_axpy(hipStream_t st, const double* w, double* u, double* sum_part, int R, int nz,
                 int M, double alpha, const double* alpha_d, const int* status, int* n_part_out) {
    dim3 grid((M + 31) / 32, (nz + 31) / 32, R);
    hipLaunchKernelGGL(k_axpy, grid, dim3(NT), 0, st, w, u, sum_part, nz, M, alpha, alpha_d,
                       status);
    if (n_part_out) *n_part_out = (int)(grid.x * grid.y);
}

// Mean over all pad atoms and layers per RHS and component, then subtraction.
__global__ void __launch_bounds__(NT) k_mean_reduce(const double* __restrict__ part, int n_part,
                                                    double* __restrict__ mean_out, double inv_n,
                                                    const int* __restrict__ status) {
    __shared__ double red[3 * NT];
    if (status && *status) return;
    const int r = blockIdx.x;
    double v[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < n_part; b += NT)
        for (int c = 0; c < 3; ++c) v[c] += part[((int64_t)r * n_part + b) * 3 + c];
    block_sum<3>(v, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) mean_out[r * 3 + c] = v[c] * inv_n;
}

__global__ void __launch_bounds__(NT) k_mean_sub(double* __restrict__ u,
                                                 const double* __restrict__ mean, int64_t per_rhs,
                                                 int R, const int* __restrict__ status) {
    if (status && *status) return;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < per_rhs * R;
         idx += (int64_t)gridDim.x * NT) {
        const int r = (int)(idx / per_rhs);
        const int64_t e = idx - (int64_t)r * per_rhs;
        u[idx] -= mean[r * 3 + (int)(e % 3)];
    }
}

void launch_mean(hipStream_t st, double* u, const double* sum_part, int n_part, double* mean_out,
                 int R, int nz, int M, const int* status) {
    const double inv_n = 1.0 / ((double)nz * (M / 3));
    hipLaunchKernelGGL(k_mean_reduce, dim3(R), dim3(NT), 0, st, sum_part, n_part, mean_out, inv_n,
                       status);
    const int64_t per_rhs = (int64_t)nz * M;
    const int64_t total = per_rhs * R;
    hipLaunchKernelGGL(k_mean_sub, dim3((unsigned)grid_blocks(total)), dim3(NT), 0, st, u,
                       mean_out, per_rhs, R, status);
}

// ----------------------------------------------------------------------------------
// Relax (Algorithm 2) on raw residuals, per RHS.  Stage 1: block partials of
// <f_k, f_{k+1} - f_k>, ||f_{k+1} - f_k||^2 and ||f_{k+1}||_inf.  Stage 2: one block per
// RHS reduces them in fixed order and sets alpha_{k+1} (alpha = 1 before the third
// iteration or without relaxation; alpha < 0 -> 1; zero denominator keeps alpha_k).
// ----------------------------------------------------------------------------------
#define RELAX_PARTS 64
__global__ void __launch_bounds__(NT) k_relax_part(const double* __restrict__ fnew,
                                                   const double* __restrict__ fprev,
                                                   double* __restrict__ part, int64_t per_rhs,
                                                   int use_prev) {
    __shared__ double red[3 * NT];
    const int r = blockIdx.y;
    const double* a = fnew + (int64_t)r * per_rhs;
    const double* b = fprev + (int64_t)r * per_rhs;
    double v[2] = {0, 0};
    double mx[1] = {0};
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < per_rhs;
         e += (int64_t)NT * gridDim.x) {
        const double x = a[e];
        mx[0] = fmax(mx[0], fabs(x));
        if (use_prev) {
            const double y = b[e];
            const double d = x - y;
            v[0] += y * d;
            v[1] += d * d;
        }
    }
    block_sum<2>(v, red);
    block_max<1>(mx, red);
    if (threadIdx.x == 0) {
        double* p = part + ((int64_t)r * gridDim.x + blockIdx.x) * 3;
        p[0] = v[0];
        p[1] = v[1];
        p[2] = mx[0];
    }
}

__global__ void __launch_bounds__(NT) k_relax_alpha(const double* __restrict__ part, int n_part,
                                                    double* __restrict__ alpha_d,
                                                    double* __restrict__ finf_d, int use_relax) {
    __shared__ double red[2 * NT];
    const int r = blockIdx.x;
    double v[2] = {0, 0};
    double mx[1] = {0};
    for (int b = threadIdx.x; b < n_part; b += NT) {
        v[0] += part[((int64_t)r * n_part + b) * 3 + 0];
        v[1] += part[((int64_t)r * n_part + b) * 3 + 1];
        mx[0] = fmax(mx[0], part[((int64_t)r * n_part + b) * 3 + 2]);
    }
    block_sum<2>(v, red);
    block_max<1>(mx, red);
    if (threadIdx.x == 0) {
        finf_d[r] = mx[0];
        double a = 1.0;
        if (use_relax) {
            const double prev = alpha_d[r];
            a = prev;
            if (v[1] > 0.0) a = -prev * v[0] / v[1];
            if (a < 0.0) a = 1.0;
        }
        alpha_d[r] = a;
    }
}

void launch_relax_alpha(hipStream_t st, const double* fnew, const double* fprev, double* part,
                        double* alpha_d, double* finf_d, int R, int64_t per_rhs, int k,
                        int relax) {
    const int use = (relax && k >= 2) ? 1 : 0;
    hipLaunchKernelGGL(k_relax_part, dim3(RELAX_PARTS, R), dim3(NT), 0, st, fnew, fprev, part,
                       per_rhs, use);
    hipLaunchKernelGGL(k_relax_alpha, dim3(R), dim3(NT), 0, st, part, RELAX_PARTS, alpha_d, finf_d,
                       use);
}

// Step bound (Algorithm 2 lines 6-8) from the per-block maxima of |w|.
__global__ void __launch_bounds__(NT) k_relax_clamp(const double* __restrict__ wmax_part,
                                                    int n_part, double* __restrict__ alpha_d,
                                                    double* __restrict__ stepinf_d, double du_max,
                                                    int use_bound) {
    __shared__ double red[NT];
    const int r = blockIdx.x;
    double mx[1] = {0};
    for (int b = threadIdx.x; b < n_part; b += NT)
        mx[0] = fmax(mx[0], wmax_part[(int64_t)r * n_part + b]);
    block_max<1>(mx, red);
    if (threadIdx.x == 0) {
        double a = alpha_d[r];
        if (use_bound && du_max > 0.0 && a * mx[0] > du_max) a = du_max / mx[0];
        alpha_d[r] = a;
        stepinf_d[r] = a * mx[0];
    }
}

void launch_relax_clamp(hipStream_t st, const double* wmax_part, int n_part, double* alpha_d,
                        double* stepinf_d, int R, double du_max, int k, int relax) {
    const int use = (relax && k >= 2) ? 1 : 0;
    hipLaunchKernelGGL(k_relax_clamp, dim3(R), dim3(NT), 0, st, wmax_part, n_part, alpha_d,
                       stepinf_d, du_max, use);
}

__global__ void __launch_bounds__(NT) k_copy(const double* __restrict__ a, double* __restrict__ b,
                                             int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        b[i] = a[i];
}

__global__ void k_relax_out(const double* __restrict__ alpha_d, const double* __restrict__ finf_d,
                            const double* __restrict__ stepinf_d, const double* __restrict__ mean_d,
                            fbc_relax_out* __restrict__ out, int R, int k, double tol_f) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    fbc_relax_out o;
    o.alpha = alpha_d[r];
    o.f_inf = finf_d[r];
    o.step_inf = stepinf_d[r];
    for (int c = 0; c < 3; ++c) o.mean_removed[c] = mean_d[r * 3 + c];
    o.converged = finf_d[r] < tol_f ? 1 : 0;
    o.k = k;
    out[r] = o;
}

void launch_relax_finish(hipStream_t st, const double* fnew, double* fprev, int64_t n,
                         const double* alpha_d, const double* finf_d, const double* stepinf_d,
                         const double* mean_d, fbc_relax_out* out, int R, int k, double tol_f) {
    hipLaunchKernelGGL(k_copy, dim3((unsigned)grid_blocks(n)), dim3(NT), 0, st, fnew, fprev,
                       n);
    if (out)
        hipLaunchKernelGGL(k_relax_out, dim3((R + 63) / 64), dim3(64), 0, st, alpha_d, finf_d,
                           stepinf_d, mean_d, out, R, k, tol_f);
}

__global__ void k_fill(double* p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        p[i] = v;
}

void launch_fill(hipStream_t st, double* p, int64_t n, double v) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill, dim3((unsigned)grid_blocks(n)), dim3(NT), 0, st, p, n, v);
}
