// Line transforms, update and reductions of the FBC pad update (Section 2.3.2,
// eq. flexbc.up=Gpipl*fipl with eq. mean(u^p)=0; the update step of Algorithm 1), and the
// residual-based relaxation (Section 2.3.3, eq. alpha, Algorithm 2).
// All reductions use a fixed partition and a fixed-order tree, so results are bitwise
// reproducible from run to run (no floating-point atomics).
#include "fft_lds.h"
#include <algorithm>
#include <mutex>
#include <set>

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
template <int NV, int NTH = NT>
__device__ inline void block_max(double (&v)[NV], double* red) {
    for (int c = 0; c < NV; ++c) red[c * NTH + threadIdx.x] = v[c];
    __syncthreads();
    for (int s = NTH / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < NV; ++c)
                red[c * NTH + threadIdx.x] = fmax(red[c * NTH + threadIdx.x], red[c * NTH + threadIdx.x + s]);
        __syncthreads();
    }
    for (int c = 0; c < NV; ++c) v[c] = red[c * NTH];
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
    // columns i = tid, tid + NT, ... in order; the loads of LU of them are issued together
    constexpr int LU = 4;
    for (int i0 = threadIdx.x; i0 < n_i; i0 += NT * LU) {
        double x[LU][3];
#pragma unroll
        for (int k = 0; k < LU; ++k) {
            const int i = i0 + k * NT;
#pragma unroll
            for (int c = 0; c < 3; ++c) x[k][c] = (i < n_i) ? row[3 * i + c] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < LU; ++k) {
            if (i0 + k * NT >= n_i) break;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[c] += x[k][c];
                v[3 + c] += fabs(x[k][c]);
                mx[0] = fmax(mx[0], fabs(x[k][c]));
                if (!isfinite(x[k][c])) v[6] = 1.0;
            }
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

// Split-FP16 form: scale exponent of the force operand of each RHS (one work group per
// RHS), from a bound on its transformed forces, |f^(m)| <= sum_n0 |f(n0)| <= Nz max|f|
// (twice that after the projection), so that the scaled values stay below 2^14.  One
// exponent per RHS: a RHS far smaller than another of the same cell (a converged one
// beside one that is not) keeps its full 22-bit split instead of falling into subnormals.
__global__ void __launch_bounds__(NT) k_bexp(const double* __restrict__ sums, int nz,
                                             int* __restrict__ bexp) {
    __shared__ double red[NT];
    const int r = blockIdx.x;
    double mx[1] = {0.0};
    for (int n0 = threadIdx.x; n0 < nz; n0 += NT)
        mx[0] = fmax(mx[0], sums[((int64_t)r * nz + n0) * NF_STRIDE + 6]);
    block_max<1>(mx, red);
    if (threadIdx.x == 0) {
        const double bound = 2.0 * nz * mx[0];
        bexp[r] = (bound > 0.0 && isfinite(bound)) ? 13 - ilogb(bound) : 0;
    }
}

// Net force of the whole cell per RHS and component (sum over layers in fixed order):
// tot[r][c].  Only this total enters the gauge (line mode 0); the check compares it with
// the total absolute force.  With shat != NULL the same block then transforms the
// per-layer net force along the line (after the projection, if any):
// shat[r][m][c] = sum_n0 (s_c(n0) - tot_c / Nz) e^{-2 pi i m n0 / Nz}, m = 0..Nz/2,
// which multiplies the subtracted row means in the inverse transform.  A layer whose net
// force lies within the rounding bound of its own summation, |s_c| <= n_i 2^-52 sum|f_c|,
// is indistinguishable from a balanced one and enters as exactly zero; shat_on[r] = 0 then
// records that the whole transform vanishes, so the compensation can be skipped.
__global__ void __launch_bounds__(NT) k_netforce_total(const double* __restrict__ sums, int nz, int logn,
                                                       int n_i, double tol, int check, int project,
                                                       double* __restrict__ tot,
                                                       const double2* __restrict__ tw,
                                                       double2* __restrict__ shat,
                                                       int* __restrict__ shat_on,
                                                       int* __restrict__ status) {
    extern __shared__ double2 lds[];             // 3 Nz (line transforms); >= 6 NT doubles
    const int r = blockIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int n0 = threadIdx.x; n0 < nz; n0 += NT)
        for (int c = 0; c < 6; ++c) v[c] += sums[((int64_t)r * nz + n0) * NF_STRIDE + c];
    block_sum<6>(v, (double*)lds);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) tot[r * 3 + c] = v[c];
        if (check && !project) {
            int bits = 0;
            for (int c = 0; c < 3; ++c)
                if (fabs(v[c]) > tol * v[3 + c]) bits |= ST_NETFORCE;
            if (bits) atomicOr(status, bits);
        }
    }
    if (!shat) return;
    // v[0..2] hold the totals in every thread after block_sum
    const double gam = (double)n_i * 0x1p-52;
    for (int e = threadIdx.x; e < 3 * nz; e += NT) {
        const int c = e / nz, n0 = e - c * nz;
        const double sub = project ? v[c] / nz : 0.0;
        const double* o = sums + ((int64_t)r * nz + n0) * NF_STRIDE;
        double s = o[c] - sub;
        if (fabs(s) <= gam * o[3 + c] && isfinite(o[3 + c])) s = 0.0;
        lds[c * nz + bitrev(n0, logn)] = make_double2(s, 0.0);
    }
    __syncthreads();
    lds_fft(lds, 3, logn, tw, false);
    const int nm = (nz >> 1) + 1;
    int any = 0;
    for (int e = threadIdx.x; e < 3 * nm; e += NT) {
        const int m = e / 3, c = e - 3 * m;
        double2 z = lds[c * nz + m];
        if (project && m == 0) z = make_double2(0.0, 0.0);
        shat[((int64_t)r * nm + m) * 3 + c] = z;
        any |= (z.x != 0.0 || z.y != 0.0);
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) shat_on[r] = any;     // 0: s^ = 0 exactly, the compensation adds 0
}

void launch_netforce(hipStream_t st, const double* f, double* sums, double* tot, double2* shat,
                     int* shat_on, int R, int nz, int n_i, double tol, int check, int project,
                     const double2* tw, int* bexp, int* status) {
    int logn = 0;
    while ((1 << logn) < nz) ++logn;
    hipLaunchKernelGGL(k_netforce, dim3(nz, R), dim3(NT), 0, st, f, sums, nz, n_i, check, status);
    const size_t lds = std::max((size_t)3 * nz * sizeof(double2), (size_t)6 * NT * sizeof(double));
    hipLaunchKernelGGL(k_netforce_total, dim3(R), dim3(NT), lds, st, sums, nz, logn, n_i, tol, check, project, tot,
                       tw, shat, shat_on, status);
    if (bexp) hipLaunchKernelGGL(k_bexp, dim3(R), dim3(NT), 0, st, sums, nz, bexp);
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
        const _Float16 hi = f64_to_f16(v);
        const _Float16 lo = f64_to_f16(v - (double)hi);
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
                const _Float16 h = f64_to_f16(v[j]);
                hi[j] = __builtin_bit_cast(unsigned short, h);
                lo[j] = __builtin_bit_cast(unsigned short, f64_to_f16(v[j] - (double)h));
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

typedef double dv2_t __attribute__((ext_vector_type(2)));

// pairs: K even and f 16-byte aligned, so two adjacent columns load as one 16-byte access
// and store as one complex LDS entry.
template <int FORM, int NTH>
__global__ void __launch_bounds__(NTH) k_line_rfft(const double* __restrict__ f,
                                                  const double* __restrict__ tot, int project,
                                                  void* __restrict__ bfrag, int nz, int logn,
                                                  int n_i, int kp, int ct, int tc,
                                                  const double2* __restrict__ tw, double inv_cnt,
                                                  const int* __restrict__ bexp, int pairs) {
    extern __shared__ double2 lds[];
    // RHS fastest across blocks: the 8 RHS of a column tile, whose 64-byte column runs
    // fill the same 1 KiB fragment blocks, are written by neighbouring blocks close in time
    const int r = blockIdx.x;
    const int esc = (FORM == FBC_FORM_SPLIT_FP16) ? bexp[r] : 0;   // power-of-two operand scale
    const int K = 3 * n_i;
    const int nseq = tc >> 1;
    const int ss = nz + 1;                  // sequence stride (complex values)
    const int nchunk = (K + tc - 1) / tc;
    double* ldsd = (double*)lds;
    for (int cy = blockIdx.y; cy < nchunk; cy += gridDim.y) {     // column chunks (grid-stride)
    const int k0 = cy * tc;
    // loads issued in batches of 8 per thread before their LDS stores (latency hiding);
    // the forces are read once per update: nontemporal loads keep them from displacing
    // the fragments the product reads next (measured: 2 % faster large step)
    constexpr int LU = 8;
    if (pairs) {
        const int hp = tc >> 1;
        for (int t0 = threadIdx.x; t0 < nz * hp; t0 += NTH * LU) {
            dv2_t v[LU];
#pragma unroll
            for (int q = 0; q < LU; ++q) {
                const int t = t0 + q * NTH;
                const int n0 = t / hp, k = k0 + 2 * (t - n0 * hp);
                v[q] = (t < nz * hp && k < K)
                           ? __builtin_nontemporal_load((const dv2_t*)(f + ((int64_t)r * nz + n0) * K + k))
                           : dv2_t{0.0, 0.0};
            }
#pragma unroll
            for (int q = 0; q < LU; ++q) {
                const int t = t0 + q * NTH;
                if (t >= nz * hp) break;
                const int n0 = t / hp, p = t - n0 * hp, k = k0 + 2 * p;
                double x0 = v[q].x, x1 = v[q].y;
                if (k < K) {
                    if (project) {                  // mean over the cell's atoms
                        x0 -= tot[r * 3 + (k % 3)] * inv_cnt;
                        x1 -= tot[r * 3 + ((k + 1) % 3)] * inv_cnt;
                    }
                    if (FORM == FBC_FORM_SPLIT_FP16) {
                        x0 = ldexp(x0, esc);
                        x1 = ldexp(x1, esc);
                    }
                }
                lds[p * ss + (int)bitrev(n0, logn)] = make_double2(x0, x1);
            }
        }
    } else
    for (int t0 = threadIdx.x; t0 < nz * tc; t0 += NTH * LU) {
        double v[LU];
#pragma unroll
        for (int q = 0; q < LU; ++q) {
            const int t = t0 + q * NTH;
            const int n0 = t / tc, c = t - n0 * tc, k = k0 + c;
            v[q] = (t < nz * tc && k < K) ? __builtin_nontemporal_load(&f[((int64_t)r * nz + n0) * K + k]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < LU; ++q) {
            const int t = t0 + q * NTH;
            if (t >= nz * tc) break;
            const int n0 = t / tc, c = t - n0 * tc, k = k0 + c;
            double x = v[q];
            if (k < K) {
                if (project) x -= tot[r * 3 + (k % 3)] * inv_cnt;     // mean over the cell's atoms
                if (FORM == FBC_FORM_SPLIT_FP16) x = ldexp(x, esc);
            }
            ldsd[2 * ((c >> 1) * ss + (int)bitrev(n0, logn)) + (c & 1)] = x;
        }
    }
    __syncthreads();
    lds_fft_s<false>(lds, nseq, ss, logn, tw);
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
        for (int t = threadIdx.x; t < nm * ng; t += NTH) {
            const int m = t / ng, g = t - m * ng;
            const int kb = k0 + g * G;
            if (kb >= K) continue;
            double vre[2 * G], vim[2 * G];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const int c = g * G + q;
                double fr = 0.0, fi = 0.0;
                if (kb + q < K) {
                    const double2 z = lds[(c >> 1) * ss + m];
                    const double2 zn = lds[(c >> 1) * ss + ((nz - m) & (nz - 1))];
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
    for (int t = threadIdx.x; t < nm * tc; t += NTH) {
        const int m = t / tc, c = t - m * tc, k = k0 + c;
        if (k >= K) continue;
        const double2 z = lds[(c >> 1) * ss + m];
        const double2 zn = lds[(c >> 1) * ss + ((nz - m) & (nz - 1))];
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
    // columns per work group: the largest power of two whose (Nz + 1) * tc doubles fit the
    // LDS budget
    constexpr int budget = 8192;          // 64 KiB
    int tc = 256;
    while (tc > 2 && tc * (nz + 1) > budget) tc >>= 1;
    // long lines: at least 8 columns (64-byte runs of each layer's forces) while the group's
    // sequences fit in 66 KiB (two groups per CU)
    while (tc < 8 && 2 * tc * (nz + 1) * 8 <= 66 * 1024) tc <<= 1;
    // lines of 1024 layers and more: 1024 threads per work group over 16 columns (128-byte
    // runs of each layer; 131 KiB of LDS at Nz = 1024, one group filling a CU with sixteen
    // waves), fewer columns where the LDS does not hold them.  Measured on the long
    // workload: 1.13-1.15 ms against 1.27 ms for 4 columns x 256 threads (and 1.39 / 1.93
    // ms for 8 / 4 columns x 1024 threads)
    const bool wide = nz >= 1024;
    if (wide) {
        tc = 16;
        while (tc > 2 && (size_t)(nz + 1) * tc * sizeof(double) > 160 * 1024) tc >>= 1;   // the CU's LDS
    }
    const int kk = (K + 1) & ~1;
    if (tc > kk) tc = kk;
    tc &= ~1;
    dim3 grid(R, (unsigned)std::min((K + tc - 1) / tc, 65535));
    const int pairs = ((K & 1) == 0 && ((uintptr_t)f & 15) == 0) ? 1 : 0;
    const size_t lds = (size_t)(nz + 1) * tc * sizeof(double);
    const double inv_cnt = 1.0 / ((double)n_i * nz);
#define RF_LAUNCH(FM)                                                                                       \
    do {                                                                                                    \
        if (wide) {                                                                                         \
            hipLaunchKernelGGL((k_line_rfft<FM, 1024>), grid, dim3(1024), lds, st, f, tot, project, bfrag, nz, logn, \
                               n_i, kp, ct, tc, tw, inv_cnt, bexp, pairs);                                  \
        } else {                                                                                            \
            hipLaunchKernelGGL((k_line_rfft<FM, NT>), grid, dim3(NT), lds, st, f, tot, project, bfrag, nz, logn, \
                               n_i, kp, ct, tc, tw, inv_cnt, bexp, pairs);                                  \
        }                                                                                                   \
    } while (0)
    switch (form) {
        case FBC_FORM_FP32: RF_LAUNCH(FBC_FORM_FP32); break;
        case FBC_FORM_SPLIT_FP16: RF_LAUNCH(FBC_FORM_SPLIT_FP16); break;
        case FBC_FORM_SPLIT_BF16: RF_LAUNCH(FBC_FORM_SPLIT_BF16); break;
        default: RF_LAUNCH(FBC_FORM_FP64); break;
    }
#undef RF_LAUNCH
}

// ----------------------------------------------------------------------------------
// Inverse rFFT along the line of the per-mode products, two RHS per complex sequence
// (Z = U_a + i U_b; U(-m) = conj U(m); the imaginary parts of modes 0 and Nz/2 are
// dropped as a real inverse transform does).
// Input layout c[ct][mp][m][16]: columns 0..7 real parts, 8..15 imaginary parts, one
// record per K slice (split_stride apart).
// ----------------------------------------------------------------------------------

// The row-gauge compensation terms R_b(m) . s^(m) of one row (atom b, component cc) for
// the two RHS of a pair, from the three entries g[d] = R_b(m)[cc][d] and s^ of each RHS:
// explicit fused multiply-adds in a fixed order, so that a kernel that stages the terms
// ahead of the product records gets the same bits as one that computes them in place.
__device__ inline void comp_core(const double2 (&g)[3], const double2 (&sa)[3], const double2 (&sb)[3],
                                 double& dar, double& dai, double& dbr, double& dbi) {
    dar = dai = dbr = dbi = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dar = fma(-g[d].y, sa[d].y, fma(g[d].x, sa[d].x, dar));
        dai = fma(g[d].y, sa[d].x, fma(g[d].x, sa[d].y, dai));
        dbr = fma(-g[d].y, sb[d].y, fma(g[d].x, sb[d].x, dbr));
        dbi = fma(g[d].y, sb[d].x, fma(g[d].x, sb[d].y, dbi));
    }
}

// The compensation is zero for RHS whose per-layer net forces all vanish (s^ = 0): skipped
// for pairs with no such RHS (shat_on[r] = 0), which saves its loads for the usual forces.
__device__ inline bool comp_on(int ra, int R, const double2* __restrict__ rowmean,
                               const int* __restrict__ shat_on) {
    return rowmean && ((ra < R && shat_on[ra]) || (ra + 1 < R && shat_on[ra + 1]));
}

__device__ inline void comp_load_s(int mm, int nm, int ra, int R, const double2* __restrict__ shat,
                                   double2 (&sa)[3], double2 (&sb)[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sa[d] = ra < R ? shat[((int64_t)ra * nm + mm) * 3 + d] : make_double2(0, 0);
        sb[d] = ra + 1 < R ? shat[((int64_t)(ra + 1) * nm + mm) * 3 + d] : make_double2(0, 0);
    }
}

__device__ inline void comp_load_g(int mm, int row, int M, const double2* __restrict__ rowmean,
                                   double2 (&g)[3]) {
    const int b = row / 3, cc = row - 3 * b;
    const double2* rm = rowmean + ((int64_t)mm * (M / 3) + b) * 6;
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = rm[sym_idx(cc, d)];
}

// split FP16: the product of RHS r carries 2^(e_A(m) + e_B(r))
__device__ inline void mode_scale(int mm, int ra, int R, const unsigned long long* __restrict__ amax,
                                  const int* __restrict__ bexp, double& ar, double& br, double& ai,
                                  double& bi) {
    if (amax) {
        const int ea = split16_exp_a(amax[mm]);
        const double sa = ldexp(1.0, -(ea + (ra < R ? bexp[ra] : 0)));
        const double sb = ldexp(1.0, -(ea + (ra + 1 < R ? bexp[ra + 1] : 0)));
        ar *= sa;
        ai *= sa;
        br *= sb;
        bi *= sb;
    }
}

// Final value of one (row, mode) of an RHS pair (columns ja, ja + 1 of the tile): K
// slices summed in fixed order, the split-FP16 scale removed, the row-gauge compensation
// + R_b(m) . s^(m) added in FP64.  v0, v1: slice 0 at columns ja and ja + 8.  Every
// kernel that consumes the product output goes through mode_scale, comp_core and the
// same additions, so they agree bit for bit.
__device__ inline void mode_adjust(int mm, int row, int M, int nm, int ra, int R,
                                   const double2* __restrict__ rowmean,
                                   const double2* __restrict__ shat,
                                   const int* __restrict__ shat_on,
                                   const unsigned long long* __restrict__ amax,
                                   const int* __restrict__ bexp,
                                   double& ar, double& br, double& ai, double& bi) {
    mode_scale(mm, ra, R, amax, bexp, ar, br, ai, bi);
    if (comp_on(ra, R, rowmean, shat_on)) {
        double2 g[3], sa[3], sb[3];
        comp_load_g(mm, row, M, rowmean, g);
        comp_load_s(mm, nm, ra, R, shat, sa, sb);
        double dar, dai, dbr, dbi;
        comp_core(g, sa, sb, dar, dai, dbr, dbi);
        ar += dar;
        ai += dai;
        br += dbr;
        bi += dbi;
    }
    if (mm == 0 || mm == nm - 1) {      // modes 0 and Nz/2 are real
        ai = 0.0;
        bi = 0.0;
    }
}

__device__ inline void mode_value(double2 v0, double2 v1, const double* __restrict__ src, int ja,
                                  int nsplit, int64_t split_stride, int mm, int row, int M, int nm,
                                  int ra, int R, const double2* __restrict__ rowmean,
                                  const double2* __restrict__ shat, const int* __restrict__ shat_on,
                                  const unsigned long long* __restrict__ amax,
                                  const int* __restrict__ bexp,
                                  double& ar, double& br, double& ai, double& bi) {
    ar = v0.x;
    br = v0.y;
    ai = v1.x;
    bi = v1.y;
    for (int ks = 1; ks < nsplit; ++ks) {
        const double* q = src + ks * split_stride;
        const double2 q0 = *(const double2*)(q + ja), q1 = *(const double2*)(q + ja + 8);
        ar += q0.x;
        br += q0.y;
        ai += q1.x;
        bi += q1.y;
    }
    mode_adjust(mm, row, M, nm, ra, R, rowmean, shat, shat_on, amax, bexp, ar, br, ai, bi);
}

// Gathers the spectra of tr rows x pp RHS pairs of one column tile into LDS (bit-reversed,
// sequence s = pj * tr + trr at s * ss) and inverse-transforms them.  Each (mode, row,
// pair) of the product output is read once, pair fastest, then mode, then row: the modes
// of a row are adjacent in the output, so a wave reads one contiguous run; the mirrored
// half of the spectrum (m > Nz/2) is written from the same values.  The first K slice's
// loads are issued LU at a time before any is used.
__device__ inline void gather_inverse(double2* lds, const double* __restrict__ c, int tile, int row0,
                                      int pair0, int tr, int pp, int ss, int R, int nz, int logn,
                                      int mp, int M, const double2* __restrict__ tw, int nsplit,
                                      int64_t split_stride, const double2* __restrict__ rowmean,
                                      const double2* __restrict__ shat, const int* __restrict__ shat_on,
                                      const unsigned long long* __restrict__ amax,
                                      const int* __restrict__ bexp) {
    const int nm = (nz >> 1) + 1;
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
            const int s = pj * tr + trr;
            const int row = row0 + trr;
            const int ja = 2 * (pair0 + pj);
            double2 z = make_double2(0, 0), zc = make_double2(0, 0);
            if (row < M) {
                const double* src = c + (((int64_t)tile * mp + row) * nm + mm) * 16;
                double ar, br, ai, bi;
                mode_value(pv0[q], pv1[q], src, ja, nsplit, split_stride, mm, row, M, nm, 8 * tile + ja, R,
                           rowmean, shat, shat_on, amax, bexp, ar, br, ai, bi);
                z = make_double2(ar - bi, ai + br);     // U_a + i U_b at m
                zc = make_double2(ar + bi, br - ai);    // conj U_a + i conj U_b at Nz - m
            }
            lds[s * ss + bitrev(mm, logn)] = z;
            if (mm > 0 && 2 * mm < nz) lds[s * ss + bitrev(nz - mm, logn)] = zc;
        }
    }
    __syncthreads();
    lds_fft_s<true>(lds, tr * pp, ss, logn, tw);
}

// Work unit of a work group of the inverse transforms: units (row group rg of column tile
// `tile`, numbered tile-major) are split into 8 contiguous ranges, one per XCD (work
// groups are dealt to the XCDs round robin by index), and the 4/pp pair groups of a unit
// take consecutive places in its XCD's sequence.  So the pair groups of a unit, which read
// disjoint parts of the same 128-byte product records, run on one XCD at about the same
// time and share those records through its L2, and so do neighbouring row groups, which
// (in the fused update) write neighbouring runs of each layer of u.  Measured on MI355X:
// the inverse transform into w at Nz = 1024 3-4 % faster than with a row x tile x pair grid.
__device__ inline bool xcd_unit(int n_units, int n_rg, int npg, int& tile, int& rg, int& pg) {
    const int u8 = (n_units + 7) >> 3;
    const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
    pg = k % npg;
    const int ul = k / npg, unit = xcd * u8 + ul;
    if (ul >= u8 || unit >= n_units) return false;
    tile = unit / n_rg;
    rg = unit - tile * n_rg;
    return true;
}

static inline int xcd_groups(int n_units, int npg) { return 8 * npg * ((n_units + 7) / 8); }

// Inverse transform into the scratch w[r][row][n0] (scaled by 1/Nz), with per row group
// and RHS the maximum |w| (the step bound of Algorithm 2).  Used by the relaxation step,
// whose step size depends on the whole of w before any update.
__global__ void __launch_bounds__(NT) k_line_irfft(const double* __restrict__ c,
                                                   double* __restrict__ w,
                                                   double* __restrict__ wmax_part, int R, int nz,
                                                   int logn, int mp, int M, int tr, int pp, int n_rg,
                                                   int n_units,
                                                   const double2* __restrict__ tw, int nsplit,
                                                   int64_t split_stride,
                                                   const double2* __restrict__ rowmean,
                                                   const double2* __restrict__ shat,
        const int* __restrict__ shat_on,
                                                   const unsigned long long* __restrict__ amax,
                                                   const int* __restrict__ bexp) {
    extern __shared__ double2 lds[];
    int tile, rg, pg;
    if (!xcd_unit(n_units, n_rg, 4 / pp, tile, rg, pg)) return;
    const int row0 = rg * tr;
    const int pair0 = pg * pp;                  // first RHS pair inside the 8-RHS tile
    const int nseq = tr * pp;
    const int ss = nz + 1;
    gather_inverse(lds, c, tile, row0, pair0, tr, pp, ss, R, nz, logn, mp, M, tw, nsplit, split_stride,
                   rowmean, shat, shat_on, amax, bexp);
    const double scale = 1.0 / nz;
    double mx[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // per RHS inside the tile
    for (int t = threadIdx.x; t < nseq * nz; t += NT) {
        const int s = t / nz, n0 = t - s * nz;
        const int pj = s / tr, trr = s - pj * tr;
        const int row = row0 + trr;
        const int ja = 2 * (pair0 + pj);
        const int ra = 8 * tile + ja;
        if (row >= M) continue;
        const double2 z = lds[s * ss + n0];
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
        // each RHS is covered by exactly one pair group
        if (rr < R && jj >= 2 * pair0 && jj < 2 * (pair0 + pp))
            wmax_part[(int64_t)rr * n_rg + rg] = mx[jj];
    }
}

// Rows and RHS pairs per work group of the inverse transform into w: 2048 complex values
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
                       const int* shat_on, const unsigned long long* amax, const int* bexp,
                       int* n_part_out) {
    (void)ct;
    int logn = 0;
    while ((1 << logn) < nz) ++logn;
    int pp, tr;
    irfft_shape(nz, &tr, &pp);
    const int n_rg = (M + tr - 1) / tr;
    const int n_units = ct_grid * n_rg;
    size_t lds = (size_t)tr * pp * (nz + 1) * sizeof(double2);
    if (lds < 8 * NT * sizeof(double)) lds = 8 * NT * sizeof(double);   // reused by the max
    hipLaunchKernelGGL(k_line_irfft, dim3(xcd_groups(n_units, 4 / pp)), dim3(NT), lds, st, c, w, wmax_part,
                       R, nz, logn, mp, M, tr, pp, n_rg, n_units, tw, nsplit, split_stride, rowmean, shat,
                       shat_on, amax, bexp);
    if (n_part_out) *n_part_out = n_rg;
}

// ----------------------------------------------------------------------------------
// Fused inverse transform and pad update (the update step of Algorithm 1):
//   u[r][n0][row] <- (read_u ? u : 0) - alpha * w[r][row][n0] - mu[r][row % 3]
// straight from the product output, without the w scratch.  A work group owns tr
// consecutive rows (one contiguous run of u per layer) and pp RHS pairs of one column
// tile, placed on the XCDs by xcd_unit: the 4/pp pair groups of a row block run on one
// XCD at about the same time and share the product records (128 bytes per row and mode)
// through its L2.
//  1. gather: the spectra in natural order (mode fastest across threads, so the LDS
//     writes are consecutive), the K slices of LU work items loaded before any is used;
//  2. decimation-in-frequency stages of half length Nz/2 .. 4 in LDS, neighbouring
//     threads on neighbouring sequences (stride Nz + 1: distinct banks);
//  3. per thread four consecutive bit-reversed slots of one sequence: the stages of half
//     length 2 and 1 in registers, then four layers n0 = bitrev(slot) of u, rows fastest
//     across threads (runs of tr values of u per layer).
// mu (mean of the updated u, from k_update_mean) may be NULL (no mean removal).  alpha_d:
// per-RHS step factors on the device in place of alpha (the relaxation step without its
// bound); wmax_part (one RHS pair per group): per RHS and row group the largest |w|.
// Skipped entirely when a data check has latched an error.  Needs Nz >= 16.
// ----------------------------------------------------------------------------------
template <int NSM, int NTH>
__global__ void __launch_bounds__(NTH) k_irfft_update(const double* __restrict__ c,
                                                     double* __restrict__ u, int R, int nz, int logn,
                                                     int mp, int M, int tr, int pp, int n_rg,
                                                     int n_units, const double2* __restrict__ tw,
                                                     int nsplit, int64_t split_stride,
                                                     const double2* __restrict__ rowmean,
                                                     const double2* __restrict__ shat,
        const int* __restrict__ shat_on,
                                                     const unsigned long long* __restrict__ amax,
                                                     const int* __restrict__ bexp, double alpha,
                                                     const double* __restrict__ alpha_d,
                                                     const double* __restrict__ mu, int read_u,
                                                     double* __restrict__ wmax_part,
                                                     const int* __restrict__ status) {
    extern __shared__ double2 lds[];
    if (status && *status) return;
    int tile, rg, pg;
    if (!xcd_unit(n_units, n_rg, 4 / pp, tile, rg, pg)) return;
    const int row0 = rg * tr, pair0 = pg * pp;
    const int ss = nz + 1;
    const int nm = (nz >> 1) + 1;
    const int nseq = tr * pp;
    // 0. row-gauge compensation (pairs with per-layer net force only): the terms of every
    //    (row, mode) staged in the LDS slots of the mode and its mirror, the s^ of a mode
    //    loaded once per 4 rows and all loads of a thread issued before any is used
    //    (computed inside the gather, each term waited for its own loads after the
    //    records': 1.5 ms more per update of the long lines)
    bool stage = false;                         // the same for the whole work group
    for (int pj = 0; pj < pp; ++pj) stage = stage || comp_on(8 * tile + 2 * (pair0 + pj), R, rowmean, shat_on);
    if (stage) {
        constexpr int CR = 4;
        const int nch = (tr + CR - 1) / CR;
        const int n0 = nm * pp * nch;
        for (int t = threadIdx.x; t < n0; t += NTH) {
            const int mm = t % nm, rest = t / nm;
            const int pj = rest % pp, ch = rest / pp;
            const int ra = 8 * tile + 2 * (pair0 + pj);
            if (!comp_on(ra, R, rowmean, shat_on)) continue;
            double2 sa[3], sb[3], g[CR][3];
            comp_load_s(mm, nm, ra, R, shat, sa, sb);
#pragma unroll
            for (int q = 0; q < CR; ++q) {
                const int trr = ch * CR + q, row = row0 + trr;
                if (trr < tr && row < M) {
                    comp_load_g(mm, row, M, rowmean, g[q]);
                } else {
                    g[q][0] = g[q][1] = g[q][2] = make_double2(0, 0);
                }
            }
#pragma unroll
            for (int q = 0; q < CR; ++q) {
                const int trr = ch * CR + q, row = row0 + trr;
                if (trr >= tr || row >= M) continue;
                double dar, dai, dbr, dbi;
                comp_core(g[q], sa, sb, dar, dai, dbr, dbi);
                double2* sq = lds + (pj * tr + trr) * ss;
                sq[mm] = make_double2(dar, dbr);
                if (mm > 0 && 2 * mm < nz) sq[nz - mm] = make_double2(dai, dbi);
            }
        }
        __syncthreads();
    }
    // 1. gather
    {
        constexpr int LU = NSM >= 8 ? 1 : 8 / NSM;
        const int nload = nm * nseq;
        for (int t0 = threadIdx.x; t0 < nload; t0 += NTH * LU) {
            double2 v0[LU][NSM], v1[LU][NSM];
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                const int t = t0 + k * NTH;
                const int mm = t % nm, rest = t / nm;
                const int pj = rest % pp, trr = rest / pp;
                const int row = row0 + trr;
                const int ja = 2 * (pair0 + pj);
                const double* src = c + (((int64_t)tile * mp + row) * nm + mm) * 16 + ja;
#pragma unroll
                for (int ks = 0; ks < NSM; ++ks) {
                    v0[k][ks] = v1[k][ks] = make_double2(0, 0);
                    if (t < nload && row < M && ks < nsplit) {
                        v0[k][ks] = *(const double2*)(src + ks * split_stride);
                        v1[k][ks] = *(const double2*)(src + ks * split_stride + 8);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                const int t = t0 + k * NTH;
                if (t >= nload) break;
                const int mm = t % nm, rest = t / nm;
                const int pj = rest % pp, trr = rest / pp;
                const int row = row0 + trr;
                const int ja = 2 * (pair0 + pj);
                double ar = v0[k][0].x, br = v0[k][0].y, ai = v1[k][0].x, bi = v1[k][0].y;
#pragma unroll
                for (int ks = 1; ks < NSM; ++ks) {     // K slices in fixed order (zeros past nsplit)
                    if (ks < nsplit) {
                        ar += v0[k][ks].x;
                        br += v0[k][ks].y;
                        ai += v1[k][ks].x;
                        bi += v1[k][ks].y;
                    }
                }
                double2 z = make_double2(0, 0), zc = make_double2(0, 0);
                double2* sq = lds + (pj * tr + trr) * ss;
                if (row < M) {
                    const int ra = 8 * tile + ja;
                    mode_scale(mm, ra, R, amax, bexp, ar, br, ai, bi);
                    if (comp_on(ra, R, rowmean, shat_on)) {     // the terms staged in step 0
                        const double2 d0 = sq[mm];
                        const double2 d1 = (mm > 0 && 2 * mm < nz) ? sq[nz - mm] : make_double2(0, 0);
                        ar += d0.x;
                        ai += d1.x;
                        br += d0.y;
                        bi += d1.y;
                    }
                    if (mm == 0 || mm == nm - 1) {      // modes 0 and Nz/2 are real
                        ai = 0.0;
                        bi = 0.0;
                    }
                    z = make_double2(ar - bi, ai + br);     // U_a + i U_b at m
                    zc = make_double2(ar + bi, br - ai);    // conj U_a + i conj U_b at Nz - m
                }
                sq[mm] = z;
                if (mm > 0 && 2 * mm < nz) sq[nz - mm] = zc;
            }
        }
    }
    __syncthreads();
    // 2. stages of half length Nz/2 .. 4; in groups of 1024 threads (one per CU, nothing
    //    else to cover the transform's latency) with the old values of u and the means for
    //    the first LV items of each thread already on their way (long lines: 3.2 against
    //    3.4 ms; 256-thread groups, four per CU, load them after the transform)
    constexpr bool early = NTH >= 1024;
    const double scale = 1.0 / nz;
    const int nq = nz >> 2;
    const int nitem = nseq * nq;
    constexpr int LV = 2;
    double oa[LV][4], ob[LV][4], ma[LV], mb[LV];
    auto load_old = [&](int t0) {
#pragma unroll
        for (int k = 0; k < LV; ++k) {
            const int t = t0 + k * NTH;
            const int trr = t % tr, rest = t / tr;
            const int g = rest % nq, pj = rest / nq;
            const int row = row0 + trr;
            const int ra = 8 * tile + 2 * (pair0 + pj);
            const bool live = t < nitem && row < M;
            ma[k] = (mu && live && ra < R) ? mu[ra * 3 + row % 3] : 0.0;
            mb[k] = (mu && live && ra + 1 < R) ? mu[(ra + 1) * 3 + row % 3] : 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                oa[k][e] = ob[k][e] = 0.0;
                if (read_u && t < nitem && row < M) {
                    const int n0 = (int)bitrev(4 * g + e, logn);
                    if (ra < R) oa[k][e] = u[((int64_t)ra * nz + n0) * M + row];
                    if (ra + 1 < R) ob[k][e] = u[((int64_t)(ra + 1) * nz + n0) * M + row];
                }
            }
        }
    };
    if (early) load_old(threadIdx.x);
    lds_fft_dif_s<true>(lds, nseq, ss, logn, 2, tw);
    // 3. last two stages in registers, then the update; with per-RHS step factors alpha_d
    //    (one RHS pair per group then) the group's largest |w| per RHS goes to wmax_part
    const double2 w0 = twid<true>(tw, 0), w1 = twid<true>(tw, nz >> 2);
    double mxw[2] = {0.0, 0.0};
    for (int t0 = threadIdx.x; t0 < nitem; t0 += NTH * LV) {
        if (!early || t0 != (int)threadIdx.x) load_old(t0);
#pragma unroll
        for (int k = 0; k < LV; ++k) {
            const int t = t0 + k * NTH;
            if (t >= nitem) break;
            const int trr = t % tr, rest = t / tr;
            const int g = rest % nq, pj = rest / nq;
            const int row = row0 + trr;
            if (row >= M) continue;
            const int ra = 8 * tile + 2 * (pair0 + pj);
            const double2* sq = lds + (pj * tr + trr) * ss + 4 * g;
            double2 x0 = sq[0], x1 = sq[1], x2 = sq[2], x3 = sq[3];
            dif(x0, x2, w0);
            dif(x1, x3, w1);
            dif(x0, x1, w0);
            dif(x2, x3, w0);
            const double2 xv[4] = {x0, x1, x2, x3};
            const double aa = (alpha_d && ra < R) ? alpha_d[ra] : alpha;
            const double ab = (alpha_d && ra + 1 < R) ? alpha_d[ra + 1] : alpha;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int n0 = (int)bitrev(4 * g + e, logn);
                const double wa = xv[e].x * scale, wb = xv[e].y * scale;
                if (wmax_part) {
                    mxw[0] = fmax(mxw[0], fabs(wa));
                    mxw[1] = fmax(mxw[1], fabs(wb));
                }
                if (ra < R) {
                    const double x = oa[k][e] - aa * wa;
                    u[((int64_t)ra * nz + n0) * M + row] = mu ? x - ma[k] : x;
                }
                if (ra + 1 < R) {
                    const double x = ob[k][e] - ab * wb;
                    u[((int64_t)(ra + 1) * nz + n0) * M + row] = mu ? x - mb[k] : x;
                }
            }
        }
    }
    if (wmax_part) {
        __syncthreads();                     // the transform buffer is free again
        block_max<2, NTH>(mxw, (double*)lds);
        const int ra = 8 * tile + 2 * pair0;
        if (threadIdx.x == 0 && ra < R) wmax_part[(int64_t)ra * n_rg + rg] = mxw[0];
        if (threadIdx.x == 0 && ra + 1 < R) wmax_part[(int64_t)(ra + 1) * n_rg + rg] = mxw[1];
    }
}

// Shape of the fused update's work groups: 8 rows (64-byte runs of u; 33 KiB of LDS at
// Nz = 256) x one RHS pair.  Measured on MI355X (medium and large workloads, autotuned
// lists): 8 rows beat 4 (fewer groups in flight are not the limit; the read amplification
// of 32-byte runs is) and match or beat 16 (half the groups per CU); one pair per group,
// the pair groups sharing the product records through L2, beats two or four pairs per
// group.  Lines of 512 and 1024 layers keep the 8 rows (66 and 131 KiB of LDS) with 1024
// threads per group (sixteen waves on the CU it fills): on the long workload 2.8-3.4 ms
// against 4.3 ms for the inverse transform into w and the transpose-update, where 256
// threads took 3.9-4.4 ms, 4 or 2 rows 4.2-7.9 ms, and 4 rows with 512 or 1024 threads (two
// groups per CU) 4.2-5.1 ms; at Nz = 256, 1024 or 512 threads are 9-40 % slower than 256.  Returns false outside 16 <= Nz <= 1024: the update then
// goes through the w scratch and the tiled transpose.
static int update_groups(int tr, int pp, int M, int ct_grid) {
    return xcd_groups(ct_grid * ((M + tr - 1) / tr), 4 / pp);
}

bool update_shape(int nz, int M, int ct_grid, int* tr, int* pp) {
    (void)M;
    (void)ct_grid;
    *pp = 1;
    *tr = 8;
    return nz >= 16 && nz <= 1024;
}

void launch_irfft_update(hipStream_t st, const double* c, double* u, int R, int nz, int mp, int M,
                         int ct_grid, const double2* tw, int nsplit, int64_t split_stride,
                         const double2* rowmean, const double2* shat, const int* shat_on,
                         const unsigned long long* amax, const int* bexp, double alpha,
                         const double* mu, int read_u, const int* status, const double* alpha_d,
                         double* wmax_part) {
    int logn = 0;
    while ((1 << logn) < nz) ++logn;
    int tr, pp;
    update_shape(nz, M, ct_grid, &tr, &pp);
    if (pp != 1) wmax_part = nullptr;        // the group's maxima are per RHS pair (never taken)
    const int n_rg = (M + tr - 1) / tr;
    const int n_units = ct_grid * n_rg;
    const int nblk = update_groups(tr, pp, M, ct_grid);
    size_t lds = (size_t)tr * pp * (nz + 1) * sizeof(double2);
    // the maxima of |w| are reduced in the same LDS: 2 values per thread
    const size_t lds_max = 2 * (size_t)(nz > 256 ? 1024 : NT) * sizeof(double);
    if (wmax_part && lds < lds_max) lds = lds_max;
    // lines of 512 and 1024 layers: 1024 threads per work group (one group per CU with its
    // 66-131 KiB of LDS), 256 below
#define UPD_CASE(NS) do {                                                                              \
    if (nz > 256) {                                                                                   \
        hipLaunchKernelGGL((k_irfft_update<NS, 1024>), dim3(nblk), dim3(1024), lds, st, c, u, R, nz, logn, mp, \
                           M, tr, pp, n_rg, n_units, tw, nsplit, split_stride, rowmean, shat, shat_on, amax, \
                           bexp, alpha, alpha_d, mu, read_u, wmax_part, status);                      \
    } else {                                                                                          \
        hipLaunchKernelGGL((k_irfft_update<NS, NT>), dim3(nblk), dim3(NT), lds, st, c, u, R, nz, logn, mp, M, \
                           tr, pp, n_rg, n_units, tw, nsplit, split_stride, rowmean, shat, shat_on, amax, \
                           bexp, alpha, alpha_d, mu, read_u, wmax_part, status);                      \
    }                                                                                                 \
} while (0)
    if (nsplit <= 1) UPD_CASE(1);
    else if (nsplit <= 2) UPD_CASE(2);
    else if (nsplit <= 4) UPD_CASE(4);
    else UPD_CASE(8);
#undef UPD_CASE
}

// ----------------------------------------------------------------------------------
// Mean of the updated pad displacement, before the update is written:
//   mean(u - alpha w) = (sum u - alpha sum w) / (Nz n_b)   per RHS and component,
// where sum_n0 w[row][n0] is the line mode 0 of the row (the inverse transform's
// constant term), so sum w needs only the mode-0 records.  k_mean_parts: partial sums
// of u and of the mode-0 values over a fixed partition (nbr blocks per RHS);
// k_update_mean: one block per RHS adds the partials in fixed order.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_mean_parts(const double* __restrict__ u, const double* __restrict__ c,
                                                   int64_t per_rhs, int nbr, int R, int nz, int mp, int M,
                                                   int nsplit, int64_t split_stride,
                                                   const double2* __restrict__ rowmean,
                                                   const double2* __restrict__ shat,
        const int* __restrict__ shat_on,
                                                   const unsigned long long* __restrict__ amax,
                                                   const int* __restrict__ bexp,
                                                   double* __restrict__ part,
                                                   const int* __restrict__ status) {
    __shared__ double red[6 * NT];
    if (status && *status) return;
    const int r = blockIdx.y, b = blockIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};     // sum u (3), sum w (3)
    {
        const int64_t len = (per_rhs + nbr - 1) / nbr;
        const int64_t e0 = (int64_t)b * len, e1 = std::min(per_rhs, e0 + len);
        const double* ur = u + (int64_t)r * per_rhs;
        constexpr int LU = 4;
        for (int64_t i0 = e0 + threadIdx.x; i0 < e1; i0 += (int64_t)NT * LU) {
            double x[LU];
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                const int64_t i = i0 + (int64_t)k * NT;
                x[k] = i < e1 ? ur[i] : 0.0;
            }
            // component (n0 M + row) % 3 = i % 3; NT % 3 = 1, so it advances by one per k
            static_assert(NT % 3 == 1, "component stepping assumes NT = 1 mod 3");
            const int c0 = (int)(i0 % 3);
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                const int64_t i = i0 + (int64_t)k * NT;
                if (i < e1) v[(c0 + k) % 3] += x[k];
            }
        }
    }
    {
        const int tile = r >> 3, ja = (r & 7) & ~1, odd = r & 1;
        const int nm = (nz >> 1) + 1;
        const int lr = (M + nbr - 1) / nbr;
        const int r1 = std::min(M, (b + 1) * lr);
        for (int row = b * lr + threadIdx.x; row < r1; row += NT) {
            const double* src = c + ((int64_t)tile * mp + row) * nm * 16;
            double ar, br, ai, bi;
            mode_value(*(const double2*)(src + ja), *(const double2*)(src + ja + 8), src, ja, nsplit,
                       split_stride, 0, row, M, nm, 8 * tile + ja, R, rowmean, shat, shat_on, amax, bexp, ar,
                       br, ai, bi);
            v[3 + row % 3] += odd ? br : ar;
        }
    }
    block_sum<6>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) part[((int64_t)r * nbr + b) * 6 + k] = v[k];
}

int mean_blocks(int64_t per_rhs) {
    const int64_t b = (per_rhs + (int64_t)NT * 32 - 1) / ((int64_t)NT * 32);
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, b));
}

__global__ void __launch_bounds__(NT) k_update_mean(const double* __restrict__ part, int nbr, int nz, int n_b,
                                                    double alpha, const double* __restrict__ alpha_d,
                                                    double* __restrict__ mu,
                                                    const int* __restrict__ status) {
    __shared__ double red[6 * NT];
    if (status && *status) return;
    const int r = blockIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nbr; b += NT)
        for (int k = 0; k < 6; ++k) v[k] += part[((int64_t)r * nbr + b) * 6 + k];
    block_sum<6>(v, red);
    if (threadIdx.x == 0) {
        const double inv_n = 1.0 / ((double)nz * n_b);
        const double a = alpha_d ? alpha_d[r] : alpha;
        for (int cc = 0; cc < 3; ++cc) mu[r * 3 + cc] = (v[cc] - a * v[3 + cc]) * inv_n;
    }
}

void launch_update_mean(hipStream_t st, const double* u, const double* c, double* part, int R, int nz,
                        int mp, int M, int nsplit, int64_t split_stride, const double2* rowmean,
                        const double2* shat, const int* shat_on, const unsigned long long* amax,
                        const int* bexp, double alpha, double* mu, const int* status,
                        const double* alpha_d) {
    const int64_t per_rhs = (int64_t)nz * M;
    const int nbr = mean_blocks(per_rhs);
    hipLaunchKernelGGL(k_mean_parts, dim3(nbr, R), dim3(NT), 0, st, u, c, per_rhs, nbr, R, nz, mp, M, nsplit,
                       split_stride, rowmean, shat, shat_on, amax, bexp, part, status);
    hipLaunchKernelGGL(k_update_mean, dim3(R), dim3(NT), 0, st, part, nbr, nz, M / 3, alpha, alpha_d, mu, status);
}

// ----------------------------------------------------------------------------------
// u[r][n0][row] -= alpha_r * w[r][row][n0] (+ mu[r][row % 3] when mu is given: the mean
// of the result, known beforehand) by a tiled transpose through LDS: tiles of 64 rows x
// 32 layers, 16-byte accesses along the contiguous axis of each array (two rows of a
// layer of u, two layers of a row of w per thread) where the arrays allow; the old values
// of u are loaded before the tile of w.  Skipped entirely when a data check has latched an
// error.
// ----------------------------------------------------------------------------------
#define AX_TR 64
#define AX_TN 32

__global__ void __launch_bounds__(NT) k_axpy(const double* __restrict__ w, double* __restrict__ u, int nz,
                                             int M, double alpha, const double* __restrict__ alpha_d,
                                             const double* __restrict__ mu, int vec,
                                             const int* __restrict__ status) {
    __shared__ double tile[AX_TR][AX_TN + 1];
    if (status && *status) return;
    const int r = blockIdx.z;
    const int row0 = blockIdx.x * AX_TR, n00 = blockIdx.y * AX_TN;
    const double a = alpha_d ? alpha_d[r] : alpha;
    const double* wr = w + (int64_t)r * M * nz;
    double* ur = u + (int64_t)r * nz * M;
    double m3[3] = {0.0, 0.0, 0.0};
    if (mu)
        for (int cc = 0; cc < 3; ++cc) m3[cc] = mu[r * 3 + cc];
    // old u: rows 2 tx, 2 tx + 1 of layers ty + 8 k
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int row = row0 + 2 * tx;
    double uo[4][2];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int n0 = n00 + ty + 8 * k;
        uo[k][0] = uo[k][1] = 0.0;
        if (n0 < nz) {
            const double* p = ur + (int64_t)n0 * M + row;
            if (vec && row + 1 < M) {
                const double2 x = *(const double2*)p;
                uo[k][0] = x.x;
                uo[k][1] = x.y;
            } else {
                if (row < M) uo[k][0] = p[0];
                if (row + 1 < M) uo[k][1] = p[1];
            }
        }
    }
    // w: layers 2 sx, 2 sx + 1 of rows sy + 16 k
    {
        const int sx = threadIdx.x & 15, sy = threadIdx.x >> 4;
        const int n0 = n00 + 2 * sx;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int rr = row0 + sy + 16 * k;
            double x0 = 0.0, x1 = 0.0;
            if (rr < M) {
                const double* p = wr + (int64_t)rr * nz + n0;
                if (vec && n0 + 1 < nz) {
                    const double2 x = *(const double2*)p;
                    x0 = x.x;
                    x1 = x.y;
                } else {
                    if (n0 < nz) x0 = p[0];
                    if (n0 + 1 < nz) x1 = p[1];
                }
            }
            tile[sy + 16 * k][2 * sx] = x0;
            tile[sy + 16 * k][2 * sx + 1] = x1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int n0 = n00 + ty + 8 * k;
        if (n0 >= nz) continue;
        double x[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int rr = row + e;
            x[e] = uo[k][e] - a * tile[2 * tx + e][ty + 8 * k];
            if (mu) x[e] -= m3[rr % 3];
        }
        double* p = ur + (int64_t)n0 * M + row;
        if (vec && row + 1 < M) {
            *(double2*)p = make_double2(x[0], x[1]);
        } else {
            if (row < M) p[0] = x[0];
            if (row + 1 < M) p[1] = x[1];
        }
    }
}

void launch_axpy(hipStream_t st, const double* w, double* u, int R, int nz, int M, double alpha,
                 const double* alpha_d, const int* status, const double* mu) {
    dim3 grid((M + AX_TR - 1) / AX_TR, (nz + AX_TN - 1) / AX_TN, R);
    // 16-byte accesses: every row pair of u and layer pair of w starts 16-byte aligned
    const int vec = ((M & 1) == 0 && (nz & 1) == 0 && ((uintptr_t)u & 15) == 0 && ((uintptr_t)w & 15) == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_axpy, grid, dim3(NT), 0, st, w, u, nz, M, alpha, alpha_d, mu, vec, status);
}

// ----------------------------------------------------------------------------------
// Relax (Algorithm 2) on raw residuals, per RHS.  Stage 1: block partials of
// <f_k, f_{k+1} - f_k>, ||f_{k+1} - f_k||^2 and ||f_{k+1}||_inf.  Stage 2: one block per
// RHS reduces them in fixed order and sets alpha_{k+1} (alpha = 1 before the third
// iteration or without relaxation; alpha < 0 -> 1; zero denominator keeps alpha_k).
// The iteration index k lives in device memory (kdev), read by the kernels and advanced
// by the last one, so a step captured into a graph replays with the current k.
// ----------------------------------------------------------------------------------
__device__ inline int relax_on(const int* __restrict__ kdev, int relax) { return (relax && *kdev >= 2) ? 1 : 0; }
#define RELAX_PARTS 64
__global__ void __launch_bounds__(NT) k_relax_part(const double* __restrict__ fnew, double* fprev,
                                                   double* __restrict__ part, int64_t per_rhs,
                                                   const int* __restrict__ kdev, int relax) {
    __shared__ double red[3 * NT];
    const int use_prev = relax_on(kdev, relax);
    const int r = blockIdx.y;
    const double* a = fnew + (int64_t)r * per_rhs;
    double* b = fprev + (int64_t)r * per_rhs;     // f_k read, then f_k+1 kept for the next step
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
        b[e] = x;
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
                                                    double* __restrict__ finf_d, const int* __restrict__ kdev,
                                                    int relax, double alpha_min) {
    __shared__ double red[2 * NT];
    const int use_relax = relax_on(kdev, relax);
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
            if (alpha_min > 0.0) a = fmax(a, alpha_min);   // Remark in Section 2.3.3
        }
        alpha_d[r] = a;
    }
}

void launch_relax_alpha(hipStream_t st, const double* fnew, double* fprev, double* part,
                        double* alpha_d, double* finf_d, int R, int64_t per_rhs, const int* kdev,
                        int relax, double alpha_min) {
    hipLaunchKernelGGL(k_relax_part, dim3(RELAX_PARTS, R), dim3(NT), 0, st, fnew, fprev, part,
                       per_rhs, kdev, relax);
    hipLaunchKernelGGL(k_relax_alpha, dim3(R), dim3(NT), 0, st, part, RELAX_PARTS, alpha_d, finf_d,
                       kdev, relax, alpha_min);
}

// Step bound (the optional bound on the step in Algorithm 2) from the per-block maxima of |w|.
__global__ void __launch_bounds__(NT) k_relax_clamp(const double* __restrict__ wmax_part,
                                                    int n_part, double* __restrict__ alpha_d,
                                                    double* __restrict__ stepinf_d, double du_max,
                                                    const int* __restrict__ kdev, int relax) {
    __shared__ double red[NT];
    const int use_bound = relax_on(kdev, relax);
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
                        double* stepinf_d, int R, double du_max, const int* kdev, int relax) {
    hipLaunchKernelGGL(k_relax_clamp, dim3(R), dim3(NT), 0, st, wmax_part, n_part, alpha_d,
                       stepinf_d, du_max, kdev, relax);
}

__global__ void k_relax_out(const double* __restrict__ alpha_d, const double* __restrict__ finf_d,
                            const double* __restrict__ stepinf_d, const double* __restrict__ mean_d,
                            fbc_relax_out* __restrict__ out, int R, const int* __restrict__ kdev,
                            double tol_f) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = *kdev;
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

// kdev[0] <- v (v >= 0), or kdev[0] + 1 (v < 0): the iteration index of the relaxation.
__global__ void k_relax_index(int* __restrict__ kdev, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) kdev[0] = v >= 0 ? v : kdev[0] + 1;
}

void launch_relax_index(hipStream_t st, int* kdev, int v) {
    hipLaunchKernelGGL(k_relax_index, dim3(1), dim3(64), 0, st, kdev, v);
}

void launch_relax_finish(hipStream_t st, const double* alpha_d, const double* finf_d, const double* stepinf_d,
                         const double* mean_d, fbc_relax_out* out, int R, int* kdev, double tol_f) {
    if (out)
        hipLaunchKernelGGL(k_relax_out, dim3((R + 63) / 64), dim3(64), 0, st, alpha_d, finf_d,
                           stepinf_d, mean_d, out, R, kdev, tol_f);
    launch_relax_index(st, kdev, -1);     // after every reader of k in this step
}

__global__ void k_fill(double* p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        p[i] = v;
}

void launch_fill(hipStream_t st, double* p, int64_t n, double v) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill, dim3((unsigned)grid_blocks(n)), dim3(NT), 0, st, p, n, v);
}

// The 1024-thread forms of the forward transform and of the fused update take more than
// the default 64 KiB of dynamic LDS: raise their limit to the CU's 160 KiB once, at context
// creation (not in a launch path, which may be under stream capture).
void apply_kernels_init() {
    static std::mutex mu;
    static std::set<int> done;               // devices whose limits are set
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(mu);
    if (!done.insert(dev).second) return;
    {
        const int lim = 160 * 1024;
        (void)hipFuncSetAttribute((const void*)k_line_rfft<FBC_FORM_FP64, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)k_line_rfft<FBC_FORM_FP32, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)k_line_rfft<FBC_FORM_SPLIT_BF16, 1024>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)k_line_rfft<FBC_FORM_SPLIT_FP16, 1024>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)k_irfft_update<1, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)k_irfft_update<2, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)k_irfft_update<4, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)k_irfft_update<8, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipGetLastError();
    }
}
