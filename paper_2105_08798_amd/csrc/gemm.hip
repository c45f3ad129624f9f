// Per-mode complex products w^(m) = G^(m) f^(m) on MFMA (Section 2.3.2,
// eq. flexbc.up=Gpipl*fipl; Section 3.2, eq. impl.up=Gpipl*fipl_mvm, one dense product
// per line mode).  The complex product is one real product: A[row][k'] holds
// (Re, Im) of G^ interleaved along k', and the B operand holds, per RHS, the two
// columns (Re f, -Im f) and (Im f, Re f), so a 16-column output tile carries the real
// parts of 8 RHS in columns 0..7 and their imaginary parts in columns 8..15.
//
// A is streamed once from HBM in MFMA fragment order (each wave-wide 16-byte load is
// 1 KiB contiguous, no LDS); B fragments are re-read by every row tile of the same
// mode and stay in L2 because the job list gives all tiles of a mode to one XCD.
// Each work group is 4 waves; a wave owns RB row blocks (16 rows each) of one mode and
// all column tiles of that mode, over the whole K.  Loads run PF steps ahead.
#include "kernels.h"

static __device__ inline void store_c_f64(double* __restrict__ c, const GemmJob& jb, int rb,
                                          int ctile, int lane, const d4_t& acc) {
    const int64_t mp = (int64_t)jb.mb * 16;
    const int col = lane & 15;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = 16 * rb + 4 * j + (lane >> 4);      // FP64 16x16x4 output order
        c[jb.c_off + ((int64_t)ctile * mp + row) * 16 + col] = acc[j];
    }
}
static __device__ inline void store_c_f32acc(double* __restrict__ c, const GemmJob& jb, int rb,
                                             int ctile, int lane, const d4_t& acc) {
    const int64_t mp = (int64_t)jb.mb * 16;
    const int col = lane & 15;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = 16 * rb + 4 * (lane >> 4) + j;      // FP32-accumulator output order
        c[jb.c_off + ((int64_t)ctile * mp + row) * 16 + col] = acc[j];
    }
}

// ------------------------------- FP64 ---------------------------------------------
template <int RB, int CTM, int PF>
__global__ void __launch_bounds__(256) k_gemm_f64(const GemmJob* __restrict__ jobs,
                                                  const double* __restrict__ A,
                                                  const double* __restrict__ B,
                                                  double* __restrict__ C) {
    const GemmJob jb = jobs[blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rbw = jb.rb0 + wave * RB;
    if (rbw >= jb.mb) return;
    const int nrb = min(RB, jb.mb - rbw);
    const int nct = jb.ct;
    const int kp8 = jb.kp >> 3;
    const double2* a = (const double2*)(A + jb.a_off) + (int64_t)rbw * kp8 * 64 + lane;
    const double2* b = (const double2*)(B + jb.b_off) + lane;
    d4_t acc[RB][CTM];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CTM; ++c) acc[r][c] = (d4_t){0, 0, 0, 0};
    double2 ab[PF][RB], bb[PF][CTM];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
            ab[u][r] = (r < nrb && u < kp8) ? a[((int64_t)r * kp8 + u) * 64] : make_double2(0, 0);
#pragma unroll
        for (int c = 0; c < CTM; ++c)
            bb[u][c] = (c < nct && u < kp8) ? b[((int64_t)c * kp8 + u) * 64] : make_double2(0, 0);
    }
    for (int p0 = 0; p0 < kp8; p0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const double2* av = ab[u];
            const double2* bv = bb[u];
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CTM; ++c) {
                    if (r < nrb && c < nct && p0 + u < kp8) {
                        acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r].x, bv[c].x, acc[r][c], 0, 0, 0);
                        acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r].y, bv[c].y, acc[r][c], 0, 0, 0);
                    }
                }
            const int pn = p0 + u + PF;
            if (pn < kp8) {
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    if (r < nrb) ab[u][r] = a[((int64_t)r * kp8 + pn) * 64];
#pragma unroll
                for (int c = 0; c < CTM; ++c)
                    if (c < nct) bb[u][c] = b[((int64_t)c * kp8 + pn) * 64];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CTM; ++c)
            if (r < nrb && c < nct) store_c_f64(C, jb, rbw + r, c, lane, acc[r][c]);
}

// ------------------------------- FP32 ---------------------------------------------
// FP32 MFMA with FP32 accumulation inside chunks of KCH*16 real k, FP64 across chunks.
template <int RB, int CTM, int PF, int KCH>
__global__ void __launch_bounds__(256) k_gemm_f32(const GemmJob* __restrict__ jobs,
                                                  const float* __restrict__ A,
                                                  const float* __restrict__ B,
                                                  double* __restrict__ C) {
    const GemmJob jb = jobs[blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rbw = jb.rb0 + wave * RB;
    if (rbw >= jb.mb) return;
    const int nrb = min(RB, jb.mb - rbw);
    const int nct = jb.ct;
    const int kq = jb.kp >> 4;
    const float4* a = (const float4*)(A + jb.a_off) + (int64_t)rbw * kq * 64 + lane;
    const float4* b = (const float4*)(B + jb.b_off) + lane;
    d4_t acc[RB][CTM];
    f4_t ac32[RB][CTM];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CTM; ++c) {
            acc[r][c] = (d4_t){0, 0, 0, 0};
            ac32[r][c] = (f4_t){0, 0, 0, 0};
        }
    float4 ab[PF][RB], bb[PF][CTM];
    const float4 z4 = make_float4(0, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < PF; ++u) {
#pragma unroll
        for (int r = 0; r < RB; ++r) ab[u][r] = (r < nrb && u < kq) ? a[((int64_t)r * kq + u) * 64] : z4;
#pragma unroll
        for (int c = 0; c < CTM; ++c) bb[u][c] = (c < nct && u < kq) ? b[((int64_t)c * kq + u) * 64] : z4;
    }
    for (int q0 = 0; q0 < kq; q0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CTM; ++c) {
                    if (r < nrb && c < nct && q0 + u < kq) {
                        f4_t t = ac32[r][c];
                        t = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[u][r].x, bb[u][c].x, t, 0, 0, 0);
                        t = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[u][r].y, bb[u][c].y, t, 0, 0, 0);
                        t = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[u][r].z, bb[u][c].z, t, 0, 0, 0);
                        t = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[u][r].w, bb[u][c].w, t, 0, 0, 0);
                        ac32[r][c] = t;
                    }
                }
            const int qn = q0 + u + PF;
            if (qn < kq) {
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    if (r < nrb) ab[u][r] = a[((int64_t)r * kq + qn) * 64];
#pragma unroll
                for (int c = 0; c < CTM; ++c)
                    if (c < nct) bb[u][c] = b[((int64_t)c * kq + qn) * 64];
            }
        }
        if (((q0 + PF) % KCH) == 0 || q0 + PF >= kq) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CTM; ++c) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[r][c][j] += (double)ac32[r][c][j];
                    ac32[r][c] = (f4_t){0, 0, 0, 0};
                }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CTM; ++c)
            if (r < nrb && c < nct) store_c_f32acc(C, jb, rbw + r, c, lane, acc[r][c]);
}

// ------------------------------- split BF16 ---------------------------------------
// G ~ G_hi + G_lo, f ~ f_hi + f_lo; products hi*hi + hi*lo + lo*hi on BF16 MFMA with
// FP32 accumulation inside chunks of KCH*32 real k, FP64 across chunks.
template <int RB, int CTM, int PF, int KCH>
__global__ void __launch_bounds__(256) k_gemm_bf16(const GemmJob* __restrict__ jobs,
                                                   const unsigned short* __restrict__ A,
                                                   const unsigned short* __restrict__ B,
                                                   double* __restrict__ C) {
    const GemmJob jb = jobs[blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rbw = jb.rb0 + wave * RB;
    if (rbw >= jb.mb) return;
    const int nrb = min(RB, jb.mb - rbw);
    const int nct = jb.ct;
    const int kt = jb.kp >> 5;
    // 16-byte units: per (block, t): hi run of 64 units then lo run of 64 units
    const bf8_t* a = (const bf8_t*)(A + jb.a_off) + (int64_t)rbw * kt * 128 + lane;
    const bf8_t* b = (const bf8_t*)(B + jb.b_off) + lane;
    d4_t acc[RB][CTM];
    f4_t ac32[RB][CTM];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CTM; ++c) {
            acc[r][c] = (d4_t){0, 0, 0, 0};
            ac32[r][c] = (f4_t){0, 0, 0, 0};
        }
    bf8_t ah[PF][RB], al[PF][RB], bh[PF][CTM], bl[PF][CTM];
    bf8_t zb;
#pragma unroll
    for (int j = 0; j < 8; ++j) zb[j] = (__bf16)0.0f;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            ah[u][r] = (r < nrb && u < kt) ? a[((int64_t)r * kt + u) * 128] : zb;
            al[u][r] = (r < nrb && u < kt) ? a[((int64_t)r * kt + u) * 128 + 64] : zb;
        }
#pragma unroll
        for (int c = 0; c < CTM; ++c) {
            bh[u][c] = (c < nct && u < kt) ? b[((int64_t)c * kt + u) * 128] : zb;
            bl[u][c] = (c < nct && u < kt) ? b[((int64_t)c * kt + u) * 128 + 64] : zb;
        }
    }
    for (int t0 = 0; t0 < kt; t0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CTM; ++c) {
                    if (r < nrb && c < nct && t0 + u < kt) {
                        f4_t t = ac32[r][c];
                        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[u][r], bh[u][c], t, 0, 0, 0);
                        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u][r], bl[u][c], t, 0, 0, 0);
                        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u][r], bh[u][c], t, 0, 0, 0);
                        ac32[r][c] = t;
                    }
                }
            const int tn = t0 + u + PF;
            if (tn < kt) {
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    if (r < nrb) {
                        ah[u][r] = a[((int64_t)r * kt + tn) * 128];
                        al[u][r] = a[((int64_t)r * kt + tn) * 128 + 64];
                    }
#pragma unroll
                for (int c = 0; c < CTM; ++c)
                    if (c < nct) {
                        bh[u][c] = b[((int64_t)c * kt + tn) * 128];
                        bl[u][c] = b[((int64_t)c * kt + tn) * 128 + 64];
                    }
            }
        }
        if (((t0 + PF) % KCH) == 0 || t0 + PF >= kt) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CTM; ++c) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[r][c][j] += (double)ac32[r][c][j];
                    ac32[r][c] = (f4_t){0, 0, 0, 0};
                }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CTM; ++c)
            if (r < nrb && c < nct) store_c_f32acc(C, jb, rbw + r, c, lane, acc[r][c]);
}

// Row blocks per wave for a given column-tile count (register budget per lane).
int gemm_rb(int form, int ctmax) {
    (void)form;
    return ctmax <= 1 ? 4 : (ctmax <= 2 ? 4 : 2);
}

void launch_gemm(hipStream_t st, int form, const GemmJob* jobs, int njobs, int ctmax,
                 const void* a, const void* b, double* c, const double2*, const int32_t* const*,
                 const int32_t* const*, const int32_t*, int, int, int) {
    if (njobs <= 0) return;
    dim3 grid(njobs), blk(256);
#define GEMM_CASE(KERN, RB, CT, ...)                                                           \
    hipLaunchKernelGGL((KERN<RB, CT, __VA_ARGS__>), grid, blk, 0, st, jobs, (const TA*)a,     \
                       (const TA*)b, c)
    if (form == FBC_FORM_FP64) {
        typedef double TA;
        if (ctmax <= 1) GEMM_CASE(k_gemm_f64, 4, 1, 4);
        else if (ctmax <= 2) GEMM_CASE(k_gemm_f64, 4, 2, 4);
        else if (ctmax <= 4) GEMM_CASE(k_gemm_f64, 2, 4, 2);
        else GEMM_CASE(k_gemm_f64, 2, 8, 2);
    } else if (form == FBC_FORM_FP32) {
        typedef float TA;
        if (ctmax <= 1) GEMM_CASE(k_gemm_f32, 4, 1, 4, 16);
        else if (ctmax <= 2) GEMM_CASE(k_gemm_f32, 4, 2, 4, 16);
        else if (ctmax <= 4) GEMM_CASE(k_gemm_f32, 2, 4, 2, 16);
        else GEMM_CASE(k_gemm_f32, 2, 8, 2, 16);
    } else {
        typedef unsigned short TA;
        if (ctmax <= 1) GEMM_CASE(k_gemm_bf16, 4, 1, 2, 8);
        else if (ctmax <= 2) GEMM_CASE(k_gemm_bf16, 4, 2, 2, 8);
        else if (ctmax <= 4) GEMM_CASE(k_gemm_bf16, 2, 4, 2, 8);
        else GEMM_CASE(k_gemm_bf16, 2, 8, 1, 8);
    }
#undef GEMM_CASE
}
