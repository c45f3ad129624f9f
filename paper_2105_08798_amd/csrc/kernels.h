// Kernel launch wrappers of the FBC library (all enqueue on `st`, no synchronisation).
#pragma once
#include "common.h"

struct BondTable {
    int n[12][3];        // primitive-basis offsets of the 12 nearest-neighbour bonds
    double p[12][6];     // k * Rhat Rhat^T in symmetric order xx yy zz xy xz yz
};

// ---- assembly (Appendix B, discrete Brillouin-zone sum) ----
void launch_dinv(hipStream_t st, double2* pk, int m0, int nmc, int nz, int m1, int m2,
                 int logL, const double* sn, const BondTable& bt);
void launch_fft_rows(hipStream_t st, double2* data, int64_t nrows, int logn, const double2* tw,
                     bool inverse);
void launch_transpose_c(hipStream_t st, const double2* in, double2* out, int batches, int rows,
                        int cols);
void launch_gather_table(hipStream_t st, const double2* t, double2* tab, int nmc, int m1, int m2,
                         int64_t n_off, const int32_t* off_d1, const int32_t* off_d2,
                         int64_t tab_mode_stride, double scale);
// Table modes are on the finest line grid of the context: cell mode m reads table mode
// m * mode_mult.
void launch_rowmean(hipStream_t st, const double2* tab, double2* rowmean, int nm, int mode_mult,
                    int64_t n_off, int n_b, int n_i, const int32_t* cols_b, const int32_t* cols_i,
                    const int32_t* lut, int d1min, int d2min, int w2);
// Per table mode: largest magnitude (amax) and the distance beyond which every block is
// below tau * amax (rhocut); both as bit patterns of non-negative doubles.
void launch_tab_rhocut(hipStream_t st, const double2* tab, int T, int64_t n_off, const int32_t* d1,
                       const int32_t* d2, double tau, unsigned long long* amax,
                       unsigned long long* rhocut);
// Compact dense store of one cell (chunk-tiles of the negligible-block windows; see
// k_build_dense): reg_pre [nm * n_tiles + 1] (prefix sums of the window lengths, in
// chunk-tiles) and win_start [nm * n_tiles] on the device; n_ct = reg_pre[last].
void launch_build_dense(hipStream_t st, int form, void* store, const double2* tab,
                        const double2* rowmean, const int64_t* reg_pre, const int32_t* win_start,
                        int nm, int n_tiles, int n_chunks, int tile_rows, int64_t n_ct, int mode_mult,
                        int64_t n_off, int n_b, int n_i, const int32_t* cols_b, const int32_t* cols_i,
                        const int32_t* lut, int d1min, int d2min, int w2, unsigned long long* amax);

// ---- apply (Section 2.3.2 update in line-mode form) ----
// Per-layer sums sums[r][n0][6] (net force, absolute force), cell totals tot[r][3] with
// the net-force check, and (shat != NULL) the line transform of the per-layer net force.
void launch_netforce(hipStream_t st, const double* f, double* sums, double* tot, double2* shat,
                     int* shat_on, int R, int nz, int n_i, double tol, int check, int project,
                     const double2* tw, int* bexp, int* status);
void launch_line_rfft(hipStream_t st, int form, const double* f, const double* tot, int project,
                      void* bfrag, int R, int nz, int n_i, int kp, int ct, const double2* tw,
                      const int* bexp);
// variant: one of gemm_variants(form, ctmax) kernel instantiations (bitwise the same result)
void launch_gemm(hipStream_t st, int form, const GemmJob* jobs, int njobs, int ctmax,
                 const void* a, const void* b, double* c,
                 const PqLists* q, int variant);   // q != NULL: persistent work-queue kernel on these lists
int gemm_variants(int form, int ctmax);
std::string gemm_shape(int form, int ctmax, int variant);
// Offset-table form: 32 pad columns x all interface columns per work group, table
// entries gathered into LDS in MFMA fragment order.
void launch_gemm_dtab(hipStream_t st, const GemmJob* jobs, int njobs, int ct, const double2* tab,
                      int64_t a_base, const double* b, double* c, const CellDev* cells,
                      const int32_t* lut, int d1min, int d2min, int w2, const int32_t* need,
                      int64_t n_off, const PqLists* q, int mixed = 0);   // q != NULL: persistent work-queue kernel
// H-matrix product step (hmat.hip): B fragments of one FP64 cell in, product records out
void hmat_enqueue_pipeline(fbc_hmat* h, const double* bfrag, int64_t bf_mode, int kp, double* rec, int mp, int nm,
                           int ct, hipStream_t st);
const fbc_ctx* hmat_context(const fbc_hmat* h);
void irfft_shape(int nz, int* tr, int* pp);
void launch_line_irfft(hipStream_t st, const double* c, double* w, double* wmax_part, int R,
                       int nz, int mp, int M, int ct, int ct_grid, const double2* tw, int nsplit,
                       int64_t split_stride, const double2* rowmean, const double2* shat,
                       const int* shat_on, const unsigned long long* amax, const int* bexp,
                       int* n_part_out);
// Raises the dynamic-LDS limit of the 1024-thread line-transform kernels on the current
// device (once per device; call outside stream capture, e.g. at context creation).
void apply_kernels_init();
// u <- u - alpha_r w - mu_r (mu optional) through a tiled transpose
void launch_axpy(hipStream_t st, const double* w, double* u, int R, int nz, int M, double alpha,
                 const double* alpha_d, const int* status, const double* mu);
// fused inverse transform + update (fbc_apply, fbc_green_apply, the relaxation step without
// a step bound), and the mean it removes; update_shape is false where the line is too long
// for the fused kernel.  alpha_d: per-RHS step factors on the device (else alpha);
// wmax_part: per RHS and row group (ceil(M / tr) of them) the largest |w|, or NULL.
bool update_shape(int nz, int M, int ct_grid, int* tr, int* pp);
void launch_irfft_update(hipStream_t st, const double* c, double* u, int R, int nz, int mp, int M,
                         int ct_grid, const double2* tw, int nsplit, int64_t split_stride,
                         const double2* rowmean, const double2* shat, const int* shat_on,
                         const unsigned long long* amax, const int* bexp, double alpha,
                         const double* mu, int read_u, const int* status,
                         const double* alpha_d = nullptr, double* wmax_part = nullptr);
int mean_blocks(int64_t per_rhs);
void launch_update_mean(hipStream_t st, const double* u, const double* c, double* part, int R, int nz,
                        int mp, int M, int nsplit, int64_t split_stride, const double2* rowmean,
                        const double2* shat, const int* shat_on, const unsigned long long* amax,
                        const int* bexp, double alpha, double* mu, const int* status,
                        const double* alpha_d = nullptr);

// ---- relax (Section 2.3.3, Algorithm 2); kdev: the iteration index on the device ----
void launch_relax_alpha(hipStream_t st, const double* fnew, double* fprev, double* part,
                        double* alpha_d, double* finf_d, int R, int64_t per_rhs, const int* kdev, int relax,
                        double alpha_min);
void launch_relax_clamp(hipStream_t st, const double* wmax_part, int n_part, double* alpha_d,
                        double* stepinf_d, int R, double du_max, const int* kdev, int relax);
// relaxation output and the index advance; the partials kernel (launch_relax_alpha) keeps
// f_k+1 in fprev for the next step
void launch_relax_finish(hipStream_t st, const double* alpha_d, const double* finf_d, const double* stepinf_d,
                         const double* mean_d, fbc_relax_out* out, int R, int* kdev, double tol_f);
// kdev <- v (v >= 0) or kdev + 1 (v < 0)
void launch_relax_index(hipStream_t st, int* kdev, int v);
void launch_fill(hipStream_t st, double* p, int64_t n, double v);
