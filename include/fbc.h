/*
 * fbc.h -- C ABI of the line-periodic flexible-boundary-condition (FBC) pad update
 * for MI355X (gfx950).
 *
 * The operation (Section 2.3.2, eq. flexbc.up=Gpipl*fipl, Algorithm 1):
 *     u^p  <-  u^p - alpha * G^{p|i+} [f_in],   then remove the mean pad displacement
 * (eq. mean(u^p)=0), for a cell that is periodic along the dislocation line
 * (Section 2.1).  G^{p|i+} is the Green matrix of the harmonic lattice (Section 3.2,
 * eq. impl.up=Gpipl*fipl_mvm); because the cell is periodic along the line and the
 * entries depend only on the separation, it is block-circulant in the layer index.
 * The library therefore works per line mode m: rFFT of the interface forces along the
 * line, one dense complex product w^(m) = G^(m) f^(m) per mode, inverse rFFT.
 *
 * Lattice and model.  fcc, lattice constant a, nearest-neighbour central springs of
 * stiffness k (the local harmonic model K_h of Section 2.2.1).  Sites are indexed in
 * the primitive basis b0 = a(1/2,-1/2,0) (along the line [1-10]), b1 = a(1/2,0,1/2),
 * b2 = a(1/2,1/2,0): site (n0, n1, n2) is atom column (n1, n2) in layer n0 mod N_z, one
 * atom per column and layer.
 *
 * Green function (Appendix B).  G^(m; dn1, dn2) is the inverse lattice Fourier
 * transform of D(q)^{-1}, D the Fourier symbol of K_h, summed over the discrete
 * Brillouin-zone grid of an M1 x M2 in-plane torus, with the singular q = 0 term
 * dropped (pseudo-inverse gauge: the Green function is unique only up to a constant,
 * Section 3.1).  The block coupling pad column b to interface column i is
 * G^(m; n_b - n_i).  The gauge is a constant 3x3 added to every block of line mode 0
 * (Section 3.1: the Green function is unique up to a constant), so forces whose net
 * force over the whole cell (all interface atoms of all layers) vanishes give a
 * gauge-free result; the check below enforces it, or the projection removes that net
 * force.  Net forces of single layers are allowed (the incompatibility forces of
 * Algorithm 1 have them).
 *
 * Conventions.
 *   f  (interface forces)  : device FP64, per cell [n_rhs][N_z][n_i][3], row-major.
 *   u  (pad displacements)  : device FP64, per cell [n_rhs][N_z][n_b][3], row-major.
 *   Cells are packed back to back in the order given to fbc_assemble_G.
 *   Forward line transform e^{-2 pi i m n0 / N_z}, unnormalised; inverse scaled 1/N_z.
 *   Column sets are host int32 arrays [n][2] of (n1, n2).
 *
 * Ownership.  The caller owns f, u, the relax output buffer and the stream.  The
 * context owns every device buffer it allocates (Green store, tables, scratch) and
 * frees them in fbc_destroy.  Nothing of the caller's is retained across calls.
 *
 * Errors.  Every entry point returns an fbc_status; nothing throws across the ABI.
 * Host-checkable arguments are validated before any device work is enqueued, so a
 * call rejected with FBC_E_ARG / FBC_E_UNSUPPORTED leaves every output untouched.
 * Data-dependent checks (non-finite forces, non-zero net force) run on the device
 * inside the enqueued work: when one fails, the kernels that write u skip their
 * writes (u is left untouched) and the failure is latched in the context; it is
 * returned by fbc_sync_status(), which synchronises the stream.  Device/runtime
 * failures give FBC_E_DEVICE with the HIP error text in fbc_last_error().
 *
 * Threads and streams.  A context may be used by one host thread and one stream at a
 * time; calls that overlap on one context race on its scratch buffers.
 */
#ifndef FBC_H
#define FBC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fbc_ctx fbc_ctx;

typedef enum {
    FBC_OK = 0,
    FBC_E_ARG = -1,          /* invalid argument (null pointer, bad size, bad enum) */
    FBC_E_NOMEM = -2,        /* device allocation failed */
    FBC_E_NETFORCE = -3,     /* |sum f| > netforce_tol * sum |f| for some RHS and component,
                                sums over all interface atoms of all layers of a cell      */
    FBC_E_NONFINITE = -4,    /* NaN or Inf in the forces */
    FBC_E_DEVICE = -5,       /* HIP runtime error (text in fbc_last_error) */
    FBC_E_STATE = -6,        /* call out of order (e.g. relax step before relax begin) */
    FBC_E_UNSUPPORTED = -7   /* valid request outside what the library implements */
} fbc_status;

/* How G^(m) is stored and applied (the per-mode product, Section 3.2 in spectral form). */
typedef enum {
    FBC_FORM_FP64 = 0,        /* dense FP64 complex blocks, FP64 MFMA                        */
    FBC_FORM_FP32 = 1,        /* dense FP32 complex blocks, FP32 MFMA, FP64 across K chunks   */
    FBC_FORM_SPLIT_BF16 = 2,  /* dense split-BF16 (hi+lo) blocks, BF16 MFMA with FP32
                                 accumulation inside K chunks and FP64 across them            */
    FBC_FORM_DTABLE_FP64 = 3, /* no dense store: FP64 table over distinct column offsets
                                 (entries depend on n_b - n_i only), gathered into LDS
                                 tiles and applied on FP64 MFMA                               */
    FBC_FORM_SURROGATE = 4,   /* offset-table product whose table is generated per mode
                                 chunk before each product: exact lattice values (kept,
                                 FP64) near the source, beyond them the continuum Green
                                 function plus a learned correction (Appendix B: exact
                                 near field, continuum far field; bands below); needs
                                 options.surrogate with MLP weights set                    */
    FBC_FORM_SPLIT_FP16 = 5   /* dense split-FP16 blocks, scaled per line mode by a power of
                                 two (hi = fp16(2^e G), lo = fp16(2^e G - hi): 22 bits at the
                                 bytes of split BF16), forces likewise scaled per call, FP16
                                 MFMA with FP32 accumulation inside K chunks, FP64 across  */
} fbc_form;

/* Learned far field (see the fbc_sur_* and fbc_mlp_* calls below). */
typedef struct fbc_sur fbc_sur;
typedef struct fbc_mlp fbc_mlp;

/* Section 2.1 (eq. flexbc.bravais) and Section 2.2.1 (K_h). */
typedef struct {
    double a;          /* lattice constant (> 0); the index-space Green function depends only
                          on bond directions and k, so a enters only the geometry      */
    double spring_k;   /* nearest-neighbour central spring stiffness (> 0) */
} fbc_lattice;

/* One line-periodic cell (Section 2.1: period l3 = N_z a / sqrt 2; Section 2.2.2: the
 * interface set Lambda^{i+} and the pad set Lambda^p, here unions of atom columns). */
typedef struct {
    int nz;                  /* layers along the line, power of two in [2, 4096]          */
    int n_i;                 /* interface columns (>= 1)                                   */
    int n_b;                 /* pad columns (>= 1)                                         */
    int n_rhs;               /* force right-hand sides applied per call, in [1, 65535]     */
    const int32_t* cols_i;   /* host [n_i][2] (n1, n2); copied, not retained               */
    const int32_t* cols_b;   /* host [n_b][2] (n1, n2); copied, not retained               */
} fbc_cell;

typedef struct {
    int form;                /* fbc_form                                                   */
    int bz_m1, bz_m2;        /* in-plane Brillouin-zone torus, powers of two in [8, 4096]  */
    int check_netforce;      /* 1: latch FBC_E_NETFORCE / FBC_E_NONFINITE (device check)   */
    int project_netforce;    /* 1: subtract from f its mean over all interface atoms of all
                                layers (per RHS and component) before applying           */
    double netforce_tol;     /* relative tolerance of the net-force check (e.g. 1e-10)     */
    int row_gauge;           /* reduced forms: store each block row minus its mean over i
                                per mode before rounding; the mean is added back in FP64
                                against sum_i f^_i(m) (exact for any f)                  */
    const fbc_sur* surrogate;/* FBC_FORM_SURROGATE: far-field object (not owned; must
                                outlive the context and keep its MLP weights); else NULL */
    int gen_modes;           /* FBC_FORM_SURROGATE: table modes generated per chunk
                                (>= 0; 0: as many as fit in 4 GiB of scratch)            */
    double skip_tol;         /* negligible blocks: at line mode m the product skips the
                                K chunks of a row tile whose blocks all lie farther than
                                the farthest offset with |G^(m)| >= skip_tol * max |G^(m)|
                                (the line-mode Green function decays with kappa rho).
                                0: default (1e-16 for the FP64 forms, at the rounding
                                of their assembly; 1e-9 for the reduced forms, two orders
                                below their rounding of ~1e-7, and for the surrogate, two
                                orders below its error of ~1e-8, just inside its learned
                                band's end at ~2e-9; there it also ends the generated part
                                of each mode); < 0: none                                  */
    int table_fp32;          /* offset-table forms (FBC_FORM_DTABLE_FP64, FBC_FORM_SURROGATE):
                                1 = the products of the line modes whose far blocks are
                                skipped (skip_tol) on FP32 MFMA -- the gathered FP64 blocks
                                and f^ rounded to FP32, FP32 sums over 8 interface columns,
                                FP64 across them -- and FP64 MFMA at the modes without
                                skipping (mode 0 among them: its long-range part carries
                                the gauge constant); error of the order of the FP32 form's.
                                0 (default) = FP64 MFMA everywhere.  FBC_E_ARG for other
                                values or forms                                           */
} fbc_options;

/* Fills *opt with defaults: FP64, 1024 x 1024 torus, check on, no projection, tol 1e-10,
 * row_gauge on, no surrogate, default skip tolerance. */
void fbc_default_options(fbc_options* opt);

/* Assembles G^(m) for m = 0..N_z/2 of every cell on the device (Appendix B, discrete
 * Brillouin-zone sum in FP64, then the chosen store), and the plan and scratch buffers.
 * Done once per geometry (Section 3.2: built once, reused).  stream: hipStream_t or
 * NULL.  Synchronises the stream before returning.  On success *out owns everything. */
fbc_status fbc_assemble_G(const fbc_lattice* lat, const fbc_cell* cells, int n_cells,
                          const fbc_options* opt, void* stream, fbc_ctx** out);

/* u <- u - alpha * G^{p|i+} f, then per RHS and Cartesian component the mean over all
 * pad atoms of all layers is removed (update step of Algorithm 1).  alpha = -1 with u = 0
 * gives u = G f minus its mean.  f, u: device pointers, packed by cell (see above).
 * Asynchronous on `stream`; data-dependent failures are latched (fbc_sync_status). */
fbc_status fbc_apply(fbc_ctx* ctx, const double* f, double* u, double alpha, void* stream);

/* Same as fbc_apply without the mean removal and with u <- -G f (u overwritten): the
 * raw harmonic response w = G^{p|i+} f (the matrix-vector product of Section 3.2).  When
 * a data check has latched an error, w is not computed (its contents are unspecified). */
fbc_status fbc_green_apply(fbc_ctx* ctx, const double* f, double* w, void* stream);

/* fbc_apply replayed from a HIP graph: the first call with a given (f, u, alpha, stream)
 * captures the whole kernel sequence of fbc_apply into a graph (one launch per update
 * afterwards); a call with other arguments re-captures.  stream must be a created
 * (non-default) stream that is not itself capturing.  Same contract as fbc_apply. */
fbc_status fbc_apply_graph(fbc_ctx* ctx, const double* f, double* u, double alpha, void* stream);

/* Autotuner of the per-mode product launch.  Times every candidate -- the product kernel
 * variants of this context (see fbc_set_kernel_variant) times the work lists: K split
 * into 1, 2, 4, 8 slices (as far as the context's output buffer holds) times the orders:
 * 0 XCD-grouped (all tiles of a mode on one XCD), 1 mode-major, 2 longest-first, 3
 * persistent (jobs longest first, taken from a device work queue by as many work groups
 * as fit on the chip), 4 persistent with one work list per XCD (the row tiles of a mode
 * one after another on one XCD, so their f^ operands are shared in its L2; a group whose
 * list is exhausted helps the others) -- with `reps` fbc_green_apply calls each on this context (input
 * f, device; w, device, same layout as u, is overwritten with G f), times the candidates
 * within 4 % of the fastest again in three interleaved rounds, keeps the one with the
 * fastest whole call over those rounds (the K slices also cost the inverse transform a
 * read each) and reports it in *out (may be NULL).  The surrogate form is refused (FBC_E_UNSUPPORTED):
 * it keeps its mode-major chunks.  Synchronises the stream. */
typedef struct {
    int nsplit;
    int order;
    double gemm_ms;       /* average product time of the chosen list */
    int n_candidates;
    double call_ms;       /* average fbc_green_apply time of the chosen list */
    int variant;          /* product kernel variant (fbc_set_kernel_variant) */
    int from_cache;       /* fbc_autotune_cached: 1 when taken from the cache file, untimed */
} fbc_tune_result;
fbc_status fbc_autotune(fbc_ctx* ctx, const double* f, double* w, int reps, fbc_tune_result* out,
                        void* stream);

/* fbc_autotune with a cache file (text, one line per tuned configuration): when the file
 * holds a result for this context's key -- form, negligible-block tolerance, row gauge,
 * in-plane torus, every cell's line length, column sets and RHS count, the product's column
 * tiles, the device's architecture name and compute-unit count, and the cache format
 * version -- it is applied without timing (from_cache = 1); otherwise the candidates are
 * timed as by fbc_autotune and the result is appended to the file (created if missing).
 * A line whose values fall outside this context's ranges is ignored.  cache_path: host
 * string; FBC_E_ARG if NULL or the file cannot be written. */
fbc_status fbc_autotune_cached(fbc_ctx* ctx, const double* f, double* w, int reps, const char* cache_path,
                               fbc_tune_result* out, void* stream);

/* Selects the product kernel variant: 0 (default) .. n-1, n from fbc_info.n_variants.  The
 * variants share the store layout and the arithmetic order (prefetch-ring depth, K steps
 * per barrier), so results are bitwise those of variant 0.  FBC_E_ARG out of range. */
fbc_status fbc_set_kernel_variant(fbc_ctx* ctx, int variant);

/* Pins the work list of the per-mode product: nsplit K slices (1 .. the context's limit,
 * fbc_info.nsplit after assembly is the default) in the given order (as listed for
 * fbc_autotune; the surrogate form accepts only its mode-major chunks, nsplit 1, with
 * order 1 (one work group per job) or 3 (default: each chunk consumed by the persistent
 * kernel, longest job first)).  Out-of-range values: FBC_E_ARG.  Results do not depend
 * on the order (every order partitions the same products); the number of K slices
 * changes only the rounding (the slices' partial sums are added in fixed order).  A
 * captured update (fbc_apply_graph) is captured again on its next call.  Synchronises
 * the stream. */
fbc_status fbc_set_work_list(fbc_ctx* ctx, int nsplit, int order, void* stream);

/* Residual-based relaxation (Section 2.3.3, eq. alpha, Algorithm 2). */
typedef struct {
    int relax;        /* 1: relax from the third iteration on (Algorithm 1)               */
    double du_max;    /* > 0: bound ||alpha G f||_inf by du_max (Algorithm 2); the bound
                         needs the whole of G f before the update, so a step with it writes
                         G f to a scratch first; <= 0: off, and lines of 16-1024 layers
                         update u straight from the product output                         */
    double tol_f;     /* convergence flag: ||f_in||_inf < tol_f (Section 2.3.3)           */
    double alpha_min; /* > 0: lower bound on alpha_{k+1} (the preprint's variant, Remark in
                         Section 2.3.3), applied after the reset of negative values and
                         before the du_max bound; 0: off                                   */
} fbc_relax_opts;

/* Per RHS, written to device memory by fbc_relax_step (packed over all cells' RHS). */
typedef struct {
    double alpha;            /* alpha_{k+1} used for this update                 */
    double f_inf;            /* ||f_in,k+1||_inf                                  */
    double step_inf;         /* ||alpha G f_in,k+1||_inf                          */
    double mean_removed[3];  /* mean pad displacement removed (per component)     */
    int32_t converged;       /* f_inf < tol_f                                     */
    int32_t k;               /* iteration index k before this step                */
} fbc_relax_out;

/* Resets the iteration: k = 0, alpha = 1 for every RHS. */
fbc_status fbc_relax_begin(fbc_ctx* ctx, const fbc_relax_opts* opts, void* stream);

/* One pass of Algorithm 1 from the relaxation on, given f_in,k+1 (computed by the caller):
 * alpha from Relax on raw residuals (k >= 2), optional step bound, pad update, mean
 * removal.  No host synchronisation.  out_dev: device array [total RHS] or NULL.  The
 * iteration index k is kept in device memory and advanced by the step's last kernel. */
fbc_status fbc_relax_step(fbc_ctx* ctx, const double* f_in, double* u,
                          fbc_relax_out* out_dev, void* stream);

/* fbc_relax_step replayed from a HIP graph (Algorithm 1's update with Algorithm 2 in one
 * launch per iteration): the first call with a given (f_in, u, out_dev, stream) captures
 * the step's kernels, later calls with the same arguments replay them; the kernels read
 * the iteration index from device memory, so every replay takes the current k.  A call
 * with other arguments, fbc_relax_begin, fbc_relax_set_state and a new work list capture
 * again.  stream must be a created (non-default) stream that is not itself capturing.
 * Same contract and results (bitwise) as fbc_relax_step. */
fbc_status fbc_relax_step_graph(fbc_ctx* ctx, const double* f_in, double* u,
                                fbc_relax_out* out_dev, void* stream);

/* Checkpoint and resume of the relaxation (Section 2.3.3): the iteration's state is the
 * options, the index k, alpha_k of every RHS and the previous raw incompatibility forces
 * f_in,k (eq. alpha takes the difference f_in,k+1 - f_in,k).  fbc_relax_get_state copies
 * it out: alpha [total RHS] and f_prev [f elements, the layout of f] are host or device
 * pointers owned by the caller; f_prev holds meaningful values only for k >= 1.
 * fbc_relax_set_state loads a saved state into a context of the same cells (a fresh one
 * after a restart), replacing fbc_relax_begin; f_prev is read only for k > 0 and may be
 * NULL otherwise.  Both synchronise `stream` before they return, so host buffers are
 * complete (get) or may be reused (set).  FBC_E_STATE from get before fbc_relax_begin or
 * set; FBC_E_ARG for NULL pointers, k < 0 or invalid options.  Steps continued from a
 * loaded state are bitwise those of the uninterrupted iteration when both contexts use
 * the same work list (fbc_set_work_list: K slices change the rounding). */
fbc_status fbc_relax_get_state(fbc_ctx* ctx, fbc_relax_opts* opts, int32_t* k, double* alpha,
                               double* f_prev, void* stream);
fbc_status fbc_relax_set_state(fbc_ctx* ctx, const fbc_relax_opts* opts, int32_t k,
                               const double* alpha, const double* f_prev, void* stream);

/* Synchronises `stream`, returns and clears the latched device-side status. */
fbc_status fbc_sync_status(fbc_ctx* ctx, void* stream);

/* Introspection (sizes in bytes of the Green store; per-cell mode counts etc.). */
typedef struct {
    int n_cells;
    int total_rhs;
    int64_t store_bytes;       /* bytes of the G^ store (dense tiles or offset table)     */
    int64_t scratch_bytes;     /* bytes of scratch owned by the context                   */
    int64_t f_elems, u_elems;  /* doubles expected in f and u                             */
    int64_t n_offsets;         /* distinct column offsets over all cells                  */
    int nsplit;                /* K slices of the per-mode product launch                 */
    int job_order;             /* work-list order (see fbc_autotune)                      */
    int n_jobs;                /* work groups of the per-mode product launch              */
    double product_bytes;      /* HBM bytes one product launch must read and write: the
                                  stored blocks of the K chunks it does not skip (dense
                                  forms) or the table (offset forms), plus f^ and w^    */
    double product_flops;      /* real flops of the blocks it does not skip (8 per
                                  complex multiply-add)                                 */
    double skipped_fraction;   /* fraction of the (row, K) block area skipped             */
    int kernel_variant;        /* product kernel variant in use                           */
    int n_variants;            /* variants of this context's product (1 for table forms)  */
    char kernel_shape[96];     /* readable shape of the product kernel in use             */
} fbc_info;
fbc_status fbc_get_info(const fbc_ctx* ctx, fbc_info* info);

/* Copies G^(m) block rows of one cell to host for testing: out[rows][3 n_i] complex
 * (interleaved re, im), rows = 3 * (b1 - b0), for pad columns b0..b1-1 at mode m, as
 * the library stores it (FP64 forms only; reduced forms return FBC_E_UNSUPPORTED). */
fbc_status fbc_copy_block_rows(fbc_ctx* ctx, int cell, int m, int b0, int b1, double* out_host);

/* Kernel timing for measurement.  When enabled, every fbc_apply / fbc_green_apply /
 * fbc_relax_step records a pair of HIP events on `stream` around the launch of the
 * per-mode product kernel (the dominant kernel); up to 4096 pairs are kept.
 * fbc_timing_read synchronises, returns the summed elapsed time in ms and the number
 * of launches timed since the last read, and resets the list. */
fbc_status fbc_timing(fbc_ctx* ctx, int enable);
fbc_status fbc_timing_read(fbc_ctx* ctx, double* gemm_ms_total, int* n_launches);

void fbc_destroy(fbc_ctx* ctx);
const char* fbc_last_error(const fbc_ctx* ctx);

/* ------------------------------------------------------------------------------------
 * Learned far field (Section 3.1 eq. cgf and Appendix B: the lattice Green function is
 * used exactly near the source and replaced by the continuum Green function G_cgf,
 * homogeneous of degree -1, far from it; their difference is a smooth, decaying
 * correction).  In the line-mode representation (theta0 = m / N_z, offset (dn1, dn2),
 * in-plane distance rho, kappa = 2 pi theta0 / c, c = a / sqrt 2):
 *     G_cgf(m; dn) = (1/c) exp(i pi theta0 dn1) G^_K(kappa, r_perp),
 * G^_K the line transform of the anisotropic Kelvin solution of the cubic continuum
 * with C11 = 2k/a, C12 = C44 = k/a (nearest-neighbour springs); m = 0 is regularised by
 * dropping the 2 G_K(t) log(kappa) divergence (a constant gauge).  A surrogate context
 * takes line mode 0 exact for every offset (a table of one mode): the exact Green function
 * lives on the in-plane torus of the context, whose images act on line mode 0 only (they
 * are damped by exp(-kappa L) at m >= 1), and no infinite-plane continuum far field can
 * follow them -- which also makes Appendix B's matching constant unnecessary.  For m >= 1
 * the offsets, sorted by in-plane distance rho, are split into bands by the lattice
 * values themselves (a context computes every mode's exact values once, at creation, to
 * find them; the values fall roughly like exp(-kappa rho), kappa = 2 pi theta0 / c, but
 * more slowly than the continuum's at large theta0):
 *   exact: rho <= r_c, and out to the last block (largest |component|) of at least
 *     exp(-s_exact) times the mode's largest block (default s_exact = 12;
 *     fbc_sur_set_exact_range); stored per mode as a ragged prefix;
 *   learned: out to the last block of at least exp(-s_learn) times the largest (default
 *     s_learn = 20; fbc_sur_set_learn_range): continuum plus the learned correction
 *       G_lgf - G_cgf = env * exp(i pi theta0 dn1) * MLP(features),
 *     features = (cos phi, sin phi, cos 2phi, sin 2phi, cos 4phi, sin 4phi, r_c / rho,
 *     8 theta0), phi the in-plane angle from [001] towards [110], env = exp(-s_exact)
 *     times the mode's largest block (the band's largest values, so the targets are of
 *     order one or less), the MLP 8 -> 128 -> 128 -> 128 -> 12 with SiLU activations
 *     giving the 6 complex components of the symmetric 3x3 block (xx, yy, zz, xy, xz,
 *     yz); applied out to the largest distance of its training data, the continuum
 *     alone beyond;
 *   continuum: out to the last block above the context's skip tolerance (the continuum
 *     value alone, zero where kappa rho > 40);  beyond: zero.
 * ------------------------------------------------------------------------------------ */

/* Last error text of the fbc_sur_* / fbc_mlp_* calls on this host thread. */
const char* fbc_learned_last_error(void);

/* Builds the continuum table H(kappa rho, phi) on the device (homogeneity: one table at
 * unit in-plane distance; 256 in-plane directions, 256 log-spaced kappa rho in
 * [1e-3, 40] plus kappa = 0; beyond 40 the continuum value is taken as zero).  r_c in
 * lattice constants (> 0).  Synchronises `stream`. */
fbc_status fbc_sur_create(const fbc_lattice* lat, double r_c, void* stream, fbc_sur** out);
void fbc_sur_destroy(fbc_sur* s);

/* Copies the network's current FP32 weights into the object as BF16 (round to nearest
 * even) for inference; later training of `net` does not change them until called again.
 * A surrogate context evaluates the learned band with them on MFMA (BF16 weights and
 * activations, FP32 accumulation, biases and SiLU in FP32); fbc_sur_eval on the SIMT
 * path (FP32 activations).  Synchronises `stream`. */
fbc_status fbc_sur_set_mlp(fbc_sur* s, const fbc_mlp* net, void* stream);

/* The same with the FP32 weights kept as they are (inference with FP32 weights, FP32
 * activations and FP32 accumulation, on the SIMT path): the control that separates the
 * BF16 rounding of weights and activations from the network's own fit in an error budget.  Replaces the BF16 weights until fbc_sur_set_mlp
 * is called again.  Synchronises `stream`. */
fbc_status fbc_sur_set_mlp_fp32(fbc_sur* s, const fbc_mlp* net, void* stream);

/* End of the learned band (exp(-s_learn) of a mode's largest block): s_learn in (0, 40];
 * default 20.  Read when a context is created and by fbc_sur_training_set. */
fbc_status fbc_sur_set_learn_range(fbc_sur* s, double s_learn);

/* End of the exact band (exp(-s_exact) of a mode's largest block): s_exact in [0, 40];
 * default 12.  Read when a context is created (it fixes the size of the context's exact
 * table, fbc_info's store_bytes) and by fbc_sur_training_set. */
fbc_status fbc_sur_set_exact_range(fbc_sur* s, double s_exact);

/* Evaluates n blocks: out[n][6] complex (interleaved re, im; device) at line wavenumber
 * theta0[n] in [0, 1/2] and column offsets dn1[n], dn2[n] (all device).  use_mlp = 0:
 * continuum value only; 1: continuum + the network's correction with env = 1 (a context
 * scales it by its per-mode envelope; rho <= r_c returns the continuum value, since the
 * exact values live in a context).  Asynchronous. */
fbc_status fbc_sur_eval(const fbc_sur* s, const double* theta0, const int32_t* dn1,
                        const int32_t* dn2, int n, int use_mlp, double* out, void* stream);

/* Training data from an FBC_FORM_DTABLE_FP64 context, whose table holds the lattice
 * values of every distinct offset and line mode of its cells: max_samples pairs
 * (table mode >= 1, offset) in the learned band of that table (rho > r_c, found from the
 * table's values as a surrogate context finds it) drawn by a host generator seeded with
 * `seed` (a mode uniformly among those whose band holds an offset, then an offset
 * uniformly in its band), each turned into
 * features x[n][8] and target t[n][12] (the correction above divided by env and rotated
 * by exp(-i pi theta0 dn1)); x, t are device FP32 buffers of max_samples rows.
 * *n_out = rows written.  Also records in s the largest in-plane distance of the band:
 * surrogate contexts apply the learned correction only out to it (no extrapolation
 * beyond the training data; the continuum alone further out).  FBC_E_ARG when no offset
 * of the context lies in the band.  Synchronises. */
fbc_status fbc_sur_training_set(fbc_sur* s, const fbc_ctx* table_ctx, int max_samples,
                                uint64_t seed, float* x, float* t, int* n_out, void* stream);

/* Trainable MLP with FP32 parameters, Adam state and a workspace for batches of up to
 * max_batch rows (<= 2^22).  Weights drawn N(0, 1/fan_in) from `seed`, biases zero.
 * Parameter layout, per layer l = 0..3: W_l [out][in] row-major, then b_l [out]. */
fbc_status fbc_mlp_create(int max_batch, uint64_t seed, fbc_mlp** out);
void fbc_mlp_destroy(fbc_mlp* m);
int fbc_mlp_num_params(void);
/* Synchronous host copies: host_in (may be NULL) replaces the parameters, then
 * host_out (may be NULL) receives them; fbc_mlp_grad copies the last gradient. */
fbc_status fbc_mlp_params(fbc_mlp* m, float* host_out, const float* host_in);
fbc_status fbc_mlp_grad(fbc_mlp* m, float* host_out);
/* Loss L = (1/n) sum_rows sum_j (y_j - t_j)^2 over a batch (x [n][8], t [n][12],
 * device FP32) and its gradient with respect to the parameters (kept in the object);
 * loss_dev: device float receiving L, or NULL.  Asynchronous. */
fbc_status fbc_mlp_loss_grad(fbc_mlp* m, const float* x, const float* t, int n,
                             float* loss_dev, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the last gradient. */
fbc_status fbc_mlp_adam_step(fbc_mlp* m, float lr, void* stream);
/* FP32 forward pass y [n][12] of x [n][8] (device). */
fbc_status fbc_mlp_forward(fbc_mlp* m, const float* x, float* y, int n, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the same forward pass (same kernels, bitwise the
 * result of fbc_mlp_forward) with the layer activations kept in a workspace of 64 MiB that
 * the library holds statically on every GPU it runs on (until the process ends) instead
 * of the network's own workspace; n is not limited by max_batch but by that workspace:
 * n in [1, fbc_mlp_forward_noalloc_max_rows()] (10591 rows), else FBC_E_ARG.  Calls no
 * allocating routine; asynchronous on `stream`.  The network's device must be current
 * (FBC_E_ARG otherwise).  All calls on one GPU share the workspace: calls that overlap on
 * one GPU (other streams, other threads) race; calls ordered on one stream do not.  Every
 * workspace value is written before it is read, so nothing carries over between calls. */
fbc_status fbc_mlp_forward_noalloc(const fbc_mlp* m, const float* x, float* y, int n, void* stream);
int fbc_mlp_forward_noalloc_max_rows(void);
/* ------------------------------------------------------------------------------------
 * Real-space periodic lattice Green function (Section 3.1, eqs. G~inf, plgf_conv,
 * plgf_poly and plgf_rich; Appendix B): an independent route to the line-periodic Green
 * function, for cross-checking the Brillouin-zone blocks and for geometries that are not
 * unions of atom columns.
 *
 * G~inf(r) is the infinite-lattice Green function for |r| <= r_cut and the continuum
 * (Kelvin) Green function beyond.  Within r_cut it is evaluated as the Green function of
 * the torus_l^3 torus of the primitive cell (Brillouin-zone sum on that grid, q = 0
 * dropped) minus a constant C, the mean of that torus function minus the continuum
 * function over the lattice vectors of the shell r_cut < |r| <= r_match; C makes the two
 * pieces join (the Green function is unique up to a constant).  The line-periodic value
 * at a lattice vector r is the Richardson extrapolation (order N, from the partial sums
 * k = n .. n + N) of G~_k(r) = sum over |i| <= k of G~inf(r + i N_z b0) - G~inf(i N_z b0).
 *
 * Lattice vectors are primitive-basis integers (n0, n1, n2) with b0 = (1, -1, 0)/2 along
 * the line, b1 = (1, 0, 1)/2, b2 = (1, 1, 0)/2 (cube axes, a = 1); radii enter as
 * 4 |r|^2 / a^2, integers, so r_cut = 5 a is r2x4_cut = 100.  Results do not depend on a.
 * Outputs are the 6 components xx yy zz xy xz yz of the symmetric 3x3 block.
 * ------------------------------------------------------------------------------------ */
typedef struct fbc_plgf fbc_plgf;

typedef struct {
    int torus_l;        /* torus edge for the near-field table: power of two in [8, 256]  */
    int r2x4_cut;       /* 4 r_cut^2 in [0, 576] (a = 1)                                  */
    int r2x4_match;     /* 4 r_match^2 in (r2x4_cut, 1024]: outer radius of the C shell   */
    int n_psi;          /* nodes of the continuum circle integral: multiple of 64 in
                           [64, 1024]                                                     */
} fbc_plgf_opts;

/* Last error text of the fbc_plgf_* calls on this host thread. */
const char* fbc_plgf_last_error(void);

/* Builds the near-field table (torus sums, one work group per lattice vector of the table
 * and the shell) and C on the device.  Synchronises `stream`.  FBC_E_ARG for out-of-range
 * options; FBC_E_NOMEM / FBC_E_DEVICE as elsewhere.  The object owns its device memory. */
fbc_status fbc_plgf_create(const fbc_lattice* lat, const fbc_plgf_opts* opts, void* stream,
                           fbc_plgf** out);
void fbc_plgf_destroy(fbc_plgf* p);

/* Synchronous host copies of the table: *n_table = number of lattice vectors with
 * |r| <= r_cut; vectors [n_table][3] (sorted by 4|r|^2, then n0, n1, n2), values
 * [n_table][6] (G_torus - C) and c [6] may each be NULL. */
fbc_status fbc_plgf_table(const fbc_plgf* p, int* n_table, int32_t* vectors, double* values,
                          double* c);

/* Line-periodic Green function at n lattice vectors disp [n][3] (device int32) for a line
 * of nz layers (period nz b0, nz in [1, 65536]); out [n][6] (device FP64).  Richardson
 * from the partial sums n_rich .. n_rich + order (n_rich >= 1, order in [0, 7],
 * n_rich + order <= 16; the paper's choice is n_rich = 1, order = 5).  Asynchronous; the
 * object holds the images of the origin for the call in flight, so calls on one object
 * must be ordered (one stream). */
fbc_status fbc_plgf_eval(fbc_plgf* p, const int32_t* disp, int64_t n, int nz, int n_rich,
                         int order, double* out, void* stream);

/* ------------------------------------------------------------------------------------
 * H-matrix form of the per-mode Green blocks (Appendix C).  For every line mode m of a
 * cell, G^(m) (3 n_b x 3 n_i complex) is split by the block partition of two cluster
 * trees: binary space partitioning of the in-plane column positions, each cluster cut
 * along the longer side of its bounding box at the median (ties by column index) until it
 * holds at most b_min columns; a block t x s is low rank when
 * min(diam t, diam s) <= gamma dist(t, s) (eq. geom_adm on the bounding boxes: diam =
 * box diagonal, dist = distance between the boxes, decided in exact integers; the text's
 * centroid distance admits touching half rings; the line direction is diagonalised
 * by the line transform, so the periodic images s+- share the in-plane position of s), a
 * dense leaf when both clusters are leaves, and subdivided otherwise.  Low-rank blocks
 * are compressed by adaptive cross approximation with partial pivoting (eq. aca; first
 * row of the block first, then the unused row of largest |u_k|; stop when
 * |u_k| |v_k| <= eps ||S_k||_F holds for two consecutive terms); rows and columns of a
 * block follow the tree order (first child's columns, then the second's).  A block that
 * needs more than max_rank terms is applied from the dense store instead.  Paper:
 * b_min = 20, gamma = 2, eps = 1e-5.
 * ------------------------------------------------------------------------------------ */
typedef struct fbc_hmat fbc_hmat;

typedef struct {
    int b_min;          /* minimal cluster size in atom columns (>= 1)                  */
    int gamma;          /* admissibility constant, integer in [1, 64]                  */
    double eps;         /* cross-approximation accuracy bound (> 0)                    */
    int max_rank;       /* rank bound per block, in [1, 512]                           */
} fbc_hmat_opts;

typedef struct {
    int n_blocks, n_low_rank, n_dense;   /* partition leaves (same for every mode)      */
    int max_rank_used;                   /* largest rank over modes and blocks          */
    int n_over_rank;                     /* (mode, block) pairs applied from the store   */
    double stored_entries;               /* complex entries of the factors and dense
                                            leaves over all modes                       */
    double dense_entries;                /* the same matrices stored densely            */
} fbc_hmat_info;

/* Last error text of the fbc_hmat_* calls on this host thread. */
const char* fbc_hmat_last_error(void);

/* Builds the H-matrices of every line mode of `ctx` (FBC_FORM_DTABLE_FP64, exactly one
 * cell; FBC_E_UNSUPPORTED otherwise) from its offset table (the entries depend on the
 * column offset only, Section 3.2, so no dense matrix is ever formed); the context must
 * outlive the object, which reads the table for dense leaves.  Trees and partition on the
 * host (geometry only), the cross approximations on the device (one work group per block
 * and mode).  Synchronises `stream`. */
fbc_status fbc_hmat_create(const fbc_ctx* ctx, const fbc_hmat_opts* opts, void* stream,
                           fbc_hmat** out);
void fbc_hmat_destroy(fbc_hmat* h);
fbc_status fbc_hmat_get_info(const fbc_hmat* h, fbc_hmat_info* info);

/* The partition as a host int32 stream: per block kind (1 low rank, 0 dense), n_t, n_s,
 * the n_t pad and the n_s interface column indices (tree order).  *n_out = its length;
 * out may be NULL to query it (else cap >= *n_out). */
fbc_status fbc_hmat_partition(const fbc_hmat* h, int32_t* out, int64_t cap, int64_t* n_out);

/* Ranks [n_modes][n_low_rank] (host; -1: over the rank bound). */
fbc_status fbc_hmat_ranks(const fbc_hmat* h, int32_t* out);

/* what = H f per mode: fhat [n_modes][3 n_i][R] and what [n_modes][3 n_b][R], complex
 * FP64 interleaved (re, im), device; R = the cell's n_rhs.  Asynchronous; calls on one
 * object must be ordered (it holds the products V^T f of the call in flight). */
fbc_status fbc_hmat_apply(fbc_hmat* h, const double* fhat, double* what, void* stream);

/* Attaches h (built from c by fbc_hmat_create) as the product step of c's pipeline:
 * fbc_apply, fbc_apply_graph, fbc_green_apply, fbc_relax_step and fbc_relax_step_graph
 * then apply the H-matrix of every line mode (Section 3.2 / Appendix C) in place of the
 * offset-table product, reading the forward transform's output and writing the records
 * the inverse transform reads (no extra pass); h = NULL detaches.  The work list is set
 * to one K slice while attached (its K slices come back on detaching); fbc_autotune and
 * fbc_set_work_list return FBC_E_STATE while an H-matrix is attached; captured graphs are
 * dropped.  fbc_hmat_destroy of an attached
 * object detaches it.  FBC_E_ARG when h was built from another context.  Synchronises
 * `stream`. */
fbc_status fbc_set_hmat(fbc_ctx* c, fbc_hmat* h, void* stream);

const char* fbc_status_string(fbc_status s);

/* Diagnostic for callers that weigh a kernel against the memory's practical rate (not part
 * of the method): reads `bytes` of the device buffer `buf` (16-byte aligned, a multiple of
 * 16 bytes) with a plain streaming-read kernel -- `groups` work groups of 256 threads, each
 * its own contiguous share, 16-byte nontemporal loads, eight in flight per thread -- once
 * untimed, then `reps` times between HIP events on `stream`, and sets *gbs to the rate in
 * GB/s (1e9 bytes).  Allocates and frees a small output buffer; synchronises `stream`.
 * FBC_E_ARG for a bad pointer, size, alignment, groups outside [1, 65536] or reps outside
 * [1, 1000]; FBC_E_NOMEM / FBC_E_DEVICE on a runtime failure. */
fbc_status fbc_probe_read(const void* buf, int64_t bytes, int groups, int reps, double* gbs, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FBC_H */
