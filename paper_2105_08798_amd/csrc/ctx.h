// Internal definitions shared by the C-ABI translation units.
#pragma once
#include <string>
#include <vector>

#include "learned.h"

struct fbc_sur;

struct fbc_ctx {
    int device = 0;
    fbc_hmat* hmat = nullptr;        // attached H-matrix: the product step of the apply pipeline
    int hmat_prev_nsplit = 1;        // K slices of the work list before attaching
    fbc_options opt{};
    fbc_lattice lat{};
    std::vector<CellPlan> cells;
    int total_rhs = 0;
    int64_t f_elems = 0, u_elems = 0;
    int ctmax = 1;
    // device buffers (all owned)
    std::vector<void*> allocs;
    void* store = nullptr;          // dense store (FP64 / FP32 / split BF16)
    int64_t store_bytes = 0;
    void* bfrag = nullptr;          // GEMM B operand
    double* cbuf = nullptr;         // GEMM output
    double* wbuf = nullptr;         // w[r][row][n0]
    double* sums = nullptr;         // per layer: net force and absolute force [r][n0][6]
    double* ftot = nullptr;         // net force of each cell per RHS [total_rhs][3]
    double2* shat = nullptr;        // line transform of the per-layer net force [r][m][3]
    int* shat_on = nullptr;         // per RHS: 0 when that transform is exactly zero [total_rhs]
    double2* rowmean = nullptr;     // row-gauge means [m][b][6] (reduced forms with row gauge)
    std::vector<int64_t> shat_off, rowmean_off;
    unsigned long long* amax = nullptr;  // split FP16: per cell mode, largest table magnitude
    std::vector<int64_t> amax_off;
    int* bexp = nullptr;            // split FP16: per RHS, force operand scale exponent [total_rhs]
    double* wmax_part = nullptr;
    double* sum_part = nullptr;
    double* mean = nullptr;         // [total_rhs][3]
    double2* tw = nullptr;          // twiddle tables
    int* status = nullptr;          // 128 bytes: [0] device latch; [16..24] counters of the
                                    // persistent product's work lists, zero between launches
    PqLists lists{};                // work lists of the persistent product (orders 3 and 4)
    GemmJob* jobs = nullptr;
    int njobs = 0;
    int nsplit = 1;                 // K slices of the per-mode product
    int nsplit_cap = 1;             // K slices the output buffer holds
    int job_order = 0;              // see build_jobs (3, 4: persistent kernel)
    int variant = 0;                // product kernel variant (gemm_variants)
    int64_t jobs_cap = 0;
    // captured update (fbc_apply_graph)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const double* g_f = nullptr;
    double* g_u = nullptr;
    double g_alpha = 0.0;
    void* g_stream = nullptr;
    int64_t scratch_bytes = 0;
    double product_bytes = 0, product_flops = 0, skipped_fraction = 0;   // see fbc_info
    int64_t n_offsets = 0;
    // offset table (kept for the offset-table form)
    int nz_max = 0;
    double2* tab = nullptr;
    int32_t* lut = nullptr;
    int d1min = 0, d2min = 0, w2 = 0;
    CellDev* celldev = nullptr;
    // surrogate form: ragged exact table, offsets by increasing distance, generated slices
    const fbc_sur* sur = nullptr;
    double2* exact_tab = nullptr;    // mode t: the first n_exact[t] offsets at ex_off[t] (x 6)
    int64_t* ex_off = nullptr;       // device [T]
    int32_t* n_exact = nullptr;      // device [T]
    int32_t* n_learn = nullptr;      // device [T]: offsets n_exact .. n_learn-1 get the learned correction
    double* env_mode = nullptr;      // device [T]: envelope of the learned correction
    std::vector<int32_t> n_exact_h, n_learn_h;   // host copies
    std::vector<int64_t> ex_off_h;
    int64_t n_near = 0;              // offsets with rho <= r_c
    int32_t* off_d1 = nullptr;       // device offsets in table order
    int32_t* off_d2 = nullptr;
    int32_t* n_need = nullptr;       // per table mode: offsets to generate (prefix)
    std::vector<int32_t> n_need_h;   // host copy
    double2* gen = nullptr;          // generated slices [chunk modes][n_off][6]
    int gen_modes = 0;               // table modes per generated chunk
    std::vector<int> chunk_job0;     // first job of each chunk (jobs sorted by table mode)
    // relax
    double* fprev = nullptr;
    double* alpha = nullptr;
    double* finf = nullptr;
    double* stepinf = nullptr;
    double* rpart = nullptr;
    double* rmean = nullptr;
    fbc_relax_opts ropt{};
    int relax_k = -1;               // -1 before fbc_relax_begin; else the host's count of steps
                                    // (the index itself lives on the device: status[4])
    // captured relaxation step (fbc_relax_step_graph)
    hipGraph_t rgraph = nullptr;
    hipGraphExec_t rgraph_exec = nullptr;
    const double* rg_f = nullptr;
    double* rg_u = nullptr;
    fbc_relax_out* rg_out = nullptr;
    void* rg_stream = nullptr;
    // per cell partial counts
    std::vector<int> npart_irfft, npart_update;
    std::vector<int64_t> wmax_off, sum_part_off, rpart_off;
    std::string err;
    // timing of the product kernel
    int timing = 0;
    std::vector<hipEvent_t> ev;      // 2 * kMaxTimed events, created on first enable
    int n_timed = 0;
};
static const int kMaxTimed = 4096;

// Learned far-field object (continuum table + inference weights).
struct fbc_sur {
    double r_c = 6.0;
    CgfConst k{};
    double2* H = nullptr;            // continuum table
    double* g0 = nullptr;
    unsigned short* wb = nullptr;    // transposed bf16 weights
    unsigned short* wm = nullptr;    // bf16 weights in MFMA fragment order (learned band)
    float* wf = nullptr;             // transposed FP32 weights (inference control)
    float* bias = nullptr;
    int has_mlp = 0;
    int mlp_fp32 = 0;                // 1: inference with the FP32 weights
    double s_exact = SUR_S_EXACT;    // end of the exact band (exp(-s_exact) of a mode's largest block)
    double s_learn = SUR_S_LEARN;    // end of the learned band (exp(-s_learn) of a mode's largest block)
    double rho_learn = INFINITY;     // largest distance of the training data (set by fbc_sur_training_set)
    std::vector<void*> allocs;
    std::string err;
    MlpInfer infer() const { return MlpInfer{wb, mlp_fp32 ? wf : nullptr, bias, wm}; }
    CgfView view() const {
        CgfView v;
        v.H = H;
        v.g0 = g0;
        v.nphi = k.nphi;
        v.ns = k.ns;
        v.ls_min = std::log(k.s_min);
        v.dls = (std::log(k.s_max) - std::log(k.s_min)) / (k.ns - 1);
        v.s_max = k.s_max;
        return v;
    }
};

// Trainable MLP (FP32 master weights, Adam state, gradient and workspace).
struct fbc_mlp {
    float* params = nullptr;
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* ws = nullptr;
    float* loss = nullptr;
    int max_batch = 0;
    int step = 0;
    int device = 0;                  // device holding the parameters
    std::vector<void*> allocs;
    std::string err;
};
