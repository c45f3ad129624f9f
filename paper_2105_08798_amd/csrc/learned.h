// Learned far-field form: continuum Green function table and MLP kernels.
#pragma once
#include "kernels.h"

#define MLP_IN 8
#define MLP_H 128
#define MLP_OUT 12
#define MLP_NPARAMS (MLP_IN * MLP_H + MLP_H + 2 * (MLP_H * MLP_H + MLP_H) + MLP_H * MLP_OUT + MLP_OUT)

// Build parameters of the continuum table H(s, phi) (unit in-plane distance).
struct CgfConst {
    double c11, c12, c44;
    double t[3];           // line direction (cubic axes)
    int npsi;              // circle-integral nodes
    int nphi;              // in-plane directions
    int nzq;               // z nodes on [-zmax, zmax]
    int ns;                // s nodes, log-spaced on [s_min, s_max]
    double zmax, dz, s_min, s_max;
};

// Read-only view used by the evaluation device function.
struct CgfView {
    const double2* H;      // [nphi][ns + 1][6]; column ns: kappa = 0 (real part)
    const double* g0;      // G_K(t), 6 components
    int nphi, ns;
    double ls_min, dls, s_max;
};

__device__ void cgf_eval(const CgfView& v, double theta0, int dn1, int dn2, double2 out[6]);

void launch_cgf_build(hipStream_t st, const CgfConst& k, const double* cpsi, const double* spsi,
                      const double* rhat, double* g0, double* g1, double* rem, const double2* ph0,
                      const double2* step, const double* k0s, double2* H);
void launch_cgf_points(hipStream_t st, const CgfView& v, const double* theta0, const int32_t* d1,
                       const int32_t* d2, int n, double2* out);

int64_t mlp_workspace_floats(int n);
void launch_mlp_forward(hipStream_t st, const float* params, const float* x, int n, float* ws,
                        float* y);
void launch_mlp_loss_grad(hipStream_t st, const float* params, const float* x, const float* t,
                          const float* w, int n, float* ws, float* grad, float* loss);
void launch_adam(hipStream_t st, float* p, const float* g, float* m, float* v, int n, float lr,
                 int step);

#define MLP_NW (MLP_H * MLP_IN + 2 * MLP_H * MLP_H + MLP_OUT * MLP_H)
#define MLP_NB (3 * MLP_H + MLP_OUT)

// Inference weights of the learned correction: transposed BF16 weights (wb), or -- the
// FP32 control -- transposed FP32 weights (wf != NULL), and FP32 biases.
struct MlpInfer {
    const unsigned short* wb;
    const float* wf;
    const float* bias;
    const unsigned short* wm;      // BF16 fragments of the MFMA inference (k_sur_learned)
};

void launch_sur_samples(hipStream_t st, const CgfView& v, const double2* tab, int64_t n_off, int nz_tab,
                        const int32_t* d1, const int32_t* d2, const int32_t* pick_t,
                        const int32_t* pick_o, int n, double r_c, const double* env_mode, float* x, float* t);
// Surrogate bands of every line mode m >= 1, by distance: exact lattice values within r_c
// and out to the last block of at least exp(-s_exact) times the mode's largest block,
// continuum + learned correction out to the last block of at least exp(-s_learn) times
// it, continuum alone out to the last block above the context's skip tolerance, zero
// beyond.
#define SUR_S_EXACT 12.0
#define SUR_S_LEARN 20.0
void launch_sur_points(hipStream_t st, const CgfView& v, const MlpInfer& w, int use_mlp, double r_c,
                       const double* theta0, const int32_t* d1,
                       const int32_t* d2, int n, double2* out);
void launch_sur_generate(hipStream_t st, const CgfView& v, const MlpInfer& w, double r_c, const double* env_mode,
                         double rho_learn, int nz_tab, int t0, int nt, const double2* exact_tab, const int64_t* ex_off,
                         const int32_t* n_exact, const int32_t* n_learn, int64_t n_off,
                         const int32_t* n_need, const int32_t* d1, const int32_t* d2, double2* out,
                         int64_t min_exact, int64_t max_exact, int64_t min_learn, int64_t max_band, int64_t max_need);
void launch_mlp_to_bf16(hipStream_t st, const float* params, unsigned short* wb, float* bias);
void launch_mlp_to_f32t(hipStream_t st, const float* params, float* wf, float* bias);
#define MLP_MFMA_ELEMS ((8 + 32 + 32 + 4) * 512)
void launch_mlp_to_mfma(hipStream_t st, const float* params, unsigned short* wm);
