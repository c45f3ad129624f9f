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

void launch_sur_samples(hipStream_t st, const CgfView& v, const double2* tab, int64_t n_off, int nz_tab,
                        const int32_t* d1, const int32_t* d2, const int32_t* pick_t,
                        const int32_t* pick_o, int n, double r_c, double env_floor,
                        const double* cmatch, float* x, float* t);
// width of the shell inside r_c over which the line-mode-0 matching constant is averaged
#define SUR_MATCH_SHELL 1.5
// the learned correction covers kappa rho <= SUR_S_LEARN (beyond it the blocks are below
// about 1e-3 of the line-mode-0 scale and the continuum value is used alone)
#define SUR_S_LEARN 6.0
void launch_sur_const(hipStream_t st, const CgfView& v, const double2* tab0, const int32_t* d1,
                      const int32_t* d2, int64_t n, double r_lo, double r_hi, double* cmatch);
void launch_sur_points(hipStream_t st, const CgfView& v, const unsigned short* wb, const float* bias,
                       int use_mlp, double r_c, double env_floor, const double* theta0,
                       const int32_t* d1, const int32_t* d2, int n, double2* out);
void launch_sur_generate(hipStream_t st, const CgfView& v, const unsigned short* wb, const float* bias,
                         double r_c, double env_floor, int nz_tab, int t0, int nt,
                         const double2* near_tab, int64_t n_near, int64_t n_off,
                         const int32_t* n_need, const int32_t* d1, const int32_t* d2, const double* cmatch,
                         double2* out, int64_t max_need);
void launch_mlp_to_bf16(hipStream_t st, const float* params, unsigned short* wb, float* bias);
