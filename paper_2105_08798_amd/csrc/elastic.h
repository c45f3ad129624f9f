// Continuum elasticity of a cubic crystal on the device: the Kelvin point-force solution
// (Section 3.1, eq. cgf: homogeneous of degree -1) shared by the learned far field and the
// real-space periodic Green function.
#pragma once
#include <hip/hip_runtime.h>

// Inverse of a symmetric 3x3 matrix in the order xx yy zz xy xz yz (adjugate / det).
__device__ inline void sym_inverse(const double g[6], double o[6]) {
    const double a = g[0], b = g[1], c = g[2], xy = g[3], xz = g[4], yz = g[5];
    const double cxx = b * c - yz * yz, cyy = a * c - xz * xz, czz = a * b - xy * xy;
    const double cxy = xz * yz - xy * c, cxz = xy * yz - b * xz, cyz = xy * xz - a * yz;
    const double inv = 1.0 / (a * cxx + xy * cxy + xz * cxz);
    o[0] = cxx * inv; o[1] = cyy * inv; o[2] = czz * inv;
    o[3] = cxy * inv; o[4] = cxz * inv; o[5] = cyz * inv;
}

// Acoustic tensor Gamma_ik(n) = C_ijkl n_j n_l of a cubic crystal in its cube axes:
// Gamma_ii = C11 n_i^2 + C44 (|n|^2 - n_i^2), Gamma_ik = (C12 + C44) n_i n_k.
__device__ inline void acoustic(const double n[3], double c11, double c12, double c44, double g[6]) {
    const double q0 = n[0] * n[0], q1 = n[1] * n[1], q2 = n[2] * n[2], tot = q0 + q1 + q2;
    g[0] = c11 * q0 + c44 * (tot - q0);
    g[1] = c11 * q1 + c44 * (tot - q1);
    g[2] = c11 * q2 + c44 * (tot - q2);
    g[3] = (c12 + c44) * n[0] * n[1];
    g[4] = (c12 + c44) * n[0] * n[2];
    g[5] = (c12 + c44) * n[1] * n[2];
}

// Orthonormal pair (u, v) normal to the unit vector xh (u = xh x e, e = e_x unless xh is
// close to it, then e_y; v = xh x u).
__device__ inline void normal_pair(const double xh[3], double u[3], double v[3]) {
    double hp[3] = {0, 0, 0};
    if (fabs(xh[0]) < 0.9) hp[0] = 1.0; else hp[1] = 1.0;
    u[0] = xh[1] * hp[2] - xh[2] * hp[1];
    u[1] = xh[2] * hp[0] - xh[0] * hp[2];
    u[2] = xh[0] * hp[1] - xh[1] * hp[0];
    const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    u[0] /= un; u[1] /= un; u[2] /= un;
    v[0] = xh[1] * u[2] - xh[2] * u[1];
    v[1] = xh[2] * u[0] - xh[0] * u[2];
    v[2] = xh[0] * u[1] - xh[1] * u[0];
}

// Kelvin solution G_K(x) = 1/(8 pi^2 |x|) * circle integral of Gamma(n)^{-1} over unit n
// normal to x, by the trapezoid rule over npsi nodes psi_l (cpsi, spsi = cos, sin psi_l);
// output xx yy zz xy xz yz.
__device__ inline void kelvin_point(const double x[3], double c11, double c12, double c44, int npsi,
                                    const double* __restrict__ cpsi, const double* __restrict__ spsi,
                                    double out[6]) {
    const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double xh[3] = {x[0] / r, x[1] / r, x[2] / r};
    double u[3], v[3];
    normal_pair(xh, u, v);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int l = 0; l < npsi; ++l) {
        const double n[3] = {cpsi[l] * u[0] + spsi[l] * v[0], cpsi[l] * u[1] + spsi[l] * v[1],
                             cpsi[l] * u[2] + spsi[l] * v[2]};
        double g[6], o[6];
        acoustic(n, c11, c12, c44, g);
        sym_inverse(g, o);
        for (int c = 0; c < 6; ++c) acc[c] += o[c];
    }
    const double sc = 1.0 / (4.0 * M_PI * npsi * r);
    for (int c = 0; c < 6; ++c) out[c] = acc[c] * sc;
}
