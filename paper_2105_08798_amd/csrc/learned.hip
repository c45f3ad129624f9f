// Learned far-field form (beyond the exact near field): the continuum Green function
// in the line-mode representation (Section 3.1, eq. cgf; Appendix B, lattice function ->
// continuum function beyond a cut-off radius), tabulated once through its homogeneity,
// and a 4-layer MLP for the correction G^_lgf - G^_cgf, with training kernels (forward,
// backward, Adam) and the on-the-fly table generator of the surrogate form.
#include <algorithm>
#include <cmath>
#include <vector>

#include "elastic.h"
#include "learned.h"

#define NTL 256

__device__ inline void kelvin(const double x[3], const CgfConst& k, const double* __restrict__ cpsi,
                              const double* __restrict__ spsi, double out[6]) {
    kelvin_point(x, k.c11, k.c12, k.c44, k.npsi, cpsi, spsi, out);
}

// G0 = G_K(t) and g1(phi_j) = (r_hat_j . grad) G_K at t (central difference, step h).
__global__ void k_cgf_g(CgfConst k, const double* __restrict__ cpsi, const double* __restrict__ spsi,
                        const double* __restrict__ rhat, double* __restrict__ g0,
                        double* __restrict__ g1) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > k.nphi) return;
    if (j == k.nphi) {
        kelvin(k.t, k, cpsi, spsi, g0);
        return;
    }
    const double h = 1e-4;
    double xp[3], xm[3], gp[6], gm[6];
    for (int a = 0; a < 3; ++a) {
        xp[a] = k.t[a] + h * rhat[3 * j + a];
        xm[a] = k.t[a] - h * rhat[3 * j + a];
    }
    kelvin(xp, k, cpsi, spsi, gp);
    kelvin(xm, k, cpsi, spsi, gm);
    for (int c = 0; c < 6; ++c) g1[6 * j + c] = (gp[c] - gm[c]) / (2.0 * h);
}

// Remainder R(phi_j, z) = G_K(r_hat_j + z t) - G0/sqrt(z^2+1) - g1_j z/(z^2+1)^{3/2}.
__global__ void __launch_bounds__(NTL) k_cgf_rem(CgfConst k, const double* __restrict__ cpsi,
                                                 const double* __restrict__ spsi,
                                                 const double* __restrict__ rhat,
                                                 const double* __restrict__ g0,
                                                 const double* __restrict__ g1,
                                                 double* __restrict__ rem) {
    const int64_t idx = (int64_t)blockIdx.x * NTL + threadIdx.x;
    if (idx >= (int64_t)k.nphi * k.nzq) return;
    const int j = (int)(idx / k.nzq);
    const int q = (int)(idx - (int64_t)j * k.nzq);
    const double z = -k.zmax + q * k.dz;
    double x[3], g[6];
    for (int a = 0; a < 3; ++a) x[a] = rhat[3 * j + a] + z * k.t[a];
    kelvin(x, k, cpsi, spsi, g);
    const double d = sqrt(z * z + 1.0);
    const double e1 = 1.0 / d, e2 = z / (d * d * d);
    for (int c = 0; c < 6; ++c) rem[idx * 6 + c] = g[c] - g0[c] * e1 - g1[6 * j + c] * e2;
}

// H(s_i, phi_j) = sum_q w_q exp(-i s_i z_q) R(phi_j, z_q) + 2 G0 K0(s) - 2 i s g1 K0(s),
// stored as e^{s_i} H; the phase advances by a complex rotation per node (host tables
// ph0, step).
// Column i = ns holds the regularised kappa = 0 value (real): sum_q w_q R + 2 G0 (log 2 - gamma).
__global__ void __launch_bounds__(NTL) k_cgf_transform(CgfConst k, const double* __restrict__ rem,
                                                       const double* __restrict__ g0,
                                                       const double* __restrict__ g1,
                                                       const double2* __restrict__ ph0,
                                                       const double2* __restrict__ step,
                                                       const double* __restrict__ k0s,
                                                       double2* __restrict__ H) {
    const int idx = blockIdx.x * NTL + threadIdx.x;
    if (idx >= k.nphi * (k.ns + 1)) return;
    const int j = idx / (k.ns + 1);
    const int i = idx - j * (k.ns + 1);
    const double* rj = rem + (int64_t)j * k.nzq * 6;
    double2 acc[6];
    for (int c = 0; c < 6; ++c) acc[c] = make_double2(0, 0);
    if (i < k.ns) {
        double2 ph = ph0[i];
        const double2 st = step[i];
        for (int q = 0; q < k.nzq; ++q) {
            const double w = (q == 0 || q == k.nzq - 1) ? 0.5 * k.dz : k.dz;
            const double pr = w * ph.x, pi = w * ph.y;
            for (int c = 0; c < 6; ++c) {
                const double r = rj[q * 6 + c];
                acc[c].x += pr * r;
                acc[c].y += pi * r;
            }
            ph = make_double2(ph.x * st.x - ph.y * st.y, ph.x * st.y + ph.y * st.x);
        }
        const double K0 = k0s[2 * i], s = k0s[2 * i + 1];      // K0(s_i), s_i (host table)
        // stored times e^{s}: the transform decays roughly like e^{-s}, and the scaled
        // function varies slowly enough for cubic interpolation between nodes
        const double es = exp(s);
        for (int c = 0; c < 6; ++c) {
            acc[c].x = (acc[c].x + 2.0 * g0[c] * K0) * es;
            acc[c].y = (acc[c].y - 2.0 * s * g1[6 * j + c] * K0) * es;
        }
    } else {
        for (int q = 0; q < k.nzq; ++q) {
            const double w = (q == 0 || q == k.nzq - 1) ? 0.5 * k.dz : k.dz;
            for (int c = 0; c < 6; ++c) acc[c].x += w * rj[q * 6 + c];
        }
        for (int c = 0; c < 6; ++c) acc[c].x += 2.0 * g0[c] * (M_LN2 - 0.57721566490153286061);
    }
    for (int c = 0; c < 6; ++c) H[(int64_t)idx * 6 + c] = acc[c];
}

// ----------------------------------------------------------------------------------
// Evaluation of the far-field block at (theta0, dn1, dn2): Catmull-Rom interpolation
// of H in (log s, phi), the small-s logarithm below s_min, zero above s_max.
// ----------------------------------------------------------------------------------
__device__ inline double cr_w(double t, int k) {
    // Catmull-Rom weights for points -1, 0, 1, 2 at parameter t in [0, 1)
    const double t2 = t * t, t3 = t2 * t;
    switch (k) {
        case 0: return 0.5 * (-t3 + 2.0 * t2 - t);
        case 1: return 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
        case 2: return 0.5 * (-3.0 * t3 + 4.0 * t2 + t);
        default: return 0.5 * (t3 - t2);
    }
}

__device__ void cgf_eval(const CgfView& v, double theta0, int dn1, int dn2, double2 out[6]) {
    const double x = 0.5 * dn1;
    const double y = (dn1 + 2.0 * dn2) * (0.5 * M_SQRT1_2);
    const double rho = sqrt(x * x + y * y);
    double phi = atan2(y, x);
    if (phi < 0.0) phi += 2.0 * M_PI;
    const double fp = phi / (2.0 * M_PI) * v.nphi;
    int jp = (int)floor(fp);
    const double tp = fp - jp;
    const double inv_c = M_SQRT2;    // 1 / c with c = a / sqrt 2, a = 1
    for (int c = 0; c < 6; ++c) out[c] = make_double2(0, 0);
    if (theta0 == 0.0) {
        for (int a = 0; a < 4; ++a) {
            const int jj = ((jp - 1 + a) % v.nphi + v.nphi) % v.nphi;
            const double wa = cr_w(tp, a);
            for (int c = 0; c < 6; ++c) out[c].x += wa * v.H[((int64_t)jj * (v.ns + 1) + v.ns) * 6 + c].x;
        }
        const double lr = log(rho);
        for (int c = 0; c < 6; ++c) out[c].x = (out[c].x - 2.0 * v.g0[c] * lr) * inv_c;
        return;
    }
    const double kappa = 2.0 * M_PI * theta0 * inv_c;
    const double s = kappa * rho;
    if (s > v.s_max) return;
    double ls = log(s);
    double extra = 0.0;       // below s_min: H(s) = H(s_min) - 2 G0 log(s / s_min)
    if (ls < v.ls_min) {
        extra = ls - v.ls_min;
        ls = v.ls_min;
    }
    const double fs = (ls - v.ls_min) / v.dls;
    int is = (int)floor(fs);
    double ts = fs - is;
    if (is >= v.ns - 1) {
        is = v.ns - 2;
        ts = 1.0;
    }
    for (int a = 0; a < 4; ++a) {
        const int jj = ((jp - 1 + a) % v.nphi + v.nphi) % v.nphi;
        const double wa = cr_w(tp, a);
        for (int b = 0; b < 4; ++b) {
            const int ii = min(max(is - 1 + b, 0), v.ns - 1);
            const double w = wa * cr_w(ts, b);
            const double2* h = v.H + ((int64_t)jj * (v.ns + 1) + ii) * 6;
            for (int c = 0; c < 6; ++c) {
                out[c].x += w * h[c].x;
                out[c].y += w * h[c].y;
            }
        }
    }
    const double unscale = exp(-exp(ls));      // table holds e^{s} H
    for (int c = 0; c < 6; ++c) {
        out[c].x *= unscale;
        out[c].y *= unscale;
    }
    if (extra != 0.0)
        for (int c = 0; c < 6; ++c) out[c].x -= 2.0 * v.g0[c] * extra;
    double sp, cp;
    sincospi(theta0 * dn1, &sp, &cp);
    for (int c = 0; c < 6; ++c) {
        const double re = out[c].x * cp - out[c].y * sp;
        const double im = out[c].x * sp + out[c].y * cp;
        out[c] = make_double2(re * inv_c, im * inv_c);
    }
}

__global__ void __launch_bounds__(NTL) k_cgf_points(CgfView v, const double* __restrict__ theta0,
                                                    const int32_t* __restrict__ d1,
                                                    const int32_t* __restrict__ d2, int n,
                                                    double2* __restrict__ out) {
    const int i = blockIdx.x * NTL + threadIdx.x;
    if (i >= n) return;
    double2 o[6];
    cgf_eval(v, theta0[i], d1[i], d2[i], o);
    for (int c = 0; c < 6; ++c) out[(int64_t)i * 6 + c] = o[c];
}

void launch_cgf_points(hipStream_t st, const CgfView& v, const double* theta0, const int32_t* d1,
                       const int32_t* d2, int n, double2* out) {
    if (n > 0)
        hipLaunchKernelGGL(k_cgf_points, dim3((n + NTL - 1) / NTL), dim3(NTL), 0, st, v, theta0, d1,
                           d2, n, out);
}

void launch_cgf_build(hipStream_t st, const CgfConst& k, const double* cpsi, const double* spsi,
                      const double* rhat, double* g0, double* g1, double* rem, const double2* ph0,
                      const double2* step, const double* k0s, double2* H) {
    hipLaunchKernelGGL(k_cgf_g, dim3((k.nphi + 1 + 63) / 64), dim3(64), 0, st, k, cpsi, spsi, rhat, g0, g1);
    const int64_t nrem = (int64_t)k.nphi * k.nzq;
    hipLaunchKernelGGL(k_cgf_rem, dim3((unsigned)((nrem + NTL - 1) / NTL)), dim3(NTL), 0, st, k, cpsi,
                       spsi, rhat, g0, g1, rem);
    const int nh = k.nphi * (k.ns + 1);
    hipLaunchKernelGGL(k_cgf_transform, dim3((nh + NTL - 1) / NTL), dim3(NTL), 0, st, k, rem, g0, g1, ph0,
                       step, k0s, H);
}

// ----------------------------------------------------------------------------------
// MLP 8 -> 128 -> 128 -> 128 -> 12, SiLU, FP32 training kernels.
// Parameter layout: per layer W [out][in] row-major, then b [out].
// ----------------------------------------------------------------------------------
__device__ inline float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float silu_d(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// out[s][o] = b[o] + sum_i in[s][i] W[o][i]; z stored, a = silu(z) unless last.
// A block takes FWD_S samples: W (transposed, [i][o]) and the input rows are staged in
// LDS, then each thread forms outputs (s, o) with o running fastest across the wave.
#define FWD_S 32
__global__ void __launch_bounds__(NTL) k_dense_fwd(const float* __restrict__ in, int n, int ni, int no,
                                                   const float* __restrict__ W,
                                                   const float* __restrict__ b,
                                                   float* __restrict__ z, float* __restrict__ a,
                                                   int last) {
    __shared__ float wt[MLP_H * MLP_H];
    __shared__ float xs[FWD_S * MLP_H];
    const int s0 = blockIdx.x * FWD_S;
    const int ns = min(FWD_S, n - s0);
    for (int e = threadIdx.x; e < ni * no; e += NTL) {
        const int o = e / ni, i = e - o * ni;
        wt[i * no + o] = W[e];
    }
    for (int e = threadIdx.x; e < ns * ni; e += NTL) xs[e] = in[(int64_t)s0 * ni + e];
    __syncthreads();
    for (int e = threadIdx.x; e < ns * no; e += NTL) {
        const int sl = e / no, o = e - sl * no;
        float acc = b[o];
        const float* x = xs + sl * ni;
        for (int i = 0; i < ni; ++i) acc = fmaf(x[i], wt[i * no + o], acc);
        const int64_t idx = (int64_t)(s0 + sl) * no + o;
        z[idx] = acc;
        a[idx] = last ? acc : silu(acc);
    }
}

// dz = da * silu'(z) (or da for the last layer).
__global__ void __launch_bounds__(NTL) k_dense_dz(const float* __restrict__ da,
                                                  const float* __restrict__ z, int64_t total,
                                                  float* __restrict__ dz, int last) {
    const int64_t idx = (int64_t)blockIdx.x * NTL + threadIdx.x;
    if (idx < total) dz[idx] = last ? da[idx] : da[idx] * silu_d(z[idx]);
}
// din[s][i] = sum_o dz[s][o] W[o][i].
__global__ void __launch_bounds__(NTL) k_dense_bwd_x(const float* __restrict__ dz, int n, int ni, int no,
                                                     const float* __restrict__ W,
                                                     float* __restrict__ din) {
    const int64_t idx = (int64_t)blockIdx.x * NTL + threadIdx.x;
    if (idx >= (int64_t)n * ni) return;
    const int s = (int)(idx / ni), i = (int)(idx - (int64_t)s * ni);
    float acc = 0.0f;
    const float* g = dz + (int64_t)s * no;
    for (int o = 0; o < no; ++o) acc = fmaf(g[o], W[(int64_t)o * ni + i], acc);
    din[idx] = acc;
}
// dW[o][i] = sum_s dz[s][o] in[s][i]; db[o] = sum_s dz[s][o].  The samples are cut into
// gridDim.y chunks; each chunk's FP64 partial sum goes to part[chunk][o * (ni + 1) + i],
// and k_dense_bwd_sum adds the chunks in fixed order (deterministic result).
__global__ void __launch_bounds__(NTL) k_dense_bwd_w(const float* __restrict__ dz,
                                                     const float* __restrict__ in, int n, int ni,
                                                     int no, int chunk, double* __restrict__ part) {
    const int idx = blockIdx.x * NTL + threadIdx.x;
    const int nw = no * (ni + 1);
    if (idx >= nw) return;
    const int o = idx / (ni + 1), i = idx - o * (ni + 1);
    const int sa = blockIdx.y * chunk, sb = min(n, sa + chunk);
    double acc = 0.0;
    if (i < ni)
        for (int s = sa; s < sb; ++s) acc += (double)dz[(int64_t)s * no + o] * in[(int64_t)s * ni + i];
    else
        for (int s = sa; s < sb; ++s) acc += dz[(int64_t)s * no + o];
    part[(int64_t)blockIdx.y * nw + idx] = acc;
}
__global__ void __launch_bounds__(NTL) k_dense_bwd_sum(const double* __restrict__ part, int nchunk, int ni,
                                                       int no, float* __restrict__ dW,
                                                       float* __restrict__ db) {
    const int idx = blockIdx.x * NTL + threadIdx.x;
    const int nw = no * (ni + 1);
    if (idx >= nw) return;
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += part[(int64_t)c * nw + idx];
    const int o = idx / (ni + 1), i = idx - o * (ni + 1);
    if (i < ni) dW[(int64_t)o * ni + i] = (float)acc;
    else db[o] = (float)acc;
}
#define BWD_CHUNKS 64

// Loss: mean over samples of sum over outputs of (w (y - t))^2; dy = 2 w^2 (y - t) / n.
__global__ void __launch_bounds__(NTL) k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              const float* __restrict__ wt, int n, int no,
                                              float* __restrict__ dy, double* __restrict__ part) {
    __shared__ double red[NTL];
    double acc = 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * NTL + threadIdx.x; idx < (int64_t)n * no;
         idx += (int64_t)gridDim.x * NTL) {
        const int s = (int)(idx / no);
        const float w = wt ? wt[s] : 1.0f;
        const float d = y[idx] - t[idx];
        dy[idx] = 2.0f * w * w * d / n;
        acc += (double)(w * d) * (w * d);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = NTL / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_loss_final(const double* __restrict__ part, int np, int n, float* __restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < np; ++i) s += part[i];
        *loss = (float)(s / n);
    }
}

__global__ void __launch_bounds__(NTL) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int n,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
    const int i = blockIdx.x * NTL + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static const int MLP_SIZES[5] = {MLP_IN, MLP_H, MLP_H, MLP_H, MLP_OUT};

static int64_t layer_off(int l) {
    int64_t off = 0;
    for (int k = 0; k < l; ++k) off += (int64_t)MLP_SIZES[k + 1] * MLP_SIZES[k] + MLP_SIZES[k + 1];
    return off;
}

// Workspace: activations z_l, a_l for l = 1..4 and gradients, n samples.
int64_t mlp_workspace_floats(int n) {
    int64_t t = 0;
    for (int l = 1; l <= 4; ++l) t += 4 * (int64_t)n * MLP_SIZES[l];   // z, a, dz, da
    // loss partials (256 doubles) and the weight-gradient chunk partials (doubles)
    return t + (int64_t)n * MLP_H + 4096 + 2LL * BWD_CHUNKS * MLP_H * (MLP_H + 1);
}

void launch_mlp_forward(hipStream_t st, const float* params, const float* x, int n, float* ws,
                        float* y) {
    const float* in = x;
    float* p = ws;
    for (int l = 0; l < 4; ++l) {
        const int ni = MLP_SIZES[l], no = MLP_SIZES[l + 1];
        float* z = p;
        float* a = (l == 3 && y) ? y : p + (int64_t)n * no;
        const int64_t tot = (int64_t)n * no;
        (void)tot;
        hipLaunchKernelGGL(k_dense_fwd, dim3((unsigned)((n + FWD_S - 1) / FWD_S)), dim3(NTL), 0, st, in, n, ni,
                           no, params + layer_off(l), params + layer_off(l) + (int64_t)no * ni, z, a,
                           l == 3 ? 1 : 0);
        in = a;
        p += 4 * (int64_t)n * no;
    }
}

void launch_mlp_loss_grad(hipStream_t st, const float* params, const float* x, const float* t,
                          const float* w, int n, float* ws, float* grad, float* loss) {
    launch_mlp_forward(st, params, x, n, ws, nullptr);
    // pointers per layer
    float* zl[4];
    float* al[4];
    float* dzl[4];
    float* dal[4];
    float* p = ws;
    for (int l = 0; l < 4; ++l) {
        const int no = MLP_SIZES[l + 1];
        zl[l] = p;
        al[l] = p + (int64_t)n * no;
        dzl[l] = p + 2 * (int64_t)n * no;
        dal[l] = p + 3 * (int64_t)n * no;
        p += 4 * (int64_t)n * no;
    }
    double* part = (double*)(p + (int64_t)n * MLP_H);
    double* wpart = part + 2048;              // after the 4096 floats of loss partials
    const int nb = 256;
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(NTL), 0, st, al[3], t, w, n, MLP_OUT, dal[3], part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, part, nb, n, loss);
    for (int l = 3; l >= 0; --l) {
        const int ni = MLP_SIZES[l], no = MLP_SIZES[l + 1];
        const float* Wl = params + layer_off(l);
        const int64_t tot = (int64_t)n * no;
        hipLaunchKernelGGL(k_dense_dz, dim3((unsigned)((tot + NTL - 1) / NTL)), dim3(NTL), 0, st, dal[l],
                           zl[l], tot, dzl[l], l == 3 ? 1 : 0);
        const float* in = (l == 0) ? x : al[l - 1];
        const int nw = no * (ni + 1);
        const int chunk = std::max(64, (n + BWD_CHUNKS - 1) / BWD_CHUNKS);
        const int nchunk = (n + chunk - 1) / chunk;
        hipLaunchKernelGGL(k_dense_bwd_w, dim3((nw + NTL - 1) / NTL, nchunk), dim3(NTL), 0, st, dzl[l], in, n,
                           ni, no, chunk, wpart);
        hipLaunchKernelGGL(k_dense_bwd_sum, dim3((nw + NTL - 1) / NTL), dim3(NTL), 0, st, wpart, nchunk, ni, no,
                           grad + layer_off(l), grad + layer_off(l) + (int64_t)no * ni);
        if (l > 0) {
            const int64_t ti = (int64_t)n * ni;
            hipLaunchKernelGGL(k_dense_bwd_x, dim3((unsigned)((ti + NTL - 1) / NTL)), dim3(NTL), 0, st, dzl[l],
                               n, ni, no, Wl, dal[l - 1]);
        }
    }
}

void launch_adam(hipStream_t st, float* p, const float* g, float* m, float* v, int n, float lr, int step) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + NTL - 1) / NTL), dim3(NTL), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1,
                       c2);
}

// ----------------------------------------------------------------------------------
// Training samples and the surrogate table generator.
// Features of (theta0, dn1, dn2): (cos phi, sin phi, cos 2phi, sin 2phi, cos 4phi,
// sin 4phi, r_c / rho, 8 theta0); the low angular harmonics of the cubic anisotropy
// are given explicitly.
// Target / output: exp(-i pi theta0 dn1) (G^_lgf - G^_cgf) / env, 6 complex components
// (xx yy zz xy xz yz) as 12 reals, with env = env_mode[t] = exp(-s_exact) times the
// largest block of table mode t: the learned band starts where the lattice blocks fall
// below that, so the targets are of order one or less and the network's absolute error
// is spread evenly over the band (the continuum is zero beyond kappa rho = 40, where the
// lattice values at large theta0 still matter; a relative envelope would vanish there).
// ----------------------------------------------------------------------------------
__device__ inline void sur_features(double theta0, int dn1, int dn2, double r_c, float f[MLP_IN],
                                    double* rho_out) {
    const double x = 0.5 * dn1;
    const double y = (dn1 + 2.0 * dn2) * (0.5 * M_SQRT1_2);
    const double rho = sqrt(x * x + y * y);
    const double c1 = x / rho, s1 = y / rho;
    const double c2 = c1 * c1 - s1 * s1, s2 = 2.0 * s1 * c1;
    f[0] = (float)c1;
    f[1] = (float)s1;
    f[2] = (float)c2;
    f[3] = (float)s2;
    f[4] = (float)(c2 * c2 - s2 * s2);
    f[5] = (float)(2.0 * s2 * c2);
    f[6] = (float)(r_c / rho);
    f[7] = (float)(8.0 * theta0);
    *rho_out = rho;
}



__global__ void __launch_bounds__(NTL) k_sur_samples(CgfView v, const double2* __restrict__ tab,
                                                     int64_t n_off, int nz_tab,
                                                     const int32_t* __restrict__ d1,
                                                     const int32_t* __restrict__ d2,
                                                     const int32_t* __restrict__ pick_t,
                                                     const int32_t* __restrict__ pick_o, int n,
                                                     double r_c, const double* __restrict__ env_mode,
                                                     float* __restrict__ x, float* __restrict__ t) {
    const int i = blockIdx.x * NTL + threadIdx.x;
    if (i >= n) return;
    const int tm = pick_t[i];
    const int64_t o = pick_o[i];
    const double theta0 = (double)tm / nz_tab;
    double2 g[6];
    cgf_eval(v, theta0, d1[o], d2[o], g);
    float f[MLP_IN];
    double rho;
    sur_features(theta0, d1[o], d2[o], r_c, f, &rho);
    const double env = env_mode[tm];
    double sp, cp;
    sincospi(theta0 * d1[o], &sp, &cp);
    const double2* l = tab + ((int64_t)tm * n_off + o) * 6;
    for (int a = 0; a < MLP_IN; ++a) x[(int64_t)i * MLP_IN + a] = f[a];
    for (int c = 0; c < 6; ++c) {
        const double dr = l[c].x - g[c].x, di = l[c].y - g[c].y;
        // multiply by exp(-i pi theta0 dn1)
        t[(int64_t)i * 12 + 2 * c] = (float)((dr * cp + di * sp) / env);
        t[(int64_t)i * 12 + 2 * c + 1] = (float)((di * cp - dr * sp) / env);
    }
}

void launch_sur_samples(hipStream_t st, const CgfView& v, const double2* tab, int64_t n_off, int nz_tab,
                        const int32_t* d1, const int32_t* d2, const int32_t* pick_t,
                        const int32_t* pick_o, int n, double r_c, const double* env_mode, float* x, float* t) {
    if (n > 0)
        hipLaunchKernelGGL(k_sur_samples, dim3((n + NTL - 1) / NTL), dim3(NTL), 0, st, v, tab, n_off, nz_tab,
                           d1, d2, pick_t, pick_o, n, r_c, env_mode, x, t);
}

// MLP forward of one sample, weights transposed ([in][out], read with wave-uniform
// addresses) in BF16 (inference) or FP32 (the control that isolates the weights'
// rounding), FP32 accumulation.  The hidden vector of each thread lives in its own LDS
// column hl[i * stride]; every layer reads its inputs from there and overwrites them with
// its outputs (the column is private to the thread, so no barrier is needed).
#define MLP_BLOCK 64
__device__ inline float wval(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ inline float wval(float x) { return x; }

template <typename WT>
struct MlpW {
    const WT* w1t;   // [8][128]
    const WT* w2t;   // [128][128]
    const WT* w3t;   // [128][128]
    const WT* w4t;   // [128][12]
    const float* b1;
    const float* b2;
    const float* b3;
    const float* b4;
};

template <typename WT>
__device__ inline MlpW<WT> mlp_view(const WT* w, const float* bias) {
    MlpW<WT> m;
    m.w1t = w;
    m.w2t = m.w1t + MLP_IN * MLP_H;
    m.w3t = m.w2t + MLP_H * MLP_H;
    m.w4t = m.w3t + MLP_H * MLP_H;
    m.b1 = bias;
    m.b2 = m.b1 + MLP_H;
    m.b3 = m.b2 + MLP_H;
    m.b4 = m.b3 + MLP_H;
    return m;
}

template <typename WT>
__device__ inline void mlp_hidden(const WT* __restrict__ wt, const float* __restrict__ b, float* hl, int stride) {
    float acc[MLP_H];
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) acc[o] = b[o];
    for (int i = 0; i < MLP_H; ++i) {
        const float v = hl[i * stride];
        const WT* w = wt + i * MLP_H;
#pragma unroll
        for (int o = 0; o < MLP_H; ++o) acc[o] = fmaf(wval(w[o]), v, acc[o]);
    }
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) hl[o * stride] = silu(acc[o]);
}

template <typename WT>
__device__ void mlp_eval(const MlpW<WT>& m, const float f[MLP_IN], float* hl, int stride, float y[MLP_OUT]) {
    {
        float acc[MLP_H];
#pragma unroll
        for (int o = 0; o < MLP_H; ++o) {
            float a = m.b1[o];
#pragma unroll
            for (int i = 0; i < MLP_IN; ++i) a = fmaf(wval(m.w1t[i * MLP_H + o]), f[i], a);
            acc[o] = a;
        }
#pragma unroll
        for (int o = 0; o < MLP_H; ++o) hl[o * stride] = silu(acc[o]);
    }
    mlp_hidden(m.w2t, m.b2, hl, stride);
    mlp_hidden(m.w3t, m.b3, hl, stride);
#pragma unroll
    for (int o = 0; o < MLP_OUT; ++o) y[o] = m.b4[o];
    for (int i = 0; i < MLP_H; ++i) {
        const float v = hl[i * stride];
#pragma unroll
        for (int o = 0; o < MLP_OUT; ++o) y[o] = fmaf(wval(m.w4t[i * MLP_OUT + o]), v, y[o]);
    }
}

// Far-field block (CGF, optionally + the network's correction with a unit envelope) at
// arbitrary points.
template <typename WT>
__global__ void __launch_bounds__(MLP_BLOCK) k_sur_points(CgfView v, const WT* __restrict__ wt,
                                                          const float* __restrict__ bias, int use_mlp,
                                                          double r_c, const double* __restrict__ theta0,
                                                          const int32_t* __restrict__ d1,
                                                          const int32_t* __restrict__ d2, int n,
                                                          double2* __restrict__ out) {
    __shared__ float hl[MLP_H * MLP_BLOCK];
    const MlpW<WT> m = mlp_view(wt, bias);
    const int i = blockIdx.x * MLP_BLOCK + threadIdx.x;
    if (i >= n) return;
    double2 g[6];
    cgf_eval(v, theta0[i], d1[i], d2[i], g);
    float f[MLP_IN], y[MLP_OUT];
    double rho;
    sur_features(theta0[i], d1[i], d2[i], r_c, f, &rho);
    if (use_mlp && rho > r_c) {
        mlp_eval(m, f, hl + threadIdx.x, MLP_BLOCK, y);
        double sp, cp;
        sincospi(theta0[i] * d1[i], &sp, &cp);
        for (int c = 0; c < 6; ++c) {
            const double cr = y[2 * c], ci = y[2 * c + 1];
            g[c].x += cr * cp - ci * sp;
            g[c].y += cr * sp + ci * cp;
        }
    }
    for (int c = 0; c < 6; ++c) out[(int64_t)i * 6 + c] = g[c];
}

void launch_sur_points(hipStream_t st, const CgfView& v, const MlpInfer& w, int use_mlp, double r_c,
                       const double* theta0, const int32_t* d1,
                       const int32_t* d2, int n, double2* out) {
    if (n <= 0) return;
    const dim3 grid((n + MLP_BLOCK - 1) / MLP_BLOCK);
    if (w.wf)
        hipLaunchKernelGGL(k_sur_points<float>, grid, dim3(MLP_BLOCK), 0, st, v, w.wf, w.bias, use_mlp, r_c,
                           theta0, d1, d2, n, out);
    else
        hipLaunchKernelGGL(k_sur_points<unsigned short>, grid, dim3(MLP_BLOCK), 0, st, v, w.wb, w.bias, use_mlp,
                           r_c, theta0, d1, d2, n, out);
}

// The exact prefix of each table mode t0 .. t0+nt-1 into the generated slice: one
// contiguous run per mode (ragged table: mode t at ex_off[t], n_exact[t] offsets).
__global__ void __launch_bounds__(256) k_sur_copy_exact(const double2* __restrict__ exact_tab,
                                                        const int64_t* __restrict__ ex_off,
                                                        const int32_t* __restrict__ n_exact, int t0, int64_t n_off,
                                                        double2* __restrict__ out) {
    const int tl = blockIdx.y, tm = t0 + tl;
    const int64_t n = (int64_t)n_exact[tm] * 6;
    const double2* src = exact_tab + ex_off[tm] * 6;
    double2* dst = out + (int64_t)tl * n_off * 6;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

// Table slice generator of the surrogate form: table modes t0 .. t0+nt-1 for every
// offset o (offsets numbered by increasing rho; every band below is a prefix).
// o < n_exact[t]: the exact lattice value (copied from the ragged table by
// k_sur_copy_exact; this kernel starts at o0, the smallest n_exact of the chunk);
// o < n_learn[t]: continuum + learned correction (only out to rho_learn, the largest distance
// of the training data: no extrapolation); o < n_need[t]: continuum alone; beyond:
// zero, not written (the product treats offsets at or beyond n_need[t] as zero).
template <typename WT>
__global__ void __launch_bounds__(MLP_BLOCK) k_sur_generate(CgfView v, const WT* __restrict__ wt,
                                                            const float* __restrict__ bias, double r_c,
                                                            const double* __restrict__ env_mode, double rho_learn,
                                                            int nz_tab, int t0,
                                                            const int32_t* __restrict__ n_exact,
                                                            const int32_t* __restrict__ n_learn,
                                                            int64_t o0, int64_t n_off,
                                                            const int32_t* __restrict__ n_need,
                                                            const int32_t* __restrict__ d1,
                                                            const int32_t* __restrict__ d2,
                                                            double2* __restrict__ out, int band_done) {
    __shared__ float hl[MLP_H * MLP_BLOCK];
    const MlpW<WT> m = mlp_view(wt, bias);
    const int tl = blockIdx.y;
    const int tm = t0 + tl;
    const int64_t o = o0 + (int64_t)blockIdx.x * MLP_BLOCK + threadIdx.x;
    if (o >= n_off) return;
    double2* dst = out + ((int64_t)tl * n_off + o) * 6;
    if (o < n_exact[tm]) return;      // copied by k_sur_copy_exact
    if (band_done && o < n_learn[tm]) return;     // made by k_sur_learned
    if (o >= n_need[tm]) return;      // zero by definition; the product does not read it
    const double theta0 = (double)tm / nz_tab;
    double2 g[6];
    cgf_eval(v, theta0, d1[o], d2[o], g);
    float f[MLP_IN], y[MLP_OUT];
    double rho;
    sur_features(theta0, d1[o], d2[o], r_c, f, &rho);
    const double env = env_mode[tm];
    if (o < n_learn[tm] && rho <= rho_learn) {
        mlp_eval(m, f, hl + threadIdx.x, MLP_BLOCK, y);
        double sp, cp;
        sincospi(theta0 * d1[o], &sp, &cp);
        for (int c = 0; c < 6; ++c) {
            const double cr = env * y[2 * c], ci = env * y[2 * c + 1];
            g[c].x += cr * cp - ci * sp;
            g[c].y += cr * sp + ci * cp;
        }
    }
    for (int c = 0; c < 6; ++c) dst[c] = g[c];
}

// ----------------------------------------------------------------------------------
// Learned band on MFMA: the network's layers are dense products over a batch of samples,
// run as v_mfma_f32_16x16x32_bf16 (weights and activations in BF16, FP32 accumulation,
// biases and SiLU in FP32).  Weights in fragment order (k_mlp_to_mfma): layer l's
// fragment (row block rb, K block kb) is 64 lanes x 8 BF16, lane L holding
// W[16 rb + L % 16][32 kb + 8 (L / 16) + j]; layers 8 -> 128 (K padded to 32), 128 ->
// 128 twice, 128 -> 12 (rows padded to 16).  One wave takes 64 samples (one per lane for
// the continuum, the features and the final combination) and runs the network on them
// in four groups of 16 (the MFMA columns); between layers the activations go through a
// per-wave LDS buffer [sample][row] (row stride 136: the lanes' 8- and 16-byte accesses
// fall on distinct banks), which turns the accumulator layout (rows 16 rb + 4 (L / 16) +
// j) into the operand layout (rows 32 kb + 8 (L / 16) + j).
// ----------------------------------------------------------------------------------
#define LRN_WAVES 4
#define LRN_ACT 136
#define LRN_FRAGS (8 + 32 + 32 + 4)

__device__ inline unsigned short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);       // round to nearest even (finite values)
    return (unsigned short)(u >> 16);
}

__device__ inline bf8_t frag_at(const unsigned short* p) { return *(const bf8_t*)p; }

// bias + SiLU of one layer's accumulators, into the activation buffer act[sample][row]
__device__ inline void put_act(unsigned short* act, const f4_t (&acc)[8], const float* __restrict__ b, int lane) {
    const int n = lane & 15, q = lane >> 4;
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
        unsigned short h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) h[j] = to_bf16(silu(acc[rb][j] + b[16 * rb + 4 * q + j]));
        uint2 pk;
        pk.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
        pk.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
        *(uint2*)(act + n * LRN_ACT + 16 * rb + 4 * q) = pk;
    }
}

// Offsets n_exact[t] .. n_learn[t] - 1 of table modes t0 .. t0 + nt - 1: continuum + the
// network's correction (within rho_learn; the continuum alone beyond), as k_sur_generate.
__global__ void __launch_bounds__(64 * LRN_WAVES) k_sur_learned(CgfView v, const unsigned short* __restrict__ wm,
                                                               const float* __restrict__ bias, double r_c,
                                                               const double* __restrict__ env_mode,
                                                               double rho_learn, int nz_tab, int t0,
                                                               const int32_t* __restrict__ n_exact,
                                                               const int32_t* __restrict__ n_learn, int64_t n_off,
                                                               const int32_t* __restrict__ d1,
                                                               const int32_t* __restrict__ d2,
                                                               double2* __restrict__ out) {
    __shared__ __align__(16) unsigned short feat[LRN_WAVES][64][8];
    __shared__ __align__(16) unsigned short act[LRN_WAVES][16 * LRN_ACT];
    __shared__ float yo[LRN_WAVES][64][MLP_OUT];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tl = blockIdx.y, tm = t0 + tl;
    const int64_t o = (int64_t)n_exact[tm] + ((int64_t)blockIdx.x * LRN_WAVES + wave) * 64 + lane;
    const bool live = o < n_learn[tm];
    const double theta0 = (double)tm / nz_tab;
    double2 g[6];
    float f[MLP_IN];
    double rho = 0.0;
    bool use = false;
    if (live) {
        cgf_eval(v, theta0, d1[o], d2[o], g);
        sur_features(theta0, d1[o], d2[o], r_c, f, &rho);
        use = rho <= rho_learn;
    }
#pragma unroll
    for (int a = 0; a < MLP_IN; ++a) feat[wave][lane][a] = use ? to_bf16(f[a]) : (unsigned short)0;
    const int any = __syncthreads_or(use ? 1 : 0);       // work-group uniform
    if (any) {
        const int n = lane & 15, q = lane >> 4;
        unsigned short* aw = act[wave];
        const f4_t zero = {0.f, 0.f, 0.f, 0.f};
        for (int sb = 0; sb < 4; ++sb) {
            f4_t acc[8];
            // layer 1: the 8 features are K rows 0..7 (the first lane quarter), zeros beyond
            bf8_t b1;
            if (q == 0) b1 = *(const bf8_t*)&feat[wave][16 * sb + n][0];
            else b1 = (bf8_t){};
#pragma unroll
            for (int rb = 0; rb < 8; ++rb)
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag_at(wm + rb * 512 + lane * 8), b1, zero, 0, 0, 0);
            put_act(aw, acc, bias, lane);
            __syncthreads();
            // layers 2 and 3
            for (int l = 0; l < 2; ++l) {
                bf8_t bk[4];
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) bk[kb] = *(const bf8_t*)(aw + n * LRN_ACT + 32 * kb + 8 * q);
                __syncthreads();             // every lane has its operands before any overwrite
                const unsigned short* wl = wm + (8 + 32 * l) * 512;
#pragma unroll
                for (int rb = 0; rb < 8; ++rb) {
                    acc[rb] = zero;
#pragma unroll
                    for (int kb = 0; kb < 4; ++kb)
                        acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag_at(wl + (rb * 4 + kb) * 512 + lane * 8),
                                                                          bk[kb], acc[rb], 0, 0, 0);
                }
                put_act(aw, acc, bias + MLP_H * (l + 1), lane);
                __syncthreads();
            }
            // layer 4: 12 outputs (rows 12..15 of the fragment are zero)
            bf8_t bk[4];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) bk[kb] = *(const bf8_t*)(aw + n * LRN_ACT + 32 * kb + 8 * q);
            f4_t a4 = zero;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                a4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag_at(wm + (72 + kb) * 512 + lane * 8), bk[kb], a4, 0, 0,
                                                             0);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 4 * q + j;
                if (row < MLP_OUT) yo[wave][16 * sb + n][row] = a4[j] + bias[3 * MLP_H + row];
            }
            __syncthreads();                 // layer 4 has read act; yo complete after the last group
        }
    }
    if (!live) return;
    if (use) {
        const double env = env_mode[tm];
        double sp, cp;
        sincospi(theta0 * d1[o], &sp, &cp);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double cr = env * yo[wave][lane][2 * c], ci = env * yo[wave][lane][2 * c + 1];
            g[c].x += cr * cp - ci * sp;
            g[c].y += cr * sp + ci * cp;
        }
    }
    double2* dst = out + ((int64_t)tl * n_off + o) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) dst[c] = g[c];
}

// FP32 weights -> BF16 fragments of k_sur_learned (round to nearest even; zeros in the
// padding).
__global__ void k_mlp_to_mfma(const float* __restrict__ params, unsigned short* __restrict__ wm) {
    for (int e = threadIdx.x; e < LRN_FRAGS * 512; e += blockDim.x) {
        const int fr = e / 512, rem = e - fr * 512, lane = rem / 8, j = rem - lane * 8;
        int l, rb, kb;
        if (fr < 8) { l = 0; rb = fr; kb = 0; }
        else if (fr < 40) { l = 1; rb = (fr - 8) / 4; kb = (fr - 8) % 4; }
        else if (fr < 72) { l = 2; rb = (fr - 40) / 4; kb = (fr - 40) % 4; }
        else { l = 3; rb = 0; kb = fr - 72; }
        const int ni = (l == 0) ? MLP_IN : MLP_H, no = (l == 3) ? MLP_OUT : MLP_H;
        int64_t off = 0;
        if (l > 0) off += (int64_t)MLP_H * MLP_IN + MLP_H;
        if (l > 1) off += (int64_t)MLP_H * MLP_H + MLP_H;
        if (l > 2) off += (int64_t)MLP_H * MLP_H + MLP_H;
        const int row = 16 * rb + (lane & 15), col = 32 * kb + 8 * (lane >> 4) + j;
        wm[e] = (row < no && col < ni) ? to_bf16(params[off + (int64_t)row * ni + col]) : (unsigned short)0;
    }
}

void launch_mlp_to_mfma(hipStream_t st, const float* params, unsigned short* wm) {
    hipLaunchKernelGGL(k_mlp_to_mfma, dim3(1), dim3(256), 0, st, params, wm);
}

void launch_sur_generate(hipStream_t st, const CgfView& v, const MlpInfer& w, double r_c, const double* env_mode,
                         double rho_learn, int nz_tab, int t0, int nt, const double2* exact_tab, const int64_t* ex_off,
                         const int32_t* n_exact, const int32_t* n_learn, int64_t n_off,
                         const int32_t* n_need, const int32_t* d1, const int32_t* d2, double2* out,
                         int64_t min_exact, int64_t max_exact, int64_t min_learn, int64_t max_band, int64_t max_need) {
    if (nt <= 0) return;
    if (max_exact > 0) {
        const int64_t per = (max_exact * 6 + 255) / 256;
        hipLaunchKernelGGL(k_sur_copy_exact, dim3((unsigned)std::min<int64_t>(per, 1024), nt), dim3(256), 0, st,
                           exact_tab, ex_off, n_exact, t0, n_off, out);
    }
    if (w.wf) {          // FP32 control: the whole non-exact prefix on the SIMT network
        if (max_need <= min_exact) return;
        dim3 grid((unsigned)((max_need - min_exact + MLP_BLOCK - 1) / MLP_BLOCK), nt);
        hipLaunchKernelGGL(k_sur_generate<float>, grid, dim3(MLP_BLOCK), 0, st, v, w.wf, w.bias, r_c, env_mode, rho_learn,
                           nz_tab, t0, n_exact, n_learn, min_exact, n_off, n_need, d1, d2, out, 0);
        return;
    }
    if (max_band > 0) {   // learned band on MFMA
        const int64_t per = (max_band + 64 * LRN_WAVES - 1) / (64 * LRN_WAVES);
        hipLaunchKernelGGL(k_sur_learned, dim3((unsigned)per, nt), dim3(64 * LRN_WAVES), 0, st, v, w.wm, w.bias, r_c,
                           env_mode, rho_learn, nz_tab, t0, n_exact, n_learn, n_off, d1, d2, out);
    }
    if (max_need <= min_learn) return;     // continuum alone beyond the learned band
    dim3 grid((unsigned)((max_need - min_learn + MLP_BLOCK - 1) / MLP_BLOCK), nt);
    hipLaunchKernelGGL(k_sur_generate<unsigned short>, grid, dim3(MLP_BLOCK), 0, st, v, w.wb, w.bias, r_c,
                       env_mode, rho_learn, nz_tab, t0, n_exact, n_learn, min_learn, n_off, n_need, d1, d2, out, 1);
}

// FP32 weights -> transposed bf16 (round to nearest even) and biases, for inference.
__global__ void k_mlp_to_bf16(const float* __restrict__ params, unsigned short* __restrict__ wb,
                              float* __restrict__ bias) {
    const int sizes[5] = {MLP_IN, MLP_H, MLP_H, MLP_H, MLP_OUT};
    int64_t off = 0, ow = 0, ob = 0;
    for (int l = 0; l < 4; ++l) {
        const int ni = sizes[l], no = sizes[l + 1];
        for (int e = threadIdx.x; e < no * ni; e += blockDim.x) {
            const int o = e / ni, i = e - o * ni;           // W [o][i] -> Wt [i][o]
            unsigned u = __float_as_uint(params[off + e]);
            u += 0x7FFFu + ((u >> 16) & 1u);
            wb[ow + (int64_t)i * no + o] = (unsigned short)(u >> 16);
        }
        for (int i = threadIdx.x; i < no; i += blockDim.x) bias[ob + i] = params[off + (int64_t)no * ni + i];
        off += (int64_t)no * ni + no;
        ow += (int64_t)no * ni;
        ob += no;
    }
}

void launch_mlp_to_bf16(hipStream_t st, const float* params, unsigned short* wb, float* bias) {
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3(1), dim3(256), 0, st, params, wb, bias);
}

// FP32 weights -> transposed FP32 weights and biases (the inference control without the
// BF16 rounding of the weights).
__global__ void k_mlp_to_f32t(const float* __restrict__ params, float* __restrict__ wf, float* __restrict__ bias) {
    const int sizes[5] = {MLP_IN, MLP_H, MLP_H, MLP_H, MLP_OUT};
    int64_t off = 0, ow = 0, ob = 0;
    for (int l = 0; l < 4; ++l) {
        const int ni = sizes[l], no = sizes[l + 1];
        for (int e = threadIdx.x; e < no * ni; e += blockDim.x) {
            const int o = e / ni, i = e - o * ni;
            wf[ow + (int64_t)i * no + o] = params[off + e];
        }
        for (int i = threadIdx.x; i < no; i += blockDim.x) bias[ob + i] = params[off + (int64_t)no * ni + i];
        off += (int64_t)no * ni + no;
        ow += (int64_t)no * ni;
        ob += no;
    }
}

void launch_mlp_to_f32t(hipStream_t st, const float* params, float* wf, float* bias) {
    hipLaunchKernelGGL(k_mlp_to_f32t, dim3(1), dim3(256), 0, st, params, wf, bias);
}
