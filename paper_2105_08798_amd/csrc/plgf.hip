// Real-space periodic lattice Green function (Section 3.1, eqs. G~inf, plgf_conv, plgf_poly,
// plgf_rich; Appendix B): the Green function of the infinite lattice within r_cut, the
// continuum (Kelvin) Green function beyond, the image sum along the line with the images
// of the origin subtracted, and Richardson extrapolation of its partial sums.
//
// Within r_cut the infinite-lattice function is taken from the L x L x L torus of the
// primitive cell: G_L(n) = L^-3 sum_{theta != 0} D(theta)^{-1} cos(2 pi theta.n), theta on
// the L^3 grid (Appendix B's inverse transform, discretised), minus the constant C that
// joins it to the continuum: C = mean of G_L - G_cgf over the lattice vectors of the shell
// r_cut < |r| <= r_match.  Lattice vectors are primitive-basis integers n (b0 along the
// line); radii are compared as 4 |B n|^2, an integer for fcc, so table membership is exact.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "elastic.h"
#include "kernels.h"

#define NTP 256
#define PLGF_MAX_IMAGES 16

static thread_local std::string g_perr;

static fbc_status pfail(fbc_status s, const std::string& m) {
    g_perr = m;
    return s;
}

#define PCHK(expr)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return pfail(FBC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct PlgfConst {
    double c11, c12, c44;
    int npsi;
    int r2x4_cut;
    int lo[3], span[3];          // index-map box: n_i in [lo_i, lo_i + span_i)
};

// 4 |B n|^2 with B n = (n0 + n1 + n2, n2 - n0, n1) / 2 in cube axes (a = 1)
__host__ __device__ inline int four_r2(int n0, int n1, int n2) {
    const int a = n0 + n1 + n2, b = n2 - n0;
    return a * a + b * b + n1 * n1;
}

__device__ inline void cube_pos(int n0, int n1, int n2, double x[3]) {
    x[0] = 0.5 * (n0 + n1 + n2);
    x[1] = 0.5 * (n2 - n0);
    x[2] = 0.5 * n1;
}

__device__ inline int table_index(const int* __restrict__ map, const PlgfConst& k, int n0, int n1, int n2) {
    const int a = n0 - k.lo[0], b = n1 - k.lo[1], c = n2 - k.lo[2];
    if (a < 0 || b < 0 || c < 0 || a >= k.span[0] || b >= k.span[1] || c >= k.span[2]) return -1;
    return map[((int64_t)a * k.span[1] + b) * k.span[2] + c];
}

// Fixed-order tree sum of six values over the work group (deterministic).
__device__ inline void block_sum6(double v[6], double* red) {
    for (int c = 0; c < 6; ++c) red[c * NTP + threadIdx.x] = v[c];
    __syncthreads();
    for (int s = NTP / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 6; ++c) red[c * NTP + threadIdx.x] += red[c * NTP + threadIdx.x + s];
        __syncthreads();
    }
    for (int c = 0; c < 6; ++c) v[c] = red[c * NTP];
    __syncthreads();
}

// G_L at the lattice vectors pts[p] (one work group per point).  D(theta) from the 12
// bonds, sin(pi j / L) and cos(2 pi j / L) from tables (phases reduced modulo L exactly).
__global__ void __launch_bounds__(NTP) k_plgf_torus(const int32_t* __restrict__ pts, int logL,
                                                    const double* __restrict__ sn,
                                                    const double* __restrict__ cs, BondTable bt,
                                                    double* __restrict__ out) {
    __shared__ double red[6 * NTP];
    const int p = blockIdx.x;
    const int mask = (1 << logL) - 1;
    const int q0 = pts[3 * p], q1 = pts[3 * p + 1], q2 = pts[3 * p + 2];
    const int64_t total = (int64_t)1 << (3 * logL);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t idx = 1 + threadIdx.x; idx < total; idx += NTP) {        // theta = 0 dropped
        const int k0 = (int)(idx >> (2 * logL)), k1 = (int)((idx >> logL) & mask), k2 = (int)(idx & mask);
        double d[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 12; ++b) {
            const double s = sn[(k0 * bt.n[b][0] + k1 * bt.n[b][1] + k2 * bt.n[b][2]) & mask];
            const double w = 2.0 * s * s;
#pragma unroll
            for (int c = 0; c < 6; ++c) d[c] += w * bt.p[b][c];
        }
        double o[6];
        sym_inverse(d, o);
        const double ph = cs[(k0 * q0 + k1 * q1 + k2 * q2) & mask];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += o[c] * ph;
    }
    block_sum6(acc, red);
    if (threadIdx.x < 6) out[6 * p + threadIdx.x] = acc[threadIdx.x] / (double)total;
}

// C = mean over the shell of G_L - G_cgf; table = G_L - C (one work group).
__global__ void __launch_bounds__(NTP) k_plgf_match(const int32_t* __restrict__ shell,
                                                    const double* __restrict__ gl_shell, int n_shell,
                                                    const double* __restrict__ gl_table, int n_table,
                                                    PlgfConst k, const double* __restrict__ cpsi,
                                                    const double* __restrict__ spsi,
                                                    double* __restrict__ c_out, double* __restrict__ table) {
    __shared__ double red[6 * NTP];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int j = threadIdx.x; j < n_shell; j += NTP) {
        double x[3], g[6];
        cube_pos(shell[3 * j], shell[3 * j + 1], shell[3 * j + 2], x);
        kelvin_point(x, k.c11, k.c12, k.c44, k.npsi, cpsi, spsi, g);
        for (int c = 0; c < 6; ++c) acc[c] += gl_shell[6 * j + c] - g[c];
    }
    block_sum6(acc, red);
    double cc[6];
    for (int c = 0; c < 6; ++c) cc[c] = acc[c] / (double)n_shell;
    if (threadIdx.x < 6) c_out[threadIdx.x] = cc[threadIdx.x];
    for (int e = threadIdx.x; e < 6 * n_table; e += NTP) table[e] = gl_table[e] - cc[e % 6];
}

// Richardson combination folded into one coefficient per image: Q0 = sum_k w_k G~_{n+k}
// and G~_k sums the images |i| <= k, so image i enters with coef_i = sum of w_k over
// n + k >= max(|i|, n).  coef[i + K], K = n + N.
struct RichC {
    double c[2 * PLGF_MAX_IMAGES + 1];
};

// 1/d by the hardware reciprocal and two Newton steps (relative error near 1 ulp).
__device__ inline double rcp_nr(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// Kelvin solution at a lattice vector by one thread (nodes in sequence; cpsi/spsi are read
// at a uniform index), the symmetric inverse with the Newton reciprocal.
__device__ inline void kelvin_thread(int n0, int n1, int n2, const PlgfConst& k, const double* __restrict__ cpsi,
                                     const double* __restrict__ spsi, double out[6]) {
    double x[3];
    cube_pos(n0, n1, n2, x);
    const double rinv = rcp_nr(sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]));
    const double xh[3] = {x[0] * rinv, x[1] * rinv, x[2] * rinv};
    double u[3], v[3];
    normal_pair(xh, u, v);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int l = 0; l < k.npsi; ++l) {
        const double cl = cpsi[l], sl = spsi[l];
        const double n[3] = {cl * u[0] + sl * v[0], cl * u[1] + sl * v[1], cl * u[2] + sl * v[2]};
        double g[6];
        acoustic(n, k.c11, k.c12, k.c44, g);
        const double a = g[0], b = g[1], c = g[2], xy = g[3], xz = g[4], yz = g[5];
        const double cxx = b * c - yz * yz, cyy = a * c - xz * xz, czz = a * b - xy * xy;
        const double cxy = xz * yz - xy * c, cxz = xy * yz - b * xz, cyz = xy * xz - a * yz;
        const double inv = rcp_nr(a * cxx + xy * cxy + xz * cxz);
        acc[0] += cxx * inv; acc[1] += cyy * inv; acc[2] += czz * inv;
        acc[3] += cxy * inv; acc[4] += cxz * inv; acc[5] += cyz * inv;
    }
    const double sc = rinv / (4.0 * M_PI * k.npsi);
    for (int c = 0; c < 6; ++c) out[c] = acc[c] * sc;
}

// One thread per displacement: Q0 = sum_i coef_i [G~inf(r + i N_z b0) - G~inf(i N_z b0)].
__global__ void __launch_bounds__(NTP) k_plgf_eval(const int32_t* __restrict__ disp, int64_t n, int nz, int K,
                                                   RichC rc, PlgfConst k, const int* __restrict__ map,
                                                   const double* __restrict__ table,
                                                   const double* __restrict__ cpsi,
                                                   const double* __restrict__ spsi,
                                                   const double* __restrict__ origin,
                                                   double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * NTP + threadIdx.x;
    if (j >= n) return;
    const int d0 = disp[3 * j], d1 = disp[3 * j + 1], d2 = disp[3 * j + 2];
    double q[6] = {0, 0, 0, 0, 0, 0};
    for (int i = -K; i <= K; ++i) {
        const int m0 = d0 + i * nz;
        double t[6];
        if (four_r2(m0, d1, d2) <= k.r2x4_cut) {
            const int ti = table_index(map, k, m0, d1, d2);
            for (int c = 0; c < 6; ++c) t[c] = (ti >= 0) ? table[6 * ti + c] : __builtin_nan("");
        } else {
            kelvin_thread(m0, d1, d2, k, cpsi, spsi, t);
        }
        const double w = rc.c[i + K];
        for (int c = 0; c < 6; ++c) q[c] = fma(w, t[c] - origin[6 * (i + K) + c], q[c]);
    }
    for (int c = 0; c < 6; ++c) out[6 * j + c] = q[c];
}

// Images of the origin, G~inf(i N_z b0) for i = -K..K (one thread per image, the same
// evaluation as the displacement terms, so a zero displacement gives exactly zero).
__global__ void __launch_bounds__(64) k_plgf_origin(int nz, int K, PlgfConst k, const int* __restrict__ map,
                                                    const double* __restrict__ table,
                                                    const double* __restrict__ cpsi,
                                                    const double* __restrict__ spsi,
                                                    double* __restrict__ origin) {
    const int i = (int)threadIdx.x - K;
    if (i > K) return;
    const int m0 = i * nz;
    double t[6];
    if (four_r2(m0, 0, 0) <= k.r2x4_cut) {
        const int ti = table_index(map, k, m0, 0, 0);
        for (int c = 0; c < 6; ++c) t[c] = (ti >= 0) ? table[6 * ti + c] : __builtin_nan("");
    } else {
        kelvin_thread(m0, 0, 0, k, cpsi, spsi, t);
    }
    for (int c = 0; c < 6; ++c) origin[6 * (i + K) + c] = t[c];
}

// ---------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------
struct fbc_plgf {
    int L = 0, logL = 0, r2x4_cut = 0, r2x4_match = 0, npsi = 0;
    int n_table = 0, n_shell = 0;
    PlgfConst kc{};
    std::vector<int32_t> vec;        // table vectors, host copy [n_table][3]
    std::vector<void*> allocs;
    int* map = nullptr;
    double* table = nullptr;
    double* c = nullptr;
    double* cpsi = nullptr;
    double* spsi = nullptr;
    double* origin = nullptr;        // [2 PLGF_MAX_IMAGES + 1][6]
};

static void plgf_free(fbc_plgf* p) {
    if (!p) return;
    for (void* a : p->allocs) (void)hipFree(a);
    delete p;
}

template <class T>
static fbc_status palloc(fbc_plgf* p, T** ptr, int64_t bytes) {
    *ptr = nullptr;
    hipError_t e = hipMalloc((void**)ptr, (size_t)std::max<int64_t>(bytes, 8));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return pfail(FBC_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + " B)");
    }
    p->allocs.push_back(*ptr);
    return FBC_OK;
}

// Lattice vectors with lo < 4|B n|^2 <= hi, sorted by (4|B n|^2, n0, n1, n2).
static std::vector<int32_t> shell_vectors(int lo, int hi) {
    const int bound = (int)std::ceil(std::sqrt(hi / 4.0) * 3.0) + 1;   // |n_i| <= 3 |x| for this basis
    struct V { int d2, a, b, c; };
    std::vector<V> v;
    for (int a = -bound; a <= bound; ++a)
        for (int b = -bound; b <= bound; ++b)
            for (int c = -bound; c <= bound; ++c) {
                const int d2 = four_r2(a, b, c);
                if (d2 > lo && d2 <= hi) v.push_back({d2, a, b, c});
            }
    std::sort(v.begin(), v.end(), [](const V& x, const V& y) {
        if (x.d2 != y.d2) return x.d2 < y.d2;
        if (x.a != y.a) return x.a < y.a;
        if (x.b != y.b) return x.b < y.b;
        return x.c < y.c;
    });
    std::vector<int32_t> out;
    out.reserve(v.size() * 3);
    for (const V& e : v) {
        out.push_back(e.a);
        out.push_back(e.b);
        out.push_back(e.c);
    }
    return out;
}

BondTable make_bonds(double k);

extern "C" const char* fbc_plgf_last_error(void) { return g_perr.c_str(); }

extern "C" fbc_status fbc_plgf_create(const fbc_lattice* lat, const fbc_plgf_opts* o, void* stream,
                                      fbc_plgf** out) {
    if (!out) return pfail(FBC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!lat || !o) return pfail(FBC_E_ARG, "lattice and options must not be NULL");
    if (!(lat->a > 0) || !(lat->spring_k > 0)) return pfail(FBC_E_ARG, "a and spring_k must be > 0");
    const int L = o->torus_l;
    if (L < 8 || L > 256 || (L & (L - 1))) return pfail(FBC_E_ARG, "torus_l must be a power of two in [8, 256]");
    if (o->r2x4_cut < 0 || o->r2x4_cut > 4 * 12 * 12) return pfail(FBC_E_ARG, "r2x4_cut must be in [0, 576]");
    if (o->r2x4_match <= o->r2x4_cut || o->r2x4_match > 4 * 16 * 16)
        return pfail(FBC_E_ARG, "r2x4_match must be in (r2x4_cut, 1024]");
    if (o->n_psi < 64 || o->n_psi > 1024 || (o->n_psi % 64))
        return pfail(FBC_E_ARG, "n_psi must be a multiple of 64 in [64, 1024]");
    hipStream_t st = (hipStream_t)stream;
    fbc_plgf* p = new (std::nothrow) fbc_plgf();
    if (!p) return pfail(FBC_E_NOMEM, "host allocation");
    p->L = L;
    while ((1 << p->logL) < L) ++p->logL;
    p->r2x4_cut = o->r2x4_cut;
    p->r2x4_match = o->r2x4_match;
    p->npsi = o->n_psi;
    const double k = lat->spring_k;
    p->kc.c11 = 2.0 * k;                 // nearest-neighbour central springs, a = 1
    p->kc.c12 = k;
    p->kc.c44 = k;
    p->kc.npsi = o->n_psi;
    p->kc.r2x4_cut = o->r2x4_cut;
    p->vec = shell_vectors(-1, o->r2x4_cut);
    const std::vector<int32_t> shell = shell_vectors(o->r2x4_cut, o->r2x4_match);
    p->n_table = (int)(p->vec.size() / 3);
    p->n_shell = (int)(shell.size() / 3);
    // index map over the bounding box of the table vectors
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int t = 0; t < p->n_table; ++t)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p->vec[3 * t + a]);
            hi[a] = std::max(hi[a], p->vec[3 * t + a]);
        }
    for (int a = 0; a < 3; ++a) {
        p->kc.lo[a] = lo[a];
        p->kc.span[a] = hi[a] - lo[a] + 1;
    }
    const int64_t map_n = (int64_t)p->kc.span[0] * p->kc.span[1] * p->kc.span[2];
    std::vector<int> map((size_t)map_n, -1);
    for (int t = 0; t < p->n_table; ++t) {
        const int a = p->vec[3 * t] - lo[0], b = p->vec[3 * t + 1] - lo[1], c = p->vec[3 * t + 2] - lo[2];
        map[((size_t)a * p->kc.span[1] + b) * p->kc.span[2] + c] = t;
    }
    std::vector<double> sn(L), cs(L), cp(o->n_psi), sp(o->n_psi);
    for (int j = 0; j < L; ++j) {
        sn[j] = std::sin(M_PI * j / L);
        cs[j] = std::cos(2.0 * M_PI * j / L);
    }
    for (int l = 0; l < o->n_psi; ++l) {
        cp[l] = std::cos(2.0 * M_PI * l / o->n_psi);
        sp[l] = std::sin(2.0 * M_PI * l / o->n_psi);
    }
    const int npts = p->n_table + p->n_shell;
    int32_t* pts = nullptr;
    double *gl = nullptr, *sn_d = nullptr, *cs_d = nullptr;
    fbc_status s;
    if ((s = palloc(p, &pts, (int64_t)npts * 12)) != FBC_OK || (s = palloc(p, &gl, (int64_t)npts * 48)) != FBC_OK ||
        (s = palloc(p, &sn_d, L * 8)) != FBC_OK || (s = palloc(p, &cs_d, L * 8)) != FBC_OK ||
        (s = palloc(p, &p->map, map_n * 4)) != FBC_OK || (s = palloc(p, &p->table, (int64_t)p->n_table * 48)) != FBC_OK ||
        (s = palloc(p, &p->c, 48)) != FBC_OK || (s = palloc(p, &p->cpsi, o->n_psi * 8)) != FBC_OK ||
        (s = palloc(p, &p->spsi, o->n_psi * 8)) != FBC_OK ||
        (s = palloc(p, &p->origin, (2 * PLGF_MAX_IMAGES + 1) * 48)) != FBC_OK) {
        plgf_free(p);
        return s;
    }
    std::vector<int32_t> all(p->vec);
    all.insert(all.end(), shell.begin(), shell.end());
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(pts, all.data(), all.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->map, map.data(), map.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sn_d, sn.data(), L * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(cs_d, cs.data(), L * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->cpsi, cp.data(), cp.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->spsi, sp.data(), sp.size() * 8, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);
        plgf_free(p);
        return pfail(FBC_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    const BondTable bt = make_bonds(k);
    hipLaunchKernelGGL(k_plgf_torus, dim3(npts), dim3(NTP), 0, st, pts, p->logL, sn_d, cs_d, bt, gl);
    hipLaunchKernelGGL(k_plgf_match, dim3(1), dim3(NTP), 0, st, pts + 3 * p->n_table, gl + 6 * p->n_table,
                       p->n_shell, gl, p->n_table, p->kc, p->cpsi, p->spsi, p->c, p->table);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        plgf_free(p);
        return pfail(FBC_E_DEVICE, std::string("table kernels: ") + hipGetErrorString(e));
    }
    *out = p;
    return FBC_OK;
}

extern "C" void fbc_plgf_destroy(fbc_plgf* p) { plgf_free(p); }

extern "C" fbc_status fbc_plgf_table(const fbc_plgf* p, int* n_table, int32_t* vectors, double* values,
                                     double* c) {
    if (!p || !n_table) return pfail(FBC_E_ARG, "object and n_table must not be NULL");
    *n_table = p->n_table;
    if (vectors) std::memcpy(vectors, p->vec.data(), p->vec.size() * 4);
    if (values) PCHK(hipMemcpy(values, p->table, (size_t)p->n_table * 48, hipMemcpyDeviceToHost));
    if (c) PCHK(hipMemcpy(c, p->c, 48, hipMemcpyDeviceToHost));
    return FBC_OK;
}

extern "C" fbc_status fbc_plgf_eval(fbc_plgf* p, const int32_t* disp, int64_t n, int nz, int n_rich,
                                    int order, double* out, void* stream) {
    if (!p) return pfail(FBC_E_ARG, "object is NULL");
    if (n < 0) return pfail(FBC_E_ARG, "n must be >= 0");
    if (n > 0 && (!disp || !out)) return pfail(FBC_E_ARG, "disp and out must be device pointers");
    if (nz < 1 || nz > 65536) return pfail(FBC_E_ARG, "nz must be in [1, 65536]");
    if (n_rich < 1 || order < 0 || order > 7 || n_rich + order > PLGF_MAX_IMAGES)
        return pfail(FBC_E_ARG, "need n_rich >= 1, 0 <= order <= 7, n_rich + order <= 16");
    if (n == 0) return FBC_OK;
    hipStream_t st = (hipStream_t)stream;
    double w[8], fact[8] = {1, 1, 2, 6, 24, 120, 720, 5040};
    for (int i = 0; i <= order; ++i)
        w[i] = std::pow((double)(n_rich + i), order) * (((i + order) & 1) ? -1.0 : 1.0) / (fact[i] * fact[order - i]);
    const int K = n_rich + order;
    RichC rc{};
    for (int i = -K; i <= K; ++i) {
        double s = 0.0;
        for (int kk = std::max(std::abs(i), n_rich); kk <= K; ++kk) s += w[kk - n_rich];
        rc.c[i + K] = s;
    }
    hipLaunchKernelGGL(k_plgf_origin, dim3(1), dim3(64), 0, st, nz, K, p->kc,
                       p->map, p->table, p->cpsi, p->spsi, p->origin);
    const int64_t blocks = (n + NTP - 1) / NTP;
    if (blocks > 0x7fffffffLL) return pfail(FBC_E_ARG, "n too large");
    hipLaunchKernelGGL(k_plgf_eval, dim3((unsigned)blocks), dim3(NTP), 0, st, disp, n, nz, K, rc, p->kc, p->map,
                       p->table, p->cpsi, p->spsi, p->origin, out);
    PCHK(hipGetLastError());
    return FBC_OK;
}
