// C ABI of the learned far-field form: continuum table, MLP training, evaluation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "ctx.h"
#include "kernels.h"

static thread_local std::string g_lerr;

static fbc_status lfail(std::string* dst, fbc_status s, const std::string& m) {
    if (dst) *dst = m;
    g_lerr = m;
    return s;
}

#define LCHK(dst, expr)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return lfail(dst, FBC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
static fbc_status lalloc(std::vector<void*>& list, std::string* err, T** p, int64_t bytes) {
    *p = nullptr;
    if (bytes <= 0) return FBC_OK;
    hipError_t e = hipMalloc((void**)p, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return lfail(err, FBC_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + " B)");
    }
    list.push_back(*p);
    return FBC_OK;
}

extern "C" const char* fbc_learned_last_error(void) { return g_lerr.c_str(); }

// ----------------------------------------------------------------------------------
// Continuum table.  Cubic constants of the nearest-neighbour central-spring crystal
// (C11 = 2k/a, C12 = C44 = k/a), line direction [1-10], in-plane axes [001] and
// [110]/sqrt2.  Grids: psi 48 nodes, phi 256 directions, z on [-400, 400] step 1/64,
// s log-spaced on [1e-3, 40] (256 nodes) plus the kappa = 0 column.
// ----------------------------------------------------------------------------------
extern "C" fbc_status fbc_sur_create(const fbc_lattice* lat, double r_c, void* stream, fbc_sur** out) {
    if (!out) return lfail(nullptr, FBC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!lat || !(lat->spring_k > 0) || !(lat->a > 0)) return lfail(nullptr, FBC_E_ARG, "lattice");
    if (!(r_c > 0) || !(r_c < 1e4)) return lfail(nullptr, FBC_E_ARG, "r_c must be in (0, 1e4)");
    fbc_sur* s = new (std::nothrow) fbc_sur();
    if (!s) return lfail(nullptr, FBC_E_NOMEM, "host allocation");
    hipStream_t st = (hipStream_t)stream;
    s->r_c = r_c;
    CgfConst& k = s->k;
    k.c11 = 2.0 * lat->spring_k / lat->a;
    k.c12 = lat->spring_k / lat->a;
    k.c44 = lat->spring_k / lat->a;
    k.t[0] = M_SQRT1_2;
    k.t[1] = -M_SQRT1_2;
    k.t[2] = 0.0;
    k.npsi = 48;
    k.nphi = 256;
    k.zmax = 400.0;
    k.dz = 1.0 / 64.0;
    k.nzq = (int)std::lround(2.0 * k.zmax / k.dz) + 1;
    k.ns = 256;
    k.s_min = 1e-3;
    k.s_max = 40.0;
    std::vector<double> cpsi(k.npsi), spsi(k.npsi), rhat(3 * k.nphi);
    for (int l = 0; l < k.npsi; ++l) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * l / k.npsi;
        cpsi[l] = (double)cosl(a);
        spsi[l] = (double)sinl(a);
    }
    const double e1[3] = {0, 0, 1}, e2[3] = {M_SQRT1_2, M_SQRT1_2, 0};
    for (int j = 0; j < k.nphi; ++j) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * j / k.nphi;
        const double c = (double)cosl(a), sn = (double)sinl(a);
        for (int q = 0; q < 3; ++q) rhat[3 * j + q] = c * e1[q] + sn * e2[q];
    }
    std::vector<double2> ph0(k.ns), step(k.ns);
    std::vector<double> k0s(2 * k.ns);
    for (int i = 0; i < k.ns; ++i) {
        const double si = k.s_min * std::pow(k.s_max / k.s_min, (double)i / (k.ns - 1));
        const long double a0 = (long double)si * k.zmax;      // exp(-i s z0), z0 = -zmax
        ph0[i] = make_double2((double)cosl(a0), (double)sinl(a0));
        const long double a1 = -(long double)si * k.dz;
        step[i] = make_double2((double)cosl(a1), (double)sinl(a1));
        k0s[2 * i] = std::cyl_bessel_k(0.0, si);
        k0s[2 * i + 1] = si;
    }
    double *d_cpsi, *d_spsi, *d_rhat, *d_g1, *d_rem, *d_k0s;
    double2 *d_ph0, *d_step;
    std::vector<void*> tmp;
    fbc_status rc;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (void* p : tmp) (void)hipFree(p);
    };
    if ((rc = lalloc(tmp, &s->err, &d_cpsi, k.npsi * 8)) || (rc = lalloc(tmp, &s->err, &d_spsi, k.npsi * 8)) ||
        (rc = lalloc(tmp, &s->err, &d_rhat, (int64_t)rhat.size() * 8)) ||
        (rc = lalloc(tmp, &s->err, &d_g1, (int64_t)k.nphi * 6 * 8)) ||
        (rc = lalloc(tmp, &s->err, &d_rem, (int64_t)k.nphi * k.nzq * 6 * 8)) ||
        (rc = lalloc(tmp, &s->err, &d_k0s, (int64_t)k0s.size() * 8)) ||
        (rc = lalloc(tmp, &s->err, &d_ph0, (int64_t)k.ns * 16)) ||
        (rc = lalloc(tmp, &s->err, &d_step, (int64_t)k.ns * 16)) ||
        (rc = lalloc(s->allocs, &s->err, &s->g0, 6 * 8)) ||
        (rc = lalloc(s->allocs, &s->err, &s->H, (int64_t)k.nphi * (k.ns + 1) * 6 * 16)) ||
        (rc = lalloc(s->allocs, &s->err, &s->wb, (int64_t)MLP_NW * 2)) ||
        (rc = lalloc(s->allocs, &s->err, &s->wm, (int64_t)MLP_MFMA_ELEMS * 2)) ||
        (rc = lalloc(s->allocs, &s->err, &s->wf, (int64_t)MLP_NW * 4)) ||
        (rc = lalloc(s->allocs, &s->err, &s->bias, (int64_t)MLP_NB * 4))) {
        cleanup();
        for (void* p : s->allocs) (void)hipFree(p);
        delete s;
        return rc;
    }
    (void)hipMemcpyAsync(d_cpsi, cpsi.data(), k.npsi * 8, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(d_spsi, spsi.data(), k.npsi * 8, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(d_rhat, rhat.data(), rhat.size() * 8, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(d_k0s, k0s.data(), k0s.size() * 8, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(d_ph0, ph0.data(), ph0.size() * 16, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(d_step, step.data(), step.size() * 16, hipMemcpyHostToDevice, st);
    launch_cgf_build(st, k, d_cpsi, d_spsi, d_rhat, s->g0, d_g1, d_rem, d_ph0, d_step, d_k0s, s->H);
    hipError_t e = hipGetLastError();
    cleanup();
    if (e != hipSuccess) {
        for (void* p : s->allocs) (void)hipFree(p);
        delete s;
        return lfail(nullptr, FBC_E_DEVICE, std::string("continuum table: ") + hipGetErrorString(e));
    }
    *out = s;
    return FBC_OK;
}

extern "C" void fbc_sur_destroy(fbc_sur* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    for (void* p : s->allocs) (void)hipFree(p);
    delete s;
}

extern "C" fbc_status fbc_sur_set_mlp(fbc_sur* s, const fbc_mlp* net, void* stream) {
    if (!s || !net) return lfail(nullptr, FBC_E_ARG, "null argument");
    launch_mlp_to_bf16((hipStream_t)stream, net->params, s->wb, s->bias);
    launch_mlp_to_mfma((hipStream_t)stream, net->params, s->wm);
    LCHK(&s->err, hipGetLastError());
    LCHK(&s->err, hipStreamSynchronize((hipStream_t)stream));
    s->has_mlp = 1;
    s->mlp_fp32 = 0;
    return FBC_OK;
}

extern "C" fbc_status fbc_sur_set_mlp_fp32(fbc_sur* s, const fbc_mlp* net, void* stream) {
    if (!s || !net) return lfail(nullptr, FBC_E_ARG, "null argument");
    launch_mlp_to_f32t((hipStream_t)stream, net->params, s->wf, s->bias);
    LCHK(&s->err, hipGetLastError());
    LCHK(&s->err, hipStreamSynchronize((hipStream_t)stream));
    s->has_mlp = 1;
    s->mlp_fp32 = 1;
    return FBC_OK;
}

extern "C" fbc_status fbc_sur_set_learn_range(fbc_sur* s, double s_learn) {
    if (!s || !(s_learn > 0) || !(s_learn <= 40.0)) return lfail(nullptr, FBC_E_ARG, "s_learn must be in (0, 40]");
    s->s_learn = s_learn;
    return FBC_OK;
}

extern "C" fbc_status fbc_sur_set_exact_range(fbc_sur* s, double s_exact) {
    if (!s || !(s_exact >= 0) || !(s_exact <= 40.0)) return lfail(nullptr, FBC_E_ARG, "s_exact must be in [0, 40]");
    s->s_exact = s_exact;
    return FBC_OK;
}

extern "C" fbc_status fbc_sur_eval(const fbc_sur* s, const double* theta0, const int32_t* dn1,
                                   const int32_t* dn2, int n, int use_mlp, double* out, void* stream) {
    if (!s || !theta0 || !dn1 || !dn2 || !out || n < 0) return lfail(nullptr, FBC_E_ARG, "null argument");
    if (use_mlp && !s->has_mlp) return lfail(nullptr, FBC_E_STATE, "no MLP weights set");
    launch_sur_points((hipStream_t)stream, s->view(), s->infer(), use_mlp ? 1 : 0, s->r_c,
                      theta0, dn1, dn2, n, (double2*)out);
    LCHK(nullptr, hipGetLastError());
    return FBC_OK;
}

// Training set from an offset-table context (its table holds lattice values for every
// distinct offset and line mode of its cells): samples (mode t >= 1, offset o) in the
// learned band of the table, drawn with a seeded generator: a line mode uniformly among
// those whose band holds an offset, then an offset uniformly in that mode's band.  The
// band is the one a surrogate context uses: offsets beyond r_c and beyond the last block
// of at least exp(-s_exact) times the mode's largest block, out to the last block of at
// least exp(-s_learn) times it.
extern "C" fbc_status fbc_sur_training_set(fbc_sur* s, const fbc_ctx* c, int max_samples,
                                           uint64_t seed, float* x, float* t, int* n_out,
                                           void* stream) {
    if (!s || !c || !x || !t || !n_out || max_samples < 1) return lfail(nullptr, FBC_E_ARG, "null argument");
    if (c->opt.form != FBC_FORM_DTABLE_FP64 || !c->tab || !c->off_d1)
        return lfail(nullptr, FBC_E_STATE, "training data needs an offset-table context");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n_off = c->n_offsets;
    const int T = c->nz_max / 2 + 1;
    std::vector<int32_t> d1(n_off), d2(n_off);
    LCHK(nullptr, hipMemcpy(d1.data(), c->off_d1, n_off * 4, hipMemcpyDeviceToHost));
    LCHK(nullptr, hipMemcpy(d2.data(), c->off_d2, n_off * 4, hipMemcpyDeviceToHost));
    std::vector<double> rho(n_off);
    for (int64_t o = 0; o < n_off; ++o) {
        const double xx = 0.5 * d1[o], yy = (d1[o] + 2.0 * d2[o]) * (0.5 * M_SQRT1_2);
        rho[o] = std::sqrt(xx * xx + yy * yy);
    }
    std::vector<int32_t> ord(n_off);
    for (int64_t o = 0; o < n_off; ++o) ord[o] = (int32_t)o;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return rho[a] < rho[b]; });
    // per table mode, the distances beyond which every block is below exp(-s_exact) and
    // exp(-s_learn) of the mode's largest block
    unsigned long long* cut_d = nullptr;
    LCHK(nullptr, hipMalloc((void**)&cut_d, (size_t)T * 8 * 3));
    launch_tab_rhocut(st, c->tab, T, n_off, c->off_d1, c->off_d2, std::exp(-s->s_exact), cut_d + 2 * T, cut_d);
    launch_tab_rhocut(st, c->tab, T, n_off, c->off_d1, c->off_d2, std::exp(-s->s_learn), cut_d + 2 * T, cut_d + T);
    std::vector<unsigned long long> bits((size_t)T * 3);     // two cuts, then the largest blocks
    const hipError_t ce = hipMemcpyAsync(bits.data(), cut_d, bits.size() * 8, hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(cut_d);
    LCHK(nullptr, ce);
    auto cut = [&](int k, int t) {
        double v;
        std::memcpy(&v, &bits[(size_t)k * T + t], 8);
        return v * (1.0 + 1e-12);              // the device and host distances may differ in the last bit
    };
    // band of line mode t in rank order: [lo, hi); line mode 0 is taken exact by the surrogate
    // (the in-plane torus of the exact Green function acts on that mode only)
    auto rank_beyond = [&](double r) {
        return (int64_t)(std::upper_bound(ord.begin(), ord.end(), r,
                                          [&](double v, int32_t o) { return v < rho[o]; }) - ord.begin());
    };
    std::vector<int> modes;
    std::vector<int64_t> lo, hi;
    const int64_t r_near = rank_beyond(s->r_c);
    for (int tm = 1; tm < T; ++tm) {
        const int64_t a = std::max(r_near, rank_beyond(cut(0, tm))), b = rank_beyond(cut(1, tm));
        if (b > a) {
            modes.push_back(tm);
            lo.push_back(a);
            hi.push_back(b);
        }
    }
    if (modes.empty())
        return lfail(nullptr, FBC_E_ARG, "no offset of the table context lies in the learned band");
    double rho_band = 0.0;
    for (size_t k = 0; k < modes.size(); ++k) rho_band = std::max(rho_band, rho[ord[hi[k] - 1]]);
    std::mt19937_64 gen(seed);
    std::uniform_int_distribution<int> pick_m(0, (int)modes.size() - 1);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    std::vector<int32_t> pt(max_samples), po(max_samples);
    for (int i = 0; i < max_samples; ++i) {
        const int k = pick_m(gen);
        int64_t r = lo[k] + (int64_t)(u01(gen) * (double)(hi[k] - lo[k]));
        r = std::min(r, hi[k] - 1);
        pt[i] = modes[k];
        po[i] = ord[r];
    }
    // envelope per table mode: exp(-s_exact) times the mode's largest block
    std::vector<double> envm(T);
    for (int tm = 0; tm < T; ++tm) {
        std::memcpy(&envm[tm], &bits[(size_t)2 * T + tm], 8);
        envm[tm] *= std::exp(-s->s_exact);
    }
    const int n = max_samples;
    {
        // envelopes and index lists
        char* buf = nullptr;
        LCHK(nullptr, hipMalloc((void**)&buf, (size_t)T * 8 + (size_t)n * 8));
        double* denv = (double*)buf;
        int32_t* dpt = (int32_t*)(buf + (size_t)T * 8);
        int32_t* dpo = dpt + n;
        (void)hipMemcpyAsync(denv, envm.data(), (size_t)T * 8, hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(dpt, pt.data(), (size_t)n * 4, hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(dpo, po.data(), (size_t)n * 4, hipMemcpyHostToDevice, st);
        launch_sur_samples(st, s->view(), c->tab, n_off, c->nz_max, c->off_d1, c->off_d2, dpt, dpo, n, s->r_c,
                           denv, x, t);
        (void)hipStreamSynchronize(st);
        (void)hipFree(buf);
    }
    s->rho_learn = rho_band;
    *n_out = n;
    LCHK(nullptr, hipGetLastError());
    return FBC_OK;
}

// ----------------------------------------------------------------------------------
// MLP training objects.
// ----------------------------------------------------------------------------------
extern "C" fbc_status fbc_mlp_create(int max_batch, uint64_t seed, fbc_mlp** out) {
    if (!out) return lfail(nullptr, FBC_E_ARG, "out is NULL");
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 22)) return lfail(nullptr, FBC_E_ARG, "max_batch in [1, 2^22]");
    fbc_mlp* m = new (std::nothrow) fbc_mlp();
    if (!m) return lfail(nullptr, FBC_E_NOMEM, "host allocation");
    m->max_batch = max_batch;
    (void)hipGetDevice(&m->device);
    fbc_status rc;
    if ((rc = lalloc(m->allocs, &m->err, &m->params, MLP_NPARAMS * 4)) ||
        (rc = lalloc(m->allocs, &m->err, &m->grad, MLP_NPARAMS * 4)) ||
        (rc = lalloc(m->allocs, &m->err, &m->m, MLP_NPARAMS * 4)) ||
        (rc = lalloc(m->allocs, &m->err, &m->v, MLP_NPARAMS * 4)) ||
        (rc = lalloc(m->allocs, &m->err, &m->loss, 64)) ||
        (rc = lalloc(m->allocs, &m->err, &m->ws, mlp_workspace_floats(max_batch) * 4))) {
        for (void* p : m->allocs) (void)hipFree(p);
        delete m;
        return rc;
    }
    // normal(0, 1/sqrt(fan_in)) weights, zero biases, from a seeded host generator
    std::vector<float> p(MLP_NPARAMS, 0.0f);
    std::mt19937_64 gen(seed);
    const int sizes[5] = {MLP_IN, MLP_H, MLP_H, MLP_H, MLP_OUT};
    int64_t off = 0;
    for (int l = 0; l < 4; ++l) {
        std::normal_distribution<double> nd(0.0, 1.0 / std::sqrt((double)sizes[l]));
        for (int i = 0; i < sizes[l + 1] * sizes[l]; ++i) p[off + i] = (float)nd(gen);
        off += (int64_t)sizes[l + 1] * sizes[l] + sizes[l + 1];
    }
    (void)hipMemcpy(m->params, p.data(), p.size() * 4, hipMemcpyHostToDevice);
    (void)hipMemset(m->m, 0, MLP_NPARAMS * 4);
    (void)hipMemset(m->v, 0, MLP_NPARAMS * 4);
    *out = m;
    return FBC_OK;
}

extern "C" void fbc_mlp_destroy(fbc_mlp* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
}

extern "C" int fbc_mlp_num_params(void) { return MLP_NPARAMS; }

extern "C" fbc_status fbc_mlp_params(fbc_mlp* m, float* host_out, const float* host_in) {
    if (!m) return lfail(nullptr, FBC_E_ARG, "null argument");
    LCHK(&m->err, hipDeviceSynchronize());
    if (host_in) LCHK(&m->err, hipMemcpy(m->params, host_in, MLP_NPARAMS * 4, hipMemcpyHostToDevice));
    if (host_out) LCHK(&m->err, hipMemcpy(host_out, m->params, MLP_NPARAMS * 4, hipMemcpyDeviceToHost));
    return FBC_OK;
}

extern "C" fbc_status fbc_mlp_grad(fbc_mlp* m, float* host_out) {
    if (!m || !host_out) return lfail(nullptr, FBC_E_ARG, "null argument");
    LCHK(&m->err, hipDeviceSynchronize());
    LCHK(&m->err, hipMemcpy(host_out, m->grad, MLP_NPARAMS * 4, hipMemcpyDeviceToHost));
    return FBC_OK;
}

extern "C" fbc_status fbc_mlp_loss_grad(fbc_mlp* m, const float* x, const float* t, int n,
                                        float* loss_dev, void* stream) {
    if (!m || !x || !t) return lfail(nullptr, FBC_E_ARG, "null argument");
    if (n < 1 || n > m->max_batch) return lfail(&m->err, FBC_E_ARG, "batch size out of range");
    launch_mlp_loss_grad((hipStream_t)stream, m->params, x, t, nullptr, n, m->ws, m->grad,
                         loss_dev ? loss_dev : m->loss);
    LCHK(&m->err, hipGetLastError());
    return FBC_OK;
}

extern "C" fbc_status fbc_mlp_adam_step(fbc_mlp* m, float lr, void* stream) {
    if (!m || !(lr > 0)) return lfail(nullptr, FBC_E_ARG, "bad argument");
    m->step += 1;
    launch_adam((hipStream_t)stream, m->params, m->grad, m->m, m->v, MLP_NPARAMS, lr, m->step);
    LCHK(&m->err, hipGetLastError());
    return FBC_OK;
}

extern "C" fbc_status fbc_mlp_forward(fbc_mlp* m, const float* x, float* y, int n, void* stream) {
    if (!m || !x || !y) return lfail(nullptr, FBC_E_ARG, "null argument");
    if (n < 1 || n > m->max_batch) return lfail(&m->err, FBC_E_ARG, "batch size out of range");
    launch_mlp_forward((hipStream_t)stream, m->params, x, n, m->ws, y);
    LCHK(&m->err, hipGetLastError());
    return FBC_OK;
}

// ----------------------------------------------------------------------------------
// Forward pass without device allocation, for callers that cannot allocate (code under
// HIP graph capture, serving loops): the layer activations go to a file-scope device
// array instead of the network's workspace.  Each GPU the library runs on holds its own
// copy of the array until the process ends; every call on that GPU shares it.
// ----------------------------------------------------------------------------------
static constexpr int64_t kNoAllocBytes = (int64_t)64 << 20;
static __device__ __align__(256) float scratch[kNoAllocBytes / 4];

// Floats of the forward workspace for n rows (z and a of every layer in the layout of
// launch_mlp_forward, 4 n x width per layer).
static int64_t forward_ws_floats(int64_t n) { return 4 * n * (3 * MLP_H + MLP_OUT); }
static const int kNoAllocRows = (int)(kNoAllocBytes / 4 / forward_ws_floats(1));

// Device address of this GPU's copy of `scratch`, looked up once per device with that
// device current; host code never passes the array's own name to a kernel.
static std::mutex g_scratch_mu;
static std::vector<float*> g_scratch_dev;

static fbc_status scratch_address(int dev, float** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return lfail(nullptr, FBC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_dev[dev] = (float*)p;
    }
    *out = g_scratch_dev[dev];
    return FBC_OK;
}

extern "C" int fbc_mlp_forward_noalloc_max_rows(void) { return kNoAllocRows; }

extern "C" fbc_status fbc_mlp_forward_noalloc(const fbc_mlp* m, const float* x, float* y, int n, void* stream) {
    if (!m || !x || !y) return lfail(nullptr, FBC_E_ARG, "null argument");
    if (n < 1 || n > kNoAllocRows)
        return lfail(nullptr, FBC_E_ARG, "n must be in [1, " + std::to_string(kNoAllocRows) +
                                             "]: the static workspace holds " + std::to_string(kNoAllocBytes) + " B");
    int dev = -1;
    LCHK(nullptr, hipGetDevice(&dev));
    if (dev != m->device)
        return lfail(nullptr, FBC_E_ARG, "the network's device (" + std::to_string(m->device) +
                                             ") must be current (current: " + std::to_string(dev) + ")");
    float* ws = nullptr;
    fbc_status s = scratch_address(dev, &ws);
    if (s != FBC_OK) return s;
    // every workspace value is written before it is read: nothing needs clearing
    launch_mlp_forward((hipStream_t)stream, m->params, x, n, ws, y);
    LCHK(nullptr, hipGetLastError());
    return FBC_OK;
}
