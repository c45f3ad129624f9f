// C ABI of the FBC pad-update library: validation, planning, device buffers, and the
// orchestration of the kernels (see include/fbc.h for the contract).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include <cmath>

#include "ctx.h"
#include "plan.h"

int gemm_tile_rows(int form, int ctmax);
extern "C" fbc_status fbc_timing(fbc_ctx* c, int enable);
extern "C" fbc_status fbc_timing_read(fbc_ctx* c, double* ms, int* n);
static void drop_relax_graph(fbc_ctx* c);



static thread_local std::string g_err;

static fbc_status fail(fbc_ctx* c, fbc_status s, const std::string& msg) {
    if (c) c->err = msg;
    g_err = msg;
    return s;
}

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, FBC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
static int ilog2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}
static int64_t roundup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

static fbc_status dev_alloc(fbc_ctx* c, void** p, int64_t bytes) {
    *p = nullptr;
    if (bytes <= 0) return FBC_OK;
    hipError_t e = hipMalloc(p, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(c, FBC_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + " B): " + hipGetErrorString(e));
    }
    c->allocs.push_back(*p);
    return FBC_OK;
}

static void free_all(fbc_ctx* c) {
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

extern "C" void fbc_default_options(fbc_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->form = FBC_FORM_FP64;
    o->bz_m1 = 1024;
    o->bz_m2 = 1024;
    o->check_netforce = 1;
    o->project_netforce = 0;
    o->netforce_tol = 1e-10;
    o->row_gauge = 1;
}

extern "C" const char* fbc_status_string(fbc_status s) {
    switch (s) {
        case FBC_OK: return "ok";
        case FBC_E_ARG: return "invalid argument";
        case FBC_E_NOMEM: return "out of device memory";
        case FBC_E_NETFORCE: return "non-zero net force of a cell (all interface atoms of all layers)";
        case FBC_E_NONFINITE: return "non-finite force";
        case FBC_E_DEVICE: return "device error";
        case FBC_E_STATE: return "call out of order";
        case FBC_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown";
}

extern "C" const char* fbc_last_error(const fbc_ctx* c) {
    return c ? c->err.c_str() : g_err.c_str();
}

// Nearest-neighbour bonds of fcc in the primitive basis b0=(1/2,-1/2,0), b1=(1/2,0,1/2),
// b2=(1/2,1/2,0) and the projectors k Rhat Rhat^T (Section 2.2.1, K_h of central springs).
BondTable make_bonds(double k) {
    BondTable bt{};
    // cubic (a = 1) basis columns
    const double B[3][3] = {{0.5, 0.5, 0.5}, {-0.5, 0.0, 0.5}, {0.0, 0.5, 0.0}};
    // inverse of B (rows), exact for this basis
    double det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                 B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                 B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    double inv[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
            inv[i][j] = (B[i1][j1] * B[i2][j2] - B[i1][j2] * B[i2][j1]) / det;
        }
    int nb = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            for (int sa = -1; sa <= 1; sa += 2)
                for (int sb = -1; sb <= 1; sb += 2) {
                    double R[3] = {0, 0, 0};
                    R[a] = 0.5 * sa;
                    R[b] = 0.5 * sb;
                    for (int i = 0; i < 3; ++i) {
                        const double v = inv[i][0] * R[0] + inv[i][1] * R[1] + inv[i][2] * R[2];
                        bt.n[nb][i] = (int)std::lround(v);
                    }
                    const double len2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
                    const int cc[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
                    for (int s = 0; s < 6; ++s) bt.p[nb][s] = k * R[cc[s][0]] * R[cc[s][1]] / len2;
                    ++nb;
                }
    return bt;
}

// exp(-2 pi i j / n), j < n/2, from extended precision.
static void twiddles(int n, std::vector<double2>& out) {
    out.resize(std::max(1, n / 2));
    for (int j = 0; j < n / 2; ++j) {
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * j / n;
        out[j] = make_double2((double)cosl(a), (double)sinl(a));
    }
    if (n / 2 == 0) out[0] = make_double2(1.0, 0.0);
}

static bool is_table_form(int form) {
    return form == FBC_FORM_DTABLE_FP64 || form == FBC_FORM_SURROGATE;
}

// Row gauge: reduced dense forms store G^_bi(m) - mean_i G^_bi(m) (smaller dynamic range
// before rounding) and add the mean back exactly (FP64) against sum_i f^_i(m).
static bool is_split16(int form) { return form == FBC_FORM_SPLIT_BF16 || form == FBC_FORM_SPLIT_FP16; }

static bool row_gauge_active(const fbc_ctx* c) {
    return c->opt.row_gauge && (c->opt.form == FBC_FORM_FP32 || is_split16(c->opt.form));
}

static int64_t store_elem_bytes(int form) {
    return form == FBC_FORM_FP64 ? 8 : (form == FBC_FORM_FP32 ? 4 : 2);
}
// Store elements (of the store type) of one chunk-tile of the compact dense store:
// rows_tile rows x 64 K' (x2 for the hi and lo parts of the split forms).
static int64_t chunk_tile_elems(int form, int rows_tile) {
    return (int64_t)rows_tile * 64 * (is_split16(form) ? 2 : 1);
}
static int64_t b_mode_elems(int form, const CellPlan& p) {
    return (int64_t)16 * p.ct * p.kp * (is_split16(form) ? 2 : 1);
}
static int64_t b_elem_bytes(int form) {
    return (form == FBC_FORM_FP64 || is_table_form(form)) ? 8 : (form == FBC_FORM_FP32 ? 4 : 2);
}

// ----------------------------------------------------------------------------------
// Assembly of one cell's offset table and store.
// ----------------------------------------------------------------------------------
using OffsetSet = PlanOffsets;

static std::vector<PlanGeom> plan_geoms(const std::vector<CellPlan>& cells) {
    std::vector<PlanGeom> g;
    for (const CellPlan& p : cells) g.push_back(PlanGeom{p.n_i, p.n_b, p.cols_i.data(), p.cols_b.data()});
    return g;
}

// Distinct column offsets n_b - n_i over every cell, indexed through a dense lookup
// table over their bounding box (row-major over (d1, d2), so the numbering is fixed).
static OffsetSet offsets_of(const std::vector<CellPlan>& cells) { return plan_offsets(plan_geoms(cells)); }

// ----------------------------------------------------------------------------------
// Negligible-block windows.  At line mode m the Green function decays with kappa rho;
// rho_cut[t] is the farthest in-plane distance (table mode t) of a block that reaches the
// skip tolerance.  A K chunk of a row tile is negligible when all its (pad, interface)
// pairs lie farther than that; the product then runs, per (mode, tile), over the cyclic
// window of chunks that contains every non-negligible one.
// ----------------------------------------------------------------------------------
static double skip_tolerance(const fbc_options& o) {
    if (o.skip_tol < 0) return -1.0;
    if (o.skip_tol > 0) return o.skip_tol;
    // FP64 forms: at the rounding of their assembly; reduced forms: two orders of
    // magnitude below their own rounding (~1e-7); the learned form likewise: two orders
    // below its own error (~1e-8), just inside the end of its learned band (blocks down to
    // exp(-s_learn) ~ 2e-9 of a mode's largest)
    return (o.form == FBC_FORM_FP32 || o.form == FBC_FORM_SPLIT_BF16 || o.form == FBC_FORM_SPLIT_FP16 ||
            o.form == FBC_FORM_SURROGATE)
               ? 1e-9
               : 1e-16;
}

static void compute_windows(fbc_ctx* c, const std::vector<double>& rho_cut, int rows_tile) {
    const bool dt = is_table_form(c->opt.form);
    for (CellPlan& p : c->cells) {
        PlanWindows w;
        plan_windows(PlanGeom{p.n_i, p.n_b, p.cols_i.data(), p.cols_b.data()}, p.nm, p.mp, p.kp, dt, rows_tile,
                     c->nz_max / p.nz, rho_cut, w);
        p.n_tiles = w.n_tiles;
        p.n_chunks = w.n_chunks;
        p.win_start.swap(w.win_start);
        p.win_len.swap(w.win_len);
        p.mode_skips.swap(w.mode_skips);
    }
}

// Builds the offset table tab[t][o][6] for every line mode t = 0..nz_max/2 of the finest
// line grid of the context (a cell with Nz layers reads table mode m * nz_max / Nz, the
// same wavenumber), then either fills the dense stores of every cell and frees the
// table, or keeps it for the offset-table form.
static fbc_status assemble_all(fbc_ctx* c, hipStream_t st, const BondTable& bt, double* sn_d,
                               int logL) {
    const int m1 = c->opt.bz_m1, m2 = c->opt.bz_m2;
    const int form = c->opt.form;
    OffsetSet os = offsets_of(c->cells);
    const bool sur = (form == FBC_FORM_SURROGATE);
    std::vector<double> rho_sorted;      // surrogate: in-plane distance of each offset, ascending
    if (sur) {
        // number offsets by increasing in-plane distance: for every line mode the exact part
        // is a prefix, and so is the part where the far field is not negligible
        const int64_t n = (int64_t)os.d1.size();
        std::vector<double> rho(n);
        for (int64_t o = 0; o < n; ++o) {
            const double xx = 0.5 * os.d1[o], yy = (os.d1[o] + 2.0 * os.d2[o]) * (0.5 * M_SQRT1_2);
            rho[o] = std::sqrt(xx * xx + yy * yy);
        }
        std::vector<int32_t> ord(n);
        for (int64_t o = 0; o < n; ++o) ord[o] = (int32_t)o;
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return rho[a] < rho[b]; });
        std::vector<int32_t> rank(n), nd1(n), nd2(n);
        for (int64_t r = 0; r < n; ++r) {
            rank[ord[r]] = (int32_t)r;
            nd1[r] = os.d1[ord[r]];
            nd2[r] = os.d2[ord[r]];
        }
        for (auto& e : os.lut)
            if (e >= 0) e = rank[e];
        os.d1.swap(nd1);
        os.d2.swap(nd2);
        c->n_near = 0;
        while (c->n_near < n && rho[ord[c->n_near]] <= c->sur->r_c) ++c->n_near;
        rho_sorted.resize(n);
        for (int64_t r = 0; r < n; ++r) rho_sorted[r] = rho[ord[r]];
    }
    const int64_t n_off = (int64_t)os.d1.size();
    c->n_offsets = n_off;
    c->d1min = os.d1min;
    c->d2min = os.d2min;
    c->w2 = os.w2;
    const int T = c->nz_max / 2 + 1;
    std::vector<void*> tmp;
    auto talloc = [&](void** ptr, int64_t bytes) -> fbc_status {
        *ptr = nullptr;
        hipError_t e = hipMalloc(ptr, (size_t)bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, FBC_E_NOMEM, "assembly scratch of " + std::to_string(bytes) + " B: " + hipGetErrorString(e));
        }
        tmp.push_back(*ptr);
        return FBC_OK;
    };
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (void* q : tmp) (void)hipFree(q);
    };
    fbc_status s;
    int32_t *d1_d, *d2_d;
    const bool keep = (form == FBC_FORM_DTABLE_FP64);
    if ((s = dev_alloc(c, (void**)&c->lut, (int64_t)os.lut.size() * 4)) != FBC_OK) return s;
    if (keep) {
        if ((s = dev_alloc(c, (void**)&c->tab, (int64_t)T * n_off * 96)) != FBC_OK) return s;
        c->store_bytes = (int64_t)T * n_off * 96;
    } else if (sur) {
        // generated slices (also the workspace of the measuring pass below): by default as many
        // table modes per chunk as fit in 4 GiB (long workload: 40 modes per chunk, 4 % faster
        // than the 21 of 2 GiB, within 1 % of 80 or 171)
        c->gen_modes = (int)std::max<int64_t>(1, std::min<int64_t>(T, ((int64_t)4 << 30) / std::max<int64_t>(1, n_off * 96)));
        if (c->opt.gen_modes > 0) c->gen_modes = std::min(c->opt.gen_modes, T);
        if ((s = dev_alloc(c, (void**)&c->gen, (int64_t)c->gen_modes * n_off * 96)) != FBC_OK) return s;
        c->scratch_bytes += (int64_t)c->gen_modes * n_off * 96;
    } else if ((s = talloc((void**)&c->tab, (int64_t)T * n_off * 96)) != FBC_OK) {
        cleanup();
        return s;
    }
    if (is_table_form(form)) {
        if ((s = dev_alloc(c, (void**)&d1_d, n_off * 4)) != FBC_OK || (s = dev_alloc(c, (void**)&d2_d, n_off * 4)) != FBC_OK)
            return s;
        c->off_d1 = d1_d;
        c->off_d2 = d2_d;
    } else if ((s = talloc((void**)&d1_d, n_off * 4)) != FBC_OK || (s = talloc((void**)&d2_d, n_off * 4)) != FBC_OK) {
        cleanup();
        return s;
    }
    HIPCHK(c, hipMemcpyAsync(c->lut, os.lut.data(), os.lut.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(d1_d, os.d1.data(), n_off * 4, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(d2_d, os.d2.data(), n_off * 4, hipMemcpyHostToDevice, st));
    std::vector<double2> tw1, tw2;
    twiddles(m1, tw1);
    twiddles(m2, tw2);
    double2 *tw1_d, *tw2_d;
    if ((s = talloc((void**)&tw1_d, (int64_t)tw1.size() * 16)) != FBC_OK ||
        (s = talloc((void**)&tw2_d, (int64_t)tw2.size() * 16)) != FBC_OK) {
        cleanup();
        return s;
    }
    HIPCHK(c, hipMemcpyAsync(tw1_d, tw1.data(), tw1.size() * 16, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(tw2_d, tw2.data(), tw2.size() * 16, hipMemcpyHostToDevice, st));
    // mode chunks sized to ~2 GiB of FFT workspace (x2 for the transpose)
    const int64_t plane = (int64_t)m1 * m2;
    const int64_t per_mode = plane * 3 * 16;
    int chunk = (int)std::max<int64_t>(1, ((int64_t)1 << 31) / per_mode);
    chunk = std::min(chunk, T);
    double2 *pk, *pt;
    if ((s = talloc((void**)&pk, per_mode * chunk)) != FBC_OK ||
        (s = talloc((void**)&pt, per_mode * chunk)) != FBC_OK) {
        cleanup();
        return s;
    }
    const double scale = 1.0 / ((double)m1 * m2);
    // the lattice Green function of table modes t0 .. t0+nmc-1 in pt: [mode][comp][d2][d1]
    auto lattice_modes = [&](int t0, int nmc) {
        launch_dinv(st, pk, t0, nmc, c->nz_max, m1, m2, logL, sn_d, bt);
        // inverse 2-D FFT: rows (m2 contiguous), transpose, rows again -> t[comp][d2][d1]
        launch_fft_rows(st, pk, (int64_t)nmc * 3 * m1, ilog2(m2), tw2_d, true);
        launch_transpose_c(st, pk, pt, nmc * 3, m1, m2);
        launch_fft_rows(st, pt, (int64_t)nmc * 3 * m2, ilog2(m1), tw1_d, true);
    };
    const double tau = skip_tolerance(c->opt);
    if (sur) {
        // Measuring pass: per table mode, the distances beyond which every block is below
        // exp(-s_exact), exp(-s_learn) and tau of the mode's largest block; they fix the
        // ragged exact prefix, the learned band and the generated prefix of every mode.
        const double taus[3] = {std::exp(-c->sur->s_exact), std::exp(-c->sur->s_learn), tau};
        const int nk = tau >= 0 ? 3 : 2;
        unsigned long long* cut_d;
        if ((s = talloc((void**)&cut_d, (int64_t)T * 8 * (nk + 1))) != FBC_OK) {
            cleanup();
            return s;
        }
        for (int t0 = 0; t0 < T; t0 += chunk) {
            const int nmc = std::min(chunk, T - t0);
            lattice_modes(t0, nmc);
            for (int a = 0; a < nmc; a += c->gen_modes) {
                const int ns = std::min(c->gen_modes, nmc - a);
                launch_gather_table(st, pt + (int64_t)a * 3 * plane, c->gen, ns, m1, m2, n_off, d1_d, d2_d, n_off * 6,
                                    scale);
                for (int k = 0; k < nk; ++k)
                    launch_tab_rhocut(st, c->gen, ns, n_off, d1_d, d2_d, taus[k], cut_d + (int64_t)nk * T + t0 + a,
                                      cut_d + (int64_t)k * T + t0 + a);
            }
        }
        std::vector<unsigned long long> bits((size_t)T * (nk + 1));     // cuts, then the largest blocks
        HIPCHK(c, hipMemcpyAsync(bits.data(), cut_d, bits.size() * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        auto cut = [&](int k, int t) {
            double v;
            std::memcpy(&v, &bits[(size_t)k * T + t], 8);
            return v * (1.0 + 1e-12);          // the device and host distances may differ in the last bit
        };
        // number of offsets (a prefix in distance order) within distance r, at least n_near
        auto within = [&](double r) {
            const int64_t k = std::upper_bound(rho_sorted.begin(), rho_sorted.end(), r) - rho_sorted.begin();
            return (int32_t)std::max<int64_t>(k, c->n_near);
        };
        std::vector<int32_t> nex(T), nle(T), need(T);
        std::vector<int64_t> exo(T);
        std::vector<double> envm(T);
        int64_t n_ex = 0;
        for (int t = 0; t < T; ++t) {
            std::memcpy(&envm[t], &bits[(size_t)nk * T + t], 8);
            envm[t] *= taus[0];
            if (t == 0) {
                nex[t] = nle[t] = need[t] = (int32_t)n_off;   // line mode 0: every offset, exact
            } else {
                nex[t] = within(cut(0, t));
                nle[t] = std::max(nex[t], within(cut(1, t)));
                need[t] = (nk == 3) ? std::max(nle[t], within(cut(2, t))) : (int32_t)n_off;
            }
            exo[t] = n_ex;
            n_ex += nex[t];
        }
        c->n_need_h = need;
        c->n_exact_h = nex;
        c->n_learn_h = nle;
        c->ex_off_h = exo;
        if ((s = dev_alloc(c, (void**)&c->exact_tab, n_ex * 96)) != FBC_OK ||
            (s = dev_alloc(c, (void**)&c->n_need, (int64_t)T * 4)) != FBC_OK ||
            (s = dev_alloc(c, (void**)&c->n_exact, (int64_t)T * 4)) != FBC_OK ||
            (s = dev_alloc(c, (void**)&c->n_learn, (int64_t)T * 4)) != FBC_OK ||
            (s = dev_alloc(c, (void**)&c->ex_off, (int64_t)T * 8)) != FBC_OK ||
            (s = dev_alloc(c, (void**)&c->env_mode, (int64_t)T * 8)) != FBC_OK) {
            cleanup();
            return s;
        }
        c->store_bytes = n_ex * 96;
        HIPCHK(c, hipMemcpyAsync(c->n_need, need.data(), (size_t)T * 4, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(c->n_exact, nex.data(), (size_t)T * 4, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(c->n_learn, nle.data(), (size_t)T * 4, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(c->ex_off, exo.data(), (size_t)T * 8, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(c->env_mode, envm.data(), (size_t)T * 8, hipMemcpyHostToDevice, st));
        // gathering pass: the exact prefix of every mode
        for (int t0 = 0; t0 < T; t0 += chunk) {
            const int nmc = std::min(chunk, T - t0);
            lattice_modes(t0, nmc);
            for (int t = t0; t < t0 + nmc; ++t)
                if (nex[t] > 0)
                    launch_gather_table(st, pt + (int64_t)(t - t0) * 3 * plane, c->exact_tab + exo[t] * 6, 1, m1, m2,
                                        nex[t], d1_d, d2_d, 0, scale);
        }
    } else {
        for (int t0 = 0; t0 < T; t0 += chunk) {
            const int nmc = std::min(chunk, T - t0);
            lattice_modes(t0, nmc);
            launch_gather_table(st, pt, c->tab + (int64_t)t0 * n_off * 6, nmc, m1, m2, n_off, d1_d, d2_d, n_off * 6,
                                scale);
        }
    }
    HIPCHK(c, hipGetLastError());
    {
        // distance cut-off per table mode, then the windows of every cell
        std::vector<double> rho_cut(T, INFINITY);
        if (sur) {
            for (int t = 1; t < T; ++t)           // zero beyond the generated prefix
                rho_cut[t] = c->n_need_h[t] > 0 ? rho_sorted[c->n_need_h[t] - 1] : 0.0;
        } else if (tau >= 0) {
            unsigned long long* st2;
            if ((s = talloc((void**)&st2, (int64_t)T * 16)) != FBC_OK) {
                cleanup();
                return s;
            }
            launch_tab_rhocut(st, c->tab, T, n_off, d1_d, d2_d, tau, st2, st2 + T);
            std::vector<unsigned long long> bits(T);
            HIPCHK(c, hipMemcpyAsync(bits.data(), st2 + T, (size_t)T * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            for (int t = 0; t < T; ++t) {
                double v;
                std::memcpy(&v, &bits[t], 8);
                rho_cut[t] = v;
            }
        }
        const int rows_tile = gemm_tile_rows(form, c->ctmax);
        compute_windows(c, rho_cut, rows_tile);
    }
    if (!keep && !sur) {
        if (form == FBC_FORM_SPLIT_FP16) {
            // per cell mode: largest table magnitude, which fixes the power-of-two scale
            int64_t na = 0;
            for (CellPlan& p : c->cells) {
                c->amax_off.push_back(na);
                na += p.nm;
            }
            if ((s = dev_alloc(c, (void**)&c->amax, na * 8)) != FBC_OK ||
                (s = dev_alloc(c, (void**)&c->bexp, (int64_t)c->total_rhs * 4)) != FBC_OK) {
                cleanup();
                return s;
            }
        }
        if (row_gauge_active(c)) {
            // kept: the inverse transform adds R_b(m) . sum_i f^_i(m) back in FP64
            int64_t tot_rm = 0;
            for (CellPlan& p : c->cells) {
                c->rowmean_off.push_back(tot_rm);
                tot_rm += (int64_t)p.nm * p.n_b * 6;
            }
            if ((s = dev_alloc(c, (void**)&c->rowmean, tot_rm * 16)) != FBC_OK) {
                cleanup();
                return s;
            }
            c->scratch_bytes += tot_rm * 16;
        }
        // compact store: the chunk-tiles of every window, cell after cell
        const int rows_tile = gemm_tile_rows(form, c->ctmax);
        const int64_t cte = chunk_tile_elems(form, rows_tile);
        int64_t a_tot = 0, max_reg = 0;
        for (CellPlan& p : c->cells) {
            const int nreg = p.nm * p.n_tiles;
            p.reg_pre.assign((size_t)nreg + 1, 0);
            for (int r = 0; r < nreg; ++r) p.reg_pre[r + 1] = p.reg_pre[r] + p.win_len[r];
            p.n_ct = p.reg_pre[nreg];
            p.a_off = a_tot;
            a_tot += p.n_ct * cte;
            max_reg = std::max<int64_t>(max_reg, nreg);
        }
        c->store_bytes = a_tot * store_elem_bytes(form);
        if ((s = dev_alloc(c, &c->store, std::max<int64_t>(c->store_bytes, 256))) != FBC_OK) {
            cleanup();
            return fail(c, FBC_E_NOMEM, "dense store of " + std::to_string(c->store_bytes) +
                                            " B (the blocks inside the negligible-block windows): " + c->err);
        }
        int64_t* reg_d;
        int32_t* ws_d;
        if ((s = talloc((void**)&reg_d, (max_reg + 1) * 8)) != FBC_OK || (s = talloc((void**)&ws_d, max_reg * 4 + 4)) != FBC_OK) {
            cleanup();
            return s;
        }
        for (size_t ci = 0; ci < c->cells.size(); ++ci) {
            CellPlan& p = c->cells[ci];
            const int mult = c->nz_max / p.nz;
            double2* rowmean = nullptr;
            if (row_gauge_active(c)) {
                rowmean = c->rowmean + c->rowmean_off[ci];
                launch_rowmean(st, c->tab, rowmean, p.nm, mult, n_off, p.n_b, p.n_i, p.cols_b_d,
                               p.cols_i_d, c->lut, os.d1min, os.d2min, os.w2);
                // no row gauge where chunks are skipped: the skipped blocks would otherwise
                // drop their share of the row mean
                for (int m = 0; m < p.nm; ++m)
                    if (p.mode_skips[m])
                        HIPCHK(c, hipMemsetAsync(rowmean + (int64_t)m * p.n_b * 6, 0, (size_t)p.n_b * 6 * 16, st));
            }
            char* base = (char*)c->store + p.a_off * store_elem_bytes(form);
            // the previous cell's build must be done with the staging lists before they change
            HIPCHK(c, hipStreamSynchronize(st));
            HIPCHK(c, hipMemcpyAsync(reg_d, p.reg_pre.data(), p.reg_pre.size() * 8, hipMemcpyHostToDevice, st));
            HIPCHK(c, hipMemcpyAsync(ws_d, p.win_start.data(), p.win_start.size() * 4, hipMemcpyHostToDevice, st));
            launch_build_dense(st, form, base, c->tab, rowmean, reg_d, ws_d, p.nm, p.n_tiles, p.n_chunks, rows_tile,
                               p.n_ct, mult, n_off, p.n_b, p.n_i, p.cols_b_d, p.cols_i_d, c->lut, os.d1min,
                               os.d2min, os.w2, form == FBC_FORM_SPLIT_FP16 ? c->amax + c->amax_off[ci] : nullptr);
            HIPCHK(c, hipGetLastError());
        }
        c->tab = nullptr;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    cleanup();
    return FBC_OK;
}

// Algorithmic bytes and flops of one product launch over the non-skipped blocks.
static void product_stats(fbc_ctx* c) {
    const int form = c->opt.form;
    const bool dt = is_table_form(form);
    const int rows_tile = dt ? 96 : gemm_tile_rows(form, c->ctmax);
    const double eb = (form == FBC_FORM_FP64) ? 8.0 : 4.0;       // stored bytes per real entry
    const double fb = (form == FBC_FORM_FP64 || dt) ? 16.0 : 8.0; // bytes per complex f^
    double bytes = 0, flops = 0, area = 0, kept = 0;
    for (const CellPlan& p : c->cells) {
        for (int m = 0; m < p.nm; ++m) {
            bytes += (double)p.R * p.K * fb + (double)p.R * p.M * 16.0;      // f^ in, w^ out
            for (int tl = 0; tl < p.n_tiles; ++tl) {
                const double rows = std::max(0, std::min(p.M, (tl + 1) * rows_tile) - tl * rows_tile);
                const int ws = p.win_start[(size_t)m * p.n_tiles + tl];
                const int wl = p.win_len[(size_t)m * p.n_tiles + tl];
                for (int ch = 0; ch < p.n_chunks; ++ch) {
                    const double kc = dt ? 3.0 * std::max(0, std::min(p.n_i, 8 * (ch + 1)) - 8 * ch)
                                         : (double)std::max(0, std::min(p.K, 32 * (ch + 1)) - 32 * ch);
                    area += rows * kc;
                    if (((ch - ws + p.n_chunks) % p.n_chunks) < wl) {
                        kept += rows * kc;
                        flops += 8.0 * rows * kc * p.R;
                        if (!dt) bytes += (double)rows_tile * 64.0 * eb;
                    }
                }
            }
        }
    }
    if (form == FBC_FORM_SURROGATE) {
        for (int t : c->n_need_h) bytes += t * 96.0;     // generated slices, read once
    } else if (dt) {
        bytes += (double)c->store_bytes;
    }
    c->product_bytes = bytes;
    c->product_flops = flops;
    c->skipped_fraction = area > 0 ? 1.0 - kept / area : 0.0;
}

// ----------------------------------------------------------------------------------
// Work list of the per-mode products.  A unit is one (cell, mode); it expands into
// row tiles x K slices.  Orders:
//   0  XCD-grouped: units, longest first, go to the least-loaded XCD (work groups are
//      dispatched round-robin over the 8 XCDs by block index), so the B fragments of a
//      mode are shared through one XCD's L2;
//   1  mode-major: units by table mode, so every XCD works on the same table slice;
//   2  longest-first: units by cost, natural order;
//   3  jobs longest first, consumed by the persistent work-queue kernel: each work group
//      takes the next job as it finishes the last (surrogate form: its mode-major chunks,
//      longest job first inside each);
//   4  one list per XCD for the persistent kernel: units, longest first, go to the least
//      loaded XCD as in order 0, and each XCD's groups take the jobs of its list in order
//      -- the row tiles of one mode after another, whose overlapping K windows share the
//      f^ fragments in that XCD's L2 -- then help the other lists.
// ----------------------------------------------------------------------------------
struct Unit {
    int cell, m, t;
    int64_t cost;
};

static void unit_jobs(const fbc_ctx* c, const Unit& u, int nsplit, std::vector<GemmJob>& out) {
    const int form = c->opt.form;
    const CellPlan& p = c->cells[u.cell];
    const bool dt = is_table_form(form);
    const int tile_rows = dt ? 96 : gemm_tile_rows(form, c->ctmax);
    const int tiles = p.mp / tile_rows;
    const int unit_k = dt ? 8 : 64;
    for (int ks = 0; ks < nsplit; ++ks)
        for (int tl = 0; tl < tiles; ++tl) {
            // the K slice ks of this tile's window (cyclic; empty slices write zeros)
            const int ws = p.win_start[(size_t)u.m * p.n_tiles + tl];
            const int wl = p.win_len[(size_t)u.m * p.n_tiles + tl];
            const int a = (int)((int64_t)wl * ks / nsplit), e = (int)((int64_t)wl * (ks + 1) / nsplit);
            GemmJob j{};
            j.a_off = dt ? (int64_t)u.t * c->n_offsets * 6
                         : p.a_off + (p.reg_pre[(size_t)u.m * p.n_tiles + tl] + a) * chunk_tile_elems(form, tile_rows);
            j.b_off = p.b_off + (int64_t)u.m * b_mode_elems(form, p);
            j.c_off = p.c_off + ks * p.c_split + (int64_t)u.m * 16;
            j.crs = p.nm * 16;
            j.mb = p.mp / 16;
            j.kp = p.kp;
            j.rb0 = tl * (tile_rows / 16);
            j.ct = p.ct;
            j.cell = u.cell;
            j.k0 = (a == e) ? 0 : unit_k * (ws + a);
            j.k1 = (a == e) ? 0 : unit_k * (ws + e);
            j.ct_active = p.ctr;
            // FP32 MFMA only at modes whose far blocks are skipped: a mode without skipping
            // (mode 0 among them) keeps its whole long-range part, gauge constant included,
            // which FP32 rounding of the blocks would not carry to 1e-6
            j.prec = (dt && c->opt.table_fp32 && p.mode_skips[u.m]) ? 1 : 0;
            out.push_back(j);
        }
}

static std::vector<GemmJob> build_jobs(const fbc_ctx* c, int nsplit, int order, int* list_start = nullptr) {
    const bool dt = is_table_form(c->opt.form);
    std::vector<Unit> units;
    for (int ci = 0; ci < (int)c->cells.size(); ++ci) {
        const CellPlan& p = c->cells[ci];
        const int mult = c->nz_max / p.nz;
        const int64_t tile_rows = dt ? 96 : gemm_tile_rows(c->opt.form, c->ctmax);
        const int64_t unit_k = dt ? 48 : 64;
        for (int m = 0; m < p.nm; ++m) {
            int64_t cost = 0;
            for (int tl = 0; tl < p.n_tiles; ++tl) cost += p.win_len[(size_t)m * p.n_tiles + tl];
            units.push_back({ci, m, m * mult, cost * tile_rows * unit_k});
        }
    }
    std::vector<GemmJob> out;
    if (order == 1 || (order == 3 && c->opt.form == FBC_FORM_SURROGATE)) {
        std::stable_sort(units.begin(), units.end(), [](const Unit& a, const Unit& b) { return a.t < b.t; });
        for (const Unit& u : units) unit_jobs(c, u, nsplit, out);
        return out;
    }
    std::stable_sort(units.begin(), units.end(), [](const Unit& a, const Unit& b) { return a.cost > b.cost; });
    if (order == 2 || order == 3) {
        for (const Unit& u : units) unit_jobs(c, u, nsplit, out);
        if (order == 3)
            std::stable_sort(out.begin(), out.end(), [](const GemmJob& a, const GemmJob& b) {
                return (a.k1 - a.k0) > (b.k1 - b.k0);
            });
        return out;
    }
    std::vector<std::vector<GemmJob>> per_xcd(8);
    std::vector<int64_t> load(8, 0);
    for (const Unit& u : units) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        const size_t before = per_xcd[x].size();
        unit_jobs(c, u, nsplit, per_xcd[x]);
        load[x] += (int64_t)(per_xcd[x].size() - before) * u.cost / std::max<int64_t>(1, nsplit);
    }
    if (order == 4) {            // the XCD lists back to back
        for (int x = 0; x < 8; ++x) {
            if (list_start) list_start[x] = (int)out.size();
            out.insert(out.end(), per_xcd[x].begin(), per_xcd[x].end());
        }
        if (list_start) list_start[8] = (int)out.size();
        return out;
    }
    size_t mx = 0;
    for (auto& v : per_xcd) mx = std::max(mx, v.size());
    out.reserve(mx * 8);
    for (size_t k = 0; k < mx; ++k)
        for (int x = 0; x < 8; ++x) {
            if (k < per_xcd[x].size()) out.push_back(per_xcd[x][k]);
            else {
                GemmJob z{};
                z.mb = 0;      // empty job: every wave returns at once
                out.push_back(z);
            }
        }
    return out;
}

static fbc_status upload_jobs(fbc_ctx* c, int nsplit, int order, hipStream_t st) {
    // the new list, its work lists and chunk starts are formed aside and take effect only
    // once the list is on the device: a failure leaves the current list in place
    int list_start[9] = {0};
    std::vector<GemmJob> jobs = build_jobs(c, nsplit, order, list_start);
    PqLists lists{};
    lists.ctr = c->status + 16;
    lists.nl = (order == 4) ? 8 : 1;
    for (int l = 0; l < 9; ++l) lists.start[l] = (order == 4) ? list_start[l] : (l ? (int)jobs.size() : 0);
    std::vector<int> chunk_job0;
    if (c->opt.form == FBC_FORM_SURROGATE && c->gen_modes > 0) {
        // jobs are in table-mode order; record where each generated chunk starts
        const int T = c->nz_max / 2 + 1;
        size_t j = 0;
        for (int t0 = 0; t0 < T; t0 += c->gen_modes) {
            while (j < jobs.size() && jobs[j].a_off < (int64_t)t0 * c->n_offsets * 6) ++j;
            chunk_job0.push_back((int)j);
        }
        chunk_job0.push_back((int)jobs.size());
        if (order == 3)      // persistent per chunk: longest job first inside each chunk
            for (size_t ch = 0; ch + 1 < chunk_job0.size(); ++ch)
                std::stable_sort(jobs.begin() + chunk_job0[ch], jobs.begin() + chunk_job0[ch + 1],
                                 [](const GemmJob& a, const GemmJob& b) { return (a.k1 - a.k0) > (b.k1 - b.k0); });
    }
    // queued launches may still read the current list: wait for them before replacing it
    HIPCHK(c, hipStreamSynchronize(st));
    GemmJob* dst = c->jobs;
    if ((int64_t)jobs.size() > c->jobs_cap) {
        // a larger list is allocated aside (the old one stays allocated until the context
        // is destroyed), so a failed allocation changes nothing
        fbc_status s = dev_alloc(c, (void**)&dst, (int64_t)jobs.size() * sizeof(GemmJob));
        if (s != FBC_OK) return s;
    }
    HIPCHK(c, hipMemcpyAsync(dst, jobs.data(), jobs.size() * sizeof(GemmJob), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (dst != c->jobs) {
        c->jobs = dst;
        c->jobs_cap = (int64_t)jobs.size();
    }
    c->lists = lists;
    c->chunk_job0.swap(chunk_job0);
    c->njobs = (int)jobs.size();
    c->nsplit = nsplit;
    c->job_order = order;
    if (c->graph_exec) {                 // the captured update refers to the old list
        (void)hipGraphExecDestroy(c->graph_exec);
        (void)hipGraphDestroy(c->graph);
        c->graph_exec = nullptr;
        c->graph = nullptr;
    }
    drop_relax_graph(c);
    return FBC_OK;
}

extern "C" fbc_status fbc_assemble_G(const fbc_lattice* lat, const fbc_cell* cells, int n_cells,
                                     const fbc_options* opt, void* stream, fbc_ctx** out) {
    if (!out) return fail(nullptr, FBC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!lat || !cells || !opt || n_cells <= 0) return fail(nullptr, FBC_E_ARG, "null argument or n_cells <= 0");
    if (!(lat->a > 0) || !(lat->spring_k > 0) || !std::isfinite(lat->a) || !std::isfinite(lat->spring_k))
        return fail(nullptr, FBC_E_ARG, "lattice constant and spring stiffness must be positive");
    if (opt->form < FBC_FORM_FP64 || opt->form > FBC_FORM_SPLIT_FP16)
        return fail(nullptr, FBC_E_ARG, "unknown form");
    if (opt->form == FBC_FORM_SURROGATE && (!opt->surrogate || !opt->surrogate->has_mlp))
        return fail(nullptr, FBC_E_ARG, "the surrogate form needs an fbc_sur with MLP weights");
    if (opt->gen_modes < 0) return fail(nullptr, FBC_E_ARG, "gen_modes must be >= 0");
    if (opt->table_fp32 != 0 && opt->table_fp32 != 1) return fail(nullptr, FBC_E_ARG, "table_fp32 must be 0 or 1");
    if (opt->table_fp32 && !is_table_form(opt->form))
        return fail(nullptr, FBC_E_ARG, "table_fp32 applies to the offset-table forms (FP64 table, surrogate)");
    if (!is_pow2(opt->bz_m1) || !is_pow2(opt->bz_m2) || opt->bz_m1 < 8 || opt->bz_m2 < 8 ||
        opt->bz_m1 > 4096 || opt->bz_m2 > 4096)
        return fail(nullptr, FBC_E_ARG, "bz_m1, bz_m2 must be powers of two in [8, 4096]");
    if (!(opt->netforce_tol >= 0)) return fail(nullptr, FBC_E_ARG, "netforce_tol must be >= 0");
    for (int i = 0; i < n_cells; ++i) {
        const fbc_cell& cl = cells[i];
        if (!is_pow2(cl.nz) || cl.nz < 2 || cl.nz > 4096)
            return fail(nullptr, FBC_E_ARG, "nz must be a power of two in [2, 4096]");
        if (cl.n_i < 1 || cl.n_b < 1 || cl.n_rhs < 1 || !cl.cols_i || !cl.cols_b)
            return fail(nullptr, FBC_E_ARG, "cell sizes must be >= 1 and column arrays non-null");
        if ((int64_t)cl.n_i * 6 > (1 << 30) || (int64_t)cl.n_b * 3 > (1 << 30))
            return fail(nullptr, FBC_E_ARG, "cell too large");
        if (cl.n_rhs > 65535) return fail(nullptr, FBC_E_ARG, "n_rhs must be <= 65535");
        if (cl.n_rhs > 64) return fail(nullptr, FBC_E_ARG, "at most 64 RHS per cell");
    }

    fbc_ctx* c = new (std::nothrow) fbc_ctx();
    if (!c) return fail(nullptr, FBC_E_NOMEM, "host allocation");
    c->opt = *opt;
    c->lat = *lat;
    c->sur = opt->surrogate;
    (void)hipGetDevice(&c->device);
    apply_kernels_init();            // dynamic-LDS limits of the long-line transforms, before any capture
    hipStream_t st = (hipStream_t)stream;
    const int form = opt->form;

    // plan: one column-tile count for the whole context (template of the product kernel),
    // rows padded to whole work-group tiles, K' padded to a multiple of 64
    int ctmax = 1;
    for (int i = 0; i < n_cells; ++i) ctmax = std::max(ctmax, (cells[i].n_rhs + 7) / 8);
    const int ctl = ctmax <= 1 ? 1 : ctmax <= 2 ? 2 : ctmax <= 4 ? 4 : 8;
    const int rows_tile = gemm_tile_rows(form, ctl);
    c->ctmax = ctl;
    int64_t f_off = 0, u_off = 0, b_off = 0, c_off = 0, w_off = 0;
    int rhs0 = 0;
    int64_t tiles_total = 0;   // (cell, mode, row tile) work items before the K split
    int kslices_max = 1 << 30;
    for (int i = 0; i < n_cells; ++i) {
        CellPlan p{};
        p.nz = cells[i].nz;
        p.nm = p.nz / 2 + 1;
        p.n_i = cells[i].n_i;
        p.n_b = cells[i].n_b;
        p.R = cells[i].n_rhs;
        p.K = 3 * p.n_i;
        p.M = 3 * p.n_b;
        if (is_table_form(form)) {
            p.kp = 6 * (int)roundup(p.n_i, 8);       // whole chunks of 8 interface columns
            p.mp = (int)roundup(p.M, 96);            // whole tiles of 32 pad columns
        } else {
            p.kp = (int)roundup(6 * (int64_t)p.n_i, 64);
            p.mp = (int)roundup(p.M, rows_tile);
        }
        p.ct = ctl;
        p.ctr = (p.R + 7) / 8;
        p.f_off = f_off;
        p.u_off = u_off;
        p.a_off = 0;
        p.b_off = b_off;
        p.c_off = c_off;
        p.w_off = w_off;
        p.rhs0 = rhs0;
        p.cols_i.assign(cells[i].cols_i, cells[i].cols_i + 2 * p.n_i);
        p.cols_b.assign(cells[i].cols_b, cells[i].cols_b + 2 * p.n_b);
        f_off += (int64_t)p.R * p.nz * p.K;
        u_off += (int64_t)p.R * p.nz * p.M;
        b_off += b_mode_elems(form, p) * p.nm;
        p.c_split = (int64_t)p.nm * p.ct * p.mp * 16;
        if (is_table_form(form)) {
            tiles_total += (int64_t)p.nm * (p.mp / 96);
            kslices_max = std::min(kslices_max, (p.n_i + 7) / 8);
        } else {
            tiles_total += (int64_t)p.nm * (p.mp / rows_tile);
            kslices_max = std::min(kslices_max, p.kp / 64);
        }
        w_off += (int64_t)p.R * p.M * p.nz;
        rhs0 += p.R;
        c->nz_max = std::max(c->nz_max, p.nz);
        c->cells.push_back(p);
    }
    // K slices: enough work items for several rounds of the resident work groups
    // (256 CUs x 3 groups), so the last round leaves little of the chip idle
    {
        const int64_t want = 6 * 768;
        int ks = (int)std::min<int64_t>((want + tiles_total - 1) / tiles_total, kslices_max);
        c->nsplit = std::max(1, std::min(ks, 8));
        // room for up to 8 slices within 4 GiB of partial outputs (the autotuner may pick more)
        int64_t per_split = 0;
        for (auto& p : c->cells) per_split += p.c_split * 8;
        int cap = (int)std::min<int64_t>(8, std::max<int64_t>(1, ((int64_t)4 << 30) / std::max<int64_t>(1, per_split)));
        cap = std::min(cap, std::max(1, kslices_max));
        c->nsplit_cap = std::max(cap, c->nsplit);
        int64_t co = 0;
        for (auto& p : c->cells) {
            p.c_off = co;
            co += p.c_split * c->nsplit_cap;
        }
        c_off = co;
    }
    c->total_rhs = rhs0;
    c->f_elems = f_off;
    c->u_elems = u_off;
    fbc_status s;
    // the dense store is allocated once the negligible-block windows are known (assembly)
    if ((s = dev_alloc(c, &c->bfrag, b_off * b_elem_bytes(form))) != FBC_OK) goto fail_out;
    if ((s = dev_alloc(c, (void**)&c->cbuf, c_off * 8)) != FBC_OK) goto fail_out;
    if ((s = dev_alloc(c, (void**)&c->wbuf, w_off * 8)) != FBC_OK) goto fail_out;
    if ((s = dev_alloc(c, (void**)&c->status, 128)) != FBC_OK) goto fail_out;
    c->scratch_bytes = b_off * b_elem_bytes(form) + c_off * 8 + w_off * 8;
    {
        // per-cell small buffers
        int64_t sums_n = 0, wmax_n = 0, sp_n = 0, rp_n = 0, shat_n = 0;
        for (auto& p : c->cells) {
            sums_n += (int64_t)p.R * p.nz * 8;
            c->shat_off.push_back(shat_n);
            shat_n += (int64_t)p.R * p.nm * 3;
            int tr, pp;
            irfft_shape(p.nz, &tr, &pp);
            const int np_ir = (p.M + tr - 1) / tr;
            int np_up = 0;                   // the fused update's row groups (relaxation without a bound)
            if (update_shape(p.nz, p.M, p.ctr, &tr, &pp)) np_up = (p.M + tr - 1) / tr;
            c->wmax_off.push_back(wmax_n);
            c->sum_part_off.push_back(sp_n);
            c->rpart_off.push_back(rp_n);
            c->npart_irfft.push_back(np_ir);
            c->npart_update.push_back(np_up);
            wmax_n += (int64_t)p.R * std::max(np_ir, np_up);
            sp_n += (int64_t)p.R * mean_blocks((int64_t)p.nz * p.M) * 6;
            rp_n += (int64_t)p.R * 64 * 3;
        }
        if ((s = dev_alloc(c, (void**)&c->sums, sums_n * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->ftot, (int64_t)c->total_rhs * 3 * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->shat, shat_n * 16)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->shat_on, (int64_t)c->total_rhs * 4)) != FBC_OK) goto fail_out;
        c->scratch_bytes += shat_n * 16 + (int64_t)c->total_rhs * 28;
        if ((s = dev_alloc(c, (void**)&c->wmax_part, wmax_n * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->sum_part, sp_n * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->rpart, rp_n * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->mean, (int64_t)c->total_rhs * 3 * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->rmean, (int64_t)c->total_rhs * 3 * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->alpha, (int64_t)c->total_rhs * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->finf, (int64_t)c->total_rhs * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&c->stepinf, (int64_t)c->total_rhs * 8)) != FBC_OK) goto fail_out;
        c->scratch_bytes += (sums_n + wmax_n + sp_n + rp_n + 5LL * c->total_rhs) * 8;
    }
    // line twiddles, per distinct nz
    {
        std::map<int, int64_t> off;
        std::vector<double2> all, t;
        for (auto& p : c->cells) {
            if (!off.count(p.nz)) {
                off[p.nz] = (int64_t)all.size();
                twiddles(p.nz, t);
                all.insert(all.end(), t.begin(), t.end());
            }
            p.tw_off = off[p.nz];
            p.tw_n = p.nz;
        }
        if ((s = dev_alloc(c, (void**)&c->tw, (int64_t)all.size() * 16)) != FBC_OK) goto fail_out;
        HIPCHK(c, hipMemcpyAsync(c->tw, all.data(), all.size() * 16, hipMemcpyHostToDevice, st));
    }
    for (auto& p : c->cells) {
        if ((s = dev_alloc(c, (void**)&p.cols_i_d, (int64_t)p.n_i * 8)) != FBC_OK) goto fail_out;
        if ((s = dev_alloc(c, (void**)&p.cols_b_d, (int64_t)p.n_b * 8)) != FBC_OK) goto fail_out;
        HIPCHK(c, hipMemcpyAsync(p.cols_i_d, p.cols_i.data(), (size_t)p.n_i * 8, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(p.cols_b_d, p.cols_b.data(), (size_t)p.n_b * 8, hipMemcpyHostToDevice, st));
    }
    {
        std::vector<CellDev> cd;
        for (auto& p : c->cells) cd.push_back(CellDev{p.cols_b_d, p.cols_i_d, p.n_b, p.n_i});
        if ((s = dev_alloc(c, (void**)&c->celldev, (int64_t)cd.size() * sizeof(CellDev))) != FBC_OK) goto fail_out;
        HIPCHK(c, hipMemcpyAsync(c->celldev, cd.data(), cd.size() * sizeof(CellDev), hipMemcpyHostToDevice, st));
    }
    HIPCHK(c, hipMemsetAsync(c->bfrag, 0, (size_t)(b_off * b_elem_bytes(form)), st));
    HIPCHK(c, hipMemsetAsync(c->status, 0, 128, st));
    {
        // sin(pi p / L) table, L = max over every line length and the torus sizes
        int L = std::max(opt->bz_m1, opt->bz_m2);
        for (auto& p : c->cells) L = std::max(L, p.nz);
        const int logL = ilog2(L);
        std::vector<double> sn(L);
        for (int q = 0; q < L; ++q)
            sn[q] = (double)sinl(3.14159265358979323846264338327950288L * q / L);
        double* sn_d = nullptr;
        if (hipMalloc((void**)&sn_d, (size_t)L * 8) != hipSuccess) {
            (void)hipGetLastError();
            s = fail(c, FBC_E_NOMEM, "sin table");
            goto fail_out;
        }
        (void)hipMemcpyAsync(sn_d, sn.data(), (size_t)L * 8, hipMemcpyHostToDevice, st);
        const BondTable bt = make_bonds(lat->spring_k);
        s = assemble_all(c, st, bt, sn_d, logL);
        if (s != FBC_OK) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(sn_d);
            goto fail_out;
        }
        (void)hipStreamSynchronize(st);
        (void)hipFree(sn_d);
    }
    product_stats(c);
    if (form == FBC_FORM_SURROGATE) c->nsplit = 1;     // slices are generated per mode chunk
    // default lists: mode-major for the offset table, mode-major chunks consumed by the
    // persistent kernel for the surrogate (1 % faster on the long workload), XCD-grouped
    // for the dense stores
    if ((s = upload_jobs(c, c->nsplit, form == FBC_FORM_SURROGATE ? 3 : is_table_form(form) ? 1 : 0, st)) != FBC_OK)
        goto fail_out;
    if ((s = dev_alloc(c, (void**)&c->fprev, c->f_elems * 8)) != FBC_OK) goto fail_out;
    HIPCHK(c, hipStreamSynchronize(st));
    HIPCHK(c, hipGetLastError());
    *out = c;
    return FBC_OK;
fail_out:
    g_err = c->err;
    (void)hipStreamSynchronize(st);
    free_all(c);
    delete c;
    return s;
}

// ----------------------------------------------------------------------------------
// Apply pipeline: net force -> line rFFT -> per-mode products -> inverse rFFT.
// ----------------------------------------------------------------------------------
// Inverse transform of one cell's product output into the w scratch, with the per-row-group
// maxima of |w| (the step bound of Algorithm 2).
static void enqueue_to_w(fbc_ctx* c, size_t ci, hipStream_t st) {
    const bool comp = row_gauge_active(c);
    const bool f16 = (c->opt.form == FBC_FORM_SPLIT_FP16);
    auto& p = c->cells[ci];
    launch_line_irfft(st, c->cbuf + p.c_off, c->wbuf + p.w_off, c->wmax_part + c->wmax_off[ci], p.R, p.nz,
                      p.mp, p.M, p.ct, p.ctr, c->tw + p.tw_off, c->nsplit, p.c_split,
                      comp ? c->rowmean + c->rowmean_off[ci] : nullptr, comp ? c->shat + c->shat_off[ci] : nullptr,
                      comp ? c->shat_on + p.rhs0 : nullptr, f16 ? c->amax + c->amax_off[ci] : nullptr,
                      f16 ? c->bexp + p.rhs0 : nullptr, nullptr);
}

static void enqueue_forward(fbc_ctx* c, const double* f, hipStream_t st) {
    const int form = c->opt.form;
    int64_t sums_off = 0;
    const bool comp = row_gauge_active(c);
    const bool f16 = (form == FBC_FORM_SPLIT_FP16);
    for (size_t ci = 0; ci < c->cells.size(); ++ci) {
        auto& p = c->cells[ci];
        const double* fc = f + p.f_off;
        double* sums = c->sums + sums_off;
        double* tot = c->ftot + 3 * p.rhs0;
        int* bexp = f16 ? c->bexp + p.rhs0 : nullptr;
        if (c->opt.check_netforce || c->opt.project_netforce || comp || f16)
            launch_netforce(st, fc, sums, tot, comp ? c->shat + c->shat_off[ci] : nullptr,
                            comp ? c->shat_on + p.rhs0 : nullptr, p.R, p.nz, p.n_i, c->opt.netforce_tol,
                            c->opt.check_netforce, c->opt.project_netforce, c->tw + p.tw_off, bexp,
                            c->status);
        void* bm = (char*)c->bfrag + p.b_off * b_elem_bytes(form);
        launch_line_rfft(st, form, fc, tot, c->opt.project_netforce, bm, p.R, p.nz, p.n_i, p.kp,
                         p.ct, c->tw + p.tw_off, bexp);
        sums_off += (int64_t)p.R * p.nz * 8;
    }
    const bool tm = c->timing && c->n_timed < kMaxTimed;
    if (tm) (void)hipEventRecord(c->ev[2 * c->n_timed], st);
    if (form == FBC_FORM_SURROGATE) {
        // generate a chunk of table modes, then run the products of those modes
        const int T = c->nz_max / 2 + 1;
        const fbc_sur* sv = c->sur;
        for (size_t ch = 0; ch + 1 < c->chunk_job0.size(); ++ch) {
            const int t0 = (int)ch * c->gen_modes;
            const int nt = std::min(c->gen_modes, T - t0);
            int64_t max_need = 0, min_exact = INT64_MAX, max_exact = 0, min_learn = INT64_MAX, max_band = 0;
            for (int t = t0; t < t0 + nt; ++t) {
                max_need = std::max<int64_t>(max_need, c->n_need_h[t]);
                min_exact = std::min<int64_t>(min_exact, c->n_exact_h[t]);
                max_exact = std::max<int64_t>(max_exact, c->n_exact_h[t]);
                min_learn = std::min<int64_t>(min_learn, c->n_learn_h[t]);
                max_band = std::max<int64_t>(max_band, (int64_t)c->n_learn_h[t] - c->n_exact_h[t]);
            }
            launch_sur_generate(st, sv->view(), sv->infer(), sv->r_c, c->env_mode, sv->rho_learn, c->nz_max, t0, nt,
                                c->exact_tab, c->ex_off, c->n_exact, c->n_learn, c->n_offsets, c->n_need,
                                c->off_d1, c->off_d2, c->gen, min_exact, max_exact, min_learn, max_band, max_need);
            const int j0 = c->chunk_job0[ch], j1 = c->chunk_job0[ch + 1];
            PqLists ql{};
            ql.ctr = c->status + 16;
            ql.nl = 1;
            for (int l = 0; l < 9; ++l) ql.start[l] = j1 - j0;
            ql.start[0] = 0;
            launch_gemm_dtab(st, c->jobs + j0, j1 - j0, c->ctmax, c->gen, (int64_t)t0 * c->n_offsets * 6,
                             (const double*)c->bfrag, c->cbuf, c->celldev, c->lut, c->d1min, c->d2min, c->w2,
                             c->n_need, c->n_offsets, c->job_order == 3 ? &ql : nullptr, c->opt.table_fp32);
        }
    } else if (form == FBC_FORM_DTABLE_FP64 && c->hmat) {
        const CellPlan& p = c->cells[0];          // one cell (checked when attached)
        hmat_enqueue_pipeline(c->hmat, (const double*)c->bfrag + p.b_off, b_mode_elems(form, p), p.kp,
                              c->cbuf + p.c_off, p.mp, p.nm, p.ct, st);
    } else if (form == FBC_FORM_DTABLE_FP64)
        launch_gemm_dtab(st, c->jobs, c->njobs, c->ctmax, c->tab, 0, (const double*)c->bfrag, c->cbuf,
                         c->celldev, c->lut, c->d1min, c->d2min, c->w2, nullptr, c->n_offsets,
                         c->job_order >= 3 ? &c->lists : nullptr, c->opt.table_fp32);
    else
        launch_gemm(st, form, c->jobs, c->njobs, c->ctmax, c->store, c->bfrag, c->cbuf,
                    c->job_order >= 3 ? &c->lists : nullptr, c->variant);
    if (tm) {
        (void)hipEventRecord(c->ev[2 * c->n_timed + 1], st);
        ++c->n_timed;
    }
}

// Fused inverse transform and update of every cell: u <- u - alpha G f minus the mean of
// the result (mean_removal), or u <- -alpha G f.
static void enqueue_update(fbc_ctx* c, double* u, double alpha, bool mean_removal, hipStream_t st) {
    const bool comp = row_gauge_active(c);
    const bool f16 = (c->opt.form == FBC_FORM_SPLIT_FP16);
    for (size_t ci = 0; ci < c->cells.size(); ++ci) {
        auto& p = c->cells[ci];
        const double2* rm = comp ? c->rowmean + c->rowmean_off[ci] : nullptr;
        const double2* sh = comp ? c->shat + c->shat_off[ci] : nullptr;
        const int* so = comp ? c->shat_on + p.rhs0 : nullptr;
        const unsigned long long* am = f16 ? c->amax + c->amax_off[ci] : nullptr;
        const int* be = f16 ? c->bexp + p.rhs0 : nullptr;
        int tr, pp;
        if (!update_shape(p.nz, p.M, p.ctr, &tr, &pp)) {
            // lines outside 16..1024 layers: inverse transform into w, then the tiled transpose-update,
            // which also removes the mean (known beforehand, as for the fused update)
            double* uc = u + p.u_off;
            double* sp = c->sum_part + c->sum_part_off[ci];
            double* mu = nullptr;
            if (mean_removal) {
                mu = c->mean + 3 * p.rhs0;
                launch_update_mean(st, uc, c->cbuf + p.c_off, sp, p.R, p.nz, p.mp, p.M, c->nsplit, p.c_split, rm,
                                   sh, so, am, be, alpha, mu, c->status);
            }
            launch_line_irfft(st, c->cbuf + p.c_off, c->wbuf + p.w_off, c->wmax_part + c->wmax_off[ci], p.R,
                              p.nz, p.mp, p.M, p.ct, p.ctr, c->tw + p.tw_off, c->nsplit, p.c_split, rm, sh,
                              so, am, be, nullptr);
            if (!mean_removal) launch_fill(st, uc, (int64_t)p.R * p.nz * p.M, 0.0);
            // the mean is known beforehand: no partial sums
            launch_axpy(st, c->wbuf + p.w_off, uc, p.R, p.nz, p.M, alpha, nullptr, c->status, mu);
            continue;
        }
        double* mu = nullptr;
        if (mean_removal) {
            mu = c->mean + 3 * p.rhs0;
            launch_update_mean(st, u + p.u_off, c->cbuf + p.c_off, c->sum_part + c->sum_part_off[ci], p.R,
                               p.nz, p.mp, p.M, c->nsplit, p.c_split, rm, sh, so, am, be, alpha, mu, c->status);
        }
        launch_irfft_update(st, c->cbuf + p.c_off, u + p.u_off, p.R, p.nz, p.mp, p.M, p.ctr,
                            c->tw + p.tw_off, c->nsplit, p.c_split, rm, sh, so, am, be, alpha, mu,
                            mean_removal ? 1 : 0, c->status);
    }
}

static fbc_status check_apply_args(fbc_ctx* c, const void* f, const void* u) {
    if (!c) return fail(nullptr, FBC_E_ARG, "ctx is NULL");
    if (!f || !u) return fail(c, FBC_E_ARG, "f and u must be device pointers");
    if (((uintptr_t)f & 7) || ((uintptr_t)u & 7)) return fail(c, FBC_E_ARG, "f and u must be 8-byte aligned");
    return FBC_OK;
}

extern "C" fbc_status fbc_apply(fbc_ctx* c, const double* f, double* u, double alpha, void* stream) {
    fbc_status s = check_apply_args(c, f, u);
    if (s != FBC_OK) return s;
    if (!std::isfinite(alpha)) return fail(c, FBC_E_ARG, "alpha must be finite");
    hipStream_t st = (hipStream_t)stream;
    // the forward half, then per cell the mean and the fused inverse transform + update
    enqueue_forward(c, f, st);
    enqueue_update(c, u, alpha, true, st);
    HIPCHK(c, hipGetLastError());
    return FBC_OK;
}

extern "C" fbc_status fbc_apply_graph(fbc_ctx* c, const double* f, double* u, double alpha,
                                      void* stream) {
    fbc_status s = check_apply_args(c, f, u);
    if (s != FBC_OK) return s;
    if (!std::isfinite(alpha)) return fail(c, FBC_E_ARG, "alpha must be finite");
    if (!stream) return fail(c, FBC_E_ARG, "graph capture needs a non-default stream");
    hipStream_t st = (hipStream_t)stream;
    if (!(c->graph_exec && c->g_f == f && c->g_u == u && c->g_alpha == alpha && c->g_stream == stream)) {
        if (c->graph_exec) {
            (void)hipGraphExecDestroy(c->graph_exec);
            (void)hipGraphDestroy(c->graph);
            c->graph_exec = nullptr;
            c->graph = nullptr;
        }
        const int timing = c->timing;
        c->timing = 0;
        HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        s = fbc_apply(c, f, u, alpha, stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        c->timing = timing;
        if (s != FBC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return fail(c, FBC_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        HIPCHK(c, hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
        c->graph = g;
        c->g_f = f;
        c->g_u = u;
        c->g_alpha = alpha;
        c->g_stream = stream;
    }
    HIPCHK(c, hipGraphLaunch(c->graph_exec, st));
    return FBC_OK;
}

static int n_variants(const fbc_ctx* c) { return is_table_form(c->opt.form) ? 1 : gemm_variants(c->opt.form, c->ctmax); }

extern "C" fbc_status fbc_autotune(fbc_ctx* c, const double* f, double* w, int reps,
                                   fbc_tune_result* out, void* stream) {
    fbc_status s = check_apply_args(c, f, w);
    if (s != FBC_OK) return s;
    if (c->hmat) return fail(c, FBC_E_STATE, "an H-matrix is attached: its product has no work list to tune");
    if (reps < 1 || reps > 1000) return fail(c, FBC_E_ARG, "reps must be in [1, 1000]");
    if (c->opt.form == FBC_FORM_SURROGATE) return fail(c, FBC_E_UNSUPPORTED, "the surrogate form keeps its mode-major list");
    hipStream_t st = (hipStream_t)stream;
    const int timing = c->timing;
    double ms0;
    int n0;
    if ((s = fbc_timing(c, 1)) != FBC_OK) return s;
    if ((s = fbc_timing_read(c, &ms0, &n0)) != FBC_OK) return s;   // drop earlier records
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, FBC_E_DEVICE, "hipEventCreate failed");
    }
    struct Cand {
        int var, order, ks;
        double call, gemm;
    };
    std::vector<Cand> cand;
    // one timing of candidate (var, order, ks): a warm-up call, then `n_rep` calls
    auto time_one = [&](Cand& x, int n_rep) -> fbc_status {
        c->variant = x.var;
        fbc_status r;
        if ((r = upload_jobs(c, x.ks, x.order, st)) != FBC_OK) return r;
        if ((r = fbc_green_apply(c, f, w, stream)) != FBC_OK) return r;       // warm-up
        if ((r = fbc_timing_read(c, &ms0, &n0)) != FBC_OK) return r;
        (void)hipEventRecord(e0, st);
        for (int k = 0; k < n_rep && r == FBC_OK; ++k) r = fbc_green_apply(c, f, w, stream);
        if (r != FBC_OK) return r;
        (void)hipEventRecord(e1, st);
        double ms;
        int n;
        if ((r = fbc_timing_read(c, &ms, &n)) != FBC_OK) return r;
        float call = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&call, e0, e1) != hipSuccess)
            return fail(c, FBC_E_DEVICE, "hipEventElapsedTime failed");
        x.call = call / n_rep;
        x.gemm = ms / std::max(1, n);
        return FBC_OK;
    };
    const int nv = n_variants(c);
    for (int var = 0; var < nv && s == FBC_OK; ++var)
        for (int order = 0; order < 5 && s == FBC_OK; ++order)
            for (int ks = 1; ks <= c->nsplit_cap && s == FBC_OK; ks *= 2) {
                Cand x{var, order, ks, 0.0, 0.0};
                if ((s = time_one(x, reps)) == FBC_OK) cand.push_back(x);
            }
    // Candidates within 4 % of the fastest are timed again, in interleaved rounds, and the
    // one with the least summed time wins: single timings of near-equal lists are decided
    // by noise otherwise.
    double best = 1e300, best_gemm = 0.0;
    int best_split = c->nsplit, best_order = c->job_order, best_var = c->variant;
    const int ncand = (int)cand.size();
    if (s == FBC_OK && ncand > 0) {
        double t_min = 1e300;
        for (const Cand& x : cand) t_min = std::min(t_min, x.call);
        std::vector<Cand> top;
        for (const Cand& x : cand)
            if (x.call <= 1.04 * t_min) top.push_back(x);
        std::vector<double> sum(top.size(), 0.0), gsum(top.size(), 0.0);
        const int rounds = top.size() > 1 ? 3 : 0;
        for (int rd = 0; rd < rounds && s == FBC_OK; ++rd)
            for (size_t q = 0; q < top.size() && s == FBC_OK; ++q) {
                Cand x = top[q];
                if ((s = time_one(x, reps)) != FBC_OK) break;
                sum[q] += x.call;
                gsum[q] += x.gemm;
            }
        for (size_t q = 0; q < top.size() && s == FBC_OK; ++q) {
            const double t = rounds ? sum[q] / rounds : top[q].call;
            if (t < best) {
                best = t;
                best_gemm = rounds ? gsum[q] / rounds : top[q].gemm;
                best_split = top[q].ks;
                best_order = top[q].order;
                best_var = top[q].var;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->variant = best_var;
    if (s == FBC_OK) s = upload_jobs(c, best_split, best_order, st);
    c->timing = timing;
    if (s != FBC_OK) return s;
    if (out) {
        out->nsplit = best_split;
        out->order = best_order;
        out->gemm_ms = best_gemm;
        out->n_candidates = ncand;
        out->call_ms = best;
        out->variant = best_var;
        out->from_cache = 0;
    }
    return FBC_OK;
}

// Key of a tuned configuration: FNV-1a over everything that decides the product's work
// (form, tolerance, row gauge, torus, cells with their column sets and RHS, column
// tiles) and the device it ran on.
static uint64_t tune_key(const fbc_ctx* c) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    const int version = 1;
    mix(&version, sizeof version);
    mix(&c->opt.form, sizeof c->opt.form);
    mix(&c->opt.skip_tol, sizeof c->opt.skip_tol);
    mix(&c->opt.row_gauge, sizeof c->opt.row_gauge);
    mix(&c->opt.bz_m1, sizeof c->opt.bz_m1);
    mix(&c->opt.bz_m2, sizeof c->opt.bz_m2);
    mix(&c->ctmax, sizeof c->ctmax);
    for (const CellPlan& p : c->cells) {
        const int hd[4] = {p.nz, p.n_i, p.n_b, p.R};
        mix(hd, sizeof hd);
        mix(p.cols_i.data(), p.cols_i.size() * 4);
        mix(p.cols_b.data(), p.cols_b.size() * 4);
    }
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
        mix(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
        mix(&prop.multiProcessorCount, sizeof prop.multiProcessorCount);
    }
    return h;
}

extern "C" fbc_status fbc_autotune_cached(fbc_ctx* c, const double* f, double* w, int reps, const char* path,
                                          fbc_tune_result* out, void* stream) {
    fbc_status s = check_apply_args(c, f, w);
    if (s != FBC_OK) return s;
    if (!path) return fail(c, FBC_E_ARG, "cache_path is NULL");
    if (c->opt.form == FBC_FORM_SURROGATE) return fail(c, FBC_E_UNSUPPORTED, "the surrogate form keeps its mode-major list");
    char key[17];
    snprintf(key, sizeof key, "%016llx", (unsigned long long)tune_key(c));
    // the last valid line for this key wins
    int var = -1, ns = 0, ord = 0;
    double gm = 0, cm = 0;
    if (FILE* fp = std::fopen(path, "r")) {
        char line[256];
        while (std::fgets(line, sizeof line, fp)) {
            char k[32];
            int v, n, o;
            double g, cc;
            if (std::sscanf(line, "fbc-tune %31s %d %d %d %lf %lf", k, &v, &n, &o, &g, &cc) == 6 &&
                std::strcmp(k, key) == 0 && v >= 0 && v < n_variants(c) && n >= 1 && n <= c->nsplit_cap && o >= 0 &&
                o <= 4) {
                var = v;
                ns = n;
                ord = o;
                gm = g;
                cm = cc;
            }
        }
        std::fclose(fp);
    }
    if (var >= 0) {
        c->variant = var;
        if ((s = upload_jobs(c, ns, ord, (hipStream_t)stream)) != FBC_OK) return s;
        if (out) *out = fbc_tune_result{ns, ord, gm, 0, cm, var, 1};
        return FBC_OK;
    }
    fbc_tune_result r{};
    if ((s = fbc_autotune(c, f, w, reps, &r, stream)) != FBC_OK) return s;
    FILE* fp = std::fopen(path, "a");
    if (!fp) return fail(c, FBC_E_ARG, std::string("cannot append to the cache file ") + path);
    std::fprintf(fp, "fbc-tune %s %d %d %d %.6f %.6f\n", key, r.variant, r.nsplit, r.order, r.gemm_ms, r.call_ms);
    std::fclose(fp);
    if (out) *out = r;
    return FBC_OK;
}

extern "C" fbc_status fbc_set_kernel_variant(fbc_ctx* c, int variant) {
    if (!c) return fail(nullptr, FBC_E_ARG, "ctx is NULL");
    if (variant < 0 || variant >= n_variants(c))
        return fail(c, FBC_E_ARG, "variant must be in [0, " + std::to_string(n_variants(c)) + ")");
    if (variant != c->variant && c->graph_exec) {      // the captured update launches the old kernel
        (void)hipGraphExecDestroy(c->graph_exec);
        (void)hipGraphDestroy(c->graph);
        c->graph_exec = nullptr;
        c->graph = nullptr;
    }
    if (variant != c->variant) drop_relax_graph(c);
    c->variant = variant;
    return FBC_OK;
}

extern "C" fbc_status fbc_set_work_list(fbc_ctx* c, int nsplit, int order, void* stream) {
    if (!c) return fail(nullptr, FBC_E_ARG, "ctx is NULL");
    if (c->hmat) return fail(c, FBC_E_STATE, "an H-matrix is attached: detach it first");
    if (nsplit < 1 || nsplit > c->nsplit_cap)
        return fail(c, FBC_E_ARG, "nsplit must be in [1, " + std::to_string(c->nsplit_cap) + "]");
    if (order < 0 || order > 4) return fail(c, FBC_E_ARG, "order must be 0, 1, 2, 3 or 4");
    if (c->opt.form == FBC_FORM_SURROGATE && (nsplit != 1 || (order != 1 && order != 3)))
        return fail(c, FBC_E_UNSUPPORTED, "the surrogate form keeps its mode-major chunks (nsplit 1, order 1 or 3)");
    return upload_jobs(c, nsplit, order, (hipStream_t)stream);
}

extern "C" fbc_status fbc_green_apply(fbc_ctx* c, const double* f, double* w, void* stream) {
    fbc_status s = check_apply_args(c, f, w);
    if (s != FBC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    enqueue_forward(c, f, st);
    enqueue_update(c, w, -1.0, false, st);
    HIPCHK(c, hipGetLastError());
    return FBC_OK;
}

static fbc_status check_relax_opts(fbc_ctx* c, const fbc_relax_opts* o) {
    if (!(o->du_max >= 0) || !(o->tol_f >= 0) || !(o->alpha_min >= 0) || !std::isfinite(o->alpha_min))
        return fail(c, FBC_E_ARG, "du_max, tol_f and alpha_min must be >= 0 (alpha_min finite)");
    return FBC_OK;
}

static void drop_relax_graph(fbc_ctx* c) {
    if (c->rgraph_exec) (void)hipGraphExecDestroy(c->rgraph_exec);
    if (c->rgraph) (void)hipGraphDestroy(c->rgraph);
    c->rgraph_exec = nullptr;
    c->rgraph = nullptr;
}

extern "C" fbc_status fbc_set_hmat(fbc_ctx* c, fbc_hmat* h, void* stream) {
    if (!c) return fail(nullptr, FBC_E_ARG, "ctx is NULL");
    if (h && hmat_context(h) != c) return fail(c, FBC_E_ARG, "the H-matrix was built from another context");
    if (h == c->hmat) return FBC_OK;
    hipStream_t st = (hipStream_t)stream;
    if (h && !c->hmat) {
        // the products land in one K slice: the inverse transform must read one; the work
        // list in place comes back on detaching
        c->hmat_prev_nsplit = c->nsplit;
        if (c->nsplit != 1) {
            fbc_status s = upload_jobs(c, 1, c->job_order, st);
            if (s != FBC_OK) return s;
        }
    } else if (!h && c->hmat_prev_nsplit != c->nsplit) {
        fbc_status s = upload_jobs(c, c->hmat_prev_nsplit, c->job_order, st);
        if (s != FBC_OK) return s;
    }
    HIPCHK(c, hipStreamSynchronize(st));        // queued applies may still use the old product
    c->hmat = h;
    if (c->graph_exec) {                        // captured updates launch the old product
        (void)hipGraphExecDestroy(c->graph_exec);
        (void)hipGraphDestroy(c->graph);
        c->graph_exec = nullptr;
        c->graph = nullptr;
    }
    drop_relax_graph(c);
    return FBC_OK;
}

extern "C" fbc_status fbc_relax_begin(fbc_ctx* c, const fbc_relax_opts* o, void* stream) {
    if (!c || !o) return fail(c, FBC_E_ARG, "null argument");
    fbc_status s = check_relax_opts(c, o);
    if (s != FBC_OK) return s;
    drop_relax_graph(c);                 // the options are kernel arguments of a captured step
    c->ropt = *o;
    c->relax_k = 0;
    launch_fill((hipStream_t)stream, c->alpha, c->total_rhs, 1.0);
    launch_relax_index((hipStream_t)stream, c->status + 4, 0);
    HIPCHK(c, hipGetLastError());
    return FBC_OK;
}

// One relaxation step, enqueued; the iteration index is read and advanced on the device.
static void enqueue_relax(fbc_ctx* c, const double* f_in, double* u, fbc_relax_out* out, hipStream_t st) {
    int* kdev = c->status + 4;
    for (size_t ci = 0; ci < c->cells.size(); ++ci) {
        auto& p = c->cells[ci];
        const int64_t per_rhs = (int64_t)p.nz * p.K;
        launch_relax_alpha(st, f_in + p.f_off, c->fprev + p.f_off, c->rpart + c->rpart_off[ci],
                           c->alpha + p.rhs0, c->finf + p.rhs0, p.R, per_rhs, kdev, c->ropt.relax,
                           c->ropt.alpha_min);
    }
    enqueue_forward(c, f_in, st);
    const bool comp = row_gauge_active(c);
    const bool f16 = (c->opt.form == FBC_FORM_SPLIT_FP16);
    for (size_t ci = 0; ci < c->cells.size(); ++ci) {
        auto& p = c->cells[ci];
        const double2* rm = comp ? c->rowmean + c->rowmean_off[ci] : nullptr;
        const double2* sh = comp ? c->shat + c->shat_off[ci] : nullptr;
        const int* so = comp ? c->shat_on + p.rhs0 : nullptr;
        const unsigned long long* am = f16 ? c->amax + c->amax_off[ci] : nullptr;
        const int* be = f16 ? c->bexp + p.rhs0 : nullptr;
        double* uc = u + p.u_off;
        double* mu = c->rmean + 3 * p.rhs0;
        double* wm = c->wmax_part + c->wmax_off[ci];
        // the mean of the updated u, (sum u - alpha_r sum w) / N with sum w from the mode-0
        // records, is known once the step factors are: the update removes it
        if (c->ropt.du_max <= 0.0 && c->npart_update[ci] > 0) {
            // no step bound: the step factors are known before w, so the fused inverse
            // transform and update takes them, and leaves the maxima of |w| for step_inf
            launch_update_mean(st, uc, c->cbuf + p.c_off, c->sum_part + c->sum_part_off[ci], p.R, p.nz, p.mp,
                               p.M, c->nsplit, p.c_split, rm, sh, so, am, be, 0.0, mu, c->status, c->alpha + p.rhs0);
            launch_irfft_update(st, c->cbuf + p.c_off, uc, p.R, p.nz, p.mp, p.M, p.ctr, c->tw + p.tw_off, c->nsplit,
                                p.c_split, rm, sh, so, am, be, 0.0, mu, 1, c->status, c->alpha + p.rhs0, wm);
            launch_relax_clamp(st, wm, c->npart_update[ci], c->alpha + p.rhs0, c->stepinf + p.rhs0, p.R,
                               c->ropt.du_max, kdev, c->ropt.relax);
            continue;
        }
        // the step bound needs the whole of w first
        enqueue_to_w(c, ci, st);
        launch_relax_clamp(st, wm, c->npart_irfft[ci], c->alpha + p.rhs0, c->stepinf + p.rhs0, p.R,
                           c->ropt.du_max, kdev, c->ropt.relax);
        launch_update_mean(st, uc, c->cbuf + p.c_off, c->sum_part + c->sum_part_off[ci], p.R, p.nz, p.mp, p.M,
                           c->nsplit, p.c_split, rm, sh, so, am, be, 0.0, mu, c->status, c->alpha + p.rhs0);
        launch_axpy(st, c->wbuf + p.w_off, uc, p.R, p.nz, p.M, 0.0, c->alpha + p.rhs0, c->status, mu);
    }
    launch_relax_finish(st, c->alpha, c->finf, c->stepinf, c->rmean, out, c->total_rhs, kdev, c->ropt.tol_f);
}

extern "C" fbc_status fbc_relax_step(fbc_ctx* c, const double* f_in, double* u, fbc_relax_out* out,
                                     void* stream) {
    fbc_status s = check_apply_args(c, f_in, u);
    if (s != FBC_OK) return s;
    if (c->relax_k < 0) return fail(c, FBC_E_STATE, "fbc_relax_begin was not called");
    enqueue_relax(c, f_in, u, out, (hipStream_t)stream);
    c->relax_k += 1;
    HIPCHK(c, hipGetLastError());
    return FBC_OK;
}

extern "C" fbc_status fbc_relax_step_graph(fbc_ctx* c, const double* f_in, double* u, fbc_relax_out* out,
                                           void* stream) {
    fbc_status s = check_apply_args(c, f_in, u);
    if (s != FBC_OK) return s;
    if (c->relax_k < 0) return fail(c, FBC_E_STATE, "fbc_relax_begin was not called");
    if (!stream) return fail(c, FBC_E_ARG, "graph capture needs a non-default stream");
    hipStream_t st = (hipStream_t)stream;
    if (!(c->rgraph_exec && c->rg_f == f_in && c->rg_u == u && c->rg_out == out && c->rg_stream == stream)) {
        drop_relax_graph(c);
        const int timing = c->timing;
        c->timing = 0;
        HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        enqueue_relax(c, f_in, u, out, st);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        c->timing = timing;
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(c, FBC_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        }
        e = hipGraphInstantiate(&c->rgraph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            c->rgraph_exec = nullptr;
            return fail(c, FBC_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        c->rgraph = g;
        c->rg_f = f_in;
        c->rg_u = u;
        c->rg_out = out;
        c->rg_stream = stream;
    }
    HIPCHK(c, hipGraphLaunch(c->rgraph_exec, st));
    c->relax_k += 1;
    return FBC_OK;
}

extern "C" fbc_status fbc_relax_get_state(fbc_ctx* c, fbc_relax_opts* opts, int32_t* k, double* alpha,
                                          double* f_prev, void* stream) {
    if (!c || !opts || !k || !alpha || !f_prev) return fail(c, FBC_E_ARG, "null argument");
    if (c->relax_k < 0) return fail(c, FBC_E_STATE, "fbc_relax_begin was not called");
    hipStream_t st = (hipStream_t)stream;
    int32_t kd = 0;
    HIPCHK(c, hipMemcpyAsync(alpha, c->alpha, (size_t)c->total_rhs * sizeof(double), hipMemcpyDefault, st));
    HIPCHK(c, hipMemcpyAsync(f_prev, c->fprev, (size_t)c->f_elems * sizeof(double), hipMemcpyDefault, st));
    HIPCHK(c, hipMemcpyAsync(&kd, c->status + 4, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    *opts = c->ropt;
    *k = kd;
    return FBC_OK;
}

extern "C" fbc_status fbc_relax_set_state(fbc_ctx* c, const fbc_relax_opts* opts, int32_t k,
                                          const double* alpha, const double* f_prev, void* stream) {
    if (!c || !opts || !alpha || (k > 0 && !f_prev)) return fail(c, FBC_E_ARG, "null argument");
    if (k < 0) return fail(c, FBC_E_ARG, "k must be >= 0");
    fbc_status s = check_relax_opts(c, opts);
    if (s != FBC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    drop_relax_graph(c);
    HIPCHK(c, hipMemcpyAsync(c->alpha, alpha, (size_t)c->total_rhs * sizeof(double), hipMemcpyDefault, st));
    if (k > 0)
        HIPCHK(c, hipMemcpyAsync(c->fprev, f_prev, (size_t)c->f_elems * sizeof(double), hipMemcpyDefault, st));
    launch_relax_index(st, c->status + 4, k);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    c->ropt = *opts;
    c->relax_k = k;
    return FBC_OK;
}

extern "C" fbc_status fbc_sync_status(fbc_ctx* c, void* stream) {
    if (!c) return fail(nullptr, FBC_E_ARG, "ctx is NULL");
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    int st = 0;
    HIPCHK(c, hipMemcpy(&st, c->status, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemset(c->status, 0, sizeof(int)));
    if (st & ST_NONFINITE) return fail(c, FBC_E_NONFINITE, "non-finite interface force");
    if (st & ST_NETFORCE)
        return fail(c, FBC_E_NETFORCE, "net force of a cell (all interface atoms of all layers) exceeds tolerance");
    return FBC_OK;
}

extern "C" fbc_status fbc_get_info(const fbc_ctx* c, fbc_info* info) {
    if (!c || !info) return FBC_E_ARG;
    info->n_cells = (int)c->cells.size();
    info->total_rhs = c->total_rhs;
    info->store_bytes = c->store_bytes;
    info->scratch_bytes = c->scratch_bytes;
    info->f_elems = c->f_elems;
    info->u_elems = c->u_elems;
    info->n_offsets = c->n_offsets;
    info->nsplit = c->nsplit;
    info->job_order = c->job_order;
    info->n_jobs = c->njobs;
    info->product_bytes = c->product_bytes;
    info->product_flops = c->product_flops;
    info->skipped_fraction = c->skipped_fraction;
    info->kernel_variant = c->variant;
    info->n_variants = n_variants(c);
    const std::string shape = is_table_form(c->opt.form) ? std::string("offset table, 32 pad columns x 8 interface columns per step")
                                                         : gemm_shape(c->opt.form, c->ctmax, c->variant);
    std::snprintf(info->kernel_shape, sizeof info->kernel_shape, "%s", shape.c_str());
    return FBC_OK;
}

extern "C" fbc_status fbc_copy_block_rows(fbc_ctx* c, int cell, int m, int b0, int b1, double* out) {
    if (!c || !out) return fail(c, FBC_E_ARG, "null argument");
    if (cell < 0 || cell >= (int)c->cells.size()) return fail(c, FBC_E_ARG, "cell out of range");
    const CellPlan& p = c->cells[cell];
    if (m < 0 || m >= p.nm || b0 < 0 || b1 > p.n_b || b0 >= b1) return fail(c, FBC_E_ARG, "range");
    if (c->opt.form == FBC_FORM_SURROGATE) return fail(c, FBC_E_UNSUPPORTED, "no stored table in the surrogate form");
    if (c->opt.form == FBC_FORM_DTABLE_FP64) {
        // reconstruct the block rows from the offset table
        const int mult = c->nz_max / p.nz;
        HIPCHK(c, hipDeviceSynchronize());
        std::vector<double2> tabm((size_t)c->n_offsets * 6);
        HIPCHK(c, hipMemcpy(tabm.data(), c->tab + (int64_t)m * mult * c->n_offsets * 6,
                            tabm.size() * 16, hipMemcpyDeviceToHost));
        OffsetSet os = offsets_of(c->cells);
        for (int b = b0; b < b1; ++b)
            for (int i = 0; i < p.n_i; ++i) {
                const int x = p.cols_b[2 * b] - p.cols_i[2 * i] - os.d1min;
                const int y = p.cols_b[2 * b + 1] - p.cols_i[2 * i + 1] - os.d2min;
                const int64_t o = os.lut[(size_t)x * os.w2 + y];
                for (int cc = 0; cc < 3; ++cc)
                    for (int d = 0; d < 3; ++d) {
                        const double2 v = tabm[o * 6 + sym_idx(cc, d)];
                        double* dst = out + ((int64_t)(3 * (b - b0) + cc) * 6 * p.n_i + 2 * (3 * i + d));
                        dst[0] = v.x;
                        dst[1] = v.y;
                    }
            }
        return FBC_OK;
    }
    if (c->opt.form != FBC_FORM_FP64) return fail(c, FBC_E_UNSUPPORTED, "FP64 forms only");
    // compact store: the row tiles covering the rows, their windows at mode m; blocks
    // outside a window are the product's zeros
    const int rows_tile = gemm_tile_rows(c->opt.form, c->ctmax);
    const int64_t cte = chunk_tile_elems(c->opt.form, rows_tile);
    const int trb = rows_tile / 16;
    const int rows = 3 * (b1 - b0);
    std::fill(out, out + (int64_t)rows * 6 * p.n_i, 0.0);
    HIPCHK(c, hipDeviceSynchronize());
    std::vector<double> reg;
    for (int tl = (3 * b0) / rows_tile; tl <= (3 * b1 - 1) / rows_tile; ++tl) {
        const int r = m * p.n_tiles + tl;
        const int ws = p.win_start[r], wl = p.win_len[r];
        if (wl == 0) continue;
        reg.resize((size_t)wl * cte);
        HIPCHK(c, hipMemcpy(reg.data(), (double*)c->store + p.a_off + p.reg_pre[r] * cte, reg.size() * 8,
                            hipMemcpyDeviceToHost));
        for (int row = std::max(3 * b0, tl * rows_tile); row < std::min(3 * b1, (tl + 1) * rows_tile); ++row) {
            const int rr = row - tl * rows_tile, blk = rr >> 4;
            for (int j = 0; j < wl; ++j) {
                const int ch = (ws + j) % p.n_chunks;
                for (int x = 0; x < 64; ++x) {
                    const int k = 64 * ch + x;
                    if (k >= 6 * p.n_i) break;
                    const int lane = ((x & 3) << 4) | (rr & 15);
                    const int64_t el = (int64_t)j * cte + ((((x >> 3) * trb + blk) * 64 + lane) << 1) + ((x >> 2) & 1);
                    out[(int64_t)(row - 3 * b0) * 6 * p.n_i + k] = reg[el];
                }
            }
        }
    }
    return FBC_OK;
}

extern "C" fbc_status fbc_timing(fbc_ctx* c, int enable) {
    if (!c) return fail(nullptr, FBC_E_ARG, "ctx is NULL");
    if (enable && c->ev.empty()) {
        c->ev.resize(2 * kMaxTimed);
        for (auto& e : c->ev) HIPCHK(c, hipEventCreate(&e));
    }
    c->timing = enable ? 1 : 0;
    return FBC_OK;
}

extern "C" fbc_status fbc_timing_read(fbc_ctx* c, double* ms, int* n) {
    if (!c || !ms || !n) return fail(c, FBC_E_ARG, "null argument");
    double tot = 0.0;
    for (int i = 0; i < c->n_timed; ++i) {
        HIPCHK(c, hipEventSynchronize(c->ev[2 * i + 1]));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev[2 * i], c->ev[2 * i + 1]));
        tot += t;
    }
    *ms = tot;
    *n = c->n_timed;
    c->n_timed = 0;
    return FBC_OK;
}

extern "C" void fbc_destroy(fbc_ctx* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    drop_relax_graph(c);
    free_all(c);
    delete c;
}
