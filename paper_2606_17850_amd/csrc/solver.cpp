// Host orchestration of the solve path: grid setup, Lanczos spectral bounds,
// the Chebyshev-preconditioned CG (Algorithm 1 + the Chebyshev algorithm of
// Section 4.3) and FP64 iterative refinement around an FP32 inner solve.
//
// Everything numeric on vectors runs in the kernels of kernels.hip.  The host
// enqueues launches on the handle's stream, reads back a few scalars or
// per-workgroup partials once per chunk of CG iterations and decides what to
// launch next.
#include "grid.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>

namespace cuth {

#define CUTH_HIP(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return Status::err(CUTH_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CUTH_TRY(expr)               \
    do {                             \
        Status s_ = (expr);          \
        if (s_.bad()) return s_;     \
    } while (0)

// Accumulate the durations of the recorded sweep events (stream already synced).
Status prof_flush(Grid &g) {
    for (size_t i = 0; i + 1 < g.pev_used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g.pev[i], g.pev[i + 1]) == hipSuccess) {
            g.prof_ms += ms;
            g.prof_count += 1;
        }
    }
    g.pev_used = 0;
    return Status::ok();
}

namespace {

template <typename P>
Status dev_alloc(P **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(P) * count);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return Status::err(CUTH_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return Status::ok();
}

template <typename P>
void dev_free(P *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

Status sync(Grid &g) {
    CUTH_HIP(hipStreamSynchronize(g.stream));
    return Status::ok();
}

template <typename T>
Status alloc_work(Work<T> &w, int64_t N) {
    if (w.ready()) return Status::ok();
    T **ps[] = {&w.x, &w.r, &w.rhat, &w.pA, &w.pB, &w.mu, &w.zA, &w.zB};
    for (T **p : ps) CUTH_TRY(dev_alloc(p, (size_t)N));
    return Status::ok();
}

template <typename T>
void free_work(Work<T> &w) {
    T **ps[] = {&w.x, &w.r, &w.rhat, &w.pA, &w.pB, &w.mu, &w.zA, &w.zB};
    for (T **p : ps) dev_free(*p);
}

// Coefficients of the Chebyshev sweeps for degree k on [lmin, lmax]: with
// theta = (lmax+lmin)/2, delta = (lmax-lmin)/2, sigma1 = theta/delta,
// rho_0 = 1/sigma1 and rho_{i+1} = 1/(2 sigma1 - rho_i) (Section 4.3), the
// two-term form z_{j+1} = z_j + rho_j [rho_{j-1}(z_j - z_{j-1}) + (2/delta)(r - A z_j)]
// (eq. final_expression_recurrence applied to A z = r from z_0 = 0) needs
// c1_j = rho_j rho_{j-1} and c2_j = 2 rho_j / delta; z_1 = r / theta.
struct ChebConsts {
    int k = 1;
    double inv_th = 0;
    std::vector<double> c1, c2;
};

ChebConsts make_cheb(double lmin, double lmax, int k) {
    ChebConsts cc;
    cc.k = k;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma1 = theta / delta;
    std::vector<double> rho(k + 1);
    rho[0] = 1.0 / sigma1;
    for (int i = 0; i < k; ++i) rho[i + 1] = 1.0 / (2.0 * sigma1 - rho[i]);
    cc.inv_th = 1.0 / theta;
    cc.c1.assign(k, 0.0);
    cc.c2.assign(k, 0.0);
    for (int j = 1; j < k; ++j) {
        cc.c1[j] = rho[j] * rho[j - 1];
        cc.c2[j] = 2.0 * rho[j] / delta;
    }
    return cc;
}

// Algorithmic bytes per unknown of each kernel (what the method must move).
template <typename T>
struct Bytes {
    double coef;   // per-cell lateral conductances read by one stencil sweep
    explicit Bytes(const Grid &g) : coef(g.per_cell ? 2.0 * sizeof(T) : 0.0) {}
    double cheb(int mode) const { return (mode == 1 ? 2 : mode == 2 ? 3 : 4) * sizeof(T) + coef; }
    double dir() const { return 4.0 * sizeof(T) + coef; }
    double update() const { return 6.0 * sizeof(T); }
    double check() const { return 3.0 * sizeof(T) + coef; }
    double scale() const { return 2.0 * sizeof(T); }
    double precond(int k) const {
        if (k == 1) return scale();
        double b = cheb(1);
        for (int j = 2; j < k; ++j) b += cheb(j == 2 ? 2 : 0);
        return b;
    }
};

// z = q(A) r by k-1 stencil sweeps (k >= 2) or one scaling (k == 1).  chk: the
// first kernel first tests convergence of CG iteration `it` from the update's
// partials (part_in, np_in).  The last kernel writes partials of r^T z to
// part_out (np_out of them).  Returns the buffer holding z.
template <typename T>
T *precond_seq(Grid &g, const OpView<T> &op, const ChebConsts &cc, const T *r, T *zA, T *zB,
               CgState<T> *st, bool chk, int it, const T *part_in, int np_in, T *part_out,
               int &np_out) {
    const Bytes<T> by(g);
    const int k = cc.k;
    if (k == 1) {
        launch_scale<T>(g.N, r, (T)cc.inv_th, zA, chk, it, st, part_in, np_in, part_out, g.stream);
        np_out = red_blocks(g.N);
        return zA;
    }
    launch_cheb<T>(op, 1, k == 2, chk, it, r, zB, r, (T)cc.c1[1], (T)cc.c2[1], (T)cc.inv_th, st,
                   part_in, np_in, part_out, g.stream);
    T *cur = zB, *prev = zA;
    for (int j = 2; j < k; ++j) {
        const int mode = (j == 2) ? 2 : 0;
        const bool timed = g.prof && j == 3 && g.pev_used + 2 <= g.pev.size();
        if (timed) (void)hipEventRecord(g.pev[g.pev_used], g.stream);
        launch_cheb<T>(op, mode, j == k - 1, false, it, cur, prev, r, (T)cc.c1[j], (T)cc.c2[j],
                       (T)cc.inv_th, st, part_in, np_in, part_out, g.stream);
        if (timed) {
            (void)hipEventRecord(g.pev[g.pev_used + 1], g.stream);
            g.pev_used += 2;
            g.prof_bytes = by.cheb(0) * (double)g.N;
        }
        std::swap(cur, prev);
    }
    np_out = stencil_blocks(op);
    return cur;
}

template <typename T>
CgState<T> *state_of(Grid &g);
template <>
CgState<float> *state_of<float>(Grid &g) { return g.st32; }
template <>
CgState<double> *state_of<double>(Grid &g) { return g.st64; }
template <typename T>
CgState<T> *hstate_of(Grid &g);
template <>
CgState<float> *hstate_of<float>(Grid &g) { return g.h_st32; }
template <>
CgState<double> *hstate_of<double>(Grid &g) { return g.h_st64; }

template <typename T>
Status write_state(Grid &g, double rr0, double tol2) {
    CgState<T> *h = hstate_of<T>(g);
    std::memset(h, 0, sizeof(CgState<T>));
    h->rr = (T)rr0;
    h->rr0 = (T)rr0;
    h->tol2 = (T)tol2;
    h->done = rr0 > 0.0 ? 0 : 1;
    CUTH_HIP(hipMemcpyAsync(state_of<T>(g), h, sizeof(CgState<T>), hipMemcpyHostToDevice, g.stream));
    return Status::ok();
}

// Read back the state and nv*np partials of slot s; host sums in a fixed order.
template <typename T>
Status read_state_and_partials(Grid &g, int s, int nv, int np, double *sums) {
    CUTH_HIP(hipMemcpyAsync(hstate_of<T>(g), state_of<T>(g), sizeof(CgState<T>),
                            hipMemcpyDeviceToHost, g.stream));
    CUTH_HIP(hipMemcpyAsync(g.h_part, g.slot<T>(s), sizeof(T) * (size_t)nv * np,
                            hipMemcpyDeviceToHost, g.stream));
    CUTH_TRY(sync(g));
    const T *p = reinterpret_cast<const T *>(g.h_part);
    for (int v = 0; v < nv; ++v) {
        double a = 0.0;
        for (int q = 0; q < np; ++q) a += (double)p[(size_t)v * np + q];
        sums[v] = a;
    }
    return Status::ok();
}

// Inner PCG on A_T x = rhat with x_0 = 0 (r = rhat on entry).  Runs chunks of
// `period` iterations; after each chunk a true-residual kernel gives the
// drift (||r_true - r_low|| >= 0.5 ||r_true||) and stagnation
// (||r_true^k|| > 0.9 ||r_true^{k-1}||) criteria of Section 4.4, evaluated
// here together with the device's convergence flag.
template <typename T>
InnerResult inner_pcg(Grid &g, const OpView<T> &op, Work<T> &w, const ChebConsts &cc, double rr0,
                      double tol2, int maxit, int period, Status &status) {
    InnerResult res;
    status = Status::ok();
    CgState<T> *st = state_of<T>(g);
    CgState<T> *hst = hstate_of<T>(g);
    const Bytes<T> by(g);
    const double n = (double)g.N;
    const int nbs = stencil_blocks(op);
    status = write_state<T>(g, rr0, tol2);
    if (status.bad()) return res;
    int np_z = 0, nchecks = 0;
    T *z = precond_seq<T>(g, op, cc, w.r, w.zA, w.zB, st, false, 0, nullptr, 0, g.slot<T>(S_CHEB),
                          np_z);
    T *pold = w.pA, *pnew = w.pB;
    int it = 0, reason = 0;
    double true_prev = -1.0, sums[2] = {0, 0};
    while (it < maxit) {
        const int nb = std::min(period, maxit - it);
        for (int q = 0; q < nb; ++q) {
            const int k = it + q;
            launch_cg_dir<T>(op, k, z, pold, pnew, w.mu, st, g.slot<T>(S_CHEB), np_z,
                             g.slot<T>(S_DIR), g.stream);
            launch_cg_update<T>(op, k, w.x, pnew, w.r, w.mu, st, g.slot<T>(S_DIR), nbs,
                                g.slot<T>(S_UPD), g.stream);
            z = precond_seq<T>(g, op, cc, w.r, w.zA, w.zB, st, true, k, g.slot<T>(S_UPD), nbs,
                               g.slot<T>(S_CHEB), np_z);
            std::swap(pold, pnew);
        }
        it += nb;
        launch_cg_check<T>(op, w.rhat, w.x, w.r, true, g.slot<T>(S_CHK), g.stream);
        ++nchecks;
        status = read_state_and_partials<T>(g, S_CHK, 2, nbs, sums);
        if (status.bad()) return res;
        if (g.prof) (void)prof_flush(g);
        const double tn = std::sqrt(sums[0]);
        if (hst->done) {
            reason = hst->done;
            break;
        }
        if (!std::isfinite(tn)) {
            reason = 4;
            break;
        }
        if (std::sqrt(sums[1]) >= 0.5 * tn) {
            reason = 2;
            break;
        }
        if (true_prev >= 0.0 && tn > 0.9 * true_prev) {
            reason = 3;
            break;
        }
        true_prev = tn;
    }
    if (reason == 0) reason = 5;
    res.iters = hst->iter;
    res.reason = reason;
    res.true_red = rr0 > 0 ? std::sqrt(sums[0] / rr0) : 0.0;
    // launches after the stopping point exit early and move no data
    const int iters = res.iters;
    const int precs_run = 1 + iters - (reason == 1 ? 1 : 0);
    res.bytes = precs_run * by.precond(cc.k) * n + iters * (by.dir() + by.update()) * n +
                nchecks * by.check() * n;
    res.stencils = (int64_t)precs_run * (cc.k - 1) + iters + nchecks;
    if (reason == 4) status = Status::err(CUTH_E_BREAKDOWN, "CG breakdown (p^T A p <= 0 or non-finite value)");
    return res;
}

struct OuterRes {
    double rr = 0, bb = 0, dinf = 0, thinf = 0, bad = 0;
};

template <typename TD, typename TI>
Status outer_residual(Grid &g, const OpView<double> &op, const double *th_in, double in_off,
                      const TD *delta, const double *P, const double *Tn, double *th_out,
                      double *r64, TI *r_in, TI *rhat, OuterRes &o) {
    launch_residual<TD, TI>(op, th_in, in_off, delta, P, Tn, g.t_amb, th_out, r64, r_in, rhat,
                            g.slot<double>(S_RES), g.stream);
    const int nb = stencil_blocks(op);
    CUTH_HIP(hipMemcpyAsync(g.h_part, g.slot<double>(S_RES), sizeof(double) * kResidualValues * nb,
                            hipMemcpyDeviceToHost, g.stream));
    CUTH_TRY(sync(g));
    const double *p = g.h_part;
    o = OuterRes();
    for (int q = 0; q < nb; ++q) {
        o.rr += p[q];
        o.bb += p[nb + q];
        o.dinf = std::max(o.dinf, p[2 * nb + q]);
        o.thinf = std::max(o.thinf, p[3 * nb + q]);
        o.bad += p[4 * nb + q];
    }
    return Status::ok();
}

int sturm_count(const std::vector<double> &a, const std::vector<double> &b, double x) {
    int cnt = 0;
    double d = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        const double off = i ? b[i - 1] * b[i - 1] / d : 0.0;
        d = a[i] - x - off;
        if (d == 0.0) d = -std::numeric_limits<double>::min();
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

double bisect_kth(const std::vector<double> &a, const std::vector<double> &b, int kth, double lo,
                  double hi) {
    // smallest x with sturm_count(x) >= kth, i.e. the kth smallest eigenvalue
    for (int it = 0; it < 300; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, mid) >= kth) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// CUTH_LOG=1: one line per refinement cycle on stderr.
bool log_on() {
    static const bool on = [] {
        const char *e = std::getenv("CUTH_LOG");
        return e && e[0] == '1';
    }();
    return on;
}

Shape shape_from_env(const char *name, Shape def, int nx, int maxvx) {
    Shape s = def;
    if (const char *e = std::getenv(name)) {
        int vx = 0, by = 0, zc = 0;
        if (std::sscanf(e, "%d,%d,%d", &vx, &by, &zc) == 3) {
            if ((vx == 1 || vx == 2 || vx == 4) && vx <= maxvx) s.vx = vx;
            if (by >= 1 && by <= kMaxBY) s.by = by;
            if (zc >= 1) s.zc = zc;
        }
    }
    while (s.vx > 1 && nx % s.vx != 0) s.vx /= 2;
    return s;
}

}  // namespace

// ---------------------------------------------------------------- tridiagonal
void tridiag_extremes(const std::vector<double> &a, const std::vector<double> &b, double &lo,
                      double &hi) {
    const size_t m = a.size();
    double glo = std::numeric_limits<double>::infinity(), ghi = -glo;
    for (size_t i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        glo = std::min(glo, a[i] - r);
        ghi = std::max(ghi, a[i] + r);
    }
    const double pad = 1e-12 * std::max(std::fabs(glo), std::fabs(ghi)) + 1e-300;
    glo -= pad;
    ghi += pad;
    lo = bisect_kth(a, b, 1, glo, ghi);
    hi = bisect_kth(a, b, (int)m, glo, ghi);
}

// ----------------------------------------------------------------- handle
Status grid_create(const cuth_grid_desc &d, hipStream_t s, Grid **out) {
    Grid *g = new Grid();
    *out = nullptr;
    auto fail = [&](Status st) {
        grid_destroy(g);
        return st;
    };
    if (hipGetDevice(&g->device) != hipSuccess) return fail(Status::err(CUTH_E_DEVICE, "hipGetDevice failed"));
    g->stream = s;
    g->nx = d.nx;
    g->ny = d.ny;
    g->nz = d.nz;
    g->N = (int64_t)d.nx * d.ny * d.nz;
    g->dx = d.dx;
    g->dy = d.dy;
    g->h_top = d.h_top;
    g->h_bot = d.h_bottom;
    g->t_amb = d.t_amb;
    g->dz.assign(d.dz, d.dz + d.nz);
    g->k_lat.assign(d.k_lat, d.k_lat + d.nz);
    g->k_vert.assign(d.k_vert, d.k_vert + d.nz);
    g->has_cap = d.heat_cap != nullptr;
    if (g->has_cap) g->cap.assign(d.heat_cap, d.heat_cap + d.nz);
    g->per_cell = d.k_lat_mult != nullptr;

    // launch shapes: one 16-byte load per lane where the row length allows, one
    // wavefront per workgroup, vertical marches of 8 layers (measured best on
    // gfx950 for the 512 x 512 x 16 stack: FP32 sweep 5.9 TB/s, FP64 6.8 TB/s);
    // CUTH_SHAPE32 / CUTH_SHAPE64 = "vx,by,zc" override them
    g->sh32 = shape_from_env("CUTH_SHAPE32", Shape{4, 1, 8}, g->nx, 4);
    g->sh64 = shape_from_env("CUTH_SHAPE64", Shape{2, 1, 8}, g->nx, 2);
    auto nblocks = [&](const Shape &sh) {
        return (size_t)tiles_x(g->nx, sh.vx) * tiles_y(g->ny, sh.by) * tiles_z(g->nz, sh.zc);
    };
    const size_t nb_max = std::max({nblocks(g->sh32), nblocks(g->sh64), (size_t)kRedBlocks});
    g->slot_doubles = 8 * nb_max;
    const size_t nb_adj = (size_t)((g->nx + kWave - 1) / kWave) * ((g->ny + 3) / 4);
    Status st;
    if ((st = dev_alloc(&g->part, g->slot_doubles * S_COUNT + (size_t)2 * g->nz * nb_adj)).bad())
        return fail(st);
    g->part_adj = g->part + g->slot_doubles * S_COUNT;
    if ((st = dev_alloc(&g->st32, 1)).bad()) return fail(st);
    if ((st = dev_alloc(&g->st64, 1)).bad()) return fail(st);
    if ((st = dev_alloc(&g->lz, 1024)).bad()) return fail(st);
    if ((st = dev_alloc(&g->adj_fac, (size_t)3 * g->nz)).bad()) return fail(st);
    if ((st = dev_alloc(&g->thA, (size_t)g->N)).bad()) return fail(st);
    if ((st = dev_alloc(&g->thB, (size_t)g->N)).bad()) return fail(st);
    if ((st = alloc_work(g->w32, g->N)).bad()) return fail(st);
    if (hipHostMalloc((void **)&g->h_st32, sizeof(CgState<float>), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->h_st64, sizeof(CgState<double>), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->h_part, g->slot_doubles * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->h_lz, 1024 * sizeof(float), hipHostMallocDefault) != hipSuccess)
        return fail(Status::err(CUTH_E_NOMEM, "hipHostMalloc failed"));
    if (hipMemset(g->st32, 0, sizeof(CgState<float>)) != hipSuccess ||
        hipMemset(g->st64, 0, sizeof(CgState<double>)) != hipSuccess)
        return fail(Status::err(CUTH_E_DEVICE, "hipMemset failed"));
    if (hipEventCreate(&g->ev0) != hipSuccess || hipEventCreate(&g->ev1) != hipSuccess ||
        hipEventCreate(&g->ev2) != hipSuccess)
        return fail(Status::err(CUTH_E_DEVICE, "hipEventCreate failed"));

    // adjoint factors: 1/k_lat[l], and dg/dk_vert[l] of the faces above / below layer l
    // (g = dx dy / (dz_a/(2 k_a) + dz_b/(2 k_b)) gives dg/dk_a = g^2 dz_a / (2 k_a^2 dx dy))
    {
        const int nz = g->nz;
        std::vector<double> fac((size_t)3 * nz, 0.0);
        const double dxdy = g->dx * g->dy;
        for (int l = 0; l < nz; ++l) {
            fac[l] = 1.0 / g->k_lat[l];
            const double kv = g->k_vert[l];
            if (l + 1 < nz) {
                const double gz = dxdy / (g->dz[l] / (2.0 * kv) + g->dz[l + 1] / (2.0 * g->k_vert[l + 1]));
                fac[nz + l] = gz * gz * g->dz[l] / (2.0 * kv * kv * dxdy);
            }
            if (l > 0) {
                const double gz = dxdy / (g->dz[l - 1] / (2.0 * g->k_vert[l - 1]) + g->dz[l] / (2.0 * kv));
                fac[2 * nz + l] = gz * gz * g->dz[l] / (2.0 * kv * kv * dxdy);
            }
        }
        if (hipMemcpy(g->adj_fac, fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return fail(Status::err(CUTH_E_DEVICE, "hipMemcpy failed"));
    }

    if (g->per_cell) {
        const int64_t N = g->N;
        if ((st = dev_alloc(&g->gx64, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->gy64, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->gx32, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->gy32, (size_t)N)).bad()) return fail(st);
        double *ddz = nullptr, *dkl = nullptr;
        unsigned long long *dmax = nullptr;
        unsigned int *dbad = nullptr;
        if ((st = dev_alloc(&ddz, (size_t)g->nz)).bad() || (st = dev_alloc(&dkl, (size_t)g->nz)).bad() ||
            (st = dev_alloc(&dmax, (size_t)g->nz)).bad() || (st = dev_alloc(&dbad, 1)).bad()) {
            dev_free(ddz); dev_free(dkl); dev_free(dmax); dev_free(dbad);
            return fail(st);
        }
        std::vector<unsigned long long> hmax(g->nz, 0ull);
        unsigned int hbad = 0;
        bool ok = hipMemcpy(ddz, g->dz.data(), g->nz * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(dkl, g->k_lat.data(), g->nz * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemset(dmax, 0, g->nz * sizeof(unsigned long long)) == hipSuccess &&
                  hipMemset(dbad, 0, sizeof(unsigned int)) == hipSuccess;
        if (ok) {
            launch_build_lateral(g->nx, g->ny, g->nz, g->dx, g->dy, ddz, dkl, d.k_lat_mult, g->gx64,
                                 g->gy64, g->gx32, g->gy32, dmax, dbad, g->stream);
            ok = hipStreamSynchronize(g->stream) == hipSuccess &&
                 hipMemcpy(hmax.data(), dmax, g->nz * sizeof(unsigned long long), hipMemcpyDeviceToHost) == hipSuccess &&
                 hipMemcpy(&hbad, dbad, sizeof(unsigned int), hipMemcpyDeviceToHost) == hipSuccess;
        }
        dev_free(ddz); dev_free(dkl); dev_free(dmax); dev_free(dbad);
        if (!ok) return fail(Status::err(CUTH_E_DEVICE, "coefficient build failed"));
        if (hbad) return fail(Status::err(CUTH_E_INVALID, "k_lat_mult has entries <= 0 or non-finite"));
        g->lat_rowmax.resize(g->nz);
        for (int l = 0; l < g->nz; ++l) {
            double v;
            std::memcpy(&v, &hmax[l], sizeof(double));
            g->lat_rowmax[l] = v;
        }
    }
    *out = g;
    return Status::ok();
}

void grid_destroy(Grid *g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    for (Setup &su : g->setups) {
        dev_free(su.lc64);
        dev_free(su.lc32);
    }
    dev_free(g->gx64);
    dev_free(g->gy64);
    dev_free(g->gx32);
    dev_free(g->gy32);
    free_work(g->w32);
    free_work(g->w64);
    dev_free(g->thA);
    dev_free(g->thB);
    dev_free(g->part);
    dev_free(g->st32);
    dev_free(g->st64);
    dev_free(g->lz);
    dev_free(g->adj_fac);
    if (g->h_st32) (void)hipHostFree(g->h_st32);
    if (g->h_st64) (void)hipHostFree(g->h_st64);
    if (g->h_part) (void)hipHostFree(g->h_part);
    if (g->h_lz) (void)hipHostFree(g->h_lz);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    if (g->ev2) (void)hipEventDestroy(g->ev2);
    for (hipEvent_t e : g->pev) (void)hipEventDestroy(e);
    delete g;
}

OpView<double> view64(const Grid &g, const Setup &su) {
    return OpView<double>{g.nx, g.ny, g.nz, g.per_cell ? g.gx64 : nullptr,
                          g.per_cell ? g.gy64 : nullptr, su.lc64, g.sh64.vx, g.sh64.by,
                          g.sh64.zc};
}

OpView<float> view32(const Grid &g, const Setup &su) {
    return OpView<float>{g.nx, g.ny, g.nz, g.per_cell ? g.gx32 : nullptr,
                         g.per_cell ? g.gy32 : nullptr, su.lc32, g.sh32.vx, g.sh32.by,
                         g.sh32.zc};
}

Setup *get_setup(Grid &g, double dt, Status &status) {
    status = Status::ok();
    for (Setup &su : g.setups)
        if (su.dt == dt) return &su;
    Setup su;
    su.dt = dt;
    const int nz = g.nz;
    const double dx = g.dx, dy = g.dy, dxdy = dx * dy;
    su.hlc.resize(nz);
    double gersh = 0.0;
    for (int l = 0; l < nz; ++l) {
        LayerCoef<double> &L = su.hlc[l];
        const double k = g.k_lat[l], d = g.dz[l];
        // series half-cell conductance of a lateral face inside a uniform layer
        L.gx = (dy * d) / (dx / (2.0 * k) + dx / (2.0 * k));
        L.gy = (dx * d) / (dy / (2.0 * k) + dy / (2.0 * k));
        L.gzu = (l + 1 < nz)
                    ? dxdy / (d / (2.0 * g.k_vert[l]) + g.dz[l + 1] / (2.0 * g.k_vert[l + 1]))
                    : 0.0;
        L.gzd = (l > 0) ? su.hlc[l - 1].gzu : 0.0;
        L.cap = (dt > 0.0) ? g.cap[l] * dxdy * d / dt : 0.0;
        L.sink = L.cap + (l == nz - 1 ? g.h_top * dxdy : 0.0) + (l == 0 ? g.h_bot * dxdy : 0.0);
        const double lat = g.per_cell ? g.lat_rowmax[l]
                                      : std::min(2, g.nx - 1) * L.gx + std::min(2, g.ny - 1) * L.gy;
        gersh = std::max(gersh, 2.0 * (lat + L.gzu + L.gzd) + L.sink);
    }
    su.gersh = gersh;
    std::vector<LayerCoef<float>> h32(nz);
    for (int l = 0; l < nz; ++l) {
        const LayerCoef<double> &L = su.hlc[l];
        h32[l] = LayerCoef<float>{(float)L.gx, (float)L.gy, (float)L.gzd, (float)L.gzu,
                                  (float)L.sink, (float)L.cap};
    }
    status = dev_alloc(&su.lc64, (size_t)nz);
    if (!status.bad()) status = dev_alloc(&su.lc32, (size_t)nz);
    if (status.bad()) {
        dev_free(su.lc64);
        dev_free(su.lc32);
        return nullptr;
    }
    if (hipMemcpy(su.lc64, su.hlc.data(), nz * sizeof(LayerCoef<double>), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(su.lc32, h32.data(), nz * sizeof(LayerCoef<float>), hipMemcpyHostToDevice) != hipSuccess) {
        dev_free(su.lc64);
        dev_free(su.lc32);
        status = Status::err(CUTH_E_DEVICE, "hipMemcpy of layer coefficients failed");
        return nullptr;
    }
    g.setups.push_back(su);
    return &g.setups.back();
}

// FP32 Lanczos on the FP32 operator (Section 4.4, component-wise precision of
// Lanczos): alpha_j = v_j^T A v_j, w = A v_j - alpha_j v_j - beta_{j-1} v_{j-1},
// beta_j = ||w||, v_{j+1} = w / beta_j.  Scalars stay on the device until the
// end; one readback returns the tridiagonal.
Status run_lanczos(Grid &g, Setup &su, int steps, const float *v0, std::vector<double> &alpha,
                   std::vector<double> &beta) {
    steps = (int)std::max<int64_t>(1, std::min<int64_t>(steps, g.N));
    steps = std::min(steps, 256);
    const OpView<float> op = view32(g, su);
    const int nbs = stencil_blocks(op), nb1 = red_blocks(g.N);
    float *pa = g.slot<float>(S_LZA), *pb = g.slot<float>(S_LZB);
    float *bufs[3] = {g.w32.pA, g.w32.pB, g.w32.mu};
    if (v0) {
        launch_norm2(g.N, v0, pa, g.stream);
        launch_scale_rsqrt(g.N, v0, pa, nb1, bufs[1], g.stream);
    } else {
        launch_fill_random(g.N, 0x2606178500ull, bufs[0], g.stream);
        launch_norm2(g.N, bufs[0], pa, g.stream);
        launch_scale_rsqrt(g.N, bufs[0], pa, nb1, bufs[1], g.stream);
    }
    int ip = 0, iv = 1, iw = 2;
    for (int j = 0; j < steps; ++j) {
        launch_lanczos_av(op, j, bufs[iv], j > 0 ? bufs[ip] : nullptr, g.lz, bufs[iw], pa, g.stream);
        launch_lanczos_orth(g.N, j, bufs[iw], bufs[iv], g.lz, pa, nbs, pb, g.stream);
        if (j == steps - 1) break;
        launch_lanczos_div(g.N, j, bufs[iw], g.lz, pb, nb1, g.stream);
        const int old = ip;
        ip = iv;
        iv = iw;
        iw = old;
    }
    CUTH_HIP(hipMemcpyAsync(g.h_lz, g.lz, 512 * sizeof(float), hipMemcpyDeviceToHost, g.stream));
    CUTH_TRY(sync(g));
    alpha.clear();
    beta.clear();
    double amax = 0.0;
    for (int j = 0; j < steps; ++j) amax = std::max(amax, std::fabs((double)g.h_lz[j]));
    for (int j = 0; j < steps; ++j) {
        const double a = g.h_lz[j];
        if (!std::isfinite(a)) break;
        alpha.push_back(a);
        if (j == steps - 1) break;
        const double b = g.h_lz[256 + j];
        // invariant subspace found (or round-off level): stop the tridiagonal here
        if (!std::isfinite(b) || b <= 1e-6 * amax) break;
        beta.push_back(b);
    }
    if (alpha.empty()) return Status::err(CUTH_E_BREAKDOWN, "Lanczos produced no finite values");
    beta.resize(alpha.size() - 1);
    return Status::ok();
}

Status ensure_bounds(Grid &g, Setup &su, int steps) {
    if (su.have_bounds && su.bounds_steps == steps) return Status::ok();
    std::vector<double> a, b;
    CUTH_TRY(run_lanczos(g, su, steps, nullptr, a, b));
    double lo, hi;
    tridiag_extremes(a, b, lo, hi);
    su.ritz_min = lo;
    su.ritz_max = hi;
    // lambda_max must bound the spectrum from above (else the polynomial
    // preconditioner loses definiteness); lambda_min is the smallest Ritz value
    su.lmax = std::min(su.gersh, 1.05 * hi);
    su.lmin = lo;
    if (!(su.lmin > 0.0) || !(su.lmax > su.lmin * (1.0 + 1e-6))) su.lmin = 0.5 * su.lmax;
    su.have_bounds = true;
    su.bounds_steps = steps;
    return Status::ok();
}

// ------------------------------------------------------------------- solve
Status solve_system(Grid &g, double dt, const double *P, const double *Tn, const double *init,
                    double init_off, double *out, double out_off, const cuth_options &o,
                    cuth_stats *stats, bool transient_defaults) {
    Status st;
    CUTH_HIP(hipEventRecord(g.ev0, g.stream));
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    CUTH_TRY(ensure_bounds(g, *su, o.lanczos_steps));
    CUTH_HIP(hipEventRecord(g.ev1, g.stream));
    const ChebConsts cc = make_cheb(su->lmin, su->lmax, o.cheb_degree);
    // tol == 0 selects the default of the precision: mixed, relative rise error
    // 1e-8; FP64, relative residual 1e-10 (steady) or 1e-12 (transient, where
    // ||b|| is dominated by the C/dt T_n term and the residual bound is looser)
    const double tol = o.tol > 0.0 ? o.tol
                                   : (o.precision == CUTH_MIXED ? 1e-8 : (dt > 0.0 ? 1e-12 : 1e-10));
    const int period = o.check_period > 0 ? o.check_period : (transient_defaults ? 5 : 20);
    const OpView<double> op64 = view64(g, *su);
    const double n = (double)g.N;
    const double coef64 = g.per_cell ? 16.0 : 0.0;
    int cycles = 0, cg_iters = 0, reason = 0;
    int64_t stencils = 0;
    double bytes = 0.0, relres = 0.0, err_est = 0.0;
    Status result = Status::ok();
    double *final_theta = nullptr;

    auto resid_bytes = [&](bool th_in, int delta_sz, int inner_sz) {
        return ((th_in ? 8.0 : 0.0) + delta_sz + 8.0 + (Tn ? 8.0 : 0.0) + 8.0 + 2.0 * inner_sz +
                coef64) * n;
    };

    if (o.precision == CUTH_MIXED) {
        const OpView<float> op32 = view32(g, *su);
        const double *th_in = init;
        double in_off = init_off;
        const float *delta = nullptr;
        double *th_out = g.thA;
        double last_red = 1.0, d_prev = 1.0, est = 1.0;
        for (int cyc = 0;; ++cyc) {
            OuterRes os;
            CUTH_TRY((outer_residual<float, float>(g, op64, th_in, in_off, delta, P, Tn, th_out,
                                                   nullptr, g.w32.r, g.w32.rhat, os)));
            bytes += resid_bytes(th_in != nullptr, delta ? 4 : 0, 4);
            ++stencils;
            final_theta = th_out;
            relres = os.bb > 0 ? std::sqrt(os.rr / os.bb) : std::sqrt(os.rr);
            if (os.bad > 0) {
                result = Status::err(CUTH_E_BREAKDOWN, "non-finite residual");
                break;
            }
            if (cyc >= 1) {
                const double d = os.thinf > 0 ? os.dinf / os.thinf : (os.dinf > 0 ? INFINITY : 0.0);
                const double q = d / d_prev;
                est = q * d;
                err_est = d;
                d_prev = d;
                // d is about the error before the last correction; that
                // correction's inner solve cut the residual by last_red, which
                // leaves an error of about last_red * d, but never less than the
                // FP32 rounding floor of the inner solve (about 16 ulps, 1e-6:
                // an FP32 residual can be exactly zero while the correction is
                // only FP32-accurate).  Stop when this is a tenth of tol, or
                // when the correction itself is below tol and cut the residual
                // at least tenfold.
                const double red_eff = std::max(last_red, 1e-6);
                if (red_eff * d <= 0.1 * tol || (d <= tol && last_red <= 0.1)) break;
            }
            if (os.rr == 0.0) break;
            if (cyc >= o.max_outer) {
                result = Status::err(CUTH_E_NOT_CONVERGED, "refinement cycle limit reached");
                break;
            }
            const double tau = cyc == 0 ? 1e-5 : std::min(0.1, std::max(1e-5, 0.1 * tol / est));
            const double rr0 = (double)(float)os.rr;
            Status is;
            InnerResult ir = inner_pcg<float>(g, op32, g.w32, cc, rr0, tau * tau * rr0,
                                              o.max_inner, period, is);
            cg_iters += ir.iters;
            stencils += ir.stencils;
            bytes += ir.bytes;
            reason = ir.reason;
            ++cycles;
            if (is.code == CUTH_E_DEVICE) return is;
            if (ir.iters == 0) {
                result = is.bad() ? is : Status::err(CUTH_E_BREAKDOWN, "inner solve made no progress");
                break;
            }
            if (log_on())
                std::fprintf(stderr,
                             "cuth: cycle %d relres %.3e tau %.1e inner %d its (stop %d) "
                             "true reduction %.3e est %.3e\n",
                             cyc, relres, tau, ir.iters, ir.reason, ir.true_red, est);
            last_red = ir.true_red;
            delta = g.w32.x;
            th_in = th_out;
            in_off = 0.0;
            th_out = (th_out == g.thA) ? g.thB : g.thA;
            if (is.bad()) result = is;   // breakdown: keep the partial correction
        }
    } else {
        CUTH_TRY(alloc_work(g.w64, g.N));
        const double *th_in = init;
        double in_off = init_off;
        const double *delta = nullptr;
        double *th_out = g.thA;
        double prev_relres = INFINITY;
        for (int cyc = 0;; ++cyc) {
            OuterRes os;
            CUTH_TRY((outer_residual<double, double>(g, op64, th_in, in_off, delta, P, Tn, th_out,
                                                     nullptr, g.w64.r, g.w64.rhat, os)));
            bytes += resid_bytes(th_in != nullptr, delta ? 8 : 0, 8);
            ++stencils;
            final_theta = th_out;
            relres = os.bb > 0 ? std::sqrt(os.rr / os.bb) : std::sqrt(os.rr);
            if (cyc >= 1 && os.thinf > 0) err_est = os.dinf / os.thinf;
            if (os.bad > 0) {
                result = Status::err(CUTH_E_BREAKDOWN, "non-finite residual");
                break;
            }
            if (relres <= tol || os.rr == 0.0) break;
            if (cyc >= o.max_outer) {
                result = Status::err(CUTH_E_NOT_CONVERGED, "restart limit reached");
                break;
            }
            // a restart that did not halve the true residual has hit the
            // attainable accuracy of FP64 for this system: report, do not loop
            if (cyc >= 1 && relres > 0.5 * prev_relres) {
                result = Status::err(CUTH_E_NOT_CONVERGED,
                                     "true residual stagnated above tol (attainable accuracy)");
                break;
            }
            prev_relres = relres;
            // hot restart: r and p recomputed from their definitions, x kept
            Status is;
            InnerResult ir = inner_pcg<double>(g, op64, g.w64, cc, os.rr, tol * tol * os.bb,
                                               o.max_inner, period, is);
            cg_iters += ir.iters;
            stencils += ir.stencils;
            bytes += ir.bytes;
            reason = ir.reason;
            ++cycles;
            if (is.code == CUTH_E_DEVICE) return is;
            if (ir.iters == 0) {
                result = is.bad() ? is : Status::err(CUTH_E_BREAKDOWN, "inner solve made no progress");
                break;
            }
            delta = g.w64.x;
            th_in = th_out;
            in_off = 0.0;
            th_out = (th_out == g.thA) ? g.thB : g.thA;
            if (is.bad()) result = is;
        }
    }
    if (final_theta) {
        launch_add_scalar(g.N, final_theta, out_off, out, g.stream);
        bytes += 16.0 * n;
    }
    CUTH_HIP(hipEventRecord(g.ev2, g.stream));
    CUTH_TRY(sync(g));
    if (stats) {
        float ms_setup = 0, ms_solve = 0;
        (void)hipEventElapsedTime(&ms_setup, g.ev0, g.ev1);
        (void)hipEventElapsedTime(&ms_solve, g.ev1, g.ev2);
        stats->outer_cycles = cycles;
        stats->cg_iters = cg_iters;
        stats->stencil_applies = stencils;
        stats->stop_reason = reason;
        stats->rel_residual = relres;
        stats->err_est = err_est;
        stats->setup_ms = ms_setup;
        stats->solve_ms = ms_solve;
        stats->alg_bytes = bytes;
        stats->lambda_min = su->lmin;
        stats->lambda_max = su->lmax;
    }
    return result;
}

Status apply_op(Grid &g, double dt, int precision, const void *x, void *y) {
    Status st;
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    if (precision == CUTH_MIXED) launch_apply<float>(view32(g, *su), (const float *)x, (float *)y, g.stream);
    else launch_apply<double>(view64(g, *su), (const double *)x, (double *)y, g.stream);
    CUTH_HIP(hipGetLastError());
    return sync(g);
}

Status residual(Grid &g, double dt, const double *b, const double *T, double *r) {
    Status st;
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    launch_residual<double, double>(view64(g, *su), T, g.t_amb, (const double *)nullptr, b, nullptr,
                                    0.0, nullptr, r, nullptr, nullptr, g.slot<double>(S_RES),
                                    g.stream);
    CUTH_HIP(hipGetLastError());
    return sync(g);
}

template <typename T>
static Status precond_typed(Grid &g, const OpView<T> &op, Work<T> &w, const ChebConsts &cc,
                            const T *r, T *z) {
    // the result lands in zA for k == 1 or odd k, in zB for even k >= 2
    const bool in_b = cc.k >= 2 && ((cc.k - 1) % 2 == 1);
    T *zA = in_b ? w.zA : z;
    T *zB = in_b ? z : w.zB;
    CUTH_TRY(write_state<T>(g, 1.0, 0.0));
    int np = 0;
    T *res = precond_seq<T>(g, op, cc, r, zA, zB, state_of<T>(g), false, 0, nullptr, 0,
                            g.slot<T>(S_CHEB), np);
    if (res != z) return Status::err(CUTH_E_DEVICE, "internal: preconditioner buffer mismatch");
    CUTH_HIP(hipGetLastError());
    return sync(g);
}

Status precond_apply(Grid &g, double dt, int precision, double lmin, double lmax, int degree,
                     const void *r, void *z) {
    Status st;
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    const ChebConsts cc = make_cheb(lmin, lmax, degree);
    if (precision == CUTH_MIXED)
        return precond_typed<float>(g, view32(g, *su), g.w32, cc, (const float *)r, (float *)z);
    CUTH_TRY(alloc_work(g.w64, g.N));
    return precond_typed<double>(g, view64(g, *su), g.w64, cc, (const double *)r, (double *)z);
}

Status adjoint(Grid &g, const double *T, const double *dL_dT, double *dL_dP, double *dL_dk,
               const cuth_options &o, cuth_stats *stats) {
    Status st = solve_system(g, 0.0, dL_dT, nullptr, nullptr, 0.0, dL_dP, 0.0, o, stats, false);
    if (st.code == CUTH_E_DEVICE || st.code == CUTH_E_INVALID || st.code == CUTH_E_NOMEM) return st;
    Status s2;
    Setup *su = get_setup(g, 0.0, s2);
    if (!su) return s2;
    launch_adjoint(view64(g, *su), dL_dP, T, g.t_amb, g.adj_fac, g.part_adj, dL_dk, g.stream);
    CUTH_HIP(hipGetLastError());
    CUTH_TRY(sync(g));
    return st;
}

}  // namespace cuth
