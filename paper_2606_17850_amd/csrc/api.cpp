// C ABI of the library (declared in include/cuth.h): argument validation on
// the host, then dispatch to the solver in solver.cpp.  Nothing unwinds across
// the boundary; every failure becomes a status code plus a thread-local message.
#include "grid.hpp"

#include <cmath>
#include <cstdio>
#include <exception>
#include <new>
#include <string>
#include <vector>

struct cuth_grid_s {
    cuth::Grid *g;
};

namespace {

thread_local std::string g_last_error;

cuth_status fail(cuth_status c, const std::string &m) {
    g_last_error = m;
    return c;
}

cuth_status report(const cuth::Status &s) {
    if (s.bad()) g_last_error = s.msg;
    return s.code;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

cuth_status check_desc(const cuth_grid_desc *d) {
    if (!d) return fail(CUTH_E_INVALID, "descriptor is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(CUTH_E_INVALID, "nx, ny, nz must be >= 1");
    if (d->nz > cuth::kMaxLayers) return fail(CUTH_E_INVALID, "nz exceeds 64");
    if ((int64_t)d->nx * d->ny * d->nz > ((int64_t)1 << 36))
        return fail(CUTH_E_INVALID, "grid too large (more than 2^36 cells)");
    if (!finite_pos(d->dx) || !finite_pos(d->dy))
        return fail(CUTH_E_INVALID, "dx and dy must be finite and > 0");
    if (!d->dz || !d->k_lat || !d->k_vert)
        return fail(CUTH_E_INVALID, "dz, k_lat and k_vert are required");
    for (int l = 0; l < d->nz; ++l) {
        if (!finite_pos(d->dz[l])) return fail(CUTH_E_INVALID, "dz[l] must be finite and > 0");
        if (!finite_pos(d->k_lat[l]) || !finite_pos(d->k_vert[l]))
            return fail(CUTH_E_INVALID, "k_lat[l] and k_vert[l] must be finite and > 0");
        if (d->heat_cap && !finite_pos(d->heat_cap[l]))
            return fail(CUTH_E_INVALID, "heat_cap[l] must be finite and > 0");
    }
    if (!std::isfinite(d->h_top) || !std::isfinite(d->h_bottom) || d->h_top < 0 || d->h_bottom < 0)
        return fail(CUTH_E_INVALID, "h_top and h_bottom must be finite and >= 0");
    if (!std::isfinite(d->t_amb)) return fail(CUTH_E_INVALID, "t_amb must be finite");
    return CUTH_OK;
}

cuth_status check_opts(const cuth_options &o) {
    if (o.precision < CUTH_FP64 || o.precision > CUTH_FP32)
        return fail(CUTH_E_INVALID, "precision must be a cuth_precision value");
    if (o.preconditioner < CUTH_PC_CHEBYSHEV || o.preconditioner > CUTH_PC_CHEBYSHEV_JACOBI)
        return fail(CUTH_E_INVALID, "preconditioner must be a cuth_preconditioner value");
    if (o.storage == CUTH_STORAGE_CSR && o.preconditioner == CUTH_PC_CHEBYSHEV_JACOBI)
        return fail(CUTH_E_INVALID, "the Jacobi-scaled Chebyshev preconditioner needs stencil storage");
    if (o.storage != CUTH_STORAGE_STENCIL && o.storage != CUTH_STORAGE_CSR)
        return fail(CUTH_E_INVALID, "storage must be a cuth_storage value");
    if (o.storage == CUTH_STORAGE_CSR && o.precision != CUTH_FP64)
        return fail(CUTH_E_INVALID, "CSR storage needs precision CUTH_FP64");
    if (!(o.tol == 0.0 || (finite_pos(o.tol) && o.tol < 1.0)))
        return fail(CUTH_E_INVALID, "tol must be 0 (default) or in (0, 1)");
    if (o.cheb_degree != CUTH_DEGREE_AUTO && (o.cheb_degree < 1 || o.cheb_degree > 256))
        return fail(CUTH_E_INVALID, "cheb_degree must be in 1..256 or CUTH_DEGREE_AUTO");
    if (o.lanczos_steps < 2 || o.lanczos_steps > 256)
        return fail(CUTH_E_INVALID, "lanczos_steps must be in 2..256");
    if (o.max_inner < 1 || o.max_outer < 1)
        return fail(CUTH_E_INVALID, "max_inner and max_outer must be >= 1");
    if (o.check_period < 0) return fail(CUTH_E_INVALID, "check_period must be >= 0");
    return CUTH_OK;
}

cuth_options resolve(const cuth_options *o, bool &ok) {
    cuth_options r;
    cuth_default_options(&r);
    if (o) {
        r = *o;
        if (r.cheb_degree == 0) r.cheb_degree = 30;
        if (r.lanczos_steps == 0) r.lanczos_steps = 30;
        if (r.max_inner == 0) r.max_inner = 2000;
        if (r.max_outer == 0) r.max_outer = 12;
    }
    ok = check_opts(r) == CUTH_OK;
    return r;
}

cuth_status check_handle(cuth_grid g) {
    if (!g || !g->g) return fail(CUTH_E_INVALID, "grid handle is NULL");
    if (!g->g->valid)
        return fail(CUTH_E_INVALID, "grid conductivities are invalid: the last "
                                    "cuth_grid_set_conductivity was rejected on the device");
    return CUTH_OK;
}

bool steady_ok(const cuth::Grid &g) { return g.h_top + g.h_bot > 0.0; }

template <typename F>
cuth_status guarded(F &&f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return fail(CUTH_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(CUTH_E_DEVICE, e.what());
    } catch (...) {
        return fail(CUTH_E_DEVICE, "unknown exception");
    }
}

}  // namespace

extern "C" {

void cuth_default_options(cuth_options *o) {
    if (!o) return;
    o->precision = CUTH_MIXED;
    o->tol = 0.0;
    o->cheb_degree = 30;
    o->lanczos_steps = 30;
    o->max_inner = 2000;
    o->max_outer = 12;
    o->use_initial_guess = 0;
    o->check_period = 0;
    o->preconditioner = CUTH_PC_CHEBYSHEV;
    o->storage = CUTH_STORAGE_STENCIL;
}

const char *cuth_last_error(void) { return g_last_error.c_str(); }

cuth_status cuth_grid_create(const cuth_grid_desc *desc, void *hip_stream, cuth_grid *out) {
    return guarded([&]() -> cuth_status {
        if (!out) return fail(CUTH_E_INVALID, "out is NULL");
        *out = nullptr;
        cuth_status c = check_desc(desc);
        if (c != CUTH_OK) return c;
        cuth::Grid *g = nullptr;
        cuth::Status s = cuth::grid_create(*desc, (hipStream_t)hip_stream, &g);
        if (s.bad()) return report(s);
        *out = new cuth_grid_s{g};
        return CUTH_OK;
    });
}

void cuth_grid_destroy(cuth_grid g) {
    if (!g) return;
    cuth::grid_destroy(g->g);
    delete g;
}

cuth_status cuth_grid_set_conductivity(cuth_grid h, const double *k_lat, const double *k_vert,
                                       const double *k_lat_mult) {
    return guarded([&]() -> cuth_status {
        if (!h || !h->g) return fail(CUTH_E_INVALID, "grid handle is NULL");
        cuth::Grid &g = *h->g;
        if (!k_lat || !k_vert) return fail(CUTH_E_INVALID, "k_lat and k_vert are required");
        for (int l = 0; l < g.nz; ++l)
            if (!finite_pos(k_lat[l]) || !finite_pos(k_vert[l]))
                return fail(CUTH_E_INVALID, "k_lat[l] and k_vert[l] must be finite and > 0");
        if (g.per_cell && !k_lat_mult)
            return fail(CUTH_E_INVALID, "the grid was created with k_lat_mult: it is required");
        if (!g.per_cell && k_lat_mult)
            return fail(CUTH_E_INVALID, "the grid was created without k_lat_mult: pass NULL");
        return report(cuth::grid_set_conductivity(g, k_lat, k_vert, k_lat_mult));
    });
}

cuth_status cuth_solve(cuth_grid h, const double *P, double *T, const cuth_options *opt,
                       cuth_stats *stats) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        bool ok;
        cuth_options o = resolve(opt, ok);
        if (!ok) return check_opts(o);
        if (!P || !T) return fail(CUTH_E_INVALID, "P and T are required");
        cuth::Grid &g = *h->g;
        if (!steady_ok(g))
            return fail(CUTH_E_INVALID, "steady solve needs a convective face (h_top + h_bottom > 0)");
        return report(cuth::solve_system(g, 0.0, P, nullptr, o.use_initial_guess ? T : nullptr,
                                         g.t_amb, T, g.t_amb, o, stats, false));
    });
}

cuth_status cuth_transient_step(cuth_grid h, double dt, const double *P_next, const double *T_n,
                                double *T_next, const cuth_options *opt, cuth_stats *stats) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        bool ok;
        cuth_options o = resolve(opt, ok);
        if (!ok) return check_opts(o);
        cuth::Grid &g = *h->g;
        if (!finite_pos(dt)) return fail(CUTH_E_INVALID, "dt must be finite and > 0");
        if (!g.has_cap) return fail(CUTH_E_INVALID, "transient step needs heat_cap in the descriptor");
        if (!P_next || !T_n || !T_next) return fail(CUTH_E_INVALID, "P_next, T_n and T_next are required");
        return report(cuth::solve_system(g, dt, P_next, T_n, T_n, g.t_amb, T_next, g.t_amb, o,
                                         stats, true));
    });
}

cuth_status cuth_solve_batch(int32_t nsys, const cuth_grid *grids, int32_t nrhs,
                             const double *const *P, double *const *T, const cuth_options *opt,
                             cuth_stats *stats) {
    return guarded([&]() -> cuth_status {
        if (nsys < 0 || nrhs < 1) return fail(CUTH_E_INVALID, "nsys >= 0 and nrhs >= 1 required");
        if (nsys == 0) return CUTH_OK;
        if (!grids || !P || !T) return fail(CUTH_E_INVALID, "grids, P and T are required");
        bool ok;
        cuth_options o = resolve(opt, ok);
        if (!ok) return check_opts(o);
        if (o.storage != CUTH_STORAGE_STENCIL)
            return fail(CUTH_E_INVALID, "batched solves use the stencil storage only");
        for (int s = 0; s < nsys; ++s) {
            if (check_handle(grids[s]) != CUTH_OK) return CUTH_E_INVALID;
            if (!P[s] || !T[s]) return fail(CUTH_E_INVALID, "P[s] and T[s] are required");
            if (!steady_ok(*grids[s]->g))
                return fail(CUTH_E_INVALID, "steady solve needs a convective face");
        }
        std::vector<cuth::Grid *> gs(nsys);
        for (int s = 0; s < nsys; ++s) {
            gs[s] = grids[s]->g;
            if (gs[s]->device != gs[0]->device)
                return fail(CUTH_E_INVALID, "all grids of a batch must be on one device");
        }
        return report(cuth::solve_batch(nsys, gs.data(), nrhs, P, T, o, stats));
    });
}

cuth_status cuth_adjoint(cuth_grid h, const double *T, const double *dL_dT, double *dL_dP,
                         double *dL_dk, const cuth_options *opt, cuth_stats *stats) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        bool ok;
        cuth_options o = resolve(opt, ok);
        if (!ok) return check_opts(o);
        if (!T || !dL_dT || !dL_dP || !dL_dk) return fail(CUTH_E_INVALID, "all vectors are required");
        cuth::Grid &g = *h->g;
        if (!steady_ok(g)) return fail(CUTH_E_INVALID, "adjoint of a steady solve needs a convective face");
        return report(cuth::adjoint(g, T, dL_dT, dL_dP, dL_dk, o, stats));
    });
}

cuth_status cuth_apply(cuth_grid h, double dt, int32_t precision, const void *x, void *y) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        cuth::Grid &g = *h->g;
        if (!x || !y) return fail(CUTH_E_INVALID, "x and y are required");
        if (precision != CUTH_FP64 && precision != CUTH_MIXED && precision != CUTH_MIXED16)
            return fail(CUTH_E_INVALID, "bad precision");
        if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(CUTH_E_INVALID, "dt must be >= 0");
        if (dt > 0.0 && !g.has_cap) return fail(CUTH_E_INVALID, "dt > 0 needs heat_cap");
        return report(cuth::apply_op(g, dt, precision, x, y));
    });
}

cuth_status cuth_residual(cuth_grid h, double dt, const double *b, const double *T, double *r) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        cuth::Grid &g = *h->g;
        if (!b || !T || !r) return fail(CUTH_E_INVALID, "b, T and r are required");
        if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(CUTH_E_INVALID, "dt must be >= 0");
        if (dt > 0.0 && !g.has_cap) return fail(CUTH_E_INVALID, "dt > 0 needs heat_cap");
        return report(cuth::residual(g, dt, b, T, r));
    });
}

cuth_status cuth_apply_csr(cuth_grid h, double dt, const double *x, double *y) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        cuth::Grid &g = *h->g;
        if (!x || !y) return fail(CUTH_E_INVALID, "x and y are required");
        if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(CUTH_E_INVALID, "dt must be >= 0");
        if (dt > 0.0 && !g.has_cap) return fail(CUTH_E_INVALID, "dt > 0 needs heat_cap");
        return report(cuth::apply_csr(g, dt, x, y));
    });
}

cuth_status cuth_precond_apply(cuth_grid h, double dt, int32_t precision, int32_t preconditioner,
                               double lmin, double lmax, int32_t degree, const void *r, void *z) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        cuth::Grid &g = *h->g;
        if (!r || !z) return fail(CUTH_E_INVALID, "r and z are required");
        if (r == z) return fail(CUTH_E_INVALID, "r and z must not alias");
        if (precision != CUTH_FP64 && precision != CUTH_MIXED && precision != CUTH_MIXED16)
            return fail(CUTH_E_INVALID, "bad precision");
        if (preconditioner < CUTH_PC_CHEBYSHEV || preconditioner > CUTH_PC_CHEBYSHEV_JACOBI)
            return fail(CUTH_E_INVALID, "preconditioner must be a cuth_preconditioner value");
        if (!finite_pos(lmin) || !finite_pos(lmax) || !(lmax > lmin))
            return fail(CUTH_E_INVALID, "need 0 < lmin < lmax");
        if (degree < 1 || degree > 256) return fail(CUTH_E_INVALID, "degree must be in 1..256");
        if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(CUTH_E_INVALID, "dt must be >= 0");
        if (dt > 0.0 && !g.has_cap) return fail(CUTH_E_INVALID, "dt > 0 needs heat_cap");
        return report(cuth::precond_apply(g, dt, precision, preconditioner, lmin, lmax, degree, r, z));
    });
}

cuth_status cuth_precond_apply_noalloc(cuth_grid h, double dt, int32_t precision,
                                       int32_t preconditioner, double lmin, double lmax,
                                       int32_t degree, const void *r, void *z) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        cuth::Grid &g = *h->g;
        if (!r || !z) return fail(CUTH_E_INVALID, "r and z are required");
        if (r == z) return fail(CUTH_E_INVALID, "r and z must not alias");
        if (precision != CUTH_FP64 && precision != CUTH_MIXED && precision != CUTH_MIXED16)
            return fail(CUTH_E_INVALID, "bad precision");
        if (preconditioner < CUTH_PC_CHEBYSHEV || preconditioner > CUTH_PC_CHEBYSHEV_JACOBI)
            return fail(CUTH_E_INVALID, "preconditioner must be a cuth_preconditioner value");
        if (!finite_pos(lmin) || !finite_pos(lmax) || !(lmax > lmin))
            return fail(CUTH_E_INVALID, "need 0 < lmin < lmax");
        if (degree < 1 || degree > 256) return fail(CUTH_E_INVALID, "degree must be in 1..256");
        if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(CUTH_E_INVALID, "dt must be >= 0");
        if (dt > 0.0 && !g.has_cap) return fail(CUTH_E_INVALID, "dt > 0 needs heat_cap");
        return report(
            cuth::precond_apply_noalloc(g, dt, precision, preconditioner, lmin, lmax, degree, r, z));
    });
}

cuth_status cuth_spectral_bounds(cuth_grid h, double dt, int32_t preconditioner, int32_t steps,
                                 const float *v0, double *alpha, double *beta, double *ritz_min,
                                 double *ritz_max, double *lmin, double *lmax) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        cuth::Grid &g = *h->g;
        if (preconditioner != CUTH_PC_CHEBYSHEV && preconditioner != CUTH_PC_CHEBYSHEV_JACOBI)
            return fail(CUTH_E_INVALID, "preconditioner must be a Chebyshev one");
        const bool scaled = preconditioner == CUTH_PC_CHEBYSHEV_JACOBI;
        if (steps < 2 || steps > 256) return fail(CUTH_E_INVALID, "steps must be in 2..256");
        if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(CUTH_E_INVALID, "dt must be >= 0");
        if (dt > 0.0 && !g.has_cap) return fail(CUTH_E_INVALID, "dt > 0 needs heat_cap");
        cuth::Status st;
        cuth::Setup *su = cuth::get_setup(g, dt, st);
        if (!su) return report(st);
        std::vector<double> a, b;
        st = cuth::run_lanczos(g, *su, steps, v0, a, b, scaled);
        if (st.bad()) return report(st);
        double lo, hi;
        cuth::tridiag_extremes(a, b, lo, hi);
        if (alpha)
            for (int j = 0; j < steps; ++j) alpha[j] = j < (int)a.size() ? a[j] : NAN;
        if (beta)
            for (int j = 0; j + 1 < steps; ++j) beta[j] = j < (int)b.size() ? b[j] : NAN;
        if (ritz_min) *ritz_min = lo;
        if (ritz_max) *ritz_max = hi;
        double lx = std::min(scaled ? 2.0 : su->gersh, 1.05 * hi), ln = lo;
        if (!(ln > 0.0) || !(lx > ln * (1.0 + 1e-6))) ln = 0.5 * lx;
        if (lmin) *lmin = ln;
        if (lmax) *lmax = lx;
        return CUTH_OK;
    });
}

cuth_status cuth_grid_reset_bounds(cuth_grid h) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        for (cuth::Setup &su : h->g->setups) su.have_bounds = false;
        return CUTH_OK;
    });
}

cuth_status cuth_profile_enable(cuth_grid h, int32_t on) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        cuth::Grid &g = *h->g;
        if (hipStreamSynchronize(g.stream) != hipSuccess)
            return fail(CUTH_E_DEVICE, "hipStreamSynchronize failed");
        if (on && g.pev.empty()) {
            g.pev.resize(512, nullptr);
            for (hipEvent_t &e : g.pev)
                if (hipEventCreate(&e) != hipSuccess) return fail(CUTH_E_DEVICE, "hipEventCreate failed");
        }
        g.prof = on != 0;
        g.pev_used = 0;
        g.prof_ms = 0.0;
        g.prof_count = 0;
        return CUTH_OK;
    });
}

cuth_status cuth_profile_read(cuth_grid h, double *total_ms, int64_t *launches,
                              double *bytes_per_launch, int32_t *fused) {
    return guarded([&]() -> cuth_status {
        if (check_handle(h) != CUTH_OK) return CUTH_E_INVALID;
        cuth::Grid &g = *h->g;
        if (hipStreamSynchronize(g.stream) != hipSuccess)
            return fail(CUTH_E_DEVICE, "hipStreamSynchronize failed");
        (void)cuth::prof_flush(g);
        if (total_ms) *total_ms = g.prof_ms;
        if (launches) *launches = g.prof_count;
        if (bytes_per_launch) *bytes_per_launch = g.prof_bytes;
        if (fused) *fused = g.prof_width - 1;
        return CUTH_OK;
    });
}

}  // extern "C"
