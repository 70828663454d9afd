// Host-side state of one grid handle and the solver entry points behind the C ABI.
#pragma once

#include "cuth_internal.hpp"
#include "../../include/cuth.h"

#include <string>
#include <vector>

namespace cuth {

// Device work vectors of one precision (each of length N).
template <typename T>
struct Work {
    T *x = nullptr, *r = nullptr, *rhat = nullptr, *pA = nullptr, *pB = nullptr, *mu = nullptr,
      *zA = nullptr, *zB = nullptr;
    bool ready() const { return x != nullptr; }
};

// Operator data that depends on dt (steady: dt == 0) plus cached spectral bounds.
struct Setup {
    double dt = 0.0;
    std::vector<LayerCoef<double>> hlc;
    LayerCoef<double> *lc64 = nullptr;
    LayerCoef<float> *lc32 = nullptr;
    bool have_bounds = false;
    int bounds_steps = 0;
    double lmin = 0, lmax = 0, ritz_min = 0, ritz_max = 0, gersh = 0;
};

// Result of one inner PCG run.
struct InnerResult {
    int iters = 0;
    int reason = 0;        // 1 tol, 2 drift, 3 stagnation, 4 breakdown, 5 iteration limit
    double true_red = 1;   // ||rhat - A x|| / ||rhat||
    int64_t stencils = 0;
    double bytes = 0;      // algorithmic bytes moved
};

struct Status {
    cuth_status code = CUTH_OK;
    std::string msg;
    static Status ok() { return Status(); }
    static Status err(cuth_status c, std::string m) {
        Status s;
        s.code = c;
        s.msg = std::move(m);
        return s;
    }
    bool bad() const { return code != CUTH_OK; }
};

// Launch shape of the stencil kernels of one precision.
struct Shape {
    int vx = 1, by = 4, zc = 64;
};

// Slots of the partials buffer (one per producer/consumer pair).
enum Slot { S_CHEB = 0, S_DIR, S_UPD, S_CHK, S_RES, S_LZA, S_LZB, S_MISC, S_COUNT };

struct Grid {
    int device = 0;
    hipStream_t stream = nullptr;
    int nx = 0, ny = 0, nz = 0;
    int64_t N = 0;
    double dx = 0, dy = 0, h_top = 0, h_bot = 0, t_amb = 0;
    std::vector<double> dz, k_lat, k_vert, cap;
    bool has_cap = false, per_cell = false;
    Shape sh32, sh64;

    double *gx64 = nullptr, *gy64 = nullptr;
    float *gx32 = nullptr, *gy32 = nullptr;
    std::vector<double> lat_rowmax;    // per layer, per-cell grids only

    std::vector<Setup> setups;
    Work<float> w32;
    Work<double> w64;
    double *thA = nullptr, *thB = nullptr;

    double *part = nullptr;           // S_COUNT slots of slot_doubles each, then the adjoint slot
    size_t slot_doubles = 0;
    double *part_adj = nullptr;
    CgState<float> *st32 = nullptr;
    CgState<double> *st64 = nullptr;
    float *lz = nullptr;              // Lanczos scalars on the device
    double *adj_fac = nullptr;        // adjoint factors [3 nz]

    // pinned host mirrors for stream-ordered readback
    CgState<float> *h_st32 = nullptr;
    CgState<double> *h_st64 = nullptr;
    double *h_part = nullptr;         // slot_doubles
    float *h_lz = nullptr;

    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;

    // kernel timing (measurement only): event pairs around the first general
    // Chebyshev sweep of each preconditioner application
    bool prof = false;
    std::vector<hipEvent_t> pev;
    size_t pev_used = 0;
    double prof_ms = 0.0, prof_bytes = 0.0;
    int64_t prof_count = 0;

    template <typename T>
    T *slot(int s) const {
        return reinterpret_cast<T *>(part + (size_t)s * slot_doubles);
    }
};

Status prof_flush(Grid &g);

Status grid_create(const cuth_grid_desc &d, hipStream_t s, Grid **out);
void grid_destroy(Grid *g);

Setup *get_setup(Grid &g, double dt, Status &st);
Status ensure_bounds(Grid &g, Setup &su, int steps);
Status run_lanczos(Grid &g, Setup &su, int steps, const float *v0, std::vector<double> &alpha,
                   std::vector<double> &beta);
void tridiag_extremes(const std::vector<double> &alpha, const std::vector<double> &beta,
                      double &lo, double &hi);

OpView<double> view64(const Grid &g, const Setup &su);
OpView<float> view32(const Grid &g, const Setup &su);

// Solve (dt == 0: G; dt > 0: C/dt + G) theta = P (+ cap*(Tn - t_amb)).  init:
// optional initial guess given as T (offset init_off).  The result is written as
// out = theta + out_off.
Status solve_system(Grid &g, double dt, const double *P, const double *Tn, const double *init,
                    double init_off, double *out, double out_off, const cuth_options &o,
                    cuth_stats *stats, bool transient_defaults);

Status precond_apply(Grid &g, double dt, int precision, double lmin, double lmax, int degree,
                     const void *r, void *z);
Status apply_op(Grid &g, double dt, int precision, const void *x, void *y);
Status residual(Grid &g, double dt, const double *b, const double *T, double *r);
Status adjoint(Grid &g, const double *T, const double *dL_dT, double *dL_dP, double *dL_dk,
               const cuth_options &o, cuth_stats *stats);

}  // namespace cuth
