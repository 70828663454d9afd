// Host-side state of one grid handle and the solver entry points behind the C ABI.
#pragma once

#include "cuth_internal.hpp"
#include "../../include/cuth.h"

#include <deque>
#include <string>
#include <vector>

namespace cuth {

// Device work vectors of one precision (each of length N).
template <typename T>
struct Work {
    T *x = nullptr, *r = nullptr, *rhat = nullptr, *pA = nullptr, *pB = nullptr, *mu = nullptr,
      *zA = nullptr, *zB = nullptr;
    T *zC = nullptr, *zD = nullptr;   // the fused sweep pairs' extra iterates (FP32)
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
    // interval of D^{-1} A for the Jacobi-scaled Chebyshev preconditioner
    // (Lanczos on D^{-1/2} A D^{-1/2}, dis = D^{-1/2} per cell in FP32)
    float *dis = nullptr;
    bool have_jbounds = false;
    int jbounds_steps = 0;
    double jlmin = 0, jlmax = 0, jritz_min = 0, jritz_max = 0;
    // CSR copy of the FP64 operator (cuth_apply_csr), built on first use
    int *csr_ptr = nullptr, *csr_col = nullptr;
    double *csr_val = nullptr;
    int64_t csr_nnz = 0;
    // CG iterations at which the last inner solve of refinement cycle c stopped
    // on its tolerance, per inner precision ([0]: FP64, [1]: FP32) and
    // preconditioner (cuth_preconditioner); 0 = unknown
    int stop_iter[2][4][16] = {};
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

// Launch shape of the stencil kernels of one precision.  fr > 0: general
// Chebyshev sweeps run as fused pairs with fr rows and fzc layers per workgroup
// and fwpr wavefronts per row (FP32 only).
struct Shape {
    int vx = 1, by = 1, zc = 8;
    int fr = 0, fzc = 8, fwpr = 1;   // fused pairs: rows per workgroup (0: off), layers, wavefronts per row
    int tr = 0, tzc = 8, twpr = 1;   // fused triples (used only with pairs on)
};

// Device descriptors, states and reduction partials for up to `cap` problems
// solved together (a single solve uses a set of one).
struct Engine {
    int cap = 0, kcap = 0;
    size_t slot_doubles = 0;
    InnerProb<float> *in32 = nullptr, *h_in32 = nullptr;
    InnerProb<double> *in64 = nullptr, *h_in64 = nullptr;
    OuterProb<float, float> *out32 = nullptr, *h_out32 = nullptr;
    OuterProb<double, double> *out64 = nullptr, *h_out64 = nullptr;
    CgState<float> *st32 = nullptr, *h_st32 = nullptr;
    CgState<double> *st64 = nullptr, *h_st64 = nullptr;
    float *cheb32 = nullptr, *h_cheb32 = nullptr;
    double *cheb64 = nullptr, *h_cheb64 = nullptr;
    double *part = nullptr, *h_part = nullptr;   // 5 slots of slot_doubles
    hipStream_t own = nullptr;                   // stream for graph capture
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // instantiated chunks of CG iterations, by launch configuration: a chunk's
    // kernel arguments depend only on that configuration and the engine's own
    // buffers (the descriptors they point to are re-uploaded per inner solve)
    std::vector<std::pair<std::string, hipGraphExec_t>> graphs;
};

// Work vectors and engine of a batched solve, kept between calls with the same
// batch signature (sizes, precision, right-hand sides): one per coefficient
// storage group, held by the batch's first grid.
struct BatchPool {
    std::string key;
    float *pool32 = nullptr;
    double *pool64 = nullptr, *poolth = nullptr;
    Engine E;
};

// Slots of a grid's own partials buffer (Lanczos, adjoint).
enum Slot { S_LZA = 0, S_LZB, S_COUNT };

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
    uint16_t *hx = nullptr, *hy = nullptr;   // FP16 planes (per-cell grids)
    std::vector<double> lat_rowmax;    // per layer, per-cell grids only
    std::vector<int> e16;              // per-layer FP16 scale exponent e_l
    double *build_tmp = nullptr;       // per-layer inputs and maxima of the plane build
    bool valid = true;                 // false after a rejected multiplier (set_conductivity)

    std::deque<Setup> setups;         // a deque: Setup pointers stay valid as dt's are added
    Work<float> w32;
    Work<double> w64;
    double *thA = nullptr, *thB = nullptr;

    double *part = nullptr;           // S_COUNT slots of slot_doubles, then the adjoint slot
    size_t slot_doubles = 0;
    double *part_adj = nullptr;
    float *lz = nullptr;              // Lanczos scalars on the device
    double *adj_fac = nullptr;        // adjoint factors [3 nz]
    float *h_lz = nullptr;
    Engine eng;                       // single-problem engine of this grid
    BatchPool batch[2];               // batches led by this grid (uniform / per-cell group)

    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;

    // kernel timing (measurement only): event pairs around the first general
    // Chebyshev sweep of each preconditioner application
    bool prof = false;
    std::vector<hipEvent_t> pev;
    std::vector<int> pev_tag;   // CG iteration of each recorded block (-1: initial)
    std::vector<int> pev_cnt;   // launches in each recorded block
    size_t pev_used = 0;
    double prof_ms = 0.0, prof_bytes = 0.0;
    int prof_width = 1;   // sweeps per timed launch (2: fused pair, 3: fused triple)
    int64_t prof_count = 0;

    template <typename T>
    T *slot(int s) const {
        return reinterpret_cast<T *>(part + (size_t)s * slot_doubles);
    }
};

Status prof_flush(Grid &g, int valid_below = 1 << 30);

Status grid_create(const cuth_grid_desc &d, hipStream_t s, Grid **out);
void grid_destroy(Grid *g);
// New layer conductivities for an existing grid, rebuilt in place (mult: the
// per-cell multiplier, required for per-cell grids and ignored otherwise).
Status grid_set_conductivity(Grid &g, const double *k_lat, const double *k_vert, const double *mult);

Setup *get_setup(Grid &g, double dt, Status &st);
// scaled: the interval of D^{-1} A (Lanczos on D^{-1/2} A D^{-1/2}), for the
// Jacobi-scaled preconditioner
Status ensure_bounds(Grid &g, Setup &su, int steps, bool scaled = false);
Status run_lanczos(Grid &g, Setup &su, int steps, const float *v0, std::vector<double> &alpha,
                   std::vector<double> &beta, bool scaled = false);
void tridiag_extremes(const std::vector<double> &alpha, const std::vector<double> &beta,
                      double &lo, double &hi);

OpView<double> view64(const Grid &g, const Setup &su);
// h16: with the FP16-stored lateral conductances (CUTH_MIXED16 sweeps)
OpView<float> view32(const Grid &g, const Setup &su, bool h16 = false);

// Solve (dt == 0: G; dt > 0: C/dt + G) theta = P (+ cap*(Tn - t_amb)).  init:
// optional initial guess given as T (offset init_off).  The result is written as
// out = theta + out_off.
Status solve_system(Grid &g, double dt, const double *P, const double *Tn, const double *init,
                    double init_off, double *out, double out_off, const cuth_options &o,
                    cuth_stats *stats, bool transient_defaults);

// Steady solves of nsys grids with nrhs right-hand sides each, all advanced
// together in batched launches.
Status solve_batch(int nsys, Grid *const *grids, int nrhs, const double *const *P,
                   double *const *T, const cuth_options &o, cuth_stats *stats);

Status precond_apply(Grid &g, double dt, int precision, int preconditioner, double lmin,
                     double lmax, int degree, const void *r, void *z);
// As precond_apply, with every device buffer beyond r, z and the grid's operator
// planes taken from the per-device scratch array (no device allocation); single
// sweeps only.
Status precond_apply_noalloc(Grid &g, double dt, int precision, int preconditioner, double lmin,
                             double lmax, int degree, const void *r, void *z);
Status apply_op(Grid &g, double dt, int precision, const void *x, void *y);
Status residual(Grid &g, double dt, const double *b, const double *T, double *r);
Status apply_csr(Grid &g, double dt, const double *x, double *y);
// Builds the setup's CSR copy of the FP64 operator if it has none.
Status ensure_csr(Grid &g, Setup &su);
Status adjoint(Grid &g, const double *T, const double *dL_dT, double *dL_dP, double *dL_dk,
               const cuth_options &o, cuth_stats *stats);

}  // namespace cuth
