// Internal types shared by the gfx950 kernels and the host-side solver.
//
// Layout: every vector is a flat array over cells in the order
// i + nx*(j + ny*l) (x fastest, then y, then layer l from the bottom).  The
// operator is the 7-point stencil of the paper's Section 3.2 written in
// difference form,
//     (A x)_c = sink_l x_c + sum_faces g_f (x_c - x_nbr),
// which equals the assembled matrix (diagonal = sum of face conductances +
// sink) and keeps every row sum exactly equal to `sink`, also in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cuth {

constexpr int kMaxLayers = 64;
constexpr int kBX = 64;            // stencil tile: one wavefront along x
constexpr int kBY = 4;             // four wavefronts along y
constexpr int kThreads = kBX * kBY;

// Per-layer coefficients (uniform within a layer).
template <typename T>
struct LayerCoef {
    T gx, gy;     // lateral face conductance of the layer (used when no per-cell planes)
    T gzd, gzu;   // vertical conductance to the layer below / above (0 at the boundary)
    T sink;       // h*dx*dy on convective layers + C*dx*dy*dz/dt for transient operators
    T cap;        // C*dx*dy*dz/dt (weight of T_n in the transient right-hand side)
};

// Operator view handed to kernels.  gx/gy are null for per-layer-uniform grids;
// otherwise gx[c] couples c and c+1 (0 on the last column), gy[c] couples c and
// c+nx (0 on the last row).
template <typename T>
struct OpView {
    int nx, ny, nz;
    const T *gx;
    const T *gy;
    const LayerCoef<T> *lc;   // device [nz]
};

// Scalars of one PCG run (Algorithm 1), resident on the device.
template <typename T>
struct CgState {
    T rz;         // r_k^T z_k
    T rz_new;     // r_{k+1}^T z_{k+1} from the last preconditioner sweep
    T alpha;
    T beta;
    T pmu;        // p^T A p
    T rr;         // recursive ||r||^2
    T rr0;        // ||rhat||^2 of the inner right-hand side
    T tol2;       // stop when rr <= tol2
    T true_rr;    // last ||rhat - A x||^2
    T drift_rr;   // last ||(rhat - A x) - r||^2
    T true_prev;  // previous true residual norm (< 0: none yet)
    int done;     // 0 running, 1 tolerance, 2 drift, 3 stagnation, 4 breakdown
    int iter;     // completed CG iterations
    int first;    // 1 until the first search direction has been formed
    int pad;
};

// FP64 quantities of one outer residual evaluation.
struct OuterStats {
    double rr;       // ||b - A theta||_2^2
    double bb;       // ||b||_2^2
    double dinf;     // ||delta||_inf of the correction just applied
    double thinf;    // ||theta||_inf after the correction
    double bad;      // count of non-finite residual entries
    double pad[3];
};

// Reduction scratch: per-block partial values and the arrival counter used by
// the last block to finish a kernel (one cross-block pass, fixed order).
struct RedScratch {
    void *partials;
    unsigned *counter;
};

// Sizes of the grid handled by one launch (tile grid over x, y).
inline dim3 tile_grid(int nx, int ny) {
    return dim3((unsigned)((nx + kBX - 1) / kBX), (unsigned)((ny + kBY - 1) / kBY), 1);
}

// ---- launchers (kernels.hip) -------------------------------------------------
template <typename T>
void launch_apply(const OpView<T> &op, const T *x, T *y, hipStream_t s);

// Chebyshev sweep z_{j+1} = z_j + c1 (z_j - z_{j-1}) + c2 (r - A z_j).
// mode 1: z_j = r*inv_th, z_{j-1} = 0 (j = 1); mode 2: z_{j-1} = r*inv_th
// (j = 2); mode 0: z_{j-1} read from zo.  The result is written to zo.
// last: also reduce r^T z_{j+1} into st->rz_new.
template <typename T>
void launch_cheb(const OpView<T> &op, int mode, bool last, const T *z, T *zo, const T *r,
                 T c1, T c2, T inv_th, CgState<T> *st, RedScratch red, hipStream_t s);

template <typename T>
void launch_scale(int64_t n, const T *x, T a, T *y, CgState<T> *st, bool set_rz_from, const T *r,
                  RedScratch red, hipStream_t s);

template <typename T>
void launch_cg_dir(const OpView<T> &op, const T *z, const T *pold, T *pnew, T *mu,
                   CgState<T> *st, RedScratch red, hipStream_t s);

template <typename T>
void launch_cg_update(const OpView<T> &op, T *x, const T *p, T *r, const T *mu,
                      CgState<T> *st, RedScratch red, hipStream_t s);

template <typename T>
void launch_cg_check(const OpView<T> &op, const T *rhat, const T *x, const T *r,
                     CgState<T> *st, int force, RedScratch red, hipStream_t s);

// theta_out = (theta_in - in_off) + delta;  b = P + cap*(Tn - tn_off);
// r = b - A theta_out (FP64); optional copies of r in the inner precision.
template <typename TD, typename TI>
void launch_residual(const OpView<double> &op, const double *th_in, double in_off,
                     const TD *delta, const double *P, const double *Tn, double tn_off,
                     double *th_out, double *r64, TI *r_in, TI *rhat, OuterStats *os,
                     CgState<TI> *st, double inner_tol, RedScratch red, hipStream_t s);

void launch_add_scalar(int64_t n, const double *x, double a, double *y, hipStream_t s);
void launch_copy_to_float(int64_t n, const double *x, float *y, hipStream_t s);

// Face conductances of a grid with a per-cell lateral multiplier.  Writes the
// FP64 and FP32 planes and the per-layer maximum lateral off-diagonal row sum
// (as the bit pattern of a positive double) for the Gershgorin bound; counts
// invalid multiplier entries into *bad.
void launch_build_lateral(int nx, int ny, int nz, double dx, double dy, const double *dz,
                          const double *k_lat, const double *mult, double *gx64, double *gy64,
                          float *gx32, float *gy32, unsigned long long *maxrow,
                          unsigned int *bad, hipStream_t s);

// Lanczos building blocks (FP32).
void launch_fill_random(int64_t n, uint64_t seed, float *v, hipStream_t s);
void launch_norm2(int64_t n, const float *v, float *out, RedScratch red, hipStream_t s);
void launch_scale_by_rsqrt(int64_t n, const float *v, const float *nrm2, float *out, hipStream_t s);
void launch_lanczos_av(const OpView<float> &op, const float *v, const float *vprev,
                       const float *beta_prev, float *w, float *alpha_out, RedScratch red,
                       hipStream_t s);
void launch_lanczos_orth(int64_t n, float *w, const float *v, const float *alpha,
                         float *beta_out, RedScratch red, hipStream_t s);
void launch_div_scalar(int64_t n, float *w, const float *den, hipStream_t s);

// Adjoint gradient sums: per layer, S_lat[l] = sum over lateral faces of
// g (la_a - la_b)(th_a - th_b) and S_vert[l] = sum over the faces between l and
// l+1 of (la_l - la_{l+1})(th_l - th_{l+1}); both FP64, written to out[0..nz) and
// out[nz..2nz).
void launch_adjoint_sums(const OpView<double> &op, const double *lam, const double *T,
                         double t_amb, double *out, RedScratch red, hipStream_t s);
void launch_adjoint_finish(int nz, const double *sums, const double *fac_lat,
                           const double *fac_vert_up, const double *fac_vert_dn, double *dL_dk,
                           hipStream_t s);

}  // namespace cuth
