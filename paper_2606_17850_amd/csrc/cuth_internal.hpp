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
constexpr int kWave = 64;          // CDNA wavefront
constexpr int kMaxBY = 8;          // rows (wavefronts) per workgroup
constexpr int kRedBlocks = 1024;   // workgroups of the 1-D (non-stencil) reduction kernels

// Per-layer coefficients (uniform within a layer).
template <typename T>
struct LayerCoef {
    T gx, gy;     // lateral face conductance of the layer (used when no per-cell planes)
    T gzd, gzu;   // vertical conductance to the layer below / above (0 at the boundary)
    T sink;       // h*dx*dy on convective layers + C*dx*dy*dz/dt for transient operators
    T cap;        // C*dx*dy*dz/dt (weight of T_n in the transient right-hand side)
    T hs;         // 2^-e_l: factor of the layer's FP16-stored lateral conductances
};

// Operator view handed to kernels.  gx/gy are null for per-layer-uniform grids;
// otherwise gx[c] couples c and c+1 (0 on the last column), gy[c] couples c and
// c+nx (0 on the last row).  vx, by, zc: launch shape (cells per lane along
// x, wavefront rows per workgroup, layers per vertical march); vx divides nx.
// hx/hy (FP16 bit patterns of gx*2^e_l, gy*2^e_l; Section 4.2, the
// half-precision copy of the in-plane diagonals) are set only where the
// Chebyshev sweeps use the FP16-stored conductances.
template <typename T>
struct OpView {
    int nx, ny, nz;
    const T *gx;
    const T *gy;
    const LayerCoef<T> *lc;   // device [nz]
    int vx, by, zc;
    const uint16_t *hx = nullptr;
    const uint16_t *hy = nullptr;
    // FP32 copies of gx/gy read by FP64 operators that promote them (the
    // paper's "FP64/32 SpMV"; set where such launches are made)
    const float *fx = nullptr;
    const float *fy = nullptr;
    // CSR copy of the FP64 operator (row r's entries at [csr_ptr[r],
    // csr_ptr[r+1])); set only where a solve runs on CSR storage
    const int *csr_ptr = nullptr;
    const int *csr_col = nullptr;
    const double *csr_val = nullptr;
};

// Where a stencil kernel's operator comes from.
enum CoefSrc : int {
    CS_OWN = 0,   // per-cell op.gx/op.gy in the operator's precision, or the per-layer constants
    CS_F16 = 1,   // op.hx/op.hy: FP16 copies at the layer's power-of-two scale (FP32 sweeps)
    CS_F32 = 2,   // op.fx/op.fy: FP32 copies, promoted (FP64 operators)
    CS_CSR = 3    // op.csr_*: every row's entries from the CSR copy, one lane per row
                  // (Section 5, Ablation I's baseline storage; FP64 operators)
};

// Number of workgroups of a stencil launch (one 64*vx by `by` tile and one
// chunk of zc layers each).
inline int tiles_x(int nx, int vx) { return (nx + kWave * vx - 1) / (kWave * vx); }
inline int tiles_y(int ny, int by) { return (ny + by - 1) / by; }
inline int tiles_z(int nz, int zc) { return (nz + zc - 1) / zc; }
template <typename T>
inline int stencil_blocks(const OpView<T> &op) {
    return tiles_x(op.nx, op.vx) * tiles_y(op.ny, op.by) * tiles_z(op.nz, op.zc);
}
// x windows of a fused launch (a pair: 2 sweeps, a triple: 3) over rows of nx
// cells.  A workgroup row holds W = wpr*64*vx cells.  When W < nx the row is
// covered by windows that overlap by halo lanes: each window computes all W
// cells and owns the W - 2*hl*vx between its hl = ceil((sweeps - 1)/vx) halo
// lanes on either side (the last sweep needs sweeps - 1 cells of halo per side);
// window t starts at x = t*(W - 2*hl*vx) - hl*vx.
__host__ __device__ inline int fused_halo_lanes(int vx, int sweeps) {
    return (sweeps - 1 + vx - 1) / vx;
}
__host__ __device__ inline int fused_windows(int nx, int vx, int wpr, int sweeps) {
    const int W = wpr * kWave * vx;
    if (W >= nx) return 1;
    const int S = W - 2 * fused_halo_lanes(vx, sweeps) * vx;
    return (nx + S - 1) / S;
}
inline int red_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > kRedBlocks ? kRedBlocks : b));
}

// Scalars of one PCG run (Algorithm 1) resident on the device.  Kernels never
// read a field that a workgroup of the same launch writes, except `done`, which
// every workgroup of a problem sets to the same value from the same data.
template <typename T>
struct CgState {
    T rz[2];      // r_k^T z_k in slot k & 1 (direction kernel of k); the host sets
                  // slot 1 to +inf before iteration 0, which marks "no previous p"
    T rr;         // last recursive ||r||^2
    T rr0;        // ||rhat||^2 of the inner right-hand side (host)
    T tol2;       // converged when rr <= tol2 (host)
    T pad;
    int done;     // 0 running, 1 tolerance, 2 drift, 3 stagnation, 4 breakdown
    int iter;     // completed CG iterations (updates followed by a convergence test)
    int pad2[2];
};

// One inner PCG problem (one system and right-hand side) of a batched launch.
// The launch covers the problems' workgroup slots [tile0, tile0 + ntiles) back
// to back; slot s is given to the workgroup of XCD-banded index s.
template <typename T>
struct InnerProb {
    OpView<T> op;
    int ntx, ntz;             // tiles along x and z (the launch shape is op.vx/by/zc)
    int tile0, ntiles;
    T *x, *r, *rhat, *mu;
    T *p[2];
    T *z[4];                  // Chebyshev iterates; z[2], z[3] only for fused sweep pairs
    CgState<T> *st;
    const T *cheb;            // 1/theta at [0], c1_j at [1 + j], c2_j at [1 + kcap + j]
    int kcap, pad;
    int f_tile0 = 0, f_ntiles = 0;   // workgroup slots of fused sweep pairs (launch_cheb2_b)
    int t_tile0 = 0, t_ntiles = 0;   // ... of fused sweep triples (launch_cheb3_b)
    // FP64 CG with an FP32 preconditioner (the paper's stage-switched scheme):
    // the update also writes r_lo = (float) r; k_promote_dot reads the
    // preconditioner's z_lo; k_reduce_conv mirrors the stop flag to *done_lo.
    float *r_lo = nullptr;
    const float *z_lo = nullptr;
    int *done_lo = nullptr;
};

// One FP64 outer-residual problem of a batched launch:
// theta_out = (theta_in - in_off) + delta;  b = P + cap*(Tn - tn_off);
// r = b - A theta_out, with optional copies of r in the inner precision.
template <typename TD, typename TI>
struct OuterProb {
    OpView<double> op;
    int ntx, ntz, tile0, ntiles;
    const double *th_in;
    double in_off;
    const TD *delta;
    const double *P;
    const double *Tn;
    double tn_off;
    double *th_out, *r64;
    TI *r_in, *rhat;
};

// ---- launchers (kernels.hip) -------------------------------------------------
// Every reduction writes one partial per workgroup slot into `part` (value v of
// slot s at part[v*nb + s], nb = total slots of the launch); the consumer (next
// kernel, or the host) sums a problem's slots in a fixed order.  A consumer
// launched with red = true instead reads problem p's sum at part_in[p], written
// by launch_reduce_b.

template <typename T>
void launch_apply(const OpView<T> &op, const T *x, T *y, hipStream_t s);

// Chebyshev sweep j (Section 4.3, two-term form):
//   z_{j+1} = z_j + c1_j (z_j - z_{j-1}) + c2_j (r - A z_j).
// mode 1 (j = 1): z_1 = r/theta and z_0 = 0 are implicit; mode 2 (j = 2):
// z_{j-1} = r/theta implicit; mode 0: z_{j-1} read.  zsel = in + 4*out: z_j is in
// z[in], z_{j-1} in z[out] (read at the cell only) and the result overwrites z[out].  last: partials of r^T z_{j+1}.  chk: the first kernel after
// a CG update reduces the update's partials (part_in) and stops converged
// problems (rr <= tol2).
// cs (CoefSrc): CS_F16 reads the FP16-stored lateral conductances (FP32,
// per-cell grids only), CS_CSR the CSR copy (FP64); otherwise CS_OWN.
// jac: the Jacobi-scaled sweep z_{j+1} = z_j + c1 (z_j - z_{j-1}) + c2 D^{-1}(r - A z_j)
// with D = diag(A) (beyond the paper); mode 3 (z_1 read from z[in], z_0 = 0)
// or 0 only, and no chk (its first kernel is the PM_JCHEB scale pass).
template <typename T>
void launch_cheb_b(const InnerProb<T> *probs, int nprob, int nb, bool pc, int cs, bool jac, int vx,
                   int by, int mode, bool last, bool chk, int j, int zsel, const T *part_in,
                   bool red, T *part_out, hipStream_t s);

// Two consecutive general sweeps j, j+1 in one pass (temporal blocking):
// zsel = N + 4 P + 16 X + 64 Y with z_j in z[N], z_{j-1} in z[P]; z_{j+1} is
// written to z[X] and z_{j+2} to z[Y] (four distinct buffers).  A workgroup is
// R + 2 rows of wpr wavefronts (whole rows of 64*vx*wpr >= nx cells) and a chunk
// of zc layers; the launch covers the problems' slots [f_tile0, f_tile0 +
// f_ntiles) with f_ntiles = ceil(ny / R) * ceil(nz / zc).  FP32; h16: the
// FP16-stored lateral conductances (per-cell grids).
template <typename T>
void launch_cheb2_b(const InnerProb<T> *probs, int nprob, int nb, bool pc, bool h16, bool jac,
                    int vx, int R, int zc, int wpr, int j, int zsel, hipStream_t s);

// Three consecutive general sweeps j, j+1, j+2 in one pass: zsel as for the
// pair, z_{j+2} written to z[X] and z_{j+3} to z[Y] (z_{j+1} stays on chip).
// A workgroup is R + 4 rows of wpr wavefronts and a chunk of zc layers; the
// launch covers the problems' slots [t_tile0, t_tile0 + t_ntiles) with
// t_ntiles = ceil(ny / R) * ceil(nz / zc); dynamic LDS 3 (2R + 6) rows of
// 64*vx*wpr values.  FP32; h16 and jac as for the pair.  At j = 2 without jac
// z_{j-1} = z_1 = r / theta is formed from r (z[P] is not read).
template <typename T>
void launch_cheb3_b(const InnerProb<T> *probs, int nprob, int nb, bool pc, bool h16, bool jac, int vx,
                    int R, int zc, int wpr, int j, int zsel, hipStream_t s);

// Single-pass preconditioner into z[0] (same chk/last behaviour as the sweeps):
// pm 0: z = r/theta (degree-1 Chebyshev), 1: z = r/diag(A) (Jacobi), 2: z = r,
// 3: z = r/(theta diag(A)) (first iterate of the Jacobi-scaled Chebyshev).
template <typename T>
void launch_scale_b(const InnerProb<T> *probs, int nprob, int nb, bool pc, int pm, int vx, int by,
                    bool chk, const T *part_in, bool red, T *part_out, hipStream_t s);

// CG iteration of parity par: rz = sum(part_in); p[par] = z[zfin] + (rz / rz_prev) p[1-par];
// mu = A p[par]; partials of p^T mu.  cs: CS_F32 (FP64, per-cell grids) promotes
// the FP32-stored conductances, CS_CSR (FP64) reads the CSR copy; else CS_OWN.
template <typename T>
void launch_dir_b(const InnerProb<T> *probs, int nprob, int nb, bool pc, int cs, int vx,
                  int by, int par, int zfin, const T *part_in, bool red, T *part_out,
                  hipStream_t s);

// f32coef (FP64 only): the product reads the FP32 copies op.fx/op.fy, promoted
// (the paper's "FP64/32 SpMV" of the early CG stage).
// z[0] = (T) z_lo with partials of r^T z (FP64 CG with an FP32 preconditioner).
template <typename T>
void launch_promote_dot(const InnerProb<T> *probs, int nprob, int nb, int vx, int by, T *part_out,
                        hipStream_t s);

// One workgroup per problem: r^T r from the update's partials, convergence
// test against st->tol2, stop flag mirrored to *done_lo.
template <typename T>
void launch_reduce_conv(const InnerProb<T> *probs, int nprob, const T *part_in, hipStream_t s);

// x += alpha p[par] (x = alpha p on the first iteration), r -= alpha mu with
// alpha = rz / p^T mu; partials of r^T r.
template <typename T>
void launch_update_b(const InnerProb<T> *probs, int nprob, int nb, int vx, int by, int par,
                     const T *part_in, bool red, T *part_out, hipStream_t s);

// red_out[p] = fixed-order sum of problem p's partials in part_in (one
// workgroup per problem).
template <typename T>
void launch_reduce_b(const InnerProb<T> *probs, int nprob, const T *part_in, T *red_out,
                     hipStream_t s);

// True residual rt = rhat - A x: partials of ||rt||^2 and ||rt - r||^2 (cs:
// CS_CSR for the CSR copy, FP64; else CS_OWN).
template <typename T>
void launch_check_b(const InnerProb<T> *probs, int nprob, int nb, bool pc, int cs, int vx, int by,
                    T *part_out, hipStream_t s);

// FP64 outer residual; partials of ||r||^2, ||b||^2, max|delta|, max|theta_out|,
// count of non-finite r.  flags: the streams every problem of the launch has
// (residual_flags), or -1 where they differ.
template <typename TD, typename TI>
void launch_residual_b(const OuterProb<TD, TI> *probs, int nprob, int nb, bool pc, int vx, int by,
                       int flags, double *part_out, hipStream_t s);
// bit 0 theta_in, bit 1 delta, bit 2 T_n, bit 3 r64 as the only output (else
// theta_out, r_in and rhat, all present); -1 for any other combination
template <typename TD, typename TI>
inline int residual_flags(const OuterProb<TD, TI> &o) {
    const bool out_api = o.r64 && !o.th_out && !o.r_in && !o.rhat;
    const bool out_outer = !o.r64 && o.th_out && o.r_in && o.rhat;
    if (!out_api && !out_outer) return -1;
    return (o.th_in ? 1 : 0) | (o.delta ? 2 : 0) | (o.Tn ? 4 : 0) | (out_api ? 8 : 0);
}
constexpr int kResidualValues = 5;
// Per-problem totals of launch_residual_b's partials (ntot: its workgroups), in
// a fixed order: out[p * kResidualValues + v].
template <typename TD, typename TI>
void launch_reduce_outer(const OuterProb<TD, TI> *probs, int nprob, const double *part, int ntot,
                         double *out, hipStream_t s);

void launch_add_scalar(int64_t n, const double *x, double a, double *y, hipStream_t s);
// y = (float) x
void launch_to_f32(int64_t n, const double *x, float *y, hipStream_t s);

// CSR copy of the FP64 operator: row r's entries at [ptr[r], ptr[r+1]) in
// ascending column order; and y = A x with one thread per row.
void launch_csr_fill(const OpView<double> &op, const int *ptr, int *col, double *val,
                     hipStream_t s);
void launch_csr_spmv(int64_t n, const int *ptr, const int *col, const double *val,
                     const double *x, double *y, hipStream_t s);

// Face conductances of a grid with a per-cell lateral multiplier.  Writes the
// FP64 and FP32 planes, the per-layer maximum lateral off-diagonal row sum (as
// the bit pattern of a positive double) for the Gershgorin bound and the
// per-layer maximum single lateral conductance (same encoding) for the FP16
// scale; counts invalid multiplier entries into *bad.
void launch_build_lateral(int nx, int ny, int nz, double dx, double dy, const double *dz,
                          const double *k_lat, const double *mult, double *gx64, double *gy64,
                          float *gx32, float *gy32, unsigned long long *maxrow,
                          unsigned long long *maxg, unsigned int *bad, hipStream_t s);

// FP16 planes: hx[c] = fp16(fp32(gx64[c] * scale[l])) (round to nearest even at
// each step; scale[l] = 2^e_l), hy likewise, as bit patterns.
void launch_build_fp16(int nx, int ny, int nz, const double *gx64, const double *gy64,
                       const double *scale, uint16_t *hx, uint16_t *hy, hipStream_t s);

// Lanczos building blocks (FP32).  lz: device scalars, alpha_j at lz[j],
// beta_j at lz[256 + j].
void launch_fill_random(int64_t n, uint64_t seed, float *v, hipStream_t s);
void launch_norm2(int64_t n, const float *v, float *part_out, hipStream_t s);
void launch_scale_rsqrt(int64_t n, const float *v, const float *part_in, int np_in, float *out,
                        hipStream_t s);
void launch_lanczos_av(const OpView<float> &op, int j, const float *v, const float *vprev,
                       const float *lz, const float *dis, float *w, float *part_out,
                       hipStream_t s);
// dis = D^{-1/2}, D = diag(A), per cell (FP32) of an FP64 operator; with dis,
// launch_lanczos_av applies D^{-1/2} A D^{-1/2}
void launch_jacobi_dis(const OpView<double> &op, float *dis, hipStream_t s);
void launch_lanczos_orth(int64_t n, int j, float *w, const float *v, float *lz,
                         const float *part_in, int np_in, float *part_out, hipStream_t s);
void launch_lanczos_div(int64_t n, int j, float *w, float *lz, const float *part_in, int np_in,
                        hipStream_t s);

// Adjoint gradient: per layer l, S_lat[l] = sum over lateral faces of
// g (la_a - la_b)(th_a - th_b) and S_vert[l] = sum over the faces between l and
// l+1 of (la_l - la_{l+1})(th_l - th_{l+1}); then
// dL_dk[l] = dL/dk_lat[l] + dL/dk_vert[l]
//          = -(fac_lat[l] S_lat[l] + fac_up[l] S_vert[l] + fac_dn[l] S_vert[l-1]).
void launch_adjoint(const OpView<double> &op, const double *lam, const double *T, double t_amb,
                    const double *fac, double *part, double *dL_dk, hipStream_t s);

// ---- allocation-free entry point (kernels.hip) --------------------------------
// Bytes of the per-device scratch array that cuth_precond_apply_noalloc takes
// every device buffer from (beyond its r, z and the grid's operator planes).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// Device address of the scratch array on `device`: looked up once per device
// with that device current, then returned from the cache.
hipError_t noalloc_scratch(int device, unsigned char **ptr);
// Copy n host bytes (a multiple of 4) to the device address dst in stream
// order, carried by kernel arguments (2 KiB per launch): no staging buffer and
// no allocation.
hipError_t launch_put(const void *src, size_t n, void *dst, hipStream_t s);

}  // namespace cuth
