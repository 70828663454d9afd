// gfx950 kernels of the layered-stencil PCG.
//
// Every stencil kernel uses the same mapping: a 64 x 4 workgroup (four
// wavefronts, one per grid row) owns a 64 x 4 column tile of the lateral grid
// and marches up through all layers, keeping the values of the layers below,
// at and above the current one in registers.  Lateral neighbours are read from
// global memory; they are the same cache lines the neighbouring lanes and rows
// load, so HBM sees each vector close to once per sweep.  Loads along x are
// unit-stride and coalesced.
//
// Reductions (dot products, norms, maxima) are done with wavefront butterflies,
// then across the four wavefronts in LDS; each workgroup writes one partial and
// the last workgroup to arrive (atomic ticket) sums all partials in a fixed
// order and writes the scalars the next kernel needs (alpha, beta, ...).  No
// host round trip is needed between kernels of a CG iteration, and results are
// run-to-run deterministic.
#include "cuth_internal.hpp"

#include <cmath>

namespace cuth {
namespace {

__device__ __forceinline__ int tid_lin() { return threadIdx.x + blockDim.x * threadIdx.y; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <typename T>
__device__ __forceinline__ T load_coherent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum (or max, for slots whose bit is set in maxmask; those values must be
// >= 0) of v[k] over the whole grid.  Returns true in the last workgroup to
// finish, where v[k] then holds the grid-wide results in every thread.
// Requires blockDim = kThreads and every thread of the workgroup to call it.
template <typename T, int NV>
__device__ __forceinline__ bool grid_reduce(T (&v)[NV], unsigned maxmask, T *partials,
                                            unsigned *counter) {
    constexpr int NW = kThreads / 64;
    __shared__ T sh[NV][NW];
    __shared__ int is_last;
    const int t = tid_lin(), lane = t & 63, w = t >> 6;
    const int nb = gridDim.x * gridDim.y;
    const int b = blockIdx.x + gridDim.x * blockIdx.y;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const bool mx = (maxmask >> k) & 1u;
        T x = mx ? wave_max(v[k]) : wave_sum(v[k]);
        if (lane == 0) sh[k][w] = x;
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const bool mx = (maxmask >> k) & 1u;
            T a = sh[k][0];
            for (int q = 1; q < NW; ++q) a = mx ? fmax(a, sh[k][q]) : a + sh[k][q];
            partials[(size_t)k * nb + b] = a;
        }
        __threadfence();
        const unsigned ticket = atomicAdd(counter, 1u);
        is_last = (ticket == (unsigned)(nb - 1));
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const bool mx = (maxmask >> k) & 1u;
        T a = T(0);
        for (int q = t; q < nb; q += kThreads) {
            const T p = load_coherent(&partials[(size_t)k * nb + q]);
            a = mx ? fmax(a, p) : a + p;
        }
        a = mx ? wave_max(a) : wave_sum(a);
        if (lane == 0) sh[k][w] = a;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const bool mx = (maxmask >> k) & 1u;
        T a = sh[k][0];
        for (int q = 1; q < NW; ++q) a = mx ? fmax(a, sh[k][q]) : a + sh[k][q];
        v[k] = a;
    }
    if (t == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// (A x)_c at cell c = (i, j, l): xc, xdn, xup are x at c, c - plane, c + plane;
// X(q) fetches x at any in-range cell q for the lateral neighbours.
template <typename T, bool PC, typename F>
__device__ __forceinline__ T stencil_at(const OpView<T> &op, const LayerCoef<T> &L, int i, int j,
                                        int l, int64_t c, T xc, T xdn, T xup, F &&X) {
    T gxm, gxp, gym, gyp;
    if constexpr (PC) {
        gxp = op.gx[c];
        gyp = op.gy[c];
        gxm = i > 0 ? op.gx[c - 1] : T(0);
        gym = j > 0 ? op.gy[c - op.nx] : T(0);
    } else {
        gxm = gxp = L.gx;
        gym = gyp = L.gy;
    }
    T a = L.sink * xc;
    if (i > 0) a += gxm * (xc - X(c - 1));
    if (i < op.nx - 1) a += gxp * (xc - X(c + 1));
    if (j > 0) a += gym * (xc - X(c - op.nx));
    if (j < op.ny - 1) a += gyp * (xc - X(c + op.nx));
    if (l > 0) a += L.gzd * (xc - xdn);
    if (l < op.nz - 1) a += L.gzu * (xc - xup);
    return a;
}

// March one (i, j) column through all layers; emit(l, c, x_c, (A x)_c).
template <typename T, bool PC, typename F, typename E>
__device__ __forceinline__ void column(const OpView<T> &op, int i, int j, F &&X, E &&emit) {
    const int64_t plane = (int64_t)op.nx * op.ny;
    int64_t c = i + (int64_t)op.nx * j;
    T xdn = T(0), xc = X(c);
    for (int l = 0; l < op.nz; ++l, c += plane) {
        const LayerCoef<T> L = op.lc[l];
        const T xup = (l + 1 < op.nz) ? X(c + plane) : T(0);
        const T ax = stencil_at<T, PC>(op, L, i, j, l, c, xc, xdn, xup, X);
        emit(l, c, xc, ax);
        xdn = xc;
        xc = xup;
    }
}

__device__ __forceinline__ void tile_ij(int &i, int &j) {
    i = blockIdx.x * kBX + threadIdx.x;
    j = blockIdx.y * kBY + threadIdx.y;
}

template <typename T>
__device__ __forceinline__ bool finite_val(T v) {
    return isfinite(v);
}

// ------------------------------------------------------------------ apply
template <typename T, bool PC>
__global__ __launch_bounds__(kThreads) void k_apply(OpView<T> op, const T *__restrict__ x,
                                                    T *__restrict__ y) {
    int i, j;
    tile_ij(i, j);
    if (i >= op.nx || j >= op.ny) return;
    column<T, PC>(
        op, i, j, [&](int64_t q) { return x[q]; },
        [&](int, int64_t c, T, T ax) { y[c] = ax; });
}

// ------------------------------------------------------------ Chebyshev sweep
template <typename T, bool PC, int MODE, bool LAST>
__global__ __launch_bounds__(kThreads) void k_cheb(OpView<T> op, const T *__restrict__ z, T *zo,
                                                   const T *__restrict__ r, T c1, T c2, T inv_th,
                                                   CgState<T> *st, T *partials,
                                                   unsigned *counter) {
    if (st->done) return;
    int i, j;
    tile_ij(i, j);
    T acc[1] = {T(0)};
    if (i < op.nx && j < op.ny) {
        auto X = [&](int64_t q) -> T {
            if constexpr (MODE == 1) return r[q] * inv_th;
            else return z[q];
        };
        column<T, PC>(op, i, j, X, [&](int, int64_t c, T zj, T az) {
            const T rc = r[c];
            T zm;
            if constexpr (MODE == 0) zm = zo[c];
            else if constexpr (MODE == 2) zm = rc * inv_th;
            else zm = T(0);
            const T zn = zj + c1 * (zj - zm) + c2 * (rc - az);
            zo[c] = zn;
            if constexpr (LAST) acc[0] += rc * zn;
        });
    }
    if constexpr (LAST) {
        if (grid_reduce<T, 1>(acc, 0u, partials, counter)) {
            if (tid_lin() == 0) {
                st->rz_new = acc[0];
                if (!(acc[0] > T(0)) || !finite_val(acc[0])) st->done = 4;
            }
        }
    }
}

// z = a*r, and r^T z into st->rz_new (degree-1 preconditioner).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale_dot(int64_t n, const T *__restrict__ r, T a,
                                                        T *__restrict__ z, CgState<T> *st,
                                                        T *partials, unsigned *counter) {
    if (st->done) return;
    T acc[1] = {T(0)};
    const int64_t stride = (int64_t)gridDim.x * gridDim.y * kThreads;
    for (int64_t q = (int64_t)(blockIdx.x + gridDim.x * blockIdx.y) * kThreads + tid_lin(); q < n;
         q += stride) {
        const T v = a * r[q];
        z[q] = v;
        acc[0] += r[q] * v;
    }
    if (grid_reduce<T, 1>(acc, 0u, partials, counter)) {
        if (tid_lin() == 0) {
            st->rz_new = acc[0];
            if (!(acc[0] > T(0)) || !finite_val(acc[0])) st->done = 4;
        }
    }
}

// ---------------------------------------------- CG: direction + SpMV + p^T A p
template <typename T, bool PC>
__global__ __launch_bounds__(kThreads) void k_cg_dir(OpView<T> op, const T *__restrict__ z,
                                                     const T *__restrict__ pold,
                                                     T *__restrict__ pnew, T *__restrict__ mu,
                                                     CgState<T> *st, T *partials,
                                                     unsigned *counter) {
    if (st->done) return;
    const int first = st->first;
    const T rz_new = st->rz_new;
    const T beta = first ? T(0) : rz_new / st->rz;
    int i, j;
    tile_ij(i, j);
    T acc[1] = {T(0)};
    if (i < op.nx && j < op.ny) {
        auto X = [&](int64_t q) -> T { return first ? z[q] : z[q] + beta * pold[q]; };
        column<T, PC>(op, i, j, X, [&](int, int64_t c, T pc, T ap) {
            pnew[c] = pc;
            mu[c] = ap;
            acc[0] += pc * ap;
        });
    }
    if (grid_reduce<T, 1>(acc, 0u, partials, counter)) {
        if (tid_lin() == 0) {
            const T pmu = acc[0];
            st->pmu = pmu;
            st->beta = beta;
            st->rz = rz_new;
            st->first = 0;
            if (!(pmu > T(0)) || !finite_val(pmu)) {
                st->done = 4;
                st->alpha = T(0);
            } else {
                st->alpha = rz_new / pmu;
            }
        }
    }
}

// ------------------------------------------------- CG: x += a p, r -= a mu, r^T r
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_update(int nx, int ny, int nz, T *__restrict__ x,
                                                        const T *__restrict__ p,
                                                        T *__restrict__ r,
                                                        const T *__restrict__ mu,
                                                        CgState<T> *st, T *partials,
                                                        unsigned *counter) {
    if (st->done) return;
    const T alpha = st->alpha;
    const bool fresh = (st->iter == 0);
    int i, j;
    tile_ij(i, j);
    T acc[1] = {T(0)};
    if (i < nx && j < ny) {
        const int64_t plane = (int64_t)nx * ny;
        int64_t c = i + (int64_t)nx * j;
        for (int l = 0; l < nz; ++l, c += plane) {
            const T xn = (fresh ? T(0) : x[c]) + alpha * p[c];
            const T rn = r[c] - alpha * mu[c];
            x[c] = xn;
            r[c] = rn;
            acc[0] += rn * rn;
        }
    }
    if (grid_reduce<T, 1>(acc, 0u, partials, counter)) {
        if (tid_lin() == 0) {
            const T rr = acc[0];
            st->rr = rr;
            st->iter = st->iter + 1;
            if (!finite_val(rr)) st->done = 4;
            else if (rr <= st->tol2) st->done = 1;
        }
    }
}

// ----------------------------- CG: true residual, drift and stagnation checks
template <typename T, bool PC>
__global__ __launch_bounds__(kThreads) void k_cg_check(OpView<T> op, const T *__restrict__ rhat,
                                                       const T *__restrict__ x,
                                                       const T *__restrict__ r, CgState<T> *st,
                                                       int force, T *partials,
                                                       unsigned *counter) {
    if (st->done && !force) return;
    const bool have_x = st->iter > 0;
    int i, j;
    tile_ij(i, j);
    T acc[2] = {T(0), T(0)};
    if (i < op.nx && j < op.ny) {
        auto X = [&](int64_t q) -> T { return have_x ? x[q] : T(0); };
        column<T, PC>(op, i, j, X, [&](int, int64_t c, T, T ax) {
            const T rt = rhat[c] - ax;
            const T d = rt - r[c];
            acc[0] += rt * rt;
            acc[1] += d * d;
        });
    }
    if (grid_reduce<T, 2>(acc, 0u, partials, counter)) {
        if (tid_lin() == 0) {
            st->true_rr = acc[0];
            st->drift_rr = acc[1];
            if (!force) {
                const T tn = sqrt(acc[0]);
                // switching criteria of Section 4.4: drift ||r_true - r_low|| >=
                // 0.5 ||r_true||, stagnation ||r_true^k|| > 0.9 ||r_true^{k-1}||
                if (!finite_val(tn)) st->done = 4;
                else if (sqrt(acc[1]) >= T(0.5) * tn) st->done = 2;
                else if (st->true_prev >= T(0) && tn > T(0.9) * st->true_prev) st->done = 3;
                st->true_prev = tn;
            }
        }
    }
}

// ------------------------------------------------------- FP64 outer residual
template <bool PC, typename TD, typename TI>
__global__ __launch_bounds__(kThreads) void k_residual(
    OpView<double> op, const double *__restrict__ th_in, double in_off,
    const TD *__restrict__ delta, const double *__restrict__ P, const double *__restrict__ Tn,
    double tn_off, double *__restrict__ th_out, double *__restrict__ r64, TI *__restrict__ r_in,
    TI *__restrict__ rhat, OuterStats *os, CgState<TI> *st, double inner_tol, double *partials,
    unsigned *counter) {
    int i, j;
    tile_ij(i, j);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < op.nx && j < op.ny) {
        auto X = [&](int64_t q) -> double {
            double v = th_in ? th_in[q] - in_off : 0.0;
            if (delta) v += (double)delta[q];
            return v;
        };
        column<double, PC>(op, i, j, X, [&](int l, int64_t c, double th, double ath) {
            double b = P[c];
            if (Tn) b += op.lc[l].cap * (Tn[c] - tn_off);
            const double rc = b - ath;
            if (th_out) th_out[c] = th;
            if (r64) r64[c] = rc;
            if (r_in) {
                const TI v = (TI)rc;
                r_in[c] = v;
                rhat[c] = v;
            }
            acc[0] += rc * rc;
            acc[1] += b * b;
            if (delta) acc[2] = fmax(acc[2], fabs((double)delta[c]));
            acc[3] = fmax(acc[3], fabs(th));
            acc[4] += isfinite(rc) ? 0.0 : 1.0;
        });
    }
    if (grid_reduce<double, 5>(acc, (1u << 2) | (1u << 3), partials, counter)) {
        if (tid_lin() == 0) {
            os->rr = acc[0];
            os->bb = acc[1];
            os->dinf = acc[2];
            os->thinf = acc[3];
            os->bad = acc[4];
            if (st) {
                const TI rr0 = (TI)acc[0];
                st->rr0 = rr0;
                st->rr = rr0;
                st->tol2 = (TI)(inner_tol * inner_tol * acc[0]);
                st->done = (acc[0] > 0.0 && acc[4] == 0.0) ? 0 : (acc[4] == 0.0 ? 1 : 4);
                st->iter = 0;
                st->first = 1;
                st->true_prev = TI(-1);
                st->true_rr = rr0;
                st->drift_rr = TI(0);
                st->rz = TI(0);
                st->rz_new = TI(0);
                st->alpha = TI(0);
                st->beta = TI(0);
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_add_scalar(int64_t n, const double *__restrict__ x,
                                                         double a, double *__restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + tid_lin(); q < n; q += stride)
        y[q] = x[q] + a;
}

__global__ __launch_bounds__(kThreads) void k_to_float(int64_t n, const double *__restrict__ x,
                                                       float *__restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + tid_lin(); q < n; q += stride)
        y[q] = (float)x[q];
}

// ------------------------------------------------------ coefficient build
__global__ __launch_bounds__(kThreads) void k_build_lateral(
    int nx, int ny, int nz, double dx, double dy, const double *__restrict__ dz,
    const double *__restrict__ k_lat, const double *__restrict__ mult, double *__restrict__ gx64,
    double *__restrict__ gy64, float *__restrict__ gx32, float *__restrict__ gy32,
    unsigned long long *maxrow, unsigned int *bad) {
    int i, j;
    tile_ij(i, j);
    if (i >= nx || j >= ny) return;
    const int64_t plane = (int64_t)nx * ny;
    int64_t c = i + (int64_t)nx * j;
    for (int l = 0; l < nz; ++l, c += plane) {
        const double kl = k_lat[l], d = dz[l];
        const double m = mult[c];
        if (!(m > 0.0) || !isfinite(m)) atomicAdd(bad, 1u);
        const double ka = kl * m;
        double gx = 0.0, gy = 0.0;
        // series half-cell conductance across the +x and +y faces
        if (i < nx - 1) gx = (dy * d) / (dx / (2.0 * ka) + dx / (2.0 * (kl * mult[c + 1])));
        if (j < ny - 1) gy = (dx * d) / (dy / (2.0 * ka) + dy / (2.0 * (kl * mult[c + nx])));
        gx64[c] = gx;
        gy64[c] = gy;
        gx32[c] = (float)gx;
        gy32[c] = (float)gy;
    }
}

// Per-layer max over cells of the lateral off-diagonal row sum, after the planes exist.
__global__ __launch_bounds__(kThreads) void k_lateral_rowmax(int nx, int ny, int nz,
                                                             const double *__restrict__ gx,
                                                             const double *__restrict__ gy,
                                                             unsigned long long *maxrow) {
    int i, j;
    tile_ij(i, j);
    const int t = tid_lin(), lane = t & 63;
    const bool act = (i < nx && j < ny);
    const int64_t plane = (int64_t)nx * ny;
    for (int l = 0; l < nz; ++l) {
        double s = 0.0;
        if (act) {
            const int64_t c = i + (int64_t)nx * j + plane * l;
            s = gx[c] + gy[c] + (i > 0 ? gx[c - 1] : 0.0) + (j > 0 ? gy[c - nx] : 0.0);
        }
        s = wave_max(s);
        if (lane == 0) atomicMax(&maxrow[l], (unsigned long long)__double_as_longlong(s));
    }
}

// --------------------------------------------------------------- Lanczos
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    // SplitMix64 (Steele, Lea, Flood 2014): counter-based, one output per index.
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ __launch_bounds__(kThreads) void k_fill_random(int64_t n, uint64_t seed,
                                                          float *__restrict__ v) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + tid_lin(); q < n; q += stride) {
        const uint64_t h = splitmix64(seed ^ (uint64_t)q * 0xD1B54A32D192ED03ull);
        // uniform in [-1, 1) from the top 24 bits
        v[q] = (float)((double)(h >> 40) * (2.0 / 16777216.0) - 1.0);
    }
}

__global__ __launch_bounds__(kThreads) void k_norm2(int64_t n, const float *__restrict__ v,
                                                    float *out, float *partials,
                                                    unsigned *counter) {
    float acc[1] = {0.f};
    const int64_t stride = (int64_t)gridDim.x * gridDim.y * kThreads;
    for (int64_t q = (int64_t)(blockIdx.x + gridDim.x * blockIdx.y) * kThreads + tid_lin(); q < n;
         q += stride)
        acc[0] += v[q] * v[q];
    if (grid_reduce<float, 1>(acc, 0u, partials, counter))
        if (tid_lin() == 0) *out = acc[0];
}

__global__ __launch_bounds__(kThreads) void k_scale_rsqrt(int64_t n, const float *__restrict__ v,
                                                          const float *nrm2,
                                                          float *__restrict__ out) {
    const float s = 1.0f / sqrtf(*nrm2);
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + tid_lin(); q < n; q += stride)
        out[q] = v[q] * s;
}

template <bool PC>
__global__ __launch_bounds__(kThreads) void k_lanczos_av(OpView<float> op,
                                                         const float *__restrict__ v,
                                                         const float *__restrict__ vprev,
                                                         const float *beta_prev,
                                                         float *__restrict__ w, float *alpha_out,
                                                         float *partials, unsigned *counter) {
    const float bp = beta_prev ? *beta_prev : 0.f;
    int i, j;
    tile_ij(i, j);
    float acc[1] = {0.f};
    if (i < op.nx && j < op.ny) {
        column<float, PC>(
            op, i, j, [&](int64_t q) { return v[q]; },
            [&](int, int64_t c, float vc, float av) {
                const float wc = vprev ? av - bp * vprev[c] : av;
                w[c] = wc;
                acc[0] += vc * wc;
            });
    }
    if (grid_reduce<float, 1>(acc, 0u, partials, counter))
        if (tid_lin() == 0) *alpha_out = acc[0];
}

__global__ __launch_bounds__(kThreads) void k_lanczos_orth(int64_t n, float *__restrict__ w,
                                                           const float *__restrict__ v,
                                                           const float *alpha, float *beta_out,
                                                           float *partials, unsigned *counter) {
    const float a = *alpha;
    float acc[1] = {0.f};
    const int64_t stride = (int64_t)gridDim.x * gridDim.y * kThreads;
    for (int64_t q = (int64_t)(blockIdx.x + gridDim.x * blockIdx.y) * kThreads + tid_lin(); q < n;
         q += stride) {
        const float wc = w[q] - a * v[q];
        w[q] = wc;
        acc[0] += wc * wc;
    }
    if (grid_reduce<float, 1>(acc, 0u, partials, counter))
        if (tid_lin() == 0) *beta_out = sqrtf(acc[0]);
}

__global__ __launch_bounds__(kThreads) void k_div_scalar(int64_t n, float *__restrict__ w,
                                                         const float *den) {
    const float s = 1.0f / *den;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + tid_lin(); q < n; q += stride) w[q] *= s;
}

// --------------------------------------------------------------- adjoint
// Per-layer sums with one partial per workgroup and layer; the last workgroup
// reduces each layer's partials in a fixed order.
template <bool PC>
__global__ __launch_bounds__(kThreads) void k_adjoint_sums(OpView<double> op,
                                                           const double *__restrict__ lam,
                                                           const double *__restrict__ T,
                                                           double t_amb, double *out,
                                                           double *partials, unsigned *counter) {
    constexpr int NW = kThreads / 64;
    __shared__ double sh[NW][2 * kMaxLayers];
    __shared__ int is_last;
    int i, j;
    tile_ij(i, j);
    const int t = tid_lin(), lane = t & 63, w = t >> 6;
    const int nb = gridDim.x * gridDim.y, b = blockIdx.x + gridDim.x * blockIdx.y;
    const bool act = (i < op.nx && j < op.ny);
    const int nz = op.nz, nx = op.nx, ny = op.ny;
    const int64_t plane = (int64_t)nx * ny;
    int64_t c = i + (int64_t)nx * j;
    for (int l = 0; l < nz; ++l, c += plane) {
        const LayerCoef<double> L = op.lc[l];
        double slat = 0.0, svert = 0.0;
        if (act) {
            const double la = lam[c], th = T[c] - t_amb;
            if (i < nx - 1) {
                const double g = PC ? op.gx[c] : L.gx;
                slat += g * (la - lam[c + 1]) * (th - (T[c + 1] - t_amb));
            }
            if (j < ny - 1) {
                const double g = PC ? op.gy[c] : L.gy;
                slat += g * (la - lam[c + nx]) * (th - (T[c + nx] - t_amb));
            }
            if (l < nz - 1) svert = (la - lam[c + plane]) * (th - (T[c + plane] - t_amb));
        }
        slat = wave_sum(slat);
        svert = wave_sum(svert);
        if (lane == 0) {
            sh[w][l] = slat;
            sh[w][kMaxLayers + l] = svert;
        }
    }
    __syncthreads();
    if (t == 0) {
        for (int l = 0; l < nz; ++l) {
            double a = 0.0, v = 0.0;
            for (int q = 0; q < NW; ++q) {
                a += sh[q][l];
                v += sh[q][kMaxLayers + l];
            }
            partials[(size_t)l * nb + b] = a;
            partials[(size_t)(nz + l) * nb + b] = v;
        }
        __threadfence();
        const unsigned ticket = atomicAdd(counter, 1u);
        is_last = (ticket == (unsigned)(nb - 1));
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    for (int k = 0; k < 2 * nz; ++k) {
        double a = 0.0;
        for (int q = t; q < nb; q += kThreads) a += load_coherent(&partials[(size_t)k * nb + q]);
        a = wave_sum(a);
        __syncthreads();
        if (lane == 0) sh[w][0] = a;
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int q = 0; q < NW; ++q) s += sh[q][0];
            out[k] = s;
        }
    }
    if (t == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_adjoint_finish(int nz, const double *__restrict__ sums,
                                 const double *__restrict__ fac_lat,
                                 const double *__restrict__ fac_up,
                                 const double *__restrict__ fac_dn, double *__restrict__ dk) {
    const int l = threadIdx.x;
    if (l >= nz) return;
    dk[l] = -fac_lat[l] * sums[l];
    double v = 0.0;
    if (l < nz - 1) v += fac_up[l] * sums[nz + l];
    if (l > 0) v += fac_dn[l] * sums[nz + l - 1];
    dk[nz + l] = -v;
}

inline unsigned blocks_1d(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

// =================================================================== launchers
template <typename T>
void launch_apply(const OpView<T> &op, const T *x, T *y, hipStream_t s) {
    const dim3 g = tile_grid(op.nx, op.ny), b(kBX, kBY);
    if (op.gx) hipLaunchKernelGGL((k_apply<T, true>), g, b, 0, s, op, x, y);
    else hipLaunchKernelGGL((k_apply<T, false>), g, b, 0, s, op, x, y);
}

template <typename T, bool PC>
static void cheb_dispatch(const OpView<T> &op, int mode, bool last, const T *z, T *zo, const T *r,
                          T c1, T c2, T inv_th, CgState<T> *st, RedScratch red, hipStream_t s) {
    const dim3 g = tile_grid(op.nx, op.ny), b(kBX, kBY);
    T *pp = (T *)red.partials;
#define CUTH_CHEB(M, LST)                                                                       \
    hipLaunchKernelGGL((k_cheb<T, PC, M, LST>), g, b, 0, s, op, z, zo, r, c1, c2, inv_th, st, pp, \
                       red.counter)
    if (mode == 0) {
        if (last) CUTH_CHEB(0, true); else CUTH_CHEB(0, false);
    } else if (mode == 1) {
        if (last) CUTH_CHEB(1, true); else CUTH_CHEB(1, false);
    } else {
        if (last) CUTH_CHEB(2, true); else CUTH_CHEB(2, false);
    }
#undef CUTH_CHEB
}

template <typename T>
void launch_cheb(const OpView<T> &op, int mode, bool last, const T *z, T *zo, const T *r, T c1,
                 T c2, T inv_th, CgState<T> *st, RedScratch red, hipStream_t s) {
    if (op.gx) cheb_dispatch<T, true>(op, mode, last, z, zo, r, c1, c2, inv_th, st, red, s);
    else cheb_dispatch<T, false>(op, mode, last, z, zo, r, c1, c2, inv_th, st, red, s);
}

template <typename T>
void launch_scale(int64_t n, const T *x, T a, T *y, CgState<T> *st, bool, const T *,
                  RedScratch red, hipStream_t s) {
    hipLaunchKernelGGL((k_scale_dot<T>), dim3(blocks_1d(n)), dim3(kBX, kBY), 0, s, n, x, a, y, st,
                       (T *)red.partials, red.counter);
}

template <typename T>
void launch_cg_dir(const OpView<T> &op, const T *z, const T *pold, T *pnew, T *mu, CgState<T> *st,
                   RedScratch red, hipStream_t s) {
    const dim3 g = tile_grid(op.nx, op.ny), b(kBX, kBY);
    if (op.gx)
        hipLaunchKernelGGL((k_cg_dir<T, true>), g, b, 0, s, op, z, pold, pnew, mu, st,
                           (T *)red.partials, red.counter);
    else
        hipLaunchKernelGGL((k_cg_dir<T, false>), g, b, 0, s, op, z, pold, pnew, mu, st,
                           (T *)red.partials, red.counter);
}

template <typename T>
void launch_cg_update(const OpView<T> &op, T *x, const T *p, T *r, const T *mu, CgState<T> *st,
                      RedScratch red, hipStream_t s) {
    const dim3 g = tile_grid(op.nx, op.ny), b(kBX, kBY);
    hipLaunchKernelGGL((k_cg_update<T>), g, b, 0, s, op.nx, op.ny, op.nz, x, p, r, mu, st,
                       (T *)red.partials, red.counter);
}

template <typename T>
void launch_cg_check(const OpView<T> &op, const T *rhat, const T *x, const T *r, CgState<T> *st,
                     int force, RedScratch red, hipStream_t s) {
    const dim3 g = tile_grid(op.nx, op.ny), b(kBX, kBY);
    if (op.gx)
        hipLaunchKernelGGL((k_cg_check<T, true>), g, b, 0, s, op, rhat, x, r, st, force,
                           (T *)red.partials, red.counter);
    else
        hipLaunchKernelGGL((k_cg_check<T, false>), g, b, 0, s, op, rhat, x, r, st, force,
                           (T *)red.partials, red.counter);
}

template <typename TD, typename TI>
void launch_residual(const OpView<double> &op, const double *th_in, double in_off, const TD *delta,
                     const double *P, const double *Tn, double tn_off, double *th_out,
                     double *r64, TI *r_in, TI *rhat, OuterStats *os, CgState<TI> *st,
                     double inner_tol, RedScratch red, hipStream_t s) {
    const dim3 g = tile_grid(op.nx, op.ny), b(kBX, kBY);
    if (op.gx)
        hipLaunchKernelGGL((k_residual<true, TD, TI>), g, b, 0, s, op, th_in, in_off, delta, P, Tn,
                           tn_off, th_out, r64, r_in, rhat, os, st, inner_tol,
                           (double *)red.partials, red.counter);
    else
        hipLaunchKernelGGL((k_residual<false, TD, TI>), g, b, 0, s, op, th_in, in_off, delta, P,
                           Tn, tn_off, th_out, r64, r_in, rhat, os, st, inner_tol,
                           (double *)red.partials, red.counter);
}

void launch_add_scalar(int64_t n, const double *x, double a, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_add_scalar, dim3(blocks_1d(n)), dim3(kBX, kBY), 0, s, n, x, a, y);
}

void launch_copy_to_float(int64_t n, const double *x, float *y, hipStream_t s) {
    hipLaunchKernelGGL(k_to_float, dim3(blocks_1d(n)), dim3(kBX, kBY), 0, s, n, x, y);
}

void launch_build_lateral(int nx, int ny, int nz, double dx, double dy, const double *dz,
                          const double *k_lat, const double *mult, double *gx64, double *gy64,
                          float *gx32, float *gy32, unsigned long long *maxrow, unsigned int *bad,
                          hipStream_t s) {
    const dim3 g = tile_grid(nx, ny), b(kBX, kBY);
    hipLaunchKernelGGL(k_build_lateral, g, b, 0, s, nx, ny, nz, dx, dy, dz, k_lat, mult, gx64,
                       gy64, gx32, gy32, maxrow, bad);
    hipLaunchKernelGGL(k_lateral_rowmax, g, b, 0, s, nx, ny, nz, (const double *)gx64,
                       (const double *)gy64, maxrow);
}

void launch_fill_random(int64_t n, uint64_t seed, float *v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_random, dim3(blocks_1d(n)), dim3(kBX, kBY), 0, s, n, seed, v);
}

void launch_norm2(int64_t n, const float *v, float *out, RedScratch red, hipStream_t s) {
    hipLaunchKernelGGL(k_norm2, dim3(blocks_1d(n)), dim3(kBX, kBY), 0, s, n, v, out,
                       (float *)red.partials, red.counter);
}

void launch_scale_by_rsqrt(int64_t n, const float *v, const float *nrm2, float *out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_scale_rsqrt, dim3(blocks_1d(n)), dim3(kBX, kBY), 0, s, n, v, nrm2, out);
}

void launch_lanczos_av(const OpView<float> &op, const float *v, const float *vprev,
                       const float *beta_prev, float *w, float *alpha_out, RedScratch red,
                       hipStream_t s) {
    const dim3 g = tile_grid(op.nx, op.ny), b(kBX, kBY);
    if (op.gx)
        hipLaunchKernelGGL((k_lanczos_av<true>), g, b, 0, s, op, v, vprev, beta_prev, w,
                           alpha_out, (float *)red.partials, red.counter);
    else
        hipLaunchKernelGGL((k_lanczos_av<false>), g, b, 0, s, op, v, vprev, beta_prev, w,
                           alpha_out, (float *)red.partials, red.counter);
}

void launch_lanczos_orth(int64_t n, float *w, const float *v, const float *alpha,
                         float *beta_out, RedScratch red, hipStream_t s) {
    hipLaunchKernelGGL(k_lanczos_orth, dim3(blocks_1d(n)), dim3(kBX, kBY), 0, s, n, w, v, alpha,
                       beta_out, (float *)red.partials, red.counter);
}

void launch_div_scalar(int64_t n, float *w, const float *den, hipStream_t s) {
    hipLaunchKernelGGL(k_div_scalar, dim3(blocks_1d(n)), dim3(kBX, kBY), 0, s, n, w, den);
}

void launch_adjoint_sums(const OpView<double> &op, const double *lam, const double *T,
                         double t_amb, double *out, RedScratch red, hipStream_t s) {
    const dim3 g = tile_grid(op.nx, op.ny), b(kBX, kBY);
    if (op.gx)
        hipLaunchKernelGGL((k_adjoint_sums<true>), g, b, 0, s, op, lam, T, t_amb, out,
                           (double *)red.partials, red.counter);
    else
        hipLaunchKernelGGL((k_adjoint_sums<false>), g, b, 0, s, op, lam, T, t_amb, out,
                           (double *)red.partials, red.counter);
}

void launch_adjoint_finish(int nz, const double *sums, const double *fac_lat,
                           const double *fac_vert_up, const double *fac_vert_dn, double *dL_dk,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_adjoint_finish, dim3(1), dim3(kMaxLayers), 0, s, nz, sums, fac_lat,
                       fac_vert_up, fac_vert_dn, dL_dk);
}

// explicit instantiations
template void launch_apply<float>(const OpView<float> &, const float *, float *, hipStream_t);
template void launch_apply<double>(const OpView<double> &, const double *, double *, hipStream_t);
template void launch_cheb<float>(const OpView<float> &, int, bool, const float *, float *,
                                 const float *, float, float, float, CgState<float> *, RedScratch,
                                 hipStream_t);
template void launch_cheb<double>(const OpView<double> &, int, bool, const double *, double *,
                                  const double *, double, double, double, CgState<double> *,
                                  RedScratch, hipStream_t);
template void launch_scale<float>(int64_t, const float *, float, float *, CgState<float> *, bool,
                                  const float *, RedScratch, hipStream_t);
template void launch_scale<double>(int64_t, const double *, double, double *, CgState<double> *,
                                   bool, const double *, RedScratch, hipStream_t);
template void launch_cg_dir<float>(const OpView<float> &, const float *, const float *, float *,
                                   float *, CgState<float> *, RedScratch, hipStream_t);
template void launch_cg_dir<double>(const OpView<double> &, const double *, const double *,
                                    double *, double *, CgState<double> *, RedScratch, hipStream_t);
template void launch_cg_update<float>(const OpView<float> &, float *, const float *, float *,
                                      const float *, CgState<float> *, RedScratch, hipStream_t);
template void launch_cg_update<double>(const OpView<double> &, double *, const double *, double *,
                                       const double *, CgState<double> *, RedScratch, hipStream_t);
template void launch_cg_check<float>(const OpView<float> &, const float *, const float *,
                                     const float *, CgState<float> *, int, RedScratch, hipStream_t);
template void launch_cg_check<double>(const OpView<double> &, const double *, const double *,
                                      const double *, CgState<double> *, int, RedScratch,
                                      hipStream_t);
template void launch_residual<float, float>(const OpView<double> &, const double *, double,
                                            const float *, const double *, const double *, double,
                                            double *, double *, float *, float *, OuterStats *,
                                            CgState<float> *, double, RedScratch, hipStream_t);
template void launch_residual<double, double>(const OpView<double> &, const double *, double,
                                              const double *, const double *, const double *,
                                              double, double *, double *, double *, double *,
                                              OuterStats *, CgState<double> *, double, RedScratch,
                                              hipStream_t);

}  // namespace cuth
