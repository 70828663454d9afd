// Host orchestration of the solve path: grid setup, Lanczos spectral bounds,
// the Chebyshev-preconditioned CG (Algorithm 1 + the Chebyshev algorithm of
// Section 4.3) and FP64 iterative refinement around an FP32 inner solve.
//
// Everything numeric on vectors runs in the kernels of kernels.hip.  The host
// enqueues launches, reads back scalars and per-workgroup partials once per
// chunk of CG iterations or refinement cycle, and decides what to launch next.
// Solves of several systems and right-hand sides advance together: each launch
// covers every active problem (a single solve is a set of one).
#include "grid.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <sstream>

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

// Accumulate the durations of the recorded blocks of sweep launches (stream
// already synced).  Blocks recorded in CG iterations at or after `valid_below`
// ran after the device-side stop and did no work; they are dropped.
Status prof_flush(Grid &g, int valid_below) {
    for (size_t i = 0; i + 1 < g.pev_used; i += 2) {
        float ms = 0.f;
        if (g.pev_tag.size() > i / 2 && g.pev_tag[i / 2] >= valid_below) continue;
        if (hipEventElapsedTime(&ms, g.pev[i], g.pev[i + 1]) == hipSuccess) {
            g.prof_ms += ms;
            g.prof_count += g.pev_cnt.size() > i / 2 ? g.pev_cnt[i / 2] : 1;
        }
    }
    g.pev_used = 0;
    return Status::ok();
}

namespace {

constexpr int P_CHEB = 0, P_DIR = 1, P_UPD = 2, P_CHK = 3, P_RES = 4, P_RED = 5, P_SLOTS = 6;

// Above this many workgroups per problem, the sums the CG kernels need are
// formed once per problem by a reduce launch (the direct way has every
// workgroup of the consumer read every partial: quadratic in the workgroups).
// A batch pays one reduce launch for all its problems, and lower: at 1024 the
// 64-stack batch (150-1500 workgroups per problem) solves 3 % faster than at
// 4096 (2.53 against 2.60 s), and no faster at 256.  CUTH_REDUCE_ABOVE
// overrides both thresholds (read at every inner solve).
int reduce_above(int nprob) {
    const char *e = std::getenv("CUTH_REDUCE_ABOVE");
    return e ? std::atoi(e) : (nprob > 1 ? 1024 : 4096);
}

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
Status host_alloc(P **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipHostMalloc((void **)p, sizeof(P) * count, hipHostMallocDefault) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return Status::err(CUTH_E_NOMEM, "hipHostMalloc failed");
    }
    return Status::ok();
}

template <typename P>
void dev_free(P *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

template <typename P>
void host_free(P *&p) {
    if (p) (void)hipHostFree((void *)p);
    p = nullptr;
}

Status sync_stream(hipStream_t s) {
    CUTH_HIP(hipStreamSynchronize(s));
    return Status::ok();
}

template <typename T>
Status alloc_work(Work<T> &w, int64_t N, bool extra_z = false) {
    if (!w.ready()) {
        T **ps[] = {&w.x, &w.r, &w.rhat, &w.pA, &w.pB, &w.mu, &w.zA, &w.zB};
        for (T **p : ps) CUTH_TRY(dev_alloc(p, (size_t)N));
    }
    if (extra_z && !w.zC) {
        CUTH_TRY(dev_alloc(&w.zC, (size_t)N));
        CUTH_TRY(dev_alloc(&w.zD, (size_t)N));
    }
    return Status::ok();
}

template <typename T>
void free_work(Work<T> &w) {
    T **ps[] = {&w.x, &w.r, &w.rhat, &w.pA, &w.pB, &w.mu, &w.zA, &w.zB, &w.zC, &w.zD};
    for (T **p : ps) dev_free(*p);
}

// CUTH_LOG=1: one line per refinement cycle on stderr.
bool log_on() {
    static const bool on = [] {
        const char *e = std::getenv("CUTH_LOG");
        return e && e[0] == '1';
    }();
    return on;
}

// CUTH_GRAPH=0/1 overrides whether chunks of CG iterations are captured into
// HIP graphs and replayed (default: batches, and single solves of grids up to
// kGraphMaxN unknowns, whose kernels are shorter than a launch from the host).
int graph_env() {
    const char *e = std::getenv("CUTH_GRAPH");
    return e ? (e[0] == '1' ? 1 : 0) : -1;
}
constexpr int64_t kGraphMaxN = int64_t(1) << 21;

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

// Sweep fusion of a shape: 3 fused triples (and pairs for what is left), 2
// fused pairs, 0 single sweeps only.
inline int fuse_level(const Shape &sh) { return sh.tr > 0 && sh.fr > 0 ? 3 : sh.fr > 0 ? 2 : 0; }

// The fusion level the preconditioner runs at in precision T (fused launches
// are FP32 only).
template <typename T>
int fuse_for(const Shape &sh, int pm) {
    (void)pm;
    return sizeof(T) == 4 ? fuse_level(sh) : 0;
}

// Number of sweeps the launch at sweep j of a degree-k preconditioner covers
// at fusion level `fuse`: fused launches end before the last sweep, which
// also forms the r^T z partials; triples start at j = 2 (forming the implicit
// z_1 = r / theta of the plain polynomial themselves), pairs at j = 3; sweep 1
// (implicit z_0 = 0, the convergence test) is always single.
inline int sweep_width(int j, int k, int fuse) {
    if (j < 2) return 1;
    if (fuse >= 3 && j + 2 < k - 1) return 3;
    if (j < 3) return 1;
    if (fuse >= 2 && j + 1 < k - 1) return 2;
    return 1;
}

// Algorithmic bytes per unknown of each kernel (what the method must move).
template <typename T>
struct Bytes {
    double coef;     // per-cell lateral conductances read by one CG stencil pass
    double coef_sw;  // ... by one Chebyshev sweep (FP16-stored: 2 x 2 B)
    explicit Bytes(bool per_cell, bool h16 = false)
        : coef(per_cell ? 2.0 * sizeof(T) : 0.0),
          coef_sw(per_cell ? (h16 ? 4.0 : 2.0 * sizeof(T)) : 0.0) {}
    double cheb(int mode) const { return (mode == 1 ? 2 : mode == 2 ? 3 : 4) * sizeof(T) + coef_sw; }
    double dir() const { return 4.0 * sizeof(T) + coef; }
    double update() const { return 6.0 * sizeof(T); }
    double check() const { return 3.0 * sizeof(T) + coef; }
    double scale() const { return 2.0 * sizeof(T); }
    // a fused pair of general sweeps: z_j, z_{j-1}, r (+ conductances) read once,
    // z_{j+1} and z_{j+2} written
    double pair() const { return 5.0 * sizeof(T) + coef_sw; }
    // a fused triple moves the same: z_{j+1} stays on chip, z_{j+2} and
    // z_{j+3} are written
    double triple() const { return pair(); }
    double precond(int k, int pm = 0, int fuse = 0) const {
        if (pm == 1) return scale() + coef;   // Jacobi: also the lateral conductances
        if (pm == 2 || (k == 1 && pm == 0)) return scale();
        // Jacobi-scaled Chebyshev: the scale pass (r and the conductances read,
        // z_1 written), then a sweep that reads z_1 and r, then general sweeps
        const bool jac = pm == 3;
        if (jac && k == 1) return scale() + coef;
        double b = jac ? scale() + coef + cheb(2) : cheb(1);
        for (int j = 2; j < k;) {
            const int wd = sweep_width(j, k, fuse);
            // at j = 2 the plain polynomial's z_1 is formed from r, not read
            const double m2 = j == 2 && !jac ? sizeof(T) : 0.0;
            b += wd == 3 ? triple() - m2 : wd == 2 ? pair() : cheb(j == 2 && !jac ? 2 : 0);
            j += wd;
        }
        return b;
    }
};

// One system and right-hand side of a solve, with its progress.
struct Problem {
    Grid *g = nullptr;
    Setup *su = nullptr;
    ChebConsts cc;
    const double *P = nullptr, *Tn = nullptr, *init = nullptr;
    double init_off = 0.0;
    double *out = nullptr;
    double out_off = 0.0;
    Work<float> w32;
    Work<double> w64;
    double *thA = nullptr, *thB = nullptr;
    double tol = 0.0;
    // progress of the refinement
    bool finished = false;
    const double *th_in = nullptr;
    double in_off = 0.0;
    bool have_delta = false;
    double *th_out = nullptr, *th_final = nullptr;
    double last_red = 1.0, d_prev = 1.0, est = 1.0, prev_relres = INFINITY;
    // mixed refinement: the previous inner solve's residual reduction, and
    // the largest measured ratio of error contraction to residual reduction
    double red_prev = 1.0, lag = 1.0;
    // mixed refinement: an inner solve has ended on the stagnation test, i.e.
    // at the FP32 floor of this system
    bool floor32 = false;
    // FP64 and stage-switched solves: a relative residual accepted when the
    // true residual stops falling above tol (0: none; the default transient
    // tolerance, which a stiff step cannot always reach in FP64)
    double tol_relax = 0.0;
    // the Chebyshev sweeps read the FP16-stored lateral conductances
    bool h16 = false;
    // preconditioner: 0 Chebyshev, 1 Jacobi, 2 none (cuth_options.preconditioner)
    int pm = 0;
    // stage-switched scheme: still in the early stage (FP32-stored coefficients
    // in the CG product, switch test (a) as the inner tolerance)
    bool early = false;
    // fixed-FP32 ablation baseline: one FP32 inner solve to tol on its own
    // recursive residual, no drift or stagnation stop, no refinement
    bool fixed32 = false;
    // FP64 products from the CSR copy of the operator (Ablation I's storage)
    bool csr = false;
    // per inner solve
    bool inner = false;
    double rr0 = 0.0, tol2 = 0.0, true_prev = -1.0, low_prev = -1.0, true_rr = 0.0;
    int stop = 0;
    // results
    int cycles = 0, cg_iters = 0, reason = 0, drift_stops = 0, stag_stops = 0;
    int64_t stencils = 0;
    double bytes = 0.0, relres = 0.0, err_est = 0.0;
    Status status;
    // slots of the current launches
    int tile0 = 0, ntiles = 0;
    // interval of the preconditioner's operator (A, or D^{-1} A when scaled)
    double ilo = 0.0, ihi = 0.0;
};

// The two Chebyshev preconditioners (the paper's, and the Jacobi-scaled one).
inline bool is_cheb(int pm) { return pm == CUTH_PC_CHEBYSHEV || pm == CUTH_PC_CHEBYSHEV_JACOBI; }

// Interval of the operator the preconditioner's polynomial acts on (bounds
// already computed).
inline void pc_interval(const Setup &su, int pm, double &lo, double &hi) {
    lo = pm == CUTH_PC_CHEBYSHEV_JACOBI ? su.jlmin : su.lmin;
    hi = pm == CUTH_PC_CHEBYSHEV_JACOBI ? su.jlmax : su.lmax;
}

template <typename T> struct Sel;
template <> struct Sel<float> {
    static InnerProb<float> *d(Engine &E) { return E.in32; }
    static InnerProb<float> *h(Engine &E) { return E.h_in32; }
    static CgState<float> *ds(Engine &E) { return E.st32; }
    static CgState<float> *hs(Engine &E) { return E.h_st32; }
    static float *dc(Engine &E) { return E.cheb32; }
    static float *hc(Engine &E) { return E.h_cheb32; }
    static Work<float> &w(Problem &p) { return p.w32; }
    static OpView<float> view(const Problem &p, const Shape &sh) {
        const Grid &g = *p.g;
        OpView<float> v{g.nx, g.ny, g.nz, g.per_cell ? g.gx32 : nullptr,
                        g.per_cell ? g.gy32 : nullptr, p.su->lc32, sh.vx, sh.by, sh.zc};
        if (p.h16 && g.per_cell) {
            v.hx = g.hx;
            v.hy = g.hy;
        }
        return v;
    }
};
template <> struct Sel<double> {
    static InnerProb<double> *d(Engine &E) { return E.in64; }
    static InnerProb<double> *h(Engine &E) { return E.h_in64; }
    static CgState<double> *ds(Engine &E) { return E.st64; }
    static CgState<double> *hs(Engine &E) { return E.h_st64; }
    static double *dc(Engine &E) { return E.cheb64; }
    static double *hc(Engine &E) { return E.h_cheb64; }
    static Work<double> &w(Problem &p) { return p.w64; }
    static OpView<double> view(const Problem &p, const Shape &sh) {
        const Grid &g = *p.g;
        OpView<double> v{g.nx, g.ny, g.nz, g.per_cell ? g.gx64 : nullptr,
                         g.per_cell ? g.gy64 : nullptr, p.su->lc64, sh.vx, sh.by, sh.zc};
        if (p.csr) {
            v.csr_ptr = p.su->csr_ptr;
            v.csr_col = p.su->csr_col;
            v.csr_val = p.su->csr_val;
        }
        return v;
    }
};

OpView<double> outer_view(const Problem &p, const Shape &sh) {
    return Sel<double>::view(p, sh);
}

int prob_tiles(const Grid &g, const Shape &sh) {
    return tiles_x(g.nx, sh.vx) * tiles_y(g.ny, sh.by) * tiles_z(g.nz, sh.zc);
}

}  // namespace

// ------------------------------------------------------------------ engine
Status engine_alloc(Engine &E, int cap, int kcap, size_t nb_max) {
    E.cap = cap;
    E.kcap = kcap;
    // the reduce slot holds three sums per problem (red_rz, red_pmu, red_rr)
    // and then the outer residual's totals (outer_totals)
    E.slot_doubles = std::max<size_t>(8 * std::max<size_t>(nb_max, 1), (size_t)(3 + kResidualValues) * cap);
    const size_t nc = (size_t)cap * (1 + 2 * kcap);
    CUTH_TRY(dev_alloc(&E.in32, cap));
    CUTH_TRY(dev_alloc(&E.in64, cap));
    CUTH_TRY(dev_alloc(&E.out32, cap));
    CUTH_TRY(dev_alloc(&E.out64, cap));
    CUTH_TRY(dev_alloc(&E.st32, cap));
    CUTH_TRY(dev_alloc(&E.st64, cap));
    CUTH_TRY(dev_alloc(&E.cheb32, nc));
    CUTH_TRY(dev_alloc(&E.cheb64, nc));
    CUTH_TRY(dev_alloc(&E.part, E.slot_doubles * P_SLOTS));
    CUTH_TRY(host_alloc(&E.h_in32, cap));
    CUTH_TRY(host_alloc(&E.h_in64, cap));
    CUTH_TRY(host_alloc(&E.h_out32, cap));
    CUTH_TRY(host_alloc(&E.h_out64, cap));
    CUTH_TRY(host_alloc(&E.h_st32, cap));
    CUTH_TRY(host_alloc(&E.h_st64, cap));
    CUTH_TRY(host_alloc(&E.h_cheb32, nc));
    CUTH_TRY(host_alloc(&E.h_cheb64, nc));
    CUTH_TRY(host_alloc(&E.h_part, E.slot_doubles));
    CUTH_HIP(hipStreamCreateWithFlags(&E.own, hipStreamNonBlocking));
    CUTH_HIP(hipEventCreateWithFlags(&E.ev_in, hipEventDisableTiming));
    CUTH_HIP(hipEventCreateWithFlags(&E.ev_out, hipEventDisableTiming));
    return Status::ok();
}

void engine_free(Engine &E) {
    if (E.own) (void)hipStreamSynchronize(E.own);
    for (auto &g : E.graphs) (void)hipGraphExecDestroy(g.second);
    E.graphs.clear();
    dev_free(E.in32);
    dev_free(E.in64);
    dev_free(E.out32);
    dev_free(E.out64);
    dev_free(E.st32);
    dev_free(E.st64);
    dev_free(E.cheb32);
    dev_free(E.cheb64);
    dev_free(E.part);
    host_free(E.h_in32);
    host_free(E.h_in64);
    host_free(E.h_out32);
    host_free(E.h_out64);
    host_free(E.h_st32);
    host_free(E.h_st64);
    host_free(E.h_cheb32);
    host_free(E.h_cheb64);
    host_free(E.h_part);
    if (E.ev_in) (void)hipEventDestroy(E.ev_in);
    if (E.ev_out) (void)hipEventDestroy(E.ev_out);
    if (E.own) (void)hipStreamDestroy(E.own);
    E = Engine();
}

namespace {

template <typename T>
T *eslot(Engine &E, int s) {
    return reinterpret_cast<T *>(E.part + (size_t)s * E.slot_doubles);
}

// Upload the Chebyshev constants of every problem (slot i of the set).
template <typename T>
Status upload_cheb(Engine &E, std::vector<Problem *> &ps, hipStream_t s) {
    const int stride = 1 + 2 * E.kcap;
    T *h = Sel<T>::hc(E);
    for (size_t i = 0; i < ps.size(); ++i) {
        const ChebConsts &cc = ps[i]->cc;
        T *c = h + i * stride;
        std::fill(c, c + stride, T(0));
        c[0] = (T)cc.inv_th;
        for (int j = 1; j < cc.k; ++j) {
            c[1 + j] = (T)cc.c1[j];
            c[1 + E.kcap + j] = (T)cc.c2[j];
        }
    }
    CUTH_HIP(hipMemcpyAsync(Sel<T>::dc(E), h, sizeof(T) * stride * ps.size(),
                            hipMemcpyHostToDevice, s));
    return Status::ok();
}

// Inner descriptors for the problems with p->inner set; cheb row = slot index in ps.
template <typename T>
int build_inner(Engine &E, std::vector<Problem *> &ps, const Shape &sh, std::vector<int> &which) {
    InnerProb<T> *h = Sel<T>::h(E);
    int tile = 0, ftile = 0, ttile = 0, n = 0;
    which.clear();
    for (size_t i = 0; i < ps.size(); ++i) {
        Problem &p = *ps[i];
        if (!p.inner) continue;
        Work<T> &w = Sel<T>::w(p);
        // every vector a kernel of this precision touches must exist
        if (!w.x || !w.r || !w.rhat || !w.mu || !w.pA || !w.pB || !w.zA || !w.zB) return -1;
        InnerProb<T> d;
        d.op = Sel<T>::view(p, sh);
        d.ntx = tiles_x(p.g->nx, sh.vx);
        d.ntz = tiles_z(p.g->nz, sh.zc);
        d.tile0 = tile;
        d.ntiles = prob_tiles(*p.g, sh);
        d.x = w.x;
        d.r = w.r;
        d.rhat = w.rhat;
        d.mu = w.mu;
        d.p[0] = w.pA;
        d.p[1] = w.pB;
        d.z[0] = w.zA;
        d.z[1] = w.zB;
        d.z[2] = w.zC;
        d.z[3] = w.zD;
        d.f_tile0 = d.f_ntiles = 0;
        d.t_tile0 = d.t_ntiles = 0;
        if (sh.fr > 0) {
            if (!w.zC || !w.zD) return -1;
            d.f_tile0 = ftile;
            d.f_ntiles = fused_windows(p.g->nx, sh.vx, sh.fwpr, 2) * tiles_y(p.g->ny, sh.fr) *
                         tiles_z(p.g->nz, sh.fzc);
            ftile += d.f_ntiles;
        }
        if (sh.tr > 0) {
            d.t_tile0 = ttile;
            d.t_ntiles = fused_windows(p.g->nx, sh.vx, sh.twpr, 3) * tiles_y(p.g->ny, sh.tr) *
                         tiles_z(p.g->nz, sh.tzc);
            ttile += d.t_ntiles;
        }
        d.st = Sel<T>::ds(E) + n;
        d.cheb = Sel<T>::dc(E) + i * (1 + 2 * E.kcap);
        d.kcap = E.kcap;
        d.pad = 0;
        h[n] = d;
        p.tile0 = tile;
        p.ntiles = d.ntiles;
        tile += d.ntiles;
        which.push_back((int)i);
        ++n;
    }
    // the check kernel writes two partials per workgroup into one slot
    if ((size_t)tile * 2 > E.slot_doubles) return -1;
    return tile;
}

// Packed buffer selection of a sweep: z_j in z[in], result over z[out].
inline int zsel(int in, int out) { return in + 4 * out; }

// The two of the four z buffers that are neither n nor p.
inline void free_pair(int n, int p, int &x, int &y) {
    x = y = -1;
    for (int b = 0; b < 4; ++b)
        if (b != n && b != p) {
            if (x < 0) x = b;
            else y = b;
        }
}

// Buffer that holds z = q(A) r after enqueue_precond (same rotation): mode 1
// writes z[1]; every single sweep writes over the older of (newest, older);
// a fused pair or triple writes the two other buffers.
int precond_final(int k, int pm, int fuse) {
    if (k == 1 || pm == 1 || pm == 2) return 0;
    if (k == 2) return 1;
    int n = 1, p = 0;   // after mode 1
    for (int j = 2; j < k;) {
        const int wd = sweep_width(j, k, fuse);
        if (wd > 1) {
            int x, y;
            free_pair(n, p, x, y);
            p = x;
            n = y;
        } else {
            std::swap(n, p);
        }
        j += wd;
    }
    return n;
}

// Per-problem sums written by launch_reduce_b (red mode): r^T z, p^T A p, r^T r.
template <typename T>
T *red_rz(Engine &E) { return eslot<T>(E, P_RED); }
template <typename T>
T *red_pmu(Engine &E) { return eslot<T>(E, P_RED) + E.cap; }
template <typename T>
T *red_rr(Engine &E) { return eslot<T>(E, P_RED) + 2 * E.cap; }
// per-problem totals of the outer residual, after the three sums above (in
// doubles, past them in either precision)
double *outer_totals(Engine &E) { return eslot<double>(E, P_RED) + 3 * E.cap; }

// z = q(A) r for every problem of the launch; returns the buffer index of z.
// chk: the first kernel also runs the convergence test on the update's r^T r.
template <typename T>
int enqueue_precond(Engine &E, int nprob, int nb, bool pc, int cs, int pm, const Shape &sh, int k,
                    bool chk, bool red, hipStream_t s, Grid *prof, int tag = -1) {
    InnerProb<T> *d = Sel<T>::d(E);
    const bool h16 = cs == CS_F16;
    const bool jac = pm == 3;   // Jacobi-scaled Chebyshev (beyond the paper)
    const T *rr_in = red ? red_rr<T>(E) : eslot<T>(E, P_UPD);
    if (pm == 1 || pm == 2 || k == 1) {
        launch_scale_b<T>(d, nprob, nb, pc, pm, sh.vx, sh.by, chk, rr_in, red, eslot<T>(E, P_CHEB), s);
        if (red) launch_reduce_b<T>(d, nprob, eslot<T>(E, P_CHEB), red_rz<T>(E), s);
        return 0;
    }
    if (jac) {
        // z_1 = D^{-1} r / theta into z[0] (with the convergence test), then
        // the first sweep from the stored z_1 into z[1]
        launch_scale_b<T>(d, nprob, nb, pc, pm, sh.vx, sh.by, chk, rr_in, red, eslot<T>(E, P_CHEB), s);
        launch_cheb_b<T>(d, nprob, nb, pc, cs, true, sh.vx, sh.by, 3, k == 2, false, 1, zsel(0, 1),
                         rr_in, red, eslot<T>(E, P_CHEB), s);
    } else {
        launch_cheb_b<T>(d, nprob, nb, pc, cs, false, sh.vx, sh.by, 1, k == 2, chk, 1, zsel(0, 1),
                         rr_in, red, eslot<T>(E, P_CHEB), s);
    }
    // fused pairs and triples of general sweeps (FP32)
    const int fuse = fuse_for<T>(sh, pm);
    int nbf = 0, nbt = 0;
    if (fuse >= 2) {
        const InnerProb<T> &last = Sel<T>::h(E)[nprob - 1];
        nbf = last.f_tile0 + last.f_ntiles;
        nbt = last.t_tile0 + last.t_ntiles;
    }
    int n = 1, p = 0;   // newest and older iterate after mode 1
    // Timed block: the launches of the one general kernel from j = 3 on (the
    // fused triples, else the fused pairs, else the sweeps before the last),
    // back to back on the stream; its duration over its launch count is the
    // average launch duration, with the two event markers spread over the
    // whole block.
    const bool timing = prof && prof->prof && prof->pev_used + 2 <= prof->pev.size();
    const int wtop = sweep_width(3, k, fuse);
    int blk = 0;
    auto in_block = [&](int jj) {
        return jj >= 3 && jj < k - 1 && sweep_width(jj, k, fuse) == wtop;
    };
    for (int j = 2; j < k;) {
        const int wd = sweep_width(j, k, fuse);
        const bool timed = timing && in_block(j);
        if (timed && blk == 0) (void)hipEventRecord(prof->pev[prof->pev_used], s);
        if (wd > 1) {
            int x, y;
            free_pair(n, p, x, y);
            if constexpr (sizeof(T) == 4) {
                if (wd == 3)
                    launch_cheb3_b<T>(d, nprob, nbt, pc, h16, jac, sh.vx, sh.tr, sh.tzc, sh.twpr, j,
                                      n + 4 * p + 16 * x + 64 * y, s);
                else
                    launch_cheb2_b<T>(d, nprob, nbf, pc, h16, jac, sh.vx, sh.fr, sh.fzc, sh.fwpr, j,
                                      n + 4 * p + 16 * x + 64 * y, s);
            }
            p = x;
            n = y;
        } else {
            // j = 2 reads z_1 where the scale pass stored it (Jacobi) or
            // takes it as r/theta (mode 2)
            const int mode = (j == 2 && !jac) ? 2 : 0;
            launch_cheb_b<T>(d, nprob, nb, pc, cs, jac, sh.vx, sh.by, mode, j == k - 1, false, j,
                             zsel(n, p), rr_in, red, eslot<T>(E, P_CHEB), s);
            std::swap(n, p);
        }
        ++blk;
        if (timed && !in_block(j + wd)) {
            (void)hipEventRecord(prof->pev[prof->pev_used + 1], s);
            const size_t slot = prof->pev_used / 2;
            if (prof->pev_tag.size() <= slot) prof->pev_tag.resize(prof->pev.size() / 2);
            if (prof->pev_cnt.size() <= slot) prof->pev_cnt.resize(prof->pev.size() / 2);
            prof->pev_tag[slot] = tag;
            prof->pev_cnt[slot] = blk;
            prof->pev_used += 2;
            // a fused pair or triple reads z_j, z_{j-1}, r (+ gx, gy) once and
            // writes two iterates
            const Bytes<T> by(pc, h16);
            prof->prof_bytes = (wd == 3 ? by.triple() : wd == 2 ? by.pair() : by.cheb(0)) * (double)prof->N;
            prof->prof_width = wd;
        }
        if (!timed) blk = 0;
        j += wd;
    }
    if (red) launch_reduce_b<T>(d, nprob, eslot<T>(E, P_CHEB), red_rz<T>(E), s);
    return n;
}

template <typename T>
void enqueue_iterations(Engine &E, int nprob, int nb, bool pc, int cs, int pm, const Shape &sh, int k,
                        int first_k, int count, int zfin, bool red, hipStream_t s, Grid *prof) {
    InnerProb<T> *d = Sel<T>::d(E);
    for (int q = 0; q < count; ++q) {
        const int par = (first_k + q) & 1;
        launch_dir_b<T>(d, nprob, nb, pc, cs == CS_CSR ? CS_CSR : CS_OWN, sh.vx, sh.by, par, zfin,
                        red ? red_rz<T>(E) : eslot<T>(E, P_CHEB), red, eslot<T>(E, P_DIR), s);
        if (red) launch_reduce_b<T>(d, nprob, eslot<T>(E, P_DIR), red_pmu<T>(E), s);
        launch_update_b<T>(d, nprob, nb, sh.vx, sh.by, par, red ? red_pmu<T>(E) : eslot<T>(E, P_DIR),
                           red, eslot<T>(E, P_UPD), s);
        if (red) launch_reduce_b<T>(d, nprob, eslot<T>(E, P_UPD), red_rr<T>(E), s);
        enqueue_precond<T>(E, nprob, nb, pc, cs, pm, sh, k, true, red, s, prof, first_k + q);
    }
}

// Host-side stop rule of an inner solve at a true-residual check (Section 4.4):
// dev_done is the device's own stop (1 tolerance, 4 breakdown), tn the norm of
// the true residual r_true = rhat - A x, dn the norm of r_true - r_low, ln the
// norm of the recursive residual r_low, and prev / lprev the true and recursive
// norms of the previous check (< 0 at the first).  Returns 0 to continue, 4 for
// a non-finite value, 2 for drift (eq. switching c: dn >= 0.5 tn), 3 for
// stagnation (eq. switching b: tn > 0.9 prev while the recursive residual
// still fell, ln < lprev: a true residual that rises with the recursive one
// is CG's own non-monotone residual, not stagnation), 5 at the iteration
// limit.  Without tests (the fixed-FP32 baseline) only the device stop,
// non-finite values and the limit apply.
int stop_rule(int dev_done, double tn, double dn, double ln, double prev, double lprev, bool tests,
              bool at_limit) {
    if (dev_done) return dev_done;
    if (!std::isfinite(tn)) return 4;
    if (tests && dn >= 0.5 * tn) return 2;
    if (tests && prev >= 0.0 && tn > 0.9 * prev && ln < lprev) return 3;
    if (at_limit) return 5;
    return 0;
}

// Inner PCG (Algorithm 1 with the Chebyshev preconditioner) on every problem
// with p->inner set: A x = rhat from x = 0, r = rhat already written by the
// residual kernel.  Chunks of `period` iterations run back to back for all
// problems; after each chunk one true-residual launch gives every problem's
// drift (||r_true - r_low|| >= 0.5 ||r_true||) and stagnation
// (||r_true^k|| > 0.9 ||r_true^{k-1}||) tests of Section 4.4.
template <typename T>
Status inner_solve(Engine &E, std::vector<Problem *> &ps, const Shape &sh, int k, int maxit,
                   int period, bool use_graph, hipStream_t s, Grid *prof) {
    std::vector<int> which;
    const int nb = build_inner<T>(E, ps, sh, which);
    if (nb < 0) return Status::err(CUTH_E_DEVICE, "internal: inner solve does not fit the engine");
    const int nprob = (int)which.size();
    if (nprob == 0) return Status::ok();
    const bool pc = ps[which[0]]->g->per_cell;
    const bool h16 = pc && ps[which[0]]->h16;
    const int cs = (sizeof(T) == 8 && ps[which[0]]->csr) ? CS_CSR : (h16 ? CS_F16 : CS_OWN);
    const int pm = ps[which[0]]->pm;
    bool red = false;
    const int above = reduce_above(nprob);
    for (int n = 0; n < nprob; ++n) red = red || ps[which[n]]->ntiles > above;
    CUTH_HIP(hipMemcpyAsync(Sel<T>::d(E), Sel<T>::h(E), sizeof(InnerProb<T>) * nprob,
                            hipMemcpyHostToDevice, s));
    CgState<T> *hs = Sel<T>::hs(E);
    for (int n = 0; n < nprob; ++n) {
        Problem &p = *ps[which[n]];
        CgState<T> &st = hs[n];
        std::memset(&st, 0, sizeof(st));
        st.rz[1] = std::numeric_limits<T>::infinity();
        st.rr = (T)p.rr0;
        st.rr0 = (T)p.rr0;
        st.tol2 = (T)p.tol2;
        st.done = p.rr0 > 0.0 ? 0 : 1;
        p.true_prev = -1.0;
        p.low_prev = -1.0;
        p.stop = 0;
    }
    CUTH_HIP(hipMemcpyAsync(Sel<T>::ds(E), hs, sizeof(CgState<T>) * nprob, hipMemcpyHostToDevice, s));
    const int zfin = enqueue_precond<T>(E, nprob, nb, pc, cs, pm, sh, k, false, red, s, prof);
    const bool graph = use_graph && period % 2 == 0;
    // instantiated chunk of `len` iterations (len even: the arguments repeat
    // with the iteration's parity), captured on first use and kept by the
    // engine for later inner solves of the same configuration
    auto chunk_graph = [&](int len, hipGraphExec_t &out) -> Status {
        std::ostringstream key;
        key << sizeof(T) << ' ' << nprob << ' ' << nb << ' ' << pc << ' ' << cs << ' ' << pm << ' '
            << k << ' ' << len << ' ' << zfin << ' ' << red << ' ' << sh.vx << ',' << sh.by << ','
            << sh.zc << ',' << sh.fr << ',' << sh.fzc << ',' << sh.fwpr << ',' << sh.tr << ','
            << sh.tzc << ',' << sh.twpr;
        for (auto &g : E.graphs)
            if (g.first == key.str()) {
                out = g.second;
                return Status::ok();
            }
        hipGraph_t gr = nullptr;
        CUTH_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        enqueue_iterations<T>(E, nprob, nb, pc, cs, pm, sh, k, 0, len, zfin, red, s, nullptr);
        CUTH_HIP(hipStreamEndCapture(s, &gr));
        const hipError_t ie = hipGraphInstantiate(&out, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ie != hipSuccess) return Status::err(CUTH_E_DEVICE, "hipGraphInstantiate failed");
        E.graphs.emplace_back(key.str(), out);
        return Status::ok();
    };
    hipGraphExec_t exec = nullptr, exec2 = nullptr;
    if (graph) CUTH_TRY(chunk_graph(period, exec));
    std::vector<double> sums(2 * (size_t)nprob, 0.0);
    int it = 0, nchecks = 0;
    Status result = Status::ok();
    // one more host check where the last inner solve of this cycle on this
    // operator stopped: a stop found on the device is only seen at the next
    // check, and every iteration launched before that runs empty (with graphs,
    // chunks of two iterations run up to the predicted stop)
    const int pi = sizeof(T) == 4 ? 1 : 0;
    Problem &p0 = *ps[which[0]];
    const int pred = nprob == 1 ? p0.su->stop_iter[pi][p0.pm][std::min(p0.cycles, 15)] : 0;
    while (it < maxit) {
        int cnt = graph ? period : std::min(period, maxit - it);
        // (graph chunks are of even length: rounded up, so that the check comes
        // at or after the predicted stop, never one iteration before it, where
        // the stagnation test could fire on the FP32 plateau)
        if (pred > it && pred - it < cnt) cnt = graph ? (pred - it + 1) & ~1 : pred - it;
        if (graph) {
            hipGraphExec_t ex = exec;
            if (cnt != period) {
                if (!exec2) CUTH_TRY(chunk_graph(2, exec2));
                ex = exec2;
            }
            for (int q = 0; q < (cnt == period ? 1 : cnt / 2); ++q) {
                const hipError_t le = hipGraphLaunch(ex, s);
                if (le != hipSuccess) {
                    result = Status::err(CUTH_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(le));
                    break;
                }
            }
            if (result.bad()) break;
        } else {
            enqueue_iterations<T>(E, nprob, nb, pc, cs, pm, sh, k, it, cnt, zfin, red, s, prof);
        }
        it += cnt;
        launch_check_b<T>(Sel<T>::d(E), nprob, nb, pc, cs, sh.vx, sh.by, eslot<T>(E, P_CHK), s);
        ++nchecks;
        CUTH_HIP(hipMemcpyAsync(hs, Sel<T>::ds(E), sizeof(CgState<T>) * nprob, hipMemcpyDeviceToHost, s));
        CUTH_HIP(hipMemcpyAsync(E.h_part, eslot<T>(E, P_CHK), sizeof(T) * 2 * (size_t)nb,
                                hipMemcpyDeviceToHost, s));
        CUTH_TRY(sync_stream(s));
        if (prof && prof->prof) {
            // a stop found on the device at CG iteration t (st.iter = t + 1, or
            // t for a breakdown in the direction kernel) empties the sweeps of
            // iteration t and later
            const int dev_stop = hs[0].done == 1 || hs[0].done == 4;
            (void)prof_flush(*prof, dev_stop ? hs[0].iter - 1 : 1 << 30);
        }
        const T *hp = reinterpret_cast<const T *>(E.h_part);
        bool all_done = true;
        for (int n = 0; n < nprob; ++n) {
            Problem &p = *ps[which[n]];
            if (p.stop) continue;
            double a = 0.0, b = 0.0;
            for (int q = p.tile0; q < p.tile0 + p.ntiles; ++q) {
                a += (double)hp[q];
                b += (double)hp[nb + q];
            }
            p.true_rr = a;
            const double tn = std::sqrt(a);
            const double ln = std::sqrt((double)hs[n].rr);
            const int why = stop_rule(hs[n].done, tn, std::sqrt(b), ln, p.true_prev, p.low_prev,
                                      !p.fixed32, it >= maxit);
            if (why && !hs[n].done) {
                // stop this problem on the device too (its launches exit early)
                hs[n].done = why;
                CUTH_HIP(hipMemcpyAsync(&Sel<T>::ds(E)[n].done, &hs[n].done, sizeof(int),
                                        hipMemcpyHostToDevice, s));
            }
            p.true_prev = tn;
            p.low_prev = ln;
            if (why) p.stop = why;
            else all_done = false;
        }
        if (all_done) break;
    }
    CUTH_TRY(sync_stream(s));
    CUTH_TRY(result);
    if (nprob == 1 && p0.stop == 1) p0.su->stop_iter[pi][p0.pm][std::min(p0.cycles, 15)] = hs[0].iter;
    // per-problem results and byte accounting (launches after a problem's stop
    // exit early and move no data)
    for (int n = 0; n < nprob; ++n) {
        Problem &p = *ps[which[n]];
        const Bytes<T> by(p.g->per_cell, p.h16);
        const double N = (double)p.g->N;
        const int iters = hs[n].iter;
        const int reason = p.stop ? p.stop : 5;
        const int precs_run = 1 + iters - (reason == 1 ? 1 : 0);
        p.cg_iters += iters;
        p.reason = reason;
        p.drift_stops += reason == 2;
        p.stag_stops += reason == 3;
        const int fused = fuse_for<T>(sh, p.pm);
        p.bytes += precs_run * by.precond(k, p.pm, fused) * N + iters * (by.dir() + by.update()) * N +
                   nchecks * by.check() * N;
        p.stencils += (int64_t)precs_run * (k - 1) + iters + nchecks;
        p.last_red = p.rr0 > 0 ? std::sqrt(p.true_rr / p.rr0) : 0.0;
        p.cycles += 1;
        p.inner = false;
        if (iters == 0) {
            p.status = Status::err(CUTH_E_BREAKDOWN, "inner solve made no progress");
            p.finished = true;
        } else if (reason == 4) {
            p.status = Status::err(CUTH_E_BREAKDOWN, "CG breakdown (p^T A p <= 0 or non-finite value)");
        }
    }
    return Status::ok();
}

// FP64 residual of every unfinished problem; fills relres, rr0 and the
// correction statistics.
template <typename TI>
Status outer_step(Engine &E, std::vector<Problem *> &ps, const Shape &sh64, hipStream_t s,
                  std::vector<double> &stats5) {
    OuterProb<TI, TI> *h = nullptr;
    OuterProb<TI, TI> *d = nullptr;
    if constexpr (sizeof(TI) == 4) {
        h = reinterpret_cast<OuterProb<TI, TI> *>(E.h_out32);
        d = reinterpret_cast<OuterProb<TI, TI> *>(E.out32);
    } else {
        h = reinterpret_cast<OuterProb<TI, TI> *>(E.h_out64);
        d = reinterpret_cast<OuterProb<TI, TI> *>(E.out64);
    }
    int tile = 0, n = 0, flags = -1;
    std::vector<int> which;
    for (size_t i = 0; i < ps.size(); ++i) {
        Problem &p = *ps[i];
        if (p.finished) continue;
        Work<TI> &w = Sel<TI>::w(p);
        OuterProb<TI, TI> o;
        o.op = outer_view(p, sh64);
        o.ntx = tiles_x(p.g->nx, sh64.vx);
        o.ntz = tiles_z(p.g->nz, sh64.zc);
        o.tile0 = tile;
        o.ntiles = prob_tiles(*p.g, sh64);
        o.th_in = p.th_in;
        o.in_off = p.in_off;
        o.delta = p.have_delta ? w.x : nullptr;
        o.P = p.P;
        o.Tn = p.Tn;
        o.tn_off = p.g->t_amb;
        o.th_out = p.th_out;
        o.r64 = nullptr;
        o.r_in = w.r;
        o.rhat = w.rhat;
        const int f = residual_flags(o);
        flags = n == 0 ? f : (flags == f ? f : -1);
        h[n] = o;
        p.tile0 = tile;
        p.ntiles = o.ntiles;
        tile += o.ntiles;
        which.push_back((int)i);
        ++n;
    }
    stats5.assign(ps.size() * kResidualValues, 0.0);
    if (n == 0) return Status::ok();
    if ((size_t)tile * kResidualValues > E.slot_doubles)
        return Status::err(CUTH_E_DEVICE, "internal: residual launch does not fit the engine");
    const bool pc = ps[which[0]]->g->per_cell;
    CUTH_HIP(hipMemcpyAsync(d, h, sizeof(OuterProb<TI, TI>) * n, hipMemcpyHostToDevice, s));
    launch_residual_b<TI, TI>(d, n, tile, pc, sh64.vx, sh64.by, flags, eslot<double>(E, P_RES), s);
    launch_reduce_outer<TI, TI>(d, n, eslot<double>(E, P_RES), tile, outer_totals(E), s);
    CUTH_HIP(hipMemcpyAsync(E.h_part, outer_totals(E), sizeof(double) * kResidualValues * (size_t)n,
                            hipMemcpyDeviceToHost, s));
    CUTH_TRY(sync_stream(s));
    for (int m = 0; m < n; ++m) {
        Problem &p = *ps[which[m]];
        double *o = &stats5[(size_t)which[m] * kResidualValues];
        for (int v = 0; v < kResidualValues; ++v) o[v] = E.h_part[(size_t)m * kResidualValues + v];
        const double N = (double)p.g->N;
        p.bytes += ((p.th_in ? 8.0 : 0.0) + (p.have_delta ? (double)sizeof(TI) : 0.0) + 8.0 +
                    (p.Tn ? 8.0 : 0.0) + 8.0 + 2.0 * sizeof(TI) + (p.g->per_cell ? 16.0 : 0.0)) * N;
        p.stencils += 1;
        p.th_final = p.th_out;
    }
    return Status::ok();
}

// Refinement decisions after a residual (Section 4.4 readings):
// mixed precision stops when the estimated remaining rise error is below
// tol/10; FP64 stops at the relative-residual tolerance.  Sets p->inner for
// the problems that need another inner solve and their tolerances.
void decide(Problem &p, const double *o, bool mixed, int max_outer) {
    const double rr = o[0], bb = o[1], dinf = o[2], thinf = o[3], bad = o[4];
    p.relres = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    p.inner = false;
    const int cyc = p.cycles;
    if (bad > 0) {
        p.status = Status::err(CUTH_E_BREAKDOWN, "non-finite residual");
        p.finished = true;
        return;
    }
    if (p.fixed32) {
        if (cyc >= 1 && thinf > 0) p.err_est = dinf / thinf;
        if (cyc >= 1 || rr == 0.0 || p.status.bad()) {
            if (!p.status.bad() && p.reason == 5)
                p.status = Status::err(CUTH_E_NOT_CONVERGED, "FP32 iteration limit reached");
            p.finished = true;
            return;
        }
        p.inner = true;
        p.rr0 = (double)(float)rr;
        p.tol2 = p.tol * p.tol * p.rr0;
        return;
    }
    if (!p.status.bad()) {
        if (mixed) {
            if (cyc >= 1) {
                const double d = thinf > 0 ? dinf / thinf : (dinf > 0 ? INFINITY : 0.0);
                // d is about the error before the last correction, and the
                // ratio of two successive corrections, q = d / d_prev, is the
                // error contraction of the inner solve before the last one;
                // against that solve's residual reduction it measures how far
                // the error lags the residual (lag).  On well-conditioned
                // stacks the error falls about as fast as the residual; with
                // condition numbers near 1/u32 the residual falls mainly in
                // the stiff modes and the error left in the smooth ones far
                // less (on a 64-layer stack with condition number 3e6 a
                // 6e3-fold residual cut came with a 20-fold error cut).
                const double q = d / p.d_prev;
                if (cyc >= 2) p.lag = std::max(p.lag, q / std::max(p.red_prev, 1e-6));
                p.red_prev = p.last_red;
                p.est = q * d;
                p.err_est = d;
                p.d_prev = d;
                // An inner solve that met its own tolerance cut the error by
                // about lag times its residual reduction, never below the FP32
                // rounding floor of the inner solve (about 16 ulps, 1e-6: an
                // FP32 residual can be exactly zero while the correction is
                // only FP32-accurate); a margin of 10 covers lags up to 10.
                // One stopped by the drift test (or the iteration limit) says
                // little about the error through its residual: its contraction
                // is taken as the last measured one, q, which needs two
                // corrections after the first solve, and the remaining error
                // as the geometric tail q / (1 - q) d.  Stop when the estimate
                // is a tenth of tol (or tol over the lag), or when the
                // correction itself is below tol and the inner solve cut the
                // error at least tenfold.
                //
                // Once an inner solve has ended on the stagnation test, the
                // FP32 system cannot resolve the error further in that solve
                // (condition number times the FP32 unit roundoff near 1): the
                // cycles then differ widely in what they achieve (one cut the
                // error 60-fold, the next not at all), so no contraction is
                // extrapolated; every later inner solve runs to the floor
                // (tau 1e-5) and the refinement stops when the correction
                // itself is a tenth of tol.
                if (p.reason == 3) p.floor32 = true;
                const double margin = std::max(p.lag, 10.0);
                bool done;
                if (p.floor32)
                    done = d <= 0.1 * p.tol;
                else if (p.reason == 1)
                    done = margin * std::max(p.last_red, 1e-6) * d <= p.tol ||
                           (d <= p.tol && margin * p.last_red <= 1.0);
                else
                    done = (cyc >= 3 && q < 1.0 && 10.0 * q / (1.0 - q) * d <= p.tol) ||
                           (d <= p.tol && margin * p.last_red <= 1.0);
                if (done) {
                    p.finished = true;
                    return;
                }
            }
        } else {
            if (cyc >= 1 && thinf > 0) p.err_est = dinf / thinf;
            if (p.relres <= p.tol) {
                p.finished = true;
                return;
            }
            // a restart that did not halve the true residual has hit the
            // attainable accuracy of FP64 for this system: report, do not loop
            // (or stop without error below the relaxed tolerance)
            if (cyc >= 1 && p.relres > 0.5 * p.prev_relres) {
                p.finished = true;
                if (p.relres <= p.tol_relax) return;
                p.status = Status::err(CUTH_E_NOT_CONVERGED,
                                       "true residual stagnated above tol (attainable accuracy)");
                return;
            }
            p.prev_relres = p.relres;
        }
    }
    if (rr == 0.0 || p.status.bad()) {
        p.finished = true;
        return;
    }
    if (cyc >= max_outer) {
        p.status = Status::err(CUTH_E_NOT_CONVERGED, "refinement cycle limit reached");
        p.finished = true;
        return;
    }
    p.inner = true;
    if (mixed) {
        // the inner tolerance that would bring the estimated error to a tenth
        // of tol, tightened by a lag beyond the margin
        const double tau =
            cyc == 0 || p.floor32
                ? 1e-5
                : std::min(0.1, std::max(1e-5, 0.1 * p.tol / (p.est * std::max(1.0, 0.1 * p.lag))));
        p.rr0 = (double)(float)rr;
        p.tol2 = tau * tau * p.rr0;
    } else {
        // hot restart: r and p recomputed from their definitions, x kept
        p.rr0 = rr;
        p.tol2 = p.tol * p.tol * bb;
    }
}

template <typename TI>
Status run_refinement(Engine &E, std::vector<Problem *> &ps, const Shape &sh_in,
                      const Shape &sh64, int k, const cuth_options &o, int period, bool use_graph,
                      hipStream_t s, Grid *prof) {
    const bool mixed = sizeof(TI) == 4;
    std::vector<double> st5;
    CUTH_TRY(upload_cheb<TI>(E, ps, s));
    for (;;) {
        CUTH_TRY(outer_step<TI>(E, ps, sh64, s, st5));
        bool any = false;
        for (size_t i = 0; i < ps.size(); ++i) {
            Problem &p = *ps[i];
            if (p.finished) continue;
            decide(p, &st5[i * kResidualValues], mixed, o.max_outer);
            if (log_on())
                std::fprintf(stderr,
                             "cuth: problem %zu cycle %d relres %.3e last reduction %.3e est %.3e "
                             "correction %.3e inner stop %d lag %.2f%s%s\n",
                             i, p.cycles, p.relres, p.last_red, p.est, p.err_est, p.reason, p.lag,
                             p.floor32 ? " floor" : "",
                             p.inner ? "" : " -> done");
            any = any || p.inner;
        }
        if (!any) break;
        std::vector<Problem *> ran;
        for (Problem *p : ps)
            if (p->inner) ran.push_back(p);
        CUTH_TRY(inner_solve<TI>(E, ps, sh_in, k, o.max_inner, period, use_graph, s, prof));
        for (Problem *p : ran) {
            if (p->finished) continue;
            // the next residual applies this correction to the current theta
            p->th_in = p->th_out;
            p->in_off = 0.0;
            p->have_delta = true;
            p->th_out = (p->th_out == p->thA) ? p->thB : p->thA;
        }
    }
    return Status::ok();
}

// ---------------------------------------------------------------------------
// The paper's stage-switched scheme (Section 4.4): CG vectors, scalars and inner
// products in FP64; the Chebyshev preconditioner in FP32 with FP16-stored
// lateral conductances; the CG product with FP32-stored conductances promoted
// to FP64 in the early stage and FP64 ones in the late stage.  The early stage
// ends at the first of: ||r_low|| <= sqrt(tol) ||b|| (eq. switching a, with the
// relative tolerance in place of the absolute one), stagnation (b) or drift (c)
// of the FP64 true residual checked every `period` iterations; the switch is a
// hot restart: r recomputed as b - A x in FP64 (x kept), p restarted.

// One FP64 inner CG with the FP32 preconditioner on the problems with
// p->inner set: A x = rhat from x = 0, r = rhat (FP64) and r_lo = (float) r
// already written.
Status inner_solve_staged(Engine &E, std::vector<Problem *> &ps, const Shape &sh32,
                          const Shape &sh64, int k, int maxit, int period, hipStream_t s) {
    std::vector<int> which32, which;
    const int nb32 = build_inner<float>(E, ps, sh32, which32);
    const int nb = build_inner<double>(E, ps, sh64, which);   // p->tile0/ntiles: FP64 tiling
    if (nb32 < 0 || nb < 0) return Status::err(CUTH_E_DEVICE, "internal: staged solve does not fit the engine");
    const int nprob = (int)which.size();
    if (nprob == 0) return Status::ok();
    const bool pc = ps[which[0]]->g->per_cell;
    const bool h16 = pc && ps[which[0]]->h16;
    const int pm = ps[which[0]]->pm;
    const bool early = ps[which[0]]->early;
    bool red = false;
    const int above = reduce_above(nprob);
    for (int n = 0; n < nprob; ++n) red = red || ps[which[n]]->ntiles > above;
    const int zfin32 = precond_final(k, pm, fuse_for<float>(sh32, pm));
    InnerProb<double> *h64 = E.h_in64;
    for (int n = 0; n < nprob; ++n) {
        Problem &p = *ps[which[n]];
        h64[n].op.fx = p.g->per_cell ? p.g->gx32 : nullptr;
        h64[n].op.fy = p.g->per_cell ? p.g->gy32 : nullptr;
        h64[n].r_lo = p.w32.r;
        h64[n].z_lo = zfin32 == 0 ? p.w32.zA : p.w32.zB;
        h64[n].done_lo = &E.st32[n].done;
    }
    CUTH_HIP(hipMemcpyAsync(E.in32, E.h_in32, sizeof(InnerProb<float>) * nprob, hipMemcpyHostToDevice, s));
    CUTH_HIP(hipMemcpyAsync(E.in64, E.h_in64, sizeof(InnerProb<double>) * nprob, hipMemcpyHostToDevice, s));
    CgState<double> *hs = E.h_st64;
    CgState<float> *hs32 = E.h_st32;
    for (int n = 0; n < nprob; ++n) {
        Problem &p = *ps[which[n]];
        std::memset(&hs[n], 0, sizeof(hs[n]));
        std::memset(&hs32[n], 0, sizeof(hs32[n]));
        hs[n].rz[1] = std::numeric_limits<double>::infinity();
        hs[n].rr = p.rr0;
        hs[n].rr0 = p.rr0;
        hs[n].tol2 = p.tol2;
        hs[n].done = p.rr0 > 0.0 ? 0 : 1;
        hs32[n].done = hs[n].done;
        p.true_prev = -1.0;
        p.low_prev = -1.0;
        p.stop = 0;
    }
    CUTH_HIP(hipMemcpyAsync(E.st64, hs, sizeof(CgState<double>) * nprob, hipMemcpyHostToDevice, s));
    CUTH_HIP(hipMemcpyAsync(E.st32, hs32, sizeof(CgState<float>) * nprob, hipMemcpyHostToDevice, s));
    InnerProb<double> *d = E.in64;
    auto precond = [&]() {
        (void)enqueue_precond<float>(E, nprob, nb32, pc, h16 ? CS_F16 : CS_OWN, pm, sh32, k, false, false, s, nullptr);
        launch_promote_dot<double>(d, nprob, nb, sh64.vx, sh64.by, eslot<double>(E, P_CHEB), s);
        if (red) launch_reduce_b<double>(d, nprob, eslot<double>(E, P_CHEB), red_rz<double>(E), s);
    };
    precond();
    int it = 0, nchecks = 0;
    while (it < maxit) {
        const int cnt = std::min(period, maxit - it);
        for (int q = 0; q < cnt; ++q) {
            const int par = (it + q) & 1;
            launch_dir_b<double>(d, nprob, nb, pc, early ? CS_F32 : CS_OWN, sh64.vx, sh64.by, par, 0,
                                 red ? red_rz<double>(E) : eslot<double>(E, P_CHEB), red,
                                 eslot<double>(E, P_DIR), s);
            if (red) launch_reduce_b<double>(d, nprob, eslot<double>(E, P_DIR), red_pmu<double>(E), s);
            launch_update_b<double>(d, nprob, nb, sh64.vx, sh64.by, par,
                                    red ? red_pmu<double>(E) : eslot<double>(E, P_DIR), red,
                                    eslot<double>(E, P_UPD), s);
            launch_reduce_conv<double>(d, nprob, eslot<double>(E, P_UPD), s);
            precond();
        }
        it += cnt;
        // FP64 true residual with the FP64 operator (switch tests b and c)
        launch_check_b<double>(d, nprob, nb, pc, CS_OWN, sh64.vx, sh64.by, eslot<double>(E, P_CHK), s);
        ++nchecks;
        CUTH_HIP(hipMemcpyAsync(hs, E.st64, sizeof(CgState<double>) * nprob, hipMemcpyDeviceToHost, s));
        CUTH_HIP(hipMemcpyAsync(E.h_part, eslot<double>(E, P_CHK), sizeof(double) * 2 * (size_t)nb,
                                hipMemcpyDeviceToHost, s));
        CUTH_TRY(sync_stream(s));
        bool all_done = true;
        for (int n = 0; n < nprob; ++n) {
            Problem &p = *ps[which[n]];
            if (p.stop) continue;
            double a = 0.0, b = 0.0;
            for (int q = p.tile0; q < p.tile0 + p.ntiles; ++q) {
                a += E.h_part[q];
                b += E.h_part[nb + q];
            }
            p.true_rr = a;
            const double tn = std::sqrt(a);
            const double ln = std::sqrt(hs[n].rr);
            const int why = stop_rule(hs[n].done, tn, std::sqrt(b), ln, p.true_prev, p.low_prev, true,
                                      it >= maxit);
            if (why && !hs[n].done) {
                hs[n].done = why;
                CUTH_HIP(hipMemcpyAsync(&E.st64[n].done, &hs[n].done, sizeof(int),
                                        hipMemcpyHostToDevice, s));
                CUTH_HIP(hipMemcpyAsync(&E.st32[n].done, &hs[n].done, sizeof(int),
                                        hipMemcpyHostToDevice, s));
            }
            p.true_prev = tn;
            p.low_prev = ln;
            if (why) p.stop = why;
            else all_done = false;
        }
        if (all_done) break;
    }
    CUTH_TRY(sync_stream(s));
    for (int n = 0; n < nprob; ++n) {
        Problem &p = *ps[which[n]];
        const double N = (double)p.g->N;
        const Bytes<float> b32(p.g->per_cell, p.h16);
        const Bytes<double> b64(p.g->per_cell);
        const int iters = hs[n].iter;
        const int reason = p.stop ? p.stop : 5;
        const int precs_run = 1 + iters - (reason == 1 ? 1 : 0);
        const double dir64 = 32.0 + (p.g->per_cell ? (p.early ? 8.0 : 16.0) : 0.0);
        p.cg_iters += iters;
        p.reason = reason;
        p.drift_stops += reason == 2;
        p.stag_stops += reason == 3;
        p.bytes += precs_run * (b32.precond(k, p.pm, fuse_for<float>(sh32, p.pm)) + 20.0) * N + iters * (dir64 + b64.update() + 4.0) * N +
                   nchecks * b64.check() * N;
        p.stencils += (int64_t)precs_run * (k - 1) + iters + nchecks;
        p.last_red = p.rr0 > 0 ? std::sqrt(p.true_rr / p.rr0) : 0.0;
        p.cycles += 1;
        p.inner = false;
        if (iters == 0 && reason != 1) {
            p.status = Status::err(CUTH_E_BREAKDOWN, "inner solve made no progress");
            p.finished = true;
        } else if (reason == 4) {
            p.status = Status::err(CUTH_E_BREAKDOWN, "CG breakdown (p^T A p <= 0 or non-finite value)");
        }
    }
    return Status::ok();
}

// Decisions of the stage-switched scheme after an FP64 residual: finished at
// ||b - A T|| <= tol ||b||; otherwise an inner solve to tol2 = tol ||b||^2 (early
// stage, switch test a) or tol^2 ||b||^2 (late stage).
void decide_staged(Problem &p, const double *o, int max_outer) {
    const double rr = o[0], bb = o[1], dinf = o[2], thinf = o[3], bad = o[4];
    p.relres = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    p.inner = false;
    if (bad > 0) {
        p.status = Status::err(CUTH_E_BREAKDOWN, "non-finite residual");
        p.finished = true;
        return;
    }
    if (p.cycles >= 1 && thinf > 0) p.err_est = dinf / thinf;
    if (!p.status.bad() && p.relres <= p.tol) {
        p.finished = true;
        return;
    }
    if (!p.status.bad() && !p.early && p.cycles >= 2 && p.relres > 0.5 * p.prev_relres) {
        p.finished = true;
        if (p.relres <= p.tol_relax) return;
        p.status = Status::err(CUTH_E_NOT_CONVERGED,
                               "true residual stagnated above tol (attainable accuracy)");
        return;
    }
    p.prev_relres = p.relres;
    if (rr == 0.0 || p.status.bad()) {
        p.finished = true;
        return;
    }
    if (p.cycles >= max_outer) {
        p.status = Status::err(CUTH_E_NOT_CONVERGED, "refinement cycle limit reached");
        p.finished = true;
        return;
    }
    p.inner = true;
    p.rr0 = rr;
    p.tol2 = p.early ? p.tol * bb : p.tol * p.tol * bb;
}

Status run_staged(Engine &E, std::vector<Problem *> &ps, const Shape &sh32, const Shape &sh64,
                  int k, const cuth_options &o, int period, hipStream_t s) {
    std::vector<double> st5;
    CUTH_TRY(upload_cheb<float>(E, ps, s));
    for (Problem *p : ps) p->early = true;
    for (;;) {
        CUTH_TRY(outer_step<double>(E, ps, sh64, s, st5));
        bool any = false;
        for (size_t i = 0; i < ps.size(); ++i) {
            Problem &p = *ps[i];
            if (p.finished) continue;
            decide_staged(p, &st5[i * kResidualValues], o.max_outer);
            if (log_on() && p.inner)
                std::fprintf(stderr, "cuth: problem %zu cycle %d %s stage relres %.3e\n", i, p.cycles,
                             p.early ? "early" : "late", p.relres);
            any = any || p.inner;
        }
        if (!any) break;
        std::vector<Problem *> ran;
        for (Problem *p : ps)
            if (p->inner) {
                ran.push_back(p);
                launch_to_f32(p->g->N, p->w64.r, p->w32.r, s);
            }
        // every problem of a launch is in the same stage (they start together
        // and each switches after its first inner solve)
        CUTH_TRY(inner_solve_staged(E, ps, sh32, sh64, k, o.max_inner, period, s));
        for (Problem *p : ran) {
            p->early = false;
            if (p->finished) continue;
            p->th_in = p->th_out;
            p->in_off = 0.0;
            p->have_delta = true;
            p->th_out = (p->th_out == p->thA) ? p->thB : p->thA;
        }
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

// A later tuning candidate replaces the best so far only when it is faster by
// more than this margin: near-ties keep the earlier candidate, so timing noise
// does not flip the chosen shape from one process to the next.
constexpr float kTuneMargin = 0.97f;
// Triples against the chosen pairs take a smaller margin: inside a solve the
// triples' lead has come out larger than in the tuner's back-to-back timing
// (512x512x16: 18 against 14 % per sweep; a batch of 64 stacks: 3.1 against
// 2.7 %), so a near-tie still favours them.
constexpr float kTuneMargin3 = 0.99f;

// Fused pairs of general FP32 Chebyshev sweeps: CUTH_FUSE=0 never, CUTH_FUSE=1
// always (shape CUTH_FUSE_SHAPE="R,zc", default 2,8), unset: chosen per grid by
// timing (tune_fuse).  A workgroup holds R + 2 rows of whole-row wavefronts (at
// most 16) and a ring of three layers of them in LDS (at most 64 KB); grids too
// wide for that keep single sweeps.
int fuse_env() {
    const char *e = std::getenv("CUTH_FUSE");
    if (!e) return -1;
    return e[0] == '0' ? 0 : 1;
}

// Fit fused shape (R, zc) to rows of max_nx cells; false when it cannot fit.
// wcap > 0: at most wcap wavefronts per row, the row split into overlapping x
// windows where it is longer (fused_windows).
int fused_wpr(int max_nx, int vx, int wcap) {
    const int whole = (max_nx + kWave * vx - 1) / (kWave * vx);
    return wcap > 0 ? std::min(whole, wcap) : whole;
}

bool fuse_fit(Shape &sh, int max_nx, int R, int zc, int wcap = 0) {
    sh.fr = 0;
    const int wpr = fused_wpr(max_nx, sh.vx, wcap);
    auto lds = [&](int r) { return (size_t)3 * (r + 2) * wpr * kWave * sh.vx * sizeof(float); };
    while (R > 1 && (wpr * (R + 2) > 16 || lds(R) > 65536)) --R;
    if (R < 1 || wpr * (R + 2) > 16 || lds(R) > 65536) return false;
    sh.fr = R;
    sh.fzc = zc;
    sh.fwpr = wpr;
    return true;
}

// Fused triples (on top of pairs): CUTH_FUSE3=0 never, CUTH_FUSE3=1 always
// where pairs run (shape CUTH_FUSE3_SHAPE="R,zc", default 4,8), unset: chosen
// by timing against the pairs (tune_fuse).  A workgroup holds R + 4 rows of
// whole-row wavefronts (at most 16) and two rings of three layers in LDS.
int fuse3_env() {
    const char *e = std::getenv("CUTH_FUSE3");
    if (!e) return -1;
    return e[0] == '0' ? 0 : 1;
}

// Dynamic LDS a workgroup may use on the current device.
size_t lds_cap() {
    static const size_t cap = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            return (size_t)65536;
        return (size_t)v;
    }();
    return cap;
}

// Fit the triple shape (R, zc) to rows of max_nx cells; false when it cannot fit.
bool fuse3_fit(Shape &sh, int max_nx, int R, int zc, int wcap = 0) {
    sh.tr = 0;
    const int wpr = fused_wpr(max_nx, sh.vx, wcap);
    auto lds = [&](int r) { return (size_t)3 * ((r + 4) + (r + 2)) * wpr * kWave * sh.vx * sizeof(float); };
    while (R > 1 && (wpr * (R + 4) > 16 || lds(R) > lds_cap())) --R;
    if (R < 1 || wpr * (R + 4) > 16 || lds(R) > lds_cap()) return false;
    sh.tr = R;
    sh.tzc = zc;
    sh.twpr = wpr;
    return true;
}

// Shapes forced from the environment (CUTH_FUSE=1, CUTH_FUSE3=1), or no fusion.
void set_fuse(Shape &sh, int max_nx) {
    sh.fr = 0;
    sh.tr = 0;
    if (fuse_env() != 1) return;
    // "R,zc" or "R,zc,wcap" (wcap: wavefronts per row, x windows where the
    // row is longer)
    auto parse = [](const char *name, int rmax, int &R, int &zc, int &wc) {
        if (const char *f = std::getenv(name)) {
            int a = 0, b = 0, c = 0;
            const int n = std::sscanf(f, "%d,%d,%d", &a, &b, &c);
            if (n >= 2 && a >= 1 && a <= rmax && b >= 1) {
                R = a;
                zc = b;
                wc = (n == 3 && c >= 1 && c <= 16) ? c : 0;
            }
        }
    };
    int R = 2, zc = 8, wc = 0;
    parse("CUTH_FUSE_SHAPE", 14, R, zc, wc);
    if (!fuse_fit(sh, max_nx, R, zc, wc) || fuse3_env() != 1) return;
    R = 4;
    zc = 8;
    wc = 0;
    parse("CUTH_FUSE3_SHAPE", 12, R, zc, wc);
    (void)fuse3_fit(sh, max_nx, R, zc, wc);
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
// adjoint factors: 1/k_lat[l], and dg/dk_vert[l] of the faces above / below layer l
// (g = dx dy / (dz_a/(2 k_a) + dz_b/(2 k_b)) gives dg/dk_a = g^2 dz_a / (2 k_a^2 dx dy))
static Status upload_adj_factors(Grid &g) {
    const int nz = g.nz;
    std::vector<double> fac((size_t)3 * nz, 0.0);
    const double dxdy = g.dx * g.dy;
    for (int l = 0; l < nz; ++l) {
        fac[l] = 1.0 / g.k_lat[l];
        const double kv = g.k_vert[l];
        if (l + 1 < nz) {
            const double gz = dxdy / (g.dz[l] / (2.0 * kv) + g.dz[l + 1] / (2.0 * g.k_vert[l + 1]));
            fac[nz + l] = gz * gz * g.dz[l] / (2.0 * kv * kv * dxdy);
        }
        if (l > 0) {
            const double gz = dxdy / (g.dz[l - 1] / (2.0 * g.k_vert[l - 1]) + g.dz[l] / (2.0 * kv));
            fac[2 * nz + l] = gz * gz * g.dz[l] / (2.0 * kv * kv * dxdy);
        }
    }
    if (hipMemcpy(g.adj_fac, fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return Status::err(CUTH_E_DEVICE, "hipMemcpy failed");
    return Status::ok();
}

// Per-cell grids: the face conductance planes from k_lat and the multiplier
// (FP64, FP32, and FP16 scaled per layer by 2^e_l), with the per-layer maxima
// of the lateral row sums; then the adjoint factors (every grid).  Writes the
// grid's allocations only (planes and build_tmp: dz, k_lat and the FP16 scales
// per layer, then the two maxima per layer and the bad-entry flag).
static Status build_coefficients(Grid &g, const double *mult) {
    CUTH_TRY(upload_adj_factors(g));
    if (!g.per_cell) return Status::ok();
    const int nz = g.nz;
    double *ddz = g.build_tmp, *dkl = ddz + nz, *dscale = dkl + nz;
    unsigned long long *dmax = reinterpret_cast<unsigned long long *>(dscale + nz);
    unsigned int *dbad = reinterpret_cast<unsigned int *>(dmax + 2 * nz);
    // dmax[0, nz): max lateral row sum per layer; dmax[nz, 2 nz): max single g
    std::vector<unsigned long long> hmax(2 * (size_t)nz, 0ull);
    unsigned int hbad = 0;
    bool ok = hipMemcpy(ddz, g.dz.data(), nz * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dkl, g.k_lat.data(), nz * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(dmax, 0, 2 * nz * sizeof(unsigned long long)) == hipSuccess &&
              hipMemset(dbad, 0, sizeof(unsigned int)) == hipSuccess;
    if (ok) {
        launch_build_lateral(g.nx, g.ny, nz, g.dx, g.dy, ddz, dkl, mult, g.gx64, g.gy64, g.gx32,
                             g.gy32, dmax, dmax + nz, dbad, g.stream);
        ok = hipStreamSynchronize(g.stream) == hipSuccess &&
             hipMemcpy(hmax.data(), dmax, 2 * nz * sizeof(unsigned long long), hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(&hbad, dbad, sizeof(unsigned int), hipMemcpyDeviceToHost) == hipSuccess;
    }
    if (ok && !hbad) {
        g.lat_rowmax.resize(nz);
        g.e16.assign(nz, 0);
        std::vector<double> scale(nz, 1.0);
        for (int l = 0; l < nz; ++l) {
            double v, m;
            std::memcpy(&v, &hmax[l], sizeof(double));
            std::memcpy(&m, &hmax[nz + l], sizeof(double));
            g.lat_rowmax[l] = v;
            // FP16 storage scale 2^e_l with e_l = 14 - ceil(log2(max g)):
            // frexp gives m = f 2^x with f in [0.5, 1), so ceil(log2 m) is
            // x, or x - 1 when f is exactly 0.5
            if (m > 0.0) {
                int x = 0;
                const double f = std::frexp(m, &x);
                g.e16[l] = 14 - (f == 0.5 ? x - 1 : x);
            }
            scale[l] = std::ldexp(1.0, g.e16[l]);
        }
        ok = hipMemcpy(dscale, scale.data(), nz * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
        if (ok) {
            launch_build_fp16(g.nx, g.ny, nz, g.gx64, g.gy64, dscale, g.hx, g.hy, g.stream);
            ok = hipStreamSynchronize(g.stream) == hipSuccess;
        }
    }
    if (!ok) return Status::err(CUTH_E_DEVICE, "coefficient build failed");
    if (hbad) return Status::err(CUTH_E_INVALID, "k_lat_mult has entries <= 0 or non-finite");
    return Status::ok();
}

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
    const size_t nb_max = std::max({(size_t)prob_tiles(*g, g->sh32), (size_t)prob_tiles(*g, g->sh64),
                                    (size_t)kRedBlocks});
    g->slot_doubles = 8 * nb_max;
    const size_t nb_adj = (size_t)((g->nx + kWave - 1) / kWave) * ((g->ny + 3) / 4);
    Status st;
    if ((st = dev_alloc(&g->part, g->slot_doubles * S_COUNT + (size_t)2 * g->nz * nb_adj)).bad())
        return fail(st);
    g->part_adj = g->part + g->slot_doubles * S_COUNT;
    if ((st = dev_alloc(&g->lz, 1024)).bad()) return fail(st);
    if ((st = dev_alloc(&g->adj_fac, (size_t)3 * g->nz)).bad()) return fail(st);
    if ((st = dev_alloc(&g->thA, (size_t)g->N)).bad()) return fail(st);
    if ((st = dev_alloc(&g->thB, (size_t)g->N)).bad()) return fail(st);
    if ((st = alloc_work(g->w32, g->N)).bad()) return fail(st);
    if ((st = host_alloc(&g->h_lz, 1024)).bad()) return fail(st);
    if ((st = engine_alloc(g->eng, 1, 256, nb_max)).bad()) return fail(st);
    if (hipEventCreate(&g->ev0) != hipSuccess || hipEventCreate(&g->ev1) != hipSuccess ||
        hipEventCreate(&g->ev2) != hipSuccess)
        return fail(Status::err(CUTH_E_DEVICE, "hipEventCreate failed"));

    if (g->per_cell) {
        const int64_t N = g->N;
        if ((st = dev_alloc(&g->gx64, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->gy64, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->gx32, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->gy32, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->hx, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->hy, (size_t)N)).bad()) return fail(st);
        if ((st = dev_alloc(&g->build_tmp, (size_t)5 * g->nz + 1)).bad()) return fail(st);
    }
    if ((st = build_coefficients(*g, d.k_lat_mult)).bad()) return fail(st);
    *out = g;
    return Status::ok();
}

void batch_pool_free(BatchPool &bp) {
    engine_free(bp.E);
    dev_free(bp.pool32);
    dev_free(bp.pool64);
    dev_free(bp.poolth);
    bp.key.clear();
}

void grid_destroy(Grid *g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    engine_free(g->eng);
    for (BatchPool &bp : g->batch) batch_pool_free(bp);
    for (Setup &su : g->setups) {
        dev_free(su.lc64);
        dev_free(su.lc32);
        dev_free(su.csr_ptr);
        dev_free(su.csr_col);
        dev_free(su.csr_val);
        dev_free(su.dis);
    }
    dev_free(g->gx64);
    dev_free(g->gy64);
    dev_free(g->gx32);
    dev_free(g->gy32);
    dev_free(g->hx);
    dev_free(g->hy);
    dev_free(g->build_tmp);
    free_work(g->w32);
    free_work(g->w64);
    dev_free(g->thA);
    dev_free(g->thB);
    dev_free(g->part);
    dev_free(g->lz);
    dev_free(g->adj_fac);
    host_free(g->h_lz);
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

OpView<float> view32(const Grid &g, const Setup &su, bool h16) {
    OpView<float> v{g.nx, g.ny, g.nz, g.per_cell ? g.gx32 : nullptr, g.per_cell ? g.gy32 : nullptr,
                    su.lc32, g.sh32.vx, g.sh32.by, g.sh32.zc};
    if (h16 && g.per_cell) {
        v.hx = g.hx;
        v.hy = g.hy;
    }
    return v;
}

// Per-layer coefficients of the operator of dt (steady: dt == 0) and the
// Gershgorin bound of its spectrum.
static void layer_coefs(const Grid &g, double dt, std::vector<LayerCoef<double>> &hlc,
                        double &gersh_out) {
    const int nz = g.nz;
    const double dx = g.dx, dy = g.dy, dxdy = dx * dy;
    hlc.assign(nz, LayerCoef<double>{});
    double gersh = 0.0;
    for (int l = 0; l < nz; ++l) {
        LayerCoef<double> &L = hlc[l];
        const double k = g.k_lat[l], d = g.dz[l];
        // series half-cell conductance of a lateral face inside a uniform layer
        L.gx = (dy * d) / (dx / (2.0 * k) + dx / (2.0 * k));
        L.gy = (dx * d) / (dy / (2.0 * k) + dy / (2.0 * k));
        L.gzu = (l + 1 < nz)
                    ? dxdy / (d / (2.0 * g.k_vert[l]) + g.dz[l + 1] / (2.0 * g.k_vert[l + 1]))
                    : 0.0;
        L.gzd = (l > 0) ? hlc[l - 1].gzu : 0.0;
        L.cap = (dt > 0.0) ? g.cap[l] * dxdy * d / dt : 0.0;
        L.sink = L.cap + (l == nz - 1 ? g.h_top * dxdy : 0.0) + (l == 0 ? g.h_bot * dxdy : 0.0);
        L.hs = g.e16.empty() ? 1.0 : std::ldexp(1.0, -g.e16[l]);
        const double lat = g.per_cell ? g.lat_rowmax[l]
                                      : std::min(2, g.nx - 1) * L.gx + std::min(2, g.ny - 1) * L.gy;
        gersh = std::max(gersh, 2.0 * (lat + L.gzu + L.gzd) + L.sink);
    }
    gersh_out = gersh;
}

// FP32 copy of the layer coefficients (each rounded once).
static std::vector<LayerCoef<float>> layer_coefs32(const std::vector<LayerCoef<double>> &hlc) {
    std::vector<LayerCoef<float>> h32(hlc.size());
    for (size_t l = 0; l < hlc.size(); ++l) {
        const LayerCoef<double> &L = hlc[l];
        h32[l] = LayerCoef<float>{(float)L.gx, (float)L.gy, (float)L.gzd, (float)L.gzu,
                                  (float)L.sink, (float)L.cap, (float)L.hs};
    }
    return h32;
}

Setup *get_setup(Grid &g, double dt, Status &status) {
    status = Status::ok();
    for (Setup &su : g.setups)
        if (su.dt == dt) return &su;
    Setup su;
    su.dt = dt;
    const int nz = g.nz;
    layer_coefs(g, dt, su.hlc, su.gersh);
    const std::vector<LayerCoef<float>> h32 = layer_coefs32(su.hlc);
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

Status grid_set_conductivity(Grid &g, const double *k_lat, const double *k_vert, const double *mult) {
    // nothing in flight may read the planes or coefficients being replaced
    CUTH_TRY(sync_stream(g.stream));
    g.valid = false;
    g.k_lat.assign(k_lat, k_lat + g.nz);
    g.k_vert.assign(k_vert, k_vert + g.nz);
    CUTH_TRY(build_coefficients(g, g.per_cell ? mult : nullptr));
    // every operator the handle holds (one per dt used so far): its layer
    // coefficients in place, its spectral intervals and stop predictions
    // dropped, the Jacobi scaling recomputed, the CSR copy rebuilt on next use
    for (Setup &su : g.setups) {
        layer_coefs(g, su.dt, su.hlc, su.gersh);
        const std::vector<LayerCoef<float>> h32 = layer_coefs32(su.hlc);
        if (hipMemcpy(su.lc64, su.hlc.data(), g.nz * sizeof(LayerCoef<double>), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(su.lc32, h32.data(), g.nz * sizeof(LayerCoef<float>), hipMemcpyHostToDevice) != hipSuccess)
            return Status::err(CUTH_E_DEVICE, "hipMemcpy of layer coefficients failed");
        su.have_bounds = false;
        su.bounds_steps = 0;
        su.have_jbounds = false;
        su.jbounds_steps = 0;
        if (su.dis) launch_jacobi_dis(view64(g, su), su.dis, g.stream);
        dev_free(su.csr_ptr);
        dev_free(su.csr_col);
        dev_free(su.csr_val);
        su.csr_nnz = 0;
        std::memset(su.stop_iter, 0, sizeof(su.stop_iter));
    }
    CUTH_HIP(hipGetLastError());
    CUTH_TRY(sync_stream(g.stream));
    g.valid = true;
    return Status::ok();
}

// FP32 Lanczos on the FP32 operator (Section 4.4, component-wise precision of
// Lanczos): alpha_j = v_j^T A v_j, w = A v_j - alpha_j v_j - beta_{j-1} v_{j-1},
// beta_j = ||w||, v_{j+1} = w / beta_j.  Scalars stay on the device until the
// end; one readback returns the tridiagonal.
Status run_lanczos(Grid &g, Setup &su, int steps, const float *v0, std::vector<double> &alpha,
                   std::vector<double> &beta, bool scaled) {
    steps = (int)std::max<int64_t>(1, std::min<int64_t>(steps, g.N));
    steps = std::min(steps, 256);
    const OpView<float> op = view32(g, su);
    if (scaled && !su.dis) {
        CUTH_TRY(dev_alloc(&su.dis, (size_t)g.N));
        launch_jacobi_dis(view64(g, su), su.dis, g.stream);
        CUTH_HIP(hipGetLastError());
    }
    const float *dis = scaled ? su.dis : nullptr;
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
        launch_lanczos_av(op, j, bufs[iv], j > 0 ? bufs[ip] : nullptr, g.lz, dis, bufs[iw], pa,
                          g.stream);
        launch_lanczos_orth(g.N, j, bufs[iw], bufs[iv], g.lz, pa, nbs, pb, g.stream);
        if (j == steps - 1) break;
        launch_lanczos_div(g.N, j, bufs[iw], g.lz, pb, nb1, g.stream);
        const int old = ip;
        ip = iv;
        iv = iw;
        iw = old;
    }
    CUTH_HIP(hipMemcpyAsync(g.h_lz, g.lz, 512 * sizeof(float), hipMemcpyDeviceToHost, g.stream));
    CUTH_TRY(sync_stream(g.stream));
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

Status ensure_bounds(Grid &g, Setup &su, int steps, bool scaled) {
    if (scaled) {
        // D^{-1} A: its spectrum lies in (0, 2] for a diagonally dominant A with
        // positive diagonal (Gershgorin: |lambda - 1| <= sum_j |a_ij| / a_ii <= 1)
        if (su.have_jbounds && su.jbounds_steps == steps) return Status::ok();
        std::vector<double> a, b;
        CUTH_TRY(run_lanczos(g, su, steps, nullptr, a, b, true));
        double lo, hi;
        tridiag_extremes(a, b, lo, hi);
        su.jritz_min = lo;
        su.jritz_max = hi;
        su.jlmax = std::min(2.0, 1.05 * hi);
        su.jlmin = lo;
        if (!(su.jlmin > 0.0) || !(su.jlmax > su.jlmin * (1.0 + 1e-6))) su.jlmin = 0.5 * su.jlmax;
        su.have_jbounds = true;
        su.jbounds_steps = steps;
        return Status::ok();
    }
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

namespace {

template <typename T>
Status tune_fuse(Engine &E, std::vector<Problem *> &ps, int k, Shape &sh, const std::string &sig);

// Chebyshev degree chosen from the preconditioner's interval [lmin, lmax]: the
// smallest k >= 2 whose polynomial damps that interval to 2 s^k <= 0.3, with
// s = (sqrt(c) - 1)/(sqrt(c) + 1), c = lmax/lmin (a degree-k Chebyshev polynomial
// leaves at most 1/T_k((c + 1)/(c - 1)) <= 2 s^k there); at most 64.  Measured on
// the 512x512x16 steady and the 1024x1024x20 transient systems, the time to
// tolerance is within a few percent of the best degree at this threshold.
int auto_degree(double lmin, double lmax) {
    const double c = lmin > 0.0 ? lmax / lmin : 0.0;
    if (!(c > 1.0) || !std::isfinite(c)) return 2;
    const double sc = std::sqrt(c), s = (sc - 1.0) / (sc + 1.0);
    int k = 2;
    while (k < 64 && 2.0 * std::pow(s, k) > 0.3) ++k;
    return k;
}

double default_tol(const cuth_options &o, double dt) {
    // tol == 0 selects the default of the precision: mixed, relative rise error
    // 1e-8; FP64, relative residual 1e-10 (steady) or 1e-12 (transient, where
    // ||b|| is dominated by the C/dt T_n term and the residual bound is looser)
    if (o.tol > 0.0) return o.tol;
    const bool mixed = o.precision == CUTH_MIXED || o.precision == CUTH_MIXED16;
    return mixed ? 1e-8 : (dt > 0.0 ? 1e-12 : 1e-10);
}

// The residual accepted when an FP64 or stage-switched solve stalls above its
// tolerance: the steady default for a transient solve left at its default.  As
// dt grows the step approaches the steady system, whose FP64 residual floor
// (about machine epsilon times the condition number) can lie above 1e-12: a
// 64-layer stack stalled at 1.1e-12 with dt = 1 s and 4.2e-12 with dt = 100 s.
double relaxed_tol(const cuth_options &o, double dt) {
    const bool fp64_like = o.precision == CUTH_FP64 || o.precision == CUTH_ADAPTIVE;
    return (o.tol > 0.0 || dt <= 0.0 || !fp64_like) ? 0.0 : 1e-10;
}

void fill_stats(const Problem &p, cuth_stats *stats, float ms_setup, float ms_solve) {
    if (!stats) return;
    stats->cheb_degree = p.cc.k > 0 ? p.cc.k : 1;
    stats->outer_cycles = p.cycles;
    stats->cg_iters = p.cg_iters;
    stats->stencil_applies = p.stencils;
    stats->stop_reason = p.reason;
    stats->drift_stops = p.drift_stops;
    stats->stagnation_stops = p.stag_stops;
    stats->rel_residual = p.relres;
    stats->err_est = p.err_est;
    stats->setup_ms = ms_setup;
    stats->solve_ms = ms_solve;
    stats->alg_bytes = p.bytes;
    stats->lambda_min = is_cheb(p.pm) ? p.ilo : p.su->lmin;
    stats->lambda_max = is_cheb(p.pm) ? p.ihi : p.su->lmax;
}

// Run the refinement for a set of problems on the engine's own stream (waiting
// for `user` first, and making `user` wait for the result).
Status run_set(Engine &E, std::vector<Problem *> &ps, hipStream_t user, const Shape &sh32,
               const Shape &sh64, const cuth_options &o, int period, bool use_graph, Grid *prof,
               const Shape *sh64_inner = nullptr) {
    const hipStream_t s = E.own;
    CUTH_HIP(hipEventRecord(E.ev_in, user));
    CUTH_HIP(hipStreamWaitEvent(s, E.ev_in, 0));
    Status st;
    // Jacobi and no preconditioning are single passes (degree-1 path)
    const int k = is_cheb(o.preconditioner) ? o.cheb_degree : 1;
    if (o.precision == CUTH_ADAPTIVE)
        st = run_staged(E, ps, sh32, sh64, k, o, period, s);
    else if (o.precision != CUTH_FP64)
        st = run_refinement<float>(E, ps, sh32, sh64, k, o, period, use_graph, s, prof);
    else
        st = run_refinement<double>(E, ps, sh64_inner ? *sh64_inner : sh64, sh64, k, o, period,
                                    use_graph, s, prof);
    if (st.code == CUTH_E_DEVICE || st.code == CUTH_E_NOMEM) return st;
    for (Problem *p : ps)
        if (p->th_final) {
            launch_add_scalar(p->g->N, p->th_final, p->out_off, p->out, s);
            p->bytes += 16.0 * (double)p->g->N;
        }
    CUTH_HIP(hipEventRecord(E.ev_out, s));
    CUTH_HIP(hipStreamWaitEvent(user, E.ev_out, 0));
    CUTH_TRY(sync_stream(s));
    return st;
}

}  // namespace

// ------------------------------------------------------------------- solve
Status solve_system(Grid &g, double dt, const double *P, const double *Tn, const double *init,
                    double init_off, double *out, double out_off, const cuth_options &o_in,
                    cuth_stats *stats, bool transient_defaults) {
    Status st;
    cuth_options o = o_in;
    if (o.cheb_degree > g.eng.kcap) return Status::err(CUTH_E_INVALID, "cheb_degree above 256");
    CUTH_HIP(hipEventRecord(g.ev0, g.stream));
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    const bool cheb = is_cheb(o.preconditioner);
    double ilo = 0.0, ihi = 0.0;
    if (cheb) {
        CUTH_TRY(ensure_bounds(g, *su, o.lanczos_steps, o.preconditioner == CUTH_PC_CHEBYSHEV_JACOBI));
        pc_interval(*su, o.preconditioner, ilo, ihi);
    }
    if (o.cheb_degree == CUTH_DEGREE_AUTO) o.cheb_degree = cheb ? auto_degree(ilo, ihi) : 1;
    CUTH_HIP(hipEventRecord(g.ev1, g.stream));
    if (o.precision == CUTH_FP64 || o.precision == CUTH_ADAPTIVE) CUTH_TRY(alloc_work(g.w64, g.N));
    Problem p;
    p.g = &g;
    p.su = su;
    p.cc = cheb ? make_cheb(ilo, ihi, o.cheb_degree) : ChebConsts{};
    p.ilo = ilo;
    p.ihi = ihi;
    p.pm = o.preconditioner;
    p.P = P;
    p.Tn = Tn;
    p.init = init;
    p.init_off = init_off;
    p.out = out;
    p.out_off = out_off;
    p.w32 = g.w32;
    p.w64 = g.w64;
    // the stage-switched scheme's preconditioner reads FP16 conductances too
    p.h16 = o.precision == CUTH_MIXED16 || o.precision == CUTH_ADAPTIVE;
    p.fixed32 = o.precision == CUTH_FP32;
    // CSR products: one row per lane (vx 1, one layer per lane, 4 wavefronts
    // per workgroup, as the plain CSR kernel); the engine grows to this shape's
    // number of workgroups if it has fewer slots
    const Shape sh_csr{1, 4, 1};
    if (o.storage == CUTH_STORAGE_CSR) {
        CUTH_TRY(ensure_csr(g, *su));
        p.csr = true;
        const size_t need = (size_t)prob_tiles(g, sh_csr);
        if (8 * need > g.eng.slot_doubles) {
            Engine bigger;
            Status es = engine_alloc(bigger, 1, g.eng.kcap, need);
            if (es.bad()) {
                engine_free(bigger);
                return es;
            }
            engine_free(g.eng);
            g.eng = bigger;
        }
    }
    p.thA = g.thA;
    p.thB = g.thB;
    p.tol = default_tol(o, dt);
    p.tol_relax = relaxed_tol(o, dt);
    p.th_in = init;
    p.in_off = init_off;
    p.th_out = g.thA;
    std::vector<Problem *> ps{&p};
    const int period = o.check_period > 0 ? o.check_period : (transient_defaults ? 5 : 20);
    const int ge = graph_env();
    const bool use_graph = !g.prof && (ge == 1 || (ge < 0 && g.N <= kGraphMaxN));
    Shape sh32 = g.sh32;
    if (o.precision != CUTH_FP64 && fuse_env() != 0) {
        // fused pairs of general sweeps where they are faster on this grid
        CUTH_TRY(alloc_work(g.w32, g.N, true));
        p.w32 = g.w32;
        std::ostringstream sig;
        sig << "single " << g.nx << 'x' << g.ny << 'x' << g.nz << (g.per_cell ? " pc" : " mf")
            << (p.h16 && g.per_cell ? "16" : "") << ' ' << g.sh32.vx << ',' << g.sh32.by << ','
            << g.sh32.zc;
        const int kk = is_cheb(o.preconditioner) ? o.cheb_degree : 1;
        CUTH_TRY(tune_fuse<float>(g.eng, ps, kk, sh32, sig.str()));
    }
    Status rs = run_set(g.eng, ps, g.stream, sh32, g.sh64, o, period, use_graph, &g,
                        p.csr ? &sh_csr : nullptr);
    if (rs.code == CUTH_E_DEVICE || rs.code == CUTH_E_NOMEM) return rs;
    CUTH_HIP(hipEventRecord(g.ev2, g.stream));
    CUTH_TRY(sync_stream(g.stream));
    float ms_setup = 0, ms_solve = 0;
    (void)hipEventElapsedTime(&ms_setup, g.ev0, g.ev1);
    (void)hipEventElapsedTime(&ms_solve, g.ev1, g.ev2);
    fill_stats(p, stats, ms_setup, ms_solve);
    return p.status;
}

// --------------------------------------------------------------- batched solve
namespace {

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tuned;

// A launch shape the batched kernels accept for every problem: whole 16-byte
// (or narrower) lanes along each row, at most kMaxBY rows, and no more
// workgroups than the candidate shapes (vx 1, by 1, zc 4) that size the slots.
template <typename T>
bool shape_fits(const std::vector<Problem *> &ps, const Shape &sh) {
    if (!(sh.vx == 1 || sh.vx == 2 || (sh.vx == 4 && sizeof(T) == 4))) return false;
    if (sh.by < 1 || sh.by > kMaxBY || sh.zc < 4) return false;
    for (const Problem *p : ps)
        if (p->g->nx % sh.vx != 0) return false;
    return true;
}

// Pick the FP32 (or FP64) launch shape of a batch by timing the general
// Chebyshev sweep of every candidate on the batch itself; results are kept per
// batch signature for the process (and in the file named by CUTH_AUTOTUNE_CACHE).
template <typename T>
Status autotune(Engine &E, std::vector<Problem *> &ps, int kcheb, const std::string &sig,
                Shape &best) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(sig);
        if (it != g_tuned.end()) {
            best = it->second;
            return Status::ok();
        }
    }
    const char *cache = std::getenv("CUTH_AUTOTUNE_CACHE");
    if (cache) {
        if (FILE *f = std::fopen(cache, "r")) {
            char line[4096];
            while (std::fgets(line, sizeof line, f)) {
                std::string s(line);
                const size_t sp = s.rfind(' ');
                if (sp == std::string::npos || s.substr(0, sp) != sig) continue;
                int vx, by, zc;
                if (std::sscanf(s.c_str() + sp + 1, "%d,%d,%d", &vx, &by, &zc) == 3 &&
                    shape_fits<T>(ps, Shape{vx, by, zc})) {
                    best = Shape{vx, by, zc};
                    std::fclose(f);
                    std::lock_guard<std::mutex> lk(g_tune_mu);
                    g_tuned[sig] = best;
                    return Status::ok();
                }
            }
            std::fclose(f);
        }
    }
    int vmax = (sizeof(T) == 4) ? 4 : 2;
    for (Problem *p : ps)
        while (vmax > 1 && p->g->nx % vmax != 0) vmax /= 2;
    std::vector<Shape> cand;
    const int vxs[3] = {4, 2, 1};
    for (int vx : vxs) {
        if (vx > vmax) continue;
        for (int by : {1, 2})
            for (int zc : {4, 8, 16}) cand.push_back(Shape{vx, by, zc});
        if (cand.size() >= 6) break;
    }
    const hipStream_t s = E.own;
    hipEvent_t e0, e1;
    CUTH_HIP(hipEventCreate(&e0));
    CUTH_HIP(hipEventCreate(&e1));
    for (Problem *p : ps) p->inner = true;
    float best_ms = INFINITY;
    for (const Shape &sh : cand) {
        std::vector<int> which;
        const int nb = build_inner<T>(E, ps, sh, which);
        if (nb < 0) return Status::err(CUTH_E_DEVICE, "internal: autotune shape does not fit the engine");
        const int n = (int)which.size();
        CUTH_HIP(hipMemcpyAsync(Sel<T>::d(E), Sel<T>::h(E), sizeof(InnerProb<T>) * n,
                                hipMemcpyHostToDevice, s));
        CUTH_HIP(hipMemsetAsync(Sel<T>::ds(E), 0, sizeof(CgState<T>) * n, s));
        const bool pc = ps[0]->g->per_cell, h16 = pc && ps[0]->h16, jac = ps[0]->pm == CUTH_PC_CHEBYSHEV_JACOBI;
        for (int rep = 0; rep < 2; ++rep)
            launch_cheb_b<T>(Sel<T>::d(E), n, nb, pc, h16 ? CS_F16 : CS_OWN, jac, sh.vx, sh.by, 0, false, false, 2, zsel(1, 0),
                             eslot<T>(E, P_UPD), false, eslot<T>(E, P_CHEB), s);
        CUTH_HIP(hipEventRecord(e0, s));
        for (int rep = 0; rep < 6; ++rep)
            launch_cheb_b<T>(Sel<T>::d(E), n, nb, pc, h16 ? CS_F16 : CS_OWN, jac, sh.vx, sh.by, 0, false, false, 2,
                             zsel(rep & 1, 1 - (rep & 1)),
                             eslot<T>(E, P_UPD), false, eslot<T>(E, P_CHEB), s);
        CUTH_HIP(hipEventRecord(e1, s));
        CUTH_TRY(sync_stream(s));
        float ms = 0;
        CUTH_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (log_on()) std::fprintf(stderr, "cuth: autotune %d,%d,%d %.3f ms\n", sh.vx, sh.by, sh.zc, ms / 6);
        if (ms < best_ms * kTuneMargin) {
            best_ms = ms;
            best = sh;
        }
    }
    for (Problem *p : ps) p->inner = false;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)kcheb;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[sig] = best;
    if (cache)
        if (FILE *f = std::fopen(cache, "a")) {
            std::fprintf(f, "%s %d,%d,%d\n", sig.c_str(), best.vx, best.by, best.zc);
            std::fclose(f);
        }
    return Status::ok();
}

// Fused pairs or single sweeps for these problems (FP32 general sweeps), then
// fused triples on top of the pairs: the environment decides if it says so
// (fuse_env, fuse3_env), else timing on the problems themselves: the faster of
// four single sweeps and two fused pairs per candidate shape, then two fused
// triples per candidate against the pairs' time per sweep.  Cached per
// signature.  Needs the four iterate buffers.
template <typename T>
Status tune_fuse(Engine &E, std::vector<Problem *> &ps, int k, Shape &sh, const std::string &sig) {
    sh.fr = 0;
    sh.tr = 0;
    if (sizeof(T) != 4 || ps.empty()) return Status::ok();
    const int fe = fuse_env();
    int max_nx = 1;
    for (Problem *p : ps) max_nx = std::max(max_nx, p->g->nx);
    if (fe == 0) return Status::ok();
    if (fe == 1) {
        set_fuse(sh, max_nx);
        return Status::ok();
    }
    if (k < 6 || !is_cheb(ps[0]->pm)) return Status::ok();   // no pair of general sweeps
    for (Problem *p : ps)
        if (!Sel<T>::w(*p).zC || !Sel<T>::w(*p).zD) return Status::ok();
    // the triple setting is part of the key: a cached choice made with
    // triples allowed must not outlive CUTH_FUSE3=0, nor the reverse
    const int f3 = fuse3_env();
    // the preconditioner is part of the key too (the Jacobi-scaled sweeps are
    // other kernels)
    const std::string key = sig + (f3 == 0 ? " fuse no3" : f3 == 1 ? " fuse 3" : " fuse") + " pm" +
                            std::to_string(ps[0]->pm);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            sh.fr = it->second.fr;
            sh.fzc = it->second.fzc;
            sh.fwpr = it->second.fwpr;
            sh.tr = it->second.tr;
            sh.tzc = it->second.tzc;
            sh.twpr = it->second.twpr;
            return Status::ok();
        }
    }
    const bool pc = ps[0]->g->per_cell, h16 = pc && ps[0]->h16, jac = ps[0]->pm == CUTH_PC_CHEBYSHEV_JACOBI;
    const hipStream_t s = E.own;
    constexpr int kRounds = 5;
    hipEvent_t ev[kRounds + 1];
    for (hipEvent_t &e : ev) CUTH_HIP(hipEventCreate(&e));
    for (Problem *p : ps) p->inner = true;
    Status st = Status::ok();
    // milliseconds per general sweep of shape c with launches of `width`
    // sweeps (1, 2 or 3), from timed rounds after a warm-up round; a negative
    // value if the shape does not fit or its launch fails
    auto per_sweep = [&](const Shape &c, int width) -> float {
        std::vector<int> which;
        const int nb = build_inner<T>(E, ps, c, which);
        if (nb < 0) return -1.f;
        const int n = (int)which.size();
        const InnerProb<T> &last = Sel<T>::h(E)[n - 1];
        const int nbf = last.f_tile0 + last.f_ntiles, nbt = last.t_tile0 + last.t_ntiles;
        if (hipMemcpyAsync(Sel<T>::d(E), Sel<T>::h(E), sizeof(InnerProb<T>) * n,
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemsetAsync(Sel<T>::ds(E), 0, sizeof(CgState<T>) * n, s) != hipSuccess) {
            st = Status::err(CUTH_E_DEVICE, "tune_fuse: upload failed");
            return -1.f;
        }
        auto round = [&]() {
            if (width == 1) {
                for (int q = 0; q < 4; ++q)
                    launch_cheb_b<T>(Sel<T>::d(E), n, nb, pc, h16 ? CS_F16 : CS_OWN, jac, c.vx, c.by, 0, false, false, 3,
                                     zsel(q & 1, 1 - (q & 1)), eslot<T>(E, P_UPD), false,
                                     eslot<T>(E, P_CHEB), s);
            } else if constexpr (sizeof(T) == 4) {
                // two launches from j = 3 over the four buffers (reads N, P; writes X, Y)
                for (int q = 0; q < 2; ++q) {
                    const int zs = q == 0 ? 0 + 4 * 1 + 16 * 2 + 64 * 3 : 3 + 4 * 2 + 16 * 0 + 64 * 1;
                    if (width == 3)
                        launch_cheb3_b<T>(Sel<T>::d(E), n, nbt, pc, h16, jac, c.vx, c.tr, c.tzc, c.twpr, 3, zs, s);
                    else
                        launch_cheb2_b<T>(Sel<T>::d(E), n, nbf, pc, h16, jac, c.vx, c.fr, c.fzc, c.fwpr, 3, zs, s);
                }
            }
        };
        round();
        if (hipGetLastError() != hipSuccess) return -1.f;   // e.g. more LDS than a launch may take
        // the median of kRounds separately timed rounds (one slow round, e.g.
        // a clock change, does not move it)
        (void)hipEventRecord(ev[0], s);
        for (int rep = 0; rep < kRounds; ++rep) {
            round();
            (void)hipEventRecord(ev[rep + 1], s);
        }
        if (hipStreamSynchronize(s) != hipSuccess) {
            st = Status::err(CUTH_E_DEVICE, "tune_fuse: timing launch failed");
            return -1.f;
        }
        float t[kRounds];
        for (int rep = 0; rep < kRounds; ++rep) {
            t[rep] = 0.f;
            (void)hipEventElapsedTime(&t[rep], ev[rep], ev[rep + 1]);
        }
        std::sort(t, t + kRounds);
        const float sw = t[kRounds / 2] / (width == 1 ? 4 : 2 * width);
        if (log_on())
            std::fprintf(stderr, "cuth: fuse width %d shape %d,%d,%d %.4f ms per sweep\n", width,
                         width == 3 ? c.tr : c.fr, width == 3 ? c.tzc : c.fzc,
                         width == 3 ? c.twpr : c.fwpr, sw);
        return sw;
    };
    float best_sw = INFINITY;
    Shape best = sh;
    // candidates (R, zc, wcap): rows per workgroup, layers per chunk, and 0 for
    // whole rows or the wavefronts per row of an x window; shapes that fit to
    // the same workgroup as an earlier candidate are skipped
    std::vector<Shape> tried;
    auto seen = [&](const Shape &c, bool triple) {
        for (const Shape &t : tried) {
            if (!triple && t.tr == 0 && t.fr == c.fr && t.fzc == c.fzc && t.fwpr == c.fwpr) return true;
            if (triple && t.tr > 0 && t.tr == c.tr && t.tzc == c.tzc && t.twpr == c.twpr) return true;
        }
        tried.push_back(c);
        return false;
    };
    const int cand[][3] = {{0, 0, 0}, {4, 8, 0}, {2, 8, 0}, {2, 16, 0}, {4, 4, 0}, {1, 16, 0},
                           {8, 8, 1}, {14, 10, 1}, {6, 8, 2}};
    for (const auto &cd : cand) {
        Shape c = sh;
        c.fr = 0;
        c.tr = 0;
        if (cd[0] > 0 && (!fuse_fit(c, max_nx, cd[0], cd[1], cd[2]) || seen(c, false))) continue;
        const float sw = per_sweep(c, cd[0] > 0 ? 2 : 1);
        if (st.bad()) break;
        if (sw >= 0.f && sw < best_sw * kTuneMargin) {
            best_sw = sw;
            best = c;
        }
    }
    // fused triples where a triple fits before the last sweep (degree 6 and
    // up: the first triple covers sweeps 2-4 and ends before the last sweep),
    // timed against the winner so far, single sweeps or pairs.  Triples run
    // with pairs for the sweeps a triple does not fill: where single sweeps
    // won, a candidate brings the pairs of the smallest shape (any leftover is
    // at most one launch per application)
    Shape base3 = best;
    bool have3 = best.fr > 0;
    if (!have3) have3 = fuse_fit(base3, max_nx, 2, 8);
    if (!st.bad() && f3 == 1 && best.fr == 0 && have3) best = base3;
    if (!st.bad() && have3 && f3 != 0 && k >= 6) {
        const int cand3[][3] = {{4, 8, 0}, {2, 8, 0}, {4, 16, 0}, {12, 10, 1}, {12, 20, 1},
                                {8, 20, 1}, {8, 10, 1}, {4, 10, 2}};
        for (const auto &cd : cand3) {
            Shape c = base3;
            if (!fuse3_fit(c, max_nx, cd[0], cd[1], cd[2]) || seen(c, true)) continue;
            const float sw = per_sweep(c, 3);
            if (st.bad()) break;
            if (sw >= 0.f && (f3 == 1 || sw < best_sw * kTuneMargin3)) {
                best_sw = sw;
                best = c;
                if (f3 == 1) break;
            }
        }
    }
    if (log_on())
        std::fprintf(stderr, "cuth: fuse choice pairs %d,%d,%d triples %d,%d,%d\n", best.fr, best.fzc,
                     best.fwpr, best.tr, best.tzc, best.twpr);
    for (Problem *p : ps) p->inner = false;
    for (hipEvent_t &e : ev) (void)hipEventDestroy(e);
    if (st.bad()) return st;
    sh = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
    return Status::ok();
}

}  // namespace

Status solve_batch(int nsys, Grid *const *grids, int nrhs, const double *const *P,
                   double *const *T, const cuth_options &o_in, cuth_stats *stats) {
    cuth_options o = o_in;
    if (o.cheb_degree > 256) return Status::err(CUTH_E_INVALID, "cheb_degree above 256");
    const bool mixed = o.precision == CUTH_MIXED || o.precision == CUTH_MIXED16 || o.precision == CUTH_FP32;
    const bool staged = o.precision == CUTH_ADAPTIVE;
    const hipStream_t user = grids[0]->stream;
    // per-system setup (Lanczos bounds cached in each grid)
    std::vector<Setup *> sus(nsys);
    for (int s = 0; s < nsys; ++s) {
        Status st;
        sus[s] = get_setup(*grids[s], 0.0, st);
        if (!sus[s]) return st;
        if (is_cheb(o.preconditioner))
            CUTH_TRY(ensure_bounds(*grids[s], *sus[s], o.lanczos_steps,
                                   o.preconditioner == CUTH_PC_CHEBYSHEV_JACOBI));
    }
    if (o.cheb_degree == CUTH_DEGREE_AUTO) {
        int k = 1;
        if (is_cheb(o.preconditioner))
            for (int s = 0; s < nsys; ++s) {
                double lo, hi;
                pc_interval(*sus[s], o.preconditioner, lo, hi);
                k = std::max(k, auto_degree(lo, hi));
            }
        o.cheb_degree = k;
    }
    // problems grouped by coefficient storage (one launch family per group)
    Status result = Status::ok();
    for (int group = 0; group < 2; ++group) {
        std::vector<int> sys;
        for (int s = 0; s < nsys; ++s)
            if ((int)grids[s]->per_cell == group) sys.push_back(s);
        if (sys.empty()) continue;
        const int np = (int)sys.size() * nrhs;
        std::vector<Problem> probs(np);
        std::vector<Problem *> ps(np);
        int64_t ntot = 0;
        for (int s : sys) ntot += grids[s]->N * nrhs;
        // FP32 pools hold two more iterates when general sweeps run as fused pairs
        const bool fuse32 = (mixed || staged) && fuse_env() != 0;
        const int nvec = fuse32 ? 10 : 8;
        std::ostringstream sig;
        const bool h16 = group == 1 && (o.precision == CUTH_MIXED16 || staged);
        sig << (mixed ? "f32" : staged ? "f64s" : "f64") << (group ? (h16 ? "pc16" : "pc") : "mf");
        for (int s : sys) sig << ' ' << grids[s]->nx << 'x' << grids[s]->ny << 'x' << grids[s]->nz;
        sig << " r" << nrhs;
        // workgroup slots: the largest of the candidate launch shapes
        size_t nb_max = kRedBlocks;
        for (int s : sys)
            nb_max += (size_t)nrhs * tiles_x(grids[s]->nx, 1) * grids[s]->ny * tiles_z(grids[s]->nz, 4);
        // the tuners' timed sweeps read the constants of sweeps up to j = 5, so
        // the constant rows hold at least 6 sweeps whatever the degree
        const int kcap = std::max(o.cheb_degree, 6);
        // pooled work vectors and the engine, kept by the first grid for the
        // next call with the same signature
        BatchPool &bp = grids[sys[0]]->batch[group];
        std::ostringstream pkey;
        pkey << sig.str() << " v" << nvec << " k" << kcap;
        Status st;
        if (bp.key != pkey.str()) {
            batch_pool_free(bp);
            st = dev_alloc(&bp.poolth, (size_t)ntot * 2);
            if (!st.bad() && (mixed || staged)) st = dev_alloc(&bp.pool32, (size_t)ntot * nvec);
            if (!st.bad() && !mixed) st = dev_alloc(&bp.pool64, (size_t)ntot * nvec);
            if (!st.bad()) st = engine_alloc(bp.E, np, kcap, nb_max);
            if (st.bad()) {
                batch_pool_free(bp);
                return st;
            }
            bp.key = pkey.str();
        }
        float *pool32 = bp.pool32;
        double *pool64 = bp.pool64, *poolth = bp.poolth;
        Engine &E = bp.E;
        int64_t off = 0;
        int n = 0;
        for (int s : sys) {
            Grid &g = *grids[s];
            for (int q = 0; q < nrhs; ++q, ++n) {
                Problem &p = probs[n];
                p.g = &g;
                p.su = sus[s];
                if (is_cheb(o.preconditioner)) {
                    pc_interval(*sus[s], o.preconditioner, p.ilo, p.ihi);
                    p.cc = make_cheb(p.ilo, p.ihi, o.cheb_degree);
                }
                p.pm = o.preconditioner;
                p.P = P[s] + (int64_t)q * g.N;
                p.out = T[s] + (int64_t)q * g.N;
                p.out_off = g.t_amb;
                p.init = o.use_initial_guess ? p.out : nullptr;
                p.init_off = g.t_amb;
                const int64_t N = g.N;
                auto carve32 = [&](Work<float> &w) {
                    float *b = pool32 + off * nvec;
                    float **v[] = {&w.x, &w.r, &w.rhat, &w.pA, &w.pB, &w.mu, &w.zA, &w.zB, &w.zC, &w.zD};
                    for (int i = 0; i < nvec; ++i) *v[i] = b + (int64_t)i * N;
                };
                auto carve64 = [&](Work<double> &w) {
                    double *b = pool64 + off * nvec;
                    double **v[] = {&w.x, &w.r, &w.rhat, &w.pA, &w.pB, &w.mu, &w.zA, &w.zB};
                    for (int i = 0; i < 8; ++i) *v[i] = b + (int64_t)i * N;
                };
                if (mixed || staged) carve32(p.w32);
                if (!mixed) carve64(p.w64);
                p.thA = poolth + off * 2;
                p.thB = p.thA + N;
                off += N;
                p.tol = default_tol(o, 0.0);
                p.h16 = h16;
                p.fixed32 = o.precision == CUTH_FP32;
                p.th_in = p.init;
                p.in_off = p.init_off;
                p.th_out = p.thA;
                ps[n] = &p;
            }
        }
        // inner shape: autotuned on the problems' own inner work vectors; the
        // FP64 residual (once per refinement cycle) uses a fixed shape in mixed
        // precision, since no FP64 work vectors exist then
        Shape sh_in, sh64{2, 1, 8};
        for (Problem *p : ps)
            while (sh64.vx > 1 && p->g->nx % sh64.vx != 0) sh64.vx /= 2;
        // (the stage-switched scheme tunes its FP32 preconditioner's shape)
        Status ts = (mixed || staged)
                        ? autotune<float>(E, ps, o.cheb_degree, sig.str() + " in", sh_in)
                        : autotune<double>(E, ps, o.cheb_degree, sig.str() + " in", sh_in);
        if (!mixed && !staged) sh64 = sh_in;
        if (fuse32 && !ts.bad()) {
            const int kk = is_cheb(o.preconditioner) ? o.cheb_degree : 1;
            for (Problem *p : ps) p->pm = o.preconditioner;
            ts = tune_fuse<float>(E, ps, kk, sh_in, sig.str());
        }
        if (!ts.bad()) {
            const int period = o.check_period > 0 ? o.check_period : 20;
            const bool use_graph = graph_env() != 0;
            ts = run_set(E, ps, user, sh_in, sh64, o, period, use_graph, nullptr);
        }
        if (ts.code == CUTH_E_DEVICE || ts.code == CUTH_E_NOMEM) batch_pool_free(bp);
        if (ts.code == CUTH_E_DEVICE || ts.code == CUTH_E_NOMEM || ts.code == CUTH_E_INVALID) return ts;
        n = 0;
        for (int s : sys)
            for (int q = 0; q < nrhs; ++q, ++n) {
                fill_stats(probs[n], stats ? &stats[(int64_t)s * nrhs + q] : nullptr, 0.f, 0.f);
                if (probs[n].status.bad() && !result.bad()) result = probs[n].status;
            }
    }
    return result;
}

// ------------------------------------------------------------ step-level calls
Status apply_op(Grid &g, double dt, int precision, const void *x, void *y) {
    Status st;
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    if (precision != CUTH_FP64)
        launch_apply<float>(view32(g, *su, precision == CUTH_MIXED16), (const float *)x, (float *)y,
                            g.stream);
    else launch_apply<double>(view64(g, *su), (const double *)x, (double *)y, g.stream);
    CUTH_HIP(hipGetLastError());
    return sync_stream(g.stream);
}

// CSR copy of a setup's FP64 operator, built once on first use: row pointers on
// the host (1 + one entry per existing face neighbour), columns and values by
// k_csr_fill on the device.
Status ensure_csr(Grid &g, Setup &su) {
    if (su.csr_ptr) return Status::ok();
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    std::vector<int> ptr((size_t)g.N + 1);
    int64_t k = 0;
    size_t r = 0;
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                ptr[r++] = (int)k;
                k += 1 + (i > 0) + (i < nx - 1) + (j > 0) + (j < ny - 1) + (l > 0) + (l < nz - 1);
                if (k >= ((int64_t)1 << 31) - 1)
                    return Status::err(CUTH_E_INVALID, "CSR needs fewer than 2^31 nonzeros");
            }
    ptr[r] = (int)k;
    int *p = nullptr, *c = nullptr;
    double *v = nullptr;
    Status st = dev_alloc(&p, ptr.size());
    if (!st.bad()) st = dev_alloc(&c, (size_t)k);
    if (!st.bad()) st = dev_alloc(&v, (size_t)k);
    if (st.bad()) {
        dev_free(p);
        dev_free(c);
        dev_free(v);
        return st;
    }
    su.csr_ptr = p;
    su.csr_col = c;
    su.csr_val = v;
    su.csr_nnz = k;
    CUTH_HIP(hipMemcpy(p, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice));
    launch_csr_fill(view64(g, su), p, c, v, g.stream);
    CUTH_HIP(hipGetLastError());
    return sync_stream(g.stream);
}

Status apply_csr(Grid &g, double dt, const double *x, double *y) {
    Status st;
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    CUTH_TRY(ensure_csr(g, *su));
    launch_csr_spmv(g.N, su->csr_ptr, su->csr_col, su->csr_val, x, y, g.stream);
    CUTH_HIP(hipGetLastError());
    return sync_stream(g.stream);
}

Status residual(Grid &g, double dt, const double *b, const double *T, double *r) {
    Status st;
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    Engine &E = g.eng;
    OuterProb<double, double> o;
    o.op = view64(g, *su);
    o.ntx = tiles_x(g.nx, g.sh64.vx);
    o.ntz = tiles_z(g.nz, g.sh64.zc);
    o.tile0 = 0;
    o.ntiles = prob_tiles(g, g.sh64);
    o.th_in = T;
    o.in_off = g.t_amb;
    o.delta = nullptr;
    o.P = b;
    o.Tn = nullptr;
    o.tn_off = 0.0;
    o.th_out = nullptr;
    o.r64 = r;
    o.r_in = nullptr;
    o.rhat = nullptr;
    E.h_out64[0] = o;
    CUTH_HIP(hipMemcpyAsync(E.out64, E.h_out64, sizeof(o), hipMemcpyHostToDevice, g.stream));
    launch_residual_b<double, double>(E.out64, 1, o.ntiles, g.per_cell, g.sh64.vx, g.sh64.by,
                                      residual_flags(o), eslot<double>(E, P_RES), g.stream);
    CUTH_HIP(hipGetLastError());
    return sync_stream(g.stream);
}

template <typename T>
static Status precond_typed(Grid &g, Setup &su, Work<T> &w, const Shape &sh, const ChebConsts &cc,
                            int pm, bool h16, const T *r, T *z) {
    // the result lands in the buffer the sweep rotation ends in (fused pairs
    // exactly where enqueue_precond uses them: FP32)
    Engine &E = g.eng;
    const bool h16e = h16 && g.per_cell;
    const int zfin = precond_final(cc.k, pm, fuse_for<T>(sh, pm));
    Problem p;
    p.g = &g;
    p.su = &su;
    p.cc = cc;
    p.pm = pm;
    p.h16 = h16e;
    Work<T> &pw = Sel<T>::w(p);
    pw = w;
    pw.r = const_cast<T *>(r);
    T **zs[4] = {&pw.zA, &pw.zB, &pw.zC, &pw.zD};
    *zs[zfin] = z;
    p.inner = true;
    std::vector<Problem *> ps{&p};
    std::vector<int> which;
    const int nb = build_inner<T>(E, ps, sh, which);
    if (nb < 0) return Status::err(CUTH_E_DEVICE, "internal: preconditioner does not fit the engine");
    CUTH_TRY(upload_cheb<T>(E, ps, g.stream));
    CUTH_HIP(hipMemcpyAsync(Sel<T>::d(E), Sel<T>::h(E), sizeof(InnerProb<T>), hipMemcpyHostToDevice,
                            g.stream));
    CgState<T> *hs = Sel<T>::hs(E);
    std::memset(hs, 0, sizeof(CgState<T>));
    CUTH_HIP(hipMemcpyAsync(Sel<T>::ds(E), hs, sizeof(CgState<T>), hipMemcpyHostToDevice, g.stream));
    const int got = enqueue_precond<T>(E, 1, nb, g.per_cell, p.h16 ? CS_F16 : CS_OWN, pm, sh, cc.k,
                                       false, false, g.stream, nullptr);
    if (got != zfin) return Status::err(CUTH_E_DEVICE, "internal: preconditioner buffer mismatch");
    CUTH_HIP(hipGetLastError());
    return sync_stream(g.stream);
}

Status precond_apply(Grid &g, double dt, int precision, int pm, double lmin, double lmax,
                     int degree, const void *r, void *z) {
    Status st;
    if (degree > g.eng.kcap) return Status::err(CUTH_E_INVALID, "degree above 256");
    Setup *su = get_setup(g, dt, st);
    if (!su) return st;
    // Jacobi and none are single passes; their degree is 1 (the constants are unused)
    const ChebConsts cc = make_cheb(lmin, lmax, is_cheb(pm) ? degree : 1);
    if (precision != CUTH_FP64) {
        Shape sh32 = g.sh32;
        set_fuse(sh32, g.nx);
        if (sh32.fr > 0) CUTH_TRY(alloc_work(g.w32, g.N, true));
        return precond_typed<float>(g, *su, g.w32, sh32, cc, pm, precision == CUTH_MIXED16,
                                    (const float *)r, (float *)z);
    }
    CUTH_TRY(alloc_work(g.w64, g.N));
    return precond_typed<double>(g, *su, g.w64, g.sh64, cc, pm, false, (const double *)r,
                                 (double *)z);
}

// Scratch layout of one allocation-free preconditioner application: each part
// starts on a 256-byte boundary.
struct NoAllocLayout {
    size_t desc = 0, state = 0, cheb = 0, layers = 0, part = 0, iter = 0, total = 0;
    size_t slot_doubles = 0;
};

template <typename T>
static NoAllocLayout noalloc_layout(const Grid &g, int kcap, int nb) {
    NoAllocLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~size_t(255);
        return o;
    };
    L.desc = take(sizeof(InnerProb<T>));
    L.state = take(sizeof(CgState<T>));
    L.cheb = take(sizeof(T) * (1 + 2 * (size_t)kcap));
    L.layers = take(sizeof(LayerCoef<T>) * (size_t)g.nz);
    L.slot_doubles = std::max<size_t>(8 * (size_t)std::max(nb, 1), 3);
    L.part = take(sizeof(double) * L.slot_doubles * P_SLOTS);
    L.iter = take(sizeof(T) * (size_t)g.N);
    L.total = off;
    return L;
}

// z = M^{-1} r as precond_typed runs it with single sweeps, but every buffer
// the kernels use besides r, z and the grid's planes (the problem descriptor,
// its state, the sweep constants, the layer coefficients of dt, the partials
// and the one iterate that is not z) lives in the scratch array; the small ones
// are written there by kernel arguments.  The state is cleared on every call.
template <typename T>
static Status precond_noalloc_typed(Grid &g, double dt, const ChebConsts &cc, int pm, bool h16,
                                    const T *r, T *z) {
    Shape sh = sizeof(T) == 4 ? g.sh32 : g.sh64;
    sh.fr = 0;
    sh.tr = 0;
    const bool h16e = sizeof(T) == 4 && h16 && g.per_cell;
    const int kcap = std::max(cc.k, 1);
    const int nb = prob_tiles(g, sh);
    const NoAllocLayout L = noalloc_layout<T>(g, kcap, nb);
    if (L.total > kNoAllocScratchBytes)
        return Status::err(CUTH_E_INVALID,
                           "allocation-free preconditioner: this grid needs " + std::to_string(L.total) +
                               " bytes of scratch, above the " +
                               std::to_string(kNoAllocScratchBytes) + " the library holds per device");
    unsigned char *base = nullptr;
    CUTH_HIP(noalloc_scratch(g.device, &base));
    // host images of the small parts
    std::vector<LayerCoef<double>> hlc;
    double gersh = 0.0;
    layer_coefs(g, dt, hlc, gersh);
    std::vector<LayerCoef<T>> hl;
    if constexpr (sizeof(T) == 4) hl = layer_coefs32(hlc);
    else hl = hlc;
    std::vector<T> hc((size_t)1 + 2 * kcap, T(0));
    hc[0] = (T)cc.inv_th;
    for (int j = 1; j < cc.k; ++j) {
        hc[1 + j] = (T)cc.c1[j];
        hc[1 + kcap + j] = (T)cc.c2[j];
    }
    const int zfin = precond_final(cc.k, pm, 0);
    T *it = reinterpret_cast<T *>(base + L.iter);
    OpView<T> v{g.nx, g.ny, g.nz, nullptr, nullptr,
                reinterpret_cast<const LayerCoef<T> *>(base + L.layers), sh.vx, sh.by, sh.zc};
    if constexpr (sizeof(T) == 4) {
        if (g.per_cell) {
            v.gx = g.gx32;
            v.gy = g.gy32;
        }
        if (h16e) {
            v.hx = g.hx;
            v.hy = g.hy;
        }
    } else if (g.per_cell) {
        v.gx = g.gx64;
        v.gy = g.gy64;
    }
    InnerProb<T> d{};
    d.op = v;
    d.ntx = tiles_x(g.nx, sh.vx);
    d.ntz = tiles_z(g.nz, sh.zc);
    d.tile0 = 0;
    d.ntiles = nb;
    // the preconditioner's kernels read r and the iterates only; the CG
    // vectors point at the scratch iterate so that none is null
    d.x = d.rhat = d.mu = it;
    d.p[0] = d.p[1] = it;
    d.r = const_cast<T *>(r);
    for (T *&zz : d.z) zz = it;
    d.z[zfin] = z;
    d.st = reinterpret_cast<CgState<T> *>(base + L.state);
    d.cheb = reinterpret_cast<const T *>(base + L.cheb);
    d.kcap = kcap;
    const CgState<T> st0{};
    CUTH_HIP(launch_put(&d, sizeof d, base + L.desc, g.stream));
    CUTH_HIP(launch_put(&st0, sizeof st0, base + L.state, g.stream));
    CUTH_HIP(launch_put(hc.data(), sizeof(T) * hc.size(), base + L.cheb, g.stream));
    CUTH_HIP(launch_put(hl.data(), sizeof(LayerCoef<T>) * hl.size(), base + L.layers, g.stream));
    // an engine of one problem over the scratch (no host arrays: single sweeps
    // never read them)
    Engine E;
    E.cap = 1;
    E.kcap = kcap;
    E.slot_doubles = L.slot_doubles;
    E.part = reinterpret_cast<double *>(base + L.part);
    if constexpr (sizeof(T) == 4) {
        E.in32 = reinterpret_cast<InnerProb<float> *>(base + L.desc);
        E.st32 = reinterpret_cast<CgState<float> *>(base + L.state);
        E.cheb32 = reinterpret_cast<float *>(base + L.cheb);
    } else {
        E.in64 = reinterpret_cast<InnerProb<double> *>(base + L.desc);
        E.st64 = reinterpret_cast<CgState<double> *>(base + L.state);
        E.cheb64 = reinterpret_cast<double *>(base + L.cheb);
    }
    const int got = enqueue_precond<T>(E, 1, nb, g.per_cell, h16e ? CS_F16 : CS_OWN, pm, sh, cc.k,
                                       false, false, g.stream, nullptr);
    if (got != zfin) return Status::err(CUTH_E_DEVICE, "internal: preconditioner buffer mismatch");
    CUTH_HIP(hipGetLastError());
    return sync_stream(g.stream);
}

Status precond_apply_noalloc(Grid &g, double dt, int precision, int pm, double lmin, double lmax,
                             int degree, const void *r, void *z) {
    const ChebConsts cc = make_cheb(lmin, lmax, is_cheb(pm) ? degree : 1);
    if (precision != CUTH_FP64)
        return precond_noalloc_typed<float>(g, dt, cc, pm, precision == CUTH_MIXED16,
                                            (const float *)r, (float *)z);
    return precond_noalloc_typed<double>(g, dt, cc, pm, false, (const double *)r, (double *)z);
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
    CUTH_TRY(sync_stream(g.stream));
    return st;
}

}  // namespace cuth
