"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: values solved
by hand (tests/golden/hand_examples.json), closed forms (series-resistance
column, single-cell backward Euler, Chebyshev trig/hyperbolic form), invariants
(symmetry, row sums, energy balance, SPD), an independent algorithm (the
separable DCT solver, the full spectrum), library routines and brute force.
Several tests plant a mistake in a copy of an oracle routine and check that the
pin rejects it.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as w
from oracle import adjoint, assembly, cpu_cg, direct, krylov, transient

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _frac(s):
    return float(Fraction(s))


def _stack_from(ex):
    nz = len(ex["dz"])
    names = [f"m{l}" for l in range(nz)]
    mult = None
    if "k_lat_mult" in ex:
        mult = np.asarray(ex["k_lat_mult"], float).reshape(nz, ex["ny"], ex["nx"])
    return w.Stack(ex["nx"], ex["ny"], names, dx=ex["dx"], dy=ex["dy"], dz=np.array(ex["dz"]),
                   k_lat_mult=mult, h_top=ex["h_top"], h_bottom=ex["h_bottom"],
                   t_amb=ex["t_amb"], k_lat=np.array(ex["k_lat"]),
                   k_vert=np.array(ex["k_vert"]),
                   heat_cap=np.array(ex.get("heat_cap", [1.0] * nz)))


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def c0():
    st, P = w.config0()
    A = assembly.assemble(st)
    return st, P, A


@pytest.fixture(scope="module")
def c4s():
    st, P = w.config4_small()
    A = assembly.assemble(st)
    return st, P, A


# ----------------------------------------------------------------- assembly
@pytest.mark.parametrize("name", ["column_1x1x3", "pair_2x1x1"])
def test_hand_solved_steady(gold, name):
    ex = gold[name]
    st = _stack_from(ex)
    A = assembly.assemble(st)
    th = direct.solve_dense(A, np.array(ex["P"]))
    T = st.t_amb + th
    exp = np.array([_frac(s) for s in ex["T"]])
    np.testing.assert_allclose(T, exp, rtol=1e-14, atol=1e-13)


def test_hand_solved_transient(gold):
    ex = gold["cell_transient"]
    st = _stack_from(ex)
    th = np.zeros(1)
    for n, s in enumerate(ex["theta_steps"]):
        th = transient.step(st, np.array(ex["P"]), th, ex["dt"], solve=direct.solve_dense)
        assert th[0] == pytest.approx(_frac(s), rel=1e-14)
        # closed form theta_n = (P/hS) (1 - (c/(c+hS))^n)
        assert th[0] == pytest.approx(2.0 * (1.0 - (8.0 / 9.0) ** (n + 1)), rel=1e-14)


def test_exact_symmetry_and_row_sums(c4s):
    st, _, A = c4s
    assert abs(A - A.T).max() == 0.0
    ones = np.ones(A.shape[0])
    sink = assembly.convective_per_cell(st)
    diag = A.diagonal()
    assert np.all(np.abs(A @ ones - sink) <= 1e-13 * diag)
    # 7-point pattern: at most 7 entries per row, off-diagonals negative
    assert np.diff(A.indptr).max() == 7
    Acoo = A.tocoo()
    offd = Acoo.data[Acoo.row != Acoo.col]
    assert np.all(offd < 0)


def test_transient_row_sums(c0):
    st, _, _ = c0
    dt = 1e-4
    At = assembly.assemble(st, dt=dt)
    sink = assembly.convective_per_cell(st) + assembly.capacity_per_cell(st, dt)
    assert np.all(np.abs(At @ np.ones(At.shape[0]) - sink) <= 1e-13 * At.diagonal())


def test_energy_balance_steady(c0, c4s):
    for st, P, A in (c0, c4s):
        th = direct.solve_splu(A, assembly.rhs_steady(P))
        hs = assembly.convective_per_cell(st)
        injected = math.fsum(P.ravel())
        leaving = math.fsum(hs * th)
        assert abs(leaving - injected) <= 1e-12 * injected


def test_energy_balance_transient(c0):
    st, P, _ = c0
    dt = 1e-4
    A = assembly.assemble(st, dt=dt)
    th0 = np.zeros(st.n)
    th1 = transient.step(st, P, th0, dt, solve=direct.solve_splu, A=A)
    th2 = transient.step(st, P, th1, dt, solve=direct.solve_splu, A=A)
    cv = assembly.capacity_per_cell(st, dt)
    hs = assembly.convective_per_cell(st)
    inj = math.fsum(P.ravel())
    out = math.fsum(hs * th2) + math.fsum(cv * (th2 - th1))
    assert abs(out - inj) <= 1e-11 * inj


def _series_column(dz, kv, dxdy, h, q):
    """Rise of a laterally uniform column by series resistances (heat only
    leaves through the top): each interface carries the power below it."""
    nz = len(dz)
    th = np.zeros(nz)
    th[-1] = q.sum() / (h * dxdy)
    for l in range(nz - 2, -1, -1):
        r_half_lo = (dz[l] / 2.0) / (kv[l] * dxdy)
        r_half_hi = (dz[l + 1] / 2.0) / (kv[l + 1] * dxdy)
        th[l] = th[l + 1] + q[: l + 1].sum() * (r_half_lo + r_half_hi)
    return th


def test_slab_closed_form():
    layers = ["Si", "BEOL", "bond", "Si", "BEOL", "bond", "TIM", "Cu"]
    st = w.uniform_stack(7, 5, layers)
    st.dz = np.array([50e-6, 10e-6, 2e-6, 100e-6, 10e-6, 2e-6, 80e-6, 300e-6])
    q = np.array([2e-3, 0, 0, 1e-3, 0, 0, 0, 0])
    P = np.broadcast_to(q[:, None, None], st.shape).copy()
    A = assembly.assemble(st)
    th = direct.solve_dense(A, P.ravel()).reshape(st.shape)
    exp = _series_column(st.dz, st.k_vert, st.dx * st.dy, st.h_top, q)
    np.testing.assert_allclose(th, np.broadcast_to(exp[:, None, None], st.shape), rtol=1e-12)
    # laterally uniform: lateral conductances play no role
    st2 = w.uniform_stack(7, 5, layers)
    st2.dz = st.dz
    st2.k_lat = st.k_lat * 10.0
    th2 = direct.solve_dense(assembly.assemble(st2), P.ravel())
    np.testing.assert_allclose(th2, th.ravel(), rtol=1e-10)


def test_spd_and_planted_negative_conductance():
    st = w.uniform_stack(8, 6, ["Si", "BEOL", "TIM", "Cu"])
    A = assembly.assemble(st)
    M = A.toarray()
    assert np.linalg.eigvalsh(M)[0] > 0
    sla.cholesky(M, lower=True)
    bad = w.uniform_stack(8, 6, ["Si", "BEOL", "TIM", "Cu"])
    bad.k_lat = bad.k_lat.copy()
    bad.k_lat[1] = -50.0          # planted: negative conductivity in one layer
    with pytest.raises(np.linalg.LinAlgError):
        sla.cholesky(assembly.assemble(bad).toarray(), lower=True)


def test_separable_spectrum_matches_dense():
    st = w.uniform_stack(6, 5, ["Si", "BEOL", "bond", "Cu"])
    for dt in (None, 1e-4):
        A = assembly.assemble(st, dt=dt).toarray()
        ev = np.linalg.eigvalsh(A)
        sep = direct.all_eigenvalues(st, dt=dt)
        np.testing.assert_allclose(sep, ev, rtol=1e-10, atol=1e-12 * ev[-1])
        lo, hi = direct.exact_extremes(st, dt=dt)
        assert lo == pytest.approx(ev[0], rel=1e-9)
        assert hi == pytest.approx(ev[-1], rel=1e-12)


def test_solvers_agree(c0):
    st, P, A = c0
    b = assembly.rhs_steady(P)
    x_lu = direct.solve_splu(A, b)
    x_sep = direct.solve_separable(st, b)
    x_cg, it, rr = cpu_cg.jacobi_cg(A, b, rtol=1e-14)
    rise = np.abs(x_lu).max()
    assert np.abs(x_sep - x_lu).max() <= 1e-12 * rise
    assert np.abs(x_cg - x_lu).max() <= 1e-12 * rise
    assert rr < 1e-10


def test_dense_vs_splu_small():
    st = w.uniform_stack(9, 7, ["Si", "BEOL", "bond", "TIM", "Cu"])
    rng = np.random.default_rng(1)
    b = rng.uniform(0, 1e-3, st.n)
    A = assembly.assemble(st)
    x1 = direct.solve_dense(A, b)
    x2 = direct.solve_splu(A, b)
    x3 = direct.solve_separable(st, b)
    np.testing.assert_allclose(x2, x1, rtol=1e-11)
    np.testing.assert_allclose(x3, x1, rtol=1e-11)


def test_separable_transient_matches_lu():
    st = w.uniform_stack(10, 9, ["Si", "Si", "BEOL", "bond", "TIM", "Cu"])
    rng = np.random.default_rng(2)
    P = rng.uniform(0, 1e-3, st.n)
    thn = rng.uniform(0, 5, st.n)
    dt = 1e-4
    A = assembly.assemble(st, dt=dt)
    b = assembly.rhs_transient(st, P, thn, dt)
    np.testing.assert_allclose(direct.solve_separable(st, b, dt=dt), direct.solve_splu(A, b),
                               rtol=1e-12)


def test_metamorphic(c4s):
    st, P, A = c4s
    b = P.ravel()
    th = direct.solve_splu(A, b)
    # positivity (M-matrix): P >= 0 -> theta >= 0
    assert th.min() >= 0
    # linearity
    rng = np.random.default_rng(3)
    Q = rng.uniform(0, 1e-3, st.n)
    th2 = direct.solve_splu(A, 2.0 * b + 3.0 * Q)
    thq = direct.solve_splu(A, Q)
    np.testing.assert_allclose(th2, 2.0 * th + 3.0 * thq, rtol=1e-10, atol=1e-12 * th.max())
    # reciprocity
    i, j = 123, 3 * 4096 + 2000
    ei = np.zeros(st.n); ei[i] = 1.0
    ej = np.zeros(st.n); ej[j] = 1.0
    assert direct.solve_splu(A, ej)[i] == pytest.approx(direct.solve_splu(A, ei)[j], rel=1e-10)
    # x mirror: flip power and multiplier along x
    stm = w.Stack(st.nx, st.ny, st.layers, k_lat_mult=st.k_lat_mult[:, :, ::-1].copy())
    thm = direct.solve_splu(assembly.assemble(stm), P[:, :, ::-1].ravel())
    np.testing.assert_allclose(thm.reshape(st.shape)[:, :, ::-1].ravel(), th, rtol=1e-10)
    # scaling k, h by s scales theta by 1/s
    s = 3.0
    sts = w.Stack(st.nx, st.ny, st.layers, k_lat_mult=st.k_lat_mult, h_top=st.h_top * s,
                  k_lat=st.k_lat * s, k_vert=st.k_vert * s)
    ths = direct.solve_splu(assembly.assemble(sts), b)
    np.testing.assert_allclose(ths * s, th, rtol=1e-10)


def test_separable_steps_match_lu_and_single_steps():
    """The trajectory stepper (operator eliminated once, right-hand side formed
    in the DCT basis) against a chain of SuperLU steps of the assembled
    transient matrix, over six steps with a floorplan switch; and one stepper
    step against the plain separable step."""
    st = w.config2_stack(24, 17)
    dt = 1e-4
    maps = [w.config2_power(st, f) for f in (0, 3)]
    A = assembly.assemble(st, dt=dt)
    stp = transient.SeparableSteps(st, dt)
    th_lu = np.zeros(st.n)
    th_hat = stp.to_hat(np.zeros(st.n))
    maps_hat = [stp.to_hat(m) for m in maps]
    for s in range(6):
        f = s // 3
        th_lu = transient.step(st, maps[f], th_lu, dt, solve=direct.solve_splu, A=A)
        th_hat = stp.step_hat(maps_hat[f], th_hat)
        got = stp.from_hat(th_hat)
        assert np.abs(got - th_lu).max() <= 1e-12 * np.abs(th_lu).max()
    one = stp.step(maps[1], th_lu)
    ref = transient.step(st, maps[1], th_lu, dt)
    assert np.abs(one - ref).max() <= 1e-13 * np.abs(ref).max()


def test_transient_converges_to_steady():
    st = w.uniform_stack(6, 6, ["Si", "BEOL", "TIM", "Cu"])
    rng = np.random.default_rng(4)
    P = rng.uniform(0, 1e-3, st.n)
    ths = direct.solve_separable(st, P)
    th = np.zeros(st.n)
    dt = 1.0   # long steps: contraction toward the fixed point
    for _ in range(400):
        th = transient.step(st, P, th, dt)
    np.testing.assert_allclose(th, ths, rtol=1e-9)


# ----------------------------------------------------------------- Chebyshev
def _cheb_recurrence(k, t):
    c0, c1 = np.ones_like(t), t.copy()
    if k == 0:
        return c0
    for _ in range(k - 1):
        c0, c1 = c1, 2.0 * t * c1 - c0
    return c1


@pytest.mark.parametrize("k", [0, 1, 2, 5, 30])
def test_chebyshev_closed_form_vs_three_term(k):
    t = np.concatenate([np.linspace(-1, 1, 41), [1.0001, 1.3, 2.5, -1.2]])
    np.testing.assert_allclose(krylov.chebyshev_first_kind(k, t), _cheb_recurrence(k, t),
                               rtol=1e-9, atol=1e-12)


def _diag_matvec(d):
    return lambda v: d * v


@pytest.mark.parametrize("k", [1, 2, 3, 10, 30])
def test_chebyshev_precondition_diagonal(k):
    rng = np.random.default_rng(k)
    lmin, lmax = 0.5, 40.0
    lam = np.concatenate([np.linspace(lmin, lmax, 50), rng.uniform(0.01, 60.0, 30)])
    r = rng.standard_normal(lam.size)
    z = krylov.chebyshev_precondition(_diag_matvec(lam), r, lmin, lmax, k)
    exp = (1.0 - krylov.chebyshev_residual_poly(lam, lmin, lmax, k)) / lam * r
    np.testing.assert_allclose(z, exp, rtol=1e-10, atol=1e-13)


def _mutant_precondition(matvec, r_cg, lmin, lmax, k, flip):
    """Copy of the algorithm with one planted mistake."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    r_ch = r_cg.copy()
    sigma1 = theta / delta
    rho = 1.0 / sigma1
    d = r_ch / theta
    z = np.zeros_like(r_ch)
    for _ in range(k):
        z = z + d
        r_ch = r_ch - matvec(d) if flip != "sign" else r_ch + matvec(d)
        rho_next = 1.0 / (2.0 * sigma1 - rho) if flip != "rho" else 1.0 / (2.0 * sigma1 + rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * r_ch
        rho = rho_next
    return z


@pytest.mark.parametrize("flip", ["sign", "rho"])
def test_chebyshev_pin_rejects_planted_mistake(flip):
    lam = np.linspace(0.5, 40.0, 60)
    r = np.random.default_rng(5).standard_normal(lam.size)
    z = _mutant_precondition(_diag_matvec(lam), r, 0.5, 40.0, 8, flip)
    exp = (1.0 - krylov.chebyshev_residual_poly(lam, 0.5, 40.0, 8)) / lam * r
    assert not np.allclose(z, exp, rtol=1e-6)


def test_chebyshev_symmetric_and_on_eigenmodes():
    st = w.uniform_stack(8, 6, ["Si", "BEOL", "TIM", "Cu"])
    A = assembly.assemble(st)
    M = A.toarray()
    ev, V = np.linalg.eigh(M)
    lmin, lmax = ev[5], 1.02 * ev[-1]
    mv = lambda v: A @ v
    rng = np.random.default_rng(6)
    u, v = rng.standard_normal((2, st.n))
    Mu = krylov.chebyshev_precondition(mv, u, lmin, lmax, 30)
    Mv = krylov.chebyshev_precondition(mv, v, lmin, lmax, 30)
    assert v @ Mu == pytest.approx(u @ Mv, rel=1e-10)
    for q in (0, 3, 50, st.n - 1):
        z = krylov.chebyshev_precondition(mv, V[:, q], lmin, lmax, 30)
        fac = (1.0 - krylov.chebyshev_residual_poly(np.array([ev[q]]), lmin, lmax, 30)[0]) / ev[q]
        np.testing.assert_allclose(z, fac * V[:, q], rtol=1e-7, atol=1e-9 * abs(fac))
        assert fac > 0


# -------------------------------------------------------------------- Lanczos
def test_lanczos_reproduces_diagonal_spectrum():
    d = np.array([1.0, 2.0, 3.5, 7.0, 11.0, 12.5])
    v0 = np.ones(d.size)
    a, b = krylov.lanczos(_diag_matvec(d), v0, d.size)
    np.testing.assert_allclose(krylov.ritz_values(a, b), d, rtol=1e-10)


def test_lanczos_ritz_interlace(c0):
    st, _, A = c0
    lo, hi = direct.exact_extremes(st)
    a, b = krylov.lanczos(lambda v: A @ v, w.lanczos_start(st.n), 30)
    ritz = krylov.ritz_values(a, b)
    assert ritz[0] >= lo * (1 - 1e-12)
    assert ritz[-1] <= hi * (1 + 1e-12)
    assert ritz[-1] >= 0.99 * hi
    lmin, lmax = krylov.spectral_bounds(A, w.lanczos_start(st.n))
    assert lmax >= hi                        # safe upper bound
    assert lmax <= krylov.gershgorin_max(A)


def test_gershgorin_bound_brute_force():
    st = w.uniform_stack(5, 4, ["Si", "BEOL", "Cu"])
    A = assembly.assemble(st)
    M = A.toarray()
    brute = max(M[i, i] + sum(abs(M[i, j]) for j in range(M.shape[0]) if j != i)
                for i in range(M.shape[0]))
    assert krylov.gershgorin_max(A) == pytest.approx(brute, rel=1e-14)
    assert np.linalg.eigvalsh(M)[-1] <= brute


# ------------------------------------------------------------------------ PCG
def test_pcg_reaches_direct_solution(c0):
    st, P, A = c0
    b = P.ravel()
    xd = direct.solve_separable(st, b)
    lmin, lmax = krylov.spectral_bounds(A, w.lanczos_start(st.n))
    M = lambda r: krylov.chebyshev_precondition(lambda v: A @ v, r, lmin, lmax, 30)
    x, k = krylov.pcg(lambda v: A @ v, b, M, np.zeros_like(b), 1e-11 * np.linalg.norm(b))
    assert np.abs(x - xd).max() <= 1e-9 * np.abs(xd).max()
    # preconditioning pays: far fewer iterations than plain CG (Table abl_pre shape)
    _, k_plain = krylov.pcg(lambda v: A @ v, b, lambda r: r, np.zeros_like(b),
                            1e-11 * np.linalg.norm(b), maxit=5000)
    assert k * 10 < k_plain


# -------------------------------------------------------------------- adjoint
def _perturbed_theta(st, theta, A, kl=None, kv=None):
    """theta' = theta - A'^{-1} (A' - A) theta  (exact perturbation solve)."""
    Ap = assembly.assemble(st, cond=assembly.conductances(st, k_lat=kl, k_vert=kv))
    return theta - direct.solve_splu(Ap, (Ap - A) @ theta)


def test_adjoint_against_perturbation_fd():
    st = w.Stack(12, 10, ["Si", "BEOL", "bond", "Si", "TIM", "Cu"])
    st.k_lat_mult = np.exp(0.3 * np.random.default_rng(7).standard_normal(st.shape))
    rng = np.random.default_rng(8)
    P = rng.uniform(0, 2e-3, st.n)
    A = assembly.assemble(st)
    th = direct.solve_splu(A, P)
    beta = 0.5
    mask = st.si_mask()
    Tf = st.t_amb + th
    gT = adjoint.lse_grad(Tf, mask, beta)
    gr = adjoint.gradient(st, th, gT, direct.solve_splu)
    L = lambda t: adjoint.lse_loss(st.t_amb + t, mask, beta)
    # dL/dP for a few cells: exact perturbation  dtheta = A^{-1} e_i dP
    for i in (0, 37, 500):
        h = 1e-4 * max(P[i], 1e-4)
        e = np.zeros(st.n); e[i] = h
        dth = direct.solve_splu(A, e)
        fd = (L(th + dth) - L(th - dth)) / (2 * h)
        assert fd == pytest.approx(gr.dP[i], rel=1e-6)
    # dL/dk_lat[l] and dL/dk_vert[l]
    for l in range(st.nz):
        for which in ("lat", "vert"):
            h = 1e-4 * (st.k_lat[l] if which == "lat" else st.k_vert[l])
            kp = (st.k_lat if which == "lat" else st.k_vert).copy()
            km = kp.copy()
            kp[l] += h
            km[l] -= h
            if which == "lat":
                tp = _perturbed_theta(st, th, A, kl=kp)
                tm = _perturbed_theta(st, th, A, kl=km)
                g = gr.dk_lat[l]
            else:
                tp = _perturbed_theta(st, th, A, kv=kp)
                tm = _perturbed_theta(st, th, A, kv=km)
                g = gr.dk_vert[l]
            fd = (L(tp) - L(tm)) / (2 * h)
            assert fd == pytest.approx(g, rel=1e-5, abs=1e-9 * abs(gr.dk_layer).max())
    # dL/dk per layer (the library's output): both conductivities of layer l
    # moved by the same step in one perturbation solve
    for l in range(st.nz):
        h = 1e-4 * st.k_lat[l]
        klp, klm = st.k_lat.copy(), st.k_lat.copy()
        kvp, kvm = st.k_vert.copy(), st.k_vert.copy()
        klp[l] += h
        kvp[l] += h
        klm[l] -= h
        kvm[l] -= h
        tp = _perturbed_theta(st, th, A, kl=klp, kv=kvp)
        tm = _perturbed_theta(st, th, A, kl=klm, kv=kvm)
        fd = (L(tp) - L(tm)) / (2 * h)
        assert fd == pytest.approx(gr.dk_layer[l], rel=1e-5, abs=1e-9 * abs(gr.dk_layer).max())


def test_adjoint_special_cases():
    st = w.uniform_stack(10, 8, ["Si", "BEOL", "Si", "TIM", "Cu"])
    P = np.random.default_rng(9).uniform(0, 2e-3, st.n)
    A = assembly.assemble(st)
    th = direct.solve_separable(st, P)
    mask = st.si_mask()
    # beta -> 0: softmax -> uniform weights over Si cells
    g0 = adjoint.lse_grad(st.t_amb + th, mask, 1e-12)
    np.testing.assert_allclose(g0[mask.ravel()], 1.0 / mask.sum(), rtol=1e-9)
    assert g0[~mask.ravel()].max() == 0.0
    # raising conductivity on the heat path lowers the smoothed peak
    gr = adjoint.gradient(st, th, adjoint.lse_grad(st.t_amb + th, mask, 0.5), direct.solve_splu)
    assert np.all(gr.dk_vert < 0)
    # dL/dP = lambda > 0 (M-matrix inverse is positive)
    assert gr.dP.min() > 0


# ------------------------------------------------------------ FP16 storage
def test_fp16_storage_rounding_bound_and_range(c4s):
    """Every stored lateral conductance is within one FP16 half-ulp (plus the
    FP32 step) of the exact value, and the scaled layer maxima sit in
    (2^13, 2^14]: normal FP16 numbers, far from overflow."""
    st = c4s[0]
    c = assembly.conductances(st)
    h = assembly.fp16_lateral(c)
    e = assembly.fp16_exponents(c)
    bound = 2.0 ** -11 * (1 + 2.0 ** -12)
    for g, gh in ((c.gx, h.gx), (c.gy, h.gy)):
        assert np.all(gh > 0)
        assert np.max(np.abs(gh - g) / g) <= bound
    for l in range(st.nz):
        m = max(c.gx[l].max(), c.gy[l].max()) * 2.0 ** e[l]
        assert 2.0 ** 13 < m <= 2.0 ** 14
    assert np.array_equal(h.gz, c.gz) and np.array_equal(h.sink, c.sink)


def test_fp16_storage_exact_for_powers_of_two():
    """dx = dy = dz = 1 and k = 2^-20 give g = 2^-20 exactly: its exponent is 34
    (2^-20 * 2^34 = 2^14) and the stored value is exact; k = 3 * 2^-20 with a
    mantissa that FP16 holds is also exact."""
    for kk, exact in ((2.0 ** -20, True), (3 * 2.0 ** -20, True), (1.0 / 3.0, False)):
        st = w.Stack(4, 3, ["Si", "Cu"], dx=1.0, dy=1.0, dz=np.array([1.0, 1.0]),
                     k_lat=np.array([kk, kk]), k_vert=np.array([1.0, 1.0]), h_top=1.0)
        c = assembly.conductances(st)
        h = assembly.fp16_lateral(c)
        assert np.allclose(c.gx, kk, rtol=1e-15)
        if exact:
            assert np.array_equal(h.gx, c.gx) and np.array_equal(h.gy, c.gy)
        else:
            assert not np.array_equal(h.gx, c.gx)
    e = assembly.fp16_exponents(assembly.conductances(
        w.Stack(4, 3, ["Si"], dx=1.0, dy=1.0, dz=np.array([1.0]), k_lat=np.array([2.0 ** -20]),
                k_vert=np.array([1.0]), h_top=1.0)))
    assert e.tolist() == [34]


def test_fp16_operator_balanced_spd_and_relative_bound():
    """The FP16-stored operator keeps every row sum equal to the sink (the
    diagonal is formed from the stored off-diagonals), stays SPD, and, as a
    relative perturbation of each edge weight by at most eps = 2^-11 of a
    Laplacian-plus-diagonal matrix, satisfies (1 - eps) A <= A16 <= (1 + eps) A:
    the generalized eigenvalues of (A16, A) lie in [1 - eps, 1 + eps].  A
    missing unscale or a wrong exponent moves them far outside."""
    st = w.uniform_stack(5, 4, ["Si", "BEOL", "TIM", "Cu"])
    st.k_lat_mult = np.random.default_rng(3).lognormal(0.0, 0.3, st.shape)
    c = assembly.conductances(st)
    h = assembly.fp16_lateral(c)
    A = assembly.assemble(st, cond=c).toarray()
    A16 = assembly.assemble(st, cond=h).toarray()
    assert np.array_equal(A16, A16.T)
    assert np.allclose(A16 @ np.ones(st.n), c.sink.ravel(), rtol=0, atol=1e-15 * np.abs(A16).max())
    ev = sla.eigh(A16, A, eigvals_only=True)
    eps = 2.0 ** -11 * (1 + 2.0 ** -12)
    assert ev.min() >= 1 - eps and ev.max() <= 1 + eps
    assert np.linalg.eigvalsh(A16).min() > 0
    # planted mistake: the scale left in the stored values
    e = assembly.fp16_exponents(c)
    bad = assembly.Conductances(h.gx * np.ldexp(1.0, e)[:, None, None], h.gy, h.gz, h.sink)
    ev_bad = sla.eigh(assembly.assemble(st, cond=bad).toarray(), A, eigvals_only=True)
    assert ev_bad.max() > 2.0


# ---------------------------------------------------------------------------
# Jacobi-scaled Chebyshev preconditioner (an extension beyond the paper)

def _scaled_closed_form(A, r, lmin, lmax, k):
    """D^{-1/2} V diag((1 - P_k(l)) / l) V^T D^{-1/2} r from a dense
    eigendecomposition of S = D^{-1/2} A D^{-1/2} and the closed-form residual
    polynomial: no recurrence and no sparse product."""
    Ad = A.toarray()
    s = 1.0 / np.sqrt(np.diag(Ad))
    S = s[:, None] * Ad * s[None, :]
    lam, V = np.linalg.eigh(S)
    f = (1.0 - krylov.chebyshev_residual_poly(lam, lmin, lmax, k)) / lam
    return s * (V @ (f * (V.T @ (s * r))))


@pytest.mark.parametrize("k", [1, 2, 7, 30])
def test_jacobi_chebyshev_matches_closed_form(k):
    """The scaled recurrence equals q_k(D^{-1} A) D^{-1} r evaluated through
    the eigenvectors of the symmetric scaling, on a small layered stack whose
    layers give the diagonal a spread of three decades."""
    st = w.Stack(6, 5, ["Si", "BEOL", "Cu", "TIM"], h_top=1e4)
    A = assembly.assemble(st)
    r = np.random.default_rng(11).standard_normal(st.n)
    lam = np.linalg.eigvalsh((A.toarray() / np.sqrt(np.outer(A.diagonal(), A.diagonal()))))
    lmin, lmax = 0.5 * lam[0], min(2.0, 1.05 * lam[-1])
    got = krylov.jacobi_chebyshev_precondition(A, r, lmin, lmax, k)
    ref = _scaled_closed_form(A, r, lmin, lmax, k)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    # a plausible mistake - scaling only the right-hand side, not the operator -
    # differs from the closed form once the polynomial has a degree (k = 1 is
    # the constant 1/theta, the same either way)
    if k > 1:
        wrong = krylov.chebyshev_precondition(lambda v: A @ v, r / A.diagonal(), lmin, lmax, k)
        assert np.abs(wrong - ref).max() > 1e-3 * np.abs(ref).max()


def test_jacobi_chebyshev_uniform_diagonal_is_plain_chebyshev():
    """With diag(A) = c I the scaled preconditioner on [a, b] is the plain one
    on [c a, c b] (the residual polynomial only sees A / c)."""
    rng = np.random.default_rng(5)
    n = 40
    B = rng.standard_normal((n, n))
    off = -np.abs(B + B.T) / (4 * n)
    np.fill_diagonal(off, 0.0)
    c = 3.7
    Ad = off + np.diag(np.full(n, c))
    import scipy.sparse as sp

    A = sp.csr_matrix(Ad)
    lam = np.linalg.eigvalsh(Ad)
    a, b = lam[0] / c, lam[-1] / c
    r = rng.standard_normal(n)
    z1 = krylov.jacobi_chebyshev_precondition(A, r, a, b, 12)
    z2 = krylov.chebyshev_precondition(lambda v: A @ v, r, c * a, c * b, 12)
    assert np.abs(z1 - z2).max() <= 1e-12 * np.abs(z2).max()


def test_jacobi_bounds_and_interlacing(c0):
    """The Lanczos interval of D^{-1} A lies inside (0, 2] and inside the
    true spectrum of S (Ritz values interlace), and the scaled spectrum is
    narrower than the unscaled one on config 0."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    st, _, A = c0
    lo, hi = krylov.jacobi_spectral_bounds(A, w.lanczos_start(st.n))
    s = 1.0 / np.sqrt(A.diagonal())
    S = (sp.diags(s) @ A @ sp.diags(s)).tocsc()
    smax = spla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0]
    smin = spla.eigsh(S, k=1, sigma=0, which="LM", return_eigenvectors=False, tol=1e-12)[0]
    assert 0.0 < smin <= lo and hi <= 2.0 and smax <= 2.0 + 1e-12
    amax = spla.eigsh(A.tocsc(), k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0]
    amin = spla.eigsh(A.tocsc(), k=1, sigma=0, which="LM", return_eigenvectors=False, tol=1e-12)[0]
    assert smax / smin < 0.5 * amax / amin


def test_jacobi_chebyshev_pcg(c0):
    """PCG with the scaled preconditioner reaches the direct solution, in
    fewer iterations than the plain Chebyshev preconditioner of the same
    degree (the point of the scaling)."""
    st, P, A = c0
    b = P.ravel()
    v0 = w.lanczos_start(st.n)
    lo, hi = krylov.jacobi_spectral_bounds(A, v0)
    Mj = lambda r: krylov.jacobi_chebyshev_precondition(A, r, lo, hi, 30)
    xj, kj = krylov.pcg(lambda v: A @ v, b, Mj, np.zeros(st.n), 1e-10 * np.linalg.norm(b))
    lmin, lmax = krylov.spectral_bounds(A, v0)
    Mc = lambda r: krylov.chebyshev_precondition(lambda v: A @ v, r, lmin, lmax, 30)
    _, kc = krylov.pcg(lambda v: A @ v, b, Mc, np.zeros(st.n), 1e-10 * np.linalg.norm(b))
    ref = direct.solve_separable(st, b)
    assert np.abs(xj - ref).max() <= 1e-8 * np.abs(ref).max()
    assert kj < kc


def _two_sided_column(dz, kv, dxdy, h_top, h_bot, l, q):
    """Rise of a laterally uniform column cooled on both faces, heated by q per
    cell in layer l only: a resistor chain whose two ends lead to ambient.
    The heat splits between the two paths in inverse proportion to their
    resistances; along each path the rise falls with the resistance left."""
    nz = len(dz)
    link = [(dz[m] / 2.0) / (kv[m] * dxdy) + (dz[m + 1] / 2.0) / (kv[m + 1] * dxdy)
            for m in range(nz - 1)]
    # resistance from layer m to ambient through the top and through the bottom
    up = [sum(link[m:]) + 1.0 / (h_top * dxdy) for m in range(nz)]
    dn = [sum(link[:m]) + 1.0 / (h_bot * dxdy) for m in range(nz)]
    th_l = q * up[l] * dn[l] / (up[l] + dn[l])
    q_up, q_dn = th_l / up[l], th_l / dn[l]
    th = np.array([q_up * up[m] if m >= l else q_dn * dn[m] for m in range(nz)])
    return th, q_up, q_dn


@pytest.mark.parametrize("l", [0, 2, 5])
def test_two_sided_cooling_closed_form(l):
    """Both faces cooled (the bottom convection term, which no hand example
    exercises): the solve matches the two-path resistor network, and the heat
    leaving each face is the network's split of the injected power."""
    layers = ["Si", "BEOL", "bond", "Si", "TIM", "Cu"]
    st = w.uniform_stack(4, 3, layers)
    st.dz = np.array([60e-6, 8e-6, 3e-6, 90e-6, 40e-6, 500e-6])
    st.h_top, st.h_bottom = 2e4, 3e3
    q = 1.5e-3
    P = np.zeros(st.shape)
    P[l] = q
    th = direct.solve_dense(assembly.assemble(st), P.ravel()).reshape(st.shape)
    dxdy = st.dx * st.dy
    exp, q_up, q_dn = _two_sided_column(st.dz, st.k_vert, dxdy, st.h_top, st.h_bottom, l, q)
    np.testing.assert_allclose(th, np.broadcast_to(exp[:, None, None], st.shape), rtol=1e-12)
    cells = st.nx * st.ny
    out_top = math.fsum((st.h_top * dxdy * th[-1]).ravel())
    out_bot = math.fsum((st.h_bottom * dxdy * th[0]).ravel())
    assert out_top == pytest.approx(cells * q_up, rel=1e-12)
    assert out_bot == pytest.approx(cells * q_dn, rel=1e-12)
    assert out_top + out_bot == pytest.approx(cells * q, rel=1e-12)


def test_single_layer_both_faces():
    """One layer cooled on both faces: the two convective conductances act on
    the same cells, so the rise is q / ((h_top + h_bottom) dx dy)."""
    st = w.uniform_stack(3, 2, ["Si"])
    st.h_top, st.h_bottom = 1e4, 2.5e3
    q = 2e-3
    th = direct.solve_dense(assembly.assemble(st), np.full(st.n, q))
    np.testing.assert_allclose(th, q / ((st.h_top + st.h_bottom) * st.dx * st.dy), rtol=1e-13)


def test_separable_two_sided_matches_lu():
    """The separable solver and eigenvalues with both faces cooled (its own
    sink term) against the assembled matrix: LU solve and dense spectrum."""
    st = w.uniform_stack(6, 5, ["Si", "BEOL", "bond", "TIM", "Cu"])
    st.h_top, st.h_bottom = 1e4, 4e3
    A = assembly.assemble(st)
    b = np.random.default_rng(9).uniform(0, 1e-3, st.n)
    x_lu = direct.solve_splu(A, b)
    x_sep = direct.solve_separable(st, b)
    assert np.abs(x_sep - x_lu).max() <= 1e-12 * np.abs(x_lu).max()
    ev = np.linalg.eigvalsh(A.toarray())
    np.testing.assert_allclose(direct.all_eigenvalues(st), ev, rtol=1e-10, atol=1e-12 * ev[-1])
