"""GPU parity: every step of the solve path through the C ABI against the CPU oracle.

Tolerances ("Parity bar"):
* FP64 operator / residual: |gpu - ref| <= 1e-14 * (|A| |x|)_i element-wise
  (a 7-term sum in a different order differs by a few ulps of the row scale);
* FP32 operator: <= 2e-6 * (|A| |x|)_i (inputs rounded to FP32, 7 terms);
* FP64 Chebyshev application: <= 1e-10 * ||z||_inf (29 sweeps of rounding
  amplified by the polynomial's norm);
* FP32 Chebyshev application: <= 4 max(k, 4) times the spread between the
  oracle's listing in FP32 and in FP64 (gpu_helpers.fp32_cheb_bar);
* solves: plain FP64 <= 1e-10 and mixed <= 1e-8 rise-relative inf-norm error.
"""

import numpy as np
import pytest
import torch

import workloads as w
from oracle import assembly, cpu_cg, direct, krylov, transient
from tests.gpu_helpers import dev, fp32_cheb_bar, grid_of, ragged_stack, rise_err, say, t32, t64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


CASES = {
    "ragged_mult": lambda: ragged_stack(70, 9, mult=True),
    "ragged_uniform": lambda: ragged_stack(131, 6, mult=False),
    "column": lambda: ragged_stack(1, 1, mult=False),
    "row": lambda: ragged_stack(67, 1, mult=True),
    "c0": lambda: w.config0()[0],
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("dt", [None, 1e-4])
def test_apply_matches_csr(case, dt):
    say(f"apply {case} dt={dt}")
    st = CASES[case]()
    A = assembly.assemble(st, dt=dt)
    Aabs = abs(A)
    g = grid_of(st)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, st.n) + 2.0
    y = g.apply(t64(x), dt=dt or 0.0).cpu().numpy()
    ref = A @ x
    scale = Aabs @ np.abs(x)
    assert np.all(np.abs(y - ref) <= 1e-14 * scale)
    # the CSR copy of the operator (storage baseline) gives the same product
    yc = g.apply_csr(t64(x), dt=dt or 0.0).cpu().numpy()
    assert np.all(np.abs(yc - ref) <= 1e-14 * scale)
    x32 = x.astype(np.float32)
    y32 = g.apply(t32(x32), dt=dt or 0.0).cpu().numpy().astype(np.float64)
    ref32 = A @ x32.astype(np.float64)
    assert np.all(np.abs(y32 - ref32) <= 2e-6 * (Aabs @ np.abs(x32.astype(np.float64))))
    g.close()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("dt", [None, 1e-4])
def test_residual_matches_oracle(case, dt):
    """Every grid shape: the even-width ones take the residual kernel built
    for this call's streams, the odd-width ones (one cell per lane) the one
    that tests its pointers at run time."""
    say(f"residual {case} dt={dt}")
    st = CASES[case]()
    A = assembly.assemble(st, dt=dt)
    g = grid_of(st)
    rng = np.random.default_rng(4)
    th = rng.uniform(0, 50, st.n)
    b = rng.uniform(0, 1e-3, st.n)
    r = g.residual(t64(b), t64(st.t_amb + th), dt=dt or 0.0).cpu().numpy()
    ref = b - A @ th
    scale = np.abs(b) + abs(A) @ np.abs(th)
    assert np.all(np.abs(r - ref) <= 2e-14 * scale)
    g.close()


@pytest.mark.parametrize("case", ["ragged_mult", "ragged_uniform", "c0"])
@pytest.mark.parametrize("degree", [1, 2, 3, 30])
def test_chebyshev_matches_oracle(case, degree):
    say(f"chebyshev {case} k={degree}")
    st = CASES[case]()
    A = assembly.assemble(st)
    g = grid_of(st)
    lmin, lmax = krylov.spectral_bounds(A, w.lanczos_start(st.n))
    rng = np.random.default_rng(5)
    r = rng.standard_normal(st.n)
    ref = krylov.chebyshev_precondition(lambda v: A @ v, r, lmin, lmax, degree)
    z = g.precond_apply(t64(r), lmin, lmax, degree).cpu().numpy()
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()
    # FP32: same polynomial in single precision
    z32 = g.precond_apply(t32(r), lmin, lmax, degree).cpu().numpy().astype(np.float64)
    assert np.abs(z32 - ref).max() <= fp32_cheb_bar(A, r, lmin, lmax, degree, ref)
    g.close()


@pytest.mark.parametrize("case", ["ragged_mult", "ragged_uniform", "c0"])
@pytest.mark.parametrize("degree", [1, 2, 3, 6, 7, 9, 30])
def test_chebyshev_jacobi_matches_oracle(monkeypatch, case, degree):
    """The Jacobi-scaled Chebyshev preconditioner (beyond the paper):
    q_k(D^{-1} A) D^{-1} r against the oracle's definition, in FP64 and FP32,
    with single sweeps, fused sweep pairs (two workgroup shapes) and fused
    triples (two shapes); the fused results also against the single sweeps."""
    say(f"chebyshev-jacobi {case} k={degree}")
    st = CASES[case]()
    A = assembly.assemble(st)
    g = grid_of(st)
    lo, hi = krylov.jacobi_spectral_bounds(A, w.lanczos_start(st.n))
    r = np.random.default_rng(7).standard_normal(st.n)
    ref = krylov.jacobi_chebyshev_precondition(A, r, lo, hi, degree)
    z = g.precond_apply(t64(r), lo, hi, degree, preconditioner="chebyshev_jacobi").cpu().numpy()
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()
    z_single = None
    bar32 = fp32_cheb_bar(A, r, lo, hi, degree, ref, jacobi=True)
    for env in ({"CUTH_FUSE": "0"}, {"CUTH_FUSE": "1", "CUTH_FUSE_SHAPE": "2,8", "CUTH_FUSE3": "0"},
                {"CUTH_FUSE": "1", "CUTH_FUSE_SHAPE": "1,1", "CUTH_FUSE3": "0"},
                {"CUTH_FUSE": "1", "CUTH_FUSE_SHAPE": "2,8", "CUTH_FUSE3": "1", "CUTH_FUSE3_SHAPE": "4,8"},
                {"CUTH_FUSE": "1", "CUTH_FUSE_SHAPE": "2,8", "CUTH_FUSE3": "1", "CUTH_FUSE3_SHAPE": "1,1"}):
        for k_, v_ in env.items():
            monkeypatch.setenv(k_, v_)
        z32 = g.precond_apply(t32(r), lo, hi, degree,
                              preconditioner="chebyshev_jacobi").cpu().numpy().astype(np.float64)
        assert np.abs(z32 - ref).max() <= bar32, env
        if z_single is None:
            z_single = z32
        else:
            # the same arithmetic in the same order as single sweeps
            assert np.abs(z32 - z_single).max() <= 1e-6 * np.abs(z_single).max(), env
    g.close()


@pytest.mark.parametrize("case", ["ragged_mult", "c0"])
def test_single_pass_preconditioners_match_oracle(case):
    """Jacobi (z = r / diag(A)) and none (z = r) through cuth_precond_apply."""
    say(f"single-pass preconditioners {case}")
    st = CASES[case]()
    A = assembly.assemble(st)
    g = grid_of(st)
    r = np.random.default_rng(9).standard_normal(st.n)
    zj = g.precond_apply(t64(r), 1.0, 2.0, 1, preconditioner="jacobi").cpu().numpy()
    np.testing.assert_allclose(zj, r / A.diagonal(), rtol=1e-14)
    zn = g.precond_apply(t64(r), 1.0, 2.0, 1, preconditioner="none").cpu().numpy()
    assert np.array_equal(zn, r)
    g.close()


@pytest.mark.parametrize("case", ["c0", "ragged_mult"])
def test_jacobi_lanczos_matches_oracle(case):
    """Lanczos on D^{-1/2} A D^{-1/2} against the oracle's, from the same start
    vector; the interval used lies in (0, 2]."""
    say(f"jacobi lanczos {case}")
    st = CASES[case]()
    A = assembly.assemble(st)
    g = grid_of(st)
    v0 = w.lanczos_start(st.n)
    b = g.spectral_bounds(steps=30, v0=t32(v0.astype(np.float32)), preconditioner="chebyshev_jacobi")
    s = 1.0 / np.sqrt(A.diagonal())
    a_ref, b_ref = krylov.lanczos(lambda v: s * (A @ (s * v)),
                                  v0.astype(np.float32).astype(np.float64), 30)
    ritz = krylov.ritz_values(a_ref, b_ref)
    np.testing.assert_allclose(b["alpha"][:5], a_ref[:5], rtol=1e-4)
    assert b["ritz_max"] == pytest.approx(ritz[-1], rel=1e-4)
    assert b["ritz_min"] == pytest.approx(ritz[0], rel=5e-2)
    assert 0.0 < b["lmin"] < b["lmax"] <= 2.0
    g.close()


def test_solve_chebyshev_jacobi():
    """Solves with the Jacobi-scaled Chebyshev preconditioner meet the parity
    bars in every precision (steady, one backward-Euler step, a two-grid
    batch), and take fewer CG iterations than the paper's preconditioner of the
    same degree on the layered stacks."""
    import paper_2606_17850_amd as cuth
    say("solve chebyshev-jacobi")
    for st, P in (w.config4_small(), w.config0()):
        ref = _ref_steady(st, P)
        g = grid_of(st)
        for prec, bar in (("fp64", 1e-10), ("mixed", 1e-8), ("mixed16", 1e-8), ("adaptive", 1e-10)):
            T, s = g.solve(t64(P), precision=prec, preconditioner="chebyshev_jacobi")
            e = rise_err(T.cpu().numpy(), ref, st.t_amb)
            _, s0 = g.solve(t64(P), precision=prec)
            say(f"  {st.shape} {prec} cg {s['cg_iters']} (chebyshev {s0['cg_iters']}) err {e:.2e} "
                f"interval {s['lambda_min']:.3e}..{s['lambda_max']:.3e}")
            assert e <= bar
            assert 0.0 < s["lambda_min"] < s["lambda_max"] <= 2.0
            if prec == "fp64":
                assert s["cg_iters"] < s0["cg_iters"]
        g.close()
    st = ragged_stack(70, 9, mult=True)
    P = np.zeros(st.shape)
    P[0] = np.random.default_rng(6).uniform(0, 2e-3, (st.ny, st.nx))
    g = grid_of(st)
    dt = 1e-4
    th0 = np.random.default_rng(8).uniform(0, 5.0, st.n)
    ref_tr = transient.step(st, P.ravel(), th0, dt)
    Tt, _ = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision="mixed",
                             preconditioner="chebyshev_jacobi")
    got = Tt.cpu().numpy() - st.t_amb
    assert np.abs(got - ref_tr).max() <= 1e-8 * np.abs(ref_tr).max()
    g.close()
    stacks = [ragged_stack(70, 9, mult=True), ragged_stack(67, 1, mult=True)]
    maps = [np.random.default_rng(40 + i).uniform(0, 2e-3, s_.n) for i, s_ in enumerate(stacks)]
    grids = [grid_of(s_) for s_ in stacks]
    Tb, _ = cuth.solve_batch(grids, [t64(m) for m in maps], nrhs=1, precision="mixed",
                             preconditioner="chebyshev_jacobi")
    for s_, m, t in zip(stacks, maps, Tb):
        assert rise_err(t.cpu().numpy(), _ref_steady(s_, m), s_.t_amb) <= 1e-8
    for gg in grids:
        gg.close()


@pytest.mark.parametrize("case", ["c0", "ragged_mult"])
def test_lanczos_matches_oracle(case):
    say(f"lanczos {case}")
    st = CASES[case]()
    A = assembly.assemble(st)
    g = grid_of(st)
    v0 = w.lanczos_start(st.n)
    b = g.spectral_bounds(steps=30, v0=t32(v0.astype(np.float32)))
    a_ref, b_ref = krylov.lanczos(lambda v: A @ v, v0.astype(np.float32).astype(np.float64), 30)
    ritz = krylov.ritz_values(a_ref, b_ref)
    # the first steps agree closely; extreme Ritz values agree to FP32-level
    np.testing.assert_allclose(b["alpha"][:5], a_ref[:5], rtol=1e-4)
    assert b["ritz_max"] == pytest.approx(ritz[-1], rel=1e-4)
    assert b["ritz_min"] == pytest.approx(ritz[0], rel=5e-2)
    # a safe upper bound and a lower bound no smaller than the spectrum
    ev_hi = krylov.gershgorin_max(A)
    assert b["lmax"] <= ev_hi * (1 + 1e-12)
    if st.k_lat_mult is None:
        lo, hi = direct.exact_extremes(st)
        assert b["lmax"] >= hi
        assert b["ritz_min"] >= lo * (1 - 1e-4)
    g.close()


def _ref_steady(st, P):
    A = assembly.assemble(st)
    b = P.ravel()
    if st.k_lat_mult is None:
        return st.t_amb + direct.solve_separable(st, b)
    if st.n <= 300000:
        return st.t_amb + direct.solve_splu(A, b)
    x, _, _ = cpu_cg.jacobi_cg(A, b, rtol=1e-14)
    return st.t_amb + x


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_solve_config0(prec, tol):
    say(f"solve c0 {prec}")
    st, P = w.config0()
    ref = _ref_steady(st, P)
    g = grid_of(st)
    T, stats = g.solve(t64(P), precision=prec)
    err = rise_err(T.cpu().numpy(), ref, st.t_amb)
    say(f"  err {err:.3e} stats {stats}")
    assert err <= tol
    # the FP64 residual of the result (the mixed path stops on the error estimate)
    assert stats["rel_residual"] < (1e-9 if prec == "fp64" else 1e-7)
    g.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_solve_lognormal_small(prec, tol):
    say(f"solve c4-small {prec}")
    st, P = w.config4_small()
    ref = _ref_steady(st, P)
    g = grid_of(st)
    T, stats = g.solve(t64(P), precision=prec)
    err = rise_err(T.cpu().numpy(), ref, st.t_amb)
    say(f"  err {err:.3e} cg {stats['cg_iters']} cycles {stats['outer_cycles']}")
    assert err <= tol
    g.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_solve_ragged(prec, tol):
    say(f"solve ragged {prec}")
    st = ragged_stack(70, 9, mult=True)
    P = np.zeros(st.shape)
    P[0] = np.random.default_rng(6).uniform(0, 2e-3, (st.ny, st.nx))
    ref = _ref_steady(st, P)
    g = grid_of(st)
    T, stats = g.solve(t64(P), precision=prec)
    assert rise_err(T.cpu().numpy(), ref, st.t_amb) <= tol
    g.close()


def test_reduce_launch_mode(monkeypatch):
    """The per-problem reduce launch (used for grids with more than 4096
    workgroups) forced on small grids: same oracle parity as the direct mode,
    and the two modes agree to the solve tolerance (their fixed summation
    orders differ).  Degree 30 on a steady ragged grid and on a two-grid batch;
    degree 1 (the scaling preconditioner, plain CG) on a backward-Euler step,
    whose system is well conditioned."""
    import paper_2606_17850_amd as cuth
    say("reduce launch mode")
    st = ragged_stack(70, 9, mult=True)
    P = np.zeros(st.shape)
    P[0] = np.random.default_rng(6).uniform(0, 2e-3, (st.ny, st.nx))
    ref = _ref_steady(st, P)
    g = grid_of(st)
    dt = 1e-4
    th0 = np.random.default_rng(8).uniform(0, 5.0, st.n)
    ref_tr = transient.step(st, P.ravel(), th0, dt)
    for prec, tol in (("mixed", 1e-8), ("fp64", 1e-10)):
        out = {}
        for mode in ("direct", "reduce"):
            if mode == "reduce":
                monkeypatch.setenv("CUTH_REDUCE_ABOVE", "0")
            else:
                monkeypatch.delenv("CUTH_REDUCE_ABOVE", raising=False)
            T, _ = g.solve(t64(P), precision=prec)
            Tt, _ = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision=prec,
                                     cheb_degree=1, max_inner=5000)
            assert rise_err(T.cpu().numpy(), ref, st.t_amb) <= tol
            got = Tt.cpu().numpy() - st.t_amb
            assert np.abs(got - ref_tr).max() <= tol * np.abs(ref_tr).max()
            out[mode] = (T.cpu().numpy(), Tt.cpu().numpy())
        assert rise_err(out["reduce"][0], out["direct"][0], st.t_amb) <= tol
    monkeypatch.setenv("CUTH_REDUCE_ABOVE", "0")
    stacks = [w.uniform_stack(64, 48, ["Si", "BEOL", "TIM", "Cu"]),
              w.uniform_stack(96, 40, ["Si", "bond", "Si", "TIM", "Cu"])]
    maps = [np.random.default_rng(20 + i).uniform(0, 2e-3, s.n) for i, s in enumerate(stacks)]
    grids = [grid_of(s) for s in stacks]
    T, _ = cuth.solve_batch(grids, [t64(m) for m in maps], nrhs=1, precision="mixed")
    for s, m, t in zip(stacks, maps, T):
        refb = s.t_amb + direct.solve_separable(s, m)
        assert rise_err(t.cpu().numpy(), refb, s.t_amb) <= 1e-8
    for gg in grids + [g]:
        gg.close()


@pytest.mark.parametrize("case", ["ragged_mult", "row"])
@pytest.mark.parametrize("dt", [None, 1e-4])
def test_apply_fp16_coefficients(case, dt):
    """The FP32 operator with FP16-stored lateral conductances against the
    oracle's operator assembled from the same rounded conductances."""
    say(f"apply fp16 {case} dt={dt}")
    st = CASES[case]()
    cond = assembly.fp16_lateral(assembly.conductances(st, dt))
    A16 = assembly.assemble(st, dt=dt, cond=cond)
    g = grid_of(st)
    x32 = (np.random.default_rng(3).uniform(-1, 1, st.n) + 2.0).astype(np.float32)
    y = g.apply(t32(x32), dt=dt or 0.0, fp16_coef=True).cpu().numpy().astype(np.float64)
    x = x32.astype(np.float64)
    assert np.all(np.abs(y - A16 @ x) <= 2e-6 * (abs(A16) @ np.abs(x)))
    # and it is not the FP32-coefficient operator (the rounding is visible)
    y32 = g.apply(t32(x32), dt=dt or 0.0).cpu().numpy().astype(np.float64)
    assert np.abs(y - y32).max() > 0
    g.close()


@pytest.mark.parametrize("degree", [3, 30])
def test_chebyshev_fp16_coefficients(degree):
    """Chebyshev application with the FP16-stored lateral conductances against
    the oracle's polynomial in the rounded operator (bounds of the exact one)."""
    say(f"chebyshev fp16 k={degree}")
    st = CASES["ragged_mult"]()
    A = assembly.assemble(st)
    A16 = assembly.assemble(st, cond=assembly.fp16_lateral(assembly.conductances(st)))
    lmin, lmax = krylov.spectral_bounds(A, w.lanczos_start(st.n))
    r = np.random.default_rng(5).standard_normal(st.n)
    ref = krylov.chebyshev_precondition(lambda v: A16 @ v, r, lmin, lmax, degree)
    g = grid_of(st)
    z = g.precond_apply(t32(r), lmin, lmax, degree, fp16_coef=True).cpu().numpy().astype(np.float64)
    assert np.abs(z - ref).max() <= fp32_cheb_bar(A16, r, lmin, lmax, degree, ref)
    g.close()


def test_solve_mixed16():
    """Solves with FP16-stored conductances in the preconditioner reach the same
    1e-8 rise error (lognormal grids, steady and one backward-Euler step, and a
    two-grid batch); on a grid without per-cell conductances the result is
    bitwise that of plain mixed precision."""
    import paper_2606_17850_amd as cuth
    say("solve mixed16")
    st, P = w.config4_small()
    ref = _ref_steady(st, P)
    g = grid_of(st)
    T, stats = g.solve(t64(P), precision="mixed16")
    err = rise_err(T.cpu().numpy(), ref, st.t_amb)
    say(f"  c4-small err {err:.3e} cg {stats['cg_iters']} cycles {stats['outer_cycles']}")
    assert err <= 1e-8
    dt = 1e-4
    th0 = np.random.default_rng(9).uniform(0, 5.0, st.n)
    ref_tr = transient.step(st, P.ravel(), th0, dt)
    Tt, _ = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision="mixed16")
    got = Tt.cpu().numpy() - st.t_amb
    assert np.abs(got - ref_tr).max() <= 1e-8 * np.abs(ref_tr).max()
    g.close()
    stacks = [ragged_stack(70, 9, mult=True), ragged_stack(67, 1, mult=True)]
    maps = [np.random.default_rng(30 + i).uniform(0, 2e-3, s.n) for i, s in enumerate(stacks)]
    grids = [grid_of(s) for s in stacks]
    Tb, _ = cuth.solve_batch(grids, [t64(m) for m in maps], nrhs=1, precision="mixed16")
    for s, m, t in zip(stacks, maps, Tb):
        assert rise_err(t.cpu().numpy(), _ref_steady(s, m), s.t_amb) <= 1e-8
    for gg in grids:
        gg.close()
    st0, P0 = w.config0()
    g0 = grid_of(st0)
    Ta, _ = g0.solve(t64(P0), precision="mixed")
    Tb0, _ = g0.solve(t64(P0), precision="mixed16")
    assert torch.equal(Ta, Tb0)
    g0.close()


def test_solve_adaptive_stage_switched():
    """The stage-switched scheme (FP64 CG, FP32/FP16 preconditioner, early
    FP32-stored product, hot restart, late FP64 product) reaches the FP64
    tolerances against the direct oracle: steady on a lognormal grid, on a
    uniform grid and on a ragged one, one backward-Euler step, and a two-grid
    batch.  At least one late-stage cycle follows the early one."""
    import paper_2606_17850_amd as cuth
    say("solve adaptive")
    for st, P in (w.config4_small(), w.config0()):
        ref = _ref_steady(st, P)
        g = grid_of(st)
        T, stats = g.solve(t64(P), precision="adaptive")
        err = rise_err(T.cpu().numpy(), ref, st.t_amb)
        say(f"  err {err:.3e} cg {stats['cg_iters']} cycles {stats['outer_cycles']} "
            f"relres {stats['rel_residual']:.2e}")
        assert err <= 1e-10
        assert stats["rel_residual"] <= 1e-10
        assert stats["outer_cycles"] >= 2
        g.close()
    st = ragged_stack(70, 9, mult=True)
    P = np.zeros(st.shape)
    P[0] = np.random.default_rng(6).uniform(0, 2e-3, (st.ny, st.nx))
    g = grid_of(st)
    T, _ = g.solve(t64(P), precision="adaptive")
    assert rise_err(T.cpu().numpy(), _ref_steady(st, P), st.t_amb) <= 1e-10
    dt = 1e-4
    th0 = np.random.default_rng(8).uniform(0, 5.0, st.n)
    ref_tr = transient.step(st, P.ravel(), th0, dt)
    Tt, _ = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision="adaptive")
    got = Tt.cpu().numpy() - st.t_amb
    assert np.abs(got - ref_tr).max() <= 1e-10 * np.abs(ref_tr).max()
    g.close()
    stacks = [ragged_stack(70, 9, mult=True), ragged_stack(67, 1, mult=True)]
    maps = [np.random.default_rng(40 + i).uniform(0, 2e-3, s.n) for i, s in enumerate(stacks)]
    grids = [grid_of(s) for s in stacks]
    Tb, sb = cuth.solve_batch(grids, [t64(m) for m in maps], nrhs=1, precision="adaptive")
    for s, m, t in zip(stacks, maps, Tb):
        assert rise_err(t.cpu().numpy(), _ref_steady(s, m), s.t_amb) <= 1e-10
    for gg in grids:
        gg.close()


def test_solve_fixed_fp32_drifts():
    """The fixed-FP32 baseline of Ablation II: one FP32 PCG to ||r|| <= 1e-10
    ||b|| on its own recursive residual, no refinement.  It takes about the FP64
    iteration count, its FP64 true residual stays far above the tolerance its
    recursive residual met, and its rise error is FP32-sized: larger than the
    mixed scheme's and the FP64 solver's, yet bounded."""
    say("solve fixed fp32")
    for st, P in (w.config4_small(), w.config0()):
        ref = _ref_steady(st, P)
        g = grid_of(st)
        T64, s64 = g.solve(t64(P), precision="fp64")
        T32, s32 = g.solve(t64(P), precision="fp32")
        Tm, _ = g.solve(t64(P), precision="mixed")
        e32 = rise_err(T32.cpu().numpy(), ref, st.t_amb)
        e64 = rise_err(T64.cpu().numpy(), ref, st.t_amb)
        em = rise_err(Tm.cpu().numpy(), ref, st.t_amb)
        say(f"  fp32 cg {s32['cg_iters']} (fp64 {s64['cg_iters']}) cycles {s32['outer_cycles']} "
            f"true relres {s32['rel_residual']:.2e} err {e32:.2e} (mixed {em:.2e}, fp64 {e64:.2e})")
        assert s32["outer_cycles"] == 1
        assert abs(s32["cg_iters"] - s64["cg_iters"]) <= 0.25 * s64["cg_iters"] + 2
        assert s32["rel_residual"] > 10 * 1e-10
        assert e32 <= 1e-3
        assert e32 > em and e32 > e64
        g.close()


@pytest.mark.parametrize("pcname", ["jacobi", "none"])
def test_baseline_preconditioners_match_oracle_pcg(pcname):
    """Jacobi-PCG and plain CG (the baselines of Ablation III) in FP64: the
    GPU's CG iteration count to ||r|| <= 1e-10 ||b|| equals the oracle's
    Algorithm 1 with M^-1 = diag(A)^-1 or the identity, within 2 (rounding near
    the threshold), and the solution meets the FP64 bar.  Mid-run true-residual
    checks are switched off so both run one uninterrupted CG."""
    say(f"baseline preconditioner {pcname}")
    st, P = w.config0()
    A = assembly.assemble(st)
    b = P.ravel()
    d = A.diagonal()
    M = (lambda r: r / d) if pcname == "jacobi" else (lambda r: r.copy())
    tol = 1e-10
    _, k_ref = krylov.pcg(lambda v: A @ v, b, M, np.zeros(st.n), tol * np.linalg.norm(b),
                          maxit=20000)
    g = grid_of(st)
    T, stats = g.solve(t64(P), precision="fp64", preconditioner=pcname, max_inner=20000,
                       check_period=20000)
    say(f"  gpu {stats['cg_iters']} oracle {k_ref}")
    assert abs(stats["cg_iters"] - k_ref) <= 2
    assert rise_err(T.cpu().numpy(), _ref_steady(st, P), st.t_amb) <= 1e-9
    # mixed precision with the same preconditioner still reaches the mixed bar
    # (the residual of plain and Jacobi CG plateaus for tens of iterations, so
    # the stagnation test runs every 200 and more refinement cycles are allowed)
    Tm, _ = g.solve(t64(P), precision="mixed", preconditioner=pcname, max_inner=20000,
                    check_period=200, max_outer=40)
    assert rise_err(Tm.cpu().numpy(), _ref_steady(st, P), st.t_amb) <= 1e-8
    # and so does the stage-switched scheme (Ablation III, optimisations on)
    Ta, sa = g.solve(t64(P), precision="adaptive", preconditioner=pcname, max_inner=20000,
                     check_period=200, max_outer=40)
    say(f"  adaptive cg {sa['cg_iters']} cycles {sa['outer_cycles']}")
    assert rise_err(Ta.cpu().numpy(), _ref_steady(st, P), st.t_amb) <= 1e-9
    assert sa["rel_residual"] <= 1e-10
    g.close()


def _auto_degree_rule(lmin, lmax):
    # the documented rule: smallest k >= 2 with 2 s^k <= 0.3, at most 64
    c = lmax / lmin
    s = (np.sqrt(c) - 1.0) / (np.sqrt(c) + 1.0)
    k = 2
    while k < 64 and 2.0 * s ** k > 0.3:
        k += 1
    return k


def test_auto_degree():
    """cheb_degree = CUTH_DEGREE_AUTO: the degree reported in the stats follows
    the documented rule from the reported interval, and the solves still meet
    the parity bars (steady mixed and FP64, one backward-Euler step, and a
    two-grid batch, which takes the largest degree of its systems)."""
    import paper_2606_17850_amd as cuth
    say("auto degree")
    for st, P in (w.config4_small(), w.config0()):
        ref = _ref_steady(st, P)
        g = grid_of(st)
        for prec, bar in (("mixed", 1e-8), ("fp64", 1e-10)):
            T, s = g.solve(t64(P), precision=prec, cheb_degree="auto")
            k = _auto_degree_rule(s["lambda_min"], s["lambda_max"])
            say(f"  {prec} degree {s['cheb_degree']} (rule {k}) cg {s['cg_iters']}")
            assert s["cheb_degree"] == k
            assert rise_err(T.cpu().numpy(), ref, st.t_amb) <= bar
        _, s30 = g.solve(t64(P), precision="mixed")
        assert s30["cheb_degree"] == 30
        g.close()
    st = ragged_stack(70, 9, mult=True)
    P = np.zeros(st.shape)
    P[0] = np.random.default_rng(6).uniform(0, 2e-3, (st.ny, st.nx))
    g = grid_of(st)
    dt = 1e-4
    th0 = np.random.default_rng(8).uniform(0, 5.0, st.n)
    ref_tr = transient.step(st, P.ravel(), th0, dt)
    Tt, s = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision="mixed", cheb_degree="auto")
    assert s["cheb_degree"] == _auto_degree_rule(s["lambda_min"], s["lambda_max"])
    got = Tt.cpu().numpy() - st.t_amb
    assert np.abs(got - ref_tr).max() <= 1e-8 * np.abs(ref_tr).max()
    g.close()
    stacks = [ragged_stack(70, 9, mult=True), ragged_stack(67, 1, mult=True)]
    maps = [np.random.default_rng(40 + i).uniform(0, 2e-3, s_.n) for i, s_ in enumerate(stacks)]
    grids = [grid_of(s_) for s_ in stacks]
    degs = []
    for gg, m in zip(grids, maps):
        _, s1 = gg.solve(t64(m), precision="mixed", cheb_degree="auto")
        degs.append(s1["cheb_degree"])
    Tb, sb = cuth.solve_batch(grids, [t64(m) for m in maps], nrhs=1, precision="mixed",
                              cheb_degree="auto")
    for s_, m, t, sd in zip(stacks, maps, Tb, sb):
        assert sd["cheb_degree"] == max(degs)
        assert rise_err(t.cpu().numpy(), _ref_steady(s_, m), s_.t_amb) <= 1e-8
    for gg in grids:
        gg.close()


@pytest.mark.parametrize("pcname", ["chebyshev", "jacobi", "none"])
def test_csr_storage_pcg(pcname):
    """The CSR baseline storage (Ablation I; Ablation III with the optimisation
    off) runs the same FP64 PCG with row-wise CSR products: the same CG
    iteration count as the stencil within 2 (sums in another order), and both
    meet the FP64 bar against the direct oracle, on config 0 and on a ragged
    grid with per-cell multipliers; one backward-Euler step on CSR matches the
    oracle too.  CSR with mixed precision, or in a batch, is refused."""
    import paper_2606_17850_amd as cuth
    say(f"csr storage {pcname}")
    for st, P in (w.config0(), (ragged_stack(70, 9, mult=True), None)):
        if P is None:
            P = np.zeros(st.shape)
            P[0] = np.random.default_rng(6).uniform(0, 2e-3, (st.ny, st.nx))
        ref = _ref_steady(st, P)
        g = grid_of(st)
        kw = dict(precision="fp64", preconditioner=pcname, max_inner=20000,
                  check_period=0 if pcname == "chebyshev" else 20000)
        Ts, ss = g.solve(t64(P), **kw)
        Tc, sc = g.solve(t64(P), storage="csr", **kw)
        ec = rise_err(Tc.cpu().numpy(), ref, st.t_amb)
        say(f"  {st.shape} stencil {ss['cg_iters']} csr {sc['cg_iters']} err {ec:.2e}")
        assert abs(sc["cg_iters"] - ss["cg_iters"]) <= 2
        assert ec <= 1e-9
        assert sc["rel_residual"] <= 1e-10
        if pcname == "chebyshev" and st.n < 10000:
            dt = 1e-4
            th0 = np.random.default_rng(8).uniform(0, 5.0, st.n)
            ref_tr = transient.step(st, P.ravel(), th0, dt)
            Tt, _ = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision="fp64",
                                     storage="csr")
            got = Tt.cpu().numpy() - st.t_amb
            assert np.abs(got - ref_tr).max() <= 1e-10 * np.abs(ref_tr).max()
        if pcname == "none":
            with pytest.raises(cuth.CuthError) as e:
                g.solve(t64(P), precision="mixed", storage="csr")
            assert e.value.status == cuth._lib.CUTH_E_INVALID
            with pytest.raises(cuth.CuthError) as e:
                cuth.solve_batch([g], [t64(P)], nrhs=1, precision="fp64", storage="csr")
            assert e.value.status == cuth._lib.CUTH_E_INVALID
        g.close()


@pytest.mark.parametrize("shape", ["2,8", "1,1", "3,4", "2,64"])
@pytest.mark.parametrize("case", ["ragged_mult", "ragged_uniform", "c0"])
def test_fused_sweep_pairs(monkeypatch, case, shape):
    """General Chebyshev sweeps fused in pairs (two sweeps per pass, halo rows
    and layers recomputed per workgroup): the FP32 preconditioner against the
    oracle's polynomial, and against the same polynomial with single sweeps,
    for degrees with no pair (5), one pair (6) and the default (30), and
    workgroup shapes from one row and one layer to chunks deeper than the stack."""
    say(f"fused sweeps {case} shape {shape}")
    st = CASES[case]()
    A = assembly.assemble(st)
    lmin, lmax = krylov.spectral_bounds(A, w.lanczos_start(st.n))
    r = np.random.default_rng(11).standard_normal(st.n)
    g = grid_of(st)
    A16 = None
    if st.k_lat_mult is not None:
        A16 = assembly.assemble(st, cond=assembly.fp16_lateral(assembly.conductances(st)))
    for degree in (5, 6, 30):
        ref = krylov.chebyshev_precondition(lambda v: A @ v, r, lmin, lmax, degree)
        monkeypatch.setenv("CUTH_FUSE", "0")
        z1 = g.precond_apply(t32(r), lmin, lmax, degree).cpu().numpy().astype(np.float64)
        monkeypatch.setenv("CUTH_FUSE", "1")
        monkeypatch.setenv("CUTH_FUSE_SHAPE", shape)
        z2 = g.precond_apply(t32(r), lmin, lmax, degree).cpu().numpy().astype(np.float64)
        assert np.abs(z2 - ref).max() <= fp32_cheb_bar(A, r, lmin, lmax, degree, ref)
        # same arithmetic in the same order as two single sweeps
        assert np.abs(z2 - z1).max() <= 1e-6 * np.abs(z1).max()
        if A16 is not None:
            # and with the FP16-stored conductances
            ref16 = krylov.chebyshev_precondition(lambda v: A16 @ v, r, lmin, lmax, degree)
            z3 = g.precond_apply(t32(r), lmin, lmax, degree, fp16_coef=True).cpu().numpy()
            assert np.abs(z3.astype(np.float64) - ref16).max() <= \
                fp32_cheb_bar(A16, r, lmin, lmax, degree, ref16)
    g.close()


@pytest.mark.parametrize("shape", ["4,8", "2,8", "1,1", "3,4", "2,64"])
@pytest.mark.parametrize("case", ["ragged_mult", "ragged_uniform", "c0"])
def test_fused_sweep_triples(monkeypatch, case, shape):
    """General Chebyshev sweeps fused in threes (z_{j+1} kept on chip, two halo
    rows and layers per side): the FP32 preconditioner against the oracle's
    polynomial and against single sweeps.  Sweep 1 is always single and the
    last sweep (which forms the r^T z partials) too; triples start at sweep 2
    (forming z_1 = r / theta themselves) and pairs fill what a triple cannot:
    degree 6 runs one triple (2-4), 7 one triple and a single sweep (5), 8 a
    triple and a pair (5-6), 9 two triples (2-4, 5-7) and 30 nine triples
    (2-28); workgroup shapes from one row and one layer to chunks deeper than
    the stack."""
    say(f"fused triples {case} shape {shape}")
    st = CASES[case]()
    A = assembly.assemble(st)
    lmin, lmax = krylov.spectral_bounds(A, w.lanczos_start(st.n))
    r = np.random.default_rng(13).standard_normal(st.n)
    g = grid_of(st)
    A16 = None
    if st.k_lat_mult is not None:
        A16 = assembly.assemble(st, cond=assembly.fp16_lateral(assembly.conductances(st)))
    for degree in (6, 7, 8, 9, 30):
        ref = krylov.chebyshev_precondition(lambda v: A @ v, r, lmin, lmax, degree)
        monkeypatch.setenv("CUTH_FUSE", "0")
        z1 = g.precond_apply(t32(r), lmin, lmax, degree).cpu().numpy().astype(np.float64)
        monkeypatch.setenv("CUTH_FUSE", "1")
        monkeypatch.setenv("CUTH_FUSE_SHAPE", "2,8")
        monkeypatch.setenv("CUTH_FUSE3", "1")
        monkeypatch.setenv("CUTH_FUSE3_SHAPE", shape)
        z2 = g.precond_apply(t32(r), lmin, lmax, degree).cpu().numpy().astype(np.float64)
        monkeypatch.delenv("CUTH_FUSE3")
        assert np.abs(z2 - ref).max() <= fp32_cheb_bar(A, r, lmin, lmax, degree, ref)
        # same arithmetic in the same order as three single sweeps
        assert np.abs(z2 - z1).max() <= 1e-6 * np.abs(z1).max()
        if A16 is not None:
            monkeypatch.setenv("CUTH_FUSE3", "1")
            ref16 = krylov.chebyshev_precondition(lambda v: A16 @ v, r, lmin, lmax, degree)
            z3 = g.precond_apply(t32(r), lmin, lmax, degree, fp16_coef=True).cpu().numpy()
            monkeypatch.delenv("CUTH_FUSE3")
            assert np.abs(z3.astype(np.float64) - ref16).max() <= \
                fp32_cheb_bar(A16, r, lmin, lmax, degree, ref16)
    g.close()


@pytest.mark.parametrize("shape", ["4,8", "1,1", "2,2"])
@pytest.mark.parametrize("dims", [(1, 1, 1), (65, 3, 1), (33, 2, 2), (70, 9, 3), (7, 21, 2)])
def test_fused_triples_shallow_and_narrow(monkeypatch, dims, shape):
    """Forced fused triples on stacks of 1-3 layers and on grids narrower or
    shorter than a workgroup (one cell, one row, a ragged lane tail): the
    closing iterations of stages B and C carry most of the work there.  The
    FP32 preconditioner equals single sweeps to 1e-6 of its scale and the
    oracle's polynomial to the FP32 bar."""
    nx, ny, nl = dims
    layers = ("Si", "BEOL", "Cu")[:nl] if nl < 3 else ("Si", "bond", "Cu")
    say(f"shallow triples {dims} shape {shape}")
    st = ragged_stack(nx, ny, layers=layers, mult=True, seed=5)
    A = assembly.assemble(st)
    lmin, lmax = krylov.spectral_bounds(A, w.lanczos_start(st.n))
    # a widened interval (a one-cell grid has lmin = lmax); both sides use it
    lmin, lmax = 0.9 * lmin, 1.05 * lmax
    r = np.random.default_rng(17).standard_normal(st.n)
    g = grid_of(st)
    for degree in (6, 9):
        ref = krylov.chebyshev_precondition(lambda v: A @ v, r, lmin, lmax, degree)
        monkeypatch.setenv("CUTH_FUSE", "0")
        z1 = g.precond_apply(t32(r), lmin, lmax, degree).cpu().numpy().astype(np.float64)
        monkeypatch.setenv("CUTH_FUSE", "1")
        monkeypatch.setenv("CUTH_FUSE_SHAPE", "2,8")
        monkeypatch.setenv("CUTH_FUSE3", "1")
        monkeypatch.setenv("CUTH_FUSE3_SHAPE", shape)
        z3 = g.precond_apply(t32(r), lmin, lmax, degree).cpu().numpy().astype(np.float64)
        monkeypatch.delenv("CUTH_FUSE3")
        assert np.abs(z3 - z1).max() <= 1e-6 * np.abs(z1).max()
        assert np.abs(z3 - ref).max() <= fp32_cheb_bar(A, r, lmin, lmax, degree, ref)
    g.close()


@pytest.mark.parametrize("dims", [(520, 7, 5, True), (1024, 6, 3, False), (262, 5, 4, True),
                                  (131, 6, 5, False)])
@pytest.mark.parametrize("pc", ["chebyshev", "chebyshev_jacobi"])
def test_fused_x_windows(monkeypatch, dims, pc):
    """Fused pairs and triples over rows longer than a workgroup row, split
    into overlapping x windows (one or two wavefronts per row, halo lanes at
    each window's edges): lane widths 4, 2 and 1, a last window that is only
    partly inside the grid, per-cell and per-layer conductances, the paper's
    polynomial and the Jacobi-scaled one.  Against single sweeps (same
    arithmetic, 1e-6 of the scale) and the oracle (FP32 bar)."""
    nx, ny, nl, mult = dims
    layers = ("Si", "BEOL", "bond", "TIM", "Cu")[:nl]
    say(f"x windows {dims} {pc}")
    st = ragged_stack(nx, ny, layers=layers, mult=mult, seed=19)
    A = assembly.assemble(st)
    jac = pc == "chebyshev_jacobi"
    if jac:
        lmin, lmax = krylov.jacobi_spectral_bounds(A, w.lanczos_start(st.n))
    else:
        lmin, lmax = krylov.spectral_bounds(A, w.lanczos_start(st.n))
    r = np.random.default_rng(23).standard_normal(st.n)
    g = grid_of(st)
    for degree in (6, 9, 30):
        if jac:
            ref = krylov.jacobi_chebyshev_precondition(A, r, lmin, lmax, degree)
        else:
            ref = krylov.chebyshev_precondition(lambda v: A @ v, r, lmin, lmax, degree)
        bar = fp32_cheb_bar(A, r, lmin, lmax, degree, ref, jacobi=jac)
        monkeypatch.setenv("CUTH_FUSE", "0")
        z1 = g.precond_apply(t32(r), lmin, lmax, degree, preconditioner=pc).cpu().numpy().astype(np.float64)
        for pair, triple in (("4,8,1", None), ("2,3,2", None), ("2,8,1", "8,4,1"), ("2,8,1", "3,16,2"),
                             ("2,8", "2,8,1")):
            monkeypatch.setenv("CUTH_FUSE", "1")
            monkeypatch.setenv("CUTH_FUSE_SHAPE", pair)
            if triple:
                monkeypatch.setenv("CUTH_FUSE3", "1")
                monkeypatch.setenv("CUTH_FUSE3_SHAPE", triple)
            z2 = g.precond_apply(t32(r), lmin, lmax, degree, preconditioner=pc).cpu().numpy().astype(np.float64)
            if triple:
                monkeypatch.delenv("CUTH_FUSE3")
            assert np.abs(z2 - z1).max() <= 1e-6 * np.abs(z1).max(), (degree, pair, triple)
            assert np.abs(z2 - ref).max() <= bar, (degree, pair, triple)
    g.close()


def test_fused_triple_solves(monkeypatch):
    """Mixed solves with fused sweep triples (and pairs for the rest) reach the
    1e-8 bar: steady on a lognormal and a uniform grid, one backward-Euler step,
    and a two-grid batch; the timed launches are the triples."""
    import paper_2606_17850_amd as cuth
    say("fused triple solves")
    monkeypatch.setenv("CUTH_FUSE", "1")
    monkeypatch.setenv("CUTH_FUSE_SHAPE", "2,8")
    monkeypatch.setenv("CUTH_FUSE3", "1")
    monkeypatch.setenv("CUTH_FUSE3_SHAPE", "4,8")
    for st, P in (w.config4_small(), w.config0()):
        g = grid_of(st)
        g.profile_enable(True)
        T, stats = g.solve(t64(P), precision="mixed")
        prof = g.profile_read()
        g.profile_enable(False)
        err = rise_err(T.cpu().numpy(), _ref_steady(st, P), st.t_amb)
        say(f"  err {err:.3e} cg {stats['cg_iters']} {prof}")
        assert err <= 1e-8
        assert prof["fused"] == 2 and prof["launches"] % 8 == 0
        dt = 1e-4
        th0 = np.random.default_rng(12).uniform(0, 5.0, st.n)
        ref_tr = transient.step(st, P.ravel(), th0, dt)
        Tt, _ = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision="mixed")
        assert np.abs(Tt.cpu().numpy() - st.t_amb - ref_tr).max() <= 1e-8 * np.abs(ref_tr).max()
        g.close()
    stacks = [ragged_stack(70, 9, mult=True), ragged_stack(131, 6, mult=False)]
    maps = [np.random.default_rng(50 + i).uniform(0, 2e-3, s.n) for i, s in enumerate(stacks)]
    grids = [grid_of(s) for s in stacks]
    Tb, _ = cuth.solve_batch(grids, [t64(m) for m in maps], nrhs=1, precision="mixed")
    for s, m, t in zip(stacks, maps, Tb):
        assert rise_err(t.cpu().numpy(), _ref_steady(s, m), s.t_amb) <= 1e-8
    for gg in grids:
        gg.close()


def test_triples_forced_through_tuner(monkeypatch):
    """CUTH_FUSE3=1 with the pair shape left to the tuner: the tuner keeps its
    pair choice and adds the first triple shape that fits; the solve meets the
    1e-8 bar with triples as the timed launches, and CUTH_FUSE3=0 keeps them
    off."""
    say("triples forced through the tuner")
    monkeypatch.delenv("CUTH_FUSE", raising=False)
    st, P = w.config4_small()
    ref = _ref_steady(st, P)
    for f3, want in (("1", 2), ("0", 1)):
        monkeypatch.setenv("CUTH_FUSE3", f3)
        g = grid_of(st)   # a fresh handle: the tuner's choice is cached per grid signature
        g.profile_enable(True)
        T, stats = g.solve(t64(P), precision="mixed")
        prof = g.profile_read()
        g.profile_enable(False)
        g.close()
        err = rise_err(T.cpu().numpy(), ref, st.t_amb)
        say(f"  CUTH_FUSE3={f3}: err {err:.3e} {prof}")
        assert err <= 1e-8
        assert prof["fused"] <= want
        if f3 == "1":
            assert prof["fused"] == 2


def test_fused_sweep_solves(monkeypatch):
    """Mixed solves with fused sweep pairs reach the 1e-8 bar: steady on a
    lognormal and a uniform grid, one backward-Euler step, and a two-grid batch."""
    import paper_2606_17850_amd as cuth
    say("fused sweep solves")
    monkeypatch.setenv("CUTH_FUSE", "1")
    for st, P in (w.config4_small(), w.config0()):
        g = grid_of(st)
        T, stats = g.solve(t64(P), precision="mixed")
        err = rise_err(T.cpu().numpy(), _ref_steady(st, P), st.t_amb)
        say(f"  err {err:.3e} cg {stats['cg_iters']}")
        assert err <= 1e-8
        dt = 1e-4
        th0 = np.random.default_rng(12).uniform(0, 5.0, st.n)
        ref_tr = transient.step(st, P.ravel(), th0, dt)
        Tt, _ = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision="mixed")
        assert np.abs(Tt.cpu().numpy() - st.t_amb - ref_tr).max() <= 1e-8 * np.abs(ref_tr).max()
        g.close()
    stacks = [ragged_stack(70, 9, mult=True), ragged_stack(131, 6, mult=False)]
    maps = [np.random.default_rng(50 + i).uniform(0, 2e-3, s.n) for i, s in enumerate(stacks)]
    grids = [grid_of(s) for s in stacks]
    Tb, _ = cuth.solve_batch(grids, [t64(m) for m in maps], nrhs=1, precision="mixed")
    for s, m, t in zip(stacks, maps, Tb):
        assert rise_err(t.cpu().numpy(), _ref_steady(s, m), s.t_amb) <= 1e-8
    for gg in grids:
        gg.close()


@pytest.mark.parametrize("fuse", ["0", "1", "3"])
def test_kernel_timing_blocks(monkeypatch, fuse):
    """The measurement hook times whole back-to-back runs of the general FP32
    kernel from sweep 3 on: at k = 30 every preconditioner application
    contributes 8 fused triples (sweeps 5-28; the first triple, 2-4, forms z_1
    itself and is not in the block), 13 fused pairs (sweeps 3-28) or 26 single
    sweeps (3-28), so the launch count is a multiple of that, and the bytes per
    launch are those of the kernel timed (28, 28 or 24 B per unknown on a
    per-cell grid)."""
    say(f"kernel timing blocks, fusion {fuse}")
    monkeypatch.setenv("CUTH_FUSE", "0" if fuse == "0" else "1")
    monkeypatch.setenv("CUTH_FUSE_SHAPE", "2,8")
    monkeypatch.setenv("CUTH_FUSE3", "1" if fuse == "3" else "0")
    monkeypatch.setenv("CUTH_FUSE3_SHAPE", "4,8")
    st, P = w.config4_small()
    g = grid_of(st)
    g.profile_enable(True)
    T, stats = g.solve(t64(P), precision="mixed", cheb_degree=30)
    prof = g.profile_read()
    g.profile_enable(False)
    g.close()
    per = {"0": 26, "1": 13, "3": 8}[fuse]
    say(f"  {prof} cg {stats['cg_iters']}")
    assert prof["fused"] == {"0": 0, "1": 1, "3": 2}[fuse]
    assert prof["launches"] >= per and prof["launches"] % per == 0
    assert prof["launches"] <= per * (stats["cg_iters"] + stats["outer_cycles"] + 1)
    assert prof["bytes_per_launch"] == (24 if fuse == "0" else 28) * st.n
    assert prof["total_ms"] > 0


def test_solve_single_cell_and_zero_power():
    say("solve single cell / zero power")
    st = w.Stack(1, 1, ["Cu"])
    g = grid_of(st)
    T, _ = g.solve(t64(np.array([2e-3])), precision="mixed")
    exact = st.t_amb + 2e-3 / (st.h_top * st.dx * st.dy)
    assert T.cpu().numpy()[0] == pytest.approx(exact, rel=1e-10)
    g.close()
    st2, _ = w.config0()
    g2 = grid_of(st2)
    T0, stats = g2.solve(t64(np.zeros(st2.n)), precision="mixed")
    assert np.all(T0.cpu().numpy() == st2.t_amb)
    g2.close()


def test_transient_steps_match_oracle():
    say("transient c0-stack 4 steps")
    st = w.uniform_stack(64, 48, ["Si", "BEOL", "bond", "Si", "BEOL", "bond", "TIM", "Cu"])
    rng = np.random.default_rng(7)
    Ps = [rng.uniform(0, 2e-3, st.n) for _ in range(2)]
    dt = 1e-4
    g = grid_of(st)
    for prec, tol in (("mixed", 1e-8), ("fp64", 1e-10)):
        th = np.zeros(st.n)
        T = t64(st.t_amb + th)
        for s in range(4):
            P = Ps[s // 2]
            ref_th = transient.step(st, P, th, dt)
            T, stats = g.transient_step(dt, t64(P), T, precision=prec)
            got = T.cpu().numpy()
            err = np.abs(got - (st.t_amb + ref_th)).max() / np.abs(ref_th).max()
            say(f"  {prec} step {s} err {err:.2e} cg {stats['cg_iters']}")
            assert err <= tol
            th = got - st.t_amb      # strict per-step parity from the GPU's own state
    g.close()


def test_invalid_and_failure_paths():
    import paper_2606_17850_amd as cuth
    say("failure paths")
    st = w.Stack(8, 8, ["Si", "Cu"], h_top=0.0)
    g = grid_of(st)
    with pytest.raises(cuth.CuthError) as e:
        g.solve(t64(np.ones(st.n) * 1e-3))
    assert e.value.status == cuth._lib.CUTH_E_INVALID
    st2, P = w.config0()
    g2 = grid_of(st2)
    with pytest.raises(cuth.CuthError) as e:
        g2.transient_step(-1.0, t64(P), t64(np.full(st2.n, 300.0)))
    assert e.value.status == cuth._lib.CUTH_E_INVALID
    bad = P.ravel().copy()
    bad[5] = np.nan
    with pytest.raises(cuth.CuthError) as e:
        g2.solve(t64(bad))
    assert e.value.status == cuth._lib.CUTH_E_BREAKDOWN
    with pytest.raises(cuth.CuthError) as e:
        g2.solve(t64(P), precision="mixed", max_inner=1, max_outer=1)
    assert e.value.status == cuth._lib.CUTH_E_NOT_CONVERGED
    assert e.value.stats is not None and e.value.stats["cg_iters"] >= 1
    g.close()
    g2.close()


def test_inner_stop_on_drift():
    """Eq. switching (c), drift: FP64 Chebyshev-PCG asked for an unattainable
    relative residual (1e-300).  Its recursive residual keeps falling
    geometrically while the true residual rhat - A x settles at the FP64
    rounding floor, so the inner solves end on ||r_true - r_low|| >=
    0.5 ||r_true|| (checked every 5 iterations).  The hot restarts after them
    cannot halve the true residual, so the call reports NOT_CONVERGED with the
    best iterate, which meets the FP64 bar against the oracle."""
    import paper_2606_17850_amd as cuth
    say("stop rule: drift")
    st, P = w.config0()
    g = grid_of(st)
    T = torch.empty(st.n, dtype=torch.float64, device=dev())
    with pytest.raises(cuth.CuthError) as e:
        g.solve(t64(P), T=T, precision="fp64", tol=1e-300, check_period=5, max_inner=5000)
    s = e.value.stats
    say(f"  {s}")
    assert e.value.status == cuth._lib.CUTH_E_NOT_CONVERGED
    # the last inner solve stopped on drift, the first one too (its recursive
    # residual falls through the floor of a true residual that started at
    # ||b||); a hot-restarted one may stop earlier, on the plateau of its true
    # residual (stagnation), which is the other test of the same floor
    assert s["stop_reason"] == 2
    assert s["drift_stops"] >= 2 and s["outer_cycles"] >= 2
    assert s["drift_stops"] + s["stagnation_stops"] == s["outer_cycles"]
    assert rise_err(T.cpu().numpy(), _ref_steady(st, P), st.t_amb) <= 1e-10
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_inner_stop_on_stagnation(prec):
    """Eq. switching (b), stagnation: plain CG (no preconditioner) with the true
    residual checked after every iteration.  On this stack plain CG's residual
    often falls by less than a tenth from one iteration to the next while the
    recursive residual still falls, so every inner solve ends on
    ||r_true|| > 0.9 ||r_true^prev|| with ||r_low|| < ||r_low^prev||, no
    earlier than the second check (the first with a previous one), and the
    refinement gives up (NOT_CONVERGED).  The best iterate is returned: the
    relative residual the call reports is that of the returned T, recomputed
    by the oracle."""
    import paper_2606_17850_amd as cuth
    say(f"stop rule: stagnation {prec}")
    st, P = w.config0()
    A = assembly.assemble(st)
    g = grid_of(st)
    T = torch.empty(st.n, dtype=torch.float64, device=dev())
    with pytest.raises(cuth.CuthError) as e:
        g.solve(t64(P), T=T, precision=prec, preconditioner="none", check_period=1, max_outer=4)
    s = e.value.stats
    say(f"  {s}")
    assert e.value.status == cuth._lib.CUTH_E_NOT_CONVERGED
    assert s["stop_reason"] == 3
    assert s["stagnation_stops"] == s["outer_cycles"] >= 1
    assert s["drift_stops"] == 0
    assert s["cg_iters"] >= 2 * s["outer_cycles"]
    th = T.cpu().numpy() - st.t_amb
    b = P.ravel()
    relres = np.linalg.norm(b - A @ th) / np.linalg.norm(b)
    assert relres == pytest.approx(s["rel_residual"], rel=1e-6)
    g.close()


def test_run_twice_bitwise_identical():
    say("determinism")
    st, P = w.config4_small()
    g = grid_of(st)
    T1, _ = g.solve(t64(P), precision="mixed")
    T2, _ = g.solve(t64(P), precision="mixed")
    assert torch.equal(T1, T2)
    g.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_graph_replays_match_eager(monkeypatch, prec):
    """Single solves replay captured chunks of CG iterations (kept by the
    handle between solves): three graph solves, with eager solves and
    synchronisations between them, each against the eager result and the
    oracle; the graph replays agree with each other bit for bit."""
    say(f"graph replays {prec}")
    st, P = w.config0()
    ref = st.t_amb + direct.solve_separable(st, P.ravel())
    g = grid_of(st)
    Pt = t64(P)
    monkeypatch.setenv("CUTH_GRAPH", "0")
    T_eager, _ = g.solve(Pt, precision=prec)
    T_eager = T_eager.clone()
    first = None
    for rep in range(3):
        monkeypatch.setenv("CUTH_GRAPH", "1")
        T, s = g.solve(Pt, precision=prec)
        torch.cuda.synchronize()
        T = T.clone()
        assert rise_err(T.cpu().numpy(), ref, st.t_amb) <= (1e-8 if prec == "mixed" else 1e-10)
        assert float((T - T_eager).abs().max()) <= 1e-12 * float((T_eager - st.t_amb).abs().max())
        if first is None:
            first = T
        else:
            assert torch.equal(T, first), rep
        # eager work between the replays
        monkeypatch.setenv("CUTH_GRAPH", "0")
        T2, _ = g.solve(Pt, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(T2, T_eager)
    g.close()


@pytest.mark.parametrize("mult", [True, False])
def test_set_conductivity_matches_new_grid(mult):
    """New layer conductivities set in place answer as a grid built with them:
    the FP64, FP32 and FP16-plane products of the steady and transient
    operators (both cached before the change), the residual, the spectral
    interval, a mixed solve, the Jacobi-scaled preconditioner and the adjoint,
    bit for bit; the solve also against the oracle at the new values."""
    import copy

    import paper_2606_17850_amd as cuth
    say(f"set_conductivity mult={mult}")
    st0 = ragged_stack(70, 9, mult=mult)
    rng = np.random.default_rng(21)
    P = np.zeros(st0.shape)
    P[0] = rng.uniform(0, 2e-3, (st0.ny, st0.nx))
    x = rng.uniform(-1, 1, st0.n) + 2.0
    dt = 1e-4
    g = grid_of(st0)
    # operators, bounds, graphs and stop predictions of the old values
    for d in (0.0, dt):
        g.apply(t64(x), dt=d)
    g.solve(t64(P), precision="mixed")
    g.solve(t64(P), precision="mixed", preconditioner="chebyshev_jacobi")
    st1 = copy.deepcopy(st0)
    st1.k_lat = st0.k_lat * rng.uniform(0.5, 2.0, st0.nz)
    st1.k_vert = st0.k_vert * rng.uniform(0.5, 2.0, st0.nz)
    g.set_conductivity(st1.k_lat, st1.k_vert)
    g1 = grid_of(st1)
    for d in (0.0, dt):
        assert torch.equal(g.apply(t64(x), dt=d), g1.apply(t64(x), dt=d))
        x32 = t64(x).float()
        assert torch.equal(g.apply(x32, dt=d), g1.apply(x32, dt=d))
        if mult:
            assert torch.equal(g.apply(x32, dt=d, fp16_coef=True), g1.apply(x32, dt=d, fp16_coef=True))
        b = t64(P)
        Tx = t64(st0.t_amb + x)
        assert torch.equal(g.residual(b, Tx, dt=d), g1.residual(b, Tx, dt=d))
    sb, sb1 = g.spectral_bounds(), g1.spectral_bounds()
    assert sb["lmin"] == sb1["lmin"] and sb["lmax"] == sb1["lmax"]
    T, s = g.solve(t64(P), precision="mixed")
    T1, s1 = g1.solve(t64(P), precision="mixed")
    assert torch.equal(T, T1) and s["cg_iters"] == s1["cg_iters"]
    assert rise_err(T.cpu().numpy(), _ref_steady(st1, P), st1.t_amb) <= 1e-8
    Tj, _ = g.solve(t64(P), precision="mixed", preconditioner="chebyshev_jacobi")
    Tj1, _ = g1.solve(t64(P), precision="mixed", preconditioner="chebyshev_jacobi")
    assert torch.equal(Tj, Tj1)
    gT = t64(rng.uniform(0, 1, st0.n))
    dP, dk, _ = g.adjoint(T, gT)
    dP1, dk1, _ = g1.adjoint(T1, gT)
    assert torch.equal(dP, dP1) and torch.equal(dk, dk1)
    g1.close()
    g.close()


def test_set_conductivity_rejections():
    """Host checks leave the grid as it was; a multiplier that the device check
    rejects leaves it refusing calls until a valid set."""
    import paper_2606_17850_amd as cuth
    st = ragged_stack(70, 9, mult=True)
    g = grid_of(st)
    x = t64(np.random.default_rng(22).uniform(1, 2, st.n))
    y0 = g.apply(x)
    bad_k = np.array(st.k_lat, dtype=np.float64)
    bad_k[1] = -1.0
    for kl, kv in ((bad_k, st.k_vert), (st.k_lat, np.full(st.nz, np.nan))):
        with pytest.raises(cuth.CuthError) as e:
            g.set_conductivity(kl, kv)
        assert e.value.status == cuth._lib.CUTH_E_INVALID
    assert torch.equal(g.apply(x), y0)
    # a uniform grid takes no multiplier
    gu = grid_of(ragged_stack(70, 9, mult=False))
    with pytest.raises(cuth.CuthError) as e:
        gu.set_conductivity(st.k_lat, st.k_vert, k_lat_mult=t64(np.ones(st.n)))
    assert e.value.status == cuth._lib.CUTH_E_INVALID
    gu.close()
    # a multiplier with a zero entry, found by the build kernel's own check
    m = np.ascontiguousarray(st.k_lat_mult, dtype=np.float64).ravel().copy()
    m[17] = 0.0
    with pytest.raises(cuth.CuthError) as e:
        g.set_conductivity(st.k_lat, st.k_vert, k_lat_mult=t64(m))
    assert e.value.status == cuth._lib.CUTH_E_INVALID
    with pytest.raises(cuth.CuthError) as e:
        g.apply(x)
    assert e.value.status == cuth._lib.CUTH_E_INVALID
    g.set_conductivity(st.k_lat, st.k_vert,
                       k_lat_mult=t64(np.ascontiguousarray(st.k_lat_mult, dtype=np.float64).ravel()))
    assert torch.equal(g.apply(x), y0)
    g.close()


def test_max_layer_count(monkeypatch):
    """64 layers, the descriptor's limit (the adjoint's per-layer sums fill
    their arrays): steady mixed and FP64 solves against the direct oracle, the
    same with fused pairs and triples forced, a backward-Euler step, and the
    adjoint's dL/dP and per-layer dL/dk against the oracle gradient.

    With the heat sink on top only, 64 layers in series give a condition
    number near 3e6, so condition number times the FP32 unit roundoff is about
    0.2 and the error of an FP32 inner solve can lag its residual by orders of
    magnitude; CG's residual also rises for stretches here, which the
    stagnation test must not take for stagnation.  The mixed solves (fixed and
    automatic Chebyshev degree) must still meet the 1e-8 bar, and the FP64
    adjoint its default tolerance."""
    import paper_2606_17850_amd as cuth
    from oracle import adjoint as oadj
    layers = (["Si", "BEOL", "bond", "TIM"] * 16)[:63] + ["Cu"]
    st = ragged_stack(20, 12, layers=layers, mult=True, seed=31)
    assert st.nz == 64
    rng = np.random.default_rng(32)
    P = np.zeros(st.shape)
    for l, name in enumerate(layers):
        if name == "Si":
            P[l] = rng.uniform(0, 2e-5, (st.ny, st.nx))
    A = assembly.assemble(st)
    th_ref = direct.solve_splu(A, P.ravel())
    g = grid_of(st)
    for prec, kw, bar in (("mixed", {}, 1e-8), ("mixed", {"cheb_degree": "auto"}, 1e-8),
                          ("mixed16", {}, 1e-8), ("fp64", {}, 1e-10), ("adaptive", {}, 1e-10)):
        T, s = g.solve(t64(P), precision=prec, **kw)
        err = rise_err(T.cpu().numpy(), st.t_amb + th_ref, st.t_amb)
        say(f"64 layers {prec} {kw} err {err:.2e} cycles {s['outer_cycles']} "
            f"stagnation stops {s['stagnation_stops']}")
        assert err <= bar
    # batched with a 5-layer stack: each system keeps its own stop decisions
    st5 = ragged_stack(70, 9, mult=True)
    P5 = np.zeros(st5.shape)
    P5[0] = 1e-5
    g5 = grid_of(st5)
    Tb, _ = cuth.solve_batch([g, g5], [t64(P), t64(P5)], nrhs=1, precision="mixed")
    assert rise_err(Tb[0].cpu().numpy(), st.t_amb + th_ref, st.t_amb) <= 1e-8
    assert rise_err(Tb[1].cpu().numpy(), _ref_steady(st5, P5), st5.t_amb) <= 1e-8
    g5.close()
    monkeypatch.setenv("CUTH_FUSE", "1")
    monkeypatch.setenv("CUTH_FUSE_SHAPE", "2,8")
    monkeypatch.setenv("CUTH_FUSE3", "1")
    monkeypatch.setenv("CUTH_FUSE3_SHAPE", "2,8")
    Tf, _ = g.solve(t64(P), precision="mixed")
    assert rise_err(Tf.cpu().numpy(), st.t_amb + th_ref, st.t_amb) <= 1e-8
    for k in ("CUTH_FUSE", "CUTH_FUSE_SHAPE", "CUTH_FUSE3", "CUTH_FUSE3_SHAPE"):
        monkeypatch.delenv(k)
    # backward-Euler steps from short to stiff: at dt = 1 s and 100 s the step
    # is nearly the steady system, whose FP64 residual floor lies above the
    # transient default of 1e-12 (the default then accepts up to 1e-10)
    th0 = rng.uniform(0, 5.0, st.n)
    for dt in (1e-4, 1.0, 100.0):
        ref_tr = transient.step(st, P.ravel(), th0, dt)
        for prec, bar in (("mixed", 1e-8), ("mixed16", 1e-8), ("fp64", 1e-10), ("adaptive", 1e-10)):
            Tt, s = g.transient_step(dt, t64(P), t64(st.t_amb + th0), precision=prec)
            err = np.abs(Tt.cpu().numpy() - st.t_amb - ref_tr).max() / np.abs(ref_tr).max()
            say(f"64 layers dt {dt:g} {prec} err {err:.2e} relres {s['rel_residual']:.1e}")
            assert err <= bar
    T, _ = g.solve(t64(P), precision="fp64")
    Tn = T.cpu().numpy()
    gT = oadj.lse_grad(Tn, st.si_mask(), 0.5)
    ref = oadj.gradient(st, Tn - st.t_amb, gT, direct.solve_splu)
    for prec in ("fp64", "mixed", "mixed16"):
        dP, dk, _ = g.adjoint(T, t64(gT), precision=prec)
        eP = np.abs(dP.cpu().numpy() - ref.dP).max() / np.abs(ref.dP).max()
        say(f"64 layers adjoint {prec} dP err {eP:.2e}")
        assert eP <= 1e-6
        assert dk.shape == (64,)
        np.testing.assert_allclose(dk.cpu().numpy(), ref.dk_layer, rtol=1e-6,
                                   atol=1e-9 * np.abs(ref.dk_layer).max())
    g.close()


def _extreme_stack(name):
    """Stacks at the edges of the solver's range (condition numbers from the
    oracle's sparse eigensolver in the comments)."""
    eight = ["Si", "BEOL", "bond", "Si", "BEOL", "bond", "TIM", "Cu"]
    if name == "column64":        # one column of 64 layers (1.3e4)
        return ragged_stack(1, 1, layers=(["Si", "BEOL", "bond", "TIM"] * 16)[:63] + ["Cu"], mult=False)
    if name == "bottom_sink":     # the heat leaves through the bottom only (5.6e4)
        st = ragged_stack(70, 9, mult=True)
        st.h_top, st.h_bottom = 0.0, 1e4
        return st
    if name == "both_sinks":      # both faces cooled (4.7e4)
        st = ragged_stack(70, 9, mult=True)
        st.h_bottom = 1e3
        return st
    st = ragged_stack(40, 24, layers=eight, mult=True)
    if name == "contrast":        # lognormal lateral multipliers, sigma 2 (4.5e6)
        st.k_lat_mult = np.exp(2.0 * np.random.default_rng(5).standard_normal(st.shape))
    elif name == "weak_layer":    # a TIM layer of 0.01 W/(m K) (2.5e6)
        st.k_vert = np.array(st.k_vert, float)
        st.k_lat = np.array(st.k_lat, float)
        st.k_vert[6] = st.k_lat[6] = 0.01
    elif name == "thin_layers":   # layers from 1 um to 1 mm thick (1.3e6)
        st.dz = np.array([5e-5, 2e-6, 1e-6, 5e-5, 2e-6, 1e-6, 2e-5, 1e-3])
    return st


@pytest.mark.parametrize("name", ["column64", "bottom_sink", "both_sinks", "contrast",
                                  "weak_layer", "thin_layers"])
def test_extreme_stacks(name):
    """Steady solves in every precision against the direct oracle on stacks
    with one cooled face or two, extreme conductivity contrast, a near-
    insulating layer and a thousandfold spread of layer thicknesses: the mixed
    modes to 1e-8 and the FP64 ones to 1e-10 rise error.  Then the adjoint
    (mixed and FP64) against the oracle gradient of the log-sum-exp of the
    silicon temperatures, to the bars of the small adjoint test."""
    from oracle import adjoint as oadj
    st = _extreme_stack(name)
    rng = np.random.default_rng(3)
    P = np.zeros(st.shape)
    for l, m in enumerate(st.layers):
        if m == "Si":
            P[l] = rng.uniform(0, 2e-5, (st.ny, st.nx))
    ref = _ref_steady(st, P)
    g = grid_of(st)
    for prec, bar in (("mixed", 1e-8), ("mixed16", 1e-8), ("fp64", 1e-10), ("adaptive", 1e-10)):
        T, s = g.solve(t64(P), precision=prec)
        err = rise_err(T.cpu().numpy(), ref, st.t_amb)
        say(f"  {name} {prec} err {err:.2e} cycles {s['outer_cycles']} cg {s['cg_iters']}")
        assert err <= bar
    Tn = ref                       # the adjoint linearises at the exact state
    gT = oadj.lse_grad(Tn, st.si_mask(), 0.5)
    gref = oadj.gradient(st, Tn - st.t_amb, gT, direct.solve_splu)
    for prec in ("mixed", "fp64"):
        dP, dk, _ = g.adjoint(t64(Tn), t64(gT), precision=prec)
        eP = np.abs(dP.cpu().numpy() - gref.dP).max() / np.abs(gref.dP).max()
        say(f"  {name} adjoint {prec} dP err {eP:.2e}")
        assert eP <= 1e-6
        np.testing.assert_allclose(dk.cpu().numpy(), gref.dk_layer, rtol=1e-6,
                                   atol=1e-9 * np.abs(gref.dk_layer).max())
    g.close()


def test_extreme_stacks_batched():
    """All six edge stacks in one batched call (a matrix-free group and a
    per-cell group), mixed and FP64: each problem keeps its own spectral
    interval, inner tolerance and stop decisions, and meets the single-solve
    bars against the direct oracle."""
    import paper_2606_17850_amd as cuth
    names = ["column64", "bottom_sink", "both_sinks", "contrast", "weak_layer", "thin_layers"]
    stacks = [_extreme_stack(n) for n in names]
    rng = np.random.default_rng(4)
    Ps, refs = [], []
    for st in stacks:
        P = np.zeros(st.shape)
        for l, m in enumerate(st.layers):
            if m == "Si":
                P[l] = rng.uniform(0, 2e-5, (st.ny, st.nx))
        Ps.append(P)
        refs.append(_ref_steady(st, P))
    grids = [grid_of(st) for st in stacks]
    for prec, bar in (("mixed", 1e-8), ("fp64", 1e-10)):
        T, stats = cuth.solve_batch(grids, [t64(P) for P in Ps], nrhs=1, precision=prec)
        for name, st, t, ref, s in zip(names, stacks, T, refs, stats):
            err = rise_err(t.cpu().numpy(), ref, st.t_amb)
            say(f"  batched {name} {prec} err {err:.2e} cycles {s['outer_cycles']} cg {s['cg_iters']}")
            assert err <= bar
    for g in grids:
        g.close()
