"""Chebyshev polynomial preconditioning, Lanczos and PCG in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``chebyshev_residual_poly`` - the closed form of the degree-k Chebyshev
  residual polynomial P_k(lambda) = C_k((theta - lambda)/delta) / C_k(theta/delta),
  theta = (beta + alpha)/2, delta = (beta - alpha)/2 (Section 4.3, eqs. for P_k
  and the three-term recurrence of C_k).  C_k(t) is cos(k acos t) on [-1, 1] and
  sign(t)^k cosh(k acosh|t|) outside.
* ``chebyshev_precondition`` - the paper's "Chebyshev Polynomial
  Preconditioning" algorithm, steps in the paper's order: z starts at zero,
  d_0 = r/theta, then k times z += d, r_cheb -= A d,
  rho_{i+1} = 1/(2 sigma_1 - rho_i), d_{i+1} = rho_{i+1} rho_i d_i +
  (2 rho_{i+1}/delta) r_cheb.  In exact arithmetic its output is
  (1 - P_k(A)) A^{-1} r, which the closed form pins.
* ``lanczos`` - m steps of the symmetric Lanczos process (no
  re-orthogonalisation) returning the tridiagonal T (Section 4.3, last
  paragraph); ``ritz_extremes`` takes its extreme eigenvalues with a library
  routine.
* ``pcg`` - Algorithm 1 (preconditioned CG) with the stopping test
  ||r_k||_2 > eps on the recursive residual.
* ``jacobi_chebyshev_precondition`` / ``jacobi_spectral_bounds`` - an
  extension beyond the paper: the same Chebyshev algorithm applied to the
  Jacobi-scaled system D^{-1} A x = D^{-1} r (D = diag(A)), i.e.
  z = q_k(D^{-1} A) D^{-1} r, with the interval of D^{-1} A (the spectrum of
  the symmetric S = D^{-1/2} A D^{-1/2}) from Lanczos on S, capped above by 2
  (Gershgorin: |lambda - 1| <= sum_{j != i} |a_ij| / a_ii <= 1 for a
  diagonally dominant A with positive diagonal).
"""

from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np

Matvec = Callable[[np.ndarray], np.ndarray]


def chebyshev_first_kind(k: int, t: np.ndarray) -> np.ndarray:
    """C_k(t) evaluated without the recurrence (trig / hyperbolic closed form)."""
    t = np.asarray(t, float)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(k * np.arccos(t[inside]))
    ti = t[~inside]
    out[~inside] = np.sign(ti) ** k * np.cosh(k * np.arccosh(np.abs(ti)))
    return out


def chebyshev_residual_poly(lam: np.ndarray, lmin: float, lmax: float, k: int) -> np.ndarray:
    """P_k(lambda) = C_k((theta - lambda)/delta) / C_k(theta/delta)."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    t = (theta - np.asarray(lam, float)) / delta
    return chebyshev_first_kind(k, t) / chebyshev_first_kind(k, np.array([theta / delta]))[0]


def chebyshev_precondition(matvec: Matvec, r_cg: np.ndarray, lmin: float, lmax: float,
                           k: int, dtype=np.float64) -> np.ndarray:
    """z_cg = M^{-1} r_cg by the paper's Chebyshev algorithm (k loop passes).

    ``dtype`` is the precision of the vectors (the scalars rho, theta, delta
    stay FP64 and are rounded where they meet a vector); with float32 and a
    float32 ``matvec`` the same steps run in single precision, which the tests
    use only as a scale for the rounding error of an FP32 application."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    r_ch = np.array(r_cg, dtype=dtype, copy=True)
    sigma1 = theta / delta
    rho = 1.0 / sigma1
    d = r_ch / theta
    z = np.zeros_like(r_ch)
    for _ in range(k):
        z = z + d
        Ad = matvec(d)
        r_ch = r_ch - Ad
        rho_next = 1.0 / (2.0 * sigma1 - rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * r_ch
        rho = rho_next
    return z


def lanczos(matvec: Matvec, v0: np.ndarray, m: int) -> Tuple[np.ndarray, np.ndarray]:
    """m-step Lanczos: diagonal alpha[m] and off-diagonal beta[m-1] of T."""
    v = np.asarray(v0, float) / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    alpha: List[float] = []
    beta: List[float] = []
    for j in range(m):
        w = matvec(v)
        a = float(v @ w)
        w = w - a * v - b_prev * v_prev
        alpha.append(a)
        if j == m - 1:
            break
        b = float(np.linalg.norm(w))
        beta.append(b)
        if b == 0.0:
            break
        v_prev, v, b_prev = v, w / b, b
    return np.array(alpha), np.array(beta)


def ritz_values(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Eigenvalues of the Lanczos tridiagonal, ascending (library eigensolver)."""
    m = len(alpha)
    T = np.diag(alpha)
    if m > 1:
        T += np.diag(beta[: m - 1], 1) + np.diag(beta[: m - 1], -1)
    return np.linalg.eigvalsh(T)


def gershgorin_max(A) -> float:
    """max_i (a_ii + sum_{j != i} |a_ij|) of a CSR matrix."""
    absrow = np.asarray(abs(A).sum(axis=1)).ravel()
    d = A.diagonal()
    return float(np.max(absrow - np.abs(d) + d))


def spectral_bounds(A, v0: np.ndarray, m: int = 30, margin: float = 1.05) -> Tuple[float, float]:
    """(lambda_min, lambda_max) as the solver uses them: the smallest Ritz value,
    and the largest Ritz value times a safety margin capped by Gershgorin."""
    a, b = lanczos(lambda x: A @ x, v0, m)
    ritz = ritz_values(a, b)
    return float(ritz[0]), float(min(gershgorin_max(A), margin * ritz[-1]))


def pcg(matvec: Matvec, b: np.ndarray, precond: Callable[[np.ndarray], np.ndarray],
        x0: np.ndarray, eps: float, maxit: int = 100000) -> Tuple[np.ndarray, int]:
    """Algorithm 1 of the paper; returns (x_k, k)."""
    x = np.array(x0, dtype=float, copy=True)
    r = b - matvec(x)
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    k = 0
    while np.linalg.norm(r) > eps and k < maxit:
        mu = matvec(p)
        alpha = rz / float(p @ mu)
        x = x + alpha * p
        r = r - alpha * mu
        z = precond(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        k += 1
    return x, k


def jacobi_chebyshev_precondition(A, r: np.ndarray, lmin: float, lmax: float,
                                  k: int, dtype=np.float64) -> np.ndarray:
    """z = q_k(D^{-1} A) D^{-1} r: ``chebyshev_precondition`` on the system
    scaled by D^{-1} = diag(A)^{-1} (beyond the paper); lmin, lmax bound the
    spectrum of D^{-1} A.  ``dtype`` as for ``chebyshev_precondition`` (A, its
    diagonal and r rounded to it first)."""
    A = A.astype(dtype)
    d = A.diagonal()
    return chebyshev_precondition(lambda v: (A @ v) / d, np.asarray(r, dtype) / d, lmin, lmax, k,
                                  dtype=dtype)


def jacobi_spectral_bounds(A, v0: np.ndarray, m: int = 30,
                           margin: float = 1.05) -> Tuple[float, float]:
    """Interval of D^{-1} A as the Jacobi-scaled preconditioner uses it: Lanczos
    on S = D^{-1/2} A D^{-1/2} (same spectrum, symmetric), the smallest Ritz
    value, and the largest times the margin capped by 2."""
    s = 1.0 / np.sqrt(A.diagonal())
    a, b = lanczos(lambda x: s * (A @ (s * x)), v0, m)
    ritz = ritz_values(a, b)
    return float(ritz[0]), float(min(2.0, margin * ritz[-1]))
