"""Krylov solver and Chebyshev-Jacobi preconditioner (Sec. 5.3).

Sec. 5.3: conjugate gradients for the symmetric viscous and pressure steps,
double precision in the outer Krylov method and single precision inside the
preconditioner, and a Chebyshev-accelerated Jacobi smoother built on the
precomputed inverse matrix diagonal, whose residuals use the operator action.
The paper gives neither the polynomial degree nor the eigenvalue interval; the
readings taken here are: degree 5, interval [lam/20, lam] with lam 1.2 times
the largest Ritz value of 20 Lanczos steps on D^-1/2 A D^-1/2 from a
reproducible U(-1,1) start vector (SplitMix64, seed 12345).  Because a
single-precision preconditioner is not exactly a fixed symmetric operator,
the outer iteration is the flexible (Polak-Ribiere) variant of CG.
Relative residual: ||b - A x|| / ||b|| from x0 = 0.  When the recursive
residual meets the tolerance the true residual is recomputed and, if it does
not, CG restarts from the current iterate (at most 3 restarts).  For the pure
Neumann Poisson problem the right-hand side, every preconditioned residual
and the solution are projected to zero mean (Sec. 3.2 sets the mean of the
right-hand side to zero in that case).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """Counter-based U(-1, 1): value i is SplitMix64's output for state
    seed + (i+1)*0x9E3779B97F4A7C15 (Steele, Lea and Flood 2014), top 53 bits
    scaled to [0, 1), then mapped to [-1, 1)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(1, n + 1, dtype=np.uint64) * _GAMMA)
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def lanczos_max(apply, dinv: np.ndarray, steps: int = 20, seed: int = 12345) -> float:
    """Largest Ritz value of `steps` Lanczos steps on S = D^-1/2 A D^-1/2."""
    s = np.sqrt(dinv)
    S = lambda v: s * apply(s * v)
    v = splitmix64_uniform(seed, len(dinv))
    v /= np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    alphas, betas = [], []
    beta = 0.0
    for _ in range(steps):
        w = S(v)
        a = float(w @ v)
        w = w - a * v - beta * v_prev
        alphas.append(a)
        beta = float(np.linalg.norm(w))
        if beta == 0.0:
            break
        betas.append(beta)
        v_prev, v = v, w / beta
    m = len(alphas)
    ev = scipy.linalg.eigvalsh_tridiagonal(np.array(alphas), np.array(betas[:m - 1]))
    return float(ev[-1])


def chebyshev_jacobi(apply, dinv: np.ndarray, r: np.ndarray, degree: int,
                     lam_hi: float, lam_lo: float) -> np.ndarray:
    """z ~ A^-1 r by `degree` steps of Chebyshev acceleration of Jacobi from
    z = 0 (degree - 1 operator applications), interval [lam_lo, lam_hi] of
    D^-1 A; three-term recurrence as in Saad, Iterative Methods, Alg. 12.1."""
    theta = 0.5 * (lam_hi + lam_lo)
    delta = 0.5 * (lam_hi - lam_lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    z = dinv * r / theta
    d = z.copy()
    for _ in range(degree - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * (r - apply(z)))
        z = z + d
        rho = rho_new
    return z


def flexible_cg(apply, b, precond, tol, max_iter, x0=None, bnorm=None, project=None):
    """Flexible preconditioned CG with beta = r_new.(z_new - z_old) / (r_old.z_old).

    Returns (x, iterations, status) with status "ok", "not_converged" or
    "breakdown"; convergence is ||r|| <= tol * bnorm for the recursive r."""
    bnorm = float(np.linalg.norm(b)) if bnorm is None else bnorm
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x) if x0 is not None else b.copy()
    if np.linalg.norm(r) <= tol * bnorm:
        return x, 0, "ok"
    z = precond(r)
    if project is not None:
        z = project(z)
    p = z.copy()
    rz = float(r @ z)
    for it in range(1, max_iter + 1):
        q = apply(p)
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            return x, it, "breakdown"
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= tol * bnorm:
            return x, it, "ok"
        z_new = precond(r)
        if project is not None:
            z_new = project(z_new)
        rz_new = float(r @ z_new)
        beta = (rz_new - float(r @ z)) / rz
        p = z_new + beta * p
        z, rz = z_new, rz_new
    return x, max_iter, "not_converged"


def solve(apply, diag: np.ndarray, b: np.ndarray, tol: float = 1e-8, max_iter: int = 2000,
          cheb_degree: int = 5, cheb_ratio: float = 20.0, safety: float = 1.2,
          lanczos_steps: int = 20, seed: int = 12345, mean_zero: bool = False,
          max_restarts: int = 3, precond_apply=None, precond=None):
    """Solve A x = b to ||b - A x|| <= tol ||b||; returns (x, info dict).

    precond_apply (default: apply) is the operator used inside the
    Chebyshev-Jacobi preconditioner, so a lower-precision action can be
    substituted there while the outer iteration stays in FP64; `precond`
    (r -> z) replaces the Chebyshev-Jacobi preconditioner altogether (the
    multigrid V-cycle of ``oracle.multigrid``)."""
    precond_apply = precond_apply or apply
    dinv = 1.0 / diag
    b = np.asarray(b, dtype=np.float64)
    project = (lambda v: v - v.mean()) if mean_zero else None
    if mean_zero:
        b = project(b)
    lam = lanczos_max(apply, dinv, lanczos_steps, seed)
    lam_hi = safety * lam
    lam_lo = lam_hi / cheb_ratio
    M = precond or (lambda r: chebyshev_jacobi(precond_apply, dinv, r, cheb_degree, lam_hi, lam_lo))
    bnorm = float(np.linalg.norm(b))
    x, its, status = flexible_cg(apply, b, M, tol, max_iter, bnorm=bnorm, project=project)
    total, restarts = its, 0
    while True:
        if mean_zero:
            x = project(x)
        rel = float(np.linalg.norm(b - apply(x)) / bnorm)
        if rel <= tol or status == "breakdown" or restarts >= max_restarts or total >= max_iter:
            break
        restarts += 1
        x, its, status = flexible_cg(apply, b, M, tol, max_iter - total, x0=x, bnorm=bnorm,
                                     project=project)
        total += its
    if rel > tol and status == "ok":
        status = "not_converged"
    return x, {"iterations": total, "rel_residual": rel, "lambda_max": lam,
               "restarts": restarts, "status": status}
