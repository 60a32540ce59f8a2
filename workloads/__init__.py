"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This module only *draws* inputs: mesh vertices, the random modes that define a
viscosity field or a background velocity, right-hand sides and request
streams.  It holds none of the discretisation's arithmetic (no basis, no
quadrature, no geometry factors, no viscosity-law evaluation at quadrature
points); both the oracle and the HIP library evaluate the fields defined here
on their own.

The workloads stand in for the paper's cavity and backward-facing-step runs
(Sec. 6.2 and 6.3): hexahedral meshes of a cube, polynomial degrees 2-5,
viscosity contrasts 1 to 1e4 and about 1e6-1e7 unknowns.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "box_vertices",
    "logfield_law",
    "carreau_law",
    "sine_law",
    "const_law",
    "uniform_vector",
    "CONFIGS",
    "config",
    "serving_requests",
]

# Side order used for boundary conditions everywhere: -x, +x, -y, +y, -z, +z.
ALL_DIRICHLET = ("D",) * 6
ALL_NEUMANN = ("N",) * 6


def box_vertices(nx: int, ny: int, nz: int, perturb: float = 0.0) -> np.ndarray | None:
    """Vertices of a structured nx*ny*nz hex mesh of the unit cube.

    Returns an array of shape ((nz+1)*(ny+1)*(nx+1), 3), vertex
    (ix, iy, iz) at row (iz*(ny+1) + iy)*(nx+1) + ix.  With perturb != 0 every
    coordinate of every vertex is moved by perturb*h*sin(2 pi x)sin(2 pi y)
    sin(2 pi z) of the unperturbed position, h = 1/max(nx, ny, nz); boundary
    vertices stay on the boundary because the product vanishes there.
    Returns None for the unperturbed (affine) box, which the library and the
    oracle both accept as "unit box with straight cells".
    """
    if perturb == 0.0:
        return None
    x = np.linspace(0.0, 1.0, nx + 1)
    y = np.linspace(0.0, 1.0, ny + 1)
    z = np.linspace(0.0, 1.0, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    h = 1.0 / max(nx, ny, nz)
    s = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(2 * np.pi * Z)
    # the product vanishes on the boundary; make that exact (sin(2 pi) != 0 in fp64)
    on_bdry = np.zeros_like(s, dtype=bool)
    on_bdry[0], on_bdry[-1] = True, True
    on_bdry[:, 0], on_bdry[:, -1] = True, True
    on_bdry[:, :, 0], on_bdry[:, :, -1] = True, True
    d = np.where(on_bdry, 0.0, perturb * h * s)
    V = np.stack([X + d, Y + d, Z + d], axis=-1)
    return np.ascontiguousarray(V.reshape(-1, 3))


def _wave_vectors(rng: np.random.Generator, n_modes: int, kmax: int) -> np.ndarray:
    """n_modes integer wave vectors drawn uniformly from {-kmax..kmax}^3 minus 0."""
    out = []
    while len(out) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            out.append(k)
    return np.array(out, dtype=np.int64)


def const_law(mu: float = 1.0) -> dict:
    return {"kind": "const", "mu": float(mu)}


def sine_law(mu: float = 1.0, amp: float = 0.5) -> dict:
    """mu(x) = mu * (1 + amp sin(2 pi x) sin(2 pi y) sin(2 pi z))."""
    return {"kind": "sine", "mu": float(mu), "amp": float(amp)}


def logfield_law(seed: int, contrast: float, n_modes: int = 8, kmax: int = 2) -> dict:
    """Smooth random log-viscosity field mu(x) = contrast ** s(x).

    s(x) = clip((r(x) - rmin) / (rmax - rmin), 0, 1) with
    r(x) = sum_m a_m cos(2 pi k_m . x + phi_m); the modes are drawn here and
    rmin / rmax are the extremes of r over a fixed 65^3 lattice of the unit
    cube, so the field does not depend on the mesh it is sampled on.
    """
    rng = np.random.default_rng(seed)
    k = _wave_vectors(rng, n_modes, kmax)
    a = rng.uniform(0.0, 1.0, size=n_modes)
    phi = rng.uniform(0.0, 2 * np.pi, size=n_modes)
    t = np.linspace(0.0, 1.0, 65)
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    r = np.cos(2 * np.pi * (P @ k.T.astype(np.float64)) + phi) @ a
    return {
        "kind": "logfield",
        "contrast": float(contrast),
        "k": k,
        "a": a,
        "phi": phi,
        "rmin": float(r.min()),
        "rmax": float(r.max()),
    }


def carreau_law(seed: int, mu0: float = 1.0, mu_inf: float = 1e-4, lam: float = 1.0,
                n_exp: float = 0.5, kappa: float = 1.0, a_exp: float = 2.0,
                n_modes: int = 8, kmax: int = 2) -> dict:
    """Generalised-Newtonian viscosity of a prescribed background velocity.

    mu = mu_inf + (mu0 - mu_inf) [kappa + (lam * gdot)^a]^((b-1)/a), b = n_exp,
    with gdot the shear rate of w(x) = sum_m v_m cos(2 pi k_m . x + phi_m),
    v_m = c_m x k_m, c_m ~ N(0, I): each mode is orthogonal to its wave vector,
    so w is divergence-free.  The cross product only builds the input field.
    """
    rng = np.random.default_rng(seed)
    k = _wave_vectors(rng, n_modes, kmax)
    c = rng.normal(0.0, 1.0, size=(n_modes, 3))
    phi = rng.uniform(0.0, 2 * np.pi, size=n_modes)
    v = np.cross(c, k.astype(np.float64))
    return {
        "kind": "carreau",
        "mu0": float(mu0), "mu_inf": float(mu_inf), "lam": float(lam),
        "n_exp": float(n_exp), "kappa": float(kappa), "a_exp": float(a_exp),
        "k": k, "v": v, "phi": phi,
    }


def penalty_parameters(nx: int, ny: int, nz: int, degree: int, vertices, seed: int,
                       cfl: float = 0.4, zeta: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Per-cell divergence and continuity penalty factors of the penalty step.

    The paper takes them from Fehn et al. (2018); the reading used here is
    tau_div = zeta |u_e| h dt / (k+1) and tau_cont = zeta |u_e| dt, with u_e
    the seeded divergence-free velocity of ``carreau_law(seed)`` at the cell
    centre (mean of the 8 vertices), h = 1/N per direction (geometric mean)
    and dt = cfl * h / max_e |u_e|.
    """
    law = carreau_law(seed)
    if vertices is None:
        Z, Y, X = np.meshgrid(np.linspace(0, 1, nz + 1), np.linspace(0, 1, ny + 1), np.linspace(0, 1, nx + 1),
                              indexing="ij")
        vertices = np.stack([X, Y, Z], axis=-1)
    V = np.asarray(vertices, dtype=np.float64).reshape(nz + 1, ny + 1, nx + 1, 3)
    centre = 0.125 * sum(V[c:nz + c, b:ny + b, a:nx + a] for a in (0, 1) for b in (0, 1) for c in (0, 1))
    x = centre.reshape(-1, 3)
    arg = 2 * np.pi * x @ law["k"].T.astype(np.float64) + law["phi"]
    w = np.cos(arg) @ law["v"]
    speed = np.linalg.norm(w, axis=1)
    h = (1.0 / nx / ny / nz) ** (1.0 / 3.0)
    dt = cfl * h / speed.max()
    return zeta * speed * h * dt / (degree + 1), zeta * speed * dt


def uniform_vector(seed: int, n: int) -> np.ndarray:
    """n values ~ U(-1, 1) from numpy's default generator."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def _cfg(name, n, degree, op, law, alpha, bc, perturb, **extra):
    d = {
        "name": name, "nx": n, "ny": n, "nz": n, "degree": degree, "op": op,
        "law": law, "alpha": float(alpha), "penalty": 1.0, "bc": tuple(bc),
        "perturb": float(perturb),
    }
    d.update(extra)
    return d


def config(name: str, n: int | None = None) -> dict:
    """The five workloads, optionally on a smaller n^3 mesh of the same kind.

    c1  4^3 affine, k=2, viscous, sine viscosity, alpha/dt = 10, Dirichlet.
    c2  32^3 perturbed (0.1 h), k=3, viscous, mu = 10^(3 s(x)), seed 2.
    c3  24^3 perturbed, k=4, viscous, Carreau of a seeded velocity, seed 3.
    c4p 20^3 affine, k=5, Poisson, all Neumann (singular, mean-zero data).
    c4v 20^3 affine, k=5, viscous, sine viscosity, Dirichlet.
    c6  16^3 perturbed, k=3, penalty step (mass + divergence and continuity
        penalties, per-cell factors from ``penalty_parameters``, seed 6).
    c7  the nonlinear viscous step: c3's mesh, degree and Carreau parameters
        with the viscosity taken from the velocity (Picard iteration), zero
        initial velocity, right-hand side ``b_scale`` U(-1, 1) with seed 7,
        b_scale = 100 alpha / (cells (k+1)^3).
    c8  one dual-splitting time step (BDF1, dt = 1e-3) of a lid-driven box
        (``lid_data``: the +z wall moves with (1, 0, 0), the others are
        no-slip): c3's mesh, velocity degree 4 (pressure 3) and Carreau
        parameters, the old velocity and body force of ``split_inputs``.
    """
    if name == "c1":
        return _cfg("c1", n or 4, 2, "viscous", sine_law(1.0, 0.5), 10.0, ALL_DIRICHLET, 0.0,
                    x_seed=1, tol=1e-10)
    if name == "c2":
        return _cfg("c2", n or 32, 3, "viscous", logfield_law(2, 1e3), 10.0, ALL_DIRICHLET, 0.1,
                    x_seed=2)
    if name == "c3":
        return _cfg("c3", n or 24, 4, "viscous", carreau_law(3), 10.0, ALL_DIRICHLET, 0.1,
                    x_seed=3, tol=1e-8)
    if name == "c4p":
        return _cfg("c4p", n or 20, 5, "poisson", const_law(1.0), 0.0, ALL_NEUMANN, 0.0,
                    x_seed=4, tol=1e-8)
    if name == "c4v":
        return _cfg("c4v", n or 20, 5, "viscous", sine_law(1.0, 0.5), 10.0, ALL_DIRICHLET, 0.0,
                    x_seed=4, tol=1e-8)
    if name == "c6":
        m = n or 16
        td, tc = penalty_parameters(m, m, m, 3, box_vertices(m, m, m, 0.1), 6)
        return _cfg("c6", m, 3, "penalty", None, 1.0, ALL_DIRICHLET, 0.1, x_seed=6, tol=1e-8,
                    tau_div=td, tau_cont=tc)
    if name == "c7":
        m = n or 24
        return _cfg("c7", m, 4, "viscous", carreau_law(3), 10.0, ALL_DIRICHLET, 0.1, x_seed=7, tol=1e-8,
                    b_scale=100.0 * 10.0 / (m ** 3 * 125), picard=True)
    if name == "c8":
        m = n or 24
        dt = 1e-3
        return _cfg("c8", m, 4, "viscous", carreau_law(3), 1.0 / dt, ALL_DIRICHLET, 0.1, x_seed=8, tol=1e-8,
                    dt=dt, split=True)
    raise KeyError(name)


def lid_data(cfg: dict) -> np.ndarray:
    """Wall data of a lid-driven box: g_u = (1, 0, 0) on the +z wall, 0 on
    the others, at every wall face point (the wall layout of the splitting
    step: sides -x, +x, -y, +y, -z, +z, (k+1)^2 points, 3 components)."""
    nx, ny, nz, n = cfg["nx"], cfg["ny"], cfg["nz"], cfg["degree"] + 1
    sizes = [ny * nz, ny * nz, nx * nz, nx * nz, nx * ny, nx * ny]
    g = np.zeros((sum(sizes), n * n, 3))
    top = sum(sizes[:5])
    g[top:top + sizes[5], :, 0] = 1.0
    return g.reshape(-1)


def node_positions(nx: int, ny: int, nz: int, degree: int, vertices=None) -> np.ndarray:
    """Physical positions (cells, (k+1)^3, 3) of the Gauss-point nodes of
    every cell (first reference direction fastest) under the trilinear map
    of its 8 vertices."""
    n = degree + 1
    g = (np.polynomial.legendre.leggauss(n)[0] + 1.0) / 2.0
    if vertices is None:
        Z, Y, X = np.meshgrid(np.linspace(0, 1, nz + 1), np.linspace(0, 1, ny + 1), np.linspace(0, 1, nx + 1),
                              indexing="ij")
        vertices = np.stack([X, Y, Z], axis=-1)
    V = np.asarray(vertices, dtype=np.float64).reshape(nz + 1, ny + 1, nx + 1, 3)
    L = np.stack([1.0 - g, g])                                  # (2, n): linear shape functions at the points
    out = np.zeros((nz, ny, nx, n, n, n, 3))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                Xc = V[c:nz + c, b:ny + b, a:nx + a]             # (nz, ny, nx, 3)
                w = L[c][:, None, None] * L[b][None, :, None] * L[a][None, None, :]   # (q3, q2, q1)
                out += Xc[:, :, :, None, None, None, :] * w[None, None, None, :, :, :, None]
    return out.reshape(nx * ny * nz, n ** 3, 3)


def split_inputs(cfg: dict, vertices=None) -> tuple[np.ndarray, np.ndarray]:
    """Old velocity and body force of the dual-splitting workload, nodal
    vectors (cells, 3, (k+1)^3): u^n = 6.4 x(1-x) y(1-y) z(1-z) w(x) with w
    the seeded smooth background velocity of ``carreau_law(x_seed)`` (zero on
    the walls), b = (sin 2 pi y, sin 2 pi z, sin 2 pi x)."""
    x = node_positions(cfg["nx"], cfg["ny"], cfg["nz"], cfg["degree"], vertices)
    law = carreau_law(cfg["x_seed"])
    arg = 2 * np.pi * x @ law["k"].T.astype(np.float64) + law["phi"]
    w = np.cos(arg) @ law["v"]
    bub = 6.4 * np.prod(x * (1.0 - x), axis=-1)
    u = bub[..., None] * w
    b = np.sin(2 * np.pi * x[..., [1, 2, 0]])
    return np.transpose(u, (0, 2, 1)).reshape(-1).copy(), np.transpose(b, (0, 2, 1)).reshape(-1).copy()


CONFIGS = ("c1", "c2", "c3", "c4p", "c4v")


def ndofs(cfg: dict) -> int:
    n = cfg["degree"] + 1
    comps = 1 if cfg["op"] == "poisson" else 3
    return cfg["nx"] * cfg["ny"] * cfg["nz"] * comps * n ** 3


def serving_requests(seed: int = 5, count: int = 256, rate: float = 20.0,
                     nmin: int = 4, nmax: int = 24) -> list[dict]:
    """Viscous-step solve requests with Poisson arrivals.

    Edge count N ~ U{nmin..nmax}, degree ~ U{2,3,4,5}, viscosity contrast
    ~ U{1, 1e2, 1e4} (mu = contrast^s(x), per-request field seed),
    alpha/dt ~ U[1, 100], all-Dirichlet, affine cube, right-hand side
    ~ U(-1, 1) with a per-request seed; arrival gaps ~ Exp(1/rate).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.integers(nmin, nmax + 1))
        k = int(rng.integers(2, 6))
        contrast = float([1.0, 1e2, 1e4][rng.integers(0, 3)])
        alpha = float(rng.uniform(1.0, 100.0))
        fseed = int(rng.integers(0, 2**31 - 1))
        bseed = int(rng.integers(0, 2**31 - 1))
        law = const_law(1.0) if contrast == 1.0 else logfield_law(fseed, contrast)
        out.append({
            "id": i, "arrival": t,
            "cfg": _cfg(f"req{i}", n, k, "viscous", law, alpha, ALL_DIRICHLET, 0.0,
                        x_seed=bseed, tol=1e-8),
        })
    return out
