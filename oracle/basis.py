"""One-dimensional Gauss rule and Lagrange basis on [0, 1].

Sec. 4 builds Q_k from tensor products of 1D shape functions and Sec. 4.1
(paragraph on viscosity storage) uses as many integration points per direction
as support points.  The reading taken here: nodes and quadrature points are
both the k+1 Gauss-Legendre points of [0, 1].
"""
from __future__ import annotations

import numpy as np


def gauss_points(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n-point Gauss-Legendre rule mapped to [0, 1] (points ascending, weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0


def lagrange_values(nodes: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """V[p, j] = l_j(pts[p]), l_j(x) = prod_{m != j} (x - x_m) / (x_j - x_m)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.atleast_1d(np.asarray(pts, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(pts), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                V[:, j] *= (pts - nodes[m]) / (nodes[j] - nodes[m])
    return V


def lagrange_derivatives(nodes: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """D[p, j] = l_j'(pts[p]) by the product rule:
    l_j'(x) = sum_{m != j} 1/(x_j - x_m) prod_{l != j, m} (x - x_l)/(x_j - x_l)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.atleast_1d(np.asarray(pts, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(pts), n))
    for j in range(n):
        for m in range(n):
            if m == j:
                continue
            term = np.full(len(pts), 1.0 / (nodes[j] - nodes[m]))
            for l in range(n):
                if l != j and l != m:
                    term *= (pts - nodes[l]) / (nodes[j] - nodes[l])
            D[:, j] += term
    return D


def tensor_tables(n: int, pts3: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Values and reference gradients of the n^3 tensor-product basis functions
    at reference points pts3 (P x 3).

    Basis function index i = i3*n^2 + i2*n + i1 (first direction fastest),
    phi_i(xi) = l_i1(xi1) l_i2(xi2) l_i3(xi3).
    Returns V (P, n^3) and G (P, n^3, 3) with G[p, i, d] = d phi_i / d xi_d.
    """
    nodes, _ = gauss_points(n)
    v = [lagrange_values(nodes, pts3[:, d]) for d in range(3)]
    g = [lagrange_derivatives(nodes, pts3[:, d]) for d in range(3)]
    P = pts3.shape[0]
    # (P, i3, i2, i1)
    V = v[2][:, :, None, None] * v[1][:, None, :, None] * v[0][:, None, None, :]
    G = np.empty((P, n, n, n, 3))
    G[..., 0] = v[2][:, :, None, None] * v[1][:, None, :, None] * g[0][:, None, None, :]
    G[..., 1] = v[2][:, :, None, None] * g[1][:, None, :, None] * v[0][:, None, None, :]
    G[..., 2] = g[2][:, :, None, None] * v[1][:, None, :, None] * v[0][:, None, None, :]
    return V.reshape(P, n ** 3), G.reshape(P, n ** 3, 3)


def cell_points(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Tensor Gauss points of the reference cell, index q = q3*n^2 + q2*n + q1,
    and their weights."""
    g, w = gauss_points(n)
    Q3, Q2, Q1 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    q1, q2, q3 = Q1.ravel(), Q2.ravel(), Q3.ravel()
    pts = np.stack([g[q1], g[q2], g[q3]], axis=1)
    return pts, w[q1] * w[q2] * w[q3]


def face_points(n: int, d: int, side: int) -> tuple[np.ndarray, np.ndarray]:
    """Tensor Gauss points on the reference face xi_d = side (0 or 1).

    The face's two tangential directions (t1 < t2) are the other two; face
    point index f = b*n + a with xi_t1 = g[a], xi_t2 = g[b].
    """
    g, w = gauss_points(n)
    t1, t2 = [t for t in range(3) if t != d]
    B, A = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    a, b = A.ravel(), B.ravel()
    pts = np.zeros((n * n, 3))
    pts[:, t1] = g[a]
    pts[:, t2] = g[b]
    pts[:, d] = float(side)
    return pts, w[a] * w[b]
