"""Structured hexahedral mesh of a box with trilinear cells.

Sec. 4 maps each reference cell to a hexahedron by chi_e.  The meshes used
here are structured boxes whose cells are trilinear in their 8 vertices
(a straight-sided cell is reproduced exactly by the degree-k mapping the
paper uses).  Cell e = (ez*ny + ey)*nx + ex; reference coordinate xi_1 runs
along x, xi_2 along y, xi_3 along z.
"""
from __future__ import annotations

import numpy as np


class Mesh:
    def __init__(self, nx: int, ny: int, nz: int, vertices: np.ndarray | None = None,
                 bc=("D",) * 6):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        if vertices is None:
            x = np.linspace(0.0, 1.0, nx + 1)
            y = np.linspace(0.0, 1.0, ny + 1)
            z = np.linspace(0.0, 1.0, nz + 1)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            vertices = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(nz + 1, ny + 1, nx + 1, 3)
        self.bc = tuple(bc)
        assert len(self.bc) == 6 and all(b in ("D", "N") for b in self.bc)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def cell_ijk(self, cells: np.ndarray):
        cells = np.asarray(cells)
        ex = cells % self.nx
        ey = (cells // self.nx) % self.ny
        ez = cells // (self.nx * self.ny)
        return ex, ey, ez

    def corners(self, cells: np.ndarray) -> np.ndarray:
        """X[e, a, b, c, :] = vertex (ex+a, ey+b, ez+c) of cell e."""
        ex, ey, ez = self.cell_ijk(cells)
        X = np.empty((len(ex), 2, 2, 2, 3))
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    X[:, a, b, c] = self.vertices[ez + c, ey + b, ex + a]
        return X

    @staticmethod
    def _shape(pts):
        """Trilinear shape functions N_abc(xi) = N_a(xi1) N_b(xi2) N_c(xi3),
        N_0(t) = 1 - t, N_1(t) = t, and their reference gradients."""
        P = pts.shape[0]
        Nv = [np.stack([1 - pts[:, d], pts[:, d]], axis=1) for d in range(3)]  # (P, 2)
        dN = np.array([-1.0, 1.0])
        N = np.einsum("pa,pb,pc->pabc", Nv[0], Nv[1], Nv[2])
        G = np.empty((P, 2, 2, 2, 3))
        G[..., 0] = np.einsum("a,pb,pc->pabc", dN, Nv[1], Nv[2])
        G[..., 1] = np.einsum("pa,b,pc->pabc", Nv[0], dN, Nv[2])
        G[..., 2] = np.einsum("pa,pb,c->pabc", Nv[0], Nv[1], dN)
        return N, G

    def map(self, cells, pts) -> np.ndarray:
        """Physical points chi_e(xi) for each cell and reference point: (E, P, 3)."""
        X = self.corners(cells)
        N, _ = self._shape(pts)
        return np.einsum("pabc,eabci->epi", N, X)

    def jacobian(self, cells, pts) -> np.ndarray:
        """J[e, p, i, d] = d x_i / d xi_d at the reference points."""
        X = self.corners(cells)
        _, G = self._shape(pts)
        return np.einsum("pabcd,eabci->epid", G, X)

    def interior_faces(self, d: int) -> tuple[np.ndarray, np.ndarray]:
        """Pairs (e_minus, e_plus) of cells sharing a face normal to direction d,
        e_plus = e_minus + unit step in direction d."""
        nx, ny, nz = self.nx, self.ny, self.nz
        ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
        lim = (nx, ny, nz)[d]
        pos = (ex, ey, ez)[d]
        keep = pos < lim - 1
        ex, ey, ez = ex[keep], ey[keep], ez[keep]
        em = (ez * ny + ey) * nx + ex
        step = (1, nx, nx * ny)[d]
        order = np.argsort(em)
        em = em[order]
        return em, em + step

    def boundary_cells(self, d: int, side: int) -> np.ndarray:
        """Cells touching the boundary plane xi_d = side of the box."""
        nx, ny, nz = self.nx, self.ny, self.nz
        ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
        lim = (nx, ny, nz)[d]
        pos = (ex, ey, ez)[d]
        keep = pos == (lim - 1 if side == 1 else 0)
        return np.sort((ez[keep] * ny + ey[keep]) * nx + ex[keep])

    @property
    def nfaces(self) -> int:
        nx, ny, nz = self.nx, self.ny, self.nz
        return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)

    def face_index(self, d: int, cells, side: int) -> np.ndarray:
        """Number of the face xi_d = side of each cell: x-faces first,
        (ez*ny + ey)*(nx+1) + fx, then y-faces (ez*(ny+1) + fy)*nx + ex,
        then z-faces (fz*ny + ey)*nx + ex, with f_d = e_d + side."""
        nx, ny, nz = self.nx, self.ny, self.nz
        ex, ey, ez = self.cell_ijk(cells)
        if d == 0:
            return (ez * ny + ey) * (nx + 1) + ex + side
        if d == 1:
            return (nx + 1) * ny * nz + (ez * (ny + 1) + ey + side) * nx + ex
        return (nx + 1) * ny * nz + nx * (ny + 1) * nz + ((ez + side) * ny + ey) * nx + ex
