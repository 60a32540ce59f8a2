"""Pins of the oracle's penalty-step operator (Sec. 4.3, "Consistent
Stabilization", eq. penalty_step): mass + divergence penalty per cell +
continuity penalty on the normal jump, with the face factor the mean of the
two cells' values (reading) and the oriented jump u - g on Dirichlet faces.
Checked against closed-form energies and structural properties."""
import numpy as np
import pytest

import workloads as W
from oracle.forms import Problem, apply, assemble, diagonal, interpolate
from oracle.mesh import Mesh


def pen(mesh, deg, td, tc, alpha=1.0):
    return Problem(mesh, deg, "penalty", alpha, 1.0, None, np.asarray(td, float), np.asarray(tc, float))


def rand_tau(ncell, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 2.0, ncell), rng.uniform(0.5, 2.0, ncell)


def test_penalty_operator_is_symmetric_positive_definite():
    m = Mesh(2, 2, 1, W.box_vertices(2, 2, 1, 0.15), ("D", "N", "D", "D", "N", "D"))
    pb = pen(m, 2, *rand_tau(4, 1))
    A = assemble(pb).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


def test_penalty_modes_and_diagonal_agree():
    m = Mesh(3, 2, 2, W.box_vertices(3, 2, 2, 0.1))
    pb = pen(m, 3, *rand_tau(12, 2))
    A = assemble(pb)
    x = W.uniform_vector(3, pb.ndof)
    np.testing.assert_allclose(apply(pb, x), A @ x, rtol=0, atol=1e-12 * np.abs(A @ x).max())
    np.testing.assert_allclose(diagonal(pb), A.diagonal(), rtol=1e-13, atol=0)


def test_penalty_with_zero_factors_is_the_mass_matrix():
    m = Mesh(2, 1, 2, W.box_vertices(2, 1, 2, 0.1))
    pb = pen(m, 2, np.zeros(4), np.zeros(4), alpha=1.7)
    A = assemble(pb).toarray()
    assert np.abs(A - np.diag(np.diag(A))).max() == 0.0
    # collocated mass: the diagonal sums to alpha * volume per component (volume 1)
    assert abs(np.diag(A).sum() - 3 * 1.7) <= 1e-13


def test_divergence_free_continuous_field_feels_only_the_mass():
    """u = curl(0, 0, x^2 y) = (x^2, -2xy, 0) is divergence-free and
    continuous: with Neumann faces A u = alpha M u exactly (k >= 2)."""
    m = Mesh(2, 2, 2, None, ("N",) * 6)
    td, tc = rand_tau(8, 4)
    pb = pen(m, 2, td, tc, alpha=1.0)
    u = interpolate(pb, lambda X: np.stack([X[:, 0] ** 2, -2 * X[:, 0] * X[:, 1], 0 * X[:, 0]], axis=1))
    M = assemble(pen(m, 2, np.zeros(8), np.zeros(8))).diagonal()
    np.testing.assert_allclose(apply(pb, u), M * u, rtol=0, atol=1e-12)


def test_divergence_penalty_energy_of_a_linear_field():
    """u = (x, 0, 0): div u = 1, no jumps: u.A u = sum_e tau_div^e |e| + alpha/3."""
    m = Mesh(2, 3, 2, None, ("N",) * 6)
    td, tc = rand_tau(12, 5)
    pb = pen(m, 1, td, tc, alpha=0.6)
    u = interpolate(pb, lambda X: np.stack([X[:, 0], 0 * X[:, 0], 0 * X[:, 0]], axis=1))
    assert abs(u @ apply(pb, u) - (td.sum() / 12 + 0.6 / 3)) <= 1e-13


@pytest.mark.parametrize("cell", [13, 0])
def test_continuity_penalty_energy_of_a_cell_indicator(cell):
    """u = e_1 on one cell, 0 elsewhere (3^3 unit cube, h = 1/3): the normal jump
    is 1 on the cell's two x-faces only, so u.A u = alpha h^3 + h^2 sum over
    those faces of tau_F, with tau_F the mean of the two cells' factors inside
    and the cell's own factor on a Dirichlet face (no mirror doubling)."""
    m = Mesh(3, 3, 3, None, ("D",) * 6)
    td, tc = rand_tau(27, 6)
    pb = pen(m, 2, td, tc, alpha=1.0)
    u = np.zeros(pb.ndof)
    nloc = pb.nloc
    u[cell * nloc:cell * nloc + pb.n ** 3] = 1.0              # component 0 on `cell`
    ex = cell % 3
    h = 1.0 / 3
    faces = 0.0
    for nb_x in (ex - 1, ex + 1):
        faces += tc[cell] if nb_x < 0 or nb_x > 2 else 0.5 * (tc[cell] + tc[cell - ex + nb_x])
    assert abs(u @ apply(pb, u) - (h ** 3 + h ** 2 * faces)) <= 1e-13
