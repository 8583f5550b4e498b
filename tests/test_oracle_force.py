"""Pins for the force oracle g = -grad(phi) (central differences, the reading
taken for the gravity-force step that follows the solve): the closed form of
the central difference of a sinusoid on the periodic level, exactness on a
linear potential through the refined level's trilinear ghosts, and agreement
of a refined level that covers the whole box with the periodic level."""
import numpy as np

from oracle import amr as A
from oracle import poisson as P


def test_periodic_sinusoid_closed_form():
    # phi = sin(2 pi x) + 2 cos(4 pi y) + 3 sin(6 pi z) at cell centres; the
    # central difference of sin(a t) is cos(a t) sin(a h) / h exactly, of
    # cos(a t) it is -sin(a t) sin(a h) / h.  Different wave numbers per axis
    # catch a transposed component.
    n = 16
    h = 1.0 / n
    x = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    a, b, c = 2 * np.pi, 4 * np.pi, 6 * np.pi
    phi = np.sin(a * X) + 2 * np.cos(b * Y) + 3 * np.sin(c * Z)
    g = P.force(phi, h)
    np.testing.assert_allclose(g[0], -np.cos(a * X) * np.sin(a * h) / h, atol=1e-12, rtol=0)
    np.testing.assert_allclose(g[1], 2 * np.sin(b * Y) * np.sin(b * h) / h, atol=1e-12, rtol=0)
    np.testing.assert_allclose(g[2], -3 * np.cos(c * Z) * np.sin(c * h) / h, atol=1e-12, rtol=0)


def test_periodic_force_of_constant_is_zero_and_sums_vanish():
    n = 8
    rng = np.random.default_rng(4)
    assert np.all(P.force(np.full((n, n, n), 3.25), 1.0 / n) == 0.0)
    g = P.force(rng.standard_normal((n, n, n)), 1.0 / n)
    # a central difference telescopes to zero over every periodic line along its axis
    for d in range(3):
        assert np.max(np.abs(g[d].sum(axis=d))) < 1e-12


def _patch_octs(lo, hi):
    r = np.arange(lo, hi)
    return np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)


def test_refined_level_linear_potential_exact():
    # a linear potential on both levels: the trilinear ghosts reproduce it, so
    # every cell, including those whose neighbours are ghosts, gets -grad.
    nc = 16
    n = 2 * nc
    parent = A.CellSet(nc)
    lin = lambda p: 0.3 + 1.5 * p[:, 0] - 2.0 * p[:, 1] + 0.75 * p[:, 2]
    octs = _patch_octs(5, 11)
    lev = A.DirichletLevel(n, octs, parent)
    assert len(lev.ghost_cell) > 0
    phi_parent = lin((parent.coords + 0.5) / nc)
    phi = lin((lev.cells.coords + 0.5) / n).reshape(-1, 8)
    g = lev.force(phi, phi_parent)
    for d, want in enumerate((-1.5, 2.0, -0.75)):
        np.testing.assert_allclose(g[d], want, atol=1e-11, rtol=0)


def test_refined_level_ghost_side_matters():
    # Changing the parent potential changes exactly the cells next to a ghost
    # face, and only the component across that face.
    nc = 8
    parent = A.CellSet(nc)
    octs = _patch_octs(1, 3)
    lev = A.DirichletLevel(2 * nc, octs, parent)
    rng = np.random.default_rng(1)
    phi = rng.standard_normal((len(octs), 8))
    pp = rng.standard_normal(len(parent))
    g0 = lev.force(phi, pp).reshape(3, -1)
    g1 = lev.force(phi, pp + 1.0).reshape(3, -1)       # every ghost value rises by 1 (weights sum to 1)
    for d in range(3):
        lo = lev.nbr[:, 2 * d] < 0
        hi = lev.nbr[:, 2 * d + 1] < 0
        want = np.zeros(lev.n_cells)
        want[hi] -= 1.0 / (2 * lev.h)
        want[lo] += 1.0 / (2 * lev.h)
        np.testing.assert_allclose(g1[d] - g0[d], want, atol=1e-9, rtol=0)


def test_full_cover_refined_level_equals_periodic():
    # a refined level that holds every oct of its box has no ghosts; with the
    # periodic wrap its force is the periodic level's force.
    n = 8
    octs = _patch_octs(0, n // 2)
    lev = A.DirichletLevel(n, octs, A.CellSet(n // 2))
    assert len(lev.ghost_cell) == 0
    rng = np.random.default_rng(2)
    dense = rng.standard_normal((n, n, n))
    cells = lev.cells.coords
    phi = dense[cells[:, 0], cells[:, 1], cells[:, 2]].reshape(-1, 8)
    g = lev.force(phi, np.zeros(len(A.CellSet(n // 2))))
    ref = P.force(dense, 1.0 / n)
    for d in range(3):
        np.testing.assert_allclose(g[d].ravel(), ref[d][cells[:, 0], cells[:, 1], cells[:, 2]], atol=1e-12, rtol=0)
