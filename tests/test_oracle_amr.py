"""Pins for the refined-level (Dirichlet) oracle: an exact special case (linear
coarse potential), symmetry and definiteness of the assembled operator, a
direct sparse solve against CG, the brute-force ghost definition, and
invariants of the masked father-cell hierarchy."""
import numpy as np
import pytest

from oracle import amr as A
from oracle import morton as M
from oracle import poisson as P
from workloads import build_amr_input


def _patch_octs(n_oct_dim, lo, hi):
    r = np.arange(lo, hi)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    return g.astype(np.int32)


def test_linear_potential_is_reproduced_exactly():
    # f = 0 and a linear coarse potential: the ghosts are exact (trilinear
    # interpolation reproduces linear functions), L_h of a linear function is 0,
    # so the level solution is that linear function at the fine cell centres.
    nc = 16                       # coarse cells per dim (full periodic parent)
    n = 2 * nc
    octs = _patch_octs(n // 2, 5, 11)     # a cube of octs away from the wrap
    parent = A.CellSet(nc)
    pc = (parent.coords + 0.5) / nc
    lin = lambda x: 0.3 + 1.5 * x[:, 0] - 2.0 * x[:, 1] + 0.75 * x[:, 2]
    phi_parent = lin(pc)
    lev = A.DirichletLevel(n, octs, parent)
    f = np.zeros((len(octs), 8))
    phi = lev.solve(f, phi_parent)
    exact = lin((lev.cells.coords + 0.5) / n).reshape(-1, 8)
    np.testing.assert_allclose(phi, exact, atol=1e-12, rtol=0)
    assert np.max(np.abs(lev.residual(exact, f, phi_parent))) < 1e-9   # L_h(linear) = 0 with exact ghosts


def test_ghost_values_match_pointwise_definition():
    nc = 8
    octs = _patch_octs(nc, 1, 4)
    parent = A.CellSet(nc)
    rng = np.random.default_rng(0)
    pp = rng.standard_normal(len(parent))
    lev = A.DirichletLevel(2 * nc, octs, parent)
    gv = lev.ghost_values(pp)
    dense = pp.reshape(nc, nc, nc)
    for t in range(0, len(gv), 7):
        g = lev.ghost_coords[t]
        Pc = g // 2
        s = np.where(g % 2 == 1, 1, -1)
        val = 0.0
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    w = (0.25 if a else 0.75) * (0.25 if b else 0.75) * (0.25 if c else 0.75)
                    q = (Pc + np.array([a * s[0], b * s[1], c * s[2]])) % nc
                    val += w * dense[q[0], q[1], q[2]]
        assert abs(val - gv[t]) < 1e-14


def test_operator_symmetric_negative_definite_and_solvers_agree():
    a = build_amr_input(base_n=16, n_refined=1, n_clumps=4)
    lv1 = a.levels[1]
    parent = A.CellSet(16)
    lev = A.DirichletLevel(32, lv1.oct_ijk, parent)
    Am = lev.matrix()
    assert abs(Am - Am.T).max() == 0
    w = np.linalg.eigvalsh(Am.toarray())
    assert w.max() < 0                      # -L is SPD: unique solution
    rng = np.random.default_rng(1)
    pp = rng.standard_normal(len(parent))
    f = rng.standard_normal((lv1.n_oct, 8))
    x1 = lev.solve(f, pp)
    b = f.ravel() - lev.ghost_sum(pp) * 32 * 32
    x2 = np.linalg.solve(Am.toarray(), b)
    np.testing.assert_allclose(x1.ravel(), x2, rtol=1e-10, atol=1e-12)
    assert lev.relres(x1, f, pp) < 1e-12


def test_level_neighbours_equal_bruteforce_cells():
    a = build_amr_input(base_n=16, n_refined=1, n_clumps=4)
    octs = a.levels[1].oct_ijk
    lev = A.DirichletLevel(32, octs, A.CellSet(16))
    # oct-level neighbours by brute force, expanded to cells
    onb = M.neighbours_bruteforce(octs, 16)
    for o in range(0, len(octs), 11):
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, c >> 2
            cell = 8 * o + c
            # -x neighbour: inside the oct when cx == 1, else cell cx=1 of the -x oct
            exp = 8 * o + (c - 1) if cx == 1 else (8 * onb[o, 0] + c + 1 if onb[o, 0] >= 0 else -1)
            assert lev.nbr[cell, 0] == exp
            exp = 8 * o + (c + 4) if cz == 0 else (8 * onb[o, 5] + c - 4 if onb[o, 5] >= 0 else -1)
            assert lev.nbr[cell, 5] == exp


def test_full_coverage_level_reduces_to_periodic_operator():
    # a refined level that covers the whole box has no ghosts: its operator is the
    # periodic 7-point Laplacian at that resolution
    n = 8
    octs = _patch_octs(n // 2, 0, n // 2)
    lev = A.DirichletLevel(n, octs, A.CellSet(n // 2))
    assert len(lev.ghost_cell) == 0
    rng = np.random.default_rng(2)
    dense = rng.standard_normal((n, n, n))
    flat = dense[lev.cells.coords[:, 0], lev.cells.coords[:, 1], lev.cells.coords[:, 2]]
    got = lev.apply(flat, np.zeros(len(lev.parent)))
    ref = P.apply_laplacian(dense, 1.0 / n)
    exp = ref[lev.cells.coords[:, 0], lev.cells.coords[:, 1], lev.cells.coords[:, 2]]
    np.testing.assert_allclose(got, exp, rtol=1e-13, atol=1e-10)


def test_masked_hierarchy_invariants():
    a = build_amr_input(base_n=16, n_refined=2, n_clumps=4)
    octs = a.levels[1].oct_ijk
    levels, fathers = A.build_hierarchy(32, octs, max_coarse_cells=64)
    assert len(levels) >= 2
    for lv, fa, nxt in zip(levels[:-1], fathers, levels[1:]):
        # one father per fine oct, all distinct, all active
        assert len(np.unique(fa)) == len(lv.oct_ijk)
        assert nxt.active.reshape(-1)[fa].all()
        assert nxt.n_active == len(lv.oct_ijk)
        # restriction: the mean of the 8 children
        r = np.random.default_rng(3).standard_normal((len(lv.oct_ijk), 8))
        rc = A.restrict_fathers(r, fa, len(nxt.oct_ijk))
        np.testing.assert_allclose(rc.reshape(-1)[fa], r.mean(axis=1), rtol=1e-15)
        # prolongation of a constant on fully-surrounded fine cells is that constant
        ec = np.where(nxt.active, 1.0, 0.0).reshape(-1, 8)
        pf = A.prolong_masked(lv, nxt, fa, ec)
        inner = (lv.nbr >= 0).all(axis=1)
        assert np.all(pf.reshape(-1) <= 1.0 + 1e-15)
        assert np.any(np.isclose(pf.reshape(-1)[inner], 1.0))


def test_nesting_violation_is_detected():
    nc = 8
    octs = np.array([[0, 0, 0]], dtype=np.int32)
    parent = A.CellSet(nc, np.array([[0, 0, 0]]))     # parent has a single oct: no full stencil
    with pytest.raises(A.NestingError):
        A.DirichletLevel(2 * nc, octs, parent)


def test_masked_level_operator_is_mirror_boundary_and_spd():
    # the coarse error operator of a masked level: an active cell whose neighbour
    # is inactive/absent sees -e_cell there (zero on the shared face); the
    # assembled operator is symmetric negative definite
    a = build_amr_input(base_n=16, n_refined=1, n_clumps=4)
    levels, fathers = A.build_hierarchy(32, a.levels[1].oct_ijk, max_coarse_cells=64)
    lv = levels[1]
    act = np.nonzero(lv.active)[0]
    N = len(lv.active)
    Mx = np.zeros((len(act), len(act)))
    for k, i in enumerate(act):
        e = np.zeros(N)
        e[i] = 1.0
        Mx[:, k] = lv.apply(e)[act]
    assert np.allclose(Mx, Mx.T)
    assert np.linalg.eigvalsh(Mx).max() < 0
    # pointwise: a cell with one active neighbour j and 5 missing ones
    e = np.random.default_rng(4).standard_normal(N) * lv.active
    out = lv.apply(e)
    for i in act[:50]:
        nb = [j for j in lv.nbr[i] if j >= 0]
        exp = (sum(e[j] for j in nb) - (6 + (6 - len(nb))) * e[i]) / lv.h ** 2
        assert abs(out[i] - exp) < 1e-9 * max(1.0, abs(exp))
