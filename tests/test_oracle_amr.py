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
    levels, fathers = A.build_hierarchy(32, octs, max_coarse_octs=8)
    assert len(levels) >= 3
    for lv, fa, nxt in zip(levels[:-1], fathers, levels[1:]):
        # one father per fine oct, all distinct; father masks are the children's means
        assert len(np.unique(fa)) == len(lv.oct_ijk)
        np.testing.assert_allclose(nxt.lsm[fa], lv.lsm.reshape(-1, 8).mean(axis=1))
        others = np.setdiff1d(np.arange(len(nxt.lsm)), fa)
        assert np.all(nxt.lsm[others] == -1.0)
        # restriction: the mean of the 8 children
        r = np.random.default_rng(3).standard_normal((len(lv.oct_ijk), 8))
        rc = A.restrict_fathers(r, fa, len(nxt.oct_ijk))
        np.testing.assert_allclose(rc.reshape(-1)[fa], r.mean(axis=1), rtol=1e-15)
    # level 1: masks are exactly +-1 and the fathers are exactly the active cells
    l1 = levels[1]
    assert set(np.unique(l1.lsm)) <= {-1.0, 1.0}
    assert l1.n_active == len(octs)
    # prolongation of a constant onto fine cells whose coarse stencil is all active is exact
    ec = np.where(l1.active, 1.0, 0.0).reshape(-1, 8)
    pf = A.prolong_masked(levels[0], l1, fathers[0], ec).reshape(-1)
    assert np.all(pf <= 1.0 + 1e-15) and np.any(np.isclose(pf, 1.0))


def test_nesting_violation_is_detected():
    nc = 8
    octs = np.array([[0, 0, 0]], dtype=np.int32)
    parent = A.CellSet(nc, np.array([[0, 0, 0]]))     # parent has a single oct: no full stencil
    with pytest.raises(A.NestingError):
        A.DirichletLevel(2 * nc, octs, parent)


def test_level_set_operator_hand_cases_and_spd():
    # two octs side by side along x at level n=8 (oct coords (1,1,1), (2,1,1));
    # crafted masks: cell c=1 of oct 0 (cx=1) has mask 0.5, its +x neighbour
    # (cell c=0 of oct 1) has mask -1  ->  theta = 0.5/1.5 = 1/3, extra 1/theta-1 = 2
    octs = np.array([[1, 1, 1], [2, 1, 1]])
    lsm = np.ones(16)
    lsm[1] = 0.5
    lsm[8 + 0] = -1.0
    lv = A.OctMGLevel(8, octs, lsm)
    # cell 1 of oct 0: neighbours -x (cell 0, active), +x (oct 1 cell 0, inactive, theta 1/3),
    # -y/+y/-z/+z: cell 3 and cell 5 are inside the oct (active); -y, -z are absent (mask -1,
    # theta = 0.5/1.5 = 1/3 each)
    assert lv.active[1] and not lv.active[8]
    np.testing.assert_allclose(lv.diag[1], 6.0 + 2.0 + 2.0 + 2.0)
    # a +1 cell next to an absent oct: theta = 1/2 -> mirror, extra 1 per such face
    # cell 0 of oct 0 (cx=cy=cz=0): -x, -y, -z absent -> diag 9
    np.testing.assert_allclose(lv.diag[0], 9.0)
    # operator on active cells: symmetric negative definite
    a = build_amr_input(base_n=16, n_refined=1, n_clumps=4)
    levels, fathers = A.build_hierarchy(32, a.levels[1].oct_ijk, max_coarse_octs=8)
    for lvl in levels[1:]:
        act = np.nonzero(lvl.active)[0]
        N = len(lvl.active)
        Mx = np.zeros((len(act), len(act)))
        for k, i in enumerate(act):
            e = np.zeros(N)
            e[i] = 1.0
            Mx[:, k] = lvl.apply(e)[act]
        assert np.allclose(Mx, Mx.T)
        assert np.linalg.eigvalsh(Mx).max() < 0


def test_cellset_index_at_deep_extent():
    # a level of 2^30 cells per dimension: coordinates far beyond what an
    # n^3 linear key holds; lookups (with periodic wrap) against a dict
    n = 1 << 30
    base = np.array([(1 << 29) + 7, 123456789, n // 2 - 5])
    octs = (base // 2 + _patch_octs(n // 2, 0, 3).astype(np.int64)).astype(np.int64)
    cs = A.CellSet(n, octs)
    table = {tuple(int(v) for v in c): i for i, c in enumerate(cs.coords)}
    rng = np.random.default_rng(5)
    q = np.concatenate([cs.coords, cs.coords + rng.integers(-2, 3, size=cs.coords.shape),
                        cs.coords + np.array([n, 0, -n])])          # wrapped copies
    got = cs.index(q)
    want = np.array([table.get(tuple(int(v) % n for v in c), -1) for c in q])
    np.testing.assert_array_equal(got, want)


def test_linear_potential_exact_on_a_deep_level():
    # the linear-potential pin at 2^25 cells per dimension, parent 2^24
    nc = 1 << 24
    n = 2 * nc
    p0 = np.array([nc // 3, nc // 2, nc // 5]) // 2 * 2 // 2          # parent oct origin
    parent = A.CellSet(nc, (p0 + _patch_octs(nc // 2, 0, 8).astype(np.int64)))
    octs = 2 * p0 + 5 + _patch_octs(n // 2, 0, 6).astype(np.int64)    # child cells of the parent's interior
    pc = (parent.coords + 0.5) / nc
    lin = lambda x: 0.3 + 1.5 * x[:, 0] - 2.0 * x[:, 1] + 0.75 * x[:, 2]
    lev = A.DirichletLevel(n, octs, parent)
    phi = lev.solve(np.zeros((len(octs), 8)), lin(pc))
    exact = lin((lev.cells.coords + 0.5) / n).reshape(-1, 8)
    np.testing.assert_allclose(phi, exact, atol=1e-12, rtol=0)


def _dense_dirichlet_system(n, octs, nc, pp):
    """Brute-force assembly of a refined level: cell list, dense matrix of the
    interior couplings and the per-cell sum of ghost values, from coordinates
    alone (a dict of cells; ghosts by the pointwise trilinear rule of the
    interpolation stencil: parent cell g // 2 and its neighbours toward g,
    weights 3/4 and 1/4 per axis)."""
    cells = []
    for o in octs:
        for c in range(8):
            cells.append((2 * int(o[0]) + (c & 1), 2 * int(o[1]) + ((c >> 1) & 1), 2 * int(o[2]) + (c >> 2)))
    where = {cc: i for i, cc in enumerate(cells)}
    N = len(cells)
    h2 = (1.0 / n) ** 2
    A = np.zeros((N, N))
    g = np.zeros(N)
    dense = np.asarray(pp).reshape(nc, nc, nc)
    for i, (x, y, z) in enumerate(cells):
        A[i, i] = -6.0 / h2
        for d in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
            q = ((x + d[0]) % n, (y + d[1]) % n, (z + d[2]) % n)
            if q in where:
                A[i, where[q]] += 1.0 / h2
            else:
                P = np.array(q) // 2
                s = np.where(np.array(q) % 2 == 1, 1, -1)
                val = 0.0
                for a in (0, 1):
                    for b in (0, 1):
                        for cc in (0, 1):
                            w = (0.25 if a else 0.75) * (0.25 if b else 0.75) * (0.25 if cc else 0.75)
                            r = (P + np.array([a * s[0], b * s[1], cc * s[2]])) % nc
                            val += w * dense[r[0], r[1], r[2]]
                g[i] += val
    colour = np.array([(x + y + z) % 2 for x, y, z in cells])
    return A, g, colour


def _sequential_gs(A, rhs, x, rows_by_colour):
    """Gauss-Seidel row substitution, the rows of each colour in index order."""
    x = x.copy()
    for rows in rows_by_colour:
        for i in rows:
            x[i] = (rhs[i] - (A[i] @ x - A[i, i] * x[i])) / A[i, i]
    return x


def test_dirichlet_gs_half_sweeps_equal_sequential_substitution():
    # equation gs_update on a refined level with inhomogeneous ghosts: red rows
    # first, then black, each row using the newest values of its neighbours and
    # the ghosts moved to the right-hand side
    nc = 8
    n = 2 * nc
    octs = _patch_octs(n // 2, 1, 4)
    parent = A.CellSet(nc)
    rng = np.random.default_rng(21)
    pp = rng.standard_normal(len(parent))
    lev = A.DirichletLevel(n, octs, parent)
    f = rng.standard_normal((len(octs), 8))
    phi0 = rng.standard_normal((len(octs), 8))
    Am, g, col = _dense_dirichlet_system(n, octs, nc, pp)
    rhs = f.ravel() - g * n * n
    want = _sequential_gs(Am, rhs, phi0.ravel(), [np.nonzero(col == 0)[0], np.nonzero(col == 1)[0]])
    got = phi0.copy()
    lev.gs_half_sweep(got, f, pp, 0)
    lev.gs_half_sweep(got, f, pp, 1)
    np.testing.assert_allclose(got.ravel(), want, rtol=1e-13, atol=1e-13)
    # the level's right-hand side is the brute-force one, and a zero guess has relres 1
    np.testing.assert_allclose(lev.rhs(f, pp), rhs, rtol=1e-14, atol=1e-12)
    assert abs(lev.relres(np.zeros_like(f), f, pp) - 1.0) < 1e-15


def test_masked_level_gs_half_sweeps_equal_sequential_substitution():
    # a father-cell level with masked cells: red then black over the active
    # cells only, inactive cells untouched, rows of the operator the level applies
    a = build_amr_input(base_n=16, n_refined=1, n_clumps=4)
    levels, _ = A.build_hierarchy(32, a.levels[1].oct_ijk, max_coarse_octs=8)
    lv = levels[1]
    assert 0 < lv.n_active < len(lv.active)
    N = len(lv.active)
    Mx = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        Mx[:, j] = lv.apply(e)
    rng = np.random.default_rng(22)
    b = rng.standard_normal(N)
    e0 = rng.standard_normal(N)
    col = lv.cells.coords.sum(axis=1) % 2
    act = lv.active
    want = _sequential_gs(Mx, b, e0, [np.nonzero(act & (col == 0))[0], np.nonzero(act & (col == 1))[0]])
    got = e0.copy()
    lv.gs_half_sweep(got, b, 0)
    lv.gs_half_sweep(got, b, 1)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(got[~act], e0[~act])


def test_prolong_masked_single_impulse_weights():
    # a coarse correction of 64 in one active coarse cell Q: the fine cells
    # 2Q + o take 27 (o in {0,1}^3), 9 (one axis one step outside), 3 (two
    # axes), 1 (three axes), 0 further away; an impulse in an inactive coarse
    # cell contributes nothing
    n = 32
    octs = _patch_octs(n // 2, 3, 9).astype(np.int64)     # coarse cells 2 and 9 per axis are not fathers
    levels, fathers = A.build_hierarchy(n, octs, max_coarse_octs=100000)
    fine, coarse = levels[0], levels[1]
    Q = np.array([4, 4, 4])
    qi = coarse.cells.index(Q[None, :])[0]
    assert qi >= 0 and coarse.active[qi]
    ec = np.zeros(len(coarse.active))
    ec[qi] = 64.0
    pf = A.prolong_masked(fine, coarse, fathers[0], ec.reshape(-1, 8)).ravel()
    hand = {(0, 0, 0): 27, (1, 1, 1): 27, (1, 0, 1): 27, (-1, 0, 0): 9, (2, 0, 0): 9, (0, -1, 1): 9,
            (1, 1, 2): 9, (-1, -1, 0): 3, (2, 2, 1): 3, (-1, 0, 2): 3, (-1, -1, -1): 1, (2, 2, 2): 1,
            (-1, 2, -1): 1, (-2, 0, 0): 0, (3, 0, 0): 0, (0, 3, 1): 0, (1, 1, -2): 0}
    for o, v in hand.items():
        i = fine.cells.index((2 * Q + np.array(o))[None, :])[0]
        assert i >= 0
        assert pf[i] == v, (o, pf[i], v)
    assert pf.sum() == 64 * 8                  # each coarse cell spreads weight 2 per axis
    # a masked (inactive) coarse cell carries no correction
    inactive = np.nonzero(~coarse.active)[0]
    assert len(inactive) > 0
    ec2 = np.zeros(len(coarse.active))
    ec2[inactive[0]] = 64.0
    assert np.all(A.prolong_masked(fine, coarse, fathers[0], ec2.reshape(-1, 8)) == 0)


def _exact_parent_chain(amr, upto):
    """(CellSet, flat potential) of level upto-1 with each level solved exactly."""
    n0 = amr.base_n
    phi = P.fft_solve(P.rhs(amr.levels[0].rho, 1.0), 1.0 / n0)
    pset, pphi = A.CellSet(n0), phi.ravel()
    for lv in amr.levels[1:upto]:
        d = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
        pphi = d.solve((lv.rho - amr.rho_mean).reshape(-1, 8), pphi).ravel()
        pset = A.CellSet(lv.n_cells_dim, lv.oct_ijk)
    return pset, pphi


@pytest.mark.parametrize("base_n,n_ref,n_clumps,level", [(16, 2, 4, 1), (16, 2, 4, 2), (32, 3, 8, 1)])
def test_refined_vcycle_converges_to_the_direct_solution(base_n, n_ref, n_clumps, level):
    # The cycle's fixed point is the level's discrete solution, which the
    # sparse direct solve fixes independently; each cycle cuts the residual
    # at least 4x (measured 0.15-0.2 after the first), where a dropped,
    # mis-scaled or sign-flipped coarse correction leaves the smoother's
    # rate (near 1) or diverges.
    amr = build_amr_input(base_n=base_n, n_refined=n_ref, n_clumps=n_clumps)
    lv = amr.levels[level]
    pset, pphi = _exact_parent_chain(amr, level)
    d = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
    f = (lv.rho - amr.rho_mean).reshape(-1, 8)
    hier = A.refined_hierarchy(d)
    assert len(hier[0]) >= 2 and not hier[2]
    phi, hist = A.refined_mg_solve(d, f, pphi, tol=1e-10, max_cycles=25)
    ref = d.solve(f, pphi)
    assert hist[-1] <= 1e-10 and len(hist) <= 20
    assert np.max(np.abs(phi - ref)) <= 1e-9 * np.max(np.abs(ref))
    rates = [hist[i + 1] / hist[i] for i in range(len(hist) - 1)]
    assert max(rates) <= 0.25, rates


def test_refined_vcycle_on_a_cut_hierarchy():
    # isolated octs: the father level holds one active cell per oct, the
    # level below none, so the hierarchy is cut and its last level only
    # smoothed; the cycle still converges to the direct solution
    base = 16
    phi0 = P.fft_solve(P.rhs(np.random.default_rng(3).lognormal(size=(base,) * 3), 1.0), 1.0 / base)
    g = np.arange(0, base, 2)
    octs = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    d = A.DirichletLevel(2 * base, octs, A.CellSet(base))
    hier = A.refined_hierarchy(d, max_coarse_octs=64)
    assert [lv.n_active for lv in hier[0]] == [8 * len(octs), len(octs)] and hier[2]
    f = np.random.default_rng(1).standard_normal((len(octs), 8))
    phi, hist = A.refined_mg_solve(d, f, phi0.ravel(), tol=1e-12, max_cycles=20, max_coarse_octs=64)
    ref = d.solve(f, phi0.ravel())
    assert hist[-1] <= 1e-12
    assert np.max(np.abs(phi - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("max_coarse_octs,coarsest", [(8, 4), (64, 8)])
def test_full_coverage_vcycle_equals_the_periodic_vcycle(max_coarse_octs, coarsest):
    # A refined level covering the whole box has no ghosts and a hierarchy
    # whose masks are +1 everywhere (diagonal 6): its V-cycle is then the
    # periodic oracle's V-cycle on the same 16^3 grid (same sweeps, residual,
    # mean restriction, trilinear prolongation, at every level of the
    # recursion), up to the constant that the periodic cycle projects out;
    # the coarsest grid's red-black sweeps converge to the pseudo-inverse
    # solution there (400 sweeps: the slowest mode of 8^3 contracts by 0.81
    # per sweep).
    n = 16
    octs = _patch_octs(n // 2, 0, n // 2)
    lev = A.DirichletLevel(n, octs, A.CellSet(n // 2))
    hier = A.refined_hierarchy(lev, max_coarse_octs=max_coarse_octs)
    assert [lv.n for lv in hier[0]][-1] == coarsest and not hier[2]
    assert all(np.all(lv.diag == 6.0) and lv.active.all() for lv in hier[0])
    rng = np.random.default_rng(4)
    f = rng.standard_normal((n, n, n))
    f -= f.mean()
    phi = rng.standard_normal((n, n, n))
    c = lev.cells.coords
    to_flat = lambda a: a[c[:, 0], c[:, 1], c[:, 2]].reshape(-1, 8)
    p_ref = phi.copy()
    P.vcycle(p_ref, f, 1.0 / n, coarsest=coarsest)
    p_got = to_flat(phi).copy()
    A.refined_vcycle(lev, hier, p_got, to_flat(f), np.zeros(len(lev.parent)), coarse_sweeps=400)
    d = p_got - to_flat(p_ref)
    assert np.max(np.abs(d - d.mean())) <= 1e-11 * np.max(np.abs(p_ref))
