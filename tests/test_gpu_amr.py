"""GPU parity of refined (Dirichlet) levels against the CPU oracle, through the C ABI.

* Morton keys and the hash-table neighbour cache are compared bit-exactly
  with the oracle's bit loop and brute-force / sorted neighbour search.
* Each refined level is solved given its parent's GPU potential; the result
  must reach relative residual <= 1e-10 under the oracle's own residual code
  and match the oracle's exact sparse solve (same parent potential) to
  max|dphi|/max|phi| <= 1e-8.
"""
import numpy as np
import pytest
import torch

from oracle import amr as A
from oracle import morton as M
from oracle import poisson as P
from paper_2604_06035_amd import abi
from workloads import build_amr_input, dense_to_oct, lognormal_density, oct_to_dense

pytestmark = pytest.mark.gpu
DEV = "cuda"


def log(*a):
    print(*a, flush=True)


def test_morton_keys_bit_exact():
    rng = np.random.default_rng(0)
    ijk = rng.integers(0, 1 << 21, size=(100003, 3)).astype(np.int32)
    ijk[:8] = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [(1 << 21) - 1] * 3, [5, 0, 0], [0, 0, 1 << 20], [3, 3, 3]]
    keys = torch.zeros(len(ijk), dtype=torch.int64, device=DEV)
    abi.mg_op_morton(torch.from_numpy(ijk).to(DEV), keys)
    torch.cuda.synchronize()
    got = keys.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, M.encode_array(ijk))


class Chain:
    """GPU handles for a base level plus refined levels, solved in order."""

    def __init__(self, amr, precision=abi.MG_PREC_FP64, load_factor=0.5, brick_shift=0):
        self.amr = amr
        self.handles, self.octs, self.rho = [], [], []
        parent = None
        for lv in amr.levels:
            if lv.level == 0:
                rho = torch.from_numpy(dense_to_oct(lv.rho)).to(DEV)
                hd = abi.mg_build_level(amr.base_n, 0, precision=precision)
                octs = None
            else:
                octs = torch.from_numpy(lv.oct_ijk).to(DEV)
                rho = torch.from_numpy(np.ascontiguousarray(lv.rho.reshape(-1))).to(DEV)
                hd = abi.mg_build_level(amr.base_n, lv.level, lv.n_oct, octs, parent, precision=precision,
                                        load_factor=load_factor, brick_shift=brick_shift)
            self.handles.append(hd)
            self.octs.append(octs)
            self.rho.append(rho)
            parent = hd

    def solve(self, tol=1e-10, max_cycles=100):
        phis, infos = [], []
        for i, hd in enumerate(self.handles):
            phi = torch.zeros_like(self.rho[i])
            pp = phis[-1] if i > 0 else None
            st, info = abi.mg_solve(hd, self.rho[i], None if i == 0 else self.amr.rho_mean, 1.0, pp, phi, tol,
                                    max_cycles)
            assert st == (abi.MG_OK if max_cycles == 100 else abi.MG_NOT_CONVERGED), (i, info)
            log(f"  level {i}: {info}")
            phis.append(phi)
            infos.append(info)
        torch.cuda.synchronize()
        return phis, infos

    def close(self):
        for hd in self.handles:
            abi.mg_destroy_level(hd)


def parent_cellset_and_phi(amr, i, phis):
    """Oracle CellSet of level i-1 and its GPU potential in the CellSet's flat layout."""
    plv = amr.levels[i - 1]
    if plv.level == 0:
        n = amr.base_n
        return A.CellSet(n), oct_to_dense(phis[i - 1].cpu().numpy(), n).ravel()
    return A.CellSet(plv.n_cells_dim, plv.oct_ijk), phis[i - 1].cpu().numpy()


@pytest.mark.parametrize("base_n,n_ref,n_clumps", [(16, 2, 4), (32, 3, 8)])
def test_neighbours_bit_exact(base_n, n_ref, n_clumps):
    amr = build_amr_input(base_n=base_n, n_refined=n_ref, n_clumps=n_clumps)
    log(f"neighbours base={base_n} octs={[l.n_oct for l in amr.levels]}")
    ch = Chain(amr)
    try:
        for i in range(1, len(amr.levels)):
            lv = amr.levels[i]
            nbr = torch.full((lv.n_oct, 6), -7, dtype=torch.int32, device=DEV)
            abi.mg_get_neighbors(ch.handles[i], nbr)
            torch.cuda.synchronize()
            got = nbr.cpu().numpy()
            ref = M.neighbours_sorted(lv.oct_ijk, lv.n_cells_dim // 2)
            np.testing.assert_array_equal(got, ref)
            if lv.n_oct <= 4096:
                np.testing.assert_array_equal(got, M.neighbours_bruteforce(lv.oct_ijk, lv.n_cells_dim // 2))
            # the father-cell level-set hierarchy: active cells per level equal the oracle's
            act = abi.mg_hierarchy_info(ch.handles[i])
            levels, _ = A.build_hierarchy(lv.n_cells_dim, lv.oct_ijk, max_coarse_octs=256)
            ref = [l.n_active for l in levels]
            if 0 in ref:   # the library's hierarchy ends above the first level without active cells
                ref = ref[:ref.index(0)]
            assert act == ref
            assert act[0] == lv.n_cells and act[1] == lv.n_oct
    finally:
        ch.close()


@pytest.mark.parametrize("precision", [abi.MG_PREC_FP64, abi.MG_PREC_MIXED])
@pytest.mark.parametrize("base_n,n_ref,n_clumps", [(16, 2, 4), (32, 3, 8)])
def test_refined_solve_matches_oracle(base_n, n_ref, n_clumps, precision):
    amr = build_amr_input(base_n=base_n, n_refined=n_ref, n_clumps=n_clumps)
    log(f"solve chain base={base_n} octs={[l.n_oct for l in amr.levels]} prec={precision}")
    ch = Chain(amr, precision)
    try:
        phis, infos = ch.solve()
        for i in range(1, len(amr.levels)):
            lv = amr.levels[i]
            pset, pphi = parent_cellset_and_phi(amr, i, phis)
            lev = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
            f = (lv.rho - amr.rho_mean).reshape(-1, 8)
            phi = phis[i].cpu().numpy().reshape(-1, 8)
            rr = lev.relres(phi, f, pphi)
            ref = lev.solve(f, pphi)
            md = float(np.max(np.abs(phi - ref)) / np.max(np.abs(ref)))
            log(f"  level {i}: oracle relres={rr:.3e} maxdiff={md:.3e}")
            assert rr <= 1e-10
            assert md <= 1e-8
    finally:
        ch.close()


def _cycles_vs_oracle(hd, rho, rho_mean, phi_parent, d, f, pphi, cycles=(1, 2, 3)):
    """GPU potential after exactly k V-cycles from zero against the oracle's
    refined V-cycle (same hierarchy, sweeps and coarsest relaxation)."""
    hier = A.refined_hierarchy(d)
    ref = np.zeros((d.n_cells // 8, 8))
    done = 0
    for k in cycles:
        phi = torch.zeros_like(rho)
        st, info = abi.mg_solve(hd, rho, rho_mean, 1.0, phi_parent, phi, 1e-30, k)
        assert st == abi.MG_NOT_CONVERGED and info["cycles"] == k
        while done < k:
            A.refined_vcycle(d, hier, ref, f, pphi)
            done += 1
        got = phi.cpu().numpy().reshape(-1, 8)
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        rr = d.relres(ref, f, pphi)
        log(f"    {k} cycles: max rel diff {err:.2e}; relres gpu {info['relres']:.4e} oracle {rr:.4e}")
        assert err <= 1e-12
        assert abs(info["relres"] - rr) <= 1e-6 * rr
    return [lv.n_active for lv in hier[0]], hier[2]


@pytest.mark.parametrize("base_n,n_ref,n_clumps", [(16, 2, 4), (32, 3, 8)])
def test_refined_cycles_match_oracle(base_n, n_ref, n_clumps):
    # one, two and three V-cycles on each refined level equal the oracle's:
    # the brick sweeps, the prolongation fused into the first post-sweep,
    # the residual + restriction and the father-cell levels, cycle by cycle
    # (a converged solve cannot see a wrong prolongation or restriction)
    amr = build_amr_input(base_n=base_n, n_refined=n_ref, n_clumps=n_clumps)
    ch = Chain(amr)
    try:
        phis, _ = ch.solve()
        for i in range(1, len(amr.levels)):
            lv = amr.levels[i]
            pset, pphi = parent_cellset_and_phi(amr, i, phis)
            d = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
            f = (lv.rho - amr.rho_mean).reshape(-1, 8)
            log(f"  level {i} ({lv.n_oct} octs)")
            act, cut = _cycles_vs_oracle(ch.handles[i], ch.rho[i], amr.rho_mean, phis[i - 1], d, f, pphi)
            assert act == abi.mg_hierarchy_info(ch.handles[i])
    finally:
        ch.close()


def test_refined_cycles_on_a_cut_hierarchy_match_oracle():
    # isolated octs: the hierarchy is cut below the father level, which is
    # then only smoothed (nu_pre + nu_post sweeps from zero)
    base = 16
    g = np.arange(0, base, 2)
    octs = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    rng = np.random.default_rng(7)
    rho0 = lognormal_density(base, seed=7)
    rho1 = rng.lognormal(size=(len(octs), 8))
    rho_mean = float(rho0.mean())
    h0 = abi.mg_build_level(base, 0)
    h1 = None
    try:
        r0 = torch.from_numpy(dense_to_oct(rho0)).to(DEV)
        p0 = torch.zeros_like(r0)
        assert abi.mg_solve(h0, r0, None, 1.0, None, p0, 1e-12, 50)[0] == abi.MG_OK
        h1 = abi.mg_build_level(base, 1, len(octs), torch.from_numpy(octs).to(DEV), h0)
        r1 = torch.from_numpy(rho1).to(DEV)
        pphi = oct_to_dense(p0.cpu().numpy(), base).ravel()
        d = A.DirichletLevel(2 * base, octs, A.CellSet(base))
        act, cut = _cycles_vs_oracle(h1, r1, rho_mean, p0, d, rho1 - rho_mean, pphi)
        assert cut and act == [8 * len(octs), len(octs)]
    finally:
        if h1:
            abi.mg_destroy_level(h1)
        abi.mg_destroy_level(h0)


@pytest.mark.parametrize("precision", [abi.MG_PREC_FP64, abi.MG_PREC_MIXED])
def test_brick_lattice_shift_does_not_change_the_iterates(precision):
    # the bricks only stage octs: on every one of the 8 lattices (forced on
    # every hierarchy level, and the automatic choice) two V-cycles per level
    # give bit-identical potentials; the sweeps with the prolongation read
    # the coarse window at the lattice's offset
    amr = build_amr_input(base_n=32, n_refined=3, n_clumps=8)
    log(f"brick shifts octs={[l.n_oct for l in amr.levels]} prec={precision}")
    ref = None
    for bs in [1, 0, 2, 3, 4, 5, 6, 7, 8]:
        ch = Chain(amr, precision, brick_shift=bs)
        try:
            phis, _ = ch.solve(max_cycles=2)
            got = [p.cpu().numpy() for p in phis]
        finally:
            ch.close()
        if ref is None:
            ref = got
            continue
        for i in range(1, len(got)):
            diff = int(np.count_nonzero(got[i].view(np.int64) != ref[i].view(np.int64)))
            log(f"  brick_shift={bs} level {i}: {diff} cells differ from the aligned lattice")
            assert diff == 0


@pytest.mark.parametrize("base_n,n_ref,n_clumps", [(16, 2, 4), (32, 3, 8)])
def test_refined_smoother_matches_oracle(base_n, n_ref, n_clumps):
    # the refined-level smoother (LDS-staged brick sweeps with Dirichlet
    # ghosts) against the oracle's red-then-black half sweeps, cell by cell,
    # for 1 and 3 sweeps from a random phi, with a random parent potential
    amr = build_amr_input(base_n=base_n, n_refined=n_ref, n_clumps=n_clumps)
    ch = Chain(amr)
    rng = np.random.default_rng(base_n + n_ref)
    try:
        for i in range(1, len(amr.levels)):
            lv = amr.levels[i]
            plv = amr.levels[i - 1]
            if plv.level == 0:
                pset = A.CellSet(amr.base_n)
                pphi_flat = rng.standard_normal(amr.base_n ** 3) * 1e-3
                pphi_dev = torch.from_numpy(dense_to_oct(pphi_flat.reshape((amr.base_n,) * 3))).to(DEV)
            else:
                pset = A.CellSet(plv.n_cells_dim, plv.oct_ijk)
                pphi_flat = rng.standard_normal(plv.n_oct * 8) * 1e-3
                pphi_dev = torch.from_numpy(pphi_flat).to(DEV)
            lev = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
            f = (lv.rho - amr.rho_mean).reshape(-1, 8)
            phi0 = rng.standard_normal((lv.n_oct, 8)) * 1e-3
            for sweeps in (1, 3):
                ref = phi0.copy()
                for _ in range(sweeps):
                    lev.gs_half_sweep(ref, f, pphi_flat, 0)
                    lev.gs_half_sweep(ref, f, pphi_flat, 1)
                phi_d = torch.from_numpy(phi0.ravel().copy()).to(DEV)
                abi.mg_level_smooth(ch.handles[i], ch.rho[i], amr.rho_mean, 1.0, pphi_dev, phi_d, sweeps)
                got = phi_d.cpu().numpy().reshape(-1, 8)
                err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
                log(f"  level {i} octs={lv.n_oct} sweeps={sweeps}: max rel diff {err:.3e}")
                assert err <= 1e-12
    finally:
        ch.close()


def test_refined_fused_norm_matches_oracle():
    # the first sweep of each cycle also returns ||f - L phi|| of the incoming
    # phi: with no cycle allowed, relres0 must be the oracle's relative
    # residual of the guess (ghosts from a random parent potential)
    amr = build_amr_input(base_n=32, n_refined=2, n_clumps=8)
    ch = Chain(amr)
    rng = np.random.default_rng(11)
    try:
        for i in range(1, len(amr.levels)):
            lv, plv = amr.levels[i], amr.levels[i - 1]
            if plv.level == 0:
                pset = A.CellSet(amr.base_n)
                pflat = rng.standard_normal(amr.base_n ** 3) * 1e-3
                pdev = torch.from_numpy(dense_to_oct(pflat.reshape((amr.base_n,) * 3))).to(DEV)
            else:
                pset = A.CellSet(plv.n_cells_dim, plv.oct_ijk)
                pflat = rng.standard_normal(plv.n_oct * 8) * 1e-3
                pdev = torch.from_numpy(pflat).to(DEV)
            lev = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
            f = (lv.rho - amr.rho_mean).reshape(-1, 8)
            phi0 = rng.standard_normal((lv.n_oct, 8)) * 1e-4
            phi_d = torch.from_numpy(phi0.ravel().copy()).to(DEV)
            st, info = abi.mg_solve(ch.handles[i], ch.rho[i], amr.rho_mean, 1.0, pdev, phi_d, 1e-10, 0)
            ref = lev.relres(phi0, f, pflat)
            log(f"  level {i}: relres0 gpu={info['relres0']:.15e} oracle={ref:.15e}")
            assert st == abi.MG_NOT_CONVERGED and info["cycles"] == 0
            assert abs(info["relres0"] - ref) <= 1e-12 * ref
            np.testing.assert_array_equal(phi_d.cpu().numpy().reshape(-1, 8), phi0)   # untouched
    finally:
        ch.close()


def test_load_factors_and_error_paths():
    amr = build_amr_input(base_n=16, n_refined=1, n_clumps=4)
    lv = amr.levels[1]
    base = abi.mg_build_level(16, 0)
    try:
        octs = torch.from_numpy(lv.oct_ijk).to(DEV)
        # the neighbour cache does not depend on the table size
        ref = M.neighbours_sorted(lv.oct_ijk, 16)
        for lf in (0.9, 0.5, 0.1):
            hd = abi.mg_build_level(16, 1, lv.n_oct, octs, base, load_factor=lf)
            nbr = torch.zeros((lv.n_oct, 6), dtype=torch.int32, device=DEV)
            abi.mg_get_neighbors(hd, nbr)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(nbr.cpu().numpy(), ref)
            abi.mg_destroy_level(hd)
        # empty refined level
        with pytest.raises(abi.MgError) as ei:
            abi.mg_build_level(16, 1, 0, octs[:0], base)
        assert ei.value.status == abi.MG_ERR_ARG
        # duplicate oct
        dup = torch.cat([octs, octs[:1]])
        with pytest.raises(abi.MgError) as ei:
            abi.mg_build_level(16, 1, lv.n_oct + 1, dup, base)
        assert ei.value.status == abi.MG_ERR_ARG and "duplicate" in str(ei.value)
        # coordinate out of range
        bad = octs.clone()
        bad[3, 1] = 16
        with pytest.raises(abi.MgError) as ei:
            abi.mg_build_level(16, 1, lv.n_oct, bad, base)
        assert ei.value.status == abi.MG_ERR_ARG
        # level 2 on top of a sparse level 1 that does not contain its stencil
        one = torch.tensor([[20, 20, 20]], dtype=torch.int32, device=DEV)
        l1 = abi.mg_build_level(16, 1, 1, torch.tensor([[5, 5, 5]], dtype=torch.int32, device=DEV), base)
        with pytest.raises(abi.MgError) as ei:
            abi.mg_build_level(16, 2, 1, one, l1)
        assert ei.value.status == abi.MG_ERR_NESTING
        abi.mg_destroy_level(l1)
        # refined solve without parent phi / mean
        hd = abi.mg_build_level(16, 1, lv.n_oct, octs, base)
        rho = torch.ones(lv.n_cells, dtype=torch.float64, device=DEV)
        phi = torch.zeros_like(rho)
        with pytest.raises(abi.MgError):
            abi.mg_solve(hd, rho, None, 1.0, torch.zeros(16 ** 3, dtype=torch.float64, device=DEV), phi, 1e-10, 5)
        with pytest.raises(abi.MgError):
            abi.mg_solve(hd, rho, 1.0, 1.0, None, phi, 1e-10, 5)
        # the direct FFT solve exists for periodic levels only
        with pytest.raises(abi.MgError) as ei:
            abi.mg_fft_solve(hd, rho, 1.0, 1.0, phi)
        assert ei.value.status == abi.MG_ERR_ARG and "periodic" in str(ei.value)
        abi.mg_destroy_level(hd)
    finally:
        abi.mg_destroy_level(base)


@pytest.mark.slow
def test_full_size_amr_chain():
    # periodic 128^3 base + 3 refined levels, 64 Plummer clumps (the full AMR workload)
    amr = build_amr_input()
    log(f"full AMR octs={[l.n_oct for l in amr.levels]}")
    ch = Chain(amr)
    try:
        phis, infos = ch.solve()
        for i in range(1, len(amr.levels)):
            lv = amr.levels[i]
            nbr = torch.zeros((lv.n_oct, 6), dtype=torch.int32, device=DEV)
            abi.mg_get_neighbors(ch.handles[i], nbr)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(nbr.cpu().numpy(), M.neighbours_sorted(lv.oct_ijk, lv.n_cells_dim // 2))
            pset, pphi = parent_cellset_and_phi(amr, i, phis)
            lev = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
            f = (lv.rho - amr.rho_mean).reshape(-1, 8)
            phi = phis[i].cpu().numpy()
            rr = lev.relres(phi, f, pphi)
            log(f"  level {i}: cells={lv.n_cells} cycles={infos[i]['cycles']} oracle relres={rr:.3e}")
            assert rr <= 1e-10
            # the force step on the solved potential, every cell against the
            # oracle: identical where both neighbours along an axis are level
            # cells, within the ghost values' rounding next to a ghost face
            g = torch.full((3, lv.n_oct, 8), np.nan, dtype=torch.float64, device=DEV)
            abi.mg_force(ch.handles[i], phis[i - 1], phis[i], g)
            got = g.cpu().numpy()
            ref = lev.force(phi.reshape(-1, 8), pphi)
            for d in range(3):
                inner = ((lev.nbr[:, 2 * d] >= 0) & (lev.nbr[:, 2 * d + 1] >= 0)).reshape(-1, 8)
                np.testing.assert_array_equal(got[d][inner], ref[d][inner])
            tol = 16 * np.finfo(np.float64).eps * max(np.abs(phi).max(), np.abs(pphi).max()) * lv.n_cells_dim / 2
            err = float(np.abs(got - ref).max())
            log(f"  level {i}: force max |diff| {err:.3e} (bound {tol:.3e})")
            assert err <= tol
    finally:
        ch.close()


@pytest.mark.parametrize("precision", [abi.MG_PREC_FP64, abi.MG_PREC_MIXED])
def test_chain_in_one_call(precision):
    # mg_solve_chain solves the hierarchy coarse to fine in one call: the same
    # solves as level by level (the mean is the GPU's FP64 mean of level 0
    # instead of the host's, so the potentials agree to rounding); with the
    # base level solved by the direct FFT the refined levels still converge
    # and agree with the multigrid chain to the multigrid tolerance
    amr = build_amr_input(base_n=32, n_refined=3, n_clumps=8)
    ch = Chain(amr, precision)
    try:
        ref, ref_infos = ch.solve()
        for base_fft in (False, True):
            phis = [torch.zeros_like(r) for r in ch.rho]
            st, infos = abi.mg_solve_chain(ch.handles, ch.rho, None, 1.0, phis, 1e-10, 100, base_fft=base_fft)
            torch.cuda.synchronize()
            assert st == abi.MG_OK
            for i, (p, r) in enumerate(zip(phis, ref)):
                d = float((p - r).abs().max() / r.abs().max())
                log(f"  base_fft={base_fft} level {i}: {infos[i]} max rel diff vs level by level {d:.2e}")
                assert infos[i]["relres"] <= 1e-10
                assert abs(infos[i]["rho_mean"] - amr.rho_mean) <= 1e-14 * amr.rho_mean
                if base_fft:
                    assert d <= 1e-8
                else:
                    assert infos[i]["cycles"] == ref_infos[i]["cycles"] and d <= 1e-12
            if base_fft:
                assert infos[0]["cycles"] == 0 and infos[0]["relres"] <= 1e-12
        # argument checks: a handle out of order
        with pytest.raises(abi.MgError, match="level-i handle"):
            abi.mg_solve_chain([ch.handles[0], ch.handles[2]], ch.rho[:1] + ch.rho[2:3], None, 1.0,
                               [torch.zeros_like(ch.rho[0]), torch.zeros_like(ch.rho[2])])
    finally:
        ch.close()


def _nested_cubes(base_n, depth, side=6, a1=5):
    """Octs of levels 1..depth: cubes of side^3 octs, each level's cube the
    refinement of the central side^3 cells of the level above (a shared
    centre), so every level is properly nested."""
    levels, a = [], a1
    r = np.arange(side)
    cube = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    for lv in range(1, depth + 1):
        levels.append((a + cube).astype(np.int32))
        a = 2 * a + (side // 2)
    return levels


def test_deep_levels_use_key_frames():
    # levels 1..21 above a 16^3 base: from level 19 on the extent passes 2^21
    # octs per axis (64-bit keys cannot hold absolute coordinates), so the
    # builder keys them in a frame near the octs.  Neighbours must still be
    # bit-exact, and each deep level's solve (ghosts from a given parent
    # potential of the h^2 scale the level's own solution has) must match the
    # oracle's exact solve; the force step too.
    base_n, depth = 16, 21
    octs = _nested_cubes(base_n, depth)
    rng = np.random.default_rng(19)
    handles = [abi.mg_build_level(base_n, 0)]
    try:
        for lv in range(1, depth + 1):
            o = torch.from_numpy(octs[lv - 1]).to(DEV)
            handles.append(abi.mg_build_level(base_n, lv, len(octs[lv - 1]), o, handles[-1]))
        for lv in (17, 18, 19, 20, 21):
            n = base_n << lv
            n_dim = n // 2
            oi = octs[lv - 1]
            nbr = torch.full((len(oi), 6), -7, dtype=torch.int32, device=DEV)
            abi.mg_get_neighbors(handles[lv], nbr)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(nbr.cpu().numpy(), M.neighbours_bruteforce(oi, n_dim))
            pset = A.CellSet(n // 2, octs[lv - 2])
            h = 1.0 / n
            pflat = rng.standard_normal(len(pset)) * (2 * h) ** 2
            lev = A.DirichletLevel(n, oi, pset)
            rho = 1.0 + rng.random((len(oi), 8))
            f = rho - 1.0
            ref = lev.solve(f, pflat)
            phi = torch.zeros(len(oi) * 8, dtype=torch.float64, device=DEV)
            # solved to 5e-11 by the library's residual, so that the oracle's
            # own residual (other rounding) has margin under the 1e-10 bar
            st, info = abi.mg_solve(handles[lv], torch.from_numpy(rho.ravel().copy()).to(DEV), 1.0, 1.0,
                                    torch.from_numpy(pflat).to(DEV), phi, 5e-11, 60)
            got = phi.cpu().numpy().reshape(-1, 8)
            rr = lev.relres(got, f, pflat)
            md = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
            log(f"  level {lv} (extent 2^{n_dim.bit_length() - 1} octs): {info['cycles']} cycles, "
                f"oracle relres {rr:.2e}, maxdiff {md:.2e}")
            assert st == abi.MG_OK and rr <= 1e-10 and md <= 1e-8
            g = torch.full((3, len(oi), 8), np.nan, dtype=torch.float64, device=DEV)
            abi.mg_force(handles[lv], torch.from_numpy(pflat).to(DEV), phi, g)
            fref = lev.force(got, pflat)
            tol = 16 * np.finfo(np.float64).eps * max(np.abs(got).max(), np.abs(pflat).max()) * n / 2
            assert float(np.abs(g.cpu().numpy() - fref).max()) <= tol
        # a deep level whose octs spread over more than the key space along x
        far = np.array([[0, 0, 0], [1 << 22, 0, 0]], dtype=np.int32) + octs[19][0]
        with pytest.raises(abi.MgError) as ei:
            abi.mg_build_level(base_n, 20, 2, torch.from_numpy(far).to(DEV), handles[19])
        assert ei.value.status == abi.MG_ERR_ARG and "2^21" in str(ei.value)
    finally:
        for hd in reversed(handles):
            abi.mg_destroy_level(hd)


@pytest.mark.parametrize("precision", [abi.MG_PREC_FP64, abi.MG_PREC_MIXED])
def test_level_driven_only_by_its_boundary(precision):
    # a refined level whose density equals the mean (f = 0) under a non-zero
    # parent potential: the solution is the discrete harmonic extension of the
    # ghosts, not zero; the relative residual is taken on the system's full
    # right-hand side (the Dirichlet terms), so the solve converges to it
    amr = build_amr_input(base_n=16, n_refined=1, n_clumps=4)
    lv = amr.levels[1]
    ch = Chain(amr, precision)
    rng = np.random.default_rng(31)
    try:
        x = (np.arange(16) + 0.5) / 16
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        pdense = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + 0.3 * np.sin(4 * np.pi * Z) + \
            1e-2 * rng.standard_normal((16, 16, 16))
        pdev = torch.from_numpy(dense_to_oct(pdense)).to(DEV)
        pset = A.CellSet(16)
        lev = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
        rho = torch.full((lv.n_oct * 8,), amr.rho_mean, dtype=torch.float64, device=DEV)
        f = np.zeros((lv.n_oct, 8))
        phi = torch.zeros_like(rho)
        st, info = abi.mg_solve(ch.handles[1], rho, amr.rho_mean, 1.0, pdev, phi, 1e-10, 100)
        torch.cuda.synchronize()
        got = phi.cpu().numpy().reshape(-1, 8)
        ref = lev.solve(f, pdense.ravel())
        rr = lev.relres(got, f, pdense.ravel())
        md = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        log(f"boundary-driven level prec={precision}: {info} oracle relres={rr:.2e} maxdiff={md:.2e}")
        assert st == abi.MG_OK and info["cycles"] > 0 and abs(info["relres0"] - 1.0) < 1e-12
        assert np.max(np.abs(ref)) > 0.1 and rr <= 1e-10 and md <= 1e-8
        rn, bn = abi.mg_residual_norm(ch.handles[1], rho, amr.rho_mean, 1.0, pdev, phi)
        assert abs(bn - lev.rhs_norm(f, pdense.ravel())) <= 1e-13 * bn
        # zero density contrast and zero parent potential: b = 0, phi = 0 at once
        zero_parent = torch.zeros_like(pdev)
        phi.fill_(1.0)
        st, info = abi.mg_solve(ch.handles[1], rho, amr.rho_mean, 1.0, zero_parent, phi, 1e-10, 100)
        torch.cuda.synchronize()
        assert st == abi.MG_OK and info["cycles"] == 0 and bool(torch.all(phi == 0.0))
    finally:
        ch.close()


@pytest.fixture(scope="module")
def full_amr_oracle_chain():
    """The full AMR workload and the oracle's own chain of exact solutions:
    the periodic base by the FFT solve, every refined level by CG (relative
    residual 1e-12) with the oracle's solution of the level above as its
    Dirichlet source (no GPU value enters)."""
    amr = build_amr_input()
    log(f"full AMR octs={[l.n_oct for l in amr.levels]}")
    n0 = amr.base_n
    f0 = P.rhs(amr.levels[0].rho, 1.0, amr.rho_mean)
    refs = [P.fft_solve(f0, 1.0 / n0)]
    pset, pphi = A.CellSet(n0), refs[0].ravel()
    levs = [None]
    for lv in amr.levels[1:]:
        lev = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
        f = (lv.rho - amr.rho_mean).reshape(-1, 8)
        refs.append(lev.solve(f, pphi, rtol=1e-12))
        log(f"  oracle level {lv.level}: relres {lev.relres(refs[-1], f, pphi):.2e}")
        levs.append(lev)
        pset, pphi = lev.cells, refs[-1].ravel()
    return amr, refs, levs


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [abi.MG_PREC_FP64, abi.MG_PREC_MIXED])
def test_full_size_amr_levels_match_oracle_chain(full_amr_oracle_chain, precision):
    # every level of the full AMR workload (128^3 base + 3 refined levels,
    # 1.47M / 1.23M / 5.13M cells), plain and mixed: relative residual <= 1e-10
    # under the oracle's residual (with the GPU parent as the level's boundary)
    # and max |dphi| / max |phi| <= 1e-8 against the oracle's own chain
    amr, refs, levs = full_amr_oracle_chain
    ch = Chain(amr, precision)
    try:
        phis, infos = ch.solve()
        phi0 = oct_to_dense(phis[0].cpu().numpy(), amr.base_n)
        md0 = P.maxdiff(phi0, refs[0])
        log(f"  level 0: maxdiff vs FFT {md0:.2e}")
        assert md0 <= 1e-8
        for i in range(1, len(amr.levels)):
            lv = amr.levels[i]
            pset, pphi = parent_cellset_and_phi(amr, i, phis)
            f = (lv.rho - amr.rho_mean).reshape(-1, 8)
            phi = phis[i].cpu().numpy().reshape(-1, 8)
            rr = levs[i].relres(phi, f, pphi)
            md = float(np.max(np.abs(phi - refs[i])) / np.max(np.abs(refs[i])))
            log(f"  level {i}: cells={lv.n_cells} cycles={infos[i]['cycles']} oracle relres={rr:.2e} "
                f"maxdiff vs oracle chain={md:.2e}")
            assert rr <= 1e-10
            assert md <= 1e-8
    finally:
        ch.close()


def test_rebuilt_levels_reuse_memory_and_give_the_same_solution():
    # A refined level built, destroyed and built again (its device blocks now
    # come back from the per-device cache, possibly holding the old level's
    # data) has the same hierarchy and gives the same potential bit for bit,
    # in either precision, also while other levels live beside it.
    amr = build_amr_input(base_n=32, n_refined=2, n_clumps=8)
    ch = Chain(amr, abi.MG_PREC_FP64)
    try:
        phis, _ = ch.solve()
        lv = amr.levels[-1]
        parent = ch.handles[-2]
        pphi = phis[-2]
        ref = {}
        for rep in range(3):
            for prec in (abi.MG_PREC_FP64, abi.MG_PREC_MIXED):
                extra = abi.mg_build_level(amr.base_n, lv.level, lv.n_oct, ch.octs[-1], parent, precision=prec)
                hd = abi.mg_build_level(amr.base_n, lv.level, lv.n_oct, ch.octs[-1], parent, precision=prec)
                try:
                    phi = torch.zeros_like(ch.rho[-1])
                    st, info = abi.mg_solve(hd, ch.rho[-1], amr.rho_mean, 1.0, pphi, phi, 1e-10, 100)
                    assert st == abi.MG_OK
                    got = (abi.mg_hierarchy_info(hd), info["cycles"], phi.cpu().numpy())
                finally:
                    abi.mg_destroy_level(hd)
                    abi.mg_destroy_level(extra)
                log(f"  rebuild {rep} precision {prec}: cycles {got[1]} hierarchy {got[0]}")
                if prec not in ref:
                    ref[prec] = got
                    continue
                assert got[0] == ref[prec][0] and got[1] == ref[prec][1]
                assert np.array_equal(got[2], ref[prec][2])
        # the first build's potential (same level, same parent) as well
        assert np.array_equal(ref[abi.MG_PREC_FP64][2], phis[-1].cpu().numpy())
    finally:
        ch.close()
