"""GPU parity of g = -grad(phi) (mg_force, mg_op_force) against the oracle's
central differences, through the C ABI.

Periodic levels: with h = 1/n the scaling by 1/(2h) = n/2 is exact on both
sides, so the result must be bit-identical, at 8^3 .. 64^3 and at the full
256^3 size.  Refined levels: cells whose neighbour is a level cell are
bit-identical too; a ghost value is a sum of 8 weighted parent values whose
rounding order may differ, so the bound there is 16 ulp of the largest
potential times n/2.
"""
import numpy as np
import pytest
import torch

from oracle import amr as A
from oracle import poisson as P
from paper_2604_06035_amd import abi
from workloads import build_amr_input, dense_to_oct, lognormal_density

pytestmark = pytest.mark.gpu
DEV = "cuda"


def log(*a):
    print(*a, flush=True)


def _periodic_ref(dense, n):
    g = P.force(dense, 1.0 / n)
    return np.stack([dense_to_oct(g[d]) for d in range(3)])


@pytest.mark.parametrize("n", [8, 16, 32, 64])
def test_periodic_force_bit_exact(n):
    rng = np.random.default_rng(n)
    dense = rng.standard_normal((n, n, n))
    phi = torch.from_numpy(dense_to_oct(dense)).to(DEV)
    ref = _periodic_ref(dense, n)
    hd = abi.mg_build_level(n, 0)
    try:
        g = torch.full((3, n ** 3 // 8, 8), np.nan, dtype=torch.float64, device=DEV)
        abi.mg_force(hd, None, phi, g)
        np.testing.assert_array_equal(g.cpu().numpy(), ref)
        g2 = torch.full_like(g, np.nan)
        abi.mg_op_force(n, 1.0 / n, phi, g2)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g2.cpu().numpy(), ref)
        log(f"force n={n}: bit-exact, max |g| = {np.abs(ref).max():.3e}")
    finally:
        abi.mg_destroy_level(hd)


def test_periodic_force_full_size_256():
    # the benchmark's grid: a solved-like smooth potential (the FFT solve of
    # the lognormal density), every cell compared
    n = 256
    rho = lognormal_density(n, seed=2)
    hd = abi.mg_build_level(n, 0)
    try:
        r = torch.from_numpy(dense_to_oct(rho)).to(DEV)
        phi = torch.zeros_like(r)
        abi.mg_fft_solve(hd, r, None, 1.0, phi)
        g = torch.full((3, r.shape[0], 8), np.nan, dtype=torch.float64, device=DEV)
        abi.mg_force(hd, None, phi, g)
        got = g.cpu().numpy()
        from workloads import oct_to_dense
        ref = _periodic_ref(oct_to_dense(phi.cpu().numpy(), n), n)
        np.testing.assert_array_equal(got, ref)
        log(f"force 256^3: bit-exact over {got.size} values")
    finally:
        abi.mg_destroy_level(hd)


def test_force_rejects_wrong_parent_arguments():
    hd = abi.mg_build_level(16, 0)
    phi = torch.zeros(16 ** 3, dtype=torch.float64, device=DEV)
    g = torch.zeros(3 * 16 ** 3, dtype=torch.float64, device=DEV)
    try:
        with pytest.raises(abi.MgError) as ei:
            abi.mg_force(hd, phi, phi, g)
        assert ei.value.status == abi.MG_ERR_ARG
    finally:
        abi.mg_destroy_level(hd)


@pytest.mark.parametrize("base_n,n_ref,n_clumps", [(16, 2, 4), (32, 3, 8)])
def test_refined_force_matches_oracle(base_n, n_ref, n_clumps):
    amr = build_amr_input(base_n=base_n, n_refined=n_ref, n_clumps=n_clumps)
    rng = np.random.default_rng(base_n * 7 + n_ref)
    handles = []
    try:
        parent = None
        for lv in amr.levels:
            if lv.level == 0:
                hd = abi.mg_build_level(amr.base_n, 0)
            else:
                octs = torch.from_numpy(lv.oct_ijk).to(DEV)
                hd = abi.mg_build_level(amr.base_n, lv.level, lv.n_oct, octs, parent)
            handles.append(hd)
            parent = hd
        for i in range(1, len(amr.levels)):
            lv, plv = amr.levels[i], amr.levels[i - 1]
            if plv.level == 0:
                pset = A.CellSet(amr.base_n)
                pflat = rng.standard_normal(amr.base_n ** 3)
                pdev = torch.from_numpy(dense_to_oct(pflat.reshape((amr.base_n,) * 3))).to(DEV)
            else:
                pset = A.CellSet(plv.n_cells_dim, plv.oct_ijk)
                pflat = rng.standard_normal(plv.n_oct * 8)
                pdev = torch.from_numpy(pflat).to(DEV)
            lev = A.DirichletLevel(lv.n_cells_dim, lv.oct_ijk, pset)
            phi = rng.standard_normal((lv.n_oct, 8))
            ref = lev.force(phi, pflat)
            g = torch.full((3, lv.n_oct, 8), np.nan, dtype=torch.float64, device=DEV)
            abi.mg_force(handles[i], pdev, torch.from_numpy(phi.ravel().copy()).to(DEV), g)
            got = g.cpu().numpy()
            tol = 16 * np.finfo(np.float64).eps * max(np.abs(phi).max(), np.abs(pflat).max()) * lv.n_cells_dim / 2
            err = np.abs(got - ref)
            # cells whose neighbour along d is a level cell: identical arithmetic
            for d in range(3):
                inner = ((lev.nbr[:, 2 * d] >= 0) & (lev.nbr[:, 2 * d + 1] >= 0)).reshape(-1, 8)
                np.testing.assert_array_equal(got[d][inner], ref[d][inner])
            log(f"  level {i} octs={lv.n_oct}: max |diff| {err.max():.3e} (bound {tol:.3e})")
            assert err.max() <= tol
            with pytest.raises(abi.MgError):
                abi.mg_force(handles[i], None, torch.zeros(lv.n_oct * 8, dtype=torch.float64, device=DEV), g)
    finally:
        for hd in handles:
            abi.mg_destroy_level(hd)
