"""Pins for the seeded input generators (shared by oracle and GPU path)."""
import numpy as np

from workloads import (array_digest, build_amr_input, dense_to_oct, gaussian_random_field,
                       lognormal_density, oct_to_dense, sinusoid_density)


def test_oct_layout_round_trip_and_indexing():
    n = 8
    a = np.arange(n ** 3, dtype=np.float64).reshape(n, n, n)
    o = dense_to_oct(a)
    assert o.shape == (64, 8)
    np.testing.assert_array_equal(oct_to_dense(o, n), a)
    # oct (ox, oy, oz) = (1, 2, 3), cell (cx, cy, cz) = (1, 0, 1)
    ox, oy, oz, cx, cy, cz = 1, 2, 3, 1, 0, 1
    assert o[(oz * 4 + oy) * 4 + ox, cx + 2 * cy + 4 * cz] == a[2 * ox + cx, 2 * oy + cy, 2 * oz + cz]


def test_grf_moments_and_spectrum():
    n = 64
    g = gaussian_random_field(n, -2.5, 1.5, seed=2)
    assert abs(g.mean()) < 1e-14
    assert abs(g.var() - 1.5) < 1e-12
    # log-binned power spectrum slope
    pk = np.abs(np.fft.rfftn(g)) ** 2
    k = np.fft.fftfreq(n, 1.0 / n)
    kz = np.fft.rfftfreq(n, 1.0 / n)
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2)
    sel = (kk >= 2) & (kk <= 20)
    bins = np.logspace(np.log10(2), np.log10(20), 10)
    idx = np.digitize(kk[sel], bins)
    xs, ys = [], []
    for b in range(1, len(bins)):
        m = idx == b
        if m.sum() > 10:
            xs.append(np.log(kk[sel][m].mean()))
            ys.append(np.log(pk[sel][m].mean()))
    slope = np.polyfit(xs, ys, 1)[0]
    assert abs(slope - (-2.5)) < 0.1


def test_generators_are_bit_reproducible():
    a = lognormal_density(32, seed=2)
    b = lognormal_density(32, seed=2)
    assert array_digest(a) == array_digest(b)
    assert abs(a.mean() - 1.0) < 0.2
    assert array_digest(lognormal_density(32, seed=3)) != array_digest(a)


def test_sinusoid():
    r = sinusoid_density(32)
    assert abs(r.mean() - 1.0) < 1e-14
    assert abs(r.max() - 1.5) < 0.01


def test_amr_input_nesting_and_counts():
    a = build_amr_input(base_n=32, n_refined=2, n_clumps=8)
    assert len(a.levels) == 3
    for lo, hi in zip(a.levels[:-1], a.levels[1:]):
        # every fine oct's father cell and its 26 neighbours exist on the coarser level
        n_lo = lo.n_cells_dim
        if lo.oct_ijk is None:
            present = None
        else:
            cells = (2 * lo.oct_ijk[:, None, :].astype(np.int64) +
                     np.array([(c & 1, (c >> 1) & 1, c >> 2) for c in range(8)])[None]).reshape(-1, 3)
            present = set(map(tuple, cells))
        for f in hi.oct_ijk[::17]:
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        q = tuple((f + np.array([dx, dy, dz])) % n_lo)
                        assert present is None or q in present
        assert hi.rho.shape == (hi.n_oct, 8)
        assert len(np.unique(hi.oct_ijk, axis=0)) == hi.n_oct
