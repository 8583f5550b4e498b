"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module generates densities and oct sets and converts between array
layouts.  It contains none of the Poisson solver's arithmetic (no stencil,
no smoother, no restriction or prolongation, no Morton keys, no hashing),
so that the CPU oracle and the GPU path can both consume its output while
sharing no solver code.

Array conventions
-----------------
* A dense field on an ``n^3`` periodic grid is a float64 array ``a[i, j, k]``
  with ``i`` along x, ``j`` along y and ``k`` along z; cell ``(i, j, k)`` has its
  centre at ``((i + 1/2) h, (j + 1/2) h, (k + 1/2) h)`` with ``h = 1/n`` on the
  unit box.
* The oct-major layout used by the library is ``[n_oct][8]``: an oct is a
  2x2x2 block of cells (the paper's "grid", section on the Morton key hash
  table), and cell ``c = cx + 2 cy + 4 cz`` inside it.  On a full periodic
  level the octs are listed lexicographically with x fastest:
  ``oct = (oz * no + oy) * no + ox`` with ``no = n / 2``.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "dense_to_oct", "oct_to_dense", "sinusoid_density", "gaussian_random_field",
    "lognormal_density", "cnn_field_params", "plummer_centres", "AmrLevel",
    "AmrInput", "build_amr_input", "array_digest", "brick_order",
]


# ----------------------------------------------------------------------------
# layouts
# ----------------------------------------------------------------------------
def dense_to_oct(a: np.ndarray) -> np.ndarray:
    """Dense ``[n,n,n]`` (x, y, z) -> oct-major ``[(n/2)^3, 8]`` (lexicographic octs)."""
    n = a.shape[0]
    assert a.shape == (n, n, n) and n % 2 == 0
    no = n // 2
    t = a.reshape(no, 2, no, 2, no, 2)           # ox cx oy cy oz cz
    t = t.transpose(4, 2, 0, 5, 3, 1)            # oz oy ox cz cy cx
    return np.ascontiguousarray(t.reshape(no ** 3, 8))


def oct_to_dense(o: np.ndarray, n: int) -> np.ndarray:
    """Inverse of :func:`dense_to_oct`."""
    no = n // 2
    t = np.asarray(o).reshape(no, no, no, 2, 2, 2)   # oz oy ox cz cy cx
    t = t.transpose(2, 5, 1, 4, 0, 3)                # ox cx oy cy oz cz
    return np.ascontiguousarray(t.reshape(n, n, n))


def array_digest(a: np.ndarray) -> str:
    """SHA-256 of an array's bytes (C order), used to pin generator outputs."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ----------------------------------------------------------------------------
# densities
# ----------------------------------------------------------------------------
def cell_centres_1d(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def sinusoid_density(n: int, amplitude: float = 0.5) -> np.ndarray:
    """rho = 1 + A sin(2 pi x) sin(2 pi y) sin(2 pi z) sampled at cell centres."""
    x = cell_centres_1d(n)
    s = np.sin(2.0 * np.pi * x)
    return 1.0 + amplitude * s[:, None, None] * s[None, :, None] * s[None, None, :]


def gaussian_random_field(n: int, slope: float, var: float, seed: int | None = None,
                          rng: np.random.Generator | None = None) -> np.ndarray:
    """Zero-mean periodic Gaussian field with P(k) ~ |k|^slope and sample variance ``var``.

    Recipe: white noise from ``numpy.random.default_rng(seed)`` -> real FFT ->
    multiply by sqrt(P(|k|)) with |k| in integer lattice units; the k = 0 mode and
    every mode on a Nyquist plane get amplitude 0 -> inverse FFT -> subtract the
    sample mean -> rescale to sample variance exactly ``var``.  float64 throughout.
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    del w
    k = np.fft.fftfreq(n, d=1.0 / n)
    kz = np.fft.rfftfreq(n, d=1.0 / n)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)     # sqrt(|k|^slope)
    del k2
    half = n // 2
    amp[half, :, :] = 0.0
    amp[:, half, :] = 0.0
    amp[:, :, half] = 0.0
    wk *= amp
    del amp
    g = np.fft.irfftn(wk, s=(n, n, n), axes=(0, 1, 2))
    del wk
    g -= g.mean()
    g *= np.sqrt(var / g.var())
    return g


def lognormal_density(n: int, slope: float = -2.5, var: float = 1.5, seed: int = 2,
                      rng: np.random.Generator | None = None) -> np.ndarray:
    """rho = exp(g - var/2) with g from :func:`gaussian_random_field` (mean ~ 1)."""
    g = gaussian_random_field(n, slope, var, seed=seed, rng=rng)
    np.subtract(g, 0.5 * var, out=g)
    np.exp(g, out=g)
    return g


def cnn_field_params(seed: int) -> tuple[float, float, np.random.Generator]:
    """Per-seed statistics of the learned-warm-start workload.

    Draws the spectral slope ~ U[-3, -2] and the variance ~ U[0.5, 2] from the
    seed's generator, which then continues to draw the field's white noise.
    """
    rng = np.random.default_rng(seed)
    slope = float(rng.uniform(-3.0, -2.0))
    var = float(rng.uniform(0.5, 2.0))
    return slope, var, rng


# ----------------------------------------------------------------------------
# oct-based AMR input (periodic base level + nested refined levels)
# ----------------------------------------------------------------------------
def plummer_centres(n_clumps: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(n_clumps, 3))


def _periodic_trilinear(g: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Periodic trilinear interpolation of a cell-centred base-grid field at points."""
    n = g.shape[0]
    u = pts * n - 0.5
    i0 = np.floor(u).astype(np.int64)
    t = u - i0
    i0 %= n
    i1 = (i0 + 1) % n
    out = np.zeros(len(pts))
    for a in (0, 1):
        wx = t[:, 0] if a else 1.0 - t[:, 0]
        ix = i1[:, 0] if a else i0[:, 0]
        for b in (0, 1):
            wy = t[:, 1] if b else 1.0 - t[:, 1]
            iy = i1[:, 1] if b else i0[:, 1]
            for c in (0, 1):
                wz = t[:, 2] if c else 1.0 - t[:, 2]
                iz = i1[:, 2] if c else i0[:, 2]
                out += wx * wy * wz * g[ix, iy, iz]
    return out


def _plummer_sum(pts: np.ndarray, centres: np.ndarray, amp: float, a: float,
                 chunk: int = 1 << 20) -> np.ndarray:
    """Sum over clumps of amp * (1 + r^2/a^2)^(-5/2), periodic minimum-image r."""
    out = np.zeros(len(pts))
    inv_a2 = 1.0 / (a * a)
    for s in range(0, len(pts), chunk):
        p = pts[s:s + chunk]
        acc = np.zeros(len(p))
        for c in centres:
            d = p - c
            d -= np.round(d)
            q = 1.0 + np.einsum("ij,ij->i", d, d) * inv_a2
            acc += 1.0 / (q * q * np.sqrt(q))
        out[s:s + chunk] = amp * acc
    return out


def brick_order(ijk: np.ndarray, n_oct_dim: int) -> np.ndarray:
    """Permutation that lists octs brick by brick (4x4x4-oct bricks, bricks and
    octs inside a brick lexicographic, x fastest), for memory locality."""
    ijk = ijk.astype(np.int64)
    nb = max(n_oct_dim // 4, 1)
    b = ijk >> 2
    r = ijk & 3
    key = ((b[:, 2] * nb + b[:, 1]) * nb + b[:, 0]) * 64 + (r[:, 2] * 16 + r[:, 1] * 4 + r[:, 0])
    return np.argsort(key, kind="stable")


@dataclass
class AmrLevel:
    level: int                     # 0 = periodic base level
    n_cells_dim: int               # cells per dimension of the level's full extent
    oct_ijk: np.ndarray | None     # [n_oct, 3] int32 oct coordinates (None on the base level)
    rho: np.ndarray                # base: dense [n,n,n]; refined: [n_oct, 8] oct-major

    @property
    def n_oct(self) -> int:
        return (self.n_cells_dim // 2) ** 3 if self.oct_ijk is None else len(self.oct_ijk)

    @property
    def n_cells(self) -> int:
        return 8 * self.n_oct


@dataclass
class AmrInput:
    base_n: int
    rho_mean: float
    levels: list = field(default_factory=list)


_OFFS27 = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)],
                   dtype=np.int64)


def _lin(c: np.ndarray, n: int) -> np.ndarray:
    c = c.astype(np.int64) % n
    return (c[:, 2] * n + c[:, 1]) * n + c[:, 0]


def _in_sorted(sorted_keys: np.ndarray, q: np.ndarray) -> np.ndarray:
    pos = np.searchsorted(sorted_keys, q)
    pos = np.minimum(pos, len(sorted_keys) - 1)
    return sorted_keys[pos] == q


def build_amr_input(base_n: int = 128, n_refined: int = 3, grf_seed: int = 3,
                    clump_seed: int = 1003, n_clumps: int = 64, slope: float = -2.5,
                    var: float = 1.5, scale_radius: float = 0.005, contrast: float = 1e4,
                    threshold: float = 8.0) -> AmrInput:
    """Periodic base grid plus ``n_refined`` nested levels refined on density.

    * rho(x) = exp(g~(x) - var/2) + sum_c A (1 + r_c^2/a^2)^(-5/2): g~ is the
      periodic trilinear interpolant of the base-grid Gaussian field (it equals
      the field at base-cell centres), r_c the periodic distance to clump c,
      a = ``scale_radius`` and A = ``contrast`` times the mean of the lognormal
      part over base cells.  Clump centres are uniform in the box.
    * rho_mean is the mean of rho over base cells (clumps included, as sampled).
    * On every level a cell is flagged when rho at its centre exceeds
      ``threshold * rho_mean``; flags are dilated by one cell (26-neighbourhood)
      among the level's cells, and a flag is dropped unless its whole
      26-neighbourhood exists on the level (proper nesting, so that every ghost
      of the next level finds a full coarse interpolation stencil).  Each kept
      flag becomes one oct of the next level; octs are listed in brick order.
    """
    g = gaussian_random_field(base_n, slope, var, seed=grf_seed)
    rho_ln = np.exp(g - 0.5 * var)
    centres = plummer_centres(n_clumps, clump_seed)
    amp = contrast * float(rho_ln.mean())
    x = cell_centres_1d(base_n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    del X, Y, Z
    rho0 = (rho_ln.ravel() + _plummer_sum(pts, centres, amp, scale_radius)).reshape(base_n, base_n, base_n)
    rho_mean = float(rho0.mean())
    out = AmrInput(base_n=base_n, rho_mean=rho_mean)
    out.levels.append(AmrLevel(0, base_n, None, rho0))

    def density(points: np.ndarray) -> np.ndarray:
        return np.exp(_periodic_trilinear(g, points) - 0.5 * var) + \
            _plummer_sum(points, centres, amp, scale_radius)

    # cells of level 0 as integer coordinates and their densities
    ii = np.arange(base_n, dtype=np.int64)
    I, J, K = np.meshgrid(ii, ii, ii, indexing="ij")
    cells = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    rho_cells = rho0.ravel()
    del I, J, K
    n = base_n
    for lev in range(n_refined):
        keys = _lin(cells, n)
        order = np.argsort(keys)
        skeys = keys[order]
        flagged = cells[rho_cells > threshold * rho_mean]
        if len(flagged) == 0:
            break
        # dilate by one cell among the cells that exist on this level
        cand = (flagged[:, None, :] + _OFFS27[None, :, :]).reshape(-1, 3) % n
        ck = np.unique(_lin(cand, n))
        ck = ck[_in_sorted(skeys, ck)]
        # proper nesting: keep flags whose 26 neighbours all exist
        fc = np.stack([ck % n, (ck // n) % n, ck // (n * n)], axis=1)
        ok = np.ones(len(fc), dtype=bool)
        for o in _OFFS27:
            ok &= _in_sorted(skeys, _lin(fc + o, n))
        fc = fc[ok]
        if len(fc) == 0:
            break
        n *= 2
        fc = fc[brick_order(fc, n // 2)]
        oct_ijk = fc.astype(np.int32)
        # cells of the new level, oct-major, c = cx + 2cy + 4cz
        sub = np.array([(c & 1, (c >> 1) & 1, (c >> 2) & 1) for c in range(8)], dtype=np.int64)
        cells = (2 * fc[:, None, :] + sub[None, :, :]).reshape(-1, 3)
        pts = (cells + 0.5) / n
        rho_cells = density(pts)
        out.levels.append(AmrLevel(lev + 1, n, oct_ijk, rho_cells.reshape(-1, 8)))
    return out
