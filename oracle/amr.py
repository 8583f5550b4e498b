"""Oracle for the Poisson solve on a refined (Dirichlet) level of an oct-based mesh.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs the multigrid V-cycle "at each AMR level" (section
"Multi-Grid Method"); a refined level's boundary values come from the
next-coarser level, and the trilinear interpolation stencil reads
neighbouring coarse cells (subsection "V-cycle algorithm and exchange
optimization").  The paper gives no ghost formula; the reading used here:

* the unknowns are the cells of the level's octs; cell (i, j, k) has spacing
  h = 1/n with n = base_n * 2^level cells per dimension over the unit box;
* a face neighbour is the level cell at (i, j, k) +- e_d, wrapped modulo n,
  when its oct exists; otherwise it is a ghost whose value is the trilinear
  (cell-centred) interpolation of the coarse potential: the ghost's coarse
  parent P = g >> 1 and, per axis, the coarse neighbour on the ghost's side
  (s_d = +1 if g_d is odd, else -1), with per-axis weights 3/4 and 1/4;
* the same equation (sum of neighbours - 6 phi_c)/h^2 = f_c holds on every
  cell, with ghosts entering as known values.  -L is then symmetric positive
  definite, so the solution is unique.

The multigrid hierarchy below a refined level (the paper only says that a
coarse cell is the average of its eight children): coarse level m+1 holds the
father cells of level m's octs, grouped in their octs.  Each cell carries a
level-set mask: +1 on every cell of the refined level; a father cell takes the
mean of its 8 children's masks, every other coarse cell -1.  Cells with a
positive mask are the unknowns of the coarse error equation; the others hold
0.  For an active cell c and an inactive or absent neighbour j the error is
taken to vanish where the mask interpolates to zero between the two centres,
at fraction theta = m_c / (m_c - m_j) (clamped to [0.1, 1]); extrapolating e
linearly through that zero gives e_j = e_c (1 - 1/theta), so c's diagonal is
-(6 + sum_j (1/theta_j - 1))/H^2.  With masks +-1 the zero lies on the shared
face.  The restriction is the mean of the 8 children's residuals; the
prolongation is trilinear with inactive or absent coarse cells counting as 0.
This hierarchy affects only the speed of convergence, not the converged
solution, which the fine-level equations fix.  (Counting inactive neighbours
as 0 one coarse cell away instead made the V-cycle diverge on the full-size
nested workload.)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .morton import DIRS

SUB = np.array([(c & 1, (c >> 1) & 1, (c >> 2) & 1) for c in range(8)], dtype=np.int64)

__all__ = ["SUB", "CellSet", "DirichletLevel", "NestingError", "OctMGLevel", "coarsen", "coarse_mask",
           "build_hierarchy", "restrict_fathers", "prolong_masked", "refined_hierarchy", "refined_vcycle",
           "refined_mg_solve"]


class NestingError(ValueError):
    """A ghost's coarse interpolation stencil is not fully present."""


class CellSet:
    """The cells of one level and a coordinate -> flat index lookup.

    A full periodic level (``oct_ijk is None``) stores values as a dense
    [n, n, n] array with flat index (i n + j) n + k; an oct level stores
    [n_oct, 8] with flat index 8 oct + c, c = cx + 2 cy + 4 cz.  Lookups wrap
    coordinates modulo n and linearise them inside the set's bounding box
    (widened by one cell on each side), so deep levels whose extent n has no
    int64 cube still index exactly; a set that is small but straddles the
    periodic boundary would need a box as wide as the level.
    """

    def __init__(self, n: int, oct_ijk: np.ndarray | None = None):
        self.n = int(n)
        if oct_ijk is None:
            ii = np.arange(n, dtype=np.int64)
            I, J, K = np.meshgrid(ii, ii, ii, indexing="ij")
            self.coords = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
            self.oct_ijk = None
        else:
            self.oct_ijk = np.asarray(oct_ijk, dtype=np.int64)
            self.coords = (2 * self.oct_ijk[:, None, :] + SUB[None, :, :]).reshape(-1, 3)
        wrapped = self.coords % self.n
        self._lo = wrapped.min(axis=0) - 1
        self._ext = wrapped.max(axis=0) - self._lo + 2
        keys = self._lin(self.coords)
        self._order = np.argsort(keys, kind="stable")
        self._sorted = keys[self._order]

    def _lin(self, c: np.ndarray) -> np.ndarray:
        """Box-linear key of each wrapped coordinate, -1 outside the box."""
        r = np.asarray(c, dtype=np.int64) % self.n - self._lo
        inside = np.all((r >= 0) & (r < self._ext), axis=1)
        k = (r[:, 2] * self._ext[1] + r[:, 1]) * self._ext[0] + r[:, 0]
        return np.where(inside, k, -1)

    def __len__(self) -> int:
        return len(self.coords)

    def index(self, q: np.ndarray) -> np.ndarray:
        """Flat index of each queried cell coordinate (wrapped mod n), -1 if absent."""
        k = self._lin(q)
        pos = np.minimum(np.searchsorted(self._sorted, k), len(self._sorted) - 1)
        hit = self._sorted[pos] == k
        out = np.full(len(k), -1, dtype=np.int64)
        out[hit] = self._order[pos[hit]]
        return out


def _ghost_stencils(ghost_cells: np.ndarray, parent: CellSet) -> tuple[np.ndarray, np.ndarray]:
    """For each ghost cell coordinate: the 8 coarse flat indices and trilinear weights."""
    P = ghost_cells >> 1
    s = np.where(ghost_cells & 1, 1, -1)
    idx = np.empty((len(ghost_cells), 8), dtype=np.int64)
    w = np.empty((len(ghost_cells), 8))
    k = 0
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                off = np.stack([a * s[:, 0], b * s[:, 1], c * s[:, 2]], axis=1)
                idx[:, k] = parent.index(P + off)
                w[:, k] = (0.25 if a else 0.75) * (0.25 if b else 0.75) * (0.25 if c else 0.75)
                k += 1
    if np.any(idx < 0):
        raise NestingError("coarse interpolation stencil of a ghost is not present")
    return idx, w


class DirichletLevel:
    """A refined level: cells of ``oct_ijk`` at ``n`` cells/dim, ghosts from ``parent``."""

    def __init__(self, n: int, oct_ijk: np.ndarray, parent: CellSet):
        self.n = int(n)
        self.h = 1.0 / n
        self.cells = CellSet(n, oct_ijk)
        self.parent = parent
        c = self.cells.coords
        self.nbr = np.stack([self.cells.index(c + DIRS[j]) for j in range(6)], axis=1)
        gc, gj = np.nonzero(self.nbr < 0)
        self.ghost_cell = gc                      # which cell the ghost face belongs to
        self.ghost_dir = gj
        self.ghost_coords = (c[gc] + DIRS[gj]) % n
        self.ghost_idx, self.ghost_w = _ghost_stencils(self.ghost_coords, parent)

    @property
    def n_cells(self) -> int:
        return len(self.cells)

    def ghost_values(self, phi_parent: np.ndarray) -> np.ndarray:
        """Trilinear ghost values from the coarse potential (flat, parent's layout)."""
        pp = np.asarray(phi_parent, dtype=np.float64).ravel()
        return np.sum(pp[self.ghost_idx] * self.ghost_w, axis=1)

    def ghost_sum(self, phi_parent: np.ndarray) -> np.ndarray:
        """Per cell: the sum of its ghost neighbour values."""
        G = np.zeros(self.n_cells)
        np.add.at(G, self.ghost_cell, self.ghost_values(phi_parent))
        return G

    def neighbour_sum(self, phi: np.ndarray, phi_parent: np.ndarray) -> np.ndarray:
        p = np.asarray(phi, dtype=np.float64).ravel()
        s = self.ghost_sum(phi_parent)
        for j in range(6):
            m = self.nbr[:, j] >= 0
            s[m] += p[self.nbr[m, j]]
        return s

    def apply(self, phi: np.ndarray, phi_parent: np.ndarray) -> np.ndarray:
        p = np.asarray(phi, dtype=np.float64).ravel()
        return (self.neighbour_sum(p, phi_parent) - 6.0 * p) / (self.h * self.h)

    def neighbour_values(self, phi: np.ndarray, phi_parent: np.ndarray) -> np.ndarray:
        """[n_cells, 6] value of each face neighbour (directions -x, +x, -y, +y,
        -z, +z): the level cell when its oct exists, else the ghost value."""
        p = np.asarray(phi, dtype=np.float64).ravel()
        V = np.empty((self.n_cells, 6))
        for j in range(6):
            m = self.nbr[:, j] >= 0
            V[m, j] = p[self.nbr[m, j]]
        V[self.ghost_cell, self.ghost_dir] = self.ghost_values(phi_parent)
        return V

    def force(self, phi: np.ndarray, phi_parent: np.ndarray) -> np.ndarray:
        """g = -grad(phi) by central differences, [3, n_oct, 8]; a neighbour
        outside the level is its ghost, the same trilinear value the solve
        uses (the reading of the periodic oracle's ``force``)."""
        V = self.neighbour_values(phi, phi_parent)
        g = np.stack([-(V[:, 2 * d + 1] - V[:, 2 * d]) / (2.0 * self.h) for d in range(3)])
        return g.reshape(3, -1, 8)

    def residual(self, phi, f, phi_parent) -> np.ndarray:
        return np.asarray(f, dtype=np.float64).ravel() - self.apply(phi, phi_parent)

    def rhs(self, f, phi_parent) -> np.ndarray:
        """Right-hand side of the level's linear system A phi = b once the known
        ghost values are moved across: b = f - (sum of ghost neighbours) / h^2.
        It is the residual of the zero potential."""
        return np.asarray(f, dtype=np.float64).ravel() - self.ghost_sum(phi_parent) / (self.h * self.h)

    def rhs_norm(self, f, phi_parent) -> float:
        return float(np.linalg.norm(self.rhs(f, phi_parent)))

    def relres(self, phi, f, phi_parent) -> float:
        """||f - L_h phi|| / ||b||: the residual relative to the system's full
        right-hand side (f with the Dirichlet terms), so a zero guess has
        relres 1 and a level whose only source is its boundary is measured on
        the scale of that boundary."""
        r = self.residual(phi, f, phi_parent)
        return float(np.linalg.norm(r) / self.rhs_norm(f, phi_parent))

    def matrix(self) -> sp.csr_matrix:
        """Sparse matrix of L restricted to the unknowns (ghost terms excluded)."""
        N = self.n_cells
        rows, cols = [], []
        for j in range(6):
            m = self.nbr[:, j] >= 0
            rows.append(np.nonzero(m)[0])
            cols.append(self.nbr[m, j])
        r = np.concatenate(rows + [np.arange(N)])
        c = np.concatenate(cols + [np.arange(N)])
        v = np.concatenate([np.ones(sum(len(x) for x in rows)), np.full(N, -6.0)])
        return sp.csr_matrix((v, (r, c)), shape=(N, N)) / (self.h * self.h)

    def solve(self, f: np.ndarray, phi_parent: np.ndarray, rtol: float = 1e-14) -> np.ndarray:
        """Exact solution (direct below 30k unknowns, else CG on the SPD system -L)."""
        A = self.matrix()
        b = self.rhs(f, phi_parent)
        if self.n_cells <= 30000:
            x = spla.spsolve(A.tocsc(), b)
        else:
            x, info = spla.cg(-A, -b, rtol=rtol, atol=0.0, maxiter=100000)
            if info != 0:
                raise RuntimeError(f"CG did not converge (info={info})")
        return x.reshape(-1, 8)

    # -- red-black Gauss-Seidel on the level (inhomogeneous Dirichlet ghosts) --
    def colour(self) -> np.ndarray:
        return self.cells.coords.sum(axis=1) % 2

    def gs_half_sweep(self, phi: np.ndarray, f: np.ndarray, phi_parent: np.ndarray, colour: int) -> None:
        """In place on phi ([n_oct, 8]): update every cell of one colour."""
        p = phi.reshape(-1)
        new = (self.neighbour_sum(p, phi_parent) - self.h * self.h * np.asarray(f).ravel()) / 6.0
        m = self.colour() == colour
        p[m] = new[m]


# ---------------------------------------------------------------------------
# masked father-cell hierarchy
# ---------------------------------------------------------------------------
class OctMGLevel:
    """One multigrid level made of octs with a level-set mask ``lsm`` [n_oct, 8].

    ``active`` = lsm > 0; ``nbr[cell, j]`` is the flat index of an active
    neighbour cell or -1; ``diag[cell]`` is 6 + sum over inactive/absent
    neighbours of (1/theta - 1).
    """

    THETA_MIN = 0.1

    def __init__(self, n: int, oct_ijk: np.ndarray, lsm: np.ndarray):
        self.n = int(n)
        self.h = 1.0 / n
        self.cells = CellSet(n, oct_ijk)
        self.oct_ijk = self.cells.oct_ijk
        self.lsm = np.asarray(lsm, dtype=np.float64).reshape(-1)
        self.active = self.lsm > 0
        c = self.cells.coords
        raw = np.stack([self.cells.index(c + DIRS[j]) for j in range(6)], axis=1)
        mj = np.where(raw >= 0, self.lsm[np.maximum(raw, 0)], -1.0)
        self.nbr = np.where((raw >= 0) & (mj > 0), raw, -1)
        mc = self.lsm[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            theta = np.clip(mc / (mc - mj), self.THETA_MIN, 1.0)
        extra = np.where(mj > 0, 0.0, 1.0 / theta - 1.0).sum(axis=1)
        self.diag = np.where(self.active, 6.0 + extra, 6.0)

    @property
    def n_active(self) -> int:
        return int(self.active.sum())

    def neighbour_sum(self, e: np.ndarray) -> np.ndarray:
        p = e.reshape(-1)
        s = np.zeros_like(p)
        for j in range(6):
            m = self.nbr[:, j] >= 0
            s[m] += p[self.nbr[m, j]]
        return s

    def apply(self, e: np.ndarray) -> np.ndarray:
        p = e.reshape(-1)
        out = (self.neighbour_sum(p) - self.diag * p) / (self.h * self.h)
        return np.where(self.active, out, 0.0)

    def residual(self, e: np.ndarray, b: np.ndarray) -> np.ndarray:
        return np.where(self.active, b.reshape(-1) - self.apply(e), 0.0)

    def gs_half_sweep(self, e: np.ndarray, b: np.ndarray, colour: int) -> None:
        p = e.reshape(-1)
        new = (self.neighbour_sum(p) - self.h * self.h * b.reshape(-1)) / self.diag
        m = self.active & (self.cells.coords.sum(axis=1) % 2 == colour)
        p[m] = new[m]


def coarsen(oct_ijk: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Father-cell coarsening: (coarse oct coords, flat father cell index per fine oct).

    The father cell of fine oct (I, J, K) is coarse cell (I, J, K), which lies
    in coarse oct (I, J, K) >> 1 at child index from the parities.
    """
    f = np.asarray(oct_ijk, dtype=np.int64)
    co = f >> 1
    nd = int(co.max()) + 1 if len(co) else 1
    key = (co[:, 2] * nd + co[:, 1]) * nd + co[:, 0]
    ukey, inv = np.unique(key, return_inverse=True)
    coarse = np.stack([ukey % nd, (ukey // nd) % nd, ukey // (nd * nd)], axis=1)
    child = (f[:, 0] & 1) + 2 * (f[:, 1] & 1) + 4 * (f[:, 2] & 1)
    return coarse, inv * 8 + child


def coarse_mask(fine: OctMGLevel, father: np.ndarray, n_coarse_oct: int) -> np.ndarray:
    """-1 everywhere; each father cell = mean of its 8 children's masks."""
    out = np.full(n_coarse_oct * 8, -1.0)
    out[father] = fine.lsm.reshape(-1, 8).mean(axis=1)
    return out


def build_hierarchy(n: int, oct_ijk: np.ndarray, max_coarse_octs: int = 256):
    """Levels (finest first) and father maps: coarsen at least once, then until
    the coarsest level has at most ``max_coarse_octs`` octs (or one oct per dimension)."""
    lv = OctMGLevel(n, oct_ijk, np.ones(len(oct_ijk) * 8))
    levels, fathers = [lv], []
    while (len(levels) == 1 or len(lv.oct_ijk) > max_coarse_octs) and lv.n // 2 > 1:
        coarse, father = coarsen(lv.oct_ijk)
        nxt = OctMGLevel(lv.n // 2, coarse, coarse_mask(lv, father, len(coarse)))
        fathers.append(father)
        levels.append(nxt)
        lv = nxt
    return levels, fathers


def restrict_fathers(r_fine: np.ndarray, father: np.ndarray, n_coarse_oct: int) -> np.ndarray:
    """Coarse right-hand side: each father cell = mean of its 8 children's residuals."""
    out = np.zeros(n_coarse_oct * 8)
    out[father] = np.asarray(r_fine).reshape(-1, 8).mean(axis=1)
    return out.reshape(-1, 8)


def prolong_masked(fine: OctMGLevel, coarse: OctMGLevel, father: np.ndarray,
                   ec: np.ndarray) -> np.ndarray:
    """Trilinear correction for every fine cell; absent/masked coarse cells count as 0."""
    ecf = np.where(coarse.active, ec.reshape(-1), 0.0)
    fc = fine.cells.coords                 # fine cell coords
    P = fc >> 1                            # coarse cell containing each fine cell
    s = np.where(fc & 1, 1, -1)
    out = np.zeros(len(fc))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                off = np.stack([a * s[:, 0], b * s[:, 1], c * s[:, 2]], axis=1)
                idx = coarse.cells.index(P + off)
                w = (0.25 if a else 0.75) * (0.25 if b else 0.75) * (0.25 if c else 0.75)
                ok = idx >= 0
                out[ok] += w * ecf[idx[ok]]
    return out.reshape(-1, 8)


# ---------------------------------------------------------------------------
# V-cycle on a refined level (Alg "GPU-accelerated V-cycle at AMR level l")
# ---------------------------------------------------------------------------
def refined_hierarchy(dlev: DirichletLevel, max_coarse_octs: int = 256):
    """The father-cell hierarchy under a refined level as its V-cycle uses it:
    (levels, fathers, smooth_only).  Built as in :func:`build_hierarchy`; a
    coarse level without active cells carries no unknowns, so the hierarchy
    ends above it and its new last level is relaxed with nu_pre + nu_post
    sweeps (``smooth_only``) instead of being solved (reading R18)."""
    levels, fathers = build_hierarchy(dlev.n, dlev.cells.oct_ijk, max_coarse_octs)
    for m in range(1, len(levels)):
        if levels[m].n_active == 0:
            return levels[:m], fathers[:m - 1], True
    return levels, fathers, False


def refined_vcycle(dlev: DirichletLevel, hier, phi: np.ndarray, f: np.ndarray, phi_parent: np.ndarray,
                   nu_pre: int = 2, nu_post: int = 2, coarse_sweeps: int = 64) -> None:
    """One V-cycle on a refined level, in place on phi ([n_oct, 8]).

    Steps in the algorithm's order: nu_pre red-black sweeps of the level
    (Dirichlet ghosts from phi_parent), residual, restriction to the father
    cells (mean of the 8 children), the coarse error equations solved by the
    same cycle from a zero guess on each masked level below, trilinear
    prolongation + correction, nu_post sweeps.  The last level is relaxed
    from zero: nu_pre + nu_post sweeps when the hierarchy was cut, otherwise
    ``coarse_sweeps`` sweeps (its approximate solve, reading R7)."""
    levels, fathers, smooth_only = hier
    n_last = len(levels) - 1

    def sweeps(k, one_half):
        for _ in range(k):
            one_half(0)
            one_half(1)

    def coarse(m: int, b: np.ndarray) -> np.ndarray:
        lv = levels[m]
        e = np.zeros(len(lv.cells))
        if m == n_last:
            sweeps(nu_pre + nu_post if smooth_only else coarse_sweeps, lambda c: lv.gs_half_sweep(e, b, c))
            return e
        sweeps(nu_pre, lambda c: lv.gs_half_sweep(e, b, c))
        bc = restrict_fathers(lv.residual(e, b), fathers[m], len(levels[m + 1].oct_ijk))
        ec = coarse(m + 1, bc.ravel())
        e += prolong_masked(lv, levels[m + 1], fathers[m], ec).ravel()
        sweeps(nu_post, lambda c: lv.gs_half_sweep(e, b, c))
        return e

    if n_last == 0:   # no coarse level with unknowns: the cycle is its sweeps
        sweeps(nu_pre + nu_post, lambda c: dlev.gs_half_sweep(phi, f, phi_parent, c))
        return
    sweeps(nu_pre, lambda c: dlev.gs_half_sweep(phi, f, phi_parent, c))
    bc = restrict_fathers(dlev.residual(phi, f, phi_parent), fathers[0], len(levels[1].oct_ijk))
    ec = coarse(1, bc.ravel())
    phi += prolong_masked(levels[0], levels[1], fathers[0], ec)
    sweeps(nu_post, lambda c: dlev.gs_half_sweep(phi, f, phi_parent, c))


def refined_mg_solve(dlev: DirichletLevel, f: np.ndarray, phi_parent: np.ndarray, tol: float = 1e-10,
                     max_cycles: int = 50, nu_pre: int = 2, nu_post: int = 2, coarse_sweeps: int = 64,
                     max_coarse_octs: int = 256):
    """V-cycles from phi = 0 until ||f - L phi|| / ||b|| <= tol (b the full
    right-hand side, :meth:`DirichletLevel.relres`).  Returns (phi, history)
    with history[i] the relative residual after i cycles."""
    hier = refined_hierarchy(dlev, max_coarse_octs)
    phi = np.zeros((dlev.n_cells // 8, 8))
    hist = [dlev.relres(phi, f, phi_parent)]
    for _ in range(max_cycles):
        if hist[-1] <= tol:
            break
        refined_vcycle(dlev, hier, phi, f, phi_parent, nu_pre, nu_post, coarse_sweeps)
        hist.append(dlev.relres(phi, f, phi_parent))
    return phi, hist
