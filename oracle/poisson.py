"""Oracle for the multigrid Poisson solve on a periodic level (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
uses this module.

What is computed (paper, section "Poisson solver optimizations", subsection
"Multi-Grid Method"; appendix "Multigrid solver implementation details";
algorithm "GPU-accelerated V-cycle at AMR level l"):

* the discrete problem: (L_h phi)_c = (sum of the 6 face neighbours - 6 phi_c)/h^2
  = f_c with f = 4 pi G (rho - rho_mean) on a periodic n^3 grid, gauge
  mean(phi) = 0.  The paper writes the source without the mean; on a periodic
  box the mean must be removed for a solution to exist.
* the exact solution of that system by an FFT with the discrete eigenvalues
  of L_h (the plain definition of the result the iteration converges to);
* the V-cycle of the correction scheme: red-black Gauss-Seidel pre-smoothing,
  residual, restriction by the mean of the 8 children, recursion, trilinear
  prolongation and correction, post-smoothing; a direct solve on the coarsest
  grid.
* the mixed-precision defect correction (FP32 V-cycles inside an FP64 outer
  loop), which the paper does not contain.

Arrays are dense [n, n, n] indexed (x, y, z); "red" cells have (i+j+k) even and
are updated first.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rhs", "neighbour_sum", "apply_laplacian", "residual", "norm2", "relres",
    "fft_solve", "colour_mask", "gs_half_sweep", "gs_sweep", "restrict", "prolong",
    "laplacian_matrix", "coarse_solve", "vcycle", "mg_solve", "mg_solve_mixed",
    "project_mean", "maxdiff", "force",
]


# ---------------------------------------------------------------------------
# the discrete problem
# ---------------------------------------------------------------------------
def rhs(rho: np.ndarray, four_pi_G: float = 1.0, rho_mean: float | None = None) -> np.ndarray:
    """f = 4 pi G (rho - rho_mean); rho_mean defaults to the FP64 mean of rho."""
    if rho_mean is None:
        rho_mean = float(np.mean(rho, dtype=np.float64))
    return four_pi_G * (rho - rho_mean)


def neighbour_sum(phi: np.ndarray) -> np.ndarray:
    """Sum of the six face neighbours with periodic wrap."""
    s = np.zeros_like(phi)
    for ax in range(3):
        s += np.roll(phi, 1, axis=ax)
        s += np.roll(phi, -1, axis=ax)
    return s


def apply_laplacian(phi: np.ndarray, h: float) -> np.ndarray:
    """7-point discrete Laplacian, periodic."""
    return (neighbour_sum(phi) - 6.0 * phi) / (h * h)


def residual(phi: np.ndarray, f: np.ndarray, h: float) -> np.ndarray:
    """r = f - L_h phi (the fused residual of the MG appendix, without the fusion)."""
    return f - apply_laplacian(phi, h)


def norm2(a: np.ndarray) -> float:
    return float(np.sqrt(np.sum(np.asarray(a, dtype=np.float64) ** 2)))


def relres(phi: np.ndarray, f: np.ndarray, h: float) -> float:
    """||f - L_h phi||_2 / ||f||_2 (denominator ||f||, so warm starts are judged fairly)."""
    return norm2(residual(np.asarray(phi, np.float64), f, h)) / norm2(f)


def project_mean(phi: np.ndarray) -> np.ndarray:
    return phi - np.mean(phi, dtype=np.float64)


def maxdiff(phi: np.ndarray, ref: np.ndarray) -> float:
    """max|phi - ref| / max|ref| after removing each field's mean."""
    a = project_mean(np.asarray(phi, np.float64))
    b = project_mean(np.asarray(ref, np.float64))
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def force(phi: np.ndarray, h: float) -> np.ndarray:
    """Gravitational acceleration g = -grad(phi), [3, n, n, n] (components x, y, z).

    The paper lists the gravity force among the per-cell routines that follow
    the solve (section "GPU offloading: approach and assessment") without
    printing its stencil; the reading taken here is the second-order central
    difference that matches the 7-point operator:
    g_d(i) = -(phi(i + e_d) - phi(i - e_d)) / (2 h), periodic wrap.
    """
    p = np.asarray(phi, dtype=np.float64)
    return np.stack([-(np.roll(p, -1, axis=ax) - np.roll(p, 1, axis=ax)) / (2.0 * h) for ax in range(3)])


def fft_solve(f: np.ndarray, h: float) -> np.ndarray:
    """Exact mean-zero solution of L_h phi = f - mean(f) with the discrete eigenvalues.

    The periodic 7-point operator is diagonalised by the DFT; its eigenvalue at
    integer wave vector k is sum_d (2 cos(2 pi k_d / n) - 2) / h^2.  The k = 0
    component (the mean) is set to zero.
    """
    n = f.shape[0]
    fk = np.fft.fftn(f)
    lam1 = (2.0 * np.cos(2.0 * np.pi * np.arange(n) / n) - 2.0) / (h * h)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    lam[0, 0, 0] = 1.0
    pk = fk / lam
    pk[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(pk))


# ---------------------------------------------------------------------------
# red-black Gauss-Seidel (equation gs_update of the MG appendix)
# ---------------------------------------------------------------------------
def colour_mask(n: int, colour: int) -> np.ndarray:
    """True where (i + j + k) mod 2 == colour (0 = red, 1 = black)."""
    i = np.arange(n)
    par = (i[:, None, None] + i[None, :, None] + i[None, None, :]) % 2
    return par == colour


def gs_half_sweep(phi: np.ndarray, b: np.ndarray, h: float, colour: int) -> None:
    """In place: phi_c <- (sum_j phi_j - h^2 b_c) / 6 on every cell of one colour.

    With n even, every face neighbour of a cell has the other colour, so
    updating all cells of one colour from the same neighbour values is exactly
    the sequential Gauss-Seidel update of those cells.
    """
    dt = phi.dtype
    h2 = dt.type(h * h)
    new = (neighbour_sum(phi) - h2 * b) / dt.type(6.0)
    m = colour_mask(phi.shape[0], colour)
    phi[m] = new[m]


def gs_sweep(phi: np.ndarray, b: np.ndarray, h: float) -> None:
    """One red-black sweep: red cells first, then black."""
    gs_half_sweep(phi, b, h, 0)
    gs_half_sweep(phi, b, h, 1)


# ---------------------------------------------------------------------------
# transfer operators
# ---------------------------------------------------------------------------
def restrict(r: np.ndarray) -> np.ndarray:
    """Coarse cell = average of its 8 children (exact mean, no full weighting)."""
    n = r.shape[0]
    c = n // 2
    return r.reshape(c, 2, c, 2, c, 2).mean(axis=(1, 3, 5), dtype=r.dtype)


def _interp_axis(a: np.ndarray, ax: int) -> np.ndarray:
    """Cell-centred linear interpolation doubling one axis (periodic).

    Fine cell 2I takes 3/4 of coarse cell I and 1/4 of I-1; fine cell 2I+1
    takes 3/4 of I and 1/4 of I+1 (the neighbour on the child's side).
    """
    dt = a.dtype.type
    lo = dt(0.75) * a + dt(0.25) * np.roll(a, 1, axis=ax)
    hi = dt(0.75) * a + dt(0.25) * np.roll(a, -1, axis=ax)
    shape = list(a.shape)
    shape[ax] *= 2
    out = np.empty(shape, dtype=a.dtype)
    sl_lo = [slice(None)] * 3
    sl_hi = [slice(None)] * 3
    sl_lo[ax] = slice(0, None, 2)
    sl_hi[ax] = slice(1, None, 2)
    out[tuple(sl_lo)] = lo
    out[tuple(sl_hi)] = hi
    return out


def prolong(ec: np.ndarray) -> np.ndarray:
    """Trilinear (cell-centred) interpolation of a coarse correction to the fine grid.

    Applying the 1-D operator along each axis gives the product weights
    27/64 (parent), 9/64 (the 3 face neighbours toward the child), 3/64 (the 3
    edge neighbours) and 1/64 (the corner).
    """
    out = ec
    for ax in range(3):
        out = _interp_axis(out, ax)
    return out


# ---------------------------------------------------------------------------
# coarsest-grid direct solve
# ---------------------------------------------------------------------------
def laplacian_matrix(n: int, h: float) -> np.ndarray:
    """Dense matrix of the periodic 7-point operator on n^3 cells (C-order ravel)."""
    N = n ** 3
    A = np.zeros((N, N))
    idx = np.arange(N).reshape(n, n, n)
    for ax in range(3):
        for s in (1, -1):
            nb = np.roll(idx, s, axis=ax).ravel()
            A[np.arange(N), nb] += 1.0
    A[np.arange(N), np.arange(N)] -= 6.0
    return A / (h * h)


_PINV_CACHE: dict = {}


def coarse_solve(b: np.ndarray, h: float) -> np.ndarray:
    """Minimum-norm (mean-zero) exact solve on the coarsest grid: phi = A^+ b."""
    n = b.shape[0]
    key = (n, h, b.dtype.str)
    if key not in _PINV_CACHE:
        _PINV_CACHE[key] = np.linalg.pinv(laplacian_matrix(n, h)).astype(b.dtype)
    return (_PINV_CACHE[key] @ b.ravel()).reshape(b.shape)


# ---------------------------------------------------------------------------
# V-cycle and the outer iteration
# ---------------------------------------------------------------------------
def vcycle(e: np.ndarray, b: np.ndarray, h: float, nu_pre: int = 2, nu_post: int = 2,
           coarsest: int = 4, project: bool = True) -> None:
    """One V-cycle of the correction scheme on L_h e = b, in place on e.

    Steps in the paper's order: nu_pre red-black sweeps, residual, restriction,
    recursive V-cycle on the coarse error equation from a zero guess,
    prolongation + correction, nu_post red-black sweeps.  The coarse operator is
    the same 7-point stencil re-discretised with spacing 2h.  On the coarsest
    grid the system is solved exactly.  ``project`` removes the mean of each
    restricted right-hand side (periodic compatibility).
    """
    n = e.shape[0]
    if n <= coarsest:
        e[...] = coarse_solve(b - np.mean(b, dtype=np.float64).astype(b.dtype) if project else b, h)
        return
    for _ in range(nu_pre):
        gs_sweep(e, b, h)
    bc = restrict(residual(e, b, h))
    if project:
        bc = bc - np.mean(bc, dtype=np.float64).astype(bc.dtype)
    ec = np.zeros_like(bc)
    vcycle(ec, bc, 2.0 * h, nu_pre, nu_post, coarsest, project)
    e += prolong(ec)
    for _ in range(nu_post):
        gs_sweep(e, b, h)


def mg_solve(f: np.ndarray, h: float, tol: float = 1e-10, max_cycles: int = 50,
             phi0: np.ndarray | None = None, nu_pre: int = 2, nu_post: int = 2,
             coarsest: int = 4):
    """Plain FP64 multigrid: repeat V-cycles until ||f - L phi|| / ||f|| <= tol.

    Returns (phi, history) where history[i] is the relative residual after i
    cycles (history[0] is that of the initial guess).  phi is mean-zero.
    """
    phi = np.zeros_like(f) if phi0 is None else np.array(phi0, dtype=np.float64)
    fn = norm2(f)
    hist = [norm2(residual(phi, f, h)) / fn]
    for _ in range(max_cycles):
        if hist[-1] <= tol:
            break
        vcycle(phi, f, h, nu_pre, nu_post, coarsest)
        phi = project_mean(phi)
        hist.append(norm2(residual(phi, f, h)) / fn)
    return phi, hist


def mg_solve_mixed(f: np.ndarray, h: float, tol: float = 1e-10, max_outer: int = 50,
                   phi0: np.ndarray | None = None, nu_pre: int = 2, nu_post: int = 2,
                   coarsest: int = 4):
    """FP32 V-cycles inside an FP64 defect-correction loop.

    Each outer step: r = f - L_h phi in FP64 (mean removed); r32 = r rounded to
    float32 (round to nearest even); one float32 V-cycle on L_h e = r32 from
    e = 0 (all inner arithmetic in float32); phi += e in FP64; remove the mean
    of phi in FP64.  Returns (phi, history) like :func:`mg_solve`.
    """
    phi = np.zeros_like(f) if phi0 is None else np.array(phi0, dtype=np.float64)
    fn = norm2(f)
    r = residual(phi, f, h)
    hist = [norm2(r) / fn]
    for _ in range(max_outer):
        if hist[-1] <= tol:
            break
        r32 = project_mean(r).astype(np.float32)
        e = np.zeros_like(r32)
        vcycle(e, r32, h, nu_pre, nu_post, coarsest)
        phi = project_mean(phi + e.astype(np.float64))
        r = residual(phi, f, h)
        hist.append(norm2(r) / fn)
    return phi, hist
