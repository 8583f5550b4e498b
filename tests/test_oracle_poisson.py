"""Pins for the periodic-level oracle, each against something other than itself:
closed forms, the dense Gauss-Seidel substitution, exact invariants and
library routines (FFT, pseudo-inverse)."""
import json
import os

import numpy as np
import pytest

from oracle import poisson as P
from workloads import lognormal_density, sinusoid_density

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sss(n):
    x = (np.arange(n) + 0.5) / n
    s = np.sin(2 * np.pi * x)
    return s[:, None, None] * s[None, :, None] * s[None, None, :]


def test_laplacian_on_discrete_eigenvector():
    # s = sin sin sin at cell centres is an eigenvector of the periodic 7-point
    # operator with eigenvalue -12 sin^2(pi h) / h^2 (product of 1-D eigenvectors).
    for n in (8, 16, 32):
        h = 1.0 / n
        lam = -12.0 * np.sin(np.pi * h) ** 2 / h ** 2
        s = sss(n)
        assert np.max(np.abs(P.apply_laplacian(s, h) - lam * s)) < 1e-9 * abs(lam)


def test_laplacian_matches_dense_matrix_built_independently():
    # matrix assembled from the index rolls vs a loop over cells and offsets
    n, h = 4, 0.25
    A = P.laplacian_matrix(n, h)
    B = np.zeros_like(A)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                r = (i * n + j) * n + k
                B[r, r] = -6.0
                for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    c = (((i + d[0]) % n) * n + (j + d[1]) % n) * n + (k + d[2]) % n
                    B[r, c] += 1.0
    np.testing.assert_array_equal(A, B / h ** 2)


def test_fft_solve_closed_form_c1():
    # C1: rho = 1 + 0.5 s, 4 pi G = 1 -> f = 0.5 s; phi = 0.5 / lambda_h * s
    n, h = 32, 1.0 / 32
    f = P.rhs(sinusoid_density(n), 1.0)
    phi = P.fft_solve(f, h)
    lam = -12.0 * np.sin(np.pi * h) ** 2 / h ** 2
    assert abs(0.5 / lam - (-0.0042353055387)) < 1e-12
    np.testing.assert_allclose(phi, 0.5 / lam * sss(n), atol=1e-16, rtol=0)


def test_paper_microbenchmark_second_order():
    g = json.load(open(os.path.join(GOLDEN, "paper_poisson_microbenchmark.json")))
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        f = g["f_amplitude"] * sss(n)
        phi, hist = P.mg_solve(f, h, tol=1e-12)
        assert hist[-1] <= 1e-12
        cont = g["phi_amplitude_continuous"] * sss(n)
        errs.append(np.max(np.abs(phi - cont)))
    # O(h^2) truncation: halving h divides the error by ~4
    assert 3.8 < errs[0] / errs[1] < 4.2
    assert errs[1] < 4e-3


def test_fft_solve_random_field_satisfies_equation():
    n, h = 16, 1.0 / 16
    f = np.random.default_rng(0).standard_normal((n, n, n))
    phi = P.fft_solve(f, h)
    assert abs(phi.mean()) < 1e-14
    np.testing.assert_allclose(P.apply_laplacian(phi, h), f - f.mean(), atol=1e-10, rtol=0)


def test_coarse_pinv_equals_fft_on_4cubed():
    h = 0.25
    b = np.random.default_rng(1).standard_normal((4, 4, 4))
    b -= b.mean()
    np.testing.assert_allclose(P.coarse_solve(b, h), P.fft_solve(b, h), atol=1e-13, rtol=0)


def test_gs_half_sweeps_equal_sequential_substitution():
    # Dense Gauss-Seidel row by row: all red rows in index order, then all black rows.
    n, h = 4, 0.25
    rng = np.random.default_rng(2)
    phi0 = rng.standard_normal((n, n, n))
    b = rng.standard_normal((n, n, n))
    A = P.laplacian_matrix(n, h)
    x = phi0.ravel().copy()
    bb = b.ravel()
    col = np.add.reduce(np.indices((n, n, n)), axis=0).ravel() % 2
    for colour in (0, 1):
        for i in np.nonzero(col == colour)[0]:
            x[i] = (bb[i] - (A[i] @ x - A[i, i] * x[i])) / A[i, i]
    phi = phi0.copy()
    P.gs_sweep(phi, b, h)
    np.testing.assert_allclose(phi.ravel(), x, rtol=1e-13, atol=1e-13)


def test_restriction_and_prolongation_invariants():
    rng = np.random.default_rng(3)
    r = rng.standard_normal((8, 8, 8))
    rc = P.restrict(r)
    assert rc.shape == (4, 4, 4)
    assert abs(rc.sum() * 8 - r.sum()) < 1e-12
    assert abs(rc[1, 2, 3] - r[2:4, 4:6, 6:8].mean()) < 1e-15
    # prolongation reproduces constants exactly
    np.testing.assert_array_equal(P.prolong(np.full((4, 4, 4), 2.5)), np.full((8, 8, 8), 2.5))
    # ... and linear functions away from the periodic wrap
    X = np.arange(4)[:, None, None] + 0.5
    Y = np.arange(4)[None, :, None] + 0.5
    Z = np.arange(4)[None, None, :] + 0.5
    lin = 1.0 + 2.0 * X - 3.0 * Y + 0.5 * Z + 0 * X * Y * Z
    fine = P.prolong(lin)
    xf = (np.arange(8)[:, None, None] + 0.5) / 2
    yf = (np.arange(8)[None, :, None] + 0.5) / 2
    zf = (np.arange(8)[None, None, :] + 0.5) / 2
    exact = 1.0 + 2.0 * xf - 3.0 * yf + 0.5 * zf
    np.testing.assert_allclose(fine[1:-1, 1:-1, 1:-1], exact[1:-1, 1:-1, 1:-1], atol=1e-13)
    # the weights of one fine cell: 27/64 parent, 9/64 face, 3/64 edge, 1/64 corner
    ec = np.zeros((4, 4, 4))
    ec[2, 2, 2] = 64.0
    f = P.prolong(ec)
    assert f[4, 4, 4] == 27 and f[3, 4, 4] == 9 and f[3, 3, 4] == 3 and f[3, 3, 3] == 1
    assert f[2, 4, 4] == 0


@pytest.mark.parametrize("n,seed", [(32, 2), (64, 5)])
def test_mg_equals_fft_and_converges(n, seed):
    h = 1.0 / n
    f = P.rhs(lognormal_density(n, seed=seed), 1.0)
    phi, hist = P.mg_solve(f, h, tol=1e-12)
    assert hist[-1] <= 1e-12
    assert P.maxdiff(phi, P.fft_solve(f, h)) < 1e-11
    factors = np.array(hist[1:]) / np.array(hist[:-1])
    assert factors.max() < 0.2            # V(2,2) red-black contraction per cycle
    assert P.relres(phi, f, h) <= 1e-12


def test_mixed_precision_outer_loop():
    n, h = 32, 1.0 / 32
    f = P.rhs(lognormal_density(n, seed=2), 1.0)
    phi, hist = P.mg_solve_mixed(f, h, tol=1e-10)
    assert hist[-1] <= 1e-10
    factors = np.array(hist[1:]) / np.array(hist[:-1])
    assert factors.max() < 0.2            # each FP32 V-cycle still cuts the FP64 residual >= 5x
    assert P.maxdiff(phi, P.fft_solve(f, h)) < 1e-8
