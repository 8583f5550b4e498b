"""GPU parity of the periodic-level path against the CPU oracle, through the C ABI.

Per-step checks (one kernel each) on grids that span several workgroups and
a partial last workgroup, then whole solves: the GPU potential must reach
relative residual <= 1e-10 (evaluated by the oracle's own residual code) and
match the oracle's exact FFT solution to max|dphi|/max|phi| <= 1e-8.
"""
import numpy as np
import pytest
import torch

from oracle import poisson as P
from paper_2604_06035_amd import abi
from workloads import dense_to_oct, lognormal_density, oct_to_dense, sinusoid_density

pytestmark = pytest.mark.gpu
DEV = "cuda"


def log(*a):
    print(*a, flush=True)


def dev(dense, dtype=torch.float64):
    return torch.from_numpy(dense_to_oct(np.ascontiguousarray(dense))).to(DEV, dtype)


def host(t, n):
    return oct_to_dense(t.double().cpu().numpy(), n)


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------------------
# kernel-level parity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,sweeps", [(4, 2), (8, 2), (16, 3), (32, 2), (64, 1), (64, 2), (128, 2)])
def test_smooth_parity(n, sweeps, dtype):
    # n >= 16 runs the fused LDS-tiled sweep (ping-pong buffers), smaller n the half-sweep kernels
    log(f"smooth n={n} sweeps={sweeps} {dtype}")
    h = 1.0 / n
    rng = np.random.default_rng(n)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    phi0 = rng.standard_normal((n, n, n)).astype(npdt)
    b = rng.standard_normal((n, n, n)).astype(npdt) * npdt(n * n)
    ref = phi0.copy()
    for _ in range(sweeps):
        P.gs_sweep(ref, b, h)
    phi_d, b_d = dev(phi0, dtype), dev(b, dtype)
    work = torch.empty_like(phi_d) if n == 64 else None      # caller-provided or library scratch
    abi.mg_op_smooth(n, h, phi_d, b_d, sweeps, work)
    torch.cuda.synchronize()
    got = host(phi_d, n)
    tol = 1e-13 if dtype == torch.float64 else 2e-5
    assert rel_err(got, ref.astype(np.float64)) < tol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [16, 32, 64, 256])
def test_repeated_sweeps_equal_single_sweeps(n, dtype):
    # k sweeps in one call (ping-pong between the caller's buffer and the work
    # buffer, a final copy when k is odd) must reproduce k one-sweep calls bit
    # for bit; n = 256 runs the z-marching kernel, smaller n the 3-D tiles
    log(f"repeated sweeps n={n} {dtype}")
    h = 1.0 / n
    rng = np.random.default_rng(300 + n)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    phi0 = rng.standard_normal((n, n, n)).astype(npdt)
    b = (rng.standard_normal((n, n, n)) * n * n).astype(npdt)
    b_d = dev(b, dtype)
    work = torch.empty_like(b_d)
    for sweeps in (2, 3, 4):
        one = dev(phi0, dtype)
        for _ in range(sweeps):
            abi.mg_op_smooth(n, h, one, b_d, 1, work)
        fused = dev(phi0, dtype)
        abi.mg_op_smooth(n, h, fused, b_d, sweeps, work)
        torch.cuda.synchronize()
        assert torch.equal(one, fused), sweeps


@pytest.mark.parametrize("n,dtype", [(256, torch.float64), (256, torch.float32), (512, torch.float64)])
def test_marching_sweep_parity(n, dtype):
    # the z-marching sweep (n >= 256; at 512^3 the launch the bandwidth figure
    # is measured on): one sweep against the oracle's red-black sweep, element
    # by element, on a field with structure at every scale
    log(f"marching sweep n={n} {dtype}")
    h = 1.0 / n
    rng = np.random.default_rng(n)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    phi0 = rng.standard_normal((n, n, n)).astype(npdt)
    b = (rng.standard_normal((n, n, n)) * n * n).astype(npdt)
    ref = phi0.astype(np.float64)
    P.gs_sweep(ref, b.astype(np.float64), h)
    phi_d, b_d = dev(phi0, dtype), dev(b, dtype)
    abi.mg_op_smooth(n, h, phi_d, b_d, 1, torch.empty_like(phi_d))
    torch.cuda.synchronize()
    tol = 1e-13 if dtype == torch.float64 else 2e-5
    assert rel_err(host(phi_d, n), ref) < tol


def test_fused_norm_of_marching_sweep_256():
    # the first sweep of each cycle also returns ||f - L phi||: with no cycle
    # allowed, relres0 must equal the oracle's relative residual of phi0
    n = 256
    rho = lognormal_density(n, seed=5)
    rng = np.random.default_rng(5)
    phi0 = rng.standard_normal((n, n, n)) * 1e-4
    st, info, phi = solve_gpu(rho, phi0=phi0, max_cycles=0)
    f = P.rhs(rho, 1.0)
    ref = P.relres(phi0, f, 1.0 / n)
    log(f"  relres0 gpu={info['relres0']:.15e} oracle={ref:.15e}")
    assert st == abi.MG_NOT_CONVERGED and info["cycles"] == 0
    assert abs(info["relres0"] - ref) <= 1e-12 * ref
    # no cycle ran: phi is the guess, only projected to mean zero
    np.testing.assert_allclose(phi, phi0 - phi0.mean(), rtol=0, atol=1e-15)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [4, 8, 32, 64, 256, 512])
def test_resid_restrict_parity(n, dtype):
    # n >= 512 runs the z-marching residual (column runs, LDS ring), 16-256
    # the 3-D tile, smaller grids one thread per oct
    log(f"resid_restrict n={n} {dtype}")
    h = 1.0 / n
    rng = np.random.default_rng(100 + n)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    phi = rng.standard_normal((n, n, n)).astype(npdt)
    b = (rng.standard_normal((n, n, n)) * n * n).astype(npdt)
    r = P.residual(phi, b, h)
    ref_c = P.restrict(r)
    ref_n2 = float(np.sum(r.astype(np.float64) ** 2))
    bc = torch.zeros((n // 2) ** 3, dtype=dtype, device=DEV)
    n2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    abi.mg_op_resid_restrict(n, h, dev(phi, dtype), dev(b, dtype), bc, n2)
    torch.cuda.synchronize()
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    assert rel_err(host(bc, n // 2), ref_c.astype(np.float64)) < tol * 10
    assert abs(n2.item() - ref_n2) / ref_n2 < tol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [8, 16, 64])
def test_prolong_parity(n, dtype):
    log(f"prolong n={n} {dtype}")
    rng = np.random.default_rng(200 + n)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    ec = rng.standard_normal((n // 2,) * 3).astype(npdt)
    e = rng.standard_normal((n,) * 3).astype(npdt)
    ref = e + P.prolong(ec)
    e_d = dev(e, dtype)
    abi.mg_op_prolong(n, dev(ec, dtype), e_d)
    torch.cuda.synchronize()
    tol = 1e-14 if dtype == torch.float64 else 1e-6
    assert rel_err(host(e_d, n), ref.astype(np.float64)) < tol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_coarse_solve_parity(dtype):
    n, h = 4, 1.0 / 4
    rng = np.random.default_rng(3)
    b = rng.standard_normal((n, n, n))
    b -= b.mean()
    ref = P.coarse_solve(b, h)
    e_d = torch.zeros(64, dtype=dtype, device=DEV)
    abi.mg_op_coarse_solve(n, h, dev(b, dtype), e_d)
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert rel_err(host(e_d, n), ref) < tol


# ---------------------------------------------------------------------------
# whole solves
# ---------------------------------------------------------------------------
def solve_gpu(rho, precision=abi.MG_PREC_FP64, tol=1e-10, phi0=None, max_cycles=50):
    n = rho.shape[0]
    L = abi.mg_build_level(n, precision=precision)
    try:
        rho_d = dev(rho)
        phi_d = torch.zeros_like(rho_d) if phi0 is None else dev(phi0)
        st, info = abi.mg_solve(L, rho_d, None, 1.0, None, phi_d, tol, max_cycles)
        torch.cuda.synchronize()
        return st, info, host(phi_d, n)
    finally:
        abi.mg_destroy_level(L)


def check_against_oracle(rho, phi, tol_relres=1e-10, tol_max=1e-8):
    n = rho.shape[0]
    h = 1.0 / n
    f = P.rhs(rho, 1.0)
    rr = P.relres(phi, f, h)
    ref = P.fft_solve(f, h)
    md = P.maxdiff(phi, ref)
    log(f"  oracle relres={rr:.3e} maxdiff={md:.3e} mean={phi.mean():.2e}")
    assert rr <= tol_relres
    assert md <= tol_max
    assert abs(phi.mean()) < 1e-12 * np.max(np.abs(ref))
    return rr, md


@pytest.mark.parametrize("precision", [abi.MG_PREC_FP64, abi.MG_PREC_MIXED])
def test_solve_sinusoid_32(precision):
    log(f"solve sinusoid 32 prec={precision}")
    n = 32
    rho = sinusoid_density(n)
    st, info, phi = solve_gpu(rho, precision)
    log(" ", info)
    assert st == abi.MG_OK and info["relres"] <= 1e-10
    assert abs(info["rho_mean"] - 1.0) < 1e-14
    check_against_oracle(rho, phi)
    # closed form: phi = 0.5 / lambda_h * s with lambda_h = -12 sin^2(pi h)/h^2
    x = (np.arange(n) + 0.5) / n
    s = np.sin(2 * np.pi * x)
    S = s[:, None, None] * s[None, :, None] * s[None, None, :]
    coef = 0.5 / (-12.0 * np.sin(np.pi / n) ** 2 * n * n)
    assert np.max(np.abs(phi - coef * S)) <= 1e-8 * abs(coef)
    # same number of cycles as the oracle's V-cycle (plain mode)
    if precision == abi.MG_PREC_FP64:
        _, hist = P.mg_solve(P.rhs(rho, 1.0), 1.0 / n, tol=1e-10)
        assert abs(info["cycles"] - (len(hist) - 1)) <= 1


@pytest.mark.parametrize("precision", [abi.MG_PREC_FP64, abi.MG_PREC_MIXED])
@pytest.mark.parametrize("n", [16, 64, 128])
def test_solve_lognormal(n, precision):
    log(f"solve lognormal n={n} prec={precision}")
    rho = lognormal_density(n, seed=2)
    st, info, phi = solve_gpu(rho, precision)
    log(" ", info)
    assert st == abi.MG_OK
    rr, _ = check_against_oracle(rho, phi)
    # the reported norm is that of the returned phi (the solve enqueues cycles
    # ahead of the norms it has read); a cycle changes it by 5x or more
    assert abs(info["relres"] - rr) <= 0.05 * rr


@pytest.mark.parametrize("max_cycles", [1, 2, 3, 6])
def test_cycle_limit_applies_exactly_that_many_cycles(max_cycles):
    # a cycle limit stops the pipelined loop after exactly max_cycles V-cycles:
    # phi equals the oracle's after the same number of cycles and the reported
    # norm is the oracle's norm of that phi
    n = 32
    h = 1.0 / n
    rho = lognormal_density(n, seed=2)
    f = P.rhs(rho, 1.0)
    st, info, phi = solve_gpu(rho, max_cycles=max_cycles)
    log(f"max_cycles={max_cycles}", info)
    assert st == abi.MG_NOT_CONVERGED and info["cycles"] == max_cycles
    ref, hist = P.mg_solve(f, h, tol=0.0, max_cycles=max_cycles)
    assert len(hist) == max_cycles + 1
    assert rel_err(phi, ref) <= 1e-10
    assert abs(info["relres"] - hist[-1]) <= 1e-6 * hist[-1]


@pytest.mark.slow
@pytest.mark.parametrize("precision", [abi.MG_PREC_FP64, abi.MG_PREC_MIXED])
def test_solve_lognormal_256_full_size(precision):
    # the full-size periodic workload: 256^3, P(k) ~ k^-2.5, variance 1.5, seed 2
    log(f"solve lognormal 256 prec={precision}")
    rho = lognormal_density(256, seed=2)
    st, info, phi = solve_gpu(rho, precision)
    log(" ", info)
    assert st == abi.MG_OK
    check_against_oracle(rho, phi)


def test_solve_lognormal_512_full_size():
    # 512^3, the size the bandwidth target is stated for: plain and mixed
    # solves of one input against the oracle's residual and exact solution
    n = 512
    h = 1.0 / n
    log(f"solve lognormal {n}, plain and mixed")
    rho = lognormal_density(n, seed=2)
    f = P.rhs(rho, 1.0)
    ref = P.fft_solve(f, h)
    for precision in (abi.MG_PREC_FP64, abi.MG_PREC_MIXED):
        st, info, phi = solve_gpu(rho, precision)
        rr, md = P.relres(phi, f, h), P.maxdiff(phi, ref)
        log(f"  prec={precision} cycles={info['cycles']} oracle relres={rr:.3e} maxdiff={md:.3e}")
        assert st == abi.MG_OK
        assert rr <= 1e-10 and md <= 1e-8
        assert abs(phi.mean()) < 1e-12 * np.max(np.abs(ref))
        del phi


def test_warm_start_and_not_converged_and_zero_rhs():
    n = 32
    rho = lognormal_density(n, seed=7)
    f = P.rhs(rho, 1.0)
    ref = P.fft_solve(f, 1.0 / n)
    st, info, phi = solve_gpu(rho, phi0=ref)
    assert st == abi.MG_OK and info["cycles"] == 0 and info["relres0"] <= 1e-10
    st, info, phi = solve_gpu(rho, max_cycles=1)
    assert st == abi.MG_NOT_CONVERGED and info["cycles"] == 1 and info["relres"] < info["relres0"]
    st, info, phi = solve_gpu(np.full((n, n, n), 3.0))
    assert st == abi.MG_OK and np.all(phi == 0.0)


def test_residual_norm_matches_oracle():
    n = 32
    rho = lognormal_density(n, seed=9)
    rng = np.random.default_rng(1)
    phi = rng.standard_normal((n, n, n)) * 1e-3
    f = P.rhs(rho, 2.5)
    L = abi.mg_build_level(n)
    try:
        rn, fn = abi.mg_residual_norm(L, dev(rho), None, 2.5, None, dev(phi))
    finally:
        abi.mg_destroy_level(L)
    assert abs(fn - P.norm2(f)) / P.norm2(f) < 1e-13
    r_ref = P.norm2(P.residual(phi, f, 1.0 / n))
    assert abs(rn - r_ref) / r_ref < 1e-12


def test_solve_argument_errors():
    n = 16
    L = abi.mg_build_level(n)
    try:
        rho = torch.ones((n // 2) ** 3 * 8, dtype=torch.float64, device=DEV)
        phi = torch.zeros_like(rho)
        with pytest.raises(abi.MgError) as ei:
            abi.mg_solve(L, rho, None, 1.0, phi, phi, 1e-10, 10)   # parent phi on a periodic level
        assert ei.value.status == abi.MG_ERR_ARG
        with pytest.raises(abi.MgError):
            abi.mg_solve(L, rho, None, 1.0, None, phi, -1.0, 10)
        rho_nan = rho.clone()
        rho_nan[5] = float("nan")
        with pytest.raises(abi.MgError) as ei:
            abi.mg_solve(L, rho_nan, None, 1.0, None, phi, 1e-10, 10)
        assert ei.value.status == abi.MG_ERR_DIVERGED
    finally:
        abi.mg_destroy_level(L)
