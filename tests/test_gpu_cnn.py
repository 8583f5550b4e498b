"""GPU parity of the learned warm start (BF16 MFMA network) against the CPU oracle.

The oracle runs in FP64 on the same bfloat16-rounded weights, input and
stored activations; the GPU accumulates in FP32.  Bars: forward relative L2
<= 1e-2; parameter and input gradients cosine >= 0.999 and relative L2
<= 3e-2; one Adam step equal to the textbook update to 1e-6.
"""
import numpy as np
import pytest
import torch

from oracle import cnn as N
from oracle import poisson as P
from paper_2604_06035_amd import abi
from workloads import dense_to_oct, lognormal_density, oct_to_dense

pytestmark = pytest.mark.gpu
DEV = "cuda"


def log(*a):
    print(*a, flush=True)


def flat_to_params(v):
    """Flat FP32 vector (mgnn.h layout) -> oracle [(w [O,C,3,3,3], b [O])]."""
    widths = [1, 24, 24, 24, 24, 1]
    out, k = [], 0
    for l in range(5):
        ci, co = widths[l], widths[l + 1]
        w = v[k:k + co * ci * 27].astype(np.float64).reshape(co, ci, 3, 3, 3)
        k += co * ci * 27
        b = v[k:k + co].astype(np.float64)
        k += co
        out.append((w, b))
    assert k == len(v)
    return out


def params_to_flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cosine(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b)))


def random_params(seed):
    rng = np.random.default_rng(seed)
    ps = N.init_params(24, 5, seed=seed)
    return [(w, rng.standard_normal(b.shape) * 0.1) for w, b in ps]


@pytest.mark.parametrize("n", [8, 16])
def test_forward_and_backward_parity(n):
    log(f"cnn parity n={n}")
    rng = np.random.default_rng(n)
    params = random_params(n)
    net = abi.mgnn_create(24, 5, 1)
    try:
        abi.mgnn_set_weights(net, params_to_flat(params))
        got_w = abi.mgnn_get_weights(net)
        np.testing.assert_array_equal(got_w, params_to_flat(params))
        x = rng.standard_normal((n, n, n))
        xd = torch.from_numpy(x.astype(np.float32).ravel()).to(DEV)
        yd = torch.zeros_like(xd)
        abi.mgnn_forward_raw(net, n, xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy().astype(np.float64).reshape(n, n, n)
        p32 = flat_to_params(params_to_flat(params))          # weights as the GPU holds them (f32 master)
        y_ref, cache = N.forward(x.astype(np.float32).astype(np.float64), p32, quantize=True)
        e = rel_l2(y, y_ref)
        log(f"  forward rel L2 = {e:.3e}")
        assert e <= 1e-2
        # backward
        dy = rng.standard_normal((n, n, n)) / n ** 3
        dyd = torch.from_numpy(dy.astype(np.float32).ravel()).to(DEV)
        dxd = torch.zeros_like(xd)
        abi.mgnn_zero_grad(net)
        abi.mgnn_backward_raw(net, n, dyd, dxd)
        torch.cuda.synchronize()
        g = flat_to_params(abi.mgnn_get_grads(net))
        g_ref, dx_ref = N.backward(dy.astype(np.float32).astype(np.float64), p32, cache, quantize=True)
        for l in range(5):
            for k, name in ((0, "W"), (1, "b")):
                a, b = g[l][k], g_ref[l][k]
                c, r = cosine(a, b), rel_l2(a, b)
                log(f"  layer {l} d{name}: cosine={c:.6f} relL2={r:.3e}")
                assert c >= 0.999 and r <= 3e-2
        dx = dxd.cpu().numpy().astype(np.float64).reshape(n, n, n)
        c, r = cosine(dx, dx_ref), rel_l2(dx, dx_ref)
        log(f"  dx: cosine={c:.6f} relL2={r:.3e}")
        assert c >= 0.999 and r <= 3e-2
        # gradients accumulate: a second backward doubles them
        abi.mgnn_backward_raw(net, n, dyd, None)
        torch.cuda.synchronize()
        g2 = abi.mgnn_get_grads(net)
        np.testing.assert_allclose(g2, 2 * params_to_flat(g), rtol=1e-5, atol=1e-12)
    finally:
        abi.mgnn_destroy(net)


def _oracle_at(x, p32, c, r=6):
    """Oracle output at cell c, from the (2r + 1)^3 periodic patch around it.
    Five 3x3x3 layers see 5 cells each way; the patch's wrapped border spoils
    one more cell inward per layer, so with r = 6 the centre is exact."""
    n = x.shape[0]
    patch = x[np.ix_(*[np.arange(ci - r, ci + r + 1) % n for ci in c])]
    y, _ = N.forward(patch, p32, quantize=True)
    return y[r, r, r]


@pytest.mark.parametrize("n", [128, 256])
def test_forward_full_size_sampled(n):
    """Sizes at which workgroups run many tiles each (prefetching the next
    tile's halo box), 256^3 being the warm-start workload: sampled outputs,
    tile corners and the periodic faces among them, against the oracle."""
    log(f"cnn sampled parity n={n}")
    rng = np.random.default_rng(1000 + n)
    params = random_params(n)
    p32 = flat_to_params(params_to_flat(params))
    x = rng.standard_normal((n, n, n)).astype(np.float32)
    net = abi.mgnn_create(24, 5, 1)
    try:
        abi.mgnn_set_weights(net, params_to_flat(params))
        xd = torch.from_numpy(x.ravel()).to(DEV)
        yd = torch.zeros_like(xd)
        abi.mgnn_forward_raw(net, n, xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy().reshape(n, n, n).astype(np.float64)
        assert np.all(np.isfinite(y))
        edge = [0, 7, 8, n // 2 - 1, n // 2, n - 8, n - 1]
        cells = [tuple(rng.choice(edge, 3)) for _ in range(24)] + [tuple(rng.integers(0, n, 3)) for _ in range(24)]
        xo = x.astype(np.float64)
        got = np.array([y[c] for c in cells])
        ref = np.array([_oracle_at(xo, p32, c) for c in cells])
        scale = float(np.sqrt(np.mean(ref ** 2)))
        err = np.abs(got - ref) / scale
        log(f"  {len(cells)} cells: rel L2 = {rel_l2(got, ref):.3e}, max |diff| / rms = {err.max():.3e}")
        assert rel_l2(got, ref) <= 1e-2
        assert err.max() <= 2e-2
    finally:
        abi.mgnn_destroy(net)


@pytest.mark.parametrize("n", [64, 256])
def test_backward_full_size_sparse(n):
    """Gradients at sizes where the weight-gradient workgroups each sum many
    tiles.  dy is non-zero at a few cells at least 11 apart (periodically), so
    the supports of their back-propagated gradients (5 cells each way) are
    disjoint and the BF16 rounding of those gradients acts on each separately;
    the oracle then gets every gradient exactly as a sum over 21^3 periodic
    patches, one per cell, of the network evaluated around that cell."""
    log(f"cnn sparse-dy backward n={n}")
    rng = np.random.default_rng(2000 + n)
    params = random_params(n + 1)
    p32 = flat_to_params(params_to_flat(params))
    x = rng.standard_normal((n, n, n)).astype(np.float32)
    h = n // 2
    cells = [(0, 0, 0), (n - 1, h, 7), (8, n - 1, h - 1), (h, 8, n - 8), (h - 1, h + 16, 16), (24, 24, h + 24)]
    vals = [1.0, -0.5, 0.75, 2.0, -1.25, 0.5]
    for i in range(len(cells)):
        for j in range(i):
            d = [min(abs(a - b), n - abs(a - b)) for a, b in zip(cells[i], cells[j])]
            assert max(d) >= 11, (cells[i], cells[j])
    dy = np.zeros((n, n, n), np.float32)
    for c, v in zip(cells, vals):
        dy[c] = v
    net = abi.mgnn_create(24, 5, 1)
    try:
        abi.mgnn_set_weights(net, params_to_flat(params))
        xd = torch.from_numpy(x.ravel()).to(DEV)
        yd = torch.zeros_like(xd)
        abi.mgnn_forward_raw(net, n, xd, yd)
        dyd = torch.from_numpy(dy.ravel()).to(DEV)
        dxd = torch.zeros_like(xd)
        abi.mgnn_zero_grad(net)
        abi.mgnn_backward_raw(net, n, dyd, dxd)
        torch.cuda.synchronize()
        g = flat_to_params(abi.mgnn_get_grads(net))
        dx = dxd.cpu().numpy().reshape(n, n, n).astype(np.float64)
    finally:
        abi.mgnn_destroy(net)
    R = 10
    xo = x.astype(np.float64)
    g_ref = [[np.zeros_like(w), np.zeros_like(b)] for w, b in p32]
    dx_ref = np.zeros((n, n, n))
    for c, v in zip(cells, vals):
        idx = np.ix_(*[np.arange(ci - R, ci + R + 1) % n for ci in c])
        _, cache = N.forward(xo[idx], p32, quantize=True)
        dyp = np.zeros((2 * R + 1,) * 3)
        dyp[R, R, R] = v
        gp, dxp = N.backward(dyp, p32, cache, quantize=True)
        for l in range(5):
            g_ref[l][0] += gp[l][0]
            g_ref[l][1] += gp[l][1]
        dx_ref[idx] += dxp
    for l in range(5):
        for k, name in ((0, "W"), (1, "b")):
            c_, r_ = cosine(g[l][k], g_ref[l][k]), rel_l2(g[l][k], g_ref[l][k])
            log(f"  layer {l} d{name}: cosine={c_:.6f} relL2={r_:.3e}")
            assert c_ >= 0.999 and r_ <= 3e-2
    c_, r_ = cosine(dx, dx_ref), rel_l2(dx, dx_ref)
    log(f"  dx: cosine={c_:.6f} relL2={r_:.3e}")
    assert c_ >= 0.999 and r_ <= 3e-2
    np.testing.assert_allclose(g[4][1], [sum(vals)], rtol=1e-6)


def test_network_io_transforms_64():
    """The oct <-> dense transforms around the network at a size with several
    tiles per axis: mgnn_forward (density in, oct-major potential out) equals
    s times the raw forward of the host-built input f / rms(f), and the
    training loss equals the host's loss of that output against phi / s."""
    n = 64
    log(f"cnn io transforms n={n}")
    rho = lognormal_density(n, seed=7)
    rho_d = torch.from_numpy(dense_to_oct(rho)).to(DEV)
    f = P.rhs(rho, 1.0)
    rms = float(np.sqrt(np.mean(f * f)))
    s = rms / n ** 2
    x = (f / rms).astype(np.float32)
    net = abi.mgnn_create(24, 5, 3)
    L = abi.mg_build_level(n)
    try:
        xd = torch.from_numpy(N.bf16_round(x.astype(np.float64)).astype(np.float32).ravel()).to(DEV)
        yd = torch.zeros_like(xd)
        abi.mgnn_forward_raw(net, n, xd, yd)
        phi0 = torch.zeros_like(rho_d)
        abi.mgnn_forward(net, n, rho_d, None, 1.0, phi0)
        torch.cuda.synchronize()
        y = yd.cpu().numpy().reshape(n, n, n).astype(np.float64)
        got = oct_to_dense(phi0.cpu().numpy(), n) / s
        e = rel_l2(got, y)
        log(f"  forward through the transforms vs raw: rel L2 = {e:.3e}")
        assert e <= 1e-3
        phi_t = torch.zeros_like(rho_d)
        st, _ = abi.mg_solve(L, rho_d, None, 1.0, None, phi_t, 1e-10, 50)
        assert st == abi.MG_OK
        loss = abi.mgnn_train_step(net, n, rho_d, None, 1.0, phi_t, 0.0)
        t = oct_to_dense(phi_t.cpu().numpy(), n) / s
        loss_ref = float(np.sum((y - t) ** 2) / np.sum(t ** 2))
        log(f"  loss gpu={loss:.8e} host={loss_ref:.8e}")
        assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    finally:
        abi.mgnn_destroy(net)
        abi.mg_destroy_level(L)


def test_adam_step_matches_textbook_update():
    n = 8
    rng = np.random.default_rng(7)
    params = random_params(3)
    net = abi.mgnn_create(24, 5, 1)
    try:
        abi.mgnn_set_weights(net, params_to_flat(params))
        x = torch.from_numpy(rng.standard_normal(n ** 3).astype(np.float32)).to(DEV)
        y = torch.zeros_like(x)
        abi.mgnn_forward_raw(net, n, x, y)
        abi.mgnn_zero_grad(net)
        abi.mgnn_backward_raw(net, n, torch.ones_like(x) / n ** 3)
        torch.cuda.synchronize()
        g = abi.mgnn_get_grads(net).astype(np.float64)
        p0 = params_to_flat(params).astype(np.float64)
        abi.mgnn_adam_step(net, 1e-3)
        torch.cuda.synchronize()
        p1 = abi.mgnn_get_weights(net).astype(np.float64)
        ref, _, _ = N.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
        np.testing.assert_allclose(p1, ref, rtol=1e-6, atol=1e-7)
    finally:
        abi.mgnn_destroy(net)


def test_training_step_loss_and_warm_start():
    # one field, multigrid target, repeated steps: the loss must fall; its first
    # value must equal the oracle's loss of the same network on the same input
    n = 32
    rho = lognormal_density(n, seed=11)
    rho_d = torch.from_numpy(dense_to_oct(rho)).to(DEV)
    L = abi.mg_build_level(n)
    net = abi.mgnn_create(24, 5, 5)
    try:
        phi_t = torch.zeros_like(rho_d)
        st, info = abi.mg_solve(L, rho_d, None, 1.0, None, phi_t, 1e-12, 50)
        assert st == abi.MG_OK
        w0 = abi.mgnn_get_weights(net)
        losses = [abi.mgnn_train_step(net, n, rho_d, None, 1.0, phi_t, 3e-3) for _ in range(30)]
        from workloads import oct_to_dense
        log(f"  losses {losses[0]:.4e} -> {losses[-1]:.4e}")
        assert losses[-1] < 0.7 * losses[0]
        # oracle loss of the initial network on the same input
        f = P.rhs(rho, 1.0)
        h = 1.0 / n
        s = h * h * np.sqrt(np.mean(f * f))
        x = N.bf16_round(f / np.sqrt(np.mean(f * f)))
        y_ref, _ = N.forward(x, flat_to_params(w0), quantize=True)
        t_ref = oct_to_dense(phi_t.cpu().numpy(), n) / s
        loss_ref = float(np.sum((y_ref - t_ref) ** 2) / np.sum(t_ref ** 2))
        log(f"  first loss gpu={losses[0]:.6e} oracle={loss_ref:.6e}")
        assert abs(losses[0] - loss_ref) <= 1e-2 * loss_ref
        # the network output equals the oracle forward of the trained weights
        w1 = abi.mgnn_get_weights(net)
        phi0 = torch.zeros_like(rho_d)
        abi.mgnn_forward(net, n, rho_d, None, 1.0, phi0)
        y1, _ = N.forward(x, flat_to_params(w1), quantize=True)
        got = oct_to_dense(phi0.cpu().numpy(), n) / s
        assert rel_l2(got, y1) <= 1e-2
        rn, fn = abi.mg_residual_norm(L, rho_d, None, 1.0, None, phi0)
        assert np.isfinite(rn) and fn > 0
        # the warm-started solve converges; the guess is kept only if it beats zero
        st, info = abi.mgnn_solve_warm(net, L, rho_d, None, 1.0, phi0, 1e-10, 50)
        assert st == abi.MG_OK and info["relres"] <= 1e-10
        assert info["used_fallback"] == (0 if rn < fn else 1)
        log(f"  warm relres0={rn / fn:.3e} cycles={info['cycles']} fallback={info['used_fallback']}")
        rel = P.relres(oct_to_dense(phi0.cpu().numpy(), n), f, h)
        assert rel <= 1e-10
    finally:
        abi.mgnn_destroy(net)
        abi.mg_destroy_level(L)
