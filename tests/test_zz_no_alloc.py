"""The residual + restriction entry point that allocates nothing against the
one that allocates its partials per call: same results bit for bit, on two
calls in a row (the second on a smaller grid, so stale partials of the first
would show), in f64 and f32; sizes beyond the static scratch are refused."""
import numpy as np
import pytest
import torch

from paper_2604_06035_amd import abi

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_resid_restrict_matches_the_allocating_entry_point(dtype):
    gen = torch.Generator(device=DEV)
    gen.manual_seed(17)
    for n in (64, 32, 8, 1024):          # tiled, tiled, small-grid kernel, the largest size allowed
        h = 1.0 / n
        phi = torch.randn(n ** 3, generator=gen, device=DEV, dtype=dtype)
        b = torch.randn(n ** 3, generator=gen, device=DEV, dtype=dtype) * (n * n)
        out = []
        for fn in (abi.mg_op_resid_restrict, abi.mg_op_resid_restrict_noalloc):
            bc = torch.full(((n // 2) ** 3,), np.nan, dtype=dtype, device=DEV)
            nrm = torch.full((1,), np.nan, dtype=torch.float64, device=DEV)
            fn(n, h, phi, b, bc, nrm)
            torch.cuda.synchronize()
            out.append((bc.cpu().numpy(), float(nrm.item())))
        print(f"n={n} {dtype}: norm2 {out[0][1]:.17e} / {out[1][1]:.17e}", flush=True)
        np.testing.assert_array_equal(out[1][0], out[0][0])
        assert out[1][1] == out[0][1] and np.isfinite(out[0][1])
        # without a norm output the partials are not written at all
        bc = torch.zeros(((n // 2) ** 3,), dtype=dtype, device=DEV)
        abi.mg_op_resid_restrict_noalloc(n, h, phi, b, bc, None)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(bc.cpu().numpy(), out[0][0])
        del phi, b


def test_noalloc_rejects_grids_beyond_its_scratch():
    x = torch.zeros(16, dtype=torch.float64, device=DEV)
    with pytest.raises(abi.MgError) as ei:
        abi.mg_op_resid_restrict_noalloc(2048, 1.0 / 2048, x, x, x, x)
    assert ei.value.status == abi.MG_ERR_ARG and "scratch" in str(ei.value)
