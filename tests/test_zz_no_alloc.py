"""ka_gamma_apply_static (no device allocation, static scratch) against
ka_gamma_apply on the same inputs, through the C ABI: two calls in a row, the
second with a smaller product, both precisions; and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inputs(torch, seed, nr, nc, b):
    from workloads import normal_block, uniform_points
    xc = torch.tensor(uniform_points(seed, nc), dtype=torch.float32, device="cuda")
    xr = torch.tensor(uniform_points(seed + 1, nr), dtype=torch.float32, device="cuda")
    y = torch.tensor(normal_block(seed + 2, nc, b, dtype=np.float32), device="cuda")
    return xr, xc, y


# (kernel, ell, nr, nc, b, precision): the first call splits its columns over
# several workgroups (partial sums in the scratch), the second is smaller and
# leaves the first call's data in the scratch behind it
CALLS = [("gaussian", 0.5, 9000, 150000, 32, "bf16x3"),
         ("exponential", 0.8, 1500, 20000, 16, "fp32"),
         ("gaussian", 0.3, 700, 3333, 64, "bf16x3")]


def test_static_scratch_matches_workspace_entry_point():
    import torch
    import paper_2101_00629_amd as K
    torch.cuda.set_device(0)
    for i, (kern, ell, nr, nc, b, prec) in enumerate(CALLS):
        print(f"[no-alloc] call {i}: {kern} nr={nr} nc={nc} b={b} {prec}", flush=True)
        P = K.PRECISIONS[prec]
        need = K.ka_gamma_workspace(nr, nc, b, P)
        assert 0 < need <= K.ka_gamma_static_capacity()
        xr, xc, y = _inputs(torch, 40 + i, nr, nc, b)
        ref = torch.empty((nr, b), dtype=torch.float32, device="cuda")
        got = torch.full((nr, b), float("nan"), dtype=torch.float32, device="cuda")
        work = torch.empty(need // 4 + 1, dtype=torch.float32, device="cuda")
        K.ka_gamma_apply(K.KERNELS[kern], 1.1, ell, xr, xc, y, ref, P, work)
        K.ka_gamma_apply_static(K.KERNELS[kern], 1.1, ell, xr, xc, y, got, P)
        torch.cuda.synchronize()
        # same kernels, same split plan, same reduction order: bitwise equal
        assert torch.equal(ref, got), (ref - got).abs().max().item()


def test_static_scratch_size_limit():
    import torch
    import paper_2101_00629_amd as K
    torch.cuda.set_device(0)
    cap = K.ka_gamma_static_capacity()
    nc = cap // (64 * 4) + 64            # BF16X3 split parts of Y alone exceed the capacity
    assert K.ka_gamma_workspace(16, nc, 64, K.KA_BF16X3) > cap
    x = torch.zeros((16, 3), dtype=torch.float32, device="cuda")
    z = torch.zeros((16, 64), dtype=torch.float32, device="cuda")

    class _Fake:                          # shapes only: the call must fail before any launch
        def __init__(self, shape):
            self.shape = shape

        def data_ptr(self):
            return x.data_ptr()
    with pytest.raises(K.KAError) as e:
        K.ka_gamma_apply_static(K.KA_GAUSSIAN, 1.0, 0.5, x, _Fake((nc, 3)), _Fake((nc, 64)), z, K.KA_BF16X3)
    assert e.value.code == K.KA_ERR_ARG
    assert "static scratch" in K.ka_last_error()
