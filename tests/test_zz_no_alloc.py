"""The allocation-free network backward (mpm_mlp_backward_noalloc: the work
buffer is the library's static device array) against the allocating one
(mpm_mlp_backward with a caller buffer), through the C-ABI, on two calls in
a row -- the second with fewer samples, so the scratch array still holds
the first call's larger layout -- and its size limit."""
import ctypes as ct

import numpy as np
import pytest

from paper_2507_04192_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(a, b):
    a, b = a.double(), b.double()
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("math", ["bf16", "f32"])
def test_noalloc_backward_matches_allocating_backward(math):
    import torch
    from paper_2507_04192_amd.native import MLP
    widths = [2, 128, 128, 1]                       # the friction-field network
    net = MLP(widths, out_act="sigmoid", math=math)
    params = torch.tensor(W.mlp_init_params(widths, 3), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(17)
    # two calls in a row, the second smaller (a floor of 193 x 97 nodes, then 4,099)
    for n in (18721, 4099):
        print(f"[case] noalloc backward {math} n={n}", flush=True)
        assert net.cache_floats(n) <= 8 * 1024 * 1024
        x = torch.tensor(rng.uniform(-1, 1, (2, n)), dtype=torch.float32, device="cuda")
        dy = torch.tensor(rng.normal(0, 1, (1, n)), dtype=torch.float32, device="cuda")
        _, cache = net.forward(params, x)
        want = net.backward(params, x, cache, dy)
        got = torch.full_like(params, float("nan"))
        net.backward_noalloc_into(params, x, cache, dy, got)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        # the weight gradient sums chunk partials with atomics: equal to
        # rounding, not bit for bit
        e = _rel(got, want)
        print(f"  rel L2 {e:.2e}", flush=True)
        assert e <= 1e-6


def test_noalloc_backward_rejects_oversize():
    import torch
    from paper_2507_04192_amd.native import MLP, lib
    widths = [2, 128, 128, 1]
    net = MLP(widths, out_act="sigmoid", math="f32")
    n = 40000                                          # 40000 x 257 floats > 8 Mi
    assert net.cache_floats(n) > 8 * 1024 * 1024
    params = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    x = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    L = lib()
    rc = L.mpm_mlp_backward_noalloc(ct.byref(net.desc), None, ct.c_void_p(params.data_ptr()), n,
                                    ct.c_void_p(x.data_ptr()), ct.c_void_p(x.data_ptr()),
                                    ct.c_void_p(x.data_ptr()), ct.c_void_p(params.data_ptr()))
    assert rc == -1
    assert b"scratch" in L.mpm_last_error(None)
