"""The allocation-free entry point siminf_mlp_ensemble_predict_static,
through the C ABI, against the allocating siminf_mlp_ensemble_predict on the
same networks and inputs: bit-identical outputs on two calls in a row, the
second with a smaller batch (the fixed workspace keeps the first call's
contents), and a request beyond the workspace rejected before any work."""
import ctypes

import numpy as np
import pytest

from paper_1605_01421_amd import workloads as W

pytestmark = pytest.mark.gpu

DIMS = (8, 256, 256, 256, 256, 156)


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1605_01421_amd import siminf
    siminf.load()
    return siminf


def test_static_ensemble_equals_allocating_one(lib):
    import torch
    torch.cuda.set_device(0)
    rng = np.random.default_rng(77)
    nets = []
    for k in range(3):
        params = [(Wl, rng.normal(scale=0.1, size=b.shape)) for Wl, b in W.mlp_init(DIMS, 90 + k)]
        net = lib.MLP(DIMS, 1024)
        net.set_params(params)
        nets.append(net)
    ymu = torch.from_numpy(rng.normal(size=DIMS[-1]).astype(np.float32)).cuda()
    ysd = torch.from_numpy(rng.uniform(0.5, 2.0, size=DIMS[-1]).astype(np.float32)).cuda()
    for B in (2500, 700):
        X = torch.from_numpy(rng.normal(size=(B, DIMS[0])).astype(np.float32)).cuda()
        Ya, da = lib.ensemble_predict(nets, X, ymu, ysd)
        Ys, ds = lib.ensemble_predict(nets, X, ymu, ysd, static=True)
        torch.cuda.synchronize()
        assert torch.equal(Ya, Ys), B
        assert torch.equal(da, ds), B
        assert bool(torch.isfinite(Ys).all()) and bool((ds > 0).all())
    # members x B x outputs above the 2^22-float workspace: rejected
    B = (1 << 22) // (3 * DIMS[-1]) + 1
    X = torch.zeros((B, DIMS[0]), dtype=torch.float32, device="cuda")
    Y = torch.zeros((B, DIMS[-1]), dtype=torch.float32, device="cuda")
    d = torch.zeros((B,), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.SiminfError) as e:
        lib.ensemble_predict(nets, X, ymu, ysd, static=True, out=(Y, d))
    assert e.value.code == -2  # SIMINF_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert not bool(Y.any()) and not bool(d.any())
    for net in nets:
        net.close()
