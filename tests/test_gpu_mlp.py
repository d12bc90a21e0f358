"""GPU checks of the surrogate network kernels against the float64 oracle.

The oracle rounds inputs, hidden activations and back-propagated gradients to
bfloat16 at the same points as the kernels, so the remaining differences come
from float32 accumulation and the float32 GELU, which can move a value across
a bfloat16 rounding boundary.  Per-tensor relative Frobenius errors must stay
below 2e-2 for gradients (5e-3 for the forward pass), and every entry within
a few bfloat16 ulps of the magnitude of its own products (see _abs_scales)."""
import numpy as np
import pytest

from oracle import mlp as ref
from paper_1605_01421_amd import workloads as W

pytestmark = pytest.mark.gpu

DIMS = (8, 256, 256, 256, 256, 156)
PROBS = (0.1, 0.5, 0.9)


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1605_01421_amd import siminf
    siminf.load()
    return siminf


def _relf(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _bf16_bits(x):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).cuda(), t.to(torch.float64).numpy()


@pytest.mark.parametrize("shape", [(70, 130, 45), (300, 264, 264), (129, 8, 256), (513, 160, 8)])
@pytest.mark.parametrize("a_trans,b_trans", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_orientations(lib, a_trans, b_trans, shape):
    """Odd leading dimensions take element loads; multiples of 8 take
    16-byte vector loads; tile edges are ragged in M, N and K."""
    import torch
    rng = np.random.default_rng(a_trans * 2 + b_trans)
    M, N, K = shape
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(K, N))
    Astore = A.T if a_trans else A          # a_trans: stored K x M
    Bstore = B if b_trans else B.T          # b_trans: stored K x N, else N x K
    Ab, Aval = _bf16_bits(Astore)
    Bb, Bval = _bf16_bits(Bstore)
    Aeff = Aval.T if a_trans else Aval
    Beff = Bval if b_trans else Bval.T
    C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    lib.gemm_bf16(Ab, Bb, M, N, K, Astore.shape[1], a_trans, Bstore.shape[1], b_trans, C, N)
    torch.cuda.synchronize()
    want = Aeff @ Beff
    assert np.max(np.abs(C.cpu().numpy() - want)) <= 1e-5 * np.max(np.abs(want))


def _setup(seed, B):
    import torch
    params = W.mlp_init(DIMS, seed)
    rng = np.random.default_rng(seed + 100)
    params = [(Wl, rng.normal(scale=0.1, size=b.shape)) for Wl, b in params]
    X = rng.normal(size=(B, DIMS[0]))
    T = rng.normal(scale=0.5, size=(B, DIMS[-1]))
    # the values the device computes with: bfloat16 weights, float32 biases
    rparams = [(ref.bf16(Wl), b.astype(np.float32).astype(np.float64)) for Wl, b in params]
    Xt = torch.from_numpy(X.astype(np.float32)).cuda()
    Tt = torch.from_numpy(T.astype(np.float32)).cuda()
    return params, rparams, X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64), Xt, Tt


def _abs_scales(rparams, X, T):
    """Per-entry magnitudes of the products behind the output and the weight
    gradients, from the oracle with every factor replaced by its absolute
    value: for an entry computed as a sum of products a*b, sum |a||b|.  A
    product with bfloat16 operands whose float32 result or GELU lands on the
    other side of a bfloat16 rounding boundary moves the next layer's operand
    by one bfloat16 ulp (2^-8 relative), so deviations are bounded by a few
    such ulps of these magnitudes, compounded over the layers."""
    Y, (A, Z) = ref.forward(rparams, X, round_bf16=True)
    L = len(rparams)
    yscale = np.abs(A[L - 1]) @ np.abs(rparams[L - 1][0]).T + np.abs(rparams[L - 1][1])
    _, dY = ref.pinball(Y, T, PROBS)
    dz = np.abs(dY)
    gscale = [None] * L
    for l in range(L - 1, -1, -1):
        gscale[l] = (dz.T @ np.abs(A[l]), dz.sum(axis=0))
        if l > 0:
            dz = (dz @ np.abs(rparams[l][0])) * np.abs(ref.gelu_grad(Z[l - 1]))
    return yscale, gscale


def test_forward_matches_oracle(lib):
    """Element by element: |Y - Y_ref| <= 4 bfloat16 ulps of sum |a||w| of
    the output layer's products (plus 1e-6 of the largest), and 5e-3 in
    relative Frobenius norm."""
    params, rparams, X, T, Xt, Tt = _setup(1, 300)
    net = lib.MLP(DIMS, 512)
    net.set_params(params)
    Y = net.forward(Xt).cpu().numpy().astype(np.float64)
    want, _ = ref.forward(rparams, X, round_bf16=True)
    assert _relf(Y, want) < 5e-3
    yscale, _ = _abs_scales(rparams, X, T)
    bound = 4 * 2.0 ** -8 * yscale + 1e-6 * yscale.max()
    over = np.abs(Y - want) > bound
    assert not over.any(), (int(over.sum()), float((np.abs(Y - want) / bound).max()))


@pytest.mark.parametrize("B", [257, 3000])
def test_gradients_match_oracle(lib, B):
    """B = 3000 splits every weight-gradient product over several K slices."""
    params, rparams, X, T, Xt, Tt = _setup(2, B)
    net = lib.MLP(DIMS, 4096)
    net.set_params(params)
    loss = net.backward(Xt, Tt, PROBS)
    wl, wgrads, _ = ref.loss_and_grads(rparams, X, T, PROBS, round_bf16=True)
    assert abs(loss - wl) / wl < 1e-3
    _, gscale = _abs_scales(rparams, X, T)
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(net.get_grads(), wgrads)):
        assert _relf(gW.astype(np.float64), rW) < 2e-2, ("W", l)
        assert _relf(gb.astype(np.float64), rb) < 2e-2, ("b", l)
        # element by element: 4 bfloat16 ulps per layer the gradient passed
        # through, of the entry's sum |dz||a| (plus 1e-6 of the largest)
        ulps = 4 * (len(DIMS) - 1 - l)
        for got, want, sc, what in ((gW, rW, gscale[l][0], "W"), (gb, rb, gscale[l][1], "b")):
            bound = ulps * 2.0 ** -8 * sc + 1e-6 * sc.max()
            over = np.abs(got.astype(np.float64) - want) > bound
            assert not over.any(), (what, l, int(over.sum()),
                                    float((np.abs(got.astype(np.float64) - want) / bound).max()))


def test_adamw_matches_oracle(lib):
    params, rparams, X, T, Xt, Tt = _setup(3, 128)
    net = lib.MLP(DIMS, 256)
    net.set_params(params)
    master = [(Wl.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
              for Wl, b in params]
    state = ref.init_state(master)
    for step in range(3):
        net.backward(Xt, Tt, PROBS, want_loss=False)
        g = [(a.astype(np.float64), b.astype(np.float64)) for a, b in net.get_grads()]
        net.adamw(1e-3, weight_decay=0.01)
        ref.adamw_step(master, g, state, 1e-3, weight_decay=0.01)
        got = net.get_params()
        for (gW, gb), (mW, mb) in zip(got, master):
            assert np.allclose(gW, mW, rtol=1e-5, atol=1e-6)
            assert np.allclose(gb, mb, rtol=1e-5, atol=1e-6)
        master = [(a.astype(np.float64), b.astype(np.float64)) for a, b in got]


def test_training_reduces_loss(lib):
    import torch
    rng = np.random.default_rng(5)
    X = rng.normal(size=(512, 8)).astype(np.float32)
    Wt = rng.normal(size=(8, 156)) / 3
    T = (np.tanh(X @ Wt) + 0.05 * rng.normal(size=(512, 156))).astype(np.float32)
    net = lib.MLP(DIMS, 512)
    net.set_params(W.mlp_init(DIMS, 7))
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    first = net.backward(Xt, Tt, PROBS)
    net.adamw(2e-3)
    for _ in range(300):
        net.backward(Xt, Tt, PROBS, want_loss=False)
        net.adamw(2e-3)
    last = net.backward(Xt, Tt, PROBS)
    assert last < 0.5 * first


def _fwd_bound(rparams, X):
    """4 bfloat16 ulps of the output layer's product magnitudes (see
    test_forward_matches_oracle)."""
    _, (A, _) = ref.forward(rparams, X, round_bf16=True)
    L = len(rparams)
    sc = np.abs(A[L - 1]) @ np.abs(rparams[L - 1][0]).T + np.abs(rparams[L - 1][1])
    return 4 * 2.0 ** -8 * sc + 1e-6 * sc.max()


@pytest.mark.parametrize("members,B", [(1, 37), (4, 300), (3, 1100)])
def test_ensemble_predict_matches_oracle(lib, members, B):
    """siminf_mlp_ensemble_predict against the oracle's members (float64,
    bfloat16-rounded where the kernels round) and its ensemble combination:
    the mean within the members' forward-pass bound times y_std, the
    disagreement within sqrt(K/(K-1)) times that bound; B = 1100 runs the
    members in slices of their largest batch (512)."""
    import torch
    rng = np.random.default_rng(40 + members)
    X = rng.normal(size=(B, DIMS[0])).astype(np.float32).astype(np.float64)
    nets, rps = [], []
    for k in range(members):
        params = [(Wl, rng.normal(scale=0.1, size=b.shape)) for Wl, b in W.mlp_init(DIMS, 60 + k)]
        net = lib.MLP(DIMS, 512)
        net.set_params(params)
        nets.append(net)
        rps.append([(ref.bf16(Wl), b.astype(np.float32).astype(np.float64)) for Wl, b in params])
    ymu = rng.normal(size=DIMS[-1]).astype(np.float32)
    ysd = rng.uniform(0.5, 2.0, size=DIMS[-1]).astype(np.float32)
    Y, dis = lib.ensemble_predict(nets, torch.from_numpy(X.astype(np.float32)).cuda(),
                                  torch.from_numpy(ymu).cuda(), torch.from_numpy(ysd).cuda())
    torch.cuda.synchronize()
    P = np.stack([ref.forward(rp, X, round_bf16=True)[0] for rp in rps])
    mean, d = ref.ensemble_combine(P, ymu, ysd)
    bound = np.max(np.stack([_fwd_bound(rp, X) for rp in rps]), axis=0) * ysd.astype(np.float64)
    Yg = Y.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Yg - mean) <= bound + 1e-6 * np.abs(mean)), float(np.max(np.abs(Yg - mean) / bound))
    dg = dis.cpu().numpy().astype(np.float64)
    if members == 1:
        assert np.all(dg == 0.0)
    else:
        dbound = (np.sqrt(members / (members - 1.0)) * bound).mean(axis=1)
        assert np.all(np.abs(dg - d) <= dbound + 1e-6 * d), float(np.max(np.abs(dg - d) / dbound))
    for net in nets:
        net.close()
