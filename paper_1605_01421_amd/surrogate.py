"""Learned surrogate for the weekly prevalence quantiles of SSA ensembles.

For a parameter set (model, rates, initial prevalence, node-size
distribution, number of nodes) the batched SSA runs R replicate trajectories;
the per-run population prevalence sum(I)/sum(N) at weeks 1..52 (the
prevalence() reduction of section 4.2, taken over all nodes) gives, over the
replicates, the 0.1/0.5/0.9 quantiles of each week -- 156 targets.  A small
multilayer perceptron (8 -> 256 x 4 -> 156, GELU, bfloat16 matrix cores with
float32 accumulation, trained by the library's own kernels on the pinball
loss with AdamW) learns the map; an ensemble of such networks gives a
disagreement estimate, and sets whose disagreement exceeds a threshold fall
back to the SSA.
"""
from __future__ import annotations

import time

import numpy as np

from . import siminf
from . import workloads as W

WEEKS = 52
PROBS = (0.1, 0.5, 0.9)
DIMS = (8, 256, 256, 256, 256, WEEKS * len(PROBS))


def ssa_quantiles(sets, replicates: int, seed: int, stream_base: int = 0, max_nodes: int = 40_000_000,
                  log=None):
    """Quantiles (n_sets, 52, 3) float32 of weekly prevalence from `replicates`
    SSA runs per set (weeks are the tspan indices 1..52 of weekly tspans),
    computed on the GPU in batches of at most `max_nodes` nodes.  Returns the
    quantiles and the device milliseconds spent (SSA + reduction)."""
    import torch
    out = np.zeros((len(sets), WEEKS, len(PROBS)), dtype=np.float32)
    dev_ms = 0.0
    i = 0
    runs_done = 0
    while i < len(sets):
        j, nodes = i, 0
        while j < len(sets) and (j == i or nodes + sets[j].spec.Nn * replicates <= max_nodes):
            nodes += sets[j].spec.Nn * replicates
            j += 1
        chunk = sets[i:j]
        t_host = time.time()
        m = siminf.Model([(s.spec, replicates) for s in chunk], record=siminf.RECORD_SUMS)
        t_host = time.time() - t_host
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        m.run(seed, stream_base + runs_done)
        q = m.prevalence_quantiles(1, (0, 1, 2), replicates, 1, WEEKS, PROBS)
        stop.record()
        rc = m.wait()
        if rc != 0:
            raise siminf.SiminfError(rc, f"ssa batch {m.error_info()}")
        torch.cuda.synchronize()
        dev_ms += start.elapsed_time(stop)
        out[i:j] = q.cpu().numpy()
        runs_done += len(chunk) * replicates
        m.close()
        if log is not None:
            log(f"  sets {i}..{j - 1}: {nodes} nodes, create {t_host:.2f}s, device {dev_ms / 1e3:.2f}s so far")
        i = j
    return out, dev_ms


class Ensemble:
    """K independently initialised networks trained on the same data."""

    def __init__(self, members: int = 4, seed: int = 0, max_batch: int = 4096, dims=DIMS):
        self.dims = tuple(dims)
        self.nets = []
        for k in range(members):
            net = siminf.MLP(self.dims, max_batch)
            net.set_params(W.mlp_init(self.dims, seed * 1000 + k))
            self.nets.append(net)
        self.max_batch = max_batch
        self.mu = self.sd = None      # input standardisation
        self.ymu = self.ysd = None    # per-output target standardisation

    @staticmethod
    def _transform(X):
        """The 8 features re-expressed without changing their information:
        (is_SISe, beta/gamma, upsilon/gamma, log gamma, log initial
        prevalence, mean and variance of log node size, log Nn)."""
        X = np.asarray(X, dtype=np.float64)
        g = X[:, 3]
        return np.stack([X[:, 0], X[:, 1] / g, X[:, 2] / g, np.log(g), np.log(np.maximum(X[:, 4], 1e-12)),
                         X[:, 5], X[:, 6], X[:, 7]], axis=1)

    def _standardise(self, X):
        return ((self._transform(X) - self.mu) / self.sd).astype(np.float32)

    def fit(self, X, Y, epochs: int = 150, batch: int = 128, lr: float = 4e-3, weight_decay: float = 1e-4,
            seed: int = 0, log=None):
        """Minibatch AdamW on the pinball loss; each member sees its own order."""
        import torch
        Z = self._transform(X)
        self.mu = Z.mean(axis=0)
        self.sd = Z.std(axis=0) + 1e-9
        Yf = Y.reshape(len(Y), -1).astype(np.float64)
        # a positive affine map of each output leaves its pinball minimiser
        # (the quantile) equivariant, so the network learns standardised targets
        self.ymu = Yf.mean(axis=0)
        self.ysd = Yf.std(axis=0) + 1e-6
        Xs = torch.from_numpy(self._standardise(X)).cuda()
        Yt = torch.from_numpy(((Yf - self.ymu) / self.ysd).astype(np.float32)).cuda()
        n = len(X)
        steps = max(1, n // batch)
        history = []
        for k, net in enumerate(self.nets):
            rng = np.random.default_rng(seed * 7919 + k)
            total = epochs * steps
            it = 0
            for ep in range(epochs):
                perm = torch.from_numpy(rng.permutation(n)).cuda()
                for s in range(steps):
                    idx = perm[s * batch:(s + 1) * batch]
                    xb, yb = Xs[idx].contiguous(), Yt[idx].contiguous()
                    want = s == steps - 1
                    loss = net.backward(xb, yb, PROBS, want_loss=want)
                    # cosine decay of the learning rate
                    cur = lr * 0.5 * (1.0 + np.cos(np.pi * it / total))
                    net.adamw(float(cur), weight_decay=weight_decay)
                    it += 1
                if log is not None and (ep % 25 == 24 or ep == epochs - 1):
                    log(f"member {k} epoch {ep + 1}/{epochs} loss {loss:.5f}")
                history.append(loss)
        return history

    def predict(self, X):
        """Mean prediction (n, 52, 3), member disagreement (n,) and device ms:
        the members' forward passes, the de-standardisation, the mean and the
        disagreement all run in the library (siminf_mlp_ensemble_predict)."""
        import torch
        Xs = torch.from_numpy(self._standardise(X)).cuda()
        ysd = torch.from_numpy(self.ysd.astype(np.float32)).cuda()
        ymu = torch.from_numpy(self.ymu.astype(np.float32)).cuda()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        mean, dis = siminf.ensemble_predict(self.nets, Xs, ymu, ysd)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        return (mean.cpu().numpy().reshape(len(X), WEEKS, len(PROBS)), dis.cpu().numpy(), ms)

    def close(self):
        for net in self.nets:
            net.close()


def mean_abs_error(Q, ref) -> np.ndarray:
    """Per-set mean absolute quantile error."""
    return np.abs(Q - ref).reshape(len(Q), -1).mean(axis=1)


def choose_threshold(dis, err, eps):
    """Largest disagreement threshold whose accepted sets (dis <= theta) have
    mean error <= eps; -inf when no set can be accepted."""
    order = np.argsort(dis, kind="stable")
    csum = np.cumsum(err[order])
    ok = np.nonzero(csum / np.arange(1, len(order) + 1) <= eps)[0]
    if len(ok) == 0:
        return -np.inf
    return float(dis[order[ok[-1]]])


def choose_threshold_combined(dis, err_nn, err_ssa):
    """Largest disagreement threshold theta for which the combined answer --
    the network on the sets with dis <= theta, the SSA on the others -- is
    no less accurate on average than the SSA alone on the same sets, i.e.
    sum over the accepted sets of (err_nn - err_ssa) <= 0; -inf when no
    prefix qualifies."""
    order = np.argsort(dis, kind="stable")
    csum = np.cumsum(err_nn[order] - err_ssa[order])
    ok = np.nonzero(csum <= 0.0)[0]
    if len(ok) == 0:
        return -np.inf
    return float(dis[order[ok[-1]]])


def make_dataset(n_train=30000, train_reps=32, n_val=1000, val_reps=64, truth_reps=256,
                 nn_range=(100, 20_000), seed=11, log=print):
    """SSA-generated training and held-out data: features X, training targets
    (train_reps-replicate quantiles), held-out ground truth (truth_reps
    replicates) and the val_reps-replicate SSA answer the surrogate competes
    with, plus the device time each took."""
    t0 = time.time()
    train = W.ensemble_sets(seed=seed, n_sets=n_train, replicates=train_reps, nn_range=nn_range)
    val = W.ensemble_sets(seed=seed + 1, n_sets=n_val, replicates=val_reps, nn_range=nn_range)
    log(f"sets generated in {time.time() - t0:.1f}s")
    Ytr, ms_train = ssa_quantiles(train, train_reps, seed=101, log=log)
    log(f"training targets: {n_train} sets x {train_reps} runs in {ms_train / 1e3:.2f}s of device time")
    truth, ms_truth = ssa_quantiles(val, truth_reps, seed=202)
    ssa, ms_ssa = ssa_quantiles(val, val_reps, seed=303)
    log(f"held-out: truth {ms_truth / 1e3:.2f}s, SSA-{val_reps} {ms_ssa / 1e3:.2f}s")
    return dict(Xtr=np.stack([s.features for s in train]), Ytr=Ytr, Xval=np.stack([s.features for s in val]),
                truth=truth, ssa=ssa, ms_train=ms_train, ms_truth=ms_truth, ms_ssa=ms_ssa,
                n_train=n_train, train_reps=train_reps, n_val=n_val, val_reps=val_reps, truth_reps=truth_reps,
                nn_range=nn_range, seed=seed)


def evaluate(ds=None, members=4, epochs=150, batch=128, lr=4e-3, weight_decay=1e-4, log=print, **data_args):
    """The surrogate experiment on a dataset from make_dataset (made here when
    not given): train the ensemble, then on the held-out sets compare (a) the
    val_reps-replicate SSA and (b) the surrogate with SSA fallback, both
    against the truth_reps-replicate ground truth.  The fixed error eps is
    (a)'s mean absolute quantile error; the disagreement threshold is set on
    the even-numbered held-out sets and the accepted fraction, error and
    speedup are reported on the odd-numbered ones."""
    if ds is None:
        ds = make_dataset(log=log, **data_args)
    n_val, val_reps = ds["n_val"], ds["val_reps"]
    val = W.ensemble_sets(seed=ds["seed"] + 1, n_sets=n_val, replicates=val_reps, nn_range=ds["nn_range"])
    ens = Ensemble(members=members, seed=ds["seed"])
    t1 = time.time()
    ens.fit(ds["Xtr"], ds["Ytr"], epochs=epochs, batch=batch, lr=lr, weight_decay=weight_decay, log=log)
    train_s = time.time() - t1
    ens.predict(ds["Xval"][:8])          # first launches load the kernels; not timed
    pred, dis, ms_inf = ens.predict(ds["Xval"])
    truth, ssa = ds["truth"], ds["ssa"]
    err_ssa = mean_abs_error(ssa, truth)
    err_nn = mean_abs_error(pred, truth)
    # the generator emits SIR sets first and SISe sets second, so the
    # calibration and test halves interleave
    cal, test = np.arange(0, n_val, 2), np.arange(1, n_val, 2)
    eps = float(err_ssa.mean())
    # the threshold keeps the combined answer (network where accepted, SSA
    # elsewhere) no less accurate than the SSA alone on the calibration half
    theta = choose_threshold_combined(dis[cal], err_nn[cal], err_ssa[cal])
    accept = dis[test] <= theta
    rej = [val[i] for i in test[~accept]]
    test_sets = [val[i] for i in test]
    ms_fb = ssa_quantiles(rej, val_reps, seed=404)[1] if rej else 0.0
    _, ms_ssa_test = ssa_quantiles(test_sets, val_reps, seed=505)
    combined = np.where(accept[:, None, None], pred[test], ssa[test])
    err_comb_sets = mean_abs_error(combined, truth[test])
    res = dict(
        n_train=ds["n_train"], train_reps=ds["train_reps"], n_val=n_val, val_reps=val_reps,
        truth_reps=ds["truth_reps"], members=members, epochs=epochs, batch=batch,
        eps_ssa=eps, err_nn_all=float(err_nn.mean()),
        err_nn_accepted=float(err_nn[test][accept].mean()) if accept.any() else None,
        err_combined=float(err_comb_sets.mean()),
        err_ssa_test=float(err_ssa[test].mean()), threshold=theta, accepted_fraction=float(accept.mean()),
        ms_ssa_test=ms_ssa_test, ms_nn_inference=ms_inf * len(test) / n_val, ms_fallback=ms_fb,
        train_wall_s=train_s, ms_train_targets=ds["ms_train"])
    # the paired standard error of (combined - SSA) over the test sets
    diff = err_comb_sets - err_ssa[test]
    res["err_combined_minus_ssa_se"] = float(diff.std(ddof=1) / np.sqrt(len(diff))) if len(diff) > 1 else 0.0
    res["ms_pipeline"] = res["ms_nn_inference"] + res["ms_fallback"]
    res["speedup"] = res["ms_ssa_test"] / res["ms_pipeline"]
    # the other reading of fixed error: the fewest SSA replicates whose error
    # on the test sets reaches the combined answer's, and their time
    matched = None
    err_nn_test = float(err_nn[test].mean())
    res["err_nn_test"] = err_nn_test
    equiv = None  # the most replicates whose SSA is no more accurate than the network alone
    for reps in (2, 4, 8, 16, 32):
        if reps >= val_reps:
            break
        q, ms = ssa_quantiles(test_sets, reps, seed=606 + reps)
        e = float(mean_abs_error(q, truth[test]).mean())
        res[f"err_ssa{reps}_test"] = e
        res[f"ms_ssa{reps}_test"] = ms
        if matched is None and e <= res["err_combined"]:
            matched = (reps, ms)
        if e >= err_nn_test:
            equiv = (reps, ms)
    if matched is None:
        matched = (val_reps, ms_ssa_test)
    res["matched_reps"] = matched[0]
    res["speedup_matched_reps"] = matched[1] / res["ms_pipeline"]
    # what the network alone gains: it answers every test set as accurately
    # as an SSA of equiv replicates, at its inference cost
    res["network_equivalent_reps"] = equiv[0] if equiv else 0
    res["speedup_network_vs_equivalent_ssa"] = (equiv[1] / res["ms_nn_inference"]) if equiv else None
    res["err_nn_test_quantiles"] = [float(x) for x in np.quantile(err_nn[test], (0.1, 0.5, 0.9))]
    res["spearman_dis_err"] = float(np.corrcoef(np.argsort(np.argsort(dis)), np.argsort(np.argsort(err_nn)))[0, 1])
    ens.close()
    return res, dict(pred=pred, dis=dis)


def main(argv=None):
    """python -m paper_1605_01421_amd.surrogate [--n-train N] ... : the whole
    experiment on cuda:0; progress lines go to stdout, the result is the
    last line (JSON)."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=200000)
    ap.add_argument("--train-reps", type=int, default=64)
    ap.add_argument("--n-val", type=int, default=2000)
    ap.add_argument("--members", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--lr", type=float, default=4e-3)
    ap.add_argument("--seed", type=int, default=11)
    args = ap.parse_args(argv)
    t0 = time.time()

    def log(msg):
        print(f"[{time.time() - t0:7.1f}s] {msg}", flush=True)

    ds = make_dataset(n_train=args.n_train, train_reps=args.train_reps, n_val=args.n_val, seed=args.seed, log=log)
    res, _ = evaluate(ds, members=args.members, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    res["wall_s"] = time.time() - t0
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
