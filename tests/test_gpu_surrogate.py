"""The surrogate pipeline end to end on the GPU, at a reduced size: SSA
targets through the library's prevalence reduction (checked against oracle
runs), an ensemble trained by the library's MFMA kernels, and the
disagreement-gated fallback.  The gain test asks that the combined answer
(network where accepted, SSA elsewhere) be no less accurate than the SSA it
replaces, and that the network alone answer every held-out set at least as
accurately as a small SSA ensemble, at a small fraction of its device
time."""
import os
import sys

import numpy as np
import pytest

from paper_1605_01421_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1605_01421_amd import siminf, surrogate
    siminf.load()
    return surrogate


def test_ssa_quantiles_match_oracle(S):
    import oracle
    import oracle.prevalence as P
    sets = W.ensemble_sets(seed=5, n_sets=3, replicates=6, nn_range=(100, 140))
    q, ms = S.ssa_quantiles(sets, 6, seed=9, stream_base=40)
    _say("quantiles", q.shape, ms)
    sums = np.zeros((18, len(sets[0].spec.tspan), 3), dtype=np.int64)
    for r in range(18):
        spec = sets[r // 6].spec
        ref = oracle.run(spec, 9, 40 + r, nthreads=min(16, os.cpu_count() or 1))
        sums[r, :, :spec.Nc] = ref["U"].astype(np.int64).sum(axis=1)
    want = P.prevalence_quantiles(sums, 1, (0, 1, 2), 6, 1, 52, S.PROBS)
    assert np.array_equal(q, want)


def test_surrogate_gain(S):
    ds = S.make_dataset(n_train=3000, train_reps=16, n_val=120, val_reps=16, truth_reps=128,
                        nn_range=(100, 400), seed=21, log=lambda m: _say(m))
    res, arr = S.evaluate(ds, members=2, epochs=60, batch=128, log=lambda m: _say(m))
    _say({k: res[k] for k in ("eps_ssa", "err_nn_all", "err_nn_accepted", "err_combined", "err_ssa_test",
                              "accepted_fraction", "speedup", "matched_reps", "speedup_matched_reps",
                              "err_nn_test", "network_equivalent_reps", "speedup_network_vs_equivalent_ssa")})
    # the networks learned the map: far better than predicting the mean target
    base = S.mean_abs_error(np.broadcast_to(ds["Ytr"].mean(axis=0), ds["truth"].shape), ds["truth"]).mean()
    assert res["err_nn_all"] < 0.3 * base
    assert np.all(arr["dis"] >= 0)
    # the gain over the SSA alone at the SSA's own error: a share of the sets
    # is answered without simulation, and answering them costs a small
    # fraction of simulating them.  (At this size the SSA is latency-bound,
    # so its time hardly shrinks with fewer sets; the throughput-regime
    # speedup is measured by the full experiment.)
    # fixed error: the threshold was set on the other half so that the
    # combined answer is no less accurate than the SSA; on the test half it
    # must hold within three paired standard errors
    assert res["err_combined"] <= res["err_ssa_test"] + 3 * res["err_combined_minus_ssa_se"]
    # the gain of the network alone: on every test set it is at least as
    # accurate as an SSA ensemble of a few replicates, at a small fraction
    # of that ensemble's device time
    assert res["network_equivalent_reps"] >= 2
    assert res["ms_nn_inference"] < 0.05 * res[f"ms_ssa{res['network_equivalent_reps']}_test"]
