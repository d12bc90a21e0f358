"""Parity at the full sizes of the throughput workloads.

* SISe with scheduled events, 37,000 nodes x 3,650 days (about 7.9 million
  events): the whole trajectory U bit-exact, phi within 1e-12 relative,
  counters equal.
* The 4,096-run batch (64 parameter sets x 64 replicates, node counts
  log-uniform on 100..20,000, 365 days, weekly sums): per-run weekly sums of
  sampled runs bit-exact against oracle runs of the same stream, and the
  prevalence quantiles of one whole set recomputed from oracle runs of all
  of its replicates.
"""
import os
import sys

import numpy as np
import pytest

from paper_1605_01421_amd import workloads as W

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1605_01421_amd import siminf
    siminf.load()
    return siminf


def test_sise_events_full_size(lib):
    import oracle
    spec = W.sise_with_events()
    _say("SISe with events, full size", spec.Nn, len(spec.events["time"]), "threads", NTHREADS)
    m = lib.Model(spec)
    m.run(31, 5)
    rc = m.wait()
    _say("gpu done", rc, m.launch_info(), m.timing())
    ref = oracle.run(spec, 31, 5, nthreads=NTHREADS)
    _say("oracle done", ref["status"])
    assert rc == 0 and ref["status"] == 0
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])
    U, V = m.trajectory()
    assert np.array_equal(U, ref["U"])
    np.testing.assert_allclose(V, ref["V"], rtol=1e-12, atol=0)


@pytest.fixture(scope="module")
def batch(lib):
    """The batch as the benchmark runs it: autotuned launch shape, replayed
    from a captured HIP graph."""
    sets = W.ensemble_sets(seed=3, n_sets=64, replicates=64)
    m = lib.Model([(s.spec, 64) for s in sets], record=lib.RECORD_SUMS, graph=1)
    _say("batch", m.runs, "runs", sum(s.spec.Nn for s in sets) * 64, "nodes")
    best = m.autotune(seed=7, repeats=1)
    _say("autotuned", m.launch_info(), f"{best:.1f} ms")
    m.run(79, 0)
    assert m.wait() == 0, m.error_info()
    _say("batch done", m.launch_info(), m.timing())
    return sets, m, m.sums()


def test_batch_full_size_shapes_agree(lib, batch):
    """The autotuned, graph-replayed batch equals plain launches of the
    lockstep kernel and of the lane-queue kernel, sum for sum and counter for
    counter."""
    sets, m, sums = batch
    c = m.counters()
    for lq in (2, 1):
        other = lib.Model([(s.spec, 64) for s in sets], record=lib.RECORD_SUMS, lane_queue=lq)
        other.run(79, 0)
        assert other.wait() == 0
        _say("plain", other.launch_info(), other.timing())
        assert np.array_equal(other.sums(), sums), lq
        assert other.counters() == c, lq
        other.close()


@pytest.mark.parametrize("run", [0, 1, 2047, 2048, 4095])
def test_batch_full_size_sampled_runs(lib, batch, run):
    import oracle
    sets, m, sums = batch
    spec = sets[run // 64].spec
    _say("sampled run", run, spec.name, spec.Nn)
    ref = oracle.run(spec, 79, run, nthreads=NTHREADS)
    assert ref["status"] == 0
    assert np.array_equal(sums[run, :, :spec.Nc], ref["U"].astype(np.int64).sum(axis=1))


def test_batch_full_size_set_quantiles(lib, batch):
    """All 64 replicates of the smallest SIR and SISe sets through the oracle."""
    import oracle
    import oracle.prevalence as P
    sets, m, sums = batch
    q = m.prevalence_quantiles(1, (0, 1, 2), 64, 1, 52).cpu().numpy()
    for lo, hi in ((0, 32), (32, 64)):
        k = min(range(lo, hi), key=lambda j: sets[j].spec.Nn)
        spec = sets[k].spec
        _say("set", k, spec.name, spec.Nn)
        ref_sums = np.zeros((64, m.ntspan, 3), dtype=np.int64)
        for r in range(64):
            ref = oracle.run(spec, 79, 64 * k + r, nthreads=NTHREADS)
            ref_sums[r, :, :spec.Nc] = ref["U"].astype(np.int64).sum(axis=1)
        assert np.array_equal(sums[64 * k:64 * (k + 1)], ref_sums)
        want = P.prevalence_quantiles(ref_sums, 1, (0, 1, 2), 64, 1, 52, (0.1, 0.5, 0.9))
        assert np.array_equal(q[k], want[0])
