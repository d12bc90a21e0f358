"""Runs replayed from a captured HIP graph (options.graph = 1).

Each replay, with ordinary (uncaptured) runs of another model and host
synchronisation in between, must equal a plainly launched run of the same
seed bit for bit, and the oracle where it is consulted."""
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


def test_graph_replays_equal_plain_runs(lib):
    import oracle
    sets = W.ensemble_sets(seed=41, n_sets=6, replicates=4, days=120, nn_range=(80, 600))
    batch = [(s.spec, 4) for s in sets]
    g = lib.Model(batch, record=lib.RECORD_SUMS, graph=1)
    plain = lib.Model(batch, record=lib.RECORD_SUMS)
    for seed in (3, 8, 3, 21):
        _say("graph replay seed", seed)
        g.run(seed, 10)
        assert g.wait() == 0
        got = g.sums()
        plain.run(seed, 10)
        assert plain.wait() == 0
        assert np.array_equal(got, plain.sums()), seed
        assert g.counters() == plain.counters()
    ref = oracle.run(sets[5].spec, 21, 10 + 23, nthreads=NTHREADS)
    assert np.array_equal(got[23, :, :2], ref["U"].astype(np.int64).sum(axis=1))


def test_graph_full_records_and_reconfigure(lib):
    import oracle
    spec = W.plain_sir()
    m = lib.Model(spec, graph=1)
    for seed in (123, 7):
        _say("graph full records seed", seed)
        m.run(seed, 0)
        assert m.wait() == 0
        ref = oracle.run(spec, seed, 0, nthreads=NTHREADS)
        U, _ = m.trajectory()
        assert np.array_equal(U, ref["U"])
    # the autotuner reconfigures the launch: the graph is captured again
    m.autotune(seed=5, repeats=1)
    m.run(9, 2)
    assert m.wait() == 0
    U, _ = m.trajectory()
    assert np.array_equal(U, oracle.run(spec, 9, 2, nthreads=NTHREADS)["U"])


def test_graph_replays_with_groups(lib):
    """Graph replay of a launch with nodes on groups of lanes and 8 nodes to
    a one-lane wavefront, against plain launches and the oracle."""
    import oracle
    spec = W.plain_sir()
    # lanes=1: no wavefront-wide nodes (the 100 equal nodes would all pass
    # the wide cut), so 40 nodes take groups and 60 one lane each
    g = lib.Model(spec, graph=1, group=40, pack=8, lanes=1)
    plain = lib.Model(spec, group=40, pack=8, lanes=1)
    assert g.launch_info()["group"] == 40
    for seed in (4, 19, 4):
        _say("graph with groups seed", seed)
        g.run(seed, 1)
        assert g.wait() == 0
        plain.run(seed, 1)
        assert plain.wait() == 0
        U, _ = g.trajectory()
        assert np.array_equal(U, plain.trajectory()[0])
    assert np.array_equal(U, oracle.run(spec, 4, 1, nthreads=NTHREADS)["U"])


def test_graph_refused_with_transfers(lib):
    spec = W.sir_with_events(seed=3, Nn=200, days=20)
    m = lib.Model(spec, graph=1)
    with pytest.raises(lib.SiminfError) as e:
        m.run(1, 0)
    assert e.value.code == -2
