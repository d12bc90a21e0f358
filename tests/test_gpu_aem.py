"""GPU parity of the all events method (section 3.4, solver 'aem') against
the oracle's: every built-in model kind, scheduled events with and without
external transfers in the free-running, barrier and dataflow kernels, a
generated three-transition model, graph replay, the first error, and the
full sizes the benchmark times (SIR with events, 10,000 nodes x 365 days,
and the 4,096-run batch, both at their autotuned launch shapes).  U must be
bit-identical and the counters and error keys equal."""
import sys

import numpy as np
import pytest

from paper_1605_01421_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def _run(lib, spec, seed, stream, **opts):
    import oracle
    _say(spec.name, "aem seed", seed, "stream", stream, opts)
    ref = oracle.run(spec, seed, stream, nthreads=16, solver="aem")
    m = lib.Model(spec, solver="aem", **opts)
    m.run(seed, stream)
    return m, ref, m.wait()


def _same(m, ref, what):
    U, V = m.trajectory()
    if not np.array_equal(U, ref["U"]):
        bad = np.argwhere(U != ref["U"])
        raise AssertionError(f"{what}: U differs at {len(bad)} entries, first {bad[:3].tolist()}")
    if V.size:
        assert np.array_equal(V, ref["V"]), what
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


def test_sir_plain(lib):
    spec = W.plain_sir()
    m, ref, rc = _run(lib, spec, 123, 0)
    assert rc == 0 and ref["status"] == 0
    _same(m, ref, "plain SIR")
    assert m.launch_info()["wide"] == 0 and m.launch_info()["group"] == 0


@pytest.mark.parametrize("mode", [1, 2])
def test_sir_with_events(lib, mode):
    spec = W.sir_with_events(seed=7, Nn=1000, days=90)
    m, ref, rc = _run(lib, spec, 49, 5, mode=mode)
    assert rc == 0 and ref["status"] == 0
    _same(m, ref, f"SIR with events mode {mode}")
    assert m.launch_info()["mode"] == mode


def test_sise_without_transfers(lib):
    spec = W.sise_with_events(seed=4, Nn=700, days=200)
    keep = spec.events["event"] != W.EXTTRANS
    spec.events = {k: v[keep] for k, v in spec.events.items()}
    m, ref, rc = _run(lib, spec, 9, 2)
    assert rc == 0 and ref["status"] == 0
    _same(m, ref, "SISe, node events only")
    assert m.launch_info()["mode"] == 0


@pytest.mark.parametrize("kind", ["sis", "birth_death", "immigration_death"])
def test_other_models(lib, kind):
    rng = np.random.default_rng(5)
    if kind == "sis":
        spec = W.sis_spec(np.stack([rng.integers(0, 60, 300), rng.integers(0, 5, 300)], 1), np.arange(0, 31),
                          0.01, 0.2)
    elif kind == "birth_death":
        spec = W.birth_death_spec(rng.integers(0, 40, 300), np.arange(0, 21), 0.2, 0.18)
    else:
        spec = W.birth_death_spec(rng.integers(0, 10, 300), np.arange(0, 21), 2.0, 0.3, immigration=True)
    m, ref, rc = _run(lib, spec, 77, 1)
    assert rc == 0
    _same(m, ref, kind)


def test_generated_model(lib):
    spec = W.mparse_spec(["S -> b*S*I/(S+I+R) -> I", "I -> g*I -> R", "R -> w*R -> S"], ["S", "I", "R"],
                         np.tile([90, 10, 0], (2000, 1)), np.arange(0, 151), gdata=dict(b=0.5, g=0.2, w=0.05))
    m, ref, rc = _run(lib, spec, 17, 3)
    assert rc == 0 and ref["status"] == 0
    _same(m, ref, "generated SIRS")


def test_graph_replay(lib):
    spec = W.plain_sir()
    import oracle
    ref = oracle.run(spec, 8, 2, nthreads=16, solver="aem")
    m = lib.Model(spec, solver="aem", graph=1)
    for r in range(3):
        m.run(8, 2)
        assert m.wait() == 0
        assert np.array_equal(m.trajectory()[0], ref["U"]), r


def test_first_error(lib):
    """A negative compartment after an exit-free transition is impossible;
    a bad rate is not: a negative beta makes the infection rate negative
    on the first day, at the oracle's key."""
    spec = W.sir_spec(np.tile([50, 5, 0], (64, 1)), np.arange(0, 11), -0.5, 0.1)
    m, ref, rc = _run(lib, spec, 1, 0)
    assert rc == ref["status"] == -6
    e = m.error_info()
    assert (e["code"], e["step"], e["phase"], e["index"]) == ref["error"]


def test_lane_queue_refused(lib):
    with pytest.raises(lib.SiminfError) as e:
        lib.Model(W.plain_sir(), solver="aem", lane_queue=1)
    assert e.value.code == -2


def test_sir_events_full_size_autotuned(lib):
    """SIR with scheduled events at full size (10,000 nodes x 365 days,
    469,539 events) at the autotuned launch shape that the benchmark times:
    U bit-exact and the counters equal."""
    import oracle
    spec = W.sir_with_events()
    m = lib.Model(spec, solver="aem")
    best = m.autotune(seed=3, repeats=1)
    _say("autotuned", m.launch_info(), f"{best:.2f} ms")
    m.run(61, 2)
    rc = m.wait()
    ref = oracle.run(spec, 61, 2, nthreads=16, solver="aem")
    assert rc == 0 and ref["status"] == 0
    _same(m, ref, "SIR with events, full size")


def test_batch_full_size_sampled_runs(lib):
    """The 4,096-run batch (64 parameter sets x 64 replicates, weekly sums)
    as the benchmark runs it with the all events method, autotuned and
    replayed from a captured graph: the weekly sums of sampled runs against
    oracle runs of the same streams."""
    import oracle
    sets = W.ensemble_sets(seed=3, n_sets=64, replicates=64)
    m = lib.Model([(s.spec, 64) for s in sets], record=lib.RECORD_SUMS, graph=1, solver="aem")
    best = m.autotune(seed=7, repeats=1)
    _say("batch autotuned", m.launch_info(), f"{best:.1f} ms")
    m.run(83, 0)
    assert m.wait() == 0, m.error_info()
    sums = m.sums()
    for run in (0, 2047, 2048, 4095):
        spec = sets[run // 64].spec
        _say("sampled run", run, spec.name, spec.Nn)
        ref = oracle.run(spec, 83, run, nthreads=16, solver="aem")
        assert ref["status"] == 0
        assert np.array_equal(sums[run, :, :spec.Nc], ref["U"].astype(np.int64).sum(axis=1)), run
