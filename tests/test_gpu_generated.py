"""GPU parity of models given as transition strings (section 5.1): the
kernels compiled at run time for the generated model type against the
oracle's own parse and evaluation.  U must be bit-identical and the counters
and error keys equal."""
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


def _oracle(spec, seed, stream):
    import oracle
    return oracle.run(spec, seed, stream, nthreads=16)


def _check(m, ref, run=0, what=""):
    U, _ = m.trajectory(run)
    if not np.array_equal(U, ref["U"]):
        bad = np.argwhere(U != ref["U"])
        raise AssertionError(f"{what}: U differs at {len(bad)} entries, first (t, node, c) = {bad[:3].tolist()}")


def _run(lib, spec, seed, stream, **opts):
    _say(spec.name, "seed", seed, "stream", stream, opts)
    ref = _oracle(spec, seed, stream)
    m = lib.Model(spec, **opts)
    m.run(seed, stream)
    return m, ref, m.wait()


def test_incidence_example(lib):
    """Section 5.1's incidence example (S, I, Icum, R), 1,000 nodes x 150
    days, free-running kernel, plain and replayed from a graph."""
    spec = W.incidence_sir(n=1000, days=150)
    m, ref, rc = _run(lib, spec, 123, 0)
    assert rc == 0 and ref["status"] == 0
    _check(m, ref, what="incidence")
    c = m.counters()
    assert (c["transitions"], c["node_days"]) == (ref["transitions"], ref["node_days"])
    assert m.launch_info()["mode"] == 0 and m.launch_info()["wide"] == 0
    g = lib.Model(spec, graph=1)
    for r in range(3):
        g.run(123, 0)
        assert g.wait() == 0
        _check(g, ref, what=f"graph replay {r}")


def test_generated_sir_equals_builtin(lib):
    """The generated SIR and the built-in SIR draw the same trajectories
    (nodes that never empty)."""
    u0 = np.tile([99, 5, 0], (2000, 1))
    a = W.mparse_spec(["S -> b*S*I/(S+I+R) -> I", "I -> g*I -> R"], ["S", "I", "R"], u0, np.arange(0, 121),
                      gdata=dict(b=0.16, g=0.077))
    b = W.sir_spec(u0, np.arange(0, 121), 0.16, 0.077)
    ma = lib.Model(a)
    mb = lib.Model(b, lanes=1)
    ma.run(5, 1)
    mb.run(5, 1)
    assert ma.wait() == 0 and mb.wait() == 0
    assert np.array_equal(ma.trajectory()[0], mb.trajectory()[0])


def test_sirs_three_transitions(lib):
    spec = W.mparse_spec(["S -> b*S*I/(S+I+R) -> I", "I -> g*I -> R", "R -> w*R -> S"], ["S", "I", "R"],
                         np.tile([90, 10, 0], (3000, 1)), np.arange(0, 201), gdata=dict(b=0.5, g=0.2, w=0.05))
    m, ref, rc = _run(lib, spec, 77, 2)
    assert rc == 0 and ref["status"] == 0
    _check(m, ref, what="SIRS")
    assert m.counters()["transitions"] == ref["transitions"]


@pytest.mark.parametrize("mode", [1, 2])
def test_event_edge_values(lib, mode):
    """Scheduled events at their edge values on a generated SIR (the select
    and shift tables compiled into the model): proportions 0 and 1, a fixed
    n equal to the selected total, proportions that round half up, events on
    emptied nodes, an enter of n = 0 and an external transfer of a whole
    node."""
    u0 = np.array([[5, 3, 2], [4, 4, 4], [7, 1, 0], [3, 1, 0], [10, 2, 1], [1, 1, 1]], np.int32)
    E_, X, IT, ET = W.ENTER, W.EXIT, W.INTTRANS, W.EXTTRANS
    rows = [(X, 1, 0, 0, 0, 1.0, 3, -1), (X, 1, 1, 0, 0, 0.0, 3, -1), (X, 1, 2, 0, 8, 0.0, 3, -1),
            (IT, 2, 3, 0, 0, 0.5, 0, 0), (ET, 2, 4, 5, 0, 1.0, 3, -1),
            (X, 3, 5, 0, 0, 0.5, 1, -1), (X, 3, 0, 0, 0, 0.5, 3, -1), (E_, 3, 1, 0, 0, 0.0, 0, -1),
            (ET, 3, 2, 3, 0, 0.5, 3, 0), (IT, 4, 4, 0, 0, 1.0, 3, 0)]
    E = np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 1]], np.int32)
    N = np.array([[1], [1], [0]], np.int32)
    # (1 + S + I + R: the emptied nodes would make S*I/(S+I+R) 0/0, an error)
    spec = W.mparse_spec(["S -> b*S*I/(1+S+I+R) -> I", "I -> g*I -> R"], ["S", "I", "R"], u0,
                         np.arange(0, 7), gdata=dict(b=0.16, g=0.077), E=E, N=N, events=W.make_events(rows))
    m, ref, rc = _run(lib, spec, 19, 3, mode=mode)
    assert rc == 0 and ref["status"] == 0
    _check(m, ref, what=f"event edges, generated, mode {mode}")
    c = m.counters()
    assert (c["transitions"], c["events"]) == (ref["transitions"], ref["events"])


@pytest.mark.parametrize("solver", ["ssm", "aem"])
def test_largest_model(lib, solver):
    """A model at the limits of the model compiler: 16 compartments in a
    chain and 32 transitions (a step forward and back between neighbours,
    an immigration into the first and a death from the last), with rates
    that read three global data; both solvers."""
    comps = [f"C{i}" for i in range(16)]
    tr = [f"C{i} -> a*C{i} -> C{i + 1}" for i in range(15)]
    tr += [f"C{i + 1} -> b*C{i + 1}/(1+C{i}) -> C{i}" for i in range(15)]
    tr += ["@ -> m -> C0", "C15 -> 0.05*C15 -> @"]
    assert len(tr) == 32
    rng = np.random.default_rng(9)
    spec = W.mparse_spec(tr, comps, rng.integers(0, 40, size=(60, 16)), np.arange(0, 31),
                         gdata=dict(a=0.3, b=0.2, m=2.5))
    import oracle
    ref = oracle.run(spec, 13, 4, nthreads=16, solver=solver)
    m = lib.Model(spec, solver=solver)
    _say("largest model", solver, m.launch_info())
    m.run(13, 4)
    assert m.wait() == 0 and ref["status"] == 0
    _check(m, ref, what=f"16 x 32 model, {solver}")
    c = m.counters()
    assert (c["transitions"], c["node_days"]) == (ref["transitions"], ref["node_days"])
    assert c["transitions"] > 10000


@pytest.mark.parametrize("mode", [1, 2])
def test_vaccination_example(lib, mode):
    """Section 5.1.2's example: five compartments (S, I, Icum, R, V), births,
    deaths and movements between 1,600 herds, vaccination as internal
    transfers shifted to V, in the barrier (1) and dataflow (2) kernels."""
    spec = W.vaccination_example(infected=16)
    m, ref, rc = _run(lib, spec, 2024, 0, mode=mode)
    assert rc == 0 and ref["status"] == 0
    _check(m, ref, what=f"vaccination mode {mode}")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])
    assert m.launch_info()["mode"] == mode


def test_vaccination_full_size_autotuned(lib):
    """The benchmark's vaccination workload (1,600 herds x 300 days, one
    infected animal) at the launch shape the benchmark times (the
    autotuner's pick): U and counters."""
    spec = W.vaccination_example()
    ref = _oracle(spec, 2026, 4)
    m = lib.Model(spec)
    best = m.autotune(seed=11, repeats=2)
    _say("vaccination, autotuned", m.launch_info(), f"{best:.2f} ms")
    m.run(2026, 4)
    assert m.wait() == 0 and ref["status"] == 0
    _check(m, ref, what=f"autotuned {m.launch_info()}")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


@pytest.mark.parametrize("mode", [1, 2])
def test_age_structured_model(lib, mode):
    """Appendix B's age categories: six compartments and six transitions,
    births, exits per category, ageing by shifted internal transfers, and
    movements."""
    spec = W.age_structured_sis()
    m, ref, rc = _run(lib, spec, 9, 4, mode=mode)
    assert rc == 0 and ref["status"] == 0
    _check(m, ref, what=f"age model mode {mode}")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


def test_invalid_propensity_error_key(lib):
    """An empty herd makes b*S*I/(S+I+R+V) 0/0: the run ends with
    SIMINF_E_BAD_RATE at the oracle's key (step, phase, node)."""
    spec = W.vaccination_example(Nn=200, days=60, infected=5)
    u0 = np.array(spec.u0, copy=True)
    u0[17] = 0
    spec.u0 = u0
    m, ref, rc = _run(lib, spec, 1, 0)
    assert ref["status"] == -6 and rc == -6
    e = m.error_info()
    assert (e["code"], e["step"], e["phase"], e["index"]) == ref["error"]


def test_batch_with_builtin_model(lib):
    """A generated model and a built-in one in one batch (two model groups
    on two streams): every run equals its oracle run."""
    a = W.incidence_sir(n=300, days=80)
    b = W.sir_spec(np.tile([200, 3, 0], (200, 1)), np.arange(1, 81), 0.3, 0.1)
    batch = [(a, 2), (b, 2)]
    m = lib.Model(batch)
    m.run(13, 7)
    assert m.wait() == 0
    r = 0
    for spec, reps in batch:
        for _ in range(reps):
            _check(m, _oracle(spec, 13, 7 + r), run=r, what=f"batch run {r}")
            r += 1


def test_lane_queue_refused(lib):
    with pytest.raises(lib.SiminfError) as e:
        lib.Model(W.incidence_sir(n=100, days=10), lane_queue=1)
    assert e.value.code == -2
