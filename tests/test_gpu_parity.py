"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer trajectories must be bit-identical, counters equal, and the real
state V within 1e-12 relative (the same IEEE operations are performed, so
it is expected to be exact as well)."""
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


def _compare(model, ref, run=0, what=""):
    U, V = model.trajectory(run)
    if not np.array_equal(U, ref["U"]):
        bad = np.argwhere(U != ref["U"])
        raise AssertionError(f"{what}: U differs at {len(bad)} entries, first (t, node, c) = {bad[:3].tolist()}")
    if V.size:
        np.testing.assert_allclose(V, ref["V"], rtol=1e-12, atol=0, err_msg=what)


def _run_both(lib, spec, seed, stream=0, **opts):
    _say(spec.name, "seed", seed, "stream", stream, opts)
    ref = oracle_run(spec, seed, stream)
    m = lib.Model(spec, **opts)
    m.run(seed, stream)
    rc = m.wait()
    return m, ref, rc


def oracle_run(spec, seed, stream):
    import oracle
    return oracle.run(spec, seed, stream, nthreads=NTHREADS)


def test_plain_sir_100_nodes(lib):
    spec = W.plain_sir()
    m, ref, rc = _run_both(lib, spec, 123)
    assert rc == 0 and ref["status"] == 0
    _compare(m, ref, what="sir-100")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], 0)
    assert m.launch_info()["mode"] == 0


@pytest.mark.parametrize("infect", [False, True])
def test_paper_five_node_event_example(lib, infect):
    spec = W.sir_event_example(infect)
    for stream in range(4):
        for mode in (1, 2):
            m, ref, rc = _run_both(lib, spec, 3, stream, mode=mode)
            assert rc == 0
            _compare(m, ref, what=f"five-node stream {stream} mode {mode}")
            assert m.counters()["events"] == ref["events"]
            assert m.launch_info()["mode"] == mode


@pytest.mark.parametrize("Nn,days,seed", [(257, 40, 1), (1000, 90, 7)])
def test_sir_with_events_small(lib, Nn, days, seed):
    spec = W.sir_with_events(seed=seed, Nn=Nn, days=days)
    m, ref, rc = _run_both(lib, spec, 42 + seed, 5)
    assert rc == 0 and ref["status"] == 0
    _compare(m, ref, what=spec.name)
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


@pytest.mark.parametrize("mode", [1, 2])
def test_sise_with_events_small(lib, mode):
    spec = W.sise_with_events(seed=4, Nn=700, days=200)
    m, ref, rc = _run_both(lib, spec, 9, 2, mode=mode)
    assert rc == 0 and ref["status"] == 0
    _compare(m, ref, what=spec.name)
    assert np.array_equal(m.trajectory()[1], ref["V"]), "phi expected bit-identical"


@pytest.mark.parametrize("kind", ["sis", "birth_death", "immigration_death", "sise_noevents"])
def test_other_models(lib, kind):
    rng = np.random.default_rng(5)
    if kind == "sis":
        spec = W.sis_spec(np.stack([rng.integers(0, 60, 300), rng.integers(0, 5, 300)], 1), np.arange(0, 31),
                          0.01, 0.2)
    elif kind == "birth_death":
        spec = W.birth_death_spec(rng.integers(0, 40, 300), np.arange(0, 21), 0.2, 0.18)
    elif kind == "immigration_death":
        spec = W.birth_death_spec(rng.integers(0, 10, 300), np.arange(0, 21), 2.0, 0.3, immigration=True)
    else:
        spec = W.sise_spec(np.stack([rng.integers(0, 80, 300), rng.integers(0, 8, 300)], 1),
                           np.arange(0, 400, 3), 0.0175, 0.1, 1.0, (0.1, 0.12, 0.1, 0.11))
    m, ref, rc = _run_both(lib, spec, 77, 1)
    assert rc == 0
    _compare(m, ref, what=kind)
    assert m.counters()["transitions"] == ref["transitions"]


@pytest.mark.parametrize("opts", [dict(block=64), dict(block=128), dict(block=256), dict(order=1),
                                  dict(mode=1), dict(mode=1, max_blocks=3), dict(mode=1, block=64, max_blocks=1),
                                  dict(mode=2, block=128), dict(pipeline=1), dict(pipeline=2),
                                  dict(mode=1, pipeline=2), dict(max_blocks=1, block=64),
                                  dict(lanes=1), dict(lanes=64, wide=1), dict(lanes=64, wide=40),
                                  dict(lanes=64, wide=600, block=256), dict(lanes=64, wide=7, block=128, pipeline=2),
                                  dict(lanes=64, wide=600, lattice=2), dict(lanes=64, wide=600, mode=1, lattice=1),
                                  dict(lanes=64, wide=90, block=64, lattice=2), dict(pipeline=2, block=128),
                                  dict(pack=16), dict(pack=32, block=128), dict(pack=16, mode=2, lanes=1),
                                  dict(pack=16, lanes=64, wide=40, block=256), dict(pack=32, mode=1),
                                  dict(pack=8, lanes=64, wide=90, block=64), dict(pack=4, block=128, pipeline=2),
                                  dict(group=-1, lanes=1), dict(group=-1, lanes=64, wide=40, pack=8),
                                  dict(group=200, mode=2, block=128), dict(group=-1, mode=1),
                                  dict(group=77, pipeline=2, block=256, pack=16)])
def test_launch_shape_does_not_change_bits(lib, opts):
    spec = W.sir_with_events(seed=11, Nn=600, days=50)
    ref = oracle_run(spec, 5, 0)
    m = lib.Model(spec, **opts)
    _say("launch", opts, m.launch_info())
    m.run(5, 0)
    assert m.wait() == 0
    _compare(m, ref, what=str(opts))
    free = W.plain_sir()
    ref0 = oracle_run(free, 8, 3)
    m0 = lib.Model(free, **opts)
    m0.run(8, 3)
    assert m0.wait() == 0
    _compare(m0, ref0, what="free " + str(opts))


@pytest.mark.parametrize("mode", [1, 2])
def test_batch_with_transfers_on_groups(lib, mode):
    """Runs with external transfers batched in one launch, every node on a
    group of lanes (dataflow kernel) or the barrier kernel, against the
    oracle run by run."""
    specs = [W.sir_with_events(seed=s, Nn=nn, days=45) for s, nn in ((5, 300), (9, 170))]
    batch = [(specs[0], 2), (specs[1], 1)]
    m = lib.Model(batch, group=-1, pack=8, mode=mode)
    info = m.launch_info()
    _say("batch with transfers", mode, info)
    assert (info["group"] > 0) == (mode == 2)
    m.run(13, 7)
    assert m.wait() == 0
    r = 0
    for spec, reps in batch:
        for _ in range(reps):
            ref = oracle_run(spec, 13, 7 + r)
            _compare(m, ref, run=r, what=f"batch run {r}")
            r += 1


def test_batch_equals_individual_runs(lib):
    a = W.sir_spec(np.tile([200, 3, 0], (70, 1)), np.arange(0, 41), 0.3, 0.1)
    b = W.sise_spec(np.tile([90, 6], (45, 1)), np.arange(0, 41), 0.02, 0.1, 1.0, (0.1, 0.12, 0.1, 0.11))
    c = W.sir_spec(np.tile([50, 1, 0], (33, 1)), np.arange(0, 41), 0.5, 0.2)
    batch = [(a, 3), (b, 2), (c, 2)]
    m = lib.Model(batch)
    _say("batch full", m.runs)
    m.run(21, 100)
    assert m.wait() == 0
    r = 0
    for spec, reps in batch:
        for _ in range(reps):
            ref = oracle_run(spec, 21, 100 + r)
            _compare(m, ref, run=r, what=f"batch run {r}")
            r += 1
    ms = lib.Model(batch, record=lib.RECORD_SUMS)
    _say("batch sums")
    ms.run(21, 100)
    assert ms.wait() == 0
    sums = ms.sums()
    r = 0
    for spec, reps in batch:
        for _ in range(reps):
            ref = oracle_run(spec, 21, 100 + r)
            want = ref["U"].astype(np.int64).sum(axis=1)
            assert np.array_equal(sums[r, :, :want.shape[1]], want), r
            r += 1


def test_prevalence_quantiles(lib):
    import oracle.prevalence as P
    sets = W.ensemble_sets(seed=9, n_sets=4, replicates=8, days=56, nn_range=(100, 400))
    m = lib.Model([(s.spec, s.replicates) for s in sets], record=lib.RECORD_SUMS)
    m.run(1234, 0)
    assert m.wait() == 0
    sums = m.sums()
    q = m.prevalence_quantiles(1, (0, 1), 8, 1, m.ntspan - 1).cpu().numpy()
    want = P.prevalence_quantiles(sums, 1, (0, 1), 8, 1, m.ntspan - 1, (0.1, 0.5, 0.9))
    assert np.array_equal(q, want)
    # and the sums themselves against oracle runs of two sampled replicates
    for r in (0, 13):
        spec = sets[r // 8].spec
        ref = oracle_run(spec, 1234, r)
        assert np.array_equal(sums[r, :, :spec.Nc], ref["U"].astype(np.int64).sum(axis=1))


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("group", [0, -1])
@pytest.mark.parametrize("case", ["overdraw_e1", "overdraw_e2", "negative_rate"])
def test_first_error_matches_oracle(lib, case, mode, group):
    u0 = np.array([[5, 0, 0], [5, 0, 0], [5, 0, 0]])
    beta = 0.0
    if case == "overdraw_e1":
        rows = [(W.EXIT, 3, 1, 0, 2, 0.0, 0, -1), (W.EXIT, 3, 2, 0, 9, 0.0, 0, -1),
                (W.EXIT, 3, 0, 0, 6, 0.0, 3, -1)]
    elif case == "overdraw_e2":
        rows = [(W.EXTTRANS, 2, 0, 1, 5, 0.0, 0, -1), (W.EXTTRANS, 2, 0, 2, 1, 0.0, 0, -1),
                (W.EXTTRANS, 2, 1, 2, 11, 0.0, 0, -1)]
    else:
        u0 = np.array([[5, 1, 0], [5, 0, 0], [5, 2, 0]])
        beta = -0.1
        rows = []
    spec = W.sir_spec(u0, [0, 1, 2, 3, 4], beta, 0.1, events=W.make_events(rows))
    m, ref, rc = _run_both(lib, spec, 1, 0, mode=mode, group=group, lanes=1 if group else 0)
    info = m.error_info()
    assert rc == ref["status"] != 0
    assert (info["code"], info["step"], info["phase"], info["index"]) == ref["error"]


@pytest.mark.parametrize("opts", [dict(pack=2), dict(pack=48), dict(block=96), dict(lanes=2), dict(lattice=3)])
def test_invalid_options_rejected(lib, opts):
    spec = W.plain_sir()
    with pytest.raises(lib.SiminfError) as e:
        lib.Model(spec, **opts)
    assert e.value.code in (-1, -2)


def test_invalid_event_rejected_at_create(lib):
    spec = W.sir_spec(np.array([[5, 0, 0]]), [0, 1], 0.1, 0.1,
                      events=W.make_events([(W.EXIT, 1, 0, 0, 1, 0.0, 9, -1)]))
    with pytest.raises(lib.SiminfError) as e:
        lib.Model(spec)
    assert e.value.code == -8


def test_trajectory_to_device(lib):
    import torch
    spec = W.sir_event_example(True)
    m, ref, rc = _run_both(lib, spec, 3, 1)
    U, V = m.trajectory(device=True)
    assert U.is_cuda and np.array_equal(U.cpu().numpy(), ref["U"])


@pytest.mark.parametrize("mode", [1, 2])
def test_sir_events_full_size(lib, mode):
    """10,000 nodes, 365 days, the benchmark workload: whole trajectory."""
    spec = W.sir_with_events()
    _say("SIR with events, full size", spec.Nn, len(spec.events["time"]))
    m, ref, rc = _run_both(lib, spec, 2024, 0, mode=mode)
    assert rc == 0 and ref["status"] == 0
    _compare(m, ref, what="SIR with events, full size")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


def test_sir_events_full_size_autotuned(lib):
    """The benchmark workload at the launch shape the benchmark times (the
    autotuner's pick): whole trajectory and counters."""
    spec = W.sir_with_events()
    ref = oracle_run(spec, 2025, 3)
    m = lib.Model(spec)
    best = m.autotune(seed=11, repeats=2)
    _say("SIR with events, full size, autotuned", m.launch_info(), f"{best:.3f} ms")
    m.run(2025, 3)
    assert m.wait() == 0 and ref["status"] == 0
    _compare(m, ref, what=f"autotuned {m.launch_info()}")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


def test_autotune_keeps_bits(lib):
    spec = W.sir_with_events(seed=13, Nn=800, days=45)
    ref = oracle_run(spec, 77, 2)
    m = lib.Model(spec)
    _say("autotune")
    best = m.autotune(seed=5, repeats=1)
    assert best > 0
    m.run(77, 2)
    assert m.wait() == 0
    _compare(m, ref, what=f"autotuned {m.launch_info()}")


def test_wait_limit_abandons_run_cleanly(lib):
    """A destination that must wait longer than options.wait_ms for its
    source ends the run with SIMINF_E_DEVICE (node 0 makes about 10^6
    transitions on day 1 before it can send; node 1 waits for it with a 1 ms
    limit).  Every kernel exits normally, and a model with the default limit
    then reproduces the oracle."""
    u0 = np.array([[500000, 500000, 0], [10, 0, 0]])
    ev = W.make_events([(W.EXTTRANS, 1, 0, 1, 1, 0.0, 0, -1)])
    spec = W.sir_spec(u0, [0, 1, 2], 1.0, 1.0, events=ev)
    m = lib.Model(spec, mode=2, wait_ms=1)
    _say("wait limit 1 ms", m.launch_info())
    m.run(3, 0)
    assert m.wait() == -4
    m2, ref, rc = _run_both(lib, spec, 3, 0, mode=2)
    assert rc == 0 and ref["status"] == 0
    _compare(m2, ref, what="after an abandoned run")


@pytest.mark.parametrize("lattice", [1, 2])
@pytest.mark.parametrize("case", ["extinction", "immigration", "sise", "sir_heavy", "neg_state", "bad_rate",
                                  "step_limit", "step_limit_full_g"])
def test_wide_node_paths(lib, case, lattice):
    """Every node on its own wavefront (lanes=64, wide=Nn), with the lattice
    walk (1) and the plain dependent chain (2): stops at lambda = 0 inside a
    window, thousands of steps per day, the SISe rates, an epidemic's
    turnover, a negative compartment after a transition, a bad rate, and the
    2^24-step guard (in both paths), all against the oracle (state, counters,
    error key)."""
    spec = _path_case(case)
    Nn = np.asarray(spec.u0).shape[0]
    m, ref, rc = _run_both(lib, spec, 23, 4, lanes=64, wide=Nn, lattice=lattice)
    info = m.launch_info()
    assert info["wide"] == Nn
    _check_path_case(m, ref, rc, case)


@pytest.mark.parametrize("case", ["extinction", "immigration", "sise", "sir_heavy", "neg_state", "bad_rate",
                                  "step_limit", "step_limit_full_g"])
def test_group_node_paths(lib, case):
    """The same cases with every node on a group of 8 lanes (eight nodes to
    a wavefront, the lattice walk three steps per pass); the immigration
    models, whose G does not mark both rates, fall back to one lane."""
    spec = _path_case(case)
    Nn = np.asarray(spec.u0).shape[0]
    m, ref, rc = _run_both(lib, spec, 23, 4, lanes=1, group=-1)
    info = m.launch_info()
    assert info["group"] == (0 if case in ("immigration", "step_limit") else Nn), info
    _check_path_case(m, ref, rc, case)


def _check_path_case(m, ref, rc, case):
    assert rc == ref["status"]
    if rc:
        e = m.error_info()
        assert (e["code"], e["step"], e["phase"], e["index"]) == ref["error"]
        return
    _compare(m, ref, what=case)
    c = m.counters()
    assert (c["transitions"], c["node_days"]) == (ref["transitions"], ref["node_days"])


def _path_case(case):
    rng = np.random.default_rng(17)
    tspan = np.arange(0, 6)
    if case == "extinction":
        spec = W.birth_death_spec(rng.integers(50, 400, 40), tspan, 0.5, 1.2)
    elif case == "immigration":
        spec = W.birth_death_spec(rng.integers(0, 10, 20), tspan, 3000.0, 0.7, immigration=True)
    elif case == "sise":
        spec = W.sise_spec(np.stack([rng.integers(1000, 20000, 20), rng.integers(0, 3000, 20)], 1),
                           np.arange(0, 40), 0.0175, 0.1, 1.0, (0.1, 0.12, 0.1, 0.11))
    elif case == "sir_heavy":
        spec = W.sir_spec(np.stack([rng.integers(2000, 9000, 20), rng.integers(1, 50, 20),
                                    np.zeros(20, int)], 1), np.arange(0, 60), 0.3, 0.1)
    elif case == "neg_state":
        spec = W.sir_spec(np.array([[500, 20, 0], [300, 4, 3]]), tspan, 0.4, 0.1)
        spec.S = np.array([[-1, 0], [1, -1], [-1, 1]])   # an infection also removes a recovered
    elif case == "bad_rate":
        spec = W.sir_spec(np.array([[500, 20, 0], [300, 4, 3]]), tspan, -0.4, 0.1)
    elif case == "step_limit_full_g":
        # SIS marks both rates after either transition, so the lattice walk
        # runs into the 2^24-draw guard (about 1e8 transitions per day)
        spec = W.sis_spec(np.array([[100000, 100000]]), np.arange(0, 2), 0.01, 0.5)
    else:
        spec = W.birth_death_spec(np.array([0, 0]), np.arange(0, 2), 3.0e7, 0.0, immigration=True)
    return spec


def _no_transfers(spec):
    ev = {k: np.asarray(v)[np.asarray(spec.events["event"]) != W.EXTTRANS] for k, v in spec.events.items()}
    return W.sir_spec(np.asarray(spec.u0), np.asarray(spec.tspan), 0.16, 0.077, events=ev, name="no-transfers")


@pytest.mark.parametrize("pipeline", [1, 2])
@pytest.mark.parametrize("case", ["events", "batch_sums", "batch_full", "error"])
def test_free_running_cases(lib, case, pipeline):
    """Runs without external transfers, with the next step's random numbers
    computed ahead (pipeline 1) or not (2): node-local events, full records,
    weekly sums over uneven runs and a failing node, against the oracle."""
    if case == "events":
        spec = _no_transfers(W.sir_with_events(seed=21, Nn=900, days=80))
        m, ref, rc = _run_both(lib, spec, 41, 3, pipeline=pipeline)
        assert rc == 0 and ref["status"] == 0
        _compare(m, ref, what=case)
        c = m.counters()
        assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])
        return
    if case == "error":
        u0 = np.array([[500, 20, 0]] * 70 + [[50, 5, 0]])
        spec = W.sir_spec(u0, np.arange(0, 12), 0.3, 0.1,
                          events=W.make_events([(W.ENTER, 6, 70, 0, 3, 0.0, 0, -1),
                                                (W.EXIT, 8, 70, 0, 400, 0.0, 0, -1)]))
        m, ref, rc = _run_both(lib, spec, 5, 0, pipeline=pipeline)
        info = m.error_info()
        assert rc == ref["status"] != 0
        assert (info["code"], info["step"], info["phase"], info["index"]) == ref["error"]
        return
    sets = W.ensemble_sets(seed=31, n_sets=6, replicates=3, days=70, nn_range=(60, 700))
    batch = [(st.spec, 3) for st in sets]
    record = lib.RECORD_SUMS if case == "batch_sums" else lib.RECORD_FULL
    m = lib.Model(batch, record=record, pipeline=pipeline)
    _say(case, m.runs, m.launch_info())
    m.run(17, 50)
    assert m.wait() == 0
    sums = m.sums() if record == lib.RECORD_SUMS else None
    for r in range(m.runs):
        spec = sets[r // 3].spec
        ref = oracle_run(spec, 17, 50 + r)
        if sums is not None:
            assert np.array_equal(sums[r, :, :spec.Nc], ref["U"].astype(np.int64).sum(axis=1)), r
        else:
            _compare(m, ref, run=r, what=f"batch run {r}")


@pytest.mark.parametrize("pack,group", [(4, 0), (16, 0), (32, 0), (64, -1), (8, 150)])
def test_packed_wavefronts_batch(lib, pack, group):
    """Fewer nodes per wavefront (the rest of its lanes idle), or nodes on
    groups of lanes: weekly sums of a batch whose runs straddle wavefronts,
    and the launch reports it."""
    sets = W.ensemble_sets(seed=37, n_sets=4, replicates=2, days=60, nn_range=(20, 300))
    batch = [(st.spec, 2) for st in sets]
    m = lib.Model(batch, record=lib.RECORD_SUMS, pack=pack, group=group)
    info = m.launch_info()
    _say("packed batch", pack, group, info)
    assert info["pack"] == pack
    assert (info["group"] > 0) == (group != 0)
    m.run(29, 4)
    assert m.wait() == 0
    sums = m.sums()
    for r in range(m.runs):
        spec = sets[r // 2].spec
        ref = oracle_run(spec, 29, 4 + r)
        assert np.array_equal(sums[r, :, :spec.Nc], ref["U"].astype(np.int64).sum(axis=1)), r


def _expected_auto_pack(info, Nn, cus, smallest):
    """The automatic packing rule, restated from the option's documentation."""
    major = info["wide"] + -(-info["group"] // 8)
    rest = Nn - info["wide"] - info["group"]
    pack = 64
    if major + -(-rest // 64) < cus:
        while pack > smallest and major + -(-rest // pack) < 4 * cus:
            pack //= 2
    return pack


@pytest.mark.parametrize("case", ["transfers-600", "generated-800", "aem-2000"])
def test_automatic_packing(lib, case):
    """With no launch option a model with fewer 64-node wavefronts than the
    device has CUs packs fewer nodes to a wavefront; the results stay the
    oracle's."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    solver = "ssm"
    if case == "transfers-600":
        spec = W.sir_with_events(seed=8, Nn=600, days=60)
    elif case == "generated-800":
        spec = W.vaccination_example(seed=4, Nn=800, days=60, infected=20)
    else:
        spec = W.sir_with_events(seed=9, Nn=2000, days=40)
        solver = "aem"
    m = lib.Model(spec, solver=solver)
    info = m.launch_info()
    _say("automatic packing", case, info, "CUs", cus)
    assert info["pack"] == _expected_auto_pack(info, spec.Nn, cus, 4)
    one_lane = spec.Nn - info["wide"] - info["group"]
    if case != "transfers-600":
        assert one_lane == spec.Nn  # one lane per node: no wide or grouped nodes
    if one_lane > 0 and info["wide"] + -(-info["group"] // 8) + -(-one_lane // 64) < cus:
        assert info["pack"] < 64
    m.run(23, 6)
    assert m.wait() == 0
    import oracle
    ref = oracle.run(spec, 23, 6, nthreads=NTHREADS, solver=solver)
    _compare(m, ref, what=case)


def _degenerate_spec(kind):
    u0 = np.array([[90, 10, 0], [50, 5, 0], [0, 0, 0], [400, 3, 1]], np.int32)
    if kind == "no_nodes":
        return W.sir_spec(np.zeros((0, 3), np.int32), np.arange(0, 11, dtype=float))
    if kind == "no_nodes_sise":
        return W.sise_spec(np.zeros((0, 2), np.int32), np.arange(0, 5, dtype=float), 0.01, 0.1, 1.0,
                           (0.1, 0.12, 0.1, 0.11))
    if kind == "one_tspan":
        return W.sir_spec(u0, np.array([0.0]))
    if kind == "one_tspan_late":
        return W.sir_spec(u0, np.array([7.0]))
    return W.sir_spec(u0, np.arange(0, 21, dtype=float))


@pytest.mark.parametrize("case", ["no_nodes", "no_nodes_sise", "one_tspan", "one_tspan_late"])
def test_degenerate_sizes(lib, case):
    """A model without nodes runs and records nothing; a single tspan point
    records the initial state and simulates no day."""
    spec = _degenerate_spec(case)
    m, ref, rc = _run_both(lib, spec, 5, 1)
    assert rc == 0 and ref["status"] == 0
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])
    if spec.Nn == 0:
        U, V = m.trajectory()
        assert U.size == 0 and V.size == 0 and c["node_days"] == 0
    else:
        _compare(m, ref, what=case)
        assert np.array_equal(ref["U"][0], spec.u0)


@pytest.mark.parametrize("lane_queue", [2, 1])
def test_batch_with_an_empty_spec(lib, lane_queue):
    """A ragged batch with a spec of no nodes between two others: every run
    equals the oracle's run of its stream (full records without the lane
    queue, weekly-style sums with it)."""
    a = W.sir_with_events(seed=3, Nn=300, days=30)
    a.events = W.empty_events()
    b = W.sir_spec(np.array([[900, 100, 0], [30, 2, 0]], np.int32), a.tspan)
    empty = W.sir_spec(np.zeros((0, 3), np.int32), a.tspan)
    batch = [(a, 2), (empty, 2), (b, 3)]
    record = lib.RECORD_FULL if lane_queue == 2 else lib.RECORD_SUMS
    m = lib.Model(batch, record=record, lane_queue=lane_queue)
    _say("batch with an empty spec", m.launch_info())
    m.run(41, 9)
    assert m.wait() == 0
    specs = [a, a, empty, empty, b, b, b]
    sums = m.sums() if record == lib.RECORD_SUMS else None
    for r, spec in enumerate(specs):
        ref = oracle_run(spec, 41, 9 + r)
        if sums is not None:
            want = ref["U"].astype(np.int64).sum(axis=1) if spec.Nn else np.zeros((len(spec.tspan), 3), np.int64)
            assert np.array_equal(sums[r, :, :3], want), r
        elif spec.Nn:
            _compare(m, ref, run=r, what=f"batch run {r}")
        else:
            U, V = m.trajectory(r)
            assert U.size == 0, r


def _event_edges_spec(rates):
    """Events at their edge values on six nodes: proportions 0 and 1, a
    fixed n equal to the selected total, proportions that round half up
    (0.5 of 3, twice), events on nodes that an earlier event emptied, an
    enter of n = 0, and an external transfer of a whole node."""
    u0 = np.array([[5, 3, 2], [4, 4, 4], [7, 1, 0], [3, 1, 0], [10, 2, 1], [1, 1, 1]], np.int32)
    E, X, IT, ET = W.ENTER, W.EXIT, W.INTTRANS, W.EXTTRANS
    rows = [(X, 1, 0, 0, 0, 1.0, 3, -1), (X, 1, 1, 0, 0, 0.0, 3, -1), (X, 1, 2, 0, 8, 0.0, 3, -1),
            (IT, 2, 3, 0, 0, 0.5, 0, 0), (ET, 2, 4, 5, 0, 1.0, 3, -1),
            (X, 3, 5, 0, 0, 0.5, 1, -1), (X, 3, 0, 0, 0, 0.5, 3, -1), (E, 3, 1, 0, 0, 0.0, 0, -1),
            (ET, 3, 2, 3, 0, 0.5, 3, 0), (IT, 4, 4, 0, 0, 1.0, 3, 0)]
    beta, gamma = (0.16, 0.077) if rates else (0.0, 0.0)
    spec = W.sir_spec(u0, np.arange(0, 7, dtype=float), beta, gamma, events=W.make_events(rows))
    spec.N = np.array([[1], [1], [0]], np.int32)  # shift: S -> I, I -> R
    return spec


@pytest.mark.parametrize("rates", [False, True])
@pytest.mark.parametrize("opts", [dict(mode=1), dict(mode=2, lanes=1), dict(mode=2, lanes=64, wide=6),
                                  dict(mode=2, lanes=1, group=-1)])
def test_event_edge_values(lib, rates, opts):
    spec = _event_edges_spec(rates)
    m, ref, rc = _run_both(lib, spec, 19, 3, **opts)
    assert rc == 0 and ref["status"] == 0
    _compare(m, ref, what=f"event edges {opts}")
    c = m.counters()
    assert (c["transitions"], c["events"]) == (ref["transitions"], ref["events"])
    if not rates:
        U = ref["U"]
        assert U[1, 0].sum() == 0 and (U[1, 1] == [4, 4, 4]).all() and U[1, 2].sum() == 0
        assert (U[2, 3] == [1, 3, 0]).all() and U[2, 4].sum() == 0 and (U[2, 5] == [11, 3, 2]).all()


@pytest.mark.parametrize("rates", [False, True])
@pytest.mark.parametrize("opts", [dict(lane_queue=1), dict(lane_queue=2), dict(lane_queue=2, lanes=64, wide=6)])
def test_event_edge_values_free_running(lib, rates, opts):
    """The same edge values without the external transfers, in the
    free-running kernels (the lane queue, the lockstep kernel, wide nodes)."""
    spec = _event_edges_spec(rates)
    keep = spec.events["event"] != W.EXTTRANS
    spec.events = {k: v[keep] for k, v in spec.events.items()}
    m, ref, rc = _run_both(lib, spec, 23, 1, **opts)
    assert rc == 0 and ref["status"] == 0
    _compare(m, ref, what=f"event edges, free running {opts}")
    c = m.counters()
    assert (c["transitions"], c["events"]) == (ref["transitions"], ref["events"])


@pytest.mark.parametrize("opts", [dict(mode=1), dict(mode=2)])
def test_event_edge_values_all_events_method(lib, opts):
    """The edge values with the all events method (one lane per node)."""
    import oracle
    spec = _event_edges_spec(True)
    ref = oracle.run(spec, 29, 2, nthreads=NTHREADS, solver="aem")
    m = lib.Model(spec, solver="aem", **opts)
    m.run(29, 2)
    assert m.wait() == 0 and ref["status"] == 0
    _compare(m, ref, what=f"event edges, aem {opts}")
    c = m.counters()
    assert (c["transitions"], c["events"]) == (ref["transitions"], ref["events"])


def test_split_run_equals_full_run(lib):
    """Draws are keyed by the absolute day: running [0, 40] and then
    [40, 90] from the saved state equals one run over [0, 90] on the GPU
    (SIR and SISe, with phi carried over)."""
    def go(spec, seed, stream):
        m = lib.Model(spec)
        m.run(seed, stream)
        assert m.wait() == 0
        return m.trajectory()
    u0 = np.tile([300, 5, 0], (50, 1))
    U, _ = go(W.sir_spec(u0, np.arange(0, 91), 0.3, 0.1), 11, 2)
    U1, _ = go(W.sir_spec(u0, np.arange(0, 41), 0.3, 0.1), 11, 2)
    U2, _ = go(W.sir_spec(U1[-1], np.arange(40, 91), 0.3, 0.1), 11, 2)
    assert np.array_equal(U[:41], U1) and np.array_equal(U[40:], U2)
    su = np.tile([60, 4], (30, 1))
    bq = (0.1, 0.12, 0.1, 0.11)
    F, FV = go(W.sise_spec(su, np.arange(0, 91), 0.02, 0.1, 1.0, bq), 3, 0)
    S1, S1V = go(W.sise_spec(su, np.arange(0, 41), 0.02, 0.1, 1.0, bq), 3, 0)
    S2, S2V = go(W.sise_spec(S1[-1], np.arange(40, 91), 0.02, 0.1, 1.0, bq, phi0=S1V[-1, :, 0]), 3, 0)
    assert np.array_equal(F[40:], S2) and np.array_equal(FV[40:], S2V)


def _without_transfers(spec):
    keep = np.asarray(spec.events["event"]) != W.EXTTRANS
    ev = {k: np.asarray(v)[keep] for k, v in spec.events.items()}
    out = W.sir_spec(np.asarray(spec.u0), np.asarray(spec.tspan), 0.16, 0.077, events=ev,
                     name=spec.name + "-no-transfers")
    out.E, out.N = spec.E, spec.N
    return out


@pytest.mark.parametrize("opts", [dict(mode=1), dict(mode=2, lanes=1), dict(mode=2, lanes=64, wide=8),
                                  dict(mode=2, lanes=1, group=-1), dict(mode=2, lanes=64, wide=8, group=-1),
                                  dict(mode=2, lanes=64, wide=8, group=-1, lattice=2)])
def test_internal_and_shifted_transfers(lib, opts):
    """Section 3.3 and Table 2 on the GPU: internal transfers with the shift
    matrix N (proportional and fixed counts), shifted external transfers,
    proportional exits and transfers (n = 0), enters into a two-row select
    column and transfers from a node to itself, in the grid-barrier and the
    dataflow kernels, with the heaviest nodes on a wavefront or on a group of
    lanes; bit-exact against the oracle (state, counters)."""
    spec = W.sir_with_shifts(seed=6)
    m, ref, rc = _run_both(lib, spec, 29, 2, **opts)
    assert rc == 0 and ref["status"] == 0
    info = m.launch_info()
    assert info["mode"] == opts["mode"], info
    if opts["mode"] == 2 and opts.get("lanes") == 64:
        assert info["wide"] == 8, info
    _compare(m, ref, what=f"shifts {opts}")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


@pytest.mark.parametrize("opts", [dict(lanes=1), dict(lanes=64, wide=8), dict(lanes=1, group=-1),
                                  dict(lanes=64, wide=8, group=-1)])
def test_internal_transfers_free_running(lib, opts):
    """The same events without the external transfers, in the free-running
    kernel: internal transfers with shifts applied by one lane, a wavefront
    or a group of lanes, bit-exact against the oracle."""
    spec = _without_transfers(W.sir_with_shifts(seed=7))
    m, ref, rc = _run_both(lib, spec, 31, 9, **opts)
    assert rc == 0 and ref["status"] == 0
    assert m.launch_info()["mode"] == 0
    _compare(m, ref, what=f"internal transfers {opts}")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


# ---- lane queue: every lane advances its own node ---------------------------

@pytest.mark.parametrize("block,chunk,lqb,pipeline", [(64, 64, 1, 2), (256, 512, 16, 1), (128, 1024, 64, 2),
                                                      (128, 256, 8, 1)])
def test_lane_queue_batch_sums(lib, block, chunk, lqb, pipeline):
    """Weekly sums of an uneven batch (SIR and SISe sets, many nodes that
    start without infection and finish at once) from the lane-queue kernel,
    against oracle runs of every replicate; counters against the lockstep
    kernel (draws included) and the oracle."""
    sets = W.ensemble_sets(seed=41, n_sets=8, replicates=3, days=80, nn_range=(50, 900))
    batch = [(st.spec, 3) for st in sets]
    m = lib.Model(batch, record=lib.RECORD_SUMS, lane_queue=1, block=block, chunk=chunk, batch=lqb,
                  pipeline=pipeline)
    info = m.launch_info()
    _say("lane queue", info)
    assert info["mode"] == 3 and info["chunk"] == chunk and info["block"] == block, info
    assert info["batch"] == lqb and info["pipeline"] == (1 if pipeline == 1 else 0), info
    m.run(19, 7)
    assert m.wait() == 0, m.error_info()
    sums = m.sums()
    c = m.counters()
    lock = lib.Model(batch, record=lib.RECORD_SUMS, lane_queue=2)
    assert lock.launch_info()["mode"] == 0
    lock.run(19, 7)
    assert lock.wait() == 0
    assert np.array_equal(sums, lock.sums())
    assert c == lock.counters()
    tr = nd = 0
    for r in range(m.runs):
        spec = sets[r // 3].spec
        ref = oracle_run(spec, 19, 7 + r)
        assert np.array_equal(sums[r, :, :spec.Nc], ref["U"].astype(np.int64).sum(axis=1)), r
        tr += ref["transitions"]
        nd += ref["node_days"]
    assert (c["transitions"], c["node_days"]) == (tr, nd)


@pytest.mark.parametrize("pipeline", [1, 2])
@pytest.mark.parametrize("case", ["shifts", "sise_events", "birth_death"])
def test_lane_queue_full_records(lib, case, pipeline):
    """Whole trajectories from the lane-queue kernel with node-local events
    (internal transfers with shifts, proportional exits, two-row enters),
    SISe with events (phi bit-identical) and linear birth-death nodes that die
    out, bit-exact against the oracle."""
    if case == "shifts":
        spec = _without_transfers(W.sir_with_shifts(seed=8, Nn=700, days=50))
    elif case == "sise_events":
        full = W.sise_with_events(seed=12, Nn=900, days=120)
        keep = np.asarray(full.events["event"]) != W.EXTTRANS
        ev = {k: np.asarray(v)[keep] for k, v in full.events.items()}
        spec = W.sise_spec(full.u0, full.tspan, 0.0175, 0.1, 1.0, (0.1, 0.12, 0.1, 0.11), events=ev,
                           name="sise-node-events")
    else:
        spec = W.birth_death_spec(np.random.default_rng(5).integers(0, 40, 1500), np.arange(0, 30), 0.3, 0.4)
    m, ref, rc = _run_both(lib, spec, 37, 11, lane_queue=1, chunk=128, block=128, pipeline=pipeline)
    assert m.launch_info()["mode"] == 3
    assert rc == 0 and ref["status"] == 0
    _compare(m, ref, what=f"lane queue {case}")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


@pytest.mark.parametrize("pipeline", [1, 2])
@pytest.mark.parametrize("case", ["overdraw_e1", "negative_rate", "neg_state", "step_limit"])
def test_lane_queue_first_error(lib, case, pipeline):
    """The first error in the serial order (day, phase, index) from the
    lane-queue kernel equals the oracle's."""
    u0 = np.tile([[500, 20, 0]], (300, 1))
    beta, rows, S = 0.3, [], None
    if case == "overdraw_e1":
        rows = [(W.EXIT, 6, 250, 0, 400, 0.0, 1, -1), (W.EXIT, 6, 40, 0, 900, 0.0, 0, -1),
                (W.EXIT, 9, 3, 0, 900, 0.0, 0, -1)]
    elif case == "negative_rate":
        beta = -0.01
    spec = W.sir_spec(u0, np.arange(0, 12), beta, 0.1, events=W.make_events(rows))
    if case == "neg_state":
        spec.S = np.array([[-1, 0], [1, -1], [-1, 1]])
    if case == "step_limit":
        # immigration at 3e7 per day: both nodes reach the 2^24-draw limit on day 0
        x0 = np.zeros(2, dtype=np.int64)
        spec = W.birth_death_spec(x0, np.arange(0, 3), 1.0, 0.5, immigration=True)
        spec.gdata = np.array([3.0e7, 0.0])
    m, ref, rc = _run_both(lib, spec, 5, 0, lane_queue=1, chunk=64, block=64, pipeline=pipeline)
    info = m.error_info()
    assert rc == ref["status"] != 0
    assert (info["code"], info["step"], info["phase"], info["index"]) == ref["error"]


def test_lane_queue_graph_replays(lib):
    """A lane-queue batch captured in a HIP graph: every replay (other work
    between them) equals a plain run."""
    sets = W.ensemble_sets(seed=43, n_sets=4, replicates=4, days=50, nn_range=(100, 600))
    batch = [(st.spec, 4) for st in sets]
    g = lib.Model(batch, record=lib.RECORD_SUMS, lane_queue=1, graph=1, chunk=256)
    plain = lib.Model(batch, record=lib.RECORD_SUMS, lane_queue=1, chunk=256)
    for seed in (3, 4, 3):
        g.run(seed, 2)
        assert g.wait() == 0
        plain.run(seed, 2)
        assert plain.wait() == 0
        assert np.array_equal(g.sums(), plain.sums()), seed


@pytest.mark.parametrize("transfers", [True, False])
@pytest.mark.parametrize("opts", [dict(lanes=64, wide=3), dict(lanes=64, wide=3, block=256, pipeline=2),
                                  dict(lanes=64, wide=3, lattice=2)])
def test_wide_node_event_windows(lib, opts, transfers):
    """Wavefront-wide nodes read their event records 64 at a time: three
    heavy nodes with hundreds of events, 150 of them on one day (the window
    is refilled in the middle of a day), exits of fixed counts and of
    proportions, births, and (dataflow kernel) transfers to the light nodes
    or (free-running kernel) none, against the oracle."""
    rng = np.random.default_rng(17)
    Nn, days = 40, 30
    u0 = np.stack([rng.integers(20, 60, Nn), rng.integers(0, 3, Nn), np.zeros(Nn, np.int64)], 1)
    u0[:3] = [[6000, 40, 0], [5000, 25, 0], [4000, 10, 0]]
    rows = []
    for node in range(3):
        for day in range(1, days + 1):
            per_day = 150 if day == 7 else int(rng.integers(0, 12))
            for _ in range(per_day):
                kind = int(rng.integers(0, 4))
                if kind == 0:
                    rows.append((W.EXIT, day, node, 0, int(rng.integers(1, 6)), 0.0, 3, -1))
                elif kind == 1:
                    rows.append((W.ENTER, day, node, 0, int(rng.integers(1, 6)), 0.0, 0, -1))
                elif kind == 2:
                    rows.append((W.EXIT, day, node, 0, 0, 0.002, 3, -1))
                else:
                    rows.append((W.EXTTRANS, day, node, int(rng.integers(3, Nn)), int(rng.integers(1, 4)), 0.0, 3, -1))
    if not transfers:
        rows = [r for r in rows if r[0] != W.EXTTRANS]
    rows.sort(key=lambda r: (r[1], r[0] == W.EXTTRANS))
    spec = W.sir_spec(u0, np.arange(0, days + 1), 0.3, 0.1, events=W.make_events(rows))
    m, ref, rc = _run_both(lib, spec, 4, 2, **opts)
    assert m.launch_info()["mode"] == (2 if transfers else 0)
    assert rc == 0 and ref["status"] == 0, (rc, ref["status"])
    assert m.launch_info()["wide"] == 3
    _compare(m, ref, what=f"event windows {opts}")
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


def test_sparse_trajectory(lib):
    """Table 1's U_sparse / V_sparse: the entries of U and V at a random
    sparse pattern (in the paper's layout: row node*width + c, column tspan
    index), empty columns included, equal the oracle's trajectory there; a
    pattern out of range is refused."""
    import scipy.sparse as sp
    spec = W.sise_with_events(seed=4, Nn=300, days=60)
    m, ref, rc = _run_both(lib, spec, 9, 2)
    assert rc == 0
    rng = np.random.default_rng(3)
    T = ref["U"].shape[0]
    for which, arr in (("U", ref["U"]), ("V", ref["V"])):
        Nn, width = arr.shape[1], arr.shape[2]
        dense = np.zeros((Nn * width, T))
        mask = rng.random(dense.shape) < 0.02
        mask[:, 5] = False  # an empty column
        dense[mask] = 1.0
        P = sp.csc_matrix(dense)
        P.sort_indices()
        got = m.trajectory_sparse(P, which)
        assert np.array_equal(got.indptr, P.indptr) and np.array_equal(got.indices, P.indices)
        want = arr.transpose(1, 2, 0).reshape(Nn * width, T)  # [node*width + c, t], the paper's layout
        cols = np.repeat(np.arange(T), np.diff(P.indptr))
        assert got.data.size == mask.sum()
        assert np.array_equal(got.data, want[P.indices, cols].astype(np.float64)), which
    bad = sp.csc_matrix(([1.0], ([spec.Nn * 2], [0])), shape=(spec.Nn * 2 + 1, T))
    with pytest.raises(lib.SiminfError):
        m.trajectory_sparse(bad, "U")
