"""GPU parity of the spatially coupled SISe model (section 4.2, eq.
envInfPressure-local-spread) against the CPU oracle.

The coupled post-time step runs in the dataflow kernel only: each node posts
phi before the step and N after the day's events, and sums its neighbours'
coupling terms in stored order.  The same IEEE operations are performed in
the same order on both sides, so U and V must be bit-identical."""
import sys

import numpy as np
import pytest

from paper_1605_01421_amd import workloads as W

pytestmark = pytest.mark.gpu

NTHREADS = 16


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
    return oracle.run(spec, seed, stream, nthreads=NTHREADS)


def _same(m, ref, run=0, what=""):
    U, V = m.trajectory(run)
    if not np.array_equal(U, ref["U"]):
        bad = np.argwhere(U != ref["U"])
        raise AssertionError(f"{what}: U differs at {len(bad)} entries, first (t, node, c) = {bad[:3].tolist()}")
    if not np.array_equal(V, ref["V"]):
        bad = np.argwhere(V != ref["V"])
        raise AssertionError(f"{what}: phi differs at {len(bad)} entries, first {bad[:3].tolist()}")


def _counters_match(m, ref):
    c = m.counters()
    assert (c["transitions"], c["node_days"], c["events"]) == (ref["transitions"], ref["node_days"], ref["events"])


def _asymmetric(spec, seed, keep=0.6):
    """Keep each stored neighbour with probability `keep`: the relation is
    then no longer symmetric (a node may read another that does not read
    it); every ninth node keeps no neighbour at all."""
    rng = np.random.default_rng(seed)
    nb = spec.neighbours
    ptr, idx, dist = nb["ptr"], nb["idx"], nb["dist"]
    Nn = len(ptr) - 1
    nptr = np.zeros(Nn + 1, np.int32)
    nidx, ndist = [], []
    for i in range(Nn):
        sel = rng.random(ptr[i + 1] - ptr[i]) < keep
        if i % 9 == 0:
            sel[:] = False
        nidx.append(idx[ptr[i]:ptr[i + 1]][sel])
        ndist.append(dist[ptr[i]:ptr[i + 1]][sel])
        nptr[i + 1] = nptr[i] + int(sel.sum())
    spec.neighbours = dict(ptr=nptr, idx=np.concatenate(nidx).astype(np.int32),
                           dist=np.concatenate(ndist).astype(np.float64))
    return spec


@pytest.mark.parametrize("Nn,days,seed", [(300, 120, 1), (900, 365, 2)])
def test_sise_sp_with_events(lib, Nn, days, seed):
    spec = W.sise_sp_with_events(seed=seed, Nn=Nn, days=days)
    _say(spec.name, "edges", len(spec.neighbours["idx"]), "events", len(spec.events["time"]))
    ref = _oracle(spec, 31 + seed, 3)
    assert ref["status"] == 0
    m = lib.Model(spec)
    assert m.launch_info()["mode"] == 2, "the coupled model runs in the dataflow kernel"
    m.run(31 + seed, 3)
    assert m.wait() == 0
    _same(m, ref, what=spec.name)
    _counters_match(m, ref)


def test_sise_sp_asymmetric_and_empty_nodes(lib):
    """Neighbour lists that are not symmetric, nodes without neighbours and
    empty nodes (whose alpha and coupling terms are 0, but which still post
    for their readers), with scheduled events that fill and empty nodes."""
    spec = W.sise_sp_with_events(seed=3, Nn=500, days=200, events=False)
    spec = _asymmetric(spec, 4)
    u0 = np.array(spec.u0, copy=True)
    u0[::7] = 0
    spec.u0 = u0
    # every second empty node is filled by births (into S, E column 0), and
    # every 11th node is emptied by an exit of all its animals (E column 2)
    rows = [(W.ENTER, 20 + i % 90, i, 0, 25, 0.0, 0, -1) for i in range(0, 500, 14)]
    rows += [(W.EXIT, 60 + i % 100, i, 0, 0, 1.0, 2, -1) for i in range(5, 500, 11)]
    rows.sort(key=lambda r: (r[1], r[2]))
    spec.events = W.make_events(rows)
    ref = _oracle(spec, 8, 1)
    assert ref["status"] == 0
    m = lib.Model(spec)
    _say("asymmetric", m.launch_info())
    m.run(8, 1)
    assert m.wait() == 0
    _same(m, ref, what="asymmetric")
    _counters_match(m, ref)


@pytest.mark.parametrize("opts", [dict(lanes=64, wide=16), dict(lanes=1, group=-1), dict(block=256),
                                  dict(pipeline=1), dict(pipeline=2), dict(pack=16)])
def test_sise_sp_launch_shapes(lib, opts):
    """Wavefront-wide nodes, nodes on groups of lanes, block sizes,
    pipelining and packing leave every bit unchanged."""
    spec = W.sise_sp_with_events(seed=5, Nn=400, days=150)
    ref = _oracle(spec, 17, 2)
    m = lib.Model(spec, **opts)
    _say("shape", opts, m.launch_info())
    m.run(17, 2)
    assert m.wait() == 0
    _same(m, ref, what=str(opts))
    _counters_match(m, ref)


def test_sise_sp_automatic_packing(lib):
    """With no packing option the coupled kernel packs at least 16 nodes to a
    wavefront (every node on one lane: fewer 64-node wavefronts than CUs
    here); bits unchanged."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    spec = W.sise_sp_with_events(seed=5, Nn=400, days=150)
    ref = _oracle(spec, 17, 2)
    m = lib.Model(spec, lanes=1)
    info = m.launch_info()
    _say("automatic packing", info, "CUs", cus)
    if cus >= 8:
        assert info["pack"] == 16
    m.run(17, 2)
    assert m.wait() == 0
    _same(m, ref, what="automatic packing")
    _counters_match(m, ref)


def test_sise_sp_replicates(lib):
    """Replicates of one coupled model in one launch: each couples only its
    own nodes."""
    spec = W.sise_sp_with_events(seed=7, Nn=250, days=100)
    m = lib.Model([(spec, 4)])
    m.run(5, 40)
    assert m.wait() == 0
    for r in range(4):
        ref = _oracle(spec, 5, 40 + r)
        _same(m, ref, run=r, what=f"replicate {r}")


def test_sise_sp_unsupported_launches(lib):
    """The grid-barrier and lane-queue kernels have no coupled post-time
    step: asking for them is refused at create."""
    spec = W.sise_sp_with_events(seed=2, Nn=100, days=20)
    for opts in (dict(mode=1), dict(lane_queue=1)):
        with pytest.raises(lib.SiminfError) as e:
            lib.Model(spec, **opts)
        assert e.value.code == -2, opts


def test_sise_sp_first_error(lib):
    """A pair of nodes a hair apart makes the coupling weight overflow: the
    post-time step's phi is not finite, and the error key (step, phase,
    node) is the oracle's."""
    spec = W.sise_sp_with_events(seed=2, Nn=200, days=60)
    nb = spec.neighbours
    dist = np.array(nb["dist"], copy=True)
    dist[len(dist) // 2] = 1e-320
    spec.neighbours = dict(ptr=nb["ptr"], idx=nb["idx"], dist=dist)
    ref = _oracle(spec, 3, 0)
    assert ref["status"] != 0
    m = lib.Model(spec)
    m.run(3, 0)
    rc = m.wait()
    assert rc == ref["status"]
    e = m.error_info()
    assert (e["code"], e["step"], e["phase"], e["index"]) == ref["error"]


def test_sise_sp_full_size(lib):
    """1,600 farms in 50 x 50 km, neighbours within 2,500 m, four years with
    births, exits and movements: the whole trajectory."""
    spec = W.sise_sp_with_events()
    _say("SISe_sp full size", spec.Nn, len(spec.neighbours["idx"]), len(spec.events["time"]))
    ref = _oracle(spec, 2016, 0)
    assert ref["status"] == 0
    m = lib.Model(spec)
    m.run(2016, 0)
    assert m.wait() == 0
    _same(m, ref, what="SISe_sp full size")
    _counters_match(m, ref)


def test_sise_sp_full_size_autotuned(lib):
    """The full-size workload at the launch shape the benchmark times (the
    autotuner's pick): whole trajectory, phi and counters."""
    spec = W.sise_sp_with_events()
    ref = _oracle(spec, 2017, 1)
    assert ref["status"] == 0
    m = lib.Model(spec)
    best = m.autotune(seed=11, repeats=2)
    _say("SISe_sp full size, autotuned", m.launch_info(), f"{best:.2f} ms")
    m.run(2017, 1)
    assert m.wait() == 0
    _same(m, ref, what=f"autotuned {m.launch_info()}")
    _counters_match(m, ref)


@pytest.mark.parametrize("Nn,days", [(400, 150), (1600, 1460)])
def test_sise_sp_all_events_method(lib, Nn, days):
    """The coupled post-time step under the all events method (one lane per
    node, the dataflow kernel): U and phi bit-identical, counters equal."""
    import oracle
    spec = W.sise_sp_with_events(seed=5, Nn=Nn, days=days)
    ref = oracle.run(spec, 17, 2, nthreads=NTHREADS, solver="aem")
    assert ref["status"] == 0
    m = lib.Model(spec, solver="aem")
    _say("SISe_sp, all events method", Nn, days, m.launch_info())
    m.run(17, 2)
    assert m.wait() == 0
    _same(m, ref, what=f"SISe_sp aem {Nn} x {days}")
    _counters_match(m, ref)
