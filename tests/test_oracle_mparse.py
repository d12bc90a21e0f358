"""Pins for the oracle's models given as transition strings (section 5.1):
its parser (oracle/mparse.py) and its postfix evaluation of the
propensities, against hand-derived matrices, the built-in SIR, invariants
of the paper's examples, and the master equation of a three-transition
model."""
import numpy as np
import pytest
from scipy import linalg

from oracle import mparse
from paper_1605_01421_amd import workloads as W

from test_oracle_ssa import _chi2_pooled


def test_incidence_example_matrices():
    """S -> b*S*I/(S+I+R) -> I + Icum, I -> g*I -> R: S has the columns
    (-1, +1, +1, 0) and (0, -1, 0, +1); both rates read I, which both
    transitions change, so G is all ones."""
    tr, comp = W.INCIDENCE_SIR
    m = mparse.compile_model(tr, comp, ["b", "g"])
    assert m["S"].tolist() == [[-1, 0], [1, -1], [1, 0], [0, 1]]
    assert m["G"].tolist() == [[1, 1], [1, 1]]


def test_sirs_dependency_graph():
    """Three transitions: rate 0 reads S, I, R; rate 1 reads I; rate 2 reads
    R.  Transition 0 changes S and I, 1 changes I and R, 2 changes R and S,
    so G's columns are (1,1,0), (1,1,1), (1,0,1); '@', '2*X' and a sum on
    one side give their counts."""
    m = mparse.compile_model(["S -> b*S*I/(S+I+R) -> I", "I -> g*I -> R", "R -> w*R -> S"], ["S", "I", "R"],
                             ["b", "g", "w"])
    assert m["G"].tolist() == [[1, 1, 1], [1, 1, 0], [0, 1, 1]]
    m2 = mparse.compile_model(["@ -> k -> 2*X + Y", "X + Y -> d*X*Y -> @"], ["X", "Y"], ["k", "d"])
    assert m2["S"].tolist() == [[2, -1], [1, -1]]
    assert m2["G"].tolist() == [[0, 0], [1, 1]]


@pytest.mark.parametrize("bad", [["S -> b*S*J -> I"], ["S -> b*S -> I -> R"], ["S -> b*S"], ["0*S -> b -> I"],
                                 ["S -> b*(S -> I"], ["S -> b*S) -> I"], ["S -> b S -> I"], ["S -> b* -> I"],
                                 ["Q -> b -> I"], ["S -> .e5 -> I"], ["S -> 1e999 -> I"]])
def test_parse_errors(bad):
    with pytest.raises(mparse.ParseError):
        mparse.compile_model(bad, ["S", "I"], ["b"])


def test_repeated_names_rejected():
    with pytest.raises(mparse.ParseError):
        mparse.compile_model(["S -> b -> I"], ["S", "I"], ["S"])


def test_operator_precedence_and_unary_minus():
    """2 - 3 * -b / (1 + 1) + -(-g) with b = 4, g = 0.5: 2 - (-12/2) + 0.5 =
    8.5, evaluated by the oracle as the rate of a constant-rate birth: the
    births of one day are Poisson(8.5)."""
    spec = W.mparse_spec(["@ -> 2 - 3 * -b / (1 + 1) + -(-g) -> X"], ["X"], np.zeros((20000, 1)), [0.0, 1.0],
                         gdata=dict(b=4.0, g=0.5))
    import oracle
    r = oracle.run(spec, 3, 0)
    assert r["status"] == 0
    x = r["U"][1][:, 0]
    assert abs(x.mean() - 8.5) < 4 * np.sqrt(8.5 / x.size)
    assert abs(x.var() - 8.5) < 0.05 * 8.5


def test_generated_sir_equals_builtin_sir():
    """The propensity b*S*I/(S+I+R) in the order the built-in SIR computes it
    ((b S) I)/((S + I) + R): with nodes that never empty, the trajectories
    are bit-identical, draw for draw."""
    import oracle
    u0 = np.tile([99, 5, 0], (300, 1))
    a = W.mparse_spec(["S -> b*S*I/(S+I+R) -> I", "I -> g*I -> R"], ["S", "I", "R"], u0, np.arange(0, 121),
                      gdata=dict(b=0.16, g=0.077))
    b = W.sir_spec(u0, np.arange(0, 121), 0.16, 0.077)
    ra, rb = oracle.run(a, 9, 3), oracle.run(b, 9, 3)
    assert ra["status"] == rb["status"] == 0
    assert np.array_equal(ra["U"], rb["U"])
    assert ra["transitions"] == rb["transitions"] > 10000


def test_incidence_counter_invariant():
    """In a closed population every infection moves one S to I and counts
    one in Icum: Icum(t) - Icum(0) = S(0) - S(t) for every node and time,
    and S + I + R is constant."""
    import oracle
    spec = W.incidence_sir(n=500, days=150)
    r = oracle.run(spec, 11, 0)
    assert r["status"] == 0
    U = r["U"].astype(np.int64)
    assert np.array_equal(U[:, :, 2] - U[0, :, 2], U[0, :, 0] - U[:, :, 0])
    assert (U[:, :, [0, 1, 3]].sum(axis=2) == 100).all()
    assert U[-1, :, 2].sum() > 1000


def _sirs_master_equation(N, S0, I0, b, g, w, times):
    states = [(s, i) for s in range(N + 1) for i in range(N + 1 - s)]
    index = {st: k for k, st in enumerate(states)}
    Q = np.zeros((len(states), len(states)))
    for (s, i), k in index.items():
        r = N - s - i
        for rate, dest in ((b * s * i / N, (s - 1, i + 1)), (g * i, (s, i - 1)), (w * r, (s + 1, i))):
            if rate > 0:
                Q[index[dest], k] += rate
                Q[k, k] -= rate
    P0 = np.zeros(len(states))
    P0[index[(S0, I0)]] = 1.0
    return states, [linalg.expm(Q * t) @ P0 for t in times]


def test_sirs_matches_master_equation():
    """A three-transition model (SIRS: waning immunity R -> S at w R) through
    the generic path: the joint law of (S, I) against the brute-force master
    equation for N = 12."""
    import oracle
    N, S0, I0, b, g, w = 12, 10, 2, 1.8, 0.6, 0.4
    n = 100_000
    times = [1.0, 3.0, 8.0]
    spec = W.mparse_spec(["S -> b*S*I/(S+I+R) -> I", "I -> g*I -> R", "R -> w*R -> S"], ["S", "I", "R"],
                         np.tile([S0, I0, N - S0 - I0], (n, 1)), [0.0] + times, gdata=dict(b=b, g=g, w=w))
    r = oracle.run(spec, 777, 1)
    assert r["status"] == 0
    states, Ps = _sirs_master_equation(N, S0, I0, b, g, w, times)
    code = {st: k for k, st in enumerate(states)}
    for m, P in enumerate(Ps, start=1):
        U = r["U"][m]
        assert (U.sum(axis=1) == N).all()
        obs = np.bincount([code[(s, i)] for s, i in U[:, :2]], minlength=len(states))
        assert _chi2_pooled(obs, P * n) > 1e-4


def test_vaccination_shift_moves_to_v():
    """The vaccination events of section 5.1.2 alone (no infection, no other
    events): on its day a herd moves floor(0.8 (S + I + R) + 0.5) animals,
    all from S here, four compartments on to V; nothing else changes."""
    import oracle
    spec = W.vaccination_example(Nn=300, days=40, b=0.0)
    keep = spec.events["event"] == W.INTTRANS
    spec.events = {k: v[keep] for k, v in spec.events.items()}
    spec.u0[:, 0] += spec.u0[:, 1]
    spec.u0[:, 1] = 0
    r = oracle.run(spec, 1, 0)
    assert r["status"] == 0
    S0 = spec.u0[:, 0].astype(np.int64)
    moved = np.floor(0.8 * S0 + 0.5).astype(np.int64)
    day = 21 + np.arange(300) // 50
    U = r["U"]
    for t in (20, 25, 30, 39):
        done = day <= t + 1  # tspan 1..40: record index t is day t + 1
        want_v = np.where(done, moved, 0)
        assert np.array_equal(U[t, :, 4], want_v), t
        assert np.array_equal(U[t, :, 0], S0 - want_v), t


def test_age_categories_move_with_ageing():
    """Appendix B's ageing as internal transfers with shifts: with no
    infection and no other events, a quarter of category 1 moves to
    category 2 every 30 days and a fifth of category 2 to category 3 every
    60 days, each floor(p n + 0.5) of the category's animals at the time."""
    import oracle
    spec = W.age_structured_sis(Nn=50, days=130, beta=0.0)
    keep = spec.events["event"] == W.INTTRANS
    spec.events = {k: v[keep] for k, v in spec.events.items()}
    r = oracle.run(spec, 2, 0)
    assert r["status"] == 0
    cat = spec.u0.reshape(50, 3, 2).sum(2).astype(np.int64)
    U = r["U"].reshape(131, 50, 3, 2).sum(3)
    for day in range(1, 131):
        for a, every, p in ((0, 30, 0.25), (1, 60, 0.2)):
            if day % every == 0:
                mv = np.floor(p * cat[:, a] + 0.5).astype(np.int64) * (cat[:, a] > 0)
                cat[:, a] -= mv
                cat[:, a + 1] += mv
        assert np.array_equal(U[day], cat), day
