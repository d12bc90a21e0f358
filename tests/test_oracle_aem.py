"""Pins for the oracle's all events method (section 3.4, the 'aem' solver):
each transition channel fires when its integrated rate reaches the running
sum of unit exponentials from its own stream.  It is an exact method, so its
law must equal the master equation's, as the direct method's does, while its
random numbers differ; and it must hold the same invariants."""
import numpy as np
import pytest

from paper_1605_01421_amd import workloads as W

from test_oracle_ssa import _chi2_pooled, _sir_master_equation, _sis_master_equation
from test_oracle_mparse import _sirs_master_equation


@pytest.mark.parametrize("N,S0,I0,beta,gamma", [(20, 18, 2, 1.5, 0.5), (12, 11, 1, 2.0, 0.7)])
def test_aem_sir_matches_master_equation(orc, N, S0, I0, beta, gamma):
    n = 100_000
    times = [1.0, 3.0, 10.0]
    spec = W.sir_spec(np.tile([S0, I0, N - S0 - I0], (n, 1)), [0.0] + times, beta, gamma)
    r = orc.run(spec, seed=2718, stream=4, solver="aem")
    assert r["status"] == 0
    states, Ps = _sir_master_equation(N, S0, I0, beta, gamma, times)
    code = {st: k for k, st in enumerate(states)}
    for m, P in enumerate(Ps, start=1):
        U = r["U"][m]
        assert (U.sum(axis=1) == N).all()
        obs = np.bincount([code[(s, i)] for s, i in U[:, :2]], minlength=len(states))
        assert _chi2_pooled(obs, P * n) > 1e-4


def test_aem_sis_matches_master_equation(orc):
    N, I0, beta, gamma = 20, 3, 0.05, 0.6
    n = 100_000
    times = [1.0, 3.0, 10.0]
    spec = W.sis_spec(np.tile([N - I0, I0], (n, 1)), [0.0] + times, beta, gamma)
    r = orc.run(spec, seed=99, stream=1, solver="aem")
    assert r["status"] == 0
    for m, P in enumerate(_sis_master_equation(N, I0, beta, gamma, times), start=1):
        obs = np.bincount(r["U"][m][:, 1], minlength=N + 1)
        assert _chi2_pooled(obs, P * n) > 1e-4


def test_aem_three_channels_match_master_equation(orc):
    """A generated three-transition model (SIRS) under the all events
    method: the law of (S, I) against the master equation."""
    N, S0, I0, b, g, w = 12, 10, 2, 1.8, 0.6, 0.4
    n = 100_000
    times = [1.0, 3.0, 8.0]
    spec = W.mparse_spec(["S -> b*S*I/(S+I+R) -> I", "I -> g*I -> R", "R -> w*R -> S"], ["S", "I", "R"],
                         np.tile([S0, I0, N - S0 - I0], (n, 1)), [0.0] + times, gdata=dict(b=b, g=g, w=w))
    r = orc.run(spec, 31, 2, solver="aem")
    assert r["status"] == 0
    states, Ps = _sirs_master_equation(N, S0, I0, b, g, w, times)
    code = {st: k for k, st in enumerate(states)}
    for m, P in enumerate(Ps, start=1):
        obs = np.bincount([code[(s, i)] for s, i in r["U"][m][:, :2]], minlength=len(states))
        assert _chi2_pooled(obs, P * n) > 1e-4


def test_aem_pure_death_is_binomial(orc):
    """I -> R alone: each individual leaves at rate gamma, so I(t) ~
    Binomial(I0, exp(-gamma t)) whatever the random numbers."""
    n, I0, gamma = 50_000, 30, 0.3
    spec = W.sir_spec(np.tile([0, I0, 0], (n, 1)), [0.0, 1.0, 3.0, 6.0], 0.0, gamma)
    r = orc.run(spec, 5, 0, solver="aem")
    from scipy import stats
    for m, t in ((1, 1.0), (2, 3.0), (3, 6.0)):
        obs = np.bincount(r["U"][m][:, 1], minlength=I0 + 1)
        exp = stats.binom.pmf(np.arange(I0 + 1), I0, np.exp(-gamma * t)) * n
        assert _chi2_pooled(obs, exp) > 1e-4


def test_aem_differs_from_ssm_but_keeps_invariants(orc):
    """The two methods draw different random numbers (the trajectories
    differ), both conserve S + I + R without events, and the aem's results
    do not depend on the thread count or on splitting the run in two."""
    u0 = np.tile([95, 5, 0], (2000, 1))
    spec = W.sir_spec(u0, np.arange(0, 61), 0.3, 0.1)
    a = orc.run(spec, 7, 0, solver="aem", nthreads=1)
    b = orc.run(spec, 7, 0, solver="ssm")
    a8 = orc.run(spec, 7, 0, solver="aem", nthreads=8)
    assert not np.array_equal(a["U"], b["U"])
    assert np.array_equal(a["U"], a8["U"])
    assert (a["U"].sum(axis=2) == 100).all()


def test_aem_with_events_runs_and_counts(orc):
    spec = W.sir_with_events(seed=3, Nn=400, days=60)
    r = orc.run(spec, 11, 2, solver="aem")
    assert r["status"] == 0 and r["events"] == len(spec.events["time"])
