"""Pins for the oracle's SSA against what the mathematics fixes.

Every test uses many independent replicate nodes in one run (the counter RNG
keys draws by node index) and a fixed seed.  Statistical tests use p > 1e-4
each (about 1e-3 over the file)."""
import math

import numpy as np
import pytest
from scipy import linalg, stats
from scipy.integrate import solve_ivp

from paper_1605_01421_amd import workloads as W


def _chi2_pooled(observed, expected, min_expected=5.0):
    """Chi-square p-value after pooling the tail bins with small expectation."""
    order = np.argsort(expected)
    obs, exp = [], []
    acc_o = acc_e = 0.0
    for k in order:
        acc_o += observed[k]
        acc_e += expected[k]
        if acc_e >= min_expected:
            obs.append(acc_o)
            exp.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 and exp:
        obs[-1] += acc_o
        exp[-1] += acc_e
    obs, exp = np.array(obs), np.array(exp)
    exp *= obs.sum() / exp.sum()
    return stats.chisquare(obs, exp).pvalue


def test_pure_recovery_is_binomial(orc):
    """P1: with beta = 0 each infected recovers after an Exp(gamma) time, so
    I(t) ~ Binomial(I0, exp(-gamma t)) exactly (day truncation is exact by
    memorylessness)."""
    n, I0, g = 100_000, 10, 0.3
    spec = W.sir_spec(np.tile([0, I0, 0], (n, 1)), [0, 1, 5, 20], beta=0.0, gamma=g)
    r = orc.run(spec, seed=2024, stream=1)
    assert r["status"] == 0
    for m, t in ((1, 1.0), (2, 5.0), (3, 20.0)):
        I = r["U"][m, :, 1]
        assert (r["U"][m].sum(axis=1) == I0).all()
        obs = np.bincount(I, minlength=I0 + 1)
        exp = stats.binom.pmf(np.arange(I0 + 1), I0, math.exp(-g * t)) * n
        assert _chi2_pooled(obs, exp) > 1e-4


def test_two_state_flip_is_binomial_mixture(orc):
    """P2: SISe with phi frozen (alpha = 0, no decay): every individual flips
    S->I at a = upsilon*phi and I->S at b = gamma independently, so
    I(t) ~ Bin(S0, a/(a+b)(1-e^{-(a+b)t})) + Bin(I0, (a+b e^{-(a+b)t})/(a+b))."""
    n, S0, I0 = 100_000, 8, 4
    ups, phi, g = 0.5, 1.0, 0.3
    spec = W.sise_spec(np.tile([S0, I0], (n, 1)), [0, 1, 2, 6], ups, g, 0.0,
                       (0.0, 0.0, 0.0, 0.0), phi0=phi)
    r = orc.run(spec, seed=77, stream=0)
    assert r["status"] == 0
    a, b = ups * phi, g
    for m, t in ((1, 1.0), (2, 2.0), (3, 6.0)):
        assert np.all(r["V"][m] == phi)
        e = math.exp(-(a + b) * t)
        p1 = a / (a + b) * (1 - e)
        p2 = (a + b * e) / (a + b)
        pmf = np.convolve(stats.binom.pmf(np.arange(S0 + 1), S0, p1),
                          stats.binom.pmf(np.arange(I0 + 1), I0, p2))
        obs = np.bincount(r["U"][m, :, 1], minlength=S0 + I0 + 1)
        assert _chi2_pooled(obs, pmf * n) > 1e-4


def test_immigration_death_is_poisson(orc):
    """P3a: from X0 = 0, X_t ~ Poisson(kappa/mu (1 - e^{-mu t}))."""
    n, kap, mu = 100_000, 3.0, 0.5
    spec = W.birth_death_spec(np.zeros(n), [0, 1, 4], kap, mu, immigration=True)
    r = orc.run(spec, seed=5, stream=3)
    assert r["status"] == 0
    for m, t in ((1, 1.0), (2, 4.0)):
        X = r["U"][m, :, 0]
        lam = kap / mu * (1 - math.exp(-mu * t))
        k = np.arange(X.max() + 1)
        obs = np.bincount(X, minlength=k.size)
        assert _chi2_pooled(obs, stats.poisson.pmf(k, lam) * n) > 1e-4


def test_linear_birth_death_moments(orc):
    """P3b: E X_t = X0 e^{(b-d)t}, Var X_t = X0 (b+d)/(b-d) e^{(b-d)t}(e^{(b-d)t}-1)."""
    n, X0, b, d, t = 100_000, 20, 0.3, 0.2, 5.0
    spec = W.birth_death_spec(np.full(n, X0), [0, t], b, d)
    r = orc.run(spec, seed=8, stream=0)
    X = r["U"][1, :, 0].astype(np.float64)
    g = math.exp((b - d) * t)
    mean, var = X0 * g, X0 * (b + d) / (b - d) * g * (g - 1)
    assert abs(X.mean() - mean) < 5 * math.sqrt(var / n)
    # variance of the sample variance ~ (mu4 - var^2)/n; use a loose 5% bound
    assert abs(X.var() - var) / var < 0.05


def _sir_master_equation(N, S0, I0, beta, gamma, times):
    """Transition-rate matrix of the SIR CTMC on {(S, I): S + I <= N} and
    P(t) = expm(Q t) P0 (the forward Kolmogorov / master equation)."""
    states = [(s, i) for s in range(N + 1) for i in range(N + 1 - s)]
    index = {st: k for k, st in enumerate(states)}
    Q = np.zeros((len(states), len(states)))
    for (s, i), k in index.items():
        r_inf = beta * s * i / N
        r_rec = gamma * i
        if r_inf > 0:
            Q[index[(s - 1, i + 1)], k] += r_inf
            Q[k, k] -= r_inf
        if r_rec > 0:
            Q[index[(s, i - 1)], k] += r_rec
            Q[k, k] -= r_rec
    P0 = np.zeros(len(states))
    P0[index[(S0, I0)]] = 1.0
    return states, [linalg.expm(Q * t) @ P0 for t in times]


@pytest.mark.parametrize("N,S0,I0,beta,gamma", [(20, 18, 2, 1.5, 0.5), (12, 11, 1, 2.0, 0.7)])
def test_sir_matches_master_equation(orc, N, S0, I0, beta, gamma):
    """P4: joint law of (S, I) of the full SIR SSA against the brute-force
    master-equation solution for a small population."""
    n = 100_000
    times = [1.0, 3.0, 10.0]
    spec = W.sir_spec(np.tile([S0, I0, N - S0 - I0], (n, 1)), [0.0] + times, beta, gamma)
    r = orc.run(spec, seed=31337, stream=2)
    assert r["status"] == 0
    states, Ps = _sir_master_equation(N, S0, I0, beta, gamma, times)
    code = {st: k for k, st in enumerate(states)}
    for m, P in enumerate(Ps, start=1):
        U = r["U"][m]
        assert (U.sum(axis=1) == N).all()
        idx = np.array([code[(s, i)] for s, i in U[:, :2]])
        obs = np.bincount(idx, minlength=len(states))
        assert _chi2_pooled(obs, P * n) > 1e-4


def _sis_master_equation(N, I0, beta, gamma, times):
    """SIS chain on I = 0..N with S = N - I (the population is closed): the
    infection S + I -> 2I at beta S I and the recovery I -> S at gamma I
    (eqs. sirtrans, SIRstoich), P(t) = expm(Q t) P0."""
    Q = np.zeros((N + 1, N + 1))
    for i in range(N + 1):
        r_inf = beta * (N - i) * i
        r_rec = gamma * i
        if r_inf > 0:
            Q[i + 1, i] += r_inf
            Q[i, i] -= r_inf
        if r_rec > 0:
            Q[i - 1, i] += r_rec
            Q[i, i] -= r_rec
    P0 = np.zeros(N + 1)
    P0[I0] = 1.0
    return [linalg.expm(Q * t) @ P0 for t in times]


@pytest.mark.parametrize("N,I0,beta,gamma", [(20, 3, 0.05, 0.6), (9, 1, 0.4, 0.9)])
def test_sis_matches_master_equation(orc, N, I0, beta, gamma):
    """P4 for the SIS rates: the law of I of the SIS SSA against the
    brute-force master-equation solution (a dropped factor, a swapped rate or
    a wrong column of S changes the law)."""
    n = 100_000
    times = [1.0, 3.0, 10.0]
    spec = W.sis_spec(np.tile([N - I0, I0], (n, 1)), [0.0] + times, beta, gamma)
    r = orc.run(spec, seed=4242, stream=5)
    assert r["status"] == 0
    for m, P in enumerate(_sis_master_equation(N, I0, beta, gamma, times), start=1):
        U = r["U"][m]
        assert (U.sum(axis=1) == N).all()
        obs = np.bincount(U[:, 1], minlength=N + 1)
        assert _chi2_pooled(obs, P * n) > 1e-4


def test_sir_large_population_follows_ode(orc):
    """P9: for large N the mean trajectory follows dx/dt = S R(x) (eq. ODE)."""
    Npop, I0, n = 100_000, 1000, 8
    beta, gamma = 0.16, 0.077
    tspan = np.arange(0, 61, 10, dtype=float)
    spec = W.sir_spec(np.tile([Npop - I0, I0, 0], (n, 1)), tspan, beta, gamma)
    r = orc.run(spec, seed=1, stream=0)

    def rhs(t, y):
        s, i, _ = y
        return [-beta * s * i, beta * s * i - gamma * i, gamma * i]

    sol = solve_ivp(rhs, (0, 60), [(Npop - I0) / Npop, I0 / Npop, 0.0], t_eval=tspan,
                    rtol=1e-10, atol=1e-12)
    mean = r["U"].mean(axis=1) / Npop
    assert np.max(np.abs(mean - sol.y.T)) < 0.01


def test_conservation_without_events(orc):
    """P5a: S+I+R (SIR) and S+I (SISe) are constant per node without events."""
    spec = W.plain_sir()
    r = orc.run(spec, seed=123, stream=0)
    tot = r["U"].sum(axis=2)
    assert (tot == 1000).all()
    assert r["transitions"] > 0 and r["node_days"] == 100 * 99
    u0 = np.stack([np.arange(10, 60), np.arange(50) % 7], axis=1)
    s2 = W.sise_spec(u0, np.arange(0, 100), 0.0175, 0.1, 1.0, (0.1, 0.12, 0.1, 0.11))
    r2 = orc.run(s2, seed=4, stream=9)
    assert (r2["U"].sum(axis=2) == u0.sum(axis=1)).all()


def test_phi_recursion_closed_form(orc):
    """P6: with no transitions (upsilon = gamma = 0) I/N is constant and within
    a season of constant decay beta the Euler update of section 2.3 gives
    phi_{n+k} = (1-beta)^k phi_n + alpha c (1 - (1-beta)^k)/beta, c = I/N; the
    season of day T is the first q with day-of-year(T) <= end_q."""
    u0 = np.array([[90, 10], [50, 50], [7, 0], [0, 3]])
    betas = (0.1, 0.2, 0.05, 0.3)
    alpha = 1.7
    spec = W.sise_spec(u0, np.arange(0, 731), 0.0, 0.0, alpha, betas, phi0=[0.5, 0.0, 2.0, 1.0])
    r = orc.run(spec, seed=1, stream=0)
    phi = r["V"][:, :, 0]
    c = u0[:, 1] / u0.sum(axis=1)

    def season(T):
        doy = (T - 1) % 365 + 1
        return 0 if doy <= 91 else 1 if doy <= 182 else 2 if doy <= 273 else 3

    T = 1
    while T <= 730:
        q = season(T)
        T2 = T
        while T2 + 1 <= 730 and season(T2 + 1) == q:
            T2 += 1
        bq = betas[q]
        k = np.arange(1, T2 - T + 2)[:, None]
        start = phi[T - 1]
        want = (1 - bq) ** k * start + alpha * c * (1 - (1 - bq) ** k) / bq
        got = phi[T:T2 + 1]
        assert np.allclose(got, want, rtol=1e-12, atol=1e-300)
        T = T2 + 1


def test_hypergeometric_event_sampling(orc):
    """Section 3.3: individuals of an exit are sampled without replacement over
    the selected compartments, so the removed counts are multivariate
    hypergeometric."""
    n, comp, take = 40_000, (30, 15, 5), 10
    u0 = np.tile(comp, (n, 1))
    ev = W.make_events([(W.EXIT, 1, i, 0, take, 0.0, 3, -1) for i in range(n)])
    spec = W.sir_spec(u0, [0, 1], beta=0.0, gamma=0.0, events=ev)
    r = orc.run(spec, seed=99, stream=0)
    assert r["status"] == 0 and r["events"] == n
    removed = np.asarray(comp) - r["U"][1]
    assert (removed.sum(axis=1) == take).all()
    obs = np.bincount(removed[:, 0], minlength=take + 1)
    exp = stats.hypergeom.pmf(np.arange(take + 1), sum(comp), comp[0], take) * n
    assert _chi2_pooled(obs, exp) > 1e-4
    pairs = removed[:, 0] * (take + 1) + removed[:, 1]
    obs2 = np.bincount(pairs, minlength=(take + 1) ** 2)
    exp2 = np.zeros((take + 1) ** 2)
    for a in range(take + 1):
        for b in range(take + 1 - a):
            c = take - a - b
            if a <= comp[0] and b <= comp[1] and c <= comp[2]:
                exp2[a * (take + 1) + b] = stats.multivariate_hypergeom.pmf([a, b, c], comp, take)
    assert _chi2_pooled(obs2, exp2 * n) > 1e-4


def test_thread_count_does_not_change_bits(orc):
    """The counter RNG makes the trajectory independent of the schedule."""
    spec = W.sir_with_events(seed=5, Nn=400, days=60)
    a = orc.run(spec, seed=42, stream=7, nthreads=1)
    b = orc.run(spec, seed=42, stream=7, nthreads=8)
    assert a["status"] == 0 and a["events"] > 100
    assert np.array_equal(a["U"], b["U"])
    assert (a["transitions"], a["events"]) == (b["transitions"], b["events"])


def test_split_run_equals_full_run(orc):
    """Draws are keyed by the absolute day, so running [0, 40] then [40, 90]
    from the saved state equals one run over [0, 90] (SIR and SISe)."""
    u0 = np.tile([300, 5, 0], (50, 1))
    full = W.sir_spec(u0, np.arange(0, 91), 0.3, 0.1)
    a = orc.run(full, 11, 2)
    first = orc.run(W.sir_spec(u0, np.arange(0, 41), 0.3, 0.1), 11, 2)
    second = orc.run(W.sir_spec(first["U"][-1], np.arange(40, 91), 0.3, 0.1), 11, 2)
    assert np.array_equal(a["U"][:41], first["U"])
    assert np.array_equal(a["U"][40:], second["U"])
    su = np.tile([60, 4], (30, 1))
    sf = W.sise_spec(su, np.arange(0, 91), 0.02, 0.1, 1.0, (0.1, 0.12, 0.1, 0.11))
    fa = orc.run(sf, 3, 0)
    s1 = orc.run(W.sise_spec(su, np.arange(0, 41), 0.02, 0.1, 1.0, (0.1, 0.12, 0.1, 0.11)), 3, 0)
    s2 = orc.run(W.sise_spec(s1["U"][-1], np.arange(40, 91), 0.02, 0.1, 1.0,
                             (0.1, 0.12, 0.1, 0.11), phi0=s1["V"][-1, :, 0]), 3, 0)
    assert np.array_equal(fa["U"][40:], s2["U"]) and np.array_equal(fa["V"][40:], s2["V"])


def test_step_limit(orc):
    """The implementation limit of 2^24 draws per node-day.  Immigration
    without death: X(1) ~ Poisson(kappa) exactly, and every draw of the day
    but the last is a transition.  Below the limit the count is Poisson
    (within 6 sd).  Above it the node has made exactly 2^24 transitions (draws
    0 .. 2^24 - 1) when it would need draw 2^24, and the run stops with
    E_STEP_LIMIT (not a rate error: the rates are valid), keyed to day step 0,
    phase SSA, node 0; node 1 (same rates) is not reached in the key order."""
    ok = W.birth_death_spec(np.array([0]), [0.0, 1.0], 1.0e7, 0.0, immigration=True)
    r = orc.run(ok, seed=4, stream=0, nthreads=1)
    assert r["status"] == 0
    x = int(r["U"][-1, 0, 0])
    assert abs(x - 1.0e7) < 6 * np.sqrt(1.0e7)
    assert r["transitions"] == x
    big = W.birth_death_spec(np.array([0]), [0.0, 1.0], 3.0e7, 0.0, immigration=True)
    r = orc.run(big, seed=4, stream=0, nthreads=1)
    assert r["status"] == -10                     # E_STEP_LIMIT
    assert r["error"] == (-10, 0, 0, 0)           # (code, day step, phase SSA, node 0)
    assert r["transitions"] == 2 ** 24
    two = W.birth_death_spec(np.array([0, 0]), [0.0, 1.0], 3.0e7, 0.0, immigration=True)
    r = orc.run(two, seed=4, stream=0, nthreads=2)
    assert r["error"] == (-10, 0, 0, 0)
