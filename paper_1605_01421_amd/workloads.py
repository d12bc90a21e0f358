"""Seeded synthetic inputs for the SimInf split-step SSA.

This module only builds input data: node populations, parameters, model
matrices and scheduled-event tables.  It holds none of the method's
arithmetic, and both the GPU library's tests and the CPU oracle's tests take
their inputs from here.

Conventions (all 0-based):

* ``u0`` has shape (Nn, Nc): row i is node i's compartment vector, so its
  C-order flattening is the paper's column-major Nc x Nn ``u0`` (Table 1).
* ``v0`` (Nn, Nv) and ``ldata`` (Nn, Nld) likewise; ``gdata`` is a vector.
* ``S`` (Nc, Nt), ``G`` (Nt, Nt), ``E`` (Nc, Ecols), ``N`` (Nc, Ncols) are the
  paper's matrices (Tables 1 and 2) as dense arrays.
* ``events`` is a dict of equal-length vectors ``event, time, node, dest, n,
  proportion, select, shift`` (Table 2) with event codes exit=0, enter=1,
  intTrans=2, extTrans=3, 0-based nodes / select / shift columns and
  ``shift = -1`` for "no shift".

The paper's datasets (``nodes``, ``u0_SISe``, ``events_SISe``, ...) are not
available; the generators below stand in for them with the shapes, sizes and
distributions of the workloads the library is measured on.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SIR, SIS, SISE, BIRTH_DEATH, IMMIGRATION_DEATH, SISE_SP = 0, 1, 2, 3, 4, 5
EXIT, ENTER, INTTRANS, EXTTRANS = 0, 1, 2, 3
EVENT_FIELDS = ("event", "time", "node", "dest", "n", "proportion", "select", "shift")


def empty_events() -> dict:
    ev = {k: np.zeros(0, dtype=np.int32) for k in EVENT_FIELDS}
    ev["proportion"] = np.zeros(0, dtype=np.float64)
    return ev


def make_events(rows) -> dict:
    """Events from rows (event, time, node, dest, n, proportion, select, shift)."""
    if len(rows) == 0:
        return empty_events()
    cols = list(zip(*rows))
    ev = {k: np.asarray(c, dtype=np.int32) for k, c in zip(EVENT_FIELDS, cols)}
    ev["proportion"] = np.asarray(cols[5], dtype=np.float64)
    return ev


def concat_events(*evs) -> dict:
    return {k: np.concatenate([e[k] for e in evs]) for k in EVENT_FIELDS}


@dataclass
class ModelSpec:
    model: int
    S: np.ndarray
    G: np.ndarray
    u0: np.ndarray
    v0: np.ndarray
    ldata: np.ndarray
    gdata: np.ndarray
    tspan: np.ndarray
    E: np.ndarray
    N: np.ndarray
    events: dict = field(default_factory=empty_events)
    name: str = ""
    # SISe_sp: the sparse distance matrix of section 4.2 in compressed
    # columns, dict(ptr (Nn+1,), idx (nnz,), dist (nnz,)); None otherwise
    neighbours: dict = None
    # a model given as transition strings (section 5.1):
    # dict(transitions, compartments, gdata_names, ldata_names, v_names);
    # S and G are then None (each side derives them from the strings)
    mparse: dict = None

    @property
    def Nn(self) -> int:
        return int(self.u0.shape[0])

    @property
    def Nc(self) -> int:
        if self.S is None:
            return len(self.mparse["compartments"])
        return int(self.S.shape[0])

    @property
    def Nv(self) -> int:
        return int(np.asarray(self.v0).reshape(self.Nn, -1).shape[1]) if self.Nn else 0

    @property
    def n_days(self) -> int:
        """Number of unit-time steps: boundaries floor(t0)+1 .. ceil(t_end)."""
        t0, t1 = float(self.tspan[0]), float(self.tspan[-1])
        return int(np.ceil(t1) - np.floor(t0)) if t1 > t0 else 0


# ---- model matrices ------------------------------------------------------

def sir_matrices():
    """SIR (eq. SIR): compartments S, I, R; transitions S->I, I->R."""
    S = np.array([[-1, 0], [1, -1], [0, 1]], dtype=np.int32)
    G = np.ones((2, 2), dtype=np.int32)
    # select matrix of the predefined SIR model (columns {S}, {I}, {R}, {S,I,R})
    E = np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 1]], dtype=np.int32)
    N = np.zeros((3, 1), dtype=np.int32)
    return S, G, E, N


def sis_matrices():
    """SIS / SISe: compartments S, I; transitions S->I, I->S (eq. SIRstoich)."""
    S = np.array([[-1, 1], [1, -1]], dtype=np.int32)
    G = np.ones((2, 2), dtype=np.int32)
    E = np.array([[1, 0, 1], [0, 1, 1]], dtype=np.int32)
    N = np.zeros((2, 1), dtype=np.int32)
    return S, G, E, N


def birth_death_matrices(immigration: bool = False):
    """One compartment X; transition 0 adds one individual, 1 removes one.

    For immigration-death the first rate is a constant, so no transition
    makes it stale (G row 0 is empty)."""
    S = np.array([[1, -1]], dtype=np.int32)
    G = np.array([[0, 0], [1, 1]] if immigration else [[1, 1], [1, 1]], dtype=np.int32)
    E = np.array([[1]], dtype=np.int32)
    N = np.zeros((1, 1), dtype=np.int32)
    return S, G, E, N


def _empty_nodes(Nn, k):
    return np.zeros((Nn, k), dtype=np.float64)


def sir_spec(u0, tspan, beta=0.16, gamma=0.077, events=None, name="SIR") -> ModelSpec:
    S, G, E, N = sir_matrices()
    u0 = np.ascontiguousarray(u0, dtype=np.int32).reshape(-1, 3)
    return ModelSpec(SIR, S, G, u0, _empty_nodes(len(u0), 0), _empty_nodes(len(u0), 0),
                     np.array([beta, gamma], dtype=np.float64),
                     np.asarray(tspan, dtype=np.float64), E, N,
                     events if events is not None else empty_events(), name)


def sis_spec(u0, tspan, beta, gamma, events=None, name="SIS") -> ModelSpec:
    S, G, E, N = sis_matrices()
    u0 = np.ascontiguousarray(u0, dtype=np.int32).reshape(-1, 2)
    return ModelSpec(SIS, S, G, u0, _empty_nodes(len(u0), 0), _empty_nodes(len(u0), 0),
                     np.array([beta, gamma], dtype=np.float64),
                     np.asarray(tspan, dtype=np.float64), E, N,
                     events if events is not None else empty_events(), name)


def sise_spec(u0, tspan, upsilon, gamma, alpha, beta_q, end_q=(91, 182, 273, 365),
              phi0=0.0, events=None, name="SISe") -> ModelSpec:
    """SISe: gdata = (upsilon, gamma, alpha, beta_1..beta_4), ldata per node =
    the day of year each of the four seasons ends, v = (phi)."""
    S, G, E, N = sis_matrices()
    u0 = np.ascontiguousarray(u0, dtype=np.int32).reshape(-1, 2)
    Nn = len(u0)
    v0 = np.broadcast_to(np.asarray(phi0, dtype=np.float64).reshape(-1, 1), (Nn, 1)).copy()
    ld = np.broadcast_to(np.asarray(end_q, dtype=np.float64), (Nn, 4)).copy()
    gd = np.array([upsilon, gamma, alpha, *beta_q], dtype=np.float64)
    return ModelSpec(SISE, S, G, u0, v0, ld, gd, np.asarray(tspan, dtype=np.float64),
                     E, N, events if events is not None else empty_events(), name)


def distance_matrix(x, y, cutoff):
    """The neighbours of each node within `cutoff` (Euclidean, same units as
    x, y) and their distances, as compressed columns dict(ptr, idx, dist):
    node i's neighbours, in increasing index, are idx[ptr[i]:ptr[i+1]] (the
    node itself excluded).  Found through a grid of cells of side cutoff."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    cx = np.floor(x / cutoff).astype(np.int64)
    cy = np.floor(y / cutoff).astype(np.int64)
    cells = {}
    for i in range(n):
        cells.setdefault((int(cx[i]), int(cy[i])), []).append(i)
    ptr = np.zeros(n + 1, dtype=np.int64)
    idx, dist = [], []
    for i in range(n):
        cand = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                cand.extend(cells.get((int(cx[i]) + dx, int(cy[i]) + dy), ()))
        cand = np.array(sorted(c for c in cand if c != i), dtype=np.int64)
        if cand.size:
            d = np.hypot(x[cand] - x[i], y[cand] - y[i])
            keep = d <= cutoff
            idx.append(cand[keep])
            dist.append(d[keep])
            ptr[i + 1] = ptr[i] + int(keep.sum())
        else:
            ptr[i + 1] = ptr[i]
    return dict(ptr=ptr.astype(np.int32),
                idx=(np.concatenate(idx) if idx else np.zeros(0)).astype(np.int32),
                dist=(np.concatenate(dist) if dist else np.zeros(0)).astype(np.float64))


def sise_sp_spec(u0, tspan, upsilon, gamma, alpha, beta_q, coupling, neighbours, end_q=(91, 182, 273, 365),
                 phi0=0.0, events=None, name="SISe_sp") -> ModelSpec:
    """SISe_sp (section 4.2): SISe with the spatial coupling of the
    environmental pressure among proximal nodes; gdata = (upsilon, gamma,
    alpha, beta_1..beta_4, coupling D), `neighbours` the sparse distance
    matrix (distance_matrix)."""
    spec = sise_spec(u0, tspan, upsilon, gamma, alpha, beta_q, end_q, phi0, events, name)
    spec.model = SISE_SP
    spec.gdata = np.append(spec.gdata, float(coupling))
    spec.neighbours = neighbours
    return spec


def sise_sp_with_events(seed: int = 6, Nn: int = 1600, days: int = 1460, density_per_km2: float = 0.64,
                        cutoff_m: float = 2500.0, upsilon=0.012, gamma=0.1, alpha=1.0,
                        beta_q=(0.10, 0.12, 0.12, 0.10), coupling=0.2, events=True) -> ModelSpec:
    """The SISe_sp example of section 4.2 on synthetic farms: Nn farms placed
    uniformly at random in a square whose side gives `density_per_km2`
    farms per km^2 (1600 farms in 50 x 50 km by default), neighbours within
    2500 m, 10% of the farms with 5% of their animals infected, phi0 = 0,
    the example's parameters (upsilon 0.012, gamma 0.1, alpha 1, beta
    0.10/0.12/0.12/0.10, coupling 0.2), herd sizes and scheduled events as in
    sise_with_events (births, exits and movements)."""
    rng = np.random.default_rng(seed)
    side_m = np.sqrt(Nn / density_per_km2) * 1000.0
    xs, ys = rng.uniform(0.0, side_m, Nn), rng.uniform(0.0, side_m, Nn)
    nb = distance_matrix(xs, ys, cutoff_m)
    size = np.maximum(np.round(rng.lognormal(np.log(40.0), 0.39, Nn)), 1).astype(np.int64)
    I0 = np.zeros(Nn, np.int64)
    inf = rng.choice(Nn, size=max(1, Nn // 10), replace=False)
    I0[inf] = np.floor(0.05 * size[inf]).astype(np.int64)
    u0 = np.stack([size - I0, I0], axis=1).astype(np.int32)
    ev = (_demographic_events(rng, Nn, size, days, birth=0.0009, exit_=0.0009, ship_frac=0.005,
                              select_all=2, birth_select=0) if events else None)
    return sise_sp_spec(u0, np.arange(0, days + 1), upsilon, gamma, alpha, beta_q, coupling, nb, events=ev,
                        name=f"sise-sp-{Nn}x{days}")


def birth_death_spec(x0, tspan, b, d, immigration=False, name=None) -> ModelSpec:
    S, G, E, N = birth_death_matrices(immigration)
    u0 = np.ascontiguousarray(x0, dtype=np.int32).reshape(-1, 1)
    return ModelSpec(IMMIGRATION_DEATH if immigration else BIRTH_DEATH, S, G, u0,
                     _empty_nodes(len(u0), 0), _empty_nodes(len(u0), 0),
                     np.array([b, d], dtype=np.float64),
                     np.asarray(tspan, dtype=np.float64), E, N, empty_events(),
                     name or ("immigration-death" if immigration else "birth-death"))


# ---- the paper's small examples -----------------------------------------

def sir_first_example(n=1000):
    """Section 4.1.1: n nodes of (999, 1, 0), tspan = 1, 8, ..., 176."""
    u0 = np.tile(np.array([999, 1, 0], dtype=np.int32), (n, 1))
    return sir_spec(u0, np.arange(1, 181, 7), 0.16, 0.077, name="sir-first-example")


def sir_event_example(infect=True):
    """Section 4.1.2: five empty nodes; enters on days 1-10 (node k gets k
    susceptibles per day), optionally one infected into node 5 on day 25,
    eleven moves of 5 individuals on days 35-45, 20% exits on days 70, 110."""
    rows = []
    for t in range(1, 11):
        for k in range(1, 6):
            rows.append((ENTER, t, k - 1, 0, k, 0.0, 0, -1))
    if infect:
        rows.append((ENTER, 25, 4, 0, 1, 0.0, 1, -1))
    src = [5, 5, 5, 5, 4, 4, 4, 3, 3, 2, 1]
    dst = [4, 3, 3, 1, 3, 2, 1, 2, 1, 1, 2]
    for t, a, b in zip(range(35, 46), src, dst):
        rows.append((EXTTRANS, t, a - 1, b - 1, 5, 0.0, 3, -1))
    for k in range(1, 6):
        for t in (70, 110):
            rows.append((EXIT, t, k - 1, 0, 0, 0.2, 3, -1))
    u0 = np.zeros((5, 3), dtype=np.int32)
    return sir_spec(u0, np.arange(1, 181), 0.16, 0.077, events=make_events(rows),
                    name="sir-event-example")


# ---- benchmark workloads --------------------------------------------------

def plain_sir() -> ModelSpec:
    """Plain SIR: 100 nodes of (990, 10, 0), beta 0.16, gamma 0.077, tspan 1..100."""
    u0 = np.tile(np.array([990, 10, 0], dtype=np.int32), (100, 1))
    return sir_spec(u0, np.arange(1, 101), 0.16, 0.077, name="sir-100-plain")


def _demographic_events(rng, Nn, tot, days, birth, exit_, ship_frac, select_all,
                        birth_select, geom_p=0.2, pareto_a=1.2):
    """Daily births (enter), exits and external transfers for Nn nodes.

    births ~ Poisson(birth * N_i) into the compartment of ``birth_select``;
    exits ~ Binomial(N_i, exit_) over all compartments; each day a fraction
    ``ship_frac`` of the nodes ship Geometric(geom_p) individuals to a
    destination drawn with probability proportional to Pareto(pareto_a)
    weights (preferential attachment), never to themselves.  The generator
    follows each node's total through the same-day order exit < enter <
    external transfer, so no event asks for more individuals than exist.
    """
    tot = tot.astype(np.int64).copy()
    w = rng.pareto(pareto_a, Nn) + 1.0
    cw = np.cumsum(w) / w.sum()
    out = {k: [] for k in EVENT_FIELDS}

    def add(kind, t, node, dest, n, sel):
        m = len(node)
        out["event"].append(np.full(m, kind, np.int32))
        out["time"].append(np.full(m, t, np.int32))
        out["node"].append(node.astype(np.int32))
        out["dest"].append(dest.astype(np.int32))
        out["n"].append(n.astype(np.int32))
        out["proportion"].append(np.zeros(m, np.float64))
        out["select"].append(np.full(m, sel, np.int32))
        out["shift"].append(np.full(m, -1, np.int32))

    idx = np.arange(Nn)
    for t in range(1, days + 1):
        ex = rng.binomial(tot, exit_)
        ex = np.minimum(ex, tot)
        sel = ex > 0
        add(EXIT, t, idx[sel], np.zeros(sel.sum()), ex[sel], select_all)
        tot -= ex
        bi = rng.poisson(birth * tot)
        sel = bi > 0
        add(ENTER, t, idx[sel], np.zeros(sel.sum()), bi[sel], birth_select)
        tot += bi
        k = rng.binomial(Nn, ship_frac)
        if k:
            srcs = rng.choice(Nn, size=k, replace=False)
            dsts = np.searchsorted(cw, rng.random(k), side="right").clip(0, Nn - 1)
            same = dsts == srcs
            while same.any():
                dsts[same] = np.searchsorted(cw, rng.random(same.sum()), side="right").clip(0, Nn - 1)
                same = dsts == srcs
            n = rng.geometric(geom_p, size=k).astype(np.int64)
            ns = np.zeros(k, np.int64)
            for j in range(k):  # sequential: a destination may ship later the same day
                a, b_ = srcs[j], dsts[j]
                ns[j] = min(n[j], tot[a])
                tot[a] -= ns[j]
                tot[b_] += ns[j]
            keep = ns > 0
            add(EXTTRANS, t, srcs[keep], dsts[keep], ns[keep], select_all)
    return {k: np.concatenate(v) if v else np.zeros(0) for k, v in out.items()}


def sir_with_events(seed: int = 1, Nn: int = 10_000, days: int = 365) -> ModelSpec:
    """SIR with scheduled events: lognormal node sizes (median 100, sigma 1,
    clipped to 1..5000), 1% infected, daily births Poisson(0.0005 N) into S,
    exits Binomial(N, 0.0003) over S/I/R, 0.5% of the nodes ship a
    Geometric(mean 5) batch per day to Pareto-weighted destinations."""
    rng = np.random.default_rng(seed)
    size = np.clip(np.round(rng.lognormal(np.log(100.0), 1.0, Nn)), 1, 5000).astype(np.int64)
    I0 = np.round(0.01 * size).astype(np.int64)
    u0 = np.stack([size - I0, I0, np.zeros(Nn, np.int64)], axis=1).astype(np.int32)
    ev = _demographic_events(rng, Nn, size, days, birth=0.0005, exit_=0.0003,
                             ship_frac=0.005, select_all=3, birth_select=0)
    return sir_spec(u0, np.arange(0, days + 1), 0.16, 0.077, events=ev,
                    name=f"sir-events-{Nn}x{days}")


def sir_with_shifts(seed: int = 5, Nn: int = 600, days: int = 60, heavy: int = 8) -> ModelSpec:
    """SIR with every kind of scheduled event and the select / shift
    machinery of Table 2 in use: births as in ``sir_with_events``, external
    transfers of a proportion of {S, I, R}, and

    * internal transfers (a vaccination-like move, as in section 5.1.2):
      select {S, I}, shift column 0 = (+2, +1, 0) (S -> R, I -> R), a
      proportion of the selected total (n = 0) or a fixed n;
    * shifted external transfers: select {S, I}, shift column 1 =
      (+1, +1, 0) (an S individual arrives in the destination's I, an I in
      its R), given as a proportion or as a fixed n;
    * exits given as a proportion (n = 0);
    * enter events into a select column with two rows, {I, R}: the
      individuals go to the first selected compartment, I;
    * same-node external transfers (source equals destination).

    The first ``heavy`` nodes are large (thousands of individuals), so that
    launches that give the heaviest nodes a wavefront or a group of lanes
    apply these events there too.  Proportions never overdraw and fixed
    counts are sized from the generator's running totals."""
    rng = np.random.default_rng(seed)
    size = np.clip(np.round(rng.lognormal(np.log(80.0), 1.0, Nn)), 1, 3000).astype(np.int64)
    size[:heavy] = rng.integers(4000, 9000, heavy)
    I0 = np.maximum(np.round(0.02 * size), 1).astype(np.int64)
    u0 = np.stack([size - I0, I0, np.zeros(Nn, np.int64)], axis=1).astype(np.int32)
    # births (fixed counts into S); every removal below is a proportion, or a
    # small fixed count from a heavy node, so that no event can overdraw
    base = _demographic_events(rng, Nn, size, days, birth=0.001, exit_=0.0,
                               ship_frac=0.0, select_all=3, birth_select=0)
    rows = []
    for t in range(1, days + 1):
        # plain external transfers of a proportion of {S, I, R}
        for node in rng.choice(Nn, size=max(1, Nn // 60), replace=False):
            rows.append((EXTTRANS, t, int(node), int(rng.integers(0, Nn)), 0, float(rng.uniform(0.01, 0.3)), 3, -1))
        # internal transfers: a proportion of {S, I}, or a fixed small n
        for node in rng.choice(Nn, size=max(1, Nn // 40), replace=False):
            rows.append((INTTRANS, t, int(node), 0, 0, float(rng.uniform(0.05, 0.5)), 4, 0))
        rows.append((INTTRANS, t, int(rng.integers(0, heavy)), 0, int(rng.integers(1, 6)), 0.0, 4, 0))
        # shifted external transfers by proportion, some to the node itself
        for node in rng.choice(Nn, size=max(1, Nn // 60), replace=False):
            dest = int(node) if rng.random() < 0.1 else int(rng.integers(0, Nn))
            rows.append((EXTTRANS, t, int(node), dest, 0, float(rng.uniform(0.01, 0.2)), 4, 1))
        # a heavy node ships a fixed count with the shift
        h = int(rng.integers(0, heavy))
        rows.append((EXTTRANS, t, h, int(rng.integers(0, Nn)), int(rng.integers(1, 4)), 0.0, 4, 1))
        # proportional exits, and enters into the {I, R} column
        for node in rng.choice(Nn, size=max(1, Nn // 50), replace=False):
            rows.append((EXIT, t, int(node), 0, 0, float(rng.uniform(0.0, 0.1)), 3, -1))
        for node in rng.choice(Nn, size=max(1, Nn // 80), replace=False):
            rows.append((ENTER, t, int(node), 0, int(rng.integers(1, 3)), 0.0, 5, -1))
    ev = concat_events(base, make_events(rows))
    S, G, _, _ = sir_matrices()
    E = np.array([[1, 0, 0, 1, 1, 0],
                  [0, 1, 0, 1, 1, 1],
                  [0, 0, 1, 1, 0, 1]], dtype=np.int32)
    N = np.array([[2, 1], [1, 1], [0, 0]], dtype=np.int32)
    spec = sir_spec(u0, np.arange(0, days + 1), 0.16, 0.077, events=ev, name=f"sir-shifts-{Nn}x{days}")
    spec.E, spec.N = E, N
    return spec


def sise_with_events(seed: int = 2, Nn: int = 37_000, days: int = 3650) -> ModelSpec:
    """SISe with events: lognormal sizes (median 40, sigma 0.39, about 1.6M
    individuals for 37,000 nodes), 10% of nodes start with floor(5% of S)
    infected, phi0 = 0, upsilon 0.0175, gamma 0.1, alpha 1, quarterly decay
    (0.1, 0.12, 0.1, 0.11); births and exits at 0.0009 per individual-day
    and 0.5% of nodes shipping per day (about 1e6 events per simulated year
    at full size)."""
    rng = np.random.default_rng(seed)
    size = np.maximum(np.round(rng.lognormal(np.log(40.0), 0.39, Nn)), 1).astype(np.int64)
    I0 = np.zeros(Nn, np.int64)
    inf = rng.choice(Nn, size=max(1, Nn // 10), replace=False)
    I0[inf] = np.floor(0.05 * size[inf]).astype(np.int64)
    u0 = np.stack([size - I0, I0], axis=1).astype(np.int32)
    ev = _demographic_events(rng, Nn, size, days, birth=0.0009, exit_=0.0009,
                             ship_frac=0.005, select_all=2, birth_select=0)
    return sise_spec(u0, np.arange(0, days + 1), 0.0175, 0.1, 1.0,
                     (0.1, 0.12, 0.1, 0.11), events=ev, name=f"sise-events-{Nn}x{days}")


@dataclass
class EnsembleSet:
    spec: ModelSpec
    replicates: int
    features: np.ndarray  # surrogate inputs (8,)


def ensemble_sets(seed: int = 3, n_sets: int = 64, replicates: int = 64, days: int = 365,
                  nn_range=(100, 20_000), record_every: int = 7) -> list:
    """Batched-ensemble parameter sets: half SIR (beta in U[0.08, 0.24],
    gamma in U[0.0385, 0.1155]), half SISe (upsilon in U[0.00875, 0.02625],
    gamma in U[0.05, 0.15]); per set a node count log-uniform on nn_range,
    lognormal node sizes (median log-uniform on [20, 1000], sigma in
    U[0.3, 1.0]) and an initial prevalence in U[0.001, 0.05]; no scheduled
    events; state recorded every ``record_every`` days."""
    rng = np.random.default_rng(seed)
    sets = []
    tspan = np.arange(0, days + 1, record_every, dtype=np.float64)
    if tspan[-1] != days:
        tspan = np.append(tspan, float(days))
    for k in range(n_sets):
        sise = k >= n_sets // 2
        Nn = int(np.floor(np.exp(rng.uniform(np.log(nn_range[0]), np.log(nn_range[1])))))
        med = float(np.exp(rng.uniform(np.log(20.0), np.log(1000.0))))
        sig = float(rng.uniform(0.3, 1.0))
        size = np.maximum(np.round(rng.lognormal(np.log(med), sig, Nn)), 1).astype(np.int64)
        prev = float(rng.uniform(0.001, 0.05))
        I0 = rng.binomial(size, prev)
        gamma = float(rng.uniform(0.05, 0.15) if sise else rng.uniform(0.0385, 0.1155))
        if sise:
            ups = float(rng.uniform(0.00875, 0.02625))
            u0 = np.stack([size - I0, I0], axis=1).astype(np.int32)
            spec = sise_spec(u0, tspan, ups, gamma, 1.0, (0.1, 0.12, 0.1, 0.11),
                             name=f"set{k}-sise")
            par = (1.0, 0.0, ups)
        else:
            beta = float(rng.uniform(0.08, 0.24))
            u0 = np.stack([size - I0, I0, np.zeros(Nn, np.int64)], axis=1).astype(np.int32)
            spec = sir_spec(u0, tspan, beta, gamma, name=f"set{k}-sir")
            par = (0.0, beta, 0.0)
        ls = np.log(size.astype(np.float64))
        feats = np.array([par[0], par[1], par[2], gamma, I0.sum() / size.sum(),
                          ls.mean(), ls.var(), np.log(Nn)], dtype=np.float64)
        sets.append(EnsembleSet(spec, replicates, feats))
    return sets


def mlp_init(dims, seed):
    """Initial surrogate weights: uniform on +-sqrt(6 / fan_in) (He-style),
    zero biases; a list of (W (out, in), b (out,)) float64 arrays."""
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(dims) - 1):
        lim = np.sqrt(6.0 / dims[i])
        params.append((rng.uniform(-lim, lim, (dims[i + 1], dims[i])), np.zeros(dims[i + 1])))
    return params


# ---- models given as transition strings (section 5.1) -------------------

MPARSE = -1  # model id of a spec whose model is given by transition strings


def mparse_spec(transitions, compartments, u0, tspan, gdata=None, ldata=None, v0=None, E=None, N=None,
                events=None, name="mparse") -> ModelSpec:
    """A spec whose model is given as transition strings "from -> propensity
    -> to" over the named compartments; gdata, ldata and v0 are dicts name ->
    value (gdata) or name -> per-node values (ldata, v0), in the order the
    names are given.  E and N (Nc x columns) are the select and shift
    matrices of the events."""
    u0 = np.ascontiguousarray(u0, dtype=np.int32).reshape(-1, len(compartments))
    Nn = len(u0)
    gdata = dict(gdata or {})
    ldata = dict(ldata or {})
    v0 = dict(v0 or {})
    ld = (np.stack([np.broadcast_to(np.asarray(x, np.float64), (Nn,)) for x in ldata.values()], 1)
          if ldata else _empty_nodes(Nn, 0))
    vv = (np.stack([np.broadcast_to(np.asarray(x, np.float64), (Nn,)) for x in v0.values()], 1)
          if v0 else _empty_nodes(Nn, 0))
    nc = len(compartments)
    E = np.zeros((nc, 0), np.int32) if E is None else np.asarray(E, dtype=np.int32).reshape(nc, -1)
    N = np.zeros((nc, 0), np.int32) if N is None else np.asarray(N, dtype=np.int32).reshape(nc, -1)
    spec = ModelSpec(MPARSE, None, None, u0, vv, ld, np.asarray(list(gdata.values()), dtype=np.float64),
                     np.asarray(tspan, dtype=np.float64), E, N,
                     events if events is not None else empty_events(), name)
    spec.mparse = dict(transitions=list(transitions), compartments=list(compartments),
                       gdata_names=list(gdata), ldata_names=list(ldata), v_names=list(v0))
    return spec


INCIDENCE_SIR = (["S -> b*S*I/(S+I+R) -> I + Icum", "I -> g*I -> R"], ["S", "I", "Icum", "R"])


def incidence_sir(n=1000, days=150, S0=99, I0=1, b=0.16, g=0.077) -> ModelSpec:
    """The incidence example of section 5.1: SIR with a counter Icum of the
    infections, n identical closed nodes (99 susceptible, 1 infected)."""
    tr, comp = INCIDENCE_SIR
    u0 = np.tile([S0, I0, 0, 0], (n, 1))
    return mparse_spec(tr, comp, u0, np.arange(1, days + 1), gdata=dict(b=b, g=g), name=f"mparse-sir-icum-{n}")


def vaccination_example(seed=21, Nn=1600, days=300, vaccinate=True, b=0.16, g=0.077, infected=1) -> ModelSpec:
    """The vaccination example of section 5.1.2 on synthetic herds: S, I,
    Icum, R, V; births into S (E column 1), deaths and movements over S, I,
    R, V (column 2), vaccination as internal transfers of 80% of S, I and R
    (column 3) shifted to V by the N column (S +4, I +3, R +1), 50 herds a
    day from day 21 until every herd is done; one infected animal in each of
    `infected` random herds (one in the example).  Herd sizes and the birth, death and movement events follow the
    SIR-with-events generator (the example's data sets are not available)."""
    rng = np.random.default_rng(seed)
    size = np.clip(np.round(rng.lognormal(np.log(100.0), 1.0, Nn)), 1, 5000).astype(np.int64)
    u0 = np.zeros((Nn, 5), np.int64)
    u0[:, 0] = size
    for j in rng.choice(Nn, size=infected, replace=False):
        take = min(int(u0[j, 0]), 1)
        u0[j, 0] -= take
        u0[j, 1] += take
    E = np.array([[1, 1, 1], [0, 1, 1], [0, 0, 0], [0, 1, 1], [0, 1, 0]], np.int32)
    N = np.array([[4], [3], [0], [1], [0]], np.int32)
    ev = _keep_nonempty(_demographic_events(rng, Nn, size, days, birth=0.0005, exit_=0.0003, ship_frac=0.005,
                                            select_all=1, birth_select=0), size)
    if vaccinate:
        rows = [(INTTRANS, 21 + k // 50, k, 0, 0, 0.8, 2, 0) for k in range(Nn) if 21 + k // 50 <= days]
        ev = concat_events(ev, make_events(rows))
    tr = ["S -> b*S*I/(S+I+R+V) -> I + Icum", "I -> g*I -> R"]
    return mparse_spec(tr, ["S", "I", "Icum", "R", "V"], u0, np.arange(1, days + 1), gdata=dict(b=b, g=g),
                       E=E, N=N, events=ev, name=f"mparse-vaccination-{Nn}x{days}")


def _keep_nonempty(ev: dict, size) -> dict:
    """The events without the exits and external transfers that would leave
    a node with no animals (the propensity b*S*I/(S+I+R+V) of the
    vaccination example is 0/0 in an empty herd).  Totals are followed in
    the order a day applies the events: every node's exits, then its
    births, then the external transfers in input order."""
    tot = np.asarray(size, dtype=np.int64).copy()
    keep = np.ones(len(ev["time"]), dtype=bool)
    order = np.lexsort((np.arange(len(ev["time"])), ev["event"] == EXTTRANS, ev["event"], ev["time"]))
    for e in order:
        ty, node, n = int(ev["event"][e]), int(ev["node"][e]), int(ev["n"][e])
        moved = n if n > 0 else int(np.floor(float(ev["proportion"][e]) * tot[node] + 0.5))
        if ty == ENTER:
            tot[node] += n
        elif ty in (EXIT, EXTTRANS):
            if moved >= tot[node]:
                keep[e] = False
                continue
            tot[node] -= moved
            if ty == EXTTRANS:
                tot[int(ev["dest"][e])] += moved
    return {k: np.asarray(v)[keep].copy() for k, v in ev.items()}


def age_structured_sis(seed=31, Nn=400, days=200, gamma=0.1, beta=0.3) -> ModelSpec:
    """An age-structured SIS in three age categories, with the compartments
    and scheduled events of the illustration in Appendix B: S1 I1 S2 I2 S3
    I3; infection within a category at beta*S_a*I/N, recovery at gamma*I_a;
    events: births into S1 (E column 1), exits from each category (columns
    4-6: {S_a, I_a}), ageing of categories 1 and 2 as internal transfers
    shifted by the N columns (S1->S2, I1->I2; S2->S3, I2->I3), and movements
    of single animals of a category between nodes.  The generator follows
    each category's total in the order a day applies the events (exits,
    births, ageing, movements out, then movements in), so no event
    overdraws."""
    rng = np.random.default_rng(seed)
    comp = ["S1", "I1", "S2", "I2", "S3", "I3"]
    Ntot = "(S1+I1+S2+I2+S3+I3)"
    Itot = "(I1+I2+I3)"
    tr = []
    for a in (1, 2, 3):
        tr.append(f"S{a} -> beta*S{a}*{Itot}/{Ntot} -> I{a}")
        tr.append(f"I{a} -> gamma*I{a} -> S{a}")
    size = np.maximum(np.round(rng.lognormal(np.log(60.0), 0.6, (Nn, 3))), 1).astype(np.int64)
    u0 = np.zeros((Nn, 6), np.int64)
    u0[:, 0], u0[:, 2], u0[:, 4] = size[:, 0], size[:, 1], size[:, 2]
    inf = rng.choice(Nn, size=max(1, Nn // 10), replace=False)
    take = np.minimum(u0[inf, 0], 2)
    u0[inf, 0] -= take
    u0[inf, 1] += take
    # E columns: 1-3 {S_a} (births into the first), 4-6 {S_a, I_a}
    E = np.zeros((6, 6), np.int32)
    for a in range(3):
        E[2 * a, a] = 1
        E[2 * a, 3 + a] = E[2 * a + 1, 3 + a] = 1
    N = np.zeros((6, 2), np.int32)
    N[0, 0] = N[1, 0] = 2  # S1 -> S2, I1 -> I2
    N[2, 1] = N[3, 1] = 2  # S2 -> S3, I2 -> I3
    tot = u0.reshape(Nn, 3, 2).sum(2)  # animals per node and category
    rows = []
    for day in range(1, days + 1):
        arriving = np.zeros_like(tot)
        for i in range(Nn):
            for a in range(3):
                if tot[i, a] > 0 and rng.random() < 0.005:
                    k = int(rng.integers(1, min(3, tot[i, a]) + 1))
                    rows.append((EXIT, day, i, 0, k, 0.0, 3 + a, -1))
                    tot[i, a] -= k
            if rng.random() < 0.02:
                k = int(rng.integers(1, 4))
                rows.append((ENTER, day, i, 0, k, 0.0, 0, -1))
                tot[i, 0] += k
            for a, every, prop in ((0, 30, 0.25), (1, 60, 0.2)):
                if day % every == 0 and tot[i, a] > 0:
                    rows.append((INTTRANS, day, i, 0, 0, prop, 3 + a, a))
                    moved = int(np.floor(prop * tot[i, a] + 0.5))
                    tot[i, a] -= moved
                    tot[i, a + 1] += moved
            if rng.random() < 0.01:
                a = int(rng.integers(0, 3))
                dst = int(rng.integers(0, Nn))
                if tot[i, a] > 1 and dst != i:
                    rows.append((EXTTRANS, day, i, dst, 1, 0.0, 3 + a, -1))
                    tot[i, a] -= 1
                    arriving[dst, a] += 1
        tot += arriving
    return mparse_spec(tr, comp, u0, np.arange(0, days + 1), gdata=dict(beta=beta, gamma=gamma),
                       E=E, N=N, events=make_events(rows), name=f"mparse-age-sis-{Nn}x{days}")
