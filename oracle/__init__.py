"""CPU oracle for the SimInf split-step SSA (arXiv 1605.01421).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow, independent
reference implementation against which the GPU library is checked; it shares
no code with the library.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.

* ``siminf_oracle.c`` -- the split-step direct-method SSA with scheduled events
  and the post-time-step update (Appendix A, section 3.3, eq. numstep3), in C
  with OpenMP over nodes as the paper's solver does (section 3.4.2).
* ``mlp.py`` -- the float64 multilayer-perceptron reference for the surrogate.
* ``prevalence.py`` -- the prevalence and quantile reductions.

This module only marshals numpy arrays to the C oracle through ctypes.  A
model specification is any object with the attributes ``model, S, G, u0, v0,
ldata, gdata, tspan, E, N, events`` (see ``run``), and for SISe_sp
``neighbours`` = dict(ptr, idx, dist), the sparse distance matrix in
compressed columns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "siminf_oracle.c")
_LIB = os.path.join(_HERE, "libsiminf_oracle.so")

MODELS = {"SIR": 0, "SIS": 1, "SISE": 2, "BIRTH_DEATH": 3, "IMMIGRATION_DEATH": 4, "SISE_SP": 5}
ERRORS = {0: "ok", -1: "E_ARG", -2: "E_UNSUPPORTED", -3: "E_ALLOC",
          -5: "E_NEG_STATE", -6: "E_BAD_RATE", -7: "E_EVENT_OVERDRAW",
          -8: "E_EVENT_INDEX", -9: "E_PTS", -10: "E_STEP_LIMIT"}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc: -O2, OpenMP, no FP contraction."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-label",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("model", "Nc", "Nt", "Nn", "Nv", "Nld", "Ngd", "Ntspan")] + [
        ("S", ctypes.c_void_p), ("G", ctypes.c_void_p), ("u0", ctypes.c_void_p),
        ("v0", ctypes.c_void_p), ("ldata", ctypes.c_void_p),
        ("gdata", ctypes.c_void_p), ("tspan", ctypes.c_void_p),
        ("Nev", ctypes.c_int32), ("Ecols", ctypes.c_int32), ("Ncols", ctypes.c_int32),
        ("ev_type", ctypes.c_void_p), ("ev_time", ctypes.c_void_p),
        ("ev_node", ctypes.c_void_p), ("ev_dest", ctypes.c_void_p),
        ("ev_n", ctypes.c_void_p), ("ev_select", ctypes.c_void_p),
        ("ev_shift", ctypes.c_void_p), ("ev_prop", ctypes.c_void_p),
        ("E", ctypes.c_void_p), ("N", ctypes.c_void_p),
        ("Nnb", ctypes.c_int32), ("nb_ptr", ctypes.c_void_p), ("nb_idx", ctypes.c_void_p),
        ("nb_dist", ctypes.c_void_p), ("prog_off", ctypes.c_void_p), ("prog", ctypes.c_void_p),
        ("consts", ctypes.c_void_p), ("solver", ctypes.c_int32)]

SOLVERS = {"ssm": 0, "aem": 1}

# the model id the C oracle reads as "generated from transition strings"
MODEL_GENERATED = 64


_lib = None


def load():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_run.argtypes = [ctypes.POINTER(_Model), ctypes.c_uint64,
                               ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_philox.restype = None
    lib.oracle_philox.argtypes = [ctypes.c_void_p] * 3
    lib.oracle_plog.restype = ctypes.c_double
    lib.oracle_plog.argtypes = [ctypes.c_double]
    lib.oracle_uniform.restype = ctypes.c_double
    lib.oracle_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _per_node(a, n: int) -> np.ndarray:
    """An (n, k) float64 view of per-node data given as (n, k) or flat;
    with no nodes, k is the given array's second dimension (0 if flat)."""
    a = np.asarray(a, dtype=np.float64)
    if n == 0:
        return a.reshape(0, a.shape[1] if a.ndim == 2 else 0)
    return a.reshape(n, -1)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def run(spec, seed: int, stream: int = 0, nthreads: int | None = None, solver: str = "ssm") -> dict:
    """Run one trajectory of ``spec`` with Philox key ``seed`` and ``stream``.

    Returns a dict with ``U`` (Ntspan, Nn, Nc) int32, ``V`` (Ntspan, Nn, Nv)
    float64, ``transitions``, ``node_days``, ``events`` and ``status`` /
    ``error`` = (code, boundary index, phase, index).
    """
    lib = load()
    if nthreads is None:
        nthreads = lib.oracle_max_threads()
    gen = None
    if getattr(spec, "mparse", None) is not None:
        from . import mparse
        mp = spec.mparse
        gen = mparse.compile_model(mp["transitions"], mp["compartments"], mp.get("gdata_names", ()),
                                   mp.get("ldata_names", ()), mp.get("v_names", ()))
        S, G = gen["S"], gen["G"]
    else:
        S, G = np.asarray(spec.S), np.asarray(spec.G)
    Nc, Nt = S.shape
    u0 = _c(spec.u0, np.int32)
    Nn = u0.shape[0]
    v0 = _c(_per_node(spec.v0, Nn), np.float64)
    ldata = _c(_per_node(spec.ldata, Nn), np.float64)
    keep = dict(
        S=_c(S.ravel(order="F"), np.int32),
        G=_c(np.asarray(G).ravel(order="F"), np.int32),
        u0=u0, v0=v0, ldata=ldata,
        gdata=_c(spec.gdata, np.float64), tspan=_c(spec.tspan, np.float64),
        E=_c(np.asarray(spec.E).ravel(order="F"), np.int32),
        N=_c(np.asarray(spec.N).ravel(order="F"), np.int32))
    ev = spec.events
    names = ("event", "time", "node", "dest", "n", "select", "shift")
    for nm in names:
        keep["ev_" + nm] = _c(ev[nm], np.int32)
    keep["ev_prop"] = _c(ev["proportion"], np.float64)
    m = _Model()
    m.model = MODEL_GENERATED if gen is not None else int(spec.model)
    m.solver = SOLVERS[solver]
    if gen is not None:
        for f in ("prog_off", "prog"):
            keep[f] = _c(gen[f], np.int32)
            setattr(m, f, _ptr(keep[f]))
        keep["consts"] = _c(gen["consts"], np.float64)
        m.consts = _ptr(keep["consts"])
    m.Nc, m.Nt, m.Nn = Nc, Nt, Nn
    m.Nv, m.Nld = v0.shape[1], ldata.shape[1]
    m.Ngd, m.Ntspan = keep["gdata"].size, keep["tspan"].size
    for f in ("S", "G", "u0", "v0", "ldata", "gdata", "tspan", "E", "N"):
        setattr(m, f, _ptr(keep[f]))
    m.Nev = keep["ev_event"].size
    m.Ecols = np.asarray(spec.E).shape[1]
    m.Ncols = np.asarray(spec.N).shape[1] if np.asarray(spec.N).ndim == 2 else 0
    m.ev_type = _ptr(keep["ev_event"])
    for nm in names[1:]:
        setattr(m, "ev_" + nm, _ptr(keep["ev_" + nm]))
    m.ev_prop = _ptr(keep["ev_prop"])
    nb = getattr(spec, "neighbours", None)
    if nb is not None:
        keep["nb_ptr"] = _c(nb["ptr"], np.int32)
        keep["nb_idx"] = _c(nb["idx"], np.int32)
        keep["nb_dist"] = _c(nb["dist"], np.float64)
        m.Nnb = keep["nb_idx"].size
        m.nb_ptr = _ptr(keep["nb_ptr"])
        m.nb_idx = _ptr(keep["nb_idx"])
        m.nb_dist = _ptr(keep["nb_dist"])
    Ntspan = keep["tspan"].size
    U = np.zeros((Ntspan, Nn, Nc), dtype=np.int32)
    V = np.zeros((Ntspan, Nn, m.Nv), dtype=np.float64)
    cnt = np.zeros(3, dtype=np.uint64)
    err = np.zeros(4, dtype=np.int64)
    rc = lib.oracle_run(ctypes.byref(m), ctypes.c_uint64(seed & (2**64 - 1)),
                        ctypes.c_uint32(stream), int(nthreads), _ptr(U), _ptr(V),
                        _ptr(cnt), _ptr(err))
    return dict(U=U, V=V, transitions=int(cnt[0]), node_days=int(cnt[1]),
                events=int(cnt[2]), status=int(rc), error=tuple(int(x) for x in err),
                nthreads=int(nthreads))


def philox(key, ctr):
    """Philox4x32-10 block for key (2 words) and counter (4 words)."""
    lib = load()
    k = np.asarray(key, dtype=np.uint32)
    c = np.asarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox(_ptr(k), _ptr(c), _ptr(out))
    return out


def plog(x: float) -> float:
    return load().oracle_plog(float(x))


def uniform(a: int, b: int) -> float:
    return load().oracle_uniform(a, b)
