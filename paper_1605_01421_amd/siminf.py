"""ctypes binding of libsiminf.so (the C ABI in include/siminf.h).

Argument marshalling only: every step of a run executes in the library's HIP
kernels.  PyTorch is used for device memory and streams where the caller
wants device-resident results.  Loading fails loudly when the library is
missing -- there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsiminf.so")

SIMINF_OK = 0
STATUS = {0: "SIMINF_OK", -1: "SIMINF_E_ARG", -2: "SIMINF_E_UNSUPPORTED", -3: "SIMINF_E_ALLOC",
          -4: "SIMINF_E_DEVICE", -5: "SIMINF_E_NEG_STATE", -6: "SIMINF_E_BAD_RATE",
          -7: "SIMINF_E_EVENT_OVERDRAW", -8: "SIMINF_E_EVENT_INDEX", -9: "SIMINF_E_PTS",
          -10: "SIMINF_E_STEP_LIMIT"}
RECORD_FULL, RECORD_SUMS = 0, 1


class SiminfError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)}")


class Spec(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("model", "Nc", "Nt", "Nn", "Nv", "Nld", "Ngd", "Ntspan")] + [
        ("S", ctypes.c_void_p), ("G", ctypes.c_void_p), ("u0", ctypes.c_void_p),
        ("v0", ctypes.c_void_p), ("ldata", ctypes.c_void_p), ("gdata", ctypes.c_void_p),
        ("tspan", ctypes.c_void_p),
        ("Nev", ctypes.c_int32), ("Ecols", ctypes.c_int32), ("Ncols", ctypes.c_int32),
        ("ev_type", ctypes.c_void_p), ("ev_time", ctypes.c_void_p), ("ev_node", ctypes.c_void_p),
        ("ev_dest", ctypes.c_void_p), ("ev_n", ctypes.c_void_p), ("ev_select", ctypes.c_void_p),
        ("ev_shift", ctypes.c_void_p), ("ev_prop", ctypes.c_void_p),
        ("E", ctypes.c_void_p), ("N", ctypes.c_void_p),
        ("Nnb", ctypes.c_int32), ("nb_ptr", ctypes.c_void_p), ("nb_idx", ctypes.c_void_p),
        ("nb_dist", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("record", ctypes.c_int32), ("block", ctypes.c_int32), ("order", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("max_blocks", ctypes.c_int32),
                ("pipeline", ctypes.c_int32), ("mode", ctypes.c_int32), ("wide", ctypes.c_int32),
                ("lattice", ctypes.c_int32), ("wait_ms", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("pack", ctypes.c_int32), ("group", ctypes.c_int32), ("lane_queue", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("batch", ctypes.c_int32), ("solver", ctypes.c_int32)]


# exported entry points: name -> (restype, argtypes)
_P = ctypes.c_void_p


class ModelDef(ctypes.Structure):
    """siminf_model_def: a model given as transition strings (section 5.1)."""
    _fields_ = [("nt", ctypes.c_int32), ("transitions", _P), ("nc", ctypes.c_int32), ("compartments", _P),
                ("ngd", ctypes.c_int32), ("gdata_names", _P), ("nld", ctypes.c_int32), ("ldata_names", _P),
                ("nv", ctypes.c_int32), ("v_names", _P), ("Ecols", ctypes.c_int32), ("E", _P),
                ("Ncols", ctypes.c_int32), ("N", _P)]
SIGNATURES = {
    "siminf_create": (ctypes.c_int, [ctypes.POINTER(Spec), ctypes.POINTER(Options), ctypes.POINTER(_P)]),
    "siminf_create_batch": (ctypes.c_int, [ctypes.POINTER(Spec), ctypes.c_int32, _P,
                                           ctypes.POINTER(Options), ctypes.POINTER(_P)]),
    "siminf_run": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint32, _P]),
    "siminf_wait": (ctypes.c_int, [_P]),
    "siminf_trajectory": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32]),
    "siminf_sums": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "siminf_trajectory_sparse": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, _P, _P,
                                                ctypes.c_int32]),
    "siminf_counters": (ctypes.c_int, [_P, _P]),
    "siminf_shape": (ctypes.c_int, [_P, _P]),
    "siminf_error_info": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "siminf_error_message": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_size_t]),
    "siminf_launch_info": (ctypes.c_int, [_P, _P]),
    "siminf_timing": (ctypes.c_int, [_P, _P]),
    "siminf_autotune": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int32, _P, _P]),
    "siminf_destroy": (None, [_P]),
    "siminf_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "siminf_prevalence_quantiles": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32,
                                                   ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                                                   _P, _P]),
    "siminf_mlp_create": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.c_int32, ctypes.POINTER(_P)]),
    "siminf_mlp_set_params": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "siminf_mlp_get_params": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "siminf_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P]),
    "siminf_mlp_backward": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P]),
    "siminf_mlp_get_grads": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "siminf_mlp_adamw": (ctypes.c_int, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, _P]),
    "siminf_mlp_destroy": (None, [_P]),
    "siminf_mlp_ensemble_predict": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "siminf_mlp_ensemble_predict_static": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P, _P, _P,
                                                          _P]),
    "siminf_define_model": (ctypes.c_int, [ctypes.POINTER(ModelDef), ctypes.POINTER(ctypes.c_int32), _P, _P,
                                           ctypes.c_char_p, ctypes.c_size_t]),
    "siminf_generated_source": (ctypes.c_int, [ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "siminf_gemm_bf16": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                                        ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                                        _P]),
}

_lib = None

# Handles still open are closed by an exit hook while the HIP runtime is
# certainly alive, rather than by __del__ during interpreter teardown.
_live = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass


def load():
    """Load libsiminf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1605_01421_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
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
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


_defined: dict = {}


def define_model(transitions, compartments, gdata_names=(), ldata_names=(), v_names=(), E=None, N=None) -> dict:
    """Parses and compiles a model given as transition strings
    "from -> propensity -> to" (siminf_define_model); returns dict(id, S, G)
    with S (Nc, Nt) and G (Nt, Nt) as the library derived them.  Definitions
    are cached per process by their text and tables."""
    nc, nt = len(compartments), len(transitions)
    E = np.zeros((nc, 0), np.int32) if E is None else np.asarray(E, dtype=np.int32).reshape(nc, -1)
    N = np.zeros((nc, 0), np.int32) if N is None else np.asarray(N, dtype=np.int32).reshape(nc, -1)
    key = (tuple(transitions), tuple(compartments), tuple(gdata_names), tuple(ldata_names), tuple(v_names),
           E.tobytes(), E.shape, N.tobytes(), N.shape)
    if key in _defined:
        return _defined[key]
    lib = load()

    def strings(xs):
        arr = (ctypes.c_char_p * max(len(xs), 1))(*[x.encode() for x in xs])
        return arr, ctypes.cast(arr, _P)

    keep = [strings(list(transitions)), strings(list(compartments)), strings(list(gdata_names)),
            strings(list(ldata_names)), strings(list(v_names))]
    Ef = _c(E.ravel(order="F"), np.int32)
    Nf = _c(N.ravel(order="F"), np.int32)
    d = ModelDef(nt, keep[0][1], nc, keep[1][1], len(gdata_names), keep[2][1], len(ldata_names), keep[3][1],
                 len(v_names), keep[4][1], E.shape[1], _ptr(Ef), N.shape[1], _ptr(Nf))
    mid = ctypes.c_int32(-1)
    S = np.zeros(nc * nt, np.int32)
    G = np.zeros(nt * nt, np.int32)
    msg = ctypes.create_string_buffer(8192)
    rc = lib.siminf_define_model(ctypes.byref(d), ctypes.byref(mid), _ptr(S), _ptr(G), msg, len(msg))
    if rc != SIMINF_OK:
        err = SiminfError(rc, "siminf_define_model: " + msg.value.decode(errors="replace"))
        raise err
    out = dict(id=int(mid.value), S=S.reshape(nc, nt, order="F"), G=G.reshape(nt, nt, order="F"))
    _defined[key] = out
    return out


def generated_source(model_id: int) -> str:
    lib = load()
    need = ctypes.c_size_t(0)
    lib.siminf_generated_source(model_id, None, 0, ctypes.byref(need))
    buf = ctypes.create_string_buffer(need.value)
    if lib.siminf_generated_source(model_id, buf, len(buf), None) != SIMINF_OK:
        raise SiminfError(SIMINF_E_ARG, "siminf_generated_source")
    return buf.value.decode()


def _marshal(spec, keep: list) -> Spec:
    """Fill a siminf_spec from a model specification object (see workloads)."""
    gen = None
    if getattr(spec, "mparse", None) is not None:
        mp = spec.mparse
        gen = define_model(mp["transitions"], mp["compartments"], mp.get("gdata_names", ()),
                           mp.get("ldata_names", ()), mp.get("v_names", ()), spec.E, spec.N)
        S, G = gen["S"], gen["G"]
    else:
        S, G = np.asarray(spec.S), np.asarray(spec.G)
    Nc, Nt = S.shape
    u0 = _c(spec.u0, np.int32)
    Nn = u0.shape[0]
    v0 = _c(_per_node(spec.v0, Nn), np.float64)
    ld = _c(_per_node(spec.ldata, Nn), np.float64)
    E = np.asarray(spec.E)
    N = np.asarray(spec.N)
    arrays = dict(S=_c(S.ravel(order="F"), np.int32), G=_c(np.asarray(G).ravel(order="F"), np.int32),
                  u0=u0, v0=v0, ldata=ld, gdata=_c(spec.gdata, np.float64),
                  tspan=_c(spec.tspan, np.float64), E=_c(E.ravel(order="F"), np.int32),
                  N=_c(N.ravel(order="F"), np.int32))
    ev = spec.events
    for k in ("event", "time", "node", "dest", "n", "select", "shift"):
        arrays["ev_" + k] = _c(ev[k], np.int32)
    arrays["ev_prop"] = _c(ev["proportion"], np.float64)
    keep.append(arrays)
    s = Spec()
    s.model = gen["id"] if gen is not None else int(spec.model)
    s.Nc, s.Nt, s.Nn = Nc, Nt, Nn
    s.Nv, s.Nld = v0.shape[1], ld.shape[1]
    s.Ngd, s.Ntspan = arrays["gdata"].size, arrays["tspan"].size
    for f in ("S", "G", "u0", "v0", "ldata", "gdata", "tspan", "E", "N"):
        setattr(s, f, _ptr(arrays[f]))
    s.Nev = arrays["ev_event"].size
    s.Ecols = E.shape[1] if E.ndim == 2 else 0
    s.Ncols = N.shape[1] if N.ndim == 2 else 0
    s.ev_type = _ptr(arrays["ev_event"])
    for k in ("time", "node", "dest", "n", "select", "shift", "prop"):
        setattr(s, "ev_" + k, _ptr(arrays["ev_" + k]))
    nb = getattr(spec, "neighbours", None)
    if nb is not None:
        arrays["nb_ptr"] = _c(nb["ptr"], np.int32)
        arrays["nb_idx"] = _c(nb["idx"], np.int32)
        arrays["nb_dist"] = _c(nb["dist"], np.float64)
        s.Nnb = arrays["nb_idx"].size
        s.nb_ptr = _ptr(arrays["nb_ptr"])
        s.nb_idx = _ptr(arrays["nb_idx"])
        s.nb_dist = _ptr(arrays["nb_dist"])
    return s


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Model:
    """A run (or a batch of runs) resident on the current HIP device.

    ``Model(spec)`` creates one run; ``Model([(spec, replicates), ...])`` a
    batch.  ``run`` enqueues the whole simulation on a HIP stream (torch's
    current stream by default); ``wait``/``trajectory``/``sums``/``counters``
    synchronise."""

    def __init__(self, spec, record: int = RECORD_FULL, block: int = 0, order: int = 0,
                 lanes: int = 0, max_blocks: int = 0, pipeline: int = 0, mode: int = 0, wide: int = 0,
                 lattice: int = 0, wait_ms: int = 0, graph: int = 0, pack: int = 0, group: int = 0,
                 lane_queue: int = 0, chunk: int = 0, batch: int = 0, solver: str = "ssm"):
        lib = load()
        self._lib = lib
        self._h = ctypes.c_void_p()
        opt = Options(record, block, order, lanes, max_blocks, pipeline, mode, wide, lattice, wait_ms, graph, pack,
                      group, lane_queue, chunk, batch, {"ssm": 0, "aem": 1}[solver])
        keep: list = []
        if isinstance(spec, (list, tuple)):
            specs = [s for s, _ in spec]
            reps = np.asarray([r for _, r in spec], dtype=np.int32)
            arr = (Spec * len(specs))(*[_marshal(s, keep) for s in specs])
            rc = lib.siminf_create_batch(arr, len(specs), _ptr(reps), ctypes.byref(opt), ctypes.byref(self._h))
            self.specs = specs
            self.replicates = [int(r) for r in reps]
        else:
            s = _marshal(spec, keep)
            rc = lib.siminf_create(ctypes.byref(s), ctypes.byref(opt), ctypes.byref(self._h))
            self.specs = [spec]
            self.replicates = [1]
        self.record = record
        if rc != SIMINF_OK:
            info = self.error_info() if self._h.value else None
            self.close()
            err = SiminfError(rc, "siminf_create")
            err.info = info
            raise err
        shape = np.zeros(6, dtype=np.int64)
        lib.siminf_shape(self._h, _ptr(shape))
        self.runs, self.total_nodes, self.ntspan, self.ncmax, self.nvmax, self.n_steps = (int(x) for x in shape)
        self.run_spec = [k for k, r in enumerate(self.replicates) for _ in range(r)]
        _live.add(self)

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.siminf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be gone at exit)
        if _finalizing():
            return  # the process is ending: the device memory goes with it
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- running -------------------------------------------------------------
    def run(self, seed: int, stream_base: int = 0, hip_stream=None):
        rc = self._lib.siminf_run(self._h, ctypes.c_uint64(seed & (2**64 - 1)),
                                  ctypes.c_uint32(stream_base), _stream_handle(hip_stream))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_run")
        return self

    def wait(self) -> int:
        return int(self._lib.siminf_wait(self._h))

    def error_info(self) -> dict:
        code = ctypes.c_int32()
        step = ctypes.c_int64()
        phase = ctypes.c_int32()
        index = ctypes.c_int64()
        run = ctypes.c_int32()
        self._lib.siminf_error_info(self._h, ctypes.byref(code), ctypes.byref(step), ctypes.byref(phase),
                                    ctypes.byref(index), ctypes.byref(run))
        buf = ctypes.create_string_buffer(256)
        self._lib.siminf_error_message(self._h, buf, len(buf))
        return dict(code=code.value, name=STATUS.get(code.value, str(code.value)), step=step.value,
                    phase=phase.value, index=index.value, run=run.value, message=buf.value.decode())

    def counters(self) -> dict:
        out = np.zeros(4, dtype=np.uint64)
        rc = self._lib.siminf_counters(self._h, _ptr(out))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_counters")
        return dict(transitions=int(out[0]), node_days=int(out[1]), events=int(out[2]), draws=int(out[3]))

    def timing(self) -> dict:
        """Milliseconds of the last run's SSA kernels and of the whole run."""
        out = np.zeros(2, dtype=np.float64)
        rc = self._lib.siminf_timing(self._h, _ptr(out))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_timing")
        return dict(kernel_ms=float(out[0]), run_ms=float(out[1]))

    def launch_info(self) -> dict:
        out = np.zeros(12, dtype=np.int32)
        self._lib.siminf_launch_info(self._h, _ptr(out))
        return dict(block=int(out[0]), blocks=int(out[1]), mode=int(out[2]), pipeline=int(out[3]),
                    order=int(out[4]), wide=int(out[5]), pack=int(out[6]), group=int(out[7]),
                    chunk=int(out[8]), lds=int(out[9]), batch=int(out[10]), groups=int(out[11]))

    def autotune(self, seed: int = 1, repeats: int = 2, hip_stream=None) -> float:
        """Pick the fastest launch shape (see siminf_autotune); returns its ms."""
        best = ctypes.c_double()
        rc = self._lib.siminf_autotune(self._h, ctypes.c_uint64(seed), repeats, _stream_handle(hip_stream),
                                       ctypes.byref(best))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_autotune")
        return best.value

    # -- results ---------------------------------------------------------------
    def trajectory(self, run: int = 0, device: bool = False):
        """U (Ntspan, Nn, Nc) int32 and V (Ntspan, Nn, Nv) float64 of one run --
        the paper's column-major U/V viewed per time point.  With
        device=True they are torch tensors on the current device."""
        spec = self.specs[self.run_spec[run]]
        Nn, Nc = spec.u0.shape
        Nv = np.asarray(spec.v0).reshape(Nn, -1).shape[1] if Nn else 0
        if device:
            import torch
            U = torch.empty((self.ntspan, Nn, Nc), dtype=torch.int32, device="cuda")
            V = torch.empty((self.ntspan, Nn, Nv), dtype=torch.float64, device="cuda")
            rc = self._lib.siminf_trajectory(self._h, run, ctypes.c_void_p(U.data_ptr()),
                                             ctypes.c_void_p(V.data_ptr()) if Nv else None, 1)
        else:
            U = np.empty((self.ntspan, Nn, Nc), dtype=np.int32)
            V = np.empty((self.ntspan, Nn, Nv), dtype=np.float64)
            rc = self._lib.siminf_trajectory(self._h, run, _ptr(U), _ptr(V), 0)
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_trajectory")
        return U, V

    def trajectory_sparse(self, pattern, which: str = "U", run: int = 0) -> np.ndarray:
        """The entries of U (or V) at the nonzeros of `pattern`, a
        scipy.sparse matrix of shape (Nn*Nc (or Nn*Nv), Ntspan) in the
        paper's layout (Table 1, U_sparse / V_sparse); returns a CSC matrix
        with the same pattern and the recorded values (binary64)."""
        import scipy.sparse as sp
        P = sp.csc_matrix(pattern)
        P.sort_indices()
        col_ptr = _c(P.indptr, np.int64)
        rows = _c(P.indices, np.int32)
        vals = np.zeros(rows.size, dtype=np.float64)
        rc = self._lib.siminf_trajectory_sparse(self._h, run, 0 if which == "U" else 1, rows.size, _ptr(col_ptr),
                                                _ptr(rows), _ptr(vals), 0)
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_trajectory_sparse")
        return sp.csc_matrix((vals, P.indices.copy(), P.indptr.copy()), shape=P.shape)

    def sums(self) -> np.ndarray:
        """Per-run compartment sums over nodes, int64 (runs, Ntspan, Nc_max)."""
        out = np.empty((self.runs, self.ntspan, self.ncmax), dtype=np.int64)
        rc = self._lib.siminf_sums(self._h, _ptr(out), 0)
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_sums")
        return out

    def prevalence_quantiles(self, case_c: int, at_risk, replicates: int, k0: int, nk: int,
                             probs=(0.1, 0.5, 0.9), hip_stream=None):
        """Type-7 quantiles over each set's replicates of the population
        prevalence sums[case_c] / sums[at_risk] at tspan indices k0..k0+nk-1.
        Returns a float32 torch tensor (sets, nk, len(probs)) on the device."""
        import torch
        mask = 0
        for c in at_risk:
            mask |= 1 << int(c)
        p = _c(probs, np.float64)
        sets = self.runs // replicates
        out = torch.empty((sets, nk, p.size), dtype=torch.float32, device="cuda")
        rc = self._lib.siminf_prevalence_quantiles(self._h, case_c, mask, replicates, k0, nk, _ptr(p), p.size,
                                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(hip_stream))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_prevalence_quantiles")
        return out


def header_symbols(header_path: str) -> list:
    """Names of the functions include/siminf.h declares."""
    import re
    text = open(header_path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(siminf_[a-z_0-9]+)\s*\(", text)))


class MLP:
    """The surrogate network of the library (siminf_mlp_*): weights and
    optimiser state live on the device; data are torch float32 CUDA tensors."""

    def __init__(self, dims, max_batch: int):
        lib = load()
        self._lib = lib
        self.dims = [int(d) for d in dims]
        d = np.asarray(self.dims, dtype=np.int32)
        self._h = ctypes.c_void_p()
        rc = lib.siminf_mlp_create(len(self.dims) - 1, _ptr(d), int(max_batch), ctypes.byref(self._h))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_mlp_create")
        self.max_batch = int(max_batch)
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.siminf_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be gone at exit)
        if _finalizing():
            return  # the process is ending: the device memory goes with it
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        for l, (W, b) in enumerate(params):
            Wf = _c(W, np.float32)
            bf = _c(b, np.float32)
            rc = self._lib.siminf_mlp_set_params(self._h, l, _ptr(Wf), _ptr(bf))
            if rc != SIMINF_OK:
                raise SiminfError(rc, "siminf_mlp_set_params")

    def get_params(self):
        out = []
        for l in range(len(self.dims) - 1):
            W = np.empty((self.dims[l + 1], self.dims[l]), dtype=np.float32)
            b = np.empty(self.dims[l + 1], dtype=np.float32)
            rc = self._lib.siminf_mlp_get_params(self._h, l, _ptr(W), _ptr(b))
            if rc != SIMINF_OK:
                raise SiminfError(rc, "siminf_mlp_get_params")
            out.append((W, b))
        return out

    def get_grads(self):
        out = []
        for l in range(len(self.dims) - 1):
            W = np.empty((self.dims[l + 1], self.dims[l]), dtype=np.float32)
            b = np.empty(self.dims[l + 1], dtype=np.float32)
            rc = self._lib.siminf_mlp_get_grads(self._h, l, _ptr(W), _ptr(b))
            if rc != SIMINF_OK:
                raise SiminfError(rc, "siminf_mlp_get_grads")
            out.append((W, b))
        return out

    def forward(self, X, Y=None, hip_stream=None):
        import torch
        B = X.shape[0]
        if Y is None:
            Y = torch.empty((B, self.dims[-1]), dtype=torch.float32, device=X.device)
        rc = self._lib.siminf_mlp_forward(self._h, ctypes.c_void_p(X.data_ptr()), B,
                                          ctypes.c_void_p(Y.data_ptr()), _stream_handle(hip_stream))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_mlp_forward")
        return Y

    def backward(self, X, T, probs=(0.1, 0.5, 0.9), want_loss=True, hip_stream=None):
        p = _c(probs, np.float64)
        loss = ctypes.c_double()
        rc = self._lib.siminf_mlp_backward(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                           X.shape[0], _ptr(p), p.size,
                                           ctypes.byref(loss) if want_loss else None, _stream_handle(hip_stream))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_mlp_backward")
        return loss.value if want_loss else None

    def adamw(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, hip_stream=None):
        rc = self._lib.siminf_mlp_adamw(self._h, lr, beta1, beta2, eps, weight_decay, _stream_handle(hip_stream))
        if rc != SIMINF_OK:
            raise SiminfError(rc, "siminf_mlp_adamw")


def ensemble_predict(nets, X, y_mean, y_std, hip_stream=None, static=False, out=None):
    """siminf_mlp_ensemble_predict (static=True: the variant that allocates
    nothing, siminf_mlp_ensemble_predict_static): mean prediction (B, N) and
    disagreement (B,) of the networks `nets` (MLP objects) on X (B, dims[0]);
    y_mean, y_std are float32 CUDA tensors of the output width.  Torch
    tensors; `out` = (Y, dis) preallocated tensors to write into."""
    import torch
    B, N = X.shape[0], nets[0].dims[-1]
    if out is None:
        Y = torch.empty((B, N), dtype=torch.float32, device=X.device)
        dis = torch.empty((B,), dtype=torch.float32, device=X.device)
    else:
        Y, dis = out
    arr = (ctypes.c_void_p * len(nets))(*[n._h.value for n in nets])
    fn = load().siminf_mlp_ensemble_predict_static if static else load().siminf_mlp_ensemble_predict
    rc = fn(ctypes.cast(arr, ctypes.c_void_p), len(nets),
                                            ctypes.c_void_p(X.data_ptr()), B,
                                            ctypes.c_void_p(y_mean.data_ptr()), ctypes.c_void_p(y_std.data_ptr()),
                                            ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(dis.data_ptr()),
                                            _stream_handle(hip_stream))
    if rc != SIMINF_OK:
        raise SiminfError(rc, "siminf_mlp_ensemble_predict")
    return Y, dis


def gemm_bf16(A_bits, B_bits, M, N, K, lda, a_trans, ldb, b_trans, C, ldc, hip_stream=None):
    """siminf_gemm_bf16 on torch int16/uint16 tensors holding bfloat16 bit patterns."""
    rc = load().siminf_gemm_bf16(M, N, K, ctypes.c_void_p(A_bits.data_ptr()), lda, a_trans,
                                 ctypes.c_void_p(B_bits.data_ptr()), ldb, b_trans,
                                 ctypes.c_void_p(C.data_ptr()), ldc, _stream_handle(hip_stream))
    if rc != SIMINF_OK:
        raise SiminfError(rc, "siminf_gemm_bf16")
