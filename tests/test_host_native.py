"""Host-side native checks (no GPU): the dataflow kernel's XCD-aware
workgroup numbering is a bijection, and the CPU oracle runs clean under
AddressSanitizer and UndefinedBehaviorSanitizer with the same bits as its
normal build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1605_01421_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NATIVE = os.path.join(HERE, "native")


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return tmp_path_factory.mktemp("native")


def test_xcd_workgroup_numbering_is_a_bijection(workdir):
    """xcd_block (the library's own header, built for the host) maps every
    grid of 1..2500 workgroups onto itself one to one, for every start of
    the renumbered range and line group, and gives each XCD g consecutive
    slots per span."""
    exe = str(workdir / "xcd_check")
    _compile(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
              "-I" + os.path.join(ROOT, "paper_1605_01421_amd", "csrc"),
              os.path.join(NATIVE, "xcd_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr


def _write_model(path, spec, seed, stream, nthreads):
    S = np.asarray(spec.S, np.int32)
    Nc, Nt = S.shape
    u0 = np.asarray(spec.u0, np.int32)
    Nn = u0.shape[0]
    v0 = np.asarray(spec.v0, np.float64).reshape(Nn, -1)
    ld = np.asarray(spec.ldata, np.float64).reshape(Nn, -1)
    E, N = np.asarray(spec.E, np.int32), np.asarray(spec.N, np.int32)
    ev = spec.events
    head = np.array([spec.model, Nc, Nt, Nn, v0.shape[1], ld.shape[1], np.asarray(spec.gdata).size,
                     np.asarray(spec.tspan).size, len(ev["event"]), E.shape[1], N.shape[1], nthreads], np.int32)
    with open(path, "wb") as f:
        head.tofile(f)
        np.array([seed], np.uint64).tofile(f)
        np.array([stream], np.uint32).tofile(f)
        for a in (S.ravel(order="F"), np.asarray(spec.G, np.int32).ravel(order="F"), u0.ravel()):
            np.ascontiguousarray(a, np.int32).tofile(f)
        for a in (v0.ravel(), ld.ravel(), np.asarray(spec.gdata, np.float64), np.asarray(spec.tspan, np.float64)):
            np.ascontiguousarray(a, np.float64).tofile(f)
        for k in ("event", "time", "node", "dest", "n", "select", "shift"):
            np.ascontiguousarray(ev[k], np.int32).tofile(f)
        np.ascontiguousarray(ev["proportion"], np.float64).tofile(f)
        np.ascontiguousarray(E.ravel(order="F"), np.int32).tofile(f)
        np.ascontiguousarray(N.ravel(order="F"), np.int32).tofile(f)
    return Nn, Nc, v0.shape[1], np.asarray(spec.tspan).size


def _cases():
    rng = np.random.default_rng(3)
    err_rows = [(W.EXTTRANS, 2, 0, 1, 5, 0.0, 0, -1), (W.EXTTRANS, 2, 0, 2, 1, 0.0, 0, -1),
                (W.EXTTRANS, 2, 1, 2, 11, 0.0, 0, -1)]
    return {
        "five-node-example": (W.sir_event_example(True), 3, 0),
        "shifts": (W.sir_with_shifts(seed=6, Nn=300, days=30), 29, 2),
        "sir-events": (W.sir_with_events(seed=4, Nn=500, days=40), 7, 1),
        "sise-events": (W.sise_with_events(seed=5, Nn=400, days=60), 9, 0),
        "overdraw": (W.sir_spec(np.array([[5, 0, 0]] * 3), [0, 1, 2, 3], 0.0, 0.1,
                                events=W.make_events(err_rows)), 1, 0),
        "bad-rate": (W.sir_spec(np.array([[5, 1, 0], [5, 2, 0]]), [0, 1, 2], -0.1, 0.1), 1, 0),
        "birth-death": (W.birth_death_spec(rng.integers(0, 50, 64), np.arange(0, 8), 0.4, 0.5), 2, 0),
    }


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_address_and_undefined_sanitizers(workdir, orc):
    """The oracle built with -fsanitize=address,undefined (errors abort) on
    the event example, shifted and proportional events, both event
    workloads, two error paths and a birth-death run, with 1 and 4 threads:
    no report, and U, V, counters and error keys equal the normal build's."""
    exe = str(workdir / "oracle_asan")
    _compile(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
              "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              os.path.join(NATIVE, "oracle_driver.c"), "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=99",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    for name, (spec, seed, stream) in _cases().items():
        for threads in (1, 4):
            fin, fout = str(workdir / f"{name}.in"), str(workdir / f"{name}.out")
            Nn, Nc, Nv, Nt = _write_model(fin, spec, seed, stream, threads)
            r = subprocess.run([exe, fin, fout], capture_output=True, text=True, env=env, timeout=300)
            assert r.returncode == 0, f"{name}: {r.stderr[-3000:]}"
            assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
            raw = np.fromfile(fout, dtype=np.uint8)
            head = raw[:64].view(np.int64)
            U = raw[64:64 + 4 * Nt * Nn * Nc].view(np.int32).reshape(Nt, Nn, Nc)
            V = raw[64 + 4 * Nt * Nn * Nc:].view(np.float64).reshape(Nt, Nn, Nv)
            ref = orc.run(spec, seed, stream, nthreads=threads)
            assert int(head[0]) == ref["status"], name
            assert tuple(int(x) for x in head[1:5]) == ref["error"], name
            assert (int(head[5]), int(head[6]), int(head[7])) == (ref["transitions"], ref["node_days"],
                                                                  ref["events"]), name
            if ref["status"] == 0:
                assert np.array_equal(U, ref["U"]), name
                assert np.array_equal(V, ref["V"]), name
