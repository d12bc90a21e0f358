"""CPU checks of the C-ABI boundary: the library loads and exports every
entry point include/siminf.h declares (no compute calls without a GPU)."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "siminf.h")


def test_library_exports_every_declared_symbol():
    from paper_1605_01421_amd import siminf
    lib = siminf.load()
    declared = siminf.header_symbols(HEADER)
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(lib, name), name
    # the binding marshals exactly the declared entry points
    assert sorted(siminf.SIGNATURES) == declared


def test_exported_symbols_are_plain_c():
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_1605_01421_amd", "libsiminf.so")],
                         check=True, capture_output=True, text=True).stdout
    names = {line.split()[-1] for line in out.splitlines() if " T " in line}
    from paper_1605_01421_amd import siminf
    for name in siminf.header_symbols(HEADER):
        assert name in names, name  # unmangled: extern "C"


def test_status_strings_without_device():
    from paper_1605_01421_amd import siminf
    lib = siminf.load()
    for code, name in siminf.STATUS.items():
        assert lib.siminf_status_string(code).decode() == name


def test_header_compiles_as_c():
    src = '#include "siminf.h"\nint main(void){ siminf_spec s; (void)s; return SIMINF_OK; }\n'
    p = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        "-x", "c", "-", "-o", "/dev/null"], input=src, text=True, capture_output=True)
    assert p.returncode == 0, p.stderr


def test_product_does_not_use_the_oracle():
    """The library and its binding never load the oracle."""
    pkg = os.path.join(ROOT, "paper_1605_01421_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "siminf_oracle" not in text, f


@pytest.mark.parametrize("opts,code", [(dict(pack=3), -1), (dict(pack=128), -1), (dict(group=-2), -1),
                                       (dict(block=96), -1), (dict(block=512), -1), (dict(lattice=3), -1),
                                       (dict(pipeline=3), -1), (dict(mode=3), -1), (dict(graph=2), -1),
                                       (dict(wait_ms=-1), -1), (dict(record=5), -1), (dict(lanes=2), -2)])
def test_invalid_options_rejected_before_the_device(opts, code):
    """siminf_create checks the launch options before it touches a device,
    so a bad value is reported the same way with or without a GPU."""
    from paper_1605_01421_amd import siminf, workloads as W
    with pytest.raises(siminf.SiminfError) as e:
        siminf.Model(W.plain_sir(), **opts)
    assert e.value.code == code
