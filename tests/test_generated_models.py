"""The library's model parser (siminf_define_model) against the oracle's:
both must derive the same S and G from the same strings and reject the same
malformed definitions.  Runs on the CPU: the definition parses and compiles
the kernels with hipRTC for gfx950, which needs no GPU."""
import numpy as np
import pytest

from oracle import mparse
from paper_1605_01421_amd import workloads as W

MODELS = [
    (W.INCIDENCE_SIR[0], W.INCIDENCE_SIR[1], ["b", "g"]),
    (["S -> b*S*I/(S+I+R) -> I", "I -> g*I -> R", "R -> w*R -> S"], ["S", "I", "R"], ["b", "g", "w"]),
    (["@ -> k -> 2*X + Y", "X + Y -> d*X*Y -> @", "Y -> 0.5e-1*Y/(1+X) -> X"], ["X", "Y"], ["k", "d"]),
]


@pytest.fixture(scope="module")
def lib():
    from paper_1605_01421_amd import siminf
    siminf.load()
    return siminf


@pytest.mark.parametrize("k", range(len(MODELS)))
def test_library_and_oracle_agree_on_s_and_g(lib, k):
    tr, comp, gd = MODELS[k]
    d = lib.define_model(tr, comp, gd)
    o = mparse.compile_model(tr, comp, gd)
    assert d["id"] >= 64
    assert np.array_equal(d["S"], o["S"]) and np.array_equal(d["G"], o["G"])


def test_generated_source_keeps_the_operation_order(lib):
    """The generated propensity is the parse tree, fully parenthesised, every
    leaf binary64, literals exact (hexadecimal)."""
    d = lib.define_model(*MODELS[2])
    src = lib.generated_source(d["id"])
    assert "((gd[1] * (double)u[0]) * (double)u[1])" in src
    assert "((0x1.999999999999ap-5 * (double)u[1]) / (0x1p+0 + (double)u[0]))" in src


@pytest.mark.parametrize("bad", [["S -> b*S*J -> I"], ["S -> b*S -> I -> R"], ["S -> b*S"], ["0*S -> b -> I"],
                                 ["S -> b*(S -> I"], ["S -> b*S) -> I"], ["S -> b S -> I"], ["S -> b* -> I"],
                                 ["Q -> b -> I"], ["S -> .e5 -> I"], ["S -> 1e999 -> I"]])
def test_both_parsers_reject(lib, bad):
    with pytest.raises(mparse.ParseError):
        mparse.compile_model(bad, ["S", "I"], ["b"])
    with pytest.raises(lib.SiminfError) as e:
        lib.define_model(bad, ["S", "I"], ["b"])
    assert e.value.code == -1
