"""The oracle's reading of a model given as transition strings (section 5.1,
the model parser): test infrastructure, independent of the library's parser.

A transition is "from -> propensity -> to".  `from` and `to` are "@" (the
empty set) or terms "X" or "k*X" (k a positive integer) joined by '+'; the
transition's column of the state-change matrix S is to - from.  The
propensity is an arithmetic expression in numbers, compartment names (the
counts, converted to binary64), global data names, local data names and
continuous state names, with + - * / (left-associative; * and / before + and
-), unary - and +, and parentheses.  It is turned into a postfix program that
the C oracle runs on a stack of binary64 values, one IEEE operation per
operator.  The dependency graph marks rate k for recomputation after
transition j (G[k, j] = 1) when propensity k reads a compartment that
transition j changes.
"""
from __future__ import annotations

import re

import numpy as np

OP_CONST, OP_U, OP_GD, OP_LD, OP_V, OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_NEG = range(10)
_BINARY = {"+": OP_ADD, "-": OP_SUB, "*": OP_MUL, "/": OP_DIV}
_TOKEN = re.compile(r"\s*(?:(?P<num>(?:\d+\.?\d*|\.\d+)(?:[eE][+-]?\d+)?)|(?P<name>[A-Za-z_][A-Za-z0-9_]*)"
                    r"|(?P<op>[-+*/()]))", re.ASCII)


class ParseError(ValueError):
    pass


def _tokens(text: str):
    pos, out = 0, []
    text = text.rstrip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            raise ParseError(f"unexpected character at {pos} in {text!r}")
        pos = m.end()
        if m.group("num") is not None:
            out.append(("num", float(m.group("num"))))
        elif m.group("name") is not None:
            out.append(("name", m.group("name")))
        else:
            out.append(("op", m.group("op")))
    return out


def expression(text: str, names: dict) -> tuple[list, list, set]:
    """Postfix program [(op, arg)], constants, and the compartment indices
    the expression reads.  names: name -> (op code, index)."""
    toks = _tokens(text)
    pos = 0
    prog, consts, comps = [], [], set()

    def peek():
        return toks[pos] if pos < len(toks) else None

    def take():
        nonlocal pos
        pos += 1
        return toks[pos - 1]

    def primary():
        t = peek()
        if t is None:
            raise ParseError(f"expression ends early: {text!r}")
        if t == ("op", "("):
            take()
            add_expr()
            if peek() != ("op", ")"):
                raise ParseError(f"missing ')' in {text!r}")
            take()
            return
        if t[0] == "num":
            take()
            if not np.isfinite(t[1]):
                raise ParseError(f"number out of range in {text!r}")
            prog.append((OP_CONST, len(consts)))
            consts.append(t[1])
            return
        if t[0] == "name":
            take()
            if t[1] not in names:
                raise ParseError(f"unknown name {t[1]!r} in {text!r}")
            op, idx = names[t[1]]
            if op == OP_U:
                comps.add(idx)
            prog.append((op, idx))
            return
        raise ParseError(f"unexpected {t[1]!r} in {text!r}")

    def unary():
        t = peek()
        if t in (("op", "-"), ("op", "+")):
            take()
            unary()
            if t[1] == "-":
                prog.append((OP_NEG, 0))
            return
        primary()

    def mul_expr():
        unary()
        while peek() in (("op", "*"), ("op", "/")):
            op = take()[1]
            unary()
            prog.append((_BINARY[op], 0))

    def add_expr():
        mul_expr()
        while peek() in (("op", "+"), ("op", "-")):
            op = take()[1]
            mul_expr()
            prog.append((_BINARY[op], 0))

    add_expr()
    if pos != len(toks):
        raise ParseError(f"unexpected {toks[pos][1]!r} in {text!r}")
    return prog, consts, comps


def side(text: str, comp: dict, nc: int) -> np.ndarray:
    cnt = np.zeros(nc, dtype=np.int64)
    text = text.strip()
    if text == "@":
        return cnt
    for term in text.split("+"):
        term = term.strip()
        k = 1
        if "*" in term:
            num, term = term.split("*", 1)
            num, term = num.strip(), term.strip()
            if not num.isdigit() or not 1 <= int(num) <= 1000000:
                raise ParseError(f"bad coefficient in {text!r}")
            k = int(num)
        if term not in comp:
            raise ParseError(f"unknown compartment {term!r} in {text!r}")
        cnt[comp[term]] += k
    return cnt


def compile_model(transitions, compartments, gdata_names=(), ldata_names=(), v_names=()) -> dict:
    """S (Nc, Nt), G (Nt, Nt), and the propensities as one program:
    prog_off (Nt + 1), prog (op | index << 8), consts."""
    names = {}
    for op, lst in ((OP_U, compartments), (OP_GD, gdata_names), (OP_LD, ldata_names), (OP_V, v_names)):
        for i, nm in enumerate(lst):
            if nm in names or not re.fullmatch(r"[A-Za-z_][A-Za-z0-9_]*", nm, re.ASCII):
                raise ParseError(f"bad or repeated name {nm!r}")
            names[nm] = (op, i)
    comp = {nm: i for i, nm in enumerate(compartments)}
    nc, nt = len(compartments), len(transitions)
    S = np.zeros((nc, nt), dtype=np.int32)
    reads = []
    prog_off, prog, consts = [0], [], []
    for j, tr in enumerate(transitions):
        parts = tr.split("->")
        if len(parts) != 3:
            raise ParseError(f"a transition needs the form 'from -> propensity -> to': {tr!r}")
        S[:, j] = side(parts[2], comp, nc) - side(parts[0], comp, nc)
        p, c, used = expression(parts[1], names)
        base = len(consts)
        for op, arg in p:
            prog.append(op | ((arg + base if op == OP_CONST else arg) << 8))
        consts.extend(c)
        prog_off.append(len(prog))
        reads.append(used)
    G = np.zeros((nt, nt), dtype=np.int32)
    for j in range(nt):
        changed = set(np.nonzero(S[:, j])[0].tolist())
        for k in range(nt):
            if reads[k] & changed:
                G[k, j] = 1
    return dict(S=S, G=G, prog_off=np.asarray(prog_off, dtype=np.int32),
                prog=np.asarray(prog, dtype=np.int32), consts=np.asarray(consts, dtype=np.float64))
