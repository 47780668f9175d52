"""General index-notation oracle (test infrastructure).

Evaluates a statement of tensor index notation (paper, Sec. II-A) of the form
``Out(free) = +- T1 +- T2 ...``, each term a product of tensor accesses, by its
plain definition: every index variable takes every coordinate of its extent,
a variable missing from the left side is summed, and a sparse operand's entry
is its stored value when the coordinate is stored and 0 otherwise.  Arithmetic
is exact (``fractions.Fraction`` over the float64 inputs) and rounded once to
float64; S, the sum of |product| over every term and summed coordinate, is
returned beside each output entry.  Only for tiny extents: the cost is the
product of all extents.

The output pattern of a sparse (CSR) left side ``A(i,j)`` is structural (the
two-phase assembly of Sec. V-B): (i, j) is stored when some term's sparse
operands that index j all store the coordinate prefix that ends at j (the
intersection within a product, the union across a sum); a term none of whose
sparse operands index j stores every j.  Values at stored coordinates follow
the definition above, so an entry whose value cancels to 0 stays stored.

Shares no code with the GPU library: its own parser, its own traversal of the
pos/crd arrays.
"""
from __future__ import annotations

import itertools
import re
from fractions import Fraction

import numpy as np

_TOKEN = re.compile(r"\s*([A-Za-z_][A-Za-z0-9_]*|[()=+\-*,])")


def parse(stmt):
    """-> (lhs, terms) with lhs = (name, [vars]) and terms a list of
    (sign, [(name, [vars]), ...])."""
    toks, pos = [], 0
    stmt = stmt.strip()
    while pos < len(stmt):
        m = _TOKEN.match(stmt, pos)
        if not m:
            raise ValueError(f"cannot read {stmt[pos:]!r}")
        toks.append(m.group(1))
        pos = m.end()
    k = 0

    def access():
        nonlocal k
        name = toks[k]
        if not re.match(r"[A-Za-z_]", name):
            raise ValueError(f"expected a tensor name, got {name!r}")
        k += 1
        vars_ = []
        if k < len(toks) and toks[k] == "(":
            k += 1
            while toks[k] != ")":
                vars_.append(toks[k])
                k += 1
                if toks[k] == ",":
                    k += 1
            k += 1
        return name, vars_

    lhs = access()
    if toks[k] != "=":
        raise ValueError("expected '='")
    k += 1
    terms, sign = [], 1
    if toks[k] in "+-":
        sign = -1 if toks[k] == "-" else 1
        k += 1
    while True:
        factors = [access()]
        while k < len(toks) and toks[k] == "*":
            k += 1
            factors.append(access())
        terms.append((sign, factors))
        if k == len(toks):
            break
        sign = -1 if toks[k] == "-" else 1
        k += 1
    return lhs, terms


class Sparse:
    """A sparse operand as the oracle sees it: stored coordinate tuples with
    their values, and the stored prefixes of each level."""

    def __init__(self, entries, prefixes, shape):
        self.entries = entries      # {(i, j[, k]): value}
        self.prefixes = prefixes    # [set of 1-tuples, set of 2-tuples, ...]
        self.shape = tuple(shape)

    @classmethod
    def csr(cls, pos, crd, vals, shape):
        entries, p1 = {}, set()
        for i in range(shape[0]):
            for p in range(int(pos[i]), int(pos[i + 1])):
                entries[(i, int(crd[p]))] = float(vals[p])
                p1.add((i, int(crd[p])))
        return cls(entries, [{(i,) for i in range(shape[0])}, p1], shape)

    @classmethod
    def csf(cls, pos1, crd1, pos2, crd2, vals, shape):
        entries, p1, p2 = {}, set(), set()
        for i in range(shape[0]):
            for f in range(int(pos1[i]), int(pos1[i + 1])):
                j = int(crd1[f])
                p1.add((i, j))
                for p in range(int(pos2[f]), int(pos2[f + 1])):
                    entries[(i, j, int(crd2[p]))] = float(vals[p])
                    p2.add((i, j, int(crd2[p])))
        return cls(entries, [{(i,) for i in range(shape[0])}, p1, p2], shape)

    @classmethod
    def ddc(cls, pos2, crd2, vals, shape):
        I, J, _ = shape
        entries, p2 = {}, set()
        for i in range(I):
            for j in range(J):
                f = i * J + j
                for p in range(int(pos2[f]), int(pos2[f + 1])):
                    entries[(i, j, int(crd2[p]))] = float(vals[p])
                    p2.add((i, j, int(crd2[p])))
        # the middle level is Dense: every (i, j) is stored
        p1 = {(i, j) for i in range(I) for j in range(J)}
        return cls(entries, [{(i,) for i in range(I)}, p1, p2], shape)


def _extents(lhs, terms, operands, out_shape):
    ext = {}
    for _, factors in terms:
        for name, vs in factors:
            t = operands[name]
            shape = t.shape if isinstance(t, Sparse) else np.asarray(t).shape
            for v, d in zip(vs, shape):
                if ext.setdefault(v, d) != d:
                    raise ValueError(f"extent of {v} disagrees")
    for v, d in zip(lhs[1], out_shape or ()):
        if ext.setdefault(v, d) != d:
            raise ValueError(f"extent of {v} disagrees")
    return ext


def _value(t, vs, env):
    idx = tuple(env[v] for v in vs)
    if isinstance(t, Sparse):
        return t.entries.get(idx, 0.0)
    return float(np.asarray(t)[idx])


def evaluate(stmt, operands, out_shape=None, rows=None):
    """Value of every output entry and its S.  `operands` maps names to
    Sparse objects or numpy arrays.  Returns (values, S) as float64 arrays
    of the output's shape (shape () for a scalar left side); with `rows`,
    only those coordinates of the left side's first index, in that order
    (the first dimension then has len(rows) entries)."""
    lhs, terms = parse(stmt)
    ext = _extents(lhs, terms, operands, out_shape)
    free = lhs[1]
    summed = [v for v in ext if v not in free]
    ranges = [range(ext[v]) for v in free]
    if rows is not None:
        ranges[0] = [int(r) for r in rows]
    shape = tuple(len(r) for r in ranges)
    vals = np.zeros(shape, dtype=np.float64)
    S = np.zeros(shape, dtype=np.float64)
    for pos_, fc in zip(itertools.product(*[range(len(r)) for r in ranges]),
                        itertools.product(*ranges)):
        tot, mag = Fraction(0), Fraction(0)
        for rc in itertools.product(*[range(ext[v]) for v in summed]):
            env = dict(zip(free, fc))
            env.update(zip(summed, rc))
            for sign, factors in terms:
                prod = Fraction(1)
                for name, vs in factors:
                    prod *= Fraction(_value(operands[name], vs, env))
                tot += sign * prod
                mag += abs(prod)
        vals[pos_] = float(tot)
        S[pos_] = float(mag)
    return vals, S


def pattern(stmt, operands, out_shape):
    """Stored coordinates of a CSR left side A(i,j): the CSR arrays (pos,
    crd) of the structural pattern defined in the module docstring."""
    lhs, terms = parse(stmt)
    i, j = lhs[1]
    n, m = out_shape
    pos, crd = [0], []
    for a in range(n):
        for b in range(m):
            stored = False
            for _, factors in terms:
                ok = True
                for name, vs in factors:
                    t = operands[name]
                    if isinstance(t, Sparse) and j in vs:
                        level = vs.index(j)
                        env = {i: a, j: b}
                        prefix = tuple(env[v] for v in vs[:level + 1])
                        ok = ok and prefix in t.prefixes[level]
                stored = stored or ok
            if stored:
                crd.append(b)
        pos.append(len(crd))
    return np.asarray(pos, dtype=np.int32), np.asarray(crd, dtype=np.int32)
