"""Symbolic SU(3) colour algebra for one quark line and k gluons.

The colour factor of every Feynman diagram of q q~ + k gluons is expanded on
the trace basis T_s = (T^{a_s1} ... T^{a_sk})_{ij}, one element per ordering s
of the gluons, using f^{abc} T^c = -i [T^a, T^b] at every three-gluon vertex
(and twice at every four-gluon vertex).  The colour matrix
C_st = sum_colours conj(T_s) T_t is evaluated exactly (rational arithmetic)
with the SU(N) Fierz identity
    T^x_{ij} T^x_{kl} = 1/2 (delta_il delta_kj - delta_ij delta_kl / N).
These are the two ingredients of the "color algebra" part of the matrix
element named in section 3 of the paper; the method itself is the textbook
colour decomposition of tree amplitudes.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from itertools import permutations
from typing import Dict, List, Tuple

NC = 3

# A colour expansion maps an ordering of gluon legs to a Gaussian-integer
# coefficient (re, im).
Expansion = Dict[Tuple[int, ...], Tuple[int, int]]


def _cmul(a: Tuple[int, int], b: Tuple[int, int]) -> Tuple[int, int]:
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def _add_into(dst: Expansion, key, c) -> None:
    old = dst.get(key, (0, 0))
    new = (old[0] + c[0], old[1] + c[1])
    if new == (0, 0):
        dst.pop(key, None)
    else:
        dst[key] = new


def leaf(leg: int) -> Expansion:
    return {(leg,): (1, 0)}


def concat(a: Expansion, b: Expansion, scale=(1, 0)) -> Expansion:
    out: Expansion = {}
    for ka, ca in a.items():
        for kb, cb in b.items():
            _add_into(out, ka + kb, _cmul(_cmul(ca, cb), scale))
    return out


def add(a: Expansion, b: Expansion) -> Expansion:
    out = dict(a)
    for k, c in b.items():
        _add_into(out, k, c)
    return out


def commutator(a: Expansion, b: Expansion, scale=(1, 0)) -> Expansion:
    """scale * (A B - B A)"""
    neg = (-scale[0], -scale[1])
    return add(concat(a, b, scale), concat(b, a, neg))


MINUS_I = (0, -1)


def three_gluon(a: Expansion, b: Expansion) -> Expansion:
    """Off-shell gluon from legs (a, b) through f^{a b e}: T^e f^{abe} = -i [T^a, T^b]."""
    return commutator(a, b, MINUS_I)


def four_gluon(a: Expansion, b: Expansion, c: Expansion, s: int) -> Expansion:
    """Off-shell gluon (index d) from legs (a, b, c) for one of the three colour
    structures of the four-gluon vertex:
       s = 0: f^{abe} f^{cde} -> -[[A, B], C]
       s = 1: f^{ace} f^{bde} -> -[[A, C], B]
       s = 2: f^{ade} f^{bce} -> -[[B, C], A]
    """
    minus = (-1, 0)
    if s == 0:
        return commutator(commutator(a, b), c, minus)
    if s == 1:
        return commutator(commutator(a, c), b, minus)
    return commutator(commutator(b, c), a, minus)


def quark_line(blocks: List[Expansion]) -> Expansion:
    out: Expansion = {(): (1, 0)}
    for b in blocks:
        out = concat(out, b)
    return out


# --------------------------------------------------------------- colour matrix
def _canon(traces: Tuple[Tuple[int, ...], ...]):
    """Canonical form of a product of traces: relabel gluon indices in order of
    first appearance, rotate each trace to its lexicographically smallest
    rotation (after relabelling), sort the traces."""
    # iterate to a fixed point: relabelling depends on the order of traces
    best = None
    for _ in range(2):
        relabel: Dict[int, int] = {}
        for t in traces:
            for x in t:
                if x not in relabel:
                    relabel[x] = len(relabel)
        rel = [tuple(relabel[x] for x in t) for t in traces]
        rot = []
        for t in rel:
            if not t:
                rot.append(t)
                continue
            rot.append(min(t[i:] + t[:i] for i in range(len(t))))
        traces = tuple(sorted(rot))
        best = traces
    return best


@lru_cache(maxsize=None)
def _trace_product(traces: Tuple[Tuple[int, ...], ...]) -> Fraction:
    """Value of prod_t Tr(T^{x_t1} ...), each index summed over 1..N^2-1
    and appearing exactly twice in total."""
    # empty traces give N, traces of a single generator vanish
    rest = []
    factor = Fraction(1)
    for t in traces:
        if len(t) == 0:
            factor *= NC
        elif len(t) == 1:
            return Fraction(0)
        else:
            rest.append(t)
    if not rest:
        return factor
    traces = tuple(rest)
    t0 = traces[0]
    x = t0[0]
    # find the partner of x
    for ti, t in enumerate(traces):
        start = 1 if ti == 0 else 0
        for pos in range(start, len(t)):
            if t[pos] == x:
                others = traces[1:ti] + traces[ti + 1:] if ti != 0 else traces[1:]
                if ti == 0:
                    # Tr(T^x B T^x C) = 1/2 [Tr(B) Tr(C) - Tr(B C) / N]
                    B = t0[1:pos]
                    C = t0[pos + 1:]
                    a = _trace_product(_canon(others + (B, C)))
                    b = _trace_product(_canon(others + (B + C,)))
                    return factor * (Fraction(1, 2) * a - Fraction(1, 2 * NC) * b)
                # Tr(T^x A) Tr(T^x B) = 1/2 [Tr(A B) - Tr(A) Tr(B) / N]
                A = t0[1:]
                Bt = t[pos + 1:] + t[:pos]
                a = _trace_product(_canon(others + (A + Bt,)))
                b = _trace_product(_canon(others + (A, Bt)))
                return factor * (Fraction(1, 2) * a - Fraction(1, 2 * NC) * b)
    raise ValueError("unpaired colour index")


def colour_matrix(orderings: List[Tuple[int, ...]]) -> List[List[Fraction]]:
    """C_st = sum_colours conj((T_s)_{ij}) (T_t)_{ij}
            = Tr(T^{s_k} ... T^{s_1} T^{t_1} ... T^{t_k})."""
    n = len(orderings)
    C = [[Fraction(0)] * n for _ in range(n)]
    for i, s in enumerate(orderings):
        for j, t in enumerate(orderings):
            if j < i:
                C[i][j] = C[j][i]
                continue
            word = tuple(reversed(s)) + tuple(t)
            C[i][j] = _trace_product(_canon((word,)))
    return C


def basis(gluon_legs: List[int]) -> List[Tuple[int, ...]]:
    return [tuple(p) for p in permutations(sorted(gluon_legs))]
