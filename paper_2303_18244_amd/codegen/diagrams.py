"""Tree-level Feynman diagrams of g g -> t t~ + n gluons (one quark line, k
gluons in total, three- and four-gluon vertices), each with its overall phase
from the Feynman rules and its colour expansion on the trace basis.

A diagram is the ordered list of gluon trees attached along the quark line,
from the outgoing quark (the ubar end) to the outgoing antiquark (the v end).
A four-gluon vertex carries three colour/Lorentz structures; every choice of
structure at every four-gluon vertex of a diagram is one "term", so a diagram
with m four-gluon vertices has 3^m terms.  The number of diagrams for k = 2..5
gluons is 3, 16, 123 and 1240.

Phases (Peskin & Schroeder rules, couplings stripped): quark-gluon vertex i,
three-gluon vertex 1, four-gluon vertex -i, quark propagator i, gluon
propagator -i.  Every term carries gs^k, applied once per event.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache
from typing import List, Tuple

from . import colour as col


@dataclass(frozen=True)
class Tree:
    kind: str                 # "leaf", "ggg" or "gggg"
    leg: int = -1             # leaf: external leg
    children: Tuple["Tree", ...] = ()
    s: int = -1               # gggg: colour/Lorentz structure 0..2
    mask: int = 0

    @property
    def key(self) -> str:
        if self.kind == "leaf":
            return f"g{self.leg}"
        inner = ",".join(c.key for c in self.children)
        if self.kind == "ggg":
            return f"V({inner})"
        return f"Q{self.s}({inner})"

    def colour(self):
        if self.kind == "leaf":
            return col.leaf(self.leg)
        cs = [c.colour() for c in self.children]
        if self.kind == "ggg":
            return col.three_gluon(cs[0], cs[1])
        return col.four_gluon(cs[0], cs[1], cs[2], self.s)

    def phase_power(self) -> int:
        """Power of i contributed by the vertices and internal propagators of
        this tree, including the propagator above its root when it is not a leaf."""
        if self.kind == "leaf":
            return 0
        p = sum(c.phase_power() for c in self.children)
        if self.kind == "gggg":
            p += 3  # vertex -i
        p += 3      # gluon propagator -i
        return p


@dataclass
class Term:
    blocks: Tuple[Tree, ...]   # quark (ubar) end first
    diagram: int
    phase: Tuple[int, int] = (1, 0)                   # i^p as Gaussian integer
    colour: dict = field(default_factory=dict)        # ordering -> Gaussian integer


def _subsets(mask: int):
    s = mask
    while True:
        yield s
        if s == 0:
            return
        s = (s - 1) & mask


@lru_cache(maxsize=None)
def gluon_trees(mask: int) -> Tuple[Tuple[Tree, ...], ...]:
    """All gluon trees joining the legs in `mask`, grouped by diagram: each
    entry is the tuple of terms (structure choices) of one tree topology."""
    if bin(mask).count("1") == 1:
        leg = mask.bit_length() - 1
        return ((Tree("leaf", leg=leg, mask=mask),),)
    low = mask & -mask
    rest = mask ^ low
    out = []
    for s in _subsets(rest):
        A = low | s
        B = mask ^ A
        if B == 0:
            continue
        for ta in gluon_trees(A):
            for tb in gluon_trees(B):
                out.append(tuple(Tree("ggg", children=(x, y), mask=mask) for x in ta for y in tb))
    for s in _subsets(rest):
        A = low | s
        R = mask ^ A
        if R == 0:
            continue
        low2 = R & -R
        for s2 in _subsets(R ^ low2):
            B = low2 | s2
            Cm = R ^ B
            if Cm == 0:
                continue
            for ta in gluon_trees(A):
                for tb in gluon_trees(B):
                    for tc in gluon_trees(Cm):
                        terms = tuple(Tree("gggg", children=(x, y, z), s=st, mask=mask)
                                      for x in ta for y in tb for z in tc for st in range(3))
                        out.append(terms)
    return tuple(out)


def _ordered_partitions(mask: int):
    if mask == 0:
        yield ()
        return
    s = mask
    while s:
        for rest in _ordered_partitions(mask ^ s):
            yield (s,) + rest
        s = (s - 1) & mask


def ipow(p: int) -> Tuple[int, int]:
    return [(1, 0), (0, 1), (-1, 0), (0, -1)][p % 4]


def enumerate_terms(gluon_legs: List[int]) -> Tuple[List[Term], int]:
    """All terms of all diagrams; returns (terms, number of diagrams)."""
    full = 0
    for leg in gluon_legs:
        full |= 1 << leg
    terms: List[Term] = []
    nd = 0
    for part in _ordered_partitions(full):
        choices = [gluon_trees(b) for b in part]
        # cartesian product over topologies per block
        def rec(i, acc):
            nonlocal nd
            if i == len(part):
                # expand structure choices: cartesian product over the terms
                def rec2(j, blocks):
                    if j == len(acc):
                        terms.append(Term(tuple(blocks), nd))
                        return
                    for t in acc[j]:
                        rec2(j + 1, blocks + [t])
                rec2(0, [])
                nd += 1
                return
            for topo in choices[i]:
                rec(i + 1, acc + [topo])
        rec(0, [])
    for t in terms:
        n = len(t.blocks)
        p = n * 1 + (n - 1) * 1 + sum(b.phase_power() for b in t.blocks)  # qqg vertices i, quark props i
        t.phase = ipow(p)
        t.colour = col.quark_line([b.colour() for b in t.blocks])
    return terms, nd
