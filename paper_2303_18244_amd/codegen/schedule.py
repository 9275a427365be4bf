"""Evaluation schedule of the Feynman diagrams of one helicity configuration.

Every term of every diagram is evaluated as one vertex contraction (the
"amplitude vertex") of off-shell currents.  Currents are shared between
diagrams whenever the same sub-tree appears:
  T  gluon tree current (three/four-gluon vertices and gluon propagators);
  K  ket chain: the antiquark spinor after absorbing the blocks G_n, ..., G_m
     attached to the quark line, each followed by a quark propagator;
  B  bra chain: the quark spinor after absorbing G_1, ..., G_m;
  F  vector current of the quark line (bra gamma^mu ket) with the gluon
     propagator, used when the amplitude vertex is the root of a gluon tree.
For each term the amplitude vertex is either a quark-gluon vertex of the
line, B . G_m . K, or the root vertex of the tree G_m contracted with F.  The
choice minimises the estimated arithmetic of the currents it adds, greedily
and then by a few passes of local improvement.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

from .diagrams import Term, Tree

# Floating-point operation counts of the device routines (add/sub 1, mul 1,
# fused multiply-add 2; complex multiply 6); see helamp.h.
FLOPS = {
    "ffv_amp": 102, "ket_prop": 138, "bra_prop": 142, "ffv_vec": 128,
    "vvv_vec": 150, "vvv_amp": 166, "vvvv_vec": 120, "vvvv_amp": 134,
    "acc": 2,
}


@dataclass
class Current:
    key: tuple
    kind: str                  # "T", "K", "B", "F"
    inputs: List[tuple]
    mask: int                  # external legs whose flow-in momenta sum to this current's momentum
    routine: str
    tree: Optional[Tree] = None
    cost: int = 0


@dataclass
class Amp:
    term: Term
    routine: str               # "ffv_amp", "vvv_amp", "vvvv_amp"
    inputs: List[tuple]
    s: int = -1                # four-gluon structure
    coeffs: List[Tuple[int, int, int]] = field(default_factory=list)  # (flow, re, im)


class Schedule:
    def __init__(self, terms: List[Term], quark_leg: int, antiquark_leg: int, flows: List[tuple]):
        self.terms = terms
        self.q = quark_leg
        self.qb = antiquark_leg
        self.flow_index = {f: i for i, f in enumerate(flows)}
        self.currents: Dict[tuple, Current] = {}
        self.choice: List[tuple] = []
        self._build()

    # ------------------------------------------------------------ current defs
    def tree_key(self, t: Tree) -> tuple:
        return ("T", t.key) if t.kind != "leaf" else ("X", t.leg)

    def _define_tree(self, t: Tree) -> tuple:
        key = self.tree_key(t)
        if t.kind == "leaf" or key in self.currents:
            return key
        ins = [self._define_tree(c) for c in t.children]
        routine = "vvv_vec" if t.kind == "ggg" else "vvvv_vec"
        self.currents[key] = Current(key, "T", ins, t.mask, routine, tree=t, cost=FLOPS[routine])
        return key

    def _define_chain(self, side: str, blocks: Tuple[Tree, ...]) -> tuple:
        """side "K": blocks absorbed from the antiquark end (first element
        absorbed first); side "B": from the quark end."""
        if not blocks:
            return ("X", self.qb if side == "K" else self.q)
        key = (side, tuple(b.key for b in blocks))
        if key in self.currents:
            return key
        prev = self._define_chain(side, blocks[:-1])
        tk = self._define_tree(blocks[-1])
        mask = 1 << (self.qb if side == "K" else self.q)
        for b in blocks:
            mask |= b.mask
        routine = "ket_prop" if side == "K" else "bra_prop"
        self.currents[key] = Current(key, side, [prev, tk], mask, routine, cost=FLOPS[routine])
        return key

    def _define_F(self, bra: tuple, ket: tuple, mask: int) -> tuple:
        key = ("F", bra, ket)
        if key not in self.currents:
            self.currents[key] = Current(key, "F", [bra, ket], mask, "ffv_vec", cost=FLOPS["ffv_vec"])
        return key

    def _candidates(self, term: Term):
        n = len(term.blocks)
        full = 0
        for b in term.blocks:
            full |= b.mask
        full |= (1 << self.q) | (1 << self.qb)
        cands = []
        for m in range(n):
            bra = self._define_chain("B", term.blocks[:m])
            ket = self._define_chain("K", tuple(reversed(term.blocks[m + 1:])))
            g = self._define_tree(term.blocks[m])
            cands.append(("ffv_amp", [bra, ket, g], -1))
            t = term.blocks[m]
            if t.kind != "leaf":
                F = self._define_F(bra, ket, full & ~t.mask)
                ch = [self._define_tree(c) for c in t.children]
                if t.kind == "ggg":
                    cands.append(("vvv_amp", ch + [F], -1))
                else:
                    cands.append(("vvvv_amp", ch + [F], t.s))
        return cands

    def _closure(self, inputs, out: set) -> None:
        for k in inputs:
            if k[0] == "X" or k in out:
                continue
            out.add(k)
            self._closure(self.currents[k].inputs, out)

    # --------------------------------------------------------------- choosing
    def _build(self) -> None:
        cands = [self._candidates(t) for t in self.terms]
        closures = [[self._closure_set(c[1]) for c in cs] for cs in cands]
        refcount: Dict[tuple, int] = {}
        choice = [-1] * len(self.terms)

        def add(i, j, sign):
            for k in closures[i][j]:
                refcount[k] = refcount.get(k, 0) + sign

        def best(i):
            bj, bc = 0, None
            for j, cs in enumerate(closures[i]):
                c = FLOPS[cands[i][j][0]] + sum(self.currents[k].cost for k in cs if refcount.get(k, 0) == 0)
                if bc is None or c < bc:
                    bj, bc = j, c
            return bj

        for i in range(len(self.terms)):
            choice[i] = best(i)
            add(i, choice[i], +1)
        for _ in range(4):
            changed = False
            for i in range(len(self.terms)):
                add(i, choice[i], -1)
                j = best(i)
                if j != choice[i]:
                    changed = True
                choice[i] = j
                add(i, j, +1)
            if not changed:
                break
        used = set()
        self.amps: List[Amp] = []
        for i, t in enumerate(self.terms):
            routine, ins, s = cands[i][choice[i]]
            used |= closures[i][choice[i]]
            coeffs = []
            for flow, c in sorted(t.colour.items(), key=lambda kv: self.flow_index[kv[0]]):
                re = t.phase[0] * c[0] - t.phase[1] * c[1]
                im = t.phase[0] * c[1] + t.phase[1] * c[0]
                coeffs.append((self.flow_index[flow], re, im))
            self.amps.append(Amp(t, routine, ins, s, coeffs))
        self.currents = {k: v for k, v in self.currents.items() if k in used}

    def _closure_set(self, inputs) -> frozenset:
        out: set = set()
        self._closure(inputs, out)
        return frozenset(out)

    # --------------------------------------------------------------- ordering
    def low_pressure_order(self, amps: Optional[List[Amp]] = None) -> List[Amp]:
        """Order of the amplitude vertices (all of them, or the subset `amps`,
        whose currents are then evaluated afresh) that keeps few currents
        alive: repeatedly take the amplitude needing the fewest new currents
        net of the currents whose last use it is (greedy list scheduling)."""
        emitted: set = set()
        live: set = set()

        def closure(keys, out):
            for k in keys:
                if k[0] == "X" or k in emitted or k in out:
                    continue
                closure(self.currents[k].inputs, out)
                out.append(k)
            return out

        if amps is None:
            amps = self.amps
            keys = list(self.currents)
        else:
            keys = closure([i for a in amps for i in a.inputs], [])
        uses: Dict[tuple, int] = {k: 0 for k in keys}
        for k in keys:
            for i in self.currents[k].inputs:
                if i in uses:
                    uses[i] += 1
        for a in amps:
            for i in a.inputs:
                if i in uses:
                    uses[i] += 1

        todo = list(range(len(amps)))
        order: List[Amp] = []
        while todo:
            best = None
            for i in todo:
                new = closure(amps[i].inputs, [])
                cnt: Dict[tuple, int] = {}
                for k in new:
                    for j in self.currents[k].inputs:
                        if j in uses:
                            cnt[j] = cnt.get(j, 0) + 1
                for j in amps[i].inputs:
                    if j in uses:
                        cnt[j] = cnt.get(j, 0) + 1
                freed = sum(1 for j, c in cnt.items() if j in live and uses[j] == c)
                score = (len(new) - freed, len(new))
                if best is None or score < best[0]:
                    best = (score, i)
            i = best[1]
            todo.remove(i)
            order.append(amps[i])
            for k in closure(amps[i].inputs, []):
                emitted.add(k)
                live.add(k)
                for j in self.currents[k].inputs:
                    if j in uses:
                        uses[j] -= 1
                        if uses[j] == 0:
                            live.discard(j)
            for j in amps[i].inputs:
                if j in uses:
                    uses[j] -= 1
                    if uses[j] == 0:
                        live.discard(j)
        return order

    # ---------------------------------------------------------------- summary
    def flops_per_helicity(self) -> int:
        f = sum(c.cost for c in self.currents.values())
        for a in self.amps:
            f += FLOPS[a.routine] + FLOPS["acc"] * len(a.coeffs)
        return f
