"""HIP source emission for one process: a kernel with one lane per event that
loops over the good helicities in lockstep, evaluates the scheduled currents
and amplitudes in straight-line code, accumulates the colour-flow amplitudes
J and adds the colour quadratic form Re(J^dagger C J) in double precision.
"""
from __future__ import annotations

from fractions import Fraction
from math import lcm
from typing import Dict, List, Optional, Tuple

from . import colour as col
from .diagrams import enumerate_terms
from .schedule import FLOPS, Schedule


class Emitter:
    def __init__(self, n_ext: int, incoming: List[bool], massive: List[bool]):
        self.n_ext = n_ext
        self.incoming = incoming
        self.massive = massive
        self.lines: List[str] = []
        self.mom: Dict[int, str] = {}
        self.den: Dict[tuple, str] = {}

    def w(self, s: str) -> None:
        self.lines.append("    " + s)

    def momentum(self, mask: int) -> str:
        """Flow-in momentum of a set of legs, as a T[4] array."""
        if mask in self.mom:
            return self.mom[mask]
        name = f"P{mask}"
        terms = []
        for i in range(self.n_ext):
            if mask >> i & 1:
                terms.append(("+" if self.incoming[i] else "-") + f"q[{i}][MU]")
        exprs = []
        for mu in range(4):
            e = " ".join(t.replace("MU", str(mu)) for t in terms)
            if e.startswith("+"):
                e = e[1:]
            exprs.append(e)
        self.w(f"const double {name}d[4] = {{{', '.join(exprs)}}};")
        self.w(f"const T {name}[4] = {{(T){name}d[0], (T){name}d[1], (T){name}d[2], (T){name}d[3]}};")
        self.mom[mask] = name
        return name

    def denominator(self, mask: int, mass: str) -> str:
        """1 / (P^2 - m^2) in double, converted to T."""
        key = (mask, mass)
        if key in self.den:
            return self.den[key]
        p = self.momentum(mask)
        name = f"d{'t' if mass != '0' else 'g'}{mask}"
        m2 = "" if mass == "0" else f" - {mass} * {mass}"
        self.w(f"const T {name} = (T)(1.0 / ({p}d[0] * {p}d[0] - {p}d[1] * {p}d[1] - {p}d[2] * {p}d[2]"
               f" - {p}d[3] * {p}d[3]{m2}));")
        self.den[key] = name
        return name


def colour_sum_lines(C: List[List[Fraction]], den: int) -> List[str]:
    """Lines computing mc += Re(J^dagger C J) * den (integer numerators) in
    the colour precision TC of the kernel."""
    n = len(C)
    out = []
    for s in range(n):
        parts_r = [f"(TC){float(C[s][s] * den)!r} * (TC)J[{s}].re"]
        parts_i = [f"(TC){float(C[s][s] * den)!r} * (TC)J[{s}].im"]
        for t in range(s + 1, n):
            v = C[s][t] * den * 2
            if v == 0:
                continue
            parts_r.append(f"(TC){float(v)!r} * (TC)J[{t}].re")
            parts_i.append(f"(TC){float(v)!r} * (TC)J[{t}].im")
        out.append(f"mc += (TC)J[{s}].re * ({' + '.join(parts_r)}) + "
                   f"(TC)J[{s}].im * ({' + '.join(parts_i)});")
    return out


class GGBody:
    """Straight-line evaluation of a list of amplitude vertices of one
    helicity configuration: external wavefunctions, the currents each
    amplitude needs (computed at first use), and the amplitude values."""

    def __init__(self, sched: Schedule, pdg: List[int], em: Emitter, fresh_externals: bool = True,
                 lds_momenta: bool = False, inplace: bool = None, mom_block: str = "MGME_ME_BLOCK",
                 ext_lds: bool = False, prefetch: bool = False):
        """lds_momenta: the momenta are read from the lane's LDS rows (fused
        kernels) instead of the register array q (one lane per event and
        helicity in the staged kernels).

        prefetch: software-pipelines the momenta and propagator denominators.
        Without it a call's LDS loads can only start after its own register
        barriers, i.e. once the previous call has finished, and with one wave
        per SIMD nothing hides their latency.  With it, the loads of each
        routine call are issued pf_dist calls earlier, right after that
        call's barriers and ahead of a scheduling barrier (FP64 only) that
        keeps the compiler from sinking them to their use; the momentum sums
        and 1/(P^2 - m^2) follow in the block of the call just before, where
        they overlap its arithmetic.  Call finish() once the body is
        complete."""
        self.sched = sched
        self.em = em
        self.lds = lds_momenta
        self.inplace = lds_momenta if inplace is None else inplace
        self.mom_block = mom_block
        self.ext_lds = ext_lds
        self.gluon = [x == 21 for x in pdg]
        self.nload = 0
        n_ext = len(pdg)
        incoming = [i < 2 for i in range(n_ext)]
        q_leg = pdg.index(6)
        self.names: Dict[tuple, str] = {}
        self.fresh_fn: Dict[str, str] = {}
        for i in range(n_ext):
            lam = f"((hc >> {n_ext - 1 - i}) & 1 ? 1 : -1)"
            if self.lds:
                em.w(f"double q{i}[4]; load_mom_lds<{mom_block}>(q{i}, smom, lane, {i});")
                qi = f"q{i}"
            else:
                qi = f"q[{i}]"
            if pdg[i] == 21:
                ext = f"ext_vec<T>({qi}, {lam}, {'false' if incoming[i] else 'true'})"
                self.fresh_fn[f"x{i}"] = "fresh_pol"
            elif i == q_leg:
                ext = f"ext_bra<T>({qi}, mt, {lam}, false)"
            else:
                ext = f"ext_ket<T>({qi}, mt, {lam}, true)"
            if self.ext_lds:
                em.w(f"store_wf_lds<T, 256>(sext, {i}, xl, {ext});")
            else:
                em.w(f"{'' if self.lds else 'const '}wf<T> x{i} = {ext};")
            self.names[("X", i)] = f"x{i}"
            if not fresh_externals:
                self.fresh_fn[f"x{i}"] = ""
        self.inmask = sum(1 << i for i in range(n_ext) if incoming[i])
        self.counter = 0
        self.prefetch = prefetch
        self.pf_dist = 1
        # den_index: denominator key -> row of the per-event table `sden`
        # (distance-2 pipelining only); the denominators are then loaded
        # instead of recomputed for every helicity
        self.den_index: Optional[Dict[tuple, int]] = None
        # kin_index: momentum mask -> row of the per-event table `skin` (T[4]
        # sums, shared by the lanes of one event); with it the denominators
        # come from a T table `sden` too, and a call's values are loaded two
        # calls ahead straight into its own registers (no sums in the loop)
        self.kin_index: Optional[Dict[int, int]] = None
        self.kin_split = False  # one load per component (load_kin_lds1)
        # kin_lazy (kernels without prefetching): every momentum sum and
        # denominator is loaded from the event's rows where it is used, rows
        # assigned in order of first use
        self.kin_lazy = False
        self.kin_rows: Dict[int, int] = {}
        self.den_rows: Dict[tuple, int] = {}
        self.calls: List[Optional[tuple]] = []  # per routine call: its momentum needs
        if prefetch:
            em.w("@@PFHEAD@@")

    def open_call(self, needs: Optional[tuple]) -> Tuple[int, str]:
        """Registers a routine call with its momentum needs; returns its index
        and the marker that finish() replaces with the prefetch of the next
        call (empty without prefetching)."""
        i = len(self.calls)
        self.calls.append(needs)
        if not self.prefetch:
            return i, ""
        self.em.w(f"@@PFDECL{i}@@")
        return i, f"@@PF{i}@@"

    def pf_decl(self, j: int) -> str:
        if self.kin_index is not None and self.pf_dist >= 2:
            return ""  # declared with the loads, pf_dist calls ahead
        return self._vec_decl(j)

    def _vec_decl(self, j: int) -> str:
        needs = self.calls[j] if j < len(self.calls) else None
        if needs is None:
            return ""
        kind = needs[0]
        vecs = {"vvv": ["k1", "k2"], "prop": ["P"], "den": [], "amp3": ["k1", "k2", "k3"]}[kind]
        parts = [f"T pf{j}_{v}[4];" for v in vecs]
        if kind != "amp3":
            parts.append(f"T pf{j}_den;")
        return " ".join(parts)

    def pf_code(self, j: int) -> str:
        needs = self.calls[j] if j < len(self.calls) else None
        if needs is not None and self.kin_index is not None:
            return self.kin_loads(j)
        return "" if needs is None else self.pf_code_split(j, needs)

    def _union(self, j: int) -> int:
        needs = self.calls[j] if j < len(self.calls) else None
        u = 0
        if needs is not None:
            for m in needs[1:]:
                if isinstance(m, int):
                    u |= m
        return u

    @staticmethod
    def den_key(needs: Optional[tuple]) -> Optional[tuple]:
        """The quantity a call's denominator is computed from: the legs of
        the propagator momentum (as two partial sums for a three-gluon
        vertex) and the mass; None if the call has no propagator."""
        if needs is None or needs[0] == "amp3":
            return None
        if needs[0] == "vvv":
            return ("vvv", needs[1], needs[2], "0.0")
        if needs[0] == "prop":
            return ("sum", needs[1], needs[2])
        return ("sum", needs[1], "0.0")

    def _legs(self, j: int) -> int:
        """Legs whose momenta call j needs in registers."""
        needs = self.calls[j] if j < len(self.calls) else None
        if needs is not None and needs[0] == "den" and self.den_index is not None:
            return 0
        return self._union(j)

    def kin_loads(self, j: int) -> str:
        """Distance 2 with the kinematics table: call j's momentum sums and
        denominator loaded from the event's rows."""
        needs = self.calls[j] if j < len(self.calls) else None
        if needs is None:
            return ""
        kind, masks = needs[0], [m for m in needs[1:] if isinstance(m, int)]
        names = {"vvv": ["k1", "k2"], "prop": ["P"], "den": [], "amp3": ["k1", "k2", "k3"]}[kind]
        fn = "load_kin_lds1" if self.kin_split else "load_kin_lds"
        out = "".join(f"{fn}<T, {self.mom_block}>(pf{j}_{v}, skin, {self.kin_index[m]}, lane); "
                      for v, m in zip(names, masks))
        k = self.den_key(needs)
        if k is not None:
            out += f"pf{j}_den = load_tden_lds<T, {self.mom_block}>(sden, {self.den_index[k]}, lane); "
        return out + "pf_barrier<T>(); "

    def pf_loads(self, j: int) -> str:
        """Distance 2: the LDS loads of call j into its raw registers."""
        if self.kin_index is not None:
            return self.kin_loads(j)
        u = self._legs(j)
        out = ""
        if u:
            out += f"load_legs_lds<{u}u, NEXT, {self.mom_block}>(pf{j}_r, smom, lane); "
        k = self.den_key(self.calls[j] if j < len(self.calls) else None)
        if self.den_index is not None and k is not None:
            out += f"pf{j}_dr = load_den_lds<{self.mom_block}>(sden, {self.den_index[k]}, lane); "
        return out + "pf_barrier<T>(); " if out else ""

    def pf_raw_decl(self, j: int) -> str:
        """Declarations of the raw registers that call j's loads fill."""
        if self.kin_index is not None:
            return self._vec_decl(j)
        parts = []
        if self._legs(j):
            parts.append(f"double pf{j}_r[NEXT][4];")
        if self.den_index is not None and self.den_key(self.calls[j] if j < len(self.calls) else None):
            parts.append(f"double pf{j}_dr;")
        return " ".join(parts)

    def pf_sums(self, j: int) -> str:
        """Distance 2: sums and denominator of call j from its raw registers."""
        needs = self.calls[j] if j < len(self.calls) else None
        if needs is None or self.kin_index is not None:
            return ""
        return "{ " + self.pf_arith(j, needs, f"pf{j}_r")

    def pf_code_split(self, j: int, needs: tuple) -> str:
        """Distance 1: prefetch whose LDS loads sit above a scheduling barrier
        (so the scheduler cannot sink them to their use) and whose arithmetic
        sits below it."""
        head = (f"{{ double r[NEXT][4]; load_legs_lds<{self._union(j)}u, NEXT, {self.mom_block}>(r, smom, lane); "
                "pf_barrier<T>(); ")
        return head + self.pf_arith(j, needs, "r")

    def pf_arith(self, j: int, needs: tuple, r: str) -> str:
        """Momentum sums and denominator of call j from the raw leg momenta in
        register array `r`; closes the block the caller opened."""
        kind, masks = needs[0], [m for m in needs[1:] if isinstance(m, int)]
        I = self.inmask
        table = self.den_index is not None
        if kind == "vvv":
            m1, m2 = masks
            den = (f"pf{j}_den = (T)pf{j}_dr; }} " if table else
                   "const double Pd[4] = {k1d[0] + k2d[0], k1d[1] + k2d[1], k1d[2] + k2d[2], k1d[3] + k2d[3]}; "
                   f"pf{j}_den = (T)inv_virt(Pd, 0.0); }} ")
            body = (f"double k1d[4]; sum_legs<{m1}u, {I}u, NEXT>(k1d, {r}); double k2d[4]; sum_legs<{m2}u, {I}u, NEXT>(k2d, {r}); "
                    f"to_t(pf{j}_k1, k1d); to_t(pf{j}_k2, k2d); " + den)
        elif kind == "prop":
            den = f"pf{j}_den = (T)pf{j}_dr; }} " if table else f"pf{j}_den = (T)inv_virt(Pd, {needs[2]}); }} "
            body = f"double Pd[4]; sum_legs<{masks[0]}u, {I}u, NEXT>(Pd, {r}); to_t(pf{j}_P, Pd); " + den
        elif kind == "den":
            body = (f"pf{j}_den = (T)pf{j}_dr; }} " if table else
                    f"double Pd[4]; sum_legs<{masks[0]}u, {I}u, NEXT>(Pd, {r}); pf{j}_den = (T)inv_virt(Pd, 0.0); }} ")
        else:
            body = " ".join(f"{{ double kd[4]; sum_legs<{m}u, {I}u, NEXT>(kd, {r}); to_t(pf{j}_{k}, kd); }}"
                            for k, m in zip(("k1", "k2", "k3"), masks)) + " } "
        return body

    def finish(self) -> None:
        """Fills the prefetch markers: block i issues the loads of call i+1;
        the first call's are issued before any block."""
        if not self.prefetch:
            return
        n = len(self.calls)
        out = []
        if self.kin_index is not None and self.pf_dist >= 2:
            # loads of finished values only: call i's block issues those of
            # call i + pf_dist into registers declared just before the block
            d = self.pf_dist
            for ln in self.em.lines:
                t = ln.strip()
                if t == "@@PFHEAD@@":
                    decl = " ".join(x for x in (self.pf_raw_decl(j) for j in range(d)) if x)
                    out.append("    " + decl + " " + "".join(self.pf_loads(j) for j in range(d)))
                    continue
                if t.startswith("@@PFDECL"):
                    i = int(t[len("@@PFDECL"):-2])
                    x = self.pf_raw_decl(i + d)
                    if x:
                        out.append("    " + x)
                    continue
                if "@@PF" in ln:
                    i = int(ln.split("@@PF", 1)[1].split("@@", 1)[0])
                    ln = ln.replace(f"@@PF{i}@@", self.pf_loads(i + d))
                out.append(ln)
            self.em.lines = out
            return
        if self.pf_dist == 2:
            for ln in self.em.lines:
                t = ln.strip()
                if t == "@@PFHEAD@@":
                    decl = [self.pf_raw_decl(j) for j in (0, 1)]
                    decl += [self.pf_decl(0)]
                    out.append("    " + " ".join(d for d in decl if d) + " " + self.pf_loads(0) + self.pf_loads(1)
                               + self.pf_sums(0).rstrip())
                    continue
                if t.startswith("@@PFDECL"):
                    i = int(t[len("@@PFDECL"):-2])
                    d = " ".join(x for x in (self.pf_decl(i + 1), self.pf_raw_decl(i + 2)) if x)
                    if d:
                        out.append("    " + d)
                    continue
                if "@@PF" in ln:
                    i = int(ln.split("@@PF", 1)[1].split("@@", 1)[0])
                    ln = ln.replace(f"@@PF{i}@@", self.pf_loads(i + 2) + self.pf_sums(i + 1))
                out.append(ln)
            self.em.lines = out
            return
        ahead = self.pf_dist  # 1, or 0: each call loads its own values at its start
        for ln in self.em.lines:
            t = ln.strip()
            if t == "@@PFHEAD@@":
                d = self.pf_decl(0) if ahead else ""
                if d:
                    out.append("    " + d + " " + self.pf_code(0).rstrip())
                continue
            if t.startswith("@@PFDECL"):
                i = int(t[len("@@PFDECL"):-2])
                d = self.pf_decl(i + ahead)
                if d:
                    out.append("    " + d)
                continue
            if "@@PF" in ln:
                i = int(ln.split("@@PF", 1)[1].split("@@", 1)[0])
                ln = ln.replace(f"@@PF{i}@@", self.pf_code(i + ahead) if i + ahead < n else "")
            out.append(ln)
        self.em.lines = out

    def kin_vec(self, var: str, mask: int) -> str:
        """Declaration and load of the momentum sum of `mask` as T[4] from
        the event's rows (lazy form)."""
        r = self.kin_rows.setdefault(mask, len(self.kin_rows))
        return f"T {var}[4]; load_kin_lds<T, {self.mom_block}>({var}, skin, {r}, lane);"

    def kin_den(self, key: tuple) -> str:
        """Load of a propagator denominator from the event's rows (lazy form)."""
        r = self.den_rows.setdefault(key, len(self.den_rows))
        return f"load_tden_lds<T, {self.mom_block}>(sden, {r}, lane)"

    def emit_current_kin(self, cur, ins, v, pre) -> None:
        """A current whose momentum sums and denominator come from the rows."""
        em, fr = self.em, self.fr
        r = cur.routine
        if r == "vvv_vec":
            c1, c2 = cur.tree.children
            em.w(f"{{ {pre}{self.kin_vec('k1', c1.mask)} {self.kin_vec('k2', c2.mask)}")
            em.w(f"  {v} = vvv_vec<T>({fr(ins[0])}, k1, {fr(ins[1])}, k2, "
                 f"{self.kin_den(('vvv', c1.mask, c2.mask, '0.0'))}); }}")
        elif r == "vvvv_vec":
            em.w(f"{{ {pre}{v} = vvvv_vec<T, {cur.tree.s}>({fr(ins[0])}, {fr(ins[1])}, {fr(ins[2])}, "
                 f"{self.kin_den(('sum', cur.mask, '0.0'))}); }}")
        elif r in ("ket_prop", "bra_prop"):
            em.w(f"{{ {pre}{self.kin_vec('P', cur.mask)}")
            em.w(f"  {v} = {r}<T>({fr(ins[0])}, {fr(ins[1])}, P, (T)mt, {self.kin_den(('sum', cur.mask, 'mt'))}); }}")
        elif r == "ffv_vec":
            em.w(f"{{ {pre}{v} = ffv_vec<T>({fr(ins[0])}, {fr(ins[1])}, {self.kin_den(('sum', cur.mask, '0.0'))}); }}")
        else:
            raise ValueError(r)

    def fr(self, v: str) -> str:
        fn = self.fresh_fn.get(v, "fresh")
        if self.inplace:
            return v  # laundered in place by prep()
        return f"{fn}({v})" if fn else v

    def prep(self, names) -> str:
        """Statements giving the inputs of the next routine call new
        identities in place (fused kernels); empty otherwise.  With the
        external wavefunctions in LDS, also their loads (see use())."""
        out = []
        for v in dict.fromkeys(names):
            if v.startswith("u"):
                continue
            if not self.inplace:
                continue
            fn = self.fresh_fn.get(v, "fresh")
            if fn == "fresh":
                out.append(f"launder({v});")
            elif fn == "fresh_pol":
                out.append(f"launder_pol({v});")
        return " ".join(out) + (" " if out else "")

    def fm(self, out: str, mask: int) -> str:
        """Statement computing the flow-in momentum of the legs in `mask`."""
        if self.lds:
            return f"flow_momentum_lds<{mask}u, {self.inmask}u, NEXT, {self.mom_block}>({out}, smom, lane);"
        return f"flow_momentum<{mask}u, {self.inmask}u, NEXT>({out}, q);"

    def mom(self, var: str, mask: int) -> str:
        return f"double {var}d[4]; {self.fm(var + 'd', mask)} T {var}[4]; to_t({var}, {var}d);"

    def leg_mask(self, k) -> int:
        return self.sched.currents[k].mask if k[0] != "X" else 1 << k[1]

    def need(self, key) -> str:
        if key[0] == "X" and self.ext_lds:
            # a fresh load of the external wavefunction for this use
            i = key[1]
            v = f"u{self.nload}"
            self.nload += 1
            fn = "load_pol_lds" if self.gluon[i] else "load_wf_lds"
            self.em.w(f"const wf<T> {v} = {fn}<T, 256>(sext, {i}, xl);")
            return v
        if key in self.names:
            return self.names[key]
        em, fr, mom = self.em, self.fr, self.mom
        cur = self.sched.currents[key]
        ins = [self.need(k) for k in cur.inputs]
        v = f"w{self.counter}"
        self.counter += 1
        em.w(f"wf<T> {v};")
        pre = self.prep(ins)
        if self.prefetch:
            self.emit_current_pf(cur, ins, v, pre)
            self.names[key] = v
            return v
        if self.kin_lazy:
            self.emit_current_kin(cur, ins, v, pre)
            self.names[key] = v
            return v
        if cur.routine == "vvv_vec":
            c1, c2 = cur.tree.children
            em.w(f"{{ {pre}{mom('k1', c1.mask)} {mom('k2', c2.mask)}")
            em.w("  const double Pd[4] = {k1d[0] + k2d[0], k1d[1] + k2d[1], k1d[2] + k2d[2], k1d[3] + k2d[3]};")
            em.w(f"  {v} = vvv_vec<T>({fr(ins[0])}, k1, {fr(ins[1])}, k2, (T)inv_virt(Pd, 0.0)); }}")
        elif cur.routine == "vvvv_vec":
            em.w(f"{{ {pre}double Pd[4]; {self.fm('Pd', cur.mask)}")
            em.w(f"  {v} = vvvv_vec<T, {cur.tree.s}>({fr(ins[0])}, {fr(ins[1])}, {fr(ins[2])}, "
                 f"(T)inv_virt(Pd, 0.0)); }}")
        elif cur.routine in ("ket_prop", "bra_prop"):
            em.w(f"{{ {pre}{mom('P', cur.mask)}")
            em.w(f"  {v} = {cur.routine}<T>({fr(ins[0])}, {fr(ins[1])}, P, (T)mt, (T)inv_virt(Pd, mt)); }}")
        elif cur.routine == "ffv_vec":
            em.w(f"{{ {pre}double Pd[4]; {self.fm('Pd', cur.mask)}")
            em.w(f"  {v} = ffv_vec<T>({fr(ins[0])}, {fr(ins[1])}, (T)inv_virt(Pd, 0.0)); }}")
        else:
            raise ValueError(cur.routine)
        self.names[key] = v
        return v

    def emit_current_pf(self, cur, ins, v, pre) -> None:
        """A current whose momenta and denominator were prefetched."""
        em, fr = self.em, self.fr
        r = cur.routine
        if r == "vvv_vec":
            c1, c2 = cur.tree.children
            j, pf = self.open_call(("vvv", c1.mask, c2.mask))
            em.w(f"{{ {pre}{pf}")
            em.w(f"  {v} = vvv_vec<T>({fr(ins[0])}, pf{j}_k1, {fr(ins[1])}, pf{j}_k2, pf{j}_den); }}")
        elif r == "vvvv_vec":
            j, pf = self.open_call(("den", cur.mask))
            em.w(f"{{ {pre}{pf}")
            em.w(f"  {v} = vvvv_vec<T, {cur.tree.s}>({fr(ins[0])}, {fr(ins[1])}, {fr(ins[2])}, pf{j}_den); }}")
        elif r in ("ket_prop", "bra_prop"):
            j, pf = self.open_call(("prop", cur.mask, "mt"))
            em.w(f"{{ {pre}{pf}")
            em.w(f"  {v} = {r}<T>({fr(ins[0])}, {fr(ins[1])}, pf{j}_P, (T)mt, pf{j}_den); }}")
        elif r == "ffv_vec":
            j, pf = self.open_call(("den", cur.mask))
            em.w(f"{{ {pre}{pf}")
            em.w(f"  {v} = ffv_vec<T>({fr(ins[0])}, {fr(ins[1])}, pf{j}_den); }}")
        else:
            raise ValueError(r)

    def amplitude(self, a) -> None:
        """Opens a block defining `a`, the amplitude value; the caller closes it."""
        em, fr = self.em, self.fr
        ins = [self.need(k) for k in a.inputs]
        pre = self.prep(ins)
        if self.prefetch:
            if a.routine == "vvv_amp":
                m1, m2, m3 = (self.leg_mask(k) for k in a.inputs)
                j, pf = self.open_call(("amp3", m1, m2, m3))
                em.w(f"{{ {pre}{pf}")
                em.w(f"  const cx<T> a = vvv_amp<T>({fr(ins[0])}, pf{j}_k1, {fr(ins[1])}, pf{j}_k2, "
                     f"{fr(ins[2])}, pf{j}_k3);")
                return
            _, pf = self.open_call(None)
            pre = pre + pf
        if a.routine == "ffv_amp":
            em.w(f"{{ {pre}const cx<T> a = ffv_amp<T>({fr(ins[0])}, {fr(ins[1])}, {fr(ins[2])});")
        elif a.routine == "vvv_amp":
            m1, m2, m3 = (self.leg_mask(k) for k in a.inputs)
            vec = self.kin_vec if self.kin_lazy else self.mom
            em.w(f"{{ {pre}{vec('k1', m1)} {vec('k2', m2)} {vec('k3', m3)}")
            em.w(f"  const cx<T> a = vvv_amp<T>({fr(ins[0])}, k1, {fr(ins[1])}, k2, {fr(ins[2])}, k3);")
        else:
            em.w(f"{{ {pre}const cx<T> a = vvvv_amp<T, {a.s}>({fr(ins[0])}, {fr(ins[1])}, {fr(ins[2])}, "
                 f"{fr(ins[3])});")


def _gg_setup(pdg: List[int]):
    n_ext = len(pdg)
    gluon_legs = [i for i, x in enumerate(pdg) if x == 21]
    terms, n_diag = enumerate_terms(gluon_legs)
    flows = col.basis(gluon_legs)
    C = col.colour_matrix(flows)
    cden = 1
    for row in C:
        for v in row:
            cden = lcm(cden, v.denominator)
    sched = Schedule(terms, pdg.index(6), pdg.index(-6), flows)
    return n_ext, gluon_legs, terms, n_diag, flows, C, cden, sched


def _gg_meta(name, pdg, n_ext, gluon_legs, terms, n_diag, ncol, cden, sched, flops_hel, body, **extra):
    incoming = [i < 2 for i in range(n_ext)]
    n_final_g = len([i for i in gluon_legs if not incoming[i]])
    meta = dict(name=name, pdg=pdg, n_ext=n_ext, n_diagrams=n_diag, n_terms=len(terms), ncol=ncol,
                cden=cden, n_currents=len(sched.currents), n_amps=len(sched.amps), gs_power=2 * len(gluon_legs),
                spin_colour_avg=4 * 64, ident=_fact(n_final_g), kind="qcd",
                flops_per_hel=flops_hel, flops_per_event=8 * 2 ** n_ext, body=body)
    meta.update(extra)
    return meta


def emit_gg_process(name: str, pdg: List[int], fp64_dist: int = 2) -> Dict:
    """g g -> t t~ + n g, fused: the colour-flow amplitudes J stay in
    registers and the colour sum runs in the same kernel.  Eight lanes share
    an event (each takes every eighth good helicity) and its kinematics.
    fp64_dist: calls ahead at which the FP64 form loads a call's values
    (g g -> t t~ g g, 524288 events: 27.75 ms at 2, 27.97 at 3, 27.88 at 4)."""
    n_ext, gluon_legs, terms, n_diag, flows, C, cden, sched = _gg_setup(pdg)
    ncol = len(flows)
    order = sched.low_pressure_order()

    # The lanes of one event share its kinematics: a probe pass over the body
    # lists every momentum sum and propagator denominator a routine call
    # needs; the kernel forms them once per event into LDS rows, and the
    # helicity body loads each call's values two calls ahead.
    probe = Emitter(n_ext, [i < 2 for i in range(n_ext)], [abs(x) == 6 for x in pdg])
    pb = GGBody(sched, pdg, probe, lds_momenta=True, prefetch=True)
    for a in order:
        pb.amplitude(a)
        probe.w(" }")
    keys = list(dict.fromkeys(k for k in map(GGBody.den_key, pb.calls) if k is not None))
    den_index = {k: i for i, k in enumerate(keys)}
    masks = list(dict.fromkeys(m for c in pb.calls if c is not None for m in c[1:] if isinstance(m, int)
                               if c[0] != "den"))
    kin_index = {m: i for i, m in enumerate(masks)}

    def helicity_body(split: bool, dist: int = 2) -> List[str]:
        em = Emitter(n_ext, [i < 2 for i in range(n_ext)], [abs(x) == 6 for x in pdg])
        body = GGBody(sched, pdg, em, lds_momenta=True, prefetch=True, mom_block="EVB")
        body.pf_dist = dist
        body.den_index = den_index
        body.kin_index = kin_index
        body.kin_split = split
        for a in order:
            body.amplitude(a)
            upd = " ".join(f"acc(J[{f}], a, {re}, {im});" for f, re, im in a.coeffs)
            em.w(f"  {upd} }}")
        body.finish()
        return ["  " + ln for ln in em.lines]

    # Each call's values are loaded from the event's rows two calls ahead.
    # The matrix-core mode, held to 256 registers for two waves per SIMD,
    # loads the four components of a sum one by one: with 16-byte loads the
    # compiler's allocation of that mode spills about 4 KB per lane (g g ->
    # t t~ g g), with 4-byte loads nothing.  Both forms give the same bits.
    lines = [f"    cx<T> J[{ncol}];", f"    for (int s = 0; s < {ncol}; ++s) J[s] = mk<T>((T)0, (T)0);"]
    if fp64_dist != 2:
        lines += ["    if constexpr (MODE != 4 && sizeof(T) == 8) {"] + helicity_body(False, fp64_dist) + ["    } else"]
    lines += (["    if constexpr (MODE != 4) {"] + helicity_body(False) + ["    } else {"] + helicity_body(True)
              + ["    }"])
    colour = (["      TC mc = (TC)0;"] + ["  " + ln for ln in colour_sum_lines(C, cden)]
              + ["      const double me = (double)mc;"])
    flops_hel = sched.flops_per_helicity() + 2 * ncol * ncol + 4 * ncol + 90 * n_ext
    return _gg_meta(name, pdg, n_ext, gluon_legs, terms, n_diag, ncol, cden, sched, flops_hel, "\n".join(lines),
                    colour="\n".join(colour), kin_prologue=kin_table_lines(masks, keys, pb.inmask),
                    n_kin=len(masks), n_den=len(keys), hel_lanes=8)


def kin_table_lines(masks: List[int], keys: List[tuple], inmask: int) -> str:
    """Kernel prologue filling the event's kinematics rows: skin row r with
    the flow-in momentum of the legs in masks[r] (as T), sden row k with
    1/(P^2 - m^2) of denominator keys[k] (computed in double, then taken to
    T).  Each value is formed exactly as the helicity loop formed it before
    (same partial sums, same order), so the rows hold the same bits; every
    lane of the event computes them, its first lane stores them."""
    B = "EVB"
    out = ["  // The event's momentum sums and propagator denominators, the same for",
           "  // every helicity: formed once here, loaded in the helicity loop.",
           f"  __shared__ T skin[{max(len(masks), 1)} * 4 * {B}];",
           f"  __shared__ T sden[{max(len(keys), 1)} * {B}];"]
    for r, m in enumerate(masks):
        out.append(f"  {{ double kd[4]; flow_momentum_lds<{m}u, {inmask}u, NEXT, {B}>(kd, smom, lane);")
        out.append(f"    if (sub == 0) {{ T* p = skin + ({r} * {B} + lane) * 4; "
                   "p[0] = (T)kd[0]; p[1] = (T)kd[1]; p[2] = (T)kd[2]; p[3] = (T)kd[3]; } }")
    for i, k in enumerate(keys):
        if k[0] == "vvv":
            _, m1, m2, mass = k
            out.append(f"  {{ double k1d[4]; flow_momentum_lds<{m1}u, {inmask}u, NEXT, {B}>(k1d, smom, lane); "
                       f"double k2d[4]; flow_momentum_lds<{m2}u, {inmask}u, NEXT, {B}>(k2d, smom, lane);")
            out.append("    const double Pd[4] = {k1d[0] + k2d[0], k1d[1] + k2d[1], k1d[2] + k2d[2], k1d[3] + k2d[3]};")
            out.append(f"    if (sub == 0) sden[{i} * {B} + lane] = (T)inv_virt(Pd, {mass}); }}")
        else:
            _, m, mass = k
            out.append(f"  {{ double Pd[4]; flow_momentum_lds<{m}u, {inmask}u, NEXT, {B}>(Pd, smom, lane); "
                       f"if (sub == 0) sden[{i} * {B} + lane] = (T)inv_virt(Pd, {mass}); }}")
    return "\n".join(out)


def emit_gg_staged(name: str, pdg: List[int], n_chunks: int, budget: int, prefetch: int = 3,
                   inplace: bool = False, lds: bool = False, kin: bool = True) -> Dict:
    """g g -> t t~ + n g, staged for processes whose colour-flow vector does
    not fit in registers.  The amplitude vertices, in low-register-pressure
    order, are split into `n_chunks` kernels.  Each kernel keeps at most
    `budget` flow accumulators in registers and folds an accumulator into the
    flow vector J in device memory when its flow gets no further contribution
    in the chunk, or when it is the open flow used furthest in the future:
      - the first write of a flow (in kernel order) is a plain store;
      - a flow written by an earlier kernel is read, added and stored, the
        read issued `prefetch` folds ahead so that it is in flight while the
        kernel keeps computing (g g -> t t~ g g g, 10 x 48, FP64 / mixed ms
        per 65536 events: 156.6 / 77.9 at 1, 142.8 / 72.0 at 2, 140.5 / 70.9
        at 3, 140.7 / 71.4 at 4, 144.4 / 76.1 at 6, 157.7 / 88.0 at 12: each
        read in flight holds registers);
      - a flow already folded in the same kernel goes to an overflow slot
        (a kernel never reads back its own stores).
    A colour kernel adds the overflow slots and forms Re(J^dagger C J).
    kin: the four waves of a block (one helicity each, the same 64 events)
    share the events' momenta, momentum sums and denominators in LDS rows,
    which each chunk fills for what it uses."""
    assert not (lds and kin), "external wavefunctions in LDS go with the register-momenta form (kin=False)"
    n_ext, gluon_legs, terms, n_diag, flows, C, cden, sched = _gg_setup(pdg)
    ncol = len(flows)
    order = sched.low_pressure_order()
    n = len(order)
    chunks = [order[i * n // n_chunks:(i + 1) * n // n_chunks] for i in range(n_chunks)]
    # each chunk evaluates its own currents: order its amplitudes afresh for
    # few live currents (for g g -> t t~ g g g the peak per chunk falls from
    # up to 30 currents to at most 14)
    chunks = [sched.low_pressure_order(c) for c in chunks]
    written: set = set()
    overflow_flow: List[int] = []
    chunk_bodies = []
    chunk_rows: List[tuple] = []  # per chunk: (mask -> row, denominator key -> row)
    flops_hel = 0
    n_rmw = 0
    for chunk in chunks:
        em = Emitter(n_ext, [i < 2 for i in range(n_ext)], [abs(x) == 6 for x in pdg])
        # External wavefunctions are used without register barriers here.  The
        # variant with barriers (empty asm statements forcing each external
        # wavefunction into VGPRs at every use) spills less, but its FP64 build
        # returned wrong values on gfx950, while the same generated code
        # compiled for the CPU is exact with and without the barriers: the
        # defect lies in the device compilation of that variant, and a CPU test
        # keeps the generator from emitting it.
        body = GGBody(sched, pdg, em, fresh_externals=False, inplace=inplace, lds_momenta=lds or kin,
                      mom_block="EV" if kin else "64", ext_lds=lds)
        body.kin_lazy = kin
        uses: Dict[int, List[int]] = {}
        for j, a in enumerate(chunk):
            for f, _, _ in a.coeffs:
                uses.setdefault(f, []).append(j)
        ptr = {f: 0 for f in uses}
        open_acc: Dict[int, str] = {}
        folded_here: set = set()
        last_fold: Dict[int, int] = {}     # flow -> index of its latest fold in this chunk
        fold_lines: List[int] = []          # line index of every fold in this chunk
        rmw: List[tuple] = []               # (fold number, flow, prefetch variable)
        nacc = [0]

        def fold(f):
            v = open_acc.pop(f)
            nonlocal n_rmw
            k = len(fold_lines)
            # a flow this kernel stored before is read back like one from an
            # earlier kernel, provided its prefetch (issued `prefetch` folds
            # ahead) comes after that store; otherwise it goes to an overflow slot
            if f in folded_here and not (k >= prefetch and last_fold[f] <= k - prefetch):
                em.w(f"Ov[{len(overflow_flow)}ll * ldp] = {v};")
                overflow_flow.append(f)
            elif f not in written:
                em.w(f"Jc[{f}ll * ldp] = {v};")
                written.add(f)
            else:
                pf = f"pf{len(rmw)}"
                rmw.append((len(fold_lines), f, pf))
                em.w(f"Jc[{f}ll * ldp] = {pf} + {v};")
                n_rmw += 1
            folded_here.add(f)
            last_fold[f] = k
            fold_lines.append(len(em.lines) - 1)

        for j, a in enumerate(chunk):
            body.amplitude(a)
            parts = []
            for f, re, im in a.coeffs:
                ptr[f] += 1
                if f in open_acc:
                    parts.append(f"acc({open_acc[f]}, a, {re}, {im});")
                else:
                    v = f"j{nacc[0]}"
                    nacc[0] += 1
                    open_acc[f] = v
                    em.lines.insert(len(em.lines) - (1 if a.routine != "vvv_amp" else 2), f"    cx<T> {v};")
                    parts.append(f"{v} = mk<T>((T)0, (T)0); acc({v}, a, {re}, {im});")
            em.w(f"  {' '.join(parts)} }}")
            for f in [f for f in open_acc if ptr[f] >= len(uses[f])]:
                fold(f)
            while len(open_acc) > budget:
                far = max(open_acc, key=lambda f: uses[f][ptr[f]])
                fold(far)
        for f in list(open_acc):
            fold(f)
        # prefetch reads of J written by earlier kernels, `prefetch` folds ahead
        inserts = []
        for k, f, pf in rmw:
            at = fold_lines[k - prefetch] + 1 if k >= prefetch else 0
            inserts.append((at, f"    const cx<T> {pf} = Jc[{f}ll * ldp];"))
        for at, line in sorted(inserts, key=lambda t: -t[0]):
            em.lines.insert(at, line)
        chunk_bodies.append("\n".join(em.lines))
        chunk_rows.append((dict(body.kin_rows), dict(body.den_rows)))
        flops_hel += sum(FLOPS[a.routine] + FLOPS["acc"] * len(a.coeffs) for a in chunk)
        flops_hel += sum(sched.currents[k].cost for k in body.names if k[0] != "X")
    assert written == set(range(ncol)), "every flow receives a contribution"
    # executed work, with the currents that several chunks recompute
    flops_exec = flops_hel + 2 * ncol * ncol + 4 * ncol + 2 * (n_rmw + len(overflow_flow)) + 90 * n_ext * n_chunks
    # algorithmic work: every current once, as in the fused kernels
    flops_hel = sched.flops_per_helicity() + 2 * ncol * ncol + 4 * ncol + 90 * n_ext
    overflow_of = [[s for s, f in enumerate(overflow_flow) if f == fl] for fl in range(ncol)]
    return _gg_meta(name, pdg, n_ext, gluon_legs, terms, n_diag, ncol, cden, sched, flops_hel, "",
                    staged=True, chunk_bodies=chunk_bodies, n_overflow=len(overflow_flow), n_rmw=n_rmw,
                    kin=kin, chunk_prologues=[staged_kin_lines(k, d, sum(1 << i for i in range(2)))
                                              for k, d in chunk_rows] if kin else None,
                    flops_exec_per_hel=flops_exec, lds=lds,
                    overflow_of=overflow_of, colour_num=[int(v * cden) for row in C for v in row])


def staged_kin_lines(kin_rows: Dict[int, int], den_rows: Dict[tuple, int], inmask: int, ngroups: int = 8) -> str:
    """Chunk prologue filling the block's kinematics rows for its EV events:
    skin row r with the flow-in momentum of its legs (as T), sden row k with
    1/(P^2 - m^2) (double, then T), each formed exactly as the chunk formed
    it per lane before.  Rows fall into ngroups groups by r % ngroups; group
    w is filled by helicity slot w % HB, each lane its event's column."""
    nwaves = ngroups
    rows = [[] for _ in range(nwaves)]
    B = "EV"
    for m, r in kin_rows.items():
        rows[r % nwaves].append(
            f"    {{ double kd[4]; flow_momentum_lds<{m}u, {inmask}u, NEXT, {B}>(kd, smom, lane); "
            f"T* p = skin + ({r} * {B} + lane) * 4; p[0] = (T)kd[0]; p[1] = (T)kd[1]; p[2] = (T)kd[2]; "
            "p[3] = (T)kd[3]; }")
    for k, r in den_rows.items():
        if k[0] == "vvv":
            _, m1, m2, mass = k
            rows[r % nwaves].append(
                f"    {{ double k1d[4]; flow_momentum_lds<{m1}u, {inmask}u, NEXT, {B}>(k1d, smom, lane); "
                f"double k2d[4]; flow_momentum_lds<{m2}u, {inmask}u, NEXT, {B}>(k2d, smom, lane); "
                "const double Pd[4] = {k1d[0] + k2d[0], k1d[1] + k2d[1], k1d[2] + k2d[2], k1d[3] + k2d[3]}; "
                f"sden[{r} * {B} + lane] = (T)inv_virt(Pd, {mass}); }}")
        else:
            _, m, mass = k
            rows[r % nwaves].append(
                f"    {{ double Pd[4]; flow_momentum_lds<{m}u, {inmask}u, NEXT, {B}>(Pd, smom, lane); "
                f"sden[{r} * {B} + lane] = (T)inv_virt(Pd, {mass}); }}")
    out = [f"  constexpr int NKIN = {max(len(kin_rows), 1)};", f"  constexpr int NDEN = {max(len(den_rows), 1)};"]
    for w in range(nwaves):
        out.append(f"  if (slot == {w} % HB) {{")
        out += rows[w]
        out.append("  }")
    return "\n".join(out)


def _fact(n: int) -> int:
    r = 1
    for i in range(2, n + 1):
        r *= i
    return r


def emit_ee_process(name: str, pdg: List[int]) -> Dict:
    """e+ e- -> mu+ mu- through s-channel photon and Z (massless leptons)."""
    lines = []
    w = lambda s: lines.append("    " + s)
    lam = lambda i: f"((hc >> {3 - i}) & 1 ? 1 : -1)"
    w("double q[4][4];")
    w("for (int i = 0; i < 4; ++i) load_mom_lds<EVB>(q[i], smom, lane, i);")
    w(f"const wf<T> x0 = ext_bra<T>(q[0], 0.0, {lam(0)}, true);   // vbar(e+)")
    w(f"const wf<T> x1 = ext_ket<T>(q[1], 0.0, {lam(1)}, false);  // u(e-)")
    w(f"const wf<T> x2 = ext_ket<T>(q[2], 0.0, {lam(2)}, true);   // v(mu+)")
    w(f"const wf<T> x3 = ext_bra<T>(q[3], 0.0, {lam(3)}, false);  // ubar(mu-)")
    w("const double sd = (q[0][0] + q[1][0]) * (q[0][0] + q[1][0]) - (q[0][1] + q[1][1]) * (q[0][1] + q[1][1])"
      " - (q[0][2] + q[1][2]) * (q[0][2] + q[1][2]) - (q[0][3] + q[1][3]) * (q[0][3] + q[1][3]);")
    w("const wf<T> je = ffv_vec_chiral<T>(x0, x1, (T)1, (T)1);")
    w("const wf<T> jm = ffv_vec_chiral<T>(x3, x2, (T)1, (T)1);")
    w("cx<T> J[1];")
    w("J[0] = (T)(args.ee_qq / sd) * mdot(je, jm);")
    w("if (args.z_enabled) {")
    w("  const wf<T> zl = ffv_vec_chiral<T>(x0, x1, (T)args.ee_gl, (T)args.ee_gr);")
    w("  const wf<T> zm = ffv_vec_chiral<T>(x3, x2, (T)args.ee_gl, (T)args.ee_gr);")
    w("  // Z propagator 1 / (s - mZ^2 + i mZ GZ); the q_mu q_nu term vanishes between massless currents")
    w("  const double dr = sd - args.mz * args.mz, di = args.mz * args.wz, dn = 1.0 / (dr * dr + di * di);")
    w("  const cx<T> prop = mk<T>((T)(args.ee_zz * dr * dn), (T)(-args.ee_zz * di * dn));")
    w("  J[0] = J[0] + prop * mdot(zl, zm);")
    w("}")
    meta = dict(name=name, pdg=pdg, n_ext=4, n_diagrams=2, n_terms=2, ncol=1, cden=1, n_currents=4,
                n_amps=2, gs_power=0, spin_colour_avg=4, ident=1, kind="ee",
                flops_per_hel=2 * 128 + 2 * 30 + 20, flops_per_event=40, body="\n".join(lines), hel_lanes=4,
                colour="      const double me = (double)((TC)J[0].re * (TC)J[0].re + (TC)J[0].im * (TC)J[0].im);")
    return meta


KERNEL_HEADER_TEMPLATE = r"""// Generated by paper_2303_18244_amd.codegen for {title}.
// {n_diagrams} Feynman diagrams ({n_terms} colour/Lorentz terms), {ncol} colour flows,
// {n_currents} shared off-shell currents and {n_amps} amplitude vertices per helicity.
#pragma once
#include "../helamp.h"
#include "../me_kernel.h"
#include "../colour_mfma.h"
#include "../events.h"

namespace mgme {{
namespace {name} {{

constexpr int NEXT = {n_ext};
constexpr int NCOL = {ncol};
// HL lanes evaluate one event, lane `sub` taking its good helicities
// sub, sub + HL, ...; a block holds EVB events.
constexpr int HL = {hel_lanes};
constexpr int EVB = MGME_ME_BLOCK / HL;

// Blocks of a launch over nevt events.
inline unsigned me_blocks(long long nevt) {{ return (unsigned)((nevt + EVB - 1) / EVB); }}

// T: precision of the diagrams; TC: precision of the colour quadratic form.
// MODE 0: |M|^2 summed over the good helicities into out[e];
// MODE 1: each helicity's contribution into out[ih*ldo + e];
// MODE 2: the colour-flow vector J of every helicity into
//         Jout[(ih*NCOL + s)*ldo + e] (single precision) for the matrix-core colour sum;
// MODE 3: as MODE 0, and for the helicity and colour choice each helicity's
//         |M_h|^2 (before normalisation) into aux[ih*lda + e] and
//         sum_h |J_s|^2 into aux[(nhel + s)*lda + e];
// MODE 4: as MODE 0, with the colour sum of every helicity on the matrix
//         cores of the wave (single-precision J split into two half-precision
//         parts, at most 32 flows).
// MODE 4 is compiled for two waves per SIMD (the FP32 diagrams fit in 256
// registers; the matrix-core accumulators would otherwise push the kernel to
// AGPRs and one wave).
template <typename T, int MODE, typename TC = double>
__global__ void __launch_bounds__(MGME_ME_BLOCK) __attribute__((amdgpu_waves_per_eu(MODE == 4 ? 2 : 1)))
me_kernel(const double* __restrict__ mom, long long nevt, long long ld, const MeArgs args, double* __restrict__ out,
          long long ldo, float2* __restrict__ Jout, double* __restrict__ aux, long long lda) {{
  const int tid = threadIdx.x;
  const int lane = tid / HL;  // the event's column in the block's LDS rows
  const int sub = tid % HL;
  const long long e_raw = (long long)blockIdx.x * EVB + lane;
  // every lane stays to the end (block barriers; MODE 4 also needs the whole
  // wave): lanes past the batch evaluate its last event and store nothing
  const bool e_live = e_raw < nevt;
  const long long e = e_live ? e_raw : nevt - 1;
  mfma_half8 cfa[MODE == 4 ? 2 : 1];
  if constexpr (MODE == 4) {{
    const mfma_half8* cf = (const mfma_half8*)args.cfrag;
    cfa[0] = cf[tid & 63];
    cfa[1] = cf[64 + (tid & 63)];
  }}
  // per-lane jamp^2 accumulators (MODE 3): in registers in FP64 (whose one
  // wave per SIMD leaves room), else in LDS, [flow][lane of the block]; the
  // event's sum over its lanes is formed in LDS at the end
  constexpr bool kJ2Regs = sizeof(T) == 8;
  __shared__ double j2[MODE == 3 ? NCOL * MGME_ME_BLOCK : 1];
  double j2r[MODE == 3 && kJ2Regs ? NCOL : 1];
  if constexpr (MODE == 3) {{
#pragma unroll
    for (int s = 0; s < NCOL; ++s) {{
      if constexpr (kJ2Regs) j2r[s] = 0.0;
      else j2[s * MGME_ME_BLOCK + tid] = 0.0;
    }}
  }}
  // The event's momenta in LDS, loaded by its lanes together; every
  // momentum-dependent quantity of the helicity loop is read from LDS where
  // it is needed instead of being held in registers across it.
  __shared__ double smom[NEXT * 4 * EVB];
  for (int k = sub; k < NEXT * 4; k += HL) smom[k * EVB + lane] = mom[(long long)k * ld + e];
  __syncthreads();
  const double mt = args.mt;
{kin_prologue}
  __syncthreads();
  double part = 0.0;
  const int nit = (args.nhel + HL - 1) / HL;
#pragma unroll 1
  for (int it = 0; it < nit; ++it) {{
    // a lane without a helicity left evaluates the last one (the wave's
    // matrix-core step in MODE 4 needs every lane) and drops the value
    int ih = it * HL + sub;
    const bool h_live = ih < args.nhel;
    if (!h_live) ih = args.nhel - 1;
    const int hc = args.hel[ih];
{body}
    // Values are pinned before a store that only some lanes make, and the
    // sums take them through selects: otherwise the compiler sinks the whole
    // evaluation into the lanes' branch, where it needs far more registers.
    if constexpr (MODE == 2) {{
#pragma unroll
      for (int s = 0; s < NCOL; ++s) {{
        pin(J[s].re);
        pin(J[s].im);
      }}
      if (e_live && h_live) {{
#pragma unroll
        for (int s = 0; s < NCOL; ++s)
          Jout[((long long)ih * NCOL + s) * ldo + e] = make_float2((float)J[s].re, (float)J[s].im);
      }}
    }} else if constexpr (MODE == 4) {{
      const double m = colour_mfma_lane<NCOL>(J, cfa);
      part += h_live ? m : 0.0;
    }} else {{
{colour}
      if constexpr (MODE == 1) {{
        double v = me * args.factor;
        pin(v);
        if (e_live && h_live) out[(long long)ih * ldo + e] = v;
      }} else {{
        part += h_live ? me : 0.0;
        if constexpr (MODE == 3) {{
          double v = me;
          pin(v);
          if (e_live && h_live) aux[(long long)ih * lda + e] = v;
#pragma unroll
          for (int s = 0; s < NCOL; ++s) {{
            const double a2 = (double)J[s].re * (double)J[s].re + (double)J[s].im * (double)J[s].im;
            if constexpr (kJ2Regs) j2r[s] += h_live ? a2 : 0.0;
            else j2[s * MGME_ME_BLOCK + tid] += h_live ? a2 : 0.0;
          }}
        }}
      }}
    }}
  }}
  // The event's sums: its lanes' partial sums added in lane order, so every
  // launch shape and batch gives the same bits.
  if constexpr (MODE == 0 || MODE == 3 || MODE == 4) {{
    __shared__ double sred[MGME_ME_BLOCK];
    sred[tid] = part;
    if constexpr (MODE == 3 && kJ2Regs) {{
#pragma unroll
      for (int s = 0; s < NCOL; ++s) j2[s * MGME_ME_BLOCK + tid] = j2r[s];
    }}
    __syncthreads();
    if (sub == 0 && e_live) {{
      double total = 0.0;
#pragma unroll
      for (int i = 0; i < HL; ++i) total += sred[lane * HL + i];
      out[e] = total * args.factor;
    }}
    if constexpr (MODE == 3) {{
      for (int s = sub; s < NCOL; s += HL) {{
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < HL; ++i) t += j2[s * MGME_ME_BLOCK + lane * HL + i];
        if (e_live) aux[(long long)(args.nhel + s) * lda + e] = t;
      }}
    }}
  }}
}}

}}  // namespace {name}
}}  // namespace mgme
"""

LAUNCH_TEMPLATE = r"""// Generated by paper_2303_18244_amd.codegen for {title}: launcher.
// The kernel instantiations of each precision sit in units of their own
// (me_{name}_<precision>.hip) so that they compile in parallel.
#include "me_{name}_kernel.h"

extern "C" hipError_t mgme_select_{name}(int prec, const double* mom, long long nevt, long long ld,
                                          const mgme::MeArgs* args, double* out, const mgme::SelectArgs* sel,
                                          const mgme::Workspace* wsp, hipStream_t stream);
extern "C" hipError_t mgme_run_{name}_d(int per_hel, dim3 grid, const double* mom, long long nevt, long long ld,
                                         const mgme::MeArgs* args, double* out, long long ldo,
                                         const mgme::Workspace* wsp, hipStream_t stream);
extern "C" hipError_t mgme_run_{name}_f(int per_hel, dim3 grid, const double* mom, long long nevt, long long ld,
                                         const mgme::MeArgs* args, double* out, long long ldo,
                                         const mgme::Workspace* wsp, hipStream_t stream);
extern "C" hipError_t mgme_run_{name}_dc(int per_hel, dim3 grid, const double* mom, long long nevt, long long ld,
                                          const mgme::MeArgs* args, double* out, long long ldo,
                                          const mgme::Workspace* wsp, hipStream_t stream);
extern "C" hipError_t mgme_run_{name}_m(dim3 grid, const double* mom, long long nevt, long long ld,
                                         const mgme::MeArgs* args, double* out, const mgme::Workspace* wsp,
                                         hipStream_t stream);

extern "C" hipError_t mgme_launch_{name}(int prec, int per_hel, const double* mom, long long nevt, long long ld,
                                          const mgme::MeArgs* args, double* out, long long ldo,
                                          const mgme::SelectArgs* sel, const mgme::Workspace* wsp,
                                          hipStream_t stream) {{
  using namespace mgme::{name};
  const dim3 block(MGME_ME_BLOCK);
  // One launch covers at most 2^28 events (2^31 lanes at eight lanes per
  // event): larger batches run as consecutive parts, each event's result
  // the same.  (The workspace paths below already run in sub-batches.)
  constexpr long long kMaxLaunch = 1ll << 28;
  const bool ws_path = sel || (prec == 2 && (per_hel || NCOL > 32));
  if (nevt > kMaxLaunch && !ws_path) {{
    hipError_t err = hipSuccess;
    for (long long s0 = 0; s0 < nevt && err == hipSuccess; s0 += kMaxLaunch) {{
      const long long n = nevt - s0 < kMaxLaunch ? nevt - s0 : kMaxLaunch;
      err = mgme_launch_{name}(prec, per_hel, mom + s0, n, ld, args, out + s0, ldo, sel, wsp, stream);
    }}
    return err;
  }}
  if (sel && prec != 2) return mgme_select_{name}(prec, mom, nevt, ld, args, out, sel, wsp, stream);
  if (prec == 2 && !sel && !per_hel && NCOL <= 32) {{
    // the colour sum on the matrix cores inside the diagram kernel
    return mgme_run_{name}_m(dim3(me_blocks(nevt)), mom, nevt, ld, args, out, wsp, stream);
  }}
  if (prec == 2) {{
    // single-precision diagrams write J, the matrix cores form the colour sum
    const int nh = args->nhel;
    const size_t per_event = (size_t)nh * (NCOL * sizeof(float2) + sizeof(double)) + (sel ? NCOL * sizeof(double) : 0);
    const long long sub = mgme::ws_sub_batch(wsp, per_event, (size_t)4 << 30, 0, nevt);
    if (sub == 0) return hipErrorInvalidValue;
    char* ws = nullptr;
    hipError_t err = mgme::ws_acquire(wsp, per_event * (size_t)sub, (void**)&ws, stream);
    if (err != hipSuccess) return err;
    float2* J = (float2*)ws;
    double* meh = (double*)(ws + (size_t)nh * NCOL * sizeof(float2) * sub);
    double* jamp2 = meh + (size_t)nh * sub;
    for (long long start = 0; start < nevt && err == hipSuccess; start += sub) {{
      const long long n = (nevt - start < sub) ? nevt - start : sub;
      me_kernel<float, 2><<<dim3(me_blocks(n)), block, 0, stream>>>(mom + start, n, ld, *args, nullptr, sub, J,
                                                                     nullptr, 0);
      err = hipGetLastError();
      if (err == hipSuccess)
        err = mgme::launch_colour_mfma(n, nh, NCOL, J, sub, args->cfrag, per_hel ? out + start : meh,
                                       per_hel ? ldo : sub, per_hel ? args->factor : 1.0, stream);
      if (err == hipSuccess && !per_hel)
        err = mgme::launch_helicity_sum(n, nh, meh, sub, args->factor, out + start, stream);
      if (err == hipSuccess && sel)
        err = mgme::launch_jamp2<float>(n, nh, NCOL, (const float*)J, sub, jamp2, sub, stream);
      if (err == hipSuccess && sel) err = mgme::launch_select(n, args, meh, sub, NCOL, jamp2, sub, sel, start, stream);
    }}
    const hipError_t ferr = mgme::ws_release(wsp, ws, stream);
    return err != hipSuccess ? err : ferr;
  }}
  const dim3 grid(me_blocks(nevt));
  if (prec == 0) return mgme_run_{name}_d(per_hel, grid, mom, nevt, ld, args, out, ldo, wsp, stream);
  if (prec == 3) return mgme_run_{name}_dc(per_hel, grid, mom, nevt, ld, args, out, ldo, wsp, stream);
  return mgme_run_{name}_f(per_hel, grid, mom, nevt, ld, args, out, ldo, wsp, stream);
}}
"""

RUN_TEMPLATE = r"""// Generated by paper_2303_18244_amd.codegen for {title}: {what}.
#include "me_{name}_kernel.h"

extern "C" hipError_t mgme_run_{name}_{tag}(int per_hel, dim3 grid, const double* mom, long long nevt, long long ld,
                                             const mgme::MeArgs* args, double* out, long long ldo,
                                             const mgme::Workspace* wsp, hipStream_t stream) {{
  using namespace mgme::{name};
  (void)wsp;
  const dim3 block(MGME_ME_BLOCK);
  if (per_hel)  // each helicity's value is written on its own
    me_kernel<{T}, 1, {TC}><<<grid, block, 0, stream>>>(mom, nevt, ld, *args, out, ldo, nullptr, nullptr, 0);
  else
    me_kernel<{T}, 0, {TC}><<<grid, block, 0, stream>>>(mom, nevt, ld, *args, out, ldo, nullptr, nullptr, 0);
  return hipGetLastError();
}}
"""

MIXED_RUN_TEMPLATE = r"""// Generated by paper_2303_18244_amd.codegen for {title}: FP32 diagrams with
// the colour sum on the matrix cores in the same kernel.
#include "me_{name}_kernel.h"

extern "C" hipError_t mgme_run_{name}_m(dim3 grid, const double* mom, long long nevt, long long ld,
                                         const mgme::MeArgs* args, double* out, const mgme::Workspace* wsp,
                                         hipStream_t stream) {{
  using namespace mgme::{name};
  (void)wsp;
  me_kernel<float, 4><<<grid, dim3(MGME_ME_BLOCK), 0, stream>>>(mom, nevt, ld, *args, out, 0, nullptr, nullptr, 0);
  return hipGetLastError();
}}
"""

SELECT_TEMPLATE = r"""// Generated by paper_2303_18244_amd.codegen for {title}: |M|^2 with the
// helicity and leading-colour choice (kernels instantiated in a unit of their
// own so that they compile in parallel with the others).
#include "me_{name}_kernel.h"

extern "C" hipError_t mgme_select_{name}(int prec, const double* mom, long long nevt, long long ld,
                                          const mgme::MeArgs* args, double* out, const mgme::SelectArgs* sel,
                                          const mgme::Workspace* wsp, hipStream_t stream) {{
  using namespace mgme::{name};
  const dim3 block(MGME_ME_BLOCK);
  const int nh = args->nhel;
  const size_t per_event = (size_t)(nh + NCOL) * sizeof(double);
  const long long sub = mgme::ws_sub_batch(wsp, per_event, (size_t)4 << 30, 0, nevt);
  if (sub == 0) return hipErrorInvalidValue;
  double* ws = nullptr;
  hipError_t err = mgme::ws_acquire(wsp, per_event * (size_t)sub, (void**)&ws, stream);
  if (err != hipSuccess) return err;
  for (long long start = 0; start < nevt && err == hipSuccess; start += sub) {{
    const long long n = (nevt - start < sub) ? nevt - start : sub;
    const dim3 grid(me_blocks(n));
    if (prec == 0)
      me_kernel<double, 3><<<grid, block, 0, stream>>>(mom + start, n, ld, *args, out + start, 0, nullptr, ws, sub);
    else if (prec == 3)
      me_kernel<double, 3, float><<<grid, block, 0, stream>>>(mom + start, n, ld, *args, out + start, 0, nullptr, ws,
                                                               sub);
    else
      me_kernel<float, 3><<<grid, block, 0, stream>>>(mom + start, n, ld, *args, out + start, 0, nullptr, ws, sub);
    err = hipGetLastError();
    if (err == hipSuccess)
      err = mgme::launch_select(n, args, ws, sub, NCOL, ws + (size_t)nh * sub, sub, sel, start, stream);
  }}
  const hipError_t ferr = mgme::ws_release(wsp, ws, stream);
  return err != hipSuccess ? err : ferr;
}}
"""


def kernel_sources(meta: Dict) -> Dict[str, str]:
    """File name -> source for a process evaluated by one fused kernel."""
    title = " ".join(str(x) for x in meta["pdg"])
    name = meta["name"]
    out = {f"me_{name}_kernel.h": KERNEL_HEADER_TEMPLATE.format(title=title, **{"kin_prologue": "", **meta}),
           f"me_{name}.hip": LAUNCH_TEMPLATE.format(title=title, name=name),
           f"me_{name}_sel.hip": SELECT_TEMPLATE.format(title=title, name=name)}
    for tag, T, TC, what in (("d", "double", "double", "FP64 diagrams and colour sum"),
                             ("f", "float", "double", "FP32 diagrams, FP64 colour sum"),
                             ("dc", "double", "float", "FP64 diagrams, FP32 colour algebra")):
        out[f"me_{name}_{tag}.hip"] = RUN_TEMPLATE.format(title=title, name=name, tag=tag, T=T, TC=TC, what=what)
    out[f"me_{name}_m.hip"] = MIXED_RUN_TEMPLATE.format(title=title, name=name)
    return out


CHUNK_TEMPLATE = r"""// Generated by paper_2303_18244_amd.codegen for {title}: diagram chunk {chunk} of {n_chunks}.
// Each lane evaluates one (event, good helicity); its colour-flow partial sums
// are stored to slots of a device buffer laid out [helicity][slot][event].
#include "../helamp.h"
#include "../me_kernel.h"

namespace mgme {{
namespace {name} {{
namespace c{chunk} {{

constexpr int NEXT = {n_ext};
constexpr long long NCOL = {ncol};
constexpr long long NOV = {n_overflow};

// A block of 256 lanes evaluates EV consecutive events (one lane column
// each) for 256 / EV helicities.
template <typename T> constexpr int kEV = sizeof(T) == 8 ? {fp64_ev} : 64;

// Held to two waves per SIMD (256 registers) where the block's LDS allows
// two blocks per CU: some values spill, but the second wave hides the
// latency of the folds and spills that a lone wave waits for (measured on
// g g -> t t~ g g g, mixed: 91.6 -> 76.0 ms per 65536 events).
template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kEV<T> < 64 || sizeof(T) == 4 ? 2 : 1)))
chunk_kernel(const double* __restrict__ mom, long long nevt, long long ld, const MeArgs args,
             cx<T>* __restrict__ Jbuf, cx<T>* __restrict__ Ovbuf, long long ldp) {{
  constexpr int EV = kEV<T>;
  constexpr int HB = 256 / EV;
  int hs = blockIdx.y * HB + (int)threadIdx.x / EV;
  if constexpr (EV == 64) hs = __builtin_amdgcn_readfirstlane(hs);  // one helicity per wave
  const long long e = (long long)blockIdx.x * EV + (threadIdx.x % EV);
{prologue}
  cx<T>* __restrict__ Jc = Jbuf + (long long)hs * NCOL * ldp + e;
  cx<T>* __restrict__ Ov = Ovbuf + (long long)hs * NOV * ldp + e;
  (void)Ov;
{body}
}}

}}  // namespace c{chunk}
}}  // namespace {name}
}}  // namespace mgme

// {T} diagrams (each precision in a unit of its own, compiled in parallel)
extern "C" hipError_t mgme_{name}_chunk{chunk}_{tag}(const double* mom, long long nevt, long long ld,
                                                    const mgme::MeArgs* args, void* Jbuf, void* Ovbuf, long long ldp,
                                                    hipStream_t stream) {{
  constexpr int EV = mgme::{name}::c{chunk}::kEV<{T}>;
  const dim3 grid((unsigned)((nevt + EV - 1) / EV), (unsigned)((args->nhel + 256 / EV - 1) / (256 / EV)));
  mgme::{name}::c{chunk}::chunk_kernel<{T}><<<grid, 256, 0, stream>>>(mom, nevt, ld, *args,
      (mgme::cx<{T}>*)Jbuf, (mgme::cx<{T}>*)Ovbuf, ldp);
  return hipGetLastError();
}}
"""

COLOUR_TEMPLATE = r"""// Generated by paper_2303_18244_amd.codegen for {title}: colour sum and driver.
// {n_diagrams} Feynman diagrams ({n_terms} colour/Lorentz terms), {ncol} colour flows, evaluated by
// {n_chunks} diagram kernels that fold their partial colour-flow sums into J in device memory
// ({n_rmw} read-modify-write folds and {n_overflow} overflow slots per (event, helicity)).
#include "../helamp.h"
#include "../me_kernel.h"
#include "../colour_mfma.h"
#include "../events.h"

namespace mgme {{
namespace {name} {{

constexpr int NCOL = {ncol};
constexpr long long NOV = {n_overflow};
constexpr int NB = {nb};  // flows per block of the quadratic form

// colour-matrix numerators (common denominator applied in the final factor),
// upper triangle of the symmetric matrix with the off-diagonal entries
// doubled: Re(J^dagger C J) = sum_s Re(conj(J_s) sum_(t >= s) kC[s][t] J_t)
__constant__ double kC[NCOL * NCOL] = {{{cnum}}};

// Adds the overflow slots to J (fixed at generation), then
// me_h = sum_st C_st Re(conj(J_s) J_t) with blocks of NB flows of C J held in
// registers while J streams from memory.
template <typename T, typename TC>
__global__ void __launch_bounds__(256) colour_kernel(long long nevt, const MeArgs args, cx<T>* __restrict__ Jbuf,
                                                    const cx<T>* __restrict__ Ovbuf, long long ldp,
                                                    double* __restrict__ out, long long ldo, double scale) {{
  const int hs = __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (threadIdx.x >> 6));
  const long long e = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
  if (hs >= args.nhel || e >= nevt) return;
  cx<T>* __restrict__ J = Jbuf + (long long)hs * NCOL * ldp + e;
  const cx<T>* __restrict__ Ov = Ovbuf + (long long)hs * NOV * ldp + e;
  (void)Ov;
{overflow_sums}
  TC me = (TC)0;
  for (int b = 0; b < NCOL; b += NB) {{
    TC yr[NB], yi[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) yr[k] = yi[k] = (TC)0;
    for (int t = b; t < NCOL; ++t) {{
      const cx<T> jt = J[(long long)t * ldp];
      const TC jr = (TC)jt.re, ji = (TC)jt.im;
#pragma unroll
      for (int k = 0; k < NB; ++k) {{
        const TC c = (TC)kC[(b + k) * NCOL + t];
        yr[k] += c * jr;
        yi[k] += c * ji;
      }}
    }}
#pragma unroll
    for (int k = 0; k < NB; ++k) {{
      const cx<T> js = J[(long long)(b + k) * ldp];
      me += (TC)js.re * yr[k] + (TC)js.im * yi[k];
    }}
  }}
  out[(long long)hs * ldo + e] = (double)me * scale;
}}

// Adds the overflow slots into J (mixed precision: before the matrix-core colour sum).
template <typename T>
__global__ void __launch_bounds__(256) fold_kernel(long long nevt, const MeArgs args, cx<T>* __restrict__ Jbuf,
                                                  const cx<T>* __restrict__ Ovbuf, long long ldp) {{
  const int hs = __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (threadIdx.x >> 6));
  const long long e = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
  if (hs >= args.nhel || e >= nevt) return;
  cx<T>* __restrict__ J = Jbuf + (long long)hs * NCOL * ldp + e;
  const cx<T>* __restrict__ Ov = Ovbuf + (long long)hs * NOV * ldp + e;
  (void)Ov;
{overflow_sums}
}}

}}  // namespace {name}
}}  // namespace mgme

{chunk_decls}

// Events are processed in sub-batches whose buffers fit the workspace bound:
// the caller's workspace when one is given, else {workspace_bytes} bytes
// from the stream-ordered allocator.
extern "C" hipError_t mgme_launch_{name}(int prec, int per_hel, const double* mom, long long nevt, long long ld,
                                          const mgme::MeArgs* args, double* out, long long ldo,
                                          const mgme::SelectArgs* sel, const mgme::Workspace* wsp,
                                          hipStream_t stream) {{
  using namespace mgme::{name};
  const int nh = args->nhel;
  const int dprec = (prec == 0 || prec == 3) ? 0 : 1;  // diagram precision
  const size_t tsize = dprec == 0 ? sizeof(mgme::cx<double>) : sizeof(mgme::cx<float>);
  const size_t per_event = (size_t)nh * ((NCOL + NOV) * tsize + sizeof(double)) + (sel ? NCOL * sizeof(double) : 0);
  const long long sub = mgme::ws_sub_batch(wsp, per_event, (size_t){workspace_bytes}, {max_sub}, nevt);
  if (sub == 0) return hipErrorInvalidValue;
  const size_t bytes = per_event * (size_t)sub;
  char* ws = nullptr;
  hipError_t err = mgme::ws_acquire(wsp, bytes, (void**)&ws, stream);
  if (err != hipSuccess) return err;
  void* Jbuf = ws;
  void* Ovbuf = ws + (size_t)nh * NCOL * tsize * sub;
  double* meh = (double*)(ws + (size_t)nh * (NCOL + NOV) * tsize * sub);
  double* jamp2 = meh + (size_t)nh * sub;  // helicity and colour choice only
  const double factor = args->factor;
  for (long long start = 0; start < nevt && err == hipSuccess; start += sub) {{
    const long long n = (nevt - start < sub) ? nevt - start : sub;
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((nh + 3) / 4));
{chunk_calls}
    if (err != hipSuccess) break;
    double* dst = per_hel ? out + start : meh;
    const long long ldd = per_hel ? ldo : sub;
    const double sc = per_hel ? factor : 1.0;
    if (prec == 0) {{
      colour_kernel<double, double><<<grid, 256, 0, stream>>>(n, *args, (mgme::cx<double>*)Jbuf,
                                                             (const mgme::cx<double>*)Ovbuf, sub, dst, ldd, sc);
    }} else if (prec == 3) {{
      colour_kernel<double, float><<<grid, 256, 0, stream>>>(n, *args, (mgme::cx<double>*)Jbuf,
                                                            (const mgme::cx<double>*)Ovbuf, sub, dst, ldd, sc);
    }} else if (prec == 1) {{
      colour_kernel<float, double><<<grid, 256, 0, stream>>>(n, *args, (mgme::cx<float>*)Jbuf,
                                                            (const mgme::cx<float>*)Ovbuf, sub, dst, ldd, sc);
    }} else {{
      fold_kernel<float><<<grid, 256, 0, stream>>>(n, *args, (mgme::cx<float>*)Jbuf,
                                                  (const mgme::cx<float>*)Ovbuf, sub);
      err = hipGetLastError();
      if (err == hipSuccess)
        err = mgme::launch_colour_mfma(n, nh, NCOL, Jbuf, sub, args->cfrag, dst, ldd, sc, stream);
    }}
    if (err == hipSuccess) err = hipGetLastError();
    if (err == hipSuccess && !per_hel) err = mgme::launch_helicity_sum(n, nh, meh, sub, factor, out + start, stream);
    if (err == hipSuccess && sel) {{
      // J now holds every flow (overflow slots folded in by the colour step)
      err = dprec == 0 ? mgme::launch_jamp2<double>(n, nh, NCOL, (const double*)Jbuf, sub, jamp2, sub, stream)
                       : mgme::launch_jamp2<float>(n, nh, NCOL, (const float*)Jbuf, sub, jamp2, sub, stream);
      if (err == hipSuccess) err = mgme::launch_select(n, args, meh, sub, NCOL, jamp2, sub, sel, start, stream);
    }}
  }}
  const hipError_t ferr = mgme::ws_release(wsp, ws, stream);
  return err != hipSuccess ? err : ferr;
}}
"""


CHUNK_PROLOGUE_REGS = r"""  if (hs >= args.nhel || e >= nevt) return;
  const int hc = args.hel[hs];
  const double mt = args.mt;
  double q[NEXT][4];
#pragma unroll
  for (int i = 0; i < NEXT; ++i)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) q[i][mu] = mom[(long long)(i * 4 + mu) * ld + e];"""

# The four waves of a block evaluate the same 64 events (one helicity each):
# their momenta are staged once in LDS; each lane's external wavefunctions
# are stored in LDS and loaded again at every use.
CHUNK_PROLOGUE_LDS = r"""  const int lane = threadIdx.x & 63;  // event within the block
  const int xl = threadIdx.x;         // lane within the block
  __shared__ double smom[NEXT * 4 * 64];
  __shared__ T sext[NEXT * 8 * 256];
  for (int k = threadIdx.x; k < NEXT * 4 * 64; k += 256) {
    const long long ev = (long long)blockIdx.x * 64 + (k & 63);
    smom[k] = ev < nevt ? mom[(long long)(k >> 6) * ld + ev] : 0.0;
  }
  __syncthreads();
  if (hs >= args.nhel || e >= nevt) return;
  const int hc = args.hel[hs];
  const double mt = args.mt;"""


# The helicity slots of a block evaluate the same EV events: the events'
# momenta are staged once in LDS, and each chunk forms the momentum sums and
# denominators it uses once per event into LDS rows (NKIN, NDEN and the
# filling code come from the chunk; see staged_kin_lines).
CHUNK_PROLOGUE_KIN = r"""  const int lane = threadIdx.x % EV;  // event within the block
  const int slot = threadIdx.x / EV;  // helicity slot within the block
  const long long ec = e < nevt ? e : nevt - 1;
@@ROWS_DECL@@
  __shared__ double smom[NEXT * 4 * EV];
  __shared__ T skin[NKIN * 4 * EV];
  __shared__ T sden[NDEN * EV];
  for (int k = slot; k < NEXT * 4; k += HB) smom[k * EV + lane] = mom[(long long)k * ld + ec];
  __syncthreads();
  const double mt = args.mt;
@@ROWS_FILL@@
  __syncthreads();
  if (hs >= args.nhel || e >= nevt) return;
  const int hc = args.hel[hs];"""


def _upper_doubled(num: List[int], n: int) -> List[int]:
    """Row-major n x n: 0 below the diagonal, the diagonal, twice the
    off-diagonal entries above it (the matrix is symmetric)."""
    return [0 if t < s else (num[s * n + t] if t == s else 2 * num[s * n + t]) for s in range(n) for t in range(n)]


def staged_sources(meta: Dict, workspace_bytes: int = 12 << 30, max_sub: int = 16384, nb: int = 30,
                   fp64_ev: int = 64) -> Dict[str, str]:
    """File name -> source for a staged process.  fp64_ev: events per block
    of the FP64 chunk kernels (64, or 32 to let two blocks share a CU; the
    FP32 ones take 64).  The 32-event form is generated but has not been
    built: the compiler's register allocation of one such chunk had not
    finished after 25 minutes."""
    assert fp64_ev in (32, 64) and (fp64_ev == 64 or meta.get("kin")), "32-event blocks need the kinematics rows"
    title = " ".join(str(x) for x in meta["pdg"])
    out = {}
    nchunk = len(meta["chunk_bodies"])
    prologue = CHUNK_PROLOGUE_LDS if meta.get("lds") else CHUNK_PROLOGUE_REGS
    for c, body in enumerate(meta["chunk_bodies"]):
        if meta.get("kin"):
            decl, fill = meta["chunk_prologues"][c].split("\n", 2)[:2], meta["chunk_prologues"][c].split("\n", 2)[2]
            prologue = CHUNK_PROLOGUE_KIN.replace("@@ROWS_DECL@@", "\n".join(decl)).replace("@@ROWS_FILL@@", fill)
        for tag, T in (("d", "double"), ("f", "float")):
            out[f"me_{meta['name']}_chunk{c}_{tag}.hip"] = CHUNK_TEMPLATE.format(
                title=title, chunk=c, n_chunks=nchunk, name=meta["name"], n_ext=meta["n_ext"],
                ncol=meta["ncol"], n_overflow=max(1, meta["n_overflow"]), body=body, prologue=prologue,
                tag=tag, T=T, fp64_ev=fp64_ev)
    sums = []
    for fl, sl in enumerate(meta["overflow_of"]):
        if not sl:
            continue
        terms_re = " + ".join(f"Ov[{k}ll * ldp].re" for k in sl)
        terms_im = " + ".join(f"Ov[{k}ll * ldp].im" for k in sl)
        sums.append(f"  {{ cx<T> v = J[{fl}ll * ldp]; v.re += {terms_re}; v.im += {terms_im}; "
                    f"J[{fl}ll * ldp] = v; }}")
    decls = "\n".join(
        f'extern "C" hipError_t mgme_{meta["name"]}_chunk{c}_{tag}(const double*, long long, long long, '
        f'const mgme::MeArgs*, void*, void*, long long, hipStream_t);' for c in range(nchunk) for tag in "df")
    calls = "\n".join(
        f"    if (err == hipSuccess) err = (dprec == 0 ? mgme_{meta['name']}_chunk{c}_d : mgme_{meta['name']}_chunk{c}_f)"
        f"(mom + start, n, ld, args, Jbuf, Ovbuf, sub, stream);" for c in range(nchunk))
    assert meta["ncol"] % nb == 0
    out[f"me_{meta['name']}.hip"] = COLOUR_TEMPLATE.format(
        title=title, name=meta["name"], n_diagrams=meta["n_diagrams"], n_terms=meta["n_terms"],
        ncol=meta["ncol"], n_chunks=nchunk, n_overflow=max(1, meta["n_overflow"]), n_rmw=meta["n_rmw"], nb=nb,
        cnum=", ".join(f"{v}.0" for v in _upper_doubled(meta["colour_num"], meta["ncol"])),
        overflow_sums="\n".join(sums),
        chunk_decls=decls, chunk_calls=calls, workspace_bytes=workspace_bytes, max_sub=max_sub)
    return out
