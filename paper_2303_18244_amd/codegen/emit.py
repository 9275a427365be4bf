"""HIP source emission for one process: a kernel with one lane per event that
loops over the good helicities in lockstep, evaluates the scheduled currents
and amplitudes in straight-line code, accumulates the colour-flow amplitudes
J and adds the colour quadratic form Re(J^dagger C J) in double precision.
"""
from __future__ import annotations

from fractions import Fraction
from math import lcm
from typing import Dict, List

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
    """Lines computing me += Re(J^dagger C J) * den (integer numerators)."""
    n = len(C)
    out = []
    for s in range(n):
        parts_r = [f"{float(C[s][s] * den)!r} * (double)J[{s}].re"]
        parts_i = [f"{float(C[s][s] * den)!r} * (double)J[{s}].im"]
        for t in range(s + 1, n):
            v = C[s][t] * den * 2
            if v == 0:
                continue
            parts_r.append(f"{float(v)!r} * (double)J[{t}].re")
            parts_i.append(f"{float(v)!r} * (double)J[{t}].im")
        out.append(f"me += (double)J[{s}].re * ({' + '.join(parts_r)}) + "
                   f"(double)J[{s}].im * ({' + '.join(parts_i)});")
    return out


def emit_gg_process(name: str, pdg: List[int]) -> Dict:
    """g g -> t t~ + n g."""
    n_ext = len(pdg)
    incoming = [i < 2 for i in range(n_ext)]
    gluon_legs = [i for i, x in enumerate(pdg) if x == 21]
    q_leg, qb_leg = pdg.index(6), pdg.index(-6)
    terms, n_diag = enumerate_terms(gluon_legs)
    flows = col.basis(gluon_legs)
    C = col.colour_matrix(flows)
    cden = 1
    for row in C:
        for v in row:
            cden = lcm(cden, v.denominator)
    sched = Schedule(terms, q_leg, qb_leg, flows)
    em = Emitter(n_ext, incoming, [abs(x) == 6 for x in pdg])

    # external wavefunctions
    names: Dict[tuple, str] = {}
    fresh_fn: Dict[str, str] = {}
    for i in range(n_ext):
        lam = f"((hc >> {n_ext - 1 - i}) & 1 ? 1 : -1)"
        if pdg[i] == 21:
            em.w(f"const wf<T> x{i} = ext_vec<T>(q[{i}], {lam}, {'false' if incoming[i] else 'true'});")
            fresh_fn[f"x{i}"] = "fresh_pol"
        elif i == q_leg:
            em.w(f"const wf<T> x{i} = ext_bra<T>(q[{i}], mt, {lam}, false);")
        else:
            em.w(f"const wf<T> x{i} = ext_ket<T>(q[{i}], mt, {lam}, true);")
        names[("X", i)] = f"x{i}"
    inmask = sum(1 << i for i in range(n_ext) if incoming[i])

    def fr(v: str) -> str:
        return f"{fresh_fn.get(v, 'fresh')}({v})"

    def mom(var: str, mask: int) -> str:
        return (f"double {var}d[4]; flow_momentum<{mask}u, {inmask}u, NEXT>({var}d, q); "
                f"T {var}[4]; to_t({var}, {var}d);")

    def leg_mask(k) -> int:
        return sched.currents[k].mask if k[0] != "X" else 1 << k[1]

    counter = [0]

    def need(key) -> str:
        if key in names:
            return names[key]
        cur = sched.currents[key]
        ins = [need(k) for k in cur.inputs]
        v = f"w{counter[0]}"
        counter[0] += 1
        em.w(f"wf<T> {v};")
        if cur.routine == "vvv_vec":
            c1, c2 = cur.tree.children
            em.w(f"{{ {mom('k1', c1.mask)} {mom('k2', c2.mask)}")
            em.w("  const double Pd[4] = {k1d[0] + k2d[0], k1d[1] + k2d[1], k1d[2] + k2d[2], k1d[3] + k2d[3]};")
            em.w(f"  {v} = vvv_vec<T>({fr(ins[0])}, k1, {fr(ins[1])}, k2, (T)inv_virt(Pd, 0.0)); }}")
        elif cur.routine == "vvvv_vec":
            em.w(f"{{ double Pd[4]; flow_momentum<{cur.mask}u, {inmask}u, NEXT>(Pd, q);")
            em.w(f"  {v} = vvvv_vec<T, {cur.tree.s}>({fr(ins[0])}, {fr(ins[1])}, {fr(ins[2])}, "
                 f"(T)inv_virt(Pd, 0.0)); }}")
        elif cur.routine in ("ket_prop", "bra_prop"):
            em.w(f"{{ {mom('P', cur.mask)}")
            em.w(f"  {v} = {cur.routine}<T>({fr(ins[0])}, {fr(ins[1])}, P, (T)mt, (T)inv_virt(Pd, mt)); }}")
        elif cur.routine == "ffv_vec":
            em.w(f"{{ double Pd[4]; flow_momentum<{cur.mask}u, {inmask}u, NEXT>(Pd, q);")
            em.w(f"  {v} = ffv_vec<T>({fr(ins[0])}, {fr(ins[1])}, (T)inv_virt(Pd, 0.0)); }}")
        else:
            raise ValueError(cur.routine)
        names[key] = v
        return v

    amps = sched.low_pressure_order()
    ncol = len(flows)
    em.w(f"cx<T> J[{ncol}];")
    em.w(f"for (int s = 0; s < {ncol}; ++s) J[s] = mk<T>((T)0, (T)0);")
    for a in amps:
        ins = [need(k) for k in a.inputs]
        if a.routine == "ffv_amp":
            em.w(f"{{ const cx<T> a = ffv_amp<T>({fr(ins[0])}, {fr(ins[1])}, {fr(ins[2])});")
        elif a.routine == "vvv_amp":
            m1, m2, m3 = (leg_mask(k) for k in a.inputs)
            em.w(f"{{ {mom('k1', m1)} {mom('k2', m2)} {mom('k3', m3)}")
            em.w(f"  const cx<T> a = vvv_amp<T>({fr(ins[0])}, k1, {fr(ins[1])}, k2, {fr(ins[2])}, k3);")
        else:
            em.w(f"{{ const cx<T> a = vvvv_amp<T, {a.s}>({fr(ins[0])}, {fr(ins[1])}, {fr(ins[2])}, "
                 f"{fr(ins[3])});")
        upd = " ".join(f"acc(J[{f}], a, {re}, {im});" for f, re, im in a.coeffs)
        em.w(f"  {upd} }}")
    em.w("double me = 0.0;")
    for line in colour_sum_lines(C, cden):
        em.w(line)

    body = "\n".join(em.lines)
    k = len(gluon_legs)
    n_final_g = len([i for i in gluon_legs if not incoming[i]])
    flops_hel = sched.flops_per_helicity() + 2 * ncol * ncol + 4 * ncol + 90 * n_ext
    meta = dict(name=name, pdg=pdg, n_ext=n_ext, n_diagrams=n_diag, n_terms=len(terms), ncol=ncol,
                cden=cden, n_currents=len(sched.currents), n_amps=len(amps), gs_power=2 * k,
                spin_colour_avg=4 * 64, ident=_fact(n_final_g), kind="qcd",
                flops_per_hel=flops_hel, flops_per_event=8 * 2 ** n_ext,
                body=body)
    return meta


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
    w("double me = (double)J[0].re * (double)J[0].re + (double)J[0].im * (double)J[0].im;")
    meta = dict(name=name, pdg=pdg, n_ext=4, n_diagrams=2, n_terms=2, ncol=1, cden=1, n_currents=4,
                n_amps=2, gs_power=0, spin_colour_avg=4, ident=1, kind="ee",
                flops_per_hel=2 * 128 + 2 * 30 + 20, flops_per_event=40, body="\n".join(lines))
    return meta


KERNEL_TEMPLATE = r"""// Generated by paper_2303_18244_amd.codegen for {title}.
// {n_diagrams} Feynman diagrams ({n_terms} colour/Lorentz terms), {ncol} colour flows,
// {n_currents} shared off-shell currents and {n_amps} amplitude vertices per helicity.
#include "../helamp.h"
#include "../me_kernel.h"

namespace mgme {{
namespace {name} {{

constexpr int NEXT = {n_ext};

template <typename T, bool PER_HEL>
__global__ void __launch_bounds__(MGME_ME_BLOCK) me_kernel(const double* __restrict__ mom, long long nevt,
                                                          long long ld, const MeArgs args,
                                                          double* __restrict__ out, long long ldo) {{
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  double p[NEXT][4];
#pragma unroll
  for (int i = 0; i < NEXT; ++i)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) p[i][mu] = mom[(long long)(i * 4 + mu) * ld + e];
  const double mt = args.mt;
  double total = 0.0;
  for (int ih = 0; ih < args.nhel; ++ih) {{
    const int hc = args.hel[ih];
    // Re-derive every momentum-dependent quantity inside the helicity loop
    // instead of holding all of them in registers across it.
    double q[NEXT][4];
#pragma unroll
    for (int i = 0; i < NEXT; ++i)
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {{
        q[i][mu] = p[i][mu];
        asm volatile("" : "+v"(q[i][mu]));
      }}
{body}
    if (PER_HEL) out[(long long)ih * ldo + e] = me * args.factor;
    else total += me;
  }}
  if (!PER_HEL) out[e] = total * args.factor;
}}

}}  // namespace {name}
}}  // namespace mgme

extern "C" hipError_t mgme_launch_{name}(int prec, int per_hel, const double* mom, long long nevt, long long ld,
                                          const mgme::MeArgs* args, double* out, long long ldo,
                                          hipStream_t stream) {{
  const dim3 block(MGME_ME_BLOCK);
  const dim3 grid((unsigned)((nevt + MGME_ME_BLOCK - 1) / MGME_ME_BLOCK));
  if (prec == 0) {{
    if (per_hel) mgme::{name}::me_kernel<double, true><<<grid, block, 0, stream>>>(mom, nevt, ld, *args, out, ldo);
    else mgme::{name}::me_kernel<double, false><<<grid, block, 0, stream>>>(mom, nevt, ld, *args, out, ldo);
  }} else {{
    if (per_hel) mgme::{name}::me_kernel<float, true><<<grid, block, 0, stream>>>(mom, nevt, ld, *args, out, ldo);
    else mgme::{name}::me_kernel<float, false><<<grid, block, 0, stream>>>(mom, nevt, ld, *args, out, ldo);
  }}
  return hipGetLastError();
}}
"""


def kernel_source(meta: Dict) -> str:
    return KERNEL_TEMPLATE.format(title=" ".join(str(x) for x in meta["pdg"]), **meta)
