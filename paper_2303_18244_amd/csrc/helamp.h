// Device routines for helicity amplitudes on gfx950: external wavefunctions,
// off-shell currents with their propagators and vertex contractions, in the
// chiral representation, templated on the floating-point type T (double or
// float).  Kinematic inputs (momenta, propagator denominators) are always
// double; wavefunctions and vertex arithmetic are in T.
//
// The matrix element is built from Feynman diagrams and helicity amplitudes
// (paper, section 1).  Conventions: metric (+,-,-,-); gamma^mu =
// [[0, sigma^mu], [sigmabar^mu, 0]], sigma^mu = (1, s_k), sigmabar^mu =
// (1, -s_k); upper spinor components are left-handed.  Every routine returns
// the bare Lorentz structure: vertex couplings and the factors of i from
// vertices and propagators are folded into one constant phase per diagram by
// the process compiler.  Momenta passed to routines are flow-in momenta (the
// momentum flowing from the current into the vertex that consumes it).
#pragma once
#include <hip/hip_runtime.h>

namespace mgme {

template <typename T> struct cx {
  T re, im;
};

template <typename T> __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.re, -a.im}; }
// i * a
template <typename T> __device__ __forceinline__ cx<T> timesi(cx<T> a) { return {-a.im, a.re}; }

// Fused multiply-adds.  Sums of complex products are written as chains of
// these: n products then take 2 multiplies and 4n - 2 FMAs, where the plain
// expression tree costs 2n multiplies, 2n FMAs and 2(n-1) additions.
template <typename T> __device__ __forceinline__ T fmaT(T a, T b, T c) {
  if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
}
// a * b
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {fmaT(a.re, b.re, -(a.im * b.im)), fmaT(a.re, b.im, a.im * b.re)};
}
// acc + a * b
template <typename T> __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
  return {fmaT(a.re, b.re, fmaT(-a.im, b.im, acc.re)), fmaT(a.re, b.im, fmaT(a.im, b.re, acc.im))};
}
// acc - a * b
template <typename T> __device__ __forceinline__ cx<T> cfms(cx<T> a, cx<T> b, cx<T> acc) {
  return {fmaT(-a.re, b.re, fmaT(a.im, b.im, acc.re)), fmaT(-a.re, b.im, fmaT(-a.im, b.re, acc.im))};
}
// acc + s * a, s real
template <typename T> __device__ __forceinline__ cx<T> sfma(T s, cx<T> a, cx<T> acc) {
  return {fmaT(s, a.re, acc.re), fmaT(s, a.im, acc.im)};
}

// Four complex components: a spinor (ket column or bra row) or a
// contravariant vector.
template <typename T> struct wf {
  cx<T> c[4];
};

// Minkowski product of two complex vectors (no conjugation).
template <typename T> __device__ __forceinline__ cx<T> mdot(const wf<T>& a, const wf<T>& b) {
  return cfms(a.c[3], b.c[3], cfms(a.c[2], b.c[2], cfms(a.c[1], b.c[1], cmul(a.c[0], b.c[0]))));
}
// Minkowski product of a real vector with a complex vector.
template <typename T> __device__ __forceinline__ cx<T> mdot(const T k[4], const wf<T>& a) {
  return sfma(-k[3], a.c[3], sfma(-k[2], a.c[2], sfma(-k[1], a.c[1], k[0] * a.c[0])));
}

// ---------------------------------------------------------------- externals
// Two-component helicity eigenvectors chi_+ and chi_- of sigma.p / |p|, with
// the fixed phase chi_+ = (0,1), chi_- = (-1,0) for p along -z.
__device__ __forceinline__ void helicity_basis(const double p[4], double chp[4], double chm[4]) {
  const double px = p[1], py = p[2], pz = p[3];
  const double pabs = sqrt(px * px + py * py + pz * pz);
  if (px == 0.0 && py == 0.0 && pz < 0.0) {
    chp[0] = 0; chp[1] = 0; chp[2] = 1; chp[3] = 0;
    chm[0] = -1; chm[1] = 0; chm[2] = 0; chm[3] = 0;
    return;
  }
  const double ppz = pz >= 0.0 ? pabs + pz : (px * px + py * py) / (pabs - pz);
  const double nrm = 1.0 / sqrt(2.0 * pabs * ppz);
  chp[0] = ppz * nrm; chp[1] = 0.0; chp[2] = px * nrm; chp[3] = py * nrm;    // (re0, im0, re1, im1)
  chm[0] = -px * nrm; chm[1] = py * nrm; chm[2] = ppz * nrm; chm[3] = 0.0;
}

// sqrt(E + |p|) and sqrt(E - |p|) with the on-shell energy sqrt(|p|^2 + m^2).
__device__ __forceinline__ void spinor_scales(const double p[4], double m, double& big, double& small) {
  const double pabs = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  const double e = m == 0.0 ? pabs : sqrt(pabs * pabs + m * m);
  big = sqrt(e + pabs);
  small = m == 0.0 ? 0.0 : m / big;
}

// Ket spinor: u(p, lam) of an incoming fermion (anti = false) or v(p, lam)
// of an outgoing antifermion (anti = true); lam = +-1 is the helicity.
template <typename T>
__device__ __forceinline__ wf<T> ext_ket(const double p[4], double m, int lam, bool anti) {
  double chp[4], chm[4], big, small;
  helicity_basis(p, chp, chm);
  spinor_scales(p, m, big, small);
  // u(+) = (small chi+, big chi+), u(-) = (big chi-, small chi-)
  // v(+) = (-big chi-, small chi-), v(-) = (small chi+, -big chi+)
  const bool plus_chi = anti ? (lam < 0) : (lam > 0);
  const double* ch = plus_chi ? chp : chm;
  double up, lo;
  if (!anti) {
    up = lam > 0 ? small : big;
    lo = lam > 0 ? big : small;
  } else {
    up = lam > 0 ? -big : small;
    lo = lam > 0 ? small : -big;
  }
  wf<T> w;
  w.c[0] = mk<T>((T)(up * ch[0]), (T)(up * ch[1]));
  w.c[1] = mk<T>((T)(up * ch[2]), (T)(up * ch[3]));
  w.c[2] = mk<T>((T)(lo * ch[0]), (T)(lo * ch[1]));
  w.c[3] = mk<T>((T)(lo * ch[2]), (T)(lo * ch[3]));
  return w;
}

// Bra spinor (Dirac adjoint, psi^dagger gamma^0): ubar(p, lam) of an outgoing
// fermion (anti = false) or vbar(p, lam) of an incoming antifermion.
template <typename T>
__device__ __forceinline__ wf<T> ext_bra(const double p[4], double m, int lam, bool anti) {
  const wf<T> k = ext_ket<T>(p, m, lam, anti);
  wf<T> b;
  b.c[0] = conjg(k.c[2]);
  b.c[1] = conjg(k.c[3]);
  b.c[2] = conjg(k.c[0]);
  b.c[3] = conjg(k.c[1]);
  return b;
}

// Polarisation vector of a massless vector boson with helicity lam:
// eps = (-lam e1 - i e2)/sqrt(2), e1 = (0, ct cp, ct sp, -st), e2 = (0, -sp, cp, 0);
// complex conjugated for an outgoing boson.
template <typename T>
__device__ __forceinline__ wf<T> ext_vec(const double p[4], int lam, bool outgoing) {
  const double px = p[1], py = p[2], pz = p[3];
  const double pt = sqrt(px * px + py * py);
  const double pabs = sqrt(px * px + py * py + pz * pz);
  const double ct = pz / pabs, st = pt / pabs;
  double cp = 1.0, sp = 0.0;
  if (pt > 0.0) {
    cp = px / pt;
    sp = py / pt;
  }
  const double r2 = 0.70710678118654752440;
  const double l = lam > 0 ? 1.0 : -1.0;
  const double sgn = outgoing ? -1.0 : 1.0;  // conjugation flips the imaginary parts
  wf<T> w;
  w.c[0] = mk<T>((T)0, (T)0);
  w.c[1] = mk<T>((T)(-l * ct * cp * r2), (T)(sgn * sp * r2));
  w.c[2] = mk<T>((T)(-l * ct * sp * r2), (T)(-sgn * cp * r2));
  w.c[3] = mk<T>((T)(l * st * r2), (T)0);
  return w;
}

// ------------------------------------------------------------ Dirac blocks
// V.sigma    = [[V0 - V3, -V1 + i V2], [-V1 - i V2, V0 + V3]]   (upper-right block of Vslash)
// V.sigmabar = [[V0 + V3,  V1 - i V2], [ V1 + i V2, V0 - V3]]   (lower-left block)
template <typename T> struct blocks2 {
  cx<T> a00, a01, a10, a11;
};
template <typename T> __device__ __forceinline__ blocks2<T> vsigma(const wf<T>& V) {
  return {V.c[0] - V.c[3], timesi(V.c[2]) - V.c[1], -V.c[1] - timesi(V.c[2]), V.c[0] + V.c[3]};
}
template <typename T> __device__ __forceinline__ blocks2<T> vsigmabar(const wf<T>& V) {
  return {V.c[0] + V.c[3], V.c[1] - timesi(V.c[2]), V.c[1] + timesi(V.c[2]), V.c[0] - V.c[3]};
}
// V.sigmabar from V.sigma: the diagonals swap and the off-diagonals change
// sign (the negation is free as an FMA operand modifier).
template <typename T> __device__ __forceinline__ blocks2<T> vsigmabar_of(const blocks2<T>& A) {
  return {A.a11, -A.a01, -A.a10, A.a00};
}

// ---------------------------------------------------------------- vertices
// Amplitude bra . Vslash . ket  (quark-gluon vertex, vector coupling).
template <typename T> __device__ __forceinline__ cx<T> ffv_amp(const wf<T>& bra, const wf<T>& ket, const wf<T>& V) {
  const blocks2<T> A = vsigma(V), B = vsigmabar_of(A);
  const cx<T> u0 = cfma(A.a01, ket.c[3], cmul(A.a00, ket.c[2]));
  const cx<T> u1 = cfma(A.a11, ket.c[3], cmul(A.a10, ket.c[2]));
  const cx<T> l0 = cfma(B.a01, ket.c[1], cmul(B.a00, ket.c[0]));
  const cx<T> l1 = cfma(B.a11, ket.c[1], cmul(B.a10, ket.c[0]));
  return cfma(bra.c[3], l1, cfma(bra.c[2], l0, cfma(bra.c[1], u1, cmul(bra.c[0], u0))));
}

// Off-shell ket: (qslash + m) Vslash ket * den, q the momentum along the fermion arrow.
template <typename T>
__device__ __forceinline__ wf<T> ket_prop(const wf<T>& ket, const wf<T>& V, const T q[4], T m, T den) {
  const blocks2<T> A = vsigma(V), B = vsigmabar_of(A);
  // x = Vslash ket
  const cx<T> x0 = cfma(A.a01, ket.c[3], cmul(A.a00, ket.c[2]));
  const cx<T> x1 = cfma(A.a11, ket.c[3], cmul(A.a10, ket.c[2]));
  const cx<T> x2 = cfma(B.a01, ket.c[1], cmul(B.a00, ket.c[0]));
  const cx<T> x3 = cfma(B.a11, ket.c[1], cmul(B.a10, ket.c[0]));
  // y = den (qslash + m) x, q real: q.sigma = [[q0-q3, -q1+iq2],[-q1-iq2, q0+q3]];
  // den is folded into the five real coefficients
  const T qa = den * (q[0] - q[3]), qb = den * (q[0] + q[3]), dm = den * m;
  const cx<T> qm = mk<T>(-den * q[1], den * q[2]);   // den (-q1 + i q2)
  const cx<T> qp = conjg(qm);                        // den (-q1 - i q2)
  wf<T> y;
  y.c[0] = cfma(qm, x3, sfma(qa, x2, dm * x0));
  y.c[1] = cfma(qp, x2, sfma(qb, x3, dm * x1));
  y.c[2] = cfms(qm, x1, sfma(qb, x0, dm * x2));
  y.c[3] = cfms(qp, x0, sfma(qa, x1, dm * x3));
  return y;
}

// Off-shell bra: bra Vslash (qslash + m) * den with q = -P (P the flow-in
// momentum of the new current).
template <typename T>
__device__ __forceinline__ wf<T> bra_prop(const wf<T>& bra, const wf<T>& V, const T P[4], T m, T den) {
  const blocks2<T> A = vsigma(V), B = vsigmabar_of(A);
  // x = bra Vslash (row): upper out = bra_lo B, lower out = bra_up A
  const cx<T> x0 = cfma(bra.c[3], B.a10, cmul(bra.c[2], B.a00));
  const cx<T> x1 = cfma(bra.c[3], B.a11, cmul(bra.c[2], B.a01));
  const cx<T> x2 = cfma(bra.c[1], A.a10, cmul(bra.c[0], A.a00));
  const cx<T> x3 = cfma(bra.c[1], A.a11, cmul(bra.c[0], A.a01));
  // y = den x (qslash + m) with q = -P: upper out = x_lo (q.sigmabar) + m x_up,
  // lower out = x_up (q.sigma) + m x_lo; den is folded into the real coefficients
  const T q0 = -den * P[0], q1 = -den * P[1], q2 = -den * P[2], q3 = -den * P[3], dm = den * m;
  const T qa = q0 - q3, qb = q0 + q3;
  const cx<T> qm = mk<T>(-q1, q2);   // den (-q1 + i q2)  (q.sigma off-diagonal 01)
  const cx<T> qp = conjg(qm);        // den (-q1 - i q2)  (q.sigma off-diagonal 10)
  // q.sigma = [[qa, qm], [qp, qb]], q.sigmabar = [[qb, -qm], [-qp, qa]]
  wf<T> y;
  y.c[0] = cfms(x3, qp, sfma(qb, x2, dm * x0));
  y.c[1] = cfms(x2, qm, sfma(qa, x3, dm * x1));
  y.c[2] = cfma(x1, qp, sfma(qa, x0, dm * x2));
  y.c[3] = cfma(x0, qm, sfma(qb, x1, dm * x3));
  return y;
}

// Vector current bra gamma^mu ket * den (contravariant index).
template <typename T> __device__ __forceinline__ wf<T> ffv_vec(const wf<T>& b, const wf<T>& k, T den) {
  // components 0 and 3 share the pairs p = b0 k2 + b3 k1 and r = b1 k3 + b2 k0
  const cx<T> p = cfma(b.c[3], k.c[1], cmul(b.c[0], k.c[2]));
  const cx<T> r = cfma(b.c[2], k.c[0], cmul(b.c[1], k.c[3]));
  const cx<T> j1 = cfms(b.c[3], k.c[0], cfms(b.c[2], k.c[1], cfma(b.c[1], k.c[2], cmul(b.c[0], k.c[3]))));
  const cx<T> j2 = cfma(b.c[2], k.c[1], cfms(b.c[3], k.c[0], cfms(b.c[0], k.c[3], cmul(b.c[1], k.c[2]))));
  wf<T> J;
  J.c[0] = den * (p + r);
  J.c[1] = den * j1;
  J.c[2] = den * timesi(j2);
  J.c[3] = den * (p - r);
  return J;
}

// Chiral vector current bra gamma^mu (gL PL + gR PR) ket (no propagator).
template <typename T>
__device__ __forceinline__ wf<T> ffv_vec_chiral(const wf<T>& b, const wf<T>& k, T gL, T gR) {
  // right-handed part: bra_up sigma^mu ket_lo; left-handed part: bra_lo sigmabar^mu ket_up
  const cx<T> r0 = b.c[0] * k.c[2] + b.c[1] * k.c[3];
  const cx<T> l0 = b.c[2] * k.c[0] + b.c[3] * k.c[1];
  const cx<T> r1 = b.c[0] * k.c[3] + b.c[1] * k.c[2];
  const cx<T> l1 = b.c[2] * k.c[1] + b.c[3] * k.c[0];
  const cx<T> r2 = b.c[1] * k.c[2] - b.c[0] * k.c[3];
  const cx<T> l2 = b.c[2] * k.c[1] - b.c[3] * k.c[0];
  const cx<T> r3 = b.c[0] * k.c[2] - b.c[1] * k.c[3];
  const cx<T> l3 = b.c[3] * k.c[1] - b.c[2] * k.c[0];
  wf<T> J;
  J.c[0] = gR * r0 + gL * l0;
  J.c[1] = gR * r1 - gL * l1;
  J.c[2] = timesi(gR * r2 + gL * l2);
  J.c[3] = gR * r3 + gL * l3;
  return J;
}

// Three-gluon vertex with leg 3 off shell, all momenta flowing in (k3 = -k1-k2):
// [(V1.V2)(k1-k2) + V2 ((k1+2k2).V1) - V1 ((2k1+k2).V2)] * den
template <typename T>
__device__ __forceinline__ wf<T> vvv_vec(const wf<T>& V1, const T k1[4], const wf<T>& V2, const T k2[4], T den) {
  T d[4], a[4], b[4];
  for (int mu = 0; mu < 4; ++mu) {
    d[mu] = k1[mu] - k2[mu];
    a[mu] = k1[mu] + 2 * k2[mu];
    b[mu] = 2 * k1[mu] + k2[mu];
  }
  const cx<T> v12 = den * mdot(V1, V2);
  const cx<T> s1 = den * mdot(a, V1);
  const cx<T> s2 = den * mdot(b, V2);
  wf<T> W;
  for (int mu = 0; mu < 4; ++mu) W.c[mu] = cfms(V1.c[mu], s2, cfma(V2.c[mu], s1, d[mu] * v12));
  return W;
}

// Three-gluon vertex amplitude, all momenta flowing in.
template <typename T>
__device__ __forceinline__ cx<T> vvv_amp(const wf<T>& V1, const T k1[4], const wf<T>& V2, const T k2[4],
                                         const wf<T>& V3, const T k3[4]) {
  T d12[4], d23[4], d31[4];
  for (int mu = 0; mu < 4; ++mu) {
    d12[mu] = k1[mu] - k2[mu];
    d23[mu] = k2[mu] - k3[mu];
    d31[mu] = k3[mu] - k1[mu];
  }
  return cfma(mdot(V3, V1), mdot(d31, V2), cfma(mdot(V2, V3), mdot(d23, V1), cmul(mdot(V1, V2), mdot(d12, V3))));
}

// Four-gluon vertex, one of its three colour structures, leg 4 off shell.
template <typename T, int S>
__device__ __forceinline__ wf<T> vvvv_vec(const wf<T>& V1, const wf<T>& V2, const wf<T>& V3, T den) {
  wf<T> W;
  if (S == 0) {  // (V1.V3) V2 - (V2.V3) V1
    const cx<T> a = den * mdot(V1, V3), b = den * mdot(V2, V3);
    for (int mu = 0; mu < 4; ++mu) W.c[mu] = cfms(b, V1.c[mu], cmul(a, V2.c[mu]));
  } else if (S == 1) {  // (V1.V2) V3 - (V2.V3) V1
    const cx<T> a = den * mdot(V1, V2), b = den * mdot(V2, V3);
    for (int mu = 0; mu < 4; ++mu) W.c[mu] = cfms(b, V1.c[mu], cmul(a, V3.c[mu]));
  } else {  // (V1.V2) V3 - (V1.V3) V2
    const cx<T> a = den * mdot(V1, V2), b = den * mdot(V1, V3);
    for (int mu = 0; mu < 4; ++mu) W.c[mu] = cfms(b, V2.c[mu], cmul(a, V3.c[mu]));
  }
  return W;
}

template <typename T, int S>
__device__ __forceinline__ cx<T> vvvv_amp(const wf<T>& V1, const wf<T>& V2, const wf<T>& V3, const wf<T>& V4) {
  if (S == 0) return cfms(mdot(V1, V4), mdot(V2, V3), cmul(mdot(V1, V3), mdot(V2, V4)));
  if (S == 1) return cfms(mdot(V1, V4), mdot(V2, V3), cmul(mdot(V1, V2), mdot(V3, V4)));
  return cfms(mdot(V1, V3), mdot(V2, V4), cmul(mdot(V1, V2), mdot(V3, V4)));
}

// Adds c * a to J for a Gaussian-integer c in {+-1, +-i} (or small integers).
template <typename T> __device__ __forceinline__ void acc(cx<T>& J, cx<T> a, int cre, int cim) {
  if (cim == 0) {
    if (cre == 1) J = J + a;
    else if (cre == -1) J = J - a;
    else J = J + (T)cre * a;
  } else if (cre == 0) {
    if (cim == 1) J = J + timesi(a);
    else if (cim == -1) J = J - timesi(a);
    else J = J + (T)cim * timesi(a);
  } else {
    J = J + (T)cre * a + (T)cim * timesi(a);
  }
}

// ------------------------------------------------------- register control
// The straight-line helicity body is evaluated in the order the process
// compiler chose to keep few wavefunctions alive.  An empty volatile asm
// statement gives a value a new identity the compiler cannot see through, so
// each routine call works on fresh copies of its inputs: the compiler can
// neither merge the arithmetic of two calls (which would stretch live ranges
// across the whole body) nor hoist a call above the previous one.
__device__ __forceinline__ double fresh(double x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ float fresh(float x) {
  asm volatile("" : "+v"(x));
  return x;
}
// Wavefunctions get fresh copies only in double precision: there merged live
// ranges spill to scratch memory (measured on gfx950), while in single
// precision the registers suffice and the copies would only cost moves.
template <typename T> __device__ __forceinline__ wf<T> fresh(const wf<T>& w) {
  if constexpr (sizeof(T) == 4) {
    return w;
  } else {
    wf<T> r = w;
    asm volatile("" : "+v"(r.c[0].re), "+v"(r.c[0].im), "+v"(r.c[1].re), "+v"(r.c[1].im), "+v"(r.c[2].re),
                 "+v"(r.c[2].im), "+v"(r.c[3].re), "+v"(r.c[3].im));
    return r;
  }
}
// External polarisation vectors have a vanishing time component and a real
// z component; those constants stay visible to the compiler.
template <typename T> __device__ __forceinline__ wf<T> fresh_pol(const wf<T>& w) {
  if constexpr (sizeof(T) == 4) {
    return w;
  } else {
    wf<T> r = w;
    asm volatile("" : "+v"(r.c[1].re), "+v"(r.c[1].im), "+v"(r.c[2].re), "+v"(r.c[2].im), "+v"(r.c[3].re));
    r.c[0] = mk<T>((T)0, (T)0);
    r.c[3].im = (T)0;
    return r;
  }
}

// Flow-in momentum of the legs in MASK (incoming legs in INMASK count with +,
// outgoing ones with -), summed from fresh copies of the external momenta.
template <unsigned MASK, unsigned INMASK, int NEXT>
__device__ __forceinline__ void flow_momentum(double out[4], const double (&q)[NEXT][4]) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NEXT; ++i)
      if (MASK & (1u << i)) {
        const double x = fresh(q[i][mu]);
        acc = (INMASK & (1u << i)) ? acc + x : acc - x;
      }
    out[mu] = acc;
  }
}

// In-place forms of the two above: the variable itself gets the new
// identity, so no copy is needed when it is used again later.  Emitted
// before every routine call for each of its inputs.
template <typename T> __device__ __forceinline__ void launder(wf<T>& w) {
  if constexpr (sizeof(T) == 8)
    asm volatile("" : "+v"(w.c[0].re), "+v"(w.c[0].im), "+v"(w.c[1].re), "+v"(w.c[1].im), "+v"(w.c[2].re),
                 "+v"(w.c[2].im), "+v"(w.c[3].re), "+v"(w.c[3].im));
}
template <typename T> __device__ __forceinline__ void launder_pol(wf<T>& w) {
  if constexpr (sizeof(T) == 8) {
    asm volatile("" : "+v"(w.c[1].re), "+v"(w.c[1].im), "+v"(w.c[2].re), "+v"(w.c[2].im), "+v"(w.c[3].re));
    w.c[0] = mk<T>((T)0, (T)0);
    w.c[3].im = (T)0;
  }
}

// Momenta staged per lane in LDS: component mu of leg i at
// smom[(i*4 + mu)*BLOCK + lane].  The lane index is laundered on every use,
// so loads of different uses are never merged and no momentum stays in a
// register between uses (a sum is read again where it is needed).
__device__ __forceinline__ int fresh_lane(int lane) {
  asm volatile("" : "+v"(lane));
  return lane;
}
template <unsigned MASK, unsigned INMASK, int NEXT, int BLOCK>
__device__ __forceinline__ void flow_momentum_lds(double out[4], const double* smom, int lane) {
  const int l = fresh_lane(lane);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NEXT; ++i)
      if (MASK & (1u << i)) {
        const double x = smom[(i * 4 + mu) * BLOCK + l];
        acc = (INMASK & (1u << i)) ? acc + x : acc - x;
      }
    out[mu] = acc;
  }
}
template <int BLOCK>
__device__ __forceinline__ void load_mom_lds(double out[4], const double* smom, int lane, int i) {
  const int l = fresh_lane(lane);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) out[mu] = smom[(i * 4 + mu) * BLOCK + l];
}

// Split form for software pipelining: the LDS loads of the legs in MASK into
// registers (one laundered lane index), issued ahead of a scheduling barrier,
// and their signed sum, which the scheduler places after it.  The sum takes
// the legs in the same order and with the same operations as
// flow_momentum_lds, so both give the same bits.
template <unsigned MASK, int NEXT, int BLOCK>
__device__ __forceinline__ void load_legs_lds(double (&r)[NEXT][4], const double* smom, int lane) {
  const int l = fresh_lane(lane);
#pragma unroll
  for (int i = 0; i < NEXT; ++i)
    if (MASK & (1u << i))
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) r[i][mu] = smom[(i * 4 + mu) * BLOCK + l];
}
// One per-event propagator denominator staged per lane in LDS, at
// s[k*BLOCK + lane] (laundered lane index, like the momenta).
template <int BLOCK> __device__ __forceinline__ double load_den_lds(const double* s, int k, int lane) {
  return s[k * BLOCK + fresh_lane(lane)];
}
// The barrier between the two, in FP64 only: there one wave per SIMD leaves
// the load latency exposed unless the loads are issued early, while the FP32
// kernels run two waves per SIMD and would lose the second one to the longer
// live ranges.
template <typename T> __device__ __forceinline__ void pf_barrier() {
  if constexpr (sizeof(T) == 8) __builtin_amdgcn_sched_barrier(0);
}
// Kinematics of one event shared by the lanes that evaluate its helicities:
// row k of the block's table holds a momentum sum as T[4] at
// s[(k*EVB + col)*4 + mu] (one contiguous 16- or 32-byte load), or a
// propagator denominator at s[k*EVB + col]; col is the event's column in the
// block, laundered like the lane index above.
template <typename T, int EVB>
__device__ __forceinline__ void load_kin_lds(T out[4], const T* s, int k, int col) {
  const T* p = s + (k * EVB + fresh_lane(col)) * 4;
  out[0] = p[0]; out[1] = p[1]; out[2] = p[2]; out[3] = p[3];
}
// The same with one load per component: four 4-byte loads instead of one
// 16-byte load into an aligned register quad, which leaves the register
// allocator more freedom where a kernel is held to 256 registers.
template <typename T, int EVB>
__device__ __forceinline__ void load_kin_lds1(T out[4], const T* s, int k, int col) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) out[mu] = s[(k * EVB + fresh_lane(col)) * 4 + mu];
}
template <typename T, int EVB> __device__ __forceinline__ T load_tden_lds(const T* s, int k, int col) {
  return s[k * EVB + fresh_lane(col)];
}
// Forces x to be computed here, in every lane, before code that only some
// lanes run (a store), instead of inside that code.
template <typename V> __device__ __forceinline__ void pin(V& x) { asm volatile("" : "+v"(x)); }
template <unsigned MASK, unsigned INMASK, int NEXT>
__device__ __forceinline__ void sum_legs(double out[4], const double (&r)[NEXT][4]) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NEXT; ++i)
      if (MASK & (1u << i)) acc = (INMASK & (1u << i)) ? acc + r[i][mu] : acc - r[i][mu];
    out[mu] = acc;
  }
}

// External wavefunctions staged per lane in LDS: the eight real components
// of leg i at s[(i*8 + k)*NL + lane].  Each use loads them again through a
// laundered lane index, so none stays in registers between uses.
template <typename T, int NL>
__device__ __forceinline__ void store_wf_lds(T* s, int i, int lane, const wf<T>& w) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    s[(i * 8 + 2 * c) * NL + lane] = w.c[c].re;
    s[(i * 8 + 2 * c + 1) * NL + lane] = w.c[c].im;
  }
}
template <typename T, int NL> __device__ __forceinline__ wf<T> load_wf_lds(const T* s, int i, int lane) {
  const int l = fresh_lane(lane);
  wf<T> w;
#pragma unroll
  for (int c = 0; c < 4; ++c) w.c[c] = mk<T>(s[(i * 8 + 2 * c) * NL + l], s[(i * 8 + 2 * c + 1) * NL + l]);
  return w;
}
// A polarisation vector: time component zero, z component real.
template <typename T, int NL> __device__ __forceinline__ wf<T> load_pol_lds(const T* s, int i, int lane) {
  const int l = fresh_lane(lane);
  wf<T> w;
  w.c[0] = mk<T>((T)0, (T)0);
  w.c[1] = mk<T>(s[(i * 8 + 2) * NL + l], s[(i * 8 + 3) * NL + l]);
  w.c[2] = mk<T>(s[(i * 8 + 4) * NL + l], s[(i * 8 + 5) * NL + l]);
  w.c[3] = mk<T>(s[(i * 8 + 6) * NL + l], (T)0);
  return w;
}

template <typename T> __device__ __forceinline__ void to_t(T out[4], const double in[4]) {
  out[0] = (T)in[0]; out[1] = (T)in[1]; out[2] = (T)in[2]; out[3] = (T)in[3];
}

// 1 / (P^2 - m^2) in double precision: the hardware reciprocal refined by
// two Newton-Raphson steps y <- y + y (1 - x y), within an ulp or two of the
// correctly rounded quotient for the normal-range denominators of these
// propagators (the IEEE division sequence takes twice the instructions).
__device__ __forceinline__ double inv_virt(const double P[4], double m) {
  const double x = P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3] - m * m;
  double y = __builtin_amdgcn_rcp(x);
  double r = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, r, y);
  r = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, r, y);
}

}  // namespace mgme
