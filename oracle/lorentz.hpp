// Oracle (test infrastructure only): explicit Dirac algebra, external states
// and Minkowski products, templated on the real type so that the same code
// runs in double and in long double.
//
// Conventions (textbook, Peskin & Schroeder): metric diag(+,-,-,-); chiral
// (Weyl) representation gamma^0 = [[0,1],[1,0]], gamma^k = [[0,s_k],[-s_k,0]],
// gamma^5 = diag(-1,-1,1,1), so that the upper two components are
// left-handed.  Helicity spinors:
//   u(p,l) = ( sqrt(E - l|p|) chi_l , sqrt(E + l|p|) chi_l ),
//   v(p,l) = ( -l sqrt(E + l|p|) chi_{-l} , l sqrt(E - l|p|) chi_{-l} ),
// where chi_l is the two-component helicity eigenvector along p, with the
// phase chi_+ = (0,1), chi_- = (-1,0) for p along -z.  Polarisation vector of
// a massless vector boson with helicity l:
//   eps(k,l) = ( -l e1 - i e2 ) / sqrt(2),
//   e1 = (0, cos(th)cos(ph), cos(th)sin(ph), -sin(th)), e2 = (0, -sin(ph), cos(ph), 0),
// with ph = 0 for k along the z axis.  These are the helicity amplitudes the
// paper's matrix elements are built from (section 1).
#pragma once
#include <array>
#include <cmath>
#include <complex>

namespace oracle {

template <class R> using cplx = std::complex<R>;
template <class R> using Vec4 = std::array<cplx<R>, 4>;  // contravariant components
template <class R> using Spin = std::array<cplx<R>, 4>;  // ket column or bra row
template <class R> using Mat4 = std::array<std::array<cplx<R>, 4>, 4>;

template <class R> inline R metric(int mu) { return mu == 0 ? R(1) : R(-1); }

template <class R> inline cplx<R> mdot(const Vec4<R>& a, const Vec4<R>& b) {
  return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

template <class R> inline Vec4<R> real_vec(const R p[4]) {
  return {cplx<R>(p[0]), cplx<R>(p[1]), cplx<R>(p[2]), cplx<R>(p[3])};
}

// gamma^mu in the chiral representation.
template <class R> Mat4<R> gamma(int mu) {
  Mat4<R> g{};
  const cplx<R> one(1), I(0, 1);
  if (mu == 0) {
    g[0][2] = g[1][3] = g[2][0] = g[3][1] = one;
  } else {
    // sigma^k blocks
    cplx<R> s[2][2];
    if (mu == 1) { s[0][0] = 0; s[0][1] = one; s[1][0] = one; s[1][1] = 0; }
    if (mu == 2) { s[0][0] = 0; s[0][1] = -I; s[1][0] = I; s[1][1] = 0; }
    if (mu == 3) { s[0][0] = one; s[0][1] = 0; s[1][0] = 0; s[1][1] = -one; }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        g[a][2 + b] = s[a][b];
        g[2 + a][b] = -s[a][b];
      }
  }
  return g;
}

template <class R> Mat4<R> gamma5() {
  Mat4<R> g{};
  g[0][0] = g[1][1] = cplx<R>(-1);
  g[2][2] = g[3][3] = cplx<R>(1);
  return g;
}

// a-slash = gamma^mu a_mu = sum_mu g_{mu mu} a^mu gamma^mu
template <class R> Mat4<R> slash(const Vec4<R>& a) {
  Mat4<R> m{};
  for (int mu = 0; mu < 4; ++mu) {
    const Mat4<R> g = gamma<R>(mu);
    const cplx<R> c = metric<R>(mu) * a[mu];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) m[i][j] += c * g[i][j];
  }
  return m;
}

template <class R> Mat4<R> identity4() {
  Mat4<R> m{};
  for (int i = 0; i < 4; ++i) m[i][i] = cplx<R>(1);
  return m;
}

template <class R> Mat4<R> matmul(const Mat4<R>& a, const Mat4<R>& b) {
  Mat4<R> m{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 4; ++k) m[i][j] += a[i][k] * b[k][j];
  return m;
}

template <class R> Mat4<R> matadd(const Mat4<R>& a, const Mat4<R>& b) {
  Mat4<R> m{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = a[i][j] + b[i][j];
  return m;
}

template <class R> Mat4<R> matscale(const Mat4<R>& a, cplx<R> c) {
  Mat4<R> m{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = c * a[i][j];
  return m;
}

template <class R> Spin<R> matvec(const Mat4<R>& a, const Spin<R>& x) {
  Spin<R> y{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) y[i] += a[i][j] * x[j];
  return y;
}

template <class R> Spin<R> vecmat(const Spin<R>& x, const Mat4<R>& a) {
  Spin<R> y{};
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) y[j] += x[i] * a[i][j];
  return y;
}

template <class R> cplx<R> braket(const Spin<R>& bra, const Spin<R>& ket) {
  cplx<R> s(0);
  for (int i = 0; i < 4; ++i) s += bra[i] * ket[i];
  return s;
}

// Dirac adjoint: bar(psi) = psi^dagger gamma^0, as a row spinor.
template <class R> Spin<R> dirac_bar(const Spin<R>& psi) {
  const Mat4<R> g0 = gamma<R>(0);
  Spin<R> row{};
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) row[j] += std::conj(psi[i]) * g0[i][j];
  return row;
}

// Two-component helicity eigenvectors chi_l(p) with sigma.p chi_l = l |p| chi_l.
template <class R> void helicity_chi(const R p[4], int l, cplx<R> chi[2]) {
  const R px = p[1], py = p[2], pz = p[3];
  const R pabs = std::sqrt(px * px + py * py + pz * pz);
  if (px == 0 && py == 0 && pz < 0) {  // p along -z: fixed phase
    if (l > 0) { chi[0] = 0; chi[1] = 1; }
    else { chi[0] = -1; chi[1] = 0; }
    return;
  }
  // |p| + pz without cancellation for pz < 0
  const R ppz = pz >= 0 ? pabs + pz : (px * px + py * py) / (pabs - pz);
  const R norm = R(1) / std::sqrt(R(2) * pabs * ppz);
  if (l > 0) {
    chi[0] = cplx<R>(ppz * norm, 0);
    chi[1] = cplx<R>(px * norm, py * norm);
  } else {
    chi[0] = cplx<R>(-px * norm, py * norm);
    chi[1] = cplx<R>(ppz * norm, 0);
  }
}

// sqrt(E - l|p|) and sqrt(E + l|p|) for a particle of mass m, computed without
// cancellation; for m == 0 the energy is taken as |p|.
template <class R> void spinor_weights(const R p[4], R m, int l, R& w_minus, R& w_plus) {
  const R pabs = std::sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  R e = m == 0 ? pabs : std::sqrt(pabs * pabs + m * m);
  const R big = std::sqrt(e + pabs);
  const R small = m == 0 ? R(0) : m / big;  // sqrt(E-|p|) = m / sqrt(E+|p|)
  if (l > 0) { w_minus = small; w_plus = big; }
  else { w_minus = big; w_plus = small; }
}

template <class R> Spin<R> spinor_u(const R p[4], R m, int l) {
  cplx<R> chi[2];
  helicity_chi(p, l, chi);
  R wm, wp;  // sqrt(E - l|p|), sqrt(E + l|p|)
  spinor_weights(p, m, l, wm, wp);
  return {wm * chi[0], wm * chi[1], wp * chi[0], wp * chi[1]};
}

template <class R> Spin<R> spinor_v(const R p[4], R m, int l) {
  cplx<R> chi[2];
  helicity_chi(p, -l, chi);
  R wm, wp;  // sqrt(E - l|p|), sqrt(E + l|p|)
  spinor_weights(p, m, l, wm, wp);
  const R sl = l > 0 ? R(1) : R(-1);
  return {-sl * wp * chi[0], -sl * wp * chi[1], sl * wm * chi[0], sl * wm * chi[1]};
}

template <class R> Vec4<R> polarisation(const R p[4], int l) {
  const R px = p[1], py = p[2], pz = p[3];
  const R pt = std::sqrt(px * px + py * py);
  const R pabs = std::sqrt(px * px + py * py + pz * pz);
  const R ct = pz / pabs, st = pt / pabs;
  R cp = 1, sp = 0;
  if (pt > 0) { cp = px / pt; sp = py / pt; }
  const R lam = l > 0 ? R(1) : R(-1);
  const R r2 = R(1) / std::sqrt(R(2));
  const cplx<R> I(0, 1);
  Vec4<R> e1 = {cplx<R>(0), cplx<R>(ct * cp), cplx<R>(ct * sp), cplx<R>(-st)};
  Vec4<R> e2 = {cplx<R>(0), cplx<R>(-sp), cplx<R>(cp), cplx<R>(0)};
  Vec4<R> eps;
  for (int mu = 0; mu < 4; ++mu) eps[mu] = r2 * (-lam * e1[mu] - I * e2[mu]);
  return eps;
}

template <class R> Vec4<R> conj4(const Vec4<R>& a) {
  return {std::conj(a[0]), std::conj(a[1]), std::conj(a[2]), std::conj(a[3])};
}

}  // namespace oracle
