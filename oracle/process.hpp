// Oracle (test infrastructure only): tree-level |M|^2 by explicit Feynman
// diagrams.  Each diagram is built from the Feynman rules, evaluated with
// explicit 4x4 Dirac matrices for every helicity configuration, dressed with
// its explicit colour tensor, squared and summed over helicities and colours
// (the paper computes the matrix element "from Feynman diagrams and helicity
// amplitudes", section 1; its "color algebra" is the part named in
// section 3).
//
// Feynman rules (Peskin & Schroeder, all vertex momenta incoming):
//   quark-gluon      i gs gamma^mu T^a
//   three-gluon      gs f^abc [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
//   four-gluon       -i gs^2 [ f^abe f^cde (g^{mu rho} g^{nu sig} - g^{mu sig} g^{nu rho})
//                            + f^ace f^bde (g^{mu nu} g^{rho sig} - g^{mu sig} g^{nu rho})
//                            + f^ade f^bce (g^{mu nu} g^{rho sig} - g^{mu rho} g^{nu sig}) ]
//   fermion-photon   -i e Q gamma^mu
//   fermion-Z        -i e/(sw cw) gamma^mu (gL PL + gR PR),  gL = T3 - Q sw^2, gR = -Q sw^2
//   quark propagator i (qslash + m) / (q^2 - m^2)         (top width zero)
//   gluon/photon     -i g_{mu nu} / q^2
//   Z                -i (g_{mu nu} - q_mu q_nu / mZ^2) / (q^2 - mZ^2 + i mZ GZ)
//
// Returned |M|^2 is averaged over initial helicities and colours and divided
// by the number of permutations of identical final-state gluons.
#pragma once
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "colour.hpp"
#include "lorentz.hpp"

namespace oracle {

struct Params {
  double alpha_s, alpha_em, sin2w, mz, wz, mt, wt;
  int z_enabled;
};

enum NodeKind { LEAF = 0, GGG = 1, GGGG = 2 };

struct GNode {
  int kind;
  int leg;       // external leg of a leaf
  int ch[3];     // children (two for GGG, three for GGGG)
  uint32_t mask; // external legs below this node
};

// One term of one diagram: the diagram's gluon trees attached along the quark
// line, plus one of the three colour/Lorentz structures for every four-gluon
// vertex of the diagram.  A diagram without four-gluon vertices has one term.
struct Term {
  int diagram;
  std::vector<int> roots;                  // from the quark (bra) end to the antiquark (ket) end
  std::vector<std::pair<int, int>> choice; // (four-gluon node, structure 0..2)
  int boson;                               // e+e- -> mu+mu-: 0 photon, 1 Z
};

inline int popcount32(uint32_t x) { return __builtin_popcount(x); }

class Process {
 public:
  enum Kind { EE_MUMU = 0, GG_TT_NG = 1 };
  int kind = 0;
  int n_ext = 0;
  std::vector<int> pdg;
  std::vector<bool> incoming;
  std::vector<double> mass;
  std::vector<int> gluon_legs;
  int quark_leg = -1, antiquark_leg = -1;
  std::vector<GNode> pool;
  std::vector<Term> terms;
  int n_diagrams = 0;
  // colour
  int ncol = 1;
  std::vector<std::vector<int>> basis;  // each flow: a permutation of the gluon legs
  std::vector<long long> cnum;          // colour matrix numerators, ncol*ncol
  long long cden = 1;                   // common denominator
  std::vector<std::vector<std::pair<int, std::complex<long long>>>> coef;  // per term
  Params par{};
  double norm = 1.0;
  int n_hel = 0;

  Process(int n, const int* pdg_in, const Params& p) : n_ext(n), pdg(pdg_in, pdg_in + n), par(p) {
    if (p.wt != 0.0) throw std::invalid_argument("top width must be zero");
    n_hel = 1 << n_ext;
    if (n == 4 && pdg[0] == -11 && pdg[1] == 11 && pdg[2] == -13 && pdg[3] == 13) {
      kind = EE_MUMU;
      incoming = {true, true, false, false};
      mass = {0, 0, 0, 0};
      terms.push_back(Term{0, {}, {}, 0});
      n_diagrams = 1;
      if (p.z_enabled) {
        terms.push_back(Term{1, {}, {}, 1});
        n_diagrams = 2;
      }
      ncol = 1;
      basis = {{}};
      cnum = {1};
      cden = 1;
      coef = std::vector<std::vector<std::pair<int, std::complex<long long>>>>(
          terms.size(), {{0, std::complex<long long>(1, 0)}});
      norm = 1.0 / 4.0;
      return;
    }
    if (n >= 4 && n <= 7 && pdg[0] == 21 && pdg[1] == 21 && pdg[2] == 6 && pdg[3] == -6) {
      for (int i = 4; i < n; ++i)
        if (pdg[i] != 21) throw std::invalid_argument("unsupported process");
      kind = GG_TT_NG;
      for (int i = 0; i < n; ++i) {
        incoming.push_back(i < 2);
        mass.push_back((i == 2 || i == 3) ? p.mt : 0.0);
        if (pdg[i] == 21) gluon_legs.push_back(i);
      }
      quark_leg = 2;
      antiquark_leg = 3;
      enumerate_diagrams();
      build_colour();
      double fact = 1.0;
      for (int k = 2; k <= n - 4; ++k) fact *= k;
      norm = 1.0 / (4.0 * 64.0 * fact);
      return;
    }
    throw std::invalid_argument("unsupported process");
  }

  // ---------------------------------------------------------------- diagrams
  std::map<uint32_t, std::vector<int>> memo;

  int new_node(int kind_, int leg, int a, int b, int c, uint32_t mask) {
    pool.push_back(GNode{kind_, leg, {a, b, c}, mask});
    return (int)pool.size() - 1;
  }

  // All gluon trees (three- and four-gluon vertices) joining the legs in mask
  // into one off-shell gluon.
  const std::vector<int>& trees(uint32_t mask) {
    auto it = memo.find(mask);
    if (it != memo.end()) return it->second;
    std::vector<int> out;
    if (popcount32(mask) == 1) {
      out.push_back(new_node(LEAF, __builtin_ctz(mask), -1, -1, -1, mask));
    } else {
      const uint32_t low = mask & (~mask + 1u);
      const uint32_t rest = mask ^ low;
      std::vector<uint32_t> subs;  // all subsets of rest
      for (uint32_t s = rest;; s = (s - 1) & rest) {
        subs.push_back(s);
        if (s == 0) break;
      }
      for (uint32_t s : subs) {  // unordered pairs {A, B}, A holds the lowest leg
        const uint32_t A = low | s, B = mask ^ A;
        if (B == 0) continue;
        const std::vector<int> ta = trees(A), tb = trees(B);
        for (int x : ta)
          for (int y : tb) out.push_back(new_node(GGG, -1, x, y, -1, mask));
      }
      for (uint32_t s : subs) {  // unordered triples {A, B, C}
        const uint32_t A = low | s, Rm = mask ^ A;
        if (Rm == 0) continue;
        const uint32_t low2 = Rm & (~Rm + 1u), rest2 = Rm ^ low2;
        for (uint32_t s2 = rest2;; s2 = (s2 - 1) & rest2) {
          const uint32_t B = low2 | s2, Cm = Rm ^ B;
          if (Cm != 0) {
            const std::vector<int> ta = trees(A), tb = trees(B), tc = trees(Cm);
            for (int x : ta)
              for (int y : tb)
                for (int z : tc) out.push_back(new_node(GGGG, -1, x, y, z, mask));
          }
          if (s2 == 0) break;
        }
      }
    }
    memo[mask] = out;
    return memo[mask];
  }

  void collect_gggg(int node, std::vector<int>& out) const {
    const GNode& g = pool[node];
    if (g.kind == GGGG) out.push_back(node);
    if (g.kind == GGG || g.kind == GGGG)
      for (int c = 0; c < (g.kind == GGG ? 2 : 3); ++c) collect_gggg(g.ch[c], out);
  }

  void enumerate_diagrams() {
    uint32_t all = 0;
    for (int l : gluon_legs) all |= 1u << l;
    std::vector<uint32_t> blocks;
    std::function<void(uint32_t)> part = [&](uint32_t remaining) {
      if (remaining == 0) {
        // cartesian product of the trees of each block
        std::vector<std::vector<int>> choices;
        for (uint32_t b : blocks) choices.push_back(trees(b));
        std::vector<int> idx(blocks.size(), 0);
        while (true) {
          std::vector<int> roots;
          for (size_t m = 0; m < blocks.size(); ++m) roots.push_back(choices[m][idx[m]]);
          add_diagram(roots);
          size_t m = 0;
          while (m < blocks.size()) {
            if (++idx[m] < (int)choices[m].size()) break;
            idx[m] = 0;
            ++m;
          }
          if (m == blocks.size()) break;
        }
        return;
      }
      for (uint32_t s = remaining; s != 0; s = (s - 1) & remaining) {
        blocks.push_back(s);
        part(remaining ^ s);
        blocks.pop_back();
      }
    };
    part(all);
  }

  void add_diagram(const std::vector<int>& roots) {
    std::vector<int> g4;
    for (int r : roots) collect_gggg(r, g4);
    int nterm = 1;
    for (size_t i = 0; i < g4.size(); ++i) nterm *= 3;
    for (int t = 0; t < nterm; ++t) {
      Term term;
      term.diagram = n_diagrams;
      term.roots = roots;
      term.boson = -1;
      int x = t;
      for (int node : g4) {
        term.choice.push_back({node, x % 3});
        x /= 3;
      }
      terms.push_back(term);
    }
    ++n_diagrams;
  }

  // ------------------------------------------------------------------ colour
  // Colour tensor of a gluon tree node for fixed external gluon colours:
  // an 8-vector over the adjoint index of the node's upper line.
  std::array<double, 8> node_colour(int node, const Term& term, const int* acol) const {
    const ColourTables& ct = colour_tables();
    const GNode& g = pool[node];
    std::array<double, 8> K{};
    if (g.kind == LEAF) {
      K[acol[g.leg]] = 1.0;
      return K;
    }
    if (g.kind == GGG) {
      const auto A = node_colour(g.ch[0], term, acol);
      const auto B = node_colour(g.ch[1], term, acol);
      for (int b = 0; b < 8; ++b) {
        if (A[b] == 0) continue;
        for (int c = 0; c < 8; ++c) {
          if (B[c] == 0) continue;
          for (int e = 0; e < 8; ++e) K[e] += ct.f[b][c][e] * A[b] * B[c];
        }
      }
      return K;
    }
    int s = -1;
    for (auto& pc : term.choice)
      if (pc.first == node) s = pc.second;
    const auto A = node_colour(g.ch[0], term, acol);
    const auto B = node_colour(g.ch[1], term, acol);
    const auto C = node_colour(g.ch[2], term, acol);
    for (int a = 0; a < 8; ++a) {
      if (A[a] == 0) continue;
      for (int b = 0; b < 8; ++b) {
        if (B[b] == 0) continue;
        for (int c = 0; c < 8; ++c) {
          if (C[c] == 0) continue;
          const double w = A[a] * B[b] * C[c];
          for (int d = 0; d < 8; ++d)
            for (int e = 0; e < 8; ++e) {
              double v = 0;
              if (s == 0) v = ct.f[a][b][e] * ct.f[c][d][e];
              if (s == 1) v = ct.f[a][c][e] * ct.f[b][d][e];
              if (s == 2) v = ct.f[a][d][e] * ct.f[b][c][e];
              K[d] += v * w;
            }
        }
      }
    }
    return K;
  }

  // Colour factor of a term for external colours: gluon colours acol[leg],
  // quark colour i (outgoing top), anticolour j (outgoing antitop).
  cd term_colour(const Term& term, const int* acol, int i, int j) const {
    if (kind == EE_MUMU) return cd(1, 0);
    const ColourTables& ct = colour_tables();
    Mat3 M = mat3_identity();
    for (int r : term.roots) {
      const auto K = node_colour(r, term, acol);
      Mat3 X{};
      for (int x = 0; x < 8; ++x)
        if (K[x] != 0)
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) X[p][q] += K[x] * ct.T[x][p][q];
      M = mat3_mul(M, X);
    }
    return M[i][j];
  }

  // Trace-basis element (T^{a_{s1}} ... T^{a_{sk}})_{ij}.
  cd basis_value(int flow, const int* acol, int i, int j) const {
    const ColourTables& ct = colour_tables();
    Mat3 M = mat3_identity();
    for (int leg : basis[flow]) M = mat3_mul(M, ct.T[acol[leg]]);
    return M[i][j];
  }

  static bool solve_hpd(std::vector<cd> G, std::vector<cd>& x, int n) {
    // Gaussian elimination with partial pivoting, G is n x n, x holds n right sides
    // stored as columns of an n x m block; here m = x.size()/n.
    const int m = (int)x.size() / n;
    for (int col = 0; col < n; ++col) {
      int piv = col;
      for (int r = col + 1; r < n; ++r)
        if (std::abs(G[r * n + col]) > std::abs(G[piv * n + col])) piv = r;
      if (std::abs(G[piv * n + col]) < 1e-12) return false;
      if (piv != col) {
        for (int c = 0; c < n; ++c) std::swap(G[col * n + c], G[piv * n + c]);
        for (int c = 0; c < m; ++c) std::swap(x[col * m + c], x[piv * m + c]);
      }
      for (int r = 0; r < n; ++r) {
        if (r == col) continue;
        const cd fac = G[r * n + col] / G[col * n + col];
        if (fac == cd(0)) continue;
        for (int c = col; c < n; ++c) G[r * n + c] -= fac * G[col * n + c];
        for (int c = 0; c < m; ++c) x[r * m + c] -= fac * x[col * m + c];
      }
    }
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < m; ++c) x[r * m + c] /= G[r * n + r];
    return true;
  }

  void build_colour() {
    const int k = (int)gluon_legs.size();
    // basis: all orderings of the gluon legs, lexicographic
    std::vector<int> perm = gluon_legs;
    std::sort(perm.begin(), perm.end());
    do basis.push_back(perm);
    while (std::next_permutation(perm.begin(), perm.end()));
    ncol = (int)basis.size();
    // Colour matrix C_st = sum over all colours of conj(V_s) V_t, brute force.
    std::vector<cd> C((size_t)ncol * ncol, cd(0));
    int acol[8] = {0};
    long long nconf = 1;
    for (int i = 0; i < k; ++i) nconf *= 8;
    const ColourTables& ct = colour_tables();
    std::vector<Mat3> P(ncol);
    const bool full = k <= 4;  // full Gram; for k = 5 only the first row
    for (long long c = 0; c < nconf; ++c) {
      long long x = c;
      for (int i = 0; i < k; ++i) {
        acol[gluon_legs[i]] = (int)(x % 8);
        x /= 8;
      }
      for (int s = 0; s < ncol; ++s) {
        Mat3 M = mat3_identity();
        for (int leg : basis[s]) M = mat3_mul(M, ct.T[acol[leg]]);
        P[s] = M;
      }
      for (int s = 0; s < (full ? ncol : 1); ++s)
        for (int t = 0; t < ncol; ++t) {
          cd acc = 0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc += std::conj(P[s][i][j]) * P[t][i][j];
          C[(size_t)s * ncol + t] += acc;
        }
    }
    if (!full) {
      // The sum over all colour labels is invariant under relabelling the
      // gluons, so C_st = C_{id, s^-1 t}.
      std::map<std::vector<int>, int> index;
      for (int s = 0; s < ncol; ++s) index[basis[s]] = s;
      const std::vector<int>& id = basis[0];
      for (int s = 1; s < ncol; ++s)
        for (int t = 0; t < ncol; ++t) {
          // relative ordering: positions of basis[t] legs within basis[s]
          std::vector<int> rel(k);
          for (int m = 0; m < k; ++m) {
            const int pos = (int)(std::find(basis[s].begin(), basis[s].end(), basis[t][m]) -
                                  basis[s].begin());
            rel[m] = id[pos];
          }
          C[(size_t)s * ncol + t] = C[index[rel]];
        }
    }
    // exact rational form: smallest denominator making every entry integral
    cden = 0;
    for (long long d = 1; d <= 100000 && cden == 0; ++d) {
      bool ok = true;
      for (const cd& v : C) {
        const double y = v.real() * (double)d;
        if (std::fabs(y - std::round(y)) > 1e-6 || std::fabs(v.imag()) > 1e-9) {
          ok = false;
          break;
        }
      }
      if (ok) cden = d;
    }
    if (cden == 0) throw std::runtime_error("colour matrix is not rational");
    cnum.resize((size_t)ncol * ncol);
    for (size_t i = 0; i < C.size(); ++i) cnum[i] = std::llround(C[i].real() * (double)cden);
    project_terms();
  }

  // Decomposition of every term's colour tensor on the trace basis, found by
  // least squares on sampled colour assignments, rounded to Gaussian integers
  // and verified on an independent sample.
  void project_terms() {
    const int k = (int)gluon_legs.size();
    const int nt = (int)terms.size();
    uint64_t rng = 0x9E3779B97F4A7C15ull;
    auto next = [&]() {
      rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
      return rng;
    };
    auto sample = [&](int nsamp, std::vector<cd>& V, std::vector<cd>& K) {
      V.assign((size_t)nsamp * ncol, cd(0));
      K.assign((size_t)nsamp * nt, cd(0));
      int acol[8] = {0};
      for (int r = 0; r < nsamp; ++r) {
        for (int m = 0; m < k; ++m) acol[gluon_legs[m]] = (int)(next() % 8);
        const int i = (int)(next() % 3), j = (int)(next() % 3);
        for (int s = 0; s < ncol; ++s) V[(size_t)r * ncol + s] = basis_value(s, acol, i, j);
        for (int t = 0; t < nt; ++t) K[(size_t)r * nt + t] = term_colour(terms[t], acol, i, j);
      }
    };
    const int ns = 8 * ncol + 64;
    std::vector<cd> V, K;
    sample(ns, V, K);
    std::vector<cd> G((size_t)ncol * ncol, cd(0));
    std::vector<cd> B((size_t)ncol * nt, cd(0));
    for (int r = 0; r < ns; ++r)
      for (int s = 0; s < ncol; ++s) {
        const cd vs = std::conj(V[(size_t)r * ncol + s]);
        if (vs == cd(0)) continue;
        for (int t = 0; t < ncol; ++t) G[(size_t)s * ncol + t] += vs * V[(size_t)r * ncol + t];
        for (int t = 0; t < nt; ++t) B[(size_t)s * nt + t] += vs * K[(size_t)r * nt + t];
      }
    if (!solve_hpd(G, B, ncol)) throw std::runtime_error("colour projection is singular");
    coef.assign(nt, {});
    for (int t = 0; t < nt; ++t)
      for (int s = 0; s < ncol; ++s) {
        const cd c = B[(size_t)s * nt + t];
        const long long re = std::llround(c.real()), im = std::llround(c.imag());
        if (std::fabs(c.real() - re) > 1e-6 || std::fabs(c.imag() - im) > 1e-6)
          throw std::runtime_error("colour coefficient is not a Gaussian integer");
        if (re != 0 || im != 0) coef[t].push_back({s, std::complex<long long>(re, im)});
      }
    // verification on a fresh sample
    sample(2 * ncol + 64, V, K);
    const int nv = 2 * ncol + 64;
    for (int r = 0; r < nv; ++r)
      for (int t = 0; t < nt; ++t) {
        cd acc = 0;
        for (auto& sc : coef[t])
          acc += cd((double)sc.second.real(), (double)sc.second.imag()) * V[(size_t)r * ncol + sc.first];
        if (std::abs(acc - K[(size_t)r * nt + t]) > 1e-10)
          throw std::runtime_error("colour decomposition does not reproduce the tensor");
      }
  }

  // --------------------------------------------------------------- kinematics
  template <class R> struct Event {
    R p[8][4];   // physical momenta
    R pin[8][4]; // momenta flowing into the diagram
  };

  template <class R> Event<R> make_event(const double* mom) const {
    Event<R> ev;
    for (int i = 0; i < n_ext; ++i)
      for (int mu = 0; mu < 4; ++mu) {
        ev.p[i][mu] = (R)mom[4 * i + mu];
        ev.pin[i][mu] = incoming[i] ? ev.p[i][mu] : -ev.p[i][mu];
      }
    return ev;
  }

  static int hel_of(int h, int leg, int n) { return ((h >> (n - 1 - leg)) & 1) ? 1 : -1; }

  // ----------------------------------------------------------- Lorentz parts
  template <class R> struct Current {
    Vec4<R> J;
    R P[4];
  };

  template <class R>
  Current<R> node_current(int node, const Term& term, const Event<R>& ev, const Vec4<R>* pol) const {
    const GNode& g = pool[node];
    const R gs = std::sqrt(R(4) * R(3.141592653589793238462643383279502884L) * (R)par.alpha_s);
    const cplx<R> I(0, 1);
    Current<R> out;
    if (g.kind == LEAF) {
      out.J = pol[g.leg];
      for (int mu = 0; mu < 4; ++mu) out.P[mu] = ev.pin[g.leg][mu];
      return out;
    }
    if (g.kind == GGG) {
      const Current<R> a = node_current(g.ch[0], term, ev, pol);
      const Current<R> b = node_current(g.ch[1], term, ev, pol);
      R k[4], p[4], q[4];
      for (int mu = 0; mu < 4; ++mu) {
        k[mu] = a.P[mu];
        p[mu] = b.P[mu];
        q[mu] = -(a.P[mu] + b.P[mu]);
        out.P[mu] = a.P[mu] + b.P[mu];
      }
      Vec4<R> kmp, pmq, qmk;
      for (int mu = 0; mu < 4; ++mu) {
        kmp[mu] = k[mu] - p[mu];
        pmq[mu] = p[mu] - q[mu];
        qmk[mu] = q[mu] - k[mu];
      }
      const cplx<R> ab = mdot(a.J, b.J), pa = mdot(pmq, a.J), qb = mdot(qmk, b.J);
      const R P2 = out.P[0] * out.P[0] - out.P[1] * out.P[1] - out.P[2] * out.P[2] - out.P[3] * out.P[3];
      const cplx<R> fac = gs * (-I / P2);
      for (int mu = 0; mu < 4; ++mu) out.J[mu] = fac * (ab * kmp[mu] + b.J[mu] * pa + a.J[mu] * qb);
      return out;
    }
    int s = -1;
    for (auto& pc : term.choice)
      if (pc.first == node) s = pc.second;
    const Current<R> a = node_current(g.ch[0], term, ev, pol);
    const Current<R> b = node_current(g.ch[1], term, ev, pol);
    const Current<R> c = node_current(g.ch[2], term, ev, pol);
    for (int mu = 0; mu < 4; ++mu) out.P[mu] = a.P[mu] + b.P[mu] + c.P[mu];
    const R P2 = out.P[0] * out.P[0] - out.P[1] * out.P[1] - out.P[2] * out.P[2] - out.P[3] * out.P[3];
    const cplx<R> ab = mdot(a.J, b.J), ac = mdot(a.J, c.J), bc = mdot(b.J, c.J);
    const cplx<R> fac = (-I * gs * gs) * (-I / P2);
    for (int mu = 0; mu < 4; ++mu) {
      cplx<R> L;
      if (s == 0) L = ac * b.J[mu] - a.J[mu] * bc;
      else if (s == 1) L = ab * c.J[mu] - a.J[mu] * bc;
      else L = ab * c.J[mu] - ac * b.J[mu];
      out.J[mu] = fac * L;
    }
    return out;
  }

  // Lorentz part (i times the amplitude, colour stripped) of every term for
  // one helicity configuration.  pol_override: leg whose polarisation is
  // replaced by its momentum (gauge test), or -1.
  template <class R>
  void term_amplitudes(const Event<R>& ev, int h, int pol_override, std::vector<cplx<R>>& amp) const {
    const cplx<R> I(0, 1);
    amp.assign(terms.size(), cplx<R>(0));
    if (kind == EE_MUMU) {
      const R pi = R(3.141592653589793238462643383279502884L);
      const R e = std::sqrt(R(4) * pi * (R)par.alpha_em);
      const R sw2 = (R)par.sin2w, cw2 = R(1) - sw2;
      const R gz = e / std::sqrt(sw2 * cw2);
      const R Q = -1, T3 = R(-0.5);
      const R gL = T3 - Q * sw2, gR = -Q * sw2;
      const Spin<R> bra_e = dirac_bar(spinor_v<R>(ev.p[0], 0, hel_of(h, 0, 4)));
      const Spin<R> ket_e = spinor_u<R>(ev.p[1], 0, hel_of(h, 1, 4));
      const Spin<R> ket_m = spinor_v<R>(ev.p[2], 0, hel_of(h, 2, 4));
      const Spin<R> bra_m = dirac_bar(spinor_u<R>(ev.p[3], 0, hel_of(h, 3, 4)));
      const Mat4<R> g5 = gamma5<R>();
      Mat4<R> PL = identity4<R>(), PR = identity4<R>();
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          PL[i][j] = (PL[i][j] - g5[i][j]) * R(0.5);
          PR[i][j] = (PR[i][j] + g5[i][j]) * R(0.5);
        }
      Vec4<R> Je_a, Jm_a, Je_z, Jm_z;
      for (int mu = 0; mu < 4; ++mu) {
        const Mat4<R> g = gamma<R>(mu);
        const Mat4<R> va = matscale(g, -I * e * Q);
        const Mat4<R> vz = matscale(matadd(matscale(matmul(g, PL), cplx<R>(gL)),
                                           matscale(matmul(g, PR), cplx<R>(gR))),
                                    -I * gz);
        Je_a[mu] = braket(bra_e, matvec(va, ket_e));
        Jm_a[mu] = braket(bra_m, matvec(va, ket_m));
        Je_z[mu] = braket(bra_e, matvec(vz, ket_e));
        Jm_z[mu] = braket(bra_m, matvec(vz, ket_m));
      }
      Vec4<R> q;
      for (int mu = 0; mu < 4; ++mu) q[mu] = cplx<R>(ev.p[0][mu] + ev.p[1][mu]);
      const cplx<R> s = mdot(q, q);
      for (size_t t = 0; t < terms.size(); ++t) {
        if (terms[t].boson == 0) {
          amp[t] = (-I / s) * mdot(Je_a, Jm_a);
        } else {
          const R mz = (R)par.mz, wz = (R)par.wz;
          const cplx<R> den = s - mz * mz + I * mz * wz;
          amp[t] = (-I / den) * (mdot(Je_z, Jm_z) - mdot(q, Je_z) * mdot(q, Jm_z) / (mz * mz));
        }
      }
      return;
    }
    const R gs = std::sqrt(R(4) * R(3.141592653589793238462643383279502884L) * (R)par.alpha_s);
    const R mt = (R)par.mt;
    Vec4<R> pol[8];
    for (int leg : gluon_legs) {
      if (leg == pol_override) {
        pol[leg] = real_vec<R>(ev.p[leg]);
      } else {
        const Vec4<R> e = polarisation<R>(ev.p[leg], hel_of(h, leg, n_ext));
        pol[leg] = incoming[leg] ? e : conj4(e);
      }
    }
    const Spin<R> bra = dirac_bar(spinor_u<R>(ev.p[quark_leg], mt, hel_of(h, quark_leg, n_ext)));
    const Spin<R> ket0 = spinor_v<R>(ev.p[antiquark_leg], mt, hel_of(h, antiquark_leg, n_ext));
    for (size_t t = 0; t < terms.size(); ++t) {
      const Term& term = terms[t];
      Spin<R> ket = ket0;
      R q[4];
      for (int mu = 0; mu < 4; ++mu) q[mu] = ev.pin[antiquark_leg][mu];
      const int n = (int)term.roots.size();
      for (int m = n - 1; m >= 0; --m) {
        const Current<R> W = node_current(term.roots[m], term, ev, pol);
        ket = matvec(matscale(slash(W.J), I * gs), ket);
        for (int mu = 0; mu < 4; ++mu) q[mu] += W.P[mu];
        if (m > 0) {
          const Vec4<R> qv = real_vec<R>(q);
          const R q2 = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3];
          Mat4<R> S = slash(qv);
          for (int i = 0; i < 4; ++i) S[i][i] += mt;
          ket = matvec(matscale(S, I / (q2 - mt * mt)), ket);
        }
      }
      amp[t] = braket(bra, ket);
    }
  }

  // Colour-flow amplitudes J_s = sum_t c_st A_t.
  template <class R>
  void flows(const std::vector<cplx<R>>& amp, std::vector<cplx<R>>& J) const {
    J.assign(ncol, cplx<R>(0));
    for (size_t t = 0; t < terms.size(); ++t)
      for (auto& sc : coef[t])
        J[sc.first] += cplx<R>((R)sc.second.real(), (R)sc.second.imag()) * amp[t];
  }

  // sum_{s,t} conj(J_s) C_st J_t
  template <class R> R colour_sum(const std::vector<cplx<R>>& J) const {
    R acc = 0;
    for (int s = 0; s < ncol; ++s) {
      cplx<R> z = 0;
      for (int t = 0; t < ncol; ++t) z += (R)cnum[(size_t)s * ncol + t] * J[t];
      acc += (std::conj(J[s]) * z).real();
    }
    return acc / (R)cden;
  }

  // Per-helicity colour-summed |M_h|^2 (normalised), colour-decomposed.
  template <class R> void me_hel(const double* mom, R* out) const {
    const Event<R> ev = make_event<R>(mom);
    std::vector<cplx<R>> amp, J;
    for (int h = 0; h < n_hel; ++h) {
      term_amplitudes(ev, h, -1, amp);
      flows(amp, J);
      out[h] = colour_sum(J) * (R)norm;
    }
  }

  // Condition number of |M|^2 with respect to relative changes of the
  // diagram amplitudes: the same helicity and colour sums with every term
  // amplitude, colour coefficient and colour-matrix entry replaced by its
  // absolute value, divided by |M|^2 itself.  Changing each amplitude by a
  // relative amount of at most eps changes |M|^2 by at most about
  // 2 eps kappa |M|^2; kappa >= 1, and it is large where diagrams cancel.
  long double condition(const double* mom) const {
    using L = long double;
    const Event<L> ev = make_event<L>(mom);
    std::vector<cplx<L>> amp, J;
    std::vector<L> Ja(ncol);
    L num = 0, den = 0;
    for (int h = 0; h < n_hel; ++h) {
      term_amplitudes(ev, h, -1, amp);
      flows(amp, J);
      den += colour_sum(J);
      std::fill(Ja.begin(), Ja.end(), (L)0);
      for (size_t t = 0; t < terms.size(); ++t)
        for (auto& sc : coef[t]) Ja[sc.first] += std::abs(cplx<L>((L)sc.second.real(), (L)sc.second.imag())) *
                                                 std::abs(amp[t]);
      L a = 0;
      for (int s = 0; s < ncol; ++s)
        for (int t = 0; t < ncol; ++t) a += std::abs((L)cnum[(size_t)s * ncol + t]) * Ja[s] * Ja[t];
      num += a / (L)cden;
    }
    return num / den;
  }

  template <class R> R me(const double* mom) const {
    std::vector<R> hel(n_hel);
    me_hel<R>(mom, hel.data());
    R s = 0;
    for (int h = 0; h < n_hel; ++h) s += hel[h];
    return s;
  }

  // ------------------------------------------------- brute-force colour sum
  std::vector<cd> ktab;  // [config][term] explicit colour factors
  long long nconf_full = 0;

  void build_full_colour_table() {
    if (!ktab.empty() || kind == EE_MUMU) return;
    const int k = (int)gluon_legs.size();
    if (k > 4) throw std::invalid_argument("brute-force colour sum limited to four gluons");
    long long ng = 1;
    for (int i = 0; i < k; ++i) ng *= 8;
    nconf_full = ng * 9;
    ktab.assign((size_t)nconf_full * terms.size(), cd(0));
    int acol[8] = {0};
    for (long long c = 0; c < nconf_full; ++c) {
      long long x = c / 9;
      for (int i = 0; i < k; ++i) {
        acol[gluon_legs[i]] = (int)(x % 8);
        x /= 8;
      }
      const int i = (int)(c % 9) / 3, j = (int)(c % 3);
      for (size_t t = 0; t < terms.size(); ++t)
        ktab[(size_t)c * terms.size() + t] = term_colour(terms[t], acol, i, j);
    }
  }

  // |M|^2 with the colour sum done over every explicit colour assignment.
  double me_brute(const double* mom) const {
    const Event<double> ev = make_event<double>(mom);
    std::vector<cd> amp;
    double total = 0;
    for (int h = 0; h < n_hel; ++h) {
      term_amplitudes(ev, h, -1, amp);
      if (kind == EE_MUMU) {
        cd m = 0;
        for (auto& a : amp) m += a;
        total += std::norm(m);
        continue;
      }
      for (long long c = 0; c < nconf_full; ++c) {
        cd m = 0;
        const cd* kt = &ktab[(size_t)c * terms.size()];
        for (size_t t = 0; t < terms.size(); ++t) m += kt[t] * amp[t];
        total += std::norm(m);
      }
    }
    return total * norm;
  }
};

}  // namespace oracle
