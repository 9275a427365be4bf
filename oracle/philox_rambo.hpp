// Oracle (test infrastructure only): counter-based random numbers and RAMBO
// flat phase space, written plainly in double precision.
//
// Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
// 32x32->64 multiplications with the constants 0xD2511F53 / 0xCD9E8D57 and a
// Weyl key schedule with increments 0x9E3779B9 / 0xBB67AE85.
//
// RAMBO follows Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359:
// n isotropic massless momenta with energies drawn from x e^{-x}, a conformal
// boost and scale to the centre-of-mass energy, and, for massive particles, a
// rescaling of the three-momenta by the root xi of sum_i sqrt(m_i^2+xi^2 E_i^2)
// = sqrt(s), found by Newton's method.
//
// The paper places phase-space sampling in the host-side framework (section 2)
// and lists moving it to the GPU as a way to cut the serial part; it gives no
// generator of its own, so the flat RAMBO generator stands in for it.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace oracle {

inline void philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {in[0], in[1], in[2], in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {  // key schedule between rounds
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    const uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    const uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

// Two uniform doubles in the open interval (0,1) from one Philox block.
// counter = (block, 0, event low word, event high word), key = (seed low, seed high);
// each double takes 64 bits (first word low), keeps the top 53 and is centred
// in its bin: u = ((x >> 11) + 0.5) * 2^-53.
inline void uniform_pair(uint64_t seed, uint64_t event, uint32_t block, double u[2]) {
  const uint32_t ctr[4] = {block, 0u, (uint32_t)event, (uint32_t)(event >> 32)};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  philox4x32_10(ctr, key, w);
  const uint64_t x0 = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
  const uint64_t x1 = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
  const double two_m53 = 1.0 / 9007199254740992.0;
  u[0] = ((double)(x0 >> 11) + 0.5) * two_m53;
  u[1] = ((double)(x1 >> 11) + 0.5) * two_m53;
}

// One RAMBO event.  p[i][mu] for the n_out final-state particles, i in [0,n_out).
// Final-state particle i uses the four uniforms of blocks 2i and 2i+1.
// Returns the phase-space weight (with the (2 pi)^(4-3n) convention).
inline double rambo_event(int n_out, const double* masses, double sqrt_s, uint64_t seed,
                          uint64_t event, double (*p)[4]) {
  const double pi = 3.141592653589793238462643383279502884;
  const int n = n_out;
  std::vector<double> q(4 * n);
  // Step 1: isotropic massless momenta with energy density q0 e^{-q0}.
  for (int i = 0; i < n; ++i) {
    double ua[2], ub[2];
    uniform_pair(seed, event, (uint32_t)(2 * i), ua);
    uniform_pair(seed, event, (uint32_t)(2 * i + 1), ub);
    const double cost = 2.0 * ua[0] - 1.0;
    const double sint = std::sqrt(1.0 - cost * cost);
    const double phi = 2.0 * pi * ua[1];
    const double e = -std::log(ub[0] * ub[1]);
    q[4 * i + 0] = e;
    q[4 * i + 1] = e * sint * std::cos(phi);
    q[4 * i + 2] = e * sint * std::sin(phi);
    q[4 * i + 3] = e * cost;
  }
  // Step 2: conformal transformation to total momentum (sqrt_s, 0, 0, 0).
  double Q[4] = {0, 0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int mu = 0; mu < 4; ++mu) Q[mu] += q[4 * i + mu];
  const double M = std::sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
  const double x = sqrt_s / M;
  const double gam = Q[0] / M;
  const double a = 1.0 / (1.0 + gam);
  for (int i = 0; i < n; ++i) {
    const double* qi = &q[4 * i];
    const double bq = b[0] * qi[1] + b[1] * qi[2] + b[2] * qi[3];
    p[i][0] = x * (gam * qi[0] + bq);
    for (int k = 0; k < 3; ++k) p[i][k + 1] = x * (qi[k + 1] + b[k] * qi[0] + a * bq * b[k]);
  }
  // Massless weight: (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!) * (2 pi)^(4-3n).
  double fact_n1 = 1.0, fact_n2 = 1.0;
  for (int k = 2; k <= n - 1; ++k) fact_n1 *= k;
  for (int k = 2; k <= n - 2; ++k) fact_n2 *= k;
  const double s = sqrt_s * sqrt_s;
  double w = std::pow(pi / 2.0, n - 1) * std::pow(s, n - 2) / (fact_n1 * fact_n2) *
             std::pow(2.0 * pi, 4 - 3 * n);
  // Step 3: masses.
  double msum = 0.0;
  bool massive = false;
  for (int i = 0; i < n; ++i) {
    msum += masses[i];
    if (masses[i] != 0.0) massive = true;
  }
  if (!massive) return w;
  double xi = std::sqrt(1.0 - (msum / sqrt_s) * (msum / sqrt_s));
  for (int it = 0; it < 50; ++it) {
    double f = -sqrt_s, fp = 0.0;
    for (int i = 0; i < n; ++i) {
      const double e = std::sqrt(masses[i] * masses[i] + xi * xi * p[i][0] * p[i][0]);
      f += e;
      fp += xi * p[i][0] * p[i][0] / e;
    }
    if (std::fabs(f) < 1e-14 * sqrt_s) break;
    xi -= f / fp;
  }
  double prod = 1.0, sum = 0.0;
  for (int i = 0; i < n; ++i) {
    const double e = std::sqrt(masses[i] * masses[i] + xi * xi * p[i][0] * p[i][0]);
    for (int k = 1; k < 4; ++k) p[i][k] *= xi;
    p[i][0] = e;
    const double kk = std::sqrt(p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
    prod *= kk / e;
    sum += kk * kk / e;
  }
  w *= std::pow(xi, 2 * n - 3) * prod * sqrt_s / sum;
  return w;
}

}  // namespace oracle
