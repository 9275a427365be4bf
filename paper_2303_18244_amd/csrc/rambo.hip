// RAMBO flat phase-space generator on gfx950, one lane per event.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed
// by the 64-bit seed, with counter (block, 0, event low, event high); each
// block yields two doubles u = ((x >> 11) + 0.5) 2^-53 from its 64-bit halves
// (first word low), so every event is reproducible from (seed, event index)
// alone, independent of the batch it is generated in.
//
// Phase space: Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359.
// Final-state particle i draws the four uniforms of blocks 2i and 2i+1:
// cos(theta) = 2 r1 - 1, phi = 2 pi r2, E = -log(r3 r4); the massless set is
// boosted and scaled to (sqrt(s), 0, 0, 0), then masses are introduced by
// rescaling three-momenta with the root of sum_i sqrt(m_i^2 + xi^2 E_i^2) =
// sqrt(s) (Newton's method).  The two initial partons are along +z and -z
// with energy sqrt(s)/2.  The paper samples phase space in the host-side
// framework (section 2); this generator is the flat stand-in that feeds the
// matrix-element kernels with device-resident momenta.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rambo.h"

namespace mgme {

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ void uniform2(unsigned long long seed, unsigned long long event, uint32_t block,
                                         double& u0, double& u1) {
  uint32_t c[4] = {block, 0u, (uint32_t)event, (uint32_t)(event >> 32)};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const unsigned long long x0 = (unsigned long long)c[0] | ((unsigned long long)c[1] << 32);
  const unsigned long long x1 = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
  const double scale = 1.1102230246251565404e-16;  // 2^-53
  u0 = ((double)(x0 >> 11) + 0.5) * scale;
  u1 = ((double)(x1 >> 11) + 0.5) * scale;
}

template <int NOUT>
__global__ void __launch_bounds__(256) rambo_kernel(RamboArgs a, long long nevt, long long ld,
                                                    double* __restrict__ mom, double* __restrict__ wgt) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  const unsigned long long ev = a.first_event + (unsigned long long)e;
  const double pi = 3.141592653589793238462643383279502884;
  double p[NOUT][4];
  double Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < NOUT; ++i) {
    double r1, r2, r3, r4;
    uniform2(a.seed, ev, (uint32_t)(2 * i), r1, r2);
    uniform2(a.seed, ev, (uint32_t)(2 * i + 1), r3, r4);
    const double c = 2.0 * r1 - 1.0;
    const double s = sqrt(1.0 - c * c);
    double sphi, cphi;
    sincos(2.0 * pi * r2, &sphi, &cphi);
    const double en = -log(r3 * r4);
    p[i][0] = en;
    p[i][1] = en * s * cphi;
    p[i][2] = en * s * sphi;
    p[i][3] = en * c;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) Q[mu] += p[i][mu];
  }
  const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  const double b1 = -Q[1] / M, b2 = -Q[2] / M, b3 = -Q[3] / M;
  const double x = a.sqrt_s / M, g = Q[0] / M, aa = 1.0 / (1.0 + g);
#pragma unroll
  for (int i = 0; i < NOUT; ++i) {
    const double bq = b1 * p[i][1] + b2 * p[i][2] + b3 * p[i][3];
    const double e0 = p[i][0];
    p[i][0] = x * (g * e0 + bq);
    p[i][1] = x * (p[i][1] + b1 * e0 + aa * bq * b1);
    p[i][2] = x * (p[i][2] + b2 * e0 + aa * bq * b2);
    p[i][3] = x * (p[i][3] + b3 * e0 + aa * bq * b3);
  }
  double w = a.massless_weight;
  if (a.massive) {
    double msum = 0.0;
#pragma unroll
    for (int i = 0; i < NOUT; ++i) msum += a.mass[i];
    double xi = sqrt(1.0 - (msum / a.sqrt_s) * (msum / a.sqrt_s));
    for (int it = 0; it < 50; ++it) {
      double f = -a.sqrt_s, fp = 0.0;
#pragma unroll
      for (int i = 0; i < NOUT; ++i) {
        const double en = sqrt(a.mass[i] * a.mass[i] + xi * xi * p[i][0] * p[i][0]);
        f += en;
        fp += xi * p[i][0] * p[i][0] / en;
      }
      if (fabs(f) < 1e-14 * a.sqrt_s) break;
      xi -= f / fp;
    }
    double prod = 1.0, sum = 0.0;
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
      const double en = sqrt(a.mass[i] * a.mass[i] + xi * xi * p[i][0] * p[i][0]);
      p[i][1] *= xi;
      p[i][2] *= xi;
      p[i][3] *= xi;
      p[i][0] = en;
      const double kk = sqrt(p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
      prod *= kk / en;
      sum += kk * kk / en;
    }
    w *= pow(xi, 2 * NOUT - 3) * prod * a.sqrt_s / sum;
  }
  const double h = 0.5 * a.sqrt_s;
  mom[(0 * 4 + 0) * ld + e] = h;
  mom[(0 * 4 + 1) * ld + e] = 0.0;
  mom[(0 * 4 + 2) * ld + e] = 0.0;
  mom[(0 * 4 + 3) * ld + e] = h;
  mom[(1 * 4 + 0) * ld + e] = h;
  mom[(1 * 4 + 1) * ld + e] = 0.0;
  mom[(1 * 4 + 2) * ld + e] = 0.0;
  mom[(1 * 4 + 3) * ld + e] = -h;
#pragma unroll
  for (int i = 0; i < NOUT; ++i)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) mom[(long long)((i + 2) * 4 + mu) * ld + e] = p[i][mu];
  if (wgt) wgt[e] = w;
}

hipError_t launch_rambo(const RamboArgs& a, int n_out, long long nevt, long long ld, double* mom, double* wgt,
                        hipStream_t stream) {
  const dim3 block(256), grid((unsigned)((nevt + 255) / 256));
  switch (n_out) {
    case 2: rambo_kernel<2><<<grid, block, 0, stream>>>(a, nevt, ld, mom, wgt); break;
    case 3: rambo_kernel<3><<<grid, block, 0, stream>>>(a, nevt, ld, mom, wgt); break;
    case 4: rambo_kernel<4><<<grid, block, 0, stream>>>(a, nevt, ld, mom, wgt); break;
    case 5: rambo_kernel<5><<<grid, block, 0, stream>>>(a, nevt, ld, mom, wgt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mgme
