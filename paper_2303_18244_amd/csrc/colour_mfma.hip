// Colour sum on the matrix cores, mixed precision: me_h = Re(J^dagger C J)
// for a batch of (event, helicity) columns, with J from single-precision
// diagrams and C the integer numerators of the colour matrix (the "color
// algebra" of section 3 of the paper, here on 16-bit MFMA).
//
// Per wave: 32 events of one helicity.  Y = C X is one GEMM with
// X = [Re J | Im J] (flows x events) as the B operand of
// v_mfma_f32_32x32x16_f16 and C as the A operand; me = sum_m X[m] Y[m].
// Precision: every column is scaled by a power of two so that max |J| lies
// in [1/2, 1), then split into two half-precision parts, hi = fp16(x) and
// lo = fp16(x - hi), so X is carried to about 2^-22 of its largest entry;
// C's numerators (|c| <= 4096) are exact in half precision.  Products are
// exact and accumulate in FP32; the final dot product X.Y, the rescaling and
// the hand-over are in double.  The relative error of me is bounded by about
// cond(C) 2^-22.
//
// Lane layout of the 32x32x16 f16 MFMA (gfx950): A[m][k] with m = lane%32,
// k = 8 (lane/32) + j; B[k][n] with n = lane%32, k = 8 (lane/32) + j;
// D[m][n] in result register i with n = lane%32,
// m = 8 (i/4) + 4 (lane/32) + i%4.
//
// The rows of C in the A operand are permuted within each 32-row tile so
// that result register i of a lane holds Y at a flow whose X the lane itself
// supplied to the B operand: row r of the tile (in register
// i = 4 (r/8) + r%4 of the lanes with lane/32 = (r/4)%2) carries flow
// 16 (i/8) + 8 (lane/32) + i%8, which is B register j = i%8 of K step i/8 of
// that tile.  The dot product X.Y then needs no data from other lanes and no
// second read of J.
#include <hip/hip_runtime.h>

#include "colour_mfma.h"

namespace mgme {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int MT, int KS>
__global__ void __launch_bounds__(256) colour_mfma_kernel(long long nevt, int nhel, int ncol,
                                                         const float2* __restrict__ J, long long ldj,
                                                         const half8* __restrict__ cfrag, double* __restrict__ out,
                                                         long long ldo, double scale) {
  const int lane = threadIdx.x & 63;
  const int hs = __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (threadIdx.x >> 6));
  if (hs >= nhel) return;  // whole wave
  const int n = lane & 31, kh = lane >> 5;
  const long long e = (long long)blockIdx.x * 32 + n;
  const bool valid = e < nevt;
  const float2* __restrict__ Jh = J + (long long)hs * ncol * ldj;

  // B operand: flows 16 ks + 8 kh + j of this lane's event
  float xr[KS][8], xi[KS][8];
  float mx = 0.0f;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int f = 16 * ks + 8 * kh + j;
      float2 v = make_float2(0.0f, 0.0f);
      if (valid && f < ncol) v = Jh[(long long)f * ldj + e];
      xr[ks][j] = v.x;
      xi[ks][j] = v.y;
      mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
  mx = fmaxf(mx, __shfl_xor(mx, 32));
  int ex = 0;
  (void)frexpf(mx, &ex);
  // 2^-ex stays finite (mx below 2^-126 keeps the factor 2^126)
  const float s = mx > 0.0f ? ldexpf(1.0f, ex < -126 ? 126 : -ex) : 1.0f;
  half8 rh[KS], rl[KS], ih[KS], il[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float a = xr[ks][j] * s, b = xi[ks][j] * s;
      const _Float16 ah = (_Float16)a, bh = (_Float16)b;
      rh[ks][j] = ah;
      rl[ks][j] = (_Float16)(a - (float)ah);
      ih[ks][j] = bh;
      il[ks][j] = (_Float16)(b - (float)bh);
    }
  static_assert(KS == 2 * MT, "two K steps per 32-row tile");
  double me = 0.0;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    floatx16 dr = {}, di = {};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const half8 a = cfrag[(mt * KS + ks) * 64 + lane];
      dr = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, rh[ks], dr, 0, 0, 0);
      dr = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, rl[ks], dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, ih[ks], di, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, il[ks], di, 0, 0, 0);
    }
    // register i holds Y at flow 32 mt + 16 (i/8) + 8 kh + i%8: the lane's
    // own B entry j = i%8 of K step 2 mt + i/8 (hi + lo: the X of the GEMM)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int ks = 2 * mt + i / 8, j = i % 8;
      const double xre = (double)(float)rh[ks][j] + (double)(float)rl[ks][j];
      const double xim = (double)(float)ih[ks][j] + (double)(float)il[ks][j];
      me += xre * (double)dr[i] + xim * (double)di[i];
    }
  }
  me += __shfl_xor(me, 32);
  if (kh == 0 && valid) out[(long long)hs * ldo + e] = me / ((double)s * (double)s) * scale;
}

int colour_mfma_tiles(int ncol, int* mt, int* ks) {
  if (ncol <= 32) {
    *mt = 1;
    *ks = 2;
  } else if (ncol <= 128) {
    *mt = 4;
    *ks = 8;
  } else {
    return -1;
  }
  return 0;
}

// Flow carried by row r (0..31) of a 32-row tile of the A operand (see the
// kernel's lane layout): register i = 4 (r/8) + r%4 of the lanes with
// lane/32 = (r/4)%2 receives it.
int colour_mfma_row_flow(int r) {
  const int i = 4 * (r / 8) + r % 4, kh = (r / 4) % 2;
  return 16 * (i / 8) + 8 * kh + i % 8;
}

void colour_mfma_fragments(int ncol, const long long* num, unsigned short* frag_half_bits) {
  int MT = 0, KS = 0;
  colour_mfma_tiles(ncol, &MT, &KS);
  for (int mt = 0; mt < MT; ++mt)
    for (int ks = 0; ks < KS; ++ks)
      for (int lane = 0; lane < 64; ++lane)
        for (int j = 0; j < 8; ++j) {
          const int m = 32 * mt + colour_mfma_row_flow(lane % 32), k = 16 * ks + 8 * (lane / 32) + j;
          const float c = (m < ncol && k < ncol) ? (float)num[(size_t)m * ncol + k] : 0.0f;
          const _Float16 h = (_Float16)c;
          unsigned short bits;
          __builtin_memcpy(&bits, &h, 2);
          frag_half_bits[(((size_t)(mt * KS + ks) * 64 + lane) * 8) + j] = bits;
        }
}

hipError_t launch_colour_mfma(long long nevt, int nhel, int ncol, const void* J, long long ldj, const void* cfrag,
                              double* out, long long ldo, double scale, hipStream_t stream) {
  const dim3 grid((unsigned)((nevt + 31) / 32), (unsigned)((nhel + 3) / 4));
  const float2* Jf = (const float2*)J;
  const half8* cf = (const half8*)cfrag;
  if (ncol <= 32)
    colour_mfma_kernel<1, 2><<<grid, 256, 0, stream>>>(nevt, nhel, ncol, Jf, ldj, cf, out, ldo, scale);
  else if (ncol <= 128)
    colour_mfma_kernel<4, 8><<<grid, 256, 0, stream>>>(nevt, nhel, ncol, Jf, ldj, cf, out, ldo, scale);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// out[e] = factor * sum over helicities of meh[h*ldh + e], in helicity order.
__global__ void __launch_bounds__(256) helicity_sum_kernel(long long nevt, int nhel, const double* __restrict__ meh,
                                                          long long ldh, double factor, double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  double s = 0.0;
  for (int h = 0; h < nhel; ++h) s += meh[(long long)h * ldh + e];
  out[e] = s * factor;
}

hipError_t launch_helicity_sum(long long nevt, int nhel, const double* meh, long long ldh, double factor, double* out,
                               hipStream_t stream) {
  helicity_sum_kernel<<<(unsigned)((nevt + 255) / 256), 256, 0, stream>>>(nevt, nhel, meh, ldh, factor, out);
  return hipGetLastError();
}

}  // namespace mgme
