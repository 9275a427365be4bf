// Mixed-precision colour sum on the matrix cores (see colour_mfma.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace mgme {

// Tile counts for a number of colour flows (at most 128): 32-row M tiles and
// 16-deep K steps of the padded colour matrix.
int colour_mfma_tiles(int ncol, int* mt, int* ks);

// Host: A-operand fragments of the colour matrix (integer numerators
// num[ncol*ncol]) as half-precision bit patterns, [mt][ks][lane][8]; the
// array holds mt*ks*64*8 entries.
void colour_mfma_fragments(int ncol, const long long* num, unsigned short* frag_half_bits);

// out[h*ldo + e] = scale * Re(J^dagger C J) for the columns (e, h) of
// J[(h*ncol + flow)*ldj + e] (complex single precision), e < nevt, h < nhel.
hipError_t launch_colour_mfma(long long nevt, int nhel, int ncol, const void* J, long long ldj, const void* cfrag,
                              double* out, long long ldo, double scale, hipStream_t stream);

// Row r (0..31) of a 32-row tile of the A operand carries colour flow
// colour_mfma_row_flow(r) (the permutation that makes result register i of a
// lane hold a flow whose J the lane supplied itself).
int colour_mfma_row_flow(int r);

typedef _Float16 mfma_half8 __attribute__((ext_vector_type(8)));
typedef float mfma_floatx16 __attribute__((ext_vector_type(16)));

// Re(J^dagger C J) (C: the integer numerators) of the wave's 64 events, one
// per lane, for a colour-flow vector of at most 32 flows held by each lane
// (J[f].re, J[f].im in single precision), on the matrix cores inside a
// diagram kernel.  Every lane of the wave must call it (lanes without an
// event pass any finite J).  cfrag: the two A-operand fragments of C
// (colour_mfma_fragments, one 32-row tile, two K steps) of this lane.
// Precision as the colour kernel: J scaled by a power of two per event and
// split into two half-precision parts; products exact, sums of C X in FP32;
// the dot product X.(C X) and the rescaling in double.
//
// Lanes L and L+32 supply the two K halves of one event's column of the B
// operand, so the wave's 64 events are two 32-event tiles: in tile 0 lane
// L+32 supplies the flows 8..15 and 24..31 of lane L's event, in tile 1 lane
// L supplies the flows 0..7 and 16..23 of lane L+32's event (exchanged with a
// swap of the wave's halves).  Each lane then holds the partial dot product
// of its K half for both tiles; the two halves of an event are added once
// more after one swap.  With at most 16 flows the second K step holds only
// zeros (of J and of C), so it is left out: the same sums, exactly, with half
// the matrix-core instructions, splits and swaps.
template <int NCOL, typename CX>
__device__ __forceinline__ double colour_mfma_lane(const CX* J, const mfma_half8 cfrag[2]) {
  static_assert(NCOL <= 32, "one 32-row tile");
  constexpr int KS = NCOL > 16 ? 2 : 1;  // K steps of 16 flows
  const int lane = threadIdx.x & 63;
  const bool upper = lane >= 32;
  float mx = 0.0f;
#pragma unroll
  for (int f = 0; f < NCOL; ++f) mx = fmaxf(mx, fmaxf(fabsf((float)J[f].re), fabsf((float)J[f].im)));
  int ex = 0;
  (void)frexpf(mx, &ex);
  const float s = mx > 0.0f ? ldexpf(1.0f, ex < -126 ? 126 : -ex) : 1.0f;
  // m_*: the K half this lane supplies for its own event (flows
  // 16 ks + 8 (lane/32) + j), x_*: the other half, which goes to the partner
  // lane (lane xor 32) and comes back as the partner event's half
  mfma_half8 m_rh[2], m_rl[2], m_ih[2], m_il[2], x_rh[2], x_rl[2], x_ih[2], x_il[2];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int f0 = 16 * ks + j, f1 = f0 + 8;
      const float r0 = f0 < NCOL ? (float)J[f0].re * s : 0.0f, i0 = f0 < NCOL ? (float)J[f0].im * s : 0.0f;
      const float r1 = f1 < NCOL ? (float)J[f1].re * s : 0.0f, i1 = f1 < NCOL ? (float)J[f1].im * s : 0.0f;
      const float a = upper ? r1 : r0, b = upper ? i1 : i0;  // own half
      const float c = upper ? r0 : r1, d = upper ? i0 : i1;  // partner's half
      const _Float16 ah = (_Float16)a, bh = (_Float16)b, ch = (_Float16)c, dh = (_Float16)d;
      m_rh[ks][j] = ah;
      m_rl[ks][j] = (_Float16)(a - (float)ah);
      m_ih[ks][j] = bh;
      m_il[ks][j] = (_Float16)(b - (float)bh);
      x_rh[ks][j] = ch;
      x_rl[ks][j] = (_Float16)(c - (float)ch);
      x_ih[ks][j] = dh;
      x_il[ks][j] = (_Float16)(d - (float)dh);
    }
  typedef int int4v __attribute__((ext_vector_type(4)));
  auto swap_halves = [](mfma_half8& v) {
    int4v w = __builtin_bit_cast(int4v, v);
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = __shfl_xor(w[q], 32);
    v = __builtin_bit_cast(mfma_half8, w);
  };
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    swap_halves(x_rh[ks]);
    swap_halves(x_rl[ks]);
    swap_halves(x_ih[ks]);
    swap_halves(x_il[ks]);
  }
  double p[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    // tile t: the events of lanes 32 t .. 32 t + 31; the lane supplies its
    // own K half if its event is in the tile, else the received one
    const bool mine = (t == 1) == upper;
    mfma_floatx16 dr = {}, di = {};
    mfma_half8 brh[2], brl[2], bih[2], bil[2];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      brh[ks] = mine ? m_rh[ks] : x_rh[ks];
      brl[ks] = mine ? m_rl[ks] : x_rl[ks];
      bih[ks] = mine ? m_ih[ks] : x_ih[ks];
      bil[ks] = mine ? m_il[ks] : x_il[ks];
      dr = __builtin_amdgcn_mfma_f32_32x32x16_f16(cfrag[ks], brh[ks], dr, 0, 0, 0);
      dr = __builtin_amdgcn_mfma_f32_32x32x16_f16(cfrag[ks], brl[ks], dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_32x32x16_f16(cfrag[ks], bih[ks], di, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_32x32x16_f16(cfrag[ks], bil[ks], di, 0, 0, 0);
    }
    // register i holds (C X) at flow 16 (i/8) + 8 kh + i%8: B entry j = i%8
    // of K step i/8 of this lane
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 8 * KS; ++i) {
      const int ks = i / 8, j = i % 8;
      const double xre = (double)(float)brh[ks][j] + (double)(float)brl[ks][j];
      const double xim = (double)(float)bih[ks][j] + (double)(float)bil[ks][j];
      acc += xre * (double)dr[i] + xim * (double)di[i];
    }
    p[t] = acc;
  }
  // lane L (< 32): p[0] is its event's lower-K half, p[1] the lower half of
  // lane L+32's event; lane L+32 holds the upper halves of the same events
  const double keep = upper ? p[1] : p[0];
  const double other = __shfl_xor(upper ? p[0] : p[1], 32);
  return (keep + other) / ((double)s * (double)s);
}

// out[e] = factor * sum_h meh[h*ldh + e] in helicity order (deterministic).
hipError_t launch_helicity_sum(long long nevt, int nhel, const double* meh, long long ldh, double factor, double* out,
                               hipStream_t stream);

}  // namespace mgme
