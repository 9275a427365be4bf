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

// out[e] = factor * sum_h meh[h*ldh + e] in helicity order (deterministic).
hipError_t launch_helicity_sum(long long nevt, int nhel, const double* meh, long long ldh, double factor, double* out,
                               hipStream_t stream);

}  // namespace mgme
