// Arguments shared by the generated matrix-element kernels and the runtime.
#pragma once
#include <hip/hip_runtime.h>

#ifndef MGME_ME_BLOCK
#define MGME_ME_BLOCK 128
#endif

#define MGME_MAX_HEL 128

namespace mgme {

// Passed by value as a kernel argument.  The helicity list is read from the
// kernel-argument segment: through the scalar unit where every lane of a wave
// evaluates the same helicity (the staged kernels), per lane where the lanes
// of one event take different ones (the fused kernels).
struct MeArgs {
  double mt;        // top-quark mass (GeV)
  double factor;    // gs^(2k) / (spin-colour average * identical-particle factor * colour denominator)
  double ee_qq;     // e^2 Q_e Q_mu (photon exchange)
  double ee_zz;     // e^2 / (sw^2 cw^2) (Z exchange)
  double ee_gl;     // T3 - Q sw^2 of the charged leptons
  double ee_gr;     // -Q sw^2
  double mz, wz;
  int z_enabled;
  const void* cfrag;        // colour matrix as half-precision MFMA A fragments (mixed precision)
  int nhel;                 // helicities to sum
  int hel[MGME_MAX_HEL];    // helicity codes: bit (n_ext-1-leg) set for helicity +1
};

// Random numbers and results of the per-event helicity and colour choice
// (device arrays indexed by event).
struct SelectArgs {
  const double* r_hel;  // uniform in (0,1): helicity choice
  const double* r_col;  // uniform in (0,1): colour-flow choice
  int* hel;             // chosen helicity code
  int* col;             // chosen colour flow (basis index)
};

// Device workspace of one launch: a buffer the caller provides (its size then
// bounds the sub-batches, and nothing is allocated), or, when ptr is NULL,
// memory from the stream-ordered allocator returned at the end of the launch.
struct Workspace {
  void* ptr;
  long long bytes;
};

// Events per sub-batch for per_event bytes of workspace per event: bounded by
// the caller's buffer when one is given, else by `cap` bytes; at most max_sub
// (when > 0) and at most nevt rounded up to 64.  0 when a caller's buffer
// cannot hold 64 events.
inline long long ws_sub_batch(const Workspace* ws, size_t per_event, size_t cap, long long max_sub, long long nevt) {
  const bool given = ws && ws->ptr;
  long long sub = (long long)((given ? (size_t)ws->bytes : cap) / per_event) / 64 * 64;
  if (sub < 64) {
    if (given) return 0;
    sub = 64;
  }
  if (max_sub > 0 && sub > max_sub) sub = max_sub;
  const long long whole = (nevt + 63) / 64 * 64;
  return sub < whole ? sub : whole;
}

inline hipError_t ws_acquire(const Workspace* ws, size_t bytes, void** p, hipStream_t stream) {
  if (ws && ws->ptr) {
    *p = ws->ptr;
    return bytes <= (size_t)ws->bytes ? hipSuccess : hipErrorInvalidValue;
  }
  return hipMallocAsync(p, bytes, stream);
}

inline hipError_t ws_release(const Workspace* ws, void* p, hipStream_t stream) {
  return (ws && ws->ptr) ? hipSuccess : hipFreeAsync(p, stream);
}

// prec: 0 FP64, 1 FP32 diagrams, 2 FP32 diagrams + 16-bit matrix-core colour sum,
// 3 FP64 diagrams + FP32 colour algebra.  per_hel: per-helicity output with
// leading dimension ldo.  sel: when not NULL, also choose a helicity and a
// colour flow per event (per_hel must be 0).  ws: caller's workspace, or NULL.
using LaunchFn = hipError_t (*)(int prec, int per_hel, const double* mom, long long nevt, long long ld,
                                const MeArgs* args, double* out, long long ldo, const SelectArgs* sel,
                                const Workspace* ws, hipStream_t stream);

}  // namespace mgme
