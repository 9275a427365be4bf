// Event-level steps after the matrix element: cross-section weights and their
// sums, hit-or-miss unweighting, and the random choice of one helicity
// configuration and one leading colour flow per event.
#pragma once
#include <hip/hip_runtime.h>

#include "me_kernel.h"

namespace mgme {

// (hbar c)^2 = 0.3893793721 GeV^2 mb (PDG), in GeV^2 pb.
constexpr double kGeV2pb = 0.3893793721e9;

// Weight factor for massless colliding partons at fixed sqrt(s): GeV^-2 -> pb
// over the flux 2 s.  Formed on the host in this order.
inline double weight_factor(double sqrt_s) { return kGeV2pb / (2.0 * sqrt_s * sqrt_s); }

// w[e] = (wgt[e] * me[e]) * k (w may be NULL); stats = (sum w, sum w^2, max w).
// The sums are formed in a fixed order for a given n (deterministic); `part`
// holds weights_partials(n) * 3 doubles of device workspace.
int weights_partials(long long n);
hipError_t launch_event_weights(long long n, const double* wgt, const double* me, double k, double* w, double* part,
                                double* stats, hipStream_t stream);

// Keeps e when r[e] * (*wref) < w[e]; idx receives the kept indices in
// increasing order, *nkept their number.  `tiles` is device workspace of
// 2 * unweight_tiles(n) long longs.
long long unweight_tiles(long long n);
hipError_t launch_unweight(long long n, const double* w, const double* r, const double* wref, long long* idx,
                           long long* nkept, long long* tiles, hipStream_t stream);

// jamp2[s*ldo + e] = sum over h < nhel of |J[(h*ncol + s)*ldj + e]|^2, J
// complex in T (float2 or double2 layout), accumulated in double in h order.
template <typename T>
hipError_t launch_jamp2(long long n, int nhel, int ncol, const T* J, long long ldj, double* jamp2, long long ldo,
                        hipStream_t stream);

// Per event: the helicity code args.hel[i] of the first good helicity i whose
// running sum of meh[i*ldh + e] exceeds r_hel[e] times the total, and the
// first colour flow s whose running sum of jamp2[s*ldj + e] exceeds r_col[e]
// times the total (the last non-zero entry when none does, code 0 / flow 0 if
// every entry is zero).
hipError_t launch_select(long long n, const MeArgs* args, const double* meh, long long ldh, int ncol,
                         const double* jamp2, long long ldj, const SelectArgs* sel, long long offset,
                         hipStream_t stream);

}  // namespace mgme
