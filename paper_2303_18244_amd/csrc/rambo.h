// RAMBO launch interface (see rambo.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace mgme {

struct RamboArgs {
  double sqrt_s;
  double massless_weight;   // (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!) (2 pi)^(4-3n)
  double mass[6];           // final-state masses
  int massive;              // any final-state mass non-zero
  unsigned long long seed;
  unsigned long long first_event;
};

hipError_t launch_rambo(const RamboArgs& a, int n_out, long long nevt, long long ld, double* mom, double* wgt,
                        hipStream_t stream);

}  // namespace mgme
