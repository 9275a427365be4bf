// Functions shared by the runtime units of libmgme.so (not exported).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/mgme.h"
#include "me_kernel.h"

namespace mgme {

// mgme_matrix_element with its workspace taken from `ws` (NULL or ws->ptr
// NULL: the stream-ordered allocator).  Same validation and errors; a
// caller's workspace smaller than workspace_min_bytes gives EINVAL.
int matrix_element_ws(const mgme_process* proc, const double* d_mom, long long nevt, long long ld, int precision,
                      double* d_me, const Workspace* ws, hipStream_t stream);

// Smallest caller workspace with which a launch of `precision` runs: one
// sub-batch of 64 events of the staging buffers (0 when the launch needs no
// staging, as the fused processes' launches never do).
long long workspace_min_bytes(const mgme_process* proc, int precision);

// Device the process was created on.
int process_device(const mgme_process* proc);

// Number of external particles of the process.
int process_n_ext(const mgme_process* proc);

// Records `msg` as the calling thread's mgme_last_error() text; returns code.
int set_error(int code, const char* msg);

}  // namespace mgme
