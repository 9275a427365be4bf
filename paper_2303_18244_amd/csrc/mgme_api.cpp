// C-ABI runtime of libmgme.so: process creation (process selection,
// couplings, good-helicity calibration), argument validation and kernel
// launches.  See include/mgme.h for the contract of every entry point.
#include "../../include/mgme.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "colour_mfma.h"
#include "me_kernel.h"
#include "rambo.h"
#include "events.h"
#include "internal.h"
#include "registry.h"

struct mgme_process {
  const mgme::ProcEntry* entry;
  int device;
  mgme::MeArgs args;      // args.hel holds the helicities summed
  int good[MGME_MAX_HEL]; // the good helicities found at creation
  int n_good;
  int n_out;
  double mass_out[6];
  double norm_factor;
  double gs;
  void* d_cfrag;          // colour matrix as half-precision MFMA fragments (device)
};

namespace {

thread_local std::string g_error;

bool valid_precision(int p) {
  return p == MGME_FP64 || p == MGME_FP32 || p == MGME_MIXED || p == MGME_FP64_FP32COLOUR;
}

int fail(int code, const std::string& msg) {
  g_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(MGME_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Reports a pending asynchronous error of an earlier launch.
int check_pending(const char* where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, where);
  return MGME_OK;
}

int select_device(int device) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != device) {
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  }
  return MGME_OK;
}

double massless_rambo_weight(int n, double sqrt_s) {
  const double pi = 3.141592653589793238462643383279502884;
  double f1 = 1.0, f2 = 1.0;
  for (int k = 2; k <= n - 1; ++k) f1 *= k;
  for (int k = 2; k <= n - 2; ++k) f2 *= k;
  const double s = sqrt_s * sqrt_s;
  return std::pow(pi / 2.0, n - 1) * std::pow(s, n - 2) / (f1 * f2) * std::pow(2.0 * pi, 4 - 3 * n);
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int launch_rambo_checked(const mgme_process* p, double sqrt_s, unsigned long long seed, unsigned long long first,
                         long long nevt, long long ld, double* d_mom, double* d_wgt, hipStream_t stream) {
  mgme::RamboArgs a{};
  a.sqrt_s = sqrt_s;
  a.massless_weight = massless_rambo_weight(p->n_out, sqrt_s);
  double msum = 0.0;
  for (int i = 0; i < p->n_out; ++i) {
    a.mass[i] = p->mass_out[i];
    msum += p->mass_out[i];
    if (p->mass_out[i] != 0.0) a.massive = 1;
  }
  if (!(sqrt_s > msum) || !std::isfinite(sqrt_s)) return fail(MGME_EINVAL, "sqrt_s must exceed the final-state masses");
  a.seed = seed;
  a.first_event = first;
  const hipError_t e = mgme::launch_rambo(a, p->n_out, nevt, ld, d_mom, d_wgt, stream);
  if (e != hipSuccess) return hip_fail(e, "rambo launch");
  return MGME_OK;
}

// Good helicities: every helicity in FP64 on 64 RAMBO events; keep those with
// a non-zero contribution on at least one event.
int calibrate(mgme_process* p) {
  const int n_ext = p->entry->n_ext;
  const int nhel = 1 << n_ext;
  const long long nev = 64;
  double *d_mom = nullptr, *d_out = nullptr;
  hipError_t e = hipMalloc(&d_mom, sizeof(double) * 4 * n_ext * nev);
  if (e != hipSuccess) return fail(MGME_ENOMEM, "calibration buffer");
  e = hipMalloc(&d_out, sizeof(double) * nhel * nev);
  if (e != hipSuccess) {
    (void)hipFree(d_mom);
    return fail(MGME_ENOMEM, "calibration buffer");
  }
  int rc = MGME_OK;
  const double sqrt_s = p->entry->kind == mgme::KIND_EE ? 500.0 : 1500.0;
  std::vector<double> h((size_t)nhel * nev);
  mgme::MeArgs all = p->args;
  all.nhel = nhel;
  for (int i = 0; i < nhel; ++i) all.hel[i] = i;
  rc = launch_rambo_checked(p, sqrt_s, 1ull, 0ull, nev, nev, d_mom, nullptr, nullptr);
  if (rc == MGME_OK) {
    e = p->entry->launch(0, 1, d_mom, nev, nev, &all, d_out, nev, nullptr, nullptr, nullptr);
    if (e != hipSuccess) rc = hip_fail(e, "calibration launch");
  }
  if (rc == MGME_OK) {
    e = hipMemcpy(h.data(), d_out, sizeof(double) * nhel * nev, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "calibration copy");
  }
  (void)hipFree(d_mom);
  (void)hipFree(d_out);
  if (rc != MGME_OK) return rc;
  int ng = 0;
  for (int hh = 0; hh < nhel; ++hh) {
    bool good = false;
    for (long long ev = 0; ev < nev; ++ev)
      if (h[(size_t)hh * nev + ev] != 0.0) good = true;
    if (good) p->args.hel[ng++] = hh;
  }
  p->args.nhel = ng;
  return MGME_OK;
}

const mgme::ProcEntry* find_process(int n_ext, const int* pdg) {
  for (int i = 0; i < mgme::kNumProcesses; ++i) {
    const mgme::ProcEntry& e = mgme::kProcesses[i];
    if (e.n_ext != n_ext) continue;
    bool same = true;
    for (int k = 0; k < n_ext; ++k)
      if (e.pdg[k] != pdg[k]) same = false;
    if (same) return &e;
  }
  return nullptr;
}

int check_batch(const mgme_process* proc, const void* a, const void* b, long long nevt, long long ld) {
  if (!proc) return fail(MGME_EINVAL, "process is NULL");
  if (nevt < 0) return fail(MGME_EINVAL, "nevt < 0");
  if (ld < nevt) return fail(MGME_EINVAL, "ld < nevt");
  if (nevt > 0 && (!a || !b)) return fail(MGME_EINVAL, "NULL device pointer");
  if (nevt > (1ll << 31) * 64) return fail(MGME_EINVAL, "nevt too large");
  return MGME_OK;
}

}  // namespace

namespace mgme {

// Staging bytes per event of a launch (0: none), as the generated launchers
// lay them out without the helicity and colour choice.  The fused processes
// (at most 32 flows) form the mixed-precision colour sum inside the diagram
// kernel and stage nothing.
long long staging_per_event(const ProcEntry& e, int nhel, int prec) {
  if (e.staged) {
    const long long tsize = (prec == MGME_FP64 || prec == MGME_FP64_FP32COLOUR) ? 16 : 8;
    return (long long)nhel * ((e.n_colour + e.n_overflow) * tsize + 8);
  }
  if (prec == MGME_MIXED && e.n_colour > 32) return (long long)nhel * (e.n_colour * 8 + 8);
  return 0;
}

// Workspace bounds of the generated launchers: staged processes take up to
// 12 GB (at most 16384 events per sub-batch), the mixed-precision path of the
// other processes up to 4 GB.
long long workspace_bytes(const ProcEntry& e, int nhel, long long nevt, int prec) {
  if (nevt <= 0) return 0;
  const long long round64 = (nevt + 63) / 64 * 64;
  if (e.staged) {
    const long long per_event = staging_per_event(e, nhel, prec);
    long long sub = (12ll << 30) / per_event / 64 * 64;
    if (sub < 64) sub = 64;
    if (sub > 16384) sub = 16384;
    if (sub > round64) sub = round64;
    return per_event * sub;
  }
  if (prec == MGME_MIXED && e.n_colour > 32) {
    const long long per_event = staging_per_event(e, nhel, prec);
    long long sub = (4ll << 30) / per_event / 64 * 64;
    if (sub < 64) sub = 64;
    if (sub > round64) sub = round64;
    return per_event * sub;
  }
  return 0;
}

long long workspace_min_bytes(const mgme_process* proc, int precision) {
  return 64 * staging_per_event(*proc->entry, proc->args.nhel, precision);
}

int process_device(const mgme_process* proc) { return proc->device; }

int process_n_ext(const mgme_process* proc) { return proc->entry->n_ext; }

int set_error(int code, const char* msg) { return fail(code, msg); }

int matrix_element_ws(const mgme_process* proc, const double* d_mom, long long nevt, long long ld, int precision,
                      double* d_me, const Workspace* ws, hipStream_t stream) {
  int rc = check_batch(proc, d_mom, d_me, nevt, ld);
  if (rc != MGME_OK) return rc;
  if (!valid_precision(precision)) return fail(MGME_EINVAL, "unknown precision");
  if (ws && ws->ptr && ws->bytes < workspace_min_bytes(proc, precision))
    return fail(MGME_EINVAL, "workspace smaller than one 64-event sub-batch of the staging buffers");
  if ((rc = check_pending("mgme_matrix_element")) != MGME_OK) return rc;
  if (nevt == 0) return MGME_OK;
  if ((rc = select_device(proc->device)) != MGME_OK) return rc;
  const hipError_t e = proc->entry->launch(precision, 0, d_mom, nevt, ld, &proc->args, d_me, 0, nullptr, ws, stream);
  if (e != hipSuccess) return hip_fail(e, "matrix element launch");
  return MGME_OK;
}

}  // namespace mgme

extern "C" {

int mgme_workspace_bytes(const mgme_process* proc, long long nevt, int precision, long long* bytes) {
  if (!proc || !bytes || nevt < 0) return fail(MGME_EINVAL, "bad argument");
  if (!valid_precision(precision)) return fail(MGME_EINVAL, "unknown precision");
  *bytes = mgme::workspace_bytes(*proc->entry, proc->args.nhel, nevt, precision);
  return MGME_OK;
}

const char* mgme_last_error(void) { return g_error.c_str(); }

int mgme_process_create(int n_in, int n_out, const int* pdg, const mgme_params* params, int device,
                        mgme_process** out) {
  if (!out) return fail(MGME_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pdg || !params) return fail(MGME_EINVAL, "NULL argument");
  if (n_in != 2 || n_out < 2 || n_out > 5) return fail(MGME_EINVAL, "need 2 initial and 2..5 final particles");
  const mgme::ProcEntry* entry = find_process(n_in + n_out, pdg);
  if (!entry) return fail(MGME_EUNSUPPORTED, "process not supported");
  const mgme_params& P = *params;
  if (P.wt != 0.0) return fail(MGME_EUNSUPPORTED, "a non-zero top width is not supported");
  if (entry->kind == mgme::KIND_QCD && !(finite_pos(P.alpha_s) && finite_pos(P.mt)))
    return fail(MGME_EINVAL, "alpha_s and mt must be positive and finite");
  if (entry->kind == mgme::KIND_EE &&
      !(finite_pos(P.alpha_em) && finite_pos(P.sin2w) && P.sin2w < 1.0 && finite_pos(P.mz) &&
        std::isfinite(P.wz) && P.wz >= 0.0))
    return fail(MGME_EINVAL, "electroweak parameters out of range");
  int ndev = 0;
  hipError_t he = hipGetDeviceCount(&ndev);
  if (he != hipSuccess) return hip_fail(he, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(MGME_EINVAL, "no such device");
  int rc = select_device(device);
  if (rc != MGME_OK) return rc;

  mgme_process* p = new (std::nothrow) mgme_process();
  if (!p) return fail(MGME_ENOMEM, "host allocation");
  p->entry = entry;
  p->device = device;
  p->n_out = n_out;
  const double pi = 3.141592653589793238462643383279502884;
  for (int i = 0; i < n_out; ++i) p->mass_out[i] = std::abs(pdg[2 + i]) == 6 ? P.mt : 0.0;
  std::memset(&p->args, 0, sizeof p->args);
  p->args.mt = P.mt;
  p->norm_factor = 1.0 / ((double)entry->spin_colour_avg * (double)entry->ident);
  if (entry->kind == mgme::KIND_QCD) {
    p->gs = std::sqrt(4.0 * pi * P.alpha_s);
    p->args.factor = std::pow(p->gs, entry->gs_power) * p->norm_factor / (double)entry->cden;
  } else {
    const double e2 = 4.0 * pi * P.alpha_em;
    const double sw2 = P.sin2w, cw2 = 1.0 - sw2;
    p->args.factor = p->norm_factor;
    p->args.ee_qq = e2;  // Q_e Q_mu = 1
    p->args.ee_zz = e2 / (sw2 * cw2);
    p->args.ee_gl = -0.5 + sw2;
    p->args.ee_gr = sw2;
    p->args.mz = P.mz;
    p->args.wz = P.wz;
    p->args.z_enabled = P.z_enabled ? 1 : 0;
  }
  // colour matrix fragments for the matrix-core colour sum
  {
    int mt = 0, ks = 0;
    if (mgme::colour_mfma_tiles(entry->n_colour, &mt, &ks) != 0) {
      delete p;
      return fail(MGME_EUNSUPPORTED, "too many colour flows");
    }
    std::vector<unsigned short> frag((size_t)mt * ks * 64 * 8);
    mgme::colour_mfma_fragments(entry->n_colour, entry->colour_num, frag.data());
    he = hipMalloc(&p->d_cfrag, frag.size() * sizeof(unsigned short));
    if (he != hipSuccess) {
      delete p;
      return fail(MGME_ENOMEM, "colour fragments");
    }
    he = hipMemcpy(p->d_cfrag, frag.data(), frag.size() * sizeof(unsigned short), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
      (void)hipFree(p->d_cfrag);
      delete p;
      return hip_fail(he, "colour fragments");
    }
    p->args.cfrag = p->d_cfrag;
  }
  rc = calibrate(p);
  if (rc != MGME_OK) {
    (void)hipFree(p->d_cfrag);
    delete p;
    return rc;
  }
  p->n_good = p->args.nhel;
  for (int i = 0; i < p->n_good; ++i) p->good[i] = p->args.hel[i];
  *out = p;
  return MGME_OK;
}

int mgme_process_destroy(mgme_process* proc) {
  if (!proc) return MGME_OK;
  if (proc->d_cfrag) {
    int rc = select_device(proc->device);
    if (rc != MGME_OK) return rc;
    const hipError_t e = hipFree(proc->d_cfrag);
    proc->d_cfrag = nullptr;
    if (e != hipSuccess) {
      delete proc;
      return hip_fail(e, "hipFree");
    }
  }
  delete proc;
  return MGME_OK;
}

int mgme_process_info(const mgme_process* proc, mgme_info* out) {
  if (!proc || !out) return fail(MGME_EINVAL, "NULL argument");
  const mgme::ProcEntry& e = *proc->entry;
  out->n_ext = e.n_ext;
  out->n_diagrams = e.n_diagrams;
  out->n_amp_terms = e.n_terms;
  out->n_colour = e.n_colour;
  out->n_hel = 1 << e.n_ext;
  out->n_good_hel = proc->args.nhel;
  out->n_currents = e.n_currents;
  out->n_amp_vertices = e.n_amps;
  out->norm_factor = proc->norm_factor;
  out->flops_per_hel = e.flops_per_hel;
  out->flops_per_event = e.flops_per_event;
  out->kernel_hash = e.kernel_hash;
  return MGME_OK;
}

int mgme_good_helicities(const mgme_process* proc, int* codes, int* n) {
  if (!proc || !codes || !n) return fail(MGME_EINVAL, "NULL argument");
  for (int i = 0; i < proc->args.nhel; ++i) codes[i] = proc->args.hel[i];
  *n = proc->args.nhel;
  return MGME_OK;
}

int mgme_set_helicities(mgme_process* proc, const int* codes, int n) {
  if (!proc) return fail(MGME_EINVAL, "process is NULL");
  if (n == 0) {
    proc->args.nhel = proc->n_good;
    for (int i = 0; i < proc->n_good; ++i) proc->args.hel[i] = proc->good[i];
    return MGME_OK;
  }
  const int nall = 1 << proc->entry->n_ext;
  if (n < 0 || n > nall || n > MGME_MAX_HEL) return fail(MGME_EINVAL, "helicity count out of range");
  if (!codes) return fail(MGME_EINVAL, "codes is NULL");
  for (int i = 0; i < n; ++i) {
    if (codes[i] < 0 || codes[i] >= nall) return fail(MGME_EINVAL, "helicity code out of range");
    if (i > 0 && codes[i] <= codes[i - 1]) return fail(MGME_EINVAL, "helicity codes not increasing");
  }
  proc->args.nhel = n;
  for (int i = 0; i < n; ++i) proc->args.hel[i] = codes[i];
  return MGME_OK;
}

int mgme_colour_matrix(const mgme_process* proc, long long* num, long long* den, int* basis) {
  if (!proc) return fail(MGME_EINVAL, "NULL argument");
  const mgme::ProcEntry& e = *proc->entry;
  if (num)
    for (int i = 0; i < e.n_colour * e.n_colour; ++i) num[i] = e.colour_num[i];
  if (den) *den = e.cden;
  if (basis)
    for (int i = 0; i < e.n_colour * e.n_gluons; ++i) basis[i] = e.basis[i];
  return MGME_OK;
}

int mgme_rambo(const mgme_process* proc, double sqrt_s, unsigned long long seed, unsigned long long first_event,
               long long nevt, long long ld, double* d_mom, double* d_wgt, void* hip_stream) {
  int rc = check_batch(proc, d_mom, d_mom, nevt, ld);
  if (rc != MGME_OK) return rc;
  if ((rc = check_pending("mgme_rambo")) != MGME_OK) return rc;
  if (nevt == 0) return MGME_OK;
  if ((rc = select_device(proc->device)) != MGME_OK) return rc;
  return launch_rambo_checked(proc, sqrt_s, seed, first_event, nevt, ld, d_mom, d_wgt, (hipStream_t)hip_stream);
}

int mgme_matrix_element(const mgme_process* proc, const double* d_mom, long long nevt, long long ld, int precision,
                        double* d_me, void* hip_stream) {
  return mgme::matrix_element_ws(proc, d_mom, nevt, ld, precision, d_me, nullptr, (hipStream_t)hip_stream);
}

int mgme_matrix_element_per_helicity(const mgme_process* proc, const double* d_mom, long long nevt, long long ld,
                                     int precision, double* d_out, long long ldo, void* hip_stream) {
  int rc = check_batch(proc, d_mom, d_out, nevt, ld);
  if (rc != MGME_OK) return rc;
  if (ldo < nevt) return fail(MGME_EINVAL, "ldo < nevt");
  if (!valid_precision(precision)) return fail(MGME_EINVAL, "unknown precision");
  if ((rc = check_pending("mgme_matrix_element_per_helicity")) != MGME_OK) return rc;
  if (nevt == 0) return MGME_OK;
  if ((rc = select_device(proc->device)) != MGME_OK) return rc;
  mgme::MeArgs all = proc->args;
  all.nhel = 1 << proc->entry->n_ext;
  for (int i = 0; i < all.nhel; ++i) all.hel[i] = i;
  const hipError_t e =
      proc->entry->launch(precision, 1, d_mom, nevt, ld, &all, d_out, ldo, nullptr, nullptr, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "matrix element launch");
  return MGME_OK;
}

int mgme_select(const mgme_process* proc, const double* d_mom, long long nevt, long long ld, int precision,
                const double* d_r_hel, const double* d_r_col, double* d_me, int* d_hel, int* d_col,
                void* hip_stream) {
  int rc = check_batch(proc, d_mom, d_me, nevt, ld);
  if (rc != MGME_OK) return rc;
  if (nevt > 0 && (!d_r_hel || !d_r_col || !d_hel || !d_col)) return fail(MGME_EINVAL, "NULL argument");
  if (!valid_precision(precision)) return fail(MGME_EINVAL, "unknown precision");
  if ((rc = check_pending("mgme_select")) != MGME_OK) return rc;
  if (nevt == 0) return MGME_OK;
  if ((rc = select_device(proc->device)) != MGME_OK) return rc;
  const mgme::SelectArgs sel{d_r_hel, d_r_col, d_hel, d_col};
  const hipError_t e =
      proc->entry->launch(precision, 0, d_mom, nevt, ld, &proc->args, d_me, 0, &sel, nullptr, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "matrix element launch");
  return MGME_OK;
}

int mgme_event_weights(double sqrt_s, const double* d_wgt, const double* d_me, long long nevt, double* d_w,
                       double* d_stats, void* hip_stream) {
  if (nevt < 0) return fail(MGME_EINVAL, "nevt < 0");
  if (!d_stats || (nevt > 0 && (!d_wgt || !d_me))) return fail(MGME_EINVAL, "NULL argument");
  if (!std::isfinite(sqrt_s) || !(sqrt_s > 0.0)) return fail(MGME_EINVAL, "sqrt_s must be positive");
  int rc = check_pending("mgme_event_weights");
  if (rc != MGME_OK) return rc;
  const hipStream_t stream = (hipStream_t)hip_stream;
  double* part = nullptr;
  hipError_t e = hipMallocAsync((void**)&part, sizeof(double) * 3 * mgme::weights_partials(nevt), stream);
  if (e != hipSuccess) return hip_fail(e, "workspace");
  e = mgme::launch_event_weights(nevt, d_wgt, d_me, mgme::weight_factor(sqrt_s), d_w, part, d_stats, stream);
  const hipError_t fe = hipFreeAsync(part, stream);
  if (e != hipSuccess) return hip_fail(e, "event weights launch");
  if (fe != hipSuccess) return hip_fail(fe, "workspace");
  return MGME_OK;
}

int mgme_unweight(const double* d_w, const double* d_r, long long nevt, const double* d_w_ref, long long* d_idx,
                  long long* d_nkept, void* hip_stream) {
  if (nevt < 0) return fail(MGME_EINVAL, "nevt < 0");
  if (!d_w_ref || !d_nkept || (nevt > 0 && (!d_w || !d_r || !d_idx))) return fail(MGME_EINVAL, "NULL argument");
  int rc = check_pending("mgme_unweight");
  if (rc != MGME_OK) return rc;
  const hipStream_t stream = (hipStream_t)hip_stream;
  const long long nt = mgme::unweight_tiles(nevt);
  long long* tiles = nullptr;
  hipError_t e = hipMallocAsync((void**)&tiles, sizeof(long long) * 2 * (nt > 0 ? nt : 1), stream);
  if (e != hipSuccess) return hip_fail(e, "workspace");
  e = mgme::launch_unweight(nevt, d_w, d_r, d_w_ref, d_idx, d_nkept, tiles, stream);
  const hipError_t fe = hipFreeAsync(tiles, stream);
  if (e != hipSuccess) return hip_fail(e, "unweighting launch");
  if (fe != hipSuccess) return hip_fail(fe, "workspace");
  return MGME_OK;
}

}  // extern "C"
