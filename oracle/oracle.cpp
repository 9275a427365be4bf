// Oracle C API (test infrastructure only); see oracle.h.
#include "oracle.h"

#include <cstring>
#include <exception>
#include <string>
#include <thread>
#include <vector>

#include "events.hpp"
#include "lorentz.hpp"
#include "philox_rambo.hpp"
#include "process.hpp"

static thread_local std::string g_err;

extern "C" {

const char* oracle_last_error(void) { return g_err.c_str(); }

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  oracle::philox4x32_10(ctr, key, out);
}

void oracle_uniform_pair(uint64_t seed, uint64_t event, uint32_t block, double out[2]) {
  oracle::uniform_pair(seed, event, block, out);
}

int oracle_rambo(int n_out, const double* masses_out, double sqrt_s, uint64_t seed,
                 uint64_t first_event, int64_t nevt, double* mom, double* wgt) {
  if (n_out < 2 || n_out > 6 || nevt < 0) return -1;
  const int n_ext = n_out + 2;
  for (int64_t e = 0; e < nevt; ++e) {
    double* pe = mom + (size_t)e * n_ext * 4;
    const double h = 0.5 * sqrt_s;
    const double p1[4] = {h, 0, 0, h}, p2[4] = {h, 0, 0, -h};
    std::memcpy(pe, p1, sizeof p1);
    std::memcpy(pe + 4, p2, sizeof p2);
    double w = oracle::rambo_event(n_out, masses_out, sqrt_s, seed, first_event + (uint64_t)e,
                                   reinterpret_cast<double(*)[4]>(pe + 8));
    if (wgt) wgt[e] = w;
  }
  return 0;
}

int oracle_external(int kind, const double p[4], double mass, int hel, double* out) {
  using namespace oracle;
  std::array<std::complex<double>, 4> v;
  switch (kind) {
    case 0: v = spinor_u<double>(p, mass, hel); break;
    case 1: v = spinor_v<double>(p, mass, hel); break;
    case 2: v = dirac_bar(spinor_u<double>(p, mass, hel)); break;
    case 3: v = dirac_bar(spinor_v<double>(p, mass, hel)); break;
    case 4: v = polarisation<double>(p, hel); break;
    default: return -1;
  }
  for (int i = 0; i < 4; ++i) {
    out[2 * i] = v[i].real();
    out[2 * i + 1] = v[i].imag();
  }
  return 0;
}

void* oracle_process_new(int n_ext, const int* pdg, const oracle_params* p) {
  try {
    oracle::Params par{p->alpha_s, p->alpha_em, p->sin2w, p->mz, p->wz, p->mt, p->wt, p->z_enabled};
    return new oracle::Process(n_ext, pdg, par);
  } catch (const std::exception& e) {
    g_err = e.what();
    return nullptr;
  }
}

void oracle_process_free(void* proc) { delete static_cast<oracle::Process*>(proc); }

int oracle_process_info(void* proc, long long info[5]) {
  auto* P = static_cast<oracle::Process*>(proc);
  info[0] = P->n_diagrams;
  info[1] = (long long)P->terms.size();
  info[2] = P->ncol;
  info[3] = P->n_hel;
  info[4] = P->cden;
  return 0;
}

int oracle_colour_matrix(void* proc, long long* num, int* basis) {
  auto* P = static_cast<oracle::Process*>(proc);
  for (size_t i = 0; i < P->cnum.size(); ++i) num[i] = P->cnum[i];
  int k = 0;
  for (auto& b : P->basis)
    for (int leg : b) basis[k++] = leg;
  return 0;
}

int oracle_me(void* proc, const double* mom, int64_t nevt, int colour_mode, int precision,
              int nthreads, double* me) {
  auto* P = static_cast<oracle::Process*>(proc);
  try {
    if (colour_mode == 1) P->build_full_colour_table();
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
  if (nthreads < 1) nthreads = 1;
  const size_t stride = (size_t)P->n_ext * 4;
  auto work = [&](int64_t begin, int64_t end) {
    for (int64_t e = begin; e < end; ++e) {
      const double* m = mom + (size_t)e * stride;
      if (colour_mode == 1) me[e] = P->me_brute(m);
      else if (precision == 1) me[e] = (double)P->me<long double>(m);
      else me[e] = P->me<double>(m);
    }
  };
  if (nthreads == 1 || nevt < 2) {
    work(0, nevt);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) {
      const int64_t b = nevt * t / nthreads, e = nevt * (t + 1) / nthreads;
      th.emplace_back(work, b, e);
    }
    for (auto& x : th) x.join();
  }
  return 0;
}

int oracle_me_hel(void* proc, const double* mom, int precision, double* me_hel) {
  auto* P = static_cast<oracle::Process*>(proc);
  if (precision == 1) {
    std::vector<long double> h(P->n_hel);
    P->me_hel<long double>(mom, h.data());
    for (int i = 0; i < P->n_hel; ++i) me_hel[i] = (double)h[i];
  } else {
    P->me_hel<double>(mom, me_hel);
  }
  return 0;
}

int oracle_condition(void* proc, const double* mom, double* kappa) {
  auto* P = static_cast<oracle::Process*>(proc);
  *kappa = (double)P->condition(mom);
  return 0;
}

int oracle_gauge(void* proc, const double* mom, int leg, double out[2]) {
  auto* P = static_cast<oracle::Process*>(proc);
  if (P->kind != oracle::Process::GG_TT_NG || leg < 0 || leg >= P->n_ext || P->pdg[leg] != 21) return -1;
  const auto ev = P->make_event<double>(mom);
  std::vector<std::complex<double>> amp, J;
  double mx_rep = 0, mx = 0;
  for (int h = 0; h < P->n_hel; ++h) {
    P->term_amplitudes(ev, h, leg, amp);
    P->flows(amp, J);
    for (auto& j : J) mx_rep = std::max(mx_rep, std::abs(j));
    P->term_amplitudes(ev, h, -1, amp);
    P->flows(amp, J);
    for (auto& j : J) mx = std::max(mx, std::abs(j));
  }
  out[0] = mx_rep;
  out[1] = mx;
  return 0;
}

int oracle_flows(void* proc, const double* mom, int hel, double* J) {
  auto* P = static_cast<oracle::Process*>(proc);
  if (hel < 0 || hel >= P->n_hel) return -1;
  const auto ev = P->make_event<double>(mom);
  std::vector<std::complex<double>> amp, flows;
  P->term_amplitudes(ev, hel, -1, amp);
  P->flows(amp, flows);
  for (int s = 0; s < P->ncol; ++s) {
    J[2 * s] = flows[s].real();
    J[2 * s + 1] = flows[s].imag();
  }
  return 0;
}

int oracle_event_weights(int64_t nevt, const double* wgt, const double* me, double sqrt_s, double* w,
                         double stats[3]) {
  if (nevt < 0 || !(sqrt_s > 0)) return -1;
  oracle::event_weights(nevt, wgt, me, sqrt_s, w);
  oracle::weight_stats(nevt, w, stats);
  return 0;
}

int64_t oracle_unweight(int64_t nevt, const double* w, const double* r, double w_ref, int64_t* idx) {
  if (nevt < 0) return -1;
  return oracle::unweight(nevt, w, r, w_ref, idx);
}

int oracle_select(void* proc, const double* mom, double r_hel, double r_col, int out[2], double margin[2]) {
  auto* P = static_cast<oracle::Process*>(proc);
  const auto ev = P->make_event<double>(mom);
  std::vector<std::complex<double>> amp, J;
  std::vector<double> me_h(P->n_hel), jamp2(P->ncol, 0.0);
  for (int h = 0; h < P->n_hel; ++h) {
    P->term_amplitudes(ev, h, -1, amp);
    P->flows(amp, J);
    me_h[h] = P->colour_sum(J) * P->norm;
    for (int s = 0; s < P->ncol; ++s) jamp2[s] += std::norm(J[s]);
  }
  out[0] = oracle::choose(me_h, r_hel, &margin[0]);
  out[1] = oracle::choose(jamp2, r_col, &margin[1]);
  return 0;
}

}  // extern "C"
