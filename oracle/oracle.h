/* Oracle C API (test infrastructure only).
 *
 * A plain, slow CPU implementation of what the GPU path computes, used only
 * by the tests, the smoke check and the CPU-baseline leg of the benchmark.
 * It shares no code with the GPU library.  Momenta are host arrays laid out
 * [event][particle][mu] with mu = (E, px, py, pz) in GeV; particles in the
 * order of the pdg list (initial state first).
 *
 * Parity pins and their tests live under tests/ (see test_oracle_*.py).
 */
#ifndef MGME_ORACLE_H
#define MGME_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double alpha_s, alpha_em, sin2w, mz, wz, mt, wt;
  int z_enabled;
} oracle_params;

/* Philox4x32-10 block function. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Two uniforms in (0,1) from block `block` of event `event`. */
void oracle_uniform_pair(uint64_t seed, uint64_t event, uint32_t block, double out[2]);
/* RAMBO events first_event .. first_event+nevt-1.  mom: [nevt][n_out+2][4]
 * (two initial partons along +z and -z with energy sqrt_s/2 first), wgt: [nevt]. */
int oracle_rambo(int n_out, const double* masses_out, double sqrt_s, uint64_t seed,
                 uint64_t first_event, int64_t nevt, double* mom, double* wgt);

/* External states (for the spinor and polarisation pins).
 * kind: 0 u, 1 v, 2 ubar, 3 vbar, 4 polarisation vector.  out: 8 doubles
 * (re, im of four components). */
int oracle_external(int kind, const double p[4], double mass, int hel, double* out);

/* Processes: returns NULL if unsupported; error text in oracle_last_error(). */
void* oracle_process_new(int n_ext, const int* pdg, const oracle_params* p);
void oracle_process_free(void* proc);
const char* oracle_last_error(void);
/* info: n_diagrams, n_terms, n_colour, n_hel, colour denominator */
int oracle_process_info(void* proc, long long info[5]);
/* Colour matrix numerators (n_colour^2) and the basis (n_colour x n_gluons legs). */
int oracle_colour_matrix(void* proc, long long* num, int* basis);

/* |M|^2 per event.  colour_mode: 0 colour-decomposed, 1 brute-force explicit
 * colour sum (up to four gluons).  precision: 0 double, 1 long double. */
int oracle_me(void* proc, const double* mom, int64_t nevt, int colour_mode, int precision,
              int nthreads, double* me);
/* Per-helicity colour-summed |M_h|^2 for one event (n_hel values). */
int oracle_me_hel(void* proc, const double* mom, int precision, double* me_hel);
/* Condition number of |M|^2 for one event: the helicity- and colour-summed
 * square with every diagram amplitude, colour coefficient and colour-matrix
 * entry replaced by its absolute value, over |M|^2 (long double inside).
 * Relative changes of at most eps in every amplitude change |M|^2 by at most
 * about 2 eps kappa relative; it scales the FP64 rounding of an event. */
int oracle_condition(void* proc, const double* mom, double* kappa);
/* Gauge test: replace the polarisation of gluon `leg` by its momentum.
 * out[0] = max over helicities and flows of |J_s| with the replacement,
 * out[1] = the same maximum without it. */
int oracle_gauge(void* proc, const double* mom, int leg, double out[2]);

/* Colour-ordered amplitudes J_s (n_colour complex values, re/im
 * interleaved, basis order of oracle_colour_matrix) of helicity `hel` for
 * one event: i times the colour-stripped amplitude, couplings included,
 * before the averaging and symmetry factor. */
int oracle_flows(void* proc, const double* mom, int hel, double* J);
/* Cross-section weights w[e] = (wgt[e] * me[e]) * (0.3893793721e9 / (2 s)) in
 * pb for massless colliding partons, and stats = (sum w, sum w^2, max w). */
int oracle_event_weights(int64_t nevt, const double* wgt, const double* me, double sqrt_s, double* w,
                         double stats[3]);
/* Hit-or-miss unweighting: indices e with r[e] * w_ref < w[e], increasing;
 * returns their number. */
int64_t oracle_unweight(int64_t nevt, const double* w, const double* r, double w_ref, int64_t* idx);
/* Helicity and leading-colour choice for one event: out[0] = helicity code
 * (chosen with probability |M_h|^2 / |M|^2, helicities in code order),
 * out[1] = colour flow in basis order (probability proportional to
 * sum_h |J_s(h)|^2); margin[i] = distance of the threshold to the nearest
 * running sum, relative to the total. */
int oracle_select(void* proc, const double* mom, double r_hel, double r_col, int out[2], double margin[2]);

#ifdef __cplusplus
}
#endif
#endif
