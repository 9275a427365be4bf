// Sanitizer driver for the oracle (test infrastructure): every entry point of
// oracle.h on a few RAMBO events of each process, built together with
// oracle/oracle.cpp under AddressSanitizer and UndefinedBehaviorSanitizer.
// Exits 0 when every result is finite and the cross-checks hold; the
// sanitizers report on stderr and fail the run on their own.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../oracle/oracle.h"

static int g_fail = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      g_fail = 1;                                                         \
    }                                                                     \
  } while (0)

int main() {
  const oracle_params par{0.118, 1.0 / 132.5, 0.2222, 91.188, 2.441, 173.0, 0.0, 1};
  struct Case {
    std::vector<int> pdg;
    double sqrt_s;
    int nevt;
    bool brute;
  };
  const Case cases[] = {{{-11, 11, -13, 13}, 500.0, 8, true},
                        {{21, 21, 6, -6}, 1500.0, 8, true},
                        {{21, 21, 6, -6, 21}, 1500.0, 4, true},
                        {{21, 21, 6, -6, 21, 21}, 1500.0, 2, false},
                        {{21, 21, 6, -6, 21, 21, 21}, 1500.0, 1, false}};
  uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0}, out[4];
  oracle_philox4x32_10(ctr, key, out);
  double u[2];
  oracle_uniform_pair(230318244ull, 5, 3, u);
  CHECK(u[0] > 0 && u[0] < 1 && u[1] > 0 && u[1] < 1);
  double ext[8];
  const double p[4] = {200.0, 30.0, -40.0, 120.0};
  for (int kind = 0; kind < 5; ++kind) CHECK(oracle_external(kind, p, kind < 4 ? 50.0 : 0.0, 1, ext) == 0);
  for (const Case& c : cases) {
    const int n_ext = (int)c.pdg.size();
    std::vector<double> masses;
    for (int i = 2; i < n_ext; ++i) masses.push_back(std::abs(c.pdg[i]) == 6 ? 173.0 : 0.0);
    std::vector<double> mom((size_t)c.nevt * n_ext * 4), wgt(c.nevt), me(c.nevt), me2(c.nevt), me_ld(c.nevt);
    CHECK(oracle_rambo(n_ext - 2, masses.data(), c.sqrt_s, 230318244ull, 0, c.nevt, mom.data(), wgt.data()) == 0);
    void* P = oracle_process_new(n_ext, c.pdg.data(), &par);
    CHECK(P != nullptr);
    if (!P) continue;
    long long info[5];
    CHECK(oracle_process_info(P, info) == 0);
    const long long ncol = info[2], nhel = info[3];
    std::vector<long long> num((size_t)(ncol * ncol));
    std::vector<int> basis((size_t)(ncol * 8));
    CHECK(oracle_colour_matrix(P, num.data(), basis.data()) == 0);
    CHECK(oracle_me(P, mom.data(), c.nevt, 0, 0, 2, me.data()) == 0);
    CHECK(oracle_me(P, mom.data(), c.nevt, 0, 1, 1, me_ld.data()) == 0);
    if (c.brute) {
      CHECK(oracle_me(P, mom.data(), c.nevt, 1, 0, 1, me2.data()) == 0);
      for (int e = 0; e < c.nevt; ++e) CHECK(std::fabs(me2[e] / me[e] - 1.0) < 1e-12);
    }
    for (int e = 0; e < c.nevt; ++e) {
      CHECK(std::isfinite(me[e]) && me[e] > 0.0);
      CHECK(std::fabs(me_ld[e] / me[e] - 1.0) < 1e-10);
    }
    std::vector<double> mh((size_t)nhel), J((size_t)(2 * ncol));
    CHECK(oracle_me_hel(P, mom.data(), 0, mh.data()) == 0);
    double sum = 0.0;
    for (double x : mh) sum += x;
    CHECK(std::fabs(sum / me[0] - 1.0) < 1e-12);
    CHECK(oracle_flows(P, mom.data(), (int)(nhel - 1), J.data()) == 0);
    int choice[2];
    double margin[2];
    CHECK(oracle_select(P, mom.data(), 0.37, 0.61, choice, margin) == 0);
    CHECK(choice[0] >= 0 && choice[0] < nhel && choice[1] >= 0 && choice[1] < ncol);
    if (c.pdg[0] == 21 && n_ext <= 6) {
      double g[2];
      CHECK(oracle_gauge(P, mom.data(), n_ext - 1 >= 4 ? n_ext - 1 : 0, g) == 0);
      CHECK(g[0] <= 1e-11 * 1500.0 * g[1]);
      CHECK(oracle_gauge(P, mom.data(), n_ext, g) != 0);  // no such leg
      CHECK(oracle_gauge(P, mom.data(), 2, g) != 0);      // not a gluon
    }
    std::vector<double> w(c.nevt), r(c.nevt, 0.5);
    double stats[3];
    CHECK(oracle_event_weights(c.nevt, wgt.data(), me.data(), c.sqrt_s, w.data(), stats) == 0);
    std::vector<int64_t> idx(c.nevt);
    const int64_t kept = oracle_unweight(c.nevt, w.data(), r.data(), stats[2], idx.data());
    CHECK(kept >= 1 && kept <= c.nevt);
    oracle_process_free(P);
  }
  // unsupported process and bad arguments
  const int bad[4] = {1, 2, 3, 4};
  CHECK(oracle_process_new(4, bad, &par) == nullptr);
  CHECK(oracle_last_error() != nullptr);
  if (!g_fail) std::printf("oracle driver: all checks passed\n");
  return g_fail;
}
