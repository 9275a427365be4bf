// Sanitizer driver for the serving scheduler (test infrastructure).  Links
// csrc/serve.cpp with stand-ins for the library calls that only the device
// executor makes, and drives the test double (no GPU): several submitting
// threads, splitting of oversize requests, injected failures, bounded
// pass-over, and destruction with work still queued.  Exits 0 when every
// check holds; ThreadSanitizer or AddressSanitizer report on stderr and fail
// the run on their own.
#include <cstdio>
#include <thread>
#include <vector>

#include "../../include/mgme.h"
#include "../../paper_2303_18244_amd/csrc/internal.h"

// Stand-ins: the test double never reaches them.
extern "C" int mgme_matrix_element(const mgme_process*, const double*, long long, long long, int, double*, void*) {
  return MGME_EUNSUPPORTED;
}
extern "C" int mgme_workspace_bytes(const mgme_process*, long long, int, long long* b) {
  *b = 0;
  return MGME_OK;
}
namespace mgme {
int matrix_element_ws(const mgme_process*, const double*, long long, long long, int, double*, const Workspace*,
                      hipStream_t) {
  return MGME_EUNSUPPORTED;
}
long long workspace_min_bytes(const mgme_process*, int) { return 0; }
int process_device(const mgme_process*) { return 0; }
int process_n_ext(const mgme_process*) { return 4; }
int set_error(int code, const char*) { return code; }
}  // namespace mgme

static int g_fail = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      g_fail = 1;                                                  \
    }                                                              \
  } while (0)

static mgme_server_config fake(int slots, long long budget, double ns, long long bytes, long long fail_n) {
  mgme_server_config c{};
  c.n_slots = slots;
  c.hbm_budget_bytes = budget;
  c.fake_executor = 1;
  c.fake_ns_per_event = ns;
  c.fake_bytes_per_event = bytes;
  c.fake_fail_nevt = fail_n;
  return c;
}

int main() {
  // several threads submitting and waiting at once, with splits and failures
  {
    mgme_server_config c = fake(3, 20000, 200.0, 10, 333);
    mgme_server* s = nullptr;
    CHECK(mgme_server_create(&c, 0, &s) == MGME_OK);
    std::vector<std::thread> th;
    std::vector<int> bad(4, 0), ok(4, 0);
    for (int k = 0; k < 4; ++k)
      th.emplace_back([&, k] {
        for (int j = 0; j < 25; ++j) {
          const long long n = (j % 5 == 0) ? 333 : (j % 7 == 0 ? 5000 : 100 + 37 * ((k * 25 + j) % 40));
          unsigned long long id = 0;
          if (mgme_server_submit(s, nullptr, nullptr, n, n, 0, nullptr, nullptr, &id) != MGME_OK) continue;
          double lat = 0;
          const int rc = mgme_server_wait(s, id, &lat);
          if (rc == MGME_OK) ok[k]++;
          else bad[k]++;
          mgme_server_stats st;
          (void)mgme_server_get_stats(s, &st);
        }
      });
    for (auto& t : th) t.join();
    mgme_server_stats st;
    CHECK(mgme_server_get_stats(s, &st) == MGME_OK);
    int nok = 0, nbad = 0;
    for (int k = 0; k < 4; ++k) {
      nok += ok[k];
      nbad += bad[k];
    }
    CHECK(nbad == 20 && nok == 80);
    CHECK(st.completed == 80 && st.failed == 20);
    CHECK(st.split_requests > 0 && st.peak_footprint_bytes <= 20000);
    CHECK(mgme_server_destroy(s) == MGME_OK);
  }
  // bounded pass-over under a stream of small requests
  {
    mgme_server_config c = fake(4, 100, 1e5, 1, 0);
    c.max_pass_over = 2;
    mgme_server* s = nullptr;
    CHECK(mgme_server_create(&c, 0, &s) == MGME_OK);
    std::vector<unsigned long long> ids;
    unsigned long long id = 0, big = 0;
    for (int i = 0; i < 3; ++i) {
      CHECK(mgme_server_submit(s, nullptr, nullptr, 30, 30, 0, nullptr, nullptr, &id) == MGME_OK);
      ids.push_back(id);
    }
    CHECK(mgme_server_submit(s, nullptr, nullptr, 90, 90, 0, nullptr, nullptr, &big) == MGME_OK);
    for (int i = 0; i < 40; ++i) {
      CHECK(mgme_server_submit(s, nullptr, nullptr, 30, 30, 0, nullptr, nullptr, &id) == MGME_OK);
      ids.push_back(id);
    }
    CHECK(mgme_server_wait(s, big, nullptr) == MGME_OK);
    for (auto x : ids) CHECK(mgme_server_wait(s, x, nullptr) == MGME_OK);
    CHECK(mgme_server_drain(s) == MGME_OK);
    CHECK(mgme_server_destroy(s) == MGME_OK);
  }
  // destruction with requests still queued (never waited for)
  {
    mgme_server_config c = fake(1, 0, 1e4, 0, 0);
    mgme_server* s = nullptr;
    CHECK(mgme_server_create(&c, 0, &s) == MGME_OK);
    unsigned long long id = 0;
    for (int i = 0; i < 10; ++i) CHECK(mgme_server_submit(s, nullptr, nullptr, 100, 100, 0, nullptr, nullptr, &id) == MGME_OK);
    CHECK(mgme_server_destroy(s) == MGME_OK);
  }
  if (!g_fail) std::printf("serve driver: all checks passed\n");
  return g_fail;
}
