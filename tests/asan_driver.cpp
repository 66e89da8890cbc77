// Host-side checks of the C ABI, run against a build of the library whose
// host code carries AddressSanitizer (tests/test_host_asan.py builds both).
// Only calls that must return before any device work are made: argument and
// option validation, NULL contexts, and the failure path of dmpt_init on a
// device ordinal that does not exist (it must free what it allocated).
#include <cstdio>
#include <cstring>

#include "dmpt.h"

static int bad = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s\n", what);
    bad = 1;
  }
}

int main() {
  dmpt_options o;
  dmpt_ctx h = nullptr;
  dmpt_stats st;
  expect(dmpt_init(nullptr, 0, 128, 1, nullptr, nullptr) == DMPT_ERR_ARG, "init without an output pointer");
  expect(dmpt_init(&h, 0, 0, 1, nullptr, nullptr) == DMPT_ERR_ARG && !h, "n_max = 0");
  expect(std::strstr(dmpt_last_error(nullptr), "n_max") != nullptr, "error text names n_max");
  expect(dmpt_init(&h, 0, 128, 99, nullptr, nullptr) == DMPT_ERR_ARG && !h, "dirs_max = 99");
  struct Bad {
    const char* what;
    void (*set)(dmpt_options*);
  } opts[] = {
      {"unknown precision", [](dmpt_options* p) { p->prec = (dmpt_prec)17; }},
      {"refine 5", [](dmpt_options* p) { p->refine = 5; }},
      {"schedule 9", [](dmpt_options* p) { p->schedule = 9; }},
      {"max_cg 1000", [](dmpt_options* p) { p->max_cg = 1000; }},
      {"acc64 3", [](dmpt_options* p) { p->acc64 = 3; }},
      {"grouped 2", [](dmpt_options* p) { p->grouped = 2; }},
      {"unknown solver", [](dmpt_options* p) { p->solver = (dmpt_solver)7; }},
  };
  for (const Bad& b : opts) {
    dmpt_default_options(&o);
    b.set(&o);
    expect(dmpt_init(&h, 0, 128, 1, &o, nullptr) == DMPT_ERR_ARG && !h, b.what);
  }
  // every entry point rejects a NULL context
  expect(dmpt_fermi_recursion(nullptr, 4, nullptr, 1.0, 0.0, 10, nullptr, &st) == DMPT_ERR_ARG, "fermi NULL");
  expect(dmpt_mu_newton(nullptr, 4, nullptr, 0, nullptr, nullptr, nullptr, 1.0, 2.0, 10, 0, nullptr, nullptr,
                        nullptr, nullptr, nullptr, nullptr) == DMPT_ERR_ARG, "mu_newton NULL");
  expect(dmpt_backward(nullptr, 4, nullptr, 1.0, 2.0, 10, nullptr, nullptr, nullptr, nullptr) == DMPT_ERR_ARG,
         "backward NULL");
  expect(dmpt_congruence(nullptr, 4, nullptr, nullptr, nullptr, 0, nullptr) == DMPT_ERR_ARG, "congruence NULL");
  expect(dmpt_finalize(nullptr) == DMPT_OK, "finalize NULL");
  // a device ordinal that does not exist: the error path of dmpt_init
  dmpt_default_options(&o);
  const dmpt_status r = dmpt_init(&h, 4096, 256, 2, &o, nullptr);
  expect(r != DMPT_OK && !h, "device 4096 is refused and leaves no context");
  expect(std::strlen(dmpt_last_error(nullptr)) > 0, "and says why");
  std::printf("asan driver: %s\n", bad ? "failures" : "ok");
  return bad;
}
