// Host-side checks of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; no GPU needed): every
// invalid-problem path of dot_plan_create, the host coarsening of
// dot_coarsen_data (mass kept, odd counts rejected), dot_footprint_bytes,
// destroy calls on null handles and argument checks of the batch, schedule,
// checkpoint and promotion calls. Exit status 0 when every expectation holds;
// the sanitizers abort on a memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "dotsocp.h"

static int g_failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s (last error: %s)\n", what, dot_last_error());
    ++g_failures;
  }
}

struct Data {
  std::vector<double> r0, r1;
  std::vector<uint8_t> mask;
};

static dot_problem base_problem(Data& d, int D, const int* n, bool masked) {
  dot_problem p;
  std::memset(&p, 0, sizeof(p));
  p.D = D;
  int64_t nx = 1;
  for (int a = 0; a <= D; ++a) p.n[a] = n[a];
  for (int a = 1; a <= D; ++a) nx *= n[a] + 1;
  std::mt19937_64 rng(1234);
  std::uniform_real_distribution<double> u(0.1, 1.0);
  d.r0.assign(nx, 0.0);
  d.r1.assign(nx, 0.0);
  double s0 = 0, s1 = 0;
  for (int64_t i = 0; i < nx; ++i) {
    d.r0[i] = u(rng);
    d.r1[i] = u(rng);
    s0 += d.r0[i];
    s1 += d.r1[i];
  }
  for (int64_t i = 0; i < nx; ++i) {
    d.r0[i] /= s0;
    d.r1[i] /= s1;
  }
  if (masked) {
    d.mask.assign(nx, 0);
    for (int64_t i = 0; i < nx; i += 7) d.mask[i] = 1;
  }
  p.rho0 = d.r0.data();
  p.rho1 = d.r1.data();
  p.mask = masked ? d.mask.data() : nullptr;
  p.tol = 1e-6;
  p.max_iter = 100;
  p.precision = DOT_FP64;
  return p;
}

static void check_invalid_problems() {
  const int n[3] = {4, 6, 5};
  Data d;
  dot_plan* P = nullptr;
  expect(dot_plan_create(nullptr, &P) == DOT_EINVAL, "null problem");
  dot_problem p = base_problem(d, 2, n, false);
  expect(dot_plan_create(&p, nullptr) == DOT_EINVAL, "null output");
  auto rejects = [&](void (*edit)(dot_problem&, Data&), const char* what) {
    Data dd;
    dot_problem q = base_problem(dd, 2, n, false);
    edit(q, dd);
    dot_plan* out = reinterpret_cast<dot_plan*>(0x1);
    const int rc = dot_plan_create(&q, &out);
    expect(rc == DOT_EINVAL, what);
    expect(out == nullptr, "output cleared on error");
    expect(std::strlen(dot_last_error()) > 0, "error message set");
  };
  rejects([](dot_problem& q, Data&) { q.D = 0; }, "D = 0");
  rejects([](dot_problem& q, Data&) { q.D = 4; }, "D = 4");
  rejects([](dot_problem& q, Data&) { q.n[1] = 0; }, "zero segments");
  rejects([](dot_problem& q, Data&) { q.n[0] = 5000; }, "too many segments");
  rejects([](dot_problem& q, Data&) { q.rho0 = nullptr; }, "null rho0");
  rejects([](dot_problem& q, Data& dd) { dd.r0[3] = -1e-3; }, "negative mass");
  rejects([](dot_problem& q, Data& dd) { dd.r1[5] = std::numeric_limits<double>::quiet_NaN(); }, "NaN mass");
  rejects([](dot_problem& q, Data& dd) { dd.r1[5] = std::numeric_limits<double>::infinity(); }, "Inf mass");
  rejects([](dot_problem& q, Data& dd) { dd.r1[0] += 1e-6; }, "mass mismatch");
  rejects([](dot_problem& q, Data& dd) {
    for (auto& v : dd.r0) v = 0.0;
    for (auto& v : dd.r1) v = 0.0;
  }, "zero total mass");
  rejects([](dot_problem& q, Data&) { q.precision = 7; }, "unknown precision");
  rejects([](dot_problem& q, Data&) { q.tau = 2.0; }, "tau = 2");
  rejects([](dot_problem& q, Data&) { q.sigma0 = -1.0; }, "negative sigma0");
  rejects([](dot_problem& q, Data&) { q.check_every = -5; }, "negative cadence");
  rejects([](dot_problem& q, Data&) { q.max_iter = -1; }, "negative max_iter");
  rejects([](dot_problem& q, Data&) { q.time_limit_s = -1.0; }, "negative time budget");
  rejects([](dot_problem& q, Data&) { q.time_limit_s = std::numeric_limits<double>::infinity(); },
          "infinite time budget");
}

static void check_coarsening() {
  const int shapes[3][4] = {{8, 16, 0, 0}, {4, 10, 6, 0}, {2, 4, 6, 8}};
  for (int D = 1; D <= 3; ++D) {
    for (int masked = 0; masked <= 1; ++masked) {
      Data d;
      dot_problem p = base_problem(d, D, shapes[D - 1], masked != 0);
      int64_t nc = 1;
      for (int a = 1; a <= D; ++a) nc *= shapes[D - 1][a] / 2 + 1;
      std::vector<double> c0(nc, -1.0), c1(nc, -1.0);
      std::vector<uint8_t> cm(nc, 9);
      const int rc = dot_coarsen_data(D, p.n, p.rho0, p.rho1, p.mask, c0.data(), c1.data(),
                                      masked ? cm.data() : nullptr);
      expect(rc == DOT_OK, "coarsen");
      double s0 = 0, s1 = 0;
      bool nonneg = true;
      for (int64_t i = 0; i < nc; ++i) {
        s0 += c0[i];
        s1 += c1[i];
        nonneg = nonneg && c0[i] >= 0 && c1[i] >= 0;
        if (masked) nonneg = nonneg && cm[i] <= 1 && (!cm[i] || (c0[i] == 0 && c1[i] == 0));
      }
      expect(nonneg, "coarse data non-negative, zero on coarse obstacle nodes");
      expect(std::fabs(s0 - 1.0) < 1e-12 && std::fabs(s1 - 1.0) < 1e-12, "coarse masses kept");
    }
  }
  Data d;
  const int odd[3] = {4, 7, 6};
  dot_problem p = base_problem(d, 2, odd, false);
  std::vector<double> o0(64), o1(64);
  expect(dot_coarsen_data(2, p.n, p.rho0, p.rho1, nullptr, o0.data(), o1.data(), nullptr) == DOT_EINVAL,
         "odd segment count rejected");
  expect(dot_coarsen_data(2, p.n, nullptr, p.rho1, nullptr, o0.data(), o1.data(), nullptr) == DOT_EINVAL,
         "null input rejected");
}

static void check_footprint_and_null_handles() {
  Data d;
  const int small[3] = {4, 6, 5}, large[3] = {8, 12, 10};
  dot_problem a = base_problem(d, 2, small, false);
  const size_t fa = dot_footprint_bytes(&a);
  Data e;
  dot_problem b = base_problem(e, 2, large, false);
  const size_t fb = dot_footprint_bytes(&b);
  expect(fa > 0 && fb > fa, "footprint grows with the grid");
  b.precision = DOT_MIXED;
  expect(dot_footprint_bytes(&b) < fb, "mixed precision needs less");
  expect(dot_footprint_bytes(nullptr) == 0, "null footprint");
  dot_plan_destroy(nullptr);
  dot_batch_destroy(nullptr);
  dot_ctx_destroy(nullptr);
  dot_schedule s;
  expect(dot_plan_get_schedule(nullptr, &s) == DOT_EINVAL, "schedule of a null plan");
  expect(dot_plan_set_schedule(nullptr, nullptr) == DOT_EINVAL, "set schedule on a null plan");
  expect(dot_batch_get_schedule(nullptr, &s) == DOT_EINVAL, "schedule of a null batch");
  double q = 0, al = 0, be = 0, sg = 0;
  expect(dot_state_export(nullptr, nullptr, &q, &al, &be, &sg, nullptr) == DOT_EINVAL, "export on a null plan");
  expect(dot_state_import(nullptr, nullptr, &q, &al, &be, 1.0, nullptr) == DOT_EINVAL, "import on a null plan");
  expect(dot_state_promote(nullptr, nullptr, nullptr, nullptr, nullptr) == DOT_EINVAL, "promote null plans");
  dot_batch* B = nullptr;
  expect(dot_batch_create(&a, 0, &B) == DOT_EINVAL, "empty batch");
  Data f;
  dot_problem pair[2] = {a, base_problem(f, 1, small, false)};
  expect(dot_batch_create(pair, 2, &B) == DOT_EINVAL && B == nullptr, "batch of different D");
  dot_ctx* C = nullptr;
  expect(dot_ctx_create(-1, 5, DOT_FP64, 1 << 20, 4, &C) == DOT_EINVAL, "context with D = 5");
}

int main() {
  check_invalid_problems();
  check_coarsening();
  check_footprint_and_null_handles();
  std::printf("%s (%d failures)\n", g_failures ? "FAILED" : "OK", g_failures);
  return g_failures ? 1 : 0;
}
