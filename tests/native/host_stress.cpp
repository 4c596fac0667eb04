// host_stress.cpp -- exercises the host side of libccm through its C ABI:
// planning of many shapes, plan reuse and replanning, invalid inputs, and
// the served form from several submitting threads with cancellation of
// queued and running jobs and destruction with work outstanding.  Meant to
// run against a build of the library whose host code is instrumented by
// AddressSanitizer or ThreadSanitizer (tests/native/build_sanitized.py); it
// checks statuses and finiteness, not values (the GPU tests check values).
//
// Exit status 0 when every call returned a status it may return.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "ccm.h"

namespace {

int g_fail = 0;
std::mutex g_mu;

void expect(bool ok, const char* what, int line) {
  if (!ok) {
    std::lock_guard<std::mutex> lk(g_mu);
    std::fprintf(stderr, "host_stress: FAILED %s (line %d)\n", what, line);
    ++g_fail;
  }
}
#define EXPECT(c) expect((c), #c, __LINE__)

// Input series: the two-species coupled logistic map.
void coupled(int64_t n, double x0, double y0, std::vector<double>& x, std::vector<double>& y) {
  x.resize(n);
  y.resize(n);
  double a = x0, b = y0;
  for (int64_t t = 0; t < n; ++t) {
    x[t] = a;
    y[t] = b;
    const double na = a * (3.8 - 3.8 * a - 0.02 * b);
    const double nb = b * (3.5 - 3.5 * b - 0.1 * a);
    a = na;
    b = nb;
  }
}

void plans(ccm_ctx* c) {
  std::vector<double> x, y;
  coupled(1500, 0.4, 0.2, x, y);
  for (int E = 1; E <= 10; E += 3)
    for (int tau = 1; tau <= 3; ++tau) {
      const int64_t L[] = {50, 200, 1400};
      const int r = 3;
      std::vector<double> a(3 * r), b(3 * r);
      int64_t le[3];
      for (int rep = 0; rep < 2; ++rep) {   // the second call reuses the plan
        EXPECT(ccm(c, x.data(), y.data(), 1500, E, tau, L, 3, r, 11, nullptr, a.data(),
                   b.data(), le) == CCM_OK);
        for (double v : a) EXPECT(std::isfinite(v));
      }
    }
  // a sweep and a causal matrix
  const int32_t Es[] = {2, 5}, Ts[] = {1, 2};
  const int64_t L[] = {100, 800};
  std::vector<double> rho(2 * 2 * 2 * 2 * 2);
  EXPECT(ccm_sweep(c, x.data(), y.data(), 1500, Es, 2, Ts, 2, L, 2, 2, 5, nullptr,
                   rho.data()) == CCM_OK);
  std::vector<double> S(3 * 1500);
  for (int m = 0; m < 3; ++m) {
    std::vector<double> u, v;
    coupled(1500, 0.3 + 0.1 * m, 0.2, u, v);
    for (int t = 0; t < 1500; ++t) S[m * 1500 + t] = u[t];
  }
  std::vector<double> rm(3 * 3 * 2 * 2);
  EXPECT(ccm_matrix(c, S.data(), 3, 1500, 3, 1, L, 2, 2, 7, nullptr, rm.data()) == CCM_OK);
  // invalid inputs
  double d[4];
  EXPECT(ccm(c, nullptr, y.data(), 1500, 2, 1, L, 2, 1, 1, nullptr, d, d, nullptr) ==
         CCM_E_INVAL);
  EXPECT(ccm(c, x.data(), y.data(), 1500, 11, 1, L, 2, 1, 1, nullptr, d, d, nullptr) ==
         CCM_E_INVAL);
  EXPECT(ccm(c, x.data(), y.data(), 1, 2, 1, L, 2, 1, 1, nullptr, d, d, nullptr) ==
         CCM_E_INVAL);
  std::vector<double> bad(x);
  bad[7] = NAN;
  EXPECT(ccm(c, bad.data(), y.data(), 1500, 2, 1, L, 2, 1, 1, nullptr, d, d, nullptr) ==
         CCM_E_INVAL);
}

struct Sub {
  uint64_t ticket;
  int nL, r;
  bool cancelled;
};

void serve(ccm_ctx* c, uint64_t budget, bool leave_outstanding) {
  ccm_server_cfg cfg{budget, 0, 0.0};
  ccm_server* s = nullptr;
  EXPECT(ccm_server_create(c, &cfg, &s) == CCM_OK);
  if (!s) return;
  std::vector<Sub> subs;
  std::mutex mu;
  auto submitter = [&](int id) {
    std::mt19937_64 rng(1000 + id);
    for (int k = 0; k < 12; ++k) {
      const int64_t n = 800 + (int64_t)(rng() % 6000);
      const int E = 1 + (int)(rng() % 10), tau = 1 + (int)(rng() % 4);
      std::vector<double> x, y;
      coupled(n, 0.2 + 0.6 * (rng() % 1000) / 1000.0, 0.3, x, y);
      const int64_t ne = n - (int64_t)(E - 1) * tau;
      const int64_t L[] = {E + 2 + 20, ne / 2, ne};
      ccm_job j{};
      j.X = x.data();
      j.Y = y.data();
      j.N = n;
      j.E = E;
      j.tau = tau;
      j.L = L;
      j.nL = 3;
      j.r = 4;
      j.seed = rng();
      if (k % 5 == 4) j.opts.flags = CCM_FLAG_TABLE;
      uint64_t t = 0;
      const ccm_status st = ccm_submit(s, &j, &t);
      EXPECT(st == CCM_OK);
      if (st != CCM_OK) continue;
      bool cancel = (k % 4 == 1);
      if (cancel) EXPECT(ccm_cancel(s, t) == CCM_OK);
      std::lock_guard<std::mutex> lk(mu);
      subs.push_back({t, 3, 4, cancel});
    }
  };
  std::vector<std::thread> th;
  for (int i = 0; i < 3; ++i) th.emplace_back(submitter, i);
  for (auto& t : th) t.join();
  if (leave_outstanding) {
    ccm_server_destroy(s);   // cancels and waits for everything
    return;
  }
  // one more cancel while jobs run, then collect everything
  if (!subs.empty()) {
    const ccm_status st = ccm_cancel(s, subs.back().ticket);
    EXPECT(st == CCM_OK || st == CCM_E_NOTFOUND);
    subs.back().cancelled = true;
  }
  for (const Sub& u : subs) {
    const ccm_status w = ccm_wait(s, u.ticket, -1);
    std::vector<double> a(u.nL * u.r), b(u.nL * u.r);
    ccm_job_stats stt{};
    if (u.cancelled) {
      EXPECT(w == CCM_OK || w == CCM_E_NOTFOUND);
      ccm_status rs = ccm_result(s, u.ticket, a.data(), b.data(), &stt);
      while (rs == CCM_E_BUSY) {
        std::this_thread::yield();
        rs = ccm_result(s, u.ticket, a.data(), b.data(), &stt);
      }
      EXPECT(rs == CCM_OK || rs == CCM_E_NOTFOUND);
    } else {
      EXPECT(w == CCM_OK);
      EXPECT(ccm_result(s, u.ticket, a.data(), b.data(), &stt) == CCM_OK);
      EXPECT(stt.t_done >= stt.t_admit && stt.t_admit >= stt.t_submit);
    }
  }
  EXPECT(ccm_wait(s, 123456789, 0) == CCM_E_NOTFOUND);
  ccm_server_destroy(s);
}

}  // namespace

int main() {
  ccm_ctx* c = nullptr;
  if (ccm_create(0, &c) != CCM_OK) {
    std::fprintf(stderr, "host_stress: no device\n");
    return 2;
  }
  std::printf("host_stress: plans\n");
  std::fflush(stdout);
  plans(c);
  std::printf("host_stress: served form, default budget\n");
  std::fflush(stdout);
  serve(c, 0, false);
  std::printf("host_stress: served form, small budget\n");
  std::fflush(stdout);
  serve(c, 64ull << 20, false);
  std::printf("host_stress: served form, destroyed with work outstanding\n");
  std::fflush(stdout);
  serve(c, 0, true);
  ccm_destroy(c);
  std::printf("host_stress: %s (%d failures)\n", g_fail ? "FAILED" : "ok", g_fail);
  return g_fail ? 1 : 0;
}
