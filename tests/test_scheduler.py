"""The fit server's scheduler (csrc/scheduler.h) on the host, with a stand-in
device: queueing, admission by free slot and HBM budget in arrival order
(staging counted while a fit is admitted, reservations that can fail),
continuous batching (one group of slots, or two evaluated alternately with
no fit released while its group is in flight), parallel admission threads, cancellation of queued
and running fits, failed admissions (on the admission thread, concurrent with the ticks), a device
failure, the ticket lifecycle with release, teardown while callers are
blocked in result(), and a fit's result being the same alone and in a mix. Built with g++ twice: with AddressSanitizer and
UndefinedBehaviorSanitizer, and with ThreadSanitizer (races between the
caller threads and the worker)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SRC = r'''
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>
#include "scheduler.h"
using namespace mxa;

static int failures = 0;
#define CHECK(c) do { if (!(c)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++failures; } } while (0)

constexpr int NT = 6;  // parameters per fit

// Stand-in device: fit k minimises sum_i w_i (theta_i - c_i)^2 with the
// centre c taken from its own "events"; kind 1 is a linear function that
// never converges (for cancellation).
struct StubDev {
  std::mutex mu;
  int max_active = 0, max_total = 0;
  int64_t fail_admit_n = -1;
  int fail_after = -1, n_eval = 0;
  int slow_us = 0;
  int64_t held = 0, peak_held = 0;  // bytes reserved (footprint + staging while admitted)
  int64_t capacity = int64_t(1) << 62;  // reservations beyond this fail
  std::vector<uint64_t> admitted;
  std::vector<std::vector<double>> g;
  void thread_init() {}
  bool reserve(Fit& f) {
    if (held + f.footprint + f.staging > capacity) return false;
    f.dev[0] = new char[16];
    f.dev[1] = new char[8];  // the staging
    held += f.footprint + f.staging;
    peak_held = std::max(peak_held, held);
    return true;
  }
  std::atomic<int> in_admit{0}, max_in_admit{0};
  int admit_us = 0;  // time one admission takes
  int32_t admit(Fit& f, int lane) {
    CHECK(f.dev[0] != nullptr && f.dev[1] != nullptr);
    CHECK(lane >= 0 && lane < 8);
    const int now = ++in_admit;
    int seen = max_in_admit.load();
    while (now > seen && !max_in_admit.compare_exchange_weak(seen, now)) {}
    if (admit_us) std::this_thread::sleep_for(std::chrono::microseconds(admit_us));
    --in_admit;
    if (f.n == fail_admit_n) return MXA_EDEVICE;
    std::lock_guard<std::mutex> lk(mu);
    admitted.push_back(f.ticket);
    return MXA_OK;
  }
  void drop_staging(Fit& f) {
    if (f.dev[1]) { delete[] static_cast<char*>(f.dev[1]); f.dev[1] = nullptr; held -= f.staging; }
  }
  void release(Fit& f) {
    {
      // never a fit whose group is in flight
      std::lock_guard<std::mutex> lk(mu);
      for (auto& fl : flight)
        for (Fit* x : fl) CHECK(x != &f);
    }
    drop_staging(f);
    if (f.dev[0]) { delete[] static_cast<char*>(f.dev[0]); f.dev[0] = nullptr; held -= f.footprint; }
  }
  int32_t tables(const std::vector<Fit*>& slots) {
    int a = 0;
    for (Fit* f : slots) a += f != nullptr;
    std::lock_guard<std::mutex> lk(mu);
    CHECK(flight[0].empty() && flight[1].empty());  // no group in flight
    if (a > max_active) max_active = a;
    return MXA_OK;
  }
  int n_groups = 2;
  std::vector<Fit*> flight[2];  // the fits of each group in flight
  int launches = 0, overlapped = 0;
  int groups() const { return n_groups; }
  int32_t launch(const std::vector<Fit*>& slots, int grp) {
    std::lock_guard<std::mutex> lk(mu);
    CHECK(grp >= 0 && grp < n_groups && flight[grp].empty());
    ++launches;
    if (!flight[1 - grp].empty()) ++overlapped;
    for (size_t sl = grp; sl < slots.size(); sl += n_groups)
      if (slots[sl]) flight[grp].push_back(slots[sl]);
    CHECK(!flight[grp].empty());
    return MXA_OK;
  }
  int32_t collect(const std::vector<Fit*>& slots, int grp, std::vector<double>& nll,
                  std::vector<const double*>& grad) {
    {
      std::lock_guard<std::mutex> lk(mu);
      CHECK(!flight[grp].empty());
      size_t k = 0;
      for (size_t sl = grp; sl < slots.size(); sl += n_groups)
        if (slots[sl]) CHECK(k < flight[grp].size() && flight[grp][k++] == slots[sl]);
      flight[grp].clear();
    }
    if (fail_after >= 0 && ++n_eval > fail_after) return MXA_EDEVICE;
    if (slow_us) std::this_thread::sleep_for(std::chrono::microseconds(slow_us));
    g.resize(slots.size(), std::vector<double>(NT));
    for (size_t sl = grp; sl < slots.size(); sl += n_groups) {
      Fit* f = slots[sl];
      if (!f) continue;
      const double* x = f->bfgs.point();
      double v = 0.0;
      for (int i = 0; i < NT; ++i) {
        if (f->t[0] > 0.5) {  // kind 1
          v += x[i];
          g[sl][i] = 1.0;
        } else {
          const double c = f->p4[i % f->p4.size()], w = 1.0 + i % 3;
          v += w * (x[i] - c) * (x[i] - c);
          g[sl][i] = 2.0 * w * (x[i] - c);
        }
      }
      nll[sl] = v;
      grad[sl] = g[sl].data();
    }
    return MXA_OK;
  }
  const char* error() { return "stand-in device failure"; }
};

static Fit* make_fit(int64_t n, double centre, int kind = 0, int max_evals = 200) {
  Fit* f = new Fit();
  f->n = n;
  f->footprint = n * 100;
  f->staging = n * 36;
  for (int i = 0; i < 4; ++i) f->p4.push_back(centre + i);
  f->t.assign(1, kind ? 1.0 : 0.0);
  f->theta0.assign(NT, 0.0);
  std::vector<int> idx;
  std::vector<double> sc;
  for (int i = 0; i < NT; ++i) { idx.push_back(i); sc.push_back(1.0); }
  f->bfgs.init(f->theta0.data(), NT, idx.data(), sc.data(), NT, max_evals, 1e-10, 0.0);
  return f;
}

static std::vector<mxa_fit_result> run_all(StubDev& dev, int max_slots, int64_t budget,
                                           const std::vector<Fit*>& fits, int n_admit = 1) {
  Scheduler s;
  s.init(max_slots, budget, NT);
  char msg[256];
  std::vector<uint64_t> t(fits.size());
  // all queued before the worker starts, so admission sees the whole queue
  for (size_t i = 0; i < fits.size(); ++i) CHECK(s.submit(fits[i], &t[i], msg, sizeof msg) == MXA_OK);
  s.start(&dev, n_admit);
  std::vector<mxa_fit_result> out(fits.size());
  for (size_t i = 0; i < fits.size(); ++i) CHECK(s.result(t[i], &out[i], true, msg, sizeof msg) == MXA_OK);
  int64_t st[8];
  s.stats(st);
  CHECK(st[2] == 0 && st[3] == 0 && st[4] == 0);  // nothing active, queued or held
  CHECK(st[5] <= budget && st[5] == dev.peak_held);
  CHECK(st[7] == static_cast<int64_t>(fits.size()));
  CHECK(dev.held == 0);
  // records go when their tickets are released
  for (size_t i = 0; i < fits.size(); ++i) CHECK(s.release(t[i], msg, sizeof msg) == MXA_OK);
  CHECK(s.release(t[0], msg, sizeof msg) == MXA_ENOTFOUND);
  s.stats(st);
  CHECK(st[7] == 0);
  s.shutdown(dev);
  return out;
}

static void batch(int n_groups = 2) {
  // 12 fits; the budget holds two of them while admitted (cache and staging)
  // and three once admitted; the slots four
  StubDev dev;
  dev.n_groups = n_groups;
  std::vector<Fit*> fits;
  for (int k = 0; k < 12; ++k) fits.push_back(make_fit(1000, 0.5 * k));
  auto out = run_all(dev, 4, 3 * 1000 * 100, fits);
  CHECK(dev.max_active <= 3 && dev.max_active >= 2);
  CHECK(dev.peak_held <= 3 * 1000 * 100);
  for (size_t i = 1; i < dev.admitted.size(); ++i) CHECK(dev.admitted[i] > dev.admitted[i - 1]);
  CHECK(dev.admitted.size() == 12);
  // with two groups, launches overlapped the other group's evaluation
  CHECK(n_groups == 1 ? dev.overlapped == 0 : dev.overlapped > 0);
  for (int k = 0; k < 12; ++k) {
    CHECK(out[k].status == MXA_FIT_CONVERGED);
    for (int i = 0; i < NT; ++i) CHECK(std::fabs(out[k].theta[i] - (0.5 * k + i % 4)) < 1e-6);
    CHECK(out[k].nll < 1e-10);
    CHECK(out[k].t_start_ns >= out[k].t_submit_ns && out[k].t_done_ns >= out[k].t_start_ns);
  }
}

static void alone_vs_mix() {
  StubDev d1, d2;
  auto a = run_all(d1, 8, int64_t(1) << 40, {make_fit(500, 1.25)});
  std::vector<Fit*> mix;
  for (int k = 0; k < 6; ++k) mix.push_back(make_fit(500 + k, k == 3 ? 1.25 : 0.3 * k));
  auto b = run_all(d2, 3, int64_t(1) << 40, mix);
  CHECK(std::memcmp(a[0].theta, b[3].theta, sizeof a[0].theta) == 0);
  CHECK(a[0].nll == b[3].nll && a[0].n_evals == b[3].n_evals);
  CHECK(std::memcmp(a[0].grad, b[3].grad, sizeof a[0].grad) == 0);
}

static void cancel_and_tickets() {
  StubDev dev;
  dev.slow_us = 200;
  Scheduler s;
  s.init(2, int64_t(1) << 40, NT);
  s.start(&dev);
  char msg[256];
  uint64_t t[5];
  for (int k = 0; k < 5; ++k) CHECK(s.submit(make_fit(100, 0.0, 1, 1 << 30), &t[k], msg, sizeof msg) == MXA_OK);
  mxa_fit_result r;
  CHECK(s.result(12345, &r, false, msg, sizeof msg) == MXA_ENOTFOUND);
  CHECK(std::strstr(msg, "unknown ticket") != nullptr);
  CHECK(s.cancel(999, msg, sizeof msg) == MXA_ENOTFOUND);
  // wait (up to 10 s, the host may be loaded) until two fits run (both
  // admitted: their staging returned) and a tick is done
  int64_t st[8];
  for (int w = 0; w < 10000; ++w) {
    s.stats(st);
    if (st[2] == 2 && st[0] > 0 && st[4] == 2 * 100 * 100) break;
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  CHECK(s.result(t[0], &r, false, msg, sizeof msg) == MXA_EAGAIN);  // running
  CHECK(s.result(t[4], &r, false, msg, sizeof msg) == MXA_EAGAIN);  // queued
  CHECK(st[2] == 2 && st[3] == 3 && st[4] == 2 * 100 * 100 && st[0] > 0 && st[6] == 2);
  for (int k : {4, 0, 3, 1, 2}) CHECK(s.cancel(t[k], msg, sizeof msg) == MXA_OK);
  for (int k = 0; k < 5; ++k) {
    CHECK(s.result(t[k], &r, true, msg, sizeof msg) == MXA_OK);
    CHECK(r.status == MXA_FIT_CANCELLED);
  }
  s.stats(st);
  CHECK(st[2] == 0 && st[3] == 0 && st[4] == 0);
  s.shutdown(dev);
}

static void parallel_admission() {
  // three admission threads: admissions overlap (at most three at once), every
  // fit is admitted once and converges, and a fit's result is the one it has
  // with a single admission thread
  StubDev d1, d3;
  d1.admit_us = d3.admit_us = 2000;
  std::vector<Fit*> a, b;
  for (int k = 0; k < 10; ++k) {
    a.push_back(make_fit(1000 + k, 0.5 * k));
    b.push_back(make_fit(1000 + k, 0.5 * k));
  }
  auto o1 = run_all(d1, 6, int64_t(1) << 40, a, 1);
  auto o3 = run_all(d3, 6, int64_t(1) << 40, b, 3);
  CHECK(d1.max_in_admit.load() == 1);
  CHECK(d3.max_in_admit.load() >= 2 && d3.max_in_admit.load() <= 3);
  CHECK(d3.admitted.size() == 10);
  for (int k = 0; k < 10; ++k) {
    CHECK(o3[k].status == MXA_FIT_CONVERGED);
    CHECK(std::memcmp(o1[k].theta, o3[k].theta, sizeof o1[k].theta) == 0 && o1[k].nll == o3[k].nll);
  }
}

static void reservation_can_fail() {
  // the device holds less than the budget says (a fragmented arena): fits
  // wait for room instead of failing, and all finish
  StubDev dev;
  dev.capacity = 2 * 1000 * 136;
  std::vector<Fit*> fits;
  for (int k = 0; k < 6; ++k) fits.push_back(make_fit(1000, 0.25 * k));
  auto out = run_all(dev, 4, int64_t(1) << 40, fits);
  for (int k = 0; k < 6; ++k) CHECK(out[k].status == MXA_FIT_CONVERGED);
  CHECK(dev.max_active <= 2);
}

static void release_rules() {
  StubDev dev;
  dev.slow_us = 100;
  Scheduler s;
  s.init(1, int64_t(1) << 40, NT);
  s.start(&dev);
  char msg[256];
  uint64_t a, b;
  CHECK(s.submit(make_fit(100, 0.0, 1, 1 << 30), &a, msg, sizeof msg) == MXA_OK);
  CHECK(s.submit(make_fit(100, 0.0, 1, 1 << 30), &b, msg, sizeof msg) == MXA_OK);
  CHECK(s.release(a, msg, sizeof msg) == MXA_EAGAIN);  // running or queued
  CHECK(s.release(b, msg, sizeof msg) == MXA_EAGAIN);
  CHECK(s.cancel(b, msg, sizeof msg) == MXA_OK);
  CHECK(s.cancel(a, msg, sizeof msg) == MXA_OK);
  mxa_fit_result r;
  CHECK(s.result(a, &r, true, msg, sizeof msg) == MXA_OK && r.status == MXA_FIT_CANCELLED);
  CHECK(s.result(b, &r, true, msg, sizeof msg) == MXA_OK && r.status == MXA_FIT_CANCELLED);
  CHECK(s.release(a, msg, sizeof msg) == MXA_OK);
  CHECK(s.release(b, msg, sizeof msg) == MXA_OK);
  CHECK(s.result(a, &r, false, msg, sizeof msg) == MXA_ENOTFOUND);
  s.shutdown(dev);
}

static void shutdown_with_waiters() {
  // callers blocked in result() while the server is torn down: they return
  // (cancelled results) and shutdown() frees the fits only after they left
  StubDev dev;
  dev.slow_us = 100;
  Scheduler* s = new Scheduler();
  s->init(2, int64_t(1) << 40, NT);
  s->start(&dev);
  char msg[256];
  std::vector<uint64_t> t(4);
  for (int k = 0; k < 4; ++k) CHECK(s->submit(make_fit(100, 0.0, 1, 1 << 30), &t[k], msg, sizeof msg) == MXA_OK);
  std::vector<int> rc(4, 123), st(4, -1);
  std::vector<std::thread> th;
  std::atomic<int> started{0};
  for (int k = 0; k < 4; ++k)
    th.emplace_back([&, k] {
      char m[256];
      mxa_fit_result r;
      started++;
      rc[k] = s->result(t[k], &r, true, m, sizeof m);
      if (rc[k] == MXA_OK) st[k] = r.status;
    });
  // every caller is inside result() (blocked) before the teardown begins
  while (started.load() < 4) std::this_thread::yield();
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  s->shutdown(dev);
  delete s;
  for (auto& x : th) x.join();
  for (int k = 0; k < 4; ++k) CHECK((rc[k] == MXA_OK && st[k] == MXA_FIT_CANCELLED) || rc[k] == MXA_EDEVICE);
}

static void failed_admission() {
  StubDev dev;
  dev.fail_admit_n = 777;
  std::vector<Fit*> fits = {make_fit(100, 0.1), make_fit(777, 0.2), make_fit(100, 0.3)};
  auto out = run_all(dev, 1, int64_t(1) << 40, fits);
  CHECK(out[0].status == MXA_FIT_CONVERGED && out[2].status == MXA_FIT_CONVERGED);
  CHECK(out[1].status == MXA_FIT_FAILED && out[1].n_evals == 0);
}

static void device_failure() {
  StubDev dev;
  dev.fail_after = 3;
  Scheduler s;
  s.init(2, int64_t(1) << 40, NT);
  s.start(&dev);
  char msg[256];
  uint64_t t;
  CHECK(s.submit(make_fit(100, 0.0, 1, 1 << 30), &t, msg, sizeof msg) == MXA_OK);
  mxa_fit_result r;
  CHECK(s.result(t, &r, true, msg, sizeof msg) == MXA_EDEVICE);
  CHECK(std::strstr(msg, "stand-in device failure") != nullptr);
  Fit* late = make_fit(100, 0.0);
  CHECK(s.submit(late, &t, msg, sizeof msg) == MXA_EDEVICE);  // the server has stopped
  s.shutdown(dev);
}

static void shutdown_with_work() {
  StubDev dev;
  dev.slow_us = 100;
  Scheduler s;
  s.init(2, int64_t(1) << 40, NT);
  s.start(&dev);
  char msg[256];
  uint64_t t;
  for (int k = 0; k < 6; ++k) CHECK(s.submit(make_fit(100, 0.0, 1, 1 << 30), &t, msg, sizeof msg) == MXA_OK);
  std::this_thread::sleep_for(std::chrono::milliseconds(5));
  s.shutdown(dev);  // must return: running fits are cancelled, queued ones dropped
}

static void concurrent_submitters() {
  StubDev dev;
  Scheduler s;
  s.init(3, int64_t(1) << 40, NT);
  s.start(&dev);
  std::vector<std::thread> th;
  std::vector<int> ok(4, 0);
  for (int c = 0; c < 4; ++c)
    th.emplace_back([&, c] {
      char msg[256];
      for (int k = 0; k < 5; ++k) {
        uint64_t t;
        if (s.submit(make_fit(100 + c, 0.1 * k + c), &t, msg, sizeof msg) != MXA_OK) continue;
        mxa_fit_result r;
        if (s.result(t, &r, true, msg, sizeof msg) == MXA_OK && r.status == MXA_FIT_CONVERGED) ++ok[c];
      }
    });
  for (auto& x : th) x.join();
  for (int c = 0; c < 4; ++c) CHECK(ok[c] == 5);
  s.shutdown(dev);
}

int main(int argc, char** argv) {
  const std::string w = argc > 1 ? argv[1] : "all";
  if (w == "all" || w == "batch") batch();
  if (w == "all" || w == "batch1") batch(1);
  if (w == "all" || w == "mix") alone_vs_mix();
  if (w == "all" || w == "cancel") cancel_and_tickets();
  if (w == "all" || w == "admit") failed_admission();
  if (w == "all" || w == "device") device_failure();
  if (w == "all" || w == "shutdown") shutdown_with_work();
  if (w == "all" || w == "threads") concurrent_submitters();
  if (w == "all" || w == "reserve") reservation_can_fail();
  if (w == "all" || w == "release") release_rules();
  if (w == "all" || w == "waiters") shutdown_with_waiters();
  if (w == "all" || w == "padmit") parallel_admission();
  printf("%s\n", failures ? "FAILED" : "ok");
  return failures ? 1 : 0;
}
'''

FLAVOURS = {
    "asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "tsan": ["-fsanitize=thread"],
}
SCENARIOS = ["batch", "batch1", "mix", "cancel", "admit", "device", "shutdown", "threads", "reserve",
             "release", "waiters", "padmit"]


@pytest.fixture(scope="module", params=sorted(FLAVOURS))
def prog(request, tmp_path_factory):
    d = tmp_path_factory.mktemp("sched")
    (d / "t.cpp").write_text(SRC)
    exe = d / f"t_{request.param}"
    r = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-pthread", *FLAVOURS[request.param],
                        "-I", os.path.join(ROOT, "paper_1702_06735_amd", "csrc"), "-o", str(exe),
                        str(d / "t.cpp")], capture_output=True, text=True)
    if r.returncode != 0 and "san" in r.stderr.lower() and "cannot find" in r.stderr.lower():
        pytest.skip("no sanitizer runtime")
    assert r.returncode == 0, r.stderr[-3000:]
    return str(exe)


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scheduler(prog, scenario):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([prog, scenario], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-4000:])
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
