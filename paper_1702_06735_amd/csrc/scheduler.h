// Fit scheduling of the fit server: the queue, admission, ticks and tickets.
//
// Host-only C++ (no HIP): the device work is a policy object, so the same
// scheduling code runs in the library and, with a stand-in evaluator, in
// host-only tests. Dev provides
//   void thread_init()      called first on the worker and each admission thread
//   bool reserve(Fit&)      set aside the fit's device memory (its footprint
//                           and its staging): false if it cannot (then the fit
//                           waits); called with the scheduler's lock held
//   int32_t admit(Fit&, int lane)
//                           build the fit's device state (MXA_OK or an error)
//                           in the reserved memory, without the lock, on
//                           admission thread `lane` (concurrently with the
//                           worker's tables() and evaluate() and with the
//                           other admission threads)
//   void drop_staging(Fit&) return the staging part after admission (lock held)
//   void release(Fit&)      free it all (also after a failed admit; idempotent;
//                           lock held)
//   int32_t tables(const std::vector<Fit*>& slots)
//                           the set of active fits changed (slot -> fit or
//                           NULL); called with no group in flight
//   int groups()            G: the slots form G groups (slot mod G), each
//                           evaluated by its own device call
//   int32_t launch(const std::vector<Fit*>& slots, int g)
//                           start the evaluation of group g's active fits at
//                           their fit->bfgs.point() (returns without waiting)
//   int32_t collect(const std::vector<Fit*>& slots, int g, std::vector<double>& nll,
//                   std::vector<const double*>& grad)
//                           wait for group g's evaluation: each of its fits'
//                           NLL and gradient (n_theta entries); +inf for a
//                           point outside the model's domain
//   const char* error()     message of the last failing call
//
// A worker thread runs ticks: it drops cancelled fits, takes queued ones in
// arrival order while a slot and the HBM budget allow (a fit holds its
// footprint while active and its staging during admission, both counted
// against the budget) and hands them to the admission threads, evaluates
// every admitted fit's next point, one device call per group of slots, feeds
// the results to each fit's minimiser and retires the fits that have
// finished, freeing their slot and budget at once. With two groups the calls
// alternate: one group's results are fed back while the device evaluates the
// other, so the host's share of a tick overlaps the device's; a change to the
// set of active fits first lets the group in flight finish. The admission threads take the reserved fits in
// arrival order and build their device states while the ticks of the others
// go on; a fit joins the ticks once it is built. A finished fit's record
// stays until its ticket is released.
//
// Teardown: shutdown() stops the worker, wakes every caller blocked in
// result() and waits until all callers inside a scheduler call have left
// before it frees the fits; no call may start once shutdown() has begun.
#pragma once

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/mixamp.h"
#include "bfgs.h"

namespace mxa {

inline int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Fit {
  uint64_t ticket = 0;
  int32_t status = MXA_FIT_QUEUED;
  int64_t n = 0;
  int64_t footprint = 0;          // device bytes while active
  int64_t staging = 0;            // device bytes during admission only
  std::vector<double> p4, t;      // host copy until admission
  const double* d_p4 = nullptr;   // or the caller's device copy, read in place
  const double* d_t = nullptr;
  std::vector<double> theta0;
  int64_t t_submit = 0, t_start = 0, t_done = 0;
  bool cancel = false;
  int slot = -1;                  // while it holds a slot
  int phase = 0;                  // QUEUED, RESERVED, ADMITTING, READY (Scheduler)
  bool staging_held = false;      // its staging is counted in the budget
  void* dev[3] = {nullptr, nullptr, nullptr};  // device state (the device layer's)
  int64_t ld = 0;
  Bfgs bfgs;
  mxa_fit_result result{};
};

class Scheduler {
 public:
  void init(int max_slots, int64_t budget, int n_theta) {
    max_slots_ = max_slots;
    budget_ = budget;
    n_theta_ = n_theta;
    slots_.assign(max_slots, nullptr);
  }

  int64_t budget() const { return budget_; }

  // Queue a fit (owned by the scheduler from here on).
  int32_t submit(Fit* f, uint64_t* ticket, char* msg, size_t nmsg) {
    f->t_submit = now_ns();
    {
      std::lock_guard<std::mutex> lk(mu_);
      Inside in(this);
      if (stop_) {
        snprintf(msg, nmsg, "server stopped: %s", worker_msg_);
        delete f;
        return MXA_EDEVICE;
      }
      f->ticket = next_ticket_++;
      fits_[f->ticket] = f;
      queue_.push_back(f);
      *ticket = f->ticket;
      ++events_;
    }
    cv_.notify_all();
    return MXA_OK;
  }

  // A finished fit's result: MXA_OK, MXA_EAGAIN while queued or running (or,
  // with wait, blocks until it has finished), MXA_ENOTFOUND, or the worker's
  // error if the server stopped.
  int32_t result(uint64_t ticket, mxa_fit_result* out, bool wait, char* msg, size_t nmsg) {
    std::unique_lock<std::mutex> lk(mu_);
    Inside in(this);
    auto it = fits_.find(ticket);
    if (it == fits_.end()) {
      snprintf(msg, nmsg, "unknown ticket %llu", (unsigned long long)ticket);
      return MXA_ENOTFOUND;
    }
    Fit* f = it->second;
    auto running = [&] { return f->status == MXA_FIT_QUEUED || f->status == MXA_FIT_RUNNING; };
    if (wait) done_cv_.wait(lk, [&] { return !running() || (stop_ && worker_error_) || closing_; });
    if (running()) {
      if (stop_ && (worker_error_ || closing_)) {
        snprintf(msg, nmsg, "server stopped: %s", worker_error_ ? worker_msg_ : "shut down");
        return worker_error_ ? worker_error_ : MXA_EDEVICE;
      }
      return MXA_EAGAIN;
    }
    *out = f->result;
    out->status = f->status;
    return MXA_OK;
  }

  int32_t cancel(uint64_t ticket, char* msg, size_t nmsg) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      Inside in(this);
      auto it = fits_.find(ticket);
      if (it == fits_.end()) {
        snprintf(msg, nmsg, "unknown ticket %llu", (unsigned long long)ticket);
        return MXA_ENOTFOUND;
      }
      it->second->cancel = true;
      ++events_;
    }
    cv_.notify_all();
    return MXA_OK;
  }

  // Forget a finished fit's record (MXA_EAGAIN while it is queued or running).
  int32_t release(uint64_t ticket, char* msg, size_t nmsg) {
    Fit* f = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu_);
      Inside in(this);
      auto it = fits_.find(ticket);
      if (it == fits_.end()) {
        snprintf(msg, nmsg, "unknown ticket %llu", (unsigned long long)ticket);
        return MXA_ENOTFOUND;
      }
      if (it->second->status == MXA_FIT_QUEUED || it->second->status == MXA_FIT_RUNNING) {
        snprintf(msg, nmsg, "fit %llu has not finished", (unsigned long long)ticket);
        return MXA_EAGAIN;
      }
      f = it->second;
      fits_.erase(it);
    }
    delete f;  // its device state went at finish()
    return MXA_OK;
  }

  // ticks, evaluations, active fits, queued fits, HBM bytes in use, the
  // largest HBM bytes in use and the most active fits since the start, fit
  // records held
  void stats(int64_t* out) {
    std::lock_guard<std::mutex> lk(mu_);
    Inside in(this);
    int active = 0;
    for (Fit* f : slots_) active += f != nullptr;
    out[0] = ticks_.load();
    out[1] = evals_.load();
    out[2] = active;
    out[3] = static_cast<int64_t>(queue_.size());
    out[4] = used_;
    out[5] = peak_used_;
    out[6] = peak_active_;
    out[7] = static_cast<int64_t>(fits_.size());
  }

  // the worker and n_admit admission threads
  template <class Dev> void start(Dev* dev, int n_admit = 1) {
    worker_ = std::thread([this, dev] { loop(*dev); });
    for (int k = 0; k < n_admit; ++k) admitters_.emplace_back([this, dev, k] { admit_loop(*dev, k); });
  }

  // Stop the worker (unfinished fits are cancelled), wait for the callers
  // inside a scheduler call to leave, then free every fit.
  template <class Dev> void shutdown(Dev& dev) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      for (Fit* f : queue_) f->cancel = true;
      for (Fit* f : slots_)
        if (f) f->cancel = true;
    }
    cv_.notify_all();
    admit_cv_.notify_all();
    if (worker_.joinable()) worker_.join();
    for (std::thread& a : admitters_)
      if (a.joinable()) a.join();
    std::unique_lock<std::mutex> lk(mu_);
    closing_ = true;
    done_cv_.notify_all();
    left_cv_.wait(lk, [&] { return inside_ == 0; });
    for (auto& kv : fits_) {
      dev.release(*kv.second);
      delete kv.second;
    }
    fits_.clear();
  }

 private:
  // Counts a caller inside a scheduler call (made and destroyed with the
  // lock held), so that shutdown() can wait for it to leave.
  struct Inside {
    Scheduler* s;
    explicit Inside(Scheduler* sc) : s(sc) { ++s->inside_; }
    ~Inside() {
      if (--s->inside_ == 0 && s->closing_) s->left_cv_.notify_all();
    }
  };

  // Retire a fit (lock held): its result, its slot and its budget.
  template <class Dev> void finish(Dev& dev, Fit* f, int32_t status) {
    f->t_done = now_ns();
    mxa_fit_result& r = f->result;
    memset(&r, 0, sizeof r);
    f->bfgs.best(r.theta);
    r.nll = f->bfgs.best_f();
    r.grad_norm = f->bfgs.grad_norm();
    r.n_evals = f->bfgs.evals();
    r.status = status;
    r.n = f->n;
    r.t_submit_ns = f->t_submit;
    r.t_start_ns = f->t_start;
    r.t_done_ns = f->t_done;
    if (f->bfgs.errors_ok()) {
      r.errors_ok = 1;
      for (int i = 0; i < f->bfgs.n_free(); ++i) r.err[f->bfgs.free_index(i)] = f->bfgs.errors()[i];
    }
    for (int i = 0; i < n_theta_ && i < MXA_MAX_THETA; ++i) r.grad[i] = f->bfgs.best_grad()[i];
    f->status = status;
    dev.release(*f);
    used_ -= f->footprint + (f->staging_held ? f->staging : 0);
    f->staging_held = false;
    if (f->slot >= 0) slots_[f->slot] = nullptr;
    f->slot = -1;
    f->phase = DONE;
  }

  template <class Dev> void fail_worker(Dev& dev) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      worker_error_ = MXA_EDEVICE;
      snprintf(worker_msg_, sizeof worker_msg_, "%s", dev.error());
      stop_ = true;
      done_cv_.notify_all();
    }
    admit_cv_.notify_all();
  }

  // An admission thread: builds the device state of the fits the worker
  // reserved, taking them in arrival order, while the ticks go on.
  template <class Dev> void admit_loop(Dev& dev, int lane) {
    dev.thread_init();
    while (true) {
      Fit* f = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        admit_cv_.wait(lk, [&] { return stop_ || !admitting_.empty(); });
        if (stop_) return;
        f = admitting_.front();
        admitting_.pop_front();
        f->phase = ADMITTING;
      }
      const int32_t rc = dev.admit(*f, lane);
      {
        std::lock_guard<std::mutex> lk(mu_);
        dev.drop_staging(*f);
        used_ -= f->staging;
        f->staging_held = false;
        if (rc != MXA_OK) {
          finish(dev, f, MXA_FIT_FAILED);
        } else {
          f->phase = READY;
        }
        admitted_ = true;
        ++events_;
        done_cv_.notify_all();
      }
      cv_.notify_all();
    }
  }

  template <class Dev> void loop(Dev& dev) {
    dev.thread_init();
    const int G = dev.groups();
    bool dirty = true;
    std::vector<double> nll(max_slots_);
    std::vector<const double*> grad(max_slots_);
    std::vector<Fit*> ready(max_slots_, nullptr);
    int inflight = -1;  // the group launched and not yet collected
    auto has_fits = [&](int g) {
      for (int sl = g; sl < max_slots_; sl += G)
        if (ready[sl]) return true;
      return false;
    };
    // wait for group g, feed its fits' minimisers, retire the finished ones
    auto collect = [&](int g) {
      if (dev.collect(ready, g, nll, grad) != MXA_OK) return false;
      int n_active = 0;
      for (int sl = g; sl < max_slots_; sl += G) n_active += ready[sl] != nullptr;
      ticks_++;
      evals_ += n_active;
      std::lock_guard<std::mutex> lk(mu_);
      for (int sl = g; sl < max_slots_; sl += G) {
        Fit* f = ready[sl];
        if (!f) continue;
        f->bfgs.tell(nll[sl], grad[sl]);
        if (f->bfgs.status() != Bfgs::RUNNING) {
          const int32_t st = f->bfgs.status() == Bfgs::CONVERGED   ? MXA_FIT_CONVERGED
                             : f->bfgs.status() == Bfgs::MAX_EVALS ? MXA_FIT_MAX_EVALS
                                                                   : MXA_FIT_FAILED;
          finish(dev, f, st);
          ready[sl] = nullptr;
          dirty = true;
        }
      }
      done_cv_.notify_all();
      return true;
    };
    while (true) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        // cancelled fits leave at once, except one being admitted, which
        // leaves when its admission has finished, and one whose group is in
        // flight, which leaves once its group has been collected
        for (int sl = 0; sl < max_slots_; ++sl) {
          Fit* f = slots_[sl];
          if (!f || !f->cancel || f->phase == ADMITTING) continue;
          if (inflight >= 0 && f->phase == READY && sl % G == inflight) continue;
          if (f->phase == RESERVED) admitting_.erase(std::find(admitting_.begin(), admitting_.end(), f));
          if (f->phase == READY) {
            dirty = true;
            ready[sl] = nullptr;
          }
          finish(dev, f, MXA_FIT_CANCELLED);
        }
        for (auto it = queue_.begin(); it != queue_.end();) {
          if ((*it)->cancel) {
            (*it)->status = MXA_FIT_CANCELLED;
            (*it)->result.status = MXA_FIT_CANCELLED;
            (*it)->t_done = now_ns();
            (*it)->phase = DONE;
            std::vector<double>().swap((*it)->p4);
            std::vector<double>().swap((*it)->t);
            it = queue_.erase(it);
          } else {
            ++it;
          }
        }
        done_cv_.notify_all();
        // admission: a free slot and room in the budget, in arrival order;
        // the admission threads build the device states
        bool handed = false;
        while (!queue_.empty() && !stop_) {
          Fit* f = queue_.front();
          int free_slot = -1;
          for (int sl = 0; sl < max_slots_; ++sl)
            if (!slots_[sl]) {
              free_slot = sl;
              break;
            }
          if (free_slot < 0 || used_ + f->footprint + f->staging > budget_) break;
          if (!dev.reserve(*f)) break;
          queue_.pop_front();
          f->slot = free_slot;
          slots_[free_slot] = f;
          used_ += f->footprint + f->staging;
          f->staging_held = true;
          peak_used_ = std::max(peak_used_, used_);
          int act = 0;
          for (Fit* a : slots_) act += a != nullptr;
          peak_active_ = std::max<int64_t>(peak_active_, act);
          f->status = MXA_FIT_RUNNING;
          f->t_start = now_ns();
          f->phase = RESERVED;
          admitting_.push_back(f);
          handed = true;
        }
        if (handed) admit_cv_.notify_all();
        if (admitted_) {
          admitted_ = false;
          dirty = true;
        }
        int n_ready = 0, n_held = 0;
        for (Fit* f : slots_) {
          n_held += f != nullptr;
          n_ready += f && f->phase == READY;
        }
        if (n_ready == 0 && inflight < 0) {
          if (stop_ && n_held == 0) return;
          // nothing to evaluate: wait for a submission, a cancellation, an
          // admission or the stop
          const uint64_t seen = events_;
          cv_.wait(lk, [&] { return stop_ || events_ != seen; });
          continue;
        }
        if (dirty && inflight < 0)
          for (int sl = 0; sl < max_slots_; ++sl)
            ready[sl] = slots_[sl] && slots_[sl]->phase == READY ? slots_[sl] : nullptr;
      }
      if (dirty) {
        // the set of active fits changed: the group in flight finishes first
        if (inflight >= 0) {
          const int g = inflight;
          inflight = -1;
          if (!collect(g)) return fail_worker(dev);
          continue;
        }
        if (dev.tables(ready) != MXA_OK) return fail_worker(dev);
        dirty = false;
      }
      // the next group with active fits after the one in flight
      int next = -1;
      for (int k = 1; k <= G; ++k) {
        const int c = ((inflight < 0 ? G - 1 : inflight) + k) % G;
        if (c != inflight && has_fits(c)) {
          next = c;
          break;
        }
      }
      if (next < 0) {
        // nothing else to launch: let the group in flight finish
        if (inflight >= 0) {
          const int g = inflight;
          inflight = -1;
          if (!collect(g)) return fail_worker(dev);
        }
        continue;
      }
      if (dev.launch(ready, next) != MXA_OK) return fail_worker(dev);
      // the previous group's results are fed back while the device runs this one
      if (inflight >= 0 && !collect(inflight)) return fail_worker(dev);
      inflight = next;
    }
  }

  enum Phase { QUEUED = 0, RESERVED, ADMITTING, READY, DONE };

  int max_slots_ = 0, n_theta_ = 0;
  int64_t budget_ = 0, used_ = 0, peak_used_ = 0, peak_active_ = 0;
  int inside_ = 0;        // callers inside a scheduler call
  bool closing_ = false;  // shutdown() is waiting for them
  std::mutex mu_;
  std::condition_variable cv_, done_cv_, left_cv_, admit_cv_;
  std::deque<Fit*> queue_;
  std::deque<Fit*> admitting_;  // reserved, waiting for an admission thread
  bool admitted_ = false;       // an admission finished since the last tick
  uint64_t events_ = 0;         // submissions, cancellations, admissions
  std::vector<Fit*> slots_;
  std::map<uint64_t, Fit*> fits_;
  uint64_t next_ticket_ = 1;
  bool stop_ = false;
  std::thread worker_;
  std::vector<std::thread> admitters_;
  std::atomic<int64_t> ticks_{0}, evals_{0};
  int32_t worker_error_ = MXA_OK;
  char worker_msg_[256] = "";
};

}  // namespace mxa
