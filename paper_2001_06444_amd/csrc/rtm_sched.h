// rtm_sched.h -- job bookkeeping of the serving engine (host code, no HIP).
//
// The migrations of the Monte Carlo loop over velocity samples arrive as
// jobs; the engine admits a queued job as soon as its working set fits the
// arena, and keeps every admitted job advancing in the shared launches
// (continuous batching).  This class holds the part of that which needs no
// GPU: the queue, the admission order, the job state machine and its
// timestamps, and the per-realization counts of jobs in flight.
//
//   submit ─> QUEUED ─(admission pass)─> RUNNING ─(finish)─> DONE | FAILED
//               │  └─(build failed, not for lack of memory)─> FAILED
//               └─(cancel)─> CANCELLED       (only while QUEUED)
//
// Admission is first come, first served with bounded bypass: a pass walks
// the queue oldest first; the first job that does not fit blocks the pass
// unless it has been passed over fewer than max_bypass times, in which case
// younger jobs may try, up to the next one that does not fit.  A candidate
// refused because the running set is full (the engine keeps the levels of
// its running jobs within the memory-side cache) ends the pass, with no
// bypass counted: jobs then start strictly in order.  A job larger
// than the whole capacity is refused at submit; a queue whose head cannot fit
// while nothing runs (and nothing is about to be freed) fails its head with
// out-of-memory rather than wait forever (fail_head).
//
// The class is not thread-safe: the runtime holds its context mutex around
// every call, and may build a candidate's working set between
// next_candidate() and admit_result() without the mutex (the candidate is
// then ADMITTING: not cancellable, still counted as queued and in flight).
// Plain C++ (no HIP): tests/host/sched_test.cpp drives it with a mock clock
// and the arena allocator under ASan/UBSan and TSan.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <utility>
#include <iterator>
#include <map>
#include <set>
#include <unordered_map>

namespace rtm {

// Job states (the C ABI's RTM_JOB_* values) and one internal state.
enum : int { kJobQueued = 0, kJobRunning = 1, kJobDone = 2, kJobFailed = 3, kJobCancelled = 4, kJobAdmitting = 5 };
// Result codes (the C ABI's RTM_OK / RTM_E_* values).
enum : int { kSchedOk = 0, kSchedInval = -1, kSchedNomem = -3, kSchedAgain = -4, kSchedNotFound = -5,
             kSchedCancelled = -8 };

struct SchedEntry {
  uint64_t ticket = 0;
  int key = 0;       // realization: jobs of one key count toward in_flight(key)
  size_t bytes = 0;  // working-set size (submit refuses more than the capacity)
  int state = kJobQueued;
  int status = kSchedOk;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int bypassed = 0;  // passes in which this job did not fit and younger jobs went ahead
};

// State of one admission pass over the queue.
struct AdmitPass {
  uint64_t last = 0;     // the last ticket handed out in this pass
  bool blocked = false;  // a job of this pass did not fit
  bool stopped = false;  // no further candidates in this pass
};

class JobBook {
 public:
  using Clock = std::function<double()>;

  JobBook(Clock clock, size_t capacity, int queue_cap = 1 << 16, int max_bypass = 8)
      : clock_(std::move(clock)), capacity_(capacity), queue_cap_(queue_cap), max_bypass_(max_bypass) {}

  // Queues a job.  kSchedNomem if bytes exceed the capacity (it could never
  // run), kSchedAgain if the queue is full.
  int submit(int key, size_t bytes, uint64_t* ticket) {
    if (bytes > capacity_) return kSchedNomem;
    if ((int)queue_.size() >= queue_cap_) return kSchedAgain;
    SchedEntry e;
    e.ticket = next_++;
    e.key = key;
    e.bytes = bytes;
    e.t_submit = clock_();
    queue_.insert(e.ticket);
    ++in_flight_[key];
    ++submitted_;
    *ticket = e.ticket;
    jobs_.emplace(e.ticket, e);
    return kSchedOk;
  }

  // Cancels a queued job.  kSchedInval once it is being admitted or later.
  int cancel(uint64_t ticket) {
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return kSchedNotFound;
    SchedEntry& e = it->second;
    if (e.state != kJobQueued) return kSchedInval;
    queue_.erase(ticket);
    e.state = kJobCancelled;
    e.status = kSchedCancelled;
    e.t_done = clock_();
    drop_in_flight(e.key);
    ++cancelled_;
    return kSchedOk;
  }

  // The next job to try in this pass (0: none), marked ADMITTING.
  uint64_t next_candidate(AdmitPass& p) {
    if (p.stopped) return 0;
    for (auto it = queue_.upper_bound(p.last); it != queue_.end(); ++it) {
      SchedEntry& e = jobs_.at(*it);
      if (e.state != kJobQueued) continue;
      e.state = kJobAdmitting;
      p.last = e.ticket;
      return e.ticket;
    }
    p.stopped = true;
    return 0;
  }

  // Outcome of trying a candidate: kSchedOk (admitted: RUNNING), kSchedNomem
  // (does not fit now: QUEUED again), kSchedAgain (the running set is full:
  // QUEUED again and the pass ends) or another code (the job fails).
  void admit_result(AdmitPass& p, uint64_t ticket, int rc) {
    SchedEntry& e = jobs_.at(ticket);
    if (rc == kSchedOk) {
      e.state = kJobRunning;
      e.t_admit = clock_();
      queue_.erase(ticket);
      ++running_;
    } else if (rc == kSchedAgain) {
      e.state = kJobQueued;
      p.stopped = true;
    } else if (rc == kSchedNomem) {
      e.state = kJobQueued;
      if (p.blocked || ++e.bypassed > max_bypass_) p.stopped = true;  // keep the blocked job from starving
      else p.blocked = true;
    } else {
      queue_.erase(ticket);
      e.state = kJobFailed;
      e.status = rc;
      e.t_done = clock_();
      drop_in_flight(e.key);
      ++failed_;
    }
  }

  // A running job finished: DONE (status kSchedOk) or FAILED.
  void finish(uint64_t ticket, int status) {
    SchedEntry& e = jobs_.at(ticket);
    if (e.state != kJobRunning) return;
    e.state = status == kSchedOk ? kJobDone : kJobFailed;
    e.status = status;
    e.t_done = clock_();
    --running_;
    drop_in_flight(e.key);
    if (status == kSchedOk) ++done_;
    else ++failed_;
  }

  // Nothing runs and nothing is being freed, yet the queue head does not
  // fit: fail it with `status` (out of memory).  Returns its ticket or 0.
  uint64_t fail_head(int status) {
    for (uint64_t t : queue_) {
      SchedEntry& e = jobs_.at(t);
      if (e.state != kJobQueued) continue;
      queue_.erase(t);
      e.state = kJobFailed;
      e.status = status;
      e.t_done = clock_();
      drop_in_flight(e.key);
      ++failed_;
      return t;
    }
    return 0;
  }

  // Shutdown: running jobs end CANCELLED.
  void cancel_running(uint64_t ticket) {
    SchedEntry& e = jobs_.at(ticket);
    if (e.state != kJobRunning) return;
    e.state = kJobCancelled;
    e.status = kSchedCancelled;
    e.t_done = clock_();
    --running_;
    drop_in_flight(e.key);
    ++cancelled_;
  }

  const SchedEntry* find(uint64_t ticket) const {
    auto it = jobs_.find(ticket);
    return it == jobs_.end() ? nullptr : &it->second;
  }

  // State as callers see it (ADMITTING reads as QUEUED).
  static int visible_state(const SchedEntry& e) { return e.state == kJobAdmitting ? kJobQueued : e.state; }
  static bool final_state(int s) { return s == kJobDone || s == kJobFailed || s == kJobCancelled; }

  // Forgets a job in a final state.  kSchedInval otherwise.
  int forget(uint64_t ticket) {
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return kSchedNotFound;
    if (!final_state(it->second.state)) return kSchedInval;
    jobs_.erase(it);
    return kSchedOk;
  }

  size_t queued() const { return queue_.size(); }
  size_t running() const { return running_; }
  bool idle() const { return queue_.empty() && running_ == 0; }
  int in_flight(int key) const {
    auto it = in_flight_.find(key);
    return it == in_flight_.end() ? 0 : it->second;
  }
  size_t capacity() const { return capacity_; }
  uint64_t submitted() const { return submitted_; }
  uint64_t done() const { return done_; }
  uint64_t failed() const { return failed_; }
  uint64_t cancelled() const { return cancelled_; }

 private:
  void drop_in_flight(int key) {
    auto it = in_flight_.find(key);
    if (it != in_flight_.end() && --it->second == 0) in_flight_.erase(it);
  }

  Clock clock_;
  size_t capacity_;
  int queue_cap_, max_bypass_;
  uint64_t next_ = 1;
  std::set<uint64_t> queue_;  // queued and admitting tickets; ticket order is arrival order
  std::unordered_map<uint64_t, SchedEntry> jobs_;
  std::map<int, int> in_flight_;
  size_t running_ = 0;
  uint64_t submitted_ = 0, done_ = 0, failed_ = 0, cancelled_ = 0;
};

}  // namespace rtm
