// Continuous-batching scheduler for solve requests (no HIP here, so the
// admission and bookkeeping logic also builds and runs on the host alone).
//
// Requests wait in arrival order.  A request is admitted when a worker slot
// is free and its device footprint fits the remaining memory budget; while
// the head of the queue does not fit, later requests that do fit may go
// first (backfill), so small solves are not held behind a large one.
// Backfill is bounded: once the head has been passed over max_bypass times,
// nothing more is admitted ahead of it, so the running requests drain until
// it fits (no request waits forever behind a stream of smaller ones).  A
// fixed pool of `slots` worker threads runs the admitted requests (in the GPU
// executor each on its own stream), so the work of all admitted requests
// overlaps on the device.  Finished requests release their slot and memory,
// and the queue is re-examined at once.  Latency = completion - arrival
// (queueing included); the statistics also give the age of the oldest
// request still queued, which completed-request percentiles cannot show.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace vie {

struct SchedJob {
    long long id = 0;
    size_t footprint = 0;
    double t_arrival = 0, t_start = 0, t_end = 0;   // seconds since the scheduler started
    int status = 0;
    bool done = false;
    std::shared_ptr<void> payload;                  // executor data (inputs, results)
};

class Scheduler {
  public:
    using RunFn = std::function<int(SchedJob&)>;

    static constexpr int kDefaultMaxBypass = 8;

    Scheduler(size_t budget, int slots, RunFn run, int max_bypass = kDefaultMaxBypass)
        : budget_(budget), slots_(std::max(1, slots)), max_bypass_(std::max(0, max_bypass)), run_(std::move(run)),
          t0_(clock::now()) {
        workers_.reserve(slots_);
        for (int i = 0; i < slots_; ++i) workers_.emplace_back([this] { worker_loop(); });
    }

    ~Scheduler() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : workers_) t.join();
    }

    double now() const { return std::chrono::duration<double>(clock::now() - t0_).count(); }

    // returns the id, or -1 when the footprint can never fit the budget
    long long submit(size_t footprint, std::shared_ptr<void> payload) {
        std::lock_guard<std::mutex> g(m_);
        if (footprint > budget_) return -1;
        auto j = std::make_shared<SchedJob>();
        j->id = next_id_++;
        j->footprint = footprint;
        j->t_arrival = now();
        j->payload = std::move(payload);
        jobs_[j->id] = j;
        queue_.push_back(j);
        cv_.notify_all();
        return j->id;
    }

    // copy of a job's state taken under the lock (false for unknown ids); once
    // done is seen, the executor's writes to the payload are visible too
    bool job(long long id, SchedJob* out) {
        std::lock_guard<std::mutex> g(m_);
        auto it = jobs_.find(id);
        if (it == jobs_.end()) return false;
        *out = *it->second;
        return true;
    }

    void wait_all() {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [this] { return queue_.empty() && running_ == 0; });
    }

    struct Stats {
        int completed = 0, queued = 0, running = 0;
        size_t in_use = 0, peak_in_use = 0;
        int peak_running = 0;
        double p50 = 0, p99 = 0, mean = 0, makespan = 0;
        double oldest_queued = 0;   // age of the oldest request still waiting (s)
    };

    // latency statistics over completed jobs with id >= first_id
    Stats stats(long long first_id = 0) {
        std::lock_guard<std::mutex> g(m_);
        Stats s;
        std::vector<double> lat;
        double t_first = 1e300, t_last = 0;
        for (auto& kv : jobs_) {
            const SchedJob& j = *kv.second;
            if (!j.done || j.id < first_id) continue;
            lat.push_back(j.t_end - j.t_arrival);
            t_first = std::min(t_first, j.t_arrival);
            t_last = std::max(t_last, j.t_end);
        }
        s.completed = (int)lat.size();
        s.queued = (int)queue_.size();
        s.running = running_;
        s.in_use = in_use_;
        s.peak_in_use = peak_in_use_;
        s.peak_running = peak_running_;
        const double t = now();
        for (auto& j : queue_) s.oldest_queued = std::max(s.oldest_queued, t - j->t_arrival);
        if (!lat.empty()) {
            std::sort(lat.begin(), lat.end());
            auto pct = [&](double p) {
                // nearest-rank percentile
                size_t k = (size_t)std::ceil(p * lat.size());
                if (k < 1) k = 1;
                return lat[std::min(k, lat.size()) - 1];
            };
            s.p50 = pct(0.50);
            s.p99 = pct(0.99);
            double sum = 0;
            for (double v : lat) sum += v;
            s.mean = sum / lat.size();
            s.makespan = t_last - t_first;
        }
        return s;
    }

  private:
    using clock = std::chrono::steady_clock;

    // each worker admits the next request that may start, runs it, releases
    // its slot and memory, and looks again; it leaves once stop_ is set
    // (queued requests that never started are dropped)
    void worker_loop() {
        std::unique_lock<std::mutex> lk(m_);
        for (;;) {
            cv_.wait(lk, [this] { return stop_ || pick() != queue_.end(); });
            if (stop_) break;
            auto it = pick();
            std::shared_ptr<SchedJob> j = *it;
            if (it != queue_.begin()) head_bypass_ += 1;   // backfilled past the head
            else head_bypass_ = 0;                          // the head itself starts
            queue_.erase(it);
            in_use_ += j->footprint;
            running_ += 1;
            peak_in_use_ = std::max(peak_in_use_, in_use_);
            peak_running_ = std::max(peak_running_, running_);
            j->t_start = now();
            lk.unlock();
            int st = 0;
            try {
                st = run_(*j);
            } catch (...) {
                st = -3;
            }
            lk.lock();
            j->status = st;
            j->t_end = now();
            j->done = true;
            in_use_ -= j->footprint;
            running_ -= 1;
            cv_.notify_all();
        }
    }

    // the request that may start now: the head when it fits; otherwise the
    // first later request that fits, unless the head has been passed over
    // max_bypass_ times already; end() when none (a free slot is implied:
    // a worker only asks when it is idle)
    std::deque<std::shared_ptr<SchedJob>>::iterator pick() {
        if (queue_.empty()) return queue_.end();
        if (in_use_ + queue_.front()->footprint <= budget_) return queue_.begin();
        if (head_bypass_ >= max_bypass_) return queue_.end();
        for (auto it = queue_.begin() + 1; it != queue_.end(); ++it)
            if (in_use_ + (*it)->footprint <= budget_) return it;
        return queue_.end();
    }

    size_t budget_;
    int slots_;
    int max_bypass_;
    RunFn run_;
    clock::time_point t0_;
    std::mutex m_;
    std::condition_variable cv_;
    std::deque<std::shared_ptr<SchedJob>> queue_;
    std::map<long long, std::shared_ptr<SchedJob>> jobs_;
    std::vector<std::thread> workers_;
    long long next_id_ = 0;
    int head_bypass_ = 0;   // admissions past the current head of the queue
    size_t in_use_ = 0, peak_in_use_ = 0;
    int running_ = 0, peak_running_ = 0;
    bool stop_ = false;
};

}  // namespace vie
