// Host-only checks of the continuous-batching scheduler with a fake executor
// (sleeps stand in for solves).  Prints "ok <case>" per passing case and
// exits non-zero on the first failure.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

#include "scheduler.hpp"

using namespace vie;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);           \
            std::fflush(stdout);                                              \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

struct Fake {
    int ms;
    int status;
    bool thrown;
};

static Scheduler::RunFn fake_run(std::atomic<int>* live = nullptr, std::atomic<int>* peak = nullptr) {
    return [live, peak](SchedJob& j) {
        auto* f = static_cast<Fake*>(j.payload.get());
        if (live) {
            int v = ++*live;
            int p = peak->load();
            while (v > p && !peak->compare_exchange_weak(p, v)) {
            }
        }
        std::this_thread::sleep_for(std::chrono::milliseconds(f->ms));
        if (live) --*live;
        if (f->thrown) throw 1;
        return f->status;
    };
}

static SchedJob get(Scheduler& s, long long id) {
    SchedJob j;
    CHECK(s.job(id, &j));
    return j;
}

static std::shared_ptr<void> job(int ms, int status = 0, bool thrown = false) {
    return std::make_shared<Fake>(Fake{ms, status, thrown});
}

int main() {
    {   // a request larger than the whole budget is refused at submission
        Scheduler s(100, 2, fake_run());
        CHECK(s.submit(101, job(1)) == -1);
        CHECK(s.submit(100, job(1)) == 0);
        s.wait_all();
        CHECK(get(s, 0).done && get(s, 0).status == 0);
        SchedJob none;
        CHECK(!s.job(7, &none));
        std::printf("ok oversize\n");
    }
    {   // slots bound concurrency and are reused as requests finish
        std::atomic<int> live{0}, peak{0};
        Scheduler s(1000, 3, fake_run(&live, &peak));
        for (int i = 0; i < 9; ++i) CHECK(s.submit(10, job(60)) == i);
        s.wait_all();
        auto st = s.stats();
        CHECK(st.completed == 9 && st.queued == 0 && st.running == 0);
        CHECK(st.peak_running == 3 && peak.load() == 3);
        CHECK(st.peak_in_use == 30);
        CHECK(st.makespan >= 0.175 && st.makespan < 0.9);   // three waves of 60 ms, not nine
        std::printf("ok slots\n");
    }
    {   // memory budget bounds concurrency even with free slots
        std::atomic<int> live{0}, peak{0};
        Scheduler s(25, 8, fake_run(&live, &peak));
        for (int i = 0; i < 6; ++i) s.submit(10, job(40));
        s.wait_all();
        auto st = s.stats();
        CHECK(st.peak_in_use <= 25 && st.peak_running == 2 && peak.load() == 2);
        std::printf("ok budget\n");
    }
    {   // backfill: a small request behind a blocked large one starts first
        Scheduler s(10, 4, fake_run());
        long long a = s.submit(8, job(300));
        std::this_thread::sleep_for(std::chrono::milliseconds(30));   // a is running
        long long b = s.submit(8, job(10));                           // does not fit beside a
        long long c = s.submit(2, job(10));                           // fits beside a
        s.wait_all();
        auto ja = get(s, a), jb = get(s, b), jc = get(s, c);
        CHECK(jc.t_start < jb.t_start);
        CHECK(jc.t_end < ja.t_end);           // finished while a still ran
        CHECK(jb.t_start >= ja.t_end - 1e-3); // b waited for a's memory
        std::printf("ok backfill\n");
    }
    {   // bounded backfill: after max_bypass admissions past a head that does
        // not fit, later requests wait behind it; the oldest queued age shows
        Scheduler s(20, 4, fake_run(), 2);
        long long a = s.submit(10, job(150));
        std::this_thread::sleep_for(std::chrono::milliseconds(30));   // a is running
        long long b = s.submit(15, job(10));                          // waits for a's memory
        std::vector<long long> c;
        for (int i = 0; i < 4; ++i) c.push_back(s.submit(2, job(150)));
        std::this_thread::sleep_for(std::chrono::milliseconds(40));
        auto mid = s.stats();
        CHECK(mid.queued == 3 && mid.oldest_queued >= 0.035);         // b, c[2], c[3] wait
        s.wait_all();
        auto ja = get(s, a), jb = get(s, b);
        CHECK(get(s, c[0]).t_start < ja.t_end && get(s, c[1]).t_start < ja.t_end);   // two bypasses
        CHECK(get(s, c[2]).t_start >= ja.t_end - 1e-3);                              // then b's turn
        CHECK(jb.t_start <= get(s, c[2]).t_start && jb.t_start <= get(s, c[3]).t_start);
        CHECK(s.stats().oldest_queued == 0.0);
        std::printf("ok aging\n");
    }
    {   // FIFO among requests that fit
        Scheduler s(100, 1, fake_run());
        std::vector<long long> ids;
        for (int i = 0; i < 5; ++i) ids.push_back(s.submit(1, job(15)));
        s.wait_all();
        for (int i = 1; i < 5; ++i) CHECK(get(s, ids[i]).t_start >= get(s, ids[i - 1]).t_end - 1e-3);
        std::printf("ok fifo\n");
    }
    {   // statuses and exceptions of the executor are recorded
        Scheduler s(100, 2, fake_run());
        long long a = s.submit(1, job(1, -4));
        long long b = s.submit(1, job(1, 0, true));
        s.wait_all();
        CHECK(get(s, a).status == -4 && get(s, b).status == -3 && get(s, b).done);
        std::printf("ok status\n");
    }
    {   // nearest-rank percentiles of latency; first_id drops a warm-up prefix
        Scheduler s(1000, 100, fake_run());
        s.submit(1, job(400));   // warm-up outlier, id 0
        for (int i = 1; i <= 10; ++i) s.submit(1, job(20 * i));
        s.wait_all();
        auto all = s.stats(0), tail = s.stats(1);
        CHECK(all.completed == 11 && tail.completed == 10);
        // latencies ~ 20 i ms: p50 = 5th = ~100 ms, p99 = 10th = ~200 ms
        CHECK(tail.p50 > 0.095 && tail.p50 < 0.16);
        CHECK(tail.p99 > 0.195 && tail.p99 < 0.30);
        CHECK(all.p99 > 0.395);
        CHECK(tail.mean > 0.105 && tail.mean < 0.17);
        std::printf("ok percentiles\n");
    }
    {   // destruction waits for running requests and drops queued ones
        std::atomic<int> live{0}, peak{0};
        {
            Scheduler s(1000, 1, fake_run(&live, &peak));
            for (int i = 0; i < 4; ++i) s.submit(1, job(50));
            std::this_thread::sleep_for(std::chrono::milliseconds(20));
        }
        CHECK(live.load() == 0);
        std::printf("ok shutdown\n");
    }
    return 0;
}
