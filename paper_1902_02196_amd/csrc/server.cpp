// Solve server: continuous batching of VIE solves on one GPU.  Each request
// carries its own grid, tissue map, dipole excitations and solver options.
// The scheduler (scheduler.hpp) admits requests by device footprint as slots
// and memory free up; every admitted request runs on its own worker thread,
// context and HIP stream, keeping its operator and Krylov state resident
// until it completes, so the work of concurrent requests overlaps on the GPU.
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "scheduler.hpp"
#include "vie.h"

using namespace vie;

namespace {

// Operators of recently used grids, kept resident for later requests on the
// same grid (key: extents, voxel size, frequency).  Each entry is a context
// that holds the operator and nothing else; requests share it with
// vie_share_grid.  Least recently used entries go when the bytes exceed the
// cap; a request still using an evicted operator keeps it alive until it
// finishes.
struct OpCache {
    using Key = std::tuple<int, int, int, double, double, double, double>;
    struct Entry {
        vie_ctx* holder;
        size_t bytes;
        unsigned long long used;
    };
    std::mutex m;
    std::map<Key, Entry> map;
    size_t cap = 0, in_use = 0;
    unsigned long long clock = 0, hits = 0, misses = 0;

    ~OpCache() {
        for (auto& kv : map) vie_destroy(kv.second.holder);
    }
    // share a cached operator into ctx; false on a miss
    bool take(const Key& k, vie_ctx* ctx) {
        std::lock_guard<std::mutex> g(m);
        auto it = map.find(k);
        if (it == map.end()) {
            ++misses;
            return false;
        }
        if (vie_share_grid(ctx, it->second.holder) != VIE_OK) return false;
        it->second.used = ++clock;
        ++hits;
        return true;
    }
    // remember ctx's operator (just assembled) under k
    void put(const Key& k, vie_ctx* ctx, int device, size_t bytes) {
        if (bytes > cap) return;
        std::lock_guard<std::mutex> g(m);
        if (map.count(k)) return;
        while (in_use + bytes > cap && !map.empty()) {
            auto lru = map.begin();
            for (auto it = map.begin(); it != map.end(); ++it)
                if (it->second.used < lru->second.used) lru = it;
            in_use -= lru->second.bytes;
            vie_destroy(lru->second.holder);
            map.erase(lru);
        }
        vie_ctx* h = nullptr;
        if (vie_create(&h, device, nullptr) != VIE_OK) return;
        if (vie_share_grid(h, ctx) != VIE_OK) {
            vie_destroy(h);
            return;
        }
        map[k] = Entry{h, bytes, ++clock};
        in_use += bytes;
    }
};

struct Request {
    vie_request r{};
    std::vector<double> eps, sig, pos, mom;
    std::vector<vie_solve_stats> stats;
    int device = 0;
    int cached = 0;
    OpCache* cache = nullptr;
    std::string error;
};

// device bytes of a grid's operator: block tensors, both octant spectra
static size_t operator_bytes(int nx, int ny, int nz, const int M[3]) {
    const size_t V = (size_t)nx * ny * nz;
    const size_t O = (size_t)(M[0] / 2 + 1) * (M[1] / 2 + 1) * (M[2] / 2 + 1);
    return 60 * V * 16 + 60 * O * 24 + (size_t)(M[0] + M[1] + M[2]) * 24;
}

int run_request(Request& q) {
    const vie_request& r = q.r;
    VIE_HIP(hipSetDevice(q.device));
    hipStream_t s = nullptr;
    VIE_HIP(hipStreamCreate(&s));
    vie_ctx* ctx = nullptr;
    void* et = nullptr;
    void* x = nullptr;
    int rc = VIE_OK;
    auto fail = [&](int code) {
        if (rc == VIE_OK) {
            rc = code;
            q.error = vie_last_error();
        }
    };
    const int nc = r.basis == 3 ? 3 : 12;
    const long long n = (long long)nc * r.nx * r.ny * r.nz * r.nrhs;
    do {
        int c = vie_create(&ctx, q.device, s);
        if (c) { fail(c); break; }
        const double D[3] = {r.dx, r.dy, r.dz};
        const OpCache::Key key{r.nx, r.ny, r.nz, D[0], D[1], D[2], r.freq_hz};
        if (q.cache && q.cache->take(key, ctx)) {
            q.cached = 1;
        } else {
            if ((c = vie_set_grid(ctx, r.nx, r.ny, r.nz, D[0], D[1], D[2], r.freq_hz, nullptr))) { fail(c); break; }
            if (q.cache) {
                int M[3];
                if (vie_fft_size(ctx, M) == VIE_OK) q.cache->put(key, ctx, q.device, operator_bytes(r.nx, r.ny, r.nz, M));
            }
        }
        if (nc != 12 && (c = vie_set_basis(ctx, nc))) { fail(c); break; }   // the operator serves both bases
        if ((c = vie_set_contrast(ctx, q.eps.data(), q.sig.data(), 0))) { fail(c); break; }
        if (hipMalloc(&et, n * sizeof(double2)) != hipSuccess || hipMalloc(&x, n * sizeof(double2)) != hipSuccess) {
            rc = VIE_ENOMEM;
            q.error = "device allocation of the request vectors failed";
            break;
        }
        if ((c = vie_incident_dipoles(ctx, r.nrhs, q.pos.data(), q.mom.data(), 4, et))) { fail(c); break; }
        vie_solve_opts o;
        vie_default_opts(&o);
        o.mode = r.mode;
        if (r.tol > 0) o.tol = r.tol;
        if (r.restart > 0) o.restart = r.restart;
        q.stats.assign(r.nrhs, vie_solve_stats{});
        c = vie_solve(ctx, &o, r.nrhs, et, x, q.stats.data());
        if (c != VIE_OK) fail(c);
        if (c != VIE_OK && c != VIE_ENOCONV) break;
        if (r.p_abs_out && (c = vie_absorbed_power(ctx, r.nrhs, x, r.p_abs_out))) { fail(c); break; }
        if (r.x_out) {
            if (hipMemcpyAsync(r.x_out, x, n * sizeof(double2), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = VIE_EDEVICE;
                q.error = "copy of the solution failed";
                break;
            }
        }
    } while (false);
    if (ctx) vie_destroy(ctx);
    if (et) (void)hipFree(et);
    if (x) (void)hipFree(x);
    (void)hipStreamDestroy(s);
    return rc;
}

}  // namespace

struct vie_server {
    int device = 0;
    OpCache cache;                       // outlives the scheduler (declared first)
    std::unique_ptr<Scheduler> sched;
};

extern "C" {

int vie_server_create(vie_server** out, int device, size_t hbm_budget, int max_slots) {
    if (!out || max_slots < 1 || hbm_budget == 0) return VIE_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return VIE_EINVAL;
    auto* s = new vie_server();
    s->device = device;
    s->cache.cap = hbm_budget / 8;
    s->sched.reset(new Scheduler(hbm_budget, max_slots, [](SchedJob& j) {
        return run_request(*static_cast<Request*>(j.payload.get()));
    }));
    *out = s;
    return VIE_OK;
}

int vie_server_submit(vie_server* s, const vie_request* r, long long* id) {
    if (!s || !r || !id) return VIE_EINVAL;
    if (r->nx < 1 || r->ny < 1 || r->nz < 1 || r->nrhs < 1 || !r->eps_re || !r->sigma || !r->pos || !r->moment ||
        !(r->dx > 0 && r->dy > 0 && r->dz > 0 && r->freq_hz > 0) ||
        (r->mode != VIE_SOLVE_FP64 && r->mode != VIE_SOLVE_FP32_IR) ||
        (r->basis != 0 && r->basis != 12 && r->basis != 3))
        return VIE_EINVAL;
    auto q = std::make_shared<Request>();
    q->r = *r;
    q->device = s->device;
    q->cache = &s->cache;
    const size_t V = (size_t)r->nx * r->ny * r->nz;
    q->eps.assign(r->eps_re, r->eps_re + V);
    q->sig.assign(r->sigma, r->sigma + V);
    q->pos.assign(r->pos, r->pos + 3 * (size_t)r->nrhs);
    q->mom.assign(r->moment, r->moment + 3 * (size_t)r->nrhs);
    size_t fp = 0;
    if (vie_footprint_bytes(r->nx, r->ny, r->nz, r->nrhs, r->mode, r->restart > 0 ? r->restart : 50, &fp) != VIE_OK)
        return VIE_EINVAL;
    fp += 2 * (size_t)(r->basis == 3 ? 3 : 12) * V * r->nrhs * sizeof(double2);   // request vectors
    const long long k = s->sched->submit(fp, q);
    if (k < 0) return VIE_ENOMEM;                      // can never fit the budget
    *id = k;
    return VIE_OK;
}

int vie_server_poll(vie_server* s, long long id, vie_request_info* info) {
    if (!s || !info) return VIE_EINVAL;
    SchedJob j;
    if (!s->sched->job(id, &j)) return VIE_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->done = j.done ? 1 : 0;
    info->status = j.status;
    info->t_arrival = j.t_arrival;
    info->t_start = j.t_start;
    info->t_end = j.t_end;
    info->footprint = j.footprint;
    if (j.done) {
        const Request& q = *static_cast<Request*>(j.payload.get());
        for (const auto& st : q.stats) {
            info->iterations = std::max(info->iterations, st.iterations);
            info->rel_residual = std::max(info->rel_residual, st.rel_residual);
        }
        std::snprintf(info->message, sizeof(info->message), "%s", q.error.c_str());
        info->operator_cached = q.cached;
    }
    return VIE_OK;
}

int vie_server_wait(vie_server* s) {
    if (!s) return VIE_EINVAL;
    s->sched->wait_all();
    return VIE_OK;
}

int vie_server_stats(vie_server* s, long long first_id, vie_serving_stats* out) {
    if (!s || !out) return VIE_EINVAL;
    Scheduler::Stats st = s->sched->stats(first_id);
    out->completed = st.completed;
    out->queued = st.queued;
    out->running = st.running;
    out->peak_running = st.peak_running;
    out->p50_s = st.p50;
    out->p99_s = st.p99;
    out->mean_s = st.mean;
    out->makespan_s = st.makespan;
    out->peak_bytes = st.peak_in_use;
    out->oldest_queued_s = st.oldest_queued;
    {
        std::lock_guard<std::mutex> g(s->cache.m);
        out->operator_hits = (long long)s->cache.hits;
        out->operator_misses = (long long)s->cache.misses;
        out->operator_cache_bytes = s->cache.in_use;
    }
    return VIE_OK;
}

int vie_server_set_operator_cache(vie_server* s, size_t bytes) {
    if (!s) return VIE_EINVAL;
    std::lock_guard<std::mutex> g(s->cache.m);
    s->cache.cap = bytes;
    while (s->cache.in_use > bytes && !s->cache.map.empty()) {
        auto lru = s->cache.map.begin();
        for (auto it = s->cache.map.begin(); it != s->cache.map.end(); ++it)
            if (it->second.used < lru->second.used) lru = it;
        s->cache.in_use -= lru->second.bytes;
        vie_destroy(lru->second.holder);
        s->cache.map.erase(lru);
    }
    return VIE_OK;
}

void vie_server_destroy(vie_server* s) { delete s; }

}  // extern "C"
