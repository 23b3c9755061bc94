// Autotuner for the launch shapes of the operator product: times each
// candidate with HIP events on the context stream and keeps the fastest per
// (precision, nrhs).  The candidates only change the work distribution (for
// the PWC basis, only the strided passes' tiles); the
// staged x-pass variant adds the terms of the block product in another order
// than the other two, so results agree to rounding.
#include <algorithm>
#include <vector>

#include "ctx.hpp"

namespace vie {

// Milliseconds per product of the installed shape: one warm-up product,
// one timed product to size the sample, then the best of up to three
// trials of enough products for about 3 ms each (a single trial of two
// products once a product takes 2 ms or more), so that products of a few
// tens of microseconds are not ranked by timer noise.
template <typename R>
static double time_apply(Ctx& c, int nrhs, const C<R>* x, C<R>* y) {
    hipEvent_t a, b;
    VIE_HIP(hipEventCreate(&a));
    VIE_HIP(hipEventCreate(&b));
    auto timed = [&](int reps) {
        VIE_HIP(hipEventRecord(a, c.stream));
        for (int i = 0; i < reps; ++i) apply_op<R>(c, OP_N, nrhs, x, y, nullptr);
        VIE_HIP(hipEventRecord(b, c.stream));
        VIE_HIP(hipEventSynchronize(b));
        float ms = 0;
        VIE_HIP(hipEventElapsedTime(&ms, a, b));
        return (double)ms / reps;
    };
    double best = 0;
    try {
        apply_op<R>(c, OP_N, nrhs, x, y, nullptr);   // warm up this shape
        const double t1 = timed(1);
        const bool shortp = t1 < 2.0;
        const int reps = shortp ? std::max(2, std::min(64, (int)(3.0 / std::max(t1, 1e-3)))) : 2;
        best = timed(reps);
        for (int trial = 1; shortp && trial < 3; ++trial) best = std::min(best, timed(reps));
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

template <typename R>
static Tune tune_t(Ctx& c, int nrhs, double* best_ms) {
    const size_t n = (size_t)c.nc * c.V * nrhs;
    C<R>* x = nullptr;
    C<R>* y = nullptr;
    VIE_HIP(hipMalloc(&x, n * sizeof(C<R>)));
    VIE_HIP(hipMalloc(&y, n * sizeof(C<R>)));
    VIE_HIP(hipMemsetAsync(x, 0, n * sizeof(C<R>), c.stream));
    const int key0 = sizeof(R) == 4 ? 0 : 1;
    std::vector<Tune> cands;
    for (int var = 0; var <= 5; ++var)
        for (int sb : {1, 2, 4}) {
            if (var >= 1 && sb != 1) continue;
            if (c.nc == 3 && var != 1) continue;   // one x-pass kernel for the PWC basis: tiles only
            if (var == 0 && p3_ct_supported(c.M[0]) && !p3_ct_fits((int)sizeof(C<R>), c.M[0])) continue;
            if (var == 2 && !p3_quad_fits((int)sizeof(C<R>), c.M[0])) continue;
            if (var == 3 && !p3_pref_fits(c.M[0])) continue;
            if (var == 5 && (nrhs < 2 || !p3_pair_fits((int)sizeof(C<R>), c.M[0]))) continue;
            for (int tz : {4, 8, 16, 32})
                for (int ty : {4, 8, 16, 32}) {
                    Tune t;
                    t.p3_variant = var;
                    t.p3_sib_blocks = sb;
                    t.tile_z = tz;
                    t.tile_y = ty;
                    if (!strided_tile_ok((int)sizeof(C<R>), c.M[2], tz) || !strided_tile_ok((int)sizeof(C<R>), c.M[1], ty))
                        continue;
                    cands.push_back(t);
                }
        }
    c.graphs.clear();   // captured products name the launch shapes
    Tune best;
    double bms = 1e30;
    // candidates are installed one by one while they are timed; a failure
    // puts back what was installed before
    const auto key = std::make_pair(key0, nrhs);
    const auto prev = c.tune.find(key);
    const bool had = prev != c.tune.end();
    const Tune saved = had ? prev->second : Tune{};
    try {
        for (const Tune& t : cands) {
            c.tune[{key0, nrhs}] = t;
            const double ms = time_apply<R>(c, nrhs, x, y);
            if (ms < bms) {
                bms = ms;
                best = t;
            }
        }
    } catch (...) {
        if (had) c.tune[key] = saved;
        else c.tune.erase(key);
        (void)hipFree(x);
        (void)hipFree(y);
        throw;
    }
    VIE_HIP(hipFree(x));
    VIE_HIP(hipFree(y));
    c.tune[{key0, nrhs}] = best;
    if (best_ms) *best_ms = bms;
    return best;
}

Tune autotune(Ctx& c, int precision, int nrhs, double* best_ms) {
    return precision == VIE_C64 ? tune_t<float>(c, nrhs, best_ms) : tune_t<double>(c, nrhs, best_ms);
}

}  // namespace vie
