// Autotuner for the launch shapes of the operator product: times each
// candidate with HIP events on the context stream and keeps the fastest per
// (precision, nrhs).  The candidates only change the work distribution (for
// the PWC basis, only the strided passes' tiles); the
// staged x-pass variant adds the terms of the block product in another order
// than the other two, so results agree to rounding.
#include <vector>

#include "ctx.hpp"

namespace vie {

template <typename R>
static double time_apply(Ctx& c, int nrhs, const C<R>* x, C<R>* y, int reps) {
    hipEvent_t a, b;
    VIE_HIP(hipEventCreate(&a));
    VIE_HIP(hipEventCreate(&b));
    apply_op<R>(c, OP_N, nrhs, x, y, nullptr);   // warm up this shape
    VIE_HIP(hipEventRecord(a, c.stream));
    for (int i = 0; i < reps; ++i) apply_op<R>(c, OP_N, nrhs, x, y, nullptr);
    VIE_HIP(hipEventRecord(b, c.stream));
    VIE_HIP(hipEventSynchronize(b));
    float ms = 0;
    VIE_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
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
    for (int var = 0; var <= 4; ++var)
        for (int sb : {1, 2, 4}) {
            if (var >= 1 && sb != 1) continue;
            if (c.nc == 3 && var != 1) continue;   // one x-pass kernel for the PWC basis: tiles only
            if (var == 0 && p3_ct_supported(c.M[0]) && !p3_ct_fits((int)sizeof(C<R>), c.M[0])) continue;
            if (var == 2 && !p3_quad_fits((int)sizeof(C<R>), c.M[0])) continue;
            if (var == 3 && !p3_pref_fits(c.M[0])) continue;
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
    const int reps = c.V * nrhs > 4000000 ? 2 : 5;
    // candidates are installed one by one while they are timed; a failure
    // puts back what was installed before
    const auto key = std::make_pair(key0, nrhs);
    const auto prev = c.tune.find(key);
    const bool had = prev != c.tune.end();
    const Tune saved = had ? prev->second : Tune{};
    try {
        for (const Tune& t : cands) {
            c.tune[{key0, nrhs}] = t;
            const double ms = time_apply<R>(c, nrhs, x, y, reps);
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
