// Library context: grid, resident operator, materials, workspaces.
#pragma once

#include <complex>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "vie.h"
#include "kernels.hpp"

namespace vie {

constexpr double kEps0 = 8.8541878128e-12;   // CODATA 2018
constexpr double kMu0 = 1.25663706212e-6;

struct FftAxis {
    FftPlan plan{};
    double2* tw128 = nullptr;
    float2* tw64 = nullptr;
};

// Device operator of one grid: block tensors, octant spectra and twiddles.
// Contexts on the same grid (extents, voxel size, frequency, fft size) may
// share one read-only copy; the last owner frees it.
struct OperatorData {
    FftAxis ax[3];
    double2* T = nullptr;
    double2* U128 = nullptr;
    float2* U64 = nullptr;
    // curl operator K (eq. 8b, 25b), built on first use by a magnetic-field
    // call or a J-M product: 30 unique tensors [30][V] and their octant
    // [Oz][Oy][30][Ox], complex128 and complex64
    double2* TK = nullptr;
    double2* UK128 = nullptr;
    float2* UK64 = nullptr;
    std::mutex curl_m;
    size_t bytes = 0;
    ~OperatorData() {
        for (auto& a : ax) {
            if (a.tw128) (void)hipFree(a.tw128);
            if (a.tw64) (void)hipFree(a.tw64);
        }
        if (T) (void)hipFree(T);
        if (U128) (void)hipFree(U128);
        if (U64) (void)hipFree(U64);
        if (TK) (void)hipFree(TK);
        if (UK128) (void)hipFree(UK128);
        if (UK64) (void)hipFree(UK64);
    }
};

// device buffer that only grows
struct Scratch {
    void* p = nullptr;
    size_t bytes = 0;
    void* get(size_t need) {
        if (need > bytes) {
            if (p) VIE_HIP(hipFree(p));
            p = nullptr;
            bytes = 0;
            VIE_HIP(hipMalloc(&p, need));
            bytes = need;
        }
        return p;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// page-locked host buffer that only grows (asynchronous device-to-host copies)
struct PinnedScratch {
    void* p = nullptr;
    size_t bytes = 0;
    void* get(size_t need) {
        if (need > bytes) {
            if (p) VIE_HIP(hipHostFree(p));
            p = nullptr;
            bytes = 0;
            VIE_HIP(hipHostMalloc(&p, need, hipHostMallocDefault));
            bytes = need;
        }
        return p;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// HIP-event timing of kernel launches, by class
struct Profiler {
    struct Rec { int kind; hipEvent_t a, b; double bytes; };
    bool on = false;
    int every = 1;                 // record one launch in `every` per class
    unsigned long long tick[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool sample(int kind) { return (tick[kind & 7]++ % (unsigned long long)every) == 0; }
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t take() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e;
        VIE_HIP(hipEventCreate(&e));
        return e;
    }
    void clear() {
        for (auto& r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
        recs.clear();
    }
    ~Profiler() {
        clear();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// RAII scope that records one launch when profiling is on
struct ProfScope {
    Profiler& p;
    hipStream_t s;
    int kind;
    double bytes;
    hipEvent_t a = nullptr;
    ProfScope(Profiler& p_, hipStream_t s_, int k, double b) : p(p_), s(s_), kind(k), bytes(b) {
        if (p.on && p.sample(k)) { a = p.take(); VIE_HIP(hipEventRecord(a, s)); }
    }
    ~ProfScope() {
        if (p.on && a) {
            hipEvent_t b_ = p.take();
            (void)hipEventRecord(b_, s);
            p.recs.push_back(Profiler::Rec{kind, a, b_, bytes});
        }
    }
};

// records one kernel launch of a class by its own dispatch timestamps (the
// launch must go through timed_launch) when profiling samples it
struct KernelTiming {
    Profiler& p;
    int kind;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    KernelTiming(Profiler& p_, int k, double by) : p(p_), kind(k), bytes(by) {
        if (p.on && p.sample(k)) {
            a = p.take();
            b = p.take();
            g_launch_timing = LaunchTiming{a, b};
        }
    }
    ~KernelTiming() {
        if (!a) return;
        if (g_launch_timing.start == a) {   // no launch took the events (an error came first)
            g_launch_timing = LaunchTiming{};
            p.pool.push_back(a);
            p.pool.push_back(b);
            return;
        }
        p.recs.push_back(Profiler::Rec{kind, a, b, bytes});
    }
};

// Captured runs of Arnoldi steps (solver.cpp), by their launch key: shapes,
// step range and the buffers the launches name.  A key seen for the first
// time runs uncaptured (which also sizes every lazily grown buffer); the
// second time it is captured on a private stream and instantiated; later
// uses replay it.  Cleared whenever the grid, materials, basis or launch
// shapes change.
struct GraphCache {
    std::map<std::vector<long long>, hipGraphExec_t> execs;
    hipStream_t cap = nullptr;   // capture stream (the context's may be the null stream)
    static constexpr size_t kMax = 512;
    void clear() {
        for (auto& kv : execs)
            if (kv.second) (void)hipGraphExecDestroy(kv.second);
        execs.clear();
    }
    ~GraphCache() {
        clear();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// Tucker form of one Toeplitz-defining tensor (tucker.hip), complex128 on
// the host: factors U_i (N_i x r_i, row-major) for x, y, z and the core
// [r_z][r_y][r_x]
struct TuckerTensor {
    int r[3] = {0, 0, 0};
    std::vector<std::vector<std::complex<double>>> U;
    std::vector<std::complex<double>> core;
    double norm = 0, rel_error = 0;   // ||T||_F and ||T - T_hat||_F / ||T||_F
};
struct TuckerForm {
    bool valid = false;
    double tol = 0;
    std::vector<TuckerTensor> tensors;   // the 60 unique tensors
    size_t values() const;               // complex values stored
    void clear() {
        valid = false;
        tensors.clear();
    }
};

// launch shapes of the operator product, chosen per (precision, nrhs) by
// the autotuner; zeros mean the built-in defaults
struct Tune {
    int p3_variant = -1;     // -1 default, 0 staged operator row, 1 light
    int p3_sib_blocks = 0;   // staged variant: workgroups per octant row
    int tile_z = 0;          // strided passes: pencils per workgroup
    int tile_y = 0;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;

    bool has_grid = false;
    int nc = 12;               // unknowns per voxel: 12 PWL, 3 PWC (l = 1 only)
    int N[3] = {0, 0, 0};
    int M[3] = {0, 0, 0};
    int O[3] = {0, 0, 0};
    double D[3] = {0, 0, 0};
    double freq = 0, omega = 0, k0 = 0;
    long long V = 0, Osz = 0;
    FftAxis ax[3];

    std::shared_ptr<OperatorData> op;   // owner of the buffers below
    double2* T = nullptr;      // [60][V] unique block tensors, d >= 0
    double2* U128 = nullptr;   // [60][Osz] octant spectra
    float2* U64 = nullptr;

    bool has_contrast = false;
    Materials mat{};
    double* sigma = nullptr;   // [V]
    // magnetic contrast of the J-M formulation (nc = 24): mu_r, chi_m, tau_m
    // in the slots of eps_r, chi, tau; unset means mu_r = 1 everywhere
    bool has_mcontrast = false;
    Materials mmat{};
    Scratch jmbuf;             // N x and K x of the J-M product

    Scratch ws;                // FFT intermediates
    Scratch small;             // reductions
    int* flag = nullptr;       // device flag word

    // solver scratch
    Scratch basis, vecs;
    PinnedScratch hpin;           // Hessenberg columns on their way to the host
    hipEvent_t col_ev[2] = {nullptr, nullptr};

    Profiler prof;
    std::map<std::pair<int, int>, Tune> tune;   // (precision, nrhs) -> shapes
    GraphCache graphs;
    TuckerForm tucker;          // compressed copy of the grid's 60 tensors

    ~Ctx();
    void free_grid();
    void free_contrast();
    void free_mcontrast();
};

// plan / twiddles (plan.cpp)
FftPlan make_plan(int n);
bool smooth235(int n);
void make_twiddles(int n, std::vector<double2>& tw);

// operator products (apply.cpp); OP_CURL: h = G^-1 (h_t + K x) with the
// curl operator, h_t passed as rhs (complex128, PWL basis)
// OP_K: y = K x, the raw curl product (the J-M product's coupling blocks)
// OP_JMS: the J-M coupled sums over nrhs / 2 vector pairs (x_j, x_m) =
// vectors (2 r, 2 r + 1): y_j = N x_j - c_e K x_m, y_m = N x_m + c_m K x_j,
// in one pass of the FFTs (only where jm_fused_supported)
enum { OP_PREC = 0, OP_A = 1, OP_N = 2, OP_RESID = 3, OP_CURL = 4, OP_K = 5, OP_JMS = 6 };
bool jm_fused_supported(const Ctx& c, size_t es);
// ws_ext: caller-owned workspace of ws_cap bytes for the FFT intermediates
// (VIE_EINVAL when the product needs more); nullptr: the context's own,
// grown on demand
template <typename R>
void apply_op(Ctx& c, int op, int nrhs, const C<R>* x, C<R>* y, const C<R>* rhs, void* ws_ext = nullptr,
              size_t ws_cap = 0);
size_t apply_workspace_bytes(const Ctx& c, int nrhs, size_t es);

// J-M formulation (nc = 24, jm.hip): the product from one N and one K
// product over the 2 nrhs 12-component halves; OP_PREC, OP_A, OP_RESID
template <typename R>
void apply_jm(Ctx& c, int op, int nrhs, const C<R>* x, C<R>* y, const C<R>* rhs, void* ws_ext, size_t ws_cap);
// P^-1 b of the J-M system from [e_t; h_t] (complex128, [nrhs][24][V])
void jm_rhs_prec(Ctx& c, int nrhs, const double2* eh_t, double2* rhs);
// mu_r = 1 everywhere (the default magnetic contrast of a J-M context)
void jm_default_mcontrast(Ctx& c);
// the component count, set for the lifetime of the guard (the J-M product
// runs its halves as 12-component products)
struct NcGuard {
    Ctx& c;
    int saved;
    NcGuard(Ctx& c_, int nc) : c(c_), saved(c_.nc) { c.nc = nc; }
    ~NcGuard() { c.nc = saved; }
};

// build the curl operator of the context's grid if it is not there yet
// (magnetic.cpp); shared operators build it once
void ensure_curl(Ctx& c);
// tested incident magnetic field of a plane wave (12 components, one
// right-hand side) into h_t (magnetic.cpp)
void planewave_h(Ctx& c, const double pol[3], const double dir[3], double amp, double2* h_t);

// fixed per-device workspace of vie_apply_noalloc (noalloc.hip): looked up
// once per device by vie_create with that device current
void noalloc_init(int device);

// status-code guard of the C entry points (capi.cpp): runs f, turns an
// exception into its status and keeps the message for vie_last_error
extern thread_local std::string g_err;
template <typename F>
int guarded(F&& f) {
    try {
        g_err.clear();
        f();
        return VIE_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return VIE_EDEVICE;
    }
}

// Tucker compression of the 60 Toeplitz-defining tensors at relative
// tolerance tol (tucker.hip), and the reconstruction T_hat [60][V] into out
void tucker_compress(Ctx& c, double tol);
void tucker_reconstruct(Ctx& c, double2* out);

// autotuner (tune.cpp): fastest launch shapes for (precision, nrhs)
Tune autotune(Ctx& c, int precision, int nrhs, double* best_ms);

// solver (solver.cpp)
int solve(Ctx& c, const vie_solve_opts& o, int nrhs, const double2* et, double2* x, vie_solve_stats* st);

}  // namespace vie

// the opaque handle of the C ABI
struct vie_ctx {
    vie::Ctx c;
};
