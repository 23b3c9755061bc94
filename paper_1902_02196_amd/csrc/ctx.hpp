// Library context: grid, resident operator, materials, workspaces.
#pragma once

#include <vector>

#include "../../include/vie.h"
#include "kernels.hpp"

namespace vie {

constexpr double kEps0 = 8.8541878128e-12;   // CODATA 2018
constexpr double kMu0 = 1.25663706212e-6;

struct FftAxis {
    FftPlan plan{};
    double2* tw128 = nullptr;
    float2* tw64 = nullptr;
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

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;

    bool has_grid = false;
    int N[3] = {0, 0, 0};
    int M[3] = {0, 0, 0};
    int O[3] = {0, 0, 0};
    double D[3] = {0, 0, 0};
    double freq = 0, omega = 0, k0 = 0;
    long long V = 0, Osz = 0;
    FftAxis ax[3];

    double2* T = nullptr;      // [60][V] unique block tensors, d >= 0
    double2* U128 = nullptr;   // [60][Osz] octant spectra
    float2* U64 = nullptr;

    bool has_contrast = false;
    Materials mat{};
    double* sigma = nullptr;   // [V]

    Scratch ws;                // FFT intermediates
    Scratch small;             // reductions
    int* flag = nullptr;       // device flag word

    // solver scratch
    Scratch basis, vecs;

    ~Ctx();
    void free_grid();
    void free_contrast();
};

// plan / twiddles (plan.cpp)
FftPlan make_plan(int n);
bool smooth235(int n);
void make_twiddles(int n, std::vector<double2>& tw);

// operator products (apply.cpp)
enum { OP_PREC = 0, OP_A = 1, OP_N = 2, OP_RESID = 3 };
template <typename R>
void apply_op(Ctx& c, int op, int nrhs, const C<R>* x, C<R>* y, const C<R>* rhs);

// solver (solver.cpp)
int solve(Ctx& c, const vie_solve_opts& o, int nrhs, const double2* et, double2* x, vie_solve_stats* st);

}  // namespace vie
