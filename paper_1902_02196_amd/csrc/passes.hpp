// Parameter blocks of the FFT-matvec passes (shared by host and device code).
#pragma once

#include "fft.hpp"

namespace vie {

// Strided 1-D FFT pass over a batch of pencils whose inner (x) index is
// contiguous.  Element k of pencil (o1, o2, t), o1 = 12 r + c (right-hand
// side r, component c):
//   input  in  + r * in_s1  + c * in_sc  + o2 * in_s2  + k * in_sk  + t
//   output out + r * out_s1 + c * out_sc + o2 * out_s2 + k * out_sk + t
// Inputs k >= n_in are implicit zeros (zero padding), outputs k >= n_out are
// not written (crop).  A workgroup handles `tile` consecutive t.
struct StridedPass {
    FftPlan plan;
    int n_in, n_out;
    int n_inner;      // extent of t
    int tile;         // pencils per workgroup
    int pitch;        // LDS row pitch (elements) >= tile
    long long in_s1, in_sc, in_s2, in_sk;
    long long out_s1, out_sc, out_s2, out_sk;
    int nc;           // unknowns per voxel: the grid's z index splits into (rhs, component)
};

// Epilogue of the last pass: y = rhs + a(v) ga[l] x + b(v) gb[l] w
// with w the transformed value, v the voxel (k = z, o2 = y, t = x), and
// l = (component mod 4) for the PWL basis, 0 for the PWC basis; a / b null
// mean the constants a_const / b_const.
template <typename R>
struct Epilogue {
    const C<R>* x;
    const C<R>* rhs;
    const C<R>* a;
    const C<R>* b;
    R a_const, b_const;
    R ga[4];
    R gb[4];
};

// Fused x pass: FFT along x of 12 component rows, per-frequency 12 x 12
// block product with the octant-folded operator, inverse FFT, crop.  The
// operator octant is stored [Oz][Oy][60][Ox]: one contiguous row of 60 Ox
// values per (xi_z, xi_y).
struct P3Params {
    FftPlan plan;     // length Mx
    int Nx, My, Mz;
    int Ox, Oy, Oz;   // octant extents M_i / 2 + 1
    int nrhs;
    long long s_r, s_c, s_z, s_y;   // strides of the [R][Mz][My][12][Nx] buffer
    long long u_e;             // stride between unique operator entries (= Ox)
    int pitch;                 // LDS row pitch (>= Mx)
    int groups;                // pencil groups (12 rows each) per LDS pass
    unsigned magic_nx;         // fast division by Nx
    unsigned magic_ox;         // fast division by Ox
    int sib_blocks;            // workgroups sharing one octant row (1, 2, 4)
    int variant;               // 0: staged operator row, 1: one pencil group per workgroup,
                               // 2: the sibling pencil groups of a row per workgroup (complex64),
                               // 3: as 1 with the operator row prefetched, 4: as 1 with two
                               // threads per frequency, 5: the pencils of two right-hand sides
                               // per workgroup
};

// workgroup size of the x pass: complex64 1024 threads (128 VGPRs each),
// complex128 512 threads (256 VGPRs each)
template <typename R> constexpr int p3_threads() { return 512; }

// LDS bytes of the x pass: operator row, twiddles, padded pencil groups
__host__ __device__ constexpr long long p3_lds_bytes(int es, int n, int g) {
    const long long rows = (long long)g * 12 * n;
    return ((long long)60 * (n / 2 + 1) + n + rows + rows / 16 + 4) * es;
}

// pencil groups per LDS pass for the compile-time-length kernels: as many as
// fit 96 KiB of LDS (and two threads per frequency column), at most four
__host__ __device__ constexpr int p3_gmax(int es, int n, int nthr) {
    int g = 4;
    while (g > 1 && (p3_lds_bytes(es, n, g) > 96 * 1024 || 2 * g * n > nthr)) --g;
    return g;
}

}  // namespace vie
