// Parameter blocks of the FFT-matvec passes (shared by host and device code).
#pragma once

#include "fft.hpp"

namespace vie {

// Strided 1-D FFT pass over a batch of pencils whose inner (x) index is
// contiguous.  Element k of pencil (o1, o2, t):
//   input  in  + o1 * in_s1  + o2 * in_s2  + k * in_sk  + t
//   output out + o1 * out_s1 + o2 * out_s2 + k * out_sk + t
// Inputs k >= n_in are implicit zeros (zero padding), outputs k >= n_out are
// not written (crop).  A workgroup handles `tile` consecutive t.
struct StridedPass {
    FftPlan plan;
    int n_in, n_out;
    int n_inner;      // extent of t
    int tile;         // pencils per workgroup
    int pitch;        // LDS row pitch (elements) >= tile
    long long in_s1, in_s2, in_sk;
    long long out_s1, out_s2, out_sk;
};

// Epilogue of the last pass: y = rhs + a(v) ga[l] x + b(v) gb[l] w
// with w the transformed value, v the voxel (k = z, o2 = y, t = x), and
// l = (component mod 4); a / b null mean the constants a_const / b_const.
template <typename R>
struct Epilogue {
    const C<R>* x;
    const C<R>* rhs;
    const C<R>* a;
    const C<R>* b;
    R a_const, b_const;
    R ga[4];
    R gb[4];
    long long s1;     // stride between components of the batch (= N_V)
};

// Fused x pass: FFT along x of 12 component rows, per-frequency 12 x 12
// block product with the octant-folded operator, inverse FFT, crop.
struct P3Params {
    FftPlan plan;     // length Mx
    int Nx, My, Mz;
    int Ox, Oy, Oz;   // octant extents M_i / 2 + 1
    int nrhs;
    long long s_b, s_z, s_y;   // strides of the [B][Mz][My][Nx] buffer
    long long u_e;             // stride between unique operator entries
    int pitch;                 // LDS row pitch (>= Mx)
};

}  // namespace vie
