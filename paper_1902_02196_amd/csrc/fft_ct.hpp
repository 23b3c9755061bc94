// Stockham FFT of rows in LDS for a compile-time length N: the radix
// sequence, loop bounds, index divisions and the butterflies per thread are
// all constants, so every pass unrolls into straight-line code.  Same
// algorithm as fft.hpp: pass s with radix r and span Ns maps butterfly j
// (k = j mod Ns) from X[j + i N/r] to Y[(j - k) r + k + i Ns], in place with
// the inputs of a pass staged in registers between two barriers.  Twiddles
// W_N^m are read from a copy of the table in LDS.
#pragma once

#include "fft.hpp"

namespace vie {

// radix of pass s for length n (0 past the last pass): 16s first, then one
// 8 / 4 / 2 for the rest of the power of two, then 3s, then 5s
__host__ __device__ constexpr int ct_radix(int n, int s) {
    int m = n, idx = 0;
    while (m % 16 == 0) { if (idx == s) return 16; m /= 16; ++idx; }
    if (m % 8 == 0) { if (idx == s) return 8; m /= 8; ++idx; }
    if (m % 4 == 0) { if (idx == s) return 4; m /= 4; ++idx; }
    if (m % 2 == 0) { if (idx == s) return 2; m /= 2; ++idx; }
    while (m % 3 == 0) { if (idx == s) return 3; m /= 3; ++idx; }
    while (m % 5 == 0) { if (idx == s) return 5; m /= 5; ++idx; }
    return 0;
}

// HIN: the inputs of the upper half of each row are zero (a zero-padded
// forward transform, first pass only): they are neither read nor added.
// HOUT: only the lower half of each row is used afterwards (a cropped inverse
// transform, last pass only): the upper half is neither stored nor, once the
// compiler drops the dead arithmetic, computed.
// Rows are pitch = N elements apart before padding (every caller).  RP is
// the padded row pitch: N + N / 16 (the lds_pad layout of a row-major block)
// or, for N a multiple of 16, any larger value, with the elements of row t
// at t RP + lds_pad(c).
template <typename R, bool FWD, int N, int RAD, int NS, int NTHR, int MAXROWS, bool HIN = false,
          bool HOUT = false, int RP = N + N / 16>
__device__ __forceinline__ void ct_pass(C<R>* buf, const C<R>* twl, int rows, int pitch, int tid) {
    static_assert(!HIN || (NS == 1 && RAD % 2 == 0), "half-zero input only on an even first pass");
    static_assert(!HOUT || (NS * RAD == N && RAD % 2 == 0), "half output only on an even last pass");
    static_assert(RP == N + N / 16 || (N % 16 == 0 && RP > N + N / 16), "row pitch");
    // element c of row t (c < N)
    auto at = [&](int t, int c) { return RP == N + N / 16 ? lds_pad(t * pitch + c) : t * RP + lds_pad(c); };
    constexpr int nb = N / RAD;
    constexpr int NB = (MAXROWS * nb + NTHR - 1) / NTHR;
    constexpr int twstep = N / (NS * RAD);
    // Padded addresses of a row made of whole 16-element blocks (N % 16 ==
    // 0): t RP + c + (c >> 4).
    // For the c a butterfly touches, c = c0 + i S with stride S, the block
    // term splits into a per-thread part and a compile-time part when S is
    // a multiple of 16, or S divides 16 and c0's position keeps c0 + i S in
    // the block of i S (every pass below): then the address is one per-thread
    // base plus constant offsets, with no per-element index arithmetic.
    constexpr int RB = RP;
    constexpr bool AFF_IN = N % 16 == 0 && (nb % 16 == 0 || 16 % nb == 0);
    constexpr bool AFF_OUT = N % 16 == 0 && (NS % 16 == 0 ||
                                             (16 % NS == 0 && ((NS * RAD) % 16 == 0 || 16 % (NS * RAD) == 0)));
    const int total = rows * nb;
    C<R> v[NB][RAD];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int idx = tid + q * NTHR;
        if (idx < total) {
            const int t = idx / nb, j = idx - t * nb;
            if constexpr (AFF_IN) {
                const C<R>* src = buf + (t * RB + j + (j >> 4));
#pragma unroll
                for (int i = 0; i < (HIN ? RAD / 2 : RAD); ++i) v[q][i] = src[i * nb + ((i * nb) >> 4)];
            } else {
#pragma unroll
                for (int i = 0; i < (HIN ? RAD / 2 : RAD); ++i) v[q][i] = buf[at(t, j + i * nb)];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int idx = tid + q * NTHR;
        if (idx < total) {
            const int t = idx / nb, j = idx - t * nb;
            const int k = j % NS;
            if constexpr (NS > 1) {
#pragma unroll
                for (int i = 1; i < RAD; ++i) {
                    C<R> w = twl[i * k * twstep];
                    if (!FWD) w.y = -w.y;
                    v[q][i] = cmul(v[q][i], w);
                }
            }
            if constexpr (HIN) dft_r_halfin<R, FWD, RAD>(v[q]);
            else dft_r<R, FWD, RAD>(v[q]);
            if constexpr (AFF_OUT) {
                const int b0 = (j - k) * RAD + k;
                C<R>* dst = buf + (t * RB + b0 + (b0 >> 4));
#pragma unroll
                for (int i = 0; i < (HOUT ? RAD / 2 : RAD); ++i) dst[i * NS + ((i * NS) >> 4)] = v[q][i];
            } else {
                const int c0 = (j - k) * RAD + k;
#pragma unroll
                for (int i = 0; i < (HOUT ? RAD / 2 : RAD); ++i) buf[at(t, c0 + i * NS)] = v[q][i];
            }
        }
    }
    __syncthreads();
}

// HIN: rows are zero beyond N / 2 (zero-padded forward transform); the
// first pass then skips the zero half when its radix is even
// HOUT: only positions below N / 2 are read after the transform (cropped
// inverse); the last pass then stores the lower half when its radix is even
template <typename R, bool FWD, int N, int S, int NS, int NTHR, int MAXROWS, bool HIN = false, bool HOUT = false,
          int RP = N + N / 16>
__device__ __forceinline__ void ct_passes(C<R>* buf, const C<R>* twl, int rows, int pitch, int tid) {
    constexpr int r = ct_radix(N, S);
    if constexpr (r > 0) {
        constexpr bool hin = HIN && S == 0 && r % 2 == 0;
        constexpr bool hout = HOUT && ct_radix(N, S + 1) == 0 && r % 2 == 0;
        ct_pass<R, FWD, N, r, NS, NTHR, MAXROWS, hin, hout, RP>(buf, twl, rows, pitch, tid);
        ct_passes<R, FWD, N, S + 1, NS * r, NTHR, MAXROWS, false, HOUT, RP>(buf, twl, rows, pitch, tid);
    }
}

// exact floor(e / d) for e * d < 2^32 with magic = ceil(2^32 / d)
__host__ __device__ __forceinline__ unsigned magic_for(unsigned d) {
    return (unsigned)((0x100000000ULL + d - 1) / d);
}
__device__ __forceinline__ int fast_div(unsigned e, unsigned magic) { return (int)__umulhi(e, magic); }

}  // namespace vie
