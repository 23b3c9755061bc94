// Mixed-radix (2, 3, 4, 5, 8, 16) Stockham FFT on pencils staged in LDS.
//
// A pencil of length n is transformed by a sequence of radix-r passes; pass
// s with span Ns (product of the radices before it) computes, for every
// butterfly j in [0, n/r):
//     k = j mod Ns,  v_i = X[j + i n/r] * W_n^{i k n/(Ns r)},  v = DFT_r(v),
//     Y[(j / Ns) Ns r + k + i Ns] = v_i
// which leaves the result in natural order after the last pass (Stockham
// autosort).  X and Y are two LDS buffers (ping-pong).  Twiddles come from a
// table W[m] = exp(-2 pi i m / n), m < n, built on the host in FP64.
#pragma once

#include "common.hpp"

namespace vie {

constexpr int kMaxPasses = 8;

struct FftPlan {
    int n;
    int npass;
    int radix[kMaxPasses];
};

// ---------------------------------------------------------------------------
// register DFTs, forward (exp(-2 pi i ...)) or inverse (exp(+...), unscaled)
// ---------------------------------------------------------------------------
template <typename R, bool FWD>
__device__ __forceinline__ void dft2(C<R>& a, C<R>& b) {
    C<R> t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <typename R, bool FWD>
__device__ __forceinline__ void dft4(C<R>& a0, C<R>& a1, C<R>& a2, C<R>& a3) {
    C<R> s02 = cadd(a0, a2), d02 = csub(a0, a2);
    C<R> s13 = cadd(a1, a3), d13 = mul_mi<FWD>(csub(a1, a3));
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    a1 = cadd(d02, d13);
    a3 = csub(d02, d13);
}

template <typename R, bool FWD>
__device__ __forceinline__ void dft3(C<R>* v) {
    const R c = R(-0.5);
    const R s = R(0.86602540378443864676);  // sin(2 pi / 3)
    C<R> t1 = cadd(v[1], v[2]);
    C<R> t2 = cadd(v[0], cscale(t1, c));
    C<R> d = cscale(csub(v[1], v[2]), s);
    C<R> t3 = mul_mi<FWD>(d);  // forward: -i s (v1 - v2)
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
}

template <typename R, bool FWD>
__device__ __forceinline__ void dft5(C<R>* v) {
    const R c1 = R(0.30901699437494742410);   // cos(2 pi/5)
    const R c2 = R(-0.80901699437494742410);  // cos(4 pi/5)
    const R s1 = R(0.95105651629515357212);   // sin(2 pi/5)
    const R s2 = R(0.58778525229247312917);   // sin(4 pi/5)
    C<R> b1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
    C<R> b2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
    C<R> a = v[0];
    C<R> r1 = cadd(a, cadd(cscale(b1, c1), cscale(b2, c2)));
    C<R> r2 = cadd(a, cadd(cscale(b1, c2), cscale(b2, c1)));
    C<R> i1 = mul_mi<FWD>(cadd(cscale(d1, s1), cscale(d2, s2)));
    C<R> i2 = mul_mi<FWD>(csub(cscale(d1, s2), cscale(d2, s1)));
    v[0] = cadd(a, cadd(b1, b2));
    v[1] = cadd(r1, i1);
    v[4] = csub(r1, i1);
    v[2] = cadd(r2, i2);
    v[3] = csub(r2, i2);
}

template <typename R, bool FWD>
__device__ __forceinline__ void dft8(C<R>* v) {
    // even / odd split, each a length-4 DFT, combined with W8^k
    C<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C<R> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<R, FWD>(e0, e1, e2, e3);
    dft4<R, FWD>(o0, o1, o2, o3);
    const R h = R(0.70710678118654752440);
    // W8^1 = (1 - i)/sqrt2 forward, (1 + i)/sqrt2 inverse; W8^2 = -i; W8^3
    C<R> w1o1 = FWD ? mk<R>(h * (o1.x + o1.y), h * (o1.y - o1.x)) : mk<R>(h * (o1.x - o1.y), h * (o1.y + o1.x));
    C<R> w2o2 = mul_mi<FWD>(o2);
    C<R> w3o3 = FWD ? mk<R>(h * (-o3.x + o3.y), h * (-o3.y - o3.x)) : mk<R>(h * (-o3.x - o3.y), h * (-o3.y + o3.x));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1o1);
    v[5] = csub(e1, w1o1);
    v[2] = cadd(e2, w2o2);
    v[6] = csub(e2, w2o2);
    v[3] = cadd(e3, w3o3);
    v[7] = csub(e3, w3o3);
}

template <typename R, bool FWD>
__device__ __forceinline__ void dft16(C<R>* v) {
    // 16 = 4 x 4: length-4 DFTs over m of a_{4m+q} for each q (in place, so
    // v[q + 4 k1] = Z_q[k1]), twiddles W16^{q k1}, length-4 DFTs over q for
    // each k1 (v[4 k1 + q] -> index k2), output index k1 + 4 k2.
#pragma unroll
    for (int q = 0; q < 4; ++q) dft4<R, FWD>(v[q], v[4 + q], v[8 + q], v[12 + q]);
    const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173);
    const R c2 = R(0.70710678118654752440);
    const R sg = FWD ? R(-1) : R(1);
    // exp(sg i 2 pi m / 16) for m = 0..9
    const C<R> w[10] = {mk<R>(1, 0),  mk<R>(c1, sg * s1),  mk<R>(c2, sg * c2),  mk<R>(s1, sg * c1),
                        mk<R>(0, sg), mk<R>(-s1, sg * c1), mk<R>(-c2, sg * c2), mk<R>(-c1, sg * s1),
                        mk<R>(-1, 0), mk<R>(-c1, -sg * s1)};
#pragma unroll
    for (int q = 1; q < 4; ++q)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) v[q + 4 * k1] = cmul(v[q + 4 * k1], w[q * k1]);
    // now DFT over q for each k1: the four values v[q + 4 k1], q = 0..3
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<R, FWD>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds output k1 + 4 k2: transpose the 4 x 4 index
    C<R> t;
    t = v[1]; v[1] = v[4]; v[4] = t;
    t = v[2]; v[2] = v[8]; v[8] = t;
    t = v[3]; v[3] = v[12]; v[12] = t;
    t = v[6]; v[6] = v[9]; v[9] = t;
    t = v[7]; v[7] = v[13]; v[13] = t;
    t = v[11]; v[11] = v[14]; v[14] = t;
}

template <typename R, bool FWD, int RAD>
__device__ __forceinline__ void dft_r(C<R>* v);

// Length-4 DFT of (a0, a1, 0, 0): the zero half of a zero-padded input is
// not added in.
template <typename R, bool FWD>
__device__ __forceinline__ void dft4z(C<R>& a0, C<R>& a1, C<R>& a2, C<R>& a3) {
    const C<R> d13 = mul_mi<FWD>(a1);
    const C<R> s = cadd(a0, a1), d = csub(a0, a1);
    a2 = d;
    a3 = csub(a0, d13);
    a1 = cadd(a0, d13);
    a0 = s;
}

// DFT of a length-RAD butterfly whose upper half of inputs is zero (the
// first forward pass over zero-padded data); same outputs as dft_r.
template <typename R, bool FWD, int RAD>
__device__ __forceinline__ void dft_r_halfin(C<R>* v) {
    if constexpr (RAD == 2) {
        v[1] = v[0];
    } else if constexpr (RAD == 4) {
        dft4z<R, FWD>(v[0], v[1], v[2], v[3]);
    } else if constexpr (RAD == 8) {
        C<R> e0 = v[0], e1 = v[2], e2, e3;
        C<R> o0 = v[1], o1 = v[3], o2, o3;
        dft4z<R, FWD>(e0, e1, e2, e3);
        dft4z<R, FWD>(o0, o1, o2, o3);
        const R h = R(0.70710678118654752440);
        C<R> w1o1 = FWD ? mk<R>(h * (o1.x + o1.y), h * (o1.y - o1.x)) : mk<R>(h * (o1.x - o1.y), h * (o1.y + o1.x));
        C<R> w2o2 = mul_mi<FWD>(o2);
        C<R> w3o3 = FWD ? mk<R>(h * (-o3.x + o3.y), h * (-o3.y - o3.x)) : mk<R>(h * (-o3.x - o3.y), h * (-o3.y + o3.x));
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, w1o1);
        v[5] = csub(e1, w1o1);
        v[2] = cadd(e2, w2o2);
        v[6] = csub(e2, w2o2);
        v[3] = cadd(e3, w3o3);
        v[7] = csub(e3, w3o3);
    } else if constexpr (RAD == 16) {
        // as dft16, whose first stage combines v[q], v[4+q], v[8+q], v[12+q]:
        // the last two are zero
#pragma unroll
        for (int q = 0; q < 4; ++q) dft4z<R, FWD>(v[q], v[4 + q], v[8 + q], v[12 + q]);
        const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173);
        const R c2 = R(0.70710678118654752440);
        const R sg = FWD ? R(-1) : R(1);
        const C<R> w[10] = {mk<R>(1, 0),  mk<R>(c1, sg * s1),  mk<R>(c2, sg * c2),  mk<R>(s1, sg * c1),
                            mk<R>(0, sg), mk<R>(-s1, sg * c1), mk<R>(-c2, sg * c2), mk<R>(-c1, sg * s1),
                            mk<R>(-1, 0), mk<R>(-c1, -sg * s1)};
#pragma unroll
        for (int q = 1; q < 4; ++q)
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) v[q + 4 * k1] = cmul(v[q + 4 * k1], w[q * k1]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) dft4<R, FWD>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
        C<R> t;
        t = v[1]; v[1] = v[4]; v[4] = t;
        t = v[2]; v[2] = v[8]; v[8] = t;
        t = v[3]; v[3] = v[12]; v[12] = t;
        t = v[6]; v[6] = v[9]; v[9] = t;
        t = v[7]; v[7] = v[13]; v[13] = t;
        t = v[11]; v[11] = v[14]; v[14] = t;
    } else {
        dft_r<R, FWD, RAD>(v);   // odd radices: no zero half
    }
}

template <typename R, bool FWD, int RAD>
__device__ __forceinline__ void dft_r(C<R>* v) {
    if constexpr (RAD == 2) dft2<R, FWD>(v[0], v[1]);
    else if constexpr (RAD == 3) dft3<R, FWD>(v);
    else if constexpr (RAD == 4) dft4<R, FWD>(v[0], v[1], v[2], v[3]);
    else if constexpr (RAD == 5) dft5<R, FWD>(v);
    else if constexpr (RAD == 8) dft8<R, FWD>(v);
    else dft16<R, FWD>(v);
}

// ---------------------------------------------------------------------------
// one Stockham pass over npen pencils in LDS.
// element k of pencil t lives at t * pstride + k * estride.
// JFAST: consecutive threads take consecutive butterflies of one pencil
// (pencils stored contiguously); otherwise consecutive pencils (tile of
// strided pencils stored [k][t]).
// ---------------------------------------------------------------------------
template <typename R, bool FWD, int RAD, bool JFAST>
__device__ __forceinline__ void stockham_pass(const C<R>* __restrict__ X, C<R>* __restrict__ Y, int n, int Ns,
                                              int npen, int pstride, int estride,
                                              const C<R>* __restrict__ tw, int tid, int nthr) {
    const int nb = n / RAD;
    const int total = nb * npen;
    const int twstep = n / (Ns * RAD);
    for (int idx = tid; idx < total; idx += nthr) {
        int t, j;
        if (JFAST) { t = idx / nb; j = idx - t * nb; }
        else { j = idx / npen; t = idx - j * npen; }
        const int k = j % Ns;
        const C<R>* src = X + t * pstride;
        C<R> v[RAD];
#pragma unroll
        for (int i = 0; i < RAD; ++i) v[i] = src[(j + i * nb) * estride];
        if (Ns > 1) {
#pragma unroll
            for (int i = 1; i < RAD; ++i) {
                C<R> w = tw[i * k * twstep];
                if (!FWD) w.y = -w.y;
                v[i] = cmul(v[i], w);
            }
        }
        dft_r<R, FWD, RAD>(v);
        C<R>* dst = Y + t * pstride;
        const int base = (j - k) * RAD + k;
#pragma unroll
        for (int i = 0; i < RAD; ++i) dst[(base + i * Ns) * estride] = v[i];
    }
}

// Full transform; data starts in buf0 and ends in the returned buffer.
template <typename R, bool FWD, bool JFAST>
__device__ C<R>* fft_lds(C<R>* buf0, C<R>* buf1, const FftPlan& plan, int npen, int pstride, int estride,
                         const C<R>* __restrict__ tw, int tid, int nthr) {
    C<R>* X = buf0;
    C<R>* Y = buf1;
    int Ns = 1;
    for (int s = 0; s < plan.npass; ++s) {
        const int r = plan.radix[s];
        switch (r) {
            case 2: stockham_pass<R, FWD, 2, JFAST>(X, Y, plan.n, Ns, npen, pstride, estride, tw, tid, nthr); break;
            case 3: stockham_pass<R, FWD, 3, JFAST>(X, Y, plan.n, Ns, npen, pstride, estride, tw, tid, nthr); break;
            case 4: stockham_pass<R, FWD, 4, JFAST>(X, Y, plan.n, Ns, npen, pstride, estride, tw, tid, nthr); break;
            case 5: stockham_pass<R, FWD, 5, JFAST>(X, Y, plan.n, Ns, npen, pstride, estride, tw, tid, nthr); break;
            case 8: stockham_pass<R, FWD, 8, JFAST>(X, Y, plan.n, Ns, npen, pstride, estride, tw, tid, nthr); break;
            default: stockham_pass<R, FWD, 16, JFAST>(X, Y, plan.n, Ns, npen, pstride, estride, tw, tid, nthr); break;
        }
        __syncthreads();
        Ns *= r;
        C<R>* t = X;
        X = Y;
        Y = t;
    }
    return X;
}

// ---------------------------------------------------------------------------
// in-place variant for rows stored contiguously (row r, element k at
// lds_pad(r * pitch + k)): every thread holds at most one butterfly per pass
// (the caller guarantees rows * n / radix <= nthr for every radix of the
// plan), loads its inputs, the block synchronises, then it writes.  LDS
// addresses are padded by one element every 16 to spread the strided
// accesses of the early passes over the banks.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int lds_pad(int a) { return a + (a >> 4); }

template <typename R, bool FWD, int RAD, int NB>
__device__ __noinline__ void stockham_rows_inplace(C<R>* buf, int n, int Ns, int nrows, int pitch,
                                                      const C<R>* __restrict__ tw, int tid, int nthr) {
    const int nb = n / RAD;
    const int total = nb * nrows;
    C<R> v[NB][RAD];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int idx = tid + q * nthr;
        if (idx < total) {
            const int t = idx / nb, j = idx - t * nb;
            const int rb = t * pitch;
#pragma unroll
            for (int i = 0; i < RAD; ++i) v[q][i] = buf[lds_pad(rb + j + i * nb)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int idx = tid + q * nthr;
        if (idx < total) {
            const int t = idx / nb, j = idx - t * nb;
            const int k = j % Ns;
            if (Ns > 1) {
                const int twstep = n / (Ns * RAD);
#pragma unroll
                for (int i = 1; i < RAD; ++i) {
                    C<R> w = tw[i * k * twstep];
                    if (!FWD) w.y = -w.y;
                    v[q][i] = cmul(v[q][i], w);
                }
            }
            dft_r<R, FWD, RAD>(v[q]);
            const int rb = t * pitch + (j - k) * RAD + k;
#pragma unroll
            for (int i = 0; i < RAD; ++i) buf[lds_pad(rb + i * Ns)] = v[q][i];
        }
    }
    __syncthreads();
}

// butterflies a thread may hold per pass: at most 16 complex registers
__host__ __device__ constexpr int rows_max_nb(int rad) { return rad >= 16 ? 1 : rad >= 8 ? 2 : rad >= 4 ? 4 : rad == 3 ? 4 : 8; }

template <typename R, bool FWD, int RAD>
__device__ __forceinline__ void stockham_rows_dispatch(C<R>* buf, int n, int Ns, int nrows, int pitch,
                                                       const C<R>* __restrict__ tw, int tid, int nthr) {
    const int total = (n / RAD) * nrows;
    constexpr int mx = rows_max_nb(RAD);
    if (total <= nthr) stockham_rows_inplace<R, FWD, RAD, 1>(buf, n, Ns, nrows, pitch, tw, tid, nthr);
    else if constexpr (mx >= 2) {
        if (mx == 2 || total <= 2 * nthr) stockham_rows_inplace<R, FWD, RAD, 2>(buf, n, Ns, nrows, pitch, tw, tid, nthr);
        else if constexpr (mx >= 4) {
            if (mx == 4 || total <= 4 * nthr)
                stockham_rows_inplace<R, FWD, RAD, 4>(buf, n, Ns, nrows, pitch, tw, tid, nthr);
            else stockham_rows_inplace<R, FWD, RAD, 8>(buf, n, Ns, nrows, pitch, tw, tid, nthr);
        }
    }
}

// rows * n / radix <= rows_max_nb(radix) * nthr for every radix of the plan
__host__ __device__ inline bool rows_fit(const FftPlan& plan, int nrows, int nthr) {
    for (int s = 0; s < plan.npass; ++s) {
        const int r = plan.radix[s];
        if ((long long)nrows * (plan.n / r) > (long long)rows_max_nb(r) * nthr) return false;
    }
    return true;
}

// whole transform of nrows rows in place (requires rows_fit)
template <typename R, bool FWD>
__device__ void fft_rows_inplace(C<R>* buf, const FftPlan& plan, int nrows, int pitch, const C<R>* __restrict__ tw,
                                 int tid, int nthr) {
    int Ns = 1;
    for (int s = 0; s < plan.npass; ++s) {
        const int r = plan.radix[s];
        switch (r) {
            case 2: stockham_rows_dispatch<R, FWD, 2>(buf, plan.n, Ns, nrows, pitch, tw, tid, nthr); break;
            case 3: stockham_rows_dispatch<R, FWD, 3>(buf, plan.n, Ns, nrows, pitch, tw, tid, nthr); break;
            case 4: stockham_rows_dispatch<R, FWD, 4>(buf, plan.n, Ns, nrows, pitch, tw, tid, nthr); break;
            case 5: stockham_rows_dispatch<R, FWD, 5>(buf, plan.n, Ns, nrows, pitch, tw, tid, nthr); break;
            case 8: stockham_rows_dispatch<R, FWD, 8>(buf, plan.n, Ns, nrows, pitch, tw, tid, nthr); break;
            default: stockham_rows_dispatch<R, FWD, 16>(buf, plan.n, Ns, nrows, pitch, tw, tid, nthr); break;
        }
        Ns *= r;
    }
}

}  // namespace vie
