// Arnoldi / GMRES vector kernels (Sec. V: restarted GMRES).  Inner products
// and norms accumulate in FP64 whatever the storage precision; reductions run
// in a fixed order (per-thread, wave, workgroup, then a separate pass over
// workgroups), so results are bitwise reproducible.
#include "kernels.hpp"
#include "vie.h"

namespace vie {

constexpr int kTpb = 256;

// Basis vectors are streamed once per Gram-Schmidt pass and a whole basis is
// larger than the caches, so their loads are non-temporal (stream_load).
// The small kernels that sum per-workgroup partials walk them lane-strided
// with the loop unrolled, so that a lane's loads are in flight together (the
// additions keep their order, so the sums keep their bits).
constexpr int kGroup = 8;   // basis vectors per workgroup of the dot kernel

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T> __device__ __forceinline__ double2 to_d2(T v) { return make_double2((double)v.x, (double)v.y); }

// Load units of the Gram-Schmidt kernels: 16 bytes (a pair of complex64, or
// one complex128) when every vector start is 16-byte aligned, i.e. the
// vector length and all strides are even in complex64; a single complex64
// otherwise (odd lengths occur with the PWC basis, 3 V unknowns).
template <typename R, bool PAIR> struct Unit;
template <> struct Unit<float, true> {
    using T = float4;
    static constexpr int per = 2;
    __device__ static double2 get(const T& u, int h) { return h ? make_double2(u.z, u.w) : make_double2(u.x, u.y); }
    __device__ static void set(T& u, int h, double2 v) {
        if (h) { u.z = (float)v.x; u.w = (float)v.y; } else { u.x = (float)v.x; u.y = (float)v.y; }
    }
};
template <> struct Unit<float, false> {
    using T = float2;
    static constexpr int per = 1;
    __device__ static double2 get(const T& u, int) { return make_double2(u.x, u.y); }
    __device__ static void set(T& u, int, double2 v) { u.x = (float)v.x; u.y = (float)v.y; }
};
template <bool PAIR> struct Unit<double, PAIR> {
    using T = double2;
    static constexpr int per = 1;
    __device__ static double2 get(const T& u, int) { return u; }
    __device__ static void set(T& u, int, double2 v) { u = v; }
};

// true when 16-byte units cover every vector exactly: complex128, or
// complex64 with an even length, even strides and 16-byte aligned bases
template <typename R>
static bool pair_units(const void* a, const void* b, long long n, long long s1, long long s2, long long s3) {
    if (sizeof(R) == 8) return true;
    return ((n | s1 | s2 | s3) & 1) == 0 && ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0;
}

// One group of G basis vectors (G compile-time, so that the G + NW loads of an
// element are issued together) against NW vectors w_q = wr + q ldwu: partial
// sums of conj(V_i) w_q over this thread's elements, reduced over the
// workgroup and written to partial[((q nrhs + r) nvec + i) nblocks + block].
template <typename R, bool PAIR, int G, int NW>
__device__ __forceinline__ void dot_group(double2* __restrict__ partial,
                                          const typename Unit<R, PAIR>::T* __restrict__ V,
                                          const typename Unit<R, PAIR>::T* __restrict__ wr, long long ldwu,
                                          long long ldu, long long nu, int i0, int nvec, int r,
                                          double (*red)[2 * 3 * kGroup]) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long stride = (long long)gridDim.x * kTpb;
    double ar[NW][G], ai[NW][G];
#pragma unroll
    for (int q = 0; q < NW; ++q)
#pragma unroll
        for (int g = 0; g < G; ++g) ar[q][g] = ai[q][g] = 0.0;
    for (long long k = blockIdx.x * (long long)kTpb + threadIdx.x; k < nu; k += stride) {
        T wu[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) wu[q] = wr[q * ldwu + k];
        T vu[G];
#pragma unroll
        for (int g = 0; g < G; ++g) vu[g] = stream_load(&V[(i0 + g) * ldu + k]);
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int h = 0; h < U::per; ++h) {
                const double2 v = U::get(vu[g], h);
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    const double2 wv = U::get(wu[q], h);
                    ar[q][g] += v.x * wv.x + v.y * wv.y;
                    ai[q][g] += v.x * wv.y - v.y * wv.x;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NW; ++q)
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double sr = wave_sum(ar[q][g]), si = wave_sum(ai[q][g]);
            if (lane == 0) { red[wave][2 * (q * G + g)] = sr; red[wave][2 * (q * G + g) + 1] = si; }
        }
    __syncthreads();
    if (threadIdx.x < NW * G) {
        const int q = threadIdx.x / G, g = threadIdx.x - q * G;
        double sr = 0, si = 0;
        for (int wv = 0; wv < kTpb / 64; ++wv) { sr += red[wv][2 * threadIdx.x]; si += red[wv][2 * threadIdx.x + 1]; }
        partial[(((long long)q * gridDim.y + r) * nvec + i0 + g) * gridDim.x + blockIdx.x] = make_double2(sr, si);
    }
    __syncthreads();
}

// partial sums of conj(V_i) w_q for i < nvec and the NW vectors w_q = w + q
// ldw: workgroup (b, r, g) takes group g of kGroup basis vectors (the last
// group may hold fewer) over its share of the elements, so the groups stream
// side by side (vectors read in units of Unit<R, PAIR>; n and the strides
// multiples of the unit)
template <typename R, bool PAIR, int NW>
__global__ void __launch_bounds__(kTpb) k_multidot(double2* __restrict__ partial, const C<R>* __restrict__ Vb,
                                                   long long ldv, int nvec, const C<R>* __restrict__ w,
                                                   long long ldw, long long n, long long rsv, long long rsw) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    __shared__ double red[kTpb / 64][2 * 3 * kGroup];
    const int r = blockIdx.y;
    const T* V = reinterpret_cast<const T*>(Vb + r * rsv);
    const T* wr = reinterpret_cast<const T*>(w + r * rsw);
    const long long nu = n / U::per, ldu = ldv / U::per, ldwu = ldw / U::per;
    static_assert(kGroup == 8, "the group sizes below cover 1 to 8");
    const int i0 = blockIdx.z * kGroup;
    switch (min(kGroup, nvec - i0)) {   // uniform over the workgroup
#define VIE_DOT_G(g_) \
    case g_: dot_group<R, PAIR, g_, NW>(partial, V, wr, ldwu, ldu, nu, i0, nvec, r, red); break;
        VIE_DOT_G(1) VIE_DOT_G(2) VIE_DOT_G(3) VIE_DOT_G(4) VIE_DOT_G(5) VIE_DOT_G(6) VIE_DOT_G(7) VIE_DOT_G(8)
#undef VIE_DOT_G
        default: break;
    }
}

template <typename R, int NW>
static void multidot_nw(double2* partial, const C<R>* Vb, long long ldv, int nvec, const C<R>* w, long long ldw,
                        long long n, long long rsv, long long rsw, int nrhs, int nblocks, hipStream_t s) {
    const unsigned ngroups = (unsigned)((nvec + kGroup - 1) / kGroup);
    if (pair_units<R>(Vb, w, n, ldv, rsv, rsw) && (ldw & 1) == 0)
        hipLaunchKernelGGL((k_multidot<R, true, NW>), dim3(nblocks, nrhs, ngroups), dim3(kTpb), 0, s, partial, Vb,
                           ldv, nvec, w, ldw, n, rsv, rsw);
    else
        hipLaunchKernelGGL((k_multidot<R, false, NW>), dim3(nblocks, nrhs, ngroups), dim3(kTpb), 0, s, partial, Vb,
                           ldv, nvec, w, ldw, n, rsv, rsw);
    VIE_HIP(hipGetLastError());
}

template <typename R>
void launch_multidot(double2* partial, const C<R>* Vb, long long ldv, int nvec, const C<R>* w, long long n,
                     long long rsv, long long rsw, int nrhs, int nblocks, hipStream_t s) {
    multidot_nw<R, 1>(partial, Vb, ldv, nvec, w, 0, n, rsv, rsw, nrhs, nblocks, s);
}

template <typename R>
void launch_multidot2(double2* partial, const C<R>* Vb, long long ldv, int nvec, const C<R>* w, long long ldw,
                      long long n, long long rsv, long long rsw, int nrhs, int nblocks, hipStream_t s) {
    multidot_nw<R, 2>(partial, Vb, ldv, nvec, w, ldw, n, rsv, rsw, nrhs, nblocks, s);
}

template <typename R>
void launch_multidot3(double2* partial, const C<R>* Vb, long long ldv, int nvec, const C<R>* w, long long ldw,
                      long long n, long long rsv, long long rsw, int nrhs, int nblocks, hipStream_t s) {
    multidot_nw<R, 3>(partial, Vb, ldv, nvec, w, ldw, n, rsv, rsw, nrhs, nblocks, s);
}

// The basis is stored unnormalised: slot i holds u_i with v_i = u_i * ivn[i]
// (ivn = 1 / ||u_i||, 0 for a zero vector).  From the partial sums of
// conj(u_i) w this forms the Hessenberg entries h_i = conj(v_i) (sw w), with
// sw = ivn[jw] (w = the operator applied to u_jw; jw < 0: sw = 1), and the
// update coefficients c_i = h_i ivn[i], so that sw w - sum_i h_i v_i =
// sw w - sum_i c_i u_i.
__global__ void k_reduce_partials(double2* __restrict__ h, double2* __restrict__ coef,
                                  const double2* __restrict__ partial, int nblocks, int nvec,
                                  const double* __restrict__ ivn, long long ivn_ld, int jw) {
    const long long row = blockIdx.x;
    const int r = (int)(row / nvec), i = (int)(row % nvec);
    const double2* p = partial + row * nblocks;
    double sr = 0, si = 0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nblocks; b += 64) { sr += p[b].x; si += p[b].y; }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (threadIdx.x == 0) {
        const double sw = jw >= 0 ? ivn[r * ivn_ld + jw] : 1.0;
        const double iv = ivn[r * ivn_ld + i];
        const double2 hv = make_double2(sr * sw * iv, si * sw * iv);
        h[row] = hv;
        coef[row] = make_double2(hv.x * iv, hv.y * iv);
    }
}

void launch_reduce_partials(double2* h, double2* coef, const double2* partial, int nvec, int nblocks, int nrhs,
                            const double* ivn, long long ivn_ld, int jw, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(nvec * nrhs), dim3(64), 0, s, h, coef, partial, nblocks, nvec, ivn,
                       ivn_ld, jw);
    VIE_HIP(hipGetLastError());
}

// w = sw w - sum_i c_i u_i (FP64 arithmetic; sw = ivn[jw], or 1 for jw < 0),
// and partial sums of |w|^2 of the stored values
template <typename R, bool PAIR>
__global__ void __launch_bounds__(kTpb) k_update(C<R>* __restrict__ w, const C<R>* __restrict__ Vb, long long ldv,
                                                 int nvec, const double2* __restrict__ h, long long n, long long rsv,
                                                 long long rsw, double* __restrict__ norm_partial,
                                                 const double* __restrict__ ivn, long long ivn_ld, int jw) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    __shared__ double red[kTpb / 64];
    const int r = blockIdx.y;
    const T* V = reinterpret_cast<const T*>(Vb + r * rsv);
    T* wr = reinterpret_cast<T*>(w + r * rsw);
    const long long nu = n / U::per, ldu = ldv / U::per;
    const double2* hr = h + (long long)r * nvec;
    const double sw = jw >= 0 ? ivn[r * ivn_ld + jw] : 1.0;
    double acc = 0.0;
    for (long long k = blockIdx.x * (long long)kTpb + threadIdx.x; k < nu; k += (long long)gridDim.x * kTpb) {
        T wu = wr[k];
        double2 wv[U::per];
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            wv[q] = U::get(wu, q);
            wv[q].x *= sw;
            wv[q].y *= sw;
        }
        // the basis vectors in blocks of 8 (their loads issued together),
        // then one at a time
        int i = 0;
        for (; i + 8 <= nvec; i += 8) {
            T vu[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) vu[u] = stream_load(&V[(i + u) * ldu + k]);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double2 hi = hr[i + u];
#pragma unroll
                for (int q = 0; q < U::per; ++q) {
                    const double2 v = U::get(vu[u], q);
                    wv[q].x -= hi.x * v.x - hi.y * v.y;
                    wv[q].y -= hi.x * v.y + hi.y * v.x;
                }
            }
        }
        for (; i < nvec; ++i) {
            const T vu = stream_load(&V[i * ldu + k]);
            const double2 hi = hr[i];
#pragma unroll
            for (int q = 0; q < U::per; ++q) {
                const double2 v = U::get(vu, q);
                wv[q].x -= hi.x * v.x - hi.y * v.y;
                wv[q].y -= hi.x * v.y + hi.y * v.x;
            }
        }
#pragma unroll
        for (int q = 0; q < U::per; ++q) U::set(wu, q, wv[q]);
        wr[k] = wu;
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            const double2 o = U::get(wu, q);   // the stored (rounded) value
            acc += o.x * o.x + o.y * o.y;
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < kTpb / 64; ++i) s += red[i];
        norm_partial[(long long)r * gridDim.x + blockIdx.x] = s;
    }
}

template <typename R>
void launch_update(C<R>* w, const C<R>* Vb, long long ldv, int nvec, const double2* h, long long n, long long rsv,
                   long long rsw, double* norm_partial, const double* ivn, long long ivn_ld, int jw, int nrhs,
                   int nblocks, hipStream_t s) {
    if (pair_units<R>(Vb, w, n, ldv, rsv, rsw))
        hipLaunchKernelGGL((k_update<R, true>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, w, Vb, ldv, nvec, h, n, rsv,
                           rsw, norm_partial, ivn, ivn_ld, jw);
    else
        hipLaunchKernelGGL((k_update<R, false>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, w, Vb, ldv, nvec, h, n, rsv,
                           rsw, norm_partial, ivn, ivn_ld, jw);
    VIE_HIP(hipGetLastError());
}

// ---- two Arnoldi steps per pass over the basis (s-step Arnoldi, s = 2) ----
//
// For the pair of steps (j, j + 1): w1 = A v_j and w2 = (A - sigma) w1 with
// sigma = h_jj = v_j^H A v_j, the Rayleigh quotient of v_j, which keeps w2
// from leaning on w1.  One dot pass gives h = V^H w1 and g = V^H w2, one
// update pass w1 - V h and w2 - V g (V = v_0..v_j).  With beta1 = ||w1 -
// V h|| the next basis vector is v_{j+1} = (w1 - V h) / beta1, and w2 is
// then orthogonalised against it alone: with d = (w1 - V h)^H (w2 - V g),
// u_{j+2} = (w2 - V g - d / beta1^2 (w1 - V h)) / beta1, whose norm is the
// subdiagonal entry h_{j+2, j+1}.  Column j + 1 of the Hessenberg matrix
// follows from A v_{j+1} = (A w1 - A V h) / beta1 = (w2 + sigma w1 - V_{j+2}
// H h) / beta1 (the Arnoldi relation for A V h; H the unrotated columns 0..j):
//   h_{i, j+1} = (g_i + sigma h_i - (H h)_i) / beta1   (i <= j)
//   h_{j+1, j+1} = d / beta1^2                          (as sigma = h_j).
// Both products are applied to stored vectors as they are (w1 to the raw
// output of the first): the stored scale of u_j, sw = ivn[j], multiplies
// both, as in the one-step update.

// one wave per (row i, slot r): h_i = conj(v_i) (sw w1) from plane 0 of the
// dot partials, g_i = conj(v_i) (sw w2_raw) - sigma h_i from plane 1, with
// sigma = h_j summed again by every wave (the same order, so the same bits),
// and the update coefficients h_i ivn[i], g_i ivn[i]
__global__ void __launch_bounds__(64) k_reduce_pair(double2* __restrict__ h, double2* __restrict__ coef,
                                                    double2* __restrict__ gcol, double2* __restrict__ coef2,
                                                    const double2* __restrict__ partial, int nblocks, int nvec,
                                                    int na, const double* __restrict__ ivn, long long ivn_ld, int jw) {
    const int i = blockIdx.x, r = blockIdx.y, lane = threadIdx.x, j = nvec - 1;
    const double2* p1 = partial + ((long long)r * nvec + i) * nblocks;
    const double2* p2 = partial + (((long long)na + r) * nvec + i) * nblocks;
    const double2* pj = partial + ((long long)r * nvec + j) * nblocks;
    double a = 0, b = 0, c = 0, d = 0, e = 0, f = 0;
#pragma unroll 8
    for (int k = lane; k < nblocks; k += 64) {
        a += p1[k].x;
        b += p1[k].y;
        c += p2[k].x;
        d += p2[k].y;
        e += pj[k].x;
        f += pj[k].y;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    d = wave_sum(d);
    e = wave_sum(e);
    f = wave_sum(f);
    if (lane == 0) {
        const double sw = ivn[r * ivn_ld + jw], iv = ivn[r * ivn_ld + i], ivj = ivn[r * ivn_ld + j];
        const double2 sigma = make_double2(e * sw * ivj, f * sw * ivj);
        const double2 hv = make_double2(a * sw * iv, b * sw * iv);
        const double2 gv = csub(make_double2(c * sw * iv, d * sw * iv), cmul(sigma, hv));
        h[(long long)r * nvec + i] = hv;
        coef[(long long)r * nvec + i] = make_double2(hv.x * iv, hv.y * iv);
        gcol[(long long)r * nvec + i] = gv;
        coef2[(long long)r * nvec + i] = make_double2(gv.x * iv, gv.y * iv);
    }
}

void launch_reduce_pair(double2* h, double2* coef, double2* gcol, double2* coef2, const double2* partial, int nvec,
                        int nblocks, int nrhs, const double* ivn, long long ivn_ld, int jw, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_pair, dim3(nvec, nrhs), dim3(64), 0, s, h, coef, gcol, coef2, partial, nblocks, nvec,
                       nrhs, ivn, ivn_ld, jw);
    VIE_HIP(hipGetLastError());
}

// w1 <- sw w1 - sum_i c_i u_i and w2 <- sw (w2 - sigma w1) - sum_i c2_i u_i
// (w2 = w1 + ldv, w1 the value before its update; sigma = h[r nvec + nvec -
// 1]), with partial sums of |w1|^2 and of conj(w1) w2 over the stored values
template <typename R, bool PAIR>
__global__ void __launch_bounds__(kTpb) k_update_pair(C<R>* __restrict__ w, const C<R>* __restrict__ Vb,
                                                      long long ldv, int nvec, const double2* __restrict__ coef,
                                                      const double2* __restrict__ coef2,
                                                      const double2* __restrict__ hcol, long long n, long long rsv,
                                                      long long rsw, double* __restrict__ norm_partial,
                                                      double2* __restrict__ dot_partial,
                                                      const double* __restrict__ ivn, long long ivn_ld, int jw) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    __shared__ double red[kTpb / 64][3];
    const int r = blockIdx.y;
    const T* V = reinterpret_cast<const T*>(Vb + r * rsv);
    T* w1p = reinterpret_cast<T*>(w + r * rsw);
    T* w2p = reinterpret_cast<T*>(w + r * rsw + ldv);
    const long long nu = n / U::per, ldu = ldv / U::per;
    const double2* c1 = coef + (long long)r * nvec;
    const double2* c2 = coef2 + (long long)r * nvec;
    const double2 sigma = hcol[(long long)r * nvec + nvec - 1];
    const double sw = ivn[r * ivn_ld + jw];
    double nacc = 0.0, dre = 0.0, dim_ = 0.0;
    for (long long k = blockIdx.x * (long long)kTpb + threadIdx.x; k < nu; k += (long long)gridDim.x * kTpb) {
        T a1 = w1p[k], a2 = w2p[k];
        double2 x1[U::per], x2[U::per];
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            const double2 o1 = U::get(a1, q), o2 = U::get(a2, q);
            const double2 t = csub(o2, cmul(sigma, o1));
            x1[q] = make_double2(sw * o1.x, sw * o1.y);
            x2[q] = make_double2(sw * t.x, sw * t.y);
        }
        int i = 0;
        for (; i + 8 <= nvec; i += 8) {
            T vu[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) vu[u] = stream_load(&V[(i + u) * ldu + k]);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double2 p = c1[i + u], q2 = c2[i + u];
#pragma unroll
                for (int q = 0; q < U::per; ++q) {
                    const double2 v = U::get(vu[u], q);
                    x1[q].x -= p.x * v.x - p.y * v.y;
                    x1[q].y -= p.x * v.y + p.y * v.x;
                    x2[q].x -= q2.x * v.x - q2.y * v.y;
                    x2[q].y -= q2.x * v.y + q2.y * v.x;
                }
            }
        }
        for (; i < nvec; ++i) {
            const T vu = stream_load(&V[i * ldu + k]);
            const double2 p = c1[i], q2 = c2[i];
#pragma unroll
            for (int q = 0; q < U::per; ++q) {
                const double2 v = U::get(vu, q);
                x1[q].x -= p.x * v.x - p.y * v.y;
                x1[q].y -= p.x * v.y + p.y * v.x;
                x2[q].x -= q2.x * v.x - q2.y * v.y;
                x2[q].y -= q2.x * v.y + q2.y * v.x;
            }
        }
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            U::set(a1, q, x1[q]);
            U::set(a2, q, x2[q]);
        }
        w1p[k] = a1;
        w2p[k] = a2;
#pragma unroll
        for (int q = 0; q < U::per; ++q) {   // the stored (rounded) values
            const double2 o1 = U::get(a1, q), o2 = U::get(a2, q);
            nacc += o1.x * o1.x + o1.y * o1.y;
            dre += o1.x * o2.x + o1.y * o2.y;
            dim_ += o1.x * o2.y - o1.y * o2.x;
        }
    }
    nacc = wave_sum(nacc);
    dre = wave_sum(dre);
    dim_ = wave_sum(dim_);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = nacc;
        red[threadIdx.x >> 6][1] = dre;
        red[threadIdx.x >> 6][2] = dim_;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0, c = 0;
        for (int i = 0; i < kTpb / 64; ++i) { a += red[i][0]; b += red[i][1]; c += red[i][2]; }
        norm_partial[(long long)r * gridDim.x + blockIdx.x] = a;
        dot_partial[(long long)r * gridDim.x + blockIdx.x] = make_double2(b, c);
    }
}

template <typename R>
void launch_update_pair(C<R>* w, const C<R>* Vb, long long ldv, int nvec, const double2* coef, const double2* coef2,
                        const double2* h, long long n, long long rsv, long long rsw, double* norm_partial,
                        double2* dot_partial, const double* ivn, long long ivn_ld, int jw, int nrhs, int nblocks,
                        hipStream_t s) {
    if (pair_units<R>(Vb, w, n, ldv, rsv, rsw))
        hipLaunchKernelGGL((k_update_pair<R, true>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, w, Vb, ldv, nvec, coef,
                           coef2, h, n, rsv, rsw, norm_partial, dot_partial, ivn, ivn_ld, jw);
    else
        hipLaunchKernelGGL((k_update_pair<R, false>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, w, Vb, ldv, nvec, coef,
                           coef2, h, n, rsv, rsw, norm_partial, dot_partial, ivn, ivn_ld, jw);
    VIE_HIP(hipGetLastError());
}

// per slot: d = sum of the conj(w1) w2 partials (lane-strided, the order of
// the norm sums), beta1 = nrm[s] (from the Givens step of column j), and
// pc[s] = (d / beta1^2, 1 / beta1), both 0 for beta1 = 0
__global__ void __launch_bounds__(64) k_pair_coef(double2* __restrict__ pc, const double2* __restrict__ dpart,
                                                  int nblocks, const double* __restrict__ nrm) {
    const int r = blockIdx.x, lane = threadIdx.x;
    double sr = 0, si = 0;
#pragma unroll 8
    for (int b = lane; b < nblocks; b += 64) {
        sr += dpart[(long long)r * nblocks + b].x;
        si += dpart[(long long)r * nblocks + b].y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
        const double b1 = nrm[r];
        const double ib = b1 > 0 ? 1.0 / b1 : 0.0;
        pc[2 * r] = make_double2(sr * ib * ib, si * ib * ib);
        pc[2 * r + 1] = make_double2(ib, b1);
    }
}

void launch_pair_coef(double2* pc, const double2* dpart, int nblocks, const double* nrm, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_coef, dim3(nrhs), dim3(64), 0, s, pc, dpart, nblocks, nrm);
    VIE_HIP(hipGetLastError());
}

// u2 <- (u2 - gamma u1) / beta1 in place (u2 = u1 + ldv; gamma, 1 / beta1
// from pc), with partial sums of |u2|^2 over the stored values
template <typename R, bool PAIR>
__global__ void __launch_bounds__(kTpb) k_axpy_pair(C<R>* __restrict__ u1, long long ldv, long long n,
                                                    long long rs, const double2* __restrict__ pc,
                                                    double* __restrict__ norm_partial) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    __shared__ double red[kTpb / 64];
    const int r = blockIdx.y;
    const T* a = reinterpret_cast<const T*>(u1 + r * rs);
    T* b = reinterpret_cast<T*>(u1 + r * rs + ldv);
    const long long nu = n / U::per;
    const double2 gm = pc[2 * r];
    const double ib = pc[2 * r + 1].x;
    double acc = 0.0;
    for (long long k = blockIdx.x * (long long)kTpb + threadIdx.x; k < nu; k += (long long)gridDim.x * kTpb) {
        const T au = a[k];
        T bu = b[k];
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            const double2 t = csub(U::get(bu, q), cmul(gm, U::get(au, q)));
            U::set(bu, q, make_double2(t.x * ib, t.y * ib));
        }
        b[k] = bu;
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            const double2 o = U::get(bu, q);
            acc += o.x * o.x + o.y * o.y;
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < kTpb / 64; ++i) t += red[i];
        norm_partial[(long long)r * gridDim.x + blockIdx.x] = t;
    }
}

template <typename R>
void launch_axpy_pair(C<R>* u1, long long ldv, long long n, long long rs, const double2* pc, double* norm_partial,
                      int nrhs, int nblocks, hipStream_t s) {
    if (pair_units<R>(u1, u1, n, ldv, rs, rs))
        hipLaunchKernelGGL((k_axpy_pair<R, true>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, u1, ldv, n, rs, pc,
                           norm_partial);
    else
        hipLaunchKernelGGL((k_axpy_pair<R, false>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, u1, ldv, n, rs, pc,
                           norm_partial);
    VIE_HIP(hipGetLastError());
}

// Hessenberg column j + 1 of a pair (entries 0..j + 1, the subdiagonal comes
// from the norm of u_{j+2}) from h (column j above the diagonal), g, sigma =
// h_j, pc and the unrotated columns 0..j (st.Hr).  One workgroup of 4 waves
// per slot: lane l takes rows l, l + 64, ..., wave w the columns k = w, w +
// 4, ... of (H h)_i = sum_k H[i, k] h_k (H[i, k] = 0 for k < i - 1), summed
// over the waves in LDS in a fixed order.
constexpr int kColWaves = 4;
constexpr int kColRows = 201;   // restart <= 200

__global__ void __launch_bounds__(64 * kColWaves) k_pair_column(ArnoldiState st, const double2* __restrict__ h,
                                                                const double2* __restrict__ gcol,
                                                                const double2* __restrict__ pc,
                                                                double2* __restrict__ col, int j) {
    __shared__ double2 part[kColWaves][kColRows];
    const int r = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6, m = st.m, nvec = j + 1;
    const double2* hr = h + (long long)r * nvec;
    const double2* Hr = st.Hr + (long long)r * m * (m + 1);
    for (int i = lane; i <= j; i += 64) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
        for (int k = wv; k <= j; k += kColWaves)
            if (k >= i - 1) acc = cadd(acc, cmul(Hr[(long long)k * (m + 1) + i], hr[k]));
        part[wv][i] = acc;
    }
    __syncthreads();
    if (wv == 0) {
        const double2 sigma = hr[j];
        const double ib = pc[2 * r + 1].x;
        double2* out = col + (long long)r * (nvec + 1);
        for (int i = lane; i <= j; i += 64) {
            double2 hh = part[0][i];
            for (int w = 1; w < kColWaves; ++w) hh = cadd(hh, part[w][i]);
            const double2 t = csub(cadd(gcol[(long long)r * nvec + i], cmul(sigma, hr[i])), hh);
            out[i] = make_double2(t.x * ib, t.y * ib);
        }
        if (lane == 0) out[j + 1] = pc[2 * r];
    }
}

void launch_pair_column(ArnoldiState st, const double2* h, const double2* gcol, const double2* pc, double2* col,
                        int j, int na, hipStream_t s) {
    VIE_REQUIRE(st.Hr != nullptr && j + 1 < st.m && j + 1 < kColRows, VIE_EINVAL,
                "pair column without the unrotated Hessenberg matrix");
    hipLaunchKernelGGL(k_pair_column, dim3(na), dim3(64 * kColWaves), 0, s, st, h, gcol, pc, col, j);
    VIE_HIP(hipGetLastError());
}

// ---- three Arnoldi steps per pass over the basis (s = 3) ----
//
// As the pair, with w1 = A u_j, w2 = A w1, w3 = A w2 (raw, in slots j + 1 ..
// j + 3) and the shifted vectors z1 = sw w1 = A v_j, z2 = (A - sigma) z1,
// z3 = (A - sigma)^2 z1 (sigma = h_jj).  One dot pass gives g_k = V^H z_k,
// one update pass y_k = z_k - V g_k with the block's Gram matrix G = Y^H Y,
// and its Cholesky factor R (G = R^H R, FP64) orthogonalises the block:
// q_k = (Y R^-1)_k.  Stored: u_{j+1} = y1 (norm R11), u_{j+2} = (y2 - R12 /
// R11 y1) / R11 and u_{j+3} = (y3 - R13 / R11 y1 - R23 / R22 (y2 - R12 / R11
// y1)) / R22, so that each norm is the subdiagonal entry of its column.
// Columns j + 1 and j + 2 follow from A z_k = z_{k+1} + sigma z_k:
//   A q1 = (z2 + sigma z1 - A V g1) / R11,
//   A q2 = (z3 + sigma z2 - A V g2 - R12 A q1) / R22,
// with A V g = V_{j+2} H g over the unrotated columns 0..j.

// one wave per (row i, slot r): g1 = h, g2, g3 (rows of V^H z_k) and the
// update coefficients g_k ivn[i], from the 3 planes of dot partials
__global__ void __launch_bounds__(64) k_reduce_triple(double2* __restrict__ g, double2* __restrict__ coef,
                                                      const double2* __restrict__ partial, int nblocks, int nvec,
                                                      int na, const double* __restrict__ ivn, long long ivn_ld,
                                                      int jw, long long gst) {
    const int i = blockIdx.x, r = blockIdx.y, lane = threadIdx.x, j = nvec - 1;
    const double2* p1 = partial + ((long long)r * nvec + i) * nblocks;
    const double2* p2 = partial + (((long long)na + r) * nvec + i) * nblocks;
    const double2* p3 = partial + (((long long)2 * na + r) * nvec + i) * nblocks;
    const double2* pj = partial + ((long long)r * nvec + j) * nblocks;
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 4
    for (int k = lane; k < nblocks; k += 64) {
        a[0] += p1[k].x;
        a[1] += p1[k].y;
        a[2] += p2[k].x;
        a[3] += p2[k].y;
        a[4] += p3[k].x;
        a[5] += p3[k].y;
        a[6] += pj[k].x;
        a[7] += pj[k].y;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = wave_sum(a[q]);
    if (lane == 0) {
        const double sw = ivn[r * ivn_ld + jw], iv = ivn[r * ivn_ld + i], ivj = ivn[r * ivn_ld + j];
        const double2 sg = make_double2(a[6] * sw * ivj, a[7] * sw * ivj);
        const double2 P1 = make_double2(a[0] * sw * iv, a[1] * sw * iv);
        const double2 P2 = make_double2(a[2] * sw * iv, a[3] * sw * iv);
        const double2 P3 = make_double2(a[4] * sw * iv, a[5] * sw * iv);
        const double2 g2 = csub(P2, cmul(sg, P1));
        const double2 g3 = cadd(csub(P3, cscale(cmul(sg, P2), 2.0)), cmul(cmul(sg, sg), P1));
        const long long o = (long long)r * nvec + i;
        g[o] = P1;
        g[gst + o] = g2;
        g[2 * gst + o] = g3;
        coef[o] = make_double2(P1.x * iv, P1.y * iv);
        coef[gst + o] = make_double2(g2.x * iv, g2.y * iv);
        coef[2 * gst + o] = make_double2(g3.x * iv, g3.y * iv);
    }
}

void launch_reduce_triple(double2* g, double2* coef, const double2* partial, int nvec, int nblocks, int nrhs,
                          const double* ivn, long long ivn_ld, int jw, long long gst, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_triple, dim3(nvec, nrhs), dim3(64), 0, s, g, coef, partial, nblocks, nvec, nrhs, ivn,
                       ivn_ld, jw, gst);
    VIE_HIP(hipGetLastError());
}

// y_k = z_k - sum_i c_k,i u_i (k = 1..3, z_k from the raw w's, in place in
// slots j + 1 .. j + 3 = w, w + ldv, w + 2 ldv), with the partial sums of
// |y1|^2 (norm_partial) and of the Gram entries (gram_partial [r][block][8]:
// G11, G12, G13, G22, G23 as re/im, G11 and G22 real)
template <typename R, bool PAIR>
__global__ void __launch_bounds__(kTpb) k_update_triple(C<R>* __restrict__ w, const C<R>* __restrict__ Vb,
                                                        long long ldv, int nvec, const double2* __restrict__ coef,
                                                        long long gst, const double2* __restrict__ g, long long n,
                                                        long long rsv, long long rsw,
                                                        double* __restrict__ norm_partial,
                                                        double* __restrict__ gram_partial,
                                                        const double* __restrict__ ivn, long long ivn_ld, int jw) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    __shared__ double red[kTpb / 64][8];
    const int r = blockIdx.y;
    const T* V = reinterpret_cast<const T*>(Vb + r * rsv);
    T* w1p = reinterpret_cast<T*>(w + r * rsw);
    T* w2p = reinterpret_cast<T*>(w + r * rsw + ldv);
    T* w3p = reinterpret_cast<T*>(w + r * rsw + 2 * ldv);
    const long long nu = n / U::per, ldu = ldv / U::per;
    const double2* c1 = coef + (long long)r * nvec;
    const double2* c2 = c1 + gst;
    const double2* c3 = c2 + gst;
    const double2 sg = g[(long long)r * nvec + nvec - 1];
    const double2 sg2 = cmul(sg, sg);
    const double sw = ivn[r * ivn_ld + jw];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long k = blockIdx.x * (long long)kTpb + threadIdx.x; k < nu; k += (long long)gridDim.x * kTpb) {
        T a1 = w1p[k], a2 = w2p[k], a3 = w3p[k];
        double2 y1[U::per], y2[U::per], y3[U::per];
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            const double2 o1 = U::get(a1, q), o2 = U::get(a2, q), o3 = U::get(a3, q);
            const double2 t2 = csub(o2, cmul(sg, o1));
            const double2 t3 = cadd(csub(o3, cscale(cmul(sg, o2), 2.0)), cmul(sg2, o1));
            y1[q] = make_double2(sw * o1.x, sw * o1.y);
            y2[q] = make_double2(sw * t2.x, sw * t2.y);
            y3[q] = make_double2(sw * t3.x, sw * t3.y);
        }
        int i = 0;
        for (; i + 8 <= nvec; i += 8) {
            T vu[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) vu[u] = stream_load(&V[(i + u) * ldu + k]);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double2 p1 = c1[i + u], p2 = c2[i + u], p3 = c3[i + u];
#pragma unroll
                for (int q = 0; q < U::per; ++q) {
                    const double2 v = U::get(vu[u], q);
                    y1[q] = csub(y1[q], cmul(p1, v));
                    y2[q] = csub(y2[q], cmul(p2, v));
                    y3[q] = csub(y3[q], cmul(p3, v));
                }
            }
        }
        for (; i < nvec; ++i) {
            const T vu = stream_load(&V[i * ldu + k]);
            const double2 p1 = c1[i], p2 = c2[i], p3 = c3[i];
#pragma unroll
            for (int q = 0; q < U::per; ++q) {
                const double2 v = U::get(vu, q);
                y1[q] = csub(y1[q], cmul(p1, v));
                y2[q] = csub(y2[q], cmul(p2, v));
                y3[q] = csub(y3[q], cmul(p3, v));
            }
        }
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            U::set(a1, q, y1[q]);
            U::set(a2, q, y2[q]);
            U::set(a3, q, y3[q]);
        }
        w1p[k] = a1;
        w2p[k] = a2;
        w3p[k] = a3;
#pragma unroll
        for (int q = 0; q < U::per; ++q) {   // the stored (rounded) values
            const double2 o1 = U::get(a1, q), o2 = U::get(a2, q), o3 = U::get(a3, q);
            acc[0] += o1.x * o1.x + o1.y * o1.y;
            acc[1] += o1.x * o2.x + o1.y * o2.y;   // conj(y1) y2
            acc[2] += o1.x * o2.y - o1.y * o2.x;
            acc[3] += o1.x * o3.x + o1.y * o3.y;   // conj(y1) y3
            acc[4] += o1.x * o3.y - o1.y * o3.x;
            acc[5] += o2.x * o2.x + o2.y * o2.y;
            acc[6] += o2.x * o3.x + o2.y * o3.y;   // conj(y2) y3
            acc[7] += o2.x * o3.y - o2.y * o3.x;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0;
        for (int wv = 0; wv < kTpb / 64; ++wv) t += red[wv][threadIdx.x];
        gram_partial[((long long)r * gridDim.x + blockIdx.x) * 8 + threadIdx.x] = t;
        if (threadIdx.x == 0) norm_partial[(long long)r * gridDim.x + blockIdx.x] = t;
    }
}

template <typename R>
void launch_update_triple(C<R>* w, const C<R>* Vb, long long ldv, int nvec, const double2* coef, long long gst,
                          const double2* g, long long n, long long rsv, long long rsw, double* norm_partial,
                          double* gram_partial, const double* ivn, long long ivn_ld, int jw, int nrhs, int nblocks,
                          hipStream_t s) {
    if (pair_units<R>(Vb, w, n, ldv, rsv, rsw))
        hipLaunchKernelGGL((k_update_triple<R, true>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, w, Vb, ldv, nvec, coef,
                           gst, g, n, rsv, rsw, norm_partial, gram_partial, ivn, ivn_ld, jw);
    else
        hipLaunchKernelGGL((k_update_triple<R, false>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, w, Vb, ldv, nvec, coef,
                           gst, g, n, rsv, rsw, norm_partial, gram_partial, ivn, ivn_ld, jw);
    VIE_HIP(hipGetLastError());
}

// per slot: the Gram sums (lane-strided, fixed order), the Cholesky factor
// and the coefficients of the stored vectors, tc[8 s ..]: (R11, R22), R12,
// R13, R23, (1 / R11, 1 / R22), a21 = R12 / R11, b31 = R13 / R11, b32 =
// R23 / R22 (zero where a pivot is not positive)
__global__ void __launch_bounds__(64) k_triple_coef(double2* __restrict__ tc, const double* __restrict__ gpart,
                                                    int nblocks) {
    const int r = blockIdx.x, lane = threadIdx.x;
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 4
    for (int b = lane; b < nblocks; b += 64) {
        const double* p = gpart + ((long long)r * nblocks + b) * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] += p[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = wave_sum(a[q]);
    if (lane == 0) {
        const double g11 = a[0], g22 = a[5];
        const double2 g12 = make_double2(a[1], a[2]), g13 = make_double2(a[3], a[4]), g23 = make_double2(a[6], a[7]);
        const double r11 = g11 > 0 ? sqrt(g11) : 0.0, i11 = r11 > 0 ? 1.0 / r11 : 0.0;
        const double2 r12 = cscale(g12, i11), r13 = cscale(g13, i11);
        const double d22 = g22 - (r12.x * r12.x + r12.y * r12.y);
        const double r22 = d22 > 0 ? sqrt(d22) : 0.0, i22 = r22 > 0 ? 1.0 / r22 : 0.0;
        const double2 r23 = cscale(csub(g23, cmulc(r12, r13)), i22);   // (G23 - conj(R12) R13) / R22
        double2* o = tc + 8 * r;
        o[0] = make_double2(r11, r22);
        o[1] = r12;
        o[2] = r13;
        o[3] = r23;
        o[4] = make_double2(i11, i22);
        o[5] = cscale(r12, i11);
        o[6] = cscale(r13, i11);
        o[7] = cscale(r23, i22);
    }
}

void launch_triple_coef(double2* tc, const double* gpart, int nblocks, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_triple_coef, dim3(nrhs), dim3(64), 0, s, tc, gpart, nblocks);
    VIE_HIP(hipGetLastError());
}

// u2 <- (y2 - a21 y1) / R11, u3 <- (y3 - b31 y1 - b32 (y2 - a21 y1)) / R22 in
// place (y_k in slots j + 1 .. j + 3 = u1, u1 + ldv, u1 + 2 ldv), with the
// partial sums of |u2|^2 and |u3|^2 over the stored values
template <typename R, bool PAIR>
__global__ void __launch_bounds__(kTpb) k_axpy_triple(C<R>* __restrict__ u1, long long ldv, long long n,
                                                      long long rs, const double2* __restrict__ tc,
                                                      double* __restrict__ np2, double* __restrict__ np3) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    __shared__ double red[kTpb / 64][2];
    const int r = blockIdx.y;
    const T* a = reinterpret_cast<const T*>(u1 + r * rs);
    T* b = reinterpret_cast<T*>(u1 + r * rs + ldv);
    T* c = reinterpret_cast<T*>(u1 + r * rs + 2 * ldv);
    const long long nu = n / U::per;
    const double2* t = tc + 8 * r;
    const double i11 = t[4].x, i22 = t[4].y;
    const double2 a21 = t[5], b31 = t[6], b32 = t[7];
    double s2 = 0.0, s3 = 0.0;
    for (long long k = blockIdx.x * (long long)kTpb + threadIdx.x; k < nu; k += (long long)gridDim.x * kTpb) {
        const T au = a[k];
        T bu = b[k], cu = c[k];
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            const double2 y1 = U::get(au, q), y2 = U::get(bu, q), y3 = U::get(cu, q);
            const double2 d2 = csub(y2, cmul(a21, y1));
            const double2 d3 = csub(csub(y3, cmul(b31, y1)), cmul(b32, d2));
            U::set(bu, q, cscale(d2, i11));
            U::set(cu, q, cscale(d3, i22));
        }
        b[k] = bu;
        c[k] = cu;
#pragma unroll
        for (int q = 0; q < U::per; ++q) {
            const double2 o2 = U::get(bu, q), o3 = U::get(cu, q);
            s2 += o2.x * o2.x + o2.y * o2.y;
            s3 += o3.x * o3.x + o3.y * o3.y;
        }
    }
    s2 = wave_sum(s2);
    s3 = wave_sum(s3);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = s2;
        red[threadIdx.x >> 6][1] = s3;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = 0;
        for (int i = 0; i < kTpb / 64; ++i) v += red[i][threadIdx.x];
        (threadIdx.x ? np3 : np2)[(long long)r * gridDim.x + blockIdx.x] = v;
    }
}

template <typename R>
void launch_axpy_triple(C<R>* u1, long long ldv, long long n, long long rs, const double2* tc, double* np2,
                        double* np3, int nrhs, int nblocks, hipStream_t s) {
    if (pair_units<R>(u1, u1, n, ldv, rs, rs))
        hipLaunchKernelGGL((k_axpy_triple<R, true>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, u1, ldv, n, rs, tc, np2,
                           np3);
    else
        hipLaunchKernelGGL((k_axpy_triple<R, false>), dim3(nblocks, nrhs), dim3(kTpb), 0, s, u1, ldv, n, rs, tc, np2,
                           np3);
    VIE_HIP(hipGetLastError());
}

// Hessenberg columns j + 1 (entries 0..j + 1) and j + 2 (entries 0..j + 2)
// of a triple into col1 [na][j + 2] and col2 [na][j + 3] (the subdiagonal
// entries come from the stored norms): one workgroup of 4 waves per slot,
// the products A V g1 and A V g2 over the unrotated columns 0..j summed by
// the waves in LDS in a fixed order, then wave 0 forms the entries
__global__ void __launch_bounds__(64 * kColWaves) k_triple_columns(ArnoldiState st, const double2* __restrict__ g,
                                                                   long long gst, const double2* __restrict__ tc,
                                                                   double2* __restrict__ col1,
                                                                   double2* __restrict__ col2, int j) {
    __shared__ double2 part[2][kColWaves][kColRows];
    const int r = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6, m = st.m, nvec = j + 1;
    const double2* g1 = g + (long long)r * nvec;
    const double2* g2 = g1 + gst;
    const double2* g3 = g2 + gst;
    const double2* Hr = st.Hr + (long long)r * m * (m + 1);
    for (int i = lane; i <= j + 1; i += 64) {
        double2 a1 = make_double2(0.0, 0.0), a2 = make_double2(0.0, 0.0);
#pragma unroll 4
        for (int k = wv; k <= j; k += kColWaves)
            if (k >= i - 1) {
                const double2 hk = Hr[(long long)k * (m + 1) + i];
                a1 = cadd(a1, cmul(hk, g1[k]));
                a2 = cadd(a2, cmul(hk, g2[k]));
            }
        part[0][wv][i] = a1;
        part[1][wv][i] = a2;
    }
    __syncthreads();
    if (wv == 0) {
        const double2* t = tc + 8 * r;
        const double r11 = t[0].x, r22 = t[0].y, i11 = t[4].x, i22 = t[4].y;
        const double2 r12 = t[1], r13 = t[2], r23 = t[3];
        const double2 sg = g1[j];
        double2* o1 = col1 + (long long)r * (j + 2);   // the strides the Givens kernel reads
        double2* o2 = col2 + (long long)r * (j + 3);
        for (int i = lane; i <= j + 1; i += 64) {
            double2 hv1 = part[0][0][i], hv2 = part[1][0][i];
            for (int w = 1; w < kColWaves; ++w) {
                hv1 = cadd(hv1, part[0][w][i]);
                hv2 = cadd(hv2, part[1][w][i]);
            }
            // column j + 1, row i: (z2 + sigma z1 - A V g1)_i / R11
            double2 c1;
            if (i <= j) c1 = cscale(csub(cadd(g2[i], cmul(sg, g1[i])), hv1), i11);
            else c1 = cscale(r12, i11);   // row j + 1: R12 / R11
            o1[i] = c1;
            // column j + 2, row i: (z3 + sigma z2 - A V g2 - R12 A q1)_i / R22
            double2 c2;
            if (i <= j) c2 = csub(cadd(g3[i], cmul(sg, g2[i])), hv2);
            else c2 = csub(cadd(r13, cmul(sg, r12)), hv2);   // row j + 1 (z1 has no q1 part beyond R11)
            c2 = csub(c2, cmul(r12, c1));
            o2[i] = cscale(c2, i22);
        }
        if (lane == 0) {
            // column j + 2, row j + 2: (R23 + sigma R22 - R12 (A q1)_{j+2}) / R22, (A q1)_{j+2} = R22 / R11
            const double2 aq = make_double2(r22 * i11, 0.0);
            o2[j + 2] = cscale(csub(cadd(r23, cscale(sg, r22)), cmul(r12, aq)), i22);
        }
        (void)r11;
    }
}

void launch_triple_columns(ArnoldiState st, const double2* g, long long gst, const double2* tc, double2* col1,
                           double2* col2, int j, int na, hipStream_t s) {
    VIE_REQUIRE(st.Hr != nullptr && j + 2 < st.m && j + 2 < kColRows, VIE_EINVAL,
                "triple columns without the unrotated Hessenberg matrix");
    hipLaunchKernelGGL(k_triple_columns, dim3(na), dim3(64 * kColWaves), 0, s, st, g, gst, tc, col1, col2, j);
    VIE_HIP(hipGetLastError());
}

// norms from partial sums of squares; with inv != nullptr also their
// reciprocals (0 for a zero norm) at inv[r * inv_ld]
__global__ void k_reduce_norm(double* __restrict__ out, const double* __restrict__ partial, int nblocks,
                              double* __restrict__ inv, long long inv_ld) {
    const int r = blockIdx.x;
    double s = 0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nblocks; b += 64) s += partial[(long long)r * nblocks + b];
    s = wave_sum(s);
    if (threadIdx.x == 0) {
        const double nv = sqrt(s);
        out[r] = nv;
        if (inv) inv[r * inv_ld] = nv > 0 ? 1.0 / nv : 0.0;
    }
}

void launch_reduce_norm(double* out, const double* partial, int nblocks, int nrhs, hipStream_t s, double* inv,
                        long long inv_ld) {
    hipLaunchKernelGGL(k_reduce_norm, dim3(nrhs), dim3(64), 0, s, out, partial, nblocks, inv, inv_ld);
    VIE_HIP(hipGetLastError());
}

template <typename R>
__global__ void k_norm_partials(double* __restrict__ partial, const C<R>* __restrict__ v, long long n,
                                long long rs) {
    __shared__ double red[kTpb / 64];
    const int r = blockIdx.y;
    const C<R>* vr = v + r * rs;
    double acc = 0;
    for (long long k = blockIdx.x * (long long)kTpb + threadIdx.x; k < n; k += (long long)gridDim.x * kTpb) {
        const double2 z = to_d2(vr[k]);
        acc += z.x * z.x + z.y * z.y;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < kTpb / 64; ++i) s += red[i];
        partial[(long long)r * gridDim.x + blockIdx.x] = s;
    }
}

template <typename R>
void launch_norm_partials(double* partial, const C<R>* v, long long n, long long rs, int nrhs, int nblocks,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_norm_partials<R>, dim3(nblocks, nrhs), dim3(kTpb), 0, s, partial, v, n, rs);
    VIE_HIP(hipGetLastError());
}

// dst = src / norm[r]
template <typename R>
__global__ void k_scale_into(C<R>* dst, const C<R>* src, const double* __restrict__ norms,
                             long long n, long long rsd, long long rss) {
    const int r = blockIdx.y;
    const double nv = norms[r];
    const double inv = nv > 0 ? 1.0 / nv : 0.0;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const double2 z = to_d2(src[r * rss + k]);
        C<R> o;
        o.x = (R)(z.x * inv);
        o.y = (R)(z.y * inv);
        dst[r * rsd + k] = o;
    }
}

template <typename R>
void launch_scale_into(C<R>* dst, const C<R>* src, const double* norms, long long n, long long rsd, long long rss,
                       int nrhs, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_scale_into<R>, dim3(nb, nrhs), dim3(256), 0, s, dst, src, norms, n, rsd, rss);
    VIE_HIP(hipGetLastError());
}

// x (complex128) += sum_i y_i V_i
template <typename R>
__global__ void k_combine(double2* __restrict__ x, const C<R>* __restrict__ Vb, long long ldv, int nvec,
                          const double2* __restrict__ y, long long n, long long rsv) {
    const int r = blockIdx.y;
    const C<R>* V = Vb + r * rsv;
    double2* xr = x + (long long)r * n;
    const double2* yr = y + (long long)r * nvec;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        double2 acc = xr[k];
        for (int i = 0; i < nvec; ++i) {
            const double2 v = to_d2(V[i * ldv + k]);
            acc.x += yr[i].x * v.x - yr[i].y * v.y;
            acc.y += yr[i].x * v.y + yr[i].y * v.x;
        }
        xr[k] = acc;
    }
}

template <typename R>
void launch_combine(double2* x, const C<R>* Vb, long long ldv, int nvec, const double2* y, long long n,
                    long long rsv, int nrhs, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_combine<R>, dim3(nb, nrhs), dim3(256), 0, s, x, Vb, ldv, nvec, y, n, rsv);
    VIE_HIP(hipGetLastError());
}

// dst (complex64) = src * scale[r]
// ---- least-squares side of the restart cycle (FP64, one thread per slot) ----

__global__ void k_arnoldi_init(ArnoldiState st, double* __restrict__ ivn, long long ivn_ld, int na) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 4) st.status[t] = 0;
    if (t < na) {
        st.g[(long long)t * (st.m + 1)] = make_double2(st.slot[t].x, 0.0);
        ivn[t * ivn_ld] = 1.0;
    }
}

void launch_arnoldi_init(ArnoldiState st, double* ivn, long long ivn_ld, int na, hipStream_t s) {
    const int n = na > 4 ? na : 4;
    hipLaunchKernelGGL(k_arnoldi_init, dim3((n + 255) / 256), dim3(256), 0, s, st, ivn, ivn_ld, na);
    VIE_HIP(hipGetLastError());
}

// One workgroup of kGivWaves waves; wave w takes slots w, w + kGivWaves, ...
// For slot s it sums the norm partials of w into ||w|| (lane-strided, the
// order of k_reduce_norm) and the reciprocal norm of the new basis vector,
// stages column j of the Hessenberg matrix (h_i, i <= j, from the
// Gram-Schmidt pass(es); h_{j+1} = ||w||) and the earlier rotations in LDS,
// and lane 0 applies the rotations, forms the new one that zeroes h_{j+1}
// and rotates g, so |g_{j+1}| is the least-squares residual after j + 1
// steps.
constexpr int kGivWaves = 4;
constexpr int kGivRows = 201;   // restart <= 200

__global__ void __launch_bounds__(64 * kGivWaves) k_givens(ArnoldiState st, const double2* __restrict__ h1,
                                                           const double2* __restrict__ h2,
                                                           const double* __restrict__ npart, int nblocks,
                                                           double* __restrict__ nrm, double* __restrict__ ivn_next,
                                                           long long ivn_ld, int j, int na) {
    __shared__ double2 lh[kGivWaves][kGivRows], lc[kGivWaves][kGivRows], ls[kGivWaves][kGivRows];
    __shared__ double lhn[kGivWaves];
    __shared__ int open, bad;
    const bool stopped = st.status[1] | st.status[2];   // uniform: stopped at an earlier column
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, m = st.m, nvec = j + 1;
    if (threadIdx.x == 0) {
        open = 0;
        bad = 0;
    }
    for (int base = 0; base < na; base += kGivWaves) {   // the same trip count in every wave
        const int s = base + wv;
        if (s < na) {
            double q = 0;
#pragma unroll 8
            for (int b = lane; b < nblocks; b += 64) q += npart[(long long)s * nblocks + b];
            q = wave_sum(q);
            if (lane == 0) {
                const double nv = sqrt(q);
                nrm[s] = nv;
                ivn_next[s * ivn_ld] = nv > 0 ? 1.0 / nv : 0.0;
                lhn[wv] = nv;
            }
            if (!stopped)
                for (int i = lane; i <= j; i += 64) {
                    double2 v = h1[(long long)s * nvec + i];
                    if (h2) v = cadd(v, h2[(long long)s * nvec + i]);
                    lh[wv][i] = v;
                    if (i < j) {
                        lc[wv][i] = st.cs[(long long)s * m + i];
                        ls[wv][i] = st.sn[(long long)s * m + i];
                    }
                }
        }
        __syncthreads();
        if (!stopped && s < na && lane == 0) {
            const double hn = lhn[wv];
            double2* Hc = st.H + ((long long)s * m + j) * (m + 1);
            double2* g = st.g + (long long)s * (m + 1);
            // earlier rotations: (a, b) <- (c a + z b, conj(c) b - conj(z) a)
            double2 a = lh[wv][0];
            for (int i = 0; i < j; ++i) {
                const double2 b = lh[wv][i + 1], c = lc[wv][i], z = ls[wv][i];
                Hc[i] = cadd(cmul(c, a), cmul(z, b));
                a = csub(cmulc(c, b), cmulc(z, a));
            }
            const double den = sqrt(a.x * a.x + a.y * a.y + hn * hn);
            double2 c, z;
            if (den == 0.0) {
                c = make_double2(1.0, 0.0);
                z = make_double2(0.0, 0.0);
            } else {
                c = make_double2(a.x / den, -a.y / den);   // conj(a) / den
                z = make_double2(hn / den, 0.0);
            }
            if (st.Hr) {   // the unrotated column, for the two-step Arnoldi
                double2* Hu = st.Hr + ((long long)s * m + j) * (m + 1);
                for (int i = 0; i <= j; ++i) Hu[i] = lh[wv][i];
                Hu[j + 1] = make_double2(hn, 0.0);
            }
            st.cs[(long long)s * m + j] = c;
            st.sn[(long long)s * m + j] = z;
            Hc[j] = make_double2(den, 0.0);
            Hc[j + 1] = make_double2(0.0, 0.0);
            const double2 gj = g[j];
            const double2 gn = make_double2(-(z.x * gj.x + z.y * gj.y), -(z.x * gj.y - z.y * gj.x));   // -conj(z) g_j
            g[j + 1] = gn;
            g[j] = cmul(c, gj);
            const double est = sqrt(gn.x * gn.x + gn.y * gn.y) / st.slot[s].x;
            if (!isfinite(est)) atomicOr(&bad, 1);
            if (!(est <= st.slot[s].y) && hn > 0.0) atomicOr(&open, 1);
        }
        __syncthreads();   // the LDS rows are reused by the next round
    }
    if (threadIdx.x == 0 && !stopped) {
        st.status[0] = nvec;
        if (bad) st.status[2] = 1;
        if (!open) st.status[1] = 1;
    }
}

void launch_givens(ArnoldiState st, const double2* h1, const double2* h2, const double* npart, int nblocks,
                   double* nrm, double* ivn_next, long long ivn_ld, int j, int na, hipStream_t s) {
    VIE_REQUIRE(j >= 0 && j + 1 < kGivRows && j < st.m, VIE_EINVAL, "Givens column beyond restart 200");
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64 * kGivWaves), 0, s, st, h1, h2, npart, nblocks, nrm, ivn_next,
                       ivn_ld, j, na);
    VIE_HIP(hipGetLastError());
}

// Back substitution R y = g for one slot per workgroup of one wave: lane l
// keeps the right-hand side rows l, l + 64, ... (nvec <= 256); column i of R
// updates the rows above i once y_i is known.
constexpr int kBackRows = 4;   // rows per lane

__global__ void __launch_bounds__(64) k_backsolve(ArnoldiState st, const double* __restrict__ ivn,
                                                  long long ivn_ld, double2* __restrict__ y, int nvec) {
    __shared__ double2 yl[64 * kBackRows];
    const int s = blockIdx.x, lane = threadIdx.x, m = st.m;
    const double2* H = st.H + (long long)s * m * (m + 1);
    const double2* g = st.g + (long long)s * (m + 1);
    double2 b[kBackRows];
#pragma unroll
    for (int q = 0; q < kBackRows; ++q) {
        const int k = lane + 64 * q;
        b[q] = k < nvec ? g[k] : make_double2(0.0, 0.0);
    }
    for (int i = nvec - 1; i >= 0; --i) {
        const double2* Hi = H + (long long)i * (m + 1);
        if (lane == (i & 63)) {
            double2 bi = b[0];
#pragma unroll
            for (int q = 1; q < kBackRows; ++q)
                if (q == (i >> 6)) bi = b[q];
            const double2 d = Hi[i];
            const double dd = d.x * d.x + d.y * d.y;
            yl[i] = dd == 0.0 ? make_double2(0.0, 0.0) : cscale(cmulc(d, bi), 1.0 / dd);   // bi / d
        }
        __syncthreads();
        const double2 yi = yl[i];
#pragma unroll
        for (int q = 0; q < kBackRows; ++q) {
            const int k = lane + 64 * q;
            if (k < i) b[q] = csub(b[q], cmul(Hi[k], yi));
        }
    }
    __syncthreads();
    for (int i = lane; i < nvec; i += 64) y[(long long)s * nvec + i] = cscale(yl[i], ivn[s * ivn_ld + i]);
}

void launch_backsolve(ArnoldiState st, const double* ivn, long long ivn_ld, double2* y, int nvec, int na,
                      hipStream_t s) {
    VIE_REQUIRE(nvec >= 1 && nvec <= 64 * kBackRows, VIE_EINVAL, "back substitution of 1..256 columns");
    hipLaunchKernelGGL(k_backsolve, dim3(na), dim3(64), 0, s, st, ivn, ivn_ld, y, nvec);
    VIE_HIP(hipGetLastError());
}

__global__ void k_cast_down(float2* __restrict__ dst, const double2* __restrict__ src, const double* __restrict__ sc,
                            long long n) {
    const int r = blockIdx.y;
    const double s = sc ? sc[r] : 1.0;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const double2 z = src[(long long)r * n + k];
        dst[(long long)r * n + k] = make_float2((float)(z.x * s), (float)(z.y * s));
    }
}

void launch_cast_down(float2* dst, const double2* src, const double* scale, long long n, int nrhs, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_cast_down, dim3(nb, nrhs), dim3(256), 0, s, dst, src, scale, n);
    VIE_HIP(hipGetLastError());
}

__global__ void k_cast_up(double2* __restrict__ dst, const float2* __restrict__ src, long long n) {
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        dst[k] = make_double2(src[k].x, src[k].y);
}

void launch_cast_up(double2* dst, const float2* src, long long n, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_cast_up, dim3(nb), dim3(256), 0, s, dst, src, n);
    VIE_HIP(hipGetLastError());
}

__global__ void k_copy(double2* __restrict__ dst, const double2* __restrict__ src, long long n) {
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

void launch_copy_c128(double2* dst, const double2* src, long long n, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, dst, src, n);
    VIE_HIP(hipGetLastError());
}

__global__ void k_nonfinite(int* flag, const double2* __restrict__ v, long long n) {
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        if (!isfinite(v[k].x) || !isfinite(v[k].y)) atomicOr(flag, 1);
}

void launch_nonfinite(int* flag, const double2* v, long long n, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_nonfinite, dim3(nb), dim3(256), 0, s, flag, v, n);
    VIE_HIP(hipGetLastError());
}

#define INST(R)                                                                                                  \
    template void launch_multidot<R>(double2*, const C<R>*, long long, int, const C<R>*, long long, long long,  \
                                     long long, int, int, hipStream_t);                                          \
    template void launch_update<R>(C<R>*, const C<R>*, long long, int, const double2*, long long, long long,   \
                                   long long, double*, const double*, long long, int, int, int, hipStream_t);    \
    template void launch_multidot2<R>(double2*, const C<R>*, long long, int, const C<R>*, long long, long long,  \
                                      long long, long long, int, int, hipStream_t);                               \
    template void launch_update_pair<R>(C<R>*, const C<R>*, long long, int, const double2*, const double2*,      \
                                        const double2*, long long, long long, long long, double*, double2*,      \
                                        const double*, long long, int, int, int, hipStream_t);                   \
    template void launch_axpy_pair<R>(C<R>*, long long, long long, long long, const double2*, double*, int, int, \
                                      hipStream_t);                                                               \
    template void launch_multidot3<R>(double2*, const C<R>*, long long, int, const C<R>*, long long, long long,  \
                                      long long, long long, int, int, hipStream_t);                               \
    template void launch_update_triple<R>(C<R>*, const C<R>*, long long, int, const double2*, long long,        \
                                          const double2*, long long, long long, long long, double*, double*,     \
                                          const double*, long long, int, int, int, hipStream_t);                 \
    template void launch_axpy_triple<R>(C<R>*, long long, long long, long long, const double2*, double*,        \
                                        double*, int, int, hipStream_t);                                          \
    template void launch_scale_into<R>(C<R>*, const C<R>*, const double*, long long, long long, long long, int, \
                                       hipStream_t);                                                             \
    template void launch_combine<R>(double2*, const C<R>*, long long, int, const double2*, long long, long long, \
                                    int, hipStream_t);                                                           \
    template void launch_norm_partials<R>(double*, const C<R>*, long long, long long, int, int, hipStream_t);
INST(float)
INST(double)

}  // namespace vie
