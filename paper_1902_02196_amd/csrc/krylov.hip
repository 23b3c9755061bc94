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

// One group of G basis vectors (G compile-time, so that the G + 1 loads of an
// element are issued together with no guard between them): FP64 sums of
// conj(V_i) w over this thread's elements, reduced over the workgroup and
// written to partial[(r * nvec + i) * nblocks + block].
template <typename R, bool PAIR, int G>
__device__ __forceinline__ void dot_group(double2* __restrict__ partial,
                                          const typename Unit<R, PAIR>::T* __restrict__ V,
                                          const typename Unit<R, PAIR>::T* __restrict__ wr, long long ldu,
                                          long long nu, int i0, int nvec, int r, double (*red)[2 * kGroup]) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long stride = (long long)gridDim.x * kTpb;
    double ar[G], ai[G];
#pragma unroll
    for (int g = 0; g < G; ++g) ar[g] = ai[g] = 0.0;
    for (long long k = blockIdx.x * (long long)kTpb + threadIdx.x; k < nu; k += stride) {
        const T wu = wr[k];
        T vu[G];
#pragma unroll
        for (int g = 0; g < G; ++g) vu[g] = stream_load(&V[(i0 + g) * ldu + k]);
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int h = 0; h < U::per; ++h) {
                const double2 v = U::get(vu[g], h), wv = U::get(wu, h);
                ar[g] += v.x * wv.x + v.y * wv.y;
                ai[g] += v.x * wv.y - v.y * wv.x;
            }
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const double sr = wave_sum(ar[g]), si = wave_sum(ai[g]);
        if (lane == 0) { red[wave][2 * g] = sr; red[wave][2 * g + 1] = si; }
    }
    __syncthreads();
    if (threadIdx.x < G) {
        const int g = threadIdx.x;
        double sr = 0, si = 0;
        for (int wv = 0; wv < kTpb / 64; ++wv) { sr += red[wv][2 * g]; si += red[wv][2 * g + 1]; }
        partial[((long long)r * nvec + i0 + g) * gridDim.x + blockIdx.x] = make_double2(sr, si);
    }
    __syncthreads();
}

// partial sums of conj(V_i) w for i < nvec: workgroup (b, r, g) takes group g
// of kGroup basis vectors (the last group may hold fewer) over its share of
// the elements, so the groups stream side by side (vectors read in units of
// Unit<R, PAIR>; n and the strides multiples of the unit)
template <typename R, bool PAIR>
__global__ void __launch_bounds__(kTpb) k_multidot(double2* __restrict__ partial, const C<R>* __restrict__ Vb,
                                                   long long ldv, int nvec, const C<R>* __restrict__ w, long long n,
                                                   long long rsv, long long rsw) {
    using U = Unit<R, PAIR>;
    using T = typename U::T;
    __shared__ double red[kTpb / 64][2 * kGroup];
    const int r = blockIdx.y;
    const T* V = reinterpret_cast<const T*>(Vb + r * rsv);
    const T* wr = reinterpret_cast<const T*>(w + r * rsw);
    const long long nu = n / U::per, ldu = ldv / U::per;
    static_assert(kGroup == 8, "the group sizes below cover 1 to 8");
    const int i0 = blockIdx.z * kGroup;
    switch (min(kGroup, nvec - i0)) {   // uniform over the workgroup
#define VIE_DOT_G(g_) \
    case g_: dot_group<R, PAIR, g_>(partial, V, wr, ldu, nu, i0, nvec, r, red); break;
        VIE_DOT_G(1) VIE_DOT_G(2) VIE_DOT_G(3) VIE_DOT_G(4) VIE_DOT_G(5) VIE_DOT_G(6) VIE_DOT_G(7) VIE_DOT_G(8)
#undef VIE_DOT_G
        default: break;
    }
}

template <typename R>
void launch_multidot(double2* partial, const C<R>* Vb, long long ldv, int nvec, const C<R>* w, long long n,
                     long long rsv, long long rsw, int nrhs, int nblocks, hipStream_t s) {
    const unsigned ngroups = (unsigned)((nvec + kGroup - 1) / kGroup);
    if (pair_units<R>(Vb, w, n, ldv, rsv, rsw))
        hipLaunchKernelGGL((k_multidot<R, true>), dim3(nblocks, nrhs, ngroups), dim3(kTpb), 0, s, partial, Vb, ldv,
                           nvec, w, n, rsv, rsw);
    else
        hipLaunchKernelGGL((k_multidot<R, false>), dim3(nblocks, nrhs, ngroups), dim3(kTpb), 0, s, partial, Vb, ldv,
                           nvec, w, n, rsv, rsw);
    VIE_HIP(hipGetLastError());
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

// norms from partial sums of squares; with inv != nullptr also their
// reciprocals (0 for a zero norm) at inv[r * inv_ld]
__global__ void k_reduce_norm(double* __restrict__ out, const double* __restrict__ partial, int nblocks,
                              double* __restrict__ inv, long long inv_ld) {
    const int r = blockIdx.x;
    double s = 0;
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
    template void launch_scale_into<R>(C<R>*, const C<R>*, const double*, long long, long long, long long, int, \
                                       hipStream_t);                                                             \
    template void launch_combine<R>(double2*, const C<R>*, long long, int, const double2*, long long, long long, \
                                    int, hipStream_t);                                                           \
    template void launch_norm_partials<R>(double*, const C<R>*, long long, long long, int, int, hipStream_t);
INST(float)
INST(double)

}  // namespace vie
