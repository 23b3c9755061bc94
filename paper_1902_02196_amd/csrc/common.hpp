// Shared definitions of the HIP library: complex helpers, error handling,
// unknown-index bookkeeping of the PWL basis.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace vie {

// ---------------------------------------------------------------------------
// complex arithmetic on float2 / double2
// ---------------------------------------------------------------------------
template <typename R> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename R> using C = typename cplx<R>::type;

template <typename R> __host__ __device__ __forceinline__ C<R> mk(R re, R im) {
    C<R> z;
    z.x = re;
    z.y = im;
    return z;
}
template <typename T> __host__ __device__ __forceinline__ T cadd(T a, T b) { T r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename T> __host__ __device__ __forceinline__ T csub(T a, T b) { T r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename T> __host__ __device__ __forceinline__ T cmul(T a, T b) {
    T r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// conj(a) * b
template <typename T> __host__ __device__ __forceinline__ T cmulc(T a, T b) {
    T r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.x * b.y - a.y * b.x;
    return r;
}
template <typename T, typename S> __host__ __device__ __forceinline__ T cscale(T a, S s) { T r; r.x = a.x * s; r.y = a.y * s; return r; }
// multiply by -i (forward) or +i (inverse)
template <bool FWD, typename T> __host__ __device__ __forceinline__ T mul_mi(T a) {
    T r;
    if (FWD) { r.x = a.y; r.y = -a.x; } else { r.x = -a.y; r.y = a.x; }
    return r;
}
// acc += a * b
// Load marked non-temporal (streaming cache policy) for data read once: it
// keeps the caches, including the 256 MB Infinity Cache, for data that is
// read again (the operator octant, the next pass's intermediates).
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
    static_assert(sizeof(T) == 8 || sizeof(T) == 16, "8- or 16-byte elements");
    if constexpr (sizeof(T) == 8) {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u2*>(p)));
    } else {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u4*>(p)));
    }
}

__host__ __device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }

// acc += a * b as four fused multiply-adds
template <typename T> __host__ __device__ __forceinline__ void cfma(T& acc, T a, T b) {
    acc.x = fma_(a.x, b.x, acc.x);
    acc.x = fma_(-a.y, b.y, acc.x);
    acc.y = fma_(a.x, b.y, acc.y);
    acc.y = fma_(a.y, b.x, acc.y);
}

// ---------------------------------------------------------------------------
// PWL unknown bookkeeping: a = 4 p + (l - 1); reflection signs
// ---------------------------------------------------------------------------
// sigma_axis(a): reflecting `axis` flips the field component along it and the
// linear function along it (scalar basis l == axis + 2).
constexpr __host__ __device__ __forceinline__ int refl_sign(int axis, int a) {
    int p = a >> 2, l = (a & 3) + 1;
    int s = 1;
    if (p == axis) s = -s;
    if (l == axis + 2) s = -s;
    return s;
}
// bit a of the mask set where prod over the folded axes of sigma_axis(a) = -1
constexpr __host__ __device__ __forceinline__ unsigned fold_mask(int fx, int fy, int fz) {
    unsigned m = 0;
    for (int a = 0; a < 12; ++a) {
        int s = 1;
        if (fx) s *= refl_sign(0, a);
        if (fy) s *= refl_sign(1, a);
        if (fz) s *= refl_sign(2, a);
        if (s < 0) m |= (1u << a);
    }
    return m;
}
// unique-entry index of N^{(p,l),(q,l')}: 10 * pq + ll, with the sign that
// relates the entry to the stored (p <= q, l <= l') one.
constexpr __host__ __device__ __forceinline__ int pq_index(int p, int q) {
    if (p > q) { int t = p; p = q; q = t; }
    // (0,0)=0 (0,1)=1 (0,2)=2 (1,1)=3 (1,2)=4 (2,2)=5
    return p == 0 ? q : (p == 1 ? 2 + q : 5);
}
constexpr __host__ __device__ __forceinline__ int ll_index(int l, int lp) {  // l, lp in 1..4
    if (l > lp) { int t = l; l = lp; lp = t; }
    // (1,1)=0 (1,2)=1 (1,3)=2 (1,4)=3 (2,2)=4 (2,3)=5 (2,4)=6 (3,3)=7 (3,4)=8 (4,4)=9
    return (l - 1) * (10 - l) / 2 + (lp - l);
}
constexpr __host__ __device__ __forceinline__ int unique_index(int a, int b) {
    return 10 * pq_index(a >> 2, b >> 2) + ll_index((a & 3) + 1, (b & 3) + 1);
}
// exchanging the scalar bases of a pulse / linear pair flips the sign
constexpr __host__ __device__ __forceinline__ int unique_sign(int a, int b) {
    int l = (a & 3) + 1, lp = (b & 3) + 1;
    return (l > lp && lp == 1) ? -1 : 1;
}

// curl operator K = curl S: K^{(p,l),(q,l')} = eps_{pkq} Q_k^{ll'}, zero for
// p = q, with the 30 unique tensors Q_k^{ll'} (l <= l') stored as 10 k + ll;
// Q_k^{l'l} = s(l) s(l') Q_k^{ll'} (exchanging the two functions reflects w)
constexpr __host__ __device__ __forceinline__ int levi(int p, int k, int q) {
    return (p == k || k == q || p == q) ? 0 : (((k - p + 3) % 3 == 1) ? 1 : -1);
}
constexpr __host__ __device__ __forceinline__ int curl_unique_index(int a, int b) {
    const int p = a >> 2, q = b >> 2;
    return p == q ? -1 : 10 * (3 - p - q) + ll_index((a & 3) + 1, (b & 3) + 1);
}
constexpr __host__ __device__ __forceinline__ int curl_unique_sign(int a, int b) {
    const int p = a >> 2, q = b >> 2;
    return p == q ? 0 : levi(p, 3 - p - q, q) * unique_sign(a, b);
}

// The dispatcher deals workgroups to the 8 XCDs round-robin by linear
// index.  This maps a linear hardware index h < n to a logical index such
// that each XCD receives one contiguous range of logical indices, taken in
// order: workgroups with neighbouring logical indices run on the same XCD at
// about the same time and share its L2.
constexpr int kXcds = 8;
__device__ __forceinline__ unsigned xcd_contiguous(unsigned h, unsigned n) {
    const unsigned q = n / kXcds, r = n % kXcds, x = h % kXcds, k = h / kXcds;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define VIE_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            throw ::vie::Error(e_ == hipErrorOutOfMemory ? -2 : -3,                         \
                               std::string(#call) + ": " + hipGetErrorString(e_));           \
    } while (0)

#define VIE_REQUIRE(cond, code, msg)                                   \
    do {                                                               \
        if (!(cond)) throw ::vie::Error((code), std::string(msg));     \
    } while (0)

}  // namespace vie
