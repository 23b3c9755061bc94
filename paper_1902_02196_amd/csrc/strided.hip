// Compiled-length strided FFT passes (Sec. IV-A): one kernel per (length,
// pencils per workgroup, direction, epilogue), kept in their own translation
// unit.
#include <mutex>

#include "fft_ct.hpp"
#include "kernels.hpp"
#include "passes.hpp"
#include "vie.h"

namespace vie {

// Compile-time-length strided pass: the tile's T pencils are held as T rows
// of N in LDS (one buffer, padded) and transformed in place by the unrolled
// Stockham passes; loads and stores run along t, T consecutive elements.
//
// Workgroup order: the (tile, row, component array) of a workgroup is taken
// from its logical index (xcd_contiguous), tiles fastest, so that
// neighbouring tiles run on one XCD together: with tiles of 8 complex64 (64
// bytes, the long lengths, where 16 would leave one workgroup per CU) the
// two tiles of each 128-byte line are then read through the same L2 instead
// of twice, once per XCD.
// LDS row pitch of a tile: one pencil per row, padded to an odd number of
// complex elements when N is a multiple of 16, so that the T pencils of one
// element index k (the loads and stores run along the pencils) fall on T
// different bank pairs
__host__ __device__ constexpr int strided_rp(int n) { return n % 16 == 0 ? ((n + n / 16) | 1) : n + n / 16; }

template <typename R, bool FWD, bool EPI, int N, int T>
__global__ void __launch_bounds__(256) k_strided_ct(const C<R>* in, C<R>* out, StridedPass p,
                                                    const C<R>* __restrict__ tw, Epilogue<R> ep) {
    constexpr int NT = 256;
    constexpr int RP = strided_rp(N);
    auto at = [](int t, int k) { return RP == N + N / 16 ? lds_pad(t * N + k) : t * RP + lds_pad(k); };
    extern __shared__ unsigned char smem_raw[];
    C<R>* twl = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf = twl + N;
    const int tid = threadIdx.x;
    const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
    const unsigned lid = xcd_contiguous(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gz);
    const unsigned bx = lid % gx, by = (lid / gx) % gy, bz = lid / gx / gy;
    const int t0 = bx * T;
    const long long o2 = by;
    const int o1 = bz, rr = o1 / p.nc, cc = o1 - p.nc * rr;
    const int tw_n = min(T, p.n_inner - t0);
    const C<R>* src = in + rr * p.in_s1 + cc * p.in_sc + o2 * p.in_s2 + t0;
    for (int m = tid; m < N; m += NT) twl[m] = tw[m];
    constexpr int LN = N * T;
    constexpr int LPT = (LN + NT - 1) / NT;
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
        const int idx = tid + i * NT;
        if (LN % NT == 0 || idx < LN) {
            const int k = idx / T, t = idx - k * T;
            C<R> v = mk<R>(0, 0);
            if (k < p.n_in && t < tw_n) v = stream_load(&src[k * p.in_sk + t]);   // last read of the input
            buf[at(t, k)] = v;
        }
    }
    __syncthreads();
    if (FWD && 2 * p.n_in <= N) ct_passes<R, FWD, N, 0, 1, NT, T, FWD, false, RP>(buf, twl, T, N, tid);   // zero-padded
    else if (!FWD && 2 * p.n_out <= N) ct_passes<R, FWD, N, 0, 1, NT, T, false, !FWD, RP>(buf, twl, T, N, tid);   // cropped
    else ct_passes<R, FWD, N, 0, 1, NT, T, false, false, RP>(buf, twl, T, N, tid);
    const long long obase = rr * p.out_s1 + cc * p.out_sc;
    C<R>* dst = out + obase + o2 * p.out_s2 + t0;
    const int l = p.nc == 12 ? (cc & 3) : 0;
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
        const int idx = tid + i * NT;
        if (LN % NT == 0 || idx < LN) {
            const int k = idx / T, t = idx - k * T;
            if (k < p.n_out && t < tw_n) {
                C<R> w = buf[at(t, k)];
                if (EPI) {
                    const long long v = o2 * p.out_s2 + k * p.out_sk + t0 + t;   // voxel
                    const long long e = obase + v;                                  // element
                    C<R> bv = ep.b ? ep.b[v] : mk<R>(ep.b_const, 0);
                    C<R> y = cscale(cmul(bv, w), ep.gb[l]);
                    if (ep.a || ep.a_const != R(0)) {
                        C<R> av = ep.a ? ep.a[v] : mk<R>(ep.a_const, 0);
                        y = cadd(y, cscale(cmul(av, ep.x[e]), ep.ga[l]));
                    }
                    if (ep.rhs) y = cadd(y, ep.rhs[e]);
                    w = y;
                }
                dst[k * p.out_sk + t] = w;
            }
        }
    }
}

template <typename R, bool FWD, bool EPI, int N, int T>
static void launch_strided_ct_nt(const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2, long long n_o1,
                                 const C<R>* tw, const Epilogue<R>& ep, hipStream_t s) {
    const size_t lds = ((size_t)N + (size_t)T * strided_rp(N) + 2) * sizeof(C<R>);
    static std::once_flag once;
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void*)k_strided_ct<R, FWD, EPI, N, T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    });
    dim3 grid((p.n_inner + T - 1) / T, (unsigned)n_o2, (unsigned)n_o1);
    VIE_REQUIRE((unsigned long long)grid.x * grid.y * grid.z < (1ULL << 32), VIE_EINVAL,
                "strided pass grid above 2^32 workgroups");
    timed_launch(k_strided_ct<R, FWD, EPI, N, T>, grid, dim3(256), (unsigned)lds, s, in, out, p, tw, ep);
    VIE_HIP(hipGetLastError());
}

template <typename R, bool FWD, bool EPI, int N>
static void launch_strided_ct_n(const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2, long long n_o1,
                                const C<R>* tw, const Epilogue<R>& ep, hipStream_t s) {
    if constexpr (N >= 512) {
        if (p.tile == 4) {
            launch_strided_ct_nt<R, FWD, EPI, N, 4>(in, out, p, n_o2, n_o1, tw, ep, s);
            return;
        }
        if (p.tile == 8) {
            launch_strided_ct_nt<R, FWD, EPI, N, 8>(in, out, p, n_o2, n_o1, tw, ep, s);
            return;
        }
    }
    if (p.tile == 16) launch_strided_ct_nt<R, FWD, EPI, N, 16>(in, out, p, n_o2, n_o1, tw, ep, s);
    else launch_strided_ct_nt<R, FWD, EPI, N, 32>(in, out, p, n_o2, n_o1, tw, ep, s);
}

// compiled strided lengths (tiles of 16 or 32 pencils; also 8 and 4 from 512
// up, where a larger tile would hold one workgroup per CU)
#define VIE_STRIDED_LENGTHS(X) X(8) X(16) X(32) X(64) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512) X(768)

bool strided_ct_fits(int es, int n, int tile) {
    if (tile != 16 && tile != 32 && !((tile == 8 || tile == 4) && n >= 512)) return false;
    switch (n) {
#define CASE(n_) case n_:
        VIE_STRIDED_LENGTHS(CASE)
#undef CASE
        return ((size_t)n + (size_t)tile * strided_rp(n) + 2) * es <= 160 * 1024;
        default: return false;
    }
}

// a tile the strided pass can run: 16 or 32 pencils with a compiled length,
// or 4, 8, 16 pencils in the generic kernel (two buffers within 96 KiB)
bool strided_tile_ok(int es, int n, int tile) {
    if (strided_ct_fits(es, n, tile)) return true;
    return (tile == 1 || tile == 2 || tile == 4 || tile == 8 || tile == 16) && 2LL * tile * n * es <= 96 * 1024;
}

// pencils per workgroup for a strided pass of length n: `preferred` when the
// compiled kernel takes it, else 16, else the largest generic tile whose two
// LDS buffers fit 96 KiB
int strided_tile_for(int es, int n, int preferred) {
    if (strided_ct_fits(es, n, preferred)) return preferred;
    if (strided_ct_fits(es, n, 16)) return 16;
    int t = 16;
    while (t > 1 && 2LL * t * n * es > 96 * 1024) t /= 2;
    return t;
}

template <typename R, bool FWD, bool EPI>
static bool launch_strided_ct(const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2, long long n_o1,
                              const C<R>* tw, const Epilogue<R>& ep, hipStream_t s) {
    if (!strided_ct_fits((int)sizeof(C<R>), p.plan.n, p.tile)) return false;
    switch (p.plan.n) {
#define CASE(n_)                                                                   \
    case n_:                                                                      \
        launch_strided_ct_n<R, FWD, EPI, n_>(in, out, p, n_o2, n_o1, tw, ep, s); \
        return true;
        VIE_STRIDED_LENGTHS(CASE)
#undef CASE
        default: return false;
    }
}

template <typename R>
bool launch_strided_compiled(bool fwd, bool epi, const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2,
                             long long n_o1, const C<R>* tw, const Epilogue<R>& ep, hipStream_t s) {
    if (epi) return !fwd && launch_strided_ct<R, false, true>(in, out, p, n_o2, n_o1, tw, ep, s);
    if (fwd) return launch_strided_ct<R, true, false>(in, out, p, n_o2, n_o1, tw, ep, s);
    return launch_strided_ct<R, false, false>(in, out, p, n_o2, n_o1, tw, ep, s);
}

template bool launch_strided_compiled<float>(bool, bool, const C<float>*, C<float>*, const StridedPass&, long long,
                                             long long, const C<float>*, const Epilogue<float>&, hipStream_t);
template bool launch_strided_compiled<double>(bool, bool, const C<double>*, C<double>*, const StridedPass&,
                                              long long, long long, const C<double>*, const Epilogue<double>&,
                                              hipStream_t);

}  // namespace vie
