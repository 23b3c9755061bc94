// FFT-matvec passes (Sec. IV-A): strided zero-padded FFT passes along z and
// y, the fused x pass with the per-frequency block product, and the epilogue
// that crops and applies contrast / Gram scaling (Sec. IV-B).
#include "kernels.hpp"
#include "passes.hpp"

namespace vie {

// ---------------------------------------------------------------------------
// strided pass
// ---------------------------------------------------------------------------
template <typename R, bool FWD, bool EPI>
__global__ void __launch_bounds__(256) k_strided(const C<R>* in, C<R>* out,
                                                 StridedPass p, const C<R>* __restrict__ tw, Epilogue<R> ep) {
    extern __shared__ unsigned char smem_raw[];
    C<R>* buf0 = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf1 = buf0 + p.plan.n * p.pitch;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int t0 = blockIdx.x * p.tile;
    const long long o2 = blockIdx.y, o1 = blockIdx.z;
    const int tw_n = min(p.tile, p.n_inner - t0);
    const C<R>* src = in + o1 * p.in_s1 + o2 * p.in_s2 + t0;
    const int n = p.plan.n;
    // load (zero-padded beyond n_in and beyond the inner extent)
    for (int idx = tid; idx < n * p.tile; idx += nthr) {
        const int k = idx / p.tile, t = idx - k * p.tile;
        C<R> v = mk<R>(0, 0);
        if (k < p.n_in && t < tw_n) v = src[k * p.in_sk + t];
        buf0[k * p.pitch + t] = v;
    }
    __syncthreads();
    C<R>* res = fft_lds<R, FWD, false>(buf0, buf1, p.plan, p.tile, 1, p.pitch, tw, tid, nthr);
    C<R>* dst = out + o1 * p.out_s1 + o2 * p.out_s2 + t0;
    for (int idx = tid; idx < p.n_out * p.tile; idx += nthr) {
        const int k = idx / p.tile, t = idx - k * p.tile;
        if (t >= tw_n) continue;
        C<R> w = res[k * p.pitch + t];
        if (EPI) {
            const long long e = o1 * p.out_s1 + o2 * p.out_s2 + k * p.out_sk + t0 + t;   // element
            const long long v = e - o1 * p.out_s1;                                       // voxel
            const int l = int(o1 % 12) & 3;
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

// ---------------------------------------------------------------------------
// fused x pass
// ---------------------------------------------------------------------------
// The 144 entries of a frequency block come from 60 unique values; the orbit
// of unique entry e lists the (row, column, sign) positions it fills.
struct OrbitMember { int a, b, s; };
struct Orbits {
    OrbitMember m[60][4];
    int cnt[60];
};
constexpr Orbits make_orbits() {
    Orbits o{};
    for (int e = 0; e < 60; ++e) o.cnt[e] = 0;
    for (int a = 0; a < 12; ++a)
        for (int b = 0; b < 12; ++b) {
            const int e = unique_index(a, b);
            o.m[e][o.cnt[e]] = OrbitMember{a, b, unique_sign(a, b)};
            o.cnt[e]++;
        }
    return o;
}

// y[a] += s u x[b] over the orbit of unique entry E (all compile time)
template <typename R, int E, int K>
__device__ __forceinline__ void orbit_member(C<R>* yv, const C<R>* xv, C<R> u) {
    constexpr Orbits o = make_orbits();
    if constexpr (K < o.cnt[E]) {
        constexpr int a = o.m[E][K].a, b = o.m[E][K].b, sg = o.m[E][K].s;
        if constexpr (sg > 0) cfma(yv[a], u, xv[b]);
        else cfma(yv[a], mk<R>(-u.x, -u.y), xv[b]);
        orbit_member<R, E, K + 1>(yv, xv, u);
    }
}

template <typename R, int E>
__device__ __forceinline__ void block_product(C<R>* yv, const C<R>* xv, const C<R>* __restrict__ Urow, long long ue,
                                              int ox) {
    if constexpr (E < 60) {
        orbit_member<R, E, 0>(yv, xv, Urow[E * ue + ox]);
        block_product<R, E + 1>(yv, xv, Urow, ue, ox);
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_p3(C<R>* __restrict__ A, const C<R>* __restrict__ U, P3Params p,
                                            const C<R>* __restrict__ tw) {
    extern __shared__ unsigned char smem_raw[];
    C<R>* buf0 = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf1 = buf0 + 12 * p.pitch;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int Mx = p.plan.n;
    const int row = blockIdx.x;            // octant row (oz, oy)
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    const C<R>* Urow = U + (long long)(oz * p.Oy + oy) * p.Ox;
    for (int r = 0; r < p.nrhs; ++r)
        for (int sz = 0; sz < nz_sib; ++sz)
            for (int sy = 0; sy < ny_sib; ++sy) {
                const int z = sz ? p.Mz - oz : oz;
                const int y = sy ? p.My - oy : oy;
                C<R>* base = A + (long long)r * 12 * p.s_b + z * p.s_z + y * p.s_y;
                for (int idx = tid; idx < 12 * Mx; idx += nthr) {
                    const int c = idx / Mx, k = idx - c * Mx;
                    buf0[c * p.pitch + k] = k < p.Nx ? base[c * p.s_b + k] : mk<R>(0, 0);
                }
                __syncthreads();
                C<R>* X = fft_lds<R, true, true>(buf0, buf1, p.plan, 12, p.pitch, 1, tw, tid, nthr);
                C<R>* Y = (X == buf0) ? buf1 : buf0;
                for (int xi = tid; xi < Mx; xi += nthr) {
                    const int fx = 2 * xi > Mx;
                    const int ox = fx ? Mx - xi : xi;
                    const unsigned mask = fold_mask(fx, sy, sz);
                    C<R> xv[12], yv[12];
#pragma unroll
                    for (int a = 0; a < 12; ++a) {
                        C<R> v = X[a * p.pitch + xi];
                        if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                        xv[a] = v;
                        yv[a] = mk<R>(0, 0);
                    }
                    block_product<R, 0>(yv, xv, Urow, p.u_e, ox);
#pragma unroll
                    for (int a = 0; a < 12; ++a) {
                        C<R> v = yv[a];
                        if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                        Y[a * p.pitch + xi] = v;
                    }
                }
                __syncthreads();
                C<R>* Z = fft_lds<R, false, true>(Y, X, p.plan, 12, p.pitch, 1, tw, tid, nthr);
                for (int idx = tid; idx < 12 * p.Nx; idx += nthr) {
                    const int c = idx / p.Nx, k = idx - c * p.Nx;
                    base[c * p.s_b + k] = Z[c * p.pitch + k];
                }
                __syncthreads();
            }
}

// ---------------------------------------------------------------------------
// contiguous full-length FFT of rows (operator set-up)
// ---------------------------------------------------------------------------
template <typename R, bool FWD>
__global__ void __launch_bounds__(256) k_rows(C<R>* __restrict__ data, long long nrows, int rows_per_block,
                                              FftPlan plan, int pitch, const C<R>* __restrict__ tw) {
    extern __shared__ unsigned char smem_raw[];
    C<R>* buf0 = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf1 = buf0 + rows_per_block * pitch;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int n = plan.n;
    const long long r0 = (long long)blockIdx.x * rows_per_block;
    const int nr = (int)min((long long)rows_per_block, nrows - r0);
    for (int idx = tid; idx < rows_per_block * n; idx += nthr) {
        const int rr = idx / n, k = idx - rr * n;
        buf0[rr * pitch + k] = rr < nr ? data[(r0 + rr) * n + k] : mk<R>(0, 0);
    }
    __syncthreads();
    C<R>* res = fft_lds<R, FWD, true>(buf0, buf1, plan, rows_per_block, pitch, 1, tw, tid, nthr);
    for (int idx = tid; idx < nr * n; idx += nthr) {
        const int rr = idx / n, k = idx - rr * n;
        data[(r0 + rr) * n + k] = res[rr * pitch + k];
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename R, bool FWD, bool EPI>
static void launch_strided_t(const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2, long long n_o1,
                             const C<R>* tw, const Epilogue<R>& ep, hipStream_t s) {
    dim3 grid((p.n_inner + p.tile - 1) / p.tile, (unsigned)n_o2, (unsigned)n_o1);
    size_t lds = 2 * (size_t)p.plan.n * p.pitch * sizeof(C<R>);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_strided<R, FWD, EPI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((k_strided<R, FWD, EPI>), grid, dim3(256), lds, s, in, out, p, tw, ep);
    VIE_HIP(hipGetLastError());
}

template <typename R>
void launch_strided(bool fwd, const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2, long long n_o1,
                    const C<R>* tw, const Epilogue<R>* ep, hipStream_t s) {
    Epilogue<R> none{};
    if (ep) {
        if (fwd) throw Error(-1, "epilogue only on the inverse pass");
        launch_strided_t<R, false, true>(in, out, p, n_o2, n_o1, tw, *ep, s);
    } else if (fwd) {
        launch_strided_t<R, true, false>(in, out, p, n_o2, n_o1, tw, none, s);
    } else {
        launch_strided_t<R, false, false>(in, out, p, n_o2, n_o1, tw, none, s);
    }
}

template <typename R>
void launch_p3(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    size_t lds = 2 * 12 * (size_t)p.pitch * sizeof(C<R>);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_p3<R>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((k_p3<R>), dim3(p.Oy * p.Oz), dim3(256), lds, s, A, U, p, tw);
    VIE_HIP(hipGetLastError());
}

template <typename R>
void launch_rows(bool fwd, C<R>* data, long long nrows, const FftPlan& plan, const C<R>* tw, hipStream_t s) {
    int rpb = std::max(1, std::min(16, 2048 / plan.n));
    int pitch = plan.n;
    size_t lds = 2 * (size_t)rpb * pitch * sizeof(C<R>);
    dim3 grid((unsigned)((nrows + rpb - 1) / rpb));
    if (fwd) hipLaunchKernelGGL((k_rows<R, true>), grid, dim3(256), lds, s, data, nrows, rpb, plan, pitch, tw);
    else hipLaunchKernelGGL((k_rows<R, false>), grid, dim3(256), lds, s, data, nrows, rpb, plan, pitch, tw);
    VIE_HIP(hipGetLastError());
}

template void launch_strided<float>(bool, const C<float>*, C<float>*, const StridedPass&, long long, long long,
                                    const C<float>*, const Epilogue<float>*, hipStream_t);
template void launch_strided<double>(bool, const C<double>*, C<double>*, const StridedPass&, long long, long long,
                                     const C<double>*, const Epilogue<double>*, hipStream_t);
template void launch_p3<float>(C<float>*, const C<float>*, const P3Params&, const C<float>*, hipStream_t);
template void launch_p3<double>(C<double>*, const C<double>*, const P3Params&, const C<double>*, hipStream_t);
template void launch_rows<double>(bool, C<double>*, long long, const FftPlan&, const C<double>*, hipStream_t);

}  // namespace vie
