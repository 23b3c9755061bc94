// FFT-matvec passes (Sec. IV-A): strided zero-padded FFT passes along z and
// y, the fused x pass with the per-frequency block product, and the epilogue
// that crops and applies contrast / Gram scaling (Sec. IV-B).
#include <mutex>
#include "kernels.hpp"
#include "passes.hpp"
#include "fft_ct.hpp"

namespace vie {

thread_local LaunchTiming g_launch_timing;

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
    const long long o2 = blockIdx.y;
    const int o1 = blockIdx.z, rr = o1 / p.nc, cc = o1 - p.nc * rr;
    const int tw_n = min(p.tile, p.n_inner - t0);
    const C<R>* src = in + rr * p.in_s1 + cc * p.in_sc + o2 * p.in_s2 + t0;
    const int n = p.plan.n;
    // load (zero-padded beyond n_in and beyond the inner extent)
    for (int idx = tid; idx < n * p.tile; idx += nthr) {
        const int k = idx / p.tile, t = idx - k * p.tile;
        C<R> v = mk<R>(0, 0);
        if (k < p.n_in && t < tw_n) v = stream_load(&src[k * p.in_sk + t]);
        buf0[k * p.pitch + t] = v;
    }
    __syncthreads();
    C<R>* res = fft_lds<R, FWD, false>(buf0, buf1, p.plan, p.tile, 1, p.pitch, tw, tid, nthr);
    const long long obase = rr * p.out_s1 + cc * p.out_sc;
    C<R>* dst = out + obase + o2 * p.out_s2 + t0;
    for (int idx = tid; idx < p.n_out * p.tile; idx += nthr) {
        const int k = idx / p.tile, t = idx - k * p.tile;
        if (t >= tw_n) continue;
        C<R> w = res[k * p.pitch + t];
        if (EPI) {
            const long long v = o2 * p.out_s2 + k * p.out_sk + t0 + t;   // voxel
            const long long e = obase + v;                                  // element
            const int l = p.nc == 12 ? (cc & 3) : 0;
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

// y += sum_b sign(A, b) U[unique(A, b)] x[b] for one output row A; the
// unique index and sign are compile-time constants
template <typename R, int A, int B>
__device__ __forceinline__ void row_dot(C<R>& y, const C<R>* xv, const C<R>* Urow, long long ue, int ox) {
    constexpr int e = unique_index(A, B);
    constexpr int sg = unique_sign(A, B);
    const C<R> u = Urow[e * ue + ox];
    if constexpr (sg > 0) cfma(y, u, xv[B]);
    else cfma(y, mk<R>(-u.x, -u.y), xv[B]);
    if constexpr (B + 1 < 12) row_dot<R, A, B + 1>(y, xv, Urow, ue, ox);
}

// the same row of the curl operator's block (30 unique tensors; the
// entries with p = q are zero and skipped)
template <typename R, int A, int B>
__device__ __forceinline__ void row_dot_curl(C<R>& y, const C<R>* xv, const C<R>* Urow, long long ue, int ox) {
    constexpr int e = curl_unique_index(A, B);
    constexpr int sg = curl_unique_sign(A, B);
    if constexpr (sg != 0) {
        const C<R> u = Urow[e * ue + ox];
        if constexpr (sg > 0) cfma(y, u, xv[B]);
        else cfma(y, mk<R>(-u.x, -u.y), xv[B]);
    }
    if constexpr (B + 1 < 12) row_dot_curl<R, A, B + 1>(y, xv, Urow, ue, ox);
}

// rows [A, AEND) of the 12 x 12 block product into yv[A - A0]
template <typename R, bool CURL, int A0, int A, int AEND>
__device__ __forceinline__ void rows_product(C<R>* yv, const C<R>* xv, const C<R>* Urow, long long ue, int ox) {
    if constexpr (A < AEND) {
        C<R> y = mk<R>(0, 0);
        if constexpr (CURL) row_dot_curl<R, A, 0>(y, xv, Urow, ue, ox);
        else row_dot<R, A, 0>(y, xv, Urow, ue, ox);
        yv[A - A0] = y;
        rows_product<R, CURL, A0, A + 1, AEND>(yv, xv, Urow, ue, ox);
    }
}

// rows [6 h, 6 h + 6) (split 2) or [3 h, 3 h + 3) (split 4)
template <typename R, int SPLIT, bool CURL = false>
__device__ __forceinline__ void part_product(int h, C<R>* yv, const C<R>* xv, const C<R>* Urow, long long ue,
                                             int ox) {
    if constexpr (SPLIT == 2) {
        if (h == 0) rows_product<R, CURL, 0, 0, 6>(yv, xv, Urow, ue, ox);
        else rows_product<R, CURL, 6, 6, 12>(yv, xv, Urow, ue, ox);
    } else {
        if (h == 0) rows_product<R, CURL, 0, 0, 3>(yv, xv, Urow, ue, ox);
        else if (h == 1) rows_product<R, CURL, 3, 3, 6>(yv, xv, Urow, ue, ox);
        else if (h == 2) rows_product<R, CURL, 6, 6, 9>(yv, xv, Urow, ue, ox);
        else rows_product<R, CURL, 9, 9, 12>(yv, xv, Urow, ue, ox);
    }
}

// One workgroup per octant row (xi_z', xi_y'): the up to four pencils
// (+-xi_y, +-xi_z) that share it, for every right-hand side.  The operator
// row (NE unique entries x Ox frequencies) is staged in LDS once.  `groups`
// pencil groups (12 component rows each) then go through LDS together:
// load (zero-padded from Nx to Mx), forward FFT in place, block product per
// frequency (SPLIT threads per column, each a slice of the 12 output rows),
// inverse FFT, store the first Nx.  CURL selects the curl operator (30
// unique tensors); its spectrum changes sign under each octant fold on top
// of the component signs (the curl is odd under reflection).
template <typename R, int SPLIT, bool CURL = false>
__global__ void __launch_bounds__(p3_threads<R>()) k_p3(C<R>* __restrict__ A, const C<R>* __restrict__ U,
                                                        P3Params p, const C<R>* __restrict__ tw) {
    constexpr int NE = CURL ? 30 : 60;
    extern __shared__ unsigned char smem_raw[];
    C<R>* Ul = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf = Ul + NE * p.Ox;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int Mx = p.plan.n;
    const int row = blockIdx.x;
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    const int nsib = ny_sib * nz_sib;
    const int nwork = nsib * p.nrhs;
    {
        const C<R>* Urow = U + (long long)(oz * p.Oy + oy) * NE * p.Ox;
        for (int idx = tid; idx < NE * p.Ox; idx += nthr) {
            const int e = idx / p.Ox, ox = idx - e * p.Ox;
            Ul[idx] = Urow[e * p.u_e + ox];
        }
    }
    constexpr int RP = 12 / SPLIT;   // output rows per thread
    for (int w0 = 0; w0 < nwork; w0 += p.groups) {
        const int G = min(p.groups, nwork - w0);
        for (int idx = tid; idx < G * 12 * Mx; idx += nthr) {
            const int g = idx / (12 * Mx), rem = idx - g * 12 * Mx;
            const int c = rem / Mx, k = rem - c * Mx;
            const int wk = w0 + g, r = wk / nsib, sib = wk - r * nsib;
            const int z = (sib / ny_sib) ? p.Mz - oz : oz;
            const int y = (sib % ny_sib) ? p.My - oy : oy;
            C<R> v = mk<R>(0, 0);
            if (k < p.Nx) v = A[(long long)r * p.s_r + c * p.s_c + z * p.s_z + y * p.s_y + k];
            buf[lds_pad((g * 12 + c) * p.pitch + k)] = v;
        }
        __syncthreads();
        fft_rows_inplace<R, true>(buf, p.plan, G * 12, p.pitch, tw, tid, nthr);
        {
            const int ncol = G * Mx;
            const bool act = tid < SPLIT * ncol;
            const int h = tid / ncol, col = tid - h * ncol;
            const int g = col / Mx, xi = col - g * Mx;
            C<R> xv[12], yv[RP];
            unsigned mask = 0, omask = 0;
            int ox = 0;
            if (act) {
                const int wk = w0 + g, sib = wk % nsib;
                const int sz = sib / ny_sib, sy = sib % ny_sib;
                const int fx = 2 * xi > Mx;
                ox = fx ? Mx - xi : xi;
                mask = fold_mask(fx, sy, sz);
                omask = (CURL && ((fx + sy + sz) & 1)) ? (mask ^ 0xFFFu) : mask;
#pragma unroll
                for (int a = 0; a < 12; ++a) {
                    C<R> v = buf[lds_pad((g * 12 + a) * p.pitch + xi)];
                    if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                    xv[a] = v;
                }
            }
            __syncthreads();
            if (act) {
                part_product<R, SPLIT, CURL>(h, yv, xv, Ul, p.Ox, ox);
#pragma unroll
                for (int i = 0; i < RP; ++i) {
                    const int a = RP * h + i;
                    C<R> v = yv[i];
                    if (omask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                    buf[lds_pad((g * 12 + a) * p.pitch + xi)] = v;
                }
            }
        }
        __syncthreads();
        fft_rows_inplace<R, false>(buf, p.plan, G * 12, p.pitch, tw, tid, nthr);
        for (int idx = tid; idx < G * 12 * p.Nx; idx += nthr) {
            const int g = idx / (12 * p.Nx), rem = idx - g * 12 * p.Nx;
            const int c = rem / p.Nx, k = rem - c * p.Nx;
            const int wk = w0 + g, r = wk / nsib, sib = wk - r * nsib;
            const int z = (sib / ny_sib) ? p.Mz - oz : oz;
            const int y = (sib % ny_sib) ? p.My - oy : oy;
            A[(long long)r * p.s_r + c * p.s_c + z * p.s_z + y * p.s_y + k] = buf[lds_pad((g * 12 + c) * p.pitch + k)];
        }
        __syncthreads();
    }
}

// Same x pass for compile-time FFT lengths N: the operator row and the
// twiddle table are staged in LDS once, global gathers and scatters keep up
// to eight loads in flight per thread (fast division by Nx), and the FFT
// passes unroll completely.
template <typename R, int N>
__global__ void __launch_bounds__(p3_threads<R>()) k_p3_ct(C<R>* __restrict__ A, const C<R>* __restrict__ U,
                                                           P3Params p, const C<R>* __restrict__ tw) {
    constexpr int NT = p3_threads<R>();
    constexpr int GMAX = p3_gmax(sizeof(C<R>), N, NT);
    constexpr int MAXROWS = 12 * GMAX;
    constexpr int OX = N / 2 + 1;
    constexpr int SPLIT = (4 * GMAX * N <= NT) ? 4 : 2;
    constexpr int RP = 12 / SPLIT;
    extern __shared__ unsigned char smem_raw[];
    C<R>* Ul = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* twl = Ul + 60 * OX;
    C<R>* buf = twl + N;
    __shared__ long long rowoff[MAXROWS];
    const int tid = threadIdx.x;
    const int row = blockIdx.x / p.sib_blocks, sb = blockIdx.x - row * p.sib_blocks;
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    const int nsib = ny_sib * nz_sib;
    // this workgroup's siblings: sb, sb + sib_blocks, ... (< nsib)
    const int my_nsib = sb < nsib ? (nsib - sb + p.sib_blocks - 1) / p.sib_blocks : 0;
    if (my_nsib == 0) return;   // uniform over the workgroup
    const int nwork = my_nsib * p.nrhs;
    {
        const C<R>* Urow = U + (long long)(oz * p.Oy + oy) * 60 * OX;
        constexpr int TOT = 60 * OX;
        for (int b0 = 0; b0 < TOT; b0 += 8 * NT) {
            C<R> v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = b0 + tid + i * NT;
                if (e < TOT) v[i] = Urow[e];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = b0 + tid + i * NT;
                if (e < TOT) Ul[e] = v[i];
            }
        }
        for (int m = tid; m < N; m += NT) twl[m] = tw[m];
    }
    for (int w0 = 0; w0 < nwork; w0 += p.groups) {
        const int G = min(p.groups, nwork - w0);
        const int rows = 12 * G;
        if (tid < rows) {
            const int g = tid / 12, c = tid - 12 * g;
            const int wk = w0 + g, r = wk / my_nsib, sib = sb + (wk - r * my_nsib) * p.sib_blocks;
            const int z = (sib / ny_sib) ? p.Mz - oz : oz;
            const int y = (sib % ny_sib) ? p.My - oy : oy;
            rowoff[tid] = (long long)r * p.s_r + (long long)c * p.s_c + (long long)z * p.s_z + (long long)y * p.s_y;
        }
        __syncthreads();
        // gather rows x Nx, zero the padding
        const int tot = rows * p.Nx;
        for (int b0 = 0; b0 < tot; b0 += 8 * NT) {
            C<R> v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = b0 + tid + i * NT;
                if (e < tot) {
                    const int rr = fast_div((unsigned)e, p.magic_nx), k = e - rr * p.Nx;
                    v[i] = A[rowoff[rr] + k];
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = b0 + tid + i * NT;
                if (e < tot) {
                    const int rr = fast_div((unsigned)e, p.magic_nx), k = e - rr * p.Nx;
                    buf[lds_pad(rr * N + k)] = v[i];
                }
            }
        }
        for (int e = tid; e < rows * N; e += NT) {
            const int rr = e / N, k = e - rr * N;
            if (k >= p.Nx) buf[lds_pad(e)] = mk<R>(0, 0);
        }
        __syncthreads();
        ct_passes<R, true, N, 0, 1, NT, MAXROWS, true>(buf, twl, rows, N, tid);   // Nx <= N / 2
        {
            const int ncol = G * N;
            const bool act = tid < SPLIT * ncol;
            const int h = tid / ncol, col = tid - h * ncol;
            const int g = col / N, xi = col - g * N;
            C<R> xv[12], yv[RP];
            unsigned mask = 0;
            int ox = 0;
            if (act) {
                const int wk = w0 + g, sib = sb + (wk % my_nsib) * p.sib_blocks;
                const int sz = sib / ny_sib, sy = sib % ny_sib;
                const int fx = 2 * xi > N;
                ox = fx ? N - xi : xi;
                mask = fold_mask(fx, sy, sz);
#pragma unroll
                for (int a = 0; a < 12; ++a) {
                    C<R> v = buf[lds_pad((g * 12 + a) * N + xi)];
                    if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                    xv[a] = v;
                }
            }
            __syncthreads();
            if (act) {
                part_product<R, SPLIT>(h, yv, xv, Ul, OX, ox);
#pragma unroll
                for (int i = 0; i < RP; ++i) {
                    const int a = RP * h + i;
                    C<R> v = yv[i];
                    if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                    buf[lds_pad((g * 12 + a) * N + xi)] = v;
                }
            }
        }
        __syncthreads();
        ct_passes<R, false, N, 0, 1, NT, MAXROWS, false, true>(buf, twl, rows, N, tid);   // crop to Nx
        for (int b0 = 0; b0 < tot; b0 += 8 * NT) {
            C<R> v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = b0 + tid + i * NT;
                if (e < tot) {
                    const int rr = fast_div((unsigned)e, p.magic_nx), k = e - rr * p.Nx;
                    v[i] = buf[lds_pad(rr * N + k)];
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = b0 + tid + i * NT;
                if (e < tot) {
                    const int rr = fast_div((unsigned)e, p.magic_nx), k = e - rr * p.Nx;
                    A[rowoff[rr] + k] = v[i];
                }
            }
        }
        __syncthreads();
    }
}

// Row copies between global memory and LDS for the x pass: one wavefront per
// row (the row address is uniform over the wave), four rows in flight per
// wave.  Row i holds Nx contiguous elements at rowp(i); in LDS it is padded
// with zeros to N.
template <typename R, int N, int NT, typename RowPtr>
__device__ __forceinline__ void rows_to_lds(C<R>* buf, int nrows, int Nx, RowPtr rowp) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int i0 = wave; i0 < nrows; i0 += 4 * NW) {
        const C<R>* src[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) src[u] = rowp(min(i0 + u * NW, nrows - 1));
        for (int k = lane; k < N; k += 64) {
            C<R> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = (i0 + u * NW < nrows && k < Nx) ? src[u][k] : mk<R>(0, 0);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i0 + u * NW < nrows) buf[lds_pad((i0 + u * NW) * N + k)] = v[u];
        }
    }
}

template <typename R, int N, int NT, typename RowPtr>
__device__ __forceinline__ void lds_to_rows(const C<R>* buf, int nrows, int Nx, RowPtr rowp) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int i0 = wave; i0 < nrows; i0 += 4 * NW) {
        C<R>* dst[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[u] = rowp(min(i0 + u * NW, nrows - 1));
        for (int k = lane; k < Nx; k += 64) {
            C<R> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = buf[lds_pad(min(i0 + u * NW, nrows - 1) * N + k)];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i0 + u * NW < nrows) dst[u][k] = v[u];
        }
    }
}

// Light variant of the x pass: one workgroup of 256 threads per pencil group
// (one right-hand side, one of the up to four sibling pencils of an octant
// row), 12 rows of N in LDS and nothing else, so that many workgroups share a
// CU.  The block product runs one thread per frequency in the orbit form: each
// of the 60 unique operator values is read once (from L2: the four siblings
// of a row read the same values) and applied to the up to four positions it
// fills.
constexpr int kP3SmallThreads = 256;

template <typename R, int E, int K>
__device__ __forceinline__ void orbit_apply(C<R>* yv, const C<R>* xv, C<R> u) {
    constexpr Orbits o = make_orbits();
    if constexpr (K < o.cnt[E]) {
        constexpr int a = o.m[E][K].a, b = o.m[E][K].b, sg = o.m[E][K].s;
        if constexpr (sg > 0) cfma(yv[a], u, xv[b]);
        else cfma(yv[a], mk<R>(-u.x, -u.y), xv[b]);
        orbit_apply<R, E, K + 1>(yv, xv, u);
    }
}

template <typename R, int E, int EEND = 60>
__device__ __forceinline__ void orbit_product(C<R>* yv, const C<R>* xv, const C<R>* __restrict__ Ur, int ox, int OXs) {
    if constexpr (E < EEND) {
        orbit_apply<R, E, 0>(yv, xv, Ur[E * OXs + ox]);
        orbit_product<R, E + 1, EEND>(yv, xv, Ur, ox, OXs);
    }
}

template <typename R, int N, int SPLIT>
__global__ void __launch_bounds__(kP3SmallThreads) k_p3_small(C<R>* __restrict__ A, const C<R>* __restrict__ U,
                                                              P3Params p, const C<R>* __restrict__ tw) {
    constexpr int NT = kP3SmallThreads;
    constexpr int OX = N / 2 + 1;
    extern __shared__ unsigned char smem_raw[];
    C<R>* twl = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf = twl + N;
    const int tid = threadIdx.x;
    // block -> (octant row, right-hand side, sibling).  Workgroups are dealt
    // to the 8 XCDs round-robin by index, so the 4 * nrhs workgroups that read
    // one operator row get indices congruent modulo 8: they run on one XCD
    // and share its L2.
    const int K = 4 * p.nrhs;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int row = (q / K) * 8 + xcd;
    if (row >= p.Oy * p.Oz) return;       // padding rows, uniform over the workgroup
    const int kk = q - (q / K) * K;
    const int r = kk >> 2, sib = kk & 3;
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    if (sib >= ny_sib * nz_sib) return;   // uniform over the workgroup
    const int sz = sib / ny_sib, sy = sib - sz * ny_sib;
    const int z = sz ? p.Mz - oz : oz;
    const int y = sy ? p.My - oy : oy;
    C<R>* base = A + (long long)r * p.s_r + (long long)z * p.s_z + (long long)y * p.s_y;   // 12 rows of Nx, stride s_c
    const long long s_c = p.s_c;
    auto rowp = [=](int c) { return base + c * s_c; };
    for (int m = tid; m < N; m += NT) twl[m] = tw[m];
    rows_to_lds<R, N, NT>(buf, 12, p.Nx, rowp);
    __syncthreads();
    ct_passes<R, true, N, 0, 1, NT, 12, true>(buf, twl, 12, N, tid);   // Nx <= N / 2
    const C<R>* Ur = U + (long long)row * 60 * OX;
    if constexpr (SPLIT == 1) {
        for (int xi = tid; xi < N; xi += NT) {
            const int fx = 2 * xi > N;
            const int ox = fx ? N - xi : xi;
            const unsigned mask = fold_mask(fx, sy, sz);
            C<R> xv[12], yv[12];
#pragma unroll
            for (int a = 0; a < 12; ++a) {
                C<R> v = buf[lds_pad(a * N + xi)];
                if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                xv[a] = v;
                yv[a] = mk<R>(0, 0);
            }
            orbit_product<R, 0>(yv, xv, Ur, ox, OX);
#pragma unroll
            for (int a = 0; a < 12; ++a) {
                C<R> v = yv[a];
                if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                buf[lds_pad(a * N + xi)] = v;   // own column: in place
            }
        }
    } else {
        // two threads per frequency column, each summing half of the 60
        // unique entries; the second half's partial sums pass through the
        // column's LDS slots.  Every thread runs every round (barriers).
        constexpr int HALF = NT / 2;
        const int h = tid / HALF;
        for (int c0 = 0; c0 < N; c0 += HALF) {
            const int xi = c0 + (tid - h * HALF);
            const bool act = xi < N;
            const int fx = 2 * xi > N;
            const int ox = fx ? N - xi : xi;
            const unsigned mask = fold_mask(fx, sy, sz);
            C<R> xv[12], yv[12];
            if (act) {
#pragma unroll
                for (int a = 0; a < 12; ++a) {
                    C<R> v = buf[lds_pad(a * N + xi)];
                    if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                    xv[a] = v;
                    yv[a] = mk<R>(0, 0);
                }
                if (h == 0) orbit_product<R, 0, 30>(yv, xv, Ur, ox, OX);
                else orbit_product<R, 30, 60>(yv, xv, Ur, ox, OX);
            }
            __syncthreads();   // the column's inputs are read by both halves
            if (act && h == 1) {
#pragma unroll
                for (int a = 0; a < 12; ++a) buf[lds_pad(a * N + xi)] = yv[a];
            }
            __syncthreads();
            if (act && h == 0) {
#pragma unroll
                for (int a = 0; a < 12; ++a) {
                    const C<R> o = buf[lds_pad(a * N + xi)];
                    C<R> v = mk<R>(yv[a].x + o.x, yv[a].y + o.y);
                    if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                    buf[lds_pad(a * N + xi)] = v;
                }
            }
        }
    }
    __syncthreads();
    ct_passes<R, false, N, 0, 1, NT, 12, false, true>(buf, twl, 12, N, tid);   // crop to Nx
    lds_to_rows<R, N, NT>(buf, 12, p.Nx, rowp);
}

// Right-hand-side pairs (variant 5, for batches): as the light variant, but
// a workgroup holds the pencils of two right-hand sides (the same sibling of
// the same octant row, 24 rows in LDS; the last of an odd batch holds one)
// and runs two work items per frequency, one per right-hand side.  The two
// items of a frequency sit in neighbouring lanes and read the same operator
// values in one load instruction, so the operator is read from L2 half as
// often as by the light variant, and every thread works in the product.
template <typename R, int N>
__global__ void __launch_bounds__(kP3SmallThreads) k_p3_pair(C<R>* __restrict__ A, const C<R>* __restrict__ U,
                                                             P3Params p, const C<R>* __restrict__ tw) {
    constexpr int NT = kP3SmallThreads;
    constexpr int OX = N / 2 + 1;
    extern __shared__ unsigned char smem_raw[];
    C<R>* twl = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf = twl + N;
    const int tid = threadIdx.x;
    // block -> (octant row, right-hand-side pair, sibling); the 4 npairs
    // workgroups of one operator row get indices congruent modulo 8
    const int npairs = (p.nrhs + 1) >> 1;
    const int K = 4 * npairs;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int row = (q / K) * 8 + xcd;
    if (row >= p.Oy * p.Oz) return;       // padding rows, uniform over the workgroup
    const int kk = q - (q / K) * K;
    const int pr = kk >> 2, sib = kk & 3;
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    if (sib >= ny_sib * nz_sib) return;   // uniform over the workgroup
    const int sz = sib / ny_sib, sy = sib - sz * ny_sib;
    const int z = sz ? p.Mz - oz : oz;
    const int y = sy ? p.My - oy : oy;
    const int nr = min(2, p.nrhs - 2 * pr);   // right-hand sides held (1 or 2)
    C<R>* base = A + (long long)(2 * pr) * p.s_r + (long long)z * p.s_z + (long long)y * p.s_y;
    const long long s_c = p.s_c, s_r = p.s_r;
    auto rowp = [=](int rr) {   // LDS row h * 12 + c: right-hand side 2 pr + h, component c
        const int h = rr >= 12, c = rr - 12 * h;
        return base + h * s_r + c * s_c;
    };
    for (int m = tid; m < N; m += NT) twl[m] = tw[m];
    rows_to_lds<R, N, NT>(buf, 12 * nr, p.Nx, rowp);
    __syncthreads();
    ct_passes<R, true, N, 0, 1, NT, 24, true>(buf, twl, 12 * nr, N, tid);   // Nx <= N / 2
    {
        const C<R>* Ur = U + (long long)row * 60 * OX;
        // each item reads and writes only its own rows of its own column
        for (int w = tid; w < 2 * N; w += NT) {
            const int xi = w >> 1, h = w & 1;
            if (h >= nr) continue;
            const int fx = 2 * xi > N;
            const int ox = fx ? N - xi : xi;
            const unsigned mask = fold_mask(fx, sy, sz);
            C<R> xv[12], yv[12];
#pragma unroll
            for (int a = 0; a < 12; ++a) {
                C<R> v = buf[lds_pad((12 * h + a) * N + xi)];
                if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                xv[a] = v;
                yv[a] = mk<R>(0, 0);
            }
            orbit_product<R, 0>(yv, xv, Ur, ox, OX);
#pragma unroll
            for (int a = 0; a < 12; ++a) {
                C<R> v = yv[a];
                if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
                buf[lds_pad((12 * h + a) * N + xi)] = v;
            }
        }
    }
    __syncthreads();
    ct_passes<R, false, N, 0, 1, NT, 24, false, true>(buf, twl, 12 * nr, N, tid);   // crop to Nx
    lds_to_rows<R, N, NT>(buf, 12 * nr, p.Nx, rowp);
}

// Prefetching variant of the light x pass (fft lengths up to 128): as the
// light variant, but the workgroup first issues the loads of its operator row
// (60 Ox values, contiguous) into registers, so that they are in flight
// during the gather and the forward FFT, then parks the row in LDS; the block
// product reads the operator from LDS.
template <typename R, int E>
__device__ __forceinline__ void orbit_product_lds(C<R>* yv, const C<R>* xv, const C<R>* Ul, int ox, int OXs) {
    if constexpr (E < 60) {
        orbit_apply<R, E, 0>(yv, xv, Ul[E * OXs + ox]);
        orbit_product_lds<R, E + 1>(yv, xv, Ul, ox, OXs);
    }
}

template <typename R, int N>
__global__ void __launch_bounds__(kP3SmallThreads) k_p3_pref(C<R>* __restrict__ A, const C<R>* __restrict__ U,
                                                             P3Params p, const C<R>* __restrict__ tw) {
    constexpr int NT = kP3SmallThreads;
    constexpr int OX = N / 2 + 1;
    constexpr int UN = 60 * OX;
    constexpr int UPT = (UN + NT - 1) / NT;   // operator values per thread
    extern __shared__ unsigned char smem_raw[];
    C<R>* twl = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* Ul = twl + N;
    C<R>* buf = Ul + UN;
    const int tid = threadIdx.x;
    const int K = 4 * p.nrhs;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int row = (q / K) * 8 + xcd;
    if (row >= p.Oy * p.Oz) return;       // padding rows, uniform over the workgroup
    const int kk = q - (q / K) * K;
    const int r = kk >> 2, sib = kk & 3;
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    if (sib >= ny_sib * nz_sib) return;   // uniform over the workgroup
    const int sz = sib / ny_sib, sy = sib - sz * ny_sib;
    const int z = sz ? p.Mz - oz : oz;
    const int y = sy ? p.My - oy : oy;
    C<R>* base = A + (long long)r * p.s_r + (long long)z * p.s_z + (long long)y * p.s_y;
    const long long s_c = p.s_c;
    auto rowp = [=](int c) { return base + c * s_c; };
    const C<R>* Ur = U + (long long)row * UN;
    C<R> upre[UPT];
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
        const int idx = tid + i * NT;
        if (idx < UN) upre[i] = Ur[idx];
    }
    for (int m = tid; m < N; m += NT) twl[m] = tw[m];
    rows_to_lds<R, N, NT>(buf, 12, p.Nx, rowp);
    __syncthreads();
    ct_passes<R, true, N, 0, 1, NT, 12, true>(buf, twl, 12, N, tid);   // Nx <= N / 2
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
        const int idx = tid + i * NT;
        if (idx < UN) Ul[idx] = upre[i];
    }
    __syncthreads();
    for (int xi = tid; xi < N; xi += NT) {
        const int fx = 2 * xi > N;
        const int ox = fx ? N - xi : xi;
        const unsigned mask = fold_mask(fx, sy, sz);
        C<R> xv[12], yv[12];
#pragma unroll
        for (int a = 0; a < 12; ++a) {
            C<R> v = buf[lds_pad(a * N + xi)];
            if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
            xv[a] = v;
            yv[a] = mk<R>(0, 0);
        }
        orbit_product_lds<R, 0>(yv, xv, Ul, ox, OX);
#pragma unroll
        for (int a = 0; a < 12; ++a) {
            C<R> v = yv[a];
            if (mask & (1u << a)) { v.x = -v.x; v.y = -v.y; }
            buf[lds_pad(a * N + xi)] = v;
        }
    }
    __syncthreads();
    ct_passes<R, false, N, 0, 1, NT, 12, false, true>(buf, twl, 12, N, tid);   // crop to Nx
    lds_to_rows<R, N, NT>(buf, 12, p.Nx, rowp);
}

// Sibling-sharing variant of the x pass: one workgroup of 256 threads per
// (octant row, right-hand side) holding the up to four sibling pencil groups
// (+-xi_y, +-xi_z) of the row in LDS.  The block product runs one work item
// per (frequency, z sibling) that serves both y siblings at once: each of the
// 60 unique operator values is read once and applied to the two vectors, so
// a row's operator values are read half as often as with one workgroup per
// sibling, and every thread has a column to work on.
template <typename R, int E, int K>
__device__ __forceinline__ void orbit_apply2(C<R>* y0, C<R>* y1, const C<R>* x0, const C<R>* x1, C<R> u) {
    constexpr Orbits o = make_orbits();
    if constexpr (K < o.cnt[E]) {
        constexpr int a = o.m[E][K].a, b = o.m[E][K].b, sg = o.m[E][K].s;
        const C<R> us = sg > 0 ? u : mk<R>(-u.x, -u.y);
        cfma(y0[a], us, x0[b]);
        cfma(y1[a], us, x1[b]);
        orbit_apply2<R, E, K + 1>(y0, y1, x0, x1, u);
    }
}

template <typename R, int E, int EEND = 60>
__device__ __forceinline__ void orbit_product2(C<R>* y0, C<R>* y1, const C<R>* x0, const C<R>* x1,
                                               const C<R>* __restrict__ Ur, int ox, int OXs) {
    if constexpr (E < EEND) {
        orbit_apply2<R, E, 0>(y0, y1, x0, x1, Ur[E * OXs + ox]);
        orbit_product2<R, E + 1, EEND>(y0, y1, x0, x1, Ur, ox, OXs);
    }
}

constexpr int kP3QuadThreads = 256;

template <typename R, int N>
__global__ void __launch_bounds__(kP3QuadThreads) k_p3_quad(C<R>* __restrict__ A, const C<R>* __restrict__ U,
                                                            P3Params p, const C<R>* __restrict__ tw) {
    constexpr int NT = kP3QuadThreads;
    constexpr int OX = N / 2 + 1;
    extern __shared__ unsigned char smem_raw[];
    C<R>* twl = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf = twl + N;
    const int tid = threadIdx.x;
    // block -> (octant row, right-hand side); the nrhs workgroups of one row
    // get indices congruent modulo 8, so they run on one XCD and share its L2
    const int K = p.nrhs;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int row = (q / K) * 8 + xcd;
    if (row >= p.Oy * p.Oz) return;   // padding rows, uniform over the workgroup
    const int r = q - (q / K) * K;
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    const int nrows = 12 * ny_sib * nz_sib;   // LDS row s * 12 + c, sibling s = sz * ny_sib + sy
    C<R>* base = A + (long long)r * p.s_r;
    const long long s_c = p.s_c, s_y = p.s_y, s_z = p.s_z;
    const int Mz = p.Mz, My = p.My;
    auto rowp = [=](int rr) {
        const int sb = rr / 12, c = rr - 12 * sb;
        const int sz = sb >= ny_sib, sy = sb - sz * ny_sib;
        const int z = sz ? Mz - oz : oz, y = sy ? My - oy : oy;
        return base + z * s_z + y * s_y + c * s_c;
    };
    for (int m = tid; m < N; m += NT) twl[m] = tw[m];
    rows_to_lds<R, N, NT>(buf, nrows, p.Nx, rowp);
    __syncthreads();
    ct_passes<R, true, N, 0, 1, NT, 48, true>(buf, twl, nrows, N, tid);   // Nx <= N / 2
    {
        const C<R>* Ur = U + (long long)row * 60 * OX;
        // Fold signs: sibling (sy, sz) and the upper half of the x range
        // (fx) read the octant value of the mirrored frequency, D T D with
        // D = diag(+-1), applied to x and y as a flip of the sign bit.  When
        // N is a multiple of 128 a wave's 64 frequencies lie in one half of
        // the x range (with the Nyquist column counted in the upper half,
        // where the block is invariant under the x fold) and in one z
        // sibling, so the masks are wave-uniform scalars and each flip is a
        // single XOR with a scalar operand.
        constexpr bool UNIFORM = N % 128 == 0 && NT % 64 == 0;
        constexpr unsigned MX = fold_mask(1, 0, 0), MY = fold_mask(0, 1, 0), MZ = fold_mask(0, 0, 1);
        for (int w = tid; w < nz_sib * N; w += NT) {
            int sz = w >= N;
            const int xi = w - sz * N;
            int fx = UNIFORM ? (2 * xi >= N) : (2 * xi > N);
            if constexpr (UNIFORM) {
                sz = __builtin_amdgcn_readfirstlane(sz);
                fx = __builtin_amdgcn_readfirstlane(fx);
            }
            const int ox = fx ? N - xi : xi;
            const int s0 = sz * ny_sib;
            const unsigned m0 = (fx ? MX : 0u) ^ (sz ? MZ : 0u);
            auto flip = [](C<R> v, unsigned m, int a) {
                if constexpr (sizeof(R) == 4) {
                    const unsigned f = ((m >> a) & 1u) << 31;
                    v.x = __uint_as_float(__float_as_uint(v.x) ^ f);
                    v.y = __uint_as_float(__float_as_uint(v.y) ^ f);
                } else if ((m >> a) & 1u) {
                    v.x = -v.x;
                    v.y = -v.y;
                }
                return v;
            };
            if (ny_sib == 2) {
                const unsigned m1 = m0 ^ MY;
                C<R> x0[12], x1[12], y0[12], y1[12];
#pragma unroll
                for (int a = 0; a < 12; ++a) {
                    x0[a] = flip(buf[lds_pad((s0 * 12 + a) * N + xi)], m0, a);
                    x1[a] = flip(buf[lds_pad(((s0 + 1) * 12 + a) * N + xi)], m1, a);
                    y0[a] = mk<R>(0, 0);
                    y1[a] = mk<R>(0, 0);
                }
                orbit_product2<R, 0>(y0, y1, x0, x1, Ur, ox, OX);
#pragma unroll
                for (int a = 0; a < 12; ++a) {
                    buf[lds_pad((s0 * 12 + a) * N + xi)] = flip(y0[a], m0, a);
                    buf[lds_pad(((s0 + 1) * 12 + a) * N + xi)] = flip(y1[a], m1, a);
                }
            } else {
                C<R> x0[12], y0[12];
#pragma unroll
                for (int a = 0; a < 12; ++a) {
                    x0[a] = flip(buf[lds_pad((s0 * 12 + a) * N + xi)], m0, a);
                    y0[a] = mk<R>(0, 0);
                }
                orbit_product<R, 0>(y0, x0, Ur, ox, OX);
#pragma unroll
                for (int a = 0; a < 12; ++a) buf[lds_pad((s0 * 12 + a) * N + xi)] = flip(y0[a], m0, a);
            }
        }
    }
    __syncthreads();
    ct_passes<R, false, N, 0, 1, NT, 48, false, true>(buf, twl, nrows, N, tid);   // crop to Nx
    lds_to_rows<R, N, NT>(buf, nrows, p.Nx, rowp);
}

// x pass of the J-M product (24 unknowns per voxel, Sec. II eq. 15): one
// workgroup per (octant row, right-hand side, sibling) holds the 12 rows of
// the electric half x_j and the 12 of the magnetic half x_m of its pencil
// (24 rows in LDS), and per frequency forms both coupled sums
//
//   s_j = N x_j + kj K x_m,   kj = -c_e = -i w eps0
//   s_m = N x_m + km K x_j,   km = +c_m = +i w mu0
//
// two work items per frequency, one per half: the 30 curl tensors applied
// to the other half, the factor (kj or km), then the 60 N tensors applied
// to its own half.  Fold signs as in the other
// x passes: D on the inputs and outputs of both blocks, and the curl's extra
// sign (-1)^(fx + fy + fz) (odd under reflection) goes into the factors.
// The two halves of right-hand side r are the vectors 2 r and 2 r + 1 of the
// buffer (stride s_r).
struct CurlOrbits {
    OrbitMember m[30][4];
    int cnt[30];
};
constexpr CurlOrbits make_curl_orbits() {
    CurlOrbits o{};
    for (int e = 0; e < 30; ++e) o.cnt[e] = 0;
    for (int a = 0; a < 12; ++a)
        for (int b = 0; b < 12; ++b) {
            const int sg = curl_unique_sign(a, b);
            if (sg == 0) continue;
            const int e = curl_unique_index(a, b);
            o.m[e][o.cnt[e]] = OrbitMember{a, b, sg};
            o.cnt[e]++;
        }
    return o;
}

template <typename R, int E, int K>
__device__ __forceinline__ void curl_orbit_apply(C<R>* yv, const C<R>* xv, C<R> u) {
    constexpr CurlOrbits o = make_curl_orbits();
    if constexpr (K < o.cnt[E]) {
        constexpr int a = o.m[E][K].a, b = o.m[E][K].b, sg = o.m[E][K].s;
        if constexpr (sg > 0) cfma(yv[a], u, xv[b]);
        else cfma(yv[a], mk<R>(-u.x, -u.y), xv[b]);
        curl_orbit_apply<R, E, K + 1>(yv, xv, u);
    }
}

template <typename R, int E>
__device__ __forceinline__ void curl_orbit_product(C<R>* yv, const C<R>* xv, const C<R>* __restrict__ Ur, int ox,
                                                   int OXs) {
    if constexpr (E < 30) {
        curl_orbit_apply<R, E, 0>(yv, xv, Ur[E * OXs + ox]);
        curl_orbit_product<R, E + 1>(yv, xv, Ur, ox, OXs);
    }
}

constexpr int kP3JmThreads = 256;

template <typename R, int N>
__global__ void __launch_bounds__(kP3JmThreads) k_p3_jm(C<R>* __restrict__ A, const C<R>* __restrict__ UN,
                                                        const C<R>* __restrict__ UK, P3Params p,
                                                        const C<R>* __restrict__ tw, C<R> kj, C<R> km) {
    constexpr int NT = kP3JmThreads;
    constexpr int OX = N / 2 + 1;
    extern __shared__ unsigned char smem_raw[];
    C<R>* twl = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf = twl + N;
    const int tid = threadIdx.x;
    // block -> (octant row, right-hand side, sibling); the 4 nrhs workgroups
    // of one operator row get indices congruent modulo 8 (one XCD, one L2)
    const int K = 4 * p.nrhs;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int row = (q / K) * 8 + xcd;
    if (row >= p.Oy * p.Oz) return;       // padding rows, uniform over the workgroup
    const int kk = q - (q / K) * K;
    const int r = kk >> 2, sib = kk & 3;
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    if (sib >= ny_sib * nz_sib) return;   // uniform over the workgroup
    const int sz = sib / ny_sib, sy = sib - sz * ny_sib;
    const int z = sz ? p.Mz - oz : oz;
    const int y = sy ? p.My - oy : oy;
    // LDS row h * 12 + c: half h (0 electric, 1 magnetic), component c
    C<R>* base = A + (long long)(2 * r) * p.s_r + (long long)z * p.s_z + (long long)y * p.s_y;
    const long long s_c = p.s_c, s_r = p.s_r;
    auto rowp = [=](int rr) {
        const int h = rr >= 12, c = rr - 12 * h;
        return base + h * s_r + c * s_c;
    };
    for (int m = tid; m < N; m += NT) twl[m] = tw[m];
    rows_to_lds<R, N, NT>(buf, 24, p.Nx, rowp);
    __syncthreads();
    ct_passes<R, true, N, 0, 1, NT, 24, true>(buf, twl, 24, N, tid);   // Nx <= N / 2
    {
        const C<R>* Un = UN + (long long)row * 60 * OX;
        const C<R>* Uk = UK + (long long)row * 30 * OX;
        // LDS address of (row, column xi): one column base plus a constant
        // per row when rows are whole 16-element blocks (no per-row index
        // arithmetic, no per-row address registers)
        auto at = [&](int rr, int xi) -> C<R>& {
            if constexpr (N % 16 == 0) return buf[rr * (N + N / 16) + xi + (xi >> 4)];
            else return buf[lds_pad(rr * N + xi)];
        };
        // sign flip of both parts where bit a of m is set (no branches)
        auto flip = [](C<R> v, unsigned m, int a) {
            if constexpr (sizeof(R) == 4) {
                const unsigned f = ((m >> a) & 1u) << 31;
                v.x = __uint_as_float(__float_as_uint(v.x) ^ f);
                v.y = __uint_as_float(__float_as_uint(v.y) ^ f);
            } else {
                const unsigned long long f = (unsigned long long)((m >> a) & 1u) << 63;
                v.x = __longlong_as_double(__double_as_longlong(v.x) ^ f);
                v.y = __longlong_as_double(__double_as_longlong(v.y) ^ f);
            }
            return v;
        };
        // two work items per frequency, item h forming the sum of half h
        // from both halves' inputs; each round reads its columns, waits,
        // then writes them (the rounds' columns are disjoint)
        for (int w0 = 0; w0 < 2 * N; w0 += NT) {
            const int w = w0 + tid;
            const bool act = w < 2 * N;
            const int xi = w >> 1, h = w & 1;
            const int fx = 2 * xi > N;
            const int ox = fx ? N - xi : xi;
            const unsigned mask = fold_mask(fx, sy, sz);
            const bool odd = (fx + sy + sz) & 1;
            C<R> xo[12], xt[12], yv[12];
            if (act) {
#pragma unroll
                for (int a = 0; a < 12; ++a) {
                    xo[a] = flip(at(12 * h + a, xi), mask, a);
                    xt[a] = flip(at(12 - 12 * h + a, xi), mask, a);
                    yv[a] = mk<R>(0, 0);
                }
                curl_orbit_product<R, 0>(yv, xt, Uk, ox, OX);   // K x_other
                C<R> f = h ? km : kj;
                if (odd) f = mk<R>(-f.x, -f.y);
#pragma unroll
                for (int a = 0; a < 12; ++a) yv[a] = cmul(f, yv[a]);
                orbit_product<R, 0>(yv, xo, Un, ox, OX);        // + N x_own
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int a = 0; a < 12; ++a) at(12 * h + a, xi) = flip(yv[a], mask, a);
            }
        }
    }
    __syncthreads();
    ct_passes<R, false, N, 0, 1, NT, 24, false, true>(buf, twl, 24, N, tid);   // crop to Nx
    lds_to_rows<R, N, NT>(buf, 24, p.Nx, rowp);
}

// compiled for complex64 at every length of the list, for complex128 up to
// 128 (beyond, its 24 rows of butterflies would not stay in registers)
template <typename R, int N>
static bool launch_p3_jm_n(C<R>* A, const C<R>* UN, const C<R>* UK, const P3Params& p, const C<R>* tw, C<R> kj,
                           C<R> km, hipStream_t s) {
    if constexpr (sizeof(R) == 8 && N > 128) {
        return false;
    } else {
    const size_t lds = ((size_t)N + lds_pad(24 * N) + 2) * sizeof(C<R>);
    if (lds > 160 * 1024) return false;
    const long long rows8 = ((long long)p.Oy * p.Oz + 7) / 8 * 8;
    const long long nblk = rows8 * 4LL * p.nrhs;
    VIE_REQUIRE(nblk < (1LL << 31), -1, "J-M x pass: too many workgroups");
    static std::once_flag once;
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void*)k_p3_jm<R, N>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    });
    timed_launch(k_p3_jm<R, N>, dim3((unsigned)nblk), dim3(kP3JmThreads), (unsigned)lds, s, A, UN, UK, p, tw, kj,
                 km);
    VIE_HIP(hipGetLastError());
    return true;
    }
}

// x pass of the PWC basis (3 unknowns per voxel, the pulse functions): one
// workgroup per (octant row, right-hand side) holds the 3 component rows of
// each of the up to four sibling pencils of the row (at most 12 rows, the LDS
// of one PWL pencil group).  The 3 x 3 block of a frequency comes from the 6
// tensors of the pulse functions, unique entries u = 10 pq (ll = 11), placed
// by the PWL orbit table restricted to the unknowns a = 4 p; one work item
// per (sibling, frequency).
template <typename R, int E, int K>
__device__ __forceinline__ void orbit_apply_pwc(C<R>* yv, const C<R>* xv, C<R> u) {
    constexpr Orbits o = make_orbits();
    if constexpr (K < o.cnt[E]) {
        constexpr int a = o.m[E][K].a, b = o.m[E][K].b, sg = o.m[E][K].s;
        static_assert(a % 4 == 0 && b % 4 == 0, "pulse-pulse entries couple the unknowns a = 4 p only");
        if constexpr (sg > 0) cfma(yv[a / 4], u, xv[b / 4]);
        else cfma(yv[a / 4], mk<R>(-u.x, -u.y), xv[b / 4]);
        orbit_apply_pwc<R, E, K + 1>(yv, xv, u);
    }
}

template <typename R, int Q>
__device__ __forceinline__ void orbit_product_pwc(C<R>* yv, const C<R>* xv, const C<R>* __restrict__ Ur, int ox,
                                                  int OXs) {
    if constexpr (Q < 6) {
        orbit_apply_pwc<R, 10 * Q, 0>(yv, xv, Ur[10 * Q * OXs + ox]);
        orbit_product_pwc<R, Q + 1>(yv, xv, Ur, ox, OXs);
    }
}

constexpr int kP3PwcThreads = 256;

template <typename R, int N>
__global__ void __launch_bounds__(kP3PwcThreads) k_p3_pwc(C<R>* __restrict__ A, const C<R>* __restrict__ U,
                                                          P3Params p, const C<R>* __restrict__ tw) {
    constexpr int NT = kP3PwcThreads;
    constexpr int OX = N / 2 + 1;
    extern __shared__ unsigned char smem_raw[];
    C<R>* twl = reinterpret_cast<C<R>*>(smem_raw);
    C<R>* buf = twl + N;
    const int tid = threadIdx.x;
    // block -> (octant row, right-hand side), rows dealt to XCDs as in the
    // sibling variant
    const int K = p.nrhs;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int row = (q / K) * 8 + xcd;
    if (row >= p.Oy * p.Oz) return;   // padding rows, uniform over the workgroup
    const int r = q - (q / K) * K;
    const int oz = row / p.Oy, oy = row - oz * p.Oy;
    const int ny_sib = (oy == 0 || 2 * oy == p.My) ? 1 : 2;
    const int nz_sib = (oz == 0 || 2 * oz == p.Mz) ? 1 : 2;
    const int nsib = ny_sib * nz_sib;
    const int nrows = 3 * nsib;   // LDS row sb * 3 + c, sibling sb = sz * ny_sib + sy
    C<R>* base = A + (long long)r * p.s_r;
    const long long s_c = p.s_c, s_y = p.s_y, s_z = p.s_z;
    const int Mz = p.Mz, My = p.My;
    auto rowp = [=](int rr) {
        const int sb = rr / 3, c = rr - 3 * sb;
        const int sz = sb >= ny_sib, sy = sb - sz * ny_sib;
        const int z = sz ? Mz - oz : oz, y = sy ? My - oy : oy;
        return base + z * s_z + y * s_y + c * s_c;
    };
    for (int m = tid; m < N; m += NT) twl[m] = tw[m];
    rows_to_lds<R, N, NT>(buf, nrows, p.Nx, rowp);
    __syncthreads();
    ct_passes<R, true, N, 0, 1, NT, 12, true>(buf, twl, nrows, N, tid);   // Nx <= N / 2
    const C<R>* Ur = U + (long long)row * 60 * OX;
    for (int w = tid; w < nsib * N; w += NT) {
        const int sb = w / N, xi = w - sb * N;
        const int sz = sb >= ny_sib, sy = sb - sz * ny_sib;
        const int fx = 2 * xi > N;
        const int ox = fx ? N - xi : xi;
        const unsigned mask = fold_mask(fx, sy, sz);
        C<R> xv[3], yv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            C<R> v = buf[lds_pad((sb * 3 + c) * N + xi)];
            if (mask & (1u << (4 * c))) { v.x = -v.x; v.y = -v.y; }
            xv[c] = v;
            yv[c] = mk<R>(0, 0);
        }
        orbit_product_pwc<R, 0>(yv, xv, Ur, ox, OX);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            C<R> v = yv[c];
            if (mask & (1u << (4 * c))) { v.x = -v.x; v.y = -v.y; }
            buf[lds_pad((sb * 3 + c) * N + xi)] = v;
        }
    }
    __syncthreads();
    ct_passes<R, false, N, 0, 1, NT, 12, false, true>(buf, twl, nrows, N, tid);   // crop to Nx
    lds_to_rows<R, N, NT>(buf, nrows, p.Nx, rowp);
}

// lengths with a compile-time kernel
#define VIE_P3_LENGTHS(X) X(8) X(16) X(32) X(64) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512)

bool p3_ct_supported(int n) {
    switch (n) {
#define CASE(n_) case n_:
        VIE_P3_LENGTHS(CASE)
#undef CASE
        return true;
        default: return false;
    }
}

int p3_ct_groups(int es, int n) { return p3_gmax(es, n, 512); }

// the staged variant holds the operator row and at least one pencil group
bool p3_ct_fits(int es, int n) { return p3_ct_supported(n) && p3_lds_bytes(es, n, 1) <= 160 * 1024; }

template <typename R, int N, int SPLIT>
static void launch_p3_small_n(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    const size_t lds = ((size_t)N + lds_pad(12 * N) + 2) * sizeof(C<R>);
    const long long rows8 = ((long long)p.Oy * p.Oz + 7) / 8 * 8;
    const long long nblk = rows8 * 4LL * p.nrhs;
    VIE_REQUIRE(nblk < (1LL << 31), -1, "x pass: too many workgroups");
    timed_launch(k_p3_small<R, N, SPLIT>, dim3((unsigned)nblk), dim3(kP3SmallThreads), (unsigned)lds, s, A, U, p, tw);
    VIE_HIP(hipGetLastError());
}

template <typename R, int N>
static void launch_p3_pair_n(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    const size_t lds = ((size_t)N + lds_pad(24 * N) + 2) * sizeof(C<R>);
    const long long rows8 = ((long long)p.Oy * p.Oz + 7) / 8 * 8;
    const long long nblk = rows8 * 4LL * ((p.nrhs + 1) / 2);
    VIE_REQUIRE(nblk < (1LL << 31), -1, "x pass: too many workgroups");
    VIE_REQUIRE(lds <= 160 * 1024, -1, "x pass: pair variant does not fit LDS");
    static std::once_flag once;
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void*)k_p3_pair<R, N>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    });
    timed_launch(k_p3_pair<R, N>, dim3((unsigned)nblk), dim3(kP3SmallThreads), (unsigned)lds, s, A, U, p, tw);
    VIE_HIP(hipGetLastError());
}

template <typename R, int N>
static void launch_p3_quad_n(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    const size_t lds = ((size_t)N + lds_pad(48 * N) + 2) * sizeof(C<R>);
    const long long rows8 = ((long long)p.Oy * p.Oz + 7) / 8 * 8;
    const long long nblk = rows8 * p.nrhs;
    VIE_REQUIRE(nblk < (1LL << 31), -1, "x pass: too many workgroups");
    VIE_REQUIRE(lds <= 160 * 1024, -1, "x pass: sibling variant does not fit LDS");
    static std::once_flag once;
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void*)k_p3_quad<R, N>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    });
    timed_launch(k_p3_quad<R, N>, dim3((unsigned)nblk), dim3(kP3QuadThreads), (unsigned)lds, s, A, U, p, tw);
    VIE_HIP(hipGetLastError());
}

template <typename R, int N>
static void launch_p3_pwc_n(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    const size_t lds = ((size_t)N + lds_pad(12 * N) + 2) * sizeof(C<R>);
    const long long rows8 = ((long long)p.Oy * p.Oz + 7) / 8 * 8;
    const long long nblk = rows8 * p.nrhs;
    VIE_REQUIRE(nblk < (1LL << 31), -1, "x pass: too many workgroups");
    VIE_REQUIRE(lds <= 160 * 1024, -1, "PWC x pass does not fit LDS");
    static std::once_flag once;
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void*)k_p3_pwc<R, N>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    });
    timed_launch(k_p3_pwc<R, N>, dim3((unsigned)nblk), dim3(kP3PwcThreads), (unsigned)lds, s, A, U, p, tw);
    VIE_HIP(hipGetLastError());
}

template <typename R, int N>
static void launch_p3_pref(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    if constexpr (N <= 128) {
        const size_t lds = ((size_t)N + 60 * (N / 2 + 1) + lds_pad(12 * N) + 2) * sizeof(C<R>);
        const long long rows8 = ((long long)p.Oy * p.Oz + 7) / 8 * 8;
        const long long nblk = rows8 * 4LL * p.nrhs;
        VIE_REQUIRE(nblk < (1LL << 31), -1, "x pass: too many workgroups");
        static std::once_flag once;
        std::call_once(once, [&] {
            (void)hipFuncSetAttribute((const void*)k_p3_pref<R, N>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
            (void)hipGetLastError();
        });
        timed_launch(k_p3_pref<R, N>, dim3((unsigned)nblk), dim3(kP3SmallThreads), (unsigned)lds, s, A, U, p, tw);
        VIE_HIP(hipGetLastError());
    } else {
        throw Error(-1, "x pass: prefetching variant needs an fft length <= 128");
    }
}

bool p3_pref_fits(int n) { return p3_ct_supported(n) && n <= 128; }

// the sibling variant is built for complex64 only (its two-vector product
// would not fit the registers in complex128)
template <typename R, int N>
static void launch_p3_quad(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    if constexpr (sizeof(R) == 4) launch_p3_quad_n<R, N>(A, U, p, tw, s);
    else throw Error(-1, "x pass: sibling variant is complex64 only");
}

bool p3_pair_fits(int es, int n) {
    return p3_ct_supported(n) && ((size_t)n + (size_t)lds_pad(24 * n) + 2) * (size_t)es <= 160 * 1024;
}

bool p3_quad_fits(int es, int n) {
    return es == 8 && p3_ct_supported(n) && ((size_t)n + lds_pad(48 * n) + 2) * es <= 160 * 1024;
}

template <typename R, int N>
static void launch_p3_ct_n(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    constexpr int NT = p3_threads<R>();
    constexpr int GMAX = p3_gmax(sizeof(C<R>), N, NT);
    VIE_REQUIRE(p.groups >= 1 && p.groups <= GMAX && p.Ox == N / 2 + 1, -1, "x pass: bad group count");
    const size_t lds = (size_t)p3_lds_bytes(sizeof(C<R>), N, p.groups);
    VIE_REQUIRE(lds <= 160 * 1024, -1, "x pass: staged variant does not fit LDS for this length");
    // allow more than the default 64 KiB of dynamic LDS (once per process;
    // the size is fixed per instantiation); a refusal shows up as a launch
    // error below, so clear the status here
    static std::once_flag once;
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void*)k_p3_ct<R, N>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    });
    VIE_REQUIRE(p.sib_blocks == 1 || p.sib_blocks == 2 || p.sib_blocks == 4, -1, "x pass: bad sibling split");
    timed_launch(k_p3_ct<R, N>, dim3(p.Oy * p.Oz * p.sib_blocks), dim3(NT), (unsigned)lds, s, A, U, p, tw);
    VIE_HIP(hipGetLastError());
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
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute((const void*)k_strided<R, FWD, EPI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  96 * 1024);
        (void)hipGetLastError();
    });
    timed_launch(k_strided<R, FWD, EPI>, grid, dim3(256), (unsigned)lds, s, in, out, p, tw, ep);
    VIE_HIP(hipGetLastError());
}

template <typename R>
void launch_strided(bool fwd, const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2, long long n_o1,
                    const C<R>* tw, const Epilogue<R>* ep, hipStream_t s) {
    Epilogue<R> none{};
    if (ep && !fwd) {
        if (launch_strided_compiled<R>(false, true, in, out, p, n_o2, n_o1, tw, *ep, s)) return;
    } else if (!ep && fwd) {
        if (launch_strided_compiled<R>(true, false, in, out, p, n_o2, n_o1, tw, none, s)) return;
    } else if (!ep) {
        if (launch_strided_compiled<R>(false, false, in, out, p, n_o2, n_o1, tw, none, s)) return;
    }
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
    // the compiled kernels skip the zero upper half of each padded row
    VIE_REQUIRE(2 * p.Nx <= p.plan.n, -1, "x pass: fft length below 2 Nx");
    switch (p.plan.n) {
#define CASE(n_)                                                                          \
    case n_:                                                                             \
        if (p.variant == 1) launch_p3_small_n<R, n_, 1>(A, U, p, tw, s);                 \
        else if (p.variant == 4) launch_p3_small_n<R, n_, 2>(A, U, p, tw, s);            \
        else if (p.variant == 2) launch_p3_quad<R, n_>(A, U, p, tw, s);                  \
        else if (p.variant == 3) launch_p3_pref<R, n_>(A, U, p, tw, s);                  \
        else if (p.variant == 5) launch_p3_pair_n<R, n_>(A, U, p, tw, s);                \
        else launch_p3_ct_n<R, n_>(A, U, p, tw, s);                                      \
        return;
        VIE_P3_LENGTHS(CASE)
#undef CASE
        default: break;
    }
    const int nt = p3_threads<R>();
    VIE_REQUIRE(rows_fit(p.plan, p.groups * 12, nt) && 2 * p.groups * p.plan.n <= nt, -1,
                "x pass: more butterflies or columns than threads");
    size_t lds = (60 * (size_t)p.Ox + lds_pad(p.groups * 12 * p.pitch) + 2) * sizeof(C<R>);
    const bool split4 = 4 * p.groups * p.plan.n <= nt;
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute((const void*)k_p3<R, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
        (void)hipFuncSetAttribute((const void*)k_p3<R, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
        (void)hipGetLastError();
    });
    if (split4) timed_launch(k_p3<R, 4>, dim3(p.Oy * p.Oz), dim3(nt), (unsigned)lds, s, A, U, p, tw);
    else timed_launch(k_p3<R, 2>, dim3(p.Oy * p.Oz), dim3(nt), (unsigned)lds, s, A, U, p, tw);
    VIE_HIP(hipGetLastError());
}

// x pass of the curl operator (the staged kernel for any length whose rows
// fit): the magnetic field's product, and the coupling blocks of the J-M
// product in both precisions
template <typename R>
void launch_p3_curl(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    const int nt = p3_threads<R>();
    VIE_REQUIRE(rows_fit(p.plan, p.groups * 12, nt) && 2 * p.groups * p.plan.n <= nt, -1,
                "magnetic product: fft length along x above 256");
    const size_t lds = (30 * (size_t)p.Ox + lds_pad(p.groups * 12 * p.pitch) + 2) * sizeof(C<R>);
    VIE_REQUIRE(lds <= 150 * 1024, -1, "magnetic product: x rows do not fit LDS");
    const bool split4 = 4 * p.groups * p.plan.n <= nt;
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute((const void*)k_p3<R, 2, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  150 * 1024);
        (void)hipFuncSetAttribute((const void*)k_p3<R, 4, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  150 * 1024);
        (void)hipGetLastError();
    });
    if (split4) timed_launch(k_p3<R, 4, true>, dim3(p.Oy * p.Oz), dim3(nt), (unsigned)lds, s, A, U, p, tw);
    else timed_launch(k_p3<R, 2, true>, dim3(p.Oy * p.Oz), dim3(nt), (unsigned)lds, s, A, U, p, tw);
    VIE_HIP(hipGetLastError());
}
template void launch_p3_curl<float>(C<float>*, const C<float>*, const P3Params&, const C<float>*, hipStream_t);
template void launch_p3_curl<double>(C<double>*, const C<double>*, const P3Params&, const C<double>*, hipStream_t);

template <typename R>
bool launch_p3_jm(C<R>* A, const C<R>* UN, const C<R>* UK, const P3Params& p, const C<R>* tw, C<R> kj, C<R> km,
                  hipStream_t s) {
    if (2 * p.Nx > p.plan.n) return false;
    switch (p.plan.n) {
#define CASE(n_)                                                       \
    case n_:                                                          \
        return launch_p3_jm_n<R, n_>(A, UN, UK, p, tw, kj, km, s);
        VIE_P3_LENGTHS(CASE)
#undef CASE
        default: break;
    }
    return false;
}
template bool launch_p3_jm<float>(C<float>*, const C<float>*, const C<float>*, const P3Params&, const C<float>*,
                                  C<float>, C<float>, hipStream_t);
template bool launch_p3_jm<double>(C<double>*, const C<double>*, const C<double>*, const P3Params&,
                                   const C<double>*, C<double>, C<double>, hipStream_t);

template <typename R>
void launch_p3_pwc(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s) {
    VIE_REQUIRE(2 * p.Nx <= p.plan.n, -1, "x pass: fft length below 2 Nx");
    switch (p.plan.n) {
#define CASE(n_)                                        \
    case n_:                                           \
        launch_p3_pwc_n<R, n_>(A, U, p, tw, s);        \
        return;
        VIE_P3_LENGTHS(CASE)
#undef CASE
        default: break;
    }
    throw Error(-1, "the PWC x pass needs an fft length along x of 8, 16, 32, 64, 96, 128, 160, 192, 256, "
                            "320, 384 or 512");
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
template void launch_p3_pwc<float>(C<float>*, const C<float>*, const P3Params&, const C<float>*, hipStream_t);
template void launch_p3_pwc<double>(C<double>*, const C<double>*, const P3Params&, const C<double>*, hipStream_t);
template void launch_rows<double>(bool, C<double>*, long long, const FftPlan&, const C<double>*, hipStream_t);

}  // namespace vie
