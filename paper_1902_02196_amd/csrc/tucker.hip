// Tucker (low multilinear rank) compression of the 60 Toeplitz-defining
// tensors N(m), m in [0, N)^3 (eq. 43; Sec. III-C, last paragraph: these
// tensors keep a low multilinear rank and can be stored compressed).
//
// Sequentially truncated HOSVD of each tensor, modes x, y, z in turn: the
// FP64 Gram matrix of the mode unfolding of the tensor as compressed so far
// (device, tiled), its eigenvectors (host, cyclic Jacobi), the smallest
// eigenvalues dropped while their sum stays within tol^2 ||T||^2 / 3, and the
// tensor projected onto the kept eigenvectors (device) before the next mode.
// The dropped eigenvalues add up to ||T - T_hat||^2 exactly (the three
// projections are orthogonal), so each tensor is kept to tol ||T||.  The 60
// tensors are compressed by a pool of host threads, each on its own stream.
//
// Expansion rebuilds T_hat = core x_x U_x x_y U_y x_z U_z on the device and
// runs it through the operator set-up (circulant embedding, 3-D FFT,
// octant), so the products use the compressed operator.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "ctx.hpp"

namespace vie {

using cd = std::complex<double>;

// a tensor [n2][n1][n0], n0 fastest (x, y, z for the Toeplitz tensors)
struct Dims3 {
    int n[3];
    __host__ __device__ long long size() const { return (long long)n[0] * n[1] * n[2]; }
};

// address of the element with coordinate a along `mode` and the other two
// coordinates flattened into k (the lower axis fastest)
__host__ __device__ __forceinline__ long long addr3(const Dims3& d, int mode, int a, long long k) {
    if (mode == 0) return k * d.n[0] + a;
    if (mode == 1) {
        const long long i0 = k % d.n[0], i2 = k / d.n[0];
        return (i2 * d.n[1] + a) * d.n[0] + i0;
    }
    return (long long)a * d.n[1] * d.n[0] + k;
}

// G[a][b] = sum_k X[a, k] conj(X[b, k]) over the mode-`mode` unfolding, one
// 16 x 16 tile of G per workgroup, k staged through LDS 32 at a time; each
// entry summed by one thread in a fixed order
constexpr int kGT = 16, kGK = 32;

__global__ void __launch_bounds__(256) k_gram(const double2* __restrict__ X, Dims3 d, int mode,
                                              double2* __restrict__ G) {
    __shared__ double2 la[kGT][kGK + 1], lb[kGT][kGK + 1];
    const int n = d.n[mode];
    const long long K = d.size() / n;
    const int a0 = blockIdx.x * kGT, b0 = blockIdx.y * kGT;
    const int tid = threadIdx.x, ta = tid % kGT, tb = tid / kGT;
    double sr = 0, si = 0;
    for (long long k0 = 0; k0 < K; k0 += kGK) {
        for (int e = tid; e < kGT * kGK; e += 256) {
            // along x the mode coordinate is contiguous, along y and z the rest
            int i, kk;
            if (mode == 0) {
                i = e % kGT;
                kk = e / kGT;
            } else {
                kk = e % kGK;
                i = e / kGK;
            }
            const long long k = k0 + kk;
            double2 va = make_double2(0, 0), vb = make_double2(0, 0);
            if (k < K) {
                if (a0 + i < n) va = X[addr3(d, mode, a0 + i, k)];
                if (b0 + i < n) vb = X[addr3(d, mode, b0 + i, k)];
            }
            la[i][kk] = va;
            lb[i][kk] = vb;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < kGK; ++kk) {
            const double2 x = la[ta][kk], y = lb[tb][kk];
            sr += x.x * y.x + x.y * y.y;   // x conj(y)
            si += x.y * y.x - x.x * y.y;
        }
        __syncthreads();
    }
    if (a0 + ta < n && b0 + tb < n) G[(long long)(a0 + ta) * n + (b0 + tb)] = make_double2(sr, si);
}

// out = X x_mode W: out[.., p, ..] = sum_q W[p][q] X[.., q, ..], W row-major P x Q
__global__ void __launch_bounds__(256) k_mode_product(const double2* __restrict__ X, Dims3 din, int mode,
                                                      const double2* __restrict__ W, int P,
                                                      double2* __restrict__ out) {
    Dims3 dout = din;
    dout.n[mode] = P;
    const long long total = dout.size();
    const int Q = din.n[mode];
    const long long stride = mode == 0 ? 1 : (mode == 1 ? din.n[0] : (long long)din.n[0] * din.n[1]);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int c[3];
        c[0] = (int)(e % dout.n[0]);
        const long long t = e / dout.n[0];
        c[1] = (int)(t % dout.n[1]);
        c[2] = (int)(t / dout.n[1]);
        const int p = c[mode];
        c[mode] = 0;
        const long long base = ((long long)c[2] * din.n[1] + c[1]) * din.n[0] + c[0];
        const double2* w = W + (long long)p * Q;
        double sr = 0, si = 0;
        for (int q = 0; q < Q; ++q) {
            const double2 a = w[q], b = X[base + q * stride];
            sr += a.x * b.x - a.y * b.y;
            si += a.x * b.y + a.y * b.x;
        }
        out[e] = make_double2(sr, si);
    }
}

static void launch_gram(const double2* X, const Dims3& d, int mode, double2* G, hipStream_t s) {
    const int n = d.n[mode];
    const unsigned t = (unsigned)((n + kGT - 1) / kGT);
    hipLaunchKernelGGL(k_gram, dim3(t, t), dim3(256), 0, s, X, d, mode, G);
    VIE_HIP(hipGetLastError());
}

static void launch_mode_product(const double2* X, const Dims3& din, int mode, const double2* W, int P, double2* out,
                                hipStream_t s) {
    Dims3 dout = din;
    dout.n[mode] = P;
    const long long total = dout.size();
    const unsigned nb = (unsigned)std::min<long long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_mode_product, dim3(nb), dim3(256), 0, s, X, din, mode, W, P, out);
    VIE_HIP(hipGetLastError());
}

// Eigen-decomposition of a Hermitian n x n matrix (row-major) by the cyclic
// Jacobi method: each rotation first turns the (p, q) entry real with a
// phase on column q, then zeroes it with a real plane rotation (the
// classical symmetric formulas).  On return w holds the eigenvalues in
// descending order and the columns of V (row-major) the eigenvectors.
static void jacobi_hermitian(int n, std::vector<cd>& A, std::vector<double>& w, std::vector<cd>& V) {
    V.assign((size_t)n * n, cd(0));
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    double fro = 0;
    for (const cd& a : A) fro += std::norm(a);
    const double tiny = 1e-32 * fro;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::norm(A[(size_t)p * n + q]);
        if (off <= tiny) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const cd apq = A[(size_t)p * n + q];
                const double m = std::abs(apq);
                if (m == 0.0) continue;
                const double app = A[(size_t)p * n + p].real(), aqq = A[(size_t)q * n + q].real();
                const cd e = apq / m;   // e^{i phi}
                const double theta = (aqq - app) / (2.0 * m);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::abs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                // U = D R: U_pp = c, U_pq = s, U_qp = -s conj(e), U_qq = c conj(e)
                const cd ec = std::conj(e);
                for (int k = 0; k < n; ++k) {   // A <- A U (columns p, q)
                    const cd akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * ec * akq;
                    A[(size_t)k * n + q] = s * akp + c * ec * akq;
                }
                for (int k = 0; k < n; ++k) {   // A <- U^H A (rows p, q)
                    const cd apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * e * aqk;
                    A[(size_t)q * n + k] = s * apk + c * e * aqk;
                }
                A[(size_t)p * n + q] = 0.0;
                A[(size_t)q * n + p] = 0.0;
                for (int k = 0; k < n; ++k) {   // V <- V U
                    const cd vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * ec * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * ec * vkq;
                }
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) {
        const double x = A[(size_t)a * n + a].real(), y = A[(size_t)b * n + b].real();
        return x > y || (x == y && a < b);
    });
    std::vector<cd> Vs((size_t)n * n);
    w.resize(n);
    for (int j = 0; j < n; ++j) {
        w[j] = A[(size_t)idx[j] * n + idx[j]].real();
        for (int k = 0; k < n; ++k) Vs[(size_t)k * n + j] = V[(size_t)k * n + idx[j]];
    }
    V.swap(Vs);
}

// fewest leading eigenvalues (descending, negatives counted as 0) whose
// dropped tail sums to at most budget; at least 1
static int truncation_rank(const std::vector<double>& w, double budget, double* dropped) {
    const int n = (int)w.size();
    std::vector<double> tail(n + 1, 0.0);
    for (int k = n - 1; k >= 0; --k) tail[k] = tail[k + 1] + std::max(w[k], 0.0);
    int r = n;
    for (int k = 0; k <= n; ++k)
        if (tail[k] <= budget) {
            r = k;
            break;
        }
    r = std::max(r, 1);
    *dropped = tail[r];
    return r;
}

// one tensor through the three modes on stream s; work buffers a, b hold
// V values each, g n_max^2
static void compress_one(const double2* T, const int N[3], double tol, hipStream_t s, double2* a, double2* b,
                         double2* g, double2* wdev, TuckerTensor& out) {
    Dims3 d{{N[0], N[1], N[2]}};
    const double2* X = T;
    double norm2 = -1, dropped_total = 0;
    out.U.clear();
    for (int mode = 0; mode < 3; ++mode) {
        const int n = d.n[mode];
        launch_gram(X, d, mode, g, s);
        std::vector<cd> G((size_t)n * n);
        VIE_HIP(hipMemcpyAsync(G.data(), g, G.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
        VIE_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i)   // Hermitian part (the two triangles are summed separately)
            for (int j = 0; j <= i; ++j) {
                const cd h = 0.5 * (G[(size_t)i * n + j] + std::conj(G[(size_t)j * n + i]));
                G[(size_t)i * n + j] = h;
                G[(size_t)j * n + i] = std::conj(h);
            }
        if (norm2 < 0) {
            norm2 = 0;
            for (int i = 0; i < n; ++i) norm2 += G[(size_t)i * n + i].real();
        }
        std::vector<double> w;
        std::vector<cd> Vm;
        jacobi_hermitian(n, G, w, Vm);
        double dropped = 0;
        const int r = truncation_rank(w, tol * tol * norm2 / 3.0, &dropped);
        dropped_total += dropped;
        out.r[mode] = r;
        // factor U (n x r, row-major) and the projection W = U^H (r x n)
        std::vector<cd> U((size_t)n * r), W((size_t)r * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < r; ++j) {
                U[(size_t)i * r + j] = Vm[(size_t)i * n + j];
                W[(size_t)j * n + i] = std::conj(Vm[(size_t)i * n + j]);
            }
        out.U.push_back(U);
        VIE_HIP(hipMemcpyAsync(wdev, W.data(), W.size() * sizeof(double2), hipMemcpyHostToDevice, s));
        double2* dst = (X == a) ? b : a;
        launch_mode_product(X, d, mode, wdev, r, dst, s);
        d.n[mode] = r;
        X = dst;
        VIE_HIP(hipStreamSynchronize(s));   // W is reused by the next mode
    }
    out.core.resize((size_t)d.size());
    VIE_HIP(hipMemcpyAsync(out.core.data(), X, out.core.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    VIE_HIP(hipStreamSynchronize(s));
    out.norm = std::sqrt(norm2);
    out.rel_error = norm2 > 0 ? std::sqrt(dropped_total / norm2) : 0.0;
}

void tucker_compress(Ctx& c, double tol) {
    const int nent = 60;
    const long long V = c.V;
    const int nmax = std::max(c.N[0], std::max(c.N[1], c.N[2]));
    VIE_HIP(hipStreamSynchronize(c.stream));   // the blocks are complete
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nthr = (int)std::min<unsigned>(std::min<unsigned>(hw, 16u), (unsigned)nent);
    std::vector<TuckerTensor> res(nent);
    std::atomic<int> next{0};
    std::vector<std::string> errs(nthr);
    std::vector<int> codes(nthr, VIE_OK);
    auto worker = [&](int w) {
        hipStream_t s = nullptr;
        double2 *a = nullptr, *b = nullptr, *g = nullptr, *wd = nullptr;
        try {
            VIE_HIP(hipSetDevice(c.device));
            VIE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            VIE_HIP(hipMalloc(&a, V * sizeof(double2)));
            VIE_HIP(hipMalloc(&b, V * sizeof(double2)));
            VIE_HIP(hipMalloc(&g, (size_t)nmax * nmax * sizeof(double2)));
            VIE_HIP(hipMalloc(&wd, (size_t)nmax * nmax * sizeof(double2)));
            for (int e = next++; e < nent; e = next++) compress_one(c.T + e * V, c.N, tol, s, a, b, g, wd, res[e]);
        } catch (const Error& ex) {
            errs[w] = ex.what();
            codes[w] = ex.code;
        } catch (const std::exception& ex) {
            errs[w] = ex.what();
            codes[w] = VIE_EDEVICE;
        }
        if (s) (void)hipStreamSynchronize(s);
        for (double2* p : {a, b, g, wd})
            if (p) (void)hipFree(p);
        if (s) (void)hipStreamDestroy(s);
    };
    std::vector<std::thread> pool;
    for (int w = 0; w < nthr; ++w) pool.emplace_back(worker, w);
    for (auto& t : pool) t.join();
    for (int w = 0; w < nthr; ++w)
        if (codes[w] != VIE_OK) throw Error(codes[w], "Tucker compression: " + errs[w]);
    c.tucker.tensors = std::move(res);
    c.tucker.tol = tol;
    c.tucker.valid = true;
}

// T_hat of tensor e into out (V values): the core expanded along z, y, x
static void reconstruct_one(const TuckerTensor& t, const int N[3], double2* out, double2* a, double2* b,
                            double2* wdev, hipStream_t s) {
    Dims3 d{{t.r[0], t.r[1], t.r[2]}};
    VIE_HIP(hipMemcpyAsync(a, t.core.data(), t.core.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    const double2* X = a;
    for (int step = 0; step < 3; ++step) {
        const int mode = 2 - step;
        const std::vector<cd>& U = t.U[mode];   // N[mode] x r, row-major: W = U
        VIE_HIP(hipMemcpyAsync(wdev, U.data(), U.size() * sizeof(double2), hipMemcpyHostToDevice, s));
        double2* dst = step == 2 ? out : (X == a ? b : a);
        launch_mode_product(X, d, mode, wdev, N[mode], dst, s);
        d.n[mode] = N[mode];
        X = dst;
        VIE_HIP(hipStreamSynchronize(s));   // wdev is reused by the next step
    }
}

void tucker_reconstruct(Ctx& c, double2* out) {
    VIE_REQUIRE(c.tucker.valid, VIE_ESTATE, "no Tucker form: call vie_tucker_compress first");
    const long long V = c.V;
    const int nmax = std::max(c.N[0], std::max(c.N[1], c.N[2]));
    double2 *a = nullptr, *b = nullptr, *wd = nullptr;
    try {
        VIE_HIP(hipMalloc(&a, V * sizeof(double2)));
        VIE_HIP(hipMalloc(&b, V * sizeof(double2)));
        VIE_HIP(hipMalloc(&wd, (size_t)nmax * nmax * sizeof(double2)));
        VIE_HIP(hipStreamSynchronize(c.stream));
        for (int e = 0; e < 60; ++e) reconstruct_one(c.tucker.tensors[e], c.N, out + e * V, a, b, wd, c.stream);
    } catch (...) {
        for (double2* p : {a, b, wd})
            if (p) (void)hipFree(p);
        throw;
    }
    for (double2* p : {a, b, wd}) (void)hipFree(p);
}

size_t TuckerForm::values() const {
    size_t v = 0;
    for (const TuckerTensor& t : tensors) {
        v += t.core.size();
        for (const auto& U : t.U) v += U.size();
    }
    return v;
}

}  // namespace vie
