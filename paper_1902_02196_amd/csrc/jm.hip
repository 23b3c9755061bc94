// The J-M formulation for objects with magnetic contrast (Sec. II, eq.
// 13-15): polarisation and magnetisation currents j = c_e chi_e e and
// m = c_m chi_m h (eq. 6-7), 24 unknowns per voxel, the electric 12 first.
// On the PWL basis, with the contrasts constant per voxel as in the
// dielectric equation,
//
//   (A x)_j = eps_r G x_j - chi_e (N x_j - c_e K x_m)
//   (A x)_m = mu_r G x_m - chi_m (N x_m + c_m K x_j)
//   b       = [c_e chi_e e_t; c_m chi_m h_t]
//
// and with the block-diagonal preconditioner P = diag(M_eps G, M_mu G)
// (the dielectric one of Sec. IV-B on each half)
//
//   P^-1 A x = [x_j - tau_e G^-1 (N x_j - c_e K x_m); x_m - tau_m G^-1 (N x_m + c_m K x_j)].
//
// A vector [nrhs][24][V] is read as 2 nrhs vectors of 12 components.  Where
// the x length has a compiled J-M x pass, the FFT passes run once over them
// and the x pass forms both coupled sums, N x_j - c_e K x_m and N x_m + c_m
// K x_j, from the two halves of a pencil together; elsewhere the product is
// one N product and one K product over the 2 nrhs vectors.  Then one
// elementwise pass applies the materials.
#include <algorithm>
#include <vector>

#include "ctx.hpp"

namespace vie {

template <typename R>
struct JmMat {
    const C<R>* epsr;   // electric: eps_r, chi_e, tau_e per voxel
    const C<R>* chie;
    const C<R>* taue;
    const C<R>* mur;    // magnetic: mu_r, chi_m, tau_m per voxel
    const C<R>* chim;
    const C<R>* taum;
};

template <typename R>
__global__ void __launch_bounds__(256) k_jm_combine(int op, const C<R>* __restrict__ x, const C<R>* __restrict__ wN,
                                                    const C<R>* __restrict__ wK, const C<R>* __restrict__ rhs,
                                                    C<R>* __restrict__ y, JmMat<R> m, R g0, R g1, R wce, R wcm,
                                                    long long V, long long n) {
    // n = nrhs * 12 V items, one (right-hand side, component a < 12, voxel)
    // each, producing both halves
    const long long V12 = 12 * V;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long r = i / V12, rem = i - r * V12;
        const int a = (int)(rem / V);
        const long long v = rem - a * V;
        const R G = (a & 3) ? g1 : g0;
        const long long ij = r * 2 * V12 + rem, im = ij + V12;
        const C<R> xj = x[ij], xm = x[im];
        // N x_j - c_e K x_m and N x_m + c_m K x_j, c = i w (eps0 | mu0):
        // from the separate products, or formed by the fused x pass (wK null)
        C<R> sj = wN[ij], sm = wN[im];
        if (wK) {
            const C<R> Kj = wK[ij], Km = wK[im];
            sj = mk<R>(sj.x + wce * Km.y, sj.y - wce * Km.x);
            sm = mk<R>(sm.x - wcm * Kj.y, sm.y + wcm * Kj.x);
        }
        C<R> yj, ym;
        if (op == OP_A) {
            yj = csub(cscale(cmul(m.epsr[v], xj), G), cmul(m.chie[v], sj));
            ym = csub(cscale(cmul(m.mur[v], xm), G), cmul(m.chim[v], sm));
        } else {   // P^-1 A x, and the refinement residual rhs - P^-1 A x
            const R ig = R(1) / G;
            yj = csub(xj, cscale(cmul(m.taue[v], sj), ig));
            ym = csub(xm, cscale(cmul(m.taum[v], sm), ig));
            if (op == OP_RESID) {
                yj = csub(rhs[ij], yj);
                ym = csub(rhs[im], ym);
            }
        }
        y[ij] = yj;
        y[im] = ym;
    }
}

// P^-1 b = [c_e tau_e G^-1 e_t; c_m tau_m G^-1 h_t] from [e_t; h_t]
__global__ void k_jm_rhs(double2* __restrict__ rhs, const double2* __restrict__ eh, const double2* __restrict__ taue,
                         const double2* __restrict__ taum, double gi0, double gi1, double wce, double wcm,
                         long long V, long long n) {
    const long long V12 = 12 * V;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long r = i / (2 * V12), rem = i - r * 2 * V12;
        const int h = rem >= V12;
        const long long q = rem - h * V12;
        const int a = (int)(q / V);
        const long long v = q - a * V;
        const double2 t = h ? taum[v] : taue[v];
        const double w = (h ? wcm : wce) * ((a & 3) ? gi1 : gi0);
        const double2 e = eh[i];
        const double2 te = cmul(t, e);
        rhs[i] = make_double2(-w * te.y, w * te.x);   // i w (tau e) / G
    }
}

static unsigned grid_for(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 16384); }

template <typename R>
void apply_jm(Ctx& c, int op, int nrhs, const C<R>* x, C<R>* y, const C<R>* rhs, void* ws_ext, size_t) {
    VIE_REQUIRE(ws_ext == nullptr, VIE_EINVAL, "the J-M product has no fixed-workspace form");
    VIE_REQUIRE(op == OP_PREC || op == OP_A || op == OP_RESID, VIE_EINVAL,
                "the J-M product is P^-1 A or A (or the refinement residual)");
    VIE_REQUIRE(c.has_contrast, VIE_ESTATE, "the J-M product needs vie_set_contrast");
    VIE_REQUIRE(c.mmat.tau != nullptr, VIE_ESTATE, "no magnetic contrast");
    ensure_curl(c);
    const long long V = c.V;
    const size_t half = (size_t)nrhs * 24 * V;   // elements of one product over the 2 nrhs halves
    C<R>* wN = static_cast<C<R>*>(c.jmbuf.get(2 * half * sizeof(C<R>)));
    C<R>* wK = nullptr;
    {
        NcGuard g(c, 12);
        if (jm_fused_supported(c, sizeof(C<R>))) {
            apply_op<R>(c, OP_JMS, 2 * nrhs, x, wN, nullptr);
        } else {
            wK = wN + half;
            apply_op<R>(c, OP_N, 2 * nrhs, x, wN, nullptr);
            apply_op<R>(c, OP_K, 2 * nrhs, x, wK, nullptr);
        }
    }
    JmMat<R> m;
    if constexpr (sizeof(R) == 4) {
        m = JmMat<R>{c.mat.epsr64, c.mat.chi64, c.mat.tau64, c.mmat.epsr64, c.mmat.chi64, c.mmat.tau64};
    } else {
        m = JmMat<R>{c.mat.eps_r, c.mat.chi, c.mat.tau, c.mmat.eps_r, c.mmat.chi, c.mmat.tau};
    }
    const double dv = c.D[0] * c.D[1] * c.D[2];
    const long long n = (long long)nrhs * 12 * V;
    hipLaunchKernelGGL((k_jm_combine<R>), dim3(grid_for(n)), dim3(256), 0, c.stream, op, x, wN, wK, rhs, y, m,
                       R(dv), R(dv / 12), R(c.omega * kEps0), R(c.omega * kMu0), V, n);
    VIE_HIP(hipGetLastError());
}

bool jm_fused_supported(const Ctx& c, size_t es) {
    const int Mx = c.M[0];
    if (!p3_ct_supported(Mx) || 2 * c.N[0] > Mx) return false;
    if (es == sizeof(C<double>) && Mx > 128) return false;
    return ((size_t)Mx + (size_t)lds_pad(24 * Mx) + 2) * es <= 160 * 1024;
}

template void apply_jm<float>(Ctx&, int, int, const C<float>*, C<float>*, const C<float>*, void*, size_t);
template void apply_jm<double>(Ctx&, int, int, const C<double>*, C<double>*, const C<double>*, void*, size_t);

void jm_rhs_prec(Ctx& c, int nrhs, const double2* eh_t, double2* rhs) {
    VIE_REQUIRE(c.has_contrast && c.mmat.tau, VIE_ESTATE, "the J-M right-hand side needs the contrasts");
    const double dv = c.D[0] * c.D[1] * c.D[2];
    const long long n = (long long)nrhs * 24 * c.V;
    hipLaunchKernelGGL(k_jm_rhs, dim3(grid_for(n)), dim3(256), 0, c.stream, rhs, eh_t, c.mat.tau, c.mmat.tau,
                       1.0 / dv, 12.0 / dv, c.omega * kEps0, c.omega * kMu0, c.V, n);
    VIE_HIP(hipGetLastError());
}

void jm_default_mcontrast(Ctx& c) {
    c.free_mcontrast();
    const size_t V = (size_t)c.V;
    double* one = static_cast<double*>(c.small.get(2 * V * sizeof(double)));
    Materials& m = c.mmat;
    VIE_HIP(hipMalloc(&m.eps_r, V * sizeof(double2)));
    VIE_HIP(hipMalloc(&m.chi, V * sizeof(double2)));
    VIE_HIP(hipMalloc(&m.tau, V * sizeof(double2)));
    VIE_HIP(hipMalloc(&m.tau64, V * sizeof(float2)));
    VIE_HIP(hipMalloc(&m.epsr64, V * sizeof(float2)));
    VIE_HIP(hipMalloc(&m.chi64, V * sizeof(float2)));
    std::vector<double> h(2 * V, 0.0);
    for (size_t v = 0; v < V; ++v) h[v] = 1.0;   // mu' = 1, mu'' = 0
    VIE_HIP(hipMemcpyAsync(one, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    VIE_HIP(hipMemsetAsync(c.flag, 0, sizeof(int), c.stream));
    launch_materials(one, one + V, 1.0, m, c.V, c.flag, c.stream);
    VIE_HIP(hipStreamSynchronize(c.stream));
    c.has_mcontrast = false;
}

}  // namespace vie
