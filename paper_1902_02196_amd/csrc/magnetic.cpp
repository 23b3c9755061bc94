// Magnetic field and the MRI quantities derived from it (Sec. II eq. 8b and
// 'tot_fields' b; Sec. III eq. 25b; Sec. V-D).
//
// With the curl operator K u = curl S u discretised on the PWL basis like N,
// K^{pl,ql'}(d) = <f_m^{pl}, K f_n^{ql'}>, the tested total magnetic field of
// the current j (coefficients x) satisfies G h = h_t + K x, h_t the tested
// incident magnetic field.  K has 30 unique tensors Q_k^{ll'} =
// <N^l, S D_k N^{l'}> (l <= l'), K^{pl,ql'} = eps_pkq Q_k^{ll'}; they are
// assembled by the same device code as N's 60, embedded with the reflection
// sign -sigma_i(a) sigma_i(b), transformed and kept as an octant, on first
// use.  The product reuses the z and y passes of N's and its own x pass.
#include <cmath>
#include <vector>

#include "ctx.hpp"

namespace vie {

void ensure_curl(Ctx& c) {
    VIE_REQUIRE(c.has_grid && c.op, VIE_ESTATE, "the magnetic operator needs vie_set_grid");
    OperatorData& op = *c.op;
    std::lock_guard<std::mutex> g(op.curl_m);
    if (op.UK128) return;
    const long long V = c.V, Mt = (long long)c.M[0] * c.M[1] * c.M[2];
    double2* TK = nullptr;
    double2* UK = nullptr;
    float2* UK64 = nullptr;
    try {
        VIE_HIP(hipMalloc(&TK, 30 * V * sizeof(double2)));
        VIE_HIP(hipMalloc(&UK, 30 * c.Osz * sizeof(double2)));
        VIE_HIP(hipMalloc(&UK64, 30 * c.Osz * sizeof(float2)));
        AssemblyTables tab = build_curl_tables(c.D, c.k0);
        assemble_blocks(TK, tab, c.N[0], c.N[1], c.N[2], c.stream);
        double2* circ = static_cast<double2*>(c.ws.get(Mt * sizeof(double2)));
        const double2* tws[3] = {c.ax[0].tw128, c.ax[1].tw128, c.ax[2].tw128};
        FftPlan plans[3] = {c.ax[0].plan, c.ax[1].plan, c.ax[2].plan};
        embed_and_transform(UK, UK64, TK, circ, c.N[0], c.N[1], c.N[2], c.M[0], c.M[1], c.M[2], plans, tws,
                            c.stream, true);
        VIE_HIP(hipStreamSynchronize(c.stream));
    } catch (...) {
        if (TK) (void)hipFree(TK);
        if (UK) (void)hipFree(UK);
        if (UK64) (void)hipFree(UK64);
        throw;
    }
    op.TK = TK;
    op.UK128 = UK;
    op.UK64 = UK64;
    op.bytes += 30 * (V + c.Osz) * sizeof(double2) + 30 * c.Osz * sizeof(float2);
}

// axis of a signed unit vector along a coordinate axis, -1 otherwise
static int unit_axis(const double v[3], double* sign) {
    int ax = -1, nz = 0;
    for (int i = 0; i < 3; ++i)
        if (v[i] != 0.0) {
            ax = i;
            ++nz;
        }
    if (nz != 1 || std::fabs(std::fabs(v[ax]) - 1.0) > 1e-12) return -1;
    *sign = v[ax] > 0 ? 1.0 : -1.0;
    return ax;
}

void planewave_h(Ctx& c, const double pol[3], const double dir[3], double amp, double2* h_t) {
    double sp = 1, sd = 1;
    const int pa = unit_axis(pol, &sp), da = unit_axis(dir, &sd);
    VIE_REQUIRE(pa >= 0 && da >= 0 && pa != da, VIE_EINVAL,
                "pol and dir must be distinct unit vectors along coordinate axes");
    // H = (1 / eta0) dir x E: polarisation dir x pol along the third axis
    const int ha = 3 - pa - da;
    const double eta0 = std::sqrt(kMu0 / kEps0);
    const double sh = sp * sd * levi(da, pa, ha);
    launch_planewave(h_t, c.N[0], c.N[1], c.N[2], c.D, c.k0, ha, da, sd, amp * sh / eta0, 12, c.stream);
}

}  // namespace vie

using namespace vie;

namespace {

void check(vie_ctx* ctx) { VIE_REQUIRE(ctx != nullptr, VIE_EINVAL, "null context"); }

bool overlap(const void* a, const void* b, size_t n) {
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + n && pb < pa + n;
}

}  // namespace

extern "C" {

int vie_incident_planewave_h(vie_ctx* ctx, const double pol[3], const double dir[3], double amp, void* h_t) {
    return guarded([&] {
        check(ctx);
        Ctx& c = ctx->c;
        VIE_HIP(hipSetDevice(c.device));
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(c.nc == 12, VIE_EINVAL,
                    "the incident magnetic field is tested on the PWL basis (a J-M context's incident calls "
                    "write both halves)");
        VIE_REQUIRE(pol && dir && h_t, VIE_EINVAL, "null argument");
        planewave_h(c, pol, dir, amp, static_cast<double2*>(h_t));
    });
}

int vie_incident_dipoles_h(vie_ctx* ctx, int nrhs, const double* pos, const double* moment, int nq, void* h_t) {
    return guarded([&] {
        check(ctx);
        Ctx& c = ctx->c;
        VIE_HIP(hipSetDevice(c.device));
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(c.nc == 12, VIE_EINVAL,
                    "the incident magnetic field is tested on the PWL basis (a J-M context's incident calls "
                    "write both halves)");
        VIE_REQUIRE(nrhs >= 1 && pos && moment && h_t, VIE_EINVAL, "bad dipole arguments");
        VIE_REQUIRE(nq >= 1 && nq <= kMaxGauss, VIE_EINVAL, "nq must be in 1..16");
        AssemblyTables tab = build_assembly_tables(c.D, c.k0);   // holds the Gauss tables
        std::vector<double> host(6 * (size_t)nrhs + 2 * nq);
        for (int i = 0; i < 3 * nrhs; ++i) {
            VIE_REQUIRE(std::isfinite(pos[i]) && std::isfinite(moment[i]), VIE_ENAN, "non-finite dipole");
            host[i] = pos[i];
            host[3 * nrhs + i] = moment[i];
        }
        for (int i = 0; i < nq; ++i) {
            host[6 * nrhs + i] = tab.gl_x[nq][i];
            host[6 * nrhs + nq + i] = tab.gl_w[nq][i];
        }
        double* dev = static_cast<double*>(c.small.get(host.size() * sizeof(double)));
        VIE_HIP(hipMemcpyAsync(dev, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
        launch_dipoles(static_cast<double2*>(h_t), nrhs, dev, dev + 3 * nrhs, nq, dev + 6 * nrhs, dev + 6 * nrhs + nq,
                       nullptr, c.N[0], c.N[1], c.N[2], c.D, c.k0, c.omega * kEps0, c.nc, c.stream, 1);
        VIE_HIP(hipStreamSynchronize(c.stream));   // the host staging buffer is reused
    });
}

int vie_magnetic_field(vie_ctx* ctx, int nrhs, const void* h_t, const void* x, void* h) {
    return guarded([&] {
        check(ctx);
        Ctx& c = ctx->c;
        VIE_HIP(hipSetDevice(c.device));
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(c.nc == 12, VIE_EINVAL, "the magnetic field is computed for the PWL basis");
        VIE_REQUIRE(nrhs >= 1 && h_t && x && h, VIE_EINVAL, "bad arguments");
        const size_t bytes = (size_t)nrhs * 12 * c.V * sizeof(double2);
        VIE_REQUIRE(!overlap(h, x, bytes), VIE_EINVAL, "h must not overlap x");
        ensure_curl(c);
        apply_op<double>(c, OP_CURL, nrhs, static_cast<const double2*>(x), static_cast<double2*>(h),
                         static_cast<const double2*>(h_t));
    });
}

int vie_b1plus(vie_ctx* ctx, int nrhs, const void* h, void* b) {
    return guarded([&] {
        check(ctx);
        Ctx& c = ctx->c;
        VIE_HIP(hipSetDevice(c.device));
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(c.nc == 12, VIE_EINVAL, "b1+ is computed for the PWL basis");
        VIE_REQUIRE(nrhs >= 1 && h && b, VIE_EINVAL, "bad arguments");
        launch_b1plus(static_cast<double2*>(b), static_cast<const double2*>(h), kMu0, c.V, nrhs, c.stream);
    });
}

int vie_magnetic_energy(vie_ctx* ctx, int nrhs, const void* h, double* w_dev, double* W_host) {
    return guarded([&] {
        check(ctx);
        Ctx& c = ctx->c;
        VIE_HIP(hipSetDevice(c.device));
        VIE_REQUIRE(c.has_contrast, VIE_ESTATE, "the magnetic energy in the body needs vie_set_contrast");
        VIE_REQUIRE(c.nc == 12, VIE_EINVAL, "the magnetic energy is computed for the PWL basis");
        VIE_REQUIRE(nrhs >= 1 && h && (w_dev || W_host), VIE_EINVAL, "bad arguments");
        const int nb = 256;
        double* part = static_cast<double*>(c.small.get((size_t)nb * nrhs * sizeof(double)));
        launch_magnetic_energy(w_dev, part, static_cast<const double2*>(h), c.mat.chi, kMu0,
                               c.D[0] * c.D[1] * c.D[2], c.V, nrhs, nb, c.stream);
        if (W_host) {
            std::vector<double> hp((size_t)nb * nrhs);
            VIE_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            VIE_HIP(hipStreamSynchronize(c.stream));
            for (int r = 0; r < nrhs; ++r) {
                double s = 0;
                for (int k = 0; k < nb; ++k) s += hp[(size_t)r * nb + k];
                W_host[r] = s;
            }
        }
    });
}

int vie_get_curl_toeplitz(vie_ctx* ctx, double* T_host) {
    return guarded([&] {
        check(ctx);
        Ctx& c = ctx->c;
        VIE_HIP(hipSetDevice(c.device));
        VIE_REQUIRE(T_host != nullptr, VIE_EINVAL, "T_host is null");
        ensure_curl(c);
        VIE_HIP(hipMemcpyAsync(T_host, c.op->TK, 30 * c.V * sizeof(double2), hipMemcpyDeviceToHost, c.stream));
        VIE_HIP(hipStreamSynchronize(c.stream));
    });
}

}  // extern "C"
