// extern "C" entry points (include/vie.h).  Every call catches exceptions and
// turns them into a status code plus a thread-local message.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.hpp"

using namespace vie;

namespace vie {

thread_local std::string g_err;

Ctx::~Ctx() {
    free_grid();
    free_contrast();
    jmbuf.release();
    ws.release();
    small.release();
    basis.release();
    vecs.release();
    hpin.release();
    for (auto& e : col_ev)
        if (e) (void)hipEventDestroy(e);
    if (flag) (void)hipFree(flag);
}

void Ctx::free_grid() {
    graphs.clear();
    tucker.clear();
    free_mcontrast();
    op.reset();   // frees the operator unless another context shares it
    for (auto& a : ax) a = FftAxis{};
    T = nullptr;
    U128 = nullptr;
    U64 = nullptr;
    has_grid = false;
}

void Ctx::free_contrast() {
    graphs.clear();
    void* ps[] = {mat.eps_r, mat.chi, mat.tau, mat.tau64, mat.epsr64, mat.chi64, sigma};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    mat = Materials{};
    sigma = nullptr;
    has_contrast = false;
}

void Ctx::free_mcontrast() {
    graphs.clear();
    void* ps[] = {mmat.eps_r, mmat.chi, mmat.tau, mmat.tau64, mmat.epsr64, mmat.chi64};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    mmat = Materials{};
    has_mcontrast = false;
}

}  // namespace vie

static void check_ctx(vie_ctx* ctx) { VIE_REQUIRE(ctx != nullptr, VIE_EINVAL, "null context"); }

static void set_device(Ctx& c) { VIE_HIP(hipSetDevice(c.device)); }

// true when the byte ranges [a, a + na) and [b, b + nb) share a byte
static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
}

extern "C" {

const char* vie_last_error(void) { return g_err.c_str(); }

int vie_create(vie_ctx** out, int device, void* stream) {
    return guarded([&] {
        VIE_REQUIRE(out != nullptr, VIE_EINVAL, "out is null");
        int n = 0;
        VIE_HIP(hipGetDeviceCount(&n));
        VIE_REQUIRE(device >= 0 && device < n, VIE_EINVAL, "no such HIP device");
        auto* ctx = new vie_ctx();
        ctx->c.device = device;
        ctx->c.stream = static_cast<hipStream_t>(stream);
        try {
            set_device(ctx->c);
            noalloc_init(device);
            VIE_HIP(hipMalloc(&ctx->c.flag, sizeof(int)));
        } catch (...) {
            delete ctx;
            throw;
        }
        *out = ctx;
    });
}

void vie_destroy(vie_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    if (ctx->c.stream) (void)hipStreamSynchronize(ctx->c.stream);
    else (void)hipDeviceSynchronize();
    delete ctx;
}

int vie_set_stream(vie_ctx* ctx, void* stream) {
    return guarded([&] {
        check_ctx(ctx);
        ctx->c.stream = static_cast<hipStream_t>(stream);
    });
}

int vie_set_grid(vie_ctx* ctx, int nx, int ny, int nz, double dx, double dy, double dz, double freq_hz,
                 const int* fft_size) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, VIE_EINVAL, "grid extents must be >= 1");
        VIE_REQUIRE(std::isfinite(dx) && std::isfinite(dy) && std::isfinite(dz) && dx > 0 && dy > 0 && dz > 0,
                    VIE_EINVAL, "voxel sizes must be positive");
        VIE_REQUIRE(std::isfinite(freq_hz) && freq_hz > 0, VIE_EINVAL, "frequency must be positive");
        const int N[3] = {nx, ny, nz};
        int M[3];
        for (int i = 0; i < 3; ++i) {
            // default: the smallest even 2/3/5-smooth length >= 2N - 1 (2N when smooth)
            M[i] = fft_size ? fft_size[i] : 2 * N[i];
            if (!fft_size)
                while (!smooth235(M[i])) M[i] += 2;
        }
        // the PWC x pass exists for the compiled lengths only: a PWC context
        // takes the smallest compiled length >= 2 Nx along x when it has one
        if (!fft_size && c.nc == 3 && !p3_ct_supported(M[0]))
            for (int m = M[0]; m <= 512; m += 2)
                if (p3_ct_supported(m)) {
                    M[0] = m;
                    break;
                }
        for (int i = 0; i < 3; ++i) {
            VIE_REQUIRE(M[i] >= 2 * N[i] - 1 && M[i] % 2 == 0 && smooth235(M[i]), VIE_EINVAL,
                        "fft size must be even, 2/3/5-smooth and >= 2N-1");
            VIE_REQUIRE(M[i] <= 4096, VIE_EINVAL, "fft size above 4096 not supported");
        }
        if (c.stream) VIE_HIP(hipStreamSynchronize(c.stream));
        c.free_grid();
        c.free_contrast();
        for (int i = 0; i < 3; ++i) {
            c.N[i] = N[i];
            c.M[i] = M[i];
            c.O[i] = M[i] / 2 + 1;
        }
        c.D[0] = dx;
        c.D[1] = dy;
        c.D[2] = dz;
        c.freq = freq_hz;
        c.omega = 2.0 * M_PI * freq_hz;
        c.k0 = c.omega * std::sqrt(kMu0 * kEps0);
        c.V = (long long)nx * ny * nz;
        c.Osz = (long long)c.O[0] * c.O[1] * c.O[2];
        auto opd = std::make_shared<OperatorData>();
        for (int i = 0; i < 3; ++i) {
            opd->ax[i].plan = make_plan(M[i]);
            std::vector<double2> tw;
            make_twiddles(M[i], tw);
            std::vector<float2> tw32(M[i]);
            for (int k = 0; k < M[i]; ++k) tw32[k] = make_float2((float)tw[k].x, (float)tw[k].y);
            VIE_HIP(hipMalloc(&opd->ax[i].tw128, M[i] * sizeof(double2)));
            VIE_HIP(hipMalloc(&opd->ax[i].tw64, M[i] * sizeof(float2)));
            VIE_HIP(hipMemcpy(opd->ax[i].tw128, tw.data(), M[i] * sizeof(double2), hipMemcpyHostToDevice));
            VIE_HIP(hipMemcpy(opd->ax[i].tw64, tw32.data(), M[i] * sizeof(float2), hipMemcpyHostToDevice));
            opd->bytes += M[i] * (sizeof(double2) + sizeof(float2));
        }
        VIE_HIP(hipMalloc(&opd->T, 60 * c.V * sizeof(double2)));
        VIE_HIP(hipMalloc(&opd->U128, 60 * c.Osz * sizeof(double2)));
        VIE_HIP(hipMalloc(&opd->U64, 60 * c.Osz * sizeof(float2)));
        opd->bytes += 60 * c.V * sizeof(double2) + 60 * c.Osz * (sizeof(double2) + sizeof(float2));
        c.op = opd;
        for (int i = 0; i < 3; ++i) c.ax[i] = opd->ax[i];
        c.T = opd->T;
        c.U128 = opd->U128;
        c.U64 = opd->U64;
        AssemblyTables tab = build_assembly_tables(c.D, c.k0);
        assemble_blocks(c.T, tab, nx, ny, nz, c.stream);
        c.has_grid = true;
        // operator spectra
        const long long Mt = (long long)M[0] * M[1] * M[2];
        double2* circ = static_cast<double2*>(c.ws.get(Mt * sizeof(double2)));
        const double2* tws[3] = {c.ax[0].tw128, c.ax[1].tw128, c.ax[2].tw128};
        FftPlan plans[3] = {c.ax[0].plan, c.ax[1].plan, c.ax[2].plan};
        embed_and_transform(c.U128, c.U64, c.T, circ, nx, ny, nz, M[0], M[1], M[2], plans, tws, c.stream);
        VIE_HIP(hipStreamSynchronize(c.stream));
    });
}

int vie_share_grid(vie_ctx* dst, const vie_ctx* src) {
    return guarded([&] {
        check_ctx(dst);
        VIE_REQUIRE(src != nullptr && src != dst, VIE_EINVAL, "bad source context");
        const Ctx& s = src->c;
        Ctx& c = dst->c;
        VIE_REQUIRE(s.has_grid, VIE_ESTATE, "source context has no grid");
        VIE_REQUIRE(s.device == c.device, VIE_EINVAL, "contexts on different devices");
        set_device(c);
        if (s.stream) VIE_HIP(hipStreamSynchronize(s.stream));   // operator complete
        if (c.stream) VIE_HIP(hipStreamSynchronize(c.stream));
        std::shared_ptr<OperatorData> keep = s.op;                // src may equal a context sharing dst's op
        c.free_grid();
        c.free_contrast();
        for (int i = 0; i < 3; ++i) {
            c.N[i] = s.N[i];
            c.M[i] = s.M[i];
            c.O[i] = s.O[i];
            c.D[i] = s.D[i];
            c.ax[i] = s.ax[i];
        }
        c.freq = s.freq;
        c.omega = s.omega;
        c.k0 = s.k0;
        c.V = s.V;
        c.Osz = s.Osz;
        c.op = keep;
        c.T = s.T;
        c.U128 = s.U128;
        c.U64 = s.U64;
        c.tune = s.tune;
        c.has_grid = true;
    });
}

int vie_set_toeplitz(vie_ctx* ctx, const double* T_host) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "vie_set_toeplitz before vie_set_grid");
        VIE_REQUIRE(c.op.use_count() == 1, VIE_ESTATE, "the operator is shared with another context");
        VIE_REQUIRE(T_host != nullptr, VIE_EINVAL, "T_host is null");
        VIE_HIP(hipMemcpyAsync(c.T, T_host, 60 * c.V * sizeof(double2), hipMemcpyHostToDevice, c.stream));
        const long long Mt = (long long)c.M[0] * c.M[1] * c.M[2];
        double2* circ = static_cast<double2*>(c.ws.get(Mt * sizeof(double2)));
        const double2* tws[3] = {c.ax[0].tw128, c.ax[1].tw128, c.ax[2].tw128};
        FftPlan plans[3] = {c.ax[0].plan, c.ax[1].plan, c.ax[2].plan};
        embed_and_transform(c.U128, c.U64, c.T, circ, c.N[0], c.N[1], c.N[2], c.M[0], c.M[1], c.M[2], plans, tws,
                            c.stream);
        VIE_HIP(hipStreamSynchronize(c.stream));
    });
}

int vie_get_toeplitz(vie_ctx* ctx, double* T_host) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(T_host != nullptr, VIE_EINVAL, "T_host is null");
        VIE_HIP(hipMemcpyAsync(T_host, c.T, 60 * c.V * sizeof(double2), hipMemcpyDeviceToHost, c.stream));
        VIE_HIP(hipStreamSynchronize(c.stream));
    });
}

int vie_tucker_compress(vie_ctx* ctx, double tol, vie_tucker_info* info) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "vie_tucker_compress before vie_set_grid");
        VIE_REQUIRE(tol >= 1e-7 && tol < 1.0, VIE_EINVAL, "tol must be in [1e-7, 1)");
        const auto t0 = std::chrono::steady_clock::now();
        tucker_compress(c, tol);
        if (info) {
            *info = vie_tucker_info{};
            double worst = 0;
            for (int e = 0; e < 60; ++e) {
                const TuckerTensor& t = c.tucker.tensors[e];
                for (int i = 0; i < 3; ++i) info->ranks[e][i] = t.r[i];
                info->rel_error[e] = t.rel_error;
                worst = std::max(worst, t.rel_error);
            }
            info->max_rel_error = worst;
            info->bytes_dense = (size_t)60 * c.V * sizeof(double2);
            info->bytes_compressed = c.tucker.values() * sizeof(double2);
            info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
    });
}

int vie_tucker_reconstruct(vie_ctx* ctx, void* out) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(out != nullptr, VIE_EINVAL, "out is null");
        VIE_REQUIRE(!overlaps(out, 60 * c.V * sizeof(double2), c.T, 60 * c.V * sizeof(double2)), VIE_EINVAL,
                    "out overlaps the context's blocks");
        tucker_reconstruct(c, static_cast<double2*>(out));
        VIE_HIP(hipStreamSynchronize(c.stream));
    });
}

int vie_tucker_expand(vie_ctx* ctx) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(c.tucker.valid, VIE_ESTATE, "no Tucker form: call vie_tucker_compress first");
        VIE_REQUIRE(c.op.use_count() == 1, VIE_ESTATE, "the operator is shared with another context");
        // T <- T_hat, then the set-up's embedding, FFT and octant
        tucker_reconstruct(c, c.T);
        const long long Mt = (long long)c.M[0] * c.M[1] * c.M[2];
        double2* circ = static_cast<double2*>(c.ws.get(Mt * sizeof(double2)));
        const double2* tws[3] = {c.ax[0].tw128, c.ax[1].tw128, c.ax[2].tw128};
        FftPlan plans[3] = {c.ax[0].plan, c.ax[1].plan, c.ax[2].plan};
        embed_and_transform(c.U128, c.U64, c.T, circ, c.N[0], c.N[1], c.N[2], c.M[0], c.M[1], c.M[2], plans, tws,
                            c.stream);
        VIE_HIP(hipStreamSynchronize(c.stream));
    });
}

int vie_set_contrast(vie_ctx* ctx, const double* eps_re, const double* sigma, int on_device) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "vie_set_contrast before vie_set_grid");
        VIE_REQUIRE(eps_re && sigma, VIE_EINVAL, "null material array");
        c.free_contrast();
        const size_t V = (size_t)c.V;
        VIE_HIP(hipMalloc(&c.mat.eps_r, V * sizeof(double2)));
        VIE_HIP(hipMalloc(&c.mat.chi, V * sizeof(double2)));
        VIE_HIP(hipMalloc(&c.mat.tau, V * sizeof(double2)));
        VIE_HIP(hipMalloc(&c.mat.tau64, V * sizeof(float2)));
        VIE_HIP(hipMalloc(&c.mat.epsr64, V * sizeof(float2)));
        VIE_HIP(hipMalloc(&c.mat.chi64, V * sizeof(float2)));
        VIE_HIP(hipMalloc(&c.sigma, V * sizeof(double)));
        double* eps_dev = static_cast<double*>(c.small.get(V * sizeof(double)));
        const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        VIE_HIP(hipMemcpyAsync(eps_dev, eps_re, V * sizeof(double), k, c.stream));
        VIE_HIP(hipMemcpyAsync(c.sigma, sigma, V * sizeof(double), k, c.stream));
        VIE_HIP(hipMemsetAsync(c.flag, 0, sizeof(int), c.stream));
        launch_materials(eps_dev, c.sigma, c.omega * kEps0, c.mat, c.V, c.flag, c.stream);
        int bad = 0;
        VIE_HIP(hipMemcpyAsync(&bad, c.flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        VIE_HIP(hipStreamSynchronize(c.stream));
        if (bad) {
            c.free_contrast();
            if (bad & 1) throw Error(VIE_ENAN, "non-finite permittivity or conductivity");
            throw Error(VIE_EINVAL, "permittivity must be > 0 and conductivity >= 0");
        }
        c.has_contrast = true;
        if (c.nc == 24 && !c.has_mcontrast) jm_default_mcontrast(c);
    });
}

int vie_set_magnetic_contrast(vie_ctx* ctx, const double* mu_re, const double* mu_im, int on_device) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "vie_set_magnetic_contrast before vie_set_grid");
        VIE_REQUIRE(c.nc == 24, VIE_EINVAL, "a magnetic contrast needs the J-M formulation (vie_set_basis 24)");
        VIE_REQUIRE(mu_re && mu_im, VIE_EINVAL, "null material array");
        c.free_mcontrast();
        const size_t V = (size_t)c.V;
        Materials& m = c.mmat;
        VIE_HIP(hipMalloc(&m.eps_r, V * sizeof(double2)));
        VIE_HIP(hipMalloc(&m.chi, V * sizeof(double2)));
        VIE_HIP(hipMalloc(&m.tau, V * sizeof(double2)));
        VIE_HIP(hipMalloc(&m.tau64, V * sizeof(float2)));
        VIE_HIP(hipMalloc(&m.epsr64, V * sizeof(float2)));
        VIE_HIP(hipMalloc(&m.chi64, V * sizeof(float2)));
        double* dev = static_cast<double*>(c.small.get(2 * V * sizeof(double)));
        const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        VIE_HIP(hipMemcpyAsync(dev, mu_re, V * sizeof(double), k, c.stream));
        VIE_HIP(hipMemcpyAsync(dev + V, mu_im, V * sizeof(double), k, c.stream));
        VIE_HIP(hipMemsetAsync(c.flag, 0, sizeof(int), c.stream));
        // mu_r = mu' - i mu'' (eq. 2): the permittivity kernel with sigma / (w eps0) -> mu''
        launch_materials(dev, dev + V, 1.0, m, c.V, c.flag, c.stream);
        int bad = 0;
        VIE_HIP(hipMemcpyAsync(&bad, c.flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        VIE_HIP(hipStreamSynchronize(c.stream));
        if (bad) {
            c.free_mcontrast();
            if (bad & 1) throw Error(VIE_ENAN, "non-finite permeability");
            throw Error(VIE_EINVAL, "mu' must be > 0 and mu'' >= 0");
        }
        c.has_mcontrast = true;
    });
}

static int axis_of(const double v[3]) {
    int ax = -1, nz = 0;
    for (int i = 0; i < 3; ++i)
        if (v[i] != 0.0) {
            ax = i;
            ++nz;
        }
    return (nz == 1 && std::fabs(std::fabs(v[ax]) - 1.0) < 1e-12) ? ax : -1;
}

static double sign_of(double v) { return v < 0 ? -1.0 : 1.0; }

int vie_incident_planewave(vie_ctx* ctx, const double pol[3], const double dir[3], double amp, void* e_t) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(pol && dir && e_t, VIE_EINVAL, "null argument");
        const int pa = axis_of(pol), da = axis_of(dir);
        VIE_REQUIRE(pa >= 0 && da >= 0 && pa != da, VIE_EINVAL,
                    "pol and dir must be distinct unit vectors along coordinate axes");
        double2* et = static_cast<double2*>(e_t);
        launch_planewave(et, c.N[0], c.N[1], c.N[2], c.D, c.k0, pa, da, dir[da] > 0 ? 1.0 : -1.0,
                         amp * sign_of(pol[pa]), c.nc == 24 ? 12 : c.nc, c.stream);
        if (c.nc == 24) planewave_h(c, pol, dir, amp, et + 12 * c.V);   // J-M: [e_t; h_t]
    });
}

int vie_incident_dipoles(vie_ctx* ctx, int nrhs, const double* pos, const double* moment, int nq, void* e_t) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid && c.has_contrast, VIE_ESTATE, "dipoles need grid and contrast");
        VIE_REQUIRE(nrhs >= 1 && pos && moment && e_t, VIE_EINVAL, "bad dipole arguments");
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
        if (c.nc == 24) {   // J-M: per right-hand side the tested e (on tissue) and h (everywhere)
            for (int r = 0; r < nrhs; ++r) {
                double2* et = static_cast<double2*>(e_t) + (long long)r * 24 * c.V;
                launch_dipoles(et, 1, dev + 3 * r, dev + 3 * nrhs + 3 * r, nq, dev + 6 * nrhs, dev + 6 * nrhs + nq,
                               c.mat.chi, c.N[0], c.N[1], c.N[2], c.D, c.k0, c.omega * kEps0, 12, c.stream);
                launch_dipoles(et + 12 * c.V, 1, dev + 3 * r, dev + 3 * nrhs + 3 * r, nq, dev + 6 * nrhs,
                               dev + 6 * nrhs + nq, nullptr, c.N[0], c.N[1], c.N[2], c.D, c.k0, c.omega * kEps0, 12,
                               c.stream, 1);
            }
        } else {
            launch_dipoles(static_cast<double2*>(e_t), nrhs, dev, dev + 3 * nrhs, nq, dev + 6 * nrhs,
                           dev + 6 * nrhs + nq, c.mat.chi, c.N[0], c.N[1], c.N[2], c.D, c.k0, c.omega * kEps0, c.nc,
                           c.stream);
        }
        VIE_HIP(hipStreamSynchronize(c.stream));   // the host staging buffer is reused
    });
}

int vie_rhs_prec(vie_ctx* ctx, int nrhs, const void* e_t, void* rhs) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_contrast, VIE_ESTATE, "no contrast");
        VIE_REQUIRE(nrhs >= 1 && e_t && rhs, VIE_EINVAL, "bad arguments");
        if (c.nc == 24) {
            jm_rhs_prec(c, nrhs, static_cast<const double2*>(e_t), static_cast<double2*>(rhs));
            return;
        }
        const double dv = c.D[0] * c.D[1] * c.D[2];
        const double ginv[4] = {1 / dv, 12 / dv, 12 / dv, 12 / dv};
        launch_rhs_prec(static_cast<double2*>(rhs), static_cast<const double2*>(e_t), c.mat.tau, ginv,
                        make_double2(0.0, c.omega * kEps0), c.V, nrhs, c.nc, c.stream);
    });
}

int vie_apply(vie_ctx* ctx, int op, int precision, int nrhs, const void* x, void* y) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(op == VIE_OP_PREC || op == VIE_OP_A || op == VIE_OP_N, VIE_EINVAL, "unknown operator");
        VIE_REQUIRE(nrhs >= 1 && x && y, VIE_EINVAL, "bad arguments");
        VIE_REQUIRE(precision == VIE_C64 || precision == VIE_C128, VIE_EINVAL,
                    "precision must be VIE_C64 or VIE_C128");
        if (c.has_grid) {
            const size_t bytes = (size_t)nrhs * c.nc * c.V * (precision == VIE_C64 ? 8 : 16);
            VIE_REQUIRE(!overlaps(x, bytes, y, bytes), VIE_EINVAL, "x and y must not overlap");
        }
        if (precision == VIE_C64)
            apply_op<float>(c, op, nrhs, static_cast<const float2*>(x), static_cast<float2*>(y), nullptr);
        else if (precision == VIE_C128)
            apply_op<double>(c, op, nrhs, static_cast<const double2*>(x), static_cast<double2*>(y), nullptr);
        else
            throw Error(VIE_EINVAL, "precision must be VIE_C64 or VIE_C128");
    });
}

void vie_default_opts(vie_solve_opts* o) {
    if (!o) return;
    o->mode = VIE_SOLVE_FP64;
    o->restart = 50;
    o->max_outer = 200;
    o->tol = 1e-6;
    o->inner_tol = 1e-5;
    o->max_refine = 400;
    o->reorth = 0;
    o->use_x0 = 0;
    o->graph = -1;
    o->sync_steps = 0;
    o->s_step = 0;
}

int vie_solve(vie_ctx* ctx, const vie_solve_opts* opts, int nrhs, const void* e_t, void* x, vie_solve_stats* stats) {
    int rc = VIE_OK;
    int g = guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid && c.has_contrast, VIE_ESTATE, "solve needs grid and contrast");
        VIE_REQUIRE(nrhs >= 1 && e_t && x, VIE_EINVAL, "bad arguments");
        vie_solve_opts o;
        if (opts) o = *opts;
        else vie_default_opts(&o);
        VIE_REQUIRE(o.restart >= 1 && o.restart <= 200, VIE_EINVAL, "restart must be in 1..200");
        VIE_REQUIRE(o.max_outer >= 1 && o.tol > 0 && o.tol < 1, VIE_EINVAL, "bad tolerance or max_outer");
        VIE_REQUIRE(o.mode == VIE_SOLVE_FP64 || o.mode == VIE_SOLVE_FP32_IR, VIE_EINVAL, "unknown mode");
        VIE_REQUIRE(o.mode != VIE_SOLVE_FP32_IR || o.max_refine >= 1, VIE_EINVAL, "max_refine must be >= 1");
        VIE_REQUIRE(o.sync_steps >= 0, VIE_EINVAL, "sync_steps must be >= 0");
        VIE_REQUIRE(o.s_step >= 0 && o.s_step <= 3, VIE_EINVAL, "s_step must be 0, 1, 2 or 3");
        rc = solve(c, o, nrhs, static_cast<const double2*>(e_t), static_cast<double2*>(x), stats);
        if (rc == VIE_ENOCONV) g_err = "solver stopped before reaching the tolerance";
        if (rc == VIE_ENAN) g_err = "non-finite residual";
    });
    return g != VIE_OK ? g : rc;
}

int vie_fields(vie_ctx* ctx, int nrhs, const void* x, void* e) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_contrast, VIE_ESTATE, "no contrast");
        VIE_REQUIRE(nrhs >= 1 && x && e, VIE_EINVAL, "bad arguments");
        if (c.nc == 24) {   // J-M: e = x_j / (c_e chi_e), h = x_m / (c_m chi_m)
            for (int r = 0; r < nrhs; ++r) {
                const long long o = (long long)r * 24 * c.V, h = 12 * c.V;
                launch_fields(static_cast<double2*>(e) + o, static_cast<const double2*>(x) + o, c.mat.chi,
                              make_double2(0.0, c.omega * kEps0), c.V, 1, 12, c.stream);
                launch_fields(static_cast<double2*>(e) + o + h, static_cast<const double2*>(x) + o + h, c.mmat.chi,
                              make_double2(0.0, c.omega * kMu0), c.V, 1, 12, c.stream);
            }
            return;
        }
        launch_fields(static_cast<double2*>(e), static_cast<const double2*>(x), c.mat.chi,
                      make_double2(0.0, c.omega * kEps0), c.V, nrhs, c.nc, c.stream);
    });
}

int vie_total_field(vie_ctx* ctx, int nrhs, const void* e_t, const void* x, void* e) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid");
        VIE_REQUIRE(c.nc != 24, VIE_EINVAL, "the total field is computed for the dielectric formulation");
        VIE_REQUIRE(nrhs >= 1 && e_t && x && e, VIE_EINVAL, "bad arguments");
        const size_t bytes = (size_t)nrhs * c.nc * c.V * sizeof(double2);
        VIE_REQUIRE(!overlaps(e, bytes, x, bytes) && !overlaps(e, bytes, e_t, bytes), VIE_EINVAL,
                    "e must not overlap x or e_t (it receives N x before e_t is read)");
        apply_op<double>(c, OP_N, nrhs, static_cast<const double2*>(x), static_cast<double2*>(e), nullptr);
        const double dv = c.D[0] * c.D[1] * c.D[2];
        const double gram[4] = {dv, dv / 12, dv / 12, dv / 12};
        launch_total_field(static_cast<double2*>(e), static_cast<const double2*>(e_t), static_cast<const double2*>(x),
                           gram, make_double2(0.0, c.omega * kEps0), c.V, nrhs, c.nc, c.stream);
    });
}

int vie_absorbed_power(vie_ctx* ctx, int nrhs, const void* x, double* p_abs_host) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_contrast, VIE_ESTATE, "no contrast");
        VIE_REQUIRE(nrhs >= 1 && x && p_abs_host, VIE_EINVAL, "bad arguments");
        const int nb = 256;
        const int halves = c.nc == 24 ? 2 : 1;
        double* part = static_cast<double*>(c.small.get((size_t)nb * nrhs * halves * sizeof(double)));
        const double dv = c.D[0] * c.D[1] * c.D[2];
        const double gram[4] = {dv, dv / 12, dv / 12, dv / 12};
        if (c.nc == 24) {   // J-M: the electric and the magnetic loss, each half on its own
            for (int r = 0; r < nrhs; ++r)
                for (int hh = 0; hh < 2; ++hh)
                    launch_power_partials(part + (size_t)(2 * r + hh) * nb,
                                          static_cast<const double2*>(x) + ((long long)r * 24 + 12 * hh) * c.V,
                                          hh ? c.mmat.chi : c.mat.chi, gram,
                                          make_double2(0.0, c.omega * (hh ? kMu0 : kEps0)), c.V, 1, 12, nb, c.stream);
        } else {
            launch_power_partials(part, static_cast<const double2*>(x), c.mat.chi, gram,
                                  make_double2(0.0, c.omega * kEps0), c.V, nrhs, c.nc, nb, c.stream);
        }
        std::vector<double> h((size_t)nb * nrhs * halves);
        VIE_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        VIE_HIP(hipStreamSynchronize(c.stream));
        for (int r = 0; r < nrhs; ++r) {
            double s = 0;
            for (int b = 0; b < nb * halves; ++b) s += h[(size_t)r * nb * halves + b];
            p_abs_host[r] = s;
        }
    });
}

int vie_power_density(vie_ctx* ctx, int nrhs, const void* e, double* p_dev) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_contrast, VIE_ESTATE, "no contrast");
        VIE_REQUIRE(c.nc != 24, VIE_EINVAL, "the power density is computed for the dielectric formulation");
        VIE_REQUIRE(nrhs >= 1 && e && p_dev, VIE_EINVAL, "bad arguments");
        launch_power_density(p_dev, static_cast<const double2*>(e), c.sigma, c.V, nrhs, c.nc, c.stream);
    });
}

int vie_copy(vie_ctx* ctx, const void* src, void* dst, long long n) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(src && dst && n >= 0, VIE_EINVAL, "bad copy arguments");
        if (n > 0) launch_copy_c128(static_cast<double2*>(dst), static_cast<const double2*>(src), n, c.stream);
    });
}

int vie_autotune(vie_ctx* ctx, int precision, int nrhs, int* choice, double* best_ms) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "autotune needs a grid");
        VIE_REQUIRE(precision == VIE_C64 || precision == VIE_C128, VIE_EINVAL, "bad precision");
        VIE_REQUIRE(nrhs >= 1, VIE_EINVAL, "nrhs must be >= 1");
        // a J-M product runs its 2 nrhs halves as 12-component products
        const int jm = c.nc == 24;
        NcGuard g(c, jm ? 12 : c.nc);
        Tune t = autotune(c, precision, jm ? 2 * nrhs : nrhs, best_ms);
        if (choice) {
            choice[0] = t.p3_variant;
            choice[1] = t.p3_sib_blocks;
            choice[2] = t.tile_z;
            choice[3] = t.tile_y;
        }
    });
}

int vie_set_basis(vie_ctx* ctx, int ncomp) {
    return guarded([&] {
        check_ctx(ctx);
        VIE_REQUIRE(ncomp == 12 || ncomp == 3 || ncomp == 24, VIE_EINVAL,
                    "ncomp must be 12 (PWL), 3 (PWC) or 24 (PWL, J-M formulation)");
        Ctx& c = ctx->c;
        set_device(c);
        c.nc = ncomp;
        c.tune.clear();
        c.graphs.clear();
        c.free_mcontrast();
        if (ncomp == 24 && c.has_contrast) jm_default_mcontrast(c);
    });
}

int vie_fft_size(vie_ctx* ctx, int* m3) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "no grid set");
        VIE_REQUIRE(m3 != nullptr, VIE_EINVAL, "null output");
        for (int i = 0; i < 3; ++i) m3[i] = c.M[i];
    });
}

int vie_set_tuning(vie_ctx* ctx, int precision, int nrhs, const int* choice) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "tuning needs a grid");
        VIE_REQUIRE(precision == VIE_C64 || precision == VIE_C128, VIE_EINVAL, "bad precision");
        VIE_REQUIRE(nrhs >= 1 && choice, VIE_EINVAL, "bad arguments");
        const int es = precision == VIE_C64 ? 8 : 16;
        Tune t;
        t.p3_variant = choice[0];
        t.p3_sib_blocks = choice[1];
        t.tile_z = choice[2];
        t.tile_y = choice[3];
        VIE_REQUIRE(t.p3_variant >= 0 && t.p3_variant <= 5, VIE_EINVAL, "unknown x-pass variant");
        VIE_REQUIRE(t.p3_variant != 5 || p3_pair_fits(es, c.M[0]), VIE_EINVAL,
                    "the right-hand-side pair variant needs a compiled x length whose 24 rows fit LDS");
        VIE_REQUIRE(t.p3_variant != 0 || !p3_ct_supported(c.M[0]) || p3_ct_fits(es, c.M[0]), VIE_EINVAL,
                    "x-pass variant 0 does not fit LDS for this fft length and precision");
        VIE_REQUIRE(t.p3_variant != 3 || p3_pref_fits(c.M[0]), VIE_EINVAL,
                    "x-pass variant 3 needs an fft length <= 128 along x");
        VIE_REQUIRE(t.p3_variant == 0 || p3_ct_supported(c.M[0]), VIE_EINVAL,
                    "x-pass variants 1 to 4 need a compiled fft length along x");
        VIE_REQUIRE(t.p3_variant != 2 || p3_quad_fits(es, c.M[0]), VIE_EINVAL,
                    "x-pass variant 2 is complex64 only and needs its rows to fit LDS");
        VIE_REQUIRE(t.p3_sib_blocks == 1 || (t.p3_variant == 0 && (t.p3_sib_blocks == 2 || t.p3_sib_blocks == 4)),
                    VIE_EINVAL, "workgroups per row must be 1 (or 2, 4 for variant 0)");
        VIE_REQUIRE(strided_tile_ok(es, c.M[2], t.tile_z) && strided_tile_ok(es, c.M[1], t.tile_y), VIE_EINVAL,
                    "tile not available for this fft size (8 or 16, or 32 with a compiled length)");
        c.graphs.clear();
        c.tune[{precision == VIE_C64 ? 0 : 1, c.nc == 24 ? 2 * nrhs : nrhs}] = t;
    });
}

int vie_profile(vie_ctx* ctx, int enable) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(enable >= 0, VIE_EINVAL, "enable must be >= 0");
        VIE_HIP(hipStreamSynchronize(c.stream));
        if (enable) c.prof.clear();
        c.prof.on = enable != 0;
        c.prof.every = enable > 0 ? enable : 1;
        for (auto& t : c.prof.tick) t = 0;
    });
}

int vie_profile_read(vie_ctx* ctx, int kind, double* total_ms, int* launches, double* bytes) {
    return guarded([&] {
        check_ctx(ctx);
        Ctx& c = ctx->c;
        set_device(c);
        VIE_REQUIRE(kind >= 0 && kind < VIE_K_COUNT, VIE_EINVAL, "unknown kernel class");
        VIE_HIP(hipStreamSynchronize(c.stream));
        double ms = 0, b = 0;
        int n = 0;
        for (const auto& r : c.prof.recs) {
            if (r.kind != kind) continue;
            float t = 0;
            VIE_HIP(hipEventElapsedTime(&t, r.a, r.b));
            ms += t;
            b += r.bytes;
            ++n;
        }
        if (total_ms) *total_ms = ms;
        if (launches) *launches = n;
        if (bytes) *bytes = b;
    });
}

size_t vie_unknowns_bytes_basis(int nx, int ny, int nz, int ncomp) {
    if (nx < 1 || ny < 1 || nz < 1 || (ncomp != 12 && ncomp != 3)) return 0;
    return (size_t)ncomp * 8 * (size_t)nx * ny * nz * 16;
}

size_t vie_unknowns_bytes_paper(int nx, int ny, int nz) { return vie_unknowns_bytes_basis(nx, ny, nz, 12); }

int vie_footprint_bytes(int nx, int ny, int nz, int nrhs, int mode, int restart, size_t* out) {
    return guarded([&] {
        VIE_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nrhs >= 1 && restart >= 1 && out, VIE_EINVAL, "bad arguments");
        const size_t V = (size_t)nx * ny * nz;
        const size_t M = 8 * V;
        const size_t O = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
        const size_t n = 12 * V;
        const size_t s = (mode == VIE_SOLVE_FP32_IR) ? 8 : 16;
        size_t b = 0;
        b += 60 * V * 16;                 // block tensors
        b += 60 * O * (16 + 8);           // octant spectra, both precisions
        b += V * (3 * 16 + 3 * 8 + 8);    // materials
        b += M * 16;                      // set-up circulant (reused as FFT workspace)
        // FFT intermediates ([B][Mz][Ny][Nx] + [B][Mz][My][Nx] = 6 n per rhs)
        const size_t fft = 6 * n * nrhs * s;
        const size_t fft128 = 6 * n * nrhs * 16;   // refinement residual in complex128
        b += (mode == VIE_SOLVE_FP32_IR) ? std::max(fft, fft128) : fft;
        b += (size_t)(restart + 1) * (n * nrhs * s + 4352);  // Krylov basis (staggered)
        b += 2 * n * nrhs * 16;                      // residual and right-hand side (complex128)
        *out = b;
    });
}

}  // extern "C"
