// The FFT-accelerated operator product (Sec. IV-A) as five passes:
//   P1  FFT along z, input zero-padded from Nz to Mz      [B][Nz][Ny][Nx] -> [B][Mz][Ny][Nx]
//   P2  FFT along y, input zero-padded from Ny to My      -> [B][Mz][My][Nx]
//   P3  FFT along x (padded), 12 x 12 block product with the circulant
//       spectrum at every frequency, inverse FFT along x, crop to Nx (in place)
//   P4  inverse FFT along y, crop to Ny                   -> [B][Mz][Ny][Nx]
//   P5  inverse FFT along z, crop to Nz, then the epilogue that forms the
//       requested operator from w = N x (Sec. IV-B):
//         PREC:  y = x - tau G^-1 w               (P^-1 A, eq. 17)
//         A:     y = eps_r G x - chi w            (eq. 24a)
//         N:     y = w                            (eq. 25a)
//         RESID: y = rhs - (x - tau G^-1 w)       (refinement residual)
// B = nc nrhs component arrays (nc = 12 unknowns per voxel for the PWL basis,
// 3 for the PWC basis, whose x pass applies the 3 x 3 blocks of the constant
// functions); the 1/(Mx My Mz) of the inverse FFT is folded into the
// epilogue.
#include <algorithm>
#include <string>

#include "ctx.hpp"
#include "fft_ct.hpp"

namespace vie {

template <typename R> static const C<R>* twid(const FftAxis& a);
template <> const C<float>* twid<float>(const FftAxis& a) { return a.tw64; }
template <> const C<double>* twid<double>(const FftAxis& a) { return a.tw128; }
template <typename R> static const C<R>* opspec(const Ctx& c);
template <> const C<float>* opspec<float>(const Ctx& c) { return c.U64; }
template <> const C<double>* opspec<double>(const Ctx& c) { return c.U128; }
template <typename R> static const C<R>* curlspec(const Ctx& c);
template <> const C<float>* curlspec<float>(const Ctx& c) { return c.op->UK64; }
template <> const C<double>* curlspec<double>(const Ctx& c) { return c.op->UK128; }

static int pick_tile(int n, size_t elem) { return strided_tile_for((int)elem, n, 16); }

// bytes of FFT intermediates one product of nrhs vectors needs (layouts below)
size_t apply_workspace_bytes(const Ctx& c, int nrhs, size_t es) {
    const long long row = (long long)c.nc * c.N[0];
    const long long sR1 = (long long)c.M[2] * ((long long)c.N[1] * row + 32) + 96;
    const long long sR2 = (long long)c.M[2] * ((long long)c.M[1] * row + 32) + 96;
    return (size_t)nrhs * (size_t)(sR1 + sR2) * es;
}

template <typename R>
void apply_op(Ctx& c, int op, int nrhs, const C<R>* x, C<R>* y, const C<R>* rhs, void* ws_ext, size_t ws_cap) {
    Tune tn;
    {
        auto it = c.tune.find({sizeof(R) == 4 ? 0 : 1, nrhs});
        if (it != c.tune.end()) tn = it->second;
    }
    VIE_REQUIRE(c.has_grid, VIE_ESTATE, "vie_apply before vie_set_grid");
    if (c.nc == 24) {   // J-M formulation: composed from N and K products
        apply_jm<R>(c, op, nrhs, x, y, rhs, ws_ext, ws_cap);
        return;
    }
    if (op != OP_N && op != OP_CURL && op != OP_K && op != OP_JMS)
        VIE_REQUIRE(c.has_contrast, VIE_ESTATE, "operator needs vie_set_contrast");
    if (op == OP_JMS) {
        VIE_REQUIRE(c.nc == 12 && nrhs % 2 == 0 && c.op && curlspec<R>(c) && jm_fused_supported(c, sizeof(C<R>)),
                    VIE_EINVAL, "the fused J-M sums need vector pairs on a compiled x length");
    }
    if (op == OP_CURL) {
        VIE_REQUIRE(sizeof(R) == 8 && c.nc == 12, VIE_EINVAL,
                    "the magnetic product is complex128 and PWL (12 unknowns per voxel) only");
        VIE_REQUIRE(c.op && c.op->UK128, VIE_ESTATE, "curl operator not built");
    }
    if (op == OP_K) {
        VIE_REQUIRE(c.nc == 12, VIE_EINVAL, "the curl product is PWL (12 unknowns per voxel) only");
        VIE_REQUIRE(c.op && curlspec<R>(c), VIE_ESTATE, "curl operator not built");
    }
    const int Nx = c.N[0], Ny = c.N[1], Nz = c.N[2];
    const int Mx = c.M[0], My = c.M[1], Mz = c.M[2];
    const int nc = c.nc;
    const long long B = (long long)nc * nrhs;
    // intermediate layouts per right-hand side [Mz][Ny|My][nc][Nx]: the nc
    // components of one (z, y) row are adjacent, so a pencil group of the x
    // pass is one contiguous block; planes are padded so that rows used
    // together are not a large power of two apart
    const long long row = (long long)nc * Nx;
    const long long pl1 = (long long)Ny * row + 32, pl2 = (long long)My * row + 32;
    const long long sR1 = (long long)Mz * pl1 + 96;   // per right-hand side, after P1 / P4
    const long long sR2 = (long long)Mz * pl2 + 96;   // after P2 / P3
    const size_t es = sizeof(C<R>);
    const size_t need = apply_workspace_bytes(c, nrhs, es);
    char* ws = nullptr;
    if (ws_ext) {
        VIE_REQUIRE(need <= ws_cap, VIE_EINVAL,
                    "product needs " + std::to_string(need) + " workspace bytes, above the fixed limit of " +
                        std::to_string(ws_cap));
        ws = static_cast<char*>(ws_ext);
    } else {
        ws = static_cast<char*>(c.ws.get(need));
    }
    C<R>* A1 = reinterpret_cast<C<R>*>(ws);
    C<R>* A2 = reinterpret_cast<C<R>*>(ws + (size_t)nrhs * sR1 * es);
    hipStream_t s = c.stream;
    const long long V = c.V;

    // P1: z
    StridedPass p1{};
    p1.plan = c.ax[2].plan;
    p1.n_in = Nz;
    p1.n_out = Mz;
    p1.n_inner = Nx;
    p1.tile = tn.tile_z ? tn.tile_z : pick_tile(Mz, es);
    p1.pitch = p1.tile;
    p1.nc = nc;
    p1.in_s1 = nc * V;
    p1.in_sc = V;
    p1.in_s2 = Nx;
    p1.in_sk = (long long)Ny * Nx;
    p1.out_s1 = sR1;
    p1.out_sc = Nx;
    p1.out_s2 = row;
    p1.out_sk = pl1;
    const double bV = (double)B * V * es, bA1 = (double)B * Mz * Ny * Nx * es, bA2 = (double)B * Mz * My * Nx * es;
    {
        KernelTiming kt(c.prof, VIE_K_FFT_Z_FWD, bV + bA1);
        launch_strided<R>(true, x, A1, p1, Ny, B, twid<R>(c.ax[2]), nullptr, s);
    }

    // P2: y
    StridedPass p2{};
    p2.plan = c.ax[1].plan;
    p2.nc = nc;
    p2.n_in = Ny;
    p2.n_out = My;
    p2.n_inner = Nx;
    p2.tile = tn.tile_y ? tn.tile_y : pick_tile(My, es);
    p2.pitch = p2.tile;
    p2.in_s1 = sR1;
    p2.in_sc = Nx;
    p2.in_s2 = pl1;
    p2.in_sk = row;
    p2.out_s1 = sR2;
    p2.out_sc = Nx;
    p2.out_s2 = pl2;
    p2.out_sk = row;
    {
        KernelTiming kt(c.prof, VIE_K_FFT_Y_FWD, bA1 + bA2);
        launch_strided<R>(true, A1, A2, p2, Mz, B, twid<R>(c.ax[1]), nullptr, s);
    }

    // P3: x, block product
    P3Params p3{};
    p3.plan = c.ax[0].plan;
    p3.Nx = Nx;
    p3.My = My;
    p3.Mz = Mz;
    p3.Ox = c.O[0];
    p3.Oy = c.O[1];
    p3.Oz = c.O[2];
    p3.nrhs = nrhs;
    p3.s_r = sR2;
    p3.s_c = Nx;
    p3.s_z = pl2;
    p3.s_y = row;
    p3.u_e = c.O[0];
    p3.pitch = Mx;
    if (op == OP_JMS) {
        // both halves of each pair in one workgroup: the 30 curl and the 60
        // N tensors per frequency
        p3.nrhs = nrhs / 2;
        KernelTiming kt(c.prof, VIE_K_BLOCK, 2 * bA2 + 90.0 * c.Osz * es);
        const bool ok = launch_p3_jm<R>(A2, opspec<R>(c), curlspec<R>(c), p3, twid<R>(c.ax[0]),
                                        mk<R>(0, R(-c.omega * kEps0)), mk<R>(0, R(c.omega * kMu0)), s);
        VIE_REQUIRE(ok, VIE_EINVAL, "J-M x pass: no compiled kernel for this length");
    } else if (op == OP_CURL || op == OP_K) {
        // curl operator: staged x pass (any length up to 256) on its 30
        // unique tensors
        const int nt = p3_threads<R>();
        const size_t ul = 30 * (size_t)c.O[0] * es;
        int g = 4;
        while (g > 1 && (ul + (size_t)lds_pad(g * 12 * Mx) * es > 80 * 1024 || !rows_fit(p3.plan, g * 12, nt) ||
                         2 * g * Mx > nt))
            --g;
        p3.groups = g;
        p3.variant = 0;
        p3.sib_blocks = 1;
        KernelTiming kt(c.prof, VIE_K_BLOCK, 2 * bA2 + 30.0 * c.Osz * es);
        launch_p3_curl<R>(A2, curlspec<R>(c), p3, twid<R>(c.ax[0]), s);
    } else if (nc == 3) {
        // PWC: 6 of the operator's unique tensors per frequency
        VIE_REQUIRE(p3_ct_supported(Mx), VIE_EINVAL,
                    "the PWC x pass needs an fft length along x of 8, 16, 32, 64, 96, 128, 160, 192, 256, 320, 384 "
                    "or 512");
        KernelTiming kt(c.prof, VIE_K_BLOCK, 2 * bA2 + 6.0 * c.Osz * es);
        launch_p3_pwc<R>(A2, opspec<R>(c), p3, twid<R>(c.ax[0]), s);
    } else {
        // as many pencil groups per LDS pass as fit 64 KiB and the
        // butterfly bound of the in-place passes (at most 4 siblings share
        // an octant row)
        // LDS holds the operator row (60 Ox) plus the pencil groups
        const int nt = p3_threads<R>();
        const size_t ul = 60 * (size_t)c.O[0] * es;
        int g = 4;
        while (g > 1 && (ul + (size_t)lds_pad(g * 12 * Mx) * es > 80 * 1024 || !rows_fit(p3.plan, g * 12, nt) ||
                         2 * g * Mx > nt))
            --g;
        p3.sib_blocks = 1;
        p3.variant = 0;
        if (p3_ct_supported(Mx)) {
            // light variant (one pencil group per workgroup) unless the
            // autotuner chose the staged one; the staged variant shares the
            // operator row among all siblings and right-hand sides of a
            // workgroup
            p3.variant = tn.p3_variant >= 0 ? tn.p3_variant : 1;
            if (p3.variant == 0 && !p3_ct_fits((int)es, Mx)) p3.variant = 1;   // staged row would not fit LDS
            p3.sib_blocks = tn.p3_sib_blocks ? tn.p3_sib_blocks : 1;
            g = std::min(p3_ct_groups((int)es, Mx), (4 / p3.sib_blocks) * nrhs);
            g = std::max(g, 1);
        } else {
            VIE_REQUIRE(rows_fit(p3.plan, 12, nt) && 2 * Mx <= nt && ul + (size_t)lds_pad(12 * Mx) * es <= 150 * 1024,
                        VIE_EINVAL, "fft size along x too large");
        }
        p3.groups = g;
        p3.magic_nx = magic_for((unsigned)Nx);
        p3.magic_ox = magic_for((unsigned)c.O[0]);
        KernelTiming kt(c.prof, VIE_K_BLOCK, 2 * bA2 + 60.0 * c.Osz * es);
        launch_p3<R>(A2, opspec<R>(c), p3, twid<R>(c.ax[0]), s);
    }

    // P4: inverse y, crop
    StridedPass p4 = p2;
    p4.n_in = My;
    p4.n_out = Ny;
    p4.in_s1 = sR2;
    p4.in_sc = Nx;
    p4.in_s2 = pl2;
    p4.in_sk = row;
    p4.out_s1 = sR1;
    p4.out_sc = Nx;
    p4.out_s2 = pl1;
    p4.out_sk = row;
    {
        KernelTiming kt(c.prof, VIE_K_FFT_Y_INV, bA2 + bA1);
        launch_strided<R>(false, A2, A1, p4, Mz, B, twid<R>(c.ax[1]), nullptr, s);
    }

    // P5: inverse z, crop, epilogue
    StridedPass p5 = p1;
    p5.n_in = Mz;
    p5.n_out = Nz;
    p5.in_s1 = sR1;
    p5.in_sc = Nx;
    p5.in_s2 = row;
    p5.in_sk = pl1;
    p5.out_s1 = nc * V;
    p5.out_sc = V;
    p5.out_s2 = Nx;
    p5.out_sk = (long long)Ny * Nx;
    Epilogue<R> ep{};
    const R scale = R(1.0 / ((double)Mx * My * Mz));
    const double dv = c.D[0] * c.D[1] * c.D[2];
    const double G[4] = {dv, dv / 12, dv / 12, dv / 12};
    const C<R>* tau = nullptr;
    const C<R>* epsr = nullptr;
    const C<R>* chi = nullptr;
    if constexpr (sizeof(R) == 4) {
        tau = c.mat.tau64;
        epsr = c.mat.epsr64;
        chi = c.mat.chi64;
    } else {
        tau = c.mat.tau;
        epsr = c.mat.eps_r;
        chi = c.mat.chi;
    }
    ep.x = x;
    for (int l = 0; l < 4; ++l) {
        switch (op) {
            case OP_PREC:
                ep.a_const = 1;
                ep.ga[l] = 1;
                ep.b = tau;
                ep.gb[l] = R(-scale / G[l]);
                break;
            case OP_A:
                ep.a = epsr;
                ep.ga[l] = R(G[l]);
                ep.b = chi;
                ep.gb[l] = -scale;
                break;
            case OP_N:
            case OP_K:
            case OP_JMS:
                ep.a_const = 0;
                ep.ga[l] = 0;
                ep.b_const = 1;
                ep.gb[l] = scale;
                break;
            case OP_RESID:
                ep.a_const = -1;
                ep.ga[l] = 1;
                ep.b = tau;
                ep.gb[l] = R(scale / G[l]);
                ep.rhs = rhs;
                break;
            case OP_CURL:   // h = (h_t + K x) / G, h_t in the epilogue's x slot
                ep.x = rhs;
                ep.a_const = 1;
                ep.ga[l] = R(1.0 / G[l]);
                ep.b_const = 1;
                ep.gb[l] = R(scale / G[l]);
                break;
        }
    }
    {
        // inverse z pass: intermediate in, result out, plus the epilogue's x,
        // right-hand side and per-voxel coefficient reads
        double extra = 0;
        if (ep.a_const != R(0) || ep.a) extra += bV;
        if (ep.rhs) extra += bV;
        if (ep.a) extra += (double)V * es;
        if (ep.b) extra += (double)V * es;
        KernelTiming kt(c.prof, VIE_K_FFT_Z_INV, bA1 + bV + extra);
        launch_strided<R>(false, A1, y, p5, Ny, B, twid<R>(c.ax[2]), &ep, s);
    }
}

template void apply_op<float>(Ctx&, int, int, const C<float>*, C<float>*, const C<float>*, void*, size_t);
template void apply_op<double>(Ctx&, int, int, const C<double>*, C<double>*, const C<double>*, void*, size_t);

}  // namespace vie
