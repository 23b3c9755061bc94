// Restarted GMRES for the left-preconditioned system P^-1 A x = P^-1 b
// (Sec. IV-B with P = M_eps G; Sec. V: GMRES, restart 50).
//
// Every restart cycle starts from the true residual r = P^-1 b - P^-1 A x
// computed with the complex128 operator product and FP64 norms; x is kept in
// complex128.  The Arnoldi process of the cycle runs either in complex128
// (mode FP64) or in complex64 (mode FP32_IR): then each cycle is one step of
// iterative refinement, the complex64 Krylov solve of P^-1 A d = r / ||r||
// followed by x += ||r|| d in FP64.  Orthogonalisation is classical
// Gram-Schmidt (optionally twice) with FP64 inner products; the Hessenberg
// matrix, Givens rotations and the small triangular solve are FP64 on the
// host.  Basis vectors after the first are stored unnormalised, each with its
// reciprocal norm beside it: the normalisation is folded into the
// Gram-Schmidt coefficients and the solution update instead of taking a pass
// over the vector of its own.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "ctx.hpp"

namespace vie {

using cd = std::complex<double>;

// workgroups of the update and norm kernels: up to 1024, at least 1024
// elements each, so that vectors of a few MB (PWC basis, small grids) still
// spread over all CUs
static int blocks_for(long long n) {
    long long b = (n + 1024 - 1) / 1024;
    return (int)std::max(1LL, std::min(1024LL, b));
}

// workgroups per group of basis vectors of the dot kernel (whose groups run
// side by side): up to 1024, at least 2048 elements each
static int dot_blocks_for(long long n) {
    long long b = (n + 2048 - 1) / 2048;
    return (int)std::max(1LL, std::min(1024LL, b));
}

// FP64 norms of nrhs vectors of length n (device result in out_dev, host copy in out)
template <typename R>
static void norms(Ctx& c, const C<R>* v, long long n, int nrhs, double* partial, double* out_dev,
                  std::vector<double>& out) {
    const int nb = blocks_for(n);
    launch_norm_partials<R>(partial, v, n, n, nrhs, nb, c.stream);
    launch_reduce_norm(out_dev, partial, nb, nrhs, c.stream);
    out.resize(nrhs);
    VIE_HIP(hipMemcpyAsync(out.data(), out_dev, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    VIE_HIP(hipStreamSynchronize(c.stream));
}

struct Layout {
    double2 *rhs, *r, *partial, *h1, *h2, *coef, *y;
    double *nrm, *npart, *inv, *bn, *rn, *ivn;
};

template <typename R>
static int run(Ctx& c, const vie_solve_opts& o, int nrhs, double2* x, const Layout& L, vie_solve_stats* st,
               std::vector<double>& bnorm) {
    const long long n = (long long)c.nc * c.V;
    const int m = o.restart;
    const bool ir = (sizeof(R) == 4);
    const int nb = blocks_for(n), nbd = dot_blocks_for(n);
    // consecutive basis vectors are staggered by a little over 4 KiB, so that
    // the j + 1 streams the Gram-Schmidt kernels read side by side do not
    // start at equal offsets modulo large powers of two
    const long long vpad = 4352 / (long long)sizeof(C<R>);
    C<R>* Vb = static_cast<C<R>*>(c.basis.get((size_t)(m + 1) * (nrhs * n + vpad) * sizeof(C<R>)));
    std::vector<int> conv(nrhs, 0);
    std::vector<double> rnorm;
    std::vector<double> last_rel(nrhs, 1.0);
    int status = VIE_ENOCONV;
    const int rchunk = std::max(1, std::min(nrhs, 4));
    // each cycle of the refinement mode is one refinement step
    const int max_cycles = ir ? std::min(o.max_outer, o.max_refine) : o.max_outer;
    for (int cycle = 0; cycle <= max_cycles; ++cycle) {
        // true residual, complex128
        for (int r0 = 0; r0 < nrhs; r0 += rchunk) {
            const int k = std::min(rchunk, nrhs - r0);
            apply_op<double>(c, OP_RESID, k, x + r0 * n, L.r + r0 * n, L.rhs + r0 * n);
            for (int r = r0; r < r0 + k; ++r)
                if (st && !conv[r]) st[r].matvecs_c128 += 1;
        }
        norms<double>(c, L.r, n, nrhs, L.npart, L.rn, rnorm);
        std::vector<int> active;
        for (int r = 0; r < nrhs; ++r) {
            if (!std::isfinite(rnorm[r])) return VIE_ENAN;
            const double rel = bnorm[r] > 0 ? rnorm[r] / bnorm[r] : 0.0;
            if (!conv[r]) last_rel[r] = rel;
            if (rel <= o.tol) conv[r] = 1;
            if (!conv[r]) active.push_back(r);
        }
        if (active.empty()) {
            status = VIE_OK;
            break;
        }
        if (cycle == max_cycles) break;
        const int na = (int)active.size();
        const long long ldv = (long long)na * n + vpad;
        // V_0 = r / ||r|| for the active right-hand sides (compacted)
        std::vector<double> inv(na);
        for (int s = 0; s < na; ++s) inv[s] = 1.0 / rnorm[active[s]];
        VIE_HIP(hipMemcpyAsync(L.inv, inv.data(), na * sizeof(double), hipMemcpyHostToDevice, c.stream));
        for (int s = 0; s < na; ++s) {
            if constexpr (sizeof(R) == 4)
                launch_cast_down(reinterpret_cast<float2*>(Vb) + s * n, L.r + active[s] * n, L.inv + s, n, 1,
                                 c.stream);
            else
                launch_scale_into<double>(reinterpret_cast<double2*>(Vb) + s * n, L.r + active[s] * n,
                                          L.rn + active[s], n, n, n, 1, c.stream);
        }
        // reciprocal norms of the stored basis vectors: 1 for V_0, the rest
        // written by the device after each step (and kept on the host for
        // the solution update)
        std::vector<double> ivn0((size_t)na * (m + 1), 0.0);
        for (int s = 0; s < na; ++s) ivn0[(size_t)s * (m + 1)] = 1.0;
        VIE_HIP(hipMemcpyAsync(L.ivn, ivn0.data(), ivn0.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
        std::vector<std::vector<double>> ivh(na, std::vector<double>(m + 1, 0.0));
        for (int s = 0; s < na; ++s) ivh[s][0] = 1.0;
        // per-slot Hessenberg / Givens state
        std::vector<std::vector<cd>> H(na, std::vector<cd>((size_t)(m + 1) * m));
        std::vector<std::vector<cd>> cs(na, std::vector<cd>(m)), sn(na, std::vector<cd>(m)),
            g(na, std::vector<cd>(m + 1));
        std::vector<double> target(na);
        std::vector<int> done(na, 0);
        for (int s = 0; s < na; ++s) {
            g[s][0] = rnorm[active[s]];
            const double need = o.tol * bnorm[active[s]] / rnorm[active[s]];
            target[s] = ir ? std::max(o.inner_tol, need) : need;
        }
        // The Arnoldi steps do not depend on the Givens rotations, so the
        // host lags the device by one step: it enqueues step j, then waits
        // for the Hessenberg column of step j - 1 (copied into page-locked
        // memory behind it on the stream) and updates the rotations and the
        // residual estimate.  A convergence found at step j - 1 leaves step j
        // computed but unused.
        int jdone = 0;
        const size_t colsz = (size_t)na * (m + 1);
        double* pin = static_cast<double*>(c.hpin.get(2 * (2 * colsz * sizeof(double2) + na * sizeof(double))));
        auto slot_h1 = [&](int sl) { return reinterpret_cast<double2*>(pin) + (size_t)sl * 2 * colsz; };
        auto slot_h2 = [&](int sl) { return slot_h1(sl) + colsz; };
        auto slot_nrm = [&](int sl) { return pin + (size_t)2 * 2 * colsz * 2 + (size_t)sl * na; };
        for (auto& e : c.col_ev)
            if (!e) VIE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        // Givens update for column j; true when every slot has converged
        auto process = [&](int j) -> int {
            const int sl = j & 1;
            VIE_HIP(hipEventSynchronize(c.col_ev[sl]));
            const int nvec = j + 1;
            const double2* h1 = slot_h1(sl);
            const double2* h2 = slot_h2(sl);
            const double* nrm = slot_nrm(sl);
            bool all = true;
            for (int s = 0; s < na; ++s) {
                cd* Hc = &H[s][(size_t)j * (m + 1)];   // column j, rows 0..j+1
                for (int i = 0; i <= j; ++i) {
                    Hc[i] = cd(h1[(size_t)s * nvec + i].x, h1[(size_t)s * nvec + i].y);
                    if (o.reorth) Hc[i] += cd(h2[(size_t)s * nvec + i].x, h2[(size_t)s * nvec + i].y);
                }
                Hc[j + 1] = nrm[s];
                ivh[s][j + 1] = nrm[s] > 0 ? 1.0 / nrm[s] : 0.0;
                for (int i = 0; i < j; ++i) {   // previous rotations
                    const cd t = cs[s][i] * Hc[i] + sn[s][i] * Hc[i + 1];
                    Hc[i + 1] = -std::conj(sn[s][i]) * Hc[i] + std::conj(cs[s][i]) * Hc[i + 1];
                    Hc[i] = t;
                }
                const double den = std::sqrt(std::norm(Hc[j]) + std::norm(Hc[j + 1]));
                if (den == 0.0) {
                    cs[s][j] = 1.0;
                    sn[s][j] = 0.0;
                } else {
                    cs[s][j] = std::conj(Hc[j]) / den;
                    sn[s][j] = std::conj(Hc[j + 1]) / den;
                }
                Hc[j] = den;
                Hc[j + 1] = 0.0;
                g[s][j + 1] = -std::conj(sn[s][j]) * g[s][j];
                g[s][j] = cs[s][j] * g[s][j];
                const double est = std::abs(g[s][j + 1]) / rnorm[active[s]];
                if (st) {
                    st[active[s]].iterations += 1;
                    if (ir) st[active[s]].matvecs_c64 += 1;
                    else st[active[s]].matvecs_c128 += 1;
                }
                if (!std::isfinite(est)) return -1;
                if (!(est <= target[s]) && nrm[s] > 0.0) all = false;
            }
            return all ? 1 : 0;
        };
        int launched = 0, stop = 0;
        for (int j = 0; j < m && !stop; ++j) {
            C<R>* vj = Vb + (long long)j * ldv;
            C<R>* w = Vb + (long long)(j + 1) * ldv;
            apply_op<R>(c, OP_PREC, na, vj, w, nullptr);
            const int nvec = j + 1;
            // Gram-Schmidt, per pass: the dot kernel reads the j + 1 basis
            // vectors and w (w once per group of 8 basis vectors); the
            // update reads them again, reads and writes w, and leaves w
            // unnormalised with its reciprocal norm in ivn[j + 1]
            const double vb = (double)na * n * sizeof(C<R>);
            const double dot_bytes = vb * (nvec + (nvec + 7) / 8);
            const double upd_bytes = vb * (nvec + 2);
            const long long ivld = m + 1;
            for (int pass = 0; pass < (o.reorth ? 2 : 1); ++pass) {
                double2* hp = pass ? L.h2 : L.h1;
                const int jw = pass ? -1 : j;
                {
                    ProfScope ps(c.prof, c.stream, VIE_K_GS_DOT, dot_bytes);
                    launch_multidot<R>(L.partial, Vb, ldv, nvec, w, n, n, n, na, nbd, c.stream);
                    launch_reduce_partials(hp, L.coef, L.partial, nvec, nbd, na, L.ivn, ivld, jw, c.stream);
                }
                {
                    ProfScope ps(c.prof, c.stream, VIE_K_GS_UPDATE, upd_bytes);
                    launch_update<R>(w, Vb, ldv, nvec, L.coef, n, n, n, L.npart, L.ivn, ivld, jw, na, nb, c.stream);
                    if (pass == (o.reorth ? 1 : 0))
                        launch_reduce_norm(L.nrm, L.npart, nb, na, c.stream, L.ivn + (j + 1), ivld);
                }
            }
            // the column's slot was last read by the host for step j - 2,
            // which process() finished before this step was enqueued
            const int sl = j & 1;
            VIE_HIP(hipMemcpyAsync(slot_h1(sl), L.h1, (size_t)na * nvec * sizeof(double2), hipMemcpyDeviceToHost,
                                   c.stream));
            if (o.reorth)
                VIE_HIP(hipMemcpyAsync(slot_h2(sl), L.h2, (size_t)na * nvec * sizeof(double2),
                                       hipMemcpyDeviceToHost, c.stream));
            VIE_HIP(hipMemcpyAsync(slot_nrm(sl), L.nrm, na * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            VIE_HIP(hipEventRecord(c.col_ev[sl], c.stream));
            launched = j + 1;
            if (j >= 1) {
                const int rc = process(j - 1);
                if (rc < 0) return VIE_ENAN;
                jdone = j;
                if (rc > 0) stop = 1;
            }
        }
        if (!stop && launched > jdone) {
            const int rc = process(launched - 1);
            if (rc < 0) return VIE_ENAN;
            jdone = launched;
        }
        // x += V y with y from the triangular system (FP64)
        std::vector<double2> yh((size_t)na * jdone);
        for (int s = 0; s < na; ++s) {
            std::vector<cd> yv(jdone);
            for (int i = jdone - 1; i >= 0; --i) {
                cd acc = g[s][i];
                for (int k = i + 1; k < jdone; ++k) acc -= H[s][(size_t)k * (m + 1) + i] * yv[k];
                const cd d = H[s][(size_t)i * (m + 1) + i];
                yv[i] = (d == 0.0) ? cd(0) : acc / d;
            }
            // V y = sum_i (y_i ivn_i) u_i over the stored vectors
            for (int i = 0; i < jdone; ++i)
                yh[(size_t)s * jdone + i] = make_double2(yv[i].real() * ivh[s][i], yv[i].imag() * ivh[s][i]);
        }
        VIE_HIP(hipMemcpyAsync(L.y, yh.data(), yh.size() * sizeof(double2), hipMemcpyHostToDevice, c.stream));
        for (int s = 0; s < na; ++s) {
            launch_combine<R>(x + (long long)active[s] * n, Vb + (long long)s * n, ldv, jdone,
                              L.y + (size_t)s * jdone, n, n, 1, c.stream);
            if (st) {
                st[active[s]].restarts += 1;
                if (ir) st[active[s]].refinements += 1;
            }
        }
        VIE_HIP(hipStreamSynchronize(c.stream));
    }
    for (int r = 0; r < nrhs; ++r)
        if (st) {
            st[r].converged = conv[r];
            st[r].rel_residual = last_rel[r];
        }
    return status;
}

int solve(Ctx& c, const vie_solve_opts& o, int nrhs, const double2* et, double2* x, vie_solve_stats* st) {
    auto t0 = std::chrono::steady_clock::now();
    const long long n = (long long)c.nc * c.V;
    const int m = o.restart;
    const int nb = blocks_for(n);
    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o_ = off;
        off += (bytes + 255) / 256 * 256;
        return o_;
    };
    const size_t o_rhs = take((size_t)nrhs * n * 16), o_r = take((size_t)nrhs * n * 16);
    const size_t o_part = take((size_t)nrhs * (m + 1) * std::max(nb, dot_blocks_for(n)) * 16);
    const size_t o_h1 = take((size_t)nrhs * (m + 1) * 16), o_h2 = take((size_t)nrhs * (m + 1) * 16);
    const size_t o_coef = take((size_t)nrhs * (m + 1) * 16), o_ivn = take((size_t)nrhs * (m + 1) * 8);
    const size_t o_y = take((size_t)nrhs * m * 16);
    const size_t o_nrm = take(nrhs * 8), o_np = take((size_t)nrhs * nb * 8), o_inv = take(nrhs * 8);
    const size_t o_bn = take(nrhs * 8), o_rn = take(nrhs * 8);
    char* base = static_cast<char*>(c.vecs.get(off));
    Layout L{};
    L.rhs = reinterpret_cast<double2*>(base + o_rhs);
    L.r = reinterpret_cast<double2*>(base + o_r);
    L.partial = reinterpret_cast<double2*>(base + o_part);
    L.h1 = reinterpret_cast<double2*>(base + o_h1);
    L.h2 = reinterpret_cast<double2*>(base + o_h2);
    L.coef = reinterpret_cast<double2*>(base + o_coef);
    L.ivn = reinterpret_cast<double*>(base + o_ivn);
    L.y = reinterpret_cast<double2*>(base + o_y);
    L.nrm = reinterpret_cast<double*>(base + o_nrm);
    L.npart = reinterpret_cast<double*>(base + o_np);
    L.inv = reinterpret_cast<double*>(base + o_inv);
    L.bn = reinterpret_cast<double*>(base + o_bn);
    L.rn = reinterpret_cast<double*>(base + o_rn);
    if (st)
        for (int r = 0; r < nrhs; ++r) st[r] = vie_solve_stats{};

    const double dv = c.D[0] * c.D[1] * c.D[2];
    const double ginv[4] = {1 / dv, 12 / dv, 12 / dv, 12 / dv};
    launch_rhs_prec(L.rhs, et, c.mat.tau, ginv, make_double2(0.0, c.omega * kEps0), c.V, nrhs, c.nc, c.stream);
    std::vector<double> bnorm;
    norms<double>(c, L.rhs, n, nrhs, L.npart, L.bn, bnorm);
    for (int r = 0; r < nrhs; ++r)
        if (!std::isfinite(bnorm[r])) return VIE_ENAN;
    if (!o.use_x0) VIE_HIP(hipMemsetAsync(x, 0, (size_t)nrhs * n * sizeof(double2), c.stream));
    int rc = (o.mode == VIE_SOLVE_FP32_IR) ? run<float>(c, o, nrhs, x, L, st, bnorm)
                                           : run<double>(c, o, nrhs, x, L, st, bnorm);
    VIE_HIP(hipStreamSynchronize(c.stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st)
        for (int r = 0; r < nrhs; ++r) st[r].seconds = secs;
    return rc;
}

}  // namespace vie
