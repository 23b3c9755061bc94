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
// columns, Givens rotations, residual estimate and the small triangular
// solve are FP64 on the device, so the host only reads a convergence flag
// every few steps, and a run of steps can be replayed from a HIP graph.
// Basis vectors after the first are stored unnormalised, each with its
// reciprocal norm beside it: the normalisation is folded into the
// Gram-Schmidt coefficients and the solution update instead of taking a pass
// over the vector of its own.
#include <chrono>
#include <cmath>
#include <cstdint>
#include <vector>

#include "ctx.hpp"

namespace vie {

// Workgroup counts of the Gram-Schmidt kernels: per_wg elements per
// workgroup, up to 1024 workgroups, and for short vectors at least
// min(n / 512, 256) of them (one 16-byte unit per thread in complex64), so
// that a vector of a few hundred kB still spreads over the CUs: there the
// kernels are bound by load latency, not bandwidth.
static int gs_blocks(long long n, long long per_wg) {
    const long long floor_ = std::min((n + 511) / 512, 256LL);
    const long long b = std::max((n + per_wg - 1) / per_wg, floor_);
    return (int)std::max(1LL, std::min(1024LL, b));
}
// update and norm kernels: 1024 elements per workgroup
static int blocks_for(long long n) { return gs_blocks(n, 1024); }
// dot kernel, per group of 8 basis vectors (the groups run side by side):
// 2048 elements per workgroup
static int dot_blocks_for(long long n) { return gs_blocks(n, 2048); }

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
    double2 *H, *cs, *sn, *g, *slot;   // least-squares state (ArnoldiState)
    int* stat;
    // two-step Arnoldi: unrotated Hessenberg columns, second coefficients,
    // conj(w1) w2 partials, norm partials of u_{j+2}, pair coefficients and
    // the assembled column j + 1
    double2 *Hr, *coef2, *dpart, *pc, *col;
    double* npart2;
    // three-step Arnoldi: g_1..3 and their coefficients (3 [na][m + 1]
    // blocks each), Gram partials, Cholesky coefficients, the two assembled
    // columns, norm partials of u_{j+3}
    double2 *g3, *coef3, *tc, *col2;
    double *gpart, *npart3;
};

// Arnoldi steps between host checks of the convergence flag: several while
// a step is short enough for the host round trip to show, one once a step
// streams tens of MB
// graph replay by default up to this many bytes per batch of vectors: there
// the launches of a step are a visible part of it (16^3 sphere: +2.7%
// solves/s replayed), above it replay measured slower (64^3: -1.9%)
constexpr long long kGraphAutoBytes = 2LL << 20;

static int auto_sync_steps(long long vec_bytes) {
    if (vec_bytes <= (2LL << 20)) return 4;
    if (vec_bytes <= (16LL << 20)) return 2;
    return 1;
}

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
        // least-squares state on the device: g_0 = ||r||, the target of each
        // slot's residual estimate, reciprocal norm 1 for V_0
        std::vector<double2> slot(na);
        for (int s = 0; s < na; ++s) {
            const double need = o.tol * bnorm[active[s]] / rnorm[active[s]];
            slot[s] = make_double2(rnorm[active[s]], ir ? std::max(o.inner_tol, need) : need);
        }
        VIE_HIP(hipMemcpyAsync(L.slot, slot.data(), na * sizeof(double2), hipMemcpyHostToDevice, c.stream));
        const ArnoldiState as{L.H, L.cs, L.sn, L.g, L.slot, L.stat, m, L.Hr};
        const long long ivld = m + 1;
        launch_arnoldi_init(as, L.ivn, ivld, na, c.stream);

        // Arnoldi step j: w = P^-1 A u_j, Gram-Schmidt against u_0..u_j
        // (w left unnormalised, its reciprocal norm in ivn[j + 1]), and the
        // Givens update of column j on the device
        auto step = [&](int j) {
            C<R>* vj = Vb + (long long)j * ldv;
            C<R>* w = Vb + (long long)(j + 1) * ldv;
            apply_op<R>(c, OP_PREC, na, vj, w, nullptr);
            const int nvec = j + 1;
            // per pass the dot kernel reads the j + 1 basis vectors and w (w
            // once per group of 8 basis vectors); the update reads them
            // again and reads and writes w
            const double vb = (double)na * n * sizeof(C<R>);
            const double dot_bytes = vb * (nvec + (nvec + 7) / 8);
            const double upd_bytes = vb * (nvec + 2);
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
                }
            }
            // ||w|| from the last pass's partials, then column j into the rotations
            launch_givens(as, L.h1, o.reorth ? L.h2 : nullptr, L.npart, nb, L.nrm, L.ivn + (j + 1), ivld, j, na,
                          c.stream);
        };

        // Arnoldi steps j and j + 1 with one pass over the basis (s-step
        // Arnoldi, s = 2; the algebra is stated with the kernels):
        // w1 = P^-1 A u_j into slot j + 1, w2 = P^-1 A w1 into slot j + 2,
        // both orthogonalised against u_0..u_j by one dot and one update
        // pass, then u_{j+2} against u_{j+1} alone
        auto pair = [&](int j) {
            C<R>* vj = Vb + (long long)j * ldv;
            C<R>* w1 = Vb + (long long)(j + 1) * ldv;
            C<R>* w2 = Vb + (long long)(j + 2) * ldv;
            apply_op<R>(c, OP_PREC, na, vj, w1, nullptr);
            apply_op<R>(c, OP_PREC, na, w1, w2, nullptr);
            const int nvec = j + 1;
            const double vb = (double)na * n * sizeof(C<R>);
            {
                ProfScope ps(c.prof, c.stream, VIE_K_GS_DOT, vb * (nvec + 2.0 * ((nvec + 7) / 8)));
                launch_multidot2<R>(L.partial, Vb, ldv, nvec, w1, ldv, n, n, n, na, nbd, c.stream);
                launch_reduce_pair(L.h1, L.coef, L.h2, L.coef2, L.partial, nvec, nbd, na, L.ivn, ivld, j, c.stream);
            }
            {   // reads the basis, reads and writes w1 and w2
                ProfScope ps(c.prof, c.stream, VIE_K_GS_UPDATE, vb * (nvec + 4));
                launch_update_pair<R>(w1, Vb, ldv, nvec, L.coef, L.coef2, L.h1, n, n, n, L.npart, L.dpart, L.ivn,
                                      ivld, j, na, nb, c.stream);
            }
            launch_givens(as, L.h1, nullptr, L.npart, nb, L.nrm, L.ivn + (j + 1), ivld, j, na, c.stream);
            launch_pair_coef(L.pc, L.dpart, nb, L.nrm, na, c.stream);
            {   // reads u_{j+1}, reads and writes u_{j+2}
                ProfScope ps(c.prof, c.stream, VIE_K_GS_PAIR, vb * 3);
                launch_axpy_pair<R>(w1, ldv, n, n, L.pc, L.npart2, na, nb, c.stream);
            }
            launch_pair_column(as, L.h1, L.h2, L.pc, L.col, j, na, c.stream);
            launch_givens(as, L.col, nullptr, L.npart2, nb, L.nrm, L.ivn + (j + 2), ivld, j + 1, na, c.stream);
        };
        // Arnoldi three steps per pass over the basis:
        // w1 = P^-1 A u_j, w2 = P^-1 A w1, w3 = P^-1 A w2 in slots j + 1 ..
        // j + 3, one dot and one update pass for the three, then u_{j+2} and
        // u_{j+3} against the block (the algebra is stated with the kernels)
        const long long gst = (long long)na * (m + 1);
        auto triple = [&](int j) {
            C<R>* vj = Vb + (long long)j * ldv;
            C<R>* w1 = Vb + (long long)(j + 1) * ldv;
            apply_op<R>(c, OP_PREC, na, vj, w1, nullptr);
            apply_op<R>(c, OP_PREC, na, w1, w1 + ldv, nullptr);
            apply_op<R>(c, OP_PREC, na, w1 + ldv, w1 + 2 * ldv, nullptr);
            const int nvec = j + 1;
            const double vb = (double)na * n * sizeof(C<R>);
            {
                ProfScope ps(c.prof, c.stream, VIE_K_GS_DOT, vb * (nvec + 3.0 * ((nvec + 7) / 8)));
                launch_multidot3<R>(L.partial, Vb, ldv, nvec, w1, ldv, n, n, n, na, nbd, c.stream);
                launch_reduce_triple(L.g3, L.coef3, L.partial, nvec, nbd, na, L.ivn, ivld, j, gst, c.stream);
            }
            {   // reads the basis, reads and writes w1..w3
                ProfScope ps(c.prof, c.stream, VIE_K_GS_UPDATE, vb * (nvec + 6));
                launch_update_triple<R>(w1, Vb, ldv, nvec, L.coef3, gst, L.g3, n, n, n, L.npart, L.gpart, L.ivn, ivld,
                                        j, na, nb, c.stream);
            }
            launch_givens(as, L.g3, nullptr, L.npart, nb, L.nrm, L.ivn + (j + 1), ivld, j, na, c.stream);
            launch_triple_coef(L.tc, L.gpart, nb, na, c.stream);
            {   // reads y1..y3, writes u_{j+2}, u_{j+3}
                ProfScope ps(c.prof, c.stream, VIE_K_GS_PAIR, vb * 5);
                launch_axpy_triple<R>(w1, ldv, n, n, L.tc, L.npart2, L.npart3, na, nb, c.stream);
            }
            launch_triple_columns(as, L.g3, gst, L.tc, L.col, L.col2, j, na, c.stream);
            launch_givens(as, L.col, nullptr, L.npart2, nb, L.nrm, L.ivn + (j + 2), ivld, j + 1, na, c.stream);
            launch_givens(as, L.col2, nullptr, L.npart3, nb, L.nrm, L.ivn + (j + 3), ivld, j + 2, na, c.stream);
        };
        // s = 3 by default (pairs and single steps fill the end of a
        // cycle), 2 or 1 on request; the second Gram-Schmidt pass runs with
        // single steps
        const long long vec_bytes = na * n * (long long)sizeof(C<R>);
        const bool two = o.s_step != 1 && !o.reorth && m >= 2;
        const bool three = (o.s_step == 0 || o.s_step == 3) && !o.reorth && m >= 3;

        // steps [j0, j1): launched one by one, or replayed from a graph
        // (the product's workspace is grown first, so that no step
        // reallocates it under a capture)
        const bool use_graph = (o.graph > 0 || (o.graph < 0 && vec_bytes <= kGraphAutoBytes)) && !c.prof.on;
        if (use_graph) c.ws.get(apply_workspace_bytes(c, na, sizeof(C<R>)));
        auto enqueue = [&](int j0, int j1) {
            auto run_steps = [&] {
                for (int j = j0; j < j1;) {
                    if (three && j + 2 < j1) {
                        triple(j);
                        j += 3;
                    } else if (two && j + 1 < j1) {
                        pair(j);
                        j += 2;
                    } else {
                        step(j);
                        j += 1;
                    }
                }
            };
            if (!use_graph) {
                run_steps();
                return;
            }
            const std::vector<long long> key{(long long)sizeof(R), na, m, o.reorth, two, three, j0, j1, n,
                                             (long long)reinterpret_cast<uintptr_t>(Vb), ldv,
                                             (long long)reinterpret_cast<uintptr_t>(L.rhs),
                                             (long long)reinterpret_cast<uintptr_t>(c.ws.p),
                                             (long long)reinterpret_cast<uintptr_t>(c.jmbuf.p), c.nc};
            auto it = c.graphs.execs.find(key);
            if (it == c.graphs.execs.end()) {
                run_steps();
                if (c.graphs.execs.size() >= GraphCache::kMax) c.graphs.clear();
                c.graphs.execs.emplace(key, nullptr);
                return;
            }
            if (!it->second) {
                if (!c.graphs.cap) VIE_HIP(hipStreamCreateWithFlags(&c.graphs.cap, hipStreamNonBlocking));
                const hipStream_t own = c.stream;
                hipGraph_t gr = nullptr;
                c.stream = c.graphs.cap;
                VIE_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
                try {
                    run_steps();
                } catch (...) {
                    (void)hipStreamEndCapture(c.stream, &gr);
                    if (gr) (void)hipGraphDestroy(gr);
                    c.stream = own;
                    throw;
                }
                const hipError_t e = hipStreamEndCapture(c.stream, &gr);
                c.stream = own;
                VIE_HIP(e);
                hipGraphExec_t ex = nullptr;
                const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                VIE_HIP(ei);
                it->second = ex;
            }
            VIE_HIP(hipGraphLaunch(it->second, c.stream));
        };

        // The host checks the device's convergence flag once per chunk of S
        // steps and keeps one chunk queued ahead of the one it waits for, so
        // the device does not idle on the round trip; a chunk queued behind
        // the converged one runs with its Givens updates turned off.
        int S = o.sync_steps > 0 ? o.sync_steps : auto_sync_steps(vec_bytes);
        if (three) S = (S + 2) / 3 * 3;   // chunks of whole triples
        else if (two) S += S & 1;        // chunks of whole pairs
        const int nch = (m + S - 1) / S;
        int* pin = static_cast<int*>(c.hpin.get(2 * 4 * sizeof(int)));
        for (auto& e : c.col_ev)
            if (!e) VIE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        auto launch_chunk = [&](int k) {
            enqueue(k * S, std::min(m, (k + 1) * S));
            VIE_HIP(hipMemcpyAsync(pin + 4 * (k & 1), L.stat, 4 * sizeof(int), hipMemcpyDeviceToHost, c.stream));
            VIE_HIP(hipEventRecord(c.col_ev[k & 1], c.stream));
        };
        int launched = 0, checked = 0, jdone = 0;
        bool stop = false;
        launch_chunk(launched++);
        while (checked < launched && !stop) {
            if (launched < nch) launch_chunk(launched++);
            VIE_HIP(hipEventSynchronize(c.col_ev[checked & 1]));
            const int* sv = pin + 4 * (checked & 1);
            ++checked;
            jdone = sv[0];
            if (sv[2]) return VIE_ENAN;
            if (sv[1]) stop = true;
        }

        // x += V y with y = R^-1 g (FP64, on the device)
        launch_backsolve(as, L.ivn, ivld, L.y, jdone, na, c.stream);
        for (int s = 0; s < na; ++s) {
            launch_combine<R>(x + (long long)active[s] * n, Vb + (long long)s * n, ldv, jdone,
                              L.y + (size_t)s * jdone, n, n, 1, c.stream);
            if (st) {
                st[active[s]].iterations += jdone;
                if (ir) st[active[s]].matvecs_c64 += jdone;
                else st[active[s]].matvecs_c128 += jdone;
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
    const size_t o_part = take((size_t)3 * nrhs * (m + 1) * std::max(nb, dot_blocks_for(n)) * 16);
    const size_t o_h1 = take((size_t)nrhs * (m + 1) * 16), o_h2 = take((size_t)nrhs * (m + 1) * 16);
    const size_t o_coef = take((size_t)nrhs * (m + 1) * 16), o_ivn = take((size_t)nrhs * (m + 1) * 8);
    const size_t o_y = take((size_t)nrhs * m * 16);
    const size_t o_nrm = take(nrhs * 8), o_np = take((size_t)nrhs * nb * 8), o_inv = take(nrhs * 8);
    const size_t o_bn = take(nrhs * 8), o_rn = take(nrhs * 8);
    const size_t o_H = take((size_t)nrhs * m * (m + 1) * 16), o_cs = take((size_t)nrhs * m * 16);
    const size_t o_sn = take((size_t)nrhs * m * 16), o_g = take((size_t)nrhs * (m + 1) * 16);
    const size_t o_slot = take((size_t)nrhs * 16), o_stat = take(4 * sizeof(int));
    const size_t o_Hr = take((size_t)nrhs * m * (m + 1) * 16), o_coef2 = take((size_t)nrhs * (m + 1) * 16);
    const size_t o_dp = take((size_t)nrhs * nb * 16), o_pc = take((size_t)nrhs * 2 * 16);
    const size_t o_col = take((size_t)nrhs * (m + 1) * 16), o_np2 = take((size_t)nrhs * nb * 8);
    const size_t o_g3 = take((size_t)3 * nrhs * (m + 1) * 16), o_coef3 = take((size_t)3 * nrhs * (m + 1) * 16);
    const size_t o_tc = take((size_t)nrhs * 8 * 16), o_col2 = take((size_t)nrhs * (m + 2) * 16);
    const size_t o_gp = take((size_t)nrhs * nb * 8 * 8), o_np3 = take((size_t)nrhs * nb * 8);
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
    L.H = reinterpret_cast<double2*>(base + o_H);
    L.cs = reinterpret_cast<double2*>(base + o_cs);
    L.sn = reinterpret_cast<double2*>(base + o_sn);
    L.g = reinterpret_cast<double2*>(base + o_g);
    L.slot = reinterpret_cast<double2*>(base + o_slot);
    L.stat = reinterpret_cast<int*>(base + o_stat);
    L.Hr = reinterpret_cast<double2*>(base + o_Hr);
    L.coef2 = reinterpret_cast<double2*>(base + o_coef2);
    L.dpart = reinterpret_cast<double2*>(base + o_dp);
    L.pc = reinterpret_cast<double2*>(base + o_pc);
    L.col = reinterpret_cast<double2*>(base + o_col);
    L.npart2 = reinterpret_cast<double*>(base + o_np2);
    L.g3 = reinterpret_cast<double2*>(base + o_g3);
    L.coef3 = reinterpret_cast<double2*>(base + o_coef3);
    L.tc = reinterpret_cast<double2*>(base + o_tc);
    L.col2 = reinterpret_cast<double2*>(base + o_col2);
    L.gpart = reinterpret_cast<double*>(base + o_gp);
    L.npart3 = reinterpret_cast<double*>(base + o_np3);
    if (st)
        for (int r = 0; r < nrhs; ++r) st[r] = vie_solve_stats{};

    const double dv = c.D[0] * c.D[1] * c.D[2];
    const double ginv[4] = {1 / dv, 12 / dv, 12 / dv, 12 / dv};
    if (c.nc == 24) {
        // J-M: the curl operator and the product's buffers exist before any
        // Arnoldi step (which may be captured)
        ensure_curl(c);
        c.jmbuf.get((size_t)2 * nrhs * 24 * c.V * sizeof(double2));
        jm_rhs_prec(c, nrhs, et, L.rhs);
    } else {
        launch_rhs_prec(L.rhs, et, c.mat.tau, ginv, make_double2(0.0, c.omega * kEps0), c.V, nrhs, c.nc, c.stream);
    }
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
