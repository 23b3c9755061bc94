// Host-side launchers of the device kernels.
#pragma once

#include <hip/hip_ext.h>

#include "assembly.hpp"
#include "passes.hpp"

namespace vie {

// Start / stop events for the next kernel launch of the operator passes:
// hipExtLaunchKernelGGL stamps them from the kernel's own dispatch, so the
// time between them is the kernel's duration without event packets around
// it.  Set by the launch profiler, consumed (and cleared) by one launch.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchTiming g_launch_timing;

template <typename F, typename... Args>
inline void timed_launch(F kernel, const dim3& grid, const dim3& block, unsigned lds, hipStream_t s, Args... args) {
    const LaunchTiming t = g_launch_timing;
    g_launch_timing = LaunchTiming{};
    if (t.start || t.stop) hipExtLaunchKernelGGL(kernel, grid, block, lds, s, t.start, t.stop, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// passes.hip
template <typename R>
void launch_strided(bool fwd, const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2, long long n_o1,
                    const C<R>* tw, const Epilogue<R>* ep, hipStream_t s);
template <typename R>
void launch_p3(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s);
// x pass of the PWC basis (3 component rows per pencil, compiled lengths only)
template <typename R>
void launch_p3_pwc(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s);
// x pass of the curl operator K (U the [Oz][Oy][30][Ox] octant)
template <typename R>
void launch_p3_curl(C<R>* A, const C<R>* U, const P3Params& p, const C<R>* tw, hipStream_t s);
// x pass of the J-M product: the coupled sums s_j = N x_j + kj K x_m and
// s_m = N x_m + km K x_j of the vector pairs (2 r, 2 r + 1), p.nrhs pairs (UN
// the 60-tensor octant, UK the 30-tensor curl octant); false when the length
// along x has no compiled kernel (the caller then composes the two products)
template <typename R>
bool launch_p3_jm(C<R>* A, const C<R>* UN, const C<R>* UK, const P3Params& p, const C<R>* tw, C<R> kj, C<R> km,
                  hipStream_t s);
bool p3_ct_supported(int n);
int p3_ct_groups(int es, int n);
bool p3_ct_fits(int es, int n);
bool p3_quad_fits(int es, int n);
bool p3_pair_fits(int es, int n);
bool p3_pref_fits(int n);
// strided.hip: compiled-length strided passes; false when (length, tile)
// has no compiled kernel
template <typename R>
bool launch_strided_compiled(bool fwd, bool epi, const C<R>* in, C<R>* out, const StridedPass& p, long long n_o2,
                             long long n_o1, const C<R>* tw, const Epilogue<R>& ep, hipStream_t s);
bool strided_ct_fits(int es, int n, int tile);
bool strided_tile_ok(int es, int n, int tile);
int strided_tile_for(int es, int n, int preferred);
template <typename R>
void launch_rows(bool fwd, C<R>* data, long long nrows, const FftPlan& plan, const C<R>* tw, hipStream_t s);

// operator.hip
AssemblyTables build_assembly_tables(const double D[3], double k0);
AssemblyTables build_curl_tables(const double D[3], double k0);
// T.nent unique tensors [nent][Nz][Ny][Nx] for offsets d >= 0
void assemble_blocks(double2* out, const AssemblyTables& T, int Nx, int Ny, int Nz, hipStream_t s);
int unique_refl_sign(int e, int axis);
int curl_refl_sign(int e, int axis);
// circulant embedding, 3-D FFT and octant [Oz][Oy][nent][Ox] of the 60 N
// tensors, or of the 30 curl tensors (curl = true; U64 may be null)
void embed_and_transform(double2* U128, float2* U64, const double2* T, double2* circ, int Nx, int Ny, int Nz,
                         int Mx, int My, int Mz, const FftPlan plans[3], const double2* const tw[3], hipStream_t s,
                         bool curl = false);

// setup.hip: materials, excitation, post-processing
struct Materials {
    double2* eps_r;   // per voxel
    double2* chi;
    double2* tau;
    float2* tau64;
    float2* epsr64;
    float2* chi64;
};
void launch_materials(const double* eps_re, const double* sigma, double omega_eps0, Materials m, long long V,
                      int* bad_flag, hipStream_t s);
// nc: unknowns per voxel (12 PWL, 3 PWC)
void launch_planewave(double2* et, int Nx, int Ny, int Nz, const double D[3], double k0, int pol, int dir,
                      double sgn, double amp, int nc, hipStream_t s);
// magnetic = 1: the dipoles' magnetic field, tested on every voxel
void launch_dipoles(double2* et, int nrhs, const double* pos_dev, const double* mom_dev, int nq,
                    const double* glx, const double* glw, const double2* chi, int Nx, int Ny, int Nz,
                    const double D[3], double k0, double omega_eps0, int nc, hipStream_t s, int magnetic = 0);
void launch_b1plus(double2* b, const double2* h, double mu0, long long V, int nrhs, hipStream_t s);
void launch_magnetic_energy(double* w, double* partial, const double2* h, const double2* chi, double mu0, double dv,
                            long long V, int nrhs, int nblocks, hipStream_t s);
void launch_rhs_prec(double2* rhs, const double2* et, const double2* tau, const double ginv[4], double2 ce,
                     long long V, int nrhs, int nc, hipStream_t s);
void launch_fields(double2* e, const double2* x, const double2* chi, double2 ce, long long V, int nrhs, int nc,
                   hipStream_t s);
void launch_total_field(double2* e, const double2* et, const double2* x, const double gram[4], double2 ce,
                        long long V, int nrhs, int nc, hipStream_t s);
void launch_power_partials(double* partial, const double2* x, const double2* chi, const double gram[4], double2 ce,
                           long long V, int nrhs, int nc, int nblocks, hipStream_t s);
void launch_power_density(double* p, const double2* e, const double* sigma, long long V, int nrhs, int nc,
                          hipStream_t s);

// krylov.hip: Gram-Schmidt and vector kernels, FP64 accumulation
template <typename R>
void launch_multidot(double2* partial, const C<R>* Vb, long long ldv, int nvec, const C<R>* w, long long n,
                     long long rstride_v, long long rstride_w, int nrhs, int nblocks, hipStream_t s);
// the basis is stored unnormalised, v_i = u_i * ivn[i] (ivn at stride ivn_ld
// per right-hand side); jw names the vector the operator was applied to
// (w = A u_jw), or jw < 0 for a second pass
void launch_reduce_partials(double2* h, double2* coef, const double2* partial, int nvec, int nblocks, int nrhs,
                            const double* ivn, long long ivn_ld, int jw, hipStream_t s);
template <typename R>
void launch_update(C<R>* w, const C<R>* Vb, long long ldv, int nvec, const double2* coef, long long n,
                   long long rstride_v, long long rstride_w, double* norm_partial, const double* ivn,
                   long long ivn_ld, int jw, int nrhs, int nblocks, hipStream_t s);
void launch_reduce_norm(double* out, const double* partial, int nblocks, int nrhs, hipStream_t s,
                        double* inv = nullptr, long long inv_ld = 0);
template <typename R>
void launch_scale_into(C<R>* dst, const C<R>* src, const double* norms, long long n, long long rstride_dst,
                       long long rstride_src, int nrhs, hipStream_t s);
template <typename R>
void launch_combine(double2* x, const C<R>* Vb, long long ldv, int nvec, const double2* y, long long n,
                    long long rstride_v, int nrhs, hipStream_t s);
template <typename R>
void launch_norm_partials(double* partial, const C<R>* v, long long n, long long rstride, int nrhs, int nblocks,
                          hipStream_t s);
// Least-squares side of one GMRES restart cycle on the device, FP64, per
// slot s of na right-hand sides (Sec. V: restarted GMRES): the rotated
// Hessenberg matrix (column-major, column j at H + (s m + j)(m + 1)), the
// Givens rotations of the columns so far, and the rotated ||r|| e_1.
struct ArnoldiState {
    double2* H;            // [na][m][m + 1]
    double2* cs;           // [na][m]
    double2* sn;           // [na][m]
    double2* g;            // [na][m + 1]
    const double2* slot;   // [na]: (||r||, target of |g_{j+1}| / ||r||)
    int* status;           // [0] columns folded in, [1] every slot has met its
                           // target, [2] a non-finite estimate was seen
    int m;
    double2* Hr;           // [na][m][m + 1]: the unrotated columns (or nullptr)
};
// zero the status, g_0 = ||r||, ivn of the first basis vector = 1
void launch_arnoldi_init(ArnoldiState st, double* ivn, long long ivn_ld, int na, hipStream_t s);
// sum the norm partials of the new vector w (npart [na][nblocks]) into
// nrm[s] and its reciprocal ivn_next[s * ivn_ld] (0 for a zero vector), then
// fold Hessenberg column j (h1 (+ h2 with a second pass) above the diagonal,
// ||w|| below) into the rotations and the residual estimate; the rotations
// are left alone once status[1] or status[2] is set
void launch_givens(ArnoldiState st, const double2* h1, const double2* h2, const double* npart, int nblocks,
                   double* nrm, double* ivn_next, long long ivn_ld, int j, int na, hipStream_t s);
// Two Arnoldi steps per pass over the basis (s-step Arnoldi with s = 2, the
// second vector shifted by the Rayleigh quotient h_jj; krylov.hip states the
// algebra).  Dot partials of V against w and w + ldw: 2 planes of
// [nrhs][nvec][nblocks].
template <typename R>
void launch_multidot2(double2* partial, const C<R>* Vb, long long ldv, int nvec, const C<R>* w, long long ldw,
                      long long n, long long rstride_v, long long rstride_w, int nrhs, int nblocks, hipStream_t s);
// h (column j above the diagonal), g (= V^H (A - h_jj) w1) and the update
// coefficients of both from the 2 planes (w1 = A u_jw)
void launch_reduce_pair(double2* h, double2* coef, double2* gcol, double2* coef2, const double2* partial, int nvec,
                        int nblocks, int nrhs, const double* ivn, long long ivn_ld, int jw, hipStream_t s);
// both updates in one pass over the basis (w2 = w + ldv), with the partial
// sums of ||w1||^2 and conj(w1) w2
template <typename R>
void launch_update_pair(C<R>* w, const C<R>* Vb, long long ldv, int nvec, const double2* coef, const double2* coef2,
                        const double2* h, long long n, long long rstride_v, long long rstride_w, double* norm_partial,
                        double2* dot_partial, const double* ivn, long long ivn_ld, int jw, int nrhs, int nblocks,
                        hipStream_t s);
// pc[2 s] = conj(w1) w2 / ||w1||^2, pc[2 s + 1] = (1 / ||w1||, ||w1||)
void launch_pair_coef(double2* pc, const double2* dpart, int nblocks, const double* nrm, int nrhs, hipStream_t s);
// u_{j+2} = (w2 - pc0 u_{j+1}) pc1 in place, with its norm partials
template <typename R>
void launch_axpy_pair(C<R>* u1, long long ldv, long long n, long long rstride, const double2* pc,
                      double* norm_partial, int nrhs, int nblocks, hipStream_t s);
// Hessenberg column j + 1 of the pair, entries 0..j + 1, into col [na][j + 2]
void launch_pair_column(ArnoldiState st, const double2* h, const double2* gcol, const double2* pc, double2* col,
                        int j, int na, hipStream_t s);
// Three Arnoldi steps per pass over the basis (s = 3; krylov.hip states the
// algebra): dot partials against w, w + ldw, w + 2 ldw (3 planes); g_k and
// their update coefficients at g + k gst, coef + k gst; the three updates in
// one pass with the block's Gram partials ([nrhs][nblocks][8]); the Cholesky
// factor and storage coefficients tc [nrhs][8]; u_{j+2}, u_{j+3} formed in
// place with their norm partials; Hessenberg columns j + 1 and j + 2.
template <typename R>
void launch_multidot3(double2* partial, const C<R>* Vb, long long ldv, int nvec, const C<R>* w, long long ldw,
                      long long n, long long rstride_v, long long rstride_w, int nrhs, int nblocks, hipStream_t s);
void launch_reduce_triple(double2* g, double2* coef, const double2* partial, int nvec, int nblocks, int nrhs,
                          const double* ivn, long long ivn_ld, int jw, long long gst, hipStream_t s);
template <typename R>
void launch_update_triple(C<R>* w, const C<R>* Vb, long long ldv, int nvec, const double2* coef, long long gst,
                          const double2* g, long long n, long long rstride_v, long long rstride_w,
                          double* norm_partial, double* gram_partial, const double* ivn, long long ivn_ld, int jw,
                          int nrhs, int nblocks, hipStream_t s);
void launch_triple_coef(double2* tc, const double* gpart, int nblocks, int nrhs, hipStream_t s);
template <typename R>
void launch_axpy_triple(C<R>* u1, long long ldv, long long n, long long rstride, const double2* tc, double* np2,
                        double* np3, int nrhs, int nblocks, hipStream_t s);
void launch_triple_columns(ArnoldiState st, const double2* g, long long gst, const double2* tc, double2* col1,
                           double2* col2, int j, int na, hipStream_t s);
// y = R^-1 g over the first nvec columns, scaled by the basis vectors'
// reciprocal norms (the coefficients of the stored vectors), y [na][nvec]
void launch_backsolve(ArnoldiState st, const double* ivn, long long ivn_ld, double2* y, int nvec, int na,
                      hipStream_t s);
void launch_cast_down(float2* dst, const double2* src, const double* scale, long long n, int nrhs, hipStream_t s);
void launch_cast_up(double2* dst, const float2* src, long long n, hipStream_t s);
void launch_copy_c128(double2* dst, const double2* src, long long n, hipStream_t s);
void launch_nonfinite(int* flag, const double2* v, long long n, hipStream_t s);

}  // namespace vie
