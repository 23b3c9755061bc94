/*
 * vie.h - C ABI of the MI355X volume-integral-equation library.
 *
 * The method: the current-based volume integral equation for a dielectric
 * body discretised with discontinuous piecewise-linear (PWL) voxel bases and
 * Galerkin testing (Georgakis et al., "A Fast Volume Integral Equation Solver
 * with Linear Basis Functions for the Accurate Computation of EM Fields in
 * MRI", IEEE TAP 2020).  Sec. III gives the system
 *     A x = b,  A = M_eps G - M_chi N,  b = c_e M_chi e_inc        (eq. 24)
 * with 12 unknowns per voxel (3 components x 4 scalar bases, eq. 19-22);
 * Sec. IV-A the FFT-accelerated product through circulant embedding of the
 * block-Toeplitz tensors (eq. 42-43); Sec. IV-B the preconditioner
 * P = M_eps G (eq. 17); Sec. IV-C fields and absorbed power (eq. 44).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Grid: Nx x Ny x Nz voxels of size dx x dy x dz (metres), box centred at
 *   the origin; voxel centres at (n_i - (N_i - 1)/2) * d_i.
 * - Vectors of unknowns ("x" layout): [nrhs][nc][Nz][Ny][Nx], x fastest,
 *   interleaved complex (real, imag).  PWL basis (nc = 12, the default):
 *   unknown index a = 4 p + (l - 1), p in {x, y, z} -> 0..2, l = 1 (pulse),
 *   2..4 (linear in x, y, z) (eq. 30).  PWC basis (nc = 3, vie_set_basis):
 *   unknown index p, the pulse coefficients alone.
 * - Per-voxel arrays: [Nz][Ny][Nx].
 * - precision: VIE_C64 (complex64, FP32 arithmetic) or VIE_C128 (complex128).
 * - Time factor exp(+i w t); eps_r = eps' - i sigma / (w eps0) (eq. 2).
 * - Device pointers are HIP device addresses (e.g. torch tensor data_ptr()).
 *   The caller owns every buffer it passes; the context owns the operator,
 *   the contrast and its workspaces.
 * - All device work is ordered on the context's stream.  Calls that return
 *   host data (norms, stats, powers) synchronise that stream.
 * - Errors: a negative vie_status is returned and a message is kept per
 *   thread (vie_last_error).  No exception crosses the ABI.  After an error
 *   the context stays usable unless the status is VIE_EDEVICE.
 */
#ifndef VIE_H
#define VIE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vie_ctx vie_ctx;

typedef enum {
    VIE_OK = 0,
    VIE_EINVAL = -1,   /* bad argument (shape, pointer, option)            */
    VIE_ENOMEM = -2,   /* device allocation failed                          */
    VIE_EDEVICE = -3,  /* HIP runtime error                                 */
    VIE_ENOCONV = -4,  /* solver stopped before the tolerance (x = best)    */
    VIE_ENAN = -5,     /* non-finite input or iterate                       */
    VIE_ESTATE = -6    /* call out of order (e.g. apply before set_grid)     */
} vie_status;

enum { VIE_C64 = 0, VIE_C128 = 1 };

/* operator selector for vie_apply */
enum {
    VIE_OP_PREC = 0,  /* y = P^-1 A x = x - tau (G^-1 N x)          (eq. 17)  */
    VIE_OP_A = 1,     /* y = A x = eps_r G x - chi (N x)            (eq. 24a) */
    VIE_OP_N = 2      /* y = N x, the Galerkin N product            (eq. 25a) */
};

/* solver precision mode */
enum {
    VIE_SOLVE_FP64 = 0,     /* GMRES in complex128                            */
    VIE_SOLVE_FP32_IR = 1   /* complex64 GMRES inside FP64 iterative refinement */
};

typedef struct {
    int mode;            /* VIE_SOLVE_FP64 or VIE_SOLVE_FP32_IR               */
    int restart;         /* GMRES restart length (paper: 50)                  */
    int max_outer;       /* max restart cycles per solve (paper: 200)         */
    double tol;          /* relative residual ||P^-1(b - A x)|| / ||P^-1 b||  */
    double inner_tol;    /* FP32_IR: relative reduction per inner solve       */
    int max_refine;      /* FP32_IR: max refinement steps (>= 1); each is one
                            complex64 GMRES(restart) cycle on the current
                            residual, so at most min(max_outer, max_refine)
                            cycles run                                        */
    int reorth;          /* 1: second Gram-Schmidt pass per Arnoldi step      */
    int use_x0;          /* 1: x holds the initial guess, 0: start from zero  */
    int graph;           /* 1: replay the Arnoldi steps from HIP graphs (a
                            run of steps is captured the second time the
                            solver reaches it with the same shapes and
                            buffers), 0: launch every kernel, -1 (default):
                            replay when a batch of vectors is at most 2 MB;
                            the results are the same bits either way          */
    int sync_steps;      /* Arnoldi steps per host check of the device-side
                            convergence flag (the Givens rotations and the
                            residual estimate run on the device); 0: chosen
                            from the vector size.  Larger values cost fewer
                            host round trips and up to 2 sync_steps - 1
                            steps computed past convergence                   */
    int s_step;          /* Arnoldi steps per pass over the basis: 1, the
                            classical step (one product, then Gram-Schmidt
                            against the basis); 2 or 3, as many products,
                            then one dot and one update pass over the basis
                            for all of them (s-step Arnoldi, the new vectors
                            shifted by the Rayleigh quotient h_jj and
                            orthogonalised among themselves in FP64), which
                            cuts the basis reads per step to about a half or
                            a third; 0 (default): 3.  reorth = 1 always runs
                            single steps.  The iterates of 1, 2 and 3 agree
                            to rounding, not bitwise                          */
} vie_solve_opts;

typedef struct {
    int converged;       /* 1 when the relative residual <= tol               */
    int iterations;      /* inner GMRES iterations (Arnoldi steps)            */
    int restarts;        /* restart cycles                                    */
    int refinements;     /* FP64 refinement steps (FP32_IR)                   */
    int matvecs_c64;     /* operator products in complex64                    */
    int matvecs_c128;    /* operator products in complex128                   */
    double rel_residual; /* final true relative residual (FP64)               */
    double seconds;      /* wall time of the solve                            */
} vie_solve_stats;

/* -- context ------------------------------------------------------------- */

/* Create a context bound to HIP device `device` and stream `stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
int vie_create(vie_ctx** out, int device, void* stream);
void vie_destroy(vie_ctx* ctx);
/* Message of the last failing call on this thread ("" if none). */
const char* vie_last_error(void);
/* Change the stream later calls are ordered on. */
int vie_set_stream(vie_ctx* ctx, void* stream);

/* -- grid and operator (Sec. III-A, III-C, IV-A) ---------------------------- */

/* Define the voxel grid and frequency and build the operator: the 60 unique
 * Toeplitz-defining block tensors N^{pl,ql'}(d), d in [0, N)^3 (eq. 42-43;
 * 60 unique, Sec. V) are assembled on the device in FP64, embedded in
 * circulants on the fft grid with the reflection signs of the PWL bases,
 * transformed, and the octant xi_i <= M_i/2 kept in complex128 and
 * complex64.  fft_size: NULL selects for each axis the smallest even
 * 2/3/5-smooth M_i >= 2 N_i (2 N_i itself when smooth); otherwise each M_i
 * must be >= 2 N_i - 1, even, 2/3/5-smooth and <= 4096.  Frees any previous
 * grid and contrast state. */
int vie_set_grid(vie_ctx* ctx, int nx, int ny, int nz, double dx, double dy, double dz,
                 double freq_hz, const int* fft_size);

/* Discretisation of later calls: ncomp = 12 selects the PWL basis (the
 * default), ncomp = 3 the piecewise-constant (PWC) basis the paper compares
 * against (Sec. I, Sec. V: 3 unknowns per voxel, 6 unique tensors).  The PWC
 * basis is the pulse function of each voxel and component, i.e. the l = 1
 * members of the PWL basis, so its Galerkin system is the PWL one restricted
 * to a = 4 p: operator tensors u = 10 pq (ll = 11) of the same assembled
 * operator, Gram dV.  Vectors of every later call hold ncomp unknowns per
 * voxel.  Clears the launch-shape choices; may be called at any time.  The
 * PWC product needs an fft length along x of 8, 16, 32, 64, 96, 128, 160,
 * 192, 256, 320, 384 or 512: a later vie_set_grid without fft_size picks the
 * smallest of them >= 2 Nx for a PWC context; products on other lengths
 * return VIE_EINVAL.
 *
 * ncomp = 24 selects the J-M formulation on the PWL basis (Sec. II, eq.
 * 13-15): objects with magnetic contrast carry polarisation and
 * magnetisation currents j = c_e chi_e e and m = c_m chi_m h (eq. 6-7,
 * c_m = i w mu0); a vector holds per right-hand side the 12 electric then
 * the 12 magnetic coefficients ([nrhs][24][Nz][Ny][Nx]).  The operator is
 *   (A x)_j = eps_r G x_j - chi_e (N x_j - c_e K x_m)
 *   (A x)_m = mu_r G x_m - chi_m (N x_m + c_m K x_j)
 * with K the curl operator (eq. 8b, 25b), preconditioned by
 * P = diag(M_eps G, M_mu G); incident calls write [e_t; h_t], vie_rhs_prec
 * and vie_solve take them, vie_fields returns [e; h], vie_absorbed_power
 * adds the magnetic loss; vie_apply takes VIE_OP_PREC and VIE_OP_A.
 * The magnetic contrast is mu_r = 1 until vie_set_magnetic_contrast.
 * vie_total_field, vie_power_density, the magnetic-field calls and
 * vie_apply_noalloc refuse a J-M context (VIE_EINVAL).  Returns VIE_EINVAL
 * for ncomp other than 12, 3 or 24. */
int vie_set_basis(vie_ctx* ctx, int ncomp);

/* Debug / parity entry: replace the operator by caller-supplied unique block
 * tensors T_host [60][Nz][Ny][Nx] complex128 (host memory), d >= 0 octant,
 * unique index u = 10 * pq + ll with pq over (xx, xy, xz, yy, yz, zz) and
 * ll over (11, 12, 13, 14, 22, 23, 24, 33, 34, 44) (l <= l'), each entry being
 * N^{(p,l),(q,l')}(d) with p <= q, l <= l'.  Requires vie_set_grid first. */
int vie_set_toeplitz(vie_ctx* ctx, const double* T_host);

/* Copy the assembled unique block tensors (layout of vie_set_toeplitz) to a
 * host buffer of 60 * Nz * Ny * Nx complex128. */
int vie_get_toeplitz(vie_ctx* ctx, double* T_host);

/* -- Tucker compression of the operator (Sec. III-C, last paragraph) ------- */

/* The Toeplitz-defining tensors of eq. 43 keep a low multilinear rank
 * (Sec. III-C, last paragraph; Sec. V leaves their memory out of the
 * footprint for that reason).  A compressed tensor is a core times one
 * factor with orthonormal columns per axis: T_hat = core x_x U_x x_y U_y
 * x_z U_z. */
typedef struct {
    int ranks[60][3];         /* (r_x, r_y, r_z) of each unique tensor          */
    double rel_error[60];     /* ||T - T_hat||_F / ||T||_F per tensor            */
    double max_rel_error;     /* the largest of them (<= tol)                    */
    size_t bytes_dense;       /* the 60 tensors, complex128                      */
    size_t bytes_compressed;  /* cores and factors, complex128                   */
    double seconds;           /* wall time of the compression                    */
} vie_tucker_info;

/* Compress the context's 60 unique tensors (layout of vie_set_toeplitz) by
 * sequentially truncated HOSVD in the axis order x, y, z: for each axis the
 * eigenvectors of the FP64 Gram matrix of the unfolding of the tensor as
 * compressed so far, keeping the fewest whose dropped eigenvalues sum to at
 * most tol^2 ||T||_F^2 / 3, then the projection onto them.  Every tensor
 * is then within tol of itself in the Frobenius norm (the dropped
 * eigenvalues add up to the squared error exactly).  The compressed form
 * (host memory, owned by the context, freed with the grid) replaces any
 * earlier one; the operator is left as it was.  tol in [1e-7, 1):
 * VIE_EINVAL otherwise; VIE_ESTATE before vie_set_grid.  info (host, may be
 * NULL) receives ranks, errors and sizes. */
int vie_tucker_compress(vie_ctx* ctx, double tol, vie_tucker_info* info);

/* Write the reconstruction T_hat of the compressed form to out (device,
 * 60 * Nz * Ny * Nx complex128, layout of vie_set_toeplitz; must not overlap
 * the context's own blocks).  VIE_ESTATE without a compressed form. */
int vie_tucker_reconstruct(vie_ctx* ctx, void* out);

/* Replace the context's blocks by T_hat and rebuild the operator from them
 * (circulant embedding, 3-D FFT, octant in complex128 and complex64, as
 * vie_set_grid does), so later products and solves use the compressed
 * operator.  VIE_ESTATE without a compressed form or when the operator is
 * shared with another context (vie_share_grid). */
int vie_tucker_expand(vie_ctx* ctx);

/* Make dst use src's grid and operator (the same device buffers, read-only,
 * freed with the last context that uses them) instead of assembling its own;
 * dst's launch-shape choices are copied from src and its contrast cleared.
 * For many solves on one grid from several contexts or streams.  Waits for
 * src's stream.  vie_set_toeplitz refuses a shared operator. */
int vie_share_grid(vie_ctx* dst, const vie_ctx* src);

/* FFT grid size {M_x, M_y, M_z} chosen by vie_set_grid (host int[3]). */
int vie_fft_size(vie_ctx* ctx, int* m3);

/* -- materials and excitation (eq. 2, 7, 17, 27, 30-31) --------------------- */

/* Per-voxel relative permittivity eps' and conductivity sigma (S/m), FP64
 * [Nz][Ny][Nx], host (on_device = 0) or device pointers.  Computes eps_r,
 * chi = eps_r - 1 and tau = chi / eps_r on the device.  VIE_ENAN on
 * non-finite input, VIE_EINVAL on eps' <= 0 or sigma < 0. */
int vie_set_contrast(vie_ctx* ctx, const double* eps_re, const double* sigma, int on_device);

/* J-M formulation (vie_set_basis 24) only: per-voxel relative permeability
 * mu_r = mu' - i mu'' (eq. 2), FP64 [Nz][Ny][Nx], host (on_device = 0) or
 * device pointers; computes chi_m = mu_r - 1 and tau_m = chi_m / mu_r.
 * VIE_ENAN on non-finite input, VIE_EINVAL on mu' <= 0, mu'' < 0 or a
 * context that is not J-M.  Replaced by mu_r = 1 when the grid or the
 * basis changes. */
int vie_set_magnetic_contrast(vie_ctx* ctx, const double* mu_re, const double* mu_im, int on_device);

/* Tested incident field of a plane wave E0 pol exp(-i k0 dir . r) (eq. 30,
 * plane wave of Sec. V-A for pol = x, dir = z), into e_t (device,
 * [nc][Nz][Ny][Nx] complex128).  pol and dir must be orthogonal unit vectors
 * along coordinate axes. */
int vie_incident_planewave(vie_ctx* ctx, const double pol[3], const double dir[3], double amp,
                           void* e_t);

/* Tested incident fields of nrhs Hertzian dipoles (current moment vectors in
 * A m at positions in m, host arrays [nrhs][3]) into e_t (device,
 * [nrhs][nc][Nz][Ny][Nx] complex128), by nq^3-point Gauss quadrature per
 * voxel on voxels with chi != 0 (others set to zero). */
int vie_incident_dipoles(vie_ctx* ctx, int nrhs, const double* pos, const double* moment, int nq,
                         void* e_t);

/* Preconditioned right-hand side P^-1 b = c_e tau G^-1 e_t (eq. 17, 31),
 * e_t and rhs complex128 device arrays in x layout. */
int vie_rhs_prec(vie_ctx* ctx, int nrhs, const void* e_t, void* rhs);

/* -- operator product (Sec. IV-A) ------------------------------------------ */

/* y = op(x) for nrhs vectors in x layout, precision VIE_C64 or VIE_C128,
 * device pointers, asynchronous on the context stream.  x and y must not
 * overlap (VIE_EINVAL when their byte ranges intersect).  Requires
 * vie_set_grid (and vie_set_contrast for OP_PREC/OP_A).  The FFT
 * intermediates live in a context workspace that grows on demand. */
int vie_apply(vie_ctx* ctx, int op, int precision, int nrhs, const void* x, void* y);

/* -- operator product without device allocation ----------------------------- */

/* Fixed size of the per-device workspace of vie_apply_noalloc: 64 MiB. */
#define VIE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid it): the same product as
 * vie_apply (same arguments, kernels and launch shapes, so the same result
 * bit for bit), with the FFT intermediates in a fixed per-device workspace of
 * VIE_NOALLOC_SCRATCH_BYTES that the library holds from load until the
 * process ends, instead of the context's growing one.  It calls no device
 * allocation or free.  The intermediates take
 *     nrhs * es * (sR1 + sR2) bytes,  es = 8 (VIE_C64) or 16 (VIE_C128),
 *     sR1 = M_z (N_y nc N_x + 32) + 96,  sR2 = M_z (M_y nc N_x + 32) + 96,
 * with nc unknowns per voxel and the fft sizes M of vie_fft_size (e.g. one
 * complex64 PWL vector on 48^3 voxels, or one complex128 on 36^3); larger
 * requests return VIE_EINVAL before any launch.  The workspace is shared by
 * every call on one GPU and keeps the last call's contents: calls on one GPU
 * that overlap in time (other contexts or streams) race and must be ordered
 * by the caller.  The context must have been set up (vie_set_grid, and
 * vie_set_contrast for OP_PREC/OP_A); launch profiling is not applied. */
int vie_apply_noalloc(vie_ctx* ctx, int op, int precision, int nrhs, const void* x, void* y);

/* -- solve (Sec. IV-B, V: GMRES(50), left preconditioner P = M_eps G) ------- */

void vie_default_opts(vie_solve_opts* opts);

/* Solve P^-1 A x = P^-1 b for nrhs right-hand sides given as tested incident
 * fields e_t (device, complex128, x layout).  x (device, complex128) receives
 * the current coefficients (eq. 19); with opts->use_x0 it also holds the
 * initial guess.  stats (host, nrhs entries, may be NULL).  Returns VIE_OK
 * when every right-hand side converged, VIE_ENOCONV otherwise (x holds the
 * last iterate). */
int vie_solve(vie_ctx* ctx, const vie_solve_opts* opts, int nrhs, const void* e_t, void* x,
              vie_solve_stats* stats);

/* -- post-processing (Sec. IV-C, eq. 44, Sec. V-C) ------------------------- */

/* Field coefficients e = x / (c_e chi) on voxels with chi != 0, zero
 * elsewhere (eq. 6); complex128 device arrays in x layout. */
int vie_fields(vie_ctx* ctx, int nrhs, const void* x, void* e);

/* Total field coefficients everywhere in the box, tissue and air, through
 * one operator product (Sec. IV-C): G e = e_t + (N - G) x / c_e, i.e.
 * e = G^-1 (e_t + (N x - G x) / c_e) with the tested incident field e_t.  On
 * tissue voxels this equals vie_fields at the exact discrete solution.
 * e_t, x and e: complex128 device arrays in x layout; e must overlap
 * neither x nor e_t (it receives N x before e_t is read): VIE_EINVAL
 * otherwise.  Requires vie_set_grid. */
int vie_total_field(vie_ctx* ctx, int nrhs, const void* e_t, const void* x, void* e);

/* Absorbed power P_abs = 1/2 Re{x^* (c_e M_chi)^-1 G x} (eq. 44) per
 * right-hand side, into p_abs_host[nrhs] (W). */
int vie_absorbed_power(vie_ctx* ctx, int nrhs, const void* x, double* p_abs_host);

/* Voxel power density 1/2 sigma |e|^2 averaged over each voxel (Sec. V-C),
 * FP64 device array [nrhs][Nz][Ny][Nx], from field coefficients e. */
int vie_power_density(vie_ctx* ctx, int nrhs, const void* e, double* p_dev);

/* -- magnetic field and MRI quantities (Sec. II eq. 8b, 'tot_fields' b;
 *    Sec. III eq. 25b; Sec. V-D) ------------------------------------------- */

/* Tested incident magnetic field of the plane wave of vie_incident_planewave
 * with the same arguments: H = (1/eta0) dir x E, i.e. amp / eta0 along
 * dir x pol (eta0 = sqrt(mu0 / eps0)); into h_t (device, complex128,
 * [nc][Nz][Ny][Nx]). */
int vie_incident_planewave_h(vie_ctx* ctx, const double pol[3], const double dir[3], double amp, void* h_t);

/* Tested incident magnetic fields of nrhs Hertzian dipoles (arguments as for
 * vie_incident_dipoles): H = curl (g I l) = (1 + i k0 R) exp(-i k0 R) /
 * (4 pi R^2) (I l x R_hat), by nq^3-point Gauss quadrature on every voxel
 * (the sources must lie outside the voxels), into h_t (device, complex128,
 * [nrhs][nc][Nz][Ny][Nx]).  Requires vie_set_grid. */
int vie_incident_dipoles_h(vie_ctx* ctx, int nrhs, const double* pos, const double* moment, int nq, void* h_t);

/* Total magnetic field h_tot = h_inc + K j (eq. 'tot_fields' b), K = curl S
 * (eq. 8b) discretised on the PWL basis (eq. 25b): the coefficients
 * h = G^-1 (h_t + K x) everywhere in the box, from the tested incident
 * magnetic field h_t and the current coefficients x (device, complex128, x
 * layout, nrhs vectors; h must not overlap x, it may alias h_t).  The 30
 * unique tensors of K (Sec. III-C) are assembled and transformed on the
 * first call for a grid (and kept with the grid's operator).  PWL basis and
 * fft lengths along x up to 256 only (VIE_EINVAL otherwise). */
int vie_magnetic_field(vie_ctx* ctx, int nrhs, const void* h_t, const void* x, void* h);

/* b1+ = mu0 (h_x + i h_y) (Sec. V-D) as PWL coefficients: b[r][l][v] =
 * mu0 (h^{x,l} + i h^{y,l}) for l = 1..4; h complex128 [nrhs][12][V],
 * b complex128 [nrhs][4][Nz][Ny][Nx] (device). */
int vie_b1plus(vie_ctx* ctx, int nrhs, const void* h, void* b);

/* Magnetic energy (Sec. V-D): the density w_m = 1/4 mu0 |h|^2 averaged over
 * each voxel into w_dev (device, FP64 [nrhs][Nz][Ny][Nx], may be NULL) and
 * W_m = 1/4 int mu0 |h|^2 dV over the voxels with chi != 0 into W_host[nrhs]
 * (J; may be NULL).  Requires vie_set_contrast. */
int vie_magnetic_energy(vie_ctx* ctx, int nrhs, const void* h, double* w_dev, double* W_host);

/* Copy the curl operator's 30 unique block tensors Q_k^{ll'}(d), d >= 0,
 * [30][Nz][Ny][Nx] complex128, entry 10 k + ll (k = x, y, z; ll over the
 * pairs l <= l' as for vie_set_toeplitz), to host memory; K^{pl,ql'} =
 * eps_pkq Q_k^{ll'}, and Q_k^{l'l} = -Q_k^{ll'} when exactly one of l, l' is
 * the pulse.  Builds the curl operator if needed. */
int vie_get_curl_toeplitz(vie_ctx* ctx, double* T_host);

/* -- utilities -------------------------------------------------------------- */

/* Device copy of n complex128 values (src, dst device pointers, not
 * overlapping) on the context stream: a plain streaming kernel of known
 * traffic (16 n bytes read, 16 n written), used to calibrate memory
 * counters. */
int vie_copy(vie_ctx* ctx, const void* src, void* dst, long long n);

/* -- autotuning ------------------------------------------------------------ */

/* Time the candidate launch shapes of the operator product (x-pass variant,
 * workgroups per octant row, pencils per workgroup of the z and y passes)
 * for this grid, precision and number of right-hand sides, and keep the
 * fastest for later calls with the same (precision, nrhs).  choice (may be
 * NULL) receives {variant, workgroups per row, z tile, y tile}; best_ms (may
 * be NULL) the time of one product with them.  Allocates two temporary
 * vectors; synchronises the stream.  Every shape computes the same sums; the
 * x-pass variants add the 144 block terms in different orders, so results
 * agree to rounding. */
int vie_autotune(vie_ctx* ctx, int precision, int nrhs, int* choice, double* best_ms);

/* Install launch shapes for (precision, nrhs) without timing, e.g. ones an
 * earlier vie_autotune returned: choice = {variant (0 staged operator row,
 * 1 one pencil group per workgroup, 2 the sibling pencil groups of a row per
 * workgroup, complex64 only, 3 as 1 with the operator row prefetched into
 * LDS, fft length <= 128 along x, 4 as 1 with two threads per frequency,
 * 5 the pencils of two right-hand sides per workgroup),
 * workgroups per row (1, 2, 4; variant 0),
 * z tile, y tile (pencils per workgroup of the strided passes: 8 or 16, or
 * 32 where the fft length has a compiled kernel)}.  VIE_EINVAL for shapes
 * this grid cannot run. */
int vie_set_tuning(vie_ctx* ctx, int precision, int nrhs, const int* choice);

/* -- profiling ------------------------------------------------------------ */

/* kernel classes timed by the built-in profiler */
enum {
    VIE_K_FFT_Z_FWD = 0,  /* zero-padded forward FFT along z                  */
    VIE_K_FFT_Y_FWD = 1,  /* zero-padded forward FFT along y                  */
    VIE_K_BLOCK = 2,      /* fused x FFT, 12 x 12 block product, inverse x FFT */
    VIE_K_FFT_Y_INV = 3,  /* inverse FFT along y with crop                    */
    VIE_K_FFT_Z_INV = 4,  /* inverse FFT along z, crop, contrast epilogue     */
    VIE_K_GS_DOT = 5,     /* Gram-Schmidt inner products (and their reduction) */
    VIE_K_GS_UPDATE = 6,  /* Gram-Schmidt update, norm and normalisation      */
    VIE_K_GS_PAIR = 7,    /* s-step Arnoldi: the later new vectors of a
                             block against its first ones (one pass)      */
    VIE_K_COUNT = 8
};

/* enable = k > 0 clears the records and starts timing launches of the
 * classes above with HIP events on the context stream, one launch in k of
 * each class (k = 1: every launch; a larger k keeps the event overhead out of
 * the timed work); enable = 0 stops. */
int vie_profile(vie_ctx* ctx, int enable);

/* Sum over the recorded launches of one class: device time (ms, from HIP
 * events), launch count, and algorithmic HBM bytes (the minimum traffic of
 * each launch: its inputs read once and its outputs written once).
 * Synchronises the stream. */
int vie_profile_read(vie_ctx* ctx, int kind, double* total_ms, int* launches, double* bytes);

/* -- serving: continuous batching of solve requests ------------------------ */

typedef struct vie_server vie_server;

/* One solve request: its own grid, tissue map (host [Nz][Ny][Nx], eps' and
 * sigma), nrhs Hertzian-dipole excitations (host [nrhs][3] positions in m and
 * current moments in A m), solver options (mode VIE_SOLVE_*, tol <= 0 for
 * 1e-6, restart <= 0 for 50) and the basis (12 PWL, 3 PWC; 0 means 12).
 * Inputs are copied at submission.  x_out (host [nrhs][basis][Nz][Ny][Nx]
 * complex128) and p_abs_out (host [nrhs]) are optional and must stay valid
 * until the request is done.  Admission counts the PWL footprint for either
 * basis (an upper bound for PWC). */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz, freq_hz;
    const double* eps_re;
    const double* sigma;
    int nrhs;
    const double* pos;
    const double* moment;
    int mode;
    double tol;
    int restart;
    double* x_out;
    double* p_abs_out;
    int basis;
} vie_request;

typedef struct {
    int done;            /* 1 when finished                                   */
    int status;          /* vie_status of the solve                           */
    double t_arrival;    /* seconds since the server started                  */
    double t_start;      /* admission time                                    */
    double t_end;        /* completion time                                   */
    size_t footprint;    /* device bytes reserved for it at admission         */
    int iterations;      /* most GMRES iterations over its right-hand sides   */
    double rel_residual; /* largest final relative residual                   */
    char message[192];   /* error text when status != VIE_OK                  */
    int operator_cached; /* 1 when the grid's operator came from the cache    */
} vie_request_info;

typedef struct {
    int completed, queued, running, peak_running;
    double p50_s, p99_s, mean_s; /* latency = completion - arrival            */
    double makespan_s;           /* first arrival to last completion          */
    size_t peak_bytes;           /* largest sum of admitted footprints         */
    long long operator_hits;     /* requests that reused a cached operator     */
    long long operator_misses;   /* requests that assembled their operator     */
    size_t operator_cache_bytes; /* device bytes held by the operator cache    */
    double oldest_queued_s;      /* age of the oldest request still queued     */
} vie_serving_stats;

/* Create a server on HIP device `device` that admits requests while the sum
 * of their footprints (vie_footprint_bytes plus the request vectors) stays
 * within hbm_budget bytes and at most max_slots run at once.  A pool of
 * max_slots worker threads runs the admitted requests, each on its own
 * context and stream.  Requests start in arrival order; one that fits may
 * start ahead of a head of the queue that does not (backfill), at most 8
 * times per head, after which the head waits for memory to drain and starts
 * next.  Operators of
 * recently used grids stay resident for later requests on the same grid
 * (extents, voxel size, frequency), in a cache of hbm_budget / 8 bytes by
 * default, held outside the budget (see vie_server_set_operator_cache). */
int vie_server_create(vie_server** out, int device, size_t hbm_budget, int max_slots);

/* Bytes the operator cache may hold (0 disables it); least recently used
 * operators are dropped to fit. */
int vie_server_set_operator_cache(vie_server* s, size_t bytes);

/* Queue a request (returns at once); *id identifies it.  VIE_ENOMEM when its
 * footprint exceeds the whole budget, VIE_EINVAL on bad arguments. */
int vie_server_submit(vie_server* s, const vie_request* r, long long* id);

/* State and timing of a request. */
int vie_server_poll(vie_server* s, long long id, vie_request_info* info);

/* Block until every submitted request has finished. */
int vie_server_wait(vie_server* s);

/* Latency percentiles (nearest rank) and counts over finished requests with
 * id >= first_id (to leave out a warm-up prefix). */
int vie_server_stats(vie_server* s, long long first_id, vie_serving_stats* out);

/* Wait for running requests, drop queued ones, free everything. */
void vie_server_destroy(vie_server* s);

/* -- memory model (Sec. V, "unknowns memory") ------------------------------ */

/* Bytes the paper counts as unknowns memory: 12 unknowns x 8 N_V padded
 * points x 16 B (complex128) = 1536 N_V (Tables III, V, VII, VIII). */
size_t vie_unknowns_bytes_paper(int nx, int ny, int nz);

/* The same count for ncomp unknowns per voxel: ncomp x 8 N_V x 16 B, with
 * ncomp = 12 (PWL) or 3 (PWC, 384 N_V B; the PWC rows of the same tables).
 * Returns 0 for other ncomp or non-positive sizes. */
size_t vie_unknowns_bytes_basis(int nx, int ny, int nz, int ncomp);

/* Device bytes this library needs to solve nrhs right-hand sides on the
 * grid with fft size 2N: resident operator, contrast, padded FFT buffers and
 * the Krylov basis of GMRES(restart) for the given mode, PWL basis (a PWC
 * solve needs a quarter of the vector, FFT and basis bytes). */
int vie_footprint_bytes(int nx, int ny, int nz, int nrhs, int mode, int restart, size_t* out);

#ifdef __cplusplus
}
#endif
#endif
