// Materials (eq. 2, 7, 17), tested incident fields (eq. 27, 30-31) and
// post-processing (Sec. IV-C, eq. 44, Sec. V-C).  Vectors hold nc unknowns per
// voxel: nc = 12 for the PWL basis (a = 4 p + l - 1), nc = 3 for the PWC basis
// (the constant functions alone, unknown p), whose coefficients are the l = 1
// ones of the PWL basis.
#include "kernels.hpp"

namespace vie {

__global__ void k_materials(const double* __restrict__ eps_re, const double* __restrict__ sigma, double weps0,
                            Materials m, long long V, int* bad) {
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= V) return;
    const double e = eps_re[v], s = sigma[v];
    if (!isfinite(e) || !isfinite(s)) { atomicOr(bad, 1); return; }
    if (!(e > 0.0) || s < 0.0) { atomicOr(bad, 2); return; }
    const double2 er = make_double2(e, -s / weps0);          // eps' - i sigma/(w eps0)
    const double2 ch = make_double2(er.x - 1.0, er.y);        // chi = eps_r - 1
    const double den = er.x * er.x + er.y * er.y;             // tau = chi / eps_r
    const double2 ta = make_double2((ch.x * er.x + ch.y * er.y) / den, (ch.y * er.x - ch.x * er.y) / den);
    m.eps_r[v] = er;
    m.chi[v] = ch;
    m.tau[v] = ta;
    m.tau64[v] = make_float2((float)ta.x, (float)ta.y);
    m.epsr64[v] = make_float2((float)er.x, (float)er.y);
    m.chi64[v] = make_float2((float)ch.x, (float)ch.y);
}

void launch_materials(const double* eps_re, const double* sigma, double weps0, Materials m, long long V, int* bad,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_materials, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, eps_re, sigma, weps0, m, V,
                       bad);
    VIE_HIP(hipGetLastError());
}

// plane wave amp pol_hat exp(-i k0 sgn r_dir), tested in closed form: the
// pulse gives dV exp(-i k0 sgn c) sin(k0 a)/(k0 a) (a = D_dir / 2); the linear
// function along dir gives -2 i sgn (sin(k0 a) - k0 a cos(k0 a)) / k0^2 times
// dV / D_dir^2 exp(-i k0 sgn c); the other two linear functions integrate
// to zero.
__global__ void k_planewave(double2* __restrict__ et, int Nx, int Ny, int Nz, double Dx, double Dy, double Dz,
                            double k0, int pol, int dir, double sgn, double amp, int nc) {
    const long long V = (long long)Nx * Ny * Nz;
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int ix = int(v % Nx), iy = int((v / Nx) % Ny), iz = int(v / ((long long)Nx * Ny));
    const double D[3] = {Dx, Dy, Dz};
    const int n[3] = {ix, iy, iz}, N[3] = {Nx, Ny, Nz};
    const double c = (n[dir] - 0.5 * (N[dir] - 1)) * D[dir];
    const double a = 0.5 * D[dir];
    const double dv = Dx * Dy * Dz;
    double s, co;
    sincos(k0 * sgn * c, &s, &co);
    const double2 ph = make_double2(co * amp, -s * amp);
    const double ka = k0 * a;
    double l1, l4;
    if (ka == 0.0) { l1 = dv; l4 = 0.0; }
    else {
        l1 = dv * sin(ka) / ka;
        l4 = -2.0 * sgn * (sin(ka) - ka * cos(ka)) / (k0 * k0) * dv / (D[dir] * D[dir]);
    }
    for (int a_ = 0; a_ < nc; ++a_) et[a_ * V + v] = make_double2(0, 0);
    if (nc == 3) {
        et[pol * V + v] = make_double2(l1 * ph.x, l1 * ph.y);
        return;
    }
    et[(4 * pol + 0) * V + v] = make_double2(l1 * ph.x, l1 * ph.y);
    // times -i: (l4 i) * ph with l4 already carrying -2 sgn ...; value = -2i sgn(...) ph
    et[(4 * pol + dir + 1) * V + v] = make_double2(-l4 * ph.y, l4 * ph.x);
}

void launch_planewave(double2* et, int Nx, int Ny, int Nz, const double D[3], double k0, int pol, int dir,
                      double sgn, double amp, int nc, hipStream_t s) {
    const long long V = (long long)Nx * Ny * Nz;
    hipLaunchKernelGGL(k_planewave, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, et, Nx, Ny, Nz, D[0], D[1],
                       D[2], k0, pol, dir, sgn, amp, nc);
    VIE_HIP(hipGetLastError());
}

// Hertzian dipole of current moment m at r0:
// E = (1/c_e) exp(-i k R)/(4 pi R^3) [(k^2 R^2 - i k R - 1) m + (3 + 3 i k R - k^2 R^2)(R_hat . m) R_hat]
// and (magnetic = 1) H = curl (g m) = (1 + i k R) exp(-i k R)/(4 pi R^2) (m x R_hat), the
// h = K j of eq. 'tot_fields' b for a point current.  The electric field is
// tested on voxels with chi != 0 (chi may be null: every voxel), the magnetic
// one on every voxel.
__global__ void k_dipoles(double2* __restrict__ et, const double* __restrict__ pos, const double* __restrict__ mom,
                          int nq, const double* __restrict__ glx, const double* __restrict__ glw,
                          const double2* __restrict__ chi, int Nx, int Ny, int Nz, double Dx, double Dy, double Dz,
                          double k0, double weps0, int nc, int magnetic) {
    const long long V = (long long)Nx * Ny * Nz;
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (v >= V) return;
    double2* out = et + (long long)r * nc * V;
    const double2 ch = chi ? chi[v] : make_double2(1.0, 0.0);
    if (!magnetic && ch.x == 0.0 && ch.y == 0.0) {
        for (int a = 0; a < nc; ++a) out[a * V + v] = make_double2(0, 0);
        return;
    }
    const int ix = int(v % Nx), iy = int((v / Nx) % Ny), iz = int(v / ((long long)Nx * Ny));
    const double cx = (ix - 0.5 * (Nx - 1)) * Dx, cy = (iy - 0.5 * (Ny - 1)) * Dy, cz = (iz - 0.5 * (Nz - 1)) * Dz;
    const double px = pos[3 * r], py = pos[3 * r + 1], pz = pos[3 * r + 2];
    const double mx = mom[3 * r], my = mom[3 * r + 1], mz = mom[3 * r + 2];
    double acc[12][2];
    for (int a = 0; a < 12; ++a) acc[a][0] = acc[a][1] = 0.0;
    const double dv = Dx * Dy * Dz;
    for (int i = 0; i < nq; ++i) {
        const double tx = glx[i] - 0.5;   // local coordinate / Dx in [-1/2, 1/2]
        for (int j = 0; j < nq; ++j) {
            const double ty = glx[j] - 0.5;
            for (int k = 0; k < nq; ++k) {
                const double tz = glx[k] - 0.5;
                const double wq = glw[i] * glw[j] * glw[k] * dv;
                const double Rx = cx + tx * Dx - px, Ry = cy + ty * Dy - py, Rz = cz + tz * Dz - pz;
                const double R = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
                const double hx = Rx / R, hy = Ry / R, hz = Rz / R;
                const double kr = k0 * R;
                double s, c;
                sincos(kr, &s, &c);
                double2 pre;
                double E[3][2];
                if (magnetic) {
                    // (1 + i kR)(c - i s) / (4 pi R^2), times m x R_hat (real)
                    const double amp = 1.0 / (4.0 * M_PI * R * R);
                    pre = make_double2((c + kr * s) * amp, (kr * c - s) * amp);
                    const double cr[3] = {my * hz - mz * hy, mz * hx - mx * hz, mx * hy - my * hx};
                    for (int p = 0; p < 3; ++p) { E[p][0] = cr[p]; E[p][1] = 0.0; }
                } else {
                    // pre = exp(-i k R)/(4 pi R^3) / (i w eps0) = exp(-i k R) * (-i) / (4 pi R^3 w eps0)
                    const double amp = 1.0 / (4.0 * M_PI * R * R * R * weps0);
                    pre = make_double2(-s * amp, -c * amp);                  // (c - i s)(-i) amp
                    const double2 A = make_double2(kr * kr - 1.0, -kr);      // k^2R^2 - i kR - 1
                    const double hm = hx * mx + hy * my + hz * mz;
                    const double2 B = make_double2((3.0 - kr * kr) * hm, 3.0 * kr * hm);
                    E[0][0] = A.x * mx + B.x * hx; E[0][1] = A.y * mx + B.y * hx;
                    E[1][0] = A.x * my + B.x * hy; E[1][1] = A.y * my + B.y * hy;
                    E[2][0] = A.x * mz + B.x * hz; E[2][1] = A.y * mz + B.y * hz;
                }
                const double nl[4] = {1.0, tx, ty, tz};
                for (int p = 0; p < 3; ++p) {
                    const double er = pre.x * E[p][0] - pre.y * E[p][1];
                    const double ei = pre.x * E[p][1] + pre.y * E[p][0];
                    for (int l = 0; l < 4; ++l) {
                        acc[4 * p + l][0] += wq * nl[l] * er;
                        acc[4 * p + l][1] += wq * nl[l] * ei;
                    }
                }
            }
        }
    }
    if (nc == 3)
        for (int p = 0; p < 3; ++p) out[p * V + v] = make_double2(acc[4 * p][0], acc[4 * p][1]);
    else
        for (int a = 0; a < 12; ++a) out[a * V + v] = make_double2(acc[a][0], acc[a][1]);
}

void launch_dipoles(double2* et, int nrhs, const double* pos, const double* mom, int nq, const double* glx,
                    const double* glw, const double2* chi, int Nx, int Ny, int Nz, const double D[3], double k0,
                    double weps0, int nc, hipStream_t s, int magnetic) {
    const long long V = (long long)Nx * Ny * Nz;
    hipLaunchKernelGGL(k_dipoles, dim3((unsigned)((V + 127) / 128), nrhs), dim3(128), 0, s, et, pos, mom, nq, glx,
                       glw, chi, Nx, Ny, Nz, D[0], D[1], D[2], k0, weps0, nc, magnetic);
    VIE_HIP(hipGetLastError());
}

// b1+ = mu0 (h_x + i h_y) per scalar basis (Sec. V-D): b[r][l][v] from the
// PWL coefficients h^{x,l}, h^{y,l}
__global__ void k_b1plus(double2* __restrict__ b, const double2* __restrict__ h, double mu0, long long V, int nrhs) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= 4 * V * nrhs) return;
    const long long r = i / (4 * V), rem = i - r * 4 * V;      // rem = l V + v
    const double2 hx = h[r * 12 * V + rem], hy = h[r * 12 * V + 4 * V + rem];
    b[i] = make_double2(mu0 * (hx.x - hy.y), mu0 * (hx.y + hy.x));
}

void launch_b1plus(double2* b, const double2* h, double mu0, long long V, int nrhs, hipStream_t s) {
    const long long n = 4 * V * nrhs;
    hipLaunchKernelGGL(k_b1plus, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b, h, mu0, V, nrhs);
    VIE_HIP(hipGetLastError());
}

// magnetic energy density w_m = 1/4 mu0 |h|^2 averaged over each voxel (Sec.
// V-D; Gram weights 1 and 1/12), into w (may be null), and per-block partial
// sums of w_m dV over the voxels with chi != 0 (W_m inside the body)
__global__ void __launch_bounds__(256) k_magnetic_energy(double* __restrict__ w, double* __restrict__ partial,
                                                         const double2* __restrict__ h,
                                                         const double2* __restrict__ chi, double mu0, double dv,
                                                         long long V) {
    __shared__ double red[256];
    const int r = blockIdx.y;
    const double2* hr = h + (long long)r * 12 * V;
    double acc = 0.0;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V;
         v += (long long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int a = 0; a < 12; ++a) {
            const double2 z = hr[a * V + v];
            s += ((a & 3) == 0 ? 1.0 : 1.0 / 12.0) * (z.x * z.x + z.y * z.y);
        }
        const double wm = 0.25 * mu0 * s;
        if (w) w[(long long)r * V + v] = wm;
        const double2 ch = chi[v];
        if (ch.x != 0.0 || ch.y != 0.0) acc += wm * dv;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[r * gridDim.x + blockIdx.x] = red[0];
}

void launch_magnetic_energy(double* w, double* partial, const double2* h, const double2* chi, double mu0, double dv,
                            long long V, int nrhs, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_magnetic_energy, dim3(nblocks, nrhs), dim3(256), 0, s, w, partial, h, chi, mu0, dv, V);
    VIE_HIP(hipGetLastError());
}

// P^-1 b = c_e tau G^-1 e_t (eq. 17, 31)
__global__ void k_rhs_prec(double2* __restrict__ rhs, const double2* __restrict__ et, const double2* __restrict__ tau,
                           double g0, double g1, double2 ce, long long V, long long n, int nc) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long v = i % V;
    const int l = nc == 12 ? int((i / V) % 12) & 3 : 0;
    const double gi = l == 0 ? g0 : g1;
    const double2 t = cmul(cmul(ce, tau[v]), et[i]);
    rhs[i] = make_double2(t.x * gi, t.y * gi);
}

void launch_rhs_prec(double2* rhs, const double2* et, const double2* tau, const double ginv[4], double2 ce,
                     long long V, int nrhs, int nc, hipStream_t s) {
    const long long n = nc * V * nrhs;
    hipLaunchKernelGGL(k_rhs_prec, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rhs, et, tau, ginv[0], ginv[1],
                       ce, V, n, nc);
    VIE_HIP(hipGetLastError());
}

// e = x / (c_e chi) where chi != 0
__global__ void k_fields(double2* __restrict__ e, const double2* __restrict__ x, const double2* __restrict__ chi,
                         double2 ce, long long V, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 ch = chi[i % V];
    if (ch.x == 0.0 && ch.y == 0.0) { e[i] = make_double2(0, 0); return; }
    const double2 q = cmul(ce, ch);
    const double den = q.x * q.x + q.y * q.y;
    const double2 xv = x[i];
    e[i] = make_double2((xv.x * q.x + xv.y * q.y) / den, (xv.y * q.x - xv.x * q.y) / den);
}

void launch_fields(double2* e, const double2* x, const double2* chi, double2 ce, long long V, int nrhs, int nc,
                   hipStream_t s) {
    const long long n = nc * V * nrhs;
    hipLaunchKernelGGL(k_fields, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, e, x, chi, ce, V, n);
    VIE_HIP(hipGetLastError());
}

// e = (e_t + (w - G x) / c_e) / G with w = N x already in e (Sec. IV-C)
__global__ void k_total_field(double2* __restrict__ e, const double2* __restrict__ et,
                              const double2* __restrict__ x, double g0, double g1, double2 inv_ce, long long V,
                              long long n, int nc) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = nc == 12 ? int((i / V) % 12) & 3 : 0;
    const double g = l == 0 ? g0 : g1;
    const double2 w = e[i], xv = x[i], ev = et[i];
    const double2 d = make_double2(w.x - g * xv.x, w.y - g * xv.y);
    const double2 t = cmul(d, inv_ce);
    e[i] = make_double2((ev.x + t.x) / g, (ev.y + t.y) / g);
}

void launch_total_field(double2* e, const double2* et, const double2* x, const double gram[4], double2 ce,
                        long long V, int nrhs, int nc, hipStream_t s) {
    const long long n = nc * V * nrhs;
    const double den = ce.x * ce.x + ce.y * ce.y;
    const double2 inv_ce = make_double2(ce.x / den, -ce.y / den);
    hipLaunchKernelGGL(k_total_field, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, e, et, x, gram[0], gram[1],
                       inv_ce, V, n, nc);
    VIE_HIP(hipGetLastError());
}

// partial sums of 1/2 Re{conj(x) G x / (c_e chi)} (eq. 44), one per block
__global__ void __launch_bounds__(256) k_power(double* __restrict__ partial, const double2* __restrict__ x,
                                               const double2* __restrict__ chi, double g0, double g1, double2 ce,
                                               long long V, int nc) {
    __shared__ double red[256];
    const int r = blockIdx.y;
    const double2* xr = x + (long long)r * nc * V;
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nc * V;
         i += (long long)gridDim.x * blockDim.x) {
        const long long v = i % V;
        const double2 ch = chi[v];
        if (ch.x == 0.0 && ch.y == 0.0) continue;
        const double2 q = cmul(ce, ch);
        const double req = q.x / (q.x * q.x + q.y * q.y);   // Re(1/q)
        const int l = nc == 12 ? int(i / V) & 3 : 0;
        const double2 xv = xr[i];
        acc += 0.5 * (l == 0 ? g0 : g1) * (xv.x * xv.x + xv.y * xv.y) * req;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[r * gridDim.x + blockIdx.x] = red[0];
}

void launch_power_partials(double* partial, const double2* x, const double2* chi, const double gram[4], double2 ce,
                           long long V, int nrhs, int nc, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_power, dim3(nblocks, nrhs), dim3(256), 0, s, partial, x, chi, gram[0], gram[1], ce, V, nc);
    VIE_HIP(hipGetLastError());
}

// 1/2 sigma (sum_p |e^{p1}|^2 + 1/12 sum_{p, l>1} |e^{pl}|^2); PWC: the first sum
__global__ void k_power_density(double* __restrict__ p, const double2* __restrict__ e,
                                const double* __restrict__ sigma, long long V, int nc) {
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (v >= V) return;
    const double2* er = e + (long long)r * nc * V;
    double acc = 0.0;
    for (int a = 0; a < nc; ++a) {
        const double2 z = er[a * V + v];
        acc += ((nc == 3 || (a & 3) == 0) ? 1.0 : 1.0 / 12.0) * (z.x * z.x + z.y * z.y);
    }
    p[(long long)r * V + v] = 0.5 * sigma[v] * acc;
}

void launch_power_density(double* p, const double2* e, const double* sigma, long long V, int nrhs, int nc,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_power_density, dim3((unsigned)((V + 255) / 256), nrhs), dim3(256), 0, s, p, e, sigma, V,
                       nc);
    VIE_HIP(hipGetLastError());
}

}  // namespace vie
