// Operator set-up (Sec. III-C, IV-A): assembly of the 60 unique
// Toeplitz-defining block tensors on the device, circulant embedding with the
// reflection signs of the PWL bases, forward FFT, octant extraction.
#include <algorithm>
#include <cmath>
#include <vector>

#include "assembly.hpp"
#include "kernels.hpp"

namespace vie {

// ---------------------------------------------------------------------------
// host: axis kernels in closed form
// ---------------------------------------------------------------------------
// measure kinds: 0 '1', 1 't/D', 2 'D(1)', 3 'D(t/D)'
static AxisKernel axis_kernel(int kt, int kb, double D) {
    AxisKernel k{};
    auto set = [&](double* c, double a0, double a1, double a2, double a3) { c[0] = a0; c[1] = a1; c[2] = a2; c[3] = a3; };
    const double D2 = D * D;
    switch (kt * 4 + kb) {
        case 0:  // (1,1): D - |w|
            set(k.left, D, 1, 0, 0); set(k.right, D, -1, 0, 0); break;
        case 4:  // (t,1): w (D - |w|) / (2D)
            set(k.left, 0, 0.5, 0.5 / D, 0); set(k.right, 0, 0.5, -0.5 / D, 0); break;
        case 1:  // (1,t): -w (D - |w|) / (2D)
            set(k.left, 0, -0.5, -0.5 / D, 0); set(k.right, 0, -0.5, 0.5 / D, 0); break;
        case 5:  // (t,t): (D^3 - 3 D^2 |w| + 2 |w|^3) / (12 D^2)
            set(k.left, D / 12, 0.25, 0, -1.0 / (6 * D2)); set(k.right, D / 12, -0.25, 0, 1.0 / (6 * D2)); break;
        case 8:  // (D1,1): +1 left, -1 right
            set(k.left, 1, 0, 0, 0); set(k.right, -1, 0, 0, 0); break;
        case 9:  // (D1,t)
            set(k.left, -0.5, -1 / D, 0, 0); set(k.right, -0.5, 1 / D, 0, 0); break;
        case 2:  // (1,D1)
            set(k.left, -1, 0, 0, 0); set(k.right, 1, 0, 0, 0); break;
        case 6:  // (t,D1)
            set(k.left, -0.5, -1 / D, 0, 0); set(k.right, -0.5, 1 / D, 0, 0); break;
        case 10:  // (D1,D1): 2 delta_0 - delta_{-D} - delta_{D}
            k.pts[0] = -1; k.pts[1] = 2; k.pts[2] = -1; break;
        case 12:  // (Dt,1): 1/2 - |w|/D
            set(k.left, 0.5, 1 / D, 0, 0); set(k.right, 0.5, -1 / D, 0, 0); break;
        case 3:  // (1,Dt)
            set(k.left, 0.5, 1 / D, 0, 0); set(k.right, 0.5, -1 / D, 0, 0); break;
        case 13:  // (Dt,t)
            set(k.left, 0.25, 0, -0.5 / D2, 0); set(k.right, -0.25, 0, 0.5 / D2, 0); break;
        case 7:  // (t,Dt)
            set(k.left, -0.25, 0, 0.5 / D2, 0); set(k.right, 0.25, 0, -0.5 / D2, 0); break;
        case 11:  // (D1,Dt)
            set(k.left, 1 / D, 0, 0, 0); set(k.right, -1 / D, 0, 0, 0); k.pts[0] = -0.5; k.pts[2] = 0.5; break;
        case 14:  // (Dt,D1)
            set(k.left, -1 / D, 0, 0, 0); set(k.right, 1 / D, 0, 0, 0); k.pts[0] = 0.5; k.pts[2] = -0.5; break;
        case 15:  // (Dt,Dt): -|w|/D^2, 1/4 delta_{-D} + 1/2 delta_0 + 1/4 delta_D
            set(k.left, 0, 1 / D2, 0, 0); set(k.right, 0, -1 / D2, 0, 0);
            k.pts[0] = 0.25; k.pts[1] = 0.5; k.pts[2] = 0.25; break;
    }
    return k;
}

static void gauss_legendre01(int n, double* x, double* w) {
    // roots of P_n by Newton from the usual cosine guesses, weights
    // 2 / ((1 - z^2) P_n'(z)^2); mapped from [-1, 1] to [0, 1]
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            const double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-15) {
                // refresh the derivative at the converged root
                p1 = 1.0; p2 = 0.0;
                for (int j = 1; j <= n; ++j) {
                    const double p3 = p2;
                    p2 = p1;
                    p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
                }
                pp = n * (z * p1 - p2) / (z * z - 1.0);
                break;
            }
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * pp * pp);
    }
}

AssemblyTables build_assembly_tables(const double D[3], double k0) {
    AssemblyTables T{};
    for (int ax = 0; ax < 3; ++ax)
        for (int kt = 0; kt < 4; ++kt)
            for (int kb = 0; kb < 4; ++kb) T.ker[ax * 16 + kt * 4 + kb] = axis_kernel(kt, kb, D[ax]);
    const double dv = D[0] * D[1] * D[2];
    T.gram[0] = dv;
    T.gram[1] = T.gram[2] = T.gram[3] = dv / 12;
    for (int pq = 0; pq < 6; ++pq) {
        static const int P[6] = {0, 0, 0, 1, 1, 2}, Q[6] = {0, 1, 2, 1, 2, 2};
        static const int L[10] = {1, 1, 1, 1, 2, 2, 2, 3, 3, 4}, LP[10] = {1, 2, 3, 4, 2, 3, 4, 3, 4, 4};
        for (int ll = 0; ll < 10; ++ll) {
            const int p = P[pq], q = Q[pq], l = L[ll], lp = LP[ll];
            EntryTerms& e = T.ent[pq * 10 + ll];
            e.nterm = 0;
            int kt[3], kb[3];
            for (int ax = 0; ax < 3; ++ax) {
                kt[ax] = (l == ax + 2) ? 1 : 0;
                kb[ax] = (lp == ax + 2) ? 1 : 0;
            }
            if (p == q && k0 != 0.0) {
                e.coef[e.nterm] = k0 * k0;
                for (int ax = 0; ax < 3; ++ax) e.ker[e.nterm][ax] = ax * 16 + kt[ax] * 4 + kb[ax];
                e.nterm++;
            }
            int ct[3] = {kt[0], kt[1], kt[2]}, cb[3] = {kb[0], kb[1], kb[2]};
            ct[p] += 2;
            cb[q] += 2;
            e.coef[e.nterm] = -1.0;
            for (int ax = 0; ax < 3; ++ax) e.ker[e.nterm][ax] = ax * 16 + ct[ax] * 4 + cb[ax];
            e.nterm++;
            e.gram_l = (p == q && l == lp) ? l - 1 : -1;
        }
    }
    for (int n = 1; n <= kMaxGauss; ++n) gauss_legendre01(n, T.gl_x[n], T.gl_w[n]);
    T.D[0] = D[0]; T.D[1] = D[1]; T.D[2] = D[2];
    T.k0 = k0;
    T.order_near = 14;
    T.order_duffy = 12;
    T.nent = 60;
    return T;
}

// the 30 unique tensors of the curl operator: entry 10 k + ll is
// Q_k^{ll'}(d) = <N^l, S D_k N^{l'}> (l <= l'), one term, no Gram part
AssemblyTables build_curl_tables(const double D[3], double k0) {
    AssemblyTables T = build_assembly_tables(D, k0);
    static const int L[10] = {1, 1, 1, 1, 2, 2, 2, 3, 3, 4}, LP[10] = {1, 2, 3, 4, 2, 3, 4, 3, 4, 4};
    for (int k = 0; k < 3; ++k)
        for (int ll = 0; ll < 10; ++ll) {
            EntryTerms& e = T.ent[10 * k + ll];
            e.nterm = 1;
            e.coef[0] = 1.0;
            for (int ax = 0; ax < 3; ++ax) {
                const int kt = (L[ll] == ax + 2) ? 1 : 0;
                const int kb = ((LP[ll] == ax + 2) ? 1 : 0) + (ax == k ? 2 : 0);
                e.ker[0][ax] = ax * 16 + kt * 4 + kb;
            }
            e.gram_l = -1;
        }
    T.nent = 30;
    return T;
}

// ---------------------------------------------------------------------------
// device: integration
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ double horner(const double* c, double w) { return ((c[3] * w + c[2]) * w + c[1]) * w + c[0]; }

// slot: 0 = density on [-D,0], 1 = density on [0,D], 2/3/4 = point at -D/0/+D
__host__ __device__ __forceinline__ bool slot_used(const AxisKernel& k, int slot) {
    if (slot == 0) return k.left[0] != 0 || k.left[1] != 0 || k.left[2] != 0 || k.left[3] != 0;
    if (slot == 1) return k.right[0] != 0 || k.right[1] != 0 || k.right[2] != 0 || k.right[3] != 0;
    return k.pts[slot - 2] != 0;
}

__host__ __device__ __forceinline__ double slot_value(const AxisKernel& k, int slot, double w) {
    if (slot == 0) return horner(k.left, w);
    if (slot == 1) return horner(k.right, w);
    return k.pts[slot - 2];
}

__host__ __device__ __forceinline__ double2 green(double r, double k0) {
    double s, c;
    sincos(k0 * r, &s, &c);
    const double a = 1.0 / (4.0 * M_PI * r);
    return make_double2(c * a, -s * a);
}

__host__ __device__ double2 integrate_geometry(const AssemblyTables& T, const AxisKernel* kx[3], const int slot[3],
                                      const int d[3], int order_far) {
    const double* D = T.D;
    // singular corner: w* = -d Delta, touching when each axis reaches it
    bool touch = true;
    for (int i = 0; i < 3; ++i) {
        const int s = slot[i];
        bool ti;
        if (s == 0) ti = (d[i] == 0 || d[i] == 1);
        else if (s == 1) ti = (d[i] == 0);
        else if (s == 2) ti = (d[i] == 1);
        else if (s == 3) ti = (d[i] == 0);
        else ti = (d[i] == -1);
        touch = touch && ti;
    }
    int dens[3], nd = 0, pt_axis = -1;
    for (int i = 0; i < 3; ++i) {
        if (slot[i] <= 1) dens[nd++] = i;
        else pt_axis = i;
    }
    double off[3] = {d[0] * D[0], d[1] * D[1], d[2] * D[2]};
    double base[3], wfix = 1.0;
    if (pt_axis >= 0) {
        base[pt_axis] = (slot[pt_axis] - 3) * D[pt_axis];
        wfix = kx[pt_axis]->pts[slot[pt_axis] - 2];
    }
    double2 acc = make_double2(0, 0);
    if (!touch) {
        const int n = order_far;
        const double* gx = T.gl_x[n];
        const double* gw = T.gl_w[n];
        double lo[3];
        for (int i = 0; i < 3; ++i) lo[i] = (slot[i] == 0) ? -D[i] : 0.0;
        if (nd == 3) {
            for (int a = 0; a < n; ++a) {
                const double wx = lo[0] + D[0] * gx[a];
                const double fx = slot_value(*kx[0], slot[0], wx) * gw[a] * D[0];
                const double rx = off[0] + wx;
                for (int b = 0; b < n; ++b) {
                    const double wy = lo[1] + D[1] * gx[b];
                    const double fy = fx * slot_value(*kx[1], slot[1], wy) * gw[b] * D[1];
                    const double ry = off[1] + wy;
                    for (int c = 0; c < n; ++c) {
                        const double wz = lo[2] + D[2] * gx[c];
                        const double f = fy * slot_value(*kx[2], slot[2], wz) * gw[c] * D[2];
                        const double rz = off[2] + wz;
                        const double2 g = green(sqrt(rx * rx + ry * ry + rz * rz), T.k0);
                        acc.x += f * g.x;
                        acc.y += f * g.y;
                    }
                }
            }
        } else {
            const int i0 = dens[0], i1 = dens[1];
            const double rp = off[pt_axis] + base[pt_axis];
            for (int a = 0; a < n; ++a) {
                const double w0 = lo[i0] + D[i0] * gx[a];
                const double f0 = slot_value(*kx[i0], slot[i0], w0) * gw[a] * D[i0] * wfix;
                const double r0 = off[i0] + w0;
                for (int b = 0; b < n; ++b) {
                    const double w1 = lo[i1] + D[i1] * gx[b];
                    const double f = f0 * slot_value(*kx[i1], slot[i1], w1) * gw[b] * D[i1];
                    const double r1 = off[i1] + w1;
                    const double2 g = green(sqrt(r0 * r0 + r1 * r1 + rp * rp), T.k0);
                    acc.x += f * g.x;
                    acc.y += f * g.y;
                }
            }
        }
        return acc;
    }
    // Duffy: the singular point is a corner of the box.  Map the box to the
    // unit cube (square) with that corner at the origin and split it into
    // pyramids (triangles) with apex there: on the piece whose far face is
    // xi_k = 1, xi_k = s and xi_j = s t_j, Jacobian s^(dim-1).
    const int n = T.order_duffy;
    const double* gx = T.gl_x[n];
    const double* gw = T.gl_w[n];
    double corner[3], ext[3];
    for (int i = 0; i < 3; ++i) {
        corner[i] = -off[i];                     // w* = -d Delta
        if (slot[i] <= 1) {
            const double lo = (slot[i] == 0) ? -D[i] : 0.0;
            ext[i] = (corner[i] == lo) ? D[i] : -D[i];
        }
    }
    if (nd == 3) {
        const double jac0 = D[0] * D[1] * D[2];
        for (int k = 0; k < 3; ++k) {
            const int j1 = (k + 1) % 3, j2 = (k + 2) % 3;
            for (int a = 0; a < n; ++a) {
                const double s = gx[a];
                for (int b = 0; b < n; ++b) {
                    const double t1 = gx[b];
                    for (int c = 0; c < n; ++c) {
                        const double t2 = gx[c];
                        double xi[3];
                        xi[k] = s;
                        xi[j1] = s * t1;
                        xi[j2] = s * t2;
                        double w[3], rr = 0, f = gw[a] * gw[b] * gw[c] * s * s * jac0;
                        for (int i = 0; i < 3; ++i) {
                            w[i] = corner[i] + ext[i] * xi[i];
                            const double ri = off[i] + w[i];
                            rr += ri * ri;
                            f *= slot_value(*kx[i], slot[i], w[i]);
                        }
                        const double2 g = green(sqrt(rr), T.k0);
                        acc.x += f * g.x;
                        acc.y += f * g.y;
                    }
                }
            }
        }
    } else {
        const int i0 = dens[0], i1 = dens[1];
        const double jac0 = D[i0] * D[i1] * wfix;
        for (int k = 0; k < 2; ++k) {
            for (int a = 0; a < n; ++a) {
                const double s = gx[a];
                for (int b = 0; b < n; ++b) {
                    const double t = gx[b];
                    const double xi0 = (k == 0) ? s : s * t;
                    const double xi1 = (k == 0) ? s * t : s;
                    const double w0 = corner[i0] + ext[i0] * xi0;
                    const double w1 = corner[i1] + ext[i1] * xi1;
                    const double r0 = off[i0] + w0, r1 = off[i1] + w1;
                    const double f = gw[a] * gw[b] * s * jac0 * slot_value(*kx[i0], slot[i0], w0) *
                                     slot_value(*kx[i1], slot[i1], w1);
                    const double2 g = green(sqrt(r0 * r0 + r1 * r1), T.k0);
                    acc.x += f * g.x;
                    acc.y += f * g.y;
                }
            }
        }
    }
    return acc;
}

__host__ __device__ __forceinline__ int far_order(int dinf, int near) {
    if (dinf <= 2) return near;
    if (dinf <= 4) return 9;
    if (dinf <= 8) return 7;
    if (dinf <= 16) return 5;
    return 4;
}

// Gauss order bands of far_order for offsets beyond the singular corner
static const int kBandLo[kFarBands] = {2, 3, 5, 9, 17};
static const int kBandHi[kFarBands] = {2, 4, 8, 16, 1 << 30};

FarTables build_far_tables(const AssemblyTables& T) {
    FarTables F{};
    for (int b = 0; b < kFarBands; ++b) {
        FarBand& B = F.band[b];
        B.dlo = kBandLo[b];
        B.dhi = kBandHi[b];
        B.n = far_order(B.dlo, T.order_near);
        B.P = 2 * B.n + 3;
        const double* gx = T.gl_x[B.n];
        const double* gw = T.gl_w[B.n];
        for (int i = 0; i < B.P; ++i) B.ispt[i] = i >= 2 * B.n;
        for (int ax = 0; ax < 3; ++ax) {
            const double D = T.D[ax];
            for (int a = 0; a < B.n; ++a) {
                B.w[ax][a] = -D + D * gx[a];
                B.w[ax][B.n + a] = D * gx[a];
            }
            for (int m = 0; m < 3; ++m) B.w[ax][2 * B.n + m] = (m - 1) * D;
            for (int k = 0; k < 16; ++k) {
                const AxisKernel& K = T.ker[ax * 16 + k];
                for (int a = 0; a < B.n; ++a) {
                    B.W[ax][k][a] = horner(K.left, B.w[ax][a]) * gw[a] * D;
                    B.W[ax][k][B.n + a] = horner(K.right, B.w[ax][B.n + a]) * gw[a] * D;
                }
                for (int m = 0; m < 3; ++m) B.W[ax][k][2 * B.n + m] = K.pts[m];
            }
        }
    }
    F.nterm = 0;
    F.npair = 0;
    F.nent = T.nent;
    for (int e = 0; e < T.nent; ++e) {
        const EntryTerms& E = T.ent[e];
        F.ent_first[e] = F.nterm;
        F.ent_count[e] = E.nterm;
        for (int t = 0; t < E.nterm; ++t) {
            const int ky = E.ker[t][1] % 16, kz = E.ker[t][2] % 16;
            int p = 0;
            while (p < F.npair && !(F.pair_ky[p] == ky && F.pair_kz[p] == kz)) ++p;
            if (p == F.npair) {
                F.pair_ky[p] = ky;
                F.pair_kz[p] = kz;
                ++F.npair;
            }
            F.term_kx[F.nterm] = E.ker[t][0] % 16;
            F.term_pair[F.nterm] = p;
            F.term_coef[F.nterm] = E.coef[t];
            ++F.nterm;
        }
    }
    return F;
}

// The separable sum of one offset evaluated serially (host reference of the
// parallel kernel below; same grid, same contraction order).
void assemble_far_serial(const FarTables& F, const AssemblyTables& T, int b, const int d[3], double2* out60) {
    const FarBand& B = F.band[b];
    const int P = B.P;
    std::vector<double2> S(F.nterm, make_double2(0, 0)), t1(P * 16), t2(F.npair);
    std::vector<double2> slab(P * P);
    for (int i = 0; i < P; ++i) {
        const double rx = d[0] * T.D[0] + B.w[0][i];
        for (int j = 0; j < P; ++j)
            for (int k = 0; k < P; ++k) {
                const double ry = d[1] * T.D[1] + B.w[1][j], rz = d[2] * T.D[2] + B.w[2][k];
                slab[j * P + k] = (B.ispt[i] + B.ispt[j] + B.ispt[k] > 1)
                                      ? make_double2(0, 0)
                                      : green(sqrt(rx * rx + ry * ry + rz * rz), T.k0);
            }
        for (int j = 0; j < P; ++j)
            for (int kz = 0; kz < 16; ++kz) {
                double2 a = make_double2(0, 0);
                for (int k = 0; k < P; ++k) {
                    a.x += B.W[2][kz][k] * slab[j * P + k].x;
                    a.y += B.W[2][kz][k] * slab[j * P + k].y;
                }
                t1[j * 16 + kz] = a;
            }
        for (int p = 0; p < F.npair; ++p) {
            double2 a = make_double2(0, 0);
            for (int j = 0; j < P; ++j) {
                a.x += B.W[1][F.pair_ky[p]][j] * t1[j * 16 + F.pair_kz[p]].x;
                a.y += B.W[1][F.pair_ky[p]][j] * t1[j * 16 + F.pair_kz[p]].y;
            }
            t2[p] = a;
        }
        for (int t = 0; t < F.nterm; ++t) {
            const double wx = B.W[0][F.term_kx[t]][i];
            S[t].x += wx * t2[F.term_pair[t]].x;
            S[t].y += wx * t2[F.term_pair[t]].y;
        }
    }
    for (int e = 0; e < F.nent; ++e) {
        double2 a = make_double2(0, 0);
        for (int t = F.ent_first[e]; t < F.ent_first[e] + F.ent_count[e]; ++t) {
            a.x += F.term_coef[t] * S[t].x;
            a.y += F.term_coef[t] * S[t].y;
        }
        out60[e] = a;
    }
}

// One wavefront per offset (grid-stride over the offsets of the cube that
// holds the band, those below the band skipped).  Per x abscissa: the (y, z) slab of Green's values, the z
// contraction for all 16 kernel pairs, the y contraction for the (ky, kz)
// pairs in use, and the x accumulation of every (entry, term) sum.
template <int P>
__global__ void __launch_bounds__(64) k_assemble_far(double2* __restrict__ out, const FarTables* __restrict__ Fg,
                                                     int b, double Dx, double Dy, double Dz, double k0, int Nx,
                                                     int Ny, int Nz, int cx, int cy, int cz) {
    __shared__ double2 slab[P * P];
    __shared__ double2 t1[P * 16];
    __shared__ double2 t2[kFarTerms];
    const FarTables& F = *Fg;
    const FarBand& B = F.band[b];
    const int tid = threadIdx.x;
    const long long V = (long long)Nx * Ny * Nz;
    const int nterm = F.nterm, npair = F.npair;
    // offsets of the band lie in the cube [0, cx) x [0, cy) x [0, cz)
    const long long ncube = (long long)cx * cy * cz;
    for (long long q = blockIdx.x; q < ncube; q += gridDim.x) {
        const int d0 = int(q % cx), d1 = int((q / cx) % cy), d2 = int(q / ((long long)cx * cy));
        const long long v = ((long long)d2 * Ny + d1) * Nx + d0;
        const int dinf = max(d0, max(d1, d2));
        if (dinf < B.dlo || dinf > B.dhi) continue;   // uniform over the workgroup
        double2 s0 = make_double2(0, 0), s1 = make_double2(0, 0);   // terms tid, tid + 64
        for (int i = 0; i < P; ++i) {
            const double rx = d0 * Dx + B.w[0][i];
            const int pi = B.ispt[i];
            for (int idx = tid; idx < P * P; idx += 64) {
                const int j = idx / P, k = idx - j * P;
                double2 g = make_double2(0, 0);
                if (pi + B.ispt[j] + B.ispt[k] <= 1) {
                    const double ry = d1 * Dy + B.w[1][j], rz = d2 * Dz + B.w[2][k];
                    g = green(sqrt(rx * rx + ry * ry + rz * rz), k0);
                }
                slab[idx] = g;
            }
            __syncthreads();
            for (int idx = tid; idx < P * 16; idx += 64) {
                const int j = idx >> 4, kz = idx & 15;
                const double* wz = B.W[2][kz];
                double2 a = make_double2(0, 0);
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const double2 g = slab[j * P + k];
                    a.x += wz[k] * g.x;
                    a.y += wz[k] * g.y;
                }
                t1[idx] = a;
            }
            __syncthreads();
            for (int p = tid; p < npair; p += 64) {
                const double* wy = B.W[1][F.pair_ky[p]];
                const int kz = F.pair_kz[p];
                double2 a = make_double2(0, 0);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const double2 u = t1[j * 16 + kz];
                    a.x += wy[j] * u.x;
                    a.y += wy[j] * u.y;
                }
                t2[p] = a;
            }
            __syncthreads();
            if (tid < nterm) {
                const double wx = B.W[0][F.term_kx[tid]][i];
                const double2 u = t2[F.term_pair[tid]];
                s0.x += wx * u.x;
                s0.y += wx * u.y;
            }
            if (tid + 64 < nterm) {
                const double wx = B.W[0][F.term_kx[tid + 64]][i];
                const double2 u = t2[F.term_pair[tid + 64]];
                s1.x += wx * u.x;
                s1.y += wx * u.y;
            }
            __syncthreads();
        }
        // combine the terms of each entry (t2 reused for the term sums)
        if (tid < nterm) t2[tid] = s0;
        if (tid + 64 < nterm) t2[tid + 64] = s1;
        __syncthreads();
        if (tid < F.nent) {
            double2 a = make_double2(0, 0);
            for (int t = F.ent_first[tid]; t < F.ent_first[tid] + F.ent_count[tid]; ++t) {
                a.x += F.term_coef[t] * t2[t].x;
                a.y += F.term_coef[t] * t2[t].y;
            }
            out[(long long)tid * V + v] = a;
        }
        __syncthreads();
    }
}

// N^{e}(d) for one unique entry and one offset d >= 0
__host__ __device__ double2 assemble_entry(const AssemblyTables& T, int e, const int d[3]) {
    const int dinf = max(d[0], max(d[1], d[2]));
    const int nfar = far_order(dinf, T.order_near);
    const EntryTerms& E = T.ent[e];
    double2 acc = make_double2(0, 0);
    for (int t = 0; t < E.nterm; ++t) {
        const AxisKernel* kx[3] = {&T.ker[E.ker[t][0]], &T.ker[E.ker[t][1]], &T.ker[E.ker[t][2]]};
        double2 part = make_double2(0, 0);
        int slot[3];
        for (slot[0] = 0; slot[0] < 5; ++slot[0]) {
            if (!slot_used(*kx[0], slot[0])) continue;
            for (slot[1] = 0; slot[1] < 5; ++slot[1]) {
                if (!slot_used(*kx[1], slot[1])) continue;
                for (slot[2] = 0; slot[2] < 5; ++slot[2]) {
                    if (!slot_used(*kx[2], slot[2])) continue;
                    const int npt = (slot[0] >= 2) + (slot[1] >= 2) + (slot[2] >= 2);
                    if (npt > 1) continue;  // does not occur for these measures
                    const double2 g = integrate_geometry(T, kx, slot, d, nfar);
                    part.x += g.x;
                    part.y += g.y;
                }
            }
        }
        acc.x += E.coef[t] * part.x;
        acc.y += E.coef[t] * part.y;
    }
    if (d[0] == 0 && d[1] == 0 && d[2] == 0 && E.gram_l >= 0) acc.x += T.gram[E.gram_l];
    return acc;
}

// entry-by-entry assembly of the offsets at the singular corner,
// d in {0, 1}^3 (those may touch the singular point; Duffy rules)
__global__ void __launch_bounds__(64) k_assemble_near(double2* __restrict__ out, const AssemblyTables* __restrict__ Tg,
                                                      int Nx, int Ny, int Nz) {
    const long long V = (long long)Nx * Ny * Nz;
    const int e = blockIdx.x;
    const int c = threadIdx.x;
    if (c >= 8) return;
    const int d[3] = {c & 1, (c >> 1) & 1, c >> 2};
    if (d[0] >= Nx || d[1] >= Ny || d[2] >= Nz) return;
    out[(long long)e * V + ((long long)d[2] * Ny + d[1]) * Nx + d[0]] = assemble_entry(*Tg, e, d);
}

// circulant embedding of one unique entry on the M grid ([Mz][My][Mx]):
// index j_i -> offset d_i = j_i (j_i < N_i), j_i - M_i (j_i > M_i - N_i),
// otherwise zero; negative offsets by reflection, T(.., -d_i, ..) =
// sigma_i(a) sigma_i(b) T(.., d_i, ..)
__global__ void k_embed(double2* __restrict__ circ, const double2* __restrict__ Te, int Nx, int Ny, int Nz, int Mx,
                        int My, int Mz, int sgnx, int sgny, int sgnz) {
    const long long M = (long long)Mx * My * Mz;
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int jx = int(j % Mx), jy = int((j / Mx) % My), jz = int(j / ((long long)Mx * My));
    int dx, dy, dz;
    double s = 1.0;
    auto map = [](int jj, int N, int MM, int sg, int& d, double& s) {
        if (jj < N) { d = jj; return true; }
        if (jj > MM - N) { d = MM - jj; s *= sg; return true; }
        return false;
    };
    double2 val = make_double2(0, 0);
    if (map(jx, Nx, Mx, sgnx, dx, s) && map(jy, Ny, My, sgny, dy, s) && map(jz, Nz, Mz, sgnz, dz, s)) {
        double2 t = Te[((long long)dz * Ny + dy) * Nx + dx];
        val = make_double2(s * t.x, s * t.y);
    }
    circ[j] = val;
}

// keep the octant xi_i <= M_i / 2 of a transformed circulant, stored as
// U[oz][oy][e][ox] (the 60 entries of one (oz, oy) row together)
__global__ void k_octant(double2* __restrict__ U128, float2* __restrict__ U64, const double2* __restrict__ circ,
                         int e, int nent, int Mx, int My, int Ox, int Oy, int Oz) {
    const long long O = (long long)Ox * Oy * Oz;
    const long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (o >= O) return;
    const int ox = int(o % Ox);
    const long long row = o / Ox;   // oz * Oy + oy
    const int oy = int(row % Oy), oz = int(row / Oy);
    const double2 v = circ[((long long)oz * My + oy) * Mx + ox];
    const long long dst = (row * nent + e) * Ox + ox;
    U128[dst] = v;
    if (U64) U64[dst] = make_float2((float)v.x, (float)v.y);
}

// ---------------------------------------------------------------------------
// host entry points
// ---------------------------------------------------------------------------
void assemble_blocks(double2* out, const AssemblyTables& T, int Nx, int Ny, int Nz, hipStream_t s) {
    const FarTables F = build_far_tables(T);
    VIE_REQUIRE(F.nterm <= kFarTerms && F.npair <= kFarTerms, -1, "assembly: term table overflow");
    AssemblyTables* dT = nullptr;
    FarTables* dF = nullptr;
    VIE_HIP(hipMalloc(&dT, sizeof(AssemblyTables)));
    VIE_HIP(hipMalloc(&dF, sizeof(FarTables)));
    VIE_HIP(hipMemcpyAsync(dT, &T, sizeof(AssemblyTables), hipMemcpyHostToDevice, s));
    VIE_HIP(hipMemcpyAsync(dF, &F, sizeof(FarTables), hipMemcpyHostToDevice, s));
    const long long V = (long long)Nx * Ny * Nz;
    hipLaunchKernelGGL(k_assemble_near, dim3(T.nent), dim3(64), 0, s, out, dT, Nx, Ny, Nz);
    VIE_HIP(hipGetLastError());
    const int dmax = std::max(Nx, std::max(Ny, Nz)) - 1;
    for (int b = 0; b < kFarBands; ++b) {
        const FarBand& B = F.band[b];
        if (B.dlo > dmax) break;
        // offsets in the band: the cube of edge min(dhi, dmax) + 1 minus the one of edge dlo
        const int hi = std::min(B.dhi, dmax) + 1;
        const int cx = std::min(hi, Nx), cy = std::min(hi, Ny), cz = std::min(hi, Nz);
        const long long cnt = (long long)cx * cy * cz -
                              (long long)std::min(B.dlo, Nx) * std::min(B.dlo, Ny) * std::min(B.dlo, Nz);
        const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>(cnt, 1 << 16));
        const double* D = T.D;
#define FAR_CASE(P_)                                                                                        \
    case P_:                                                                                                \
        hipLaunchKernelGGL(k_assemble_far<P_>, dim3(grid), dim3(64), 0, s, out, dF, b, D[0], D[1], D[2], T.k0, \
                           Nx, Ny, Nz, cx, cy, cz);                                                         \
        break;
        switch (B.P) {
            FAR_CASE(31)
            FAR_CASE(21)
            FAR_CASE(17)
            FAR_CASE(13)
            FAR_CASE(11)
            default: throw Error(-1, "assembly: unsupported Gauss order band");
        }
#undef FAR_CASE
        VIE_HIP(hipGetLastError());
    }
    VIE_HIP(hipStreamSynchronize(s));
    VIE_HIP(hipFree(dT));
    VIE_HIP(hipFree(dF));
}

// reflection sign of unique entry e along an axis (same for its whole orbit)
int unique_refl_sign(int e, int axis) {
    static const int P[6] = {0, 0, 0, 1, 1, 2}, Q[6] = {0, 1, 2, 1, 2, 2};
    static const int L[10] = {1, 1, 1, 1, 2, 2, 2, 3, 3, 4}, LP[10] = {1, 2, 3, 4, 2, 3, 4, 3, 4, 4};
    const int pq = e / 10, ll = e % 10;
    const int a = 4 * P[pq] + L[ll] - 1, b = 4 * Q[pq] + LP[ll] - 1;
    return refl_sign(axis, a) * refl_sign(axis, b);
}

// reflection sign of curl tensor e = 10 k + ll along an axis: the linear
// functions along the axis change sign, and d_k g is odd along k, so
// K(.., -d_i, ..) = -sigma_i(a) sigma_i(b) K(.., d_i, ..)
int curl_refl_sign(int e, int axis) {
    static const int L[10] = {1, 1, 1, 1, 2, 2, 2, 3, 3, 4}, LP[10] = {1, 2, 3, 4, 2, 3, 4, 3, 4, 4};
    const int k = e / 10, ll = e % 10;
    int s = 1;
    if (L[ll] == axis + 2) s = -s;
    if (LP[ll] == axis + 2) s = -s;
    if (k == axis) s = -s;
    return s;
}

void embed_and_transform(double2* U128, float2* U64, const double2* T, double2* circ, int Nx, int Ny, int Nz,
                         int Mx, int My, int Mz, const FftPlan plans[3], const double2* const tw[3],
                         hipStream_t s, bool curl) {
    const long long V = (long long)Nx * Ny * Nz;
    const long long M = (long long)Mx * My * Mz;
    const int Ox = Mx / 2 + 1, Oy = My / 2 + 1, Oz = Mz / 2 + 1;
    const long long O = (long long)Ox * Oy * Oz;
    const int nent = curl ? 30 : 60;
    for (int e = 0; e < nent; ++e) {
        int sg[3];
        for (int ax = 0; ax < 3; ++ax) sg[ax] = curl ? curl_refl_sign(e, ax) : unique_refl_sign(e, ax);
        hipLaunchKernelGGL(k_embed, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, circ, T + e * V, Nx, Ny, Nz,
                           Mx, My, Mz, sg[0], sg[1], sg[2]);
        VIE_HIP(hipGetLastError());
        // z pass: pencils along z, inner x (full length)
        StridedPass pz{};
        pz.plan = plans[2];
        pz.n_in = pz.n_out = Mz;
        pz.n_inner = Mx;
        pz.tile = strided_tile_for((int)sizeof(double2), Mz, 16);
        pz.pitch = pz.tile;
        pz.in_s1 = pz.out_s1 = 0;
        pz.in_sc = pz.out_sc = 0;
        pz.in_s2 = pz.out_s2 = Mx;          // o2 = y
        pz.in_sk = pz.out_sk = (long long)Mx * My;
        launch_strided<double>(true, circ, circ, pz, My, 1, tw[2], nullptr, s);
        StridedPass py{};
        py.plan = plans[1];
        py.n_in = py.n_out = My;
        py.n_inner = Mx;
        py.tile = strided_tile_for((int)sizeof(double2), My, 16);
        py.pitch = py.tile;
        py.in_s1 = py.out_s1 = 0;
        py.in_sc = py.out_sc = 0;
        py.in_s2 = py.out_s2 = (long long)Mx * My;   // o2 = z
        py.in_sk = py.out_sk = Mx;
        launch_strided<double>(true, circ, circ, py, Mz, 1, tw[1], nullptr, s);
        launch_rows<double>(true, circ, (long long)My * Mz, plans[0], tw[0], s);
        hipLaunchKernelGGL(k_octant, dim3((unsigned)((O + 255) / 256)), dim3(256), 0, s, U128, U64, circ, e, nent,
                           Mx, My, Ox, Oy, Oz);
        VIE_HIP(hipGetLastError());
    }
}

}  // namespace vie
