// Tables for the on-device assembly of the Galerkin blocks (Sec. III-C).
//
// The curl operator K = curl S (eq. 8b, 25b) is assembled by the same code
// from its own table: unique entry Q_k^{ll'}(d) = <N^l, S D_k N^{l'}>
// (the derivative of g moved onto the basis function by parts), from which
// K^{pl,ql'} = sum_k eps_pkq Q_k^{ll'}.
//
// Each entry N^{pl,ql'}(d) = delta_{d0} Gram + k0^2 delta_pq S^{ll'}(d) - C^{pl,ql'}(d)
// (curl curl S = k0^2 S + grad div S + I, with grad div moved onto the test
// and basis functions by parts).  Both S and C are 6-D integrals of
// g(d Delta + u - v) times a product over the three axes of 1-D weights; each
// pair of 1-D integrals collapses to one integral over w = u - v against the
// correlation of the two 1-D weights ("axis kernel").  An axis kernel is a
// cubic density on [-D, 0], a cubic on [0, D], and point masses at -D, 0, D.
#pragma once

namespace vie {

// 1-D measures: 0 = pulse '1', 1 = linear 't/D', 2 = derivative of the pulse
// restricted to the voxel, 3 = derivative of the linear function.
struct AxisKernel {
    double left[4];   // c0 + c1 w + c2 w^2 + c3 w^3 on [-D, 0]
    double right[4];  // on [0, D]
    double pts[3];    // masses at w = -D, 0, +D
};

struct EntryTerms {
    int nterm;
    double coef[2];
    int ker[2][3];    // axis-kernel index per term and axis (axis * 16 + pair)
    int gram_l;       // -1, or the scalar basis (0..3) of a Gram diagonal entry
};

constexpr int kMaxGauss = 16;

struct AssemblyTables {
    AxisKernel ker[48];
    int nent;          // unique entries: 60 for N, 30 for the curl operator K
    EntryTerms ent[60];
    double gl_x[kMaxGauss + 1][kMaxGauss];   // Gauss-Legendre on [0, 1]
    double gl_w[kMaxGauss + 1][kMaxGauss];
    double D[3];
    double k0;
    double gram[4];
    int order_near;     // Gauss order for offsets with max |d_i| <= 2
    int order_duffy;    // order of each Duffy factor
};

// Separable far-field assembly.  Away from the singular corner (max |d_i| >= 2)
// every geometry of every entry is integrated with the same Gauss order n on
// each axis, so all 60 entries sample the Green's function on one common
// tensor grid per offset: per axis, n points on [-D, 0], n on [0, D] and the
// three point-mass abscissae -D, 0, D (P = 2 n + 3 in all).  An entry term is
// then sum_{ijk} Wx[kx][i] Wy[ky][j] Wz[kz][k] g(d Delta + w_ijk), the W the
// axis-kernel weights at the grid points (zero where the kernel has no
// support); points with two or more point-mass axes carry no weight and are
// left out.  The sum is contracted one axis at a time.
constexpr int kFarBands = 5;
constexpr int kFarPMax = 31;       // 2 * 14 + 3
constexpr int kFarTerms = 120;     // (entry, term) pairs, at most 2 terms per entry

struct FarBand {
    int n, P;                      // Gauss order, grid points per axis
    int dlo, dhi;                  // offsets with dlo <= max |d_i| <= dhi
    double w[3][kFarPMax];         // abscissae per axis
    double W[3][16][kFarPMax];     // weight of axis kernel pair (kt, kb) at each abscissa
    int ispt[kFarPMax];            // 1 for the point-mass abscissae
};

struct FarTables {
    FarBand band[kFarBands];
    int nent;                      // unique entries (60 N, 30 K)
    int nterm;                     // flattened (entry, term) list
    int term_kx[kFarTerms];        // axis-kernel pair along x
    int term_pair[kFarTerms];      // index into the (ky, kz) pair list
    double term_coef[kFarTerms];
    int ent_first[60], ent_count[60];
    int npair;
    int pair_ky[kFarTerms], pair_kz[kFarTerms];
};

}  // namespace vie
