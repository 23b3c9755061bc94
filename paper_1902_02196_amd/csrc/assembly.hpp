// Tables for the on-device assembly of the Galerkin blocks (Sec. III-C).
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
    EntryTerms ent[60];
    double gl_x[kMaxGauss + 1][kMaxGauss];   // Gauss-Legendre on [0, 1]
    double gl_w[kMaxGauss + 1][kMaxGauss];
    double D[3];
    double k0;
    double gram[4];
    int order_near;     // Gauss order for offsets with max |d_i| <= 2
    int order_duffy;    // order of each Duffy factor
};

}  // namespace vie
