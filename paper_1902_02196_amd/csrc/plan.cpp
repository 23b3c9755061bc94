// FFT plans: radix sequence and FP64 twiddle tables.
#include <cmath>
#include <vector>

#include "ctx.hpp"

namespace vie {

bool smooth235(int n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

// radices: 16 while possible, then 8 / 4 / 2 for the remaining power of two,
// then 3s and 5s
FftPlan make_plan(int n) {
    VIE_REQUIRE(smooth235(n), VIE_EINVAL, "fft length must be 2/3/5-smooth");
    FftPlan p{};
    p.n = n;
    p.npass = 0;
    int m = n;
    auto push = [&](int r) {
        VIE_REQUIRE(p.npass < kMaxPasses, VIE_EINVAL, "fft length has too many factors");
        p.radix[p.npass++] = r;
        m /= r;
    };
    while (m % 16 == 0) push(16);
    if (m % 8 == 0) push(8);
    if (m % 4 == 0) push(4);
    if (m % 2 == 0) push(2);
    while (m % 3 == 0) push(3);
    while (m % 5 == 0) push(5);
    VIE_REQUIRE(p.npass > 0, VIE_EINVAL, "fft length must be >= 2");
    return p;
}

// W[m] = exp(-2 pi i m / n), evaluated in extended precision and rounded
void make_twiddles(int n, std::vector<double2>& tw) {
    tw.resize(n);
    for (int m = 0; m < n; ++m) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
        tw[m].x = (double)std::cos(a);
        tw[m].y = -(double)std::sin(a);
    }
}

}  // namespace vie
