// Host check of the near-field sweep's table exponential (cexp_tab.h): the
// tables are filled with correctly rounded values from long double, and the
// result is compared with expl, cosl and sinl on random arguments.  Prints the
// largest error relative to |e^z| per range and exits nonzero above 1e-15.
#include "cexp_tab.h"

#include <cmath>
#include <cstdio>
#include <random>

int main()
{
    lmfmm::CexpTab tb;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < 64; ++j) {
        tb.t2[j] = (double)exp2l(j / 64.0L);
        tb.sn[j] = (double)sinl(pi * j / 32.0L);
        tb.cs[j] = (double)cosl(pi * j / 32.0L);
    }
    std::mt19937_64 g(7);
    const double ranges[][4] = {{-1, 1, -4, 4},      {-700, 300, -1000, 1000}, {-5, 5, -1e5, 1e5},
                                {-1e-3, 1e-3, -1e-3, 1e-3}, {-40, 40, 2e5, 3e5}};
    double worst = 0;
    for (const auto &rg : ranges) {
        std::uniform_real_distribution<double> da(rg[0], rg[1]), db(rg[2], rg[3]);
        double w = 0;
        for (int i = 0; i < 200000; ++i) {
            const double a = da(g), b = db(g);
            const lmfmm::cx<double> z = lmfmm::cexp_tab(a, b, tb);
            const long double ea = expl((long double)a), cr = ea * cosl((long double)b), ci = ea * sinl((long double)b);
            const long double err = sqrtl((z.re - cr) * (z.re - cr) + (z.im - ci) * (z.im - ci)) / ea;
            if ((double)err > w) w = (double)err;
        }
        printf("a in [%g, %g], b in [%g, %g]: max error %.3g\n", rg[0], rg[1], rg[2], rg[3], w);
        worst = w > worst ? w : worst;
    }
    // the ends: underflow to zero, overflow to infinity, as e^a does
    const lmfmm::cx<double> lo = lmfmm::cexp_tab(-5000.0, 1.0, tb), hi = lmfmm::cexp_tab(800.0, 0.0, tb);
    const bool ends = lo.re == 0.0 && lo.im == 0.0 && std::isinf(hi.re);
    printf("ends %s\n", ends ? "ok" : "wrong");
    return worst < 1e-15 && ends ? 0 : 1;
}
