// Complex exponential from small tables, for the near-field sweep (host and
// device, so that its accuracy can be checked on the host).
//
// Method: table-driven reduction in the manner of Tang's exponential (P. T. P.
// Tang, "Table-driven implementation of the exponential function in IEEE
// floating-point arithmetic", ACM TOMS 15(2), 1989: a 2^{j/32}-type table plus
// a short polynomial on the reduced argument), applied here with 64 entries to
// e^a and, with a table of sin and cos at multiples of pi/32, to e^{ib}; the
// argument reductions subtract the multiple of the step in several parts
// (Cody and Waite, "Software Manual for the Elementary Functions", 1980).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "lmfmm_internal.h"

namespace lmfmm {

// Complex exponential e^{a + ib} for the sweep, from small tables in LDS:
//   e^a  = 2^m 2^{j/64} e^r  with a = (64m + j) ln2/64 + r, |r| <= ln2/128, and
//          e^r by its Taylor polynomial to r^5 (remainder < 4e-17 relative);
//   e^ib = e^{i n pi/32} e^{i r'}  with b = n pi/32 + r', |r'| <= pi/64, and
//          sin r', cos r' by Taylor polynomials to r'^9 and r'^8 (remainder
//          < 1e-20 relative).
// The reductions subtract k ln2/64 and n pi/32 in parts whose leading pieces
// carry 32 significant bits, so that k and n times them are exact below 2^21
// (ln2/64 in two parts; pi/32 in three; the constants are the binary
// expansions of ln2/64 and pi/32 cut after 32 bits, the next 32 bits, and the
// rounded rest).  |b| above 1e5 takes the library sincos.
struct CexpTab {
    double t2[64];  // 2^{j/64}
    double sn[64];  // sin(j pi/32)
    double cs[64];  // cos(j pi/32)
};

__host__ __device__ inline cx<double> cexp_tab(double a, double b, const CexpTab &tb)
{
    constexpr double INV_LN2_64 = 0x1.71547652b82fep+6, LN2_64_HI = 0x1.62e42fee00000p-7,
                     LN2_64_LO = 0x1.a39ef35793c76p-39;
    constexpr double INV_PI32 = 0x1.45f306dc9c883p+3, PI32_1 = 0x1.921fb54400000p-4,
                     PI32_2 = 0x1.0b4611a600000p-38, PI32_3 = 0x1.3198a2e037073p-73;
    a = fmin(fmax(a, -2000.0), 2000.0);  // beyond: 0 or inf either way
    const double kd = rint(a * INV_LN2_64);
    const double r = fma(-kd, LN2_64_LO, fma(-kd, LN2_64_HI, a));
    const int k = (int)kd;
    const double pr = fma(r, fma(r, fma(r, fma(r, fma(r, 1.0 / 120, 1.0 / 24), 1.0 / 6), 0.5), 1.0), 1.0);
    const double ea = ldexp(tb.t2[k & 63] * pr, k >> 6);
    double sb, cb;
    if (fabs(b) <= 1.0e5) {
        const double nd = rint(b * INV_PI32);
        const double rr = fma(-nd, PI32_3, fma(-nd, PI32_2, fma(-nd, PI32_1, b)));
        const int jn = (int)nd & 63;
        const double z = rr * rr;
        const double sr =
            rr * fma(z, fma(z, fma(z, fma(z, 1.0 / 362880, -1.0 / 5040), 1.0 / 120), -1.0 / 6), 1.0);
        const double cr = fma(z, fma(z, fma(z, fma(z, 1.0 / 40320, -1.0 / 720), 1.0 / 24), -0.5), 1.0);
        const double S = tb.sn[jn], C = tb.cs[jn];
        sb = fma(S, cr, C * sr);
        cb = fma(C, cr, -S * sr);
    } else {
        sincos(b, &sb, &cb);
    }
    return {ea * cb, ea * sb};
}

// x-slabs of a leaf column of n points: one if they fit in LDS, else slabs of
// about half the capacity each
__device__ inline int sweep_slabs(int n, int nmax) { return n <= nmax ? 1 : (n + nmax / 2 - 1) / (nmax / 2); }

// slab of position x in a leaf column starting at xl, K slabs of width 1/sc:
// nondecreasing in x, so slab order is x order
__device__ inline int slab_of(double x, double xl, double sc, int K)
{
    int b = (int)floor((x - xl) * sc);
    return b < 0 ? 0 : (b >= K ? K - 1 : b);
}

}  // namespace lmfmm
