// FP64 Box-Muller transform of two Philox words, written out so that each
// normal costs a few dozen FP64 operations instead of the general-purpose
// log and sincospi:
//
//   z0 = sqrt(-2 ln u1) cos(2 pi u2),  z1 = sqrt(-2 ln u1) sin(2 pi u2),
//   u1 = (wa + 1) 2^-32 in (0, 1],  u2 = wb 2^-32 in [0, 1).
//
// ln u1: table-driven reduction (Tang, "Table-driven implementation of the
// logarithm function in IEEE floating-point arithmetic", ACM TOMS 16, 1990):
// u1 = 2^e m with m in [3/4, 3/2), F = round(256 m) / 256 (a grid point that
// includes 1, so u1 near 1 keeps its relative accuracy), r = (m - F) / F with
// |r| <= 1/384, and ln u1 = e ln 2 + ln F + ln(1 + r), the last from its
// Taylor series to r^7 (remainder below 3e-22). The table holds 1/F and ln F
// for the 193 grid points; ln 2 is split into a head with 32 significant bits
// (exact when multiplied by |e| <= 32) and a tail.
//
// cos, sin of 2 pi u2 = pi x, x = wb 2^-31 in [0, 2): x = q/2 + t with q =
// round(2x) and t in [-1/4, 1/4] (both exact), sin(pi t) and cos(pi t) from
// their Taylor series to t^17 and t^18 (remainders below 1e-19), and the
// quarter turns q mod 4 applied by swapping and negating.
//
// Functions are host and device, so that the host can check them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace icm {

constexpr int kLogTab = 193;  // grid points 192/256 .. 384/256

// Entry j of the table: inv[j] = 256 / (192 + j), lnf[j] = ln((192 + j) / 256).
__host__ __device__ inline void log_table_entry(int j, double* inv, double* lnf) {
    const double jd = (double)(192 + j);
    inv[j] = 256.0 / jd;
    lnf[j] = log(jd * 0.00390625);
}

// ln u for u in [2^-32, 1] (a multiple of 2^-32), with the table above.
__host__ __device__ inline double log_unit(double u, const double* inv, const double* lnf) {
    int e;
    double m = frexp(u, &e);  // u = m 2^e, m in [1/2, 1)
    if (m < 0.75) {
        m *= 2.0;
        e -= 1;
    }
    const double jd = rint(m * 256.0);
    const int j = (int)jd - 192;
    const double r = (m - jd * 0.00390625) * inv[j];  // m - F is exact
    // ln(1 + r) = r + r^2 (-1/2 + r (1/3 + r (-1/4 + r (1/5 + r (-1/6 + r / 7)))))
    double p = fma(r, 1.0 / 7.0, -1.0 / 6.0);
    p = fma(r, p, 1.0 / 5.0);
    p = fma(r, p, -0.25);
    p = fma(r, p, 1.0 / 3.0);
    p = fma(r, p, -0.5);
    p = fma(r * r, p, r);
    const double ln2_hi = 6.9314718036912381649e-01;  // 32 significant bits
    const double ln2_lo = 1.9082149292705877000e-10;
    const double de = (double)e;
    return fma(de, ln2_hi, fma(de, ln2_lo, lnf[j] + p));
}

// sin(pi x) and cos(pi x) for x in [0, 2) a multiple of 2^-31.
__host__ __device__ inline void sincospi_unit(double x, double* s, double* c) {
    const double q = rint(2.0 * x);
    const double t = fma(-0.5, q, x);
    const double t2 = t * t;
    // sin(pi t) / t and cos(pi t): coefficients (-1)^k pi^(2k+1) / (2k+1)! and
    // (-1)^k pi^(2k) / (2k)!
    double ps = 7.952054001475513e-07;
    ps = fma(t2, ps, -2.1915353447830217e-05);
    ps = fma(t2, ps, 4.6630280576761255e-04);
    ps = fma(t2, ps, -7.3704309457143504e-03);
    ps = fma(t2, ps, 8.214588661112823e-02);
    ps = fma(t2, ps, -5.992645293207921e-01);
    ps = fma(t2, ps, 2.5501640398773455e+00);
    ps = fma(t2, ps, -5.16771278004997e+00);
    ps = fma(t2, ps, 3.141592653589793e+00);
    const double S = ps * t;
    double pc = -1.3878952462213771e-07;
    pc = fma(t2, pc, 4.303069587032947e-06);
    pc = fma(t2, pc, -1.046381049248457e-04);
    pc = fma(t2, pc, 1.9295743094039231e-03);
    pc = fma(t2, pc, -2.580689139001406e-02);
    pc = fma(t2, pc, 2.353306303588932e-01);
    pc = fma(t2, pc, -1.3352627688545895e+00);
    pc = fma(t2, pc, 4.0587121264167685e+00);
    pc = fma(t2, pc, -4.934802200544679e+00);
    const double C = fma(t2, pc, 1.0);
    // quarter turns: (sin, cos) of pi (t + n/2), n = q mod 4
    const int n = (int)q & 3;
    const double sa = (n & 1) ? C : S, ca = (n & 1) ? S : C;
    *s = (n & 2) ? -sa : sa;
    *c = ((n + 1) & 2) ? -ca : ca;
}

__host__ __device__ inline void box_muller64(uint32_t wa, uint32_t wb, const double* inv, const double* lnf,
                                             double& z0, double& z1) {
    const double u1 = ((double)wa + 1.0) * 2.3283064365386963e-10;
    const double x = (double)wb * 4.6566128730773926e-10;  // 2 u2
    const double r = sqrt(-2.0 * log_unit(u1, inv, lnf));
    double s, c;
    sincospi_unit(x, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

}  // namespace icm
