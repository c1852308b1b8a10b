// Device helpers shared by the libigabem kernels: a complex type, the
// fundamental solutions, Bernstein bases and rational Bezier tile evaluation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace igb {

struct cd {
    double re, im;
};

__host__ __device__ inline cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cd operator-(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cd operator*(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline cd operator*(cd a, double b) { return {a.re * b, a.im * b}; }
__host__ __device__ inline cd operator*(double b, cd a) { return {a.re * b, a.im * b}; }
__host__ __device__ inline cd &operator+=(cd &a, cd b) { a.re += b.re; a.im += b.im; return a; }
__host__ __device__ inline cd &operator-=(cd &a, cd b) { a.re -= b.re; a.im -= b.im; return a; }

template <class T> __host__ __device__ inline T zero();
template <> __host__ __device__ inline double zero<double>() { return 0.0; }
template <> __host__ __device__ inline cd zero<cd>() { return {0.0, 0.0}; }

__host__ __device__ inline double conj_(double a) { return a; }
__host__ __device__ inline cd conj_(cd a) { return {a.re, -a.im}; }
__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline double abs2(cd a) { return a.re * a.re + a.im * a.im; }

// sin t and cos t for |t| < 2^19: the Helmholtz phase kappa |x - y| between surface points (the operator
// checks kappa times the size of the geometry at creation).  Branch-free.
//  * Range reduction after Cody and Waite: t = n pi + y with n the integer nearest t/pi, |y| <= pi/2 up
//    to rounding.  n comes from adding 1.5 2^52 in the fused multiply-add t (1/pi) + 1.5 2^52, whose
//    result has unit spacing, so its lowest mantissa bit is the parity of n.  pi = C1 + C2 with C1 of 30
//    significant bits, so n C1 is exact for |n| < 2^23 and t - n C1 is exact as well (Sterbenz: n C1 is
//    within a factor two of t for n != 0); C2 is the rest rounded to 53 bits and enters by one fused
//    multiply-add, which rounds once and leaves |n (pi - C1 - C2)| < 6e-21.
//  * On |y| <= pi/2 the Taylor series of sin (through y^21) and of cos (through y^20), evaluated by
//    Horner's rule in z = y^2; the first omitted terms, (pi/2)^23/23! and (pi/2)^22/22!, are below 2^-55.
//  * sin(n pi + y) = (-1)^n sin y and cos(n pi + y) = (-1)^n cos y: the parity of n flips both sign bits.
__host__ __device__ inline void sincos_red(double t, double *sn, double *cs)
{
    const double m = fma(t, 0x1.45f306dc9c883p-2, 0x1.8p52);  // t (1/pi) + 1.5 2^52
    const double n = m - 0x1.8p52;
    double y = fma(-n, 0x1.921fb548p+1, t);            // C1
    y = fma(-n, -0x1.de973dcb3b39ap-30, y);            // C2
    const double z = y * y;
    double ps = 0x1.71b8ef6dcf572p-66;                 //  1/21!
    ps = fma(ps, z, -0x1.2f49b46814157p-57);           // -1/19!
    ps = fma(ps, z, 0x1.952c77030ad4ap-49);            //  1/17!
    ps = fma(ps, z, -0x1.ae7f3e733b81fp-41);           // -1/15!
    ps = fma(ps, z, 0x1.6124613a86d09p-33);            //  1/13!
    ps = fma(ps, z, -0x1.ae64567f544e4p-26);           // -1/11!
    ps = fma(ps, z, 0x1.71de3a556c734p-19);            //  1/9!
    ps = fma(ps, z, -0x1.a01a01a01a01ap-13);           // -1/7!
    ps = fma(ps, z, 0x1.1111111111111p-7);             //  1/5!
    ps = fma(ps, z, -0x1.5555555555555p-3);            // -1/3!
    const double sy = fma(y * z, ps, y);               // sin y = y + y^3 (-1/3! + z/5! - ...)
    double pc = 0x1.e542ba4020225p-62;                 //  1/20!
    pc = fma(pc, z, -0x1.6827863b97d97p-53);           // -1/18!
    pc = fma(pc, z, 0x1.ae7f3e733b81fp-45);            //  1/16!
    pc = fma(pc, z, -0x1.93974a8c07c9dp-37);           // -1/14!
    pc = fma(pc, z, 0x1.1eed8eff8d898p-29);            //  1/12!
    pc = fma(pc, z, -0x1.27e4fb7789f5cp-22);           // -1/10!
    pc = fma(pc, z, 0x1.a01a01a01a01ap-16);            //  1/8!
    pc = fma(pc, z, -0x1.6c16c16c16c17p-10);           // -1/6!
    pc = fma(pc, z, 0x1.5555555555555p-5);             //  1/4!
    const double cy = fma(z * z, pc, fma(z, -0.5, 1.0));  // cos y = 1 - z/2 + z^2 (1/4! - z/6! + ...)
    const unsigned long long flip = __builtin_bit_cast(unsigned long long, m) << 63;
    *sn = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, sy) ^ flip);
    *cs = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, cy) ^ flip);
}

// sin t and cos t for 0 <= t <= 2^19 from a table of 256 pairs tab[j] = (sin(j pi/128), cos(j pi/128)),
// j < 256 (one period, 16-byte aligned): t = n pi/128 + y with |y| <= pi/256 (Cody-Waite reduction with
// pi/128 = C1 + C2: C1 has 29 bits, so n C1 is exact for n < 2^24 and t - n C1 is exact by Sterbenz; C2
// is the rest rounded to 53 bits and enters by one fused multiply-add, leaving |n (pi/128 - C1 - C2)| <
// 6e-21), sin y by its Taylor series through y^5 and cos y - 1 through y^6 (truncation below 1e-17), then
// the angle-sum formulas sin(a + y) = sin a (1 + (cos y - 1)) + cos a sin y and cos(a + y) = cos a (1 +
// (cos y - 1)) - sin a sin y with entry j = n mod 256.  Fifteen double operations against twenty-nine
// for sincos_red.
typedef double v2d_tab __attribute__((ext_vector_type(2)));
__device__ inline void sincos_tab(double t, const double *tab, double *sn, double *cs)
{
    const double m = fma(t, 0x1.45f306dc9c883p+5, 0x1.8p52);  // t (128/pi) + 1.5 2^52: n in the low bits
    const double n = m - 0x1.8p52;
    double y = fma(-n, 0x1.921fb54p-6, t);
    y = fma(-n, 0x1.10b4611a62633p-36, y);
    const int j = (int)(__builtin_bit_cast(unsigned long long, m) & 255u);
    const v2d_tab e = reinterpret_cast<const v2d_tab *>(tab)[j];
    const double sa = e.x, ca = e.y;
    const double z = y * y;
    const double sy = fma(y * z, fma(z, 0x1.1111111111111p-7, -0x1.5555555555555p-3), y);
    const double cm = z * fma(z, fma(z, -0x1.6c16c16c16c17p-10, 0x1.5555555555555p-5), -0.5);
    *sn = fma(sa, cm, fma(ca, sy, sa));
    *cs = fma(ca, cm, fma(-sa, sy, ca));
}

// Fundamental solutions of Sec. 3.1 (eq. fundament1 / fundament2) at distance r.
template <class T> __device__ inline T green(double r, double kappa);
template <> __device__ inline double green<double>(double r, double) { return 0.07957747154594767 / r; }
template <> __device__ inline cd green<cd>(double r, double kappa)
{
    double s, c;
    sincos_red(kappa * r, &s, &c);
    double f = 0.07957747154594767 / r;
    return {c * f, s * f};
}

// The same at any distance (evaluation points off the surface are not bounded by the geometry's size).
template <class T> __device__ inline T green_any(double r, double kappa);
template <> __device__ inline double green_any<double>(double r, double) { return 0.07957747154594767 / r; }
template <> __device__ inline cd green_any<cd>(double r, double kappa)
{
    double s, c;
    sincos(kappa * r, &s, &c);
    double f = 0.07957747154594767 / r;
    return {c * f, s * f};
}

// Bernstein polynomials of degree p at t (and derivatives), p <= 8.
__device__ inline void bernstein(int p, double t, double *B)
{
    double s = 1.0 - t;
    B[0] = 1.0;
    for (int k = 1; k <= p; ++k) {
        B[k] = t * B[k - 1];
        for (int i = k - 1; i >= 1; --i) B[i] = s * B[i] + t * B[i - 1];
        B[0] = s * B[0];
    }
}

__device__ inline void bernstein_d(int p, double t, double *B, double *dB)
{
    if (p == 0) {
        B[0] = 1.0;
        dB[0] = 0.0;
        return;
    }
    double lo[9];
    double s = 1.0 - t;
    lo[0] = 1.0;
    for (int k = 1; k < p; ++k) {
        lo[k] = t * lo[k - 1];
        for (int i = k - 1; i >= 1; --i) lo[i] = s * lo[i] + t * lo[i - 1];
        lo[0] = s * lo[0];
    }
    B[p] = t * lo[p - 1];
    for (int i = p - 1; i >= 1; --i) B[i] = s * lo[i] + t * lo[i - 1];
    B[0] = s * lo[0];
    dB[0] = -p * lo[0];
    for (int i = 1; i < p; ++i) dB[i] = p * (lo[i - 1] - lo[i]);
    dB[p] = p * lo[p - 1];
}

// Rational Bezier tile (homogeneous control points H[(j*(pu+1)+i)*4 + c]) at
// element-local (u, v): point X and surface measure w.r.t. (u, v).
__device__ inline void tile_point(const double *H, int pu, int pv, double u, double v, double X[3], double *kap)
{
    double Bu[9], dBu[9], Bv[9], dBv[9];
    bernstein_d(pu, u, Bu, dBu);
    bernstein_d(pv, v, Bv, dBv);
    double S0 = 0, S1 = 0, S2 = 0, S3 = 0, U0 = 0, U1 = 0, U2 = 0, U3 = 0, V0 = 0, V1 = 0, V2 = 0, V3 = 0;
    for (int j = 0; j <= pv; ++j) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, d0 = 0, d1 = 0, d2 = 0, d3 = 0;
        const double *h = H + 4 * j * (pu + 1);
        for (int i = 0; i <= pu; ++i) {
            double b = Bu[i], db = dBu[i];
            a0 += b * h[4 * i];
            a1 += b * h[4 * i + 1];
            a2 += b * h[4 * i + 2];
            a3 += b * h[4 * i + 3];
            d0 += db * h[4 * i];
            d1 += db * h[4 * i + 1];
            d2 += db * h[4 * i + 2];
            d3 += db * h[4 * i + 3];
        }
        double bv = Bv[j], dbv = dBv[j];
        S0 += bv * a0; S1 += bv * a1; S2 += bv * a2; S3 += bv * a3;
        U0 += bv * d0; U1 += bv * d1; U2 += bv * d2; U3 += bv * d3;
        V0 += dbv * a0; V1 += dbv * a1; V2 += dbv * a2; V3 += dbv * a3;
    }
    double iw = 1.0 / S3;
    double x0 = S0 * iw, x1 = S1 * iw, x2 = S2 * iw;
    double u0 = (U0 - x0 * U3) * iw, u1 = (U1 - x1 * U3) * iw, u2 = (U2 - x2 * U3) * iw;
    double v0 = (V0 - x0 * V3) * iw, v1 = (V1 - x1 * V3) * iw, v2 = (V2 - x2 * V3) * iw;
    X[0] = x0;
    X[1] = x1;
    X[2] = x2;
    double n0 = u1 * v2 - u2 * v1, n1 = u2 * v0 - u0 * v2, n2 = u0 * v1 - u1 * v0;
    *kap = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
}

// Compile-time-degree Bernstein values and derivatives (loops fully unrolled).
template <int P>
__device__ inline void bernstein_t(double t, double *B)
{
    double s = 1.0 - t;
    B[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= P; ++k) {
        B[k] = t * B[k - 1];
#pragma unroll
        for (int i = k - 1; i >= 1; --i) B[i] = s * B[i] + t * B[i - 1];
        B[0] = s * B[0];
    }
}

template <int P>
__device__ inline void bernstein_d_t(double t, double *B, double *dB)
{
    if constexpr (P == 0) {
        B[0] = 1.0;
        dB[0] = 0.0;
    } else {
        double lo[P];
        bernstein_t<P - 1>(t, lo);
        double s = 1.0 - t;
        B[P] = t * lo[P - 1];
#pragma unroll
        for (int i = P - 1; i >= 1; --i) B[i] = s * lo[i] + t * lo[i - 1];
        B[0] = s * lo[0];
        dB[0] = -P * lo[0];
#pragma unroll
        for (int i = 1; i < P; ++i) dB[i] = P * (lo[i - 1] - lo[i]);
        dB[P] = P * lo[P - 1];
    }
}

// Rational Bezier tile of bidegree (PG, PG) at element-local (u, v): point and
// surface measure w.r.t. (u, v).
template <int PG>
__device__ inline void tile_point_t(const double *H, double u, double v, double X[3], double *kap)
{
    constexpr int G1 = PG + 1;
    double Bu[G1], dBu[G1], Bv[G1], dBv[G1];
    bernstein_d_t<PG>(u, Bu, dBu);
    bernstein_d_t<PG>(v, Bv, dBv);
    double S0 = 0, S1 = 0, S2 = 0, S3 = 0, U0 = 0, U1 = 0, U2 = 0, U3 = 0, V0 = 0, V1 = 0, V2 = 0, V3 = 0;
#pragma unroll
    for (int j = 0; j < G1; ++j) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, d0 = 0, d1 = 0, d2 = 0, d3 = 0;
        const double *h = H + 4 * j * G1;
#pragma unroll
        for (int i = 0; i < G1; ++i) {
            double b = Bu[i], db = dBu[i];
            a0 += b * h[4 * i];
            a1 += b * h[4 * i + 1];
            a2 += b * h[4 * i + 2];
            a3 += b * h[4 * i + 3];
            d0 += db * h[4 * i];
            d1 += db * h[4 * i + 1];
            d2 += db * h[4 * i + 2];
            d3 += db * h[4 * i + 3];
        }
        double bv = Bv[j], dbv = dBv[j];
        S0 += bv * a0; S1 += bv * a1; S2 += bv * a2; S3 += bv * a3;
        U0 += bv * d0; U1 += bv * d1; U2 += bv * d2; U3 += bv * d3;
        V0 += dbv * a0; V1 += dbv * a1; V2 += dbv * a2; V3 += dbv * a3;
    }
    double iw = 1.0 / S3;
    double x0 = S0 * iw, x1 = S1 * iw, x2 = S2 * iw;
    double u0 = (U0 - x0 * U3) * iw, u1 = (U1 - x1 * U3) * iw, u2 = (U2 - x2 * U3) * iw;
    double v0 = (V0 - x0 * V3) * iw, v1 = (V1 - x1 * V3) * iw, v2 = (V2 - x2 * V3) * iw;
    X[0] = x0;
    X[1] = x1;
    X[2] = x2;
    double n0 = u1 * v2 - u2 * v1, n1 = u2 * v0 - u0 * v2, n2 = u0 * v1 - u1 * v0;
    *kap = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
}

template <class T> struct NComp { static constexpr int value = 1; };
template <> struct NComp<cd> { static constexpr int value = 2; };

__device__ inline double re_(double a) { return a; }
__device__ inline double re_(cd a) { return a.re; }
__device__ inline double im_(double) { return 0.0; }
__device__ inline double im_(cd a) { return a.im; }

}  // namespace igb
