// Device arithmetic shared by the kernels: complex helpers and the evaluation of
// the Helmholtz kernel G_k(r) = e^{ikr} / (4 pi r) in FP64 and FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace ige {
namespace dm {

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
// acc + a b as four fused multiply-adds (no separate product and sum)
// surface element |d_uF x d_vF|
__device__ inline double surf_elem(const double Fu[3], const double Fv[3])
{
    const double nx = Fu[1] * Fv[2] - Fu[2] * Fv[1], ny = Fu[2] * Fv[0] - Fu[0] * Fv[2], nz = Fu[0] * Fv[1] - Fu[1] * Fv[0];
    return sqrt(fma(nx, nx, fma(ny, ny, nz * nz)));
}
__device__ inline double2 cmac(double2 acc, double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
__device__ inline float2 cmac(float2 acc, float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}

// FP64 (near-field quadrature, potential): 1/r by the hardware reciprocal square root and two Newton steps
// y <- y (3/2 - r^2 y^2 / 2); sin and cos of kappa r by Cody-Waite reduction
// t = kappa r - k pi/2 (pi/2 split into three doubles, products exact through
// fused multiply-add) and the Taylor polynomials of sin (to t^17) and cos (to t^18)
// on |t| <= pi/4, truncation below 1e-19; the quadrant k mod 4 selects signs.
// Valid for kappa r < 2^30.
__device__ inline double2 helmholtz_r2(double kappa, double r2)
{
    constexpr double kTwoOverPi = 0.6366197723675814;
    constexpr double kPio2_1 = 1.5707963267948966;
    constexpr double kPio2_2 = 6.123233995736766e-17;
    constexpr double kPio2_3 = -1.4973849048591698e-33;
    constexpr double kInv4Pi = 0.07957747154594767;
    double y = __builtin_amdgcn_rsq(r2);
    const double hh = 0.5 * r2;
    y = y * fma(-hh * y, y, 1.5);
    y = y * fma(-hh * y, y, 1.5);
    const double x = kappa * (r2 * y);
    const double k = rint(x * kTwoOverPi);
    double t = fma(-k, kPio2_1, x);
    t = fma(-k, kPio2_2, t);
    t = fma(-k, kPio2_3, t);
    const double z = t * t;
    double ps = -1.0 / 355687428096000.0;             // -1/17!
    ps = fma(ps, z, 1.0 / 1307674368000.0);           //  1/15!
    ps = fma(ps, z, -1.0 / 6227020800.0);             // -1/13!
    ps = fma(ps, z, 1.0 / 39916800.0);                //  1/11!
    ps = fma(ps, z, -1.0 / 362880.0);                 // -1/9!
    ps = fma(ps, z, 1.0 / 5040.0);                    //  1/7!
    ps = fma(ps, z, -1.0 / 120.0);                    // -1/5!
    ps = fma(ps, z, 1.0 / 6.0);                       //  1/3!
    const double s = fma(-t * z, ps, t);              // t - t z (1/3! - z/5! + ...)
    double pc = 1.0 / 6402373705728000.0;             //  1/18!
    pc = fma(pc, z, -1.0 / 20922789888000.0);         // -1/16!
    pc = fma(pc, z, 1.0 / 87178291200.0);             //  1/14!
    pc = fma(pc, z, -1.0 / 479001600.0);              // -1/12!
    pc = fma(pc, z, 1.0 / 3628800.0);                 //  1/10!
    pc = fma(pc, z, -1.0 / 40320.0);                  // -1/8!
    pc = fma(pc, z, 1.0 / 720.0);                     //  1/6!
    pc = fma(pc, z, -1.0 / 24.0);                     // -1/4!
    pc = fma(pc, z, 0.5);                             //  1/2!
    const double c = fma(-z, pc, 1.0);                // 1 - z (1/2! - z/4! + ...)
    const int q = (int)k & 3;
    double sn = (q & 1) ? c : s;
    double cs = (q & 1) ? s : c;
    if (q & 2) sn = -sn;
    if ((q + 1) & 2) cs = -cs;
    const double f = kInv4Pi * y;
    return make_double2(cs * f, sn * f);
}

// The same kernel with a table-driven sine and cosine (angle addition): x = kappa r is
// reduced by k = rint(x 128/pi) multiples of pi/128 in one fused multiply-add with the
// double nearest pi/128 (the reduced t is exact up to k times that double's error,
// 9.6e-19, that is 0.18 ulp(x) at most: below the rounding already in x = kappa r), so
// |t| <= pi/256; sin t from its Taylor series to t^5 (the next term is below 1e-17),
// cos t to t^6 (next term below 2e-20); tab[k mod 256] = (cos, sin)(k pi/128) / (4 pi)
// gives e^{ix} / (4 pi) = (C c - S s, S c + C s).  1/r from the hardware reciprocal
// square root y0 and one third-order step y = y0 (1 + e/2 + 3e^2/8), e = 1 - r^2 y0^2
// (the next term, 5e^3/16, is below 1e-21 for the hardware estimate's |e| < 1e-7).
// Valid for |kappa r| < 5e7 (k fits an int).  Measured against long-double sine and
// cosine over x in [0, 2000] and [1e-6, 1e6]: within 1.12 ulp(x) of e^{ix}.
__device__ inline double2 helmholtz_r2_tab(double kappa, double r2, const double2 *tab)
{
    constexpr double kInvStep = 40.74366543152521;   // 128/pi
    constexpr double kStep = 0.02454369260617026;    // pi/128 rounded to double
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e = fma(-(r2 * y0), y0, 1.0);
    const double y = fma(e * y0, fma(e, 0.375, 0.5), y0);
    const double x = kappa * (r2 * y);
    const double k = rint(x * kInvStep);
    const double t = fma(-k, kStep, x);
    const double2 cs = tab[(int)k & 255];
    const double z = t * t;
    const double ps = fma(z, 1.0 / 120.0, -1.0 / 6.0);   // 1/5!, -1/3!
    const double s = fma(t * z, ps, t);
    double pc = -1.0 / 720.0;                         // -1/6!
    pc = fma(pc, z, 1.0 / 24.0);                      //  1/4!
    pc = fma(pc, z, -0.5);                            // -1/2!
    const double c = fma(z, pc, 1.0);
    return make_double2(fma(cs.x, c, -cs.y * s) * y, fma(cs.y, c, cs.x * s) * y);
}

// FP32 counterpart (relative error about kappa r 2^-23 from the rounding of r):
// one Newton step on the FP32 reciprocal square root, pi/2 split into three
// floats, Taylor polynomials of sin to t^9 and cos to t^10 (truncation < 2e-9).
__device__ inline float2 helmholtz_r2(float kappa, float r2)
{
    constexpr float kTwoOverPi = 0.63661975f;
    constexpr float kPio2_1 = 1.5707963705062866f;
    constexpr float kPio2_2 = -4.371138828673793e-08f;
    constexpr float kPio2_3 = -1.7151245100058819e-15f;
    constexpr float kInv4Pi = 0.07957747f;
    float y = __builtin_amdgcn_rsqf(r2);
    y = y * fmaf(-0.5f * r2 * y, y, 1.5f);
    const float x = kappa * (r2 * y);
    const float k = rintf(x * kTwoOverPi);
    float t = fmaf(-k, kPio2_1, x);
    t = fmaf(-k, kPio2_2, t);
    t = fmaf(-k, kPio2_3, t);
    const float z = t * t;
    float ps = 1.0f / 362880.0f;                      //  1/9!
    ps = fmaf(ps, z, -1.0f / 5040.0f);                // -1/7!
    ps = fmaf(ps, z, 1.0f / 120.0f);                  //  1/5!
    ps = fmaf(ps, z, -1.0f / 6.0f);                   // -1/3!
    const float s = fmaf(t * z, ps, t);               // t + t z (-1/3! + z/5! - ...)
    float pc = -1.0f / 3628800.0f;                    // -1/10!
    pc = fmaf(pc, z, 1.0f / 40320.0f);                //  1/8!
    pc = fmaf(pc, z, -1.0f / 720.0f);                 // -1/6!
    pc = fmaf(pc, z, 1.0f / 24.0f);                   //  1/4!
    pc = fmaf(pc, z, -0.5f);                          // -1/2!
    const float c = fmaf(z, pc, 1.0f);
    const int q = (int)k & 3;
    float sn = (q & 1) ? c : s;
    float cs = (q & 1) ? s : c;
    if (q & 2) sn = -sn;
    if ((q + 1) & 2) cs = -cs;
    const float f = kInv4Pi * y;
    return make_float2(cs * f, sn * f);
}

template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };

__device__ inline double2 to_c(double2 a, double) { return a; }
__device__ inline float2 to_c(double2 a, float) { return make_float2((float)a.x, (float)a.y); }
__device__ inline double2 to_d(double2 a) { return a; }
__device__ inline double2 to_d(float2 a) { return make_double2(a.x, a.y); }

// Sum V values over the 64 lanes of a wave by recursive halving: at each step a
// lane keeps half of its values and adds the partner's copy of that half.  On exit
// every lane holds the total of value index lane >> (6 - log2 V).
template <int V>
struct Halve {
    static __device__ double run(const double *a, int lane, int off)
    {
        constexpr int H = V / 2;
        double b[H];
        const bool hi = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double send = hi ? a[i] : a[H + i];
            const double keep = hi ? a[H + i] : a[i];
            b[i] = keep + __shfl_xor(send, off, 64);
        }
        return Halve<H>::run(b, lane, off >> 1);
    }
};
template <>
struct Halve<1> {
    static __device__ double run(const double *a, int, int off)
    {
        double v = a[0];
        for (; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        return v;
    }
};
template <int V>
constexpr int log2c()
{
    return V <= 1 ? 0 : 1 + log2c<V / 2>();
}

}  // namespace dm
}  // namespace ige
