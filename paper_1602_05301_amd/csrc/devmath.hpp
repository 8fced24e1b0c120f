// Complex arithmetic and Bessel/Hankel sequences for the gfx950 kernels.
//
// Hankel functions H_n^{(1)}(x) = J_n(x) + i Y_n(x) of real argument: H_0 and
// H_1 from their ascending series for x <= 4 and from the HIP device math
// library (j0, y0, j1, y1) above, higher orders by the
// upward three-term recurrence H_{n+1} = (2n/x) H_n - H_{n-1}, which is
// stable because Y_n dominates.  J_n by Miller's backward recurrence,
// normalised against whichever of J_0(x), J_1(x) is larger in magnitude.
#pragma once

#include <hip/hip_runtime.h>

namespace qbx {

struct cd {
    double x, y;
};

// complex float, for the translation tables of the FP32 far field
struct cf {
    float x, y;
};

__host__ __device__ __forceinline__ cd mk(double a, double b) { return {a, b}; }
__host__ __device__ __forceinline__ cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
// Complex product with explicit fused multiply-adds: the library is built
// without automatic contraction, so every rounding is written in the source
// and results do not depend on how the compiler schedules a kernel.
__host__ __device__ __forceinline__ cd operator*(cd a, cd b)
{
    return {fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}
__host__ __device__ __forceinline__ cd operator*(double s, cd a) { return {s * a.x, s * a.y}; }
__host__ __device__ __forceinline__ cd operator*(cd a, double s) { return {s * a.x, s * a.y}; }
__host__ __device__ __forceinline__ cd conj(cd a) { return {a.x, -a.y}; }
__host__ __device__ __forceinline__ cd neg(cd a) { return {-a.x, -a.y}; }
// acc += a * b
__host__ __device__ __forceinline__ void cfma(cd &acc, cd a, cd b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
__host__ __device__ __forceinline__ cd cdiv(cd a, cd b)
{
    double d = b.x * b.x + b.y * b.y;
    return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

// Miller start index M for J_0..J_N at argument x (the recurrence starts
// from f_{M+1} = 0).  Starting there leaves a relative error of about
// ((M+1)/n) (J_{M+1}/J_n)^2 in J_n.  For orders k + 1 >= x the ratios obey
// J_{k+1}/J_k = x / (2(k+1) - x J_{k+2}/J_{k+1}) <= x / (2(k+1) - x), so
// from k0 = max(N, ceil x) their product bounds J_M / J_k0; M is the first
// order where it falls below 1e-10.  For small x that is a few orders above
// N, which keeps the recurrence short and its dynamic range small.  M never
// exceeds the classical max(x, N) + 24 + 4 cbrt(max(x, N) + 1), which is
// what governs when x is near or above N (there the bound decays slowly).
__host__ __device__ __forceinline__ int miller_start(double x, int N)
{
    double m = x > (double)N ? x : (double)N;
    int cap = (int)m + 24 + (int)(4.0 * cbrt(m + 1.0));
    int k = (int)ceil(m);
    double bound = 1.0;
    while (k < cap && bound > 1e-10) {
        bound *= x / (2.0 * (k + 1) - x);
        ++k;
    }
    return k;
}

// J_n(x), n = 0..N, written to out[n * stride].  x >= 0.
__device__ inline void besselj_seq(double x, int N, double *out, long long stride)
{
    if (x == 0.0) {
        out[0] = 1.0;
        for (int n = 1; n <= N; ++n) out[n * stride] = 0.0;
        return;
    }
    int M = miller_start(x, N);
    double inv = 2.0 / x;
    double fp1 = 0.0, f = 1e-280, f1 = 0.0;
    for (int n = M; n > 0; --n) {
        if (n <= N) out[n * stride] = f;
        if (n == 1) f1 = f;
        double fm = (n * inv) * f - fp1;
        fp1 = f;
        f = fm;
        if (fabs(f) > 1e250) {
            f *= 1e-250;
            fp1 *= 1e-250;
            f1 *= 1e-250;
            for (int m = n; m <= N; ++m) out[m * stride] *= 1e-250;
        }
    }
    double jz = j0(x), jo = j1(x);
    double s = fabs(jz) >= fabs(jo) ? jz / f : jo / f1;
    out[0] = jz;
    for (int n = 1; n <= N; ++n) out[n * stride] *= s;
}

__device__ __attribute__((noinline)) void hankel01_lib(double x, cd &h0, cd &h1)
{
    h0 = mk(j0(x), y0(x));
    h1 = mk(j1(x), y1(x));
}

constexpr double kSeriesMaxX = 4.0;

// J0, J1, Y0, Y1 for 0 < x <= kSeriesMaxX from their ascending series
// (DLMF 10.2.2 and 10.8.1), t = x^2/4, H_k the harmonic numbers:
//   J0 = sum_k (-t)^k/(k!)^2,           J1 = (x/2) sum_k (-t)^k/(k!(k+1)!)
//   Y0 = (2/pi)[(ln(x/2) + gamma) J0 - sum_k H_k (-t)^k/(k!)^2]
//   Y1 = -2/(pi x) + (2/pi)(ln(x/2) + gamma) J1
//        - (x/(2 pi)) sum_k (H_k + H_{k+1}) (-t)^k/(k!(k+1)!)
// Terms up to k = 18: at x = 4 the first omitted one is below 1e-22 (the
// error against SciPy over (0, 4] is the same as with more terms, about
// 2e-15 of |H|, all rounding); the largest term is 4, so at most a few ulps
// are lost to cancellation.
__device__ __forceinline__ void hankel01_series(double x, cd &h0, cd &h1)
{
    const double t = -0.25 * x * x;
    double c = 1.0, d = 1.0;                      // (-t)^k/(k!)^2, (-t)^k/(k!(k+1)!)
    double sj0 = 1.0, sj1 = 1.0, sy0 = 0.0, sy1 = 1.0;
    double Hk = 0.0;
#pragma unroll
    for (int k = 1; k <= 18; ++k) {
        c *= t * (1.0 / ((double)k * k));
        d *= t * (1.0 / ((double)k * (k + 1)));
        Hk += 1.0 / k;
        double Hk1 = Hk + 1.0 / (k + 1);
        sj0 += c;
        sj1 += d;
        sy0 = fma(Hk, c, sy0);
        sy1 = fma(Hk + Hk1, d, sy1);
    }
    const double two_pi = 0.63661977236758134308;       // 2/pi
    const double euler_gamma = 0.57721566490153286061;
    double L = log(0.5 * x) + euler_gamma;
    double J0 = sj0, J1 = 0.5 * x * sj1;
    double Y0 = two_pi * (L * J0 - sy0);
    double Y1 = -two_pi / x + two_pi * L * J1 - (0.5 / 3.14159265358979323846) * x * sy1;
    h0 = mk(J0, Y0);
    h1 = mk(J1, Y1);
}

__device__ __forceinline__ void hankel01(double x, cd &h0, cd &h1)
{
    if (x <= kSeriesMaxX) hankel01_series(x, h0, h1);
    else hankel01_lib(x, h0, h1);
}

// A_n = tau^n H_n(x), n = 0..N, written to out[n * stride].  With
// tau = min(1, x/2) the sequence stays below (n-1)! in magnitude.
__device__ inline void scaled_hankel_seq(double x, double tau, int N, cd *out, long long stride)
{
    cd h0, h1;
    hankel01(x, h0, h1);
    cd a0 = h0, a1 = tau * h1;
    out[0] = a0;
    if (N >= 1) out[stride] = a1;
    double t2 = tau * tau;
    double c = 2.0 * tau / x;                 // one division, outside the recurrence
    for (int n = 1; n < N; ++n) {
        cd a2 = (((double)n * c) * a1) - (t2 * a0);
        out[(n + 1) * stride] = a2;
        a0 = a1;
        a1 = a2;
    }
}

}  // namespace qbx
