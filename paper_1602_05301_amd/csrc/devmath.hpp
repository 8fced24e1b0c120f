// Complex arithmetic and Bessel/Hankel sequences for the gfx950 kernels.
//
// Hankel functions H_n^{(1)}(x) = J_n(x) + i Y_n(x) of real argument: H_0 and
// H_1 from the HIP device math library (j0, y0, j1, y1), higher orders by the
// upward three-term recurrence H_{n+1} = (2n/x) H_n - H_{n-1}, which is
// stable because Y_n dominates.  J_n by Miller's backward recurrence,
// normalised against whichever of J_0(x), J_1(x) is larger in magnitude.
#pragma once

#include <hip/hip_runtime.h>

namespace qbx {

struct cd {
    double x, y;
};

__host__ __device__ __forceinline__ cd mk(double a, double b) { return {a, b}; }
__host__ __device__ __forceinline__ cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ __forceinline__ cd operator*(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
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

// Miller start index for J_0..J_N at argument x.
__host__ __device__ __forceinline__ int miller_start(double x, int N)
{
    double m = x > (double)N ? x : (double)N;
    return (int)m + 24 + (int)(4.0 * cbrt(m + 1.0));
}

// J_n(x), n = 0..N, written to out[n * stride].  x >= 0.
__device__ inline void besselj_seq(double x, int N, double *out, int stride)
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

__device__ __forceinline__ void hankel01(double x, cd &h0, cd &h1)
{
    h0 = mk(j0(x), y0(x));
    h1 = mk(j1(x), y1(x));
}

// A_n = tau^n H_n(x), n = 0..N, written to out[n * stride].  With
// tau = min(1, x/2) the sequence stays below (n-1)! in magnitude.
__device__ inline void scaled_hankel_seq(double x, double tau, int N, cd *out, int stride)
{
    cd h0, h1;
    hankel01(x, h0, h1);
    cd a0 = h0, a1 = tau * h1;
    out[0] = a0;
    if (N >= 1) out[stride] = a1;
    double t2 = tau * tau;
    for (int n = 1; n < N; ++n) {
        cd a2 = ((2.0 * n * tau / x) * a1) - (t2 * a0);
        out[(n + 1) * stride] = a2;
        a0 = a1;
        a1 = a2;
    }
}

}  // namespace qbx
