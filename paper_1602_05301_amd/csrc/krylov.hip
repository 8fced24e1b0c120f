// Device building blocks of GMRES on the QBX-FMM matvec (Sec. 8.3): the
// Arnoldi step's Gram-Schmidt products over the stored Krylov vectors, the
// normalisation, and the interpolation of densities to oversampled panels
// (Sec. 3.2, Table 1).  Every sum runs in a fixed order, so results do not
// depend on timing.  These loops stream the Krylov basis from HBM once per
// call: they are bandwidth-bound.
#include <hip/hip_runtime.h>

#include "krylov.hpp"

namespace qbx {

namespace {

__device__ __forceinline__ cd kc_mul(cd a, cd b) { return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)}; }
__device__ __forceinline__ cd kc_cmul(cd a, cd b)     // conj(a) b
{
    return {fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -a.y * b.x)};
}

constexpr int KD_THREADS = 256;
constexpr int KD_COLS = 4;                    // columns per thread
constexpr int KD_CHUNK = KD_THREADS * KD_COLS;
constexpr int KD_ROWS = 8;                    // Krylov vectors per block

// partial[r * nchunk + c] = sum over chunk c of conj(V[r][j]) w[j], for the
// KD_ROWS rows of block y.  Within a block, lanes sum their columns in
// order and the block sums lanes by a fixed tree.
__global__ void __launch_bounds__(KD_THREADS) k_kdot_partial(long long n, int k, const cd *V, long long ldv,
                                                             const cd *w, cd *partial, int nchunk)
{
    __shared__ cd red[KD_THREADS];
    int c = blockIdx.x, r0 = blockIdx.y * KD_ROWS;
    long long j0 = (long long)c * KD_CHUNK + threadIdx.x;
    cd wj[KD_COLS];
#pragma unroll
    for (int t = 0; t < KD_COLS; ++t) {
        long long j = j0 + (long long)t * KD_THREADS;
        wj[t] = j < n ? w[j] : cd{0.0, 0.0};
    }
    for (int rr = 0; rr < KD_ROWS; ++rr) {
        int r = r0 + rr;
        if (r >= k) break;                      // uniform across the block
        const cd *vr = V + (long long)r * ldv;
        cd acc{0.0, 0.0};
#pragma unroll
        for (int t = 0; t < KD_COLS; ++t) {
            long long j = j0 + (long long)t * KD_THREADS;
            if (j < n) {
                cd p = kc_cmul(vr[j], wj[t]);
                acc.x += p.x;
                acc.y += p.y;
            }
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = KD_THREADS / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                red[threadIdx.x].x += red[threadIdx.x + s].x;
                red[threadIdx.x].y += red[threadIdx.x + s].y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(long long)r * nchunk + c] = red[0];
        __syncthreads();
    }
}

// h[r] = sum over chunks of partial[r][.], in chunk order.
__global__ void k_kdot_final(int k, const cd *partial, int nchunk, cd *h)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    cd acc{0.0, 0.0};
    for (int c = 0; c < nchunk; ++c) {
        cd p = partial[(long long)r * nchunk + c];
        acc.x += p.x;
        acc.y += p.y;
    }
    h[r] = acc;
}

constexpr int KU_THREADS = 256;
constexpr int KU_HTILE = 256;                 // coefficients staged in LDS at a time

// w[j] -= sum_i h[i] V[i][j], i in order.
__global__ void __launch_bounds__(KU_THREADS) k_kupdate(long long n, int k, const cd *V, long long ldv,
                                                        const cd *h, cd *w)
{
    __shared__ cd hs[KU_HTILE];
    long long j = (long long)blockIdx.x * KU_THREADS + threadIdx.x;
    cd acc{0.0, 0.0};
    for (int i0 = 0; i0 < k; i0 += KU_HTILE) {
        int m = min(KU_HTILE, k - i0);
        __syncthreads();
        if ((int)threadIdx.x < m) hs[threadIdx.x] = h[i0 + threadIdx.x];
        __syncthreads();
        if (j < n) {
            const cd *v = V + (long long)i0 * ldv + j;
            for (int i = 0; i < m; ++i) {
                cd p = kc_mul(hs[i], v[(long long)i * ldv]);
                acc.x += p.x;
                acc.y += p.y;
            }
        }
    }
    if (j < n) {
        cd x = w[j];
        w[j] = cd{x.x - acc.x, x.y - acc.y};
    }
}

// v[j] = w[j] / sqrt(Re nrm2[0]) (0 when the norm is 0).
__global__ void k_knormalize(long long n, const cd *w, const cd *nrm2, cd *v)
{
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = nrm2[0].x;
    double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    cd x = w[j];
    v[j] = cd{inv * x.x, inv * x.y};
}

// Panel p's density at its q nodes, x[p q + b], carried to its qs nodes:
// yd[p qs + a] = sum_b L[a q + b] x[p q + b]; ys = alpha yd.
__global__ void k_upsample(long long n_panels, int q, int qs, const double *L, cd alpha, const cd *x, cd *ys,
                           cd *yd)
{
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_panels * qs) return;
    long long p = t / qs;
    int a = (int)(t - p * qs);
    const cd *xp = x + p * q;
    const double *La = L + (long long)a * q;
    cd acc{0.0, 0.0};
    for (int b = 0; b < q; ++b) {
        acc.x = fma(La[b], xp[b].x, acc.x);
        acc.y = fma(La[b], xp[b].y, acc.y);
    }
    if (yd) yd[t] = acc;
    if (ys) ys[t] = kc_mul(alpha, acc);
}

}  // namespace

int krylov_dot_chunks(long long n) { return (int)((n + KD_CHUNK - 1) / KD_CHUNK); }

hipError_t launch_krylov_dot(long long n, int k, const cd *V, long long ldv, const cd *w, cd *partial, cd *h,
                             hipStream_t s)
{
    if (k <= 0) return hipSuccess;
    int nchunk = krylov_dot_chunks(n);
    if (nchunk > 0) {
        dim3 grid(nchunk, (k + KD_ROWS - 1) / KD_ROWS);
        k_kdot_partial<<<grid, KD_THREADS, 0, s>>>(n, k, V, ldv, w, partial, nchunk);
    }
    k_kdot_final<<<(k + 255) / 256, 256, 0, s>>>(k, partial, nchunk, h);
    return hipGetLastError();
}

hipError_t launch_krylov_update(long long n, int k, const cd *V, long long ldv, const cd *h, cd *w, hipStream_t s)
{
    if (n <= 0 || k <= 0) return hipSuccess;
    k_kupdate<<<(unsigned)((n + KU_THREADS - 1) / KU_THREADS), KU_THREADS, 0, s>>>(n, k, V, ldv, h, w);
    return hipGetLastError();
}

hipError_t launch_krylov_normalize(long long n, const cd *w, const cd *nrm2, cd *v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_knormalize<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, w, nrm2, v);
    return hipGetLastError();
}

hipError_t launch_upsample(long long n_panels, int q, int qs, const double *L, cd alpha, const cd *x, cd *ys,
                           cd *yd, hipStream_t s)
{
    long long t = n_panels * qs;
    if (t <= 0) return hipSuccess;
    k_upsample<<<(unsigned)((t + 255) / 256), 256, 0, s>>>(n_panels, q, qs, L, alpha, x, ys, yd);
    return hipGetLastError();
}

}  // namespace qbx
