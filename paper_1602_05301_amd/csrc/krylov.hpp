// Launchers of the GMRES building blocks (krylov.hip).  Pointers are device
// pointers; complex values are interleaved (re, im) doubles.
#pragma once

#include <hip/hip_runtime.h>

#include "devmath.hpp"

namespace qbx {

// Chunks of the first stage of krylov_dot (its partial sums need k * chunks
// complex values of workspace).
int krylov_dot_chunks(long long n);
hipError_t launch_krylov_dot(long long n, int k, const cd *V, long long ldv, const cd *w, cd *partial, cd *h,
                             hipStream_t s);
hipError_t launch_krylov_update(long long n, int k, const cd *V, long long ldv, const cd *h, cd *w, hipStream_t s);
hipError_t launch_krylov_normalize(long long n, const cd *w, const cd *nrm2, cd *v, hipStream_t s);
hipError_t launch_upsample(long long n_panels, int q, int qs, const double *L, cd alpha, const cd *x, cd *ys,
                           cd *yd, hipStream_t s);

}  // namespace qbx
