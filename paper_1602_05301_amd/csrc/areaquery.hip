// Area queries (Sec. 5) and target association through them (Sec. 6.1).
//
// An area query returns the leaves meeting a closed square C_r(c).  It first
// descends from the root along the boxes holding c while the box radius is
// at least 2r, stopping at the first box b with |b|/2 < r <= |b| or where no
// child holds c: the guiding box.  Its peers (Sec. 5 definition: adjacent,
// at least as large, and finest such) cover the 3 x 3 block of cells of b's
// level around it, which holds C_r(c) because c lies in b and r <= |b|.
// The leaves below the peers are then tested against the square.
//
// Peers are found per cell of that block: the finest box of level <= l(b)
// holding the cell.  The tree leaves out children without points, so the
// descent to a cell can stop at a box that has children but none on the
// cell's side; that quadrant holds no leaf (an area query skips it) and is
// kept as a region of its own for association lists.  No peer is then an
// ancestor of another, so every leaf is visited at most once.
#include "areaquery.hpp"

#include <cmath>

namespace qbx {
namespace {

// DFS stack: at most 9 peers, then at most 3 pending siblings per level
// below them (31 levels at most).
constexpr int kAqStack = 128;
// Relative margin of the subtree pruning test, so that rounding in the
// stored box centres never cuts off a leaf that meets the square.
constexpr double kAqSlack = 1e-12;

__device__ __forceinline__ double aq_rad(const AQTree &t, int l) { return ldexp(t.R0, -l); }

// The closed box of centre (mx, my) and radius rb meets C_r(c).
__device__ __forceinline__ bool aq_meets(double mx, double my, double rb, double cx, double cy, double r)
{
    double lim = r + rb;
    return fabs(mx - cx) <= lim && fabs(my - cy) <= lim;
}

__device__ __forceinline__ bool aq_may_meet(double mx, double my, double rb, double cx, double cy, double r)
{
    double lim = (r + rb) * (1.0 + kAqSlack);
    return fabs(mx - cx) <= lim && fabs(my - cy) <= lim;
}

struct Guide {
    int b, l, ix, iy;     // box, level, integer position at that level
};

__device__ Guide aq_guide(const AQTree &t, double cx, double cy, double r)
{
    Guide gd{0, 0, 0, 0};
    // a centre outside the root square: the root guides, so all its leaves
    // are examined (the paper takes c in the root)
    if (!(fabs(cx - t.bcx[0]) <= t.R0 && fabs(cy - t.bcy[0]) <= t.R0)) return gd;
    // r > |b0| stops at the root as well: descending could only shrink b
    while (!(r > 0.5 * aq_rad(t, gd.l)) && !t.leaf[gd.b]) {
        int qx = cx >= t.bcx[gd.b], qy = cy >= t.bcy[gd.b];
        int c = t.child4[4 * gd.b + qx + 2 * qy];
        if (c < 0) break;
        gd.b = c;
        gd.ix = 2 * gd.ix + qx;
        gd.iy = 2 * gd.iy + qy;
        ++gd.l;
    }
    return gd;
}

// Calls emit(key, b) for every leaf b meeting C_r(c) (key 5b + 4) and, with
// regions, emit(key, -1) for every empty quadrant (key 5b + q) meeting it.
template <class F>
__device__ void aq_visit(const AQTree &t, double cx, double cy, double r, bool regions, int *err, F emit)
{
    Guide gd = aq_guide(t, cx, cy, r);
    int stack[kAqStack];
    int sp = 0;
    int seen[9];
    int nseen = 0;
    int n = 1 << gd.l;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            int jx = gd.ix + dx, jy = gd.iy + dy;
            if (jx < 0 || jy < 0 || jx >= n || jy >= n) continue;
            int pb = 0, key = -1;
            for (int k = 0; k < gd.l; ++k) {
                int sh = gd.l - 1 - k;
                int q = ((jx >> sh) & 1) | (((jy >> sh) & 1) << 1);
                int c = t.child4[4 * pb + q];
                if (c < 0) {
                    if (!t.leaf[pb]) key = kAqKeysPerBox * pb + q;
                    break;
                }
                pb = c;
            }
            if (key < 0) key = kAqKeysPerBox * pb + 4;     // a box of level l(b), or a coarser leaf
            bool dup = false;
            for (int i = 0; i < nseen; ++i) dup |= seen[i] == key;
            if (dup) continue;
            seen[nseen++] = key;
            if (key % kAqKeysPerBox == 4) {
                stack[sp++] = pb;
            } else if (regions) {
                int q = key % kAqKeysPerBox;
                double h = 0.5 * aq_rad(t, t.blev[pb]);
                if (aq_may_meet(t.bcx[pb] + ((q & 1) ? h : -h), t.bcy[pb] + ((q & 2) ? h : -h), h, cx, cy, r))
                    emit(key, -1);
            }
        }
    while (sp > 0) {
        int b = stack[--sp];
        double rb = aq_rad(t, t.blev[b]);
        if (t.leaf[b]) {
            if (regions ? aq_may_meet(t.bcx[b], t.bcy[b], rb, cx, cy, r)
                        : aq_meets(t.bcx[b], t.bcy[b], rb, cx, cy, r))
                emit(kAqKeysPerBox * b + 4, b);
            continue;
        }
        if (!aq_may_meet(t.bcx[b], t.bcy[b], rb, cx, cy, r)) continue;
        double h = 0.5 * rb;
        for (int q = 3; q >= 0; --q) {
            int c = t.child4[4 * b + q];
            if (c >= 0) {
                if (sp == kAqStack) {          // cannot happen within 31 levels; reported, not dropped silently
                    atomicOr(err, 1);
                    return;
                }
                stack[sp++] = c;
            } else if (regions &&
                       aq_may_meet(t.bcx[b] + ((q & 1) ? h : -h), t.bcy[b] + ((q & 2) ? h : -h), h, cx, cy, r)) {
                emit(kAqKeysPerBox * b + q, -1);
            }
        }
    }
}

__global__ void k_area_query(AQTree t, int64_t n, const double *qx, const double *qy, const double *qr,
                             int32_t *cnt, const int64_t *start, int32_t *list, int *err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = qr[i];
    int32_t c = 0;
    if (r >= 0.0) {                             // negative or NaN radius: empty square
        int32_t *dst = list ? list + start[i] : nullptr;
        aq_visit(t, qx[i], qy[i], r, false, err, [&](int, int b) {
            if (dst) dst[c] = b;
            ++c;
        });
    }
    if (!list) cnt[i] = c;
}

__global__ void k_region_lists(AQTree t, int64_t n, const double *x, const double *y, const double *rad,
                               double scale, int32_t *kcnt, const int64_t *kstart, int32_t *kcur,
                               int32_t *list, int *err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = rad[i] * scale;
    if (!(r >= 0.0)) return;
    aq_visit(t, x[i], y[i], r, true, err, [&](int key, int) {
        if (!list) atomicAdd(&kcnt[key], 1);
        else list[kstart[key] + atomicAdd(&kcur[key], 1)] = (int32_t)i;
    });
}

// A point of the disk lies in the square and so in a leaf meeting it.  The
// leaves are taken with the widened test (the traversal's region mode, whose
// empty quadrants hold no points and are skipped), so that rounding in the
// stored box centres cannot drop a point on a leaf's edge; the point test
// itself is exact.
__global__ void k_points_near(AQTree t, int64_t n, const double *qx, const double *qy, const double *qr,
                              const int *pbeg, const int *pend, const double *px, const double *py,
                              int32_t *hit, int *err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = qx[i], y = qy[i], r = qr[i];
    int32_t h = 0;
    if (r >= 0.0) {
        double r2 = r * r;
        aq_visit(t, x, y, r, true, err, [&](int, int b) {
            if (b < 0) return;
            for (int k = pbeg[b]; k < pend[b] && !h; ++k) {
                double dx = px[k] - x, dy = py[k] - y;
                if (dx * dx + dy * dy <= r2) h = 1;
            }
        });
    }
    hit[i] = h;
}

// Region (key) holding the point clamped to the root square.  A square
// about a point of the root that holds the target holds the clamped point
// too, so the region's list has every candidate of the target.
__device__ int aq_region_of(const AQTree &t, double x, double y)
{
    x = fmin(fmax(x, t.bcx[0] - t.R0), t.bcx[0] + t.R0);
    y = fmin(fmax(y, t.bcy[0] - t.R0), t.bcy[0] + t.R0);
    int b = 0;
    while (!t.leaf[b]) {
        int q = (x >= t.bcx[b]) | ((y >= t.bcy[b]) << 1);
        int c = t.child4[4 * b + q];
        if (c < 0) return kAqKeysPerBox * b + q;
        b = c;
    }
    return kAqKeysPerBox * b + 4;
}

__global__ void k_associate(AQTree t, AQAssoc a, int64_t n, const double *tx, const double *ty, int32_t *out,
                            unsigned long long *nfail)
{
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double x = tx[m], y = ty[m];
    int key = aq_region_of(t, x, y);
    // the host planner's rule, with its roundings (no contraction here)
    int best = -1;
    double bestd = 0.0;
    for (int64_t e = a.cstart[key]; e < a.cstart[key + 1]; ++e) {
        int k = a.clist[e];
        double dx = x - a.cx[k], dy = y - a.cy[k];
        double d2 = dx * dx + dy * dy;
        double lim = a.cr[k] * (1.0 + a.ea);
        int u = a.ctr_user[k];
        if (d2 <= lim * lim && (best < 0 || d2 < bestd || (d2 == bestd && u < best))) {
            best = u;
            bestd = d2;
        }
    }
    out[m] = best;
    if (best >= 0) return;
    bool near = false;
    for (int64_t e = a.sstart[key]; e < a.sstart[key + 1]; ++e) {
        int j = a.slist[e];
        double dx = x - a.sx[j], dy = y - a.sy[j];
        double q = 0.25 * a.sh[j];
        if (dx * dx + dy * dy <= q * q) near = true;
    }
    if (near) atomicAdd(nfail, 1ull);
}

constexpr int kAqThreads = 256;

unsigned aq_blocks(int64_t n) { return (unsigned)((n + kAqThreads - 1) / kAqThreads); }

}  // namespace

hipError_t launch_area_query(const AQTree &t, int64_t n, const double *qx, const double *qy,
                             const double *qr, int32_t *cnt, const int64_t *start, int32_t *list,
                             int *err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_area_query<<<aq_blocks(n), kAqThreads, 0, s>>>(t, n, qx, qy, qr, cnt, start, list, err);
    return hipGetLastError();
}

hipError_t launch_region_lists(const AQTree &t, int64_t n, const double *x, const double *y,
                               const double *rad, double scale, int32_t *kcnt,
                               const int64_t *kstart, int32_t *kcur, int32_t *list, int *err,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_region_lists<<<aq_blocks(n), kAqThreads, 0, s>>>(t, n, x, y, rad, scale, kcnt, kstart, kcur, list, err);
    return hipGetLastError();
}

hipError_t launch_points_near(const AQTree &t, int64_t n, const double *qx, const double *qy,
                              const double *qr, const int *pbeg, const int *pend, const double *px,
                              const double *py, int32_t *hit, int *err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_points_near<<<aq_blocks(n), kAqThreads, 0, s>>>(t, n, qx, qy, qr, pbeg, pend, px, py, hit, err);
    return hipGetLastError();
}

hipError_t launch_associate(const AQTree &t, const AQAssoc &a, int64_t n, const double *tx,
                            const double *ty, int32_t *out, unsigned long long *nfail,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_associate<<<aq_blocks(n), kAqThreads, 0, s>>>(t, a, n, tx, ty, out, nfail);
    return hipGetLastError();
}

}  // namespace qbx
