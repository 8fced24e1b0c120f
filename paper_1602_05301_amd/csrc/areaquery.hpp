// Area queries on the resident quad-tree (Sec. 5: area query, peer boxes,
// the guiding-box algorithm) and target association through them (Sec. 6.1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qbx {

// The tree as the area queries read it (device pointers, boxes in the
// plan's (level, Morton) numbering).  Box b at level l is the closed square
// of radius R0 2^-l about (bcx[b], bcy[b]); child4[4b + q] is its child in
// quadrant q = qx + 2 qy (qx = 1 on the side of larger x) or -1.
struct AQTree {
    const double *bcx, *bcy;
    const int *blev, *leaf, *child4;
    double R0;
};

// Result lists are keyed by region: 5b + 4 for leaf b, 5b + q for the empty
// quadrant q of a box b that has children (the tree leaves out children
// without points, so such a quadrant belongs to no leaf).
constexpr int kAqKeysPerBox = 5;

// Area queries for n squares C_r(c), c = (qx[i], qy[i]), r = qr[i].
// count pass (list == nullptr): cnt[i] = number of leaves met;
// fill pass: the leaves of query i go to list[start[i] ..], in the order the
// query enumerates them.
// *err is set (atomic or) if a traversal would outgrow its stack, which the
// depth limit of the tree rules out.
hipError_t launch_area_query(const AQTree &t, int64_t n, const double *qx, const double *qy,
                             const double *qr, int32_t *cnt, const int64_t *start, int32_t *list,
                             int *err, hipStream_t s);

// Inverted lists for association: every point i (x, y) with square radius
// rad[i] * scale is entered in the list of each region (leaf or empty
// quadrant, keyed as above) its square meets.  count pass (list == nullptr):
// kcnt[key] += 1 (atomic); fill pass: list[kstart[key] + slot] = i with the
// slot taken from kcur[key] (atomic; order within a key is arbitrary).
hipError_t launch_region_lists(const AQTree &t, int64_t n, const double *x, const double *y,
                               const double *rad, double scale, int32_t *kcnt,
                               const int64_t *kstart, int32_t *kcur, int32_t *list, int *err,
                               hipStream_t s);

// Disk tests: hit[i] = 1 if one of the points (px, py) lies within
// distance qr[i] of (qx[i], qy[i]), else 0.  The points are the tree's
// sources or centres in tree order, those of box b at [pbeg[b], pend[b]);
// only the leaves an area query over the disk's bounding square returns are
// scanned.
hipError_t launch_points_near(const AQTree &t, int64_t n, const double *qx, const double *qy,
                              const double *qr, const int *pbeg, const int *pend, const double *px,
                              const double *py, int32_t *hit, int *err, hipStream_t s);

// Association of n targets (device tx, ty) by the rule of the host planner:
// the nearest centre k with |t - c_k|^2 <= (cr_k (1 + ea))^2, ties to the
// lower user index ctr_user[k]; out[m] = that user index or -1.  A target
// with no such centre but within sh_j / 4 of a source j counts in *nfail.
struct AQAssoc {
    const double *cx, *cy, *cr;          // sorted centres and their radii
    const int *ctr_user;                 // sorted -> user centre index
    const double *sx, *sy, *sh;          // sorted sources and their panel lengths
    const int64_t *cstart, *sstart;      // region list offsets (5 nb + 1)
    const int32_t *clist, *slist;        // sorted centre / source indices per region
    double ea;
};
hipError_t launch_associate(const AQTree &t, const AQAssoc &a, int64_t n, const double *tx,
                            const double *ty, int32_t *out, unsigned long long *nfail,
                            hipStream_t s);

}  // namespace qbx
