// Device-side view of a resident geometry and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "devmath.hpp"

namespace qbx {

// All pointers are device pointers.  Points are in tree (Morton) order.
struct DevGeom {
    int ns, nc, nt, nb, nlev, p, n_smooth;
    int max_leaf_ctr;                          // most centres in one leaf
    double omega;
    const double *sx, *sy, *sw, *snx, *sny;   // sorted sources
    const int *src_perm;                       // sorted -> user source index
    const double *cx, *cy;                     // sorted centres
    const int *ctr_perm;                       // sorted -> user centre index
    const double *tx, *ty;                     // targets, user order
    const int *tgt_cs;                         // per target: sorted centre or -1
    const int *smooth_list;                    // targets served by the smooth rule
    const double *bcx, *bcy;                   // box centres
    const int *blev, *leaf, *parent, *child_begin, *child_count;
    const int *src_begin, *src_end, *ctr_begin, *ctr_end;
    const int *level_start;
    const int *U_start, *U_idx, *V_start, *V_idx, *V_off, *W_start, *W_idx, *X_start, *X_idx;
    // near list of a leaf = U list + W boxes summed directly; far W = the rest
    const int *near_start, *near_idx, *wf_start, *wf_idx;
    // near-list sources of the i-th leaf of the P2QBXL list: qsrc_idx[qsrc_start[i]..]
    const int *qsrc_start, *qsrc_idx;
    // X-list sources of the i-th box of the X-list P2L list: xsrc_idx[xsrc_start[i]..]
    const int *xsrc_start, *xsrc_idx;
    const int *src_box, *ctr_box;              // leaf (level >= 2) of each source / centre, or -1
    const int *Plev;                           // FMM order per level
    const int *Woff;                           // per level offset into Wtab/invW/logW
    const double *Wtab, *invW, *logW;
    const long long *box_off;                  // per box, in coefficients of one density
    // M2M / L2L scaled matrices per (parent level, child quadrant) in MFMA
    // A-operand order; child4[b*4+q] = child of b in quadrant q or -1
    const cd *m2m_mf, *l2l_mf;
    const long long *m2m_mf_off, *l2l_mf_off;  // [level*4+q]
    const int *child4;
    // per position of the M2M parent list: children's box_off by quadrant
    // (-1 = none) and the parent's; per position of the L2L child list: the
    // parent's and the child's box_off, the vy row of its first V-list entry
    // and the entry count (the entries' rows follow each other)
    const long long *m2m_coff, *m2m_poff;
    const long long *l2l_poff, *l2l_coff, *l2l_vy0;
    const int *l2l_nv;
    // M2L as batched GEMM: per (level, offset) matrices in MFMA tile order,
    // V-list positions grouped by (level, offset), per-position output offsets.
    const cd *m2l_mf;                          // tiled scaled M2L matrices
    // FP32 far field (eps >= 1e-6): M2L and L2L tables in complex float, same
    // tile order and offsets as the FP64 ones; null when off
    int far32;
    const cf *m2l_mf32, *l2l_mf32;
    const long long *m2l_mf_off;               // [level*40+o]
    const int *vpair_sorted;                   // V-list positions sorted by (level, offset)
    const long long *vy_off;                   // per V-list position: output row offset
    const long long *m2l_src, *m2l_dst;        // per sorted position: box_off of the source, vy_off
};

// One M2M / L2L GEMM tile: up to 16 (box, density) columns taken from a box
// list (parents of one level, or the children of one level in quadrant q).
struct TTile {
    int q;            // child quadrant (L2L)
    int start;        // first position of the list
    int col0;         // first column of the tile
    int ncol;         // columns in this tile (<= 16)
};

// One M2L GEMM tile: up to 16 (pair, density) columns of one (level, offset) group.
struct M2LTile {
    int lo;           // level * 40 + offset id
    int pair_start;   // first position in vpair_sorted of the group
    int col0;         // first column of the tile within the group
    int ncol;         // columns in this tile (<= 16)
};

hipError_t launch_fill_zero(cd *p, long long n, hipStream_t s);
hipError_t launch_charges(const DevGeom &g, int nd, const cd *ss, const cd *sd, cd *qs, cd *qd,
                          hipStream_t s);
hipError_t launch_p2m(const DevGeom &g, int nd, const int *list, int n, int Pmax, const cd *qs,
                      const cd *qd, double *srad, int srad_rows, cd *mp, hipStream_t s);
hipError_t launch_m2m_mfma(const DevGeom &g, int nd, int l, const TTile *tiles, int ntiles,
                           int nrb, const int *plist, cd *mp, hipStream_t s);
hipError_t launch_l2l_mfma(const DevGeom &g, int nd, int L, const TTile *tiles, int ntiles, int nrb,
                           const int *clist, const cd *vy, cd *loc, hipStream_t s);
// nw > 0: columns staged in LDS, nw waves per tile (row blocks spread over
// them); nw = 0 (or staging beyond the LDS budget): one wave per (tile, row
// block) with operands straight from memory.  Same sums, same order.
hipError_t launch_m2l_mfma(const DevGeom &g, int nd, const M2LTile *tiles, int ntiles, int Pmax,
                           int nw, const cd *mp, cd *vy, hipStream_t s);
hipError_t launch_down(const DevGeom &g, int nd, int l, int nbox, const cd *vy, cd *loc,
                       hipStream_t s);
hipError_t launch_p2l_x(const DevGeom &g, int nd, const int *list, int n, int Pmax, const cd *qs,
                        const cd *qd, cd *loc, hipStream_t s);
hipError_t launch_p2qbxl(const DevGeom &g, int nd, const int *list, int n, const cd *qs,
                         const cd *qd, cd *coef, hipStream_t s);
hipError_t launch_p2qbxl_direct(const DevGeom &g, int nd, const cd *qs, const cd *qd, cd *coef,
                                hipStream_t s);
hipError_t launch_m2qbxl(const DevGeom &g, int nd, const int2 *pairs, const long long *pair_off,
                         int npairs, int PWmax, const cd *mp, cd *wy, const int *leaf_list,
                         const int *leaf_pair_start, int nleaf, cd *coef, hipStream_t s);
// J_n sequences of the L2QBXL centres (leaves of level >= 2), into crad
hipError_t launch_ctr_rad(const DevGeom &g, int nleaf, double *crad, int crad_rows, hipStream_t s);
hipError_t launch_l2qbxl(const DevGeom &g, int nd, const int *list, int n, int Pmax, double *crad,
                         int crad_rows, const cd *loc, cd *coef, hipStream_t s);
hipError_t launch_qbx_eval(const DevGeom &g, int nd, const cd *coef, cd *u, hipStream_t s);
hipError_t launch_smooth(const DevGeom &g, int nd, const cd *qs, const cd *qd, cd *u, hipStream_t s);
hipError_t launch_coef_out(const DevGeom &g, int nd, const cd *coef, cd *out, hipStream_t s);

}  // namespace qbx
