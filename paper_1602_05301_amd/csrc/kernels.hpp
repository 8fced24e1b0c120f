// Device-side view of a resident geometry and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "devmath.hpp"

namespace qbx {

// Pointers into device memory.  In the kernels' device code they carry the
// global address space, as a kernel's own pointer arguments do, also when
// the view is read from memory (fused launches): loads through them stay
// scalar or global, never flat.  Host code sees plain pointers; the layout
// is the same.
#if defined(__HIP_DEVICE_COMPILE__) && defined(QBX_KERNELS_TU)
#define QBX_G __attribute__((address_space(1)))
#else
#define QBX_G
#endif

// All pointers are device pointers.  Points are in tree (Morton) order.
struct DevGeom {
    int ns, nc, nt, nb, nlev, p, n_smooth;
    int max_leaf_ctr;                          // most centres in one leaf
    double omega;
    const QBX_G double *sx, *sy, *sw, *snx, *sny;   // sorted sources
    const QBX_G int *src_perm;                       // sorted -> user source index
    const QBX_G double *cx, *cy;                     // sorted centres
    const QBX_G int *ctr_perm;                       // sorted -> user centre index
    const QBX_G double *tx, *ty;                     // targets, user order
    const QBX_G int *tgt_cs;                         // per target: sorted centre or -1
    const QBX_G int *smooth_list;                    // targets served by the smooth rule
    // where the evaluation writes: u[d * u_stride + tgt_out[m]] (tgt_out null:
    // the target's own index m); a geometry that serves some targets of
    // another writes into that one's output
    const QBX_G int *tgt_out;
    long long u_stride;
    const QBX_G double *bcx, *bcy;                   // box centres
    const QBX_G int *blev, *leaf, *parent, *child_begin, *child_count;
    const QBX_G int *src_begin, *src_end, *ctr_begin, *ctr_end;
    const QBX_G int *level_start;
    const QBX_G int *U_start, *U_idx, *V_start, *V_idx, *V_off, *W_start, *W_idx, *X_start, *X_idx;
    // near list of a leaf = U list + W boxes summed directly; far W = the rest
    const QBX_G int *near_start, *near_idx, *wf_start, *wf_idx;
    // near-list sources of the leaves with centres, one run per leaf; a
    // P2QBXL work item names its leaf's run
    const QBX_G int *qsrc_idx;
    // X-list sources of the i-th box of the X-list P2L list: xsrc_idx[xsrc_start[i]..]
    const QBX_G int *xsrc_start, *xsrc_idx;
    const QBX_G int *src_box, *ctr_box;              // leaf (level >= 2) of each source / centre, or -1
    // Geometry-only bases, built on the first evaluation and kept: the P2M
    // row of every source in a leaf b of level >= 2, L_n(s - m_b) for
    // n = 0..P_b+1 at sbas[s * srow + n]; the X-list P2L row of every
    // flattened X-list position q (source xsrc_idx[q] for box xsrc_box[q]),
    // S_n O_n(s - m_b) for n = -(P_b+1)..P_b+1 at xbas[xbas_off[q] + P_b+1 + n]
    // (rows of 2 P_b + 3; the positions of one box are consecutive rows).
    // xbas is null when too large to keep: rows are then built in every
    // evaluation.
    const QBX_G cd *sbas, *xbas;
    const QBX_G int *xsrc_box;
    const QBX_G long long *xbas_off;
    int srow;
    const QBX_G int *Plev;                           // FMM order per level
    const QBX_G int *Woff;                           // per level offset into Wtab/invW/logW
    const QBX_G double *Wtab, *invW, *logW;
    const QBX_G long long *box_off;                  // per box, in coefficients of one density
    // M2M / L2L scaled matrices per (parent level, child quadrant) in MFMA
    // A-operand order; child4[b*4+q] = child of b in quadrant q or -1
    const QBX_G cd *m2m_mf, *l2l_mf;
    const QBX_G long long *m2m_mf_off, *l2l_mf_off;  // [level*4+q]
    const QBX_G int *child4;
    // per position of the M2M parent list: children's box_off by quadrant
    // (-1 = none) and the parent's; per position of the L2L child list: the
    // parent's and the child's box_off, the vy row of its first V-list entry
    // and the entry count (the entries' rows follow each other)
    const QBX_G long long *m2m_coff, *m2m_poff;
    const QBX_G long long *l2l_poff, *l2l_coff, *l2l_vy0;
    const QBX_G int *l2l_nv;
    // M2L as batched GEMM: per (level, offset) matrices in MFMA tile order,
    // V-list positions grouped by (level, offset), per-position output offsets.
    const QBX_G cd *m2l_mf;                          // tiled scaled M2L matrices
    // FP32 far field (eps >= 1e-6): M2L and L2L tables in complex float, same
    // tile order and offsets as the FP64 ones; null when off
    int far32;
    const QBX_G cf *m2l_mf32, *l2l_mf32;
    const QBX_G long long *m2l_mf_off;               // [level*40+o]
    const QBX_G int *vpair_sorted;                   // V-list positions sorted by (level, offset)
    const QBX_G long long *vy_off;                   // per V-list position: output row offset
    const QBX_G long long *m2l_src, *m2l_dst;        // per sorted position: box_off of the source, vy_off
    // per sorted position: r with offset = R^r (group's offset), R the
    // rotation by 90 degrees; the pair's matrix is diag(i^{rj}) M diag(i^{rk})
    const QBX_G int *m2l_rot;
};

// Block index of a workgroup within one geometry's part of a launch: x
// fastest, y above it, nx = blocks along x.  A single-geometry launch passes
// (blockIdx.x, blockIdx.y, gridDim.x).
struct BlockId {
    int x, y, nx;
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

// ---------------------------------------------------------------------------
// Fused launches: one grid per stage over several geometries.  The grid is
// the concatenation of each geometry's own grid for the stage; map[block]
// names the record of the geometry a block belongs to, and the record holds
// that geometry's arguments and its first block.  A block then runs the same
// body as in the geometry's own launch, with its local block index, so each
// geometry's results are bitwise those of its own launch.
// ---------------------------------------------------------------------------
struct FRec {
    const DevGeom *g;          // device copy of the geometry's view
    int first, nx;             // first block of the geometry in the grid; its blocks along x
    int nd, i0;                // densities per column; a stage integer (level, pass size, ...)
    long long n64;             // a count (fill)
    const QBX_G void *in0, *in1, *in2, *in3;
    QBX_G void *out0, *out1;
};

enum FKind {
    FK_FILL, FK_CHARGES, FK_SRC_BAS, FK_X_BAS, FK_CTR_RAD, FK_P2M, FK_M2M, FK_M2L, FK_DOWN, FK_L2L, FK_P2L_X,
    FK_P2QBXL, FK_P2QBXL_DIRECT, FK_M2QBXL, FK_WSUM, FK_L2QBXL, FK_EVAL, FK_SMOOTH,
    // chosen by the planner
    FK_M2L_DIRECT, FK_M2L32, FK_L2L32, FK_P2L_XC
};

// One geometry's part of a stage, as the host describes it.  The record's
// g, nd, i0, in*, out* are the stage's arguments (their meaning per stage is
// listed at fused_plan); n, P and aux size the geometry's grid.
struct FItem {
    const DevGeom *h;          // host copy of the geometry's view
    FRec r;
    long long n;               // work items (boxes, tiles, pairs, elements)
    int P;                     // largest expansion order involved
    int aux;                   // row blocks (M2M, L2L), waves per tile (M2L), J_n rows (L2QBXL)
    int split = 0;             // M2L: leading tiles whose order needs the direct kernel
    int Psplit = 0;            // M2L: largest order among those tiles (P: the others)
};

struct FLaunch {
    int kind, variant, threads, nblocks;
    size_t lds, rec_off, map_off;
};

// Records and block maps of a set of fused launches, uploaded in one copy.
struct FBuf {
    std::vector<unsigned char> bytes;
    std::vector<FLaunch> launches;
};

// Appends the launches of one stage (one per kernel variant the items need,
// none if they have no work) and their indices to ids.
hipError_t fused_plan(FBuf &fb, int kind, const std::vector<FItem> &items, std::vector<int> &ids);
// Launches fb.launches[i] with its records at dev (the device copy of fb.bytes).
hipError_t fused_launch(const FLaunch &L, const unsigned char *dev, hipStream_t s);

hipError_t launch_fill_zero(cd *p, long long n, hipStream_t s);
hipError_t launch_charges(const DevGeom &g, int nd, const cd *ss, const cd *sd, cd *qs, cd *qd,
                          hipStream_t s);
// The geometry-only bases of P2M (into sbas, g.srow per source) and of the
// X-list P2L (into xbas, rows at g.xbas_off; nx flattened positions).
hipError_t launch_src_bas(const DevGeom &g, cd *sbas, hipStream_t s);
hipError_t launch_x_bas(const DevGeom &g, int nx, cd *xbas, hipStream_t s);
hipError_t launch_p2m(const DevGeom &g, int nd, const int *list, int n, int Pmax, const cd *qs,
                      const cd *qd, cd *mp, hipStream_t s);
hipError_t launch_m2m_mfma(const DevGeom &g, int nd, int l, const TTile *tiles, int ntiles,
                           int nrb, const int *plist, cd *mp, hipStream_t s);
// vy = null: the children's V-list rows are already summed into loc
hipError_t launch_l2l_mfma(const DevGeom &g, int nd, int L, const TTile *tiles, int ntiles, int nrb,
                           const int *clist, const cd *vy, cd *loc, hipStream_t s);
// nw > 0: columns staged in LDS, nw waves per tile (row blocks spread over
// them); nw = 0: one wave per (tile, row block) with operands straight from
// memory.  Same sums, same order.  The first nsplit tiles (orders up to
// Pdirect) have columns beyond the LDS budget and always take the direct
// kernel; the rest have orders up to Pstaged <= m2l_staged_pmax().
hipError_t launch_m2l_mfma(const DevGeom &g, int nd, const M2LTile *tiles, int ntiles, int nsplit,
                           int Pdirect, int Pstaged, int nw, const cd *mp, cd *vy, hipStream_t s);
// Largest order whose M2L columns the staged kernel holds in LDS.
int m2l_staged_pmax();
// V-list sums of the nbox boxes from the first of level 2 on (every level
// >= 2) in one launch, nd (1-4) densities; launch_l2l_mfma with vy = null
// then leaves them out of its epilogue.
hipError_t launch_down_all(const DevGeom &g, int nd, int nbox, const cd *vy, cd *loc, hipStream_t s);
// X-list P2L into the locals of the listed boxes.  beside: the launch runs
// concurrently with the other stream's chain (a short launch is then capped
// so that the chain's launches find room on every CU).
hipError_t launch_p2l_x(const DevGeom &g, int nd, const int *list, int n, int Pmax, const cd *qs,
                        const cd *qd, cd *loc, bool beside, hipStream_t s);
// P2QBXL: one workgroup of P2Q_THREADS lanes per work item.  An item is
// four ints {c0, c1, q0, q1}: centres [c0, c1) of one leaf (sorted order) and
// that leaf's near-list sources qsrc_idx[q0, q1).  The lanes form
// CG = min(c1 - c0, P2Q_THREADS / 2) centre slots of P2Q_THREADS / CG parts.
constexpr int P2Q_THREADS = 128;
// beside: the launch runs concurrently with the other stream's chain (its
// grid is then capped so that the chain's launches find room on every CU)
hipError_t launch_p2qbxl(const DevGeom &g, int nd, const int *items, int n, const cd *qs,
                         const cd *qd, cd *coef, bool beside, hipStream_t s);
hipError_t launch_p2qbxl_direct(const DevGeom &g, int nd, const cd *qs, const cd *qd, cd *coef,
                                hipStream_t s);
hipError_t launch_m2qbxl(const DevGeom &g, int nd, const int2 *pairs, const long long *pair_off,
                         int npairs, int PWmax, const cd *mp, cd *wy, const int *leaf_list,
                         const int *leaf_pair_start, int nleaf, cd *coef, hipStream_t s);
// J_n sequences of the L2QBXL centres (leaves of level >= 2), into crad
hipError_t launch_ctr_rad(const DevGeom &g, int nleaf, double *crad, int crad_rows, hipStream_t s);
// L2QBXL work items: L2Q_SEGS runs {c0, c1} of consecutive centres, each run
// inside one leaf of level >= 2 (c0 == c1: unused), at most `cap` centres in
// all.  l2qbxl_item_cap gives the largest cap (<= L2Q_CAP_MAX) whose staging
// fits the LDS budget for leaves of order up to Pmax and J_n rows of `rows`.
constexpr int L2Q_SEGS = 4;
constexpr int L2Q_CAP_MAX = 16;
int l2qbxl_item_cap(int Pmax, int rows);
hipError_t launch_l2qbxl(const DevGeom &g, int nd, const int *items, int n, int Pmax, double *crad,
                         int crad_rows, int cap, const cd *loc, cd *coef, hipStream_t s);
hipError_t launch_qbx_eval(const DevGeom &g, int nd, const cd *coef, cd *u, hipStream_t s);
hipError_t launch_smooth(const DevGeom &g, int nd, const cd *qs, const cd *qd, cd *u, hipStream_t s);
hipError_t launch_coef_out(const DevGeom &g, int nd, const cd *coef, cd *out, hipStream_t s);

}  // namespace qbx
