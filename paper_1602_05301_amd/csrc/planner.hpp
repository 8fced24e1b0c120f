// Host-side planning for FMM-accelerated Global QBX: quadtree, interaction
// lists, per-level expansion orders, target association and the scaled
// translation matrices that the device kernels consume.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qbxfmm.h"

namespace qbx {

constexpr int kMaxLevel = 30;     // Morton coordinates carry 30 bits per axis
constexpr int kMaxP = 40;         // QBX order limit
constexpr int kMaxOrder = 1024;   // FMM order limit
constexpr int kNumV = 40;         // V-list offsets: [-3,3]^2 minus [-1,1]^2

struct Error {
    qbx_status status;
    std::string msg;
};

// Index of a V-list offset (dx, dy) in [-3,3]^2 \ [-1,1]^2, in 0..39.
int v_offset_id(int dx, int dy);
void v_offset_from_id(int id, int *dx, int *dy);

struct Plan {
    // ---- inputs ----
    double omega = 0, eps = 0;
    qbx_options opt{};
    int64_t ns = 0, nc = 0, nt = 0;
    std::vector<double> sx, sy, w, nx, ny, sh, cx, cy, cr, tx, ty;

    // ---- tree (boxes in (level, Morton) order) ----
    double R0 = 0;                       // root radius |b0|
    int nlev = 0;                        // levels 0..nlev-1
    std::vector<int64_t> src_order;      // sorted position -> user source index
    std::vector<int64_t> ctr_order;      // sorted position -> user centre index
    std::vector<int32_t> lev, bix, biy, parent, leaf, child_begin, child_count;
    std::vector<int32_t> src_begin, src_end, ctr_begin, ctr_end;
    std::vector<int32_t> level_start;    // boxes of level l: [level_start[l], level_start[l+1])
    std::vector<int32_t> colleagues;     // 9 per box, -1 padded

    // ---- lists, CSR ----
    std::vector<int32_t> U_start, U_idx, V_start, V_idx, V_off, W_start, W_idx, X_start, X_idx;

    // ---- orders ----
    int p = 0, p_add = 0;
    std::vector<int32_t> P;              // per level
    std::vector<int32_t> pfmm;           // per level, before p_add

    // ---- association (user numbering) ----
    std::vector<int32_t> tgt_ctr;        // centre per target or -1

    int n_boxes() const { return (int)lev.size(); }
    double box_radius(int level) const;
    void box_center(int b, double *x, double *y) const;
};

// Validates inputs, builds tree, lists, orders and association.
Error build_plan(Plan &pl, double omega, double eps, const qbx_options &opt, int64_t ns,
                 const double *sx, const double *sy, const double *w, const double *nx,
                 const double *ny, const double *sh, int64_t nc, const double *cx,
                 const double *cy, const double *cr, int64_t nt, const double *tx,
                 const double *ty, const int32_t *tgt_ctr);

int default_p_add(int p, double eps);
int fmm_order(double omega, double R, double eps);

// Per-level scale factors W_k = min(1, sigma^k / k!), sigma = omega R_l / sqrt(2),
// k = 0..P_l.  Multipoles are stored as a_k / W_|k| and locals as g_k W_|k|.
std::vector<double> level_scales(double omega, double R, int P);

// Scaled translation matrices (row-major [out][in], complex<double>).
// M2M: child (level l+1, quadrant q) -> parent (level l).
std::vector<std::complex<double>> m2m_matrix(const Plan &pl, int l, int quadrant);
// L2L: parent (level l) -> child (level l+1, quadrant q).
std::vector<std::complex<double>> l2l_matrix(const Plan &pl, int l, int quadrant);
// M2L at level l for source box offset (dx, dy) (in box sides) from the target box.
std::vector<std::complex<double>> m2l_matrix(const Plan &pl, int l, int dx, int dy);

}  // namespace qbx
