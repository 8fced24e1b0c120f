// Host-only part of the C ABI: options, errors and planning queries.
#include <algorithm>
#include <cstring>
#include <new>

#include "abi_common.hpp"

namespace qbx {

static thread_local std::string g_last_error;
static thread_local unsigned long long g_error_seq = 0;

void set_error(const std::string &msg)
{
    g_last_error = msg;
    ++g_error_seq;
}

std::string error_msg() { return g_last_error; }

unsigned long long error_seq() { return g_error_seq; }

qbx_status fail(qbx_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

void fill_stats(const Plan &pl, qbx_stats *out)
{
    std::memset(out, 0, sizeof(*out));
    out->n_src = pl.ns;
    out->n_ctr = pl.nc;
    out->n_tgt = pl.nt;
    out->n_levels = pl.nlev;
    out->n_boxes = pl.n_boxes();
    out->p = pl.p;
    out->p_add = pl.p_add;
    out->root_radius = pl.R0;
    int nb = pl.n_boxes();
    for (int b = 0; b < nb; ++b) {
        out->n_leaves += pl.leaf[b];
        int nct = pl.ctr_end[b] - pl.ctr_begin[b];
        for (int i = pl.U_start[b]; i < pl.U_start[b + 1]; ++i) {
            int c = pl.U_idx[i];
            out->n_p2qbxl_pairs += (int64_t)nct * (pl.src_end[c] - pl.src_begin[c]);
        }
        out->n_m2qbxl_pairs += (int64_t)nct * (pl.W_start[b + 1] - pl.W_start[b]);
        for (int i = pl.X_start[b]; i < pl.X_start[b + 1]; ++i) {
            int c = pl.X_idx[i];
            out->n_x_src_pairs += pl.src_end[c] - pl.src_begin[c];
        }
    }
    out->n_u_pairs = pl.U_idx.size();
    out->n_v_pairs = pl.V_idx.size();
    out->n_w_pairs = pl.W_idx.size();
    out->n_x_pairs = pl.X_idx.size();
    for (int64_t m = 0; m < pl.nt; ++m) out->n_smooth_targets += pl.tgt_ctr[m] < 0;
}

}  // namespace qbx

using namespace qbx;

extern "C" {

int32_t qbx_abi_version(void) { return QBX_ABI_VERSION; }

const char *qbx_last_error(void)
{
    static thread_local std::string copy;
    copy = g_last_error;
    return copy.c_str();
}

void qbx_options_default(qbx_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->p = 12;
    opt->p_add = -1;
    opt->leaf_max = 32;
    opt->direct = 0;
    opt->far_fp32 = 0;
    opt->w_direct = -1;
    opt->level_restrict = 1;
    opt->keep_x_rows = 1;
    opt->eps_assoc = 0.05;
}

qbx_status qbx_plan_create(double omega, double eps, const qbx_options *opt, int64_t n_src,
                           const double *sx, const double *sy, const double *w,
                           const double *nx, const double *ny, const double *sh,
                           int64_t n_ctr, const double *cx, const double *cy,
                           const double *cr, int64_t n_tgt, const double *tx,
                           const double *ty, const int32_t *tgt_ctr, qbx_plan *out)
{
    if (!out) return fail(QBX_E_INVAL, "out is NULL");
    *out = nullptr;
    qbx_options o;
    if (opt) o = *opt;
    else qbx_options_default(&o);
    try {
        auto *p = new qbx_plan_s();
        Error e = build_plan(p->pl, omega, eps, o, n_src, sx, sy, w, nx, ny, sh, n_ctr, cx, cy,
                             cr, n_tgt, tx, ty, tgt_ctr);
        if (e.status != QBX_OK) {
            delete p;
            return fail(e.status, e.msg);
        }
        *out = p;
        return QBX_OK;
    } catch (const std::bad_alloc &) {
        return fail(QBX_E_NOMEM, "host allocation failed while planning");
    } catch (...) {
        return fail(QBX_E_INVAL, "unexpected exception while planning");
    }
}

qbx_status qbx_plan_destroy(qbx_plan plan)
{
    delete plan;
    return QBX_OK;
}

qbx_status qbx_plan_stats(qbx_plan plan, qbx_stats *out)
{
    if (!plan || !out) return fail(QBX_E_INVAL, "null argument");
    fill_stats(plan->pl, out);
    return QBX_OK;
}

qbx_status qbx_plan_boxes(qbx_plan plan, int32_t *level, int32_t *ix, int32_t *iy,
                          int32_t *parent, int32_t *leaf, int32_t *n_src_in, int32_t *n_ctr_in)
{
    if (!plan) return fail(QBX_E_INVAL, "null plan");
    const Plan &pl = plan->pl;
    int nb = pl.n_boxes();
    for (int b = 0; b < nb; ++b) {
        if (level) level[b] = pl.lev[b];
        if (ix) ix[b] = pl.bix[b];
        if (iy) iy[b] = pl.biy[b];
        if (parent) parent[b] = pl.parent[b];
        if (leaf) leaf[b] = pl.leaf[b];
        if (n_src_in) n_src_in[b] = pl.src_end[b] - pl.src_begin[b];
        if (n_ctr_in) n_ctr_in[b] = pl.ctr_end[b] - pl.ctr_begin[b];
    }
    return QBX_OK;
}

qbx_status qbx_plan_list(qbx_plan plan, int32_t which, int32_t *start, int32_t *idx)
{
    if (!plan || !start) return fail(QBX_E_INVAL, "null argument");
    const Plan &pl = plan->pl;
    const std::vector<int32_t> *s = nullptr, *v = nullptr;
    switch (which) {
    case QBX_LIST_U: s = &pl.U_start; v = &pl.U_idx; break;
    case QBX_LIST_V: s = &pl.V_start; v = &pl.V_idx; break;
    case QBX_LIST_W: s = &pl.W_start; v = &pl.W_idx; break;
    case QBX_LIST_X: s = &pl.X_start; v = &pl.X_idx; break;
    default: return fail(QBX_E_INVAL, "unknown list");
    }
    std::copy(s->begin(), s->end(), start);
    if (idx) std::copy(v->begin(), v->end(), idx);
    return QBX_OK;
}

qbx_status qbx_plan_orders(qbx_plan plan, int32_t *P)
{
    if (!plan || !P) return fail(QBX_E_INVAL, "null argument");
    std::copy(plan->pl.P.begin(), plan->pl.P.end(), P);
    return QBX_OK;
}

qbx_status qbx_plan_association(qbx_plan plan, int32_t *tgt_ctr_out)
{
    if (!plan || (!tgt_ctr_out && plan->pl.nt)) return fail(QBX_E_INVAL, "null argument");
    std::copy(plan->pl.tgt_ctr.begin(), plan->pl.tgt_ctr.end(), tgt_ctr_out);
    return QBX_OK;
}

}  // extern "C"
