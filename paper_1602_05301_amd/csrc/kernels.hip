// gfx950 kernels for FMM-accelerated Global QBX (2D Helmholtz S + D).
//
// Notation (Sec. 7 of the paper, translation formulas derived from Graf's
// addition theorem, Sec. 2.1):
//   O_n(z) = H_n(w|z|) e^{i n arg z},  I_n(z) = J_n(w|z|) e^{i n arg z},
//   L_n(z) = J_n(w|z|) e^{-i n arg z}  (the paper's J-expansion basis).
// Charges: qS = (i/4) w sigma_S, qD = (i/4) w sigma_D; nu = n_x + i n_y.
// Box expansions are stored scaled: multipole a_k / W_|k|, local g_k W_|k|,
// with the per-level W_k = min(1, s^k/k!), s = w R_l / sqrt(2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <vector>

#define QBX_KERNELS_TU
#include "devmath.hpp"
#include "kernels.hpp"

namespace qbx {

// ---------------------------------------------------------------------------
// Utilities
// ---------------------------------------------------------------------------

__device__ __forceinline__ void fill_zero_body(cd *p, long long n, BlockId bid)
{
    long long i = (long long)bid.x * blockDim.x + threadIdx.x;
    long long step = (long long)bid.nx * blockDim.x;
    for (; i < n; i += step) p[i] = mk(0.0, 0.0);
}

__global__ void k_fill_zero(cd *p, long long n)
{
    fill_zero_body(p, n, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// qS[d][j] = (i/4) w_j sigma_S[d][perm[j]] (sorted source order); same for qD.
__device__ __forceinline__ void charges_body(const DevGeom &g, int nd, const cd *sig_s, const cd *sig_d, cd *qs, cd *qd, BlockId bid)
{
    long long idx = (long long)bid.x * blockDim.x + threadIdx.x;
    long long n = (long long)nd * g.ns;
    if (idx >= n) return;
    int d = (int)(idx / g.ns), j = (int)(idx % g.ns);
    int u = g.src_perm[j];
    double s = 0.25 * g.sw[j];
    cd a = sig_s ? sig_s[(long long)d * g.ns + u] : mk(0.0, 0.0);
    cd b = sig_d ? sig_d[(long long)d * g.ns + u] : mk(0.0, 0.0);
    qs[idx] = mk(-s * a.y, s * a.x);
    qd[idx] = mk(-s * b.y, s * b.x);
}

__global__ void k_charges(DevGeom g, int nd, const cd *sig_s, const cd *sig_d, cd *qs, cd *qd)
{
    charges_body(g, nd, sig_s, sig_d, qs, qd, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

constexpr int QBLK = 8;       // l values per lane; the planner keeps P_l >= p + QBLK

// ---------------------------------------------------------------------------
// Radial sequences, one lane per source / centre (so every lane does a
// whole recurrence), written n-major: element n of item i at rad[n * count + i].
//   (k_src_bas, P2M's basis, is built the same way, below)
//   k_ctr_rad: J_n(omega |m_b - c|), n = 0..P_b+p+7, c in such a leaf
// Miller's recurrence rewrites earlier values when it rescales and
// normalises at the end, so it runs in LDS ([rows][lanes]) and each lane
// then copies its own column out.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void src_bas_body(const DevGeom &g, cd *bas, BlockId bid)
{
    extern __shared__ double lds_raw[];
    int lanes = blockDim.x;
    int s = bid.x * lanes + threadIdx.x;
    if (s >= g.ns) return;
    int b = g.src_box[s];
    if (b < 0) return;
    int N = g.Plev[g.blev[b]] + 1;
    double dx = g.sx[s] - g.bcx[b], dy = g.sy[s] - g.bcy[b];
    double r = sqrt(dx * dx + dy * dy);
    double *J = lds_raw + threadIdx.x;
    besselj_seq(g.omega * r, N, J, lanes);
    // L_n = J_n(x) conj(v)^n, the phase from one sincos per run of orders
    double th = r > 0.0 ? atan2(dy, dx) : 0.0;
    cd v = r > 0.0 ? mk(dx / r, dy / r) : mk(1.0, 0.0);
    cd *row = bas + (long long)s * g.srow;
    for (int n0 = 0; n0 <= N; n0 += 8) {
        double sn, cs;
        sincos((double)n0 * th, &sn, &cs);
        cd ph = mk(cs, -sn);
        for (int n = n0; n < n0 + 8 && n <= N; ++n) {
            row[n] = J[n * lanes] * ph;
            ph = ph * conj(v);
        }
    }
}

__global__ void k_src_bas(DevGeom g, cd *bas)
{
    src_bas_body(g, bas, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

__device__ __forceinline__ void ctr_rad_body(const DevGeom &g, int rows, double *rad, BlockId bid)
{
    extern __shared__ double lds_raw[];
    int lanes = blockDim.x;
    int c = bid.x * lanes + threadIdx.x;
    int N = -1;
    if (c < g.nc) {
        int b = g.ctr_box[c];
        if (b >= 0) {
            N = g.Plev[g.blev[b]] + g.p + QBLK - 1;
            double dx = g.bcx[b] - g.cx[c], dy = g.bcy[b] - g.cy[c];
            besselj_seq(g.omega * sqrt(dx * dx + dy * dy), N, lds_raw + threadIdx.x, lanes);
        }
    }
    (void)rows;
    for (int n = 0; n <= N; ++n) rad[(long long)n * g.nc + c] = lds_raw[n * lanes + threadIdx.x];
}

__global__ void k_ctr_rad(DevGeom g, int rows, double *rad)
{
    ctr_rad_body(g, rows, rad, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// lanes per block of a Miller kernel: [rows][lanes] doubles within 64 KiB
static int rad_lanes(int rows)
{
    int lanes = 64;
    while (lanes > 1 && (size_t)rows * lanes * sizeof(double) > 64 * 1024) lanes >>= 1;
    return lanes;
}

// ---------------------------------------------------------------------------
// Shared layout of the per-source expansion tables (P2M, X-list P2L).
// One wave per box.  A pass takes up to CH sources; for each, row t of T
// holds the 2P+3 basis values of orders n = -(P+1)..P+1 at
// T[t*(2P+3) + P+1 + n], built in two steps: one lane per source runs the
// radial recurrence into the non-negative half, then lanes (source, run of
// PT_SEG orders) attach the phases (one sincos per run, running products
// after it) and fill the negative orders.  Per-source weights of the three
// terms (charge, and the dipole's two neighbours) sit in Wt[t][d][3].  Each
// lane then owns output orders lane, lane + 64, ..., sums the pass's sources
// in source order and adds the result to the box's expansion (the first pass
// writes it).  One wave per box keeps many boxes in flight per CU, so the
// serial recurrences of some overlap the sums of others.
// ---------------------------------------------------------------------------
constexpr int PT_SEG = 8;
constexpr size_t PT_LDS = 24 * 1024;   // LDS per box: several boxes per CU

size_t ptab_lds_bytes(int nd, int P, int ch)
{
    return (size_t)ch * ((2 * (size_t)P + 3) * sizeof(cd) + 3 * (size_t)nd * sizeof(cd) + sizeof(cd) +
                         3 * sizeof(double)) +
           ((size_t)P + 2) * sizeof(double);
}

// ---------------------------------------------------------------------------
// Stage 2a: P2M at leaves, a_k = sum_j qS_j L_k(s_j - m) +
// (omega/2) qD_j (conj(nu_j) L_{k-1} - nu_j L_{k+1}), stored as a_k / W_|k|.
// L_n(z) = J_n(x) conj(v)^n with z = (x/omega) v, |v| = 1, and
// L_{-n} = (-1)^n J_n v^n.
// ---------------------------------------------------------------------------
// P2M reads each source's row of orders n = 0..P+1 (J_n is real, so
// L_{-n} = (-1)^n conj(L_n)) from the rows k_src_bas keeps with the
// geometry.  One wave per (box, run of 64 orders k >= 0): lane k sums the
// box's sources in order for the orders k and -k, which need the same three
// row entries (L_{-n} = (-1)^n conj(L_n)), read straight from those rows
// (neighbouring lanes read neighbouring entries); only the sources' weights,
// a pass of P2M_CH at a time, go through LDS.  The grid has boxes x runs of
// orders, enough waves to cover the loads' latency.
constexpr int P2M_CH = 64;
constexpr int BATCH = 8;      // sources whose basis loads are in flight together

size_t p2m_lds_bytes(int nd) { return (size_t)P2M_CH * 3 * (size_t)nd * sizeof(cd); }

int order_runs(int Pmax) { return (2 * Pmax + 1 + 63) / 64; }

// P2M lanes take the orders k and -k together: runs of 64 over k = 0..P.
int half_order_runs(int Pmax) { return (Pmax + 1 + 63) / 64; }

// u^k for a unit complex u and any integer k (u^{-1} = conj(u)) by binary
// powering, at most 2 log2|k| products.  Where a lane needs one phase per
// long run of orders, sincos of k theta is as cheap and needs no loop; this
// pays where it replaces the angle altogether.
__device__ __forceinline__ cd unit_ipow(cd u, int k)
{
    cd v = k >= 0 ? u : conj(u);
    int n = k >= 0 ? k : -k;
    cd r = mk(1.0, 0.0);
    while (n) {
        if (n & 1) r = r * v;
        v = v * v;
        n >>= 1;
    }
    return r;
}

// L_m from the row entry v = L_|m| (L_{-n} = (-1)^n conj(L_n)): f = 0 for
// m >= 0, 1 for even m < 0 (conjugate), 2 for odd m < 0 (minus the
// conjugate).  Sign changes only, so exact.
__device__ __forceinline__ cd bfix(cd v, int f) { return mk(f == 2 ? -v.x : v.x, f == 1 ? -v.y : v.y); }

template <int ND>
__device__ __forceinline__ void p2m_body(const DevGeom &g, const int *list, const cd *qs, const cd *qd, cd *mp, BlockId bid)
{
    extern __shared__ double lds_raw[];
    cd *Wt = reinterpret_cast<cd *>(lds_raw);           // [P2M_CH][ND][3]
    int b = list[bid.x];
    int l = g.blev[b];
    int P = g.Plev[l], np = 2 * P + 1;
    if (bid.y * 64 > P) return;                         // uniform: a run past this box's orders
    // lane k forms orders k and -k from the same three row entries
    int tid = threadIdx.x, k = bid.y * 64 + tid;
    bool active = k <= P;
    double hw = 0.5 * g.omega;
    const double *iw = g.invW + g.Woff[l];
    cd *out = mp + g.box_off[b] * ND;
    int s_begin = g.src_begin[b], s_end = g.src_end[b];
    // entries a = L_|k-1| (L_1 when k = 0), b = L_k, c = L_{k+1}; then
    //   order k:   L_{k-1} = a (k >= 1) or -conj(a) (k = 0), L_k = b, L_{k+1} = c
    //   order -k:  L_{-k-1}, L_{-k}, L_{-k+1} from c, b, a by bfix (a as is for k = 1)
    int ia = k == 0 ? 1 : k - 1;
    int fa = k == 0 ? 2 : 0;
    int fc_n = (k + 1) & 1 ? 2 : 1, fb_n = k & 1 ? 2 : 1, fa_n = k == 1 ? 0 : ((k - 1) & 1 ? 2 : 1);
    cd accp[ND], accn[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) accp[d] = accn[d] = mk(0.0, 0.0);
    auto add = [&](cd ea, cd eb, cd ec, const cd *w) {
        cd lm = bfix(ea, fa), mm = bfix(ec, fc_n), m0 = bfix(eb, fb_n), mp_ = bfix(ea, fa_n);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            cfma(accp[d], w[3 * d], eb);
            cfma(accp[d], w[3 * d + 1], lm);
            cfma(accp[d], w[3 * d + 2], ec);
            cfma(accn[d], w[3 * d], m0);
            cfma(accn[d], w[3 * d + 1], mm);
            cfma(accn[d], w[3 * d + 2], mp_);
        }
    };
    for (int s0 = s_begin; s0 < s_end; s0 += P2M_CH) {
        int cnt = min(P2M_CH, s_end - s0);
        __syncthreads();
        if (tid < cnt) {
            int j = s0 + tid;
            cd nu = mk(g.snx[j], g.sny[j]);
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                cd c = qd[(long long)d * g.ns + j];
                cd *w = Wt + (tid * ND + d) * 3;
                w[0] = qs[(long long)d * g.ns + j];
                w[1] = hw * (c * conj(nu));
                w[2] = neg(hw * (c * nu));
            }
        }
        __syncthreads();
        if (active) {
            // the sources of a box are consecutive, so are their rows.  The
            // entries of BATCH sources are loaded before any is used, so a
            // lane waits for memory once per batch, not once per source.
            const cd *rows = g.sbas + (long long)s0 * g.srow;
            int t = 0;
            for (; t + BATCH <= cnt; t += BATCH) {
                cd E[BATCH][3];
#pragma unroll
                for (int u = 0; u < BATCH; ++u) {
                    const cd *row = rows + (long long)(t + u) * g.srow;
                    E[u][0] = row[ia];
                    E[u][1] = row[k];
                    E[u][2] = row[k + 1];
                }
#pragma unroll
                for (int u = 0; u < BATCH; ++u) add(E[u][0], E[u][1], E[u][2], Wt + (t + u) * ND * 3);
            }
            for (; t < cnt; ++t) {
                const cd *row = rows + (long long)t * g.srow;
                add(row[ia], row[k], row[k + 1], Wt + t * ND * 3);
            }
        }
    }
    if (active) {
        // a leaf without sources gets a zero expansion
        double f = iw[k];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            out[d * np + P + k] = mk(f * accp[d].x, f * accp[d].y);
            if (k > 0) out[d * np + P - k] = mk(f * accn[d].x, f * accn[d].y);
        }
    }
}

template <int ND>
__global__ void __launch_bounds__(64) k_p2m(DevGeom g, const int *list, const cd *qs, const cd *qd, cd *mp)
{
    p2m_body<ND>(g, list, qs, qd, mp, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// ---------------------------------------------------------------------------
// Stage 4 as batched complex GEMM on FP64 MFMA.  For one (level, offset)
// group the scaled M2L matrix M (n x n, n = 2P+1) multiplies up to 16
// columns, each the scaled multipole of one V-list source box for one
// density; column c of the result is that pair's contribution to the target
// box's local, written to its own output row (vy) and summed in a fixed
// order by the downward pass.  Complex product with three real MFMAs
// (Gauss's form): P += Mr Xr, Q += Mi Xi, S += (Mr + Mi)(Xr + Xi), then
//   Yr = P - Q,  Yi = S - P - Q.
// v_mfma_f64_16x16x4f64 operands: lane l holds A[l%16][l/16], B[l/16][l%16];
// result D[4i + l/16][l%16] in element i.  The matrix is stored in that
// A-operand order, 16x4 blocks of 64 complex values, block (rb, kb) at
// (rb * NK + kb) * 64.
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
#ifndef QBX_TB_U
#define QBX_TB_U 2
#endif
constexpr int TB_U = QBX_TB_U;   // k-blocks whose table operands are loaded ahead

// Keeps the loads issued above it ahead of the matrix-core work below it:
// left alone, the scheduler sinks the next k-blocks' loads below the wait
// for the current ones, and the loop then waits on a full memory round trip
// every step.
#ifdef QBX_NO_FENCE
#define QBX_LOADS_AHEAD() ((void)0)
#else
#define QBX_LOADS_AHEAD() __builtin_amdgcn_sched_barrier(0)
#endif

// Workgroups are handed to the 8 XCDs round-robin (workgroup b to XCD b % 8).
// Map them so that XCD x works through its own contiguous range of tiles:
// the tiles of one (level, offset) group then share that XCD's L2 copy of
// the group's matrix instead of every XCD fetching every matrix.
constexpr int kNumXcd = 8;

__device__ __forceinline__ int xcd_contiguous(int b, int n)
{
    int per = n / kNumXcd, rem = n % kNumXcd;
    int x = b % kNumXcd, i = b / kNumXcd;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + i;
}

// V-list part of the downward pass: local = X-list part (already in loc)
// + the box's V-list contributions in list order.  Block bid.x takes box
// level_start[l] + bid.x, so a launch of nb - level_start[2] blocks from
// l = 2 covers every level at once.  L2L, given no V-list rows, then adds its
// translation to these sums: the same terms in the same order as when its
// epilogue summed the rows, with one bandwidth-bound launch in place of the
// epilogues' loads in every latency-bound L2L level.
__device__ __forceinline__ void down_body(const DevGeom &g, int nd, int l, const cd *vy, cd *loc, BlockId bid)
{
    int b = g.level_start[l] + bid.x;
    int P = g.Plev[g.blev[b]], n = 2 * P + 1;
    cd *out = loc + g.box_off[b] * nd;
    int v0 = g.V_start[b], nv = g.V_start[b + 1] - v0;
    if (nv == 0) return;
    // the box's V-list rows follow each other, n * nd apart
    const cd *vr = vy + g.vy_off[v0] * nd;
    long long vs = (long long)n * nd;
    for (int i = threadIdx.x; i < nd * n; i += blockDim.x) {
        cd acc = out[i];
#pragma unroll 4
        for (int v = 0; v < nv; ++v) acc = acc + vr[v * vs + i];
        out[i] = acc;
    }
}

// V-list sums of every box from level 2 on (one block of 64 lanes per
// density per box)
__global__ void __launch_bounds__(256) k_down_all(DevGeom g, int nd, const cd *vy, cd *loc)
{
    down_body(g, nd, 2, vy, loc, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// Part of one 16x16 output block of a scaled translation on FP64 MFMA: rows
// rb*16.. (Arow points at the row block), k-blocks [kb0, kb1), the lane's
// column given by bptr (nin complex inputs, NULL = 0).  The table is in
// A-operand order (see k_m2l_mfma).  Operands of the next TB_U k-blocks are
// loaded while the current ones go through the matrix core.
// z i^e (e taken mod 4): a swap and sign changes, exact
__device__ __forceinline__ cd mul_ipow(cd z, int e)
{
    bool sw = e & 1, ng = e & 2;
    double re = sw ? -z.y : z.x, im = sw ? z.x : z.y;
    return ng ? mk(-re, -im) : mk(re, im);
}

__device__ __forceinline__ void tb_load(const cd *Arow, int kb, int kb1, const cd *bs, bool bvalid,
                                        int nin, int lane, cd *a, cd *b)
{
    // unconditional loads at clamped addresses, out-of-range operands
    // replaced by zero afterwards: no branches, so the loads stay in flight
    int bk = lane >> 4;
#pragma unroll
    for (int u = 0; u < TB_U; ++u) {
        int kbu = kb + u;
        bool ok = kbu < kb1;
        int kbc = ok ? kbu : kb1 - 1;
        int k = kbc * 4 + bk;
        a[u] = Arow[kbc * 64 + lane];
        cd v = bs[min(k, nin - 1)];
        b[u] = (ok && bvalid && k < nin) ? v : mk(0.0, 0.0);
    }
}

// Complex products in three real ones (Gauss): P += ar br, Q += ai bi,
// S += (ar + ai)(br + bi); then Re = P - Q and Im = S - P - Q (cplx3_done).
// Three matrix-core operations per k-block instead of four, and three
// independent accumulation chains.  The imaginary part's rounding error is
// a few ulps of (|ar| + |ai|)(|br| + |bi|), the same order as the plain
// product's.
struct Acc3 {
    d4 p, q, s;
};

__device__ __forceinline__ Acc3 cplx3_zero()
{
    return Acc3{{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
}

__device__ __forceinline__ void cplx3_mfma(cd a, cd b, Acc3 &y)
{
    y.p = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, y.p, 0, 0, 0);
    y.q = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, y.q, 0, 0, 0);
    y.s = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x + b.y, y.s, 0, 0, 0);
}

__device__ __forceinline__ void cplx3_done(const Acc3 &y, d4 &yr, d4 &yi)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        yr[i] = y.p[i] - y.q[i];
        yi[i] = (y.s[i] - y.p[i]) - y.q[i];
    }
}

// ROT: the input coefficients of order k enter times i^{rot k}.  A lane
// always holds the same k mod 4 (lane / 16), so the factor is one per lane
// (e, taken mod 4), applied as the operand goes in, after its load.
template <bool ROT = false>
__device__ __forceinline__ void tb_mfma(const cd *a, const cd *b, Acc3 &y, int e = 0)
{
#pragma unroll
    for (int u = 0; u < TB_U; ++u) cplx3_mfma(a[u], ROT ? mul_ipow(b[u], e) : b[u], y);
}

// Two register sets alternate: one is multiplied while the other loads.
template <bool ROT = false>
__device__ __forceinline__ void trans_block(const cd *Arow, int kb0, int kb1, const cd *bptr, int nin,
                                            int lane, d4 &yr, d4 &yi, int rot = 0, int P = 0)
{
    if (kb0 >= kb1) return;
    const cd *bs = bptr ? bptr : Arow;          // any readable address when the column is empty
    bool bvalid = bptr != nullptr;
    cd a0[TB_U], b0[TB_U], a1[TB_U], b1[TB_U];
    Acc3 y = cplx3_zero();
    int e = rot * ((lane >> 4) - P);            // order k = 4 kb + lane/16 - P
    tb_load(Arow, kb0, kb1, bs, bvalid, nin, lane, a0, b0);
    for (int kb = kb0; kb < kb1; kb += 2 * TB_U) {
        tb_load(Arow, kb + TB_U, kb1, bs, bvalid, nin, lane, a1, b1);
        QBX_LOADS_AHEAD();
        tb_mfma<ROT>(a0, b0, y, e);
        tb_load(Arow, kb + 2 * TB_U, kb1, bs, bvalid, nin, lane, a0, b0);
        QBX_LOADS_AHEAD();
        if (kb + TB_U < kb1) tb_mfma<ROT>(a1, b1, y, e);
    }
    cplx3_done(y, yr, yi);
}

// M2L: one workgroup per 16-column tile, nw waves over its row blocks
// (rb = wave, wave + nw, ...).  The tile's columns (the source boxes'
// multipoles) are staged once in LDS through host-precomputed offsets and
// serve every row block; table fragments stream from memory with the next
// TB_U k-blocks in flight.  Workgroups run in XCD-contiguous order so that the
// tiles of one (level, offset) group share an XCD's L2 copy of its matrix.
constexpr int M2L_XS = 17;    // LDS row stride of the staged columns (padded)

__device__ __forceinline__ void m2l_mfma_body(const DevGeom &g, int nd, const M2LTile *tiles, const cd *mp, cd *vy, BlockId bid)
{
    extern __shared__ double lds_raw[];
    cd *X = reinterpret_cast<cd *>(lds_raw);    // [4 NK][M2L_XS]
    M2LTile t = tiles[xcd_contiguous(bid.x, bid.nx)];
    int l = t.lo / 40;
    int P = g.Plev[l], n = 2 * P + 1;
    int NK = (n + 3) / 4, NR = (n + 15) / 16;
    int nw = blockDim.x >> 6;
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int bk = lane >> 4, bc = lane & 15;
    {
        // blockDim/16 threads per column, consecutive k per column
        int tpc = blockDim.x >> 4;
        int sc = threadIdx.x / tpc, sr = threadIdx.x - sc * tpc;
        const cd *col = nullptr;
        int rot = 0;
        if (sc < t.ncol) {
            int cc = t.col0 + sc;
            col = mp + g.m2l_src[t.pair_start + cc / nd] * nd + (long long)(cc % nd) * n;
            rot = g.m2l_rot[t.pair_start + cc / nd];
        }
        // the column of a rotated offset enters as i^{rk} a_k
        for (int k = sr; k < 4 * NK; k += tpc)
            X[k * M2L_XS + sc] = (col && k < n) ? mul_ipow(col[k], rot * (k - P)) : mk(0.0, 0.0);
    }
    __syncthreads();
    const cd *A = g.m2l_mf + g.m2l_mf_off[t.lo];
    for (int rb = wave; rb < NR; rb += nw) {
        const cd *Ab = A + (long long)rb * NK * 64 + lane;
        Acc3 y = cplx3_zero();
        cd a0[TB_U], a1[TB_U];
#pragma unroll
        for (int u = 0; u < TB_U; ++u) a0[u] = Ab[min(u, NK - 1) * 64];
        for (int kb = 0; kb < NK; kb += 2 * TB_U) {
#pragma unroll
            for (int u = 0; u < TB_U; ++u) a1[u] = Ab[min(kb + TB_U + u, NK - 1) * 64];
            QBX_LOADS_AHEAD();
#pragma unroll
            for (int u = 0; u < TB_U; ++u) {
                int kk = kb + u;
                cd bv = X[(min(kk, NK - 1) * 4 + bk) * M2L_XS + bc];
                if (kk >= NK) bv = mk(0.0, 0.0);
                cplx3_mfma(a0[u], bv, y);
            }
#pragma unroll
            for (int u = 0; u < TB_U; ++u) a0[u] = Ab[min(kb + 2 * TB_U + u, NK - 1) * 64];
            QBX_LOADS_AHEAD();
            if (kb + TB_U < NK) {
#pragma unroll
                for (int u = 0; u < TB_U; ++u) {
                    int kk = kb + TB_U + u;
                    cd bv = X[(min(kk, NK - 1) * 4 + bk) * M2L_XS + bc];
                    if (kk >= NK) bv = mk(0.0, 0.0);
                    cplx3_mfma(a1[u], bv, y);
                }
            }
        }
        d4 yr, yi;
        cplx3_done(y, yr, yi);
        if (bc < t.ncol) {
            int col = t.col0 + bc;
            cd *o = vy + g.m2l_dst[t.pair_start + col / nd] * nd + (long long)(col % nd) * n;
            int rot = g.m2l_rot[t.pair_start + col / nd];
            for (int i = 0; i < 4; ++i) {
                int row = rb * 16 + 4 * i + bk;
                if (row < n) o[row] = mul_ipow(mk(yr[i], yi[i]), rot * (row - P));
            }
        }
    }
}

__global__ void __launch_bounds__(1024) k_m2l_mfma(DevGeom g, int nd, const M2LTile *tiles, const cd *mp, cd *vy)
{
    m2l_mfma_body(g, nd, tiles, mp, vy, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// M2L for orders whose staged columns exceed the LDS budget: one wave per
// (tile, row block), operands straight from memory with the
// loads of the next TB_U k-blocks in flight (trans_block).  1-D grid of
// ntiles * nrmax waves in XCD-contiguous order, the row blocks of a tile
// consecutive, so that a tile's columns and a group's matrix are fetched
// into one XCD's L2; waves past the tile's row count exit at once.
__device__ __forceinline__ void m2l_mfma_direct_body(const DevGeom &g, int nd, const M2LTile *tiles, int nrmax, const cd *mp, cd *vy, BlockId bid)
{
    int c = xcd_contiguous(bid.x, bid.nx);
    M2LTile t = tiles[c / nrmax];
    int rb = c % nrmax;
    int l = t.lo / 40;
    int P = g.Plev[l], n = 2 * P + 1;
    int NK = (n + 3) / 4, NR = (n + 15) / 16;
    if (rb >= NR) return;
    int lane = threadIdx.x;
    int bk = lane >> 4, bc = lane & 15;
    int col = t.col0 + bc;
    bool valid = bc < t.ncol;
    const cd *bptr = valid ? mp + g.m2l_src[t.pair_start + col / nd] * nd + (long long)(col % nd) * n : nullptr;
    int rot = valid ? g.m2l_rot[t.pair_start + col / nd] : 0;
    d4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
    trans_block<true>(g.m2l_mf + g.m2l_mf_off[t.lo] + (long long)rb * NK * 64, 0, NK, bptr, n, lane, yr, yi,
                      rot, P);
    if (!valid) return;
    cd *o = vy + g.m2l_dst[t.pair_start + col / nd] * nd + (long long)(col % nd) * n;
    for (int i = 0; i < 4; ++i) {
        int row = rb * 16 + 4 * i + bk;
        if (row < n) o[row] = mul_ipow(mk(yr[i], yi[i]), rot * (row - P));
    }
}

__global__ void __launch_bounds__(64) k_m2l_mfma_direct(DevGeom g, int nd, const M2LTile *tiles, int nrmax, const cd *mp, cd *vy)
{
    m2l_mfma_direct_body(g, nd, tiles, nrmax, mp, vy, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// ---------------------------------------------------------------------------
// FP32 far field (eps >= 1e-6): the same translations on v_mfma_f32_16x16x4f32
// with complex-float tables.  Inputs are rounded to float as they load and
// results return to the FP64 expansion arrays.  Operand layout as in the FP64
// instruction; the result layout differs: element i of lane l is
// D[4 (l/16) + i][l%16].
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void tb_load32(const cf *Arow, int kb, int kb1, const cd *bs, bool bvalid,
                                          int nin, int lane, cf *a, cf *b)
{
    int bk = lane >> 4;
#pragma unroll
    for (int u = 0; u < TB_U; ++u) {
        int kbu = kb + u;
        bool ok = kbu < kb1;
        int kbc = ok ? kbu : kb1 - 1;
        int k = kbc * 4 + bk;
        a[u] = Arow[kbc * 64 + lane];
        cd v = bs[min(k, nin - 1)];
        b[u] = (ok && bvalid && k < nin) ? cf{(float)v.x, (float)v.y} : cf{0.f, 0.f};
    }
}

// The same three-product form as the FP64 translations (cplx3_mfma).
struct Acc3f {
    f4 p, q, s;
};

__device__ __forceinline__ cf mul_ipow32(cf z, int e)
{
    bool sw = e & 1, ng = e & 2;
    float re = sw ? -z.y : z.x, im = sw ? z.x : z.y;
    return ng ? cf{-re, -im} : cf{re, im};
}

template <bool ROT = false>
__device__ __forceinline__ void tb_mfma32(const cf *a, const cf *b, Acc3f &y, int e = 0)
{
#pragma unroll
    for (int u = 0; u < TB_U; ++u) {
        cf bb = ROT ? mul_ipow32(b[u], e) : b[u];
        y.p = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u].x, bb.x, y.p, 0, 0, 0);
        y.q = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u].y, bb.y, y.q, 0, 0, 0);
        y.s = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u].x + a[u].y, bb.x + bb.y, y.s, 0, 0, 0);
    }
}

template <bool ROT = false>
__device__ __forceinline__ void trans_block32(const cf *Arow, int kb0, int kb1, const cd *bptr, int nin,
                                              int lane, f4 &yr, f4 &yi, int rot = 0, int P = 0)
{
    if (kb0 >= kb1) return;
    const cd *bs = bptr ? bptr : reinterpret_cast<const cd *>(Arow);
    bool bvalid = bptr != nullptr;
    cf a0[TB_U], b0[TB_U], a1[TB_U], b1[TB_U];
    Acc3f y{{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    int e = rot * ((lane >> 4) - P);            // order k = 4 kb + lane/16 - P
    tb_load32(Arow, kb0, kb1, bs, bvalid, nin, lane, a0, b0);
    for (int kb = kb0; kb < kb1; kb += 2 * TB_U) {
        tb_load32(Arow, kb + TB_U, kb1, bs, bvalid, nin, lane, a1, b1);
        QBX_LOADS_AHEAD();
        tb_mfma32<ROT>(a0, b0, y, e);
        tb_load32(Arow, kb + 2 * TB_U, kb1, bs, bvalid, nin, lane, a0, b0);
        QBX_LOADS_AHEAD();
        if (kb + TB_U < kb1) tb_mfma32<ROT>(a1, b1, y, e);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        yr[i] = y.p[i] - y.q[i];
        yi[i] = (y.s[i] - y.p[i]) - y.q[i];
    }
}

__device__ __forceinline__ void m2l_mfma32_body(const DevGeom &g, int nd, const M2LTile *tiles, int nrmax, const cd *mp, cd *vy, BlockId bid)
{
    int c = xcd_contiguous(bid.x, bid.nx);
    M2LTile t = tiles[c / nrmax];
    int rb = c % nrmax;
    int l = t.lo / 40;
    int P = g.Plev[l], n = 2 * P + 1;
    int NK = (n + 3) / 4, NR = (n + 15) / 16;
    if (rb >= NR) return;
    int lane = threadIdx.x;
    int bk = lane >> 4, bc = lane & 15;
    int col = t.col0 + bc;
    bool valid = bc < t.ncol;
    const cd *bptr = valid ? mp + g.m2l_src[t.pair_start + col / nd] * nd + (long long)(col % nd) * n : nullptr;
    int rot = valid ? g.m2l_rot[t.pair_start + col / nd] : 0;
    f4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
    trans_block32<true>(g.m2l_mf32 + g.m2l_mf_off[t.lo] + (long long)rb * NK * 64, 0, NK, bptr, n, lane, yr, yi,
                        rot, P);
    if (!valid) return;
    cd *o = vy + g.m2l_dst[t.pair_start + col / nd] * nd + (long long)(col % nd) * n;
    for (int i = 0; i < 4; ++i) {
        int row = rb * 16 + 4 * bk + i;
        if (row < n) o[row] = mul_ipow(mk((double)yr[i], (double)yi[i]), rot * (row - P));
    }
}

__global__ void __launch_bounds__(64) k_m2l_mfma32(DevGeom g, int nd, const M2LTile *tiles, int nrmax, const cd *mp, cd *vy)
{
    m2l_mfma32_body(g, nd, tiles, nrmax, mp, vy, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// k-block range of part h of NK split in KS near-equal parts
__device__ __forceinline__ void ksplit(int NK, int KS, int h, int *kb0, int *kb1)
{
    int c = (NK + KS - 1) / KS;
    *kb0 = min(NK, h * c);
    *kb1 = min(NK, *kb0 + c);
}

// Partial 16x16 blocks of the waves of one workgroup: element i of lane l is
// D[4i + l/16][l%16]; padded to 9 doubles per lane against bank conflicts.
__device__ __forceinline__ void tb_store(double (*part)[9], int lane, const d4 &yr, const d4 &yi)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) { part[lane][i] = yr[i]; part[lane][4 + i] = yi[i]; }
}

// Sum of the nw partial blocks (in wave order) at output row r, column c.
__device__ __forceinline__ cd tb_sum(const double (*part)[64][9], int nw, int r, int c)
{
    int ln = (r & 3) * 16 + c, i = r >> 2;
    cd y = mk(0.0, 0.0);
    for (int w = 0; w < nw; ++w) y = y + mk(part[w][ln][i], part[w][ln][4 + i]);
    return y;
}

// Stage 2b: M2M into the non-leaf boxes of level l.  Block = (tile of 16
// (parent, density) columns, row block); wave w applies the child-quadrant
// (w % 4) matrix over part w / 4 of its k-blocks (M2M_KS parts); the partial
// blocks are summed in wave order.  One part (four waves, 18 KiB of LDS) lets
// the workgroups of a level find room beside the near field on the other
// stream: the step 0.452 to 0.446 ms, though each level alone is slower than
// with two parts (M2M in order 101 against 105 us).
constexpr int M2M_KS = 1;

__device__ __forceinline__ void m2m_mfma_body(const DevGeom &g, int nd, int l, const TTile *tiles, const int *plist, cd *mp, BlockId bid)
{
    __shared__ double part[4 * M2M_KS][64][9];
    TTile t = tiles[bid.x];
    int rb = bid.y;
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = w & 3, h = w >> 2;
    int np = 2 * g.Plev[l] + 1, nc = 2 * g.Plev[l + 1] + 1;
    int NKc = (nc + 3) / 4;
    int bc = lane & 15;
    int col = t.col0 + bc;
    bool valid = bc < t.ncol;
    int d = col % nd;
    long long coff = valid ? g.m2m_coff[(long long)(t.start + col / nd) * 4 + q] : -1;
    const cd *bptr = coff >= 0 ? mp + coff * nd + (long long)d * nc : nullptr;
    d4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
    int kb0, kb1;
    ksplit(NKc, M2M_KS, h, &kb0, &kb1);
    if (__any(coff >= 0))
        trans_block(g.m2m_mf + g.m2m_mf_off[l * 4 + q] + (long long)rb * NKc * 64, kb0, kb1, bptr, nc,
                    lane, yr, yi);
    tb_store(part[w], lane, yr, yi);
    __syncthreads();
    int tid = threadIdx.x;
    if (tid < 256) {
        int r = tid >> 4, c = tid & 15;
        int row = rb * 16 + r;
        if (c < t.ncol && row < np) {
            int oc = t.col0 + c;
            mp[g.m2m_poff[t.start + oc / nd] * nd + (long long)(oc % nd) * np + row] =
                tb_sum(part, 4 * M2M_KS, r, c);
        }
    }
}

__global__ void __launch_bounds__(256 * M2M_KS) k_m2m_mfma(DevGeom g, int nd, int l, const TTile *tiles, const int *plist, cd *mp)
{
    m2m_mfma_body(g, nd, l, tiles, plist, mp, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// Stage 7 (levels >= 3): local of a child = X-list part (already in loc) +
// its V-list contributions in list order + L2L of the parent's local.
// Block = (tile of 16 (child, density) columns of one quadrant, row block);
// the four waves take a quarter of the k-blocks each.
constexpr int L2L_KS = 4;

__device__ __forceinline__ void l2l_mfma_body(const DevGeom &g, int nd, int L, const TTile *tiles, const int *clist, const cd *vy, cd *loc, BlockId bid)
{
    __shared__ double part[L2L_KS][64][9];
    TTile t = tiles[bid.x];
    int rb = bid.y;
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int nc = 2 * g.Plev[L] + 1, np = 2 * g.Plev[L - 1] + 1;
    int NKp = (np + 3) / 4;
    int bc = lane & 15;
    int col = t.col0 + bc;
    bool valid = bc < t.ncol;
    int d = col % nd;
    const cd *bptr = valid ? loc + g.l2l_poff[t.start + col / nd] * nd + (long long)d * np : nullptr;
    // The child's local that this thread completes, loaded ahead of the
    // K loop (it is not written in this launch: the loop reads the
    // parents' level), so that its round trip overlaps the loop.
    int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    int row = rb * 16 + r;
    bool own = c < t.ncol && row < nc;
    int oc = t.col0 + c;
    int pos = t.start + oc / nd;
    long long dr = (long long)(oc % nd) * nc + row;
    long long base = own ? g.l2l_coff[pos] * nd + dr : 0;
    cd acc = own ? loc[base] : mk(0.0, 0.0);
    d4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
    int kb0, kb1;
    ksplit(NKp, L2L_KS, w, &kb0, &kb1);
    trans_block(g.l2l_mf + g.l2l_mf_off[(L - 1) * 4 + t.q] + (long long)rb * NKp * 64, kb0, kb1, bptr,
                np, lane, yr, yi);
    tb_store(part[w], lane, yr, yi);
    __syncthreads();
    if (!own) return;
    // V-list rows of the child follow each other, nc * nd apart
    // vy null: the V-list rows are already in loc
    const cd *vr = vy ? vy + g.l2l_vy0[pos] * nd + dr : nullptr;
    int nv = vy ? g.l2l_nv[pos] : 0;
    long long vs = (long long)nc * nd;
#pragma unroll 4
    for (int v = 0; v < nv; ++v) acc = acc + vr[v * vs];
    loc[base] = acc + tb_sum(part, L2L_KS, r, c);
}

__global__ void __launch_bounds__(64 * L2L_KS) k_l2l_mfma(DevGeom g, int nd, int L, const TTile *tiles, const int *clist, const cd *vy, cd *loc)
{
    l2l_mfma_body(g, nd, L, tiles, clist, vy, loc, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// FP32 variant of k_l2l_mfma (FP32 far field): same work split; the partial
// blocks are stored in double in the FP32 result layout.
__device__ __forceinline__ cd tb_sum32(const double (*part)[64][9], int nw, int r, int c)
{
    int ln = (r >> 2) * 16 + c, i = r & 3;
    cd y = mk(0.0, 0.0);
    for (int w = 0; w < nw; ++w) y = y + mk(part[w][ln][i], part[w][ln][4 + i]);
    return y;
}

__device__ __forceinline__ void l2l_mfma32_body(const DevGeom &g, int nd, int L, const TTile *tiles, const cd *vy, cd *loc, BlockId bid)
{
    __shared__ double part[L2L_KS][64][9];
    TTile t = tiles[bid.x];
    int rb = bid.y;
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int nc = 2 * g.Plev[L] + 1, np = 2 * g.Plev[L - 1] + 1;
    int NKp = (np + 3) / 4;
    int bc = lane & 15;
    int col = t.col0 + bc;
    bool valid = bc < t.ncol;
    int d = col % nd;
    const cd *bptr = valid ? loc + g.l2l_poff[t.start + col / nd] * nd + (long long)d * np : nullptr;
    // the child's local this thread completes, loaded ahead of the K loop
    int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    int row = rb * 16 + r;
    bool own = c < t.ncol && row < nc;
    int oc = t.col0 + c;
    int pos = t.start + oc / nd;
    long long dr = (long long)(oc % nd) * nc + row;
    long long base = own ? g.l2l_coff[pos] * nd + dr : 0;
    cd acc = own ? loc[base] : mk(0.0, 0.0);
    f4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
    int kb0, kb1;
    ksplit(NKp, L2L_KS, w, &kb0, &kb1);
    trans_block32(g.l2l_mf32 + g.l2l_mf_off[(L - 1) * 4 + t.q] + (long long)rb * NKp * 64, kb0, kb1, bptr,
                  np, lane, yr, yi);
#pragma unroll
    for (int i = 0; i < 4; ++i) { part[w][lane][i] = (double)yr[i]; part[w][lane][4 + i] = (double)yi[i]; }
    __syncthreads();
    if (!own) return;
    // vy null: the V-list rows are already in loc
    const cd *vr = vy ? vy + g.l2l_vy0[pos] * nd + dr : nullptr;
    int nv = vy ? g.l2l_nv[pos] : 0;
    long long vs = (long long)nc * nd;
#pragma unroll 4
    for (int v = 0; v < nv; ++v) acc = acc + vr[v * vs];
    loc[base] = acc + tb_sum32(part, L2L_KS, r, c);
}

__global__ void __launch_bounds__(64 * L2L_KS) k_l2l_mfma32(DevGeom g, int nd, int L, const TTile *tiles, const cd *vy, cd *loc)
{
    l2l_mfma32_body(g, nd, L, tiles, vy, loc, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// ---------------------------------------------------------------------------
// Stage 6: X-list P2L, g_l += qS O_l(s - m_b) + (omega/2) qD (nu O_{l-1} -
// conj(nu) O_{l+1}), stored as W_|l| g_l.  O_n = H_n(x) v^n and
// O_{-n} = (-1)^n H_n(x) conj(v)^n.  Row entry n holds S_n O_n with
// S_n = W_min(|n|,P), built from A_n = tau^n H_n (tau = min(1, x/2)) and
// S_n tau^{-n} (one exp per run of orders, ratios of the W table after it);
// the two dipole sums are rescaled by W_|l| / S_{l-+1} at the end.  The
// sources of all X-list boxes of b are taken in list order (flattened on
// the host).
// ---------------------------------------------------------------------------
// The X-list P2L row of flattened X-list position q, as p2l_x_body builds
// it in LDS when it is not cached: S_n O_n(s - m_b), n = -(P+1)..P+1, at
// xbas[xbas_off[q] + P + 1 + n].  One lane per position.
__device__ __forceinline__ void x_bas_body(const DevGeom &g, int nx, cd *xbas, BlockId bid)
{
    int q = bid.x * blockDim.x + threadIdx.x;
    if (q >= nx) return;
    int b = g.xsrc_box[q], j = g.xsrc_idx[q];
    int l = g.blev[b];
    int P = g.Plev[l];
    const double *Wl = g.Wtab + g.Woff[l], *iWl = g.invW + g.Woff[l], *lWl = g.logW + g.Woff[l];
    double dx = g.sx[j] - g.bcx[b], dy = g.sy[j] - g.bcy[b];
    double r = sqrt(dx * dx + dy * dy);
    double x = g.omega * r;
    double tau = fmin(1.0, 0.5 * x);
    cd *row = xbas + g.xbas_off[q] + P + 1;
    scaled_hankel_seq(x, tau, P + 1, row, 1);
    cd v = mk(dx / r, dy / r);
    double th = atan2(dy, dx), lt = log(tau), itau = 1.0 / tau;
    for (int n0 = 0; n0 <= P + 1; n0 += PT_SEG) {
        double sn, cs;
        sincos((double)n0 * th, &sn, &cs);
        cd ph = mk(cs, sn);                            // v^n
        double sc = exp(lWl[min(n0, P)] - n0 * lt);    // S_n tau^{-n}
        for (int n = n0; n < n0 + PT_SEG && n <= P + 1; ++n) {
            cd e = sc * row[n];
            row[n] = e * ph;
            if (n > 0) {
                cd m = e * conj(ph);
                row[-n] = (n & 1) ? neg(m) : m;
            }
            ph = ph * v;
            sc *= (Wl[min(n + 1, P)] * iWl[min(n, P)]) * itau;
        }
    }
}

__global__ void k_x_bas(DevGeom g, int nx, cd *xbas)
{
    x_bas_body(g, nx, xbas, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

template <int ND>
__device__ __forceinline__ void p2l_x_body(const DevGeom &g, const int *list, const cd *qs, const cd *qd, cd *loc, int CH, BlockId bid)
{
    extern __shared__ double lds_raw[];
    int b = list[bid.x];
    int l = g.blev[b];
    int P = g.Plev[l], np = 2 * P + 1, NT = 2 * P + 3;
    cd *T = reinterpret_cast<cd *>(lds_raw);           // [CH][NT]
    cd *Wt = T + CH * NT;                              // [CH][ND][3]
    cd *V = Wt + CH * ND * 3;                          // [CH]
    double *TH = reinterpret_cast<double *>(V + CH);   // [CH]
    double *LT = TH + CH;                              // [CH] log tau
    double *TAU = LT + CH;                             // [CH]
    double *RW = TAU + CH;                             // [P+2] S_{n+1} / S_n
    const double *Wl = g.Wtab + g.Woff[l], *iWl = g.invW + g.Woff[l], *lWl = g.logW + g.Woff[l];
    int tid = threadIdx.x;
    for (int n = tid; n <= P + 1; n += blockDim.x) RW[n] = Wl[min(n + 1, P)] * iWl[min(n, P)];
    double mx = g.bcx[b], my = g.bcy[b], hw = 0.5 * g.omega;
    cd *out = loc + g.box_off[b] * ND;
    int q0 = g.xsrc_start[bid.x], total = g.xsrc_start[bid.x + 1] - q0;
    int nseg = (P + 2 + PT_SEG - 1) / PT_SEG;
    for (int f0 = 0; f0 < total; f0 += CH) {
        int cnt = min(CH, total - f0);
        __syncthreads();
        if (tid < cnt) {
            int j = g.xsrc_idx[q0 + f0 + tid];
            double dx = g.sx[j] - mx, dy = g.sy[j] - my;
            double r = sqrt(dx * dx + dy * dy);
            double x = g.omega * r;
            double tau = fmin(1.0, 0.5 * x);
            scaled_hankel_seq(x, tau, P + 1, T + tid * NT + P + 1, 1);
            V[tid] = mk(dx / r, dy / r);
            TH[tid] = atan2(dy, dx);
            LT[tid] = log(tau);
            TAU[tid] = tau;
            cd nu = mk(g.snx[j], g.sny[j]);
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                cd c = qd[(long long)d * g.ns + j];
                cd *w = Wt + (tid * ND + d) * 3;
                w[0] = qs[(long long)d * g.ns + j];
                w[1] = hw * (c * nu);
                w[2] = neg(hw * (c * conj(nu)));
            }
        }
        __syncthreads();
        for (int it = tid; it < cnt * nseg; it += blockDim.x) {
            int t = it % cnt, n0 = (it / cnt) * PT_SEG;
            cd v = V[t];
            double itau = 1.0 / TAU[t];
            double sn, cs;
            sincos((double)n0 * TH[t], &sn, &cs);
            cd ph = mk(cs, sn);                        // v^n
            double sc = exp(lWl[min(n0, P)] - n0 * LT[t]);   // S_n tau^{-n}
            cd *row = T + t * NT + P + 1;
            for (int n = n0; n < n0 + PT_SEG && n <= P + 1; ++n) {
                cd e = sc * row[n];
                row[n] = e * ph;
                if (n > 0) {
                    cd m = e * conj(ph);
                    row[-n] = (n & 1) ? neg(m) : m;
                }
                ph = ph * v;
                sc *= RW[n] * itau;
            }
        }
        __syncthreads();
        bool first = f0 == 0;
        for (int kk = tid; kk < np; kk += blockDim.x) {
            cd acc[3][ND];
#pragma unroll
            for (int e = 0; e < 3; ++e)
#pragma unroll
                for (int d = 0; d < ND; ++d) acc[e][d] = mk(0.0, 0.0);
            for (int t = 0; t < cnt; ++t) {
                const cd *row = T + t * NT + kk + 1;   // order l = kk - P at row[0]
                cd om = row[-1], o0 = row[0], op = row[1];
                const cd *w = Wt + t * ND * 3;
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    cfma(acc[0][d], w[3 * d], o0);
                    cfma(acc[1][d], w[3 * d + 1], om);
                    cfma(acc[2][d], w[3 * d + 2], op);
                }
            }
            int ell = kk - P, al = ell < 0 ? -ell : ell;
            int am = ell - 1 < 0 ? 1 - ell : ell - 1, ap = ell + 1 < 0 ? -ell - 1 : ell + 1;
            double rm = Wl[al] * iWl[min(am, P)], rp = Wl[al] * iWl[min(ap, P)];
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                cd v = mk(fma(rp, acc[2][d].x, fma(rm, acc[1][d].x, acc[0][d].x)),
                          fma(rp, acc[2][d].y, fma(rm, acc[1][d].y, acc[0][d].y)));
                if (!first) v = out[d * np + kk] + v;
                out[d * np + kk] = v;
            }
        }
    }
}

template <int ND>
__global__ void __launch_bounds__(64) k_p2l_x(DevGeom g, const int *list, const cd *qs, const cd *qd, cd *loc, int CH)
{
    p2l_x_body<ND>(g, list, qs, qd, loc, CH, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// X-list P2L from the rows kept with the geometry (x_bas_body): one wave per
// (box, run of 64 output orders), as P2M.  Lane kk reads its three entries of
// each position's row straight from memory (neighbouring lanes, neighbouring
// entries); the weights of a pass of XC_CH positions go through LDS.  Sums
// run over the box's positions in list order and are scaled once at the end.
constexpr int XC_CH = 64;

size_t p2l_xc_lds_bytes(int nd) { return (size_t)XC_CH * 3 * (size_t)nd * sizeof(cd); }

template <int ND>
__device__ __forceinline__ void p2l_xc_body(const DevGeom &g, const int *list, const cd *qs, const cd *qd, cd *loc, BlockId bid)
{
    extern __shared__ double lds_raw[];
    cd *Wt = reinterpret_cast<cd *>(lds_raw);          // [XC_CH][ND][3]
    int b = list[bid.x];
    int l = g.blev[b];
    int P = g.Plev[l], np = 2 * P + 1, NT = 2 * P + 3;
    if (bid.y * 64 >= np) return;                      // uniform: a run past this box's orders
    int tid = threadIdx.x, kk = bid.y * 64 + tid;
    const double *Wl = g.Wtab + g.Woff[l], *iWl = g.invW + g.Woff[l];
    double hw = 0.5 * g.omega;
    cd *out = loc + g.box_off[b] * ND;
    int q0 = g.xsrc_start[bid.x], total = g.xsrc_start[bid.x + 1] - q0;
    cd acc[3][ND];
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int d = 0; d < ND; ++d) acc[e][d] = mk(0.0, 0.0);
    for (int f0 = 0; f0 < total; f0 += XC_CH) {
        int cnt = min(XC_CH, total - f0);
        __syncthreads();
        if (tid < cnt) {
            int j = g.xsrc_idx[q0 + f0 + tid];
            cd nu = mk(g.snx[j], g.sny[j]);
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                cd c = qd[(long long)d * g.ns + j];
                cd *w = Wt + (tid * ND + d) * 3;
                w[0] = qs[(long long)d * g.ns + j];
                w[1] = hw * (c * nu);
                w[2] = neg(hw * (c * conj(nu)));
            }
        }
        __syncthreads();
        if (kk < np) {
            // one box's positions are consecutive rows of NT entries; order
            // l = kk - P sits at entry kk + 1 of a row.  Loads of BATCH
            // positions go out before any is used (as in P2M).
            const cd *rows = g.xbas + g.xbas_off[q0 + f0] + kk + 1;
            int t = 0;
            for (; t + BATCH <= cnt; t += BATCH) {
                cd O[BATCH][3];
#pragma unroll
                for (int u = 0; u < BATCH; ++u) {
                    const cd *row = rows + (long long)(t + u) * NT;
                    O[u][0] = row[-1];
                    O[u][1] = row[0];
                    O[u][2] = row[1];
                }
#pragma unroll
                for (int u = 0; u < BATCH; ++u) {
                    const cd *w = Wt + (t + u) * ND * 3;
#pragma unroll
                    for (int d = 0; d < ND; ++d) {
                        cfma(acc[0][d], w[3 * d], O[u][1]);
                        cfma(acc[1][d], w[3 * d + 1], O[u][0]);
                        cfma(acc[2][d], w[3 * d + 2], O[u][2]);
                    }
                }
            }
            for (; t < cnt; ++t) {
                const cd *row = rows + (long long)t * NT;
                cd om = row[-1], o0 = row[0], op = row[1];
                const cd *w = Wt + t * ND * 3;
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    cfma(acc[0][d], w[3 * d], o0);
                    cfma(acc[1][d], w[3 * d + 1], om);
                    cfma(acc[2][d], w[3 * d + 2], op);
                }
            }
        }
    }
    if (kk < np) {
        int ell = kk - P, al = ell < 0 ? -ell : ell;
        int am = ell - 1 < 0 ? 1 - ell : ell - 1, ap = ell + 1 < 0 ? -ell - 1 : ell + 1;
        double rm = Wl[al] * iWl[min(am, P)], rp = Wl[al] * iWl[min(ap, P)];
#pragma unroll
        for (int d = 0; d < ND; ++d)
            out[d * np + kk] = mk(fma(rp, acc[2][d].x, fma(rm, acc[1][d].x, acc[0][d].x)),
                                  fma(rp, acc[2][d].y, fma(rm, acc[1][d].y, acc[0][d].y)));
    }
}

template <int ND>
__global__ void __launch_bounds__(64) k_p2l_xc(DevGeom g, const int *list, const cd *qs, const cd *qd, cd *loc)
{
    p2l_xc_body<ND>(g, list, qs, qd, loc, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// The capped form beside the other stream: the grid walks the boxes back and
// forth, as the near field does.  (Its loop keeps more registers live, 96
// against 64 VGPRs, so launches that are not capped take the plain form.)
template <int ND>
__global__ void __launch_bounds__(64) k_p2l_xc_capped(DevGeom g, int n, const int *list, const cd *qs, const cd *qd, cd *loc)
{
    int G = gridDim.x;
    for (int r = 0; r * G < n; ++r) {
        int b = r * G + ((r & 1) ? G - 1 - (int)blockIdx.x : (int)blockIdx.x);
        if (b < n) p2l_xc_body<ND>(g, list, qs, qd, loc, BlockId{b, (int)blockIdx.y, n});
    }
}

// ---------------------------------------------------------------------------
// Stage 3: P2QBXL.  alpha_l(c) += qS O_l(s-c) + qD (w/2)(nu O_{l-1} - conj(nu) O_{l+1}).
// With z = s - c = (x/omega) u, |u| = 1, O_{+-m} = (+-1)^m H_m u^{+-m} and the
// recurrence H_{m+1} = (2m/x) H_m - H_{m-1}, the dipole pair folds into two
// terms per order.  Writing c = (w/2) qD, v = nu conj(u), A = 2 Re(v) c,
// B = (2/x) c conj(v), B' = (2/x) c v:
//   alpha_0  += qS H_0 - A H_1,
//   alpha_m  += u^m [(qS - m B) H_m + A H_{m-1}],
//   alpha_-m += (-1)^m conj(u)^m [(qS - m B') H_m + A H_{m-1}],   m >= 1,
// so only H_0..H_p are needed.
// ---------------------------------------------------------------------------
template <int PB>
__device__ __forceinline__ void p2qbxl_pair(double omega, int p, double cx, double cy, double sx,
                                            double sy, double nx, double ny, cd qS, cd qD, cd *acc)
{
    double dx = sx - cx, dy = sy - cy;
    double r = sqrt(dx * dx + dy * dy);
    double x = omega * r;
    double ir = 1.0 / r;
    cd u = mk(dx * ir, dy * ir);
    cd H0, H1;
    hankel01(x, H0, H1);
    cd c = (0.5 * omega) * qD;
    cd v = mk(nx, ny) * conj(u);
    cd A = (2.0 * v.x) * c;
    double ix2 = 2.0 / x;
    cd B = ix2 * (c * conj(v));
    cd Bp = ix2 * (c * v);
    {
        cd t = qS * H0;
        cfma(t, neg(A), H1);
        acc[PB] = acc[PB] + t;
    }
    cd Hprev = H0, Hcur = H1;           // H_{m-1}, H_m
    cd cp = qS - B, cm = qS - Bp;       // qS - m B, qS - m B'
    cd up = u;                          // u^m
    // all PB orders, without branches; orders above p are discarded by the caller
#pragma unroll
    for (int m = 1; m <= PB; ++m) {
        cd AH = A * Hprev;
        cd P = AH, M = AH;
        cfma(P, cp, Hcur);
        cfma(M, cm, Hcur);
        cfma(acc[PB + m], up, P);
        cfma(acc[PB - m], (m & 1) ? neg(conj(up)) : conj(up), M);
        if (m < PB) {
            cp = cp - B;
            cm = cm - Bp;
            up = up * u;
            cd Hn = (((double)m * ix2) * Hcur) - Hprev;
            Hprev = Hcur;
            Hcur = Hn;
        }
    }
}

__device__ __forceinline__ double shfl_xor_d(double v, int m)
{
    return __shfl_xor(v, m, 64);
}

template <int PB>
__device__ void p2qbxl_finish(cd *acc, int G, int p, bool write, cd *dst, long long stride, bool add)
{
    // reduce over the lanes that share a centre (lane bits >= log2 G)
#pragma unroll
    for (int e = 0; e < 2 * PB + 1; ++e) {
        double re = acc[e].x, im = acc[e].y;
        for (int m = G; m < 64; m <<= 1) {
            re += shfl_xor_d(re, m);
            im += shfl_xor_d(im, m);
        }
        acc[e] = mk(re, im);
    }
    if (write) {
#pragma unroll
        for (int e = 0; e < 2 * PB + 1; ++e) {
            int ell = e - PB;
            if (ell < -p || ell > p) continue;
            cd *o = dst + (long long)(ell + p) * stride;
            *o = add ? (*o + acc[e]) : acc[e];
        }
    }
}

// One workgroup of P2Q_THREADS lanes per work item (a group of one leaf's
// centres): lane = (centre slot, part) with CG = (centres in the item, at
// most P2Q_THREADS / 2) slots and P2Q_THREADS / CG parts, so few lanes idle
// whatever the centre count.  The leaf's near-list sources (flattened on the
// host) are staged in LDS P2Q_SCH at a time and go round-robin to the parts.
// The parts of a centre are then summed in part order through LDS, P2Q_RED
// coefficients at a time ([coefficient][lane] layout: conflict-free writes
// and reads).  The host splits a leaf into several items when one would give
// a lane many more pairs than the typical leaf.
constexpr int P2Q_SCH = 256;
constexpr int P2Q_RED = 8;         // coefficients per reduction round

size_t p2qbxl_lds_bytes()
{
    return sizeof(cd) * ((size_t)P2Q_RED * P2Q_THREADS + 2 * P2Q_SCH) + sizeof(double) * 4 * P2Q_SCH;
}

template <int PB>
__device__ __forceinline__ void p2qbxl_body(const DevGeom &g, int nd, const int *items, const cd *qs, const cd *qd, cd *coef, BlockId bid)
{
    extern __shared__ double lds_raw[];
    constexpr int NE = 2 * PB + 1;
    cd *red = reinterpret_cast<cd *>(lds_raw);          // [P2Q_RED][P2Q_THREADS]
    cd *QS = red + P2Q_RED * P2Q_THREADS;               // [P2Q_SCH]
    cd *QD = QS + P2Q_SCH;                              // [P2Q_SCH]
    double *SX = reinterpret_cast<double *>(QD + P2Q_SCH);
    double *SY = SX + P2Q_SCH, *NX = SY + P2Q_SCH, *NY = NX + P2Q_SCH;
    const int *it = items + 4 * bid.x;
    int c0 = it[0], c1 = it[1], q0 = it[2], total = it[3] - q0;
    int CG = max(1, min(c1 - c0, P2Q_THREADS / 2));
    int parts = P2Q_THREADS / CG;
    int tid = threadIdx.x;
    int gi = tid % CG, part = tid / CG;
    int p = g.p;
    long long ncoef = 2 * p + 1;
    for (int cg = c0; cg < c1; cg += CG) {
        int i = cg + gi, ncg = min(CG, c1 - cg);
        bool active = part < parts && i < c1;
        double cx = active ? g.cx[i] : 0.0, cy = active ? g.cy[i] : 0.0;
        for (int d = 0; d < nd; ++d) {
            cd acc[NE];
#pragma unroll
            for (int e = 0; e < NE; ++e) acc[e] = mk(0.0, 0.0);
            for (int f0 = 0; f0 < total; f0 += P2Q_SCH) {
                int cnt = min(P2Q_SCH, total - f0);
                __syncthreads();
                for (int f = tid; f < cnt; f += blockDim.x) {
                    int j = g.qsrc_idx[q0 + f0 + f];
                    SX[f] = g.sx[j];
                    SY[f] = g.sy[j];
                    NX[f] = g.snx[j];
                    NY[f] = g.sny[j];
                    QS[f] = qs[(long long)d * g.ns + j];
                    QD[f] = qd[(long long)d * g.ns + j];
                }
                __syncthreads();
                if (active) {
#pragma unroll 1
                    for (int f = part; f < cnt; f += parts)
                        p2qbxl_pair<PB>(g.omega, p, cx, cy, SX[f], SY[f], NX[f], NY[f], QS[f], QD[f], acc);
                }
            }
            // sum the parts of each centre in part order
#pragma unroll
            for (int e0 = 0; e0 < NE; e0 += P2Q_RED) {
                __syncthreads();
#pragma unroll
                for (int e = 0; e < P2Q_RED; ++e)
                    if (e0 + e < NE) red[e * P2Q_THREADS + tid] = acc[e0 + e];
                __syncthreads();
                for (int it = tid; it < ncg * P2Q_RED; it += blockDim.x) {
                    int e = it / ncg, c = it - e * ncg;
                    int ell = e0 + e - PB;
                    if (e0 + e >= NE || ell < -p || ell > p) continue;
                    const cd *r = red + e * P2Q_THREADS + c;
                    cd sum = r[0];
                    for (int jp = 1; jp < parts; ++jp) sum = sum + r[jp * CG];
                    coef[((long long)d * ncoef + ell + p) * g.nc + cg + c] = sum;
                }
            }
        }
    }
}

template <int PB>
__global__ void __launch_bounds__(P2Q_THREADS) k_p2qbxl(DevGeom g, int nd, const int *items, const cd *qs, const cd *qd, cd *coef)
{
    p2qbxl_body<PB>(g, nd, items, qs, qd, coef, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// A capped grid: workgroup b takes items b, 2G-1-b, 2G+b, ... (G = gridDim.x),
// back and forth over the list, which the host sorts by decreasing work, so
// the workgroups' totals stay close.  Each item's body begins and ends its LDS
// use behind barriers, so items follow each other in a workgroup safely.  (The
// loop costs registers, 231 against 228 VGPRs with a little scratch, so
// launches that are not capped take the plain form.)
template <int PB>
__global__ void __launch_bounds__(P2Q_THREADS) k_p2qbxl_capped(DevGeom g, int nd, int n_items, const int *items, const cd *qs, const cd *qd, cd *coef)
{
    int G = gridDim.x;
    for (int r = 0; r * G < n_items; ++r) {
        int b = r * G + ((r & 1) ? G - 1 - (int)blockIdx.x : (int)blockIdx.x);
        if (b < n_items) p2qbxl_body<PB>(g, nd, items, qs, qd, coef, BlockId{b, 0, n_items});
    }
}

// Direct mode: all sources to every centre (Sec. 3.2, oversampled coefficient sum).
template <int PB>
__device__ __forceinline__ void p2qbxl_direct_body(const DevGeom &g, int nd, int G, const cd *qs, const cd *qd, cd *coef, BlockId bid)
{
    int parts = 64 / G;
    int lane = threadIdx.x, gi = lane % G, part = lane / G;
    int i = bid.x * G + gi;
    bool active = i < g.nc;
    int p = g.p;
    long long ncoef = 2 * p + 1;
    double cx = active ? g.cx[i] : 0.0, cy = active ? g.cy[i] : 0.0;
    for (int d = 0; d < nd; ++d) {
        cd acc[2 * PB + 1];
#pragma unroll
        for (int e = 0; e < 2 * PB + 1; ++e) acc[e] = mk(0.0, 0.0);
        if (active)
#pragma unroll 1
            for (int j = part; j < g.ns; j += parts)
                p2qbxl_pair<PB>(g.omega, p, cx, cy, g.sx[j], g.sy[j], g.snx[j], g.sny[j],
                                qs[(long long)d * g.ns + j], qd[(long long)d * g.ns + j], acc);
        p2qbxl_finish<PB>(acc, G, p, active && part == 0,
                          coef + (long long)d * ncoef * g.nc + (active ? i : 0), g.nc, false);
    }
}

template <int PB>
__global__ void __launch_bounds__(64) k_p2qbxl_direct(DevGeom g, int nd, int G, const cd *qs, const cd *qd, cd *coef)
{
    p2qbxl_direct_body<PB>(g, nd, G, qs, qd, coef, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// ---------------------------------------------------------------------------
// Stage 5 (new): M2QBXL.  beta_l(c) += (-1)^l sum_k a_k O_{k+l}(c - m_w) for
// every W box w of the leaf holding c, |l| <= p.
// With z = c - m_w = |z| e^{i theta}, u = e^{i theta}, x = omega |z|,
// tau = min(1, x/2) and the scaled Hankel values Hs_n = tau^n H_n(x), and the
// stored multipole ahat_k = a_k / W_|k|:
//   beta_l = u^l [ (-1)^l tau^{-l} S+_l + tau^l S-_l ],
//   S+_l = sum_{n >= 0} v+_{n-l} Hs_n,  v+_k = ahat_k W_|k| tau^{-k} u^k,
//   S-_l = sum_{n >= 1} v-_{-n-l} Hs_n, v-_k = ahat_k W_|k| tau^{k} (-u)^k,
// (v = 0 outside |k| <= P_w).  The weights W_|k| tau^{-+k} stay <= 1 and are
// carried as running products.  One lane holds 8 consecutive l of one
// centre; the v values enter a sliding register window, so each step costs
// one Hs load and one ahat load for 8 complex multiply-adds.
// ---------------------------------------------------------------------------
constexpr size_t LDS_BUDGET = 64 * 1024;
constexpr int QCG_MAX = 16;   // centres per group (upper bound)

size_t m2qbxl_lds_bytes(int nd, int Pw, int p, int cg)
{
    (void)nd;
    int nw = 2 * Pw + 1, N = Pw + p;
    return sizeof(cd) * ((size_t)nw + (size_t)cg * (N + 1) + cg) +
           sizeof(double) * (2 * (size_t)nw + 3 * (size_t)cg);
}

// One workgroup per (leaf, far W box) pair; lanes = (centre, 8-wide l
// block, quarter of the n range).  The four quarters of an item are adjacent
// lanes and are summed by shuffles; the pair's coefficients go to its own
// output rows (wy), summed per leaf in list order by k_wsum.
constexpr int QSPLIT = 4;

__device__ __forceinline__ void chunk_of(int lo, int hi, int s, int *a, int *b)
{
    int len = hi - lo + 1;
    int cs = (len + QSPLIT - 1) / QSPLIT;
    *a = lo + s * cs;
    *b = min(*a + cs - 1, hi);
}

__device__ __forceinline__ void m2qbxl_body(const DevGeom &g, int nd, const int2 *pairs, const long long *pair_off, const cd *mp, cd *wy, int QCG, BlockId bid)
{
    extern __shared__ double lds_raw[];
    int2 pr = pairs[bid.x];
    int b = pr.x, w = pr.y;
    int c0 = g.ctr_begin[b], c1 = g.ctr_end[b], nct = c1 - c0;
    int p = g.p, nq = 2 * p + 1;
    int nblk = (nq + QBLK - 1) / QBLK;
    int tid = threadIdx.x;
    int lw = g.blev[w];
    int Pw = g.Plev[lw], nw = 2 * Pw + 1;
    int N = Pw + p;
    cd *Aw = reinterpret_cast<cd *>(lds_raw);          // [nw]
    cd *Hs = Aw + nw;                                  // [QCG][N+1]
    cd *U = Hs + QCG * (N + 1);                        // [QCG]
    double *rup = reinterpret_cast<double *>(U + QCG); // [nw], W_|k+1| / W_|k|
    double *rdn = rup + nw;                            // [nw], W_|k-1| / W_|k|
    double *TAU = rdn + nw;                            // [QCG]
    double *LT = TAU + QCG;                            // [QCG]
    double *TH = LT + QCG;                             // [QCG]
    const double *Wt = g.Wtab + g.Woff[lw], *iW = g.invW + g.Woff[lw];
    const double *logW = g.logW + g.Woff[lw];
    for (int i = tid; i < nw; i += blockDim.x) {
        int k = i - Pw, ak = k < 0 ? -k : k;
        int kp = k + 1, km = k - 1;
        rup[i] = k < Pw ? Wt[kp < 0 ? -kp : kp] * iW[ak] : 0.0;
        rdn[i] = k > -Pw ? Wt[km < 0 ? -km : km] * iW[ak] : 0.0;
    }
    double mx = g.bcx[w], my = g.bcy[w];
    cd *out_pair = wy + pair_off[bid.x] * nd;
    // this workgroup's group of centres (bid.y); the Hankel sequences
    // depend on the geometry only and serve every density
    int cg0 = c0 + bid.y * QCG;
    if (cg0 >= c1) return;
    int cnt = min(QCG, c1 - cg0);
    if (tid < cnt) {
        int i = cg0 + tid;
        double dx = g.cx[i] - mx, dy = g.cy[i] - my;
        double r = sqrt(dx * dx + dy * dy);
        double x = g.omega * r;
        double tau = fmin(1.0, 0.5 * x);
        scaled_hankel_seq(x, tau, N, Hs + tid * (N + 1), 1);
        U[tid] = mk(dx / r, dy / r);
        TAU[tid] = tau;
        LT[tid] = log(tau);
        TH[tid] = atan2(dy, dx);
    }
    for (int d = 0; d < nd; ++d) {
        const cd *src = mp + g.box_off[w] * nd + (long long)d * nw;
        {
            __syncthreads();
            for (int i = tid; i < nw; i += blockDim.x) Aw[i] = src[i];
            __syncthreads();
            int items = cnt * nblk;
            for (int it0 = 0; it0 < items; it0 += 256 / QSPLIT) {
                int it = it0 + tid / QSPLIT, sp = tid % QSPLIT;
                bool active = it < items;
                int t = active ? it % cnt : 0;
                int l0 = active ? -p + QBLK * (it / cnt) : -p;
                cd beta[QBLK];
#pragma unroll
                for (int e = 0; e < QBLK; ++e) beta[e] = mk(0.0, 0.0);
                const cd *hs = Hs + t * (N + 1);
                cd u = U[t];
                double tau = TAU[t], lt = LT[t], th = TH[t], itau = 1.0 / tau;
                const cd *A = Aw + Pw;
                const double *ru = rup + Pw, *rd = rdn + Pw;
                cd acc[QBLK], win[QBLK];
                if (active) {
                    // ---- S+ over n in this lane's quarter of [0, nmax] ----
                    int nmax = min(Pw + l0 + QBLK - 1, N);
                    int na, nb;
                    chunk_of(0, nmax, sp, &na, &nb);
#pragma unroll
                    for (int e = 0; e < QBLK; ++e) { acc[e] = mk(0.0, 0.0); win[e] = mk(0.0, 0.0); }
                    if (na <= nb) {
                        int k = na - QBLK - l0;                   // first element
                        int ak = k < 0 ? -k : k;
                        double mag = exp(logW[ak] - k * lt);      // W_|k| tau^{-k}
                        double sn, cs;
                        sincos((double)k * th, &sn, &cs);
                        cd ph = mk(cs, sn);                       // u^k
                        for (int n0 = na - QBLK; n0 <= nb; n0 += QBLK) {
#pragma unroll
                            for (int s = 0; s < QBLK; ++s) {
                                int n = n0 + s;
                                int kk = n - l0;
                                cd v = mk(0.0, 0.0);
                                if (kk >= -Pw && kk <= Pw) {
                                    v = (mag * A[kk]) * ph;
                                    mag *= ru[kk] * itau;
                                }
                                ph = ph * u;
                                win[s] = v;
                                if (n >= na && n <= nb) {
                                    cd h = hs[n];
#pragma unroll
                                    for (int e = 0; e < QBLK; ++e) cfma(acc[e], win[(s - e + QBLK) % QBLK], h);
                                }
                            }
                        }
                    }
                    {
                        double sn0, cs0;
                        sincos((double)l0 * th, &sn0, &cs0);
                        cd ul = mk(cs0, sn0);
                        double f = exp(-l0 * lt);
#pragma unroll
                        for (int e = 0; e < QBLK; ++e) {
                            double fe = ((l0 + e) & 1) ? -f : f;
                            beta[e] = beta[e] + fe * (ul * acc[e]);
                            ul = ul * u;
                            f *= itau;
                        }
                    }
                    // ---- S- over n in this lane's quarter of [1, nmax] ----
                    nmax = min(Pw - l0, N);
                    chunk_of(1, nmax, sp, &na, &nb);
#pragma unroll
                    for (int e = 0; e < QBLK; ++e) { acc[e] = mk(0.0, 0.0); win[e] = mk(0.0, 0.0); }
                    if (na <= nb) {
                        int k = -na - l0;                         // element m = na
                        int ak = k < 0 ? -k : k;
                        double mag = exp(logW[ak] + k * lt);      // W_|k| tau^{k}
                        double sn, cs;
                        sincos((double)k * th, &sn, &cs);
                        cd ph = mk(cs, sn);
                        if (k & 1) ph = neg(ph);                   // (-u)^k
                        cd mub = neg(conj(u));                     // (-u)^{-1}
                        for (int n0 = na - QBLK; n0 <= nb; n0 += QBLK) {
#pragma unroll
                            for (int s = 0; s < QBLK; ++s) {
                                int n = n0 + s;
                                // use elements m = n .. n+7 first: the new one
                                // (m = n + 8) takes the slot of m = n
                                if (n >= na && n <= nb) {
                                    cd h = hs[n];
#pragma unroll
                                    for (int e = 0; e < QBLK; ++e) cfma(acc[e], win[(s + e) % QBLK], h);
                                }
                                int kk = -(n + QBLK) - l0;
                                cd v = mk(0.0, 0.0);
                                if (kk >= -Pw && kk <= Pw) v = (mag * A[kk]) * ph;
                                if (kk > -Pw && kk <= Pw) mag *= rd[kk] * itau;
                                ph = ph * mub;
                                win[s] = v;
                            }
                        }
                    }
                    {
                        double sn0, cs0;
                        sincos((double)l0 * th, &sn0, &cs0);
                        cd ul = mk(cs0, sn0);
                        double f = exp(l0 * lt);
#pragma unroll
                        for (int e = 0; e < QBLK; ++e) {
                            beta[e] = beta[e] + f * (ul * acc[e]);
                            ul = ul * u;
                            f *= tau;
                        }
                    }
                }
                // sum the quarters (adjacent lanes)
#pragma unroll
                for (int e = 0; e < QBLK; ++e) {
                    double re = beta[e].x, im = beta[e].y;
                    for (int m = 1; m < QSPLIT; m <<= 1) {
                        re += __shfl_xor(re, m, 64);
                        im += __shfl_xor(im, m, 64);
                    }
                    beta[e] = mk(re, im);
                }
                if (active && sp == 0) {
                    int ci = cg0 - c0 + t;
                    cd *o = out_pair + ((long long)d * nct + ci) * nq;
#pragma unroll
                    for (int e = 0; e < QBLK; ++e) {
                        int ell = l0 + e;
                        if (ell <= p) o[ell + p] = beta[e];
                    }
                }
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_m2qbxl(DevGeom g, int nd, const int2 *pairs, const long long *pair_off, const cd *mp, cd *wy, int QCG)
{
    m2qbxl_body(g, nd, pairs, pair_off, mp, wy, QCG, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// coef[d][l][i] += sum over the leaf's far-W pairs (list order) of their rows.
__device__ __forceinline__ void wsum_body(const DevGeom &g, int nd, const int *leaf_list, const int *leaf_pair_start, const long long *pair_off, const cd *wy, cd *coef, BlockId bid)
{
    int li = bid.x;
    int b = leaf_list[li];
    int c0 = g.ctr_begin[b], nct = g.ctr_end[b] - c0;
    int p = g.p, nq = 2 * p + 1;
    int q0 = leaf_pair_start[li], np_ = leaf_pair_start[li + 1] - q0;
    // the leaf's pair rows follow each other, nct * nq * nd apart
    const cd *wr = wy + pair_off[q0] * nd;
    long long ws = (long long)nct * nq * nd;
    for (int idx = threadIdx.x; idx < nd * nct * nq; idx += blockDim.x) {
        int d = idx / (nct * nq), rem = idx % (nct * nq);
        int ci = rem / nq, l = rem % nq;
        cd acc = mk(0.0, 0.0);
#pragma unroll 4
        for (int q = 0; q < np_; ++q) acc = acc + wr[q * ws + idx];
        cd *o = coef + ((long long)d * nq + l) * g.nc + c0 + ci;
        *o = *o + acc;
    }
}

__global__ void k_wsum(DevGeom g, int nd, const int *leaf_list, const int *leaf_pair_start, const long long *pair_off, const cd *wy, cd *coef)
{
    wsum_body(g, nd, leaf_list, leaf_pair_start, pair_off, wy, coef, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// ---------------------------------------------------------------------------
// L2QBXL: gamma_l(c) += sum_k g_k I_{l-k}(z), z = m_b - c, with the box local
// g_k = ghat_k / W_|k|.  Writing z = (x/omega) u, |u| = 1, and
// I_n(z) = J_n(x) u^n with J_{-n} = (-1)^n J_n,
//   gamma_l = u^l sum_n gt_{l-n} J_n(x),   gt_k = g_k conj(u)^k,
// a real-by-complex correlation.  One lane holds 8 consecutive l of one
// centre and a quarter of the n range; gt enters a sliding register window
// (its phase is a running product), J_n comes from an LDS table filled by
// Miller's recurrence, one lane per centre.
//
// Work items pack centres: an item is up to L2Q_SEGS runs of consecutive
// centres, each run inside one leaf, at most `cap` centres in all (the host
// splits large leaves into runs and packs the runs, largest first, best
// fit).  A leaf's centres alone would leave a third of the lanes idle on a
// typical curve (about 11 centres per leaf against 16 slots).  Each centre's
// arithmetic is the same whichever item it lands in.
// ---------------------------------------------------------------------------
constexpr int L2Q_THREADS = 256;   // lanes per item: 16 slots x 4 l-blocks x 4 quarters

size_t l2qbxl_lds_bytes(int P, int cap, int rows)
{
    // one density's locals of every run, the centres' directions, their J_n rows
    return sizeof(cd) * ((size_t)L2Q_SEGS * (2 * P + 1) + (size_t)cap) + sizeof(double) * (size_t)cap * rows;
}

int l2qbxl_item_cap(int Pmax, int rows)
{
    int cap = L2Q_CAP_MAX;
    while (cap > 1 && l2qbxl_lds_bytes(Pmax, cap, rows) > LDS_BUDGET) cap >>= 1;
    return cap;
}

__device__ __forceinline__ void l2qbxl_body(const DevGeom &g, int nd, const int *items, const double *crad,
                                            const cd *loc, cd *coef, int cap, int rows, BlockId bid)
{
    extern __shared__ double lds_raw[];
    const int *it = items + 2 * L2Q_SEGS * bid.x;
    // runs: centres [c0, c1) of leaf b, slots [so, so + c1 - c0), locals at Gb + go
    int rc0[L2Q_SEGS], rb[L2Q_SEGS], rP[L2Q_SEGS], so[L2Q_SEGS + 1], go[L2Q_SEGS];
    int T = 0, gsum = 0;
#pragma unroll
    for (int r = 0; r < L2Q_SEGS; ++r) {
        int c0 = it[2 * r], c1 = it[2 * r + 1];
        rc0[r] = c0;
        so[r] = T;
        go[r] = gsum;
        rb[r] = c1 > c0 ? g.ctr_box[c0] : 0;
        rP[r] = c1 > c0 ? g.Plev[g.blev[rb[r]]] : 0;
        if (c1 > c0) {
            T += c1 - c0;
            gsum += 2 * rP[r] + 1;
        }
    }
    so[L2Q_SEGS] = T;
    int p = g.p, nq = 2 * p + 1;
    int nblk = (nq + QBLK - 1) / QBLK;
    int tid = threadIdx.x;
    cd *Gb = reinterpret_cast<cd *>(lds_raw);          // [gsum]: run r's local at go[r]
    cd *U = Gb + gsum;                                 // [cap]
    double *Jt = reinterpret_cast<double *>(U + cap);  // [cap][rows]
    auto run_of = [&](int t) {
        int r = 0;
#pragma unroll
        for (int q = 1; q < L2Q_SEGS; ++q) r += t >= so[q];
        return r;
    };
    for (int t = tid; t < T; t += blockDim.x) {
        int r = run_of(t), b = rb[r], i = rc0[r] + t - so[r];
        double dx = g.bcx[b] - g.cx[i], dy = g.bcy[b] - g.cy[i];
        double rr = sqrt(dx * dx + dy * dy);
        U[t] = rr > 0.0 ? mk(dx / rr, dy / rr) : mk(1.0, 0.0);
    }
    for (int i = tid; i < T * rows; i += blockDim.x) {
        int n = i / T, t = i - n * T;
        int r = run_of(t);
        if (n <= rP[r] + p + QBLK - 1)
            Jt[t * rows + n] = crad[(long long)n * g.nc + rc0[r] + t - so[r]];
    }
    for (int d = 0; d < nd; ++d) {
        if (d > 0) __syncthreads();                    // the previous density's readers are done
        for (int i = tid; i < gsum; i += blockDim.x) {
            int r = 0;
#pragma unroll
            for (int q = 1; q < L2Q_SEGS; ++q) r += i >= go[q] && so[q] < T;
            int P = rP[r], np = 2 * P + 1, k = i - go[r] - P;
            const double *iw = g.invW + g.Woff[g.blev[rb[r]]];
            Gb[i] = iw[k < 0 ? -k : k] * loc[g.box_off[rb[r]] * nd + (long long)d * np + k + P];
        }
        __syncthreads();
        int nitems = T * nblk;
        for (int it0 = 0; it0 < nitems; it0 += (int)blockDim.x / QSPLIT) {
            int iq = it0 + tid / QSPLIT, sp = tid % QSPLIT;
            bool active = iq < nitems;
            int t = active ? iq % T : 0;
            int l0 = -p + QBLK * (active ? iq / T : 0);
            int r = run_of(t);
            int P = rP[r];
            cd acc[QBLK], win[QBLK];
#pragma unroll
            for (int e = 0; e < QBLK; ++e) { acc[e] = mk(0.0, 0.0); win[e] = mk(0.0, 0.0); }
            const double *jt = Jt + t * rows;
            const cd *G = Gb + go[r] + P;
            cd u = U[t];
            int ci = rc0[r] + t - so[r];
            if (active) {
                int na, nb;
                chunk_of(l0 - P, l0 + QBLK - 1 + P, sp, &na, &nb);
                if (na <= nb) {
                    int k = l0 - (na - QBLK);                 // element of the first step
                    cd ph = unit_ipow(conj(u), k);            // conj(u)^k
#pragma unroll 1
                    for (int n0 = na - QBLK; n0 <= nb; n0 += QBLK) {
#pragma unroll
                        for (int s = 0; s < QBLK; ++s) {
                            int n = n0 + s;
                            int kk = l0 - n;
                            cd v = mk(0.0, 0.0);
                            if (kk >= -P && kk <= P) v = G[kk] * ph;
                            ph = ph * u;
                            win[s] = v;
                            if (n >= na && n <= nb) {
                                int an = n < 0 ? -n : n;
                                double jn = jt[an];
                                if (n < 0 && (an & 1)) jn = -jn;
#pragma unroll
                                for (int e = 0; e < QBLK; ++e) {
                                    cd w = win[(s - e + QBLK) % QBLK];
                                    acc[e].x = fma(w.x, jn, acc[e].x);
                                    acc[e].y = fma(w.y, jn, acc[e].y);
                                }
                            }
                        }
                    }
                }
            }
            // sum the quarters (adjacent lanes)
#pragma unroll
            for (int e = 0; e < QBLK; ++e) {
                double re = acc[e].x, im = acc[e].y;
                for (int m = 1; m < QSPLIT; m <<= 1) {
                    re += __shfl_xor(re, m, 64);
                    im += __shfl_xor(im, m, 64);
                }
                acc[e] = mk(re, im);
            }
            if (active && sp == 0) {
                cd ul = unit_ipow(u, l0);                     // u^l
#pragma unroll
                for (int e = 0; e < QBLK; ++e) {
                    int ell = l0 + e;
                    if (ell <= p) {
                        cd *o = coef + ((long long)d * nq + ell + p) * g.nc + ci;
                        *o = *o + ul * acc[e];
                    }
                    ul = ul * u;
                }
            }
        }
    }
}

__global__ void __launch_bounds__(L2Q_THREADS) k_l2qbxl(DevGeom g, int nd, const int *items, const double *crad, const cd *loc, cd *coef, int cap, int rows)
{
    l2qbxl_body(g, nd, items, crad, loc, coef, cap, rows, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// ---------------------------------------------------------------------------
// QBX evaluation at associated targets: u = sum_{|l|<=p} alpha_l J_l(w rho) e^{-i l theta}.
// Miller's recurrence runs downward and the series is summed on the fly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void qbx_eval_body(const DevGeom &g, int nd, const cd *coef, cd *u, BlockId bid)
{
    int m = bid.x * blockDim.x + threadIdx.x;
    if (m >= g.nt) return;
    int i = g.tgt_cs[m];
    if (i < 0) return;
    int p = g.p;
    long long nq = 2 * p + 1;
    double dx = g.tx[m] - g.cx[i], dy = g.ty[m] - g.cy[i];
    double rho = sqrt(dx * dx + dy * dy);
    double x = g.omega * rho;
    cd v = rho > 0.0 ? mk(dx / rho, dy / rho) : mk(1.0, 0.0);    // e^{i theta}
    long long o = g.tgt_out ? (long long)g.tgt_out[m] : (long long)m;
    for (int d = 0; d < nd; ++d) {
        const cd *a = coef + (long long)d * nq * g.nc + i;
        cd a0 = a[(long long)p * g.nc];
        if (x == 0.0) {
            u[(long long)d * g.u_stride + o] = a0;
            continue;
        }
        int M = miller_start(x, p);
        double inv = 2.0 / x;
        double fp1 = 0.0, f = 1e-280, f1 = 0.0;
        cd S = mk(0.0, 0.0);
        cd ep = unit_ipow(conj(v), p);  // e^{-i n theta} at n = p, stepped down with n
        for (int n = M; n > 0; --n) {
            if (n <= p) {
                cd t = a[(long long)(p + n) * g.nc] * ep;
                cd tm = a[(long long)(p - n) * g.nc] * conj(ep);
                if (n & 1) tm = neg(tm);
                S = S + f * (t + tm);
                ep = ep * v;
            }
            if (n == 1) f1 = f;
            double fm = (n * inv) * f - fp1;
            fp1 = f;
            f = fm;
            if (fabs(f) > 1e250) {
                f *= 1e-250; fp1 *= 1e-250; f1 *= 1e-250;
                S = 1e-250 * S;
            }
        }
        double jz = j0(x), jo = j1(x);
        double s = fabs(jz) >= fabs(jo) ? jz / f : jo / f1;
        u[(long long)d * g.u_stride + o] = s * S + jz * a0;
    }
}

__global__ void k_qbx_eval(DevGeom g, int nd, const cd *coef, cd *u)
{
    qbx_eval_body(g, nd, coef, u, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// Smooth (unmodified Gauss) rule at unassociated targets, over all sources.
// One wave per smooth-rule target: lane i takes sources i, i + 64, ...,
// evaluates each Hankel pair once for all densities of the pass, and the
// wave sums its lanes by a fixed butterfly.
constexpr int SMOOTH_ND = 4;                  // densities per pass (the pipeline's chunk)

__device__ __forceinline__ void smooth_body(const DevGeom &g, int nd, const cd *qs, const cd *qd, cd *u, BlockId bid)
{
    int idx = bid.x;
    if (idx >= g.n_smooth) return;                    // uniform across the wave
    int lane = threadIdx.x;
    int m = g.smooth_list[idx];
    double tx = g.tx[m], ty = g.ty[m];
    for (int d0 = 0; d0 < nd; d0 += SMOOTH_ND) {
        int dn = min(SMOOTH_ND, nd - d0);
        cd acc[SMOOTH_ND];
#pragma unroll
        for (int e = 0; e < SMOOTH_ND; ++e) acc[e] = mk(0.0, 0.0);
        for (int j = lane; j < g.ns; j += 64) {
            double dx = tx - g.sx[j], dy = ty - g.sy[j];
            double r = sqrt(dx * dx + dy * dy);
            double x = g.omega * r;
            cd h0, h1;
            hankel01(x, h0, h1);
            cd dh = (g.omega * (dx * g.snx[j] + dy * g.sny[j]) / r) * h1;
#pragma unroll
            for (int e = 0; e < SMOOTH_ND; ++e)
                if (e < dn) {
                    cfma(acc[e], qs[(long long)(d0 + e) * g.ns + j], h0);
                    cfma(acc[e], qd[(long long)(d0 + e) * g.ns + j], dh);
                }
        }
#pragma unroll
        for (int e = 0; e < SMOOTH_ND; ++e) {
            double re = acc[e].x, im = acc[e].y;
            for (int s = 32; s > 0; s >>= 1) {
                re += __shfl_xor(re, s, 64);
                im += __shfl_xor(im, s, 64);
            }
            if (lane == 0 && e < dn) u[(long long)(d0 + e) * g.nt + m] = mk(re, im);
        }
    }
}

__global__ void __launch_bounds__(64) k_smooth(DevGeom g, int nd, const cd *qs, const cd *qd, cd *u)
{
    smooth_body(g, nd, qs, qd, u, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}

// coef_user[d][l][user(i)] = coef[d][l][i]
__device__ __forceinline__ void coef_out_body(const DevGeom &g, int nd, const cd *coef, cd *out, BlockId bid)
{
    long long idx = (long long)bid.x * blockDim.x + threadIdx.x;
    long long nq = 2 * g.p + 1;
    long long n = nd * nq * g.nc;
    if (idx >= n) return;
    long long row = idx / g.nc;
    int i = (int)(idx % g.nc);
    out[row * g.nc + g.ctr_perm[i]] = coef[idx];
}

__global__ void k_coef_out(DevGeom g, int nd, const cd *coef, cd *out)
{
    coef_out_body(g, nd, coef, out, BlockId{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x});
}


// ---------------------------------------------------------------------------
// Fused launches (one grid per stage over several geometries)
// ---------------------------------------------------------------------------
// Records, maps and geometry views are read through the constant address
// space: they are never written while a launch runs, so the loads are
// scalar and the values stay in scalar registers, as kernel arguments do.
#ifdef __HIP_DEVICE_COMPILE__
#define QBX_CONST __attribute__((address_space(4)))
#else
#define QBX_CONST
#endif

__device__ __forceinline__ FRec fused_rec(const FRec *recs, const int *map, BlockId &bid)
{
    int gi = __builtin_amdgcn_readfirstlane(((const QBX_CONST int *)map)[blockIdx.x]);
    FRec r = ((const QBX_CONST FRec *)recs)[gi];
    int loc = (int)blockIdx.x - r.first;
    bid.x = loc % r.nx;
    bid.y = loc / r.nx;
    bid.nx = r.nx;
    return r;
}

// The geometry's view is copied at the top, before any store, so its fields
// load once like kernel arguments.
#define FUSED_BEGIN                                     \
    BlockId bid;                                        \
    const FRec r = fused_rec(recs, map, bid);           \
    const DevGeom g = *(const QBX_CONST DevGeom *)r.g;

#define CP(T, x) ((T)(r.x))

__global__ void kf_fill(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    (void)g;
    fill_zero_body(CP(cd *, out0), r.n64, bid);
}

__global__ void kf_charges(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    charges_body(g, r.nd, CP(const cd *, in0), CP(const cd *, in1), CP(cd *, out0), CP(cd *, out1), bid);
}

__global__ void kf_src_bas(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    src_bas_body(g, CP(cd *, out0), bid);
}

__global__ void kf_x_bas(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    x_bas_body(g, (int)r.n64, CP(cd *, out0), bid);
}

__global__ void kf_ctr_rad(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    ctr_rad_body(g, r.i0, CP(double *, out0), bid);
}

template <int ND>
__global__ void __launch_bounds__(64) kf_p2m(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    p2m_body<ND>(g, CP(const int *, in0), CP(const cd *, in1), CP(const cd *, in2), CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(256 * M2M_KS) kf_m2m(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    m2m_mfma_body(g, r.nd, r.i0, CP(const TTile *, in0), CP(const int *, in1), CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(1024) kf_m2l(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    m2l_mfma_body(g, r.nd, CP(const M2LTile *, in0), CP(const cd *, in1), CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(64) kf_m2l_direct(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    m2l_mfma_direct_body(g, r.nd, CP(const M2LTile *, in0), r.i0, CP(const cd *, in1), CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(64) kf_m2l32(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    m2l_mfma32_body(g, r.nd, CP(const M2LTile *, in0), r.i0, CP(const cd *, in1), CP(cd *, out0), bid);
}

__global__ void kf_down(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    down_body(g, r.nd, r.i0, CP(const cd *, in0), CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(64 * L2L_KS) kf_l2l(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    l2l_mfma_body(g, r.nd, r.i0, CP(const TTile *, in0), CP(const int *, in1), CP(const cd *, in2),
                  CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(64 * L2L_KS) kf_l2l32(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    l2l_mfma32_body(g, r.nd, r.i0, CP(const TTile *, in0), CP(const cd *, in2), CP(cd *, out0), bid);
}

template <int ND>
__global__ void __launch_bounds__(64) kf_p2l_x(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    p2l_x_body<ND>(g, CP(const int *, in0), CP(const cd *, in1), CP(const cd *, in2), CP(cd *, out0), r.i0, bid);
}

template <int ND>
__global__ void __launch_bounds__(64) kf_p2l_xc(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    p2l_xc_body<ND>(g, CP(const int *, in0), CP(const cd *, in1), CP(const cd *, in2), CP(cd *, out0), bid);
}

template <int PB>
__global__ void __launch_bounds__(P2Q_THREADS) kf_p2qbxl(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    p2qbxl_body<PB>(g, r.nd, CP(const int *, in0), CP(const cd *, in1), CP(const cd *, in2), CP(cd *, out0), bid);
}

template <int PB>
__global__ void __launch_bounds__(64) kf_p2qbxl_direct(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    p2qbxl_direct_body<PB>(g, r.nd, r.i0, CP(const cd *, in0), CP(const cd *, in1), CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(256) kf_m2qbxl(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    m2qbxl_body(g, r.nd, CP(const int2 *, in0), CP(const long long *, in1), CP(const cd *, in2), CP(cd *, out0),
                r.i0, bid);
}

__global__ void kf_wsum(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    wsum_body(g, r.nd, CP(const int *, in0), CP(const int *, in1), CP(const long long *, in2), CP(const cd *, in3),
              CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(L2Q_THREADS) kf_l2qbxl(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    l2qbxl_body(g, r.nd, CP(const int *, in0), CP(const double *, in1), CP(const cd *, in2), CP(cd *, out0), r.i0,
                (int)r.n64, bid);
}

__global__ void kf_eval(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    qbx_eval_body(g, r.nd, CP(const cd *, in0), CP(cd *, out0), bid);
}

__global__ void __launch_bounds__(64) kf_smooth(const FRec *recs, const int *map)
{
    FUSED_BEGIN
    smooth_body(g, r.nd, CP(const cd *, in0), CP(const cd *, in1), CP(cd *, out0), bid);
}

#undef CP
#undef FUSED_BEGIN

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define QBX_LAUNCH_CHECK()                                   \
    do {                                                     \
        hipError_t e_ = hipGetLastError();                   \
        if (e_ != hipSuccess) return e_;                     \
    } while (0)

hipError_t launch_fill_zero(cd *p, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    k_fill_zero<<<blocks, 256, 0, s>>>(p, n);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_charges(const DevGeom &g, int nd, const cd *ss, const cd *sd, cd *qs, cd *qd,
                          hipStream_t s)
{
    long long n = (long long)nd * g.ns;
    if (n == 0) return hipSuccess;
    k_charges<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, nd, ss, sd, qs, qd);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

// Sources per pass, sized for the largest density count so that the order
// of the sums (and so every bit of the result) does not depend on how many
// densities share a launch.
static int pick_ch(int Pmax)
{
    int ch = 64;
    while (ch > 1 && ptab_lds_bytes(4, Pmax, ch) > PT_LDS) --ch;
    return ch;
}

hipError_t launch_src_bas(const DevGeom &g, cd *sbas, hipStream_t s)
{
    if (!g.ns) return hipSuccess;
    int lanes = rad_lanes(g.srow);
    k_src_bas<<<(g.ns + lanes - 1) / lanes, lanes, (size_t)g.srow * lanes * sizeof(double), s>>>(g, sbas);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_x_bas(const DevGeom &g, int nx, cd *xbas, hipStream_t s)
{
    if (nx <= 0 || !xbas) return hipSuccess;    // no kept rows: P2L builds them itself
    k_x_bas<<<(nx + 63) / 64, 64, 0, s>>>(g, nx, xbas);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_p2m(const DevGeom &g, int nd, const int *list, int n, int Pmax, const cd *qs,
                      const cd *qd, cd *mp, hipStream_t s)
{
    if (!n) return hipSuccess;
    if (nd < 1 || nd > 4) return hipErrorInvalidValue;
    if (!g.sbas) return hipErrorInvalidValue;
    dim3 grid(n, half_order_runs(Pmax));
    size_t lds = p2m_lds_bytes(nd);
    switch (nd) {
    case 1: k_p2m<1><<<grid, 64, lds, s>>>(g, list, qs, qd, mp); break;
    case 2: k_p2m<2><<<grid, 64, lds, s>>>(g, list, qs, qd, mp); break;
    case 3: k_p2m<3><<<grid, 64, lds, s>>>(g, list, qs, qd, mp); break;
    default: k_p2m<4><<<grid, 64, lds, s>>>(g, list, qs, qd, mp); break;
    }
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

// Compute units of the current device (cached per device).
static int device_cu_count()
{
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

hipError_t launch_m2m_mfma(const DevGeom &g, int nd, int l, const TTile *tiles, int ntiles,
                           int nrb, const int *plist, cd *mp, hipStream_t s)
{
    if (!ntiles) return hipSuccess;
    k_m2m_mfma<<<dim3(ntiles, nrb), 256 * M2M_KS, 0, s>>>(g, nd, l, tiles, plist, mp);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_l2l_mfma(const DevGeom &g, int nd, int L, const TTile *tiles, int ntiles, int nrb,
                           const int *clist, const cd *vy, cd *loc, hipStream_t s)
{
    if (!ntiles) return hipSuccess;
    if (g.far32) k_l2l_mfma32<<<dim3(ntiles, nrb), 64 * L2L_KS, 0, s>>>(g, nd, L, tiles, vy, loc);
    else k_l2l_mfma<<<dim3(ntiles, nrb), 64 * L2L_KS, 0, s>>>(g, nd, L, tiles, clist, vy, loc);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

static size_t m2l_staged_lds(int P) { return sizeof(cd) * 4 * ((2 * (size_t)P + 1 + 3) / 4) * M2L_XS; }

int m2l_staged_pmax()
{
    int P = 0;
    while (m2l_staged_lds(P + 1) <= LDS_BUDGET) ++P;
    return P;
}

hipError_t launch_m2l_mfma(const DevGeom &g, int nd, const M2LTile *tiles, int ntiles, int nsplit,
                           int Pdirect, int Pstaged, int nw, const cd *mp, cd *vy, hipStream_t s)
{
    if (!ntiles) return hipSuccess;
    int Pmax = std::max(Pdirect, Pstaged);
    auto direct = [&](const M2LTile *t, int n, int P) -> hipError_t {
        int nrmax = (2 * P + 1 + 15) / 16;
        long long nblk = (long long)n * nrmax;
        if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
        if (nblk > 0) k_m2l_mfma_direct<<<(unsigned)nblk, 64, 0, s>>>(g, nd, t, nrmax, mp, vy);
        return hipSuccess;
    };
    if (g.far32) {
        int nrmax = (2 * Pmax + 1 + 15) / 16;
        long long nblk = (long long)ntiles * nrmax;
        if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
        k_m2l_mfma32<<<(unsigned)nblk, 64, 0, s>>>(g, nd, tiles, nrmax, mp, vy);
    } else if (nw > 0) {
        nw = std::min(nw, 16);
        hipError_t e = direct(tiles, nsplit, Pdirect);
        if (e != hipSuccess) return e;
        if (ntiles > nsplit) {
            size_t lds = m2l_staged_lds(Pstaged);
            if (lds > LDS_BUDGET) return hipErrorInvalidValue;
            k_m2l_mfma<<<ntiles - nsplit, 64 * nw, lds, s>>>(g, nd, tiles + nsplit, mp, vy);
        }
    } else {
        hipError_t e = direct(tiles, ntiles, Pmax);
        if (e != hipSuccess) return e;
    }
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_down_all(const DevGeom &g, int nd, int nbox, const cd *vy, cd *loc, hipStream_t s)
{
    if (!nbox) return hipSuccess;
    if (nd < 1 || nd > 4) return hipErrorInvalidValue;
    k_down_all<<<nbox, 64 * nd, 0, s>>>(g, nd, vy, loc);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

// The X-list P2L beside the other stream, like the near field after it, is
// capped so that the first M2M levels and P2M find room: 4 waves per CU (one
// per SIMD), while the launch has at most 32 waves per CU (the star: 2466
// boxes x 2 runs of orders, 19 per CU).  Step 0.446 to 0.440 ms; 2 waves per
// CU: 0.475 ms.
#ifndef XC_WAVES_PER_CU
#define XC_WAVES_PER_CU 4
#endif
constexpr int XC_CAP_WAVES_PER_CU = 32;

hipError_t launch_p2l_x(const DevGeom &g, int nd, const int *list, int n, int Pmax, const cd *qs,
                        const cd *qd, cd *loc, bool beside, hipStream_t s)
{
    if (!n) return hipSuccess;
    if (nd < 1 || nd > 4) return hipErrorInvalidValue;
    if (g.xbas) {
        // rows kept with the geometry (launch_x_bas)
        int runs = order_runs(Pmax), cus = device_cu_count();
        size_t lds = p2l_xc_lds_bytes(nd);
        if (beside && XC_WAVES_PER_CU > 0 && (long long)n * runs <= (long long)XC_CAP_WAVES_PER_CU * cus) {
            dim3 grid(std::min(n, std::max(1, XC_WAVES_PER_CU * cus / runs)), runs);
            switch (nd) {
            case 1: k_p2l_xc_capped<1><<<grid, 64, lds, s>>>(g, n, list, qs, qd, loc); break;
            case 2: k_p2l_xc_capped<2><<<grid, 64, lds, s>>>(g, n, list, qs, qd, loc); break;
            case 3: k_p2l_xc_capped<3><<<grid, 64, lds, s>>>(g, n, list, qs, qd, loc); break;
            default: k_p2l_xc_capped<4><<<grid, 64, lds, s>>>(g, n, list, qs, qd, loc); break;
            }
            QBX_LAUNCH_CHECK();
            return hipSuccess;
        }
        dim3 grid(n, runs);
        switch (nd) {
        case 1: k_p2l_xc<1><<<grid, 64, lds, s>>>(g, list, qs, qd, loc); break;
        case 2: k_p2l_xc<2><<<grid, 64, lds, s>>>(g, list, qs, qd, loc); break;
        case 3: k_p2l_xc<3><<<grid, 64, lds, s>>>(g, list, qs, qd, loc); break;
        default: k_p2l_xc<4><<<grid, 64, lds, s>>>(g, list, qs, qd, loc); break;
        }
        QBX_LAUNCH_CHECK();
        return hipSuccess;
    }
    int ch = pick_ch(Pmax);
    size_t lds = ptab_lds_bytes(nd, Pmax, ch);
    if (lds > LDS_BUDGET) return hipErrorInvalidValue;
    switch (nd) {
    case 1: k_p2l_x<1><<<n, 64, lds, s>>>(g, list, qs, qd, loc, ch); break;
    case 2: k_p2l_x<2><<<n, 64, lds, s>>>(g, list, qs, qd, loc, ch); break;
    case 3: k_p2l_x<3><<<n, 64, lds, s>>>(g, list, qs, qd, loc, ch); break;
    default: k_p2l_x<4><<<n, 64, lds, s>>>(g, list, qs, qd, loc, ch); break;
    }
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

// Workgroups per CU of the near-field launch when it runs beside the other
// stream.  At 228 VGPRs a lane two of its waves fill a SIMD's registers; with
// one workgroup per item the near field takes every CU, and the latency-bound
// M2M levels of the other stream wait for it to drain before their workgroups
// get one.  Two workgroups per CU (one wave per SIMD) leave room for them.
// Measured on the 32768-node star: 0.470 ms a step against 0.487-0.490 with
// one workgroup per item (1: 0.522, 3: 0.495, 4: 0.486).  Alone on the
// device (in order) the launch takes one workgroup per item.
#ifndef P2Q_WG_PER_CU
#define P2Q_WG_PER_CU 2
#endif
// The cap pays only while the near field is short next to the other
// stream's chain (the 32768-node star: 3454 items, 13.5 per CU).  With many
// items per CU, as on the 606k-node multiscale set with leaves of 64, the
// near field is the longer stream, and capped it becomes the critical path.
#ifndef P2Q_CAP_ITEMS_PER_CU
#define P2Q_CAP_ITEMS_PER_CU 16
#endif


template <int PB>
static hipError_t p2qbxl_dispatch(const DevGeom &g, int nd, const int *items, int n, const cd *qs,
                                  const cd *qd, cd *coef, bool beside, hipStream_t s)
{
    int cus = device_cu_count();
    if (beside && P2Q_WG_PER_CU > 0 && n <= P2Q_CAP_ITEMS_PER_CU * cus)
        k_p2qbxl_capped<PB><<<std::min(n, P2Q_WG_PER_CU * cus), P2Q_THREADS, p2qbxl_lds_bytes(), s>>>(
            g, nd, n, items, qs, qd, coef);
    else
        k_p2qbxl<PB><<<n, P2Q_THREADS, p2qbxl_lds_bytes(), s>>>(g, nd, items, qs, qd, coef);
    return hipGetLastError();
}

hipError_t launch_p2qbxl(const DevGeom &g, int nd, const int *items, int n, const cd *qs,
                         const cd *qd, cd *coef, bool beside, hipStream_t s)
{
    if (!n) return hipSuccess;
    if (g.p <= 8) return p2qbxl_dispatch<8>(g, nd, items, n, qs, qd, coef, beside, s);
    if (g.p <= 12) return p2qbxl_dispatch<12>(g, nd, items, n, qs, qd, coef, beside, s);
    if (g.p <= 14) return p2qbxl_dispatch<14>(g, nd, items, n, qs, qd, coef, beside, s);
    if (g.p <= 16) return p2qbxl_dispatch<16>(g, nd, items, n, qs, qd, coef, beside, s);
    if (g.p <= 24) return p2qbxl_dispatch<24>(g, nd, items, n, qs, qd, coef, beside, s);
    if (g.p <= 32) return p2qbxl_dispatch<32>(g, nd, items, n, qs, qd, coef, beside, s);
    return p2qbxl_dispatch<40>(g, nd, items, n, qs, qd, coef, beside, s);
}

// Centres per wave of the direct sum: one when there are few centres (the
// sources of each then spread over all 64 lanes, and the grid has a wave per
// centre), four for large sets.
static int direct_centres_per_wave(long long nc) { return nc >= 16384 ? 4 : (nc >= 4096 ? 2 : 1); }

template <int PB>
static hipError_t p2qbxl_direct_dispatch(const DevGeom &g, int nd, const cd *qs, const cd *qd,
                                         cd *coef, hipStream_t s)
{
    int G = direct_centres_per_wave(g.nc);
    int blocks = (g.nc + G - 1) / G;
    k_p2qbxl_direct<PB><<<blocks, 64, 0, s>>>(g, nd, G, qs, qd, coef);
    return hipGetLastError();
}

hipError_t launch_p2qbxl_direct(const DevGeom &g, int nd, const cd *qs, const cd *qd, cd *coef,
                                hipStream_t s)
{
    if (!g.nc) return hipSuccess;
    if (g.p <= 8) return p2qbxl_direct_dispatch<8>(g, nd, qs, qd, coef, s);
    if (g.p <= 12) return p2qbxl_direct_dispatch<12>(g, nd, qs, qd, coef, s);
    if (g.p <= 14) return p2qbxl_direct_dispatch<14>(g, nd, qs, qd, coef, s);
    if (g.p <= 16) return p2qbxl_direct_dispatch<16>(g, nd, qs, qd, coef, s);
    if (g.p <= 24) return p2qbxl_direct_dispatch<24>(g, nd, qs, qd, coef, s);
    if (g.p <= 32) return p2qbxl_direct_dispatch<32>(g, nd, qs, qd, coef, s);
    return p2qbxl_direct_dispatch<40>(g, nd, qs, qd, coef, s);
}

static int pick_cg(size_t (*bytes)(int, int, int, int), int nd, int P, int p)
{
    int cg = QCG_MAX;
    while (cg > 1 && bytes(nd, P, p, cg) > LDS_BUDGET) cg >>= 1;
    return cg;
}

hipError_t launch_m2qbxl(const DevGeom &g, int nd, const int2 *pairs, const long long *pair_off,
                         int npairs, int PWmax, const cd *mp, cd *wy, const int *leaf_list,
                         const int *leaf_pair_start, int nleaf, cd *coef, hipStream_t s)
{
    if (!npairs) return hipSuccess;
    int cg = 16;
    while (cg > 1 && m2qbxl_lds_bytes(nd, PWmax, g.p, cg) > LDS_BUDGET) cg >>= 1;
    size_t lds = m2qbxl_lds_bytes(nd, PWmax, g.p, cg);
    if (lds > LDS_BUDGET) return hipErrorInvalidValue;
    // centre groups per leaf: at most ceil(max centres per leaf / cg)
    k_m2qbxl<<<dim3(npairs, (g.max_leaf_ctr + cg - 1) / cg), 256, lds, s>>>(g, nd, pairs, pair_off, mp, wy, cg);
    QBX_LAUNCH_CHECK();
    k_wsum<<<nleaf, 256, 0, s>>>(g, nd, leaf_list, leaf_pair_start, pair_off, wy, coef);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_ctr_rad(const DevGeom &g, int nleaf, double *crad, int crad_rows, hipStream_t s)
{
    if (!nleaf || !g.nc) return hipSuccess;
    int lanes = rad_lanes(crad_rows);
    k_ctr_rad<<<(g.nc + lanes - 1) / lanes, lanes, (size_t)crad_rows * lanes * sizeof(double), s>>>(
        g, crad_rows, crad);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_l2qbxl(const DevGeom &g, int nd, const int *items, int n, int Pmax, double *crad,
                         int crad_rows, int cap, const cd *loc, cd *coef, hipStream_t s)
{
    if (!n) return hipSuccess;
    if (Pmax + g.p + QBLK > crad_rows || cap < 1 || cap > L2Q_CAP_MAX) return hipErrorInvalidValue;
    size_t lds = l2qbxl_lds_bytes(Pmax, cap, crad_rows);
    if (lds > LDS_BUDGET) return hipErrorInvalidValue;
    k_l2qbxl<<<n, L2Q_THREADS, lds, s>>>(g, nd, items, crad, loc, coef, cap, crad_rows);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_qbx_eval(const DevGeom &g, int nd, const cd *coef, cd *u, hipStream_t s)
{
    if (!g.nt) return hipSuccess;
    k_qbx_eval<<<(g.nt + 255) / 256, 256, 0, s>>>(g, nd, coef, u);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_smooth(const DevGeom &g, int nd, const cd *qs, const cd *qd, cd *u, hipStream_t s)
{
    if (!g.n_smooth) return hipSuccess;
    k_smooth<<<g.n_smooth, 64, 0, s>>>(g, nd, qs, qd, u);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_coef_out(const DevGeom &g, int nd, const cd *coef, cd *out, hipStream_t s)
{
    long long n = (long long)nd * (2 * g.p + 1) * g.nc;
    if (!n) return hipSuccess;
    k_coef_out<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, nd, coef, out);
    QBX_LAUNCH_CHECK();
    return hipSuccess;
}


// ---------------------------------------------------------------------------
// Fused-launch planning.  Record fields per stage, besides g and nd (item
// sizes n, P, aux in brackets):
//   FILL           out0 = array, n64 = elements                      [n = elements]
//   CHARGES        in0 = sigma_S, in1 = sigma_D, out0 = qS, out1 = qD
//   SRC_RAD        i0 = rows, out0 = J table                         [n = P2M leaves]
//   CTR_RAD        i0 = rows, out0 = J table                         [n = L2QBXL items]
//   P2M            in0 = leaf list, in1 = qS, in2 = qD, in3 = J table, out0 = multipoles  [n, P]
//   M2M            i0 = level, in0 = its tiles, in1 = parent list, out0 = multipoles   [n = tiles, aux = row blocks]
//   M2L            in0 = tiles, in1 = multipoles, out0 = pair rows  [n = tiles, P, aux = waves per tile]
//   DOWN           i0 = level, in0 = pair rows, out0 = locals        [n = boxes of the level]
//   L2L            i0 = level, in0 = its tiles, in1 = child list, in2 = pair rows, out0 = locals  [n, aux = row blocks]
//   P2L_X          in0 = box list, in1 = qS, in2 = qD, out0 = locals [n, P]
//   P2QBXL         in0 = leaf list, in1 = qS, in2 = qD, out0 = coefficients  [n]
//   P2QBXL_DIRECT  in0 = qS, in1 = qD, out0 = coefficients
//   M2QBXL         in0 = pairs, in1 = pair row offsets, in2 = multipoles, out0 = pair rows  [n = pairs, P = largest W order]
//   WSUM           in0 = leaf list, in1 = per-leaf first pair, in2 = pair row offsets, in3 = pair rows,
//                  out0 = coefficients                               [n = leaves]
//   L2QBXL         i0 = item capacity, in0 = items, in1 = J table, in2 = locals, out0 = coefficients  [n, P, aux = J table rows]
//   EVAL           in0 = coefficients, out0 = u
//   SMOOTH         in0 = qS, in1 = qD, out0 = u
// Per geometry, pass sizes, centre groups and tile shapes are those of its
// own launch; block size and LDS are the largest any geometry needs.
// ---------------------------------------------------------------------------
namespace {

int p2q_bucket(int p)
{
    return p <= 8 ? 8 : p <= 12 ? 12 : p <= 14 ? 14 : p <= 16 ? 16 : p <= 24 ? 24 : p <= 32 ? 32 : 40;
}

// Appends one launch: records (first block filled in) and the block map.
// Returns its index, -1 without blocks, -2 when the grid is too large.
int fb_add(FBuf &fb, int kind, int variant, int threads, size_t lds, std::vector<FRec> recs,
           const std::vector<long long> &blocks)
{
    long long total = 0;
    for (size_t i = 0; i < recs.size(); ++i) {
        recs[i].first = (int)total;
        total += blocks[i];
        if (total > 0x7fffffffLL) return -2;
    }
    if (total == 0) return -1;
    auto align = [&](size_t a) { fb.bytes.resize((fb.bytes.size() + a - 1) / a * a, 0); };
    align(256);
    FLaunch L{kind, variant, threads, (int)total, lds, fb.bytes.size(), 0};
    size_t rb = recs.size() * sizeof(FRec);
    fb.bytes.resize(L.rec_off + rb);
    std::memcpy(fb.bytes.data() + L.rec_off, recs.data(), rb);
    align(256);
    L.map_off = fb.bytes.size();
    fb.bytes.resize(L.map_off + (size_t)total * sizeof(int));
    int *m = reinterpret_cast<int *>(fb.bytes.data() + L.map_off);
    for (size_t i = 0; i < recs.size(); ++i)
        for (long long b = 0; b < blocks[i]; ++b) *m++ = (int)i;
    fb.launches.push_back(L);
    return (int)fb.launches.size() - 1;
}

}  // namespace

hipError_t fused_plan(FBuf &fb, int kind, const std::vector<FItem> &items, std::vector<int> &ids)
{
    struct Row {
        int kind, variant, threads;
        FRec r;
        long long blocks;
        size_t lds;
    };
    std::vector<Row> rows;
    auto add = [&](int k, int v, FRec r, long long blocks, long long nx, size_t lds, int threads) {
        if (blocks <= 0) return;
        r.nx = (int)std::max<long long>(nx, 1);
        rows.push_back({k, v, threads, r, blocks, lds});
    };
    switch (kind) {
    case FK_FILL:
        for (const auto &it : items) {
            FRec r = it.r;
            r.n64 = it.n;
            long long b = std::min<long long>((it.n + 255) / 256, 1024);
            add(kind, 0, r, b, b, 0, 256);
        }
        break;
    case FK_CHARGES:
        for (const auto &it : items) {
            long long b = ((long long)it.r.nd * it.h->ns + 255) / 256;
            add(kind, 0, it.r, b, b, 0, 256);
        }
        break;
    case FK_SRC_BAS:
    case FK_CTR_RAD: {
        int rmax = 1;
        for (const auto &it : items) rmax = std::max(rmax, kind == FK_SRC_BAS ? it.h->srow : it.r.i0);
        int lanes = rad_lanes(rmax);
        size_t lds = (size_t)rmax * lanes * sizeof(double);
        for (const auto &it : items) {
            long long cnt = it.n > 0 ? (kind == FK_SRC_BAS ? it.h->ns : it.h->nc) : 0;
            long long b = (cnt + lanes - 1) / lanes;
            add(kind, 0, it.r, b, b, lds, lanes);
        }
        break;
    }
    case FK_X_BAS:
        for (const auto &it : items) {
            long long b = (it.r.n64 + 63) / 64;
            add(kind, 0, it.r, b, b, 0, 64);
        }
        break;
    case FK_P2M:
        for (const auto &it : items) {
            int nd = it.r.nd;
            if (nd < 1 || nd > 4) return hipErrorInvalidValue;
            add(kind, nd, it.r, it.n * half_order_runs(it.P), it.n, p2m_lds_bytes(nd), 64);
        }
        break;
    case FK_M2M:
        for (const auto &it : items) add(kind, 0, it.r, it.n * it.aux, it.n, 0, 256 * M2M_KS);
        break;
    case FK_M2L: {
        // per geometry: the leading tiles whose orders exceed the staged
        // kernel's LDS always go direct; the rest share one staged launch
        // (direct if no geometry asks for waves per tile)
        int nw = 0;
        size_t lmax = 0;
        for (const auto &it : items)
            if (!it.h->far32 && it.n > it.split) {
                nw = std::max(nw, std::min(it.aux, 16));
                lmax = std::max(lmax, m2l_staged_lds(it.P));
            }
        bool staged = nw > 0 && lmax <= LDS_BUDGET;
        for (const auto &it : items) {
            if (it.h->far32) {
                int nrmax = (2 * std::max(it.P, it.Psplit) + 1 + 15) / 16;
                FRec r = it.r;
                r.i0 = nrmax;
                add(FK_M2L32, 0, r, it.n * nrmax, it.n * nrmax, 0, 64);
                continue;
            }
            if (it.split > 0) {
                int nrd = (2 * it.Psplit + 1 + 15) / 16;
                FRec r = it.r;
                r.i0 = nrd;
                add(FK_M2L_DIRECT, 0, r, it.split * (long long)nrd, it.split * (long long)nrd, 0, 64);
            }
            long long rest = it.n - it.split;
            if (rest <= 0) continue;
            FRec r = it.r;
            r.in0 = static_cast<const QBX_G M2LTile *>(it.r.in0) + it.split;
            int nrmax = (2 * it.P + 1 + 15) / 16;
            r.i0 = nrmax;
            if (staged) add(FK_M2L, 0, r, rest, rest, lmax, 64 * nw);
            else add(FK_M2L_DIRECT, 0, r, rest * nrmax, rest * nrmax, 0, 64);
        }
        break;
    }
    case FK_DOWN:
        for (const auto &it : items) add(kind, 0, it.r, it.n, it.n, 0, 256);
        break;
    case FK_L2L:
        for (const auto &it : items)
            add(it.h->far32 ? FK_L2L32 : FK_L2L, 0, it.r, it.n * it.aux, it.n, 0, 64 * L2L_KS);
        break;
    case FK_P2L_X:
        for (const auto &it : items) {
            int nd = it.r.nd;
            if (nd < 1 || nd > 4) return hipErrorInvalidValue;
            if (it.h->xbas) {
                add(FK_P2L_XC, nd, it.r, it.n * order_runs(it.P), it.n, p2l_xc_lds_bytes(nd), 64);
                continue;
            }
            int ch = pick_ch(it.P);
            size_t lds = ptab_lds_bytes(nd, it.P, ch);
            if (lds > LDS_BUDGET) return hipErrorInvalidValue;
            FRec r = it.r;
            r.i0 = ch;
            add(kind, nd, r, it.n, it.n, lds, 64);
        }
        break;
    case FK_P2QBXL:
        for (const auto &it : items) {
            int pb = p2q_bucket(it.h->p);
            add(kind, pb, it.r, it.n, it.n, p2qbxl_lds_bytes(), P2Q_THREADS);
        }
        break;
    case FK_P2QBXL_DIRECT:
        for (const auto &it : items) {
            FRec r = it.r;
            r.i0 = direct_centres_per_wave(it.h->nc);
            long long b = (it.h->nc + r.i0 - 1) / r.i0;
            add(kind, p2q_bucket(it.h->p), r, b, b, 0, 64);
        }
        break;
    case FK_M2QBXL:
        for (const auto &it : items) {
            int cg = QCG_MAX;
            while (cg > 1 && m2qbxl_lds_bytes(it.r.nd, it.P, it.h->p, cg) > LDS_BUDGET) cg >>= 1;
            size_t lds = m2qbxl_lds_bytes(it.r.nd, it.P, it.h->p, cg);
            if (lds > LDS_BUDGET) return hipErrorInvalidValue;
            FRec r = it.r;
            r.i0 = cg;
            long long ny = (it.h->max_leaf_ctr + cg - 1) / cg;
            add(kind, 0, r, it.n * ny, it.n, lds, 256);
        }
        break;
    case FK_WSUM:
        for (const auto &it : items) add(kind, 0, it.r, it.n, it.n, 0, 256);
        break;
    case FK_L2QBXL:
        // r.i0: the items' centre capacity; aux: the J_n table's rows
        for (const auto &it : items) {
            if (it.P + it.h->p + QBLK > it.aux || it.r.i0 < 1 || it.r.i0 > L2Q_CAP_MAX) return hipErrorInvalidValue;
            size_t lds = l2qbxl_lds_bytes(it.P, it.r.i0, it.aux);
            if (lds > LDS_BUDGET) return hipErrorInvalidValue;
            FRec r = it.r;
            r.n64 = it.aux;
            add(kind, 0, r, it.n, it.n, lds, L2Q_THREADS);
        }
        break;
    case FK_EVAL:
        for (const auto &it : items) {
            long long b = ((long long)it.h->nt + 255) / 256;
            add(kind, 0, it.r, b, b, 0, 256);
        }
        break;
    case FK_SMOOTH:
        for (const auto &it : items) add(kind, 0, it.r, it.h->n_smooth, it.h->n_smooth, 0, 64);
        break;
    default:
        return hipErrorInvalidValue;
    }
    // one launch per (kernel, variant), in order of first appearance
    std::vector<char> done(rows.size(), 0);
    for (size_t i = 0; i < rows.size(); ++i) {
        if (done[i]) continue;
        std::vector<FRec> recs;
        std::vector<long long> blocks;
        size_t lds = 0;
        for (size_t j = i; j < rows.size(); ++j)
            if (!done[j] && rows[j].kind == rows[i].kind && rows[j].variant == rows[i].variant) {
                done[j] = 1;
                recs.push_back(rows[j].r);
                blocks.push_back(rows[j].blocks);
                lds = std::max(lds, rows[j].lds);
            }
        int id = fb_add(fb, rows[i].kind, rows[i].variant, rows[i].threads, lds, recs, blocks);
        if (id == -2) return hipErrorInvalidValue;
        if (id >= 0) ids.push_back(id);
    }
    return hipSuccess;
}

hipError_t fused_launch(const FLaunch &L, const unsigned char *dev, hipStream_t s)
{
    const FRec *recs = reinterpret_cast<const FRec *>(dev + L.rec_off);
    const int *map = reinterpret_cast<const int *>(dev + L.map_off);
    dim3 grid((unsigned)L.nblocks), block((unsigned)L.threads);
    size_t lds = L.lds;
#define FL(...) __VA_ARGS__<<<grid, block, lds, s>>>(recs, map)
    switch (L.kind) {
    case FK_FILL: FL(kf_fill); break;
    case FK_CHARGES: FL(kf_charges); break;
    case FK_SRC_BAS: FL(kf_src_bas); break;
    case FK_X_BAS: FL(kf_x_bas); break;
    case FK_CTR_RAD: FL(kf_ctr_rad); break;
    case FK_P2M:
        switch (L.variant) {
        case 1: FL(kf_p2m<1>); break;
        case 2: FL(kf_p2m<2>); break;
        case 3: FL(kf_p2m<3>); break;
        default: FL(kf_p2m<4>); break;
        }
        break;
    case FK_M2M: FL(kf_m2m); break;
    case FK_M2L: FL(kf_m2l); break;
    case FK_M2L_DIRECT: FL(kf_m2l_direct); break;
    case FK_M2L32: FL(kf_m2l32); break;
    case FK_DOWN: FL(kf_down); break;
    case FK_L2L: FL(kf_l2l); break;
    case FK_L2L32: FL(kf_l2l32); break;
    case FK_P2L_XC:
        switch (L.variant) {
        case 1: FL(kf_p2l_xc<1>); break;
        case 2: FL(kf_p2l_xc<2>); break;
        case 3: FL(kf_p2l_xc<3>); break;
        default: FL(kf_p2l_xc<4>); break;
        }
        break;
    case FK_P2L_X:
        switch (L.variant) {
        case 1: FL(kf_p2l_x<1>); break;
        case 2: FL(kf_p2l_x<2>); break;
        case 3: FL(kf_p2l_x<3>); break;
        default: FL(kf_p2l_x<4>); break;
        }
        break;
    case FK_P2QBXL:
        switch (L.variant) {
        case 8: FL(kf_p2qbxl<8>); break;
        case 12: FL(kf_p2qbxl<12>); break;
        case 14: FL(kf_p2qbxl<14>); break;
        case 16: FL(kf_p2qbxl<16>); break;
        case 24: FL(kf_p2qbxl<24>); break;
        case 32: FL(kf_p2qbxl<32>); break;
        default: FL(kf_p2qbxl<40>); break;
        }
        break;
    case FK_P2QBXL_DIRECT:
        switch (L.variant) {
        case 8: FL(kf_p2qbxl_direct<8>); break;
        case 12: FL(kf_p2qbxl_direct<12>); break;
        case 14: FL(kf_p2qbxl_direct<14>); break;
        case 16: FL(kf_p2qbxl_direct<16>); break;
        case 24: FL(kf_p2qbxl_direct<24>); break;
        case 32: FL(kf_p2qbxl_direct<32>); break;
        default: FL(kf_p2qbxl_direct<40>); break;
        }
        break;
    case FK_M2QBXL: FL(kf_m2qbxl); break;
    case FK_WSUM: FL(kf_wsum); break;
    case FK_L2QBXL: FL(kf_l2qbxl); break;
    case FK_EVAL: FL(kf_eval); break;
    case FK_SMOOTH: FL(kf_smooth); break;
    default: return hipErrorInvalidValue;
    }
#undef FL
    return hipGetLastError();
}

}  // namespace qbx
