// Device part of the C ABI: contexts, resident geometries and evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "abi_common.hpp"
#include "areaquery.hpp"
#include "kernels.hpp"
#include "krylov.hpp"

using namespace qbx;

// The evaluation buffers of qbx_eval_noalloc: one static array per device,
// held until the process ends.  In host code its name stands for the
// array, not its device address; that comes from hipGetSymbolAddress,
// once per device (noalloc_base), and only that address is used.
static __device__ __align__(256) unsigned char noalloc_scratch[QBX_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char *g_noalloc_base[kMaxDevices] = {};

// Device address of the static evaluation buffers on `device` (current),
// looked up on the first call per device.  Null on failure.
unsigned char *noalloc_base(int device, hipError_t *err)
{
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_base[device]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
        if (*err != hipSuccess) return nullptr;
        g_noalloc_base[device] = static_cast<unsigned char *>(ptr);
    }
    return g_noalloc_base[device];
}

}  // namespace

// A side stream and the events that fork it from, and join it back to, the
// stream an evaluation is enqueued on.
struct QbxLane {
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_x = nullptr, ev_q = nullptr, ev_m = nullptr;
};

struct qbx_ctx_s {
    // the caller's handle and every geometry made on the context hold a
    // reference; the context is torn down when the last one goes, so a
    // geometry destroyed after qbx_ctx_destroy still finds its streams
    std::atomic<int> refs{1};
    int device = 0;
    hipStream_t stream = nullptr;
    // the side stream of plain evaluations: the near field and the X-list
    // P2L depend on the charges only and overlap the latency-bound
    // upward/downward passes; events fork it from and join it back to the
    // caller's stream
    QbxLane lane;
    // captured evaluations run on a stream of the library's own (the caller's
    // may be the null stream, which cannot be captured), joined to the
    // caller's stream by events
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // fused batch launches: records and block maps, staged in pinned host
    // memory and copied to the device once per qbx_eval_batch call
    unsigned char *fz_host = nullptr, *fz_dev = nullptr;
    size_t fz_cap = 0;
    hipEvent_t fz_copied = nullptr;   // the last copy out of fz_host
    hipEvent_t fz_done = nullptr;     // the last launch reading fz_dev was enqueued before this
    bool fz_used = false;
    // workspace of qbx_krylov_dot (partial sums), grown on demand
    cd *kw = nullptr;
    size_t kw_cap = 0;
    // the thread inside a call on this context (nested calls of that thread
    // count in depth), and the message of the last failed call
    std::atomic<std::thread::id> owner{};
    int depth = 0;
    std::mutex err_mu;
    std::string err;
};

namespace {

void ctx_release(qbx_ctx_s *ctx);

// One call on a context.  It holds a reference, so a context dropped inside
// it (its last geometry destroyed) lives until the call returns, and a
// message the call sets becomes the context's last error.  An exclusive call
// (evaluations and what else uses the context's streams, events and
// buffers) admits one thread at a time: a second thread that enters while
// another is inside one gets QBX_E_BUSY.  Geometry set-up, area queries and
// the plain kernels of GMRES touch none of that state and run alongside.
class CtxCall {
public:
    CtxCall(qbx_ctx_s *c, bool exclusive) : c_(c), seq_(error_seq())
    {
        if (exclusive) {
            std::thread::id me = std::this_thread::get_id(), none{};
            if (c_->owner.load() == me) {
                ++c_->depth;
                excl_ = true;
            } else if (c_->owner.compare_exchange_strong(none, me)) {
                c_->depth = 1;
                excl_ = true;
            } else {
                return;
            }
        }
        ok_ = true;
        ++c_->refs;
    }
    ~CtxCall()
    {
        if (!ok_) return;
        if (error_seq() != seq_) {
            std::lock_guard<std::mutex> lk(c_->err_mu);
            c_->err = error_msg();
        }
        if (excl_ && --c_->depth == 0) c_->owner.store(std::thread::id{});
        ctx_release(c_);
    }
    bool ok() const { return ok_; }
    CtxCall(const CtxCall &) = delete;
    CtxCall &operator=(const CtxCall &) = delete;

private:
    qbx_ctx_s *c_;
    unsigned long long seq_;
    bool ok_ = false, excl_ = false;
};

#define QBX_CTX_CALL(c) CtxCall ctx_call_(c, false)
#define QBX_CTX_EXCLUSIVE(c)                                                               \
    CtxCall ctx_call_(c, true);                                                            \
    if (!ctx_call_.ok()) return fail(QBX_E_BUSY, "the context is inside a call from another thread")

// Whether a caller's array is memory the context's device reads in place
// (its own device memory, or managed memory).  Host memory, pinned or not,
// is not: qbx_eval stages it, the other entry points refuse it.
bool device_readable(const void *p, int device)
{
    if (!p) return true;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();            // unregistered host memory
        return false;
    }
    if (a.type == hipMemoryTypeManaged || a.type == hipMemoryTypeUnified) return true;
    return a.type == hipMemoryTypeDevice && a.device == device;
}

bool lane_create(QbxLane &L)
{
    if (hipStreamCreateWithFlags(&L.side, hipStreamNonBlocking) != hipSuccess) { L.side = nullptr; return false; }
    for (hipEvent_t *e : {&L.ev_fork, &L.ev_x, &L.ev_q, &L.ev_m})
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) { *e = nullptr; return false; }
    return true;
}

void lane_destroy(QbxLane &L)
{
    if (L.side) (void)hipStreamSynchronize(L.side);
    for (hipEvent_t e : {L.ev_fork, L.ev_x, L.ev_q, L.ev_m})
        if (e) (void)hipEventDestroy(e);
    if (L.side) (void)hipStreamDestroy(L.side);
    L = QbxLane{};
}

constexpr int kDensChunk = 4;   // densities per pass through the pipeline
// The X-list P2L basis is kept when it takes at most this much device memory
// (else its rows are rebuilt in every evaluation).
constexpr size_t kXBasisCap = size_t(1) << 30;
constexpr int kM2LTileCols = 16; // columns per M2L tile (one MFMA column block)

// Device memory of one geometry.  The resident part is built in two passes
// of the same code: a sizing pass (`sizing`: nothing is allocated or copied,
// offsets are counted) and a packed pass into one allocation of that size,
// staged in host memory and copied once (commit).  Without a reserved block
// every request is its own allocation (the evaluation scratch).
struct DeviceArena {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    hipError_t err = hipSuccess;
    bool sizing = false;
    unsigned char *block = nullptr;          // packed pass: the one allocation
    size_t cap = 0, off = 0;
    std::vector<unsigned char> stage;        // its host image
    static size_t aligned(size_t n) { return (n + 255) & ~(size_t)255; }
    void *take(size_t n, const void *src, size_t nsrc)
    {
        if (err != hipSuccess) return nullptr;
        n = std::max<size_t>(n, 16);
        if (sizing) {
            size_t o = off;
            off += aligned(n);
            bytes = off;
            return reinterpret_cast<void *>((uintptr_t)256 + o);   // never dereferenced
        }
        if (block) {
            if (off + n > cap) {
                err = hipErrorInvalidValue;            // sizing and packed passes disagree
                return nullptr;
            }
            void *p = block + off;
            if (nsrc) std::memcpy(stage.data() + off, src, nsrc);
            off += aligned(n);
            return p;
        }
        void *p = nullptr;
        err = hipMalloc(&p, n);
        if (err != hipSuccess) return nullptr;
        ptrs.push_back(p);
        bytes += n;
        if (nsrc) err = hipMemcpy(p, src, nsrc, hipMemcpyHostToDevice);
        return p;
    }
    template <class T>
    T *upload(const std::vector<T> &v)
    {
        return static_cast<T *>(take(std::max<size_t>(v.size(), 1) * sizeof(T), v.data(), v.size() * sizeof(T)));
    }
    void *alloc(size_t n) { return take(n, nullptr, 0); }
    // packed pass: one allocation of the sized bytes (the sizing pass's offset)
    hipError_t reserve(size_t n)
    {
        cap = std::max<size_t>(n, 256);
        err = hipMalloc((void **)&block, cap);
        if (err != hipSuccess) { block = nullptr; return err; }
        ptrs.push_back(block);
        stage.assign(cap, 0);
        off = 0;
        bytes += cap;
        return hipSuccess;
    }
    hipError_t commit()
    {
        if (err == hipSuccess && block && off) err = hipMemcpy(block, stage.data(), off, hipMemcpyHostToDevice);
        stage.clear();
        stage.shrink_to_fit();
        block = nullptr;   // later requests are allocations of their own
        return err;
    }
    void release()
    {
        if (!sizing)
            for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
        off = 0;
        block = nullptr;
    }
};

struct WorkList {
    int *d = nullptr;
    int n = 0;
    int Pmax = 0;
};

// Largest (centre, source) pair count a P2QBXL lane is given before its leaf
// is split over several workgroups (about twice the typical leaf's).
constexpr long long kP2qLanePairs = 8;

}  // namespace

struct qbx_geom_s {
    qbx_ctx ctx = nullptr;
    Plan pl;
    DevGeom g{};
    const DevGeom *d_self = nullptr;   // device copy of g (fused launches)
    DeviceArena arena;
    WorkList p2m, xl, qbx, wl, l2q;
    long long total_coef = 0;     // sum over boxes of (2 P_l + 1)
    // M2L GEMM groups: (level*40 + offset, start in vpair_sorted, pairs)
    struct Group {
        int key, start, count;
    };
    std::vector<Group> m2l_groups;
    int m2l_Pmax = 0;
    int m2l_nw = 1;                                // waves per M2L tile (0 = direct kernel)
    int m2l_nw_default = 1;                        // the common row-block count
    long long total_vy = 0;       // sum over V-list positions of (2 P_l + 1)
    std::vector<int32_t> near_start, near_idx, wf_start, wf_idx;   // host copies
    // M2QBXL work: (leaf, far W) pairs, their output rows and per-leaf ranges
    int n_wpairs = 0;
    long long total_wy = 0;
    int2 *d_wpairs = nullptr;
    long long *d_wpair_off = nullptr;
    int *d_wleaf_start = nullptr;
    cd *wy = nullptr;
    M2LTile *m2l_tiles[kDensChunk + 1] = {};
    int m2l_ntiles[kDensChunk + 1] = {};
    // M2L tiles come in two runs: those of orders beyond the staged kernel's
    // LDS (direct kernel, orders up to m2l_Pdirect), then the rest (orders up
    // to m2l_Pstaged)
    int m2l_split[kDensChunk + 1] = {};
    int m2l_Pdirect = 0, m2l_Pstaged = 0;
    // M2M parents per level, L2L children per (level, quadrant), and their tiles
    std::vector<int> par_list, par_lvl, chl_list, chl_lvl;
    std::vector<long long> box_off_h, vy_off_h;   // host copies of box_off, vy_off
    int *d_par_list = nullptr, *d_chl_list = nullptr;
    TTile *m2m_tiles[kDensChunk + 1] = {}, *l2l_tiles[kDensChunk + 1] = {};
    std::vector<int> m2m_tstart[kDensChunk + 1], l2l_tstart[kDensChunk + 1];   // per level
    cd *vy = nullptr;
    // per-eval scratch, sized for kDensChunk densities
    DeviceArena scratch;
    cd *qs = nullptr, *qd = nullptr, *mp = nullptr, *loc = nullptr, *coef = nullptr;
    // radial sequences: J_n per P2M source and per L2QBXL centre (n-major)
    // geometry-only sequences, resident: the P2M and X-list P2L bases (in
    // the view g) and J_n(omega |m_b - c|) per L2QBXL centre (n-major),
    // built on the first evaluation
    int srad_rows = 0, crad_rows = 0;
    int l2q_cap = 1;              // centres per L2QBXL item (at most)
    cd *sbas = nullptr, *xbas = nullptr;
    double *crad = nullptr;
    int n_xpos = 0;                 // flattened X-list positions
    // the radial sequences depend on the geometry only: computed on the
    // first evaluation (once the scratch exists) and kept, like the tables
    bool rad_ready = false;
    // FMM mode: the targets no expansion disk holds are the centres of an
    // order-0 geometry on the same sources (each target bound to its own
    // centre), which writes their potentials into this geometry's output:
    // its P2QBXL, M2QBXL and L2QBXL are then the point FMM's near-field sum,
    // M2P and L2P (Sec. 7) at those targets
    qbx_geom_s *sub = nullptr;
    std::vector<int32_t> out_map;   // of a sub-geometry: the owner's target per target
    long long out_stride = 0;       // of a sub-geometry: the owner's target count
    // captured evaluations (qbx_geom_graph), keyed by their arguments
    struct GraphRec {
        int n_dens;
        const void *ss, *sd;
        void *u, *coef;
        hipGraphExec_t exec;
        uint64_t used;
    };
    bool graph_on = false;
    std::vector<GraphRec> graphs;
    uint64_t graph_clock = 0;
    // per-stage HIP-event timing (qbx_geom_profile)
    struct StageRec {
        int stage;
        hipEvent_t a, b;
        int launches;
    };
    bool profile = false;
    std::vector<StageRec> pending;
    std::vector<hipEvent_t> spare;
    double acc_ms[QBX_N_STAGES] = {};
    int64_t acc_n[QBX_N_STAGES] = {};
    ~qbx_geom_s()
    {
        for (auto &r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : spare) (void)hipEventDestroy(e);
        for (auto &r : graphs) (void)hipGraphExecDestroy(r.exec);
    }
};

namespace {

// Whether a W-list box's sources enter the centres' coefficients directly
// (P2QBXL) rather than through M2QBXL.  Automatic rule: per centre, direct
// costs about 3(2p+1) + 48 complex multiply-adds per source (coefficient
// updates plus Bessel values), M2QBXL (2p+1)(2P_w+1).
bool w_is_direct(const Plan &pl, int w)
{
    int ns = pl.src_end[w] - pl.src_begin[w];
    int wd = pl.opt.w_direct;
    if (wd == 0) return false;
    if (wd > 0) return ns <= wd;
    long long q = 2 * pl.p + 1, Pw = pl.P[pl.lev[w]];
    return (long long)ns * (3 * q + 48) <= q * (2 * Pw + 1);
}

template <class F>
WorkList make_list(DeviceArena &ar, const Plan &pl, F pred)
{
    std::vector<int> v;
    WorkList w;
    for (int b = 0; b < pl.n_boxes(); ++b)
        if (pred(b)) {
            v.push_back(b);
            w.Pmax = std::max(w.Pmax, pl.P[pl.lev[b]]);
        }
    w.n = (int)v.size();
    w.d = ar.upload(v);
    return w;
}

qbx_status upload(qbx_geom_s *G)
{
    const Plan &pl = G->pl;
    DeviceArena &ar = G->arena;
    DevGeom &g = G->g;
    int nb = pl.n_boxes();
    long long xbas_total = 0;     // entries of the cached X-list basis
    g.ns = (int)pl.ns; g.nc = (int)pl.nc; g.nt = (int)pl.nt; g.nb = nb; g.nlev = pl.nlev;
    g.p = pl.p; g.omega = pl.omega;
    g.max_leaf_ctr = 1;
    for (int b = 0; b < nb; ++b)
        if (pl.leaf[b]) g.max_leaf_ctr = std::max(g.max_leaf_ctr, pl.ctr_end[b] - pl.ctr_begin[b]);

    std::vector<double> a(pl.ns), bq(pl.ns), c(pl.ns), d(pl.ns), e(pl.ns);
    std::vector<int> perm(pl.ns);
    for (int64_t j = 0; j < pl.ns; ++j) {
        int64_t u = pl.src_order[j];
        a[j] = pl.sx[u]; bq[j] = pl.sy[u]; c[j] = pl.w[u]; d[j] = pl.nx[u]; e[j] = pl.ny[u];
        perm[j] = (int)u;
    }
    g.sx = ar.upload(a); g.sy = ar.upload(bq); g.sw = ar.upload(c); g.snx = ar.upload(d); g.sny = ar.upload(e);
    g.src_perm = ar.upload(perm);

    std::vector<double> ccx(pl.nc), ccy(pl.nc);
    std::vector<int> cperm(pl.nc), rank(pl.nc);
    for (int64_t i = 0; i < pl.nc; ++i) {
        int64_t u = pl.ctr_order[i];
        ccx[i] = pl.cx[u]; ccy[i] = pl.cy[u]; cperm[i] = (int)u; rank[u] = (int)i;
    }
    g.cx = ar.upload(ccx); g.cy = ar.upload(ccy); g.ctr_perm = ar.upload(cperm);

    std::vector<int> tcs(pl.nt), smooth;
    for (int64_t m = 0; m < pl.nt; ++m) {
        int v = pl.tgt_ctr[m];
        tcs[m] = v >= 0 ? rank[v] : -1;
        if (v < 0) smooth.push_back((int)m);
    }
    g.tx = ar.upload(pl.tx); g.ty = ar.upload(pl.ty); g.tgt_cs = ar.upload(tcs);
    g.smooth_list = ar.upload(smooth);
    // in FMM mode the order-0 sub-geometry serves these targets
    g.n_smooth = pl.opt.direct ? (int)smooth.size() : 0;
    g.tgt_out = G->out_map.empty() ? nullptr : ar.upload(G->out_map);
    g.u_stride = G->out_stride > 0 ? G->out_stride : (long long)pl.nt;

    std::vector<double> bcx(nb), bcy(nb);
    for (int b = 0; b < nb; ++b) pl.box_center(b, &bcx[b], &bcy[b]);
    g.bcx = ar.upload(bcx); g.bcy = ar.upload(bcy);
    g.blev = ar.upload(pl.lev); g.leaf = ar.upload(pl.leaf); g.parent = ar.upload(pl.parent);
    g.child_begin = ar.upload(pl.child_begin); g.child_count = ar.upload(pl.child_count);
    g.src_begin = ar.upload(pl.src_begin); g.src_end = ar.upload(pl.src_end);
    g.ctr_begin = ar.upload(pl.ctr_begin); g.ctr_end = ar.upload(pl.ctr_end);
    g.level_start = ar.upload(pl.level_start);
    g.U_start = ar.upload(pl.U_start); g.U_idx = ar.upload(pl.U_idx);
    g.V_start = ar.upload(pl.V_start); g.V_idx = ar.upload(pl.V_idx); g.V_off = ar.upload(pl.V_off);
    g.W_start = ar.upload(pl.W_start); g.W_idx = ar.upload(pl.W_idx);
    g.X_start = ar.upload(pl.X_start); g.X_idx = ar.upload(pl.X_idx);
    g.Plev = ar.upload(pl.P);

    std::vector<int> woff(pl.nlev + 1, 0);
    std::vector<double> W, iW, lW;
    for (int l = 0; l < pl.nlev; ++l) {
        woff[l] = (int)W.size();
        auto s = level_scales(pl.omega, pl.box_radius(l), pl.P[l]);
        for (double v : s) { W.push_back(v); iW.push_back(1.0 / v); lW.push_back(std::log(v)); }
    }
    woff[pl.nlev] = (int)W.size();
    g.Woff = ar.upload(woff); g.Wtab = ar.upload(W); g.invW = ar.upload(iW); g.logW = ar.upload(lW);

    std::vector<long long> boff(nb);
    long long tot = 0;
    for (int b = 0; b < nb; ++b) { boff[b] = tot; tot += 2 * pl.P[pl.lev[b]] + 1; }
    G->total_coef = tot;
    g.box_off = ar.upload(boff);
    G->box_off_h = boff;

    // translation tables, [in][out] (column of the scaled matrix per input index)
    std::vector<cd> m2m, l2l, m2l;
    std::vector<long long> m2m_off(4 * (size_t)std::max(pl.nlev, 1), -1),
        l2l_off(4 * (size_t)std::max(pl.nlev, 1), -1), m2l_off(40 * (size_t)std::max(pl.nlev, 1), -1);
    // V-list positions: target box, grouping by (level, offset), output rows
    int nv = (int)pl.V_idx.size();
    std::vector<int> vtgt(nv), vpos(nv);
    std::vector<long long> vy_off(std::max(nv, 1));
    long long vy_tot = 0;
    for (int b = 0; b < nb; ++b)
        for (int v = pl.V_start[b]; v < pl.V_start[b + 1]; ++v) {
            vtgt[v] = b;
            vy_off[v] = vy_tot;
            vy_tot += 2 * pl.P[pl.lev[b]] + 1;
        }
    G->total_vy = vy_tot;
    std::iota(vpos.begin(), vpos.end(), 0);
    // The V offsets fall into 10 orbits of 4 under rotations by 90 degrees.
    // Rotating the translation vector by r quarter turns multiplies O_n by
    // i^{rn}, so the matrix of offset R^r c is diag(i^{rj}) M(c) diag(i^{rk}):
    // pairs are grouped by (level, representative c) and carry r.  The
    // representative of an orbit is its offset with dx > 0, dy >= 0.
    int vrep[40], vrot[40];
    for (int id = 0; id < 40; ++id) {
        int x, y;
        v_offset_from_id(id, &x, &y);
        vrep[id] = -1;
        vrot[id] = 0;
        for (int r = 0; r < 4; ++r) {
            if (x > 0 && y >= 0) { vrep[id] = v_offset_id(x, y); vrot[id] = r; break; }
            int t = x; x = y; y = -t;   // a quarter turn back (clockwise)
        }
    }
    auto vkey = [&](int v) { return pl.lev[vtgt[v]] * 40 + vrep[pl.V_off[v]]; };
    std::stable_sort(vpos.begin(), vpos.end(), [&](int a, int b) { return vkey(a) < vkey(b); });
    G->m2l_groups.clear();
    G->m2l_Pmax = 0;
    G->m2l_nw = 1;
    G->m2l_Pdirect = G->m2l_Pstaged = 0;
    const int pstaged_max = m2l_staged_pmax();
    for (int i = 0; i < nv;) {
        int j = i;
        while (j < nv && vkey(vpos[j]) == vkey(vpos[i])) ++j;
        G->m2l_groups.push_back({vkey(vpos[i]), i, j - i});
        int P = pl.P[vkey(vpos[i]) / 40];
        G->m2l_Pmax = std::max(G->m2l_Pmax, P);
        if (P > pstaged_max) G->m2l_Pdirect = std::max(G->m2l_Pdirect, P);
        else G->m2l_Pstaged = std::max(G->m2l_Pstaged, P);
        i = j;
    }
    {
        // waves per M2L tile: the row-block count of most V pairs, so that
        // those tiles have one row block per wave
        std::vector<long long> cnt(64, 0);
        for (const auto &grp : G->m2l_groups) {
            int nr = (2 * pl.P[grp.key / 40] + 1 + 15) / 16;
            cnt[std::min(nr, 63)] += grp.count;
        }
        G->m2l_nw = (int)(std::max_element(cnt.begin(), cnt.end()) - cnt.begin());
        G->m2l_nw = std::max(1, std::min(G->m2l_nw, 16));
        G->m2l_nw_default = G->m2l_nw;
    }
    g.vpair_sorted = ar.upload(vpos);
    g.vy_off = ar.upload(vy_off);
    G->vy_off_h = vy_off;
    {
        // per sorted position: source box multipole offset, output row
        // offset, quarter turns from the group's offset
        std::vector<long long> src(std::max(nv, 1)), dst(std::max(nv, 1));
        std::vector<int> rot(std::max(nv, 1), 0);
        for (int i = 0; i < nv; ++i) {
            src[i] = boff[pl.V_idx[vpos[i]]];
            dst[i] = vy_off[vpos[i]];
            rot[i] = vrot[pl.V_off[vpos[i]]];
        }
        g.m2l_src = ar.upload(src);
        g.m2l_dst = ar.upload(dst);
        g.m2l_rot = ar.upload(rot);
    }
    // Row-major [out][in] matrix -> v_mfma_f64_16x16x4f64 A-operand order:
    // 16x4 blocks of 64 values, block (rb, kb) at (rb * NK + kb) * 64, lane l
    // holding element (rb*16 + l%16, kb*4 + l/16), zero outside the matrix.
    auto append_tiled = [](std::vector<cd> &dst, const std::vector<std::complex<double>> &M, int nout,
                           int nin) {
        int NR = (nout + 15) / 16, NK = (nin + 3) / 4;
        long long off = (long long)dst.size();
        dst.resize(dst.size() + (size_t)NR * NK * 64, mk(0.0, 0.0));
        for (int rb = 0; rb < NR; ++rb)
            for (int kb = 0; kb < NK; ++kb)
                for (int lane = 0; lane < 64; ++lane) {
                    int row = rb * 16 + lane % 16, k = kb * 4 + lane / 16;
                    if (row < nout && k < nin) {
                        const auto &v = M[(size_t)row * nin + k];
                        dst[off + ((size_t)rb * NK + kb) * 64 + lane] = mk(v.real(), v.imag());
                    }
                }
        return off;
    };
    if (!pl.opt.direct) {
        for (int l = 2; l + 1 < pl.nlev; ++l)
            for (int q = 0; q < 4; ++q) {
                int np = 2 * pl.P[l] + 1, nc = 2 * pl.P[l + 1] + 1;
                m2m_off[l * 4 + q] = append_tiled(m2m, m2m_matrix(pl, l, q), np, nc);
                l2l_off[l * 4 + q] = append_tiled(l2l, l2l_matrix(pl, l, q), nc, np);
            }
        for (const auto &grp : G->m2l_groups) {
            int l = grp.key / 40, o = grp.key % 40;
            int dx, dy;
            v_offset_from_id(o, &dx, &dy);
            int n = 2 * pl.P[l] + 1;
            m2l_off[grp.key] = append_tiled(m2l, m2l_matrix(pl, l, dx, dy), n, n);
        }
    }
    g.m2m_mf = ar.upload(m2m); g.l2l_mf = ar.upload(l2l); g.m2l_mf = ar.upload(m2l);
    g.far32 = pl.opt.far_fp32 ? 1 : 0;
    g.m2l_mf32 = g.l2l_mf32 = nullptr;
    if (g.far32) {
        // the scaled entries are bounded by one, so complex float holds them
        auto to32 = [](const std::vector<cd> &v) {
            std::vector<cf> o(v.size());
            for (size_t i = 0; i < v.size(); ++i) o[i] = cf{(float)v[i].x, (float)v[i].y};
            return o;
        };
        g.m2l_mf32 = ar.upload(to32(m2l));
        g.l2l_mf32 = ar.upload(to32(l2l));
    }
    g.m2m_mf_off = ar.upload(m2m_off); g.l2l_mf_off = ar.upload(l2l_off); g.m2l_mf_off = ar.upload(m2l_off);

    // children by quadrant; M2M parent lists and L2L child lists per level
    {
        std::vector<int> child4((size_t)nb * 4, -1);
        for (int b = 0; b < nb; ++b)
            for (int c = pl.child_begin[b]; c >= 0 && c < pl.child_begin[b] + pl.child_count[b]; ++c)
                child4[(size_t)b * 4 + ((pl.bix[c] & 1) | ((pl.biy[c] & 1) << 1))] = c;
        g.child4 = ar.upload(child4);
        // Parents of each level ordered by which of their four children
        // exist, so that most M2M tiles hold parents with the same children:
        // the waves of a child quadrant missing from a whole tile then skip
        // their product instead of multiplying zeros.  Each parent's sum is
        // the same whichever tile it lands in.
        auto cmask = [&](int b) {
            int m = 0;
            for (int c = pl.child_begin[b]; c < pl.child_begin[b] + pl.child_count[b]; ++c)
                m |= 1 << ((pl.bix[c] & 1) | ((pl.biy[c] & 1) << 1));
            return m;
        };
        G->par_list.clear();
        G->par_lvl.assign(pl.nlev + 1, 0);
        for (int l = 0; l < pl.nlev; ++l) {
            size_t s0 = G->par_list.size();
            G->par_lvl[l] = (int)s0;
            for (int b = pl.level_start[l]; b < pl.level_start[l + 1]; ++b)
                if (!pl.leaf[b] && l >= 2) G->par_list.push_back(b);
            std::stable_sort(G->par_list.begin() + s0, G->par_list.end(),
                             [&](int a, int c) { return cmask(a) < cmask(c); });
        }
        G->par_lvl[pl.nlev] = (int)G->par_list.size();
        G->chl_list.clear();
        G->chl_lvl.assign((size_t)(pl.nlev + 1) * 4, 0);
        for (int L = 0; L < pl.nlev; ++L)
            for (int q = 0; q < 4; ++q) {
                G->chl_lvl[L * 4 + q] = (int)G->chl_list.size();
                for (int c = pl.level_start[L]; c < pl.level_start[L + 1]; ++c)
                    if (L >= 3 && ((pl.bix[c] & 1) | ((pl.biy[c] & 1) << 1)) == q) G->chl_list.push_back(c);
            }
        G->chl_lvl[pl.nlev * 4] = (int)G->chl_list.size();
        G->d_par_list = ar.upload(G->par_list);
        G->d_chl_list = ar.upload(G->chl_list);
        // per list position, the offsets the translation kernels need, so that
        // they start with one load instead of a chain of dependent ones
        std::vector<long long> mc(std::max<size_t>(G->par_list.size() * 4, 1)),
            mpo(std::max<size_t>(G->par_list.size(), 1));
        for (size_t i = 0; i < G->par_list.size(); ++i) {
            int b = G->par_list[i];
            mpo[i] = G->box_off_h[b];
            for (int q = 0; q < 4; ++q) mc[i * 4 + q] = -1;
            for (int c = pl.child_begin[b]; c < pl.child_begin[b] + pl.child_count[b]; ++c)
                mc[i * 4 + ((pl.bix[c] & 1) | ((pl.biy[c] & 1) << 1))] = G->box_off_h[c];
        }
        size_t nch = std::max<size_t>(G->chl_list.size(), 1);
        std::vector<long long> lpo(nch), lco(nch), lvy(nch);
        std::vector<int> lnv(nch);
        for (size_t i = 0; i < G->chl_list.size(); ++i) {
            int c = G->chl_list[i];
            lpo[i] = G->box_off_h[pl.parent[c]];
            lco[i] = G->box_off_h[c];
            int v0 = pl.V_start[c], v1 = pl.V_start[c + 1];
            lvy[i] = v1 > v0 ? G->vy_off_h[v0] : 0;
            lnv[i] = v1 - v0;
        }
        g.m2m_coff = ar.upload(mc);
        g.m2m_poff = ar.upload(mpo);
        g.l2l_poff = ar.upload(lpo);
        g.l2l_coff = ar.upload(lco);
        g.l2l_vy0 = ar.upload(lvy);
        g.l2l_nv = ar.upload(lnv);
    }

    auto has_ctr = [&](int b) { return pl.ctr_end[b] > pl.ctr_begin[b]; };
    G->p2m = make_list(ar, pl, [&](int b) { return pl.leaf[b] && pl.lev[b] >= 2; });
    {
        // the same leaves, the most sources first (long workgroups start early)
        std::vector<int> v;
        for (int b = 0; b < nb; ++b)
            if (pl.leaf[b] && pl.lev[b] >= 2) v.push_back(b);
        std::stable_sort(v.begin(), v.end(), [&](int a, int c) {
            return pl.src_end[a] - pl.src_begin[a] > pl.src_end[c] - pl.src_begin[c];
        });
        G->p2m.d = ar.upload(v);
    }
    // the X-list P2L list: boxes with an X list, the most X-list sources
    // first, so that long workgroups start early and short ones fill the
    // tail (each box's result is independent of the order)
    std::vector<int> xorder;
    {
        std::vector<long long> xw(nb, 0);
        for (int b = 0; b < nb; ++b) {
            if (pl.X_start[b + 1] <= pl.X_start[b]) continue;
            for (int i = pl.X_start[b]; i < pl.X_start[b + 1]; ++i)
                xw[b] += pl.src_end[pl.X_idx[i]] - pl.src_begin[pl.X_idx[i]];
            xorder.push_back(b);
        }
        std::stable_sort(xorder.begin(), xorder.end(), [&](int a, int c) { return xw[a] > xw[c]; });
        G->xl.n = (int)xorder.size();
        G->xl.Pmax = 0;
        for (int b : xorder) G->xl.Pmax = std::max(G->xl.Pmax, pl.P[pl.lev[b]]);
        G->xl.d = ar.upload(xorder);
    }
    G->l2q = make_list(ar, pl, [&](int b) { return pl.leaf[b] && has_ctr(b) && pl.lev[b] >= 2; });
    {
        // L2QBXL items: the same leaves' centres in runs of at most `cap`
        // (one leaf each), packed largest first into items of at most cap
        // centres and L2Q_SEGS runs, each run into the open item it fills
        // best.  The largest items come first, so long workgroups start early.
        std::vector<int> leaves;
        for (int b = 0; b < nb; ++b)
            if (pl.leaf[b] && has_ctr(b) && pl.lev[b] >= 2) leaves.push_back(b);
        std::stable_sort(leaves.begin(), leaves.end(), [&](int a, int c) {
            return pl.ctr_end[a] - pl.ctr_begin[a] > pl.ctr_end[c] - pl.ctr_begin[c];
        });
        int cap = l2qbxl_item_cap(G->l2q.Pmax, G->l2q.Pmax + pl.p + 8);
        std::vector<std::pair<int, int>> runs;
        for (int b : leaves)
            for (int c = pl.ctr_begin[b]; c < pl.ctr_end[b]; c += cap)
                runs.push_back({c, std::min(c + cap, (int)pl.ctr_end[b])});
        std::stable_sort(runs.begin(), runs.end(), [](const std::pair<int, int> &a, const std::pair<int, int> &c) {
            return a.second - a.first > c.second - c.first;
        });
        std::vector<int> items, used, nrun;
        std::vector<std::vector<int>> open(cap + 1);   // open[f]: items with f free slots and a free run
        for (const auto &r : runs) {
            int sz = r.second - r.first, pick = -1;
            for (int f = sz; f < cap && pick < 0; ++f)
                if (!open[f].empty()) {
                    pick = open[f].back();
                    open[f].pop_back();
                }
            if (pick < 0) {
                pick = (int)used.size();
                items.insert(items.end(), 2 * L2Q_SEGS, 0);
                used.push_back(0);
                nrun.push_back(0);
            }
            items[(size_t)pick * 2 * L2Q_SEGS + 2 * nrun[pick]] = r.first;
            items[(size_t)pick * 2 * L2Q_SEGS + 2 * nrun[pick] + 1] = r.second;
            ++nrun[pick];
            used[pick] += sz;
            if (used[pick] < cap && nrun[pick] < L2Q_SEGS) open[cap - used[pick]].push_back(pick);
        }
        G->l2q.n = (int)used.size();
        G->l2q.d = ar.upload(items);
        G->l2q_cap = cap;
    }
    // Split every leaf's W list: boxes summed directly join the near list
    // (P2QBXL), the others go through M2QBXL.
    {
        std::vector<int32_t> ns(nb + 1, 0), nidx, ws(nb + 1, 0), widx;
        for (int b = 0; b < nb; ++b) {
            for (int i = pl.U_start[b]; i < pl.U_start[b + 1]; ++i) nidx.push_back(pl.U_idx[i]);
            for (int i = pl.W_start[b]; i < pl.W_start[b + 1]; ++i) {
                int w = pl.W_idx[i];
                if (w_is_direct(pl, w)) nidx.push_back(w);
                else widx.push_back(w);
            }
            ns[b + 1] = (int)nidx.size();
            ws[b + 1] = (int)widx.size();
        }
        G->near_start = ns; G->near_idx = nidx; G->wf_start = ws; G->wf_idx = widx;
        g.near_start = ar.upload(ns); g.near_idx = ar.upload(nidx);
        g.wf_start = ar.upload(ws); g.wf_idx = ar.upload(widx);
        // The P2QBXL work list (items {c0, c1, q0, q1} as the kernel takes
        // them).  An item of CG = min(centres, P2Q_THREADS / 2) slots gives a
        // lane ceil(sources / (P2Q_THREADS / CG)) pairs per pass over its
        // centres; a leaf whose near list would give a lane more than
        // kP2qLanePairs is split into the fewest groups of consecutive
        // centres that stay within it, so that one crowded leaf does not hold
        // its workgroup long after the rest have drained.  Items run in order
        // of decreasing lane work (each centre's result is independent of the
        // order and of the split).
        auto lane_pairs = [](long long n_c, long long n_s) {
            long long cg = std::max(1LL, std::min(n_c, (long long)P2Q_THREADS / 2));
            long long parts = P2Q_THREADS / cg;
            return ((n_s + parts - 1) / parts) * ((n_c + cg - 1) / cg);
        };
        std::vector<int32_t> qidx;
        std::vector<std::array<int32_t, 4>> qitems;
        std::vector<long long> qwork;
        G->qbx.Pmax = 0;
        for (int b = 0; b < nb; ++b) {
            if (!(pl.leaf[b] && has_ctr(b))) continue;
            G->qbx.Pmax = std::max(G->qbx.Pmax, pl.P[pl.lev[b]]);
            int q0 = (int)qidx.size();
            for (int i = ns[b]; i < ns[b + 1]; ++i)
                for (int j = pl.src_begin[nidx[i]]; j < pl.src_end[nidx[i]]; ++j) qidx.push_back(j);
            int q1 = (int)qidx.size();
            long long nc = pl.ctr_end[b] - pl.ctr_begin[b], nsrc = q1 - q0, ng = 1;
            while (ng < nc && lane_pairs((nc + ng - 1) / ng, nsrc) > kP2qLanePairs) ++ng;
            for (long long k = 0; k < ng; ++k) {
                int a = pl.ctr_begin[b] + (int)(k * nc / ng), e = pl.ctr_begin[b] + (int)((k + 1) * nc / ng);
                qitems.push_back({a, e, q0, q1});
                qwork.push_back(lane_pairs(e - a, nsrc));
            }
        }
        std::vector<int> qord(qitems.size());
        for (size_t i = 0; i < qord.size(); ++i) qord[i] = (int)i;
        std::stable_sort(qord.begin(), qord.end(), [&](int a, int b) { return qwork[a] > qwork[b]; });
        std::vector<int32_t> qflat;
        for (int i : qord) qflat.insert(qflat.end(), qitems[i].begin(), qitems[i].end());
        G->qbx.n = (int)qord.size();
        G->qbx.d = ar.upload(qflat);
        g.qsrc_idx = ar.upload(qidx);
        // sources of all X-list boxes of every box of the X-list P2L list, in list order
        std::vector<int32_t> xs0(1, 0), xidx;
        for (int b : xorder) {
            for (int i = pl.X_start[b]; i < pl.X_start[b + 1]; ++i)
                for (int j = pl.src_begin[pl.X_idx[i]]; j < pl.src_end[pl.X_idx[i]]; ++j) xidx.push_back(j);
            xs0.push_back((int32_t)xidx.size());
        }
        g.xsrc_start = ar.upload(xs0);
        g.xsrc_idx = ar.upload(xidx);
        // the cached X-list basis: per position its box and the start of its
        // row of 2 P_b + 3 entries (a box's positions are consecutive rows)
        std::vector<int32_t> xbox(std::max<size_t>(xidx.size(), 1), -1);
        std::vector<long long> xoff(std::max<size_t>(xidx.size(), 1), 0);
        for (size_t i = 0; i + 1 < xs0.size(); ++i) {
            int b = xorder[i];
            for (int q = xs0[i]; q < xs0[i + 1]; ++q) {
                xbox[q] = b;
                xoff[q] = xbas_total;
                xbas_total += 2 * pl.P[pl.lev[b]] + 3;
            }
        }
        G->n_xpos = (int)xidx.size();
        g.xsrc_box = ar.upload(xbox);
        g.xbas_off = ar.upload(xoff);
        // the leaf (level >= 2) of every source and of every centre, else -1
        std::vector<int32_t> sbox(std::max<int64_t>(pl.ns, 1), -1), cbox(std::max<int64_t>(pl.nc, 1), -1);
        for (int b = 0; b < nb; ++b) {
            if (!pl.leaf[b] || pl.lev[b] < 2) continue;
            for (int j = pl.src_begin[b]; j < pl.src_end[b]; ++j) sbox[j] = b;
            for (int c = pl.ctr_begin[b]; c < pl.ctr_end[b]; ++c) cbox[c] = b;
        }
        g.src_box = ar.upload(sbox);
        g.ctr_box = ar.upload(cbox);
    }
    G->wl = make_list(ar, pl, [&](int b) { return pl.leaf[b] && has_ctr(b) && G->wf_start[b + 1] > G->wf_start[b]; });
    // (leaf, far W box) pairs in leaf order, their output rows, per-leaf ranges
    {
        std::vector<int2> pairs;
        std::vector<long long> off;
        std::vector<int> lstart(1, 0);
        long long tot = 0;
        int nq = 2 * pl.p + 1;
        for (int b = 0; b < nb; ++b) {
            if (!(pl.leaf[b] && has_ctr(b) && G->wf_start[b + 1] > G->wf_start[b])) continue;
            for (int i = G->wf_start[b]; i < G->wf_start[b + 1]; ++i) {
                pairs.push_back(make_int2(b, G->wf_idx[i]));
                off.push_back(tot);
                tot += (long long)(pl.ctr_end[b] - pl.ctr_begin[b]) * nq;
            }
            lstart.push_back((int)pairs.size());
        }
        G->n_wpairs = (int)pairs.size();
        G->total_wy = tot;
        G->d_wpairs = ar.upload(pairs);
        G->d_wpair_off = ar.upload(off);
        G->d_wleaf_start = ar.upload(lstart);
    }
    // the W list needs the largest order among W boxes, not among the leaves
    int pw = 0;
    for (int b = 0; b < nb; ++b)
        if (pl.leaf[b] && has_ctr(b))
            for (int i = G->wf_start[b]; i < G->wf_start[b + 1]; ++i) pw = std::max(pw, pl.P[pl.lev[G->wf_idx[i]]]);
    G->wl.Pmax = pw;

    G->srad_rows = G->p2m.Pmax + 2;
    G->crad_rows = G->l2q.Pmax + pl.p + 8;
    if (!pl.opt.direct) {
        g.srow = G->srad_rows;
        G->sbas = (cd *)ar.alloc(sizeof(cd) * (size_t)G->srad_rows * std::max<int64_t>(pl.ns, 1));
        G->crad = (double *)ar.alloc(sizeof(double) * (size_t)G->crad_rows * std::max<int64_t>(pl.nc, 1));
        g.sbas = G->sbas;
        bool keep = pl.opt.keep_x_rows && xbas_total > 0 && xbas_total * sizeof(cd) <= kXBasisCap;
        G->xbas = keep ? (cd *)ar.alloc(sizeof(cd) * xbas_total) : nullptr;
        g.xbas = G->xbas;
    }
    G->d_self = ar.upload(std::vector<DevGeom>{g});
    if (ar.err != hipSuccess) return fail(ar.err == hipErrorOutOfMemory ? QBX_E_NOMEM : QBX_E_DEVICE,
                                          std::string("device upload failed: ") + hipGetErrorString(ar.err));
    return QBX_OK;
}

// Bytes of each evaluation buffer for chunks of c densities.
struct ScratchPlan {
    size_t qs, qd, coef, mp, loc, vy, wy;
    size_t total() const { return qs + qd + coef + mp + loc + vy + wy; }
};

ScratchPlan scratch_plan(const qbx_geom_s *G, int c)
{
    const Plan &pl = G->pl;
    const size_t cdb = sizeof(cd);
    auto at1 = [](long long n) { return (size_t)std::max<long long>(n, 1); };
    ScratchPlan sp{};
    sp.qs = sp.qd = cdb * c * at1(pl.ns);
    sp.coef = cdb * c * (2 * pl.p + 1) * at1(pl.nc);
    if (!pl.opt.direct) {
        sp.mp = sp.loc = cdb * c * at1(G->total_coef);
        sp.vy = cdb * c * at1(G->total_vy);
        sp.wy = cdb * c * at1(G->total_wy);
    }
    return sp;
}

qbx_status ensure_scratch(qbx_geom_s *G)
{
    if (G->sub && !G->sub->qs) {
        qbx_status q = ensure_scratch(G->sub);
        if (q != QBX_OK) return q;
    }
    if (G->qs) return QBX_OK;
    DeviceArena &s = G->scratch;
    ScratchPlan sp = scratch_plan(G, kDensChunk);
    G->qs = (cd *)s.alloc(sp.qs);
    G->qd = (cd *)s.alloc(sp.qd);
    G->coef = (cd *)s.alloc(sp.coef);
    if (!G->pl.opt.direct) {
        G->mp = (cd *)s.alloc(sp.mp);
        G->loc = (cd *)s.alloc(sp.loc);
        G->vy = (cd *)s.alloc(sp.vy);
        G->wy = (cd *)s.alloc(sp.wy);
    }
    if (s.err != hipSuccess) {
        hipError_t e = s.err;
        s.release();
        s.err = hipSuccess;
        G->qs = G->qd = G->coef = G->mp = G->loc = G->vy = G->wy = nullptr;
        return fail(e == hipErrorOutOfMemory ? QBX_E_NOMEM : QBX_E_DEVICE,
                    std::string("scratch allocation failed: ") + hipGetErrorString(e));
    }
    return QBX_OK;
}

// M2L GEMM tiles for nd densities: each (level, offset) group's columns are
// its (pair, density) combinations, cut into tiles of 16.
qbx_status ensure_tiles(qbx_geom_s *G, int nd)
{
    if (G->sub) {
        qbx_status q = ensure_tiles(G->sub, nd);
        if (q != QBX_OK) return q;
    }
    if (G->m2m_tiles[nd]) return QBX_OK;
    std::vector<M2LTile> t;
    const int pstaged_max = m2l_staged_pmax();
    for (int pass = 0; pass < 2; ++pass) {
        // the groups whose columns exceed the staged kernel's LDS first
        for (const auto &grp : G->m2l_groups) {
            if ((G->pl.P[grp.key / 40] > pstaged_max) != (pass == 0)) continue;
            int cols = grp.count * nd;
            for (int c0 = 0; c0 < cols; c0 += kM2LTileCols)
                t.push_back({grp.key, grp.start, c0, std::min(kM2LTileCols, cols - c0)});
        }
        if (pass == 0) G->m2l_split[nd] = (int)t.size();
    }
    G->m2l_tiles[nd] = G->arena.upload(t);
    G->m2l_ntiles[nd] = (int)t.size();
    // M2M: per parent level, 16-column tiles of (parent, density)
    int nlev = G->pl.nlev;
    std::vector<TTile> tm, tl;
    G->m2m_tstart[nd].assign(nlev + 1, 0);
    for (int l = 0; l < nlev; ++l) {
        G->m2m_tstart[nd][l] = (int)tm.size();
        int s0 = G->par_lvl[l], cols = (G->par_lvl[l + 1] - s0) * nd;
        for (int c0 = 0; c0 < cols; c0 += 16) tm.push_back({0, s0, c0, std::min(16, cols - c0)});
    }
    G->m2m_tstart[nd][nlev] = (int)tm.size();
    // L2L: per child level, per quadrant, 16-column tiles of (child, density)
    G->l2l_tstart[nd].assign(nlev + 1, 0);
    for (int L = 0; L < nlev; ++L) {
        G->l2l_tstart[nd][L] = (int)tl.size();
        for (int q = 0; q < 4; ++q) {
            int s0 = G->chl_lvl[L * 4 + q], cols = (G->chl_lvl[L * 4 + q + 1] - s0) * nd;
            for (int c0 = 0; c0 < cols; c0 += 16) tl.push_back({q, s0, c0, std::min(16, cols - c0)});
        }
    }
    G->l2l_tstart[nd][nlev] = (int)tl.size();
    G->m2m_tiles[nd] = G->arena.upload(tm);
    G->l2l_tiles[nd] = G->arena.upload(tl);
    if (G->arena.err != hipSuccess) {
        hipError_t e = G->arena.err;
        G->arena.err = hipSuccess;
        G->m2l_tiles[nd] = nullptr;
        return fail(QBX_E_DEVICE, std::string("tile upload failed: ") + hipGetErrorString(e));
    }
    return QBX_OK;
}

#define CHK(expr)                                                                    \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) return fail(QBX_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

hipEvent_t take_event(qbx_geom_s *G)
{
    if (!G->spare.empty()) {
        hipEvent_t e = G->spare.back();
        G->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records events around one stage's launches when profiling is on.
struct StageTimer {
    qbx_geom_s *G;
    int stage;
    int launches = 0;
    hipEvent_t a = nullptr;
    StageTimer(qbx_geom_s *g, int s, bool on) : G(g), stage(s)
    {
        if (on && (a = take_event(G))) (void)hipEventRecord(a, G->ctx->stream);
    }
    ~StageTimer()
    {
        if (!a) return;
        hipEvent_t b = take_event(G);
        if (!b) { G->spare.push_back(a); return; }
        (void)hipEventRecord(b, G->ctx->stream);
        G->pending.push_back({stage, a, b, launches});
    }
};

qbx_status harvest(qbx_geom_s *G)
{
    for (auto &r : G->pending) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        G->acc_ms[r.stage] += ms;
        G->acc_n[r.stage] += r.launches;
        G->spare.push_back(r.a);
        G->spare.push_back(r.b);
    }
    G->pending.clear();
    return QBX_OK;
}

#define STAGE(id) StageTimer timer_##id(G, id, B.timing)
#define LAUNCH(id, n, expr)        \
    do {                           \
        if ((n) > 0) timer_##id.launches++; \
        CHK(expr);                 \
    } while (0)

// The evaluation buffers of one pass through the pipeline: the geometry's
// own scratch, or parts of a caller-provided region (qbx_eval_noalloc).
struct EvalBufs {
    cd *qs, *qd, *mp, *loc, *coef, *vy, *wy;
    const EvalBufs *sub;        // the order-0 geometry's buffers (null: its own)
    bool timing;                // per-stage events, every stage in order on one stream
};

EvalBufs own_bufs(qbx_geom_s *G)
{
    return {G->qs, G->qd, G->mp, G->loc, G->coef, G->vy, G->wy, nullptr,
            G->profile};
}

qbx_status run_pipeline(qbx_geom_s *G, int nd, const cd *ss, const cd *sd, cd *u, cd *coef_out,
                        hipStream_t st, const QbxLane &lane, const EvalBufs *bufs = nullptr)
{
    const Plan &pl = G->pl;
    const DevGeom &g = G->g;
    EvalBufs own;
    if (!bufs) {
        own = own_bufs(G);
        bufs = &own;
    }
    const EvalBufs &B = *bufs;
    {
        STAGE(QBX_STAGE_CHARGES);
        LAUNCH(QBX_STAGE_CHARGES, pl.ns, launch_charges(g, nd, ss, sd, B.qs, B.qd, st));
    }
    if (pl.opt.direct) {
        STAGE(QBX_STAGE_DIRECT);
        LAUNCH(QBX_STAGE_DIRECT, pl.nc, launch_p2qbxl_direct(g, nd, B.qs, B.qd, B.coef, st));
    } else {
        qbx_status ts = ensure_tiles(G, nd);
        if (ts != QBX_OK) return ts;
        if (B.timing || !lane.side) {
            // in order: the locals are zeroed with the charges (X-list P2L
            // and L2L both add into them); concurrently, on the side stream
            STAGE(QBX_STAGE_CHARGES);
            LAUNCH(QBX_STAGE_CHARGES, G->total_coef, launch_fill_zero(B.loc, (long long)nd * G->total_coef, st));
        }
        // Fork: the side stream takes the centre J sequences, the X-list P2L,
        // the near field and (once M2M is done) M2QBXL while this stream runs
        // P2M, M2M, M2L and L2L.  With stage profiling on everything stays on
        // one stream, in order.
        const QbxLane *C = &lane;
        bool conc = !B.timing && C->side;
        hipStream_t s1 = conc ? C->side : st;
        if (conc) {
            CHK(hipEventRecord(C->ev_fork, st));
            CHK(hipStreamWaitEvent(s1, C->ev_fork, 0));
            if (!G->rad_ready) {
                CHK(launch_ctr_rad(g, G->l2q.n, G->crad, G->crad_rows, s1));
                CHK(launch_x_bas(g, G->n_xpos, G->xbas, s1));
            }
            CHK(launch_fill_zero(B.loc, (long long)nd * G->total_coef, s1));
            CHK(launch_p2l_x(g, nd, G->xl.d, G->xl.n, G->xl.Pmax, B.qs, B.qd, B.loc, true, s1));
            if (G->n_wpairs > 0) CHK(hipEventRecord(C->ev_x, s1));
            CHK(launch_p2qbxl(g, nd, G->qbx.d, G->qbx.n, B.qs, B.qd, B.coef, true, s1));
            // Without M2QBXL work one event marks the end of the side stream
            // and the caller's stream waits for it once, before L2L: each
            // event costs the waiting stream a few microseconds, and the near
            // field is done long before the downward pass.
            if (G->n_wpairs == 0) CHK(hipEventRecord(C->ev_q, s1));
        }
        {
            STAGE(QBX_STAGE_P2M);
            if (!G->rad_ready) LAUNCH(QBX_STAGE_P2M, pl.ns, launch_src_bas(g, G->sbas, st));
            LAUNCH(QBX_STAGE_P2M, G->p2m.n, launch_p2m(g, nd, G->p2m.d, G->p2m.n, G->p2m.Pmax, B.qs, B.qd, B.mp, st));
        }
        {
            STAGE(QBX_STAGE_M2M);
            for (int l = pl.nlev - 2; l >= 2; --l) {
                int t0 = G->m2m_tstart[nd][l], nt = G->m2m_tstart[nd][l + 1] - t0;
                int nrb = (2 * pl.P[l] + 1 + 15) / 16;
                LAUNCH(QBX_STAGE_M2M, nt, launch_m2m_mfma(g, nd, l, G->m2m_tiles[nd] + t0, nt, nrb, G->d_par_list, B.mp, st));
            }
        }
        if (conc && G->n_wpairs > 0) {
            // multipoles complete: M2QBXL joins the side stream after the near field
            CHK(hipEventRecord(C->ev_m, st));
            CHK(hipStreamWaitEvent(s1, C->ev_m, 0));
            CHK(launch_m2qbxl(g, nd, G->d_wpairs, G->d_wpair_off, G->n_wpairs, G->wl.Pmax, B.mp, B.wy,
                              G->wl.d, G->d_wleaf_start, G->wl.n, B.coef, s1));
            CHK(hipEventRecord(C->ev_q, s1));
        }
        {
            STAGE(QBX_STAGE_M2L);
            LAUNCH(QBX_STAGE_M2L, G->m2l_ntiles[nd],
                   launch_m2l_mfma(g, nd, G->m2l_tiles[nd], G->m2l_ntiles[nd], G->m2l_split[nd],
                                   G->m2l_Pdirect, G->m2l_Pstaged, G->m2l_nw,
                                   B.mp, B.vy, st));
        }
        if (conc) {
            CHK(hipStreamWaitEvent(st, G->n_wpairs > 0 ? C->ev_x : C->ev_q, 0));
        } else {
            STAGE(QBX_STAGE_P2L_X);
            if (!G->rad_ready) LAUNCH(QBX_STAGE_P2L_X, G->n_xpos, launch_x_bas(g, G->n_xpos, G->xbas, st));
            LAUNCH(QBX_STAGE_P2L_X, G->xl.n, launch_p2l_x(g, nd, G->xl.d, G->xl.n, G->xl.Pmax, B.qs, B.qd, B.loc, false, st));
        }
        {
            // V-list sums in list order for every level at once, then L2L
            // from the parent, level by level
            STAGE(QBX_STAGE_L2L);
            if (pl.nlev > 2) {
                int nbox = pl.level_start[pl.nlev] - pl.level_start[2];
                LAUNCH(QBX_STAGE_L2L, nbox, launch_down_all(g, nd, nbox, B.vy, B.loc, st));
            }
            for (int L = 3; L < pl.nlev; ++L) {
                int t0 = G->l2l_tstart[nd][L], nt = G->l2l_tstart[nd][L + 1] - t0;
                int nrb = (2 * pl.P[L] + 1 + 15) / 16;
                LAUNCH(QBX_STAGE_L2L, nt, launch_l2l_mfma(g, nd, L, G->l2l_tiles[nd] + t0, nt, nrb, G->d_chl_list, nullptr, B.loc, st));
            }
        }
        if (conc) {
            if (G->n_wpairs > 0) CHK(hipStreamWaitEvent(st, C->ev_q, 0));
        } else {
            {
                STAGE(QBX_STAGE_P2QBXL);
                LAUNCH(QBX_STAGE_P2QBXL, G->qbx.n, launch_p2qbxl(g, nd, G->qbx.d, G->qbx.n, B.qs, B.qd, B.coef, false, st));
            }
            STAGE(QBX_STAGE_M2QBXL);
            LAUNCH(QBX_STAGE_M2QBXL, G->n_wpairs,
                   launch_m2qbxl(g, nd, G->d_wpairs, G->d_wpair_off, G->n_wpairs, G->wl.Pmax, B.mp,
                                 B.wy, G->wl.d, G->d_wleaf_start, G->wl.n, B.coef, st));
        }
        {
            STAGE(QBX_STAGE_L2QBXL);
            if (!conc && !G->rad_ready) LAUNCH(QBX_STAGE_L2QBXL, G->l2q.n, launch_ctr_rad(g, G->l2q.n, G->crad, G->crad_rows, st));
            LAUNCH(QBX_STAGE_L2QBXL, G->l2q.n, launch_l2qbxl(g, nd, G->l2q.d, G->l2q.n, G->l2q.Pmax, G->crad, G->crad_rows,
                                                               G->l2q_cap, B.loc, B.coef, st));
        }
        // both radial sequences are enqueued ahead of every later evaluation
        // on this geometry (P2M and L2QBXL of later calls follow them in
        // stream order)
        G->rad_ready = true;
    }
    {
        STAGE(QBX_STAGE_EVAL);
        LAUNCH(QBX_STAGE_EVAL, pl.nt, launch_qbx_eval(g, nd, B.coef, u, st));
    }
    if (G->sub) {
        // the targets outside every expansion disk, through the order-0
        // geometry (it writes into u at their indices)
        STAGE(QBX_STAGE_SMOOTH);
        timer_QBX_STAGE_SMOOTH.launches++;
        qbx_status q = run_pipeline(G->sub, nd, ss, sd, u, nullptr, st, lane, B.sub);
        if (q != QBX_OK) return q;
    } else {
        STAGE(QBX_STAGE_SMOOTH);
        LAUNCH(QBX_STAGE_SMOOTH, G->g.n_smooth, launch_smooth(g, nd, B.qs, B.qd, u, st));
    }
    if (coef_out) {
        STAGE(QBX_STAGE_COEF_OUT);
        LAUNCH(QBX_STAGE_COEF_OUT, pl.nc, launch_coef_out(g, nd, B.coef, coef_out, st));
    }
    return QBX_OK;
}

// Algorithmic flops per stage for nd densities (conventions in qbxfmm.h).
void stage_work(const qbx_geom_s *G, int nd, double *f)
{
    const Plan &pl = G->pl;
    for (int s = 0; s < QBX_N_STAGES; ++s) f[s] = 0;
    double cq = 2.0 * pl.p + 1;
    auto nP = [&](int b) { return 2.0 * pl.P[pl.lev[b]] + 1; };
    int64_t n_assoc = 0;
    for (int64_t m = 0; m < pl.nt; ++m) n_assoc += pl.tgt_ctr[m] >= 0;
    f[QBX_STAGE_EVAL] = 8.0 * cq * n_assoc;
    f[QBX_STAGE_SMOOTH] = 16.0 * (double)(pl.nt - n_assoc) * pl.ns;
    if (pl.opt.direct) {
        f[QBX_STAGE_DIRECT] = 24.0 * cq * (double)pl.nc * pl.ns;
    } else {
        for (int b = 0; b < pl.n_boxes(); ++b) {
            int ns_b = pl.src_end[b] - pl.src_begin[b], nc_b = pl.ctr_end[b] - pl.ctr_begin[b];
            if (pl.lev[b] >= 2 && pl.leaf[b]) f[QBX_STAGE_P2M] += 24.0 * nP(b) * ns_b;
            if (pl.lev[b] >= 3) {
                double t = 8.0 * nP(b) * nP(pl.parent[b]);
                f[QBX_STAGE_M2M] += t;
                f[QBX_STAGE_L2L] += t;
            }
            f[QBX_STAGE_M2L] += 8.0 * nP(b) * nP(b) * (pl.V_start[b + 1] - pl.V_start[b]);
            for (int i = pl.X_start[b]; i < pl.X_start[b + 1]; ++i) {
                int c = pl.X_idx[i];
                f[QBX_STAGE_P2L_X] += 24.0 * nP(b) * (pl.src_end[c] - pl.src_begin[c]);
            }
            if (!pl.leaf[b] || nc_b == 0) continue;
            for (int i = G->near_start[b]; i < G->near_start[b + 1]; ++i) {
                int c = G->near_idx[i];
                f[QBX_STAGE_P2QBXL] += 24.0 * cq * nc_b * (pl.src_end[c] - pl.src_begin[c]);
            }
            for (int i = G->wf_start[b]; i < G->wf_start[b + 1]; ++i)
                f[QBX_STAGE_M2QBXL] += 8.0 * cq * nc_b * nP(G->wf_idx[i]);
            if (pl.lev[b] >= 2) f[QBX_STAGE_L2QBXL] += 8.0 * cq * nc_b * nP(b);
        }
    }
    for (int s = 0; s < QBX_N_STAGES; ++s) f[s] *= nd;
    if (G->sub) {
        // FMM mode: the smooth-rule targets go through the order-0 geometry
        double fs[QBX_N_STAGES];
        stage_work(G->sub, nd, fs);
        f[QBX_STAGE_SMOOTH] = 0.0;
        for (int s = 0; s < QBX_N_STAGES; ++s) f[QBX_STAGE_SMOOTH] += fs[s];
    }
}


// ---------------------------------------------------------------------------
// Batched evaluation: one fused launch per stage over all geometries of a
// pass (see FRec).  A pass holds each geometry at most once (its scratch is
// per geometry) with one chunk of up to kDensChunk densities; the stages run
// in the order and on the streams of run_pipeline.
// ---------------------------------------------------------------------------
struct BItem {
    qbx_geom_s *G;
    int nd;
    const cd *ss, *sd;
    cd *u;
};

// one step of a planned batch: a fused launch, an event record or a wait,
// on the caller's stream (0) or the side stream (1)
struct FOp {
    enum { LAUNCH, RECORD, WAIT } type;
    int launch;
    int stream;
    hipEvent_t ev;
};

qbx_status plan_pass(const std::vector<BItem> &B, const QbxLane &L, bool conc, FBuf &fb, std::vector<FOp> &ops)
{
    auto item = [](const BItem &b) {
        FItem it{};
        it.h = &b.G->g;
        it.r.g = b.G->d_self;
        it.r.nd = b.nd;
        return it;
    };
    auto stage = [&](int kind, const std::vector<FItem> &v, int stream) -> qbx_status {
        if (v.empty()) return QBX_OK;
        std::vector<int> ids;
        hipError_t e = fused_plan(fb, kind, v, ids);
        if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("fused launch plan: ") + hipGetErrorString(e));
        for (int id : ids) ops.push_back({FOp::LAUNCH, id, stream, nullptr});
        return QBX_OK;
    };
    auto record = [&](hipEvent_t e, int stream) { ops.push_back({FOp::RECORD, -1, stream, e}); };
    auto wait = [&](int stream, hipEvent_t e) { ops.push_back({FOp::WAIT, -1, stream, e}); };
#define QQ(expr)                          \
    do {                                  \
        qbx_status q_ = (expr);           \
        if (q_ != QBX_OK) return q_;      \
    } while (0)
    std::vector<FItem> v;
    for (const auto &b : B) {
        FItem it = item(b);
        it.r.in0 = b.ss;
        it.r.in1 = b.sd;
        it.r.out0 = b.G->qs;
        it.r.out1 = b.G->qd;
        v.push_back(it);
    }
    QQ(stage(FK_CHARGES, v, 0));
    v.clear();
    for (const auto &b : B)
        if (b.G->pl.opt.direct) {
            FItem it = item(b);
            it.r.in0 = b.G->qs;
            it.r.in1 = b.G->qd;
            it.r.out0 = b.G->coef;
            v.push_back(it);
        }
    QQ(stage(FK_P2QBXL_DIRECT, v, 0));
    std::vector<const BItem *> F;
    int maxlev = 0;
    for (const auto &b : B)
        if (!b.G->pl.opt.direct) {
            F.push_back(&b);
            maxlev = std::max(maxlev, b.G->pl.nlev);
        }
    auto over = [&](auto fill) {
        std::vector<FItem> w;
        for (const BItem *b : F) {
            FItem it = item(*b);
            if (fill(*b, it)) w.push_back(it);
        }
        return w;
    };
    auto v_ctr_rad = [&]() {
        return over([](const BItem &b, FItem &it) {
            it.r.i0 = b.G->crad_rows; it.r.out0 = b.G->crad; it.n = b.G->l2q.n;
            return it.n > 0 && !b.G->rad_ready;
        });
    };
    auto v_fill = [&]() {
        return over([](const BItem &b, FItem &it) {
            it.r.out0 = b.G->loc; it.n = (long long)b.nd * b.G->total_coef;
            return true;
        });
    };
    auto v_x_bas = [&]() {
        return over([](const BItem &b, FItem &it) {
            it.r.out0 = b.G->xbas; it.r.n64 = b.G->n_xpos; it.n = b.G->n_xpos;
            return it.n > 0 && b.G->xbas && !b.G->rad_ready;
        });
    };
    auto v_p2l_x = [&]() {
        return over([](const BItem &b, FItem &it) {
            const qbx_geom_s *G = b.G;
            it.r.in0 = G->xl.d; it.r.in1 = G->qs; it.r.in2 = G->qd; it.r.out0 = G->loc;
            it.n = G->xl.n; it.P = G->xl.Pmax;
            return it.n > 0;
        });
    };
    auto v_p2qbxl = [&]() {
        return over([](const BItem &b, FItem &it) {
            const qbx_geom_s *G = b.G;
            it.r.in0 = G->qbx.d; it.r.in1 = G->qs; it.r.in2 = G->qd; it.r.out0 = G->coef;
            it.n = G->qbx.n;
            return it.n > 0;
        });
    };
    auto v_m2qbxl = [&]() {
        return over([](const BItem &b, FItem &it) {
            const qbx_geom_s *G = b.G;
            it.r.in0 = G->d_wpairs; it.r.in1 = G->d_wpair_off; it.r.in2 = G->mp; it.r.out0 = G->wy;
            it.n = G->n_wpairs; it.P = G->wl.Pmax;
            return it.n > 0;
        });
    };
    auto v_wsum = [&]() {
        return over([](const BItem &b, FItem &it) {
            const qbx_geom_s *G = b.G;
            it.r.in0 = G->wl.d; it.r.in1 = G->d_wleaf_start; it.r.in2 = G->d_wpair_off; it.r.in3 = G->wy;
            it.r.out0 = G->coef; it.n = G->wl.n;
            return G->n_wpairs > 0 && it.n > 0;
        });
    };
    if (!F.empty()) {
        int s1 = conc ? 1 : 0;
        if (conc) {
            record(L.ev_fork, 0);
            wait(1, L.ev_fork);
            QQ(stage(FK_CTR_RAD, v_ctr_rad(), 1));
            QQ(stage(FK_FILL, v_fill(), 1));
            QQ(stage(FK_X_BAS, v_x_bas(), 1));
            QQ(stage(FK_P2L_X, v_p2l_x(), 1));
            record(L.ev_x, 1);
            QQ(stage(FK_P2QBXL, v_p2qbxl(), 1));
        }
        QQ(stage(FK_SRC_BAS, over([](const BItem &b, FItem &it) {
                     it.r.out0 = b.G->sbas; it.n = b.G->p2m.n;
                     return it.n > 0 && !b.G->rad_ready;
                 }), 0));
        QQ(stage(FK_P2M, over([](const BItem &b, FItem &it) {
                     const qbx_geom_s *G = b.G;
                     it.r.in0 = G->p2m.d; it.r.in1 = G->qs; it.r.in2 = G->qd; it.r.out0 = G->mp;
                     it.n = G->p2m.n; it.P = G->p2m.Pmax;
                     return it.n > 0;
                 }), 0));
        for (int l = maxlev - 2; l >= 2; --l)
            QQ(stage(FK_M2M, over([l](const BItem &b, FItem &it) {
                         const qbx_geom_s *G = b.G;
                         if (l > G->pl.nlev - 2) return false;
                         int t0 = G->m2m_tstart[b.nd][l], nt = G->m2m_tstart[b.nd][l + 1] - t0;
                         it.r.i0 = l; it.r.in0 = G->m2m_tiles[b.nd] + t0; it.r.in1 = G->d_par_list; it.r.out0 = G->mp;
                         it.n = nt; it.aux = (2 * G->pl.P[l] + 1 + 15) / 16;
                         return nt > 0;
                     }), 0));
        if (conc) {
            record(L.ev_m, 0);
            wait(1, L.ev_m);
            QQ(stage(FK_M2QBXL, v_m2qbxl(), 1));
            QQ(stage(FK_WSUM, v_wsum(), 1));
            record(L.ev_q, 1);
        }
        QQ(stage(FK_M2L, over([](const BItem &b, FItem &it) {
                     const qbx_geom_s *G = b.G;
                     it.r.in0 = G->m2l_tiles[b.nd]; it.r.in1 = G->mp; it.r.out0 = G->vy;
                     it.n = G->m2l_ntiles[b.nd]; it.P = G->m2l_Pstaged; it.aux = G->m2l_nw;
                     it.split = G->m2l_split[b.nd]; it.Psplit = G->m2l_Pdirect;
                     return it.n > 0;
                 }), 0));
        if (conc) {
            wait(0, L.ev_x);
        } else {
            QQ(stage(FK_FILL, v_fill(), 0));
            QQ(stage(FK_X_BAS, v_x_bas(), 0));
            QQ(stage(FK_P2L_X, v_p2l_x(), 0));
        }
        QQ(stage(FK_DOWN, over([](const BItem &b, FItem &it) {
                     const Plan &pl = b.G->pl;
                     if (pl.nlev <= 2) return false;
                     // level 2 only: the fused L2L levels sum their own V-list rows
                     it.r.i0 = 2; it.r.in0 = b.G->vy; it.r.out0 = b.G->loc;
                     it.n = pl.level_start[3] - pl.level_start[2];
                     return it.n > 0;
                 }), 0));
        for (int Lv = 3; Lv < maxlev; ++Lv)
            QQ(stage(FK_L2L, over([Lv](const BItem &b, FItem &it) {
                         const qbx_geom_s *G = b.G;
                         if (Lv >= G->pl.nlev) return false;
                         int t0 = G->l2l_tstart[b.nd][Lv], nt = G->l2l_tstart[b.nd][Lv + 1] - t0;
                         it.r.i0 = Lv; it.r.in0 = G->l2l_tiles[b.nd] + t0; it.r.in1 = G->d_chl_list;
                         it.r.in2 = G->vy; it.r.out0 = G->loc;
                         it.n = nt; it.aux = (2 * G->pl.P[Lv] + 1 + 15) / 16;
                         return nt > 0;
                     }), 0));
        if (conc) {
            wait(0, L.ev_q);
        } else {
            QQ(stage(FK_P2QBXL, v_p2qbxl(), 0));
            QQ(stage(FK_M2QBXL, v_m2qbxl(), 0));
            QQ(stage(FK_WSUM, v_wsum(), 0));
            QQ(stage(FK_CTR_RAD, v_ctr_rad(), 0));
        }
        (void)s1;
        QQ(stage(FK_L2QBXL, over([](const BItem &b, FItem &it) {
                     const qbx_geom_s *G = b.G;
                     it.r.in0 = G->l2q.d; it.r.in1 = G->crad; it.r.in2 = G->loc; it.r.out0 = G->coef;
                     it.r.i0 = G->l2q_cap;
                     it.n = G->l2q.n; it.P = G->l2q.Pmax; it.aux = G->crad_rows;
                     return it.n > 0;
                 }), 0));
    }
    v.clear();
    for (const auto &b : B) {
        FItem it = item(b);
        it.r.in0 = b.G->coef;
        it.r.out0 = b.u;
        v.push_back(it);
    }
    QQ(stage(FK_EVAL, v, 0));
    v.clear();
    for (const auto &b : B) {
        FItem it = item(b);
        it.r.in0 = b.G->qs;
        it.r.in1 = b.G->qd;
        it.r.out0 = b.u;
        v.push_back(it);
    }
    QQ(stage(FK_SMOOTH, v, 0));
#undef QQ
    return QBX_OK;
}

// Copies the planned records and maps to the device (one copy on st).
qbx_status fused_upload(qbx_ctx_s *C, const FBuf &fb, hipStream_t st)
{
    size_t n = fb.bytes.size();
    // the staging buffer is free once the previous copy out of it is done,
    // the device buffer once the launches of the previous batch have run
    if (C->fz_used) {
        CHK(hipEventSynchronize(C->fz_copied));
        CHK(hipStreamWaitEvent(st, C->fz_done, 0));
    }
    if (n > C->fz_cap) {
        if (C->fz_used) CHK(hipEventSynchronize(C->fz_done));
        if (C->fz_host) (void)hipHostFree(C->fz_host);
        if (C->fz_dev) (void)hipFree(C->fz_dev);
        C->fz_host = C->fz_dev = nullptr;
        C->fz_cap = 0;
        size_t cap = std::max<size_t>(n + n / 2, 1 << 20);
        hipError_t e = hipHostMalloc((void **)&C->fz_host, cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void **)&C->fz_dev, cap);
        if (e != hipSuccess) {
            if (C->fz_host) (void)hipHostFree(C->fz_host);
            C->fz_host = nullptr;
            return fail(e == hipErrorOutOfMemory ? QBX_E_NOMEM : QBX_E_DEVICE,
                        std::string("batch launch records: ") + hipGetErrorString(e));
        }
        C->fz_cap = cap;
    }
    std::memcpy(C->fz_host, fb.bytes.data(), n);
    CHK(hipMemcpyAsync(C->fz_dev, C->fz_host, n, hipMemcpyHostToDevice, st));
    CHK(hipEventRecord(C->fz_copied, st));
    C->fz_used = true;
    return QBX_OK;
}

}  // namespace

extern "C" {

qbx_status qbx_ctx_create(int32_t device, void *stream, qbx_ctx *out)
{
    if (!out) return fail(QBX_E_INVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0)
        return fail(QBX_E_DEVICE, std::string("no HIP device available (hipGetDeviceCount: ") +
                                      hipGetErrorString(e) + ", count " + std::to_string(n) + ")");
    if (device < 0 || device >= n) return fail(QBX_E_INVAL, "device index out of range");
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    // set-up of the static buffers of qbx_eval_noalloc on this device
    if (!noalloc_base(device, &e))
        return fail(QBX_E_DEVICE, std::string("hipGetSymbolAddress (static evaluation buffers): ") +
                                      hipGetErrorString(e));
    auto *c = new (std::nothrow) qbx_ctx_s();
    if (!c) return fail(QBX_E_NOMEM, "host allocation failed");
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    // default priority on purpose; without the streams the pipeline runs in order
    if (!lane_create(c->lane) ||
        hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fz_copied, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fz_done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        lane_destroy(c->lane);
        if (c->ev_in) (void)hipEventDestroy(c->ev_in);
        if (c->ev_out) (void)hipEventDestroy(c->ev_out);
        if (c->gstream) (void)hipStreamDestroy(c->gstream);
        if (c->fz_copied) (void)hipEventDestroy(c->fz_copied);
        if (c->fz_done) (void)hipEventDestroy(c->fz_done);
        c->gstream = nullptr;
        c->ev_in = c->ev_out = c->fz_copied = c->fz_done = nullptr;
    }
    *out = c;
    return QBX_OK;
}

const char *qbx_ctx_last_error(qbx_ctx ctx)
{
    static thread_local std::string copy;
    if (!ctx) {
        copy.clear();
        return copy.c_str();
    }
    std::lock_guard<std::mutex> lk(ctx->err_mu);
    copy = ctx->err;
    return copy.c_str();
}

qbx_status qbx_ctx_set_stream(qbx_ctx ctx, void *stream)
{
    if (!ctx) return fail(QBX_E_INVAL, "null context");
    QBX_CTX_EXCLUSIVE(ctx);
    ctx->stream = static_cast<hipStream_t>(stream);
    return QBX_OK;
}

namespace {

void ctx_release(qbx_ctx_s *ctx)
{
    if (--ctx->refs > 0) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    if (ctx->lane.side) (void)hipStreamSynchronize(ctx->lane.side);
    lane_destroy(ctx->lane);
    if (ctx->fz_copied) (void)hipEventDestroy(ctx->fz_copied);
    if (ctx->fz_done) (void)hipEventDestroy(ctx->fz_done);
    if (ctx->fz_host) (void)hipHostFree(ctx->fz_host);
    if (ctx->fz_dev) (void)hipFree(ctx->fz_dev);
    if (ctx->gstream) {
        (void)hipStreamSynchronize(ctx->gstream);
        (void)hipStreamDestroy(ctx->gstream);
    }
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->kw) (void)hipFree(ctx->kw);
    delete ctx;
}

}  // namespace

qbx_status qbx_ctx_destroy(qbx_ctx ctx)
{
    if (!ctx) return QBX_OK;
    ctx_release(ctx);
    return QBX_OK;
}

namespace {

void free_geom(qbx_geom_s *G)
{
    if (!G) return;
    free_geom(G->sub);
    G->sub = nullptr;
    G->scratch.release();
    G->arena.release();
    delete G;
}

// FMM mode with targets outside every expansion disk: the plan of the
// order-0 geometry that serves them (sources as pl's, centres at those
// targets, each target bound to its own centre, p = 0; the same tolerance
// and tree options), and the targets' indices.  False when there is none.
bool smooth_sub_plan(const Plan &pl, Plan &out, std::vector<int32_t> &idx, Error &err)
{
    err = {QBX_OK, ""};
    idx.clear();
    if (pl.opt.direct) return false;
    for (int64_t m = 0; m < pl.nt; ++m)
        if (pl.tgt_ctr[m] < 0) idx.push_back((int32_t)m);
    if (idx.empty()) return false;
    int64_t n = (int64_t)idx.size();
    std::vector<double> px(n), py(n), pr(n, 1e-300);
    std::vector<int32_t> own(n);
    for (int64_t i = 0; i < n; ++i) {
        px[i] = pl.tx[idx[i]];
        py[i] = pl.ty[idx[i]];
        own[i] = (int32_t)i;
    }
    qbx_options o = pl.opt;
    o.p = 0;
    o.p_add = -1;
    err = build_plan(out, pl.omega, pl.eps, o, pl.ns, pl.sx.data(), pl.sy.data(), pl.w.data(), pl.nx.data(),
                     pl.ny.data(), pl.sh.data(), n, px.data(), py.data(), pr.data(), n, px.data(), py.data(),
                     own.data());
    return true;
}

qbx_status build_device(qbx_geom_s *G);

qbx_status make_smooth_sub(qbx_geom_s *G)
{
    qbx_geom_s *S = new qbx_geom_s();
    Error e;
    std::vector<int32_t> idx;
    if (!smooth_sub_plan(G->pl, S->pl, idx, e)) {
        delete S;
        return QBX_OK;
    }
    if (e.status != QBX_OK) {
        delete S;
        return fail(e.status, "order-0 geometry of the smooth-rule targets: " + e.msg);
    }
    S->ctx = G->ctx;
    S->out_map = idx;
    S->out_stride = G->pl.nt;
    qbx_status st = build_device(S);
    if (st != QBX_OK) {
        free_geom(S);
        return st;
    }
    G->sub = S;
    return QBX_OK;
}

// Resident data of G without allocating: the bytes its packed allocation
// takes (G->pl, out_map and out_stride set; G itself is not modified), and
// optionally those of its evaluation scratch.
qbx_status sized_resident(qbx_geom_s *G, size_t *bytes, size_t *scratch_bytes = nullptr)
{
    qbx_geom_s D;
    D.ctx = G->ctx;
    std::swap(D.pl, G->pl);
    D.out_map = G->out_map;
    D.out_stride = G->out_stride;
    D.arena.sizing = true;
    qbx_status st = upload(&D);
    for (int nd = 1; st == QBX_OK && !D.pl.opt.direct && nd <= kDensChunk; ++nd) st = ensure_tiles(&D, nd);
    if (scratch_bytes) *scratch_bytes = scratch_plan(&D, kDensChunk).total();
    std::swap(D.pl, G->pl);
    *bytes = D.arena.off;
    return st;
}

// G's resident device data (G->pl, out_map and out_stride set): points,
// tree, lists, tables and the GEMM tile lists of every chunk size, made now
// so that evaluations (qbx_eval_noalloc in particular) never allocate them,
// in one allocation filled by one copy; then the order-0 geometry of the
// smooth-rule targets.
qbx_status build_device(qbx_geom_s *G)
{
    size_t need = 0;
    qbx_status st = sized_resident(G, &need);
    if (st != QBX_OK) return st;
    hipError_t e = G->arena.reserve(need);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? QBX_E_NOMEM : QBX_E_DEVICE,
                    std::string("device allocation of the geometry: ") + hipGetErrorString(e));
    st = upload(G);
    for (int nd = 1; st == QBX_OK && !G->pl.opt.direct && nd <= kDensChunk; ++nd) st = ensure_tiles(G, nd);
    e = G->arena.commit();
    if (st != QBX_OK) return st;
    if (e != hipSuccess)
        return fail(QBX_E_DEVICE, std::string("geometry upload: ") + hipGetErrorString(e));
    return make_smooth_sub(G);
}

}  // namespace

qbx_status qbx_geom_from_plan(qbx_ctx ctx, qbx_plan plan, qbx_geom *out)
{
    if (!ctx || !plan || !out) return fail(QBX_E_INVAL, "null argument");
    QBX_CTX_CALL(ctx);
    *out = nullptr;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    qbx_geom_s *G = nullptr;
    try {
        G = new qbx_geom_s();
        G->ctx = ctx;
        G->pl = plan->pl;
        qbx_status st = build_device(G);
        if (st != QBX_OK) {
            free_geom(G);
            return st;
        }
    } catch (const std::bad_alloc &) {
        free_geom(G);
        return fail(QBX_E_NOMEM, "host allocation failed while building tables");
    }
    ++ctx->refs;
    *out = G;
    return QBX_OK;
}

qbx_status qbx_geom_create(qbx_ctx ctx, double omega, double eps, const qbx_options *opt,
                           int64_t n_src, const double *sx, const double *sy, const double *w,
                           const double *nx, const double *ny, const double *sh, int64_t n_ctr,
                           const double *cx, const double *cy, const double *cr, int64_t n_tgt,
                           const double *tx, const double *ty, const int32_t *tgt_ctr,
                           qbx_geom *out)
{
    if (!out) return fail(QBX_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(QBX_E_INVAL, "null context");
    QBX_CTX_CALL(ctx);
    qbx_plan plan = nullptr;
    qbx_status st = qbx_plan_create(omega, eps, opt, n_src, sx, sy, w, nx, ny, sh, n_ctr, cx, cy,
                                    cr, n_tgt, tx, ty, tgt_ctr, &plan);
    if (st != QBX_OK) return st;
    st = qbx_geom_from_plan(ctx, plan, out);
    qbx_plan_destroy(plan);
    return st;
}

qbx_status qbx_geom_destroy(qbx_geom G)
{
    if (!G) return QBX_OK;
    QBX_CTX_CALL(G->ctx);
    (void)hipSetDevice(G->ctx->device);
    if (G->ctx->stream) (void)hipStreamSynchronize(G->ctx->stream);
    else (void)hipDeviceSynchronize();
    if (G->ctx->gstream) (void)hipStreamSynchronize(G->ctx->gstream);
    if (G->ctx->lane.side) (void)hipStreamSynchronize(G->ctx->lane.side);
    qbx_ctx_s *ctx = G->ctx;
    free_geom(G);
    ctx_release(ctx);
    return QBX_OK;
}

qbx_status qbx_geom_stats(qbx_geom G, qbx_stats *out)
{
    if (!G || !out) return fail(QBX_E_INVAL, "null argument");
    fill_stats(G->pl, out);
    out->device_bytes = G->arena.bytes + G->scratch.bytes;
    if (G->sub) out->device_bytes += G->sub->arena.bytes + G->sub->scratch.bytes;
    return QBX_OK;
}

size_t qbx_geom_bytes(qbx_geom G, int32_t n_dens)
{
    if (!G) return 0;
    if (G->sub) {
        // the order-0 geometry of the smooth-rule targets, counted once
        qbx_geom_s *S = G->sub;
        G->sub = nullptr;
        size_t b = qbx_geom_bytes(G, n_dens) + qbx_geom_bytes(S, n_dens);
        G->sub = S;
        return b;
    }
    // the scratch serves chunks of kDensChunk densities; the GEMM tile lists are resident
    (void)n_dens;
    return G->arena.bytes + scratch_plan(G, kDensChunk).total();
}

size_t qbx_plan_bytes(qbx_plan plan, int32_t n_dens)
{
    if (!plan) return 0;
    (void)n_dens;
    try {
        size_t total = 0;
        qbx_geom_s G;
        G.pl = plan->pl;
        size_t res = 0, scr = 0;
        if (sized_resident(&G, &res, &scr) != QBX_OK) return 0;
        total = res + scr;
        qbx_geom_s S;
        Error e;
        std::vector<int32_t> idx;
        if (smooth_sub_plan(G.pl, S.pl, idx, e)) {
            if (e.status != QBX_OK) return 0;
            S.out_map = idx;
            S.out_stride = G.pl.nt;
            if (sized_resident(&S, &res, &scr) != QBX_OK) return 0;
            total += res + scr;
        }
        return total;
    } catch (const std::bad_alloc &) {
        return 0;
    }
}

qbx_status qbx_geom_association(qbx_geom G, int32_t *tgt_ctr_out)
{
    if (!G || (!tgt_ctr_out && G->pl.nt)) return fail(QBX_E_INVAL, "null argument");
    std::copy(G->pl.tgt_ctr.begin(), G->pl.tgt_ctr.end(), tgt_ctr_out);
    return QBX_OK;
}

qbx_status qbx_geom_profile(qbx_geom G, int32_t enable)
{
    if (!G) return fail(QBX_E_INVAL, "null geometry");
    QBX_CTX_CALL(G->ctx);
    G->profile = enable != 0;
    return QBX_OK;
}

qbx_status qbx_geom_stage_times(qbx_geom G, double *ms, int64_t *launches, int32_t reset)
{
    if (!G) return fail(QBX_E_INVAL, "null geometry");
    QBX_CTX_CALL(G->ctx);
    qbx_status st = harvest(G);
    if (st != QBX_OK) return st;
    for (int s = 0; s < QBX_N_STAGES; ++s) {
        if (ms) ms[s] = G->acc_ms[s];
        if (launches) launches[s] = G->acc_n[s];
        if (reset) { G->acc_ms[s] = 0; G->acc_n[s] = 0; }
    }
    return QBX_OK;
}

qbx_status qbx_geom_work(qbx_geom G, int32_t n_dens, double *flops)
{
    if (!G || !flops || n_dens < 1) return fail(QBX_E_INVAL, "invalid argument");
    stage_work(G, n_dens, flops);
    return QBX_OK;
}

// All chunks of one evaluation, enqueued on stream st.
qbx_status eval_chunks(qbx_geom_s *G, int32_t n_dens, const void *sigma_s, const void *sigma_d, void *u,
                       void *coef, hipStream_t st, const QbxLane &lane)
{
    const Plan &pl = G->pl;
    long long nq = 2 * pl.p + 1;
    for (int d0 = 0; d0 < n_dens; d0 += kDensChunk) {
        int nd = std::min(kDensChunk, n_dens - d0);
        const cd *ss = sigma_s ? static_cast<const cd *>(sigma_s) + (long long)d0 * pl.ns : nullptr;
        const cd *sd = sigma_d ? static_cast<const cd *>(sigma_d) + (long long)d0 * pl.ns : nullptr;
        cd *uu = static_cast<cd *>(u) + (long long)d0 * pl.nt;
        cd *co = coef ? static_cast<cd *>(coef) + (long long)d0 * nq * pl.nc : nullptr;
        qbx_status q = run_pipeline(G, nd, ss, sd, uu, co, st, lane);
        if (q != QBX_OK) return q;
    }
    return QBX_OK;
}

constexpr size_t kMaxGraphs = 8;   // captured argument sets kept per geometry

// The captured evaluation for these arguments, capturing it on first use.
qbx_status graph_for(qbx_geom_s *G, int32_t n_dens, const void *sigma_s, const void *sigma_d, void *u,
                     void *coef, hipGraphExec_t *out)
{
    for (auto &r : G->graphs)
        if (r.n_dens == n_dens && r.ss == sigma_s && r.sd == sigma_d && r.u == u && r.coef == coef) {
            r.used = ++G->graph_clock;
            *out = r.exec;
            return QBX_OK;
        }
    // everything that allocates happens before the capture
    for (int d0 = 0; d0 < n_dens; d0 += kDensChunk) {
        qbx_status q = ensure_tiles(G, std::min(kDensChunk, n_dens - d0));
        if (q != QBX_OK) return q;
    }
    hipStream_t gs = G->ctx->gstream;
    hipError_t e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    // A captured pipeline only records the radial-sequence launches; they run
    // when the graph does.  Until then the flag that lets later evaluations
    // skip them must not stand (the caller clears it again if the launch
    // fails).
    bool rad0 = G->rad_ready, srad0 = G->sub && G->sub->rad_ready;
    auto undo = [&]() {
        G->rad_ready = rad0;
        if (G->sub) G->sub->rad_ready = srad0;
    };
    qbx_status q = eval_chunks(G, n_dens, sigma_s, sigma_d, u, coef, gs, G->ctx->lane);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(gs, &graph);
    if (q != QBX_OK) {
        undo();
        if (graph) (void)hipGraphDestroy(graph);
        return q;
    }
    if (e != hipSuccess) {
        undo();
        return fail(QBX_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        undo();
        return fail(QBX_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (G->graphs.size() >= kMaxGraphs) {
        size_t lru = 0;
        for (size_t i = 1; i < G->graphs.size(); ++i)
            if (G->graphs[i].used < G->graphs[lru].used) lru = i;
        // the evicted graph may still run: wait for the library's stream
        (void)hipStreamSynchronize(gs);
        (void)hipGraphExecDestroy(G->graphs[lru].exec);
        G->graphs.erase(G->graphs.begin() + lru);
    }
    G->graphs.push_back({n_dens, sigma_s, sigma_d, u, coef, exec, ++G->graph_clock});
    *out = exec;
    return QBX_OK;
}

}  // extern "C"

namespace {

// qbx_eval with some arrays in host memory: those are copied through device
// buffers of the call's own on the context's stream, and the call returns
// once the results are back in host memory (the device-memory form returns
// at once).  The copies cross PCIe: for repeated evaluations keep the arrays
// in device memory.
qbx_status eval_staged(qbx_geom_s *G, int n_dens, const void *sigma_s, const void *sigma_d, void *u, void *coef)
{
    const Plan &pl = G->pl;
    const int dev = G->ctx->device;
    hipStream_t st = G->ctx->stream;
    const size_t nq = 2 * (size_t)pl.p + 1;
    struct Arg {
        const void *host_in;   // copied in before the evaluation
        void *host_out;        // copied out after it
        size_t bytes;
        void *dev = nullptr;
    };
    Arg a[4] = {{sigma_s, nullptr, sigma_s ? sizeof(cd) * (size_t)n_dens * pl.ns : 0},
                {sigma_d, nullptr, sigma_d ? sizeof(cd) * (size_t)n_dens * pl.ns : 0},
                {nullptr, u, u ? sizeof(cd) * (size_t)n_dens * pl.nt : 0},
                {nullptr, coef, coef ? sizeof(cd) * (size_t)n_dens * nq * pl.nc : 0}};
    const void *where[4] = {sigma_s, sigma_d, u, coef};
    auto cleanup = [&]() {
        for (Arg &x : a)
            if (x.dev) (void)hipFree(x.dev);
    };
    hipError_t e = hipSuccess;
    for (int i = 0; i < 4 && e == hipSuccess; ++i) {
        if (!where[i] || a[i].bytes == 0 || device_readable(where[i], dev)) {
            a[i].host_in = nullptr;
            a[i].host_out = nullptr;
            continue;
        }
        e = hipMalloc(&a[i].dev, a[i].bytes);
        if (e == hipSuccess && a[i].host_in)
            e = hipMemcpyAsync(a[i].dev, a[i].host_in, a[i].bytes, hipMemcpyHostToDevice, st);
    }
    if (e != hipSuccess) {
        cleanup();
        return fail(e == hipErrorOutOfMemory ? QBX_E_NOMEM : QBX_E_DEVICE,
                    std::string("staging host arrays: ") + hipGetErrorString(e));
    }
    auto pick = [&](int i) { return a[i].dev ? a[i].dev : const_cast<void *>(where[i]); };
    qbx_status q = ensure_scratch(G);
    if (q == QBX_OK) q = eval_chunks(G, n_dens, pick(0), pick(1), pick(2), pick(3), st, G->ctx->lane);
    for (int i = 2; i < 4 && q == QBX_OK && e == hipSuccess; ++i)
        if (a[i].dev) e = hipMemcpyAsync(a[i].host_out, a[i].dev, a[i].bytes, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    cleanup();
    if (q != QBX_OK) return q;
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("staged evaluation: ") + hipGetErrorString(e));
    return QBX_OK;
}

}  // namespace

extern "C" {

qbx_status qbx_eval(qbx_geom G, int32_t n_dens, const void *sigma_s, const void *sigma_d, void *u,
                    void *coef)
{
    if (!G) return fail(QBX_E_INVAL, "null geometry");
    QBX_CTX_EXCLUSIVE(G->ctx);
    if (n_dens < 1 || n_dens > 64) return fail(QBX_E_INVAL, "n_dens must lie in 1..64");
    if (!u && G->pl.nt) return fail(QBX_E_INVAL, "u is NULL");
    if (!sigma_s && !sigma_d) return fail(QBX_E_INVAL, "both densities are NULL");
    hipError_t e = hipSetDevice(G->ctx->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    const int dev = G->ctx->device;
    if (!device_readable(sigma_s, dev) || !device_readable(sigma_d, dev) || !device_readable(u, dev) ||
        !device_readable(coef, dev))
        return eval_staged(G, n_dens, sigma_s, sigma_d, u, coef);
    qbx_status st = ensure_scratch(G);
    if (st != QBX_OK) return st;
    const qbx_ctx_s *C = G->ctx;
    if (G->graph_on && !G->profile && C->gstream) {
        hipGraphExec_t exec = nullptr;
        st = graph_for(G, n_dens, sigma_s, sigma_d, u, coef, &exec);
        if (st != QBX_OK) return st;
        e = hipEventRecord(C->ev_in, C->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(C->gstream, C->ev_in, 0);
        if (e == hipSuccess) e = hipGraphLaunch(exec, C->gstream);
        if (e != hipSuccess) {
            // the radial sequences recorded in the graph may never have run
            G->rad_ready = false;
            if (G->sub) G->sub->rad_ready = false;
            return fail(QBX_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        }
        CHK(hipEventRecord(C->ev_out, C->gstream));
        CHK(hipStreamWaitEvent(C->stream, C->ev_out, 0));
        return QBX_OK;
    }
    return eval_chunks(G, n_dens, sigma_s, sigma_d, u, coef, C->stream, C->lane);
}

namespace {

// Evaluation buffers of G (and of its order-0 geometry) for chunks of c
// densities, laid out from `base` at 256-byte boundaries.  Returns the end
// offset; with base null only sizes are computed.
size_t carve_bufs(const qbx_geom_s *G, int c, unsigned char *base, size_t off, EvalBufs *B, EvalBufs *Bsub)
{
    ScratchPlan sp = scratch_plan(G, c);
    auto take = [&](size_t n) {
        off = (off + 255) & ~(size_t)255;
        unsigned char *p = base ? base + off : nullptr;
        off += n;
        return p;
    };
    B->qs = (cd *)take(sp.qs);
    B->qd = (cd *)take(sp.qd);
    B->coef = (cd *)take(sp.coef);
    B->mp = (cd *)take(sp.mp);
    B->loc = (cd *)take(sp.loc);
    B->vy = (cd *)take(sp.vy);
    B->wy = (cd *)take(sp.wy);
    B->timing = false;
    B->sub = nullptr;
    if (G->sub) {
        off = carve_bufs(G->sub, c, base, off, Bsub, nullptr);
        B->sub = Bsub;
    }
    return off;
}

}  // namespace

qbx_status qbx_eval_noalloc(qbx_geom G, int32_t n_dens, const void *sigma_s, const void *sigma_d, void *u,
                            void *coef)
{
    if (!G) return fail(QBX_E_INVAL, "null geometry");
    QBX_CTX_EXCLUSIVE(G->ctx);
    if (n_dens < 1 || n_dens > 64) return fail(QBX_E_INVAL, "n_dens must lie in 1..64");
    if (!u && G->pl.nt) return fail(QBX_E_INVAL, "u is NULL");
    if (!sigma_s && !sigma_d) return fail(QBX_E_INVAL, "both densities are NULL");
    const qbx_ctx_s *C = G->ctx;
    hipError_t e = hipSetDevice(C->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    if (!device_readable(sigma_s, C->device) || !device_readable(sigma_d, C->device) ||
        !device_readable(u, C->device) || !device_readable(coef, C->device))
        return fail(QBX_E_INVAL, "qbx_eval_noalloc: every array must be device memory of the context's device");
    unsigned char *base = noalloc_base(C->device, &e);
    if (!base) return fail(QBX_E_DEVICE, std::string("static evaluation buffers: ") + hipGetErrorString(e));
    // the largest chunk of densities whose buffers fit the static array
    EvalBufs B{}, Bs{};
    int c = std::min<int>(kDensChunk, n_dens);
    for (; c >= 1; --c)
        if (carve_bufs(G, c, nullptr, 0, &B, &Bs) <= (size_t)QBX_NOALLOC_SCRATCH_BYTES) break;
    if (c < 1) {
        size_t need = carve_bufs(G, 1, nullptr, 0, &B, &Bs);
        return fail(QBX_E_UNSUPPORTED, "qbx_eval_noalloc: the geometry needs " + std::to_string(need) +
                                           " bytes of evaluation buffers for one density, more than the " +
                                           std::to_string((size_t)QBX_NOALLOC_SCRATCH_BYTES) +
                                           " of the static array; use qbx_eval");
    }
    carve_bufs(G, c, base, 0, &B, &Bs);
    const Plan &pl = G->pl;
    long long nq = 2 * pl.p + 1;
    for (int d0 = 0; d0 < n_dens; d0 += c) {
        int nd = std::min(c, n_dens - d0);
        const cd *ss = sigma_s ? static_cast<const cd *>(sigma_s) + (long long)d0 * pl.ns : nullptr;
        const cd *sd = sigma_d ? static_cast<const cd *>(sigma_d) + (long long)d0 * pl.ns : nullptr;
        cd *uu = static_cast<cd *>(u) + (long long)d0 * pl.nt;
        cd *co = coef ? static_cast<cd *>(coef) + (long long)d0 * nq * pl.nc : nullptr;
        qbx_status q = run_pipeline(G, nd, ss, sd, uu, co, C->stream, C->lane, &B);
        if (q != QBX_OK) return q;
    }
    return QBX_OK;
}

qbx_status qbx_eval_batch(qbx_ctx ctx, int32_t n_geom, const qbx_geom *geoms, const int32_t *n_dens,
                          const void *const *sigma_s, const void *const *sigma_d, void *const *u)
{
    if (!ctx || n_geom < 0 || (n_geom && (!geoms || !n_dens || !u))) return fail(QBX_E_INVAL, "invalid argument");
    QBX_CTX_EXCLUSIVE(ctx);
    if (n_geom == 0) return QBX_OK;
    for (int i = 0; i < n_geom; ++i) {
        qbx_geom G = geoms[i];
        if (!G || G->ctx != ctx) return fail(QBX_E_INVAL, "geometry missing or from another context");
        if (n_dens[i] < 1 || n_dens[i] > 64) return fail(QBX_E_INVAL, "n_dens must lie in 1..64");
        if (!u[i] && G->pl.nt) return fail(QBX_E_INVAL, "u is NULL");
        if ((!sigma_s || !sigma_s[i]) && (!sigma_d || !sigma_d[i])) return fail(QBX_E_INVAL, "both densities are NULL");
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    auto dens = [&](const void *const *a, int i) { return a ? a[i] : nullptr; };
    for (int i = 0; i < n_geom; ++i)
        if (!device_readable(dens(sigma_s, i), ctx->device) || !device_readable(dens(sigma_d, i), ctx->device) ||
            !device_readable(u[i], ctx->device))
            return fail(QBX_E_INVAL, "qbx_eval_batch: entry " + std::to_string(i) +
                                         " has an array outside the context's device memory");
    bool serial = !ctx->fz_copied;
    for (int i = 0; i < n_geom; ++i) serial = serial || geoms[i]->profile || geoms[i]->graph_on;
    if (serial) {
        // stage profiling or graph replay on some geometry: one after another
        for (int i = 0; i < n_geom; ++i) {
            qbx_status q = qbx_eval(geoms[i], n_dens[i], dens(sigma_s, i), dens(sigma_d, i), u[i], nullptr);
            if (q != QBX_OK) return q;
        }
        return QBX_OK;
    }
    // passes: the k-th chunk that names a geometry goes to pass k (a
    // geometry's scratch serves one chunk at a time)
    std::vector<std::vector<BItem>> passes;
    std::vector<std::pair<qbx_geom_s *, int>> seen;
    for (int d0 = 0;; d0 += kDensChunk) {
        bool any = false;
        for (int i = 0; i < n_geom; ++i) {
            if (n_dens[i] <= d0) continue;
            any = true;
            qbx_geom_s *G = geoms[i];
            qbx_status q = ensure_scratch(G);
            if (q != QBX_OK) return q;
            int nd = std::min(kDensChunk, n_dens[i] - d0);
            if (!G->pl.opt.direct && (q = ensure_tiles(G, nd)) != QBX_OK) return q;
            int k = 0;
            for (auto &sv : seen)
                if (sv.first == G) k = ++sv.second;
            if (k == 0) seen.push_back({G, 0});
            if ((int)passes.size() <= k) passes.resize(k + 1);
            const Plan &pl = G->pl;
            const void *ss = dens(sigma_s, i), *sd = dens(sigma_d, i);
            BItem it{G, nd, ss ? static_cast<const cd *>(ss) + (long long)d0 * pl.ns : nullptr,
                     sd ? static_cast<const cd *>(sd) + (long long)d0 * pl.ns : nullptr,
                     static_cast<cd *>(u[i]) + (long long)d0 * pl.nt};
            passes[k].push_back(it);
            if (G->sub) {
                // the smooth-rule targets: the order-0 geometry in the same
                // pass, writing into the same output
                it.G = G->sub;
                passes[k].push_back(it);
            }
        }
        if (!any) break;
    }
    FBuf fb;
    std::vector<FOp> ops;
    bool conc = ctx->lane.side != nullptr;
    for (const auto &B : passes) {
        qbx_status q = plan_pass(B, ctx->lane, conc, fb, ops);
        if (q != QBX_OK) return q;
    }
    hipStream_t st = ctx->stream;
    qbx_status q = fused_upload(ctx, fb, st);
    if (q != QBX_OK) return q;
    for (const FOp &op : ops) {
        hipStream_t s = op.stream ? ctx->lane.side : st;
        switch (op.type) {
        case FOp::LAUNCH: CHK(fused_launch(fb.launches[op.launch], ctx->fz_dev, s)); break;
        case FOp::RECORD: CHK(hipEventRecord(op.ev, s)); break;
        case FOp::WAIT: CHK(hipStreamWaitEvent(s, op.ev, 0)); break;
        }
    }
    // the geometry-only sequences of every geometry in the batch are now
    // enqueued ahead of any later evaluation
    for (const auto &P : passes)
        for (const auto &b : P)
            if (!b.G->pl.opt.direct) b.G->rad_ready = true;
    CHK(hipEventRecord(ctx->fz_done, st));
    return QBX_OK;
}

qbx_status qbx_geom_autotune(qbx_geom G, int32_t n_dens, int32_t *choice_out)
{
    if (!G) return fail(QBX_E_INVAL, "null geometry");
    QBX_CTX_EXCLUSIVE(G->ctx);
    if (n_dens < 1 || n_dens > 64) return fail(QBX_E_INVAL, "n_dens must lie in 1..64");
    hipError_t e = hipSetDevice(G->ctx->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    if (G->pl.opt.direct || G->g.far32 || G->m2l_groups.empty()) {
        if (choice_out) *choice_out = G->m2l_nw;
        return QBX_OK;
    }
    qbx_status st = ensure_scratch(G);
    if (st != QBX_OK) return st;
    // Whole evaluations with zero densities, timed with HIP events on the
    // context's stream: the M2L configuration that makes the evaluation
    // fastest in context (caches and the overlapped side stream included).
    // Candidates: the common row-block count, about half of it, and the
    // direct-load kernel (0).  They compute the same sums in the same order.
    const Plan &pl = G->pl;
    size_t ns = sizeof(cd) * (size_t)n_dens * std::max<int64_t>(pl.ns, 1);
    size_t nu = sizeof(cd) * (size_t)n_dens * std::max<int64_t>(pl.nt, 1);
    void *dsig = nullptr, *du = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s = G->ctx->stream;
    auto cleanup = [&]() {
        if (dsig) (void)hipFree(dsig);
        if (du) (void)hipFree(du);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    };
    if (hipMalloc(&dsig, ns) != hipSuccess || hipMalloc(&du, nu) != hipSuccess ||
        hipMemsetAsync(dsig, 0, ns, s) != hipSuccess || hipEventCreate(&a) != hipSuccess ||
        hipEventCreate(&b) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(QBX_E_NOMEM, "autotune buffers");
    }
    int nr = G->m2l_nw_default;
    std::vector<int> cand = {nr, (nr + 1) / 2, 0};
    bool prof = G->profile, graph = G->graph_on;
    G->profile = false;
    G->graph_on = false;
    // passes over the candidates in turn (drift of clocks and caches hits
    // them alike); a sample is kEvals evaluations back to back and each
    // candidate keeps its fastest sample; the first pass warms up.  Another
    // candidate replaces the default only when it is kMargin faster: the
    // candidates differ by a few per cent of an evaluation at most, about
    // the spread of single samples.
    constexpr int kRounds = 9, kEvals = 4;
    constexpr double kMargin = 0.99;
    std::vector<double> best_of(cand.size(), 1e300);
    for (int rep = 0; rep < kRounds; ++rep)
        for (size_t ci = 0; ci < cand.size(); ++ci) {
            G->m2l_nw = cand[ci];
            bool ok = hipEventRecord(a, s) == hipSuccess;
            for (int k = 0; ok && k < kEvals; ++k)
                ok = eval_chunks(G, n_dens, dsig, nullptr, du, nullptr, s, G->ctx->lane) == QBX_OK;
            ok = ok && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
            float ms = 0.f;
            if (ok && rep > 0 && hipEventElapsedTime(&ms, a, b) == hipSuccess)
                best_of[ci] = std::min(best_of[ci], (double)ms);
        }
    int pick = nr;
    double best = best_of[0] * kMargin;
    for (size_t ci = 1; ci < cand.size(); ++ci)
        if (best_of[ci] < best) { best = best_of[ci]; pick = cand[ci]; }
    G->profile = prof;
    G->graph_on = graph;
    G->m2l_nw = pick;
    (void)hipStreamSynchronize(s);
    cleanup();
    if (choice_out) *choice_out = pick;
    return QBX_OK;
}

qbx_status qbx_geom_graph(qbx_geom G, int32_t enable)
{
    if (!G) return fail(QBX_E_INVAL, "null geometry");
    QBX_CTX_CALL(G->ctx);
    if (!G->ctx->gstream) return fail(QBX_E_UNSUPPORTED, "graph stream unavailable");
    G->graph_on = enable != 0;
    return QBX_OK;
}

}  // extern "C"

// ---- area queries and association on the device ---------------------------
namespace {

// Temporary device buffers of one call, freed when it returns.
struct DevTmp {
    std::vector<void *> ptrs;
    hipError_t err = hipSuccess;
    template <class T> T *alloc(size_t n)
    {
        void *q = nullptr;
        if (err == hipSuccess) err = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
        if (err != hipSuccess) return nullptr;
        ptrs.push_back(q);
        return static_cast<T *>(q);
    }
    ~DevTmp()
    {
        for (void *q : ptrs) (void)hipFree(q);
    }
};

AQTree aq_tree(const qbx_geom_s *G)
{
    AQTree t;
    t.bcx = G->g.bcx;
    t.bcy = G->g.bcy;
    t.blev = G->g.blev;
    t.leaf = G->g.leaf;
    t.child4 = G->g.child4;
    t.R0 = G->pl.R0;
    return t;
}

// Exclusive scan of n device counts into start[0..n] (device), on the host.
hipError_t scan_counts(const int32_t *cnt, int64_t n, int64_t *start, int64_t *total, hipStream_t s)
{
    std::vector<int32_t> h((size_t)n);
    std::vector<int64_t> st((size_t)n + 1, 0);
    hipError_t e = n ? hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s) : hipSuccess;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int64_t i = 0; i < n; ++i) st[i + 1] = st[i] + h[i];
    *total = st[n];
    e = hipMemcpyAsync(start, st.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

qbx_status aq_check(hipError_t e, const int *d_err, hipStream_t s, const char *what)
{
    int herr = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    if (herr) return fail(QBX_E_DEVICE, std::string(what) + ": traversal stack exceeded");
    return QBX_OK;
}

}  // namespace

extern "C" {

qbx_status qbx_geom_area_query(qbx_geom G, int64_t n, const double *qx, const double *qy,
                               const double *qr, int64_t *start, int32_t *leaves, int64_t *total_out)
{
    if (!G || n < 0 || !start || (n > 0 && (!qx || !qy || !qr))) return fail(QBX_E_INVAL, "area query: bad argument");
    QBX_CTX_CALL(G->ctx);
    hipError_t e = hipSetDevice(G->ctx->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    hipStream_t s = G->ctx->stream;
    AQTree t = aq_tree(G);
    DevTmp tmp;
    int32_t *cnt = tmp.alloc<int32_t>((size_t)n);
    int *err = tmp.alloc<int>(1);
    if (tmp.err != hipSuccess) return fail(QBX_E_NOMEM, "area query buffers");
    e = hipMemsetAsync(err, 0, sizeof(int), s);
    if (e == hipSuccess) e = launch_area_query(t, n, qx, qy, qr, cnt, nullptr, nullptr, err, s);
    qbx_status st = aq_check(e, err, s, "area query (count)");
    if (st != QBX_OK) return st;
    int64_t total = 0;
    e = scan_counts(cnt, n, start, &total, s);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("area query (scan): ") + hipGetErrorString(e));
    if (total_out) *total_out = total;
    if (!leaves) return QBX_OK;
    e = launch_area_query(t, n, qx, qy, qr, nullptr, start, leaves, err, s);
    return aq_check(e, err, s, "area query (fill)");
}

qbx_status qbx_geom_points_near(qbx_geom G, int32_t which, int64_t n, const double *qx, const double *qy,
                                const double *qr, int32_t *hit_out)
{
    if (!G || n < 0 || (which != 0 && which != 1) || (n > 0 && (!qx || !qy || !qr || !hit_out)))
        return fail(QBX_E_INVAL, "points_near: bad argument");
    QBX_CTX_CALL(G->ctx);
    hipError_t e = hipSetDevice(G->ctx->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    hipStream_t s = G->ctx->stream;
    DevTmp tmp;
    int *err = tmp.alloc<int>(1);
    if (tmp.err != hipSuccess) return fail(QBX_E_NOMEM, "points_near buffers");
    const DevGeom &g = G->g;
    e = hipMemsetAsync(err, 0, sizeof(int), s);
    if (e == hipSuccess)
        e = which == 0 ? launch_points_near(aq_tree(G), n, qx, qy, qr, g.src_begin, g.src_end, g.sx, g.sy, hit_out, err, s)
                       : launch_points_near(aq_tree(G), n, qx, qy, qr, g.ctr_begin, g.ctr_end, g.cx, g.cy, hit_out, err, s);
    return aq_check(e, err, s, "points_near");
}

qbx_status qbx_geom_associate(qbx_geom G, int64_t n_tgt, const double *tx, const double *ty,
                              int32_t *tgt_ctr_out, int64_t *n_fail_out)
{
    if (!G || n_tgt < 0 || (n_tgt > 0 && (!tx || !ty || !tgt_ctr_out))) return fail(QBX_E_INVAL, "associate: bad argument");
    QBX_CTX_CALL(G->ctx);
    hipError_t e = hipSetDevice(G->ctx->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    hipStream_t s = G->ctx->stream;
    const Plan &pl = G->pl;
    AQTree t = aq_tree(G);
    int64_t nkey = (int64_t)kAqKeysPerBox * pl.n_boxes();
    // radii in tree order
    std::vector<double> hcr((size_t)pl.nc), hsh((size_t)pl.ns);
    for (int64_t k = 0; k < pl.nc; ++k) hcr[k] = pl.cr[pl.ctr_order[k]];
    for (int64_t k = 0; k < pl.ns; ++k) hsh[k] = pl.sh[pl.src_order[k]];
    DevTmp tmp;
    double *dcr = tmp.alloc<double>(hcr.size()), *dsh = tmp.alloc<double>(hsh.size());
    int32_t *ccnt = tmp.alloc<int32_t>(nkey), *scnt = tmp.alloc<int32_t>(nkey);
    int64_t *cstart = tmp.alloc<int64_t>(nkey + 1), *sstart = tmp.alloc<int64_t>(nkey + 1);
    int *err = tmp.alloc<int>(1);
    unsigned long long *nfail = tmp.alloc<unsigned long long>(1);
    if (tmp.err != hipSuccess) return fail(QBX_E_NOMEM, "associate buffers");
    e = hipMemcpyAsync(dcr, hcr.data(), sizeof(double) * hcr.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dsh, hsh.data(), sizeof(double) * hsh.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(ccnt, 0, sizeof(int32_t) * nkey, s);
    if (e == hipSuccess) e = hipMemsetAsync(scnt, 0, sizeof(int32_t) * nkey, s);
    if (e == hipSuccess) e = hipMemsetAsync(err, 0, sizeof(int), s);
    if (e == hipSuccess) e = hipMemsetAsync(nfail, 0, sizeof(unsigned long long), s);
    // every centre enters the regions its eligibility square meets, every
    // source those its sh/4 square meets (squares a relative 1e-12 wider:
    // the final tests are exact)
    const double widen = 1.0 + 1e-12, ea = pl.opt.eps_assoc;
    if (e == hipSuccess)
        e = launch_region_lists(t, pl.nc, G->g.cx, G->g.cy, dcr, (1.0 + ea) * widen, ccnt, nullptr, nullptr,
                                nullptr, err, s);
    if (e == hipSuccess)
        e = launch_region_lists(t, pl.ns, G->g.sx, G->g.sy, dsh, 0.25 * widen, scnt, nullptr, nullptr, nullptr,
                                err, s);
    qbx_status st = aq_check(e, err, s, "associate (count)");
    if (st != QBX_OK) return st;
    int64_t ctot = 0, stot = 0;
    e = scan_counts(ccnt, nkey, cstart, &ctot, s);
    if (e == hipSuccess) e = scan_counts(scnt, nkey, sstart, &stot, s);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("associate (scan): ") + hipGetErrorString(e));
    int32_t *clist = tmp.alloc<int32_t>((size_t)ctot), *slist = tmp.alloc<int32_t>((size_t)stot);
    if (tmp.err != hipSuccess) return fail(QBX_E_NOMEM, "associate lists");
    // the count arrays serve again as fill cursors
    e = hipMemsetAsync(ccnt, 0, sizeof(int32_t) * nkey, s);
    if (e == hipSuccess) e = hipMemsetAsync(scnt, 0, sizeof(int32_t) * nkey, s);
    if (e == hipSuccess)
        e = launch_region_lists(t, pl.nc, G->g.cx, G->g.cy, dcr, (1.0 + ea) * widen, nullptr, cstart, ccnt,
                                clist, err, s);
    if (e == hipSuccess)
        e = launch_region_lists(t, pl.ns, G->g.sx, G->g.sy, dsh, 0.25 * widen, nullptr, sstart, scnt, slist,
                                err, s);
    AQAssoc a;
    a.cx = G->g.cx; a.cy = G->g.cy; a.cr = dcr; a.ctr_user = G->g.ctr_perm;
    a.sx = G->g.sx; a.sy = G->g.sy; a.sh = dsh;
    a.cstart = cstart; a.sstart = sstart; a.clist = clist; a.slist = slist;
    a.ea = ea;
    if (e == hipSuccess) e = launch_associate(t, a, n_tgt, tx, ty, tgt_ctr_out, nfail, s);
    st = aq_check(e, err, s, "associate");
    if (st != QBX_OK) return st;
    unsigned long long hf = 0;
    e = hipMemcpyAsync(&hf, nfail, sizeof(hf), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("associate: ") + hipGetErrorString(e));
    if (n_fail_out) *n_fail_out = (int64_t)hf;
    return QBX_OK;
}

}  // extern "C"

// ---- GMRES building blocks ---------------------------------------------------

qbx_status qbx_krylov_dot(qbx_ctx ctx, int64_t n, int32_t k, const void *V, int64_t ldv, const void *w, void *h)
{
    if (!ctx) return fail(QBX_E_INVAL, "null context");
    QBX_CTX_EXCLUSIVE(ctx);
    if (n < 0 || k < 0 || ldv < n) return fail(QBX_E_INVAL, "qbx_krylov_dot: need n >= 0, k >= 0, ldv >= n");
    if (k == 0) return QBX_OK;
    if (!h || (n > 0 && (!V || !w))) return fail(QBX_E_INVAL, "qbx_krylov_dot: null array");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(QBX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    size_t need = (size_t)k * std::max(krylov_dot_chunks(n), 1);
    if (need > ctx->kw_cap) {
        // the previous workspace may still be read by enqueued work
        if (ctx->kw) {
            CHK(hipStreamSynchronize(ctx->stream));
            CHK(hipFree(ctx->kw));
            ctx->kw = nullptr;
            ctx->kw_cap = 0;
        }
        size_t cap = std::max(need, ctx->kw_cap * 2);
        e = hipMalloc((void **)&ctx->kw, cap * sizeof(cd));
        if (e != hipSuccess) return fail(QBX_E_NOMEM, std::string("krylov workspace: ") + hipGetErrorString(e));
        ctx->kw_cap = cap;
    }
    CHK(launch_krylov_dot(n, k, static_cast<const cd *>(V), ldv, static_cast<const cd *>(w), ctx->kw,
                          static_cast<cd *>(h), ctx->stream));
    return QBX_OK;
}

qbx_status qbx_krylov_update(qbx_ctx ctx, int64_t n, int32_t k, const void *V, int64_t ldv, const void *h,
                             void *w)
{
    if (!ctx) return fail(QBX_E_INVAL, "null context");
    QBX_CTX_CALL(ctx);
    if (n < 0 || k < 0 || ldv < n) return fail(QBX_E_INVAL, "qbx_krylov_update: need n >= 0, k >= 0, ldv >= n");
    if (n == 0 || k == 0) return QBX_OK;
    if (!V || !h || !w) return fail(QBX_E_INVAL, "qbx_krylov_update: null array");
    CHK(hipSetDevice(ctx->device));
    CHK(launch_krylov_update(n, k, static_cast<const cd *>(V), ldv, static_cast<const cd *>(h),
                             static_cast<cd *>(w), ctx->stream));
    return QBX_OK;
}

qbx_status qbx_krylov_normalize(qbx_ctx ctx, int64_t n, const void *w, const void *nrm2, void *v)
{
    if (!ctx) return fail(QBX_E_INVAL, "null context");
    QBX_CTX_CALL(ctx);
    if (n < 0) return fail(QBX_E_INVAL, "qbx_krylov_normalize: n < 0");
    if (n == 0) return QBX_OK;
    if (!w || !nrm2 || !v) return fail(QBX_E_INVAL, "qbx_krylov_normalize: null array");
    CHK(hipSetDevice(ctx->device));
    CHK(launch_krylov_normalize(n, static_cast<const cd *>(w), static_cast<const cd *>(nrm2),
                                static_cast<cd *>(v), ctx->stream));
    return QBX_OK;
}

qbx_status qbx_upsample(qbx_ctx ctx, int64_t n_panels, int32_t q, int32_t qs, const double *L, double alpha_re,
                        double alpha_im, const void *x, void *ys, void *yd)
{
    if (!ctx) return fail(QBX_E_INVAL, "null context");
    QBX_CTX_CALL(ctx);
    if (n_panels < 0 || q < 1 || qs < 1) return fail(QBX_E_INVAL, "qbx_upsample: need n_panels >= 0, q, qs >= 1");
    if (n_panels == 0) return QBX_OK;
    if (!L || !x || (!ys && !yd)) return fail(QBX_E_INVAL, "qbx_upsample: null array");
    CHK(hipSetDevice(ctx->device));
    CHK(launch_upsample(n_panels, q, qs, L, mk(alpha_re, alpha_im), static_cast<const cd *>(x),
                        static_cast<cd *>(ys), static_cast<cd *>(yd), ctx->stream));
    return QBX_OK;
}
