// Host planning for FMM-accelerated Global QBX.  See planner.hpp.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <unordered_map>
#include <unordered_set>

namespace qbx {

namespace {

inline uint64_t spread_bits(uint32_t v)
{
    uint64_t x = v & 0x3fffffffu;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// Morton key: x in even bits, y in odd bits; child quadrant q = xbit | ybit << 1.
inline uint64_t morton(uint32_t ix, uint32_t iy) { return spread_bits(ix) | (spread_bits(iy) << 1); }

// Integer coordinate of a point at the finest level: floor(u 2^30),
// u = (x + R0) / (2 R0).
inline uint32_t fine_coord(double x, double R0)
{
    double u = (x + R0) / (2.0 * R0);
    return (uint32_t)(u * 1073741824.0);
}

bool all_finite(const double *a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

}  // namespace

int v_offset_id(int dx, int dy)
{
    // enumerate (dy, dx) row-major over [-3,3]^2 skipping the inner 3x3
    int id = 0;
    for (int y = -3; y <= 3; ++y)
        for (int x = -3; x <= 3; ++x) {
            if (std::abs(x) <= 1 && std::abs(y) <= 1) continue;
            if (x == dx && y == dy) return id;
            ++id;
        }
    return -1;
}

void v_offset_from_id(int id, int *dx, int *dy)
{
    int k = 0;
    for (int y = -3; y <= 3; ++y)
        for (int x = -3; x <= 3; ++x) {
            if (std::abs(x) <= 1 && std::abs(y) <= 1) continue;
            if (k == id) { *dx = x; *dy = y; return; }
            ++k;
        }
    *dx = *dy = 0;
}

double Plan::box_radius(int level) const { return std::ldexp(R0, -level); }

void Plan::box_center(int b, double *x, double *y) const
{
    double side = std::ldexp(2.0 * R0, -lev[b]);
    *x = -R0 + (bix[b] + 0.5) * side;
    *y = -R0 + (biy[b] + 0.5) * side;
}

int default_p_add(int p, double eps)
{
    // Sec. 7.1 determines p_add empirically; its table (p = 2, 4, 6, 8 ->
    // 5, 5, 15, 20) is reproduced within a few orders by the same procedure
    // run on star curves against direct QBX, which also shows a dependence
    // on eps.  Least-squares fit of the smallest increment that kept the
    // relative l2 error below eps/4 (p = 4..20, eps = 1e-4..1e-12), plus 4.
    // Compared over every target of 256 curves of 512-16k nodes whose panels
    // meet omega h <= 5 (Sec. 5, Condition 4), of the 32768-node star and of
    // the 606k-node set, the increment keeps the relative l2 error below eps
    // and the largest error below 10 eps on all of them; the fit alone (4
    // less) fails 14 of the 256 curves at eps = 1e-10.
    double d = -std::log10(eps);
    double v = 2.358 * p + 1.4875 * d - 9.626 + 4.0;
    return std::max(5, (int)std::ceil(v));
}

int fmm_order(double omega, double R, double eps)
{
    // Smallest P with |H_n(3 omega R) J_n(sqrt(2) omega R)| <= eps for all n > P
    // (Sec. 7.1).  Long double keeps H_n finite far past the decay point.
    long double x = 3.0L * omega * R, y = std::sqrt(2.0L) * omega * R;
    int N = (int)x + 120;
    long double hm = j0l(x), hmi = y0l(x);        // H_{n-1}
    long double h = j1l(x), hi = y1l(x);          // H_n
    int last = 0;
    for (int n = 0; n <= N; ++n) {
        long double hr, him;
        if (n == 0) { hr = hm; him = hmi; }
        else if (n == 1) { hr = h; him = hi; }
        else {
            long double f = 2.0L * (n - 1) / x;
            long double nr = f * h - hm, ni = f * hi - hmi;
            hm = h; hmi = hi; h = nr; hi = ni;
            hr = h; him = hi;
        }
        long double jv = jnl(n, y);
        long double t = std::sqrt(hr * hr + him * him) * std::fabs(jv);
        if (!(t <= eps)) last = n;  // also catches overflow to inf
    }
    return std::max(last, 1);
}

std::vector<double> level_scales(double omega, double R, int P)
{
    std::vector<double> W(P + 1);
    double lsig = std::log(omega * R / std::sqrt(2.0));
    for (int k = 0; k <= P; ++k) {
        double lw = std::min(0.0, k * lsig - std::lgamma(k + 1.0));
        lw = std::max(lw, -600.0);   // any positive scale is valid; keep it normal
        W[k] = std::exp(lw);
    }
    return W;
}

namespace {

std::vector<long double> level_scales_ld(double omega, double R, int P)
{
    std::vector<long double> W(P + 1);
    long double lsig = std::log((long double)omega * R / std::sqrt(2.0L));
    for (int k = 0; k <= P; ++k) {
        long double lw = std::min(0.0L, k * lsig - std::lgamma(k + 1.0L));
        lw = std::max(lw, -600.0L);
        W[k] = std::exp(lw);
    }
    return W;
}

// J_n(x) e^{i n theta} for n = -N..N (index n + N), long double.
std::vector<std::complex<long double>> incoming_ld(double omega, double zx, double zy, int N)
{
    long double r = std::sqrt((long double)zx * zx + (long double)zy * zy);
    long double th = std::atan2((long double)zy, (long double)zx);
    std::vector<std::complex<long double>> out(2 * N + 1);
    for (int n = 0; n <= N; ++n) {
        long double j = jnl(n, omega * r);
        std::complex<long double> ph(std::cos(n * th), std::sin(n * th));
        out[N + n] = j * ph;
        long double jm = (n & 1) ? -j : j;
        out[N - n] = jm * std::conj(ph);
    }
    return out;
}

// H_n(omega|z|) e^{i n theta} for n = -N..N (index n + N), long double.
std::vector<std::complex<long double>> outgoing_ld(double omega, double zx, double zy, int N)
{
    long double r = std::sqrt((long double)zx * zx + (long double)zy * zy);
    long double th = std::atan2((long double)zy, (long double)zx);
    long double x = omega * r;
    std::vector<std::complex<long double>> H(N + 2);
    H[0] = {j0l(x), y0l(x)};
    H[1] = {j1l(x), y1l(x)};
    for (int n = 1; n <= N; ++n) H[n + 1] = (2.0L * n / x) * H[n] - H[n - 1];
    std::vector<std::complex<long double>> out(2 * N + 1);
    for (int n = 0; n <= N; ++n) {
        std::complex<long double> ph(std::cos(n * th), std::sin(n * th));
        out[N + n] = H[n] * ph;
        std::complex<long double> hm = (n & 1) ? -H[n] : H[n];
        out[N - n] = hm * std::conj(ph);
    }
    return out;
}

}  // namespace

std::vector<std::complex<double>> m2m_matrix(const Plan &pl, int l, int q)
{
    // a_n(parent) = sum_k a_k(child) I_{k-n}(m_p - m_c)        (Stage 2)
    int Pp = pl.P[l], Pc = pl.P[l + 1];
    double Rc = pl.box_radius(l + 1);
    double dx = (q & 1) ? Rc : -Rc, dy = (q & 2) ? Rc : -Rc;   // m_c - m_p
    auto Wp = level_scales_ld(pl.omega, pl.box_radius(l), Pp);
    auto Wc = level_scales_ld(pl.omega, Rc, Pc);
    int N = Pp + Pc;
    auto I = incoming_ld(pl.omega, -dx, -dy, N);
    int np = 2 * Pp + 1, nc = 2 * Pc + 1;
    std::vector<std::complex<double>> T((size_t)np * nc);
    for (int j = -Pp; j <= Pp; ++j)
        for (int k = -Pc; k <= Pc; ++k) {
            std::complex<long double> v = I[k - j + N] * (Wc[std::abs(k)] / Wp[std::abs(j)]);
            T[(size_t)(j + Pp) * nc + (k + Pc)] = std::complex<double>((double)v.real(), (double)v.imag());
        }
    return T;
}

std::vector<std::complex<double>> l2l_matrix(const Plan &pl, int l, int q)
{
    // g'_j = sum_k g_k I_{j-k}(m_p - m_c)                        (Stage 7)
    int Pp = pl.P[l], Pc = pl.P[l + 1];
    double Rc = pl.box_radius(l + 1);
    double dx = (q & 1) ? Rc : -Rc, dy = (q & 2) ? Rc : -Rc;
    auto Wp = level_scales_ld(pl.omega, pl.box_radius(l), Pp);
    auto Wc = level_scales_ld(pl.omega, Rc, Pc);
    int N = Pp + Pc;
    auto I = incoming_ld(pl.omega, -dx, -dy, N);
    int np = 2 * Pp + 1, nc = 2 * Pc + 1;
    std::vector<std::complex<double>> T((size_t)nc * np);
    for (int j = -Pc; j <= Pc; ++j)
        for (int k = -Pp; k <= Pp; ++k) {
            std::complex<long double> v = I[j - k + N] * (Wc[std::abs(j)] / Wp[std::abs(k)]);
            T[(size_t)(j + Pc) * np + (k + Pp)] = std::complex<double>((double)v.real(), (double)v.imag());
        }
    return T;
}

std::vector<std::complex<double>> m2l_matrix(const Plan &pl, int l, int dx, int dy)
{
    // g_j = (-1)^j sum_k a_k O_{k+j}(c - m)                      (Stage 4)
    int P = pl.P[l];
    double side = 2.0 * pl.box_radius(l);
    auto W = level_scales_ld(pl.omega, pl.box_radius(l), P);
    int N = 2 * P;
    auto O = outgoing_ld(pl.omega, -dx * side, -dy * side, N);
    int n = 2 * P + 1;
    std::vector<std::complex<double>> T((size_t)n * n);
    for (int j = -P; j <= P; ++j) {
        long double sg = (j & 1) ? -1.0L : 1.0L;
        for (int k = -P; k <= P; ++k) {
            std::complex<long double> v = O[k + j + N] * (sg * W[std::abs(j)] * W[std::abs(k)]);
            T[(size_t)(j + P) * n + (k + P)] = std::complex<double>((double)v.real(), (double)v.imag());
        }
    }
    return T;
}

namespace {

bool touch(const Plan &pl, int a, int b)
{
    int L = std::max(pl.lev[a], pl.lev[b]);
    int sa = L - pl.lev[a], sb = L - pl.lev[b];
    int64_t ax0 = (int64_t)pl.bix[a] << sa, ax1 = (int64_t)(pl.bix[a] + 1) << sa;
    int64_t ay0 = (int64_t)pl.biy[a] << sa, ay1 = (int64_t)(pl.biy[a] + 1) << sa;
    int64_t bx0 = (int64_t)pl.bix[b] << sb, bx1 = (int64_t)(pl.bix[b] + 1) << sb;
    int64_t by0 = (int64_t)pl.biy[b] << sb, by1 = (int64_t)(pl.biy[b] + 1) << sb;
    return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
}

void to_csr(const std::vector<std::vector<int32_t>> &L, std::vector<int32_t> &start,
            std::vector<int32_t> &idx)
{
    start.assign(L.size() + 1, 0);
    for (size_t b = 0; b < L.size(); ++b) start[b + 1] = start[b] + (int32_t)L[b].size();
    idx.resize(start.back());
    for (size_t b = 0; b < L.size(); ++b) std::copy(L[b].begin(), L[b].end(), idx.begin() + start[b]);
}

// Location code of box (l, ix, iy): a leading one above its 2l Morton bits,
// unique across levels.
inline uint64_t loc_code(int l, uint32_t ix, uint32_t iy) { return (1ull << (2 * l)) | morton(ix, iy); }

// Source and centre ranges of box (l, ix, iy) in the Morton-sorted keys.
struct Ranges {
    int s0, s1, c0, c1;
    int count() const { return s1 - s0 + c1 - c0; }
};

Ranges box_ranges(const std::vector<uint64_t> &sk, const std::vector<uint64_t> &ck, int l, uint32_t ix,
                  uint32_t iy)
{
    int shift = 2 * (kMaxLevel - l);
    uint64_t pref = morton(ix, iy);
    uint64_t k0 = pref << shift, k1 = (pref + 1) << shift;
    Ranges r;
    r.s0 = (int)(std::lower_bound(sk.begin(), sk.end(), k0) - sk.begin());
    r.s1 = (int)(std::lower_bound(sk.begin(), sk.end(), k1) - sk.begin());
    r.c0 = (int)(std::lower_bound(ck.begin(), ck.end(), k0) - ck.begin());
    r.c1 = (int)(std::lower_bound(ck.begin(), ck.end(), k1) - ck.begin());
    return r;
}

// Level restriction (2:1 balance; the paper's experiments use level-
// restricted trees, Sec. 8): no leaf may touch a box two or more levels
// finer than itself.  Returns the location codes of the leaves of the
// adaptive tree (lev, bix, biy, leaf as built) that must be split for that,
// found in one sweep from the finest level up.  A box d at level m >= 2 can
// only be touched by a too-coarse leaf through one of the level-(m-2) cells
// around its grandparent; the box covering such a cell, if it is a leaf at
// level <= m-2, is split, and so are its children covering the cell, down
// to level m-1.  Splits only create boxes coarser than m, so the sweep
// visits them later.
std::unordered_set<uint64_t> balance_splits(const Plan &pl, const std::vector<uint64_t> &sk,
                                            const std::vector<uint64_t> &ck)
{
    std::unordered_map<uint64_t, bool> split;   // code -> has children
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> at(kMaxLevel + 1);
    int nb = pl.n_boxes();
    for (int b = 0; b < nb; ++b) {
        split[loc_code(pl.lev[b], pl.bix[b], pl.biy[b])] = !pl.leaf[b];
        at[pl.lev[b]].push_back({(uint32_t)pl.bix[b], (uint32_t)pl.biy[b]});
    }
    std::unordered_set<uint64_t> forced;
    auto force = [&](int l, uint32_t ix, uint32_t iy) {
        uint64_t code = loc_code(l, ix, iy);
        split[code] = true;
        forced.insert(code);
        for (int q = 0; q < 4; ++q) {
            uint32_t jx = 2 * ix + (q & 1), jy = 2 * iy + (q >> 1);
            if (box_ranges(sk, ck, l + 1, jx, jy).count() == 0) continue;
            split.emplace(loc_code(l + 1, jx, jy), false);
            at[l + 1].push_back({jx, jy});
        }
    };
    for (int m = kMaxLevel; m >= 2; --m) {
        for (size_t i = 0; i < at[m].size(); ++i) {
            uint32_t dx = at[m][i].first, dy = at[m][i].second;
            int64_t gx = dx >> 2, gy = dy >> 2, n = 1ll << (m - 2);
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int64_t cx = gx + ox, cy = gy + oy;
                    if ((ox == 0 && oy == 0) || cx < 0 || cy < 0 || cx >= n || cy >= n) continue;
                    // closed squares in level-m units: cell [4cx, 4cx+4], d [dx, dx+1]
                    if (4 * cx > (int64_t)dx + 1 || (int64_t)dx > 4 * cx + 4) continue;
                    if (4 * cy > (int64_t)dy + 1 || (int64_t)dy > 4 * cy + 4) continue;
                    // deepest existing box holding the cell
                    int k = m - 2;
                    while (k > 0 && !split.count(loc_code(k, (uint32_t)(cx >> (m - 2 - k)), (uint32_t)(cy >> (m - 2 - k))))) --k;
                    for (; k <= m - 2; ++k) {
                        uint32_t ax = (uint32_t)(cx >> (m - 2 - k)), ay = (uint32_t)(cy >> (m - 2 - k));
                        auto it = split.find(loc_code(k, ax, ay));
                        if (it == split.end()) break;       // empty quadrant: nothing there
                        if (!it->second) force(k, ax, ay);
                    }
                }
        }
    }
    return forced;
}

void build_tree(Plan &pl, const std::unordered_set<uint64_t> *forced, std::vector<uint64_t> *sk_out,
                std::vector<uint64_t> *ck_out)
{
    double m = 0.0;
    for (int64_t i = 0; i < pl.ns; ++i) m = std::max(m, std::max(std::fabs(pl.sx[i]), std::fabs(pl.sy[i])));
    for (int64_t i = 0; i < pl.nc; ++i) m = std::max(m, std::max(std::fabs(pl.cx[i]), std::fabs(pl.cy[i])));
    if (m == 0.0) m = 1.0;
    pl.R0 = m * (1.0 + 1e-12);

    std::vector<uint64_t> skey(pl.ns), ckey(pl.nc);
    for (int64_t i = 0; i < pl.ns; ++i) skey[i] = morton(fine_coord(pl.sx[i], pl.R0), fine_coord(pl.sy[i], pl.R0));
    for (int64_t i = 0; i < pl.nc; ++i) ckey[i] = morton(fine_coord(pl.cx[i], pl.R0), fine_coord(pl.cy[i], pl.R0));
    pl.src_order.resize(pl.ns);
    pl.ctr_order.resize(pl.nc);
    std::iota(pl.src_order.begin(), pl.src_order.end(), 0);
    std::iota(pl.ctr_order.begin(), pl.ctr_order.end(), 0);
    std::stable_sort(pl.src_order.begin(), pl.src_order.end(),
                     [&](int64_t a, int64_t b) { return skey[a] < skey[b]; });
    std::stable_sort(pl.ctr_order.begin(), pl.ctr_order.end(),
                     [&](int64_t a, int64_t b) { return ckey[a] < ckey[b]; });
    std::vector<uint64_t> sk(pl.ns), ck(pl.nc);
    for (int64_t i = 0; i < pl.ns; ++i) sk[i] = skey[pl.src_order[i]];
    for (int64_t i = 0; i < pl.nc; ++i) ck[i] = ckey[pl.ctr_order[i]];

    auto push = [&](int l, int ix, int iy, int par, int s0, int s1, int c0, int c1) {
        pl.lev.push_back(l); pl.bix.push_back(ix); pl.biy.push_back(iy); pl.parent.push_back(par);
        pl.src_begin.push_back(s0); pl.src_end.push_back(s1);
        pl.ctr_begin.push_back(c0); pl.ctr_end.push_back(c1);
        pl.child_begin.push_back(-1); pl.child_count.push_back(0);
    };
    push(0, 0, 0, -1, 0, (int)pl.ns, 0, (int)pl.nc);
    pl.level_start = {0};
    int lo = 0, hi = 1, l = 0;
    while (lo < hi) {
        pl.level_start.push_back(hi);
        for (int b = lo; b < hi; ++b) {
            int cnt = (pl.src_end[b] - pl.src_begin[b]) + (pl.ctr_end[b] - pl.ctr_begin[b]);
            bool must = forced && forced->count(loc_code(l, pl.bix[b], pl.biy[b]));
            if ((cnt <= pl.opt.leaf_max && !must) || l >= kMaxLevel) continue;
            int shift = 2 * (kMaxLevel - (l + 1));
            uint64_t pref = morton((uint32_t)pl.bix[b], (uint32_t)pl.biy[b]);
            for (int q = 0; q < 4; ++q) {
                uint64_t cp = (pref << 2) | (uint64_t)q;
                uint64_t k0 = cp << shift, k1 = (cp + 1) << shift;
                int s0 = (int)(std::lower_bound(sk.begin() + pl.src_begin[b], sk.begin() + pl.src_end[b], k0) - sk.begin());
                int s1 = (int)(std::lower_bound(sk.begin() + pl.src_begin[b], sk.begin() + pl.src_end[b], k1) - sk.begin());
                int c0 = (int)(std::lower_bound(ck.begin() + pl.ctr_begin[b], ck.begin() + pl.ctr_end[b], k0) - ck.begin());
                int c1 = (int)(std::lower_bound(ck.begin() + pl.ctr_begin[b], ck.begin() + pl.ctr_end[b], k1) - ck.begin());
                if (s1 - s0 + c1 - c0 == 0) continue;
                if (pl.child_begin[b] < 0) pl.child_begin[b] = (int)pl.lev.size();
                pl.child_count[b]++;
                push(l + 1, 2 * pl.bix[b] + (q & 1), 2 * pl.biy[b] + (q >> 1), b, s0, s1, c0, c1);
            }
        }
        lo = hi;
        hi = (int)pl.lev.size();
        ++l;
    }
    // level_start has one entry per level plus a final sentinel
    pl.nlev = (int)pl.level_start.size() - 1;
    pl.level_start.back() = (int)pl.lev.size();
    while (pl.nlev > 0 && pl.level_start[pl.nlev - 1] == pl.level_start[pl.nlev]) {
        pl.level_start.pop_back();
        pl.nlev--;
    }
    int nb = pl.n_boxes();
    pl.leaf.resize(nb);
    for (int b = 0; b < nb; ++b) pl.leaf[b] = pl.child_count[b] == 0;
    if (sk_out) sk_out->swap(sk);
    if (ck_out) ck_out->swap(ck);
}

void clear_tree(Plan &pl)
{
    for (auto *v : {&pl.lev, &pl.bix, &pl.biy, &pl.parent, &pl.leaf, &pl.child_begin, &pl.child_count,
                    &pl.src_begin, &pl.src_end, &pl.ctr_begin, &pl.ctr_end, &pl.level_start})
        v->clear();
}

void build_tree(Plan &pl)
{
    std::vector<uint64_t> sk, ck;
    build_tree(pl, nullptr, &sk, &ck);
    if (!pl.opt.level_restrict) return;
    std::unordered_set<uint64_t> forced = balance_splits(pl, sk, ck);
    if (forced.empty()) return;
    clear_tree(pl);
    build_tree(pl, &forced, nullptr, nullptr);
}

void build_lists(Plan &pl)
{
    int nb = pl.n_boxes();
    pl.colleagues.assign((size_t)nb * 9, -1);
    pl.colleagues[0] = 0;
    for (int b = 1; b < nb; ++b) {
        int par = pl.parent[b], k = 0;
        for (int t = 0; t < 9; ++t) {
            int c = pl.colleagues[(size_t)par * 9 + t];
            if (c < 0) continue;
            for (int d = pl.child_begin[c]; d >= 0 && d < pl.child_begin[c] + pl.child_count[c]; ++d)
                if (std::abs(pl.bix[d] - pl.bix[b]) <= 1 && std::abs(pl.biy[d] - pl.biy[b]) <= 1)
                    pl.colleagues[(size_t)b * 9 + k++] = d;
        }
        std::sort(pl.colleagues.begin() + (size_t)b * 9, pl.colleagues.begin() + (size_t)b * 9 + k);
    }

    std::vector<std::vector<int32_t>> U(nb), V(nb), W(nb), X(nb), Voff(nb);
    for (int b = 1; b < nb; ++b) {
        int par = pl.parent[b];
        std::vector<std::pair<int, int>> vv;
        for (int t = 0; t < 9; ++t) {
            int c = pl.colleagues[(size_t)par * 9 + t];
            if (c < 0) continue;
            for (int d = pl.child_begin[c]; d >= 0 && d < pl.child_begin[c] + pl.child_count[c]; ++d) {
                int dx = pl.bix[d] - pl.bix[b], dy = pl.biy[d] - pl.biy[b];
                if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
                vv.push_back({d, v_offset_id(dx, dy)});
            }
        }
        std::sort(vv.begin(), vv.end());
        for (auto &e : vv) { V[b].push_back(e.first); Voff[b].push_back(e.second); }
    }
    for (int b = 0; b < nb; ++b) {
        if (!pl.leaf[b]) continue;
        for (int t = 0; t < 9; ++t) {
            int c = pl.colleagues[(size_t)b * 9 + t];
            if (c < 0 || c == b) continue;
            if (pl.leaf[c]) { U[b].push_back(c); continue; }
            std::vector<int> stack;
            for (int d = pl.child_begin[c]; d < pl.child_begin[c] + pl.child_count[c]; ++d) stack.push_back(d);
            while (!stack.empty()) {
                int d = stack.back();
                stack.pop_back();
                if (touch(pl, b, d)) {
                    if (pl.leaf[d]) U[b].push_back(d);
                    else
                        for (int e = pl.child_begin[d]; e < pl.child_begin[d] + pl.child_count[d]; ++e) stack.push_back(e);
                } else {
                    W[b].push_back(d);
                }
            }
        }
    }
    // U is symmetric between leaves: a finer leaf adjacent to b sees b too.
    for (int b = 0; b < nb; ++b) {
        if (!pl.leaf[b]) continue;
        size_t n0 = U[b].size();
        for (size_t i = 0; i < n0; ++i) {
            int c = U[b][i];
            if (pl.lev[c] > pl.lev[b]) U[c].push_back(b);
        }
    }
    for (int b = 0; b < nb; ++b) {
        if (pl.leaf[b]) U[b].push_back(b);
        std::sort(U[b].begin(), U[b].end());
        std::sort(W[b].begin(), W[b].end());
        for (int d : W[b]) X[d].push_back(b);
    }
    for (int b = 0; b < nb; ++b) std::sort(X[b].begin(), X[b].end());
    to_csr(U, pl.U_start, pl.U_idx);
    to_csr(V, pl.V_start, pl.V_idx);
    std::vector<int32_t> dummy;
    to_csr(Voff, dummy, pl.V_off);
    to_csr(W, pl.W_start, pl.W_idx);
    to_csr(X, pl.X_start, pl.X_idx);
}

// Uniform-grid lookup used by the association (exactly the brute-force rule,
// restricted to the cells that can hold a candidate).
struct Grid {
    double x0 = 0, y0 = 0, cell = 1;
    std::vector<uint64_t> key;
    std::vector<int64_t> idx;
    static uint64_t pack(int64_t i, int64_t j) { return ((uint64_t)(i + (1ll << 31)) << 32) | (uint64_t)(j + (1ll << 31)); }
    void build(const double *x, const double *y, int64_t n, double c)
    {
        cell = c > 0 ? c : 1.0;
        x0 = y0 = 0;
        std::vector<std::pair<uint64_t, int64_t>> kv(n);
        for (int64_t i = 0; i < n; ++i) kv[i] = {pack(cx(x[i]), cx(y[i])), i};
        std::sort(kv.begin(), kv.end());
        key.resize(n); idx.resize(n);
        for (int64_t i = 0; i < n; ++i) { key[i] = kv[i].first; idx[i] = kv[i].second; }
    }
    int64_t cx(double v) const { return (int64_t)std::floor(v / cell); }
    template <class F> void visit(double px, double py, F f) const
    {
        int64_t i0 = cx(px), j0 = cx(py);
        for (int64_t i = i0 - 1; i <= i0 + 1; ++i)
            for (int64_t j = j0 - 1; j <= j0 + 1; ++j) {
                uint64_t k = pack(i, j);
                auto it = std::lower_bound(key.begin(), key.end(), k);
                for (; it != key.end() && *it == k; ++it) f(idx[it - key.begin()]);
            }
    }
};

Error associate(Plan &pl, const int32_t *tgt_ctr)
{
    pl.tgt_ctr.assign(pl.nt, -1);
    bool any_free = false;
    for (int64_t m = 0; m < pl.nt; ++m) {
        int32_t v = tgt_ctr ? tgt_ctr[m] : -1;
        if (v < -1 || v >= pl.nc) return {QBX_E_INVAL, "tgt_ctr entry out of range"};
        pl.tgt_ctr[m] = v;
        any_free |= (v == -1);
    }
    if (!any_free) return {QBX_OK, ""};
    double ea = pl.opt.eps_assoc;
    double rmax = 0.0, hmax = 0.0;
    for (int64_t i = 0; i < pl.nc; ++i) rmax = std::max(rmax, pl.cr[i] * (1.0 + ea));
    for (int64_t j = 0; j < pl.ns; ++j) hmax = std::max(hmax, 0.25 * pl.sh[j]);
    Grid gc, gs;
    gc.build(pl.cx.data(), pl.cy.data(), pl.nc, rmax * (1.0 + 1e-9));
    gs.build(pl.sx.data(), pl.sy.data(), pl.ns, hmax * (1.0 + 1e-9));
    int64_t nfail = 0;
    for (int64_t m = 0; m < pl.nt; ++m) {
        if (pl.tgt_ctr[m] != -1) continue;
        double tx = pl.tx[m], ty = pl.ty[m];
        int64_t best = -1;
        double bestd = 0.0;
        gc.visit(tx, ty, [&](int64_t i) {
            double dx = tx - pl.cx[i], dy = ty - pl.cy[i];
            double d2 = dx * dx + dy * dy;
            double lim = pl.cr[i] * (1.0 + ea);
            if (d2 <= lim * lim && (best < 0 || d2 < bestd || (d2 == bestd && i < best))) { best = i; bestd = d2; }
        });
        if (best >= 0) { pl.tgt_ctr[m] = (int32_t)best; continue; }
        bool near = false;
        if (pl.ns > 0)
            gs.visit(tx, ty, [&](int64_t j) {
                double dx = tx - pl.sx[j], dy = ty - pl.sy[j];
                double q = 0.25 * pl.sh[j];
                if (dx * dx + dy * dy <= q * q) near = true;
            });
        if (near) ++nfail;
    }
    if (nfail) return {QBX_E_ASSOC, std::to_string(nfail) + " target(s) in Gamma_near have no eligible QBX centre"};
    return {QBX_OK, ""};
}

}  // namespace

Error build_plan(Plan &pl, double omega, double eps, const qbx_options &opt, int64_t ns,
                 const double *sx, const double *sy, const double *w, const double *nx,
                 const double *ny, const double *sh, int64_t nc, const double *cx,
                 const double *cy, const double *cr, int64_t nt, const double *tx,
                 const double *ty, const int32_t *tgt_ctr)
{
    if (ns < 0 || nc < 0 || nt < 0) return {QBX_E_INVAL, "negative count"};
    if (ns > INT32_MAX / 2 || nc > INT32_MAX / 2 || nt > INT32_MAX / 2) return {QBX_E_INVAL, "count too large"};
    if (!(omega > 0) || !std::isfinite(omega)) return {QBX_E_INVAL, "omega must be a positive real number"};
    if (!(eps >= 1e-15 && eps <= 1e-2)) return {QBX_E_INVAL, "eps must lie in [1e-15, 1e-2]"};
    if (opt.p < 0 || opt.p > kMaxP) return {QBX_E_INVAL, "p must lie in 0..40"};
    if (opt.leaf_max < 1) return {QBX_E_INVAL, "leaf_max must be >= 1"};
    if (opt.far_fp32 != 0 && opt.far_fp32 != 1) return {QBX_E_INVAL, "far_fp32 must be 0 or 1"};
    if (opt.far_fp32 && eps < 1e-6) return {QBX_E_INVAL, "far_fp32 needs eps >= 1e-6"};
    if (!(opt.eps_assoc >= 0 && opt.eps_assoc < 1)) return {QBX_E_INVAL, "eps_assoc must lie in [0, 1)"};
    if (opt.p_add < -1 || opt.p_add > 200) return {QBX_E_INVAL, "p_add must be -1 or in 0..200"};
    if (opt.w_direct < -1) return {QBX_E_INVAL, "w_direct must be -1, 0 or a positive source count"};
    if (opt.level_restrict != 0 && opt.level_restrict != 1) return {QBX_E_INVAL, "level_restrict must be 0 or 1"};
    if (opt.keep_x_rows != 0 && opt.keep_x_rows != 1) return {QBX_E_INVAL, "keep_x_rows must be 0 or 1"};
    if (ns && (!sx || !sy || !w || !nx || !ny || !sh)) return {QBX_E_INVAL, "null source array"};
    if (nc && (!cx || !cy || !cr)) return {QBX_E_INVAL, "null centre array"};
    if (nt && (!tx || !ty)) return {QBX_E_INVAL, "null target array"};
    for (const double *a : {sx, sy, w, nx, ny, sh})
        if (ns && !all_finite(a, ns)) return {QBX_E_INVAL, "non-finite source data"};
    for (const double *a : {cx, cy, cr})
        if (nc && !all_finite(a, nc)) return {QBX_E_INVAL, "non-finite centre data"};
    for (const double *a : {tx, ty})
        if (nt && !all_finite(a, nt)) return {QBX_E_INVAL, "non-finite target data"};
    for (int64_t j = 0; j < ns; ++j) {
        if (w[j] < 0 || sh[j] < 0) return {QBX_E_INVAL, "negative weight or panel length"};
        double nn = nx[j] * nx[j] + ny[j] * ny[j];
        if (std::fabs(nn - 1.0) > 2e-6) return {QBX_E_INVAL, "normals must be unit vectors"};
    }
    for (int64_t i = 0; i < nc; ++i)
        if (!(cr[i] > 0)) return {QBX_E_INVAL, "expansion radii must be positive"};

    pl.omega = omega; pl.eps = eps; pl.opt = opt;
    pl.ns = ns; pl.nc = nc; pl.nt = nt;
    pl.sx.assign(sx, sx + ns); pl.sy.assign(sy, sy + ns); pl.w.assign(w, w + ns);
    pl.nx.assign(nx, nx + ns); pl.ny.assign(ny, ny + ns); pl.sh.assign(sh, sh + ns);
    pl.cx.assign(cx, cx + nc); pl.cy.assign(cy, cy + nc); pl.cr.assign(cr, cr + nc);
    pl.tx.assign(tx, tx + nt); pl.ty.assign(ty, ty + nt);

    Error e = associate(pl, tgt_ctr);
    if (e.status != QBX_OK) return e;

    build_tree(pl);
    build_lists(pl);

    pl.p = opt.p;
    pl.p_add = opt.p_add >= 0 ? opt.p_add : default_p_add(opt.p, eps);
    pl.P.assign(pl.nlev, 0);
    pl.pfmm.assign(pl.nlev, 0);
    for (int l = 0; l < pl.nlev; ++l) {
        pl.pfmm[l] = fmm_order(omega, pl.box_radius(l), eps);
        // the M2QBXL kernel's 8-wide l window needs P_l >= p + 8 (more terms
        // only add accuracy)
        pl.P[l] = std::max(pl.pfmm[l] + pl.p_add, pl.p + 8);
        if (pl.P[l] > kMaxOrder && l >= 2)
            return {QBX_E_UNSUPPORTED, "FMM order at level " + std::to_string(l) + " exceeds 1024 (omega * box size too large)"};
        pl.P[l] = std::min(pl.P[l], kMaxOrder);
    }
    return {QBX_OK, ""};
}

}  // namespace qbx
