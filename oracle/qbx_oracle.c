/*
 * Direct (O(N_s * N_c)) Global QBX for the 2D Helmholtz single- and
 * double-layer potentials, in plain FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product library never does.  It shares
 * no code with the GPU path: its Bessel functions come from the C library
 * (j0, j1, y0, y1, jn) and the textbook three-term recurrence.
 *
 * What it computes (Rachh, Kloeckner, O'Neil, "Fast algorithms for
 * Quadrature by Expansion I"):
 *
 *   G(x, x') = (i/4) H0(omega |x - x'|)                  (Sec. 1, Green's fn)
 *   charges   qS_j = (i/4) w_j sigmaS_j,  qD_j = (i/4) w_j sigmaD_j
 *   O_l(z)  = H_l(omega |z|) e^{i l arg z}       (outgoing wave, Sec. 7.1)
 *
 *   alpha_{l}(c) = sum_j [ qS_j O_l(s_j - c)
 *                  + qD_j (omega/2) (nu_j O_{l-1}(s_j - c)
 *                                   - conj(nu_j) O_{l+1}(s_j - c)) ]
 *        for |l| <= p, over ALL sources (Sec. 3.2, oversampled coefficient
 *        sum; Sec. 2.1, eq. (graf-coefficient)).  nu_j = n_x + i n_y.  The
 *        double-layer term is the normal derivative (with respect to the
 *        source) of the single-layer one, using
 *        d/dz O_l = (omega/2) O_{l-1}, d/dzbar O_l = -(omega/2) O_{l+1},
 *        n . grad = nu d/dz + conj(nu) d/dzbar (the paper only says that
 *        "similar expansions exist" for other layer potentials).
 *
 *   u(t) = sum_{|l|<=p} alpha_l(c) J_l(omega |t-c|) e^{-i l arg(t-c)}
 *        (Sec. 2.1, eq. (phiapprox)) for a target t associated with centre c.
 *
 *   u(t) = sum_j qS_j H0(omega r) + qD_j omega H1(omega r) ((t-s_j).n_j)/r
 *        (Sec. 3.2, eq. (gauss-layerpot), plus its double-layer analogue)
 *        for targets served by the smooth rule.
 *
 *   Association (Sec. 6.1, algorithm "Associate volume/surface targets"),
 *   by brute force: the centres whose disks, enlarged by (1 + eps_assoc),
 *   contain t are eligible; the nearest wins, ties to the lowest index.
 *   With no eligible centre, t fails if it lies in Gamma_near, i.e. within
 *   h_k/4 of a node of panel k (Sec. 6.1 distance approximation), and is
 *   served by the smooth rule otherwise.
 *
 * Complex arrays are interleaved (re, im) doubles, i.e. numpy complex128.
 */
#define _DEFAULT_SOURCE 1  /* j0, j1, y0, y1, jn are XSI extensions of math.h */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef double complex cplx;

/* H_n^{(1)}(x), n = 0..nmax, x > 0: J_0, J_1, Y_0, Y_1 from the C library,
 * then H_{n+1} = (2n/x) H_n - H_{n-1}. */
static void hankel_seq(double x, int nmax, cplx *h)
{
    h[0] = j0(x) + I * y0(x);
    if (nmax >= 1) h[1] = j1(x) + I * y1(x);
    for (int n = 1; n < nmax; ++n) h[n + 1] = (2.0 * n / x) * h[n] - h[n - 1];
}

int oracle_hankel1_seq(double x, int nmax, double *out)
{
    if (!(x > 0.0) || nmax < 0) return -1;
    cplx *h = (cplx *)malloc(sizeof(cplx) * (size_t)(nmax + 2));
    if (!h) return -2;
    hankel_seq(x, nmax, h);
    for (int n = 0; n <= nmax; ++n) { out[2 * n] = creal(h[n]); out[2 * n + 1] = cimag(h[n]); }
    free(h);
    return 0;
}

/* J_n(x), n = 0..nmax, straight from the C library's jn. */
int oracle_besselj_seq(double x, int nmax, double *out)
{
    if (nmax < 0) return -1;
    for (int n = 0; n <= nmax; ++n) out[n] = jn(n, x);
    return 0;
}

/* O_l(z) for l = -L..L written to o[l + L], from |z| and arg z. */
static void outgoing_seq(double omega, double dx, double dy, int L, cplx *hbuf, cplx *o)
{
    double r = sqrt(dx * dx + dy * dy);
    double th = atan2(dy, dx);
    hankel_seq(omega * r, L, hbuf);
    for (int l = -L; l <= L; ++l) {
        int n = l < 0 ? -l : l;
        double sgn = (l < 0 && (n & 1)) ? -1.0 : 1.0;   /* H_{-n} = (-1)^n H_n */
        o[l + L] = sgn * hbuf[n] * cexp(I * (double)l * th);
    }
}

/*
 * alpha[d][l+p][i], d < nd, |l| <= p, i < nc.  sigS / sigD may be NULL.
 * Returns 0, or -1 when a source coincides with a centre.
 */
int oracle_qbx_coefficients(double omega, int p, int64_t ns,
                            const double *sx, const double *sy, const double *w,
                            const double *nx, const double *ny,
                            int nd, const double *sigS, const double *sigD,
                            int64_t nc, const double *cx, const double *cy,
                            double *alpha_out, int nthreads)
{
    const int L = p + 1;
    const int64_t ncoef = 2 * (int64_t)p + 1;
    int bad = 0;
    cplx *alpha = (cplx *)alpha_out;
    const cplx *qs_in = (const cplx *)sigS;
    const cplx *qd_in = (const cplx *)sigD;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(| : bad)
    for (int64_t i = 0; i < nc; ++i) {
        cplx *hbuf = (cplx *)malloc(sizeof(cplx) * (size_t)(L + 2));
        cplx *o = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * L + 1));
        cplx *acc = (cplx *)calloc((size_t)(nd * ncoef), sizeof(cplx));
        for (int64_t j = 0; j < ns; ++j) {
            double dx = sx[j] - cx[i], dy = sy[j] - cy[i];
            if (dx == 0.0 && dy == 0.0) { bad = 1; continue; }
            outgoing_seq(omega, dx, dy, L, hbuf, o);
            cplx nu = nx[j] + I * ny[j];
            for (int d = 0; d < nd; ++d) {
                cplx qs = qs_in ? 0.25 * I * w[j] * qs_in[(int64_t)d * ns + j] : 0.0;
                cplx qd = qd_in ? 0.25 * I * w[j] * qd_in[(int64_t)d * ns + j] : 0.0;
                for (int l = -p; l <= p; ++l) {
                    cplx term = qs * o[l + L]
                              + qd * (0.5 * omega) * (nu * o[l - 1 + L] - conj(nu) * o[l + 1 + L]);
                    acc[d * ncoef + (l + p)] += term;
                }
            }
        }
        for (int d = 0; d < nd; ++d)
            for (int64_t l = 0; l < ncoef; ++l)
                alpha[((int64_t)d * ncoef + l) * nc + i] = acc[d * ncoef + l];
        free(hbuf); free(o); free(acc);
    }
    return bad ? -1 : 0;
}

/* u[d][m] = sum_l alpha[d][l+p][ctr[m]] J_l(omega rho) e^{-i l theta} for
 * targets with ctr[m] >= 0; other entries of u are left untouched. */
int oracle_qbx_eval(double omega, int p, int64_t nc, const double *cx, const double *cy,
                    int nd, const double *alpha_in, int64_t nt, const double *tx,
                    const double *ty, const int32_t *ctr, double *u_out, int nthreads)
{
    const int64_t ncoef = 2 * (int64_t)p + 1;
    const cplx *alpha = (const cplx *)alpha_in;
    cplx *u = (cplx *)u_out;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t m = 0; m < nt; ++m) {
        int64_t i = ctr[m];
        if (i < 0 || i >= nc) continue;
        double dx = tx[m] - cx[i], dy = ty[m] - cy[i];
        double rho = sqrt(dx * dx + dy * dy);
        double th = atan2(dy, dx);
        for (int d = 0; d < nd; ++d) {
            cplx s = 0.0;
            for (int l = -p; l <= p; ++l) {
                int n = l < 0 ? -l : l;
                double jl = jn(n, omega * rho);
                if (l < 0 && (n & 1)) jl = -jl;             /* J_{-n} = (-1)^n J_n */
                s += alpha[((int64_t)d * ncoef + (l + p)) * nc + i] * jl
                     * cexp(-I * (double)l * th);
            }
            u[(int64_t)d * nt + m] = s;
        }
    }
    return 0;
}

/* Smooth (unmodified Gauss) rule at targets with ctr[m] == -1 (all targets
 * when ctr is NULL).  Returns -1 if a target coincides with a source. */
int oracle_smooth(double omega, int64_t ns, const double *sx, const double *sy,
                  const double *w, const double *nx, const double *ny, int nd,
                  const double *sigS, const double *sigD, int64_t nt,
                  const double *tx, const double *ty, const int32_t *ctr,
                  double *u_out, int nthreads)
{
    const cplx *qs_in = (const cplx *)sigS;
    const cplx *qd_in = (const cplx *)sigD;
    cplx *u = (cplx *)u_out;
    int bad = 0;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(| : bad)
    for (int64_t m = 0; m < nt; ++m) {
        if (ctr && ctr[m] != -1) continue;
        cplx *acc = (cplx *)calloc((size_t)nd, sizeof(cplx));
        for (int64_t j = 0; j < ns; ++j) {
            double dx = tx[m] - sx[j], dy = ty[m] - sy[j];
            double r = sqrt(dx * dx + dy * dy);
            if (r == 0.0) { bad = 1; continue; }
            cplx h0 = j0(omega * r) + I * y0(omega * r);
            cplx h1 = j1(omega * r) + I * y1(omega * r);
            double cosang = (dx * nx[j] + dy * ny[j]) / r;
            for (int d = 0; d < nd; ++d) {
                cplx qs = qs_in ? 0.25 * I * w[j] * qs_in[(int64_t)d * ns + j] : 0.0;
                cplx qd = qd_in ? 0.25 * I * w[j] * qd_in[(int64_t)d * ns + j] : 0.0;
                acc[d] += qs * h0 + qd * omega * h1 * cosang;
            }
        }
        for (int d = 0; d < nd; ++d) u[(int64_t)d * nt + m] = acc[d];
        free(acc);
    }
    return bad ? -1 : 0;
}

/*
 * Brute-force association.  ctr_out[m] = nearest eligible centre, -1 for the
 * smooth rule, -2 for a failed association.  Distances are compared squared:
 * centre i is eligible iff |t-c_i|^2 <= (r_i (1 + eps_assoc))^2; t is in
 * Gamma_near iff |t-s_j|^2 <= (h_j/4)^2 for some node j.
 * Returns the number of failed targets.
 */
int64_t oracle_associate(int64_t nt, const double *tx, const double *ty,
                         int64_t nc, const double *cx, const double *cy, const double *cr,
                         int64_t ns, const double *sx, const double *sy, const double *sh,
                         double eps_assoc, int32_t *ctr_out, int nthreads)
{
    int64_t nfail = 0;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(+ : nfail)
    for (int64_t m = 0; m < nt; ++m) {
        int64_t best = -1;
        double bestd = 0.0;
        for (int64_t i = 0; i < nc; ++i) {
            double dx = tx[m] - cx[i], dy = ty[m] - cy[i];
            double d2 = dx * dx + dy * dy;
            double lim = cr[i] * (1.0 + eps_assoc);
            if (d2 <= lim * lim && (best < 0 || d2 < bestd)) { best = i; bestd = d2; }
        }
        if (best >= 0) { ctr_out[m] = (int32_t)best; continue; }
        int near = 0;
        for (int64_t j = 0; j < ns && !near; ++j) {
            double dx = tx[m] - sx[j], dy = ty[m] - sy[j];
            double q = 0.25 * sh[j];
            if (dx * dx + dy * dy <= q * q) near = 1;
        }
        ctr_out[m] = near ? -2 : -1;
        nfail += near;
    }
    return nfail;
}
