/*
 * COLATUS plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library.
 * Only the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with
 * the HIP library, and the HIP library never calls it.
 *
 * Everything here is deliberately slow and literal: scalar loops in FP64,
 * IEEE sqrt and divide, Neumaier-compensated sums in index order, adaptive
 * Simpson quadrature in a.  The only parallelism is an OpenMP loop over
 * independent target particles, which does not change any sum's order.
 *
 * Paper: Stalder et al., "A new gravitational N-body simulation algorithm
 * for investigation of cosmological chaotic advection" (arXiv:1208.3444).
 *
 * Readings of the paper taken here:
 *  - Eq. (1) prints the pair term as m_j (x_k - x_j); that is repulsive.  The
 *    attractive form m_j (x_j - x_k) is used.
 *  - Eqs. (6)-(9): the canonical momentum is p = a^2 v (per unit mass), the
 *    drift is dx/dt = p/a^2 and the kick is dp/dt = g/a, where
 *    g = G sum_j m_j (x_j - x_k) r^-3 is the comoving pair sum without the
 *    a^-3 factor.  This is Eq. (1) rewritten for p; the printed Eq. (8)
 *    (p^2 in the drift, phi' instead of its gradient in the kick) is read as
 *    a typesetting slip.
 *  - The background term (a^2 a_ddot |x|^2 / 2) of Eq. (6) is off by
 *    default: the force is Eq. (1) exactly, in an open (non-periodic) box.
 *    On request it is the removal of the mean matter density's pull about
 *    a centre, b (x - c) with b = Om_M H0^2 / 2 (see oracle_background_add).
 *  - The step is kick(half) - drift - kick(half) built from the drift and
 *    kick operators of Eq. (9); steps are uniform in ln a and the half-step
 *    point is the midpoint in ln a.
 *  - Softening is Plummer, in comoving units, as written in Eq. (1).
 *  - Static limit: H0 == 0 keeps a fixed at a_begin; then the "a_end"
 *    argument of the run is the total elapsed time and dt = a_end/n_steps.
 *  - Eq. (10)'s deformation term is a fixed attractor of strength S = C psi
 *    at x_psi, softened with the same eps and added to g with the attractive
 *    sign of Eq. (1) (see oracle_attractor_add).
 *
 * Parity pins for every function live in the tests (closed forms,
 * invariants, brute force, finite differences).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Compensated summation (Neumaier 1974).                                   */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;

static void ksum_add(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v))
        k->c += (k->s - t) + v;
    else
        k->c += (v - t) + k->s;
    k->s = t;
}

static double ksum_value(const ksum *k) { return k->s + k->c; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing the oracle on one core). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Friedmann equation, Eq. (2):                                             */
/*   H(a) = H0 sqrt(Om_R a^-4 + Om_M a^-3 + Om_K a^-2 + Om_L).              */
/* No renormalisation of the density parameters.  Returns NaN if H^2 < 0.   */
/* ------------------------------------------------------------------------ */
typedef struct { double H0, OmR, OmM, OmK, OmL; } cosmo;

double oracle_hubble(double a, double H0, double OmR, double OmM, double OmK,
                     double OmL)
{
    double e2 = OmR / (a * a * a * a) + OmM / (a * a * a) + OmK / (a * a) + OmL;
    if (e2 < 0.0)
        return NAN;
    return H0 * sqrt(e2);
}

/* Integrand 1/(a^k H(a)) of the three time integrals:
 *   k = 1: cosmic time       dt       = da / (a H)
 *   k = 2: kick factor       dt / a   = da / (a^2 H)   (Eq. (9), K)
 *   k = 3: drift factor      dt / a^2 = da / (a^3 H)   (Eq. (9), D)      */
static double integrand(const cosmo *c, int k, double a)
{
    double h = oracle_hubble(a, c->H0, c->OmR, c->OmM, c->OmK, c->OmL);
    double ak = a;
    for (int i = 1; i < k; ++i)
        ak *= a;
    return 1.0 / (ak * h);
}

static double simpson_rec(const cosmo *c, int k, double lo, double hi,
                          double flo, double fmid, double fhi, double whole,
                          double tol, int depth)
{
    double mid = 0.5 * (lo + hi);
    double lm = 0.5 * (lo + mid), rm = 0.5 * (mid + hi);
    double flm = integrand(c, k, lm), frm = integrand(c, k, rm);
    double left = (mid - lo) / 6.0 * (flo + 4.0 * flm + fmid);
    double right = (hi - mid) / 6.0 * (fmid + 4.0 * frm + fhi);
    double delta = left + right - whole;
    if (depth <= 0 || fabs(delta) <= 15.0 * tol)
        return left + right + delta / 15.0;
    return simpson_rec(c, k, lo, mid, flo, flm, fmid, left, 0.5 * tol, depth - 1) +
           simpson_rec(c, k, mid, hi, fmid, frm, fhi, right, 0.5 * tol, depth - 1);
}

/* Adaptive Simpson in a of 1/(a^k H) from a1 to a2, to ~1e-14 relative.   */
static double time_integral(const cosmo *c, int k, double a1, double a2)
{
    if (a1 == a2)
        return 0.0;
    double sign = 1.0;
    if (a2 < a1) {
        double t = a1;
        a1 = a2;
        a2 = t;
        sign = -1.0;
    }
    /* Split into 64 equal panels first so the tolerance is relative to a
     * sensible scale even for wide ranges; each panel is then refined.    */
    const int panels = 64;
    double h = (a2 - a1) / panels;
    double rough = 0.0;
    for (int i = 0; i < panels; ++i) {
        double lo = a1 + i * h, hi = (i == panels - 1) ? a2 : a1 + (i + 1) * h;
        double flo = integrand(c, k, lo), fhi = integrand(c, k, hi);
        double fm = integrand(c, k, 0.5 * (lo + hi));
        rough += (hi - lo) / 6.0 * (flo + 4.0 * fm + fhi);
    }
    double tol = 1e-15 * fabs(rough) / panels;
    ksum total = {0.0, 0.0};
    for (int i = 0; i < panels; ++i) {
        double lo = a1 + i * h, hi = (i == panels - 1) ? a2 : a1 + (i + 1) * h;
        double flo = integrand(c, k, lo), fhi = integrand(c, k, hi);
        double fm = integrand(c, k, 0.5 * (lo + hi));
        double whole = (hi - lo) / 6.0 * (flo + 4.0 * fm + fhi);
        ksum_add(&total, simpson_rec(c, k, lo, hi, flo, fm, fhi, whole, tol, 48));
    }
    return sign * ksum_value(&total);
}

/* Public: kind 1 = cosmic time, 2 = kick factor, 3 = drift factor.        */
double oracle_time_integral(int kind, double a1, double a2, double H0,
                            double OmR, double OmM, double OmK, double OmL)
{
    cosmo c = {H0, OmR, OmM, OmK, OmL};
    if (kind < 1 || kind > 3)
        return NAN;
    return time_integral(&c, kind, a1, a2);
}

/* ------------------------------------------------------------------------ */
/* Pair sums of Eq. (1).                                                    */
/* ------------------------------------------------------------------------ */

/* acc_k = a^-3 G sum_{j != k} m_j (x_j - x_k) / (|x_j - x_k|^2 + eps^2)^{3/2}
 * x is SoA: x[0..N) = x-components, x[N..2N) = y, x[2N..3N) = z.
 * The self pair j == k is excluded (the "k != j" of Eq. (1)).             */
void oracle_forces(const double *x, const double *m, int64_t N, double eps,
                   double G, double a, double *acc)
{
    const double *px = x, *py = x + N, *pz = x + 2 * N;
    const double eps2 = eps * eps;
    const double scale = G / (a * a * a);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < N; ++k) {
        ksum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
        for (int64_t j = 0; j < N; ++j) {
            if (j == k)
                continue;
            double dx = px[j] - px[k];
            double dy = py[j] - py[k];
            double dz = pz[j] - pz[k];
            double s = dx * dx + dy * dy + dz * dz + eps2;
            double rinv = 1.0 / sqrt(s);
            double r3 = rinv * rinv * rinv;
            ksum_add(&sx, m[j] * dx * r3);
            ksum_add(&sy, m[j] * dy * r3);
            ksum_add(&sz, m[j] * dz * r3);
        }
        acc[k] = scale * ksum_value(&sx);
        acc[N + k] = scale * ksum_value(&sy);
        acc[2 * N + k] = scale * ksum_value(&sz);
    }
}

/* Same sum for a subset of targets (index list), used to check a large
 * force evaluation on sampled particles.  acc is [3][n_targets].          */
void oracle_forces_targets(const double *x, const double *m, int64_t N,
                           const int64_t *targets, int64_t n_targets,
                           double eps, double G, double a, double *acc)
{
    const double *px = x, *py = x + N, *pz = x + 2 * N;
    const double eps2 = eps * eps;
    const double scale = G / (a * a * a);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n_targets; ++t) {
        int64_t k = targets[t];
        ksum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
        for (int64_t j = 0; j < N; ++j) {
            if (j == k)
                continue;
            double dx = px[j] - px[k];
            double dy = py[j] - py[k];
            double dz = pz[j] - pz[k];
            double s = dx * dx + dy * dy + dz * dz + eps2;
            double rinv = 1.0 / sqrt(s);
            double r3 = rinv * rinv * rinv;
            ksum_add(&sx, m[j] * dx * r3);
            ksum_add(&sy, m[j] * dy * r3);
            ksum_add(&sz, m[j] * dz * r3);
        }
        acc[t] = scale * ksum_value(&sx);
        acc[n_targets + t] = scale * ksum_value(&sy);
        acc[2 * n_targets + t] = scale * ksum_value(&sz);
    }
}

/* Softened comoving potential whose negative gradient is the Eq. (1) sum:
 *   phi_k = -G sum_{j != k} m_j / sqrt(|x_j - x_k|^2 + eps^2).            */
void oracle_potential(const double *x, const double *m, int64_t N, double eps,
                      double G, double *phi)
{
    const double *px = x, *py = x + N, *pz = x + 2 * N;
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < N; ++k) {
        ksum s = {0, 0};
        for (int64_t j = 0; j < N; ++j) {
            if (j == k)
                continue;
            double dx = px[j] - px[k];
            double dy = py[j] - py[k];
            double dz = pz[j] - pz[k];
            double r2 = dx * dx + dy * dy + dz * dz + eps2;
            ksum_add(&s, m[j] / sqrt(r2));
        }
        phi[k] = -G * ksum_value(&s);
    }
}

/* Vector-Jacobian product of the comoving pair sum g(x) (Eq. (1) without
 * the a^-3 factor).  With d = x_j - x_k, s = |d|^2 + eps^2 and
 *   M(d) = s^{-3/2} I - 3 s^{-5/2} d d^T,
 * the derivative is dg_k/dx_j = G m_j M(d) for j != k and
 * dg_k/dx_k = -G sum_j m_j M(d), so
 *   (J^T lam)_k = G sum_{j != k} M(d_kj) (m_k lam_j - m_j lam_k).         */
void oracle_force_vjp(const double *x, const double *m, int64_t N, double eps,
                      double G, const double *lam, double *out)
{
    const double *px = x, *py = x + N, *pz = x + 2 * N;
    const double *lx = lam, *ly = lam + N, *lz = lam + 2 * N;
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < N; ++k) {
        ksum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
        for (int64_t j = 0; j < N; ++j) {
            if (j == k)
                continue;
            double dx = px[j] - px[k];
            double dy = py[j] - py[k];
            double dz = pz[j] - pz[k];
            double s = dx * dx + dy * dy + dz * dz + eps2;
            double rinv = 1.0 / sqrt(s);
            double r3 = rinv * rinv * rinv;
            double r5 = r3 * rinv * rinv;
            double ux = m[k] * lx[j] - m[j] * lx[k];
            double uy = m[k] * ly[j] - m[j] * ly[k];
            double uz = m[k] * lz[j] - m[j] * lz[k];
            double du = dx * ux + dy * uy + dz * uz;
            ksum_add(&sx, r3 * ux - 3.0 * r5 * du * dx);
            ksum_add(&sy, r3 * uy - 3.0 * r5 * du * dy);
            ksum_add(&sz, r3 * uz - 3.0 * r5 * du * dz);
        }
        out[k] = G * ksum_value(&sx);
        out[N + k] = G * ksum_value(&sy);
        out[2 * N + k] = G * ksum_value(&sz);
    }
}

/* ------------------------------------------------------------------------ */
/* Periodic boundaries (Section II: the motion equations are solved in a   */
/* periodic box), by Ewald summation.                                       */
/* ------------------------------------------------------------------------ */
/* The periodic comoving field in a box of side L, with the mean density
 * removed (the images of every particle fill space; the uniform background
 * of the same mean density is subtracted, so the field is that of the
 * density contrast), is for particle k
 *   g_k = G sum_{j != k} m_j E(x_j - x_k),
 * E(d) = sum_{n in Z^3} (d + nL) / |d + nL|^3                (summed with
 *        the background, i.e. Ewald's split):
 *      = sum_n (d + nL) C(alpha |d + nL|) / |d + nL|^3
 *        + (4 pi / L^3) sum_{q != 0} (q / q^2) exp(-q^2 / (4 alpha^2)) sin(q . d)
 * with C(u) = erfc(u) + (2u / sqrt(pi)) exp(-u^2), q = 2 pi n / L over the
 * integer vectors n != 0, for any splitting parameter alpha > 0.  The
 * particle's own images pull it nowhere (they cancel in pairs), so j == k
 * adds nothing.  Softening: the nearest image d* of each pair (minimum
 * image) takes the Plummer law of Eq. (1) instead of the Newtonian one, i.e.
 *   + d* [(|d*|^2 + eps^2)^{-3/2} - |d*|^{-3}]   (0 for d* = 0).
 * The comoving potential (its negative gradient times m_k is m_k g_k):
 *   phi_k = -G [ sum_{j != k} m_j Psi(x_j - x_k) + m_k Psi_self ],
 *   Psi(d) = sum_n erfc(alpha r_n) / r_n + [(|d*|^2 + eps^2)^{-1/2} - 1/|d*|]
 *            + (4 pi / L^3) sum_q exp(-q^2 / 4 alpha^2) / q^2 cos(q . d)
 *            - pi / (alpha^2 L^3),
 *   Psi_self = sum_{n != 0} erfc(alpha |n| L) / (|n| L) + (4 pi / L^3) sum_q
 *            exp(-q^2 / 4 alpha^2) / q^2 - pi / (alpha^2 L^3) - 2 alpha / sqrt(pi)
 * (the interaction with its own images and with the background; a
 * constant: for one particle in a unit box Psi_self is the simple cubic
 * lattice's Madelung constant).  For two coincident particles (d* = 0) the
 * nearest-image potential is the limit 1/eps - 2 alpha / sqrt(pi).
 * Real space: images n with |n_i| <= n_img around the nearest one; reciprocal
 * space: |n| <= n_kmax.  Each term's definition above; the reciprocal sums
 * are written with the structure factor S(q) = sum_j m_j exp(i q . x_j), so
 * that sum_j m_j sin(q . (x_j - x_k)) = Im(exp(-i q . x_k) S(q)) and
 * sum_j m_j cos(q . (x_j - x_k)) = Re(exp(-i q . x_k) S(q)) (j == k included:
 * sin 0 = 0 for the force, cos 0 = 1 is the self part of the potential).
 * targets: NULL (all particles, out [3][N]) or an index list (out
 * [3][n_targets]); phi: NULL or [n_targets].  acc = g / a^3.              */
static const double kPi = 3.14159265358979323846;

static double ewald_c(double u)
{
    return erfc(u) + 2.0 / sqrt(kPi) * u * exp(-u * u);
}

void oracle_forces_periodic(const double *x, const double *m, int64_t N, double eps,
                            double G, double a, double L, double alpha, int n_img,
                            int n_kmax, const int64_t *targets, int64_t n_targets,
                            double *acc, double *phi)
{
    const double *px = x, *py = x + N, *pz = x + 2 * N;
    const double eps2 = eps * eps;
    const double scale = G / (a * a * a);
    const double vol = L * L * L;
    const int64_t nt = targets ? n_targets : N;
    /* reciprocal vectors and their structure factors */
    int64_t nq = 0;
    for (int i = -n_kmax; i <= n_kmax; ++i)
        for (int j = -n_kmax; j <= n_kmax; ++j)
            for (int l = -n_kmax; l <= n_kmax; ++l)
                if ((i || j || l) && i * i + j * j + l * l <= n_kmax * n_kmax)
                    ++nq;
    double *qv = (double *)malloc((size_t)(nq > 0 ? nq : 1) * 6 * sizeof(double));
    int64_t c = 0;
    for (int i = -n_kmax; i <= n_kmax; ++i)
        for (int j = -n_kmax; j <= n_kmax; ++j)
            for (int l = -n_kmax; l <= n_kmax; ++l)
                if ((i || j || l) && i * i + j * j + l * l <= n_kmax * n_kmax) {
                    double *q = qv + 6 * c++;
                    q[0] = 2.0 * kPi * i / L;
                    q[1] = 2.0 * kPi * j / L;
                    q[2] = 2.0 * kPi * l / L;
                    const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
                    /* weight (4 pi / L^3) exp(-q^2 / 4 alpha^2) / q^2 */
                    q[3] = 4.0 * kPi / vol * exp(-q2 / (4.0 * alpha * alpha)) / q2;
                }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nq; ++t) {
        double *q = qv + 6 * t;
        ksum sr = {0, 0}, si = {0, 0};
        for (int64_t j = 0; j < N; ++j) {
            const double ph = q[0] * px[j] + q[1] * py[j] + q[2] * pz[j];
            ksum_add(&sr, m[j] * cos(ph));
            ksum_add(&si, m[j] * sin(ph));
        }
        q[4] = ksum_value(&sr);
        q[5] = ksum_value(&si);
    }
    ksum mt = {0, 0};
    for (int64_t j = 0; j < N; ++j)
        ksum_add(&mt, m[j]);
    const double M = ksum_value(&mt);
    /* self part of the real-space potential (constant) */
    ksum ss = {0, 0};
    for (int i = -n_img; i <= n_img; ++i)
        for (int j = -n_img; j <= n_img; ++j)
            for (int l = -n_img; l <= n_img; ++l)
                if (i || j || l) {
                    const double r = L * sqrt((double)(i * i + j * j + l * l));
                    ksum_add(&ss, erfc(alpha * r) / r);
                }
    const double psi_self_real = ksum_value(&ss) - 2.0 * alpha / sqrt(kPi);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t k = targets ? targets[t] : t;
        ksum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, fp = {0, 0};
        for (int64_t j = 0; j < N; ++j) {
            if (j == k)
                continue;
            double d[3] = {px[j] - px[k], py[j] - py[k], pz[j] - pz[k]};
            for (int c3 = 0; c3 < 3; ++c3)
                d[c3] -= L * nearbyint(d[c3] / L);  /* nearest image d* */
            const double rs2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            for (int i = -n_img; i <= n_img; ++i)
                for (int jj = -n_img; jj <= n_img; ++jj)
                    for (int l = -n_img; l <= n_img; ++l) {
                        const double e[3] = {d[0] + i * L, d[1] + jj * L, d[2] + l * L};
                        const double r2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                        if (r2 == 0.0)
                            continue; /* coincident pair: handled below */
                        const double r = sqrt(r2);
                        const double w = m[j] * ewald_c(alpha * r) / (r2 * r);
                        ksum_add(&fx, w * e[0]);
                        ksum_add(&fy, w * e[1]);
                        ksum_add(&fz, w * e[2]);
                        ksum_add(&fp, m[j] * erfc(alpha * r) / r);
                    }
            /* softening of the nearest image */
            if (rs2 > 0.0) {
                const double rs = sqrt(rs2);
                const double sp = 1.0 / sqrt(rs2 + eps2);
                const double w = m[j] * (sp * sp * sp - 1.0 / (rs2 * rs));
                ksum_add(&fx, w * d[0]);
                ksum_add(&fy, w * d[1]);
                ksum_add(&fz, w * d[2]);
                ksum_add(&fp, m[j] * (sp - 1.0 / rs));
            } else {
                ksum_add(&fp, m[j] * (1.0 / eps - 2.0 * alpha / sqrt(kPi)));
            }
        }
        ksum_add(&fp, m[k] * psi_self_real);
        for (int64_t u = 0; u < nq; ++u) {
            const double *q = qv + 6 * u;
            const double ph = q[0] * px[k] + q[1] * py[k] + q[2] * pz[k];
            const double cs = cos(ph), sn = sin(ph);
            /* Im(exp(-i q.x_k) S) and Re(exp(-i q.x_k) S) */
            const double im = cs * q[5] - sn * q[4];
            const double re = cs * q[4] + sn * q[5];
            ksum_add(&fx, q[3] * q[0] * im);
            ksum_add(&fy, q[3] * q[1] * im);
            ksum_add(&fz, q[3] * q[2] * im);
            ksum_add(&fp, q[3] * re);
        }
        ksum_add(&fp, -kPi * M / (alpha * alpha * vol));
        acc[t] = scale * ksum_value(&fx);
        acc[nt + t] = scale * ksum_value(&fy);
        acc[2 * nt + t] = scale * ksum_value(&fz);
        if (phi)
            phi[t] = -G * ksum_value(&fp);
    }
    free(qv);
}

/* ------------------------------------------------------------------------ */
/* Deformation attractor of Eq. (10).                                       */
/* ------------------------------------------------------------------------ */
/* Eq. (10) adds to the gradient of Eq. (1) the term
 *   -C psi (x_k - x_psi) / (|x_k - x_psi|^2 + eps^2)^{3/2},
 * the pull of a fixed point at x_psi (the paper notes it acts like a mass
 * particle at a fixed position).  C and psi enter only as their product, the
 * strength S = C psi (units of G m).  With the attractive reading of Eq. (1)
 * the comoving field added to g is
 *   f_k = S (x_psi - x_k) / (|x_psi - x_k|^2 + eps^2)^{3/2},
 * its potential phi_k = -S / sqrt(|x_psi - x_k|^2 + eps^2) (an external
 * field: the energy is sum m phi, not half of it), and its derivative
 * df_k/dx_k = -S M(d), d = x_psi - x_k.  att_x == NULL: no attractor.
 * Adds f into g and (phi != NULL) phi_ext into phi.                       */
void oracle_attractor_add(const double *x, int64_t N, double eps, double S,
                          const double *att_x, double *g, double *phi)
{
    if (!att_x)
        return;
    const double eps2 = eps * eps;
    for (int64_t k = 0; k < N; ++k) {
        double dx = att_x[0] - x[k];
        double dy = att_x[1] - x[N + k];
        double dz = att_x[2] - x[2 * N + k];
        double s = dx * dx + dy * dy + dz * dz + eps2;
        double r = sqrt(s);
        double r3 = 1.0 / (s * r);
        if (g) {
            g[k] += S * dx * r3;
            g[N + k] += S * dy * r3;
            g[2 * N + k] += S * dz * r3;
        }
        if (phi)
            phi[k] += -S / r;
    }
}

/* M(d) lam with M(d) = s^{-3/2} I - 3 s^{-5/2} d d^T, s = |d|^2 + eps^2,
 * d = x_psi - x_k; also returns lam . d s^{-3/2} (= lam . f_k / S).        */
static void attractor_m(const double *x, int64_t N, int64_t k, double eps2,
                        const double *att_x, const double *lam, double out[3],
                        double *lam_f)
{
    double dx = att_x[0] - x[k];
    double dy = att_x[1] - x[N + k];
    double dz = att_x[2] - x[2 * N + k];
    double s = dx * dx + dy * dy + dz * dz + eps2;
    double rinv = 1.0 / sqrt(s);
    double r3 = rinv * rinv * rinv;
    double r5 = r3 * rinv * rinv;
    double lx = lam[k], ly = lam[N + k], lz = lam[2 * N + k];
    double dl = dx * lx + dy * ly + dz * lz;
    out[0] = r3 * lx - 3.0 * r5 * dl * dx;
    out[1] = r3 * ly - 3.0 * r5 * dl * dy;
    out[2] = r3 * lz - 3.0 * r5 * dl * dz;
    *lam_f = dl * r3;
}

/* out += (d f / d x)^T lam = -S M(d_k) lam_k for every particle.          */
static void attractor_vjp_add(const double *x, int64_t N, double eps, double S,
                              const double *att_x, const double *lam, double *out)
{
    if (!att_x)
        return;
    for (int64_t k = 0; k < N; ++k) {
        double mv[3], lf;
        attractor_m(x, N, k, eps * eps, att_x, lam, mv, &lf);
        out[k] += -S * mv[0];
        out[N + k] += -S * mv[1];
        out[2 * N + k] += -S * mv[2];
    }
}

/* Parameter derivatives of lam . f:  grad[0] += c sum_k lam_k . f_k / S
 * (f is linear in S) and grad[1..3] += c sum_k S M(d_k) lam_k (df_k/dx_psi
 * = S M(d_k)), c being the kick factor that multiplied f.                 */
static void attractor_grad_add(const double *x, int64_t N, double eps, double S,
                               const double *att_x, const double *lam, double c,
                               double *grad)
{
    if (!att_x || !grad)
        return;
    ksum g[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int64_t k = 0; k < N; ++k) {
        double mv[3], lf;
        attractor_m(x, N, k, eps * eps, att_x, lam, mv, &lf);
        ksum_add(&g[0], lf);
        ksum_add(&g[1], S * mv[0]);
        ksum_add(&g[2], S * mv[1]);
        ksum_add(&g[3], S * mv[2]);
    }
    for (int q = 0; q < 4; ++q)
        grad[q] += c * ksum_value(&g[q]);
}

/* out = (d f / d x)^T lam alone.                                          */
void oracle_attractor_vjp(const double *x, int64_t N, double eps, double S,
                          const double *att_x, const double *lam, double *out)
{
    for (int64_t i = 0; i < 3 * N; ++i)
        out[i] = 0.0;
    attractor_vjp_add(x, N, eps, S, att_x, lam, out);
}

/* ------------------------------------------------------------------------ */
/* Background term of Eq. (6).  The comoving potential there is the         */
/* particles' own plus a term a^2 (d^2 a/dt^2) |x|^2 / 2 (the |x|^2 factor  */
/* is lost in the printed equation).  It is what makes the comoving         */
/* equations exact Newtonian dynamics about a centre c; once the uniform    */
/* Lambda and radiation backgrounds, which the particle sum leaves out, act */
/* on the particles too, what remains is the removal of the mean matter     */
/* density's pull: a comoving field added to g of                           */
/*   f_k = b (x_k - c),   b = Om_M H0^2 / 2 = (4 pi G / 3) rho_comoving,     */
/* with potential -b |x_k - c|^2 / 2 (external: counted once in the energy) */
/* and derivative df_k/dx_k = b I.  It scales with a like the pair sum, so  */
/* it joins g before the a^-3 (or kick-integral) factor.  bg_c == NULL:     */
/* none.  Adds f into g and (phi != NULL) the potential into phi.           */
/* ------------------------------------------------------------------------ */
void oracle_background_add(const double *x, int64_t N, double b, const double *bg_c,
                           double *g, double *phi)
{
    if (!bg_c)
        return;
    for (int64_t k = 0; k < N; ++k) {
        double d[3];
        for (int c = 0; c < 3; ++c)
            d[c] = x[(size_t)c * N + k] - bg_c[c];
        if (g)
            for (int c = 0; c < 3; ++c)
                g[(size_t)c * N + k] += b * d[c];
        if (phi)
            phi[k] += -0.5 * b * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
}

/* out += (df/dx)^T lam = b lam (bg_c == NULL: nothing).                    */
static void background_vjp_add(int64_t N, double b, const double *bg_c, const double *lam,
                               double *out)
{
    if (!bg_c)
        return;
    for (size_t i = 0; i < 3 * (size_t)N; ++i)
        out[i] += b * lam[i];
}

/* ------------------------------------------------------------------------ */
/* Time grid and step coefficients.                                         */
/* ------------------------------------------------------------------------ */

/* a_n = a_begin exp(n Delta), Delta = ln(a_end/a_begin)/n_steps, and
 * a_{n_steps} is a_end exactly.  In the static limit a is constant.       */
static double grid_a(const cosmo *c, double a_begin, double a_end,
                     int64_t n_steps, double n)
{
    if (c->H0 == 0.0)
        return a_begin;
    if (n == (double)n_steps)
        return a_end;
    double delta = log(a_end / a_begin) / (double)n_steps;
    return a_begin * exp(n * delta);
}

typedef struct { double k1, d, k2, dt; } step_coef;

/* Kick-drift-kick coefficients of step n (Eq. (9)):
 *   k1 = int_{a_n}^{a_n+1/2} dt/a,  d = int_{a_n}^{a_n+1} dt/a^2,
 *   k2 = int_{a_n+1/2}^{a_n+1} dt/a,  dt = elapsed cosmic time.          */
static step_coef step_coefficients(const cosmo *c, double a_begin, double a_end,
                                   int64_t n_steps, int64_t n)
{
    step_coef s;
    if (c->H0 == 0.0) {
        double dt = a_end / (double)n_steps;
        double a = a_begin;
        s.k1 = 0.5 * dt / a;
        s.k2 = 0.5 * dt / a;
        s.d = dt / (a * a);
        s.dt = dt;
        return s;
    }
    double a0 = grid_a(c, a_begin, a_end, n_steps, (double)n);
    double ah = grid_a(c, a_begin, a_end, n_steps, (double)n + 0.5);
    double a1 = grid_a(c, a_begin, a_end, n_steps, (double)(n + 1));
    s.k1 = time_integral(c, 2, a0, ah);
    s.k2 = time_integral(c, 2, ah, a1);
    s.d = time_integral(c, 3, a0, a1);
    s.dt = time_integral(c, 1, a0, a1);
    return s;
}

/* Public: the four coefficients of step n, for tests. out = {k1, d, k2, dt}. */
void oracle_step_coefficients(double H0, double OmR, double OmM, double OmK,
                              double OmL, double a_begin, double a_end,
                              int64_t n_steps, int64_t n, double *out)
{
    cosmo c = {H0, OmR, OmM, OmK, OmL};
    step_coef s = step_coefficients(&c, a_begin, a_end, n_steps, n);
    out[0] = s.k1;
    out[1] = s.d;
    out[2] = s.k2;
    out[3] = s.dt;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                             */
/* Row layout (11 doubles): a, t, K, U, LI, P[3], L[3].                     */
/*   K = 1/2 sum m |p|^2 / a^2            (kinetic energy, p = a^2 v)       */
/*   U = (1/(2a)) sum m_k phi_k           (potential energy)                */
/*   LI = E - E_first + sum trapezoid(2K + U) d ln a  (Layzer-Irvine)       */
/*   P = sum m p,  L = sum m x cross p.                                     */
/* ------------------------------------------------------------------------ */
#define DIAG_W 11

static void energies(const double *x, const double *p, const double *m,
                     int64_t N, double eps, double G, double a, double S,
                     const double *att_x, double bg_b, const double *bg_c, double *K,
                     double *U, double *P, double *L)
{
    double *phi = (double *)malloc(sizeof(double) * (size_t)N);
    double *phe = (double *)calloc((size_t)N, sizeof(double));
    oracle_potential(x, m, N, eps, G, phi);
    oracle_attractor_add(x, N, eps, S, att_x, NULL, phe);
    oracle_background_add(x, N, bg_b, bg_c, NULL, phe);
    ksum kk = {0, 0}, uu = {0, 0}, ue = {0, 0};
    ksum pp[3] = {{0, 0}, {0, 0}, {0, 0}}, ll[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t k = 0; k < N; ++k) {
        double X = x[k], Y = x[N + k], Z = x[2 * N + k];
        double px = p[k], py = p[N + k], pz = p[2 * N + k];
        ksum_add(&kk, 0.5 * m[k] * (px * px + py * py + pz * pz));
        ksum_add(&uu, m[k] * phi[k]);
        ksum_add(&ue, m[k] * phe[k]);
        ksum_add(&pp[0], m[k] * px);
        ksum_add(&pp[1], m[k] * py);
        ksum_add(&pp[2], m[k] * pz);
        ksum_add(&ll[0], m[k] * (Y * pz - Z * py));
        ksum_add(&ll[1], m[k] * (Z * px - X * pz));
        ksum_add(&ll[2], m[k] * (X * py - Y * px));
    }
    *K = ksum_value(&kk) / (a * a);
    *U = (0.5 * ksum_value(&uu) + ksum_value(&ue)) / a;
    for (int i = 0; i < 3; ++i) {
        P[i] = ksum_value(&pp[i]);
        L[i] = ksum_value(&ll[i]);
    }
    free(phi);
    free(phe);
}

/* ------------------------------------------------------------------------ */
/* Tracer tracks: the state of chosen particles at every grid point a run   */
/* visits, so that a single particle's velocity can be followed step by     */
/* step (the purpose the introduction gives the method).  Row r of a track  */
/* holds [2][3][T] doubles: x_c of particle trk[t] at [0][c][t], its         */
/* comoving velocity v_c = dx/dt at [1][c][t].  The velocity is given as   */
/* v itself (scale 1) or as p = a^2 v (scale 1/a^2).                       */
/* ------------------------------------------------------------------------ */
static void record_track(const double *x, const double *vel, double a, int use_p,
                         int64_t N, const int64_t *trk, int64_t T, double *row)
{
    for (int64_t t = 0; t < T; ++t) {
        int64_t k = trk[t];
        for (int c = 0; c < 3; ++c) {
            row[(size_t)c * T + t] = x[(size_t)c * N + k];
            double w = vel[(size_t)c * N + k];
            row[(size_t)(3 + c) * T + t] = use_p ? w / (a * a) : w;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Run: kick-drift-kick steps first_step..last_step-1 of the global grid.   */
/*   p = a_n^2 v;  p += k1 g(x_n);  x += d p;  p += k2 g(x_{n+1}).          */
/* On return x, v hold the state at a_{last_step} (v = p/a^2).              */
/* diag (optional) receives last-first+1 rows of DIAG_W doubles; track      */
/* (optional, with trk[n_trk]) the same rows of tracer states.              */
/* ------------------------------------------------------------------------ */
int oracle_run(double *x, double *v, const double *m, int64_t N, double eps,
               double G, double H0, double OmR, double OmM, double OmK,
               double OmL, double a_begin, double a_end, int64_t n_steps,
               int64_t first_step, int64_t last_step, double *diag, double att_S,
               const double *att_x, double bg_b, const double *bg_c, const int64_t *trk,
               int64_t n_trk, double *track)
{
    cosmo c = {H0, OmR, OmM, OmK, OmL};
    if (N < 1 || n_steps < 1 || first_step < 0 || last_step <= first_step ||
        last_step > n_steps)
        return -1;
    size_t n3 = 3 * (size_t)N;
    double *p = (double *)malloc(sizeof(double) * n3);
    double *g = (double *)malloc(sizeof(double) * n3);
    double a = grid_a(&c, a_begin, a_end, n_steps, (double)first_step);
    for (size_t i = 0; i < n3; ++i)
        p[i] = a * a * v[i];
    oracle_forces(x, m, N, eps, G, 1.0, g);
    oracle_attractor_add(x, N, eps, att_S, att_x, g, NULL);
    oracle_background_add(x, N, bg_b, bg_c, g, NULL);
    const size_t trow = 6 * (size_t)n_trk;
    if (track)
        record_track(x, v, a, 0, N, trk, n_trk, track);

    double t = 0.0, E0 = 0.0, li_int = 0.0, prev_src = 0.0;
    if (diag) {
        double K, U, P[3], L[3];
        energies(x, p, m, N, eps, G, a, att_S, att_x, bg_b, bg_c, &K, &U, P, L);
        E0 = K + U;
        prev_src = 2.0 * K + U;
        double *row = diag;
        row[0] = a; row[1] = 0.0; row[2] = K; row[3] = U; row[4] = 0.0;
        for (int i = 0; i < 3; ++i) { row[5 + i] = P[i]; row[8 + i] = L[i]; }
    }
    for (int64_t n = first_step; n < last_step; ++n) {
        step_coef s = step_coefficients(&c, a_begin, a_end, n_steps, n);
        for (size_t i = 0; i < n3; ++i)
            p[i] += s.k1 * g[i];
        for (size_t i = 0; i < n3; ++i)
            x[i] += s.d * p[i];
        oracle_forces(x, m, N, eps, G, 1.0, g);
        oracle_attractor_add(x, N, eps, att_S, att_x, g, NULL);
        oracle_background_add(x, N, bg_b, bg_c, g, NULL);
        for (size_t i = 0; i < n3; ++i)
            p[i] += s.k2 * g[i];
        double a_prev = a;
        a = grid_a(&c, a_begin, a_end, n_steps, (double)(n + 1));
        t += s.dt;
        if (track)
            record_track(x, p, a, 1, N, trk, n_trk, track + (size_t)(n + 1 - first_step) * trow);
        if (diag) {
            double K, U, P[3], L[3];
            energies(x, p, m, N, eps, G, a, att_S, att_x, bg_b, bg_c, &K, &U, P, L);
            double src = 2.0 * K + U;
            double dlna = (c.H0 == 0.0) ? 0.0 : log(a) - log(a_prev);
            li_int += 0.5 * (prev_src + src) * dlna;
            prev_src = src;
            double *row = diag + (size_t)(n + 1 - first_step) * DIAG_W;
            row[0] = a; row[1] = t; row[2] = K; row[3] = U;
            row[4] = K + U - E0 + li_int;
            for (int i = 0; i < 3; ++i) { row[5 + i] = P[i]; row[8 + i] = L[i]; }
        }
    }
    for (size_t i = 0; i < n3; ++i)
        v[i] = p[i] / (a * a);
    free(p);
    free(g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The paper's difference equations, Eqs. (3)-(5) (Hockney-Eastwood):       */
/*   x^{n+1/2} = x^n + tau v^n / 2                                          */
/*   v^{n+1}   = v^n (1 - H tau)/(1 + H tau)                                */
/*               + g(x^{n+1/2}) tau / (a^3 (1 + H tau))                     */
/*   x^{n+1}   = x^{n+1/2} + tau v^{n+1} / 2                                */
/* with v = dx/dt the comoving velocity, g the comoving force sum (the      */
/* gradient term of Eq. (4) read with the attractive sign, as Eq. (1)),     */
/* tau the cosmic time of the step and H, a taken at the step's half time   */
/* t^{n+1/2} = t^n + tau/2.  The steps use the same grid a_n as the run.    */
/* ------------------------------------------------------------------------ */

/* (tau, a_h, H_h) of step n: tau = t(a_{n+1}) - t(a_n); a_h solves
 * t(a_h) - t(a_n) = tau / 2 (bisection on the monotone time integral);
 * H_h = H(a_h).  Static limit: tau = dt, a_h = a, H_h = 0.                 */
typedef struct { double tau, ah, Hh; } he_coef;

static he_coef he_coefficients(const cosmo *c, double a_begin, double a_end,
                               int64_t n_steps, int64_t n)
{
    he_coef h;
    if (c->H0 == 0.0) {
        h.tau = a_end / (double)n_steps;
        h.ah = a_begin;
        h.Hh = 0.0;
        return h;
    }
    double a0 = grid_a(c, a_begin, a_end, n_steps, (double)n);
    double a1 = grid_a(c, a_begin, a_end, n_steps, (double)(n + 1));
    h.tau = time_integral(c, 1, a0, a1);
    double half = 0.5 * h.tau;
    double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
    for (int it = 0; it < 200 && hi > lo; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        double t = time_integral(c, 1, a0, mid);
        /* t grows with mid for a0 < a1 (expanding) and shrinks otherwise */
        int below = (a0 < a1) ? (t < half) : (t > half);
        if (below)
            lo = mid;
        else
            hi = mid;
    }
    h.ah = 0.5 * (lo + hi);
    h.Hh = oracle_hubble(h.ah, c->H0, c->OmR, c->OmM, c->OmK, c->OmL);
    return h;
}

void oracle_he_coefficients(double H0, double OmR, double OmM, double OmK, double OmL,
                            double a_begin, double a_end, int64_t n_steps, int64_t n,
                            double *out)
{
    cosmo c = {H0, OmR, OmM, OmK, OmL};
    he_coef h = he_coefficients(&c, a_begin, a_end, n_steps, n);
    out[0] = h.tau;
    out[1] = h.ah;
    out[2] = h.Hh;
}

/* Steps first_step..last_step-1 of Eqs. (3)-(5) in place on x, v; diag as in
 * oracle_run (the state at the integer points, K = 1/2 sum m a^2 |v|^2).   */
int oracle_run_he(double *x, double *v, const double *m, int64_t N, double eps,
                  double G, double H0, double OmR, double OmM, double OmK,
                  double OmL, double a_begin, double a_end, int64_t n_steps,
                  int64_t first_step, int64_t last_step, double *diag, double att_S,
                  const double *att_x, double bg_b, const double *bg_c, const int64_t *trk,
                  int64_t n_trk, double *track)
{
    cosmo c = {H0, OmR, OmM, OmK, OmL};
    if (N < 1 || n_steps < 1 || first_step < 0 || last_step <= first_step ||
        last_step > n_steps)
        return -1;
    size_t n3 = 3 * (size_t)N;
    double *g = (double *)malloc(sizeof(double) * n3);
    double *p = (double *)malloc(sizeof(double) * n3);
    double a = grid_a(&c, a_begin, a_end, n_steps, (double)first_step);
    double t = 0.0, E0 = 0.0, li_int = 0.0, prev_src = 0.0;
    const size_t trow = 6 * (size_t)n_trk;
    if (track)
        record_track(x, v, a, 0, N, trk, n_trk, track);
    if (diag) {
        double K, U, P[3], L[3];
        for (size_t i = 0; i < n3; ++i)
            p[i] = a * a * v[i];
        energies(x, p, m, N, eps, G, a, att_S, att_x, bg_b, bg_c, &K, &U, P, L);
        E0 = K + U;
        prev_src = 2.0 * K + U;
        double *row = diag;
        row[0] = a; row[1] = 0.0; row[2] = K; row[3] = U; row[4] = 0.0;
        for (int i = 0; i < 3; ++i) { row[5 + i] = P[i]; row[8 + i] = L[i]; }
    }
    for (int64_t n = first_step; n < last_step; ++n) {
        he_coef h = he_coefficients(&c, a_begin, a_end, n_steps, n);
        double tau = h.tau, Ht = h.Hh * h.tau;
        for (size_t i = 0; i < n3; ++i)
            x[i] += 0.5 * tau * v[i];
        oracle_forces(x, m, N, eps, G, 1.0, g);
        oracle_attractor_add(x, N, eps, att_S, att_x, g, NULL);
        oracle_background_add(x, N, bg_b, bg_c, g, NULL);
        double drag = (1.0 - Ht) / (1.0 + Ht);
        double kick = tau / (h.ah * h.ah * h.ah * (1.0 + Ht));
        for (size_t i = 0; i < n3; ++i)
            v[i] = v[i] * drag + g[i] * kick;
        for (size_t i = 0; i < n3; ++i)
            x[i] += 0.5 * tau * v[i];
        double a_prev = a;
        a = grid_a(&c, a_begin, a_end, n_steps, (double)(n + 1));
        t += tau;
        if (track)
            record_track(x, v, a, 0, N, trk, n_trk, track + (size_t)(n + 1 - first_step) * trow);
        if (diag) {
            double K, U, P[3], L[3];
            for (size_t i = 0; i < n3; ++i)
                p[i] = a * a * v[i];
            energies(x, p, m, N, eps, G, a, att_S, att_x, bg_b, bg_c, &K, &U, P, L);
            double src = 2.0 * K + U;
            double dlna = (c.H0 == 0.0) ? 0.0 : log(a) - log(a_prev);
            li_int += 0.5 * (prev_src + src) * dlna;
            prev_src = src;
            double *row = diag + (size_t)(n + 1 - first_step) * DIAG_W;
            row[0] = a; row[1] = t; row[2] = K; row[3] = U;
            row[4] = K + U - E0 + li_int;
            for (int i = 0; i < 3; ++i) { row[5 + i] = P[i]; row[8 + i] = L[i]; }
        }
    }
    free(g);
    free(p);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Velocity power spectrum of a tracer's track: the periodogram of its      */
/* velocity series over the M rows (the "energy power spectrum" of a single */
/* particle's velocity that the introduction names as the method's goal):   */
/*   E(k) = (1/M) sum_c | sum_{n<M} w_c[n] exp(-2 pi i k n / M) |^2,        */
/*   k = 0 .. M/2,  w_c[n] = v_c at row n, less its mean over the rows if   */
/*   remove_mean.  The rows are the run's grid points, uniform in ln a, so  */
/*   k counts cycles per M steps of that grid.  The phase k n is reduced    */
/*   modulo M exactly before the angle is formed.                           */
/* out[t][k], (M/2 + 1) values per tracer.                                  */
/* ------------------------------------------------------------------------ */
void oracle_velocity_spectrum(const double *track, int64_t M, int64_t T, int remove_mean,
                              double *out)
{
    const int64_t K = M / 2 + 1;
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < T; ++t) {
        double *w = (double *)malloc(sizeof(double) * (size_t)M);
        for (int64_t k = 0; k < K; ++k)
            out[t * K + k] = 0.0;
        for (int c = 0; c < 3; ++c) {
            ksum mean = {0, 0};
            for (int64_t n = 0; n < M; ++n) {
                w[n] = track[(size_t)n * 6 * T + (size_t)(3 + c) * T + t];
                ksum_add(&mean, w[n]);
            }
            double mu = remove_mean ? ksum_value(&mean) / (double)M : 0.0;
            for (int64_t n = 0; n < M; ++n)
                w[n] -= mu;
            for (int64_t k = 0; k < K; ++k) {
                ksum re = {0, 0}, im = {0, 0};
                for (int64_t n = 0; n < M; ++n) {
                    int64_t j = (k * n) % M;
                    double ang = two_pi * (double)j / (double)M;
                    ksum_add(&re, w[n] * cos(ang));
                    ksum_add(&im, -w[n] * sin(ang));
                }
                double r = ksum_value(&re), i = ksum_value(&im);
                out[t * K + k] += (r * r + i * i) / (double)M;
            }
        }
        free(w);
    }
}

/* The same periodogram at chosen bins only (n_bins values per tracer,     */
/* out[t][b] = E(bins[b])), for series too long for every bin.             */
void oracle_velocity_spectrum_bins(const double *track, int64_t M, int64_t T, int remove_mean,
                                   const int64_t *bins, int64_t n_bins, double *out)
{
    const double two_pi = 6.283185307179586476925286766559;
    double *w = (double *)malloc(sizeof(double) * (size_t)M);
    for (int64_t t = 0; t < T; ++t) {
        for (int64_t b = 0; b < n_bins; ++b)
            out[t * n_bins + b] = 0.0;
        for (int c = 0; c < 3; ++c) {
            ksum mean = {0, 0};
            for (int64_t n = 0; n < M; ++n) {
                w[n] = track[(size_t)n * 6 * T + (size_t)(3 + c) * T + t];
                ksum_add(&mean, w[n]);
            }
            double mu = remove_mean ? ksum_value(&mean) / (double)M : 0.0;
            for (int64_t n = 0; n < M; ++n)
                w[n] -= mu;
#pragma omp parallel for schedule(static)
            for (int64_t b = 0; b < n_bins; ++b) {
                const int64_t k = bins[b];
                ksum re = {0, 0}, im = {0, 0};
                for (int64_t n = 0; n < M; ++n) {
                    int64_t j = (k * n) % M;
                    double ang = two_pi * (double)j / (double)M;
                    ksum_add(&re, w[n] * cos(ang));
                    ksum_add(&im, -w[n] * sin(ang));
                }
                double r = ksum_value(&re), i = ksum_value(&im);
                out[t * n_bins + b] += (r * r + i * i) / (double)M;
            }
        }
    }
    free(w);
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint (reverse mode of the run map, every state stored).      */
/* Forward step n:  p' = p_n + k1 g(x_n);  x_{n+1} = x_n + d p';            */
/*                  p_{n+1} = p' + k2 g(x_{n+1}).                           */
/* Reverse step n:  lx += k2 J(x_{n+1})^T lp;  lp += d lx;                  */
/*                  lx += k1 J(x_n)^T lp.                                   */
/* Boundary maps: p_0 = a_0^2 v_0, v_N = p_N / a_N^2.                       */
/* For each of n_cot cotangent pairs (lam_xN, lam_vN) [n_cot][3][N] the     */
/* gradients with respect to x_0 and v_0 are written to grad_x0, grad_v0.   */
/* xN, vN (optional) receive the forward end state.                         */
/* ------------------------------------------------------------------------ */
int oracle_adjoint(const double *x0, const double *v0, const double *m,
                   int64_t N, double eps, double G, double H0, double OmR,
                   double OmM, double OmK, double OmL, double a_begin,
                   double a_end, int64_t n_steps, int32_t n_cot,
                   const double *lam_xN, const double *lam_vN, double *grad_x0,
                   double *grad_v0, double *xN, double *vN, double att_S,
                   const double *att_x, double bg_b, const double *bg_c, double *grad_att)
{
    cosmo c = {H0, OmR, OmM, OmK, OmL};
    if (N < 1 || n_steps < 1 || n_cot < 1)
        return -1;
    size_t n3 = 3 * (size_t)N;
    double *xs = (double *)malloc(sizeof(double) * n3 * (size_t)(n_steps + 1));
    double *p = (double *)malloc(sizeof(double) * n3);
    double *g = (double *)malloc(sizeof(double) * n3);
    step_coef *coef = (step_coef *)malloc(sizeof(step_coef) * (size_t)n_steps);
    double a0 = grid_a(&c, a_begin, a_end, n_steps, 0.0);
    double aN = grid_a(&c, a_begin, a_end, n_steps, (double)n_steps);

    memcpy(xs, x0, sizeof(double) * n3);
    for (size_t i = 0; i < n3; ++i)
        p[i] = a0 * a0 * v0[i];
    oracle_forces(xs, m, N, eps, G, 1.0, g);
    oracle_attractor_add(xs, N, eps, att_S, att_x, g, NULL);
    oracle_background_add(xs, N, bg_b, bg_c, g, NULL);
    for (int64_t n = 0; n < n_steps; ++n) {
        coef[n] = step_coefficients(&c, a_begin, a_end, n_steps, n);
        double *xn = xs + (size_t)n * n3, *xn1 = xs + (size_t)(n + 1) * n3;
        for (size_t i = 0; i < n3; ++i)
            p[i] += coef[n].k1 * g[i];
        for (size_t i = 0; i < n3; ++i)
            xn1[i] = xn[i] + coef[n].d * p[i];
        oracle_forces(xn1, m, N, eps, G, 1.0, g);
        oracle_attractor_add(xn1, N, eps, att_S, att_x, g, NULL);
        oracle_background_add(xn1, N, bg_b, bg_c, g, NULL);
        for (size_t i = 0; i < n3; ++i)
            p[i] += coef[n].k2 * g[i];
    }
    if (xN)
        memcpy(xN, xs + (size_t)n_steps * n3, sizeof(double) * n3);
    if (vN)
        for (size_t i = 0; i < n3; ++i)
            vN[i] = p[i] / (aN * aN);

    double *lx = (double *)malloc(sizeof(double) * n3);
    double *lp = (double *)malloc(sizeof(double) * n3);
    double *w = (double *)malloc(sizeof(double) * n3);
    for (int32_t ci = 0; ci < n_cot; ++ci) {
        const double *lxN = lam_xN + (size_t)ci * n3;
        const double *lvN = lam_vN + (size_t)ci * n3;
        double *ga = grad_att ? grad_att + 4 * (size_t)ci : NULL;
        if (ga)
            for (int q = 0; q < 4; ++q)
                ga[q] = 0.0;
        for (size_t i = 0; i < n3; ++i) {
            lx[i] = lxN[i];
            lp[i] = lvN[i] / (aN * aN);
        }
        for (int64_t n = n_steps - 1; n >= 0; --n) {
            double *xn = xs + (size_t)n * n3, *xn1 = xs + (size_t)(n + 1) * n3;
            oracle_force_vjp(xn1, m, N, eps, G, lp, w);
            attractor_vjp_add(xn1, N, eps, att_S, att_x, lp, w);
            background_vjp_add(N, bg_b, bg_c, lp, w);
            attractor_grad_add(xn1, N, eps, att_S, att_x, lp, coef[n].k2, ga);
            for (size_t i = 0; i < n3; ++i)
                lx[i] += coef[n].k2 * w[i];
            for (size_t i = 0; i < n3; ++i)
                lp[i] += coef[n].d * lx[i];
            oracle_force_vjp(xn, m, N, eps, G, lp, w);
            attractor_vjp_add(xn, N, eps, att_S, att_x, lp, w);
            background_vjp_add(N, bg_b, bg_c, lp, w);
            attractor_grad_add(xn, N, eps, att_S, att_x, lp, coef[n].k1, ga);
            for (size_t i = 0; i < n3; ++i)
                lx[i] += coef[n].k1 * w[i];
        }
        double *gx = grad_x0 + (size_t)ci * n3, *gv = grad_v0 + (size_t)ci * n3;
        for (size_t i = 0; i < n3; ++i) {
            gx[i] = lx[i];
            gv[i] = a0 * a0 * lp[i];
        }
    }
    free(lx);
    free(lp);
    free(w);
    free(xs);
    free(p);
    free(g);
    free(coef);
    return 0;
}
