/*
 * Calls every entry point of the CPU oracle on a small input, for a build
 * of the oracle under the address and undefined-behaviour sanitizers (test
 * infrastructure: the oracle is checked, not used).  Exits 0 when every
 * call returned and every output is finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_num_threads(void);
void oracle_set_num_threads(int n);
double oracle_hubble(double a, double H0, double OmR, double OmM, double OmK, double OmL);
double oracle_time_integral(int kind, double a1, double a2, double H0, double OmR, double OmM,
                            double OmK, double OmL);
void oracle_forces(const double *x, const double *m, int64_t N, double eps, double G, double a,
                   double *acc);
void oracle_forces_targets(const double *x, const double *m, int64_t N, const int64_t *targets,
                           int64_t n_targets, double eps, double G, double a, double *acc);
void oracle_potential(const double *x, const double *m, int64_t N, double eps, double G,
                      double *phi);
void oracle_force_vjp(const double *x, const double *m, int64_t N, double eps, double G,
                      const double *lam, double *out);
void oracle_attractor_add(const double *x, int64_t N, double eps, double S, const double *att_x,
                          double *g, double *phi);
void oracle_attractor_vjp(const double *x, int64_t N, double eps, double S, const double *att_x,
                          const double *lam, double *out);
void oracle_background_add(const double *x, int64_t N, double b, const double *bg_c, double *g,
                           double *phi);
void oracle_step_coefficients(double H0, double OmR, double OmM, double OmK, double OmL,
                              double a_begin, double a_end, int64_t n_steps, int64_t n,
                              double *out);
int oracle_run(double *x, double *v, const double *m, int64_t N, double eps, double G, double H0,
               double OmR, double OmM, double OmK, double OmL, double a_begin, double a_end,
               int64_t n_steps, int64_t first_step, int64_t last_step, double *diag,
               double att_S, const double *att_x, double bg_b, const double *bg_c,
               const int64_t *trk, int64_t n_trk, double *track);
void oracle_he_coefficients(double H0, double OmR, double OmM, double OmK, double OmL,
                            double a_begin, double a_end, int64_t n_steps, int64_t n,
                            double *out);
int oracle_run_he(double *x, double *v, const double *m, int64_t N, double eps, double G,
                  double H0, double OmR, double OmM, double OmK, double OmL, double a_begin,
                  double a_end, int64_t n_steps, int64_t first_step, int64_t last_step,
                  double *diag, double att_S, const double *att_x, double bg_b,
                  const double *bg_c, const int64_t *trk, int64_t n_trk, double *track);
void oracle_velocity_spectrum(const double *track, int64_t M, int64_t T, int remove_mean,
                              double *out);
void oracle_velocity_spectrum_bins(const double *track, int64_t M, int64_t T, int remove_mean,
                                   const int64_t *bins, int64_t n_bins, double *out);
int oracle_adjoint(const double *x0, const double *v0, const double *m, int64_t N, double eps,
                   double G, double H0, double OmR, double OmM, double OmK, double OmL,
                   double a_begin, double a_end, int64_t n_steps, int32_t n_cot,
                   const double *lam_xN, const double *lam_vN, double *grad_x0,
                   double *grad_v0, double *xN, double *vN, double att_S, const double *att_x,
                   double bg_b, const double *bg_c, double *grad_att);

#define N 7
#define STEPS 4
#define DIAG_W 11

static int bad = 0;

static void check(const char *what, const double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) {
            fprintf(stderr, "%s: non-finite output at %zu\n", what, i);
            bad = 1;
            return;
        }
}

static double lcg(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

int main(void)
{
    const double H0 = 1.6, OmR = 0.0, OmM = 0.3, OmK = 0.0, OmL = 0.7;
    const double eps = 0.05, G = 0.9;
    uint64_t seed = 12345;
    double x[3 * N], v[3 * N], m[N], lam[3 * N];
    for (int i = 0; i < 3 * N; ++i) {
        x[i] = lcg(&seed);
        v[i] = 0.1 * lcg(&seed);
        lam[i] = lcg(&seed);
    }
    for (int i = 0; i < N; ++i)
        m[i] = (1.0 + lcg(&seed)) / N;
    const double att_x[3] = {0.3, -0.2, 0.1}, bg_c[3] = {0.0, 0.0, 0.0};

    oracle_set_num_threads(2);
    if (oracle_num_threads() < 1)
        bad = 1;
    double h = oracle_hubble(0.5, H0, OmR, OmM, OmK, OmL);
    double t[3];
    for (int k = 1; k <= 3; ++k)
        t[k - 1] = oracle_time_integral(k, 0.2, 0.9, H0, OmR, OmM, OmK, OmL);
    check("hubble", &h, 1);
    check("time_integral", t, 3);

    double acc[3 * N], phi[N], out[3 * N], g[3 * N] = {0}, ph[N] = {0};
    int64_t targets[3] = {0, 3, 6};
    double acc_t[9];
    oracle_forces(x, m, N, eps, G, 0.5, acc);
    oracle_forces_targets(x, m, N, targets, 3, eps, G, 0.5, acc_t);
    oracle_potential(x, m, N, eps, G, phi);
    oracle_force_vjp(x, m, N, eps, G, lam, out);
    oracle_attractor_add(x, N, eps, 0.2, att_x, g, ph);
    oracle_background_add(x, N, 1.1, bg_c, g, ph);
    check("forces", acc, 3 * N);
    check("forces_targets", acc_t, 9);
    check("potential", phi, N);
    check("force_vjp", out, 3 * N);
    check("external terms", g, 3 * N);
    check("external potential", ph, N);
    oracle_attractor_vjp(x, N, eps, 0.2, att_x, lam, out);
    check("attractor_vjp", out, 3 * N);

    double coef[4], hec[3];
    oracle_step_coefficients(H0, OmR, OmM, OmK, OmL, 0.2, 1.0, STEPS, 1, coef);
    oracle_he_coefficients(H0, OmR, OmM, OmK, OmL, 0.2, 1.0, STEPS, 1, hec);
    check("step_coefficients", coef, 4);
    check("he_coefficients", hec, 3);

    const int64_t trk[2] = {1, 5};
    double diag[(STEPS + 1) * DIAG_W], track[(STEPS + 1) * 6 * 2];
    for (int scheme = 0; scheme < 2; ++scheme) {
        double xs[3 * N], vs[3 * N];
        for (int i = 0; i < 3 * N; ++i) {
            xs[i] = x[i];
            vs[i] = v[i];
        }
        int rc = scheme == 0 ? oracle_run(xs, vs, m, N, eps, G, H0, OmR, OmM, OmK, OmL, 0.2,
                                          1.0, STEPS, 0, STEPS, diag, 0.2, att_x, 1.1, bg_c,
                                          trk, 2, track)
                             : oracle_run_he(xs, vs, m, N, eps, G, H0, OmR, OmM, OmK, OmL,
                                             0.2, 1.0, STEPS, 0, STEPS, diag, 0.2, att_x, 1.1,
                                             bg_c, trk, 2, track);
        if (rc != 0)
            bad = 1;
        check("run state", xs, 3 * N);
        check("run diag", diag, (STEPS + 1) * DIAG_W);
        check("run track", track, (STEPS + 1) * 6 * 2);
    }
    double spec[2 * ((STEPS + 1) / 2 + 1)], specb[4];
    const int64_t bins[2] = {0, 2};
    oracle_velocity_spectrum(track, STEPS + 1, 2, 1, spec);
    oracle_velocity_spectrum_bins(track, STEPS + 1, 2, 0, bins, 2, specb);
    check("spectrum", spec, 2 * ((STEPS + 1) / 2 + 1));
    check("spectrum bins", specb, 4);

    double lx[2 * 3 * N], lv[2 * 3 * N], gx[2 * 3 * N], gv[2 * 3 * N], xN[3 * N], vN[3 * N];
    double ga[2 * 4];
    for (int i = 0; i < 2 * 3 * N; ++i) {
        lx[i] = lcg(&seed);
        lv[i] = lcg(&seed);
    }
    if (oracle_adjoint(x, v, m, N, eps, G, H0, OmR, OmM, OmK, OmL, 0.2, 1.0, STEPS, 2, lx, lv,
                       gx, gv, xN, vN, 0.2, att_x, 1.1, bg_c, ga) != 0)
        bad = 1;
    check("adjoint grad_x", gx, 2 * 3 * N);
    check("adjoint grad_v", gv, 2 * 3 * N);
    check("adjoint grad_att", ga, 8);
    if (bad)
        return 1;
    printf("oracle driver ok\n");
    return 0;
}
