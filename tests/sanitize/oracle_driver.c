/* Drives the FP64 oracle (oracle/rbe_oracle.c) through every function on
 * small inputs, for an AddressSanitizer / UndefinedBehaviorSanitizer build
 * on the CPU.  Exit status 0 when every call returned sane values. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double oracle_H_direct(double, double);
double oracle_H_dual(double, double);
double oracle_S(double, double);
double oracle_S_bruteforce(double, double, int);
void oracle_philox4x32_10(const uint32_t *, const uint32_t *, uint32_t *);
int oracle_mode_range(double, double);
void oracle_mode_cdf(double, double, double *);
int oracle_sample_modes(double, double, int, uint64_t, uint64_t, int32_t *);
int oracle_sample_modes_mh(double, double, int, uint64_t, uint64_t, int32_t *, int32_t *, int);
void oracle_rho(int, const double *, const double *, double, int, const int32_t *, double *, double *);
void oracle_kspace_force(int, const double *, const double *, double, int, const int32_t *, const double *,
                         double, double *);
void oracle_kspace_force_subset(int, const double *, const double *, double, int, const int32_t *,
                                const double *, double, int, const int32_t *, double *);
double oracle_kspace_energy(int, const double *, const double *, double, int, const int32_t *, const double *,
                            double);
void oracle_rbe_weights(double, double, int, double *);
int oracle_ewald_modes(double, double, int, int32_t *, double *, int);
void oracle_real_force_ex(int, const double *, const double *, double, double, double, double, double, double,
                          double, const double *, int, int, const int32_t *, double *, double *, double *,
                          double *);
void oracle_forces_vjp(int, const double *, const double *, double, double, double, double, double, double,
                       double, int, const int32_t *, const double *, const double *, double, int, double *,
                       double *);
void oracle_pair_histogram(int, const double *, const double *, double, double, int, int64_t *);

#define N 64
#define P 12

int main(void)
{
    double pos[3 * N], q[N], F[3 * N], F2[3 * N], gF[3 * N], gq[N], gr[3 * N], er[N], el[N], vir[N], diam[N];
    int32_t modes[3 * P], state[3] = {0, 0, 0}, idx[3] = {N - 1, 0, 7};
    double w[P], re[P], im[P], Fs[9], cdf[4096];
    int64_t counts[3 * 20] = {0};
    const double L = 8.0, alpha = 0.9;
    srand(7);
    for (int i = 0; i < N; ++i) {
        for (int d = 0; d < 3; ++d) pos[d * N + i] = L * (double)rand() / RAND_MAX;
        q[i] = (i % 2) ? 1.0 : -1.0;
        diam[i] = i == 0 ? 2.0 : 1.0;
        for (int d = 0; d < 3; ++d) gF[d * N + i] = 0.01 * (d + 1);
    }
    int bad = 0;
    bad |= !(fabs(oracle_H_direct(alpha, L) - oracle_H_dual(alpha, L)) < 1e-10);
    bad |= !(oracle_S(alpha, L) > 0 && oracle_S_bruteforce(alpha, L, 6) > 0);
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    int M = oracle_mode_range(alpha, L);
    bad |= !(2 * M + 1 <= 4096);
    oracle_mode_cdf(alpha, L, cdf);
    oracle_sample_modes(alpha, L, P, 9, 1, modes);
    oracle_sample_modes_mh(alpha, L, P, 9, 1, state, modes, 0);
    oracle_rbe_weights(alpha, L, P, w);
    oracle_rho(N, pos, q, L, P, modes, re, im);
    oracle_kspace_force(N, pos, q, L, P, modes, w, 1.0, F);
    oracle_kspace_force_subset(N, pos, q, L, P, modes, w, 1.0, 3, idx, Fs);
    bad |= !(Fs[0] == F[N - 1]);
    bad |= !isfinite(oracle_kspace_energy(N, pos, q, L, P, modes, w, 1.0));
    int nm = oracle_ewald_modes(alpha, L, 4, NULL, NULL, 0);
    int32_t *em = malloc(sizeof(int32_t) * 3 * nm);
    double *ew = malloc(sizeof(double) * nm);
    oracle_ewald_modes(alpha, L, 4, em, ew, nm);
    free(em);
    free(ew);
    oracle_real_force_ex(N, pos, q, L, alpha, 2.5, 1.0, 1.0, 0.3, 1.0, NULL, 0, N, NULL, F, er, el, vir);
    oracle_real_force_ex(N, pos, q, L, alpha, 2.5, 1.0, 1.0, 0.3, 1.0, NULL, 1, N, NULL, F2, er, el, vir);
    oracle_real_force_ex(N, pos, q, L, alpha, 2.5, 1.0, 1.0, 0.3, 0.3, diam, 1, 3, idx, F2, er, el, vir);
    oracle_forces_vjp(N, pos, q, L, alpha, 2.5, 1.0, 1.0, 0.3, 1.0, P, modes, w, gF, 0.5, 3, gq, gr);
    oracle_pair_histogram(N, pos, q, L, 4.0, 20, counts);
    for (int k = 0; k < 3 * N; ++k) bad |= !isfinite(F[k]) || !isfinite(gr[k]);
    printf("oracle driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
