/*
 * rbe_oracle.c -- plain FP64 CPU oracle for the random batch Ewald (RBE)
 * method of Jin, Li, Xu & Zhao, "A random batch Ewald method for particle
 * systems with Coulomb interactions" (arXiv:2010.01559).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Everything is double precision and written as the paper states it: sums
 * over particles and modes in their natural order, libm for erfc/exp/sin/cos,
 * no blocking or fusion.  OpenMP only parallelises independent particles.
 *
 * Conventions (paper Sec. 2):
 *   - cubic box of side L, V = L^3; positions are SoA: x[0..n), y[n..2n),
 *     z[2n..3n); forces use the same layout;
 *   - r_ij = r_j - r_i (Sec. 2, text before eq. 2.3);
 *   - k = 2*pi*m/L with integer m (Sec. 2, Fourier convention);
 *   - the k = 0 term is dropped (conducting boundary, text after eq. 2.7);
 *   - reduced units with Coulomb potential q/r (Sec. 4.1), times the scalar
 *     prefactor `coulomb` (the Bjerrum length l_B of Sec. 4.2, 1 otherwise);
 *   - k_B = 1 (Sec. 3.3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------ */
/* Normaliser S and the 1-D factor H: Sec. 3.1, eqs. (3.1)-(3.2).           */
/* ------------------------------------------------------------------------ */

/* H = sum_{m in Z} exp(-pi^2 m^2 / (alpha L^2)), summed directly (eq. 3.2,
 * left-hand form) until the terms no longer change the sum. */
double oracle_H_direct(double alpha, double L)
{
    double a = ORC_PI * ORC_PI / (alpha * L * L);
    double h = 1.0;
    for (long m = 1; m < 100000000; ++m) {
        double t = exp(-a * (double)m * (double)m);
        if (t == 0.0 || t < h * 1e-20) break;
        h += 2.0 * t;
    }
    return h;
}

/* H = sqrt(alpha L^2 / pi) * sum_{m in Z} exp(-alpha m^2 L^2), the Poisson
 * dual form (eq. 3.2, right-hand form). */
double oracle_H_dual(double alpha, double L)
{
    double b = alpha * L * L;
    double h = 1.0;
    for (long m = 1; m < 100000000; ++m) {
        double t = exp(-b * (double)m * (double)m);
        if (t == 0.0 || t < h * 1e-20) break;
        h += 2.0 * t;
    }
    return sqrt(alpha * L * L / ORC_PI) * h;
}

/* S = sum_{k != 0} exp(-k^2/(4 alpha)) = H^3 - 1 (eq. 3.1). */
double oracle_S(double alpha, double L)
{
    double h = oracle_H_direct(alpha, L);
    return h * h * h - 1.0;
}

/* S by brute force over the 3-D lattice |m_d| <= mmax (for pinning eq. 3.1
 * against its own definition on small boxes). */
double oracle_S_bruteforce(double alpha, double L, int mmax)
{
    double s = 0.0;
    for (int a = -mmax; a <= mmax; ++a)
        for (int b = -mmax; b <= mmax; ++b)
            for (int c = -mmax; c <= mmax; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                double kx = 2.0 * ORC_PI * a / L, ky = 2.0 * ORC_PI * b / L, kz = 2.0 * ORC_PI * c / L;
                double k2 = kx * kx + ky * ky + kz * kz;
                s += exp(-k2 / (4.0 * alpha));
            }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from the   */
/* published description: 10 rounds of two 32x32->64 multiplications with   */
/* multipliers 0xD2511F53 and 0xCD9E8D57, a word permutation, and a Weyl key */
/* schedule with increments 0x9E3779B9 and 0xBB67AE85.                      */
/* ------------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream tags occupying the top byte of counter word 1: they keep the random
 * numbers of different purposes apart under one (seed, step) key. */
#define ORC_TAG_KSAMPLE  0x01000000u
#define ORC_TAG_LANGEVIN 0x02000000u
#define ORC_TAG_ANDERSEN 0x03000000u
#define ORC_TAG_MH       0x04000000u

/* 53-bit uniform in [0,1) from two 32-bit words: 27 high bits of a, 26 of b. */
static double orc_u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

static void orc_draw(uint32_t idx, uint32_t word1, uint64_t seed, uint64_t step, uint32_t out[4])
{
    uint32_t ctr[4] = { idx, word1, (uint32_t)step, (uint32_t)(step >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    oracle_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Importance sampling of the modes: Sec. 3.1, eqs. (3.3)-(3.5).             */
/* ------------------------------------------------------------------------ */

/* 1-D target P(m) proportional to exp(-pi^2 m^2/(alpha L^2)) (eq. 3.4).  Its
 * standard deviation as a continuous Gaussian is sigma = sqrt(alpha L^2/(2 pi^2)).
 * The table spans |m| <= M with M = ceil(10 sigma) + 1, beyond which the mass
 * is below exp(-50) relative. */
int oracle_mode_range(double alpha, double L)
{
    double sigma = sqrt(alpha * L * L / (2.0 * ORC_PI * ORC_PI));
    return (int)ceil(10.0 * sigma) + 1;
}

/* Cumulative table cdf[k], k = 0..2M, for m = k - M: partial sums of the
 * unnormalised weights accumulated from m = -M upwards, divided by the total. */
static double *orc_cdf_table(double alpha, double L, int *M_out)
{
    int M = oracle_mode_range(alpha, L);
    int K = 2 * M + 1;
    double a = ORC_PI * ORC_PI / (alpha * L * L);
    double *w = (double *)malloc(sizeof(double) * K);
    double tot = 0.0;
    for (int k = 0; k < K; ++k) {
        double m = (double)(k - M);
        w[k] = exp(-a * m * m);
    }
    for (int k = 0; k < K; ++k) tot += w[k];
    double run = 0.0;
    for (int k = 0; k < K; ++k) {
        run += w[k];
        w[k] = run / tot;
    }
    *M_out = M;
    return w;
}

void oracle_mode_cdf(double alpha, double L, double *cdf_out /* [2M+1] */)
{
    int M;
    double *t = orc_cdf_table(alpha, L, &M);
    memcpy(cdf_out, t, sizeof(double) * (2 * M + 1));
    free(t);
}

/* Inverse CDF: the smallest m whose cumulative mass exceeds u. */
static int orc_invert(const double *cdf, int M, double u)
{
    int K = 2 * M + 1;
    for (int k = 0; k < K; ++k)
        if (u < cdf[k]) return k - M;
    return M;
}

/* Exact i.i.d. sampler of P_k (eq. 3.3).  The 3-D weight factorises into the
 * 1-D weights of eq. (3.4), so each component is drawn independently by
 * inverting the 1-D cumulative table; the all-zero vector is discarded and
 * drawn again (Sec. 3.1).  Draw l, attempt a uses Philox counters
 * (l, TAG_KSAMPLE | 2a, step) and (l, TAG_KSAMPLE | 2a+1, step) under key
 * `seed`; the three 53-bit uniforms are (w0,w1), (w2,w3) of the first block
 * and (w0,w1) of the second.  modes is [3][p] (SoA).  Returns the number of
 * discarded zero vectors. */
int oracle_sample_modes(double alpha, double L, int p, uint64_t seed, uint64_t step, int32_t *modes)
{
    int M;
    double *cdf = orc_cdf_table(alpha, L, &M);
    int rejected = 0;
    for (int l = 0; l < p; ++l) {
        for (uint32_t a = 0;; ++a) {
            uint32_t r0[4], r1[4];
            orc_draw((uint32_t)l, ORC_TAG_KSAMPLE | (2u * a), seed, step, r0);
            orc_draw((uint32_t)l, ORC_TAG_KSAMPLE | (2u * a + 1u), seed, step, r1);
            int mx = orc_invert(cdf, M, orc_u53(r0[0], r0[1]));
            int my = orc_invert(cdf, M, orc_u53(r0[2], r0[3]));
            int mz = orc_invert(cdf, M, orc_u53(r1[0], r1[1]));
            if (mx == 0 && my == 0 && mz == 0) { ++rejected; continue; }
            modes[l] = mx; modes[p + l] = my; modes[2 * p + l] = mz;
            break;
        }
    }
    free(cdf);
    return rejected;
}

/* The three uniforms used by draw l, attempt a (for tests that check how
 * close a draw came to a table boundary). */
void oracle_sample_uniforms(uint64_t seed, uint64_t step, int l, int a, double u[3])
{
    uint32_t r0[4], r1[4];
    orc_draw((uint32_t)l, ORC_TAG_KSAMPLE | (2u * (uint32_t)a), seed, step, r0);
    orc_draw((uint32_t)l, ORC_TAG_KSAMPLE | (2u * (uint32_t)a + 1u), seed, step, r1);
    u[0] = orc_u53(r0[0], r0[1]);
    u[1] = orc_u53(r0[2], r0[3]);
    u[2] = orc_u53(r1[0], r1[1]);
}

/* Proposal mass of the paper's Metropolis-Hastings variant, eq. (3.5): the
 * probability that round(x*) = m* for x* ~ N(0, alpha L^2/(2 pi^2)). */
double oracle_mh_proposal_mass(double alpha, double L, int mstar)
{
    double w = sqrt(alpha * L * L / (ORC_PI * ORC_PI));
    int am = mstar < 0 ? -mstar : mstar;
    if (am == 0) return erf(0.5 / w);
    return 0.5 * (erf((am + 0.5) / w) - erf((am - 0.5) / w));
}

/* Round half away from zero (ties have measure zero). */
static int orc_round(double x)
{
    return x >= 0.0 ? (int)floor(x + 0.5) : -(int)floor(-x + 0.5);
}

/* The paper's Metropolis-Hastings sampler (Sec. 3.1), one independent chain
 * per component.  Proposal m* = round(x*), x* ~ N(0, alpha L^2/(2 pi^2));
 * standard independence-chain acceptance
 *   min{1, P(m*) qbar(m) / (P(m) qbar(m*))}
 * with qbar of eq. (3.5) and P of eq. (3.4).  `state` holds the three chain
 * states across calls.  All-zero vectors are discarded.  Attempt a of draw l
 * uses Philox blocks (l, TAG_MH | 4a + j, step), j = 0..3: block j < 3 gives
 * component j's Box-Muller uniforms 1 - u53(w0,w1) and u53(w2,w3) -> x*, and
 * words w0..w2 of block 3 times 2^-32 are the three acceptance uniforms.  If skip_accept is nonzero every proposal is
 * accepted (a planted mistake for tests). */
int oracle_sample_modes_mh(double alpha, double L, int p, uint64_t seed, uint64_t step,
                           int32_t state[3], int32_t *modes, int skip_accept)
{
    double a2 = ORC_PI * ORC_PI / (alpha * L * L);
    double sd = sqrt(alpha * L * L / (2.0 * ORC_PI * ORC_PI));
    int accepted = 0;
    for (int l = 0; l < p; ++l) {
        for (uint32_t a = 0;; ++a) {
            uint32_t r[4][4];
            for (int j = 0; j < 4; ++j)
                orc_draw((uint32_t)l, ORC_TAG_MH | (4u * a + (uint32_t)j), seed, step, r[j]);
            double acc_u[3] = { (double)r[3][0] * (1.0 / 4294967296.0),
                                (double)r[3][1] * (1.0 / 4294967296.0),
                                (double)r[3][2] * (1.0 / 4294967296.0) };
            for (int d = 0; d < 3; ++d) {
                double u1 = 1.0 - orc_u53(r[d][0], r[d][1]); /* (0,1] */
                double u2 = orc_u53(r[d][2], r[d][3]);
                double x = sd * sqrt(-2.0 * log(u1)) * cos(2.0 * ORC_PI * u2);
                int ms = orc_round(x);
                int mc = state[d];
                double ratio = exp(-a2 * ((double)ms * ms - (double)mc * mc)) *
                               oracle_mh_proposal_mass(alpha, L, mc) /
                               oracle_mh_proposal_mass(alpha, L, ms);
                if (skip_accept || acc_u[d] < ratio) { state[d] = ms; ++accepted; }
            }
            if (state[0] == 0 && state[1] == 0 && state[2] == 0) continue;
            modes[l] = state[0]; modes[p + l] = state[1]; modes[2 * p + l] = state[2];
            break;
        }
    }
    return accepted;
}

/* ------------------------------------------------------------------------ */
/* Structure factor and Fourier-space force/energy: Sec. 2, eqs. (2.6),      */
/* (2.7), (2.11); Sec. 3.1, eq. (3.6).                                       */
/* ------------------------------------------------------------------------ */

/* Phase k.r_j = 2 pi (m . r_j / L) taken modulo one revolution before the
 * trigonometric functions are applied. */
static double orc_phase(const int32_t *modes, int nm, int l, const double *pos, int n, int j, double L)
{
    double s = ((double)modes[l] * pos[j] + (double)modes[nm + l] * pos[n + j] +
                (double)modes[2 * nm + l] * pos[2 * n + j]) / L;
    s -= floor(s);
    return 2.0 * ORC_PI * s;
}

/* rho(k_l) = sum_j q_j exp(i k_l . r_j) (eq. 2.7); re[l] + i im[l]. */
void oracle_rho(int n, const double *pos, const double *q, double L, int nm, const int32_t *modes,
                double *re, double *im)
{
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nm; ++l) {
        double c = 0.0, s = 0.0;
        for (int j = 0; j < n; ++j) {
            double th = orc_phase(modes, nm, l, pos, n, j, L);
            c += q[j] * cos(th);
            s += q[j] * sin(th);
        }
        re[l] = c;
        im[l] = s;
    }
}

/* Fourier-space force with a per-mode weight (eq. 2.11, first term):
 *   F_i = -coulomb * sum_l weight_l * (4 pi q_i k_l / (V k_l^2)) * Im(exp(-i k_l.r_i) rho(k_l)).
 * weight_l = exp(-k^2/(4 alpha)) over an enumerated list gives the classical
 * Ewald sum; weight_l = S/p over p sampled modes gives the random batch
 * estimator of eq. (3.6).  F is [3][n] and is overwritten. */
void oracle_kspace_force(int n, const double *pos, const double *q, double L, int nm,
                         const int32_t *modes, const double *weight, double coulomb, double *F)
{
    double *re = (double *)malloc(sizeof(double) * nm);
    double *im = (double *)malloc(sizeof(double) * nm);
    oracle_rho(n, pos, q, L, nm, modes, re, im);
    double V = L * L * L;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int l = 0; l < nm; ++l) {
            double kx = 2.0 * ORC_PI * modes[l] / L;
            double ky = 2.0 * ORC_PI * modes[nm + l] / L;
            double kz = 2.0 * ORC_PI * modes[2 * nm + l] / L;
            double k2 = kx * kx + ky * ky + kz * kz;
            double th = orc_phase(modes, nm, l, pos, n, i, L);
            /* Im(exp(-i th) (re + i im)) = cos(th) im - sin(th) re */
            double imag = cos(th) * im[l] - sin(th) * re[l];
            double f = weight[l] * 4.0 * ORC_PI * q[i] / (V * k2) * imag;
            fx -= f * kx;
            fy -= f * ky;
            fz -= f * kz;
        }
        F[i] = coulomb * fx;
        F[n + i] = coulomb * fy;
        F[2 * n + i] = coulomb * fz;
    }
    free(re);
    free(im);
}

/* The same Fourier-space force on the listed particles only (rho still sums
 * over all n particles); F is [3][nsub]. */
void oracle_kspace_force_subset(int n, const double *pos, const double *q, double L, int nm,
                                const int32_t *modes, const double *weight, double coulomb,
                                int nsub, const int32_t *idx, double *F)
{
    double *re = (double *)malloc(sizeof(double) * nm);
    double *im = (double *)malloc(sizeof(double) * nm);
    oracle_rho(n, pos, q, L, nm, modes, re, im);
    double V = L * L * L;
#pragma omp parallel for schedule(static)
    for (int t = 0; t < nsub; ++t) {
        int i = idx[t];
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int l = 0; l < nm; ++l) {
            double kx = 2.0 * ORC_PI * modes[l] / L;
            double ky = 2.0 * ORC_PI * modes[nm + l] / L;
            double kz = 2.0 * ORC_PI * modes[2 * nm + l] / L;
            double k2 = kx * kx + ky * ky + kz * kz;
            double th = orc_phase(modes, nm, l, pos, n, i, L);
            double imag = cos(th) * im[l] - sin(th) * re[l];
            double f = weight[l] * 4.0 * ORC_PI * q[i] / (V * k2) * imag;
            fx -= f * kx;
            fy -= f * ky;
            fz -= f * kz;
        }
        F[t] = coulomb * fx;
        F[nsub + t] = coulomb * fy;
        F[2 * nsub + t] = coulomb * fz;
    }
    free(re);
    free(im);
}

/* Fourier-space energy with the same per-mode weights (eq. 2.6 without the
 * self term): coulomb * sum_l weight_l * (2 pi/(V k_l^2)) |rho(k_l)|^2. */
double oracle_kspace_energy(int n, const double *pos, const double *q, double L, int nm,
                            const int32_t *modes, const double *weight, double coulomb)
{
    double *re = (double *)malloc(sizeof(double) * nm);
    double *im = (double *)malloc(sizeof(double) * nm);
    oracle_rho(n, pos, q, L, nm, modes, re, im);
    double V = L * L * L, e = 0.0;
    for (int l = 0; l < nm; ++l) {
        double k2 = 4.0 * ORC_PI * ORC_PI *
                    ((double)modes[l] * modes[l] + (double)modes[nm + l] * modes[nm + l] +
                     (double)modes[2 * nm + l] * modes[2 * nm + l]) / (L * L);
        e += weight[l] * 2.0 * ORC_PI / (V * k2) * (re[l] * re[l] + im[l] * im[l]);
    }
    free(re);
    free(im);
    return coulomb * e;
}

/* Self-energy term -sqrt(alpha/pi) sum_i q_i^2 of eq. (2.6), times coulomb. */
double oracle_self_energy(int n, const double *q, double alpha, double coulomb)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += q[i] * q[i];
    return -coulomb * sqrt(alpha / ORC_PI) * s;
}

/* Random batch weights: every sampled mode carries S/p (eq. 3.6). */
void oracle_rbe_weights(double alpha, double L, int p, double *weight)
{
    double S = oracle_S(alpha, L);
    for (int l = 0; l < p; ++l) weight[l] = S / (double)p;
}

/* Classical Ewald mode list: all m != 0 with |m|^2 <= mmax2 (ball reading of
 * the cutoff k_c), weights exp(-k^2/(4 alpha)).  Returns the count; if modes
 * is NULL only counts.  modes is [3][cap]. */
int oracle_ewald_modes(double alpha, double L, int mmax2, int32_t *modes, double *weight, int cap)
{
    int R = (int)floor(sqrt((double)mmax2)) + 1;
    int cnt = 0;
    for (int a = -R; a <= R; ++a)
        for (int b = -R; b <= R; ++b)
            for (int c = -R; c <= R; ++c) {
                int m2 = a * a + b * b + c * c;
                if (m2 == 0 || m2 > mmax2) continue;
                if (modes) {
                    if (cnt >= cap) return -1;
                    modes[cnt] = a;
                    modes[cap + cnt] = b;
                    modes[2 * cap + cnt] = c;
                    double k2 = 4.0 * ORC_PI * ORC_PI * m2 / (L * L);
                    weight[cnt] = exp(-k2 / (4.0 * alpha));
                }
                ++cnt;
            }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Real space: eq. (2.9) third term and eq. (2.11) second term; shifted      */
/* Lennard-Jones of eq. (4.1) with r_off = (d_i + d_j)/2 - sigma.            */
/* ------------------------------------------------------------------------ */

/* G(r) of eq. (2.11). */
static double orc_G(double r, double alpha)
{
    double b = sqrt(alpha);
    return erfc(b * r) / (r * r) + 2.0 * b * exp(-alpha * r * r) / (sqrt(ORC_PI) * r);
}

/* Shifted LJ of eq. (4.1) at centre distance r with offset roff:
 * s = r - roff, V = 4 eps ((sig/s)^12 - (sig/s)^6) + V_shift for s < rc,
 * V_shift chosen so that V = 0 at s = rc.  *V is the energy, *dV = dV/dr. */
static void orc_lj(double r, double roff, double eps, double sig, double rc, double *V, double *dV)
{
    double s = r - roff;
    double sr6 = pow(sig / s, 6.0), sr12 = sr6 * sr6;
    double sc6 = pow(sig / rc, 6.0), sc12 = sc6 * sc6;
    *V = 4.0 * eps * (sr12 - sr6) - 4.0 * eps * (sc12 - sc6);
    *dV = 4.0 * eps * (-12.0 * sr12 + 6.0 * sr6) / s;
}

/* Parameters of the real-space sum. */
typedef struct {
    double L, alpha, rc, coulomb, lj_eps, lj_sigma, lj_rc;
    const double *diam;   /* per-particle diameters d_i, or NULL (d_i = sigma, r_off = 0) */
} orc_rs;

/* r_off of eq. (4.1) for the pair (i, j). */
static double orc_roff(const orc_rs *P, int i, int j)
{
    return P->diam ? 0.5 * (P->diam[i] + P->diam[j]) - P->lj_sigma : 0.0;
}

/* Largest centre distance at which some pair still interacts. */
static double orc_rmax(const orc_rs *P, int n)
{
    double rm = P->rc;
    if (P->lj_eps != 0.0) {
        double d1 = P->lj_sigma, d2 = P->lj_sigma;   /* two largest diameters */
        if (P->diam) {
            d1 = d2 = -1e300;
            for (int i = 0; i < n; ++i) {
                if (P->diam[i] > d1) { d2 = d1; d1 = P->diam[i]; }
                else if (P->diam[i] > d2) d2 = P->diam[i];
            }
            if (n < 2) d2 = d1;
        }
        double rl = 0.5 * (d1 + d2) - P->lj_sigma + P->lj_rc;
        if (rl > rm) rm = rl;
    }
    return rm;
}

/* One image of the pair (i, j) at displacement d = r_j - r_i + nL, |d| = r:
 * adds the force on i (coefficient times d), half the pair energies and
 * half of r_ij . F_ij (the pair virial).  Coulomb acts for r <= rc
 * (eq. 2.9), LJ for r - r_off < lj_rc (eq. 4.1). */
static void orc_pair(const orc_rs *P, const double *q, int i, int j, double dx, double dy, double dz, double r,
                     double f[3], double *ur, double *ul, double *vir)
{
    double c = 0.0;
    if (r <= P->rc) {
        c += -P->coulomb * q[i] * q[j] * orc_G(r, P->alpha) / r;
        *ur += 0.5 * P->coulomb * q[i] * q[j] * erfc(sqrt(P->alpha) * r) / r;
    }
    if (P->lj_eps != 0.0) {
        double roff = orc_roff(P, i, j);
        if (r - roff < P->lj_rc) {
            double V, dV;
            orc_lj(r, roff, P->lj_eps, P->lj_sigma, P->lj_rc, &V, &dV);
            c += dV / r;
            *ul += 0.5 * V;
        }
    }
    f[0] += c * dx;
    f[1] += c * dy;
    f[2] += c * dz;
    *vir += 0.5 * c * r * r;
}

/* Minimum-image displacement r_j - r_i. */
static void orc_min_image(const double *pos, int n, int i, int j, double L, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double x = pos[a * n + j] - pos[a * n + i];
        d[a] = x - L * floor(x / L + 0.5);
    }
}

/* Every image within reach, O(N^2) per listed particle.  Images other than
 * the minimum one lie at least L/2 away per axis, so for rmax < L/2 only the
 * minimum image is visited. */
static void orc_real_direct(int n, const double *pos, const double *q, const orc_rs *P, int nsub,
                            const int32_t *idx, double *Fsub, double *e_real, double *e_lj, double *vir)
{
    double L = P->L, rmax = orc_rmax(P, n);
    int nimg = rmax < 0.5 * L ? 0 : (int)ceil(rmax / L) + 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int t = 0; t < nsub; ++t) {
        int i = idx ? idx[t] : t;
        double f[3] = {0, 0, 0}, ur = 0, ul = 0, w = 0;
        for (int j = 0; j < n; ++j) {
            double d0[3];
            orc_min_image(pos, n, i, j, L, d0);
            for (int a = -nimg; a <= nimg; ++a)
                for (int b = -nimg; b <= nimg; ++b)
                    for (int c = -nimg; c <= nimg; ++c) {
                        if (j == i && a == 0 && b == 0 && c == 0) continue;
                        double dx = d0[0] + a * L, dy = d0[1] + b * L, dz = d0[2] + c * L;
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        if (r > rmax) continue;
                        orc_pair(P, q, i, j, dx, dy, dz, r, f, &ur, &ul, &w);
                    }
        }
        Fsub[t] = f[0]; Fsub[nsub + t] = f[1]; Fsub[2 * nsub + t] = f[2];
        if (e_real) e_real[t] = ur;
        if (e_lj) e_lj[t] = ul;
        if (vir) vir[t] = w;
    }
}

/* Linked-cell list (a neighbour search of our own; the paper only says the
 * real-space sum is local): nc^3 cells of side L/nc >= rmax, nc >= 3, so the
 * 27 cells around a particle's cell are distinct and hold every partner
 * within rmax (minimum image, rmax <= L/3).  head[c] is the first particle
 * of cell c, next[i] the one after i. */
static void orc_real_cells(int n, const double *pos, const double *q, const orc_rs *P, int nc, int nsub,
                           const int32_t *idx, double *Fsub, double *e_real, double *e_lj, double *vir)
{
    double L = P->L, rmax = orc_rmax(P, n);
    int ncell = nc * nc * nc;
    int *head = (int *)malloc(sizeof(int) * ncell);
    int *next = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *cell = (int *)malloc(sizeof(int) * 3 * (n > 0 ? n : 1));
    for (int c = 0; c < ncell; ++c) head[c] = -1;
    for (int i = n - 1; i >= 0; --i) {
        int cc[3];
        for (int a = 0; a < 3; ++a) {
            double s = pos[a * n + i] / L;
            s -= floor(s);
            int k = (int)(s * nc);
            cc[a] = k < 0 ? 0 : (k >= nc ? nc - 1 : k);
            cell[3 * i + a] = cc[a];
        }
        int c = (cc[2] * nc + cc[1]) * nc + cc[0];
        next[i] = head[c];
        head[c] = i;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int t = 0; t < nsub; ++t) {
        int i = idx ? idx[t] : t;
        double f[3] = {0, 0, 0}, ur = 0, ul = 0, w = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int cx = (cell[3 * i] + dx + nc) % nc, cy = (cell[3 * i + 1] + dy + nc) % nc,
                        cz = (cell[3 * i + 2] + dz + nc) % nc;
                    for (int j = head[(cz * nc + cy) * nc + cx]; j >= 0; j = next[j]) {
                        if (j == i) continue;
                        double d[3];
                        orc_min_image(pos, n, i, j, L, d);
                        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                        if (r > rmax) continue;
                        orc_pair(P, q, i, j, d[0], d[1], d[2], r, f, &ur, &ul, &w);
                    }
                }
        Fsub[t] = f[0]; Fsub[nsub + t] = f[1]; Fsub[2 * nsub + t] = f[2];
        if (e_real) e_real[t] = ur;
        if (e_lj) e_lj[t] = ul;
        if (vir) vir[t] = w;
    }
    free(head);
    free(next);
    free(cell);
}

/* Cells per box side for the linked-cell list, or 0 when fewer than three
 * cells of side >= rmax fit (the direct sum is used then). */
static int orc_cells_per_side(const orc_rs *P, int n)
{
    double rmax = orc_rmax(P, n);
    int nc = (int)floor(P->L / rmax);
    if (nc > 256) nc = 256;
    return nc >= 3 ? nc : 0;
}

/* Real-space Coulomb (erfc) plus shifted LJ forces, half pair energies and
 * half pair virials r_ij . F_ij on the particles listed in idx (all
 * particles when idx is NULL, nsub = n).  Every periodic image within the
 * cutoffs counts.  method 0: the O(N^2) direct sum; 1: the linked-cell list
 * (falls back to the direct sum when fewer than three cells fit).  diam is
 * NULL or the per-particle diameters of eq. (4.1).  Fsub is [3][nsub];
 * e_real, e_lj and vir are optional [nsub]. */
void oracle_real_force_ex(int n, const double *pos, const double *q, double L, double alpha, double rc,
                          double coulomb, double lj_eps, double lj_sigma, double lj_rc, const double *diam,
                          int method, int nsub, const int32_t *idx, double *Fsub, double *e_real, double *e_lj,
                          double *vir)
{
    orc_rs P = {L, alpha, rc, coulomb, lj_eps, lj_sigma, lj_rc, diam};
    int nc = method == 1 ? orc_cells_per_side(&P, n) : 0;
    if (nc)
        orc_real_cells(n, pos, q, &P, nc, nsub, idx, Fsub, e_real, e_lj, vir);
    else
        orc_real_direct(n, pos, q, &P, nsub, idx, Fsub, e_real, e_lj, vir);
}

/* The direct sum without diameters (r_off = 0). */
void oracle_real_force(int n, const double *pos, const double *q, double L, double alpha, double rc,
                       double coulomb, double lj_eps, double lj_sigma, double lj_rc,
                       int nsub, const int32_t *idx, double *Fsub, double *e_real, double *e_lj)
{
    oracle_real_force_ex(n, pos, q, L, alpha, rc, coulomb, lj_eps, lj_sigma, lj_rc, NULL, 0, nsub, idx, Fsub,
                         e_real, e_lj, NULL);
}

/* ------------------------------------------------------------------------ */
/* Proposition 1 (Sec. 3.2, eq. 3.10): the exact variance of the random      */
/* batch force of particle i, by a full sum over the enumerated modes        */
/* (weights exp(-k^2/4alpha)); returns E|chi_i|^2 for each listed particle.  */
/* ------------------------------------------------------------------------ */
void oracle_rbe_force_variance(int n, const double *pos, const double *q, double L, double alpha,
                               int p, double coulomb, int nm, const int32_t *modes, const double *weight,
                               int nsub, const int32_t *idx, double *var)
{
    double *re = (double *)malloc(sizeof(double) * nm);
    double *im = (double *)malloc(sizeof(double) * nm);
    oracle_rho(n, pos, q, L, nm, modes, re, im);
    double V = L * L * L;
    double S = oracle_S(alpha, L);
#pragma omp parallel for schedule(static)
    for (int t = 0; t < nsub; ++t) {
        int i = idx[t];
        double second = 0.0, fx = 0, fy = 0, fz = 0;
        for (int l = 0; l < nm; ++l) {
            double kx = 2.0 * ORC_PI * modes[l] / L;
            double ky = 2.0 * ORC_PI * modes[nm + l] / L;
            double kz = 2.0 * ORC_PI * modes[2 * nm + l] / L;
            double k2 = kx * kx + ky * ky + kz * kz;
            double th = orc_phase(modes, nm, l, pos, n, i, L);
            double imag = cos(th) * im[l] - sin(th) * re[l];
            double c4 = 4.0 * ORC_PI * q[i] * coulomb;
            second += c4 * c4 * S / (V * V * k2) * weight[l] * imag * imag;
            double f = weight[l] * c4 / (V * k2) * imag;
            fx -= f * kx; fy -= f * ky; fz -= f * kz;
        }
        var[t] = (second - (fx * fx + fy * fy + fz * fz)) / (double)p;
    }
    free(re);
    free(im);
}

/* ------------------------------------------------------------------------ */
/* Langevin dynamics (Sec. 3.2 theorem statement and Sec. 3.3):              */
/*   dr = v dt,  m dv = (F - gamma v) dt + sqrt(2 gamma kT) dW.              */
/* The paper gives only the SDE; the discretisation read here is BAOAB       */
/* (Leimkuhler & Matthews 2013): half kick, half drift, exact Ornstein-      */
/* Uhlenbeck velocity update, half drift, new force, half kick.              */
/* ------------------------------------------------------------------------ */

/* Three standard normals for particle i at step `step`: one Philox block
 * (i, TAG_LANGEVIN, step) gives four 32-bit words; Box-Muller on
 * u1 = (w0 + 1) 2^-32 in (0,1], u2 = w1 2^-32 gives the first two, and on
 * u1' = (w2 + 1) 2^-32, u2' = w3 2^-32 the cosine branch gives the third. */
void oracle_langevin_normals(uint64_t seed, uint64_t step, int i, double xi[3])
{
    uint32_t r[4];
    orc_draw((uint32_t)i, ORC_TAG_LANGEVIN, seed, step, r);
    double u1 = ((double)r[0] + 1.0) * (1.0 / 4294967296.0);
    double u2 = (double)r[1] * (1.0 / 4294967296.0);
    double u3 = ((double)r[2] + 1.0) * (1.0 / 4294967296.0);
    double u4 = (double)r[3] * (1.0 / 4294967296.0);
    double a = sqrt(-2.0 * log(u1)), b = sqrt(-2.0 * log(u3));
    xi[0] = a * cos(2.0 * ORC_PI * u2);
    xi[1] = a * sin(2.0 * ORC_PI * u2);
    xi[2] = b * cos(2.0 * ORC_PI * u4);
}

/* Parameters of one oracle MD system. */
typedef struct {
    int n, p;
    double L, alpha, rc, coulomb;
    double lj_eps, lj_sigma, lj_rc;
    double kT, gamma, dt, mass;
    uint64_t seed;
    const double *diam;   /* per-particle diameters of eq. (4.1), or NULL */
    int n_fixed;          /* particles 0 .. n_fixed-1 do not move (e.g. the colloid of Sec. 4.2) */
} oracle_sys;

/* Total force used inside the MD loop: random batch Fourier part with the
 * modes of sample index `step` (Algorithm 1: a fresh batch every step), plus
 * the real-space erfc and LJ parts.  Positions are wrapped into [0, L). */
void oracle_total_force(const oracle_sys *s, const double *pos, const double *q, uint64_t step, double *F)
{
    int n = s->n, p = s->p;
    int32_t *modes = (int32_t *)malloc(sizeof(int32_t) * 3 * p);
    double *w = (double *)malloc(sizeof(double) * p);
    double *Fr = (double *)malloc(sizeof(double) * 3 * n);
    oracle_sample_modes(s->alpha, s->L, p, s->seed, step, modes);
    oracle_rbe_weights(s->alpha, s->L, p, w);
    oracle_kspace_force(n, pos, q, s->L, p, modes, w, s->coulomb, F);
    oracle_real_force_ex(n, pos, q, s->L, s->alpha, s->rc, s->coulomb, s->lj_eps, s->lj_sigma, s->lj_rc, s->diam,
                         1, n, NULL, Fr, NULL, NULL, NULL);
    for (int k = 0; k < 3 * n; ++k) F[k] += Fr[k];
    free(modes); free(w); free(Fr);
}

/* One BAOAB step (steps numbered by `step`).  On entry F = F(pos); on exit
 * pos, vel and F are advanced, with F(pos_new) computed using the mode sample
 * and the noise of index `step`. */
void oracle_baoab_step(const oracle_sys *s, double *pos, double *vel, const double *q, double *F, uint64_t step)
{
    int n = s->n;
    double h = 0.5 * s->dt;
    double c1 = exp(-s->gamma * s->dt / s->mass);
    double c2 = sqrt((1.0 - c1 * c1) * s->kT / s->mass);
    for (int i = s->n_fixed; i < n; ++i) {
        double xi[3];
        oracle_langevin_normals(s->seed, step, i, xi);
        for (int d = 0; d < 3; ++d) {
            double v = vel[d * n + i] + h * F[d * n + i] / s->mass; /* B */
            double r = pos[d * n + i] + h * v;                      /* A */
            v = c1 * v + c2 * xi[d];                                /* O */
            r += h * v;                                             /* A */
            r -= s->L * floor(r / s->L);                            /* wrap into [0, L) */
            if (r >= s->L) r -= s->L;
            pos[d * n + i] = r;
            vel[d * n + i] = v;
        }
    }
    oracle_total_force(s, pos, q, step, F);
    for (int d = 0; d < 3; ++d)
        for (int i = s->n_fixed; i < n; ++i) vel[d * n + i] += h * F[d * n + i] / s->mass; /* B */
}

/* Andersen thermostat with the leapfrog scheme (Sec. 3.1, loop body (1)-(3)):
 * v^{n+1/2} = v^{n-1/2} + F^n dt / m; r^{n+1} = r^n + v^{n+1/2} dt; then each
 * particle's velocity is redrawn from N(0, kT/m) with probability nu*dt.
 * On entry F = F(pos) with sample index step; on exit F = F(pos_new) with
 * sample index step+1.  Collision test: u = w0 2^-32 of block
 * (i, TAG_ANDERSEN, step) compared with nu*dt; the new velocity uses the three
 * Langevin normals of (i, step). */
void oracle_leapfrog_andersen_step(const oracle_sys *s, double nu, double *pos, double *vel, const double *q,
                                   double *F, uint64_t step)
{
    int n = s->n;
    double dt = s->dt;
    for (int i = s->n_fixed; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            double v = vel[d * n + i] + dt * F[d * n + i] / s->mass;
            double r = pos[d * n + i] + dt * v;
            r -= s->L * floor(r / s->L);
            if (r >= s->L) r -= s->L;
            pos[d * n + i] = r;
            vel[d * n + i] = v;
        }
        uint32_t w[4];
        orc_draw((uint32_t)i, ORC_TAG_ANDERSEN, s->seed, step, w);
        double u = (double)w[0] * (1.0 / 4294967296.0);
        if (u < nu * dt) {
            double xi[3];
            oracle_langevin_normals(s->seed, step, i, xi);
            for (int d = 0; d < 3; ++d) vel[d * n + i] = sqrt(s->kT / s->mass) * xi[d];
        }
    }
    oracle_total_force(s, pos, q, step + 1, F);
}

/* ------------------------------------------------------------------------ */
/* Adjoint (vector-Jacobian product) of the forces at a fixed mode sample.   */
/* Given G_i = dLoss/dF_i and gE = dLoss/dU, returns dLoss/dq_i and          */
/* dLoss/dr_i.  Derived from eqs. (2.6), (2.7), (2.11), (3.6) and (4.1):     */
/*                                                                           */
/* Fourier part, with W_l = weight_l 4 pi coulomb/(V k_l^2),                 */
/*   w_il = W_l G_i.k_l,  A_l = sum_i q_i w_il cos th_il,                    */
/*   B_l = sum_i q_i w_il sin th_il,                                         */
/*   dq_i = -sum_l w_il (cos th_il S_l - sin th_il C_l)                      */
/*          - sum_l (A_l sin th_il - B_l cos th_il),                         */
/*   dr_i = q_i sum_l k_l [w_il (sin th S + cos th C) - A_l cos th - B_l sin th]*/
/* where rho_l = C_l + i S_l.  Energy part: dU/dq_i =                        */
/*   sum_l W_l (C_l cos th_il + S_l sin th_il) - 2 coulomb sqrt(alpha/pi) q_i */
/*   + real-space potential;  dU/dr_i = -F_i.                                */
/*                                                                           */
/* Real part: the pair force on i is phi(r) d with d = r_j - r_i,            */
/*   phi = -coulomb q_i q_j G(r)/r + V_LJ'(r)/r, so                          */
/*   dq_i = -coulomb sum_j q_j (G/r)(G_i - G_j).d,                           */
/*   dr_i = sum_j [ -(phi'(r)/r)((G_i - G_j).d) d - phi (G_i - G_j) ].       */
/* ------------------------------------------------------------------------ */
void oracle_forces_vjp(int n, const double *pos, const double *q, double L, double alpha, double rc,
                       double coulomb, double lj_eps, double lj_sigma, double lj_rc,
                       int nm, const int32_t *modes, const double *weight,
                       const double *gF, double gE, int parts, double *gq, double *gr)
{
    double V = L * L * L;
    memset(gq, 0, sizeof(double) * n);
    memset(gr, 0, sizeof(double) * 3 * n);
    if (parts & 1) {
        double *re = (double *)malloc(sizeof(double) * nm);
        double *im = (double *)malloc(sizeof(double) * nm);
        double *A = (double *)calloc(nm, sizeof(double));
        double *B = (double *)calloc(nm, sizeof(double));
        oracle_rho(n, pos, q, L, nm, modes, re, im);
#pragma omp parallel for schedule(static)
        for (int l = 0; l < nm; ++l) {
            double kx = 2.0 * ORC_PI * modes[l] / L, ky = 2.0 * ORC_PI * modes[nm + l] / L,
                   kz = 2.0 * ORC_PI * modes[2 * nm + l] / L;
            double Wl = weight[l] * 4.0 * ORC_PI * coulomb / (V * (kx * kx + ky * ky + kz * kz));
            double a = 0, b = 0;
            for (int i = 0; i < n; ++i) {
                double th = orc_phase(modes, nm, l, pos, n, i, L);
                double w = Wl * (gF[i] * kx + gF[n + i] * ky + gF[2 * n + i] * kz);
                a += q[i] * w * cos(th);
                b += q[i] * w * sin(th);
            }
            A[l] = a;
            B[l] = b;
        }
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double dq = 0, rx = 0, ry = 0, rz = 0;
            for (int l = 0; l < nm; ++l) {
                double kx = 2.0 * ORC_PI * modes[l] / L, ky = 2.0 * ORC_PI * modes[nm + l] / L,
                       kz = 2.0 * ORC_PI * modes[2 * nm + l] / L;
                double Wl = weight[l] * 4.0 * ORC_PI * coulomb / (V * (kx * kx + ky * ky + kz * kz));
                double th = orc_phase(modes, nm, l, pos, n, i, L);
                double c = cos(th), s = sin(th);
                double w = Wl * (gF[i] * kx + gF[n + i] * ky + gF[2 * n + i] * kz);
                dq += -w * (c * im[l] - s * re[l]) - (A[l] * s - B[l] * c);
                dq += gE * Wl * (re[l] * c + im[l] * s);
                double t = w * (s * im[l] + c * re[l]) - A[l] * c - B[l] * s;
                rx += kx * t; ry += ky * t; rz += kz * t;
            }
            gq[i] += dq - gE * 2.0 * coulomb * sqrt(alpha / ORC_PI) * q[i];
            gr[i] += q[i] * rx;
            gr[n + i] += q[i] * ry;
            gr[2 * n + i] += q[i] * rz;
        }
        free(re); free(im); free(A); free(B);
    }
    if (parts & 2) {
        double rmax = rc > lj_rc ? rc : lj_rc;
        int nimg = rmax < 0.5 * L ? 0 : (int)ceil(rmax / L) + 1;
        double b = sqrt(alpha), sp = sqrt(ORC_PI);
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n; ++i) {
            double dq = 0, rx = 0, ry = 0, rz = 0;
            for (int j = 0; j < n; ++j) {
                double dx0 = pos[j] - pos[i], dy0 = pos[n + j] - pos[n + i], dz0 = pos[2 * n + j] - pos[2 * n + i];
                dx0 -= L * floor(dx0 / L + 0.5);
                dy0 -= L * floor(dy0 / L + 0.5);
                dz0 -= L * floor(dz0 / L + 0.5);
                double Gx = gF[i] - gF[j], Gy = gF[n + i] - gF[n + j], Gz = gF[2 * n + i] - gF[2 * n + j];
                for (int a = -nimg; a <= nimg; ++a)
                    for (int bb = -nimg; bb <= nimg; ++bb)
                        for (int c = -nimg; c <= nimg; ++c) {
                            if (j == i && a == 0 && bb == 0 && c == 0) continue;
                            double dx = dx0 + a * L, dy = dy0 + bb * L, dz = dz0 + c * L;
                            double r = sqrt(dx * dx + dy * dy + dz * dz);
                            double phi = 0.0, dphi = 0.0; /* phi(r) and phi'(r) */
                            if (r <= rc) {
                                double e = exp(-alpha * r * r), ec = erfc(b * r);
                                double g = ec / (r * r * r) + 2.0 * b * e / (sp * r * r); /* G/r */
                                double dg = -3.0 * ec / (r * r * r * r) - 6.0 * b * e / (sp * r * r * r) -
                                            4.0 * b * b * b * e / (sp * r);
                                phi += -coulomb * q[i] * q[j] * g;
                                dphi += -coulomb * q[i] * q[j] * dg;
                                double GD = Gx * dx + Gy * dy + Gz * dz;
                                dq += -coulomb * q[j] * g * GD;
                                dq += gE * coulomb * q[j] * ec / r;
                            }
                            if (lj_eps != 0.0 && r < lj_rc) {
                                double sr6 = pow(lj_sigma / r, 6.0), sr12 = sr6 * sr6;
                                /* V'(r)/r and its derivative in r */
                                double vr = 4.0 * lj_eps * (-12.0 * sr12 + 6.0 * sr6) / (r * r);
                                double dvr = 4.0 * lj_eps * (168.0 * sr12 - 48.0 * sr6) / (r * r * r);
                                phi += vr;
                                dphi += dvr;
                            }
                            if (phi != 0.0 || dphi != 0.0) {
                                double GD = Gx * dx + Gy * dy + Gz * dz;
                                rx += -(dphi / r) * GD * dx - phi * Gx;
                                ry += -(dphi / r) * GD * dy - phi * Gy;
                                rz += -(dphi / r) * GD * dz - phi * Gz;
                            }
                        }
            }
            gq[i] += dq;
            gr[i] += rx;
            gr[n + i] += ry;
            gr[2 * n + i] += rz;
        }
    }
    /* dU/dr = -F contributes -gE * F: added by the caller's force, see tests */
}

/* Kinetic energy sum_i m |v_i|^2 / 2. */
double oracle_kinetic_energy(int n, const double *vel, double mass)
{
    double e = 0.0;
    for (int k = 0; k < 3 * n; ++k) e += 0.5 * mass * vel[k] * vel[k];
    return e;
}

/* ------------------------------------------------------------------------ */
/* Observables of Sec. 4.1 (eq. 4.3): the pair virial and its Fourier part,  */
/* and pair-distance counts for the charge-charge correlation.               */
/* ------------------------------------------------------------------------ */

/* Sum over unordered pairs (all periodic images within the cutoffs) of
 * r_ij . F_ij with r_ij = r_j - r_i and F_ij the force of j on i, for the
 * real-space Coulomb part (returned in *w_real) and the shifted LJ part
 * (*w_lj).  Eq. (4.3) uses half of this sum. */
void oracle_pair_virial(int n, const double *pos, const double *q, double L, double alpha, double rc,
                        double coulomb, double lj_eps, double lj_sigma, double lj_rc, double *w_real, double *w_lj)
{
    double rmax = rc > lj_rc ? rc : lj_rc;
    int nimg = rmax < 0.5 * L ? 0 : (int)ceil(rmax / L) + 1;
    double wr = 0.0, wl = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double dx0 = pos[j] - pos[i], dy0 = pos[n + j] - pos[n + i], dz0 = pos[2 * n + j] - pos[2 * n + i];
            dx0 -= L * floor(dx0 / L + 0.5);
            dy0 -= L * floor(dy0 / L + 0.5);
            dz0 -= L * floor(dz0 / L + 0.5);
            for (int a = -nimg; a <= nimg; ++a)
                for (int b = -nimg; b <= nimg; ++b)
                    for (int c = -nimg; c <= nimg; ++c) {
                        if (j == i && a == 0 && b == 0 && c == 0) continue;
                        double dx = dx0 + a * L, dy = dy0 + b * L, dz = dz0 + c * L;
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        /* F_ij = -coulomb q_i q_j G(r) r_ij / r, so r_ij . F_ij = -coulomb q_i q_j G(r) r */
                        if (r <= rc) wr += 0.5 * (-coulomb * q[i] * q[j] * orc_G(r, alpha) * r);
                        if (lj_eps != 0.0 && r < lj_rc) {
                            double V, dV;
                            orc_lj(r, 0.0, lj_eps, lj_sigma, lj_rc, &V, &dV);
                            /* F_ij = dV/dr r_ij / r: r_ij . F_ij = r dV/dr */
                            wl += 0.5 * r * dV;
                        }
                    }
        }
    *w_real = wr;
    *w_lj = wl;
}

/* Fourier part of the same sum for the mode list with weights w_l: each mode
 * contributes e_l (2 pi^2 |m|^2 / (alpha L^2) - 1), where e_l is its energy
 * term coulomb w_l |rho_l|^2 / (2 pi L |m|^2) (the volume derivative of
 * eq. 2.6's Fourier sum at fixed scaled positions, in the sign convention of
 * the pair sum above). */
double oracle_kspace_virial(int n, const double *pos, const double *q, double L, double alpha, int nm,
                            const int32_t *modes, const double *weight, double coulomb)
{
    double *re = (double *)malloc(sizeof(double) * nm);
    double *im = (double *)malloc(sizeof(double) * nm);
    oracle_rho(n, pos, q, L, nm, modes, re, im);
    double w = 0.0;
    for (int l = 0; l < nm; ++l) {
        double m2 = (double)modes[l] * modes[l] + (double)modes[nm + l] * modes[nm + l] +
                    (double)modes[2 * nm + l] * modes[2 * nm + l];
        double e = coulomb * weight[l] * (re[l] * re[l] + im[l] * im[l]) / (2.0 * ORC_PI * L * m2);
        w += e * (2.0 * ORC_PI * ORC_PI * m2 / (alpha * L * L) - 1.0);
    }
    free(re);
    free(im);
    return w;
}

/* Counts of unordered pairs i < j (minimum image, r_max <= L/2) by distance
 * bin of width dr = r_max / nbins and by charge class: 0 both q > 0, 1 one
 * of each, 2 both q <= 0.  counts is [3][nbins], added to.  A pair at
 * distance r < r_max falls in bin floor(r / dr) (the definition of a
 * histogram of g(r), Sec. 4.1), with r = sqrt(dx^2 + dy^2 + dz^2) from the
 * minimum-image displacement, every operation rounded on its own. */
void oracle_pair_histogram(int n, const double *pos, const double *q, double L, double r_max, int nbins,
                           int64_t *counts)
{
    double dr = r_max / nbins;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double dx = pos[j] - pos[i], dy = pos[n + j] - pos[n + i], dz = pos[2 * n + j] - pos[2 * n + i];
            dx = dx - L * rint(dx / L);
            dy = dy - L * rint(dy / L);
            dz = dz - L * rint(dz / L);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (!(r < r_max)) continue;
            int b = (int)floor(r / dr);
            if (b >= nbins) continue;
            int cls = 2 - ((q[i] > 0.0) + (q[j] > 0.0));
            counts[(int64_t)cls * nbins + b] += 1;
        }
}

/* Threads of the OpenMP loops (for timing the oracle single-threaded and
 * with every core); returns the count in effect afterwards. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
