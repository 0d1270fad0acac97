/*
 * rbe.h -- C ABI of librbe, an MI355X (gfx950) implementation of the random
 * batch Ewald (RBE) method of Jin, Li, Xu & Zhao, "A random batch Ewald
 * method for particle systems with Coulomb interactions" (arXiv:2010.01559).
 *
 * Problem statement (paper Sec. 2, eqs. 2.1-2.3 and 2.11): N point charges
 * q_i at positions r_i in a cubic periodic box of side L, sum q_i = 0, with
 * Coulomb potential coulomb * q_i q_j / r (reduced units, Sec. 4.1; `coulomb`
 * is the Bjerrum length of Sec. 4.2, 1 otherwise).  The force splits into a
 * Fourier part (eq. 2.11, first term) -- estimated by the random batch of P
 * modes drawn from exp(-k^2/4 alpha) (Sec. 3.1, eqs. 3.3 and 3.6) -- and an
 * exact real-space erfc part inside r_cut (eq. 2.11, second term), plus an
 * optional shifted Lennard-Jones repulsion (eq. 4.1; r_off = 0 unless
 * per-particle diameters are given, then r_off = (d_i + d_j)/2 - sigma).
 *
 * Conventions shared by every entry point:
 *   - Arrays are device memory owned by the caller, contiguous, SoA:
 *     positions/velocities/forces/gradients are [3][N_tot] (x block, then y,
 *     then z), charges are [N_tot].  Element type is float for RBE_FP32 and
 *     double for RBE_FP64.  For a batch of R systems the particles of system
 *     r occupy [off_r, off_r + n_r) inside each block, in creation order.
 *   - Modes are integer vectors m with k = 2 pi m / L (Sec. 2), stored
 *     [3][M_tot] int32 with system r's p_r modes at [moff_r, moff_r + p_r).
 *   - All calls are asynchronous on the stream given at creation, except
 *     rbe_create*, rbe_destroy, rbe_energy and rbe_get_rho, which synchronise.
 *   - Hot calls (sample, forces, step, vjp) never allocate: every workspace
 *     is sized at creation.
 *   - Functions return an rbe_status and never abort; rbe_last_error gives
 *     the message.  Argument validation happens on the host before any
 *     device work is enqueued, so an error return leaves the stream
 *     untouched.
 *   - Positions may lie outside [0, L); they are wrapped periodically.
 */
#ifndef RBE_H
#define RBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbe_ctx rbe_ctx;

typedef enum rbe_status {
    RBE_OK = 0,
    RBE_ERR_INVALID = -1,      /* bad argument or parameter */
    RBE_ERR_NOT_NEUTRAL = -2,  /* |sum q| > 1e-6 sum |q| (eq. 2.1) */
    RBE_ERR_CUTOFF = -3,       /* r_cut or the LJ cutoff exceeds L/2 */
    RBE_ERR_OOM = -4,          /* device allocation failed at creation */
    RBE_ERR_HIP = -5,          /* a HIP runtime call failed */
    RBE_ERR_NONFINITE = -6,    /* non-finite value seen by a kernel, or (single precision) a
                                  real-space force of 2^20 or more, beyond which the exact
                                  fixed-point pair sums lose exactness (overlapping particles) */
    RBE_ERR_STATE = -7,        /* call not valid in the current state */
    RBE_ERR_NO_DEVICE = -8,    /* no usable gfx950 device */
    RBE_ERR_TIMEOUT = -9       /* a bounded device-side wait of a neighbour-list rebuild gave
                                  up (or a rebuild index fell outside its system): the forces
                                  of the steps since the last check are not valid; the
                                  library repairs its cell state and the next step rebuilds */
} rbe_status;

enum { RBE_FP32 = 0, RBE_FP64 = 1 };

/* Integrator for rbe_step. */
enum { RBE_LANGEVIN_BAOAB = 0, RBE_LEAPFROG_ANDERSEN = 1 };

/* Mode sampler. */
enum { RBE_SAMPLER_EXACT = 0, RBE_SAMPLER_MH = 1, RBE_SAMPLER_FIXED = 2 };

/* Parts selector for rbe_forces_vjp. */
enum { RBE_PART_KSPACE = 1, RBE_PART_REAL = 2, RBE_PART_ALL = 3 };

/* Parameters of one system (paper notation in brackets). */
typedef struct rbe_params {
    int32_t n;           /* particles [N], >= 1 */
    int32_t p;           /* batch size [p], >= 1 (Sec. 3.1) */
    double box;          /* box side [L] > 0 */
    double alpha;        /* Ewald splitting [alpha] > 0 (Sec. 2) */
    double r_cut;        /* real-space cutoff [r_c], 0 < r_cut <= L/2 (eq. 2.8) */
    double coulomb;      /* Coulomb prefactor: 1 (Sec. 4.1) or l_B (Sec. 4.2) */
    double lj_eps;       /* shifted LJ [epsilon] (eq. 4.1); 0 disables LJ */
    double lj_sigma;     /* [sigma] */
    double lj_rcut;      /* LJ cutoff [R_c] on r - r_off; the largest pair reach
                            r_off + R_c must not exceed L/2 when LJ is on */
    double kT;           /* bath temperature [T], k_B = 1 (Sec. 3.3) */
    double gamma;        /* Langevin friction [gamma] (Sec. 3.3) */
    double dt;           /* time step [Delta t] */
    double mass;         /* particle mass [m_i], equal for all particles */
    double nu;           /* Andersen collision frequency [nu] (Sec. 3.3) */
    double skin;         /* neighbour-list skin for rbe_step, >= 0.  With skin > 0 the
                            real-space pass of a step reads a list of the pairs within
                            max(r_cut, lj_rcut) + skin, rebuilt on the device whenever a
                            particle has moved more than skin/2 since the last build; the
                            cell side is at least cutoff + skin.  0 rebuilds the cell
                            list at every step.  Either way every pair inside the
                            cutoffs is counted exactly once (no effect on the result
                            beyond summation order). */
    uint64_t seed;       /* key of the counter-based generator */
    int32_t precision;   /* RBE_FP32 or RBE_FP64 (all systems of a batch alike) */
    int32_t integrator;  /* RBE_LANGEVIN_BAOAB or RBE_LEAPFROG_ANDERSEN */
    int32_t sampler;     /* RBE_SAMPLER_EXACT, RBE_SAMPLER_MH, or RBE_SAMPLER_FIXED: rbe_step keeps
                            the active list of rbe_set_k / rbe_sample_k every step instead of drawing
                            a new batch (with the classical Ewald list of rbe_set_k: Ewald dynamics on
                            the same kernels); single-system contexts only */
    int32_t flags;       /* reserved, 0 */
    int32_t n_fixed;     /* particles 0 .. n_fixed-1 of the system never move (the fixed
                            colloid of Sec. 4.2): no kicks, drifts, noise or collisions;
                            0 <= n_fixed <= n */
    int32_t reserved;    /* 0 */
    const double *diameter; /* host [n] diameters d_i of eq. (4.1), read only during creation,
                            or NULL (every d_i = sigma, so r_off = 0).  With diameters the
                            LJ term acts for r - r_off < R_c with r_off = (d_i + d_j)/2 - sigma;
                            rbe_forces_vjp then refuses the real-space part (RBE_ERR_STATE) */
} rbe_params;

/* Energies of one system (all double, host memory). */
typedef struct rbe_energy_t {
    double e_kspace;   /* random batch estimate of the Fourier sum (eq. 2.6 without
                          the self term) on the active modes */
    double e_self;     /* -coulomb sqrt(alpha/pi) sum q_i^2 (eq. 2.6) */
    double e_real;     /* truncated real-space erfc sum (eq. 2.9, third term) */
    double e_lj;       /* shifted LJ energy (eq. 4.1) */
    double e_kin;      /* sum m |v_i|^2 / 2 (0 when vel is NULL) */
    double virial;     /* sum over real-space and LJ pairs of r_ij . F_ij (pair part of eq. 4.3) */
    double virial_kspace; /* Fourier part of the same sum on the active modes: sum over modes of
                          e_l (2 pi^2 |m_l|^2 / (alpha L^2) - 1), e_l the mode's term of e_kspace
                          (scaling derivative of the Fourier sum); eq. 4.3 uses
                          vir = (virial + virial_kspace) / 2 */
    double charge_sum; /* sum q_i, for the neutrality check */
    int32_t nonfinite; /* non-zero if any kernel met a non-finite force (or a single-precision
                          real-space force of 2^20 or more) since the last check */
    int32_t timeout;   /* non-zero if a list rebuild's bounded wait gave up since the last check */
} rbe_energy_t;

/* Tile shapes of the kernels; 0 fields mean "library default". */
typedef struct rbe_tiles {
    int32_t rho_chunk;     /* particles staged per structure-factor block (<= 2048) */
    int32_t rho_block;     /* threads per structure-factor block: 256, 512 or 1024 */
    int32_t force_split;   /* waves sharing one particle in the force pass: 1, 2 or 4 */
    int32_t real_split;    /* lanes per particle in the neighbour-list pass of rbe_step: 1, 2, 4 or 8 */
} rbe_tiles;

/* Normaliser of the importance distribution (Sec. 3.1, eqs. 3.1-3.2):
 * H = sum_m exp(-pi^2 m^2/(alpha L^2)) and S = H^3 - 1.  Host only; needs no
 * device.  Returns RBE_ERR_INVALID for non-positive or non-finite inputs. */
rbe_status rbe_normalizer(double alpha, double box, double *H, double *S);

/* Create a context for one system.  stream is a hipStream_t (NULL = default
 * stream).  Validates params (RBE_ERR_INVALID / RBE_ERR_CUTOFF), selects the
 * current HIP device, allocates every workspace.  On failure *out is NULL
 * and rbe_last_error(NULL) describes the failure. */
rbe_status rbe_create(const rbe_params *params, void *stream, rbe_ctx **out);

/* Create a context for R independent systems (each with its own N, L, alpha,
 * P, seed ...) that every call processes together in single launches.
 * params is [R]; precision must agree. */
rbe_status rbe_batch_create(const rbe_params *params, int32_t R, void *stream, rbe_ctx **out);

/* Release the context and its device memory.  NULL is ignored. */
void rbe_destroy(rbe_ctx *ctx);

/* Message of the last failed call on ctx, or of the last failed creation on
 * this thread when ctx is NULL.  Never NULL. */
const char *rbe_last_error(const rbe_ctx *ctx);

/* Number of systems, total particles and total modes of the context. */
int32_t rbe_num_systems(const rbe_ctx *ctx);
int64_t rbe_num_particles(const rbe_ctx *ctx);
int32_t rbe_num_modes(const rbe_ctx *ctx);

/* Draw a fresh batch of p modes per system from P_k (Sec. 3.1, eq. 3.3;
 * "renew the batch at every time step"), keyed by (seed, step), and make it
 * the active batch with weights S/p (eq. 3.6).  The exact sampler inverts
 * the 1-D cumulative table of eq. (3.4) per component and redraws the zero
 * vector; the MH sampler follows the paper's Metropolis-Hastings recipe
 * (eq. 3.5) with chains that persist in the context.  modes_out, if not
 * NULL, is device memory [3][M_tot] int32 that receives the modes.  With
 * the exact sampler and no modes_out the draw is recorded and made by the
 * next launch that needs the modes (the structure-factor pass of the next
 * force, energy or adjoint call draws them itself); the modes are the same
 * either way. */
rbe_status rbe_sample_k(rbe_ctx *ctx, uint64_t step, int32_t *modes_out);

/* Make an explicit mode list active for a single-system context: modes is
 * host [3][nm] int32 (no zero vector), weights host [nm] or NULL.  NULL
 * weights mean the random batch weight S/nm; explicit weights w_l turn the
 * Fourier pass into sum_l w_l (4 pi k_l q_i/(V k_l^2)) Im(...) -- with
 * w_l = exp(-k_l^2/4 alpha) over all 0 < |m| <= m_c it is the classical
 * Ewald sum (eq. 2.11).  nm must not exceed the capacity fixed at creation
 * (max(p, 1) unless rbe_reserve_modes raised it). */
rbe_status rbe_set_k(rbe_ctx *ctx, const int32_t *modes, int32_t nm, const double *weights);

/* Classical Ewald comparator (eq. 2.9, second term, with the Fourier sum
 * truncated to 0 < |m|^2 <= mmax2, m = k L / (2 pi) integer).
 * rbe_ewald_radius2: the largest mmax2 whose Gaussian factor
 * exp(-pi^2 |m|^2 / (alpha L^2)) = exp(-k^2/4 alpha) is still >= tol, tol in
 * (0, 1).  rbe_ewald_modes: every such mode, m_x outermost and m_z innermost
 * from -floor(sqrt(mmax2)) up, with its weight exp(-k^2/4 alpha); modes is
 * host [3][cap] int32 (row stride cap), weights host [cap]; with both NULL
 * only *nm is written (the count), else cap must hold *nm.  Both host only
 * (no device); errors in rbe_last_error(NULL).  rbe_set_k_ewald: that list
 * made active on a single-system context with the context's alpha and L
 * (rbe_set_k with these weights; raises the mode capacity when needed, which
 * allocates: not a hot call); *nm_out (may be NULL) gets the count. */
rbe_status rbe_ewald_radius2(double alpha, double box, double tol, int32_t *mmax2);
rbe_status rbe_ewald_modes(double alpha, double box, int32_t mmax2, int32_t *modes, double *weights, int32_t cap,
                           int32_t *nm);
rbe_status rbe_set_k_ewald(rbe_ctx *ctx, int32_t mmax2, int32_t *nm_out);

/* Raise the mode capacity of a single-system context to cap (allocates;
 * not a hot call). */
rbe_status rbe_reserve_modes(rbe_ctx *ctx, int32_t cap);

/* Fourier-space force on every particle with the active modes (eq. 3.6):
 *   F_i = -coulomb * sum_l w_l (4 pi q_i k_l / (V k_l^2)) Im(exp(-i k_l.r_i) rho(k_l)),
 * rho(k) = sum_j q_j exp(i k.r_j) (eq. 2.7).  force is overwritten, or added
 * to when accumulate != 0.  The structure factors are kept for rbe_get_rho,
 * rbe_energy and rbe_forces_vjp. */
rbe_status rbe_kspace_forces(rbe_ctx *ctx, const void *pos, const void *q, void *force, int32_t accumulate);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * Fourier-space force of rbe_kspace_forces for one system described by
 * params (n, p, box, alpha, coulomb, precision; other fields ignored) and
 * the caller's modes (device [3][p] int32, no zero vector), each with the
 * random batch weight S/p, enqueued on `stream` (a hipStream_t, NULL = the
 * default stream) without a context.  pos [3][n], q [n] and force [3][n]
 * are the caller's device arrays in the precision of params; force is
 * overwritten or accumulated.  Same kernels as a context, with the built-in
 * tile shapes (never the tile cache): rho_chunk = ceil(n/256) rounded up to a
 * multiple of 8 and clamped to [64, 512], rho_block 1024, force_split 4 (2
 * for n >= 500000); the result equals rbe_set_k + rbe_kspace_forces of a
 * context on those shapes bit for bit.
 * The workspace is a fixed device array inside the library, one per GPU,
 * held until the process ends (about 17 MB); calls never allocate.  Limits:
 * n <= 2^20, p <= 512 (RBE_ERR_INVALID beyond, with the limit in the
 * message of rbe_last_error(NULL)).  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (concurrent streams or threads) race
 * and must be ordered by the caller.  Non-finite forces are not reported
 * (there is no context to hold the state). */
rbe_status rbe_kspace_forces_noalloc(const rbe_params *params, const int32_t *modes, const void *pos,
                                     const void *q, void *force, int32_t accumulate, void *stream);

/* Real-space force (eq. 2.11, second term, pairs with |r_ij + nL| <= r_cut,
 * minimum image) plus shifted LJ (eq. 4.1), on a cell list built on the fly
 * (all pairs when fewer than 3 cells fit along the box).  force is
 * overwritten or accumulated. */
rbe_status rbe_real_forces(rbe_ctx *ctx, const void *pos, const void *q, void *force, int32_t accumulate);

/* Advance nsteps time steps (Algorithm 1 of the paper).  Step s = first_step
 * + t draws its modes and noise with index s.  RBE_LANGEVIN_BAOAB: half
 * kick, half drift, exact Ornstein-Uhlenbeck velocity update, half drift,
 * force, half kick (the Langevin equation of Sec. 3.3).  On entry force must
 * hold F(pos) (e.g. from rbe_kspace_forces + rbe_real_forces); on exit pos,
 * vel, force hold the new state, positions wrapped into [0, L).
 * RBE_LEAPFROG_ANDERSEN: the leapfrog + Andersen loop of Sec. 3.1 with vel
 * the half-step velocity; the force computed at the end of step s uses the
 * modes of index s + 1.  With RBE_SAMPLER_FIXED no modes are drawn: every
 * step uses the active list (RBE_ERR_STATE if there is none).  The time step
 * is dt, or the schedule set by rbe_set_dt.  Results do not depend on how a
 * run is split into calls (bit for bit in FP32).  Asynchronous; no
 * allocation. */
rbe_status rbe_step(rbe_ctx *ctx, void *pos, void *vel, const void *q, void *force, uint64_t first_step,
                    int32_t nsteps);

/* Same as rbe_step; the name used for multi-system contexts. */
rbe_status rbe_batch_step(rbe_ctx *ctx, void *pos, void *vel, const void *q, void *force, uint64_t first_step,
                          int32_t nsteps);

/* Energies of every system with the active modes (Sec. 2, eqs. 2.6 and 2.9;
 * Sec. 4.1, eqs. 4.1 and 4.3).  vel may be NULL.  out is host [R].
 * Synchronises the stream.  Returns RBE_ERR_NOT_NEUTRAL if some system has
 * |sum q| > 1e-6 sum |q| (energies are still filled in), RBE_ERR_NONFINITE if
 * a kernel met a non-finite force, RBE_ERR_TIMEOUT if a list rebuild gave up,
 * since the previous check (see rbe_check). */
rbe_status rbe_energy(rbe_ctx *ctx, const void *pos, const void *q, const void *vel, rbe_energy_t *out);

/* Pending device-side errors since the previous check (by this call, rbe_energy or
 * rbe_list_builds): RBE_ERR_NONFINITE if a kernel met a non-finite force or
 * (single precision) a real-space force of 2^20 or more, RBE_ERR_TIMEOUT if a list rebuild's bounded wait gave up (then the cell
 * state is cleared and the next step rebuilds from scratch), else RBE_OK.
 * Clears what it reports.  Synchronises the stream.  Time steps are
 * asynchronous and cannot return these errors themselves. */
rbe_status rbe_check(rbe_ctx *ctx);

/* Bound on the spin iterations of each device-side wait inside a list
 * rebuild (default 2^24, far beyond any real wait).  Every wait ends: a wait
 * that reaches the bound gives up, raises RBE_ERR_TIMEOUT for the next
 * check and leaves the step's forces invalid; 0 makes every wait give up at
 * once, which exercises that path without any kernel hanging or faulting.
 * RBE_ERR_INVALID for a negative bound.  Synchronises the stream. */
rbe_status rbe_set_wait_limit(rbe_ctx *ctx, int32_t limit);

/* Structure factors of the last Fourier evaluation: host [M_tot][2] double
 * (real, imaginary).  Synchronises the stream. */
rbe_status rbe_get_rho(rbe_ctx *ctx, double *rho);

/* Vector-Jacobian product of the forces at the active modes: given
 * grad_force = dLoss/dF ([3][N_tot]), writes grad_pos = dLoss/dr ([3][N_tot])
 * and grad_q = dLoss/dq ([N_tot]) through the Fourier part (eq. 3.6 with the
 * structure factor of eq. 2.7) and/or the real-space and LJ parts (eq. 2.11,
 * eq. 4.1), selected by parts (RBE_PART_*).  Outputs are overwritten. */
rbe_status rbe_forces_vjp(rbe_ctx *ctx, const void *pos, const void *q, const void *grad_force, void *grad_pos,
                          void *grad_q, int32_t parts);

/* Number of neighbour-list builds made by rbe_step since creation (the first
 * step after creation, after rbe_real_forces / rbe_energy / rbe_forces_vjp,
 * and whenever a particle had moved more than skin/2 or a list overflowed),
 * or -1 when the context does not use the list.  Synchronises the stream.
 * Returns RBE_ERR_TIMEOUT (builds still written) when a rebuild gave up since
 * the previous check (see rbe_check). */
rbe_status rbe_list_builds(rbe_ctx *ctx, int64_t *builds);

/* Time step of every system from the next rbe_step on.  anneal = 0: the
 * fixed step dt.  anneal > 0: the annealed burn-in schedule of Sec. 4.2
 * (Example 2), where the step with index n (the step numbers rbe_step
 * receives) uses dt_n = anneal / ln(1 + n), n taken as at least 1; the
 * paper's burn-in uses anneal = 0.01 with the Andersen thermostat, then a
 * fixed dt.  The schedule is evaluated on the device for every step (BAOAB
 * coefficients and the Andersen collision probability nu dt_n included).
 * RBE_ERR_INVALID for a negative or non-finite value.  Synchronises the
 * stream. */
rbe_status rbe_set_dt(rbe_ctx *ctx, double dt, double anneal);

/* Pair-distance counts of every system (Sec. 4.1: the pair correlations
 * g_++, g_+- behind the charge-charge correlation rho(r) = g_++ - g_+-).
 * Adds to counts (device, int64 [R][3][nbins]) the number of pairs i < j of
 * each system at minimum-image distance r < r_max, in bin floor(r / dr) with
 * dr = r_max / nbins (r = sqrt(dx^2 + dy^2 + dz^2) of the minimum-image
 * displacement in FP64, each operation rounded on its own), by
 * class: 0 both q > 0, 1 one of each sign, 2 both q <= 0.  pos, q: the
 * context's precision, original order.  All pairs are visited (O(N^2) per
 * system): an analysis call, not a time-step kernel.  RBE_ERR_INVALID unless
 * 0 < r_max <= L/2 for every system and 1 <= nbins <= 4096.  Asynchronous. */
rbe_status rbe_pair_histogram(rbe_ctx *ctx, const void *pos, const void *q, double r_max, int32_t nbins,
                              int64_t *counts);

/* Graph replay of rbe_step (default off).  With a neighbour list and the
 * exact sampler, the steps of one rbe_step call after its first and before
 * its last are replayed 16 at a time from a captured hipGraph of their
 * launches (captured on a stream the library owns, on first use for a given
 * set of buffers, tiles and list parity; at most four kept per context until
 * it is destroyed, the tiles change or enable = 0).  The step numbers reach
 * the replayed kernels through a device counter, so the results are those of
 * separate launches (bit for bit in FP32).  Measured on MI355X with ROCm 7,
 * separate launches on one stream were slightly faster at N = 1e5, hence the
 * default.  enable = 0 drops the graphs.  Synchronises the stream. */
rbe_status rbe_use_graphs(rbe_ctx *ctx, int32_t enable);

/* Tile shapes: read or set (validated; 0 fields keep the current value). */
rbe_status rbe_get_tiles(const rbe_ctx *ctx, rbe_tiles *tiles);
rbe_status rbe_set_tiles(rbe_ctx *ctx, const rbe_tiles *tiles);

/* Time the Fourier pass under every candidate tile shape on the given inputs
 * (hipEvents on the context stream, reps repetitions each), keep the fastest
 * and return it in *best (may be NULL).  The result also goes to the
 * process's tile cache (see rbe_tune_lookup), so later contexts of the same
 * key start from it, and is appended to the cache file when $RBE_TUNE_CACHE
 * names one (the file shipped beside the library is never written).  Not a
 * hot call. */
rbe_status rbe_autotune(rbe_ctx *ctx, const void *pos, const void *q, int32_t reps, rbe_tiles *best);

/* Tile cache: shapes found by rbe_autotune, keyed by device architecture
 * (e.g. "gfx950"), precision, floor(log2 ntot), floor(log2 max_p) and
 * whether R > 1.  rbe_create / rbe_batch_create take their tile shapes from
 * it when it holds their key (else the built-in defaults).  It is read once
 * per process from the file named by $RBE_TUNE_CACHE, or else from
 * rbe_tiles.txt in the directory of the library.  Host only; writes the
 * cached shapes to *out and returns RBE_OK, or RBE_ERR_STATE when the key is
 * absent, RBE_ERR_INVALID for bad arguments. */
rbe_status rbe_tune_lookup(const char *arch, int32_t precision, int64_t ntot, int32_t max_p, int32_t R,
                           rbe_tiles *out);

/* Per-kernel timing while enabled: each logical kernel's launches carry
 * hipEvents on their own dispatches (hipExtLaunchKernel), so the elapsed
 * time is the kernels' execution as a kernel trace reports it, with no
 * packets added between launches. */
rbe_status rbe_profile_enable(rbe_ctx *ctx, int32_t enable);
/* Accumulated milliseconds and launch count of kernel `id` since enabling;
 * synchronises.  Returns RBE_ERR_INVALID for an unknown id. */
rbe_status rbe_profile_read(rbe_ctx *ctx, int32_t id, double *total_ms, int64_t *launches);
/* Name of kernel `id` (0 .. rbe_profile_count()-1), NULL if out of range. */
const char *rbe_profile_name(int32_t id);
int32_t rbe_profile_count(void);

/* Throughput micro-benchmarks of the current device, for the rooflines of
 * the kernels (the paper's cost model counts operations per particle-mode
 * pair, Sec. 3.1): compiled with the library's own flags (no packed FP32
 * instructions).  kind 0: hardware sine/cosine of revolutions (v_sin_f32 and
 * v_cos_f32 alternating), lane operations per second; 1: FP32 fused
 * multiply-add, lane operations per second; 2: FP64 fused multiply-add, lane
 * operations per second; 3: device-to-device copy, bytes read plus written
 * per second.  *rate receives the best of `reps` timed launches (reps >= 1).
 * Allocates and frees a scratch buffer (kind 3: 2 x 256 MiB); not a hot call.
 * Synchronises the device.  RBE_ERR_INVALID for an unknown kind. */
rbe_status rbe_calibrate(int32_t kind, int32_t reps, double *rate);

#ifdef __cplusplus
}
#endif

#endif /* RBE_H */
