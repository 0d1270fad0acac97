// rbe_internal.h -- data layout shared by the host code and the kernels of
// librbe.  Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbe.h"

namespace rbe {

// Events of the kernel being timed (set by the host around one logical
// kernel while per-kernel timing is on, null otherwise).  Every launch goes
// through launch_k, which attaches them to the dispatch itself: the first
// launch of the logical kernel records the start, each launch the stop, so
// the elapsed time is the kernels' execution, as a kernel trace reports it,
// with no extra packets between launches.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool started = false;
};
LaunchEvents &launch_events();

template <typename F, typename... Args>
inline void launch_k(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t stream, Args... args)
{
    LaunchEvents &e = launch_events();
    hipEvent_t a = (e.start && !e.started) ? e.start : nullptr;
    if (a) e.started = true;
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, a, e.stop, 0u, args...);
}

constexpr double kPi = 3.14159265358979323846264338327950288;

// Tags in the top byte of Philox counter word 1; they separate the random
// streams of different purposes under one (seed, step) key.
constexpr uint32_t kTagSample = 0x01000000u;
constexpr uint32_t kTagLangevin = 0x02000000u;
constexpr uint32_t kTagAndersen = 0x03000000u;
constexpr uint32_t kTagMH = 0x04000000u;

// Bits of the device error word (Workspace::flag[0]).
constexpr int32_t kFlagNonFinite = 1;   // a kernel met a non-finite force
constexpr int32_t kFlagTimeout = 2;     // a bounded wait of a list rebuild gave up
constexpr int32_t kFlagBounds = 4;      // a rebuild index fell outside its system (skipped)
constexpr int32_t kFlagRange = 8;       // a single-precision real-space partial sum left the exact range

// Default bound on the spin iterations of a device-side wait.
constexpr int32_t kWaitLimit = 1 << 24;

// Per-system constants, resident in device memory and read by every kernel.
struct SysDev {
    int32_t n;          // particles
    int32_t p;          // active modes
    int32_t off;        // first particle in the concatenated arrays
    int32_t moff;       // first mode in the concatenated mode arrays
    int32_t cdf_off;    // first entry of this system's cumulative table
    int32_t M;          // table covers m = -M..M
    int32_t nc;         // cells per box side (1 => all-pairs real space)
    int32_t cell_off;   // first cell of this system
    int32_t lj_on;
    int32_t integrator;
    int32_t mh_state_off;  // three int32 chain states at this offset
    int32_t ncell;         // nc^3
    int32_t use_list;      // neighbour list in rbe_step (skin > 0 and nc >= 3)
    int32_t hi_bits;       // FP32 phases: box fractions split as hi (multiple of 2^-hi_bits) + lo
    float hi_scale, hi_inv;  // 2^hi_bits, 2^-hi_bits
    int32_t n_fixed;       // particles 0 .. n_fixed-1 never move
    int32_t diam_on;       // per-particle diameters: LJ with r_off = (d_i + d_j)/2 - sigma
    double L, invL;
    double alpha, beta;     // beta = sqrt(alpha)
    double rc2;             // r_cut^2
    double coulomb;
    double S;               // normaliser H^3 - 1
    double lj_eps, lj_sig2, lj_rc2, lj_shift;  // sigma^2, cutoff^2, V_shift
    double lj_sig, lj_rc;   // sigma and the cutoff R_c on r - r_off
    double rsearch2;        // largest pair reach squared: max(r_cut, max_pairs r_off + R_c)^2
    double kT, gamma, dt, mass;
    double c1, c2;          // Ornstein-Uhlenbeck factors exp(-gamma dt/m), sqrt((1-c1^2) kT/m)
    double nu_dt;           // Andersen collision probability per step
    double nu;              // Andersen collision frequency
    double anneal;          // > 0: the step of index n uses dt = anneal / ln(1 + n) instead of dt
    double rlist2;          // (largest cutoff + skin)^2
    double half_skin2;      // (skin / 2)^2
    uint64_t seed;
};

// A contiguous run of particles of one system processed by one block.
struct Tile {
    int32_t sys;
    int32_t start;   // first particle, relative to the system
    int32_t count;
    int32_t aux;     // structure-factor tiles: index of this tile within its system
};

// Per-mode constants for the force pass (single precision path): the mode
// (small integers, exact in float), the force coefficients
// a = w 2 m/(L^2 |m|^2) and the structure factor (C, S).
struct KModeF {
    float m[3];
    float a[3];
    float C, S;
};

struct KModeD {
    double m[3];
    double a[3];
    double C, S;
};

// Per-mode constants of the adjoint gather pass.
struct KVjpF {
    double m[3];
    float a[3];
    float k[3];     // 2 pi m / L
    float C, S, A, B;
    float pad[3];
};

struct KVjpD {
    double m[3];
    double a[3];
    double k[3];
    double C, S, A, B;
};

// Kernel ids for per-launch event timing.
enum KernelId {
    K_SAMPLE = 0,   // stand-alone mode sampling
    K_STAGE,        // [integrate] + [bin] + [sample] + structure-factor partials
    K_MID,          // structure-factor totals + cell scan
    K_KFORCE,       // Fourier force [+ scatter]
    K_SCATTER,      // stand-alone scatter into cell order
    K_REAL,         // real space [+ kick]
    K_ENERGY,
    K_VJP_REDUCE,
    K_VJP_GATHER,
    K_VJP_REAL,
    K_MISC,
    K_COUNT
};

// Most blocks a long mode list is split over per particle chunk (classical
// Ewald through rbe_set_k).
constexpr int kMaxModeSplit = 32;

// Device workspace of a context.
struct Workspace {
    SysDev *sys;           // [R]
    Tile *rho_tiles;       // structure-factor tiles
    Tile *force_tiles;     // force-pass tiles (64 particles)
    Tile *part_tiles;      // 256-particle tiles for elementwise kernels
    Tile *real_tiles;      // real-space tiles (aux 0: cell-sorted rows, 1: all pairs)
    int32_t *modes;        // [3][Mcap]
    double *mode_w;        // [Mcap] weights (S/p or explicit)
    double *partial;       // structure-factor tile partials
    int32_t *partial_off;  // [2R]: first partial row of each system, then its tile count
    double *rho;           // [Mcap][2] structure factors
    double *ab;            // [Mcap][2] adjoint reductions (A_l, B_l)
    void *kmode;           // KModeF[Mcap] or KModeD[Mcap]
    void *kvjp;            // KVjpF[Mcap] or KVjpD[Mcap]
    double *cdf;           // concatenated cumulative tables
    int32_t *mh_state;     // [R][3]
    int32_t *cell_count;   // [ncell_tot] (cell offsets padded to multiples of 4)
    int32_t *cell_start;   // [ncell_tot + R]
    int32_t *cellid;       // [Ntot] global cell of each particle
    int32_t *rank;         // [Ntot]
    int32_t *sorted_idx;   // [Ntot] particle at each sorted slot
    void *packed;          // [Ntot] wrapped position + charge, original order
    void *sorted;          // [Ntot] same, sorted by cell
    int32_t *modes_alt;    // the next step's modes and weights when the totals launch draws them
    double *mode_w_alt;
    double *energy_part;   // [real tiles][8]
    int32_t *flag;         // [4] word 0: kFlag* error bits
    // neighbour list of rbe_step (allocated when some system uses it)
    Tile *list_tiles;      // list-pass tiles (aux 2: cell-sorted slots, 1: all pairs)
    int32_t *slot_of;      // [Ntot] sorted slot of each particle at the last build
    void *ref;             // [Ntot] record of each particle at the last build (original order)
    int32_t *nbr;          // [kmax][Ntot] partner slots, column k of slot s at k * Ntot + s
    int32_t *nnb;          // [Ntot] partners of each slot
    int32_t *lflag;        // [8]: rebuild request for even / odd steps, list overflow, builds, scan ready,
                           //      binning blocks done, poison (a rebuild gave up: the cell counts are
                           //      stale until the force launch clears them, and the next step rebuilds)
    uint64_t *step_base;   // [1]: step number of a graph replay (see ListStep)
    void *fpart;           // [kMaxModeSplit][3][Ntot] partial forces of mode-split force passes (long
                           // mode lists only; NULL until rbe_reserve_modes raises the capacity)
    double *diam;          // [Ntot] per-particle diameters (original order), or NULL
};

struct LaunchCfg {
    hipStream_t stream;
    int R;
    int prec;
    int64_t ntot;
    int mcap;
    int n_rho_tiles, n_force_tiles, n_part_tiles, n_real_tiles;
    int max_sys_rho_tiles;   // most structure-factor tiles of one system
    int rho_chunk, rho_block, force_split, real_split;
    int ncell_tot;
    int max_cells;   // largest cell count of one system
    int max_p;
    int max_table;   // largest cumulative table (2M + 1)
    int list_on;     // some system uses the neighbour list
    int kmax;        // list capacity per particle
    int n_list_tiles;
    int wait_limit;  // spin bound of the device-side waits of a list rebuild
};

// Device view of the neighbour-list state for one step.
struct ListStep {
    int32_t *rebuild;        // request flag of this step (read)
    int32_t *rebuild_next;   // request flag of the next step
    int32_t *overflow;
    int32_t *rebuilds;       // count of list builds
    int32_t *ready;          // rebuild: cell scan done (raised in the totals launch, reset by the staging launch)
    int32_t *bins_done;      // rebuild: binning blocks finished (same)
    int32_t *poison;         // a rebuild gave up (see Workspace::lflag)
    int force_rebuild;
    // graph replays: the step numbers passed to the launches are offsets
    // from *step_base (device), which the force launch advances by `bump`
    const uint64_t *step_base = nullptr;
    uint64_t *step_bump = nullptr;
    uint32_t bump = 0;
};

// What one launch of the staging kernel does.
struct StageRequest {
    void *pos;
    void *vel;
    const void *force;
    const void *q;
    uint64_t step;         // integrator noise index
    uint64_t sample_step;  // mode sample index
    int integrate, bin, sample, rho;
    const ListStep *list;  // integrate in list mode: update cell-order records, test displacements
    int kick = 0;          // integrate: first apply the previous step's closing half kick (deferred)
    int mode_split = 1;    // no integration/binning/sampling: split the modes over this many blocks per chunk
};

// ---- launchers (rbe_kspace.hip, rbe_real.hip) ----
hipError_t launch_sample(const LaunchCfg &c, const Workspace &w, uint64_t step, int use_mh);
hipError_t launch_stage(const LaunchCfg &c, const Workspace &w, const StageRequest &rq);
size_t stage_lds_bytes(const LaunchCfg &c, int sample_in_kernel, int *table_lds, int *tab_max);
hipError_t launch_mid(const LaunchCfg &c, const Workspace &w, int do_final, int do_scan,
                      const int32_t *scan_gate = nullptr, const int32_t *bin_gate = nullptr,
                      int32_t *clear_flag = nullptr, int sample_next = 0, uint64_t sample_step = 0,
                      const ListStep *ls = nullptr);
hipError_t launch_kforce(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q, void *force,
                         int accumulate, int scatter, int mode_split = 1);
hipError_t launch_scatter(const LaunchCfg &c, const Workspace &w);
hipError_t launch_set_step(const LaunchCfg &c, const Workspace &w, uint64_t step);
hipError_t launch_pair_hist(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q, double r_max,
                            int nbins, int64_t *counts);
hipError_t launch_real_step(const LaunchCfg &c, const Workspace &w, const ListStep &ls, void *force, void *vel_kick,
                            uint64_t kick_step = 0);
hipError_t launch_real(const LaunchCfg &c, const Workspace &w, void *force, int accumulate, void *vel_kick,
                       uint64_t kick_step = 0);
hipError_t launch_energy(const LaunchCfg &c, const Workspace &w, const void *q, const void *vel);
hipError_t launch_vjp_reduce(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                             const void *gF);
hipError_t launch_vjp_final(const LaunchCfg &c, const Workspace &w);
hipError_t launch_vjp_gather(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                             const void *gF, void *gpos, void *gq);
hipError_t launch_vjp_real(const LaunchCfg &c, const Workspace &w, const void *gF, void *gpos, void *gq,
                           int accumulate);
hipError_t launch_fill_zero(hipStream_t s, void *ptr, int64_t nbytes);
hipError_t launch_static_setup(const LaunchCfg &c, const Workspace &w, const SysDev &sys);
int real_rows_per_tile();
int real_allpairs_per_tile();

}  // namespace rbe
