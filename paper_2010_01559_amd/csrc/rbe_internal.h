// rbe_internal.h -- data layout shared by the host code and the kernels of
// librbe.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbe.h"

namespace rbe {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Tags in the top byte of Philox counter word 1; they separate the random
// streams of different purposes under one (seed, step) key.
constexpr uint32_t kTagSample = 0x01000000u;
constexpr uint32_t kTagLangevin = 0x02000000u;
constexpr uint32_t kTagAndersen = 0x03000000u;
constexpr uint32_t kTagMH = 0x04000000u;

// Per-system constants, resident in device memory and read by every kernel.
struct SysDev {
    int32_t n;          // particles
    int32_t p;          // active modes
    int32_t off;        // first particle in the concatenated arrays
    int32_t moff;       // first mode in the concatenated mode arrays
    int32_t cdf_off;    // first entry of this system's cumulative table
    int32_t M;          // table covers m = -M..M
    int32_t nc;         // cells per box side (0 => all-pairs real space)
    int32_t cell_off;   // first cell of this system
    int32_t lj_on;
    int32_t integrator;
    int32_t mh_state_off;  // three int32 chain states at this offset
    int32_t ncell;         // nc^3
    double L, invL;
    double alpha, beta;     // beta = sqrt(alpha)
    double rc2;             // r_cut^2
    double coulomb;
    double S;               // normaliser H^3 - 1
    double lj_eps, lj_sig2, lj_rc2, lj_shift;  // sigma^2, cutoff^2, V_shift
    double kT, gamma, dt, mass;
    double c1, c2;          // Ornstein-Uhlenbeck factors exp(-gamma dt/m), sqrt((1-c1^2) kT/m)
    double nu_dt;           // Andersen collision probability per step
    uint64_t seed;
};

// A contiguous run of particles of one system processed by one block.
struct Tile {
    int32_t sys;
    int32_t start;   // first particle, relative to the system
    int32_t count;
    int32_t aux;     // structure-factor tiles: index of this tile within its system
};

// Per-mode constants for the force pass (single precision path).  The phase
// uses the mode in double; the force coefficients a = w 2 m/(L^2 |m|^2) and
// the structure factor (C, S) are in float.
struct KModeF {
    double m[3];
    float a[3];
    float C, S;
    float pad;
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
    K_SAMPLE = 0,
    K_RHO,
    K_RHO_FINAL,
    K_KFORCE,
    K_BIN,
    K_SCAN,
    K_SCATTER,
    K_CELLSORT,
    K_REAL,
    K_INTEGRATE,
    K_ENERGY,
    K_VJP_REDUCE,
    K_VJP_GATHER,
    K_VJP_REAL,
    K_MISC,
    K_COUNT
};

// Device workspace of a context.
struct Workspace {
    SysDev *sys;           // [R]
    Tile *rho_tiles;       // structure-factor tiles
    Tile *force_tiles;     // force-pass tiles (64 particles per wave slot)
    Tile *part_tiles;      // 256-particle tiles for elementwise kernels
    int32_t *modes;        // [3][Mcap]
    double *mode_w;        // [Mcap] weights (S/p or explicit)
    double *partial;       // [rho tiles][modes][2] (sized for the maximum over systems)
    int32_t *partial_off;  // [R] first partial row of each system
    double *rho;           // [Mcap][2] structure factors
    double *ab;            // [Mcap][2] adjoint reductions (A_l, B_l)
    void *kmode;           // KModeF[Mcap] or KModeD[Mcap]
    void *kvjp;            // KVjpF[Mcap] or KVjpD[Mcap]
    double *cdf;           // concatenated cumulative tables
    int32_t *mh_state;     // [R][3]
    int32_t *cell_count;   // [ncell_tot]
    int32_t *cell_start;   // [ncell_tot + R]
    int32_t *cellid;       // [Ntot] global cell of each particle
    int32_t *rank;         // [Ntot]
    int32_t *sorted_idx;   // [Ntot] particle at each sorted slot
    void *packed;          // [Ntot] wrapped position + charge, original order
    void *sorted;          // [Ntot] same, sorted by cell
    double *energy_part;   // [part tiles][8]
    int32_t *flag;         // [1] non-finite flag
};

// ---- launchers implemented in rbe_kernels.hip ----
struct LaunchCfg {
    hipStream_t stream;
    int R;
    int prec;
    int64_t ntot;
    int mcap;
    int n_rho_tiles, n_force_tiles, n_part_tiles;
    int rho_chunk, rho_block, force_split, real_split;
    int ncell_tot;
    int max_cells;   // largest cell count of one system
    int max_p;
};

hipError_t launch_sample(const LaunchCfg &c, const Workspace &w, uint64_t step, int use_mh);
hipError_t launch_set_weights(const LaunchCfg &c, const Workspace &w);
hipError_t launch_rho(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q);
hipError_t launch_rho_final(const LaunchCfg &c, const Workspace &w);
hipError_t launch_kforce(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q, void *force,
                         int accumulate);
hipError_t launch_bin(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q);
hipError_t launch_scan(const LaunchCfg &c, const Workspace &w);
hipError_t launch_scatter(const LaunchCfg &c, const Workspace &w);
hipError_t launch_cellsort(const LaunchCfg &c, const Workspace &w);
hipError_t launch_real(const LaunchCfg &c, const Workspace &w, void *force, int accumulate, void *vel_kick);
hipError_t launch_integrate(const LaunchCfg &c, const Workspace &w, void *pos, void *vel, const void *force,
                            uint64_t step);
hipError_t launch_energy(const LaunchCfg &c, const Workspace &w, const void *q, const void *vel);
hipError_t launch_vjp_reduce(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                             const void *gF);
hipError_t launch_vjp_final(const LaunchCfg &c, const Workspace &w);
hipError_t launch_vjp_gather(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                             const void *gF, void *gpos, void *gq);
hipError_t launch_vjp_real(const LaunchCfg &c, const Workspace &w, const void *gF, void *gpos, void *gq,
                           int accumulate);
hipError_t launch_fill_zero(hipStream_t s, void *ptr, int64_t nbytes);

}  // namespace rbe
