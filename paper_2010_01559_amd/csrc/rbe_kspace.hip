// rbe_kspace.hip -- Fourier-space kernels of librbe (gfx950).
//
// Paper: Jin, Li, Xu & Zhao, "A random batch Ewald method for particle
// systems with Coulomb interactions", arXiv:2010.01559, Sec. 3.1.
//
// The random batch force (eq. 3.6) with k = 2 pi m / L reads
//   F_i = -q_i sum_l a_l (cos th_il S_l - sin th_il C_l),
//   a_l = coulomb w_l 2 m_l / (L^2 |m_l|^2),  th_il = 2 pi m_l . r_i / L,
//   rho_l = C_l + i S_l = sum_j q_j exp(i th_jl)       (eq. 2.7)
// with w_l = S/p for sampled modes.  Only integer modes and one scalar per
// mode enter.  Single-precision phases are formed exactly from a split of
// the box fraction (phase_split in rbe_device.h) and fed to the hardware
// sine/cosine in revolutions; the FP64 path wraps in double.
//
// Kernels:
//   k_sample_exact  draw the modes of every system (standalone call)
//   k_sample_mh     the paper's Metropolis-Hastings chains
//   k_stage_rho     [closing kick + integrate + list bookkeeping] + [bin] +
//                   [draw modes] + structure-factor partials per particle
//                   chunk (one launch; a lean instantiation for launches
//                   that only compute structure factors)
//   k_mid           structure-factor totals + per-mode force constants,
//                   the next step's modes, the exclusive scan of the cell
//                   counts, and the gated list rebuild (one launch)
//   k_kforce        force pass + [scatter into cell order]; long mode lists
//                   split over blocks (grid y) and summed by k_fsum
//   k_vjp_*         adjoint of the force at a fixed mode sample
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "rbe_device.h"
#include "rbe_internal.h"
#include "rbe_roles.h"

namespace rbe {

// ---------------------------------------------------------------------------
// Sampling (Sec. 3.1, eqs. 3.3-3.5)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sample_exact(const SysDev *__restrict__ sys, const double *__restrict__ cdf,
                                                      int32_t *__restrict__ modes, double *__restrict__ mode_w,
                                                      int mcap, uint64_t step, int table_lds)
{
    extern __shared__ double tab[];
    const SysDev S = sys[blockIdx.y];
    const int K = 2 * S.M + 1;
    const double *t = cdf + S.cdf_off;
    if (table_lds) {
        for (int k = threadIdx.x; k < K; k += blockDim.x) tab[k] = t[k];
        __syncthreads();
        t = tab;
    }
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= S.p) return;
    int mx, my, mz;
    sample_mode(t, S.M, (uint32_t)l, S.seed, step, mx, my, mz);
    const int o = S.moff + l;
    modes[o] = mx;
    modes[mcap + o] = my;
    modes[2 * mcap + o] = mz;
    mode_w[o] = S.S / (double)S.p;
}

// Proposal mass of eq. (3.5): P(round(x*) = m) for x* ~ N(0, alpha L^2/(2 pi^2)).
__device__ double mh_qbar(double w, int m)
{
    const int am = m < 0 ? -m : m;
    if (am == 0) return erf(0.5 / w);
    return 0.5 * (erf((am + 0.5) / w) - erf((am - 0.5) / w));
}

// One wave per system, lanes 0..2 the three component chains, whose states
// persist in the context.  Attempt a of draw l: lane d uses Philox block
// (l, TAG_MH | 4a + d, step) for its Box-Muller proposal and word d of block
// (l, TAG_MH | 4a + 3, step) as its acceptance uniform; the all-zero vector
// is discarded.
__global__ __launch_bounds__(64) void k_sample_mh(const SysDev *__restrict__ sys, int32_t *__restrict__ state,
                                                  int32_t *__restrict__ modes, double *__restrict__ mode_w,
                                                  int mcap, uint64_t step)
{
    const SysDev S = sys[blockIdx.x];
    const int d = threadIdx.x;
    const double a2 = kPi * kPi / (S.alpha * S.L * S.L);
    const double sd = sqrt(S.alpha * S.L * S.L / (2.0 * kPi * kPi));
    const double w = sqrt(S.alpha * S.L * S.L / (kPi * kPi));
    int cur = d < 3 ? state[S.mh_state_off + d] : 1;
    for (int l = 0; l < S.p; ++l) {
        for (uint32_t a = 0; a < (1u << 20); ++a) {
            const U4 acc = draw((uint32_t)l, kTagMH | (4u * a + 3u), S.seed, step);
            if (d < 3) {
                const U4 r = draw((uint32_t)l, kTagMH | (4u * a + (uint32_t)d), S.seed, step);
                const double u1 = 1.0 - u53(r.x, r.y), u2 = u53(r.z, r.w);
                const double x = sd * sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
                const int ms = x >= 0.0 ? (int)floor(x + 0.5) : -(int)floor(-x + 0.5);
                const double ratio =
                    exp(-a2 * ((double)ms * ms - (double)cur * cur)) * mh_qbar(w, cur) / mh_qbar(w, ms);
                const uint32_t word = d == 0 ? acc.x : (d == 1 ? acc.y : acc.z);
                if ((double)word * (1.0 / 4294967296.0) < ratio) cur = ms;
            }
            if (__ballot(d < 3 && cur != 0)) break;
        }
        if (d < 3) modes[d * mcap + S.moff + l] = cur;
    }
    if (d < 3) state[S.mh_state_off + d] = cur;
    if (d == 0)
        for (int l = 0; l < S.p; ++l) mode_w[S.moff + l] = S.S / (double)S.p;
}

// ---------------------------------------------------------------------------
// k_stage_rho: one block per particle chunk of one system.
//  1. (integrate) BAOA of the Langevin step (reading: BAOAB) or the leapfrog
//     + Andersen update, positions wrapped into [0, L), arithmetic in double;
//  2. (bin) cell index, atomic rank within the cell and the packed record;
//  3. stage fractional coordinates + charge of the chunk in LDS;
//  4. (sample) draw the system's modes into LDS (the cumulative table is
//     staged in LDS when small); the first chunk of the system publishes them;
//  5. structure-factor partials: each thread owns one mode and one residue
//     class g of the chunk (G = blockDim / P classes); per-thread sums are
//     blocked in T over runs of 8 particles and folded into double; the G
//     partials of a mode are combined in LDS in a fixed order.
// ---------------------------------------------------------------------------
template <typename T>
struct StageArgs {
    const SysDev *sys;
    const Tile *tiles;
    T *pos;
    T *vel;
    const T *F;
    const T *q;
    int64_t ntot;
    const double *cdf;
    int32_t *modes;
    double *mode_w;
    int mcap;
    double *partial;
    const int32_t *part_off;
    int32_t *count;
    int32_t *cellid;
    int32_t *rank;
    void *packed;
    uint64_t step;         // integrator noise index
    uint64_t sample_step;  // mode sample index
    int do_integrate, do_bin, do_sample, table_lds, do_rho;
    int kick;   // deferred closing half kick of the previous step
    int chunk;
    int single_n;          // single-system context (SINGLE launches): its particle count
    int single_p;          // and its mode count
    int tab_max;           // LDS doubles reserved for the table
    // neighbour-list mode of a time step
    int list_mode;
    ListStep ls;
    const int32_t *slot_of;
    void *sorted;
    const void *ref;
};

template <typename T>
__device__ __forceinline__ void bin_one(const SysDev &S, int64_t i, double sx, double sy, double sz, T qi,
                                        int32_t *count, int32_t *cellid, int32_t *rank, void *packed)
{
    int cx, cy, cz;
    if constexpr (sizeof(T) == 4) {
        const PackF v{to_fix(sx), to_fix(sy), to_fix(sz), (float)qi};
        reinterpret_cast<PackF *>(packed)[i] = v;
        cx = cell_of_fix(v.x, S.nc);
        cy = cell_of_fix(v.y, S.nc);
        cz = cell_of_fix(v.z, S.nc);
    } else {
        reinterpret_cast<PartD *>(packed)[i] = PartD{sx, sy, sz, (double)qi};
        cx = cell_of_frac(sx, S.nc);
        cy = cell_of_frac(sy, S.nc);
        cz = cell_of_frac(sz, S.nc);
    }
    const int c = S.cell_off + (cz * S.nc + cy) * S.nc + cx;
    cellid[i] = c;
    rank[i] = atomicAdd(&count[c], 1);
}

// List mode: store the new record in original and cell order and test the
// displacement since the last list build against skin/2.
template <typename T>
__device__ __forceinline__ bool list_update(const SysDev &S, int64_t i, double sx, double sy, double sz, T qi,
                                            const StageArgs<T> &a, const ListRef &lr)
{
    return record_update<T>(S, i, sx, sy, sz, qi, a.packed, a.sorted, lr);
}

// LDS record of the structure-factor pass: fractional coordinates in double
// and the charge in the working precision.
template <typename T>
struct RhoRec;
template <>
struct RhoRec<float> {
    struct type {
        float hx, hy, hz, lx, ly, lz, q, pad;   // split box fractions, charge
    };
};
template <>
struct RhoRec<double> {
    using type = PartD;
};

__device__ __forceinline__ void rho_record(const SysDev &S, double sx, double sy, double sz, float q,
                                           RhoRec<float>::type &v)
{
    split_frac(sx, S, v.hx, v.lx);
    split_frac(sy, S, v.hy, v.ly);
    split_frac(sz, S, v.hz, v.lz);
    v.q = q;
    v.pad = 0.0f;
}

__device__ __forceinline__ void rho_record(const SysDev &, double sx, double sy, double sz, double q, PartD &v)
{
    v.x = sx;
    v.y = sy;
    v.z = sz;
    v.q = q;
}

// One particle-mode term of the structure factor, added to (c, s).
__device__ __forceinline__ void rho_term(const RhoRec<float>::type &v, float mx, float my, float mz, float &c,
                                         float &s)
{
    const float rf = phase_split(mx, my, mz, v.hx, v.hy, v.hz, v.lx, v.ly, v.lz);
    const float sn = __builtin_amdgcn_sinf(rf), cs = __builtin_amdgcn_cosf(rf);
    c = fmaf(v.q, cs, c);
    s = fmaf(v.q, sn, s);
}

__device__ __forceinline__ void rho_term(const PartD &v, double mx, double my, double mz, double &c, double &s)
{
    const double ph = wrap_rev(fma(mx, v.x, fma(my, v.y, mz * v.z)));
    double sn, cs;
    sincospi(2.0 * ph, &sn, &cs);
    c = fma(v.q, cs, c);
    s = fma(v.q, sn, s);
}

// Particle groups per block are capped so that the zero-charge padding of a
// chunk (up to 8 records per group) stays small.
constexpr int kRhoGroupsMax = 32;
constexpr int kRhoUnroll = 8;

// VAR = 0 compiles a lean variant for launches that only stage the
// particles and compute structure factors (force calls, energies, long
// Ewald lists): without the integrator, binning, sampling and list code it
// needs far fewer registers, so more blocks share a compute unit.  VAR = 1
// adds the mode draw (force calls after rbe_sample_k), VAR = 2 is the full
// time-step variant.  SINGLE (single-system contexts) forms the block's tile
// from its index, as the host builds it, instead of loading it, so that the
// first particle loads do not wait for the tile and system constants.
template <typename T, int BS, int VAR, bool SINGLE>
__global__ __launch_bounds__(BS, VAR == 2 ? 1 : 8) void k_stage_rho(StageArgs<T> a)
{
    constexpr bool FULL = VAR == 2;     // integrator, binning, list bookkeeping
    constexpr bool SAMPLE = VAR >= 1;   // draws the modes in the launch
    extern __shared__ __align__(16) unsigned char smem[];
    const int bx = (int)blockIdx.x;
    const Tile t = SINGLE ? Tile{0, bx * a.chunk, min(a.chunk, a.single_n - bx * a.chunk), bx} : a.tiles[bx];
    SysDev S = a.sys[SINGLE ? 0 : t.sys];
    if constexpr (SINGLE) {
        // the single system's offsets are 0, its mode count comes with the
        // launch, and a list step implies that it uses the list: no particle,
        // list or mode load waits for the system constants
        S.off = 0;
        S.moff = 0;
        S.p = a.single_p;
        if (a.list_mode) S.use_list = 1;
    }
    using RR = typename RhoRec<T>::type;
    RR *sp = reinterpret_cast<RR *>(smem);
    double2 *red = reinterpret_cast<double2 *>(smem + sizeof(RR) * (a.chunk + kRhoUnroll * kRhoGroupsMax));
    double *tab = reinterpret_cast<double *>(red + BS);
    int *smode = reinterpret_cast<int *>(tab + a.tab_max);  // [3][BS]
    const int tid = threadIdx.x;
    const int count = t.count;
    const int K = 2 * S.M + 1;
    if (SAMPLE && a.do_sample && a.table_lds)
        for (int k = tid; k < K; k += BS) tab[k] = a.cdf[S.cdf_off + k];
    if (FULL && a.list_mode && blockIdx.x == 0 && tid == 0) {
        // the rebuild of this step (in the totals launch) starts from zero
        *a.ls.ready = 0;
        *a.ls.bins_done = 0;
    }
    bool moved = false;
    const uint64_t base = FULL && a.list_mode && a.ls.step_base ? *a.ls.step_base : 0;
    const uint64_t step = a.step + base, sample_step = a.sample_step + base;
    for (int j = tid; j < count; j += BS) {
        const int il = t.start + j;
        const int64_t i = S.off + il;
        double x[3];
        // single precision loads the list reference before integrating; in
        // double the extra live registers would spill
        constexpr bool EARLY = sizeof(T) == 4;
        ListRef lr;
        if (FULL && EARLY && a.list_mode) load_list_ref<T>(S, i, a.slot_of, a.ref, lr);
        if (FULL && a.do_integrate) {
            integrate_one<T>(S, il, i, a.ntot, a.pos, a.vel, a.F, step, a.kick != 0, x);
        } else {
            x[0] = (double)a.pos[i];
            x[1] = (double)a.pos[a.ntot + i];
            x[2] = (double)a.pos[2 * a.ntot + i];
        }
        const double sx = frac01(x[0] * S.invL), sy = frac01(x[1] * S.invL), sz = frac01(x[2] * S.invL);
        const T qi = a.q[i];
        RR v;
        if constexpr (sizeof(T) == 4) {
            if (FULL && a.list_mode) {
                // the force pass reads the stored 32-bit records: take the
                // phases of the structure factor from the same fractions
                split_fix(to_fix(sx), S, v.hx, v.lx);
                split_fix(to_fix(sy), S, v.hy, v.ly);
                split_fix(to_fix(sz), S, v.hz, v.lz);
                v.q = qi;
                v.pad = 0.0f;
            } else {
                rho_record(S, sx, sy, sz, qi, v);
            }
        } else {
            rho_record(S, sx, sy, sz, qi, v);
        }
        sp[j] = v;
        if (FULL && a.do_bin) bin_one<T>(S, i, sx, sy, sz, qi, a.count, a.cellid, a.rank, a.packed);
        if (FULL && !EARLY && a.list_mode) load_list_ref<T>(S, i, a.slot_of, a.ref, lr);
        if (FULL && a.list_mode) moved |= list_update<T>(S, i, sx, sy, sz, qi, a, lr);
    }
    if (FULL && a.list_mode) {
        // one request per block; block 0 adds the host's and the overflow's
        const int any = __syncthreads_or(moved ? 1 : 0);
        if (tid == 0) {
            // a rebuild that gave up in the step before is redone
            const bool req =
                any || (blockIdx.x == 0 && (a.ls.force_rebuild || *a.ls.overflow != 0 || *a.ls.poison != 0));
            if (req) atomicOr(a.ls.rebuild, 1);
        }
    } else {
        __syncthreads();
    }
    if (!a.do_rho) return;
    const int P = S.p;
    // modes [mb, me) of this block: a launch with gridDim.y > 1 splits long
    // mode lists (classical Ewald) over blocks; it never integrates, bins or
    // samples, so every y-block may stage the chunk on its own
    const int ys = (int)gridDim.y;
    const int mb = (int)(((int64_t)P * blockIdx.y) / ys), me = (int)(((int64_t)P * (blockIdx.y + 1)) / ys);
    const int Pm = me - mb;
    if (Pm <= 0) return;
    const int Pt = Pm < BS ? Pm : BS;
    const int G = BS / Pt < kRhoGroupsMax ? BS / Pt : kRhoGroupsMax;
    // zero-charge records up to a multiple of 8 G, so the unrolled loop
    // below needs no bounds tests
    const int cpad = (count + kRhoUnroll * G - 1) / (kRhoUnroll * G) * (kRhoUnroll * G);
    for (int j = count + tid; j < cpad; j += BS) {
        RR z{};
        sp[j] = z;
    }
    const double *tabp = a.table_lds ? tab : a.cdf + S.cdf_off;
    double *prow = a.partial + 2 * ((SINGLE ? 0 : (int64_t)a.part_off[t.sys]) + (int64_t)t.aux * P);
    for (int m0 = mb; m0 < me; m0 += Pt) {
        // modes of this tile into LDS: drawn here or read from the mode arrays
        if (tid < Pt && m0 + tid < me) {
            const int l = m0 + tid;
            int mx, my, mz;
            if (SAMPLE && a.do_sample) {
                sample_mode(tabp, S.M, (uint32_t)l, S.seed, sample_step, mx, my, mz);
                if (t.aux == 0) {
                    const int o = S.moff + l;
                    a.modes[o] = mx;
                    a.modes[a.mcap + o] = my;
                    a.modes[2 * a.mcap + o] = mz;
                    a.mode_w[o] = S.S / (double)P;
                }
            } else {
                const int o = S.moff + l;
                mx = a.modes[o];
                my = a.modes[a.mcap + o];
                mz = a.modes[2 * a.mcap + o];
            }
            smode[tid] = mx;
            smode[BS + tid] = my;
            smode[2 * BS + tid] = mz;
        }
        __syncthreads();
        const int lt = tid % Pt, g = tid / Pt;
        const int l = m0 + lt;
        const bool act = g < G && l < me;
        double C = 0.0, Sn = 0.0;
        if (act) {
            const T mx = (T)smode[lt], my = (T)smode[BS + lt], mz = (T)smode[2 * BS + lt];
            for (int j0 = g; j0 < cpad; j0 += kRhoUnroll * G) {
                T c8 = 0, s8 = 0;
#pragma unroll
                for (int u = 0; u < kRhoUnroll; ++u) rho_term(sp[j0 + u * G], mx, my, mz, c8, s8);
                C += (double)c8;
                Sn += (double)s8;
            }
        }
        red[tid] = make_double2(C, Sn);
        __syncthreads();
        if (tid < Pt && l < me) {
            double c = 0.0, s = 0.0;
            for (int gg = 0; gg < G; ++gg) {
                const double2 v = red[gg * Pt + lt];
                c += v.x;
                s += v.y;
            }
            prow[2 * l] = c;
            prow[2 * l + 1] = s;
        }
        // the next mode tile reuses smode and red; after the last one the
        // block ends without waiting for its stores
        if (m0 + Pt < me) __syncthreads();
    }
}

__global__ void k_set_step(uint64_t *base, uint64_t step)
{
    if (threadIdx.x == 0) *base = step;
}

// Sets the device step number that graph-replayed steps add to their step
// offsets (a kernel, so that no memset or copy node is needed).
hipError_t launch_set_step(const LaunchCfg &c, const Workspace &w, uint64_t step)
{
    launch_k(k_set_step, 1, 64, 0, c.stream, w.step_base, step);
    return hipGetLastError();
}


int final_waves_log2(int max_tiles_per_system) { return max_tiles_per_system > 64 ? 2 : 0; }

// ---------------------------------------------------------------------------
// k_mid: independent jobs in one launch (roles in rbe_roles.h), in block
// order: final structure factors (one or four waves per (system, mode) add
// the tile partials in a fixed order and fill the per-mode force constants); gated
// binning of a neighbour-list rebuild; the next step's modes (one block per
// system); then either the gated rebuild's scan and scatter blocks or, for
// cell-list force calls, one cell-scan block per system.
// ---------------------------------------------------------------------------
// LEAN: the structure-factor totals only (force, energy and adjoint calls).
template <typename KM, bool LEAN>
__global__ __launch_bounds__(1024) void k_mid(MidArgs<KM> a)
{
    extern __shared__ double mid_tab[];
    if (!LEAN && blockIdx.x == 0 && threadIdx.x == 0 && a.clear_flag) *a.clear_flag = 0;
    if ((int)blockIdx.x < a.n_final_blocks) {
        mid_final<KM>(a, blockIdx.x);
        return;
    }
    if constexpr (LEAN) return;
    const int b = blockIdx.x - a.n_final_blocks;
    if (b < a.n_bin_blocks) {
        if (*a.bin_gate == 0) return;
        mid_bin<KM>(a, b);
        if (a.reb) {
            // publish this block's counts, cell ids and ranks
            block_stores_done();
            if (threadIdx.x == 0) __hip_atomic_fetch_add(a.rb.bins_done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    const int b2 = b - a.n_bin_blocks;
    if (b2 < a.n_sample_blocks) {
        mid_sample<KM>(a, b2, a.table_lds ? mid_tab : nullptr);
        return;
    }
    const int b3 = b2 - a.n_sample_blocks;
    if (a.reb) {
        if (*a.bin_gate == 0) return;
        using Rec = typename std::conditional<sizeof(KM) == sizeof(KModeF), PackF, PartD>::type;
        if (b3 == 0)
            rebuild_scan<16>(a.rb);
        else
            rebuild_scatter<Rec>(a.rb, b3 - 1, a.n_reb_scatter);
        return;
    }
    if (!a.do_scan) return;
    if (a.scan_gate && *a.scan_gate == 0) return;
    mid_scan<16>(a.sys[b3], b3, a.count, a.start);
}

// ---------------------------------------------------------------------------
// k_kforce: one lane per particle; a block holds 4 waves, each group of
// SPLIT waves shares one 64-particle tile and splits its modes; partial
// forces are combined in LDS in a fixed order.  Mode constants are
// wave-uniform scalar loads.  With scatter on, the lane also moves its
// particle record into cell order (slot = cell start + rank).
// ---------------------------------------------------------------------------
template <typename T, typename KM>
struct ForceArgs {
    const SysDev *sys;
    const Tile *tiles;
    int ntiles;
    const T *pos;
    const T *q;
    int64_t ntot;
    const KM *km;
    T *F;
    int accumulate;
    int32_t *flag;
    // scatter
    int do_scatter;
    const int32_t *start;
    const int32_t *cellid;
    const int32_t *rank;
    const void *packed;
    int32_t *sorted_idx;
    void *sorted;
    // gridDim.y > 1: the mode list is split over y; partial sums go to
    // fpart[y][3][ntot] and k_fsum finishes the particles
    T *fpart;
    int single_n;   // single-system context (SINGLE launches): its particle count
    int single_p;   // and its mode count
};

template <typename T, typename KM, int SPLIT, bool SINGLE>
__global__ __launch_bounds__(256) void k_kforce(ForceArgs<T, KM> a)
{
    __shared__ T red[4][3][64];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int group = wave / SPLIT, part = wave % SPLIT;
    const int ti = blockIdx.x * (4 / SPLIT) + group;
    T fx = 0, fy = 0, fz = 0;
    int64_t i = -1;
    T qi = 0;
    int sysi = 0;
    if (ti < a.ntiles) {
        // SINGLE: the host's 64-particle tile of a single system, formed here
        const Tile t = SINGLE ? Tile{0, 64 * ti, min(64, a.single_n - 64 * ti), 0} : a.tiles[ti];
        sysi = t.sys;
        SysDev S = a.sys[SINGLE ? 0 : t.sys];
        if constexpr (SINGLE) {
            // offsets 0 and the mode count from the launch: the position and
            // mode-constant loads do not wait for the system constants
            S.off = 0;
            S.moff = 0;
            S.p = a.single_p;
        }
        double s3[3] = {0.0, 0.0, 0.0};
        if (lane < t.count) {
            i = S.off + t.start + lane;
            for (int d = 0; d < 3; ++d) s3[d] = frac01((double)a.pos[d * a.ntot + i] * S.invL);
            qi = a.q[i];
        }
        const int64_t nparts = (int64_t)SPLIT * gridDim.y, gp = (int64_t)blockIdx.y * SPLIT + part;
        const int l0 = (int)((S.p * gp) / nparts), l1 = (int)((S.p * (gp + 1)) / nparts);
        const KM *kk = a.km + S.moff;
        T f[3] = {0, 0, 0};
        if constexpr (sizeof(T) == 4) {
            float h[3], lo[3];
            for (int d = 0; d < 3; ++d) split_frac(s3[d], S, h[d], lo[d]);
            fourier_range(kk, l0, l1, h, lo, f);
        } else {
            fourier_range(kk, l0, l1, s3, f);
        }
        fx = f[0];
        fy = f[1];
        fz = f[2];
    }
    if constexpr (SPLIT > 1) {
        red[wave][0][lane] = fx;
        red[wave][1][lane] = fy;
        red[wave][2][lane] = fz;
        __syncthreads();
        if (part != 0) return;
        for (int s = 1; s < SPLIT; ++s) {
            fx += red[wave + s][0][lane];
            fy += red[wave + s][1][lane];
            fz += red[wave + s][2][lane];
        }
    }
    if (i < 0) return;
    if (gridDim.y > 1) {
        T *fp = a.fpart + (int64_t)blockIdx.y * 3 * a.ntot;
        fp[i] = fx;
        fp[a.ntot + i] = fy;
        fp[2 * a.ntot + i] = fz;
        return;
    }
    fx *= -qi;
    fy *= -qi;
    fz *= -qi;
    if (!isfinite(fx + fy + fz)) atomicOr(a.flag, kFlagNonFinite);
    if (a.accumulate) {
        fx += a.F[i];
        fy += a.F[a.ntot + i];
        fz += a.F[2 * a.ntot + i];
    }
    a.F[i] = fx;
    a.F[a.ntot + i] = fy;
    a.F[2 * a.ntot + i] = fz;
    if (a.do_scatter) {
        const int slot = a.start[a.cellid[i] + sysi] + a.rank[i];
        const SysDev &S = a.sys[sysi];
        if (slot < S.off || slot >= S.off + S.n) {
            atomicOr(a.flag, kFlagBounds);
            return;
        }
        a.sorted_idx[slot] = (int32_t)i;
        if constexpr (sizeof(T) == 4)
            reinterpret_cast<PackF *>(a.sorted)[slot] = reinterpret_cast<const PackF *>(a.packed)[i];
        else
            reinterpret_cast<PartD *>(a.sorted)[slot] = reinterpret_cast<const PartD *>(a.packed)[i];
    }
}

// Sum of the mode-split partial forces in a fixed order, then the charge
// factor, the finiteness check and the store (or accumulation).
template <typename T>
__global__ __launch_bounds__(256) void k_fsum(const T *__restrict__ fpart, int ysplit, const T *__restrict__ q,
                                              int64_t ntot, T *__restrict__ F, int accumulate, int32_t *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    T f[3] = {0, 0, 0};
    for (int y = 0; y < ysplit; ++y)
        for (int d = 0; d < 3; ++d) f[d] += fpart[((int64_t)y * 3 + d) * ntot + i];
    const T qi = q[i];
    for (int d = 0; d < 3; ++d) f[d] *= -qi;
    if (!isfinite(f[0] + f[1] + f[2])) atomicOr(flag, kFlagNonFinite);
    for (int d = 0; d < 3; ++d) F[d * ntot + i] = accumulate ? F[d * ntot + i] + f[d] : f[d];
}

// ---------------------------------------------------------------------------
// Adjoint of the force at a fixed mode sample.  With G_i = dLoss/dF_i,
//   w_il = G_i . a_l,  A_l = sum_i q_i w_il cos th_il,  B_l = sum_i q_i w_il sin th_il,
//   dLoss/dq_i = -sum_l [w_il (cos th S_l - sin th C_l) + A_l sin th - B_l cos th],
//   dLoss/dr_i = q_i sum_l k_l [w_il (sin th S_l + cos th C_l) - A_l cos th - B_l sin th],
// k_l = 2 pi m_l / L.  The (A, B) reduction has the shape of the structure
// factor and reuses its tiling; the gather has the shape of the force pass.
// ---------------------------------------------------------------------------
// LDS record of the adjoint reduction: the particle's phase inputs and
// q_i G_i.  Single precision takes the phase from the exact split of the box
// fraction (the same phases as the forward passes), double the fraction.
template <typename T>
struct VjpRec;
template <>
struct VjpRec<float> {
    struct alignas(16) type {
        float hx, hy, hz, lx, ly, lz, gx, gy, gz, pad[3];
    };
};
template <>
struct VjpRec<double> {
    struct alignas(16) type {
        double x, y, z, gx, gy, gz;
    };
};

__device__ __forceinline__ void vjp_record(const SysDev &S, double sx, double sy, double sz, float gx, float gy,
                                           float gz, VjpRec<float>::type &v)
{
    split_frac(sx, S, v.hx, v.lx);
    split_frac(sy, S, v.hy, v.ly);
    split_frac(sz, S, v.hz, v.lz);
    v.gx = gx;
    v.gy = gy;
    v.gz = gz;
    v.pad[0] = v.pad[1] = v.pad[2] = 0.0f;
}

__device__ __forceinline__ void vjp_record(const SysDev &, double sx, double sy, double sz, double gx, double gy,
                                           double gz, VjpRec<double>::type &v)
{
    v.x = sx;
    v.y = sy;
    v.z = sz;
    v.gx = gx;
    v.gy = gy;
    v.gz = gz;
}

// sin and cos of a record's phase for mode m.
__device__ __forceinline__ void vjp_sincos(const VjpRec<float>::type &v, float mx, float my, float mz, float &sn,
                                           float &cs)
{
    const float rf = phase_split(mx, my, mz, v.hx, v.hy, v.hz, v.lx, v.ly, v.lz);
    sn = __builtin_amdgcn_sinf(rf);
    cs = __builtin_amdgcn_cosf(rf);
}

__device__ __forceinline__ void vjp_sincos(const VjpRec<double>::type &v, double mx, double my, double mz,
                                           double &sn, double &cs)
{
    sincospi(2.0 * wrap_rev(fma(mx, v.x, fma(my, v.y, mz * v.z))), &sn, &cs);
}

template <typename T, typename KM, int BS>
__global__ __launch_bounds__(BS) void k_vjp_reduce(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                   const T *__restrict__ pos, const T *__restrict__ q,
                                                   const T *__restrict__ gF, int64_t ntot,
                                                   const KM *__restrict__ km, double *__restrict__ partial,
                                                   const int32_t *__restrict__ part_off)
{
    using VR = typename VjpRec<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    const SysDev S = sys[t.sys];
    VR *sp = reinterpret_cast<VR *>(smem);
    double2 *red = reinterpret_cast<double2 *>(smem + sizeof(VR) * t.count);
    const int tid = threadIdx.x;
    const int count = t.count;
    for (int j = tid; j < count; j += BS) {
        const int64_t i = S.off + t.start + j;
        const T qi = q[i];
        VR v;
        vjp_record(S, frac01((double)pos[i] * S.invL), frac01((double)pos[ntot + i] * S.invL),
                   frac01((double)pos[2 * ntot + i] * S.invL), qi * gF[i], qi * gF[ntot + i],
                   qi * gF[2 * ntot + i], v);
        sp[j] = v;
    }
    __syncthreads();
    const int P = S.p;
    const int Pt = P < BS ? P : BS;
    const int G = BS / Pt;
    double *prow = partial + 2 * ((int64_t)part_off[t.sys] + (int64_t)t.aux * P);
    for (int m0 = 0; m0 < P; m0 += Pt) {
        const int lt = tid % Pt, g = tid / Pt;
        const int l = m0 + lt;
        const bool act = g < G && l < P;
        double A = 0.0, B = 0.0;
        if (act) {
            const KM k = km[S.moff + l];
            const T mx = (T)k.m[0], my = (T)k.m[1], mz = (T)k.m[2];
            const T ax = (T)k.a[0], ay = (T)k.a[1], az = (T)k.a[2];
            for (int j0 = g; j0 < count; j0 += 8 * G) {
                T a8 = 0, b8 = 0;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int j = j0 + u * G;
                    if (j < count) {
                        const VR v = sp[j];
                        T sn, cs;
                        vjp_sincos(v, mx, my, mz, sn, cs);
                        const T w = fma(v.gx, ax, fma(v.gy, ay, v.gz * az));
                        a8 = fma(w, cs, a8);
                        b8 = fma(w, sn, b8);
                    }
                }
                A += (double)a8;
                B += (double)b8;
            }
        }
        red[tid] = make_double2(A, B);
        __syncthreads();
        if (tid < Pt && l < P) {
            double av = 0.0, bv = 0.0;
            for (int gg = 0; gg < G; ++gg) {
                const double2 v = red[gg * Pt + lt];
                av += v.x;
                bv += v.y;
            }
            prow[2 * l] = av;
            prow[2 * l + 1] = bv;
        }
        if (m0 + Pt < P) __syncthreads();   // red is reused by the next mode tile
    }
}

template <typename KM, typename KV>
__global__ __launch_bounds__(64) void k_vjp_final(const SysDev *__restrict__ sys, const double *__restrict__ partial,
                                                  const int32_t *__restrict__ part_off, int R,
                                                  const KM *__restrict__ km, double *__restrict__ ab,
                                                  KV *__restrict__ kv)
{
    const int r = blockIdx.y;
    const SysDev S = sys[r];
    const int l = blockIdx.x;
    if (l >= S.p) return;
    const int nt = part_off[R + r];
    const double *base = partial + 2 * (int64_t)part_off[r];
    double av = 0.0, bv = 0.0;
    for (int t = threadIdx.x; t < nt; t += 64) {
        av += base[2 * ((int64_t)t * S.p + l)];
        bv += base[2 * ((int64_t)t * S.p + l) + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        av += __shfl_down(av, off, 64);
        bv += __shfl_down(bv, off, 64);
    }
    if (threadIdx.x == 0) {
        const int o = S.moff + l;
        ab[2 * o] = av;
        ab[2 * o + 1] = bv;
        const KM k = km[o];
        KV v;
        const double tp = 2.0 * kPi * S.invL;
        for (int d = 0; d < 3; ++d) {
            v.m[d] = k.m[d];
            v.a[d] = k.a[d];
            v.k[d] = tp * k.m[d];
        }
        v.C = k.C;
        v.S = k.S;
        v.A = av;
        v.B = bv;
        if constexpr (sizeof(KV) == sizeof(KVjpF)) v.pad[0] = v.pad[1] = v.pad[2] = 0.0f;
        kv[o] = v;
    }
}

template <typename T, typename KV, int SPLIT>
__global__ __launch_bounds__(256) void k_vjp_gather(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                    int ntiles, const T *__restrict__ pos, const T *__restrict__ q,
                                                    const T *__restrict__ gF, int64_t ntot,
                                                    const KV *__restrict__ kv, T *__restrict__ gpos,
                                                    T *__restrict__ gq)
{
    __shared__ T red[4][4][64];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int group = wave / SPLIT, part = wave % SPLIT;
    const int ti = blockIdx.x * (4 / SPLIT) + group;
    T dq = 0, rx = 0, ry = 0, rz = 0;
    int64_t i = -1;
    T qi = 0;
    if (ti < ntiles) {
        const Tile t = tiles[ti];
        const SysDev S = sys[t.sys];
        double sx = 0.0, sy = 0.0, sz = 0.0;
        T gx = 0, gy = 0, gz = 0;
        if (lane < t.count) {
            i = S.off + t.start + lane;
            sx = frac01((double)pos[i] * S.invL);
            sy = frac01((double)pos[ntot + i] * S.invL);
            sz = frac01((double)pos[2 * ntot + i] * S.invL);
            qi = q[i];
            gx = gF[i];
            gy = gF[ntot + i];
            gz = gF[2 * ntot + i];
        }
        const int64_t nparts = (int64_t)SPLIT * gridDim.y, gp = (int64_t)blockIdx.y * SPLIT + part;
        const int l0 = (int)((S.p * gp) / nparts), l1 = (int)((S.p * (gp + 1)) / nparts);
        const KV *kk = kv + S.moff;
        typename VjpRec<T>::type rec;
        vjp_record(S, sx, sy, sz, (T)0, (T)0, (T)0, rec);
#pragma unroll 2
        for (int l = l0; l < l1; ++l) {
            const KV k = kk[l];
            T sn, cs;
            vjp_sincos(rec, (T)k.m[0], (T)k.m[1], (T)k.m[2], sn, cs);
            const T w = fma(gx, (T)k.a[0], fma(gy, (T)k.a[1], gz * (T)k.a[2]));
            const T Ck = (T)k.C, Sk = (T)k.S, Ak = (T)k.A, Bk = (T)k.B;
            dq -= fma(w, cs * Sk - sn * Ck, Ak * sn - Bk * cs);
            const T tt = fma(w, sn * Sk + cs * Ck, -(Ak * cs + Bk * sn));
            rx = fma(tt, (T)k.k[0], rx);
            ry = fma(tt, (T)k.k[1], ry);
            rz = fma(tt, (T)k.k[2], rz);
        }
    }
    if constexpr (SPLIT > 1) {
        red[wave][0][lane] = dq;
        red[wave][1][lane] = rx;
        red[wave][2][lane] = ry;
        red[wave][3][lane] = rz;
        __syncthreads();
        if (part != 0) return;
        for (int s = 1; s < SPLIT; ++s) {
            dq += red[wave + s][0][lane];
            rx += red[wave + s][1][lane];
            ry += red[wave + s][2][lane];
            rz += red[wave + s][3][lane];
        }
    }
    if (i < 0) return;
    gq[i] = dq;
    gpos[i] = qi * rx;
    gpos[ntot + i] = qi * ry;
    gpos[2 * ntot + i] = qi * rz;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_sample(const LaunchCfg &c, const Workspace &w, uint64_t step, int use_mh)
{
    if (use_mh) {
        launch_k(k_sample_mh, dim3(c.R), dim3(64), 0, c.stream, w.sys, w.mh_state, w.modes, w.mode_w, c.mcap, step);
    } else {
        const int table_lds = c.max_table <= 8192 ? 1 : 0;
        const size_t sm = table_lds ? sizeof(double) * c.max_table : 0;
        dim3 g((c.max_p + 255) / 256, c.R);
        launch_k(k_sample_exact, g, dim3(256), sm, c.stream, w.sys, w.cdf, w.modes, w.mode_w, c.mcap, step, table_lds);
    }
    return hipGetLastError();
}

size_t stage_lds_bytes(const LaunchCfg &c, int sample_in_kernel, int *table_lds, int *tab_max)
{
    size_t base = sizeof(PartD) * (c.rho_chunk + kRhoUnroll * kRhoGroupsMax) + sizeof(double2) * c.rho_block +
                  sizeof(int) * 3 * c.rho_block;
    *table_lds = 0;
    *tab_max = 0;
    if (sample_in_kernel && base + sizeof(double) * c.max_table <= 64 * 1024) {
        *table_lds = 1;
        *tab_max = c.max_table;
    }
    return base + sizeof(double) * (*tab_max);
}

template <typename T, int BS, bool SINGLE>
static void stage_launch_bs(int var, dim3 g, size_t sm, hipStream_t st, const StageArgs<T> &a)
{
    if (var == 2)
        launch_k(k_stage_rho<T, BS, 2, SINGLE>, g, BS, sm, st, a);
    else if (var == 1)
        launch_k(k_stage_rho<T, BS, 1, SINGLE>, g, BS, sm, st, a);
    else
        launch_k(k_stage_rho<T, BS, 0, SINGLE>, g, BS, sm, st, a);
}

template <typename T, bool SINGLE>
static void stage_launch(int block, int var, dim3 g, size_t sm, hipStream_t st, const StageArgs<T> &a)
{
    if (block == 256)
        stage_launch_bs<T, 256, SINGLE>(var, g, sm, st, a);
    else if (block == 512)
        stage_launch_bs<T, 512, SINGLE>(var, g, sm, st, a);
    else
        stage_launch_bs<T, 1024, SINGLE>(var, g, sm, st, a);
}

template <typename T>
static hipError_t stage_dispatch(const LaunchCfg &c, const Workspace &w, const StageRequest &rq)
{
    StageArgs<T> a;
    a.sys = w.sys;
    a.tiles = w.rho_tiles;
    a.pos = (T *)rq.pos;
    a.vel = (T *)rq.vel;
    a.F = (const T *)rq.force;
    a.q = (const T *)rq.q;
    a.ntot = c.ntot;
    a.cdf = w.cdf;
    a.modes = w.modes;
    a.mode_w = w.mode_w;
    a.mcap = c.mcap;
    a.partial = w.partial;
    a.part_off = w.partial_off;
    a.count = w.cell_count;
    a.cellid = w.cellid;
    a.rank = w.rank;
    a.packed = w.packed;
    a.step = rq.step;
    a.sample_step = rq.sample_step;
    a.do_integrate = rq.integrate;
    a.kick = rq.kick;
    a.do_bin = rq.bin;
    a.do_sample = rq.sample;
    a.do_rho = rq.rho;
    a.chunk = c.rho_chunk;
    a.list_mode = rq.list ? 1 : 0;
    if (rq.list) a.ls = *rq.list;
    a.slot_of = w.slot_of;
    a.sorted = w.sorted;
    a.ref = w.ref;
    int table_lds, tab_max;
    const size_t sm = stage_lds_bytes(c, rq.sample, &table_lds, &tab_max);
    a.table_lds = table_lds;
    a.tab_max = tab_max;
    a.single_n = c.R == 1 ? (int)c.ntot : 0;
    a.single_p = c.R == 1 ? c.max_p : 0;
    dim3 g(c.n_rho_tiles, rq.mode_split > 1 ? rq.mode_split : 1);
    const int var = (rq.integrate || rq.bin || rq.list) ? 2 : (rq.sample ? 1 : 0);
    if (c.R == 1)
        stage_launch<T, true>(c.rho_block, var, g, sm, c.stream, a);
    else
        stage_launch<T, false>(c.rho_block, var, g, sm, c.stream, a);
    return hipGetLastError();
}

hipError_t launch_stage(const LaunchCfg &c, const Workspace &w, const StageRequest &rq)
{
    return c.prec == RBE_FP64 ? stage_dispatch<double>(c, w, rq) : stage_dispatch<float>(c, w, rq);
}

// Binning and scatter blocks of a list rebuild (each also capped at one per
// four 256-particle tiles).  On steps without a rebuild each costs its
// dispatch; with the flag hand-offs free of L2 write-backs and invalidations
// the rebuild itself scales with them (measured at N = 1e5 and 1e6: 16 -> 128
// blocks, step 41.3 -> 40.5 and 260 -> 255 us).
constexpr int kRebBlocks = 128;

template <typename KM>
static hipError_t mid_dispatch(const LaunchCfg &c, const Workspace &w, int do_final, int do_scan,
                               const int32_t *gate, const int32_t *bin_gate, int32_t *clear_flag, int sample_next,
                               uint64_t sample_step, const ListStep *ls)
{
    MidArgs<KM> a;
    a.sys = w.sys;
    a.R = c.R;
    a.max_p = c.max_p;
    a.final_lw = final_waves_log2(c.max_sys_rho_tiles);
    const int final_modes = 16 >> a.final_lw;   // modes per totals block
    a.n_final_blocks = do_final ? (c.R * c.max_p + final_modes - 1) / final_modes : 0;
    a.single_p = c.R == 1 ? c.max_p : 0;
    a.single_nt = c.n_rho_tiles;
    a.partial = w.partial;
    a.part_off = w.partial_off;
    a.modes = w.modes;
    a.mode_w = w.mode_w;
    a.mcap = c.mcap;
    a.rho = w.rho;
    a.km = (KM *)w.kmode;
    a.count = w.cell_count;
    a.start = w.cell_start;
    a.do_scan = do_scan;
    a.scan_gate = gate;
    a.bin_gate = bin_gate;
    a.n_bin_blocks = bin_gate ? std::min(kRebBlocks, (c.n_part_tiles + 3) / 4) : 0;
    a.part_tiles = w.part_tiles;
    a.n_part_tiles = c.n_part_tiles;
    a.packed = w.packed;
    a.cellid = w.cellid;
    a.rank = w.rank;
    a.n_sample_blocks = sample_next ? c.R : 0;
    a.sample_step = sample_step;
    a.cdf = w.cdf;
    a.table_lds = sample_next && c.max_table <= 6144 ? 1 : 0;
    a.modes_next = w.modes_alt;
    a.mode_w_next = w.mode_w_alt;
    a.clear_flag = clear_flag;
    a.step_base = ls ? ls->step_base : nullptr;
    // a list step: the gated rebuild runs in this launch
    a.reb = ls && bin_gate ? 1 : 0;
    a.n_reb_scatter = a.reb ? std::min(kRebBlocks, (c.n_part_tiles + 3) / 4) : 0;
    if (a.reb) {
        RebuildArgs &r = a.rb;
        r.sys = w.sys;
        r.R = c.R;
        r.gate = bin_gate;
        r.ready = ls->ready;
        r.count = w.cell_count;
        r.start = w.cell_start;
        r.part_tiles = w.part_tiles;
        r.n_part_tiles = c.n_part_tiles;
        r.cellid = w.cellid;
        r.rank = w.rank;
        r.packed = w.packed;
        r.sorted_idx = w.sorted_idx;
        r.sorted = w.sorted;
        r.slot_of = w.slot_of;
        r.ref = w.ref;
        r.overflow = ls->overflow;
        r.builds = ls->rebuilds;
        r.flag = w.flag;
        r.bins_done = ls->bins_done;
        r.n_bin = a.n_bin_blocks;
        r.poison = ls->poison;
        r.wait_limit = c.wait_limit;
    }
    const size_t sm = a.table_lds ? sizeof(double) * c.max_table : 0;
    const int nb = a.n_final_blocks + a.n_bin_blocks + a.n_sample_blocks + (do_scan ? c.R : 0) +
                   (a.reb ? 1 + a.n_reb_scatter : 0);
    if (nb == 0) return hipSuccess;
    const bool lean = !do_scan && !a.n_bin_blocks && !a.n_sample_blocks && !a.reb && !clear_flag;
    if (lean)
        launch_k(k_mid<KM, true>, nb, 1024, sm, c.stream, a);
    else
        launch_k(k_mid<KM, false>, nb, 1024, sm, c.stream, a);
    return hipGetLastError();
}

hipError_t launch_mid(const LaunchCfg &c, const Workspace &w, int do_final, int do_scan, const int32_t *gate,
                      const int32_t *bin_gate, int32_t *clear_flag, int sample_next, uint64_t sample_step,
                      const ListStep *ls)
{
    return c.prec == RBE_FP64 ? mid_dispatch<KModeD>(c, w, do_final, do_scan, gate, bin_gate, clear_flag,
                                                     sample_next, sample_step, ls)
                              : mid_dispatch<KModeF>(c, w, do_final, do_scan, gate, bin_gate, clear_flag,
                                                     sample_next, sample_step, ls);
}

template <typename T, typename KM, bool SINGLE>
static void kforce_launch(int split, int n, int ys, hipStream_t st, const ForceArgs<T, KM> &a)
{
    switch (split) {
    case 1:
        launch_k(k_kforce<T, KM, 1, SINGLE>, dim3((n + 3) / 4, ys), 256, 0, st, a);
        break;
    case 2:
        launch_k(k_kforce<T, KM, 2, SINGLE>, dim3((n + 1) / 2, ys), 256, 0, st, a);
        break;
    default:
        launch_k(k_kforce<T, KM, 4, SINGLE>, dim3(n, ys), 256, 0, st, a);
        break;
    }
}

template <typename T, typename KM>
static hipError_t kforce_dispatch(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q, void *F,
                                  int acc, int scatter, int mode_split)
{
    ForceArgs<T, KM> a;
    a.fpart = (T *)w.fpart;
    a.sys = w.sys;
    a.tiles = w.force_tiles;
    a.ntiles = c.n_force_tiles;
    a.pos = (const T *)pos;
    a.q = (const T *)q;
    a.ntot = c.ntot;
    a.km = (const KM *)w.kmode;
    a.F = (T *)F;
    a.accumulate = acc;
    a.flag = w.flag;
    a.do_scatter = scatter;
    a.start = w.cell_start;
    a.cellid = w.cellid;
    a.rank = w.rank;
    a.packed = w.packed;
    a.sorted_idx = w.sorted_idx;
    a.sorted = w.sorted;
    const int n = c.n_force_tiles;
    const int ys = mode_split > 1 && w.fpart ? mode_split : 1;
    a.single_n = c.R == 1 ? (int)c.ntot : 0;
    a.single_p = c.R == 1 ? c.max_p : 0;
    if (c.R == 1)
        kforce_launch<T, KM, true>(c.force_split, n, ys, c.stream, a);
    else
        kforce_launch<T, KM, false>(c.force_split, n, ys, c.stream, a);
    if (ys > 1)
        launch_k(k_fsum<T>, (int)((c.ntot + 255) / 256), 256, 0, c.stream, (const T *)w.fpart, ys, (const T *)q, c.ntot,
                                                                      (T *)F, acc, w.flag);
    return hipGetLastError();
}

hipError_t launch_kforce(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q, void *force,
                         int accumulate, int scatter, int mode_split)
{
    return c.prec == RBE_FP64 ? kforce_dispatch<double, KModeD>(c, w, pos, q, force, accumulate, scatter, mode_split)
                              : kforce_dispatch<float, KModeF>(c, w, pos, q, force, accumulate, scatter, mode_split);
}

template <typename T, typename KM>
static hipError_t vjp_reduce_dispatch(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                                      const void *gF)
{
    const size_t sm = sizeof(typename VjpRec<T>::type) * c.rho_chunk + sizeof(double2) * c.rho_block;
    const T *p = (const T *)pos, *qq = (const T *)q, *g = (const T *)gF;
    const KM *km = (const KM *)w.kmode;
    dim3 gr(c.n_rho_tiles);
    switch (c.rho_block) {
    case 256:
        launch_k(k_vjp_reduce<T, KM, 256>, gr, 256, sm, c.stream, w.sys, w.rho_tiles, p, qq, g, c.ntot, km, w.partial,
                                                            w.partial_off);
        break;
    case 512:
        launch_k(k_vjp_reduce<T, KM, 512>, gr, 512, sm, c.stream, w.sys, w.rho_tiles, p, qq, g, c.ntot, km, w.partial,
                                                            w.partial_off);
        break;
    default:
        launch_k(k_vjp_reduce<T, KM, 1024>, gr, 1024, sm, c.stream, w.sys, w.rho_tiles, p, qq, g, c.ntot, km, w.partial,
                                                              w.partial_off);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_vjp_reduce(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                             const void *gF)
{
    return c.prec == RBE_FP64 ? vjp_reduce_dispatch<double, KModeD>(c, w, pos, q, gF)
                              : vjp_reduce_dispatch<float, KModeF>(c, w, pos, q, gF);
}

hipError_t launch_vjp_final(const LaunchCfg &c, const Workspace &w)
{
    dim3 g(c.max_p, c.R);
    if (c.prec == RBE_FP64)
        launch_k(k_vjp_final<KModeD, KVjpD>, g, 64, 0, c.stream, w.sys, w.partial, w.partial_off, c.R,
                                                           (const KModeD *)w.kmode, w.ab, (KVjpD *)w.kvjp);
    else
        launch_k(k_vjp_final<KModeF, KVjpF>, g, 64, 0, c.stream, w.sys, w.partial, w.partial_off, c.R,
                                                           (const KModeF *)w.kmode, w.ab, (KVjpF *)w.kvjp);
    return hipGetLastError();
}

template <typename T, typename KV>
static hipError_t vjp_gather_dispatch(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                                      const void *gF, void *gpos, void *gq)
{
    const T *p = (const T *)pos, *qq = (const T *)q, *g = (const T *)gF;
    const KV *kv = (const KV *)w.kvjp;
    const int n = c.n_force_tiles;
    switch (c.force_split) {
    case 1:
        launch_k(k_vjp_gather<T, KV, 1>, (n + 3) / 4, 256, 0, c.stream, w.sys, w.force_tiles, n, p, qq, g, c.ntot, kv,
                                                                  (T *)gpos, (T *)gq);
        break;
    case 2:
        launch_k(k_vjp_gather<T, KV, 2>, (n + 1) / 2, 256, 0, c.stream, w.sys, w.force_tiles, n, p, qq, g, c.ntot, kv,
                                                                  (T *)gpos, (T *)gq);
        break;
    default:
        launch_k(k_vjp_gather<T, KV, 4>, n, 256, 0, c.stream, w.sys, w.force_tiles, n, p, qq, g, c.ntot, kv, (T *)gpos,
                                                        (T *)gq);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_vjp_gather(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                             const void *gF, void *gpos, void *gq)
{
    return c.prec == RBE_FP64 ? vjp_gather_dispatch<double, KVjpD>(c, w, pos, q, gF, gpos, gq)
                              : vjp_gather_dispatch<float, KVjpF>(c, w, pos, q, gF, gpos, gq);
}

}  // namespace rbe

namespace rbe {

// ---------------------------------------------------------------------------
// Context-free Fourier force (the no-allocation entry point): the system
// constants, the tiles of both passes, the partial offsets and the weights
// S/p are written by this kernel into the workspace the caller points to
// (kernel arguments are copied at launch, so no host buffer outlives the
// call).  Tiles follow the same rules as a context's.
// ---------------------------------------------------------------------------
__global__ void k_static_setup(SysDev sys, int chunk, int nrho, int nforce, SysDev *sysp, Tile *rho_tiles,
                               Tile *force_tiles, int32_t *part_off, double *mode_w)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *sysp = sys;
        part_off[0] = 0;
        part_off[1] = nrho;
    }
    if (i < nrho) rho_tiles[i] = Tile{0, i * chunk, min(chunk, sys.n - i * chunk), i};
    if (i < nforce) force_tiles[i] = Tile{0, i * 64, min(64, sys.n - i * 64), 0};
    if (i < sys.p) mode_w[i] = sys.S / (double)sys.p;
}

hipError_t launch_static_setup(const LaunchCfg &c, const Workspace &w, const SysDev &sys)
{
    const int most = std::max(std::max(c.n_rho_tiles, c.n_force_tiles), std::max(sys.p, 1));
    launch_k(k_static_setup, (most + 255) / 256, 256, 0, c.stream, sys, c.rho_chunk, c.n_rho_tiles, c.n_force_tiles,
                                                             w.sys, w.rho_tiles, w.force_tiles, w.partial_off,
                                                             w.mode_w);
    return hipGetLastError();
}

}  // namespace rbe
