// Device roles of the launch that follows the staging launch (k_mid):
// structure-factor totals and per-mode force constants, the next step's
// modes, and the gated neighbour-list rebuild (binning, cell scan, scatter
// into cell order).  Loops that depend on the block size take their shape
// from blockDim.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "rbe_device.h"
#include "rbe_internal.h"

namespace rbe {

// What the force constants of one mode take besides its structure factor:
// the mode, its weight and the system's constants, and its index o in the
// mode arrays.  The totals load these before the partial sums, so that their
// latency overlaps the sums.
struct KModeIn {
    double mx, my, mz, w, coulomb, L;
    int o;
};

__device__ __forceinline__ KModeIn kmode_in(const SysDev &S, int moff, int l, const int32_t *modes,
                                            const double *mode_w, int mcap)
{
    KModeIn in;
    in.o = moff + l;
    in.mx = modes[in.o];
    in.my = modes[mcap + in.o];
    in.mz = modes[2 * mcap + in.o];
    in.w = mode_w[in.o];
    in.coulomb = S.coulomb;
    in.L = S.L;
    return in;
}

// Structure factor totals and force constants of mode in.o:
//   a_l = coulomb w_l 2 m_l / (L^2 |m_l|^2)   (eq. 3.6 with k = 2 pi m / L).
template <typename KM>
__device__ __forceinline__ void make_kmode(const KModeIn &in, double c, double s, double *rho, KM *km)
{
    const int o = in.o;
    rho[2 * o] = c;
    rho[2 * o + 1] = s;
    const double mx = in.mx, my = in.my, mz = in.mz;
    const double m2 = mx * mx + my * my + mz * mz;
    const double f = in.coulomb * in.w * 2.0 / (in.L * in.L * m2);
    KM k;
    k.m[0] = mx;
    k.m[1] = my;
    k.m[2] = mz;
    k.a[0] = f * mx;
    k.a[1] = f * my;
    k.a[2] = f * mz;
    k.C = c;
    k.S = s;
    km[o] = k;
}

// Gated list rebuild: binning blocks, then one scan block, then scatter
// blocks, ordered by bounded device flags.
struct RebuildArgs {
    const SysDev *sys;
    int R;
    const int32_t *gate;
    int32_t *ready;
    int32_t *count;
    int32_t *start;
    const Tile *part_tiles;
    int n_part_tiles;
    const int32_t *cellid;
    const int32_t *rank;
    const void *packed;
    int32_t *sorted_idx;
    void *sorted;
    int32_t *slot_of;
    void *ref;
    int32_t *overflow;
    int32_t *builds;
    int32_t *flag;
    int32_t *bins_done;     // binning blocks finished (reset by the staging launch)
    int n_bin;              // binning blocks of the launch
    int32_t *poison;        // raised when a wait gives up, cleared by a complete scan
    int wait_limit;         // spin bound of every wait
};

template <typename KM>
struct MidArgs {
    const SysDev *sys;
    int R, max_p;
    int n_final_blocks;   // blocks doing the structure-factor totals
    int single_p;         // single-system context: its mode count (else 0) ...
    int single_nt;        // ... and its structure-factor tile count
    int final_lw;         // log2 of the waves per mode of the totals (0 or 2)
    const double *partial;
    const int32_t *part_off;   // [2R]: partial offsets, then tile counts
    const int32_t *modes;
    const double *mode_w;
    int mcap;
    double *rho;
    KM *km;
    int32_t *count;
    int32_t *start;
    int do_scan;
    const int32_t *scan_gate;   // when set, the scan runs only if *scan_gate != 0
    // binning of a list rebuild (blocks after the totals), only if *bin_gate != 0
    const int32_t *bin_gate;
    int n_bin_blocks;
    const Tile *part_tiles;
    int n_part_tiles;
    const void *packed;
    int32_t *cellid;
    int32_t *rank;
    // the next step's modes (one block per system), and a flag to clear
    int n_sample_blocks;
    uint64_t sample_step;
    const double *cdf;
    int table_lds;
    int32_t *modes_next;
    double *mode_w_next;
    int32_t *clear_flag;
    const uint64_t *step_base;   // added to sample_step when set
    // list rebuild (gated by bin_gate): one scan block and n_reb_scatter
    // scatter blocks after all the others
    int reb;
    int n_reb_scatter;
    RebuildArgs rb;
};

// Up to 128 blocks, each striding over the 256-particle tiles: on the many
// steps where nothing is binned the launch costs only their dispatch.  A thread
// takes up to kRebBatch tiles at once: it loads all their records, then
// issues all the counter atomics, then stores the cell ids and ranks, so
// that the memory latencies of its particles overlap instead of adding up.
constexpr int kRebBatch = 8;

template <typename KM>
__device__ void mid_bin(const MidArgs<KM> &a, int b)
{
    const int k = threadIdx.x & 255;
    const int tpb = (int)(blockDim.x >> 8);   // 256-particle tiles per block and round
    const int stride = tpb * a.n_bin_blocks;
    for (int t0 = tpb * b + (int)(threadIdx.x >> 8); t0 < a.n_part_tiles; t0 += kRebBatch * stride) {
        int64_t idx[kRebBatch];
        int cell[kRebBatch];
#pragma unroll
        for (int u = 0; u < kRebBatch; ++u) {
            idx[u] = -1;
            cell[u] = 0;
            const int ti = t0 + u * stride;
            if (ti >= a.n_part_tiles) continue;
            const Tile t = a.part_tiles[ti];
            if (k >= t.count) continue;
            const SysDev &S = a.sys[t.sys];
            const int64_t i = S.off + t.start + k;
            int cx, cy, cz;
            if constexpr (sizeof(KM) == sizeof(KModeF)) {
                const PackF v = reinterpret_cast<const PackF *>(a.packed)[i];
                cx = cell_of_fix(v.x, S.nc);
                cy = cell_of_fix(v.y, S.nc);
                cz = cell_of_fix(v.z, S.nc);
            } else {
                const PartD v = reinterpret_cast<const PartD *>(a.packed)[i];
                cx = cell_of_frac(v.x, S.nc);
                cy = cell_of_frac(v.y, S.nc);
                cz = cell_of_frac(v.z, S.nc);
            }
            idx[u] = i;
            cell[u] = S.cell_off + (cz * S.nc + cy) * S.nc + cx;
        }
        int rk[kRebBatch];
#pragma unroll
        for (int u = 0; u < kRebBatch; ++u) rk[u] = idx[u] >= 0 ? atomicAdd(&a.count[cell[u]], 1) : 0;
#pragma unroll
        for (int u = 0; u < kRebBatch; ++u)
            if (idx[u] >= 0) {
                a.cellid[idx[u]] = cell[u];
                a.rank[idx[u]] = rk[u];
            }
    }
}


// Structure-factor totals, W = 2^final_lw waves per mode (1 or 4) and 16 / W
// modes per 1024-thread block: the wave of part q sums the tile partials of
// its mode in runs of 64 tiles q, q + W, q + 2W, ... (a lane its tile of
// each run, in order), the waves reduce across lanes, and the mode's first
// wave adds the W part sums in order and writes the force constants.  The
// partials of one mode sit a tile row apart (one cache line per tile), so
// four waves per mode quarter the chain of dependent load batches of a long
// tile list; a context whose systems all have at most 64 tiles takes one
// wave per mode and a quarter of the blocks.
int final_waves_log2(int max_tiles_per_system);

template <typename KM>
__device__ void mid_final(const MidArgs<KM> &a, int blk)
{
    __shared__ double2 q_sum[16];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lw = a.final_lw, W = 1 << lw;
    const int gm = (blk << (4 - lw)) + (wave >> lw);
    const int q = wave & (W - 1);
    const int r = gm / a.max_p, l = gm % a.max_p;
    // a single system's mode and tile counts come with the launch, so that
    // the partial loads do not wait for the system constants and offsets
    bool ok = r < a.R;
    int P = 0, nt = 0;
    const double *base = a.partial;
    if (ok) {
        P = a.single_p ? a.single_p : a.sys[r].p;
        ok = l < P;
        nt = a.single_p ? a.single_nt : a.part_off[a.R + r];
        base = a.partial + (a.single_p ? 0 : 2 * (int64_t)a.part_off[r]);
    }
    // the inputs of the force constants, loaded by the thread that forms them
    KModeIn in{};
    if (ok && q == 0 && lane == 0) {
        const SysDev &S = a.sys[r];
        in = kmode_in(S, a.single_p ? 0 : S.moff, l, a.modes, a.mode_w, a.mcap);
    }
    double c = 0.0, s = 0.0;
    if (ok) {
        // eight loads are issued before they are added, so their latencies overlap
        const int STRIDE = 64 * W;
        for (int t0 = 64 * q + lane; t0 < nt; t0 += 8 * STRIDE) {
            double2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + STRIDE * u;
                if (t < nt) v[u] = *reinterpret_cast<const double2 *>(base + 2 * ((int64_t)t * P + l));
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (t0 + STRIDE * u < nt) {
                    c += v[u].x;
                    s += v[u].y;
                }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            c += __shfl_down(c, off, 64);
            s += __shfl_down(s, off, 64);
        }
    }
    if (lane == 0) q_sum[wave] = make_double2(c, s);
    __syncthreads();
    if (ok && q == 0 && lane == 0) {
        double cc = 0.0, ss = 0.0;
        for (int k = 0; k < W; ++k) {
            cc += q_sum[wave + k].x;
            ss += q_sum[wave + k].y;
        }
        make_kmode<KM>(in, cc, ss, a.rho, a.km);
    }
}

// Exclusive scan of one system's cell counts with NW waves (64 NW threads).
// Cells are processed in passes of NCH chunks x 256 NW; thread t owns cells
// [base + g*256 NW + 4t, +4) of chunk g.  Cell offsets are padded to
// multiples of 4 so the counts load as int4.  Fewer chunks per pass hold
// fewer registers.
constexpr int kScanChunks = 8;

template <int NW, int NCH = kScanChunks>
__device__ void mid_scan(const SysDev &S, int r, int32_t *count, int32_t *start)
{
    constexpr int CH = 256 * NW;              // cells per chunk
    constexpr int NT = NCH * NW;              // wave totals per pass (at most 128)
    static_assert(NT <= 128, "one wave prefixes the wave totals, two per lane");
    __shared__ int wtot[NT];
    __shared__ int gpre[NT + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int32_t *cnt = count + S.cell_off;
    int32_t *st = start + S.cell_off + r;
    const int ncell = S.ncell;
    int carry = 0;
    for (int base = 0; base < ncell; base += NCH * CH) {
        int v[NCH][4];
        int s[NCH], incl[NCH];
#pragma unroll
        for (int g = 0; g < NCH; ++g) {
            const int idx = base + g * CH + 4 * tid;
            if (idx + 3 < ncell) {
                const int4 x = *reinterpret_cast<const int4 *>(cnt + idx);
                v[g][0] = x.x;
                v[g][1] = x.y;
                v[g][2] = x.z;
                v[g][3] = x.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) v[g][j] = (idx + j < ncell) ? cnt[idx + j] : 0;
            }
            s[g] = v[g][0] + v[g][1] + v[g][2] + v[g][3];
        }
#pragma unroll
        for (int g = 0; g < NCH; ++g) {
            incl[g] = wave_incl_scan(s[g]);
            if (lane == 63) wtot[g * NW + wave] = incl[g];
        }
        __syncthreads();
        if (wave == 0) {
            // exclusive prefix of the NT wave totals in (chunk, wave) order
            const int x0 = 2 * lane < NT ? wtot[2 * lane] : 0;
            const int x1 = 2 * lane + 1 < NT ? wtot[2 * lane + 1] : 0;
            const int inc = wave_incl_scan(x0 + x1);
            if (2 * lane < NT) gpre[2 * lane] = inc - x0 - x1;
            if (2 * lane + 1 < NT) gpre[2 * lane + 1] = inc - x1;
            if (lane == 63) gpre[NT] = inc;
        }
        __syncthreads();
#pragma unroll
        for (int g = 0; g < NCH; ++g) {
            const int idx = base + g * CH + 4 * tid;
            const int run = S.off + carry + gpre[g * NW + wave] + incl[g] - s[g];
            const int o[4] = {run, run + v[g][0], run + v[g][0] + v[g][1], run + v[g][0] + v[g][1] + v[g][2]};
            if (idx + 3 < ncell) {
                // whole groups of four: 16-byte stores (the starts of system
                // r are shifted by r entries, so they are aligned when r % 4 == 0)
                *reinterpret_cast<int4 *>(cnt + idx) = make_int4(0, 0, 0, 0);
                if ((r & 3) == 0) {
                    *reinterpret_cast<int4 *>(st + idx) = make_int4(o[0], o[1], o[2], o[3]);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) st[idx + j] = o[j];
                }
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (idx + j < ncell) {
                        st[idx + j] = o[j];
                        cnt[idx + j] = 0;
                    }
            }
        }
        carry += gpre[NT];
        __syncthreads();
    }
    if (tid == 0) st[ncell] = S.off + carry;
}

// ---------------------------------------------------------------------------
// List rebuild inside the totals launch (work only when the step's rebuild
// flag is set).  The binning blocks count their particles into the cells and
// then each adds one to bins_done; the scan block, which comes after them in
// block order, waits for all of them, scans every system's counts and raises
// `ready`; the scatter blocks, last in block order, wait for it and stride
// over the 256-particle tiles, moving records into cell order.  A block only
// waits for blocks of lower index, which are dispatched before it and do not
// wait for it, so every wait ends (with one block per compute unit the last
// scatter blocks of a large launch start when earlier blocks finish); the
// waits are bounded anyway.  A wait that reaches its bound gives up: it
// raises the timeout bit of the error word and the poison flag, and its
// block skips its work.  The
// force launch of that step then clears the cell counts (the scan that would
// have cleared them did not run) and the next step's staging launch asks for
// a rebuild; the cell pass of the failed step reads the previous cell starts,
// clamped to the system, so every access stays in bounds.  The staging
// launch of each step resets bins_done and ready.
// ---------------------------------------------------------------------------

// Thread 0 waits (at most `limit` polls) until *p reaches want; the block
// learns the outcome.  The polls are relaxed loads and one acquire follows
// the last: on gfx950 an agent-scope acquire invalidates the XCD's L2, so
// acquiring on every poll would keep evicting the data that the blocks still
// working on that XCD read.  The block's waves share thread 0's compute unit
// and L1, and the barrier orders their loads after its invalidation.
__device__ bool block_wait(int32_t *p, int want, int limit, int32_t *flag, int32_t *poison)
{
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        int ok = 0;
        for (int it = 0; it < limit; ++it) {
            if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) {
                ok = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (ok) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_s_waitcnt(0);   // the invalidation is done before the barrier
        } else {
            atomicOr(flag, kFlagTimeout);
            atomicOr(poison, 1);
        }
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Publishing a block's stores to the other blocks of the launch: every wave
// waits until its stores have reached the L2 (a workgroup barrier alone does
// not wait for them), then thread 0 alone writes the XCD's L2 back (an
// agent-scope release fence, which writes back every dirty line of that L2;
// issued by every wave, these write-backs took 15-30 us per hand-off).
// Thread 0 then raises the block's flag.
__device__ __forceinline__ void block_stores_done()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __builtin_amdgcn_s_waitcnt(0);   // the write-back has completed before the flag
    }
}

// Scan block of a rebuild: waits for every binning block, turns the cell
// counts of all systems into slot starts, clears the overflow flag, counts
// the build and releases the scatter blocks.
template <int NW, int NCH = kScanChunks>
__device__ void rebuild_scan(const RebuildArgs &a)
{
    if (!block_wait(a.bins_done, a.n_bin, a.wait_limit, a.flag, a.poison)) return;
    for (int r = 0; r < a.R; ++r) mid_scan<NW, NCH>(a.sys[r], r, a.count, a.start);
    __syncthreads();
    if (threadIdx.x == 0) {
        *a.overflow = 0;
        *a.builds += 1;
        *a.poison = 0;
    }
    block_stores_done();
    if (threadIdx.x == 0) __hip_atomic_store(a.ready, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Scatter block b of nb: moves records into cell order once the scan is out,
// and records each particle's slot and list reference record.  As in the
// binning, a thread loads everything for up to kScatBatch tiles before it
// stores (fewer than there: each holds a whole record).
constexpr int kScatBatch = 4;

template <typename Rec>
__device__ void rebuild_scatter(const RebuildArgs &a, int b, int nb)
{
    if (!block_wait(a.ready, 1, a.wait_limit, a.flag, a.poison)) return;
    const int k = threadIdx.x & 255;
    const int tpb = (int)(blockDim.x >> 8);
    const int stride = tpb * nb;
    // records move as 16-byte words (PackF: one, PartD: two)
    constexpr int W = (int)(sizeof(Rec) / sizeof(uint4));
    for (int t0 = tpb * b + (int)(threadIdx.x >> 8); t0 < a.n_part_tiles; t0 += kScatBatch * stride) {
        int idx[kScatBatch], cell[kScatBatch], rk[kScatBatch], sys[kScatBatch];
        uint4 v[kScatBatch][W];
#pragma unroll
        for (int u = 0; u < kScatBatch; ++u) {
            idx[u] = -1;
            sys[u] = 0;
            cell[u] = 0;
            rk[u] = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) v[u][q] = make_uint4(0, 0, 0, 0);
            const int ti = t0 + u * stride;
            if (ti < a.n_part_tiles) {
                const Tile t = a.part_tiles[ti];
                if (k < t.count) {
                    const int i = a.sys[t.sys].off + t.start + k;
                    idx[u] = i;
                    sys[u] = t.sys;
                    cell[u] = a.cellid[i];
                    rk[u] = a.rank[i];
#pragma unroll
                    for (int q = 0; q < W; ++q) v[u][q] = reinterpret_cast<const uint4 *>(a.packed)[(int64_t)i * W + q];
                }
            }
        }
        int slot[kScatBatch];
#pragma unroll
        for (int u = 0; u < kScatBatch; ++u) slot[u] = idx[u] >= 0 ? a.start[cell[u] + sys[u]] + rk[u] : 0;
#pragma unroll
        for (int u = 0; u < kScatBatch; ++u)
            if (idx[u] >= 0) {
                // a slot outside the system can only come from stale counts
                const SysDev &S = a.sys[sys[u]];
                if (slot[u] < S.off || slot[u] >= S.off + S.n) {
                    atomicOr(a.flag, kFlagBounds);
                    continue;
                }
                a.sorted_idx[slot[u]] = idx[u];
                a.slot_of[idx[u]] = slot[u];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    reinterpret_cast<uint4 *>(a.sorted)[(int64_t)slot[u] * W + q] = v[u][q];
                    reinterpret_cast<uint4 *>(a.ref)[(int64_t)idx[u] * W + q] = v[u][q];
                }
            }
    }
}


// Next step's modes of system b (exact sampler), drawn by one block; the
// cumulative table is read from tab when given (the caller has room for it in
// LDS), else from global memory.
template <typename KM>
__device__ void mid_sample(const MidArgs<KM> &a, int b, double *tab)
{
    const SysDev S = a.sys[b];
    const double *t = a.cdf + S.cdf_off;
    if (tab) {
        for (int k = threadIdx.x; k < 2 * S.M + 1; k += blockDim.x) tab[k] = t[k];
        __syncthreads();
        t = tab;
    }
    for (int l = threadIdx.x; l < S.p; l += blockDim.x) {
        int mx, my, mz;
        sample_mode(t, S.M, (uint32_t)l, S.seed, a.sample_step + (a.step_base ? *a.step_base : 0), mx, my, mz);
        const int o = S.moff + l;
        a.modes_next[o] = mx;
        a.modes_next[a.mcap + o] = my;
        a.modes_next[2 * a.mcap + o] = mz;
        a.mode_w_next[o] = S.S / (double)S.p;
    }
}

}  // namespace rbe
