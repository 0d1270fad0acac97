// rbe_kernels.hip -- gfx950 kernels of librbe.
//
// Paper: Jin, Li, Xu & Zhao, "A random batch Ewald method for particle
// systems with Coulomb interactions", arXiv:2010.01559.
//
// Data layout: SoA particle arrays [3][N_tot]; systems of a batch are
// contiguous runs inside each block.  Every launch covers all systems of a
// context through a tile list (system, first particle, count).
//
// Single-precision path: phases are formed in double from fractional
// coordinates s = frac(r/L) and the integer modes, wrapped to [-1/2, 1/2)
// revolutions, and only then rounded to float for the hardware sine/cosine
// (which take revolutions); sums over particles are blocked in float and
// folded into double; the cross-block reduction is double.  Real space keeps
// positions as 32-bit fixed-point fractions of the box, so that an unsigned
// difference reinterpreted as signed is the minimum-image displacement.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "rbe_internal.h"

namespace rbe {

// ---------------------------------------------------------------------------
// Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11)
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c.x;
        uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        uint32_t lo1 = 0xCD9E8D57u * c.z;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        U4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ U4 draw(uint32_t idx, uint32_t word1, uint64_t seed, uint64_t step)
{
    U4 c{idx, word1, (uint32_t)step, (uint32_t)(step >> 32)};
    return philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 53-bit uniform in [0,1): 27 bits of a, 26 bits of b.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Three standard normals for particle i at step: Box-Muller on
// u1 = (w0+1) 2^-32, u2 = w1 2^-32 (two normals) and on (w2+1) 2^-32, w3 2^-32
// (cosine branch), in double.
__device__ __forceinline__ void normals3(uint32_t i, uint64_t seed, uint64_t step, double xi[3])
{
    U4 r = draw(i, kTagLangevin, seed, step);
    const double k = 1.0 / 4294967296.0;
    double u1 = ((double)r.x + 1.0) * k, u2 = (double)r.y * k;
    double u3 = ((double)r.z + 1.0) * k, u4 = (double)r.w * k;
    double a = sqrt(-2.0 * log(u1)), b = sqrt(-2.0 * log(u3));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    xi[0] = a * c;
    xi[1] = a * s;
    xi[2] = b * cospi(2.0 * u4);
}

// ---------------------------------------------------------------------------
// Trigonometry of a phase given in revolutions
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_rev(double r, float *s, float *c)
{
    // r in [-1/2, 1/2]; v_sin/v_cos take revolutions
    float rf = (float)r;
    *s = __builtin_amdgcn_sinf(rf);
    *c = __builtin_amdgcn_cosf(rf);
}

__device__ __forceinline__ void sincos_rev(double r, double *s, double *c)
{
    sincospi(2.0 * r, s, c);
}

__device__ __forceinline__ double wrap_rev(double ph)
{
    return ph - rint(ph);
}

__device__ __forceinline__ double frac01(double x)
{
    double f = x - floor(x);
    return f >= 1.0 ? 0.0 : f;
}

// ---------------------------------------------------------------------------
// Mode sampling (Sec. 3.1, eqs. 3.3-3.5)
// ---------------------------------------------------------------------------

// Smallest table index whose cumulative mass exceeds u (the last entry is 1).
__device__ __forceinline__ int invert_cdf(const double *t, int K, double u)
{
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (u < t[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

__global__ void k_sample_exact(const SysDev *__restrict__ sys, const double *__restrict__ cdf,
                               int32_t *__restrict__ modes, double *__restrict__ mode_w, int mcap, uint64_t step)
{
    const SysDev &S = sys[blockIdx.y];
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= S.p) return;
    const double *t = cdf + S.cdf_off;
    const int K = 2 * S.M + 1;
    int mx = 0, my = 0, mz = 0;
    for (uint32_t a = 0; a < (1u << 22); ++a) {
        U4 r0 = draw((uint32_t)l, kTagSample | (2u * a), S.seed, step);
        U4 r1 = draw((uint32_t)l, kTagSample | (2u * a + 1u), S.seed, step);
        mx = invert_cdf(t, K, u53(r0.x, r0.y)) - S.M;
        my = invert_cdf(t, K, u53(r0.z, r0.w)) - S.M;
        mz = invert_cdf(t, K, u53(r1.x, r1.y)) - S.M;
        if (mx | my | mz) break;
    }
    const int o = S.moff + l;
    modes[o] = mx;
    modes[mcap + o] = my;
    modes[2 * mcap + o] = mz;
    mode_w[o] = S.S / (double)S.p;
}

// Proposal mass of eq. (3.5): P(round(x*) = m), x* ~ N(0, alpha L^2/(2 pi^2)).
__device__ double mh_qbar(double w, int m)
{
    int am = m < 0 ? -m : m;
    if (am == 0) return erf(0.5 / w);
    return 0.5 * (erf((am + 0.5) / w) - erf((am - 0.5) / w));
}

// The paper's Metropolis-Hastings chains, one wave per system, lanes 0..2 the
// three components; the chain states persist across calls.
__global__ void k_sample_mh(const SysDev *__restrict__ sys, int32_t *__restrict__ state, int32_t *__restrict__ modes,
                            double *__restrict__ mode_w, int mcap, uint64_t step)
{
    const SysDev &S = sys[blockIdx.x];
    const int d = threadIdx.x;
    const double a2 = kPi * kPi / (S.alpha * S.L * S.L);
    const double sd = sqrt(S.alpha * S.L * S.L / (2.0 * kPi * kPi));
    const double w = sqrt(S.alpha * S.L * S.L / (kPi * kPi));
    int cur = d < 3 ? state[S.mh_state_off + d] : 1;
    for (int l = 0; l < S.p; ++l) {
        for (uint32_t a = 0; a < (1u << 20); ++a) {
            U4 acc = draw((uint32_t)l, kTagMH | (4u * a + 3u), S.seed, step);
            if (d < 3) {
                U4 r = draw((uint32_t)l, kTagMH | (4u * a + (uint32_t)d), S.seed, step);
                double u1 = 1.0 - u53(r.x, r.y), u2 = u53(r.z, r.w);
                double x = sd * sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
                int ms = x >= 0.0 ? (int)floor(x + 0.5) : -(int)floor(-x + 0.5);
                double ratio = exp(-a2 * ((double)ms * ms - (double)cur * cur)) * mh_qbar(w, cur) / mh_qbar(w, ms);
                uint32_t word = d == 0 ? acc.x : (d == 1 ? acc.y : acc.z);
                if ((double)word * (1.0 / 4294967296.0) < ratio) cur = ms;
            }
            // the all-zero vector is discarded
            uint64_t nz = __ballot(d < 3 && cur != 0);
            if (nz) break;
        }
        if (d < 3) modes[d * mcap + S.moff + l] = cur;
    }
    if (d < 3) state[S.mh_state_off + d] = cur;
    if (d == 0)
        for (int l = 0; l < S.p; ++l) mode_w[S.moff + l] = S.S / (double)S.p;
}

// ---------------------------------------------------------------------------
// Structure factor rho(k_l) = sum_j q_j exp(i k_l.r_j) (eq. 2.7), stage 1.
// A block stages a chunk of particles (fractional coordinates in double and
// the charge) in LDS; each thread owns one mode l and a residue class g of
// the chunk (G = blockDim / P classes), so no cross-lane traffic is needed
// inside the loop.  Per-thread sums are blocked in T over runs of 8
// particles and folded into double; the G partial sums of a mode are
// combined in LDS and one (C, S) pair per mode and tile is written.
// ---------------------------------------------------------------------------
struct alignas(16) PartD {
    double x, y, z, q;
};

template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_rho(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                            const T *__restrict__ pos, const T *__restrict__ q, int64_t ntot,
                                            const int32_t *__restrict__ modes, int mcap,
                                            double *__restrict__ partial, const int32_t *__restrict__ part_off)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    const SysDev &S = sys[t.sys];
    PartD *sp = reinterpret_cast<PartD *>(smem);
    double2 *red = reinterpret_cast<double2 *>(smem + sizeof(PartD) * t.count);
    const int tid = threadIdx.x;
    const int count = t.count;
    for (int j = tid; j < count; j += BS) {
        const int64_t i = S.off + t.start + j;
        PartD v;
        v.x = frac01((double)pos[i] * S.invL);
        v.y = frac01((double)pos[ntot + i] * S.invL);
        v.z = frac01((double)pos[2 * ntot + i] * S.invL);
        v.q = (double)q[i];
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
        double C = 0.0, Sn = 0.0;
        if (act) {
            const int o = S.moff + l;
            const double mx = (double)modes[o], my = (double)modes[mcap + o], mz = (double)modes[2 * mcap + o];
            for (int j0 = g; j0 < count; j0 += 8 * G) {
                T c8 = 0, s8 = 0;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int j = j0 + u * G;
                    if (j < count) {
                        const PartD v = sp[j];
                        const double ph = wrap_rev(fma(mx, v.x, fma(my, v.y, mz * v.z)));
                        T sn, cs;
                        sincos_rev(ph, &sn, &cs);
                        const T qq = (T)v.q;
                        c8 = fma(qq, cs, c8);
                        s8 = fma(qq, sn, s8);
                    }
                }
                C += (double)c8;
                Sn += (double)s8;
            }
        }
        red[tid] = make_double2(C, Sn);
        __syncthreads();
        if (tid < Pt && l < P) {
            double c = 0.0, s = 0.0;
            for (int gg = 0; gg < G; ++gg) {
                const double2 v = red[gg * Pt + lt];
                c += v.x;
                s += v.y;
            }
            prow[2 * l] = c;
            prow[2 * l + 1] = s;
        }
        __syncthreads();
    }
}

// Stage 2: one wave per (system, mode) sums the tile partials in double in a
// fixed order, stores rho, and fills the per-mode constants of the force
// pass: a_l = coulomb w_l 2 m_l/(L^2 |m_l|^2), which equals
// coulomb w_l 4 pi k_l/(V k_l^2) for k_l = 2 pi m_l/L (eq. 3.6).
template <typename KM>
__global__ __launch_bounds__(64) void k_rho_final(const SysDev *__restrict__ sys, const double *__restrict__ partial,
                                                  const int32_t *__restrict__ part_off,
                                                  const int32_t *__restrict__ ntiles, const int32_t *__restrict__ modes,
                                                  const double *__restrict__ mode_w, int mcap,
                                                  double *__restrict__ rho, KM *__restrict__ km)
{
    const int r = blockIdx.y;
    const SysDev &S = sys[r];
    const int l = blockIdx.x;
    if (l >= S.p) return;
    const int nt = ntiles[r];
    const double *base = partial + 2 * (int64_t)part_off[r];
    double c = 0.0, s = 0.0;
    for (int t = threadIdx.x; t < nt; t += 64) {
        c += base[2 * ((int64_t)t * S.p + l)];
        s += base[2 * ((int64_t)t * S.p + l) + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        s += __shfl_down(s, off, 64);
    }
    if (threadIdx.x == 0) {
        const int o = S.moff + l;
        rho[2 * o] = c;
        rho[2 * o + 1] = s;
        const double mx = modes[o], my = modes[mcap + o], mz = modes[2 * mcap + o];
        const double m2 = mx * mx + my * my + mz * mz;
        const double f = S.coulomb * mode_w[o] * 2.0 / (S.L * S.L * m2);
        KM k;
        k.m[0] = mx;
        k.m[1] = my;
        k.m[2] = mz;
        k.a[0] = f * mx;
        k.a[1] = f * my;
        k.a[2] = f * mz;
        k.C = c;
        k.S = s;
        if constexpr (sizeof(KM) == sizeof(KModeF)) k.pad = 0.0f;
        km[o] = k;
    }
}

// ---------------------------------------------------------------------------
// Fourier-space force (eq. 3.6):  F_i = -q_i sum_l (cos th_il S_l - sin th_il C_l) a_l.
// One lane per particle; a block holds 4 waves, each group of SPLIT waves
// shares one 64-particle tile and splits its modes, and the partial forces
// are combined in LDS in a fixed order.  Mode constants are wave-uniform and
// come through scalar loads.
// ---------------------------------------------------------------------------
template <typename T, typename KM, int SPLIT>
__global__ __launch_bounds__(256) void k_kforce(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                int ntiles, const T *__restrict__ pos, const T *__restrict__ q,
                                                int64_t ntot, const KM *__restrict__ km, T *__restrict__ F,
                                                int accumulate, int32_t *__restrict__ flag)
{
    __shared__ T red[4][3][64];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int group = wave / SPLIT, part = wave % SPLIT;
    const int ti = blockIdx.x * (4 / SPLIT) + group;
    T fx = 0, fy = 0, fz = 0;
    int64_t i = -1;
    T qi = 0;
    if (ti < ntiles) {
        const Tile t = tiles[ti];
        const SysDev &S = sys[t.sys];
        const bool act = lane < t.count;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        if (act) {
            i = S.off + t.start + lane;
            sx = frac01((double)pos[i] * S.invL);
            sy = frac01((double)pos[ntot + i] * S.invL);
            sz = frac01((double)pos[2 * ntot + i] * S.invL);
            qi = q[i];
        }
        const int l0 = (S.p * part) / SPLIT, l1 = (S.p * (part + 1)) / SPLIT;
        const KM *kk = km + S.moff;
        for (int l = l0; l < l1; ++l) {
            const KM k = kk[l];
            const double ph = wrap_rev(fma(k.m[0], sx, fma(k.m[1], sy, k.m[2] * sz)));
            T sn, cs;
            sincos_rev(ph, &sn, &cs);
            const T im = cs * (T)k.S - sn * (T)k.C;
            fx = fma(im, (T)k.a[0], fx);
            fy = fma(im, (T)k.a[1], fy);
            fz = fma(im, (T)k.a[2], fz);
        }
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
    fx *= -qi;
    fy *= -qi;
    fz *= -qi;
    if (!isfinite(fx + fy + fz)) atomicOr(flag, 1);
    if (accumulate) {
        fx += F[i];
        fy += F[ntot + i];
        fz += F[2 * ntot + i];
    }
    F[i] = fx;
    F[ntot + i] = fy;
    F[2 * ntot + i] = fz;
}

// ---------------------------------------------------------------------------
// Cell list (bin, scan, scatter, per-cell sort).
// Single precision keeps each wrapped position as three 32-bit fractions of
// the box (u = floor(s 2^32)) plus the charge bits; double precision keeps
// the wrapped fractional coordinates in double.
// ---------------------------------------------------------------------------
struct alignas(16) PackF {
    uint32_t x, y, z;
    float q;
};

__device__ __forceinline__ uint32_t to_fix(double s)
{
    double v = s * 4294967296.0;
    return v >= 4294967295.0 ? 4294967295u : (uint32_t)v;
}

__device__ __forceinline__ int cell_of_fix(uint32_t u, int nc)
{
    return (int)(((uint64_t)u * (uint64_t)nc) >> 32);
}

__device__ __forceinline__ int cell_of_frac(double s, int nc)
{
    int c = (int)(s * nc);
    return c >= nc ? nc - 1 : c;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bin(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                             const T *__restrict__ pos, const T *__restrict__ q, int64_t ntot,
                                             int32_t *__restrict__ count, int32_t *__restrict__ cellid,
                                             int32_t *__restrict__ rank, void *__restrict__ packed)
{
    const Tile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const SysDev &S = sys[t.sys];
    const int64_t i = S.off + t.start + threadIdx.x;
    const double sx = frac01((double)pos[i] * S.invL);
    const double sy = frac01((double)pos[ntot + i] * S.invL);
    const double sz = frac01((double)pos[2 * ntot + i] * S.invL);
    int cx, cy, cz;
    if constexpr (sizeof(T) == 4) {
        PackF v{to_fix(sx), to_fix(sy), to_fix(sz), (float)q[i]};
        reinterpret_cast<PackF *>(packed)[i] = v;
        cx = cell_of_fix(v.x, S.nc);
        cy = cell_of_fix(v.y, S.nc);
        cz = cell_of_fix(v.z, S.nc);
    } else {
        reinterpret_cast<PartD *>(packed)[i] = PartD{sx, sy, sz, (double)q[i]};
        cx = cell_of_frac(sx, S.nc);
        cy = cell_of_frac(sy, S.nc);
        cz = cell_of_frac(sz, S.nc);
    }
    const int c = S.cell_off + (cz * S.nc + cy) * S.nc + cx;
    cellid[i] = c;
    rank[i] = atomicAdd(&count[c], 1);
}

// Exclusive scan of the cell counts of one system per block; start entries
// are global slot indices (S.off + prefix).  System r's starts live at
// [cell_off + r, cell_off + r + ncells].  Counts are cleared for the next use.
__global__ __launch_bounds__(1024) void k_scan(const SysDev *__restrict__ sys, int32_t *__restrict__ count,
                                               int32_t *__restrict__ start)
{
    __shared__ int32_t part[1024];
    const int r = blockIdx.x;
    const SysDev &S = sys[r];
    const int ncell = S.ncell;
    const int per = (ncell + 1023) / 1024;
    const int b = threadIdx.x * per;
    const int e = min(b + per, ncell);
    int32_t *cnt = count + S.cell_off;
    int32_t *st = start + S.cell_off + r;
    int sum = 0;
    for (int c = b; c < e; ++c) sum += cnt[c];
    part[threadIdx.x] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 thread sums
    for (int off = 1; off < 1024; off <<= 1) {
        int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = S.off + (threadIdx.x ? part[threadIdx.x - 1] : 0);
    for (int c = b; c < e; ++c) {
        st[c] = run;
        run += cnt[c];
        cnt[c] = 0;
    }
    if (threadIdx.x == 1023) st[ncell] = S.off + part[1023];
}

template <typename P>
__global__ __launch_bounds__(256) void k_scatter(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                 const int32_t *__restrict__ start, const int32_t *__restrict__ cellid,
                                                 const int32_t *__restrict__ rank, const P *__restrict__ packed,
                                                 int32_t *__restrict__ sorted_idx, P *__restrict__ sorted)
{
    const Tile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const int64_t i = sys[t.sys].off + t.start + threadIdx.x;
    const int slot = start[cellid[i] + t.sys] + rank[i];
    sorted_idx[slot] = (int32_t)i;
    sorted[slot] = packed[i];
}

// Insertion sort of each cell's slots by particle index, so that the order of
// the real-space sums does not depend on the order of the atomic increments.
template <typename P>
__global__ __launch_bounds__(256) void k_cellsort(const SysDev *__restrict__ sys, const int32_t *__restrict__ start,
                                                  int32_t *__restrict__ sorted_idx, P *__restrict__ sorted)
{
    const int r = blockIdx.y;
    const SysDev &S = sys[r];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= S.ncell) return;
    const int32_t *st = start + S.cell_off + r;
    const int b = st[c], e = st[c + 1];
    for (int a = b + 1; a < e; ++a) {
        const int32_t key = sorted_idx[a];
        const P val = sorted[a];
        int k = a - 1;
        while (k >= b && sorted_idx[k] > key) {
            sorted_idx[k + 1] = sorted_idx[k];
            sorted[k + 1] = sorted[k];
            --k;
        }
        sorted_idx[k + 1] = key;
        sorted[k + 1] = val;
    }
}

// ---------------------------------------------------------------------------
// Real space (eq. 2.11, second term) and shifted LJ (eq. 4.1, r_off = 0).
// Pair force on i: phi(r) d, d = r_j - r_i (minimum image), with
//   phi = -coulomb q_i q_j (erfc(beta r)/r + 2 beta/sqrt(pi) exp(-alpha r^2))/r^2
//         + 4 eps (6 (sigma/r)^6 - 12 (sigma/r)^12)/r^2      (LJ, r < R_c).
// One thread per sorted slot; the 27 neighbouring cells are scanned (one
// cell holding everything when fewer than 3 cells fit along the box).  The
// optional kick adds dt/(2m) times the total force to the velocity (the last
// B of the Langevin step).
// ---------------------------------------------------------------------------
struct PairAcc {
    double e_real, e_lj, vir;
};

template <bool ENERGY>
__device__ __forceinline__ void pair_f32(const SysDev &S, float qi, float qj, float dx, float dy, float dz, float r2,
                                         float &fx, float &fy, float &fz, PairAcc &acc, float rc2, float ljrc2)
{
    float phi = 0.0f;
    if (r2 <= rc2) {
        const float r = sqrtf(r2);
        const float beta = (float)S.beta;
        const float ec = erfcf(beta * r);
        const float ex = expf(-(float)S.alpha * r2);
        const float inv_r2 = 1.0f / r2;
        const float g = (ec / r + (float)(2.0 / 1.7724538509055160273) * beta * ex) * inv_r2;
        const float cq = (float)S.coulomb * qi * qj;
        phi = -cq * g;
        if constexpr (ENERGY) acc.e_real += 0.5 * (double)(cq * ec / r);
    }
    if (S.lj_on && r2 < ljrc2) {
        const float sr2 = (float)S.lj_sig2 / r2;
        const float sr6 = sr2 * sr2 * sr2;
        const float eps = (float)S.lj_eps;
        phi += 4.0f * eps * (6.0f * sr6 - 12.0f * sr6 * sr6) / r2;
        if constexpr (ENERGY) acc.e_lj += 0.5 * (4.0 * (double)eps * ((double)sr6 * sr6 - sr6) + S.lj_shift);
    }
    fx = fma(phi, dx, fx);
    fy = fma(phi, dy, fy);
    fz = fma(phi, dz, fz);
    if constexpr (ENERGY) acc.vir += 0.5 * (double)(phi * r2);
}

template <bool ENERGY>
__device__ __forceinline__ void pair_f64(const SysDev &S, double qi, double qj, double dx, double dy, double dz,
                                         double r2, double &fx, double &fy, double &fz, PairAcc &acc)
{
    double phi = 0.0;
    if (r2 <= S.rc2) {
        const double r = sqrt(r2);
        const double ec = erfc(S.beta * r);
        const double ex = exp(-S.alpha * r2);
        const double g = (ec / r + 2.0 / 1.7724538509055160273 * S.beta * ex) / r2;
        const double cq = S.coulomb * qi * qj;
        phi = -cq * g;
        if constexpr (ENERGY) acc.e_real += 0.5 * cq * ec / r;
    }
    if (S.lj_on && r2 < S.lj_rc2) {
        const double sr2 = S.lj_sig2 / r2;
        const double sr6 = sr2 * sr2 * sr2;
        phi += 4.0 * S.lj_eps * (6.0 * sr6 - 12.0 * sr6 * sr6) / r2;
        if constexpr (ENERGY) acc.e_lj += 0.5 * (4.0 * S.lj_eps * (sr6 * sr6 - sr6) + S.lj_shift);
    }
    fx = fma(phi, dx, fx);
    fy = fma(phi, dy, fy);
    fz = fma(phi, dz, fz);
    if constexpr (ENERGY) acc.vir += 0.5 * phi * r2;
}

// Walk the neighbour cells of the particle in sorted slot `slot` and
// accumulate its real-space force (and energies when ENERGY).
template <typename T, bool ENERGY>
__device__ __forceinline__ void real_one(const SysDev &S, int r, int slot, const int32_t *__restrict__ start,
                                         const void *__restrict__ sortedv, T &fx, T &fy, T &fz, PairAcc &acc)
{
    const int32_t *st = start + S.cell_off + r;
    const int nc = S.nc;
    if constexpr (sizeof(T) == 4) {
        const PackF *sorted = reinterpret_cast<const PackF *>(sortedv);
        const PackF pi = sorted[slot];
        const int cx = cell_of_fix(pi.x, nc), cy = cell_of_fix(pi.y, nc), cz = cell_of_fix(pi.z, nc);
        // fixed-point units: one unit is L 2^-32
        const float scale = (float)(S.L * (1.0 / 4294967296.0));
        const double inv_u2 = 1.0 / ((double)scale * (double)scale);
        const float rc2u = (float)(S.rc2 * inv_u2);
        const float ljrc2u = S.lj_on ? (float)(S.lj_rc2 * inv_u2) : 0.0f;
        const float rmax2u = fmaxf(rc2u, ljrc2u);
        const float rc2 = (float)S.rc2, ljrc2 = (float)S.lj_rc2;
        const int nd = nc >= 3 ? 1 : 0;
        for (int dz = -nd; dz <= nd; ++dz) {
            const int zz = (cz + dz + nc) % nc;
            for (int dy = -nd; dy <= nd; ++dy) {
                const int yy = (cy + dy + nc) % nc;
                for (int dxc = -nd; dxc <= nd; ++dxc) {
                    const int xx = (cx + dxc + nc) % nc;
                    const int c = (zz * nc + yy) * nc + xx;
                    const int b = st[c], e = st[c + 1];
                    for (int j = b; j < e; ++j) {
                        if (j == slot) continue;
                        const PackF pj = sorted[j];
                        const float ux = (float)(int32_t)(pj.x - pi.x);
                        const float uy = (float)(int32_t)(pj.y - pi.y);
                        const float uz = (float)(int32_t)(pj.z - pi.z);
                        const float r2u = fma(ux, ux, fma(uy, uy, uz * uz));
                        if (r2u <= rmax2u) {
                            const float dx = ux * scale, dy2 = uy * scale, dz2 = uz * scale;
                            const float r2 = fma(dx, dx, fma(dy2, dy2, dz2 * dz2));
                            pair_f32<ENERGY>(S, pi.q, pj.q, dx, dy2, dz2, r2, fx, fy, fz, acc, rc2, ljrc2);
                        }
                    }
                }
            }
        }
    } else {
        const PartD *sorted = reinterpret_cast<const PartD *>(sortedv);
        const PartD pi = sorted[slot];
        const int cx = cell_of_frac(pi.x, nc), cy = cell_of_frac(pi.y, nc), cz = cell_of_frac(pi.z, nc);
        const double rmax2 = S.lj_on ? fmax(S.rc2, S.lj_rc2) : S.rc2;
        const int nd = nc >= 3 ? 1 : 0;
        for (int dz = -nd; dz <= nd; ++dz) {
            const int zz = (cz + dz + nc) % nc;
            for (int dy = -nd; dy <= nd; ++dy) {
                const int yy = (cy + dy + nc) % nc;
                for (int dxc = -nd; dxc <= nd; ++dxc) {
                    const int xx = (cx + dxc + nc) % nc;
                    const int c = (zz * nc + yy) * nc + xx;
                    const int b = st[c], e = st[c + 1];
                    for (int j = b; j < e; ++j) {
                        if (j == slot) continue;
                        const PartD pj = sorted[j];
                        double sx = pj.x - pi.x, sy = pj.y - pi.y, sz = pj.z - pi.z;
                        sx -= rint(sx);
                        sy -= rint(sy);
                        sz -= rint(sz);
                        const double dx = sx * S.L, dy2 = sy * S.L, dz2 = sz * S.L;
                        const double r2 = dx * dx + dy2 * dy2 + dz2 * dz2;
                        if (r2 <= rmax2) pair_f64<ENERGY>(S, pi.q, pj.q, dx, dy2, dz2, r2, fx, fy, fz, acc);
                    }
                }
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_real(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                              const int32_t *__restrict__ start,
                                              const int32_t *__restrict__ sorted_idx, const void *__restrict__ sorted,
                                              int64_t ntot, T *__restrict__ F, int accumulate, T *__restrict__ vel,
                                              int32_t *__restrict__ flag)
{
    const Tile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const SysDev &S = sys[t.sys];
    const int slot = S.off + t.start + threadIdx.x;
    T fx = 0, fy = 0, fz = 0;
    PairAcc acc{0, 0, 0};
    real_one<T, false>(S, t.sys, slot, start, sorted, fx, fy, fz, acc);
    const int64_t i = sorted_idx[slot];
    if (!isfinite(fx + fy + fz)) atomicOr(flag, 1);
    if (accumulate) {
        fx += F[i];
        fy += F[ntot + i];
        fz += F[2 * ntot + i];
    }
    F[i] = fx;
    F[ntot + i] = fy;
    F[2 * ntot + i] = fz;
    if (vel) {
        const double h = 0.5 * S.dt / S.mass;
        vel[i] = (T)((double)vel[i] + h * (double)fx);
        vel[ntot + i] = (T)((double)vel[ntot + i] + h * (double)fy);
        vel[2 * ntot + i] = (T)((double)vel[2 * ntot + i] + h * (double)fz);
    }
}

// ---------------------------------------------------------------------------
// Integrators.
// BAOAB (reading of the Langevin equation of Sec. 3.3): B, A, O, A here; the
// force and the final B follow in the force kernels.
// Leapfrog + Andersen (Sec. 3.1 loop body, Sec. 3.3): v += dt F/m,
// r += dt v, then a collision with probability nu dt resets v ~ N(0, kT/m).
// Positions are wrapped into [0, L).  Arithmetic in double.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_integrate(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                   T *__restrict__ pos, T *__restrict__ vel,
                                                   const T *__restrict__ F, int64_t ntot, uint64_t step)
{
    const Tile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const SysDev &S = sys[t.sys];
    const int il = t.start + threadIdx.x;
    const int64_t i = S.off + il;
    double xi[3];
    if (S.integrator == RBE_LANGEVIN_BAOAB) {
        normals3((uint32_t)il, S.seed, step, xi);
        const double h = 0.5 * S.dt;
        for (int d = 0; d < 3; ++d) {
            const int64_t k = d * ntot + i;
            double v = (double)vel[k] + h * (double)F[k] / S.mass;
            double x = (double)pos[k] + h * v;
            v = S.c1 * v + S.c2 * xi[d];
            x += h * v;
            x -= S.L * floor(x * S.invL);
            T xs = (T)x;
            if (xs >= (T)S.L || xs < (T)0) xs = (T)0;
            pos[k] = xs;
            vel[k] = (T)v;
        }
    } else {
        U4 w = draw((uint32_t)il, kTagAndersen, S.seed, step);
        const bool hit = (double)w.x * (1.0 / 4294967296.0) < S.nu_dt;
        if (hit) normals3((uint32_t)il, S.seed, step, xi);
        const double sv = sqrt(S.kT / S.mass);
        for (int d = 0; d < 3; ++d) {
            const int64_t k = d * ntot + i;
            double v = (double)vel[k] + S.dt * (double)F[k] / S.mass;
            double x = (double)pos[k] + S.dt * v;
            x -= S.L * floor(x * S.invL);
            T xs = (T)x;
            if (xs >= (T)S.L || xs < (T)0) xs = (T)0;
            pos[k] = xs;
            vel[k] = (T)(hit ? sv * xi[d] : v);
        }
    }
}

// ---------------------------------------------------------------------------
// Energies (eqs. 2.6, 2.9, 4.1, 4.3): per-block double partial sums of the
// real-space energy, LJ energy, pair virial, kinetic energy, sum q^2,
// sum q and sum |q|; the host adds them up per system.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_energy(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                const int32_t *__restrict__ start,
                                                const int32_t *__restrict__ sorted_idx,
                                                const void *__restrict__ sorted, const T *__restrict__ q,
                                                const T *__restrict__ vel, int64_t ntot, double *__restrict__ out)
{
    __shared__ double red[8][256];
    const Tile t = tiles[blockIdx.x];
    const SysDev &S = sys[t.sys];
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if ((int)threadIdx.x < t.count) {
        const int slot = S.off + t.start + threadIdx.x;
        T fx = 0, fy = 0, fz = 0;
        PairAcc acc{0, 0, 0};
        real_one<T, true>(S, t.sys, slot, start, sorted, fx, fy, fz, acc);
        v[0] = acc.e_real;
        v[1] = acc.e_lj;
        v[2] = acc.vir;
        const int64_t i = S.off + t.start + threadIdx.x;  // original order for the one-body sums
        if (vel) {
            const double a = vel[i], b = vel[ntot + i], c = vel[2 * ntot + i];
            v[3] = 0.5 * S.mass * (a * a + b * b + c * c);
        }
        const double qq = (double)q[i];
        v[4] = qq * qq;
        v[5] = qq;
        v[6] = fabs(qq);
        (void)sorted_idx;
    }
    for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 8) out[8 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Adjoint of the forces at a fixed mode sample.  With G_i = dLoss/dF_i and
// the force of eq. (3.6) written F_i = -q_i sum_l (cos th_il S_l - sin th_il C_l) a_l
// (rho_l = C_l + i S_l, a_l = coulomb w_l 4 pi k_l/(V k_l^2)):
//   w_il = G_i.a_l,  A_l = sum_i q_i w_il cos th_il,  B_l = sum_i q_i w_il sin th_il,
//   dLoss/dq_i = -sum_l [w_il (cos th S_l - sin th C_l) + A_l sin th - B_l cos th],
//   dLoss/dr_i = q_i sum_l k_l [w_il (sin th S_l + cos th C_l) - A_l cos th - B_l sin th].
// The reduction over particles (A, B) has the shape of the structure factor
// and reuses its tiling; the gather has the shape of the force pass.
// ---------------------------------------------------------------------------
struct alignas(16) PartG {
    double x, y, z, gx, gy, gz;   // fractional position and q_i G_i
};

template <typename T, typename KM, int BS>
__global__ __launch_bounds__(BS) void k_vjp_reduce(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                   const T *__restrict__ pos, const T *__restrict__ q,
                                                   const T *__restrict__ gF, int64_t ntot,
                                                   const KM *__restrict__ km, double *__restrict__ partial,
                                                   const int32_t *__restrict__ part_off)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    const SysDev &S = sys[t.sys];
    PartG *sp = reinterpret_cast<PartG *>(smem);
    double2 *red = reinterpret_cast<double2 *>(smem + sizeof(PartG) * t.count);
    const int tid = threadIdx.x;
    const int count = t.count;
    for (int j = tid; j < count; j += BS) {
        const int64_t i = S.off + t.start + j;
        const double qi = (double)q[i];
        PartG v;
        v.x = frac01((double)pos[i] * S.invL);
        v.y = frac01((double)pos[ntot + i] * S.invL);
        v.z = frac01((double)pos[2 * ntot + i] * S.invL);
        v.gx = qi * (double)gF[i];
        v.gy = qi * (double)gF[ntot + i];
        v.gz = qi * (double)gF[2 * ntot + i];
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
            const T ax = (T)k.a[0], ay = (T)k.a[1], az = (T)k.a[2];
            for (int j0 = g; j0 < count; j0 += 8 * G) {
                T a8 = 0, b8 = 0;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int j = j0 + u * G;
                    if (j < count) {
                        const PartG v = sp[j];
                        const double ph = wrap_rev(fma(k.m[0], v.x, fma(k.m[1], v.y, k.m[2] * v.z)));
                        T sn, cs;
                        sincos_rev(ph, &sn, &cs);
                        const T w = fma((T)v.gx, ax, fma((T)v.gy, ay, (T)v.gz * az));
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
            double a = 0.0, b = 0.0;
            for (int gg = 0; gg < G; ++gg) {
                const double2 v = red[gg * Pt + lt];
                a += v.x;
                b += v.y;
            }
            prow[2 * l] = a;
            prow[2 * l + 1] = b;
        }
        __syncthreads();
    }
}

template <typename KM, typename KV>
__global__ __launch_bounds__(64) void k_vjp_final(const SysDev *__restrict__ sys, const double *__restrict__ partial,
                                                  const int32_t *__restrict__ part_off,
                                                  const int32_t *__restrict__ ntiles, const KM *__restrict__ km,
                                                  double *__restrict__ ab, KV *__restrict__ kv)
{
    const int r = blockIdx.y;
    const SysDev &S = sys[r];
    const int l = blockIdx.x;
    if (l >= S.p) return;
    const int nt = ntiles[r];
    const double *base = partial + 2 * (int64_t)part_off[r];
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < nt; t += 64) {
        a += base[2 * ((int64_t)t * S.p + l)];
        b += base[2 * ((int64_t)t * S.p + l) + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    if (threadIdx.x == 0) {
        const int o = S.moff + l;
        ab[2 * o] = a;
        ab[2 * o + 1] = b;
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
        v.A = a;
        v.B = b;
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
        const SysDev &S = sys[t.sys];
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
        const int l0 = (S.p * part) / SPLIT, l1 = (S.p * (part + 1)) / SPLIT;
        const KV *kk = kv + S.moff;
        for (int l = l0; l < l1; ++l) {
            const KV k = kk[l];
            const double ph = wrap_rev(fma(k.m[0], sx, fma(k.m[1], sy, k.m[2] * sz)));
            T sn, cs;
            sincos_rev(ph, &sn, &cs);
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

// Real-space and LJ adjoint.  Pair force on i is phi(r) d with d = r_j - r_i;
// with dG = G_i - G_j:
//   dLoss/dq_i += -coulomb sum_j q_j (G(r)/r) dG.d
//   dLoss/dr_i += sum_j [ -(phi'(r)/r)(dG.d) d - phi dG ]
// where G(r)/r = erfc(beta r)/r^3 + 2 beta exp(-alpha r^2)/(sqrt(pi) r^2) and
// its derivative is -3 erfc/r^4 - 6 beta e/(sqrt(pi) r^3) - 4 beta^3 e/(sqrt(pi) r).
template <typename T>
__device__ __forceinline__ void vjp_pair(const SysDev &S, T qi, T qj, T dx, T dy, T dz, T r2, T Gx, T Gy, T Gz,
                                         T &dq, T &rx, T &ry, T &rz)
{
    T phi = 0, dphi_r = 0;   // phi and phi'(r)/r
    const T GD = Gx * dx + Gy * dy + Gz * dz;
    if (r2 <= (T)S.rc2) {
        const T r = sqrt(r2);
        const T beta = (T)S.beta;
        const T ec = erfc(beta * r);
        const T ex = exp(-(T)S.alpha * r2);
        const T isp = (T)(1.0 / 1.7724538509055160273);
        const T inv_r = (T)1 / r, inv_r2 = inv_r * inv_r;
        const T g = (ec * inv_r + (T)2 * beta * isp * ex) * inv_r2;
        const T dg = -(T)3 * ec * inv_r2 * inv_r2 - (T)6 * beta * isp * ex * inv_r2 * inv_r -
                     (T)4 * beta * beta * beta * isp * ex * inv_r;
        const T cq = (T)S.coulomb * qi * qj;
        phi = -cq * g;
        dphi_r = -cq * dg * inv_r;
        dq -= (T)S.coulomb * qj * g * GD;
    }
    if (S.lj_on && r2 < (T)S.lj_rc2) {
        const T sr2 = (T)S.lj_sig2 / r2;
        const T sr6 = sr2 * sr2 * sr2, sr12 = sr6 * sr6;
        const T eps4 = (T)(4.0 * S.lj_eps);
        phi += eps4 * ((T)6 * sr6 - (T)12 * sr12) / r2;
        dphi_r += eps4 * ((T)168 * sr12 - (T)48 * sr6) / (r2 * r2);
    }
    rx -= dphi_r * GD * dx + phi * Gx;
    ry -= dphi_r * GD * dy + phi * Gy;
    rz -= dphi_r * GD * dz + phi * Gz;
}

template <typename T>
__global__ __launch_bounds__(256) void k_vjp_real(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                  const int32_t *__restrict__ start,
                                                  const int32_t *__restrict__ sorted_idx,
                                                  const void *__restrict__ sortedv, const T *__restrict__ gF,
                                                  int64_t ntot, T *__restrict__ gpos, T *__restrict__ gq,
                                                  int accumulate)
{
    const Tile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const SysDev &S = sys[t.sys];
    const int slot = S.off + t.start + threadIdx.x;
    const int64_t i = sorted_idx[slot];
    const int32_t *st = start + S.cell_off + t.sys;
    const int nc = S.nc;
    const T Gix = gF[i], Giy = gF[ntot + i], Giz = gF[2 * ntot + i];
    T dq = 0, rx = 0, ry = 0, rz = 0;
    const int nd = nc >= 3 ? 1 : 0;
    int cx, cy, cz;
    if constexpr (sizeof(T) == 4) {
        const PackF *sorted = reinterpret_cast<const PackF *>(sortedv);
        const PackF pi = sorted[slot];
        cx = cell_of_fix(pi.x, nc);
        cy = cell_of_fix(pi.y, nc);
        cz = cell_of_fix(pi.z, nc);
        const float scale = (float)(S.L * (1.0 / 4294967296.0));
        const double inv_u2 = 1.0 / ((double)scale * (double)scale);
        const float rmax2u = (float)((S.lj_on ? fmax(S.rc2, S.lj_rc2) : S.rc2) * inv_u2);
        for (int dz = -nd; dz <= nd; ++dz)
            for (int dy = -nd; dy <= nd; ++dy)
                for (int dxc = -nd; dxc <= nd; ++dxc) {
                    const int c = (((cz + dz + nc) % nc) * nc + ((cy + dy + nc) % nc)) * nc + ((cx + dxc + nc) % nc);
                    const int b = st[c], e = st[c + 1];
                    for (int j = b; j < e; ++j) {
                        if (j == slot) continue;
                        const PackF pj = sorted[j];
                        const float ux = (float)(int32_t)(pj.x - pi.x);
                        const float uy = (float)(int32_t)(pj.y - pi.y);
                        const float uz = (float)(int32_t)(pj.z - pi.z);
                        if (fma(ux, ux, fma(uy, uy, uz * uz)) <= rmax2u) {
                            const int64_t jj = sorted_idx[j];
                            const float dx = ux * scale, dy2 = uy * scale, dz2 = uz * scale;
                            const float r2 = fma(dx, dx, fma(dy2, dy2, dz2 * dz2));
                            vjp_pair<float>(S, pi.q, pj.q, dx, dy2, dz2, r2, Gix - gF[jj], Giy - gF[ntot + jj],
                                            Giz - gF[2 * ntot + jj], dq, rx, ry, rz);
                        }
                    }
                }
    } else {
        const PartD *sorted = reinterpret_cast<const PartD *>(sortedv);
        const PartD pi = sorted[slot];
        cx = cell_of_frac(pi.x, nc);
        cy = cell_of_frac(pi.y, nc);
        cz = cell_of_frac(pi.z, nc);
        const double rmax2 = S.lj_on ? fmax(S.rc2, S.lj_rc2) : S.rc2;
        for (int dz = -nd; dz <= nd; ++dz)
            for (int dy = -nd; dy <= nd; ++dy)
                for (int dxc = -nd; dxc <= nd; ++dxc) {
                    const int c = (((cz + dz + nc) % nc) * nc + ((cy + dy + nc) % nc)) * nc + ((cx + dxc + nc) % nc);
                    const int b = st[c], e = st[c + 1];
                    for (int j = b; j < e; ++j) {
                        if (j == slot) continue;
                        const PartD pj = sorted[j];
                        double sx = pj.x - pi.x, sy = pj.y - pi.y, sz = pj.z - pi.z;
                        sx -= rint(sx);
                        sy -= rint(sy);
                        sz -= rint(sz);
                        const double dx = sx * S.L, dy2 = sy * S.L, dz2 = sz * S.L;
                        const double r2 = dx * dx + dy2 * dy2 + dz2 * dz2;
                        if (r2 <= rmax2) {
                            const int64_t jj = sorted_idx[j];
                            vjp_pair<double>(S, pi.q, pj.q, dx, dy2, dz2, r2, Gix - gF[jj], Giy - gF[ntot + jj],
                                             Giz - gF[2 * ntot + jj], dq, rx, ry, rz);
                        }
                    }
                }
    }
    if (accumulate) {
        dq += gq[i];
        rx += gpos[i];
        ry += gpos[ntot + i];
        rz += gpos[2 * ntot + i];
    }
    gq[i] = dq;
    gpos[i] = rx;
    gpos[ntot + i] = ry;
    gpos[2 * ntot + i] = rz;
}

__global__ void k_fill_zero(uint32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_zero(hipStream_t s, void *ptr, int64_t nbytes)
{
    int64_t n = nbytes / 4;
    if (n <= 0) return hipSuccess;
    k_fill_zero<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>((uint32_t *)ptr, n);
    return hipGetLastError();
}

hipError_t launch_sample(const LaunchCfg &c, const Workspace &w, uint64_t step, int use_mh)
{
    if (use_mh) {
        k_sample_mh<<<dim3(c.R), dim3(64), 0, c.stream>>>(w.sys, w.mh_state, w.modes, w.mode_w, c.mcap, step);
    } else {
        dim3 g((c.max_p + 63) / 64, c.R);
        k_sample_exact<<<g, dim3(64), 0, c.stream>>>(w.sys, w.cdf, w.modes, w.mode_w, c.mcap, step);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t rho_dispatch(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q)
{
    const size_t sm = sizeof(PartD) * c.rho_chunk + sizeof(double2) * c.rho_block;
    const T *p = (const T *)pos, *qq = (const T *)q;
    dim3 g(c.n_rho_tiles);
    switch (c.rho_block) {
    case 256:
        k_rho<T, 256><<<g, 256, sm, c.stream>>>(w.sys, w.rho_tiles, p, qq, c.ntot, w.modes, c.mcap, w.partial,
                                               w.partial_off);
        break;
    case 512:
        k_rho<T, 512><<<g, 512, sm, c.stream>>>(w.sys, w.rho_tiles, p, qq, c.ntot, w.modes, c.mcap, w.partial,
                                               w.partial_off);
        break;
    default:
        k_rho<T, 1024><<<g, 1024, sm, c.stream>>>(w.sys, w.rho_tiles, p, qq, c.ntot, w.modes, c.mcap, w.partial,
                                                 w.partial_off);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_rho(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q)
{
    return c.prec == RBE_FP64 ? rho_dispatch<double>(c, w, pos, q) : rho_dispatch<float>(c, w, pos, q);
}

hipError_t launch_rho_final(const LaunchCfg &c, const Workspace &w)
{
    dim3 g(c.max_p, c.R);
    // the per-system tile counts sit right after the partial offsets
    const int32_t *ntiles = w.partial_off + c.R;
    if (c.prec == RBE_FP64)
        k_rho_final<KModeD><<<g, 64, 0, c.stream>>>(w.sys, w.partial, w.partial_off, ntiles, w.modes, w.mode_w,
                                                   c.mcap, w.rho, (KModeD *)w.kmode);
    else
        k_rho_final<KModeF><<<g, 64, 0, c.stream>>>(w.sys, w.partial, w.partial_off, ntiles, w.modes, w.mode_w,
                                                   c.mcap, w.rho, (KModeF *)w.kmode);
    return hipGetLastError();
}

template <typename T, typename KM>
static hipError_t kforce_dispatch(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q, void *F,
                                  int acc)
{
    const T *p = (const T *)pos, *qq = (const T *)q;
    const KM *km = (const KM *)w.kmode;
    T *f = (T *)F;
    const int n = c.n_force_tiles;
    switch (c.force_split) {
    case 1:
        k_kforce<T, KM, 1><<<(n + 3) / 4, 256, 0, c.stream>>>(w.sys, w.force_tiles, n, p, qq, c.ntot, km, f, acc,
                                                              w.flag);
        break;
    case 2:
        k_kforce<T, KM, 2><<<(n + 1) / 2, 256, 0, c.stream>>>(w.sys, w.force_tiles, n, p, qq, c.ntot, km, f, acc,
                                                              w.flag);
        break;
    default:
        k_kforce<T, KM, 4><<<n, 256, 0, c.stream>>>(w.sys, w.force_tiles, n, p, qq, c.ntot, km, f, acc, w.flag);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_kforce(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q, void *force,
                         int accumulate)
{
    return c.prec == RBE_FP64 ? kforce_dispatch<double, KModeD>(c, w, pos, q, force, accumulate)
                              : kforce_dispatch<float, KModeF>(c, w, pos, q, force, accumulate);
}

hipError_t launch_bin(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q)
{
    if (c.prec == RBE_FP64)
        k_bin<double><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, (const double *)pos,
                                                            (const double *)q, c.ntot, w.cell_count, w.cellid,
                                                            w.rank, w.packed);
    else
        k_bin<float><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, (const float *)pos,
                                                           (const float *)q, c.ntot, w.cell_count, w.cellid, w.rank,
                                                           w.packed);
    return hipGetLastError();
}

hipError_t launch_scan(const LaunchCfg &c, const Workspace &w)
{
    k_scan<<<c.R, 1024, 0, c.stream>>>(w.sys, w.cell_count, w.cell_start);
    return hipGetLastError();
}

hipError_t launch_scatter(const LaunchCfg &c, const Workspace &w)
{
    if (c.prec == RBE_FP64)
        k_scatter<PartD><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, w.cell_start, w.cellid, w.rank,
                                                               (const PartD *)w.packed, w.sorted_idx,
                                                               (PartD *)w.sorted);
    else
        k_scatter<PackF><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, w.cell_start, w.cellid, w.rank,
                                                               (const PackF *)w.packed, w.sorted_idx,
                                                               (PackF *)w.sorted);
    return hipGetLastError();
}

hipError_t launch_cellsort(const LaunchCfg &c, const Workspace &w)
{
    dim3 g((c.max_cells + 255) / 256, c.R);
    if (c.prec == RBE_FP64)
        k_cellsort<PartD><<<g, 256, 0, c.stream>>>(w.sys, w.cell_start, w.sorted_idx, (PartD *)w.sorted);
    else
        k_cellsort<PackF><<<g, 256, 0, c.stream>>>(w.sys, w.cell_start, w.sorted_idx, (PackF *)w.sorted);
    return hipGetLastError();
}

hipError_t launch_real(const LaunchCfg &c, const Workspace &w, void *force, int accumulate, void *vel_kick)
{
    if (c.prec == RBE_FP64)
        k_real<double><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, w.cell_start, w.sorted_idx,
                                                             w.sorted, c.ntot, (double *)force, accumulate,
                                                             (double *)vel_kick, w.flag);
    else
        k_real<float><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, w.cell_start, w.sorted_idx,
                                                            w.sorted, c.ntot, (float *)force, accumulate,
                                                            (float *)vel_kick, w.flag);
    return hipGetLastError();
}

hipError_t launch_integrate(const LaunchCfg &c, const Workspace &w, void *pos, void *vel, const void *force,
                            uint64_t step)
{
    if (c.prec == RBE_FP64)
        k_integrate<double><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, (double *)pos,
                                                                  (double *)vel, (const double *)force, c.ntot, step);
    else
        k_integrate<float><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, (float *)pos, (float *)vel,
                                                                 (const float *)force, c.ntot, step);
    return hipGetLastError();
}

hipError_t launch_energy(const LaunchCfg &c, const Workspace &w, const void *q, const void *vel)
{
    if (c.prec == RBE_FP64)
        k_energy<double><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, w.cell_start, w.sorted_idx,
                                                               w.sorted, (const double *)q, (const double *)vel,
                                                               c.ntot, w.energy_part);
    else
        k_energy<float><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, w.cell_start, w.sorted_idx,
                                                              w.sorted, (const float *)q, (const float *)vel, c.ntot,
                                                              w.energy_part);
    return hipGetLastError();
}

template <typename T, typename KM>
static hipError_t vjp_reduce_dispatch(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q,
                                      const void *gF)
{
    const size_t sm = sizeof(PartG) * c.rho_chunk + sizeof(double2) * c.rho_block;
    const T *p = (const T *)pos, *qq = (const T *)q, *g = (const T *)gF;
    const KM *km = (const KM *)w.kmode;
    dim3 gr(c.n_rho_tiles);
    switch (c.rho_block) {
    case 256:
        k_vjp_reduce<T, KM, 256><<<gr, 256, sm, c.stream>>>(w.sys, w.rho_tiles, p, qq, g, c.ntot, km, w.partial,
                                                            w.partial_off);
        break;
    case 512:
        k_vjp_reduce<T, KM, 512><<<gr, 512, sm, c.stream>>>(w.sys, w.rho_tiles, p, qq, g, c.ntot, km, w.partial,
                                                            w.partial_off);
        break;
    default:
        k_vjp_reduce<T, KM, 1024><<<gr, 1024, sm, c.stream>>>(w.sys, w.rho_tiles, p, qq, g, c.ntot, km, w.partial,
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
    const int32_t *ntiles = w.partial_off + c.R;
    if (c.prec == RBE_FP64)
        k_vjp_final<KModeD, KVjpD><<<g, 64, 0, c.stream>>>(w.sys, w.partial, w.partial_off, ntiles,
                                                           (const KModeD *)w.kmode, w.ab, (KVjpD *)w.kvjp);
    else
        k_vjp_final<KModeF, KVjpF><<<g, 64, 0, c.stream>>>(w.sys, w.partial, w.partial_off, ntiles,
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
        k_vjp_gather<T, KV, 1><<<(n + 3) / 4, 256, 0, c.stream>>>(w.sys, w.force_tiles, n, p, qq, g, c.ntot, kv,
                                                                  (T *)gpos, (T *)gq);
        break;
    case 2:
        k_vjp_gather<T, KV, 2><<<(n + 1) / 2, 256, 0, c.stream>>>(w.sys, w.force_tiles, n, p, qq, g, c.ntot, kv,
                                                                  (T *)gpos, (T *)gq);
        break;
    default:
        k_vjp_gather<T, KV, 4><<<n, 256, 0, c.stream>>>(w.sys, w.force_tiles, n, p, qq, g, c.ntot, kv, (T *)gpos,
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

hipError_t launch_vjp_real(const LaunchCfg &c, const Workspace &w, const void *gF, void *gpos, void *gq,
                           int accumulate)
{
    if (c.prec == RBE_FP64)
        k_vjp_real<double><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, w.cell_start, w.sorted_idx,
                                                                 w.sorted, (const double *)gF, c.ntot,
                                                                 (double *)gpos, (double *)gq, accumulate);
    else
        k_vjp_real<float><<<c.n_part_tiles, 256, 0, c.stream>>>(w.sys, w.part_tiles, w.cell_start, w.sorted_idx,
                                                                w.sorted, (const float *)gF, c.ntot, (float *)gpos,
                                                                (float *)gq, accumulate);
    return hipGetLastError();
}

}  // namespace rbe
