// rbe_real.hip -- real-space kernels of librbe (gfx950).
//
// Paper: Jin, Li, Xu & Zhao, arXiv:2010.01559: the truncated erfc sum of
// eq. (2.9) and the second term of eq. (2.11); the shifted Lennard-Jones
// repulsion of eq. (4.1), with r_off = 0 or, from per-particle diameters,
// r_off = (d_i + d_j)/2 - sigma (Sec. 4.2).  The paper leaves the neighbour
// search open; here it is a cell list with cells of side >= the largest
// cutoff (+ skin), rebuilt for every stand-alone evaluation, and inside
// rbe_step a Verlet list of the pairs within cutoff + skin, rebuilt on the
// device whenever some particle has moved more than skin/2 since the last
// build (the rebuild step evaluates the forces on the cell list and writes
// the list in the same pass).
//
// Pair force on particle i: phi(r) d with d = r_j - r_i (minimum image),
//   phi = -coulomb q_i q_j (erfc(beta r)/r + 2 beta exp(-alpha r^2)/sqrt(pi)) / r^2
//         + 4 eps (6 (sigma/r)^6 - 12 (sigma/r)^12) / r^2        (r < R_c)
// with beta = sqrt(alpha); the Coulomb part acts for r <= r_c.
//
// Work decomposition ("row lanes"): the 27-cell stencil of a particle is
// nine rows of three x-adjacent cells, and each row is one lane.  A wave
// holds seven particles x nine rows; the rows are contiguous ranges of the
// cell-sorted particle array (two ranges where the row wraps in x), read
// straight from global memory, where the array stays cache-resident.  A lane
// first marks the partners within the largest cutoff in a 64-bit mask (a
// cheap distance test, no branches) and then evaluates the pair terms over
// the set bits, so the expensive terms do not diverge on the cutoff test.
// Each lane accumulates its FP32 pair terms exactly (on a fixed grid, see
// qterm); the nine row sums are added in a fixed order, so the result does not
// depend on the order of the particles inside a cell (which comes from atomic
// counters) nor on the path (cell or list pass).  Systems with fewer than
// three cells per side use all-pairs tiles.
//
// List pass: LPP lanes per particle walk its list in strides of LPP; the
// LPP partial sums are combined by a fixed butterfly.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "rbe_device.h"
#include "rbe_internal.h"

namespace rbe {

constexpr int RL_BS = 256;                  // threads per block: 4 waves
constexpr int RL_PPW = 7;                   // particles per wave (9 lanes each)
constexpr int RL_PPB = 4 * RL_PPW;          // particles per block
constexpr int RL_ALLPAIRS = 256;            // particles per all-pairs tile

int real_rows_per_tile() { return RL_PPB; }
int real_allpairs_per_tile() { return RL_ALLPAIRS; }

template <typename T>
struct RBT;
template <>
struct RBT<float> {
    using Rec = PackF;
};
template <>
struct RBT<double> {
    using Rec = PartD;
};

struct PairE {
    double e_real, e_lj;
};

// Single-precision pair terms are added on a fixed grid of 2^-32 (as integers
// held in double): every partial sum is exact, so a particle's real-space
// force does not depend on the order in which its partners are visited (cell
// ranks come from atomic counters; list and cell passes order partners
// differently).  This holds while partial sums stay below 2^21 in magnitude
// (an LJ wall at r = 0.45 sigma, far inside anything these systems reach);
// the grid is far below single-precision rounding of the forces.
// A pair's force component phi * d on that grid.  In single precision the
// scale is applied to phi first (a power of two, so (phi 2^32) d rounds to
// the same float as (phi d) 2^32), and the rounding to an integer is done in
// single precision, where it is exact: the same values as
// rint((double)(phi d) * 2^32) with fewer double-precision instructions.
__device__ __forceinline__ float qphi(float phi) { return phi * 0x1p32f; }

// Flags a single-precision partial sum (in units of 2^-32) that has reached
// 2^52, half the range in which the grid sums are exact (checked at the end
// of each lane's sum and after the lanes of a particle are combined): only
// particles pressed far into each other's LJ wall get there (a force of
// 2^20), and then the forces are reported as unusable instead of silently
// losing exactness.
__device__ __forceinline__ void range_check(double x, double y, double z, int32_t *flag)
{
    if (fmax(fabs(x), fmax(fabs(y), fabs(z))) >= 0x1p52) atomicOr(flag, kFlagRange);
}
__device__ __forceinline__ double qphi(double phi) { return phi; }
__device__ __forceinline__ double qterm(float scaled) { return (double)rintf(scaled); }
__device__ __forceinline__ double qterm(double v) { return v; }
template <typename T>
__device__ __forceinline__ double qscale()
{
    return sizeof(T) == 4 ? 0x1p-32 : 1.0;
}

// Single-precision constants of one system's pair terms, held in registers.
struct PairConstF {
    float rc2, lj_rc2, beta, nalpha_log2e, two_beta_rsqrtpi, coulomb, lj_sig2, eps4, lj_shift;
    int lj_on;
};

__device__ __forceinline__ PairConstF pair_const_f(const SysDev &S)
{
    PairConstF c;
    c.rc2 = (float)S.rc2;
    c.lj_rc2 = (float)S.lj_rc2;
    c.beta = (float)S.beta;
    c.nalpha_log2e = (float)(-S.alpha * 1.4426950408889634074);
    c.two_beta_rsqrtpi = (float)(2.0 * S.beta / 1.7724538509055160273);
    c.coulomb = (float)S.coulomb;
    c.lj_sig2 = (float)S.lj_sig2;
    c.eps4 = (float)(4.0 * S.lj_eps);
    c.lj_shift = (float)S.lj_shift;
    c.lj_on = S.lj_on && !S.diam_on;   // with diameters the LJ term is formed in double (lj_offset)
    return c;
}

// erfc(x) exp(x^2) = t * sum_k c_k t^k with t = 1/(1 + 0.47047 x), x >= 0: the
// form of Abramowitz & Stegun 7.1.26 refitted to degree 9 for a relative
// error of erfc below 4e-7 in single precision on [0, 8] (fit_erfc.py).
__device__ __forceinline__ float erfc_scaled_f32(float x)
{
    const float t = __builtin_amdgcn_rcpf(fmaf(0.47047f, x, 1.0f));
    float s = -4.859511559e-02f;
    s = fmaf(s, t, 2.750724646e-01f);
    s = fmaf(s, t, -5.785352996e-01f);
    s = fmaf(s, t, 4.823851487e-01f);
    s = fmaf(s, t, -1.365632976e-01f);
    s = fmaf(s, t, 2.525006764e-01f);
    s = fmaf(s, t, 2.213245585e-01f);
    s = fmaf(s, t, 2.670528048e-01f);
    s = fmaf(s, t, 2.653580831e-01f);
    return s * t;
}

// phi(r) of one pair in single precision (r2 = |d|^2 in box units); both
// terms are evaluated and selected, so a wave does not branch on the
// per-lane cutoff tests.  With ENERGY, half the pair energies are added to e.
template <bool ENERGY>
__device__ __forceinline__ float pair_phi(const PairConstF &c, float qi, float qj, float r2, PairE &e)
{
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv;
    const bool in_c = r2 <= c.rc2;
    const bool in_lj = c.lj_on && r2 < c.lj_rc2;
    const float r = r2 * rinv;
    const float ex = __builtin_amdgcn_exp2f(c.nalpha_log2e * r2);   // exp(-alpha r^2)
    const float ec = erfc_scaled_f32(c.beta * r) * ex;               // erfc(beta r)
    const float g = fmaf(ec, rinv, c.two_beta_rsqrtpi * ex) * rinv2;
    const float cq = c.coulomb * qi * qj;
    const float sr2 = c.lj_sig2 * rinv2;
    const float sr6 = sr2 * sr2 * sr2;
    const float plj = c.eps4 * fmaf(-12.0f, sr6, 6.0f) * sr6 * rinv2;
    if constexpr (ENERGY) {
        if (in_c) e.e_real += 0.5 * (double)(cq * ec * rinv);
        if (in_lj) e.e_lj += 0.5 * ((double)c.eps4 * ((double)sr6 * sr6 - sr6) + c.lj_shift);
    }
    return (in_c ? -cq * g : 0.0f) + (in_lj ? plj : 0.0f);
}

// The same in double precision (libm erfc/exp).
template <bool ENERGY>
__device__ __forceinline__ double pair_phi(const SysDev &S, double qi, double qj, double r2, PairE &e)
{
    double phi = 0.0;
    if (r2 <= S.rc2) {
        const double r = sqrt(r2);
        const double ec = erfc(S.beta * r);
        const double ex = exp(-S.alpha * r2);
        const double g = (ec / r + 2.0 / 1.7724538509055160273 * S.beta * ex) / r2;
        const double cq = S.coulomb * qi * qj;
        phi = -cq * g;
        if constexpr (ENERGY) e.e_real += 0.5 * cq * ec / r;
    }
    if (S.lj_on && !S.diam_on && r2 < S.lj_rc2) {
        const double sr2 = S.lj_sig2 / r2;
        const double sr6 = sr2 * sr2 * sr2;
        phi += 4.0 * S.lj_eps * (6.0 * sr6 - 12.0 * sr6 * sr6) / r2;
        if constexpr (ENERGY) e.e_lj += 0.5 * (4.0 * S.lj_eps * (sr6 * sr6 - sr6) + S.lj_shift);
    }
    return phi;
}

// Shifted LJ of eq. (4.1) with r_off = (d_i + d_j)/2 - sigma from the two
// diameters, in double: s = r - r_off is a small difference of two
// distances that can be fifty times larger (a colloid against an ion), so r
// comes from the exact displacement and s is formed in double.  Returns
// dV/dr / r (the coefficient of d in the force on i) and adds half the pair
// energy when ENERGY.
template <bool ENERGY>
__device__ __forceinline__ double lj_offset(const SysDev &S, double di, double dj, double r2, PairE &e)
{
    const double r = sqrt(r2);
    const double sv = r - (0.5 * (di + dj) - S.lj_sig);
    if (!(sv < S.lj_rc)) return 0.0;
    const double sr2 = S.lj_sig2 / (sv * sv);
    const double sr6 = sr2 * sr2 * sr2;
    if constexpr (ENERGY) e.e_lj += 0.5 * (4.0 * S.lj_eps * (sr6 * sr6 - sr6) + S.lj_shift);
    return 4.0 * S.lj_eps * (6.0 * sr6 - 12.0 * sr6 * sr6) / (sv * r);
}

// |d|^2 of two records in double: exact wrapped integer differences for
// PackF, the wrapped double difference for PartD.
__device__ __forceinline__ double r2_double(const PackF &a, const PackF &b, double L)
{
    const double u = L * (1.0 / 4294967296.0);
    const double dx = (double)(int32_t)(b.x - a.x) * u, dy = (double)(int32_t)(b.y - a.y) * u,
                 dz = (double)(int32_t)(b.z - a.z) * u;
    return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ double r2_double(const PartD &a, const PartD &b, double L)
{
    double sx = b.x - a.x, sy = b.y - a.y, sz = b.z - a.z;
    sx = (sx - rint(sx)) * L;
    sy = (sy - rint(sy)) * L;
    sz = (sz - rint(sz)) * L;
    return sx * sx + sy * sy + sz * sz;
}

// Displacement between two records.  rmax2 is the largest cutoff squared in
// the record's own units (fixed-point units for PackF).
struct Geo {
    float scale;     // PackF: box length of one fixed-point unit
    float rmax2u;    // PackF: search radius^2 in fixed-point units
    double rmax2;    // PartD: search radius^2
    double L;
};

template <typename T>
__device__ __forceinline__ Geo make_geo(const SysDev &S)
{
    Geo g;
    const double rmax2 = S.rsearch2;
    g.scale = (float)(S.L * (1.0 / 4294967296.0));
    g.rmax2u = (float)(rmax2 / ((double)g.scale * (double)g.scale));
    g.rmax2 = rmax2;
    g.L = S.L;
    return g;
}

// The same with the list radius (cutoff + skin) as search radius.
__device__ __forceinline__ Geo list_geo(const SysDev &S)
{
    Geo g;
    g.scale = (float)(S.L * (1.0 / 4294967296.0));
    g.rmax2u = (float)(S.rlist2 / ((double)g.scale * (double)g.scale));
    g.rmax2 = S.rlist2;
    g.L = S.L;
    return g;
}

__device__ __forceinline__ bool near_test(const PackF &pa, const PackF &pb, const Geo &g)
{
    const float ux = (float)(int32_t)(pb.x - pa.x);
    const float uy = (float)(int32_t)(pb.y - pa.y);
    const float uz = (float)(int32_t)(pb.z - pa.z);
    return fmaf(ux, ux, fmaf(uy, uy, uz * uz)) <= g.rmax2u;
}

__device__ __forceinline__ void displacement(const PackF &pa, const PackF &pb, const Geo &g, float &dx, float &dy,
                                             float &dz, float &r2)
{
    dx = (float)(int32_t)(pb.x - pa.x) * g.scale;
    dy = (float)(int32_t)(pb.y - pa.y) * g.scale;
    dz = (float)(int32_t)(pb.z - pa.z) * g.scale;
    r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

__device__ __forceinline__ void displacement(const PartD &pa, const PartD &pb, const Geo &g, double &dx, double &dy,
                                             double &dz, double &r2)
{
    double sx = pb.x - pa.x, sy = pb.y - pa.y, sz = pb.z - pa.z;
    sx -= rint(sx);
    sy -= rint(sy);
    sz -= rint(sz);
    dx = sx * g.L;
    dy = sy * g.L;
    dz = sz * g.L;
    r2 = dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ bool near_test(const PartD &pa, const PartD &pb, const Geo &g)
{
    double dx, dy, dz, r2;
    displacement(pa, pb, g, dx, dy, dz, r2);
    return r2 <= g.rmax2;
}

template <typename T>
__device__ __forceinline__ void cell_coords(const PackF &p, int nc, int &cx, int &cy, int &cz)
{
    cx = cell_of_fix(p.x, nc);
    cy = cell_of_fix(p.y, nc);
    cz = cell_of_fix(p.z, nc);
}

template <typename T>
__device__ __forceinline__ void cell_coords(const PartD &p, int nc, int &cx, int &cy, int &cz)
{
    cx = cell_of_frac(p.x, nc);
    cy = cell_of_frac(p.y, nc);
    cz = cell_of_frac(p.z, nc);
}

// One stencil row of a particle: cells cx-1..cx+1 of row (yy, zz), x taken
// modulo nc, as one or two contiguous ranges of cell-sorted slots.  Ranges of
// at most 64 slots are scanned into hit masks (records within the search
// radius, self excluded); longer ranges are left for a direct walk.
struct RowScan {
    int b0[2], b1[2];
    uint64_t m[2];
    int nseg;
    bool walk;   // some range exceeds 64 slots
};

template <typename Rec>
__device__ __forceinline__ void row_scan(const Rec &pa, int self, int cx, int yy, int zz, int nc,
                                         const int32_t *st, const Rec *gs, const Geo &geo, RowScan &rs, int lo,
                                         int hi)
{
    const int base = (zz * nc + yy) * nc;
    if (cx >= 1 && cx + 1 < nc) {
        rs.b0[0] = st[base + cx - 1];
        rs.b1[0] = st[base + cx + 2];
        rs.nseg = 1;
    } else if (cx == 0) {
        rs.b0[0] = st[base];
        rs.b1[0] = st[base + 2];
        rs.b0[1] = st[base + nc - 1];
        rs.b1[1] = st[base + nc];
        rs.nseg = 2;
    } else {
        rs.b0[0] = st[base + nc - 2];
        rs.b1[0] = st[base + nc];
        rs.b0[1] = st[base];
        rs.b1[1] = st[base + 1];
        rs.nseg = 2;
    }
    rs.walk = false;
    rs.m[0] = rs.m[1] = 0;
    if (rs.nseg == 1) rs.b0[1] = rs.b1[1] = lo;
    // cell starts come from the last complete scan; clamped to the system's
    // slots [lo, hi) every range stays in bounds whatever they hold
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        rs.b0[s] = min(max(rs.b0[s], lo), hi);
        rs.b1[s] = min(max(rs.b1[s], rs.b0[s]), hi);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int b0 = rs.b0[s], b1 = rs.b1[s];
        uint64_t m = 0;
        if (b1 - b0 <= 64) {
            // two candidates per round, both loaded and tested without
            // branches; their two bits enter the mask with one shift.  The
            // second record is read even one past the segment (the record
            // array ends with a padding record) and its bit dropped there;
            // the particle itself is dropped once, after the loop
            for (int b = b0; b < b1; b += 2) {
                const Rec p0 = gs[b];
                const Rec p1 = gs[b + 1];
                const uint32_t h0 = (uint32_t)near_test(pa, p0, geo);
                const uint32_t h1 = (uint32_t)near_test(pa, p1, geo) & (uint32_t)(b + 1 < b1);
                m |= (uint64_t)(h0 | (h1 << 1)) << (b - b0);
            }
            if (self >= b0 && self < b1) m &= ~(1ull << (self - b0));
        } else {
            rs.walk = true;
        }
        rs.m[s] = m;
    }
}

// Calls f(pb, b) for every hit of a scanned row (masks, then direct walks).
template <typename Rec, typename F>
__device__ __forceinline__ void row_visit(const Rec &pa, int self, const RowScan &rs, const Rec *gs, const Geo &geo,
                                          F &&f)
{
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int b0 = rs.b0[s], b1 = rs.b1[s];
        if (b1 - b0 <= 64) {
            uint64_t m = rs.m[s];
            while (m) {
                const int o = __builtin_ctzll(m);
                m &= m - 1;
                f(gs[b0 + o], b0 + o);
            }
        } else {
            for (int b = b0; b < b1; ++b) {
                if (b == self) continue;
                const Rec pb = gs[b];
                if (near_test(pa, pb, geo)) f(pb, b);
            }
        }
    }
}

template <typename T>
struct RealArgs {
    const SysDev *sys;
    const Tile *tiles;       // aux = 0: row-lane tile of RL_PPB sorted slots; 1: all-pairs tile
    const int32_t *start;
    const int32_t *sorted_idx;
    const void *sorted;
    const void *packed;      // original order (all-pairs tiles)
    const T *q;              // energies: charges in original order
    int64_t ntot;
    T *F;
    int accumulate;
    T *vel;                  // kick target (may be NULL); velocities for kinetic energy when ENERGY
    int32_t *flag;
    double *epart;           // ENERGY: [tiles][8]
    const void *km;          // per-mode force constants (KModeF / KModeD) for the fused Fourier force
    uint64_t kick_step;      // index of the step whose closing half kick is applied (its time step)
    const double *diam;      // per-particle diameters (original order) when some system has them
};

// Neighbour-list state seen by the real-space pass of a step.
struct ListArgs {
    ListStep ls;
    int32_t *count;          // cell counts, cleared here after a rebuild gave up
    int ncell_tot;
    const Tile *list_tiles;
    int n_rows, n_list;      // tiles of the cell pass and of the list pass
    int32_t *nbr;            // [kmax][Ntot] partner slots, column k of slot s at k * Ntot + s
    int32_t *nnb;
    int kmax;
    int single_n, single_p;  // single-system context (SINGLE launches): its particle and mode counts
};

// Store (or add) the real-space force of particle i and apply the optional
// half kick; with ENERGY add the one-body sums to ev instead.
template <typename T, bool ENERGY>
__device__ __forceinline__ void finish_particle(const RealArgs<T> &a, const SysDev &S, int64_t i, double fxd,
                                                double fyd, double fzd, double *ev)
{
    if constexpr (ENERGY) {
        if (a.vel) {
            const double x = a.vel[i], y = a.vel[a.ntot + i], z = a.vel[2 * a.ntot + i];
            ev[3] += 0.5 * S.mass * (x * x + y * y + z * z);
        }
        const double qq = (double)a.q[i];
        ev[4] += qq * qq;
        ev[5] += qq;
        ev[6] += fabs(qq);
        return;
    }
    if (i < S.off || i >= (int64_t)S.off + S.n) {
        // the slot's particle index is stale (a rebuild gave up before its scatter)
        atomicOr(a.flag, kFlagBounds);
        return;
    }
    T fx = (T)fxd, fy = (T)fyd, fz = (T)fzd;
    if (!isfinite(fx + fy + fz)) atomicOr(a.flag, kFlagNonFinite);
    if (a.accumulate) {
        fx += a.F[i];
        fy += a.F[a.ntot + i];
        fz += a.F[2 * a.ntot + i];
    }
    a.F[i] = fx;
    a.F[a.ntot + i] = fy;
    a.F[2 * a.ntot + i] = fz;
    if (a.vel && i - S.off >= S.n_fixed) {
        // the same rounding as the deferred kick of the integrator
        const double h = 0.5 * step_dt(S, a.kick_step) / S.mass;
        a.vel[i] = (T)fma(h, (double)fx, (double)a.vel[i]);
        a.vel[a.ntot + i] = (T)fma(h, (double)fy, (double)a.vel[a.ntot + i]);
        a.vel[2 * a.ntot + i] = (T)fma(h, (double)fz, (double)a.vel[2 * a.ntot + i]);
    }
}

template <typename T>
struct PairCT {
    using type = SysDev;
};
template <>
struct PairCT<float> {
    using type = PairConstF;
};

template <typename T>
__device__ __forceinline__ typename PairCT<T>::type pair_consts(const SysDev &S);
template <>
__device__ __forceinline__ PairConstF pair_consts<float>(const SysDev &S)
{
    return pair_const_f(S);
}
template <>
__device__ __forceinline__ SysDev pair_consts<double>(const SysDev &S)
{
    return S;
}

// ---------------------------------------------------------------------------
// Fourier force fused into the real-space pass of a step (eq. 3.6).  Wave w of
// the block sums the modes of quarter w, [w P/4, (w+1) P/4), in mode order for
// every particle of the tile (64 per pass, one per lane; the mode constants are
// wave-uniform), and leaves the partial sum in LDS; the particle's lane adds
// the quarters in a fixed order when it finishes the particle.  The decomposition
// is the same on every tile shape, so the Fourier force of a particle does not
// depend on the real-space path.
// ---------------------------------------------------------------------------
constexpr int FT_MAX = 256;   // particles per tile, any shape

template <typename T>
struct KMT;
template <>
struct KMT<float> {
    using type = KModeF;
};
template <>
struct KMT<double> {
    using type = KModeD;
};

template <typename T>
using Four = T (*)[FT_MAX][3];

template <typename T>
__device__ __forceinline__ void fourier_tile(const RealArgs<T> &a, const SysDev &S, const void *recs, int first,
                                             int count, Four<T> s4)
{
    using Rec = typename RBT<T>::Rec;
    using KM = typename KMT<T>::type;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int l0 = (S.p * wave) / 4, l1 = (S.p * (wave + 1)) / 4;
    const KM *kk = reinterpret_cast<const KM *>(a.km) + S.moff;
    const Rec *rp = reinterpret_cast<const Rec *>(recs) + first;
    for (int p0 = 0; p0 < count; p0 += 64) {
        const int p = p0 + lane;
        T f[3] = {0, 0, 0};
        if (p < count) {
            const Rec r = rp[p];
            if constexpr (sizeof(T) == 4) {
                float h[3], lo[3];
                split_fix(r.x, S, h[0], lo[0]);
                split_fix(r.y, S, h[1], lo[1]);
                split_fix(r.z, S, h[2], lo[2]);
                fourier_range(kk, l0, l1, h, lo, f);
            } else {
                const double s3[3] = {r.x, r.y, r.z};
                fourier_range(kk, l0, l1, s3, f);
            }
            s4[wave][p][0] = f[0];
            s4[wave][p][1] = f[1];
            s4[wave][p][2] = f[2];
        }
    }
}

// Adds the Fourier force of tile particle k (charge qi) to (fx, fy, fz).
template <typename T>
__device__ __forceinline__ void add_fourier(Four<T> s4, int k, T qi, double &fx, double &fy, double &fz)
{
    if (!s4) return;
    T g[3];
    for (int d = 0; d < 3; ++d) g[d] = ((s4[0][k][d] + s4[1][k][d]) + s4[2][k][d]) + s4[3][k][d];
    fx += (double)(-qi * g[0]);
    fy += (double)(-qi * g[1]);
    fz += (double)(-qi * g[2]);
}

// All-pairs tile: particles [start, start + count) of a one-cell system, one
// per thread, partners in original index order.  DIAM compiles the
// per-particle-diameter LJ (only launches of contexts with diameters).
template <typename T, bool ENERGY, bool DIAM>
__device__ __forceinline__ void allpairs_body(const RealArgs<T> &a, const Tile &t, const SysDev &S, double *ev,
                                              Four<T> s4 = nullptr)
{
    using Rec = typename RBT<T>::Rec;
    const Geo geo = make_geo<T>(S);
    const auto pc = pair_consts<T>(S);
    const Rec *pk = reinterpret_cast<const Rec *>(a.packed) + S.off;
    if ((int)threadIdx.x >= t.count) return;
    const int il = t.start + threadIdx.x;
    const Rec pa = pk[il];
    const double da = DIAM && S.diam_on ? a.diam[S.off + il] : 0.0;
    double fx = 0, fy = 0, fz = 0;
    PairE e{0, 0};
    for (int j = 0; j < S.n; ++j) {
        if (j == il) continue;
        const Rec pb = pk[j];
        if (!near_test(pa, pb, geo)) continue;
        T dx, dy, dz, r2;
        displacement(pa, pb, geo, dx, dy, dz, r2);
        T phi = pair_phi<ENERGY>(pc, (T)pa.q, (T)pb.q, r2, e);
        if (DIAM && S.diam_on) phi += (T)lj_offset<ENERGY>(S, da, a.diam[S.off + j], r2_double(pa, pb, S.L), e);
        const T ph = qphi(phi);
        fx += qterm(ph * dx);
        fy += qterm(ph * dy);
        fz += qterm(ph * dz);
        if constexpr (ENERGY) ev[2] += 0.5 * (double)(phi * r2);
    }
    if constexpr (ENERGY) {
        ev[0] += e.e_real;
        ev[1] += e.e_lj;
    }
    if constexpr (sizeof(T) == 4) range_check(fx, fy, fz, a.flag);
    fx *= qscale<T>();
    fy *= qscale<T>();
    fz *= qscale<T>();
    add_fourier<T>(s4, (int)threadIdx.x, (T)pa.q, fx, fy, fz);
    finish_particle<T, ENERGY>(a, S, S.off + il, fx, fy, fz, ev);
}

// Row-lane tile on the cell list.  With BUILD the rows are scanned with the
// list radius and every hit is also written to the particle's list: the nine
// row counts are prefixed in LDS so that the list keeps row order.
template <typename T, bool ENERGY, bool BUILD, bool DIAM>
__device__ __forceinline__ void rows_body(const RealArgs<T> &a, const ListArgs *la, const Tile &t, const SysDev &S,
                                          double *ev, Four<T> s4 = nullptr)
{
    using Rec = typename RBT<T>::Rec;
    __shared__ double s_red[ENERGY ? 6 : 3][RL_BS];
    __shared__ int s_cnt[BUILD ? RL_BS : 1];
    const Geo geo = BUILD ? list_geo(S) : make_geo<T>(S);
    const auto pc = pair_consts<T>(S);
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int p = lane / 9, r = lane - 9 * (lane / 9);
    const int k = wave * RL_PPW + p;
    const bool act = lane < 9 * RL_PPW && k < t.count;
    double fx = 0, fy = 0, fz = 0, vir = 0;
    PairE e{0, 0};
    int slot = -1;
    const Rec *gs = reinterpret_cast<const Rec *>(a.sorted);
    Rec pa{};
    RowScan rs;
    rs.nseg = 0;
    rs.walk = false;
    rs.b0[0] = rs.b0[1] = rs.b1[0] = rs.b1[1] = 0;
    rs.m[0] = rs.m[1] = 0;
    int64_t iorig = 0;   // original index, loaded with the record (see list_body)
    if (act) {
        slot = S.off + t.start + k;
        pa = gs[slot];
        iorig = a.sorted_idx[slot];
        const int nc = S.nc;
        int cx, cy, cz;
        cell_coords<T>(pa, nc, cx, cy, cz);
        const int zz = (cz + r / 3 - 1 + nc) % nc, yy = (cy + r % 3 - 1 + nc) % nc;
        const int32_t *st = a.start + S.cell_off + t.sys;
        row_scan(pa, slot, cx, yy, zz, nc, st, gs, geo, rs, S.off, S.off + S.n);
    }
    const double da = DIAM && act && S.diam_on ? a.diam[iorig] : 0.0;
    int pos = 0, total = 0;
    if constexpr (BUILD) {
        const int cnt = __builtin_popcountll(rs.m[0]) + __builtin_popcountll(rs.m[1]);
        s_cnt[tid] = cnt + (rs.walk ? (1 << 20) : 0);   // a walked row cannot be listed
        __syncthreads();
        if (act) {
            const int first = tid - r;
            for (int j = 0; j < 9; ++j) {
                const int v = s_cnt[first + j];
                if (j < r) pos += v;
                total += v;
            }
        }
    }
    if (act) {
        row_visit(pa, slot, rs, gs, geo, [&](const Rec &pb, int b) {
            T dx, dy, dz, r2;
            displacement(pa, pb, geo, dx, dy, dz, r2);
            T phi = pair_phi<ENERGY>(pc, (T)pa.q, (T)pb.q, r2, e);
            if (DIAM && S.diam_on)
                phi += (T)lj_offset<ENERGY>(S, da, a.diam[a.sorted_idx[b]], r2_double(pa, pb, S.L), e);
            const T ph = qphi(phi);
            fx += qterm(ph * dx);
            fy += qterm(ph * dy);
            fz += qterm(ph * dz);
            if constexpr (ENERGY) vir += 0.5 * (double)(phi * r2);
            if constexpr (BUILD) {
                if (pos < la->kmax) la->nbr[(int64_t)pos * a.ntot + slot] = b;
                ++pos;
            }
        });
    }
    if constexpr (sizeof(T) == 4) range_check(fx, fy, fz, a.flag);
    // add the nine row sums of each particle in row order
    s_red[0][tid] = fx;
    s_red[1][tid] = fy;
    s_red[2][tid] = fz;
    if constexpr (ENERGY) {
        s_red[3][tid] = e.e_real;
        s_red[4][tid] = e.e_lj;
        s_red[5][tid] = vir;
    }
    __syncthreads();
    if (act && r == 0) {
        double sx = 0, sy = 0, sz = 0;
        for (int j = 0; j < 9; ++j) {
            sx += s_red[0][tid + j];
            sy += s_red[1][tid + j];
            sz += s_red[2][tid + j];
        }
        if constexpr (sizeof(T) == 4) range_check(sx, sy, sz, a.flag);
        if constexpr (ENERGY)
            for (int j = 0; j < 9; ++j) {
                ev[0] += s_red[3][tid + j];
                ev[1] += s_red[4][tid + j];
                ev[2] += s_red[5][tid + j];
            }
        if constexpr (BUILD) {
            // an overflowing list is never read (the next step rebuilds)
            const bool ok = total <= la->kmax;
            la->nnb[slot] = ok ? total : 0;
            if (!ok) atomicOr(la->ls.overflow, 1);
        }
        sx *= qscale<T>();
        sy *= qscale<T>();
        sz *= qscale<T>();
        add_fourier<T>(s4, k, (T)pa.q, sx, sy, sz);
        finish_particle<T, ENERGY>(a, S, iorig, sx, sy, sz, ev);
    }
}

// Block partials of the energy sums.
__device__ __forceinline__ void energy_block(double *ev, double *out)
{
    __shared__ double s_blk[8][RL_BS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = 0; k < 8; ++k) {
        double v = ev[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) s_blk[k][wave] = v;
    }
    __syncthreads();
    if (tid < 8) {
        double v = 0.0;
        for (int w = 0; w < RL_BS / 64; ++w) v += s_blk[tid][w];
        out[tid] = v;
    }
}

template <typename T, bool ENERGY, bool DIAM>
__global__ __launch_bounds__(RL_BS) void k_real_rows(RealArgs<T> a)
{
    const Tile t = a.tiles[blockIdx.x];
    const SysDev S = a.sys[t.sys];
    double ev[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (t.aux == 1)
        allpairs_body<T, ENERGY, DIAM>(a, t, S, ev);
    else
        rows_body<T, ENERGY, false, DIAM>(a, nullptr, t, S, ev);
    if constexpr (ENERGY) energy_block(ev, a.epart + 8 * blockIdx.x);
}

// List tile: LPP lanes per cell-sorted slot, U partners per lane and round.
constexpr int kListU = 4;

// What the list pass of a tile particle loads before its partners: its
// record, original index (where its force goes) and list length, and the
// raw partner slots of its first round.  None depends on the Fourier part,
// so the force launch issues these loads before it and their latency
// overlaps the Fourier arithmetic.  The first round's slots are read whatever
// the length (its columns, below 4 LPP <= 32, lie inside the list's kmax
// columns; a clamp keeps them there) and replaced by the particle's own slot
// past the length before any is used.
template <typename T>
struct ListHead {
    typename RBT<T>::Rec pa;
    int64_t iorig;
    int n, slot;
    int b[kListU];
};

template <typename T, int LPP>
__device__ __forceinline__ void list_head(const RealArgs<T> &a, const ListArgs &la, const Tile &t, const SysDev &S,
                                          ListHead<T> &h)
{
    using Rec = typename RBT<T>::Rec;
    const int tid = threadIdx.x;
    const int k = tid / LPP, sub = tid % LPP;
    h.n = 0;
    h.slot = 0;
    h.iorig = 0;
    h.pa = Rec{};
    if (k < t.count) {
        h.slot = S.off + t.start + k;
        h.pa = reinterpret_cast<const Rec *>(a.sorted)[h.slot];
        h.iorig = a.sorted_idx[h.slot];
        h.n = la.nnb[h.slot];
        const int32_t *nb = la.nbr + h.slot;
#pragma unroll
        for (int u = 0; u < kListU; ++u) h.b[u] = nb[(int64_t)min(sub + u * LPP, la.kmax - 1) * a.ntot];
    }
}

// Real-space force of tile particle k from its list, summed over the
// particle's LPP lanes (each of them holds the sum).
template <typename T, int LPP, bool DIAM>
__device__ __forceinline__ void list_pairs(const RealArgs<T> &a, const ListArgs &la, const Tile &t, const SysDev &S,
                                           const ListHead<T> &h, double &fx, double &fy, double &fz)
{
    using Rec = typename RBT<T>::Rec;
    const Geo geo = make_geo<T>(S);
    const auto pc = pair_consts<T>(S);
    const int tid = threadIdx.x;
    const int k = tid / LPP, sub = tid % LPP;
    fx = 0;
    fy = 0;
    fz = 0;
    const Rec pa = h.pa;
    const int slot = h.slot, n = h.n;
    if (k < t.count) {
        const Rec *gs = reinterpret_cast<const Rec *>(a.sorted);
        const double da = DIAM && S.diam_on ? a.diam[h.iorig] : 0.0;
        const int32_t *nb = la.nbr + slot;
        PairE e{0, 0};
        constexpr int U = kListU;
        int b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) b[u] = sub + u * LPP < n ? h.b[u] : slot;
        for (int j = sub; j < n; j += U * LPP) {
            // this round's partner records, then the next round's partner
            // slots, so that those loads overlap this round's pairs
            Rec pb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) pb[u] = gs[b[u]];
            int bn[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int jj = j + U * LPP + u * LPP;
                bn[u] = jj < n ? nb[(int64_t)jj * a.ntot] : slot;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (j + u * LPP < n) {
                    T dx, dy, dz, r2;
                    displacement(pa, pb[u], geo, dx, dy, dz, r2);
                    T phi = pair_phi<false>(pc, (T)pa.q, (T)pb[u].q, r2, e);
                    if (DIAM && S.diam_on)
                        phi += (T)lj_offset<false>(S, da, a.diam[a.sorted_idx[b[u]]], r2_double(pa, pb[u], S.L), e);
                    const T ph = qphi(phi);
                    fx += qterm(ph * dx);
                    fy += qterm(ph * dy);
                    fz += qterm(ph * dz);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) b[u] = bn[u];
        }
    }
    if constexpr (sizeof(T) == 4) range_check(fx, fy, fz, a.flag);
#pragma unroll
    for (int o = 1; o < LPP; o <<= 1) {
        fx += __shfl_xor(fx, o, 64);
        fy += __shfl_xor(fy, o, 64);
        fz += __shfl_xor(fz, o, 64);
    }
}

// Last step of a list particle (its first lane): scale of the real-space sum,
// the Fourier force from the tile's quarter sums, store.
template <typename T, int LPP>
__device__ __forceinline__ void list_finish(const RealArgs<T> &a, const Tile &t, const SysDev &S, const ListHead<T> &h,
                                            Four<T> s4, double fx, double fy, double fz)
{
    const int tid = threadIdx.x;
    const int k = tid / LPP, sub = tid % LPP;
    if (k < t.count && sub == 0) {
        if constexpr (sizeof(T) == 4) range_check(fx, fy, fz, a.flag);
        fx *= qscale<T>();
        fy *= qscale<T>();
        fz *= qscale<T>();
        add_fourier<T>(s4, k, (T)h.pa.q, fx, fy, fz);
        finish_particle<T, false>(a, S, h.iorig, fx, fy, fz, nullptr);
    }
}

// Slot of the calling wave on its SIMD: bits 3:0 (WAVE_ID) of the HW_ID
// hardware register, read with s_getreg_b32 (operand: (size - 1) << 11 |
// offset << 6 | register, HW_ID being register 4).  It only orders
// independent work; no result depends on it.
__device__ __forceinline__ int wave_slot() { return __builtin_amdgcn_s_getreg((4 - 1) << 11 | 0 << 6 | 4); }

// Force pass of one time step: the Fourier force plus the real-space force,
// on the cell list with list build when the step's rebuild flag is set, else
// on the list; then the closing half kick on the last step of a call.  Tiles
// are taken in XCD order (xcd_tile).  On the list, a particle's real-space sum
// stays in registers and its Fourier force in the tile's LDS quarter sums
// until the finish, which adds them in a fixed order, so the order of the
// two phases does not change any result.  SINGLE (a single-system context, which
// has no all-pairs tiles when it runs list steps) forms the tile from its
// index as the host builds it, and takes the system's particle and mode
// offsets (both 0) and its mode count from the launch, so that the record and
// mode-constant loads do not wait for the tile and the system constants.
template <typename T, int LPP, bool DIAM, bool SINGLE>
__global__ __launch_bounds__(RL_BS) void k_real_step(RealArgs<T> a, ListArgs la)
{
    __shared__ T s4[4][FT_MAX][3];
    // both flags are read before anything is stored, so that neither read
    // waits for the other
    const int poison = *la.ls.poison;
    const int rebuild = *la.ls.rebuild;
    // no launch of this kernel reads the step number: advance the replay's
    // base for the next steps
    if (la.ls.step_bump && blockIdx.x == 0 && threadIdx.x == 0) *la.ls.step_bump += la.ls.bump;
    if (poison) {
        // this step's rebuild gave up before its scan cleared the cell counts
        for (int k = blockIdx.x * RL_BS + threadIdx.x; k < la.ncell_tot; k += gridDim.x * RL_BS) la.count[k] = 0;
    }
    const int nb = rebuild ? la.n_rows : la.n_list;
    if ((int)blockIdx.x >= nb) return;
    const int ti = xcd_tile((int)blockIdx.x, nb);
    Tile t;
    if constexpr (SINGLE) {
        const int per = rebuild ? RL_PPB : 256 / LPP;
        t = Tile{0, ti * per, min(per, la.single_n - ti * per), rebuild ? 0 : 2};
    } else {
        t = rebuild ? a.tiles[ti] : la.list_tiles[ti];
    }
    SysDev S = a.sys[t.sys];
    if constexpr (SINGLE) {
        S.off = 0;
        S.moff = 0;
        S.p = la.single_p;
    }
    const bool allpairs = t.aux == 1;
    if (!allpairs && !rebuild) {
        ListHead<T> h;
        list_head<T, LPP>(a, la, t, S, h);
        double fx, fy, fz;
        // the two phases are independent until the finish: waves in odd
        // slots of their SIMD take the list pairs first, the others the
        // Fourier terms, so that the waves sharing a SIMD do not all wait on
        // loads at the same time
        if (wave_slot() & 1) {
            list_pairs<T, LPP, DIAM>(a, la, t, S, h, fx, fy, fz);
            fourier_tile<T>(a, S, a.sorted, S.off + t.start, t.count, s4);
        } else {
            fourier_tile<T>(a, S, a.sorted, S.off + t.start, t.count, s4);
            list_pairs<T, LPP, DIAM>(a, la, t, S, h, fx, fy, fz);
        }
        __syncthreads();
        list_finish<T, LPP>(a, t, S, h, s4, fx, fy, fz);
        return;
    }
    fourier_tile<T>(a, S, allpairs ? a.packed : a.sorted, S.off + t.start, t.count, s4);
    __syncthreads();
    if (allpairs)
        allpairs_body<T, false, DIAM>(a, t, S, nullptr, s4);
    else
        rows_body<T, false, true, DIAM>(a, &la, t, S, nullptr, s4);
}

// Stand-alone scatter into cell order (force and energy calls; a time step
// on the neighbour list scatters inside the totals launch).
template <typename Rec>
__global__ __launch_bounds__(256) void k_scatter(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                 const int32_t *__restrict__ start, const int32_t *__restrict__ cellid,
                                                 const int32_t *__restrict__ rank, const Rec *__restrict__ packed,
                                                 int32_t *__restrict__ sorted_idx, Rec *__restrict__ sorted)
{
    const Tile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const int64_t i = sys[t.sys].off + t.start + threadIdx.x;
    const int slot = start[cellid[i] + t.sys] + rank[i];
    const Rec v = packed[i];
    sorted_idx[slot] = (int32_t)i;
    sorted[slot] = v;
}

// ---------------------------------------------------------------------------
// Real-space and LJ adjoint.  With dG = G_i - G_j and the pair force phi d:
//   dLoss/dq_i += -coulomb sum_j q_j (G(r)/r) dG.d
//   dLoss/dr_i += sum_j [ -(phi'(r)/r)(dG.d) d - phi dG ]
// G(r)/r = erfc(beta r)/r^3 + 2 beta exp(-alpha r^2)/(sqrt(pi) r^2), whose
// derivative is -3 erfc/r^4 - 6 beta e/(sqrt(pi) r^3) - 4 beta^3 e/(sqrt(pi) r).
// Same row-lane decomposition as the force.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void vjp_pair(const SysDev &S, T qi, T qj, T dx, T dy, T dz, T r2, T Gx, T Gy, T Gz,
                                         double &dq, double &rx, double &ry, double &rz)
{
    T phi = 0, dphi_r = 0, gq = 0;   // phi, phi'(r)/r, and the charge term
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
        gq = -(T)S.coulomb * qj * g * GD;
    }
    if (S.lj_on && r2 < (T)S.lj_rc2) {
        const T sr2 = (T)S.lj_sig2 / r2;
        const T sr6 = sr2 * sr2 * sr2, sr12 = sr6 * sr6;
        const T eps4 = (T)(4.0 * S.lj_eps);
        phi += eps4 * ((T)6 * sr6 - (T)12 * sr12) / r2;
        dphi_r += eps4 * ((T)168 * sr12 - (T)48 * sr6) / (r2 * r2);
    }
    dq += (double)gq;
    rx -= (double)(dphi_r * GD * dx + phi * Gx);
    ry -= (double)(dphi_r * GD * dy + phi * Gy);
    rz -= (double)(dphi_r * GD * dz + phi * Gz);
}

template <typename T>
__global__ __launch_bounds__(RL_BS) void k_vjp_real(RealArgs<T> a, const T *__restrict__ gF, T *__restrict__ gpos,
                                                    T *__restrict__ gq, int accumulate)
{
    using Rec = typename RBT<T>::Rec;
    __shared__ double s_red[4][RL_BS];
    const Tile t = a.tiles[blockIdx.x];
    const SysDev S = a.sys[t.sys];
    const Geo geo = make_geo<T>(S);
    const int tid = threadIdx.x;
    const int64_t ntot = a.ntot;
    auto finish = [&](int64_t i, double dq, double rx, double ry, double rz) {
        if (accumulate) {
            dq += gq[i];
            rx += gpos[i];
            ry += gpos[ntot + i];
            rz += gpos[2 * ntot + i];
        }
        gq[i] = (T)dq;
        gpos[i] = (T)rx;
        gpos[ntot + i] = (T)ry;
        gpos[2 * ntot + i] = (T)rz;
    };
    if (t.aux == 1) {
        const Rec *pk = reinterpret_cast<const Rec *>(a.packed) + S.off;
        if (tid < t.count) {
            const int il = t.start + tid;
            const int64_t i = S.off + il;
            const Rec pa = pk[il];
            const T Gix = gF[i], Giy = gF[ntot + i], Giz = gF[2 * ntot + i];
            double dq = 0, rx = 0, ry = 0, rz = 0;
            for (int j = 0; j < S.n; ++j) {
                if (j == il) continue;
                const Rec pb = pk[j];
                if (!near_test(pa, pb, geo)) continue;
                T dx, dy, dz, r2;
                displacement(pa, pb, geo, dx, dy, dz, r2);
                const int64_t jj = S.off + j;
                vjp_pair<T>(S, (T)pa.q, (T)pb.q, dx, dy, dz, r2, Gix - gF[jj], Giy - gF[ntot + jj],
                            Giz - gF[2 * ntot + jj], dq, rx, ry, rz);
            }
            finish(i, dq, rx, ry, rz);
        }
        return;
    }
    const int wave = tid >> 6, lane = tid & 63;
    const int p = lane / 9, r = lane - 9 * (lane / 9);
    const int k = wave * RL_PPW + p;
    const bool act = lane < 9 * RL_PPW && k < t.count;
    double dq = 0, rx = 0, ry = 0, rz = 0;
    int slot = -1;
    if (act) {
        slot = S.off + t.start + k;
        const Rec *gs = reinterpret_cast<const Rec *>(a.sorted);
        const Rec pa = gs[slot];
        const int64_t i = a.sorted_idx[slot];
        const T Gix = gF[i], Giy = gF[ntot + i], Giz = gF[2 * ntot + i];
        const int nc = S.nc;
        int cx, cy, cz;
        cell_coords<T>(pa, nc, cx, cy, cz);
        const int zz = (cz + r / 3 - 1 + nc) % nc, yy = (cy + r % 3 - 1 + nc) % nc;
        const int32_t *st = a.start + S.cell_off + t.sys;
        RowScan rs;
        row_scan(pa, slot, cx, yy, zz, nc, st, gs, geo, rs, S.off, S.off + S.n);
        row_visit(pa, slot, rs, gs, geo, [&](const Rec &pb, int b) {
            T dx, dy, dz, r2;
            displacement(pa, pb, geo, dx, dy, dz, r2);
            const int64_t jj = a.sorted_idx[b];
            vjp_pair<T>(S, (T)pa.q, (T)pb.q, dx, dy, dz, r2, Gix - gF[jj], Giy - gF[ntot + jj],
                        Giz - gF[2 * ntot + jj], dq, rx, ry, rz);
        });
    }
    s_red[0][tid] = dq;
    s_red[1][tid] = rx;
    s_red[2][tid] = ry;
    s_red[3][tid] = rz;
    __syncthreads();
    if (act && r == 0) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int j = 0; j < 9; ++j) {
            a0 += s_red[0][tid + j];
            a1 += s_red[1][tid + j];
            a2 += s_red[2][tid + j];
            a3 += s_red[3][tid + j];
        }
        finish(a.sorted_idx[slot], a0, a1, a2, a3);
    }
}

__global__ void k_fill_zero(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_zero(hipStream_t s, void *ptr, int64_t nbytes)
{
    const int64_t n = nbytes / 4;
    if (n <= 0) return hipSuccess;
    launch_k(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t *)ptr, n);
    return hipGetLastError();
}

hipError_t launch_scatter(const LaunchCfg &c, const Workspace &w)
{
    if (c.prec == RBE_FP64)
        launch_k(k_scatter<PartD>, c.n_part_tiles, 256, 0, c.stream, w.sys, w.part_tiles, w.cell_start, w.cellid, w.rank,
                                                               (const PartD *)w.packed, w.sorted_idx,
                                                               (PartD *)w.sorted);
    else
        launch_k(k_scatter<PackF>, c.n_part_tiles, 256, 0, c.stream, w.sys, w.part_tiles, w.cell_start, w.cellid, w.rank,
                                                               (const PackF *)w.packed, w.sorted_idx,
                                                               (PackF *)w.sorted);
    return hipGetLastError();
}

template <typename T>
static RealArgs<T> real_args(const LaunchCfg &c, const Workspace &w, void *force, int accumulate, void *vel,
                             const void *q, uint64_t kick_step = 0)
{
    RealArgs<T> a;
    a.kick_step = kick_step;
    a.sys = w.sys;
    a.tiles = w.real_tiles;
    a.start = w.cell_start;
    a.sorted_idx = w.sorted_idx;
    a.sorted = w.sorted;
    a.packed = w.packed;
    a.q = (const T *)q;
    a.ntot = c.ntot;
    a.F = (T *)force;
    a.accumulate = accumulate;
    a.vel = (T *)vel;
    a.flag = w.flag;
    a.epart = w.energy_part;
    a.km = w.kmode;
    a.diam = w.diam;
    return a;
}

hipError_t launch_real(const LaunchCfg &c, const Workspace &w, void *force, int accumulate, void *vel_kick,
                       uint64_t kick_step)
{
    // the per-particle-diameter LJ only in launches that need it: it costs
    // the others registers (and with them resident blocks)
    const bool diam = w.diam != nullptr;
    if (c.prec == RBE_FP64)
        launch_k(diam ? k_real_rows<double, false, true> : k_real_rows<double, false, false>, c.n_real_tiles, RL_BS, 0,
                 c.stream, real_args<double>(c, w, force, accumulate, vel_kick, nullptr, kick_step));
    else
        launch_k(diam ? k_real_rows<float, false, true> : k_real_rows<float, false, false>, c.n_real_tiles, RL_BS, 0,
                 c.stream, real_args<float>(c, w, force, accumulate, vel_kick, nullptr, kick_step));
    return hipGetLastError();
}

template <typename T, int LPP>
static void real_step_launch(const LaunchCfg &c, const RealArgs<T> &a, const ListArgs &la)
{
    const int nb = la.n_rows > la.n_list ? la.n_rows : la.n_list;
    if (c.R == 1) {
        if (a.diam)
            launch_k(k_real_step<T, LPP, true, true>, nb, RL_BS, 0, c.stream, a, la);
        else
            launch_k(k_real_step<T, LPP, false, true>, nb, RL_BS, 0, c.stream, a, la);
    } else {
        if (a.diam)
            launch_k(k_real_step<T, LPP, true, false>, nb, RL_BS, 0, c.stream, a, la);
        else
            launch_k(k_real_step<T, LPP, false, false>, nb, RL_BS, 0, c.stream, a, la);
    }
}

template <typename T>
static void real_step_dispatch(const LaunchCfg &c, const RealArgs<T> &a, const ListArgs &la)
{
    switch (c.real_split) {
    case 1:
        real_step_launch<T, 1>(c, a, la);
        break;
    case 2:
        real_step_launch<T, 2>(c, a, la);
        break;
    case 8:
        real_step_launch<T, 8>(c, a, la);
        break;
    default:
        real_step_launch<T, 4>(c, a, la);
        break;
    }
}

hipError_t launch_real_step(const LaunchCfg &c, const Workspace &w, const ListStep &ls, void *force, void *vel_kick,
                            uint64_t kick_step)
{
    ListArgs la;
    la.ls = ls;
    la.list_tiles = w.list_tiles;
    la.n_rows = c.n_real_tiles;
    la.n_list = c.n_list_tiles;
    la.nbr = w.nbr;
    la.nnb = w.nnb;
    la.kmax = c.kmax;
    la.count = w.cell_count;
    la.ncell_tot = c.ncell_tot;
    la.single_n = c.R == 1 ? (int)c.ntot : 0;
    la.single_p = c.R == 1 ? c.max_p : 0;
    if (c.prec == RBE_FP64)
        real_step_dispatch<double>(c, real_args<double>(c, w, force, 0, vel_kick, nullptr, kick_step), la);
    else
        real_step_dispatch<float>(c, real_args<float>(c, w, force, 0, vel_kick, nullptr, kick_step), la);
    return hipGetLastError();
}

hipError_t launch_energy(const LaunchCfg &c, const Workspace &w, const void *q, const void *vel)
{
    const bool diam = w.diam != nullptr;
    if (c.prec == RBE_FP64)
        launch_k(diam ? k_real_rows<double, true, true> : k_real_rows<double, true, false>, c.n_real_tiles, RL_BS, 0,
                 c.stream, real_args<double>(c, w, nullptr, 0, (void *)vel, q));
    else
        launch_k(diam ? k_real_rows<float, true, true> : k_real_rows<float, true, false>, c.n_real_tiles, RL_BS, 0,
                 c.stream, real_args<float>(c, w, nullptr, 0, (void *)vel, q));
    return hipGetLastError();
}

hipError_t launch_vjp_real(const LaunchCfg &c, const Workspace &w, const void *gF, void *gpos, void *gq,
                           int accumulate)
{
    if (c.prec == RBE_FP64)
        launch_k(k_vjp_real<double>, c.n_real_tiles, RL_BS, 0, c.stream, real_args<double>(c, w, nullptr, 0, nullptr,
                                                                                     nullptr),
                                                                   (const double *)gF, (double *)gpos,
                                                                   (double *)gq, accumulate);
    else
        launch_k(k_vjp_real<float>, c.n_real_tiles, RL_BS, 0, c.stream, real_args<float>(c, w, nullptr, 0, nullptr,
                                                                                   nullptr),
                                                                  (const float *)gF, (float *)gpos, (float *)gq,
                                                                  accumulate);
    return hipGetLastError();
}

}  // namespace rbe
