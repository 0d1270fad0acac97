// rbe_device.h -- device helpers shared by the kernels of librbe.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbe_internal.h"

namespace rbe {

// ---------------------------------------------------------------------------
// Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror & Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
// 32x32 -> 64-bit products with multipliers 0xD2511F53 and 0xCD9E8D57, a word
// permutation, and a Weyl key schedule (0x9E3779B9, 0xBB67AE85).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
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

// Counter (idx, word1, step low, step high) under key `seed`.
__device__ __forceinline__ U4 draw(uint32_t idx, uint32_t word1, uint64_t seed, uint64_t step)
{
    U4 c{idx, word1, (uint32_t)step, (uint32_t)(step >> 32)};
    return philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 53-bit uniform in [0,1): 27 high bits of a, 26 of b.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Three standard normals for particle i at step: Box-Muller on
// u1 = (w0 + 1) 2^-32, u2 = w1 2^-32 (two normals) and on (w2 + 1) 2^-32,
// w3 2^-32 (cosine branch), in double.
// Component d of those normals.
__device__ __forceinline__ double normal_comp(uint32_t i, uint64_t seed, uint64_t step, int d)
{
    const U4 r = draw(i, kTagLangevin, seed, step);
    const double k = 1.0 / 4294967296.0;
    if (d < 2) {
        const double u1 = ((double)r.x + 1.0) * k, u2 = (double)r.y * k;
        const double a = sqrt(-2.0 * log(u1));
        double s, c;
        sincospi(2.0 * u2, &s, &c);
        return d == 0 ? a * c : a * s;
    }
    const double u3 = ((double)r.z + 1.0) * k, u4 = (double)r.w * k;
    const double b = sqrt(-2.0 * log(u3));
    return b * cospi(2.0 * u4);
}

// The same normals in single precision (hardware log2, sqrt and sine/cosine
// of revolutions), for single-precision systems: relative error ~1e-7.
__device__ __forceinline__ float normal_comp_f32(uint32_t i, uint64_t seed, uint64_t step, int d)
{
    const U4 r = draw(i, kTagLangevin, seed, step);
    const float k = 1.0f / 4294967296.0f;
    const uint32_t wa = d < 2 ? r.x : r.z, wb = d < 2 ? r.y : r.w;
    const float u1 = ((float)wa + 1.0f) * k, u2 = (float)wb * k;
    const float a = __builtin_amdgcn_sqrtf(-2.0f * 0.693147180559945309f * __builtin_amdgcn_logf(u1));
    return d == 1 ? a * __builtin_amdgcn_sinf(u2) : a * __builtin_amdgcn_cosf(u2);
}

template <typename T>
__device__ __forceinline__ double normal_t(uint32_t i, uint64_t seed, uint64_t step, int d)
{
    if constexpr (sizeof(T) == 4)
        return (double)normal_comp_f32(i, seed, step, d);
    else
        return normal_comp(i, seed, step, d);
}

// All three components of normal_t at once, from one draw and in
// straight-line code (the same operations per component).
template <typename T>
__device__ __forceinline__ void normal3_t(uint32_t i, uint64_t seed, uint64_t step, double xi[3])
{
    const U4 r = draw(i, kTagLangevin, seed, step);
    if constexpr (sizeof(T) == 4) {
        const float k = 1.0f / 4294967296.0f;
        const float u1 = ((float)r.x + 1.0f) * k, u2 = (float)r.y * k;
        const float u3 = ((float)r.z + 1.0f) * k, u4 = (float)r.w * k;
        const float a = __builtin_amdgcn_sqrtf(-2.0f * 0.693147180559945309f * __builtin_amdgcn_logf(u1));
        const float b = __builtin_amdgcn_sqrtf(-2.0f * 0.693147180559945309f * __builtin_amdgcn_logf(u3));
        xi[0] = (double)(a * __builtin_amdgcn_cosf(u2));
        xi[1] = (double)(a * __builtin_amdgcn_sinf(u2));
        xi[2] = (double)(b * __builtin_amdgcn_cosf(u4));
    } else {
        const double k = 1.0 / 4294967296.0;
        const double u1 = ((double)r.x + 1.0) * k, u2 = (double)r.y * k;
        const double a = sqrt(-2.0 * log(u1));
        double s, c;
        sincospi(2.0 * u2, &s, &c);
        xi[0] = a * c;
        xi[1] = a * s;
        const double u3 = ((double)r.z + 1.0) * k, u4 = (double)r.w * k;
        const double b = sqrt(-2.0 * log(u3));
        xi[2] = b * cospi(2.0 * u4);
    }
}

// For each of three uniforms u, the smallest index k of the cumulative table
// t[0..K) with u < t[k] (the last entry is 1 and u < 1, so the answer is in
// range), by bisection.  The three bisections advance together, so that
// their table reads are in flight at the same time instead of one after
// another: an interval of n entries needs at most ceil(log2 n) halvings, and
// a finished bisection only rereads its entry.
__device__ __forceinline__ void invert_cdf3(const double *t, int K, const double u[3], int out[3])
{
    int lo[3] = {0, 0, 0}, hi[3] = {K - 1, K - 1, K - 1};
    for (int n = K; n > 1; n = (n + 1) >> 1) {
        double v[3];
        int mid[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            mid[d] = (lo[d] + hi[d]) >> 1;
            v[d] = t[mid[d]];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool below = u[d] < v[d];
            if (lo[d] < hi[d]) {
                hi[d] = below ? mid[d] : hi[d];
                lo[d] = below ? lo[d] : mid[d] + 1;
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) out[d] = lo[d];
}

// One exact draw from the importance distribution (Sec. 3.1, eq. 3.3): each
// component inverts the 1-D cumulative table of eq. (3.4); the zero vector
// is drawn again.  Attempt a of draw l uses counters (l, TAG | 2a, step) and
// (l, TAG | 2a + 1, step).
__device__ __forceinline__ void sample_mode(const double *t, int M, uint32_t l, uint64_t seed, uint64_t step,
                                            int &mx, int &my, int &mz)
{
    const int K = 2 * M + 1;
    mx = my = mz = 0;
    for (uint32_t a = 0; a < (1u << 22); ++a) {
        const U4 r0 = draw(l, kTagSample | (2u * a), seed, step);
        const U4 r1 = draw(l, kTagSample | (2u * a + 1u), seed, step);
        const double u[3] = {u53(r0.x, r0.y), u53(r0.z, r0.w), u53(r1.x, r1.y)};
        int c[3];
        invert_cdf3(t, K, u, c);
        mx = c[0] - M;
        my = c[1] - M;
        mz = c[2] - M;
        if (mx | my | mz) break;
    }
}

// ---------------------------------------------------------------------------
// Phases and trigonometry.  A phase is m.s in revolutions, formed in double
// from integer modes and fractional coordinates, wrapped to [-1/2, 1/2].
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wrap_rev(double ph) { return ph - rint(ph); }

__device__ __forceinline__ double frac01(double x)
{
    const double f = x - floor(x);
    return f >= 1.0 ? 0.0 : f;
}

// Single precision: the hardware sine/cosine take revolutions directly
// (measured absolute error below 1.3e-7 on [-1/2, 1/2]).
__device__ __forceinline__ void sincos_rev(double r, float *s, float *c)
{
    const float rf = (float)r;
    *s = __builtin_amdgcn_sinf(rf);
    *c = __builtin_amdgcn_cosf(rf);
}

__device__ __forceinline__ void sincos_rev(double r, double *s, double *c) { sincospi(2.0 * r, s, c); }

// ---------------------------------------------------------------------------
// Particle records.
// PartD: fractional coordinates (double) and charge, for the Fourier passes
// and the double-precision real space.
// PackF: 32-bit fixed-point fractions of the box u = floor(s 2^32) and the
// charge; the unsigned difference of two records, read as signed, is the
// minimum-image displacement in units of L 2^-32.
// ---------------------------------------------------------------------------
struct alignas(16) PartD {
    double x, y, z, q;
};

struct alignas(16) PackF {
    uint32_t x, y, z;
    float q;
};

// Non-finite or negative input maps to 0, so that a non-finite position can
// never index outside the cell arrays (the force kernels flag it instead).
__device__ __forceinline__ uint32_t to_fix(double s)
{
    const double v = s * 4294967296.0;
    if (!(v >= 0.0)) return 0u;
    return v >= 4294967295.0 ? 4294967295u : (uint32_t)v;
}

__device__ __forceinline__ int cell_of_fix(uint32_t u, int nc) { return (int)(((uint64_t)u * (uint64_t)nc) >> 32); }

__device__ __forceinline__ int cell_of_frac(double s, int nc)
{
    if (!(s >= 0.0)) return 0;
    const int c = s < 1.0 ? (int)(s * nc) : nc - 1;
    return c >= nc ? nc - 1 : c;
}

// ---------------------------------------------------------------------------
// Single-precision phases without loss: a box fraction s in [0, 1) is split
// as s = hi + lo with hi a multiple of 2^-b (b = SysDev::hi_bits) and
// 0 <= lo < 2^-b.  For integer modes with |m| < 2^(22-b) the three products
// m_d hi_d and their sum are exact in float, so frac(m . hi) is exact; m . lo
// is small and carries only float rounding.  The phase in revolutions is
// frac(m . hi) + m . lo (range (-0.01, 1.01) at most, fine for the hardware
// sine, which takes revolutions).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split_frac(double s, const SysDev &S, float &hi, float &lo)
{
    const double h = floor(s * (double)S.hi_scale) * (double)S.hi_inv;
    hi = (float)h;
    lo = (float)(s - h);
}

__device__ __forceinline__ void split_fix(uint32_t u, const SysDev &S, float &hi, float &lo)
{
    const int sh = 32 - S.hi_bits;
    hi = (float)(u >> sh) * S.hi_inv;
    lo = (float)(u & ((1u << sh) - 1u)) * (1.0f / 4294967296.0f);
}

__device__ __forceinline__ float phase_split(float mx, float my, float mz, float hx, float hy, float hz, float lx,
                                             float ly, float lz)
{
    const float hi = fmaf(mx, hx, fmaf(my, hy, mz * hz));
    const float lo = fmaf(mx, lx, fmaf(my, ly, mz * lz));
    return __builtin_amdgcn_fractf(hi) + lo;
}

// Fourier force of the modes [l0, l1) of one system on one particle, summed
// in mode order (eq. 3.6 without the factor -q_i).  kk is wave-uniform.
// Mode constants are the same for every lane and do not change while a force
// launch runs: read them through the constant address space from a
// wave-uniform pointer, so that they arrive by scalar loads (one per wave)
// instead of a 64-lane vector load of the same bytes.
template <typename KM>
__device__ __forceinline__ const __attribute__((address_space(4))) KM *uniform_modes(const KM *kk)
{
    const uint64_t p = (uint64_t)kk;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    return (const __attribute__((address_space(4))) KM *)(((uint64_t)hi << 32) | lo);
}

template <typename KM>
__device__ __forceinline__ KM load_mode(const __attribute__((address_space(4))) KM *kk, int l)
{
    KM k;
    for (int d = 0; d < 3; ++d) {
        k.m[d] = kk[l].m[d];
        k.a[d] = kk[l].a[d];
    }
    k.C = kk[l].C;
    k.S = kk[l].S;
    return k;
}

__device__ __forceinline__ void fourier_range(const KModeF *kk0, int l0, int l1, const float h[3], const float lo[3],
                                              float f[3])
{
    const auto kk = uniform_modes(kk0);
    l0 = __builtin_amdgcn_readfirstlane(l0);
    l1 = __builtin_amdgcn_readfirstlane(l1);
#pragma unroll 4
    for (int l = l0; l < l1; ++l) {
        const KModeF k = load_mode(kk, l);
        const float rf = phase_split(k.m[0], k.m[1], k.m[2], h[0], h[1], h[2], lo[0], lo[1], lo[2]);
        const float sn = __builtin_amdgcn_sinf(rf), cs = __builtin_amdgcn_cosf(rf);
        const float im = cs * k.S - sn * k.C;
        f[0] = fmaf(im, k.a[0], f[0]);
        f[1] = fmaf(im, k.a[1], f[1]);
        f[2] = fmaf(im, k.a[2], f[2]);
    }
}

__device__ __forceinline__ void fourier_range(const KModeD *kk0, int l0, int l1, const double s[3], double f[3])
{
    const auto kk = uniform_modes(kk0);
    l0 = __builtin_amdgcn_readfirstlane(l0);
    l1 = __builtin_amdgcn_readfirstlane(l1);
#pragma unroll 2
    for (int l = l0; l < l1; ++l) {
        const KModeD k = load_mode(kk, l);
        const double ph = wrap_rev(fma(k.m[0], s[0], fma(k.m[1], s[1], k.m[2] * s[2])));
        double sn, cs;
        sincospi(2.0 * ph, &sn, &cs);
        const double im = cs * k.S - sn * k.C;
        f[0] = fma(im, k.a[0], f[0]);
        f[1] = fma(im, k.a[1], f[1]);
        f[2] = fma(im, k.a[2], f[2]);
    }
}

// ---------------------------------------------------------------------------
// One particle's position/velocity update up to the force evaluation, in
// double from the stored values: BAOA of the BAOAB Langevin step (half kick,
// half drift, exact Ornstein-Uhlenbeck velocity update with the normals of
// (particle il, step), half drift), or the leapfrog + Andersen update; the
// position is wrapped into [0, L).  x receives the new position.
// ---------------------------------------------------------------------------
// Component d of that update; xi is the component's normal (Langevin) or,
// for Andersen, the normal used when the particle collides (`hit`).
// Workgroups are dispatched round-robin over the 8 XCDs of the chip (each
// with its own L2).  For a grid of n tiles laid out in space order, block b
// (b < n) takes tile xcd_tile(b, n): XCD x = b mod 8 gets the x-th contiguous
// eighth of the tiles, so spatial neighbours share an L2.  A bijection of
// [0, n) for any n.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + k;
}

// Time step of the integrator step with index n: the fixed dt, or the
// annealed burn-in schedule anneal / ln(1 + n) (Sec. 4.2, Example 2; n is
// taken as at least 1).
__device__ __forceinline__ double step_dt(const SysDev &S, uint64_t n)
{
    if (S.anneal <= 0.0) return S.dt;
    return S.anneal / log1p(n < 1 ? 1.0 : (double)n);
}

template <typename T>
__device__ __forceinline__ void integrate_comp(const SysDev &S, T p0, T v0, T f, double xi, bool hit, bool kick,
                                               double dt, double dt_prev, double c1, double c2, T &p1, T &v1)
{
    if (S.integrator == RBE_LANGEVIN_BAOAB) {
        const double h = 0.5 * dt;
        // the previous step's closing half kick, rounded to T as if it had
        // been stored by the force pass
        if (kick) v0 = (T)fma(0.5 * dt_prev / S.mass, (double)f, (double)v0);
        double v = (double)v0 + h * (double)f / S.mass;         // B
        double r = (double)p0 + h * v;                          // A
        v = c1 * v + c2 * xi;                                   // O
        r += h * v;                                             // A
        r -= S.L * floor(r * S.invL);
        T rs = (T)r;
        if (rs >= (T)S.L || rs < (T)0) rs = (T)0;
        p1 = rs;
        v1 = (T)v;
        return;
    }
    const double sv = sqrt(S.kT / S.mass);
    const double v = (double)v0 + dt * (double)f / S.mass;
    double r = (double)p0 + dt * v;
    r -= S.L * floor(r * S.invL);
    T rs = (T)r;
    if (rs >= (T)S.L || rs < (T)0) rs = (T)0;
    p1 = rs;
    v1 = (T)(hit ? sv * xi : v);
}

// Andersen collision of particle il at step.
__device__ __forceinline__ bool andersen_hit(const SysDev &S, int il, uint64_t step)
{
    const U4 w = draw((uint32_t)il, kTagAndersen, S.seed, step);
    return (double)w.x * (1.0 / 4294967296.0) < (S.anneal > 0.0 ? S.nu * step_dt(S, step) : S.nu_dt);
}

template <typename T>
__device__ __forceinline__ void integrate_one(const SysDev &S, int il, int64_t i, int64_t ntot, T *pos, T *vel,
                                              const T *F, uint64_t step, bool kick, double x[3])
{
    // all nine loads first, before the branches on the system constants (so
    // they do not wait for them), and since the stores of one component
    // cannot be proven apart from the loads of the next
    T p0[3], v0[3], f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p0[d] = pos[d * ntot + i];
        v0[d] = vel[d * ntot + i];
        f[d] = F[d * ntot + i];
    }
    if (il < S.n_fixed) {
        // an immobile particle (the colloid of Sec. 4.2): no kick, drift,
        // noise or collision; its stored state is left as it is
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] = (double)p0[d];
        return;
    }
    const bool hit = S.integrator == RBE_LANGEVIN_BAOAB ? false : andersen_hit(S, il, step);
    const bool noise = S.integrator == RBE_LANGEVIN_BAOAB || hit;
    const double dt = step_dt(S, step), dt_prev = kick ? step_dt(S, step - 1) : 0.0;
    double c1 = S.c1, c2 = S.c2;
    if (S.anneal > 0.0 && S.integrator == RBE_LANGEVIN_BAOAB) {
        c1 = exp(-S.gamma * dt / S.mass);
        c2 = sqrt((1.0 - c1 * c1) * S.kT / S.mass);
    }
    // the three normals come from one draw outside the component loop, so
    // that the loop unrolls and its arrays stay in registers
    double xi[3] = {0.0, 0.0, 0.0};
    if (noise) normal3_t<T>((uint32_t)il, S.seed, step, xi);
    T p1[3], v1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        integrate_comp<T>(S, p0[d], v0[d], f[d], xi[d], hit, kick, dt, dt_prev, c1, c2, p1[d], v1[d]);
        x[d] = (double)p1[d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pos[d * ntot + i] = p1[d];
        vel[d * ntot + i] = v1[d];
    }
}

// What the displacement test of a list system needs besides the new
// position: the particle's cell-order slot and its record at the last list
// build (kept as plain words).  Neither depends on the integration, so the
// caller loads them before it and their latency overlaps the integrator's.
struct ListRef {
    int32_t slot;
    uint32_t w[8];   // the record's words (PackF: 4, PartD: 8)
};

template <typename T>
__device__ __forceinline__ void load_list_ref(const SysDev &S, int64_t i, const int32_t *slot_of, const void *ref,
                                              ListRef &r)
{
    r.slot = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r.w[k] = 0;
    if (S.use_list) {
        r.slot = slot_of[i];
        if constexpr (sizeof(T) == 4) {
            const uint4 v = reinterpret_cast<const uint4 *>(ref)[i];
            r.w[0] = v.x;
            r.w[1] = v.y;
            r.w[2] = v.z;
            r.w[3] = v.w;
        } else {
            const uint4 *p = reinterpret_cast<const uint4 *>(ref) + 2 * i;
            const uint4 a = p[0], b = p[1];
            r.w[0] = a.x;
            r.w[1] = a.y;
            r.w[2] = a.z;
            r.w[3] = a.w;
            r.w[4] = b.x;
            r.w[5] = b.y;
            r.w[6] = b.z;
            r.w[7] = b.w;
        }
    }
}

// Stored record of a particle (original order, and cell order for list
// systems) and the displacement test against skin/2 since the last build.
template <typename T>
__device__ __forceinline__ bool record_update(const SysDev &S, int64_t i, double sx, double sy, double sz, T qi,
                                              void *packed, void *sorted, const ListRef &lr)
{
    bool moved = false;
    if constexpr (sizeof(T) == 4) {
        const PackF v{to_fix(sx), to_fix(sy), to_fix(sz), (float)qi};
        reinterpret_cast<PackF *>(packed)[i] = v;
        if (S.use_list) {
            reinterpret_cast<PackF *>(sorted)[lr.slot] = v;
            const uint32_t rx = lr.w[0], ry = lr.w[1], rz = lr.w[2];
            const double u = 1.0 / 4294967296.0 * S.L;
            const double dx = (double)(int32_t)(v.x - rx) * u;
            const double dy = (double)(int32_t)(v.y - ry) * u;
            const double dz = (double)(int32_t)(v.z - rz) * u;
            moved = dx * dx + dy * dy + dz * dz > S.half_skin2;
        }
    } else {
        const PartD v{sx, sy, sz, (double)qi};
        reinterpret_cast<PartD *>(packed)[i] = v;
        if (S.use_list) {
            reinterpret_cast<PartD *>(sorted)[lr.slot] = v;
            auto word2 = [&](int k) { return __hiloint2double((int)lr.w[k + 1], (int)lr.w[k]); };
            double dx = v.x - word2(0), dy = v.y - word2(2), dz = v.z - word2(4);
            dx = (dx - rint(dx)) * S.L;
            dy = (dy - rint(dy)) * S.L;
            dz = (dz - rint(dz)) * S.L;
            moved = dx * dx + dy * dy + dz * dz > S.half_skin2;
        }
    }
    return moved;
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

}  // namespace rbe
