// rbe_analysis.hip -- analysis kernels that are not part of a time step.
//
// Pair-distance counts by charge class (Sec. 4.1: the pair correlations
// g_++ and g_+- of the charge-charge correlation rho(r) = g_++ - g_+-).
// One block per 256-particle tile of a system in original order; every
// thread owns one particle i and visits the partners j > i of its system,
// which the block stages through LDS 256 at a time.  Counts go to an LDS
// histogram (32-bit atomics), then once per block to the global int64
// counts.  A pair at distance r < r_max falls in bin floor(r / dr), with r
// the square root of dx^2 + dy^2 + dz^2 of the minimum-image displacement
// in FP64, every operation rounded on its own (contraction into fused
// multiply-adds is switched off), so that the bin is the one the plain
// definition gives.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "rbe_internal.h"

namespace rbe {

constexpr int kHistTile = 256;

template <typename T>
__global__ __launch_bounds__(kHistTile) void k_pair_hist(const SysDev *__restrict__ sys, const Tile *__restrict__ tiles,
                                                         const T *__restrict__ pos, const T *__restrict__ q,
                                                         int64_t ntot, double r_max, int nbins,
                                                         unsigned long long *__restrict__ counts)
{
#pragma clang fp contract(off)
    extern __shared__ unsigned int hist[];   // [3][nbins]
    __shared__ double sx[kHistTile], sy[kHistTile], sz[kHistTile];
    __shared__ int spos[kHistTile];
    const Tile t = tiles[blockIdx.x];
    const SysDev S = sys[t.sys];
    const int tid = threadIdx.x;
    for (int k = tid; k < 3 * nbins; k += kHistTile) hist[k] = 0u;
    const int il = t.start + tid;
    const bool act = tid < t.count;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    int pi = 0;
    if (act) {
        const int64_t i = S.off + il;
        xi = (double)pos[i];
        yi = (double)pos[ntot + i];
        zi = (double)pos[2 * ntot + i];
        pi = q[i] > (T)0 ? 1 : 0;
    }
    const double L = S.L, dr = r_max / nbins;
    for (int j0 = t.start; j0 < S.n; j0 += kHistTile) {
        __syncthreads();
        if (j0 + tid < S.n) {
            const int64_t j = S.off + j0 + tid;
            sx[tid] = (double)pos[j];
            sy[tid] = (double)pos[ntot + j];
            sz[tid] = (double)pos[2 * ntot + j];
            spos[tid] = q[j] > (T)0 ? 1 : 0;
        }
        __syncthreads();
        const int m = S.n - j0 < kHistTile ? S.n - j0 : kHistTile;
        if (!act) continue;
        for (int u = 0; u < m; ++u) {
            if (j0 + u <= il) continue;
            double dx = sx[u] - xi, dy = sy[u] - yi, dz = sz[u] - zi;
            dx = dx - L * rint(dx / L);
            dy = dy - L * rint(dy / L);
            dz = dz - L * rint(dz / L);
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (!(r < r_max)) continue;
            const int b = (int)floor(r / dr);
            if (b >= nbins) continue;
            const int cls = 2 - (pi + spos[u]);
            atomicAdd(&hist[cls * nbins + b], 1u);
        }
    }
    __syncthreads();
    unsigned long long *out = counts + (int64_t)t.sys * 3 * nbins;
    for (int k = tid; k < 3 * nbins; k += kHistTile)
        if (hist[k]) atomicAdd(&out[k], (unsigned long long)hist[k]);
}

hipError_t launch_pair_hist(const LaunchCfg &c, const Workspace &w, const void *pos, const void *q, double r_max,
                            int nbins, int64_t *counts)
{
    const size_t sm = sizeof(unsigned int) * 3 * (size_t)nbins;
    if (c.prec == RBE_FP64)
        launch_k(k_pair_hist<double>, c.n_part_tiles, kHistTile, sm, c.stream, 
            w.sys, w.part_tiles, (const double *)pos, (const double *)q, c.ntot, r_max, nbins,
            reinterpret_cast<unsigned long long *>(counts));
    else
        launch_k(k_pair_hist<float>, c.n_part_tiles, kHistTile, sm, c.stream, 
            w.sys, w.part_tiles, (const float *)pos, (const float *)q, c.ntot, r_max, nbins,
            reinterpret_cast<unsigned long long *>(counts));
    return hipGetLastError();
}

}  // namespace rbe
