// rbe_api.cpp -- host side of librbe: validation, context and workspace
// management, and the C-ABI entry points declared in include/rbe.h.
//
// Paper: Jin, Li, Xu & Zhao, arXiv:2010.01559.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rbe.h"
#include "rbe_internal.h"

using namespace rbe;

namespace rbe {
LaunchEvents &launch_events()
{
    thread_local LaunchEvents e;
    return e;
}
}  // namespace rbe

namespace {

// Message of the last failed call that has no context (creation, or the
// no-allocation entry point), in a fixed buffer so that setting it from the
// no-allocation path allocates nothing.
struct NullError {
    char buf[512] = "no error";
    NullError &operator=(const std::string &m) { return *this = m.c_str(); }
    NullError &operator=(const char *m)
    {
        std::snprintf(buf, sizeof buf, "%s", m);
        return *this;
    }
    const char *c_str() const { return buf; }
};
thread_local NullError g_create_error;

void null_errf(const char *f, ...)
{
    va_list ap;
    va_start(ap, f);
    std::vsnprintf(g_create_error.buf, sizeof g_create_error.buf, f, ap);
    va_end(ap);
}

const char *kKernelNames[K_COUNT] = {"sample", "stage",      "mid",        "kforce",   "scatter", "real",
                                     "energy", "vjp_reduce", "vjp_gather", "vjp_real", "misc"};

std::string fmt(const char *f, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

// 1-D factor of the normaliser (Sec. 3.1, eq. 3.2, direct form).
double normaliser_H(double alpha, double L)
{
    const double a = kPi * kPi / (alpha * L * L);
    double h = 1.0;
    for (long m = 1; m < 100000000L; ++m) {
        const double t = std::exp(-a * (double)m * (double)m);
        if (t == 0.0 || t < h * 1e-20) break;
        h += 2.0 * t;
    }
    return h;
}

// Half-width M of the 1-D mode table: the continuous Gaussian of eq. (3.4)
// has standard deviation sqrt(alpha L^2/(2 pi^2)); beyond 10 of them the
// mass is below exp(-50).
int table_half_width(double alpha, double L)
{
    const double sigma = std::sqrt(alpha * L * L / (2.0 * kPi * kPi));
    return (int)std::ceil(10.0 * sigma) + 1;
}

// Cumulative table of the 1-D weights exp(-pi^2 m^2/(alpha L^2)) for
// m = -M..M: running sums from m = -M upwards over the total.
void build_cdf(double alpha, double L, std::vector<double> &out)
{
    const int M = table_half_width(alpha, L);
    const int K = 2 * M + 1;
    const double a = kPi * kPi / (alpha * L * L);
    std::vector<double> w(K);
    for (int k = 0; k < K; ++k) {
        const double m = (double)(k - M);
        w[k] = std::exp(-a * m * m);
    }
    double tot = 0.0;
    for (int k = 0; k < K; ++k) tot += w[k];
    double run = 0.0;
    for (int k = 0; k < K; ++k) {
        run += w[k];
        out.push_back(run / tot);
    }
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// The constants of one system that the Fourier passes read: sizes, box,
// splitting, normaliser S = H^3 - 1 (eqs. 3.1-3.2), the mode table bound and
// the single-precision phase split (|m| <= 2M must satisfy |m| < 2^(22 - hi_bits)).
void fourier_constants(const rbe_params &p, SysDev &s)
{
    s.n = p.n;
    s.p = p.p;
    s.M = table_half_width(p.alpha, p.box);
    s.L = p.box;
    s.invL = 1.0 / p.box;
    s.alpha = p.alpha;
    s.beta = std::sqrt(p.alpha);
    s.coulomb = p.coulomb;
    const double H = normaliser_H(p.alpha, p.box);
    s.S = H * H * H - 1.0;
    int bm = 0;
    while ((1 << bm) <= 2 * s.M) ++bm;
    s.hi_bits = std::min(14, 22 - bm);
    s.hi_scale = std::ldexp(1.0f, s.hi_bits);
    s.hi_inv = std::ldexp(1.0f, -s.hi_bits);
}

// Default tile shapes for ntot particles: one structure-factor block per
// compute unit when the particles allow (the block's registers leave room
// for one 1024-thread block per CU); four waves share a 64-particle tile in
// the force pass while the tiles alone would not fill the chip several
// times over, two beyond.
int default_rho_chunk(int64_t ntot)
{
    return (int)std::min<int64_t>(512, std::max<int64_t>(64, ((ntot + 255) / 256 + 7) / 8 * 8));
}

int default_force_split(int64_t ntot) { return ntot >= 500000 ? 2 : 4; }

// ---------------------------------------------------------------------------
// Tile cache: shapes picked by rbe_autotune, keyed by device architecture,
// precision, the power-of-two buckets of the total particle count and of the
// largest batch size, and whether the context holds several systems.  It is
// read at the first context creation from $RBE_TUNE_CACHE, or else from
// rbe_tiles.txt beside the library, and consulted by every creation;
// rbe_autotune adds its result and appends it to the file when it can.
// Lines: "arch precision n_bucket p_bucket batched rho_chunk rho_block
// force_split real_split"; '#' starts a comment.
// ---------------------------------------------------------------------------
struct TuneKey {
    std::string arch;
    int prec, nb, pb, batched;
    bool operator<(const TuneKey &o) const
    {
        if (arch != o.arch) return arch < o.arch;
        if (prec != o.prec) return prec < o.prec;
        if (nb != o.nb) return nb < o.nb;
        if (pb != o.pb) return pb < o.pb;
        return batched < o.batched;
    }
};

struct TuneCache {
    std::mutex mu;
    bool loaded = false;
    bool persist = false;   // rbe_autotune appends to the file (only one named by RBE_TUNE_CACHE)
    std::string path;
    std::map<TuneKey, rbe_tiles> m;
};

TuneCache &tune_cache()
{
    static TuneCache t;
    return t;
}

int log2_bucket(int64_t v)
{
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

// The architecture name without its feature suffixes ("gfx950:sramecc+" -> "gfx950").
TuneKey tune_key(const char *arch, int prec, int64_t ntot, int max_p, int R)
{
    std::string a = arch;
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a.resize(colon);
    return TuneKey{a, prec, log2_bucket(ntot), log2_bucket(max_p), R > 1 ? 1 : 0};
}

void tune_load_locked(TuneCache &t)
{
    if (t.loaded) return;
    t.loaded = true;
    if (const char *env = std::getenv("RBE_TUNE_CACHE")) {
        t.path = env;
        t.persist = true;
    } else {
        Dl_info info;
        if (dladdr((void *)&tune_cache, &info) && info.dli_fname) {
            std::string lib = info.dli_fname;
            const size_t slash = lib.rfind('/');
            t.path = (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/rbe_tiles.txt";
        }
    }
    FILE *f = t.path.empty() ? nullptr : std::fopen(t.path.c_str(), "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (char *hash = std::strchr(line, '#')) *hash = 0;
        char arch[32];
        TuneKey k;
        rbe_tiles v;
        if (std::sscanf(line, "%31s %d %d %d %d %d %d %d %d", arch, &k.prec, &k.nb, &k.pb, &k.batched, &v.rho_chunk,
                        &v.rho_block, &v.force_split, &v.real_split) == 9) {
            k.arch = arch;
            t.m[k] = v;
        }
    }
    std::fclose(f);
}

bool tune_lookup(const TuneKey &k, rbe_tiles *out)
{
    TuneCache &t = tune_cache();
    std::lock_guard<std::mutex> lock(t.mu);
    tune_load_locked(t);
    auto it = t.m.find(k);
    if (it == t.m.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const TuneKey &k, const rbe_tiles &v)
{
    TuneCache &t = tune_cache();
    std::lock_guard<std::mutex> lock(t.mu);
    tune_load_locked(t);
    t.m[k] = v;
    if (!t.persist || t.path.empty()) return;
    if (FILE *f = std::fopen(t.path.c_str(), "a")) {
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", k.arch.c_str(), k.prec, k.nb, k.pb, k.batched, v.rho_chunk,
                     v.rho_block, v.force_split, v.real_split);
        std::fclose(f);
    }
}

// Whether a tile shape fits the kernels' dynamic LDS: the adjoint
// reduction stages 48 bytes per particle and 16 per thread, the staging
// kernel 32 per particle (plus 256 padding records) and 28 per thread (its
// table falls back to global memory when it does not fit).
bool tiles_fit(const rbe_tiles &n)
{
    return n.rho_chunk >= 64 && n.rho_chunk <= 2048 && n.rho_chunk % 8 == 0 &&
           (n.rho_block == 256 || n.rho_block == 512 || n.rho_block == 1024) &&
           (n.force_split == 1 || n.force_split == 2 || n.force_split == 4) &&
           (n.real_split == 1 || n.real_split == 2 || n.real_split == 4 || n.real_split == 8) &&
           48 * (size_t)n.rho_chunk + 16 * (size_t)n.rho_block <= 64 * 1024 &&
           32 * ((size_t)n.rho_chunk + 256) + 28 * (size_t)n.rho_block <= 64 * 1024;
}

// Largest centre distance at which the shifted LJ of eq. (4.1) still acts:
// R_c without diameters (r_off = 0), else r_off + R_c of the pair of the two
// largest diameters, r_off = (d_i + d_j)/2 - sigma.
double lj_reach(const rbe_params &p)
{
    if (!p.diameter || p.n < 2) return p.lj_rcut;
    double d1 = -1e300, d2 = -1e300;
    for (int i = 0; i < p.n; ++i) {
        const double d = p.diameter[i];
        if (d > d1) {
            d2 = d1;
            d1 = d;
        } else if (d > d2) {
            d2 = d;
        }
    }
    return 0.5 * (d1 + d2) - p.lj_sigma + p.lj_rcut;
}

rbe_status validate(const rbe_params &p, std::string &err)
{
    if (p.n < 1) return err = fmt("n must be >= 1 (got %d)", p.n), RBE_ERR_INVALID;
    if (p.p < 1) return err = fmt("p must be >= 1 (got %d)", p.p), RBE_ERR_INVALID;
    if (!finite_pos(p.box)) return err = "box must be finite and > 0", RBE_ERR_INVALID;
    if (!finite_pos(p.alpha)) return err = "alpha must be finite and > 0", RBE_ERR_INVALID;
    if (!finite_pos(p.r_cut)) return err = "r_cut must be finite and > 0", RBE_ERR_INVALID;
    if (!std::isfinite(p.coulomb)) return err = "coulomb must be finite", RBE_ERR_INVALID;
    if (p.r_cut > 0.5 * p.box)
        return err = fmt("r_cut %.6g exceeds half the box %.6g (minimum image)", p.r_cut, 0.5 * p.box),
               RBE_ERR_CUTOFF;
    if (!std::isfinite(p.lj_eps) || p.lj_eps < 0.0) return err = "lj_eps must be finite and >= 0", RBE_ERR_INVALID;
    if (p.diameter)
        for (int i = 0; i < p.n; ++i)
            if (!finite_pos(p.diameter[i])) return err = fmt("diameter[%d] must be finite and > 0", i), RBE_ERR_INVALID;
    if (p.lj_eps > 0.0) {
        if (!finite_pos(p.lj_sigma) || !finite_pos(p.lj_rcut))
            return err = "lj_sigma and lj_rcut must be finite and > 0 when lj_eps > 0", RBE_ERR_INVALID;
        if (lj_reach(p) > 0.5 * p.box)
            return err = fmt("the LJ reach r_off + lj_rcut = %.6g exceeds half the box", lj_reach(p)), RBE_ERR_CUTOFF;
    }
    if (p.n_fixed < 0 || p.n_fixed > p.n) return err = fmt("n_fixed must be in [0, n] (got %d)", p.n_fixed), RBE_ERR_INVALID;
    if (p.reserved != 0) return err = "reserved must be 0", RBE_ERR_INVALID;
    if (!std::isfinite(p.kT) || p.kT < 0.0) return err = "kT must be finite and >= 0", RBE_ERR_INVALID;
    if (!std::isfinite(p.gamma) || p.gamma < 0.0) return err = "gamma must be finite and >= 0", RBE_ERR_INVALID;
    if (!std::isfinite(p.dt) || p.dt < 0.0) return err = "dt must be finite and >= 0", RBE_ERR_INVALID;
    if (!finite_pos(p.mass)) return err = "mass must be finite and > 0", RBE_ERR_INVALID;
    if (!std::isfinite(p.nu) || p.nu < 0.0) return err = "nu must be finite and >= 0", RBE_ERR_INVALID;
    if (!std::isfinite(p.skin) || p.skin < 0.0) return err = "skin must be finite and >= 0", RBE_ERR_INVALID;
    if (p.precision != RBE_FP32 && p.precision != RBE_FP64) return err = "unknown precision", RBE_ERR_INVALID;
    if (p.integrator != RBE_LANGEVIN_BAOAB && p.integrator != RBE_LEAPFROG_ANDERSEN)
        return err = "unknown integrator", RBE_ERR_INVALID;
    if (p.sampler != RBE_SAMPLER_EXACT && p.sampler != RBE_SAMPLER_MH && p.sampler != RBE_SAMPLER_FIXED)
        return err = "unknown sampler", RBE_ERR_INVALID;
    if (p.flags != 0) return err = "flags must be 0", RBE_ERR_INVALID;
    const double H = normaliser_H(p.alpha, p.box);
    if (1.0 / (H * H * H) > 0.5)
        return err = fmt("alpha L^2 = %.3g is too small: the zero mode would carry most of the mass",
                         p.alpha * p.box * p.box),
               RBE_ERR_INVALID;
    if (table_half_width(p.alpha, p.box) > (1 << 20)) return err = "alpha L^2 too large for the mode table", RBE_ERR_INVALID;
    if (p.precision == RBE_FP32 && table_half_width(p.alpha, p.box) > 4095)
        return err = fmt("alpha L^2 = %.3g needs modes beyond |m| = 8191, past the single-precision phase "
                         "split; use RBE_FP64", p.alpha * p.box * p.box),
               RBE_ERR_INVALID;
    return RBE_OK;
}

}  // namespace

struct rbe_ctx {
    int R = 0;
    int prec = RBE_FP32;
    int device = 0;
    std::string arch;               // gcnArchName of the device
    bool tiles_from_cache = false;  // creation took its tile shapes from the tile cache
    hipStream_t stream = nullptr;
    std::vector<rbe_params> prm;
    std::vector<SysDev> sysh;
    std::vector<int> ntiles_rho;   // per system
    std::vector<int> real_sys;     // system of each real-space tile
    int64_t ntot = 0;
    int mtot = 0;                  // active modes in total
    int mcap = 0;                  // capacity of the mode arrays
    int max_p = 0;
    bool modes_valid = false;
    bool list_valid = false;       // the neighbour list matches the cell order in `sorted`
    uint64_t list_gen = 0;         // steps taken in list mode (selects the rebuild flag)
    bool any_mh = false;
    bool fixed = false;            // rbe_step keeps the active mode list
    // rbe_sample_k with the exact sampler only records the draw; the next
    // structure-factor launch draws the modes itself (or a sampling launch
    // runs first where that launch cannot)
    bool sample_pending = false;
    uint64_t sample_step = 0;
    // The active modes are the exact sample of step cur_step (cur_drawn), and
    // the totals launch of a force call draws the sample of cur_step + 1 into
    // the alternate mode arrays (next_ready, next_step), so that an
    // rbe_sample_k for that step only swaps the arrays.
    bool cur_drawn = false;
    uint64_t cur_step = 0;
    bool next_ready = false;
    uint64_t next_step = 0;
    LaunchCfg cfg{};
    Workspace w{};
    size_t partial_cap = 0;        // doubles allocated for partial
    std::vector<void *> allocs;
    std::string err = "no error";
    // profiling
    bool prof = false;
    struct Pend {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Pend> pend;
    std::vector<hipEvent_t> pool;
    double prof_ms[K_COUNT] = {};
    int64_t prof_n[K_COUNT] = {};
    // host staging
    std::vector<double> epart_h;
    // graphs of steady-state list steps, keyed by everything their
    // kernel arguments were taken from
    bool graphs = false;
    hipStream_t cap_stream = nullptr;
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        LaunchCfg cfg{};
        Workspace w{};
        const void *pos, *vel, *q, *force;
        int par;
        bool andersen;
        uint64_t used;
    };
    std::vector<StepGraph> step_graphs;
    uint64_t graph_clock = 0;
};

namespace {

rbe_status set_err(rbe_ctx *c, rbe_status st, const std::string &m)
{
    if (c) c->err = m;
    return st;
}

rbe_status hip_fail(rbe_ctx *c, hipError_t e, const char *what)
{
    return set_err(c, RBE_ERR_HIP, fmt("%s: %s", what, hipGetErrorString(e)));
}

#define HIPCHK(ctx, call)                                    \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

template <typename F>
rbe_status run(rbe_ctx *c, int id, F &&f)
{
    if (c->prof) {
        hipEvent_t a, b;
        if (c->pool.size() >= 2) {
            a = c->pool.back();
            c->pool.pop_back();
            b = c->pool.back();
            c->pool.pop_back();
        } else {
            HIPCHK(c, hipEventCreate(&a));
            HIPCHK(c, hipEventCreate(&b));
        }
        // the launches of f record a and b themselves (launch_k)
        LaunchEvents &le = launch_events();
        le = LaunchEvents{a, b, false};
        hipError_t e = f();
        const bool launched = le.started;
        le = LaunchEvents{};
        if (e != hipSuccess) return hip_fail(c, e, kKernelNames[id]);
        if (!launched) {
            c->pool.push_back(a);
            c->pool.push_back(b);
            return RBE_OK;
        }
        c->pend.push_back({id, a, b});
        if (c->pend.size() > 4096) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            for (auto &p : c->pend) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, p.a, p.b);
                c->prof_ms[p.id] += ms;
                c->prof_n[p.id] += 1;
                c->pool.push_back(p.a);
                c->pool.push_back(p.b);
            }
            c->pend.clear();
        }
        return RBE_OK;
    }
    hipError_t e = f();
    if (e != hipSuccess) return hip_fail(c, e, kKernelNames[id]);
    return RBE_OK;
}

#define RUN(ctx, id, expr)                                       \
    do {                                                         \
        rbe_status s_ = run(ctx, id, [&]() { return (expr); }); \
        if (s_ != RBE_OK) return s_;                             \
    } while (0)

template <typename T>
rbe_status dalloc(rbe_ctx *c, T **p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(c, RBE_ERR_OOM, fmt("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e)));
    }
    c->allocs.push_back(q);
    *p = (T *)q;
    return RBE_OK;
}

void drop_graphs(rbe_ctx *c)
{
    for (auto &g : c->step_graphs) (void)hipGraphExecDestroy(g.exec);
    c->step_graphs.clear();
}

void free_all(rbe_ctx *c)
{
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

// Structure-factor tiles for the current chunk size, their partial offsets
// (in (C,S) pairs) and per-system tile counts.
void build_rho_tiles(rbe_ctx *c, std::vector<Tile> &tiles, std::vector<int32_t> &poff, int chunk, int pcap_of_sys0)
{
    tiles.clear();
    poff.assign(2 * c->R, 0);
    c->ntiles_rho.assign(c->R, 0);
    int64_t run = 0;
    for (int r = 0; r < c->R; ++r) {
        const int n = c->sysh[r].n;
        const int nt = (n + chunk - 1) / chunk;
        c->ntiles_rho[r] = nt;
        poff[r] = (int32_t)run;
        poff[c->R + r] = nt;
        for (int k = 0; k < nt; ++k) tiles.push_back(Tile{r, k * chunk, std::min(chunk, n - k * chunk), k});
        const int pc = (c->R == 1) ? pcap_of_sys0 : c->sysh[r].p;
        run += (int64_t)nt * pc;
    }
}

size_t partial_need(rbe_ctx *c, int chunk)
{
    int64_t run = 0;
    for (int r = 0; r < c->R; ++r) {
        const int nt = (c->sysh[r].n + chunk - 1) / chunk;
        const int pc = (c->R == 1) ? c->mcap : c->sysh[r].p;
        run += (int64_t)nt * pc;
    }
    return (size_t)run * 2;
}

// Real-space tiles: runs of RL_PPB cell-sorted slots for systems with at least
// three cells per side (aux = 0), runs of 256 particles in original order for
// the all-pairs systems (aux = 1).
void build_real_tiles(rbe_ctx *c, std::vector<Tile> &out, std::vector<int> &tile_sys)
{
    out.clear();
    tile_sys.clear();
    for (int r = 0; r < c->R; ++r) {
        const SysDev &s = c->sysh[r];
        const int aux = s.nc == 1 ? 1 : 0;
        const int step = aux ? real_allpairs_per_tile() : real_rows_per_tile();
        for (int k = 0; k < s.n; k += step) {
            out.push_back(Tile{r, k, std::min(step, s.n - k), aux});
            tile_sys.push_back(r);
        }
    }
}

// List-pass tiles: runs of 256/LPP cell-sorted slots (aux = 2) for list
// systems, all-pairs runs (aux = 1) for one-cell systems.
void build_list_tiles(rbe_ctx *c, int lpp, std::vector<Tile> &out)
{
    out.clear();
    for (int r = 0; r < c->R; ++r) {
        const SysDev &s = c->sysh[r];
        const int aux = s.nc == 1 ? 1 : 2;
        const int step = aux == 1 ? real_allpairs_per_tile() : 256 / lpp;
        for (int k = 0; k < s.n; k += step) out.push_back(Tile{r, k, std::min(step, s.n - k), aux});
    }
}

rbe_status upload_list_tiles(rbe_ctx *c)
{
    if (!c->cfg.list_on) return RBE_OK;
    std::vector<Tile> lt;
    build_list_tiles(c, c->cfg.real_split, lt);
    c->cfg.n_list_tiles = (int)lt.size();
    HIPCHK(c, hipMemcpy(c->w.list_tiles, lt.data(), lt.size() * sizeof(Tile), hipMemcpyHostToDevice));
    return RBE_OK;
}

rbe_status upload_rho_tiles(rbe_ctx *c)
{
    std::vector<Tile> tiles;
    std::vector<int32_t> poff;
    build_rho_tiles(c, tiles, poff, c->cfg.rho_chunk, c->mcap);
    c->cfg.n_rho_tiles = (int)tiles.size();
    c->cfg.max_sys_rho_tiles = 0;
    for (int nt : c->ntiles_rho) c->cfg.max_sys_rho_tiles = std::max(c->cfg.max_sys_rho_tiles, nt);
    HIPCHK(c, hipMemcpy(c->w.rho_tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->w.partial_off, poff.data(), poff.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return RBE_OK;
}

rbe_status upload_sys(rbe_ctx *c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->w.sys, c->sysh.data(), c->sysh.size() * sizeof(SysDev), hipMemcpyHostToDevice));
    return RBE_OK;
}

void refresh_cfg_modes(rbe_ctx *c)
{
    c->mtot = 0;
    c->max_p = 0;
    for (auto &s : c->sysh) {
        c->mtot += s.p;
        c->max_p = std::max(c->max_p, s.p);
    }
    c->cfg.max_p = c->max_p;
    c->cfg.mcap = c->mcap;
}

bool check_device_ptr(const void *p) { return p != nullptr; }

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

rbe_status rbe_normalizer(double alpha, double box, double *H, double *S)
{
    if (!finite_pos(alpha) || !finite_pos(box) || !H || !S) return RBE_ERR_INVALID;
    const double h = normaliser_H(alpha, box);
    *H = h;
    *S = h * h * h - 1.0;
    return RBE_OK;
}

const char *rbe_last_error(const rbe_ctx *ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

int32_t rbe_num_systems(const rbe_ctx *ctx) { return ctx ? ctx->R : 0; }
int64_t rbe_num_particles(const rbe_ctx *ctx) { return ctx ? ctx->ntot : 0; }
int32_t rbe_num_modes(const rbe_ctx *ctx) { return ctx ? ctx->mtot : 0; }

rbe_status rbe_batch_create(const rbe_params *params, int32_t R, void *stream, rbe_ctx **out)
{
    if (out) *out = nullptr;
    if (!params || !out || R < 1) {
        g_create_error = "params and out must be non-NULL and R >= 1";
        return RBE_ERR_INVALID;
    }
    int64_t ntot = 0;
    for (int r = 0; r < R; ++r) {
        std::string e;
        rbe_status st = validate(params[r], e);
        if (st != RBE_OK) {
            g_create_error = fmt("system %d: %s", r, e.c_str());
            return st;
        }
        if (params[r].precision != params[0].precision) {
            g_create_error = "all systems of a batch must share one precision";
            return RBE_ERR_INVALID;
        }
        ntot += params[r].n;
    }
    if (ntot >= (int64_t)1 << 31) {
        g_create_error = "total particle count must be below 2^31";
        return RBE_ERR_INVALID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        g_create_error = "no HIP device available";
        return RBE_ERR_NO_DEVICE;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        g_create_error = "hipGetDevice failed";
        return RBE_ERR_NO_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess || std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = fmt("device %d is not gfx950 (%s)", dev, prop.gcnArchName);
        return RBE_ERR_NO_DEVICE;
    }

    rbe_ctx *c = new rbe_ctx();
    c->R = R;
    c->prec = params[0].precision;
    c->device = dev;
    c->stream = (hipStream_t)stream;
    c->prm.assign(params, params + R);
    c->ntot = ntot;

    // ---- per-system constants ----
    std::vector<double> cdf;
    int64_t off = 0;
    int moff = 0, cell_off = 0, max_cells = 0, max_table = 0;
    // the neighbour list is used only when every system of the batch asks for it
    bool all_skin = true;
    for (int r = 0; r < R; ++r) all_skin = all_skin && params[r].skin > 0.0;
    int kmax = 0;
    bool any_diam = false;
    for (int r = 0; r < R; ++r) {
        const rbe_params &p = params[r];
        SysDev s{};
        fourier_constants(p, s);
        s.off = (int32_t)off;
        s.moff = moff;
        s.cdf_off = (int32_t)cdf.size();
        build_cdf(p.alpha, p.box, cdf);
        const double rmax = std::max(p.r_cut, p.lj_eps > 0.0 ? lj_reach(p) : 0.0);
        const double rlist = rmax + p.skin;
        int nc = (int)std::floor(p.box / rlist);
        nc = std::min(nc, 128);
        if (nc < 3) nc = 1;   // fewer than 3 cells along the box: one cell, all pairs
        s.nc = nc;
        s.ncell = nc * nc * nc;
        s.cell_off = cell_off;   // kept a multiple of 4 for vector loads of the counts
        s.lj_on = p.lj_eps > 0.0 ? 1 : 0;
        s.integrator = p.integrator;
        s.mh_state_off = 3 * r;
        s.rc2 = p.r_cut * p.r_cut;
        s.lj_eps = p.lj_eps;
        s.lj_sig2 = p.lj_sigma * p.lj_sigma;
        s.lj_rc2 = p.lj_rcut * p.lj_rcut;
        s.lj_sig = p.lj_sigma;
        s.lj_rc = p.lj_rcut;
        s.rsearch2 = rmax * rmax;
        s.n_fixed = p.n_fixed;
        s.diam_on = (p.diameter && s.lj_on) ? 1 : 0;
        any_diam = any_diam || s.diam_on;
        if (s.lj_on) {
            const double sr6 = std::pow(p.lj_sigma / p.lj_rcut, 6.0);
            s.lj_shift = -4.0 * p.lj_eps * (sr6 * sr6 - sr6);
        }
        s.kT = p.kT;
        s.gamma = p.gamma;
        s.dt = p.dt;
        s.mass = p.mass;
        s.c1 = std::exp(-p.gamma * p.dt / p.mass);
        s.c2 = std::sqrt((1.0 - s.c1 * s.c1) * p.kT / p.mass);
        s.nu_dt = p.nu * p.dt;
        s.nu = p.nu;
        s.anneal = 0.0;
        s.seed = p.seed;
        s.use_list = (all_skin && nc >= 3) ? 1 : 0;
        s.rlist2 = rlist * rlist;
        s.half_skin2 = 0.25 * p.skin * p.skin;
        if (s.use_list) {
            const double dens = (double)p.n / (p.box * p.box * p.box);
            const double mean = dens * 4.0 / 3.0 * kPi * rlist * rlist * rlist;
            kmax = std::max(kmax, (int)std::ceil(1.5 * mean + 32.0));
        }
        c->sysh.push_back(s);
        if (p.sampler == RBE_SAMPLER_MH) c->any_mh = true;
        if (p.sampler == RBE_SAMPLER_FIXED) c->fixed = true;
        off += p.n;
        moff += p.p;
        cell_off += (s.ncell + 3) & ~3;
        max_cells = std::max(max_cells, s.ncell);
        max_table = std::max(max_table, 2 * s.M + 1);
    }
    if (c->fixed && R != 1) {
        g_create_error = "the fixed sampler needs a single-system context";
        delete c;
        return RBE_ERR_INVALID;
    }
    c->mcap = moff;
    refresh_cfg_modes(c);

    // ---- launch configuration ----
    LaunchCfg &g = c->cfg;
    g.stream = c->stream;
    g.R = R;
    g.prec = c->prec;
    g.ntot = ntot;
    g.mcap = c->mcap;
    g.rho_chunk = default_rho_chunk(ntot);
    g.rho_block = 1024;
    g.force_split = default_force_split(ntot);
    g.real_split = 4;
    g.kmax = std::min((kmax + 7) & ~7, 1024);
    g.list_on = 0;
    for (int r = 0; r < R; ++r) g.list_on |= c->sysh[r].use_list;
    g.ncell_tot = cell_off;
    g.max_cells = max_cells;
    g.max_p = c->max_p;
    g.max_table = max_table;
    g.wait_limit = kWaitLimit;

    std::vector<Tile> ftiles, ptiles;
    for (int r = 0; r < R; ++r) {
        const int n = c->sysh[r].n;
        for (int k = 0; k < n; k += 64) ftiles.push_back(Tile{r, k, std::min(64, n - k), 0});
        for (int k = 0; k < n; k += 256) ptiles.push_back(Tile{r, k, std::min(256, n - k), 0});
    }
    g.n_force_tiles = (int)ftiles.size();
    g.n_part_tiles = (int)ptiles.size();
    std::vector<Tile> rtiles;
    build_real_tiles(c, rtiles, c->real_sys);
    g.n_real_tiles = (int)rtiles.size();

    // ---- device memory ----
    const size_t esz = c->prec == RBE_FP64 ? 8 : 4;
    const size_t pack_sz = c->prec == RBE_FP64 ? 32 : 16;
    const size_t km_sz = c->prec == RBE_FP64 ? sizeof(KModeD) : sizeof(KModeF);
    const size_t kv_sz = c->prec == RBE_FP64 ? sizeof(KVjpD) : sizeof(KVjpF);
    (void)esz;
    // the largest rho tile list is the one for the smallest chunk (64)
    int64_t max_rho_tiles = 0;
    for (int r = 0; r < R; ++r) max_rho_tiles += (c->sysh[r].n + 63) / 64;
    c->partial_cap = partial_need(c, 64);
    Workspace &w = c->w;
    rbe_status st = RBE_OK;
#define ALLOC(ptr, bytes)                                   \
    do {                                                    \
        if ((st = dalloc(c, &(ptr), (bytes))) != RBE_OK) {  \
            g_create_error = c->err;                        \
            free_all(c);                                    \
            delete c;                                       \
            return st;                                      \
        }                                                   \
    } while (0)
    ALLOC(w.sys, sizeof(SysDev) * R);
    ALLOC(w.rho_tiles, sizeof(Tile) * max_rho_tiles);
    ALLOC(w.force_tiles, sizeof(Tile) * ftiles.size());
    ALLOC(w.part_tiles, sizeof(Tile) * ptiles.size());
    ALLOC(w.real_tiles, sizeof(Tile) * rtiles.size());
    ALLOC(w.modes, sizeof(int32_t) * 3 * c->mcap);
    ALLOC(w.mode_w, sizeof(double) * c->mcap);
    ALLOC(w.partial, sizeof(double) * c->partial_cap);
    ALLOC(w.partial_off, sizeof(int32_t) * 2 * R);
    ALLOC(w.rho, sizeof(double) * 2 * c->mcap);
    ALLOC(w.ab, sizeof(double) * 2 * c->mcap);
    ALLOC(w.kmode, km_sz * c->mcap);
    ALLOC(w.kvjp, kv_sz * c->mcap);
    ALLOC(w.cdf, sizeof(double) * cdf.size());
    ALLOC(w.mh_state, sizeof(int32_t) * 3 * R);
    ALLOC(w.cell_count, sizeof(int32_t) * cell_off);
    ALLOC(w.cell_start, sizeof(int32_t) * (cell_off + R));
    ALLOC(w.cellid, sizeof(int32_t) * ntot);
    ALLOC(w.rank, sizeof(int32_t) * ntot);
    ALLOC(w.sorted_idx, sizeof(int32_t) * ntot);
    ALLOC(w.packed, pack_sz * ntot);
    // one padding record after the last slot: the cell pass's row scan reads
    // candidates two at a time and may read one past a segment's end
    ALLOC(w.sorted, pack_sz * (ntot + 1));
    ALLOC(w.modes_alt, sizeof(int32_t) * 3 * c->mcap);
    ALLOC(w.mode_w_alt, sizeof(double) * c->mcap);
    ALLOC(w.energy_part, sizeof(double) * 8 * rtiles.size());
    ALLOC(w.flag, sizeof(int32_t) * 4);
    ALLOC(w.lflag, sizeof(int32_t) * 8);
    ALLOC(w.step_base, sizeof(uint64_t));
    if (any_diam) ALLOC(w.diam, sizeof(double) * ntot);
    {
        // list-pass tiles: at most one per 32 slots (the 8-lane shape)
        int64_t nl = 0;
        for (int r = 0; r < R; ++r) nl += (c->sysh[r].n + 31) / 32;
        const int64_t nlist = g.list_on ? ntot : 1;
        ALLOC(w.list_tiles, sizeof(Tile) * (g.list_on ? nl : 1));
        ALLOC(w.slot_of, sizeof(int32_t) * nlist);
        ALLOC(w.ref, pack_sz * nlist);
        ALLOC(w.nbr, sizeof(int32_t) * (g.list_on ? (int64_t)g.kmax * ntot : 1));
        ALLOC(w.nnb, sizeof(int32_t) * nlist);
    }
#undef ALLOC
    c->epart_h.resize(8 * rtiles.size());

    auto up = [&](void *dst, const void *src, size_t bytes) -> bool {
        return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = up(w.sys, c->sysh.data(), sizeof(SysDev) * R) &&
              up(w.force_tiles, ftiles.data(), sizeof(Tile) * ftiles.size()) &&
              up(w.part_tiles, ptiles.data(), sizeof(Tile) * ptiles.size()) &&
              up(w.real_tiles, rtiles.data(), sizeof(Tile) * rtiles.size()) &&
              up(w.cdf, cdf.data(), sizeof(double) * cdf.size()) &&
              hipMemset(w.mh_state, 0, sizeof(int32_t) * 3 * R) == hipSuccess &&
              hipMemset(w.cell_count, 0, sizeof(int32_t) * cell_off) == hipSuccess &&
              hipMemset(w.flag, 0, sizeof(int32_t) * 4) == hipSuccess &&
              hipMemset(w.lflag, 0, sizeof(int32_t) * 8) == hipSuccess &&
              hipMemset(w.cell_start, 0, sizeof(int32_t) * (cell_off + R)) == hipSuccess &&
              hipMemset(w.modes, 0, sizeof(int32_t) * 3 * c->mcap) == hipSuccess;
    if (ok) {
        // every slot names a particle of its own system until the first scatter
        std::vector<int32_t> iota(ntot);
        for (int64_t i = 0; i < ntot; ++i) iota[i] = (int32_t)i;
        ok = up(w.sorted_idx, iota.data(), sizeof(int32_t) * ntot);
    }
    if (ok && any_diam) {
        std::vector<double> d(ntot);
        for (int r = 0; r < R; ++r) {
            const rbe_params &p = params[r];
            for (int i = 0; i < p.n; ++i) d[c->sysh[r].off + i] = p.diameter ? p.diameter[i] : p.lj_sigma;
        }
        ok = up(w.diam, d.data(), sizeof(double) * ntot);
    }
    {
        // shapes from the tile cache, when it holds this configuration
        rbe_tiles t;
        c->arch = prop.gcnArchName;
        if (tune_lookup(tune_key(prop.gcnArchName, c->prec, ntot, c->max_p, R), &t) && tiles_fit(t)) {
            g.rho_chunk = t.rho_chunk;
            g.rho_block = t.rho_block;
            g.force_split = t.force_split;
            g.real_split = t.real_split;
            c->tiles_from_cache = true;
        }
    }
    if (ok) ok = upload_rho_tiles(c) == RBE_OK;
    if (ok) ok = upload_list_tiles(c) == RBE_OK;
    if (ok && g.list_on) {
        // in-bounds slots and zeroed records until the first build replaces them
        std::vector<int32_t> iota(ntot);
        for (int64_t i = 0; i < ntot; ++i) iota[i] = (int32_t)i;
        ok = up(w.slot_of, iota.data(), sizeof(int32_t) * ntot) &&
             hipMemset(w.ref, 0, pack_sz * ntot) == hipSuccess &&
             hipMemset(w.nnb, 0, sizeof(int32_t) * ntot) == hipSuccess;
    }
    if (ok) ok = hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        g_create_error = "uploading the context constants failed";
        free_all(c);
        delete c;
        return RBE_ERR_HIP;
    }
    *out = c;
    return RBE_OK;
}

rbe_status rbe_create(const rbe_params *params, void *stream, rbe_ctx **out)
{
    return rbe_batch_create(params, 1, stream, out);
}

void rbe_destroy(rbe_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &p : ctx->pend) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    free_all(ctx);
    delete ctx;
}

rbe_status rbe_reserve_modes(rbe_ctx *c, int32_t cap)
{
    if (!c) return RBE_ERR_INVALID;
    if (c->R != 1) return set_err(c, RBE_ERR_STATE, "rbe_reserve_modes needs a single-system context");
    if (cap < 1 || cap > (1 << 24)) return set_err(c, RBE_ERR_INVALID, "capacity must be in [1, 2^24]");
    if (cap <= c->mcap) return RBE_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const size_t km_sz = c->prec == RBE_FP64 ? sizeof(KModeD) : sizeof(KModeF);
    const size_t kv_sz = c->prec == RBE_FP64 ? sizeof(KVjpD) : sizeof(KVjpF);
    // replace the mode-sized buffers
    auto swap_alloc = [&](void **slot, size_t bytes) -> rbe_status {
        void *old = *slot;
        void *nw = nullptr;
        rbe_status s = dalloc(c, &nw, bytes);
        if (s != RBE_OK) return s;
        auto it = std::find(c->allocs.begin(), c->allocs.end(), old);
        if (it != c->allocs.end()) c->allocs.erase(it);
        (void)hipFree(old);
        *slot = nw;
        return RBE_OK;
    };
    drop_graphs(c);
    c->sample_pending = false;
    c->cur_drawn = c->next_ready = false;
    const int old_cap = c->mcap;
    c->mcap = cap;
    rbe_status s;
    if ((s = swap_alloc((void **)&c->w.modes, sizeof(int32_t) * 3 * cap)) != RBE_OK ||
        (s = swap_alloc((void **)&c->w.mode_w, sizeof(double) * cap)) != RBE_OK ||
        (s = swap_alloc((void **)&c->w.modes_alt, sizeof(int32_t) * 3 * cap)) != RBE_OK ||
        (s = swap_alloc((void **)&c->w.mode_w_alt, sizeof(double) * cap)) != RBE_OK ||
        (s = swap_alloc((void **)&c->w.rho, sizeof(double) * 2 * cap)) != RBE_OK ||
        (s = swap_alloc((void **)&c->w.ab, sizeof(double) * 2 * cap)) != RBE_OK ||
        (s = swap_alloc(&c->w.kmode, km_sz * cap)) != RBE_OK || (s = swap_alloc(&c->w.kvjp, kv_sz * cap)) != RBE_OK) {
        c->mcap = old_cap;
        c->modes_valid = false;
        return s;
    }
    // sized for the current chunk (a long list at a small chunk would need
    // tiles x cap partials); rbe_set_tiles refuses smaller chunks afterwards
    c->partial_cap = partial_need(c, c->cfg.rho_chunk);
    if ((s = swap_alloc((void **)&c->w.partial, sizeof(double) * c->partial_cap)) != RBE_OK) return s;
    if (cap > 1024) {
        // partial forces of mode-split force passes
        const size_t esz = c->prec == RBE_FP64 ? sizeof(double) : sizeof(float);
        if ((s = swap_alloc(&c->w.fpart, esz * 3 * (size_t)kMaxModeSplit * c->ntot)) != RBE_OK) return s;
    }
    c->modes_valid = false;
    refresh_cfg_modes(c);
    return upload_rho_tiles(c);
}

rbe_status rbe_sample_k(rbe_ctx *c, uint64_t step, int32_t *modes_out)
{
    if (!c) return RBE_ERR_INVALID;
    bool dirty = false;
    for (int r = 0; r < c->R; ++r)
        if (c->sysh[r].p != c->prm[r].p) {
            c->sysh[r].p = c->prm[r].p;
            dirty = true;
        }
    if (dirty) {
        c->next_ready = false;
        rbe_status s = upload_sys(c);
        if (s != RBE_OK) return s;
        refresh_cfg_modes(c);
        if ((s = upload_rho_tiles(c)) != RBE_OK) return s;
    }
    c->modes_valid = true;
    c->cur_drawn = !c->any_mh;
    c->cur_step = step;
    if (!c->any_mh && c->next_ready && c->next_step == step) {
        // drawn already by the totals launch of the last force call
        std::swap(c->w.modes, c->w.modes_alt);
        std::swap(c->w.mode_w, c->w.mode_w_alt);
        c->next_ready = false;
        c->sample_pending = false;
    } else if (!c->any_mh && !modes_out) {
        c->sample_pending = true;
        c->sample_step = step;
        return RBE_OK;
    } else {
        c->sample_pending = false;
        RUN(c, K_SAMPLE, launch_sample(c->cfg, c->w, step, c->any_mh ? 1 : 0));
    }
    if (modes_out) {
        for (int d = 0; d < 3; ++d)
            HIPCHK(c, hipMemcpyAsync(modes_out + (size_t)d * c->mtot, c->w.modes + (size_t)d * c->mcap,
                                     sizeof(int32_t) * c->mtot, hipMemcpyDeviceToDevice, c->stream));
    }
    return RBE_OK;
}

rbe_status rbe_set_k(rbe_ctx *c, const int32_t *modes, int32_t nm, const double *weights)
{
    if (!c) return RBE_ERR_INVALID;
    if (c->R != 1) return set_err(c, RBE_ERR_STATE, "rbe_set_k needs a single-system context");
    if (!modes || nm < 1) return set_err(c, RBE_ERR_INVALID, "modes must be non-NULL and nm >= 1");
    if (nm > c->mcap)
        return set_err(c, RBE_ERR_INVALID, fmt("nm = %d exceeds the mode capacity %d (rbe_reserve_modes)", nm, c->mcap));
    std::vector<int32_t> m(3 * (size_t)c->mcap, 0);
    std::vector<double> wv(nm);
    const double S = c->sysh[0].S;
    for (int l = 0; l < nm; ++l) {
        const int32_t a = modes[l], b = modes[nm + l], d = modes[2 * nm + l];
        if (a == 0 && b == 0 && d == 0) return set_err(c, RBE_ERR_INVALID, fmt("mode %d is the zero vector", l));
        m[l] = a;
        m[c->mcap + l] = b;
        m[2 * (size_t)c->mcap + l] = d;
        wv[l] = weights ? weights[l] : S / (double)nm;
        if (!std::isfinite(wv[l])) return set_err(c, RBE_ERR_INVALID, "non-finite weight");
    }
    c->sample_pending = false;
    c->cur_drawn = c->next_ready = false;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->w.modes, m.data(), sizeof(int32_t) * m.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->w.mode_w, wv.data(), sizeof(double) * nm, hipMemcpyHostToDevice));
    if (c->sysh[0].p != nm) {
        c->sysh[0].p = nm;
        rbe_status s = upload_sys(c);
        if (s != RBE_OK) return s;
        refresh_cfg_modes(c);
        if ((s = upload_rho_tiles(c)) != RBE_OK) return s;
    }
    c->modes_valid = true;
    return RBE_OK;
}

// ---- classical Ewald mode lists (eq. 2.9, second term, truncated) ----

rbe_status rbe_ewald_radius2(double alpha, double box, double tol, int32_t *mmax2)
{
    if (!finite_pos(alpha) || !finite_pos(box) || !(tol > 0.0 && tol < 1.0) || !mmax2) {
        null_errf("alpha and box must be positive, tol in (0, 1), mmax2 non-NULL");
        return RBE_ERR_INVALID;
    }
    // exp(-pi^2 |m|^2 / (alpha L^2)) >= tol  <=>  |m|^2 <= ln(1/tol) alpha L^2 / pi^2
    const double v = std::log(1.0 / tol) * alpha * box * box / (M_PI * M_PI);
    if (!(v < 2.0e9)) {
        null_errf("the mode radius for alpha = %g, L = %g, tol = %g is beyond 32 bits", alpha, box, tol);
        return RBE_ERR_INVALID;
    }
    *mmax2 = (int32_t)std::floor(v);
    return RBE_OK;
}

rbe_status rbe_ewald_modes(double alpha, double box, int32_t mmax2, int32_t *modes, double *weights, int32_t cap,
                           int32_t *nm)
{
    if (!finite_pos(alpha) || !finite_pos(box) || mmax2 < 1 || !nm) {
        null_errf("alpha and box must be positive, mmax2 >= 1, nm non-NULL");
        return RBE_ERR_INVALID;
    }
    int R = 0;
    while ((int64_t)(R + 1) * (R + 1) <= mmax2) ++R;
    int64_t count = 0;
    for (int64_t a = -R; a <= R; ++a)
        for (int64_t b = -R; b <= R; ++b)
            for (int64_t d = -R; d <= R; ++d) {
                const int64_t m2 = a * a + b * b + d * d;
                count += m2 > 0 && m2 <= mmax2;
            }
    if (count > INT32_MAX) {
        null_errf("%lld modes do not fit 32-bit counts", (long long)count);
        return RBE_ERR_INVALID;
    }
    *nm = (int32_t)count;
    if (!modes && !weights) return RBE_OK;
    if (!modes || !weights || cap < count) {
        null_errf("modes and weights need room for %lld modes (cap = %d)", (long long)count, cap);
        return RBE_ERR_INVALID;
    }
    // Ewald weight of mode m: exp(-k^2 / (4 alpha)) with k = 2 pi |m| / L
    const double g = M_PI * M_PI / (alpha * box * box);
    int64_t l = 0;
    for (int64_t a = -R; a <= R; ++a)
        for (int64_t b = -R; b <= R; ++b)
            for (int64_t d = -R; d <= R; ++d) {
                const int64_t m2 = a * a + b * b + d * d;
                if (m2 == 0 || m2 > mmax2) continue;
                modes[l] = (int32_t)a;
                modes[(int64_t)cap + l] = (int32_t)b;
                modes[2 * (int64_t)cap + l] = (int32_t)d;
                weights[l] = std::exp(-g * (double)m2);
                ++l;
            }
    return RBE_OK;
}

rbe_status rbe_set_k_ewald(rbe_ctx *c, int32_t mmax2, int32_t *nm_out)
{
    if (!c) return RBE_ERR_INVALID;
    if (c->R != 1) return set_err(c, RBE_ERR_STATE, "rbe_set_k_ewald needs a single-system context");
    const double alpha = c->sysh[0].alpha, L = c->sysh[0].L;
    int32_t nm = 0;
    if (rbe_ewald_modes(alpha, L, mmax2, nullptr, nullptr, 0, &nm) != RBE_OK || nm < 1)
        return set_err(c, RBE_ERR_INVALID, fmt("no Ewald modes with 0 < |m|^2 <= %d", mmax2));
    std::vector<int32_t> m(3 * (size_t)nm);
    std::vector<double> w(nm);
    if (rbe_ewald_modes(alpha, L, mmax2, m.data(), w.data(), nm, &nm) != RBE_OK)
        return set_err(c, RBE_ERR_INVALID, g_create_error.c_str());
    if (nm > c->mcap) {
        rbe_status s = rbe_reserve_modes(c, nm);
        if (s != RBE_OK) return s;
    }
    rbe_status s = rbe_set_k(c, m.data(), nm, w.data());
    if (s == RBE_OK && nm_out) *nm_out = nm;
    return s;
}

// Structure factors of pos with the active modes (one staging launch and
// the reduction), then the force pass when force is given.
// Long mode lists (classical Ewald) are split over blocks so that a launch
// holds a few blocks per compute unit even for small N.
static int mode_split(int blocks, int modes, int modes_per_part)
{
    if (blocks >= 512) return 1;
    const int want = (512 + blocks - 1) / blocks;
    const int most = (modes + modes_per_part - 1) / modes_per_part;
    return std::max(1, std::min(std::min(want, most), kMaxModeSplit));
}

// Draw a recorded sample now, with its own launch.
static rbe_status materialize_sample(rbe_ctx *c)
{
    if (!c->sample_pending) return RBE_OK;
    c->sample_pending = false;
    RUN(c, K_SAMPLE, launch_sample(c->cfg, c->w, c->sample_step, 0));
    return RBE_OK;
}

static rbe_status kspace_impl(rbe_ctx *c, const void *pos, const void *q, void *force, int accumulate)
{
    StageRequest rq{const_cast<void *>(pos), nullptr, nullptr, q, 0, 0, 0, 0, 0, 1};
    rq.mode_split = mode_split(c->cfg.n_rho_tiles, c->max_p, 256);
    if (c->sample_pending) {
        int table_lds = 0, tab_max = 0;
        // fused when the launch has at most two blocks per CU: every block
        // draws the modes it needs, which costs more than one sampling
        // launch once there are many blocks
        if (c->cfg.n_rho_tiles <= 512 && stage_lds_bytes(c->cfg, 1, &table_lds, &tab_max) <= 64 * 1024) {
            // the staging launch draws the recorded sample (every block the
            // modes it needs; the first tile of each system stores them)
            rq.sample = 1;
            rq.sample_step = c->sample_step;
            rq.mode_split = 1;
            c->sample_pending = false;
        } else {
            rbe_status st = materialize_sample(c);
            if (st != RBE_OK) return st;
        }
    }
    RUN(c, K_STAGE, launch_stage(c->cfg, c->w, rq));
    // the totals launch also draws the sample of the next step into the
    // alternate mode arrays (one block per system, beside the totals blocks)
    const bool predict = c->cur_drawn && !c->any_mh && !c->fixed &&
                         !(c->next_ready && c->next_step == c->cur_step + 1);
    RUN(c, K_MID, launch_mid(c->cfg, c->w, 1, 0, nullptr, nullptr, nullptr, predict ? 1 : 0, c->cur_step + 1));
    if (predict) {
        c->next_ready = true;
        c->next_step = c->cur_step + 1;
    }
    const int fblocks = (c->cfg.n_force_tiles * c->cfg.force_split + 3) / 4;
    const int fs = c->w.fpart ? mode_split(fblocks, c->max_p, 1024) : 1;
    if (force) RUN(c, K_KFORCE, launch_kforce(c->cfg, c->w, pos, q, force, accumulate, 0, fs));
    return RBE_OK;
}

// Cell list of pos: bin (staging launch without the structure factor),
// scan, scatter into cell order.
static rbe_status cells_impl(rbe_ctx *c, const void *pos, const void *q)
{
    c->list_valid = false;   // the cell order changes under the list
    StageRequest rq{const_cast<void *>(pos), nullptr, nullptr, q, 0, 0, 0, 1, 0, 0};
    RUN(c, K_STAGE, launch_stage(c->cfg, c->w, rq));
    RUN(c, K_MID, launch_mid(c->cfg, c->w, 0, 1));
    RUN(c, K_SCATTER, launch_scatter(c->cfg, c->w));
    return RBE_OK;
}

rbe_status rbe_kspace_forces(rbe_ctx *c, const void *pos, const void *q, void *force, int32_t accumulate)
{
    if (!c) return RBE_ERR_INVALID;
    if (!pos || !q || !force) return set_err(c, RBE_ERR_INVALID, "pos, q and force must be non-NULL");
    if (!c->modes_valid) return set_err(c, RBE_ERR_STATE, "no active modes: call rbe_sample_k or rbe_set_k first");
    return kspace_impl(c, pos, q, force, accumulate);
}

rbe_status rbe_real_forces(rbe_ctx *c, const void *pos, const void *q, void *force, int32_t accumulate)
{
    if (!c) return RBE_ERR_INVALID;
    if (!pos || !q || !force) return set_err(c, RBE_ERR_INVALID, "pos, q and force must be non-NULL");
    rbe_status s = cells_impl(c, pos, q);
    if (s != RBE_OK) return s;
    RUN(c, K_REAL, launch_real(c->cfg, c->w, force, accumulate, nullptr));
    return RBE_OK;
}

// The three launches of one list-mode step (plus the sampling launch of a
// call's first step when it is not fused).  With base set (graph capture),
// s and ks are offsets from the device step number *base, and the force
// launch advances it by bump.
static rbe_status list_step(rbe_ctx *c, void *pos, void *vel, const void *q, void *force, uint64_t s, uint64_t ks,
                            bool first, bool last, bool fuse_sample, bool andersen, uint64_t *base, uint32_t bump)
{
    const int par = (int)(c->list_gen & 1);
    ListStep ls{c->w.lflag + par, c->w.lflag + (1 - par), c->w.lflag + 2, c->w.lflag + 3, c->w.lflag + 4,
                c->w.lflag + 5, c->w.lflag + 6, c->list_valid ? 0 : 1};
    ls.step_base = base;
    ls.step_bump = bump ? base : nullptr;
    ls.bump = bump;
    // the staging launch integrates (in particle order); the modes of every
    // step after the first of a call were drawn by the totals launch of the
    // step before (exact sampler)
    const bool drawn = c->fixed || (!first && !c->any_mh);
    if (!drawn && !fuse_sample) RUN(c, K_SAMPLE, launch_sample(c->cfg, c->w, ks, c->any_mh ? 1 : 0));
    StageRequest rq{pos, vel, force, q, s, ks, 1, 0, (!drawn && fuse_sample) ? 1 : 0, 1, &ls};
    // BAOAB: the closing half kick of a step is applied by the next step's
    // integrator (the force pass would touch the velocities in scattered
    // original order); only the last step of a call kicks in the force pass
    rq.kick = !first && !andersen;
    RUN(c, K_STAGE, launch_stage(c->cfg, c->w, rq));
    const bool draw_next = !c->any_mh && !c->fixed && !last;
    RUN(c, K_MID, launch_mid(c->cfg, c->w, 1, 0, nullptr, ls.rebuild, ls.rebuild_next, draw_next ? 1 : 0, ks + 1,
                             &ls));
    RUN(c, K_REAL, launch_real_step(c->cfg, c->w, ls, force, (andersen || !last) ? nullptr : vel, s));
    c->list_valid = true;
    ++c->list_gen;
    if (draw_next) {
        std::swap(c->w.modes, c->w.modes_alt);
        std::swap(c->w.mode_w, c->w.mode_w_alt);
    }
    return RBE_OK;
}

static bool same_bytes(const void *a, const void *b, size_t n) { return std::memcmp(a, b, n) == 0; }

// Step pairs per captured graph (a replay covers 2 * kGraphPairs steps).
constexpr int kGraphPairs = 8;

// Graph of 2 * kGraphPairs steady-state list steps (neither the first nor the last of a
// call, modes drawn by the step before, list valid) for the current buffers
// and parity; captured on first use.
static rbe_status step_graph(rbe_ctx *c, void *pos, void *vel, const void *q, void *force, bool andersen,
                             hipGraphExec_t *out)
{
    const int par = (int)(c->list_gen & 1);
    LaunchCfg cfg = c->cfg;
    for (auto &g : c->step_graphs)
        if (g.pos == pos && g.vel == vel && g.q == q && g.force == force && g.par == par && g.andersen == andersen &&
            same_bytes(&g.w, &c->w, sizeof(Workspace)) && same_bytes(&g.cfg, &cfg, sizeof(LaunchCfg))) {
            g.used = ++c->graph_clock;
            *out = g.exec;
            return RBE_OK;
        }
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    rbe_ctx::StepGraph g;
    g.cfg = c->cfg;
    g.w = c->w;
    g.pos = pos;
    g.vel = vel;
    g.q = q;
    g.force = force;
    g.par = par;
    g.andersen = andersen;
    // capture on the context's own stream, leaving the state as it was
    const uint64_t gen = c->list_gen;
    const Workspace w0 = c->w;
    c->cfg.stream = c->cap_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    rbe_status st = RBE_OK;
    if (e == hipSuccess) {
        // kGraphPairs copies of the two steps; each pair's second force
        // launch advances the device step number by 2
        const uint64_t k0 = andersen ? 1 : 0;
        for (int k = 0; k < kGraphPairs && st == RBE_OK; ++k) {
            st = list_step(c, pos, vel, q, force, 0, k0, false, false, false, andersen, c->w.step_base, 0);
            if (st == RBE_OK)
                st = list_step(c, pos, vel, q, force, 1, k0 + 1, false, false, false, andersen, c->w.step_base, 2);
        }
        e = hipStreamEndCapture(c->cap_stream, &graph);
    }
    c->cfg.stream = cfg.stream;
    c->list_gen = gen;
    c->w = w0;
    if (st != RBE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(c, e, "capturing the step graph");
    if (c->step_graphs.size() >= 4) {
        auto lru = std::min_element(c->step_graphs.begin(), c->step_graphs.end(),
                                    [](const auto &a, const auto &b) { return a.used < b.used; });
        (void)hipGraphExecDestroy(lru->exec);
        c->step_graphs.erase(lru);
    }
    g.used = ++c->graph_clock;
    c->step_graphs.push_back(g);
    *out = g.exec;
    return RBE_OK;
}

rbe_status rbe_step(rbe_ctx *c, void *pos, void *vel, const void *q, void *force, uint64_t first_step,
                    int32_t nsteps)
{
    if (!c) return RBE_ERR_INVALID;
    if (!pos || !vel || !q || !force) return set_err(c, RBE_ERR_INVALID, "pos, vel, q and force must be non-NULL");
    if (nsteps < 0) return set_err(c, RBE_ERR_INVALID, "nsteps must be >= 0");
    const bool andersen = c->prm[0].integrator == RBE_LEAPFROG_ANDERSEN;
    for (int r = 1; r < c->R; ++r)
        if ((c->prm[r].integrator == RBE_LEAPFROG_ANDERSEN) != andersen)
            return set_err(c, RBE_ERR_INVALID, "all systems of a batch must use one integrator");
    if (c->fixed && !c->modes_valid)
        return set_err(c, RBE_ERR_STATE, "fixed sampler: set the modes with rbe_set_k or rbe_sample_k first");
    if (c->fixed) {
        rbe_status st = materialize_sample(c);
        if (st != RBE_OK) return st;
    } else if (nsteps > 0) {
        c->sample_pending = false;   // the first step draws its own modes
        c->cur_drawn = false;
    }
    // time steps draw the next step's modes into the alternate arrays
    if (nsteps > 0) c->next_ready = false;
    for (int r = 0; r < c->R && !c->fixed; ++r)
        if (c->sysh[r].p != c->prm[r].p) {
            // explicit modes were set: stepping resamples, so restore p
            c->sysh[r].p = c->prm[r].p;
            rbe_status s = upload_sys(c);
            if (s != RBE_OK) return s;
            refresh_cfg_modes(c);
            if ((s = upload_rho_tiles(c)) != RBE_OK) return s;
        }
    // one step on the cell list = four launches: [closing kick of the step
    // before + integrate + bin + draw modes + structure-factor partials] ->
    // [totals + cell scan] -> [Fourier force + scatter] -> [real space + LJ
    // (+ the closing half kick on the last step of the call)].  In list mode, three: [closing
    // kick + integrate + list bookkeeping + partials] -> [totals + next
    // step's modes + binning, cell scan and scatter] -> [Fourier + real space
    // + LJ (+ closing kick on the last step)], where binning, scan and
    // scatter do work only on rebuild steps (decided on the device).  With graphs on, the
    // steady-state steps of a call (after the first, before the last) are
    // replayed from a captured graph.
    int table_lds = 0, tab_max = 0;
    const size_t lds = stage_lds_bytes(c->cfg, 1, &table_lds, &tab_max);
    const bool fuse_sample = !c->any_mh && lds <= 64 * 1024;
    const bool list = c->cfg.list_on != 0;
    const bool graphs = list && c->graphs && !c->any_mh && !c->prof;
    for (int32_t t = 0; t < nsteps;) {
        const uint64_t s = first_step + (uint64_t)t;
        const uint64_t ks = andersen ? s + 1 : s;
        if (list) {
            const int32_t reps = (nsteps - 1 - t) / (2 * kGraphPairs);
            if (graphs && t > 0 && c->list_valid && reps > 0) {
                hipGraphExec_t exec;
                rbe_status st = step_graph(c, pos, vel, q, force, andersen, &exec);
                if (st != RBE_OK) return st;
                RUN(c, K_MISC, launch_set_step(c->cfg, c->w, s));
                for (int32_t k = 0; k < reps; ++k) HIPCHK(c, hipGraphLaunch(exec, c->stream));
                c->list_gen += 2 * (uint64_t)kGraphPairs * reps;
                t += 2 * kGraphPairs * reps;
                continue;
            }
            rbe_status st = list_step(c, pos, vel, q, force, s, ks, t == 0, t == nsteps - 1, fuse_sample, andersen,
                                      nullptr, 0);
            if (st != RBE_OK) return st;
        } else {
            if (!c->fixed && !fuse_sample) RUN(c, K_SAMPLE, launch_sample(c->cfg, c->w, ks, c->any_mh ? 1 : 0));
            StageRequest rq{pos, vel, force, q, s, ks, 1, 1, (!c->fixed && fuse_sample) ? 1 : 0, 1};
            rq.kick = t > 0 && !andersen;
            RUN(c, K_STAGE, launch_stage(c->cfg, c->w, rq));
            RUN(c, K_MID, launch_mid(c->cfg, c->w, 1, 1));
            RUN(c, K_KFORCE, launch_kforce(c->cfg, c->w, pos, q, force, 0, 1));
            const bool last = t == nsteps - 1;
            RUN(c, K_REAL, launch_real(c->cfg, c->w, force, 1, (andersen || !last) ? nullptr : vel, s));
        }
        ++t;
    }
    if (nsteps > 0) c->modes_valid = true;
    return RBE_OK;
}

rbe_status rbe_pair_histogram(rbe_ctx *c, const void *pos, const void *q, double r_max, int32_t nbins,
                              int64_t *counts)
{
    if (!c) return RBE_ERR_INVALID;
    if (!pos || !q || !counts) return set_err(c, RBE_ERR_INVALID, "pos, q and counts must be non-NULL");
    if (nbins < 1 || nbins > 4096) return set_err(c, RBE_ERR_INVALID, "nbins must be in [1, 4096]");
    if (!std::isfinite(r_max) || r_max <= 0.0) return set_err(c, RBE_ERR_INVALID, "r_max must be > 0");
    for (int r = 0; r < c->R; ++r)
        if (r_max > 0.5 * c->sysh[r].L)
            return set_err(c, RBE_ERR_INVALID, fmt("r_max %.6g exceeds half the box of system %d", r_max, r));
    RUN(c, K_MISC, launch_pair_hist(c->cfg, c->w, pos, q, r_max, nbins, counts));
    return RBE_OK;
}

rbe_status rbe_set_dt(rbe_ctx *c, double dt, double anneal)
{
    if (!c) return RBE_ERR_INVALID;
    if (!std::isfinite(dt) || dt < 0.0) return set_err(c, RBE_ERR_INVALID, "dt must be finite and >= 0");
    if (!std::isfinite(anneal) || anneal < 0.0) return set_err(c, RBE_ERR_INVALID, "anneal must be finite and >= 0");
    for (int r = 0; r < c->R; ++r) {
        rbe_params &p = c->prm[r];
        SysDev &s = c->sysh[r];
        p.dt = dt;
        s.dt = dt;
        s.c1 = std::exp(-p.gamma * dt / p.mass);
        s.c2 = std::sqrt((1.0 - s.c1 * s.c1) * p.kT / p.mass);
        s.nu_dt = p.nu * dt;
        s.anneal = anneal;
    }
    return upload_sys(c);
}

rbe_status rbe_use_graphs(rbe_ctx *c, int32_t enable)
{
    if (!c) return RBE_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->graphs = enable != 0;
    if (!c->graphs) drop_graphs(c);
    return RBE_OK;
}

rbe_status rbe_batch_step(rbe_ctx *c, void *pos, void *vel, const void *q, void *force, uint64_t first_step,
                          int32_t nsteps)
{
    return rbe_step(c, pos, vel, q, force, first_step, nsteps);
}

// Reads the device error word and clears the bits in `mask` (synchronises).
// After a timeout the neighbour list is marked stale so that the next step
// rebuilds from the cell counts, which the force launch of the failed step
// cleared.
static rbe_status take_device_errors(rbe_ctx *c, int32_t *bits, int32_t mask = -1)
{
    int32_t flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, c->w.flag, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flag & mask) {
        const int32_t keep = flag & ~mask;
        HIPCHK(c, hipMemcpy(c->w.flag, &keep, sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (flag & mask & (kFlagTimeout | kFlagBounds)) c->list_valid = false;
    *bits = flag & mask;
    return RBE_OK;
}

static rbe_status device_error_status(rbe_ctx *c, int32_t bits)
{
    if (bits & kFlagTimeout)
        return set_err(c, RBE_ERR_TIMEOUT, "a bounded wait of a neighbour-list rebuild gave up; the forces of the "
                                           "steps since the last check are not valid");
    if (bits & kFlagBounds)
        return set_err(c, RBE_ERR_TIMEOUT, "a neighbour-list rebuild met stale cell counts; the forces of the "
                                           "steps since the last check are not valid");
    if (bits & kFlagNonFinite) return set_err(c, RBE_ERR_NONFINITE, "a kernel met a non-finite force");
    if (bits & kFlagRange)
        return set_err(c, RBE_ERR_NONFINITE, "a real-space force reached 2^20 (overlapping particles): single-precision "
                                             "pair sums are no longer exact and the forces are not valid");
    return RBE_OK;
}

rbe_status rbe_check(rbe_ctx *c)
{
    if (!c) return RBE_ERR_INVALID;
    int32_t bits = 0;
    rbe_status s = take_device_errors(c, &bits);
    if (s != RBE_OK) return s;
    return device_error_status(c, bits);
}

rbe_status rbe_set_wait_limit(rbe_ctx *c, int32_t limit)
{
    if (!c) return RBE_ERR_INVALID;
    if (limit < 0) return set_err(c, RBE_ERR_INVALID, "the wait limit must be >= 0");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cfg.wait_limit = limit;
    return RBE_OK;
}

rbe_status rbe_energy(rbe_ctx *c, const void *pos, const void *q, const void *vel, rbe_energy_t *out)
{
    if (!c) return RBE_ERR_INVALID;
    if (!pos || !q || !out) return set_err(c, RBE_ERR_INVALID, "pos, q and out must be non-NULL");
    if (!c->modes_valid) return set_err(c, RBE_ERR_STATE, "no active modes: call rbe_sample_k or rbe_set_k first");
    rbe_status s = kspace_impl(c, pos, q, nullptr, 0);
    if (s != RBE_OK) return s;
    if ((s = cells_impl(c, pos, q)) != RBE_OK) return s;
    RUN(c, K_ENERGY, launch_energy(c->cfg, c->w, q, vel));
    std::vector<double> rho(2 * (size_t)c->mtot), wts(c->mtot);
    std::vector<int32_t> modes(3 * (size_t)c->mcap);
    int32_t flag[4] = {0, 0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(c->epart_h.data(), c->w.energy_part, sizeof(double) * c->epart_h.size(),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(rho.data(), c->w.rho, sizeof(double) * rho.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(wts.data(), c->w.mode_w, sizeof(double) * wts.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(modes.data(), c->w.modes, sizeof(int32_t) * modes.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    {
        rbe_status es = take_device_errors(c, &flag[0]);
        if (es != RBE_OK) return es;
    }
    std::vector<double> acc(8 * (size_t)c->R, 0.0);
    for (size_t tile = 0; tile < c->real_sys.size(); ++tile) {
        const int r = c->real_sys[tile];
        for (int j = 0; j < 8; ++j) acc[8 * r + j] += c->epart_h[8 * tile + j];
    }
    rbe_status ret = RBE_OK;
    for (int r = 0; r < c->R; ++r) {
        const SysDev &S = c->sysh[r];
        double ek = 0.0, wk = 0.0;
        for (int l = 0; l < S.p; ++l) {
            const int o = S.moff + l;
            const double mx = modes[o], my = modes[c->mcap + o], mz = modes[2 * (size_t)c->mcap + o];
            const double m2 = mx * mx + my * my + mz * mz;
            const double rr = rho[2 * o] * rho[2 * o] + rho[2 * o + 1] * rho[2 * o + 1];
            // (2 pi/(V k^2)) |rho|^2 with k = 2 pi m/L  ==  |rho|^2 / (2 pi L |m|^2)
            const double el = wts[o] * rr / (2.0 * kPi * S.L * m2);
            ek += el;
            // lambda dE/dlambda under r -> lambda r, L -> lambda L at fixed alpha
            wk += el * (2.0 * kPi * kPi * m2 / (S.alpha * S.L * S.L) - 1.0);
        }
        rbe_energy_t &e = out[r];
        e.e_kspace = S.coulomb * ek;
        e.virial_kspace = S.coulomb * wk;
        e.e_self = -S.coulomb * std::sqrt(S.alpha / kPi) * acc[8 * r + 4];
        e.e_real = acc[8 * r + 0];
        e.e_lj = acc[8 * r + 1];
        e.virial = acc[8 * r + 2];
        e.e_kin = vel ? acc[8 * r + 3] : 0.0;
        e.charge_sum = acc[8 * r + 5];
        e.nonfinite = (flag[0] & (kFlagNonFinite | kFlagRange)) ? 1 : 0;
        e.timeout = (flag[0] & (kFlagTimeout | kFlagBounds)) ? 1 : 0;
        if (std::fabs(acc[8 * r + 5]) > 1e-6 * acc[8 * r + 6] && ret == RBE_OK) {
            ret = set_err(c, RBE_ERR_NOT_NEUTRAL,
                          fmt("system %d is not neutral: sum q = %.6g, sum |q| = %.6g", r, acc[8 * r + 5],
                              acc[8 * r + 6]));
        }
    }
    if (flag[0]) ret = device_error_status(c, flag[0]);
    return ret;
}

rbe_status rbe_get_rho(rbe_ctx *c, double *rho)
{
    if (!c || !rho) return c ? set_err(c, RBE_ERR_INVALID, "rho must be non-NULL") : RBE_ERR_INVALID;
    HIPCHK(c, hipMemcpyAsync(rho, c->w.rho, sizeof(double) * 2 * c->mtot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBE_OK;
}

rbe_status rbe_forces_vjp(rbe_ctx *c, const void *pos, const void *q, const void *grad_force, void *grad_pos,
                          void *grad_q, int32_t parts)
{
    if (!c) return RBE_ERR_INVALID;
    if (!pos || !q || !grad_force || !grad_pos || !grad_q)
        return set_err(c, RBE_ERR_INVALID, "pointers must be non-NULL");
    if (parts < 1 || parts > 3) return set_err(c, RBE_ERR_INVALID, "parts must be RBE_PART_KSPACE, _REAL or _ALL");
    if ((parts & RBE_PART_KSPACE) && !c->modes_valid)
        return set_err(c, RBE_ERR_STATE, "no active modes: call rbe_sample_k or rbe_set_k first");
    if (parts & RBE_PART_REAL)
        for (int r = 0; r < c->R; ++r)
            if (c->sysh[r].diam_on)
                return set_err(c, RBE_ERR_STATE, "the real-space adjoint does not cover per-particle diameters");
    if (parts & RBE_PART_KSPACE) {
        rbe_status s = kspace_impl(c, pos, q, nullptr, 0);
        if (s != RBE_OK) return s;
        RUN(c, K_VJP_REDUCE, launch_vjp_reduce(c->cfg, c->w, pos, q, grad_force));
        RUN(c, K_VJP_REDUCE, launch_vjp_final(c->cfg, c->w));
        RUN(c, K_VJP_GATHER, launch_vjp_gather(c->cfg, c->w, pos, q, grad_force, grad_pos, grad_q));
    }
    if (parts & RBE_PART_REAL) {
        rbe_status s = cells_impl(c, pos, q);
        if (s != RBE_OK) return s;
        RUN(c, K_VJP_REAL, launch_vjp_real(c->cfg, c->w, grad_force, grad_pos, grad_q,
                                           (parts & RBE_PART_KSPACE) ? 1 : 0));
    }
    return RBE_OK;
}

rbe_status rbe_list_builds(rbe_ctx *c, int64_t *builds)
{
    if (!c || !builds) return RBE_ERR_INVALID;
    int32_t v = 0;
    HIPCHK(c, hipMemcpyAsync(&v, c->w.lflag + 3, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *builds = c->cfg.list_on ? (int64_t)v : -1;
    // a non-finite force is left for rbe_energy / rbe_check to report
    int32_t bits = 0;
    rbe_status s = take_device_errors(c, &bits, kFlagTimeout | kFlagBounds);
    if (s != RBE_OK) return s;
    return device_error_status(c, bits);
}

rbe_status rbe_get_tiles(const rbe_ctx *c, rbe_tiles *t)
{
    if (!c || !t) return RBE_ERR_INVALID;
    t->rho_chunk = c->cfg.rho_chunk;
    t->rho_block = c->cfg.rho_block;
    t->force_split = c->cfg.force_split;
    t->real_split = c->cfg.real_split;
    return RBE_OK;
}

rbe_status rbe_set_tiles(rbe_ctx *c, const rbe_tiles *t)
{
    if (!c || !t) return RBE_ERR_INVALID;
    rbe_tiles n{c->cfg.rho_chunk, c->cfg.rho_block, c->cfg.force_split, c->cfg.real_split};
    if (t->rho_chunk) n.rho_chunk = t->rho_chunk;
    if (t->rho_block) n.rho_block = t->rho_block;
    if (t->force_split) n.force_split = t->force_split;
    if (t->real_split) n.real_split = t->real_split;
    if (n.rho_chunk < 64 || n.rho_chunk > 2048 || (n.rho_chunk % 8))
        return set_err(c, RBE_ERR_INVALID, "rho_chunk must be a multiple of 8 in [64, 2048]");
    if (n.rho_block != 256 && n.rho_block != 512 && n.rho_block != 1024)
        return set_err(c, RBE_ERR_INVALID, "rho_block must be 256, 512 or 1024");
    if (n.force_split != 1 && n.force_split != 2 && n.force_split != 4)
        return set_err(c, RBE_ERR_INVALID, "force_split must be 1, 2 or 4");
    if (n.real_split != 1 && n.real_split != 2 && n.real_split != 4 && n.real_split != 8)
        return set_err(c, RBE_ERR_INVALID, "real_split must be 1, 2, 4 or 8");
    if (!tiles_fit(n)) return set_err(c, RBE_ERR_INVALID, "rho_chunk and rho_block need more than 64 KB of LDS");
    if (partial_need(c, n.rho_chunk) > c->partial_cap)
        return set_err(c, RBE_ERR_INVALID, "rho_chunk too small for the structure-factor partials of the reserved "
                                           "mode capacity");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cfg.rho_chunk = n.rho_chunk;
    c->cfg.rho_block = n.rho_block;
    c->cfg.force_split = n.force_split;
    c->cfg.real_split = n.real_split;
    rbe_status st = upload_rho_tiles(c);
    if (st != RBE_OK) return st;
    return upload_list_tiles(c);
}

rbe_status rbe_tune_lookup(const char *arch, int32_t precision, int64_t ntot, int32_t max_p, int32_t R,
                           rbe_tiles *out)
{
    if (!arch || !out || ntot < 1 || max_p < 1 || R < 1) return RBE_ERR_INVALID;
    return tune_lookup(tune_key(arch, precision, ntot, max_p, R), out) ? RBE_OK : RBE_ERR_STATE;
}

rbe_status rbe_autotune(rbe_ctx *c, const void *pos, const void *q, int32_t reps, rbe_tiles *best)
{
    if (!c) return RBE_ERR_INVALID;
    if (!pos || !q) return set_err(c, RBE_ERR_INVALID, "pos and q must be non-NULL");
    if (!c->modes_valid) return set_err(c, RBE_ERR_STATE, "no active modes: call rbe_sample_k or rbe_set_k first");
    if (reps < 1) reps = 10;
    {
        rbe_status st = materialize_sample(c);
        if (st != RBE_OK) return st;
    }
    const bool prof = c->prof;
    c->prof = false;
    hipEvent_t a, b;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    auto timeit = [&](auto &&body, float *ms) -> rbe_status {
        rbe_status s = body();  // warm-up
        if (s != RBE_OK) return s;
        HIPCHK(c, hipEventRecord(a, c->stream));
        for (int k = 0; k < reps; ++k)
            if ((s = body()) != RBE_OK) return s;
        HIPCHK(c, hipEventRecord(b, c->stream));
        HIPCHK(c, hipEventSynchronize(b));
        HIPCHK(c, hipEventElapsedTime(ms, a, b));
        return RBE_OK;
    };
    rbe_tiles cur;
    rbe_get_tiles(c, &cur);
    rbe_tiles win = cur;
    float best_rho = 1e30f, best_f = 1e30f;
    const int fill = (int)std::min<int64_t>(2048, std::max<int64_t>(64, ((c->ntot + 255) / 256 + 7) / 8 * 8));
    const int chunks[] = {128, 256, 512, 1024, fill};
    const int blocks[] = {256, 512, 1024};
    rbe_status s = RBE_OK;
    for (int ch : chunks)
        for (int bl : blocks) {
            rbe_tiles t{ch, bl, cur.force_split, 0};
            if (rbe_set_tiles(c, &t) != RBE_OK) continue;   // shape does not fit
            float ms = 0.f;
            s = timeit(
                [&]() -> rbe_status {
                    StageRequest rq{const_cast<void *>(pos), nullptr, nullptr, q, 0, 0, 0, 0, 0, 1};
                    RUN(c, K_STAGE, launch_stage(c->cfg, c->w, rq));
                    RUN(c, K_MID, launch_mid(c->cfg, c->w, 1, 0));
                    return RBE_OK;
                },
                &ms);
            if (s != RBE_OK) break;
            if (ms < best_rho) {
                best_rho = ms;
                win.rho_chunk = ch;
                win.rho_block = bl;
            }
        }
    if (s == RBE_OK) {
        rbe_tiles t{win.rho_chunk, win.rho_block, 0, 0};
        s = rbe_set_tiles(c, &t);
    }
    void *fbuf = nullptr;
    if (s == RBE_OK) {
        const size_t esz = c->prec == RBE_FP64 ? 8 : 4;
        // the force pass needs an output: borrow the sorted workspace, which
        // is large enough (16 or 32 bytes per particle >= 3 elements); the
        // neighbour list reads that workspace, so it must be rebuilt
        fbuf = c->w.sorted;
        c->list_valid = false;
        (void)esz;
        for (int sp : {1, 2, 4}) {
            rbe_tiles t{0, 0, sp, 0};
            if ((s = rbe_set_tiles(c, &t)) != RBE_OK) break;
            float ms = 0.f;
            s = timeit(
                [&]() -> rbe_status {
                    RUN(c, K_KFORCE, launch_kforce(c->cfg, c->w, pos, q, fbuf, 0, 0));
                    return RBE_OK;
                },
                &ms);
            if (s != RBE_OK) break;
            if (ms < best_f) {
                best_f = ms;
                win.force_split = sp;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    c->prof = prof;
    if (s != RBE_OK) return s;
    if ((s = rbe_set_tiles(c, &win)) != RBE_OK) return s;
    tune_store(tune_key(c->arch.c_str(), c->prec, c->ntot, c->max_p, c->R), win);
    if (best) *best = win;
    return RBE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Fourier force without allocation.  Its workspace (system constants, tiles,
// structure-factor partials and totals, per-mode constants) is one
// file-scope device array of fixed size: each GPU the library runs on holds
// its own copy until the process ends.  Host code never uses the array's
// name as an address; each device's address is taken once, with that device
// current, by hipGetSymbolAddress, and only that pointer reaches kernels.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kStaticMaxN = 1 << 20;     // particles
constexpr int kStaticMaxP = 512;             // modes
constexpr int kStaticMaxRhoTiles = 2048;     // structure-factor tiles of default_rho_chunk up to kStaticMaxN
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kOffSys = 0;
constexpr size_t kOffPartOff = kOffSys + align256(sizeof(SysDev));
constexpr size_t kOffFlag = kOffPartOff + 256;
constexpr size_t kOffRhoTiles = kOffFlag + 256;
constexpr size_t kOffForceTiles = kOffRhoTiles + align256(sizeof(Tile) * kStaticMaxRhoTiles);
constexpr size_t kOffModeW = kOffForceTiles + align256(sizeof(Tile) * (kStaticMaxN / 64));
constexpr size_t kOffRho = kOffModeW + align256(sizeof(double) * kStaticMaxP);
constexpr size_t kOffKmode = kOffRho + align256(sizeof(double) * 2 * kStaticMaxP);
constexpr size_t kOffPartial = kOffKmode + align256(sizeof(KModeD) * kStaticMaxP);
constexpr size_t kStaticBytes = kOffPartial + sizeof(double) * 2 * (size_t)kStaticMaxRhoTiles * kStaticMaxP;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (the device must be current).  The first
// call on a device checks that it is a gfx950 and takes the address.
rbe_status scratch_of_device(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        null_errf("device %d is beyond the %d devices this entry point tracks", dev, kMaxDevices);
        return RBE_ERR_NO_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess || std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            (void)hipGetLastError();
            null_errf("device %d is not gfx950", dev);
            return RBE_ERR_NO_DEVICE;
        }
        unsigned char *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            null_errf("hipGetSymbolAddress of the static workspace failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return RBE_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RBE_OK;
}
}  // namespace

extern "C" {

rbe_status rbe_kspace_forces_noalloc(const rbe_params *params, const int32_t *modes, const void *pos,
                                     const void *q, void *force, int32_t accumulate, void *stream)
{
    if (!params || !modes || !pos || !q || !force) {
        g_create_error = "params, modes, pos, q and force must be non-NULL";
        return RBE_ERR_INVALID;
    }
    const rbe_params &p = *params;
    if (p.n < 1 || p.n > kStaticMaxN) {
        null_errf("n = %d is outside [1, %lld], the size of this entry point's fixed workspace", p.n,
                  (long long)kStaticMaxN);
        return RBE_ERR_INVALID;
    }
    if (p.p < 1 || p.p > kStaticMaxP) {
        null_errf("p = %d is outside [1, %d], the size of this entry point's fixed workspace", p.p, kStaticMaxP);
        return RBE_ERR_INVALID;
    }
    if (!finite_pos(p.box) || !finite_pos(p.alpha) || !std::isfinite(p.coulomb)) {
        null_errf("box and alpha must be finite and > 0, coulomb finite");
        return RBE_ERR_INVALID;
    }
    if (p.precision != RBE_FP32 && p.precision != RBE_FP64) {
        null_errf("unknown precision %d", p.precision);
        return RBE_ERR_INVALID;
    }
    const double H = normaliser_H(p.alpha, p.box);
    if (1.0 / (H * H * H) > 0.5 || (p.precision == RBE_FP32 && table_half_width(p.alpha, p.box) > 4095)) {
        null_errf("alpha L^2 = %.3g is outside the range of the mode table", p.alpha * p.box * p.box);
        return RBE_ERR_INVALID;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        null_errf("no HIP device available");
        return RBE_ERR_NO_DEVICE;
    }
    unsigned char *base = nullptr;
    rbe_status st = scratch_of_device(dev, &base);
    if (st != RBE_OK) return st;

    SysDev sys{};
    fourier_constants(p, sys);
    LaunchCfg c{};
    c.stream = (hipStream_t)stream;
    c.R = 1;
    c.prec = p.precision;
    c.ntot = p.n;
    c.mcap = p.p;
    c.max_p = p.p;
    c.rho_chunk = default_rho_chunk(p.n);
    c.rho_block = 1024;
    c.force_split = default_force_split(p.n);
    c.n_rho_tiles = (p.n + c.rho_chunk - 1) / c.rho_chunk;
    c.max_sys_rho_tiles = c.n_rho_tiles;
    c.n_force_tiles = (p.n + 63) / 64;
    if (c.n_rho_tiles > kStaticMaxRhoTiles) {
        null_errf("internal: %d structure-factor tiles exceed the fixed workspace", c.n_rho_tiles);
        return RBE_ERR_INVALID;
    }
    Workspace w{};
    w.sys = reinterpret_cast<SysDev *>(base + kOffSys);
    w.partial_off = reinterpret_cast<int32_t *>(base + kOffPartOff);
    w.flag = reinterpret_cast<int32_t *>(base + kOffFlag);
    w.rho_tiles = reinterpret_cast<Tile *>(base + kOffRhoTiles);
    w.force_tiles = reinterpret_cast<Tile *>(base + kOffForceTiles);
    w.mode_w = reinterpret_cast<double *>(base + kOffModeW);
    w.rho = reinterpret_cast<double *>(base + kOffRho);
    w.kmode = base + kOffKmode;
    w.partial = reinterpret_cast<double *>(base + kOffPartial);
    w.modes = const_cast<int32_t *>(modes);

    auto hip_err = [](hipError_t e, const char *what) {
        null_errf("%s: %s", what, hipGetErrorString(e));
        return RBE_ERR_HIP;
    };
    hipError_t e = launch_static_setup(c, w, sys);
    if (e != hipSuccess) return hip_err(e, "static workspace set-up");
    StageRequest rq{const_cast<void *>(pos), nullptr, nullptr, q, 0, 0, 0, 0, 0, 1};
    rq.mode_split = mode_split(c.n_rho_tiles, p.p, 256);
    if ((e = launch_stage(c, w, rq)) != hipSuccess) return hip_err(e, "structure-factor launch");
    if ((e = launch_mid(c, w, 1, 0)) != hipSuccess) return hip_err(e, "totals launch");
    if ((e = launch_kforce(c, w, pos, q, force, accumulate, 0, 1)) != hipSuccess) return hip_err(e, "force launch");
    return RBE_OK;
}

rbe_status rbe_profile_enable(rbe_ctx *c, int32_t enable)
{
    if (!c) return RBE_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pend) {
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pend.clear();
    for (int k = 0; k < K_COUNT; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    c->prof = enable != 0;
    return RBE_OK;
}

rbe_status rbe_profile_read(rbe_ctx *c, int32_t id, double *total_ms, int64_t *launches)
{
    if (!c) return RBE_ERR_INVALID;
    if (id < 0 || id >= K_COUNT) return set_err(c, RBE_ERR_INVALID, "unknown kernel id");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pend) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, p.a, p.b));
        c->prof_ms[p.id] += ms;
        c->prof_n[p.id] += 1;
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pend.clear();
    if (total_ms) *total_ms = c->prof_ms[id];
    if (launches) *launches = c->prof_n[id];
    return RBE_OK;
}

const char *rbe_profile_name(int32_t id)
{
    if (id < 0 || id >= K_COUNT) return nullptr;
    return kKernelNames[id];
}

int32_t rbe_profile_count(void) { return K_COUNT; }

}  // extern "C"
