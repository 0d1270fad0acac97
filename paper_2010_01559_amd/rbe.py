"""Thin ctypes binding over librbe (declared in include/rbe.h).

Every function marshals torch device tensors into raw pointers and calls the
C entry point of the same name; all arithmetic runs in the library's HIP
kernels.  There is no fallback: if ``librbe.so`` is missing or no gfx950
device is present the calls raise.

Array conventions follow the C ABI: positions, velocities, forces and
gradients are ``[3, N_tot]`` contiguous tensors, charges ``[N_tot]``, float32
for ``RBE_FP32`` contexts and float64 for ``RBE_FP64``; modes are
``[3, M_tot]`` int32.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbe.so")

RBE_OK = 0
RBE_ERR_INVALID = -1
RBE_ERR_NOT_NEUTRAL = -2
RBE_ERR_CUTOFF = -3
RBE_ERR_OOM = -4
RBE_ERR_HIP = -5
RBE_ERR_NONFINITE = -6
RBE_ERR_STATE = -7
RBE_ERR_NO_DEVICE = -8
RBE_ERR_TIMEOUT = -9
RBE_FP32, RBE_FP64 = 0, 1
RBE_LANGEVIN_BAOAB, RBE_LEAPFROG_ANDERSEN = 0, 1
RBE_SAMPLER_EXACT, RBE_SAMPLER_MH, RBE_SAMPLER_FIXED = 0, 1, 2
RBE_PART_KSPACE, RBE_PART_REAL, RBE_PART_ALL = 1, 2, 3

STATUS_NAMES = {0: "RBE_OK", -1: "RBE_ERR_INVALID", -2: "RBE_ERR_NOT_NEUTRAL", -3: "RBE_ERR_CUTOFF",
                -4: "RBE_ERR_OOM", -5: "RBE_ERR_HIP", -6: "RBE_ERR_NONFINITE", -7: "RBE_ERR_STATE",
                -8: "RBE_ERR_NO_DEVICE", -9: "RBE_ERR_TIMEOUT"}

# every symbol the header declares
EXPORTED = ["rbe_normalizer", "rbe_create", "rbe_batch_create", "rbe_destroy", "rbe_last_error",
            "rbe_num_systems", "rbe_num_particles", "rbe_num_modes", "rbe_sample_k", "rbe_set_k",
            "rbe_reserve_modes", "rbe_kspace_forces", "rbe_real_forces", "rbe_step", "rbe_batch_step",
            "rbe_energy", "rbe_check", "rbe_set_wait_limit", "rbe_get_rho", "rbe_forces_vjp", "rbe_list_builds", "rbe_pair_histogram", "rbe_set_dt", "rbe_use_graphs", "rbe_get_tiles",
            "rbe_set_tiles", "rbe_autotune", "rbe_profile_enable", "rbe_profile_read", "rbe_profile_name",
            "rbe_profile_count", "rbe_kspace_forces_noalloc", "rbe_calibrate", "rbe_tune_lookup",
            "rbe_ewald_radius2", "rbe_ewald_modes", "rbe_set_k_ewald"]


class RBEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class rbe_params(C.Structure):
    _fields_ = [("n", C.c_int32), ("p", C.c_int32), ("box", C.c_double), ("alpha", C.c_double),
                ("r_cut", C.c_double), ("coulomb", C.c_double), ("lj_eps", C.c_double), ("lj_sigma", C.c_double),
                ("lj_rcut", C.c_double), ("kT", C.c_double), ("gamma", C.c_double), ("dt", C.c_double),
                ("mass", C.c_double), ("nu", C.c_double), ("skin", C.c_double), ("seed", C.c_uint64), ("precision", C.c_int32),
                ("integrator", C.c_int32), ("sampler", C.c_int32), ("flags", C.c_int32),
                ("n_fixed", C.c_int32), ("reserved", C.c_int32), ("diameter", C.c_void_p)]


class rbe_energy_t(C.Structure):
    _fields_ = [("e_kspace", C.c_double), ("e_self", C.c_double), ("e_real", C.c_double), ("e_lj", C.c_double),
                ("e_kin", C.c_double), ("virial", C.c_double), ("virial_kspace", C.c_double),
                ("charge_sum", C.c_double),
                ("nonfinite", C.c_int32), ("timeout", C.c_int32)]


class rbe_tiles(C.Structure):
    _fields_ = [("rho_chunk", C.c_int32), ("rho_block", C.c_int32), ("force_split", C.c_int32),
                ("real_split", C.c_int32)]


_lib = None


def lib():
    """Load librbe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_01559_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    L.rbe_normalizer.argtypes = [d, d, C.POINTER(d), C.POINTER(d)]
    L.rbe_create.argtypes = [C.POINTER(rbe_params), vp, C.POINTER(vp)]
    L.rbe_batch_create.argtypes = [C.POINTER(rbe_params), i32, vp, C.POINTER(vp)]
    L.rbe_destroy.argtypes = [vp]
    L.rbe_destroy.restype = None
    L.rbe_last_error.argtypes = [vp]
    L.rbe_last_error.restype = C.c_char_p
    L.rbe_num_systems.argtypes = [vp]
    L.rbe_num_systems.restype = i32
    L.rbe_num_particles.argtypes = [vp]
    L.rbe_num_particles.restype = i64
    L.rbe_num_modes.argtypes = [vp]
    L.rbe_num_modes.restype = i32
    L.rbe_sample_k.argtypes = [vp, u64, vp]
    L.rbe_set_k.argtypes = [vp, vp, i32, vp]
    L.rbe_reserve_modes.argtypes = [vp, i32]
    L.rbe_ewald_radius2.argtypes = [C.c_double, C.c_double, C.c_double, vp]
    L.rbe_ewald_modes.argtypes = [C.c_double, C.c_double, i32, vp, vp, i32, vp]
    L.rbe_set_k_ewald.argtypes = [vp, i32, vp]
    L.rbe_kspace_forces.argtypes = [vp, vp, vp, vp, i32]
    L.rbe_real_forces.argtypes = [vp, vp, vp, vp, i32]
    L.rbe_step.argtypes = [vp, vp, vp, vp, vp, u64, i32]
    L.rbe_batch_step.argtypes = [vp, vp, vp, vp, vp, u64, i32]
    L.rbe_energy.argtypes = [vp, vp, vp, vp, C.POINTER(rbe_energy_t)]
    L.rbe_get_rho.argtypes = [vp, vp]
    L.rbe_check.argtypes = [vp]
    L.rbe_calibrate.argtypes = [i32, i32, C.POINTER(d)]
    L.rbe_tune_lookup.argtypes = [C.c_char_p, i32, i64, i32, i32, C.POINTER(rbe_tiles)]
    L.rbe_kspace_forces_noalloc.argtypes = [C.POINTER(rbe_params), vp, vp, vp, vp, i32, vp]
    L.rbe_set_wait_limit.argtypes = [vp, i32]
    L.rbe_forces_vjp.argtypes = [vp, vp, vp, vp, vp, vp, i32]
    L.rbe_list_builds.argtypes = [vp, C.POINTER(i64)]
    L.rbe_use_graphs.argtypes = [vp, i32]
    L.rbe_set_dt.argtypes = [vp, C.c_double, C.c_double]
    L.rbe_pair_histogram.argtypes = [vp, vp, vp, C.c_double, i32, vp]
    L.rbe_get_tiles.argtypes = [vp, C.POINTER(rbe_tiles)]
    L.rbe_set_tiles.argtypes = [vp, C.POINTER(rbe_tiles)]
    L.rbe_autotune.argtypes = [vp, vp, vp, i32, C.POINTER(rbe_tiles)]
    L.rbe_profile_enable.argtypes = [vp, i32]
    L.rbe_profile_read.argtypes = [vp, i32, C.POINTER(d), C.POINTER(i64)]
    L.rbe_profile_name.argtypes = [i32]
    L.rbe_profile_name.restype = C.c_char_p
    L.rbe_profile_count.argtypes = []
    L.rbe_profile_count.restype = i32
    for name in EXPORTED:
        f = getattr(L, name)
        if f.restype is C.c_int:  # default: status functions
            f.restype = C.c_int
    _lib = L
    return L


def _check(st, ctx=None):
    if st != RBE_OK:
        raise RBEError(st, lib().rbe_last_error(ctx).decode())


@dataclass
class Params:
    """Python mirror of rbe_params (paper notation in the field comments of
    include/rbe.h)."""
    n: int
    p: int
    box: float
    alpha: float
    r_cut: float
    coulomb: float = 1.0
    lj_eps: float = 0.0
    lj_sigma: float = 1.0
    lj_rcut: float = 2.5
    kT: float = 1.0
    gamma: float = 1.0
    dt: float = 1e-3
    mass: float = 1.0
    nu: float = 0.0
    skin: float = 0.0
    seed: int = 0
    precision: int = RBE_FP32
    integrator: int = RBE_LANGEVIN_BAOAB
    sampler: int = RBE_SAMPLER_EXACT
    flags: int = 0
    n_fixed: int = 0
    diameter: np.ndarray | None = None   # [n] diameters of eq. (4.1), read at creation

    def to_c(self):
        dp = None
        if self.diameter is not None:
            self.diameter = np.ascontiguousarray(self.diameter, dtype=np.float64)
            if self.diameter.shape != (self.n,):
                raise ValueError("diameter must have shape (n,)")
            dp = self.diameter.ctypes.data
        return rbe_params(self.n, self.p, self.box, self.alpha, self.r_cut, self.coulomb, self.lj_eps,
                          self.lj_sigma, self.lj_rcut, self.kT, self.gamma, self.dt, self.mass, self.nu,
                          self.skin, self.seed, self.precision, self.integrator, self.sampler, self.flags,
                          self.n_fixed, 0, dp)


DEFAULT_SKIN_FRACTION = 0.14


def params_from_system(s, precision=RBE_FP32, **over):
    """Params for a workloads.System; the neighbour-list skin defaults to
    0.14 of the largest cutoff (the fastest N = 1e5 electrolyte step: a
    thinner skin rebuilds more often, a thicker one lists more pairs).
    Per-particle diameters and immobile leading particles come from
    ``s.extra`` ("diameter", "n_fixed") when present."""
    rmax = max(s.r_cut, s.lj[2] if s.lj[0] > 0 else 0.0)
    kw = dict(n=s.n, p=s.p, box=s.L, alpha=s.alpha, r_cut=s.r_cut, coulomb=s.coulomb, lj_eps=s.lj[0],
              lj_sigma=s.lj[1], lj_rcut=s.lj[2], kT=s.kT, gamma=s.gamma, dt=s.dt, mass=s.mass, seed=s.seed,
              skin=DEFAULT_SKIN_FRACTION * rmax, precision=precision,
              n_fixed=int(s.extra.get("n_fixed", 0)), diameter=s.extra.get("diameter"))
    kw.update(over)
    return Params(**kw)


class Context:
    """Owns an rbe_ctx handle."""

    def __init__(self, handle, params, stream):
        self.handle = handle
        self.params = params
        self.stream = stream
        self.precision = params[0].precision
        self.R = lib().rbe_num_systems(handle)
        self.ntot = lib().rbe_num_particles(handle)
        self.offsets = np.concatenate([[0], np.cumsum([p.n for p in params])]).astype(np.int64)

    @property
    def nmodes(self):
        return lib().rbe_num_modes(self.handle)

    def close(self):
        if self.handle:
            lib().rbe_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _torch():
    import torch
    return torch


def _dtype(ctx):
    torch = _torch()
    return torch.float64 if ctx.precision == RBE_FP64 else torch.float32


def _ptr(t, ctx, shape, dtype=None, name="tensor"):
    torch = _torch()
    dtype = dtype or _dtype(ctx)
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _vec3(ctx, t, name):
    return _ptr(t, ctx, (3, ctx.ntot), name=name)


def _scal(ctx, t, name):
    return _ptr(t, ctx, (ctx.ntot,), name=name)


# -- entry points (same names as the C ABI) --------------------------------------

def rbe_normalizer(alpha, box):
    H, S = C.c_double(), C.c_double()
    _check(lib().rbe_normalizer(alpha, box, C.byref(H), C.byref(S)))
    return H.value, S.value


def rbe_batch_create(params, stream=None):
    """params: list of Params; stream: a torch.cuda.Stream (default: current)."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    arr = (rbe_params * len(params))(*[p.to_c() for p in params])
    h = C.c_void_p()
    _check(lib().rbe_batch_create(arr, len(params), C.c_void_p(stream.cuda_stream), C.byref(h)))
    return Context(h, list(params), stream)


def rbe_create(params, stream=None):
    return rbe_batch_create([params], stream)


def rbe_destroy(ctx):
    ctx.close()


def rbe_sample_k(ctx, step, modes_out=None):
    mp = None
    if modes_out is not None:
        torch = _torch()
        mp = _ptr(modes_out, ctx, (3, sum(p.p for p in ctx.params)), torch.int32, "modes_out")
    _check(lib().rbe_sample_k(ctx.handle, step, mp), ctx.handle)


def rbe_set_k(ctx, modes, weights=None):
    m = np.ascontiguousarray(modes, dtype=np.int32)
    if m.ndim != 2 or m.shape[0] != 3:
        raise ValueError("modes must be [3, nm]")
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if w is not None and w.shape != (m.shape[1],):
        raise ValueError("weights must be [nm]")
    _check(lib().rbe_set_k(ctx.handle, m.ctypes.data_as(C.c_void_p), m.shape[1],
                           None if w is None else w.ctypes.data_as(C.c_void_p)), ctx.handle)


def rbe_reserve_modes(ctx, cap):
    _check(lib().rbe_reserve_modes(ctx.handle, cap), ctx.handle)


def rbe_ewald_radius2(alpha, box, tol):
    v = C.c_int32()
    _check(lib().rbe_ewald_radius2(float(alpha), float(box), float(tol), C.byref(v)))
    return v.value


def rbe_ewald_modes(alpha, box, mmax2):
    """(modes int32 [3, nm], weights float64 [nm]) of the classical Ewald list."""
    nm = C.c_int32()
    _check(lib().rbe_ewald_modes(float(alpha), float(box), int(mmax2), None, None, 0, C.byref(nm)))
    m = np.zeros((3, nm.value), dtype=np.int32)
    w = np.zeros(nm.value, dtype=np.float64)
    _check(lib().rbe_ewald_modes(float(alpha), float(box), int(mmax2), m.ctypes.data_as(C.c_void_p),
                                 w.ctypes.data_as(C.c_void_p), nm.value, C.byref(nm)))
    return m, w


def rbe_set_k_ewald(ctx, mmax2):
    nm = C.c_int32()
    _check(lib().rbe_set_k_ewald(ctx.handle, int(mmax2), C.byref(nm)), ctx.handle)
    return nm.value


def rbe_kspace_forces(ctx, pos, q, force, accumulate=False):
    _check(lib().rbe_kspace_forces(ctx.handle, _vec3(ctx, pos, "pos"), _scal(ctx, q, "q"),
                                   _vec3(ctx, force, "force"), int(accumulate)), ctx.handle)


def rbe_kspace_forces_noalloc(params, modes, pos, q, force, accumulate=False, stream=None):
    """Context-free Fourier force with the caller's modes ([3, p] int32 on the
    GPU); nothing is allocated (the library's fixed workspace is used)."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    dt = torch.float64 if params.precision == RBE_FP64 else torch.float32
    n = params.n

    def ptr(t, shape, dtype, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dtype or \
                tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} GPU tensor of shape {tuple(shape)}")
        return C.c_void_p(t.data_ptr())

    cp = params.to_c()
    st = lib().rbe_kspace_forces_noalloc(C.byref(cp), ptr(modes, (3, params.p), torch.int32, "modes"),
                                         ptr(pos, (3, n), dt, "pos"), ptr(q, (n,), dt, "q"),
                                         ptr(force, (3, n), dt, "force"), int(accumulate),
                                         C.c_void_p(stream.cuda_stream))
    _check(st)


def rbe_real_forces(ctx, pos, q, force, accumulate=False):
    _check(lib().rbe_real_forces(ctx.handle, _vec3(ctx, pos, "pos"), _scal(ctx, q, "q"),
                                 _vec3(ctx, force, "force"), int(accumulate)), ctx.handle)


def rbe_step(ctx, pos, vel, q, force, first_step, nsteps):
    _check(lib().rbe_step(ctx.handle, _vec3(ctx, pos, "pos"), _vec3(ctx, vel, "vel"), _scal(ctx, q, "q"),
                          _vec3(ctx, force, "force"), first_step, nsteps), ctx.handle)


def rbe_batch_step(ctx, pos, vel, q, force, first_step, nsteps):
    _check(lib().rbe_batch_step(ctx.handle, _vec3(ctx, pos, "pos"), _vec3(ctx, vel, "vel"), _scal(ctx, q, "q"),
                                _vec3(ctx, force, "force"), first_step, nsteps), ctx.handle)


def rbe_energy(ctx, pos, q, vel=None, allow_status=(RBE_OK,)):
    """Returns (status, list of dicts per system)."""
    out = (rbe_energy_t * ctx.R)()
    vp = None if vel is None else _vec3(ctx, vel, "vel")
    st = lib().rbe_energy(ctx.handle, _vec3(ctx, pos, "pos"), _scal(ctx, q, "q"), vp, out)
    if st not in allow_status:
        _check(st, ctx.handle)
    res = []
    for e in out:
        res.append({k: getattr(e, k) for k, _ in rbe_energy_t._fields_})
    return st, res


def rbe_check(ctx):
    """Raises RBEError for a pending device error (non-finite force, or a list
    rebuild whose bounded wait gave up); clears it.  Synchronises."""
    _check(lib().rbe_check(ctx.handle), ctx.handle)


def rbe_check_status(ctx):
    """The status rbe_check would raise for (RBE_OK if none); clears it."""
    return lib().rbe_check(ctx.handle)


def rbe_set_wait_limit(ctx, limit):
    """Spin bound of the device-side waits of a list rebuild (0: give up at once)."""
    _check(lib().rbe_set_wait_limit(ctx.handle, int(limit)), ctx.handle)


def rbe_get_rho(ctx):
    n = ctx.nmodes
    buf = np.zeros((n, 2), np.float64)
    _check(lib().rbe_get_rho(ctx.handle, buf.ctypes.data_as(C.c_void_p)), ctx.handle)
    return buf


def rbe_forces_vjp(ctx, pos, q, grad_force, grad_pos, grad_q, parts=RBE_PART_ALL):
    _check(lib().rbe_forces_vjp(ctx.handle, _vec3(ctx, pos, "pos"), _scal(ctx, q, "q"),
                                _vec3(ctx, grad_force, "grad_force"), _vec3(ctx, grad_pos, "grad_pos"),
                                _scal(ctx, grad_q, "grad_q"), parts), ctx.handle)


def rbe_list_builds(ctx, allow_status=(RBE_OK,)):
    """Neighbour-list builds made by rbe_step so far (-1: no list).  With
    RBE_ERR_TIMEOUT in allow_status, returns (status, builds) instead."""
    v = C.c_int64()
    st = lib().rbe_list_builds(ctx.handle, C.byref(v))
    if st not in allow_status:
        _check(st, ctx.handle)
    return (st, v.value) if len(allow_status) > 1 else v.value


def rbe_pair_histogram(ctx, pos, q, r_max, nbins, counts):
    """Adds pair counts to counts (device int64 [R, 3, nbins]; classes ++, +-, --)."""
    torch = _torch()
    cp = _ptr(counts, ctx, (ctx.R, 3, int(nbins)), torch.int64, "counts")
    _check(lib().rbe_pair_histogram(ctx.handle, _vec3(ctx, pos, "pos"), _scal(ctx, q, "q"), float(r_max),
                                    int(nbins), cp), ctx.handle)


def rbe_set_dt(ctx, dt, anneal=0.0):
    """Fixed time step dt, or (anneal > 0) the burn-in schedule dt_n = anneal / ln(1 + n)."""
    _check(lib().rbe_set_dt(ctx.handle, float(dt), float(anneal)), ctx.handle)
    for p in ctx.params:
        p.dt = float(dt)


def rbe_use_graphs(ctx, enable):
    """Replay the steady-state steps of rbe_step from captured graphs (default) or not."""
    _check(lib().rbe_use_graphs(ctx.handle, int(bool(enable))), ctx.handle)


def rbe_get_tiles(ctx):
    t = rbe_tiles()
    _check(lib().rbe_get_tiles(ctx.handle, C.byref(t)), ctx.handle)
    return {k: getattr(t, k) for k, _ in rbe_tiles._fields_}


def rbe_set_tiles(ctx, rho_chunk=0, rho_block=0, force_split=0, real_split=0):
    t = rbe_tiles(rho_chunk, rho_block, force_split, real_split)
    _check(lib().rbe_set_tiles(ctx.handle, C.byref(t)), ctx.handle)


def rbe_autotune(ctx, pos, q, reps=10):
    t = rbe_tiles()
    _check(lib().rbe_autotune(ctx.handle, _vec3(ctx, pos, "pos"), _scal(ctx, q, "q"), reps, C.byref(t)),
           ctx.handle)
    return {k: getattr(t, k) for k, _ in rbe_tiles._fields_}


def rbe_tune_lookup(arch, precision, ntot, max_p, R=1):
    """Tile shapes the cache holds for this configuration, or None."""
    t = rbe_tiles()
    st = lib().rbe_tune_lookup(arch.encode(), int(precision), int(ntot), int(max_p), int(R), C.byref(t))
    if st == RBE_ERR_STATE:
        return None
    _check(st)
    return {k: getattr(t, k) for k, _ in rbe_tiles._fields_}


def rbe_profile_enable(ctx, enable=True):
    _check(lib().rbe_profile_enable(ctx.handle, int(enable)), ctx.handle)


def rbe_profile_read(ctx):
    """{kernel name: (total ms, launches)} since enabling."""
    out = {}
    for k in range(lib().rbe_profile_count()):
        ms, n = C.c_double(), C.c_int64()
        _check(lib().rbe_profile_read(ctx.handle, k, C.byref(ms), C.byref(n)), ctx.handle)
        out[lib().rbe_profile_name(k).decode()] = (ms.value, n.value)
    return out


CALIBRATION_KINDS = {0: "sin_cos_lane_ops_per_s", 1: "fp32_fma_lane_ops_per_s", 2: "fp64_fma_lane_ops_per_s",
                     3: "copy_bytes_per_s"}


def rbe_calibrate(kind, reps=5):
    """Device throughput micro-benchmark (see include/rbe.h); returns the rate."""
    r = C.c_double()
    _check(lib().rbe_calibrate(int(kind), int(reps), C.byref(r)))
    return r.value


# -- conveniences ------------------------------------------------------------------

def to_device(a, ctx, dtype=None):
    torch = _torch()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or _dtype(ctx), device="cuda").contiguous()
