"""FP64 CPU oracle for the random batch Ewald method (arXiv:2010.01559).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check of
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The product
library never imports, links or calls anything here.

The arithmetic lives in ``rbe_oracle.c`` (plain C, double precision, written
from the paper); this module compiles it with gcc on first use and exposes
thin numpy wrappers.  Positions, forces and gradients are SoA ``[3, n]``
float64 arrays; modes are ``[3, p]`` int32 arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile ``rbe_oracle.c`` into ``liboracle.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OracleSys(C.Structure):
    _fields_ = [("n", C.c_int), ("p", C.c_int), ("L", C.c_double), ("alpha", C.c_double),
                ("rc", C.c_double), ("coulomb", C.c_double), ("lj_eps", C.c_double),
                ("lj_sigma", C.c_double), ("lj_rc", C.c_double), ("kT", C.c_double),
                ("gamma", C.c_double), ("dt", C.c_double), ("mass", C.c_double),
                ("seed", C.c_uint64), ("diam", C.c_void_p), ("n_fixed", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.oracle_H_direct.restype = C.c_double
        L.oracle_H_direct.argtypes = [C.c_double, C.c_double]
        L.oracle_H_dual.restype = C.c_double
        L.oracle_H_dual.argtypes = [C.c_double, C.c_double]
        L.oracle_S.restype = C.c_double
        L.oracle_S.argtypes = [C.c_double, C.c_double]
        L.oracle_S_bruteforce.restype = C.c_double
        L.oracle_S_bruteforce.argtypes = [C.c_double, C.c_double, C.c_int]
        L.oracle_philox4x32_10.restype = None
        L.oracle_philox4x32_10.argtypes = [np.ctypeslib.ndpointer(np.uint32), np.ctypeslib.ndpointer(np.uint32),
                                           np.ctypeslib.ndpointer(np.uint32)]
        L.oracle_mode_range.restype = C.c_int
        L.oracle_mode_range.argtypes = [C.c_double, C.c_double]
        L.oracle_mode_cdf.restype = None
        L.oracle_mode_cdf.argtypes = [C.c_double, C.c_double, _dp]
        L.oracle_sample_modes.restype = C.c_int
        L.oracle_sample_modes.argtypes = [C.c_double, C.c_double, C.c_int, C.c_uint64, C.c_uint64, _ip]
        L.oracle_sample_uniforms.restype = None
        L.oracle_sample_uniforms.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.c_int, _dp]
        L.oracle_mh_proposal_mass.restype = C.c_double
        L.oracle_mh_proposal_mass.argtypes = [C.c_double, C.c_double, C.c_int]
        L.oracle_sample_modes_mh.restype = C.c_int
        L.oracle_sample_modes_mh.argtypes = [C.c_double, C.c_double, C.c_int, C.c_uint64, C.c_uint64, _ip, _ip,
                                             C.c_int]
        L.oracle_rho.restype = None
        L.oracle_rho.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, _ip, _dp, _dp]
        L.oracle_kspace_force.restype = None
        L.oracle_kspace_force.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, _ip, _dp, C.c_double, _dp]
        L.oracle_kspace_force_subset.restype = None
        L.oracle_kspace_force_subset.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, _ip, _dp, C.c_double,
                                                 C.c_int, _ip, _dp]
        L.oracle_kspace_energy.restype = C.c_double
        L.oracle_kspace_energy.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, _ip, _dp, C.c_double]
        L.oracle_self_energy.restype = C.c_double
        L.oracle_self_energy.argtypes = [C.c_int, _dp, C.c_double, C.c_double]
        L.oracle_rbe_weights.restype = None
        L.oracle_rbe_weights.argtypes = [C.c_double, C.c_double, C.c_int, _dp]
        L.oracle_ewald_modes.restype = C.c_int
        L.oracle_ewald_modes.argtypes = [C.c_double, C.c_double, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
        L.oracle_real_force.restype = None
        L.oracle_real_force.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_double, C.c_int, C.c_void_p, _dp,
                                        C.c_void_p, C.c_void_p]
        L.oracle_real_force_ex.restype = None
        L.oracle_real_force_ex.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_int, C.c_int,
                                           C.c_void_p, _dp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_rbe_force_variance.restype = None
        L.oracle_rbe_force_variance.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_double,
                                                C.c_int, _ip, _dp, C.c_int, _ip, _dp]
        L.oracle_langevin_normals.restype = None
        L.oracle_langevin_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_int, _dp]
        L.oracle_total_force.restype = None
        L.oracle_total_force.argtypes = [C.POINTER(OracleSys), _dp, _dp, C.c_uint64, _dp]
        L.oracle_baoab_step.restype = None
        L.oracle_baoab_step.argtypes = [C.POINTER(OracleSys), _dp, _dp, _dp, _dp, C.c_uint64]
        L.oracle_leapfrog_andersen_step.restype = None
        L.oracle_leapfrog_andersen_step.argtypes = [C.POINTER(OracleSys), C.c_double, _dp, _dp, _dp, _dp,
                                                    C.c_uint64]
        L.oracle_forces_vjp.restype = None
        L.oracle_forces_vjp.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_double, C.c_int, _ip, _dp, _dp, C.c_double,
                                        C.c_int, _dp, _dp]
        L.oracle_kinetic_energy.restype = C.c_double
        L.oracle_kinetic_energy.argtypes = [C.c_int, _dp, C.c_double]
        L.oracle_pair_virial.restype = None
        L.oracle_pair_virial.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]
        L.oracle_kspace_virial.restype = C.c_double
        L.oracle_kspace_virial.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_int, _ip, _dp,
                                           C.c_double]
        L.oracle_set_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_pair_histogram.restype = None
        L.oracle_pair_histogram.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_int,
                                            np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")]
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# -- normaliser ---------------------------------------------------------------

def H_direct(alpha, L):
    return lib().oracle_H_direct(alpha, L)


def H_dual(alpha, L):
    return lib().oracle_H_dual(alpha, L)


def S(alpha, L):
    return lib().oracle_S(alpha, L)


def S_bruteforce(alpha, L, mmax):
    return lib().oracle_S_bruteforce(alpha, L, mmax)


# -- random numbers and sampling ---------------------------------------------

def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(np.ascontiguousarray(ctr, np.uint32), np.ascontiguousarray(key, np.uint32), out)
    return out


def mode_range(alpha, L):
    return lib().oracle_mode_range(alpha, L)


def mode_cdf(alpha, L):
    M = mode_range(alpha, L)
    out = np.zeros(2 * M + 1)
    lib().oracle_mode_cdf(alpha, L, out)
    return out


def sample_modes(alpha, L, p, seed, step):
    m = np.zeros((3, p), np.int32)
    rej = lib().oracle_sample_modes(alpha, L, p, seed, step, m)
    return m, rej


def sample_uniforms(seed, step, l, attempt=0):
    u = np.zeros(3)
    lib().oracle_sample_uniforms(seed, step, l, attempt, u)
    return u


def mh_proposal_mass(alpha, L, m):
    return lib().oracle_mh_proposal_mass(alpha, L, int(m))


def sample_modes_mh(alpha, L, p, seed, step, state=None, skip_accept=False):
    st = np.zeros(3, np.int32) if state is None else _i32(state).copy()
    m = np.zeros((3, p), np.int32)
    acc = lib().oracle_sample_modes_mh(alpha, L, p, seed, step, st, m, int(skip_accept))
    return m, st, acc


# -- Fourier space -------------------------------------------------------------

def rho(pos, q, L, modes):
    pos, q, modes = _f64(pos), _f64(q), _i32(modes)
    n, nm = q.shape[0], modes.shape[1]
    re, im = np.zeros(nm), np.zeros(nm)
    lib().oracle_rho(n, pos, q, L, nm, modes, re, im)
    return re, im


def rbe_weights(alpha, L, p):
    w = np.zeros(p)
    lib().oracle_rbe_weights(alpha, L, p, w)
    return w


def kspace_force(pos, q, L, modes, weight, coulomb=1.0):
    pos, q, modes, weight = _f64(pos), _f64(q), _i32(modes), _f64(weight)
    n, nm = q.shape[0], modes.shape[1]
    F = np.zeros((3, n))
    lib().oracle_kspace_force(n, pos, q, L, nm, modes, weight, coulomb, F)
    return F


def kspace_force_subset(pos, q, L, modes, weight, idx, coulomb=1.0):
    pos, q, modes, weight, idx = _f64(pos), _f64(q), _i32(modes), _f64(weight), _i32(idx)
    F = np.zeros((3, idx.shape[0]))
    lib().oracle_kspace_force_subset(q.shape[0], pos, q, L, modes.shape[1], modes, weight, coulomb, idx.shape[0],
                                     idx, F)
    return F


def kspace_energy(pos, q, L, modes, weight, coulomb=1.0):
    pos, q, modes, weight = _f64(pos), _f64(q), _i32(modes), _f64(weight)
    return lib().oracle_kspace_energy(q.shape[0], pos, q, L, modes.shape[1], modes, weight, coulomb)


def self_energy(q, alpha, coulomb=1.0):
    q = _f64(q)
    return lib().oracle_self_energy(q.shape[0], q, alpha, coulomb)


def rbe_kspace_force(pos, q, L, alpha, modes, coulomb=1.0):
    return kspace_force(pos, q, L, modes, rbe_weights(alpha, L, modes.shape[1]), coulomb)


def ewald_modes(alpha, L, mmax2):
    cnt = lib().oracle_ewald_modes(alpha, L, mmax2, None, None, 0)
    m = np.zeros((3, cnt), np.int32)
    w = np.zeros(cnt)
    lib().oracle_ewald_modes(alpha, L, mmax2, m.ctypes.data, w.ctypes.data, cnt)
    return m, w


# -- real space ------------------------------------------------------------------

def real_force(pos, q, L, alpha, rc, coulomb=1.0, lj=(0.0, 1.0, 2.5), idx=None, diam=None, cells=False,
               virial=False):
    """Real-space Coulomb + shifted LJ (eq. 2.11 second term, eq. 4.1).

    Returns (F [3,nsub], e_real [nsub], e_lj [nsub]) -- half pair energies per
    listed particle -- plus the half pair virials [nsub] when ``virial``.
    ``diam``: per-particle diameters (r_off = (d_i + d_j)/2 - sigma), or None.
    ``cells``: use the linked-cell list instead of the direct sum (same
    result up to summation order when three or more cells fit).
    """
    pos, q = _f64(pos), _f64(q)
    n = q.shape[0]
    if idx is None:
        nsub, ip = n, None
    else:
        idx = _i32(idx)
        nsub, ip = idx.shape[0], idx.ctypes.data
    dp = None
    if diam is not None:
        diam = _f64(diam)
        assert diam.shape == (n,)
        dp = diam.ctypes.data
    F = np.zeros((3, nsub))
    er, el, vr = np.zeros(nsub), np.zeros(nsub), np.zeros(nsub)
    lib().oracle_real_force_ex(n, pos, q, L, alpha, rc, coulomb, lj[0], lj[1], lj[2], dp, 1 if cells else 0,
                               nsub, ip, F, er.ctypes.data, el.ctypes.data, vr.ctypes.data)
    return (F, er, el, vr) if virial else (F, er, el)


def rbe_force_variance(pos, q, L, alpha, p, ewald_mmax2, idx, coulomb=1.0):
    pos, q, idx = _f64(pos), _f64(q), _i32(idx)
    m, w = ewald_modes(alpha, L, ewald_mmax2)
    var = np.zeros(idx.shape[0])
    lib().oracle_rbe_force_variance(q.shape[0], pos, q, L, alpha, p, coulomb, m.shape[1], m, w, idx.shape[0],
                                    idx, var)
    return var


# -- dynamics ---------------------------------------------------------------------

def make_sys(n, p, L, alpha, rc, coulomb=1.0, lj=(0.0, 1.0, 2.5), kT=1.0, gamma=1.0, dt=1e-3, mass=1.0,
             seed=0, diam=None, n_fixed=0):
    """Oracle system; ``diam`` (per-particle diameters) is kept alive on the
    returned structure."""
    s = OracleSys(n, p, L, alpha, rc, coulomb, lj[0], lj[1], lj[2], kT, gamma, dt, mass, seed, None, n_fixed)
    if diam is not None:
        s._diam = _f64(diam)
        assert s._diam.shape == (n,)
        s.diam = s._diam.ctypes.data
    return s


def langevin_normals(seed, step, i):
    xi = np.zeros(3)
    lib().oracle_langevin_normals(seed, step, i, xi)
    return xi


def total_force(sys, pos, q, step):
    F = np.zeros((3, sys.n))
    lib().oracle_total_force(C.byref(sys), _f64(pos), _f64(q), step, F)
    return F


def baoab_step(sys, pos, vel, q, F, step):
    """Advances pos, vel, F in place (float64 contiguous arrays)."""
    lib().oracle_baoab_step(C.byref(sys), pos, vel, _f64(q), F, step)


def leapfrog_andersen_step(sys, nu, pos, vel, q, F, step):
    lib().oracle_leapfrog_andersen_step(C.byref(sys), nu, pos, vel, _f64(q), F, step)


def forces_vjp(pos, q, L, alpha, rc, modes, weight, gF, coulomb=1.0, lj=(0.0, 1.0, 2.5), gE=0.0, parts=3):
    """dLoss/dq [n], dLoss/dr [3,n] of a loss of the forces (and energy)."""
    pos, q, modes, weight, gF = _f64(pos), _f64(q), _i32(modes), _f64(weight), _f64(gF)
    n = q.shape[0]
    gq, gr = np.zeros(n), np.zeros((3, n))
    lib().oracle_forces_vjp(n, pos, q, L, alpha, rc, coulomb, lj[0], lj[1], lj[2], modes.shape[1], modes,
                            weight, gF, gE, parts, gq, gr)
    return gq, gr


def kinetic_energy(vel, mass=1.0):
    vel = _f64(vel)
    return lib().oracle_kinetic_energy(vel.shape[1], vel, mass)


# -- observables (Sec. 4.1, eq. 4.3; charge-charge correlation) --------------------

def pair_virial(pos, q, L, alpha, rc, coulomb=1.0, lj=(0.0, 1.0, 2.5)):
    """(real-space Coulomb, LJ) sums over unordered pairs of r_ij . F_ij."""
    wr, wl = C.c_double(), C.c_double()
    lib().oracle_pair_virial(_f64(q).shape[0], _f64(pos), _f64(q), L, alpha, rc, coulomb, lj[0], lj[1], lj[2],
                             C.byref(wr), C.byref(wl))
    return wr.value, wl.value


def kspace_virial(pos, q, L, alpha, modes, weight, coulomb=1.0):
    """Fourier part of the pair sum of r_ij . F_ij for a weighted mode list."""
    pos, q, modes, weight = _f64(pos), _f64(q), _i32(modes), _f64(weight)
    return lib().oracle_kspace_virial(q.shape[0], pos, q, L, alpha, modes.shape[1], modes, weight, coulomb)


def pair_histogram(pos, q, L, r_max, nbins):
    """[3, nbins] int64 counts of pairs i < j by bin and class (++, +-, --)."""
    counts = np.zeros((3, nbins), np.int64)
    lib().oracle_pair_histogram(_f64(q).shape[0], _f64(pos), _f64(q), L, r_max, nbins, counts)
    return counts


def set_threads(n):
    """OpenMP threads of the oracle's loops (n <= 0 leaves them); returns the count."""
    return lib().oracle_set_threads(int(n))
