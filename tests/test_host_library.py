"""Host-side checks of librbe that need no GPU: the library loads and
exports every entry point the header declares, the host-only normaliser
matches the oracle, parameter validation rejects bad input before touching a
device, and the single-precision erfc table of the real-space kernel meets
its error bound against the library erfc of scipy.

Paper: Sec. 3.1, eqs. (3.1)-(3.2) (normaliser); eq. (2.9) (erfc kernel).
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2010_01559_amd.rbe as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbe.h")
REAL_SRC = os.path.join(ROOT, "paper_2010_01559_amd", "csrc", "rbe_real.hip")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(R.LIB_PATH):
        from paper_2010_01559_amd import build
        build.build()
    return R.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(rbe_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(R.EXPORTED) == names


def test_normaliser_matches_oracle(lib):
    for alpha, L in [(1.0, 10.0), (0.5, 31.0723), (0.663332, 100.0), (0.6633, 215.443)]:
        H, S = R.rbe_normalizer(alpha, L)
        assert H == pytest.approx(O.H_direct(alpha, L), rel=1e-14)
        assert S == pytest.approx(O.S(alpha, L), rel=1e-13)


def test_normaliser_rejects_bad_input(lib):
    H, S = C.c_double(), C.c_double()
    for a, L in [(0.0, 10.0), (-1.0, 10.0), (1.0, 0.0), (float("nan"), 10.0), (1.0, float("inf"))]:
        assert lib.rbe_normalizer(a, L, C.byref(H), C.byref(S)) == R.RBE_ERR_INVALID


def _create(lib, **over):
    p = R.Params(n=100, p=10, box=10.0, alpha=1.0, r_cut=3.5)
    for k, v in over.items():
        setattr(p, k, v)
    h = C.c_void_p()
    arr = (R.rbe_params * 1)(p.to_c())
    st = lib.rbe_batch_create(arr, 1, None, C.byref(h))
    return st, h, lib.rbe_last_error(None).decode()


@pytest.mark.parametrize("over,status,word", [
    (dict(n=0), R.RBE_ERR_INVALID, "n must"),
    (dict(p=0), R.RBE_ERR_INVALID, "p must"),
    (dict(box=-1.0), R.RBE_ERR_INVALID, "box"),
    (dict(alpha=0.0), R.RBE_ERR_INVALID, "alpha"),
    (dict(r_cut=6.0), R.RBE_ERR_CUTOFF, "half the box"),
    (dict(lj_eps=1.0, lj_rcut=5.5), R.RBE_ERR_CUTOFF, "lj_rcut"),
    (dict(skin=-0.1), R.RBE_ERR_INVALID, "skin"),
    (dict(dt=float("nan")), R.RBE_ERR_INVALID, "dt"),
    (dict(precision=7), R.RBE_ERR_INVALID, "precision"),
    (dict(integrator=5), R.RBE_ERR_INVALID, "integrator"),
    (dict(sampler=9), R.RBE_ERR_INVALID, "sampler"),
    (dict(flags=1), R.RBE_ERR_INVALID, "flags"),
    (dict(alpha=1e-4), R.RBE_ERR_INVALID, "alpha L^2"),
    (dict(n_fixed=-1), R.RBE_ERR_INVALID, "n_fixed"),
    (dict(n_fixed=101), R.RBE_ERR_INVALID, "n_fixed"),
    (dict(lj_eps=1.0, lj_rcut=1.12, diameter=np.full(100, 6.0)), R.RBE_ERR_CUTOFF, "LJ reach"),
    (dict(lj_eps=1.0, lj_rcut=1.12, diameter=np.r_[np.full(99, 4.0), -1.0]), R.RBE_ERR_INVALID, "diameter[99]"),
])
def test_create_validates_before_any_device_work(lib, over, status, word):
    st, h, msg = _create(lib, **over)
    assert st == status and not h.value
    assert word in msg


def test_create_without_a_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h, msg = _create(lib)
    assert st == R.RBE_ERR_NO_DEVICE and not h.value
    assert msg


def test_null_arguments(lib):
    assert lib.rbe_batch_create(None, 1, None, None) == R.RBE_ERR_INVALID
    assert lib.rbe_sample_k(None, 0, None) == R.RBE_ERR_INVALID
    assert lib.rbe_step(None, None, None, None, None, 0, 1) == R.RBE_ERR_INVALID
    assert lib.rbe_num_systems(None) == 0
    assert lib.rbe_profile_name(-1) is None
    assert lib.rbe_profile_count() >= 10


def erfc_table():
    """The coefficients and scale of the single-precision erfc as compiled."""
    src = open(REAL_SRC).read()
    body = src[src.index("float erfc_scaled_f32"):]
    body = body[:body.index("return s * t;")]
    p = float(re.search(r"fmaf\(([0-9.e+-]+)f, x, 1\.0f\)", body).group(1))
    first = float(re.search(r"float s = ([0-9.e+-]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"s = fmaf\(s, t, ([0-9.e+-]+)f\);", body)]
    return p, [first] + rest   # highest power first


def erfc_f32(x, p, coef):
    """Emulate the kernel's evaluation with float32 rounding at every step."""
    f = np.float32
    x = np.asarray(x, f)
    t = (f(1) / (f(p) * x + f(1))).astype(f)
    s = np.full_like(x, f(coef[0]))
    for c in coef[1:]:
        s = (s * t + f(c)).astype(f)
    ex = np.exp(-(x.astype(np.float64) ** 2)).astype(f)
    return (s * t).astype(f) * ex


def test_erfc_table_error_bound():
    from scipy.special import erfc
    p, coef = erfc_table()
    assert len(coef) == 9
    x = np.linspace(0.0, 8.0, 200001)
    # the rational form in exact arithmetic: fit quality
    t = 1.0 / (1.0 + p * x)
    s = np.zeros_like(x)
    for c in coef:
        s = s * t + c
    rel = np.abs(s * t * np.exp(-x * x) - erfc(x)) / erfc(x)
    assert rel.max() < 3e-7
    # with single-precision arithmetic at every step, against erfc of the
    # same (float-rounded) argument; the exponential is taken as correctly
    # rounded here, the hardware one adds its own ulp
    xf = x.astype(np.float32).astype(np.float64)
    rel32 = np.abs(erfc_f32(xf, p, coef).astype(np.float64) - erfc(xf)) / erfc(xf)
    assert rel32.max() < 1e-6


def test_erfc_fit_reproduces_the_table():
    """fit_erfc.py regenerates the coefficients compiled into the kernel."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "fit_erfc", os.path.join(ROOT, "paper_2010_01559_amd", "csrc", "fit_erfc.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    c = m.fit()
    p, coef = erfc_table()
    assert p == m.P
    np.testing.assert_allclose(coef, c[::-1], rtol=1e-8)


def test_tile_cache_file_is_read(tmp_path):
    """The tile cache (filled by rbe_autotune, consulted at creation) reads
    its file once per process; keys are power-of-two buckets of N and P."""
    import subprocess
    import sys
    cache = tmp_path / "tiles.txt"
    cache.write_text("# arch prec n_bucket p_bucket batched rho_chunk rho_block force_split real_split\n"
                     "gfx950 0 16 6 0 392 1024 4 4\n"
                     "gfx950 0 19 8 1 256 512 2 8   # a batch\n"
                     "garbage line\n")
    code = ("import paper_2010_01559_amd.rbe as R, json; "
            "print(json.dumps([R.rbe_tune_lookup('gfx950:sramecc+:xnack-', 0, 100000, 100), "
            "R.rbe_tune_lookup('gfx950', 0, 600000, 300, 64), R.rbe_tune_lookup('gfx950', 1, 100000, 100), "
            "R.rbe_tune_lookup('gfx950', 0, 200000, 100)]))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=dict(os.environ, RBE_TUNE_CACHE=str(cache)),
                         capture_output=True, text=True, check=True).stdout
    import json
    a, b, c, d = json.loads(out.strip().splitlines()[-1])
    assert a == {"rho_chunk": 392, "rho_block": 1024, "force_split": 4, "real_split": 4}
    assert b == {"rho_chunk": 256, "rho_block": 512, "force_split": 2, "real_split": 8}
    assert c is None and d is None   # other precision; other N bucket


def committed_tile_cache():
    """Entries of the tile cache that ships beside the library."""
    rows = []
    with open(os.path.join(ROOT, "paper_2010_01559_amd", "rbe_tiles.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                assert len(line) == 9, line
                rows.append((line[0], *map(int, line[1:])))
    return rows


def test_committed_tile_cache_is_well_formed(tmp_path):
    """Every shipped entry is a shape the kernels accept (the bounds of
    rbe_set_tiles and the 64 KiB of dynamic LDS), and the default lookup
    (no RBE_TUNE_CACHE) finds the last entry of each key."""
    import json
    import subprocess
    import sys
    rows = committed_tile_cache()
    assert rows
    last = {}
    for arch, prec, nb, pb, batched, chunk, block, fsplit, rsplit in rows:
        assert arch == "gfx950" and prec in (0, 1) and batched in (0, 1)
        assert 64 <= chunk <= 2048 and chunk % 8 == 0 and block in (256, 512, 1024)
        assert fsplit in (1, 2, 4) and rsplit in (1, 2, 4, 8)
        assert 48 * chunk + 16 * block <= 65536 and 32 * (chunk + 256) + 28 * block <= 65536
        last[(prec, nb, pb, batched)] = dict(rho_chunk=chunk, rho_block=block, force_split=fsplit,
                                             real_split=rsplit)
    keys = sorted(last)
    code = ("import paper_2010_01559_amd.rbe as R, json; print(json.dumps([R.rbe_tune_lookup('gfx950', p, 2**nb, "
            "2**pb, 2 if b else 1) for p, nb, pb, b in %r]))" % (keys,))
    env = {k: v for k, v in os.environ.items() if k != "RBE_TUNE_CACHE"}
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         check=True).stdout
    got = json.loads(out.strip().splitlines()[-1])
    assert got == [last[k] for k in keys]
