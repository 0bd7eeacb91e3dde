"""FP64 CPU oracle of the approximate Kappa sampler (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never does, and this package imports
nothing from the product.  See kappa_oracle.c for the method and citations.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

MODE_FP64 = 0
MODE_FP32 = 1
MODE_FP32_NOTAIL = 2

SIDE_LOW = 0
SIDE_HIGH = 1

# Indices of the parameter block returned by params().
PARAM_NAMES = ("kstar", "a", "b", "c", "b_over_c", "da", "db", "dc", "lnbeta")

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # A test may point the oracle at a deliberately mutated build of itself.
    path = os.environ.get("KAPPA_ORACLE_LIB", LIB)
    if path == LIB and not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    ip = ctypes.POINTER(ctypes.c_int)
    c_u64, c_u32, c_d, c_int = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_philox_blocks.argtypes = [c_u64, c_u64, c_u64, c_u32, c_u32, u32p]
    lib.oracle_philox_blocks.restype = None
    lib.oracle_digamma.argtypes = [c_d]
    lib.oracle_digamma.restype = c_d
    lib.oracle_params.argtypes = [c_d, dp]
    lib.oracle_params.restype = None
    lib.oracle_speed_uniform.argtypes = [c_int, c_u32, c_u32, ip, dp]
    lib.oracle_speed_uniform.restype = c_int
    lib.oracle_speed.argtypes = [c_d, c_int, c_d]
    lib.oracle_speed.restype = c_d
    lib.oracle_G.argtypes = [c_d, c_d, dp, dp]
    lib.oracle_G.restype = None
    lib.oracle_g_pdf.argtypes = [c_d, c_d]
    lib.oracle_g_pdf.restype = c_d
    lib.oracle_sample.argtypes = [c_d, c_d, dp, c_u64, c_u64, c_u64, c_u32, c_int, dp, dp, dp]
    lib.oracle_sample.restype = c_u64
    lib.oracle_sample_indices.argtypes = [c_d, c_d, dp, u64p, c_u64, c_u64, c_u32, c_int, dp, dp, dp]
    lib.oracle_sample_indices.restype = None
    lib.oracle_positions.argtypes = [dp, dp, c_u64, c_u64, c_u64, c_u32, c_int, dp, dp, dp]
    lib.oracle_positions.restype = None
    lib.oracle_position_coord.argtypes = [c_d, c_d, c_u32, c_int]
    lib.oracle_position_coord.restype = c_d
    lib.oracle_backward.argtypes = [c_d, c_d, c_u64, c_u64, c_u64, c_u32, c_int, fp, fp, fp, dp]
    lib.oracle_backward.restype = None
    lib.oracle_find_tails.argtypes = [c_u64, c_u64, c_u64, c_u32, u64p, c_u64]
    lib.oracle_find_tails.restype = c_u64
    lib.oracle_dot.argtypes = [c_d, c_d, c_u64, c_u64, c_u64, c_u32, c_int, fp, fp, fp]
    lib.oracle_dot.restype = c_d
    lib.oracle_speed_histogram_f32.argtypes = [fp, fp, fp, c_u64, c_d, c_d, c_u32, u64p]
    lib.oracle_speed_histogram_f32.restype = None
    lib.oracle_speed_histogram_f64.argtypes = [dp, dp, dp, c_u64, c_d, c_d, c_u32, u64p]
    lib.oracle_speed_histogram_f64.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = c_int
    lib.oracle_set_num_threads.argtypes = [c_int]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox(ctr, key):
    """One Philox4x32-10 block: ctr (4 words), key (2 words) -> 4 words."""
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def philox_blocks(n, seed, counter_offset=0, seg=0, draw=0):
    """Blocks for particles counter_offset..+n-1: array (n, 4) of uint32."""
    lib = _load()
    out = np.zeros((n, 4), dtype=np.uint32)
    lib.oracle_philox_blocks(n, seed, counter_offset, seg, draw, _ptr(out, ctypes.c_uint32))
    return out


def digamma(x):
    return _load().oracle_digamma(float(x))


def params(kappa):
    """Setup block of Table 1 plus kappa-derivatives, as a dict."""
    p = np.zeros(len(PARAM_NAMES), dtype=np.float64)
    _load().oracle_params(float(kappa), _ptr(p, ctypes.c_double))
    return dict(zip(PARAM_NAMES, p.tolist()))


def speed_uniform(mode, r0, r3):
    """(tail_taken, side, small uniform) for words r0, r3 in the given mode."""
    side = ctypes.c_int(0)
    u = ctypes.c_double(0.0)
    tail = _load().oracle_speed_uniform(mode, int(r0), int(r3), ctypes.byref(side), ctypes.byref(u))
    return bool(tail), side.value, u.value


def speed(kappa, side, u):
    """V/theta at U1 = u (side low) or 1 - U1 = u (side high)."""
    return _load().oracle_speed(float(kappa), int(side), float(u))


def G(kappa, x):
    """(G(x), 1 - G(x)) of the approximate CDF."""
    g = ctypes.c_double(0.0)
    h = ctypes.c_double(0.0)
    _load().oracle_G(float(kappa), float(x), ctypes.byref(g), ctypes.byref(h))
    return g.value, h.value


def g_pdf(kappa, x):
    return _load().oracle_g_pdf(float(kappa), float(x))


def sample(kappa, theta, n, seed, counter_offset=0, seg=0, mode=MODE_FP64, drift=None):
    """(vx, vy, vz, tails) for particles counter_offset..+n-1 of segment seg (FP64 arrays)."""
    lib = _load()
    vx = np.empty(n, dtype=np.float64)
    vy = np.empty(n, dtype=np.float64)
    vz = np.empty(n, dtype=np.float64)
    d = None if drift is None else np.ascontiguousarray(drift, dtype=np.float64)
    dptr = None if d is None else _ptr(d, ctypes.c_double)
    tails = lib.oracle_sample(float(kappa), float(theta), dptr, n, seed, counter_offset, seg, mode,
                              _ptr(vx, ctypes.c_double), _ptr(vy, ctypes.c_double), _ptr(vz, ctypes.c_double))
    return vx, vy, vz, int(tails)


def positions(lo, size, n, seed, counter_offset=0, seg=0, mode=MODE_FP64):
    """(px, py, pz): particles counter_offset..+n-1 of segment seg placed
    uniformly in the box [lo, lo + size) (draw 1 of the counter)."""
    lib = _load()
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    size = np.ascontiguousarray(size, dtype=np.float64)
    out = [np.empty(n, dtype=np.float64) for _ in range(3)]
    lib.oracle_positions(_ptr(lo, ctypes.c_double), _ptr(size, ctypes.c_double), n, seed, counter_offset, seg,
                         mode, *(_ptr(a, ctypes.c_double) for a in out))
    return tuple(out)


def position_coord(lo, size, r, mode=MODE_FP64):
    """One coordinate of a position in the box [lo, lo + size) from the
    Philox word r (what positions() does per axis)."""
    return float(_load().oracle_position_coord(float(lo), float(size), int(r), mode))


def sample_indices(kappa, theta, idx, seed, seg=0, mode=MODE_FP64, drift=None):
    """(vx, vy, vz) at the particle indices idx (uint64 array)."""
    lib = _load()
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    m = idx.size
    vx = np.empty(m, dtype=np.float64)
    vy = np.empty(m, dtype=np.float64)
    vz = np.empty(m, dtype=np.float64)
    d = None if drift is None else np.ascontiguousarray(drift, dtype=np.float64)
    dptr = None if d is None else _ptr(d, ctypes.c_double)
    lib.oracle_sample_indices(float(kappa), float(theta), dptr, _ptr(idx, ctypes.c_uint64), m, seed, seg, mode,
                              _ptr(vx, ctypes.c_double), _ptr(vy, ctypes.c_double), _ptr(vz, ctypes.c_double))
    return vx, vy, vz


def backward(kappa, theta, n, seed, gx, gy, gz, counter_offset=0, seg=0, mode=MODE_FP64):
    """(sum g.dv/dkappa, sum g.dv/dtheta) for FP32 upstream-gradient arrays gx, gy, gz."""
    lib = _load()
    gx = np.ascontiguousarray(gx, dtype=np.float32)
    gy = np.ascontiguousarray(gy, dtype=np.float32)
    gz = np.ascontiguousarray(gz, dtype=np.float32)
    assert gx.size == n and gy.size == n and gz.size == n
    out = np.zeros(2, dtype=np.float64)
    lib.oracle_backward(float(kappa), float(theta), n, seed, counter_offset, seg, mode,
                        _ptr(gx, ctypes.c_float), _ptr(gy, ctypes.c_float), _ptr(gz, ctypes.c_float),
                        _ptr(out, ctypes.c_double))
    return float(out[0]), float(out[1])


def find_tails(n, seed, counter_offset=0, seg=0, max_out=4096):
    """Particle indices whose FP32-mode uniform takes the FP64 tail."""
    out = np.zeros(max_out, dtype=np.uint64)
    found = _load().oracle_find_tails(n, seed, counter_offset, seg, _ptr(out, ctypes.c_uint64), max_out)
    return out[:min(found, max_out)].copy()


def dot(kappa, theta, n, seed, gx, gy, gz, counter_offset=0, seg=0, mode=MODE_FP64):
    """sum_i g_i . v_i over the samples, in FP64."""
    gx = np.ascontiguousarray(gx, dtype=np.float32)
    gy = np.ascontiguousarray(gy, dtype=np.float32)
    gz = np.ascontiguousarray(gz, dtype=np.float32)
    assert gx.size == n and gy.size == n and gz.size == n
    return _load().oracle_dot(float(kappa), float(theta), n, seed, counter_offset, seg, mode,
                              _ptr(gx, ctypes.c_float), _ptr(gy, ctypes.c_float), _ptr(gz, ctypes.c_float))


def speed_histogram(vx, vy, vz, theta, bin_width, nbins, counts=None):
    """Counts of |v| per bin (nbins + 1 uint64, the last the overflow), in the
    precision of the arrays (float32 or float64)."""
    lib = _load()
    if counts is None:
        counts = np.zeros(nbins + 1, dtype=np.uint64)
    if np.asarray(vx).dtype == np.float32:
        a = [np.ascontiguousarray(v, dtype=np.float32) for v in (vx, vy, vz)]
        lib.oracle_speed_histogram_f32(*[_ptr(v, ctypes.c_float) for v in a], a[0].size, float(theta),
                                       float(bin_width), nbins, _ptr(counts, ctypes.c_uint64))
    else:
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (vx, vy, vz)]
        lib.oracle_speed_histogram_f64(*[_ptr(v, ctypes.c_double) for v in a], a[0].size, float(theta),
                                       float(bin_width), nbins, _ptr(counts, ctypes.c_uint64))
    return counts


def num_threads():
    return _load().oracle_num_threads()


def set_num_threads(n):
    _load().oracle_set_num_threads(int(n))
