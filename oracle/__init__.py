"""CPU oracle for compressed out-of-core stencil sweeps.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
(`paper_2204_11315_amd`) never imports it and shares no code with it; the C
sources here are compiled with gcc into their own shared object.

What each function follows (Shen et al., "Compression-Based Optimizations for
Out-of-Core GPU Stencil Computation"):

* `star7_run`, `star7_grad`   -- the stencil update of Sec. 3.1 (7-point star,
  zero ghosts) and its adjoint; plain definitions in FP64.
* `wave25_run`                -- the 25-point acoustic-wave update of the Sec. 6
  workload (Table 1: halo 4), FP64.
* `compress` / `decompress`   -- the fixed-rate block codec (Sec. 4.2, Sec. 5:
  fixed user-specified rate); format defined step by step in codec_ref.c.
* `compressed_sweeps`         -- the compressed out-of-core path as a
  composition: the data lives compressed on the host, each residency decodes,
  runs k steps and encodes again (Sec. 1, Sec. 4.2, Algorithm 1).  The slab
  decomposition does not enter: blocks are coded independently and halos are
  whole blocks.  Pinned by the closed form of block-constant fields under a
  diagonal-only stencil (exact codec, one FP32 rounding per residency).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = ["codec_ref.c", "stencil_ref.c", "wave_ref.c"]
_LIB_PATH = os.path.join(_HERE, "_build", "libocref.so")
_lock = threading.Lock()
_lib = None

OK, ERR_ARG, ERR_SHAPE, ERR_NONFINITE = 0, -1, -2, -5


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp] + [os.path.join(_HERE, s) for s in _SRCS] + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        newest = max(os.path.getmtime(os.path.join(_HERE, s)) for s in _SRCS + ["ocref.h"])
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        sig = {
            "ocref_star7_step": (None, [P, P, I64, I64, I64, P, P]),
            "ocref_star7_step_T": (None, [P, P, I64, I64, I64, P, P]),
            "ocref_star7_run": (ctypes.c_int, [P, I64, I64, I64, P, P, I64]),
            "ocref_star7_grad": (ctypes.c_int, [P, I64, I64, I64, P, P, I64, P, P, P, P]),
            "ocref_wave25_run": (ctypes.c_int, [P, P, P, I64, I64, I64, D, D, P, D, D, I64, I64]),
            "ocref_ricker": (D, [D, D, D]),
            "ocref_block_encode": (ctypes.c_int, [P, ctypes.c_int, P, P]),
            "ocref_block_decode": (ctypes.c_int, [P, ctypes.c_int, P]),
            "ocref_compress": (ctypes.c_int, [P, I64, I64, I64, ctypes.c_int, P]),
            "ocref_decompress": (ctypes.c_int, [P, I64, I64, I64, ctypes.c_int, P]),
            "ocref_fwd_xform": (None, [P]),
            "ocref_inv_xform": (None, [P]),
            "ocref_fwd_lift_line": (None, [P]),
            "ocref_inv_lift_line": (None, [P]),
            "ocref_to_negabinary": (ctypes.c_uint32, [ctypes.c_int32]),
            "ocref_from_negabinary": (ctypes.c_int32, [ctypes.c_uint32]),
            "ocref_unread_mean": (ctypes.c_int32, [ctypes.c_int]),
            "ocref_sequency_order": (None, [P]),
            "ocref_quantize": (ctypes.c_int, [P, P, P]),
            "ocref_set_threads": (ctypes.c_int, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def set_threads(n: int) -> int:
    """Set the host threads of the oracle's OpenMP loops (calling thread);
    returns the previous count.  For timing the oracle on fewer cores."""
    return int(_load().ocref_set_threads(int(n)))


def _check(st: int, what: str):
    if st != OK:
        raise OracleError("%s failed with status %d" % (what, st))


def _coeffs(c) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    if c.shape != (7,):
        raise ValueError("c must hold 7 coefficients: c0, c-x, c+x, c-y, c+y, c-z, c+z")
    return c


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---- stencil (Sec. 3.1) ---------------------------------------------------
def star7_step(u, c, c0f=None, transpose=False) -> np.ndarray:
    """One application of A (or A^T) to a [nz][ny][nx] field, FP64."""
    lib = _load()
    u = _f64(u)
    nz, ny, nx = u.shape
    out = np.empty_like(u)
    cc = _coeffs(c)
    c0 = None if c0f is None else _f64(c0f)
    fn = lib.ocref_star7_step_T if transpose else lib.ocref_star7_step
    fn(_ptr(u), _ptr(out), nx, ny, nz, _ptr(cc), None if c0 is None else _ptr(c0))
    return out


def star7_run(u0, c, steps: int, c0f=None) -> np.ndarray:
    """u_T = A^steps u0 in FP64 (inputs promoted)."""
    lib = _load()
    u = _f64(u0).copy()
    nz, ny, nx = u.shape
    cc = _coeffs(c)
    c0 = None if c0f is None else _f64(c0f)
    _check(lib.ocref_star7_run(_ptr(u), nx, ny, nz, _ptr(cc), None if c0 is None else _ptr(c0),
                               int(steps)), "star7_run")
    return u


def star7_grad(u0, c, steps: int, c0f=None):
    """(L, u_T, dL/du0, dL/dc0) for L = 1/2 sum_{top plane} u_T^2, FP64."""
    lib = _load()
    u = _f64(u0)
    nz, ny, nx = u.shape
    cc = _coeffs(c)
    c0 = None if c0f is None else _f64(c0f)
    uT, gu, gc = np.empty_like(u), np.empty_like(u), np.empty_like(u)
    loss = np.zeros(1)
    _check(lib.ocref_star7_grad(_ptr(u), nx, ny, nz, _ptr(cc), None if c0 is None else _ptr(c0),
                                int(steps), _ptr(uT), _ptr(gu), _ptr(gc), _ptr(loss)),
           "star7_grad")
    return float(loss[0]), uT, gu, gc


# ---- acoustic wave (Sec. 6 workload) -------------------------------------
def ricker(t: float, f_peak: float, t0: float) -> float:
    return _load().ocref_ricker(float(t), float(f_peak), float(t0))


def wave25_run(p_prev, p_cur, vel, h, dt, src, f_peak, t0, n0: int, steps: int):
    """Advance (p^{n0-1}, p^{n0}) by `steps` steps; returns the new pair."""
    lib = _load()
    pp, pc, v = _f64(p_prev).copy(), _f64(p_cur).copy(), _f64(vel)
    nz, ny, nx = pc.shape
    s = np.ascontiguousarray(np.asarray(src, dtype=np.int64))
    _check(lib.ocref_wave25_run(_ptr(pp), _ptr(pc), _ptr(v), nx, ny, nz, float(h), float(dt),
                                _ptr(s), float(f_peak), float(t0), int(n0), int(steps)),
           "wave25_run")
    return pp, pc


# ---- codec (fixed rate) --------------------------------------------------
def codec_bytes(nx: int, ny: int, nz: int, R: int) -> int:
    return (nx // 4) * (ny // 4) * (nz // 4) * 8 * R


def compress(f, R: int) -> np.ndarray:
    lib = _load()
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float32))
    nz, ny, nx = f.shape
    out = np.zeros(codec_bytes(nx, ny, nz, R), dtype=np.uint8)
    _check(lib.ocref_compress(_ptr(f), nx, ny, nz, int(R), _ptr(out)), "compress")
    return out


def decompress(buf, shape, R: int) -> np.ndarray:
    lib = _load()
    nz, ny, nx = shape
    buf = np.ascontiguousarray(np.asarray(buf, dtype=np.uint8))
    if buf.size < codec_bytes(nx, ny, nz, R):
        raise ValueError("compressed buffer too small")
    f = np.empty((nz, ny, nx), dtype=np.float32)
    _check(lib.ocref_decompress(_ptr(buf), nx, ny, nz, int(R), _ptr(f)), "decompress")
    return f


def block_encode(v, R: int):
    """Encode one block of 64 FP32 values; returns (slot bytes, full stream bits)."""
    lib = _load()
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float32).reshape(64))
    slot = np.zeros(8 * R, dtype=np.uint8)
    nbits = np.zeros(1, dtype=np.int64)
    _check(lib.ocref_block_encode(_ptr(v), int(R), _ptr(slot), _ptr(nbits)), "block_encode")
    return slot, int(nbits[0])


def block_decode(slot, R: int) -> np.ndarray:
    lib = _load()
    slot = np.ascontiguousarray(np.asarray(slot, dtype=np.uint8))
    v = np.empty(64, dtype=np.float32)
    _check(lib.ocref_block_decode(_ptr(slot), int(R), _ptr(v)), "block_decode")
    return v


def fwd_xform(q) -> np.ndarray:
    q = np.ascontiguousarray(np.asarray(q, dtype=np.int32).reshape(64)).copy()
    _load().ocref_fwd_xform(_ptr(q))
    return q


def inv_xform(q) -> np.ndarray:
    q = np.ascontiguousarray(np.asarray(q, dtype=np.int32).reshape(64)).copy()
    _load().ocref_inv_xform(_ptr(q))
    return q


def fwd_lift_line(x) -> np.ndarray:
    """The transform of one line of four integers (step 4, one axis)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(4)).copy()
    _load().ocref_fwd_lift_line(_ptr(x))
    return x


def inv_lift_line(x) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(4)).copy()
    _load().ocref_inv_lift_line(_ptr(x))
    return x


def to_negabinary(c: int) -> int:
    return int(_load().ocref_to_negabinary(int(c)))


def from_negabinary(u: int) -> int:
    return int(_load().ocref_from_negabinary(int(u)))


def unread_mean(d: int) -> int:
    """Value added at decode to a significant coefficient with d unread digits."""
    return int(_load().ocref_unread_mean(int(d)))


def sequency_order() -> np.ndarray:
    perm = np.zeros(64, dtype=np.int32)
    _load().ocref_sequency_order(_ptr(perm))
    return perm


def quantize(v):
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float32).reshape(64))
    q = np.zeros(64, dtype=np.int32)
    eb = np.zeros(1, dtype=np.int32)
    _check(_load().ocref_quantize(_ptr(v), _ptr(q), _ptr(eb)), "quantize")
    return q, int(eb[0])


# ---- compressed out-of-core path as a composition ------------------------
def compressed_sweeps(u0, c, steps: int, k: int, R: int, c0f=None, load_rate: int = 0) -> np.ndarray:
    """Dec(Enc(S^{k_last} ... Dec(Enc(S^k(Dec(Enc(u0))))))) with S = FP64 stencil.

    The host holds the field compressed: loading encodes the FP32 input (at
    `load_rate` when it is set, else at R); every residency decodes the codes
    it finds (the first one at the load rate), runs k steps (the last one runs
    steps mod k when k does not divide steps), and encodes its FP32-rounded
    result at R; storing decodes the last codes at their rate.
    """
    u0 = np.ascontiguousarray(np.asarray(u0, dtype=np.float32))
    shape = u0.shape
    rate = load_rate if load_rate else R
    buf = compress(u0, rate)
    done = 0
    while done < steps:
        s = min(k, steps - done)
        u = decompress(buf, shape, rate)
        u = star7_run(u, c, s, c0f)
        rate = R
        buf = compress(u.astype(np.float32), rate)
        done += s
    return decompress(buf, shape, rate)
