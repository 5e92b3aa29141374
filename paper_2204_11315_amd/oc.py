"""ctypes binding of the C ABI in include/oc.h (argument marshalling only).

Every step of the compute path runs in the HIP library `liboc.so`; torch is
used only to own device memory (the arena), pinned host memory (the host
levels) and streams.  If the library has not been built, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
import warnings

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboc.so")

OC_OK, OC_ERR_ARG, OC_ERR_SHAPE, OC_ERR_BUDGET = 0, -1, -2, -3
OC_ERR_HIP, OC_ERR_NONFINITE, OC_ERR_STATE, OC_ERR_UNSUPPORTED, OC_ERR_HOST = -4, -5, -6, -7, -8
OC_ERR_TOO_LARGE = -9
OC_STAR7, OC_WAVE25 = 1, 2

C_CONFIG1 = (0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1)


class OCError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str = ""):
        self.status = status
        super().__init__("%s failed: %s (%d)%s" % (what, msg, status, ""))


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Stencil(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c", ctypes.c_float * 7), ("c0_is_field", ctypes.c_int32),
                ("h", ctypes.c_float), ("dt", ctypes.c_float), ("src", ctypes.c_int64 * 3),
                ("f_peak", ctypes.c_float), ("t0", ctypes.c_float)]


class Config(ctypes.Structure):
    _fields_ = [("dev_arena", ctypes.c_void_p), ("dev_budget", ctypes.c_size_t),
                ("streams", ctypes.c_void_p * 3), ("host_level", ctypes.c_void_p * 2),
                ("host_level_bytes", ctypes.c_size_t), ("host_aux", ctypes.c_void_p),
                ("host_aux_bytes", ctypes.c_size_t), ("k", ctypes.c_int32),
                ("slab_planes", ctypes.c_int32), ("rate_bits", ctypes.c_int32),
                ("single_buffer", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("ring_slots", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("fuse_steps", ctypes.c_int32), ("copy_back", ctypes.c_int32),
                ("share_overlap", ctypes.c_int32), ("in_place", ctypes.c_int32),
                ("error_budget", ctypes.c_float), ("error_steps", ctypes.c_int32),
                ("fused_codec", ctypes.c_int32), ("load_rate_bits", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("gcell_per_s", ctypes.c_double),
                ("bytes_h2d", ctypes.c_uint64), ("bytes_d2h", ctypes.c_uint64),
                ("peak_dev_bytes", ctypes.c_uint64), ("slab_visits", ctypes.c_uint64),
                ("slab_planes", ctypes.c_int64), ("halo_planes", ctypes.c_int64),
                ("n_slabs", ctypes.c_int64), ("n_ops", ctypes.c_uint64),
                ("ms_decode", ctypes.c_double), ("ms_stencil", ctypes.c_double),
                ("ms_encode", ctypes.c_double), ("ms_h2d", ctypes.c_double),
                ("ms_d2h", ctypes.c_double), ("n_decode", ctypes.c_uint64),
                ("n_stencil", ctypes.c_uint64), ("n_encode", ctypes.c_uint64),
                ("n_h2d", ctypes.c_uint64), ("n_d2h", ctypes.c_uint64),
                ("cells_stencil", ctypes.c_uint64), ("bytes_stencil", ctypes.c_uint64),
                ("blocks_decode", ctypes.c_uint64),
                ("blocks_encode", ctypes.c_uint64),
                ("host_ms_kernels", ctypes.c_double), ("host_ms_copies", ctypes.c_double),
                ("host_ms_events", ctypes.c_double), ("host_ms_sync", ctypes.c_double),
                ("rate_bits", ctypes.c_int64), ("pilot_rel_l2", ctypes.c_double),
                ("pilot_planes", ctypes.c_int64), ("pilot_runs", ctypes.c_int64),
                ("ms_fused", ctypes.c_double), ("n_fused", ctypes.c_uint64)]


_lock = threading.Lock()
_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_SIGS = {
    "oc_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "oc_host_level_bytes": (_SZ, [_P, _P, _I32]),
    "oc_host_aux_bytes": (_SZ, [_P, _P, _I32]),
    "oc_plan_bytes": (_SZ, [_P, _P, _P]),
    "oc_create": (ctypes.c_int, [_P, _P, _P, _P]),
    "oc_load": (ctypes.c_int, [_P, _P, _P, _P]),
    "oc_run": (ctypes.c_int, [_P, _I64]),
    "oc_store": (ctypes.c_int, [_P, _P, _P]),
    "oc_stats_get": (ctypes.c_int, [_P, _P]),
    "oc_destroy": (ctypes.c_int, [_P]),
    "oc_codec_bytes": (_SZ, [_I64, _I64, _I64, _I32]),
    "oc_codec_compress": (ctypes.c_int, [_P, _I64, _I64, _I64, _I32, _P, _SZ, _P]),
    "oc_codec_decompress": (ctypes.c_int, [_P, _I64, _I64, _I64, _I32, _P, _P]),
    "oc_codec_status": (ctypes.c_int, [_P]),
    "oc_codec_error_work_bytes": (_SZ, [_I64, _I64, _I64, _I32]),
    "oc_codec_error": (ctypes.c_int, [_P, _I64, _I64, _I64, _I32, _P, _SZ, _P, _P]),
    "oc_codec_error_noalloc": (ctypes.c_int, [_P, _I64, _I64, _I64, _I32, _P, _P]),
    "oc_star7_incore": (ctypes.c_int, [_P, _P, _P, _I64, _I64, _I64, _P, _P, _I64, _P]),
    "oc_wave25_incore": (ctypes.c_int, [_P, _P, _P, _P, _I64, _I64, _I64, _P, _I64, _I64, _P]),
    "oc_debug_fail_after": (ctypes.c_int, [_P, _I64]),
    "oc_set_timing": (ctypes.c_int, [_P, _I32]),
    "oc_adjoint_host_bytes": (_SZ, [_P, _I64, _I32, _I32]),
    "oc_forward_ckpt": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _SZ]),
    "oc_adjoint": (ctypes.c_int, [_P, _P, _P, _P]),
    "oc_debug_check_adjoint": (_I64, [_P, _P, _P, _I64, _I32, _I32, _I32, _I64]),
    "oc_debug_check_plan": (_I64, [_P, _P, _P, _I64, _I32, _I64]),
    "oc_debug_serialize": (_I32, [_P, _I32]),
    "oc_debug_check_plan_ckpt": (_I64, [_P, _P, _P, _I64, _I32, _I32, _I64]),
    "oc_debug_plan_ops": (_I64, [_P, _P, _P, _I64, _P]),
    "oc_debug_plan_dump": (_I64, [_P, _P, _P, _I64, ctypes.c_char_p, _SZ]),
    "oc_debug_timeline": (_I64, [_P, _P, _P, _P, _P, _I64]),
    "oc_debug_copy_to_host": (ctypes.c_int, [_P, _SZ, _P, _SZ, _I32, _P]),
    "oc_debug_codec_star7": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, _I64, _I64, _I64, _I64, _I32, _I32,
                                            _P, _P]),
    "oc_stream_overlap": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
}
EXPORTED = tuple(_SIGS)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise OCError(OC_ERR_STATE, "load",
                              "HIP library %s is missing; build it with __graft_entry__.build()"
                              % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
        return _lib


def status_str(st: int) -> str:
    return lib().oc_status_str(int(st)).decode()


def _check(st: int, what: str):
    if st != OC_OK:
        raise OCError(st, what, status_str(st))


def _ref(x):
    return ctypes.cast(ctypes.byref(x), ctypes.c_void_p)


def make_grid(shape) -> Grid:
    nz, ny, nx = (int(v) for v in shape)
    return Grid(nx, ny, nz)


def make_wave25(h: float, dt: float, src, f_peak: float, t0: float) -> Stencil:
    """25-point acoustic wave: grid spacing h (m), time step dt (s), Ricker source
    at cell src = (x, y, z) with peak frequency f_peak (Hz) and delay t0 (s)."""
    st = Stencil()
    st.kind = OC_WAVE25
    st.h = float(h)
    st.dt = float(dt)
    for i, v in enumerate(src):
        st.src[i] = int(v)
    st.f_peak = float(f_peak)
    st.t0 = float(t0)
    return st


def make_star7(c=C_CONFIG1, c0_field: bool = False) -> Stencil:
    st = Stencil()
    st.kind = OC_STAR7
    for i, v in enumerate(c):
        st.c[i] = float(v)
    st.c0_is_field = 1 if c0_field else 0
    return st


# ---- planner queries (no GPU needed) --------------------------------------
def host_level_bytes(shape, stencil: Stencil, rate: int) -> int:
    g = make_grid(shape)
    return int(lib().oc_host_level_bytes(_ref(g), _ref(stencil), int(rate)))


def host_aux_bytes(shape, stencil: Stencil, rate: int) -> int:
    g = make_grid(shape)
    return int(lib().oc_host_aux_bytes(_ref(g), _ref(stencil), int(rate)))


def plan_config(k: int, slab_planes: int, rate: int, single_buffer: bool = True,
                budget: int = 0, ring_slots: int = 0, prefetch: int = 0, fuse: int = 0,
                share: bool = False, in_place: bool = False, error_budget: float = 0.0,
                error_steps: int = 0, fused_codec: bool = False, load_rate: int = 0) -> Config:
    """A Config carrying only the plan fields."""
    cfg = Config()
    cfg.k = int(k)
    cfg.slab_planes = int(slab_planes)
    cfg.rate_bits = int(rate)
    cfg.single_buffer = 1 if single_buffer else 0
    cfg.dev_budget = int(budget)
    cfg.ring_slots = int(ring_slots)
    cfg.prefetch = int(prefetch)
    cfg.fuse_steps = int(fuse)
    cfg.share_overlap = 1 if share else -1
    cfg.in_place = 1 if in_place else 0
    cfg.error_budget = float(error_budget)
    cfg.error_steps = int(error_steps)
    cfg.fused_codec = 1 if fused_codec else 0
    cfg.load_rate_bits = int(load_rate)
    return cfg


def plan_bytes(shape, stencil: Stencil, k: int, slab_planes: int, rate: int,
               single_buffer: bool = True, budget: int = 0, ring_slots: int = 0,
               prefetch: int = 0, fuse: int = 0, share: bool = False,
               error_budget: float = 0.0, error_steps: int = 0, fused_codec: bool = False,
               load_rate: int = 0, in_place: bool = False) -> int:
    """Device bytes of the plan (with an error budget: at least the pilot's
    sample within `budget`); 0 if no plan exists."""
    g = make_grid(shape)
    cfg = plan_config(k, slab_planes, rate, single_buffer, budget, ring_slots, prefetch, fuse, share,
                      in_place, error_budget=error_budget, error_steps=error_steps,
                      fused_codec=fused_codec, load_rate=load_rate)
    return int(lib().oc_plan_bytes(_ref(g), _ref(stencil), _ref(cfg)))


def check_plan(shape, stencil: Stencil, k: int, slab_planes: int, rate: int, sweeps: int,
               single_buffer: bool = True, budget: int = 0, mutate: int = 0, i: int = 0,
               ring_slots: int = 0, prefetch: int = 0, fuse: int = 0, share: bool = False,
               in_place: bool = False, fused_codec: bool = False, load_rate: int = 0) -> int:
    g = make_grid(shape)
    cfg = plan_config(k, slab_planes, rate, single_buffer, budget, ring_slots, prefetch, fuse, share,
                      in_place, fused_codec=fused_codec, load_rate=load_rate)
    return int(lib().oc_debug_check_plan(_ref(g), _ref(stencil), _ref(cfg), int(sweeps),
                                         int(mutate), int(i)))


def check_plan_ckpt(shape, stencil: Stencil, k: int, slab_planes: int, sweeps: int, ckpt_rate: int,
                    budget: int = 0, mutate: int = 0, i: int = 0, fuse: int = 0,
                    share: bool = False) -> int:
    """check_plan for an uncompressed op list whose last sweep also writes a
    checkpoint (codes at ckpt_rate, or raw planes for 0); mutate=0, i=-1
    returns the number of waits."""
    g = make_grid(shape)
    cfg = plan_config(k, slab_planes, 0, True, budget, fuse=fuse, share=share)
    return int(lib().oc_debug_check_plan_ckpt(_ref(g), _ref(stencil), _ref(cfg), int(sweeps),
                                              int(ckpt_rate), int(mutate), int(i)))


def plan_ops(shape, stencil: Stencil, k: int, slab_planes: int, rate: int, sweeps: int,
             single_buffer: bool = True, budget: int = 0, ring_slots: int = 0, prefetch: int = 0,
             fuse: int = 0, share: bool = False,
             in_place: bool = False, fused_codec: bool = False, load_rate: int = 0):
    g = make_grid(shape)
    cfg = plan_config(k, slab_planes, rate, single_buffer, budget, ring_slots, prefetch, fuse, share,
                      in_place, fused_codec=fused_codec, load_rate=load_rate)
    nw = ctypes.c_int64(0)
    n = int(lib().oc_debug_plan_ops(_ref(g), _ref(stencil), _ref(cfg), int(sweeps), _ref(nw)))
    return n, int(nw.value)


def plan_dump(shape, stencil: Stencil, k: int, slab_planes: int, rate: int, sweeps: int,
              single_buffer: bool = True, budget: int = 0, ring_slots: int = 0,
              prefetch: int = 0, fuse: int = 0, share: bool = False,
              in_place: bool = False, fused_codec: bool = False, load_rate: int = 0) -> str:
    """Text listing of the operation list the executor would issue."""
    g = make_grid(shape)
    cfg = plan_config(k, slab_planes, rate, single_buffer, budget, ring_slots, prefetch, fuse, share,
                      in_place, fused_codec=fused_codec, load_rate=load_rate)
    n = int(lib().oc_debug_plan_dump(_ref(g), _ref(stencil), _ref(cfg), int(sweeps), None, 0))
    if n < 0:
        raise OCError(n, "oc_debug_plan_dump", status_str(n))
    buf = ctypes.create_string_buffer(n)
    lib().oc_debug_plan_dump(_ref(g), _ref(stencil), _ref(cfg), int(sweeps), buf, n)
    return buf.value.decode()


def check_adjoint_plan(shape, stencil: Stencil, steps: int, ckpt_every: int, ckpt_rate: int,
                       budget: int = 0, slab_planes: int = 0, mutate: int = 0, i: int = 0,
                       share: bool = False) -> int:
    """Race check of the adjoint's reverse-sweep operation list (see oc.h);
    mutate=0, i=-1 returns the number of waits."""
    g = make_grid(shape)
    cfg = plan_config(1, slab_planes, 0, True, budget, share=share)
    return int(lib().oc_debug_check_adjoint(_ref(g), _ref(stencil), _ref(cfg), int(steps),
                                            int(ckpt_every), int(ckpt_rate), int(mutate), int(i)))


def codec_bytes(shape, rate: int) -> int:
    nz, ny, nx = shape
    return int(lib().oc_codec_bytes(int(nx), int(ny), int(nz), int(rate)))


# ---- device-buffer entry points (need torch + a GPU) -----------------------
def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


_stream_pool = {}
_stream_overlap = {}


def pipeline_streams(device=None):
    """The three streams (copy-in, kernels, copy-back) every handle on `device`
    shares.  Created once per process: each new stream takes a hardware queue,
    and once there are more streams than queues, streams share queues; the
    kernel and copy-back streams must not share one (the copy-back kernel
    would then run in line with the decode / stencil / encode kernels), so a
    program should call this before it creates streams of its own.  On
    creation the two are probed (oc_stream_overlap) and a RuntimeWarning is
    raised when they turn out serialized."""
    torch = _torch()
    dev = torch.device(device if device is not None else "cuda")
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    with _lock:
        streams = _stream_pool.get(dev)
        created = streams is None
        if created:
            streams = _stream_pool[dev] = [torch.cuda.Stream(device=dev) for _ in range(3)]
    if created:
        with torch.cuda.device(dev):
            ov = stream_overlap(streams[1], streams[2])
        _stream_overlap[dev] = ov
        if ov < 0.5:
            warnings.warn(
                "the kernel and copy-back streams on %s run one after the other (probe overlap %.2f): "
                "they share a hardware queue, so the copy-back kernel runs in line with the "
                "decode / stencil / encode kernels and jobs slow down; call "
                "oc.pipeline_streams() before the program creates streams of its own" % (dev, ov),
                RuntimeWarning, stacklevel=2)
    return streams


def pipeline_stream_overlap(device=None) -> float:
    """The probe overlap measured when pipeline_streams() created the streams
    of `device` (about 1: the kernel and copy-back streams run side by side)."""
    torch = _torch()
    dev = torch.device(device if device is not None else "cuda")
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    pipeline_streams(dev)
    return _stream_overlap.get(dev, float("nan"))


def stream_overlap(a, b) -> float:
    """Share of a 2 ms one-wave kernel's run on stream a or b (the shorter)
    during which the same kernel ran on the other stream, both launched at
    once: about 1 when the two streams run side by side, 0 when serialized."""
    r = ctypes.c_double(0.0)
    _check(lib().oc_stream_overlap(_stream_handle(a), _stream_handle(b), ctypes.byref(r)), "oc_stream_overlap")
    return float(r.value)


def _dev(t, dtype, what):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("%s must be a contiguous CUDA tensor of %s" % (what, dtype))
    return ctypes.c_void_p(t.data_ptr())


def compress(d_in, rate: int, out=None, stream=None):
    """Fixed-rate encode of a [nz][ny][nx] float32 CUDA tensor; returns uint8 codes."""
    torch = _torch()
    nz, ny, nx = d_in.shape
    nbytes = codec_bytes(d_in.shape, rate)
    if nbytes == 0:
        raise OCError(OC_ERR_SHAPE, "compress", "dims must be multiples of 4, rate 1..32")
    if out is None:
        out = torch.empty(nbytes, dtype=torch.uint8, device=d_in.device)
    _check(lib().oc_codec_compress(_dev(d_in, torch.float32, "d_in"), nx, ny, nz, int(rate),
                                   _dev(out, torch.uint8, "out"), out.numel(),
                                   _stream_handle(stream)), "oc_codec_compress")
    return out


def decompress(d_codes, shape, rate: int, out=None, stream=None):
    torch = _torch()
    nz, ny, nx = shape
    if d_codes.numel() < codec_bytes(shape, rate):
        raise ValueError("code buffer too small")
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=d_codes.device)
    _check(lib().oc_codec_decompress(_dev(d_codes, torch.uint8, "d_codes"), nx, ny, nz, int(rate),
                                     _dev(out, torch.float32, "out"), _stream_handle(stream)),
           "oc_codec_decompress")
    return out


def codec_error(d_in, rate: int, stream=None):
    """Codec round trip at `rate` of a [nz][ny][nx] float32 CUDA tensor, on the
    device: (sum of squared errors, sum of squared inputs, max abs error)."""
    torch = _torch()
    nz, ny, nx = d_in.shape
    nw = int(lib().oc_codec_error_work_bytes(nx, ny, nz, int(rate)))
    if nw == 0:
        raise OCError(OC_ERR_SHAPE, "codec_error", "dims must be multiples of 4, rate 1..32")
    work = torch.empty(nw, dtype=torch.uint8, device=d_in.device)
    out = torch.empty(3, dtype=torch.float64, device=d_in.device)
    _check(lib().oc_codec_error(_dev(d_in, torch.float32, "d_in"), nx, ny, nz, int(rate),
                                ctypes.c_void_p(work.data_ptr()), nw, ctypes.c_void_p(out.data_ptr()),
                                _stream_handle(stream)), "oc_codec_error")
    torch.cuda.synchronize(d_in.device)
    return tuple(float(v) for v in out.cpu())


def codec_error_noalloc(d_in, rate: int, out=None, stream=None):
    """codec_error through the allocation-free entry point: no workspace; the
    three FP64 results go to `out` (a CUDA float64 tensor of 3, allocated here
    if None) and are returned as a tuple after a synchronisation."""
    torch = _torch()
    nz, ny, nx = d_in.shape
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=d_in.device)
    _check(lib().oc_codec_error_noalloc(_dev(d_in, torch.float32, "d_in"), nx, ny, nz, int(rate),
                                        _dev(out, torch.float64, "out"), _stream_handle(stream)),
           "oc_codec_error_noalloc")
    torch.cuda.synchronize(d_in.device)
    return tuple(float(v) for v in out.cpu())


def codec_star7(codes, shape, gz0: int, nz: int, rate: int, steps: int, c=C_CONFIG1, lay=None, out=None,
                stream=None):
    """The fused codec kernel on one slab (tuning aid): `codes` holds the slab's
    layers (shape = (planes, ny, nx), one halo layer on either side of the
    interior); returns the interior's codes after `steps` 7-point steps.
    lay = (lay_lo, lay_hi): the coded layers (default all)."""
    torch = _torch()
    planes, ny, nx = shape
    nl = planes // 4
    out_nl = nl - 2
    lb = codec_bytes((4, ny, nx), rate)
    if out is None:
        out = torch.empty(out_nl * lb, dtype=torch.uint8, device=codes.device)
    lo, hi = lay if lay is not None else (0, nl)
    cc = (ctypes.c_float * 7)(*c)
    _check(lib().oc_debug_codec_star7(_dev(codes, torch.uint8, "codes"), _dev(out, torch.uint8, "out"), nx, ny,
                                      int(nz), int(gz0), out_nl, int(lo), int(hi), int(rate), int(steps), cc,
                                      _stream_handle(stream)), "oc_debug_codec_star7")
    return out


def copy_to_host(host_dst, host_off: int, dev_src, nbytes: int, workgroups: int = 4, stream=None):
    """Enqueues the pipeline's copy-back kernel: `nbytes` from the start of a
    CUDA tensor to byte `host_off` of a pinned CPU tensor (tuning aid for the
    host-link probe)."""
    torch = _torch()
    if not (isinstance(host_dst, torch.Tensor) and host_dst.is_pinned()):
        raise ValueError("host_dst must be a pinned CPU tensor")
    if host_off < 0 or host_off + nbytes > host_dst.numel() * host_dst.element_size() or \
            nbytes > dev_src.numel() * dev_src.element_size():
        raise ValueError("copy range outside the tensors")
    _check(lib().oc_debug_copy_to_host(ctypes.c_void_p(host_dst.data_ptr()), int(host_off),
                                       ctypes.c_void_p(dev_src.data_ptr()), int(nbytes),
                                       int(workgroups), _stream_handle(stream)),
           "oc_debug_copy_to_host")


def codec_status(stream=None) -> int:
    return int(lib().oc_codec_status(_stream_handle(stream)))


def star7_incore(d_in, c, steps: int, c0f=None, stream=None):
    """A^steps on a device field; returns a new CUDA tensor."""
    torch = _torch()
    nz, ny, nx = d_in.shape
    out = torch.empty_like(d_in)
    tmp = torch.empty_like(d_in) if steps > 1 else None
    cc = (ctypes.c_float * 7)(*[float(v) for v in c])
    _check(lib().oc_star7_incore(_dev(d_in, torch.float32, "d_in"), _dev(out, torch.float32, "out"),
                                 None if tmp is None else ctypes.c_void_p(tmp.data_ptr()),
                                 nx, ny, nz, ctypes.cast(cc, ctypes.c_void_p),
                                 None if c0f is None else _dev(c0f, torch.float32, "c0f"),
                                 int(steps), _stream_handle(stream)), "oc_star7_incore")
    return out


def wave25_incore(d_prev, d_cur, d_vel, stencil: Stencil, n0: int, steps: int, stream=None):
    """Advances (p^{n0-1}, p^{n0}) in place on the device; returns (d_prev, d_cur)."""
    torch = _torch()
    nz, ny, nx = d_cur.shape
    tmp = torch.empty_like(d_cur) if steps % 2 else None
    _check(lib().oc_wave25_incore(_dev(d_prev, torch.float32, "d_prev"), _dev(d_cur, torch.float32, "d_cur"),
                                  _dev(d_vel, torch.float32, "d_vel"),
                                  None if tmp is None else ctypes.c_void_p(tmp.data_ptr()),
                                  nx, ny, nz, _ref(stencil), int(n0), int(steps),
                                  _stream_handle(stream)), "oc_wave25_incore")
    return d_prev, d_cur


class OutOfCore:
    """Out-of-core time stepping of a host-resident field.

    shape = (nz, ny, nx).  stencil = a Stencil (make_star7 / make_wave25); when
    None, the 7-point star with coefficients `c` (and a c0 field if c0_field).
    budget = bytes of device memory the library may use; one torch allocation of
    exactly the bytes the plan needs (of the whole budget with full_arena: the
    adjoint's reverse sweeps plan their own slabs within it).
    rate = 0 keeps raw FP32 on the host; 1..32 keeps fixed-rate codes.  k =
    steps per residency; slab_planes = S (0 = largest that fits the budget).
    fuse = 7-point steps per stencil launch (0 = 4); copy_back = workgroups of
    the copy-back kernel (0 = 4, -1 = runtime copies); share = region sharing
    (the overlap of consecutive slabs stays on the device); in_place = one host
    level updated in place (needs sharing, or one slab).  error_budget > 0
    (7-point only): `rate` is the largest rate allowed, and load() picks the
    smallest rate whose relative L2 error after error_steps steps stays within
    the budget, from a pilot run of the job's process on a z-sample of the
    field; stats() reports the rate ("rate_bits") and the pilot's error.
    """

    def __init__(self, shape, c=C_CONFIG1, k: int = 4, rate: int = 0, budget: int = 512 << 20,
                 slab_planes: int = 0, single_buffer: bool = True, c0_field: bool = False,
                 timing: bool = False, ring_slots: int = 0, prefetch: int = 0, device=None,
                 stencil: Stencil = None, fuse: int = 0, copy_back: int = 0, share: bool = True,
                 in_place: bool = False, full_arena: bool = False, error_budget: float = 0.0,
                 error_steps: int = 0, fused_codec: bool = False, load_rate: int = 0):
        torch = _torch()
        self.shape = tuple(int(v) for v in shape)
        self.rate = int(rate)
        self.k = int(k)
        self.stencil = stencil if stencil is not None else make_star7(c, c0_field)
        self.wave = self.stencil.kind == OC_WAVE25
        self.grid = make_grid(self.shape)
        self.device = torch.device(device if device is not None else "cuda")
        need = plan_bytes(self.shape, self.stencil, k, slab_planes, rate, single_buffer, budget,
                          ring_slots, prefetch, fuse, share, error_budget=error_budget,
                          error_steps=error_steps, fused_codec=fused_codec, load_rate=load_rate)
        if need == 0:
            if load_rate and (rate == 0 or load_rate > 32 or (load_rate < rate and not error_budget)):
                raise OCError(OC_ERR_ARG, "plan", "the load rate must lie in rate..32 on a coded run")
            if load_rate > rate and (self.stencil.kind != OC_STAR7 or fused_codec):
                raise OCError(OC_ERR_UNSUPPORTED, "plan",
                              "a separate load rate needs the 7-point stencil and three kernels")
            if fused_codec and not (rate > 0 and self.stencil.kind == OC_STAR7 and not c0_field
                                    and k <= 4 and rate <= 16):
                raise OCError(OC_ERR_UNSUPPORTED, "plan",
                              "the fused codec kernel needs a coded 7-point run with constant c0, "
                              "k <= 4 and rate <= 16")
            raise OCError(OC_ERR_BUDGET, "plan", "no slab depth fits the budget")
        # the plan's bytes fit `budget`; planning again with exactly those bytes
        # as the budget picks the same slab depth (plan bytes grow with it)
        arena_bytes = int(budget) if full_arena else int(need)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        self.streams = pipeline_streams(self.device)
        # host levels hold codes at the larger of the rate and the load rate
        lb = host_level_bytes(self.shape, self.stencil, max(int(rate), int(load_rate)))
        self.levels = [torch.empty(lb, dtype=torch.uint8, pin_memory=True)
                       for _ in range(1 if in_place else 2)]
        ab = host_aux_bytes(self.shape, self.stencil, rate)
        self.aux = torch.empty(ab, dtype=torch.uint8, pin_memory=True) if ab else None
        cfg = Config()
        cfg.dev_arena = self.arena.data_ptr()
        cfg.dev_budget = arena_bytes
        for i, s in enumerate(self.streams):
            cfg.streams[i] = s.cuda_stream
        cfg.host_level[0] = self.levels[0].data_ptr()
        cfg.host_level[1] = None if in_place else self.levels[1].data_ptr()
        cfg.host_level_bytes = lb
        cfg.host_aux = self.aux.data_ptr() if self.aux is not None else None
        cfg.host_aux_bytes = ab
        cfg.k = int(k)
        cfg.slab_planes = int(slab_planes)
        cfg.rate_bits = int(rate)
        cfg.single_buffer = 1 if single_buffer else 0
        cfg.timing = 1 if timing else 0
        cfg.ring_slots = int(ring_slots)
        cfg.prefetch = int(prefetch)
        cfg.fuse_steps = int(fuse)
        cfg.copy_back = int(copy_back)
        cfg.share_overlap = 1 if share else -1
        cfg.in_place = 1 if in_place else 0
        cfg.error_budget = float(error_budget)
        cfg.error_steps = int(error_steps)
        cfg.fused_codec = 1 if fused_codec else 0
        cfg.load_rate_bits = int(load_rate)
        self.cfg = cfg
        h = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        _check(lib().oc_create(_ref(self.grid), _ref(self.stencil), _ref(cfg), ctypes.byref(h)),
               "oc_create")
        self.h = h

    def _host_f32(self, a):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        if a.shape != self.shape:
            raise ValueError("expected shape %s, got %s" % (self.shape, a.shape))
        return a

    def load(self, u, aux=None, vel=None):
        """STAR7: u = field, aux = c0 field (if any).  WAVE25: u = p^0,
        aux = p^{-1}, vel = velocity."""
        u = self._host_f32(u)
        a = None if aux is None else self._host_f32(aux)
        v = None if vel is None else self._host_f32(vel)
        _check(lib().oc_load(self.h, ctypes.c_void_p(u.ctypes.data),
                             None if a is None else ctypes.c_void_p(a.ctypes.data),
                             None if v is None else ctypes.c_void_p(v.ctypes.data)), "oc_load")

    def run(self, steps: int):
        _check(lib().oc_run(self.h, int(steps)), "oc_run")

    def store(self):
        """STAR7: the field.  WAVE25: (p^n, p^{n-1})."""
        out = np.empty(self.shape, dtype=np.float32)
        if self.wave:
            prev = np.empty(self.shape, dtype=np.float32)
            _check(lib().oc_store(self.h, ctypes.c_void_p(out.ctypes.data),
                                  ctypes.c_void_p(prev.ctypes.data)), "oc_store")
            return out, prev
        _check(lib().oc_store(self.h, ctypes.c_void_p(out.ctypes.data), None), "oc_store")
        return out

    def stats(self) -> dict:
        s = Stats()
        _check(lib().oc_stats_get(self.h, _ref(s)), "oc_stats_get")
        return {name: getattr(s, name) for name, _ in Stats._fields_}

    def timeline(self):
        """Per timed op of the last run (timing on): (class, sweep*100000+slab,
        start ms, end ms) arrays; classes 0 decode, 1 stencil, 2 encode, 3 H2D, 4 D2H."""
        n = int(lib().oc_debug_timeline(self.h, None, None, None, None, 0))
        if n < 0:
            raise OCError(n, "oc_debug_timeline", status_str(n))
        kind = np.zeros(n, np.int32)
        slab = np.zeros(n, np.int64)
        t0 = np.zeros(n, np.float64)
        t1 = np.zeros(n, np.float64)
        if n:
            m = int(lib().oc_debug_timeline(self.h, kind.ctypes.data, slab.ctypes.data,
                                            t0.ctypes.data, t1.ctypes.data, n))
            if m < 0:
                raise OCError(m, "oc_debug_timeline", status_str(m))
        return kind, slab, t0, t1

    def set_timing(self, on: bool):
        _check(lib().oc_set_timing(self.h, 1 if on else 0), "oc_set_timing")

    def fail_after(self, n: int):
        _check(lib().oc_debug_fail_after(self.h, int(n)), "oc_debug_fail_after")

    def serialize(self, on: bool):
        """Test hook: every operation completes before the next is issued."""
        _check(lib().oc_debug_serialize(self.h, 1 if on else 0), "oc_debug_serialize")

    def close(self):
        if getattr(self, "h", None):
            lib().oc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Adjoint:
    """Forward with checkpoints, then gradients of a loss of u_T (7-point star).

    Wraps an uncompressed OutOfCore handle (the forward is exact); checkpoints
    every `ckpt_every` steps are kept on the host as codes at `ckpt_rate`
    bits/value (0 = raw), u_0 exactly.  share = region sharing in the forward
    and the reverse sweeps; fuse = stencil steps per launch in the forward and
    in the reverse sweeps' recomputation (0 = 4)."""

    def __init__(self, shape, c=C_CONFIG1, steps: int = 64, k: int = 4, ckpt_every: int = 8,
                 ckpt_rate: int = 16, budget: int = 512 << 20, slab_planes: int = 0,
                 c0_field: bool = True, device=None, share: bool = True, fuse: int = 0):
        torch = _torch()
        self.steps, self.ckpt_every, self.ckpt_rate = int(steps), int(ckpt_every), int(ckpt_rate)
        self.ooc = OutOfCore(shape, c, k=k, rate=0, budget=budget, slab_planes=slab_planes,
                             c0_field=c0_field, device=device, share=share, fuse=fuse,
                             full_arena=True)
        n = int(lib().oc_adjoint_host_bytes(self.ooc.h, self.steps, self.ckpt_every,
                                            self.ckpt_rate))
        if n == 0:
            raise OCError(OC_ERR_BUDGET, "oc_adjoint_host_bytes", "no adjoint plan fits")
        self.work = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        self.shape = self.ooc.shape
        # forwards started on this runner; the checkpoints backward() uses are
        # those of forward number `generation`
        self.generation = 0

    def forward(self, u0, c0=None) -> np.ndarray:
        self.generation += 1
        self.ooc.load(u0, c0)
        _check(lib().oc_forward_ckpt(self.ooc.h, self.steps, self.ckpt_every, self.ckpt_rate,
                                     ctypes.c_void_p(self.work.data_ptr()), self.work.numel()),
               "oc_forward_ckpt")
        return self.ooc.store()

    def backward(self, gT):
        gT = self.ooc._host_f32(gT)
        g_u0 = np.empty(self.shape, np.float32)
        g_c0 = np.empty(self.shape, np.float32)
        _check(lib().oc_adjoint(self.ooc.h, ctypes.c_void_p(gT.ctypes.data),
                                ctypes.c_void_p(g_u0.ctypes.data), ctypes.c_void_p(g_c0.ctypes.data)),
               "oc_adjoint")
        return g_u0, g_c0

    def close(self):
        self.ooc.close()


def stencil_function():
    """torch.autograd.Function: u_T = A(c0)^steps u0 with host-resident CPU
    float32 tensors; backward returns dL/du0 and dL/dc0 from the adjoint."""
    torch = _torch()

    class OCStencilFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, u0, c0, runner):
            uT = runner.forward(u0.detach().cpu().numpy(), c0.detach().cpu().numpy())
            ctx.runner = runner
            ctx.generation = runner.generation
            return torch.from_numpy(uT)

        @staticmethod
        def backward(ctx, gT):
            # the runner keeps the checkpoints of its latest forward only
            if ctx.runner.generation != ctx.generation:
                raise RuntimeError(
                    "OCStencilFn.backward: the runner ran another forward (number %d) after "
                    "this one (number %d) and no longer holds its checkpoints; use one runner "
                    "per pending backward" % (ctx.runner.generation, ctx.generation))
            g_u0, g_c0 = ctx.runner.backward(gT.detach().to(torch.float32).cpu().numpy())
            return torch.from_numpy(g_u0), torch.from_numpy(g_c0), None

    return OCStencilFn
