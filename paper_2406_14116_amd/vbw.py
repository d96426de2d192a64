"""Python binding of ``libvbw.so`` (C ABI in ``include/vbw.h``).

Argument marshalling only: every step of the filtering runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.  There is no CPU
fallback: if the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VBW_LIBRARY", os.path.join(HERE, "libvbw.so"))
HEADER = os.path.join(os.path.dirname(HERE), "include", "vbw.h")

VBW_OK, VBW_EINVAL, VBW_ERANGE, VBW_ENOMEM, VBW_EDEVICE, VBW_EUNSUPPORTED, VBW_ETOOLARGE = 0, -1, -2, -3, -4, -5, -6
NOALLOC_SCRATCH_BYTES = 2 << 20
DTYPES = {"c64": 0, "f16": 1, "bf16": 2, "r32": 3}
ENGINES = {"fft": 0, "gemm": 1}
NO_PRUNE, GRAPH, F32_OUT, HOST_ONLY, AUTOTUNE, STREAM = 1, 2, 4, 8, 16, 32
(Q_N_CHANNELS, Q_N_ITEMS, Q_TOTAL_BLOCKS, Q_TOTAL_SAMPLES, Q_WORKGROUP, Q_LDS_BYTES, Q_GRID, Q_VARIANT,
 Q_N_VARIANTS) = range(9)


class vbw_channel(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("hop", ctypes.c_int32), ("lv", ctypes.c_int32),
                ("v_offset", ctypes.c_int32), ("k1", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("len", ctypes.c_int64)]


class vbw_plan_desc(ctypes.Structure):
    _fields_ = [("n_channels", ctypes.c_int32), ("n_v", ctypes.c_int32),
                ("channels", ctypes.POINTER(vbw_channel)), ("v_pool", ctypes.POINTER(ctypes.c_double)),
                ("dtype", ctypes.c_int32), ("engine", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("max_workgroups", ctypes.c_int32), ("tune_cache", ctypes.c_char_p), ("reserved", ctypes.c_int32)]


class vbw_band_switch(ctypes.Structure):
    _fields_ = [("channel", ctypes.c_int32), ("k1", ctypes.c_int32), ("from_block", ctypes.c_int64)]


class VbwError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


_LIB = None


def lib():
    """Load libvbw.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the HIP library is the only compute path)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.vbw_plan.argtypes = [ctypes.POINTER(vbw_plan_desc), ctypes.POINTER(P)]
        L.vbw_plan.restype = ctypes.c_int
        L.vbw_set_bandwidth.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
        L.vbw_set_bandwidth.restype = ctypes.c_int
        L.vbw_filter.argtypes = [P, P, P, P]
        L.vbw_filter.restype = ctypes.c_int
        L.vbw_filter_timed.argtypes = [P, P, P, P, P, P]
        L.vbw_filter_timed.restype = ctypes.c_int
        L.vbw_destroy.argtypes = [P]
        L.vbw_destroy.restype = None
        L.vbw_strerror.argtypes = [ctypes.c_int]
        L.vbw_strerror.restype = ctypes.c_char_p
        L.vbw_plan_query.argtypes = [P, ctypes.c_int32]
        L.vbw_plan_query.restype = ctypes.c_int64
        L.vbw_block_k1.argtypes = [P, ctypes.c_int32, ctypes.c_int64]
        L.vbw_block_k1.restype = ctypes.c_int32
        L.vbw_copy.argtypes = [P, P, ctypes.c_int64, P]
        L.vbw_copy.restype = ctypes.c_int
        L.vbw_twiddle_table.argtypes = [ctypes.c_int32, P]
        L.vbw_twiddle_table.restype = ctypes.c_int
        L.vbw_stream_reset.argtypes = [P, P]
        L.vbw_stream_reset.restype = ctypes.c_int
        L.vbw_filter_noalloc.argtypes = [ctypes.POINTER(vbw_plan_desc), ctypes.c_int32,
                                         ctypes.POINTER(vbw_band_switch), P, P, P]
        L.vbw_filter_noalloc.restype = ctypes.c_int
        L.vbw_plan_set_variant.argtypes = [P, ctypes.c_int32]
        L.vbw_plan_set_variant.restype = ctypes.c_int
        L.vbw_test_fail_device_alloc.argtypes = [ctypes.c_int32]
        L.vbw_test_fail_device_alloc.restype = None
        _LIB = L
    return _LIB


def header_functions() -> list:
    """Names of the functions include/vbw.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vbw_[a-z0-9_]+)\s*\(", text)))


def test_fail_device_alloc(k: int) -> None:
    """Test hook: the k-th device allocation of every later vbw_plan on this
    thread fails (0: off)."""
    lib().vbw_test_fail_device_alloc(int(k))


def strerror(status: int) -> str:
    return lib().vbw_strerror(int(status)).decode()


def twiddle_table(n: int) -> np.ndarray:
    out = np.empty(2 * n, dtype=np.float32)
    rc = lib().vbw_twiddle_table(int(n), out.ctypes.data_as(ctypes.c_void_p))
    if rc != VBW_OK:
        raise VbwError(rc, "vbw_twiddle_table")
    return out.reshape(n, 2)


def copy(src, dst, stream=None) -> None:
    """Streaming device copy of src into dst (torch tensors of equal byte size)."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy: size mismatch")
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = lib().vbw_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    if rc != VBW_OK:
        raise VbwError(rc, "vbw_copy")


def _channel_array(channels):
    """ctypes array of vbw_channel and the channel lengths, from dicts (len)
    or objects (length) with n, hop, lv, v_offset, k1."""
    chans = list(channels)
    arr = (vbw_channel * max(1, len(chans)))()
    lengths = []
    for i, c in enumerate(chans):
        g = (lambda k, c=c: c[k]) if isinstance(c, dict) else (lambda k, c=c: getattr(c, k))
        length = c["len"] if isinstance(c, dict) else c.length
        arr[i] = vbw_channel(int(g("n")), int(g("hop")), int(g("lv")), int(g("v_offset")),
                             int(g("k1")), 0, int(length))
        lengths.append(int(length))
    return arr, lengths


def filter_noalloc(channels, v_pool, xs, ys, dtype: str = "c64", engine: str = "fft", flags: int = 0,
                   switches=(), stream=None, max_workgroups: int = 0) -> None:
    """vbw_filter_noalloc: plan, band switches (channel, k1, from_block) and
    filter in one call that allocates no device memory.  xs / ys: device
    tensors as for Plan.filter (checked here the same way)."""
    arr, lengths = _channel_array(channels)
    pool = np.ascontiguousarray(np.asarray(v_pool, dtype=np.float64))
    desc = vbw_plan_desc(len(lengths), int(pool.size), arr,
                         pool.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if pool.size else None,
                         DTYPES[dtype], ENGINES[engine], int(flags), int(max_workgroups), None, 0)
    _check_tensors(lengths, dtype, int(flags), xs, ys)
    sw = list(switches)
    sarr = (vbw_band_switch * max(1, len(sw)))(*[vbw_band_switch(int(c), int(k), int(b)) for c, k, b in sw])
    n = max(1, len(lengths))
    xp = (ctypes.c_void_p * n)(*[t.data_ptr() or None for t in xs])
    yp = (ctypes.c_void_p * n)(*[t.data_ptr() or None for t in ys])
    rc = lib().vbw_filter_noalloc(ctypes.byref(desc), len(sw), sarr, ctypes.cast(xp, ctypes.c_void_p),
                                  ctypes.cast(yp, ctypes.c_void_p), _stream_handle(stream) or None)
    if rc != VBW_OK:
        raise VbwError(rc, "vbw_filter_noalloc")


def _check_tensors(lengths, dtype, flags, xs, ys) -> None:
    """The kernels address len samples of the storage type from each pointer:
    check element types and sizes before handing pointers over."""
    import torch
    if len(xs) != len(lengths) or len(ys) != len(lengths):
        raise ValueError("one input and one output tensor per channel")
    in_types = {"c64": (torch.complex64,), "f16": (torch.float16,), "bf16": (torch.bfloat16,),
                "r32": (torch.float32,)}[dtype]
    f32_out = bool(flags & F32_OUT) and dtype in ("f16", "bf16")
    out_types = (torch.complex64, torch.float32) if f32_out else in_types
    in_bytes = {"c64": 8, "f16": 4, "bf16": 4, "r32": 4}[dtype]
    out_bytes = 8 if f32_out else in_bytes
    for i, (x, y) in enumerate(zip(xs, ys)):
        if x.dtype not in in_types or y.dtype not in out_types:
            raise ValueError(f"channel {i}: input must be {in_types}, output {out_types} for {dtype} "
                             f"storage (got {x.dtype}, {y.dtype})")
        if x.numel() * x.element_size() < lengths[i] * in_bytes or \
                y.numel() * y.element_size() < lengths[i] * out_bytes:
            raise ValueError(f"channel {i}: tensors hold fewer than len = {lengths[i]} samples")
    for t in list(xs) + list(ys):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("tensors must be contiguous and on the GPU")


def _event_handles(start, stop):
    """HIP event handles of two torch.cuda.Event (or raw handles)."""
    if start is None or stop is None:
        raise ValueError("both events are needed")
    handles = [int(e.cuda_event) if hasattr(e, "cuda_event") else int(e) for e in (start, stop)]
    if not all(handles):
        raise ValueError("events must exist: record each once before passing it")
    return handles[0], handles[1]


def _stream_handle(stream) -> int:
    """hipStream_t of a torch stream, an integer handle, or (None) torch's
    current stream."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Plan:
    """One vbw_plan: channels, shared V pool, storage dtype, engine, flags.

    ``channels`` is a sequence of dicts or objects with n, hop, lv, v_offset,
    k1 and len (or ``length``).
    """

    def __init__(self, channels, v_pool, dtype: str = "c64", engine: str = "fft", flags: int = 0,
                 tune_cache: str | None = None, max_workgroups: int = 0):
        arr, self.lengths = _channel_array(channels)
        self.n_channels = len(self.lengths)
        self.v_pool = np.ascontiguousarray(np.asarray(v_pool, dtype=np.float64))
        self.dtype = dtype
        self.flags = int(flags)
        desc = vbw_plan_desc(self.n_channels, int(self.v_pool.size), arr,
                             self.v_pool.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                             if self.v_pool.size else None,
                             DTYPES[dtype], ENGINES[engine], self.flags, int(max_workgroups),
                             os.fsencode(tune_cache) if tune_cache else None, 0)
        h = ctypes.c_void_p()
        rc = lib().vbw_plan(ctypes.byref(desc), ctypes.byref(h))
        if rc != VBW_OK:
            raise VbwError(rc, "vbw_plan")
        self._h = h
        self._xp = (ctypes.c_void_p * max(1, self.n_channels))()
        self._yp = (ctypes.c_void_p * max(1, self.n_channels))()

    @classmethod
    def from_workload(cls, w, dtype: str | None = None, engine: str = "fft", flags: int = 0, **kw):
        pool, offs = w.v_pool()
        chans = [dict(n=c.n, hop=c.hop, lv=c.lv, v_offset=offs[c.v_key], k1=c.k1, len=c.length)
                 for c in w.channels]
        if dtype is None:
            dtype = {"c64": "c64", "c128": "c64", "f16": "f16", "bf16": "bf16", "r32": "r32"}[w.storage]
        p = cls(chans, pool, dtype=dtype, engine=engine, flags=flags, **kw)
        for i, c in enumerate(w.channels):
            for frm, k1 in c.schedule:
                p.set_bandwidth(i, k1, frm)
        return p

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def set_variant(self, variant: int) -> None:
        """vbw_plan_set_variant: fix the launch variant."""
        rc = lib().vbw_plan_set_variant(self.handle, int(variant))
        if rc != VBW_OK:
            raise VbwError(rc, "vbw_plan_set_variant")

    def set_bandwidth(self, channel: int, k1: int, from_block: int) -> None:
        rc = lib().vbw_set_bandwidth(self.handle, int(channel), int(k1), int(from_block))
        if rc != VBW_OK:
            raise VbwError(rc, "vbw_set_bandwidth")

    def filter_ptrs(self, x_ptrs, y_ptrs, stream: int | None = 0) -> None:
        """Raw form: integer device addresses, integer hipStream_t (0 = null stream)."""
        for i in range(self.n_channels):
            self._xp[i] = x_ptrs[i] or None
            self._yp[i] = y_ptrs[i] or None
        rc = lib().vbw_filter(self.handle, ctypes.cast(self._xp, ctypes.c_void_p),
                              ctypes.cast(self._yp, ctypes.c_void_p), stream or None)
        if rc != VBW_OK:
            raise VbwError(rc, "vbw_filter")

    def filter(self, xs, ys, stream=None) -> None:
        """Filter torch tensors: complex64 (c64 storage), (len, 2) float16 /
        bfloat16 (16-bit storage) or 1-D float32 (r32, real input); outputs
        likewise, or (len, 2) float32 / complex64 with F32_OUT.  Runs on ``stream`` (default: torch's current)."""
        self._check_tensors(xs, ys)
        self.filter_ptrs([t.data_ptr() for t in xs], [t.data_ptr() for t in ys], _stream_handle(stream))

    def filter_timed(self, xs, ys, start, stop, stream=None) -> None:
        """vbw_filter_timed: as ``filter``; ``start`` / ``stop`` (torch.cuda.Event
        with timing, already created, i.e. recorded once) take the kernels' own
        start and end time, so ``start.elapsed_time(stop)`` is their duration."""
        self._check_tensors(xs, ys)
        for i, t in enumerate(xs):
            self._xp[i] = t.data_ptr() or None
        for i, t in enumerate(ys):
            self._yp[i] = t.data_ptr() or None
        a, b = _event_handles(start, stop)
        rc = lib().vbw_filter_timed(self.handle, ctypes.cast(self._xp, ctypes.c_void_p),
                                    ctypes.cast(self._yp, ctypes.c_void_p), _stream_handle(stream) or None, a, b)
        if rc != VBW_OK:
            raise VbwError(rc, "vbw_filter_timed")

    def bind(self, xs, ys):
        """Check the tensors once and return ``run(stream=None, start=None,
        stop=None)``, which filters them again on every call with nothing but
        the library call: the form for fixed buffers whose contents change
        (ring-buffered streaming, a serving loop).  With ``start`` and ``stop``
        (events as for ``filter_timed``) the call is vbw_filter_timed.  ``run``
        keeps the tensors alive."""
        self._check_tensors(xs, ys)
        n = max(1, self.n_channels)
        xp = (ctypes.c_void_p * n)(*[t.data_ptr() or None for t in xs])
        yp = (ctypes.c_void_p * n)(*[t.data_ptr() or None for t in ys])
        xpp, ypp = ctypes.cast(xp, ctypes.c_void_p), ctypes.cast(yp, ctypes.c_void_p)
        call, call_timed = lib().vbw_filter, lib().vbw_filter_timed

        def run(stream=None, start=None, stop=None):
            if start is None and stop is None:
                rc = call(self.handle, xpp, ypp, _stream_handle(stream) or None)   # raises once the plan is closed
            else:
                a, b = _event_handles(start, stop)
                rc = call_timed(self.handle, xpp, ypp, _stream_handle(stream) or None, a, b)
            if rc != VBW_OK:
                raise VbwError(rc, "vbw_filter" if start is None and stop is None else "vbw_filter_timed")
        run.tensors = (list(xs), list(ys), xp, yp)
        return run

    def _check_tensors(self, xs, ys) -> None:
        _check_tensors(self.lengths, self.dtype, self.flags, xs, ys)

    def stream_reset(self, stream=None) -> None:
        """Restart every channel's stream (STREAM plans) on ``stream``
        (default: torch's current stream)."""
        rc = lib().vbw_stream_reset(self.handle, _stream_handle(stream) or None)
        if rc != VBW_OK:
            raise VbwError(rc, "vbw_stream_reset")

    def query(self, q: int) -> int:
        return int(lib().vbw_plan_query(self.handle, int(q)))

    def block_k1(self, channel: int, block: int) -> int:
        return int(lib().vbw_block_k1(self.handle, int(channel), int(block)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().vbw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False
