"""ctypes binding of libkdeplugin (argument marshalling only).

Every function has the name of the C entry point it calls (declared in
``include/kdeplugin.h``); the work itself runs in the HIP library.  Samples may
be numpy arrays (host memory) or torch tensors on the GPU (device memory, used
in place on torch's current stream).  Importing this module loads
``libkdeplugin.so`` and raises ImportError if it has not been built: there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkdeplugin.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libkdeplugin.so not found at {LIB_PATH}; build it with "
        "`python -c 'import __graft_entry__ as g; g.build()'` or "
        "`python paper_1505_02100_amd/build.py`")

# torch first: the library's HIP runtime dependency then resolves to the
# runtime torch already loaded, so tensors, streams and kernels share one HIP
# runtime instance.
import torch as _torch_mod  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


def _mapped_hip_runtimes():
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


if len(_mapped_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are loaded in this process: " + ", ".join(_mapped_hip_runtimes()))

KDE_OK = 0
KDE_EINVAL = -1
KDE_ENONFINITE = -2
KDE_EDEGENERATE = -3
KDE_ENOMEM = -4
KDE_EDEVICE = -5
KDE_ETIMEOUT = -6
KDE_EBUSY = -7

KDE_FP64_PLAIN = 0
KDE_FP32_COMP = 1
KDE_FP32_COMP_EXACT = 2
KDE_FP32_POLYEXP = 3
KDE_Q32_32 = 4
KDE_MEM_HOST = 0
KDE_MEM_DEVICE = 1
KDE_F64 = 0
KDE_F32 = 1
KDE_NUM_STAGES = 4  # entries of kde_ctx_last_timeline


class kde_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mem_budget", ctypes.c_int64), ("tune_table", ctypes.c_char_p),
                ("rows_per_lane", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("target_items", ctypes.c_int32), ("wait_limit_us", ctypes.c_int32),
                ("pair_budget", ctypes.c_int64)]


class kde_result(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("mean", ctypes.c_double), ("sigma", ctypes.c_double),
                ("psi8", ctypes.c_double), ("g1", ctypes.c_double), ("psi6", ctypes.c_double),
                ("g2", ctypes.c_double), ("psi4", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}

    def __repr__(self):
        return "kde_result(" + ", ".join(f"{k}={v!r}" for k, v in self.as_dict().items()) + ")"


class kde_server_options(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_int64), ("step_pairs", ctypes.c_int64),
                ("max_active", ctypes.c_int32), ("policy", ctypes.c_int32),
                ("aging_ms", ctypes.c_int64), ("fill", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class kde_completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("n", ctypes.c_int64), ("result", kde_result),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double)]


class kde_server_stats(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("inflight_steps", ctypes.c_int32), ("failed_steps", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("arena_used", ctypes.c_int64),
                ("completed_unread", ctypes.c_int64), ("pairs_done", ctypes.c_double),
                ("pairs_issued", ctypes.c_double)]


KDE_SERVE_FCFS = 0
KDE_SERVE_SJF = 1
KDE_FILL_SHARE = 0
KDE_FILL_PRIORITY = 1


class KdeError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.kde_last_error_message().decode(errors="replace")
        super().__init__(f"{where}: {kde_strerror(code)} ({code}): {msg}")
        self.code = code


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PI32 = ctypes.POINTER(ctypes.c_int32)


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_sig("kde_version", ctypes.c_char_p)
_sig("kde_last_error", ctypes.c_int)
_sig("kde_last_error_message", ctypes.c_char_p)
_sig("kde_strerror", ctypes.c_char_p, ctypes.c_int)
_sig("kde_options_init", None, ctypes.POINTER(kde_options))
_sig("kde_ctx_create", ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(kde_options))
_sig("kde_ctx_destroy", None, _P)
_sig("kde_ctx_config", ctypes.c_int, _P, _PI32, _PI32, _PI32, _PI32)
_sig("kde_ctx_last_launch", ctypes.c_int, _P, _PI32, _PI32)
_sig("kde_psi", _D, ctypes.POINTER(_D), _I64, ctypes.c_int, _D)
_sig("kde_plugin_bandwidth", _D, ctypes.POINTER(_D), _I64)
_sig("kde_psi_ex", ctypes.c_int, _P, _P, _I64, ctypes.c_int, _D, ctypes.c_int, ctypes.c_int, _P,
     ctypes.POINTER(_D))
_sig("kde_plugin_bandwidth_ex", ctypes.c_int, _P, _P, _I64, ctypes.c_int, ctypes.c_int, _P,
     ctypes.POINTER(kde_result))
_sig("kde_plugin_bandwidth_batch", ctypes.c_int, _P, ctypes.POINTER(_P), _PI64, _I64, ctypes.c_int,
     ctypes.POINTER(kde_result), _P)
_sig("kde_plugin_bandwidth_noalloc", ctypes.c_int, _P, _P, _I64, ctypes.c_int, _P, ctypes.POINTER(kde_result))
_sig("kde_ctx_last_timeline", ctypes.c_int, _P, _I64, ctypes.POINTER(_D))
_sig("kde_ctx_last_device_ms", _D, _P)
_sig("kde_psi_num_items", _I64, _P, _I64)
_sig("kde_server_options_init", None, ctypes.POINTER(kde_server_options))
_sig("kde_server_create", ctypes.c_int, ctypes.POINTER(_P), _P, ctypes.POINTER(kde_server_options))
_sig("kde_server_destroy", None, _P)
_sig("kde_server_submit", ctypes.c_int, _P, _P, _I64, ctypes.c_int, _P, _PI64)
_sig("kde_server_cancel", ctypes.c_int, _P, _I64)
_sig("kde_server_step", ctypes.c_int, _P, _I32, ctypes.POINTER(kde_server_stats))
_sig("kde_server_poll", ctypes.c_int, _P, ctypes.POINTER(kde_completion), _I32, _PI32)
_sig("kde_server_drain", ctypes.c_int, _P)
_sig("kde_server_fail_next_step", ctypes.c_int, _P, _I32)
_sig("kde_autotune", ctypes.c_int, ctypes.POINTER(kde_options), _PI64, _I32, _I32, _I32, ctypes.c_char_p,
     _I32)
_sig("kde_psi_item_geometry", ctypes.c_int, _P, _I64, _I64, _PI64, _PI64, _PI64, _PI64)
_sig("kde_psi_range", ctypes.c_int, _P, _P, _I64, ctypes.c_int, _D, ctypes.c_int, ctypes.c_int,
     _I64, _I64, _P, ctypes.POINTER(_D))
_sig("kde_eval_ex", ctypes.c_int, _P, _P, _I64, ctypes.c_int, ctypes.c_int, _P, _I64, ctypes.c_int, _D, _P,
     _P)
_sig("kde_eval", ctypes.c_int, ctypes.POINTER(_D), _I64, ctypes.POINTER(_D), _I64, _D, ctypes.POINTER(_D))


def kde_version() -> str:
    return _lib.kde_version().decode()


def kde_strerror(code: int) -> str:
    return _lib.kde_strerror(int(code)).decode()


def kde_last_error() -> int:
    return _lib.kde_last_error()


def kde_last_error_message() -> str:
    return _lib.kde_last_error_message().decode(errors="replace")


def _check(code: int, where: str) -> None:
    if code != KDE_OK:
        raise KdeError(code, where)


# ------------------------------------------------------------ marshalling
class _Samples:
    """Pointer, length, memory kind, dtype and stream for one sample array.
    Keeps a reference to whatever owns the memory for the call's duration."""

    def __init__(self, x):
        self.keep = x
        if _is_torch(x):
            if x.device.type == "cuda":
                if not x.is_contiguous():
                    x = x.contiguous()
                    self.keep = x
                if x.dtype not in (_torch().float64, _torch().float32):
                    raise TypeError("samples must be float64 or float32")
                self.ptr = x.data_ptr()
                self.n = x.numel()
                self.mem = KDE_MEM_DEVICE
                self.dtype = KDE_F64 if x.dtype == _torch().float64 else KDE_F32
                self.stream = _current_stream(x.device)
                return
            x = x.detach().cpu().numpy()
        a = np.asarray(x)
        if a.dtype not in (np.float64, np.float32):
            a = a.astype(np.float64)
        a = np.ascontiguousarray(a).reshape(-1)
        self.keep = a
        self.ptr = a.ctypes.data
        self.n = a.size
        self.mem = KDE_MEM_HOST
        self.dtype = KDE_F64 if a.dtype == np.float64 else KDE_F32
        self.stream = None


def _torch():
    import torch
    return torch


def _current_stream(device) -> int:
    """The raw HIP stream torch currently uses on `device` (the call is
    ordered after the tensor's producers on that stream)."""
    t = _torch()
    raw = getattr(t._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return raw(device.index if device.index is not None else t.cuda.current_device())
    return t.cuda.current_stream(device).cuda_stream


def _is_torch(x) -> bool:
    mod = type(x).__module__
    return mod.startswith("torch") and hasattr(x, "data_ptr")


def _host_f64(x) -> np.ndarray:
    if _is_torch(x):
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64)).reshape(-1)


# ------------------------------------------------------------- literal calls
def kde_psi(x, r: int, g: float) -> float:
    """Psi_r(g) (equations (6)-(7)) on the default FP64 context; NaN on error."""
    a = _host_f64(x)
    return _lib.kde_psi(a.ctypes.data_as(ctypes.POINTER(_D)), a.size, int(r), float(g))


def kde_plugin_bandwidth(x) -> float:
    """h of Algorithm 1 on the default FP64 context; NaN on error."""
    a = _host_f64(x)
    return _lib.kde_plugin_bandwidth(a.ctypes.data_as(ctypes.POINTER(_D)), a.size)


# -------------------------------------------------------------- contexts
def kde_options_init() -> kde_options:
    o = kde_options()
    _lib.kde_options_init(ctypes.byref(o))
    return o


def kde_ctx_create(precision: int = KDE_FP64_PLAIN, device: int = 0, mem_budget: int = 0,
                   rows_per_lane: int = 0, blocks_per_cu: int = 0, target_items: int = 0,
                   tune_table: Optional[str] = None, pair_budget: int = 0, wait_limit_us: int = 0) -> int:
    o = kde_options_init()
    o.device = device
    o.precision = precision
    o.mem_budget = mem_budget
    o.rows_per_lane = rows_per_lane
    o.blocks_per_cu = blocks_per_cu
    o.target_items = target_items
    o.pair_budget = pair_budget
    o.wait_limit_us = wait_limit_us
    o.tune_table = tune_table.encode() if tune_table else None
    h = _P()
    _check(_lib.kde_ctx_create(ctypes.byref(h), ctypes.byref(o)), "kde_ctx_create")
    return h.value


def kde_ctx_destroy(ctx: int) -> None:
    _lib.kde_ctx_destroy(ctx)


def kde_ctx_last_launch(ctx: int) -> dict:
    b, w = _I32(), _I32()
    _check(_lib.kde_ctx_last_launch(ctx, ctypes.byref(b), ctypes.byref(w)), "kde_ctx_last_launch")
    return dict(blocks=b.value, waves_per_simd=w.value)


def kde_ctx_config(ctx: int) -> dict:
    v = [_I32() for _ in range(4)]
    _check(_lib.kde_ctx_config(ctx, *[ctypes.byref(t) for t in v]), "kde_ctx_config")
    return dict(rows_per_lane=v[0].value, block_threads=v[1].value, tile_rows=v[2].value,
                blocks_per_cu=v[3].value)


def kde_ctx_last_timeline(ctx: int, sample: int = 0) -> List[float]:
    """Milliseconds from the sample's first item to each stage's publication
    (mean; sigma and g1; Psi6 and g2; Psi4 and h)."""
    ms = (_D * KDE_NUM_STAGES)()
    _check(_lib.kde_ctx_last_timeline(ctx, int(sample), ms), "kde_ctx_last_timeline")
    return list(ms)


def kde_ctx_last_device_ms(ctx: int) -> float:
    """Device time (ms) of the last call's launch, from HIP events on its stream."""
    return _lib.kde_ctx_last_device_ms(ctx)


def kde_psi_ex(ctx: int, x, r: int, g: float) -> float:
    s = _Samples(x)
    out = _D()
    _check(_lib.kde_psi_ex(ctx, s.ptr, s.n, int(r), float(g), s.mem, s.dtype, s.stream,
                           ctypes.byref(out)), "kde_psi_ex")
    return out.value


def kde_plugin_bandwidth_ex(ctx: int, x, check: bool = True) -> kde_result:
    s = _Samples(x)
    res = kde_result()
    code = _lib.kde_plugin_bandwidth_ex(ctx, s.ptr, s.n, s.mem, s.dtype, s.stream, ctypes.byref(res))
    if check:
        _check(code, "kde_plugin_bandwidth_ex")
    return res


def _device_batch(xs: Sequence):
    """(pointers, sizes, stream) of a list of contiguous CUDA float64 tensors on
    one device, or None if xs is anything else; one pass, no per-sample stream
    lookups (the batch runs on the current stream of the samples' device)."""
    if not xs or not all(_is_torch(x) for x in xs):
        return None
    t = _torch()
    dev = xs[0].device
    if dev.type != "cuda":
        return None
    for x in xs:
        if x.device != dev or x.dtype != t.float64 or not x.is_contiguous():
            return None
    m = len(xs)
    ptrs = (_P * m)(*[x.data_ptr() for x in xs])
    ns = (_I64 * m)(*[x.numel() for x in xs])
    return ptrs, ns, _current_stream(dev)


def kde_plugin_bandwidth_batch(ctx: int, xs: Sequence) -> List[kde_result]:
    """All samples host (numpy) or all device (torch CUDA float64) arrays."""
    xs = list(xs)
    m = len(xs)
    fast = _device_batch(xs)
    if fast is not None:
        ptrs, ns, stream = fast
        out = (kde_result * m)()
        _check(_lib.kde_plugin_bandwidth_batch(ctx, ptrs, ns, m, KDE_MEM_DEVICE, out, stream),
               "kde_plugin_bandwidth_batch")
        return list(out)
    ss = [_Samples(x if _is_torch(x) else _host_f64(x)) for x in xs]
    mems = {s.mem for s in ss}
    if len(mems) != 1:
        raise ValueError("batch samples must be all host or all device arrays")
    if any(s.dtype != KDE_F64 for s in ss):
        raise TypeError("batch samples must be float64")
    ptrs = (_P * m)(*[s.ptr for s in ss])
    ns = (_I64 * m)(*[s.n for s in ss])
    out = (kde_result * m)()
    stream = ss[0].stream
    _check(_lib.kde_plugin_bandwidth_batch(ctx, ptrs, ns, m, ss[0].mem, out, stream),
           "kde_plugin_bandwidth_batch")
    return list(out)


def kde_plugin_bandwidth_batch_async(ctx: int, xs: Sequence, out) -> None:
    """Enqueue a batch of device samples (torch CUDA float64 tensors) on torch's
    current stream; the results land in ``out`` (a torch tensor in device
    memory or pinned host memory of at least len(xs) * sizeof(kde_result)
    bytes) when the stream gets there.  The caller synchronizes the stream
    and reads them with ``batch_results(out, len(xs))``."""
    ss = [_Samples(x) for x in xs]
    if any(s.mem != KDE_MEM_DEVICE or s.dtype != KDE_F64 for s in ss):
        raise TypeError("asynchronous batches take torch CUDA float64 tensors")
    m = len(ss)
    if out.numel() * out.element_size() < m * ctypes.sizeof(kde_result):
        raise ValueError("output buffer too small")
    ptrs = (_P * m)(*[s.ptr for s in ss])
    ns = (_I64 * m)(*[s.n for s in ss])
    _check(_lib.kde_plugin_bandwidth_batch(ctx, ptrs, ns, m, KDE_MEM_DEVICE,
                                           ctypes.cast(out.data_ptr(), ctypes.POINTER(kde_result)),
                                           ss[0].stream), "kde_plugin_bandwidth_batch")


KDE_NOALLOC_MAX_ITEMS = 262144
KDE_NOALLOC_SCRATCH_BYTES = 13634816


def kde_plugin_bandwidth_noalloc(ctx: int, x, out) -> None:
    """Enqueue one selection of the device sample ``x`` (torch CUDA float64 or
    float32 tensor) on torch's current stream without any allocation by the
    library; the kde_result lands in ``out`` (a torch tensor in device memory
    or pinned host memory of at least sizeof(kde_result) bytes) when the
    stream gets there.  Read it with ``batch_results(out, 1)[0]`` after
    synchronizing the stream."""
    s = _Samples(x)
    if s.mem != KDE_MEM_DEVICE:
        raise TypeError("kde_plugin_bandwidth_noalloc takes a torch CUDA tensor")
    if out.numel() * out.element_size() < ctypes.sizeof(kde_result):
        raise ValueError("output buffer too small")
    _check(_lib.kde_plugin_bandwidth_noalloc(ctx, s.ptr, s.n, s.dtype, s.stream,
                                             ctypes.cast(out.data_ptr(), ctypes.POINTER(kde_result))),
           "kde_plugin_bandwidth_noalloc")


def batch_results(out, count: int) -> List[kde_result]:
    """kde_result records from a buffer written by an asynchronous batch (after
    the caller has synchronized its stream)."""
    host = out.cpu() if out.device.type == "cuda" else out
    raw = bytes(host.contiguous().view(-1).numpy().view(np.uint8)[: count * ctypes.sizeof(kde_result)])
    arr = (kde_result * count).from_buffer_copy(raw)
    return list(arr)


def kde_psi_num_items(ctx: int, n: int) -> int:
    v = _lib.kde_psi_num_items(ctx, int(n))
    if v < 0:
        raise KdeError(kde_last_error(), "kde_psi_num_items")
    return v


def kde_psi_item_geometry(ctx: int, n: int, item: int):
    v = [_I64() for _ in range(4)]
    _check(_lib.kde_psi_item_geometry(ctx, int(n), int(item), *[ctypes.byref(t) for t in v]),
           "kde_psi_item_geometry")
    return tuple(t.value for t in v)


def kde_psi_range(ctx: int, x, r: int, g: float, item_begin: int, item_end: int) -> float:
    s = _Samples(x)
    out = _D()
    _check(_lib.kde_psi_range(ctx, s.ptr, s.n, int(r), float(g), s.mem, s.dtype, int(item_begin),
                              int(item_end), s.stream, ctypes.byref(out)), "kde_psi_range")
    return out.value


def kde_eval(x, y, h: float) -> np.ndarray:
    """Density estimate (equation (1)) at the points y on the default FP64
    context (host arrays)."""
    a = _host_f64(x)
    b = _host_f64(y)
    out = np.empty_like(b)
    _check(_lib.kde_eval(a.ctypes.data_as(ctypes.POINTER(_D)), a.size, b.ctypes.data_as(ctypes.POINTER(_D)),
                         b.size, float(h), out.ctypes.data_as(ctypes.POINTER(_D))), "kde_eval")
    return out


def kde_eval_ex(ctx: int, x, y, h: float):
    """Density estimate at the points y.  A CUDA float64 tensor y gives a CUDA
    tensor result (device path, on the current stream of y's device);
    anything else is taken as host points and gives a numpy array."""
    s = _Samples(x)
    if _is_torch(y) and y.device.type == "cuda":
        torch = _torch()
        yy = y.contiguous()
        if yy.dtype != torch.float64:
            raise TypeError("evaluation points must be float64")
        out = torch.empty_like(yy)
        stream = _current_stream(yy.device)
        _check(_lib.kde_eval_ex(ctx, s.ptr, s.n, s.mem, s.dtype, yy.data_ptr(), yy.numel(), KDE_MEM_DEVICE,
                                float(h), stream, out.data_ptr()), "kde_eval_ex")
        return out
    b = _host_f64(y)
    out = np.empty_like(b)
    _check(_lib.kde_eval_ex(ctx, s.ptr, s.n, s.mem, s.dtype, b.ctypes.data, b.size, KDE_MEM_HOST, float(h),
                            s.stream, out.ctypes.data), "kde_eval_ex")
    return out


def kde_server_options_init() -> kde_server_options:
    o = kde_server_options()
    _lib.kde_server_options_init(ctypes.byref(o))
    return o


def kde_server_create(ctx: int, opts: kde_server_options) -> int:
    h = _P()
    _check(_lib.kde_server_create(ctypes.byref(h), ctx, ctypes.byref(opts)), "kde_server_create")
    return h.value


def kde_server_destroy(srv: int) -> None:
    _lib.kde_server_destroy(srv)


def kde_server_submit(srv: int, ptr: int, n: int, mem_kind: int, producer=None) -> int:
    """producer: the raw HIP stream that writes a device sample (None: the null
    stream); the server's work on the sample is ordered after it."""
    rid = _I64()
    _check(_lib.kde_server_submit(srv, ptr, int(n), int(mem_kind), producer, ctypes.byref(rid)),
           "kde_server_submit")
    return rid.value


def kde_server_cancel(srv: int, rid: int) -> None:
    _check(_lib.kde_server_cancel(srv, int(rid)), "kde_server_cancel")


def kde_server_step(srv: int, block: bool = False) -> kde_server_stats:
    st = kde_server_stats()
    _check(_lib.kde_server_step(srv, int(bool(block)), ctypes.byref(st)), "kde_server_step")
    return st


def kde_server_poll(srv: int, max_items: int = 4096) -> List[kde_completion]:
    buf = (kde_completion * max_items)()
    got = _I32()
    _check(_lib.kde_server_poll(srv, buf, max_items, ctypes.byref(got)), "kde_server_poll")
    return [buf[k] for k in range(got.value)]


def kde_server_drain(srv: int) -> None:
    _check(_lib.kde_server_drain(srv), "kde_server_drain")


def kde_server_fail_next_step(srv: int, code: int) -> None:
    _check(_lib.kde_server_fail_next_step(srv, int(code)), "kde_server_fail_next_step")


KDE_TUNE_SINGLE = 0
KDE_TUNE_BATCH = 1


def kde_autotune(precision: int, ns: Sequence[int], out_path: str, mode: int = KDE_TUNE_SINGLE,
                 reps: int = 5, device: int = 0, verbose: bool = False) -> dict:
    """Run the library's tile-configuration search and return the table."""
    import json
    o = kde_options_init()
    o.device = device
    o.precision = precision
    arr = (_I64 * len(ns))(*[int(v) for v in ns])
    _check(_lib.kde_autotune(ctypes.byref(o), arr, len(ns), int(mode), int(reps), out_path.encode(),
                             int(verbose)), "kde_autotune")
    with open(out_path) as f:
        return json.load(f)


class Context:
    """Owning wrapper of a kde_ctx handle."""

    def __init__(self, precision: int = KDE_FP64_PLAIN, **kw):
        self.handle = kde_ctx_create(precision=precision, **kw)
        self.precision = precision

    def close(self):
        if self.handle:
            kde_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def config(self):
        return kde_ctx_config(self.handle)

    def last_launch(self):
        return kde_ctx_last_launch(self.handle)

    def last_timeline(self, sample: int = 0):
        return kde_ctx_last_timeline(self.handle, sample)

    def last_device_ms(self):
        return kde_ctx_last_device_ms(self.handle)

    def psi(self, x, r, g):
        return kde_psi_ex(self.handle, x, r, g)

    def plugin_bandwidth(self, x, check=True):
        return kde_plugin_bandwidth_ex(self.handle, x, check=check)

    def plugin_bandwidth_batch(self, xs: Iterable):
        return kde_plugin_bandwidth_batch(self.handle, list(xs))

    def plugin_bandwidth_batch_async(self, xs: Iterable, out):
        return kde_plugin_bandwidth_batch_async(self.handle, list(xs), out)

    def plugin_bandwidth_noalloc(self, x, out):
        return kde_plugin_bandwidth_noalloc(self.handle, x, out)

    def psi_num_items(self, n):
        return kde_psi_num_items(self.handle, n)

    def psi_item_geometry(self, n, item):
        return kde_psi_item_geometry(self.handle, n, item)

    def eval(self, x, y, h):
        return kde_eval_ex(self.handle, x, y, h)

    def psi_range(self, x, r, g, b, e):
        return kde_psi_range(self.handle, x, r, g, b, e)
