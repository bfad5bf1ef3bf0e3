"""Python binding of the C ABI in include/rsort.h (ctypes; marshalling only).

Every function here converts torch tensors to device pointers and calls the
entry point of the same name in ``librsort.so``; all sorting work runs in the
library's HIP kernels.  If the library is missing the import-time loader raises
instead of falling back to anything else.

torch is imported before the library is loaded so that the library binds to
the HIP runtime torch already mapped (both carry the same soname), which makes
torch's device pointers and streams valid handles for the library.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsort.so")

RSORT_OK = 0
RSORT_EINVAL = -1
RSORT_ENOMEM = -2
RSORT_EDEVICE = -3
RSORT_EBUSY = -4
RSORT_EUNSUPPORTED = -5

RSORT_U32 = 0
RSORT_U64 = 1
RSORT_I32 = 2
RSORT_F32 = 3
RSORT_I64 = 4
RSORT_F64 = 5
KEY_TYPES = {"u32": RSORT_U32, "u64": RSORT_U64, "i32": RSORT_I32, "f32": RSORT_F32,
             "i64": RSORT_I64, "f64": RSORT_F64}

RSORT_AUTO = 0
RSORT_LSD_R8 = 1
RSORT_LSD_R16 = 2
RSORT_SAMPLE_REGULAR = 3

ALGOS = {"auto": RSORT_AUTO, "lsd8": RSORT_LSD_R8, "pr4": RSORT_LSD_R8,
         "lsd16": RSORT_LSD_R16, "pr2": RSORT_LSD_R16,
         "sample": RSORT_SAMPLE_REGULAR, "gsd": RSORT_SAMPLE_REGULAR}

# Every symbol include/rsort.h declares; the loader checks they all exist.
EXPORTED = ("rsort_create", "rsort_destroy", "rsort_status_string", "rsort_last_error",
            "rsort_workspace_bytes", "rsort_sort", "rsort_sort_noalloc", "rsort_set_pr4_rounds",
            "rsort_histogram",
            "rsort_synchronize",
            "rsort_profile_enable", "rsort_profile_read", "rsort_profile_set_period",
            "rsort_segmented_sort",
            "rsort_segmented_workspace_bytes", "rsort_segmented_set_split",
            "rsort_segmented_tune", "rsort_segmented_set_small_sort",
            "rsort_segmented_get_small_sort", "rsort_segmented_set_tile",
            "rsort_segmented_get_config", "rsort_segmented_set_launch", "rsort_set_tune_cache",
            "rsort_debug_fail_alloc", "rsort_sample_sort", "rsort_sample_sort_workspace_bytes",
            "rsort_sample_sort_stats", "rsort_sample_sort_random",
            "rsort_sample_sort_random_workspace_bytes", "rsort_sample_sort_gvr",
            "rsort_sample_sort_gvr_workspace_bytes", "rsort_segmented_sort_device",
            "rsort_segmented_device_workspace_bytes", "rsort_server_create", "rsort_server_submit",
            "rsort_server_submit_async", "rsort_server_reserve", "rsort_server_memory",
            "rsort_server_fail_next",
            "rsort_server_poll", "rsort_server_wait", "rsort_server_latency",
            "rsort_server_reset_stats", "rsort_server_destroy")

RSORT_PR4_COUNTED = 0
RSORT_PR4_SINGLE_READ = 1
PR4_ROUNDS = {"counted": RSORT_PR4_COUNTED, "single_read": RSORT_PR4_SINGLE_READ}

RSORT_SMALL_RADIX = 0
RSORT_SMALL_BTN = 1
RSORT_SMALL_OET = 2
SMALL_SORTS = {"radix": RSORT_SMALL_RADIX, "btn": RSORT_SMALL_BTN, "oet": RSORT_SMALL_OET}

RSORT_KERNEL_ROUND = 0
RSORT_KERNEL_HIST = 1
RSORT_KERNEL_COUNT = 2
RSORT_KERNEL_TILESCAN = 3
RSORT_KERNEL_SMALL = 4
RSORT_KERNEL_GROUP = 5


class RsortError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = "%s failed: %s (%d)" % (where, _status_string(status), status)
        if detail:
            msg += ": " + detail
        super().__init__(msg)


_lib = None
_lib_lock = threading.Lock()


def load_library():
    """Load librsort.so and declare the C signatures.  Raises if it is absent."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError("HIP library %s is not built; run "
                              "`python -m paper_1808_10292_amd.build`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        vp, sz, i, u32p = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p
        for name in EXPORTED:
            getattr(lib, name)  # AttributeError if a declared symbol is missing
        lib.rsort_create.argtypes = [i, ctypes.POINTER(vp)]
        lib.rsort_destroy.argtypes = [vp]
        lib.rsort_status_string.argtypes = [i]
        lib.rsort_status_string.restype = ctypes.c_char_p
        lib.rsort_last_error.argtypes = [vp]
        lib.rsort_last_error.restype = ctypes.c_char_p
        lib.rsort_workspace_bytes.argtypes = [vp, i, i, sz, i, ctypes.POINTER(sz)]
        lib.rsort_sort.argtypes = [vp, i, vp, vp, u32p, u32p, sz, i, i, i, vp, sz, vp]
        lib.rsort_histogram.argtypes = [vp, i, vp, sz, i, i, i, u32p, vp]
        lib.rsort_set_pr4_rounds.argtypes = [vp, i]
        lib.rsort_sort_noalloc.argtypes = [vp, i, vp, vp, u32p, u32p, sz, i, i, vp]
        lib.rsort_synchronize.argtypes = [vp, vp]
        lib.rsort_profile_enable.argtypes = [vp, i]
        lib.rsort_profile_set_period.argtypes = [vp, ctypes.c_uint32]
        lib.rsort_segmented_sort.argtypes = [vp, i, vp, vp, u32p, u32p, vp, sz, vp, sz, vp]
        lib.rsort_segmented_workspace_bytes.argtypes = [vp, i, i, vp, sz, ctypes.POINTER(sz)]
        lib.rsort_segmented_set_split.argtypes = [vp, ctypes.c_uint32]
        lib.rsort_segmented_set_small_sort.argtypes = [vp, i]
        lib.rsort_segmented_get_small_sort.argtypes = [vp, ctypes.POINTER(i)]
        lib.rsort_segmented_set_tile.argtypes = [vp, i]
        lib.rsort_segmented_set_launch.argtypes = [vp, i]
        lib.rsort_segmented_get_config.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32),
                                                   ctypes.POINTER(i), ctypes.POINTER(i),
                                                   ctypes.POINTER(i), ctypes.POINTER(i)]
        lib.rsort_segmented_tune.argtypes = [vp, i, vp, vp, u32p, u32p, vp, sz, i, vp,
                                             ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(ctypes.c_double)]
        lib.rsort_set_tune_cache.argtypes = [vp, ctypes.c_char_p]
        lib.rsort_debug_fail_alloc.argtypes = [i]
        lib.rsort_sample_sort.argtypes = [vp, i, vp, vp, u32p, u32p, sz, i, i, vp, sz, vp]
        lib.rsort_sample_sort_workspace_bytes.argtypes = [vp, i, i, sz, i, i, ctypes.POINTER(sz)]
        lib.rsort_sample_sort_stats.argtypes = [vp, i, ctypes.POINTER(i), vp, vp, vp, vp]
        lib.rsort_sample_sort_random.argtypes = [vp, i, vp, vp, u32p, u32p, sz, i, i,
                                                 ctypes.c_uint64, vp, sz, vp]
        lib.rsort_sample_sort_random_workspace_bytes.argtypes = [vp, i, i, sz, i, i,
                                                                 ctypes.POINTER(sz)]
        lib.rsort_sample_sort_gvr.argtypes = lib.rsort_sample_sort_random.argtypes
        lib.rsort_sample_sort_gvr_workspace_bytes.argtypes = \
            lib.rsort_sample_sort_random_workspace_bytes.argtypes
        lib.rsort_segmented_sort_device.argtypes = [vp, i, vp, vp, u32p, u32p, vp, sz, sz, vp, sz,
                                                    vp]
        lib.rsort_segmented_device_workspace_bytes.argtypes = [vp, i, i, sz, sz, ctypes.POINTER(sz)]
        lib.rsort_server_create.argtypes = [i, sz, i, ctypes.POINTER(vp)]
        lib.rsort_server_submit.argtypes = [vp, i, vp, vp, sz, ctypes.POINTER(ctypes.c_uint64)]
        lib.rsort_server_submit_async.argtypes = [vp, i, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_uint64)]
        lib.rsort_server_reserve.argtypes = [vp, i, sz]
        lib.rsort_server_fail_next.argtypes = [vp]
        lib.rsort_server_memory.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
        lib.rsort_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i)]
        lib.rsort_server_wait.argtypes = [vp, ctypes.c_uint64]
        lib.rsort_server_latency.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_uint64)]
        lib.rsort_server_reset_stats.argtypes = [vp]
        lib.rsort_server_destroy.argtypes = [vp]
        lib.rsort_profile_read.argtypes = [vp, i, ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_double)]
        for name in EXPORTED:
            f = getattr(lib, name)
            if f.restype is ctypes.c_int or f.restype is None:
                f.restype = i
        lib.rsort_status_string.restype = ctypes.c_char_p
        lib.rsort_last_error.restype = ctypes.c_char_p
        _lib = lib
        return lib


def _status_string(status: int) -> str:
    try:
        return load_library().rsort_status_string(status).decode()
    except Exception:  # noqa: BLE001 - only used to format an error
        return "status"


class Context:
    """An rsort_ctx bound to one HIP device."""

    def __init__(self, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        rc = lib.rsort_create(int(device), ctypes.byref(h))
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_create")
        self.handle = h
        self.device = int(device)
        self._lib = lib

    def check(self, rc: int, where: str):
        if rc != RSORT_OK:
            detail = self._lib.rsort_last_error(self.handle).decode()
            raise RsortError(rc, where, detail)

    def close(self):
        if self.handle:
            self._lib.rsort_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


_contexts: dict = {}


def context(device=None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if isinstance(device, torch.device):
        device = device.index if device.index is not None else torch.cuda.current_device()
    ctx = _contexts.get(device)
    if ctx is None:
        ctx = _contexts[device] = Context(device)
    return ctx


def _key_type(t: torch.Tensor, key_type=None) -> int:
    """Integer tensors sort their bit patterns as unsigned unless key_type
    ("i32", "i64", ...) says otherwise; float32 / float64 sort by IEEE
    totalOrder."""
    if key_type is not None:
        kt = KEY_TYPES[key_type] if isinstance(key_type, str) else int(key_type)
        width = 4 if kt in (RSORT_U32, RSORT_I32, RSORT_F32) else 8
        if t.element_size() != width:
            raise TypeError("key_type %s needs %d-byte elements, got %s" % (key_type, width, t.dtype))
        return kt
    if t.dtype in (torch.int32, torch.uint32):
        return RSORT_U32
    if t.dtype in (torch.int64, torch.uint64):
        return RSORT_U64
    if t.dtype == torch.float32:
        return RSORT_F32
    if t.dtype == torch.float64:
        return RSORT_F64
    raise TypeError("keys must be a 32- or 64-bit integer or float tensor, got %s" % t.dtype)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_tensor(t, n, name):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be contiguous with %d elements" % (name, n))


# ---------------------------------------------------------------------------
# Entry points under their C names.

def rsort_workspace_bytes(key_dtype, has_vals: bool, n: int, algo="auto", device=None,
                          key_type=None) -> int:
    ctx = context(device)
    kt = _key_type(torch.empty(0, dtype=key_dtype), key_type)
    out = ctypes.c_size_t()
    ctx.check(ctx._lib.rsort_workspace_bytes(ctx.handle, kt, int(bool(has_vals)), int(n),
                                             ALGOS[algo] if isinstance(algo, str) else int(algo),
                                             ctypes.byref(out)), "rsort_workspace_bytes")
    return out.value


def rsort_sort(keys_in, keys_out, vals_in=None, vals_out=None, begin_bit=0, end_bit=None,
               algo="auto", workspace=None, stream=None, key_type=None):
    """Stable sort of keys_in into keys_out (may be the same tensor).
    key_type: "u32" / "u64" (default for integer tensors), "i32" / "i64"
    (signed), "f32" / "f64" (default for float tensors)."""
    kt = _key_type(keys_in, key_type)
    n = keys_in.numel()
    if keys_out.dtype != keys_in.dtype:
        raise TypeError("keys_out must have the dtype of keys_in")
    _check_tensor(keys_in, n, "keys_in")
    _check_tensor(keys_out, n, "keys_out")
    if (vals_in is None) != (vals_out is None):
        raise ValueError("vals_in and vals_out must both be given or both be None")
    if vals_in is not None:
        for t, name in ((vals_in, "vals_in"), (vals_out, "vals_out")):
            if t.dtype not in (torch.int32, torch.uint32):
                raise TypeError("%s must be a 32-bit integer tensor" % name)
            _check_tensor(t, n, name)
    if end_bit is None:
        end_bit = 8 * keys_in.element_size()
    ctx = context(keys_in.device)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = _ptr(workspace), workspace.numel() * workspace.element_size()
    rc = ctx._lib.rsort_sort(ctx.handle, kt, _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                             _ptr(vals_out), n, int(begin_bit), int(end_bit),
                             ALGOS[algo] if isinstance(algo, str) else int(algo),
                             ws_ptr, ws_bytes, _stream_handle(stream))
    ctx.check(rc, "rsort_sort")
    return keys_out, vals_out


def rsort_sort_noalloc(keys_in, keys_out, vals_in=None, vals_out=None, begin_bit=0, end_bit=None,
                       stream=None, key_type=None):
    """rsort_sort (radix 2^8) with the library's own scratch array as workspace:
    the call allocates nothing.  Arguments as in rsort_sort."""
    kt = _key_type(keys_in, key_type)
    n = keys_in.numel()
    if keys_out.dtype != keys_in.dtype:
        raise TypeError("keys_out must have the dtype of keys_in")
    _check_tensor(keys_in, n, "keys_in")
    _check_tensor(keys_out, n, "keys_out")
    if (vals_in is None) != (vals_out is None):
        raise ValueError("vals_in and vals_out must both be given or both be None")
    if vals_in is not None:
        for t, name in ((vals_in, "vals_in"), (vals_out, "vals_out")):
            if t.dtype not in (torch.int32, torch.uint32):
                raise TypeError("%s must be a 32-bit integer tensor" % name)
            _check_tensor(t, n, name)
    if end_bit is None:
        end_bit = 8 * keys_in.element_size()
    ctx = context(keys_in.device)
    rc = ctx._lib.rsort_sort_noalloc(ctx.handle, kt, _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                     _ptr(vals_out), n, int(begin_bit), int(end_bit),
                                     _stream_handle(stream))
    ctx.check(rc, "rsort_sort_noalloc")
    return keys_out, vals_out


def rsort_set_pr4_rounds(kind, device=None):
    """Round kind of RSORT_LSD_R8: "counted" (default) or "single_read"."""
    ctx = context(device)
    ctx.check(ctx._lib.rsort_set_pr4_rounds(ctx.handle, PR4_ROUNDS[kind] if isinstance(kind, str)
                                            else int(kind)), "rsort_set_pr4_rounds")


def rsort_histogram(keys, digit_bits=8, begin_bit=0, end_bit=None, out=None, stream=None):
    """Counts of every digit of every count-sort round, shape (rounds, 2^digit_bits)."""
    kt = _key_type(keys)
    if end_bit is None:
        end_bit = 32 if kt == RSORT_U32 else 64
    rounds = (end_bit - begin_bit + digit_bits - 1) // digit_bits if end_bit > begin_bit else 0
    if out is None:
        out = torch.zeros((rounds, 1 << digit_bits), dtype=torch.int32, device=keys.device)
    ctx = context(keys.device)
    rc = ctx._lib.rsort_histogram(ctx.handle, kt, _ptr(keys), keys.numel(), int(digit_bits),
                                  int(begin_bit), int(end_bit), _ptr(out), _stream_handle(stream))
    ctx.check(rc, "rsort_histogram")
    return out


def rsort_synchronize(stream=None, device=None):
    ctx = context(device)
    ctx.check(ctx._lib.rsort_synchronize(ctx.handle, _stream_handle(stream)),
              "rsort_synchronize")


def rsort_profile_enable(enable=True, kinds=None, device=None):
    """Start (or stop, enable=False) kernel timing; kinds: iterable of
    RSORT_KERNEL_* values to time (default: every kind)."""
    ctx = context(device)
    mask = 0
    if enable:
        mask = -1 if kinds is None else sum(1 << int(k) for k in set(kinds))
    ctx.check(ctx._lib.rsort_profile_enable(ctx.handle, int(mask)), "rsort_profile_enable")


def rsort_profile_set_period(period, device=None):
    """Time only launches 0, period, 2 period, ... of each timed kind."""
    ctx = context(device)
    ctx.check(ctx._lib.rsort_profile_set_period(ctx.handle, int(period)),
              "rsort_profile_set_period")


def rsort_profile_read(kind=RSORT_KERNEL_ROUND, device=None):
    """(timed launches, summed milliseconds) for one kernel kind."""
    ctx = context(device)
    launches = ctypes.c_uint64()
    ms = ctypes.c_double()
    ctx.check(ctx._lib.rsort_profile_read(ctx.handle, int(kind), ctypes.byref(launches),
                                          ctypes.byref(ms)), "rsort_profile_read")
    return launches.value, ms.value


def _host_offsets(seg_offsets):
    import numpy as np
    off = np.ascontiguousarray(np.asarray(seg_offsets, dtype=np.uint64))
    if off.ndim != 1 or off.size < 1:
        raise ValueError("seg_offsets must be a 1-D array of num_segs + 1 offsets")
    return off


def rsort_segmented_sort(keys_in, keys_out, seg_offsets, vals_in=None, vals_out=None,
                         workspace=None, stream=None):
    """Sort every segment [off[s], off[s+1]) of keys_in independently into keys_out.
    seg_offsets: host sequence (numpy/list) of num_segs + 1 offsets."""
    kt = _key_type(keys_in)
    off = _host_offsets(seg_offsets)
    n = keys_in.numel()
    if int(off[-1]) > n:
        raise ValueError("seg_offsets end beyond the key array")
    _check_tensor(keys_in, n, "keys_in")
    _check_tensor(keys_out, n, "keys_out")
    if (vals_in is None) != (vals_out is None):
        raise ValueError("vals_in and vals_out must both be given or both be None")
    if vals_in is not None:
        _check_tensor(vals_in, n, "vals_in")
        _check_tensor(vals_out, n, "vals_out")
    ctx = context(keys_in.device)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = _ptr(workspace), workspace.numel() * workspace.element_size()
    rc = ctx._lib.rsort_segmented_sort(ctx.handle, kt, _ptr(keys_in), _ptr(keys_out),
                                       _ptr(vals_in), _ptr(vals_out),
                                       ctypes.c_void_p(off.ctypes.data), off.size - 1,
                                       ws_ptr, ws_bytes, _stream_handle(stream))
    ctx.check(rc, "rsort_segmented_sort")
    return keys_out, vals_out


def rsort_segmented_workspace_bytes(key_dtype, has_vals, seg_offsets, device=None):
    ctx = context(device)
    kt = _key_type(torch.empty(0, dtype=key_dtype))
    off = _host_offsets(seg_offsets)
    out = ctypes.c_size_t()
    ctx.check(ctx._lib.rsort_segmented_workspace_bytes(ctx.handle, kt, int(bool(has_vals)),
                                                       ctypes.c_void_p(off.ctypes.data),
                                                       off.size - 1, ctypes.byref(out)),
              "rsort_segmented_workspace_bytes")
    return out.value


def rsort_segmented_sort_device(keys_in, keys_out, seg_offsets, vals_in=None, vals_out=None,
                                workspace=None, stream=None):
    """Segmented sort with the offsets in a device tensor (int32/uint32,
    num_segs + 1 entries)."""
    kt = _key_type(keys_in)
    n = _check_kv(keys_in, keys_out, vals_in, vals_out)
    if not seg_offsets.is_cuda or seg_offsets.dtype not in (torch.int32, torch.uint32) or \
            not seg_offsets.is_contiguous() or seg_offsets.dim() != 1 or seg_offsets.numel() < 1:
        raise ValueError("seg_offsets must be a contiguous 1-D 32-bit device tensor")
    ctx = context(keys_in.device)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = _ptr(workspace), workspace.numel() * workspace.element_size()
    rc = ctx._lib.rsort_segmented_sort_device(ctx.handle, kt, _ptr(keys_in), _ptr(keys_out),
                                              _ptr(vals_in), _ptr(vals_out), _ptr(seg_offsets),
                                              seg_offsets.numel() - 1, n, ws_ptr, ws_bytes,
                                              _stream_handle(stream))
    ctx.check(rc, "rsort_segmented_sort_device")
    return keys_out, vals_out


def rsort_segmented_device_workspace_bytes(key_dtype, has_vals, num_segs, total_n, device=None):
    ctx = context(device)
    kt = _key_type(torch.empty(0, dtype=key_dtype))
    out = ctypes.c_size_t()
    ctx.check(ctx._lib.rsort_segmented_device_workspace_bytes(ctx.handle, kt, int(bool(has_vals)),
                                                              int(num_segs), int(total_n),
                                                              ctypes.byref(out)),
              "rsort_segmented_device_workspace_bytes")
    return out.value


def rsort_segmented_set_split(small_max, device=None):
    ctx = context(device)
    ctx.check(ctx._lib.rsort_segmented_set_split(ctx.handle, int(small_max)),
              "rsort_segmented_set_split")


def rsort_segmented_set_small_sort(small_sort, device=None):
    """Sorter of the small segments: "radix", "btn", "oet" (or RSORT_SMALL_*)."""
    ctx = context(device)
    v = SMALL_SORTS[small_sort] if isinstance(small_sort, str) else int(small_sort)
    ctx.check(ctx._lib.rsort_segmented_set_small_sort(ctx.handle, v),
              "rsort_segmented_set_small_sort")


def rsort_segmented_get_small_sort(device=None):
    ctx = context(device)
    out = ctypes.c_int()
    ctx.check(ctx._lib.rsort_segmented_get_small_sort(ctx.handle, ctypes.byref(out)),
              "rsort_segmented_get_small_sort")
    return out.value


def rsort_segmented_set_tile(tile_threads, device=None):
    """Tile workgroup of the large segments' rounds: 256, 512 or 1024 threads
    (0 = default)."""
    ctx = context(device)
    ctx.check(ctx._lib.rsort_segmented_set_tile(ctx.handle, int(tile_threads)),
              "rsort_segmented_set_tile")


SEG_LAUNCHES = {"rounds": 0, "persistent": 1}


def rsort_segmented_set_launch(launch, device=None):
    """Launch mode of the segmented sort with host offsets: "rounds" (kernels
    per round, default) or "persistent" (one persistent launch)."""
    ctx = context(device)
    code = SEG_LAUNCHES[launch] if isinstance(launch, str) else int(launch)
    ctx.check(ctx._lib.rsort_segmented_set_launch(ctx.handle, code), "rsort_segmented_set_launch")


def rsort_segmented_get_config(device=None):
    """dict(split, small_sort, tile_threads, radix_bits, launch) of the
    segmented sort."""
    ctx = context(device)
    sm, ss, tt, rb, ln = (ctypes.c_uint32(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(),
                          ctypes.c_int())
    ctx.check(ctx._lib.rsort_segmented_get_config(ctx.handle, ctypes.byref(sm), ctypes.byref(ss),
                                                  ctypes.byref(tt), ctypes.byref(rb),
                                                  ctypes.byref(ln)),
              "rsort_segmented_get_config")
    names = {v: k for k, v in SMALL_SORTS.items()}
    launches = {v: k for k, v in SEG_LAUNCHES.items()}
    return {"split": sm.value, "small_sort": names.get(ss.value, ss.value),
            "tile_threads": tt.value, "radix_bits": rb.value,
            "launch": launches.get(ln.value, ln.value)}


def rsort_segmented_tune(keys_in, keys_out, seg_offsets, vals_in=None, vals_out=None, reps=3,
                         stream=None):
    """Pick the fastest small/large split, small-segment sorter and tile
    workgroup of the large path for this batch (all left set); returns
    (split, ms) -- the rest through rsort_segmented_get_config()."""
    kt = _key_type(keys_in)
    off = _host_offsets(seg_offsets)
    ctx = context(keys_in.device)
    split = ctypes.c_uint32()
    ms = ctypes.c_double()
    rc = ctx._lib.rsort_segmented_tune(ctx.handle, kt, _ptr(keys_in), _ptr(keys_out),
                                       _ptr(vals_in), _ptr(vals_out),
                                       ctypes.c_void_p(off.ctypes.data), off.size - 1, int(reps),
                                       _stream_handle(stream), ctypes.byref(split),
                                       ctypes.byref(ms))
    ctx.check(rc, "rsort_segmented_tune")
    return split.value, ms.value


def rsort_set_tune_cache(path, device=None):
    """Tune cache file of the device's context (None: none); see include/rsort.h."""
    ctx = context(device)
    arg = None if path is None else os.fsencode(path)
    ctx.check(ctx._lib.rsort_set_tune_cache(ctx.handle, arg), "rsort_set_tune_cache")


def rsort_debug_fail_alloc(k):
    """Make the k-th device allocation of the library from now on fail as out
    of memory (0 disarms); a test hook for the error paths."""
    lib = load_library()
    rc = lib.rsort_debug_fail_alloc(int(k))
    if rc:
        raise RsortError(rc, "rsort_debug_fail_alloc")


def _check_kv(keys_in, keys_out, vals_in, vals_out):
    n = keys_in.numel()
    if keys_out.dtype != keys_in.dtype:
        raise TypeError("keys_out must have the dtype of keys_in")
    _check_tensor(keys_in, n, "keys_in")
    _check_tensor(keys_out, n, "keys_out")
    if (vals_in is None) != (vals_out is None):
        raise ValueError("vals_in and vals_out must both be given or both be None")
    if vals_in is not None:
        for t, name in ((vals_in, "vals_in"), (vals_out, "vals_out")):
            if t.dtype not in (torch.int32, torch.uint32):
                raise TypeError("%s must be a 32-bit integer tensor" % name)
            _check_tensor(t, n, name)
    return n


def rsort_sample_sort(keys_in, keys_out, vals_in=None, vals_out=None, p=256, r=32,
                      workspace=None, stream=None):
    """GSD sample sort (p buckets, oversampling factor r) of 32-bit keys."""
    kt = _key_type(keys_in)
    n = _check_kv(keys_in, keys_out, vals_in, vals_out)
    ctx = context(keys_in.device)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = _ptr(workspace), workspace.numel() * workspace.element_size()
    rc = ctx._lib.rsort_sample_sort(ctx.handle, kt, _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                    _ptr(vals_out), n, int(p), int(r), ws_ptr, ws_bytes,
                                    _stream_handle(stream))
    ctx.check(rc, "rsort_sample_sort")
    return keys_out, vals_out


def rsort_sample_sort_workspace_bytes(key_dtype, has_vals, n, p=256, r=32, device=None):
    ctx = context(device)
    kt = _key_type(torch.empty(0, dtype=key_dtype))
    out = ctypes.c_size_t()
    ctx.check(ctx._lib.rsort_sample_sort_workspace_bytes(ctx.handle, kt, int(bool(has_vals)),
                                                         int(n), int(p), int(r),
                                                         ctypes.byref(out)),
              "rsort_sample_sort_workspace_bytes")
    return out.value


def _random_sample_sort(name, keys_in, keys_out, vals_in, vals_out, p, s, seed, workspace,
                        stream):
    kt = _key_type(keys_in)
    n = _check_kv(keys_in, keys_out, vals_in, vals_out)
    ctx = context(keys_in.device)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = _ptr(workspace), workspace.numel() * workspace.element_size()
    rc = getattr(ctx._lib, name)(ctx.handle, kt, _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                 _ptr(vals_out), n, int(p), int(s),
                                 int(seed) & 0xFFFFFFFFFFFFFFFF, ws_ptr, ws_bytes,
                                 _stream_handle(stream))
    ctx.check(rc, name)
    return keys_out, vals_out


def _random_sample_ws(name, key_dtype, has_vals, n, p, s, device):
    ctx = context(device)
    kt = _key_type(torch.empty(0, dtype=key_dtype))
    out = ctypes.c_size_t()
    ctx.check(getattr(ctx._lib, name)(ctx.handle, kt, int(bool(has_vals)), int(n), int(p),
                                      int(s), ctypes.byref(out)), name)
    return out.value


def rsort_sample_sort_random(keys_in, keys_out, vals_in=None, vals_out=None, p=256, s=0,
                             seed=0x18081029, workspace=None, stream=None):
    """GER sample sort (p buckets, s p - 1 random sample keys, s = 0: default)."""
    return _random_sample_sort("rsort_sample_sort_random", keys_in, keys_out, vals_in, vals_out,
                               p, s, seed, workspace, stream)


def rsort_sample_sort_random_workspace_bytes(key_dtype, has_vals, n, p=256, s=0, device=None):
    return _random_sample_ws("rsort_sample_sort_random_workspace_bytes", key_dtype, has_vals, n,
                             p, s, device)


def rsort_sample_sort_gvr(keys_in, keys_out, vals_in=None, vals_out=None, p=256, s=0,
                          seed=0x18081029, workspace=None, stream=None):
    """GVR sample sort (p <= 256 buckets, s p - 1 random input positions,
    s = 0: default)."""
    return _random_sample_sort("rsort_sample_sort_gvr", keys_in, keys_out, vals_in, vals_out, p,
                               s, seed, workspace, stream)


def rsort_sample_sort_gvr_workspace_bytes(key_dtype, has_vals, n, p=256, s=0, device=None):
    return _random_sample_ws("rsort_sample_sort_gvr_workspace_bytes", key_dtype, has_vals, n, p,
                             s, device)


def rsort_sample_sort_stats(p_cap=1024, device=None):
    """Split of the last sample sort: dict with p, cnt (p x p), bucket (p),
    split_key and split_index (p - 1), as numpy uint32 arrays."""
    import numpy as np
    ctx = context(device)
    used = ctypes.c_int()
    cnt = np.zeros(p_cap * p_cap, dtype=np.uint32)
    bucket = np.zeros(p_cap, dtype=np.uint32)
    sk = np.zeros(p_cap, dtype=np.uint32)
    si = np.zeros(p_cap, dtype=np.uint32)
    rc = ctx._lib.rsort_sample_sort_stats(ctx.handle, int(p_cap), ctypes.byref(used),
                                          ctypes.c_void_p(cnt.ctypes.data),
                                          ctypes.c_void_p(bucket.ctypes.data),
                                          ctypes.c_void_p(sk.ctypes.data),
                                          ctypes.c_void_p(si.ctypes.data))
    ctx.check(rc, "rsort_sample_sort_stats")
    p = used.value
    return {"p": p, "cnt": cnt[:p * p].reshape(p, p), "bucket": bucket[:p],
            "split_key": sk[:max(p - 1, 0)], "split_index": si[:max(p - 1, 0)]}


class Server:
    """rsort_server: continuous-batching sort server on one device.  Methods
    carry the C names without the prefix; submit takes torch tensors and keeps
    references to them until the request is waited on."""

    def __init__(self, hbm_cap_bytes, num_streams=4, device=None):
        lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        rc = lib.rsort_server_create(int(device), int(hbm_cap_bytes), int(num_streams),
                                     ctypes.byref(h))
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_create")
        self.handle = h
        self._lib = lib
        self._held = {}
        self._lock = threading.Lock()

    def submit(self, keys_in, keys_out, stream=None):
        """Queue a sort that starts after the work already enqueued on `stream`
        (default: torch's current stream), e.g. the kernel that wrote keys_in."""
        kt = _key_type(keys_in)
        n = keys_in.numel()
        if keys_out.dtype != keys_in.dtype:
            raise TypeError("keys_out must have the dtype of keys_in")
        _check_tensor(keys_in, n, "keys_in")
        _check_tensor(keys_out, n, "keys_out")
        t = ctypes.c_uint64()
        rc = self._lib.rsort_server_submit_async(self.handle, kt, _ptr(keys_in), _ptr(keys_out), n,
                                                 _stream_handle(stream), ctypes.byref(t))
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_submit_async")
        with self._lock:
            self._held[t.value] = (keys_in, keys_out)
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int()
        rc = self._lib.rsort_server_poll(self.handle, int(ticket), ctypes.byref(done))
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_poll")
        if done.value:
            with self._lock:
                self._held.pop(int(ticket), None)
        return bool(done.value)

    def wait(self, ticket):
        rc = self._lib.rsort_server_wait(self.handle, int(ticket))
        with self._lock:
            self._held.pop(int(ticket), None)
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_wait")

    def latency(self):
        """(p50 us, p99 us, keys/s, completed requests)"""
        p50, p99, kps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        done = ctypes.c_uint64()
        rc = self._lib.rsort_server_latency(self.handle, ctypes.byref(p50), ctypes.byref(p99),
                                            ctypes.byref(kps), ctypes.byref(done))
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_latency")
        return p50.value, p99.value, kps.value, done.value

    def reserve(self, key_type, max_n):
        """Allocate every slot's workspace for requests of up to max_n keys now."""
        rc = self._lib.rsort_server_reserve(self.handle, KEY_TYPES[key_type], int(max_n))
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_reserve")

    def fail_next(self):
        """Test hook: the next radix-path request completes with RSORT_EDEVICE."""
        rc = self._lib.rsort_server_fail_next(self.handle)
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_fail_next")

    def memory(self):
        """(bytes in flight, max bytes in flight, bytes the server holds)"""
        a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        rc = self._lib.rsort_server_memory(self.handle, ctypes.byref(a), ctypes.byref(b),
                                           ctypes.byref(c))
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_memory")
        return a.value, b.value, c.value

    def reset_stats(self):
        rc = self._lib.rsort_server_reset_stats(self.handle)
        if rc != RSORT_OK:
            raise RsortError(rc, "rsort_server_reset_stats")

    def destroy(self):
        if self.handle:
            self._lib.rsort_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


# ---------------------------------------------------------------------------
# Convenience wrapper.

def sort(keys, values=None, algo="auto", begin_bit=0, end_bit=None, stream=None, key_type=None):
    """Return (sorted_keys, moved_values or None) as new tensors."""
    ko = torch.empty_like(keys)
    vo = None if values is None else torch.empty_like(values)
    rsort_sort(keys, ko, values, vo, begin_bit, end_bit, algo, stream=stream, key_type=key_type)
    return ko, vo
