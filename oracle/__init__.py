"""CPU reference ("oracle") for the integer sorts of arXiv 1808.10292.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  The GPU library never calls it and shares no code with it.

The arithmetic lives in ``sr4.c`` (plain serial C, built with gcc into
``liboracle.so``); this file only marshals numpy arrays through ctypes.

* ``lsd_sort``      -- Section 3.2 SR4 (digit_bits=8) and the serial form of
                       PR2's rounds (digit_bits=16), over a key-bit range.
* ``digit_counts``  -- the counting loop of one count-sort round.
* ``gsd``           -- Section 3.3 Algorithm 1 (GSD) steps 1-5, returning the
                       intermediate split counts and splitters as well.
* ``ger``, ``gvr``   -- Section 3.3 Algorithms 2 and 3 with their random draws
                       passed in as positions.
* ``segmented``     -- SR4 on every CSR segment.
* ``sort_signed_or_float`` -- stable comparison sort of signed integer or IEEE
                       float keys (totalOrder); not in the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sr4.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile sr4.c into liboracle.so with gcc (plain -O2, no tuning)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _configure(lib):
    """Declare the C signatures on a loaded copy of the oracle library."""
    vp, sz, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    for name in ("lsd_u32", "lsd_u64"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, sz, i, i, i, vp, vp]
        f.restype = i
    for name in ("digit_counts_u32", "digit_counts_u64"):
        f = getattr(lib, name)
        f.argtypes = [vp, sz, i, i, vp]
        f.restype = i
    for name in ("segmented_u32", "segmented_u64"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, sz, vp, vp]
        f.restype = i
    lib.gsd_u32.argtypes = [vp, vp, sz, i, i, vp, vp, vp, vp, vp,
                            ctypes.POINTER(ctypes.c_int)]
    lib.gsd_u32.restype = i
    lib.ger_u32.argtypes = [vp, vp, sz, i, i, vp, sz, vp, vp, vp, vp, vp,
                            ctypes.POINTER(ctypes.c_int)]
    lib.ger_u32.restype = i
    lib.sort_kind.argtypes = [vp, vp, sz, i, i]
    lib.sort_kind.restype = i
    lib.gvr_u32.argtypes = [vp, vp, sz, i, i, vp, sz, vp, vp, vp, vp, vp,
                            ctypes.POINTER(ctypes.c_int)]
    lib.gvr_u32.restype = i
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _key_kind(keys: np.ndarray):
    if keys.dtype == np.uint32:
        return "u32", 32
    if keys.dtype == np.uint64:
        return "u64", 64
    raise TypeError("keys must be uint32 or uint64, got %s" % keys.dtype)


def lsd_sort(keys, vals=None, digit_bits: int = 8, begin_bit: int = 0, end_bit=None):
    """Stable LSD radix sort of ``keys`` (uint32/uint64) on bits [begin_bit, end_bit),
    carrying ``vals`` (uint32) along.  Returns (keys_out, vals_out or None)."""
    keys = np.ascontiguousarray(keys)
    kind, width = _key_kind(keys)
    if end_bit is None:
        end_bit = width
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        assert vals.shape == keys.shape
    ko = np.empty_like(keys)
    vo = None if vals is None else np.empty_like(vals)
    f = getattr(_load(), "lsd_" + kind)
    rc = f(_ptr(keys), _ptr(vals), keys.size, digit_bits, begin_bit, end_bit,
           _ptr(ko), _ptr(vo))
    if rc:
        raise ValueError("oracle lsd_%s failed (%d)" % (kind, rc))
    return ko, vo


def sr4(keys, vals=None):
    """SR4: four (u32) or eight (u64) stable count-sort rounds of radix 256."""
    return lsd_sort(keys, vals, 8)


def digit_counts(keys, shift: int, width: int) -> np.ndarray:
    """counts[v] = number of keys whose bits [shift, shift+width) equal v."""
    keys = np.ascontiguousarray(keys)
    kind, _ = _key_kind(keys)
    out = np.empty(1 << width, dtype=np.uint64)
    rc = getattr(_load(), "digit_counts_" + kind)(_ptr(keys), keys.size, shift, width,
                                                 _ptr(out))
    if rc:
        raise ValueError("oracle digit_counts failed (%d)" % rc)
    return out


def segmented(keys, vals, offsets):
    """SR4 applied to each segment [offsets[s], offsets[s+1])."""
    keys = np.ascontiguousarray(keys)
    kind, _ = _key_kind(keys)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
    ko = np.empty_like(keys)
    vo = None if vals is None else np.empty_like(vals)
    rc = getattr(_load(), "segmented_" + kind)(_ptr(keys), _ptr(vals), _ptr(offsets),
                                              offsets.size - 1, _ptr(ko), _ptr(vo))
    if rc:
        raise ValueError("oracle segmented failed (%d)" % rc)
    return ko, vo


def gsd(keys, vals, p: int, r: int):
    """GSD (Algorithm 1) on uint32 keys.  Returns a dict with the sorted
    ``keys``/``vals``, ``p`` actually used (min(p, n)), ``cnt`` (p x p,
    cnt[k, j] = |X_{k,j}|), ``split_key``/``split_g`` (the p-1 splitter
    composites) and ``bucket`` (|Y_j| = column sums of cnt)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    n = keys.size
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
    pmax = max(1, min(p, n))
    ko = np.empty_like(keys)
    vo = None if vals is None else np.empty_like(vals)
    cnt = np.zeros(pmax * pmax, dtype=np.uint64)
    sk = np.zeros(max(pmax - 1, 1), dtype=np.uint32)
    sg = np.zeros(max(pmax - 1, 1), dtype=np.uint64)
    used = ctypes.c_int(0)
    rc = _load().gsd_u32(_ptr(keys), _ptr(vals), n, p, r, _ptr(ko), _ptr(vo), _ptr(cnt),
                         _ptr(sk), _ptr(sg), ctypes.byref(used))
    if rc:
        raise ValueError("oracle gsd failed (%d)" % rc)
    pu = used.value
    cnt = cnt.reshape(pu, pu)
    return {"keys": ko, "vals": vo, "p": pu, "cnt": cnt,
            "split_key": sk[:pu - 1], "split_g": sg[:pu - 1],
            "bucket": cnt.sum(axis=0)}


def gvr(keys, vals, p: int, s: int, positions):
    """GVR (Algorithm 3) on uint32 keys with the random draws given:
    ``positions`` (at least s*min(p, n) - 1, each < n) index the INPUT.
    cnt[k, j] = elements of input block k in bucket j.  Same dict as ``gsd``."""
    return _skeleton_random("gvr_u32", keys, vals, p, s, positions)


def ger(keys, vals, p: int, s: int, positions):
    """GER (Algorithm 2) on uint32 keys with the random draws given:
    ``positions`` (uint32, at least s*min(p, n) - 1 of them, each < n) are the
    sample positions into the locally sorted blocks.  Returns the same dict as
    ``gsd``."""
    return _skeleton_random("ger_u32", keys, vals, p, s, positions)


def _skeleton_random(fn, keys, vals, p: int, s: int, positions):
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    n = keys.size
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
    pos = np.ascontiguousarray(positions, dtype=np.uint32)
    pmax = max(1, min(p, n))
    ko = np.empty_like(keys)
    vo = None if vals is None else np.empty_like(vals)
    cnt = np.zeros(pmax * pmax, dtype=np.uint64)
    sk = np.zeros(max(pmax - 1, 1), dtype=np.uint32)
    sg = np.zeros(max(pmax - 1, 1), dtype=np.uint64)
    used = ctypes.c_int(0)
    rc = getattr(_load(), fn)(_ptr(keys), _ptr(vals), n, p, s, _ptr(pos), pos.size, _ptr(ko),
                              _ptr(vo), _ptr(cnt), _ptr(sk), _ptr(sg), ctypes.byref(used))
    if rc:
        raise ValueError("oracle %s failed (%d)" % (fn, rc))
    pu = used.value
    cnt = cnt.reshape(pu, pu)
    return {"keys": ko, "vals": vo, "p": pu, "cnt": cnt,
            "split_key": sk[:pu - 1], "split_g": sg[:pu - 1],
            "bucket": cnt.sum(axis=0)}


def sort_signed_or_float(keys, vals=None, kind="signed"):
    """Stable sort of int32/int64 (kind "signed") or float32/float64 (kind
    "float", IEEE totalOrder) keys by comparison; returns (keys, vals)."""
    keys = np.ascontiguousarray(keys)
    bits = keys.dtype.itemsize * 8
    k = keys.view(np.uint32 if bits == 32 else np.uint64).astype(np.uint64)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    rc = _load().sort_kind(_ptr(k), _ptr(v), k.size, bits, 1 if kind == "signed" else 2)
    if rc:
        raise ValueError("oracle sort_kind failed (%d)" % rc)
    out = k.astype(np.uint32 if bits == 32 else np.uint64).view(keys.dtype)
    return out, v
