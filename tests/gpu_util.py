"""Helpers for the GPU parity tests: move numpy arrays to the device and back
with their exact bit patterns, and print which case is about to run."""
import sys

import numpy as np


def announce(*parts):
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t) -> np.ndarray:
    return t.cpu().numpy()


def check_kv_invariants(keys_in, keys_out, vals_out):
    """With vals = original index these four facts prove keys_out/vals_out is
    the unique stable sort of keys_in (no oracle needed, any size)."""
    n = keys_in.size
    assert keys_out.size == n and vals_out.size == n
    if n == 0:
        return
    assert np.all(keys_out[1:] >= keys_out[:-1]), "not nondecreasing"
    assert int(vals_out.max()) < n
    seen = np.zeros(n, dtype=bool)
    seen[vals_out] = True
    assert seen.all(), "payload is not a permutation"
    assert np.array_equal(keys_out, keys_in[vals_out]), "payload does not travel with its key"
    tie = keys_out[1:] == keys_out[:-1]
    assert np.all(vals_out[1:][tie] > vals_out[:-1][tie]), "ties not in input order"
