"""GPU parity of signed and floating-point keys (rsort_sort with RSORT_I32,
RSORT_F32, RSORT_I64, RSORT_F64) against the oracle's comparison sort
(two's complement order; IEEE totalOrder for floats: -NaN < -inf < ... < -0 <
+0 < ... < +inf < +NaN).  Bit-exact on keys and payloads: radix 2^8 and 2^16,
in place and not, one to many tiles, special values, and argument errors.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 77, 8192, 8193, 100003, (1 << 20) + 3]


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    return rsort


def make_keys(dtype, n, seed):
    rng = np.random.default_rng(seed)
    if np.issubdtype(dtype, np.integer):
        info = np.iinfo(dtype)
        k = rng.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
        if n > 8:
            k[:4] = [info.min, info.max, 0, -1]
    else:
        k = (rng.standard_normal(n) * 1e3).astype(dtype)
        if n > 16:
            k[::7] = np.round(k[::7])                  # duplicates, and some -0.0
            k[:10] = [0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, 1.0, -1.0,
                      np.finfo(dtype).tiny, -np.finfo(dtype).tiny]
    if n > 64:
        k[n // 2: n // 2 + 32] = k[5]                  # a run of equal keys
    return k


def as_tensor(k):
    """Device tensor with the bit patterns of k (int32/int64/float32/float64)."""
    return dev(k)


def kind_of(dtype):
    return "signed" if np.issubdtype(dtype, np.integer) else "float"


def key_type_of(dtype):
    return {np.int32: "i32", np.int64: "i64", np.float32: "f32", np.float64: "f64"}[dtype]


@pytest.mark.parametrize("algo", ["lsd8", "lsd16"])
@pytest.mark.parametrize("dtype", [np.int32, np.float32, np.int64, np.float64])
def test_kv_matches_oracle(rs, dtype, algo):
    import torch
    for n in SIZES:
        announce("key types", dtype.__name__, algo, n)
        k = make_keys(dtype, n, 50 + n)
        vals = np.arange(n, dtype=np.uint32)
        wk, wv = oracle.sort_signed_or_float(k, vals, kind_of(dtype))
        dk, dv = as_tensor(k), dev(vals)
        ko, vo = torch.empty_like(dk), torch.empty_like(dv)
        rs.rsort_sort(dk, ko, dv, vo, algo=algo, key_type=key_type_of(dtype))
        rs.rsort_synchronize()
        got = host(ko)
        assert np.array_equal(got.view(np.uint8), wk.view(np.uint8)), (dtype, algo, n)
        assert np.array_equal(host(vo).view(np.uint32), wv), (dtype, algo, n)


@pytest.mark.parametrize("dtype", [np.int32, np.float32, np.int64, np.float64])
def test_in_place_and_keys_only(rs, dtype):
    n = 300007
    announce("key types in place", dtype.__name__)
    k = make_keys(dtype, n, 7)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.sort_signed_or_float(k, vals, kind_of(dtype))
    dk, dv = as_tensor(k), dev(vals)
    rs.rsort_sort(dk, dk, dv, dv, key_type=key_type_of(dtype))
    rs.rsort_synchronize()
    assert np.array_equal(host(dk).view(np.uint8), wk.view(np.uint8))
    assert np.array_equal(host(dv).view(np.uint32), wv)
    dk = as_tensor(k)
    ko, _ = rs.sort(dk, key_type=key_type_of(dtype))
    rs.rsort_synchronize()
    assert np.array_equal(host(ko).view(np.uint8), wk.view(np.uint8))



@pytest.mark.parametrize("algo", ["lsd8", "lsd16"])
@pytest.mark.parametrize("dtype", [np.int32, np.float32, np.int64, np.float64])
def test_all_equal_payloads_in_place(rs, dtype, algo):
    """Equal keys (every round the identity) with the payloads sorted in
    place and the keys not: the mapped keys must still reach keys_out before
    the inverse map."""
    import torch
    n = 40009
    announce("key types equal, payloads in place", dtype.__name__, algo)
    k = np.full(n, -3, dtype=dtype)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.sort_signed_or_float(k, vals, kind_of(dtype))
    dk, dv = as_tensor(k), dev(vals)
    ko = torch.empty_like(dk)
    rs.rsort_sort(dk, ko, dv, dv, algo=algo, key_type=key_type_of(dtype))
    rs.rsort_synchronize()
    assert np.array_equal(host(ko).view(np.uint8), wk.view(np.uint8))
    assert np.array_equal(host(dv).view(np.uint32), wv)

def test_float_tensors_default_to_total_order(rs):
    import torch
    k = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, np.nan, -np.nan, -0.0, 0.0],
                 dtype=np.float32)
    ko, vo = rs.sort(dev(k), torch.arange(k.size, dtype=torch.int32, device="cuda"))
    rs.rsort_synchronize()
    assert host(vo).tolist() == [7, 3, 5, 1, 8, 0, 9, 4, 2, 6]


def test_errors_and_workspace(rs):
    import torch
    k = dev(make_keys(np.int32, 1000, 3))
    o = torch.empty_like(k)
    with pytest.raises(rs.RsortError) as e:
        rs.rsort_sort(k, o, begin_bit=0, end_bit=16, key_type="i32")
    assert e.value.status == rs.RSORT_EUNSUPPORTED
    with pytest.raises(rs.RsortError) as e:
        rs.rsort_sort(k, o, algo="sample", key_type="i32")
    assert e.value.status == rs.RSORT_EUNSUPPORTED
    with pytest.raises(TypeError):
        rs.rsort_sort(k, o, key_type="i64")
    need_u = rs.rsort_workspace_bytes(torch.int32, True, 1000)
    need_i = rs.rsort_workspace_bytes(torch.int32, True, 1000, key_type="i32")
    assert need_i >= need_u + 4000
    ws = torch.empty(need_i, dtype=torch.uint8, device="cuda")
    kk = make_keys(np.int32, 1000, 3)
    rs.rsort_sort(dev(kk), o, workspace=ws, key_type="i32")
    rs.rsort_synchronize()
    assert np.array_equal(host(o), oracle.sort_signed_or_float(kk, None, "signed")[0])
