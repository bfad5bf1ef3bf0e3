"""rsort_sort_noalloc (the entry point for callers that cannot allocate) against
rsort_sort, bit-exact, through the C ABI: two calls in a row on the shared
scratch array, the second smaller than the first, so that the second call runs
on what the first left there; and the size limit, rejected on the host."""
import numpy as np
import pytest

import keygen
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    return rsort


def both(rs, keys, vals=None, begin_bit=0, end_bit=None, key_type=None):
    """(noalloc keys, noalloc vals, rsort_sort keys, rsort_sort vals) on the host."""
    import torch
    dk = dev(keys)
    dv = dev(vals) if vals is not None else None
    ka, va = torch.empty_like(dk), (torch.empty_like(dv) if dv is not None else None)
    rs.rsort_sort_noalloc(dk, ka, dv, va, begin_bit, end_bit, key_type=key_type)
    kb, vb = torch.empty_like(dk), (torch.empty_like(dv) if dv is not None else None)
    rs.rsort_sort(dk, kb, dv, vb, begin_bit, end_bit, algo="lsd8", key_type=key_type)
    rs.rsort_synchronize()
    return (host(ka), host(va) if va is not None else None,
            host(kb), host(vb) if vb is not None else None)


def test_two_calls_second_smaller(rs):
    n1 = 3000017
    keys = keygen.uniform_u32(n1, 21)
    vals = np.arange(n1, dtype=np.uint32)
    announce("noalloc u32 kv", n1)
    ka, va, kb, vb = both(rs, keys, vals)
    assert np.array_equal(ka, kb) and np.array_equal(va, vb)
    assert np.all(ka[1:] >= ka[:-1])
    n2 = 500009
    keys2 = keygen.kv_keys("zipf", n2, 22)
    announce("noalloc u32 keys", n2)
    ka, _, kb, _ = both(rs, keys2)
    assert np.array_equal(ka, kb)
    assert np.array_equal(ka, np.sort(keys2, kind="stable"))


def test_key_types_and_ranges(rs):
    n = 700001
    k64 = keygen.uniform_u64(n, 23)
    announce("noalloc u64", n)
    ka, _, kb, _ = both(rs, k64)
    assert np.array_equal(ka, kb)
    f32 = (keygen.unit_doubles(24, n) * 2.0 - 1.0).astype(np.float32)
    announce("noalloc f32", n)
    ka, _, kb, _ = both(rs, f32, key_type="f32")
    assert np.array_equal(ka.view(np.uint32), kb.view(np.uint32))
    keys = keygen.uniform_u32(n, 25)
    vals = np.arange(n, dtype=np.uint32)
    announce("noalloc bits [4, 20)", n)
    ka, va, kb, vb = both(rs, keys, vals, 4, 20)
    assert np.array_equal(ka, kb) and np.array_equal(va, vb)
    announce("noalloc n = 1 and n = 0")
    ka, _, kb, _ = both(rs, keys[:1])
    assert np.array_equal(ka, kb)
    ka, _, kb, _ = both(rs, keys[:0])
    assert ka.size == 0


def test_size_beyond_scratch_is_rejected(rs):
    import torch
    n = 1 << 24   # about 66 MiB of workspace for uint32 keys
    announce("noalloc beyond the scratch", n)
    dk = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(rs.RsortError) as e:
        rs.rsort_sort_noalloc(dk, torch.empty_like(dk), key_type="u32")
    assert e.value.status == rs.RSORT_EUNSUPPORTED
