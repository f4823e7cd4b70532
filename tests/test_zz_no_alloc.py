"""The allocation-free top-k (cf_top_k_noalloc, static per-GPU scratch) against
the context's cf_top_k, bit for bit, on two calls in a row (the second smaller,
so it runs over the first call's leftovers in the shared scratch), with the
oracle's ordering as a third witness.  Also: oversized k is refused before any
launch, and a call ordered after an earlier one on the same stream allocates
no device memory."""
import sys

import numpy as np
import pytest

import oracle
from helpers import weights

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _values(n, seed):
    rng = np.random.default_rng(seed)
    v = np.round(rng.normal(6, 1.5, size=n), 2).astype(np.float32)   # many exact ties
    v[rng.integers(0, n, size=max(1, n // 50))] = np.nan
    v[:3] = [0.0, -0.0, 0.0]
    return v


def _noalloc(values, k):
    import torch
    from paper_2104_04547_amd import cfabi
    idx = torch.empty(k, dtype=torch.int32, device="cuda")
    val = torch.empty(k, dtype=torch.float32, device="cuda")
    cfabi.cf_top_k_noalloc(values.data_ptr(), values.numel(), k, idx.data_ptr(), val.data_ptr(),
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return idx, val


def test_top_k_noalloc_matches_cf_top_k_twice():
    import torch
    from paper_2104_04547_amd import Scorer
    arch, w = weights("tiny")
    s = Scorer(arch, w, "fp32")
    try:
        for n, k, seed in ((1_000_000, 1024, 11), (20_000, 100, 12)):
            _say(f"cf_top_k_noalloc n={n} k={k} vs cf_top_k")
            v = _values(n, seed)
            vd = torch.from_numpy(v).cuda()
            got_i, got_v = _noalloc(vd, k)
            ref_i, ref_v = s.top_k(vd, k)
            s.check()
            np.testing.assert_array_equal(got_i.cpu().numpy(), ref_i.cpu().numpy())
            np.testing.assert_array_equal(got_v.cpu().numpy().view(np.uint32), ref_v.cpu().numpy().view(np.uint32))
            np.testing.assert_array_equal(got_i.cpu().numpy(), oracle.top_k(v.astype(np.float64), k))
    finally:
        s.close()


def test_top_k_noalloc_refuses_k_beyond_the_static_scratch():
    import torch
    from paper_2104_04547_amd import cfabi
    _say("cf_top_k_noalloc k=1025")
    v = torch.zeros(4096, device="cuda")
    idx = torch.empty(1025, dtype=torch.int32, device="cuda")
    with pytest.raises(cfabi.CfError) as e:
        cfabi.cf_top_k_noalloc(v.data_ptr(), 4096, 1025, idx.data_ptr(), None,
                               torch.cuda.current_stream().cuda_stream)
    assert e.value.code == cfabi.CF_ERR_UNSUPPORTED


def test_top_k_noalloc_leaves_device_memory_unchanged():
    import torch
    _say("cf_top_k_noalloc device memory before / after")
    v = torch.from_numpy(_values(300_000, 13)).cuda()
    _noalloc(v, 64)                       # first call on the device looks up the scratch address
    idx = torch.empty(500, dtype=torch.int32, device="cuda")
    val = torch.empty(500, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    from paper_2104_04547_amd import cfabi
    for _ in range(3):
        cfabi.cf_top_k_noalloc(v.data_ptr(), v.numel(), 500, idx.data_ptr(), val.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    np.testing.assert_array_equal(idx.cpu().numpy(), oracle.top_k(v.cpu().numpy().astype(np.float64), 500))
