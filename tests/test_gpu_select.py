"""Post-scoring selection on the GPU vs the oracle, bit for bit: per-compound
best pose (segmented max with lowest-index ties, NaNs ignored) and top-k
(descending, lowest index on ties, NaN last), including a million values."""
import sys

import numpy as np
import pytest

import oracle
from helpers import weights

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def scorer():
    from paper_2104_04547_amd import Scorer
    arch, w = weights("tiny")
    s = Scorer(arch, w, "fp32")
    yield s
    s.close()


def test_compound_max_bit_exact(scorer):
    import torch
    _say("cf_compound_max 5000 compounds, 1..40 poses, ties and NaNs")
    rng = np.random.default_rng(3)
    lens = rng.integers(0, 41, size=5000)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    s = np.round(rng.normal(6, 1.5, size=int(off[-1])), 1).astype(np.float32)
    s[rng.integers(0, len(s), size=300)] = np.nan
    best, idx = scorer.compound_max(torch.from_numpy(s).cuda(), torch.from_numpy(off))
    scorer.check()
    wb, wi = oracle.compound_best(s.astype(np.float64), off)
    np.testing.assert_array_equal(idx.cpu().numpy(), wi)
    np.testing.assert_array_equal(best.cpu().numpy().astype(np.float64), wb)


def test_compound_max_reports_bad_offsets(scorer):
    import torch
    from paper_2104_04547_amd import cfabi
    _say("cf_compound_max malformed offsets")
    s = torch.zeros(10, device="cuda")
    scorer.compound_max(s, torch.tensor([0, 5, 12], dtype=torch.int32))
    assert scorer.status()[0] == cfabi.CF_ERR_INVALID_ARG


@pytest.mark.parametrize("n,k", [(1, 1), (1000, 1000), (100_000, 100), (1_000_000, 100), (1_000_000, 1024)])
def test_top_k_bit_exact(scorer, n, k):
    import torch
    _say(f"cf_top_k n={n} k={k}")
    rng = np.random.default_rng(n + k)
    v = np.round(rng.normal(6, 1.5, size=n), 2).astype(np.float32)   # many exact ties
    if n > 10:
        v[rng.integers(0, n, size=n // 50)] = np.nan
        v[:3] = [0.0, -0.0, 0.0]
    idx, val = scorer.top_k(torch.from_numpy(v).cuda(), k)
    vd = v.astype(np.float64)
    want = oracle.top_k(vd, k)
    np.testing.assert_array_equal(idx.cpu().numpy(), want)
    np.testing.assert_array_equal(val.cpu().numpy(), v[want])
