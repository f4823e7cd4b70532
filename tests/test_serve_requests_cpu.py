"""Host logic of the serving load generator: each request is a contiguous span of
the pose pool, materialised as views with rebased offsets, identical to copying
the same poses out of the pool."""
import numpy as np

import synth
from paper_2104_04547_amd.serve import Requests


def test_request_spans_equal_copied_poses():
    pool = synth.make_poses("c5", 300)
    reqs = Requests(pool, 40, np.random.default_rng(3), max_poses=32, grids=(48, 64))
    assert len(reqs) == 40 and reqs.total_poses == int(reqs.k.sum())
    seen_G = set()
    for i, (span, G) in enumerate(reqs):
        k, st = int(reqs.k[i]), int(reqs.start[i])
        assert span.n_poses == k and 1 <= k <= 32 and st + k <= pool.n_poses
        ref = pool.select(list(range(st, st + k)))
        assert np.array_equal(span.atom_off, ref.atom_off) and span.atom_off[0] == 0
        assert np.array_equal(span.xyz, ref.xyz) and np.array_equal(span.feat, ref.feat)
        assert np.array_equal(span.is_lig, ref.is_lig)
        assert np.shares_memory(span.xyz, pool.xyz) or span.n_atoms == 0
        seen_G.add(G)
    assert seen_G <= {48, 64}
    # consecutive requests continue where the previous one stopped, modulo the period
    assert all(int(reqs.start[i + 1]) == (int(reqs.start[i]) + int(reqs.k[i])) % reqs.period for i in range(39))
