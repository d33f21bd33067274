"""The no-allocation top-K entry point (bmf_topk_dev_noalloc) against
bmf_topk_dev: the same items and scores bit for bit, in all three precisions,
on two calls in a row (the second with fewer users, so it runs over what
the first left in the fixed workspace), through the C ABI; oversized
requests and a missing BF16 table are refused without running anything."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True, file=sys.stderr)


def test_noalloc_topk_equals_topk_dev():
    import torch
    from paper_1907_07410_amd import binding as B
    rng = np.random.default_rng(77)
    m, n, k, K = 3000, 20000, 64, 100
    G = B.Model(m, n, k, 4)
    G.set_factors(rng.normal(0, .3, (m, k)).astype(np.float32), rng.normal(0, .3, (n, k)).astype(np.float32),
                  rng.normal(0, .3, m).astype(np.float32), rng.normal(0, .3, n).astype(np.float32), 3.5)
    # the BF16 table's memory does not exist yet: refused, nothing run
    u0 = torch.from_numpy(rng.integers(0, m, 5).astype(np.int32)).cuda()
    it0 = torch.zeros((5, K), dtype=torch.int32, device="cuda")
    sc0 = torch.zeros((5, K), dtype=torch.float32, device="cuda")
    with pytest.raises(B.BmfError) as ex:
        G.topk_dev_noalloc(u0, K, 1, 0, it0, sc0)
    assert ex.value.status == B.BMF_E_STATE
    # a request larger than the fixed workspace: refused
    big = torch.zeros(200000, dtype=torch.int32, device="cuda")
    with pytest.raises(B.BmfError) as ex:
        G.topk_dev_noalloc(big, K, 0, 0, it0, sc0)
    assert ex.value.status == B.BMF_E_NOMEM
    for precision in (0, 1, 2):
        for nu in (1500, 37):  # the second call is smaller than the first
            log("precision", precision, "users", nu)
            users = torch.from_numpy(rng.integers(0, m, nu).astype(np.int32)).cuda()
            ia = torch.full((nu, K), -7, dtype=torch.int32, device="cuda")
            sa = torch.zeros((nu, K), dtype=torch.float32, device="cuda")
            ib = torch.full((nu, K), -9, dtype=torch.int32, device="cuda")
            sb = torch.ones((nu, K), dtype=torch.float32, device="cuda")
            G.topk_dev(users, K, precision, 0, ia, sa)
            G.synchronize()
            G.topk_dev_noalloc(users, K, precision, 0, ib, sb)
            G.synchronize()
            a_i, a_s, b_i, b_s = ia.cpu().numpy(), sa.cpu().numpy(), ib.cpu().numpy(), sb.cpu().numpy()
            assert np.array_equal(a_i, b_i)
            assert np.array_equal(a_s.view(np.uint32), b_s.view(np.uint32))
            assert np.all(a_i >= 0) and np.all(np.diff(a_s, axis=1) <= 0)
    G.close()
