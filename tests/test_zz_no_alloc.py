"""The allocation-free entry point (ot_assign_dev_noalloc) against ot_assign_dev.

Both run the same one-workgroup engine on the same inputs, so every output is
bit-identical; two calls in a row (the second smaller) show that the static
scratch keeps no state that changes a later result.
"""
import numpy as np
import pytest

import oracle
from paper_2005_01182_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _solve(ot, fn, C, **kw):
    import torch
    n = C.shape[0]
    dC = torch.from_numpy(C).cuda()
    out = (torch.full((n,), -1, dtype=torch.int32, device="cuda"), torch.zeros(1, dtype=torch.int64, device="cuda"),
           torch.zeros(n, dtype=torch.int64, device="cuda"), torch.zeros(n, dtype=torch.int64, device="cuda"))
    st = ot.stats_tensor(1)
    fn(dC, *out, st[0], **kw)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out] + [st.cpu().numpy()[0]]


@pytest.mark.parametrize("sizes", [(1000, 300), (4096, 65)])
def test_noalloc_matches_ot_assign_dev(otkm_gpu, sizes):
    for n in sizes:
        C = wl.geometric_assignment(n, seed=n) if n % 2 == 0 else wl.uniform_assignment(n, seed=n, hi=5000)
        print("noalloc n =", n, flush=True)
        a = _solve(otkm_gpu, otkm_gpu.ot_assign_dev_noalloc, C)
        b = _solve(otkm_gpu, otkm_gpu.ot_assign_dev, C, wgs=1)
        assert a[4][7] == 0 and b[4][7] == 0
        for x, y in zip(a[:4], b[:4]):
            assert np.array_equal(x, y)
        assert oracle.certify_assign(C, a[0], a[2], a[3]) == 0
        if n <= 1000:
            assert int(a[1][0]) == oracle.assign(C)[1]


def test_noalloc_rejects_what_it_cannot_do(otkm_gpu):
    import torch
    C = torch.zeros((8, 8), dtype=torch.int32, device="cuda")
    plan = torch.empty(8, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    for kw in ({"max_paths": -1}, {"block": 100}):
        with pytest.raises(otkm_gpu.OtError) as e:
            otkm_gpu.ot_assign_dev_noalloc(C, plan, cost, **kw)
        assert e.value.code == otkm_gpu.OT_EINVAL
    big = torch.zeros((4097, 4097), dtype=torch.int32, device="cuda")
    with pytest.raises(otkm_gpu.OtError) as e:
        otkm_gpu.ot_assign_dev_noalloc(big, plan, cost)
    assert e.value.code == otkm_gpu.OT_ETOOBIG
