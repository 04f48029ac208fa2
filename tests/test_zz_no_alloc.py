"""gbs_prob_exact_dev_noalloc (the entry point that allocates nothing: its
partial sums live in a fixed device array) against gbs_prob_exact_dev on the
same device inputs, through the C ABI: two calls in a row, the second with a
smaller batch (the fixed array keeps the first call's contents), then a batch
beyond the array's capacity, which is refused."""
import numpy as np
import pytest

import paper_2106_01445_amd as g
from paper_2106_01445_amd import gbs
from workloads import make_workload

pytestmark = pytest.mark.gpu


def _run(ctx, wl, noalloc):
    import torch
    dev = torch.device("cuda")
    off = torch.tensor(wl.offsets, dtype=torch.int32, device=dev)
    mod = torch.tensor(wl.modes, dtype=torch.int32, device=dev)
    P = wl.P
    out = [torch.full((P,), -1.0, dtype=torch.float64, device=dev) for _ in range(3)]
    st = torch.full((P,), -1, dtype=torch.int32, device=dev)
    rc = ctx.gbs_prob_exact_dev(off, mod, int(np.diff(wl.offsets).max()), out[0], out[1], out[2], st,
                                noalloc=noalloc)
    assert rc == 0
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out] + [st.cpu().numpy()]


def test_noalloc_matches_allocating_entry_point(gpu_ctx):
    full = make_workload(2)                              # 4096 rows, 6-14 clicks
    gpu_ctx.gbs_set_model(full.U, full.r, full.eta)
    for wl in (full.subset(range(1500)), full.subset(range(700, 900))):
        ref = _run(gpu_ctx, wl, noalloc=False)
        got = _run(gpu_ctx, wl, noalloc=True)
        assert np.array_equal(got[3], ref[3])
        assert np.all(ref[3] == 0)
        for a, b in zip(got[:3], ref[:3]):
            assert np.array_equal(a, b)


def test_noalloc_refuses_batches_beyond_its_scratch(gpu_ctx):
    import torch
    wl = make_workload(2).subset(range(300))
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    dev = torch.device("cuda")
    off = torch.tensor(wl.offsets, dtype=torch.int32, device=dev)
    mod = torch.tensor(wl.modes, dtype=torch.int32, device=dev)
    p = torch.empty(wl.P, dtype=torch.float64, device=dev)
    st = torch.empty(wl.P, dtype=torch.int32, device=dev)
    # 300 rows x 2^12 work items (max_clicks 30) > 2^20
    with pytest.raises(g.GBSError) as e:
        gpu_ctx.gbs_prob_exact_dev(off, mod, 30, p, None, None, st, noalloc=True)
    assert e.value.code == gbs.GBS_E_INVAL
