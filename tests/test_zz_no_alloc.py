"""tip_decompose_noalloc (scratch in a static device array, no allocation in
the call) against tip_decompose_async (caller's workspace) on the same
inputs: identical tip numbers, on two calls in a row, the second with a
smaller graph, and both equal to the oracle.  The scratch holds no
fine-grained pair rows, so the no-alloc call walks every fine-grained
update: its work counters equal those of tip_decompose_async with
TIP_FLAG_FD_WALK.  A graph whose workspace exceeds the scratch is refused
with TIP_ENOMEM."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2010_08695_amd import graphgen as gg
from paper_2010_08695_amd import tip

pytestmark = pytest.mark.gpu

WORK_KEYS = ("wedges_count", "wedges_cd", "wedges_fd", "pair_updates", "rounds", "subsets", "fd_levels")


def _run_both(g, side, stream):
    import torch
    dev = torch.device("cuda:0")
    d_eu = torch.from_numpy(g.eu).to(dev)
    d_ev = torch.from_numpy(g.ev).to(dev)
    n = g.n_u if side == 0 else g.n_v
    walk = tip.TIP_FLAG_FD_WALK
    assert tip.workspace_size(g.n_u, g.n_v, g.m, side, flags=walk) <= tip.NOALLOC_SCRATCH_BYTES
    ws = torch.empty(tip.workspace_size(g.n_u, g.n_v, g.m, side), dtype=torch.uint8, device=dev)
    th_a = torch.full((max(n, 1),), -1, dtype=torch.int64, device=dev)
    th_w = torch.full((max(n, 1),), -3, dtype=torch.int64, device=dev)
    th_n = torch.full((max(n, 1),), -2, dtype=torch.int64, device=dev)
    tip.decompose_async(d_eu, d_ev, g.n_u, g.n_v, side, th_a, ws, stream)
    st_w = tip.decompose_async(d_eu, d_ev, g.n_u, g.n_v, side, th_w, ws, stream, flags=walk)
    st_n = tip.decompose_noalloc(d_eu, d_ev, g.n_u, g.n_v, side, th_n, stream)
    stream.synchronize()
    np.testing.assert_array_equal(th_w[:n].cpu().numpy(), th_a[:n].cpu().numpy())
    return th_a[:n].cpu().numpy(), th_n[:n].cpu().numpy(), st_w, st_n


def test_noalloc_matches_async_on_two_calls(gpu_lib):
    import torch
    stream = torch.cuda.Stream()
    big = gg.chung_lu(60_000, 12_000, 600_000, 2.5, 2.1, seed=12, cap_v=3e3)
    small = gg.chung_lu(5_000, 1_000, 40_000, 2.3, 2.0, seed=81)
    for g, side in ((big, 0), (small, 1)):
        print(f"noalloc vs async: {g.name} side {side} m={g.m}", flush=True)
        a, n, sa, sn = _run_both(g, side, stream)
        np.testing.assert_array_equal(n, a)
        np.testing.assert_array_equal(n, oracle.bup(g, side)[0])
        for k in WORK_KEYS:
            assert sa[k] == sn[k], k


def test_noalloc_refuses_graphs_beyond_the_scratch(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    n_u, n_v, m = 4_000_000, 1_000, 8
    assert tip.workspace_size(n_u, n_v, m, 0, flags=tip.TIP_FLAG_FD_WALK) > tip.NOALLOC_SCRATCH_BYTES
    d_e = torch.zeros(m, dtype=torch.int32, device=dev)
    d_theta = torch.empty(n_u, dtype=torch.int64, device=dev)
    with pytest.raises(tip.TipError) as ei:
        tip.decompose_noalloc(d_e, d_e, n_u, n_v, 0, d_theta)
    assert ei.value.status == tip.TIP_ENOMEM and "scratch" in str(ei.value)
