"""The allocation-free hash-grid query (ddf_hash_query_static) against the workspace query
(ddf_hash_query with ws) through the C ABI: the same kernels, so the answers must be equal bit
for bit, on two calls in a row (the second with fewer rays, so a stale tail of the first call's
staged lookups would show), and a batch beyond the static capacity is refused before anything
is written."""
import numpy as np
import pytest
import torch

from oracle import hashgrid_oracle as H
from paper_2606_00817_amd import ddf
from paper_2606_00817_amd import inputs as I
from tests.helpers import cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("desc", [I.HASH_PAPER, I.HASH_SMALL], ids=["paper-16-level", "6-level"])
def test_static_hash_query_equals_workspace_query(desc):
    dev = cuda()
    params = torch.from_numpy(I.hash_params(desc, H.table_entries(desc), 31, table_std=0.3)).to(dev)
    sc = I.scene_mixed(256, 2)
    cap = ddf.hash_query_static_max_rays()
    assert cap == 1 << 19
    for n, seed in ((cap - 3, 12), (1000, 13)):
        rays = torch.from_numpy(I.shadow_rays(sc, n, seed)).to(dev)
        t_s = torch.full((n,), float("nan"), device=dev)
        x_s = torch.full((n,), float("nan"), device=dev)
        ddf.hash_query_static(desc, params, rays, t_s, x_s)
        ws = torch.empty(ddf.hash_query_workspace_bytes(desc, n), dtype=torch.uint8, device=dev)
        t_w, x_w = ddf.hash_query(desc, params, rays, ws=ws)
        torch.cuda.synchronize()
        print(f"static vs workspace query, {desc.n_levels} levels, n = {n}: "
              f"{int((t_s != t_w).sum())} t and {int((x_s != x_w).sum())} xi differ")
        assert torch.equal(t_s, t_w) and torch.equal(x_s, x_w)
    # beyond the capacity: refused, outputs untouched
    n = cap + 1
    rays = torch.zeros((6, n), dtype=torch.float32, device=dev)
    rays[5] = 1.0
    t_s = torch.full((n,), -7.0, device=dev)
    x_s = torch.full((n,), -7.0, device=dev)
    with pytest.raises(ddf.DDFError, match="static workspace"):
        ddf.hash_query_static(desc, params, rays, t_s, x_s)
    torch.cuda.synchronize()
    assert bool((t_s == -7.0).all()) and bool((x_s == -7.0).all())
