"""Graph capture of the query paths (the sparse-query regime, where launch cost matters): a
captured dense bf16 query and two-pass hash query, replayed several times with eager work and
new inputs in between, equal the eager results bit for bit on every replay.  The library
records no memset and allocates nothing inside these calls."""
import numpy as np
import pytest
import torch

from oracle import hashgrid_oracle as H
from paper_2606_00817_amd import ddf
from paper_2606_00817_amd import inputs as I
from tests.helpers import cuda

pytestmark = pytest.mark.gpu


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def test_graph_replays_match_eager():
    dev = cuda()
    n = 1000
    sc = I.scene_mixed(256, 2)
    desc = I.NET_FULL
    master = _t(I.he_init(desc, 0), dev)
    packed = ddf.pack(desc, "bf16", master)
    dc = ddf.desc_c(desc, "bf16")
    hd = I.HASH_PAPER
    hp = _t(I.hash_params(hd, H.table_entries(hd), 60, table_std=0.3), dev)
    batches = [_t(I.shadow_rays(sc, n, 61 + k), dev) for k in range(4)]
    rays = batches[0].clone()
    t1 = torch.empty(n, device=dev); x1 = torch.empty(n, device=dev)
    t2 = torch.empty(n, device=dev); x2 = torch.empty(n, device=dev)
    ws = torch.empty(ddf.hash_query_workspace_bytes(hd, n), dtype=torch.uint8, device=dev)

    def step():
        ddf.query_into(dc, packed, rays, t1, x1)
        ddf.hash_query(hd, hp, rays, ws=ws, t=t2, xi=x2)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for k in range(1, 4):
        rays.copy_(batches[k])
        g.replay()
        torch.cuda.synchronize()
        got = [x.clone() for x in (t1, x1, t2, x2)]
        # eager work between replays, then the eager answers for the same rays
        ddf.query_into(dc, packed, batches[(k + 1) % 4], t1, x1)
        step()
        torch.cuda.synchronize()
        for a, b in zip(got, (t1, x1, t2, x2)):
            assert torch.equal(a, b), f"replay {k} differs from eager"
