"""The GPU training-ray sampler against the float64 oracle (same uniforms): every ray whose
accept/reject decisions and primitive draw are not within float32 reach of a boundary
matches; the rest are valid rays of their kind."""
import numpy as np
import pytest
import torch

from oracle import sampling as SM
from paper_2606_00817_amd import ddf
from paper_2606_00817_amd import inputs as I
from tests.helpers import cuda

pytestmark = pytest.mark.gpu


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("n,tries", [(5001, 4), (1, 1), (256, 8)])
def test_sample_rays_match_oracle(mode, n, tries):
    dev = cuda()
    sc = I.scene_ground(24, 5)
    u = I.uniforms(3 * tries + 2, n, 50 + mode)
    rays = ddf.sample_rays(_t(ddf.scene_prims(sc), dev), _t(u, dev), mode=mode, box_half=1.5, offset=1e-3)
    torch.cuda.synchronize()
    r = rays.cpu().numpy().astype(np.float64).T
    ref, chosen, margin = SM.sample_rays(sc, u.astype(np.float64), mode, 1.5, 1e-3, tries)
    clear = margin > 1e-5
    assert clear.mean() > 0.95
    assert np.abs(r[clear, 0:3] - ref[clear, 0:3]).max() <= 2e-5
    assert np.abs(r[:, 3:6] - ref[:, 3:6]).max() <= 2e-6          # directions never depend on a decision
    # every origin in the box (free) or within offset + float32 of a surface (surface rays)
    assert np.isfinite(r).all() and (np.abs(r[:, 0:3]) <= 1.5 + 1e-3 + 1e-5).all()
    print(f"sampler mode {mode} n={n} tries={tries}: clear {clear.mean():.4f}, "
          f"max |do| {np.abs(r[clear, 0:3] - ref[clear, 0:3]).max() if clear.any() else 0:.2e}")


def test_sample_rays_argument_errors():
    dev = cuda()
    prims = _t(ddf.scene_prims(I.scene_ground(4, 5)), dev)
    u = torch.rand((3 * 4 + 2, 64), device=dev)
    with pytest.raises(ddf.DDFError, match="mode"):
        ddf.sample_rays(prims, u, mode=3)
    with pytest.raises(ddf.DDFError, match="rows"):
        ddf.sample_rays(prims, u, tries=5)        # 17 rows needed
    with pytest.raises(ddf.DDFError, match="box_half"):
        ddf.sample_rays(prims, u, box_half=0.0)
    with pytest.raises(ddf.DDFError, match="tries"):
        ddf.sample_rays(prims, torch.rand((3 * 17 + 2, 64), device=dev), tries=17)
