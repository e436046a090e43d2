"""GPU light baking through the C ABI against the oracle (Sec. 3 single-scatter
source of a directional light; reading A17).  FP64 both sides; the GPU sums
the optical depth with a wave scan instead of a running sum and uses the
device exp, so values agree to rounding (<= 1e-13 relative)."""
import numpy as np
import pytest

import oracle
from synth import media

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_1403_8105_amd")
torch = pytest.importorskip("torch")


def gpu_bake(st, al, h, light=1.0):
    dev = torch.device("cuda:0")
    d_st = torch.from_numpy(np.ascontiguousarray(st)).to(dev)
    d_al = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(al, st.shape))).to(dev)
    d_q = torch.full_like(d_st, np.nan)
    F.fld_light_bake(d_st.data_ptr(), d_al.data_ptr(), light, st.shape, h, d_q.data_ptr(),
                     torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    return d_q.cpu().numpy()


@pytest.mark.parametrize("shape", [(7, 5, 300), (3, 4, 1), (16, 16, 64), (9, 7, 130), (1, 1, 65)])
def test_bake_matches_oracle(shape):
    rng = np.random.default_rng(sum(shape))
    st = rng.uniform(0.0, 40.0, shape) * (rng.random(shape) > 0.25)   # vacuum voxels too
    al = rng.uniform(0.3, 1.0, shape)
    h = 1.0 / max(shape)
    q = gpu_bake(st, al, h, light=1.7)
    ref = oracle.light_bake(st, al, h, light=1.7)
    assert np.all(np.isfinite(q))
    np.testing.assert_allclose(q, ref, rtol=1e-13, atol=1e-300)


def test_bake_full_size_cloud():
    # the 256^3 bench cloud: every voxel against the oracle
    st, al, _, h = media.config("cloud256")
    q = gpu_bake(st, al, h)
    ref = oracle.light_bake(st, al, h)
    np.testing.assert_allclose(q, ref, rtol=1e-12, atol=1e-300)
