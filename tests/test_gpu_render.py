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


def gpu_render(st, al, src, phi, h, background=0.0):
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(np.ascontiguousarray(np.broadcast_to(a, st.shape))).to(dev)
         for a in (st, al, src, phi)]
    img = torch.full(st.shape[:2], np.nan, dtype=torch.float64, device=dev)
    F.fld_render(*[x.data_ptr() for x in t], background, st.shape, h, img.data_ptr(),
                 torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    return img.cpu().numpy()


@pytest.mark.parametrize("shape", [(7, 5, 300), (3, 4, 1), (16, 16, 64), (9, 7, 130)])
def test_render_matches_oracle(shape):
    rng = np.random.default_rng(3 * sum(shape))
    st = rng.uniform(0.0, 30.0, shape) * (rng.random(shape) > 0.25)
    al = rng.uniform(0.3, 1.0, shape)
    src = rng.uniform(0.0, 5.0, shape)
    phi = rng.uniform(0.0, 2.0, shape)
    h = 1.0 / max(shape)
    img = gpu_render(st, al, src, phi, h, background=0.4)
    ref = oracle.render(st, al, src, phi, h, background=0.4)
    np.testing.assert_allclose(img, ref, rtol=1e-13, atol=1e-300)


def test_render_full_size_cloud():
    st, al, Q, h = media.config("cloud256")
    phi = np.random.default_rng(1).uniform(0.0, 1.0, st.shape)
    img = gpu_render(st, al, Q, phi, h, background=1.0)
    ref = oracle.render(st, al, Q, phi, h, background=1.0)
    np.testing.assert_allclose(img, ref, rtol=1e-12, atol=1e-300)


def test_pipeline_bake_solve_render():
    # bake -> FP64 multigrid solve -> render, all on the GPU, against the same
    # three steps of the oracle
    st, al, _, h = media.config("cloud128", n=32)
    q = gpu_bake(st, al, h)
    s = F.Solver(st.shape, h, tol=1e-9, max_iters=500)
    s.set_medium(st, al, q)
    phi, rep = s.solve()
    s.close()
    assert rep["status"] == F.FLD_OK
    img = gpu_render(st, al, q, phi, h, background=0.5)
    q_ref = oracle.light_bake(st, al, h)
    prob = oracle.setup(st, al, q_ref, h)
    ref = oracle.solve(prob, method="mg", tol=1e-9, max_iters=500)
    img_ref = oracle.render(st, al, q_ref, ref.phi, h, background=0.5)
    np.testing.assert_allclose(img, img_ref, rtol=1e-8)
