"""The allocation-free residual entry point against fld_residual_device.

fld_residual_device_noalloc keeps its temporaries in a fixed per-GPU scratch
area instead of allocating them; on the same context and fluence it must give
the same bits as fld_residual_device, also on a second call with a smaller
grid (the scratch then still holds the first call's larger contents), and it
must refuse a grid above its limit.
"""
import numpy as np
import pytest

from synth import media

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_1403_8105_amd")
torch = pytest.importorskip("torch")


def ragged_cloud(shape, seed):
    v = media.value_noise(shape, 4, seed)
    st = media.cloud_extinction(v, 200.0, 0.4)
    al = np.full(shape, 0.99)
    h = 1.0 / max(shape)
    return st, al, media.beer_lambert_source(st, al, h), h


def one_call(shape, seed, **opts):
    st, al, Q, h = ragged_cloud(shape, seed)
    s = F.Solver(shape, h, tol=0.0, max_iters=3, **opts)
    s.set_medium(st, al, Q)
    s.solve()                                   # a current fluence for the NULL case
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 1.0, shape) * (rng.random(shape) > 0.05)
    dev = torch.device("cuda:0")
    d_phi = torch.from_numpy(phi).to(dev)
    r_ref = torch.empty_like(d_phi)
    r_new = torch.full_like(d_phi, float("nan"))
    torch.cuda.synchronize()
    rel_ref = F.fld_residual_device(s.ctx, d_phi.data_ptr(), r_ref.data_ptr())
    rel_new = F.fld_residual_device_noalloc(s.ctx, d_phi.data_ptr(), r_new.data_ptr())
    torch.cuda.synchronize()
    assert rel_new == rel_ref
    assert torch.equal(r_new, r_ref)
    assert np.isfinite(rel_ref) and rel_ref > 0
    # the context's current fluence, and no residual field requested
    assert F.fld_residual_device_noalloc(s.ctx) == F.fld_residual_device(s.ctx)
    s.close()


def test_noalloc_residual_matches_two_calls_second_smaller():
    one_call((48, 40, 64), 3, precision="mixed")    # 122880 cells, quad paths
    one_call((21, 18, 13), 4, method="rbsor")       # smaller, one-cell-per-thread paths


def test_noalloc_residual_rejects_grids_above_its_limit():
    shape = (130, 128, 128)                   # above FLD_NOALLOC_MAX_CELLS = 128^3
    s = F.Solver(shape, 1.0 / 130, method="rbsor")
    st = np.full(shape, 1.0)
    s.set_medium(st, np.full(shape, 0.5), np.ones(shape))
    with pytest.raises(F.FldError) as ei:
        F.fld_residual_device_noalloc(s.ctx)
    assert ei.value.status == F.FLD_ERR_INVALID_ARGUMENT
    s.close()
