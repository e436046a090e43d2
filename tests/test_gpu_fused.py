"""The fused passes against the separate ones.  The limiter-residual pass
(fuse_lr = 1) against the separate limiter and residual passes (fuse_lr = 0,
the default): the same D and r per cell,
so the same iterates, and residual norms that differ only in the grouping of
their partial sums.  Shapes with partial tiles (rows not a multiple of 16,
z not a multiple of 32, x not a multiple of 32), both precisions and both outer
steps, a batch of uneven volumes, and the oracle's iterates at 1e-10."""
import numpy as np
import pytest

import oracle
from synth import media

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_1403_8105_amd")


def ragged_cloud(shape, seed):
    v = media.value_noise(shape, 4, seed)
    st = media.cloud_extinction(v, 200.0, 0.4)
    al = np.full(shape, 0.99)
    h = 1.0 / max(shape)
    return st, al, media.beer_lambert_source(st, al, h), h


def solve(st, al, Q, h, **kw):
    s = F.Solver(st.shape, h, **kw)
    s.set_medium(st, al, Q)
    out = s.solve()
    s.close()
    return out


# multigrid shapes (coarsest level at most 512 cells) with partial tiles:
# rows not a multiple of 16, z not a multiple of 32 (40: natural order in the
# mixed form; 48, 16: colour-split), x not a multiple of 32
CASES = [
    ("cloud", (32, 32, 32), dict(aa_m=4)),
    ("ragged", (40, 56, 40), dict(aa_m=4)),
    ("ragged", (72, 40, 48), dict(precision="mixed", aa_m=4)),
    ("ragged", (72, 40, 48), dict(precision="mixed")),
    ("ragged", (40, 40, 16), dict(precision="mixed", aa_m=2, nu1=3, nu2=3, omega_s=1.15)),
]


@pytest.mark.parametrize("kind,shape,kw", CASES)
def test_fused_equals_separate_passes(kind, shape, kw):
    if kind == "cloud":
        st, al, Q, h = media.config("cloud256", n=shape[0])
    else:
        st, al, Q, h = ragged_cloud(shape, seed=sum(shape))
    a, ra = solve(st, al, Q, h, tol=0.0, max_iters=12, fuse_lr=1, **kw)
    b, rb = solve(st, al, Q, h, tol=0.0, max_iters=12, fuse_lr=0, **kw)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_allclose(ra["history"], rb["history"], rtol=1e-13)


@pytest.mark.parametrize("shape", [(40, 56, 40), (72, 40, 48)])
def test_fused_fp64_iterates_match_oracle(shape):
    st, al, Q, h = ragged_cloud(shape, seed=7 + sum(shape))
    prob = oracle.setup(st, al, Q, h)
    for k in (1, 5):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, aa_m=3)
        phi, rep = solve(st, al, Q, h, tol=0.0, max_iters=k, aa_m=3, fuse_lr=1)
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-8)
        assert np.linalg.norm(phi - ref.phi) <= 1e-10 * np.linalg.norm(ref.phi), k


def test_fused_residual_entry_matches_oracle_after_solve():
    # the solve's last residual (fused) and the oracle's evaluation of its fluence
    st, al, Q, h = ragged_cloud((40, 56, 40), seed=3)
    prob = oracle.setup(st, al, Q, h)
    phi, rep = solve(st, al, Q, h, precision="mixed", tol=1e-8, max_iters=3000, aa_m=4,
                     fuse_lr=1)
    assert rep["status"] == F.FLD_OK
    _, rel_o, _ = oracle.nonlinear_residual(prob, phi)
    assert rel_o == pytest.approx(rep["rel"], rel=1e-9)


def test_fused_batch_equals_separate_passes():
    vols = media.batch_config(nvol=3, size_scale=0.25, seed=5)
    dims = [(v["n"],) * 3 for v in vols]
    outs = []
    for fuse in (1, 0):
        o = F.fld_default_options(precision="mixed", tol=0.0, max_iters=8, aa_m=4, fuse_lr=fuse)
        b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
        for i, v in enumerate(vols):
            F.fld_batch_set_volume(b, i, v["sigma_t"], v["albedo"], v["Q"])
        res, iters, rep = F.fld_batch_solve(b, [d for d in dims for _ in range(3)])
        F.fld_batch_destroy(b)
        outs.append(res)
    for x, y in zip(*outs):
        np.testing.assert_array_equal(x, y)


# single-pass red-black sweeps of the finest level (fuse_rb = 1) against the
# half-sweeps: odd and even sweep counts (an odd sweep left over runs as
# half-sweeps), both storage orders in the mixed form (nz = 48 and 16:
# colour-split; 40: natural), FP64, over-relaxation
RB_CASES = [
    ("cloud", (32, 32, 32), dict(precision="mixed", aa_m=4, nu1=4, nu2=4, omega_s=1.15)),
    ("ragged", (72, 40, 48), dict(precision="mixed", aa_m=4, nu1=3, nu2=2)),
    ("ragged", (40, 56, 40), dict(precision="mixed", nu1=2, nu2=2)),
    ("ragged", (40, 40, 16), dict(precision="mixed", aa_m=2, nu1=1, nu2=2, omega_s=1.3)),
    ("ragged", (40, 56, 40), dict(aa_m=4, nu1=2, nu2=2, omega_s=1.15)),
]


@pytest.mark.parametrize("kind,shape,kw", RB_CASES)
def test_fused_sweep_equals_half_sweeps(kind, shape, kw):
    if kind == "cloud":
        st, al, Q, h = media.config("cloud256", n=shape[0])
    else:
        st, al, Q, h = ragged_cloud(shape, seed=11 + sum(shape))
    a, ra = solve(st, al, Q, h, tol=0.0, max_iters=10, fuse_rb=1, **kw)
    b, rb = solve(st, al, Q, h, tol=0.0, max_iters=10, fuse_rb=0, **kw)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ra["history"], rb["history"])


def test_fused_sweep_fp64_iterates_match_oracle():
    st, al, Q, h = ragged_cloud((72, 40, 48), seed=5)
    prob = oracle.setup(st, al, Q, h)
    for k in (1, 5):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, nu1=2, nu2=2)
        phi, rep = solve(st, al, Q, h, tol=0.0, max_iters=k, nu1=2, nu2=2, fuse_rb=1)
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
        assert np.linalg.norm(phi - ref.phi) <= 1e-10 * np.linalg.norm(ref.phi), k


def test_fused_sweep_batch_and_graphs():
    vols = media.batch_config(nvol=3, size_scale=0.25, seed=6)
    dims = [(v["n"],) * 3 for v in vols]
    outs = []
    for fuse, graph in ((1, 1), (0, 1), (1, 0)):
        o = F.fld_default_options(precision="mixed", tol=0.0, max_iters=8, aa_m=4, nu1=4, nu2=4,
                                  fuse_rb=fuse, graph=graph)
        b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
        for i, v in enumerate(vols):
            F.fld_batch_set_volume(b, i, v["sigma_t"], v["albedo"], v["Q"])
        res, iters, rep = F.fld_batch_solve(b, [d for d in dims for _ in range(3)])
        F.fld_batch_destroy(b)
        outs.append(res)
    for other in outs[1:]:
        for x, y in zip(outs[0], other):
            np.testing.assert_array_equal(x, y)
