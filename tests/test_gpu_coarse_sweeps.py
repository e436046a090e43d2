"""Extra smoothing sweeps on the coarse levels (options nu_coarse, coarse_from)
on the GPU against the oracle's V-cycle with the same rule, through the C ABI.

The levels from coarse_from on are swept nu_coarse times before and after the
coarse correction.  On a 64^3 grid (levels 64, 32, 16, 8, 4) the 32^3 level
runs in the work-list kernels and the 16^3 and 8^3 levels in the one-workgroup
tail, or with deep_cells = 32768 from 32^3 on in the deep kernels, so each
place that sweeps a level is covered.  FP64: same options and iteration count
=> the fluence to 1e-10 relative L2, residual histories to 1e-9 (1e-8 with
Anderson acceleration).  A batch equals its problems solved one at a time.
"""
import numpy as np
import pytest

import oracle
from synth import media

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_1403_8105_amd")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def solve_gpu(st, al, Q, h, **kw):
    s = F.Solver(st.shape, h, **kw)
    s.set_medium(st, al, Q)
    out = s.solve()
    s.close()
    return out


@pytest.mark.parametrize("nu_coarse,coarse_from,deep", [(6, 1, 4096), (6, 2, 4096),
                                                        (5, 3, 4096), (6, 1, 32768)])
def test_coarse_sweeps_iterate_parity(nu_coarse, coarse_from, deep, parity_record):
    st, al, Q, h = media.config("cloud256", n=64)
    prob = oracle.setup(st, al, Q, h)
    kw = dict(nu1=3, nu2=3, omega_s=1.15, corr_scale=1.4, nu_coarse=nu_coarse,
              coarse_from=coarse_from)
    for k in (1, 3, 8):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, **kw)
        phi, rep = solve_gpu(st, al, Q, h, tol=0.0, max_iters=k, deep_cells=deep, **kw)
        err = rel_l2(phi, ref.phi)
        parity_record(test="coarse_sweeps_fp64_iterates", n=64, nu_coarse=nu_coarse,
                      coarse_from=coarse_from, deep_cells=deep, iterations=k, rel_l2=err)
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
        assert err <= 1e-10, k


def test_coarse_sweeps_change_the_iteration():
    # the option is live on each path: the iterate after 3 outer iterations
    # differs from the plain schedule's
    st, al, Q, h = media.config("cloud256", n=64)
    base, _ = solve_gpu(st, al, Q, h, tol=0.0, max_iters=3, nu1=3, nu2=3)
    for cf, deep in ((1, 4096), (3, 4096), (1, 32768)):
        phi, _ = solve_gpu(st, al, Q, h, tol=0.0, max_iters=3, nu1=3, nu2=3, nu_coarse=6,
                           coarse_from=cf, deep_cells=deep)
        assert rel_l2(phi, base) > 1e-12, (cf, deep)


def test_coarse_sweeps_with_anderson_iterate_parity(parity_record):
    st, al, Q, h = media.config("cloud256", n=32)
    prob = oracle.setup(st, al, Q, h)
    kw = dict(nu1=4, nu2=4, omega_s=1.15, corr_scale=2.0, aa_m=4, nu_coarse=10, coarse_from=2)
    for k in (1, 5, 12):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, **kw)
        phi, rep = solve_gpu(st, al, Q, h, tol=0.0, max_iters=k, **kw)
        err = rel_l2(phi, ref.phi)
        parity_record(test="coarse_sweeps_anderson_fp64_iterates", n=32, iterations=k,
                      rel_l2=err)
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-8)
        assert err <= 1e-10, k


def test_coarse_sweeps_mixed_reaches_the_oracle_fixed_point(parity_record):
    st, al, Q, h = media.config("cloud256", n=64)
    prob = oracle.setup(st, al, Q, h)
    ref = oracle.solve(prob, method="mg", tol=1e-10, max_iters=3000)
    assert ref.status == "converged"
    phi, rep = solve_gpu(st, al, Q, h, precision="mixed", tol=1e-10, max_iters=3000, nu1=4,
                         nu2=4, omega_s=1.15, corr_scale=2.0, aa_m=6, nu_coarse=12,
                         coarse_from=1)
    assert rep["status"] == F.FLD_OK
    err = rel_l2(phi, ref.phi)
    _, rel_o, _ = oracle.nonlinear_residual(prob, phi)
    parity_record(test="coarse_sweeps_mixed_vs_oracle", n=64, gpu_iterations=rep["iterations"],
                  rel_l2=err, gpu_rel_by_oracle=rel_o)
    assert err <= 1e-5
    assert rel_o <= 1.5e-10


def test_coarse_sweeps_batch_equals_single_solves():
    vols = media.batch_config(nvol=3, size_scale=0.25, seed=3)
    dims = [(v["n"],) * 3 for v in vols]
    kw = dict(precision="mixed", tol=1e-6, max_iters=3000, aa_m=4, nu_coarse=8, coarse_from=1)
    o = F.fld_default_options(**kw)
    b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
    for i, v in enumerate(vols):
        F.fld_batch_set_volume(b, i, v["sigma_t"], v["albedo"], v["Q"])
    outs, iters, rep = F.fld_batch_solve(b, [d for d in dims for _ in range(3)])
    F.fld_batch_destroy(b)
    assert rep["status"] == F.FLD_OK
    q = 0
    for v in vols:
        for c in range(3):
            phi, r = solve_gpu(v["sigma_t"], v["albedo"][c], v["Q"][c], v["h"], **kw)
            assert r["iterations"] == iters[q]
            np.testing.assert_array_equal(outs[q], phi)
            q += 1
