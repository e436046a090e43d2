"""Anderson-accelerated outer iteration (aa_m > 0) on the GPU against the
oracle's, through the C ABI.

FP64: same options and iteration count => the fluence to 1e-10 relative L2
and residual histories to 1e-8 (the least-squares coefficients come from sums
whose rounding order differs between the two sides, and the comparison stops
at a few tens of iterations, before that difference can grow).  Mixed: converged
fluence against the FP64 oracle's fixed point, 1e-5.  Launch-structure
variants (graphs, colour-split storage, batches, resume) give the same bits.
"""
import numpy as np
import pytest

import oracle
from synth import media

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_1403_8105_amd")

TUNED = dict(nu1=4, nu2=4, omega_s=1.15, corr_scale=2.0)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def solve_gpu(st, al, Q, h, **kw):
    s = F.Solver(st.shape, h, **kw)
    s.set_medium(st, al, Q)
    out = s.solve()
    s.close()
    return out


@pytest.mark.parametrize("sched", ["default", "tuned"])
@pytest.mark.parametrize("m", [1, 4])
def test_anderson_fp64_iterate_parity(m, sched, parity_record):
    # the 256^3 generator at 32^3: vacuum clusters (deflation) and residual
    # growth in the first iterations (restarts)
    st, al, Q, h = media.config("cloud256", n=32)
    prob = oracle.setup(st, al, Q, h)
    kw = dict(TUNED) if sched == "tuned" else {}
    for k in (1, 3, 10, 25):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, aa_m=m, **kw)
        phi, rep = solve_gpu(st, al, Q, h, tol=0.0, max_iters=k, aa_m=m, **kw)
        err = rel_l2(phi, ref.phi)
        parity_record(test="anderson_fp64_iterates", m=m, schedule=sched, iterations=k,
                      rel_l2=err)
        # the residual histories agree to 1e-8: the least-squares coefficients
        # amplify the rounding-order difference of the Gram sums (1e-16)
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-8)
        assert err <= 1e-10, k


@pytest.mark.parametrize("n", [32, 64])
def test_anderson_mixed_against_fp64_oracle(n, parity_record):
    st, al, Q, h = media.config("cloud128", n=n)
    prob = oracle.setup(st, al, Q, h)
    ref = oracle.solve(prob, method="mg", tol=1e-10, max_iters=3000)
    assert ref.status == "converged"
    phi, rep = solve_gpu(st, al, Q, h, precision="mixed", tol=1e-10, max_iters=3000, aa_m=4,
                         **TUNED)
    assert rep["status"] == F.FLD_OK
    err = rel_l2(phi, ref.phi)
    _, rel_o, _ = oracle.nonlinear_residual(prob, phi)
    parity_record(test="anderson_mixed_vs_oracle", n=n, gpu_iterations=rep["iterations"],
                  oracle_cg_iterations=ref.iterations, rel_l2=err, gpu_rel_by_oracle=rel_o)
    assert err <= 1e-5
    assert rel_o <= 1.5e-10


def test_anderson_launch_variants_are_bit_identical():
    # graph replay, timing events, colour-split storage and resume change how
    # the iteration is launched and stored, not what it computes
    st, al, Q, h = media.config("cloud256", n=32)
    outs = []
    for graph, timing, split in ((0, 0, 1), (1, 0, 1), (1, 1, 1), (1, 0, 0)):
        outs.append(solve_gpu(st, al, Q, h, precision="mixed", tol=0.0, max_iters=11, aa_m=4,
                              graph=graph, timing=timing, colour_split=split))
    for phi, rep in outs[1:]:
        np.testing.assert_array_equal(phi, outs[0][0])
        np.testing.assert_array_equal(rep["history"], outs[0][1]["history"])
    # 5 iterations, then 5 more resumed == 10 in one call
    s = F.Solver(st.shape, h, precision="mixed", tol=0.0, max_iters=5, aa_m=4)
    s.set_medium(st, al, Q)
    s.solve()
    part, rep = s.resume()
    s.close()
    assert rep["iterations"] == 10
    full, _ = solve_gpu(st, al, Q, h, precision="mixed", tol=0.0, max_iters=10, aa_m=4)
    np.testing.assert_array_equal(part, full)


def test_anderson_fp64_colour_split_is_bit_identical():
    # the FP64 form's colour-split finest fields under Anderson acceleration,
    # deflation and graph replay
    st, al, Q, h = media.config("cloud256", n=32)
    outs = [solve_gpu(st, al, Q, h, precision="fp64", tol=0.0, max_iters=9, aa_m=4,
                      colour_split=split) for split in (0, 1)]
    np.testing.assert_array_equal(outs[1][0], outs[0][0])
    np.testing.assert_array_equal(outs[1][1]["history"], outs[0][1]["history"])


def test_anderson_batch_equals_single_solves():
    vols = media.batch_config(nvol=3, size_scale=0.25, seed=3)
    dims = [(v["n"],) * 3 for v in vols]
    o = F.fld_default_options(precision="mixed", tol=1e-6, max_iters=3000, aa_m=4)
    b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
    for i, v in enumerate(vols):
        F.fld_batch_set_volume(b, i, v["sigma_t"], v["albedo"], v["Q"])
    outs, iters, rep = F.fld_batch_solve(b, [d for d in dims for _ in range(3)])
    F.fld_batch_destroy(b)
    assert rep["status"] == F.FLD_OK
    q = 0
    for v in vols:
        for c in range(3):
            phi, r = solve_gpu(v["sigma_t"], v["albedo"][c], v["Q"][c], v["h"],
                               precision="mixed", tol=1e-6, max_iters=3000, aa_m=4)
            assert r["iterations"] == iters[q]
            np.testing.assert_array_equal(outs[q], phi)
            q += 1
