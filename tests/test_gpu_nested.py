"""GPU parity of grid sequencing (options.nested_tol): the 2:1 coarse solve and
the fine solve started from its fluence, against the oracle's nested solve.
FP64 form: the coarse iteration count and the fine iterates (fixed count)
agree, relative L2 <= 1e-10.  Mixed form: the converged fluence against the
FP64 oracle solved to its floor, relative L2 <= 1e-5.
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
    try:
        s.set_medium(st, al, Q)
        return s.solve()
    finally:
        s.close()


@pytest.mark.parametrize("shape", [(32, 32, 32), (16, 24, 32)])
def test_nested_fp64_iterate_parity(shape):
    st, al, Q, h = media.cloud_medium(shape, 4, 200.0, 0.4, 0.99, 21)
    prob = oracle.setup(st, al, Q, h)
    for k in (1, 6):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, nested_tol=1e-3)
        phi, rep = solve_gpu(st, al, Q, h, tol=0.0, max_iters=k, nested_tol=1e-3)
        assert rep["nested_iterations"] == ref.nested_iterations > 0
        assert rep["iterations"] == ref.iterations == k
        assert rel_l2(phi, ref.phi) <= 1e-10, k


def test_nested_inherit_fp64_iterate_parity():
    # the coarse solve with the fine solve's schedule (Anderson window, sweeps,
    # coarse-level sweeps one level up) against the oracle's
    st, al, Q, h = media.cloud_medium((32, 32, 32), 4, 200.0, 0.4, 0.99, 21)
    prob = oracle.setup(st, al, Q, h)
    kw = dict(nu1=3, nu2=3, omega_s=1.15, corr_scale=1.4, aa_m=4, nu_coarse=6, coarse_from=2)
    plain = oracle.solve(prob, method="mg", tol=0.0, max_iters=1, nested_tol=1e-3, **kw)
    for k in (1, 6):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, nested_tol=1e-3,
                           nested_inherit=True, **kw)
        phi, rep = solve_gpu(st, al, Q, h, tol=0.0, max_iters=k, nested_tol=1e-3,
                             nested_inherit=1, **kw)
        assert rep["nested_iterations"] == ref.nested_iterations > 0
        assert ref.nested_iterations != plain.nested_iterations
        assert rep["iterations"] == ref.iterations == k
        assert rel_l2(phi, ref.phi) <= 1e-10, k


def test_nested_mixed_reaches_the_fp64_fixed_point():
    st, al, Q, h = media.config("cloud128", n=32)
    prob = oracle.setup(st, al, Q, h)
    ref = oracle.solve(prob, method="mg", tol=1e-13, max_iters=5000)
    phi, rep = solve_gpu(st, al, Q, h, precision="mixed", tol=1e-8, max_iters=5000,
                         nested_tol=1e-3)
    assert rep["status"] == F.FLD_OK and rep["nested_iterations"] > 0
    assert rel_l2(phi, ref.phi) <= 1e-5


def test_nested_is_skipped_with_a_start_state():
    # an explicit initial fluence bypasses the coarse solve
    st, al, Q, h = media.config("cloud128", n=16)
    phi0 = np.full(st.shape, 1e-3)
    s = F.Solver(st.shape, h, tol=0.0, max_iters=3, nested_tol=1e-3)
    try:
        s.set_medium(st, al, Q)
        phi, rep = s.solve(phi_init=phi0)
    finally:
        s.close()
    assert rep["nested_iterations"] == 0
    ref = oracle.solve(oracle.setup(st, al, Q, h), method="mg", phi=phi0, tol=0.0, max_iters=3)
    assert rep["iterations"] == ref.iterations == 3
    assert rel_l2(phi, ref.phi) <= 1e-10


def test_nested_batch_equals_individual_nested_solves():
    # the coarse batch and the coarse context of a single solve compute the
    # same bits, and so do the fine solves started from their fluence
    vols = media.batch_config(nvol=3, size_scale=0.25, seed=3)
    dims = [(v["n"],) * 3 for v in vols]
    o = F.fld_default_options(precision="mixed", tol=1e-6, max_iters=3000, nested_tol=1e-2)
    b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
    try:
        for i, v in enumerate(vols):
            F.fld_batch_set_volume(b, i, v["sigma_t"], v["albedo"], v["Q"])
        shapes = [d for d in dims for _ in range(3)]
        outs, iters, rep = F.fld_batch_solve(b, shapes)
    finally:
        F.fld_batch_destroy(b)
    assert rep["status"] == F.FLD_OK and rep["nested_iterations"] > 0
    q = 0
    for v in vols:
        for c in range(3):
            phi, r = solve_gpu(v["sigma_t"], v["albedo"][c], v["Q"][c], v["h"],
                               precision="mixed", tol=1e-6, max_iters=3000, nested_tol=1e-2)
            assert r["nested_iterations"] > 0
            assert r["iterations"] == iters[q]
            np.testing.assert_array_equal(outs[q], phi)
            q += 1
