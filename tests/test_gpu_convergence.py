"""GPU parity of Algorithm 1 (red-black SOR, Sec. 5) on the convergence test
case of Fig. 3: the spherical cloud in vacuum with a noise emission field,
over-relaxed (omega != 1), with a non-default extinction floor sigma_eps, and
on a case that diverges.  FP64 iterates against the oracle, relative L2
<= 1e-12 for the same iteration count.
"""
import numpy as np
import pytest

import oracle
from synth import media

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_1403_8105_amd")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run_gpu(st, al, Q, h, **kw):
    s = F.Solver(st.shape, h, method="rbsor", **kw)
    try:
        s.set_medium(st, al, Q)
        return s.solve(allow=(F.FLD_OK, F.FLD_ERR_NOT_CONVERGED, F.FLD_ERR_DIVERGED))
    finally:
        s.close()


@pytest.mark.parametrize("shape,lim,omega", [((17, 17, 17), "lp", 1.4),
                                             ((21, 19, 23), "lp", 1.7),
                                             ((17, 17, 17), "cda", 1.9),
                                             ((20, 20, 20), "kershaw", 1.2)])
def test_alg1_sphere_over_relaxed_iterates(shape, lim, omega):
    st, al, Q, h = media.sphere_cloud(shape)
    prob = oracle.setup(st, al, Q, h, limiter=lim)
    for k in (1, 7, 60):
        ref = oracle.solve(prob, method="alg1", omega=omega, tol=0.0, max_iters=k,
                           check_every=10 ** 6)
        phi, rep = run_gpu(st, al, Q, h, limiter=lim, omega=omega, tol=0.0, max_iters=k,
                           check_every=10 ** 6)
        assert rep["iterations"] == ref.iterations == k
        assert rel_l2(phi, ref.phi) <= 1e-12, k
        assert rep["rel_sweep"] == pytest.approx(ref.rel_sweep, rel=1e-9)


@pytest.mark.parametrize("floor", [1e-1, 1e-5])
def test_alg1_sphere_to_tolerance_with_extinction_floor(floor):
    # Fig. 3c varies sigma_eps = floor / L; both sides stop on the same check
    st, al, Q, h = media.sphere_cloud(17)
    se = floor / (h * 17)
    prob = oracle.setup(st, al, Q, h, sigma_eps=se)
    ref = oracle.solve(prob, method="alg1", omega=1.3, tol=1e-6, max_iters=20000, check_every=1)
    phi, rep = run_gpu(st, al, Q, h, omega=1.3, tol=1e-6, max_iters=20000, check_every=1,
                       sigma_eps=se)
    assert ref.status == "converged" and rep["status"] == F.FLD_OK
    assert rep["iterations"] == ref.iterations
    assert rel_l2(phi, ref.phi) <= 1e-10
    np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-8)


def test_alg1_divergence_is_reported():
    # LP with omega = 1.9 on the 17^3 sphere grows without bound on both
    # sides; the GPU stops with FLD_ERR_DIVERGED once the residual is not
    # finite, as the oracle does
    st, al, Q, h = media.sphere_cloud(17)
    prob = oracle.setup(st, al, Q, h)
    ref = oracle.solve(prob, method="alg1", omega=1.9, tol=1e-6, max_iters=5000, check_every=1)
    _, rep = run_gpu(st, al, Q, h, omega=1.9, tol=1e-6, max_iters=5000, check_every=1)
    assert ref.status == "diverged"
    assert rep["status"] == F.FLD_ERR_DIVERGED
    assert abs(rep["iterations"] - ref.iterations) <= 0.05 * ref.iterations
    # the unstable mode grows about 1.4x per iteration and amplifies the
    # rounding differences of the two sides alike, so the histories agree
    # closely only over the first few dozen iterations
    np.testing.assert_allclose(rep["history"][:30], ref.history[:30], rtol=1e-6)
