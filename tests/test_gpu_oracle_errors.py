"""GPU results against the FP64 CPU oracle at the sizes of the benchmark
workloads, with every measured error recorded (``parity_record``).

* Batched form (16 cloud volumes of sizes {64..192}^3 x 3 colour channels,
  one shared extinction per volume, albedo 0.99 / 0.95 / 0.9; Sec. 6's
  per-channel albedo pattern): volumes of that generator at 64^3 and 96^3,
  FP64 batch iterates against the oracle solving each (volume, channel) alone,
  and the mixed batch solved to 1e-10 against the oracle solved to its floor.
* 128^3 cloud, plain FP64 multigrid V(2,2) to 1e-8, and the mixed form to
  1e-10, against the oracle's fixed point.
* Multigrid on grids whose z extent is not a multiple of 4 (one cell per
  thread, natural order) or of 8 (quads without the colour-split storage).

Gates: FP64 iterates 1e-10 relative L2 (same method, options and iteration
count); a converged mixed result 1e-5 against the FP64 oracle at its residual
floor.  A result solved only to a looser tolerance (the 1e-8 of the 128^3
FP64 workload) is checked against the error that tolerance allows and the
measured value is recorded.
"""
import numpy as np
import pytest

import oracle
from synth import media

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_1403_8105_amd")

ALBEDOS = (0.99, 0.95, 0.9)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


_fixed = {}


def oracle_floor(key, prob, tol, max_iters=3000, **kw):
    """The oracle's multigrid solve to `tol`, cached per key.  Any schedule
    reaches the same fixed point.  The residual floor of these media lies
    between 1e-13 and 3e-11 depending on the medium, so the references stop at
    1e-10: such a solution differs from the one at the floor by 5e-12 to 3e-11
    (relative L2, measured on the 64^3 batch volumes and the small ragged
    grids), far below the 1e-5 gate."""
    if key not in _fixed:
        r = oracle.solve(prob, method="mg", tol=tol, max_iters=max_iters, **kw)
        assert r.status == "converged", (key, r.status, r.rel)
        _fixed[key] = r
    return _fixed[key]


def c3_volumes():
    return [media.batch_volume(64, 0, ALBEDOS), media.batch_volume(96, 1, ALBEDOS)]


def make_batch(vols, **kw):
    o = F.fld_default_options(**kw)
    b = F.fld_batch_create(o, [(v["n"],) * 3 for v in vols], [v["h"] for v in vols],
                           len(ALBEDOS))
    for q, v in enumerate(vols):
        F.fld_batch_set_volume(b, q, v["sigma_t"], v["albedo"], v["Q"])
    return b


def test_batch_fp64_iterates_match_oracle_at_batch_sizes(parity_record):
    vols = c3_volumes()
    shapes = [(v["n"],) * 3 for v in vols for _ in ALBEDOS]
    for k in (2, 6):
        b = make_batch(vols, tol=0.0, max_iters=k)
        outs, iters, _ = F.fld_batch_solve(b, shapes)
        F.fld_batch_destroy(b)
        q = 0
        for v in vols:
            for c, a in enumerate(ALBEDOS):
                prob = oracle.setup(v["sigma_t"], v["albedo"][c], v["Q"][c], v["h"])
                ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k)
                err = rel_l2(outs[q], ref.phi)
                parity_record(test="batch_fp64_iterates", n=v["n"], albedo=a, iterations=k,
                              rel_l2=err)
                assert iters[q] == ref.iterations == k
                assert err <= 1e-10, (v["n"], a, k, err)
                q += 1


def test_batch_mixed_to_1e10_against_oracle_floor(parity_record):
    vols = c3_volumes()
    shapes = [(v["n"],) * 3 for v in vols for _ in ALBEDOS]
    b = make_batch(vols, precision="mixed", tol=1e-10, max_iters=4000)
    outs, iters, rep = F.fld_batch_solve(b, shapes)
    F.fld_batch_destroy(b)
    assert rep["status"] == F.FLD_OK
    q = 0
    for v in vols:
        for c, a in enumerate(ALBEDOS):
            prob = oracle.setup(v["sigma_t"], v["albedo"][c], v["Q"][c], v["h"])
            # the residual floor of these media lies between 1e-11 and 3e-11;
            # the oracle stops at 1e-10 (about 300-600 iterations)
            ref = oracle_floor(("c3", v["n"], a), prob, 1e-10)
            err = rel_l2(outs[q], ref.phi)
            _, rel_o, _ = oracle.nonlinear_residual(prob, outs[q])
            parity_record(test="batch_mixed_vs_oracle_floor", n=v["n"], albedo=a,
                          gpu_iterations=int(iters[q]), oracle_iterations=ref.iterations,
                          oracle_rel=ref.rel, gpu_rel_by_oracle=rel_o, rel_l2=err)
            assert err <= 1e-5, (v["n"], a, err)
            assert rel_o <= 1.5e-10
            q += 1


# the oracle's reference solve at 128^3 uses the schedule tuned for that grid
# (about 300 iterations instead of 669; same fixed point)
FAST128 = dict(nu1=2, nu2=2, omega_s=1.15, corr_scale=1.4, nested_tol=1e-2)


def cloud128():
    st, al, Q, h = media.config("cloud128")
    return st, al, Q, h, oracle.setup(st, al, Q, h)


def test_c1_fp64_128_iterates_and_error_at_1e8(parity_record):
    st, al, Q, h, prob = cloud128()
    ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=3)
    s = F.Solver(st.shape, h, tol=0.0, max_iters=3)
    s.set_medium(st, al, Q)
    phi, rep = s.solve()
    s.close()
    np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
    err_it = rel_l2(phi, ref.phi)
    assert err_it <= 1e-10
    # the 128^3 workload: plain FP64 V(2,2) (defaults) to 1e-8
    s = F.Solver(st.shape, h, tol=1e-8, max_iters=5000)
    s.set_medium(st, al, Q)
    phi, rep = s.solve()
    s.close()
    assert rep["status"] == F.FLD_OK and rep["rel"] <= 1e-8
    fixed = oracle_floor("cloud128", prob, 1e-10, **FAST128)
    err = rel_l2(phi, fixed.phi)
    parity_record(test="c1_fp64_128_to_1e-8_vs_oracle_floor", gpu_iterations=rep["iterations"],
                  gpu_rel=rep["rel"], oracle_iterations=fixed.iterations, oracle_rel=fixed.rel,
                  rel_l2=err, iterate_rel_l2=err_it)
    # a residual of 1e-8 leaves an error of the order of 1e-8 times the
    # conditioning of the near-vacuum operator
    assert err <= 1e-4


def test_mixed_128_to_1e10_against_oracle_floor(parity_record):
    st, al, Q, h, prob = cloud128()
    s = F.Solver(st.shape, h, precision="mixed", tol=1e-10, max_iters=5000)
    s.set_medium(st, al, Q)
    phi, rep = s.solve()
    s.close()
    assert rep["status"] == F.FLD_OK
    fixed = oracle_floor("cloud128", prob, 1e-10, **FAST128)
    err = rel_l2(phi, fixed.phi)
    _, rel_o, _ = oracle.nonlinear_residual(prob, phi)
    parity_record(test="mixed_128_to_1e-10_vs_oracle_floor", gpu_iterations=rep["iterations"],
                  gpu_rel=rep["rel"], gpu_rel_by_oracle=rel_o, oracle_iterations=fixed.iterations,
                  oracle_rel=fixed.rel, rel_l2=err)
    assert err <= 1e-5
    assert rel_o <= 1.5e-10


def ragged_cloud(shape, seed):
    v = media.value_noise(shape, 4, seed)
    st = media.cloud_extinction(v, 200.0, 0.4)
    al = np.full(shape, 0.99)
    h = 1.0 / max(shape)
    return st, al, media.beer_lambert_source(st, al, h), h


@pytest.mark.parametrize("shape", [(16, 16, 10), (16, 24, 10), (24, 16, 20)])
def test_mg_iterates_on_grids_off_the_quad_and_split_paths(shape, parity_record):
    # nz = 10: one cell per thread in every finest pass and the smoother's pair
    # walk; nz = 20: quads in natural order (no colour-split storage)
    st, al, Q, h = ragged_cloud(shape, seed=sum(shape))
    prob = oracle.setup(st, al, Q, h)
    for k in (1, 4, 12):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k)
        s = F.Solver(shape, h, tol=0.0, max_iters=k)
        s.set_medium(st, al, Q)
        phi, rep = s.solve()
        s.close()
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
        assert rel_l2(phi, ref.phi) <= 1e-10, k
    fixed = oracle_floor(("ragged", shape), prob, 1e-10)
    s = F.Solver(shape, h, precision="mixed", tol=1e-10, max_iters=3000)
    s.set_medium(st, al, Q)
    phi, rep = s.solve()
    s.close()
    assert rep["status"] == F.FLD_OK
    err = rel_l2(phi, fixed.phi)
    parity_record(test="mixed_off_quad_paths_vs_oracle_floor", shape=list(shape),
                  gpu_iterations=rep["iterations"], rel_l2=err)
    assert err <= 1e-5
