"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

FP64 form: same method, options and iteration count => relative L2 error
<= 1e-10 (expected ~1e-13; differences come only from the summation order of
reductions and from library exp/sqrt).  Mixed form (FP32 V-cycle, FP64
outer residual and update): the converged fluence against the oracle solved
to its residual floor, relative L2 <= 1e-5.
"""
import numpy as np
import pytest

import oracle
from synth import media

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_1403_8105_amd")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_solver(shape, h, st, al, Q, **kw):
    s = F.Solver(shape, h, **kw)
    s.set_medium(st, al, Q)
    return s


def ragged_cloud(shape, seed=11, sigma_max=200.0, p_vac=0.4, albedo=0.99):
    v = media.value_noise(shape, 4, seed)
    st = media.cloud_extinction(v, sigma_max, p_vac)
    al = np.full(shape, albedo)
    h = 1.0 / max(shape)
    return st, al, media.beer_lambert_source(st, al, h), h


@pytest.mark.parametrize("lim", ["lp", "cda", "kershaw", "larsen"])
def test_residual_parity(lim):
    shape = (21, 18, 13)
    st, al, Q, h = ragged_cloud(shape)
    rng = np.random.default_rng(1)
    phi = rng.uniform(0.0, 1.0, shape) * (rng.random(shape) > 0.05)   # some zero voxels
    prob = oracle.setup(st, al, Q, h, limiter=lim)
    r_ref, rel_ref, _ = oracle.nonlinear_residual(prob, phi)
    s = gpu_solver(shape, h, st, al, Q, limiter=lim, method="rbsor")
    r, rel = s.residual(phi)
    assert np.max(np.abs(r - r_ref)) <= 1e-12 * np.max(np.abs(r_ref))
    assert rel == pytest.approx(rel_ref, rel=1e-12)


@pytest.mark.parametrize("case", ["point16", "ragged", "cloud32"])
def test_alg1_iterate_parity(case):
    if case == "point16":
        st, al, Q, h = media.point_source(16)
    elif case == "ragged":
        st, al, Q, h = ragged_cloud((19, 23, 17))
    else:
        st, al, Q, h = media.config("cloud128", n=32)
    prob = oracle.setup(st, al, Q, h)
    for k in (1, 2, 7, 40):
        ref = oracle.solve(prob, method="alg1", tol=0.0, max_iters=k, check_every=10 ** 6)
        s = gpu_solver(st.shape, h, st, al, Q, method="rbsor", tol=0.0, max_iters=k,
                       check_every=10 ** 6)
        phi, rep = s.solve()
        assert rep["iterations"] == ref.iterations == k
        assert rel_l2(phi, ref.phi) <= 1e-12, k
        assert rep["rel_sweep"] == pytest.approx(ref.rel_sweep, rel=1e-9)


def test_c0_point_source_alg1_to_tolerance():
    # 32^3, sigma_t = 10, albedo 0.9, unit point source, Red-black GS to 1e-10.
    st, al, Q, h = media.point_source(32)
    for lim in ("lp", "cda"):
        prob = oracle.setup(st, al, Q, h, limiter=lim)
        ref = oracle.solve(prob, method="alg1", tol=1e-10, max_iters=20000, check_every=10)
        s = gpu_solver(st.shape, h, st, al, Q, limiter=lim, method="rbsor", tol=1e-10,
                       max_iters=20000, check_every=10)
        phi, rep = s.solve()
        assert rep["status"] == F.FLD_OK
        assert rep["iterations"] == ref.iterations
        assert rel_l2(phi, ref.phi) <= 1e-10
        assert rep["rel"] <= 1e-10


@pytest.mark.parametrize("shape,lim", [((32, 32, 32), "lp"), ((32, 32, 32), "cda"),
                                       ((32, 16, 24), "lp"), ((24, 24, 24), "lp")])
def test_mg_fp64_iterate_parity(shape, lim):
    st, al, Q, h = ragged_cloud(shape, seed=5)
    prob = oracle.setup(st, al, Q, h, limiter=lim)
    for k in (1, 2, 5, 12):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k)
        s = gpu_solver(shape, h, st, al, Q, limiter=lim, tol=0.0, max_iters=k)
        phi, rep = s.solve()
        assert rep["iterations"] == ref.iterations == k
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
        assert rel_l2(phi, ref.phi) <= 1e-10, k


def test_mg_fp64_converged_matches_oracle_fixed_point():
    # the residual floor of this medium is ~3e-12; both solve to 1e-11
    st, al, Q, h = media.config("cloud128", n=32)
    prob = oracle.setup(st, al, Q, h)
    ref = oracle.solve(prob, method="mg", tol=1e-11, max_iters=1000)
    assert ref.status == "converged"
    s = gpu_solver(st.shape, h, st, al, Q, tol=1e-11, max_iters=1000)
    phi, rep = s.solve()
    assert rep["status"] == F.FLD_OK and rep["rel"] <= 1e-11
    assert abs(rep["iterations"] - ref.iterations) <= 2
    assert rel_l2(phi, ref.phi) <= 1e-9


@pytest.mark.parametrize("n", [32, 64])
def test_mg_mixed_against_fp64_oracle(n):
    st, al, Q, h = media.config("cloud128", n=n)
    prob = oracle.setup(st, al, Q, h)
    # reference: FP64 oracle to 1e-11 (its error is ~1e-12 relative; the
    # residual floor of these media is ~1e-11)
    ref = oracle.solve(prob, method="mg", tol=1e-11, max_iters=2000)
    assert ref.status == "converged"
    s = gpu_solver(st.shape, h, st, al, Q, precision="mixed", tol=1e-10, max_iters=2000)
    phi, rep = s.solve()
    assert rep["status"] == F.FLD_OK
    err = rel_l2(phi, ref.phi)
    print(f"mixed n={n}: iterations {rep['iterations']}, rel {rep['rel']:.2e}, err {err:.2e}")
    assert err <= 1e-5
    # the oracle confirms the claimed residual of the GPU fluence
    _, rel_o, _ = oracle.nonlinear_residual(prob, phi)
    assert rel_o <= 1.5e-10


def test_resume_is_bit_exact():
    # k iterations, stop, resume for k more == 2k iterations in one go
    st, al, Q, h = ragged_cloud((32, 32, 32), seed=3)
    for prec in ("fp64", "mixed"):
        c = gpu_solver(st.shape, h, st, al, Q, precision=prec, tol=0.0, max_iters=3)
        c.solve()
        part, rep = c.resume()
        assert rep["iterations"] == 6
        d = gpu_solver(st.shape, h, st, al, Q, precision=prec, tol=0.0, max_iters=6)
        six, _ = d.solve()
        np.testing.assert_array_equal(part, six)


def test_phi_init_and_zero_emission():
    st, al, Q, h = media.point_source(16)
    prob = oracle.setup(st, al, Q, h)
    start = np.full(st.shape, 0.5)
    ref = oracle.solve(prob, method="mg", phi=start, tol=0.0, max_iters=3)
    s = gpu_solver(st.shape, h, st, al, Q, tol=0.0, max_iters=3)
    phi, _ = s.solve(phi_init=start)
    assert rel_l2(phi, ref.phi) <= 1e-10
    z = gpu_solver(st.shape, h, st, al, np.zeros_like(Q))
    phi, rep = z.solve()
    assert rep["status"] == F.FLD_OK and np.all(phi == 0.0)


def test_batch_equals_individual_solves():
    vols = media.batch_config(nvol=3, size_scale=0.25, seed=3)
    dims = [(v["n"],) * 3 for v in vols]
    o = F.fld_default_options(precision="mixed", tol=1e-6, max_iters=3000)
    b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
    for i, v in enumerate(vols):
        F.fld_batch_set_volume(b, i, v["sigma_t"], v["albedo"], v["Q"])
    shapes = [d for d in dims for _ in range(3)]
    outs, iters, rep = F.fld_batch_solve(b, shapes)
    F.fld_batch_destroy(b)
    assert rep["status"] == F.FLD_OK
    q = 0
    for v in vols:
        for c in range(3):
            s = gpu_solver((v["n"],) * 3, v["h"], v["sigma_t"], v["albedo"][c], v["Q"][c],
                           precision="mixed", tol=1e-6, max_iters=3000)
            phi, r = s.solve()
            assert r["iterations"] == iters[q]
            np.testing.assert_array_equal(outs[q], phi)
            q += 1


def test_solve_before_medium_is_state_error():
    s = F.Solver((8, 8, 8), 0.125)
    with pytest.raises(F.FldError) as ei:
        s.solve()
    assert ei.value.status == F.FLD_ERR_STATE


def test_invalid_medium_is_rejected():
    st, al, Q, h = media.point_source(8)
    s = F.Solver(st.shape, h)
    bad = al.copy()
    bad[1, 2, 3] = 1.5
    with pytest.raises(F.FldError) as ei:
        s.set_medium(st, bad, Q)
    assert ei.value.status == F.FLD_ERR_INVALID_ARGUMENT
    assert "albedo[" in str(ei.value)


def test_not_converged_still_writes_phi():
    st, al, Q, h = media.point_source(16)
    s = gpu_solver(st.shape, h, st, al, Q, tol=1e-14, max_iters=2)
    phi, rep = s.solve()
    assert rep["status"] == F.FLD_ERR_NOT_CONVERGED and rep["iterations"] == 2
    assert np.all(np.isfinite(phi)) and phi.max() > 0


@pytest.mark.parametrize("tau", [0.0, 1.0])
def test_mg_deflation_iterate_parity(tau):
    # the 256^3-generator medium has strongly coupled vacuum clusters
    st, al, Q, h = media.config("cloud256", n=32)
    prob = oracle.setup(st, al, Q, h)
    lab, K = oracle.clusters(prob, 1.0)
    assert K > 0
    for k in (1, 2, 6, 15):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, deflate_tau=tau)
        s = gpu_solver(st.shape, h, st, al, Q, tol=0.0, max_iters=k, deflate_tau=tau)
        phi, rep = s.solve()
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
        assert rel_l2(phi, ref.phi) <= 1e-10, k


def test_mg_deflated_solve_converges_like_the_oracle():
    st, al, Q, h = media.config("cloud256", n=32)
    prob = oracle.setup(st, al, Q, h)
    ref = oracle.solve(prob, method="mg", tol=1e-8, max_iters=3000)
    for prec in ("fp64", "mixed"):
        s = gpu_solver(st.shape, h, st, al, Q, precision=prec, tol=1e-8, max_iters=3000)
        phi, rep = s.solve()
        assert rep["status"] == F.FLD_OK
        assert rep["iterations"] <= 1.25 * ref.iterations
        assert rel_l2(phi, ref.phi) <= (1e-6 if prec == "mixed" else 1e-7)


def test_graph_replay_is_bit_identical():
    # outer iterations replayed from captured HIP graphs give the same bits
    # as launching every kernel; checked over several replays of both graphs
    st, al, Q, h = media.config("cloud256", n=32)
    outs = []
    for graph in (0, 1):
        for timing in (0, 1):
            s = gpu_solver(st.shape, h, st, al, Q, precision="mixed", tol=0.0, max_iters=9,
                           graph=graph, timing=timing)
            phi, rep = s.solve()
            outs.append((phi, rep))
            if timing:
                assert rep["kernel_launches"][0] > 0 and rep["kernel_ms"][0] > 0
    for phi, rep in outs[1:]:
        np.testing.assert_array_equal(phi, outs[0][0])
        np.testing.assert_array_equal(rep["history"], outs[0][1]["history"])
    # events recorded inside the graphs time the same launches as eager ones
    assert outs[3][1]["kernel_launches"] == outs[1][1]["kernel_launches"]
    assert outs[3][1]["kernel_bytes"] == outs[1][1]["kernel_bytes"]
    # finest half-sweep in FP32: black e, all of D, red b and sa, red e written
    rep = outs[1][1]
    assert rep["kernel_bytes"][0] == rep["kernel_launches"][0] * 12.0 * st.size


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("shape,omega_s", [((32, 32, 32), 1.0), ((24, 16, 40), 1.0),
                                           ((16, 16, 8), 1.0), ((32, 24, 16), 1.2)])
def test_colour_split_is_bit_identical(shape, omega_s, precision):
    # the red/black storage of the V-cycle's finest fields (FP32 in the mixed
    # form, FP64 in the FP64 form) changes where values live, not how they
    # are computed
    st, al, Q, h = ragged_cloud(shape, seed=7)
    outs = []
    for split in (0, 1):
        s = gpu_solver(shape, h, st, al, Q, precision=precision, tol=0.0, max_iters=8,
                       omega_s=omega_s, colour_split=split)
        outs.append(s.solve())
    np.testing.assert_array_equal(outs[1][0], outs[0][0])
    np.testing.assert_array_equal(outs[1][1]["history"], outs[0][1]["history"])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_launch_shapes_are_bit_identical(prec):
    # task sizes and the one-workgroup deep part of the V-cycle change where
    # and how work is launched, not what is computed
    st, al, Q, h = ragged_cloud((32, 32, 48), seed=9)
    outs = []
    for tc0, cb, deep in ((4096, 2048, 0), (512, 64, 4096), (65536, 65536, 100000),
                          (4096, 2048, 1)):
        s = gpu_solver(st.shape, h, st, al, Q, precision=prec, tol=0.0, max_iters=6,
                       task_cells0=tc0, coarse_blocks=cb, deep_cells=deep)
        outs.append(s.solve())
    for phi, rep in outs[1:]:
        np.testing.assert_array_equal(phi, outs[0][0])
        np.testing.assert_array_equal(rep["history"], outs[0][1]["history"])


def test_batch_deep_cycle_bit_identical():
    vols = media.batch_config(nvol=3, size_scale=0.25, seed=5)
    dims = [(v["n"],) * 3 for v in vols]
    shapes = [d for d in dims for _ in range(3)]
    res = []
    for deep in (0, 4096):
        o = F.fld_default_options(precision="mixed", tol=0.0, max_iters=5, deep_cells=deep)
        b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
        for i, v in enumerate(vols):
            F.fld_batch_set_volume(b, i, v["sigma_t"], v["albedo"], v["Q"])
        outs, _, _ = F.fld_batch_solve(b, shapes)
        F.fld_batch_destroy(b)
        res.append(outs)
    for a, b_ in zip(*res):
        np.testing.assert_array_equal(a, b_)


def test_batch_mixing_split_and_natural_volumes():
    # nz % 8 == 0 volumes use the colour-split storage, the 24x16x20 one the
    # natural order; one batch holds both and each result equals its own solve
    shapes = [(16, 16, 16), (24, 16, 20), (16, 24, 32)]
    vols = [ragged_cloud(sh, seed=20 + q) for q, sh in enumerate(shapes)]
    albs = (0.99, 0.9)
    o = F.fld_default_options(precision="mixed", tol=0.0, max_iters=7)
    b = F.fld_batch_create(o, shapes, [v[3] for v in vols], len(albs))
    for q, (st, _, _, h) in enumerate(vols):
        al = [np.full(st.shape, a) for a in albs]
        F.fld_batch_set_volume(b, q, st, al, [media.beer_lambert_source(st, x, h) for x in al])
    outs, iters, rep = F.fld_batch_solve(b, [sh for sh in shapes for _ in albs])
    F.fld_batch_destroy(b)
    r = 0
    for st, _, _, h in vols:
        for a in albs:
            al = np.full(st.shape, a)
            s = gpu_solver(st.shape, h, st, al, media.beer_lambert_source(st, al, h),
                           precision="mixed", tol=0.0, max_iters=7)
            phi, rep1 = s.solve()
            assert iters[r] == rep1["iterations"] == 7
            np.testing.assert_array_equal(outs[r], phi)
            r += 1


@pytest.mark.parametrize("nu1,nu2,omega_s,growth,scale", [
    (1, 1, 1.0, 2.0, 1.0), (2, 1, 1.0, 2.0, 1.0), (1, 2, 1.0, 2.0, 1.0), (3, 3, 1.0, 10.0, 1.0),
    (2, 2, 1.15, 2.0, 1.4), (3, 3, 1.15, 10.0, 1.6), (2, 2, 1.0, 0.0, 1.4),
    (3, 3, 1.15, 2.0, 2.0), (4, 4, 1.15, 2.0, 2.0), (3, 3, 1.3, 10.0, 1.8)])
def test_mg_schedules_iterate_parity(nu1, nu2, omega_s, growth, scale):
    # every schedule, restart factor and correction factor the autotuner may
    # pick (and every cached one) follows the oracle
    st, al, Q, h = media.config("cloud256", n=32)
    prob = oracle.setup(st, al, Q, h)
    kw = dict(nu1=nu1, nu2=nu2, omega_s=omega_s, restart_growth=growth, corr_scale=scale)
    for k in (1, 3, 10, 30):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k, **kw)
        s = gpu_solver(st.shape, h, st, al, Q, tol=0.0, max_iters=k, **kw)
        phi, rep = s.solve()
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
        assert rel_l2(phi, ref.phi) <= 1e-10, k
    # and the mixed form still converges with it
    s = gpu_solver(st.shape, h, st, al, Q, precision="mixed", tol=1e-6, max_iters=1000, **kw)
    _, rep = s.solve()
    assert rep["status"] == F.FLD_OK


def test_full_size_256_in_the_bench_configuration():
    # the bench's grid and options: FP64 multigrid iterates follow the oracle,
    # and the mixed solve's fluence has, per the oracle, the residual it reports
    from paper_1403_8105_amd.autotune import tuned_options

    st, al, Q, h = media.config("cloud256")
    prob = oracle.setup(st, al, Q, h)
    ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=2)
    s = gpu_solver(st.shape, h, st, al, Q, tol=0.0, max_iters=2)
    phi, rep = s.solve()
    s.close()
    np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
    assert rel_l2(phi, ref.phi) <= 1e-10
    opts = tuned_options(st.shape, "mixed", "lp")
    s = gpu_solver(st.shape, h, st, al, Q, precision="mixed", tol=1e-6, max_iters=5000, **opts)
    phi, rep = s.solve()
    s.close()
    assert rep["status"] == F.FLD_OK and rep["rel"] <= 1e-6
    _, rel_o, _ = oracle.nonlinear_residual(prob, phi)
    assert rel_o == pytest.approx(rep["rel"], rel=1e-9)


@pytest.mark.parametrize("lim", ["sum", "max"])
def test_residual_parity_remaining_limiters(lim):
    shape = (21, 18, 13)
    st, al, Q, h = ragged_cloud(shape)
    rng = np.random.default_rng(2)
    phi = rng.uniform(0.0, 1.0, shape) * (rng.random(shape) > 0.05)
    prob = oracle.setup(st, al, Q, h, limiter=lim)
    r_ref, rel_ref, _ = oracle.nonlinear_residual(prob, phi)
    s = gpu_solver(shape, h, st, al, Q, limiter=lim, method="rbsor")
    r, rel = s.residual(phi)
    assert np.max(np.abs(r - r_ref)) <= 1e-12 * np.max(np.abs(r_ref))
    assert rel == pytest.approx(rel_ref, rel=1e-12)


@pytest.mark.parametrize("g", [0.3, 0.8])
def test_anisotropy_iterate_parity(g):
    # reduced extinction in D and R: FP64 multigrid iterates follow the oracle
    st, al, Q, h = ragged_cloud((32, 24, 32), seed=13)
    prob = oracle.setup(st, al, Q, h, aniso_g=g)
    for k in (1, 4, 12):
        ref = oracle.solve(prob, method="mg", tol=0.0, max_iters=k)
        s = gpu_solver(st.shape, h, st, al, Q, tol=0.0, max_iters=k, anisotropy_g=g)
        phi, rep = s.solve()
        np.testing.assert_allclose(rep["history"], ref.history, rtol=1e-9)
        assert rel_l2(phi, ref.phi) <= 1e-10, k
    # Algorithm 1 as well
    ref = oracle.solve(prob, method="alg1", tol=0.0, max_iters=20, check_every=10 ** 6)
    s = gpu_solver(st.shape, h, st, al, Q, method="rbsor", tol=0.0, max_iters=20,
                   check_every=10 ** 6, anisotropy_g=g)
    phi, _ = s.solve()
    assert rel_l2(phi, ref.phi) <= 1e-12
