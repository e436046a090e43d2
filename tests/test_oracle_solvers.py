"""Pins of the oracle's solvers: Algorithm 1 (red-black SOR, Sec. 5) and the
Picard-multigrid/nonlinear-PCG solve.

References: scipy's sparse direct solver on the CDA system (a special case
that reduces to a library routine), a brute-force Picard iteration with an
exact sparse solve per step for FLD on small grids, agreement of the two
different iterations on the same fixed point, the closed-form CDA Green's
function of a point source (Sec. 4.1, equation cda_greensfunction) with its
second-order approach under grid refinement, and the discrete power balance
at convergence.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spl

from synth import media
from test_oracle_operator import assemble

EPS = 1e-20
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def direct_cda(prob, h):
    D = np.full(prob.shape, (1.0 / 3.0)) / prob.sig_hat
    M = assemble(D, prob.sig_a, h, EPS * h).tocsc()
    return spl.spsolve(M, prob.j.ravel() * h * h).reshape(prob.shape)


@pytest.mark.parametrize("case", ["point", "cloud"])
def test_cda_matches_sparse_direct_solve(oracle_mod, case):
    if case == "point":
        st, al, Q, h = media.point_source(12, sigma_t=10.0, albedo=0.5)
    else:
        st, al, Q, h = media.config("cloud128", n=16)
    prob = oracle_mod.setup(st, al, Q, h, limiter="cda")
    ref = direct_cda(prob, h)
    mg = oracle_mod.solve(prob, method="mg", tol=1e-14, max_iters=400)
    assert mg.status == "converged"
    assert np.linalg.norm(mg.phi - ref) <= 1e-11 * np.linalg.norm(ref)
    if case == "point":
        a1 = oracle_mod.solve(prob, method="alg1", tol=1e-14, max_iters=20000, check_every=25)
        assert a1.status == "converged"
        assert np.linalg.norm(a1.phi - ref) <= 1e-11 * np.linalg.norm(ref)


def picard_direct(oracle_mod, prob, h, iters=400, tol=1e-14):
    """FLD fixed point by Picard iteration with an exact sparse solve each step."""
    phi, _ = prob.init_state()
    for _ in range(iters):
        D = oracle_mod.limiter_pass(prob, phi)
        M = assemble(D, prob.sig_a, h, EPS * h).tocsc()
        new = spl.spsolve(M, prob.j.ravel() * h * h).reshape(prob.shape)
        if np.linalg.norm(new - phi) <= tol * np.linalg.norm(new):
            return new
        phi = new
    raise AssertionError("brute-force Picard did not settle")


@pytest.mark.parametrize("case", ["point", "cloud"])
def test_fld_fixed_point_brute_force(oracle_mod, case):
    if case == "point":
        st, al, Q, h = media.point_source(8, sigma_t=10.0, albedo=0.9)
    else:
        st, al, Q, h = media.config("cloud128", n=8)
    prob = oracle_mod.setup(st, al, Q, h, limiter="lp")
    ref = picard_direct(oracle_mod, prob, h)
    # residual floor of these systems is ~1e-13 (the reference itself sits there)
    mg = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=2000)
    assert mg.status == "converged"
    assert np.linalg.norm(mg.phi - ref) <= 1e-10 * np.linalg.norm(ref)
    a1 = oracle_mod.solve(prob, method="alg1", tol=1e-12, max_iters=200000, check_every=50)
    assert a1.status == "converged"
    assert np.linalg.norm(a1.phi - ref) <= 1e-10 * np.linalg.norm(ref)


def test_alg1_and_multigrid_share_the_fixed_point(oracle_mod):
    st, al, Q, h = media.point_source(16, sigma_t=10.0, albedo=0.9)
    prob = oracle_mod.setup(st, al, Q, h, limiter="lp")
    a1 = oracle_mod.solve(prob, method="alg1", tol=1e-13, max_iters=100000, check_every=20)
    mg = oracle_mod.solve(prob, method="mg", tol=1e-13, max_iters=400)
    assert a1.status == mg.status == "converged"
    assert np.linalg.norm(a1.phi - mg.phi) <= 1e-10 * np.linalg.norm(mg.phi)


def closed_form(r, sigma_t=10.0, albedo=0.9):
    # CDA Green's function of a unit-power point source, Sec. 4.1
    # (cda_greensfunction): phi = 3 sigma_t^2 exp(-sqrt(3(1-a)) tau) / (4 pi tau).
    tau = sigma_t * r
    return 3 * sigma_t ** 2 * np.exp(-np.sqrt(3 * (1 - albedo)) * tau) / (4 * np.pi * tau)


def test_golden_closed_form_table():
    with open(os.path.join(GOLDEN, "cda_point_source_closed_form.json")) as f:
        g = json.load(f)
    for r, v in zip(g["r"], g["phi"]):
        assert closed_form(r, g["sigma_t"], g["albedo"]) == pytest.approx(v, rel=1e-14)


def test_point_source_cda_closed_form_and_refinement(oracle_mod):
    # Measured on the 32^3 grid: +5.8, +3.2, +1.8, +1.0 % along the axes at
    # 3..6 voxels, and down to -3.0 % on the diagonals (2,2,2) voxels away;
    # the gates sit just above these.  A stencil with the wrong neighbour set
    # or face average breaks the diagonal points first.
    errs, diag = {}, {}
    offsets = [(2, 2, 0), (2, 2, 1), (2, 2, 2), (3, 2, 1), (3, 3, 0), (4, 3, 2), (3, 3, 3),
               (4, 4, 0)]
    for n in (32, 64):
        st, al, Q, h = media.point_source(n)
        prob = oracle_mod.setup(st, al, Q, h, limiter="cda")
        phi = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=400).phi
        c, s = n // 2, n // 32
        for rr in (3 / 32, 4 / 32, 5 / 32, 6 / 32):
            m = int(round(rr * n))
            along = [phi[c + m, c, c], phi[c - m, c, c], phi[c, c + m, c], phi[c, c, c - m]]
            errs[(n, rr)] = max(abs(v / closed_form(rr) - 1) for v in along)
        for a, b, d in offsets:
            r = np.sqrt(a * a + b * b + d * d) / 32
            pts = [phi[c + a * s, c + b * s, c + d * s], phi[c - a * s, c - b * s, c - d * s],
                   phi[c + d * s, c - a * s, c + b * s], phi[c - b * s, c + d * s, c + a * s]]
            diag[(n, (a, b, d))] = max(abs(v / closed_form(r) - 1) for v in pts)
    for rr, gate in zip((3 / 32, 4 / 32, 5 / 32, 6 / 32), (0.065, 0.036, 0.021, 0.012)):
        assert errs[(32, rr)] < gate, (rr, errs[(32, rr)])
    for off in offsets:
        assert diag[(32, off)] < 0.033, (off, diag[(32, off)])
    # second order: the error at r = 3h(32) falls ~4x with each halving of h,
    # on the axes and on the space diagonal
    assert errs[(64, 3 / 32)] < errs[(32, 3 / 32)] / 4.0
    assert diag[(64, (2, 2, 2))] < diag[(32, (2, 2, 2))] / 2.5


def test_analytic_dirichlet_closes_the_gap(oracle_mod):
    # Fig. 4a: with Dirichlet data from the closed form the CDA solve matches
    # the theory better than with phi = 0 on the boundary.
    n = 32
    st, al, Q, h = media.point_source(n)
    c = n // 2
    fn = lambda I, J, K: closed_form(h * np.sqrt((I - c) ** 2 + (J - c) ** 2 + (K - c) ** 2) + 1e-300)
    from test_oracle_operator import ghost_fill
    g = ghost_fill(np.zeros((n, n, n)), fn)
    zero = oracle_mod.setup(st, al, Q, h, limiter="cda")
    exact = oracle_mod.setup(st, al, Q, h, limiter="cda", ghost_phi=g, mirror_d=True)
    p0 = oracle_mod.solve(zero, method="alg1", tol=1e-11, max_iters=50000, check_every=50).phi
    p1 = oracle_mod.solve(exact, method="alg1", tol=1e-11, max_iters=50000, check_every=50).phi
    err1 = []
    for m in range(9, 16):
        cf = closed_form(m * h)
        for v0, v1 in ((p0[c + m, c, c], p1[c + m, c, c]), (p0[c, c - m, c], p1[c, c - m, c])):
            assert abs(v1 / cf - 1) < abs(v0 / cf - 1)
            assert abs(v1 / cf - 1) < 0.011
        err1.append(abs(p1[c + m, c, c] / cf - 1))
    assert np.all(np.diff(err1) < 0)   # only the near-source discretisation error is left


def test_power_balance_at_convergence(oracle_mod):
    st, al, Q, h = media.point_source(24, sigma_t=10.0, albedo=0.9)
    for lim in ("cda", "lp"):
        prob = oracle_mod.setup(st, al, Q, h, limiter=lim)
        res = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=400)
        D = oracle_mod.limiter_pass(prob, res.phi)
        absorbed = (prob.sig_a * res.phi).sum() * h ** 3
        leak = 0.0
        for ax in range(3):
            for end in (0, -1):
                sl = [slice(None)] * 3
                sl[ax] = end
                leak += (0.5 * (D[tuple(sl)] + EPS * h) * res.phi[tuple(sl)]).sum() * h
        assert absorbed + leak == pytest.approx(1.0, rel=1e-9)   # unit emitted power


def test_zero_emission_returns_boundary_value(oracle_mod):
    st, al, Q, h = media.point_source(8)
    prob = oracle_mod.setup(st, al, np.zeros_like(Q), h, phi_b=0.0)
    for method in ("alg1", "mg"):
        res = oracle_mod.solve(prob, method=method)
        assert res.status == "converged" and res.rel == 0.0
        assert np.all(res.phi == 0.0)


def test_multigrid_levels_rule(oracle_mod):
    lv, ok = oracle_mod.mg_levels(32, 32, 32)
    assert ok and lv == [(32, 32, 32), (16, 16, 16), (8, 8, 8), (4, 4, 4)]
    assert oracle_mod.mg_levels(96, 96, 96)[0][-1] == (6, 6, 6)
    assert oracle_mod.mg_levels(160, 160, 160)[0][-1] == (5, 5, 5)
    assert len(oracle_mod.mg_levels(512, 512, 512)[0]) == 8
    assert not oracle_mod.mg_levels(100, 100, 100)[1]          # 25^3 coarsest > 512
    assert oracle_mod.mg_levels(64, 32, 16)[0][-1] == (16, 8, 4)


def test_cholesky_against_numpy(oracle_mod):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 40))
    M = A @ A.T + 40 * np.eye(40)
    np.testing.assert_allclose(oracle_mod.cholesky(M), np.linalg.cholesky(M), rtol=1e-12, atol=1e-13)
    b = rng.standard_normal(40)
    np.testing.assert_allclose(oracle_mod.cholesky_solve(M, b), np.linalg.solve(M, b), rtol=1e-11)


def test_single_level_vcycle_is_exact(oracle_mod):
    rng = np.random.default_rng(4)
    n, h = 6, 1.0 / 6
    D = rng.uniform(0.01, 3.0, (n, n, n))
    sa = rng.uniform(0.0, 2.0, (n, n, n))
    b = rng.standard_normal((n, n, n))
    e = oracle_mod.linear_vcycle(D, sa, b, h, EPS * h)
    M = assemble(D, sa, h, EPS * h).tocsc()
    ref = spl.spsolve(M, b.ravel() * h * h).reshape(b.shape)
    np.testing.assert_allclose(e, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_clusters_match_connected_components(oracle_mod):
    # Clusters = connected components of the graph of strong faces (classical
    # coefficient ((1/3)/sig_p + (1/3)/sig_s)/2 > tau * L), computed here with scipy.
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    st, al, Q, h = media.config("cloud256", n=24)
    prob = oracle_mod.setup(st, al, Q, h)
    for tau in (0.3, 1.0, 5.0):
        lab, K = oracle_mod.clusters(prob, tau)
        n = st.size
        idx = np.arange(n).reshape(st.shape)
        Dc = (1.0 / 3.0) / prob.sig_hat
        rows, cols = [], []
        for ax in range(3):
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax], hi[ax] = slice(0, -1), slice(1, None)
            F = 0.5 * (Dc[tuple(lo)] + Dc[tuple(hi)])
            m = F > tau * h * 24
            rows.append(idx[tuple(lo)][m])
            cols.append(idx[tuple(hi)][m])
        r, c = np.concatenate(rows), np.concatenate(cols)
        G = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
        nc, comp = connected_components(G, directed=False)
        sizes = np.bincount(comp)
        in_cluster = sizes[comp] > 1
        assert K == int((sizes > 1).sum())
        np.testing.assert_array_equal(lab.ravel() >= 0, in_cluster)
        # same partition: equal labels <=> equal components
        a, b = lab.ravel()[in_cluster], comp[in_cluster]
        pairs = set(zip(a.tolist(), b.tolist()))
        assert len(pairs) == K == len(set(a.tolist())) == len(set(b.tolist()))
        # numbering: by first voxel in index order
        first = [int(np.argmax(lab.ravel() == q)) for q in range(K)]
        assert first == sorted(first)


def test_deflation_keeps_the_fixed_point(oracle_mod):
    st, al, Q, h = media.config("cloud256", n=32)
    prob = oracle_mod.setup(st, al, Q, h)
    a = oracle_mod.solve(prob, method="mg", tol=1e-11, max_iters=3000, deflate_tau=0.0)
    b = oracle_mod.solve(prob, method="mg", tol=1e-11, max_iters=3000, deflate_tau=1.0)
    assert a.status == b.status == "converged"
    assert b.iterations < a.iterations / 2          # the point of deflating
    assert np.linalg.norm(a.phi - b.phi) <= 1e-9 * np.linalg.norm(a.phi)


def test_direction_restarts_keep_the_fixed_point(oracle_mod):
    # restarting the conjugate direction changes the path, not the solution;
    # a growth factor of 1 restarts after every increase of the residual
    st, al, Q, h = media.config("cloud256", n=32)
    prob = oracle_mod.setup(st, al, Q, h)
    runs = [oracle_mod.solve(prob, method="mg", tol=1e-11, max_iters=3000, restart_growth=g)
            for g in (0.0, 1.0, 2.0)]
    assert all(r.status == "converged" for r in runs)
    for r in runs[1:]:
        assert np.linalg.norm(r.phi - runs[0].phi) <= 1e-9 * np.linalg.norm(runs[0].phi)
    # the restart rule is active: with factor 1 the path differs from no restarts
    assert runs[1].iterations != runs[0].iterations or \
        not np.array_equal(runs[1].history, runs[0].history)


def test_reduced_extinction_point_source(oracle_mod):
    # Anisotropy (Sec. 7): D uses sigma_t' = sigma_t (1 - a g), absorption
    # stays (1 - a) sigma_t, so CDA's Green's function has D = 1/(3 sigma_t')
    # and kappa = sqrt(sigma_a / D): phi = exp(-kappa r) / (4 pi D r).  With
    # analytic Dirichlet data the discrete solve follows it within 1.1 % at
    # 9..15 voxels; dropping g, or reducing the absorption too, misses by far.
    n, g = 32, 0.5
    st, al, Q, h = media.point_source(n)
    sig_r = 10.0 * (1 - 0.9 * g)
    D, sa = 1.0 / (3.0 * sig_r), (1 - 0.9) * 10.0
    kappa = np.sqrt(sa / D)
    cf = lambda r: np.exp(-kappa * r) / (4 * np.pi * D * r)
    c = n // 2
    fn = lambda I, J, K: cf(h * np.sqrt((I - c) ** 2 + (J - c) ** 2 + (K - c) ** 2) + 1e-300)
    from test_oracle_operator import ghost_fill
    gh = ghost_fill(np.zeros((n, n, n)), fn)
    prob = oracle_mod.setup(st, al, Q, h, limiter="cda", ghost_phi=gh, mirror_d=True, aniso_g=g)
    phi = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=400).phi
    for m in range(9, 16):
        for v in (phi[c + m, c, c], phi[c, c - m, c], phi[c, c, c + m]):
            assert abs(v / cf(m * h) - 1) < 0.011
    iso = oracle_mod.setup(st, al, Q, h, limiter="cda", ghost_phi=gh, mirror_d=True)
    phi0 = oracle_mod.solve(iso, method="mg", tol=1e-12, max_iters=400).phi
    assert abs(phi0[c + 12, c, c] / cf(12 * h) - 1) > 0.05


@pytest.mark.parametrize("case", ["sphere", "point"])
def test_alg1_sor_rate_follows_young(oracle_mod, case):
    # With CDA the discretised equation is linear (D = 1/(3 sigma_hat) after
    # the first sweep), and red-black ordering of the 7-point stencil is
    # consistently ordered.  Young's theory of SOR then fixes the asymptotic
    # error reduction per iteration from the Jacobi spectral radius rho_J of
    # the matrix alone: for 1 <= omega <= omega_opt it is
    # ((omega rho_J + sqrt(omega^2 rho_J^2 - 4 (omega - 1))) / 2)^2, which is
    # rho_J^2 for Gauss-Seidel.  rho_J comes from an independent assembly; the
    # oracle's residual history must decay at exactly that rate.
    import scipy.sparse as sp
    n = 17
    st, al, Q, h = media.sphere_cloud(n) if case == "sphere" else media.point_source(n)
    prob = oracle_mod.setup(st, al, Q, h, limiter="cda")
    M = assemble((1.0 / 3.0) / prob.sig_hat, prob.sig_a, h, EPS * h)
    d = M.diagonal()
    s = sp.diags(1.0 / np.sqrt(d))
    rho_j = spl.eigsh(s @ (sp.diags(d) - M) @ s, k=1, which="LA",
                      return_eigenvectors=False)[0]
    assert 0.9 < rho_j < 1.0
    for omega in (1.0, 1.2, 1.4):
        r = oracle_mod.solve(prob, method="alg1", omega=omega, tol=1e-13, max_iters=20000,
                             check_every=1)
        assert r.status == "converged"
        hist = r.history
        a, b = len(hist) // 2, (9 * len(hist)) // 10
        observed = (hist[b] / hist[a]) ** (1.0 / (b - a))
        x = omega * rho_j
        predicted = ((x + np.sqrt(x * x - 4.0 * (omega - 1.0))) / 2.0) ** 2
        assert abs(observed / predicted - 1.0) < 1e-5, (omega, observed, predicted)


def test_alg1_converges_over_a_range_of_sor_factors(oracle_mod):
    # Sec. 5, Fig. 3a: on the spherical cloud in vacuum Algorithm 1 converges
    # for a broad range of SOR factors, and over-relaxation pays: omega = 1.4
    # needs fewer iterations than Gauss-Seidel.  (With the LP limiter omega
    # near 2 does diverge here; the sweep of the GPU benchmark records where.)
    st, al, Q, h = media.sphere_cloud(17)
    prob = oracle_mod.setup(st, al, Q, h, limiter="lp")
    its = {}
    for omega in (1.0, 1.2, 1.4, 1.6):
        r = oracle_mod.solve(prob, method="alg1", omega=omega, tol=1e-6, max_iters=20000,
                             check_every=1)
        assert r.status == "converged" and r.rel <= 1e-6, omega
        its[omega] = r.iterations
    assert its[1.4] < its[1.0]


def test_grid_sequencing_problem_and_fixed_point(oracle_mod):
    # Grid sequencing (our design): the 2:1 coarse medium averages 8 children.
    # It conserves the total emission and absorption (sum over cells times
    # cell volume), maps a homogeneous medium onto itself, and a solve started
    # from the prolongated coarse fluence lands on the plain solve's fixed point.
    st, al, Q, h = media.config("cloud128", n=32)
    prob = oracle_mod.setup(st, al, Q, h)
    c = oracle_mod.nested_problem(prob)
    assert c.shape == (16, 16, 16) and c.params.h == 2 * h
    for fine, coarse in ((prob.j, c.j), (prob.sig_a, c.sig_a)):
        assert abs(coarse.sum() * (2 * h) ** 3 - fine.sum() * h ** 3) <= 1e-12 * fine.sum() * h ** 3
    st1, al1, Q1, h1 = media.point_source(16, sigma_t=7.0, albedo=0.8)
    p1 = oracle_mod.nested_problem(oracle_mod.setup(st1, al1, np.full_like(Q1, 2.0), h1))
    np.testing.assert_allclose(p1.sig_hat, 7.0, rtol=1e-15)
    np.testing.assert_allclose(p1.sig_a, 0.2 * 7.0, rtol=1e-14)
    plain = oracle_mod.solve(prob, method="mg", tol=1e-10, max_iters=3000)
    nest = oracle_mod.solve(prob, method="mg", tol=1e-10, max_iters=3000, nested_tol=1e-3)
    assert nest.status == "converged" and nest.nested_iterations > 0
    assert np.linalg.norm(nest.phi - plain.phi) <= 1e-8 * np.linalg.norm(plain.phi)


def gmres_iterates(oracle_mod, D, sa, b, h, d_ghost, x0, k, **vk):
    """Left-preconditioned GMRES for M A x = M b (M: one V-cycle, A: the
    finest operator of frozen D), written here with numpy: the Arnoldi
    process on the operator v -> M A v and the small least-squares problem;
    returns the iterates x_0 .. x_k."""
    shape = b.shape

    def A(x):
        return -oracle_mod.level_residual(D, sa, np.zeros(shape), x, h, d_ghost)

    def M(r):
        return oracle_mod.linear_vcycle(D, sa, r, h, d_ghost, **vk)

    r0 = M(b - A(x0)).ravel()
    beta = np.linalg.norm(r0)
    V = [r0 / beta]
    H = np.zeros((k + 1, k))
    xs = [x0.copy()]
    for j in range(k):
        w = M(A(V[j].reshape(shape))).ravel()
        for i in range(j + 1):
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j])
        e1 = np.zeros(j + 2)
        e1[0] = beta
        y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
        xs.append(x0 + (np.stack(V[:j + 1], axis=1) @ y).reshape(shape))
    return xs


def test_anderson_on_a_linear_map_follows_gmres(oracle_mod):
    # Walker and Ni (SIAM J. Numer. Anal. 2011), Thm 2.2: without truncation,
    # Anderson acceleration of x -> g(x) = x + M(b - A x) yields
    # x^AA_{k+1} = g(x^GMRES_k), GMRES applied to M A x = M b from the same
    # start.  CDA makes D constant, so the outer iteration is that linear map
    # (no deflation, no restarts, no regularisation).
    st, al, Q, h = media.config("cloud128", n=16)
    prob = oracle_mod.setup(st, al, Q, h, limiter="cda")
    phi0, _ = prob.init_state()
    D = oracle_mod.limiter_pass(prob, phi0)
    vk = dict(deflate_tau=0.0)
    xs = gmres_iterates(oracle_mod, D, prob.sig_a, prob.j, h, EPS * h, phi0, 6)
    for k in range(1, 7):
        aa = oracle_mod.solve(prob, method="mg", tol=0.0, max_iters=k, aa_m=16, aa_reg=0.0,
                              restart_growth=0.0, **vk)
        x = xs[k - 1]
        g = x + oracle_mod.linear_vcycle(D, prob.sig_a, prob.j - (-oracle_mod.level_residual(
            D, prob.sig_a, np.zeros(x.shape), x, h, EPS * h)), h, EPS * h, **vk)
        assert np.linalg.norm(aa.phi - g) <= 1e-8 * np.linalg.norm(g), k


@pytest.mark.parametrize("case", ["point", "cloud"])
def test_anderson_reaches_the_brute_force_fixed_point(oracle_mod, case):
    if case == "point":
        st, al, Q, h = media.point_source(8, sigma_t=10.0, albedo=0.9)
    else:
        st, al, Q, h = media.config("cloud128", n=8)
    prob = oracle_mod.setup(st, al, Q, h, limiter="lp")
    ref = picard_direct(oracle_mod, prob, h)
    aa = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=2000, aa_m=4)
    assert aa.status == "converged"
    assert np.linalg.norm(aa.phi - ref) <= 1e-10 * np.linalg.norm(ref)


def test_coarse_level_sweeps_change_the_path_not_the_fixed_point(oracle_mod):
    # nu_coarse sweeps on the coarse levels (the 8^3 level of a 16^3 grid; the
    # 4^3 level is solved) change the V-cycle; the multigrid still lands on the
    # brute-force Picard fixed point
    st, al, Q, h = media.config("cloud128", n=16)
    prob = oracle_mod.setup(st, al, Q, h, limiter="lp")
    ref = picard_direct(oracle_mod, prob, h)
    base = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=2000)
    # nu_coarse equal to nu1 = nu2 is the same cycle, bit for bit
    same = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=2000, nu_coarse=2,
                            coarse_from=1)
    np.testing.assert_array_equal(same.phi, base.phi)
    for m in (1, 8):
        r = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=2000, nu_coarse=m,
                             coarse_from=1)
        assert r.status == "converged"
        assert np.linalg.norm(r.phi - ref) <= 1e-10 * np.linalg.norm(ref)
        assert r.iterations != base.iterations or not np.array_equal(r.history, base.history)
    # from level 2 on there is nothing to smooth on this grid: the default cycle
    r = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=2000, nu_coarse=8,
                         coarse_from=2)
    np.testing.assert_array_equal(r.phi, base.phi)


def test_inherited_grid_sequencing_keeps_the_fixed_point(oracle_mod):
    # the coarse solve of grid sequencing with the fine solve's schedule
    # (nested_inherit) takes another path to the same fixed point
    st, al, Q, h = media.config("cloud128", n=16)
    prob = oracle_mod.setup(st, al, Q, h, limiter="lp")
    kw = dict(nu1=3, nu2=3, omega_s=1.15, corr_scale=1.4, aa_m=4, nu_coarse=6, coarse_from=2)
    plain = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=2000, nested_tol=1e-3, **kw)
    inh = oracle_mod.solve(prob, method="mg", tol=1e-12, max_iters=2000, nested_tol=1e-3,
                           nested_inherit=True, **kw)
    assert plain.status == inh.status == "converged"
    assert inh.nested_iterations != plain.nested_iterations
    assert np.linalg.norm(inh.phi - plain.phi) <= 1e-10 * np.linalg.norm(plain.phi)


def test_anderson_and_conjugate_gradient_share_the_fixed_point(oracle_mod):
    # the 256^3 generator at 32^3 has vacuum clusters (deflation active) and
    # residual growth in the first iterations (restarts active)
    st, al, Q, h = media.config("cloud256", n=32)
    prob = oracle_mod.setup(st, al, Q, h)
    cg = oracle_mod.solve(prob, method="mg", tol=1e-10, max_iters=3000)
    for m in (1, 4):
        aa = oracle_mod.solve(prob, method="mg", tol=1e-10, max_iters=3000, aa_m=m)
        assert aa.status == cg.status == "converged"
        assert np.linalg.norm(aa.phi - cg.phi) <= 1e-8 * np.linalg.norm(cg.phi)
    assert aa.iterations < cg.iterations
