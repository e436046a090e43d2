"""Pins of the oracle's discrete operator (Sec. 5: gradient, guarded Knudsen
number, D update, discretised FLD equation and its residual) and of the
multigrid coarse operator.

References other than the oracle itself: exactness of central differences on
linear fields, the guard branches worked out by hand, the flux-limiting
bound |E| <= phi (Sec. 4), symmetry of the discrete operator, the exact
discrete power balance obtained by summing the discretised equation
(first line of the moment equations, Sec. 3: energy conservation), an
independent scipy assembly of the same linear system, and the Galerkin
identity A_1 = P^T A_0 P / 8 computed with plain numpy.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from synth import media

EPS = 1e-20


def ghost_fill(phi, fn):
    """Padded array with phi inside and fn(i,j,k) (0-based unknown indices) in the ghost layer."""
    nx, ny, nz = phi.shape
    g = np.zeros((nx + 2, ny + 2, nz + 2))
    I, J, K = np.meshgrid(np.arange(-1, nx + 1), np.arange(-1, ny + 1), np.arange(-1, nz + 1),
                          indexing="ij")
    g[...] = fn(I, J, K)
    g[1:-1, 1:-1, 1:-1] = phi
    return g


def test_knudsen_exact_on_linear_field(oracle_mod):
    n, h = 9, 0.1
    a, b = np.array([0.3, -0.2, 0.5]), 2.0
    lin = lambda I, J, K: b + h * (a[0] * I + a[1] * J + a[2] * K)
    I, J, K = np.indices((n, n, n))
    phi = lin(I, J, K)
    st = np.full((n, n, n), 4.0)
    st[2, 3, 4] = 0.5
    Q = np.ones((n, n, n))
    prob = oracle_mod.setup(st, np.zeros_like(st), Q, h, ghost_phi=ghost_fill(phi, lin))
    R = oracle_mod.knudsen(prob, phi)
    expect = np.linalg.norm(a) / (prob.sig_hat * phi)
    np.testing.assert_allclose(R, expect, rtol=1e-13)


def test_knudsen_guard_branches(oracle_mod):
    n, h = 5, 0.2
    st = np.full((n, n, n), 2.0)
    Q = np.zeros((n, n, n))
    Q[2, 2, 2] = 1.0
    prob = oracle_mod.setup(st, np.zeros_like(st), Q, h)
    jbar = prob.jbar
    assert jbar == pytest.approx(np.sqrt(1.0 / n ** 3), rel=1e-15)
    floor = EPS * jbar
    # zero fluence everywhere (ghost 0): both guards active -> R = 1
    R = oracle_mod.knudsen(prob, np.zeros((n, n, n)))
    np.testing.assert_array_equal(R, np.ones((n, n, n)))
    # constant fluence inside, zero ghosts: interior gradient 0 -> numerator floored
    c = 3.0
    R = oracle_mod.knudsen(prob, np.full((n, n, n), c))
    assert R[2, 2, 2] == pytest.approx(floor / (2.0 * c), rel=1e-15)


def test_knudsen_guards_worked(oracle_mod):
    # Worked by hand: 1-voxel-thin features so that each guard branch is hit.
    n, h = 5, 0.5
    st = np.full((n, n, n), 2.0)
    Q = np.zeros((n, n, n))
    Q[0, 0, 0] = 5.0
    prob = oracle_mod.setup(st, np.zeros_like(st), Q, h)
    floor = EPS * prob.jbar
    phi = np.full((n, n, n), 1.0)
    phi[2, 2, 2] = 1e-40                   # sigma*phi < floor, gradient 0 (neighbours equal)
    R = oracle_mod.knudsen(prob, phi)
    assert R[2, 2, 2] == floor / floor     # both guards -> 1
    phi[2, 2, 3] = 3.0                     # now gradient along z at (2,2,2) = (3-1)/(2h)
    R = oracle_mod.knudsen(prob, phi)
    assert R[2, 2, 2] == pytest.approx((2.0 / (2 * h)) / floor, rel=1e-15)


def test_limiter_pass_respects_flux_bound(oracle_mod):
    # After a limiter pass, |E| = D |grad phi| <= phi wherever the guards are
    # inactive (R F(R) <= 1 for every limiter of Table 2).
    rng = np.random.default_rng(5)
    n, h = 12, 1.0 / 12
    st = rng.uniform(0.0, 50.0, (n, n, n))
    phi = rng.uniform(0.01, 1.0, (n, n, n))
    I = np.indices((n, n, n))
    for kind in ["lp", "sum", "max", "kershaw", "larsen"]:
        prob = oracle_mod.setup(st, np.full_like(st, 0.5), np.ones_like(st), h, limiter=kind)
        D = oracle_mod.limiter_pass(prob, phi)
        p = np.pad(phi, 1)
        g = np.stack([(p[2:, 1:-1, 1:-1] - p[:-2, 1:-1, 1:-1]),
                      (p[1:-1, 2:, 1:-1] - p[1:-1, :-2, 1:-1]),
                      (p[1:-1, 1:-1, 2:] - p[1:-1, 1:-1, :-2])]) / (2 * h)
        E = D * np.linalg.norm(g, axis=0)
        assert np.all(E <= phi * (1 + 1e-14)), kind
        # CDA-sized coefficients where the medium is optically thick and smooth
        assert np.all(D <= 1.0 / (3.0 * prob.sig_hat) * (1 + 1e-15))


def assemble(D, sa, h, d_ghost, mirror=False):
    """Sparse h^2-scaled operator M = h^2 A of the discretised equation, written with numpy."""
    shape = D.shape
    N = D.size
    idx = np.arange(N).reshape(shape)
    diag = sa.ravel() * h * h
    rows, cols, vals = [], [], []
    for ax in range(3):
        for sgn in (-1, 1):
            Ds = D.copy() if mirror else np.full(shape, d_ghost)
            nb = np.full(shape, -1)
            dst = [slice(None)] * 3
            src = [slice(None)] * 3
            dst[ax], src[ax] = (slice(0, -1), slice(1, None)) if sgn == 1 else (slice(1, None), slice(0, -1))
            Ds[tuple(dst)] = D[tuple(src)]
            nb[tuple(dst)] = idx[tuple(src)]
            F = 0.5 * (D + Ds)
            diag = diag + F.ravel()
            m = nb.ravel() >= 0
            rows.append(idx.ravel()[m]); cols.append(nb.ravel()[m]); vals.append(-F.ravel()[m])
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def test_residual_matches_independent_assembly(oracle_mod):
    rng = np.random.default_rng(7)
    n, h = 8, 1.0 / 8
    D = rng.uniform(0.01, 2.0, (n, n, n))
    sa = rng.uniform(0.0, 3.0, (n, n, n))
    b = rng.standard_normal((n, n, n))
    e = rng.standard_normal((n, n, n))
    for mirror in (False, True):
        r = oracle_mod.level_residual(D, sa, b, e, h, EPS * h, mirror)
        M = assemble(D, sa, h, EPS * h, mirror)
        expect = b.ravel() - (M @ e.ravel()) / (h * h)
        np.testing.assert_allclose(r.ravel(), expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


def test_operator_symmetric_and_m_matrix(oracle_mod):
    rng = np.random.default_rng(8)
    n, h = 7, 0.1
    D = rng.uniform(0.001, 5.0, (n, n, n))
    sa = rng.uniform(0.0, 1.0, (n, n, n))
    A = lambda x: -oracle_mod.level_residual(D, sa, np.zeros_like(x), x, h, EPS * h)
    x, y = rng.standard_normal((2, n, n, n))
    assert abs((x * A(y)).sum() - (y * A(x)).sum()) < 1e-11 * abs((x * A(y)).sum())
    # M-matrix: A x >= 0 with x >= 0 impossible to be negative on the diagonal; check
    # that the inverse of the assembled matrix is entrywise non-negative (small case).
    M = assemble(D[:4, :4, :4], sa[:4, :4, :4], h, EPS * h).toarray()
    assert np.all(np.linalg.inv(M) >= -1e-14)


def test_discrete_power_balance(oracle_mod):
    # Summing the discretised equation over all unknowns, interior face fluxes
    # cancel pairwise: sum r = sum j - sum sigma_a phi - boundary leakage.
    rng = np.random.default_rng(9)
    n, h = 10, 0.07
    st = rng.uniform(0.0, 20.0, (n, n, n))
    al = rng.uniform(0.0, 1.0, (n, n, n))
    Q = rng.uniform(0.0, 3.0, (n, n, n))
    phi_b = 0.25
    prob = oracle_mod.setup(st, al, Q, h, phi_b=phi_b)
    phi = rng.uniform(0.0, 2.0, (n, n, n))
    D = oracle_mod.limiter_pass(prob, phi)
    r, _ = oracle_mod.residual(prob, phi, D)
    leak = 0.0
    for ax in range(3):
        for end in (0, -1):
            sl = [slice(None)] * 3
            sl[ax] = end
            Fb = 0.5 * (D[tuple(sl)] + EPS * h)
            leak += (Fb * (phi[tuple(sl)] - phi_b)).sum() / h ** 2
    lhs = r.sum()
    rhs = Q.sum() - (prob.sig_a * phi).sum() - leak
    scale = Q.sum() + (prob.sig_a * phi).sum() + abs(leak)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_galerkin_coarse_operator(oracle_mod):
    # A_1 x = (1/8) P^T A_0 (P x), P = copy each coarse value to its 8 children.
    rng = np.random.default_rng(10)
    n, h = 8, 1.0 / 8
    D = rng.uniform(0.001, 300.0, (n, n, n))
    sa = rng.uniform(0.0, 2.0, (n, n, n))
    x1 = rng.standard_normal((n // 2,) * 3)
    for mirror in (False, True):
        Px = np.repeat(np.repeat(np.repeat(x1, 2, 0), 2, 1), 2, 2)
        A0Px = -oracle_mod.level_residual(D, sa, np.zeros_like(Px), Px, h, EPS * h, mirror)
        expect = A0Px.reshape(n // 2, 2, n // 2, 2, n // 2, 2).mean(axis=(1, 3, 5))
        got = oracle_mod.coarse_apply(D, sa, x1, h, EPS * h, mirror)
        np.testing.assert_allclose(got, expect, rtol=1e-11, atol=1e-11 * np.abs(expect).max())


def test_homogeneity_bit_exact(oracle_mod):
    # R and F are scale-free and the init/guards scale with j-bar, so scaling
    # Q by 2^k scales every iterate by 2^k exactly.
    st, al, Q, h = media.config("cloud128", n=16)
    base = oracle_mod.setup(st, al, Q, h)
    scaled = oracle_mod.setup(st, al, Q * 8.0, h)
    for method, kw in (("alg1", dict(max_iters=7, check_every=100)), ("mg", dict(max_iters=4))):
        a = oracle_mod.solve(base, method=method, tol=0.0, **kw)
        b = oracle_mod.solve(scaled, method=method, tol=0.0, **kw)
        np.testing.assert_array_equal(b.phi, 8.0 * a.phi)


def test_axis_permutation_symmetry(oracle_mod):
    # Point source on the diagonal of a cubic grid: the problem and the
    # red-black colouring are invariant under axis permutations.
    st, al, Q, h = media.point_source(12)
    prob = oracle_mod.setup(st, al, Q, h)
    for method in ("alg1", "mg"):
        phi = oracle_mod.solve(prob, method=method, tol=0.0, max_iters=6).phi
        for perm in ((1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)):
            np.testing.assert_allclose(phi.transpose(perm), phi, rtol=1e-13, atol=0)
