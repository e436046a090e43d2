"""Pins of the oracle's set-up step (Algorithm 1 set-up; Sec. 5, extinction
tolerance; Sec. 7, reduced extinction) against values worked out by hand.

The paper clamps the extinction to sigma_eps, the inverse of a mean free path
of 1000 box lengths, so sigma_eps = 1e-3 / L with L the box extent; the
clamped value replaces sigma everywhere Algorithm 1 uses it, the absorption
(1 - albedo) sigma included.  The grid below is deliberately non-cubic with a
voxel edge that is not 1/n, so a box extent taken in voxels (10 instead of
0.5), along the wrong axis (h * min n = 0.1) or from the voxel size alone
would give a different floor; voxels of zero, sub-floor and ordinary
extinction hit both branches of the clamp.  Expected values are literals
computed by hand from those numbers.
"""
import numpy as np
import pytest

SHAPE = (4, 10, 2)          # L = h * max(n) = 0.05 * 10 = 0.5  ->  sigma_eps = 2e-3
H = 0.05


def medium():
    st = np.full(SHAPE, 7.0)
    al = np.full(SHAPE, 0.5)
    Q = np.zeros(SHAPE)
    cases = {
        # voxel: (sigma_t, albedo)
        (0, 0, 0): (0.0, 0.25),      # vacuum
        (1, 9, 1): (0.001, 0.5),     # below the floor
        (2, 3, 0): (3.0, 0.9),       # ordinary
        (3, 5, 1): (0.003, 0.8),     # above the floor, below it once reduced by g = 0.5
        (0, 7, 1): (0.0021, 1.0),    # just above the floor, pure scatterer
    }
    for v, (s, a) in cases.items():
        st[v], al[v] = s, a
    Q[1, 2, 0], Q[3, 9, 1] = 3.0, 4.0
    return st, al, Q


def test_extinction_floor_and_absorption(oracle_mod):
    st, al, Q = medium()
    prob = oracle_mod.setup(st, al, Q, H)
    assert prob.sigma_eps == pytest.approx(2e-3, rel=1e-15)
    expect = {
        (0, 0, 0): (2e-3, 1.5e-3),
        (1, 9, 1): (2e-3, 1e-3),
        (2, 3, 0): (3.0, 0.3),
        (3, 5, 1): (3e-3, 6e-4),
        (0, 7, 1): (2.1e-3, 0.0),
        (1, 1, 1): (7.0, 3.5),       # the background voxel
    }
    for v, (sh, sa) in expect.items():
        assert prob.sig_hat[v] == pytest.approx(sh, rel=1e-15), v
        assert prob.sig_a[v] == pytest.approx(sa, rel=1e-15, abs=0.0), v
    # the floor never lowers a value and is reached exactly where it binds
    assert np.all(prob.sig_hat >= 2e-3) and np.all(prob.sig_hat >= st)
    # RMS emission over all 80 voxels and the 2-norm: sqrt(9 + 16) = 5
    assert prob.jnorm == pytest.approx(5.0, rel=1e-15)
    assert prob.jbar == pytest.approx(5.0 / np.sqrt(80.0), rel=1e-15)


def test_reduced_extinction_keeps_absorption(oracle_mod):
    # with anisotropy g the diffusion coefficient and the Knudsen number use
    # sigma_t (1 - albedo g), floored; the absorption stays (1 - albedo)
    # max(sigma_t, sigma_eps)
    st, al, Q = medium()
    prob = oracle_mod.setup(st, al, Q, H, aniso_g=0.5)
    expect = {
        (0, 0, 0): (2e-3, 1.5e-3),
        (1, 9, 1): (2e-3, 1e-3),
        (2, 3, 0): (1.65, 0.3),      # 3 * (1 - 0.45)
        (3, 5, 1): (2e-3, 6e-4),     # 0.003 * 0.6 = 0.0018 < floor; absorption from 0.003
        (0, 7, 1): (2e-3, 0.0),      # 0.0021 * 0.5 below the floor
        (1, 1, 1): (5.25, 3.5),      # 7 * 0.75
    }
    for v, (sh, sa) in expect.items():
        assert prob.sig_hat[v] == pytest.approx(sh, rel=1e-15), v
        assert prob.sig_a[v] == pytest.approx(sa, rel=1e-15, abs=0.0), v


def test_explicit_floor_overrides_the_box_rule(oracle_mod):
    st, al, Q = medium()
    prob = oracle_mod.setup(st, al, Q, H, sigma_eps=0.01)
    assert prob.sigma_eps == 0.01
    assert prob.sig_hat[0, 0, 0] == 0.01 and prob.sig_hat[3, 5, 1] == 0.01
    assert prob.sig_a[0, 0, 0] == pytest.approx(0.0075, rel=1e-15)
    assert prob.sig_hat[2, 3, 0] == 3.0


def test_floor_scales_with_the_longest_axis(oracle_mod):
    # the same medium transposed so the long axis is x, and a cubic 10^3 box
    # of the same extent: the floor follows L only
    st, al, Q = medium()
    t = oracle_mod.setup(np.ascontiguousarray(st.transpose(1, 0, 2)),
                         np.ascontiguousarray(al.transpose(1, 0, 2)),
                         np.ascontiguousarray(Q.transpose(1, 0, 2)), H)
    assert t.sigma_eps == pytest.approx(2e-3, rel=1e-15)
    c = oracle_mod.setup(np.zeros((10, 10, 10)), np.zeros((10, 10, 10)), np.ones((10, 10, 10)), H)
    assert c.sigma_eps == pytest.approx(2e-3, rel=1e-15)
    d = oracle_mod.setup(np.zeros((4, 4, 4)), np.zeros((4, 4, 4)), np.ones((4, 4, 4)), 0.25)
    assert d.sigma_eps == pytest.approx(1e-3, rel=1e-15)     # unit box
