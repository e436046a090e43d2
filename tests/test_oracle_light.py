"""Pins of the oracle's light baking (Sec. 3 single-scatter source of a
directional light, q = L sigma_s T, T towards the light; reading A17: light
along +z from the z = 0 face, midpoint transmittance of each voxel)."""
import numpy as np
import pytest


def test_homogeneous_column_closed_form(oracle_mod):
    # constant sigma: T_k = exp(-sigma h (k + 1/2)) exactly
    n, h, sig, alb, L = 40, 1.0 / 40, 7.5, 0.8, 2.5
    st = np.full((3, 2, n), sig)
    q = oracle_mod.light_bake(st, alb, h, light=L)
    k = np.arange(n)
    want = L * alb * sig * np.exp(-sig * h * (k + 0.5))
    for i in range(3):
        for j in range(2):
            np.testing.assert_allclose(q[i, j], want, rtol=1e-13)


def test_product_form_of_transmittance(oracle_mod):
    # T is the product of the attenuation of every voxel the light crossed and
    # of half the voxel itself: an independent evaluation of the same quantity
    rng = np.random.default_rng(4)
    shape, h = (4, 3, 29), 0.05
    st = rng.uniform(0.0, 30.0, shape) * (rng.random(shape) > 0.3)
    al = rng.uniform(0.5, 1.0, shape)
    q = oracle_mod.light_bake(st, al, h)
    T = np.ones(shape)
    for k in range(shape[2]):
        T[:, :, k] = np.prod(np.exp(-h * st[:, :, :k]), axis=2) * np.exp(-0.5 * h * st[:, :, k])
    np.testing.assert_allclose(q, al * st * T, rtol=1e-12, atol=0.0)


def test_vacuum_and_linearity(oracle_mod):
    rng = np.random.default_rng(5)
    st = rng.uniform(0.0, 10.0, (5, 5, 16))
    st[:, :, :4] = 0.0                        # a vacuum layer casts no shadow and emits nothing
    q1 = oracle_mod.light_bake(st, 0.9, 0.1, light=1.0)
    q3 = oracle_mod.light_bake(st, 0.45, 0.1, light=6.0)
    assert np.all(q1[:, :, :4] == 0.0)
    np.testing.assert_allclose(q3, 3.0 * q1, rtol=1e-15)
    # the first voxel past the vacuum sees the full light
    s = st[:, :, 4]
    np.testing.assert_allclose(q1[:, :, 4], 0.9 * s * np.exp(-0.05 * s), rtol=1e-14)


def test_uses_extinction_not_scattering_for_the_shadow(oracle_mod):
    # albedo scales the emitted source, never the attenuation
    st = np.full((1, 1, 8), 4.0)
    qa = oracle_mod.light_bake(st, 1.0, 0.25)
    qb = oracle_mod.light_bake(st, 0.25, 0.25)
    np.testing.assert_allclose(qb, 0.25 * qa, rtol=1e-15)


def test_render_homogeneous_column_closed_form(oracle_mod):
    # constant sigma, albedo, src and phi: the sum is a geometric series
    n, h, sig, alb, src, phi, bg = 24, 0.125, 3.0, 0.7, 2.0, 5.0, 0.6
    shape = (2, 3, n)
    img = oracle_mod.render(np.full(shape, sig), alb, np.full(shape, src), np.full(shape, phi), h,
                            background=bg)
    Q = (src + alb * sig * phi) / (4.0 * np.pi)
    a = np.exp(-sig * h)
    series = np.exp(-0.5 * sig * h) * (1.0 - a ** n) / (1.0 - a)     # sum_k exp(-sig h (k + 1/2))
    want = bg * a ** n + h * Q * series
    np.testing.assert_allclose(img, want, rtol=1e-13)


def test_render_vacuum_and_order(oracle_mod):
    rng = np.random.default_rng(8)
    shape, h = (3, 2, 10), 0.1
    st = np.zeros(shape)
    src = rng.uniform(0.0, 1.0, shape)
    phi = rng.uniform(0.0, 1.0, shape)
    # vacuum: nothing attenuates and nothing scatters; the image is bg + h sum src / 4 pi
    img = oracle_mod.render(st, 0.9, src, phi, h, background=0.25)
    np.testing.assert_allclose(img, 0.25 + h * src.sum(axis=2) / (4 * np.pi), rtol=1e-14)
    # an absorbing voxel in front of (z above) a source hides it; behind it, it does not
    st = np.zeros((1, 1, 6))
    src = np.zeros((1, 1, 6))
    src[0, 0, 1] = 1.0
    front = st.copy()
    front[0, 0, 4] = 50.0
    behind = st.copy()
    behind[0, 0, 0] = 50.0
    z = np.zeros_like(st)
    i_front = oracle_mod.render(front, 0.0, src, z, 1.0)
    i_behind = oracle_mod.render(behind, 0.0, src, z, 1.0)
    assert i_front[0, 0] < 1e-20 and i_behind[0, 0] == pytest.approx(1.0 / (4 * np.pi), rel=1e-15)
