"""Pins of the oracle's flux limiters (Sec. 4, Table 2; CDA F = 1/3).

Independent reference: the closed forms of Table 2 evaluated by mpmath at
50 significant digits.  Also the limits F -> 1/3 (R -> 0) and R F -> 1
(R -> inf) and the flux-limiting bound F <= 1/R that the paper requires of
every limiter (Sec. 4, equations F_limits and F_constraint).
"""
import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 50

R_VALUES = np.concatenate([np.array([0.0, 1e-12, 1e-8, 1e-4, 1e-3, 0.01, 0.05, 0.09, 0.0999999,
                                     0.1, 0.1000001, 0.11, 0.2, 0.5, 1.0, 2.0, 3.0, 3.0000001,
                                     5.0, 10.0, 30.0, 100.0, 1e3, 1e5, 1e8, 1e12, 1e20]),
                           np.logspace(-6, 6, 97)])


def exact(kind, R, n=2.0):
    R = mp.mpf(R)
    if kind == "cda":
        return mp.mpf(1) / 3
    if kind == "lp":
        if R == 0:
            return mp.mpf(1) / 3
        return (mp.coth(R) - 1 / R) / R
    if kind == "sum":
        return 1 / (3 + R)
    if kind == "max":
        return 1 / mp.mpf(max(3, R))
    if kind == "kershaw":
        return 2 / (3 + mp.sqrt(9 + 4 * R * R))
    if kind == "larsen":
        n = mp.mpf(n)
        return (mp.mpf(3) ** n + R ** n) ** (-1 / n)
    raise KeyError(kind)


@pytest.mark.parametrize("kind,tol", [("cda", 1e-16), ("lp", 6e-16), ("sum", 2e-16),
                                      ("max", 2e-16), ("kershaw", 4e-16)])
def test_limiter_matches_closed_form(oracle_mod, kind, tol):
    F = oracle_mod.limiter(kind, R_VALUES)
    for R, f in zip(R_VALUES, F):
        ref = exact(kind, R)
        assert abs(f - float(ref)) <= tol * float(ref), (kind, R, f, ref)


@pytest.mark.parametrize("n", [1.0, 2.0, 3.0, 4.5])
def test_larsen_matches_closed_form(oracle_mod, n):
    F = oracle_mod.limiter("larsen", R_VALUES, n)
    for R, f in zip(R_VALUES, F):
        ref = exact("larsen", R, n)
        assert abs(f - float(ref)) <= 2e-15 * float(ref), (n, R, f, ref)


def test_lp_small_r_branch_is_accurate(oracle_mod):
    # The continued-fraction branch (R < 2) must agree with the closed form
    # to rounding over its whole range, including next to the switch.
    R = np.concatenate([np.linspace(0.0, 1.9999999, 301), [2.0, 2.0000001, 2.5]])
    F = oracle_mod.limiter("lp", R)
    err = max(abs(f - float(exact("lp", r))) / float(exact("lp", r)) for r, f in zip(R, F))
    assert err < 5e-16


@pytest.mark.parametrize("kind", ["lp", "sum", "max", "kershaw", "larsen"])
def test_limiter_limits_and_bound(oracle_mod, kind):
    F0 = oracle_mod.limiter(kind, [0.0])[0]
    assert abs(F0 - 1.0 / 3.0) < 1e-15
    big = np.array([1e6, 1e9, 1e12])
    RF = big * oracle_mod.limiter(kind, big)
    assert np.all(np.abs(RF - 1.0) < 1e-5)
    F = oracle_mod.limiter(kind, R_VALUES)
    assert np.all(F <= 1.0 / 3.0 + 1e-16)
    pos = R_VALUES > 0
    assert np.all(F[pos] * R_VALUES[pos] <= 1.0 + 1e-15)     # |E| <= phi
    srt = np.sort(R_VALUES)
    Fs = oracle_mod.limiter(kind, srt)
    assert np.all(np.diff(Fs) <= 1e-16)                       # non-increasing


def test_cda_is_constant(oracle_mod):
    assert np.all(oracle_mod.limiter("cda", R_VALUES) == 1.0 / 3.0)
