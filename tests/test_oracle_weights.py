"""Pins of the oracle's comparison weights (the paper's Sec. 5 comparison of
GENO with WENO-Z and TENO on the same three sub-stencils): special cases
with closed forms, invariants, the TENO cut-off threshold solved exactly, and
the paper's two extreme scenarios (smooth extremum, discontinuity)."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def prm(oracle):
    return oracle.params(ndim=1)


D = np.array([1.0, 8.0, 1.0]) / 10.0     # linear weights, normalised


def test_equal_indicators_give_the_linear_weights(oracle, prm):
    for s in (0.0, 1e-20, 1e-3, 1.0, 1e6):
        w = oracle.weights(prm, [s, s, s])
        assert np.allclose(w["wz"], D, rtol=0, atol=1e-15) and w["chi_z"] == pytest.approx(1.0, abs=1e-15)
        assert np.allclose(w["wt"], D, rtol=0, atol=1e-15) and w["chi_t"] == 1.0
        assert w["chi_geno"] == 1.0


def test_wenoz_equal_outer_indicators_and_scaling(oracle, prm):
    # tau_Z = |IS_1 - IS_3| = 0: the linear weights whatever IS_2 is
    w = oracle.weights(prm, [2.0, 50.0, 2.0])
    assert np.allclose(w["wz"], D, atol=1e-15)
    # scaling all indicators (eps negligible) leaves the weights unchanged
    a = oracle.weights(prm, [1.0, 3.0, 7.0])["wz"]
    b = oracle.weights(prm, [1e3, 3e3, 7e3])["wz"]
    assert np.allclose(a, b, rtol=1e-13) and a.sum() == pytest.approx(1.0, abs=1e-15)
    # a discontinuity in S_3 (IS_3 -> infinity) removes its weight; the others
    # approach d_k (1 + tau/IS_k) renormalised, here tau/IS_k -> infinity too,
    # so the two smooth stencils share in the ratio d_1 : d_2 / (IS_1 : IS_2)
    w = oracle.weights(prm, [1.0, 1.0, 1e12])["wz"]
    assert w[2] < 1e-11 and w[0] / w[1] == pytest.approx(D[0] / D[1], rel=1e-9)


def test_teno_cut_threshold(oracle, prm):
    # IS = (s, s, phi s): gamma_3 = phi^-7 / (2 + phi^-7) <= C_T exactly when
    # phi >= ((1 - C_T) / (2 C_T))^(1/7)
    ct = 1e-6
    phi = ((1.0 - ct) / (2.0 * ct)) ** (1.0 / 7.0)
    s = 1.0
    below = oracle.weights(prm, [s, s, phi * (1 - 1e-9) * s], ct=ct)
    above = oracle.weights(prm, [s, s, phi * (1 + 1e-9) * s], ct=ct)
    assert below["chi_t"] == 1.0 and np.allclose(below["wt"], D, atol=1e-15)
    assert above["chi_t"] == 0.0
    assert np.allclose(above["wt"], [D[0] / (D[0] + D[1]), D[1] / (D[0] + D[1]), 0.0], atol=1e-15)


def test_smooth_extremum_scenario(oracle, prm):
    # IS^max = phi IS^min with IS^tau = |(IS_2 + IS_3)/2 - IS_1| = 0 (the
    # paper's smooth-extremum case): GENO keeps the linear reconstruction
    # (chi = 1 exactly), TENO drops to the low-order one once phi is large,
    # WENO-Z deviates for every phi > 1
    for phi in (2.0, 10.0, 100.0, 1e4):
        IS = [0.5 * (1.0 + phi), 1.0, phi]
        w = oracle.weights(prm, IS)
        assert w["chi_geno"] == 1.0
        assert w["chi_z"] < 1.0
        if phi >= 10.0:
            assert w["chi_t"] == 0.0


def test_discontinuity_scenario(oracle, prm):
    # IS^tau ~ IS^max: all three leave the linear reconstruction as phi grows,
    # and keep it as phi -> 1 (resolved data)
    for phi, lin in ((1.0 + 1e-9, True), (1e6, False)):
        w = oracle.weights(prm, [1.0, phi, phi])
        if lin:
            assert w["chi_geno"] > 0.999 and w["chi_z"] > 0.999 and w["chi_t"] == 1.0
        else:
            assert w["chi_geno"] < 1e-3 and w["chi_z"] < 1e-3 and w["chi_t"] == 0.0


def test_path_function_hand_worked_value(oracle):
    # Eq. (5) with r = 2 and Eq. (4), C = 20, for the compact scheme's IS^tau
    # (Eq. (14)) from indicators worked by hand: IS = (IS_1, IS_2, IS_3) =
    # (1, 13, 11) gives IS^H = 13, IS^L = 1, IS^tau = |(13 + 11)/2 - 1| = 11;
    # alpha^H = 1 + (11/13)^2 = 290/169, alpha^L = 1 + 11^2 = 122 (eps
    # negligible), alpha = 2 alpha^H / (alpha^H + alpha^L) = 580/20908 =
    # 145/5227 = 0.0277405...; tanh(20) rounds to 1, so chi = tanh(2900/5227) =
    # (e^1.10962 - 1) / (e^1.10962 + 1) = 2.03321 / 4.03321 = 0.504118...
    w = oracle.weights(oracle.params(), np.array([1.0, 13.0, 11.0]))
    assert abs(w["chi_geno"] - 0.5041176819) < 2e-10, w["chi_geno"]
    assert abs(w["chi_geno"] - math.tanh(20.0 * 145.0 / 5227.0) / math.tanh(20.0)) < 1e-14
