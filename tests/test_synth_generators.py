"""Pins of the seeded input generators.

The U(1) heat-bath is checked against the exact infinite-volume plaquette of
two-dimensional U(1) lattice gauge theory, <cos theta_P> = I_1(beta)/I_0(beta),
and against the string-tension lengths the paper prints for its beta = 6 and
beta = 10 ensembles: the area law of 2d U(1) gives
l_sigma = [-ln(I_1/I_0)]^(-1/2) per plaquette (golden values, numerical-test
section).
"""
import json
import os

import numpy as np
import pytest
from scipy.special import iv

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _measure(beta, L=32, therm=60, meas=120, seed=0):
    rng = synth.rng_for(97, int(100 * beta), L, L, seed)
    th = synth.u1_heatbath(L, L, beta, therm, rng)
    vals = []
    for _ in range(meas):
        th = synth.u1_heatbath(L, L, beta, 1, rng, theta=th)
        vals.append(synth.u1_mean_plaquette(th))
    return np.mean(vals), np.std(vals) / np.sqrt(meas), th


@pytest.mark.parametrize("beta", [3.0, 6.0, 10.0])
def test_heatbath_plaquette_matches_bessel_ratio(beta):
    mean, err, th = _measure(beta)
    exact = iv(1, beta) / iv(0, beta)
    assert abs(mean - exact) < max(6 * err, 1.5e-3), (mean, exact, err)
    q = synth.u1_topological_charge(th)
    assert abs(q - round(q)) < 1e-10


def test_string_tension_lengths_match_paper():
    with open(GOLDEN) as f:
        gold = json.load(f)["string_tension_length"]
    for beta, l_paper in zip(gold["beta"], gold["l_sigma"]):
        mean, err, _ = _measure(beta, meas=150, seed=1)
        l_meas = (-np.log(mean)) ** -0.5
        # closed form (exact) agrees with the printed value to its 3 digits
        l_exact = (-np.log(iv(1, beta) / iv(0, beta))) ** -0.5
        assert round(l_exact, 2) == pytest.approx(l_paper, abs=1e-9)
        assert abs(l_meas - l_paper) < 0.05, (beta, l_meas, l_paper)


def test_cold_start_and_charge_is_integer():
    th = synth.u1_cold(8, 6)
    assert synth.u1_mean_plaquette(th) == 1.0
    rng = synth.rng_for(3)
    th = synth.u1_heatbath(16, 16, 1.0, 30, rng)
    q = synth.u1_topological_charge(th)
    assert abs(q - round(q)) < 1e-10


def test_heatbath_is_seed_deterministic():
    a = synth.u1_heatbath(8, 8, 6.0, 5, synth.rng_for(1, 600, 8, 8, 0))
    b = synth.u1_heatbath(8, 8, 6.0, 5, synth.rng_for(1, 600, 8, 8, 0))
    assert np.array_equal(a, b)


def test_tiling_keeps_plaquettes():
    th = synth.u1_heatbath(8, 8, 6.0, 10, synth.rng_for(4))
    t = synth.tile_u1(th, 2, 3)
    assert t.shape == (2, 24, 16)
    p0 = np.cos(synth.u1_plaquette_angles(th))
    p1 = np.cos(synth.u1_plaquette_angles(t))
    assert np.allclose(np.tile(p0, (3, 2)), p1)


def test_su3_haar_and_stout():
    U = synth.su3_haar((4, 2, 2, 2, 2), synth.rng_for(5))
    eye = np.eye(3)
    assert np.allclose(U @ np.conj(np.swapaxes(U, -1, -2)), eye, atol=1e-13)
    assert np.allclose(np.linalg.det(U), 1.0, atol=1e-13)
    p0 = synth.su3_mean_plaquette(U)
    Us = synth.su3_stout_smear(U, 0.1, 3)
    assert np.allclose(Us @ np.conj(np.swapaxes(Us, -1, -2)), eye, atol=1e-12)
    assert np.allclose(np.linalg.det(Us), 1.0, atol=1e-12)
    p1 = synth.su3_mean_plaquette(Us)
    assert p1 > p0 + 0.1
    # Haar: <(1/3) Re tr U_P> = 0 in expectation (small sample, loose bound)
    assert abs(p0) < 0.1


@pytest.mark.parametrize("Q", [0, 1, 4, -3])
def test_flux_background_has_charge_q_and_uniform_flux(Q):
    """The constant-flux start: every plaquette angle is 2 pi Q / V and the
    charge is exactly Q; a short heat-bath at beta = 10 from it keeps Q."""
    L1, L2 = 16, 12
    th = synth.u1_flux(L1, L2, Q)
    a = np.angle(np.exp(1j * synth.u1_plaquette_angles(th)))
    assert np.abs(a - 2 * np.pi * Q / (L1 * L2)).max() < 1e-12
    assert synth.u1_topological_charge(th) == pytest.approx(Q, abs=1e-9)
    th2 = synth.u1_heatbath(L1, L2, 10.0, 5, synth.rng_for(9, Q + 10), th)
    assert round(synth.u1_topological_charge(th2)) == Q
