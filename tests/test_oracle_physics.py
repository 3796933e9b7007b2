"""Pins of the oracle's closed-form interaction models.

The paper keeps DPM's physics without printing it (section 2.1); the models are
this project's closed forms for synthetic pseudo-element materials.  Each is
pinned against something other than itself: textbook limits, a differential
cross section integrated numerically against its closed-form total, energy-loss
identities linking two formulas, and published data where the model should be
close (ballpark tolerances, marked as such)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from paper_1107_3355_amd.inputs import AIR, BONE, LUNG, MATERIALS, WATER, Material

MC2 = 0.51099895
RE = 2.8179403262e-13
NA = 6.02214076e23
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "reference_values.json")))


def test_thomson_limit():
    st = GOLD["thomson_cross_section_cm2"]["value"]
    for k in (1e-3, 3e-3):
        s = oracle.phys(oracle.SIGMA_KN, WATER, k * MC2)
        # low-energy expansion sigma_KN = sigma_T (1 - 2k + 26k^2/5 - 133k^3/10 + O(k^4))
        assert abs(s / st - (1 - 2 * k + 5.2 * k * k - 13.3 * k ** 3)) < 50 * k ** 4 + 1e-8  # 1e-8: cancellation in the closed form at small k


def test_kn_high_energy_asymptote():
    k = 1e5
    s = oracle.phys(oracle.SIGMA_KN, WATER, k * MC2)
    asym = math.pi * RE ** 2 / k * (math.log(2 * k) + 0.5)
    assert abs(s / asym - 1) < 1e-3


@pytest.mark.parametrize("e", [0.06, 0.3, 1.0, 2.0, 6.0, 20.0])
def test_kn_total_is_integral_of_differential(e):
    k = e / MC2
    e0 = 1 / (1 + 2 * k)
    # integrate in ln(eps): the 1/eps part peaks at the lower end
    tot = quad(lambda y: math.exp(y) * oracle.phys(oracle.DSIGMA_KN, WATER, e, math.exp(y)),
               math.log(e0), 0.0, epsrel=1e-13, limit=200)[0]
    assert abs(tot / oracle.phys(oracle.SIGMA_KN, WATER, e) - 1) < 1e-9
    mu = oracle.phys(oracle.MU_COMPTON, WATER, e)
    assert abs(mu / (NA * WATER.z_over_a * tot) - 1) < 1e-9


def test_photoelectric_and_pair_shapes():
    for m in MATERIALS:
        a = oracle.phys(oracle.MU_PHOTO, m, 0.1)
        b = oracle.phys(oracle.MU_PHOTO, m, 0.2)
        assert abs(a / b - 8.0) < 1e-12
        assert oracle.phys(oracle.MU_PAIR, m, 2 * MC2) == 0.0
        assert oracle.phys(oracle.MU_PAIR, m, 1.0) == 0.0
        x0 = oracle.phys(oracle.X0, m, 1.0)
        hi = oracle.phys(oracle.MU_PAIR, m, 1e6)
        assert abs(hi / (0.35 * 7 / 9 / x0) - 1) < 1e-5
    assert oracle.phys(oracle.MU_PHOTO, BONE, 0.1) / oracle.phys(oracle.MU_PHOTO, WATER, 0.1) == \
        pytest.approx((13.0 / 7.42) ** 3 * (0.5148 / 0.55508), rel=1e-12)


def test_radiation_length_against_pdg():
    g = GOLD["radiation_length_g_cm2"]
    for name, v in g["elements"].items():
        m = Material(name, v["z"], v["z"] / v["a"], 80.0, 1.0)
        x0 = oracle.phys(oracle.X0, m, 1.0)
        assert abs(x0 / v["x0"] - 1) < g["tolerance"], name


def _rohrlich_carlson(m, t):
    """Unrestricted electron collision stopping power (no density effect)."""
    tau = t / MC2
    g = tau + 1
    b2 = 1 - 1 / g ** 2
    im = m.i_ev * 1e-6 / MC2
    f = 1 - b2 + (tau ** 2 / 8 - (2 * tau + 1) * math.log(2)) / (tau + 1) ** 2
    return 2 * math.pi * RE ** 2 * MC2 * NA * m.z_over_a / b2 * (
        math.log(tau ** 2 * (tau + 2) / (2 * im ** 2)) + f)


@pytest.mark.parametrize("m", MATERIALS, ids=lambda m: m.name)
@pytest.mark.parametrize("t", [0.25, 0.5, 1.0, 5.0, 20.0])
def test_restricted_loss_reduces_to_unrestricted(m, t):
    full = oracle.phys(oracle.L_RESTRICTED, m, t, 1e9)
    assert abs(full / _rohrlich_carlson(m, t) - 1) < 1e-12


@pytest.mark.parametrize("m", [WATER, BONE], ids=lambda m: m.name)
@pytest.mark.parametrize("t", [0.5, 1.0, 5.0, 20.0])
def test_restricted_loss_plus_hard_moller_loss_is_total(m, t):
    wcc = 0.2
    lr = oracle.phys(oracle.L_RESTRICTED, m, t, wcc)
    lu = oracle.phys(oracle.L_RESTRICTED, m, t, 1e9)
    # energy lost to Moller deltas above wcc: n * int W dsigma/dW dW = n T int eps dsigma/deps
    # (integrated in ln eps: the 1/eps^2 part peaks at the lower end)
    hard = NA * m.z_over_a * t * quad(
        lambda y: math.exp(2 * y) * oracle.phys(oracle.DSIGMA_MOLLER, m, t, math.exp(y)),
        math.log(wcc / t), math.log(0.5), epsrel=1e-13, limit=200)[0]
    assert abs((lr + hard) / lu - 1) < 1e-9


@pytest.mark.parametrize("t", [0.45, 1.0, 3.0, 20.0])
def test_moller_total_is_integral_of_differential(t):
    wcc = 0.2
    tot = quad(lambda y: math.exp(y) * oracle.phys(oracle.DSIGMA_MOLLER, WATER, t, math.exp(y)),
               math.log(wcc / t), math.log(0.5), epsrel=1e-13, limit=200)[0]
    mu = oracle.phys(oracle.MU_MOLLER, WATER, t, wcc)
    assert abs(mu / (NA * WATER.z_over_a * tot) - 1) < 1e-9
    assert oracle.phys(oracle.MU_MOLLER, WATER, 0.39, wcc) == 0.0


@pytest.mark.parametrize("t", [0.3, 1.0, 6.0, 20.0])
def test_bremsstrahlung_integrals(t):
    wcb = 0.05
    f = lambda k: oracle.phys(oracle.DMU_BREMS, WATER, t, k)
    hard = quad(f, wcb, t, epsrel=1e-12)[0]
    assert abs(oracle.phys(oracle.MU_BREMS, WATER, t, wcb) / hard - 1) < 1e-10
    soft = quad(lambda k: k * f(k), 0, wcb, epsrel=1e-12)[0]
    assert abs(oracle.phys(oracle.S_RAD_SOFT, WATER, t, wcb) / soft - 1) < 1e-10
    # complete screening: total radiative stopping power is T / X0
    tot = quad(lambda k: k * f(k), 0, t, epsrel=1e-12)[0]
    assert abs(tot / (t / oracle.phys(oracle.X0, WATER, 1.0)) - 1) < 1e-10


@pytest.mark.parametrize("m", [WATER, BONE], ids=lambda m: m.name)
def test_hard_attenuation_increases_with_energy(m):
    ts = np.exp(np.linspace(np.log(0.2), np.log(25.0), 3000))
    mh = [oracle.phys(oracle.MU_MOLLER, m, t, 0.2) + oracle.phys(oracle.MU_BREMS, m, t, 0.05)
          for t in ts]
    assert np.all(np.diff(mh) >= 0)


@pytest.mark.parametrize("m", [WATER, BONE], ids=lambda m: m.name)
@pytest.mark.parametrize("t", [0.3, 1.0, 10.0])
def test_transport_cross_section_of_screened_rutherford(m, t):
    """1/lambda_1 equals the integral of (1 - cos) against the screened
    Rutherford cross section with Moliere's screening parameter."""
    al = 1 / 137.035999084
    pc2 = t * (t + 2 * MC2)
    g = 1 + t / MC2
    b2 = 1 - 1 / g ** 2
    a_s = 0.25 * (al * m.z ** (1 / 3) * MC2 / (0.885 * math.sqrt(pc2))) ** 2 * (
        1.13 + 3.76 * (al * m.z) ** 2 / b2)
    kk = m.z * (m.z + 1) * RE ** 2 * MC2 ** 2 / (b2 * pc2)
    # dsigma/dOmega = kk / (1 - cos + 2 A)^2 ; integrate in x = 1 - cos over [0, 2]
    s1 = 2 * math.pi * kk * quad(lambda x: x / (x + 2 * a_s) ** 2, 0, 2, points=[2 * a_s, 20 * a_s],
                                 epsrel=1e-12, limit=400)[0]
    inv = NA / (m.z / m.z_over_a) * s1
    assert abs(oracle.phys(oracle.INV_LAMBDA1, m, t) / inv - 1) < 1e-8


def test_water_values_against_estar_ballpark():
    g = GOLD["water_electron_1MeV"]
    lc = oracle.phys(oracle.L_RESTRICTED, WATER, 1.0, 1e9)
    assert abs(lc / g["collision_stopping_power_MeV_cm2_g"] - 1) < g["tolerance"]
    rng = oracle.path_length(WATER, 0.01, 1.0, 1e9, 0.0)
    assert abs(rng / g["csda_range_g_cm2"] - 1) < g["tolerance"]


@pytest.mark.parametrize("m", [WATER, BONE, AIR], ids=lambda m: m.name)
def test_path_length_matches_independent_quadrature(m):
    s = lambda e: oracle.phys(oracle.S_TOTAL, m, e, 0.2, 0.05)
    for a, b in [(0.2, 1.0), (0.3, 0.5), (15.0, 20.0), (0.2, 25.0)]:
        ref = quad(lambda e: 1 / s(e), a, b, points=[0.4] if a < 0.4 < b else None,
                   epsrel=1e-13, limit=200)[0]
        assert abs(oracle.path_length(m, a, b) / ref - 1) < 1e-11


@pytest.mark.parametrize("m", [WATER, BONE], ids=lambda m: m.name)
def test_csda_energy_inverts_path_length(m):
    for t0, q in [(1.0, 0.05), (20.0, 2.0), (0.3, 0.01), (5.0, 1e-6)]:
        t = oracle.csda_energy(m, t0, q)
        assert t < t0
        assert abs(oracle.path_length(m, t, t0) - q) < 1e-12 * q + 1e-14


@pytest.mark.parametrize("a", [1e-8, 1e-4, 0.01, 0.3, 5.0, 2e3, 1e6])
def test_mw_mean_is_mean_of_pdf(a):
    # substitute x = ln(mu + A): the integrand becomes A(1+A)(1 - A e^-x), smooth
    num = a * (1 + a) * quad(lambda x: 1 - a * math.exp(-x), math.log(a), math.log1p(a),
                             epsrel=1e-13, limit=200)[0]
    assert abs(oracle.phys(oracle.MW_MEAN, WATER, 1.0, a) / num - 1) < 1e-9


@pytest.mark.parametrize("t", [1e-7, 1e-3, 0.1, 1.0, 5.0, 15.0])
def test_mw_screening_matches_lewis_first_moment(t):
    a = oracle.mw_A(t)
    assert abs(oracle.phys(oracle.MW_MEAN, WATER, 1.0, a) / (-0.5 * math.expm1(-t)) - 1) < 1e-9
