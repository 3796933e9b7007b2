"""Pins of the oracle's random choices and of the kinematics of its photon
interactions.

Choice rules (section 2.1's transport: Woodcock tracking against a majorant,
the interaction type by its share of the attenuation, delta scattering of the
hard electron events against a step-start majorant, Moller or bremsstrahlung
by their share of the hard cross section).  Each choice picks outcome i with a
probability p_i that the oracle computes from the closed forms at that moment;
over a run, N_i - sum p_i is a martingale with variance sum p_i (1 - p_i), so
z = (N_i - sum p_i) / sqrt(sum p_i (1 - p_i)) is close to standard normal
whatever the energies at which the choices were made.  A wrong branch order,
a wrong normalisation or swapped outcomes moves z by many units.

Kinematics: pair production splits E - 2 mc^2 uniformly and conserves energy;
the Compton electron leaves at cot(theta_e) = (1 + k) tan(theta_gamma / 2), the
two-body relation of free-electron Compton scattering.

The hard-event free path: with angular deflections off, an electron slowing
down from T_0 has its first real hard event after a number of mean free paths
distributed as Exp(1), so the probability that a history has no hard event at
all is exp(-integral_{E_abs}^{T_0} mu_h(T) / S_r(T) dT), summed over the
layers crossed (the density cancels inside a layer).  This pins the hard-event
counter across voxel faces and the acceptance against the majorant."""
import math

import numpy as np
import pytest
from scipy import stats as sst
from scipy.integrate import quad
from scipy.optimize import brentq

import oracle
from paper_1107_3355_amd import inputs as I

MC2 = 0.51099895
MATS = I.MATERIALS


def _z_scores(r, min_var=20.0):
    out = {}
    for name, (n, p, v) in r["choices"].items():
        if v >= min_var:
            out[name] = (n - p) / math.sqrt(v)
    return out


@pytest.mark.parametrize("case", ["slab_photon", "slab_electron", "ct", "pair_rich"])
def test_choice_counts_follow_their_probabilities(case):
    if case == "slab_photon":
        w = I.slab_photon(n=40, d=0.75)
        r = oracle.run(MATS, w.phantom, w.source, n_hist=60_000, seed=21)
        need = ("flight_real", "flight_virtual", "compton", "pair", "hard_real", "moller", "brems")
    elif case == "slab_electron":
        w = I.slab_electron(n=40, d=0.75)
        r = oracle.run(MATS, w.phantom, w.source, n_hist=6_000, seed=22)
        need = ("hard_real", "hard_virtual", "moller", "brems", "flight_real", "compton")
    elif case == "ct":
        ph = I.ct_phantom((40, 40, 20), (1.0, 1.0, 1.25))
        src = I.Source(I.PHOTON, I.triangular_spectrum(), I.imrt_plan(ph, nb=8))
        r = oracle.run(MATS, ph, src, n_hist=60_000, seed=23)
        need = ("flight_real", "flight_virtual", "compton", "photo", "moller", "brems")
    else:
        # 20 MeV photons in bone: pair production is a large share of the real
        # interactions (one material at one density: every flight is real)
        ph = I.homogeneous((12, 12, 40), (1.0, 1.0, 1.0), I.ID_BONE, 1.85)
        src = I.Source(I.PHOTON, I.mono(20.0), [I.parallel_beam_z(ph, 4.0)])
        r = oracle.run(MATS, ph, src, n_hist=20_000, seed=24, flags=oracle.KERMA)
        need = ("compton", "pair", "photo")
        assert r["choices"]["flight_virtual"][0] == 0
    z = _z_scores(r)
    print(case, {k: round(v, 2) for k, v in z.items()},
          {k: r["choices"][k][0] for k in r["choices"]})
    for k in need:
        assert k in z, (k, r["choices"][k])
    for k, v in z.items():
        assert abs(v) < 4.5, (case, k, v)
    # every choice is counted once: outcomes of one choice sum to the choices
    # made (a flight that leaves the phantom makes no choice)
    c = {k: v[0] for k, v in r["choices"].items()}
    assert c["flight_real"] + c["flight_virtual"] <= r["events"]["flights"]
    assert c["flight_real"] == r["events"]["real"] == c["compton"] + c["photo"] + c["pair"]
    assert c["hard_real"] + c["hard_virtual"] == r["events"]["hard_cand"]
    assert c["hard_real"] == r["events"]["hard"] == c["moller"] + c["brems"]


def test_choice_counts_detect_a_planted_mistake():
    """The statistic is sensitive: the same run's counts tested against the
    probabilities of the swapped outcomes (as if the branches were exchanged)
    give |z| far above the acceptance bound."""
    w = I.slab_photon(n=40, d=0.75)
    r = oracle.run(MATS, w.phantom, w.source, n_hist=20_000, seed=25)
    n_m, p_m, v_m = r["choices"]["moller"]
    n_b, p_b, v_b = r["choices"]["brems"]
    assert abs((n_m - p_b) / math.sqrt(v_b)) > 10
    n_c, p_c, v_c = r["choices"]["compton"]
    n_p, p_p, v_p = r["choices"]["pair"]
    assert abs((n_c - (p_c + p_p)) / math.sqrt(v_c)) > 10 or abs((n_p - 0.0) / math.sqrt(v_p)) > 10


@pytest.mark.parametrize("e", [1.5, 6.0, 25.0])
def test_pair_split_uniform_and_energy_conserving(e):
    frac, de = oracle.sample(6, e, n=200_000, seed=31)
    assert frac.min() > 0.0 and frac.max() < 1.0
    assert sst.kstest(frac, "uniform").pvalue > 1e-4
    # T- + T+ + a = E up to double rounding (the positron keeps a = E - K)
    assert np.all(np.abs(de) <= 4e-16 * e)


@pytest.mark.parametrize("e", [0.1, 1.0, 6.0, 20.0])
def test_compton_electron_direction(e):
    """cot(theta_e) = (1 + k) tan(theta_gamma / 2), i.e.
    cos_e (1 + cos_g) = (1 + k) sin_g sin_e, and the electron moves forward."""
    k = e / MC2
    ce, cg = oracle.sample(7, e, n=100_000, seed=33)
    se = np.sqrt(np.maximum(0.0, 1 - ce * ce))
    sg = np.sqrt(np.maximum(0.0, 1 - cg * cg))
    lhs, rhs = ce * (1 + cg), (1 + k) * sg * se
    assert np.all(np.abs(lhs - rhs) <= 1e-9 * (1 + k))
    assert np.all(ce >= -1e-12)
    # the sampler's photon angle is the Klein-Nishina one: <cos> against quadrature
    f = lambda x: oracle.phys(oracle.DSIGMA_KN, I.WATER, e, x)
    e0 = 1 / (1 + 2 * k)
    norm = quad(f, e0, 1, epsrel=1e-12)[0]
    mean_cos = quad(lambda x: f(x) * (1 - (1 - x) / (k * x)), e0, 1, epsrel=1e-12)[0] / norm
    assert abs(cg.mean() - mean_cos) < 5 * cg.std() / math.sqrt(len(cg))


def _mfp_integral(mat, ta, tb, wcc=0.2, wcb=0.05):
    """integral_{ta}^{tb} mu_h(T) / S_r(T) dT, from the closed forms"""
    def f(t):
        mu = oracle.phys(oracle.MU_MOLLER, mat, t, wcc) + oracle.phys(oracle.MU_BREMS, mat, t, wcb)
        return mu / oracle.phys(oracle.S_TOTAL, mat, t, wcc, wcb)
    pts = [x for x in (2 * wcc,) if ta < x < tb]
    return quad(f, ta, tb, points=pts or None, epsrel=1e-11, limit=200)[0]


def _layered(mats, rhos, dz, lateral=2.0):
    ph = I.homogeneous((1, 1, len(mats)), (lateral, lateral, dz), I.ID_WATER, 1.0)
    ph.mat[:, 0, 0] = mats
    ph.rho[:, 0, 0] = rhos
    return ph


@pytest.mark.parametrize("hetero", [False, True])
def test_hard_event_free_path(hetero):
    t0, dz, ecut = 3.0, 0.05, 0.2
    if hetero:
        mats = [I.ID_WATER] * 6 + [I.ID_BONE] * 6 + [I.ID_LUNG] * 30 + [I.ID_WATER] * 60
    else:
        mats = [I.ID_WATER] * 80
    rhos = np.array([MATS[m].rho_nominal for m in mats], dtype=np.float32)
    ph = _layered(mats, rhos, dz)
    src = I.Source(I.ELECTRON, I.mono(t0), [I.parallel_beam_z(ph, 0.01)])
    n = 40_000
    r = oracle.run(MATS, ph, src, n_hist=n, seed=35, flags=oracle.NO_MS, want_hist=True,
                   want_hist_hard=True)
    # mean free paths along the slowing-down path, layer by layer (T at the
    # faces from the range integral, solved independently of the oracle)
    tau, t = 0.0, t0
    for m, rho in zip(mats, rhos.astype(np.float64)):
        mat = MATS[m]
        s = lambda e: oracle.phys(oracle.S_TOTAL, mat, e, 0.2, 0.05)
        path = lambda a, b: quad(lambda e: 1 / s(e), a, b, points=[0.4] if a < 0.4 < b else None,
                                 epsrel=1e-12, limit=200)[0]
        q = rho * dz
        t1 = ecut if path(ecut, t) <= q else brentq(lambda x: path(x, t) - q, ecut, t, xtol=1e-14)
        tau += _mfp_integral(mat, t1, t)
        t = t1
        if t <= ecut:
            break
    p = math.exp(-tau)
    k = int((r["hist_hard"] == 0).sum())
    print("no hard event", k / n, "expected", p, "tau", tau)
    assert abs(k - n * p) < 4.5 * math.sqrt(n * p * (1 - p))
    # a history without a hard event deposits exactly its energy, along the axis
    assert np.allclose(r["hist"][r["hist_hard"] == 0, 0], t0, rtol=1e-12)
