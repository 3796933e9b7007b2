"""Transport-level pins of the oracle: special cases of the full method that
reduce to closed forms, exact energy conservation, determinism, and the
calibration of the acceptance statistics (section 3.1) on oracle-vs-oracle runs.
"""
import math

import numpy as np
import pytest
from scipy import stats as sst
from scipy.integrate import quad
from scipy.optimize import brentq

import oracle
from paper_1107_3355_amd import inputs as I
from tests import stats as S

MC2 = 0.51099895


def _layered(mats, rhos, dz, lateral=2.0):
    nz = len(mats)
    ph = I.homogeneous((1, 1, nz), (lateral, lateral, dz), I.ID_WATER, 1.0)
    ph.mat[:, 0, 0] = mats
    ph.rho[:, 0, 0] = rhos
    return ph


def test_photoelectric_only_layers_follow_beer_lambert():
    """Photoelectric absorption only, E below the electron absorption energy:
    each photon deposits E where it is absorbed, so the fraction absorbed in
    layer i is exp(-tau_i) - exp(-tau_{i+1}) with tau the optical depth. The
    densities alternate, so Woodcock's majorant rejects many flights."""
    nz, dz, e = 24, 0.5, 0.06
    rhos = np.where(np.arange(nz) % 2 == 0, 1.85, 0.6).astype(np.float32)
    ph = _layered([I.ID_BONE] * nz, rhos, dz)
    src = I.Source(I.PHOTON, I.mono(e), [I.parallel_beam_z(ph, 0.5)])
    n = 100_000
    r = oracle.run(I.MATERIALS, ph, src, n_hist=n, flags=oracle.NO_COMPTON | oracle.NO_PAIR)
    counts = np.append(r["batch_edep"].sum(axis=0) / e, r["e_esc"] / e)
    assert np.allclose(counts, np.round(counts), atol=1e-6)
    mu = oracle.phys(oracle.MU_PHOTO, I.BONE, e)
    tau = np.concatenate([[0.0], np.cumsum(rhos * mu * dz)])
    p = np.append(np.exp(-tau[:-1]) - np.exp(-tau[1:]), np.exp(-tau[-1]))
    assert sst.chisquare(np.round(counts), p * n).pvalue > 1e-4


def test_narrow_beam_uncollided_fraction():
    """Pencil beam, full photon physics in kerma mode: a history deposits
    nothing iff its primary crosses without a real interaction, so that
    fraction is exp(-sum mu_i L_i) (binomial)."""
    mats = [I.ID_WATER] * 6 + [I.ID_BONE] * 4 + [I.ID_LUNG] * 6 + [I.ID_WATER] * 4
    rhos = np.array([I.MATERIALS[m].rho_nominal for m in mats], dtype=np.float32)
    dz, e = 1.0, 2.0
    ph = _layered(mats, rhos, dz)
    src = I.Source(I.PHOTON, I.mono(e), [I.parallel_beam_z(ph, 0.01)])
    n = 200_000
    r = oracle.run(I.MATERIALS, ph, src, n_hist=n, flags=oracle.KERMA, want_hist=True)
    k = int((r["hist"][:, 0] == 0.0).sum())
    mu = lambda m: sum(oracle.phys(w, I.MATERIALS[m], e)
                       for w in (oracle.MU_COMPTON, oracle.MU_PHOTO, oracle.MU_PAIR))
    p = math.exp(-sum(rho * mu(m) * dz for m, rho in zip(mats, rhos)))
    assert abs(k - n * p) < 4 * math.sqrt(n * p * (1 - p))


def _csda_profile(mats, rhos, dz, t0, ecut=0.2):
    """Energy deposited per layer by a straight electron losing energy
    continuously: T(z) from integral dT/S_r = rho dz, solved independently."""
    dep = []
    t = t0
    for m, rho in zip(mats, rhos):
        mat = I.MATERIALS[m]
        if t <= ecut:
            dep.append(0.0)
            continue
        s = lambda e: oracle.phys(oracle.S_TOTAL, mat, e, 0.2, 0.05)
        path = lambda a, b: quad(lambda e: 1 / s(e), a, b, points=[0.4] if a < 0.4 < b else None,
                                 epsrel=1e-13, limit=200)[0]
        q = rho * dz
        if path(ecut, t) <= q:
            dep.append(t)
            t = 0.0
        else:
            t1 = brentq(lambda x: path(x, t) - q, ecut, t, xtol=1e-15, rtol=1e-15)
            dep.append(t - t1)
            t = t1
    return np.array(dep)


@pytest.mark.parametrize("hetero", [False, True])
def test_electron_csda_pencil_deposits_exact(hetero):
    """Hard events and deflections off: an electron moves straight and loses
    energy by the restricted stopping power only, so the energy left in each
    layer is fixed by the range integral (deterministic)."""
    nz, dz, t0 = 30, 0.1, 3.0
    if hetero:
        mats = [I.ID_WATER] * 5 + [I.ID_BONE] * 5 + [I.ID_LUNG] * 10 + [I.ID_WATER] * 10
    else:
        mats = [I.ID_WATER] * nz
    rhos = np.array([I.MATERIALS[m].rho_nominal for m in mats], dtype=np.float32)
    ph = _layered(mats, rhos, dz)
    src = I.Source(I.ELECTRON, I.mono(t0), [I.parallel_beam_z(ph, 0.01)])
    r = oracle.run(I.MATERIALS, ph, src, n_hist=20, n_batches=2, n_threads=1,
                   flags=oracle.NO_MS | oracle.NO_MOLLER | oracle.NO_BREMS)
    got = r["batch_edep"].sum(axis=0) / 20
    exp = _csda_profile(mats, rhos.astype(np.float64), dz, t0)
    assert np.allclose(got, exp, rtol=1e-9, atol=1e-12)
    assert r["e_esc"] == 0.0


def _balance(r):
    return abs(r["e_dep"] + r["e_esc"] - r["e_in"]) / r["e_in"]


def _small_ct():
    ph = I.ct_phantom((48, 48, 24), (1.0, 1.0, 1.25))
    return I.Source(I.PHOTON, I.triangular_spectrum(), I.imrt_plan(ph, nb=10)), ph


@pytest.mark.parametrize("case", ["water", "slab_photon", "slab_electron", "ct", "pairs"])
def test_energy_conservation(case):
    if case == "water":
        w = I.water_cube_2mev(4000)
        ph, src, n = w.phantom, w.source, w.n_hist
    elif case == "slab_photon":
        w = I.slab_photon(3000, n=50, d=0.6)
        ph, src, n = w.phantom, w.source, w.n_hist
    elif case == "slab_electron":
        w = I.slab_electron(200, n=50, d=0.6)
        ph, src, n = w.phantom, w.source, w.n_hist
    elif case == "ct":
        src, ph = _small_ct()
        n = 3000
    else:
        ph = I.homogeneous((10, 10, 10), (1.0, 1.0, 1.0), I.ID_BONE, 1.85)
        src = I.Source(I.PHOTON, I.mono(15.0), [I.parallel_beam_z(ph, 4.0)])
        n = 1000
    r = oracle.run(I.MATERIALS, ph, src, n_hist=n, want_hist=True)
    assert _balance(r) < 1e-12
    e_in = oracle.sample_source(src, ph, n=n)[:, 0]
    h = r["hist"]
    assert np.allclose(h[:, 0] + h[:, 1], e_in, rtol=1e-12, atol=0)
    assert np.all(r["dose"] >= 0) and np.all(r["sigma"] >= 0)
    if case == "pairs":
        assert r["events"]["pushes"] > 0


def test_determinism_and_thread_independence():
    w = I.water_cube_2mev(3000)
    a = oracle.run(I.MATERIALS, w.phantom, w.source, n_hist=w.n_hist, n_threads=4)
    b = oracle.run(I.MATERIALS, w.phantom, w.source, n_hist=w.n_hist, n_threads=4)
    c = oracle.run(I.MATERIALS, w.phantom, w.source, n_hist=w.n_hist, n_threads=1)
    assert np.array_equal(a["dose"], b["dose"])
    assert np.allclose(a["dose"], c["dose"], rtol=1e-12, atol=1e-300)
    assert a["events"] == c["events"]


def test_batches_are_contiguous_rounds():
    """History h goes to batch floor(h / R) mod N_b; the per-history tallies of
    a run reproduce its per-batch energy sums."""
    w = I.water_cube_2mev(1000)
    r = oracle.run(I.MATERIALS, w.phantom, w.source, n_hist=1000, n_batches=4, round_size=100,
                   want_hist=True)
    dep = r["hist"][:, 0]
    per = [dep[np.arange(1000) // 100 % 4 == b].sum() for b in range(4)]
    assert np.allclose(r["batch_edep"].sum(axis=1), per, rtol=1e-12)


def test_oracle_vs_oracle_statistics_calibration():
    """Two independent runs (different seeds) of the same method: the per-voxel
    t-test passes at about the nominal rate for N_b = 10 and t_{0.975,9}, and
    the batch-resolved region sums agree within their standard error."""
    w = I.water_cube_2mev(200_000)
    a = oracle.run(I.MATERIALS, w.phantom, w.source, seed=1, n_hist=w.n_hist)
    b = oracle.run(I.MATERIALS, w.phantom, w.source, seed=2, n_hist=w.n_hist)
    rate, nreg = S.pass_rate(a["dose"], a["sigma"], b["dose"], b["sigma"])
    assert nreg > 1000
    assert 0.93 <= rate <= 0.99, rate
    region = np.maximum(a["dose"], b["dose"]) > 0.1 * max(a["dose"].max(), b["dose"].max())
    nb = w.n_hist / 10
    diff, se = S.region_sum_test(a["batch_edep"], nb, b["batch_edep"], nb, region)
    assert abs(diff) < 3 * se
    assert abs(a["e_in"] - b["e_in"]) == 0.0  # monoenergetic source
