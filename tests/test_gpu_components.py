"""GPU components against the oracle, through the C ABI test entry points.

The device and the oracle draw the same Philox streams, so each sample can be
compared one by one: the generator bit for bit, samplers and the source to
single-precision rounding (a rare sample may take the other branch of a
rejection test when a single-precision value lands next to the threshold),
table lookups to the interpolation tolerance of section 2.2.2."""
import math

import numpy as np
import pytest
from scipy import stats as sst
from scipy.integrate import quad

import oracle
from paper_1107_3355_amd import inputs as I
from tests.gpu_common import report

pytestmark = pytest.mark.gpu


def test_philox_bit_identical(gctx):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(100_000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 0, 0, 1]]
    for key in ([0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [12345, 67890]):
        out = gctx.philox(key, ctr)
        ref = np.array([oracle.philox(key, [int(v) for v in c]) for c in ctr[::10]], dtype=np.uint32)
        assert np.array_equal(out[::10], ref)


def test_philox_known_answer_vectors(gctx):
    """The device generator against the published Philox4x32-10 vectors."""
    import json
    import os
    kat = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")))
    for vec in kat["vectors"]:
        ctr = np.array([[int(x, 16) for x in vec["ctr"]]], dtype=np.uint32)
        out = gctx.philox([int(x, 16) for x in vec["key"]], ctr)
        assert [int(v) for v in out[0]] == [int(x, 16) for x in vec["out"]]


def _close(a, b, rel):
    return np.abs(a - b) <= rel * np.maximum(np.abs(b), 1e-30)


@pytest.mark.parametrize("e", [0.06, 0.5, 2.0, 10.0, 25.0])
def test_compton_lockstep(gctx, e):
    n = 200_000
    ga, gb = gctx.sample(0, e, n=n, seed=5)
    oa, ob = oracle.sample(0, e, n=n, seed=5)
    frac = np.mean(_close(ga, oa, 2e-5))
    report("compton", e=e, lockstep=frac)
    assert frac > 0.999
    k = e / 0.51099895
    edges = np.linspace(1 / (1 + 2 * k), 1, 41)
    f = lambda x: oracle.phys(oracle.DSIGMA_KN, I.WATER, e, x)
    w = np.array([quad(f, a, b)[0] for a, b in zip(edges[:-1], edges[1:])])
    h, _ = np.histogram(ga, edges)
    assert sst.chisquare(h, w / w.sum() * h.sum()).pvalue > 1e-4


@pytest.mark.parametrize("t", [0.5, 3.0, 20.0])
def test_moller_lockstep(gctx, t):
    ga, gb = gctx.sample(1, t, 0.2, n=100_000, seed=7)
    oa, ob = oracle.sample(1, t, 0.2, n=100_000, seed=7)
    frac = np.mean(_close(ga, oa, 2e-5) & _close(gb, ob, 2e-5))
    report("moller", t=t, lockstep=frac)
    assert frac > 0.999


@pytest.mark.parametrize("t", [0.3, 6.0, 20.0])
def test_bremsstrahlung_lockstep(gctx, t):
    ga, _ = gctx.sample(2, t, 0.05, n=100_000, seed=9)
    oa, _ = oracle.sample(2, t, 0.05, n=100_000, seed=9)
    frac = np.mean(_close(ga, oa, 2e-5))
    report("brems", t=t, lockstep=frac)
    assert frac > 0.999
    # the photon never takes more than the electron's energy (the hardware
    # log2 and exp2 could round past T for draws next to 1; the sampler clamps)
    assert ga.min() >= 0.05 and ga.max() <= np.float32(t)


@pytest.mark.parametrize("t", [1e-6, 1e-3, 0.1, 2.0, 19.0, 25.0])
def test_mw_deflection_lockstep(gctx, t):
    ga, _ = gctx.sample(3, t, n=100_000, seed=11)
    oa, _ = oracle.sample(3, t, n=100_000, seed=11)
    frac = np.mean(np.abs(ga - oa) <= 2e-4 * np.maximum(oa, 1e-12) + 1e-12)
    report("mw", t=t, lockstep=frac)
    assert frac > 0.99
    assert abs(ga.mean() - (-0.5 * math.expm1(-t))) < 5 * ga.std() / math.sqrt(len(ga))


@pytest.mark.parametrize("t,nh", [(0.05, 10), (0.5, 4)])
def test_multiple_scattering_first_moment(gctx, t, nh):
    c, norm = gctx.sample(4, t, 0.0, nh, n=100_000, seed=13)
    assert np.allclose(norm, 1.0, atol=1e-5)
    assert abs(c.mean() - math.exp(-nh * t)) < 5 * c.std() / math.sqrt(len(c))


def test_annihilation(gctx):
    c, dot = gctx.sample(5, 0.0, n=100_000, seed=17)
    oc, _ = oracle.sample(5, 0.0, n=100_000, seed=17)
    assert np.allclose(dot, -1.0, atol=1e-5)
    assert np.allclose(c, oc, atol=1e-6)


@pytest.mark.parametrize("mi", range(4))
def test_lookups_match_closed_forms(gctx, mi):
    m = I.MATERIALS[mi]
    e = np.exp(np.random.default_rng(mi).uniform(np.log(0.21), np.log(29.0), 400)).astype(np.float32)
    ed = e.astype(np.float64)
    mu = gctx.lookup(0, mi, e)
    ref = np.array([sum(oracle.phys(w, m, x) for w in (0, 1, 2)) for x in ed])
    assert np.max(np.abs(mu / ref - 1)) < 1e-4
    rng = gctx.lookup(1, mi, e)
    rref = np.array([oracle.path_length(m, 0.2, x) for x in ed])
    assert np.all(np.abs(rng - rref) < 1e-4 * rref + 1e-6)
    il = gctx.lookup(4, mi, e)
    iref = np.array([oracle.phys(oracle.INV_LAMBDA1, m, x) for x in ed])
    assert np.max(np.abs(il / iref - 1)) < 1e-4
    hi = ed > 0.45
    mh = gctx.lookup(2, mi, e)
    href = np.array([oracle.phys(oracle.MU_MOLLER, m, x, 0.2) + oracle.phys(oracle.MU_BREMS, m, x, 0.05)
                     for x in ed])
    assert np.max(np.abs(mh[hi] / href[hi] - 1)) < 1e-4
    # inverse range: E(R(E)) = E
    back = gctx.lookup(5, mi, rng)
    assert np.max(np.abs(back[hi] / e[hi] - 1)) < 2e-4


def test_mw_screening_lookup(gctx):
    t = np.exp(np.linspace(np.log(1e-8), np.log(15.0), 60)).astype(np.float32)
    a = gctx.lookup(6, 0, t)
    ref = np.array([oracle.mw_A(float(x)) for x in t])
    assert np.max(np.abs(a / ref - 1)) < 3e-4


def _source_cases():
    w1 = I.water_cube_2mev(1)
    w2 = I.slab_photon(1)
    w3 = I.slab_electron(1)
    return [("water_parallel", w1.phantom, w1.source), ("slab_point", w2.phantom, w2.source),
            ("slab_electron", w3.phantom, w3.source)]


@pytest.mark.parametrize("case", [0, 1, 2, 3, 4])
def test_source_lockstep(gctx, case):
    if case < 3:
        name, ph, src = _source_cases()[case]
    elif case == 3:
        w = I.ct_imrt()
        name, ph, src = "ct_imrt_full", w.phantom, w.source
    else:
        # the serving form's 180-control-point arc: 288,000 beamlets
        ph = I.ct_imrt().phantom
        name, src = "ct_vmat180_full", I.Source(I.PHOTON, I.triangular_spectrum(), I.vmat_arc(ph))
    p = gctx.phantom(ph)
    s = gctx.source(src)
    n = 20_000
    g = gctx.sample_source(p, s, n=n, hist0=12345)
    o = oracle.sample_source(src, ph, n=n, hist0=12345)
    p.close()
    s.close()
    assert np.array_equal(g[:, 1], o[:, 1].astype(np.float32))      # same beamlet
    inside = o[:, 1] >= 0
    # the inverse CDF is ill-conditioned where the pdf vanishes (spectrum ends):
    # single precision moves a rare sample by up to 1e-4 relative there
    rel = np.abs(g[:, 0] / o[:, 0] - 1)
    assert np.mean(rel < 2e-6) > 0.999 and rel.max() < 1e-4
    np.testing.assert_allclose(g[inside, 2:5], o[inside, 2:5], atol=2e-4)
    np.testing.assert_allclose(g[inside, 5:8], o[inside, 5:8], atol=2e-5)
    report("source", case=name, inside=float(inside.mean()))


def test_metropolis_source_lockstep(gctx):
    """Metropolis beamlet chains (Algorithm A1) on the device against the
    oracle's: the same beamlet for every history of every chain (integer,
    exact), on the full-size 9-beam CT plan with zero-intensity beamlets added,
    over four steps of each chain from a first history that is not a multiple
    of the chain count."""
    import dataclasses
    w = I.ct_imrt()
    beams = []
    for k, b in enumerate(w.source.beams):
        f = np.array(b.intensity, dtype=np.float32, copy=True)
        f.ravel()[k::7] = 0.0
        beams.append(dataclasses.replace(b, intensity=f))
    src = I.Source(w.source.particle, w.source.spectrum, beams, beamlet_sampler=1)
    p = gctx.phantom(w.phantom)
    s = gctx.source(src)
    n = 4 * oracle.METRO_CHAINS + 777
    g = gctx.sample_source(p, s, n=n, hist0=98765)
    o = oracle.sample_source(src, w.phantom, n=n, hist0=98765)
    p.close()
    s.close()
    assert np.array_equal(g[:, 1], o[:, 1].astype(np.float32))
    inside = o[:, 1] >= 0
    np.testing.assert_allclose(g[inside, 2:5], o[inside, 2:5], atol=2e-4)
    zero = np.concatenate([np.asarray(b.intensity).ravel() == 0 for b in beams])
    assert not zero[o[inside, 1].astype(int)].any()
    report("metropolis source", inside=float(inside.mean()))


@pytest.mark.parametrize("shape", [0, 1])
def test_stratified_source_lockstep(gctx, shape):
    """Energy intervals (section 2.3.2): for one round of n histories the device
    and the oracle put every history in the same interval and give it the same
    energy to single-precision rounding (uniform inside the interval, shape 0,
    or the spectrum's shape, 1); the beamlets are unchanged."""
    import dataclasses
    w = I.ct_imrt()
    K = 16
    src = dataclasses.replace(w.source, spectrum_strata=K, strata_shape=shape)
    p = gctx.phantom(w.phantom)
    s = gctx.source(src)
    n = 50_001
    g = gctx.sample_source(p, s, n=n, hist0=4242)
    o = oracle.sample_source(src, w.phantom, n=n, hist0=4242)
    p.close()
    s.close()
    assert np.array_equal(g[:, 1], o[:, 1].astype(np.float32))
    sp = src.spectrum
    edges = sp.e[0] + (sp.e[-1] - sp.e[0]) * np.arange(K + 1) / K
    kg = np.clip(np.searchsorted(edges, g[:, 0], side="right") - 1, 0, K - 1)
    ko = np.clip(np.searchsorted(edges, o[:, 0], side="right") - 1, 0, K - 1)
    assert np.mean(kg == ko) > 0.9999                  # an energy on an edge may round across
    rel = np.abs(g[:, 0] / o[:, 0] - 1)
    assert np.mean(rel < 2e-6) > 0.999 and rel.max() < 1e-4
    assert np.all(np.diff(ko) >= 0)


def test_phase_space_source_lockstep(gctx):
    """Phase-space primaries (section 2.3.3) on the device against the oracle:
    the same record per history, the same entry points (single precision) and
    the same escapes, over more histories than records."""
    w = I.ct_imrt()
    ps = I.point_phase_space(w.phantom, 30_000, seed=8, inside_frac=0.2)
    ps[:50, 3:6] *= -1.0                         # a few rays that miss the phantom
    src = I.Source(I.PHOTON, I.mono(1.0), [], phase_space=ps)
    p = gctx.phantom(w.phantom)
    s = gctx.source(src)
    n = 70_001
    g = gctx.sample_source(p, s, n=n, hist0=123)
    o = oracle.sample_source(src, w.phantom, n=n, hist0=123)
    p.close()
    s.close()
    assert np.array_equal(g[:, 1], o[:, 1].astype(np.float32))
    inside = o[:, 1] >= 0
    assert 0.9 < inside.mean() < 1.0
    np.testing.assert_allclose(g[inside, 2:5], o[inside, 2:5], atol=2e-4)
    np.testing.assert_array_equal(g[:, 0], o[:, 0].astype(np.float32))


@pytest.mark.parametrize("e", [1.5, 6.0, 25.0])
def test_pair_split(gctx, e):
    """The kernel's pair split: T-/K uniform (same draws as the oracle's, so
    equal to single-precision rounding) and T- + T+ = K exactly."""
    ga, gb = gctx.sample(6, e, n=200_000, seed=19)
    oa, _ = oracle.sample(6, e, n=200_000, seed=19)
    assert np.all(gb == 0.0)
    assert np.all(np.abs(ga - oa) <= 2e-6)
    assert sst.kstest(ga, "uniform").pvalue > 1e-4


@pytest.mark.parametrize("e", [0.1, 1.0, 6.0, 20.0])
def test_compton_electron_direction(gctx, e):
    """The kernel's Compton electron direction against the oracle's on the same
    streams, and the two-body relation cot(theta_e) = (1 + k) tan(theta_g / 2)
    to single precision."""
    k = e / 0.51099895
    ce, cg = gctx.sample(7, e, n=100_000, seed=23)
    oe, og = oracle.sample(7, e, n=100_000, seed=23)
    frac = np.mean((np.abs(ce - oe) <= 1e-4) & (np.abs(cg - og) <= 1e-4))
    report("compton electron", e=e, lockstep=frac)
    assert frac > 0.999
    ce, cg = ce.astype(np.float64), cg.astype(np.float64)
    se, sg = np.sqrt(np.maximum(0, 1 - ce * ce)), np.sqrt(np.maximum(0, 1 - cg * cg))
    # single precision: cosines near 1 carry about 1e-7 absolute, sines near 0 about 5e-4
    assert np.median(np.abs(ce * (1 + cg) - (1 + k) * sg * se)) < 1e-5 * (1 + k)
    assert np.mean(np.abs(ce * (1 + cg) - (1 + k) * sg * se) < 1e-3 * (1 + k)) > 0.999


@pytest.mark.parametrize("case", ["slab_photon", "slab_electron"])
def test_solo_lanes_same_physics(case):
    """The one-particle-per-wavefront measurement form runs the same kernels'
    code with one lane busy: every particle takes the same path, so the physics
    event counts are equal and the dose equals the normal form's up to the
    order of the FP64 tally additions."""
    from paper_1107_3355_amd import gdpm as G
    from tests.gpu_common import gpu_run, physics_events
    w = I.slab_photon(n=40, d=0.75) if case == "slab_photon" else I.slab_electron(n=40, d=0.75)
    n = 20_000 if case == "slab_photon" else 4_000
    out = []
    for opts in ('{}', '{"solo_lanes": 1, "graphs": 0}'):
        ctx = G.Context(0, opts=opts, materials=I.MATERIALS)
        try:
            out.append(gpu_run(ctx, w.phantom, w.source, n_hist=n, seed=5))
        finally:
            ctx.close()
    a, b = out
    assert physics_events(a) == physics_events(b)
    assert a["interactions"] == b["interactions"]
    err = np.abs(a["dose"] - b["dose"]).max() / a["dose"].max()
    report(f"solo lanes {case}", max_rel_diff=f"{err:.2e}", t_normal=f"{a['t_kernel_s']:.4f}",
           t_solo=f"{b['t_kernel_s']:.4f}")
    assert err < 1e-9
    assert b["transport_anomalies"] == 0
