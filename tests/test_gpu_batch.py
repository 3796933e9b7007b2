"""Many jobs through one engine: the batched form (gdpm_run_batch) and the
server (gdpm_server_*).

A job's particles draw only from the job's own Philox streams (seed, job_id),
so its dose in a mix must equal its dose alone up to the order of the FP64
tally additions; that is checked to a relative 1e-9 of the job's maximum dose.
Energy balance is checked per job.  Plus admission by slots and footprint, the
online autotuner (which may change launch settings, never results), and error
paths."""
import time

import numpy as np
import pytest

from paper_1107_3355_amd import gdpm as G
from paper_1107_3355_amd import inputs as I
from tests.gpu_common import balance, physics_events, report

pytestmark = pytest.mark.gpu
MATS = I.MATERIALS


def small_jobs(n=5, seed=4101):
    """Uneven small jobs: photons and electrons, spectra and lines, fixed and
    target-uncertainty mode."""
    ws = I.batch_jobs(n, seed=seed, side=(12, 28), d=0.5, hist=(3e3, 4e4))
    out = []
    for k, w in enumerate(ws):
        kw = dict(seed=11 + k, job_id=k, n_hist=w.n_hist, n_batches=10)
        if k == 1:
            # super-rounds until 5% (about 1e6 histories on these cubes)
            kw.update(target_unc=0.05, n_hist=20_000, max_histories=5_000_000)
        out.append((w, kw))
    return out


def same_dose(a, b, what):
    scale = max(np.abs(a).max(), np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max() / scale
    report(what, max_rel_diff=f"{err:.2e}")
    assert err < 1e-9, what


def solo(ctx, w, kw):
    p, s = ctx.phantom(w.phantom), ctx.source(w.source)
    try:
        return ctx.run(p, s, **kw)
    finally:
        p.close()
        s.close()


def test_batch_equals_solo(gctx):
    jobs = small_jobs()
    handles = [(gctx.phantom(w.phantom), gctx.source(w.source), kw) for w, kw in jobs]
    try:
        res = gctx.run_batch(handles)
    finally:
        for p, s, _ in handles:
            p.close()
            s.close()
    for (w, kw), r in zip(jobs, res):
        assert r["status"] in ("GDPM_OK", "GDPM_E_NOT_CONVERGED")
        a = solo(gctx, w, kw)
        assert r["histories"] == a["histories"], w.name
        assert balance(r) < 1e-6, w.name
        same_dose(r["dose"], a["dose"], f"batch vs solo {w.name}")
        same_dose(r["sigma"], a["sigma"], f"batch vs solo sigma {w.name}")
        assert abs(r["e_in"] - a["e_in"]) <= 1e-12 * a["e_in"]
        if kw.get("target_unc"):
            assert r["status"] == "GDPM_OK" and r["unc"] <= kw["target_unc"]
            assert r["rounds"] > 10   # more than one super-round


def test_batch_source_modes_equal_solo(gctx):
    """The source modes in a shared batch: Metropolis chains (run to a target
    over several super-rounds, so the chains carry on across rounds), energy
    intervals, a phase space and a plain job side by side; each job's dose
    equals its dose alone (the chain state is the job's own, the interval of a
    history depends on its place in its own round)."""
    ph = I.ellipsoid_phantom(20, 0.5, seed=77)
    plan = I.imrt_plan(ph, n_beams=5, nb=6, seed=78)
    jobs = [
        ("metropolis", I.Source(I.PHOTON, I.triangular_spectrum(), plan, beamlet_sampler=1),
         dict(n_hist=20_000, target_unc=0.06, max_histories=4_000_000)),
        ("intervals", I.Source(I.PHOTON, I.triangular_spectrum(), plan, spectrum_strata=8),
         dict(n_hist=35_001)),
        ("phase_space", I.Source(I.PHOTON, I.mono(1.0), [], phase_space=I.point_phase_space(ph, 5_000, seed=79)),
         dict(n_hist=30_000)),
        ("plain", I.Source(I.ELECTRON, I.mono(9.0), [I.parallel_beam_z(ph, 6.0)]), dict(n_hist=8_000)),
    ]
    handles = []
    for k, (name, src, kw) in enumerate(jobs):
        handles.append((gctx.phantom(ph), gctx.source(src), dict(kw, seed=31 + k, job_id=k, n_batches=10)))
    try:
        res = gctx.run_batch(handles)
        for (name, _, _), (p, s, kw), r in zip(jobs, handles, res):
            a = gctx.run(p, s, **kw)
            assert r["histories"] == a["histories"], name
            assert balance(r) < 1e-6, name
            same_dose(r["dose"], a["dose"], f"batch vs solo {name}")
            if name == "metropolis":   # more than one super-round: chains carried across
                assert r["status"] in ("GDPM_OK", "GDPM_E_NOT_CONVERGED") and r["rounds"] > 10
    finally:
        for p, s, _ in handles:
            p.close()
            s.close()


def test_batch_graphs_equal_direct_launches():
    """The batched form with each iteration replayed from a recorded HIP graph
    (the default) against direct launches: same doses, same events.  A small
    history budget per iteration makes many iterations of the same launch
    configuration, so that recordings are replayed whatever the jobs' event
    counts."""
    jobs = small_jobs(seed=4103)
    res = {}
    for graphs in (0, 1):
        c2 = G.Context(0, opts=f'{{"graphs": {graphs}, "pass_histories": 4000}}', materials=MATS)
        handles = [(c2.phantom(w.phantom), c2.source(w.source), kw) for w, kw in jobs]
        try:
            res[graphs] = c2.run_batch(handles)
        finally:
            for p, s, _ in handles:
                p.close()
                s.close()
            c2.close()
    for (w, kw), a, b in zip(jobs, res[0], res[1]):
        report(f"graphs vs direct {w.name}", histories=(a["histories"], b["histories"]),
               unc=(a["unc"], b["unc"]), rounds=(a["rounds"], b["rounds"]),
               graph_launches=b["graph_launches"])
    # a job's event counters are the engine's running totals when the job
    # finishes, which depend on when the others' work ran; the totals at the
    # end (the largest over the jobs) are the physics of the whole batch
    def totals(rs):
        return {k: max(physics_events(r)[k] for r in rs) for k in physics_events(rs[0]) if k != "histories"}
    assert totals(res[0]) == totals(res[1])
    for (w, _), a, b in zip(jobs, res[0], res[1]):
        assert a["graph_launches"] == 0 and b["graph_launches"] > 0, w.name
        assert a["histories"] == b["histories"], w.name
        same_dose(b["dose"], a["dose"], f"graphs vs direct {w.name}")
        assert balance(b) < 1e-6


@pytest.mark.parametrize("extra", ["", ', "fused_passes": 1', ', "rebin_bins": 8',
                                   ', "rebin_bins": 8, "rebin_space": 1, "fused_passes": 1, "photon_waves": 4'],
                         ids=["default", "fused", "energy_bins", "space_bins_fused"])
def test_accounting_check_finds_nothing(gctx, extra):
    """The diagnostic accounting check (every iteration: live queue records of
    each job against its births less deaths) on the batched form, several jobs
    sharing the queues with re-binning, and on a multi-round target job; with
    both passes in one launch and with bins within a job as well.  Each job's
    dose equals the job run alone with the default settings."""
    jobs = small_jobs(seed=4107)
    c2 = G.Context(0, opts='{"check_accounting": 1, "pass_histories": 3000, "ring_capacity_log2": 21' + extra + '}',
                   materials=MATS)
    handles = [(c2.phantom(w.phantom), c2.source(w.source), kw) for w, kw in jobs]
    try:
        res = c2.run_batch(handles)
    finally:
        for p, s, _ in handles:
            p.close()
            s.close()
        c2.close()
    for (w, kw), r in zip(jobs, res):
        report(f"accounting check {w.name}", mismatches=r["accounting_mismatches"], passes=r["passes"],
               rebinned=r["passes_rebinned"])
        assert r["accounting_mismatches"] == 0 and r["transport_anomalies"] == 0, w.name
        assert balance(r) < 1e-6
        a = solo(gctx, w, kw)
        assert r["histories"] == a["histories"], w.name
        same_dose(r["dose"], a["dose"], f"batch{extra} vs solo {w.name}")


def test_batch_more_jobs_than_slots(gctx):
    """300 tiny jobs: admitted 256 at a time, the rest as slots free up."""
    ph = I.homogeneous((6, 6, 6), (1.0, 1.0, 1.0), I.ID_WATER, 1.0)
    src = I.Source(I.PHOTON, I.mono(1.25), [I.parallel_beam_z(ph, 4.0)])
    p, s = gctx.phantom(ph), gctx.source(src)
    try:
        res = gctx.run_batch([(p, s, dict(seed=5, job_id=k, n_hist=300 + k, n_batches=2))
                              for k in range(300)])
        ref = gctx.run(p, s, seed=5, job_id=299, n_hist=599, n_batches=2)
    finally:
        p.close()
        s.close()
    assert all(r["status"] == "GDPM_OK" for r in res)
    assert [r["histories"] for r in res] == [300 + k for k in range(300)]
    assert max(balance(r) for r in res) < 1e-6
    same_dose(res[-1]["dose"], ref["dose"], "job 299 of 300 vs solo")


def test_autotune_changes_speed_not_results():
    ws = I.batch_jobs(3, seed=4201, side=(32, 40), d=0.5, hist=(2e5, 4e5))
    # iterations of this small batch hold about 1e6 transport events: score them all
    ctx = G.Context(0, opts='{"autotune": 1, "autotune_min_events": 100000, "pass_histories": 30000}',
                    materials=MATS)
    try:
        hs = [(ctx.phantom(w.phantom), ctx.source(w.source),
               dict(seed=3 + k, job_id=k, n_hist=w.n_hist)) for k, w in enumerate(ws)]
        res = ctx.run_batch(hs)
        st = ctx.settings()
        cand, score, kept = ctx.tuning()
        report("autotune", **st, candidates=cand, scores=[f"{x:.3g}" for x in score], kept=kept)
        # the tuner's candidate set; it keeps the best-scored one once every
        # candidate was scored, and the context then runs with it
        assert sorted(cand) == [(8, 1), (8, 16), (12, 1), (12, 16)]
        assert (st["waves_per_cu"], st["rebin_bins"]) in cand
        assert kept >= 0   # every candidate was scored twice and one was kept
        assert all(x > 0 for x in score)
        assert score[kept] == max(score)
        assert (st["waves_per_cu"], st["rebin_bins"]) == cand[kept]
        assert 21 <= st["ring_capacity_log2"] <= 26
        for p, s, _ in hs:
            p.close()
            s.close()
    finally:
        ctx.close()
    ctx2 = G.Context(0, materials=MATS)
    try:
        for k, (w, r) in enumerate(zip(ws, res)):
            a = solo(ctx2, w, dict(seed=3 + k, job_id=k, n_hist=w.n_hist))
            same_dose(r["dose"], a["dose"], f"autotuned batch vs solo {w.name}")
    finally:
        ctx2.close()


def test_server_alone_and_in_the_mix():
    """Job A alone, then job B (longer) with A submitted again while B runs:
    A's dose is the same both times and B's equals B alone."""
    wa = I.water_cube_2mev(30_000)
    wb = I.batch_jobs(1, seed=4301, side=(40, 40), d=0.5, hist=(2e6, 2e6))[0]
    ka = dict(seed=21, job_id=1, n_hist=wa.n_hist)
    kb = dict(seed=22, job_id=2, n_hist=wb.n_hist)
    ctx = G.Context(0, materials=MATS)
    try:
        pa, sa = ctx.phantom(wa.phantom), ctx.source(wa.source)
        pb, sb = ctx.phantom(wb.phantom), ctx.source(wb.source)
        srv = G.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=8)
        try:
            alone = srv.submit(pa, sa, **ka).wait()
            jb = srv.submit(pb, sb, **kb)
            ja = srv.submit(pa, sa, **ka)
            mixed = ja.wait()
            rb = jb.wait()
            info = srv.info()
        finally:
            srv.close()
        solo_b = ctx.run(pb, sb, **kb)   # the server is gone: the context runs again
        for h in (pa, sa, pb, sb):
            h.close()
    finally:
        ctx.close()
    report("server", latency_alone=f"{alone['t_total_s']:.3f}", latency_mixed=f"{mixed['t_total_s']:.3f}",
           **{k: info[k] for k in ("submitted", "finished", "histories")})
    assert info["submitted"] == 3 and info["finished"] == 3
    assert info["histories"] == 2 * wa.n_hist + wb.n_hist
    assert info["high_water_bytes"] > 0 and info["footprint_bytes"] == 0
    same_dose(mixed["dose"], alone["dose"], "server: A in the mix vs alone")
    same_dose(rb["dose"], solo_b["dose"], "server: B vs gdpm_run")
    for r in (alone, mixed, rb):
        assert balance(r) < 1e-6


def test_server_admission_waits_for_memory():
    """A budget that holds one job at a time: the second job is queued until the
    first leaves, and still gets the same dose."""
    w = I.water_cube_2mev(20_000)
    ctx = G.Context(0, materials=MATS)
    try:
        p, s = ctx.phantom(w.phantom), ctx.source(w.source)
        nv = w.phantom.nvox
        one_job = 10 * nv * 8 + 2 * nv * 8 + 64 * 1024
        srv = G.Server(ctx, hbm_budget_bytes=int(1.5 * one_job), max_slots=8)
        try:
            j1 = srv.submit(p, s, seed=31, job_id=1, n_hist=w.n_hist)
            j2 = srv.submit(p, s, seed=32, job_id=2, n_hist=w.n_hist)
            r1, r2 = j1.wait(), j2.wait()
            info = srv.info()
        finally:
            srv.close()
        solo2 = ctx.run(p, s, seed=32, job_id=2, n_hist=w.n_hist)
        p.close()
        s.close()
    finally:
        ctx.close()
    assert info["high_water_bytes"] <= 1.5 * one_job
    same_dose(r2["dose"], solo2["dose"], "server: queued job vs solo")
    assert balance(r1) < 1e-6 and balance(r2) < 1e-6


def test_oldest_first_share_rejected():
    """The oldest-job-first sharing policy can overflow the queues (one job
    takes a whole iteration's history budget); it is refused at creation."""
    with pytest.raises(G.GdpmError) as e:
        G.Context(0, opts='{"share": 0}', materials=MATS)
    assert e.value.status == 1 and "share" in str(e.value)


def test_server_errors():
    w = I.water_cube_2mev(1000)
    ctx = G.Context(0, materials=MATS)
    try:
        p, s = ctx.phantom(w.phantom), ctx.source(w.source)
        with pytest.raises(G.GdpmError) as e:
            G.Server(ctx, hbm_budget_bytes=0)
        assert e.value.status == 1
        srv = G.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=2)
        try:
            with pytest.raises(G.GdpmError) as e:   # the context belongs to the server
                ctx.run(p, s, n_hist=100)
            assert e.value.status == 5
            j = srv.submit(p, s, seed=1, n_hist=2000)
            with pytest.raises(G.GdpmError) as e:   # other cutoffs than the first job
                srv.submit(p, s, seed=1, n_hist=100, ecut_e=0.3)
            assert e.value.status == 1
            assert j.wait()["histories"] == 2000
        finally:
            srv.close()
        p.close()
        s.close()
    finally:
        ctx.close()


def _vs_oracle(r, ph, src, kw, name):
    """A job's result from the batched or served form against the oracle:
    (1) the same job (seed, job_id) on the oracle's streams: the per-voxel
    energies agree to within the histories that leave lockstep (a few per
    cent of the incident energy at most; a job transported with another job's
    phantom, source or key would differ by the whole deposited energy);
    (2) an independent oracle run: the section 3.1 t-test passes in 95-99% of
    the voxels above 10% of D_max."""
    from tests import stats as S
    from tests.gpu_common import oracle_run
    n, nb = kw["n_hist"], kw.get("n_batches", 10)
    assert n % nb == 0
    rho = ph.rho.ravel().astype(np.float64)
    e_g = r["dose"] * rho * (ph.dx * ph.dy * ph.dz) * n
    same = oracle_run(MATS, ph, src, seed=kw["seed"], job_id=kw["job_id"], n_hist=n, n_batches=nb)
    l1 = np.abs(e_g - same["batch_edep"].sum(axis=0)).sum() / same["e_in"]
    indep = oracle_run(MATS, ph, src, seed=kw["seed"] + 1000, job_id=kw["job_id"], n_hist=n, n_batches=nb)
    # air voxels (below 0.1 g/cm^3) are left out of D_max and the region: their
    # dose estimates are dominated by rare local deposits
    rate, nreg = S.pass_rate(r["dose"], r["sigma"], indep["dose"], indep["sigma"], nb, mask=rho >= 0.1)
    report(f"{name} vs oracle", voxel_l1=f"{l1:.3g}", pass_rate=round(rate, 4), voxels=nreg)
    assert abs(r["e_in"] - same["e_in"]) <= 1e-5 * same["e_in"]
    assert l1 < 0.03
    assert nreg >= 500 and 0.95 <= rate <= 0.99


def test_batch_and_served_jobs_match_oracle(gctx):
    """One job of a mixed batch (photons and electrons together) and one job
    served beside another, each compared with the oracle directly."""
    wa = I.water_cube_2mev()
    wb = I.slab_electron(n=50, d=0.6)
    ct = I.ct_phantom((48, 48, 24), (1.0, 1.0, 1.25))
    src_c = I.Source(I.PHOTON, I.triangular_spectrum(), I.imrt_plan(ct, nb=10))
    ka = dict(seed=61, job_id=7, n_hist=200_000)
    kb = dict(seed=62, job_id=8, n_hist=20_000)
    kc = dict(seed=63, job_id=9, n_hist=150_000)
    handles = [(gctx.phantom(wa.phantom), gctx.source(wa.source), ka),
               (gctx.phantom(wb.phantom), gctx.source(wb.source), kb),
               (gctx.phantom(ct), gctx.source(src_c), kc)]
    try:
        res = gctx.run_batch(handles)
    finally:
        for p, s, _ in handles:
            p.close()
            s.close()
    _vs_oracle(res[0], wa.phantom, wa.source, ka, "batched water")
    _vs_oracle(res[1], wb.phantom, wb.source, kb, "batched slab electrons")
    ctx = G.Context(0, materials=MATS)
    try:
        pc, sc = ctx.phantom(ct), ctx.source(src_c)
        pa, sa = ctx.phantom(wa.phantom), ctx.source(wa.source)
        srv = G.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=8)
        try:
            ja = srv.submit(pa, sa, **dict(ka, job_id=17))
            jc = srv.submit(pc, sc, **kc)
            rc = jc.wait()
            ja.wait()
        finally:
            srv.close()
        for h in (pc, sc, pa, sa):
            h.close()
    finally:
        ctx.close()
    _vs_oracle(rc, ct, src_c, kc, "served CT")


@pytest.mark.parametrize("mode", [1, 2])
def test_server_admit_draining(mode):
    """Admission only while every running job drains (mode 1: any super-round,
    2: its last one; the second job runs to a target, so it has two): jobs
    still finish with the dose they have alone."""
    wa = I.water_cube_2mev(400_000)
    wb = I.batch_jobs(1, seed=4302, side=(40, 40), d=0.5, hist=(1.5e6, 1.5e6))[0]
    ctx = G.Context(0, opts=f'{{"admit_draining": {mode}, "issue_order": 2}}', materials=MATS)
    try:
        pa, sa = ctx.phantom(wa.phantom), ctx.source(wa.source)
        pb, sb = ctx.phantom(wb.phantom), ctx.source(wb.source)
        kws = [(pa, sa, dict(seed=31 + k, job_id=k, n_hist=wa.n_hist)) if k % 2 == 0 else
               (pb, sb, dict(seed=31 + k, job_id=k, n_hist=200_000, target_unc=0.05,
                             max_histories=20_000_000)) for k in range(4)]
        srv = G.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=8)
        try:
            jobs = [srv.submit(p, s, **kw) for p, s, kw in kws]
            res = [j.wait() for j in jobs]
            info = srv.info()
        finally:
            srv.close()
        alone = [ctx.run(p, s, **kw) for p, s, kw in kws]
        for h in (pa, sa, pb, sb):
            h.close()
    finally:
        ctx.close()
    assert info["submitted"] == 4 and info["finished"] == 4
    for k, (r, a) in enumerate(zip(res, alone)):
        same_dose(r["dose"], a["dose"], f"admit_draining: job {k} served vs alone")
        assert balance(r) < 1e-6


def test_admit_draining_validated():
    with pytest.raises(G.GdpmError):
        G.Context(0, opts='{"admit_draining": 3}', materials=MATS)
