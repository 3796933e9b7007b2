"""Host-side logic without a GPU: argument checks of the batched and serving
entry points, and the synthetic workloads of the batched and serving forms
(sizes, history counts and mixes as the workloads define them)."""
import ctypes as C

import numpy as np
import pytest

from paper_1107_3355_amd import gdpm as G
from paper_1107_3355_amd import inputs as I


def test_batch_and_server_entry_points_reject_null():
    L = G.lib()
    assert L.gdpm_run_batch(None, 1, None, None, None) == 1
    out = C.c_void_p()
    assert L.gdpm_server_create(None, 1 << 30, 4, C.byref(out)) == 1
    assert L.gdpm_server_submit(None, None, C.byref(out)) == 1
    assert L.gdpm_server_info_get(None, None) == 1
    assert L.gdpm_server_destroy(None) == 1
    assert L.gdpm_context_settings(None, (C.c_int * 5)()) == 1
    assert L.gdpm_job_wait(None, None) == 1
    assert b"NULL" in L.gdpm_last_error() or L.gdpm_last_error()


def test_job_desc_layout_matches_header():
    # phantom, source (pointers), run parameters, two host pointers
    assert G.JobDesc.params.offset == 16
    assert G.JobDesc.dose.offset == 16 + C.sizeof(G.RunParams)
    assert C.sizeof(G.JobDesc) == 16 + C.sizeof(G.RunParams) + 16


def test_batch_jobs_follow_the_batched_form():
    ws = I.batch_jobs(64, side=(48, 256), hist=(1e5, 1e7))
    sides = np.array([w.phantom.nx for w in ws])
    hist = np.array([w.n_hist for w in ws])
    assert all(w.phantom.nx == w.phantom.ny == w.phantom.nz for w in ws)
    assert sides.min() >= 48 and sides.max() <= 256
    assert hist.min() >= 1e5 and hist.max() <= 1e7
    # log-uniform histories: the median sits near the geometric mean 1e6
    assert 2e5 < np.median(hist) < 5e6
    kinds = [w.source.spectrum.kind for w in ws]
    assert 16 <= sum(1 for k in kinds if k == 1) <= 48   # about half use the spectrum
    electrons = sum(1 for w in ws if w.source.particle == I.ELECTRON)
    assert 4 <= electrons <= 28
    # a different seed gives different jobs, the same seed the same ones
    assert [w.n_hist for w in I.batch_jobs(8, seed=9)] == [w.n_hist for w in I.batch_jobs(8, seed=9)]
    assert [w.n_hist for w in I.batch_jobs(8, seed=9)] != [w.n_hist for w in I.batch_jobs(8, seed=10)]


def test_serving_requests_are_a_poisson_stream():
    ct = I.homogeneous((8, 8, 4), (0.2, 0.2, 0.25), I.ID_WATER, 1.0)
    small = I.homogeneous((4, 4, 2), (0.4, 0.4, 0.5), I.ID_WATER, 1.0)
    reqs = I.serving_requests(duration_s=300.0, rate=2.0, ct=ct, small_ct=small)
    t = np.array([r[0] for r in reqs])
    assert np.all(np.diff(t) > 0) and t[-1] < 300.0
    # 600 expected arrivals: Poisson count within 4 sigma
    assert abs(len(reqs) - 600) < 4 * np.sqrt(600)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.5) < 0.06
    vmat = [w for _, w in reqs if w.phantom is ct]
    assert abs(len(vmat) / len(reqs) - 0.5) < 0.1
    assert all(len(w.source.beams) == 180 for w in vmat)
    assert {w.target_unc for _, w in reqs} == {0.01, 0.02}
