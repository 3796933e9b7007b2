"""The benchmark's profile arithmetic on synthetic counter files (no GPU):
the event-cost fit recovers known per-event costs and the per-history cost of
the CT pair, and the traffic summary applies the copy calibration."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KNAMES = {"k_photon": "void gdpm::k_photon<true, true>(gdpm::Ctl*, gdpm::Tables, gdpm::RunDev)",
          "k_electron": "void gdpm::k_electron<true, true>(gdpm::Ctl*, gdpm::Tables, gdpm::RunDev)"}


def _runs(rng, n):
    runs = []
    for i in range(n):
        h = 1_000_000 if i < 2 else int(rng.integers(50_000, 500_000))
        if i == 1:
            h = 2_000_000
        s = h / 1e6
        runs.append({"name": "ct_imrt" if i < 2 else f"w{i}", "histories": h,
                     "passes_photon": 4 if i < 2 else int(rng.integers(1, 6)),
                     "passes_electron": 4 if i < 2 else int(rng.integers(1, 6)),
                     "events": {"flights": int(rng.uniform(2, 9) * h), "esteps": int(rng.uniform(1, 9) * h),
                                "real": 0, "hard_cand": 0, "hard": 0, "deposits": 0, "pushes": 0,
                                "histories": h},
                     "interactions": {k: int(rng.uniform(0.01, 2) * h) for k in
                                      ("compton", "photo", "pair", "moller", "brems")},
                     "records_loaded": [int(rng.uniform(1, 3) * h), int(rng.uniform(1, 3) * h)],
                     "records_stored": [int(rng.uniform(0.5, 1.5) * h), int(rng.uniform(0.1, 0.5) * h)],
                     "records_requeued": [0, 0], "deposits": [int(rng.uniform(0, 1) * h), int(rng.uniform(1, 8) * h)]})
        del s
    return runs


def test_event_cost_fit_recovers_costs(tmp_path, capsys):
    rng = np.random.default_rng(7)
    runs = _runs(rng, 14)
    true = {k: rng.uniform(20, 600, len(bench.EVENT_TERMS[k])) for k in KNAMES}
    rows, did = [], 0
    for r in runs:
        for k, passes in (("k_photon", "passes_photon"), ("k_electron", "passes_electron")):
            x = np.array(bench.event_regressors(r, k))
            per = float(true[k][1:] @ x) / r[passes]
            for _ in range(r[passes]):
                did += 1
                rows.append((did, KNAMES[k], "SQ_WAVES", 3072.0))
                rows.append((did, KNAMES[k], "SQ_INSTS_VALU", per + true[k][0] * 3072.0))
            did += 1
            rows.append((did, "void gdpm::k_source(...)", "SQ_INSTS_VALU", 5.0))
            rows.append((did, "void gdpm::k_source(...)", "SQ_WAVES", 1.0))
    csv = tmp_path / "c.csv"
    with open(csv, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, n, c, v in rows:
            f.write(f'{d},"{n}",{c},{float(v)!r}\n')
    js = tmp_path / "r.json"
    js.write_text(json.dumps({"event_cost_runs": runs}) + "\n")
    bench.event_cost_fit(str(csv), str(js))
    out = capsys.readouterr().out
    kv = dict(l.split(": ", 1) for l in out.splitlines() if ": " in l and not l.startswith(" "))
    for k in KNAMES:
        got = [float(kv[f"{k}_cost_{t}"]) for t in bench.EVENT_TERMS[k]]
        np.testing.assert_allclose(got[1:], true[k][1:], atol=2e-3)  # printed to 3 decimals
        # per history: the instruction difference of the two CT runs over 1e6
        a, b = runs[0], runs[1]
        xa, xb = np.array(bench.event_regressors(a, k)), np.array(bench.event_regressors(b, k))
        want = float(true[k][1:] @ (xb - xa)) / 1e6
        assert abs(float(kv[f"{k}_valu_per_history"]) - want) < 0.01


def test_traffic_summary_scales_by_the_copy(tmp_path, capsys):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    f.write_text(hdr + '1,"__amd_rocclr_copyBuffer",FETCH_SIZE,524288\n'
                 '2,"void gdpm::k_photon<true, false>(x)",FETCH_SIZE,1000\n'
                 '3,"void gdpm::k_photon<true, false>(x)",FETCH_SIZE,3000\n')
    w.write_text(hdr + '1,"__amd_rocclr_copyBuffer",WRITE_SIZE,1048576\n'
                 '2,"void gdpm::k_photon<true, false>(x)",WRITE_SIZE,500\n'
                 '3,"void gdpm::k_photon<true, false>(x)",WRITE_SIZE,1500\n')
    bench.summarize_traffic(str(f), str(w), 1024)
    out = capsys.readouterr().out
    kv = dict(l.split(": ", 1) for l in out.splitlines() if ": " in l and not l.startswith(" "))
    # fetch scaled by 2 (the copy read 1 GiB, the counter said 0.5), write by 1
    assert abs(float(kv["k_photon_hbm_bytes_per_launch"]) - (2000 * 2 + 1000) * 1024) < 1e-3 * 5e6
