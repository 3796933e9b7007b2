"""Helpers shared by the GPU tests: run a workload on the GPU and on the
oracle, and compare them per history (same Philox streams) or statistically
(independent streams, section 3.1 t-test)."""
import os

import numpy as np

import oracle
from tests import stats as S

ORACLE_THREADS = int(os.environ.get("GDPM_ORACLE_THREADS", "16"))


def gpu_run(ctx, ph, src, **kw):
    p = ctx.phantom(ph)
    s = ctx.source(src)
    try:
        return ctx.run(p, s, **kw)
    finally:
        p.close()
        s.close()


def oracle_run(materials, ph, src, **kw):
    kw.setdefault("n_threads", ORACLE_THREADS)
    return oracle.run(materials, ph, src, **kw)


def balance(r):
    # a sound run never needs its particle accounting repaired
    assert r.get("accounting_repairs", 0) == 0, r.get("accounting_gap")
    assert r.get("transport_anomalies", 0) == 0
    return abs(r["e_dep"] + r["e_esc"] - r["e_in"]) / r["e_in"]


def lockstep_fraction(hg, ho, e_in, rel=1e-4):
    """Fraction of histories whose deposited and escaped energies agree."""
    tol = rel * e_in + 1e-6
    ok = (np.abs(hg[:, 0] - ho[:, 0]) <= tol) & (np.abs(hg[:, 1] - ho[:, 1]) <= tol)
    return float(ok.mean())


def report(name, **vals):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v}" for k, v in vals.items()), flush=True)


def statistical(g, o, n_batches, frac=0.1):
    rate, nreg = S.pass_rate(g["dose"], g["sigma"], o["dose"], o["sigma"], n_batches, frac)
    dmax = max(g["dose"].max(), o["dose"].max())
    region = np.maximum(g["dose"], o["dose"]) > frac * dmax
    nb_hist = None
    return rate, nreg, region


def physics_events(r):
    """Event counts that follow from the physics alone.  'deposits' counts the
    FP64 tally additions, which depend on scheduling: a lane merges deposits of
    consecutive steps in one voxel, and a particle handed to the next pass or a
    wavefront changing jobs flushes its sum early."""
    return {k: v for k, v in r["events"].items() if k != "deposits"}
