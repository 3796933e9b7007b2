"""The allocation-free entry point (gdpm_run_noalloc) against gdpm_run_async.

gdpm_run_noalloc runs the same engine and kernels with its queues, control
blocks and batch tallies in the library's static scratch array.  A particle's
random stream depends only on (seed, job, history, path), so the same job must
give the same physics events and the same dose and standard error as through
gdpm_run_async, up to the order of the FP64 tally additions (relative 1e-12).
Two calls in a row, the second on a smaller input, check that the scratch
array is cleared between calls; sizes beyond the array's limit and table sets
that are not resident are rejected with GDPM_E_INVALID."""
import numpy as np
import pytest

from paper_1107_3355_amd import gdpm as G
from paper_1107_3355_amd import inputs as I
from tests.gpu_common import balance, physics_events, report

pytestmark = pytest.mark.gpu
MATS = I.MATERIALS


class _DeviceArrays:
    """Caller-owned device outputs (hipMalloc through the HIP runtime the
    library uses), zeroed before each call."""

    def __init__(self, nv, n=2):
        import ctypes as C
        self.C = C
        self.hip = C.CDLL("libamdhip64.so")
        self.nbytes = C.c_size_t(nv * 8)
        self.nv = nv
        self.bufs = [C.c_void_p() for _ in range(n)]
        for b in self.bufs:
            assert self.hip.hipMalloc(C.byref(b), self.nbytes) == 0

    def zero(self):
        for b in self.bufs:
            assert self.hip.hipMemset(b, 0, self.nbytes) == 0
        assert self.hip.hipDeviceSynchronize() == 0

    def ptrs(self):
        return [b.value for b in self.bufs]

    def read(self, i):
        out = np.empty(self.nv)
        assert self.hip.hipDeviceSynchronize() == 0
        assert self.hip.hipMemcpy(out.ctypes.data_as(self.C.c_void_p), self.bufs[i], self.nbytes, 2) == 0
        return out

    def close(self):
        for b in self.bufs:
            if b.value:
                self.hip.hipFree(b)
        self.bufs = []


def _device_run(fn, ctx, ph, src, **kw):
    arr = _DeviceArrays(ph.desc.nvox)
    try:
        arr.zero()
        st = fn(ph, src, *arr.ptrs(), **kw)
        st["dose"], st["sigma"] = arr.read(0), arr.read(1)
    finally:
        arr.close()
    return st


def _same(a, b, what):
    for k in ("dose", "sigma"):
        scale = max(np.abs(a[k]).max(), 1e-300)
        err = np.abs(a[k] - b[k]).max() / scale
        report(f"noalloc {what} {k}", max_rel_diff=f"{err:.2e}")
        assert err < 1e-12, (what, k)
    assert physics_events(a) == physics_events(b), what
    assert a["histories"] == b["histories"]
    assert balance(a) < 1e-6


def test_noalloc_equals_run_async_twice_smaller_second():
    big = I.slab_photon(n=50, d=0.6)                       # 125,000 voxels, photons
    small = I.water_cube_2mev()                           # 32^3 voxels
    ctx = G.Context(0, materials=MATS)
    try:
        cases = [("slab50 photon", big.phantom, big.source, dict(seed=41, n_hist=120_000)),
                 ("water32 2 MeV", small.phantom, small.source, dict(seed=42, n_hist=30_000, n_batches=4))]
        for name, ph_d, src_d, kw in cases:
            ph, src = ctx.phantom(ph_d), ctx.source(src_d)
            try:
                ref = _device_run(ctx.run_async, ctx, ph, src, **kw)
                got = _device_run(ctx.run_noalloc, ctx, ph, src, **kw)
            finally:
                ph.close()
                src.close()
            assert got["graph_launches"] == 0 and got["graphs_recorded"] == 0
            _same(got, ref, name)
    finally:
        ctx.close()


def test_noalloc_electrons_and_target_mode():
    """Electrons (the other source queue) and a run to a target uncertainty
    over several super-rounds, through the scratch memory."""
    w = I.slab_electron(n=50, d=0.6)
    ctx = G.Context(0, materials=MATS)
    try:
        ph, src = ctx.phantom(w.phantom), ctx.source(w.source)
        try:
            for kw in (dict(seed=43, n_hist=15_000),
                       dict(seed=44, n_hist=4_000, target_unc=0.04, max_histories=2_000_000)):
                ref = _device_run(ctx.run_async, ctx, ph, src, **kw)
                got = _device_run(ctx.run_noalloc, ctx, ph, src, **kw)
                _same(got, ref, f"slab50 electron {kw}")
        finally:
            ph.close()
            src.close()
    finally:
        ctx.close()


def test_noalloc_limits():
    ctx = G.Context(0, materials=MATS)
    arr = None
    try:
        # 10 batches x 3,375,000 voxels of FP64 tallies: above the 255 MiB of the scratch array
        ph_d = I.homogeneous((150, 150, 150), (0.1, 0.1, 0.1), I.ID_WATER, 1.0)
        src_d = I.Source(I.PHOTON, I.mono(1.0), [I.parallel_beam_z(ph_d, 5.0)])
        ph, src = ctx.phantom(ph_d), ctx.source(src_d)
        arr = _DeviceArrays(ph_d.nvox)
        d, s = arr.ptrs()
        with pytest.raises(G.GdpmError) as e:
            ctx.run_noalloc(ph, src, d, s, n_hist=1000, n_batches=10)
        assert e.value.status == 1 and "scratch" in str(e.value)
        # 9 batches fit (30,375,000 doubles)
        r = ctx.run_noalloc(ph, src, d, s, n_hist=2000, n_batches=9, seed=3)
        assert r["histories"] == 2000 and balance(r) < 1e-6
        # other absorption energies: their tables are not resident yet
        with pytest.raises(G.GdpmError) as e:
            ctx.run_noalloc(ph, src, d, s, n_hist=1000, n_batches=2, ecut_e=0.3)
        assert e.value.status == 1 and "resident" in str(e.value)
        ctx.run_async(ph, src, d, s, n_hist=100, n_batches=2, ecut_e=0.3)
        r = ctx.run_noalloc(ph, src, d, s, n_hist=1000, n_batches=2, ecut_e=0.3)
        assert r["histories"] == 1000
        ph.close()
        src.close()
    finally:
        if arr is not None:
            arr.close()
        ctx.close()
