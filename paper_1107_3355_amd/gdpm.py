"""ctypes binding of libgdpm (include/gdpm.h): argument marshalling only.

Every step of the transport runs in the library's HIP kernels; this module only
converts numpy arrays and the input descriptions of ``inputs`` into the C
structures and back.  It raises if the library is not built or the call fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgdpm.so")
_lib = None

NO_COMPTON, NO_PHOTO, NO_PAIR, NO_MS, NO_MOLLER, NO_BREMS, KERMA = 1, 2, 4, 8, 16, 32, 64
EV_NAMES = ("flights", "real", "esteps", "hard_cand", "hard", "deposits", "pushes", "histories")
INTERACTION_NAMES = ("compton", "photo", "pair", "moller", "brems")
STATUS = {0: "GDPM_OK", 1: "GDPM_E_INVALID", 2: "GDPM_E_NOMEM", 3: "GDPM_E_DEVICE",
          4: "GDPM_E_OVERFLOW", 5: "GDPM_E_BUSY", 6: "GDPM_E_NOT_CONVERGED"}
EXPORTS = ("gdpm_context_create", "gdpm_context_destroy", "gdpm_last_error", "gdpm_set_materials",
           "gdpm_phantom_create", "gdpm_phantom_destroy", "gdpm_source_create",
           "gdpm_source_destroy", "gdpm_run", "gdpm_run_async", "gdpm_job_wait",
           "gdpm_job_release", "gdpm_tables_host", "gdpm_test_philox", "gdpm_test_sample",
           "gdpm_test_atomic_rate", "gdpm_test_source", "gdpm_test_lookup", "gdpm_run_batch", "gdpm_context_settings",
           "gdpm_server_create", "gdpm_server_submit", "gdpm_server_info_get",
           "gdpm_server_destroy", "gdpm_run_noalloc", "gdpm_context_tuning")


class GdpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Material(C.Structure):
    _fields_ = [("z", C.c_double), ("z_over_a", C.c_double), ("i_ev", C.c_double)]


class Spectrum(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_pts", C.c_int), ("e_mev", C.POINTER(C.c_double)),
                ("pdf", C.POINTER(C.c_double)), ("e_mono", C.c_double)]


class Beam(C.Structure):
    _fields_ = [("iso_cm", C.c_double * 3), ("dir", C.c_double * 3), ("e1", C.c_double * 3),
                ("sad_cm", C.c_double), ("nbx", C.c_int), ("nby", C.c_int),
                ("bw_cm", C.c_double), ("bh_cm", C.c_double), ("intensity", C.POINTER(C.c_float))]


class SourceDesc(C.Structure):
    _fields_ = [("particle", C.c_int), ("spectrum", Spectrum), ("n_beams", C.c_int),
                ("beams", C.POINTER(Beam)), ("beamlet_sampler", C.c_int),
                ("spectrum_strata", C.c_int), ("n_phase_space", C.c_uint64),
                ("phase_space", C.POINTER(C.c_float)), ("strata_shape", C.c_int)]


class RunParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("job_id", C.c_uint32), ("n_histories", C.c_uint64),
                ("target_unc", C.c_double), ("n_batches", C.c_int),
                ("ecut_photon_mev", C.c_double), ("ecut_electron_mev", C.c_double),
                ("max_histories", C.c_uint64), ("flags", C.c_uint32),
                ("round_size", C.c_uint64), ("hist0", C.c_uint64),
                ("stat_min_density", C.c_double), ("split_log2", C.c_int)]


class RunStats(C.Structure):
    _fields_ = [("histories", C.c_uint64), ("e_in", C.c_double), ("e_dep", C.c_double),
                ("e_esc", C.c_double), ("unc_mean_over_dmax", C.c_double), ("dmax", C.c_double),
                ("t_total_s", C.c_double), ("t_kernel_s", C.c_double),
                ("t_photon_s", C.c_double), ("t_electron_s", C.c_double),
                ("events", C.c_uint64 * 8), ("passes", C.c_uint32), ("rounds", C.c_uint32),
                ("passes_photon", C.c_uint32), ("passes_electron", C.c_uint32),
                ("records_loaded", C.c_uint64 * 2), ("records_stored", C.c_uint64 * 2),
                ("deposits", C.c_uint64 * 2), ("accounting_repairs", C.c_uint32),
                ("accounting_gap", C.c_int64), ("transport_anomalies", C.c_uint64),
                ("graph_launches", C.c_uint32), ("graphs_recorded", C.c_uint32),
                ("accounting_mismatches", C.c_uint32), ("interactions", C.c_uint64 * 5),
                ("records_requeued", C.c_uint64 * 2), ("passes_rebinned", C.c_uint32)]


class JobDesc(C.Structure):
    _fields_ = [("phantom", C.c_void_p), ("source", C.c_void_p), ("params", RunParams),
                ("dose", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double))]


class ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("finished", C.c_uint64), ("running", C.c_uint64),
                ("queued", C.c_uint64), ("histories", C.c_uint64),
                ("footprint_bytes", C.c_double), ("high_water_bytes", C.c_double),
                ("resident_bytes", C.c_double)]


def lib():
    """Load libgdpm.so (built in-tree by build.py); raises when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_1107_3355_amd/build.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, dp, fp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_float)
        u32p = C.POINTER(C.c_uint32)
        sig = {
            "gdpm_context_create": [C.c_int, C.c_char_p, C.POINTER(vp)],
            "gdpm_context_destroy": [vp],
            "gdpm_set_materials": [vp, C.POINTER(Material), C.c_int, C.c_int],
            "gdpm_phantom_create": [vp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                    C.c_double, C.POINTER(C.c_uint8), fp, C.POINTER(vp)],
            "gdpm_phantom_destroy": [vp],
            "gdpm_source_create": [vp, C.POINTER(SourceDesc), C.POINTER(vp)],
            "gdpm_source_destroy": [vp],
            "gdpm_run": [vp, vp, vp, C.POINTER(RunParams), dp, dp, dp, dp, C.POINTER(RunStats)],
            "gdpm_run_async": [vp, vp, vp, C.POINTER(RunParams), vp, vp, vp, C.POINTER(vp)],
            "gdpm_run_noalloc": [vp, vp, vp, C.POINTER(RunParams), vp, vp, vp, C.POINTER(RunStats)],
            "gdpm_job_wait": [vp, C.POINTER(RunStats)],
            "gdpm_job_release": [vp],
            "gdpm_tables_host": [C.POINTER(Material), C.c_int, C.c_int, C.c_double, C.c_double,
                                 C.c_uint32, C.c_int, fp, C.c_size_t, C.POINTER(C.c_size_t), dp],
            "gdpm_test_philox": [vp, u32p, u32p, u32p, C.c_int],
            "gdpm_test_atomic_rate": [vp, C.c_uint64, C.POINTER(C.c_double)],
            "gdpm_test_sample": [vp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_uint64,
                                 C.c_int, fp, fp],
            "gdpm_test_source": [vp, vp, vp, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, fp],
            "gdpm_test_lookup": [vp, C.c_double, C.c_double, C.c_uint32, C.c_int, C.c_int, fp, fp,
                                 C.c_int],
            "gdpm_run_batch": [vp, C.c_int, C.POINTER(JobDesc), C.POINTER(RunStats),
                               C.POINTER(C.c_int)],
            "gdpm_context_settings": [vp, C.POINTER(C.c_int)],
            "gdpm_context_tuning": [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), dp,
                                    C.POINTER(C.c_int)],
            "gdpm_server_create": [vp, C.c_uint64, C.c_int, C.POINTER(vp)],
            "gdpm_server_submit": [vp, C.POINTER(JobDesc), C.POINTER(vp)],
            "gdpm_server_info_get": [vp, C.POINTER(ServerInfo)],
            "gdpm_server_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.gdpm_last_error.argtypes = []
        L.gdpm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st):
    if st != 0 and st != 6:
        raise GdpmError(st, lib().gdpm_last_error().decode())
    return st


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _fp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))


def _materials(mats):
    return (Material * len(mats))(*[Material(m.z, m.z_over_a, m.i_ev) for m in mats])


def tables_host(materials, which, n_grid=1024, ecut_g=0.05, ecut_e=0.2, flags=0):
    """Interpolation tables as built by the library (host only, no GPU needed)."""
    L = lib()
    m = _materials(materials)
    n = C.c_size_t()
    g = (C.c_double * 4)()
    _check(L.gdpm_tables_host(m, len(materials), n_grid, ecut_g, ecut_e, flags, which, None, 0,
                              C.byref(n), g))
    out = np.empty(n.value, dtype=np.float32)
    _check(L.gdpm_tables_host(m, len(materials), n_grid, ecut_g, ecut_e, flags, which, _fp(out),
                              n.value, C.byref(n), g))
    return out, tuple(g)


class Phantom:
    def __init__(self, ctx, ph):
        self.ctx = ctx
        self.desc = ph
        self.handle = C.c_void_p()
        mat = np.ascontiguousarray(ph.mat, dtype=np.uint8)
        rho = np.ascontiguousarray(ph.rho, dtype=np.float32)
        _check(lib().gdpm_phantom_create(ctx.handle, ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz,
                                         mat.ctypes.data_as(C.POINTER(C.c_uint8)), _fp(rho),
                                         C.byref(self.handle)))

    def close(self):
        if self.handle:
            lib().gdpm_phantom_destroy(self.handle)
            self.handle = C.c_void_p()


class Source:
    def __init__(self, ctx, src):
        self.ctx = ctx
        self.desc = src
        keep = []
        beams = (Beam * len(src.beams))()
        for i, b in enumerate(src.beams):
            beams[i].iso_cm[:] = list(map(float, b.iso))
            beams[i].dir[:] = list(map(float, b.dir))
            beams[i].e1[:] = list(map(float, b.e1))
            beams[i].sad_cm = b.sad
            beams[i].nbx, beams[i].nby = b.nbx, b.nby
            beams[i].bw_cm, beams[i].bh_cm = b.bw, b.bh
            if b.intensity is not None:
                f = np.ascontiguousarray(b.intensity, dtype=np.float32).ravel()
                keep.append(f)
                beams[i].intensity = _fp(f)
        sp = src.spectrum
        spec = Spectrum(sp.kind, 0, None, None, sp.e_mono)
        if sp.kind == 1:
            e = np.ascontiguousarray(sp.e, dtype=np.float64)
            p = np.ascontiguousarray(sp.p, dtype=np.float64)
            keep += [e, p]
            spec.n_pts = len(e)
            spec.e_mev, spec.pdf = _dp(e), _dp(p)
        d = SourceDesc(src.particle, spec, len(src.beams), beams, getattr(src, "beamlet_sampler", 0),
                       getattr(src, "spectrum_strata", 0))
        d.strata_shape = getattr(src, "strata_shape", 0)
        ps = getattr(src, "phase_space", None)
        if ps is not None:
            ps = np.ascontiguousarray(ps, dtype=np.float32).reshape(-1, 7)
            keep.append(ps)
            d.n_phase_space = len(ps)
            d.phase_space = _fp(ps)
        self.handle = C.c_void_p()
        _check(lib().gdpm_source_create(ctx.handle, C.byref(d), C.byref(self.handle)))

    def close(self):
        if self.handle:
            lib().gdpm_source_destroy(self.handle)
            self.handle = C.c_void_p()


def _stats_dict(st):
    return {"histories": int(st.histories), "e_in": st.e_in, "e_dep": st.e_dep, "e_esc": st.e_esc,
            "unc": st.unc_mean_over_dmax, "dmax": st.dmax, "t_total_s": st.t_total_s,
            "t_kernel_s": st.t_kernel_s, "t_photon_s": st.t_photon_s,
            "t_electron_s": st.t_electron_s, "passes": int(st.passes), "rounds": int(st.rounds),
            "passes_photon": int(st.passes_photon), "passes_electron": int(st.passes_electron),
            "events": {k: int(st.events[i]) for i, k in enumerate(EV_NAMES)},
            "records_loaded": [int(v) for v in st.records_loaded],
            "records_stored": [int(v) for v in st.records_stored],
            "deposits": [int(v) for v in st.deposits],
            "accounting_repairs": int(st.accounting_repairs),
            "accounting_gap": int(st.accounting_gap),
            "transport_anomalies": int(st.transport_anomalies),
            "graph_launches": int(st.graph_launches), "graphs_recorded": int(st.graphs_recorded),
            "accounting_mismatches": int(st.accounting_mismatches),
            "interactions": {k: int(st.interactions[i]) for i, k in enumerate(INTERACTION_NAMES)},
            "records_requeued": [int(v) for v in st.records_requeued],
            "passes_rebinned": int(st.passes_rebinned)}


class Context:
    """A libgdpm context on one HIP device."""

    def __init__(self, device: int = 0, opts: Optional[str] = None, materials=None, n_grid=1024):
        self.handle = C.c_void_p()
        _check(lib().gdpm_context_create(device, opts.encode() if opts else None,
                                         C.byref(self.handle)))
        if materials is not None:
            self.set_materials(materials, n_grid)

    def set_materials(self, materials, n_grid=1024):
        self.materials = list(materials)
        _check(lib().gdpm_set_materials(self.handle, _materials(materials), len(materials), n_grid))

    def phantom(self, ph) -> Phantom:
        return Phantom(self, ph)

    def source(self, src) -> Source:
        return Source(self, src)

    def settings(self):
        """Launch settings in use (after any autotuning)."""
        a = (C.c_int * 5)()
        _check(lib().gdpm_context_settings(self.handle, a))
        return dict(zip(("waves_per_cu", "rebin_bins", "ring_capacity_log2", "pass_histories",
                         "autotune"), list(a)))

    def tuning(self):
        """The autotuner's record: candidates (waves_per_cu, rebin_bins), their
        mean scores (events per kernel second) and the index kept (-1: undecided)."""
        n, kept = C.c_int(), C.c_int()
        cand = (C.c_int * 128)()
        score = (C.c_double * 64)()
        _check(lib().gdpm_context_tuning(self.handle, 64, C.byref(n), cand, score, C.byref(kept)))
        return ([(cand[2 * i], cand[2 * i + 1]) for i in range(n.value)],
                [score[i] for i in range(n.value)], kept.value)

    def run_batch(self, jobs, want_dose=True):
        """Run several jobs together.  jobs: sequence of (phantom, source, params dict);
        params take the keyword arguments of run().  Returns one result dict per job."""
        n = len(jobs)
        descs = (JobDesc * n)()
        outs = []
        for i, (ph, src, kw) in enumerate(jobs):
            prm = _params(kw)
            nv = ph.desc.nvox
            dose = np.zeros(nv) if want_dose else None
            sigma = np.zeros(nv) if want_dose else None
            descs[i] = JobDesc(ph.handle, src.handle, prm, _dp(dose), _dp(sigma))
            outs.append((dose, sigma))
        stats = (RunStats * n)()
        status = (C.c_int * n)()
        _check(lib().gdpm_run_batch(self.handle, n, descs, stats, status))
        res = []
        for i in range(n):
            r = _stats_dict(stats[i])
            r["status"] = STATUS[status[i]]
            r["dose"], r["sigma"] = outs[i]
            res.append(r)
        return res

    def run(self, phantom: Phantom, source: Source, *, seed=1, n_hist=1000, n_batches=10,
            round_size=0, hist0=0, job_id=0, ecut_g=0.05, ecut_e=0.2, flags=0, target_unc=0.0,
            max_histories=0, stat_min_density=0.0, want_batches=False, want_hist=False,
            want_dose=True, split_log2=0):
        nv = phantom.desc.nvox
        prm = RunParams(seed, job_id, n_hist, target_unc, n_batches, ecut_g, ecut_e,
                        max_histories, flags, round_size, hist0, stat_min_density, split_log2)
        dose = np.zeros(nv) if want_dose else None
        sigma = np.zeros(nv) if want_dose else None
        batch = np.zeros((n_batches, nv)) if want_batches else None
        hist = np.zeros((n_hist, 2)) if want_hist else None
        st = RunStats()
        rc = _check(lib().gdpm_run(self.handle, phantom.handle, source.handle, C.byref(prm),
                                   _dp(dose), _dp(sigma), _dp(batch), _dp(hist), C.byref(st)))
        out = _stats_dict(st)
        out["status"] = STATUS[rc]
        out["dose"], out["sigma"] = dose, sigma
        if want_batches:
            out["batch_edep"] = batch
        if want_hist:
            out["hist"] = hist
        return out

    def run_async(self, phantom: Phantom, source: Source, d_dose: int, d_sigma: int,
                  stream: int = 0, **kw):
        """Device outputs (e.g. torch tensors' data_ptr()); returns run statistics."""
        prm = RunParams(kw.get("seed", 1), kw.get("job_id", 0), kw.get("n_hist", 1000),
                        kw.get("target_unc", 0.0), kw.get("n_batches", 10),
                        kw.get("ecut_g", 0.05), kw.get("ecut_e", 0.2),
                        kw.get("max_histories", 0), kw.get("flags", 0),
                        kw.get("round_size", 0), kw.get("hist0", 0),
                        kw.get("stat_min_density", 0.0), kw.get("split_log2", 0))
        job = C.c_void_p()
        _check(lib().gdpm_run_async(self.handle, phantom.handle, source.handle, C.byref(prm),
                                    C.c_void_p(d_dose), C.c_void_p(d_sigma),
                                    C.c_void_p(stream) if stream else None, C.byref(job)))
        st = RunStats()
        rc = lib().gdpm_job_wait(job, C.byref(st))
        lib().gdpm_job_release(job)
        _check(rc)
        out = _stats_dict(st)
        out["status"] = STATUS[rc]
        return out

    def run_noalloc(self, phantom: Phantom, source: Source, d_dose: int, d_sigma: int,
                    stream: int = 0, **kw):
        """gdpm_run_noalloc: device outputs, the library's scratch memory, no
        allocation; blocking.  Returns run statistics."""
        st = RunStats()
        rc = _check(lib().gdpm_run_noalloc(self.handle, phantom.handle, source.handle,
                                           C.byref(_params(kw)), C.c_void_p(d_dose),
                                           C.c_void_p(d_sigma),
                                           C.c_void_p(stream) if stream else None, C.byref(st)))
        out = _stats_dict(st)
        out["status"] = STATUS[rc]
        return out

    # --- test entry points ---
    def atomic_rate(self, nbytes: int) -> float:
        """Scattered FP64 atomic additions per second into an array of nbytes."""
        out = C.c_double()
        _check(lib().gdpm_test_atomic_rate(self.handle, nbytes, C.byref(out)))
        return out.value

    def philox(self, key: Sequence[int], ctr: np.ndarray) -> np.ndarray:
        ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
        out = np.empty_like(ctr)
        k = (C.c_uint32 * 2)(*key)
        _check(lib().gdpm_test_philox(self.handle, k, ctr.ctypes.data_as(C.POINTER(C.c_uint32)),
                                      out.ctypes.data_as(C.POINTER(C.c_uint32)), len(ctr)))
        return out

    def sample(self, which, e, p1=0.0, p2=0.0, seed=1, n=1000):
        a = np.empty(n, dtype=np.float32)
        b = np.empty(n, dtype=np.float32)
        _check(lib().gdpm_test_sample(self.handle, which, e, p1, p2, seed, n, _fp(a), _fp(b)))
        return a, b

    def sample_source(self, phantom: Phantom, source: Source, seed=1, job=0, hist0=0, n=1000):
        out = np.empty((n, 8), dtype=np.float32)
        _check(lib().gdpm_test_source(self.handle, phantom.handle, source.handle, seed, job, hist0,
                                      n, _fp(out)))
        return out

    def lookup(self, which, mat, x, ecut_g=0.05, ecut_e=0.2, flags=0):
        x = np.ascontiguousarray(x, dtype=np.float32)
        out = np.empty_like(x)
        _check(lib().gdpm_test_lookup(self.handle, ecut_g, ecut_e, flags, which, mat, _fp(x),
                                      _fp(out), len(x)))
        return out

    def close(self):
        if self.handle:
            lib().gdpm_context_destroy(self.handle)
            self.handle = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _params(kw):
    return RunParams(kw.get("seed", 1), kw.get("job_id", 0), kw.get("n_hist", 1000),
                     kw.get("target_unc", 0.0), kw.get("n_batches", 10), kw.get("ecut_g", 0.05),
                     kw.get("ecut_e", 0.2), kw.get("max_histories", 0), kw.get("flags", 0),
                     kw.get("round_size", 0), kw.get("hist0", 0), kw.get("stat_min_density", 0.0),
                     kw.get("split_log2", 0))


class ServerJob:
    """A queued or running job of a Server; wait() returns its result dict."""

    def __init__(self, handle, dose, sigma, desc):
        self.handle, self.dose, self.sigma = handle, dose, sigma
        self._desc = desc   # keeps the descriptor's arrays alive until the job ends

    def wait(self):
        st = RunStats()
        rc = lib().gdpm_job_wait(self.handle, C.byref(st))
        msg = lib().gdpm_last_error().decode() if rc not in (0, 6) else ""
        lib().gdpm_job_release(self.handle)
        self.handle = None
        if rc not in (0, 6):
            raise GdpmError(rc, msg)
        r = _stats_dict(st)
        r["status"] = STATUS[rc]
        r["dose"], r["sigma"] = self.dose, self.sigma
        return r


class Server:
    """Request loop of libgdpm on a context: admission by device footprint and
    slots, continuous batching of the admitted jobs (gdpm_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int = 64):
        self.ctx = ctx
        self.handle = C.c_void_p()
        _check(lib().gdpm_server_create(ctx.handle, int(hbm_budget_bytes), max_slots,
                                        C.byref(self.handle)))

    def submit(self, phantom: Phantom, source: Source, want_dose=True, **kw) -> ServerJob:
        nv = phantom.desc.nvox
        dose = np.zeros(nv) if want_dose else None
        sigma = np.zeros(nv) if want_dose else None
        desc = JobDesc(phantom.handle, source.handle, _params(kw), _dp(dose), _dp(sigma))
        job = C.c_void_p()
        _check(lib().gdpm_server_submit(self.handle, C.byref(desc), C.byref(job)))
        return ServerJob(job, dose, sigma, desc)

    def info(self):
        i = ServerInfo()
        _check(lib().gdpm_server_info_get(self.handle, C.byref(i)))
        return {k: getattr(i, k) for k, _ in ServerInfo._fields_}

    def close(self):
        if self.handle:
            _check(lib().gdpm_server_destroy(self.handle))
            self.handle = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
