"""ctypes binding of the reference CPU transport in ``oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the GPU library or its Python binding.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NO_COMPTON, NO_PHOTO, NO_PAIR, NO_MS, NO_MOLLER, NO_BREMS, KERMA = 1, 2, 4, 8, 16, 32, 64
EV_NAMES = ("flights", "real", "esteps", "hard_cand", "hard", "deposits", "pushes", "histories")
(MU_COMPTON, MU_PHOTO, MU_PAIR, L_RESTRICTED, S_RAD_SOFT, MU_MOLLER, MU_BREMS, INV_LAMBDA1,
 X0, S_TOTAL, SIGMA_KN, DSIGMA_KN, DSIGMA_MOLLER, DMU_BREMS, MW_MEAN) = range(15)


class Material(C.Structure):
    _fields_ = [("z", C.c_double), ("z_over_a", C.c_double), ("i_ev", C.c_double)]


class Phantom(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("mat", C.POINTER(C.c_uint8)), ("rho", C.POINTER(C.c_float))]


class Beam(C.Structure):
    _fields_ = [("iso", C.c_double * 3), ("dir", C.c_double * 3), ("e1", C.c_double * 3),
                ("sad", C.c_double), ("nbx", C.c_int), ("nby", C.c_int),
                ("bw", C.c_double), ("bh", C.c_double), ("intensity", C.POINTER(C.c_float))]


METRO_CHAINS = 16384   # ORC_METRO_CHAINS of oracle.h


class Source(C.Structure):
    _fields_ = [("particle", C.c_int), ("spec_kind", C.c_int), ("spec_n", C.c_int),
                ("spec_e", C.POINTER(C.c_double)), ("spec_p", C.POINTER(C.c_double)),
                ("e_mono", C.c_double), ("n_beams", C.c_int), ("beams", C.POINTER(Beam)),
                ("beamlet_sampler", C.c_int), ("spectrum_strata", C.c_int),
                ("n_phsp", C.c_uint64), ("phsp", C.POINTER(C.c_float)), ("strata_shape", C.c_int)]


class Params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("job_id", C.c_uint32), ("n_hist", C.c_uint64),
                ("hist0", C.c_uint64), ("round_size", C.c_uint64), ("n_batches", C.c_int),
                ("ecut_g", C.c_double), ("ecut_e", C.c_double), ("flags", C.c_uint32),
                ("n_threads", C.c_int), ("split_log2", C.c_int)]


TYPE_NAMES = ("flight_real", "flight_virtual", "compton", "photo", "pair", "hard_real",
              "hard_virtual", "moller", "brems")


class Stats(C.Structure):
    _fields_ = [("e_in", C.c_double), ("e_dep", C.c_double), ("e_esc", C.c_double),
                ("ev", C.c_uint64 * 8), ("n_type", C.c_uint64 * len(TYPE_NAMES)),
                ("p_type", C.c_double * len(TYPE_NAMES)), ("v_type", C.c_double * len(TYPE_NAMES))]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} is not built; run oracle/build.py or __graft_entry__.build()")
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_run.argtypes = [C.POINTER(Material), C.c_int, C.POINTER(Phantom), C.POINTER(Source),
                              C.POINTER(Params), dp, dp, dp, dp, C.POINTER(C.c_uint32),
                              C.POINTER(Stats)]
        L.orc_run.restype = C.c_int
        L.orc_phys.argtypes = [C.c_int, C.POINTER(Material), C.c_double, C.c_double, C.c_double]
        L.orc_phys.restype = C.c_double
        L.orc_path_length.argtypes = [C.POINTER(Material)] + [C.c_double] * 4
        L.orc_path_length.restype = C.c_double
        L.orc_csda_energy.argtypes = [C.POINTER(Material)] + [C.c_double] * 4
        L.orc_csda_energy.restype = C.c_double
        L.orc_mw_A.argtypes = [C.c_double]
        L.orc_mw_A.restype = C.c_double
        L.orc_philox.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_philox.restype = None
        L.orc_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32,
                                   C.c_int, dp]
        L.orc_uniforms.restype = None
        L.orc_spawn_path.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32,
                                     C.c_int]
        L.orc_spawn_path.restype = C.c_uint32
        L.orc_sample.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_int,
                                 dp, dp]
        L.orc_sample.restype = None
        L.orc_sample_source.argtypes = [C.POINTER(Source), C.POINTER(Phantom), C.c_uint64,
                                        C.c_uint32, C.c_uint64, C.c_int, dp]
        L.orc_sample_source.restype = C.c_int
        _lib = L
    return _lib


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _material(m):
    return Material(m.z, m.z_over_a, m.i_ev)


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self):
        self.refs = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.refs.append(a)
        return a


def _phantom(ph, keep):
    mat = keep.arr(ph.mat, np.uint8)
    rho = keep.arr(ph.rho, np.float32)
    return Phantom(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz,
                   mat.ctypes.data_as(C.POINTER(C.c_uint8)),
                   rho.ctypes.data_as(C.POINTER(C.c_float)))


def _source(src, keep):
    beams = (Beam * len(src.beams))()
    for i, b in enumerate(src.beams):
        beams[i].iso[:] = list(b.iso)
        beams[i].dir[:] = list(b.dir)
        beams[i].e1[:] = list(b.e1)
        beams[i].sad = b.sad
        beams[i].nbx, beams[i].nby = b.nbx, b.nby
        beams[i].bw, beams[i].bh = b.bw, b.bh
        if b.intensity is not None:
            f = keep.arr(b.intensity, np.float32).ravel()
            beams[i].intensity = f.ctypes.data_as(C.POINTER(C.c_float))
    keep.refs.append(beams)
    sp = src.spectrum
    s = Source(src.particle, sp.kind, 0, None, None, sp.e_mono, len(src.beams), beams,
               getattr(src, "beamlet_sampler", 0), getattr(src, "spectrum_strata", 0))
    s.strata_shape = getattr(src, "strata_shape", 0)
    ps = getattr(src, "phase_space", None)
    if ps is not None:
        ps = keep.arr(ps, np.float32).reshape(-1, 7)
        s.n_phsp = len(ps)
        s.phsp = ps.ctypes.data_as(C.POINTER(C.c_float))
    if sp.kind == 1:
        e = keep.arr(sp.e, np.float64)
        p = keep.arr(sp.p, np.float64)
        s.spec_n = len(e)
        s.spec_e, s.spec_p = _dptr(e), _dptr(p)
    return s


def run(materials, phantom, source, *, seed=1, n_hist=1000, n_batches=10, round_size=None,
        hist0=0, job_id=0, ecut_g=0.05, ecut_e=0.2, flags=0, n_threads=None,
        want_batches=True, want_hist=False, want_hist_hard=False, split_log2=0):
    """Run the reference transport; returns a dict of numpy arrays and stats."""
    L = lib()
    keep = _Keep()
    mats = (Material * len(materials))(*[_material(m) for m in materials])
    ph = _phantom(phantom, keep)
    src = _source(source, keep)
    if round_size is None:
        round_size = -(-n_hist // n_batches)
    if n_threads is None:
        n_threads = min(os.cpu_count() or 1, 16)
    prm = Params(seed, job_id, n_hist, hist0, round_size, n_batches, ecut_g, ecut_e, flags,
                 n_threads, split_log2)
    nv = phantom.nvox
    batch = np.zeros((n_batches, nv)) if want_batches else None
    dose = np.zeros(nv)
    sigma = np.zeros(nv)
    hist = np.zeros((n_hist, 2)) if want_hist else None
    hard = np.zeros(n_hist, dtype=np.uint32) if want_hist_hard else None
    st = Stats()
    rc = L.orc_run(mats, len(materials), C.byref(ph), C.byref(src), C.byref(prm),
                   _dptr(batch), _dptr(dose), _dptr(sigma), _dptr(hist),
                   None if hard is None else hard.ctypes.data_as(C.POINTER(C.c_uint32)),
                   C.byref(st))
    if rc != 0:
        raise ValueError("oracle rejected its inputs")
    out = {"dose": dose, "sigma": sigma, "e_in": st.e_in, "e_dep": st.e_dep, "e_esc": st.e_esc,
           "events": {k: int(st.ev[i]) for i, k in enumerate(EV_NAMES)},
           "choices": {k: (int(st.n_type[i]), st.p_type[i], st.v_type[i])
                       for i, k in enumerate(TYPE_NAMES)}}
    if want_hist_hard:
        out["hist_hard"] = hard
    if want_batches:
        out["batch_edep"] = batch
    if want_hist:
        out["hist"] = hist
    return out


def phys(which, material, e, p1=0.0, p2=0.0):
    m = _material(material)
    return lib().orc_phys(which, C.byref(m), e, p1, p2)


def path_length(material, ta, tb, wcc=0.2, wcb=0.05):
    m = _material(material)
    return lib().orc_path_length(C.byref(m), ta, tb, wcc, wcb)


def csda_energy(material, t0, q, wcc=0.2, wcb=0.05):
    m = _material(material)
    return lib().orc_csda_energy(C.byref(m), t0, q, wcc, wcb)


def mw_A(t):
    return lib().orc_mw_A(t)


def philox(key, ctr):
    k = (C.c_uint32 * 2)(*key)
    c = (C.c_uint32 * 4)(*ctr)
    o = (C.c_uint32 * 4)()
    lib().orc_philox(k, c, o)
    return list(o)


def uniforms(seed, job, hist, path, ctr0, n):
    out = np.empty(n)
    lib().orc_uniforms(seed, job, hist, path, ctr0, n, _dptr(out))
    return out


def spawn_path(seed, job, hist, path, ctr, word):
    return lib().orc_spawn_path(seed, job, hist, path, ctr, word)


def sample(which, e, p1=0.0, p2=0.0, seed=1, n=1000):
    a = np.empty(n)
    b = np.empty(n)
    lib().orc_sample(which, e, p1, p2, seed, n, _dptr(a), _dptr(b))
    return a, b


def sample_source(source, phantom, seed=1, job=0, hist0=0, n=1000):
    keep = _Keep()
    ph = _phantom(phantom, keep)
    src = _source(source, keep)
    out = np.empty((n, 8))
    rc = lib().orc_sample_source(C.byref(src), C.byref(ph), seed, job, hist0, n, _dptr(out))
    if rc != 0:
        raise ValueError("oracle rejected its inputs")
    return out
