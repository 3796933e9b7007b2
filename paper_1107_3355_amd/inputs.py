"""Seeded synthetic inputs: materials, phantoms, beams and spectra.

This module only builds input data (arrays and plain descriptions).  It holds
none of the transport arithmetic, imports neither the GPU binding nor the
oracle, and is the one module both of them are fed from.

The paper's clinical inputs (patient CTs, Eclipse plans, the measured 6 MV
spectrum; sections 3.1 and 3.2) are not available, so the generators below make
stand-ins of the same shapes: slab phantoms of water/lung/bone along depth
(section 3.1), a point source at SSD 90 cm with a 10x10 cm field at SAD 100 cm
(section 3.1), a piecewise-linear photon spectrum, an ellipsoid CT phantom with
a 9-field coplanar fluence-map plan (section 3.2, fluence maps of section 2.3.1).

Units: cm, MeV, g/cm^3.  Voxel index v = ix + nx*(iy + ny*iz); arrays are
stored with shape (nz, ny, nx) so that ``arr.ravel()`` follows that order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# materials: pseudo-elements (Z_eff, Z/A, mean excitation energy I)
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class Material:
    name: str
    z: float
    z_over_a: float
    i_ev: float
    rho_nominal: float


AIR = Material("air", 7.64, 0.49919, 85.7, 0.0012)
LUNG = Material("lung", 7.42, 0.55508, 75.0, 0.26)
WATER = Material("water", 7.42, 0.55508, 75.0, 1.00)
BONE = Material("bone", 13.0, 0.5148, 106.4, 1.85)
MATERIALS: List[Material] = [AIR, LUNG, WATER, BONE]
ID_AIR, ID_LUNG, ID_WATER, ID_BONE = 0, 1, 2, 3

# ---------------------------------------------------------------------------
# phantom, beams, source
# ---------------------------------------------------------------------------


@dataclass
class Phantom:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    mat: np.ndarray  # uint8, shape (nz, ny, nx)
    rho: np.ndarray  # float32, shape (nz, ny, nx)

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def extent(self):
        return (self.nx * self.dx, self.ny * self.dy, self.nz * self.dz)


@dataclass
class Beam:
    iso: Sequence[float]     # isocentre (cm)
    dir: Sequence[float]     # unit central axis, source -> isocentre
    e1: Sequence[float]      # unit beamlet-column axis in the isocentre plane
    sad: float               # source-axis distance; <= 0 for a parallel beam
    nbx: int
    nby: int
    bw: float
    bh: float
    intensity: Optional[np.ndarray] = None  # float32 (nby, nbx) relative fluence, None = open


@dataclass
class Spectrum:
    kind: int = 0            # 0 monoenergetic, 1 piecewise-linear pdf
    e_mono: float = 1.0
    e: Optional[np.ndarray] = None
    p: Optional[np.ndarray] = None


@dataclass
class Source:
    particle: int            # 0 photon, 1 electron
    spectrum: Spectrum
    beams: List[Beam] = field(default_factory=list)
    beamlet_sampler: int = 0  # 0 cumulative-probability search, 1 Metropolis chains (Algorithm A1)
    spectrum_strata: int = 0  # 0 plain spectrum sampling, K > 0 energy intervals (section 2.3.2)
    strata_shape: int = 0     # inside an interval: 0 uniform energy (section 2.3.2), 1 the spectrum's shape
    # (n, 7) float32 records x, y, z, u, v, w, E: a phase space (section 2.3.3);
    # history h starts as record h mod n, and beams and spectrum are unused
    phase_space: Optional[np.ndarray] = None


PHOTON, ELECTRON = 0, 1

# ---------------------------------------------------------------------------
# generators
# ---------------------------------------------------------------------------


def homogeneous(n: Sequence[int], d: Sequence[float], mat_id: int, rho: float) -> Phantom:
    nx, ny, nz = n
    mat = np.full((nz, ny, nx), mat_id, dtype=np.uint8)
    den = np.full((nz, ny, nx), rho, dtype=np.float32)
    return Phantom(nx, ny, nz, *map(float, d), mat, den)


def slab_phantom(n: int = 100, d: float = 0.3,
                 layers=((ID_WATER, 17), (ID_LUNG, 17), (ID_BONE, 17), (ID_WATER, 49))) -> Phantom:
    """Layers along z (depth), thicknesses in voxels; nominal densities."""
    assert sum(t for _, t in layers) == n
    mat = np.empty((n, n, n), dtype=np.uint8)
    rho = np.empty((n, n, n), dtype=np.float32)
    z = 0
    for mid, t in layers:
        mat[z:z + t] = mid
        rho[z:z + t] = MATERIALS[mid].rho_nominal
        z += t
    return Phantom(n, n, n, d, d, d, mat, rho)


def hu_to_material(hu: np.ndarray):
    """HU -> (material id, density): air < -950 <= lung < -400 <= water < 150 <= bone."""
    mat = np.full(hu.shape, ID_BONE, dtype=np.uint8)
    mat[hu < 150] = ID_WATER
    mat[hu < -400] = ID_LUNG
    mat[hu < -950] = ID_AIR
    rho = np.where(hu <= 0, np.maximum(0.0012, 1.0 + hu / 1000.0), 1.0 + 0.00085 * hu)
    return mat, rho.astype(np.float32)


def _ellipsoid(shape, d, centre, semi):
    nz, ny, nx = shape
    x = (np.arange(nx) + 0.5) * d[0] - centre[0]
    y = (np.arange(ny) + 0.5) * d[1] - centre[1]
    z = (np.arange(nz) + 0.5) * d[2] - centre[2]
    return ((z[:, None, None] / semi[2]) ** 2 + (y[None, :, None] / semi[1]) ** 2
            + (x[None, None, :] / semi[0]) ** 2) <= 1.0


def ct_phantom(n=(256, 256, 128), d=(0.2, 0.2, 0.25), seed: int = 1003) -> Phantom:
    """Ellipsoid 'patient': body 0 HU, two lungs -800 HU, spine and 12 ribs
    +1000 HU, air outside, Gaussian noise sigma 20 HU; 4 materials + density."""
    nx, ny, nz = n
    lx, ly, lz = nx * d[0], ny * d[1], nz * d[2]
    c = (lx / 2, ly / 2, lz / 2)
    shape = (nz, ny, nx)
    hu = np.full(shape, -1000.0, dtype=np.float64)
    body = _ellipsoid(shape, d, c, (0.42 * lx, 0.32 * ly, 0.48 * lz))
    hu[body] = 0.0
    for sx in (-1, 1):
        lung = _ellipsoid(shape, d, (c[0] + sx * 0.13 * lx, c[1] + 0.03 * ly, c[2]),
                          (0.09 * lx, 0.12 * ly, 0.30 * lz))
        hu[lung & body] = -800.0
    spine = _ellipsoid(shape, d, (c[0], c[1] - 0.20 * ly, c[2]), (0.03 * lx, 0.04 * ly, 0.5 * lz))
    hu[spine & body] = 1000.0
    for k in range(12):
        a = 2 * math.pi * (k + 0.5) / 12
        rc = (c[0] + 0.40 * lx * math.cos(a), c[1] + 0.30 * ly * math.sin(a), c[2])
        rib = _ellipsoid(shape, d, rc, (0.015 * lx, 0.015 * ly, 0.30 * lz))
        hu[rib & body] = 1000.0
    rng = np.random.Generator(np.random.PCG64(seed))
    hu += rng.normal(0.0, 20.0, size=shape)
    mat, rho = hu_to_material(hu)
    return Phantom(nx, ny, nz, d[0], d[1], d[2], mat, rho)


def ellipsoid_phantom(n: int, d: float, seed: int, n_blobs: int = 6) -> Phantom:
    """Water cube with random lung and bone ellipsoids at nominal densities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n, n)
    L = n * d
    mat = np.full(shape, ID_WATER, dtype=np.uint8)
    rho = np.full(shape, WATER.rho_nominal, dtype=np.float32)
    for _ in range(n_blobs):
        mid = ID_LUNG if rng.random() < 0.5 else ID_BONE
        centre = rng.uniform(0.2 * L, 0.8 * L, size=3)
        semi = rng.uniform(0.05 * L, 0.2 * L, size=3)
        m = _ellipsoid(shape, (d, d, d), centre, semi)
        mat[m] = mid
        rho[m] = MATERIALS[mid].rho_nominal
    return Phantom(n, n, n, d, d, d, mat, rho)


def triangular_spectrum(lo: float = 0.25, peak: float = 1.2, hi: float = 6.0) -> Spectrum:
    """6 MV-like stand-in: piecewise-linear pdf, zero at lo and hi, peak at `peak`."""
    return Spectrum(kind=1, e=np.array([lo, peak, hi], dtype=np.float64),
                    p=np.array([0.0, 1.0, 0.0], dtype=np.float64))


def mono(e: float) -> Spectrum:
    return Spectrum(kind=0, e_mono=float(e))


def parallel_beam_z(ph: Phantom, field: float) -> Beam:
    """Parallel beam along +z into the z = 0 face, square field centred in x, y."""
    lx, ly, lz = ph.extent
    return Beam(iso=(lx / 2, ly / 2, lz / 2), dir=(0.0, 0.0, 1.0), e1=(1.0, 0.0, 0.0),
                sad=0.0, nbx=1, nby=1, bw=field, bh=field)


def point_beam_z(ph: Phantom, field: float = 10.0, ssd: float = 90.0, sad: float = 100.0) -> Beam:
    """Point source on the z axis at SSD from the z = 0 face, field defined at SAD."""
    lx, ly, _ = ph.extent
    return Beam(iso=(lx / 2, ly / 2, sad - ssd), dir=(0.0, 0.0, 1.0), e1=(1.0, 0.0, 0.0),
                sad=sad, nbx=1, nby=1, bw=field, bh=field)


def gantry_beam(ph: Phantom, gantry_deg: float, nb: int = 40, bsize: float = 0.5,
                sad: float = 100.0, intensity: Optional[np.ndarray] = None) -> Beam:
    """Coplanar beam rotated by the gantry angle about the phantom z axis through
    its centre; beamlet columns in the x-y plane, rows along z."""
    lx, ly, lz = ph.extent
    t = math.radians(gantry_deg)
    d = (math.sin(t), -math.cos(t), 0.0)
    e1 = (math.cos(t), math.sin(t), 0.0)
    return Beam(iso=(lx / 2, ly / 2, lz / 2), dir=d, e1=e1, sad=sad, nbx=nb, nby=nb,
                bw=bsize, bh=bsize, intensity=intensity)


def linac_beam(ph: Phantom, gantry_deg: float, collimator_deg: float = 0.0, couch_deg: float = 0.0,
               nb: int = 40, bsize: float = 0.5, sad: float = 100.0,
               intensity: Optional[np.ndarray] = None) -> Beam:
    """Beam of a linac with gantry, collimator and couch angles (section 2.3:
    the plan's geometry rotates the gantry, the collimator and the couch).
    Phantom frame: z along the couch, y vertical (gantry 0 irradiates along -y),
    isocentre at the phantom centre.  The gantry turns the beam about z (as
    gantry_beam); the collimator turns the fluence map about the central axis
    by collimator_deg (from e1 towards e2 = dir x e1); the couch turns the
    patient about the vertical y axis by couch_deg, i.e. the beam by
    -couch_deg.  Angles 0, 0 give gantry_beam's beam."""
    b = gantry_beam(ph, gantry_deg, nb=nb, bsize=bsize, sad=sad, intensity=intensity)
    d = np.array(b.dir, dtype=np.float64)
    e1 = np.array(b.e1, dtype=np.float64)
    e2 = np.cross(d, e1)
    c = math.radians(collimator_deg)
    e1 = math.cos(c) * e1 + math.sin(c) * e2
    t = math.radians(-couch_deg)
    ry = np.array([[math.cos(t), 0.0, math.sin(t)], [0.0, 1.0, 0.0], [-math.sin(t), 0.0, math.cos(t)]])
    iso = np.array(b.iso, dtype=np.float64)
    return Beam(iso=tuple(iso), dir=tuple(ry @ d), e1=tuple(ry @ e1), sad=sad, nbx=nb, nby=nb,
                bw=bsize, bh=bsize, intensity=intensity)


def noncoplanar_plan(ph: Phantom, nb: int = 40, seed: int = 1009) -> List[Beam]:
    """Eight non-coplanar fields (the paper's head-and-neck IMRT plan had eight,
    section 3.2): gantry, couch and collimator angles below, intensities
    uniform in [0, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fields = [(0, 0, 0), (45, 20, 15), (90, 40, 30), (135, -20, 45), (180, 0, 90), (225, 30, 10),
              (270, -40, 60), (315, 10, 5)]
    return [linac_beam(ph, g, coll, couch, nb=nb,
                       intensity=rng.uniform(0.0, 1.0, size=(nb, nb)).astype(np.float32))
            for g, couch, coll in fields]


def point_phase_space(ph: Phantom, n: int, seed: int, sad: float = 100.0, field: float = 10.0,
                      spectrum: Optional[Spectrum] = None, inside_frac: float = 0.0) -> np.ndarray:
    """Synthetic phase space (section 2.3.3 stands in for a linac's): n records
    of a point source SAD cm above the phantom centre (along -y, gantry 0),
    directions uniform over a square field of `field` cm at the isocentre,
    energies from `spectrum` (default 6 MV-like triangular) by numpy's PCG64;
    records scored on a plane 5 cm above the phantom, plus a fraction of
    records placed inside the phantom on the same rays.  float32, unit
    directions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lx, ly, lz = ph.extent
    iso = np.array([lx / 2, ly / 2, lz / 2])
    src = iso + np.array([0.0, sad, 0.0])
    a = rng.uniform(-field / 2, field / 2, size=(n, 2))
    tgt = iso[None, :] + np.stack([a[:, 0], np.zeros(n), a[:, 1]], axis=1)
    d = tgt - src
    d /= np.linalg.norm(d, axis=1)[:, None]
    t = (src[1] - (ly + 5.0)) / -d[:, 1]            # the scoring plane y = ly + 5
    inside = rng.random(n) < inside_frac
    t = np.where(inside, (src[1] - ly / 2) / -d[:, 1], t)
    pos = src[None, :] + t[:, None] * d
    sp = spectrum or triangular_spectrum()
    if sp.kind == 0:
        e = np.full(n, sp.e_mono)
    else:   # inverse CDF on a fine grid of the piecewise-linear pdf
        grid = np.linspace(sp.e[0], sp.e[-1], 4097)
        pg = np.interp(grid, sp.e, sp.p)
        cg = np.concatenate([[0.0], np.cumsum(0.5 * (pg[1:] + pg[:-1]) * np.diff(grid))])
        e = np.interp(rng.random(n) * cg[-1], cg, grid)
    out = np.concatenate([pos, d, e[:, None]], axis=1).astype(np.float32)
    out[:, 3:6] /= np.linalg.norm(out[:, 3:6].astype(np.float64), axis=1)[:, None].astype(np.float32)
    return out


def imrt_plan(ph: Phantom, n_beams: int = 9, nb: int = 40, seed: int = 1003) -> List[Beam]:
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    beams = []
    for k in range(n_beams):
        f = rng.uniform(0.0, 1.0, size=(nb, nb)).astype(np.float32)
        beams.append(gantry_beam(ph, 360.0 * k / n_beams, nb=nb, intensity=f))
    return beams


def vmat_arc(ph: Phantom, n_cp: int = 180, nb: int = 40, seed: int = 1005) -> List[Beam]:
    rng = np.random.Generator(np.random.PCG64(seed + 11))
    return [gantry_beam(ph, 360.0 * k / n_cp, nb=nb,
                        intensity=rng.uniform(0.0, 1.0, size=(nb, nb)).astype(np.float32))
            for k in range(n_cp)]

# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    phantom: Phantom
    source: Source
    n_hist: int
    n_batches: int = 10
    ecut_g: float = 0.05
    ecut_e: float = 0.2
    seed: int = 1
    target_unc: float = 0.0


def water_cube_2mev(n_hist: int = 200_000) -> Workload:
    """32^3 water voxels of 0.5 cm, 2 MeV parallel photons, 5x5 cm field."""
    ph = homogeneous((32, 32, 32), (0.5, 0.5, 0.5), ID_WATER, 1.0)
    src = Source(PHOTON, mono(2.0), [parallel_beam_z(ph, 5.0)])
    return Workload("water32_2MeV_parallel", ph, src, n_hist)


def slab_photon(n_hist: int = 10_000_000, n: int = 100, d: float = 0.3) -> Workload:
    """Slab heterogeneity phantom, 6 MV-like spectrum, point source, 10x10 cm."""
    ph = slab_phantom(n, d) if n == 100 else _scaled_slab(n, d)
    src = Source(PHOTON, triangular_spectrum(), [point_beam_z(ph)])
    return Workload("slab100_6MVlike_point", ph, src, n_hist)


def slab_electron(n_hist: int = 10_000_000, n: int = 100, d: float = 0.3) -> Workload:
    """Slab heterogeneity phantom, 20 MeV electrons, point source, 10x10 cm."""
    ph = slab_phantom(n, d) if n == 100 else _scaled_slab(n, d)
    src = Source(ELECTRON, mono(20.0), [point_beam_z(ph)])
    return Workload("slab100_20MeV_electron", ph, src, n_hist)


def _scaled_slab(n: int, d: float) -> Phantom:
    t = [round(n * f) for f in (0.17, 0.17, 0.17)]
    return slab_phantom(n, d, ((ID_WATER, t[0]), (ID_LUNG, t[1]), (ID_BONE, t[2]),
                               (ID_WATER, n - sum(t))))


def ct_imrt(n_hist: int = 100_000_000, n=(256, 256, 128), d=(0.2, 0.2, 0.25),
            target_unc: float = 0.01) -> Workload:
    """Synthetic CT with a 9-beam coplanar IMRT plan (40x40 beamlets of 0.5 cm)."""
    ph = ct_phantom(n, d)
    src = Source(PHOTON, triangular_spectrum(), imrt_plan(ph))
    return Workload("ct256x256x128_imrt9_6MVlike", ph, src, n_hist, target_unc=target_unc)


def batch_jobs(n_jobs: int = 64, seed: int = 4001, side=(48, 256), d: float = 0.25,
               hist=(1e5, 1e7), target_unc: float = 0.0) -> List[Workload]:
    """Independent dose jobs of uneven size for the batched form: cubes of side
    uniform in `side` voxels of `d` cm with random lung/bone ellipsoids;
    histories log-uniform in `hist`; half the jobs use the 6 MV-like spectrum,
    the others a monoenergetic 1-20 MeV beam, photons or electrons with equal
    odds; a parallel 10x10 cm field along +z, clipped to the phantom."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n_jobs):
        n = int(rng.integers(side[0], side[1] + 1))
        ph = ellipsoid_phantom(n, d, seed=seed * 1000 + k)
        field = min(10.0, n * d)
        if rng.random() < 0.5:
            src = Source(PHOTON, triangular_spectrum(), [parallel_beam_z(ph, field)])
            kind = "6MVlike"
        else:
            e = float(rng.uniform(1.0, 20.0))
            particle = PHOTON if rng.random() < 0.5 else ELECTRON
            src = Source(particle, mono(e), [parallel_beam_z(ph, field)])
            kind = f"{'photon' if particle == PHOTON else 'electron'}{e:.1f}MeV"
        nh = int(round(10 ** rng.uniform(np.log10(hist[0]), np.log10(hist[1]))))
        out.append(Workload(f"cube{n}_{kind}", ph, src, nh, target_unc=target_unc))
    return out


def serving_requests(duration_s: float = 300.0, rate: float = 2.0, seed: int = 5001,
                     ct=None, small_ct=None):
    """Poisson request stream of the serving form: arrival times at `rate` jobs/s
    over `duration_s`; each request is a VMAT-like arc (180 control points, 40x40
    fluence per point) on the 256x256x128 CT or a 9-beam IMRT job on a
    128x128x64 CT of 0.4x0.4x0.5 cm voxels (same extent), with equal odds, at a
    requested uncertainty of 1% or 2% with equal odds.  Returns (arrival time,
    Workload) pairs; phantoms are shared between requests of the same kind."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ct = ct if ct is not None else ct_phantom()
    small_ct = small_ct if small_ct is not None else ct_phantom((128, 128, 64), (0.4, 0.4, 0.5))
    t, out = 0.0, []
    k = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration_s:
            break
        unc = 0.01 if rng.random() < 0.5 else 0.02
        if rng.random() < 0.5:
            src = Source(PHOTON, triangular_spectrum(), vmat_arc(ct, seed=seed + 7 * k))
            w = Workload(f"vmat180_ct256_{unc:.0%}", ct, src, 20_000_000, target_unc=unc)
        else:
            src = Source(PHOTON, triangular_spectrum(), imrt_plan(small_ct, seed=seed + 7 * k))
            w = Workload(f"imrt9_ct128_{unc:.0%}", small_ct, src, 5_000_000, target_unc=unc)
        out.append((t, w))
        k += 1
    return out
