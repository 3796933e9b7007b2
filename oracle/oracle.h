/*
 * oracle.h -- reference CPU transport for coupled photon/electron Monte Carlo dose.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this library.  It shares no
 * code with the GPU library (no headers, helpers, tables or constants): every
 * formula here is written out independently, in double precision, one particle
 * at a time with a LIFO stack of secondaries.
 *
 * What it computes (paper, sections 2.1 and 2.2.1): the expected energy
 * absorbed per voxel per source history, by photon Woodcock tracking and
 * class-II condensed-history electron transport, over N_b batches, with the
 * per-voxel mean and its standard error (section 3.1).
 *
 * Units: cm, MeV, g/cm^3.  Voxel index v = ix + nx*(iy + ny*iz).
 */
#ifndef GDPM_ORACLE_H
#define GDPM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double z, z_over_a, i_ev; } orc_material;

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    const uint8_t* mat;   /* nx*ny*nz material ids */
    const float* rho;     /* nx*ny*nz densities, > 0 */
} orc_phantom;

typedef struct {
    double iso[3];        /* isocentre (cm, phantom frame) */
    double dir[3];        /* unit central axis, source -> isocentre */
    double e1[3];         /* unit beamlet-column axis in the isocentre plane; e2 = dir x e1 */
    double sad;           /* source-axis distance; <= 0 means a parallel beam */
    int nbx, nby;         /* beamlets along e1, e2 */
    double bw, bh;        /* beamlet size at the isocentre plane (cm) */
    const float* intensity; /* nbx*nby relative intensities >= 0 (index jx + nbx*jy) */
} orc_beam;

typedef struct {
    int particle;         /* 0 photon, 1 electron */
    int spec_kind;        /* 0 monoenergetic, 1 piecewise-linear pdf */
    int spec_n;
    const double* spec_e; /* spec_n increasing energies */
    const double* spec_p; /* spec_n pdf values >= 0 */
    double e_mono;
    int n_beams;
    const orc_beam* beams;
    int beamlet_sampler;  /* 0: cumulative-probability search; 1: Metropolis chains
                             (Algorithm A1, section 2.3.1; see ORC_METRO_CHAINS) */
    int spectrum_strata;  /* 0: each history samples the spectrum; K > 0 (piecewise-linear
                             spectra, K <= 64): section 2.3.2's energy intervals, K of
                             equal width over the spectrum's support; a round of R
                             histories gives positions C_k <= i < C_{k+1}, C_k =
                             floor(R F(e_k) + 1/2), to interval k, in increasing energy,
                             and inside the interval the energy is uniform (strata_shape
                             0, the paper's) or follows the spectrum (strata_shape 1) */
    uint64_t n_phsp;      /* > 0: a phase space (section 2.3.3, the open source
                             interface): history h starts as record h mod n_phsp of
                             phsp; beams and spectrum are then unused */
    const float* phsp;    /* n_phsp records x, y, z, u, v, w, E (cm, unit vector, MeV): a
                             record inside the phantom starts where it is, one outside
                             moves forward to its entry point or escapes; no draws */
    int strata_shape;     /* energy inside an interval: 0 uniform, 1 the spectrum's shape */
} orc_source;

/* Metropolis beamlet sampling: the run's histories form this many chains,
 * history h on chain h mod ORC_METRO_CHAINS, each taken in increasing h from
 * the run's first history (hist0). */
#define ORC_METRO_CHAINS 16384

/* physics switches (test cases that reduce to closed forms) */
#define ORC_NO_COMPTON 1u
#define ORC_NO_PHOTO   2u
#define ORC_NO_PAIR    4u
#define ORC_NO_MS      8u
#define ORC_NO_MOLLER  16u
#define ORC_NO_BREMS   32u
#define ORC_KERMA      64u

typedef struct {
    uint64_t seed;
    uint32_t job_id;
    uint64_t n_hist;      /* histories simulated: ids hist0 .. hist0+n_hist-1 */
    uint64_t hist0;
    uint64_t round_size;  /* R: history h goes to batch ((h-hist0)/R) mod n_batches */
    int n_batches;
    double ecut_g;        /* photon absorption energy = bremsstrahlung threshold */
    double ecut_e;        /* electron absorption energy = Moller threshold */
    uint32_t flags;
    int n_threads;
    int split_log2;       /* primary splitting (variance reduction): each history's
                             primary becomes 2^k copies of weight 2^-k, copy i on stream
                             path i from the draw after the source's; 0..6 (0: none) */
} orc_params;

/* event counters */
enum { ORC_EV_FLIGHTS = 0, ORC_EV_REAL, ORC_EV_ESTEPS, ORC_EV_HARD_CAND, ORC_EV_HARD,
       ORC_EV_DEPOSITS, ORC_EV_PUSHES, ORC_EV_HISTORIES };

/* the random choices of the transport, counted by outcome (a test of each
 * choice rule: the count of an outcome minus the sum of its probabilities over
 * the choices made is a martingale with variance sum p (1 - p)) */
enum { ORC_TYPE_FLIGHT_REAL = 0, ORC_TYPE_FLIGHT_VIRTUAL,      /* Woodcock acceptance */
       ORC_TYPE_COMPTON, ORC_TYPE_PHOTO, ORC_TYPE_PAIR,         /* real photon interactions */
       ORC_TYPE_HARD_REAL, ORC_TYPE_HARD_VIRTUAL,               /* hard-event acceptance */
       ORC_TYPE_MOLLER, ORC_TYPE_BREMS,                         /* real hard events */
       ORC_NTYPES };

typedef struct {
    double e_in, e_dep, e_esc;
    uint64_t ev[8];
    uint64_t n_type[ORC_NTYPES];   /* choices by outcome */
    double p_type[ORC_NTYPES];     /* sum of the outcome's probability over its choices */
    double v_type[ORC_NTYPES];     /* sum of p (1 - p) over the same choices */
} orc_stats;

/* Full run.  batch_edep (n_batches*nvox, MeV), dose and sigma (nvox, MeV/g per
 * history), hist_out (2*n_hist: deposited, escaped energy per history) and
 * hist_hard (n_hist: real hard events per history) may each be NULL.  Returns
 * 0 on success, nonzero on invalid input. */
int orc_run(const orc_material* mats, int n_mat, const orc_phantom* ph,
            const orc_source* src, const orc_params* prm,
            double* batch_edep, double* dose, double* sigma,
            double* hist_out, uint32_t* hist_hard, orc_stats* st);

/* ---- hooks used by the pin tests ---- */
enum { ORC_MU_COMPTON = 0, ORC_MU_PHOTO, ORC_MU_PAIR, ORC_L_RESTRICTED, ORC_S_RAD_SOFT,
       ORC_MU_MOLLER, ORC_MU_BREMS, ORC_INV_LAMBDA1, ORC_X0, ORC_S_TOTAL, ORC_SIGMA_KN,
       ORC_DSIGMA_KN, ORC_DSIGMA_MOLLER, ORC_DMU_BREMS, ORC_MW_MEAN };
/* which: quantity; E: energy (MeV); p1, p2: cutoffs or the secondary variable */
double orc_phys(int which, const orc_material* m, double E, double p1, double p2);
double orc_path_length(const orc_material* m, double ta, double tb, double wcc, double wcb);
double orc_csda_energy(const orc_material* m, double t0, double q, double wcc, double wcb);
double orc_mw_A(double t);
void orc_philox(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]);
void orc_uniforms(uint64_t seed, uint32_t job, uint64_t hist, uint32_t path, uint32_t ctr0,
                  int n, double* out);
uint32_t orc_spawn_path(uint64_t seed, uint32_t job, uint64_t hist, uint32_t path,
                        uint32_t ctr, int word);
/* which: 0 Compton (E) -> eps, cos; 1 Moller (T, wcc) -> eps; 2 bremsstrahlung
 * (T, wcb) -> k; 3 MW deflection (t) -> mu; 4 multiple-scattering walk of p2
 * hinges of t each -> Omega.Omega0; 5 annihilation pair -> cos1, dot(dir1, dir2);
 * 6 pair production (E) -> T-/(E - 2mc^2), T- + T+ + a - E; 7 Compton (E) ->
 * cos of the electron, cos of the photon (both against the incident direction).
 * Samplers 0, 1, 2, 6 and 7 run the transport's own code on a particle along +z. */
void orc_sample(int which, double e, double p1, double p2, uint64_t seed, int n,
                double* out1, double* out2);
/* source: n histories from hist0; out is n*8: E, beamlet, x, y, z, u, v, w
 * (beamlet -1 and x..w = NaN for a particle that misses the phantom) */
int orc_sample_source(const orc_source* src, const orc_phantom* ph, uint64_t seed,
                      uint32_t job, uint64_t hist0, int n, double* out);

#ifdef __cplusplus
}
#endif
#endif
