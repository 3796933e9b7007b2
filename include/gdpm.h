/*
 * gdpm.h -- C ABI of libgdpm: coupled photon/electron Monte Carlo dose on one
 * AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows the paper (Jia et al., "GPU-based fast Monte
 * Carlo simulation for radiotherapy dose calculation", gDPM v2.0):
 *   - a voxelised geometry with a material and a density per voxel, material
 *     properties and cross-section data (section 2.2.1);
 *   - a source with an energy spectrum (section 2.3.2), fluence maps grouped
 *     over all beam angles into beamlets of intensity f_I (section 2.3.1) and
 *     the linac geometry (gantry, collimator and couch rotations: any beam
 *     axis, section 2.3), sampled by search or by Metropolis chains (Algorithm
 *     A1) and optionally by energy intervals (section 2.3.2); or a phase space
 *     of primaries (the open source interface, section 2.3.3);
 *   - a number of histories split evenly into N_b batches (section 2.2.1),
 *     or an uncertainty target on the mean of sigma/D_max over voxels above
 *     half the maximum dose (section 3.1);
 *   - out: per-voxel mean dose and its standard error over the batches
 *     (section 2.2.1).
 * Transport: photon Woodcock tracking; class-II condensed-history electrons;
 * positrons as electrons with two photons at the end (section 2.1); absorption
 * energies (section 3.1); single precision transport (section 2.2.2) with
 * double-precision dose tallies.
 *
 * Conventions
 *   Units: cm, MeV, g/cm^3.  Dose is MeV/g per source history (multiply by
 *   1.602176634e-10 for Gy).  Voxel index v = ix + nx*(iy + ny*iz); the
 *   phantom occupies [0, nx*dx) x [0, ny*dy) x [0, nz*dz).
 *   Every function returns a gdpm_status; no exception crosses the ABI.  On
 *   failure gdpm_last_error() describes the cause (thread-local, valid until
 *   the next call on the same thread).
 *   Host input arrays are copied before a call returns; the caller keeps
 *   ownership of everything it passes.  Handles are destroyed explicitly;
 *   destroying a context invalidates its phantoms, sources and jobs.
 *   A context is bound to one HIP device and is not thread-safe: calls on one
 *   context must not overlap.
 */
#ifndef GDPM_H
#define GDPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GDPM_OK = 0,
    GDPM_E_INVALID = 1,        /* an argument is out of range or inconsistent */
    GDPM_E_NOMEM = 2,          /* a device or host allocation failed */
    GDPM_E_DEVICE = 3,         /* a HIP call failed */
    GDPM_E_OVERFLOW = 4,       /* a particle queue filled up; outputs are not valid */
    GDPM_E_BUSY = 5,           /* the context has a job in flight */
    GDPM_E_NOT_CONVERGED = 6   /* target uncertainty not reached within max_histories;
                                  outputs are written and valid for the histories run */
} gdpm_status;

typedef struct gdpm_context_s* gdpm_context;
typedef struct gdpm_phantom_s* gdpm_phantom;
typedef struct gdpm_source_s* gdpm_source;
typedef struct gdpm_job_s* gdpm_job;

/* Material as a pseudo-element (the paper keeps DPM's material data, section
 * 2.1, which is not reproduced; the closed-form models need Z, Z/A and I). */
typedef struct {
    double z;         /* effective atomic number, > 0 */
    double z_over_a;  /* electrons per nucleon (mol/g per mol of electrons), > 0 */
    double i_ev;      /* mean excitation energy (eV), > 0 */
} gdpm_material;

/* Energy spectrum (section 2.3.2). kind 0: monoenergetic e_mono.  kind 1:
 * piecewise-linear pdf through (e_mev[i], pdf[i]), i < n_pts, energies strictly
 * increasing, pdf >= 0 with positive area; sampled by exact inverse CDF. */
typedef struct {
    int kind;
    int n_pts;
    const double* e_mev;
    const double* pdf;
    double e_mono;
} gdpm_spectrum;

/* One beam (one gantry angle / control point) with its fluence map (section
 * 2.3.1).  The isocentre plane is spanned by e1 and e2 = dir x e1; beamlet
 * (jx, jy) covers [jx*bw - nbx*bw/2, (jx+1)*bw - nbx*bw/2) along e1 and the
 * same with bh, nby along e2.  sad_cm > 0: point source at iso - sad*dir;
 * sad_cm <= 0: parallel beam along dir.  intensity: nbx*nby values >= 0,
 * index jx + nbx*jy, or NULL for an open field (all 1). */
typedef struct {
    double iso_cm[3];
    double dir[3];      /* unit vector, source -> isocentre */
    double e1[3];       /* unit vector orthogonal to dir */
    double sad_cm;
    int nbx, nby;
    double bw_cm, bh_cm;
    const float* intensity;
} gdpm_beam;

typedef struct {
    int particle;            /* 0 photon, 1 electron */
    gdpm_spectrum spectrum;  /* energies within (ecut, 30] MeV */
    int n_beams;             /* >= 1; beamlets of all beams form one index I */
    const gdpm_beam* beams;
    /* how a history picks its beamlet (section 2.3.1): 0, the search of the
     * cumulative probability P(I) <= r < P(I+1); 1, Metropolis sampling
     * (Algorithm A1): a job's histories form GDPM_METRO_CHAINS chains, history
     * h on chain h mod GDPM_METRO_CHAINS, each taken in increasing h from the
     * job's first history and started at a beamlet drawn with equal
     * probability among those of nonzero intensity (stream: history id
     * (2^32-1)*2^32 + chain, path 0); at history h, after the energy, h's
     * stream gives a trial beamlet J (equal probability among nonzero ones)
     * and r, and the chain moves to J when r f_prev < f_J.  The chains
     * converge to f_I (the first histories of a chain carry their start's
     * bias); a chain's state lives with the job on the device. */
    int beamlet_sampler;
    /* how a history picks its energy (section 2.3.2): 0, by sampling the
     * spectrum; K in 1..64 (piecewise-linear spectra), from K energy intervals
     * of equal width over the spectrum's support: a round of R histories gives
     * positions C_k <= i < C_{k+1}, C_k = floor(R F(e_k) + 1/2), to interval k
     * (F the spectrum's CDF at the interval's lower edge), so a round runs
     * through the intervals in increasing energy; inside its interval a
     * history's energy is uniform or follows the spectrum (strata_shape). */
    int spectrum_strata;
    /* the open source interface (section 2.3.3): n_phase_space > 0 records of
     * 7 floats each, x, y, z (cm, phantom frame), u, v, w (unit vector, norm
     * within 1e-5 of 1), E (MeV, in (0, 30]), copied at creation.  History h
     * starts as record h mod n_phase_space: inside the phantom where it is,
     * outside at the point where its forward ray enters the phantom (or it
     * escapes); no random draws are spent on it.  Spectrum, beams and the two
     * modes above are then unused (n_beams may be 0). */
    uint64_t n_phase_space;
    const float* phase_space;
    /* energy inside an interval of spectrum_strata: 0, uniform between the
     * interval's edges (the paper's rule, section 2.3.2: the spectrum becomes
     * its histogram over the intervals); 1, the spectrum's own shape (inverse
     * CDF at F_k + u (F_{k+1} - F_k): the spectrum exactly). */
    int strata_shape;
} gdpm_source_desc;

#define GDPM_METRO_CHAINS 16384

/* run flags: physics switches used by the tests' closed-form special cases */
#define GDPM_NO_COMPTON 1u
#define GDPM_NO_PHOTO 2u
#define GDPM_NO_PAIR 4u
#define GDPM_NO_MS 8u
#define GDPM_NO_MOLLER 16u
#define GDPM_NO_BREMS 32u
#define GDPM_KERMA 64u   /* charged secondaries deposited where they are created */

typedef struct {
    uint64_t seed;             /* Philox key: (seed lo32, seed hi32 ^ job_id) */
    uint32_t job_id;
    uint64_t n_histories;      /* fixed history count, or the first estimate if target_unc > 0 */
    double target_unc;         /* 0: run n_histories; > 0: run until mean(sigma/D_max over
                                  D > D_max/2) <= target_unc */
    int n_batches;             /* N_b >= 2 (0 means 10) */
    double ecut_photon_mev;    /* photon absorption energy = bremsstrahlung threshold (0 -> 0.05) */
    double ecut_electron_mev;  /* electron absorption energy = Moller threshold (0 -> 0.2) */
    uint64_t max_histories;    /* cap in target mode (0 -> 100 * n_histories) */
    uint32_t flags;            /* GDPM_NO_* / GDPM_KERMA */
    uint64_t round_size;       /* histories per round; 0: n_histories / n_batches.  In fixed
                                  mode history h goes to batch floor(h/round_size) mod N_b */
    uint64_t hist0;            /* id of the first history (fixed mode) */
    double stat_min_density;   /* voxels below this density (g/cm^3) are left out of D_max and
                                  of the uncertainty statistic (0: all voxels) */
    int split_log2;            /* primary splitting, a variance reduction (the paper's
                                  section 4 names particle splitting as one): each history's
                                  source particle becomes S = 2^k copies of weight 1/S, copy
                                  i on stream path i from the draw after the source's (copy 0
                                  is the unsplit primary); deposits and escapes of a copy and
                                  its secondaries count with its weight, so the dose keeps its
                                  expectation and each history its energy exactly.  0..6
                                  (0: none).  The queues hold S records per history. */
} gdpm_run_params;

enum { GDPM_EV_FLIGHTS = 0, GDPM_EV_REAL, GDPM_EV_ESTEPS, GDPM_EV_HARD_CAND, GDPM_EV_HARD,
       GDPM_EV_DEPOSITS, GDPM_EV_PUSHES, GDPM_EV_HISTORIES };

typedef struct {
    uint64_t histories;
    double e_in, e_dep, e_esc;   /* MeV: source kinetic energy, deposited, escaped */
    double unc_mean_over_dmax;   /* mean sigma/D_max over D > D_max/2 (voxels at or above
                                    stat_min_density) */
    double dmax;                 /* MeV/g per history, same voxels */
    double t_total_s;            /* wall time of the call */
    double t_kernel_s;           /* device time of the transport kernels (HIP events) */
    double t_photon_s, t_electron_s;  /* device time per pass type, when the passes are
                                         launched apart (0 with fused_passes) */
    uint64_t events[8];          /* GDPM_EV_* counters of the run (for a job of a batch or a
                                    server: the engine's totals, all jobs, when it finished;
                                    events[GDPM_EV_HISTORIES] is the job's own) */
    uint32_t passes;             /* transport passes, photon and electron (a fused launch
                                    runs one of each) */
    uint32_t rounds;
    uint32_t passes_photon;      /* photon passes (t_photon_s covers them when launched apart) */
    uint32_t passes_electron;    /* electron passes (likewise t_electron_s) */
    /* per pass type (0 photon, 1 electron): 64-byte queue records the passes
     * loaded and stored (secondaries and particles handed to the next pass),
     * and FP64 tally deposits; the memory traffic the passes cannot avoid */
    uint64_t records_loaded[2], records_stored[2], deposits[2];
    /* consistency of the particle accounting: the number of times the run
     * found the queues empty while the job's particle births and deaths
     * differed, and the summed difference (births - deaths); 0 and 0 in a
     * sound run.  A nonzero gap is also visible in the energy balance. */
    uint32_t accounting_repairs;
    int64_t accounting_gap;
    /* particles ended by a safety net of the transport kernels (a non-finite
     * or absurd energy, a wavefront past its iteration bound) and queue
     * records dropped because they belong to no running job; 0 in a sound
     * run; counted over the whole run, like events and passes */
    uint64_t transport_anomalies;
    /* scheduler iterations launched as a replayed HIP graph, and the graphs
     * recorded for them (option "graphs"; 0 and 0 when it is off) */
    uint32_t graph_launches, graphs_recorded;
    /* option "check_accounting": iterations after which some job's live queue
     * records differed from its births less its deaths (0 in a sound run, and
     * always 0 with the option off) */
    uint32_t accounting_mismatches;
    /* real interactions by type over the run (Compton, photoelectric, pair,
     * Moller, bremsstrahlung), counted like events */
    uint64_t interactions[5];
    /* records handed to the next pass of the same type (0 photon, 1 electron):
     * particles still held by a wavefront at the tail of a large pass, or when
     * it switched jobs */
    uint64_t records_requeued[2];
    /* transport passes whose queue was re-binned by job first (every pass in
     * which more than one job holds particles), counted like passes */
    uint32_t passes_rebinned;
} gdpm_run_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `hip_device`.  opts_json may be NULL or a
 * flat JSON object with any of: "ring_capacity_log2" (queue records per type,
 * 2^k, default 25), "waves_per_cu" (wavefronts of the persistent workgroup
 * each CU runs, 1..12, default 12), "photon_waves_per_cu" (the same for the
 * photon pass alone, at most waves_per_cu, 0..12, default 0: waves_per_cu),
 * "rebin_bins" (bins per job of the queue re-binning, 0..64, default 1:
 * records are grouped by job only, which measured faster than energy order),
 * "rebin_space" (0, default: the bins are intervals of log2 E; 1: they are
 * boxes of the phantom, space^3 with space^3 the largest cube within the bins),
 * "rebin_photons", "rebin_electrons" (1: re-bin the queue of that particle type
 * also when a single job holds all the particles; default 0: then the queues
 * are read unsorted, which measured faster), "lds_tables" (1: stage
 * interpolation tables in LDS when they fit, together with each wavefront's
 * next claimed queue records, default; 0: read the tables through the caches
 * and load records directly), "pass_histories" (new histories started per
 * scheduler iteration, default 0 = half the queue capacity less what the
 * fuller queue holds; a larger
 * value can overflow the queues, which gdpm_run reports as GDPM_E_OVERFLOW).
 * Each wavefront reserves queue slots 256 at a time, so a queue needs well
 * over 256 slots per wavefront of the grid (2^21 and up on a 256-CU device
 * with 12 wavefronts per CU); smaller queues overflow.
 * "share" (how the jobs run together share the new histories of an iteration:
 * 1, the only value accepted, evenly; 0, oldest job first, is rejected with
 * GDPM_E_INVALID: a job taking the whole history budget of an iteration can
 * overflow the queues, whose budget assumes few secondaries per history),
 * "issue_order" (which jobs of a batch or server start their histories
 * first: 0, default, an even share of each iteration's budget for every job
 * still starting histories; 1, the job with the fewest histories left in its
 * planned super-round first, taking what it can use, then the next: shortest
 * remaining work first, so that a small job admitted beside a large one is
 * not slowed down by it; 2, the earliest admitted job first, taking what it
 * can use, then the next: arrival order, with later jobs filling the room an
 * earlier job leaves, e.g. while its super-round drains; a job's new
 * histories per iteration are bounded by its source in every order),
 * "autotune" (see gdpm_context_settings), "autotune_min_events" (transport
 * events, photon flights plus electron steps, an iteration must have for the
 * autotuner to score it; default 4000000), "graphs" (1, default: a
 * scheduler iteration's launches, copies included, are recorded as a HIP
 * graph the second time their launch configuration occurs in a run, and
 * replayed from then on, on the stream of the run; each run, batch or server
 * keeps its own recordings; 0: launched one by one),
 * "check_accounting" (1: after every iteration count each job's live queue
 * records on the device and compare them with its births less its deaths; a
 * disagreement is printed to stderr and counted in the run statistics; a
 * diagnostic, default 0), "ring_start" (queue position, 0 <= p < 2^32, at
 * which runs start; positions advance with every record and wrap modulo
 * 2^32, which a value near 2^32 brings forward; default 0),
 * "admit_draining" (servers: 1 admits a job only while every running job has
 * issued all the histories of its current super-round, 2 only while every
 * running job drains the super-round planned as its last (the one sized by
 * the sigma ~ N^-1/2 estimate to reach its target, or a fixed-count job's
 * only one), so that a new job fills the queues a running job leaves as it
 * drains instead of sharing the device with jobs large enough to fill it
 * alone; default 0: admission by slots and device footprint only), "solo_lanes" (1: a measurement form of
 * the transport kernels in which a wavefront carries one particle at a time,
 * so that it executes exactly the instructions of that particle's path; very
 * slow; needs "lds_tables" on and "autotune" off; default 0), "fused_passes"
 * (1: both transport passes of an iteration in one launch, the photon pass on
 * "photon_waves" wavefronts of each workgroup at first (default -1: half) and
 * the electron pass on the others, each wavefront turning to the other pass
 * when its own has nothing left; each pass then transports what its queue held
 * at the start of the iteration; needs the electron tables staged in LDS;
 * 0: the photon pass, then the electron pass).
 * Results do not depend on any of these options (each particle draws from its
 * own random stream), only the speed does. */
gdpm_status gdpm_context_create(int hip_device, const char* opts_json, gdpm_context* out);

/* The launch settings the context uses now, after any autotuning ("autotune":
 * 1 in opts_json makes gdpm_run_batch and servers size the queues from the
 * submitted work and try block sizes and energy-bin counts on the first
 * iterations, keeping the fastest for the rest of the run and for later runs
 * of the context).  out: waves_per_cu, rebin_bins, ring_capacity_log2,
 * pass_histories, autotune. */
gdpm_status gdpm_context_settings(gdpm_context ctx, int out[5]);
/* The autotuner's record of the context's latest tuned run (inspection):
 * *n candidates, the first min(cap, *n) written as (waves_per_cu, rebin_bins)
 * pairs to cand[2i], cand[2i+1] with their mean score in transport events
 * (photon flights and electron steps) per second of transport kernel time in
 * score[i] (0 while unmeasured); *kept is the index of the candidate kept for
 * the rest of the run, -1 while the tuner has not decided (and *n = 0 if no
 * tuned run happened). */
gdpm_status gdpm_context_tuning(gdpm_context ctx, int cap, int* n, int* cand, double* score,
                                int* kept);
gdpm_status gdpm_context_destroy(gdpm_context ctx);
const char* gdpm_last_error(void);

/* Material table shared by all phantoms of the context (ids 0..n-1, n <= 8).
 * n_grid: nodes of the interpolation grid uniform in ln E (256..8192; 0 ->
 * 1024).  Tables are generated from closed forms in double precision and
 * stored in single precision; interpolation is linear (section 2.2.2). */
gdpm_status gdpm_set_materials(gdpm_context ctx, const gdpm_material* m, int n, int n_grid);

/* ---- phantom ------------------------------------------------------------ */

/* nx, ny <= 2048, nz <= 1024 and nx*ny*nz <= 2^31 - 1 (the linear voxel index
 * is a signed 32-bit integer on the device); mat[v] < number of materials;
 * density[v] in [2^-16, 2^16) g/cm^3 (a voxel is stored in 4 bytes: the
 * density's exact single-precision value and the material).  Both arrays
 * (nx*ny*nz) are copied to device memory.  The sizes are checked before anything else (a NULL context with
 * bad sizes reports the sizes). */
gdpm_status gdpm_phantom_create(gdpm_context ctx, int nx, int ny, int nz, double dx, double dy,
                                double dz, const uint8_t* mat, const float* density,
                                gdpm_phantom* out);
gdpm_status gdpm_phantom_destroy(gdpm_phantom ph);

/* ---- source ------------------------------------------------------------- */

/* The descriptor and everything it points to are copied.  The beamlet
 * probabilities P(I) are normalised prefix sums of f_I in double precision. */
gdpm_status gdpm_source_create(gdpm_context ctx, const gdpm_source_desc* desc, gdpm_source* out);
gdpm_status gdpm_source_destroy(gdpm_source src);

/* ---- runs --------------------------------------------------------------- */

/* Blocking run.  dose and sigma: host arrays of nx*ny*nz doubles (either may
 * be NULL).  batch_edep: NULL or host n_batches*nx*ny*nz doubles receiving the
 * energy (MeV) deposited per batch and voxel.  hist_out: NULL or host
 * 2*n_histories doubles receiving (deposited, escaped) energy per history
 * (fixed mode only, n_histories <= 2^24).  stats may be NULL. */
gdpm_status gdpm_run(gdpm_context ctx, gdpm_phantom ph, gdpm_source src,
                     const gdpm_run_params* prm, double* dose, double* sigma,
                     double* batch_edep, double* hist_out, gdpm_run_stats* stats);

/* Same computation with device outputs: d_dose, d_sigma are device pointers
 * (nx*ny*nz doubles, e.g. a torch tensor's data_ptr()); work is ordered on
 * hip_stream (NULL = the context's own stream).  The call returns once the
 * work is queued or finished; gdpm_job_wait blocks until the outputs are
 * complete. */
gdpm_status gdpm_run_async(gdpm_context ctx, gdpm_phantom ph, gdpm_source src,
                           const gdpm_run_params* prm, double* d_dose, double* d_sigma,
                           void* hip_stream, gdpm_job* out);
/* Wait for a job of gdpm_run_async or of a server; returns the job's status
 * (its message through gdpm_last_error).  Releasing a server job that has not
 * finished returns GDPM_E_BUSY. */
gdpm_status gdpm_job_wait(gdpm_job job, gdpm_run_stats* stats);
gdpm_status gdpm_job_release(gdpm_job job);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * computation of gdpm_run_async, blocking (it returns once d_dose and d_sigma
 * are written, after a synchronisation of hip_stream), with nothing allocated
 * by the call.  The run's queues, control blocks, Woodcock majorant,
 * Metropolis chain states and batch tallies live in a static scratch array of
 * 512 MiB that every device the library runs on holds from the first context
 * created on it until the process ends; the caller still passes the outputs.
 * d_dose, d_sigma: device arrays of nx*ny*nz doubles (caller-owned, written in
 * full).  hip_stream: NULL = the context's stream.  stats may be NULL.
 * Limits (GDPM_E_INVALID beyond them, before any work): n_batches * nx*ny*nz
 * <= 33,423,360 (255 MiB of FP64 batch tallies: 10 batches of 3.3e6 voxels);
 * queues of 2^21 records per particle type (GDPM_E_OVERFLOW if a pass does not
 * fit, with the outputs invalid); no per-history or per-batch output; the
 * table set of the run's absorption energies and physics flags must be
 * resident (the default energies' set is made by gdpm_set_materials, any
 * other by a first run of another entry point with them), else
 * GDPM_E_INVALID.  Iterations are launched directly (no graph is recorded)
 * and the queues are never re-binned.  Every call on one device shares that
 * device's scratch array, which keeps the last call's contents (each call
 * clears what must start at zero): calls that overlap on one device, from any
 * context or thread, race and corrupt each other's results. */
gdpm_status gdpm_run_noalloc(gdpm_context ctx, gdpm_phantom ph, gdpm_source src,
                             const gdpm_run_params* prm, double* d_dose, double* d_sigma,
                             void* hip_stream, gdpm_run_stats* stats);

/* ---- many jobs ------------------------------------------------------------
 * Several dose jobs transported together: every kernel launch advances the
 * particles of all admitted jobs (shared photon and electron queues whose
 * records carry the job, one persistent grid per pass).  Each job keeps its
 * phantom, source, random key (seed, job_id), batches and statistics, and its
 * dose equals the dose of the same job run alone (the same particles draw the
 * same random numbers; only the order of the FP64 tally additions differs).
 * Jobs run together must use the same cutoffs and physics flags (bits 0-5);
 * the KERMA flag may differ.  In the returned gdpm_run_stats, histories,
 * e_in, e_dep, e_esc, unc_mean_over_dmax, dmax, rounds and t_total_s are the
 * job's own; events, passes, timings and the per-pass counters are totals of
 * the engine over the call. */

/* One job: handles of the caller's context; dose and sigma are host arrays of
 * nx*ny*nz doubles (either may be NULL), written when the job finishes. */
typedef struct {
    gdpm_phantom phantom;
    gdpm_source source;
    gdpm_run_params params;
    double* dose;
    double* sigma;
} gdpm_job_desc;

/* Blocking batched run of n jobs (n >= 1).  Up to 256 jobs are admitted at
 * once, more as earlier ones finish.  stats: NULL or n entries; status: NULL
 * or n entries receiving each job's result (GDPM_OK, GDPM_E_NOT_CONVERGED...).
 * Returns GDPM_OK when every job finished with GDPM_OK or
 * GDPM_E_NOT_CONVERGED, else the first other error (a device error or queue
 * overflow ends every job). */
gdpm_status gdpm_run_batch(gdpm_context ctx, int n, const gdpm_job_desc* jobs,
                           gdpm_run_stats* stats, gdpm_status* status);

/* ---- serving ---------------------------------------------------------------
 * A server owns the context's device (the context answers GDPM_E_BUSY to
 * other runs while the server exists) and runs a request loop on its own host
 * thread: queued jobs are admitted in arrival order while fewer than
 * max_slots jobs run and their device footprint (batch tallies, dose and
 * sigma, majorant) fits in hbm_budget_bytes (a job that alone exceeds the
 * budget is admitted when nothing else runs); admitted jobs share every
 * kernel launch (as in gdpm_run_batch) and each leaves as soon as its own
 * uncertainty target or history count is reached, freeing its slot and
 * memory for the next request.  Phantoms, sources and tables stay resident
 * on the device.  Jobs must share cutoffs and physics flags (bits 0-5) with
 * the first job submitted. */
typedef struct gdpm_server_s* gdpm_server;

typedef struct {
    uint64_t submitted, finished, running, queued;
    uint64_t histories;           /* histories of finished jobs */
    double footprint_bytes;       /* device bytes held by admitted jobs now */
    double high_water_bytes;      /* largest footprint_bytes so far */
    double resident_bytes;        /* queues, control blocks, tables, phantoms and
                                     sources of the context */
} gdpm_server_info;

/* max_slots in 1..256; hbm_budget_bytes > 0. */
gdpm_status gdpm_server_create(gdpm_context ctx, uint64_t hbm_budget_bytes, int max_slots,
                               gdpm_server* out);
/* Queue one job; returns at once.  The descriptor is copied; its handles and
 * host output arrays must stay valid until gdpm_job_wait returns.  The job's
 * gdpm_run_stats.t_total_s is its latency from submission to completion. */
gdpm_status gdpm_server_submit(gdpm_server srv, const gdpm_job_desc* job, gdpm_job* out);
gdpm_status gdpm_server_info_get(gdpm_server srv, gdpm_server_info* info);
/* Waits until every queued and running job has finished, then stops the
 * loop.  Job handles stay valid until gdpm_job_release. */
gdpm_status gdpm_server_destroy(gdpm_server srv);

/* ---- inspection and test entry points ------------------------------------
 * These expose the pieces of the transport so that tests can compare them
 * with an independent reference; they are not needed to compute dose. */

/* Host-only: build the interpolation tables for a material set and return
 * them.  which: 0 photon {muC, muPE, muPair, muTot} (cm^2/g) per material and
 * node of the photon grid; 1 electron {R (g/cm^2), muHard, muMoller,
 * 1/lambda1 (cm^2/g)} per material and node of the electron grid; 2 inverse
 * range E(w) on w = sqrt(R) per material; 3 MW screening log2 A on log2 t;
 * 4 Klein-Nishina inverse distribution function (section 2.1's Compton
 * scattering, material independent): ln(eps/eps0)/ln(1/eps0) of the eps =
 * E'/E at which the distribution function reaches u, on log2 E nodes (rows)
 * and u = j/(columns - 1), eps0 = 1/(1 + 2E/mc^2).
 * grid[0..3] receives (ln-grid start, spacing, node count, materials), for
 * which 4 (log2 E start, spacing, rows, columns).
 * out: cap floats; *len receives the number needed. */
gdpm_status gdpm_tables_host(const gdpm_material* m, int n, int n_grid, double ecut_g,
                             double ecut_e, uint32_t flags, int which, float* out, size_t cap,
                             size_t* len, double grid[4]);

/* Device Philox4x32-10 on n counters: key2 (2 words), ctr (4n words), out (4n
 * words); host arrays. */
gdpm_status gdpm_test_philox(gdpm_context ctx, const uint32_t key[2], const uint32_t* ctr,
                             uint32_t* out, int n);

/* Device samplers, n samples, sample i drawn from the stream of history i,
 * path 0 of `seed`: which 0 Compton (E) -> eps, cos; 1 Moller (T) -> W/T, cos
 * of the primary; 2 bremsstrahlung (T) -> k; 3 MW deflection (t) -> mu;
 * 4 multiple-scattering walk of (int)p2 hinges of t each -> Omega.Omega0;
 * 5 annihilation pair -> cos of photon 1, dir1.dir2; 6 pair production (E) ->
 * T-/(E - 2mc^2), T- + T+ - (E - 2mc^2) (0: the split is exact); 7 Compton (E)
 * -> cos of the electron, cos of the photon (against the incident direction).
 * out1/out2: host arrays of n floats (out2 may be NULL). */
gdpm_status gdpm_test_sample(gdpm_context ctx, int which, double e, double p1, double p2,
                             uint64_t seed, int n, float* out1, float* out2);

/* Device source sampling: n histories from hist0 of (seed, job); out: host
 * n*8 floats E, beamlet, x, y, z, u, v, w (beamlet -1 if the particle misses
 * the phantom). */
gdpm_status gdpm_test_source(gdpm_context ctx, gdpm_phantom ph, gdpm_source src, uint64_t seed,
                             uint32_t job, uint64_t hist0, int n, float* out);

/* Measured rate of scattered FP64 atomic additions (the tally's access
 * pattern, no transport) into a zeroed device array of `bytes` bytes
 * (8 B .. 16 GiB; the library allocates and frees it): *ops_per_s receives
 * additions per second of the second of two launches of 8 blocks of 256
 * threads per CU, 64 additions each.  GDPM_E_DEVICE if the array does not sum
 * to the additions made.  The peak against which the benchmark prices the
 * transport kernels' tally atomics. */
gdpm_status gdpm_test_atomic_rate(gdpm_context ctx, uint64_t bytes, double* ops_per_s);

/* Device table lookups at n energies for material mat (ecut/flags select the
 * table set): which 0 muTot photon, 1 R, 2 muHard, 3 muMoller, 4 1/lambda1,
 * 5 inverse range (input is R), 6 MW A (input is t). */
gdpm_status gdpm_test_lookup(gdpm_context ctx, double ecut_g, double ecut_e, uint32_t flags,
                             int which, int mat, const float* in, float* out, int n);

#ifdef __cplusplus
}
#endif
#endif /* GDPM_H */
