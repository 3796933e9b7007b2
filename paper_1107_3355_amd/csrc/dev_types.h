// Plain data shared by the host runtime and the HIP kernels of libgdpm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

namespace gdpm {

constexpr int kMaxMaterials = 8;
constexpr uint32_t kPushChunk = 256;    // ring slots a wavefront reserves at a time
constexpr uint32_t kClaimMin = 32;      // smallest number of queue items a wavefront claims
                                        // with one atomic, and the largest, per particle type:
constexpr uint32_t kClaimMaxPhoton = 2048;   // a photon record lasts a few short iterations, so
constexpr uint32_t kClaimMaxElectron = 256;  // photon wavefronts claim often: larger chunks keep
                                             // them off the shared claim counter
constexpr int kMaxBins = 64;            // energy bins of the queue re-binning
constexpr int kMaxJobs = 256;           // dose jobs transported together
constexpr int kMaxKeys = 4096;          // re-binning keys (job x energy bin)
constexpr uint32_t kTailLanes = 16;     // a drained wavefront with fewer particles
                                        // than this hands them to the next pass ...
constexpr uint32_t kTailMinPerLane = 4; // ... if the pass had this many per lane
#ifndef GDPM_HARD_BATCH
#define GDPM_HARD_BATCH 12
#endif
constexpr uint32_t kHardBatch = GDPM_HARD_BATCH;  // electron hard events sampled together
#ifndef GDPM_REAL_BATCH
#define GDPM_REAL_BATCH 22
#endif
constexpr uint32_t kRealBatch = GDPM_REAL_BATCH;  // photon interactions sampled together
constexpr uint32_t kRefillMin = 12;     // empty lanes a wavefront refills at once
constexpr float kMaxEnergy = 1.0e6f;    // MeV; a larger or non-finite energy marks a
                                        // damaged record
constexpr uint32_t kMaxWaveIterations = 1u << 21;  // bound of a wavefront's loop in one
                                        // pass (about 1e3 in practice)

// event counters (same order as the GDPM_EV_* enumeration of the C ABI)
enum { EV_FLIGHTS = 0, EV_REAL, EV_ESTEPS, EV_HARD_CAND, EV_HARD, EV_DEPOSITS, EV_PUSHES,
       EV_HISTORIES };

// An empty queue position carries exactly this energy.  A particle's own
// energy never does: it is >= 0, or a rounding below 0 by a few ulps that the
// transport ends as an absorption, so such a record must still be read as a
// particle (an empty-slot test of e < 0 would lose it: born, never ended).
constexpr float kEmptyEnergy = -1.0f;
__host__ __device__ inline bool record_empty(float e) { return e == kEmptyEnergy; }

// A particle record: 64 bytes, four 16-byte vectors.
struct alignas(16) Particle {
    float x, y, z, e;        // position (cm), kinetic energy (MeV); kEmptyEnergy marks an empty slot
    float u, v, w, nh;       // direction; hard-event mean free paths left (< 0: unset)
    uint32_t hlo, hhi;       // history id
    uint32_t path, ctr;      // Philox stream path id and draw counter
    uint32_t vox;            // charged particles: ix | iy << 11 | iz << 22
    float a;                 // positron: energy of its two annihilation photons together
    uint32_t flags;          // bit 0: positron
    uint32_t job;            // bits 0-7: job slot; 8-15: the slot's generation; 16-31: batch slot
};
static_assert(sizeof(Particle) == 64, "particle record is 64 bytes");

// One queue (ring buffer of 2^k records, indices wrap modulo 2^32).
struct RingCtl {
    uint32_t head, tail;     // records in [head, tail)
    uint32_t begin, count;   // input of the running pass: [begin, begin + count)
    uint32_t claim;          // claim counter of the running pass
    uint32_t permuted;       // 1: the pass reads its input through the permutation
    uint32_t next_head;      // head after a permuted pass (the tail before it)
};

// Device-resident control block of the transport (the host reads it back
// after every scheduler iteration).
struct Ctl {
    RingCtl ring[2];                  // 0 photons, 1 electrons/positrons
    uint32_t overflow;
    uint32_t n_valid;                 // records kept by the last compaction
    unsigned long long ev[8];
    unsigned long long pass_ev[2][4];  // per pass type: records loaded, records
                                       // stored, tally deposits, records handed
                                       // to the next pass of the same type
    unsigned long long itype[5];      // real interactions: Compton, photoelectric,
                                       // pair, Moller, bremsstrahlung
    double red[4];                    // statistics reductions
    unsigned long long dmax_bits;
    unsigned long long anomalies;     // particles ended by a loop bound (0 in a sound run)
};

// Per-job counters and the job segments of the running pass.  The first four
// arrays are read back by the host after every iteration: a job whose births
// equal its deaths has no particle left in the queues.
struct JobCtl {
    unsigned long long births[kMaxJobs];   // queue records created (primaries, secondaries)
    unsigned long long deaths[kMaxJobs];   // particles ended (absorbed, escaped)
    double e_in[kMaxJobs];                 // source kinetic energy (MeV)
    double e_esc[kMaxJobs];                // energy leaving the phantom (MeV)
    // per particle type [ri] (the two passes of an iteration may run at once):
    uint32_t seg_begin[2][kMaxJobs];       // the job's records in the pass input:
    uint32_t seg_count[2][kMaxJobs];       //   [seg_begin, seg_begin + seg_count)
    uint32_t claim[2][kMaxJobs];           // claim counter of the job's segment
    unsigned long long left[2][kMaxJobs / 64];  // jobs with unclaimed records
    uint32_t bin_count[kMaxKeys];
    uint32_t bin_cursor[kMaxKeys];
};

// Interpolation tables (single precision, linear in log2 E).
struct Tables {
    const float4* phot;    // [mat][pg_n] {muC, muPE, muPair, muTot} cm^2/g
    const float* mumax;    // [pg_n] Woodcock majorant of the phantom, 1/cm
    float pg_lo, pg_inv;   // node i at log2 E = pg_lo + i / pg_inv
    int pg_n;
    const float4* elec;    // [mat][eg_n] {R g/cm^2, muHard, muMoller, 1/lambda1 cm^2/g}
    float eg_lo, eg_inv;
    int eg_n;
    const float* rinv;     // [mat][nr] E at w = sqrt(R), w uniform from 0
    const float* rinv_scale;  // [mat] (nr - 1) / w_max
    int nr;
    const float* aw;       // [aw_n] log2 A at log2 t = aw_lo + i / aw_inv
    float aw_lo, aw_inv;
    int aw_n;
    int n_mat;
    const float* kn;       // [kn_ne][kn_nu] Klein-Nishina inverse: ln(eps/eps0)/ln(1/eps0)
    float kn_lo, kn_inv;   // at log2 E = kn_lo + i / kn_inv and u = j / (kn_nu - 1)
    int kn_ne, kn_nu;
};

// A voxel of the phantom in 4 bytes: the density's single-precision mantissa
// (bits 0-22), its exponent less kVoxExpBias (bits 23-27: densities in
// [2^-16, 2^16) g/cm^3, every single-precision value there exactly) and the
// material id (bits 28-31).  Half the bytes of a {density, material} pair, so
// the random voxel gathers of the transport touch half the cache lines.
constexpr uint32_t kVoxExpBias = 111u;   // single-precision exponent field of 2^-16
static_assert(kMaxMaterials <= 16, "material ids take 4 bits of a packed voxel");
__host__ __device__ inline bool voxel_density_ok(float rho) {
    const float lo = 1.0f / 65536.0f, hi = 65536.0f;
    return rho >= lo && rho < hi;
}
__host__ __device__ inline uint32_t pack_voxel(float rho, uint32_t mat) {
    uint32_t bits;
    memcpy(&bits, &rho, 4);
    return (bits - (kVoxExpBias << 23)) | (mat << 28);
}
__host__ __device__ inline float voxel_density(uint32_t w) {
    const uint32_t bits = (w & 0x0FFFFFFFu) + (kVoxExpBias << 23);
    float r;
    memcpy(&r, &bits, 4);
    return r;
}
__host__ __device__ inline int voxel_material(uint32_t w) { return (int)(w >> 28); }

struct Geom {
    const uint32_t* vox;   // packed voxels (pack_voxel)
    int nx, ny, nz;
    float dx, dy, dz;
    float idx, idy, idz;   // 1 / voxel size
    float lx, ly, lz;      // extent
};

struct BeamDev {
    float iso[3], dir[3], e1[3], e2[3];
    float sad, bw, bh, hx, hy;   // hx = nbx * bw / 2, hy = nby * bh / 2
    int nbx, nby, off;
};

struct SourceDev {
    int particle, spec_kind, spec_n;
    float e_mono;
    const float* spec_e;
    const float* spec_p;
    const float* spec_c;       // cumulative area at spec_e
    const double* cdf;         // nf + 1 beamlet probabilities P(I)
    int nf;
    const uint32_t* guide;     // guide[k]: I with P(I) <= k / n_guide (start of the search)
    int n_guide;
    const BeamDev* beams;
    const uint16_t* beam_of;   // beamlet -> beam
    int n_beams;
    int metro;                 // 1: Metropolis beamlet chains (Algorithm A1)
    int n_nz;                  // beamlets of nonzero intensity ...
    const uint32_t* nz;        // ... their indices
    const float* f;            // [nf] intensities (negative ones as 0)
    int strata;                // K > 0: energy intervals of a round (section 2.3.2)
    const double* strata_F;    // [K + 1] spectrum CDF at the interval edges
    int strata_shape;          // inside an interval: 0 uniform energy, 1 the spectrum's shape
    float strata_lo, strata_w; // lower edge of the first interval, interval width (MeV)
    const float* phsp;         // [n_phsp][7] phase-space records, or null (section 2.3.3)
    unsigned long long n_phsp;
};

constexpr uint32_t kMetroChains = 16384;   // Metropolis chains of a job

// One dose job: its phantom, source, random key and tallies.
struct JobDev {
    Geom G;
    SourceDev S;
    const float* mumax;        // [pg_n] Woodcock majorant of the job's phantom, 1/cm
    double* tally;             // [n_batches][nv] energy tallies (MeV per voxel)
    unsigned long long nv;     // voxels of the phantom
    double* hist;              // per-history (deposited, escaped) or null
    unsigned long long hist0;  // history id of hist[0]
    uint32_t k0, k1;           // Philox key
    uint32_t flags;            // GDPM_* run flags
    uint32_t gen;              // generation of the slot (8 bits): records of an earlier
                               // job in the same slot carry another one
    uint32_t* chains;          // [kMetroChains] Metropolis chain states, or null
    uint32_t split;            // primary splitting: 2^split copies of each history's primary
                               // (tallied at weight 1; the host scales the job's sums by 2^-split)
};

// A run of new histories for the source pass: ids [h0, h0 + n) of job `job`,
// batch slot `batch`, written to queue slots tail + off + i.
struct SrcSeg {
    unsigned long long h0;
    uint32_t n, off;
    uint32_t job, batch;
    uint32_t rpos, rsize;      // position of h0 in its round, and the round's size
};

// the source pass of one particle type in one scheduler iteration: segments
// and histories; read by the kernels from device memory, so that a recorded
// launch sequence stays valid while these change
struct SrcHdr {
    uint32_t nseg, total;
    uint32_t pad0, pad1;
};

// The re-binning leaves the records where they are.  Each queue has a
// re-binning buffer of 2C 32-bit words, C the queue capacity: each input
// position's key (kEmptyKey for an empty position, kOrphanKey for a record of a
// job no longer running), then the permutation, the queue positions of the
// pass's input in key order, which the pass reads its input through.
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu, kOrphanKey = 0xFFFFFFFEu;
constexpr size_t kBinWordsPerSlot = 2;
__host__ __device__ inline uint32_t* bin_keys(uint32_t* bin) { return bin; }
__host__ __device__ inline uint32_t* bin_perm(uint32_t* bin, uint32_t mask) { return bin + ((size_t)mask + 1u); }

struct RunDev {
    float ecut_g, ecut_e;      // shared by every job (the tables depend on them)
    const JobDev* jobs;
    JobCtl* jc;
    int n_jobs;                // job slots in use
    int nb;                    // energy bins per job of the re-binning
    Particle* buf[2];          // the queues' records [ring]
    uint32_t* bin[2];          // their re-binning buffers (2 words per queue slot), or null
    uint32_t mask[2];          // capacity - 1
    uint32_t hard[2];          // fill above which a reservation fails
};

}  // namespace gdpm
