// Plain data shared by the host runtime and the HIP kernels of libgdpm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gdpm {

constexpr int kMaxMaterials = 8;
constexpr uint32_t kPushChunk = 256;    // ring slots a wavefront reserves at a time
constexpr uint32_t kClaimMin = 32;      // smallest and largest number of queue items a
constexpr uint32_t kClaimMax = 256;     // wavefront claims with one atomic
constexpr int kMaxBins = 64;            // energy bins of the queue re-binning
constexpr uint32_t kTailLanes = 32;     // a drained wavefront with fewer particles
                                        // than this hands them to the next pass ...
constexpr uint32_t kTailMinPerLane = 4; // ... if the pass had this many per lane

// event counters (same order as the GDPM_EV_* enumeration of the C ABI)
enum { EV_FLIGHTS = 0, EV_REAL, EV_ESTEPS, EV_HARD_CAND, EV_HARD, EV_DEPOSITS, EV_PUSHES,
       EV_HISTORIES };

// A particle record: 64 bytes, four 16-byte vectors.
struct alignas(16) Particle {
    float x, y, z, e;        // position (cm), kinetic energy (MeV); e < 0 marks an empty slot
    float u, v, w, nh;       // direction; hard-event mean free paths left (< 0: unset)
    uint32_t hlo, hhi;       // history id
    uint32_t path, ctr;      // Philox stream path id and draw counter
    uint32_t vox;            // charged particles: ix | iy << 11 | iz << 22
    float a;                 // positron: energy of its two annihilation photons together
    uint32_t flags;          // bit 0: positron
    uint32_t pad;
};
static_assert(sizeof(Particle) == 64, "particle record is 64 bytes");

// One queue (ring buffer of 2^k records, indices wrap modulo 2^32).
struct RingCtl {
    uint32_t head, tail;     // records in [head, tail)
    uint32_t begin, count;   // input of the running pass: [begin, begin + count)
    uint32_t claim;          // claim counter of the running pass
    uint32_t cur;            // which of the two buffers holds the ring
};

// Device-resident control block of a run.
struct Ctl {
    RingCtl ring[2];                  // 0 photons, 1 electrons/positrons
    uint32_t overflow;
    uint32_t pad0;
    unsigned long long ev[8];
    unsigned long long pass_ev[2][3];  // per pass type: records loaded, records
                                       // stored, tally deposits
    double e_in, e_esc;
    uint32_t bin_count[kMaxBins];
    uint32_t bin_cursor[kMaxBins];
    uint32_t n_valid;
    uint32_t pad1;
    double red[4];                    // statistics reductions
    unsigned long long dmax_bits;
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
};

struct Geom {
    const uint2* vox;      // {float bits of density, material id}
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
};

struct RunDev {
    uint32_t k0, k1;           // Philox key
    float ecut_g, ecut_e;
    uint32_t flags;
    uint32_t pad;
    double* tally;             // energy tally of the active batch slot (MeV per voxel)
    double* hist;              // per-history (deposited, escaped) or null
    unsigned long long hist0;
    Particle* buf[2][2];       // [ring][buffer]
    uint32_t mask[2];          // capacity - 1
    uint32_t hard[2];          // fill above which a reservation fails
};

}  // namespace gdpm
