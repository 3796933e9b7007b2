// Host runtime behind the C ABI of include/gdpm.h: device resources, the pass
// scheduler and the batch statistics.
//
// Scheduling follows the paper's batch loop (section 2.2.1, Fig. 1): histories
// are split into N_b batches; within a batch the photon and electron kernels
// alternate until the source is exhausted and both secondary queues are empty;
// per-voxel mean dose and its uncertainty come from the batch tallies.  Here a
// batch slot is filled by one or more rounds of histories, the queues are ring
// buffers sized for HBM, and the host only reads a few counters between passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <tuple>
#include <vector>

#include "gdpm.h"
#include "dev_types.h"
#include "tables.h"

namespace gdpm {
hipError_t launch_setup(hipStream_t st, Ctl* ctl, const RunDev& R, int ri, int rebinned, int lone);
hipError_t launch_source(hipStream_t st, int blocks, Ctl* ctl, const RunDev& R, const SrcSeg* segs,
                         const SrcHdr* hdr, int ri);
hipError_t launch_finish(hipStream_t st, Ctl* ctl, int ri);
size_t transport_lds_bytes(int ri, const Tables& T, int waves);
hipError_t transport_lds_optin(size_t bytes);
hipError_t launch_transport(hipStream_t st, int ri, int blocks, int threads, bool lds, bool solo, bool permuted,
                            Ctl* ctl, const Tables& T, const RunDev& R);
hipError_t launch_rebin(hipStream_t st, int blocks, Ctl* ctl, const RunDev& R, int ri, int nb,
                        float lo, float inv, int space);
hipError_t launch_fused(hipStream_t st, int blocks, int threads, int photon_waves, bool permuted, Ctl* ctl,
                        const Tables& T, const RunDev& R);
hipError_t launch_count_records(hipStream_t st, int blocks, const Ctl* ctl, const RunDev& R,
                                unsigned long long* counts);
hipError_t launch_stats(hipStream_t st, int blocks, Ctl* ctl, const double* slots, size_t nvox,
                        int nb, const double* inv_n, const uint32_t* vox, double vvox, float min_rho,
                        double* dose, double* sigma);
hipError_t launch_test_philox(hipStream_t st, uint32_t k0, uint32_t k1, const uint4* ctr, uint4* out,
                              int n);
hipError_t launch_test_sample(hipStream_t st, const Tables& T, int which, float e, float p1, float p2,
                              uint32_t k0, uint32_t k1, int n, float* out1, float* out2);
hipError_t launch_test_source(hipStream_t st, const SourceDev& S, const Geom& G, uint32_t k0,
                              uint32_t k1, unsigned long long hist0, int n, float* out);
hipError_t launch_test_lookup(hipStream_t st, const Tables& T, int which, int m, const float* in,
                              float* out, int n);
hipError_t launch_atomic_rate(hipStream_t st, int blocks, double* buf, uint32_t n, uint32_t iters);
hipError_t launch_metro_init(hipStream_t st, const SourceDev& S, uint32_t k0, uint32_t k1, uint32_t* chains);
}  // namespace gdpm

using namespace gdpm;

// ---------------------------------------------------------------------------
// scratch memory of the allocation-free entry point (gdpm_run_noalloc): one
// array per device, held from the library's first use on that device until the
// process ends.  Host code never uses the array's name as an address: each
// device's address comes from hipGetSymbolAddress at context creation.
// Layout: control blocks, majorant and chain states (1 MiB), the two particle
// queues of 2^21 records each (256 MiB), then the batch tallies (255 MiB).
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = (size_t)512 << 20;
constexpr int kScratchRingLog2 = 21;
constexpr size_t kScratchCtlBytes = (size_t)1 << 20;
constexpr size_t kScratchRingBytes = ((size_t)1 << kScratchRingLog2) * sizeof(Particle);
constexpr size_t kScratchTallyBytes = kScratchBytes - kScratchCtlBytes - 2 * kScratchRingBytes;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
// each device's address of `scratch`, looked up once per device with that
// device current (every device holds its own copy of the array)
std::mutex g_scratch_mutex;
std::map<int, unsigned char*> g_scratch_addr;

hipError_t scratch_address(int device, unsigned char** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    *out = static_cast<unsigned char*>(p);
    g_scratch_addr[device] = *out;
    return hipSuccess;
}
}  // namespace

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_err;

gdpm_status fail(gdpm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? GDPM_E_NOMEM : GDPM_E_DEVICE, "%s: %s",  \
                        #call, hipGetErrorString(e_));                                       \
    } while (0)

// device allocation owned by a unique_ptr-like holder
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t n) {
        reset();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) bytes = n;
        else p = nullptr;
        return e;
    }
    hipError_t ensure(size_t n) { return n <= bytes ? hipSuccess : alloc(n); }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

template <class T>
hipError_t upload(DevBuf& b, const std::vector<T>& v) {
    hipError_t e = b.alloc(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    return hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

struct TableKey {
    double ecut_g, ecut_e;
    uint32_t flags;
    bool operator<(const TableKey& o) const {
        return std::tie(ecut_g, ecut_e, flags) < std::tie(o.ecut_g, o.ecut_e, o.flags);
    }
};

struct DevTables {
    HostTables host;
    DevBuf phot, elec, rinv, rinv_scale, aw, kn;
    Tables view(const float* mumax) const {
        Tables t;
        t.phot = phot.as<const float4>();
        t.mumax = mumax;
        t.pg_lo = (float)host.pg_lo;
        t.pg_inv = (float)(1.0 / host.pg_step);
        t.pg_n = host.pg_n;
        t.elec = elec.as<const float4>();
        t.eg_lo = (float)host.eg_lo;
        t.eg_inv = (float)(1.0 / host.eg_step);
        t.eg_n = host.eg_n;
        t.rinv = rinv.as<const float>();
        t.rinv_scale = rinv_scale.as<const float>();
        t.nr = host.nr;
        t.aw = aw.as<const float>();
        t.aw_lo = (float)host.aw_lo;
        t.aw_inv = (float)(1.0 / host.aw_step);
        t.aw_n = host.aw_n;
        t.n_mat = host.n_mat;
        t.kn = kn.as<const float>();
        t.kn_lo = (float)host.kn_lo;
        t.kn_inv = (float)(1.0 / host.kn_step);
        t.kn_ne = host.kn_ne;
        t.kn_nu = host.kn_nu;
        return t;
    }
};

int json_int(const char* js, const char* key, int dflt) {
    if (!js) return dflt;
    std::string k = std::string("\"") + key + "\"";
    const char* p = strstr(js, k.c_str());
    if (!p) return dflt;
    p = strchr(p + k.size(), ':');
    if (!p) return dflt;
    return atoi(p + 1);
}

unsigned long long json_u64(const char* js, const char* key, unsigned long long dflt) {
    if (!js) return dflt;
    std::string k = std::string("\"") + key + "\"";
    const char* p = strstr(js, k.c_str());
    if (!p) return dflt;
    p = strchr(p + k.size(), ':');
    if (!p) return dflt;
    return strtoull(p + 1, nullptr, 10);
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
// Everything that fixes one scheduler iteration's launch sequence (grids,
// kernel arguments, copy sizes); equal keys replay the same recorded graph.
// Compared bytewise: built on a zeroed object.
struct StepGraphKey {
    hipStream_t st;
    int seg_copy[2];     // source segments copied per particle type (0: no source pass)
    int src_blocks[2];
    int rebin[2], lds[2];
    int lone;            // the one job holding particles (queues not re-binned), or -1
    int blocks, threads, nb, space;
    int threads_photon;        // block size of the photon pass (separate launches)
    int fused, photon_waves;   // both passes in one launch; its photon-first wavefronts
    float blo, binv;
    RunDev R;
    Tables T;
};
struct StepGraph {
    StepGraphKey key;
    hipGraphExec_t exec;   // null: seen once, not recorded yet
    uint64_t last_use;
};

struct gdpm_context_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    int ring_log2 = 25;
    int waves_per_cu = 12;
    int rebin_bins = 1;          // bins per job of the re-binning (1: by job only)
    int rebin_space = 0;         // 1: the bins are boxes of the phantom, not energy intervals
    int lds_tables = 1;          // stage interpolation tables in LDS when they fit
    int pass_histories = 0;      // new histories per iteration (0: half a queue less its fill)
    int autotune = 0;            // tune block size and re-binning online, queues from the work
    int autotune_min_events = 4000000;   // transport events an iteration needs to be scored
    int share = 1;               // new histories: evenly over the jobs (the only policy)
    int issue_order = 0;         // 0 even shares, 1 least work left first, 2 admission order first
    int rebin_photons = 0;       // 1: re-bin the photon queue also when one job holds all particles
    int rebin_electrons = 0;     // 1: the same for the electron queue
    int graphs = 1;              // replay each iteration's launches as a recorded HIP graph
    int check_accounting = 0;    // after every iteration, count each job's live records
    int solo_lanes = 0;          // measurement form: one particle per wavefront at a time
    int fused_passes = 0;        // 1: both passes of an iteration in one launch (k_transport)
    int photon_waves_per_cu = 0; // wavefronts per CU of the photon pass (at most
                                 // waves_per_cu; 0: waves_per_cu)
    int photon_waves = -1;       // wavefronts per workgroup that start with photons (fused; -1: half)
    int admit_draining = 0;      // server: admit a job only while every running job drains (1: any
                                 // super-round, 2: its last one)
    uint32_t ring_start = 0;     // queue position a run starts at (positions run modulo 2^32)
    int max_lds = 0;             // dynamic LDS bytes a workgroup may use
    bool lds_optin = false;
    std::vector<MaterialParams> mats;
    int n_grid = 1024;
    std::map<TableKey, std::unique_ptr<DevTables>> tables;
    DevBuf rings[2];   // the queues' records
    DevBuf bins[2];    // their re-binning buffers
    DevBuf ctl;
    Ctl* host_ctl = nullptr;   // pinned mirror
    DevBuf jobs_dev, jc, segs, inv_n, counts;
    JobDev* h_jobs = nullptr;  // pinned: job table, source segments, the read-back
    SrcSeg* h_segs = nullptr;  // part of the job counters, statistics reductions
    DevBuf src_hdr;            // per particle type: segments and histories of the
    SrcHdr* h_hdr = nullptr;   // iteration's source pass (device, pinned host)
    void* h_jc = nullptr;
    double* h_red = nullptr;
    double resident_bytes = 0.0;   // phantoms and sources alive in the context
    unsigned char* scratch = nullptr;  // this device's scratch array (gdpm_run_noalloc)
    // the autotuner's latest record: candidates, mean scores, the one kept (-1: undecided)
    std::vector<std::pair<int, int>> tune_cand;
    std::vector<double> tune_score;
    int tune_kept = -1;
    std::vector<hipEvent_t> events;
    bool busy = false;
};

struct gdpm_phantom_s {
    gdpm_context ctx;
    int nx, ny, nz;
    double dx, dy, dz;
    DevBuf vox;
    std::vector<double> rho_max;   // per material, 0 if absent
};

struct gdpm_source_s {
    gdpm_context ctx;
    int particle;
    double e_max;
    int spec_kind, spec_n;
    float e_mono;
    DevBuf spec_e, spec_p, spec_c, cdf, guide, beams, beam_of;
    DevBuf fl, nz;               // intensities and nonzero beamlets (Metropolis chains)
    DevBuf strata_F;             // spectrum CDF at the energy-interval edges
    DevBuf phsp;                 // phase-space records (the open source interface)
    unsigned long long n_phsp = 0;
    int nf, n_guide, n_beams;
    int metro = 0, n_nz = 0, strata = 0, strata_shape = 0;
    float strata_lo = 0.0f, strata_w = 0.0f;   // lower edge and width of the intervals
    SourceDev view() const {
        SourceDev s;
        s.particle = particle;
        s.spec_kind = spec_kind;
        s.spec_n = spec_n;
        s.e_mono = e_mono;
        s.spec_e = spec_e.as<const float>();
        s.spec_p = spec_p.as<const float>();
        s.spec_c = spec_c.as<const float>();
        s.cdf = cdf.as<const double>();
        s.nf = nf;
        s.guide = guide.as<const uint32_t>();
        s.n_guide = n_guide;
        s.beams = beams.as<const BeamDev>();
        s.beam_of = beam_of.as<const uint16_t>();
        s.n_beams = n_beams;
        s.metro = metro;
        s.n_nz = n_nz;
        s.nz = nz.as<const uint32_t>();
        s.f = fl.as<const float>();
        s.strata = strata;
        s.strata_F = strata_F.as<const double>();
        s.strata_shape = strata_shape;
        s.strata_lo = strata_lo;
        s.strata_w = strata_w;
        s.phsp = phsp.as<const float>();
        s.n_phsp = n_phsp;
        return s;
    }
};


namespace {

constexpr int kMaxBlockThreads = 768;   // launch bound of the transport kernels
constexpr int kMaxSegs = 4096;          // source segments per iteration (both types)
constexpr int kMaxBatches = 1000;       // N_b of a job
constexpr int kMaxGrid = 8192;          // nodes of an interpolation grid
constexpr size_t kMaxStepGraphs = 32;   // launch settings an engine remembers
uint64_t pow2_at_least(uint64_t n, uint64_t lo) {
    uint64_t p = lo;
    while (p < n) p <<= 1;
    return p;
}
// the host reads back the first four arrays of JobCtl after every iteration
struct JobCtlMirror {
    unsigned long long births[kMaxJobs], deaths[kMaxJobs];
    double e_in[kMaxJobs], e_esc[kMaxJobs];
};
constexpr size_t kJcMirrorBytes = sizeof(JobCtlMirror);
static_assert(offsetof(JobCtl, seg_begin) == kJcMirrorBytes, "JobCtl starts with the read-back arrays");

Geom geom_of(const gdpm_phantom_s* ph) {
    Geom g;
    g.vox = ph->vox.as<const uint32_t>();
    g.nx = ph->nx;
    g.ny = ph->ny;
    g.nz = ph->nz;
    g.dx = (float)ph->dx;
    g.dy = (float)ph->dy;
    g.dz = (float)ph->dz;
    g.idx = (float)(1.0 / ph->dx);
    g.idy = (float)(1.0 / ph->dy);
    g.idz = (float)(1.0 / ph->dz);
    g.lx = (float)(ph->nx * ph->dx);
    g.ly = (float)(ph->ny * ph->dy);
    g.lz = (float)(ph->nz * ph->dz);
    return g;
}

gdpm_status get_tables(gdpm_context ctx, double ecut_g, double ecut_e, uint32_t flags,
                       DevTables** out) {
    if (ctx->mats.empty()) return fail(GDPM_E_INVALID, "no materials set");
    TableKey key{ecut_g, ecut_e, flags & 0x3Fu};
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) {
        *out = it->second.get();
        return GDPM_OK;
    }
    auto t = std::make_unique<DevTables>();
    std::string err;
    if (!build_tables(ctx->mats, ctx->n_grid, ecut_g, ecut_e, key.flags, &t->host, &err))
        return fail(GDPM_E_INVALID, "%s", err.c_str());
    HIP_TRY(upload(t->phot, t->host.phot));
    HIP_TRY(upload(t->elec, t->host.elec));
    HIP_TRY(upload(t->rinv, t->host.rinv));
    HIP_TRY(upload(t->rinv_scale, t->host.rinv_scale));
    HIP_TRY(upload(t->aw, t->host.aw));
    HIP_TRY(upload(t->kn, t->host.kn));
    *out = t.get();
    ctx->tables[key] = std::move(t);
    return GDPM_OK;
}

gdpm_status ensure_rings(gdpm_context ctx) {
    const size_t cap = (size_t)1 << ctx->ring_log2;
    for (int r = 0; r < 2; ++r) {
        HIP_TRY(ctx->rings[r].ensure(cap * sizeof(Particle)));
        HIP_TRY(ctx->bins[r].ensure(cap * kBinWordsPerSlot * sizeof(uint32_t)));
    }
    return GDPM_OK;
}

// The device memory an engine runs in: the context's own buffers (queues
// sized by ring_capacity_log2, each with its re-binning buffer), or fixed
// memory given to the engine (no re-binning buffer: such an engine never
// re-bins, records no graph and allocates nothing).
struct EngineMem {
    Particle* ring[2];
    uint32_t* bin[2];
    int ring_log2;
    Ctl* ctl;
    JobDev* jobs;
    JobCtl* jc;
    SrcSeg* segs;
    SrcHdr* hdr;
    double* inv_n;                 // kMaxBatches doubles
    unsigned long long* counts;    // kMaxJobs counters
    bool fixed;                    // given memory: no allocation, no graph, no re-binning
};

gdpm_status context_mem(gdpm_context ctx, EngineMem* m) {
    gdpm_status e = ensure_rings(ctx);
    if (e) return e;
    memset(m, 0, sizeof *m);
    for (int r = 0; r < 2; ++r) {
        m->ring[r] = ctx->rings[r].as<Particle>();
        m->bin[r] = ctx->bins[r].as<uint32_t>();
    }
    m->ring_log2 = ctx->ring_log2;
    m->ctl = ctx->ctl.as<Ctl>();
    m->jobs = ctx->jobs_dev.as<JobDev>();
    m->jc = ctx->jc.as<JobCtl>();
    m->segs = ctx->segs.as<SrcSeg>();
    m->hdr = ctx->src_hdr.as<SrcHdr>();
    m->inv_n = ctx->inv_n.as<double>();
    m->counts = ctx->counts.as<unsigned long long>();
    m->fixed = false;
    return GDPM_OK;
}

// persistent transport grid: one workgroup of waves_per_cu wavefronts per CU
int grid_blocks(gdpm_context ctx) { return std::max(1, ctx->cu_count); }
int block_threads(gdpm_context ctx) { return std::min(kMaxBlockThreads, 64 * ctx->waves_per_cu); }

// ---------------------------------------------------------------------------
// one run
// ---------------------------------------------------------------------------
struct RunPlan {
    uint64_t n_hist;
    int nb;
    int split;          // primary splitting: 2^split copies per history
    double ecut_g, ecut_e;
    uint32_t flags;
    bool target;
};

gdpm_status validate_params(const gdpm_run_params* p, const gdpm_source_s* src, RunPlan* plan) {
    if (!p) return fail(GDPM_E_INVALID, "run parameters are NULL");
    plan->nb = p->n_batches == 0 ? 10 : p->n_batches;
    if (plan->nb < 2 || plan->nb > kMaxBatches)
        return fail(GDPM_E_INVALID, "n_batches must be in [2, %d]", kMaxBatches);
    plan->ecut_g = p->ecut_photon_mev == 0.0 ? 0.05 : p->ecut_photon_mev;
    plan->ecut_e = p->ecut_electron_mev == 0.0 ? 0.2 : p->ecut_electron_mev;
    if (!(plan->ecut_g > 0.0 && plan->ecut_g < 1.0) || !(plan->ecut_e > 0.0 && plan->ecut_e < 5.0))
        return fail(GDPM_E_INVALID, "absorption energies out of range");
    plan->target = p->target_unc > 0.0;
    if (!(p->target_unc >= 0.0) || !std::isfinite(p->target_unc))
        return fail(GDPM_E_INVALID, "target_unc must be finite and >= 0");
    if (p->n_histories == 0) return fail(GDPM_E_INVALID, "n_histories must be > 0");
    if (p->n_histories > ((uint64_t)1 << 48)) return fail(GDPM_E_INVALID, "n_histories too large");
    plan->n_hist = p->n_histories;
    plan->flags = p->flags;
    if (p->flags & ~0x7Fu) return fail(GDPM_E_INVALID, "unknown flag bits");
    if (!(p->stat_min_density >= 0.0) || !std::isfinite(p->stat_min_density))
        return fail(GDPM_E_INVALID, "stat_min_density must be finite and >= 0");
    if (src->particle == 1 && (p->flags & GDPM_KERMA))
        return fail(GDPM_E_INVALID, "kerma mode needs a photon source");
    if (p->split_log2 < 0 || p->split_log2 > 6) return fail(GDPM_E_INVALID, "split_log2 in [0, 6]");
    plan->split = p->split_log2;
    return GDPM_OK;
}

struct Timers {
    double photon = 0, electron = 0;
    double fused = 0;   // both passes in one launch
    uint32_t passes = 0, passes_photon = 0, passes_electron = 0;
    uint32_t graph_launches = 0, graphs_recorded = 0;
    uint32_t passes_rebinned = 0;
};

// ---------------------------------------------------------------------------
// the transport engine: up to kMaxJobs dose jobs share the particle queues and
// every kernel launch.  Each job keeps its own phantom, source, random key,
// batch tallies and statistics; a job's results do not depend on which other
// jobs run beside it (its particles draw only from the job's own streams).
//
// Batches follow the paper's scheme (section 2.2.1): a job's histories are cut
// into super-rounds of N_b rounds, round b of a super-round feeding batch
// slot b.  Records carry their batch slot, so rounds and jobs overlap in the
// queues; a super-round is complete when all its histories were started and
// the job's particle births equal its deaths.
// ---------------------------------------------------------------------------
struct EJob {
    gdpm_phantom_s* ph = nullptr;
    gdpm_source_s* src = nullptr;
    gdpm_run_params prm{};
    RunPlan plan{};
    int slot = -1;
    size_t nv = 0;
    DevBuf tally, mumax, hist, dose_buf, sigma_buf;
    DevBuf chains;               // Metropolis chain states of the job's source
    // the job's device arrays: set by admit() from the buffers above, or given
    // beforehand (an engine on fixed memory)
    double* tally_p = nullptr;
    float* mumax_p = nullptr;
    uint32_t* chains_p = nullptr;
    double* d_dose = nullptr;   // outputs in device memory
    double* d_sigma = nullptr;
    uint64_t hbase = 0;         // id of the job's first history
    uint64_t issued = 0;        // histories started (relative ids [0, issued))
    uint64_t sr_start = 0, sr_end = 0;  // the running super-round
    bool sr_final = false;              // planned as the job's last super-round
    uint64_t round_size = 0;
    uint64_t max_hist = 0;
    std::vector<double> nhist;  // histories per batch slot
    uint32_t rounds = 0;
    double unc = 0, dmax = 0, edep = 0, e_in = 0, e_esc = 0;
    unsigned long long births = 0, deaths = 0;
    long long death_offset = 0;   // counter repairs (see Engine::settle)
    uint32_t repairs = 0;
    gdpm_status status = GDPM_OK;
    bool done = false;
    std::string err;
    double t_submit = 0, t_admit = 0, t_done = 0;
    uint64_t seq = 0;           // admission order
    size_t footprint = 0;       // device bytes the job owns while admitted
};

size_t job_footprint(const gdpm_phantom_s* ph, const RunPlan& plan, bool own_outputs, int pg_n) {
    const size_t nv = (size_t)ph->nx * ph->ny * ph->nz;
    return (size_t)plan.nb * nv * sizeof(double) + (own_outputs ? 2 * nv * sizeof(double) : 0) +
           (size_t)pg_n * sizeof(float);
}

struct Engine {
    gdpm_context ctx = nullptr;
    hipStream_t st = nullptr;
    EngineMem M{};              // device memory of the engine's queues and control blocks
    DevTables* tab = nullptr;
    TableKey key{};
    RunDev R{};
    Tables T{};
    std::vector<EJob*> slots;
    int n_slots = 0;            // slots in use: [0, n_slots)
    std::vector<uint32_t> slot_gen = std::vector<uint32_t>(kMaxJobs, 0u);   // 8-bit generations
    Timers tm;
    uint32_t iter = 0, idle = 0;
    StepGraphKey last{};        // launch settings of the latest iteration
    // recorded iterations, by launch settings; an engine records and replays
    // them on the one thread that drives it, and they end with it
    std::vector<StepGraph> graphs;
    uint64_t graph_clock = 0;
    Engine() = default;
    Engine(const Engine&) = delete;
    Engine& operator=(const Engine&) = delete;
    ~Engine() { drop_graphs(); }
    void drop_graphs() {
        for (auto& g : graphs)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    uint32_t mismatches = 0;    // iterations whose record count disagreed (check_accounting)
    gdpm_status check_accounting();
    uint64_t admitted = 0;
    // online autotuning: launch settings change nothing in the results, so
    // candidate (waves per CU, energy bins) pairs are tried on live iterations
    // and the fastest, in transport events per kernel second, is kept
    struct Tuner {
        bool on = false, fixed = false;
        std::vector<std::pair<int, int>> cand;
        std::vector<double> score;
        std::vector<int> samples;
        int cur = 0;
        unsigned long long last_events = 0;
        double last_time = 0.0;
    } tune;
    void tune_begin();
    void tune_account();

    gdpm_status init(gdpm_context c, hipStream_t s, const RunPlan& plan, const EngineMem* mem = nullptr);
    gdpm_status admit(EJob* j);
    gdpm_status step();
    gdpm_status issue(const StepGraphKey& k, bool recording);
    gdpm_status replay(const StepGraphKey& k);
    gdpm_status settle();       // super-round ends, statistics, finished jobs
    void release(EJob* j);
    bool any_active() const {
        for (int i = 0; i < n_slots; ++i)
            if (slots[i] && !slots[i]->done) return true;
        return false;
    }
};

void Engine::tune_begin() {
    tune = Tuner{};
    tune.on = ctx->autotune != 0 && !M.fixed;
    if (!tune.on) return;
    for (int w : {8, 12})
        for (int b : {1, 16}) tune.cand.emplace_back(w, b);
    tune.score.assign(tune.cand.size(), 0.0);
    tune.samples.assign(tune.cand.size(), 0);
    ctx->waves_per_cu = tune.cand[0].first;
    ctx->rebin_bins = tune.cand[0].second;
    ctx->tune_cand = tune.cand;
    ctx->tune_score.assign(tune.cand.size(), 0.0);
    ctx->tune_kept = -1;
}

// after an iteration: score the candidate it ran with, move to the next
void Engine::tune_account() {
    if (!tune.on || tune.fixed) return;
    const Ctl* hc = ctx->host_ctl;
    const unsigned long long ev = hc->ev[GDPM_EV_FLIGHTS] + hc->ev[GDPM_EV_ESTEPS];
    const double t = tm.photon + tm.electron + tm.fused;
    const unsigned long long dev = ev - tune.last_events;
    const double dt = t - tune.last_time;
    tune.last_events = ev;
    tune.last_time = t;
    if (dev < (unsigned long long)ctx->autotune_min_events || dt <= 0.0) return;   // too little work to score
    tune.score[tune.cur] += (double)dev / dt;
    tune.samples[tune.cur]++;
    ctx->tune_score[tune.cur] = tune.score[tune.cur] / tune.samples[tune.cur];
    const int n = (int)tune.cand.size();
    tune.cur = (tune.cur + 1) % n;
    if (*std::min_element(tune.samples.begin(), tune.samples.end()) >= 2) {
        int best = 0;
        for (int i = 1; i < n; ++i)
            if (tune.score[i] / tune.samples[i] > tune.score[best] / tune.samples[best]) best = i;
        tune.cur = best;
        tune.fixed = true;
        ctx->tune_kept = best;
    }
    ctx->waves_per_cu = tune.cand[tune.cur].first;
    ctx->rebin_bins = tune.cand[tune.cur].second;
}

gdpm_status Engine::init(gdpm_context c, hipStream_t s, const RunPlan& plan, const EngineMem* mem) {
    drop_graphs();
    ctx = c;
    st = s;
    slots.assign(kMaxJobs, nullptr);
    n_slots = 0;
    key = TableKey{plan.ecut_g, plan.ecut_e, plan.flags & 0x3Fu};
    gdpm_status e = GDPM_OK;
    if (mem) {
        // fixed memory: the table set must already be resident
        auto it = ctx->tables.find(key);
        if (it == ctx->tables.end())
            return fail(GDPM_E_INVALID,
                        "no resident tables for cutoffs (%g, %g) MeV and flags 0x%x: the default set is "
                        "made by gdpm_set_materials, others by a first run of any other entry point",
                        plan.ecut_g, plan.ecut_e, key.flags);
        tab = it->second.get();
        M = *mem;
    } else {
        e = get_tables(ctx, plan.ecut_g, plan.ecut_e, plan.flags, &tab);
        if (e) return e;
        e = context_mem(ctx, &M);
        if (e) return e;
    }
    T = tab->view(nullptr);
    Ctl* hc = ctx->host_ctl;
    memset(hc, 0, sizeof(Ctl));
    for (int r = 0; r < 2; ++r) hc->ring[r].head = hc->ring[r].tail = hc->ring[r].begin = ctx->ring_start;
    HIP_TRY(hipMemcpyAsync(M.ctl, hc, sizeof(Ctl), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(M.jc, 0, sizeof(JobCtl), st));
    memset(ctx->h_jc, 0, kJcMirrorBytes);
    memset(&R, 0, sizeof R);
    R.ecut_g = (float)plan.ecut_g;
    R.ecut_e = (float)plan.ecut_e;
    R.jobs = M.jobs;
    R.jc = M.jc;
    R.n_jobs = 0;
    const uint32_t cap = 1u << M.ring_log2;
    for (int r = 0; r < 2; ++r) {
        R.buf[r] = M.ring[r];
        R.bin[r] = M.bin[r];
        R.mask[r] = cap - 1u;
        R.hard[r] = cap;
    }
    tm = Timers{};
    iter = idle = 0;
    tune_begin();
    return GDPM_OK;
}

// validate a job against the engine and give it a slot, buffers and its first super-round
gdpm_status Engine::admit(EJob* j) {
    if (!j->ph || !j->src) return fail(GDPM_E_INVALID, "NULL handle");
    if (j->ph->ctx != ctx || j->src->ctx != ctx) return fail(GDPM_E_INVALID, "handle of another context");
    if (TableKey{j->plan.ecut_g, j->plan.ecut_e, j->plan.flags & 0x3Fu} < key ||
        key < TableKey{j->plan.ecut_g, j->plan.ecut_e, j->plan.flags & 0x3Fu})
        return fail(GDPM_E_INVALID, "jobs run together must share cutoffs and physics flags");
    if ((int)j->ph->rho_max.size() > tab->host.n_mat)
        return fail(GDPM_E_INVALID, "phantom uses more materials than the context has");
    int slot = -1;
    for (int i = 0; i < kMaxJobs; ++i)
        if (!slots[i]) {
            slot = i;
            break;
        }
    if (slot < 0) return fail(GDPM_E_BUSY, "all %d job slots are in use", kMaxJobs);
    const RunPlan& plan = j->plan;
    const size_t nv = (size_t)j->ph->nx * j->ph->ny * j->ph->nz;
    j->nv = nv;
    j->slot = slot;
    // Woodcock majorant of this job's phantom
    std::vector<double> rmax(tab->host.n_mat, 0.0);
    for (size_t m = 0; m < j->ph->rho_max.size(); ++m) rmax[m] = j->ph->rho_max[m];
    const std::vector<float> mm = build_majorant(tab->host, rmax);
    if (M.fixed && (!j->mumax_p || !j->tally_p || !j->d_dose || !j->d_sigma))
        return fail(GDPM_E_INVALID, "a job of an engine on fixed memory needs its arrays given");
    if (!j->mumax_p) {
        HIP_TRY(j->mumax.alloc(mm.size() * sizeof(float)));
        j->mumax_p = j->mumax.as<float>();
    }
    HIP_TRY(hipMemcpyAsync(j->mumax_p, mm.data(), mm.size() * sizeof(float), hipMemcpyHostToDevice, st));
    if (!j->tally_p) {
        HIP_TRY(j->tally.alloc((size_t)plan.nb * nv * sizeof(double)));
        j->tally_p = j->tally.as<double>();
    }
    HIP_TRY(hipMemsetAsync(j->tally_p, 0, (size_t)plan.nb * nv * sizeof(double), st));
    if (!j->d_dose) {
        HIP_TRY(j->dose_buf.alloc(nv * sizeof(double)));
        j->d_dose = j->dose_buf.as<double>();
    }
    if (!j->d_sigma) {
        HIP_TRY(j->sigma_buf.alloc(nv * sizeof(double)));
        j->d_sigma = j->sigma_buf.as<double>();
    }
    double* hist = nullptr;
    if (j->hist.bytes) {
        HIP_TRY(hipMemsetAsync(j->hist.p, 0, j->hist.bytes, st));
        hist = j->hist.as<double>();
    }
    JobDev& d = ctx->h_jobs[slot];
    memset(&d, 0, sizeof d);
    d.G = geom_of(j->ph);
    d.S = j->src->view();
    d.mumax = j->mumax_p;
    d.tally = j->tally_p;
    d.nv = nv;
    d.hist = hist;
    d.hist0 = j->prm.hist0;
    d.k0 = (uint32_t)j->prm.seed;
    d.k1 = (uint32_t)(j->prm.seed >> 32) ^ j->prm.job_id;
    d.flags = plan.flags;
    d.split = (uint32_t)plan.split;
    // a new generation of the slot: records of the slot's earlier jobs (none
    // in a sound run) are then recognised as such and dropped
    slot_gen[slot] = (slot_gen[slot] + 1u) & 0xFFu;
    d.gen = slot_gen[slot];
    if (j->src->metro) {
        // the job's Metropolis chains start afresh at its first history
        if (!j->chains_p) {
            if (M.fixed) return fail(GDPM_E_INVALID, "a job of an engine on fixed memory needs its chain states given");
            HIP_TRY(j->chains.alloc(kMetroChains * sizeof(uint32_t)));
            j->chains_p = j->chains.as<uint32_t>();
        }
        HIP_TRY(launch_metro_init(st, d.S, d.k0, d.k1, j->chains_p));
        d.chains = j->chains_p;
    }
    HIP_TRY(hipMemcpyAsync(M.jobs + slot, &d, sizeof d, hipMemcpyHostToDevice, st));
    // the job's counters start from zero
    JobCtl* dj = M.jc;
    HIP_TRY(hipMemsetAsync(&dj->births[slot], 0, sizeof(unsigned long long), st));
    HIP_TRY(hipMemsetAsync(&dj->deaths[slot], 0, sizeof(unsigned long long), st));
    HIP_TRY(hipMemsetAsync(&dj->e_in[slot], 0, sizeof(double), st));
    HIP_TRY(hipMemsetAsync(&dj->e_esc[slot], 0, sizeof(double), st));
    j->births = j->deaths = 0;
    // schedule: fixed mode is one super-round; target mode starts from n_histories
    j->hbase = plan.target ? 0 : j->prm.hist0;
    j->issued = 0;
    j->nhist.assign(plan.nb, 0.0);
    j->max_hist = j->prm.max_histories ? j->prm.max_histories : 100 * plan.n_hist;
    j->round_size = j->prm.round_size ? j->prm.round_size : (plan.n_hist + plan.nb - 1) / plan.nb;
    j->sr_start = 0;
    j->sr_end = plan.target ? (uint64_t)plan.nb * j->round_size
                            : std::min<uint64_t>(plan.n_hist, (uint64_t)plan.nb * j->round_size);
    j->sr_final = !plan.target;   // a fixed-count job runs one super-round
    j->done = false;
    j->status = GDPM_OK;
    j->t_admit = now_s();
    j->seq = admitted++;
    slots[slot] = j;
    n_slots = std::max(n_slots, slot + 1);
    return GDPM_OK;
}

void Engine::release(EJob* j) {
    if (j->slot >= 0 && slots[j->slot] == j) slots[j->slot] = nullptr;
    while (n_slots > 0 && !slots[n_slots - 1]) --n_slots;
    j->slot = -1;
}

// one scheduler iteration: new histories, a photon pass, an electron pass
gdpm_status Engine::step() {
    Ctl* hc = ctx->host_ctl;
    const int blocks = grid_blocks(ctx);
    const uint32_t cap = 1u << M.ring_log2;
    // new histories: at most half a queue (or pass_histories) less what the
    // fuller queue holds, split evenly over the jobs that still start
    // histories (issue_order 0), or given to one job first, which takes what it
    // can use, the next job the rest, and so on: the job with the least work
    // left first (issue_order 1: the histories left of its planned
    // super-round), or the earliest admitted first (issue_order 2)
    const uint32_t budget = ctx->pass_histories > 0 ? (uint32_t)ctx->pass_histories : cap / 2u;
    const uint32_t fill = std::max(hc->ring[0].tail - hc->ring[0].head, hc->ring[1].tail - hc->ring[1].head);
    uint64_t room = fill < budget ? budget - fill : 0u;
    std::vector<EJob*> want;
    for (int i = 0; i < n_slots; ++i) {
        EJob* j = slots[i];
        if (j && !j->done && j->issued < j->sr_end) want.push_back(j);
    }
    std::stable_sort(want.begin(), want.end(), [](const EJob* a, const EJob* b) { return a->seq < b->seq; });
    const bool greedy = ctx->issue_order != 0;
    if (ctx->issue_order == 1)
        std::stable_sort(want.begin(), want.end(), [](const EJob* a, const EJob* b) {
            return a->sr_end - a->issued < b->sr_end - b->issued;
        });
    int nseg[2] = {0, 0};
    uint32_t total[2] = {0u, 0u};
    SrcSeg* hs = ctx->h_segs;
    const int seg_cap = kMaxSegs / 2;   // per source type
    for (size_t k = 0; k < want.size() && room > 0; ++k) {
        EJob* j = want[k];
        const uint64_t share = greedy ? room : std::max<uint64_t>(1, room / (want.size() - k));
        uint64_t n = std::min<uint64_t>(share, j->sr_end - j->issued);
        // A pass holds its input and the secondaries it creates: the budget
        // assumes about one charged secondary per photon history below 7 MeV.
        // Electron sources (a 20 MeV electron leaves about six records of
        // secondaries, deltas and their own) and harder photon spectra start
        // fewer histories per iteration, so that a job alone cannot overflow.
        const double per_history = j->src->particle == 1 ? 8.0 : std::max(1.0, j->src->e_max / 7.0);
        n = std::min<uint64_t>(n, (uint64_t)((double)budget / per_history));
        // a split history takes 2^split queue records
        const uint32_t copies = 1u << j->plan.split;
        n = std::min<uint64_t>(n, room / copies);
        const int ri = j->src->particle == 0 ? 0 : 1;
        while (n > 0 && nseg[ri] < seg_cap) {
            const uint64_t rel = j->issued - j->sr_start;
            const uint32_t b = (uint32_t)std::min<uint64_t>(rel / j->round_size, j->plan.nb - 1);
            const uint64_t round_end = std::min(j->sr_end, j->sr_start + (b + 1) * j->round_size);
            const uint64_t m = std::min(n, round_end - j->issued);
            SrcSeg& sg = hs[ri * seg_cap + nseg[ri]++];
            sg.h0 = j->hbase + j->issued;
            sg.n = (uint32_t)m;
            const uint64_t round_start = j->sr_start + (uint64_t)b * j->round_size;
            sg.rpos = (uint32_t)(j->issued - round_start);
            sg.rsize = (uint32_t)(round_end - round_start);
            sg.off = total[ri];   // in records: history i's copy c at off + i 2^split + c
            sg.job = (uint32_t)j->slot;
            sg.batch = b;
            total[ri] += (uint32_t)(m * copies);
            j->issued += m;
            j->nhist[b] += (double)m;
            room -= m * copies;
            n -= m;
        }
    }
    R.n_jobs = std::max(n_slots, 1);
    for (int ri = 0; ri < 2; ++ri) ctx->h_hdr[ri] = SrcHdr{(uint32_t)nseg[ri], total[ri], 0u, 0u};
    // bins per job so that jobs x bins fits the re-binning keys; boxes of the
    // phantom come as space^3 (the largest cube within the bins)
    int nb = std::max(1, std::min(std::min(ctx->rebin_bins, kMaxBins), kMaxKeys / R.n_jobs));
    int space = 0;
    if (ctx->rebin_space) {
        space = 1;
        while ((space + 1) * (space + 1) * (space + 1) <= nb) ++space;
        nb = space * space * space;
    }
    const float blo = -5.0f, bhi = 5.0f;  // log2 E range of the bins (0.03 .. 32 MeV)
    // The jobs that hold particles in this iteration: live records after the
    // last one (births less deaths) or new histories now.  With one such job
    // the queues need no re-binning: they are all its segment.
    int holders = 0, lone = -1, first_slot = -1;
    {
        const JobCtlMirror* m = reinterpret_cast<const JobCtlMirror*>(ctx->h_jc);
        std::vector<char> fresh(n_slots, 0);
        for (int ri = 0; ri < 2; ++ri)
            for (int q = 0; q < nseg[ri]; ++q) fresh[hs[ri * seg_cap + q].job] = 1;
        for (int i = 0; i < n_slots; ++i) {
            if (!slots[i]) continue;
            if (first_slot < 0) first_slot = i;
            const long long live =
                (long long)(m->births[i] - m->deaths[i]) - slots[i]->death_offset;
            if (live != 0 || fresh[i]) {
                ++holders;
                lone = i;
            }
        }
        if (holders == 0) lone = first_slot;   // queues hold no particle at all
    }
    // A graph needs a launch sequence that does not change between iterations:
    // copy sizes and source grids are rounded up to powers of two (the kernels
    // read the true counts from the header), so a few recordings serve a run.
    // (A null stream cannot record; it never reaches here, a run without a
    // stream of its own uses the context's.)
    const bool graph = ctx->graphs != 0 && st != nullptr && !M.fixed;
    StepGraphKey k;
    memset(&k, 0, sizeof k);
    k.st = st;
    for (int ri = 0; ri < 2; ++ri) {
        if (!nseg[ri]) continue;
        const uint64_t need = std::min<uint64_t>((total[ri] + 255) / 256, 4u * (uint64_t)blocks);
        k.seg_copy[ri] = graph ? (int)std::min<uint64_t>(pow2_at_least(nseg[ri], 8), seg_cap) : nseg[ri];
        k.src_blocks[ri] = (int)(graph ? std::min<uint64_t>(pow2_at_least(need, 1), 4u * (uint64_t)blocks) : need);
    }
    k.blocks = blocks;
    k.threads = block_threads(ctx);
    k.threads_photon = ctx->photon_waves_per_cu ? std::min(k.threads, 64 * ctx->photon_waves_per_cu) : k.threads;
    k.nb = nb;
    k.space = space;
    k.blo = blo;
    k.binv = nb / (bhi - blo);
    for (int ri = 0; ri < 2; ++ri) {
        // sort the queue's positions by job (and bin, rebin_bins > 1), dropping
        // empty ones, so that each job's records form a segment of the pass's
        // input (read through the permutation); skipped when one job holds
        // all particles (measured faster: with lanes refilled every iteration
        // energy order gains nothing, and push order keeps some spatial
        // locality), the pass then reads the queue as it is, empty slots included
        k.rebin[ri] = !M.fixed && ((ri == 0 ? ctx->rebin_photons : ctx->rebin_electrons) || holders > 1 || lone < 0);
        if (k.rebin[ri]) tm.passes_rebinned++;
        const int tpb = ri == 0 ? k.threads_photon : k.threads;
        k.lds[ri] = ctx->lds_tables && transport_lds_bytes(ri, T, tpb / 64) <= (size_t)ctx->max_lds;
        tm.passes++;
        (ri == 0 ? tm.passes_photon : tm.passes_electron)++;
    }
    k.lone = (k.rebin[0] && k.rebin[1]) ? -1 : lone;
    // both passes in one launch: needs the electron tables staged (the photon
    // tables are read through the caches); not in the one-particle form
    k.fused = ctx->fused_passes && !ctx->solo_lanes && k.lds[1];
    if (k.fused) {
        const int waves = k.threads / 64;
        k.photon_waves = ctx->photon_waves < 0 ? waves / 2 : std::min(ctx->photon_waves, waves);
        k.lds[0] = 0;
    }
    k.R = R;
    k.T = T;
    {
        const gdpm_status s = graph ? replay(k) : issue(k, false);
        if (s != GDPM_OK) return s;
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (k.fused) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]));
        tm.fused += ms * 1e-3;
    } else {
        for (int ri = 0; ri < 2; ++ri) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->events[2 * ri], ctx->events[2 * ri + 1]));
            (ri == 0 ? tm.photon : tm.electron) += ms * 1e-3;
        }
    }
    ++iter;
    last = k;
    tune_account();
    if (ctx->check_accounting && !hc->overflow) {
        const gdpm_status s = check_accounting();
        if (s != GDPM_OK) return s;
    }
    if (hc->overflow)
        return fail(GDPM_E_OVERFLOW, "a particle queue filled up (capacity 2^%d); raise ring_capacity_log2",
                    M.ring_log2);
    return GDPM_OK;
}

// Diagnostic (option check_accounting): after an iteration every job's live
// records in the queues must equal its particle births less its deaths.  A
// disagreement is printed with the iteration's launch settings and queue state
// and counted in the run statistics; the run goes on.
gdpm_status Engine::check_accounting() {
    HIP_TRY(hipMemsetAsync(M.counts, 0, kMaxJobs * sizeof(unsigned long long), st));
    HIP_TRY(launch_count_records(st, 4 * grid_blocks(ctx), M.ctl, R, M.counts));
    std::vector<unsigned long long> live(kMaxJobs);
    HIP_TRY(hipMemcpyAsync(live.data(), M.counts, kMaxJobs * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const JobCtlMirror* m = reinterpret_cast<const JobCtlMirror*>(ctx->h_jc);
    const Ctl* hc = ctx->host_ctl;
    for (int i = 0; i < n_slots; ++i) {
        const EJob* j = slots[i];
        if (!j || j->done) continue;
        const long long expect = (long long)m->births[i] - (long long)m->deaths[i] - j->death_offset;
        if (expect == (long long)live[i]) continue;
        ++mismatches;
        fprintf(stderr,
                "[gdpm] accounting check: iteration %u, slot %d (job %u): births %llu deaths %llu "
                "(offset %lld) but %llu live records; slots %d, source segments %d/%d, re-binned %d/%d, "
                "queues [%u, %u) [%u, %u), graph %d\n",
                iter, i, j->prm.job_id, (unsigned long long)m->births[i], (unsigned long long)m->deaths[i],
                (long long)j->death_offset, live[i], n_slots, last.seg_copy[0], last.seg_copy[1],
                last.rebin[0], last.rebin[1], hc->ring[0].head, hc->ring[0].tail, hc->ring[1].head,
                hc->ring[1].tail, ctx->graphs);
    }
    return GDPM_OK;
}

// the launch sequence of one iteration: source passes, then for photons and
// electrons re-binning, set-up, transport (between two timing events) and
// completion, then the read-back of the counters
gdpm_status Engine::issue(const StepGraphKey& k, bool recording) {
    Ctl* dc = M.ctl;
    SrcHdr* dh = M.hdr;
    const int seg_cap = kMaxSegs / 2;
    HIP_TRY(hipMemcpyAsync(dh, ctx->h_hdr, 2 * sizeof(SrcHdr), hipMemcpyHostToDevice, st));
    for (int ri = 0; ri < 2; ++ri) {
        if (!k.seg_copy[ri]) continue;
        SrcSeg* dseg = M.segs + ri * seg_cap;
        HIP_TRY(hipMemcpyAsync(dseg, ctx->h_segs + ri * seg_cap, k.seg_copy[ri] * sizeof(SrcSeg),
                               hipMemcpyHostToDevice, st));
        HIP_TRY(launch_source(st, k.src_blocks[ri], dc, k.R, dseg, dh + ri, ri));
    }
    if (k.fused) {
        // both queues set up, then one launch runs both passes
        for (int ri = 0; ri < 2; ++ri) {
            if (k.rebin[ri]) HIP_TRY(launch_rebin(st, 4 * k.blocks, dc, k.R, ri, k.nb, k.blo, k.binv, k.space));
            HIP_TRY(launch_setup(st, dc, k.R, ri, k.rebin[ri], k.lone));
        }
        HIP_TRY(recording ? hipEventRecordWithFlags(ctx->events[0], st, hipEventRecordExternal)
                          : hipEventRecord(ctx->events[0], st));
        HIP_TRY(launch_fused(st, k.blocks, k.threads, k.photon_waves, k.rebin[0] || k.rebin[1], dc, k.T, k.R));
        HIP_TRY(recording ? hipEventRecordWithFlags(ctx->events[1], st, hipEventRecordExternal)
                          : hipEventRecord(ctx->events[1], st));
        for (int ri = 0; ri < 2; ++ri) HIP_TRY(launch_finish(st, dc, ri));
        HIP_TRY(hipMemcpyAsync(ctx->host_ctl, dc, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(ctx->h_jc, M.jc, kJcMirrorBytes, hipMemcpyDeviceToHost, st));
        return GDPM_OK;
    }
    for (int ri = 0; ri < 2; ++ri) {
        if (k.rebin[ri]) HIP_TRY(launch_rebin(st, 4 * k.blocks, dc, k.R, ri, k.nb, k.blo, k.binv, k.space));
        HIP_TRY(launch_setup(st, dc, k.R, ri, k.rebin[ri], k.lone));
        // a recorded event becomes a node of the graph that records it at replay
        HIP_TRY(recording ? hipEventRecordWithFlags(ctx->events[2 * ri], st, hipEventRecordExternal)
                          : hipEventRecord(ctx->events[2 * ri], st));
        HIP_TRY(launch_transport(st, ri, k.blocks, ri == 0 ? k.threads_photon : k.threads, k.lds[ri] != 0,
                                 ctx->solo_lanes != 0, k.rebin[ri] != 0, dc, k.T, k.R));
        HIP_TRY(recording ? hipEventRecordWithFlags(ctx->events[2 * ri + 1], st, hipEventRecordExternal)
                          : hipEventRecord(ctx->events[2 * ri + 1], st));
        HIP_TRY(launch_finish(st, dc, ri));
    }
    HIP_TRY(hipMemcpyAsync(ctx->host_ctl, dc, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(ctx->h_jc, M.jc, kJcMirrorBytes, hipMemcpyDeviceToHost, st));
    return GDPM_OK;
}

// launch the iteration as a graph: settings seen for the first time launch
// directly, the second time they are recorded, from then on replayed (the
// least recently used of kMaxStepGraphs settings makes room for a new one)
gdpm_status Engine::replay(const StepGraphKey& k) {
    StepGraph* hit = nullptr;
    for (auto& g : graphs)
        if (memcmp(&g.key, &k, sizeof k) == 0) hit = &g;
    if (!hit) {
        if (graphs.size() >= kMaxStepGraphs) {
            auto old = std::min_element(graphs.begin(), graphs.end(), [](const StepGraph& a, const StepGraph& b) {
                return a.last_use < b.last_use;
            });
            if (old->exec) (void)hipGraphExecDestroy(old->exec);
            graphs.erase(old);
        }
        graphs.push_back(StepGraph{k, nullptr, ++graph_clock});
        return issue(k, false);
    }
    if (!hit->exec) {
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const gdpm_status s = issue(k, true);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &graph);
        if (s != GDPM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess) return fail(GDPM_E_DEVICE, "recording an iteration: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(GDPM_E_DEVICE, "instantiating an iteration: %s", hipGetErrorString(ei));
        hit->exec = exec;
        tm.graphs_recorded++;
    }
    hit->last_use = ++graph_clock;
    HIP_TRY(hipGraphLaunch(hit->exec, st));
    tm.graph_launches++;
    return GDPM_OK;
}

gdpm_status compute_stats(gdpm_context ctx, const EngineMem& M, EJob* j, hipStream_t st) {
    const int nb = j->plan.nb;
    const size_t nv = j->nv;
    std::vector<double> inv(nb);
    // a split job's tallies hold 2^split copies at weight 1 each
    for (int b = 0; b < nb; ++b) inv[b] = j->nhist[b] > 0 ? std::ldexp(1.0 / j->nhist[b], -j->plan.split) : 0.0;
    HIP_TRY(hipMemcpyAsync(M.inv_n, inv.data(), nb * sizeof(double), hipMemcpyHostToDevice, st));
    Ctl* dc = M.ctl;
    double* red = ctx->h_red;
    memset(red, 0, 4 * sizeof(double) + sizeof(unsigned long long));
    HIP_TRY(hipMemcpyAsync(&dc->red[0], red, 4 * sizeof(double) + sizeof(unsigned long long),
                           hipMemcpyHostToDevice, st));
    const int blocks = (int)std::min<size_t>((nv + 255) / 256, 8192);
    HIP_TRY(launch_stats(st, blocks, dc, j->tally_p, nv, nb, M.inv_n,
                         j->ph->vox.as<const uint32_t>(), j->ph->dx * j->ph->dy * j->ph->dz,
                         (float)j->prm.stat_min_density, j->d_dose, j->d_sigma));
    HIP_TRY(hipMemcpyAsync(red, &dc->red[0], 4 * sizeof(double) + sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double dm;
    memcpy(&dm, red + 4, sizeof dm);
    j->dmax = dm;
    j->edep = std::ldexp(red[0], -j->plan.split);
    j->unc = (red[2] > 0 && dm > 0) ? red[1] / red[2] / dm : 0.0;
    return GDPM_OK;
}

// after an iteration: jobs whose super-round is complete get their statistics
// and either finish or start the next super-round
gdpm_status Engine::settle() {
    bool progress = false;
    const JobCtlMirror* m = reinterpret_cast<const JobCtlMirror*>(ctx->h_jc);
    for (int i = 0; i < n_slots; ++i) {
        EJob* j = slots[i];
        if (!j || j->done) continue;
        j->births = m->births[i];
        j->deaths = m->deaths[i] + (unsigned long long)j->death_offset;
        j->e_in = m->e_in[i];
        j->e_esc = std::ldexp(m->e_esc[i], -j->plan.split);
        if (j->issued < j->sr_end || j->births != j->deaths) continue;
        progress = true;
        gdpm_status s = compute_stats(ctx, M, j, st);
        if (s) return s;
        j->rounds += (uint32_t)j->plan.nb;
        const gdpm_run_params& p = j->prm;
        bool finished = !j->plan.target || j->unc <= p.target_unc;
        if (!finished && j->issued >= j->max_hist) {
            finished = true;
            j->status = GDPM_E_NOT_CONVERGED;
            char buf[160];
            snprintf(buf, sizeof buf, "uncertainty %.4g above target after %llu histories", j->unc,
                     (unsigned long long)j->issued);
            j->err = buf;
        }
        if (finished) {
            j->done = true;
            j->t_done = now_s();
            continue;
        }
        // histories still needed, from sigma ~ 1/sqrt(N), with a 5% margin
        const double done = (double)j->issued;
        const double need = done * ((j->unc / p.target_unc) * (j->unc / p.target_unc) * 1.05 - 1.0);
        uint64_t more = (uint64_t)std::ceil(std::max(need, 0.02 * done));
        more = std::min<uint64_t>(more, j->max_hist - j->issued);
        j->round_size = std::max<uint64_t>(1, (more + j->plan.nb - 1) / j->plan.nb);
        j->sr_start = j->issued;
        j->sr_end = j->issued + (uint64_t)j->plan.nb * j->round_size;
        j->sr_final = true;   // sized to reach the target (or the history cap)
    }
    // nothing left anywhere but a job still waits: the bookkeeping is broken
    const Ctl* hc = ctx->host_ctl;
    const bool empty = hc->ring[0].tail == hc->ring[0].head && hc->ring[1].tail == hc->ring[1].head;
    bool issuing = false;
    for (int i = 0; i < n_slots; ++i)
        if (slots[i] && !slots[i]->done && slots[i]->issued < slots[i]->sr_end) issuing = true;
    idle = (!progress && empty && !issuing) ? idle + 1 : 0;
    if (idle > 2) {
        // The queues are empty and nothing starts, yet a job's births and
        // deaths differ.  Count the job's records on the device: if none is
        // left the counters drifted; align them and record the repair (it is
        // reported in the job's statistics), else stop with the numbers.
        HIP_TRY(hipMemsetAsync(M.counts, 0, kMaxJobs * sizeof(unsigned long long), st));
        HIP_TRY(launch_count_records(st, 4 * grid_blocks(ctx), M.ctl, R, M.counts));
        std::vector<unsigned long long> live(kMaxJobs);
        HIP_TRY(hipMemcpyAsync(live.data(), M.counts, kMaxJobs * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        int repaired = 0;
        for (int i = 0; i < n_slots; ++i) {
            EJob* j = slots[i];
            if (!j || j->done || j->births == j->deaths) continue;
            if (live[i] || j->repairs >= 3)
                return fail(GDPM_E_DEVICE,
                            "transport made no progress: job %d has %llu particles born, %llu ended, "
                            "%llu records queued, %u repairs", i, (unsigned long long)j->births,
                            (unsigned long long)j->deaths, (unsigned long long)live[i], j->repairs);
            j->death_offset += (long long)j->births - (long long)j->deaths;
            j->repairs++;
            repaired++;
        }
        if (!repaired) return fail(GDPM_E_DEVICE, "transport made no progress (no job left to finish)");
        idle = 0;
    }
    return GDPM_OK;
}

void fill_stats(const Engine& E, const EJob* j, double t_start, gdpm_run_stats* out) {
    memset(out, 0, sizeof *out);
    const Ctl* hc = E.ctx->host_ctl;
    out->histories = j->issued;
    out->e_in = j->e_in;
    out->e_esc = j->e_esc;
    out->e_dep = j->edep;
    out->unc_mean_over_dmax = j->unc;
    out->dmax = j->dmax;
    for (int i = 0; i < 8; ++i) out->events[i] = hc->ev[i];
    out->events[GDPM_EV_HISTORIES] = j->issued;
    out->passes = E.tm.passes;
    out->passes_photon = E.tm.passes_photon;
    out->passes_electron = E.tm.passes_electron;
    for (int k = 0; k < 2; ++k) {
        out->records_loaded[k] = hc->pass_ev[k][0];
        out->records_stored[k] = hc->pass_ev[k][1];
        out->deposits[k] = hc->pass_ev[k][2];
    }
    out->rounds = j->rounds;
    out->accounting_repairs = j->repairs;
    out->accounting_gap = j->death_offset;
    out->transport_anomalies = hc->anomalies;
    out->graph_launches = E.tm.graph_launches;
    out->graphs_recorded = E.tm.graphs_recorded;
    out->passes_rebinned = E.tm.passes_rebinned;
    out->accounting_mismatches = E.mismatches;
    // the kernels count photoelectric, pair and Moller events; Compton and
    // bremsstrahlung are the rest of the real interactions and hard events
    out->interactions[1] = hc->itype[1];
    out->interactions[2] = hc->itype[2];
    out->interactions[3] = hc->itype[3];
    out->interactions[0] = hc->ev[GDPM_EV_REAL] - hc->itype[1] - hc->itype[2];
    out->interactions[4] = hc->ev[GDPM_EV_HARD] - hc->itype[3];
    for (int k = 0; k < 2; ++k) out->records_requeued[k] = hc->pass_ev[k][3];
    out->t_photon_s = E.tm.photon;
    out->t_electron_s = E.tm.electron;
    out->t_kernel_s = E.tm.photon + E.tm.electron + E.tm.fused;
    out->t_total_s = (j->t_done > 0 ? j->t_done : now_s()) - t_start;
}

gdpm_status make_job(gdpm_context ctx, gdpm_phantom ph, gdpm_source src, const gdpm_run_params* prm,
                     EJob* j) {
    if (!ph || !src) return fail(GDPM_E_INVALID, "NULL handle");
    if (ph->ctx != ctx || src->ctx != ctx) return fail(GDPM_E_INVALID, "handle of another context");
    gdpm_status s = validate_params(prm, src, &j->plan);
    if (s) return s;
    j->ph = ph;
    j->src = src;
    j->prm = *prm;
    return GDPM_OK;
}

// one job through the engine, blocking; outputs stay in device memory
// the scratch array carved into the engine's memory and one job's arrays
// (see kScratchBytes); false if the job's batch tallies do not fit
bool scratch_layout(unsigned char* base, EJob* j, EngineMem* M) {
    if ((size_t)j->plan.nb * j->nv * sizeof(double) > kScratchTallyBytes) return false;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base + off;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    memset(M, 0, sizeof *M);
    M->ctl = reinterpret_cast<Ctl*>(take(sizeof(Ctl)));
    M->jobs = reinterpret_cast<JobDev*>(take(kMaxJobs * sizeof(JobDev)));
    M->jc = reinterpret_cast<JobCtl*>(take(sizeof(JobCtl)));
    M->segs = reinterpret_cast<SrcSeg*>(take(kMaxSegs * sizeof(SrcSeg)));
    M->hdr = reinterpret_cast<SrcHdr*>(take(2 * sizeof(SrcHdr)));
    M->inv_n = reinterpret_cast<double*>(take(kMaxBatches * sizeof(double)));
    M->counts = reinterpret_cast<unsigned long long*>(take(kMaxJobs * sizeof(unsigned long long)));
    j->mumax_p = reinterpret_cast<float*>(take(kMaxGrid * sizeof(float)));
    j->chains_p = reinterpret_cast<uint32_t*>(take(kMetroChains * sizeof(uint32_t)));
    if (off > kScratchCtlBytes) return false;   // (a layout error; see the static sizes)
    for (int r = 0; r < 2; ++r) {
        M->ring[r] = reinterpret_cast<Particle*>(base + kScratchCtlBytes + r * kScratchRingBytes);
        M->bin[r] = nullptr;
    }
    M->ring_log2 = kScratchRingLog2;
    j->tally_p = reinterpret_cast<double*>(base + kScratchCtlBytes + 2 * kScratchRingBytes);
    M->fixed = true;
    return true;
}

// one job through the engine, blocking; outputs stay in device memory.  With
// `scr` (this device's scratch array) the engine's queues, control blocks and
// the job's arrays live there and nothing is allocated.
gdpm_status do_run(gdpm_context ctx, gdpm_phantom ph, gdpm_source src, const gdpm_run_params* prm,
                   double* d_dose, double* d_sigma, double* h_batch, double* h_hist,
                   hipStream_t st, gdpm_run_stats* out, EJob* keep, unsigned char* scr = nullptr) {
    const double t_start = now_s();
    if (!ctx) return fail(GDPM_E_INVALID, "NULL context");
    EJob local;
    EJob* j = keep ? keep : &local;
    gdpm_status s = make_job(ctx, ph, src, prm, j);
    if (s) return s;
    if (h_hist && (j->plan.target || j->plan.n_hist > ((uint64_t)1 << 24)))
        return fail(GDPM_E_INVALID, "per-history output needs fixed mode and <= 2^24 histories");
    j->d_dose = d_dose;
    j->d_sigma = d_sigma;
    EngineMem sm;
    if (scr) {
        j->nv = (size_t)ph->nx * ph->ny * ph->nz;
        if (h_batch || h_hist) return fail(GDPM_E_INVALID, "no batch or history output from scratch memory");
        if (!scratch_layout(scr, j, &sm))
            return fail(GDPM_E_INVALID,
                        "batch tallies of %zu bytes (n_batches %d x %zu voxels x 8) exceed the %zu bytes "
                        "of the scratch memory", (size_t)j->plan.nb * j->nv * sizeof(double), j->plan.nb,
                        j->nv, kScratchTallyBytes);
    }
    if (h_hist) HIP_TRY(j->hist.alloc(j->plan.n_hist * 2 * sizeof(double)));
    Engine E;
    s = E.init(ctx, st, j->plan, scr ? &sm : nullptr);
    if (s) return s;
    s = E.admit(j);
    if (s) return s;
    while (!j->done) {
        s = E.step();
        if (s) return s;
        s = E.settle();
        if (s) return s;
    }
    const size_t nv = j->nv;
    if (h_batch)
        HIP_TRY(hipMemcpyAsync(h_batch, j->tally_p, (size_t)j->plan.nb * nv * sizeof(double),
                               hipMemcpyDeviceToHost, st));
    if (h_hist)
        HIP_TRY(hipMemcpyAsync(h_hist, j->hist.p, j->plan.n_hist * 2 * sizeof(double),
                               hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (j->plan.split) {
        // the device sums hold each copy at weight 1 (see compute_stats)
        if (h_batch)
            for (size_t i = 0, n = (size_t)j->plan.nb * nv; i < n; ++i) h_batch[i] = std::ldexp(h_batch[i], -j->plan.split);
        if (h_hist)
            for (size_t i = 0, n = (size_t)j->plan.n_hist * 2; i < n; ++i) h_hist[i] = std::ldexp(h_hist[i], -j->plan.split);
    }
    if (out) fill_stats(E, j, t_start, out);
    E.release(j);
    if (j->status == GDPM_E_NOT_CONVERGED) fail(GDPM_E_NOT_CONVERGED, "%s", j->err.c_str());
    return j->status;
}

}  // namespace

// a job of gdpm_run_async (finished when created) or of a server
struct gdpm_job_s {
    gdpm_context ctx = nullptr;
    gdpm_status status = GDPM_OK;
    gdpm_run_stats stats{};
    std::string err;
    gdpm_server_s* srv = nullptr;
    std::unique_ptr<EJob> ej;
    double* dose = nullptr;    // host outputs of a server job
    double* sigma = nullptr;
    bool finished = true;
};

// the request loop of a server (see gdpm_server_create)
struct gdpm_server_s {
    gdpm_context ctx = nullptr;
    uint64_t budget = 0;
    int max_slots = 0;
    std::thread th;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<gdpm_job_s*> pending;
    std::vector<gdpm_job_s*> running;
    bool stop = false;
    bool key_set = false;
    TableKey key{};
    size_t used = 0, high_water = 0;
    uint64_t submitted = 0, finished = 0, histories = 0;
    void loop();
};

namespace {
void finish_server_job(gdpm_server_s* S, gdpm_job_s* job, gdpm_status st, const std::string& msg) {
    job->status = st;
    job->err = msg;
    job->finished = true;
    S->finished++;
    S->cv_done.notify_all();
}
}  // namespace

void gdpm_server_s::loop() {
    (void)hipSetDevice(ctx->device);
    hipStream_t st = ctx->stream;
    Engine E;
    bool ready = false;
    std::unique_lock<std::mutex> lk(m);
    for (;;) {
        // admission in arrival order, by slots and device footprint; with
        // admit_draining 1, only while every running job has issued all the
        // histories of its current super-round (its particles drain from the
        // queues, or it waits for its statistics), with 2 only while every
        // running job drains the super-round planned as its last: a new job
        // then fills the device a finishing job leaves instead of sharing it
        // with jobs that could fill it alone
        while (!pending.empty() && (int)running.size() < max_slots) {
            if (ctx->admit_draining && !running.empty()) {
                bool busy = false;
                for (gdpm_job_s* r : running) {
                    const EJob* q = r->ej.get();
                    const bool draining = q->issued >= q->sr_end && (ctx->admit_draining == 1 || q->sr_final);
                    busy = busy || (!q->done && !draining);
                }
                if (busy) break;
            }
            gdpm_job_s* job = pending.front();
            EJob* j = job->ej.get();
            const size_t fp = job_footprint(j->ph, j->plan, true, ready ? E.tab->host.pg_n : 0);
            if (used + fp > budget && !running.empty()) break;
            pending.pop_front();
            gdpm_status s = GDPM_OK;
            if (!ready) {
                s = E.init(ctx, st, j->plan);
                ready = s == GDPM_OK;
            }
            if (!s) s = E.admit(j);
            if (s) {
                finish_server_job(this, job, s, g_err);
                continue;
            }
            j->footprint = fp;
            used += fp;
            high_water = std::max(high_water, used);
            running.push_back(job);
        }
        if (running.empty()) {
            if (stop && pending.empty()) break;
            cv_work.wait(lk, [&] { return stop || !pending.empty(); });
            continue;
        }
        lk.unlock();
        gdpm_status s = E.step();
        if (!s) s = E.settle();
        lk.lock();
        if (s) {
            // a device error or an overflow ends every running job
            const std::string msg = g_err;
            for (gdpm_job_s* job : running) {
                E.release(job->ej.get());
                finish_server_job(this, job, s, msg);
            }
            running.clear();
            used = 0;
            ready = false;
            continue;
        }
        for (size_t i = 0; i < running.size();) {
            gdpm_job_s* job = running[i];
            EJob* j = job->ej.get();
            if (!j->done) {
                ++i;
                continue;
            }
            gdpm_status cs = GDPM_OK;
            if (job->dose && hipMemcpyAsync(job->dose, j->d_dose, j->nv * sizeof(double),
                                            hipMemcpyDeviceToHost, st) != hipSuccess)
                cs = GDPM_E_DEVICE;
            if (job->sigma && hipMemcpyAsync(job->sigma, j->d_sigma, j->nv * sizeof(double),
                                             hipMemcpyDeviceToHost, st) != hipSuccess)
                cs = GDPM_E_DEVICE;
            if (hipStreamSynchronize(st) != hipSuccess) cs = GDPM_E_DEVICE;
            fill_stats(E, j, j->t_submit, &job->stats);
            E.release(j);
            j->tally.reset();
            j->dose_buf.reset();
            j->sigma_buf.reset();
            j->mumax.reset();
            j->chains.reset();
            used -= j->footprint;
            histories += j->issued;
            finish_server_job(this, job, cs ? cs : j->status, cs ? "copying the outputs failed" : j->err);
            running.erase(running.begin() + i);
        }
    }
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* gdpm_last_error(void) { return g_err.c_str(); }

gdpm_status gdpm_context_create(int hip_device, const char* opts_json, gdpm_context* out) {
    if (!out) return fail(GDPM_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (hip_device < 0 || hip_device >= n) return fail(GDPM_E_INVALID, "no HIP device %d", hip_device);
    HIP_TRY(hipSetDevice(hip_device));
    auto ctx = std::make_unique<gdpm_context_s>();
    ctx->device = hip_device;
    HIP_TRY(scratch_address(hip_device, &ctx->scratch));
    ctx->ring_log2 = json_int(opts_json, "ring_capacity_log2", 25);
    ctx->waves_per_cu = json_int(opts_json, "waves_per_cu", 12);
    ctx->rebin_bins = json_int(opts_json, "rebin_bins", 1);
    ctx->rebin_space = json_int(opts_json, "rebin_space", 0);
    ctx->lds_tables = json_int(opts_json, "lds_tables", 1);
    ctx->pass_histories = json_int(opts_json, "pass_histories", 0);
    ctx->autotune = json_int(opts_json, "autotune", 0);
    ctx->autotune_min_events = json_int(opts_json, "autotune_min_events", 4000000);
    ctx->share = json_int(opts_json, "share", 1);
    ctx->issue_order = json_int(opts_json, "issue_order", 0);
    ctx->rebin_photons = json_int(opts_json, "rebin_photons", 0);
    ctx->rebin_electrons = json_int(opts_json, "rebin_electrons", 0);
    ctx->graphs = json_int(opts_json, "graphs", 1);
    ctx->check_accounting = json_int(opts_json, "check_accounting", 0);
    ctx->solo_lanes = json_int(opts_json, "solo_lanes", 0);
    ctx->fused_passes = json_int(opts_json, "fused_passes", 0);
    ctx->photon_waves_per_cu = json_int(opts_json, "photon_waves_per_cu", 0);
    ctx->photon_waves = json_int(opts_json, "photon_waves", -1);
    ctx->admit_draining = json_int(opts_json, "admit_draining", 0);
    const unsigned long long ring_start = json_u64(opts_json, "ring_start", 0);
    if (ring_start >= (1ull << 32)) return fail(GDPM_E_INVALID, "ring_start below 2^32");
    ctx->ring_start = (uint32_t)ring_start;
    if (ctx->ring_log2 < 12 || ctx->ring_log2 > 28) return fail(GDPM_E_INVALID, "ring_capacity_log2 in [12, 28]");
    if (ctx->waves_per_cu < 1 || ctx->waves_per_cu > kMaxBlockThreads / 64)
        return fail(GDPM_E_INVALID, "waves_per_cu in [1, %d]", kMaxBlockThreads / 64);
    if (ctx->rebin_bins < 0 || ctx->rebin_bins > kMaxBins) return fail(GDPM_E_INVALID, "rebin_bins in [0, 64]");
    if (ctx->rebin_space != 0 && ctx->rebin_space != 1) return fail(GDPM_E_INVALID, "rebin_space must be 0 or 1");
    if (ctx->pass_histories < 0) return fail(GDPM_E_INVALID, "pass_histories must be >= 0");
    if (ctx->autotune_min_events < 1) return fail(GDPM_E_INVALID, "autotune_min_events must be >= 1");
    if (ctx->issue_order < 0 || ctx->issue_order > 2)
        return fail(GDPM_E_INVALID, "issue_order must be 0 (even shares), 1 (least work left first) or 2 "
                    "(admission order first)");
    if (ctx->share != 1)
        return fail(GDPM_E_INVALID, "share must be 1: the oldest-job-first policy (0) can overflow the queues");
    if (ctx->admit_draining < 0 || ctx->admit_draining > 2) return fail(GDPM_E_INVALID, "admit_draining is 0, 1 or 2");
    if (ctx->solo_lanes != 0 && (ctx->solo_lanes != 1 || !ctx->lds_tables || ctx->autotune))
        return fail(GDPM_E_INVALID, "solo_lanes is 0 or 1 and needs lds_tables on and autotune off");
    if (ctx->fused_passes != 0 && ctx->fused_passes != 1) return fail(GDPM_E_INVALID, "fused_passes is 0 or 1");
    if (ctx->photon_waves_per_cu < 0 || ctx->photon_waves_per_cu > kMaxBlockThreads / 64)
        return fail(GDPM_E_INVALID, "photon_waves_per_cu in [0, %d]", kMaxBlockThreads / 64);
    if (ctx->photon_waves != -1 && (ctx->photon_waves < 0 || ctx->photon_waves > ctx->waves_per_cu))
        return fail(GDPM_E_INVALID, "photon_waves in [0, waves_per_cu] (or -1: half)");
    HIP_TRY(hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, hip_device));
    HIP_TRY(hipDeviceGetAttribute(&ctx->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device));
    if (ctx->lds_tables) {
        // the staged kernels may use all of it (above 64 KB an opt-in is needed)
        if (transport_lds_optin((size_t)ctx->max_lds) != hipSuccess) ctx->lds_tables = 0;
        (void)hipGetLastError();
    }
    HIP_TRY(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    HIP_TRY(ctx->ctl.alloc(sizeof(Ctl)));
    HIP_TRY(hipHostMalloc((void**)&ctx->host_ctl, sizeof(Ctl), hipHostMallocDefault));
    memset(ctx->host_ctl, 0, sizeof(Ctl));
    HIP_TRY(ctx->jobs_dev.alloc(kMaxJobs * sizeof(JobDev)));
    HIP_TRY(ctx->jc.alloc(sizeof(JobCtl)));
    HIP_TRY(ctx->segs.alloc(kMaxSegs * sizeof(SrcSeg)));
    HIP_TRY(hipHostMalloc((void**)&ctx->h_jobs, kMaxJobs * sizeof(JobDev), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void**)&ctx->h_segs, kMaxSegs * sizeof(SrcSeg), hipHostMallocDefault));
    memset(ctx->h_segs, 0, kMaxSegs * sizeof(SrcSeg));
    HIP_TRY(ctx->src_hdr.alloc(2 * sizeof(SrcHdr)));
    HIP_TRY(hipHostMalloc((void**)&ctx->h_hdr, 2 * sizeof(SrcHdr), hipHostMallocDefault));
    memset(ctx->h_hdr, 0, 2 * sizeof(SrcHdr));
    HIP_TRY(hipHostMalloc(&ctx->h_jc, kJcMirrorBytes, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void**)&ctx->h_red, 8 * sizeof(double), hipHostMallocDefault));
    HIP_TRY(ctx->inv_n.alloc(kMaxBatches * sizeof(double)));
    HIP_TRY(ctx->counts.alloc(kMaxJobs * sizeof(unsigned long long)));
    for (int i = 0; i < 4; ++i) {   // timing events of the two transport passes
        hipEvent_t ev;
        HIP_TRY(hipEventCreate(&ev));
        ctx->events.push_back(ev);
    }
    *out = ctx.release();
    return GDPM_OK;
}

gdpm_status gdpm_context_destroy(gdpm_context ctx) {
    if (!ctx) return fail(GDPM_E_INVALID, "NULL context");
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto e : ctx->events) (void)hipEventDestroy(e);
    if (ctx->h_hdr) (void)hipHostFree(ctx->h_hdr);
    if (ctx->host_ctl) (void)hipHostFree(ctx->host_ctl);
    if (ctx->h_jobs) (void)hipHostFree(ctx->h_jobs);
    if (ctx->h_segs) (void)hipHostFree(ctx->h_segs);
    if (ctx->h_jc) (void)hipHostFree(ctx->h_jc);
    if (ctx->h_red) (void)hipHostFree(ctx->h_red);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return GDPM_OK;
}

gdpm_status gdpm_set_materials(gdpm_context ctx, const gdpm_material* m, int n, int n_grid) {
    if (!ctx || !m) return fail(GDPM_E_INVALID, "NULL argument");
    if (n < 1 || n > kMaxMaterials) return fail(GDPM_E_INVALID, "1..%d materials", kMaxMaterials);
    if (n_grid == 0) n_grid = 1024;
    if (n_grid < 256 || n_grid > kMaxGrid) return fail(GDPM_E_INVALID, "n_grid in [256, %d]", kMaxGrid);
    std::vector<MaterialParams> mats(n);
    for (int i = 0; i < n; ++i) {
        if (!(m[i].z > 0) || !(m[i].z_over_a > 0) || !(m[i].i_ev > 0) || !std::isfinite(m[i].z) ||
            !std::isfinite(m[i].z_over_a) || !std::isfinite(m[i].i_ev))
            return fail(GDPM_E_INVALID, "material %d: parameters must be positive and finite", i);
        mats[i] = {m[i].z, m[i].z_over_a, m[i].i_ev};
    }
    ctx->mats = mats;
    ctx->n_grid = n_grid;
    ctx->tables.clear();
    // the table set of the default absorption energies, resident from now on
    HIP_TRY(hipSetDevice(ctx->device));
    DevTables* t = nullptr;
    return get_tables(ctx, 0.05, 0.2, 0u, &t);
}

gdpm_status gdpm_phantom_create(gdpm_context ctx, int nx, int ny, int nz, double dx, double dy,
                                double dz, const uint8_t* mat, const float* density,
                                gdpm_phantom* out) {
    if (!out) return fail(GDPM_E_INVALID, "NULL argument");
    *out = nullptr;
    // the sizes first (host-only checks, testable without a device)
    if (nx < 1 || ny < 1 || nz < 1 || nx > 2048 || ny > 2048 || nz > 1024)
        return fail(GDPM_E_INVALID, "dimensions must be in [1,2048]x[1,2048]x[1,1024]");
    if ((uint64_t)nx * (uint64_t)ny * (uint64_t)nz > (uint64_t)INT32_MAX)
        return fail(GDPM_E_INVALID, "%d x %d x %d voxels: at most 2^31 - 1 voxels (the linear voxel "
                    "index is a signed 32-bit integer)", nx, ny, nz);
    if (!(dx > 0) || !(dy > 0) || !(dz > 0) || !std::isfinite(dx) || !std::isfinite(dy) ||
        !std::isfinite(dz))
        return fail(GDPM_E_INVALID, "voxel sizes must be positive");
    if (!ctx || !mat || !density) return fail(GDPM_E_INVALID, "NULL argument");
    if (ctx->mats.empty()) return fail(GDPM_E_INVALID, "set materials first");
    const size_t nv = (size_t)nx * ny * nz;
    std::vector<uint32_t> vox(nv);
    std::vector<double> rmax(ctx->mats.size(), 0.0);
    for (size_t v = 0; v < nv; ++v) {
        const float r = density[v];
        if (mat[v] >= ctx->mats.size())
            return fail(GDPM_E_INVALID, "voxel %zu: material %d not defined", v, (int)mat[v]);
        if (!voxel_density_ok(r))
            return fail(GDPM_E_INVALID, "voxel %zu: density %g outside [2^-16, 2^16) g/cm^3", v, (double)r);
        vox[v] = pack_voxel(r, mat[v]);
        rmax[mat[v]] = std::max(rmax[mat[v]], (double)r);
    }
    HIP_TRY(hipSetDevice(ctx->device));
    auto ph = std::make_unique<gdpm_phantom_s>();
    ph->ctx = ctx;
    ph->nx = nx;
    ph->ny = ny;
    ph->nz = nz;
    ph->dx = dx;
    ph->dy = dy;
    ph->dz = dz;
    ph->rho_max = rmax;
    HIP_TRY(upload(ph->vox, vox));
    ctx->resident_bytes += (double)ph->vox.bytes;
    *out = ph.release();
    return GDPM_OK;
}

gdpm_status gdpm_phantom_destroy(gdpm_phantom ph) {
    if (!ph) return fail(GDPM_E_INVALID, "NULL phantom");
    ph->ctx->resident_bytes -= (double)ph->vox.bytes;
    delete ph;
    return GDPM_OK;
}

gdpm_status gdpm_source_create(gdpm_context ctx, const gdpm_source_desc* d, gdpm_source* out) {
    if (!ctx || !d || !out) return fail(GDPM_E_INVALID, "NULL argument");
    *out = nullptr;
    if (d->particle != 0 && d->particle != 1) return fail(GDPM_E_INVALID, "particle must be 0 or 1");
    if (d->n_phase_space > 0) {
        // the open source interface: a phase space replaces beams and spectrum
        if (!d->phase_space) return fail(GDPM_E_INVALID, "phase_space is NULL");
        if (d->n_phase_space > ((uint64_t)1 << 31)) return fail(GDPM_E_INVALID, "at most 2^31 phase-space records");
        auto src = std::make_unique<gdpm_source_s>();
        src->ctx = ctx;
        src->particle = d->particle;
        double emax = 0.0;
        for (uint64_t k = 0; k < d->n_phase_space; ++k) {
            const float* r = d->phase_space + 7 * k;
            const double nn = (double)r[3] * r[3] + (double)r[4] * r[4] + (double)r[5] * r[5];
            if (!(r[6] > 0.0f) || r[6] > kEmax || !(std::fabs(nn - 1.0) < 1e-5) || !std::isfinite(r[0]) ||
                !std::isfinite(r[1]) || !std::isfinite(r[2]))
                return fail(GDPM_E_INVALID, "phase-space record %llu: energy in (0, 30] MeV, unit direction, "
                            "finite position", (unsigned long long)k);
            emax = std::max(emax, (double)r[6]);
        }
        src->spec_kind = 0;
        src->e_mono = 0.0f;
        src->e_max = emax;
        src->spec_n = 0;
        src->nf = 0;
        src->n_guide = 0;
        src->n_beams = 0;
        std::vector<float> recs(d->phase_space, d->phase_space + 7 * d->n_phase_space);
        HIP_TRY(hipSetDevice(ctx->device));
        HIP_TRY(upload(src->phsp, recs));
        src->n_phsp = d->n_phase_space;
        *out = src.release();
        return GDPM_OK;
    }
    if (d->n_beams < 1 || !d->beams) return fail(GDPM_E_INVALID, "need at least one beam");
    if (d->n_beams > 65535) return fail(GDPM_E_INVALID, "at most 65535 beams");
    if (d->beamlet_sampler != 0 && d->beamlet_sampler != 1)
        return fail(GDPM_E_INVALID, "beamlet_sampler must be 0 (search) or 1 (Metropolis)");
    if (d->spectrum_strata < 0 || d->spectrum_strata > 64)
        return fail(GDPM_E_INVALID, "spectrum_strata in [0, 64]");
    if (d->spectrum_strata > 0 && d->spectrum.kind != 1)
        return fail(GDPM_E_INVALID, "energy intervals need a piecewise-linear spectrum");
    if (d->strata_shape != 0 && d->strata_shape != 1)
        return fail(GDPM_E_INVALID, "strata_shape must be 0 (uniform) or 1 (the spectrum's shape)");
    std::vector<double> strata_F;
    auto src = std::make_unique<gdpm_source_s>();
    src->ctx = ctx;
    src->particle = d->particle;
    const gdpm_spectrum& sp = d->spectrum;
    src->spec_kind = sp.kind;
    std::vector<float> se, spp, sc;
    if (sp.kind == 0) {
        if (!(sp.e_mono > 0) || sp.e_mono > kEmax)
            return fail(GDPM_E_INVALID, "monoenergetic energy must be in (0, 30] MeV");
        src->e_mono = (float)sp.e_mono;
        src->e_max = sp.e_mono;
        src->spec_n = 0;
    } else if (sp.kind == 1) {
        if (sp.n_pts < 2 || !sp.e_mev || !sp.pdf) return fail(GDPM_E_INVALID, "spectrum needs >= 2 points");
        double area = 0.0;
        sc.push_back(0.0f);
        std::vector<double> c(sp.n_pts, 0.0);
        for (int i = 0; i < sp.n_pts; ++i) {
            if (!(sp.e_mev[i] > 0) || sp.e_mev[i] > kEmax || !(sp.pdf[i] >= 0) || !std::isfinite(sp.pdf[i]))
                return fail(GDPM_E_INVALID, "spectrum point %d out of range", i);
            if (i > 0 && !(sp.e_mev[i] > sp.e_mev[i - 1]))
                return fail(GDPM_E_INVALID, "spectrum energies must increase");
            if (i > 0) {
                area += 0.5 * (sp.pdf[i - 1] + sp.pdf[i]) * (sp.e_mev[i] - sp.e_mev[i - 1]);
                c[i] = area;
            }
        }
        if (!(area > 0)) return fail(GDPM_E_INVALID, "spectrum has zero area");
        for (int i = 0; i < sp.n_pts; ++i) {
            se.push_back((float)sp.e_mev[i]);
            spp.push_back((float)sp.pdf[i]);
        }
        sc.clear();
        for (int i = 0; i < sp.n_pts; ++i) sc.push_back((float)c[i]);
        // section 2.3.2: CDF of the spectrum at the edges of K equal-width
        // intervals over its support (area of the pdf below e over the total)
        if (d->spectrum_strata > 0) {
            const int K = d->spectrum_strata;
            const double e0 = sp.e_mev[0], e1 = sp.e_mev[sp.n_pts - 1];
            strata_F.assign(K + 1, 0.0);
            for (int k = 1; k < K; ++k) {
                const double e = e0 + (e1 - e0) * k / K;
                int j = 0;
                while (j < sp.n_pts - 2 && sp.e_mev[j + 1] <= e) ++j;
                const double t = (e - sp.e_mev[j]) / (sp.e_mev[j + 1] - sp.e_mev[j]);
                const double pe = sp.pdf[j] + t * (sp.pdf[j + 1] - sp.pdf[j]);
                strata_F[k] = (c[j] + 0.5 * (sp.pdf[j] + pe) * (e - sp.e_mev[j])) / area;
            }
            strata_F[K] = 1.0;
        }
        src->spec_n = sp.n_pts;
        src->e_mono = 0.0f;
        src->e_max = sp.e_mev[sp.n_pts - 1];
    } else {
        return fail(GDPM_E_INVALID, "spectrum kind must be 0 or 1");
    }
    // beams and the beamlet cumulative probabilities P(I): normalised prefix
    // sums of f_I over all beams (section 2.3.1), in double precision
    std::vector<BeamDev> beams(d->n_beams);
    size_t nf = 0;
    for (int b = 0; b < d->n_beams; ++b) {
        const gdpm_beam& bm = d->beams[b];
        if (bm.nbx < 1 || bm.nby < 1 || !(bm.bw_cm > 0) || !(bm.bh_cm > 0))
            return fail(GDPM_E_INVALID, "beam %d: bad beamlet grid", b);
        double dn = 0, en = 0, de = 0;
        for (int i = 0; i < 3; ++i) {
            dn += bm.dir[i] * bm.dir[i];
            en += bm.e1[i] * bm.e1[i];
            de += bm.dir[i] * bm.e1[i];
            if (!std::isfinite(bm.iso_cm[i])) return fail(GDPM_E_INVALID, "beam %d: bad isocentre", b);
        }
        if (std::fabs(dn - 1) > 1e-6 || std::fabs(en - 1) > 1e-6 || std::fabs(de) > 1e-6)
            return fail(GDPM_E_INVALID, "beam %d: dir and e1 must be orthonormal", b);
        nf += (size_t)bm.nbx * bm.nby;
    }
    if (nf > ((size_t)1 << 30)) return fail(GDPM_E_INVALID, "too many beamlets");
    std::vector<double> cdf(nf + 1, 0.0);
    std::vector<uint16_t> beam_of(nf);
    std::vector<float> fl(nf);
    std::vector<uint32_t> nzl;
    double tot = 0.0;
    size_t gi = 0;
    for (int b = 0; b < d->n_beams; ++b) {
        const gdpm_beam& bm = d->beams[b];
        BeamDev& o = beams[b];
        const double e2[3] = {bm.dir[1] * bm.e1[2] - bm.dir[2] * bm.e1[1],
                              bm.dir[2] * bm.e1[0] - bm.dir[0] * bm.e1[2],
                              bm.dir[0] * bm.e1[1] - bm.dir[1] * bm.e1[0]};
        for (int i = 0; i < 3; ++i) {
            o.iso[i] = (float)bm.iso_cm[i];
            o.dir[i] = (float)bm.dir[i];
            o.e1[i] = (float)bm.e1[i];
            o.e2[i] = (float)e2[i];
        }
        o.sad = (float)bm.sad_cm;
        o.bw = (float)bm.bw_cm;
        o.bh = (float)bm.bh_cm;
        o.hx = (float)(0.5 * bm.nbx * bm.bw_cm);
        o.hy = (float)(0.5 * bm.nby * bm.bh_cm);
        o.nbx = bm.nbx;
        o.nby = bm.nby;
        o.off = (int)gi;
        for (int j = 0; j < bm.nbx * bm.nby; ++j, ++gi) {
            double f = bm.intensity ? (double)bm.intensity[j] : 1.0;
            if (!std::isfinite(f)) return fail(GDPM_E_INVALID, "beam %d: intensity not finite", b);
            if (f < 0.0) f = 0.0;
            cdf[gi] = tot;
            beam_of[gi] = (uint16_t)b;
            fl[gi] = (float)f;
            if (f > 0.0) nzl.push_back((uint32_t)gi);
            tot += f;
        }
    }
    if (!(tot > 0.0)) return fail(GDPM_E_INVALID, "fluence maps are all zero");
    for (size_t i = 0; i < nf; ++i) cdf[i] /= tot;
    cdf[nf] = 1.0;
    // guide table (indexed search): guide[k] = I with P(I) <= k / G < P(I+1)
    const size_t ng = std::max<size_t>(1, nf);
    std::vector<uint32_t> guide(ng);
    size_t I = 0;
    for (size_t k = 0; k < ng; ++k) {
        const double r = (double)k / (double)ng;
        while (I + 1 < nf && cdf[I + 1] <= r) ++I;
        guide[k] = (uint32_t)I;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(upload(src->spec_e, se));
    HIP_TRY(upload(src->spec_p, spp));
    HIP_TRY(upload(src->spec_c, sc));
    HIP_TRY(upload(src->cdf, cdf));
    HIP_TRY(upload(src->guide, guide));
    HIP_TRY(upload(src->beams, beams));
    HIP_TRY(upload(src->beam_of, beam_of));
    src->strata = d->spectrum_strata;
    if (src->strata) {
        HIP_TRY(upload(src->strata_F, strata_F));
        src->strata_shape = d->strata_shape;
        const double e0 = sp.e_mev[0], e1 = sp.e_mev[sp.n_pts - 1];
        src->strata_lo = (float)e0;
        src->strata_w = (float)((e1 - e0) / src->strata);
    }
    src->metro = d->beamlet_sampler;
    if (src->metro) {
        HIP_TRY(upload(src->fl, fl));
        HIP_TRY(upload(src->nz, nzl));
        src->n_nz = (int)nzl.size();
    }
    src->nf = (int)nf;
    src->n_guide = (int)ng;
    src->n_beams = d->n_beams;
    *out = src.release();
    return GDPM_OK;
}

gdpm_status gdpm_source_destroy(gdpm_source src) {
    if (!src) return fail(GDPM_E_INVALID, "NULL source");
    delete src;
    return GDPM_OK;
}

gdpm_status gdpm_run(gdpm_context ctx, gdpm_phantom ph, gdpm_source src, const gdpm_run_params* prm,
                     double* dose, double* sigma, double* batch_edep, double* hist_out,
                     gdpm_run_stats* stats) {
    if (!ctx) return fail(GDPM_E_INVALID, "NULL context");
    if (ctx->busy) return fail(GDPM_E_BUSY, "context busy");
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->busy = true;
    EJob job;
    gdpm_status s = do_run(ctx, ph, src, prm, nullptr, nullptr, batch_edep, hist_out, ctx->stream,
                           stats, &job);
    ctx->busy = false;
    if (s != GDPM_OK && s != GDPM_E_NOT_CONVERGED) return s;
    const std::string msg = g_err;
    if (dose) HIP_TRY(hipMemcpy(dose, job.d_dose, job.nv * sizeof(double), hipMemcpyDeviceToHost));
    if (sigma) HIP_TRY(hipMemcpy(sigma, job.d_sigma, job.nv * sizeof(double), hipMemcpyDeviceToHost));
    g_err = msg;
    return s;
}

gdpm_status gdpm_run_async(gdpm_context ctx, gdpm_phantom ph, gdpm_source src,
                           const gdpm_run_params* prm, double* d_dose, double* d_sigma,
                           void* hip_stream, gdpm_job* out) {
    if (!ctx || !out) return fail(GDPM_E_INVALID, "NULL argument");
    *out = nullptr;
    if (ctx->busy) return fail(GDPM_E_BUSY, "context busy");
    HIP_TRY(hipSetDevice(ctx->device));
    auto job = std::make_unique<gdpm_job_s>();
    job->ctx = ctx;
    memset(&job->stats, 0, sizeof job->stats);
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    ctx->busy = true;
    job->status = do_run(ctx, ph, src, prm, d_dose, d_sigma, nullptr, nullptr, st, &job->stats, nullptr);
    ctx->busy = false;
    if (job->status != GDPM_OK && job->status != GDPM_E_NOT_CONVERGED) return job->status;
    *out = job.release();
    return GDPM_OK;
}

gdpm_status gdpm_run_noalloc(gdpm_context ctx, gdpm_phantom ph, gdpm_source src,
                             const gdpm_run_params* prm, double* d_dose, double* d_sigma,
                             void* hip_stream, gdpm_run_stats* stats) {
    if (!ctx || !d_dose || !d_sigma) return fail(GDPM_E_INVALID, "NULL context or output");
    if (ctx->busy) return fail(GDPM_E_BUSY, "context busy");
    if (!ctx->scratch) return fail(GDPM_E_DEVICE, "no scratch memory on device %d", ctx->device);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    ctx->busy = true;
    const gdpm_status s = do_run(ctx, ph, src, prm, d_dose, d_sigma, nullptr, nullptr, st, stats,
                                 nullptr, ctx->scratch);
    ctx->busy = false;
    return s;
}

gdpm_status gdpm_run_batch(gdpm_context ctx, int n, const gdpm_job_desc* jobs,
                           gdpm_run_stats* stats, gdpm_status* status) {
    if (!ctx || !jobs || n < 1) return fail(GDPM_E_INVALID, "need a context and n >= 1 jobs");
    if (ctx->busy) return fail(GDPM_E_BUSY, "context busy");
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<std::unique_ptr<EJob>> ej;
    for (int i = 0; i < n; ++i) {
        ej.emplace_back(new EJob);
        gdpm_status s = make_job(ctx, jobs[i].phantom, jobs[i].source, &jobs[i].params, ej.back().get());
        if (s) return fail(s, "job %d: %s", i, g_err.c_str());
    }
    if (status)
        for (int i = 0; i < n; ++i) status[i] = GDPM_OK;
    ctx->busy = true;
    struct Busy {
        gdpm_context c;
        ~Busy() { c->busy = false; }
    } busy{ctx};
    hipStream_t st = ctx->stream;
    const double t0 = now_s();
    if (ctx->autotune) {
        // queue capacity from the work submitted: room for the first
        // super-rounds of all jobs in a few iterations (2^21 .. 2^26 records)
        double work = 0.0;
        for (auto& j : ej) work += (double)j->plan.n_hist;
        const int lg = (int)std::ceil(std::log2(std::max(work, 1.0)));
        ctx->ring_log2 = std::min(26, std::max(21, lg));
    }
    Engine E;
    gdpm_status s = E.init(ctx, st, ej[0]->plan);
    if (s) return s;
    int next = 0, left = n;
    gdpm_status first_err = GDPM_OK;
    while (left > 0) {
        // admit while slots and memory allow
        while (next < n) {
            EJob* j = ej[next].get();
            s = E.admit(j);
            if (s == GDPM_E_BUSY || (s == GDPM_E_NOMEM && E.any_active())) {
                (void)hipGetLastError();
                break;
            }
            if (s) return fail(s, "job %d: %s", next, g_err.c_str());
            ++next;
        }
        s = E.step();
        if (!s) s = E.settle();
        if (s) {
            first_err = s;
            break;
        }
        for (int i = 0; i < next; ++i) {
            EJob* j = ej[i].get();
            if (!j->done || j->slot < 0) continue;
            // outputs of a finished job, then its device memory goes back
            if (jobs[i].dose)
                HIP_TRY(hipMemcpyAsync(jobs[i].dose, j->d_dose, j->nv * sizeof(double), hipMemcpyDeviceToHost, st));
            if (jobs[i].sigma)
                HIP_TRY(hipMemcpyAsync(jobs[i].sigma, j->d_sigma, j->nv * sizeof(double), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (stats) fill_stats(E, j, t0, &stats[i]);
            if (status) status[i] = j->status;
            E.release(j);
            j->tally.reset();
            j->dose_buf.reset();
            j->sigma_buf.reset();
            j->mumax.reset();
            j->chains.reset();
            --left;
        }
    }
    if (first_err) {
        const std::string msg = g_err;
        if (status)
            for (int i = 0; i < n; ++i)
                if (!ej[i]->done) status[i] = first_err;
        (void)hipStreamSynchronize(st);
        g_err = msg;
        return first_err;
    }
    return GDPM_OK;
}

gdpm_status gdpm_context_settings(gdpm_context ctx, int out[5]) {
    if (!ctx || !out) return fail(GDPM_E_INVALID, "NULL argument");
    out[0] = ctx->waves_per_cu;
    out[1] = ctx->rebin_bins;
    out[2] = ctx->ring_log2;
    out[3] = ctx->pass_histories;
    out[4] = ctx->autotune;
    return GDPM_OK;
}

gdpm_status gdpm_context_tuning(gdpm_context ctx, int cap, int* n, int* cand, double* score, int* kept) {
    if (!ctx || !n || !kept || cap < 0 || (cap > 0 && (!cand || !score)))
        return fail(GDPM_E_INVALID, "NULL argument");
    *n = (int)ctx->tune_cand.size();
    *kept = ctx->tune_kept;
    for (int i = 0; i < std::min(cap, *n); ++i) {
        cand[2 * i] = ctx->tune_cand[i].first;
        cand[2 * i + 1] = ctx->tune_cand[i].second;
        score[i] = ctx->tune_score[i];
    }
    return GDPM_OK;
}

gdpm_status gdpm_job_wait(gdpm_job job, gdpm_run_stats* stats) {
    if (!job) return fail(GDPM_E_INVALID, "NULL job");
    if (job->srv) {
        std::unique_lock<std::mutex> lk(job->srv->m);
        job->srv->cv_done.wait(lk, [&] { return job->finished; });
    }
    if (stats) *stats = job->stats;
    if (job->status != GDPM_OK) g_err = job->err;
    return job->status;
}

gdpm_status gdpm_job_release(gdpm_job job) {
    if (!job) return fail(GDPM_E_INVALID, "NULL job");
    if (job->srv) {
        std::lock_guard<std::mutex> lk(job->srv->m);
        if (!job->finished) return fail(GDPM_E_BUSY, "the job has not finished");
    }
    delete job;
    return GDPM_OK;
}

gdpm_status gdpm_server_create(gdpm_context ctx, uint64_t hbm_budget_bytes, int max_slots,
                               gdpm_server* out) {
    if (!ctx || !out) return fail(GDPM_E_INVALID, "NULL argument");
    *out = nullptr;
    if (max_slots < 1 || max_slots > kMaxJobs) return fail(GDPM_E_INVALID, "max_slots in [1, %d]", kMaxJobs);
    if (hbm_budget_bytes == 0) return fail(GDPM_E_INVALID, "hbm_budget_bytes must be > 0");
    if (ctx->busy) return fail(GDPM_E_BUSY, "context busy");
    HIP_TRY(hipSetDevice(ctx->device));
    auto srv = std::make_unique<gdpm_server_s>();
    srv->ctx = ctx;
    srv->budget = hbm_budget_bytes;
    srv->max_slots = max_slots;
    ctx->busy = true;
    try {
        srv->th = std::thread([s = srv.get()] { s->loop(); });
    } catch (...) {
        ctx->busy = false;
        return fail(GDPM_E_NOMEM, "cannot start the server thread");
    }
    *out = srv.release();
    return GDPM_OK;
}

gdpm_status gdpm_server_submit(gdpm_server srv, const gdpm_job_desc* d, gdpm_job* out) {
    if (!srv || !d || !out) return fail(GDPM_E_INVALID, "NULL argument");
    *out = nullptr;
    auto job = std::make_unique<gdpm_job_s>();
    job->ctx = srv->ctx;
    job->srv = srv;
    job->ej.reset(new EJob);
    gdpm_status s = make_job(srv->ctx, d->phantom, d->source, &d->params, job->ej.get());
    if (s) return s;
    const EJob& j = *job->ej;
    const TableKey k{j.plan.ecut_g, j.plan.ecut_e, j.plan.flags & 0x3Fu};
    job->dose = d->dose;
    job->sigma = d->sigma;
    job->finished = false;
    job->ej->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(srv->m);
        if (srv->stop) return fail(GDPM_E_INVALID, "the server is stopping");
        if (!srv->key_set) {
            srv->key = k;
            srv->key_set = true;
        } else if (k < srv->key || srv->key < k) {
            return fail(GDPM_E_INVALID, "jobs of a server must share cutoffs and physics flags");
        }
        srv->pending.push_back(job.get());
        srv->submitted++;
    }
    srv->cv_work.notify_all();
    *out = job.release();
    return GDPM_OK;
}

gdpm_status gdpm_server_info_get(gdpm_server srv, gdpm_server_info* info) {
    if (!srv || !info) return fail(GDPM_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->m);
    memset(info, 0, sizeof *info);
    info->submitted = srv->submitted;
    info->finished = srv->finished;
    info->running = srv->running.size();
    info->queued = srv->pending.size();
    info->histories = srv->histories;
    info->footprint_bytes = (double)srv->used;
    info->high_water_bytes = (double)srv->high_water;
    gdpm_context ctx = srv->ctx;
    double res = (double)(ctx->ctl.bytes + ctx->jobs_dev.bytes + ctx->jc.bytes + ctx->segs.bytes);
    for (int r = 0; r < 2; ++r) res += (double)(ctx->rings[r].bytes + ctx->bins[r].bytes);
    for (auto& t : ctx->tables)
        res += (double)(t.second->phot.bytes + t.second->elec.bytes + t.second->rinv.bytes +
                        t.second->rinv_scale.bytes + t.second->aw.bytes + t.second->kn.bytes);
    res += ctx->resident_bytes;
    info->resident_bytes = res;
    return GDPM_OK;
}

gdpm_status gdpm_server_destroy(gdpm_server srv) {
    if (!srv) return fail(GDPM_E_INVALID, "NULL server");
    {
        std::lock_guard<std::mutex> lk(srv->m);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->th.joinable()) srv->th.join();
    srv->ctx->busy = false;
    delete srv;
    return GDPM_OK;
}

gdpm_status gdpm_tables_host(const gdpm_material* m, int n, int n_grid, double ecut_g, double ecut_e,
                             uint32_t flags, int which, float* out, size_t cap, size_t* len,
                             double grid[4]) {
    if (!m || !len) return fail(GDPM_E_INVALID, "NULL argument");
    if (n < 1 || n > kMaxMaterials) return fail(GDPM_E_INVALID, "1..%d materials", kMaxMaterials);
    if (n_grid == 0) n_grid = 1024;
    std::vector<MaterialParams> mats(n);
    for (int i = 0; i < n; ++i) mats[i] = {m[i].z, m[i].z_over_a, m[i].i_ev};
    HostTables T;
    std::string err;
    if (!build_tables(mats, n_grid, ecut_g, ecut_e, flags & 0x3Fu, &T, &err))
        return fail(GDPM_E_INVALID, "%s", err.c_str());
    const std::vector<float>* v = nullptr;
    double g[4] = {0, 0, 0, (double)n};
    switch (which) {
    case 0: v = &T.phot; g[0] = T.pg_lo; g[1] = T.pg_step; g[2] = T.pg_n; break;
    case 1: v = &T.elec; g[0] = T.eg_lo; g[1] = T.eg_step; g[2] = T.eg_n; break;
    case 2: v = &T.rinv; g[0] = 0.0; g[1] = 0.0; g[2] = T.nr; break;
    case 3: v = &T.aw; g[0] = T.aw_lo; g[1] = T.aw_step; g[2] = T.aw_n; break;
    case 4: v = &T.kn; g[0] = T.kn_lo; g[1] = T.kn_step; g[2] = T.kn_ne; g[3] = T.kn_nu; break;
    default: return fail(GDPM_E_INVALID, "which must be 0..4");
    }
    if (which == 2) {
        // the grid spacing of the inverse range differs per material: return w_max of material 0
        g[1] = 1.0 / T.rinv_scale[0];
    }
    *len = v->size();
    if (grid) memcpy(grid, g, sizeof g);
    if (out) {
        if (cap < v->size()) return fail(GDPM_E_INVALID, "output holds %zu floats, %zu needed", cap, v->size());
        memcpy(out, v->data(), v->size() * sizeof(float));
    }
    return GDPM_OK;
}

gdpm_status gdpm_test_philox(gdpm_context ctx, const uint32_t key[2], const uint32_t* ctr,
                             uint32_t* out, int n) {
    if (!ctx || !key || !ctr || !out || n < 1) return fail(GDPM_E_INVALID, "bad arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    DevBuf a, b;
    HIP_TRY(a.alloc((size_t)n * 16));
    HIP_TRY(b.alloc((size_t)n * 16));
    HIP_TRY(hipMemcpy(a.p, ctr, (size_t)n * 16, hipMemcpyHostToDevice));
    HIP_TRY(launch_test_philox(ctx->stream, key[0], key[1], a.as<const uint4>(), b.as<uint4>(), n));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(out, b.p, (size_t)n * 16, hipMemcpyDeviceToHost));
    return GDPM_OK;
}

gdpm_status gdpm_test_atomic_rate(gdpm_context ctx, uint64_t bytes, double* ops_per_s) {
    if (!ctx || !ops_per_s || bytes < 8 || bytes > (1ull << 34))
        return fail(GDPM_E_INVALID, "bad arguments (8 B <= footprint <= 16 GiB)");
    HIP_TRY(hipSetDevice(ctx->device));
    const uint64_t n = bytes / 8;
    const int blocks = 8 * grid_blocks(ctx);
    const uint32_t iters = 64;
    DevBuf buf;
    HIP_TRY(buf.alloc(n * 8));
    HIP_TRY(hipMemsetAsync(buf.p, 0, n * 8, ctx->stream));
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    float ms = 0.0f;
    hipError_t e = hipSuccess;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the second launch is timed
        e = hipEventRecord(a, ctx->stream);
        if (e == hipSuccess) e = launch_atomic_rate(ctx->stream, blocks, buf.as<double>(), (uint32_t)n, iters);
        if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    HIP_TRY(e);
    // every addition landed: the array sums to the number made (exact in FP64)
    std::vector<double> h(n);
    HIP_TRY(hipMemcpy(h.data(), buf.p, n * 8, hipMemcpyDeviceToHost));
    double sum = 0.0;
    for (double v : h) sum += v;
    const double ops = (double)blocks * 256.0 * iters;
    if (sum != 2.0 * ops) return fail(GDPM_E_DEVICE, "atomic probe lost additions: %.0f of %.0f", sum, 2.0 * ops);
    *ops_per_s = ms > 0.0f ? ops / (ms * 1e-3) : 0.0;
    return GDPM_OK;
}

gdpm_status gdpm_test_sample(gdpm_context ctx, int which, double e, double p1, double p2,
                             uint64_t seed, int n, float* out1, float* out2) {
    if (!ctx || !out1 || n < 1 || which < 0 || which > 7) return fail(GDPM_E_INVALID, "bad arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    DevTables* tab = nullptr;
    gdpm_status s = get_tables(ctx, 0.05, 0.2, 0u, &tab);
    if (s) return s;
    DevBuf a, b;
    HIP_TRY(a.alloc((size_t)n * 4));
    HIP_TRY(b.alloc((size_t)n * 4));
    HIP_TRY(launch_test_sample(ctx->stream, tab->view(nullptr), which, (float)e, (float)p1, (float)p2,
                               (uint32_t)seed, (uint32_t)(seed >> 32), n, a.as<float>(), b.as<float>()));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(out1, a.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (out2) HIP_TRY(hipMemcpy(out2, b.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    return GDPM_OK;
}

gdpm_status gdpm_test_source(gdpm_context ctx, gdpm_phantom ph, gdpm_source src, uint64_t seed,
                             uint32_t job, uint64_t hist0, int n, float* out) {
    if (!ctx || !ph || !src || !out || n < 1) return fail(GDPM_E_INVALID, "bad arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    DevBuf a;
    HIP_TRY(a.alloc((size_t)n * 32));
    HIP_TRY(launch_test_source(ctx->stream, src->view(), geom_of(ph), (uint32_t)seed,
                               (uint32_t)(seed >> 32) ^ job, (unsigned long long)hist0, n, a.as<float>()));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(out, a.p, (size_t)n * 32, hipMemcpyDeviceToHost));
    return GDPM_OK;
}

gdpm_status gdpm_test_lookup(gdpm_context ctx, double ecut_g, double ecut_e, uint32_t flags, int which,
                             int mat, const float* in, float* out, int n) {
    if (!ctx || !in || !out || n < 1 || which < 0 || which > 6) return fail(GDPM_E_INVALID, "bad arguments");
    if (mat < 0 || mat >= (int)ctx->mats.size()) return fail(GDPM_E_INVALID, "material out of range");
    HIP_TRY(hipSetDevice(ctx->device));
    DevTables* tab = nullptr;
    gdpm_status s = get_tables(ctx, ecut_g, ecut_e, flags, &tab);
    if (s) return s;
    DevBuf a, b;
    HIP_TRY(a.alloc((size_t)n * 4));
    HIP_TRY(b.alloc((size_t)n * 4));
    HIP_TRY(hipMemcpy(a.p, in, (size_t)n * 4, hipMemcpyHostToDevice));
    HIP_TRY(launch_test_lookup(ctx->stream, tab->view(nullptr), which, mat, a.as<const float>(),
                               b.as<float>(), n));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(out, b.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    return GDPM_OK;
}

}  // extern "C"
