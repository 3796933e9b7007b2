// Transport kernels of libgdpm for gfx950 (CDNA4, 64-wide wavefronts).
//
// The paper separates photon and electron transport into different kernel
// launches so that threads of a warp follow the same physics (section 2.2.1,
// Fig. 1): particles live in a particle array and two secondary stacks, and the
// host alternates source generation, photon kernels and electron kernels.
// Here the same separation is kept (one queue per particle type, one kernel per
// type) but the launch shape is built for CDNA:
//   - a kernel is a persistent grid of wavefronts; each lane holds one
//     particle and advances it by one event per iteration (one Woodcock flight
//     for a photon, one condensed-history step for an electron); a lane whose
//     particle ends takes the next one from the queue (or starts a new source
//     history), so lanes stay busy instead of idling until the slowest particle
//     of the wave finishes;
//   - queue traffic is per wavefront: a ballot + mbcnt prefix gives each lane
//     its slot and one atomic per 256 records reserves ring space, one atomic
//     per 64 items claims input;
//   - dose goes into double-precision tallies with hardware FP64 atomics, one
//     per voxel visit of a charged particle (deposits merged in registers).
// Random numbers: Philox4x32-10 (Salmon et al., SC'11); a particle owns the
// stream (history id, path id) and the draw order of each event is fixed, so
// results do not depend on scheduling.
// Energy is conserved exactly in single precision: when an energy X splits in
// two, the larger part L >= X/2 is computed and the smaller is X - L, which is
// exact (Sterbenz).  This unit is therefore compiled without floating-point
// contraction; fused multiply-adds are written out with fmaf.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_types.h"

namespace gdpm {

#define GDPM_DEV __device__ __forceinline__
#define GDPM_HD __host__ __device__ inline

constexpr float kMec2f = 0.51099895f;
constexpr float kTwoMec2f = 1.0219979f;
constexpr float kLn2f = 0.693147180559945f;
constexpr float kMwIsoF = 20.0f;

// ---------------------------------------------------------------------------
// hardware math (v_log_f32 is log2, v_exp_f32 is 2^x, v_sin/v_cos take turns)
// ---------------------------------------------------------------------------
GDPM_DEV float hlog2(float x) { return __builtin_amdgcn_logf(x); }
GDPM_DEV float hexp2(float x) { return __builtin_amdgcn_exp2f(x); }
GDPM_DEV float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
GDPM_DEV float hrsq(float x) { return __builtin_amdgcn_rsqf(x); }
GDPM_DEV float hrcp(float x) { return __builtin_amdgcn_rcpf(x); }
GDPM_DEV float sin_turns(float t) { return __builtin_amdgcn_sinf(t); }
GDPM_DEV float cos_turns(float t) { return __builtin_amdgcn_cosf(t); }
GDPM_DEV float neg_ln(float u) { return -kLn2f * hlog2(u); }

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------
GDPM_DEV uint32_t lane_id() { return __lane_id(); }
GDPM_DEV uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
GDPM_DEV uint64_t ballot(bool p) { return __ballot(p); }
GDPM_DEV uint32_t first_lane(uint64_t m) { return (uint32_t)(__ffsll((unsigned long long)m) - 1); }
GDPM_DEV uint32_t bcast(uint32_t v, uint32_t lane) { return __builtin_amdgcn_readlane(v, lane); }
// device-coherent load of a counter, made wave-uniform
GDPM_DEV uint32_t load_agent(const uint32_t* p) {
    return __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

GDPM_DEV double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
GDPM_DEV uint32_t wave_sum(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------
// Philox4x32-10
// ---------------------------------------------------------------------------
GDPM_DEV void philox(uint32_t k0, uint32_t k1, uint32_t& x0, uint32_t& x1, uint32_t& x2,
                     uint32_t& x3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product per multiplier
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x0 = y0;
        x1 = (uint32_t)p1;
        x2 = y2;
        x3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// A lane's stream: key (k0, k1), counter (hist lo, hist hi, path, draw >> 2);
// draw d is word d & 3 of its block.  A (block `blk`, next word `i`, 4 = used
// up) is followed by at most one queued block C (blk + 1, flag `qc`).  Blocks
// are generated with the wavefront converged: rng_topup once per iteration
// and at the start of a batch of interactions (A has a word left and C is
// queued: at least 5 draws, enough for a flight or an electron step, and for
// a photon interaction, which draws at most 4 with the inverse-CDF Compton
// sampler).  A lane that still runs out (a rejection loop of an electron hard
// event) takes the out-of-line path, which costs a whole wavefront's Philox
// for the few lanes in it.  Blocks are only ever generated in counter order,
// so the draws are the same whatever is buffered.
struct Rng {
    uint32_t hlo, hhi, path;
    uint32_t blk, i, skip;
    uint32_t a0, a1, a2, a3;
    uint32_t c0, c1, c2, c3;
    bool qc;
};

// counter of the next draw
GDPM_DEV uint32_t rng_ctr(const Rng& r) { return 4u * r.blk + r.i; }

// position the stream at draw `ctr` (no block generated yet)
GDPM_DEV void rng_start(Rng& r, uint32_t hlo, uint32_t hhi, uint32_t path, uint32_t ctr) {
    r.hlo = hlo;
    r.hhi = hhi;
    r.path = path;
    r.blk = (ctr >> 2) - 1u;  // A is "used up"; the next block is ctr >> 2
    r.i = 4u;
    r.skip = ctr & 3u;
    r.qc = false;
}

__device__ __attribute__((noinline)) uint4 rng_block_slow(uint32_t k0, uint32_t k1, uint32_t hlo,
                                                         uint32_t hhi, uint32_t path, uint32_t blk) {
    uint32_t x0 = hlo, x1 = hhi, x2 = path, x3 = blk;
    philox(k0, k1, x0, x1, x2, x3);
    return make_uint4(x0, x1, x2, x3);
}

GDPM_DEV uint4 rng_block(uint32_t k0, uint32_t k1, const Rng& r, uint32_t blk) {
    uint32_t x0 = r.hlo, x1 = r.hhi, x2 = r.path, x3 = blk;
    philox(k0, k1, x0, x1, x2, x3);
    return make_uint4(x0, x1, x2, x3);
}

// A used up: the next block becomes A (from the queue, else generated here,
// inline or out of line)
GDPM_DEV void rng_advance(Rng& r, uint32_t k0, uint32_t k1, bool inline_block) {
    if (r.qc) {
        r.a0 = r.c0; r.a1 = r.c1; r.a2 = r.c2; r.a3 = r.c3;
        r.qc = false;
    } else {
        const uint4 b = inline_block ? rng_block(k0, k1, r, r.blk + 1u)
                                     : rng_block_slow(k0, k1, r.hlo, r.hhi, r.path, r.blk + 1u);
        r.a0 = b.x; r.a1 = b.y; r.a2 = b.z; r.a3 = b.w;
    }
    r.blk += 1u;
    r.i = r.skip;
    r.skip = 0u;
}

// queue the next block (C)
GDPM_DEV void rng_queue(Rng& r, uint32_t k0, uint32_t k1) {
    const uint4 b = rng_block(k0, k1, r, r.blk + 1u);
    r.c0 = b.x; r.c1 = b.y; r.c2 = b.z; r.c3 = b.w;
    r.qc = true;
}

// make sure A has a word left and C is queued
GDPM_DEV void rng_topup(Rng& r, uint32_t k0, uint32_t k1) {
    if (r.i == 4u) rng_advance(r, k0, k1, true);
    if (!r.qc) rng_queue(r, k0, k1);
}

// (2 (x >> 9) + 1) 2^-24: exact in single and double precision, inside (0, 1)
GDPM_DEV float uniform(Rng& r, uint32_t k0, uint32_t k1) {
    if (r.i == 4u) rng_advance(r, k0, k1, false);
    const uint32_t w = r.i;
    const uint32_t x = w == 0u ? r.a0 : (w == 1u ? r.a1 : (w == 2u ? r.a2 : r.a3));
    r.i = w + 1u;
    return (float)(x >> 9) * 0x1p-23f + 0x1p-24f;
}

// path id of the secondary created in role `word` at the parent's current counter
GDPM_DEV uint32_t spawn_path(const Rng& r, uint32_t k0, uint32_t k1, int word) {
    uint32_t x0 = r.hlo, x1 = r.hhi, x2 = r.path, x3 = 0x80000000u | rng_ctr(r);
    philox(k0, k1, x0, x1, x2, x3);
    return word == 0 ? x0 : (word == 1 ? x1 : (word == 2 ? x2 : x3));
}

// non-exact division through the hardware reciprocal (about 1 ulp)
GDPM_DEV float fdiv(float a, float b) { return a * hrcp(b); }

// ---------------------------------------------------------------------------
// table lookups (linear in log2 E)
// ---------------------------------------------------------------------------
GDPM_DEV void grid(float lg, float lo, float inv, int n, int& i, float& t) {
    float f = (lg - lo) * inv;
    f = fminf(fmaxf(f, 0.0f), (float)(n - 1));
    i = min((int)f, n - 2);
    t = f - (float)i;
}

GDPM_DEV float4 lerp4(const float4* tab, int i, float t) {
    const float4 a = tab[i], b = tab[i + 1];
    return make_float4(fmaf(t, b.x - a.x, a.x), fmaf(t, b.y - a.y, a.y), fmaf(t, b.z - a.z, a.z),
                       fmaf(t, b.w - a.w, a.w));
}

GDPM_DEV float lerp1(const float* tab, int i, float t) {
    const float a = tab[i], b = tab[i + 1];
    return fmaf(t, b - a, a);
}

GDPM_DEV float4 elec_at(const Tables& T, const float4* etab, int m, float e) {
    int i;
    float t;
    grid(hlog2(e), T.eg_lo, T.eg_inv, T.eg_n, i, t);
    return lerp4(etab + m * T.eg_n, i, t);
}
GDPM_DEV float4 elec_at(const Tables& T, int m, float e) { return elec_at(T, T.elec, m, e); }

// energy whose residual range is r (g/cm^2); rtab holds the material's nodes
// followed (after all materials) by the per-material scales
GDPM_DEV float range_inv(const Tables& T, const float* rtab, const float* rscale, int m, float r) {
    const float f = fminf(hsqrt(fmaxf(r, 0.0f)) * rscale[m], (float)(T.nr - 1));
    const int i = min((int)f, T.nr - 2);
    return lerp1(rtab + m * T.nr, i, f - (float)i);
}
GDPM_DEV float range_inv(const Tables& T, int m, float r) {
    return range_inv(T, T.rinv, T.rinv_scale, m, r);
}

// screening A of the modified-Wentzel law for t = s / lambda_1 (t < t_iso)
GDPM_DEV float mw_screening(const Tables& T, float tt) {
    const float f = fminf((hlog2(tt) - T.aw_lo) * T.aw_inv, (float)(T.aw_n - 1));
    const int i = min(max((int)f, 0), T.aw_n - 2);  // f < 0 extrapolates the first cell
    return hexp2(lerp1(T.aw, i, f - (float)i));
}

// modified-Wentzel deflection mu = (1 - cos)/2 for t = s / lambda_1
GDPM_DEV float mw_mu(const Tables& T, float tt, float u) {
    if (!(tt < kMwIsoF)) return u;
    const float a = mw_screening(T, tt);
    return fdiv(a * u, 1.0f + a - u);
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
GDPM_DEV void rotate(float& u, float& v, float& w, float ct, float st, float turns) {
    const float cp = cos_turns(turns), sp = sin_turns(turns);
    const float r2 = u * u + v * v;
    float nu, nv, nw;
    if (r2 > 1e-12f) {
        const float ir = hrsq(r2), r = r2 * ir;
        nu = u * ct + st * (u * w * cp - v * sp) * ir;
        nv = v * ct + st * (v * w * cp + u * sp) * ir;
        nw = w * ct - st * cp * r;
    } else {
        nu = st * cp;
        nv = st * sp;
        nw = (w >= 0.0f ? ct : -ct);
    }
    const float n = hrsq(nu * nu + nv * nv + nw * nw);
    u = nu * n;
    v = nv * n;
    w = nw * n;
}

GDPM_DEV int clampi(int x, int n) { return min(max(x, 0), n - 1); }

GDPM_DEV int voxel_of(const Geom& G, float x, float y, float z, int& ix, int& iy, int& iz) {
    ix = clampi((int)floorf(x * G.idx), G.nx);
    iy = clampi((int)floorf(y * G.idy), G.ny);
    iz = clampi((int)floorf(z * G.idz), G.nz);
    return ix + G.nx * (iy + G.ny * iz);
}

GDPM_DEV uint32_t pack_vox(int ix, int iy, int iz) {
    return (uint32_t)ix | ((uint32_t)iy << 11) | ((uint32_t)iz << 22);
}

GDPM_DEV bool outside(const Geom& G, float x, float y, float z) {
    return !(x >= 0.0f && x < G.lx && y >= 0.0f && y < G.ly && z >= 0.0f && z < G.lz);
}

// distance to the exit face of voxel (ix, iy, iz) along the direction; axis of that face
GDPM_DEV float face_dist(const Geom& G, float x, float y, float z, float u, float v, float w,
                         int ix, int iy, int iz, int& ax) {
    float best = 3.0e38f;
    ax = 0;
    if (u != 0.0f) {
        const float d = fdiv((u > 0.0f ? (float)(ix + 1) : (float)ix) * G.dx - x, u);
        best = d;
    }
    if (v != 0.0f) {
        const float d = fdiv((v > 0.0f ? (float)(iy + 1) : (float)iy) * G.dy - y, v);
        if (d < best) {
            best = d;
            ax = 1;
        }
    }
    if (w != 0.0f) {
        const float d = fdiv((w > 0.0f ? (float)(iz + 1) : (float)iz) * G.dz - z, w);
        if (d < best) {
            best = d;
            ax = 2;
        }
    }
    return fmaxf(best, 0.0f);
}

// ---------------------------------------------------------------------------
// source: history h -> primary particle (section 2.3)
// ---------------------------------------------------------------------------
GDPM_DEV float spectrum_energy(const SourceDev& S, float u) {
    if (S.spec_kind == 0) return S.e_mono;
    const int n = S.spec_n;
    const float r = u * S.spec_c[n - 1];
    int j = 0;
    while (j < n - 2 && S.spec_c[j + 1] <= r) ++j;
    const float e0 = S.spec_e[j], e1 = S.spec_e[j + 1];
    const float p0 = S.spec_p[j], sl = (S.spec_p[j + 1] - p0) / (e1 - e0);
    const float d = r - S.spec_c[j];
    const float den = p0 + hsqrt(fmaxf(0.0f, p0 * p0 + 2.0f * sl * d));
    const float x = den > 0.0f ? 2.0f * d / den : 0.0f;
    return fminf(fmaxf(e0 + x, e0), e1);
}

// beamlet I with P(I) <= r < P(I+1); start from the guide table, walk both ways
GDPM_DEV int beamlet_of(const SourceDev& S, float u) {
    const double r = (double)u;
    int k = (int)(r * (double)S.n_guide);
    k = min(k, S.n_guide - 1);
    int i = (int)S.guide[k];
    while (i > 0 && S.cdf[i] > r) --i;
    while (i < S.nf - 1 && S.cdf[i + 1] <= r) ++i;
    return i;
}

struct Primary {
    float x, y, z, u, v, w, e;
    int beamlet;
    bool in;
};

// one step of a Metropolis chain (Algorithm A1, section 2.3.1): trial beamlet J
// with equal probability among those of nonzero intensity, then r; the chain
// moves to J when r < f_J / f_prev, tested as r f_prev < f_J in double
// precision (exact for single-precision r and f)
GDPM_DEV int metropolis_step(const SourceDev& S, float uj, float r, uint32_t& prev) {
    const uint32_t J = S.nz[min((int)((double)uj * (double)S.n_nz), S.n_nz - 1)];
    if ((double)r * (double)S.f[prev] < (double)S.f[J]) prev = J;
    return (int)prev;
}

// chain start: a beamlet drawn with equal probability among those of nonzero
// intensity, from the chain's own stream (history id (2^32-1) 2^32 + chain)
GDPM_DEV uint32_t metropolis_start(const SourceDev& S, uint32_t chain, uint32_t k0, uint32_t k1) {
    Rng r;
    rng_start(r, chain, 0xFFFFFFFFu, 0u, 0u);
    const float u = uniform(r, k0, k1);
    return S.nz[min((int)((double)u * (double)S.n_nz), S.n_nz - 1)];
}

// section 2.3.2: energy of the history at position i of a round of `size`:
// interval k with C_k <= i < C_{k+1}, C_k = floor(size F_k + 1/2); inside it
// the energy is uniform (strata_shape 0) or the spectrum's inverse CDF at
// F_k + u (F_{k+1} - F_k) (strata_shape 1)
GDPM_DEV float stratified_energy(const SourceDev& S, uint32_t i, uint32_t size, float u) {
    int k = 0;
    while (k < S.strata - 1 && floor((double)size * S.strata_F[k + 1] + 0.5) <= (double)i) ++k;
    if (S.strata_shape == 0) return fmaf(u, S.strata_w, fmaf((float)k, S.strata_w, S.strata_lo));
    const double f0 = S.strata_F[k], f1 = S.strata_F[k + 1];
    return spectrum_energy(S, (float)(f0 + (double)u * (f1 - f0)));
}

// section 2.3.3: the history whose stream is r starts as phase-space record
// h mod n: inside the phantom where it is, outside where its forward ray
// enters (else it escapes); the record number stands in for the beamlet
GDPM_DEV Primary phase_space_primary(const SourceDev& S, const Geom& G, const Rng& rg) {
    const unsigned long long h = (unsigned long long)rg.hhi << 32 | rg.hlo;
    const unsigned long long k = h % S.n_phsp;
    const float* rec = S.phsp + 7 * k;
    Primary p;
    p.beamlet = (int)k;
    p.e = rec[6];
    p.u = rec[3];
    p.v = rec[4];
    p.w = rec[5];
    const float o[3] = {rec[0], rec[1], rec[2]}, d[3] = {p.u, p.v, p.w}, L[3] = {G.lx, G.ly, G.lz};
    p.x = o[0];
    p.y = o[1];
    p.z = o[2];
    p.in = true;
    if (o[0] >= 0.0f && o[0] < G.lx && o[1] >= 0.0f && o[1] < G.ly && o[2] >= 0.0f && o[2] < G.lz) return p;
    float tmin = 0.0f, tmax = 3.0e38f;
    int ax = -1;
    bool miss = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (d[i] != 0.0f) {
            const float ta = (0.0f - o[i]) / d[i], tb = (L[i] - o[i]) / d[i];
            const float tn = fminf(ta, tb), tf = fmaxf(ta, tb);
            if (tn > tmin) {
                tmin = tn;
                ax = i;
            }
            tmax = fminf(tmax, tf);
        } else if (o[i] < 0.0f || o[i] > L[i]) {
            miss = true;
        }
    }
    p.in = !miss && tmax > tmin;
    p.x = o[0] + tmin * p.u;
    p.y = o[1] + tmin * p.v;
    p.z = o[2] + tmin * p.w;
    if (ax == 0) p.x = p.u > 0.0f ? 0.0f : G.lx;
    if (ax == 1) p.y = p.v > 0.0f ? 0.0f : G.ly;
    if (ax == 2) p.z = p.w > 0.0f ? 0.0f : G.lz;
    return p;
}

// the primary of the history whose stream is r; `chain` (Metropolis sources
// only) holds the state of the history's chain and is advanced; rpos and
// rsize (stratified spectra only) place the history in its round
GDPM_DEV Primary make_primary(const SourceDev& S, const Geom& G, Rng& r, uint32_t k0, uint32_t k1,
                              uint32_t* chain = nullptr, uint32_t rpos = 0u, uint32_t rsize = 1u) {
    if (S.n_phsp) return phase_space_primary(S, G, r);
    Primary p;
    const float ue = uniform(r, k0, k1);
    p.e = S.strata ? stratified_energy(S, rpos, rsize, ue) : spectrum_energy(S, ue);
    int gi;
    if (chain) {
        const float uj = uniform(r, k0, k1);
        gi = metropolis_step(S, uj, uniform(r, k0, k1), *chain);
    } else {
        gi = beamlet_of(S, uniform(r, k0, k1));
    }
    const float ux = uniform(r, k0, k1), uy = uniform(r, k0, k1);
    p.beamlet = gi;
    const BeamDev& b = S.beams[S.beam_of[gi]];
    const int j = gi - b.off;
    const int jx = j % b.nbx, jy = j / b.nbx;
    const float px = ((float)jx + ux) * b.bw - b.hx;
    const float py = ((float)jy + uy) * b.bh - b.hy;
    const float qx = b.iso[0] + px * b.e1[0] + py * b.e2[0];
    const float qy = b.iso[1] + px * b.e1[1] + py * b.e2[1];
    const float qz = b.iso[2] + px * b.e1[2] + py * b.e2[2];
    float ox, oy, oz, tlo;
    if (b.sad > 0.0f) {
        ox = b.iso[0] - b.sad * b.dir[0];
        oy = b.iso[1] - b.sad * b.dir[1];
        oz = b.iso[2] - b.sad * b.dir[2];
        const float dx = qx - ox, dy = qy - oy, dz = qz - oz;
        const float n = hrsq(dx * dx + dy * dy + dz * dz);
        p.u = dx * n;
        p.v = dy * n;
        p.w = dz * n;
        tlo = 0.0f;
    } else {
        ox = qx;
        oy = qy;
        oz = qz;
        p.u = b.dir[0];
        p.v = b.dir[1];
        p.w = b.dir[2];
        tlo = -3.0e38f;
    }
    // slab-method ray-box entry
    float tmin = tlo, tmax = 3.0e38f;
    int ax = -1;
    bool miss = false;
    const float o[3] = {ox, oy, oz}, d[3] = {p.u, p.v, p.w}, L[3] = {G.lx, G.ly, G.lz};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (d[i] != 0.0f) {
            const float ta = (0.0f - o[i]) / d[i], tb = (L[i] - o[i]) / d[i];
            const float tn = fminf(ta, tb), tf = fmaxf(ta, tb);
            if (tn > tmin) {
                tmin = tn;
                ax = i;
            }
            tmax = fminf(tmax, tf);
        } else if (o[i] < 0.0f || o[i] > L[i]) {
            miss = true;
        }
    }
    p.in = !miss && tmax > tmin;
    p.x = ox + tmin * p.u;
    p.y = oy + tmin * p.v;
    p.z = oz + tmin * p.w;
    if (ax == 0) p.x = p.u > 0.0f ? 0.0f : G.lx;
    if (ax == 1) p.y = p.v > 0.0f ? 0.0f : G.ly;
    if (ax == 2) p.z = p.w > 0.0f ? 0.0f : G.lz;
    return p;
}

// ---------------------------------------------------------------------------
// queue reservation and claiming (wave-uniform state)
// ---------------------------------------------------------------------------
struct PushState {
    uint32_t next, end;  // reserved, unused ring slots [next, end)
};

// Reserve `n` consecutive logical positions for this wave; item j of the wave
// lands in slot slot_of(j).  Returns false if the ring would exceed its hard
// limit (the run is then marked overflowed and the items are dropped).
struct Reservation {
    uint32_t old_next, old_avail, new_base;
    bool ok;
};

GDPM_DEV Reservation reserve(PushState& ps, RingCtl* rc, uint32_t head, uint32_t hard, uint32_t n,
                             Ctl* ctl) {
    Reservation r;
    r.old_next = ps.next;
    r.old_avail = ps.end - ps.next;
    r.new_base = 0;
    r.ok = true;
    if (n <= r.old_avail) {
        ps.next += n;
        return r;
    }
    const uint32_t leader = first_lane(ballot(true));
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&rc->tail, kPushChunk);
    base = bcast(base, leader);
    if (base + kPushChunk - head > hard) {
        if (lane_id() == leader) atomicOr(&ctl->overflow, 1u);
        r.ok = false;
        ps.next = ps.end;
        return r;
    }
    r.new_base = base;
    ps.next = base + (n - r.old_avail);
    ps.end = base + kPushChunk;
    return r;
}

GDPM_DEV uint32_t slot_of(const Reservation& r, uint32_t j) {
    return j < r.old_avail ? r.old_next + j : r.new_base + (j - r.old_avail);
}

GDPM_DEV void store(Particle* buf, uint32_t mask, uint32_t slot, const Particle& p) {
    float4* d = reinterpret_cast<float4*>(buf + (slot & mask));
    const float4* s = reinterpret_cast<const float4*>(&p);
    d[0] = s[0];
    d[1] = s[1];
    d[2] = s[2];
    d[3] = s[3];
}

GDPM_DEV Particle load(const Particle* buf, uint32_t mask, uint32_t slot) {
    Particle p;
    const float4* s = reinterpret_cast<const float4*>(buf + (slot & mask));
    float4* d = reinterpret_cast<float4*>(&p);
    d[0] = s[0];
    d[1] = s[1];
    d[2] = s[2];
    d[3] = s[3];
    return p;
}

// mark the unused tail of this wave's reservation as empty slots
GDPM_DEV void release(PushState& ps, Particle* buf, uint32_t mask) {
    // by offset from ps.next: queue positions run modulo 2^32, and a reserved
    // run may straddle the wrap (then ps.end < ps.next as numbers)
    const uint32_t n = ps.end - ps.next;
    for (uint32_t o = lane_id(); o < n; o += 64u)
        reinterpret_cast<float*>(buf + ((ps.next + o) & mask))[3] = kEmptyEnergy;
    ps.next = ps.end;
}

// Counters kept per wavefront (scalar registers): updated only where the
// wavefront is converged, from ballots of the lanes concerned.
struct WaveTally {
    uint32_t events;      // flights (photon pass) or steps (electron pass)
    uint32_t pushes;      // secondaries written, all jobs
    uint32_t ld, rq;      // records loaded from the queue, records handed on
    uint32_t born, died;  // records created and particles ended, current job
    uint32_t bad;         // particles ended by the iteration bound of a wavefront
    uint32_t it[2];       // real interactions by type (photons: photoelectric,
                          // pair; electrons: Moller); Compton and bremsstrahlung
                          // are the rest of the real interactions and hard events
};

// Hand particles to the next pass of the same type (the record keeps the whole
// state, random stream position included, so nothing physical changes).
// Returns true in the lanes that wrote a record.
GDPM_DEV bool requeue(bool active, PushState& ps, uint32_t head, Ctl* ctl, RingCtl* rc, uint32_t hard,
                      Particle* buf, uint32_t mask, const Particle& p, WaveTally& c) {
    const uint64_t b = ballot(active);
    const uint32_t n = (uint32_t)__popcll(b);
    if (n == 0) return false;
    const Reservation res = reserve(ps, rc, head, hard, n, ctl);
    if (res.ok) c.rq += n;
    if (!res.ok || !active) return false;
    store(buf, mask, slot_of(res, mbcnt(b)), p);
    return true;
}

// ---------------------------------------------------------------------------
// the job a wavefront works on: loaded when the wavefront switches jobs and
// held in scalar registers (a wavefront only ever holds one job's particles)
// ---------------------------------------------------------------------------
struct WJob {
    Geom G;
    const float* mumax;
    double* tally;
    unsigned long long nv;
    double* hist;
    unsigned long long hist0;
    uint32_t k0, k1, flags;
    int j;
    int ri;                          // the particle type of the pass the wavefront works in
    uint32_t tag;                    // slot | generation << 8: low half of the records' job word
    uint32_t seg_begin, seg_count;   // the job's records in the running pass
};

template <class T>
GDPM_DEV T uniform_copy(const T& v) {
    static_assert(sizeof(T) % 4 == 0, "word-sized fields");
    T out;
    const uint32_t* a = reinterpret_cast<const uint32_t*>(&v);
    uint32_t* b = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) b[i] = __builtin_amdgcn_readfirstlane(a[i]);
    return out;
}

GDPM_DEV void load_job(WJob& w, const RunDev& R, int j, int ri) {
    j = __builtin_amdgcn_readfirstlane(j);
    const JobDev& d = R.jobs[j];
    w.G = uniform_copy(d.G);
    w.mumax = uniform_copy(d.mumax);
    w.tally = uniform_copy(d.tally);
    w.nv = uniform_copy(d.nv);
    w.hist = uniform_copy(d.hist);
    w.hist0 = uniform_copy(d.hist0);
    w.k0 = __builtin_amdgcn_readfirstlane(d.k0);
    w.k1 = __builtin_amdgcn_readfirstlane(d.k1);
    w.flags = __builtin_amdgcn_readfirstlane(d.flags);
    w.j = j;
    w.ri = ri;
    w.tag = (uint32_t)j | ((__builtin_amdgcn_readfirstlane(d.gen) & 0xFFu) << 8);
    w.seg_begin = __builtin_amdgcn_readfirstlane(R.jc->seg_begin[ri][j]);
    w.seg_count = __builtin_amdgcn_readfirstlane(R.jc->seg_count[ri][j]);
}

// first job of a wavefront: the pass input is split over the wavefronts of the
// grid in proportion to the jobs' record counts; -1 if the pass is empty
GDPM_DEV int first_job(const RunDev& R, uint32_t total, int ri) {
    if (total == 0) return -1;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t pos = (uint32_t)(((unsigned long long)w * total + total / 2) / waves);
    int lo = 0, hi = R.n_jobs - 1;   // last job whose segment starts at or before pos
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (__builtin_amdgcn_readfirstlane(R.jc->seg_begin[ri][mid]) <= pos) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

GDPM_DEV unsigned long long load_agent64(const unsigned long long* p) {
    const unsigned long long v = __hip_atomic_load(const_cast<unsigned long long*>(p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (unsigned long long)hi << 32 | lo;
}

// the next job after j (cyclically) with unclaimed records in this pass, or -1
GDPM_DEV int next_job(const JobCtl* jc, int j, int n_jobs, int ri) {
    if (n_jobs <= 1) return -1;
    const int nw = (n_jobs + 63) >> 6;
    for (int k = 0; k <= nw; ++k) {
        const int wi = ((j >> 6) + k) % nw;
        unsigned long long m = load_agent64(&jc->left[ri][wi]);
        if (k == 0) {
            const int b = j & 63;   // only jobs after j in j's own word
            m = b == 63 ? 0ull : m & (~0ull << (b + 1));
        } else if (k == nw) {
            m &= (1ull << (j & 63)) - 1ull;   // jobs before j in j's word, last
        }
        if (m) {
            const int c = wi * 64 + (__ffsll(m) - 1);
            if (c < n_jobs && c != j) return c;
        }
    }
    return -1;
}

// the job's majorant table: a copy in this wavefront's LDS slice `lmw`, or the
// global array when there is no slice
GDPM_DEV const float* job_majorant(const WJob& W, float* lmw, int n) {
    if (lmw == nullptr) return W.mumax;
    for (int i = (int)lane_id(); i < n; i += 64) lmw[i] = W.mumax[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return lmw;
}

struct ClaimState {
    uint32_t next, end;  // claimed positions of the job's segment not yet handed out
    uint32_t seen;       // the job's claim counter as this wave last saw it
    bool done;           // the job's segment has nothing left to claim
    uint32_t st_lo, st_hi;  // positions whose records are staged in the wave's LDS slice
};

// ---------------------------------------------------------------------------
// per-lane tallies
// ---------------------------------------------------------------------------
struct LaneTally {
    int dv;          // voxel of the pending deposit (-1 none)
    double de;       // pending deposit (MeV)
    double e_esc;    // escaped energy of the current job
    double h_dep, h_esc;  // per-history accumulators (test mode)
    uint32_t ev[7];
};


// deposits go to the batch slot `pb` of the particle's history; a split job's
// particles are tallied at weight 1 and the host scales the sums by 2^-split
// (exact: a power of two commutes with every rounding of the sum)
GDPM_DEV void tally_flush(LaneTally& t, const WJob& W, uint32_t pb) {
    if (t.dv >= 0 && t.de != 0.0) {
        unsafeAtomicAdd(&W.tally[(unsigned long long)pb * W.nv + (unsigned)t.dv], t.de);
        t.ev[EV_DEPOSITS]++;
    }
    t.dv = -1;
    t.de = 0.0;
}

GDPM_DEV void deposit(LaneTally& t, const WJob& W, uint32_t pb, int v, float e) {
    if (v != t.dv) tally_flush(t, W, pb);
    t.dv = v;
    t.de += (double)e;
    t.h_dep += (double)e;
}

GDPM_DEV void history_flush(LaneTally& t, const WJob& W, uint32_t hlo, uint32_t hhi) {
    if (W.hist) {
        const unsigned long long h = ((unsigned long long)hhi << 32 | hlo) - W.hist0;
        if (t.h_dep != 0.0) unsafeAtomicAdd(&W.hist[2 * h], t.h_dep);
        if (t.h_esc != 0.0) unsafeAtomicAdd(&W.hist[2 * h + 1], t.h_esc);
    }
    t.h_dep = 0.0;
    t.h_esc = 0.0;
}

GDPM_DEV void tally_init(LaneTally& t) {
    t.dv = -1;
    t.de = 0.0;
    t.e_esc = t.h_dep = t.h_esc = 0.0;
#pragma unroll
    for (int i = 0; i < 7; ++i) t.ev[i] = 0u;
}

// fold the per-job counters into the job's (before a switch, at the end)
GDPM_DEV void job_flush(LaneTally& t, WaveTally& c, const WJob& W, JobCtl* jc) {
    const double esc = wave_sum(t.e_esc);
    if (lane_id() == 0) {
        if (esc != 0.0) unsafeAtomicAdd(&jc->e_esc[W.j], esc);
        if (c.born) atomicAdd(&jc->births[W.j], (unsigned long long)c.born);
        if (c.died) atomicAdd(&jc->deaths[W.j], (unsigned long long)c.died);
    }
    t.e_esc = 0.0;
    c.pushes += c.born;
    c.born = c.died = 0u;
}

// fold the pass counters into the run's; `ri` is the pass's particle type
GDPM_DEV void pass_finish(LaneTally& t, const WaveTally& c, Ctl* ctl, int ri) {
    uint32_t ev[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) ev[i] = wave_sum(t.ev[i]);
    ev[ri == 0 ? EV_FLIGHTS : EV_ESTEPS] += c.events;
    ev[EV_PUSHES] += c.pushes;
    if (lane_id() == 0) {
        if (c.bad) atomicAdd(&ctl->anomalies, (unsigned long long)c.bad);
#pragma unroll
        for (int i = 0; i < 7; ++i)
            if (ev[i]) atomicAdd(&ctl->ev[i], (unsigned long long)ev[i]);
        atomicAdd(&ctl->pass_ev[ri][0], (unsigned long long)c.ld);
        atomicAdd(&ctl->pass_ev[ri][1], (unsigned long long)(c.pushes + c.rq));
        atomicAdd(&ctl->pass_ev[ri][2], (unsigned long long)ev[EV_DEPOSITS]);
        if (c.rq) atomicAdd(&ctl->pass_ev[ri][3], (unsigned long long)c.rq);
        if (ri == 0) {
            if (c.it[0]) atomicAdd(&ctl->itype[1], (unsigned long long)c.it[0]);
            if (c.it[1]) atomicAdd(&ctl->itype[2], (unsigned long long)c.it[1]);
        } else if (c.it[0]) {
            atomicAdd(&ctl->itype[3], (unsigned long long)c.it[0]);
        }
    }
}

// ---------------------------------------------------------------------------
// samplers (the draw order is part of the contract with the reference)
// ---------------------------------------------------------------------------

// Klein-Nishina: eps = E'/E where the distribution function reaches one
// uniform draw u, from the tabulated inverse (bilinear in log2 E and u, of
// q = ln(eps/eps0)/ln(1/eps0), so that eps = eps0^(1 - q)); then
// t = 1 - cos(theta) and the azimuth (in turns).  No rejection: every lane
// of a wavefront runs the same instructions.
GDPM_DEV void sample_compton(const Tables& T, Rng& r, uint32_t k0, uint32_t k1, float e, float& eps,
                             float& t, float& turns) {
    const float k = e * (1.0f / kMec2f);
    const float u = uniform(r, k0, k1);
    float fe = (hlog2(e) - T.kn_lo) * T.kn_inv;
    fe = fminf(fmaxf(fe, 0.0f), (float)(T.kn_ne - 1));
    const int i = min((int)fe, T.kn_ne - 2);
    const float a = fe - (float)i;
    const float fu = u * (float)(T.kn_nu - 1);
    const int j = min((int)fu, T.kn_nu - 2);
    const float b = fu - (float)j;
    const float* p = T.kn + (i * T.kn_nu + j);
    const float q0 = fmaf(b, p[1] - p[0], p[0]);
    const float q1 = fmaf(b, p[T.kn_nu + 1] - p[T.kn_nu], p[T.kn_nu]);
    const float q = fmaf(a, q1 - q0, q0);
    eps = fminf(hexp2(-hlog2(1.0f + 2.0f * k) * (1.0f - q)), 1.0f);
    t = (1.0f - eps) * hrcp(k) * hrcp(eps);
    turns = uniform(r, k0, k1);
}

// Moller: eps = W/T by a 1/eps^2 proposal on [W_cc/T, 1/2] and rejection
// eps^2 B(eps) / 2.25; then the azimuth
GDPM_DEV void sample_moller(Rng& r, uint32_t k0, uint32_t k1, float tt, float wcc, float& eps,
                            float& turns) {
    const float g = 1.0f + tt * (1.0f / kMec2f), e0 = fdiv(wcc, tt);
    const float ig = hrcp(g);
    const float c1 = (g - 1.0f) * ig, c2 = (2.0f * g - 1.0f) * ig * ig;
    for (;;) {
        const float ua = uniform(r, k0, k1);
        eps = fdiv(e0, 1.0f - ua * (1.0f - 2.0f * e0));
        const float ub = uniform(r, k0, k1);
        const float ie = hrcp(eps), io = hrcp(1.0f - eps);
        const float br = c1 * c1 + ie * (ie - c2) + io * (io - c2);
        if (ub * 2.25f <= eps * eps * br) break;
    }
    turns = uniform(r, k0, k1);
}

// bremsstrahlung photon energy: 1/k proposal on [W_cb, T], rejection by the
// complete-screening spectrum
GDPM_DEV float sample_brems(Rng& r, uint32_t k0, uint32_t k1, float tt, float wcb) {
    const float lr = hlog2(tt) - hlog2(wcb);
    const float it = hrcp(tt);
    float kph;
    for (;;) {
        const float ua = uniform(r, k0, k1);
        // the hardware log2 and exp2 are within about an ulp each, so near
        // ua = 1 their product could exceed T by a few ulps and leave the
        // electron a negative energy: the photon takes at most T
        kph = fminf(wcb * hexp2(ua * lr), tt);
        const float ub = uniform(r, k0, k1);
        const float yy = kph * it;
        if (ub * (4.0f / 3.0f) <= 4.0f / 3.0f - 4.0f / 3.0f * yy + yy * yy) break;
    }
    return kph;
}

// isotropic direction of the first annihilation photon (cos, then azimuth)
GDPM_DEV void sample_iso(Rng& r, uint32_t k0, uint32_t k1, float& du, float& dv, float& dw) {
    const float ct = 2.0f * uniform(r, k0, k1) - 1.0f;
    const float turns = uniform(r, k0, k1);
    const float st = hsqrt((1.0f - ct) * (1.0f + ct));
    du = st * cos_turns(turns);
    dv = st * sin_turns(turns);
    dw = ct;
}

// Compton electron: along the momentum transfer E d0 - E' d of a photon
// turned from d0 to d with E -> E' (no binding: momentum conservation)
GDPM_DEV void compton_electron_dir(float e, float e1, float u0, float v0, float w0, float u, float v,
                                   float w, float& eu, float& ev, float& ew) {
    eu = e * u0 - e1 * u;
    ev = e * v0 - e1 * v;
    ew = e * w0 - e1 * w;
    const float nn = eu * eu + ev * ev + ew * ew;
    if (nn > 0.0f) {
        const float in = hrsq(nn);
        eu *= in; ev *= in; ew *= in;
    } else {
        eu = u0; ev = v0; ew = w0;
    }
}

// pair production: K = E - 2 mc^2 split at the uniform u (T- = u K), the
// larger part computed and the smaller taken as K minus it, so that
// T- + T+ = K exactly; the positron keeps a = E - K
GDPM_DEV void pair_split(float e, float u, float& tm, float& tp, float& aa) {
    const float kk = e - kTwoMec2f;
    aa = e - kk;
    const float tc = u * kk;
    if (2.0f * tc >= kk) {
        tm = tc;
        tp = kk - tc;
    } else {
        tp = kk - tc;
        tm = kk - tp;
    }
}

// ---------------------------------------------------------------------------
// secondaries of one event, pushed once per iteration with the wave converged
// ---------------------------------------------------------------------------
// charged: up to two; the second (a positron) shares the first one's direction
struct PendCharged {
    int n;
    float e0, du, dv, dw;   // first particle and the common direction
    float a0;               // first particle: annihilation energy if it is a positron
    uint32_t role, flag0;   // first particle: role word, positron flag
    float e1, a1;           // second particle (always the pair positron, role 1)
};
// photons: one (role word wb) or two back to back (roles wb, wb + 1)
struct PendPhoton {
    int n;
    float e, u, v, w;
    uint32_t wb;
};

GDPM_DEV void write_particle(Particle* buf, uint32_t mask, uint32_t slot, float x, float y, float z,
                             float e, float u, float v, float w, uint32_t hlo, uint32_t hhi,
                             uint32_t path, uint32_t vox, float a, uint32_t flags, uint32_t job) {
    float4* d = reinterpret_cast<float4*>(buf + (slot & mask));
    d[0] = make_float4(x, y, z, e);
    d[1] = make_float4(u, v, w, -1.0f);
    d[2] = make_float4(__uint_as_float(hlo), __uint_as_float(hhi), __uint_as_float(path), 0.0f);
    d[3] = make_float4(__uint_as_float(vox), a, __uint_as_float(flags), __uint_as_float(job));
}

// secondaries inherit the job and the batch slot (`jb`) of their history
GDPM_DEV void push_charged(PendCharged& q, PushState& ps, uint32_t head, Ctl* ctl, const RunDev& R,
                           const WJob& W, uint32_t jb, Particle* buf, float x, float y, float z,
                           uint32_t vox, const Rng& rng, WaveTally& c) {
    const uint64_t b0 = ballot(q.n >= 1), b1 = ballot(q.n >= 2);
    const uint32_t n0 = (uint32_t)__popcll(b0), n = n0 + (uint32_t)__popcll(b1);
    if (n == 0) return;
    const Reservation res = reserve(ps, &ctl->ring[1], head, R.hard[1], n, ctl);
    if (res.ok && q.n > 0) {
        write_particle(buf, R.mask[1], slot_of(res, mbcnt(b0)), x, y, z, q.e0, q.du, q.dv, q.dw,
                       rng.hlo, rng.hhi, spawn_path(rng, W.k0, W.k1, (int)q.role), vox, q.a0,
                       q.flag0, jb);
        if (q.n > 1)
            write_particle(buf, R.mask[1], slot_of(res, n0 + mbcnt(b1)), x, y, z, q.e1, q.du, q.dv,
                           q.dw, rng.hlo, rng.hhi, spawn_path(rng, W.k0, W.k1, 1), vox, q.a1, 1u, jb);
    }
    if (res.ok) c.born += n;
    q.n = 0;
}

GDPM_DEV void push_photons(PendPhoton& q, PushState& ps, uint32_t head, Ctl* ctl, const RunDev& R,
                           const WJob& W, uint32_t jb, Particle* buf, float x, float y, float z,
                           const Rng& rng, WaveTally& c) {
    const uint64_t b0 = ballot(q.n >= 1), b1 = ballot(q.n >= 2);
    const uint32_t n0 = (uint32_t)__popcll(b0), n = n0 + (uint32_t)__popcll(b1);
    if (n == 0) return;
    const Reservation res = reserve(ps, &ctl->ring[0], head, R.hard[0], n, ctl);
    if (res.ok && q.n > 0) {
        write_particle(buf, R.mask[0], slot_of(res, mbcnt(b0)), x, y, z, q.e, q.u, q.v, q.w,
                       rng.hlo, rng.hhi, spawn_path(rng, W.k0, W.k1, (int)q.wb), 0u, 0.0f, 0u, jb);
        if (q.n > 1)
            write_particle(buf, R.mask[0], slot_of(res, n0 + mbcnt(b1)), x, y, z, q.e, -q.u, -q.v,
                           -q.w, rng.hlo, rng.hhi, spawn_path(rng, W.k0, W.k1, (int)q.wb + 1), 0u,
                           0.0f, 0u, jb);
    }
    if (res.ok) c.born += n;
    q.n = 0;
}

// ---------------------------------------------------------------------------
// pass set-up and completion (one block, between passes): the job segments
// come from the re-binning that precedes every pass
// ---------------------------------------------------------------------------
// rebinned = 0: the queue was not re-binned because only job `lone` holds
// particles: the whole queue, empty slots included, is that job's segment and
// the other jobs' segments are empty (they start at its end, so that a
// wavefront's first job is `lone`)
__global__ void __launch_bounds__(256) k_setup(Ctl* ctl, RunDev R, int ri, int rebinned, int lone) {
    JobCtl* jc = R.jc;
    RingCtl& r = ctl->ring[ri];
    // a permuted pass reads positions [0, n_valid) of the permutation; its
    // records stay in [head, tail), which it consumes whole
    const bool perm = rebinned && r.permuted;
    const uint32_t count = ctl->overflow ? 0u : (perm ? ctl->n_valid : r.tail - r.head);
    if (!rebinned)
        for (int j = threadIdx.x; j < R.n_jobs; j += blockDim.x) {
            jc->seg_begin[ri][j] = j <= lone ? 0u : count;
            jc->seg_count[ri][j] = j == lone ? count : 0u;
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        r.begin = perm ? 0u : r.head;
        r.count = count;
        r.claim = 0u;
        r.next_head = r.tail;
        if (!perm) r.permuted = 0u;
    }
    for (int j = threadIdx.x; j < R.n_jobs; j += blockDim.x) jc->claim[ri][j] = 0u;
    const int nw = (R.n_jobs + 63) >> 6;
    for (int k = threadIdx.x; k < kMaxJobs / 64; k += blockDim.x) {
        unsigned long long m = 0ull;
        if (k < nw && !ctl->overflow)
            for (int b = 0; b < 64 && k * 64 + b < R.n_jobs; ++b)
                if (jc->seg_count[ri][k * 64 + b] > 0u) m |= 1ull << b;
        jc->left[ri][k] = m;
    }
}

__global__ void k_finish(Ctl* ctl, int ri) {
    RingCtl& r = ctl->ring[ri];
    r.head = r.permuted ? r.next_head : r.begin + r.count;
    r.count = 0u;
    r.permuted = 0u;
}

// ---------------------------------------------------------------------------
// claiming input: positions [0, seg_count) of the job's segment
// ---------------------------------------------------------------------------
GDPM_DEV void claim_refill(ClaimState& cs, JobCtl* jc, const WJob& W, const Ctl* ctl) {
    if (cs.done || cs.next != cs.end) return;
    // the wave has used up its items: claim a new chunk if the job has more.
    // Chunks shrink as the segment drains (guided self-scheduling), so that the
    // last items spread over many wavefronts.  The shared counters are touched
    // once per claim, never per iteration.
    const uint32_t count = W.seg_count;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    const uint32_t left = count - min(cs.seen, count);
    const uint32_t chunk = min(max(left / (2u * waves), kClaimMin), W.ri == 0 ? kClaimMaxPhoton : kClaimMaxElectron);
    if (load_agent(&ctl->overflow)) {   // a queue overflowed: the run is void
        cs.done = true;
        return;
    }
    const uint32_t leader = first_lane(ballot(true));
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&jc->claim[W.ri][W.j], chunk);
    base = bcast(base, leader);
    cs.seen = base + chunk;
    if (base >= count) {
        if (lane_id() == leader) atomicAnd(&jc->left[W.ri][W.j >> 6], ~(1ull << (W.j & 63)));
        cs.done = true;
        return;
    }
    cs.next = base;
    cs.end = min(base + chunk, count);
}

// Records of the wave's claimed chunk are staged in its LDS slice (kStage
// records, 64 bytes each) by direct-to-LDS loads issued right after a refill,
// so the next refills read them from LDS instead of waiting for memory.
constexpr uint32_t kStage = 64;
constexpr uint32_t kStageLow = 24;   // restage when fewer staged records are left

GDPM_DEV Particle load_staged(const float4* st, uint32_t k) {
    Particle p;
    float4* d = reinterpret_cast<float4*>(&p);
    d[0] = st[4 * k];
    d[1] = st[4 * k + 1];
    d[2] = st[4 * k + 2];
    d[3] = st[4 * k + 3];
    return p;
}

// the queue position of input position `pos` of a pass: itself, or through the
// permutation of a pass re-binned by job (`perm` non-null); both masked, so
// that any value reads inside the queue
GDPM_DEV uint32_t input_slot(const uint32_t* perm, uint32_t mask, uint32_t pos) {
    return (perm ? perm[pos & mask] : pos) & mask;
}

// stage the records of positions [cs.next, cs.next + kStage) (every lane: 4
// loads of 16 bytes; lane L of load c fetches piece L % 4 of record 16 c + L / 4,
// which lands at float4 64 c + L of the slice).  Positions past the chunk are
// loaded too (the ring index is masked) and never used.
GDPM_DEV void stage_records(ClaimState& cs, float4* st, const Particle* buf, uint32_t mask,
                            uint32_t first, const uint32_t* perm) {
    // the refill's reads of the slice are complete before it is overwritten
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
    const uint32_t l = lane_id();
    for (uint32_t c = 0; c < 4; ++c) {
        const uint32_t rec = 16u * c + (l >> 2);
        const float4* src = reinterpret_cast<const float4*>(buf + input_slot(perm, mask, first + cs.next + rec)) +
                            (l & 3u);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(st + 64u * c), 16, 0, 0);
    }
    cs.st_lo = cs.next;
    cs.st_hi = cs.next + kStage;
}

// refill the lanes without a particle from the wave's claimed items; returns
// true in the lanes that loaded a record.  Lanes wait until kRefillMin of them
// are empty (or no lane is busy): a refill stalls the wavefront on record
// loads, so it pays to do it for several lanes at once.  With a staging slice
// (`st`, LDS) the records come from it when they are staged.  kSolo (a
// measurement form): one particle per wavefront at a time, so the wavefront
// executes exactly the instructions of that particle's path.
template <bool kSolo>
GDPM_DEV bool refill(bool active, ClaimState& cs, JobCtl* jc, const WJob& W, uint32_t begin,
                     Ctl* ctl, const Particle* buf, uint32_t mask, const uint32_t* perm, Particle& p,
                     WaveTally& c, float4* st) {
    if (cs.done) return false;
    const uint64_t need = ballot(!active);
    if (!need) return false;
    if constexpr (kSolo) {
        if (ballot(active)) return false;
    } else {
        if ((uint32_t)__popcll(need) < kRefillMin && ballot(active)) return false;
    }
    claim_refill(cs, jc, W, ctl);
    const uint32_t have = cs.end - cs.next;
    const uint32_t rank = mbcnt(need);
    const uint32_t take = kSolo ? min(have, 1u) : min(have, (uint32_t)__popcll(need));
    const uint32_t first = begin + W.seg_begin;
    const bool staged = st != nullptr && take > 0u && cs.next >= cs.st_lo &&
                        cs.next + take <= cs.st_hi;
    if (staged) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the staging loads have landed
    bool got = false;
    if (!active && rank < take) {
        p = staged ? load_staged(st, cs.next + rank - cs.st_lo)
                   : load(buf, mask, input_slot(perm, mask, first + cs.next + rank));
        got = !record_empty(p.e);
        if (got && (p.job & 0xFFFFu) != W.tag) {
            // a record of another job (or of an earlier job in this slot) in
            // this job's segment: only a broken bookkeeping puts it there; it
            // is dropped and counted
            atomicAdd(&ctl->anomalies, 1ull);
            got = false;
        }
    }
    cs.next += take;
    c.ld += take;
    if (st != nullptr && cs.next < cs.end) {
        // positions of a pass's segment do not wrap: plain comparisons
        const uint32_t left = cs.next >= cs.st_lo && cs.next < cs.st_hi ? cs.st_hi - cs.next : 0u;
        if (left <= kStageLow) stage_records(cs, st, buf, mask, first, perm);
    }
    return got;
}

// ---------------------------------------------------------------------------
// source pass: segments of new histories (job, first id, count, batch slot) ->
// primaries appended to the queue of the source particle type (section 2.3);
// a primary whose ray misses the phantom leaves an empty slot and counts as
// escaped
// ---------------------------------------------------------------------------
GDPM_DEV double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane_id() == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += sh[i];
    return s;
}

__global__ void __launch_bounds__(256) k_source(Ctl* ctl, RunDev R, const SrcSeg* segs,
                                                const SrcHdr* hdr, int ri) {
    __shared__ double sh[4];
    if (ctl->overflow) return;
    const int nseg = (int)__builtin_amdgcn_readfirstlane(hdr->nseg);
    const uint32_t total = __builtin_amdgcn_readfirstlane(hdr->total);
    const RingCtl& r = ctl->ring[ri];
    const uint32_t tail = r.tail;
    if (tail + total - r.head > R.hard[ri]) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctl->overflow, 1u);
        return;
    }
    Particle* buf = R.buf[ri];
    const uint32_t nthreads = gridDim.x * blockDim.x;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int s = 0; s < nseg; ++s) {
        const SrcSeg sg = uniform_copy(segs[s]);
        const JobDev& d = R.jobs[sg.job];
        const Geom G = uniform_copy(d.G);
        const SourceDev S = uniform_copy(d.S);
        const uint32_t k0 = __builtin_amdgcn_readfirstlane(d.k0);
        const uint32_t k1 = __builtin_amdgcn_readfirstlane(d.k1);
        double* hist = uniform_copy(d.hist);
        const unsigned long long hist0 = uniform_copy(d.hist0);
        const uint32_t jb = sg.job | ((__builtin_amdgcn_readfirstlane(d.gen) & 0xFFu) << 8) | (sg.batch << 16);
        const uint32_t copies = 1u << __builtin_amdgcn_readfirstlane(d.split);
        double e_in = 0.0, e_esc = 0.0, born = 0.0;
        // history sg.h0 + i; `chain` holds its Metropolis chain (or is null).
        // A split history writes its 2^split copies to consecutive records,
        // copy c on stream path c (copy 0 is the unsplit primary).
        auto one = [&](uint32_t i, uint32_t* chain) {
            const unsigned long long h = sg.h0 + i;
            Rng rng;
            rng_start(rng, (uint32_t)h, (uint32_t)(h >> 32), 0u, 0u);
            rng_topup(rng, k0, k1);
            const Primary pr = make_primary(S, G, rng, k0, k1, chain, sg.rpos + i, sg.rsize);
            e_in += (double)pr.e;
            uint32_t vox = 0u;
            if (pr.in && ri == 1) {
                int ix, iy, iz;
                voxel_of(G, pr.x, pr.y, pr.z, ix, iy, iz);
                vox = pack_vox(ix, iy, iz);
            }
            for (uint32_t c = 0; c < copies; ++c) {
                float4* q = reinterpret_cast<float4*>(buf + ((tail + sg.off + i * copies + c) & R.mask[ri]));
                if (pr.in) {
                    // the stream continues at the draw after the source's draws
                    q[0] = make_float4(pr.x, pr.y, pr.z, pr.e);
                    q[1] = make_float4(pr.u, pr.v, pr.w, -1.0f);
                    q[2] = make_float4(__uint_as_float(rng.hlo), __uint_as_float(rng.hhi), __uint_as_float(c),
                                       __uint_as_float(rng_ctr(rng)));
                    q[3] = make_float4(__uint_as_float(vox), 0.0f, 0.0f, __uint_as_float(jb));
                } else {
                    reinterpret_cast<float*>(q)[3] = kEmptyEnergy;
                }
            }
            if (pr.in) {
                born += (double)copies;
            } else {
                // all copies escape: weight 1 each, like the tallies
                const double out = (double)pr.e * (double)copies;
                e_esc += out;
                if (hist) unsafeAtomicAdd(&hist[2 * (h - hist0) + 1], out);
            }
        };
        if (S.metro) {
            // a chain's histories in increasing order, by one thread (a chain
            // runs across segments and iterations through its stored state)
            uint32_t* chains = uniform_copy(d.chains);
            for (uint32_t c = tid; c < kMetroChains; c += nthreads) {
                uint32_t state = chains[c];
                const uint32_t first = (uint32_t)((c + kMetroChains - sg.h0 % kMetroChains) % kMetroChains);
                for (uint32_t i = first; i < sg.n; i += kMetroChains) one(i, &state);
                chains[c] = state;
            }
        } else {
            for (uint32_t i = tid; i < sg.n; i += nthreads) one(i, nullptr);
        }
        e_in = block_sum(e_in, sh);
        e_esc = block_sum(e_esc, sh);
        born = block_sum(born, sh);
        if (threadIdx.x == 0) {
            if (e_in != 0.0) unsafeAtomicAdd(&R.jc->e_in[sg.job], e_in);
            if (e_esc != 0.0) unsafeAtomicAdd(&R.jc->e_esc[sg.job], e_esc);
            if (born != 0.0) atomicAdd(&R.jc->births[sg.job], (unsigned long long)born);
        }
    }
}

// make the records written by the source pass part of the queue
__global__ void k_commit(Ctl* ctl, int ri, const SrcHdr* hdr) {
    if (ctl->overflow) return;
    ctl->ring[ri].tail += hdr->total;
}

// ---------------------------------------------------------------------------
// photon pass: Woodcock tracking (section 2.1), one flight per iteration
// ---------------------------------------------------------------------------
// Interpolation tables are staged in LDS (kLds) when they fit; one workgroup
// per CU shares them, and each wavefront keeps its job's majorant in its own
// LDS slice.
extern __shared__ float4 lds_tables[];

// LDS layout of a transport workgroup (float4 units): the tables (photons: the
// cross sections, then one majorant slice of pg_n floats per wavefront;
// electrons: the stopping and scattering data, the inverse range and its
// scales), then one slice of kStage staged records per wavefront
GDPM_HD uint32_t stage_offset(int ri, const Tables& T, int waves) {
    const uint32_t floats = ri == 0 ? (uint32_t)(waves * T.pg_n)
                                    : (uint32_t)(T.n_mat * T.nr + T.n_mat);
    const uint32_t tab = ri == 0 ? (uint32_t)(T.n_mat * T.pg_n) : (uint32_t)(T.n_mat * T.eg_n);
    return tab + (floats + 3u) / 4u;
}

// One wavefront's share of a photon pass.  ptab: the cross sections (LDS or
// global); lmw: the wavefront's LDS slice for its job's majorant (null: the
// global array); stage: its LDS slice for staged records (null: none).
template <bool kSolo, bool kPerm>
GDPM_DEV void photon_pass(Ctl* ctl, const Tables& T, const RunDev& R, const float4* ptab, float* lmw,
                          float4* stage) {
    RingCtl* rc = &ctl->ring[0];
    const uint32_t begin = rc->begin, count = rc->count;
    // a re-binned pass reads its input through the permutation (only the kPerm
    // form has that code: the passes of a lone job keep the plain reads)
    const uint32_t* perm_in =
        kPerm && __builtin_amdgcn_readfirstlane(rc->permuted) ? bin_perm(R.bin[0], R.mask[0]) : nullptr;
    const bool big = !kSolo && count >= kTailMinPerLane * gridDim.x * blockDim.x;
    Particle* bufg = R.buf[0];
    Particle* bufe = R.buf[1];
    const uint32_t head_g = ctl->ring[0].head, head_e = ctl->ring[1].head;
    JobCtl* jc = R.jc;
    const float ecut_e = R.ecut_e, ecut_g = R.ecut_g;

    int j = first_job(R, count, 0);
    PushState pg{0u, 0u}, pe{0u, 0u};
    LaneTally tl;
    tally_init(tl);
    WaveTally wt{0u, 0u, 0u, 0u, 0u, 0u, 0u, {0u, 0u}};
    uint32_t iters = 0u;
    bool last_job = false;   // no other job has records left in this pass
    // one job at a time: a wavefront switches jobs with all its lanes empty
    while (j >= 0) {
        WJob W;
        load_job(W, R, j, 0);
        const float* mtab = job_majorant(W, lmw, T.pg_n);
        ClaimState cs{0u, 0u, 0u, false, 0u, 0u};
        bool active = false;
        float x = 0, y = 0, z = 0, u = 0, v = 0, w = 0, e = 0;
        uint32_t pb = 0u;   // batch slot of the lane's history
        int pm = -1;        // >= 0: a real interaction waits, in a voxel of this material
        Rng rng;
        rng_start(rng, 0u, 0u, 0u, 0u);
        int next = -1;
        for (;;) {
            const uint32_t k0 = W.k0, k1 = W.k1;
            const bool kerma = (W.flags & 64u) != 0u;
            Particle p;
            if (refill<kSolo>(active, cs, jc, W, begin, ctl, bufg, R.mask[0], perm_in, p, wt, stage)) {
                x = p.x; y = p.y; z = p.z; e = p.e;
                u = p.u; v = p.v; w = p.w;
                pb = p.job >> 16;
                rng_start(rng, p.hlo, p.hhi, p.path, p.ctr);
                active = true;
            }
            if (!ballot(active)) {
                if (cs.done && last_job) break;
                if (!cs.done) continue;
            } else {
            rng_topup(rng, k0, k1);
            const uint64_t act0 = ballot(active);

            PendCharged qe;
            PendPhoton qg;
            qe.n = 0;
            qg.n = 0;
            int ix = 0, iy = 0, iz = 0;
            if (active && !(e <= kMaxEnergy)) {
                // a non-finite energy can only come from a damaged record: end the
                // particle (counted as an anomaly) rather than feed it to a
                // rejection sampler that would never accept
                atomicAdd(&ctl->anomalies, 1ull);
                active = false;
                pm = -1;
            }
            // energy grid cell of the flight and of a waiting interaction (the
            // energy is unchanged in between); computed on every lane, since the
            // grid clamps any energy, 0 and non-finite ones included, into the table
            int gi;
            float gt;
            grid(hlog2(e), T.pg_lo, T.pg_inv, T.pg_n, gi, gt);
            const float mumax = lerp1(mtab, gi, gt);
            wt.events += (uint32_t)__popcll(ballot(active && pm < 0 && !(e < ecut_g)));
            if (active && pm < 0) {
                if (e < ecut_g) {
                    const int vv = voxel_of(W.G, x, y, z, ix, iy, iz);
                    deposit(tl, W, pb, vv, e);
                    tally_flush(tl, W, pb);
                    active = false;
                } else {
                    const float s = neg_ln(uniform(rng, k0, k1)) * hrcp(mumax);
                    x = fmaf(s, u, x);
                    y = fmaf(s, v, y);
                    z = fmaf(s, w, z);
                    if (outside(W.G, x, y, z)) {
                        tl.e_esc += (double)e;
                        tl.h_esc += (double)e;
                        active = false;
                    } else {
                        const int vv = voxel_of(W.G, x, y, z, ix, iy, iz);
                        const uint32_t vx = W.G.vox[vv];
                        const float rho = voxel_density(vx);
                        const int m = voxel_material(vx);
                        const float4 mu = lerp4(ptab + m * T.pg_n, gi, gt);
                        if (uniform(rng, k0, k1) * mumax < rho * mu.w) {
                            tl.ev[EV_REAL]++;
                            pm = m;   // the interaction waits (see below)
                        }
                    }
                }
                if (!active) {
                        history_flush(tl, W, rng.hlo, rng.hhi);
                }
            }
            // Real interactions are sampled together once kRealBatch lanes have
            // one (or the wavefront has no other live lane, or the pass has
            // nothing left to claim): the lanes of a wavefront share their
            // sampling code instead of a few running it each iteration.  A lane
            // waits where it is without drawing, so each particle's draws keep
            // their order; the voxel and the cross sections are recomputed from
            // the same inputs (the energy grid cell from this iteration's lookup).
            {
                const uint64_t br = ballot(pm >= 0);
                if (br && (cs.done || (uint32_t)__popcll(br) >= kRealBatch || br == ballot(active))) {
                    int itype = -1;   // the interaction sampled by this lane
                    if (pm >= 0) {
                        rng_topup(rng, k0, k1);
                        const int vv = voxel_of(W.G, x, y, z, ix, iy, iz);
                        const float4 mu = lerp4(ptab + pm * T.pg_n, gi, gt);
                        const float r = uniform(rng, k0, k1) * mu.w;
                        itype = r < mu.x ? 0 : (r < mu.x + mu.y ? 1 : 2);
                        if (itype == 0) {
                            float eps, t, turns;
                            sample_compton(T, rng, k0, k1, e, eps, t, turns);
                            const float u0 = u, v0 = v, w0 = w;
                            rotate(u, v, w, 1.0f - t, hsqrt(fmaxf(0.0f, t * (2.0f - t))), turns);
                            // exact split of E into E' and T (the unit is built without
                            // contraction, so the product is rounded on its own)
                            const float ec = eps * e;
                            float e1, te;
                            if (2.0f * ec >= e) {
                                e1 = ec;
                                te = e - ec;
                            } else {
                                te = e - ec;
                                e1 = e - te;
                            }
                            if (kerma || te <= ecut_e) {
                                deposit(tl, W, pb, vv, te);
                            } else {
                                float eu, ev, ew;
                                compton_electron_dir(e, e1, u0, v0, w0, u, v, w, eu, ev, ew);
                                qe.n = 1; qe.e0 = te; qe.du = eu; qe.dv = ev; qe.dw = ew;
                                qe.a0 = 0.0f; qe.role = 0u; qe.flag0 = 0u;
                            }
                            e = e1;
                        } else if (itype == 1) {
                            // photoelectric: the electron takes E along the photon
                            if (kerma || e <= ecut_e) {
                                deposit(tl, W, pb, vv, e);
                            } else {
                                qe.n = 1; qe.e0 = e; qe.du = u; qe.dv = v; qe.dw = w;
                                qe.a0 = 0.0f; qe.role = 0u; qe.flag0 = 0u;
                            }
                            active = false;
                        } else {
                            // pair: uniform split of E - 2 mc^2; the positron keeps a = E - K
                            float tm, tp, aa;
                            pair_split(e, uniform(rng, k0, k1), tm, tp, aa);
                            const bool e_local = kerma || tm <= ecut_e;
                            const bool p_local = kerma || tp <= ecut_e;
                            if (p_local) {
                                float du, dv, dw;
                                sample_iso(rng, k0, k1, du, dv, dw);
                                deposit(tl, W, pb, vv, tp);
                                qg.n = 2; qg.e = 0.5f * aa; qg.u = du; qg.v = dv; qg.w = dw; qg.wb = 2u;
                            }
                            if (e_local) deposit(tl, W, pb, vv, tm);
                            qe.du = u; qe.dv = v; qe.dw = w;
                            if (!e_local) {
                                qe.n = 1; qe.e0 = tm; qe.a0 = 0.0f; qe.role = 0u; qe.flag0 = 0u;
                                if (!p_local) {
                                    qe.n = 2; qe.e1 = tp; qe.a1 = aa;
                                }
                            } else if (!p_local) {
                                qe.n = 1; qe.e0 = tp; qe.a0 = aa; qe.role = 1u; qe.flag0 = 1u;
                            }
                            active = false;
                        }
                        tally_flush(tl, W, pb);
                        if (!active) history_flush(tl, W, rng.hlo, rng.hhi);
                        pm = -1;
                    }
                    wt.it[0] += (uint32_t)__popcll(ballot(itype == 1));
                    wt.it[1] += (uint32_t)__popcll(ballot(itype == 2));
                }
            }
            // secondaries: electrons/positrons to queue 1, annihilation photons to queue 0
            wt.died += (uint32_t)__popcll(act0 & ~ballot(active));
            const uint32_t jb = W.tag | (pb << 16);
            push_charged(qe, pe, head_e, ctl, R, W, jb, bufe, x, y, z, pack_vox(ix, iy, iz), rng, wt);
            push_photons(qg, pg, head_g, ctl, R, W, jb, bufg, x, y, z, rng, wt);
            }
            if (++iters > kMaxWaveIterations) {
                // safety net, never reached in a sound run: end the particles
                // still held (counted as anomalies) so the grid always drains
                const uint32_t n = (uint32_t)__popcll(ballot(active));
                wt.died += n;
                wt.bad += n;
                active = false;
                last_job = true;
                break;
            }
            if (cs.done) {
                // this job has nothing left to claim in the pass: move to a job
                // that has records left, or at the tail of a large pass stop
                // early; the particles still held go to the next pass
                int nj = -1;
                if (!last_job) {
                    nj = next_job(jc, W.j, R.n_jobs, 0);
                    last_job = nj < 0;
                }
                if (nj >= 0 || (big && __popcll(ballot(active)) < kTailLanes)) {
                    Particle q;
                    q.x = x; q.y = y; q.z = z; q.e = e;
                    q.u = u; q.v = v; q.w = w; q.nh = -1.0f;
                    q.hlo = rng.hlo; q.hhi = rng.hhi; q.path = rng.path; q.ctr = rng_ctr(rng);
                    q.vox = 0u; q.a = 0.0f; q.flags = 0u; q.job = W.tag | (pb << 16);
                    if (requeue(active, pg, head_g, ctl, &ctl->ring[0], R.hard[0], bufg, R.mask[0], q, wt)) {
                        history_flush(tl, W, rng.hlo, rng.hhi);
                    }
                    active = false;
                    next = nj;
                    break;
                }
            }
        }
        tally_flush(tl, W, pb);
        job_flush(tl, wt, W, jc);
        j = next;
    }
    // no staging load may still be writing the slice when the wave moves on
    if (stage != nullptr) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    release(pe, bufe, R.mask[1]);
    release(pg, bufg, R.mask[0]);
    pass_finish(tl, wt, ctl, 0);
}

template <bool kLds, bool kSolo, bool kPerm>
__global__ void __launch_bounds__(768) k_photon(Ctl* ctl, Tables T, RunDev R) {
    const float4* ptab = T.phot;
    float* lmw = nullptr;
    float4* stage = nullptr;
    if constexpr (kLds) {
        const int np = T.n_mat * T.pg_n;
        for (int i = threadIdx.x; i < np; i += blockDim.x) lds_tables[i] = T.phot[i];
        const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        lmw = reinterpret_cast<float*>(lds_tables + np) + wave * T.pg_n;
        stage = lds_tables + stage_offset(0, T, blockDim.x >> 6) + wave * (4u * kStage);
        __syncthreads();
        ptab = lds_tables;
    }
    photon_pass<kSolo, kPerm>(ctl, T, R, ptab, lmw, stage);
}

// ---------------------------------------------------------------------------
// electron pass: class-II condensed history with a random hinge, one step per
// iteration (section 2.1)
// ---------------------------------------------------------------------------
// One wavefront's share of an electron pass.  etab, rtab, rscale: the
// stopping and scattering data, the inverse range and its scales (LDS or
// global); stage: the wavefront's LDS slice for staged records (null: none).
template <bool kSolo, bool kPerm>
GDPM_DEV void electron_pass(Ctl* ctl, const Tables& T, const RunDev& R, const float4* etab, const float* rtab,
                            const float* rscale, float4* stage) {
    RingCtl* rc = &ctl->ring[1];
    const uint32_t begin = rc->begin, count = rc->count;
    const uint32_t* perm_in =
        kPerm && __builtin_amdgcn_readfirstlane(rc->permuted) ? bin_perm(R.bin[1], R.mask[1]) : nullptr;
    const bool big = !kSolo && count >= kTailMinPerLane * gridDim.x * blockDim.x;
    Particle* bufg = R.buf[0];
    Particle* bufe = R.buf[1];
    const uint32_t head_g = ctl->ring[0].head, head_e = ctl->ring[1].head;
    JobCtl* jc = R.jc;
    const float ecut = R.ecut_e;

    int j = first_job(R, count, 1);
    PushState pg{0u, 0u}, pe{0u, 0u};
    LaneTally tl;
    tally_init(tl);
    WaveTally wt{0u, 0u, 0u, 0u, 0u, 0u, 0u, {0u, 0u}};
    uint32_t iters = 0u;
    bool last_job = false;   // no other job has records left in this pass
    // one job at a time: a wavefront switches jobs with all its lanes empty
    while (j >= 0) {
        WJob W;
        load_job(W, R, j, 1);
        ClaimState cs{0u, 0u, 0u, false, 0u, 0u};
        bool active = false;
        float x = 0, y = 0, z = 0, u = 0, v = 0, w = 0, e = 0, nh = -1.0f, aa = 0.0f;
        int ix = 0, iy = 0, iz = 0;
        float rho = 1.0f;   // density and material of the current voxel, reloaded
        int mat = 0;        // when the particle enters a voxel
        bool positron = false;
        float hq = -1.0f;   // >= 0: a hard event waits; the step-start mu_h per g/cm^2
        uint32_t pb = 0u;   // batch slot of the lane's history
        Rng rng;
        rng_start(rng, 0u, 0u, 0u, 0u);
        int next = -1;
        for (;;) {
            const uint32_t k0 = W.k0, k1 = W.k1;
            const bool no_ms = (W.flags & 8u) != 0u;
            Particle p;
            if (refill<kSolo>(active, cs, jc, W, begin, ctl, bufe, R.mask[1], perm_in, p, wt, stage)) {
                x = p.x; y = p.y; z = p.z; e = p.e;
                u = p.u; v = p.v; w = p.w; nh = p.nh;
                ix = (int)(p.vox & 2047u);
                iy = (int)((p.vox >> 11) & 2047u);
                iz = (int)(p.vox >> 22);
                aa = p.a;
                positron = (p.flags & 1u) != 0u;
                pb = p.job >> 16;
                rng_start(rng, p.hlo, p.hhi, p.path, p.ctr);
                const uint32_t vx = W.G.vox[ix + W.G.nx * (iy + W.G.ny * iz)];
                rho = voxel_density(vx);
                mat = voxel_material(vx);
                active = true;
            }
            if (!ballot(active)) {
                if (cs.done && last_job) break;
                if (!cs.done) continue;
            } else {
            rng_topup(rng, k0, k1);
            const uint64_t act0 = ballot(active);
            wt.events += (uint32_t)__popcll(ballot(active && hq < 0.0f && !(e <= ecut)));

            PendCharged qe;
            PendPhoton qg;
            qe.n = 0;
            qg.n = 0;
            if (active && !(e <= kMaxEnergy)) {
                // a non-finite energy can only come from a damaged record (see the
                // photon pass)
                atomicAdd(&ctl->anomalies, 1ull);
                active = false;
                hq = -1.0f;
            }
            if (active && hq < 0.0f) {
                const int vv = ix + W.G.nx * (iy + W.G.ny * iz);
                if (e <= ecut) {
                    // absorption; a positron annihilates at rest into two photons
                    deposit(tl, W, pb, vv, e);
                    if (positron) {
                        float du, dv, dw;
                        sample_iso(rng, k0, k1, du, dv, dw);
                        qg.n = 2; qg.e = 0.5f * aa; qg.u = du; qg.v = dv; qg.w = dw; qg.wb = 0u;
                    }
                    active = false;
                } else {
                    const float irho = hrcp(rho);
                    const int m = mat;
                    if (nh < 0.0f) nh = neg_ln(uniform(rng, k0, k1));
                    const float t0 = e;
                    const float4 q0 = elec_at(T, etab, m, t0);
                    const float mus = rho * q0.y;
                    const float sh = mus > 0.0f ? nh * hrcp(mus) : 3.0e38f;
                    const float tfl = fmaxf(0.75f * t0, ecut);
                    const float rfl = tfl > ecut ? elec_at(T, etab, m, tfl).x : 0.0f;
                    const float se = (q0.x - rfl) * irho;
                    const bool hard = sh < se;
                    const float s = hard ? sh : se;
                    const float xi = uniform(rng, k0, k1);
                    const float s1 = xi * s, s2 = s - s1;
                    const float tend = hard ? fminf(fmaxf(range_inv(T, rtab, rscale, m, q0.x - rho * s), tfl), t0) : tfl;
                    // first half: to the hinge, or to the voxel face if that comes
                    // first.  Lanes that cross and lanes that reach the hinge share
                    // one move, one range lookup and one deposit.
                    int ax;
                    float db = face_dist(W.G, x, y, z, u, v, w, ix, iy, iz, ax);
                    bool crossed = db < s1;
                    float travelled = db;
                    {
                        const float d1 = crossed ? db : s1;
                        x = fmaf(d1, u, x); y = fmaf(d1, v, y); z = fmaf(d1, w, z);
                        const float t1 = fminf(fmaxf(range_inv(T, rtab, rscale, m, q0.x - rho * d1), tend), e);
                        deposit(tl, W, pb, vv, e - t1);
                        e = t1;
                    }
                    if (!crossed) {
                        // hinge: modified-Wentzel deflection for the whole step
                        if (!no_ms) {
                            const float tmid = 0.5f * (t0 + tend);
                            const float tt = s * rho * elec_at(T, etab, m, tmid).w;
                            const float mu = mw_mu(T, tt, uniform(rng, k0, k1));
                            const float turns = uniform(rng, k0, k1);
                            rotate(u, v, w, 1.0f - 2.0f * mu, 2.0f * hsqrt(mu * (1.0f - mu)), turns);
                        }
                        // second half: to the step end or the face; a lane that
                        // reaches the end loses exactly the energy left above tend
                        db = face_dist(W.G, x, y, z, u, v, w, ix, iy, iz, ax);
                        crossed = db < s2;
                        travelled = s1 + db;
                        const float d2 = crossed ? db : s2;
                        x = fmaf(d2, u, x); y = fmaf(d2, v, y); z = fmaf(d2, w, z);
                        float t2 = tend;
                        if (crossed) t2 = fminf(fmaxf(range_inv(T, rtab, rscale, m, q0.x - rho * travelled), tend), e);
                        deposit(tl, W, pb, vv, e - t2);
                        e = t2;
                    }
                    if (crossed) {
                        nh -= mus * travelled;
                        // move onto the face and into the next voxel
                        if (ax == 0) {
                            const int st = u > 0.0f ? 1 : -1;
                            x = (float)(st > 0 ? ix + 1 : ix) * W.G.dx;
                            ix += st;
                        } else if (ax == 1) {
                            const int st = v > 0.0f ? 1 : -1;
                            y = (float)(st > 0 ? iy + 1 : iy) * W.G.dy;
                            iy += st;
                        } else {
                            const int st = w > 0.0f ? 1 : -1;
                            z = (float)(st > 0 ? iz + 1 : iz) * W.G.dz;
                            iz += st;
                        }
                        if (ix < 0 || ix >= W.G.nx || iy < 0 || iy >= W.G.ny || iz < 0 || iz >= W.G.nz) {
                            // a positron takes its annihilation energy along (summed in FP64)
                            const double out = (double)e + (positron ? (double)aa : 0.0);
                            tl.e_esc += out;
                            tl.h_esc += out;
                            active = false;
                        } else {
                            // the next voxel's density and material, needed by the next step
                            const uint32_t vx = W.G.vox[ix + W.G.nx * (iy + W.G.ny * iz)];
                            rho = voxel_density(vx);
                            mat = voxel_material(vx);
                        }
                    } else if (hard) {
                        hq = q0.y;   // the hard event waits (see below)
                    } else {
                        nh -= mus * s;
                    }
                }
                if (!active) {
                        tally_flush(tl, W, pb);
                    history_flush(tl, W, rng.hlo, rng.hhi);
                }
            }
            // Hard events are rare (a few per hundred steps): run as they come,
            // their sampling would occupy the whole wavefront for one or two
            // lanes in most iterations.  A lane with one waits, where it is and
            // without drawing, until kHardBatch lanes wait, the wavefront has no
            // other live lane, or the pass has nothing left to claim; then they
            // are sampled together.  Each particle's draws keep their order.
            {
                const uint64_t bh = ballot(hq >= 0.0f);
                if (bh && (cs.done || (uint32_t)__popcll(bh) >= kHardBatch || bh == ballot(active))) {
                    int htype = -1;   // the hard event sampled by this lane
                    if (hq >= 0.0f) {
                        // delta scattering against the step-start majorant
                        // (mu_h grows with T; the step ended at e)
                        const int vv = ix + W.G.nx * (iy + W.G.ny * iz);
                        tl.ev[EV_HARD_CAND]++;
                        const float4 q1 = elec_at(T, etab, mat, e);
                        if (uniform(rng, k0, k1) * hq < q1.y) {
                            tl.ev[EV_HARD]++;
                            htype = uniform(rng, k0, k1) * q1.y < q1.z ? 0 : 1;
                            if (htype == 0) {
                                float eps, turns;
                                const float tt = e;
                                sample_moller(rng, k0, k1, tt, ecut, eps, turns);
                                const float tp = tt - eps * tt;   // >= T/2
                                const float wd = tt - tp;         // exact
                                const float tm2 = tt + kTwoMec2f;
                                const float itt = hrcp(tt);
                                const float cd = hsqrt(wd * tm2 * itt * hrcp(wd + kTwoMec2f));
                                const float cpr = hsqrt(tp * tm2 * itt * hrcp(tp + kTwoMec2f));
                                float du = u, dv = v, dw = w;
                                rotate(du, dv, dw, cd, hsqrt(fmaxf(0.0f, 1.0f - cd * cd)), turns);
                                rotate(u, v, w, cpr, hsqrt(fmaxf(0.0f, 1.0f - cpr * cpr)), turns + 0.5f);
                                if (wd <= ecut) {
                                    deposit(tl, W, pb, vv, wd);
                                } else {
                                    qe.n = 1; qe.e0 = wd; qe.du = du; qe.dv = dv; qe.dw = dw;
                                    qe.a0 = 0.0f; qe.role = 0u; qe.flag0 = 0u;
                                }
                                e = tp;
                            } else {
                                const float tt = e;
                                const float kph = sample_brems(rng, k0, k1, tt, R.ecut_g);
                                float kp, el;
                                if (2.0f * kph >= tt) {
                                    kp = kph;
                                    el = tt - kph;
                                } else {
                                    el = tt - kph;
                                    kp = tt - el;
                                }
                                qg.n = 1; qg.e = kp; qg.u = u; qg.v = v; qg.w = w; qg.wb = 0u;
                                e = el;
                            }
                        }
                        nh = -1.0f;
                        hq = -1.0f;
                    }
                    wt.it[0] += (uint32_t)__popcll(ballot(htype == 0));
                }
            }
            wt.died += (uint32_t)__popcll(act0 & ~ballot(active));
            const uint32_t jb = W.tag | (pb << 16);
            push_charged(qe, pe, head_e, ctl, R, W, jb, bufe, x, y, z, pack_vox(ix, iy, iz), rng, wt);
            push_photons(qg, pg, head_g, ctl, R, W, jb, bufg, x, y, z, rng, wt);
            }
            if (++iters > kMaxWaveIterations) {
                // safety net, never reached in a sound run: end the particles
                // still held (counted as anomalies) so the grid always drains
                const uint32_t n = (uint32_t)__popcll(ballot(active));
                wt.died += n;
                wt.bad += n;
                active = false;
                last_job = true;
                break;
            }
            if (cs.done) {
                // this job has nothing left to claim in the pass: move to a job
                // that has records left, or at the tail of a large pass stop
                // early; the particles still held go to the next pass
                int nj = -1;
                if (!last_job) {
                    nj = next_job(jc, W.j, R.n_jobs, 1);
                    last_job = nj < 0;
                }
                if (nj >= 0 || (big && __popcll(ballot(active)) < kTailLanes)) {
                    Particle q;
                    q.x = x; q.y = y; q.z = z; q.e = e;
                    q.u = u; q.v = v; q.w = w; q.nh = nh;
                    q.hlo = rng.hlo; q.hhi = rng.hhi; q.path = rng.path; q.ctr = rng_ctr(rng);
                    q.vox = pack_vox(ix, iy, iz); q.a = aa; q.flags = positron ? 1u : 0u;
                    q.job = W.tag | (pb << 16);
                    if (requeue(active, pe, head_e, ctl, &ctl->ring[1], R.hard[1], bufe, R.mask[1], q, wt)) {
                        history_flush(tl, W, rng.hlo, rng.hhi);
                    }
                    active = false;
                    next = nj;
                    break;
                }
            }
        }
        tally_flush(tl, W, pb);
        job_flush(tl, wt, W, jc);
        j = next;
    }
    // no staging load may still be writing the slice when the wave moves on
    if (stage != nullptr) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    release(pe, bufe, R.mask[1]);
    release(pg, bufg, R.mask[0]);
    pass_finish(tl, wt, ctl, 1);
}

template <bool kLds, bool kSolo, bool kPerm>
__global__ void __launch_bounds__(768) k_electron(Ctl* ctl, Tables T, RunDev R) {
    const float4* etab = T.elec;
    const float* rtab = T.rinv;
    const float* rscale = T.rinv_scale;
    float4* stage = nullptr;
    if constexpr (kLds) {
        const int ne = T.n_mat * T.eg_n, nr = T.n_mat * T.nr;
        stage = lds_tables + stage_offset(1, T, blockDim.x >> 6) +
                __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * (4u * kStage);
        for (int i = threadIdx.x; i < ne; i += blockDim.x) lds_tables[i] = T.elec[i];
        float* lr = reinterpret_cast<float*>(lds_tables + ne);
        for (int i = threadIdx.x; i < nr; i += blockDim.x) lr[i] = T.rinv[i];
        for (int i = threadIdx.x; i < T.n_mat; i += blockDim.x) lr[nr + i] = T.rinv_scale[i];
        __syncthreads();
        etab = lds_tables;
        rtab = lr;
        rscale = lr + nr;
    }
    electron_pass<kSolo, kPerm>(ctl, T, R, etab, rtab, rscale, stage);
}

// ---------------------------------------------------------------------------
// both passes of an iteration in one launch: the first `photon_waves`
// wavefronts of each workgroup start with the photon pass, the others with the
// electron pass, and a wavefront that has finished its first pass helps with
// the other.  The photon pass mostly waits on its random voxel reads and the
// electron pass mostly issues vector instructions, so a CU runs one while the
// other waits.  The electron tables and the wavefronts' staging slices are in
// LDS; the photon cross sections and majorants are read through the caches.
// Each pass reads what its queue held at the set-up: what either pass pushes
// is transported in the next iteration.
// ---------------------------------------------------------------------------
template <bool kPerm>
__global__ void __launch_bounds__(768) k_transport(Ctl* ctl, Tables T, RunDev R, int photon_waves) {
    const int ne = T.n_mat * T.eg_n, nr = T.n_mat * T.nr;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float4* stage = lds_tables + stage_offset(1, T, blockDim.x >> 6) + wave * (4u * kStage);
    for (int i = threadIdx.x; i < ne; i += blockDim.x) lds_tables[i] = T.elec[i];
    float* lr = reinterpret_cast<float*>(lds_tables + ne);
    for (int i = threadIdx.x; i < nr; i += blockDim.x) lr[i] = T.rinv[i];
    for (int i = threadIdx.x; i < T.n_mat; i += blockDim.x) lr[nr + i] = T.rinv_scale[i];
    __syncthreads();
    for (int k = 0; k < 2; ++k) {
        const bool photons = ((int)wave < photon_waves) == (k == 0);
        if (photons)
            photon_pass<false, kPerm>(ctl, T, R, T.phot, nullptr, stage);
        else
            electron_pass<false, kPerm>(ctl, T, R, lds_tables, lr, lr + nr, stage);
    }
}

// ---------------------------------------------------------------------------
// queue re-binning: counting sort of the positions [head, tail) by the key job x
// bin (bins: log2-energy intervals, or boxes of the phantom with `space` > 0).
// The records stay where they are: the count pass keeps each position's key,
// the scatter writes the permutation, in key order, of the positions that hold
// a running job's record (empty ones are dropped), and the pass reads its input
// through it.  Each job's records form one segment of the permutation.
// ---------------------------------------------------------------------------
GDPM_DEV int energy_bin(float e, float lo, float inv, int nb) {
    const int b = (int)((hlog2(e) - lo) * inv);
    return min(max(b, 0), nb - 1);
}

// the box of a position when the phantom is cut into space^3 equal boxes
// (x fastest); positions on or past the far faces fall in the last box
GDPM_DEV int space_bin(const Geom& G, float x, float y, float z, int space) {
    const float sc = (float)space;
    const int bx = min(max((int)(x * G.idx * sc / (float)G.nx), 0), space - 1);
    const int by = min(max((int)(y * G.idy * sc / (float)G.ny), 0), space - 1);
    const int bz = min(max((int)(z * G.idz * sc / (float)G.nz), 0), space - 1);
    return bx + space * (by + space * bz);
}

// the slot of a record's job if that job is running in it (slot below n_jobs,
// same generation), else -1
GDPM_DEV int record_job(const RunDev& R, uint32_t job_word) {
    const int slot = (int)(job_word & 0xFFu);
    if (slot >= R.n_jobs) return -1;
    const uint32_t gen = R.jobs[slot].gen & 0xFFu;
    return ((job_word >> 8) & 0xFFu) == gen ? slot : -1;
}

// re-binning key word of the record in `slot`: job x nb + bin, kEmptyKey for an
// empty position, kOrphanKey for a record of no running job
GDPM_DEV uint32_t record_key(const RunDev& R, const Particle* buf, uint32_t mask, uint32_t slot, int nb,
                             float lo, float inv, int space) {
    const float4 w0 = reinterpret_cast<const float4*>(buf + (slot & mask))[0];
    const float4 w3 = reinterpret_cast<const float4*>(buf + (slot & mask))[3];
    if (record_empty(w0.w)) return kEmptyKey;
    const int j = record_job(R, __float_as_uint(w3.w));
    if (j < 0) return kOrphanKey;
    const int b = space > 0 ? space_bin(R.jobs[j].G, w0.x, w0.y, w0.z, space) : energy_bin(w0.w, lo, inv, nb);
    return (uint32_t)(j * nb + b);
}

__global__ void __launch_bounds__(256) k_bin_count(Ctl* ctl, RunDev R, int ri, int nb, float lo,
                                                   float inv, int space) {
    if (ctl->overflow) return;
    extern __shared__ uint32_t hist[];
    const int nk = R.n_jobs * nb;
    for (int i = threadIdx.x; i < nk; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const RingCtl& r = ctl->ring[ri];
    const uint32_t n = r.tail - r.head;
    const Particle* buf = R.buf[ri];
    // each position's key is kept (4 B), so that the scatter does not read
    // the records again
    uint32_t* kw = bin_keys(R.bin[ri]);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t k = record_key(R, buf, R.mask[ri], r.head + i, nb, lo, inv, space);
        if (k < kOrphanKey) atomicAdd(&hist[k], 1u);
        kw[i] = k;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nk; i += blockDim.x)
        if (hist[i]) atomicAdd(&R.jc->bin_count[i], hist[i]);
}

// exclusive scan of the key counts (one block of 1024 threads, <= 4 keys each);
// also the jobs' segments and the number of records kept
__global__ void __launch_bounds__(1024) k_bin_scan(Ctl* ctl, RunDev R, int nb, int ri) {
    if (ctl->overflow) return;
    __shared__ uint32_t part[1024];
    JobCtl* jc = R.jc;
    const int nk = R.n_jobs * nb;
    const int per = (nk + 1023) / 1024;
    const int k0 = threadIdx.x * per;
    uint32_t s = 0u;
    for (int k = k0; k < k0 + per && k < nk; ++k) s += jc->bin_count[k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
        const uint32_t a = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += a;
        __syncthreads();
    }
    uint32_t acc = part[threadIdx.x] - s;
    for (int k = k0; k < k0 + per && k < nk; ++k) {
        jc->bin_cursor[k] = acc;
        acc += jc->bin_count[k];
        jc->bin_count[k] = 0u;
    }
    __syncthreads();
    const uint32_t total = part[1023];
    for (int j = threadIdx.x; j < R.n_jobs; j += blockDim.x) {
        const uint32_t b0 = jc->bin_cursor[j * nb];
        const uint32_t b1 = j + 1 < R.n_jobs ? jc->bin_cursor[(j + 1) * nb] : total;
        jc->seg_begin[ri][j] = b0;
        jc->seg_count[ri][j] = b1 - b0;
    }
    if (threadIdx.x == 0) ctl->n_valid = total;
}

__global__ void __launch_bounds__(256) k_bin_scatter(Ctl* ctl, RunDev R, int ri, int nb) {
    if (ctl->overflow) return;
    extern __shared__ uint32_t cnt[];   // [nk] this block's counts, then ranks; [nk] its bases
    const int nk = R.n_jobs * nb;
    uint32_t* base = cnt + nk;
    const RingCtl& r = ctl->ring[ri];
    const uint32_t n = r.tail - r.head;
    const uint32_t mask = R.mask[ri];
    const uint32_t* kw = bin_keys(R.bin[ri]);
    uint32_t* perm = bin_perm(R.bin[ri], mask);
    // each block takes one contiguous share of the positions: it counts its
    // keys, takes its place in every key's run with one atomic per key, then
    // writes its positions (one global atomic per key and block, not per tile)
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint32_t i0 = min(n, blockIdx.x * per), i1 = min(n, i0 + per);
    for (int q = threadIdx.x; q < nk; q += blockDim.x) cnt[q] = 0u;
    __syncthreads();
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const uint32_t k = kw[i];
        if (k < kOrphanKey) atomicAdd(&cnt[k], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nk; q += blockDim.x) {
        base[q] = cnt[q] ? atomicAdd(&R.jc->bin_cursor[q], cnt[q]) : 0u;
        cnt[q] = 0u;
    }
    __syncthreads();
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const uint32_t k = kw[i];
        if (k < kOrphanKey) {
            perm[(base[k] + atomicAdd(&cnt[k], 1u)) & mask] = r.head + i;
        } else if (k == kOrphanKey) {
            // a record of a job no longer running: only a broken bookkeeping
            // leaves one; it is dropped (the count pass skipped it) and counted
            atomicAdd(&ctl->anomalies, 1ull);
        }
    }
}

// live records per job in both queues (a consistency check of the host's
// particle accounting; counts[j] += records of job j)
__global__ void __launch_bounds__(256) k_count_records(const Ctl* ctl, RunDev R,
                                                       unsigned long long* counts) {
    for (int ri = 0; ri < 2; ++ri) {
        const RingCtl& r = ctl->ring[ri];
        const uint32_t n = r.tail - r.head;
        const Particle* buf = R.buf[ri];
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            const float4* q = reinterpret_cast<const float4*>(buf + ((r.head + i) & R.mask[ri]));
            const int j = !record_empty(q[0].w) ? record_job(R, __float_as_uint(q[3].w)) : -1;
            if (j >= 0) atomicAdd(&counts[j], 1ull);
        }
    }
}

// after the re-binning the pass reads the queue through the permutation
__global__ void k_bin_swap(Ctl* ctl, int ri) {
    if (ctl->overflow) return;
    ctl->ring[ri].permuted = 1u;
}


// ---------------------------------------------------------------------------
// batch statistics (section 2.2.1, section 3.1): per voxel the mean over the
// batches of D_b = E_b / (rho V n_b) and its standard error
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_dose_stats(Ctl* ctl, const double* slots, size_t nvox,
                                                    int nb, const double* inv_mass_n,
                                                    const uint32_t* vox, double vvox, float min_rho,
                                                    double* dose, double* sigma) {
    double emax = 0.0, edep = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox;
         i += (size_t)gridDim.x * blockDim.x) {
        const double rho = (double)voxel_density(vox[i]);
        const double im = 1.0 / (rho * vvox);
        double s = 0.0, s2 = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double eb = slots[(size_t)b * nvox + i];
            edep += eb;
            const double d = eb * im * inv_mass_n[b];
            s += d;
        }
        const double mean = s / nb;
        for (int b = 0; b < nb; ++b) {
            const double d = slots[(size_t)b * nvox + i] * im * inv_mass_n[b] - mean;
            s2 += d * d;
        }
        if (dose) dose[i] = mean;
        if (sigma) sigma[i] = nb > 1 ? sqrt(s2 / ((double)nb * (nb - 1))) : 0.0;
        if (rho >= (double)min_rho) emax = fmax(emax, mean);
    }
    // block reductions
    __shared__ double sh[256];
    sh[threadIdx.x] = emax;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(&ctl->dmax_bits, (unsigned long long)__double_as_longlong(sh[0]));
    __syncthreads();
    sh[threadIdx.x] = edep;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(&ctl->red[0], sh[0]);
}

// mean of sigma / D_max over voxels with D > D_max / 2
__global__ void __launch_bounds__(256) k_unc(Ctl* ctl, const double* dose, const double* sigma,
                                             const uint32_t* vox, float min_rho, size_t nvox) {
    const double dmax = __longlong_as_double((long long)ctl->dmax_bits);
    double s = 0.0, c = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox;
         i += (size_t)gridDim.x * blockDim.x) {
        if (dose[i] > 0.5 * dmax && voxel_density(vox[i]) >= min_rho) {
            s += sigma[i];
            c += 1.0;
        }
    }
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = s;
    sh[1][threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsafeAtomicAdd(&ctl->red[1], sh[0][0]);
        unsafeAtomicAdd(&ctl->red[2], sh[1][0]);
    }
}

// ---------------------------------------------------------------------------
// test kernels
// ---------------------------------------------------------------------------
__global__ void k_test_philox(uint32_t k0, uint32_t k1, const uint4* ctr, uint4* out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 c = ctr[i];
    philox(k0, k1, c.x, c.y, c.z, c.w);
    out[i] = c;
}

__global__ void k_test_sample(Tables T, int which, float e, float p1, float p2, uint32_t k0,
                              uint32_t k1, int n, float* out1, float* out2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rng r;
    rng_start(r, (uint32_t)i, 0u, 0u, 0u);
    rng_topup(r, k0, k1);
    float a = 0.0f, b = 0.0f;
    if (which == 0) {
        float eps, t, turns;
        sample_compton(T, r, k0, k1, e, eps, t, turns);
        a = eps;
        b = 1.0f - t;
    } else if (which == 1) {
        float eps, turns;
        sample_moller(r, k0, k1, e, p1, eps, turns);
        const float tt = e, tp = tt - eps * tt, wd = tt - tp;
        a = wd / tt;
        b = hsqrt(tp * (tt + kTwoMec2f) / (tt * (tp + kTwoMec2f)));
    } else if (which == 2) {
        a = sample_brems(r, k0, k1, e, p1);
    } else if (which == 3) {
        a = mw_mu(T, e, uniform(r, k0, k1));
    } else if (which == 4) {
        float u = 0.0f, v = 0.0f, w = 1.0f;
        const int nh = (int)p2;
        for (int k = 0; k < nh; ++k) {
            const float mu = mw_mu(T, e, uniform(r, k0, k1));
            const float turns = uniform(r, k0, k1);
            rotate(u, v, w, 1.0f - 2.0f * mu, 2.0f * hsqrt(mu * (1.0f - mu)), turns);
        }
        a = w;
        b = u * u + v * v + w * w;
    } else if (which == 5) {
        float du, dv, dw;
        sample_iso(r, k0, k1, du, dv, dw);
        a = dw;
        b = -(du * du + dv * dv + dw * dw);
    } else if (which == 6) {
        float tm, tp, aa;
        pair_split(e, uniform(r, k0, k1), tm, tp, aa);
        a = tm / (e - kTwoMec2f);
        b = (tm + tp) - (e - kTwoMec2f);   // 0: the split is exact
    } else if (which == 7) {
        // the photon interaction's kinematics on a photon along +z
        float eps, t, turns;
        sample_compton(T, r, k0, k1, e, eps, t, turns);
        float u = 0.0f, v = 0.0f, w = 1.0f;
        rotate(u, v, w, 1.0f - t, hsqrt(fmaxf(0.0f, t * (2.0f - t))), turns);
        const float e1 = eps * e;
        float eu, ev, ew;
        compton_electron_dir(e, e1, 0.0f, 0.0f, 1.0f, u, v, w, eu, ev, ew);
        a = ew;
        b = w;
    }
    out1[i] = a;
    if (out2) out2[i] = b;
}

GDPM_DEV void test_source_one(const SourceDev& S, const Geom& G, uint32_t k0, uint32_t k1,
                              unsigned long long hist0, int i, int n, float* out, uint32_t* chain) {
    const unsigned long long h = hist0 + i;
    Rng r;
    rng_start(r, (uint32_t)h, (uint32_t)(h >> 32), 0u, 0u);
    rng_topup(r, k0, k1);
    const Primary p = make_primary(S, G, r, k0, k1, chain, (uint32_t)i, (uint32_t)n);
    float* o = out + 8 * (size_t)i;
    o[0] = p.e;
    o[1] = p.in ? (float)p.beamlet : -1.0f;
    o[2] = p.x; o[3] = p.y; o[4] = p.z;
    o[5] = p.u; o[6] = p.v; o[7] = p.w;
}

// histories hist0 .. hist0+n-1 as a job starting at hist0 samples them; with
// Metropolis chains one thread per chain, the chains freshly started
__global__ void k_test_source(SourceDev S, Geom G, uint32_t k0, uint32_t k1,
                              unsigned long long hist0, int n, float* out) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (S.metro) {
        if (t >= kMetroChains) return;
        uint32_t state = metropolis_start(S, t, k0, k1);
        const uint32_t first = (uint32_t)((t + kMetroChains - hist0 % kMetroChains) % kMetroChains);
        for (uint32_t i = first; i < (uint32_t)n; i += kMetroChains)
            test_source_one(S, G, k0, k1, hist0, (int)i, n, out, &state);
        return;
    }
    if ((int)t >= n) return;
    test_source_one(S, G, k0, k1, hist0, (int)t, n, out, nullptr);
}

// the start of every Metropolis chain of a job
__global__ void k_metro_init(SourceDev S, uint32_t k0, uint32_t k1, uint32_t* chains) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < kMetroChains) chains[c] = metropolis_start(S, c, k0, k1);
}

__global__ void k_test_lookup(Tables T, int which, int m, const float* in, float* out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = in[i];
    float r = 0.0f;
    if (which == 0) {
        int gi;
        float gt;
        grid(hlog2(x), T.pg_lo, T.pg_inv, T.pg_n, gi, gt);
        r = lerp4(T.phot + m * T.pg_n, gi, gt).w;
    } else if (which >= 1 && which <= 4) {
        const float4 q = elec_at(T, m, x);
        r = which == 1 ? q.x : (which == 2 ? q.y : (which == 3 ? q.z : q.w));
    } else if (which == 5) {
        r = range_inv(T, m, x);
    } else if (which == 6) {
        r = mw_screening(T, x);
    }
    out[i] = r;
}

// ---------------------------------------------------------------------------
// host launchers (the host runtime calls these; kernels stay in this unit)
// ---------------------------------------------------------------------------
hipError_t launch_setup(hipStream_t st, Ctl* ctl, const RunDev& R, int ri, int rebinned, int lone) {
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, st, ctl, R, ri, rebinned, lone);
    return hipGetLastError();
}
hipError_t launch_source(hipStream_t st, int blocks, Ctl* ctl, const RunDev& R, const SrcSeg* segs,
                         const SrcHdr* hdr, int ri) {
    hipLaunchKernelGGL(k_source, dim3(blocks), dim3(256), 0, st, ctl, R, segs, hdr, ri);
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(1), 0, st, ctl, ri, hdr);
    return hipGetLastError();
}
hipError_t launch_finish(hipStream_t st, Ctl* ctl, int ri) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1), 0, st, ctl, ri);
    return hipGetLastError();
}
// LDS bytes the table staging of a pass needs with `waves` wavefronts per block
size_t transport_lds_bytes(int ri, const Tables& T, int waves) {
    return ((size_t)stage_offset(ri, T, waves) + (size_t)waves * 4u * kStage) * sizeof(float4);
}

// allow the staged kernels to use `bytes` of dynamic LDS
hipError_t transport_lds_optin(size_t bytes) {
    const void* kernels[] = {(const void*)k_photon<true, false, false>, (const void*)k_electron<true, false, false>,
                             (const void*)k_photon<true, false, true>,  (const void*)k_electron<true, false, true>,
                             (const void*)k_photon<true, true, false>,  (const void*)k_electron<true, true, false>,
                             (const void*)k_photon<true, true, true>,   (const void*)k_electron<true, true, true>,
                             (const void*)k_transport<false>,           (const void*)k_transport<true>};
    for (const void* k : kernels) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
template <bool kPerm>
void launch_transport_form(hipStream_t st, int ri, int blocks, int threads, bool lds, bool solo, size_t bytes,
                           Ctl* ctl, const Tables& T, const RunDev& R) {
    if (ri == 0) {
        if (solo)
            hipLaunchKernelGGL((k_photon<true, true, kPerm>), dim3(blocks), dim3(threads), bytes, st, ctl, T, R);
        else if (lds)
            hipLaunchKernelGGL((k_photon<true, false, kPerm>), dim3(blocks), dim3(threads), bytes, st, ctl, T, R);
        else
            hipLaunchKernelGGL((k_photon<false, false, kPerm>), dim3(blocks), dim3(threads), 0, st, ctl, T, R);
    } else {
        if (solo)
            hipLaunchKernelGGL((k_electron<true, true, kPerm>), dim3(blocks), dim3(threads), bytes, st, ctl, T, R);
        else if (lds)
            hipLaunchKernelGGL((k_electron<true, false, kPerm>), dim3(blocks), dim3(threads), bytes, st, ctl, T, R);
        else
            hipLaunchKernelGGL((k_electron<false, false, kPerm>), dim3(blocks), dim3(threads), 0, st, ctl, T, R);
    }
}
}  // namespace

// `solo`: the one-particle-per-wavefront measurement form (staged tables only);
// `permuted`: the pass follows a re-binning by job alone (its input is read
// through the permutation)
hipError_t launch_transport(hipStream_t st, int ri, int blocks, int threads, bool lds, bool solo, bool permuted,
                            Ctl* ctl, const Tables& T, const RunDev& R) {
    const size_t bytes = lds ? transport_lds_bytes(ri, T, threads / 64) : 0;
    if (solo && !lds) return hipErrorInvalidValue;
    if (permuted)
        launch_transport_form<true>(st, ri, blocks, threads, lds, solo, bytes, ctl, T, R);
    else
        launch_transport_form<false>(st, ri, blocks, threads, lds, solo, bytes, ctl, T, R);
    return hipGetLastError();
}
// both passes in one launch (k_transport); its LDS is the electron pass's
// layout (transport_lds_bytes(1, T, threads / 64))
hipError_t launch_fused(hipStream_t st, int blocks, int threads, int photon_waves, bool permuted, Ctl* ctl,
                        const Tables& T, const RunDev& R) {
    const size_t bytes = transport_lds_bytes(1, T, threads / 64);
    if (permuted)
        hipLaunchKernelGGL((k_transport<true>), dim3(blocks), dim3(threads), bytes, st, ctl, T, R, photon_waves);
    else
        hipLaunchKernelGGL((k_transport<false>), dim3(blocks), dim3(threads), bytes, st, ctl, T, R, photon_waves);
    return hipGetLastError();
}

// nb bins per job (energy intervals, or space^3 boxes with space > 0);
// R.n_jobs * nb <= kMaxKeys
hipError_t launch_rebin(hipStream_t st, int blocks, Ctl* ctl, const RunDev& R, int ri, int nb,
                        float lo, float inv, int space) {
    const size_t nk = (size_t)R.n_jobs * nb;
    hipLaunchKernelGGL(k_bin_count, dim3(blocks), dim3(256), nk * sizeof(uint32_t), st, ctl, R, ri,
                       nb, lo, inv, space);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, ctl, R, nb, ri);
    hipLaunchKernelGGL(k_bin_scatter, dim3(blocks), dim3(256), 2 * nk * sizeof(uint32_t), st, ctl, R,
                       ri, nb);
    hipLaunchKernelGGL(k_bin_swap, dim3(1), dim3(1), 0, st, ctl, ri);
    return hipGetLastError();
}
hipError_t launch_count_records(hipStream_t st, int blocks, const Ctl* ctl, const RunDev& R,
                                unsigned long long* counts) {
    hipLaunchKernelGGL(k_count_records, dim3(blocks), dim3(256), 0, st, ctl, R, counts);
    return hipGetLastError();
}
hipError_t launch_stats(hipStream_t st, int blocks, Ctl* ctl, const double* slots, size_t nvox,
                        int nb, const double* inv_n, const uint32_t* vox, double vvox, float min_rho,
                        double* dose, double* sigma) {
    hipLaunchKernelGGL(k_dose_stats, dim3(blocks), dim3(256), 0, st, ctl, slots, nvox, nb, inv_n,
                       vox, vvox, min_rho, dose, sigma);
    hipLaunchKernelGGL(k_unc, dim3(blocks), dim3(256), 0, st, ctl, (const double*)dose,
                       (const double*)sigma, vox, min_rho, nvox);
    return hipGetLastError();
}
hipError_t launch_test_philox(hipStream_t st, uint32_t k0, uint32_t k1, const uint4* ctr, uint4* out,
                              int n) {
    hipLaunchKernelGGL(k_test_philox, dim3((n + 255) / 256), dim3(256), 0, st, k0, k1, ctr, out, n);
    return hipGetLastError();
}
hipError_t launch_test_sample(hipStream_t st, const Tables& T, int which, float e, float p1, float p2,
                              uint32_t k0, uint32_t k1, int n, float* out1, float* out2) {
    hipLaunchKernelGGL(k_test_sample, dim3((n + 255) / 256), dim3(256), 0, st, T, which, e, p1, p2,
                       k0, k1, n, out1, out2);
    return hipGetLastError();
}
hipError_t launch_test_source(hipStream_t st, const SourceDev& S, const Geom& G, uint32_t k0,
                              uint32_t k1, unsigned long long hist0, int n, float* out) {
    const int blocks = S.metro ? (int)(kMetroChains / 256) : (n + 255) / 256;
    hipLaunchKernelGGL(k_test_source, dim3(blocks), dim3(256), 0, st, S, G, k0, k1, hist0, n, out);
    return hipGetLastError();
}
hipError_t launch_metro_init(hipStream_t st, const SourceDev& S, uint32_t k0, uint32_t k1, uint32_t* chains) {
    hipLaunchKernelGGL(k_metro_init, dim3(kMetroChains / 256), dim3(256), 0, st, S, k0, k1, chains);
    return hipGetLastError();
}
// scattered FP64 atomic additions: `iters` per thread at hashed addresses of
// an array of n words (the dose tally's access pattern without the transport)
__global__ void __launch_bounds__(256) k_atomic_rate(double* buf, uint32_t n, uint32_t iters) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t k = 0; k < iters; ++k) {
        uint32_t h = t * 0x9E3779B9u + k * 0x85EBCA6Bu;
        h ^= h >> 16;
        h *= 0x7FEB352Du;
        h ^= h >> 15;
        h *= 0x846CA68Bu;
        h ^= h >> 16;
        unsafeAtomicAdd(&buf[h % n], 1.0);
    }
}

hipError_t launch_atomic_rate(hipStream_t st, int blocks, double* buf, uint32_t n, uint32_t iters) {
    hipLaunchKernelGGL(k_atomic_rate, dim3(blocks), dim3(256), 0, st, buf, n, iters);
    return hipGetLastError();
}

hipError_t launch_test_lookup(hipStream_t st, const Tables& T, int which, int m, const float* in,
                              float* out, int n) {
    hipLaunchKernelGGL(k_test_lookup, dim3((n + 255) / 256), dim3(256), 0, st, T, which, m, in, out, n);
    return hipGetLastError();
}

}  // namespace gdpm
