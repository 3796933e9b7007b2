/*
 * oracle.c -- reference CPU transport (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow, double-precision Monte Carlo of coupled photon/electron
 * transport through a voxel phantom, one particle at a time with a LIFO stack
 * of secondaries.  It follows the paper's method:
 *   - photon Woodcock (delta) tracking against a majorant (section 2.1);
 *   - class-II condensed-history electrons: hard Moller and bremsstrahlung
 *     events above cutoffs simulated one by one, continuous slowing down with
 *     the restricted stopping power below them (section 2.1);
 *   - positrons transported as electrons, two photons created at the end of
 *     the track (section 2.1);
 *   - absorption energies 200 keV (electrons) and 50 keV (photons) (section 3.1);
 *   - N_b batches, per-voxel mean dose and its uncertainty (sections 2.2.1, 3.1);
 *   - fluence-map beamlets chosen by the cumulative-probability search
 *     P(I) <= r < P(I+1) (section 2.3.1).
 * The paper keeps DPM's physics but does not print it; the closed-form models
 * written out below are this project's reading (stated in the design notes),
 * evaluated directly in FP64, never from tables.  The random numbers are
 * Philox4x32-10 (Salmon et al., SC'11), a counter-based generator, keyed so
 * that every particle owns a stream that does not depend on scheduling.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load
 * this library.  It shares no code with the GPU library.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 constants */
#define MC2 0.51099895          /* electron rest energy, MeV */
#define RE 2.8179403262e-13     /* classical electron radius, cm */
#define NAV 6.02214076e23       /* Avogadro constant, 1/mol */
#define ALPHA (1.0 / 137.035999084)
#define PI 3.14159265358979323846

/* ======================================================================== */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                         */
/* ======================================================================== */

void orc_philox(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {           /* Weyl key schedule */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* A particle's stream: key = (seed lo, seed hi ^ job); counter = (history lo,
 * history hi, path, draw >> 2); draw d takes word d & 3 of that block. */
typedef struct {
    uint32_t key[2];
    uint64_t hist;
    uint32_t path;
    uint32_t ctr;
} stream_t;

static stream_t stream_make(uint64_t seed, uint32_t job, uint64_t hist, uint32_t path) {
    stream_t s;
    s.key[0] = (uint32_t)seed;
    s.key[1] = (uint32_t)(seed >> 32) ^ job;
    s.hist = hist;
    s.path = path;
    s.ctr = 0;
    return s;
}

/* uniform on the open interval (0,1): (2*(x >> 9) + 1) * 2^-24 */
static double draw(stream_t* s) {
    uint32_t c[4] = {(uint32_t)s->hist, (uint32_t)(s->hist >> 32), s->path, s->ctr >> 2};
    uint32_t o[4];
    orc_philox(s->key, c, o);
    uint32_t x = o[s->ctr & 3u];
    s->ctr += 1;
    return (2.0 * (double)(x >> 9) + 1.0) * (1.0 / 16777216.0);
}

/* stream of the secondary created in role `word` (0..3) by a parent whose
 * draw counter currently stands at parent->ctr */
static stream_t spawn(const stream_t* parent, int word) {
    uint32_t c[4] = {(uint32_t)parent->hist, (uint32_t)(parent->hist >> 32), parent->path,
                     0x80000000u | parent->ctr};
    uint32_t o[4];
    orc_philox(parent->key, c, o);
    stream_t s = *parent;
    s.path = o[word];
    s.ctr = 0;
    return s;
}

void orc_uniforms(uint64_t seed, uint32_t job, uint64_t hist, uint32_t path, uint32_t ctr0,
                  int n, double* out) {
    stream_t s = stream_make(seed, job, hist, path);
    s.ctr = ctr0;
    for (int i = 0; i < n; ++i) out[i] = draw(&s);
}

uint32_t orc_spawn_path(uint64_t seed, uint32_t job, uint64_t hist, uint32_t path,
                        uint32_t ctr, int word) {
    stream_t s = stream_make(seed, job, hist, path);
    s.ctr = ctr;
    return spawn(&s, word).path;
}

/* ======================================================================== */
/* Materials and closed-form physics                                         */
/* ======================================================================== */

typedef struct {
    double z, za, i_mev;
    double a;    /* A = Z / (Z/A), g/mol */
    double x0;   /* radiation length, g/cm^2 */
    double ne;   /* electrons per gram, N_A Z/A */
} mat_t;

static mat_t mat_make(const orc_material* m) {
    mat_t r;
    r.z = m->z;
    r.za = m->z_over_a;
    r.i_mev = m->i_ev * 1e-6;
    r.a = m->z / m->z_over_a;
    /* radiation length, Dahl's approximation as quoted by the PDG */
    r.x0 = 716.4 * r.a / (r.z * (r.z + 1.0) * log(287.0 / sqrt(r.z)));
    r.ne = NAV * m->z_over_a;
    return r;
}

/* Klein-Nishina total cross section per free electron (cm^2), k = E/mc^2 */
static double sigma_kn(double k) {
    double a = 1.0 + 2.0 * k;
    double l = log(a);
    return 2.0 * PI * RE * RE *
           ((1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - l / k) + l / (2.0 * k) -
            (1.0 + 3.0 * k) / (a * a));
}

/* Klein-Nishina dsigma/deps per electron, eps = E'/E */
static double dsigma_kn(double k, double eps) {
    double t = (1.0 - eps) / (k * eps);
    double sin2 = t * (2.0 - t);
    return PI * RE * RE / k * (1.0 / eps + eps) * (1.0 - eps * sin2 / (1.0 + eps * eps));
}

static double mu_compton(const mat_t* m, double e) { return m->ne * sigma_kn(e / MC2); }

static double mu_photo(const mat_t* m, double e) {
    double r = m->z / 7.42;
    return 2.8e-6 * r * r * r * (m->za / 0.55508) / (e * e * e);
}

static double mu_pair(const mat_t* m, double e) {
    if (e <= 2.0 * MC2) return 0.0;
    double f = 1.0 - 2.0 * MC2 / e;
    return 0.35 * (7.0 / 9.0) / m->x0 * f * f * f;
}

/* restricted collision stopping power (MeV cm^2/g), Berger-Seltzer form with
 * no density effect; energy transfers up to min(wcc, T/2) */
static double l_restricted(const mat_t* m, double t, double wcc) {
    double tau = t / MC2, g = tau + 1.0, b2 = 1.0 - 1.0 / (g * g);
    double dl = fmin(wcc, 0.5 * t) / MC2;
    double im = m->i_mev / MC2;
    double br = log(2.0 * (tau + 2.0) / (im * im)) - 1.0 - b2 + log((tau - dl) * dl) +
                tau / (tau - dl) + (0.5 * dl * dl + (2.0 * tau + 1.0) * log(1.0 - dl / tau)) / (g * g);
    return 2.0 * PI * RE * RE * MC2 * m->ne / b2 * br;
}

/* bremsstrahlung, complete-screening spectrum dmu/dk = (1/X0)(1/k)(4/3 - 4/3 y + y^2) */
static double dmu_brems(const mat_t* m, double t, double k) {
    double y = k / t;
    return (4.0 / 3.0 - 4.0 / 3.0 * y + y * y) / (m->x0 * k);
}

/* radiative stopping power below the hard threshold: integral of k dmu/dk on [0, min(wcb,T)] */
static double s_rad_soft(const mat_t* m, double t, double wcb) {
    double w = fmin(wcb, t);
    return (4.0 / 3.0 * w - 2.0 / 3.0 * w * w / t + w * w * w / (3.0 * t * t)) / m->x0;
}

/* hard bremsstrahlung attenuation (cm^2/g): integral of dmu/dk on [wcb, T] */
static double mu_brems(const mat_t* m, double t, double wcb) {
    if (t <= wcb) return 0.0;
    double y = wcb / t;
    return (4.0 / 3.0 * log(t / wcb) - 4.0 / 3.0 * (1.0 - y) + 0.5 * (1.0 - y * y)) / m->x0;
}

/* Moller dsigma/deps per electron, eps = W/T of the less energetic electron */
static double dsigma_moller(double t, double eps) {
    double g = 1.0 + t / MC2, b2 = 1.0 - 1.0 / (g * g);
    double c1 = (g - 1.0) / g;
    double c2 = (2.0 * g - 1.0) / (g * g);
    double br = c1 * c1 + 1.0 / eps * (1.0 / eps - c2) + 1.0 / (1.0 - eps) * (1.0 / (1.0 - eps) - c2);
    return 2.0 * PI * RE * RE * MC2 / (b2 * t) * br;
}

/* hard Moller attenuation (cm^2/g): closed-form integral over eps in [wcc/T, 1/2] */
static double mu_moller(const mat_t* m, double t, double wcc) {
    if (t <= 2.0 * wcc) return 0.0;
    double g = 1.0 + t / MC2, b2 = 1.0 - 1.0 / (g * g);
    double e0 = wcc / t;
    double c1 = (g - 1.0) / g;
    double s = c1 * c1 * (0.5 - e0) + 1.0 / e0 - 1.0 / (1.0 - e0) -
               (2.0 * g - 1.0) / (g * g) * log((1.0 - e0) / e0);
    return m->ne * 2.0 * PI * RE * RE * MC2 / (b2 * t) * s;
}

/* inverse transport mean free path per g/cm^2: screened Rutherford with
 * Moliere's screening parameter, Z(Z+1) to include atomic electrons */
static double inv_lambda1(const mat_t* m, double t) {
    double pc2 = t * (t + 2.0 * MC2);
    double g = 1.0 + t / MC2, b2 = 1.0 - 1.0 / (g * g);
    double q = ALPHA * cbrt(m->z) * MC2 / (0.885 * sqrt(pc2));
    double as = 0.25 * q * q * (1.13 + 3.76 * ALPHA * ALPHA * m->z * m->z / b2);
    return NAV / m->a * 2.0 * PI * m->z * (m->z + 1.0) * RE * RE * MC2 * MC2 / (b2 * pc2) *
           (log(1.0 + 1.0 / as) - 1.0 / (1.0 + as));
}

static double s_total(const mat_t* m, double t, double wcc, double wcb) {
    return l_restricted(m, t, wcc) + s_rad_soft(m, t, wcb);
}

/* ---- 8-point Gauss-Legendre nodes, computed by Newton on P_8 ---- */
static double gl_x[8], gl_w[8];
static pthread_once_t gl_once = PTHREAD_ONCE_INIT;

static void gl_init(void) {
    const int n = 8;
    for (int i = 1; i <= n / 2; ++i) {
        double z = cos(PI * (i - 0.25) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        gl_x[i - 1] = -z;
        gl_x[n - i] = z;
        gl_w[i - 1] = gl_w[n - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* integral of dE / S_r(E) from a to b (a <= b), in ln E, split at the kinks
 * of the restricted loss (T = 2 wcc) and of the soft radiative loss (T = wcb) */
static double path_piece(const mat_t* m, double a, double b, double wcc, double wcb) {
    double la = log(a), lb = log(b);
    int np = (int)ceil((lb - la) / 0.1);
    if (np < 1) np = 1;
    double h = (lb - la) / np, sum = 0.0;
    for (int k = 0; k < np; ++k) {
        double c = la + (k + 0.5) * h;
        for (int i = 0; i < 8; ++i) {
            double e = exp(c + 0.5 * h * gl_x[i]);
            sum += gl_w[i] * 0.5 * h * e / s_total(m, e, wcc, wcb);
        }
    }
    return sum;
}

static double path_length(const mat_t* m, double a, double b, double wcc, double wcb) {
    pthread_once(&gl_once, gl_init);
    if (b <= a) return 0.0;
    double cuts[2] = {fmin(wcb, 2.0 * wcc), fmax(wcb, 2.0 * wcc)};
    double sum = 0.0, lo = a;
    for (int i = 0; i < 2; ++i) {
        if (cuts[i] > lo && cuts[i] < b) {
            sum += path_piece(m, lo, cuts[i], wcc, wcb);
            lo = cuts[i];
        }
    }
    return sum + path_piece(m, lo, b, wcc, wcb);
}

/* kinetic energy left after a mass thickness q (g/cm^2) of continuous slowing
 * down from t0: the T' with integral_{T'}^{t0} dE/S_r = q.  lo must satisfy
 * integral_{lo}^{t0} >= q.  Newton on f(x) = integral_x^{t0} - q, f' = -1/S_r,
 * safeguarded by bisection on [lo, t0]. */
static double csda_energy_in(const mat_t* m, double t0, double q, double lo, double wcc,
                             double wcb) {
    if (q <= 0.0) return t0;
    double hi = t0;
    double x = t0 - q * s_total(m, t0, wcc, wcb);
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        double f = path_length(m, x, t0, wcc, wcb) - q; /* decreasing in x */
        if (f > 0.0) lo = x; else hi = x;
        double xn = x + f * s_total(m, x, wcc, wcb);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-15 * x) { x = xn; break; }
        x = xn;
    }
    return x;
}

static double csda_energy(const mat_t* m, double t0, double q, double wcc, double wcb) {
    double lo = 0.5 * t0;
    while (path_length(m, lo, t0, wcc, wcb) < q) {
        lo *= 0.5;
        if (lo < 1e-4) return lo;
    }
    return csda_energy_in(m, t0, q, lo, wcc, wcb);
}

/* ---- modified-Wentzel angular distribution p(mu) = A(1+A)/(mu+A)^2, mu = (1-cos)/2 ---- */
static double mw_mean(double a) {
    if (a > 1e3) { /* series in 1/A: sum_{n>=1} (-1)^(n+1) A^(1-n) / (n(n+1)) */
        double x = 1.0 / a, s = 0.0, p = 1.0;
        for (int n = 1; n <= 8; ++n) {
            s += ((n & 1) ? 1.0 : -1.0) * p / (n * (n + 1.0));
            p *= x;
        }
        return s;
    }
    return a * ((1.0 + a) * log1p(1.0 / a) - 1.0);
}

#define MW_T_ISO 20.0 /* beyond this the deflection is isotropic */

/* screening A with <mu> = (1 - exp(-t))/2, so that <cos> = exp(-t) (Lewis) */
double orc_mw_A(double t) {
    double target = -0.5 * expm1(-t);
    double lo = -90.0, hi = 90.0; /* ln A */
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mw_mean(exp(mid)) < target) lo = mid; else hi = mid;
        if (hi - lo < 1e-15) break;
    }
    return exp(0.5 * (lo + hi));
}

static double sample_mw(double t, stream_t* s) {
    double u = draw(s);
    if (t >= MW_T_ISO) return u;
    double a = orc_mw_A(t);
    return a * u / (1.0 + a - u);
}

/* ======================================================================== */
/* Geometry helpers                                                          */
/* ======================================================================== */

/* turn direction d by polar (cos, sin) and azimuth phi */
static void rotate(double d[3], double ct, double st, double phi) {
    double cp = cos(phi), sp = sin(phi);
    double u = d[0], v = d[1], w = d[2];
    double r2 = u * u + v * v;
    if (r2 > 1e-12) {
        double r = sqrt(r2);
        d[0] = u * ct + st * (u * w * cp - v * sp) / r;
        d[1] = v * ct + st * (v * w * cp + u * sp) / r;
        d[2] = w * ct - st * cp * r;
    } else {
        d[0] = st * cp;
        d[1] = st * sp;
        d[2] = (w >= 0.0 ? 1.0 : -1.0) * ct;
    }
}

/* ======================================================================== */
/* Run context                                                               */
/* ======================================================================== */

typedef struct {
    int type;  /* 0 photon, 1 electron, 2 positron */
    double x[3], d[3];
    double e;  /* kinetic energy */
    double a;  /* positron: energy of its annihilation photons together */
    double nh; /* hard-event mean free paths left */
    int nh_set;
    int iv[3]; /* electron voxel */
    stream_t s;
    double wt; /* statistical weight (1, or 2^-k for a split primary and its secondaries) */
} particle_t;

typedef struct {
    const orc_phantom* ph;
    int n_mat;
    mat_t* mats;
    double rho_max[256];
    int present[256];
    double d[3], len[3];
    int n[3];
    const orc_source* src;
    double* cdf;      /* nf + 1 cumulative beamlet probabilities */
    int* beam_of;     /* beamlet -> beam */
    int* beam_off;    /* first global beamlet of each beam */
    int nf;
    double* spec_c;   /* cumulative spectrum at spec_e */
    double* f;        /* beamlet intensities (negative ones as 0) */
    double* strata_F; /* spectrum CDF at the K + 1 interval edges (stratified spectra) */
    double* strata_e; /* the K + 1 interval edges (MeV) */
    int* metro_bl;    /* Metropolis mode: beamlet of history metro_h0 + i */
    uint64_t metro_h0;
    orc_params prm;
} ctx_t;

typedef struct {
    particle_t* st;
    int n, cap;
    double* tally;
    double e_in, e_esc, h_dep, h_esc;
    uint64_t ev[8];
    uint64_t n_type[ORC_NTYPES];   /* choices made, by type */
    double p_type[ORC_NTYPES];     /* sum of each type's probability over the choices */
    double v_type[ORC_NTYPES];     /* sum of p (1 - p) over the choices */
    uint32_t h_hard;               /* real hard events of the running history */
    double wt;                     /* statistical weight of the particle being tracked */
} work_t;

/* record one choice among `n` types (probabilities p[0..n-1], summing to 1)
 * that picked `chosen`; `first` is the index of p[0] among ORC_TYPE_* */
static void count_choice(work_t* w, int first, int n, const double* p, int chosen) {
    w->n_type[first + chosen]++;
    for (int i = 0; i < n; ++i) {
        w->p_type[first + i] += p[i];
        w->v_type[first + i] += p[i] * (1.0 - p[i]);
    }
}

static void push(work_t* w, const particle_t* p) {
    if (w->n == w->cap) {
        w->cap = w->cap ? 2 * w->cap : 64;
        w->st = (particle_t*)realloc(w->st, (size_t)w->cap * sizeof(particle_t));
    }
    w->st[w->n] = *p;
    w->st[w->n].wt = w->wt;   /* a particle's secondaries carry its weight */
    w->n++;
    w->ev[ORC_EV_PUSHES]++;
}

/* energy deposited and escaping, both scaled by the particle's weight */
static void deposit(work_t* w, int v, double e) {
    if (e <= 0.0) return;
    w->tally[v] += e * w->wt;
    w->h_dep += e * w->wt;
    w->ev[ORC_EV_DEPOSITS]++;
}

static void escape(work_t* w, double e) {
    w->e_esc += e * w->wt;
    w->h_esc += e * w->wt;
}

static int vox_of(const ctx_t* c, const double x[3], int iv[3]) {
    for (int i = 0; i < 3; ++i) {
        int k = (int)floor(x[i] / c->d[i]);
        if (k < 0) k = 0;
        if (k > c->n[i] - 1) k = c->n[i] - 1;
        iv[i] = k;
    }
    return iv[0] + c->n[0] * (iv[1] + c->n[1] * iv[2]);
}

static int lin(const ctx_t* c, const int iv[3]) {
    return iv[0] + c->n[0] * (iv[1] + c->n[1] * iv[2]);
}

static int outside(const ctx_t* c, const double x[3]) {
    for (int i = 0; i < 3; ++i)
        if (x[i] < 0.0 || x[i] >= c->len[i]) return 1;
    return 0;
}

/* photon mass attenuation coefficients of material m with the test switches */
static void photon_mus(const ctx_t* c, int m, double e, double* mc, double* mp, double* mq) {
    uint32_t f = c->prm.flags;
    *mc = (f & ORC_NO_COMPTON) ? 0.0 : mu_compton(&c->mats[m], e);
    *mp = (f & ORC_NO_PHOTO) ? 0.0 : mu_photo(&c->mats[m], e);
    *mq = (f & ORC_NO_PAIR) ? 0.0 : mu_pair(&c->mats[m], e);
}

/* Woodcock majorant: max over the materials present of mu_m(E) times their largest density */
static double mu_max(const ctx_t* c, double e) {
    double best = 0.0;
    for (int m = 0; m < c->n_mat; ++m) {
        if (!c->present[m]) continue;
        double a, b, q;
        photon_mus(c, m, e, &a, &b, &q);
        double v = c->rho_max[m] * (a + b + q);
        if (v > best) best = v;
    }
    return best;
}

static double muh_moller(const ctx_t* c, int m, double t) {
    return (c->prm.flags & ORC_NO_MOLLER) ? 0.0 : mu_moller(&c->mats[m], t, c->prm.ecut_e);
}

static double muh_brems(const ctx_t* c, int m, double t) {
    return (c->prm.flags & ORC_NO_BREMS) ? 0.0 : mu_brems(&c->mats[m], t, c->prm.ecut_g);
}

/* two photons of a/2, back to back, isotropic, at x: draws cos then phi */
static void annihilate(work_t* w, particle_t* parent, const double x[3], double a, int word0) {
    double ct = 2.0 * draw(&parent->s) - 1.0;
    double phi = 2.0 * PI * draw(&parent->s);
    double st = sqrt((1.0 - ct) * (1.0 + ct));
    double dir[3] = {st * cos(phi), st * sin(phi), ct};
    for (int k = 0; k < 2; ++k) {
        particle_t g;
        memset(&g, 0, sizeof g);
        g.type = 0;
        memcpy(g.x, x, sizeof g.x);
        for (int i = 0; i < 3; ++i) g.d[i] = k == 0 ? dir[i] : -dir[i];
        g.e = 0.5 * a;
        g.s = spawn(&parent->s, word0 + k);
        push(w, &g);
    }
}

static void make_charged(particle_t* q, int type, const particle_t* parent, const double dir[3],
                         double t, double a, const int iv[3], int word) {
    memset(q, 0, sizeof *q);
    q->type = type;
    memcpy(q->x, parent->x, sizeof q->x);
    memcpy(q->d, dir, sizeof q->d);
    q->e = t;
    q->a = a;
    q->nh_set = 0;
    memcpy(q->iv, iv, sizeof q->iv);
    q->s = spawn(&parent->s, word);
}

/* ======================================================================== */
/* Photon transport                                                          */
/* ======================================================================== */

/* Klein-Nishina in eps = E'/E on [1/(1+2k), 1] (free electron): density
 * proportional to 1/x + x - t(2 - t) with t = (1/x - 1)/k = 1 - cos(theta);
 * kn_cum is its antiderivative, written out term by term:
 * ln x + x^2/2 - (2/k)(ln x - x) + (-1/x - 2 ln x + x)/k^2 */
static double kn_density(double x, double k) {
    double t = (1.0 / x - 1.0) / k;
    return 1.0 / x + x - t * (2.0 - t);
}

static double kn_cum(double x, double k) {
    double l = log(x);
    return l + 0.5 * x * x - 2.0 / k * (l - x) + (-1.0 / x - 2.0 * l + x) / (k * k);
}

/* eps with F(eps) = u, F the normalised Klein-Nishina distribution function:
 * Newton steps kept inside a shrinking bracket (bisection where a step would
 * leave it), from the log-uniform guess e0^(1 - u), to full double precision */
static double kn_inverse(double k, double u) {
    double e0 = 1.0 / (1.0 + 2.0 * k);
    double g0 = kn_cum(e0, k), span = kn_cum(1.0, k) - g0;
    double lo = e0, hi = 1.0, x = pow(e0, 1.0 - u);
    for (int it = 0; it < 200; ++it) {
        double f = (kn_cum(x, k) - g0) / span - u;
        if (f > 0.0) hi = x;
        else lo = x;
        double xn = x - f * span / kn_density(x, k);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-15 * x || hi - lo <= 1e-15 * x) return xn;
        x = xn;
    }
    return x;
}

/* Compton scattering of photon p (section 2.1's photon physics, read as
 * free-electron Klein-Nishina): eps = E'/E by inversion of the distribution
 * function at one uniform draw, then an azimuth; the photon turned and left
 * with E' = eps E; the electron takes T = E - E' along E d0 - E' d (momentum
 * conservation). */
static void compton(particle_t* p, double* te, double de[3]) {
    double k = p->e / MC2;
    double eps = kn_inverse(k, draw(&p->s));
    double t = (1.0 - eps) / (k * eps);
    double phi = 2.0 * PI * draw(&p->s);
    double d0[3] = {p->d[0], p->d[1], p->d[2]};
    rotate(p->d, 1.0 - t, sqrt(fmax(0.0, t * (2.0 - t))), phi);
    double e1 = eps * p->e;
    *te = p->e - e1;
    double nn = 0.0;
    for (int i = 0; i < 3; ++i) {
        de[i] = p->e * d0[i] - e1 * p->d[i];
        nn += de[i] * de[i];
    }
    nn = sqrt(nn);
    for (int i = 0; i < 3; ++i) de[i] = nn > 0.0 ? de[i] / nn : d0[i];
    p->e = e1;
}

/* pair production by photon p: the kinetic energy K = E - 2 mc^2 split
 * uniformly (T- = u K, T+ = K - T-); the positron keeps its annihilation
 * energy a = E - K */
static void pair_split(particle_t* p, double* tm, double* tp, double* a) {
    double kk = p->e - 2.0 * MC2;
    *a = p->e - kk;
    *tm = draw(&p->s) * kk;
    *tp = kk - *tm;
}

static void track_photon(ctx_t* c, work_t* w, particle_t* p) {
    const double ecut_g = c->prm.ecut_g, ecut_e = c->prm.ecut_e;
    const int kerma = (c->prm.flags & ORC_KERMA) != 0;
    for (;;) {
        int iv[3];
        if (p->e < ecut_g) {
            deposit(w, vox_of(c, p->x, iv), p->e);
            return;
        }
        /* free flight against the majorant */
        double mmax = mu_max(c, p->e);
        double s = -log(draw(&p->s)) / mmax;
        w->ev[ORC_EV_FLIGHTS]++;
        for (int i = 0; i < 3; ++i) p->x[i] += s * p->d[i];
        if (outside(c, p->x)) {
            escape(w, p->e);
            return;
        }
        int v = vox_of(c, p->x, iv);
        int m = c->ph->mat[v];
        double rho = c->ph->rho[v];
        double mc, mp, mq;
        photon_mus(c, m, p->e, &mc, &mp, &mq);
        double mt = mc + mp + mq;
        /* real with probability rho mu / mu_max, else fictitious */
        const int real = draw(&p->s) * mmax < rho * mt;
        const double pr[2] = {rho * mt / mmax, 1.0 - rho * mt / mmax};
        count_choice(w, ORC_TYPE_FLIGHT_REAL, 2, pr, real ? 0 : 1);
        if (!real) continue;
        w->ev[ORC_EV_REAL]++;
        /* the interaction: Compton, photoelectric or pair with probabilities mu_i / mu */
        double r = draw(&p->s) * mt;
        int type = r < mc ? 0 : (r < mc + mp ? 1 : 2);
        const double pt[3] = {mc / mt, mp / mt, mq / mt};
        count_choice(w, ORC_TYPE_COMPTON, 3, pt, type);
        if (type == 0) {
            double te, de[3];
            compton(p, &te, de);
            if (kerma || te <= ecut_e) deposit(w, v, te);
            else {
                particle_t q;
                make_charged(&q, 1, p, de, te, 0.0, iv, 0);
                push(w, &q);
            }
        } else if (type == 1) {
            /* photoelectric: the electron takes all the energy, along the photon */
            if (kerma || p->e <= ecut_e) deposit(w, v, p->e);
            else {
                particle_t q;
                make_charged(&q, 1, p, p->d, p->e, 0.0, iv, 0);
                push(w, &q);
            }
            return;
        } else {
            /* pair: both particles along the photon */
            double tm, tp, a;
            pair_split(p, &tm, &tp, &a);
            int pos_local = kerma || tp <= ecut_e;
            double ct = 0.0, phi = 0.0;
            if (pos_local) {
                ct = 2.0 * draw(&p->s) - 1.0;
                phi = 2.0 * PI * draw(&p->s);
            }
            if (kerma || tm <= ecut_e) deposit(w, v, tm);
            else {
                particle_t q;
                make_charged(&q, 1, p, p->d, tm, 0.0, iv, 0);
                push(w, &q);
            }
            if (pos_local) {
                deposit(w, v, tp);
                double st = sqrt((1.0 - ct) * (1.0 + ct));
                double dir[3] = {st * cos(phi), st * sin(phi), ct};
                for (int kq = 0; kq < 2; ++kq) {
                    particle_t g;
                    memset(&g, 0, sizeof g);
                    memcpy(g.x, p->x, sizeof g.x);
                    for (int i = 0; i < 3; ++i) g.d[i] = kq == 0 ? dir[i] : -dir[i];
                    g.e = 0.5 * a;
                    g.s = spawn(&p->s, 2 + kq);
                    push(w, &g);
                }
            } else {
                particle_t q;
                make_charged(&q, 2, p, p->d, tp, a, iv, 1);
                push(w, &q);
            }
            return;
        }
    }
}

/* ======================================================================== */
/* Electron / positron transport: class II, random hinge, voxel-limited      */
/* ======================================================================== */

static double face_dist(const ctx_t* c, const particle_t* p, int* axis) {
    double best = INFINITY;
    int ax = 0;
    for (int i = 0; i < 3; ++i) {
        double di;
        if (p->d[i] > 0.0) di = ((p->iv[i] + 1) * c->d[i] - p->x[i]) / p->d[i];
        else if (p->d[i] < 0.0) di = (p->iv[i] * c->d[i] - p->x[i]) / p->d[i];
        else continue;
        if (di < best) {
            best = di;
            ax = i;
        }
    }
    *axis = ax;
    return best < 0.0 ? 0.0 : best;
}

/* place the particle on the face it reached and step its voxel; 1 if it left the grid */
static int cross_face(const ctx_t* c, particle_t* p, int ax) {
    int step = p->d[ax] > 0.0 ? 1 : -1;
    p->x[ax] = (step > 0 ? p->iv[ax] + 1 : p->iv[ax]) * c->d[ax];
    p->iv[ax] += step;
    return p->iv[ax] < 0 || p->iv[ax] >= c->n[ax];
}

static void move(particle_t* p, double s) {
    for (int i = 0; i < 3; ++i) p->x[i] += s * p->d[i];
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

static void moller(ctx_t* c, work_t* w, particle_t* p, int v) {
    double t = p->e, wcc = c->prm.ecut_e;
    double g = 1.0 + t / MC2, e0 = wcc / t;
    double c1 = (g - 1.0) / g, c2 = (2.0 * g - 1.0) / (g * g);
    double eps;
    for (;;) {
        double ua = draw(&p->s);
        eps = e0 / (1.0 - ua * (1.0 - 2.0 * e0)); /* proposal ~ 1/eps^2 on [e0, 1/2] */
        double ub = draw(&p->s);
        double br = c1 * c1 + 1.0 / eps * (1.0 / eps - c2) + 1.0 / (1.0 - eps) * (1.0 / (1.0 - eps) - c2);
        if (ub * 2.25 <= eps * eps * br) break;
    }
    double phi = 2.0 * PI * draw(&p->s);
    double wd = eps * t, tp = t - wd;
    double cd = sqrt(wd * (t + 2.0 * MC2) / (t * (wd + 2.0 * MC2)));
    double cpr = sqrt(tp * (t + 2.0 * MC2) / (t * (tp + 2.0 * MC2)));
    double dd[3] = {p->d[0], p->d[1], p->d[2]};
    rotate(dd, cd, sqrt(fmax(0.0, 1.0 - cd * cd)), phi);
    rotate(p->d, cpr, sqrt(fmax(0.0, 1.0 - cpr * cpr)), phi + PI);
    if (wd <= c->prm.ecut_e) deposit(w, v, wd);
    else {
        particle_t q;
        make_charged(&q, 1, p, dd, wd, 0.0, p->iv, 0);
        push(w, &q);
    }
    p->e = tp;
}

static void brems(ctx_t* c, work_t* w, particle_t* p) {
    double t = p->e, wcb = c->prm.ecut_g, k;
    for (;;) {
        double ua = draw(&p->s);
        k = wcb * pow(t / wcb, ua); /* proposal ~ 1/k on [wcb, T] */
        double ub = draw(&p->s);
        double y = k / t;
        if (ub * (4.0 / 3.0) <= 4.0 / 3.0 - 4.0 / 3.0 * y + y * y) break;
    }
    particle_t g;
    memset(&g, 0, sizeof g);
    memcpy(g.x, p->x, sizeof g.x);
    memcpy(g.d, p->d, sizeof g.d);
    g.e = k;
    g.s = spawn(&p->s, 0);
    push(w, &g);
    p->e = t - k;
}

static void track_electron(ctx_t* c, work_t* w, particle_t* p) {
    const double ecut_e = c->prm.ecut_e, wcc = c->prm.ecut_e, wcb = c->prm.ecut_g;
    for (;;) {
        int v = lin(c, p->iv);
        if (p->e <= ecut_e) {
            deposit(w, v, p->e);
            if (p->type == 2) annihilate(w, p, p->x, p->a, 0);
            return;
        }
        int m = c->ph->mat[v];
        double rho = c->ph->rho[v];
        const mat_t* mt = &c->mats[m];
        if (!p->nh_set) {
            p->nh = -log(draw(&p->s));
            p->nh_set = 1;
        }
        w->ev[ORC_EV_ESTEPS]++;
        double t0 = p->e;
        double muh0 = muh_moller(c, m, t0) + muh_brems(c, m, t0);
        double mus = rho * muh0;
        double sh = mus > 0.0 ? p->nh / mus : INFINITY;
        double tfl = fmax(0.75 * t0, ecut_e);
        double se = path_length(mt, tfl, t0, wcc, wcb) / rho;
        int hard = sh < se;
        double s = hard ? sh : se;
        double xi = draw(&p->s);
        double s1 = xi * s, s2 = s - s1;
        double tend = hard ? clampd(csda_energy_in(mt, t0, rho * s, tfl, wcc, wcb), tfl, t0) : tfl;
        int ax;
        /* segment 1 */
        double db = face_dist(c, p, &ax);
        if (db < s1) {
            move(p, db);
            double t1 = clampd(csda_energy_in(mt, t0, rho * db, tfl, wcc, wcb), tend, p->e);
            deposit(w, v, p->e - t1);
            p->e = t1;
            p->nh -= mus * db;
            if (cross_face(c, p, ax)) {
                escape(w, p->e + (p->type == 2 ? p->a : 0.0));
                return;
            }
            continue;
        }
        move(p, s1);
        double t1 = clampd(csda_energy_in(mt, t0, rho * s1, tfl, wcc, wcb), tend, p->e);
        deposit(w, v, p->e - t1);
        p->e = t1;
        /* hinge */
        if (!(c->prm.flags & ORC_NO_MS)) {
            double tmid = 0.5 * (t0 + tend);
            double tt = s * rho * inv_lambda1(mt, tmid);
            double mu = sample_mw(tt, &p->s);
            double phi = 2.0 * PI * draw(&p->s);
            rotate(p->d, 1.0 - 2.0 * mu, 2.0 * sqrt(mu * (1.0 - mu)), phi);
        }
        /* segment 2 */
        db = face_dist(c, p, &ax);
        if (db < s2) {
            move(p, db);
            double t2 = clampd(csda_energy_in(mt, t0, rho * (s1 + db), tfl, wcc, wcb), tend, p->e);
            deposit(w, v, p->e - t2);
            p->e = t2;
            p->nh -= mus * (s1 + db);
            if (cross_face(c, p, ax)) {
                escape(w, p->e + (p->type == 2 ? p->a : 0.0));
                return;
            }
            continue;
        }
        move(p, s2);
        deposit(w, v, p->e - tend);
        p->e = tend;
        if (hard) {
            /* delta scattering against the step-start majorant; mu_h grows with T */
            w->ev[ORC_EV_HARD_CAND]++;
            double mm = muh_moller(c, m, tend);
            double muh1 = mm + muh_brems(c, m, tend);
            const int accept = draw(&p->s) * muh0 < muh1;
            const double pa[2] = {muh1 / muh0, 1.0 - muh1 / muh0};
            count_choice(w, ORC_TYPE_HARD_REAL, 2, pa, accept ? 0 : 1);
            if (accept) {
                w->ev[ORC_EV_HARD]++;
                w->h_hard++;
                /* Moller with probability mu_Moller / mu_hard, else bremsstrahlung */
                const int type = draw(&p->s) * muh1 < mm ? 0 : 1;
                const double pm[2] = {mm / muh1, 1.0 - mm / muh1};
                count_choice(w, ORC_TYPE_MOLLER, 2, pm, type);
                if (type == 0) moller(c, w, p, v);
                else brems(c, w, p);
            }
            p->nh_set = 0;
        } else {
            p->nh -= mus * s;
        }
    }
}

/* ======================================================================== */
/* Source                                                                     */
/* ======================================================================== */

static double spectrum_energy(const ctx_t* c, double u) {
    const orc_source* s = c->src;
    if (s->spec_kind == 0) return s->e_mono;
    int n = s->spec_n;
    double r = u * c->spec_c[n - 1];
    int j = 0;
    while (j < n - 2 && c->spec_c[j + 1] <= r) ++j;
    double p0 = s->spec_p[j];
    double sl = (s->spec_p[j + 1] - s->spec_p[j]) / (s->spec_e[j + 1] - s->spec_e[j]);
    double d = r - c->spec_c[j];
    double den = p0 + sqrt(fmax(0.0, p0 * p0 + 2.0 * sl * d));
    double x = den > 0.0 ? 2.0 * d / den : 0.0;
    return clampd(s->spec_e[j] + x, s->spec_e[j], s->spec_e[j + 1]);
}

/* spectrum CDF F(e), the area of the piecewise-linear pdf below e over its total */
static double spectrum_cdf(const ctx_t* c, double e) {
    const orc_source* s = c->src;
    int n = s->spec_n;
    if (e <= s->spec_e[0]) return 0.0;
    if (e >= s->spec_e[n - 1]) return 1.0;
    int j = 0;
    while (j < n - 2 && s->spec_e[j + 1] <= e) ++j;
    double t = (e - s->spec_e[j]) / (s->spec_e[j + 1] - s->spec_e[j]);
    double pe = s->spec_p[j] + t * (s->spec_p[j + 1] - s->spec_p[j]);
    return (c->spec_c[j] + 0.5 * (s->spec_p[j] + pe) * (e - s->spec_e[j])) / c->spec_c[n - 1];
}

/* section 2.3.2: the K energy intervals of equal width over the support */
static void strata_setup(ctx_t* c) {
    const orc_source* s = c->src;
    int K = s->spectrum_strata;
    c->strata_F = (double*)malloc(sizeof(double) * (K + 1));
    c->strata_e = (double*)malloc(sizeof(double) * (K + 1));
    double e0 = s->spec_e[0], e1 = s->spec_e[s->spec_n - 1];
    for (int k = 0; k <= K; ++k) {
        c->strata_e[k] = e0 + (e1 - e0) * k / K;
        c->strata_F[k] = spectrum_cdf(c, c->strata_e[k]);
    }
    c->strata_F[0] = 0.0;
    c->strata_F[K] = 1.0;
    c->strata_e[K] = e1;
}

/* energy of history h in a stratified run: its position i in its round of R
 * histories picks the interval k with C_k <= i < C_{k+1}, C_k = floor(R F_k +
 * 1/2) (the round's histories shared among the intervals by the spectrum, in
 * increasing energy); inside the interval the energy is uniform, e_k + u
 * (e_{k+1} - e_k) (the paper's rule), or, with strata_shape 1, the spectrum's
 * inverse CDF at F_k + u (F_{k+1} - F_k) */
static double stratified_energy(const ctx_t* c, uint64_t h, double u) {
    uint64_t off = h - c->prm.hist0, R = c->prm.round_size, N = c->prm.n_hist;
    uint64_t a = off / R * R, b = a + R < N ? a + R : N;
    double i = (double)(off - a), size = (double)(b - a);
    int K = c->src->spectrum_strata, k = 0;
    while (k < K - 1 && floor(size * c->strata_F[k + 1] + 0.5) <= i) ++k;
    if (c->src->strata_shape == 0)
        return c->strata_e[k] + u * (c->strata_e[k + 1] - c->strata_e[k]);
    return spectrum_energy(c, c->strata_F[k] + u * (c->strata_F[k + 1] - c->strata_F[k]));
}

/* beamlet I with P(I) <= r < P(I+1), by bisection on the cumulative array */
static int beamlet_search(const ctx_t* c, double r) {
    int lo = 0, hi = c->nf; /* P[lo] <= r < P[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (c->cdf[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

/* Algorithm A1 (section 2.3.1), Metropolis sampling of the beamlet index,
 * for histories h0 .. h0+n-1.  The histories form ORC_METRO_CHAINS chains,
 * history h on chain h mod ORC_METRO_CHAINS, each taken in increasing h.  A
 * chain starts at a beamlet drawn with equal probability among those of
 * nonzero intensity, from a stream of its own (history id (2^32-1)*2^32 +
 * chain, path 0, a history id no run reaches).  At history h, after the draw
 * of the energy, h's stream gives the trial beamlet J (equal probability among
 * nonzero beamlets) and r; the chain moves to J when r < f_J / f_prev, tested
 * as r f_prev < f_J, exact in double precision. */
static int metropolis_chains(ctx_t* c, uint64_t h0, uint64_t n) {
    int n_nz = 0;
    for (int i = 0; i < c->nf; ++i) n_nz += c->f[i] > 0.0;
    if (n_nz == 0) return 1;
    int* nz = (int*)malloc(sizeof(int) * n_nz);
    for (int i = 0, k = 0; i < c->nf; ++i)
        if (c->f[i] > 0.0) nz[k++] = i;
    c->metro_bl = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    c->metro_h0 = h0;
    const uint64_t C = ORC_METRO_CHAINS;
    for (uint64_t ch = 0; ch < C; ++ch) {
        stream_t s0 = stream_make(c->prm.seed, c->prm.job_id, (0xFFFFFFFFull << 32) | ch, 0);
        int prev = nz[(int)floor(draw(&s0) * n_nz)];
        for (uint64_t h = h0 + (ch + C - h0 % C) % C; h < h0 + n; h += C) {
            stream_t s = stream_make(c->prm.seed, c->prm.job_id, h, 0);
            (void)draw(&s);   /* the energy's draw */
            int J = nz[(int)floor(draw(&s) * n_nz)];
            double r = draw(&s);
            int I = r * c->f[prev] < c->f[J] ? J : prev;
            c->metro_bl[h - h0] = I;
            prev = I;
        }
    }
    free(nz);
    return 0;
}

/* section 2.3.3: history h starts as phase-space record h mod n_phsp, inside
 * the phantom where it is, outside at the point where its forward ray enters
 * the phantom (none: the particle escapes); the record number is reported in
 * place of a beamlet */
static int phase_space_particle(const ctx_t* c, uint64_t h, particle_t* p, int* beamlet) {
    const orc_source* s = c->src;
    uint64_t k = h % s->n_phsp;
    const float* r = s->phsp + 7 * k;
    *beamlet = (int)k;
    p->e = r[6];
    double o[3] = {r[0], r[1], r[2]};
    for (int i = 0; i < 3; ++i) p->d[i] = r[3 + i];
    int inside = 1;
    for (int i = 0; i < 3; ++i)
        if (!(o[i] >= 0.0 && o[i] < c->len[i])) inside = 0;
    if (inside) {
        for (int i = 0; i < 3; ++i) p->x[i] = o[i];
        vox_of(c, p->x, p->iv);
        return 1;
    }
    double tmin = 0.0, tmax = INFINITY;
    int ax = -1;
    for (int i = 0; i < 3; ++i) {
        if (p->d[i] != 0.0) {
            double ta = (0.0 - o[i]) / p->d[i], tb = (c->len[i] - o[i]) / p->d[i];
            double tn = fmin(ta, tb), tf = fmax(ta, tb);
            if (tn > tmin) {
                tmin = tn;
                ax = i;
            }
            if (tf < tmax) tmax = tf;
        } else if (o[i] < 0.0 || o[i] > c->len[i]) {
            return 0;
        }
    }
    if (!(tmax > tmin)) return 0;
    for (int i = 0; i < 3; ++i) p->x[i] = o[i] + tmin * p->d[i];
    if (ax >= 0) p->x[ax] = p->d[ax] > 0.0 ? 0.0 : c->len[ax];
    vox_of(c, p->x, p->iv);
    return 1;
}

/* sample the primary of history h; returns 1 if it enters the phantom */
static int source_particle(const ctx_t* c, uint64_t h, particle_t* p, int* beamlet) {
    const orc_source* s = c->src;
    memset(p, 0, sizeof *p);
    p->s = stream_make(c->prm.seed, c->prm.job_id, h, 0);
    p->type = s->particle == 0 ? 0 : 1;
    if (s->n_phsp) return phase_space_particle(c, h, p, beamlet);
    p->e = c->strata_F ? stratified_energy(c, h, draw(&p->s)) : spectrum_energy(c, draw(&p->s));
    int gi;
    if (c->metro_bl) {
        (void)draw(&p->s);   /* J and r of the chain step */
        (void)draw(&p->s);
        gi = c->metro_bl[h - c->metro_h0];
    } else {
        gi = beamlet_search(c, draw(&p->s));
    }
    double ux = draw(&p->s), uy = draw(&p->s);
    *beamlet = gi;
    int b = c->beam_of[gi];
    const orc_beam* bm = &s->beams[b];
    int j = gi - c->beam_off[b];
    int jx = j % bm->nbx, jy = j / bm->nbx;
    double px = (jx + ux) * bm->bw - 0.5 * bm->nbx * bm->bw;
    double py = (jy + uy) * bm->bh - 0.5 * bm->nby * bm->bh;
    double e2[3] = {bm->dir[1] * bm->e1[2] - bm->dir[2] * bm->e1[1],
                    bm->dir[2] * bm->e1[0] - bm->dir[0] * bm->e1[2],
                    bm->dir[0] * bm->e1[1] - bm->dir[1] * bm->e1[0]};
    double pt[3], o[3], tlo;
    for (int i = 0; i < 3; ++i) pt[i] = bm->iso[i] + px * bm->e1[i] + py * e2[i];
    if (bm->sad > 0.0) {
        double nn = 0.0;
        for (int i = 0; i < 3; ++i) {
            o[i] = bm->iso[i] - bm->sad * bm->dir[i];
            p->d[i] = pt[i] - o[i];
            nn += p->d[i] * p->d[i];
        }
        nn = sqrt(nn);
        for (int i = 0; i < 3; ++i) p->d[i] /= nn;
        tlo = 0.0;
    } else {
        for (int i = 0; i < 3; ++i) {
            o[i] = pt[i];
            p->d[i] = bm->dir[i];
        }
        tlo = -INFINITY;
    }
    /* slab-method ray-box entry */
    double tmin = tlo, tmax = INFINITY;
    int ax = -1;
    for (int i = 0; i < 3; ++i) {
        if (p->d[i] != 0.0) {
            double ta = (0.0 - o[i]) / p->d[i], tb = (c->len[i] - o[i]) / p->d[i];
            double tn = fmin(ta, tb), tf = fmax(ta, tb);
            if (tn > tmin) {
                tmin = tn;
                ax = i;
            }
            if (tf < tmax) tmax = tf;
        } else if (o[i] < 0.0 || o[i] > c->len[i]) {
            return 0;
        }
    }
    if (!(tmax > tmin)) return 0;
    for (int i = 0; i < 3; ++i) p->x[i] = o[i] + tmin * p->d[i];
    if (ax >= 0) p->x[ax] = p->d[ax] > 0.0 ? 0.0 : c->len[ax];
    vox_of(c, p->x, p->iv);
    return 1;
}

/* ======================================================================== */
/* Runs: histories split over threads, tallies merged in a fixed order        */
/* ======================================================================== */

typedef struct {
    ctx_t* c;
    work_t w;
    uint64_t h0, h1;
    double* hist_out;
    uint32_t* hist_hard;
} job_t;

static void run_history(ctx_t* c, work_t* w, uint64_t h, double* hist_out, uint32_t* hist_hard) {
    particle_t p;
    int beamlet;
    w->h_dep = w->h_esc = 0.0;
    w->h_hard = 0;
    w->ev[ORC_EV_HISTORIES]++;
    int in = source_particle(c, h, &p, &beamlet);
    w->e_in += p.e;
    w->wt = 1.0;
    if (!in) {
        escape(w, p.e);
    } else {
        /* primary splitting: S = 2^k copies of the source particle, each of
         * weight 1/S; copy i continues on stream path i at the draw after the
         * source's (copy 0 is the unsplit primary) */
        const int S = 1 << c->prm.split_log2;
        w->n = 0;
        w->wt = 1.0 / S;
        for (int i = S - 1; i >= 0; --i) {
            particle_t q = p;
            q.s.path = (uint32_t)i;
            w->ev[ORC_EV_PUSHES]--; /* the primaries are not secondaries */
            push(w, &q);
        }
        while (w->n > 0) {
            particle_t q = w->st[--w->n];
            w->wt = q.wt;
            if (q.type == 0) track_photon(c, w, &q);
            else track_electron(c, w, &q);
        }
    }
    if (hist_out) {
        uint64_t i = h - c->prm.hist0;
        hist_out[2 * i] = w->h_dep;
        hist_out[2 * i + 1] = w->h_esc;
    }
    if (hist_hard) hist_hard[h - c->prm.hist0] = w->h_hard;
}

static void* thread_main(void* arg) {
    job_t* j = (job_t*)arg;
    for (uint64_t h = j->h0; h < j->h1; ++h) run_history(j->c, &j->w, h, j->hist_out, j->hist_hard);
    return NULL;
}

static int validate(const orc_material* mats, int n_mat, const orc_phantom* ph,
                    const orc_source* src, const orc_params* prm) {
    if (!mats || n_mat < 1 || n_mat > 256 || !ph || !src || !prm) return 1;
    if (ph->nx < 1 || ph->ny < 1 || ph->nz < 1) return 1;
    if (!(ph->dx > 0) || !(ph->dy > 0) || !(ph->dz > 0) || !ph->mat || !ph->rho) return 1;
    size_t nv = (size_t)ph->nx * ph->ny * ph->nz;
    for (size_t v = 0; v < nv; ++v)
        if (ph->mat[v] >= n_mat || !(ph->rho[v] > 0.0f)) return 1;
    if (src->n_phsp > 0) {
        if (!src->phsp) return 1;
        for (uint64_t k = 0; k < src->n_phsp; ++k) {
            const float* r = src->phsp + 7 * k;
            double nn = (double)r[3] * r[3] + (double)r[4] * r[4] + (double)r[5] * r[5];
            if (!(r[6] > 0.0f) || !(fabs(nn - 1.0) < 1e-5) || !isfinite(r[0]) || !isfinite(r[1]) ||
                !isfinite(r[2]))
                return 1;
        }
    } else {
        if (src->n_beams < 1 || !src->beams) return 1;
        if (src->beamlet_sampler != 0 && src->beamlet_sampler != 1) return 1;
        if (src->spectrum_strata < 0 || src->spectrum_strata > 64) return 1;
        if (src->spectrum_strata > 0 && src->spec_kind != 1) return 1;
        if (src->strata_shape != 0 && src->strata_shape != 1) return 1;
        if (src->spec_kind == 0 && !(src->e_mono > 0)) return 1;
        if (src->spec_kind == 1 && (src->spec_n < 2 || !src->spec_e || !src->spec_p)) return 1;
    }
    if (prm->n_batches < 1 || prm->round_size < 1) return 1;
    if (prm->split_log2 < 0 || prm->split_log2 > 6) return 1;
    if (src->particle == 1 && (prm->flags & ORC_KERMA)) return 1;
    return 0;
}

int orc_run(const orc_material* mats, int n_mat, const orc_phantom* ph, const orc_source* src,
            const orc_params* prm, double* batch_edep, double* dose, double* sigma,
            double* hist_out, uint32_t* hist_hard, orc_stats* st) {
    if (validate(mats, n_mat, ph, src, prm)) return 1;
    pthread_once(&gl_once, gl_init);
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.ph = ph;
    c.n_mat = n_mat;
    c.src = src;
    c.prm = *prm;
    c.mats = (mat_t*)malloc(sizeof(mat_t) * n_mat);
    for (int m = 0; m < n_mat; ++m) c.mats[m] = mat_make(&mats[m]);
    c.n[0] = ph->nx; c.n[1] = ph->ny; c.n[2] = ph->nz;
    c.d[0] = ph->dx; c.d[1] = ph->dy; c.d[2] = ph->dz;
    for (int i = 0; i < 3; ++i) c.len[i] = c.n[i] * c.d[i];
    size_t nv = (size_t)ph->nx * ph->ny * ph->nz;
    for (size_t v = 0; v < nv; ++v) {
        int m = ph->mat[v];
        c.present[m] = 1;
        if (ph->rho[v] > c.rho_max[m]) c.rho_max[m] = ph->rho[v];
    }
    /* beamlet cumulative probabilities, summed in beam-major, row-major order */
    c.nf = 0;
    for (int b = 0; b < src->n_beams; ++b) c.nf += src->beams[b].nbx * src->beams[b].nby;
    c.cdf = (double*)malloc(sizeof(double) * (c.nf + 1));
    c.f = (double*)malloc(sizeof(double) * c.nf);
    c.beam_of = (int*)malloc(sizeof(int) * c.nf);
    c.beam_off = (int*)malloc(sizeof(int) * src->n_beams);
    double tot = 0.0;
    int gi = 0;
    for (int b = 0; b < src->n_beams; ++b) {
        c.beam_off[b] = gi;
        const orc_beam* bm = &src->beams[b];
        for (int j = 0; j < bm->nbx * bm->nby; ++j, ++gi) {
            double f = bm->intensity ? (double)bm->intensity[j] : 1.0;
            if (f < 0.0) f = 0.0;
            c.cdf[gi] = tot;
            c.f[gi] = f;
            c.beam_of[gi] = b;
            tot += f;
        }
    }
    int bad = !(tot > 0.0) && src->n_phsp == 0;
    if (!bad && src->n_phsp == 0 && src->beamlet_sampler == 1)
        bad = metropolis_chains(&c, prm->hist0, prm->n_hist);
    for (int i = 0; i < c.nf; ++i) c.cdf[i] /= tot;
    c.cdf[c.nf] = 1.0;
    if (src->spec_kind == 1) {
        c.spec_c = (double*)malloc(sizeof(double) * src->spec_n);
        c.spec_c[0] = 0.0;
        for (int j = 0; j + 1 < src->spec_n; ++j)
            c.spec_c[j + 1] = c.spec_c[j] + 0.5 * (src->spec_p[j] + src->spec_p[j + 1]) *
                                                (src->spec_e[j + 1] - src->spec_e[j]);
        if (!(c.spec_c[src->spec_n - 1] > 0.0)) bad = 1;
        else if (src->spectrum_strata > 0) strata_setup(&c);
    }
    if (bad) {
        free(c.mats); free(c.cdf); free(c.beam_of); free(c.beam_off); free(c.spec_c);
        free(c.f); free(c.metro_bl); free(c.strata_F); free(c.strata_e);
        return 1;
    }

    int nb = prm->n_batches;
    int nt = prm->n_threads > 0 ? prm->n_threads : 1;
    double* slots = batch_edep ? batch_edep : (double*)malloc(sizeof(double) * nv * nb);
    memset(slots, 0, sizeof(double) * nv * nb);
    double* nhist = (double*)calloc(nb, sizeof(double));
    job_t* jobs = (job_t*)calloc(nt, sizeof(job_t));
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nt);
    for (int t = 0; t < nt; ++t) {
        jobs[t].c = &c;
        jobs[t].w.tally = (double*)malloc(sizeof(double) * nv);
        jobs[t].hist_out = hist_out;
        jobs[t].hist_hard = hist_hard;
    }
    uint64_t R = prm->round_size, N = prm->n_hist;
    for (uint64_t r = 0; r * R < N; ++r) {
        uint64_t a = prm->hist0 + r * R;
        uint64_t b = prm->hist0 + (r * R + R < N ? r * R + R : N);
        int slot = (int)(r % (uint64_t)nb);
        nhist[slot] += (double)(b - a);
        uint64_t chunk = (b - a + nt - 1) / nt;
        for (int t = 0; t < nt; ++t) {
            memset(jobs[t].w.tally, 0, sizeof(double) * nv);
            jobs[t].h0 = a + chunk * t < b ? a + chunk * t : b;
            jobs[t].h1 = a + chunk * (t + 1) < b ? a + chunk * (t + 1) : b;
            if (nt > 1) pthread_create(&th[t], NULL, thread_main, &jobs[t]);
            else thread_main(&jobs[t]);
        }
        for (int t = 0; t < nt; ++t) {
            if (nt > 1) pthread_join(th[t], NULL);
            double* dst = slots + (size_t)slot * nv;
            for (size_t v = 0; v < nv; ++v) dst[v] += jobs[t].w.tally[v];
        }
    }
    orc_stats acc;
    memset(&acc, 0, sizeof acc);
    for (int t = 0; t < nt; ++t) {
        acc.e_in += jobs[t].w.e_in;
        acc.e_esc += jobs[t].w.e_esc;
        for (int k = 0; k < 8; ++k) acc.ev[k] += jobs[t].w.ev[k];
        for (int k = 0; k < ORC_NTYPES; ++k) {
            acc.n_type[k] += jobs[t].w.n_type[k];
            acc.p_type[k] += jobs[t].w.p_type[k];
            acc.v_type[k] += jobs[t].w.v_type[k];
        }
        free(jobs[t].w.tally);
        free(jobs[t].w.st);
    }
    for (size_t i = 0; i < nv * nb; ++i) acc.e_dep += slots[i];
    /* dose per history in each batch, batch mean and its standard error */
    double vvox = ph->dx * ph->dy * ph->dz;
    if (dose || sigma) {
        for (size_t v = 0; v < nv; ++v) {
            double mass = ph->rho[v] * vvox, mean = 0.0;
            for (int k = 0; k < nb; ++k)
                mean += nhist[k] > 0 ? slots[(size_t)k * nv + v] / (mass * nhist[k]) : 0.0;
            mean /= nb;
            double ss = 0.0;
            for (int k = 0; k < nb; ++k) {
                double dk = nhist[k] > 0 ? slots[(size_t)k * nv + v] / (mass * nhist[k]) : 0.0;
                ss += (dk - mean) * (dk - mean);
            }
            if (dose) dose[v] = mean;
            if (sigma) sigma[v] = nb > 1 ? sqrt(ss / ((double)nb * (nb - 1))) : 0.0;
        }
    }
    if (st) *st = acc;
    if (!batch_edep) free(slots);
    free(nhist); free(jobs); free(th);
    free(c.mats); free(c.cdf); free(c.beam_of); free(c.beam_off); free(c.spec_c);
    free(c.f); free(c.metro_bl); free(c.strata_F); free(c.strata_e);
    return 0;
}

/* ======================================================================== */
/* Hooks for the pin tests                                                    */
/* ======================================================================== */

double orc_phys(int which, const orc_material* mm, double e, double p1, double p2) {
    mat_t m = mat_make(mm);
    switch (which) {
    case ORC_MU_COMPTON: return mu_compton(&m, e);
    case ORC_MU_PHOTO: return mu_photo(&m, e);
    case ORC_MU_PAIR: return mu_pair(&m, e);
    case ORC_L_RESTRICTED: return l_restricted(&m, e, p1);
    case ORC_S_RAD_SOFT: return s_rad_soft(&m, e, p1);
    case ORC_MU_MOLLER: return mu_moller(&m, e, p1);
    case ORC_MU_BREMS: return mu_brems(&m, e, p1);
    case ORC_INV_LAMBDA1: return inv_lambda1(&m, e);
    case ORC_X0: return m.x0;
    case ORC_S_TOTAL: return s_total(&m, e, p1, p2);
    case ORC_SIGMA_KN: return sigma_kn(e / MC2);
    case ORC_DSIGMA_KN: return dsigma_kn(e / MC2, p1);
    case ORC_DSIGMA_MOLLER: return dsigma_moller(e, p1);
    case ORC_DMU_BREMS: return dmu_brems(&m, e, p1);
    case ORC_MW_MEAN: return mw_mean(p1);
    default: return NAN;
    }
}

double orc_path_length(const orc_material* mm, double ta, double tb, double wcc, double wcb) {
    mat_t m = mat_make(mm);
    return path_length(&m, ta, tb, wcc, wcb);
}

double orc_csda_energy(const orc_material* mm, double t0, double q, double wcc, double wcb) {
    pthread_once(&gl_once, gl_init);
    mat_t m = mat_make(mm);
    return csda_energy(&m, t0, q, wcc, wcb);
}

void orc_sample(int which, double e, double p1, double p2, uint64_t seed, int n, double* out1,
                double* out2) {
    for (int i = 0; i < n; ++i) {
        stream_t s = stream_make(seed, 0, (uint64_t)i, 0);
        double a = NAN, b = NAN;
        if (which == 0 || which == 7) {
            /* the transport's Compton interaction on a photon along +z */
            particle_t p;
            memset(&p, 0, sizeof p);
            p.e = e;
            p.d[2] = 1.0;
            p.s = s;
            double te, de[3];
            compton(&p, &te, de);
            if (which == 0) {
                a = p.e / e;
                b = p.d[2];
            } else {
                a = de[2];   /* electron direction cosine */
                b = p.d[2];  /* photon direction cosine */
            }
        } else if (which == 1) {
            /* run the transport's Moller sampler on a scratch particle */
            ctx_t c;
            work_t w;
            memset(&c, 0, sizeof c);
            memset(&w, 0, sizeof w);
            c.prm.ecut_e = p1;
            double tally = 0.0;
            w.tally = &tally;
            particle_t p;
            memset(&p, 0, sizeof p);
            p.e = e;
            p.d[2] = 1.0;
            p.s = s;
            moller(&c, &w, &p, 0);
            a = (e - p.e) / e;
            b = p.d[2];
            free(w.st);
        } else if (which == 2) {
            ctx_t c;
            work_t w;
            memset(&c, 0, sizeof c);
            memset(&w, 0, sizeof w);
            c.prm.ecut_g = p1;
            particle_t p;
            memset(&p, 0, sizeof p);
            p.e = e;
            p.d[2] = 1.0;
            p.s = s;
            brems(&c, &w, &p);
            a = e - p.e;
            free(w.st);
        } else if (which == 3) {
            a = sample_mw(e, &s);
        } else if (which == 4) {
            double d[3] = {0.0, 0.0, 1.0};
            int nh = (int)p2;
            for (int k = 0; k < nh; ++k) {
                double mu = sample_mw(e, &s);
                double phi = 2.0 * PI * draw(&s);
                rotate(d, 1.0 - 2.0 * mu, 2.0 * sqrt(mu * (1.0 - mu)), phi);
            }
            a = d[2];
            b = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        } else if (which == 5) {
            work_t w;
            memset(&w, 0, sizeof w);
            particle_t p;
            memset(&p, 0, sizeof p);
            p.s = s;
            double x[3] = {0, 0, 0};
            annihilate(&w, &p, x, 2.0 * MC2, 0);
            a = w.st[0].d[2];
            b = w.st[0].d[0] * w.st[1].d[0] + w.st[0].d[1] * w.st[1].d[1] + w.st[0].d[2] * w.st[1].d[2];
            free(w.st);
        } else if (which == 6) {
            /* the transport's pair split of a photon of energy e */
            particle_t p;
            memset(&p, 0, sizeof p);
            p.e = e;
            p.s = s;
            double tm, tp, aa;
            pair_split(&p, &tm, &tp, &aa);
            a = tm / (e - 2.0 * MC2);
            b = (tm + tp + aa) - e;   /* energy conservation */
        }
        out1[i] = a;
        if (out2) out2[i] = b;
    }
}

int orc_sample_source(const orc_source* src, const orc_phantom* ph, uint64_t seed, uint32_t job,
                      uint64_t hist0, int n, double* out) {
    orc_material dummy = {7.42, 0.55508, 75.0};
    orc_params prm;
    memset(&prm, 0, sizeof prm);
    prm.seed = seed;
    prm.job_id = job;
    prm.n_batches = 1;
    prm.hist0 = hist0;
    prm.n_hist = n > 0 ? (uint64_t)n : 1;    /* the n histories form one round */
    prm.round_size = prm.n_hist;
    if (validate(&dummy, 256, ph, src, &prm)) return 1;
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.ph = ph;
    c.src = src;
    c.prm = prm;
    c.n[0] = ph->nx; c.n[1] = ph->ny; c.n[2] = ph->nz;
    c.d[0] = ph->dx; c.d[1] = ph->dy; c.d[2] = ph->dz;
    for (int i = 0; i < 3; ++i) c.len[i] = c.n[i] * c.d[i];
    c.nf = 0;
    for (int b = 0; b < src->n_beams; ++b) c.nf += src->beams[b].nbx * src->beams[b].nby;
    c.cdf = (double*)malloc(sizeof(double) * (c.nf + 1));
    c.f = (double*)malloc(sizeof(double) * c.nf);
    c.beam_of = (int*)malloc(sizeof(int) * c.nf);
    c.beam_off = (int*)malloc(sizeof(int) * src->n_beams);
    double tot = 0.0;
    int gi = 0;
    for (int b = 0; b < src->n_beams; ++b) {
        c.beam_off[b] = gi;
        const orc_beam* bm = &src->beams[b];
        for (int j = 0; j < bm->nbx * bm->nby; ++j, ++gi) {
            double f = bm->intensity ? (double)bm->intensity[j] : 1.0;
            if (f < 0.0) f = 0.0;
            c.cdf[gi] = tot;
            c.f[gi] = f;
            c.beam_of[gi] = b;
            tot += f;
        }
    }
    if (src->n_phsp == 0 && src->beamlet_sampler == 1 && metropolis_chains(&c, hist0, (uint64_t)n)) {
        free(c.cdf); free(c.f); free(c.beam_of); free(c.beam_off);
        return 1;
    }
    for (int i = 0; i < c.nf; ++i) c.cdf[i] /= tot;
    c.cdf[c.nf] = 1.0;
    if (src->spec_kind == 1) {
        c.spec_c = (double*)malloc(sizeof(double) * src->spec_n);
        c.spec_c[0] = 0.0;
        for (int j = 0; j + 1 < src->spec_n; ++j)
            c.spec_c[j + 1] = c.spec_c[j] + 0.5 * (src->spec_p[j] + src->spec_p[j + 1]) *
                                                (src->spec_e[j + 1] - src->spec_e[j]);
        if (src->spectrum_strata > 0) strata_setup(&c);
    }
    for (int i = 0; i < n; ++i) {
        particle_t p;
        int bl;
        int in = source_particle(&c, hist0 + i, &p, &bl);
        double* o = out + 8 * (size_t)i;
        o[0] = p.e;
        o[1] = in ? bl : -1;
        for (int k = 0; k < 3; ++k) {
            o[2 + k] = in ? p.x[k] : NAN;
            o[5 + k] = in ? p.d[k] : NAN;
        }
    }
    free(c.cdf); free(c.beam_of); free(c.beam_off); free(c.spec_c);
    free(c.f); free(c.metro_bl); free(c.strata_F); free(c.strata_e);
    return 0;
}
