// Closed-form interaction models of the pseudo-element materials and the
// single-precision interpolation tables built from them.
//
// The paper keeps DPM's physics (section 2.1) without printing it; the models
// are this project's closed forms: free-electron Klein-Nishina Compton, a
// Z^3 E^-3 photoelectric law, a threshold pair law scaled by the radiation
// length, the restricted collision stopping power (Berger-Seltzer, no density
// effect), complete-screening bremsstrahlung, Moller above the cutoff, and
// screened-Rutherford transport cross sections with Moliere screening for the
// modified-Wentzel hinge deflection.  Cross sections are interpolated linearly
// on a grid uniform in log E, as the paper replaces DPM's cubic splines by
// linear interpolation (section 2.2.2).
#include "tables.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace gdpm {
namespace {

constexpr double kMec2 = 0.51099895;         // MeV
constexpr double kRe = 2.8179403262e-13;     // cm
constexpr double kAvogadro = 6.02214076e23;  // 1/mol
constexpr double kAlpha = 1.0 / 137.035999084;
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPiRe2 = 2.0 * kPi * kRe * kRe;

// One pseudo-element with its derived constants and cutoffs.
class Model {
public:
    Model(const MaterialParams& m, double wcb, double wcc, uint32_t flags)
        : z_(m.z), za_(m.z_over_a), imev_(m.i_ev * 1e-6), wcb_(wcb), wcc_(wcc), flags_(flags) {
        a_ = z_ / za_;
        x0_ = 716.4 * a_ / (z_ * (z_ + 1.0) * std::log(287.0 / std::sqrt(z_)));
        ne_ = kAvogadro * za_;
    }

    // photon mass attenuation coefficients (cm^2/g)
    double compton(double e) const {
        if (flags_ & 1u) return 0.0;
        const double k = e / kMec2, b = 1.0 + 2.0 * k, lb = std::log(b);
        const double s = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / b - lb / k) + lb / (2.0 * k) -
                         (1.0 + 3.0 * k) / (b * b);
        return ne_ * kTwoPiRe2 * s;
    }
    double photo(double e) const {
        if (flags_ & 2u) return 0.0;
        const double zr = z_ / 7.42;
        return 2.8e-6 * zr * zr * zr * (za_ / 0.55508) / (e * e * e);
    }
    double pair(double e) const {
        if ((flags_ & 4u) || e <= 2.0 * kMec2) return 0.0;
        const double f = 1.0 - 2.0 * kMec2 / e;
        return 0.35 * (7.0 / 9.0) * f * f * f / x0_;
    }

    // restricted stopping power, collision part with transfers below min(wcc, T/2)
    double collision(double t) const {
        const double tau = t / kMec2, gam = tau + 1.0, beta2 = 1.0 - 1.0 / (gam * gam);
        const double d = std::min(wcc_, 0.5 * t) / kMec2, ir = imev_ / kMec2;
        const double f = -1.0 - beta2 + std::log((tau - d) * d) + tau / (tau - d) +
                         (0.5 * d * d + (2.0 * tau + 1.0) * std::log(1.0 - d / tau)) / (gam * gam);
        return kTwoPiRe2 * kMec2 * ne_ / beta2 * (std::log(2.0 * (tau + 2.0) / (ir * ir)) + f);
    }
    // radiative part below the bremsstrahlung threshold
    double radiative_soft(double t) const {
        const double w = std::min(wcb_, t);
        return (4.0 / 3.0 * w - 2.0 / 3.0 * w * w / t + w * w * w / (3.0 * t * t)) / x0_;
    }
    double stopping(double t) const { return collision(t) + radiative_soft(t); }

    double moller(double t) const {
        if ((flags_ & 16u) || t <= 2.0 * wcc_) return 0.0;
        const double gam = 1.0 + t / kMec2, beta2 = 1.0 - 1.0 / (gam * gam), x = wcc_ / t;
        const double g1 = (gam - 1.0) / gam;
        const double s = g1 * g1 * (0.5 - x) + 1.0 / x - 1.0 / (1.0 - x) -
                         (2.0 * gam - 1.0) / (gam * gam) * std::log((1.0 - x) / x);
        return ne_ * kTwoPiRe2 * kMec2 / (beta2 * t) * s;
    }
    double brems(double t) const {
        if ((flags_ & 32u) || t <= wcb_) return 0.0;
        const double y = wcb_ / t;
        return (4.0 / 3.0 * std::log(1.0 / y) - 4.0 / 3.0 * (1.0 - y) + 0.5 * (1.0 - y * y)) / x0_;
    }
    // 1 / lambda_1 per g/cm^2
    double inv_transport(double t) const {
        const double p2 = t * (t + 2.0 * kMec2), gam = 1.0 + t / kMec2;
        const double beta2 = 1.0 - 1.0 / (gam * gam);
        const double q = kAlpha * std::cbrt(z_) * kMec2 / (0.885 * std::sqrt(p2));
        const double as = 0.25 * q * q * (1.13 + 3.76 * (kAlpha * z_) * (kAlpha * z_) / beta2);
        const double rut = kAvogadro / a_ * kTwoPiRe2 * z_ * (z_ + 1.0) * kMec2 * kMec2 / (beta2 * p2);
        return rut * (std::log1p(1.0 / as) - 1.0 / (1.0 + as));
    }

    // integral of dE / S over [a, b] (a <= b): Simpson in ln E, split at the
    // kinks of the restricted losses
    double path(double a, double b) const {
        if (b <= a) return 0.0;
        double cuts[2] = {std::min(wcb_, 2.0 * wcc_), std::max(wcb_, 2.0 * wcc_)};
        double sum = 0.0, lo = a;
        for (double c : cuts) {
            if (c > lo && c < b) {
                sum += simpson(lo, c);
                lo = c;
            }
        }
        return sum + simpson(lo, b);
    }

private:
    double simpson(double a, double b) const {
        const double la = std::log(a), lb = std::log(b);
        int n = 2 * std::max(4, (int)std::ceil((lb - la) / 0.004));
        const double h = (lb - la) / n;
        auto f = [&](double l) {
            const double e = std::exp(l);
            return e / stopping(e);
        };
        double s = f(la) + f(lb);
        for (int i = 1; i < n; ++i) s += (i & 1 ? 4.0 : 2.0) * f(la + i * h);
        return s * h / 3.0;
    }

    double z_, za_, imev_, wcb_, wcc_;
    uint32_t flags_;
    double a_, x0_, ne_;
};

// mean of mu = (1 - cos)/2 under the modified-Wentzel law with screening A
double mw_mean(double a) {
    if (a > 1e3) {
        const double x = 1.0 / a;
        // A [ (1+A) ln(1 + 1/A) - 1 ] expanded in x = 1/A
        return 0.5 - x / 6.0 + x * x / 12.0 - x * x * x / 20.0 + x * x * x * x / 30.0;
    }
    return a * ((1.0 + a) * std::log1p(1.0 / a) - 1.0);
}

// screening A with mean deflection (1 - e^-t)/2, by bisection on log A
double mw_screening(double t) {
    const double target = -0.5 * std::expm1(-t);
    double lo = std::log(1e-40), hi = std::log(1e40);
    for (int i = 0; i < 300 && hi - lo > 1e-14; ++i) {
        const double mid = 0.5 * (lo + hi);
        (mw_mean(std::exp(mid)) < target ? lo : hi) = mid;
    }
    return std::exp(0.5 * (lo + hi));
}

}  // namespace

void build_kn_table(double log2_lo, HostTables& T);

bool build_tables(const std::vector<MaterialParams>& mats, int n_grid, double ecut_g,
                  double ecut_e, uint32_t flags, HostTables* out, std::string* err) {
    if (mats.empty() || (int)mats.size() > 8) {
        *err = "need 1..8 materials";
        return false;
    }
    if (n_grid < 256 || n_grid > 8192) {
        *err = "n_grid must lie in [256, 8192]";
        return false;
    }
    if (!(ecut_g > 0.0) || !(ecut_e > 0.0) || ecut_g >= kEmax || ecut_e >= kEmax) {
        *err = "absorption energies must lie in (0, 30) MeV";
        return false;
    }
    for (const auto& m : mats) {
        if (!(m.z > 0.0) || !(m.z_over_a > 0.0) || !(m.i_ev > 0.0) || !std::isfinite(m.z) ||
            !std::isfinite(m.z_over_a) || !std::isfinite(m.i_ev)) {
            *err = "material parameters must be positive and finite";
            return false;
        }
    }
    HostTables& T = *out;
    const int nm = (int)mats.size();
    T.n_mat = nm;
    std::vector<Model> model;
    for (const auto& m : mats) model.emplace_back(m, ecut_g, ecut_e, flags);

    // photon tables
    T.pg_n = n_grid;
    T.pg_lo = std::log2(0.999 * ecut_g);
    T.pg_step = (std::log2(kEmax) - T.pg_lo) / (n_grid - 1);
    T.phot.assign((size_t)nm * n_grid * 4, 0.0f);
    T.mu_tot.assign((size_t)nm * n_grid, 0.0);
    for (int m = 0; m < nm; ++m) {
        for (int i = 0; i < n_grid; ++i) {
            const double e = std::exp2(T.pg_lo + i * T.pg_step);
            const double c = model[m].compton(e), p = model[m].photo(e), q = model[m].pair(e);
            float* o = &T.phot[((size_t)m * n_grid + i) * 4];
            o[0] = (float)c;
            o[1] = (float)p;
            o[2] = (float)q;
            o[3] = (float)(c + p + q);
            T.mu_tot[(size_t)m * n_grid + i] = c + p + q;
        }
    }

    // electron tables; node 0 sits at the absorption energy, where R = 0
    T.eg_n = n_grid;
    T.eg_lo = std::log2(ecut_e);
    T.eg_step = (std::log2(kEmax) - T.eg_lo) / (n_grid - 1);
    T.elec.assign((size_t)nm * n_grid * 4, 0.0f);
    T.nr = n_grid;
    T.rinv.assign((size_t)nm * T.nr, 0.0f);
    T.rinv_scale.assign(nm, 0.0f);
    std::vector<double> energy(n_grid), range(n_grid);
    for (int i = 0; i < n_grid; ++i) energy[i] = std::exp2(T.eg_lo + i * T.eg_step);
    energy[0] = ecut_e;
    for (int m = 0; m < nm; ++m) {
        const Model& md = model[m];
        range[0] = 0.0;
        for (int i = 1; i < n_grid; ++i) range[i] = range[i - 1] + md.path(energy[i - 1], energy[i]);
        double prev_hard = 0.0;
        for (int i = 0; i < n_grid; ++i) {
            const double e = energy[i];
            const double mm = md.moller(e), hard = mm + md.brems(e);
            if (hard < prev_hard) {
                *err = "hard-event attenuation must not decrease with energy";
                return false;
            }
            prev_hard = hard;
            float* o = &T.elec[((size_t)m * n_grid + i) * 4];
            o[0] = (float)range[i];
            o[1] = (float)hard;
            o[2] = (float)mm;
            o[3] = (float)md.inv_transport(e);
        }
        // inverse range on w = sqrt(R): E(w_k), w_k = k w_max / (nr - 1)
        const double wmax = std::sqrt(range[n_grid - 1]);
        T.rinv_scale[m] = (float)((T.nr - 1) / wmax);
        int j = 0;
        for (int k = 0; k < T.nr; ++k) {
            const double w = wmax * k / (T.nr - 1), r = w * w;
            if (k == 0) {
                T.rinv[(size_t)m * T.nr] = (float)ecut_e;
                continue;
            }
            if (k == T.nr - 1) {
                T.rinv[(size_t)m * T.nr + k] = (float)energy[n_grid - 1];
                continue;
            }
            while (j + 1 < n_grid - 1 && range[j + 1] <= r) ++j;
            // solve R(E) = r inside [energy[j], energy[j+1]] by safeguarded Newton
            double lo = energy[j], hi = energy[j + 1];
            double e = lo + (r - range[j]) / (range[j + 1] - range[j]) * (hi - lo);
            for (int it = 0; it < 60; ++it) {
                const double f = range[j] + md.path(energy[j], e) - r;
                (f < 0.0 ? lo : hi) = e;
                double en = e - f * md.stopping(e);
                if (!(en > lo && en < hi)) en = 0.5 * (lo + hi);
                if (std::fabs(en - e) < 1e-15 * e) {
                    e = en;
                    break;
                }
                e = en;
            }
            T.rinv[(size_t)m * T.nr + k] = (float)e;
        }
    }

    // modified-Wentzel screening table: log2 A on log2 t in [1e-9, t_iso]
    T.aw_n = 4096;
    T.aw_lo = std::log2(1e-9);
    T.aw_step = (std::log2(kMwIsotropic) - T.aw_lo) / (T.aw_n - 1);
    T.aw.assign(T.aw_n, 0.0f);
    for (int i = 0; i < T.aw_n; ++i)
        T.aw[i] = (float)std::log2(mw_screening(std::exp2(T.aw_lo + i * T.aw_step)));

    // Compton: the inverse of the Klein-Nishina distribution function on the
    // photon energy range
    build_kn_table(T.pg_lo, T);
    return true;
}

// Klein-Nishina mass of eps' in [eps, 1] (unnormalised), in terms of a = 1/eps:
// the density 1/eps + eps - t(2 - t), t = (a - 1)/k, times |d eps| = da / a^2,
// integrated from 1 to a:
// [ln a - 1/(2a^2)] - (2/k)[ln a + 1/a - 1] + (1/k^2)[a - 2 ln a - 1/a]  (+ 1/2 from a = 1)
double kn_upper_mass(double a, double k) {
    const double la = std::log(a);
    return (la - 0.5 / (a * a) + 0.5) - (2.0 / k) * (la + 1.0 / a - 1.0) + (a - 2.0 * la - 1.0 / a) / (k * k);
}

// eps with F(eps) = u, F the Klein-Nishina distribution function on [eps0, 1]:
// Newton steps on F (its derivative is the density over the total) inside a
// bracket that every evaluation narrows, bisecting where a step leaves it
double kn_quantile(double k, double u) {
    const double eps0 = 1.0 / (1.0 + 2.0 * k);
    const double total = kn_upper_mass(1.0 + 2.0 * k, k);
    double lo = eps0, hi = 1.0, x = std::pow(eps0, 1.0 - u);
    for (int it = 0; it < 200; ++it) {
        const double f = 1.0 - kn_upper_mass(1.0 / x, k) / total - u;
        if (f < 0.0) lo = x;
        else hi = x;
        const double t = (1.0 / x - 1.0) / k;
        const double dens = (1.0 / x + x - t * (2.0 - t)) / total;
        double xn = x - f / dens;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 1e-15 * x || hi - lo <= 1e-15 * hi) return xn;
        x = xn;
    }
    return x;
}

void build_kn_table(double log2_lo, HostTables& T) {
    T.kn_ne = 256;
    T.kn_nu = 1025;
    T.kn_lo = log2_lo;
    T.kn_step = (std::log2(kEmax) - log2_lo) / (T.kn_ne - 1);
    T.kn.assign((size_t)T.kn_ne * T.kn_nu, 0.0f);
    for (int i = 0; i < T.kn_ne; ++i) {
        const double k = std::exp2(T.kn_lo + i * T.kn_step) / kMec2;
        const double l0 = std::log(1.0 + 2.0 * k);   // ln(1/eps0)
        for (int j = 0; j < T.kn_nu; ++j) {
            const double u = (double)j / (T.kn_nu - 1);
            const double q = j == 0 ? 0.0 : (j == T.kn_nu - 1 ? 1.0 : std::log(kn_quantile(k, u) * (1.0 + 2.0 * k)) / l0);
            T.kn[(size_t)i * T.kn_nu + j] = (float)q;
        }
    }
}

std::vector<float> build_majorant(const HostTables& t, const std::vector<double>& rho_max) {
    std::vector<float> mm(t.pg_n, 0.0f);
    for (int i = 0; i < t.pg_n; ++i) {
        double best = 0.0;
        for (int m = 0; m < t.n_mat && m < (int)rho_max.size(); ++m) {
            // majorant of what the device evaluates: rho (float) times the float table value
            const double v = rho_max[m] * (double)t.phot[((size_t)m * t.pg_n + i) * 4 + 3];
            best = std::max(best, v);
        }
        mm[i] = (float)(best * (1.0 + 1e-6));
    }
    return mm;
}

}  // namespace gdpm
