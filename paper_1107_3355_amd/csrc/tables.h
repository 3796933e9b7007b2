// Interpolation tables of the transport, generated on the host from closed
// forms in double precision and stored in single precision.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace gdpm {

struct MaterialParams {
    double z, z_over_a, i_ev;
};

struct HostTables {
    int n_mat = 0;
    // photon grid: node i at log2 E = pg_lo + i * pg_step
    double pg_lo = 0, pg_step = 0;
    int pg_n = 0;
    std::vector<float> phot;   // n_mat * pg_n * 4
    // electron grid: node 0 at the absorption energy
    double eg_lo = 0, eg_step = 0;
    int eg_n = 0;
    std::vector<float> elec;   // n_mat * eg_n * 4
    int nr = 0;
    std::vector<float> rinv;   // n_mat * nr
    std::vector<float> rinv_scale;
    double aw_lo = 0, aw_step = 0;
    int aw_n = 0;
    std::vector<float> aw;
    // photon mass attenuation (double) kept for the majorant
    std::vector<double> mu_tot;  // n_mat * pg_n
    // Klein-Nishina inverse distribution function (material independent):
    // kn[i * kn_nu + j] = ln(eps / eps0) / ln(1 / eps0) of the eps with F(eps) = u,
    // at log2 E = kn_lo + i * kn_step and u = j / (kn_nu - 1); eps0 = 1/(1 + 2k)
    double kn_lo = 0, kn_step = 0;
    int kn_ne = 0, kn_nu = 0;
    std::vector<float> kn;
};

// Largest kinetic energy the tables cover (MeV).
constexpr double kEmax = 30.0;
// Beyond this t = s / lambda_1 the hinge deflection is isotropic.
constexpr double kMwIsotropic = 20.0;

// Builds every table; returns false with a message on an inconsistent input.
bool build_tables(const std::vector<MaterialParams>& mats, int n_grid, double ecut_g,
                  double ecut_e, uint32_t flags, HostTables* out, std::string* err);

// Woodcock majorant of a phantom on the photon grid: max over materials of the
// largest density times mu_tot, rounded up to single precision.
std::vector<float> build_majorant(const HostTables& t, const std::vector<double>& rho_max);

}  // namespace gdpm
