// Host-side FP64 cosmology tables for the PM step (no GPU code).
//
// Growth: flat LambdaCDM growing mode in integral form,
//   D~(a) = (5 Om / 2) E(a) int_0^a da' / (a' E(a'))^3,   D = D~ / D~(1),
// evaluated by composite Gauss-Legendre quadrature after the substitution
// a' = a u^2 (smooth integrand).  G(a) = a^3 E(a) dD/da is the momentum growth.
// Linear spectrum: Eisenstein & Hu (1998) no-wiggle transfer function,
// P = A k^n_s T^2 with A fixed by sigma_8 (top hat R = 8 Mpc/h).
// Time stepping: kick/drift factors exact for linear growth (FastPM lineage,
// cited by the pmwd paper via FastPM-vmad).
// Second-order (2LPT) growth at a_0: D2 = -(3/7) D^2 Omega_m(a)^(-1/143)
// (Bouchet et al. 1995 fit) and G2 = a^3 E dD2/da.
#pragma once
#include <vector>

namespace pmx {

struct Cosmo {
    double omega_m, omega_b, h, sigma8, n_s, T_cmb;
};

struct Growth {
    double D, dD, G;
};

// D(a), dD/da and G(a) for flat LambdaCDM.
Growth growth(double a, double omega_m);

// Linear P(k) at a = 1, k in h/Mpc; amplitude from sigma_8.
double pk_amplitude(const Cosmo& c);
double pk_linear(double k, const Cosmo& c, double amplitude);

struct Schedule {
    std::vector<double> a;          // a_n, n = 0..N
    std::vector<double> kick_a, drift, kick_b;   // n = 0..N-1
    double D0 = 0, G0 = 0;
    double D20 = 0, G20 = 0;        // second-order growth D2, G2 at a_0
    std::vector<double> D, dD, G;   // at a_n
};

Schedule schedule(double omega_m, double a_start, double a_stop, int n_steps);

// Central differences in Omega_m (step 1e-5 Omega_m) of every schedule entry.
Schedule schedule_domega(double omega_m, double a_start, double a_stop, int n_steps);

// P_lin(k_n) for k_n = 2 pi sqrt(n2) / box, n2 = 0 .. n2_max (0 at n2 = 0).
std::vector<double> pk_table(const Cosmo& c, double box, int n2_max);

// d/dOmega_m of pk_table (central differences, sigma_8 held fixed).
std::vector<double> pk_table_domega(const Cosmo& c, double box, int n2_max);

}  // namespace pmx
