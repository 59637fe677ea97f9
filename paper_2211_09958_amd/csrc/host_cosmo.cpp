// Host-side FP64 cosmology tables; see host_cosmo.h.
#include "host_cosmo.h"

#include <cmath>

namespace pmx {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Legendre polynomial P_n(z) and its derivative, by the three-term recurrence.
void legendre(int n, double z, double* p, double* dp) {
    double p0 = 1.0, p1 = 0.0;
    for (int k = 1; k <= n; ++k) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
    }
    *p = p0;
    *dp = n * (z * p0 - p1) / (z * z - 1.0);
}

// Gauss-Legendre nodes/weights on [-1, 1]: Newton iteration on the roots of P_n.
struct GaussLegendre {
    std::vector<double> x, w;
    explicit GaussLegendre(int n) : x(n), w(n) {
        for (int i = 0; i < n; ++i) {
            double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), p, dp;
            for (int it = 0; it < 100; ++it) {
                legendre(n, z, &p, &dp);
                double dz = p / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            legendre(n, z, &p, &dp);
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

const GaussLegendre& gl20() {
    static const GaussLegendre g(20);
    return g;
}

// Composite Gauss-Legendre of f over [lo, hi] with `panels` equal panels.
template <class F>
double integrate(F f, double lo, double hi, int panels) {
    const GaussLegendre& g = gl20();
    double h = (hi - lo) / panels, sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        double c = lo + (p + 0.5) * h, acc = 0.0;
        for (size_t i = 0; i < g.x.size(); ++i) acc += g.w[i] * f(c + 0.5 * h * g.x[i]);
        sum += 0.5 * h * acc;
    }
    return sum;
}

double hubble(double a, double om) { return std::sqrt(om / (a * a * a) + (1.0 - om)); }

// D~(a) and dD~/da from the integral form.
void growth_raw(double a, double om, double* d, double* dd) {
    // int_0^a da'/(a'E)^3 with a' = a u^2, da' = 2 a u du
    auto f = [&](double u) {
        if (u <= 0.0) return 0.0;
        double ap = a * u * u;
        double ae = ap * hubble(ap, om);
        return 2.0 * a * u / (ae * ae * ae);
    };
    double I = integrate(f, 0.0, 1.0, 64);
    double E = hubble(a, om);
    double dE = -1.5 * om / (a * a * a * a * E);
    double ae = a * E;
    *d = 2.5 * om * E * I;
    *dd = 2.5 * om * (dE * I + E / (ae * ae * ae));
}

double transfer(double k, const Cosmo& c) {
    double om_h2 = c.omega_m * c.h * c.h;
    double ob_h2 = c.omega_b * c.h * c.h;
    double fb = c.omega_b / c.omega_m;
    double theta = c.T_cmb / 2.7;
    double s = 44.5 * std::log(9.83 / om_h2) / std::sqrt(1.0 + 10.0 * std::pow(ob_h2, 0.75));
    double alpha = 1.0 - 0.328 * std::log(431.0 * om_h2) * fb +
                   0.38 * std::log(22.3 * om_h2) * fb * fb;
    double ks = 0.43 * k * c.h * s;
    double gamma = c.omega_m * c.h * (alpha + (1.0 - alpha) / (1.0 + ks * ks * ks * ks));
    double q = k * theta * theta / gamma;
    double L0 = std::log(2.0 * std::exp(1.0) + 1.8 * q);
    double C0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
    return L0 / (L0 + C0 * q * q);
}

double tophat(double x) {
    if (std::fabs(x) < 1e-3) return 1.0 - x * x / 10.0 + x * x * x * x / 280.0;
    return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

Schedule schedule_shift(double omega_m, double a_start, double a_stop, int n_steps) {
    Schedule s;
    double d1, dd1;
    growth_raw(1.0, omega_m, &d1, &dd1);
    auto gr = [&](double a) {
        double d, dd;
        growth_raw(a, omega_m, &d, &dd);
        Growth g;
        g.D = d / d1;
        g.dD = dd / d1;
        g.G = a * a * a * hubble(a, omega_m) * g.dD;
        return g;
    };
    s.a.resize(n_steps + 1);
    s.D.resize(n_steps + 1);
    s.dD.resize(n_steps + 1);
    s.G.resize(n_steps + 1);
    for (int n = 0; n <= n_steps; ++n) {
        s.a[n] = a_start + (a_stop - a_start) * n / n_steps;
        Growth g = gr(s.a[n]);
        s.D[n] = g.D;
        s.dD[n] = g.dD;
        s.G[n] = g.G;
    }
    s.kick_a.resize(n_steps);
    s.drift.resize(n_steps);
    s.kick_b.resize(n_steps);
    for (int n = 0; n < n_steps; ++n) {
        Growth h = gr(0.5 * (s.a[n] + s.a[n + 1]));
        s.kick_a[n] = (h.G - s.G[n]) / s.D[n];
        s.drift[n] = (s.D[n + 1] - s.D[n]) / h.G;
        s.kick_b[n] = (s.G[n + 1] - h.G) / s.D[n + 1];
    }
    s.D0 = s.D[0];
    s.G0 = s.G[0];
    // second order: D2 = -(3/7) D^2 Om(a)^(-1/143), G2 = a^3 E dD2/da with
    // dln D2/da = 2 D'/D + (3/143) (1 - Om(a)) / a
    const double a0 = s.a[0], E0 = hubble(a0, omega_m);
    const double om_a = omega_m / (a0 * a0 * a0 * E0 * E0);
    s.D20 = -3.0 / 7.0 * s.D[0] * s.D[0] * std::pow(om_a, -1.0 / 143.0);
    s.G20 = a0 * a0 * a0 * E0 * s.D20 *
            (2.0 * s.dD[0] / s.D[0] + 3.0 / 143.0 * (1.0 - om_a) / a0);
    return s;
}

}  // namespace

Growth growth(double a, double omega_m) {
    double d1, dd1, d, dd;
    growth_raw(1.0, omega_m, &d1, &dd1);
    growth_raw(a, omega_m, &d, &dd);
    Growth g;
    g.D = d / d1;
    g.dD = dd / d1;
    g.G = a * a * a * hubble(a, omega_m) * g.dD;
    return g;
}

double pk_amplitude(const Cosmo& c) {
    const double R = 8.0;
    auto f = [&](double lnk) {
        double k = std::exp(lnk);
        double t = transfer(k, c);
        double w = tophat(k * R);
        return k * k * k * std::pow(k, c.n_s) * t * t * w * w;
    };
    double var = integrate(f, std::log(1e-5), std::log(1e2), 4000) / (2.0 * kPi * kPi);
    return c.sigma8 * c.sigma8 / var;
}

double pk_linear(double k, const Cosmo& c, double amplitude) {
    if (k <= 0.0) return 0.0;
    double t = transfer(k, c);
    return amplitude * std::pow(k, c.n_s) * t * t;
}

Schedule schedule(double omega_m, double a_start, double a_stop, int n_steps) {
    return schedule_shift(omega_m, a_start, a_stop, n_steps);
}

Schedule schedule_domega(double omega_m, double a_start, double a_stop, int n_steps) {
    double h = 1e-5 * omega_m;
    Schedule up = schedule_shift(omega_m + h, a_start, a_stop, n_steps);
    Schedule dn = schedule_shift(omega_m - h, a_start, a_stop, n_steps);
    Schedule d = up;
    double inv = 1.0 / (2.0 * h);
    for (int n = 0; n < n_steps; ++n) {
        d.kick_a[n] = (up.kick_a[n] - dn.kick_a[n]) * inv;
        d.drift[n] = (up.drift[n] - dn.drift[n]) * inv;
        d.kick_b[n] = (up.kick_b[n] - dn.kick_b[n]) * inv;
    }
    for (int n = 0; n <= n_steps; ++n) {
        d.D[n] = (up.D[n] - dn.D[n]) * inv;
        d.dD[n] = (up.dD[n] - dn.dD[n]) * inv;
        d.G[n] = (up.G[n] - dn.G[n]) * inv;
    }
    d.D0 = (up.D0 - dn.D0) * inv;
    d.G0 = (up.G0 - dn.G0) * inv;
    d.D20 = (up.D20 - dn.D20) * inv;
    d.G20 = (up.G20 - dn.G20) * inv;
    return d;
}

std::vector<double> pk_table(const Cosmo& c, double box, int n2_max) {
    std::vector<double> t(n2_max + 1, 0.0);
    double amp = pk_amplitude(c);
    double kf = 2.0 * kPi / box;
    for (int n2 = 1; n2 <= n2_max; ++n2) t[n2] = pk_linear(kf * std::sqrt((double)n2), c, amp);
    return t;
}

std::vector<double> pk_table_domega(const Cosmo& c, double box, int n2_max) {
    double h = 1e-5 * c.omega_m;
    Cosmo up = c, dn = c;
    up.omega_m += h;
    dn.omega_m -= h;
    std::vector<double> a = pk_table(up, box, n2_max), b = pk_table(dn, box, n2_max);
    for (int i = 0; i <= n2_max; ++i) a[i] = (a[i] - b[i]) / (2.0 * h);
    return a;
}

}  // namespace pmx
