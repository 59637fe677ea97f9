// Host-only driver of the library's cosmology tables, built with g++ and the
// address and undefined-behaviour sanitizers by tests/test_host_sanitize.py.
// Prints the schedule, its Omega_m derivatives, the second-order growth at a_0
// and a P(k) table so the test can compare them with the library's own output.
#include <cstdio>
#include <vector>

#include "host_cosmo.h"

int main() {
    using namespace pmx;
    const Cosmo c{0.3, 0.05, 0.7, 0.8, 0.96, 2.7255};
    for (int steps : {1, 10, 63}) {
        Schedule s = schedule(c.omega_m, 1.0 / 64, 1.0, steps);
        Schedule d = schedule_domega(c.omega_m, 1.0 / 64, 1.0, steps);
        std::printf("steps %d\n", steps);
        for (int n = 0; n < steps; ++n)
            std::printf("%.17g %.17g %.17g %.17g %.17g %.17g\n", s.kick_a[n], s.drift[n],
                        s.kick_b[n], d.kick_a[n], d.drift[n], d.kick_b[n]);
        std::printf("ic %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", s.D0, s.G0, s.D20,
                    s.G20, d.D0, d.G0, d.D20, d.G20);
    }
    std::vector<double> pk = pk_table(c, 64.0, 3 * 16 * 16);
    std::printf("pk %zu\n", pk.size());
    for (double v : pk) std::printf("%.17g\n", v);
    return 0;
}
