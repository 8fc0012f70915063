// Runs libpd's host set-up routines (filter and profile construction, status
// strings) over valid and invalid arguments, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer.  Prints OK.
#include <cmath>
#include <cstdio>
#include <vector>

#include "pd.h"

int main()
{
    for (int m = -1; m <= 12; ++m) {
        std::vector<double> h(2 * (m > 0 ? m : 1) + 2, 0.0);
        const int rc = pd_symmlet(m, h.data());
        if ((m >= 1 && m <= 10) != (rc == PD_OK)) return 1;
        if (rc == PD_OK) {
            double s = 0.0;
            for (int k = 0; k < 2 * m; ++k) s += h[k];
            if (std::fabs(s - std::sqrt(2.0)) > 1e-9) return 1;
        }
    }
    if (pd_symmlet(6, nullptr) == PD_OK) return 1;
    const int n2s[] = {1, 2, 8, 64, 513};
    const double sig[] = {-1.0, 0.0, 0.5, 3.0, 12.0};
    const double mass[] = {0.0, 0.5, 0.99, 1.0, 1.5};
    for (int n2 : n2s)
        for (double sm : sig)
            for (double ms : mass) {
                int R = -1;
                if (pd_op1_taps(n2, sm, ms, &R, nullptr) != PD_OK) continue;
                if (R < 0 || R > 100000) return 1;
                std::vector<double> t((size_t)n2 * (2 * R + 1));
                if (pd_op1_taps(n2, sm, ms, &R, t.data()) != PD_OK) return 1;
                for (double v : t)
                    if (!std::isfinite(v)) return 1;
            }
    if (pd_op1_taps(16, 3.0, 0.99, nullptr, nullptr) == PD_OK) return 1;
    for (int code = -12; code <= 2; ++code)
        if (!pd_strerror(code)) return 1;
    std::printf("OK\n");
    return 0;
}
