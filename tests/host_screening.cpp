// Host build of the library's reduced screening length (physics.hpp) for a
// CPU test against the oracle: for each I_TFD value a read from stdin, prints
// a, L_R and ln L_R.
#include <cstdio>

#include "physics.hpp"

int main() {
    double a;
    while (std::scanf("%lf", &a) == 1) {
        const cmc::phys::Reduced r = cmc::phys::reduced_length_log(a);
        std::printf("%.17g %.17g %.17g\n", a, r.Lr, r.lnLr);
    }
    return 0;
}
