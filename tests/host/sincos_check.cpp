// Host check of cia::fast_sincosf against double-precision sin/cos: prints
// the largest absolute errors over a dense sweep and random angles.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <random>

#include "../../paper_2203_16657_amd/csrc/fastmath.h"

int main() {
    double es = 0.0, ec = 0.0, es_big = 0.0, ec_big = 0.0;
    auto check = [](float t, double &a, double &b) {
        float s, c;
        cia::fast_sincosf(t, &s, &c);
        a = std::fmax(a, std::fabs((double)s - std::sin((double)t)));
        b = std::fmax(b, std::fabs((double)c - std::cos((double)t)));
    };
    for (int64_t k = -20000000; k <= 20000000; k++) check((float)(k * 2.5e-6), es, ec);   // [-50, 50]
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> u(-2.0e4, 2.0e4);
    for (int k = 0; k < 20000000; k++) check((float)u(g), es_big, ec_big);
    std::printf("%.3e %.3e %.3e %.3e\n", es, ec, es_big, ec_big);
    return 0;
}
