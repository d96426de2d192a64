// Host build of the in-register butterflies (fft_small.h): each size and
// direction against a float64 DFT of the same float32 inputs (eq. (4) signs).
// Prints "R INV max_relative_error" lines.
#include "fft_small.h"
#include <cstdio>
#include <cmath>
#include <random>
using namespace vbw::fft;
template <int R, bool INV> double check(std::mt19937 &g) {
    std::normal_distribution<float> nd(0.f, 1.f);
    double worst = 0;
    for (int trial = 0; trial < 200; ++trial) {
        float2 a[R];
        double xr[R], xi[R];
        for (int i = 0; i < R; ++i) { a[i] = make_float2(nd(g), nd(g)); xr[i] = a[i].x; xi[i] = a[i].y; }
        dft_small<R, INV>(a);
        double num = 0, den = 0;
        for (int k = 0; k < R; ++k) {
            double yr = 0, yi = 0;
            for (int n = 0; n < R; ++n) {
                const double th = (INV ? 2.0 : -2.0) * M_PI * double((k * n) % R) / R;
                yr += xr[n] * std::cos(th) - xi[n] * std::sin(th);
                yi += xr[n] * std::sin(th) + xi[n] * std::cos(th);
            }
            num += (a[k].x - yr) * (a[k].x - yr) + (a[k].y - yi) * (a[k].y - yi);
            den += yr * yr + yi * yi;
        }
        worst = std::fmax(worst, std::sqrt(num / den));
    }
    return worst;
}
int main() {
    std::mt19937 g(1234);
    printf("2 0 %.3e\n", check<2, false>(g)); printf("2 1 %.3e\n", check<2, true>(g));
    printf("4 0 %.3e\n", check<4, false>(g)); printf("4 1 %.3e\n", check<4, true>(g));
    printf("8 0 %.3e\n", check<8, false>(g)); printf("8 1 %.3e\n", check<8, true>(g));
    printf("16 0 %.3e\n", check<16, false>(g)); printf("16 1 %.3e\n", check<16, true>(g));
}
