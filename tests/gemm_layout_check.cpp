// Host model of the matrix-core engine's data flow for one N = 256 block:
// the lane layout and DFT-matrix exponents of gemm_layout.h, the real
// 16x16x32 products (S1's contraction entries (re, im) interleaved as the
// samples are stored, the other products' in (real | imaginary) halves), the
// twiddles, H_R and the kept output rows, in float64.  Prints the largest error against
// a direct float64 overlap-save block (forward DFT, H_R, inverse DFT, phase
// as a delay of D samples) for a few band edges.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "gemm_layout.h"

using namespace vbw::gemm;
typedef std::complex<double> cd;

struct Op {          // one operand register set: 64 lanes x 8 contraction entries
    double v[64][8];
};
struct Acc {         // accumulator: 64 lanes x 4 slots
    double v[64][4];
};

// D = A B: lane (g, c) of A holds row c, of B column c, entries 8g..8g+7;
// D lane (g, c) slot r = row 4g + r, column c.
static Acc mfma(const Op &a, const Op &b) {
    Acc d{};
    for (int g = 0; g < 4; ++g)
        for (int c = 0; c < 16; ++c)
            for (int r = 0; r < 4; ++r) {
                const int row = 4 * g + r;
                double s = 0;
                for (int gg = 0; gg < 4; ++gg)
                    for (int k = 0; k < 8; ++k) s += a.v[16 * gg + row][k] * b.v[16 * gg + c][k];
                d.v[16 * g + c][r] = s;
            }
    return d;
}

static cd w16(int e) { return std::polar(1.0, -2 * M_PI * e / 16); }
static cd w256(int e) { return std::polar(1.0, -2 * M_PI * e / 256); }

// constant operand (a0, b0, a1, b1, ...) from per-(lane, j) entries: S1's,
// whose contraction entries pair with the samples as stored, (re, im) each
template <class F> static Op make_op_interleaved(F f) {
    Op o{};
    for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 4; ++j) {
            const std::pair<double, double> p = f(l >> 4, l & 15, j);
            o.v[l][2 * j] = p.first;
            o.v[l][2 * j + 1] = p.second;
        }
    return o;
}
// constant operand [a | b] from per-(lane, j) entries
template <class F> static Op make_op(F f) {
    Op o{};
    for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 4; ++j) {
            const std::pair<double, double> p = f(l >> 4, l & 15, j);
            o.v[l][j] = p.first;
            o.v[l][4 + j] = p.second;
        }
    return o;
}
static Op data_op(const Acc &re, const Acc &im) {
    Op o{};
    for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 4; ++j) {
            o.v[l][j] = re.v[l][j];
            o.v[l][4 + j] = im.v[l][j];
        }
    return o;
}

int main() {
    std::mt19937 rng(5);
    std::normal_distribution<double> nd;
    const int N = 256;
    double worst = 0;
    for (int trial = 0; trial < 6; ++trial) {
        const int hop = trial < 4 ? 192 : (trial == 4 ? 128 : 254);
        const int lv = 8, k1 = 5 + 17 * trial;
        const int D = (N - hop) / 2;
        std::vector<double> V(lv);
        for (int r = 0; r < lv; ++r) V[r] = 1.0 - (r + 0.5) / lv;
        std::vector<cd> x(N);
        for (auto &s : x) s = cd(nd(rng), nd(rng));
        auto hr = [&](int k) {   // eq. (6) with the mirror
            const int kk = k <= N / 2 ? k : N - k;
            if (kk < k1) return 1.0;
            if (kk <= k1 + lv - 1) return V[kk - k1];
            return 0.0;
        };
        // reference: z0 = IDFT(H_R DFT(x)), kept samples z0(D + j)
        std::vector<cd> X(N), z(N);
        for (int k = 0; k < N; ++k) {
            cd s = 0;
            for (int n = 0; n < N; ++n) s += x[n] * std::polar(1.0, -2 * M_PI * double((n * k) % N) / N);
            X[k] = s * hr(k);
        }
        for (int n = 0; n < N; ++n) {
            cd s = 0;
            for (int k = 0; k < N; ++k) s += X[k] * std::polar(1.0, 2 * M_PI * double((n * k) % N) / N);
            z[n] = s / double(N);
        }
        // the engine's data flow
        Op xa{};   // the samples as loaded: (re, im) of slot j at entries 2j, 2j + 1
        for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 4; ++j) {
                const cd s = x[16 * in_row(l >> 4, j) + (l & 15)];
                xa.v[l][2 * j] = s.real();
                xa.v[l][2 * j + 1] = s.imag();
            }
        const Op s1r = make_op_interleaved([](int g, int c, int j) { cd w = w16(s1_w(g, c, j)); return std::make_pair(w.real(), -w.imag()); });
        const Op s1i = make_op_interleaved([](int g, int c, int j) { cd w = w16(s1_w(g, c, j)); return std::make_pair(w.imag(), w.real()); });
        const Op s2r = make_op([](int g, int c, int j) { cd w = w16(s2_w(g, c, j)); return std::make_pair(w.real(), -w.imag()); });
        const Op s2i = make_op([](int g, int c, int j) { cd w = w16(s2_w(g, c, j)); return std::make_pair(w.imag(), w.real()); });
        const Op s4r = make_op([](int g, int c, int j) { cd w = w16(s4_w(g, c, j)); return std::make_pair(w.real(), w.imag()); });
        const Op s4i = make_op([](int g, int c, int j) { cd w = w16(s4_w(g, c, j)); return std::make_pair(-w.imag(), w.real()); });
        Acc dr = mfma(xa, s1r), di = mfma(xa, s1i);
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
                const cd v = cd(dr.v[l][r], di.v[l][r]) * w256(tw_e(l >> 4, l & 15, r));
                dr.v[l][r] = v.real();
                di.v[l][r] = v.imag();
            }
        const Op b1 = data_op(dr, di);
        Acc qr = mfma(s2r, b1), qi = mfma(s2i, b1);
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
                const double f = hr((l & 15) + 16 * (4 * (l >> 4) + r)) / N;
                qr.v[l][r] *= f;
                qi.v[l][r] *= f;
            }
        // S3 = sum Y conj W = conj(sum conj(Y) W), with S2's entries
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) qi.v[l][r] = -qi.v[l][r];
        const Op a2 = data_op(qr, qi);
        dr = mfma(a2, s2r);
        di = mfma(a2, s2i);
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
                const cd v = cd(dr.v[l][r], -di.v[l][r]) * std::conj(w256(tw_e(l >> 4, l & 15, r)));
                dr.v[l][r] = v.real();
                di.v[l][r] = v.imag();
            }
        const Op b3 = data_op(dr, di);
        qr = mfma(s4r, b3);
        qi = mfma(s4i, b3);
        int kept = 0;
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * out_row(l >> 4, r) + (l & 15) - D;   // kept output sample
                if (j < 0 || j >= hop) continue;
                ++kept;
                worst = std::max(worst, std::abs(cd(qr.v[l][r], qi.v[l][r]) - z[D + j]));
            }
        if (kept != hop) worst = 1e9;
    }
    std::printf("%.3e\n", worst);
    return 0;
}
