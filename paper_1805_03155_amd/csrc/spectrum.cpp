// Eigenvalues from probe time series (host, FP64).
//
// The paper reads eigenfrequencies off the Fourier transform of the wave
// function recorded at a point over the run (Sec. 3.1 and Tables 2-4).  The
// unstated details follow one reading: conjugated complex series per probe,
// symmetric 4-term Blackman-Harris window, zero padding to
// 2^ceil(log2(8 Ns)), power summed over probes, local maxima above 1e-8 of
// the largest, the lowest ones refined to the zero of the derivative of the
// windowed DTFT power by bisection.
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/spstd.h"

namespace {

using cd = std::complex<double>;

// Self-sorting radix-2 FFT (forward, unnormalised), ping-pong buffers.
void fft_pow2(std::vector<cd>& a) {
    const size_t n = a.size();
    std::vector<cd> b(n), tw(n / 2 > 0 ? n / 2 : 1);
    for (size_t k = 0; k < n / 2; ++k) {
        long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)n;
        tw[k] = cd((double)cosl(ang), (double)sinl(ang));
    }
    cd* x = a.data();
    cd* y = b.data();
    // Stockham: at stage with span s (s = 1, 2, 4, ...), m = n / (2 s)
    for (size_t s = 1; s < n; s <<= 1) {
        const size_t m = n / (2 * s);
        for (size_t q = 0; q < m; ++q) {
            const cd w = tw[q * s];
            for (size_t p = 0; p < s; ++p) {
                const cd u = x[p + s * q];
                const cd v = x[p + s * (q + m)];
                y[p + s * (2 * q)] = u + v;
                y[p + s * (2 * q + 1)] = (u - v) * w;
            }
        }
        std::swap(x, y);
    }
    if (x != a.data()) a.assign(x, x + n);
}

struct Probe {
    std::vector<cd> ws;   // window * conj(series)
};

// F(theta) = sum_p |X_p|^2 and dF/dtheta with X_p = sum_n ws[n] e^{-i theta n}
void power_slope(const std::vector<Probe>& pr, double th, double* F, double* dF) {
    double f = 0.0, df = 0.0;
    for (const Probe& p : pr) {
        cd X(0.0, 0.0), dX(0.0, 0.0);
        const size_t ns = p.ws.size();
        for (size_t n = 0; n < ns; ++n) {
            const double ang = -th * (double)n;
            const cd e(std::cos(ang), std::sin(ang));
            const cd t = p.ws[n] * e;
            X += t;
            dX += cd(0.0, -(double)n) * t;
        }
        f += std::norm(X);
        df += 2.0 * std::real(std::conj(X) * dX);
    }
    *F = f;
    *dF = df;
}

}  // namespace

extern "C" spstd_status spstd_spectrum(const double* series, int64_t nsamples, int nprobes, double dt,
                                       double hbar, int nlevels, double* E_out, double* amp_out,
                                       int* nfound) {
    if (!series || nsamples < 4 || nprobes < 1 || nprobes > SPSTD_MAX_PROBES || !(dt > 0.0) ||
        !(hbar > 0.0) || nlevels < 1 || !E_out || !nfound)
        return SPSTD_ERR_ARG;
    *nfound = 0;
    const size_t ns = (size_t)nsamples;
    // symmetric 4-term Blackman-Harris window (Harris 1978)
    const double a0 = 0.35875, a1 = 0.48829, a2 = 0.14128, a3 = 0.01168;
    std::vector<double> w(ns);
    double wsum = 0.0;
    for (size_t n = 0; n < ns; ++n) {
        const double t = 2.0 * 3.14159265358979323846 * (double)n / (double)(ns - 1);
        w[n] = a0 - a1 * std::cos(t) + a2 * std::cos(2.0 * t) - a3 * std::cos(3.0 * t);
        wsum += w[n];
    }
    std::vector<Probe> pr(nprobes);
    for (int p = 0; p < nprobes; ++p) {
        pr[p].ws.resize(ns);
        for (size_t n = 0; n < ns; ++n) {
            const double re = series[(n * nprobes + p) * 2 + 0];
            const double im = series[(n * nprobes + p) * 2 + 1];
            if (!std::isfinite(re) || !std::isfinite(im)) return SPSTD_ERR_NONFINITE;
            pr[p].ws[n] = w[n] * cd(re, -im);
        }
    }
    size_t M = 1;
    while (M < 8 * ns) M <<= 1;
    std::vector<double> power(M / 2, 0.0);
    std::vector<cd> buf(M);
    for (int p = 0; p < nprobes; ++p) {
        std::fill(buf.begin(), buf.end(), cd(0.0, 0.0));
        for (size_t n = 0; n < ns; ++n) buf[n] = pr[p].ws[n];
        fft_pow2(buf);
        for (size_t k = 0; k < M / 2; ++k) power[k] += std::norm(buf[k]);
    }
    double pmax = 0.0;
    for (double v : power) pmax = std::fmax(pmax, v);
    const double thr = 1e-8 * pmax;
    const double dth = 2.0 * 3.14159265358979323846 / (double)M;
    int found = 0;
    for (size_t k = 1; k + 1 < M / 2 && found < nlevels; ++k) {
        const double pk = power[k];
        if (!(pk > thr && pk > power[k - 1] && pk >= power[k + 1])) continue;
        double a = (double)(k - 1) * dth, b = (double)(k + 1) * dth, F, da, db;
        power_slope(pr, a, &F, &da);
        power_slope(pr, b, &F, &db);
        double th;
        if (da > 0.0 && db < 0.0) {
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (a + b);
                if (mid <= a || mid >= b) break;
                double dm;
                power_slope(pr, mid, &F, &dm);
                if (dm > 0.0) a = mid;
                else b = mid;
            }
            th = 0.5 * (a + b);
        } else {
            th = (double)k * dth;
        }
        power_slope(pr, th, &F, &da);
        E_out[found] = hbar * th / dt;
        if (amp_out) amp_out[found] = std::sqrt(F) / wsum;
        ++found;
    }
    *nfound = found;
    return SPSTD_OK;
}
