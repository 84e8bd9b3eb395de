// croft_plan.cpp -- host-side planning helpers: supported lengths, radix
// factorisation, the FP64 twiddle generator and Bluestein's tables.
#include <cmath>
#include <utility>
#include <vector>

#include "croft_internal.h"

namespace croft {

bool smooth_length(int n) {
    if (n < 1 || n > kMaxLength) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Same factorisation rule as the kernels' compile-time plans: the 5s, the 3s,
// then the power of two as radix-8 stages plus one radix-4 or radix-16 stage
// for the remainder (a lone 2 or 4 for n = 2, 4).
int factorize(int n, int *radix) {
    if (!smooth_length(n)) return 0;
    int m = n, c5 = 0, c3 = 0, a2 = 0, s = 0;
    while (m % 5 == 0) { m /= 5; ++c5; }
    while (m % 3 == 0) { m /= 3; ++c3; }
    while (m % 2 == 0) { m /= 2; ++a2; }
    for (int i = 0; i < c5; ++i) radix[s++] = 5;
    for (int i = 0; i < c3; ++i) radix[s++] = 3;
    const int k = a2 / 3, rem = a2 % 3;
    if (rem == 1 && k >= 1) {
        for (int i = 0; i < k - 1; ++i) radix[s++] = 8;
        radix[s++] = 16;
    } else {
        for (int i = 0; i < k; ++i) radix[s++] = 8;
        if (rem == 1) radix[s++] = 2;
        if (rem == 2) radix[s++] = 4;
    }
    return s;
}

// w[m] = exp(-2 pi i m / n).  The angle 2 pi m / n is split into q quarter
// turns plus phi = (pi/2) r / n with r = 4m - q n in [0, n); phi is folded into
// [0, pi/4] (cos and sin swap beyond it) so that libm only sees small angles,
// values at multiples of pi/4 come out exactly symmetric, and the quarter
// turns are applied exactly by swapping and negating.
void twiddles_fp64(int n, double *out) {
    const double half_pi = 1.57079632679489661923132169163975144;
    for (int m = 0; m < n; ++m) {
        const long long q = (4LL * m) / n;
        const long long r = 4LL * m - q * n;
        double c, s;
        if (2 * r == n) {
            c = s = 0.70710678118654752440084436210484904;
        } else if (2 * r < n) {
            const double phi = half_pi * (double)r / (double)n;
            c = std::cos(phi);
            s = std::sin(phi);
        } else {
            const double phi = half_pi * (double)(n - r) / (double)n;
            c = std::sin(phi);
            s = std::cos(phi);
        }
        double C, S;
        switch (q & 3) {
            case 0: C = c; S = s; break;
            case 1: C = -s; S = c; break;
            case 2: C = -c; S = -s; break;
            default: C = s; S = -c; break;
        }
        out[2 * m] = C;
        out[2 * m + 1] = -S;
    }
}

// The FP64 values rounded once, to nearest even, to the FP32 the c64 and
// half-storage kernels compute in.
void round_to_fp32(const double *in, size_t count, float *out) {
    for (size_t i = 0; i < count; ++i) out[i] = static_cast<float>(in[i]);
}

int bluestein_length(int n) {
    int m = 1;
    while (m < 2 * n - 1) m *= 2;
    return m;
}

// Bluestein (1970): with j k = (j^2 + k^2 - (k - j)^2) / 2,
//   sum_j x[j] exp(-2 pi i j k / n) = c[k] sum_j (x[j] c[j]) conj(c[k - j]),
// c[j] = exp(-pi i j^2 / n): a circular convolution of length m >= 2n - 1
// once the kernel conj(c[i]), |i| < n, is wrapped into [0, m).
void bluestein_tables_fp64(int n, int m, double *chirp, double *bhat) {
    // c[j] = exp(-2 pi i r / (2n)), r = j^2 mod 2n: the length-2n twiddle table
    std::vector<double> w(4 * (size_t)n);
    twiddles_fp64(2 * n, w.data());
    for (int j = 0; j < n; ++j) {
        const long long r = ((long long)j * j) % (2LL * n);
        chirp[2 * j] = w[2 * r];
        chirp[2 * j + 1] = w[2 * r + 1];
    }
    std::vector<double> re(m, 0.0), im(m, 0.0);
    for (int i = 0; i < n; ++i) {
        re[i] = chirp[2 * i];
        im[i] = -chirp[2 * i + 1];
        if (i > 0) {
            re[m - i] = chirp[2 * i];
            im[m - i] = -chirp[2 * i + 1];
        }
    }
    // iterative radix-2 FFT (decimation in time), exp(-2 pi i ...) sign
    for (int i = 1, j = 0; i < m; ++i) {
        int bit = m >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            std::swap(re[i], re[j]);
            std::swap(im[i], im[j]);
        }
    }
    std::vector<double> tw(2 * (size_t)m);
    twiddles_fp64(m, tw.data());
    for (int len = 2; len <= m; len *= 2) {
        const int step = m / len;
        for (int i = 0; i < m; i += len) {
            for (int k = 0; k < len / 2; ++k) {
                const double wr = tw[2 * (size_t)k * step], wi = tw[2 * (size_t)k * step + 1];
                const int a = i + k, b = i + k + len / 2;
                const double xr = re[b] * wr - im[b] * wi, xi = re[b] * wi + im[b] * wr;
                re[b] = re[a] - xr;
                im[b] = im[a] - xi;
                re[a] += xr;
                im[a] += xi;
            }
        }
    }
    for (int i = 0; i < m; ++i) {
        bhat[2 * i] = re[i] / m;
        bhat[2 * i + 1] = im[i] / m;
    }
}

}  // namespace croft
