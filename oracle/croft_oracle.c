/*
 * croft_oracle.c -- plain FP64 CPU oracle for the complex-to-complex 3D DFT.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the GPU library (which never loads it).
 *
 * What it computes (the paper, Section 2.1):
 *   forward,  Eq. (1):  Y(k) = sum_j X(j) exp(-2 pi i (kx jx/Nx + ky jy/Ny + kz jz/Nz))
 *   backward, Eq. (2):  the same sum with exp(+2 pi i ...), scaled by 1/(Nx Ny Nz).
 * The functions below take the sign of the exponent (-1 forward, +1 backward)
 * and never normalise: the backward sum of Eq. (2) *without* the 1/N factor is
 * what they return, and the caller divides by N where Eq. (2) is wanted.
 *
 * Method: the 3D sum is separable (Section 2.1: a 3D FFT is 1D transforms
 * along each dimension), so dft3d applies a naive O(n^2) 1D DFT along x, then
 * y, then z, in place.  dft3d_brute evaluates the triple sum of Eq. (1)
 * directly, with no separation, for tiny grids.  dft3d_lines evaluates exact
 * output lines of a large grid (all kx for chosen (ky,kz)) in O(N) each.
 *
 * Layout: element (x,y,z) of a grid is at index x + nx*(y + ny*z); complex
 * values are interleaved (re, im) doubles.
 *
 * Parity pins for every function live in tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static const double kTwoPi = 6.283185307179586476925286766559;

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* One naive 1D DFT of a length-n line read with element stride `es` (in
 * complex elements) starting at `base`, written back in place.
 *   T[k] = sum_{j<n} X[j] * (c[(j k) mod n] + i*sign*s[(j k) mod n])
 * with c[m] = cos(2 pi m / n), s[m] = sin(2 pi m / n); that is
 * T[k] = sum_j X[j] exp(sign * 2 pi i j k / n).  Accumulation is sequential in
 * j, in FP64.  `tmp` holds 2n doubles of scratch. */
static void dft_line(double *data, long base, long es, int n, int sign,
                     const double *c, const double *s, double *tmp)
{
    for (int k = 0; k < n; ++k) {
        double acc_re = 0.0, acc_im = 0.0;
        int m = 0;                       /* m = (j*k) mod n, kept by add-and-wrap */
        for (int j = 0; j < n; ++j) {
            const double *x = data + 2 * (base + (long)j * es);
            const double wr = c[m], wi = sign * s[m];
            acc_re += x[0] * wr - x[1] * wi;
            acc_im += x[0] * wi + x[1] * wr;
            m += k;
            if (m >= n) m -= n;
        }
        tmp[2 * k] = acc_re;
        tmp[2 * k + 1] = acc_im;
    }
    for (int k = 0; k < n; ++k) {
        double *y = data + 2 * (base + (long)k * es);
        y[0] = tmp[2 * k];
        y[1] = tmp[2 * k + 1];
    }
}

static void make_table(int n, double *c, double *s)
{
    for (int m = 0; m < n; ++m) {
        c[m] = cos(kTwoPi * (double)m / (double)n);
        s[m] = sin(kTwoPi * (double)m / (double)n);
    }
}

/* Transform, in place, `count` lines along `axis` (0 = x, 1 = y, 2 = z),
 * starting at line number `first`.  Lines along an axis are numbered in the
 * natural order of the two remaining coordinates (the lower axis fastest):
 *   axis 0: line l = y + ny*z         axis 1: l = x + nx*z
 *   axis 2: l = x + nx*y
 * Returns 0, or -1 on bad arguments or allocation failure. */
int oracle_dft_axis_lines(int nx, int ny, int nz, double *data, int axis,
                          long first, long count, int sign)
{
    if (nx < 1 || ny < 1 || nz < 1 || axis < 0 || axis > 2 || (sign != 1 && sign != -1))
        return -1;
    const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const long es = axis == 0 ? 1 : (axis == 1 ? nx : (long)nx * ny);
    const long nlines = (long)nx * ny * nz / n;
    if (first < 0 || count < 0 || first + count > nlines) return -1;
    double *tab = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    if (!tab) return -1;
    make_table(n, tab, tab + n);
    int failed = 0;
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        if (!tmp) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (long l = first; l < first + count; ++l) {
                long base;
                if (axis == 0) base = l * nx;                       /* (0, y, z) */
                else if (axis == 1) base = (l % nx) + (l / nx) * (long)nx * ny; /* (x, 0, z) */
                else base = l;                                       /* (x, y, 0) */
                dft_line(data, base, es, n, sign, tab, tab + n, tmp);
            }
            free(tmp);
        }
    }
    free(tab);
    return failed ? -1 : 0;
}

/* Full 3D DFT, in place: x, then y, then z (separability, Section 2.1).
 * sign -1 gives Eq. (1); sign +1 gives N times Eq. (2). */
int oracle_dft3d(int nx, int ny, int nz, double *data, int sign)
{
    if (oracle_dft_axis_lines(nx, ny, nz, data, 0, 0, (long)ny * nz, sign)) return -1;
    if (oracle_dft_axis_lines(nx, ny, nz, data, 1, 0, (long)nx * nz, sign)) return -1;
    if (oracle_dft_axis_lines(nx, ny, nz, data, 2, 0, (long)nx * ny, sign)) return -1;
    return 0;
}

/* Same transform, axes taken in the order z, y, x (used to check that the
 * result does not depend on the order of the separable passes). */
int oracle_dft3d_zyx(int nx, int ny, int nz, double *data, int sign)
{
    if (oracle_dft_axis_lines(nx, ny, nz, data, 2, 0, (long)nx * ny, sign)) return -1;
    if (oracle_dft_axis_lines(nx, ny, nz, data, 1, 0, (long)nx * nz, sign)) return -1;
    if (oracle_dft_axis_lines(nx, ny, nz, data, 0, 0, (long)ny * nz, sign)) return -1;
    return 0;
}

/* Direct triple sum of Eq. (1) (sign -1) or of Eq. (2) without 1/N (sign +1),
 * O(N^2): no separation into axes.  The phase of each term is
 *   2 pi ((kx jx mod Nx)/Nx + (ky jy mod Ny)/Ny + (kz jz mod Nz)/Nz)
 * evaluated in FP64 and passed to cos/sin as one angle.  Out of place. */
int oracle_dft3d_brute(int nx, int ny, int nz, const double *in, double *out, int sign)
{
    if (nx < 1 || ny < 1 || nz < 1 || (sign != 1 && sign != -1) || in == out) return -1;
    const long N = (long)nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 4)
    for (long kk = 0; kk < N; ++kk) {
        const long kx = kk % nx, ky = (kk / nx) % ny, kz = kk / ((long)nx * ny);
        double acc_re = 0.0, acc_im = 0.0;
        for (long jj = 0; jj < N; ++jj) {
            const long jx = jj % nx, jy = (jj / nx) % ny, jz = jj / ((long)nx * ny);
            const double phase = kTwoPi * ((double)((kx * jx) % nx) / nx +
                                           (double)((ky * jy) % ny) / ny +
                                           (double)((kz * jz) % nz) / nz);
            const double wr = cos(phase), wi = sign * sin(phase);
            const double xr = in[2 * jj], xi = in[2 * jj + 1];
            acc_re += xr * wr - xi * wi;
            acc_im += xr * wi + xi * wr;
        }
        out[2 * kk] = acc_re;
        out[2 * kk + 1] = acc_im;
    }
    return 0;
}

/* The inner O(N) reduction of an exact output line: for each of the `nsamp`
 * pairs (ky[i], kz[i]) it writes, for every x,
 *   red[i*nx + x] = sum_z e_z(kz z) sum_y e_y(ky y) X(x,y,z)
 * (interleaved complex), e_a(m) = exp(sign 2 pi i m / Na) -- the y and z sums
 * of Eq. (1) (sign -1) or of Eq. (2) without 1/N (sign +1), done before any
 * sum over x.  Parallel over (i, block of XB consecutive x); the x loop is
 * innermost so rows are read contiguously.  For each x the sums run in the
 * order written above.  `in` is not modified. */
int oracle_yz_sums(int nx, int ny, int nz, const double *in, int sign,
                   int nsamp, const int *ky, const int *kz, double *red)
{
    if (nx < 1 || ny < 1 || nz < 1 || (sign != 1 && sign != -1) || nsamp < 0) return -1;
    for (int i = 0; i < nsamp; ++i)
        if (ky[i] < 0 || ky[i] >= ny || kz[i] < 0 || kz[i] >= nz) return -1;
    double *ty = (double *)malloc(sizeof(double) * 2 * (size_t)ny);
    double *tz = (double *)malloc(sizeof(double) * 2 * (size_t)nz);
    if (!ty || !tz) { free(ty); free(tz); return -1; }
    make_table(ny, ty, ty + ny);
    make_table(nz, tz, tz + nz);
    enum { XB = 64 };
    const int nxb = (nx + XB - 1) / XB;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int i = 0; i < nsamp; ++i) {
        for (int xb = 0; xb < nxb; ++xb) {
            const int x0 = xb * XB, x1 = (x0 + XB < nx) ? x0 + XB : nx;
            double sr[XB], si[XB], pr[XB], pi[XB];
            for (int x = x0; x < x1; ++x) sr[x - x0] = si[x - x0] = 0.0;
            int mz = 0;
            for (int z = 0; z < nz; ++z) {
                for (int x = x0; x < x1; ++x) pr[x - x0] = pi[x - x0] = 0.0;
                int my = 0;
                for (int y = 0; y < ny; ++y) {
                    const double wr = ty[my], wi = sign * ty[ny + my];
                    const double *v = in + 2 * ((long)nx * (y + (long)ny * z));
                    for (int x = x0; x < x1; ++x) {
                        pr[x - x0] += v[2 * x] * wr - v[2 * x + 1] * wi;
                        pi[x - x0] += v[2 * x] * wi + v[2 * x + 1] * wr;
                    }
                    my += ky[i];
                    if (my >= ny) my -= ny;
                }
                const double wr = tz[mz], wi = sign * tz[nz + mz];
                for (int x = x0; x < x1; ++x) {
                    sr[x - x0] += pr[x - x0] * wr - pi[x - x0] * wi;
                    si[x - x0] += pr[x - x0] * wi + pi[x - x0] * wr;
                }
                mz += kz[i];
                if (mz >= nz) mz -= nz;
            }
            for (int x = x0; x < x1; ++x) {
                red[2 * ((long)i * nx + x)] = sr[x - x0];
                red[2 * ((long)i * nx + x) + 1] = si[x - x0];
            }
        }
    }
    free(ty); free(tz);
    return 0;
}

/* Exact output lines of a large grid: for each of the `nsamp` pairs
 * (ky[i], kz[i]) it writes the nx values Y(kx, ky[i], kz[i]), kx = 0..nx-1,
 * to out[i*nx + kx] (interleaved complex).  By Eq. (1),
 *   Y(kx,ky,kz) = sum_x e_x(kx x) * [ sum_z e_z(kz z) sum_y e_y(ky y) X(x,y,z) ]
 * where e_a(m) = exp(sign 2 pi i m / Na).  The bracket is the O(N) reduction
 * of oracle_yz_sums, one value per x; a naive DFT over x then gives the line.
 * `in` is not modified. */
int oracle_dft3d_lines(int nx, int ny, int nz, const double *in, int sign,
                       int nsamp, const int *ky, const int *kz, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || (sign != 1 && sign != -1) || nsamp < 0) return -1;
    double *tx = (double *)malloc(sizeof(double) * 2 * (size_t)nx);
    double *red = (double *)malloc(sizeof(double) * 2 * (size_t)nx * (size_t)(nsamp > 0 ? nsamp : 1));
    if (!tx || !red) { free(tx); free(red); return -1; }
    make_table(nx, tx, tx + nx);
    if (oracle_yz_sums(nx, ny, nz, in, sign, nsamp, ky, kz, red)) { free(tx); free(red); return -1; }
    for (int i = 0; i < nsamp; ++i) {
        for (int kx = 0; kx < nx; ++kx) {
            double ar = 0.0, ai = 0.0;
            int m = 0;
            for (int x = 0; x < nx; ++x) {
                const double *v = red + 2 * ((long)i * nx + x);
                const double wr = tx[m], wi = sign * tx[nx + m];
                ar += v[0] * wr - v[1] * wi;
                ai += v[0] * wi + v[1] * wr;
                m += kx;
                if (m >= nx) m -= nx;
            }
            out[2 * ((long)i * nx + kx)] = ar;
            out[2 * ((long)i * nx + kx) + 1] = ai;
        }
    }
    free(tx); free(red);
    return 0;
}
