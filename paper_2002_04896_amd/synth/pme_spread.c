/*
 * pme_spread.c -- seeded synthetic input: point charges spread onto a
 * periodic grid with the order-4 cardinal B-spline.
 *
 * This is input generation only; it holds no part of the transform.  It
 * models the charge grids that the forward FFT of particle-mesh Ewald
 * consumes (the application the paper targets, Section 1): charges +-1 at
 * random positions, one charge per grid cell on average, stratified so that
 * every 4x4x4 block of cells receives as many charges as it has cells, with
 * positions uniform inside the block.
 *
 * B-spline: M_2(u) = 1 - |u - 1| on [0, 2], and for n > 2
 *   M_n(u) = u/(n-1) M_{n-1}(u) + (n-u)/(n-1) M_{n-1}(u-1)
 * (smooth PME, Essmann et al., J. Chem. Phys. 103, 8577 (1995)).  A charge at
 * scaled coordinate u adds q * M_4(u - k) to grid point k, for the four k with
 * u - k in [0, 4), wrapped periodically.  The four weights sum to one.
 *
 * Random numbers: a counter-based splitmix64 stream, value c of charge i is
 * splitmix64(seed * 0x9E3779B97F4A7C15 + 4*i + c), so the grid does not depend
 * on the number of threads.  Charges are numbered block by block (x-block
 * fastest), and within a block in order.
 *
 * Determinism: blocks are processed in slabs of constant z-block index; two
 * slabs run concurrently only if the z-planes they touch are disjoint (phases
 * by parity of the z-block index, with the last block in a phase of its own
 * when the count is odd), so every grid value is summed in one fixed order.
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

static inline uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline double unit_double(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

/* M_n evaluated by the recurrence above. */
static double bspline(int n, double u)
{
    if (n == 2) return (u < 0.0 || u > 2.0) ? 0.0 : 1.0 - fabs(u - 1.0);
    return (u * bspline(n - 1, u) + (n - u) * bspline(n - 1, u - 1.0)) / (n - 1);
}

/* Weights for the 4 grid points floor(u)-3 .. floor(u) (w[0] is floor(u)). */
static void weights4(double u, long *k0, double w[4])
{
    const double fl = floor(u);
    const double f = u - fl;
    *k0 = (long)fl;
    for (int t = 0; t < 4; ++t) w[t] = bspline(4, f + t);
}

static inline long wrap(long k, long n) { k %= n; return k < 0 ? k + n : k; }

static void spread_slab(int nx, int ny, int nz, int bz, uint64_t seed, double *grid,
                        double *qsum)
{
    const int nbx = (nx + 3) / 4, nby = (ny + 3) / 4;
    const int z0 = 4 * bz, dz = (nz - z0 < 4) ? nz - z0 : 4;
    double qs = 0.0;
    for (int by = 0; by < nby; ++by) {
        const int y0 = 4 * by, dy = (ny - y0 < 4) ? ny - y0 : 4;
        for (int bx = 0; bx < nbx; ++bx) {
            const int x0 = 4 * bx, dx = (nx - x0 < 4) ? nx - x0 : 4;
            const long block = bx + (long)nbx * (by + (long)nby * bz);
            const int cnt = dx * dy * dz;
            for (int c = 0; c < cnt; ++c) {
                /* charge index: 64 slots per block, of which `cnt` are used */
                const uint64_t idx = (uint64_t)block * 64u + (uint64_t)c;
                const uint64_t key = seed * 0x9E3779B97F4A7C15ull + 4u * idx;
                const double ux = x0 + dx * unit_double(splitmix64(key + 0));
                const double uy = y0 + dy * unit_double(splitmix64(key + 1));
                const double uz = z0 + dz * unit_double(splitmix64(key + 2));
                const double q = (splitmix64(key + 3) >> 63) ? 1.0 : -1.0;
                qs += q;
                long kx, ky, kz;
                double wx[4], wy[4], wz[4];
                weights4(ux, &kx, wx);
                weights4(uy, &ky, wy);
                weights4(uz, &kz, wz);
                for (int c2 = 0; c2 < 4; ++c2) {
                    const long gz = wrap(kz - c2, nz);
                    for (int b2 = 0; b2 < 4; ++b2) {
                        const long gy = wrap(ky - b2, ny);
                        const double qyz = q * wz[c2] * wy[b2];
                        double *row = grid + (long)nx * (gy + (long)ny * gz);
                        for (int a2 = 0; a2 < 4; ++a2)
                            row[wrap(kx - a2, nx)] += qyz * wx[a2];
                    }
                }
            }
        }
    }
    *qsum = qs;
}

/* Fill `grid` (nx*ny*nz doubles, zeroed here) and return the total charge in
 * *total_charge.  Returns 0, or -1 on bad sizes. */
int synth_pme_spread(int nx, int ny, int nz, uint64_t seed, double *grid, double *total_charge)
{
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    const long N = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) grid[i] = 0.0;
    const int nbz = (nz + 3) / 4;
    double qtot = 0.0;
    /* phase 0: even bz, phase 1: odd bz, phase 2: the last bz when nbz is odd
     * and > 1 (it would otherwise touch the planes of bz = 0 through the wrap).
     * With nbz <= 2 every slab runs on its own. */
    for (int phase = 0; phase < 3; ++phase) {
        double qphase = 0.0;
        const int odd_tail = (nbz % 2 == 1) && nbz > 1;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : qphase) if (nbz > 2)
        for (int bz = 0; bz < nbz; ++bz) {
            int ph;
            if (odd_tail && bz == nbz - 1) ph = 2;
            else ph = bz % 2;
            if (ph != phase) continue;
            double qs;
            spread_slab(nx, ny, nz, bz, seed, grid, &qs);
            qphase += qs;
        }
        qtot += qphase;
    }
    *total_charge = qtot;
    return 0;
}
