// croft_tune.cpp -- wisdom: remembered kernel choices per (length, pass kind,
// dtype), the FFTW-style cache of the autotuner's results.
//
// The choice is a compiled candidate configuration and the persistent grid
// size (in resident-block waves; 0 = one block per tile).  Choices measured in
// this process are kept in memory; when the environment variable CROFT_WISDOM
// names a file, plans also read it and CROFT_MEASURE plans append to it.
// File format, one choice per line:  n kind dtype candidate waves [axis]
// (and "slabs nx ny nz dtype K" for the slab count of a grid, below)
// A strided pass also has a choice of its own per grid axis (1 = y, 2 = z:
// their strides differ, and so can their best tiles); a line without an axis
// serves every axis.  Lookup order: the CROFT_WISDOM file, choices measured
// in this process, for forward plans the forward-only built-in choices, the
// per-axis built-in choices, the built-in table below (measured on an MI355X
// with CROFT_MEASURE on cubic grids; kinds 2 and 3, the real x pass and the
// fused multiply pass, on real and convolution plans of cubic grids), then
// candidate 0 with one resident wave.  At each step an entry for the pass's
// axis comes before one for any axis.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "croft_internal.h"

namespace croft {
namespace {
struct Builtin {
    int n, kind, dtype, cand, waves;
};
// n kind dtype candidate waves
const Builtin kBuiltin[] = {
    // complex64 (384: from a sweep of the 384^3 grid, too large for the
    // Infinity Cache: the non-temporal contiguous tile, x 186 -> 163 us; the
    // 32-line wide strided tile on one wave of resident blocks, y 212 -> 173
    // and z 222 -> 176 us, both directions)
    {32, 0, 0, 0, 1}, {32, 1, 0, 0, 1}, {48, 0, 0, 0, 0}, {48, 1, 0, 0, 2}, {60, 0, 0, 0, 4}, {60, 1, 0, 0, 0},
    {64, 0, 0, 0, 4}, {64, 1, 0, 0, 4}, {72, 0, 0, 0, 1}, {72, 1, 0, 0, 0}, {80, 0, 0, 0, 0}, {80, 1, 0, 0, 4},
    {96, 0, 0, 0, 1}, {96, 1, 0, 0, 1}, {100, 0, 0, 0, 2}, {100, 1, 0, 0, 4}, {128, 0, 0, 1, 2},
    {128, 1, 0, 5, 1}, {256, 0, 0, 1, 0}, {256, 1, 0, 1, 0}, {384, 0, 0, 3, 0}, {384, 1, 0, 2, 1},
    // (the real x pass of the 512^3 real grid, length 256 above: the non-temporal
    // candidate, forward 0.613 -> 0.587 ms, backward 0.675 -> 0.640, convolution
    // 1.207 -> 1.194)
    // complex64 at the larger compiled 2^a 3^b 5^c lengths (one forward sweep of
    // n^3): the streaming contiguous tile for x except at 576; the strided tile
    // in the XCD-contiguous order where it pays (576: 2.80 -> 2.22 ms, 640:
    // 4.15 -> 3.16, 720: 5.76 -> 5.52, 768: 6.42 -> 4.89, 960: 12.70 -> 11.43)
    {400, 0, 0, 3, 0}, {480, 0, 0, 3, 0}, {576, 1, 0, 6, 0}, {640, 0, 0, 3, 0}, {640, 1, 0, 6, 0},
    {720, 0, 0, 3, 0}, {720, 1, 0, 7, 0}, {768, 0, 0, 3, 0}, {768, 1, 0, 6, 0}, {960, 0, 0, 3, 0},
    {960, 1, 0, 7, 0},
    {512, 0, 0, 3, 0}, {512, 1, 0, 4, 4}, {1024, 0, 0, 3, 0}, {1024, 1, 0, 7, 1}, {32, 2, 0, 0, 0},
    {64, 2, 0, 0, 2}, {64, 3, 0, 0, 2}, {128, 2, 0, 0, 1}, {128, 3, 0, 0, 2}, {256, 2, 0, 1, 0},
    {256, 3, 0, 0, 1}, {512, 3, 0, 0, 2},
    // complex64 batched tile shapes (kinds 4 and 5: the batched kernel's
    // contiguous and strided passes; candidate = shape), the majority of six
    // CROFT_MEASURE runs (both directions) on the 64-grid PME batch; the
    // lengths not listed keep shape 0
    {60, 4, 0, 1, 0}, {60, 5, 0, 1, 0}, {64, 4, 0, 1, 0}, {64, 5, 0, 1, 0}, {72, 4, 0, 1, 0}, {72, 5, 0, 1, 0},
    {80, 4, 0, 1, 0}, {80, 5, 0, 1, 0}, {96, 4, 0, 1, 0}, {96, 5, 0, 1, 0}, {100, 5, 0, 1, 0},
    // complex128
    {32, 0, 1, 0, 4}, {32, 1, 1, 0, 0}, {48, 0, 1, 0, 2}, {48, 1, 1, 0, 4}, {60, 0, 1, 0, 2}, {60, 1, 1, 0, 2},
    {64, 0, 1, 0, 0}, {64, 1, 1, 0, 4}, {72, 0, 1, 0, 1}, {72, 1, 1, 0, 0}, {80, 0, 1, 0, 1}, {80, 1, 1, 0, 0},
    {96, 0, 1, 0, 2}, {96, 1, 1, 0, 1}, {100, 0, 1, 0, 4}, {100, 1, 1, 0, 1}, {128, 0, 1, 3, 2},
    {128, 1, 1, 5, 4}, {256, 0, 1, 3, 0}, {256, 1, 1, 5, 0}, {384, 0, 1, 0, 0}, {384, 1, 1, 0, 2},
    // complex128 at the larger compiled lengths (one forward sweep of n^3): the
    // streaming x tile and the XCD-ordered strided tile with prefetch (640:
    // 7.43 -> 5.87 ms with the strided choice alone, 768: 12.80 -> 10.59);
    // 720 keeps the default, which none of the others beat
    {400, 0, 1, 3, 0}, {400, 1, 1, 7, 0}, {480, 0, 1, 3, 0}, {480, 1, 1, 7, 0}, {576, 0, 1, 3, 0},
    {576, 1, 1, 7, 0}, {640, 0, 1, 3, 0}, {640, 1, 1, 7, 0}, {768, 0, 1, 3, 0}, {768, 1, 1, 7, 0},
    {512, 0, 1, 3, 0}, {512, 1, 1, 4, 2}, {1024, 0, 1, 2, 0}, {1024, 1, 1, 5, 0}, {32, 2, 1, 0, 2},
    {64, 2, 1, 0, 1}, {64, 3, 1, 0, 0}, {128, 2, 1, 0, 1}, {128, 3, 1, 1, 1}, {256, 2, 1, 0, 2},
    {256, 3, 1, 0, 2}, {512, 3, 1, 0, 1},
    // FP16 storage (400-768: the XCD-ordered strided tile, one FP16 forward
    // sweep, BF16 the same: 640^3 3.70 -> 2.56 ms, 768^3 5.80 -> 4.00;
    // 512 x: the non-temporal contiguous tile on four waves of
    // resident blocks, 0.217 -> 0.195 ms in both directions; the same for BF16)
    {32, 0, 2, 0, 2}, {32, 1, 2, 0, 0}, {48, 0, 2, 0, 0}, {48, 1, 2, 0, 2}, {60, 0, 2, 0, 1}, {60, 1, 2, 0, 0},
    {64, 0, 2, 0, 0}, {64, 1, 2, 0, 1}, {72, 0, 2, 0, 2}, {72, 1, 2, 0, 0}, {80, 0, 2, 0, 4}, {80, 1, 2, 0, 2},
    {96, 0, 2, 0, 4}, {96, 1, 2, 0, 0}, {100, 0, 2, 0, 1}, {100, 1, 2, 0, 4}, {128, 0, 2, 1, 1},
    {128, 1, 2, 1, 4}, {256, 0, 2, 1, 0}, {256, 1, 2, 2, 1}, {384, 0, 2, 0, 0}, {384, 1, 2, 0, 1},
    {512, 0, 2, 3, 4}, {512, 1, 2, 6, 1}, {1024, 0, 2, 3, 4}, {1024, 1, 2, 7, 1},
    {400, 1, 2, 6, 0}, {576, 1, 2, 6, 0}, {640, 1, 2, 6, 0}, {720, 0, 2, 3, 0}, {720, 1, 2, 7, 0},
    {768, 1, 2, 7, 0},
    // BF16 storage
    {32, 0, 3, 0, 0}, {32, 1, 3, 0, 2}, {48, 0, 3, 0, 2}, {48, 1, 3, 0, 2}, {60, 0, 3, 0, 4}, {60, 1, 3, 0, 1},
    {64, 0, 3, 0, 2}, {64, 1, 3, 0, 4}, {72, 0, 3, 0, 4}, {72, 1, 3, 0, 4}, {80, 0, 3, 0, 1}, {80, 1, 3, 0, 2},
    {96, 0, 3, 0, 0}, {96, 1, 3, 0, 2}, {100, 0, 3, 0, 2}, {100, 1, 3, 0, 0}, {128, 0, 3, 1, 2},
    {128, 1, 3, 1, 0}, {256, 0, 3, 1, 0}, {256, 1, 3, 2, 1}, {384, 0, 3, 0, 0}, {384, 1, 3, 0, 1},
    {512, 0, 3, 3, 4}, {512, 1, 3, 6, 1}, {1024, 0, 3, 3, 4}, {1024, 1, 3, 7, 1},
    {400, 1, 3, 6, 0}, {576, 1, 3, 6, 0}, {640, 1, 3, 6, 0}, {720, 0, 3, 3, 0}, {720, 1, 3, 7, 0},
    {768, 1, 3, 7, 0},
};

// Forward-only choices, looked up before the table above by forward plans:
// where the best configuration for both directions together is not the best
// forward one (512 strided complex64 passes with no per-axis choice, such as
// the convolution plan's: the 1024-thread wide tile is the fastest forward
// but spills in its inverse).
const Builtin kBuiltinForward[] = {
    {512, 1, 0, 2, 1},
};

// Per-axis choices (n kind dtype axis candidate waves), looked up before
// the two tables above, all one line per lane; at 512 in 256-thread blocks
// (two share a CU), one block per tile, unless noted: the y pass (4 KiB
// stride for complex64) with non-temporal loads, complex64 with the tiles
// in reverse order (0.377 -> 0.350 ms), 16-bit storage in the
// XCD-contiguous order (0.230 -> 0.213 ms); a real grid's half-spectrum y
// pass, whose rows are not whole 128-byte lines, takes the plain twin (the
// XCD-ordered plain kernel, 0.20 ms); the complex64 z pass (2 MiB stride)
// with non-temporal loads and stores.
struct BuiltinAxis {
    int n, kind, dtype, axis, cand, waves;
};
const BuiltinAxis kBuiltinAxis[] = {
    // complex64 at 1024, 512-thread blocks, one block per tile: y in the
    // XCD-contiguous order (3.40 -> 3.29 ms), z non-temporal (4.16 -> 3.97)
    {1024, 1, 0, 1, 8, 0},
    {1024, 1, 0, 2, 7, 0},
    // 16-bit storage at 1024: y in dispatch order, plain (2.29 -> 2.23 ms
    // FP16, 2.25 -> 2.16 BF16); z in XCD-contiguous order, non-temporal, one
    // block per tile (2.91 -> 2.86)
    {1024, 1, 2, 1, 6, 1},
    {1024, 1, 2, 2, 9, 0},
    {1024, 1, 3, 1, 6, 1},
    {1024, 1, 3, 2, 9, 0},
    {512, 1, 0, 1, 15, 0},
    // complex64 z at 512: the same 256-thread blocks, non-temporal, the
    // candidate that copies half a tile into LDS, one block per tile (so each
    // block copies the first half of its own tile): 0.400 -> 0.382 ms on two
    // waves of resident blocks, then 0.382 -> 0.371 ms with one block per
    // tile (both directions, two GPUs; real plans 0.618 -> 0.615 ms forward,
    // 0.684 -> 0.677 ms backward)
    {512, 1, 0, 2, 18, 0},
    {512, 1, 2, 1, 14, 0},
    {512, 1, 3, 1, 14, 0},
    // complex128 y at 512: the wide tile with fewer threads, one block per
    // tile.  The 16-line tile in the XCD-contiguous order (candidate 6) runs
    // the y pass itself faster (0.79-0.80 against 0.80-0.81 ms), but the z
    // pass after it takes 0.91 against 0.86 ms: the transform is faster with
    // this one (2.404-2.423 against 2.440-2.461 ms, both directions)
    {512, 1, 1, 1, 4, 0},
    // 16-bit storage z at 512: 64-line tiles loading the next tile into
    // registers during the current one (BF16 0.272-0.277 -> 0.264-0.268 ms,
    // FP16 the same within the spread, both directions, two GPUs); FP16 with
    // the non-temporal hint on those loads (0.242-0.243 -> 0.238-0.239 ms,
    // transform 0.675-0.679 -> 0.665-0.666 ms; on BF16 the hint gains nothing)
    {512, 1, 2, 2, 23, 1},
    {512, 1, 3, 2, 20, 1},
};

std::mutex g_mu;
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_mem;  // (n, kind, dtype, axis or -1)

// The last matching line for this axis (axis >= 0) or for any axis (axis -1).
bool read_file(const char *path, int n, int kind, int dtype, int axis, int *cand, int *waves) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    int a, b, c, d, e, x;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        const int got = std::sscanf(line, "%d %d %d %d %d %d", &a, &b, &c, &d, &e, &x);
        if (got < 5 || a != n || b != kind || c != dtype) continue;
        if ((axis < 0 && got == 5) || (axis >= 0 && got == 6 && x == axis)) {
            *cand = d;
            *waves = e;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}
}  // namespace

bool wisdom_lookup(int n, int kind, int dtype, int dir, int axis, int *cand, int *waves) {
    std::lock_guard<std::mutex> lk(g_mu);
    const char *path = std::getenv("CROFT_WISDOM");
    if (path && *path) {
        if (axis >= 0 && read_file(path, n, kind, dtype, axis, cand, waves)) return true;
        if (read_file(path, n, kind, dtype, -1, cand, waves)) return true;
    }
    const int axes[2] = {axis, -1};
    for (int i = axis >= 0 ? 0 : 1; i < 2; ++i) {
        auto it = g_mem.find({n, kind, dtype, axes[i]});
        if (it != g_mem.end()) {
            *cand = it->second.first;
            *waves = it->second.second;
            return true;
        }
    }
    if (axis >= 0) {
        for (const BuiltinAxis &b : kBuiltinAxis) {
            if (b.n == n && b.kind == kind && b.dtype == dtype && b.axis == axis) {
                *cand = b.cand;
                *waves = b.waves;
                return true;
            }
        }
    }
    if (dir == -1) {
        for (const Builtin &b : kBuiltinForward) {
            if (b.n == n && b.kind == kind && b.dtype == dtype) {
                *cand = b.cand;
                *waves = b.waves;
                return true;
            }
        }
    }
    for (const Builtin &b : kBuiltin) {
        if (b.n == n && b.kind == kind && b.dtype == dtype) {
            *cand = b.cand;
            *waves = b.waves;
            return true;
        }
    }
    return false;
}

void wisdom_record(int n, int kind, int dtype, int axis, int cand, int waves, bool persist) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_mem[{n, kind, dtype, axis}] = {cand, waves};
    const char *path = std::getenv("CROFT_WISDOM");
    if (!persist || !path || !*path) return;
    if (FILE *f = std::fopen(path, "a")) {
        if (axis >= 0) std::fprintf(f, "%d %d %d %d %d %d\n", n, kind, dtype, cand, waves, axis);
        else std::fprintf(f, "%d %d %d %d %d\n", n, kind, dtype, cand, waves);
        std::fclose(f);
    }
}

// ---- slab count K of the pipelined schedule ----
// File lines "slabs nx ny nz dtype K"; the same lookup order as the pass
// choices (file, this process, built-in).  No built-in grid takes K > 1: on
// an MI355X the measured gain of the slab schedule at 512^3 and 1024^3 is
// within the spread of repeated runs.
namespace {
std::map<std::tuple<int, int, int, int>, int> g_slabs;  // (nx, ny, nz, dtype) -> K

bool read_slabs(const char *path, int nx, int ny, int nz, int dtype, int *k) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    int a, b, c, d, e;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "slabs %d %d %d %d %d", &a, &b, &c, &d, &e) != 5) continue;
        if (a == nx && b == ny && c == nz && d == dtype && e >= 1 && nz % e == 0) {
            *k = e;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}
}  // namespace

bool slab_wisdom_lookup(int nx, int ny, int nz, int dtype, int *k) {
    std::lock_guard<std::mutex> lk(g_mu);
    const char *path = std::getenv("CROFT_WISDOM");
    if (path && *path && read_slabs(path, nx, ny, nz, dtype, k)) return true;
    auto it = g_slabs.find({nx, ny, nz, dtype});
    if (it != g_slabs.end()) {
        *k = it->second;
        return true;
    }
    return false;
}

void slab_wisdom_record(int nx, int ny, int nz, int dtype, int k, bool persist) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_slabs[{nx, ny, nz, dtype}] = k;
    const char *path = std::getenv("CROFT_WISDOM");
    if (!persist || !path || !*path) return;
    if (FILE *f = std::fopen(path, "a")) {
        std::fprintf(f, "slabs %d %d %d %d %d\n", nx, ny, nz, dtype, k);
        std::fclose(f);
    }
}

}  // namespace croft
