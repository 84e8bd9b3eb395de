// croft_internal.h -- declarations shared by the planner, the C ABI and the
// HIP kernels of the 3D FFT library (not installed; include/croft.h is the
// public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace croft {

constexpr int kMaxStages = 12;
constexpr int kMaxLength = 4096;

enum Dtype { kC64 = 0, kC128 = 1, kC16F = 2, kC16B = 3 };
enum PassKind { kContiguous = 0, kStrided = 1 };

inline size_t element_bytes(int dtype) {
    return dtype == kC128 ? 16 : (dtype == kC64 ? 8 : 4);
}

// How one axis pass is launched.  The kernels see a grid as lines of length n
// (the transformed axis) with element stride `es` (in elements):
//   contiguous (es == 1): line l starts at element l * n, l < nlines;
//   strided    (es  > 1): line (p, w) starts at p + w * es * n, p < es,
//                         w < nw; consecutive p are adjacent in memory and a
//                         block takes a tile of `lines` consecutive p.
struct KernelConfig {
    const void *func = nullptr;  // the __global__ function
    bool generic = false;        // runtime-radix kernel
    int threads_per_line = 0;    // T
    int lines = 0;               // L, lines per block
    int block = 0;               // T * L
    size_t lds = 0;              // dynamic LDS bytes per block
    int nstages = 0;
    int radix[kMaxStages] = {};
};

// Exponent addressing of the half-storage form.  For an element at line
// coordinate q (contiguous: q = l; strided: q = p) and position j in the line,
// with line-block index w (strided only, 0 otherwise):
//   input exponent index  = (q % qmod) * a0 + (q / qmod) * a1 + w * a2 + j * a3
//   output exponent index = (q % qmod) * b0 + (q / qmod) * b1 + w * b2
struct ExpMap {
    long long qmod = 1LL << 40;
    long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    long long b0 = 0, b1 = 0, b2 = 0;
};

// One launch of one pass over (a slab of) a grid.
struct PassLaunch {
    int axis = 0;
    int n = 1;
    int kind = kContiguous;
    long long es = 1;      // element stride
    long long nlines = 0;  // contiguous: lines; strided: es (the p range)
    long long nw = 1;      // strided: number of w
    KernelConfig cfg;
    const void *tw = nullptr;  // device twiddle table of length n (dtype's compute type)
    ExpMap em;
};

struct Geometry {
    int nx, ny, nz;
};

// ---- kernels (croft_kernels.hip) ----
// Look up the compiled configuration for a pass; generic == true falls back
// to the runtime-radix kernel.  Returns false if no kernel can run it.
bool select_kernel(int n, int kind, int dtype, bool force_generic, KernelConfig *cfg);

// Launch one pass.  `in`/`out` point at the first element of the lines the
// launch covers; exponent pointers likewise (half storage only).
hipError_t launch_pass(const PassLaunch &pl, int dtype, const void *in, void *out,
                       const int8_t *in_exp, int8_t *out_exp, int inverse, hipStream_t stream);

// ---- planner (croft_plan.cpp) ----
bool smooth_length(int n);
int factorize(int n, int *radix);  // returns stage count, 0 if unsupported
// Forward twiddles w[m] = exp(-2 pi i m / n), m < n, computed in FP64 with
// octant symmetry, written as interleaved doubles (2n values).
void twiddles_fp64(int n, double *out);

}  // namespace croft
