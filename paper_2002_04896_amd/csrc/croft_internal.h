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
// kRealX: the x pass of a real transform; contiguous geometry over the
// half-length complex view of the real lines (n = nx / 2), spectra of
// n + 1 elements per line.
// kConvZ: the fused forward FFT / multiply / inverse FFT pass of a
// convolution plan; strided geometry on the half spectrum.
enum PassKind { kContiguous = 0, kStrided = 1, kRealX = 2, kConvZ = 3 };

// Line geometry of a pass kind: strided (lines (p, w), stride es) or
// contiguous (lines l, stride 1).
inline bool strided_kind(int kind) { return kind == kStrided || kind == kConvZ; }

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
    const void *func = nullptr;      // the __global__ function (forward)
    const void *func_inv = nullptr;  // the same configuration, inverse direction
    bool generic = false;            // runtime-radix kernel
    int candidate = 0;               // index among the compiled configurations
    int plain = -1;                  // non-temporal or whole-tile: the candidate to run instead where
                                     // rows are not whole 128-byte lines or tiles are not whole
    bool whole_tiles = false;        // needs es to be a multiple of the lines per tile
    int threads_per_line = 0;        // T
    int lines = 0;                   // L, lines per block
    int block = 0;                   // T * L
    size_t lds = 0;                  // dynamic LDS bytes per block
    int nstages = 0;
    int radix[kMaxStages] = {};
    int bluestein = 0;   // > 0: Bluestein's algorithm with this power-of-two
                         // convolution length (nstages / radix describe it)
    int resident = 0;    // blocks the device holds at once (0: unknown)
    int grid_waves = 1;  // static kernels: launch min(tiles, resident * grid_waves)
                         // blocks looping over tiles; 0 launches one block per tile
};

// Exponent addressing of the half-storage form.  For an element at line
// coordinate q (contiguous: q = l; strided: q = p) and position j in the line,
// with line-block index w (strided only, 0 otherwise):
//   input exponent index  = (q % qmod) * a0 + (q / qmod) * a1 + w * a2 + j * a3
//   output exponent index = (q % qmod) * b0 + (q / qmod) * b1 + w * b2
// Every q is below 2^31 (grids hold fewer than 2^31 elements), so q / qmod is
// (q qmul) >> qshift with qmul = floor(2^(31 + l) / qmod) + 1 and
// l = ceil(log2 qmod), qshift = 31 + l: exact for q < 2^31 (Granlund and
// Montgomery, division by invariant integers using multiplication, 1994,
// theorem 4.2).  qmod = 2^31 leaves q whole (no wrap); set it with
// set_exp_qmod.
struct ExpMap {
    long long qmod = 1LL << 31;
    unsigned long long qmul = (1ULL << 31) + 1;
    int qshift = 62;
    long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    long long b0 = 0, b1 = 0, b2 = 0;
};

inline void set_exp_qmod(ExpMap &m, long long qmod) {
    int l = 0;
    while ((1LL << l) < qmod) ++l;
    m.qmod = qmod;
    m.qmul = (unsigned long long)(((unsigned __int128)1 << (31 + l)) / (unsigned long long)qmod) + 1;
    m.qshift = 31 + l;
}

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
    const void *tw2 = nullptr; // kRealX: device twiddle table of length 2 n
    ExpMap em;
    const void *chirp = nullptr;  // Bluestein: exp(-pi i j^2 / n), j < n
    const void *bhat = nullptr;   // Bluestein: DFT of the conjugate chirp kernel, / m
    int dir = 0;               // 0: the plan's direction; else CROFT_FORWARD / CROFT_BACKWARD
    long long hx = 0;          // kConvZ: spectrum elements per x-line
};

struct Geometry {
    int nx, ny, nz;
};

// ---- kernels (croft_kernels.hip) ----
// Number of compiled static configurations for (n, kind, dtype).
int kernel_candidates(int n, int kind, int dtype);
// Look up compiled configuration `cand` (0 = default; an unknown index falls
// back to 0) for a pass; with force_generic, or when no static kernel exists,
// the runtime-radix kernel.  Returns false if no kernel can run it.
bool select_kernel(int n, int kind, int dtype, bool force_generic, int cand, KernelConfig *cfg);
// Tiles (blocks of work) of one launch of a pass.
long long pass_tiles(const PassLaunch &pl);
// Launch one pass.  `in`/`out` point at the first element of the lines the
// launch covers; exponent pointers likewise (half storage only).
// mul / partial: the multiplier and the energy partials of a kConvZ pass.
hipError_t launch_pass(const PassLaunch &pl, int dtype, const void *in, void *out,
                       const int8_t *in_exp, int8_t *out_exp, int inverse, hipStream_t stream,
                       const void *mul = nullptr, double *partial = nullptr);

// The runtime-radix fused multiply pass (kConvZ) for a 2^a 3^b 5^c length
// without a compiled one; false for other lengths and for half storage.
bool select_generic_conv(int n, int dtype, KernelConfig *cfg);

// Blocks a pass launches (persistent grids loop over the tiles).
long long pass_blocks(const PassLaunch &pl);

// energy[0] = sum of partial[0..n) in a fixed order (one block).
hipError_t launch_sum_partials(const double *partial, int n, double *energy, hipStream_t stream);

// ---- batched form (croft_batch.hip) ----
struct BatchConfig {
    int n = 0, kind = 0, shape = 0, threads_per_line = 0, lines = 0;
    size_t lds = 0;
};
// Tile shapes the batched kernel compiles per (length, kind) for a dtype
// (shape 0 is the default; the autotuner picks among them), and the wisdom
// kinds that record the choice: kBatchWisdomKind + kind.
int batch_shape_count(int dtype);
constexpr int kBatchWisdomKind = 4;
// Code of a (length, kind, shape) the batched kernel compiles, -1 if none.
int batch_code(int n, int kind, int shape = 0);
bool batch_config(int code, int dtype, BatchConfig *c);
const void *batch_kernel(int dtype, int inverse);
size_t batch_item_bytes();
void batch_item_fill(void *dst, long long offset, long long tile_begin, long long es, long long nlines,
                     long long nw, long long ntiles, long long total, const void *tw, int code, int from_in);
const void *batch_coop_kernel(int dtype, int inverse);
// One cooperative launch of `blocks` blocks (all resident) over every pass of
// every grid in the table: segments of pass p at [item_begin[p],
// item_begin[p+1]), tiles[p] tiles each, the passes separated by grid-wide
// barriers.
hipError_t launch_batch_coop(const void *items, const int item_begin[4], const long long tiles[3], int blocks,
                             size_t lds, int dtype, int inverse, const void *in, void *out, hipStream_t stream);
// One launch over `tiles` tiles described by the device array `items`.
hipError_t launch_batch(const void *items, int nitems, long long tiles, size_t lds, int dtype, int inverse,
                        const void *in, void *out, hipStream_t stream);

// ---- standalone transpose of the unfused schedule (croft_transpose.hip) ----
// Permute a complex64/complex128 3D array: input element (i0, i1, i2) of
// dims d (i0 fastest) goes to output offset i0 so[0] + i1 so[1] + i2 so[2];
// input axis b (1 or 2) must be the output's fastest (so[b] == 1).  Out of
// place.
hipError_t launch_permute(int dtype, const void *in, void *out, const long long d[3], const long long so[3], int b,
                          hipStream_t stream);

// ---- allocation-free half-storage execute (croft_noalloc.hip) ----
// Bytes of the static per-GPU scratch array that holds the intermediate
// exponents of croft_execute_scaled_noalloc.
constexpr size_t kNoAllocScratchBytes = (size_t)4 << 20;
// The address of `device`'s copy of that array (looked up with
// hipGetSymbolAddress on the first call for a device, which must then be
// the current one; cached afterwards).
hipError_t noalloc_scratch(int device, int8_t **ptr);

// ---- wisdom (croft_tune.cpp) ----
// dir: -1 forward, +1 backward, 0 a pass that runs in both directions (the
// forward-only built-in choices apply to -1 only).  axis: the grid axis of a
// strided pass (a choice for that axis first, then one for any axis), -1
// for the other kinds.
bool wisdom_lookup(int n, int kind, int dtype, int dir, int axis, int *cand, int *waves);
void wisdom_record(int n, int kind, int dtype, int axis, int cand, int waves, bool persist);
// Slab count K of the pipelined schedule for a grid and dtype (K divides nz).
bool slab_wisdom_lookup(int nx, int ny, int nz, int dtype, int *k);
void slab_wisdom_record(int nx, int ny, int nz, int dtype, int k, bool persist);
// The axis a pass's wisdom is keyed on.
inline int wisdom_axis(int kind, int axis) { return kind == kStrided ? axis : -1; }

// ---- planner (croft_plan.cpp) ----
bool smooth_length(int n);
int factorize(int n, int *radix);  // returns stage count, 0 if unsupported
// Forward twiddles w[m] = exp(-2 pi i m / n), m < n, computed in FP64 with
// octant symmetry, written as interleaved doubles (2n values).
void twiddles_fp64(int n, double *out);
// out[i] = in[i] rounded to nearest even FP32 (the tables of FP32-compute
// plans are the FP64 values rounded once).
void round_to_fp32(const double *in, size_t count, float *out);
// Bluestein's tables for length n and convolution length m >= 2n - 1:
// chirp[j] = exp(-pi i j^2 / n), j < n (2n doubles), and bhat = the m-point
// DFT of b, b[i] = b[m - i] = conj chirp[i] for i < n (zero elsewhere),
// divided by m (2m doubles).  All in FP64.
void bluestein_tables_fp64(int n, int m, double *chirp, double *bhat);
// Smallest power of two >= 2n - 1.
int bluestein_length(int n);
// The Bluestein kernel of a pass kind and dtype whose convolution has length
// m (a power of two, 16 .. 8192) with its launch shape: T threads per line,
// L lines per block, LDS bytes; func is NULL for any other m and where two
// line buffers do not fit in LDS (FP64 at 8192).
struct BluesteinLaunch {
    const void *func = nullptr;
    int T = 0, L = 0;
    size_t lds = 0;
};
BluesteinLaunch bluestein_kernel(int kind, int dtype, int m);

}  // namespace croft
