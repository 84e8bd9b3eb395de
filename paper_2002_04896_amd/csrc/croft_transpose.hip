// croft_transpose.hip -- the standalone transpose of the unfused schedule
// (CROFT_UNFUSED): the paper's Option 2, a plan without overlap whose
// pack / all-to-all / unpack between the axis passes are separate sweeps
// (Section 5.1).  On one GPU each exchange becomes a permutation of the
// whole grid through LDS tiles, kept only as the measured baseline of the
// fused passes.
#include <hip/hip_runtime.h>

#include "croft_internal.h"

namespace croft {
namespace {

// Input element (i0, i1, i2) (dims d0, d1, d2, i0 fastest) goes to output
// offset i0 so0 + i1 so1 + i2 so2, where input axis b is the output's
// fastest (so_b == 1) and c is the remaining axis.  A block moves a tile of
// 64 values of axis 0 by 64 values of axis b at one value of axis c: it
// reads 64 rows along axis 0 (contiguous in the input), and writes 64 rows
// along axis b (contiguous in the output) out of LDS.
struct PermuteArgs {
    const void *in;
    void *out;
    long long d[3];
    long long so[3];
    int b, c;
    long long ta, tb;  // tiles along axis 0 and axis b
};

constexpr int kTile = 64;

template <typename E>
__global__ void __launch_bounds__(256) permute_tiles(const PermuteArgs a) {
    __shared__ E tile[kTile][kTile + 1];  // [row along axis b][value along axis 0]; padded
    const E *in = reinterpret_cast<const E *>(a.in);
    E *out = reinterpret_cast<E *>(a.out);
    long long blk = blockIdx.x;
    const long long ia = blk % a.ta;
    blk /= a.ta;
    const long long ib = blk % a.tb;
    const long long ic = blk / a.tb;
    const long long a0 = ia * kTile, b0 = ib * kTile;
    const long long si[3] = {1, a.d[0], a.d[0] * a.d[1]};
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long db = a.d[a.b];
    const long long base_in = ic * si[a.c] + b0 * si[a.b] + a0;
#pragma unroll 4
    for (int r = w; r < kTile; r += 4) {
        if (a0 + lane < a.d[0] && b0 + r < db) tile[r][lane] = in[base_in + (long long)r * si[a.b] + lane];
    }
    __syncthreads();
    const long long base_out = ic * a.so[a.c] + a0 * a.so[0] + b0;
#pragma unroll 4
    for (int r = w; r < kTile; r += 4) {
        if (a0 + r < a.d[0] && b0 + lane < db) out[base_out + (long long)r * a.so[0] + lane] = tile[lane][r];
    }
}

}  // namespace

hipError_t launch_permute(int dtype, const void *in, void *out, const long long d[3], const long long so[3], int b,
                          hipStream_t stream) {
    if (b != 1 && b != 2) return hipErrorInvalidValue;
    PermuteArgs a;
    a.in = in;
    a.out = out;
    for (int i = 0; i < 3; ++i) {
        a.d[i] = d[i];
        a.so[i] = so[i];
    }
    a.b = b;
    a.c = 3 - b;
    a.ta = (d[0] + kTile - 1) / kTile;
    a.tb = (d[b] + kTile - 1) / kTile;
    const long long blocks = a.ta * a.tb * d[a.c];
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    void *args[] = {&a};
    const void *f = dtype == kC128 ? reinterpret_cast<const void *>(&permute_tiles<double2>)
                                   : reinterpret_cast<const void *>(&permute_tiles<float2>);
    if (dtype != kC64 && dtype != kC128) return hipErrorInvalidValue;
    return hipLaunchKernel(f, dim3((unsigned)blocks), dim3(256), args, 0, stream);
}

}  // namespace croft
