// croft_batch.hip -- the batched form: one launch per axis pass covering the
// tiles of every grid in a batch, or one cooperative launch for all passes
// (compiled lengths 48, 60, 64, 72, 80, 96, 100, 128; complex64 and
// complex128).
#include <hip/hip_runtime.h>

#include "croft_device.h"
#include "croft_internal.h"

namespace croft {
using namespace dev;

namespace {
}  // namespace

int batch_code(int n, int kind, int shape) {
    if (shape < 0 || shape >= kBatchShapes) return -1;
    for (int i = 0; i < 8; ++i)
        if (kBatchLengths[i] == n) return 2 * i + (kind == kStrided ? 1 : 0) + 16 * shape;
    return -1;
}

namespace {
template <class St>
void config_of(int code, BatchConfig *c) {
    const int i = (code % 16) / 2;
    const int kind = code % 2;
    const int shape = code / 16;
    c->n = kBatchLengths[i];
    c->kind = kind;
    c->shape = shape;
    c->threads_per_line = batch_threads(c->n, shape);
    c->lines = 256 / c->threads_per_line;
    size_t lds = 0;
    switch (code) {
#define CROFT_LDS(I, SH)                                                               \
    case 2 * I + 16 * SH: lds = BCfg<kBatchLengths[I], kContiguous, St, SH>::kLds; break; \
    case 2 * I + 1 + 16 * SH: lds = BCfg<kBatchLengths[I], kStrided, St, SH>::kLds; break;
        CROFT_LDS(0, 0) CROFT_LDS(1, 0) CROFT_LDS(2, 0) CROFT_LDS(3, 0) CROFT_LDS(4, 0) CROFT_LDS(5, 0)
        CROFT_LDS(6, 0) CROFT_LDS(7, 0) CROFT_LDS(0, 1) CROFT_LDS(1, 1) CROFT_LDS(2, 1) CROFT_LDS(3, 1)
        CROFT_LDS(4, 1) CROFT_LDS(5, 1) CROFT_LDS(6, 1) CROFT_LDS(7, 1)
#undef CROFT_LDS
        default: break;
    }
    c->lds = lds;
}
}  // namespace

bool batch_config(int code, int dtype, BatchConfig *c) {
    if (code < 0 || code >= 16 * batch_shape_count(dtype)) return false;
    if (dtype == kC64) config_of<StC64>(code, c);
    else if (dtype == kC128) config_of<StC128>(code, c);
    else return false;
    return true;
}

int batch_shape_count(int dtype) {
    return dtype == kC64 ? batch_shapes<StC64>() : (dtype == kC128 ? batch_shapes<StC128>() : 0);
}

const void *batch_kernel(int dtype, int inverse) {
    if (dtype == kC64)
        return inverse ? reinterpret_cast<const void *>(&fft_batch<StC64, true>)
                       : reinterpret_cast<const void *>(&fft_batch<StC64, false>);
    if (dtype == kC128)
        return inverse ? reinterpret_cast<const void *>(&fft_batch<StC128, true>)
                       : reinterpret_cast<const void *>(&fft_batch<StC128, false>);
    return nullptr;
}

hipError_t launch_batch(const void *items, int nitems, long long tiles, size_t lds, int dtype, int inverse,
                        const void *in, void *out, hipStream_t stream) {
    if (tiles <= 0 || nitems <= 0) return hipSuccess;
    if (tiles > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    BatchArgs b;
    b.items = reinterpret_cast<const BatchItem *>(items);
    b.nitems = nitems;
    b.in = in;
    b.out = out;
    void *args[] = {&b};
    return hipLaunchKernel(batch_kernel(dtype, inverse), dim3((unsigned)tiles), dim3(256), args, lds, stream);
}

size_t batch_item_bytes() { return sizeof(BatchItem); }

const void *batch_coop_kernel(int dtype, int inverse) {
    if (dtype == kC64)
        return inverse ? reinterpret_cast<const void *>(&fft_batch_coop<StC64, true>)
                       : reinterpret_cast<const void *>(&fft_batch_coop<StC64, false>);
    if (dtype == kC128)
        return inverse ? reinterpret_cast<const void *>(&fft_batch_coop<StC128, true>)
                       : reinterpret_cast<const void *>(&fft_batch_coop<StC128, false>);
    return nullptr;
}

hipError_t launch_batch_coop(const void *items, const int item_begin[4], const long long tiles[3], int blocks,
                             size_t lds, int dtype, int inverse, const void *in, void *out, hipStream_t stream) {
    if (tiles[0] + tiles[1] + tiles[2] <= 0) return hipSuccess;
    if (blocks < 1) return hipErrorInvalidConfiguration;
    BatchCoopArgs b;
    b.items = reinterpret_cast<const BatchItem *>(items);
    for (int i = 0; i < 4; ++i) b.item_begin[i] = item_begin[i];
    for (int i = 0; i < 3; ++i) b.tiles[i] = tiles[i];
    b.in = in;
    b.out = out;
    void *args[] = {&b};
    return hipLaunchCooperativeKernel(batch_coop_kernel(dtype, inverse), dim3((unsigned)blocks), dim3(256), args,
                                      (unsigned)lds, stream);
}

void batch_item_fill(void *dst, long long offset, long long tile_begin, long long es, long long nlines,
                     long long nw, long long ntiles, long long total, const void *tw, int code, int from_in) {
    BatchItem it;
    it.offset = offset;
    it.tile_begin = tile_begin;
    it.es = es;
    it.nlines = nlines;
    it.nw = nw;
    it.ntiles = ntiles;
    it.total = total;
    it.tw = tw;
    it.code = code;
    it.from_in = from_in;
    *reinterpret_cast<BatchItem *>(dst) = it;
}

}  // namespace croft
