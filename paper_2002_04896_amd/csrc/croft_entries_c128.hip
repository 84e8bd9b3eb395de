// croft_entries_c128.hip -- compiled static configurations for complex128 storage (FP64 compute).
// Candidate 0 of every length is the default; the autotuner (CROFT_MEASURE)
// and the wisdom tables choose among the others.
#include <vector>

#include "croft_device.h"

namespace croft {
namespace dev {

#define DEF(N) make_entry<N, kContiguous, StC128, 16, kC128>(0), make_entry<N, kStrided, StC128, 16, kC128>(0), make_real_entry<N, StC128, 16, kC128>(), \
               make_conv_entry<N, StC128, 16, kC128>(0)
// contiguous: 1 padded LDS lines, 2 no prefetch;
// strided: 1 no prefetch, 2 wide tile (EW elements per thread, LW lines), 3 wide tile with prefetch,
// 4 wide tile with fewer threads (EW2 elements per thread, LW2 lines),
// 5 wide tile with non-temporal loads and stores; contiguous 3: non-temporal;
// fused multiply pass: 0 default shape, 1 wide tile (EW, LW); strided 512: 6, 7, 8 are 1, 2, 4
// with each XCD taking a contiguous run of tiles, 9 and 10 are 4 and 8 with non-temporal loads
// and stores
#define CAND(N, EW, LW, EW2, LW2)                                                \
    make_entry<N, kContiguous, StC128, 16, kC128, 0, 0, 1, 1>(1),                 \
        make_entry<N, kContiguous, StC128, 16, kC128, 0, 0, 0, 0>(2),             \
        make_entry<N, kStrided, StC128, 16, kC128, 0, 0, 0, 0>(1),                \
        make_entry<N, kStrided, StC128, 16, kC128, EW, LW, 0, 0>(2),              \
        make_entry<N, kStrided, StC128, 16, kC128, EW, LW, 0, 1>(3),              \
        make_entry<N, kStrided, StC128, 16, kC128, EW2, LW2, 0, 0>(4), \
        make_entry<N, kContiguous, StC128, 16, kC128, 0, 0, 0, 1, 1>(3), \
        make_entry<N, kStrided, StC128, 16, kC128, EW, LW, 0, 0, 1>(5), \
        make_conv_entry<N, StC128, 16, kC128, EW, LW>(1)

// the larger compiled 2^a 3^b 5^c lengths: the streaming contiguous tile, the
// strided tile without prefetch, and both strided tiles in the XCD-contiguous
// order (numbered as the complex64 ones)
#define XCAND(N)                                                                   \
    make_entry<N, kContiguous, StC128, 16, kC128, 0, 0, 0, 1, 1>(3),               \
        make_entry<N, kStrided, StC128, 16, kC128, 0, 0, 0, 0>(1),                 \
        make_entry<N, kStrided, StC128, 16, kC128, 0, 0, 0, 0, 0, 1>(6),           \
        make_entry<N, kStrided, StC128, 16, kC128, 0, 0, 0, 1, 0, 1>(7)

std::vector<Entry> entries_c128() {
    return {
        DEF(2),   DEF(4),   DEF(8),   DEF(16),   DEF(32),   DEF(64),   DEF(128),
        DEF(256), DEF(512), DEF(1024), DEF(2048), DEF(4096), DEF(48),  DEF(60),
        DEF(72),  DEF(80),  DEF(96),  DEF(100), DEF(384), DEF(120), DEF(160),
        DEF(192), DEF(240), DEF(320), DEF(480), DEF(200), DEF(288), DEF(360),
        DEF(400), DEF(576), DEF(640), DEF(720), DEF(768), DEF(960),
        CAND(128, 8, 16, 16, 16), CAND(256, 8, 16, 16, 16), CAND(512, 8, 16, 16, 16), CAND(1024, 16, 8, 32, 8),
        make_entry<512, kStrided, StC128, 16, kC128, 0, 0, 0, 0, 0, 1>(6),
        make_entry<512, kStrided, StC128, 16, kC128, 8, 16, 0, 0, 0, 1>(7),
        make_entry<512, kStrided, StC128, 16, kC128, 16, 16, 0, 0, 0, 1>(8),
        make_entry<512, kStrided, StC128, 16, kC128, 16, 16, 0, 0, 1>(9),
        make_entry<512, kStrided, StC128, 16, kC128, 16, 16, 0, 0, 1, 1>(10),
        XCAND(400), XCAND(480), XCAND(576), XCAND(640), XCAND(720), XCAND(768), XCAND(960),
        make_real_entry<256, StC128, 16, kC128, 1>(),
    };
}

}  // namespace dev
}  // namespace croft
