// croft_entries_c64.hip -- compiled static configurations for complex64 storage (FP32 compute).
// Candidate 0 of every length is the default; the autotuner (CROFT_MEASURE)
// and the wisdom tables choose among the others.
#include <vector>

#include "croft_device.h"

namespace croft {
namespace dev {

#define DEF(N) make_entry<N, kContiguous, StC64, 8, kC64>(0), make_entry<N, kStrided, StC64, 8, kC64>(0), make_real_entry<N, StC64, 8, kC64>(), \
               make_conv_entry<N, StC64, 8, kC64>(0)
// contiguous: 1 padded LDS lines, 2 no prefetch;
// strided: 1 no prefetch, 2 wide tile (EW elements per thread, LW lines), 3 wide tile with prefetch,
// 4 wide tile with fewer threads (EW2 elements per thread, LW2 lines),
// 5 wide tile with non-temporal loads and stores, 6 and 7 (lengths 512 and 1024) one
// line per lane (7 non-temporal), 8 and 9 (length 512) the same in 256-thread blocks
// (9 non-temporal), 10 and 11 those with an XCD-contiguous tile order (11 non-temporal);
// 12 and 13 (length 512) 8 with the non-temporal hint on the loads only and on the
// stores only, 14 is 12 in the XCD-contiguous order, 15 and 16 are 12 and 8 with the
// tiles in reverse order, 17 and 18 are 8 and 9 copying the first half of the next tile into LDS
// during the current one (whole tiles, persistent grids), 19 and 20 are 17 with the
// non-temporal hint on the loads only and on the stores only; at 1024, 8 and 9 are 6 and 7 with the
// XCD-contiguous order, 10 to 12 are 6 with that copy (non-temporal stores in 11, loads and stores
// in 12); contiguous 3:
// non-temporal;
// fused multiply pass: 0 default shape, 1 wide tile (EW, LW); strided 384: 6 and 7 are 1 and 0
// (without and with prefetch) in the XCD-contiguous tile order
#define CAND(N, EW, LW, EW2, LW2)                                                \
    make_entry<N, kContiguous, StC64, 8, kC64, 0, 0, 1, 1>(1),                 \
        make_entry<N, kContiguous, StC64, 8, kC64, 0, 0, 0, 0>(2),             \
        make_entry<N, kStrided, StC64, 8, kC64, 0, 0, 0, 0>(1),                \
        make_entry<N, kStrided, StC64, 8, kC64, EW, LW, 0, 0>(2),              \
        make_entry<N, kStrided, StC64, 8, kC64, EW, LW, 0, 1>(3),              \
        make_entry<N, kStrided, StC64, 8, kC64, EW2, LW2, 0, 0>(4), \
        make_entry<N, kContiguous, StC64, 8, kC64, 0, 0, 0, 1, 1>(3), \
        make_entry<N, kStrided, StC64, 8, kC64, EW, LW, 0, 0, 1>(5), \
        make_conv_entry<N, StC64, 8, kC64, EW, LW>(1)

// the larger compiled 2^a 3^b 5^c lengths (16-line strided tiles): the
// streaming contiguous tile, the strided tile without prefetch, and both
// strided tiles in the XCD-contiguous order (numbered as at 384)
#define XCAND(N)                                                                  \
    make_entry<N, kContiguous, StC64, 8, kC64, 0, 0, 0, 1, 1>(3),                 \
        make_entry<N, kStrided, StC64, 8, kC64, 0, 0, 0, 0>(1),                   \
        make_entry<N, kStrided, StC64, 8, kC64, 0, 0, 0, 0, 0, 1>(6),             \
        make_entry<N, kStrided, StC64, 8, kC64, 0, 0, 0, 1, 0, 1>(7)

std::vector<Entry> entries_c64() {
    return {
        DEF(2),   DEF(4),   DEF(8),   DEF(16),   DEF(32),   DEF(64),   DEF(128),
        DEF(256), DEF(512), DEF(1024), DEF(2048), DEF(4096), DEF(48),  DEF(60),
        DEF(72),  DEF(80),  DEF(96),  DEF(100), DEF(384), DEF(120), DEF(160),
        DEF(192), DEF(240), DEF(320), DEF(480), DEF(200), DEF(288), DEF(360),
        DEF(400), DEF(576), DEF(640), DEF(720), DEF(768), DEF(960),
        CAND(128, 16, 32, 32, 32), CAND(256, 16, 32, 32, 32), CAND(512, 16, 32, 32, 32), CAND(1024, 32, 16, 64, 16),
        make_lanes_entry<512, StC64, kC64, 0>(6), with_plain(make_lanes_entry<512, StC64, kC64, 3>(7), 6),
        make_lanes_entry<512, StC64, kC64, 0, 256>(8), with_plain(make_lanes_entry<512, StC64, kC64, 3, 256>(9), 8),
        make_lanes_entry<512, StC64, kC64, 0, 256, true>(10), with_plain(make_lanes_entry<512, StC64, kC64, 3, 256, true>(11), 10),
        with_plain(make_lanes_entry<512, StC64, kC64, 1, 256>(12), 8), with_plain(make_lanes_entry<512, StC64, kC64, 2, 256>(13), 8),
        with_plain(make_lanes_entry<512, StC64, kC64, 1, 256, true>(14), 10),
        with_plain(make_lanes_entry<512, StC64, kC64, 1, 256, false, true>(15), 10),
        make_lanes_entry<512, StC64, kC64, 0, 256, false, true>(16),
        make_lanes_entry<1024, StC64, kC64, 0>(6), with_plain(make_lanes_entry<1024, StC64, kC64, 3>(7), 6),
        make_lanes_entry<1024, StC64, kC64, 0, 512, true>(8), with_plain(make_lanes_entry<1024, StC64, kC64, 3, 512, true>(9), 8),
        with_plain(make_lanes_entry<1024, StC64, kC64, 0, 512, false, false, true>(10), 6),
        with_plain(make_lanes_entry<1024, StC64, kC64, 2, 512, false, false, true>(11), 6),
        with_plain(make_lanes_entry<1024, StC64, kC64, 3, 512, false, false, true>(12), 6),
        with_plain(make_lanes_entry<512, StC64, kC64, 0, 256, false, false, true>(17), 8),
        with_plain(make_lanes_entry<512, StC64, kC64, 3, 256, false, false, true>(18), 8),
        with_plain(make_lanes_entry<512, StC64, kC64, 1, 256, false, false, true>(19), 8),
        with_plain(make_lanes_entry<512, StC64, kC64, 2, 256, false, false, true>(20), 8),
        CAND(384, 16, 32, 32, 32),
        make_entry<384, kStrided, StC64, 8, kC64, 0, 0, 0, 0, 0, 1>(6),
        make_entry<384, kStrided, StC64, 8, kC64, 0, 0, 0, 1, 0, 1>(7),
        XCAND(400), XCAND(480), XCAND(576), XCAND(640), XCAND(720), XCAND(768), XCAND(960),
        make_real_entry<256, StC64, 8, kC64, 1>(), make_real_entry<512, StC64, 8, kC64, 1>(),
    };
}

}  // namespace dev
}  // namespace croft
