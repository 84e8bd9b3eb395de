// croft_entries_c16b.hip -- compiled static configurations for BF16 pair storage with per-line exponents (FP32 compute).
// Candidate 0 of every length is the default; the autotuner (CROFT_MEASURE)
// and the wisdom tables choose among the others.
#include <vector>

#include "croft_device.h"

namespace croft {
namespace dev {

#define DEF(N) make_entry<N, kContiguous, StHalf<true>, 4, kC16B>(0), make_entry<N, kStrided, StHalf<true>, 4, kC16B>(0)
// contiguous: 1 padded LDS lines, 2 no prefetch;
// strided: 1 no prefetch, 2 wide tile (EW elements per thread, LW lines), 3 wide tile with prefetch,
// 4 wide tile with fewer threads (EW2 elements per thread, LW2 lines),
// 5 wide tile with non-temporal loads and stores, 6 and 7 (lengths 512 and 1024) one
// line per lane (7 non-temporal), 8 and 9 (length 512) the same in 256-thread blocks
// (9 non-temporal), 10 and 11 those with an XCD-contiguous tile order (11 non-temporal),
// 12 and 13 8 with the non-temporal hint on the loads only and on the stores only, 14 is
// 12 in the XCD-contiguous order, 15 and 16 are 6 with the hint on the loads only and on
// the stores only; 17 and 18 are 6 and 16 copying the first half of the next tile into LDS
// during the current one (whole tiles, persistent grids); 19 and 20 are 16 and 6 loading
// the next tile into registers during the current one (persistent grids); 21 and 22
// are 8 and 9 with the copy of 17 (256-thread blocks, two per CU); 23 and 24 are 20 with
// the non-temporal hint on the loads and on the loads and stores; 25 and 26 are 12 and 8
// with the tiles in reverse order;
// at 1024, 8 and 9 are 6 and 7 with the XCD-contiguous order, 10 and 11 are 6 and 7 with that
// copy; contiguous 3: non-temporal
#define CAND(N, EW, LW, EW2, LW2)                                                \
    make_entry<N, kContiguous, StHalf<true>, 4, kC16B, 0, 0, 1, 1>(1),                 \
        make_entry<N, kContiguous, StHalf<true>, 4, kC16B, 0, 0, 0, 0>(2),             \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B, 0, 0, 0, 0>(1),                \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B, EW, LW, 0, 0>(2),              \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B, EW, LW, 0, 1>(3),              \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B, EW2, LW2, 0, 0>(4), \
        make_entry<N, kContiguous, StHalf<true>, 4, kC16B, 0, 0, 0, 1, 1>(3), \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B, EW, LW, 0, 0, 1>(5)

// the larger compiled 2^a 3^b 5^c lengths: the streaming contiguous tile, the
// strided tile without prefetch, and both strided tiles in the XCD-contiguous
// order (numbered as the complex64 ones)
#define XCAND(N)                                                                     \
    make_entry<N, kContiguous, StHalf<true>, 4, kC16B, 0, 0, 0, 1, 1>(3),                 \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B, 0, 0, 0, 0>(1),                   \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B, 0, 0, 0, 0, 0, 1>(6),             \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B, 0, 0, 0, 1, 0, 1>(7)

std::vector<Entry> entries_c16b() {
    return {
        DEF(2),   DEF(4),   DEF(8),   DEF(16),   DEF(32),   DEF(64),   DEF(128),
        DEF(256), DEF(512), DEF(1024), DEF(2048), DEF(4096), DEF(48),  DEF(60),
        DEF(72),  DEF(80),  DEF(96),  DEF(100), DEF(384), DEF(120), DEF(160),
        DEF(192), DEF(240), DEF(320), DEF(480), DEF(200), DEF(288), DEF(360),
        DEF(400), DEF(576), DEF(640), DEF(720), DEF(768), DEF(960),
        CAND(128, 16, 64, 32, 64), CAND(256, 16, 64, 32, 64), CAND(512, 16, 32, 32, 32), CAND(1024, 32, 16, 64, 16),
        make_lanes_entry<512, StHalf<true>, kC16B, 0>(6), with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 3>(7), 6),
        make_lanes_entry<512, StHalf<true>, kC16B, 0, 256>(8), with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 3, 256>(9), 8),
        make_lanes_entry<512, StHalf<true>, kC16B, 0, 256, true>(10), with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 3, 256, true>(11), 10),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 1, 256>(12), 8), with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 2, 256>(13), 8),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 1, 256, true>(14), 10),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 1>(15), 6), with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 2>(16), 6),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 0, 512, false, false, true>(17), 6),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 2, 512, false, false, true>(18), 6),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 2, 512, false, false, false, true>(19), 20),
        make_lanes_entry<512, StHalf<true>, kC16B, 0, 512, false, false, false, true>(20),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 0, 256, false, false, true>(21), 8),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 3, 256, false, false, true>(22), 8),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 1, 512, false, false, false, true>(23), 20),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 3, 512, false, false, false, true>(24), 20),
        with_plain(make_lanes_entry<512, StHalf<true>, kC16B, 1, 256, false, true>(25), 26),
        make_lanes_entry<512, StHalf<true>, kC16B, 0, 256, false, true>(26),
        make_lanes_entry<1024, StHalf<true>, kC16B, 0>(6), with_plain(make_lanes_entry<1024, StHalf<true>, kC16B, 3>(7), 6),
        make_lanes_entry<1024, StHalf<true>, kC16B, 0, 512, true>(8), with_plain(make_lanes_entry<1024, StHalf<true>, kC16B, 3, 512, true>(9), 8),
        with_plain(make_lanes_entry<1024, StHalf<true>, kC16B, 0, 512, false, false, true>(10), 6),
        with_plain(make_lanes_entry<1024, StHalf<true>, kC16B, 3, 512, false, false, true>(11), 6),
        XCAND(400), XCAND(480), XCAND(576), XCAND(640), XCAND(720), XCAND(768), XCAND(960),
    };
}

}  // namespace dev
}  // namespace croft
