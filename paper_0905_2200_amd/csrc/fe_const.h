// fe_const.h -- sizes and classes shared by the host runtime, the device
// kernels and the host-only algorithms (plain C++: constexpr functions are
// usable from device code too).  Not part of the public ABI.
#pragma once

namespace fe {

constexpr int WAVE = 64;
constexpr int NMAX = 8;          // largest episode size
constexpr int KMAX = 16;         // slot-table entries kept per (candidate, segment)
// List-depth classes of the exact machine: classes 0..3 keep 1, 2, 4, 8
// windows per list in registers; class DEEP_CLS holds the candidates with a
// hop whose window bound hi/(hi-lo+1)+1 exceeds 8, whose lists are ring
// buffers in device memory (k_deep).
constexpr int NDCLS = 5;
constexpr int DEEP_CLS = 4;
constexpr int NKEYS = NMAX * NDCLS;
constexpr int TICK_LIMIT = 1 << 30;
constexpr int WPB = 4;           // waves per block in the Map kernels

// device status bits
constexpr int ST_UNSORTED = 1;
constexpr int ST_RANGE = 2;
constexpr int ST_BADCAND = 4;
constexpr int ST_INTERNAL = 8;

inline constexpr int dcls_depth(int c) { return 1 << c; }
// list-depth class of a candidate whose largest window bound is `bound`
inline constexpr int depth_class(int bound)
{
    return bound <= 1 ? 0 : bound <= 2 ? 1 : bound <= 4 ? 2 : bound <= 8 ? 3 : DEEP_CLS;
}
// live windows of one exact list for a hop (lo, hi]: hi/(hi-lo+1)+1
inline constexpr int window_bound(int lo, int hi) { return hi / (hi - lo + 1) + 1; }
// ints in one packed tile record: types[N][64], lo[N-1][64], hi[N-1][64]
inline constexpr int rec_ints(int N) { return (3 * N - 2) * WAVE; }

}  // namespace fe
