// Arrival counters in the workspace's control region (shared by the kernels
// and the host-side workspace layout).
#pragma once

namespace ms {

// Eight group counters (one per XCD: workgroup id mod 8) and a top counter,
// one 128-byte cache line each: atomics are serialised per line at the memory
// side, so counters sharing a line would queue behind each other.
constexpr int kArriveGroups = 8;
constexpr int kArriveWords = kArriveGroups + 1;
constexpr int kArriveStride = 32;  // words
// word offsets of the two counter sets (forward and reverse scans)
constexpr int kCountersFilter = 0, kCountersTraj = kArriveWords * kArriveStride;
// the numeric status word (MAP_CHECK_FINITE) on a line of its own after them
constexpr int kStatusWord = 2 * kArriveWords * kArriveStride;
// the segment queue of the segment-local schedule (reset by its order kernel)
constexpr int kQueueWord = kStatusWord + kArriveStride;
constexpr int kCounterWords = kQueueWord + kArriveStride;

}  // namespace ms
