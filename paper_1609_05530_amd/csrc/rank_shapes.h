// rank_shapes.h — launch shapes of the workgroup rank kernel (rank_wg.h)
// and the built-in / candidate choices per size class.
#pragma once

namespace cpc {

constexpr int kRankClasses = 4;  // size classes of the workgroup path

// Launch shapes of the rank kernel (threads, items per thread, packed
// exchange): a subset of up to threads * items rows fits a shape. Ranks are
// exact integers under every shape, so the choice (made by the autotuner per
// size class) only affects speed. 64-bit keys always use the class's default
// shape, unpacked.
struct RankShape {
  int threads, items, cap, packed, merge;  // merge: merge sort instead of radix passes
  int trunc;  // radix passes over this many leading varying key bits, runs then ordered by counting (0: all)
};
constexpr int kNumRankShapes = 16;
constexpr RankShape kRankShapes[kNumRankShapes] = {
    {64, 8, 512, 0, 0, 0},      {256, 8, 2048, 0, 0, 0},    {128, 16, 2048, 0, 0, 0}, {512, 16, 8192, 0, 0, 0},
    {256, 32, 8192, 0, 0, 0},   {1024, 16, 16384, 0, 0, 0}, {512, 32, 16384, 0, 0, 0},
    {64, 8, 512, 1, 0, 0},      {256, 8, 2048, 1, 0, 0},    {128, 16, 2048, 1, 0, 0}, {512, 16, 8192, 1, 0, 0},
    {256, 32, 8192, 1, 0, 0},   {1024, 16, 16384, 1, 0, 0}, {512, 32, 16384, 1, 0, 0},
    {64, 8, 512, 0, 1, 0},
    {64, 8, 512, 0, 0, 24}};
// built-in choices (measured fastest on MI355X: packed words pay off where
// several workgroups share a CU, not at one workgroup per CU)
constexpr int kRankDefaultShape[kRankClasses] = {7, 9, 10, 5};
// Candidate shapes per size class (-1 terminated): one wave or one larger
// workgroup per subset for the smallest class, two thread / item splits for
// the others; each unpacked and packed; and, for the smallest class, the
// one-wave merge sort (measured on MI355X: about 5% faster than the radix
// passes below 512 rows, but 1.5x to 2.4x slower at 256 to 1024 threads,
// where its chains of dependent LDS reads are not hidden) and the one-wave
// sort truncated to 24 leading key bits (about 10% faster below 512 rows; at
// 256 to 1024 threads the ordering of the runs cost what the two skipped
// passes saved).
constexpr int kRankCandidates[kRankClasses][6] = {{7, 8, 0, 1, 14, 15}, {9, 8, 2, 1, -1, -1}, {10, 11, 3, 4, -1, -1},
                                                 {5, 6, 12, 13, -1, -1}};

}  // namespace cpc
