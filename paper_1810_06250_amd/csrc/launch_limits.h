// Launch-size arithmetic shared by the kernel launchers (plain C++, no HIP
// types, so that it can be checked on the host).
//
// A dispatch packet counts its grid in work-items with 32 bits per
// dimension, so one launch of B-thread workgroups holds at most
// floor((2^32 - 1) / B) workgroups.  Launchers whose grid grows with the
// number of lines of sight split the work into batches that respect this.
#pragma once

#include <stdint.h>

constexpr int64_t kMaxGridItems = 0xffffffffLL;

// Largest number of workgroups of `block_threads` work-items in one launch.
constexpr int64_t max_blocks(int64_t block_threads) { return kMaxGridItems / block_threads; }

// Largest number of items in one launch when every workgroup of
// `block_threads` work-items handles `items_per_block` of them.
constexpr int64_t max_items(int64_t items_per_block, int64_t block_threads)
{
    return max_blocks(block_threads) * items_per_block;
}

// LOS per launch of a tiled transform kernel: LOS tiles of `tile_los` lines
// of sight times `tiles_n` phi tiles, one workgroup each.  At least one LOS
// tile (a grid of tiles_n workgroups always fits: tiles_n < 2^13 for the
// largest phi grid a plan accepts).
constexpr int64_t max_los_tiled(int64_t tiles_n, int64_t tile_los, int64_t block_threads)
{
    const int64_t m = max_blocks(block_threads) / tiles_n;
    return (m > 0 ? m : 1) * tile_los;
}
