// Data layouts shared by the batch planner (host only) and the kernels: work
// items, pool queues and seeds, LDS pages of an NPDU sector, and the layout
// of a batch plan's device workspace.  Plain C++ (no HIP headers), so the
// planner builds and is tested on a machine without a GPU; the constexpr
// functions are usable in device code as well.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace afps {

// NPDU readings other than the default one, for points Sec. III-C leaves open
// (bit flags of the NPDU entry points and of a work item):
//   kNpduFirstFull : the first iteration updates every point of the sector;
//   kNpduShiftEdges: a window that would cross a sector edge is moved inward
//                    (keeping its size) instead of being truncated;
//   kNpduKWithSelf : the k updated points include the sample; the host turns
//                    it into k - 1 without the flag (the same window), so the
//                    kernels never see it.
constexpr int kNpduFirstFull = 1;
constexpr int kNpduShiftEdges = 2;
constexpr int kNpduKWithSelf = 4;
// Work-item flag set by the planner (not a reading): the sector's coordinates
// stay in global memory (L2) and only its distances take LDS, for a sector
// small enough to hold its coordinates in LDS too.
constexpr int kItemXyzInL2 = 1 << 8;

// One sector's work, as the batch queue hands it out (40 bytes).
struct WorkItem {
    int64_t xyz_offset;   // first point of the sector, in points, into xyz_all
    int64_t out_offset;   // first output of the sector, in indices, into out_all
    int32_t n;            // points in the sector
    int32_t c;            // samples of the sector
    int32_t k;            // NPDU window parameter, < 0 = off
    int32_t start;        // local start point (start mod n)
    int32_t base;         // index of the sector's first point inside its cloud
    int32_t flags;        // NPDU readings (kNpdu*) and kItemXyzInL2; 0 without NPDU
};
static_assert(sizeof(WorkItem) == 40, "work item layout");

// LDS of an NPDU sector of n points: one record per point ({D, x, y, z}, 16
// bytes, or D alone, 4 bytes), padded with one empty block of 64 points.
constexpr int npdu_padded_points(int n) { return ((n + 63) / 64 + 1) * 64; }
constexpr int npdu_lds_words(int n, bool xyz_in_lds) { return (xyz_in_lds ? 4 : 1) * npdu_padded_points(n); }

// Blocks of 64 points per lane register (R) of the NPDU sampler holding a
// sector of n points; 0 if n is too large.  Coordinates can stay in LDS only
// for R <= 2 (up to 8192 points).
constexpr int npdu_r_for(int n) { return n <= 4096 ? 1 : n <= 8192 ? 2 : n <= 16384 ? 4 : n <= 32768 ? 8 : 0; }
constexpr int kMaxNpduSector = 32768;
constexpr int kMaxNpduLdsXyz = 8192;   // largest sector whose coordinates fit in LDS records

// Pooled NPDU kernel: a workgroup owns a pool of LDS pages of 1 KB (64
// records of 16 bytes); a sector holds exactly npdu_pool_pages contiguous pages.
constexpr int kPoolPageBytes = 1024;
constexpr int kMaxPoolPages = 160;      // pages per workgroup, at most (used-mask of 3 words)
constexpr int kMaxPoolQueues = 128;     // two per lane in the queue scan
constexpr int kMaxPoolWaves = 16;
constexpr int kMaxPoolSeedGroups = 512;
constexpr int kSeedSleepCycles = 127 * 64;   // one s_sleep(127)

// Whether a pooled NPDU sector keeps its coordinates in LDS, from its item flags.
constexpr bool npdu_item_xyz_in_lds(int n, int flags) {
    return npdu_r_for(n) <= 2 && (flags & kItemXyzInL2) == 0;
}
constexpr int npdu_pool_pages(int n, bool xyz_in_lds) {
    return (4 * npdu_lds_words(n, xyz_in_lds) + kPoolPageBytes - 1) / kPoolPageBytes;
}
// Pages of the sector the built-in placement gives (coordinates in LDS up to 8192 points).
constexpr int npdu_pool_pages(int n) { return npdu_pool_pages(n, npdu_r_for(n) <= 2); }

// A queue of pooled sectors that all need the same pages, longest first:
// items [first, first + count) of the plan, of which the first `seeded` are
// the first sectors of waves in round 0 (they are not queued in that round).
struct PoolQueue {
    int32_t first;
    int32_t count;
    int32_t pages;     // pages every item of the queue needs
    int32_t seeded;
};
// Queue counters of one round of a pooled launch (one per queue).
constexpr int kRoundCounters = 128;
static_assert(sizeof(PoolQueue) == 16, "pool queue layout");

// First sector of each pooled wave, assigned when the plan is built: the
// item, its first page and how many sleep periods (kSeedSleepCycles each) the
// wave waits before loading it; item -1 if none.
struct PoolSeed {
    int32_t item;
    int16_t page;
    int16_t sleeps;
};
static_assert(sizeof(PoolSeed) == 8, "pool seed layout");

// One cloud's points, for the optional input check.
struct CheckSeg {
    int64_t offset;   // first point of the cloud, in points
    int32_t n;
    int32_t pad;
};

// Device workspace of a batch plan:
//   [bucket counters (63) | status word | pool queue counters (128) |
//    pool queue table (128 x 16 B) | pool seeds (512 x 16 x 8 B) | work items]
constexpr size_t kCounterBytes = 256;
constexpr int kStatusWord = (int)(kCounterBytes / sizeof(unsigned)) - 1;   // set by a wave that gave up
constexpr int kMaxBuckets = kStatusWord;
constexpr size_t kPoolCounterOffset = kCounterBytes;
constexpr size_t kPoolTableOffset = kPoolCounterOffset + kMaxPoolQueues * sizeof(unsigned);
constexpr size_t kPoolSeedOffset = kPoolTableOffset + kMaxPoolQueues * sizeof(PoolQueue);
constexpr size_t kItemsOffset = kPoolSeedOffset + (size_t)kMaxPoolSeedGroups * kMaxPoolWaves * sizeof(PoolSeed);
static_assert(kItemsOffset % 256 == 0, "work items start 256-byte aligned");
constexpr int kResetWords = (int)(kPoolTableOffset / sizeof(unsigned));   // counters and status, cleared per launch

constexpr size_t workspace_bytes_for_items(int64_t items) {
    return items <= 0 ? 0 : ((kItemsOffset + (size_t)items * sizeof(WorkItem)) + 255) / 256 * 256;
}
// A launch of several rounds adds the queue counters of every round after
// the work items.
constexpr size_t round_counters_bytes(int64_t rounds) {
    return rounds <= 0 ? 0 : ((size_t)rounds * kRoundCounters * sizeof(unsigned) + 255) / 256 * 256;
}

}  // namespace afps
