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
// stay out of LDS, for a sector small enough to hold them in LDS too; only its
// distances take LDS.  The pooled kernels of at most two waves per SIMD hold
// such a sector's coordinates in registers when it has at most 4096 points and
// k <= 64; otherwise they read them from global memory (L2).
constexpr int kItemXyzNotInLds = 1 << 8;

// One sector's work, as the batch queue hands it out (40 bytes).
struct WorkItem {
    int64_t xyz_offset;   // first point of the sector, in points, into xyz_all
    int64_t out_offset;   // first output of the sector, in indices, into out_all
    int32_t n;            // points in the sector
    int32_t c;            // samples of the sector
    int32_t k;            // NPDU window parameter, < 0 = off
    int32_t start;        // local start point (start mod n)
    int32_t base;         // index of the sector's first point inside its cloud
    int32_t flags;        // NPDU readings (kNpdu*) and kItemXyzNotInLds; 0 without NPDU
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
constexpr int kMaxPoolWaves = 16;
constexpr int kMaxPoolGroups = 512;     // pooled workgroups of one launch, at most
constexpr int kMaxLocalQueues = 64;     // queues of one pooled workgroup (one per lane)
constexpr int kRoundRing = 4;           // rounds a pooled workgroup takes sectors from at once
static_assert((kRoundRing & (kRoundRing - 1)) == 0, "ring slots by mask");
// LDS the pooled kernel declares statically (page mask, lock, the claim
// counters of kRoundRing rounds, round and exit words), bounded: the pool
// takes the rest of the CU's LDS.
constexpr int kPoolStaticLdsBytes = 2048;
// LDS pages of each of `groups` pooled workgroups sharing a CU that holds
// cu_pool_pages pages next to one workgroup's static LDS (each further
// workgroup brings its own static LDS).
constexpr int pool_pages_per_group(int cu_pool_pages, int groups) {
    return (cu_pool_pages * kPoolPageBytes - (groups - 1) * kPoolStaticLdsBytes) / (groups * kPoolPageBytes);
}
constexpr int kSeedSleepCycles = 127 * 64;   // one s_sleep(127)

// Whether a pooled NPDU sector keeps its coordinates in LDS, from its item flags.
constexpr bool npdu_item_xyz_in_lds(int n, int flags) {
    return npdu_r_for(n) <= 2 && (flags & kItemXyzNotInLds) == 0;
}
constexpr int npdu_pool_pages(int n, bool xyz_in_lds) {
    return (4 * npdu_lds_words(n, xyz_in_lds) + kPoolPageBytes - 1) / kPoolPageBytes;
}
// Pages of the sector the built-in placement gives (coordinates in LDS up to 8192 points).
constexpr int npdu_pool_pages(int n) { return npdu_pool_pages(n, npdu_r_for(n) <= 2); }
// Sectors the light pooled kernels serve (the narrow loop with coordinates
// read from L2 is all they hold, which keeps them small enough for six or
// eight waves per SIMD): at most 4096 points, 0 <= k <= 64, coordinates out
// of LDS.
constexpr bool npdu_item_lite(int n, int k, int flags) {
    return n <= 4096 && k >= 0 && k <= 64 && (flags & kItemXyzNotInLds) != 0;
}

// A pooled launch assigns every sector to one workgroup when the plan is
// built (balanced by estimated cost), for every round alike.  Inside a
// workgroup its sectors are queued by the pages they take: a queue holds
// items [first, first + count) of the plan, longest first, that all take
// `pages` pages (at least what each needs); the first `seeded` are the first
// sectors of the workgroup's waves in round 0 (not queued in that round).
struct PoolQueue {
    int32_t first;
    int32_t count;
    int32_t pages;
    int32_t seeded;
};
static_assert(sizeof(PoolQueue) == 16, "pool queue layout");

// A pooled workgroup's queues: [queue_first, queue_first + queues) of the
// plan's queue table, highest priority first, at most kMaxLocalQueues.
struct PoolGroup {
    int32_t queue_first;
    int32_t queues;
};
static_assert(sizeof(PoolGroup) == 8, "pool group layout");

// First sector of each pooled wave, assigned when the plan is built: the
// item, its first page, the pages it takes and how many sleep periods
// (kSeedSleepCycles each) the wave waits before loading it; item -1 if none.
struct PoolSeed {
    int32_t item;
    int16_t page;
    uint8_t pages;
    uint8_t sleeps;
};
static_assert(sizeof(PoolSeed) == 8, "pool seed layout");
static_assert(kMaxPoolPages < 256, "seed pages in a byte");

// One cloud's points, for the optional input check.
struct CheckSeg {
    int64_t offset;   // first point of the cloud, in points
    int32_t n;
    int32_t pad;
};

// Device workspace of a batch plan:
//   [bucket counters (63) | status word | pool groups (512 x 8 B) |
//    pool seeds (512 x 16 x 8 B) | work items | pool queues (at most one per item)]
constexpr size_t kCounterBytes = 256;
constexpr int kStatusWord = (int)(kCounterBytes / sizeof(unsigned)) - 1;   // set by a wave that gave up
constexpr int kMaxBuckets = kStatusWord;
constexpr size_t kPoolGroupOffset = kCounterBytes;
constexpr size_t kPoolSeedOffset = kPoolGroupOffset + (size_t)kMaxPoolGroups * sizeof(PoolGroup);
constexpr size_t kItemsOffset = kPoolSeedOffset + (size_t)kMaxPoolGroups * kMaxPoolWaves * sizeof(PoolSeed);
static_assert(kItemsOffset % 256 == 0, "work items start 256-byte aligned");
constexpr int kResetWords = (int)(kCounterBytes / sizeof(unsigned));   // counters and status, cleared per launch

// The pool queue table follows the work items (16-byte aligned).
constexpr size_t pool_queue_offset(int64_t items) {
    return (kItemsOffset + (size_t)(items < 0 ? 0 : items) * sizeof(WorkItem) + 15) / 16 * 16;
}
// Workspace of a plan of `items` work items: room for a queue per item, the
// most a plan can have.
constexpr size_t workspace_bytes_for_items(int64_t items) {
    return items <= 0 ? 0 : (pool_queue_offset(items) + (size_t)items * sizeof(PoolQueue) + 255) / 256 * 256;
}

}  // namespace afps
