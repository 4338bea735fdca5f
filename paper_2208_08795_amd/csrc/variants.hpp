// Host-visible tables of compiled kernel variants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

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

// One sector's work, as the batch queue hands it out (40 bytes).
struct WorkItem {
    int64_t xyz_offset;   // first point of the sector, in points, into xyz_all
    int64_t out_offset;   // first output of the sector, in indices, into out_all
    int32_t n;            // points in the sector
    int32_t c;            // samples of the sector
    int32_t k;            // NPDU window parameter, < 0 = off
    int32_t start;        // local start point (start mod n)
    int32_t base;         // index of the sector's first point inside its cloud
    int32_t flags;        // NPDU readings (kNpdu* below), 0 without NPDU
};
static_assert(sizeof(WorkItem) == 40, "work item layout");

// Full-update sector kernels (kernels.hip): W waves, P slots per thread.
struct VariantEntry {
    int waves;              // W: waves per workgroup (64*W threads)
    int slots;              // P: point slots per thread; a sector holds <= 64*W*P points
    int lds_bytes;          // dynamic LDS (distances kept in LDS), 0 = in registers
    const void* direct;     // direct_kernel<P, W, DL>
    const void* persistent; // persistent_kernel<P, W, DL>
};

void register_variants_w1(std::vector<VariantEntry>& v);
void register_variants_w2(std::vector<VariantEntry>& v);
void register_variants_w4(std::vector<VariantEntry>& v);
void register_variants_w8(std::vector<VariantEntry>& v);
void register_variants_w16(std::vector<VariantEntry>& v);

// NPDU sector kernels (kernels_npdu.hip): one wave, blocks of 64 points whose
// maxima live in R registers (one block per lane).
struct NpduEntry {
    int chunk64;            // R: a sector holds <= 64*64*R points
    int xyz_in_lds;         // 1: x,y,z and D in LDS (16 B/point); 0: only D (4 B/point)
    const void* direct;
};
void register_npdu_variants(std::vector<NpduEntry>& v);

// LDS of an NPDU sector of n points: x, y, z (if held in LDS) and D arrays,
// each padded with one empty block of 64 points.
__host__ __device__ constexpr int npdu_padded_points(int n) { return ((n + 63) / 64 + 1) * 64; }
__host__ __device__ constexpr int npdu_lds_words(int n, bool xyz_in_lds) {
    return (xyz_in_lds ? 4 : 1) * npdu_padded_points(n);
}

// Pooled NPDU kernel (kernels_pool.hip): one workgroup per CU owns the CU's
// LDS (or two own half of it each) as pages of 1 KB (64 records of 16
// bytes); each of its W waves takes
// sectors from priority queues and holds exactly the pages its sector needs.
struct PoolQueue {
    int32_t first;     // items [first, first + count) of the plan, longest first
    int32_t count;
    int32_t pages;     // pages every item of the queue needs
    int32_t pad;
};
static_assert(sizeof(PoolQueue) == 16, "pool queue layout");
constexpr int kPoolPageBytes = 1024;
constexpr int kMaxPoolPages = 160;      // pages per workgroup, at most (used-mask of 3 words)
constexpr int kMaxPoolQueues = 128;     // two per lane in the queue scan
// First sector of each wave, assigned when the plan is built (no queue
// atomics at the start of a launch): the item, its first page and how many
// sleep periods (kSeedSleepCycles each) the wave waits before loading it;
// item -1 if none.  Seeds cover workgroups below kMaxPoolSeedGroups,
// kMaxPoolWaves waves each.
struct PoolSeed {
    int32_t item;
    int16_t page;
    int16_t sleeps;
};
static_assert(sizeof(PoolSeed) == 8, "pool seed layout");
constexpr int kSeedSleepCycles = 127 * 64;   // one s_sleep(127)
constexpr int kMaxPoolWaves = 8;
constexpr int kMaxPoolSeedGroups = 512;
// Timestamps of one sector of a pooled launch (afps_plan_launch_stamped):
// the shader clock (s_memtime, cycles) when its wave took it, when its points
// were in LDS and when its last pick was written; the constant-rate clock
// (s_memrealtime) at take and end, which gives the shader clock's rate; the
// wave's hardware id register (CU, SIMD, wave slot) and XCC id.
struct SectorStamp {
    uint64_t take, loaded, end;
    uint64_t take_rt, end_rt;
    int32_t item, n, c, k;
    uint32_t hw_id, xcc_id;
};
static_assert(sizeof(SectorStamp) == 64, "sector stamp layout");

// Arguments of the pooled NPDU kernel (passed by value).
struct PoolArgs {
    const float* xyz_all;
    int32_t* out_all;
    const WorkItem* items;
    const PoolQueue* queues;
    unsigned* qtaken;          // one counter per queue
    const PoolSeed* seeds;
    unsigned* status;          // the plan's status word (workspace), set when a wave gives up
    unsigned* dev_status;      // the device's failure word, set alike
    SectorStamp* stamps;       // per plan item, or nullptr
    int nq, seed_groups, pool_pages;
    unsigned spin_limit;
};

struct PoolEntry {
    int waves;
    const void* kernel;
};
void register_pool_variants(std::vector<PoolEntry>& v);

// Blocks of 64 points per lane register (R) of the NPDU kernel holding a
// sector of n points, and whether x, y, z live in LDS (R <= 2) or are read
// from global memory (R >= 4); 0 if n is too large.
__host__ __device__ constexpr int npdu_r_for(int n) {
    return n <= 4096 ? 1 : n <= 8192 ? 2 : n <= 16384 ? 4 : n <= 32768 ? 8 : 0;
}
// Pages of the pool a sector of n points occupies.
__host__ __device__ constexpr int npdu_pool_pages(int n) {
    return (4 * npdu_lds_words(n, npdu_r_for(n) <= 2) + kPoolPageBytes - 1) / kPoolPageBytes;
}

// Point validation pass (check.hip): one workgroup per cloud, up to
// kCheckClouds clouds per launch; per cloud the first point with a non-finite
// coordinate and the order keys of the smallest and largest x, y, z.
struct CheckSeg {
    int64_t offset;   // first point of the cloud, in points
    int32_t n;
    int32_t pad;
};
constexpr int kCheckClouds = 64;
struct CheckBatch {
    CheckSeg seg[kCheckClouds];   // passed by value (1 KB of kernel arguments)
};
struct CheckResult {
    unsigned long long first_bad;   // ~0 if every coordinate is finite
    uint32_t lo[3], hi[3];          // order keys: unsigned order of the keys = float order
};
static_assert(sizeof(CheckResult) == 32, "check result layout");
const void* check_points_kernel();

// Grouping around the samples (group.hip): the ball-query kernel.
const void* ball_query_kernel_ptr();

// Binning along one axis (binning.hip): a stable counting sort by bin.
constexpr int kBinChunk = 1024;   // points per histogram chunk (one scatter wave each)
constexpr int kMaxBins = 8192;    // bins counted in LDS
struct BinHeader {
    uint32_t lo_key, hi_key;      // order keys of the smallest and largest coordinate
    uint32_t pad[62];
};
static_assert(sizeof(BinHeader) == 256, "binning header");
struct BinKernels {
    const void *reset, *range, *count, *scan_rows, *scan_totals, *scatter;
};
BinKernels bin_kernels();

// Multi-workgroup plain FPS (fps_grid.hip).
struct GridVariant {
    int waves, slots;
    const void* kernel;
};
void register_grid_variants(std::vector<GridVariant>& v);
const void* grid_reset_kernel();
const void* queue_reset_kernel();
constexpr int kMaxGridGroups = 64;     // workgroups meeting at the grid barrier
constexpr int kGridSyncBytes = 256 + 2 * kMaxGridGroups * 32;   // one barrier block

}  // namespace afps
