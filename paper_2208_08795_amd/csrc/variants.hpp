// Host-visible tables of compiled kernel variants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "layout.hpp"

namespace afps {

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

// Inputs and outputs of one round of a launch of several rounds (one DEVICE
// entry per round; the same layout as afps_round in afps.h).
struct PoolRound {
    const float* xyz_all;
    int32_t* out_all;
};
static_assert(sizeof(PoolRound) == 16, "round layout");

// Arguments of the pooled NPDU kernel (passed by value).
struct PoolArgs {
    const float* xyz_all;      // a single round's points and outputs (rounds == nullptr)
    int32_t* out_all;
    const PoolRound* rounds;   // several rounds: per-round points and outputs, or nullptr
    const WorkItem* items;
    const PoolGroup* groups;   // one per workgroup
    const PoolQueue* queues;
    const PoolSeed* seeds;     // W per workgroup, workgroup-major
    unsigned* status;          // the plan's status word (workspace), set when a wave gives up
    unsigned* dev_status;      // the device's failure word, set alike
    SectorStamp* stamps;       // per plan item (single round only), or nullptr
    int nrounds, pool_pages;
    unsigned spin_limit;
    int seed_priority;         // issue priority (0..3) of the wave running its workgroup's first seed
};

struct PoolEntry {
    int waves;
    bool lite;   // only the narrow loop with coordinates from L2 (npdu_item_lite sectors)
    const void* kernel;
};
void register_pool_variants(std::vector<PoolEntry>& v);

// Point validation pass (check.hip): one workgroup per cloud, up to
// kCheckClouds clouds per launch; per cloud the first point with a non-finite
// coordinate and the order keys of the smallest and largest x, y, z.
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
