// Batch planner: host-only logic of a batch plan (no HIP calls), so that it
// can be built and exercised on a machine without a GPU.
//
// From the clouds' descriptors it validates sizes, cuts every cloud into its
// Sec. III-B sectors (work items), chooses per NPDU sector where its
// coordinates live (LDS records or L2), groups the NPDU sectors into page
// queues for the pooled launch and seeds each pooled wave with its first
// sector, groups the full-update sectors by kernel variant and sizes each
// persistent grid, and lays out the device workspace.  What it needs to know
// about the device and the compiled kernels comes in PlannerEnv.
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "afps.h"
#include "layout.hpp"

namespace afps {

// A full-update (FPS / AFPS) kernel variant as the planner sees it.
struct FullVariantInfo {
    int id;          // index into the caller's table of compiled variants
    int waves;       // waves per workgroup
    int slots;       // point slots per thread
    int lds_bytes;   // dynamic LDS of the persistent kernel
};

// Where an NPDU sector's coordinates live, for sectors of at most n_max
// points and windows k <= k_max: LDS records (xyz_in_lds = 1) or outside LDS
// (0: registers in pooled shapes of at most 8 waves for sectors of at most
// 4096 points with k <= 64, else L2).  The first entry (ascending n_max, then
// k_max) that covers a sector decides; sectors no entry covers keep their
// coordinates in LDS up to 8192 points.
struct NpduPlacement {
    int n_max, k_max, xyz_in_lds;
};

// Tunable policy of the pooled NPDU launch.
struct PoolPolicy {
    float waves_per_simd = 0.0f;   // plan occupancy budget (0 = built-in rule)
    int waves = 0;                 // explicit shape: waves per workgroup (0 = from the budget)
    int groups = 0;                // explicit shape: workgroups per CU (0 = from the budget)
    bool seed_sleep = true;        // seeds with slack before the critical sector wait before loading
    int seed_priority = 3;         // issue priority of the wave running its workgroup's first seed
    std::vector<NpduPlacement> placement;
};

struct PlannerEnv {
    int cu_count = 0;        // compute units
    int cu_pool_pages = 0;   // LDS pages of a whole CU for pooled workgroups (<= kMaxPoolPages)
    PoolPolicy pool;
    // Batch variant for a full-update sector of n points (false: none holds it).
    std::function<bool(int n, FullVariantInfo*)> choose_full;
    // Workgroups of a full-update variant resident per CU (0: cannot run).
    std::function<int(const FullVariantInfo&)> blocks_per_cu;
};

struct PlannedBucket {
    int variant;      // full-update variant id; -1 = the pooled NPDU launch
    int block;        // threads per workgroup
    int lds_bytes;    // dynamic LDS per workgroup
    int first, count; // items [first, first + count)
    int grid;         // workgroups launched
    double cost;      // estimated cycles of all its items
    double longest;   // estimated cycles of its longest item
    bool pool() const { return variant < 0; }
};

struct PlanTables {
    std::vector<WorkItem> items;
    std::vector<PlannedBucket> buckets;   // largest estimated cost first
    std::vector<PoolGroup> groups;        // each pooled workgroup's queues
    std::vector<PoolQueue> queues;        // every workgroup's queues, highest priority first
    std::vector<PoolSeed> seeds;          // first sector of each pooled wave, workgroup-major
    std::vector<CheckSeg> clouds;         // each descriptor's points
    int pool_pages = 0;                   // LDS pages of one pooled workgroup
    int pool_groups = 0;                  // pooled workgroups per CU (0 without NPDU sectors)
    int pool_waves = 0;                   // waves per pooled workgroup
    bool pool_lite = false;               // the light kernel (two workgroups of 12 or 16 waves per CU)
    int seed_priority = 0;
    size_t ws_bytes = 0;
};

// Argument checks shared with the single-cloud calls; on failure they return
// the afps status and set *err.
int check_sizes(int32_t n, int32_t c, int32_t m, int32_t start, std::string* err);
// NPDU reading flags checked; "k counting the sample" rewritten as k - 1.
int npdu_readings(int32_t* k, int32_t* flags, std::string* err);
int32_t largest_sector(int32_t n, int32_t m);
// Windows wider than twice the sector behave exactly like 2 n_s.
int32_t clamp_k(int32_t k, int32_t n_s);
// Pooled launch shapes: one workgroup per CU of 4, 8, 12 or 16 waves (one to
// four per SIMD), two of 4 waves each owning half of the CU's pages, or two
// of 12 or 16 waves (six or eight per SIMD: light kernels, for plans whose
// NPDU sectors all qualify, npdu_item_lite).
bool valid_pool_shape(int waves, int groups);
bool pool_shape_needs_lite(int waves, int groups);
// Coordinates of an NPDU sector of n points with window k in LDS?
bool npdu_xyz_in_lds(const PoolPolicy& policy, int n, int k);

// Build the plan; AFPS_OK or a status with *err naming the first bad descriptor.
int build_plan(const afps_cloud_desc* descs, int32_t batch, const PlannerEnv& env, PlanTables* out,
               std::string* err);

}  // namespace afps
