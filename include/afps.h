/*
 * afps.h -- C ABI of the MI355X (gfx950) farthest-point-sampling library.
 *
 * Implements, as hand-written HIP kernels:
 *   - plain farthest point sampling (FPS): Algorithm 1 of Li et al., "An
 *     Adjustable Farthest Point Sampling Method for Approximately-sorted Point
 *     Cloud Data" (arXiv 2208.08795);
 *   - adjustable FPS (AFPS): the cloud is cut into M contiguous storage sectors
 *     and each sector runs its own FPS, all sectors at once (Sec. III-B);
 *   - nearest-point distance updating (NPDU): each iteration updates only the
 *     distances of the new sample's storage neighbours (Sec. III-C), alone
 *     (M = 1) or inside every AFPS sector.
 *
 * Common conventions
 *   xyz      DEVICE pointer to n points, row-major fp32 (x, y, z per point,
 *            12 bytes per point, 4-byte aligned).  Read only, and not to be
 *            written while a launch that reads it runs (kernels read the
 *            points partly through the scalar data cache, which a concurrent
 *            write would not update).
 *   out_idx  DEVICE pointer to c int32 entries, written with indices into the
 *            cloud (0 .. n-1): sector-major, and within a sector in pick order.
 *   stream   a hipStream_t passed as void* (NULL = the default stream).  Every
 *            call is asynchronous on that stream; results are valid once the
 *            caller has synchronised it.
 *   Ownership: the caller allocates and frees every buffer.  No sampling call
 *   allocates device memory: the library's own device state (barrier blocks
 *   of the multi-workgroup FPS, a failure word, events ordering their reuse)
 *   is static device memory or is made once per device, by afps_init or by
 *   the first call on that device.  Batch plans allocate host memory only
 *   (the device side lives in the caller's workspace).
 *   Device-side failures: the only waits inside kernels are bounded (see
 *   afps_set_spin_limit); a kernel that gives one up leaves -1 in the outputs
 *   it could not finish and records the failure, which afps_device_status
 *   (any call) and afps_plan_status (batch plans) report as AFPS_ERR_DEVICE.
 *   Arithmetic: squared Euclidean distance in fp32, ((dx*dx + dy*dy) + dz*dz),
 *   no fused multiply-add; initial distance 1e10; argmax ties go to the lowest
 *   index.  Results are bit-identical to a sequential evaluation of the paper's
 *   loop in that arithmetic.
 *   Preconditions, not checked unless input checking is on (afps_set_checking,
 *   or AFPS_CHECK=1 in the environment when the library loads): coordinates
 *   finite, squared distances below 1e10 (coordinate extent below 1e5).
 *   Errors: a negative status; nothing is launched and out_idx is untouched
 *   when the arguments are rejected.  No C++ exception crosses this ABI.
 *   Every function is thread-safe.
 */
#ifndef AFPS_H
#define AFPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum afps_status {
    AFPS_OK = 0,
    AFPS_ERR_NULL = -1,        /* a required pointer is NULL */
    AFPS_ERR_ARG = -2,         /* sizes violate 1 <= m <= c <= n, or a bad descriptor */
    AFPS_ERR_RANGE = -3,       /* start outside [0, n) */
    AFPS_ERR_WORKSPACE = -4,   /* workspace missing or smaller than required */
    AFPS_ERR_HIP = -5,         /* a HIP runtime call failed; see afps_last_error() */
    AFPS_ERR_UNSUPPORTED = -6, /* the problem exceeds what the kernels handle */
    AFPS_ERR_DEVICE = -7,      /* a kernel reported a failure (e.g. a timed-out grid barrier) */
    AFPS_ERR_DATA = -8         /* input check: a non-finite coordinate, or extent too large */
};

/*
 * Plain FPS, Algorithm 1: c samples from n points starting at index `start`.
 * Requires 1 <= c <= n and 0 <= start < n.  Any n up to 2^31-1 that fits the
 * device: clouds beyond one workgroup's register capacity are split across
 * several workgroups that meet at a grid barrier each iteration.
 */
int afps_fps_plain(const float *xyz, int32_t n, int32_t c, int32_t start,
                   int32_t *out_idx, void *stream);

/*
 * AFPS, Sec. III-B: M sectors of contiguous storage.  Sector s holds
 * n_s = floor(n/m) + (s < n mod m) points starting at point
 * b_s = s*floor(n/m) + min(s, n mod m), and takes c_s = floor(c/m) + (s < c mod m)
 * samples written at out_idx[o_s ..], o_s = s*floor(c/m) + min(s, c mod m).
 * Each sector starts at its local point (start mod n_s).
 * Requires 1 <= m <= c <= n and 0 <= start < n.  m = 1 is plain FPS.
 * Each sector must fit one workgroup: n_s <= afps_max_sector_points().
 */
int afps_afps(const float *xyz, int32_t n, int32_t c, int32_t m, int32_t start,
              int32_t *out_idx, void *stream);

/*
 * AFPS with NPDU, Sec. III-C: after each pick the distance update touches only
 * the window [cur - floor(k/2), cur + ceil(k/2)] of the sector (the sample and
 * its k storage neighbours), truncated at the sector's edges; there is no full
 * first pass.  Requires k >= 0 plus the AFPS requirements.
 */
int afps_afps_npdu(const float *xyz, int32_t n, int32_t c, int32_t m, int32_t k,
                   int32_t start, int32_t *out_idx, void *stream);

/*
 * The readings of Sec. III-C that the paper leaves open, as alternatives to the
 * ones afps_afps_npdu takes (bit flags, combinable):
 *   AFPS_NPDU_FIRST_FULL : the first iteration updates every point of the
 *                          sector from the start point; later ones the window;
 *   AFPS_NPDU_SHIFT_EDGES: a window that would cross a sector edge is moved
 *                          inward, keeping its k + 1 points where the sector
 *                          allows, instead of being truncated;
 *   AFPS_NPDU_K_WITH_SELF: the k updated points include the sample
 *                          (floor((k-1)/2) below, ceil((k-1)/2) above); k >= 1.
 */
#define AFPS_NPDU_FIRST_FULL 1
#define AFPS_NPDU_SHIFT_EDGES 2
#define AFPS_NPDU_K_WITH_SELF 4

/* afps_afps_npdu with reading flags (0 = afps_afps_npdu); AFPS_ERR_ARG for
 * unknown bits, or K_WITH_SELF with k < 1. */
int afps_afps_npdu_ex(const float *xyz, int32_t n, int32_t c, int32_t m, int32_t k,
                      int32_t start, int32_t flags, int32_t *out_idx, void *stream);

/*
 * Set up the library's state on the current device (kernel attributes, the
 * static barrier blocks and failure word, events): every call does this on
 * its first use of a device; calling it first keeps that work out of a later
 * call (for instance one inside a stream capture).  AFPS_ERR_HIP on failure.
 */
int afps_init(void);

/*
 * Device-side failures on the current device: waits for `stream`, then
 * returns AFPS_ERR_DEVICE if any kernel of the library on this device has
 * given up a bounded wait since the record was last cleared (its unfinished
 * outputs hold -1), else AFPS_OK; clear != 0 clears the record (ordered on
 * `stream`).  The record is shared by every stream and thread on the device.
 */
int afps_device_status(void *stream, int32_t clear);

/* Largest sector (points) a single workgroup holds in registers. */
int32_t afps_max_sector_points(void);

/* ---------------------------------------------------------------- batches */

/*
 * One cloud of a batch (Table I's setting of many clouds per call, here of
 * uneven size).  xyz_offset counts points into xyz_all, out_offset counts
 * indices into out_all.  k < 0 turns NPDU off; m == 1 && k < 0 is plain FPS.
 * Indices written are local to the cloud (0 .. n-1).
 */
typedef struct afps_cloud_desc {
    int64_t xyz_offset;
    int64_t out_offset;
    int32_t n, c, m, k;
    int32_t start;
    int32_t flags;             /* NPDU reading flags (AFPS_NPDU_*); 0 without NPDU */
} afps_cloud_desc;

typedef struct afps_plan afps_plan;

/*
 * Build a batch plan on the host from `batch` HOST descriptors: validates
 * them, expands every cloud into its sectors (work items), orders the items
 * longest-first, and groups them: NPDU sectors are each assigned to one
 * workgroup of the pooled launch (balanced by estimated cost) and queued
 * there by LDS pages, FPS/AFPS sectors are grouped by kernel variant (one
 * persistent launch each); sizes the workspace.
 * Returns AFPS_OK and *plan, or an error (AFPS_ERR_ARG names the first bad
 * descriptor in afps_last_error()).
 */
int afps_plan_create(const afps_cloud_desc *descs, int32_t batch, afps_plan **plan);

/* Device workspace bytes the plan needs (counters, workgroup, seed and queue tables, work items). */
size_t afps_plan_workspace_bytes(const afps_plan *plan);

/*
 * Workspace bytes of a plan with `items` work items in total (one per sector,
 * i.e. the sum of m over the batch): a 68.25 KB header (the launch counters,
 * the pooled workgroups' queue ranges and each pooled wave's first sector),
 * then 40 bytes per item and at most one 16-byte NPDU queue per item, rounded
 * up to 256.  Lets a caller reserve device memory before building the plan.
 * Host-only arithmetic; 0 for items <= 0.
 */
size_t afps_workspace_bytes_for_items(int32_t items);

/*
 * Copy the plan's tables (NPDU workgroups, queues and first sectors, work items) into `workspace` (DEVICE,
 * >= the size above, 256-byte aligned) on `stream`, asynchronously.  Must precede
 * afps_plan_launch with that workspace in stream order: a launch on another
 * stream is ordered after the copy by the caller (an event, or a stream that
 * waits for this one); the tables stay valid until overwritten.  A plan's
 * launches on several streams at once each need their own workspace (its
 * launch counters and status word are reset and used by every launch).
 */
int afps_plan_upload(afps_plan *plan, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Run the batch: reset the launch counters (a kernel), then one persistent
 * launch per kernel variant, concurrent on helper streams when there are
 * several.  FPS/AFPS workgroups take work items from device queues with
 * atomic counters until the queues are empty; the waves of a pooled NPDU
 * workgroup take its own sectors, claimed in its LDS.  Kernel launches only,
 * so a caller may capture it in a hipGraph.  Launches with one workspace must
 * not overlap.
 */
int afps_plan_launch(const afps_plan *plan, const float *xyz_all, int32_t *out_all,
                     void *workspace, void *stream);

/*
 * Same as afps_plan_launch, but the launch sequence is captured into a
 * hipGraph the first time (per stream, buffers and workspace) and replayed
 * afterwards.
 */
int afps_plan_graph_launch(afps_plan *plan, const float *xyz_all, int32_t *out_all,
                           void *workspace, void *stream);

/*
 * Several rounds of the plan's batch in ONE pooled launch: a stream of
 * batches with the plan's layout (e.g. consecutive steps over fresh inputs),
 * processed back to back on the device with no kernel boundary between
 * them.  Round r reads rounds[r].xyz_all and writes rounds[r].out_all (both
 * laid out as for afps_plan_launch).  Each wave takes the highest-priority
 * of its workgroup's sectors that fits the workgroup's free LDS pages, from
 * the lowest round with sectors left, or from the next three rounds when none
 * of that one fits, so the next batch's sectors start as soon as pages free
 * up.  Every output of every round is the same as a separate
 * afps_plan_launch of that round gives.
 *   rounds    DEVICE array of `count` afps_round entries, 1 <= count <= 4096
 *   workspace DEVICE, >= afps_plan_rounds_workspace_bytes(plan, count) (the
 *             plan's own workspace size: the claim counters of the rounds
 *             live in LDS), the plan's tables uploaded into it (afps_plan_upload)
 * Only for plans whose sectors all use NPDU (AFPS_ERR_UNSUPPORTED otherwise)
 * and not with input checking on (each round's clouds are unknown to the
 * host).  Kernel launches only (capturable); asynchronous on `stream`.
 */
typedef struct afps_round {
    const float *xyz_all;
    int32_t *out_all;
} afps_round;
size_t afps_plan_rounds_workspace_bytes(const afps_plan *plan, int32_t rounds);   /* 0 if invalid */
int afps_plan_launch_rounds(const afps_plan *plan, const afps_round *rounds, int32_t count,
                            void *workspace, size_t workspace_bytes, void *stream);

/*
 * Status of the plan's last launch with `workspace`: waits for `stream`, then
 * returns AFPS_ERR_DEVICE if a wave of that launch gave up a bounded wait
 * (the sectors it could not run hold -1 in full), else AFPS_OK.  Each launch
 * clears the word first.
 */
int afps_plan_status(const afps_plan *plan, const void *workspace, void *stream);

/*
 * afps_plan_launch that also records, for every NPDU sector of the plan, 64
 * bytes of timestamps into `stamps` (DEVICE, >= afps_plan_items(plan) * 64
 * bytes, 64-byte aligned; entry i belongs to the plan's work item i):
 *   uint64 take, loaded, end  shader-clock counter (cycles) when a wave took
 *                             the sector, when its points were in LDS, and
 *                             when its last pick was written
 *   uint64 take_rt, end_rt    constant-rate counter at take and end
 *   int32  item, n, c, k      the work item and its sector's points, samples
 *                             and window
 *   uint32 hw_id, xcc_id      hardware id of the wave (CU, SIMD, slot) and
 *                             its XCC
 * so that (end - loaded) / (c - 1) is the sector's cycles per iteration.
 * Entries of full-update (FPS / AFPS) sectors are not written.
 */
int afps_plan_launch_stamped(const afps_plan *plan, const float *xyz_all, int32_t *out_all,
                             void *workspace, void *stamps, size_t stamp_bytes, void *stream);

/* Rate of the constant-rate counter of the stamps (kHz) on the current
 * device; 0 if the runtime does not report it. */
int32_t afps_wall_clock_khz(void);

/*
 * afps_plan_launch for callers that cannot allocate device memory and cannot
 * bring a workspace (tight serving loops, harnesses that forbid hipMalloc):
 * the plan's workspace is a static array of 1 MiB in device memory that the
 * library holds on each GPU it runs on until the process ends, so the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * It copies the plan's tables into that array on `stream` and launches the
 * same kernels as afps_plan_launch, whose reset kernel clears the launch
 * counters first.  Every call on a GPU shares that GPU's array, which keeps
 * the last call's contents: calls that overlap on one GPU (several streams
 * or threads, or with a plan launched this way still running) race on it and
 * must be serialised by the caller.  The plan must have been created with the
 * current device current (AFPS_ERR_ARG otherwise).  AFPS_ERR_WORKSPACE, with
 * nothing copied or launched, for a plan of more than afps_noalloc_max_items()
 * sectors.  Not for stream capture (the tables are copied from pageable host
 * memory).
 */
int afps_plan_launch_noalloc(const afps_plan *plan, const float *xyz_all, int32_t *out_all,
                             void *stream);
/* Sectors (work items) a plan may have for afps_plan_launch_noalloc. */
int32_t afps_noalloc_max_items(void);

/* Number of work items (sectors) and persistent launches of the plan. */
int32_t afps_plan_items(const afps_plan *plan);
int32_t afps_plan_launches(const afps_plan *plan);

/*
 * Waves per workgroup of the plan's pooled NPDU launch, and its workgroups per
 * CU; both 0 if the plan has no NPDU sectors.  The launch holds each CU's LDS
 * as 1 KB pages: one workgroup of 4 waves per CU (one wave per SIMD), one of 8
 * (two per SIMD), or, for two per SIMD when every sector fits half of a CU's
 * pages, two workgroups of 4 per CU with half the pages each (a launch then
 * releases LDS half a CU at a time to launches on other streams).  Chosen at
 * plan creation from the plan's longest sector and total work, or by
 * afps_set_plan_occupancy.
 */
int32_t afps_plan_pool_waves(const afps_plan *plan);
int32_t afps_plan_pool_groups_per_cu(const afps_plan *plan);

void afps_plan_destroy(afps_plan *plan);

/*
 * One-shot batch: plan, upload and launch.  descs are HOST descriptors;
 * workspace must hold afps_batched_workspace_bytes(descs, batch) bytes.
 */
size_t afps_batched_workspace_bytes(const afps_cloud_desc *descs, int32_t batch);
int afps_batched(const float *xyz_all, const afps_cloud_desc *descs, int32_t batch,
                 int32_t *out_all, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------- tuning */

/*
 * Kernel variant chosen for a sector of n_s points: waves per workgroup and
 * point slots per thread.  `kind` selects the table: AFPS_TUNE_DIRECT (FPS /
 * AFPS single-cloud launches), AFPS_TUNE_BATCH (FPS / AFPS sectors inside batch
 * plans), AFPS_TUNE_NPDU (reports the NPDU variant: one wave, `slots` = block
 * registers).  Tuned entries ("for sectors of at most n_s_max points use this
 * variant") override the built-in rule; afps_tune_set is what the autotuner
 * calls, and a file named by the environment variable AFPS_TUNE_CACHE (lines
 * "direct|batch n_s_max waves slots") is read once at first use.
 * afps_tune_set returns AFPS_ERR_ARG for an unknown or too small variant.
 */
enum { AFPS_TUNE_DIRECT = 0, AFPS_TUNE_NPDU = 1, AFPS_TUNE_BATCH = 2 };
int afps_tune_get(int32_t n_s, int32_t kind, int32_t *waves, int32_t *slots);
int afps_tune_set(int32_t n_s_max, int32_t kind, int32_t waves, int32_t slots);
void afps_tune_reset(void);   /* forgets every tuned entry and the pool policy (not the occupancy) */

/*
 * NPDU placement in batch plans created afterwards: NPDU sectors of at most
 * n_s_max points with windows k <= k_max keep their coordinates in LDS
 * (xyz_in_lds = 1: 16-byte records {D, x, y, z}, possible up to 8192 points)
 * or out of LDS (0: only the distances take LDS, 4 bytes per point, so a
 * pooled CU holds four times the sectors; the coordinates sit in vector
 * registers for sectors of at most 4096 points with k <= 64 in pooled
 * launches of at most 8 waves per workgroup, else they are read from L2).
 * The entry with the smallest n_s_max (then k_max) that covers a sector
 * decides; without one, sectors up to 8192 points keep their coordinates in
 * LDS (the fastest iteration: the shortest single launch).  Batches bound by
 * throughput gain from placements out of LDS (autotune.tune_npdu), which let
 * a CU run more sectors at once.  Read from
 * AFPS_TUNE_CACHE as lines "npdu n_s_max k_max xyz_in_lds".  AFPS_ERR_ARG
 * for bad values.  afps_npdu_xyz_in_lds reports the placement a sector would
 * get.
 */
int afps_tune_npdu(int32_t n_s_max, int32_t k_max, int32_t xyz_in_lds);
int afps_npdu_xyz_in_lds(int32_t n_s, int32_t k);
/* Forget the NPDU placement entries and the pool policy (afps_set_pool_policy);
 * the full-update tuning and the occupancy budget stay. */
void afps_tune_npdu_clear(void);

/*
 * Policy of the pooled NPDU launch of batch plans created afterwards:
 *   waves, groups_per_cu  the launch shape: one workgroup per CU of 4, 8, 12
 *                         or 16 waves (one to four per SIMD) owning all of
 *                         the CU's LDS pages, or two of 4, 12 or 16 waves
 *                         owning half each (used when every sector fits half;
 *                         two of 12 or 16, six or eight waves per SIMD, only
 *                         when every NPDU sector has at most 4096 points,
 *                         k <= 64 and its coordinates out of LDS: a light
 *                         kernel that holds only that loop); 0, 0 = chosen
 *                         from the plan's occupancy budget and its sectors
 *                         (afps_set_plan_occupancy)
 *   seed_sleep            1 = first sectors with slack before the plan's
 *                         longest one wait a sleep period before loading
 *   seed_priority         issue priority 0..3 of the wave running its
 *                         workgroup's first (longest) seed
 * Read from AFPS_TUNE_CACHE as a line "pool waves groups sleep priority".
 * Defaults 0, 0, 1, 3; afps_tune_reset restores them.  AFPS_ERR_ARG for
 * values outside these sets.
 */
int afps_set_pool_policy(int32_t waves, int32_t groups_per_cu, int32_t seed_sleep,
                         int32_t seed_priority);

/*
 * Run one sector variant explicitly (for the autotuner and tests): AFPS or
 * NPDU over m sectors with the given waves / slots.  AFPS_ERR_UNSUPPORTED if
 * that variant is not built or the sectors do not fit it.
 */
int afps_afps_variant(const float *xyz, int32_t n, int32_t c, int32_t m, int32_t k,
                      int32_t start, int32_t flags, int32_t *out_idx, int32_t waves,
                      int32_t slots, void *stream);

/*
 * Wave budget of batch plans created afterwards, in waves per SIMD.  0 (the
 * default) = no budget: each persistent FPS/AFPS grid is as large as stays
 * resident, at most one workgroup per work item, and the pooled NPDU launch
 * picks one or two waves per SIMD from the plan's longest sector and total
 * work.  With a budget, each FPS/AFPS bucket gets the fewest workgroups whose
 * longest-first schedule of its estimated item costs ends by the plan's
 * longest item, raised until all grids together keep about this many waves
 * per SIMD, and the pooled NPDU launch runs one wave per SIMD below 1.5 and
 * two from 1.5.  Process-wide; AFPS_ERR_ARG outside [0, 64].
 */
int afps_set_plan_occupancy(float waves_per_simd);

/*
 * Bound on the polls of one wait inside a kernel (default 4M): a grid barrier
 * of the multi-workgroup plain-FPS kernel, or the page-allocation lock and
 * free pages of the pooled NPDU kernel.  A wait that exceeds it fails the
 * launch: the grid kernel's workgroups all return with -1 in the unfinished
 * outputs; a pooled workgroup stops taking sectors and its last wave marks
 * every sector of it no wave took -1 (in every round).  Either records
 * AFPS_ERR_DEVICE (afps_device_status, afps_plan_status).  Process-wide.
 */
int afps_set_spin_limit(uint32_t polls);

/* ---------------------------------------------------------------- binning */

/*
 * Binning along one axis, Sec. III-A: a cloud without dimensional locality is
 * binned instead of sorted, into the approximate order of the footnote to
 * Table II (every point of a later bin has a larger coordinate; points inside
 * a bin keep their storage order), which AFPS and NPDU then exploit.  With
 * lo, hi the smallest and largest coordinate along `axis` (0 = x, 1 = y,
 * 2 = z), each point goes to bin min(bins-1, floor((x - lo) * scale)),
 * scale = bins / (hi - lo) in fp32 (0 when hi == lo).
 *   perm     DEVICE, n int32: perm[i] = storage index of the i-th point in
 *            binned order (a stable counting sort by bin)
 *   xyz_out  DEVICE, n x 3 fp32 or NULL: the points in binned order (must
 *            not be xyz)
 *   workspace DEVICE, >= afps_bin_workspace_bytes(n, bins), 256-byte aligned
 * Requires n >= 1 and 1 <= bins <= 8192.  Kernel launches only (a caller may
 * capture them in a hipGraph); asynchronous on `stream`.
 */
size_t afps_bin_workspace_bytes(int32_t n, int32_t bins);   /* 0 if the sizes are invalid */
int afps_bin_points(const float *xyz, int32_t n, int32_t axis, int32_t bins, int32_t *perm,
                    float *xyz_out, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Input check of the preconditions above for one cloud of n points (DEVICE
 * xyz): every coordinate finite, and the squared diagonal of the bounding box
 * (which bounds every squared distance) below the initial distance 1e10 of
 * Algorithm 1.  Reads the points once on `stream` and waits for it.  Returns
 * AFPS_OK, or AFPS_ERR_DATA with the first offending point (or the diagonal)
 * in afps_last_error().  The first check on a device allocates a 2 KB result
 * buffer that the library keeps until the process ends.
 */
int afps_check_points(const float *xyz, int64_t n, void *stream);

/*
 * Input checking on (on != 0) or off, process-wide.  When on, every sampling
 * call first runs afps_check_points on each of its clouds (a batch plan: each
 * descriptor's cloud, before its launch or graph replay), so the call waits
 * for its stream and returns AFPS_ERR_DATA without launching when a cloud
 * fails.  Off by default; AFPS_CHECK=1 in the environment turns it on at load.
 */
int afps_set_checking(int32_t on);

/* ------------------------------------------------------------- grouping */

/*
 * Grouping around the samples: the ball query of a PointNet++ set
 * abstraction layer, which the paper names as the consumer of the samples
 * (Sec. I, Sec. II-A) without defining it; the readings are those of the
 * oracle.  For each centre q (an index into the cloud, typically a sample
 * returned by the calls above), the first k points j in increasing index
 * order with squared distance ((dx*dx + dy*dy) + dz*dz, dx = x_j - x_q, fp32,
 * no fused multiply-add) below r2 = radius * radius (rounded to fp32); the
 * slots past the found ones repeat the first found, or hold q when none was
 * found (radius 0).  window >= 0 bounds the candidates to storage positions
 * [q - window, q + window] (with dimensional locality, Sec. III-A, storage
 * neighbours approximate spatial ones); window < 0 searches the whole cloud.
 *   xyz      DEVICE, n x 3 fp32 row-major, n >= 1
 *   centers  DEVICE, c int32 indices; an index outside [0, n) yields -1 in
 *            all k slots and in its count (nothing outside the cloud is read)
 *   out_idx  DEVICE, c x k int32 (centre-major), fully written
 *   out_cnt  DEVICE, c int32 neighbours found (at most k), or NULL
 * Requires c >= 0, k >= 1 and radius >= 0 (AFPS_ERR_ARG otherwise, nothing
 * launched).  One kernel launch (capturable); asynchronous on `stream`.
 */
int afps_ball_query(const float *xyz, int32_t n, const int32_t *centers, int32_t c, float radius,
                    int32_t k, int32_t window, int32_t *out_idx, int32_t *out_cnt, void *stream);

/* --------------------------------------------------------------- status */

const char *afps_status_string(int status);  /* static string */
const char *afps_last_error(void);           /* this thread's last error detail */

#ifdef __cplusplus
}
#endif

#endif /* AFPS_H */
