// Host side of the C ABI declared in include/afps.h.
//
// Responsibilities: argument validation (before anything touches the GPU),
// the sector plan of Sec. III-B, the choice of kernel variant per sector size
// (built-in rule or tuned override), launches on the caller's stream, batch
// plans (work-item tables for the persistent kernels, per-variant buckets on
// helper streams, optional hipGraph capture/replay) and the grid-barrier pool
// of the multi-workgroup plain-FPS kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "afps.h"
#include "planner.hpp"
#include "variants.hpp"

using namespace afps;

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return AFPS_ERR_HIP;
}

#define AFPS_HIP(call)                                    \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------------ variants

struct Registry {
    std::vector<VariantEntry> full;   // full-update sector kernels
    std::vector<NpduEntry> npdu;      // NPDU sector kernels, ascending capacity
    std::vector<GridVariant> grid;    // multi-workgroup plain FPS
    std::vector<PoolEntry> pool;      // pooled NPDU kernel of batch plans, by waves
    Registry() {
        register_variants_w1(full);
        register_variants_w2(full);
        register_variants_w4(full);
        register_variants_w8(full);
        register_variants_w16(full);
        register_npdu_variants(npdu);
        register_grid_variants(grid);
        register_pool_variants(pool);
    }
};

Registry& registry() {
    static Registry r;
    return r;
}

const VariantEntry* find_full(int waves, int slots) {
    for (const auto& v : registry().full)
        if (v.waves == waves && v.slots == slots) return &v;
    return nullptr;
}

int capacity(const VariantEntry& v) { return 64 * v.waves * v.slots; }
int capacity(const NpduEntry& v) { return 64 * 64 * v.chunk64; }

constexpr int kMaxFullSector = 32768;   // W = 16, P = 32 with distances in LDS

// Built-in rule for a full-update sector of n points: about 512 points per
// wave (a power of two number of waves, at most 16), then the smallest slot
// count that holds the sector.
const VariantEntry* rule_full(int n) {
    int waves = 1;
    while (waves < 16 && waves * 512 < n) waves *= 2;
    const VariantEntry* best = nullptr;
    for (const auto& v : registry().full)
        if (v.waves == waves && capacity(v) >= n && (!best || v.slots < best->slots)) best = &v;
    if (!best)   // fall back to any variant that holds it, fewest slots first
        for (const auto& v : registry().full)
            if (capacity(v) >= n && (!best || capacity(v) < capacity(*best))) best = &v;
    return best;
}

struct Tuned {
    int n_max, waves, slots;
};
// Tuned full-update variants: [0] single-cloud (direct) launches, [1] batch
// plans (persistent launches); each ascending in n_max.
std::mutex g_tune_mu;
std::vector<Tuned> g_tuned[2];
bool g_tune_loaded = false;
// Policy of pooled NPDU launches in batch plans (occupancy budget, shape,
// seeding, coordinate placement); guarded by g_tune_mu.
PoolPolicy g_pool_policy;

void sort_placement(std::vector<NpduPlacement>& tab) {
    std::sort(tab.begin(), tab.end(), [](const NpduPlacement& a, const NpduPlacement& b) {
        return a.n_max != b.n_max ? a.n_max < b.n_max : a.k_max < b.k_max;
    });
}

bool valid_pool_policy(int waves, int groups, int sleep, int prio) {
    const bool shape = (waves == 0 && groups == 0) || valid_pool_shape(waves, groups);
    return shape && (sleep == 0 || sleep == 1) && prio >= 0 && prio <= 3;
}

void load_tune_file_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("AFPS_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    // lines: "<direct|batch> <n_max> <waves> <slots>", "npdu <n_max> <k_max> <xyz_in_lds>",
    //        "pool <waves> <groups> <seed_sleep> <seed_priority>"
    char kind[16];
    while (std::fscanf(f, "%15s", kind) == 1) {
        int a = 0, b = 0, c = 0, d = 0;
        if (std::strcmp(kind, "pool") == 0) {
            if (std::fscanf(f, "%d %d %d %d", &a, &b, &c, &d) != 4) break;
            if (valid_pool_policy(a, b, c, d)) {
                g_pool_policy.waves = a;
                g_pool_policy.groups = b;
                g_pool_policy.seed_sleep = c != 0;
                g_pool_policy.seed_priority = d;
            }
            continue;
        }
        if (std::fscanf(f, "%d %d %d", &a, &b, &c) != 3) break;
        if (std::strcmp(kind, "npdu") == 0) {
            if (a >= 1 && b >= 0 && (c == 0 || c == 1)) g_pool_policy.placement.push_back({a, b, c});
            continue;
        }
        const int t = std::strcmp(kind, "direct") == 0 ? 0 : std::strcmp(kind, "batch") == 0 ? 1 : -1;
        const VariantEntry* v = find_full(b, c);
        if (t >= 0 && v && capacity(*v) >= a) g_tuned[t].push_back({a, b, c});
    }
    std::fclose(f);
    for (auto& tab : g_tuned)
        std::sort(tab.begin(), tab.end(), [](const Tuned& x, const Tuned& y) { return x.n_max < y.n_max; });
    sort_placement(g_pool_policy.placement);
}

// Variant for a full-update sector of n points; batch = persistent launch.
const VariantEntry* choose_full(int n, bool batch = false) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_file_locked();
        for (const auto& t : g_tuned[batch ? 1 : 0])
            if (n <= t.n_max) {
                const VariantEntry* v = find_full(t.waves, t.slots);
                if (v && capacity(*v) >= n) return v;
                break;
            }
    }
    return rule_full(n);
}

// The batch (persistent) variant of a full-update sector of n points.
bool batch_variant(int n, FullVariantInfo* out) {
    const VariantEntry* v = n <= kMaxFullSector ? choose_full(n, true) : nullptr;
    if (!v) return false;
    out->id = (int)(v - registry().full.data());
    out->waves = v->waves;
    out->slots = v->slots;
    out->lds_bytes = v->lds_bytes;
    return true;
}

const NpduEntry* choose_npdu(int n) {
    for (const auto& v : registry().npdu)
        if (capacity(v) >= n) return &v;
    return nullptr;
}

int npdu_lds_bytes(const NpduEntry& v, int n) { return 4 * npdu_lds_words(n, v.xyz_in_lds != 0); }

// ------------------------------------------------------------ devices

// Workspace of afps_plan_launch_noalloc, for callers that cannot allocate
// device memory: static device memory, one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it names a stand-in, not device memory): it uses the address that
// hipGetSymbolAddress returns on each device (DeviceState::scratch).
constexpr size_t kScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kHelperStreams = 4;
constexpr int kMaxRounds = 4096;   // rounds of one pooled launch
constexpr int kGridBlocks = 16;

// The barrier blocks of the multi-workgroup plain-FPS kernel and the
// device's failure word (device_words[0]: set by any kernel whose bounded
// wait gave up; afps_device_status reads it), in static device memory held
// until the process ends, so that no sampling call allocates.
static __device__ __align__(256) unsigned char grid_blocks[kGridBlocks * kGridSyncBytes];
static __device__ __align__(256) unsigned device_words[64];

struct DeviceState {
    bool ready = false;
    int cu_count = 0;
    size_t max_lds = 0;
    int pool_pages = 0;                      // LDS pages of one pooled-NPDU workgroup
    std::vector<hipStream_t> helpers;        // bucket streams for batch plans
    void* grid_pool = nullptr;               // this device's copy of grid_blocks
    unsigned* status = nullptr;              // this device's failure word (device_words[0])
    CheckResult* check_buf = nullptr;        // validation results (kCheckClouds), on first use
    std::mutex check_mu;                     // one validation at a time per device
    std::vector<hipEvent_t> grid_events;     // last user of each block
    int grid_next = 0;
    void* scratch = nullptr;                 // this device's copy of `scratch`
};

std::mutex g_dev_mu;
std::map<int, DeviceState> g_devices;

int device_state(DeviceState** out) {
    int dev = 0;
    AFPS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceState& d = g_devices[dev];
    if (!d.ready) {
        // The device address of this GPU's static scratch (with this device
        // current, as hipGetDevice reported it above).
        void* sp = nullptr;
        AFPS_HIP(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
        if (!sp) return fail(AFPS_ERR_HIP, "hipGetSymbolAddress(scratch) returned no address");
        d.scratch = sp;
        void* gp = nullptr;
        void* wp = nullptr;
        AFPS_HIP(hipGetSymbolAddress(&gp, HIP_SYMBOL(grid_blocks)));
        AFPS_HIP(hipGetSymbolAddress(&wp, HIP_SYMBOL(device_words)));
        if (!gp || !wp) return fail(AFPS_ERR_HIP, "hipGetSymbolAddress returned no address");
        d.grid_pool = gp;
        d.status = (unsigned*)wp;
        // Events that order the reuse of each barrier block, created here so
        // that no sampling call creates a runtime object.
        while ((int)d.grid_events.size() < kGridBlocks) {
            hipEvent_t e;
            AFPS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            d.grid_events.push_back(e);
        }
        int cus = 0, lds = 0;
        AFPS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        AFPS_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        d.cu_count = cus;
        d.max_lds = (size_t)lds;
        // The pool takes a CU's whole LDS, less the kernel's static LDS.
        int per_cu = 0;
        if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            per_cu <= 0)
            per_cu = lds;
        d.pool_pages = std::min(kMaxPoolPages, (per_cu - kPoolStaticLdsBytes) / kPoolPageBytes);
        // Kernels that take more than the default dynamic LDS.
        for (const auto& v : registry().full)
            if (v.lds_bytes > 0) {
                (void)hipFuncSetAttribute(v.direct, hipFuncAttributeMaxDynamicSharedMemorySize, v.lds_bytes);
                (void)hipFuncSetAttribute(v.persistent, hipFuncAttributeMaxDynamicSharedMemorySize, v.lds_bytes);
            }
        for (const auto& v : registry().npdu) {
            const int b = npdu_lds_bytes(v, capacity(v));
            (void)hipFuncSetAttribute(v.direct, hipFuncAttributeMaxDynamicSharedMemorySize, b);
        }
        for (const auto& v : registry().pool)
            (void)hipFuncSetAttribute(v.kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      d.pool_pages * kPoolPageBytes);
        (void)hipGetLastError();
        d.ready = true;
    }
    *out = &d;
    return AFPS_OK;
}

int helper_streams(DeviceState* d) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    while ((int)d->helpers.size() < kHelperStreams) {
        hipStream_t s;
        AFPS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        d->helpers.push_back(s);
    }
    return AFPS_OK;
}

// ------------------------------------------------------------ validation

int check_sizes(int32_t n, int32_t c, int32_t m, int32_t start) {
    std::string e;
    const int rc = afps::check_sizes(n, c, m, start, &e);
    return rc ? fail(rc, e) : AFPS_OK;
}

int npdu_readings(int32_t* k, int32_t* flags) {
    std::string e;
    const int rc = afps::npdu_readings(k, flags, &e);
    return rc ? fail(rc, e) : AFPS_OK;
}

// ------------------------------------------------------------ launches

int launch_full_direct(const VariantEntry& v, const float* xyz, int32_t n, int32_t c, int32_t m,
                       int32_t start, int32_t* out, hipStream_t stream) {
    void* args[] = {(void*)&xyz, (void*)&n, (void*)&c, (void*)&m, (void*)&start, (void*)&out};
    AFPS_HIP(hipLaunchKernel(v.direct, dim3(m), dim3(64 * v.waves), args, v.lds_bytes, stream));
    return AFPS_OK;
}

int launch_npdu_direct(const NpduEntry& v, const float* xyz, int32_t n, int32_t c, int32_t m,
                       int32_t k, int32_t start, int32_t flags, int32_t* out, hipStream_t stream) {
    const int lds = npdu_lds_bytes(v, largest_sector(n, m));
    void* args[] = {(void*)&xyz, (void*)&n, (void*)&c, (void*)&m, (void*)&k, (void*)&start, (void*)&flags,
                    (void*)&out};
    AFPS_HIP(hipLaunchKernel(v.direct, dim3(m), dim3(64), args, lds, stream));
    return AFPS_OK;
}

unsigned g_spin_limit = 1u << 22;

// Validate inputs before every sampling call (AFPS_CHECK=1 in the
// environment at load, or afps_set_checking).
bool env_checking() {
    const char* e = std::getenv("AFPS_CHECK");
    return e && *e && std::strcmp(e, "0") != 0;
}
bool g_checking = env_checking();

float unkey(uint32_t k) {
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    float f;
    std::memcpy(&f, &b, sizeof(f));
    return f;
}

// Preconditions of the distance arithmetic for each cloud [offset, offset+n)
// of xyz_all: finite coordinates, and a squared bounding-box diagonal below
// the initial distance 1e10 (it bounds every squared distance).  Waits for
// the stream.  `names[i]` says which cloud a failure refers to.
int check_clouds(const float* xyz_all, const std::vector<CheckSeg>& segs, hipStream_t stream,
                 const std::vector<std::string>& names) {
    DeviceState* d;
    int rc = device_state(&d);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(d->check_mu);
    if (!d->check_buf) AFPS_HIP(hipMalloc((void**)&d->check_buf, kCheckClouds * sizeof(CheckResult)));
    CheckResult host[kCheckClouds];
    for (size_t first = 0; first < segs.size(); first += kCheckClouds) {
        const int count = (int)std::min<size_t>(kCheckClouds, segs.size() - first);
        CheckBatch batch{};
        for (int i = 0; i < count; ++i) batch.seg[i] = segs[first + i];
        CheckResult* buf = d->check_buf;
        void* args[] = {(void*)&xyz_all, &batch, &buf};
        AFPS_HIP(hipLaunchKernel(check_points_kernel(), dim3(count), dim3(256), args, 0, stream));
        AFPS_HIP(hipMemcpyAsync(host, buf, count * sizeof(CheckResult), hipMemcpyDeviceToHost, stream));
        AFPS_HIP(hipStreamSynchronize(stream));
        for (int i = 0; i < count; ++i) {
            const CheckResult& r = host[i];
            const std::string& who = names[first + i];
            if (r.first_bad != ~0ull)
                return fail(AFPS_ERR_DATA, who + "point " + std::to_string(r.first_bad) +
                                               " has a non-finite coordinate");
            if (segs[first + i].n == 0) continue;
            double diag2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double e = (double)unkey(r.hi[a]) - (double)unkey(r.lo[a]);
                diag2 += e * e;
            }
            if (diag2 >= 1e10) {
                char msg[160];
                std::snprintf(msg, sizeof(msg),
                              "squared bounding-box diagonal %.6g is not below the initial distance 1e10",
                              diag2);
                return fail(AFPS_ERR_DATA, who + msg);
            }
        }
    }
    return AFPS_OK;
}

int maybe_check_cloud(const float* xyz, int32_t n, void* stream) {
    if (!g_checking) return AFPS_OK;
    return check_clouds(xyz, {CheckSeg{0, n, 0}}, (hipStream_t)stream, {""});
}

int launch_grid_fps(const float* xyz, int32_t n, int32_t c, int32_t start, int32_t* out,
                     hipStream_t stream) {
    const GridVariant* gv = nullptr;
    int groups = 0;
    // About 8192 points per workgroup; wider blocks once 64 workgroups are not enough.
    for (const auto& v : registry().grid) {
        const int chunk = 64 * v.waves * v.slots;
        const int g = (int)(((int64_t)n + chunk - 1) / chunk);
        if (v.slots >= 8 && g <= kMaxGridGroups) { gv = &v; groups = g; break; }
    }
    if (!gv)
        return fail(AFPS_ERR_UNSUPPORTED, "cloud of " + std::to_string(n) +
                                              " points exceeds the multi-workgroup FPS capacity");
    // Balance the blocks (the last one is not nearly empty); recount so that
    // every workgroup owns at least one point.  Block indices travel in 16
    // bits of the barrier word, so a block holds at most 65536 points.
    const int32_t chunk = (int32_t)(((int64_t)n + groups - 1) / groups);
    groups = (int)(((int64_t)n + chunk - 1) / chunk);
    if (chunk > 65536) return fail(AFPS_ERR_UNSUPPORTED, "grid block too large");
    DeviceState* d;
    int rc = device_state(&d);
    if (rc) return rc;
    void* block;
    hipEvent_t ev;
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        const int slot = d->grid_next;
        d->grid_next = (slot + 1) % kGridBlocks;
        block = (char*)d->grid_pool + (size_t)slot * kGridSyncBytes;
        ev = d->grid_events[slot];
        // The block's previous user (possibly on another stream) must be done.
        AFPS_HIP(hipStreamWaitEvent(stream, ev, 0));
        void* rargs[] = {&block};
        AFPS_HIP(hipLaunchKernel(grid_reset_kernel(), dim3(1), dim3(64), rargs, 0, stream));
        unsigned spin = g_spin_limit;
        unsigned* status = d->status;
        void* args[] = {(void*)&xyz, (void*)&n, (void*)&c, (void*)&start, (void*)&chunk,
                        (void*)&out, &block, &spin, &status};
        AFPS_HIP(hipLaunchCooperativeKernel(gv->kernel, dim3(groups), dim3(64 * gv->waves), args, 0,
                                            stream));
        AFPS_HIP(hipEventRecord(ev, stream));
    }
    return AFPS_OK;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

const char* afps_status_string(int status) {
    switch (status) {
        case AFPS_OK: return "ok";
        case AFPS_ERR_NULL: return "null pointer argument";
        case AFPS_ERR_ARG: return "invalid size arguments";
        case AFPS_ERR_RANGE: return "start index out of range";
        case AFPS_ERR_WORKSPACE: return "workspace missing or too small";
        case AFPS_ERR_HIP: return "HIP runtime error";
        case AFPS_ERR_UNSUPPORTED: return "problem exceeds the kernels' capacity";
        case AFPS_ERR_DEVICE: return "device-side failure";
        case AFPS_ERR_DATA: return "input coordinates violate the preconditions";
        default: return "unknown status";
    }
}

const char* afps_last_error(void) { return g_last_error.c_str(); }

int32_t afps_max_sector_points(void) { return kMaxFullSector; }

}  // extern "C"

namespace {

// afps_afps after argument validation (and the optional input check).
int afps_impl(const float* xyz, int32_t n, int32_t c, int32_t m, int32_t start, int32_t* out_idx,
              void* stream) {
    int rc;
    const int32_t ns = largest_sector(n, m);
    if (ns > kMaxFullSector) {
        if (m == 1) return launch_grid_fps(xyz, n, c, start, out_idx, (hipStream_t)stream);
        return fail(AFPS_ERR_UNSUPPORTED, "sector of " + std::to_string(ns) +
                                              " points exceeds one workgroup (use more sectors)");
    }
    DeviceState* d;
    if ((rc = device_state(&d))) return rc;
    const VariantEntry* v = choose_full(ns);
    if (!v) return fail(AFPS_ERR_UNSUPPORTED, "no kernel variant holds the sector");
    return launch_full_direct(*v, xyz, n, c, m, start, out_idx, (hipStream_t)stream);
}

}  // namespace

extern "C" {

int afps_afps(const float* xyz, int32_t n, int32_t c, int32_t m, int32_t start, int32_t* out_idx,
              void* stream) {
    if (!xyz || !out_idx) return fail(AFPS_ERR_NULL, "xyz and out_idx must be non-null");
    int rc = check_sizes(n, c, m, start);
    if (rc) return rc;
    if ((rc = maybe_check_cloud(xyz, n, stream))) return rc;
    return afps_impl(xyz, n, c, m, start, out_idx, stream);
}

int afps_afps_npdu_ex(const float* xyz, int32_t n, int32_t c, int32_t m, int32_t k, int32_t start,
                      int32_t flags, int32_t* out_idx, void* stream) {
    if (!xyz || !out_idx) return fail(AFPS_ERR_NULL, "xyz and out_idx must be non-null");
    int rc = check_sizes(n, c, m, start);
    if (rc) return rc;
    if (k < 0) return fail(AFPS_ERR_ARG, "NPDU needs k >= 0");
    if ((rc = npdu_readings(&k, &flags))) return rc;
    const int32_t ns = largest_sector(n, m);
    const NpduEntry* v = choose_npdu(ns);
    if (!v)
        return fail(AFPS_ERR_UNSUPPORTED, "NPDU sector of " + std::to_string(ns) +
                                              " points exceeds one workgroup (use more sectors)");
    if ((rc = maybe_check_cloud(xyz, n, stream))) return rc;
    DeviceState* d;
    if ((rc = device_state(&d))) return rc;
    return launch_npdu_direct(*v, xyz, n, c, m, clamp_k(k, ns), start, flags, out_idx, (hipStream_t)stream);
}

int afps_afps_npdu(const float* xyz, int32_t n, int32_t c, int32_t m, int32_t k, int32_t start,
                   int32_t* out_idx, void* stream) {
    return afps_afps_npdu_ex(xyz, n, c, m, k, start, 0, out_idx, stream);
}

int afps_fps_plain(const float* xyz, int32_t n, int32_t c, int32_t start, int32_t* out_idx,
                   void* stream) {
    if (!xyz || !out_idx) return fail(AFPS_ERR_NULL, "xyz and out_idx must be non-null");
    int rc = check_sizes(n, c, 1, start);
    if (rc) return rc;
    if ((rc = maybe_check_cloud(xyz, n, stream))) return rc;
    return afps_impl(xyz, n, c, 1, start, out_idx, stream);
}

int afps_afps_variant(const float* xyz, int32_t n, int32_t c, int32_t m, int32_t k, int32_t start,
                      int32_t flags, int32_t* out_idx, int32_t waves, int32_t slots, void* stream) {
    if (!xyz || !out_idx) return fail(AFPS_ERR_NULL, "xyz and out_idx must be non-null");
    int rc = check_sizes(n, c, m, start);
    if (rc) return rc;
    if ((rc = npdu_readings(&k, &flags))) return rc;
    if ((rc = maybe_check_cloud(xyz, n, stream))) return rc;
    const int32_t ns = largest_sector(n, m);
    DeviceState* d;
    if ((rc = device_state(&d))) return rc;
    if (k >= 0) {
        // NPDU: `slots` selects the chunk size in units of 64 points.
        for (const auto& v : registry().npdu)
            if (v.chunk64 == slots && capacity(v) >= ns && waves == 1)
                return launch_npdu_direct(v, xyz, n, c, m, clamp_k(k, ns), start, flags, out_idx,
                                          (hipStream_t)stream);
        return fail(AFPS_ERR_UNSUPPORTED, "no such NPDU variant for this sector size");
    }
    const VariantEntry* v = find_full(waves, slots);
    if (!v || capacity(*v) < ns) return fail(AFPS_ERR_UNSUPPORTED, "no such variant for this sector size");
    return launch_full_direct(*v, xyz, n, c, m, start, out_idx, (hipStream_t)stream);
}

int afps_tune_get(int32_t n_s, int32_t kind, int32_t* waves, int32_t* slots) {
    if (!waves || !slots) return fail(AFPS_ERR_NULL, "waves and slots must be non-null");
    if (n_s < 1) return fail(AFPS_ERR_ARG, "n_s must be positive");
    if (kind == AFPS_TUNE_NPDU) {
        const NpduEntry* v = choose_npdu(n_s);
        if (!v) return fail(AFPS_ERR_UNSUPPORTED, "sector too large");
        *waves = 1;
        *slots = v->chunk64;
        return AFPS_OK;
    }
    if (kind != AFPS_TUNE_DIRECT && kind != AFPS_TUNE_BATCH) return fail(AFPS_ERR_ARG, "unknown tuning kind");
    const VariantEntry* v = n_s <= kMaxFullSector ? choose_full(n_s, kind == AFPS_TUNE_BATCH) : nullptr;
    if (!v) return fail(AFPS_ERR_UNSUPPORTED, "sector too large");
    *waves = v->waves;
    *slots = v->slots;
    return AFPS_OK;
}

int afps_tune_set(int32_t n_s_max, int32_t kind, int32_t waves, int32_t slots) {
    if (kind != AFPS_TUNE_DIRECT && kind != AFPS_TUNE_BATCH)
        return fail(AFPS_ERR_ARG, "only full-update variants are tuned (NPDU uses one wave per sector)");
    const VariantEntry* v = find_full(waves, slots);
    if (!v || capacity(*v) < n_s_max) return fail(AFPS_ERR_ARG, "variant does not exist or is too small");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto& tab = g_tuned[kind == AFPS_TUNE_BATCH ? 1 : 0];
    tab.erase(std::remove_if(tab.begin(), tab.end(), [&](const Tuned& t) { return t.n_max == n_s_max; }),
              tab.end());
    tab.push_back({n_s_max, waves, slots});
    std::sort(tab.begin(), tab.end(), [](const Tuned& a, const Tuned& b) { return a.n_max < b.n_max; });
    return AFPS_OK;
}

void afps_tune_reset(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& tab : g_tuned) tab.clear();
    const float occupancy = g_pool_policy.waves_per_simd;
    g_pool_policy = PoolPolicy();
    g_pool_policy.waves_per_simd = occupancy;
    g_tune_loaded = true;   // forget the cache file too
}

int afps_set_plan_occupancy(float waves_per_simd) {
    if (!(waves_per_simd >= 0.0f) || waves_per_simd > 64.0f)
        return fail(AFPS_ERR_ARG, "waves per SIMD must be 0 (no budget) or in (0, 64]");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_pool_policy.waves_per_simd = waves_per_simd;
    return AFPS_OK;
}

int afps_tune_npdu(int32_t n_s_max, int32_t k_max, int32_t xyz_in_lds) {
    if (n_s_max < 1 || k_max < 0 || (xyz_in_lds != 0 && xyz_in_lds != 1))
        return fail(AFPS_ERR_ARG, "need n_s_max >= 1, k_max >= 0 and xyz_in_lds 0 or 1");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto& tab = g_pool_policy.placement;
    tab.erase(std::remove_if(tab.begin(), tab.end(),
                             [&](const NpduPlacement& e) { return e.n_max == n_s_max && e.k_max == k_max; }),
              tab.end());
    tab.push_back({n_s_max, k_max, xyz_in_lds});
    sort_placement(tab);
    return AFPS_OK;
}

int afps_set_pool_policy(int32_t waves, int32_t groups_per_cu, int32_t seed_sleep, int32_t seed_priority) {
    if (!valid_pool_policy(waves, groups_per_cu, seed_sleep, seed_priority))
        return fail(AFPS_ERR_ARG, "pool shape must be (0, 0), (4|8|12|16 waves, 1 group) or (4|12|16 waves, 2 groups); "
                                  "seed_sleep 0|1; seed_priority 0..3");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    g_pool_policy.waves = waves;
    g_pool_policy.groups = groups_per_cu;
    g_pool_policy.seed_sleep = seed_sleep != 0;
    g_pool_policy.seed_priority = seed_priority;
    return AFPS_OK;
}

void afps_tune_npdu_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    const float occupancy = g_pool_policy.waves_per_simd;
    g_pool_policy = PoolPolicy();
    g_pool_policy.waves_per_simd = occupancy;
}

int afps_npdu_xyz_in_lds(int32_t n_s, int32_t k) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    return npdu_xyz_in_lds(g_pool_policy, n_s, k) ? 1 : 0;
}

size_t afps_bin_workspace_bytes(int32_t n, int32_t bins) {
    if (n < 1 || bins < 1 || bins > kMaxBins) return 0;
    const size_t chunks = ((size_t)n + kBinChunk - 1) / kBinChunk;
    auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
    // header, bin sizes / first positions, per-chunk histograms
    return sizeof(BinHeader) + r256((size_t)bins * sizeof(uint32_t)) + r256(chunks * (size_t)bins * sizeof(uint32_t));
}

int afps_bin_points(const float* xyz, int32_t n, int32_t axis, int32_t bins, int32_t* perm, float* xyz_out,
                    void* workspace, size_t workspace_bytes, void* stream_) {
    if (!xyz || !perm) return fail(AFPS_ERR_NULL, "xyz and perm must be non-null");
    if (n < 1) return fail(AFPS_ERR_ARG, "n must be >= 1");
    if (axis < 0 || axis > 2) return fail(AFPS_ERR_ARG, "axis must be 0, 1 or 2");
    if (bins < 1 || bins > kMaxBins) return fail(AFPS_ERR_ARG, "bins must be in [1, " + std::to_string(kMaxBins) + "]");
    if (xyz_out == xyz) return fail(AFPS_ERR_ARG, "xyz_out must not be xyz");
    const size_t need = afps_bin_workspace_bytes(n, bins);
    if (!workspace || workspace_bytes < need)
        return fail(AFPS_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace & 255) != 0) return fail(AFPS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    int rc = maybe_check_cloud(xyz, n, stream_);
    if (rc) return rc;
    hipStream_t stream = (hipStream_t)stream_;
    const BinKernels k = bin_kernels();
    BinHeader* h = (BinHeader*)workspace;
    uint32_t* totals = (uint32_t*)((char*)workspace + sizeof(BinHeader));
    uint32_t* hist = totals + ((size_t)bins * sizeof(uint32_t) + 255) / 256 * 64;
    int chunks = (int)(((int64_t)n + kBinChunk - 1) / kBinChunk);
    void* a0[] = {&h};
    AFPS_HIP(hipLaunchKernel(k.reset, dim3(1), dim3(64), a0, 0, stream));
    void* a1[] = {(void*)&xyz, &n, &axis, &h};
    AFPS_HIP(hipLaunchKernel(k.range, dim3(std::min(chunks, 1024)), dim3(256), a1, 0, stream));
    void* a2[] = {(void*)&xyz, &n, &axis, &bins, &h, &hist};
    AFPS_HIP(hipLaunchKernel(k.count, dim3(chunks), dim3(256), a2, 0, stream));
    void* a3[] = {&hist, &totals, &chunks, &bins};
    AFPS_HIP(hipLaunchKernel(k.scan_rows, dim3((bins + 3) / 4), dim3(256), a3, 0, stream));
    void* a4[] = {&totals, &bins};
    AFPS_HIP(hipLaunchKernel(k.scan_totals, dim3(1), dim3(1024), a4, 0, stream));
    void* a5[] = {(void*)&xyz, &n, &axis, &bins, &h, &hist, &totals, &perm, &xyz_out};
    AFPS_HIP(hipLaunchKernel(k.scatter, dim3(chunks), dim3(64), a5, 0, stream));
    return AFPS_OK;
}

int afps_ball_query(const float* xyz, int32_t n, const int32_t* centers, int32_t c, float radius, int32_t k,
                    int32_t window, int32_t* out_idx, int32_t* out_cnt, void* stream) {
    if (!xyz || !centers || !out_idx) return fail(AFPS_ERR_NULL, "xyz, centers and out_idx must be non-null");
    if (n < 1) return fail(AFPS_ERR_ARG, "n must be >= 1");
    if (c < 0) return fail(AFPS_ERR_ARG, "c must be >= 0");
    if (k < 1) return fail(AFPS_ERR_ARG, "k must be >= 1");
    if (!(radius >= 0.0f)) return fail(AFPS_ERR_ARG, "radius must be >= 0");
    if (c == 0) return AFPS_OK;
    int rc = maybe_check_cloud(xyz, n, stream);
    if (rc) return rc;
    const float r2 = radius * radius;   // fp32, as the oracle rounds it
    uint32_t r2_bits;
    std::memcpy(&r2_bits, &r2, sizeof(r2_bits));
    DeviceState* ds = nullptr;
    if ((rc = device_state(&ds))) return rc;
    const int waves = 4;   // one centre per wave, four waves per workgroup
    const int grid = (int)std::min<int64_t>(((int64_t)c + waves - 1) / waves, (int64_t)ds->cu_count * 16);
    void* args[] = {(void*)&xyz, &n, (void*)&centers, &c, &r2_bits, &k, &window, &out_idx, &out_cnt};
    AFPS_HIP(hipLaunchKernel(ball_query_kernel_ptr(), dim3(grid), dim3(64 * waves), args, 0, (hipStream_t)stream));
    return AFPS_OK;
}

int afps_check_points(const float* xyz, int64_t n, void* stream) {
    if (!xyz) return fail(AFPS_ERR_NULL, "xyz must be non-null");
    if (n < 0 || n > INT32_MAX) return fail(AFPS_ERR_ARG, "n must be in [0, 2^31-1]");
    if (n == 0) return AFPS_OK;
    return check_clouds(xyz, {CheckSeg{0, (int32_t)n, 0}}, (hipStream_t)stream, {""});
}

int afps_set_checking(int32_t on) {
    g_checking = on != 0;
    return AFPS_OK;
}

int afps_set_spin_limit(uint32_t polls) {
    if (polls == 0) return fail(AFPS_ERR_ARG, "spin limit must be positive");
    g_spin_limit = polls;
    return AFPS_OK;
}

}  // extern "C"

// ================================================================ batch plans

// A batch plan: the planner's tables (host logic, planner.cpp) plus the
// kernels they map to and the HIP objects of its launches.
struct afps_plan {
    std::vector<WorkItem> items;
    std::vector<PlannedBucket> buckets;
    std::vector<const void*> kernels;  // the kernel of each bucket
    std::vector<PoolGroup> groups;    // each pooled workgroup's queues
    std::vector<PoolQueue> queues;    // every pooled workgroup's queues, highest priority first
    std::vector<PoolSeed> seeds;      // first sector of each pool wave (workgroup-major)
    std::vector<CheckSeg> clouds;     // each descriptor's points, for the optional input check
    int pool_pages = 0;               // LDS pages of one pooled workgroup
    int pool_groups = 0;              // pooled workgroups per CU (1 or 2; 0 without NPDU sectors)
    int pool_waves = 0;
    bool pool_lite = false;           // the light pooled kernel (every NPDU sector npdu_item_lite)
    int seed_priority = 0;
    size_t ws_bytes = 0;
    int device = 0;
    std::vector<hipEvent_t> events;   // fork / join events (1 + helper streams)
    std::mutex mu;
    hipGraphExec_t exec = nullptr;
    const void* g_xyz = nullptr;
    void* g_out = nullptr;
    void* g_ws = nullptr;
    hipStream_t capture = nullptr;   // stream the graph is captured on
    ~afps_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (capture) (void)hipStreamDestroy(capture);
        for (auto e : events) (void)hipEventDestroy(e);
    }
};

extern "C" {

int afps_plan_create(const afps_cloud_desc* descs, int32_t batch, afps_plan** plan_out) {
    if (!plan_out || (!descs && batch > 0)) return fail(AFPS_ERR_NULL, "descs and plan must be non-null");
    *plan_out = nullptr;
    if (batch < 0) return fail(AFPS_ERR_ARG, "batch must be >= 0");
    // Validation and sector expansion first (host only): a bad descriptor is
    // reported before anything touches a device.
    PlannerEnv env;
    env.cu_count = 1;
    env.cu_pool_pages = kMaxPoolPages;
    PlanTables pre;
    std::string err;
    env.choose_full = [](int n, FullVariantInfo* v) { return batch_variant(n, v); };
    env.blocks_per_cu = [](const FullVariantInfo&) { return 1; };
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_file_locked();
        env.pool = g_pool_policy;
    }
    int rc = build_plan(descs, batch, env, &pre, &err);
    if (rc && rc != AFPS_ERR_UNSUPPORTED) return fail(rc, err);
    std::unique_ptr<afps_plan> plan(new afps_plan());
    DeviceState* ds = nullptr;
    if (batch > 0) {
        if ((rc = device_state(&ds))) return rc;
        AFPS_HIP(hipGetDevice(&plan->device));
        env.cu_count = ds->cu_count;
        env.cu_pool_pages = ds->pool_pages;
    }
    env.blocks_per_cu = [](const FullVariantInfo& v) {
        int per_cu = 0;
        const VariantEntry& e = registry().full[v.id];
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, e.persistent, 64 * e.waves, e.lds_bytes) !=
            hipSuccess)
            return 0;
        return per_cu;
    };
    PlanTables t;
    if ((rc = build_plan(descs, batch, env, &t, &err))) return fail(rc, err);
    plan->items = std::move(t.items);
    plan->buckets = std::move(t.buckets);
    plan->groups = std::move(t.groups);
    plan->queues = std::move(t.queues);
    plan->seeds = std::move(t.seeds);
    plan->clouds = std::move(t.clouds);
    plan->pool_pages = t.pool_pages;
    plan->pool_groups = t.pool_groups;
    plan->pool_waves = t.pool_waves;
    plan->pool_lite = t.pool_lite;
    plan->seed_priority = t.seed_priority;
    plan->ws_bytes = t.ws_bytes;
    for (const auto& bk : plan->buckets) {
        const void* k = nullptr;
        if (bk.pool()) {
            for (const auto& v : registry().pool)
                if (v.waves == plan->pool_waves && v.lite == plan->pool_lite) k = v.kernel;
        } else {
            k = registry().full[bk.variant].persistent;
        }
        if (!k) return fail(AFPS_ERR_UNSUPPORTED, "a planned kernel is not built");
        plan->kernels.push_back(k);
    }
    if (!plan->buckets.empty()) {
        if (plan->buckets.size() > 1) {
            int hrc = helper_streams(ds);   // created outside any stream capture
            if (hrc) return hrc;
        }
        const int n_events = 1 + kHelperStreams;
        for (int i = 0; i < n_events; ++i) {
            hipEvent_t e;
            AFPS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            plan->events.push_back(e);
        }
    }
    *plan_out = plan.release();
    return AFPS_OK;
}

size_t afps_plan_workspace_bytes(const afps_plan* plan) { return plan ? plan->ws_bytes : 0; }

size_t afps_workspace_bytes_for_items(int32_t items) { return workspace_bytes_for_items(items); }
int32_t afps_plan_items(const afps_plan* plan) { return plan ? (int32_t)plan->items.size() : 0; }

int32_t afps_plan_launches(const afps_plan* plan) { return plan ? (int32_t)plan->buckets.size() : 0; }

int32_t afps_plan_pool_waves(const afps_plan* plan) { return plan ? plan->pool_waves : 0; }

int32_t afps_plan_pool_groups_per_cu(const afps_plan* plan) { return plan ? plan->pool_groups : 0; }

void afps_plan_destroy(afps_plan* plan) { delete plan; }

}  // extern "C"

namespace {

// Copy the plan's tables (pool groups, queues and seeds, work items) into a
// workspace.  Pageable sources: the copies have consumed the host tables when
// this returns.
int upload_tables(const afps_plan* plan, void* workspace, hipStream_t stream) {
    if (!plan->groups.empty())
        AFPS_HIP(hipMemcpyAsync((char*)workspace + kPoolGroupOffset, plan->groups.data(),
                                plan->groups.size() * sizeof(PoolGroup), hipMemcpyHostToDevice, stream));
    if (!plan->queues.empty())
        AFPS_HIP(hipMemcpyAsync((char*)workspace + pool_queue_offset((int64_t)plan->items.size()),
                                plan->queues.data(), plan->queues.size() * sizeof(PoolQueue),
                                hipMemcpyHostToDevice, stream));
    if (!plan->seeds.empty())
        AFPS_HIP(hipMemcpyAsync((char*)workspace + kPoolSeedOffset, plan->seeds.data(),
                                plan->seeds.size() * sizeof(PoolSeed), hipMemcpyHostToDevice, stream));
    AFPS_HIP(hipMemcpyAsync((char*)workspace + kItemsOffset, plan->items.data(),
                            plan->items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, stream));
    return AFPS_OK;
}

}  // namespace

extern "C" {

int afps_plan_upload(afps_plan* plan, void* workspace, size_t workspace_bytes, void* stream) {
    if (!plan) return fail(AFPS_ERR_NULL, "plan must be non-null");
    if (plan->items.empty()) return AFPS_OK;
    if (!workspace || workspace_bytes < plan->ws_bytes)
        return fail(AFPS_ERR_WORKSPACE, "workspace needs " + std::to_string(plan->ws_bytes) + " bytes");
    if (((uintptr_t)workspace & 255) != 0) return fail(AFPS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    return upload_tables(plan, workspace, (hipStream_t)stream);
}

}  // extern "C"

namespace {

int check_plan_clouds(const afps_plan* plan, const float* xyz_all, hipStream_t stream) {
    std::vector<std::string> names;
    for (size_t i = 0; i < plan->clouds.size(); ++i) names.push_back("cloud " + std::to_string(i) + ": ");
    return check_clouds(xyz_all, plan->clouds, stream, names);
}

// Clear `words` counters on `stream` with a kernel (a memset node would
// misbehave in a replayed graph).
int reset_words(unsigned* words, int count, hipStream_t stream) {
    void* args[] = {&words, &count};
    AFPS_HIP(hipLaunchKernel(queue_reset_kernel(), dim3((count + 255) / 256), dim3(256), args, 0, stream));
    return AFPS_OK;
}

// afps_plan_launch after argument checks: launches only (capturable).
// `stamps`: per-item timestamps of the pooled NPDU launch, or nullptr.
// `rounds`/`nrounds`: a launch of several rounds (pooled plans only): per-round
// inputs and outputs (DEVICE).
int plan_launch_impl(const afps_plan* plan, const float* xyz_all, int32_t* out_all, void* workspace,
                     hipStream_t stream, SectorStamp* stamps = nullptr, const PoolRound* rounds = nullptr,
                     int nrounds = 1) {
    DeviceState* d;
    int rc = device_state(&d);
    if (rc) return rc;
    unsigned* counters = (unsigned*)workspace;
    const PoolGroup* groups = (const PoolGroup*)((char*)workspace + kPoolGroupOffset);
    const PoolQueue* queues = (const PoolQueue*)((char*)workspace + pool_queue_offset((int64_t)plan->items.size()));
    const PoolSeed* seeds = (const PoolSeed*)((char*)workspace + kPoolSeedOffset);
    const WorkItem* items = (const WorkItem*)((char*)workspace + kItemsOffset);
    int nb = (int)plan->buckets.size();
    if ((rc = reset_words(counters, kResetWords, stream))) return rc;

    auto launch_bucket = [&](int b, hipStream_t s) -> int {
        const PlannedBucket& bk = plan->buckets[b];
        const void* kernel = plan->kernels[b];
        if (bk.pool()) {
            PoolArgs pa{};
            pa.xyz_all = xyz_all;
            pa.out_all = out_all;
            pa.rounds = rounds;
            pa.nrounds = nrounds;
            pa.items = items;
            pa.groups = groups;
            pa.queues = queues;
            pa.seeds = seeds;
            pa.status = counters + kStatusWord;
            pa.dev_status = d->status;
            pa.stamps = stamps;
            pa.pool_pages = plan->pool_pages;
            pa.spin_limit = g_spin_limit;
            pa.seed_priority = plan->seed_priority;
            void* args[] = {&pa};
            AFPS_HIP(hipLaunchKernel(kernel, dim3(bk.grid), dim3(bk.block), args, bk.lds_bytes, s));
            return AFPS_OK;
        }
        const WorkItem* first = items + bk.first;
        int count = bk.count;
        unsigned* counter = counters + b;
        void* args[] = {(void*)&xyz_all, (void*)&out_all, (void*)&first, (void*)&count, (void*)&counter};
        AFPS_HIP(hipLaunchKernel(kernel, dim3(bk.grid), dim3(bk.block), args, bk.lds_bytes, s));
        return AFPS_OK;
    };
    if (nb == 1) return launch_bucket(0, stream);

    // Several variants: run them concurrently on helper streams (fork / join
    // through events, which a stream capture records as graph edges).
    if ((rc = helper_streams(d))) return rc;
    AFPS_HIP(hipEventRecord(plan->events[0], stream));
    const int used = std::min(nb, kHelperStreams);
    for (int h = 0; h < used; ++h) AFPS_HIP(hipStreamWaitEvent(d->helpers[h], plan->events[0], 0));
    for (int b = 0; b < nb; ++b)
        if ((rc = launch_bucket(b, d->helpers[b % kHelperStreams]))) return rc;
    for (int h = 0; h < used; ++h) {
        AFPS_HIP(hipEventRecord(plan->events[1 + h], d->helpers[h]));
        AFPS_HIP(hipStreamWaitEvent(stream, plan->events[1 + h], 0));
    }
    return AFPS_OK;
}

int plan_launch_args(const afps_plan* plan, const float* xyz_all, int32_t* out_all, void* workspace) {
    if (!plan) return fail(AFPS_ERR_NULL, "plan must be non-null");
    if (plan->items.empty()) return AFPS_OK;
    if (!xyz_all || !out_all) return fail(AFPS_ERR_NULL, "xyz_all and out_all must be non-null");
    if (!workspace) return fail(AFPS_ERR_WORKSPACE, "workspace must be non-null");
    return AFPS_OK;
}

}  // namespace

extern "C" {

int afps_plan_launch(const afps_plan* plan, const float* xyz_all, int32_t* out_all, void* workspace,
                     void* stream) {
    int rc = plan_launch_args(plan, xyz_all, out_all, workspace);
    if (rc || plan->items.empty()) return rc;
    if (g_checking && (rc = check_plan_clouds(plan, xyz_all, (hipStream_t)stream))) return rc;
    return plan_launch_impl(plan, xyz_all, out_all, workspace, (hipStream_t)stream);
}

int afps_plan_graph_launch(afps_plan* plan, const float* xyz_all, int32_t* out_all, void* workspace,
                           void* stream_) {
    int rc0 = plan_launch_args(plan, xyz_all, out_all, workspace);
    if (rc0 || plan->items.empty()) return rc0;
    hipStream_t stream = (hipStream_t)stream_;
    // The check synchronises the stream, so it runs before the replay, never
    // inside the capture.
    if (g_checking && (rc0 = check_plan_clouds(plan, xyz_all, stream))) return rc0;
    std::lock_guard<std::mutex> lk(plan->mu);
    if (!plan->exec || plan->g_xyz != xyz_all || plan->g_out != out_all || plan->g_ws != workspace) {
        if (plan->exec) {
            (void)hipGraphExecDestroy(plan->exec);
            plan->exec = nullptr;
        }
        // Capture on the plan's own stream (the caller's may be the null
        // stream, which cannot be captured); replay on the caller's stream.
        if (!plan->capture) AFPS_HIP(hipStreamCreateWithFlags(&plan->capture, hipStreamNonBlocking));
        AFPS_HIP(hipStreamBeginCapture(plan->capture, hipStreamCaptureModeThreadLocal));
        int rc = plan_launch_impl(plan, xyz_all, out_all, workspace, plan->capture);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(plan->capture, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        plan->g_xyz = xyz_all;
        plan->g_out = out_all;
        plan->g_ws = workspace;
    }
    AFPS_HIP(hipGraphLaunch(plan->exec, stream));
    return AFPS_OK;
}

int afps_plan_launch_noalloc(const afps_plan* plan, const float* xyz_all, int32_t* out_all, void* stream_) {
    if (!plan) return fail(AFPS_ERR_NULL, "plan must be non-null");
    if (plan->items.empty()) return AFPS_OK;
    if (!xyz_all || !out_all) return fail(AFPS_ERR_NULL, "xyz_all and out_all must be non-null");
    if (plan->ws_bytes > kScratchBytes)
        return fail(AFPS_ERR_WORKSPACE, "the plan needs " + std::to_string(plan->ws_bytes) +
                                            " bytes of workspace; the static scratch holds " +
                                            std::to_string(kScratchBytes) + " (at most " +
                                            std::to_string(afps_noalloc_max_items()) + " sectors)");
    DeviceState* d;
    int rc = device_state(&d);
    if (rc) return rc;
    int dev = 0;
    AFPS_HIP(hipGetDevice(&dev));
    if (dev != plan->device)
        return fail(AFPS_ERR_ARG, "the plan was built on device " + std::to_string(plan->device) +
                                      ", the current device is " + std::to_string(dev));
    hipStream_t stream = (hipStream_t)stream_;
    if (g_checking && (rc = check_plan_clouds(plan, xyz_all, stream))) return rc;
    // The tables go into this device's scratch on the launch stream, then the
    // same launches as afps_plan_launch; the reset kernel clears the counters.
    if ((rc = upload_tables(plan, d->scratch, stream))) return rc;
    return plan_launch_impl(plan, xyz_all, out_all, d->scratch, stream);
}

int32_t afps_noalloc_max_items(void) {
    // the largest count whose workspace (a queue per item at most) fits the scratch
    int32_t lo = 0, hi = (int32_t)(kScratchBytes / sizeof(WorkItem));
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (workspace_bytes_for_items(mid) <= kScratchBytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

int afps_plan_launch_stamped(const afps_plan* plan, const float* xyz_all, int32_t* out_all, void* workspace,
                             void* stamps, size_t stamp_bytes, void* stream) {
    int rc = plan_launch_args(plan, xyz_all, out_all, workspace);
    if (rc || plan->items.empty()) return rc;
    if (!stamps) return fail(AFPS_ERR_NULL, "stamps must be non-null");
    const size_t need = plan->items.size() * sizeof(SectorStamp);
    if (stamp_bytes < need) return fail(AFPS_ERR_WORKSPACE, "stamps need " + std::to_string(need) + " bytes");
    if (((uintptr_t)stamps & 63) != 0) return fail(AFPS_ERR_WORKSPACE, "stamps must be 64-byte aligned");
    if (g_checking && (rc = check_plan_clouds(plan, xyz_all, (hipStream_t)stream))) return rc;
    return plan_launch_impl(plan, xyz_all, out_all, workspace, (hipStream_t)stream, (SectorStamp*)stamps);
}

size_t afps_plan_rounds_workspace_bytes(const afps_plan* plan, int32_t rounds) {
    if (!plan || plan->items.empty() || rounds < 1 || rounds > kMaxRounds) return 0;
    return plan->ws_bytes;   // the claim counters of a pooled launch live in LDS
}

int afps_plan_launch_rounds(const afps_plan* plan, const afps_round* rounds, int32_t count, void* workspace,
                            size_t workspace_bytes, void* stream) {
    if (!plan) return fail(AFPS_ERR_NULL, "plan must be non-null");
    if (plan->items.empty()) return AFPS_OK;
    if (!rounds) return fail(AFPS_ERR_NULL, "rounds must be non-null");
    if (count < 1 || count > kMaxRounds)
        return fail(AFPS_ERR_ARG, "rounds must be in [1, " + std::to_string(kMaxRounds) + "]");
    if (plan->buckets.size() != 1 || !plan->buckets[0].pool())
        return fail(AFPS_ERR_UNSUPPORTED, "launches of several rounds take plans whose sectors all use NPDU");
    const size_t need = afps_plan_rounds_workspace_bytes(plan, count);
    if (!workspace || workspace_bytes < need)
        return fail(AFPS_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace & 255) != 0) return fail(AFPS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (g_checking)
        return fail(AFPS_ERR_UNSUPPORTED, "input checking cannot read the device round table; "
                                          "check each round's clouds with afps_check_points");
    static_assert(sizeof(afps_round) == sizeof(PoolRound), "round table layout");
    return plan_launch_impl(plan, nullptr, nullptr, workspace, (hipStream_t)stream, nullptr,
                            (const PoolRound*)rounds, count);
}

int afps_plan_status(const afps_plan* plan, const void* workspace, void* stream_) {
    if (!plan) return fail(AFPS_ERR_NULL, "plan must be non-null");
    if (plan->items.empty()) return AFPS_OK;
    if (!workspace) return fail(AFPS_ERR_WORKSPACE, "workspace must be non-null");
    hipStream_t stream = (hipStream_t)stream_;
    unsigned word = 0;
    AFPS_HIP(hipMemcpyAsync(&word, (const unsigned*)workspace + kStatusWord, sizeof(word), hipMemcpyDeviceToHost,
                            stream));
    AFPS_HIP(hipStreamSynchronize(stream));
    if (word) return fail(AFPS_ERR_DEVICE, "a wave of the plan's last launch gave up a bounded wait; "
                                           "the sectors it could not run hold -1");
    return AFPS_OK;
}

int afps_device_status(void* stream_, int32_t clear) {
    DeviceState* d;
    int rc = device_state(&d);
    if (rc) return rc;
    hipStream_t stream = (hipStream_t)stream_;
    unsigned word = 0;
    AFPS_HIP(hipMemcpyAsync(&word, d->status, sizeof(word), hipMemcpyDeviceToHost, stream));
    if (clear) AFPS_HIP(hipMemsetAsync(d->status, 0, sizeof(unsigned), stream));
    AFPS_HIP(hipStreamSynchronize(stream));
    if (word) return fail(AFPS_ERR_DEVICE, "a kernel gave up a bounded wait on this device; "
                                           "its unfinished outputs hold -1");
    return AFPS_OK;
}

int32_t afps_wall_clock_khz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return khz;
}

int afps_init(void) {
    DeviceState* d;
    return device_state(&d);
}

size_t afps_batched_workspace_bytes(const afps_cloud_desc* descs, int32_t batch) {
    afps_plan* p = nullptr;
    if (afps_plan_create(descs, batch, &p) != AFPS_OK) return 0;
    const size_t b = p->ws_bytes;
    afps_plan_destroy(p);
    return b;
}

int afps_batched(const float* xyz_all, const afps_cloud_desc* descs, int32_t batch, int32_t* out_all,
                 void* workspace, size_t workspace_bytes, void* stream) {
    if (batch > 0 && (!xyz_all || !out_all)) return fail(AFPS_ERR_NULL, "xyz_all and out_all must be non-null");
    afps_plan* p = nullptr;
    int rc = afps_plan_create(descs, batch, &p);
    if (rc) return rc;
    rc = afps_plan_upload(p, workspace, workspace_bytes, stream);
    if (!rc) rc = afps_plan_launch(p, xyz_all, out_all, workspace, stream);
    afps_plan_destroy(p);
    return rc;
}

}  // extern "C"
