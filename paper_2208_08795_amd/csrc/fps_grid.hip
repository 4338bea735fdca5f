// Plain FPS (Algorithm 1) on a cloud larger than one workgroup holds.
//
// G workgroups (launched cooperatively, so all are resident) each keep a
// contiguous block of `chunk` points in registers.  Every iteration each
// workgroup updates its block and finds its lowest-index maximum, then
// publishes it as ONE 64-bit word in its slot:
//
//     bits 63..32  distance (fp32 bits)
//     bits 31..16  iteration tag (i mod 2^16)
//     bits 15..0   index inside the workgroup's block (chunk <= 2^16)
//
// with a relaxed device-scope atomic store.  Every wave then polls all G
// slots with relaxed device-scope atomic loads until each carries this
// iteration's tag: the poll that completes the barrier also delivers every
// candidate, and since each slot is a single atomic word no other memory
// ordering is needed.  The winner is the maximum distance, ties to the lowest
// workgroup (blocks are in index order) and within it the reported lowest
// index; its coordinates are read from the (read-only) input.  Slots are
// double-buffered by iteration parity: a workgroup can only overwrite a
// parity-p slot after every workgroup published the next iteration, i.e.
// after every workgroup read the parity-p slots.
//
// Every wait is bounded: after `spin_limit` polls a wave marks the launch
// failed (and the device's failure word, which afps_device_status reports)
// and returns; the other workgroups notice the mark and return too, and the
// waves of its own workgroup return together with it (a flag in LDS, read
// after the next candidate exchange, so that no wave goes on with a
// candidate its sibling never wrote).  Workgroup 0 fills the unfinished
// outputs with -1.  This per-iteration synchronisation is the cost the
// paper's sectors avoid (Sec. III-B).
#include "sampler.hpp"
#include "variants.hpp"

namespace afps {

struct GridSync {
    unsigned failed;        // set when a workgroup gave up waiting
    unsigned pad[63];
    uint64_t slot[2][kMaxGridGroups];
    uint64_t spare[(kGridSyncBytes - 256) / 8 - 2 * kMaxGridGroups];
};
static_assert(sizeof(GridSync) == kGridSyncBytes, "barrier block layout");

template <int P, int W>
__global__ __launch_bounds__(64 * W) void fps_grid_kernel(const float* __restrict__ xyz, int n,
                                                          int c, int start, int chunk,
                                                          int32_t* __restrict__ out, GridSync* gs,
                                                          unsigned spin_limit, unsigned* dev_status) {
    constexpr int T = 64 * W;
    __shared__ Candidate lds[2 * W];
    __shared__ unsigned gave_up;   // a wave of this workgroup gave up waiting and returned
    const int G = gridDim.x;
    const int g = blockIdx.x;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int first = g * chunk;
    const int cnt = min(chunk, n - first);
    const int ns = (cnt + T - 1) / T;
    if (W > 1) {
        if (t == 0) gave_up = 0u;
        __syncthreads();
    }

    float X[P], Y[P], Z[P];
    Dist<P, T, false> D;
    load_points<P, T, false>(xyz + 3 * (int64_t)first, cnt, ns, t, X, Y, Z, D);
    float px = xyz[3 * (int64_t)start + 0], py = xyz[3 * (int64_t)start + 1],
          pz = xyz[3 * (int64_t)start + 2];
    // Picks are buffered one per lane (pick i in lane i mod 64); wave 0 of
    // workgroup 0 writes them 64 at a time.
    uint32_t picks = (uint32_t)start;
    // Leave at iteration i without its pick: workgroup 0's wave 0 writes the
    // buffered picks before i and -1 from i on.
    auto leave = [&](int i) {
        if (g == 0 && w == 0) {
            const int done = i & ~63;   // picks before `done` are written
            if (lane < (i & 63)) out[done + lane] = (int32_t)picks;
            for (int j = i + lane; j < c; j += 64) out[j] = -1;
        }
    };

    for (int i = 1; i < c; ++i) {
        const Pick mine = update_and_pick<P, T, false>(ns, w, lane, X, Y, Z, D, px, py, pz);
        const Pick p = combine_waves<W>(mine, lds, i & 1, w, lane);
        // After the exchange's barrier: a sibling that gave up has returned
        // (and no longer writes its candidate), so this wave returns too.
        if (W > 1 && __hip_atomic_load(&gave_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            leave(i);
            return;
        }
        const uint64_t tag = (uint64_t)(i & 0xFFFF);
        uint64_t* slots = gs->slot[i & 1];
        if (t == 0)
            __hip_atomic_store(&slots[g], ((uint64_t)p.d << 32) | (tag << 16) | (uint64_t)p.idx,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // Poll every slot (lane l reads workgroup l's) until all carry tag i.
        uint64_t v = 0;
        bool ok = true;
        for (unsigned spins = 0;; ++spins) {
            if (lane < G) v = __hip_atomic_load(&slots[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool ready = lane >= G || ((v >> 16) & 0xFFFF) == tag;
            if (ballot(!ready) == 0) break;
            if (spins >= spin_limit ||
                ((spins & 255u) == 255u &&
                 __hip_atomic_load(&gs->failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ok) {
            if (lane == 0) {
                __hip_atomic_store(&gs->failed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_or(dev_status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (W > 1) __hip_atomic_store(&gave_up, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            // the flag is in LDS before this wave ends (its siblings read it
            // after their next barrier, which this wave no longer holds up)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            leave(i);
            return;
        }
        const uint32_t d = lane < G ? (uint32_t)(v >> 32) : 0u;
        const uint32_t best = wave_max(d);
        const int win = (int)__builtin_ctzll(ballot(lane < G && d == best));
        const int cur = win * chunk + (int)(readlane((uint32_t)(v & 0xFFFF), win));
        px = xyz[3 * (int64_t)cur + 0];
        py = xyz[3 * (int64_t)cur + 1];
        pz = xyz[3 * (int64_t)cur + 2];
        const int slot = i & 63;
        picks = lane == slot ? (uint32_t)cur : picks;
        if (slot == 63 && g == 0 && w == 0) out[i - 63 + lane] = (int32_t)picks;
    }
    const int tail = (c - 1) & 63;   // picks of the last, partial group
    if (g == 0 && w == 0 && tail != 63 && lane <= tail) out[(c - 1) - tail + lane] = (int32_t)picks;
}

__global__ void grid_reset(GridSync* gs) {
    const int t = threadIdx.x;
    if (t == 0) gs->failed = 0u;
    if (t < kMaxGridGroups) {
        gs->slot[0][t] = 0ull;
        gs->slot[1][t] = 0ull;
    }
}

const void* grid_reset_kernel() { return (const void*)&grid_reset; }

void register_grid_variants(std::vector<GridVariant>& v) {
    v.push_back({16, 4, (const void*)&fps_grid_kernel<4, 16>});
    v.push_back({16, 8, (const void*)&fps_grid_kernel<8, 16>});
    v.push_back({16, 16, (const void*)&fps_grid_kernel<16, 16>});
}

}  // namespace afps
