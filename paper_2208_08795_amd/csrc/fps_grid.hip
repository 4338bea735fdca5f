// Plain FPS (Algorithm 1) on a cloud larger than one workgroup holds.
//
// G workgroups (launched cooperatively, so all are resident) each keep a
// contiguous block of `chunk` points in registers.  Every iteration each
// workgroup updates its block and finds its lowest-index maximum, publishes
// it in a per-workgroup slot, and arrives at a grid barrier (a release add on
// one counter; the waiters spin with acquire loads).  After the barrier every
// workgroup reads all G slots and takes the maximum, ties to the lowest
// index: every workgroup reaches the same pick without a second barrier.
// Slots are double-buffered by iteration parity: a workgroup can only
// overwrite a parity-p slot after everybody passed the next barrier, i.e.
// after everybody read it.  This per-iteration synchronisation is the cost
// that the paper's sectors avoid (Sec. III-B).
//
// Every wait is bounded: after `spin_limit` polls a workgroup marks the
// launch failed, returns, and the others notice the mark and return too;
// workgroup 0 then fills the unfinished outputs with -1.
#include "sampler.hpp"
#include "variants.hpp"

namespace afps {

struct GridSync {
    unsigned arrive;        // barrier arrivals since the reset
    unsigned failed;        // set when a workgroup gave up waiting
    unsigned pad[62];
    Candidate cand[2][kMaxGridGroups];
};
static_assert(sizeof(GridSync) == kGridSyncBytes, "barrier block layout");

template <int P, int W>
__global__ __launch_bounds__(64 * W) void fps_grid_kernel(const float* __restrict__ xyz, int n,
                                                          int c, int start, int chunk,
                                                          int32_t* __restrict__ out, GridSync* gs,
                                                          unsigned spin_limit) {
    constexpr int T = 64 * W;
    __shared__ Candidate lds[2 * W];
    __shared__ unsigned go;
    const int G = gridDim.x;
    const int g = blockIdx.x;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int first = g * chunk;
    const int cnt = min(chunk, n - first);
    const int ns = (cnt + T - 1) / T;

    float X[P], Y[P], Z[P];
    Dist<P, T, false> D;
    load_points<P, T, false>(xyz + 3 * (int64_t)first, cnt, ns, t, X, Y, Z, D);
    float px = xyz[3 * (int64_t)start + 0], py = xyz[3 * (int64_t)start + 1],
          pz = xyz[3 * (int64_t)start + 2];
    // Picks are buffered one per lane (pick i in lane i mod 64); wave 0 of
    // workgroup 0 writes them 64 at a time.
    uint32_t picks = (uint32_t)start;

    for (int i = 1; i < c; ++i) {
        const Pick mine = update_and_pick<P, T, false>(ns, w, lane, X, Y, Z, D, px, py, pz);
        const Pick p = combine_waves<W>(mine, lds, i & 1, w, lane);
        if (t == 0) {
            Candidate* slot = &gs->cand[i & 1][g];
            slot->d = p.d;
            slot->idx = (uint32_t)first + p.idx;
            slot->x = p.x; slot->y = p.y; slot->z = p.z;
            __hip_atomic_fetch_add(&gs->arrive, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (unsigned)G * (unsigned)i;
            unsigned ok = 1, spins = 0;
            while (__hip_atomic_load(&gs->arrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins >= spin_limit ||
                    ((spins & 255u) == 0 &&
                     __hip_atomic_load(&gs->failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                    ok = 0;
                    break;
                }
            }
            if (!ok) __hip_atomic_store(&gs->failed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            go = ok;
        }
        __syncthreads();
        if (!go) {
            if (g == 0) {
                const int done = i & ~63;   // picks before `done` are written
                if (w == 0 && lane < (i & 63)) out[done + lane] = (int32_t)picks;
                for (int j = i + t; j < c; j += T) out[j] = -1;
            }
            return;
        }
        // Acquire in every wave before reading the other workgroups' slots.
        (void)__hip_atomic_load(&gs->arrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t ld = 0, li = 0xFFFFFFFFu;
        float lx = 0.f, ly = 0.f, lz = 0.f;
        if (lane < G) {
            const Candidate* e = &gs->cand[i & 1][lane];
            ld = e->d; li = e->idx; lx = e->x; ly = e->y; lz = e->z;
        }
        const uint32_t best = wave_max(ld);
        const uint64_t tie = __ballot(lane < G && ld == best);
        int win = (int)__builtin_ctzll(tie);
        if (tie & (tie - 1)) {
            const uint32_t key = ((tie >> lane) & 1) ? li : 0xFFFFFFFFu;
            const uint32_t lowest = wave_min(key);
            win = (int)__builtin_ctzll(__ballot(key == lowest));
        }
        const int cur = (int)readlane(li, win);
        px = readlane(lx, win); py = readlane(ly, win); pz = readlane(lz, win);
        const int slot = i & 63;
        picks = lane == slot ? (uint32_t)cur : picks;
        if (slot == 63 && g == 0 && w == 0) out[i - 63 + lane] = (int32_t)picks;
    }
    const int tail = (c - 1) & 63;   // picks of the last, partial group
    if (g == 0 && w == 0 && tail != 63 && lane <= tail) out[(c - 1) - tail + lane] = (int32_t)picks;
}

__global__ void grid_reset(GridSync* gs) {
    if (threadIdx.x == 0) { gs->arrive = 0u; gs->failed = 0u; }
}

const void* grid_reset_kernel() { return (const void*)&grid_reset; }

void register_grid_variants(std::vector<GridVariant>& v) {
    v.push_back({16, 4, (const void*)&fps_grid_kernel<4, 16>});
    v.push_back({16, 8, (const void*)&fps_grid_kernel<8, 16>});
    v.push_back({16, 16, (const void*)&fps_grid_kernel<16, 16>});
}

}  // namespace afps
