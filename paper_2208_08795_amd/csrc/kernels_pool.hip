// Pooled NPDU kernel (Sec. III-C sectors of a whole batch in one launch).
//
// One workgroup per CU takes the CU's whole LDS as a pool of 1 KB pages (64
// sector records of 16 bytes), or two take half of it each (the plan's
// choice; pool_pages is the workgroup's share).  Its W waves work
// independently: a wave
// allocates exactly the pages of one sector (first fit, contiguous), samples
// it with the one-wave NPDU sampler, frees the pages and takes the next
// sector.  Sectors wait in priority queues, one per page count, ordered by
// their longest sector first; a wave takes the first queue whose sectors fit
// in the largest free run of its pool, so the long sectors (the critical path
// of the batch) start first and the short ones fill the pages left over.
//
// Each wave's first sector (its seed) and that sector's pages are chosen when
// the plan is built, by the same policy played out for the moment all waves
// start; the seeds' pages are marked used before the workgroup's start
// barrier, so a launch begins without every wave contending for the same
// queue counter.  A seed with slack before the plan's longest sector would
// end waits a few sleep periods first, so that the longest sectors load their
// points with less competition for memory bandwidth.
//
// Allocation is serialised per workgroup by an LDS lock; frees are atomic
// ANDs on the used-mask and need no lock.  Every wait (for the lock, or for
// pages another wave of the workgroup still holds) polls at most spin_limit
// times; a wave that gives up sets the plan's status word and the device's
// failure word, marks every sector still queued as failed (outputs -1) so
// that no output is left unwritten, and exits.
//
// With a stamp buffer (afps_plan_launch_stamped), lane 0 of each wave records
// per sector the shader clock when it took the sector, when the sector was in
// LDS and when its last pick was written (plus the constant-rate clock, for
// the shader clock's rate): cycles per iteration measured on the device.
#include "sampler.hpp"
#include "variants.hpp"

namespace afps {

namespace {

// Number of consecutive 1 bits of x from bit 0.
__device__ __forceinline__ int ones_from_bottom(uint64_t x) {
    return ~x == 0ull ? 64 : (int)__builtin_ctzll(~x);
}
// Free pages from page 64*w + lane onwards, for the three words of the
// used-mask u (bit set = page in use); pages past the pool are marked used.
__device__ __forceinline__ int free_run(int w, int lane, uint64_t u0, uint64_t u1, uint64_t u2) {
    const uint64_t uw = w == 0 ? u0 : (w == 1 ? u1 : u2);
    int run = ones_from_bottom(~uw >> lane);
    if (run < 64 - lane) return run;        // a used page inside this word ends the run
    run = 64 - lane;
    if (w < 1) {
        const int r1 = ones_from_bottom(~u1);
        run += r1;
        if (r1 < 64) return run;
    }
    if (w < 2) run += ones_from_bottom(~u2);
    return run;
}
// Bits of pages [s, s + p) inside word w of the used-mask.
__device__ __forceinline__ uint64_t page_bits(int w, int s, int p) {
    const int lo = max(s, 64 * w), hi = min(s + p, 64 * w + 64);
    if (lo >= hi) return 0ull;
    const int len = hi - lo;
    const uint64_t ones = len == 64 ? ~0ull : ((1ull << len) - 1ull);
    return ones << (lo - 64 * w);
}

__device__ __forceinline__ void fail_item(const WorkItem& wi, int32_t* out_all, int lane) {
    int32_t* out = out_all + wi.out_offset;
    for (int j = lane; j < wi.c; j += 64) out[j] = -1;
}

// Pages a work item's sector occupies (its coordinates in LDS or not).
__device__ __forceinline__ int item_pages(const WorkItem& wi) {
    return npdu_pool_pages(wi.n, npdu_item_xyz_in_lds(wi.n, wi.flags));
}

// Sample one sector with the NPDU variant its size and coordinate placement
// call for; `lds` is the first of its pages.
__device__ __forceinline__ void run_item(const float* __restrict__ xyz_all, int32_t* __restrict__ out_all,
                                         const WorkItem& wi, uint32_t* lds, uint64_t* t_loaded) {
    const float* xyz = xyz_all + 3 * wi.xyz_offset;
    int32_t* out = out_all + wi.out_offset;
    const int f = wi.flags & ~kItemXyzInL2;
    const bool in_lds = npdu_item_xyz_in_lds(wi.n, wi.flags);
    switch (npdu_r_for(wi.n)) {
        case 1:
            if (in_lds) sample_sector_npdu<1, true>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            else sample_sector_npdu<1, false>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            break;
        case 2:
            if (in_lds) sample_sector_npdu<2, true>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            else sample_sector_npdu<2, false>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            break;
        case 4: sample_sector_npdu<4, false>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded); break;
        default: sample_sector_npdu<8, false>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded); break;
    }
}

// run_item, timed into a.stamps[item] when the launch records stamps.
__device__ __forceinline__ void run_stamped(const PoolArgs& a, int item, const WorkItem& wi, uint32_t* lds,
                                            int lane) {
    if (!a.stamps) {
        run_item(a.xyz_all, a.out_all, wi, lds, nullptr);
        return;
    }
    const uint64_t take_rt = __builtin_amdgcn_s_memrealtime();
    const uint64_t take = __builtin_amdgcn_s_memtime();
    uint64_t loaded = take;
    run_item(a.xyz_all, a.out_all, wi, lds, &loaded);
    const uint64_t end = __builtin_amdgcn_s_memtime();
    const uint64_t end_rt = __builtin_amdgcn_s_memrealtime();
    if (lane == 0) {
        SectorStamp st;
        st.take = take;
        st.loaded = loaded;
        st.end = end;
        st.take_rt = take_rt;
        st.end_rt = end_rt;
        st.item = item;
        st.n = wi.n;
        st.c = wi.c;
        st.k = wi.k;
        // HW_ID (register 4) and XCC_ID (register 20), whole 32-bit registers
        st.hw_id = (uint32_t)__builtin_amdgcn_s_getreg((31 << 11) | 4);
        st.xcc_id = (uint32_t)__builtin_amdgcn_s_getreg((31 << 11) | 20);
        a.stamps[item] = st;
    }
}

}  // namespace

template <int W>
__global__ __launch_bounds__(64 * W) void pooled_npdu_kernel(const PoolArgs a) {
    static_assert(W <= kMaxPoolWaves, "seed table holds kMaxPoolWaves waves per workgroup");
    extern __shared__ __attribute__((aligned(16))) uint32_t pool[];
    __shared__ uint64_t used[3];
    __shared__ uint32_t lock;
    const int lane = threadIdx.x & 63;
    const int nq = a.nq;
    const unsigned spin_limit = a.spin_limit;
    const WorkItem* __restrict__ items = a.items;
    const PoolQueue* __restrict__ queues = a.queues;
    unsigned* qtaken = a.qtaken;
    const bool seeded = (int)blockIdx.x < a.seed_groups;
    if (threadIdx.x < 3) {
        const int wd = (int)threadIdx.x, lo = 64 * wd;
        uint64_t u = a.pool_pages <= lo ? ~0ull : (a.pool_pages >= lo + 64 ? 0ull : (~0ull << (a.pool_pages - lo)));
        if (seeded)
            for (int w = 0; w < W; ++w) {
                const PoolSeed sd = a.seeds[blockIdx.x * W + w];
                if (sd.item >= 0) u |= page_bits(wd, sd.page, item_pages(items[sd.item]));
            }
        used[wd] = u;
    }
    if (threadIdx.x == 0) lock = 0u;
    __syncthreads();   // the only workgroup barrier: from here on waves are independent

    // ---- the wave's seed: pages already marked, no lock
    if (seeded) {
        const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const PoolSeed sd = a.seeds[blockIdx.x * W + wv];
        if (sd.item >= 0) {
            for (int z = 0; z < sd.sleeps; ++z) __builtin_amdgcn_s_sleep(127);   // kSeedSleepCycles each
            const WorkItem wi = items[sd.item];
            const int p = item_pages(wi);
            // Wave 0's seed is its workgroup's longest sector (the first round
            // of seeds takes the longest sectors): with a seed priority, its
            // instructions go first when a SIMD has another wave ready too.
            const bool raise = wv == 0 && a.seed_priority > 0;
            if (raise) {
                switch (a.seed_priority) {
                    case 1: __builtin_amdgcn_s_setprio(1); break;
                    case 2: __builtin_amdgcn_s_setprio(2); break;
                    default: __builtin_amdgcn_s_setprio(3); break;
                }
            }
            run_stamped(a, sd.item, wi, pool + sd.page * (kPoolPageBytes / 4), lane);
            if (raise) __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");   // this sector's accesses are done
            if (lane == 0)
                for (int wd = 0; wd < 3; ++wd) {
                    const uint64_t m = page_bits(wd, sd.page, p);
                    if (m) __hip_atomic_fetch_and(&used[wd], ~m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
        }
    }

    // This lane's two queues (lane, lane + 64): their page counts and sizes.
    const int q0 = lane, q1 = lane + 64;
    const int pages0 = q0 < nq ? queues[q0].pages : 0x7FFFFFFF, count0 = q0 < nq ? queues[q0].count : 0;
    const int pages1 = q1 < nq ? queues[q1].pages : 0x7FFFFFFF, count1 = q1 < nq ? queues[q1].count : 0;

    unsigned spins = 0;
    bool failed = false;
    for (;;) {
        // ---- take the allocation lock (lane 0 polls; the wave follows)
        int got = 0;
        if (lane == 0) {
            for (;;) {
                uint32_t expected = 0u;
                if (__hip_atomic_compare_exchange_strong(&lock, &expected, 1u, __ATOMIC_ACQUIRE,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                    got = 1;
                    break;
                }
                if (++spins >= spin_limit) break;
                __builtin_amdgcn_s_sleep(1);
            }
        }
        spins = (unsigned)__builtin_amdgcn_readfirstlane((int)spins);
        if (!__builtin_amdgcn_readfirstlane(got)) {
            failed = true;
            break;
        }

        // ---- largest free run of pages, per start page (three per lane)
        const uint64_t u0 = __hip_atomic_load(&used[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint64_t u1 = __hip_atomic_load(&used[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint64_t u2 = __hip_atomic_load(&used[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int r0 = free_run(0, lane, u0, u1, u2);
        const int r1 = free_run(1, lane, u0, u1, u2);
        const int r2 = free_run(2, lane, u0, u1, u2);
        const int longest = (int)wave_max((uint32_t)max(r0, max(r1, r2)));

        // ---- first queue (highest priority) with sectors left that fits
        const unsigned t0 = q0 < nq ? __hip_atomic_load(&qtaken[q0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        const unsigned t1 = q1 < nq ? __hip_atomic_load(&qtaken[q1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        const bool left0 = t0 < (unsigned)count0, left1 = t1 < (unsigned)count1;
        if ((ballot(left0) | ballot(left1)) == 0ull) {           // every queue is drained
            if (lane == 0) __hip_atomic_store(&lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            break;
        }
        const uint64_t fit0 = ballot(left0 && pages0 <= longest), fit1 = ballot(left1 && pages1 <= longest);
        int q = -1;
        if (fit0) q = (int)__builtin_ctzll(fit0);
        else if (fit1) q = 64 + (int)__builtin_ctzll(fit1);
        int item = -1;
        if (q >= 0) {
            unsigned idx = 0;
            if (lane == 0) idx = atomicAdd(&qtaken[q], 1u);
            idx = (unsigned)__builtin_amdgcn_readfirstlane((int)idx);
            const PoolQueue Q = queues[q];
            if (idx < (unsigned)Q.count) item = Q.first + (int)idx;
        }
        if (item < 0) {
            // Nothing fits now (pages held by other waves of this workgroup),
            // or the queue emptied meanwhile: release and poll again.
            if (lane == 0) __hip_atomic_store(&lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (q < 0) {
                if (++spins >= spin_limit) {
                    failed = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            continue;
        }

        // ---- first fit of the item's pages, marked used, lock released
        const int p = q < 64 ? __builtin_amdgcn_readlane(pages0, q) : __builtin_amdgcn_readlane(pages1, q - 64);
        const uint64_t b0 = ballot(r0 >= p), b1 = ballot(r1 >= p), b2 = ballot(r2 >= p);
        const int s = b0 ? (int)__builtin_ctzll(b0) : (b1 ? 64 + (int)__builtin_ctzll(b1) : 128 + (int)__builtin_ctzll(b2));
        const uint64_t m0 = page_bits(0, s, p), m1 = page_bits(1, s, p), m2 = page_bits(2, s, p);
        if (lane == 0) {
            if (m0) __hip_atomic_fetch_or(&used[0], m0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (m1) __hip_atomic_fetch_or(&used[1], m1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (m2) __hip_atomic_fetch_or(&used[2], m2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(&lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // the previous owner's accesses are done
        spins = 0;                                                // the limit bounds each wait

        const WorkItem wi = items[item];
        run_stamped(a, item, wi, pool + s * (kPoolPageBytes / 4), lane);

        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");   // this sector's accesses are done
        if (lane == 0) {
            if (m0) __hip_atomic_fetch_and(&used[0], ~m0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (m1) __hip_atomic_fetch_and(&used[1], ~m1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (m2) __hip_atomic_fetch_and(&used[2], ~m2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    if (!failed) return;
    // Gave up waiting: report it, take every sector still queued and mark it failed.
    if (lane == 0) {
        __hip_atomic_fetch_or(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_or(a.dev_status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int q = 0; q < nq; ++q) {
        const PoolQueue Q = queues[q];
        for (;;) {
            unsigned idx = 0;
            if (lane == 0) idx = atomicAdd(&qtaken[q], 1u);
            idx = (unsigned)__builtin_amdgcn_readfirstlane((int)idx);
            if (idx >= (unsigned)Q.count) break;
            fail_item(items[Q.first + (int)idx], a.out_all, lane);
        }
    }
}

void register_pool_variants(std::vector<PoolEntry>& v) {
    v.push_back({4, (const void*)&pooled_npdu_kernel<4>});
    v.push_back({8, (const void*)&pooled_npdu_kernel<8>});
}

}  // namespace afps
