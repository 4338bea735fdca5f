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

// A work item with every field read from the first active lane (wave-uniform).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ WorkItem uniform_item(const WorkItem& w) {
    WorkItem u;
    u.xyz_offset = uniform64(w.xyz_offset);
    u.out_offset = uniform64(w.out_offset);
    u.n = __builtin_amdgcn_readfirstlane(w.n);
    u.c = __builtin_amdgcn_readfirstlane(w.c);
    u.k = __builtin_amdgcn_readfirstlane(w.k);
    u.start = __builtin_amdgcn_readfirstlane(w.start);
    u.base = __builtin_amdgcn_readfirstlane(w.base);
    u.flags = __builtin_amdgcn_readfirstlane(w.flags);
    return u;
}

// A pointer rebuilt from its bits, known to address global memory (so that
// its accesses compile to global, not flat, instructions).
template <class T>
__device__ __forceinline__ T* global_ptr(int64_t bits) {
    return (T*)(__attribute__((address_space(1))) T*)bits;
}

// Pages a work item's sector occupies (its coordinates in LDS or not).
__device__ __forceinline__ int item_pages(const WorkItem& wi) {
    return npdu_pool_pages(wi.n, npdu_item_xyz_in_lds(wi.n, wi.flags));
}

// Sample one sector with the NPDU variant its size and coordinate placement
// call for; `lds` is the first of its pages; LR points per lane in flight
// while the sector loads.
template <int LR>
__device__ __forceinline__ void run_item(const float* __restrict__ xyz_all, int32_t* __restrict__ out_all,
                                         const WorkItem& wi, uint32_t* lds, uint64_t* t_loaded) {
    const float* xyz = xyz_all + 3 * wi.xyz_offset;
    int32_t* out = out_all + wi.out_offset;
    const int f = wi.flags & ~kItemXyzInL2;
    const bool in_lds = npdu_item_xyz_in_lds(wi.n, wi.flags);
    switch (npdu_r_for(wi.n)) {
        case 1:
            if (in_lds) sample_sector_npdu<1, true, LR>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            else sample_sector_npdu<1, false, LR>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            break;
        case 2:
            if (in_lds) sample_sector_npdu<2, true, LR>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            else sample_sector_npdu<2, false, LR>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            break;
        case 4: sample_sector_npdu<4, false, LR>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded); break;
        default: sample_sector_npdu<8, false, LR>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded); break;
    }
}

}  // namespace

// Rounds past a wave's lowest round with queued sectors that it may take
// sectors from when none of that round fits its pool.
constexpr int kRoundLookahead = 2;

template <int W>
__global__ __launch_bounds__(64 * W) void pooled_npdu_kernel(const PoolArgs a) {
    static_assert(W <= kMaxPoolWaves, "seed table holds kMaxPoolWaves waves per workgroup");
    extern __shared__ __attribute__((aligned(16))) uint32_t pool[];
    __shared__ uint64_t used[3];
    __shared__ uint32_t lock;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nq = a.nq;
    const int nrounds = a.nrounds;
    const unsigned spin_limit = a.spin_limit;
    const WorkItem* __restrict__ items = a.items;
    const PoolQueue* __restrict__ queues = a.queues;
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

    // This lane's two queues (lane, lane + 64): page counts, items per round
    // (round 0 without the seeded ones) and their first items.
    const int q0 = lane, q1 = lane + 64;
    PoolQueue Q0{0, 0, 0x7FFFFFFF, 0}, Q1{0, 0, 0x7FFFFFFF, 0};
    if (q0 < nq) Q0 = queues[q0];
    if (q1 < nq) Q1 = queues[q1];

    // The sector in hand: the wave's seed first (round 0, pages marked
    // before the barrier), then whatever the queues hand out.
    int item = -1, page = 0, pages = 0, round = 0, sleeps = 0;
    bool first_seed = false;
    if (seeded) {
        const PoolSeed sd = a.seeds[blockIdx.x * W + wv];
        if (sd.item >= 0) {
            item = sd.item;
            page = sd.page;
            pages = item_pages(items[item]);
            sleeps = sd.sleeps;
            first_seed = true;
        }
    }
    int low = 0;   // lowest round that may still have queued sectors
    unsigned spins = 0;
    bool failed = false;
    for (;;) {
        if (item < 0) {
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

            // ---- the first queue (highest priority) with sectors left that
            // fits, in the lowest round with sectors left, else up to
            // kRoundLookahead rounds further
            int q = -1, qr = 0;
            for (int r = low; r < nrounds && r < low + kRoundLookahead; r = __builtin_amdgcn_readfirstlane(r + 1)) {
                unsigned* ctr = a.qtaken + (size_t)r * kRoundCounters;
                const int avail0 = r == 0 ? Q0.count - Q0.seeded : Q0.count;
                const int avail1 = r == 0 ? Q1.count - Q1.seeded : Q1.count;
                const unsigned t0 = q0 < nq ? __hip_atomic_load(&ctr[q0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
                const unsigned t1 = q1 < nq ? __hip_atomic_load(&ctr[q1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
                const bool left0 = t0 < (unsigned)avail0, left1 = t1 < (unsigned)avail1;
                if ((ballot(left0) | ballot(left1)) == 0ull) {   // round r is drained for good
                    if (r == low) low = r + 1;
                    continue;
                }
                const uint64_t fit0 = ballot(left0 && Q0.pages <= longest), fit1 = ballot(left1 && Q1.pages <= longest);
                if (fit0 | fit1) {
                    q = fit0 ? (int)__builtin_ctzll(fit0) : 64 + (int)__builtin_ctzll(fit1);
                    qr = r;
                    break;
                }
            }
            if (low >= nrounds) {   // every round is drained
                if (lane == 0) __hip_atomic_store(&lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                break;
            }
            if (q >= 0) {
                unsigned idx = 0;
                if (lane == 0) idx = atomicAdd(&a.qtaken[(size_t)qr * kRoundCounters + q], 1u);
                idx = (unsigned)__builtin_amdgcn_readfirstlane((int)idx);
                const PoolQueue Q = queues[q];
                const int skip = qr == 0 ? Q.seeded : 0;
                if (idx < (unsigned)(Q.count - skip)) {
                    item = Q.first + skip + (int)idx;
                    pages = Q.pages;
                    round = qr;
                }
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
            const uint64_t b0 = ballot(r0 >= pages), b1 = ballot(r1 >= pages), b2 = ballot(r2 >= pages);
            page = b0 ? (int)__builtin_ctzll(b0) : (b1 ? 64 + (int)__builtin_ctzll(b1) : 128 + (int)__builtin_ctzll(b2));
            const uint64_t m0 = page_bits(0, page, pages), m1 = page_bits(1, page, pages), m2 = page_bits(2, page, pages);
            if (lane == 0) {
                if (m0) __hip_atomic_fetch_or(&used[0], m0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (m1) __hip_atomic_fetch_or(&used[1], m1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (m2) __hip_atomic_fetch_or(&used[2], m2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_store(&lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // the previous owner's accesses are done
            spins = 0;                                                // the limit bounds each wait
        }

        // ---- sample the sector in hand (the one call site of the samplers)
        for (int z = 0; z < sleeps; ++z) __builtin_amdgcn_s_sleep(127);   // kSeedSleepCycles each
        // Wave 0's seed is its workgroup's longest sector (the first round of
        // seeds takes the longest sectors): with a seed priority, its
        // instructions go first when a SIMD has another wave ready too.
        const bool raise = first_seed && wv == 0 && a.seed_priority > 0;
        if (raise) {
            switch (a.seed_priority) {
                case 1: __builtin_amdgcn_s_setprio(1); break;
                case 2: __builtin_amdgcn_s_setprio(2); break;
                default: __builtin_amdgcn_s_setprio(3); break;
            }
        }
        // Everything the sampler is given is wave-uniform: stated, so that the
        // compiler keeps the loop's index arithmetic scalar (through the loop
        // around the allocation it cannot prove it).
        item = __builtin_amdgcn_readfirstlane(item);
        page = __builtin_amdgcn_readfirstlane(page);
        round = __builtin_amdgcn_readfirstlane(round);
        const WorkItem wi = uniform_item(items[item]);
        const float* xyz_r = global_ptr<const float>(
            uniform64(reinterpret_cast<int64_t>(a.rounds ? a.rounds[round].xyz_all : a.xyz_all)));
        int32_t* out_r = global_ptr<int32_t>(
            uniform64(reinterpret_cast<int64_t>(a.rounds ? a.rounds[round].out_all : a.out_all)));
        const uint64_t take_rt = __builtin_amdgcn_s_memrealtime();
        const uint64_t take = __builtin_amdgcn_s_memtime();
        uint64_t loaded = take;
        run_item<(W > 8 ? 16 : kLoadRound)>(xyz_r, out_r, wi, pool + page * (kPoolPageBytes / 4), &loaded);
        if (a.stamps) {
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
        if (raise) __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");   // this sector's accesses are done
        if (lane == 0)
            for (int wd = 0; wd < 3; ++wd) {
                const uint64_t m = page_bits(wd, page, pages);
                if (m) __hip_atomic_fetch_and(&used[wd], ~m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        item = -1;
        sleeps = 0;
        first_seed = false;
    }
    if (!failed) return;
    // Gave up waiting: report it, take every sector still queued in any round
    // and mark it failed.
    if (lane == 0) {
        __hip_atomic_fetch_or(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_or(a.dev_status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int r = 0; r < nrounds; ++r) {
        int32_t* out_r = a.rounds ? a.rounds[r].out_all : a.out_all;
        for (int q = 0; q < nq; ++q) {
            const PoolQueue Q = queues[q];
            const int skip = r == 0 ? Q.seeded : 0;
            for (;;) {
                unsigned idx = 0;
                if (lane == 0) idx = atomicAdd(&a.qtaken[(size_t)r * kRoundCounters + q], 1u);
                idx = (unsigned)__builtin_amdgcn_readfirstlane((int)idx);
                if (idx >= (unsigned)(Q.count - skip)) break;
                fail_item(items[Q.first + skip + (int)idx], out_r, lane);
            }
        }
    }
}

// Four or eight waves per workgroup load sectors 32 points per lane at a time
// (at most two waves per SIMD fit their registers); twelve or sixteen (three
// or four per SIMD) load 16 at a time, which keeps them within the registers.
void register_pool_variants(std::vector<PoolEntry>& v) {
    v.push_back({4, (const void*)&pooled_npdu_kernel<4>});
    v.push_back({8, (const void*)&pooled_npdu_kernel<8>});
    v.push_back({12, (const void*)&pooled_npdu_kernel<12>});
    v.push_back({16, (const void*)&pooled_npdu_kernel<16>});
}

}  // namespace afps
