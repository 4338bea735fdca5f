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

// Sample one sector with the NPDU variant its size and coordinate placement
// call for; `lds` is the first of its pages; LR points per lane in flight
// while the sector loads.  Coordinates kept out of LDS live in registers
// (REGS: kernels of at most two waves per SIMD, sectors of at most 4096
// points, k <= 64), else they are read from L2 (by the narrow loop for such
// sectors without REGS).
// The narrow loop with coordinates from L2 (k <= 64): windows of at most 64
// points (k <= 63) update their own 64 lanes, the widest its two blocks.
__device__ __forceinline__ void run_narrow_l2(const float* __restrict__ xyz, int32_t* __restrict__ out,
                                              const WorkItem& wi, int f, uint32_t* lds, uint64_t* t_loaded) {
    const bool first_full = (f & kNpduFirstFull) != 0;
    if (wi.k <= 63) {
        if (f & kNpduShiftEdges)
            sample_sector_npdu_narrow_l2<true, true>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, first_full,
                                                     t_loaded);
        else
            sample_sector_npdu_narrow_l2<false, true>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, first_full,
                                                      t_loaded);
    } else {
        if (f & kNpduShiftEdges)
            sample_sector_npdu_narrow_l2<true, false>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, first_full,
                                                      t_loaded);
        else
            sample_sector_npdu_narrow_l2<false, false>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, first_full,
                                                       t_loaded);
    }
}

template <int LR, bool REGS, bool LITE>
__device__ __forceinline__ void run_item(const float* __restrict__ xyz_all, int32_t* __restrict__ out_all,
                                         const WorkItem& wi, uint32_t* lds, uint64_t* t_loaded) {
    const float* xyz = xyz_all + 3 * wi.xyz_offset;
    int32_t* out = out_all + wi.out_offset;
    const int f = wi.flags & ~kItemXyzNotInLds;
    if constexpr (LITE) {   // the plan holds npdu_item_lite sectors only
        run_narrow_l2(xyz, out, wi, f, lds, t_loaded);
        return;
    }
    const bool in_lds = npdu_item_xyz_in_lds(wi.n, wi.flags);
    switch (npdu_r_for(wi.n)) {
        case 1:
            if (in_lds) {
                sample_sector_npdu<1, true, LR>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            } else if (REGS && wi.k <= 64) {
                if (f & kNpduShiftEdges)
                    sample_sector_npdu_regs<true>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds,
                                                  (f & kNpduFirstFull) != 0, t_loaded);
                else
                    sample_sector_npdu_regs<false>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds,
                                                   (f & kNpduFirstFull) != 0, t_loaded);
            } else if (wi.k <= 64) {
                run_narrow_l2(xyz, out, wi, f, lds, t_loaded);
            } else {
                sample_sector_npdu<1, false, LR>(xyz, wi.n, wi.c, wi.k, wi.start, wi.base, out, lds, f, t_loaded);
            }
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

// The pooled NPDU kernel: one persistent workgroup of W waves per CU (or two
// of four, twelve or sixteen), every wave one sector at a time.  The light
// variant (LITE) holds only the narrow loop with coordinates from L2, so that
// two workgroups of twelve or sixteen waves fit a CU's registers.  The plan
// gave each workgroup its own sectors (the same for every round) in queues
// by page count; a wave claims the next one under the workgroup's lock,
// entirely in LDS (the claim counters of kRoundRing rounds at once and the
// page mask), so no device-wide atomic is touched per sector: on MI355X
// those cross the XCDs.
template <int W, bool LITE>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(LITE ? W / 2 : 1)))
void pooled_npdu_kernel(const PoolArgs a) {
    static_assert(W <= kMaxPoolWaves, "seed table holds kMaxPoolWaves waves per workgroup");
    static_assert(kMaxLocalQueues == 64, "one queue per lane");
    extern __shared__ __attribute__((aligned(16))) uint32_t pool[];
    __shared__ uint64_t used[3];                              // page mask, bit set = in use
    __shared__ uint32_t lock;
    __shared__ uint32_t taken[kRoundRing][kMaxLocalQueues];   // claims per queue of round r in slot r % kRoundRing
    __shared__ int32_t low;                                   // rounds below have every sector claimed
    __shared__ uint32_t exited;                               // waves that left the work loop
    __shared__ uint32_t gave_up;                              // a wave of this workgroup gave up a bounded wait
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nrounds = a.nrounds;
    const unsigned spin_limit = a.spin_limit;
    const WorkItem* __restrict__ items = a.items;
    const PoolGroup grp = a.groups[blockIdx.x];
    // This lane's queue: first item, items per round (round 0 without the
    // seeded ones), pages; lanes past the workgroup's queues hold none.
    PoolQueue Q{0, 0, 0x7FFFFFFF, 0};
    if (lane < grp.queues) Q = a.queues[grp.queue_first + lane];
    const PoolSeed* seeds = a.seeds + (size_t)blockIdx.x * W;
    if (threadIdx.x < 3) {
        const int wd = (int)threadIdx.x, lo = 64 * wd;
        uint64_t u = a.pool_pages <= lo ? ~0ull : (a.pool_pages >= lo + 64 ? 0ull : (~0ull << (a.pool_pages - lo)));
        for (int w = 0; w < W; ++w) {
            const PoolSeed sd = seeds[w];
            if (sd.item >= 0) u |= page_bits(wd, sd.page, sd.pages);
        }
        used[wd] = u;
    }
    for (int i = threadIdx.x; i < kRoundRing * kMaxLocalQueues; i += 64 * W) (&taken[0][0])[i] = 0u;
    if (threadIdx.x == 0) {
        lock = 0u;
        low = 0;
        exited = 0u;
        gave_up = 0u;
    }
    __syncthreads();   // the only workgroup barrier: from here on waves are independent

    // The sector in hand: the wave's seed first (round 0, pages marked
    // before the barrier), then whatever the workgroup's queues hand out.
    int item = -1, page = 0, pages = 0, sleeps = 0;
    bool first_seed = false;
    WorkItem wi{};
    PoolRound rp{a.xyz_all, a.out_all};
    {
        const PoolSeed sd = seeds[wv];
        if (sd.item >= 0) {
            item = sd.item;
            page = sd.page;
            pages = sd.pages;
            sleeps = sd.sleeps;
            first_seed = true;
            wi = items[item];
            if (a.rounds) rp = a.rounds[0];
        }
    }
    unsigned spins = 0;
    bool failed = false;
    for (;;) {
        if (item < 0) {
            if (__hip_atomic_load(&gave_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
            // ---- the workgroup lock (lane 0 polls; the wave follows)
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
            // ---- under the lock: the longest free run of pages, then the
            // first queue (highest priority) with sectors left that fits it, in
            // the lowest round with sectors left, else up to kRoundRing - 1
            // rounds further.  Rounds at the front with every sector claimed
            // pass their counter slot on to round r + kRoundRing.
            const uint64_t u0 = __hip_atomic_load(&used[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const uint64_t u1 = __hip_atomic_load(&used[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const uint64_t u2 = __hip_atomic_load(&used[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int r0 = free_run(0, lane, u0, u1, u2);
            const int r1 = free_run(1, lane, u0, u1, u2);
            const int r2 = free_run(2, lane, u0, u1, u2);
            const int longest = (int)wave_max((uint32_t)max(r0, max(r1, r2)));
            const int lw = __builtin_amdgcn_readfirstlane(__hip_atomic_load(&low, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            int lw_new = lw;
            int q = -1, qr = 0;
            unsigned idx = 0u;
            bool front = true;
#pragma unroll
            for (int i = 0; i < kRoundRing; ++i) {
                const int r = lw + i;
                if (q < 0 && r < nrounds) {
                    uint32_t* const slot = taken[r & (kRoundRing - 1)];
                    const uint32_t t = __hip_atomic_load(&slot[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    const int avail = r == 0 ? Q.count - Q.seeded : Q.count;
                    const uint64_t left = ballot(t < (uint32_t)avail);
                    if (left == 0ull) {
                        if (front) {   // round r is claimed for good: the slot is round r + kRoundRing's
                            __hip_atomic_store(&slot[lane], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            lw_new = r + 1;
                        }
                    } else {
                        front = false;
                        const uint64_t fit = left & ballot(Q.pages <= longest);
                        if (fit) {
                            q = (int)__builtin_ctzll(fit);
                            qr = r;
                            idx = (uint32_t)__builtin_amdgcn_readlane((int)t, q);
                            if (lane == q)
                                __hip_atomic_store(&slot[lane], t + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                }
            }
            if (lw_new != lw && lane == 0) __hip_atomic_store(&low, lw_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (q < 0) {
                if (lane == 0) __hip_atomic_store(&lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (lw_new >= nrounds) break;   // every sector of every round is claimed
                // Nothing left fits the free pages now (they are held by
                // other waves of this workgroup): poll again.
                if (++spins >= spin_limit) {
                    failed = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                continue;
            }
            // ---- the first fit of the queue's pages, marked used; lock released
            q = __builtin_amdgcn_readfirstlane(q);
            qr = __builtin_amdgcn_readfirstlane(qr);
            const int q_pages = __builtin_amdgcn_readlane(Q.pages, q);
            const uint64_t b0 = ballot(r0 >= q_pages), b1 = ballot(r1 >= q_pages), b2 = ballot(r2 >= q_pages);
            page = b0 ? (int)__builtin_ctzll(b0) : (b1 ? 64 + (int)__builtin_ctzll(b1) : 128 + (int)__builtin_ctzll(b2));
            const uint64_t m0 = page_bits(0, page, q_pages), m1 = page_bits(1, page, q_pages),
                           m2 = page_bits(2, page, q_pages);
            if (lane == 0) {
                if (m0) __hip_atomic_fetch_or(&used[0], m0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (m1) __hip_atomic_fetch_or(&used[1], m1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (m2) __hip_atomic_fetch_or(&used[2], m2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_store(&lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // the pages' previous owner is done with them
            spins = 0;                                                // the limit bounds each wait
            const int skip = qr == 0 ? __builtin_amdgcn_readlane(Q.seeded, q) : 0;
            item = __builtin_amdgcn_readlane(Q.first, q) + skip + (int)idx;
            pages = q_pages;
            wi = items[item];
            if (a.rounds) rp = a.rounds[qr];
        }

        // ---- sample the sector in hand (the one call site of the samplers)
        for (int z = 0; z < sleeps; ++z) __builtin_amdgcn_s_sleep(127);   // kSeedSleepCycles each
        // Wave 0's seed is its workgroup's longest sector (the seeds take
        // the longest sectors first): with a seed priority, its instructions
        // go first when a SIMD has another wave ready too.
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
        const WorkItem wu = uniform_item(wi);
        const float* xyz_r = global_ptr<const float>(uniform64(reinterpret_cast<int64_t>(rp.xyz_all)));
        int32_t* out_r = global_ptr<int32_t>(uniform64(reinterpret_cast<int64_t>(rp.out_all)));
        const uint64_t take_rt = __builtin_amdgcn_s_memrealtime();
        const uint64_t take = __builtin_amdgcn_s_memtime();
        uint64_t loaded = take;
        run_item<(W > 8 ? 16 : kLoadRound), (W <= 8), LITE>(xyz_r, out_r, wu, pool + page * (kPoolPageBytes / 4),
                                                            &loaded);
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
                st.n = wu.n;
                st.c = wu.c;
                st.k = wu.k;
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
        // not carried past the sampler in registers: set again by the next claim
        wi = WorkItem{};
        rp = PoolRound{a.xyz_all, a.out_all};
    }

    // ---- leaving.  A wave that gave up reports it and stops the workgroup
    // claiming; the last wave out then marks every sector no wave claimed
    // failed (every claimed sector ran to its end).
    if (failed && lane == 0) {
        __hip_atomic_fetch_or(&gave_up, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_or(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_or(a.dev_status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned before = 0u;
    if (lane == 0) before = __hip_atomic_fetch_add(&exited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    before = (unsigned)__builtin_amdgcn_readfirstlane((int)before);
    if (before != (unsigned)(W - 1)) return;
    if (!__hip_atomic_load(&gave_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return;
    const int lw = __builtin_amdgcn_readfirstlane(__hip_atomic_load(&low, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    for (int r = lw; r < nrounds; ++r) {
        int32_t* out_r = global_ptr<int32_t>(uniform64(reinterpret_cast<int64_t>(a.rounds ? a.rounds[r].out_all : a.out_all)));
        const uint32_t t = r < lw + kRoundRing
                               ? __hip_atomic_load(&taken[r & (kRoundRing - 1)][lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                               : 0u;
        for (int q = 0; q < grp.queues; ++q) {
            const int skip = r == 0 ? __builtin_amdgcn_readlane(Q.seeded, q) : 0;
            const int first = __builtin_amdgcn_readlane(Q.first, q), count = __builtin_amdgcn_readlane(Q.count, q);
            for (int i = first + skip + __builtin_amdgcn_readlane((int)t, q); i < first + count; ++i)
                fail_item(uniform_item(items[i]), out_r, lane);
        }
    }
}

// Four or eight waves per workgroup load sectors 32 points per lane at a time
// (at most two waves per SIMD fit their registers); twelve or sixteen (three
// or four per SIMD) load 16 at a time, which keeps them within the registers.
// The light twelve- and sixteen-wave kernels run two workgroups per CU (six
// or eight waves per SIMD).
void register_pool_variants(std::vector<PoolEntry>& v) {
    v.push_back({4, false, (const void*)&pooled_npdu_kernel<4, false>});
    v.push_back({8, false, (const void*)&pooled_npdu_kernel<8, false>});
    v.push_back({12, false, (const void*)&pooled_npdu_kernel<12, false>});
    v.push_back({16, false, (const void*)&pooled_npdu_kernel<16, false>});
    v.push_back({12, true, (const void*)&pooled_npdu_kernel<12, true>});
    v.push_back({16, true, (const void*)&pooled_npdu_kernel<16, true>});
}

}  // namespace afps
