// Randomised check of the batch planner (paper_2208_08795_amd/csrc/planner.cpp)
// on the CPU, built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_planner_host.py.  For random batches (clouds of 1..32768 points,
// mixed plain FPS / AFPS / NPDU with every reading flag, random starts), every
// occupancy budget and pool policy, it asserts that the plan covers every
// sector exactly once with the Sec. III-B split, that every pooled sector
// belongs to exactly one workgroup's queues, that every work item, queue,
// seed and page range stays inside the workspace and the LDS pool, and that
// corrupted descriptors are rejected.  Exit status 0 = every check held.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "planner.hpp"

using namespace afps;

static int g_failures = 0;

#define CHECK(cond, ...)                                              \
    do {                                                              \
        if (!(cond)) {                                                \
            std::fprintf(stderr, "check failed: %s: ", #cond);       \
            std::fprintf(stderr, __VA_ARGS__);                        \
            std::fprintf(stderr, "\n");                               \
            if (++g_failures > 20) std::exit(1);                      \
        }                                                             \
    } while (0)

namespace {

// Compiled full-update variants of the library: W waves x P slots.
struct FakeVariant {
    int waves, slots, lds;
};
std::vector<FakeVariant> fake_variants() {
    std::vector<FakeVariant> v;
    for (int w : {1, 2, 4, 8, 16})
        for (int p : {1, 2, 4, 8, 12, 16, 24, 32}) v.push_back({w, p, (w == 16 && p == 32) ? 32 * 64 * 16 * 4 : 0});
    return v;
}

PlannerEnv make_env(std::mt19937_64& rng, const std::vector<FakeVariant>& vars) {
    PlannerEnv env;
    env.cu_count = std::uniform_int_distribution<int>(1, 256)(rng);
    env.cu_pool_pages = std::uniform_int_distribution<int>(0, 3)(rng) == 0
                            ? std::uniform_int_distribution<int>(20, kMaxPoolPages)(rng)
                            : 159;
    const float occ[] = {0.0f, 1.0f, 1.5f, 2.0f, 4.0f};
    env.pool.waves_per_simd = occ[std::uniform_int_distribution<int>(0, 4)(rng)];
    if (std::uniform_int_distribution<int>(0, 2)(rng) == 0) {
        const int shapes[][2] = {{4, 1}, {8, 1}, {4, 2}, {8, 2}, {12, 1}, {16, 1}, {12, 2}, {16, 2}};
        const auto& sh = shapes[std::uniform_int_distribution<int>(0, 7)(rng)];
        env.pool.waves = sh[0];
        env.pool.groups = sh[1];
    }
    env.pool.seed_sleep = std::uniform_int_distribution<int>(0, 1)(rng) != 0;
    env.pool.seed_priority = std::uniform_int_distribution<int>(0, 3)(rng);
    const int entries = std::uniform_int_distribution<int>(0, 3)(rng);
    for (int i = 0; i < entries; ++i)
        env.pool.placement.push_back({std::uniform_int_distribution<int>(64, 9000)(rng),
                                      std::uniform_int_distribution<int>(0, 200)(rng),
                                      std::uniform_int_distribution<int>(0, 1)(rng)});
    std::sort(env.pool.placement.begin(), env.pool.placement.end(), [](const NpduPlacement& a, const NpduPlacement& b) {
        return a.n_max != b.n_max ? a.n_max < b.n_max : a.k_max < b.k_max;
    });
    env.choose_full = [vars](int n, FullVariantInfo* out) {
        int best = -1;
        for (size_t i = 0; i < vars.size(); ++i) {
            const int cap = 64 * vars[i].waves * vars[i].slots;
            if (cap >= n && (best < 0 || cap < 64 * vars[best].waves * vars[best].slots)) best = (int)i;
        }
        if (best < 0) return false;
        *out = FullVariantInfo{best, vars[best].waves, vars[best].slots, vars[best].lds};
        return true;
    };
    env.blocks_per_cu = [](const FullVariantInfo& v) { return std::max(1, 32 / v.waves); };
    return env;
}

int log_uniform(std::mt19937_64& rng, int lo, int hi) {
    std::uniform_real_distribution<double> u(std::log((double)lo), std::log((double)hi + 1.0));
    return std::min(hi, std::max(lo, (int)std::exp(u(rng))));
}

std::vector<afps_cloud_desc> random_batch(std::mt19937_64& rng) {
    const int batch = std::uniform_int_distribution<int>(0, 3)(rng) == 0 ? std::uniform_int_distribution<int>(1, 4)(rng)
                                                                         : std::uniform_int_distribution<int>(1, 300)(rng);
    std::vector<afps_cloud_desc> d(batch);
    int64_t xo = 0, oo = 0;
    for (auto& c : d) {
        c.n = log_uniform(rng, 1, 32768);
        const int kind = std::uniform_int_distribution<int>(0, 3)(rng);   // fps, afps, npdu, npdu
        c.c = std::uniform_int_distribution<int>(1, c.n)(rng);
        c.m = kind == 0 ? 1 : std::uniform_int_distribution<int>(1, std::min(c.c, 64))(rng);
        c.k = kind < 2 ? -1 : (std::uniform_int_distribution<int>(0, 5)(rng) == 0 ? std::uniform_int_distribution<int>(0, 2 * c.n + 5)(rng)
                                                                               : std::uniform_int_distribution<int>(0, 130)(rng));
        c.flags = kind < 2 ? 0 : std::uniform_int_distribution<int>(0, 7)(rng);
        if ((c.flags & AFPS_NPDU_K_WITH_SELF) && c.k < 1) c.k = 1;
        c.start = std::uniform_int_distribution<int>(0, c.n - 1)(rng);
        c.xyz_offset = xo;
        c.out_offset = oo;
        xo += c.n;
        oo += c.c;
    }
    return d;
}

void check_plan(const std::vector<afps_cloud_desc>& d, const PlannerEnv& env, const PlanTables& t) {
    // every sector of every cloud exactly once, with the Sec. III-B split
    std::map<std::pair<int64_t, int64_t>, const WorkItem*> by_offsets;
    for (const auto& it : t.items) {
        auto key = std::make_pair(it.xyz_offset, it.out_offset);
        CHECK(!by_offsets.count(key), "item at %lld/%lld twice", (long long)it.xyz_offset, (long long)it.out_offset);
        by_offsets[key] = &it;
    }
    size_t sectors = 0;
    for (size_t b = 0; b < d.size(); ++b) {
        const auto& c = d[b];
        int32_t k = c.k, flags = c.flags;
        if (flags & AFPS_NPDU_K_WITH_SELF) {
            k -= 1;
            flags &= ~AFPS_NPDU_K_WITH_SELF;
        }
        for (int s = 0; s < c.m; ++s) {
            const int ns = c.n / c.m + (s < c.n % c.m), bs = s * (c.n / c.m) + std::min(s, c.n % c.m);
            const int cs = c.c / c.m + (s < c.c % c.m), os = s * (c.c / c.m) + std::min(s, c.c % c.m);
            auto f = by_offsets.find({c.xyz_offset + bs, c.out_offset + os});
            CHECK(f != by_offsets.end(), "cloud %zu sector %d missing", b, s);
            if (f == by_offsets.end()) continue;
            const WorkItem& it = *f->second;
            CHECK(it.n == ns && it.c == cs && it.base == bs, "cloud %zu sector %d split", b, s);
            CHECK(it.c >= 1 && it.c <= it.n, "cloud %zu sector %d samples %d of %d", b, s, it.c, it.n);
            CHECK(it.start == c.start % ns, "cloud %zu sector %d start", b, s);
            CHECK(it.k == (k < 0 ? -1 : std::min(k, 2 * ns)), "cloud %zu sector %d k", b, s);
            CHECK((it.flags & ~kItemXyzNotInLds) == (k < 0 ? 0 : flags), "cloud %zu sector %d flags", b, s);
            const bool out = (it.flags & kItemXyzNotInLds) != 0;
            CHECK(!out || (k >= 0 && npdu_r_for(ns) <= 2), "placement flag on a sector that cannot hold it");
            if (k >= 0 && npdu_r_for(ns) <= 2)
                CHECK(out == !npdu_xyz_in_lds(env.pool, ns, it.k), "placement of cloud %zu sector %d", b, s);
            CHECK(it.out_offset + it.c <= c.out_offset + c.c && it.xyz_offset + it.n <= c.xyz_offset + c.n,
                  "sector outside its cloud");
            ++sectors;
        }
    }
    CHECK(sectors == t.items.size(), "%zu sectors, %zu items", sectors, t.items.size());
    CHECK(t.clouds.size() == d.size(), "clouds");
    CHECK(t.ws_bytes >= kItemsOffset + t.items.size() * sizeof(WorkItem) && t.ws_bytes % 256 == 0, "workspace size");
    CHECK(t.ws_bytes == workspace_bytes_for_items((int64_t)t.items.size()), "workspace formula");
    CHECK((int)t.buckets.size() <= kMaxBuckets, "buckets");

    // buckets partition the items; the pool bucket covers the NPDU items
    std::vector<int> owner(t.items.size(), -1);
    int pool_buckets = 0;
    for (size_t b = 0; b < t.buckets.size(); ++b) {
        const auto& bk = t.buckets[b];
        CHECK(bk.first >= 0 && bk.count >= 1 && bk.first + bk.count <= (int)t.items.size(), "bucket range");
        CHECK(bk.grid >= 1 && bk.grid <= bk.count, "bucket %zu grid %d of %d items", b, bk.grid, bk.count);
        for (int i = bk.first; i < bk.first + bk.count && i < (int)t.items.size(); ++i) {
            CHECK(owner[i] < 0, "item %d in two buckets", i);
            owner[i] = (int)b;
            CHECK((t.items[i].k >= 0) == bk.pool(), "item %d in the wrong kind of bucket", i);
        }
        if (bk.pool()) {
            ++pool_buckets;
            CHECK(bk.first == 0, "pool bucket first");
            CHECK(bk.block == 64 * t.pool_waves && valid_pool_shape(t.pool_waves, t.pool_groups), "pool shape");
            CHECK(bk.lds_bytes == t.pool_pages * kPoolPageBytes, "pool LDS");
            CHECK(t.pool_groups == 1 || t.pool_groups == 2, "pool groups");
            CHECK(t.pool_pages >= 1 && t.pool_pages * t.pool_groups <= env.cu_pool_pages, "pool pages");
            // every workgroup of the shape fits one CU's LDS with its static part
            CHECK(t.pool_groups * (t.pool_pages * kPoolPageBytes + kPoolStaticLdsBytes) <=
                      env.cu_pool_pages * kPoolPageBytes + kPoolStaticLdsBytes, "pool LDS per CU");
            bool all_lite = true;
            for (int i = bk.first; i < bk.first + bk.count && i < (int)t.items.size(); ++i)
                all_lite = all_lite && npdu_item_lite(t.items[i].n, t.items[i].k, t.items[i].flags);
            CHECK(t.pool_lite == pool_shape_needs_lite(t.pool_waves, t.pool_groups), "light kernel choice");
            CHECK(!t.pool_lite || all_lite, "light kernel with sectors it cannot serve");
            CHECK(bk.grid <= t.pool_groups * env.cu_count, "pool grid");
            CHECK(t.seed_priority >= 0 && t.seed_priority <= 3, "priority");
        }
    }
    for (size_t i = 0; i < owner.size(); ++i) CHECK(owner[i] >= 0, "item %zu in no bucket", i);
    CHECK(pool_buckets <= 1, "pool buckets");

    // workgroups, queues and seeds: together exactly the NPDU items, pages in the pool
    int npdu_items = 0;
    for (const auto& it : t.items) npdu_items += it.k >= 0;
    int pool_grid = 0;
    for (const auto& bk : t.buckets)
        if (bk.pool()) pool_grid = bk.grid;
    CHECK((int)t.groups.size() == pool_grid && pool_grid <= kMaxPoolGroups, "%zu workgroups, grid %d",
          t.groups.size(), pool_grid);
    std::vector<int> seen(t.items.size(), 0);
    std::vector<int> in_queue(t.items.size(), 0);
    std::vector<int> group_of(t.items.size(), -1);
    int next_first = 0, next_queue = 0;
    for (size_t g = 0; g < t.groups.size(); ++g) {
        const PoolGroup& grp = t.groups[g];
        CHECK(grp.queue_first == next_queue && grp.queues >= 1 && grp.queues <= kMaxLocalQueues,
              "workgroup %zu queues [%d, +%d)", g, grp.queue_first, grp.queues);
        next_queue = grp.queue_first + grp.queues;
        std::set<int> pages_seen;
        for (int qi = grp.queue_first; qi < grp.queue_first + grp.queues && qi < (int)t.queues.size(); ++qi) {
            const PoolQueue& q = t.queues[qi];
            CHECK(q.first >= 0 && q.count >= 1 && q.first + q.count <= npdu_items, "queue range");
            CHECK(q.seeded >= 0 && q.seeded <= q.count, "queue seeded %d of %d", q.seeded, q.count);
            CHECK(q.pages >= 1 && q.pages <= t.pool_pages, "queue pages %d of %d", q.pages, t.pool_pages);
            CHECK(q.first == next_first, "queues tile the NPDU items in order");
            CHECK(pages_seen.insert(q.pages).second, "two queues of %d pages in workgroup %zu", q.pages, g);
            next_first = q.first + q.count;
            for (int i = q.first; i < q.first + q.count && i < (int)t.items.size(); ++i) {
                ++in_queue[i];
                group_of[i] = (int)g;
                if (i >= q.first + q.seeded) ++seen[i];   // round 0 queues only the unseeded ones
                const WorkItem& it = t.items[i];
                CHECK(npdu_pool_pages(it.n, npdu_item_xyz_in_lds(it.n, it.flags)) <= q.pages, "item pages");
            }
        }
    }
    CHECK(next_queue == (int)t.queues.size(), "workgroups cover the queues");
    CHECK(next_first == npdu_items, "queues cover the NPDU items");
    for (int i = 0; i < npdu_items; ++i) CHECK(in_queue[i] == 1, "NPDU item %d in %d queues (later rounds)", i, in_queue[i]);
    if (npdu_items) {
        const int waves = t.pool_waves;
        CHECK((int)t.seeds.size() == pool_grid * waves, "seed table shape");
        for (int g = 0; g < pool_grid; ++g) {
            std::vector<std::pair<int, int>> ranges;
            for (int w = 0; w < waves; ++w) {
                const PoolSeed& sd = t.seeds[(size_t)g * waves + w];
                if (sd.item < 0) continue;
                CHECK(sd.item < npdu_items, "seed item");
                if (sd.item >= npdu_items) continue;
                CHECK(group_of[sd.item] == g, "seed %d of workgroup %d is another workgroup's", sd.item, g);
                bool front = false;   // a seed is among the first `seeded` items of its queue, and takes its pages
                const PoolGroup& grp = t.groups[g];
                for (int qi = grp.queue_first; qi < grp.queue_first + grp.queues; ++qi) {
                    const PoolQueue& q = t.queues[qi];
                    if (sd.item >= q.first && sd.item < q.first + q.seeded) front = sd.pages == q.pages;
                }
                CHECK(front, "seed %d is not at the front of its queue with its pages", sd.item);
                ++seen[sd.item];
                CHECK(sd.page >= 0 && sd.page + sd.pages <= t.pool_pages, "seed pages [%d, %d) of %d", sd.page,
                      sd.page + sd.pages, t.pool_pages);
                CHECK(sd.sleeps == 0 || (sd.sleeps == 1 && env.pool.seed_sleep && w > 0), "seed sleeps");
                ranges.push_back({sd.page, sd.page + sd.pages});
            }
            std::sort(ranges.begin(), ranges.end());
            for (size_t r = 1; r < ranges.size(); ++r) CHECK(ranges[r - 1].second <= ranges[r].first, "seed pages overlap");
        }
    }
    for (int i = 0; i < npdu_items; ++i) CHECK(seen[i] == 1, "NPDU item %d queued or seeded %d times", i, seen[i]);
}

}  // namespace

int main(int argc, char** argv) {
    const int iters = argc > 1 ? std::atoi(argv[1]) : 1500;
    const uint64_t seed = argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 1;
    std::mt19937_64 rng(seed);
    const auto vars = fake_variants();
    int planned = 0, rejected = 0;
    for (int it = 0; it < iters; ++it) {
        const PlannerEnv env = make_env(rng, vars);
        auto d = random_batch(rng);
        PlanTables t;
        std::string err;
        const int rc = build_plan(d.data(), (int32_t)d.size(), env, &t, &err);
        // valid descriptors fail only where a sector exceeds the LDS pool of a
        // (small, random) device
        if (rc != AFPS_OK) {
            CHECK(rc == AFPS_ERR_UNSUPPORTED, "iteration %d: status %d (%s)", it, rc, err.c_str());
            ++rejected;
        } else {
            check_plan(d, env, t);
            ++planned;
        }
        // a corrupted copy is rejected with a descriptor error, never accepted
        if (!d.empty()) {
            auto bad = d;
            auto& c = bad[std::uniform_int_distribution<size_t>(0, bad.size() - 1)(rng)];
            switch (std::uniform_int_distribution<int>(0, 5)(rng)) {
                case 0: c.m = 0; break;
                case 1: c.c = c.n + 1; break;
                case 2: c.start = c.n; break;
                case 3: c.xyz_offset = -1; break;
                case 4: c.k = std::max(c.k, 0); c.flags = 8; break;
                default: c.m = c.c + 1; break;
            }
            PlanTables t2;
            const int rc2 = build_plan(bad.data(), (int32_t)bad.size(), env, &t2, &err);
            CHECK(rc2 == AFPS_ERR_ARG || rc2 == AFPS_ERR_RANGE, "iteration %d: corrupted batch got %d", it, rc2);
            CHECK(err.find("descriptor") != std::string::npos, "error names the descriptor: %s", err.c_str());
        }
    }
    // empty batch, null descriptors
    PlanTables t;
    std::string err;
    PlannerEnv env = make_env(rng, vars);
    CHECK(build_plan(nullptr, 0, env, &t, &err) == AFPS_OK && t.items.empty() && t.ws_bytes == 0, "empty batch");
    CHECK(build_plan(nullptr, 3, env, &t, &err) == AFPS_ERR_NULL, "null descriptors");
    CHECK(build_plan(nullptr, -1, env, &t, &err) == AFPS_ERR_ARG, "negative batch");
    std::printf("planner fuzz: %d plans checked, %d rejected by the device limits, %d failures\n", planned, rejected,
                g_failures);
    return g_failures ? 1 : 0;
}
