// Batch planner (see planner.hpp): plain C++, no HIP calls.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <utility>

namespace afps {

namespace {

// Estimated cycles of one NPDU iteration of one wave (window within two
// blocks) with another wave on its SIMD, by block registers and coordinate
// placement: measured per-sector cycles per iteration of pooled launches.
// Coordinates in registers (sectors of at most 4096 points, k <= 64) cost
// the lane selects of the register sets; from L2 they cost a round trip per
// iteration where LDS would serve.
double npdu_iter_cycles(int n, bool xyz_in_lds, int k) {
    switch (npdu_r_for(n)) {
        case 1: return xyz_in_lds ? 520.0 : (k <= 64 ? 640.0 : 1300.0);
        case 2: return xyz_in_lds ? 650.0 : 1300.0;
        case 4: return 830.0;
        default: return 1000.0;
    }
}

// Estimated cycles of a full-update sector of c samples on a variant: per
// iteration 12 VALU ops per slot on each of the ceil(W/4) waves sharing a
// SIMD (4 cycles each), plus the reduction and, for W > 1, the LDS exchange.
double full_cost(int c, const FullVariantInfo& v) {
    const int per_simd = (v.waves + 3) / 4;
    return (double)c * (48.0 * v.slots * per_simd + (v.waves > 1 ? 600.0 : 250.0));
}

struct Staged {
    WorkItem item;
    FullVariantInfo full;   // full-update variant (full.id >= 0), or NPDU (id -1)
    int pages;              // NPDU: pool pages
    double cost;            // estimated cycles
};

}  // namespace

int check_sizes(int32_t n, int32_t c, int32_t m, int32_t start, std::string* err) {
    if (m < 1 || c < m || n < c) {
        *err = "sizes must satisfy 1 <= m <= c <= n (n=" + std::to_string(n) + ", c=" + std::to_string(c) +
               ", m=" + std::to_string(m) + ")";
        return AFPS_ERR_ARG;
    }
    if (start < 0 || start >= n) {
        *err = "start " + std::to_string(start) + " outside [0, n)";
        return AFPS_ERR_RANGE;
    }
    return AFPS_OK;
}

int npdu_readings(int32_t* k, int32_t* flags, std::string* err) {
    if (*flags & ~(AFPS_NPDU_FIRST_FULL | AFPS_NPDU_SHIFT_EDGES | AFPS_NPDU_K_WITH_SELF)) {
        *err = "unknown NPDU reading flags";
        return AFPS_ERR_ARG;
    }
    if (*flags && *k < 0) {
        *err = "NPDU reading flags need NPDU (k >= 0)";
        return AFPS_ERR_ARG;
    }
    if (*flags & AFPS_NPDU_K_WITH_SELF) {
        if (*k < 1) {
            *err = "k must be >= 1 when it counts the sample";
            return AFPS_ERR_ARG;
        }
        *k -= 1;
        *flags &= ~AFPS_NPDU_K_WITH_SELF;
    }
    return AFPS_OK;
}

int32_t largest_sector(int32_t n, int32_t m) { return n / m + (n % m ? 1 : 0); }

int32_t clamp_k(int32_t k, int32_t n_s) { return k > 2 * n_s ? 2 * n_s : k; }

bool valid_pool_shape(int waves, int groups) {
    return (waves == 4 && (groups == 1 || groups == 2)) || ((waves == 8 || waves == 12 || waves == 16) && groups == 1) ||
           ((waves == 12 || waves == 16) && groups == 2);
}

bool pool_shape_needs_lite(int waves, int groups) { return groups == 2 && waves >= 12; }

bool npdu_xyz_in_lds(const PoolPolicy& policy, int n, int k) {
    if (npdu_r_for(n) > 2) return false;
    for (const auto& e : policy.placement)
        if (n <= e.n_max && k <= e.k_max) return e.xyz_in_lds != 0;
    // built-in: 16-byte records in LDS (the fastest iteration, so the
    // shortest single launch); throughput-bound batches tune a placement out
    // of LDS (registers or L2), which lets a CU hold more sectors at once
    (void)k;
    return true;
}

int build_plan(const afps_cloud_desc* descs, int32_t batch, const PlannerEnv& env, PlanTables* out,
               std::string* err) {
    PlanTables& plan = *out;
    plan = PlanTables();
    if (batch < 0) {
        *err = "batch must be >= 0";
        return AFPS_ERR_ARG;
    }
    if (batch > 0 && !descs) {
        *err = "descs must be non-null";
        return AFPS_ERR_NULL;
    }

    // ---- every cloud cut into its sectors (Sec. III-B), each a work item
    std::vector<Staged> staged;
    for (int32_t b = 0; b < batch; ++b) {
        const afps_cloud_desc& d = descs[b];
        const std::string where = "descriptor " + std::to_string(b) + ": ";
        if (d.xyz_offset < 0 || d.out_offset < 0) {
            *err = where + "negative offset";
            return AFPS_ERR_ARG;
        }
        std::string e;
        int rc = check_sizes(d.n, d.c, d.m, d.start, &e);
        int32_t dk = d.k, dflags = d.flags;
        if (!rc) rc = npdu_readings(&dk, &dflags, &e);
        if (rc) {
            *err = where + e;
            return rc;
        }
        plan.clouds.push_back(CheckSeg{d.xyz_offset, d.n, 0});
        const int32_t qn = d.n / d.m, rn = d.n % d.m, qc = d.c / d.m, rc_ = d.c % d.m;
        for (int32_t s = 0; s < d.m; ++s) {
            Staged st{};
            WorkItem& it = st.item;
            const int32_t ns = qn + (s < rn ? 1 : 0), bs = s * qn + std::min(s, rn);
            const int32_t cs = qc + (s < rc_ ? 1 : 0), os = s * qc + std::min(s, rc_);
            it.xyz_offset = d.xyz_offset + bs;
            it.out_offset = d.out_offset + os;
            it.n = ns;
            it.c = cs;
            it.k = dk < 0 ? -1 : clamp_k(dk, ns);
            it.start = d.start % ns;
            it.base = bs;
            it.flags = dflags;
            if (dk >= 0) {
                if (npdu_r_for(ns) == 0) {
                    *err = where + "NPDU sector too large";
                    return AFPS_ERR_UNSUPPORTED;
                }
                const bool in_lds = npdu_xyz_in_lds(env.pool, ns, it.k);
                if (!in_lds && npdu_r_for(ns) <= 2) it.flags |= kItemXyzNotInLds;
                st.full.id = -1;
                st.pages = npdu_pool_pages(ns, in_lds);
                // windows wider than two blocks re-reduce one more block pair per extra 128
                st.cost = (double)cs * npdu_iter_cycles(ns, in_lds, it.k) * (1.0 + std::max(0, it.k - 64) / 128.0);
            } else {
                FullVariantInfo v{};
                if (!env.choose_full || !env.choose_full(ns, &v)) {
                    *err = where + "sector of " + std::to_string(ns) +
                           " points exceeds one workgroup (split into more sectors)";
                    return AFPS_ERR_UNSUPPORTED;
                }
                st.full = v;
                st.cost = full_cost(cs, v);
            }
            staged.push_back(st);
        }
    }
    if (staged.empty()) return AFPS_OK;
    if (env.cu_count < 1 || env.cu_pool_pages < 1 || env.cu_pool_pages > kMaxPoolPages) {
        *err = "device facts out of range";
        return AFPS_ERR_ARG;
    }
    plan.pool_pages = env.cu_pool_pages;

    // ---- NPDU sectors: one pooled launch.
    std::vector<Staged> npdu, full;
    for (auto& st : staged) (st.full.id < 0 ? npdu : full).push_back(st);
    for (const auto& st : npdu)
        if (st.pages > plan.pool_pages) {
            *err = "NPDU sector of " + std::to_string(st.item.n) + " points exceeds the LDS of one CU";
            return AFPS_ERR_UNSUPPORTED;
        }

    // Full-update sectors: one bucket per (variant, LDS), longest first inside.
    std::stable_sort(full.begin(), full.end(), [](const Staged& a, const Staged& b) {
        if (a.full.id != b.full.id) return a.full.id < b.full.id;
        if (a.full.lds_bytes != b.full.lds_bytes) return a.full.lds_bytes < b.full.lds_bytes;
        return a.cost > b.cost;
    });

    plan.items.reserve(staged.size());
    std::vector<double> item_cost;   // estimated cycles, aligned with plan.items
    item_cost.reserve(staged.size());
    if (!npdu.empty()) {
        PlannedBucket bk{-1, 0, 0, 0, 0, 0, 0.0, 0.0};
        int max_pages = 0;
        bool all_lite = true;
        for (const auto& st : npdu) {
            bk.cost += st.cost;
            bk.longest = std::max(bk.longest, st.cost);
            max_pages = std::max(max_pages, st.pages);
            all_lite = all_lite && npdu_item_lite(st.item.n, st.item.k, st.item.flags);
        }
        bk.count = (int)npdu.size();
        // Waves per CU: one per SIMD keeps the longest sectors at full speed;
        // two per SIMD give more throughput (about 1.7x) when the batch is
        // bound by total work rather than by its longest sector.
        const double cus = (double)env.cu_count;
        const double span4 = std::max(bk.longest, bk.cost / (4.0 * cus));
        const double span8 = std::max(1.18 * bk.longest, bk.cost / (6.8 * cus));
        int waves = span8 < span4 ? 8 : 4;
        if (env.pool.waves_per_simd > 0.0f) waves = env.pool.waves_per_simd < 1.5f ? 4 : 8;
        // Two waves per SIMD run as two workgroups of four per CU, each owning
        // half of the CU's pages, whenever every sector fits half: one launch
        // runs as fast either way, but a launch then gives its LDS back half
        // a CU at a time, so a launch queued behind it on another stream
        // starts sooner.
        plan.pool_groups = waves == 8 && max_pages <= pool_pages_per_group(plan.pool_pages, 2) ? 2 : 1;
        if (plan.pool_groups == 2) waves = 4;
        if (env.pool.waves > 0 && env.pool.groups > 0) {   // an explicit (tuned) shape
            const bool ok = valid_pool_shape(env.pool.waves, env.pool.groups) &&
                            max_pages <= pool_pages_per_group(plan.pool_pages, env.pool.groups) &&
                            (all_lite || !pool_shape_needs_lite(env.pool.waves, env.pool.groups));
            if (ok) {
                waves = env.pool.waves;
                plan.pool_groups = env.pool.groups;
            }
        }
        plan.pool_pages = pool_pages_per_group(plan.pool_pages, plan.pool_groups);
        plan.pool_waves = waves;
        plan.pool_lite = pool_shape_needs_lite(waves, plan.pool_groups);   // all_lite holds then
        plan.seed_priority = std::max(0, std::min(3, env.pool.seed_priority));
        bk.block = 64 * waves;
        bk.lds_bytes = plan.pool_pages * kPoolPageBytes;
        const int G = std::min({plan.pool_groups * env.cu_count, bk.count, kMaxPoolGroups});
        bk.grid = G;

        // Every sector goes to one workgroup for good (and so for every
        // round alike): longest-processing-time first, each to the workgroup
        // that is least loaded, counting a workgroup's load as its estimated
        // cycles over its waves or its page-weighted cycles over its pages,
        // whichever is larger (large sectors run fewer at a time).  Claims
        // then stay inside the workgroup's LDS: no device-wide counter is
        // touched per sector.
        std::vector<int> order(npdu.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return npdu[x].cost > npdu[y].cost; });
        std::vector<double> load_c(G, 0.0), load_p(G, 0.0);
        auto key = [&](int g) { return std::max(load_c[g] / waves, load_p[g] / plan.pool_pages); };
        auto later = [&](int x, int y) { return key(x) > key(y) || (key(x) == key(y) && x > y); };
        std::vector<int> heap(G);
        for (int g = 0; g < G; ++g) heap[g] = g;
        std::make_heap(heap.begin(), heap.end(), later);
        std::vector<std::vector<int>> members(G);
        for (int i : order) {
            std::pop_heap(heap.begin(), heap.end(), later);
            const int g = heap.back();
            members[g].push_back(i);   // in descending cost
            load_c[g] += npdu[i].cost;
            load_p[g] += npdu[i].cost * npdu[i].pages;
            std::push_heap(heap.begin(), heap.end(), later);
        }

        // Inside a workgroup: queues by pages (rounded up to fewer distinct
        // counts if there would be more than kMaxLocalQueues), longest first,
        // the queues ordered by their longest sector.  Seeds: the queue
        // policy of the kernel played out for the moment every wave starts
        // (wave 0 first, each taking the first queue with sectors left that
        // fits the workgroup's pages), so that a launch starts without a rush
        // on the workgroup's lock.  A workgroup's seeds sit in consecutive
        // pages from page 0; the seeded sectors are the front of their queues,
        // which in round 0 start after them.  Seeds after the first whose
        // estimated cost leaves room before the plan's longest sector wait
        // one sleep period before loading: the first sectors then load with
        // less competition for bandwidth, and the wait cannot lengthen the
        // launch by the cost model.
        std::vector<double> item_cost_npdu;
        plan.seeds.assign((size_t)G * waves, PoolSeed{-1, 0, 0, 0});
        for (int g = 0; g < G; ++g) {
            std::vector<int> distinct;
            for (int i : members[g]) distinct.push_back(npdu[i].pages);
            std::sort(distinct.begin(), distinct.end());
            distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
            int step = 1;
            auto rounded = [&](int p) { return std::min(plan.pool_pages, (p + step - 1) / step * step); };
            for (;;) {
                std::vector<int> r;
                for (int p : distinct) r.push_back(rounded(p));
                r.erase(std::unique(r.begin(), r.end()), r.end());
                if ((int)r.size() <= kMaxLocalQueues) break;
                ++step;
            }
            std::vector<std::pair<int, std::vector<int>>> lq;   // (pages, members in descending cost)
            for (int i : members[g]) {
                const int p = rounded(npdu[i].pages);
                auto it = std::find_if(lq.begin(), lq.end(), [p](const auto& e) { return e.first == p; });
                if (it == lq.end()) {
                    lq.push_back({p, {}});
                    it = lq.end() - 1;
                }
                it->second.push_back(i);
            }
            // members are in descending cost, so each queue's first item is its
            // longest and the queues come out ordered by it
            PoolGroup grp{(int)plan.queues.size(), (int)lq.size()};
            plan.groups.push_back(grp);
            std::vector<int> qfirst;
            for (const auto& e : lq) {
                qfirst.push_back((int)plan.items.size());
                for (int i : e.second) {
                    plan.items.push_back(npdu[i].item);
                    item_cost_npdu.push_back(npdu[i].cost);
                }
                plan.queues.push_back(PoolQueue{qfirst.back(), (int)e.second.size(), e.first, 0});
            }
            int used = 0;
            for (int w = 0; w < waves; ++w)
                for (size_t q = 0; q < lq.size(); ++q) {
                    PoolQueue& Q = plan.queues[grp.queue_first + q];
                    if (Q.seeded < Q.count && used + Q.pages <= plan.pool_pages) {
                        const int item = Q.first + Q.seeded;
                        const bool slack = env.pool.seed_sleep && w > 0 &&
                                           item_cost_npdu[item] + kSeedSleepCycles <= bk.longest;
                        plan.seeds[(size_t)g * waves + w] =
                            PoolSeed{item, (int16_t)used, (uint8_t)Q.pages, (uint8_t)(slack ? 1 : 0)};
                        used += Q.pages;
                        ++Q.seeded;
                        break;
                    }
                }
        }
        for (double c : item_cost_npdu) item_cost.push_back(c);
        plan.buckets.push_back(bk);
    }
    for (size_t i = 0; i < full.size();) {
        size_t j = i;
        PlannedBucket bk{full[i].full.id, 64 * full[i].full.waves, full[i].full.lds_bytes, (int)plan.items.size(),
                         0, 0, 0.0, 0.0};
        while (j < full.size() && full[j].full.id == bk.variant && full[j].full.lds_bytes == bk.lds_bytes) {
            bk.cost += full[j].cost;
            bk.longest = std::max(bk.longest, full[j].cost);
            plan.items.push_back(full[j].item);
            item_cost.push_back(full[j].cost);
            ++j;
        }
        bk.count = (int)(j - i);
        plan.buckets.push_back(bk);
        i = j;
    }
    if ((int)plan.buckets.size() > kMaxBuckets) {
        *err = "too many kernel variants in one plan";
        return AFPS_ERR_UNSUPPORTED;
    }
    // Largest bucket first: it gets the first helper stream.
    std::stable_sort(plan.buckets.begin(), plan.buckets.end(),
                     [](const PlannedBucket& a, const PlannedBucket& b) { return a.cost > b.cost; });

    // ---- full-update persistent grids.  Makespan model: the queue hands out
    // items longest first, so a bucket run by g workgroups finishes when the
    // longest-processing-time (LPT) schedule of its item costs on g machines
    // does.  Take the critical path T = the longest item of the plan, give
    // each bucket the fewest workgroups whose LPT schedule ends by T, and
    // raise T until all buckets together stay within the wave budget (waves
    // per SIMD x SIMDs).  Never more workgroups than items or than fit.
    const float budget_simd = env.pool.waves_per_simd;
    const double budget = std::max(1.0, (double)budget_simd * 4.0 * env.cu_count);
    std::vector<int> cap(plan.buckets.size(), 0);
    double T = 0.0;
    for (size_t b = 0; b < plan.buckets.size(); ++b) {
        PlannedBucket& bk = plan.buckets[b];
        T = std::max(T, bk.longest);
        if (bk.pool()) continue;
        FullVariantInfo v{bk.variant, bk.block / 64, 0, bk.lds_bytes};
        const int per_cu = env.blocks_per_cu ? env.blocks_per_cu(v) : 0;
        if (per_cu < 1) {
            *err = "a kernel variant cannot be resident";
            return AFPS_ERR_UNSUPPORTED;
        }
        cap[b] = std::min(bk.count, per_cu * env.cu_count);
    }
    auto lpt_makespan = [&](const PlannedBucket& bk, int g) {
        std::vector<double> load(g, 0.0);   // min-heap of machine loads
        double span = 0.0;
        for (int i = 0; i < bk.count; ++i) {
            std::pop_heap(load.begin(), load.end(), std::greater<double>());
            load.back() += item_cost[bk.first + i];
            span = std::max(span, load.back());
            std::push_heap(load.begin(), load.end(), std::greater<double>());
        }
        return span;
    };
    auto workgroups_for = [&](size_t b, double t) {
        const PlannedBucket& bk = plan.buckets[b];
        int lo = (int)std::min<double>(cap[b], std::max(1.0, std::ceil(bk.cost / t)));
        int hi = cap[b];
        if (lpt_makespan(bk, lo) <= t * 1.0001) return lo;
        while (lo + 1 < hi) {   // smallest g in (lo, hi] meeting t
            const int mid = lo + (hi - lo) / 2;
            if (lpt_makespan(bk, mid) <= t * 1.0001) hi = mid;
            else lo = mid;
        }
        return hi;
    };
    if (budget_simd <= 0.0f) {
        for (size_t b = 0; b < plan.buckets.size(); ++b)
            if (!plan.buckets[b].pool()) plan.buckets[b].grid = cap[b];
    } else {
        for (int round = 0; round < 200; ++round) {
            double waves = 0.0;
            for (size_t b = 0; b < plan.buckets.size(); ++b) {
                PlannedBucket& bk = plan.buckets[b];
                if (!bk.pool()) bk.grid = workgroups_for(b, T);
                waves += (double)bk.grid * (bk.block / 64);
            }
            if (waves <= budget) break;
            T *= 1.05;
        }
    }
    plan.ws_bytes = workspace_bytes_for_items((int64_t)plan.items.size());
    return AFPS_OK;
}

}  // namespace afps
