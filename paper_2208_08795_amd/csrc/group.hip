// Grouping around the samples: the ball query of a PointNet++ set
// abstraction layer, the consumer of the samples that the paper names
// (Sec. I, Sec. II-A).  For each centre (a sampled point's index), the first
// k points in index order whose squared fp32 distance to it is below
// radius^2, padded with the first found (the centre itself when none is).
// With a storage window w, only points within w positions of the centre are
// candidates (Sec. III-A: with dimensional locality, storage neighbours
// approximate spatial neighbours), which bounds the search to 2w + 1 points.
//
// One wave per centre.  The wave scans its candidates 256 at a time (four
// coalesced 64-point rows in flight), a ballot per row gives the hits, and
// each hit's slot is the number of hits before it (lower rows, then lower
// lanes), so the output keeps index order without any sorting.  The scan
// stops at the first group of rows that completes k.
#include "sampler.hpp"
#include "variants.hpp"

namespace afps {

namespace {

constexpr int kGroupRows = 4;   // 64-point rows loaded together

}  // namespace

__global__ __launch_bounds__(256) void ball_query_kernel(const float* __restrict__ xyz, int n,
                                                         const int32_t* __restrict__ centers, int c,
                                                         uint32_t r2_bits, int k, int window,
                                                         int32_t* __restrict__ out_idx,
                                                         int32_t* __restrict__ out_cnt) {
    const int lane = threadIdx.x & 63;
    const int waves = (int)(blockDim.x >> 6);
    const uint64_t below = (1ull << lane) - 1ull;
    for (int q = blockIdx.x * waves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); q < c;
         q += gridDim.x * waves) {
        int32_t* row = out_idx + (int64_t)q * k;
        const int ci = __builtin_amdgcn_readfirstlane(centers[q]);
        if (ci < 0 || ci >= n) {   // not a point of the cloud: the centre's outputs are -1
            for (int l = lane; l < k; l += 64) row[l] = -1;
            if (out_cnt && lane == 0) out_cnt[q] = -1;
            continue;
        }
        const float px = xyz[3 * (int64_t)ci], py = xyz[3 * (int64_t)ci + 1], pz = xyz[3 * (int64_t)ci + 2];
        int lo = 0, hi = n - 1;
        if (window >= 0) {
            lo = ci - window < 0 ? 0 : ci - window;
            hi = ci > n - 1 - window ? n - 1 : ci + window;
        }
        int found = 0, first = ci;
        // 64-bit positions: the last group may reach past 2^31 - 1
        for (int64_t j0 = lo; j0 <= hi && found < k; j0 += 64 * kGroupRows) {
            float x[kGroupRows], y[kGroupRows], z[kGroupRows];
#pragma unroll
            for (int u = 0; u < kGroupRows; ++u) {
                const int64_t j = min(j0 + 64 * u + lane, (int64_t)hi);   // past hi: point hi again, never a hit
                x[u] = xyz[3 * j];
                y[u] = xyz[3 * j + 1];
                z[u] = xyz[3 * j + 2];
            }
#pragma unroll
            for (int u = 0; u < kGroupRows; ++u) {
                const int64_t j = j0 + 64 * u + lane;
                const bool hit = j <= hi && sq_dist_bits(x[u], y[u], z[u], px, py, pz) < r2_bits;
                const uint64_t m = ballot(hit);
                if (m != 0ull && found == 0) first = (int)(j0 + 64 * u + (int)__builtin_ctzll(m));
                const int slot = found + (int)__popcll(m & below);
                if (hit && slot < k) row[slot] = (int32_t)j;
                found += (int)__popcll(m);
            }
        }
        const int cnt = min(found, k);
        for (int l = cnt + lane; l < k; l += 64) row[l] = first;
        if (out_cnt && lane == 0) out_cnt[q] = cnt;
    }
}

const void* ball_query_kernel_ptr() { return (const void*)&ball_query_kernel; }

}  // namespace afps
