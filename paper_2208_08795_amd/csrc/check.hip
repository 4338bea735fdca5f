// Validation of the inputs' preconditions (the distance arithmetic assumes
// finite coordinates and squared distances below the initial 1e10 of
// Algorithm 1).  Run on request only: it reads every point once more and the
// host then waits for the result.
#include "variants.hpp"

namespace afps {

namespace {

// Unsigned key with the order of the (finite) float.
__device__ __forceinline__ uint32_t order_key(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

}  // namespace

__global__ __launch_bounds__(256) void check_points(const float* __restrict__ xyz_all, CheckBatch batch,
                                                    CheckResult* __restrict__ res) {
    __shared__ unsigned long long s_bad;
    __shared__ uint32_t s_lo[3], s_hi[3];
    const CheckSeg sg = batch.seg[blockIdx.x];
    if (threadIdx.x == 0) {
        s_bad = ~0ull;
        for (int a = 0; a < 3; ++a) {
            s_lo[a] = ~0u;
            s_hi[a] = 0u;
        }
    }
    __syncthreads();
    const float* p = xyz_all + 3 * sg.offset;
    unsigned long long bad = ~0ull;
    uint32_t lo[3] = {~0u, ~0u, ~0u}, hi[3] = {0u, 0u, 0u};
    for (int64_t j = threadIdx.x; j < sg.n; j += blockDim.x) {
        const float v[3] = {p[3 * j], p[3 * j + 1], p[3 * j + 2]};
        if (!(__builtin_isfinite(v[0]) && __builtin_isfinite(v[1]) && __builtin_isfinite(v[2]))) {
            bad = min(bad, (unsigned long long)j);
            continue;
        }
        for (int a = 0; a < 3; ++a) {
            const uint32_t k = order_key(v[a]);
            lo[a] = min(lo[a], k);
            hi[a] = max(hi[a], k);
        }
    }
    atomicMin(&s_bad, bad);
    for (int a = 0; a < 3; ++a) {
        atomicMin(&s_lo[a], lo[a]);
        atomicMax(&s_hi[a], hi[a]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        CheckResult r;
        r.first_bad = s_bad;
        for (int a = 0; a < 3; ++a) {
            r.lo[a] = s_lo[a];
            r.hi[a] = s_hi[a];
        }
        res[blockIdx.x] = r;
    }
}

const void* check_points_kernel() { return (const void*)&check_points; }

}  // namespace afps
