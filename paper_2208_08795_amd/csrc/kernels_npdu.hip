// NPDU sector kernels (Sec. III-C) of single-cloud calls: one workgroup of
// one wave per sector, sector in LDS; dynamic LDS (XYZ_IN_LDS ? 16 : 4) bytes
// per point of the largest sector.  Batch plans run their NPDU sectors in the
// pooled kernel (kernels_pool.hip).
#include "sampler.hpp"
#include "variants.hpp"

namespace afps {

template <int R, bool XYZ>
__global__ __launch_bounds__(64) void direct_npdu_kernel(const float* __restrict__ xyz, int n, int c,
                                                         int m, int k, int start, int flags,
                                                         int32_t* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint32_t dyn_lds[];
    const int s = blockIdx.x;
    const int qn = n / m, rn = n % m, qc = c / m, rc = c % m;
    const int ns = qn + (s < rn ? 1 : 0), b = s * qn + min(s, rn);
    const int cs = qc + (s < rc ? 1 : 0), o = s * qc + min(s, rc);
    sample_sector_npdu<R, XYZ>(xyz + 3 * (int64_t)b, ns, cs, k, start % ns, b, out + o, dyn_lds, flags);
}

template <int R, bool XYZ>
static void add(std::vector<NpduEntry>& v) {
    v.push_back({R, XYZ ? 1 : 0, (const void*)&direct_npdu_kernel<R, XYZ>});
}

void register_npdu_variants(std::vector<NpduEntry>& v) {
    add<1, true>(v);    // n <= 4096,  64 KB LDS
    add<2, true>(v);    // n <= 8192, 128 KB LDS
    add<4, false>(v);   // n <= 16384, 64 KB LDS (x,y,z from L2)
    add<8, false>(v);   // n <= 32768, 128 KB LDS
}

// Queue counters live in the caller's workspace; a kernel (not a memset)
// clears them so the whole batch pipeline can be captured in a graph.
__global__ void queue_reset(unsigned* counters, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) counters[i] = 0u;
}
const void* queue_reset_kernel() { return (const void*)&queue_reset; }

}  // namespace afps
