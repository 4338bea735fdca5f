// NPDU sector kernels (Sec. III-C): one wave per sector, sector in LDS.
//
// direct_npdu_kernel     : one workgroup per sector of one cloud.
// persistent_npdu_kernel : workgroups take sector work items from a device
//                          queue until it is empty.
// Dynamic LDS: (XYZ_IN_LDS ? 16 : 4) bytes per point of the largest sector.
#include "sampler.hpp"
#include "variants.hpp"

namespace afps {

template <int R, bool XYZ>
__global__ __launch_bounds__(64) void direct_npdu_kernel(const float* __restrict__ xyz, int n, int c,
                                                         int m, int k, int start,
                                                         int32_t* __restrict__ out) {
    extern __shared__ uint32_t dyn_lds[];
    const int s = blockIdx.x;
    const int qn = n / m, rn = n % m, qc = c / m, rc = c % m;
    const int ns = qn + (s < rn ? 1 : 0), b = s * qn + min(s, rn);
    const int cs = qc + (s < rc ? 1 : 0), o = s * qc + min(s, rc);
    sample_sector_npdu<R, XYZ>(xyz + 3 * (int64_t)b, ns, cs, k, start % ns, b, out + o, dyn_lds);
}

template <int R, bool XYZ>
__global__ __launch_bounds__(64) void persistent_npdu_kernel(const float* __restrict__ xyz_all,
                                                             int32_t* __restrict__ out_all,
                                                             const WorkItem* __restrict__ items,
                                                             int n_items, unsigned* counter) {
    extern __shared__ uint32_t dyn_lds[];
    for (;;) {
        unsigned v = 0;
        if (threadIdx.x == 0) v = atomicAdd(counter, 1u);
        const unsigned it = (unsigned)__builtin_amdgcn_readfirstlane((int)v);
        if (it >= (unsigned)n_items) break;   // every workgroup ends once the queue is drained
        const WorkItem wi = items[it];
        sample_sector_npdu<R, XYZ>(xyz_all + 3 * wi.xyz_offset, wi.n, wi.c, wi.k, wi.start, wi.base,
                                   out_all + wi.out_offset, dyn_lds);
        __syncthreads();   // LDS of this item is dead before the next item's load
    }
}

template <int R, bool XYZ>
static void add(std::vector<NpduEntry>& v) {
    v.push_back({R, XYZ ? 1 : 0, (const void*)&direct_npdu_kernel<R, XYZ>,
                 (const void*)&persistent_npdu_kernel<R, XYZ>});
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
