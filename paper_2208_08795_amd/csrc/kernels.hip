// Full-update sector kernels (FPS / AFPS) for one wave count (AFPS_WAVES),
// every slot count.
//
// direct_kernel     : one workgroup per sector of one cloud; the sector plan
//                     (Sec. III-B split) is evaluated from blockIdx.
// persistent_kernel : a fixed grid of workgroups that take sector work items
//                     from a device queue (one atomic per item, not per
//                     iteration) until it is empty; items arrive sorted
//                     longest-first, so the tail is short.
//
// This file is compiled once per wave count so the instantiations build in
// parallel; each build registers its kernels in the host-side variant table.
#include "sampler.hpp"
#include "variants.hpp"

#ifndef AFPS_WAVES
#error "AFPS_WAVES must be defined"
#endif

namespace afps {

template <int P, int W, bool DL>
__global__ __launch_bounds__(64 * W) void direct_kernel(const float* __restrict__ xyz, int n, int c,
                                                        int m, int start,
                                                        int32_t* __restrict__ out) {
    __shared__ Candidate lds[2 * W];
    extern __shared__ uint32_t dyn_lds[];
    const int s = blockIdx.x;
    const int qn = n / m, rn = n % m, qc = c / m, rc = c % m;
    const int ns = qn + (s < rn ? 1 : 0), b = s * qn + min(s, rn);
    const int cs = qc + (s < rc ? 1 : 0), o = s * qc + min(s, rc);
    sample_sector<P, W, DL>(xyz + 3 * (int64_t)b, ns, cs, start % ns, b, out + o, lds, dyn_lds);
}

template <int P, int W, bool DL>
__global__ __launch_bounds__(64 * W) void persistent_kernel(const float* __restrict__ xyz_all,
                                                            int32_t* __restrict__ out_all,
                                                            const WorkItem* __restrict__ items,
                                                            int n_items, unsigned* counter) {
    __shared__ Candidate lds[2 * W];
    __shared__ unsigned next;
    extern __shared__ uint32_t dyn_lds[];
    for (;;) {
        unsigned it;
        if (W == 1) {
            unsigned v = 0;
            if (threadIdx.x == 0) v = atomicAdd(counter, 1u);
            it = (unsigned)__builtin_amdgcn_readfirstlane((int)v);
        } else {
            if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
            __syncthreads();
            it = next;
            __syncthreads();
        }
        if (it >= (unsigned)n_items) break;   // every workgroup ends once the queue is drained
        const WorkItem wi = items[it];
        sample_sector<P, W, DL>(xyz_all + 3 * wi.xyz_offset, wi.n, wi.c, wi.start, wi.base,
                                out_all + wi.out_offset, lds, dyn_lds);
    }
}

template <int P, bool DL = false>
static void add(std::vector<VariantEntry>& v) {
    constexpr int W = AFPS_WAVES;
    v.push_back({W, P, DL ? P * 64 * W * 4 : 0, (const void*)&direct_kernel<P, W, DL>,
                 (const void*)&persistent_kernel<P, W, DL>});
}

#define AFPS_CAT2(a, b) a##b
#define AFPS_CAT(a, b) AFPS_CAT2(a, b)

void AFPS_CAT(register_variants_w, AFPS_WAVES)(std::vector<VariantEntry>& v) {
    add<1>(v);
    add<2>(v);
    add<4>(v);
    add<8>(v);
    add<12>(v);
    add<16>(v);
    add<24>(v);
#if AFPS_WAVES < 16
    add<32>(v);   // 4*32 data registers only fit below 4 waves per SIMD
#else
    add<32, true>(v);   // 32768 points: x,y,z in registers, distances in 128 KB of LDS
#endif
}

}  // namespace afps
