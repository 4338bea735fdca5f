// Binning of a cloud along one axis (Sec. III-A: a cloud without dimensional
// locality can be binned instead of sorted, into the approximate order of the
// footnote to Table II: every point of a later bin has a larger coordinate,
// points inside a bin keep their storage order).
//
// A stable counting sort by bin, in six launches (kernels only, so a caller
// may capture them in a graph):
//   bin_reset       : the range keys start empty;
//   bin_range       : smallest and largest coordinate (order keys, atomics);
//   bin_count       : per chunk of kBinChunk (1024) points, a histogram of the
//                     bins (LDS), stored bin-major;
//   bin_scan_rows   : one wave per bin: its chunks' counts become offsets
//                     inside the bin, and the bin's size;
//   bin_scan_totals : one workgroup: the bin sizes become the bins' first
//                     output positions (bins in order);
//   bin_scatter     : one wave per chunk loads its points at once, then walks
//                     them in storage order, 64 at a time; a point's rank
//                     among the lanes of its bin comes from one ballot per bit
//                     of the bin, so the order inside a bin is the storage
//                     order.
// The bin of a point is decided in fp32: scale = bins / (hi - lo) (correctly
// rounded), t = (x - lo) * scale, bin = min(bins - 1, floor(t)).
#include "sampler.hpp"
#include "variants.hpp"

namespace afps {

namespace {

__device__ __forceinline__ uint32_t order_key(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float from_key(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

struct BinRange {
    float lo, scale;
};
__device__ __forceinline__ BinRange bin_range_of(const BinHeader* h, int bins) {
    const float lo = from_key(h->lo_key), hi = from_key(h->hi_key);
    return {lo, hi > lo ? __fdiv_rn((float)bins, hi - lo) : 0.f};
}
__device__ __forceinline__ int bin_of(float x, BinRange r, int bins) {
    const float t = (x - r.lo) * r.scale;
    return min(bins - 1, (int)t);   // t >= 0: the conversion truncates, i.e. floors
}

}  // namespace

__global__ void bin_reset(BinHeader* h) {
    if (threadIdx.x == 0) {
        h->lo_key = ~0u;
        h->hi_key = 0u;
    }
}

__global__ __launch_bounds__(256) void bin_range(const float* __restrict__ xyz, int n, int axis, BinHeader* h) {
    __shared__ uint32_t s_lo, s_hi;
    if (threadIdx.x == 0) {
        s_lo = ~0u;
        s_hi = 0u;
    }
    __syncthreads();
    uint32_t lo = ~0u, hi = 0u;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const uint32_t k = order_key(xyz[3 * (int64_t)j + axis]);
        lo = min(lo, k);
        hi = max(hi, k);
    }
    atomicMin(&s_lo, lo);
    atomicMax(&s_hi, hi);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMin(&h->lo_key, s_lo);
        atomicMax(&h->hi_key, s_hi);
    }
}

__global__ __launch_bounds__(256) void bin_count(const float* __restrict__ xyz, int n, int axis, int bins,
                                                 const BinHeader* h, uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[kMaxBins];
    for (int b = threadIdx.x; b < bins; b += blockDim.x) cnt[b] = 0u;
    __syncthreads();
    const BinRange r = bin_range_of(h, bins);
    const int first = blockIdx.x * kBinChunk, last = min(n, first + kBinChunk);
    for (int j = first + threadIdx.x; j < last; j += blockDim.x)
        atomicAdd(&cnt[bin_of(xyz[3 * (int64_t)j + axis], r, bins)], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < bins; b += blockDim.x) hist[(int64_t)b * gridDim.x + blockIdx.x] = cnt[b];
}

// Row scan, one wave per bin: hist[b][c] (count of bin b in chunk c; a bin's
// chunks are contiguous) becomes the number of bin-b points in chunks before
// c, and totals[b] the bin's size.
__global__ __launch_bounds__(256) void bin_scan_rows(uint32_t* __restrict__ hist, uint32_t* __restrict__ totals,
                                                     int chunks, int bins) {
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (b >= bins) return;
    uint32_t* row = hist + (int64_t)b * chunks;
    uint32_t carry = 0u;
    for (int c0 = 0; c0 < chunks; c0 += 64) {
        const int c = c0 + lane;
        const uint32_t v = c < chunks ? row[c] : 0u;
        uint32_t incl = v;   // inclusive prefix inside the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t up = (uint32_t)__shfl_up((int)incl, d, 64);
            incl += lane >= d ? up : 0u;
        }
        if (c < chunks) row[c] = carry + incl - v;
        carry += readlane(incl, 63);
    }
    if (lane == 0) totals[b] = carry;
}

// Exclusive scan of the bin sizes (bins in order): totals[b] becomes the first
// output position of bin b.
__global__ __launch_bounds__(1024) void bin_scan_totals(uint32_t* __restrict__ totals, int bins) {
    __shared__ uint32_t part[1024];
    constexpr int kPer = kMaxBins / 1024;   // bins per thread
    uint32_t tot[kPer];
    uint32_t mine = 0u;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = threadIdx.x * kPer + u;
        tot[u] = b < bins ? totals[b] : 0u;
        mine += tot[u];
    }
    part[threadIdx.x] = mine;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t base = part[threadIdx.x] - mine;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = threadIdx.x * kPer + u;
        if (b < bins) totals[b] = base;
        base += tot[u];
    }
}

__global__ __launch_bounds__(64) void bin_scatter(const float* __restrict__ xyz, int n, int axis, int bins,
                                                  const BinHeader* h, const uint32_t* __restrict__ hist,
                                                  const uint32_t* __restrict__ bin_first,
                                                  int32_t* __restrict__ perm, float* __restrict__ xyz_out) {
    __shared__ uint32_t next[kMaxBins];   // next output position per bin, this chunk
    const int lane = threadIdx.x;
    for (int b = lane; b < bins; b += 64) next[b] = bin_first[b] + hist[(int64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const BinRange r = bin_range_of(h, bins);
    const int nbits = 32 - __builtin_clz((unsigned)max(bins - 1, 1));
    const uint64_t below = (1ull << lane) - 1ull;
    const int first = blockIdx.x * kBinChunk, last = min(n, first + kBinChunk);
    // The chunk's points, 16 per lane, all loads in flight together (indices
    // past the chunk read its last point and are not written).
    constexpr int kPer = kBinChunk / 64;
    float px[kPer], py[kPer], pz[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = min(first + 64 * u + lane, last - 1);
        px[u] = xyz[3 * (int64_t)j];
        py[u] = xyz[3 * (int64_t)j + 1];
        pz[u] = xyz[3 * (int64_t)j + 2];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = first + 64 * u + lane;
        const bool valid = j < last;
        const float x = axis == 0 ? px[u] : (axis == 1 ? py[u] : pz[u]);
        const int b = valid ? bin_of(x, r, bins) : 0;
        // lanes holding the same bin: agree on every bit of it
        uint64_t peers = ballot(valid);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (b >> bit) & 1;
            const uint64_t m = ballot(on);
            peers &= on ? m : ~m;
        }
        const uint32_t base = valid ? next[b] : 0u;
        if (valid && (peers & below) == 0ull) next[b] = base + (uint32_t)__popcll(peers);   // lowest lane of the bin
        if (valid) {
            const uint32_t pos = base + (uint32_t)__popcll(peers & below);
            perm[pos] = j;
            if (xyz_out) {
                xyz_out[3 * (int64_t)pos] = px[u];
                xyz_out[3 * (int64_t)pos + 1] = py[u];
                xyz_out[3 * (int64_t)pos + 2] = pz[u];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");   // this group's bin updates before the next reads
    }
}

BinKernels bin_kernels() {
    return {(const void*)&bin_reset, (const void*)&bin_range, (const void*)&bin_count,
            (const void*)&bin_scan_rows, (const void*)&bin_scan_totals, (const void*)&bin_scatter};
}

}  // namespace afps
