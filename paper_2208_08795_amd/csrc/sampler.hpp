// Device-side sector samplers for gfx950 (CDNA4, wave64).
//
// Both run the farthest-point loop of Algorithm 1 on one sector of a cloud
// (Sec. III-B: AFPS runs it on every sector at once; M = 1 is plain FPS).
//
// sample_sector (full distance update: FPS / AFPS)
//   One workgroup of W waves (T = 64*W threads), sector of n <= P*T points.
//   Point j lives in thread (j mod T), register slot (j div T): x, y, z and the
//   running distance D are VGPR arrays of P entries, loaded once (consecutive
//   threads read consecutive 12-byte points) and resident for the whole loop.
//   Per iteration every thread updates its P points, takes its lane-local max
//   (lowest slot on ties), the wave takes a DPP max and the lowest
//   (slot, lane) at that max; W > 1 waves exchange one candidate each through
//   LDS (double-buffered by iteration parity: one barrier per iteration).
//
// sample_sector_npdu (Sec. III-C: update only the window around the sample)
//   One wave, sector in LDS (x, y, z and D), cut into at most 64 chunks of
//   64*Q consecutive points; lane q keeps chunk q's maximum and the lowest
//   index reaching it.  Per iteration the wave updates the window (one lane
//   per point), re-reduces only the chunks whose recorded maximum lay inside
//   the window (distances only decrease, so no other chunk maximum can
//   change), and takes the max over the 64 chunk lanes; chunk order is index
//   order, so the lowest lane at the max holds the lowest index.
//
// Distances are kept as fp32 bit patterns: every distance is >= +0, so
// unsigned order equals float order and min / max are exact integer ops.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "variants.hpp"

#pragma clang fp contract(off)

namespace afps {

// Algorithm 1 initialises every distance to 1e10 (exact in fp32).
constexpr float kInitialDistance = 1e10f;

struct alignas(16) Candidate {
    uint32_t d;      // fp32 bits of the distance
    uint32_t idx;    // sector-local index
    float x, y, z;   // coordinates of the point
    uint32_t pad[3];
};

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ float readlane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Max / min inside each row of 16 lanes: quad xor-1, quad xor-2, half-row
// mirror, row mirror.  Every lane of a row ends with the row's value.
__device__ __forceinline__ uint32_t row_max(uint32_t v) {
    v = max(v, dpp<0xB1>(v));    // quad_perm [1,0,3,2]
    v = max(v, dpp<0x4E>(v));    // quad_perm [2,3,0,1]
    v = max(v, dpp<0x141>(v));   // row_half_mirror
    v = max(v, dpp<0x140>(v));   // row_mirror
    return v;
}
__device__ __forceinline__ uint32_t row_min(uint32_t v) {
    v = min(v, dpp<0xB1>(v));
    v = min(v, dpp<0x4E>(v));
    v = min(v, dpp<0x141>(v));
    v = min(v, dpp<0x140>(v));
    return v;
}
// Whole-wave max, returned wave-uniform.
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    v = row_max(v);
    uint32_t a = readlane(v, 0), b = readlane(v, 16), c = readlane(v, 32), d = readlane(v, 48);
    return max(max(a, b), max(c, d));
}
// Whole-wave min, returned wave-uniform.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = row_min(v);
    uint32_t a = readlane(v, 0), b = readlane(v, 16), c = readlane(v, 32), d = readlane(v, 48);
    return min(min(a, b), min(c, d));
}

__device__ __forceinline__ uint32_t sq_dist_bits(float x, float y, float z,
                                                 float px, float py, float pz) {
    const float dx = x - px;
    const float dy = y - py;
    const float dz = z - pz;
    const float xx = dx * dx;
    const float yy = dy * dy;
    const float zz = dz * dz;
    return __float_as_uint((xx + yy) + zz);
}

// Call f(std::integral_constant<int, S>) for the wave-uniform slot s in
// [LO, HI], by binary search over scalar branches, so that every register
// array access inside f has a compile-time index (a dynamic VGPR index would
// become a select chain over all slots).
template <int LO, int HI, class F>
__device__ __forceinline__ void with_slot(int s, F&& f) {
    if constexpr (LO == HI) {
        f(std::integral_constant<int, LO>{});
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (s <= MID) with_slot<LO, MID>(s, f);
        else with_slot<MID + 1, HI>(s, f);
    }
}

// Wave-uniform description of a candidate point.
struct Pick {
    uint32_t d;      // fp32 bits of its distance
    uint32_t idx;    // index (sector-local or global, as the caller defines)
    float x, y, z;
};

// Running distances of a sector, P slots per thread: in VGPRs, or (DL) in
// LDS at word s*T + t (for sectors whose four arrays exceed the register file).
template <int P, int T, bool DL>
struct Dist {
    uint32_t r[DL ? 1 : P];
    uint32_t* l;
    __device__ __forceinline__ uint32_t get(int s) const {
        if constexpr (DL) return l[s * T];
        else return r[s];
    }
    __device__ __forceinline__ void set(int s, uint32_t v) {
        if constexpr (DL) l[s * T] = v;
        else r[s] = v;
    }
};

// Load points [0, n) of a sector into the interleaved register layout.
template <int P, int T, bool DL>
__device__ __forceinline__ void load_points(const float* __restrict__ xyz, int n, int ns, int t,
                                            float (&X)[P], float (&Y)[P], float (&Z)[P],
                                            Dist<P, T, DL>& D) {
#pragma unroll
    for (int s = 0; s < P; ++s) {
        const int j = s * T + t;
        X[s] = 0.f; Y[s] = 0.f; Z[s] = 0.f;
        // Slots past the sector hold D = +0: they never beat a real point,
        // whose distance is >= +0 and whose index is lower.
        uint32_t d = 0u;
        if (s < ns && j < n) {
            X[s] = xyz[3 * j + 0];
            Y[s] = xyz[3 * j + 1];
            Z[s] = xyz[3 * j + 2];
            d = __float_as_uint(kInitialDistance);
        }
        D.set(s, d);
    }
}

// Algorithm 1 distance update of every point against (px, py, pz), then this
// wave's lowest-index maximum.  Index = slot*T + 64*w + lane.
template <int P, int T, bool DL>
__device__ __forceinline__ Pick update_and_pick(int ns, int w, int lane,
                                                const float (&X)[P], const float (&Y)[P],
                                                const float (&Z)[P], Dist<P, T, DL>& D,
                                                float px, float py, float pz) {
    uint32_t m = 0u;
    int sl = 0;
#pragma unroll
    for (int s = 0; s < P; ++s) {
        if (s < ns) {
            const uint32_t d = min(D.get(s), sq_dist_bits(X[s], Y[s], Z[s], px, py, pz));
            D.set(s, d);
            // lane-local maximum, lowest slot on ties (ascending, strict >)
            if (s == 0 || d > m) { m = d; sl = s; }
        }
    }
    Pick p;
    p.d = wave_max(m);
    const uint64_t at_max = __ballot(m == p.d);
    int l = (int)__builtin_ctzll(at_max);
    int sw = (int)readlane((uint32_t)sl, l);
    if (at_max & (at_max - 1)) {
        // several lanes at the maximum: lowest (slot, lane) pair
        const uint32_t key = (m == p.d) ? (uint32_t)(sl * 64 + lane) : 0xFFFFFFFFu;
        const uint32_t lowest = wave_min(key);
        sw = (int)(lowest >> 6);
        l = (int)(lowest & 63);
    }
    p.idx = (uint32_t)(sw * T + 64 * w + l);
    with_slot<0, P - 1>(sw, [&](auto S) {
        p.x = readlane(X[S], l);
        p.y = readlane(Y[S], l);
        p.z = readlane(Z[S], l);
    });
    return p;
}

// Combine the W waves' picks through LDS (double-buffered by `parity`, one
// barrier): the maximum distance, ties to the lowest index.  W <= 16, so all
// candidates sit in row 0 of the wave.
template <int W>
__device__ __forceinline__ Pick combine_waves(Pick mine, Candidate* lds, int parity, int w,
                                             int lane) {
    if constexpr (W == 1) {
        return mine;
    } else {
        Candidate* buf = lds + parity * W;
        if (lane == 0) {
            buf[w].d = mine.d; buf[w].idx = mine.idx;
            buf[w].x = mine.x; buf[w].y = mine.y; buf[w].z = mine.z;
        }
        __syncthreads();
        uint32_t ld = 0, li = 0xFFFFFFFFu;
        float lx = 0.f, ly = 0.f, lz = 0.f;
        if (lane < W) {
            ld = buf[lane].d; li = buf[lane].idx;
            lx = buf[lane].x; ly = buf[lane].y; lz = buf[lane].z;
        }
        const uint32_t g = readlane(row_max(ld), 0);
        const uint64_t tie = __ballot(lane < W && ld == g);
        int win = (int)__builtin_ctzll(tie);
        if (tie & (tie - 1)) {
            const uint32_t key = ((tie >> lane) & 1) ? li : 0xFFFFFFFFu;
            const uint32_t lowest = readlane(row_min(key), 0);
            win = (int)__builtin_ctzll(__ballot(key == lowest));
        }
        Pick p;
        p.d = g;
        p.idx = readlane(li, win);
        p.x = readlane(lx, win); p.y = readlane(ly, win); p.z = readlane(lz, win);
        return p;
    }
}

// Run the sampling loop of one sector (full distance update).
//   xyz   : the sector's first point (row-major fp32 x,y,z)
//   n, c  : points and samples of the sector (1 <= c <= n <= P*T)
//   cur   : local start point (0 <= cur < n)
//   base  : added to local indices on output
//   out   : c outputs
//   lds   : 2*W candidates of shared memory (unused when W == 1)
//   dl    : DL only: P*T words of shared memory for the distances
template <int P, int W, bool DL = false>
__device__ __forceinline__ void sample_sector(const float* __restrict__ xyz, int n, int c, int cur,
                                              int base, int32_t* __restrict__ out,
                                              Candidate* lds, uint32_t* dl = nullptr) {
    constexpr int T = 64 * W;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int ns = (n + T - 1) / T;   // slots holding at least one point

    float X[P], Y[P], Z[P];
    Dist<P, T, DL> D;
    if constexpr (DL) D.l = dl + t;
    load_points<P, T, DL>(xyz, n, ns, t, X, Y, Z, D);

    float px = xyz[3 * cur + 0], py = xyz[3 * cur + 1], pz = xyz[3 * cur + 2];
    if (t == 0) out[0] = base + cur;

    for (int i = 1; i < c; ++i) {
        const Pick mine = update_and_pick<P, T, DL>(ns, w, lane, X, Y, Z, D, px, py, pz);
        const Pick p = combine_waves<W>(mine, lds, i & 1, w, lane);
        cur = (int)p.idx;
        px = p.x; py = p.y; pz = p.z;
        if (t == 0) out[i] = base + cur;
    }
}

// Replace lane `lane` of `old` by the wave-uniform `v`.
__device__ __forceinline__ uint32_t writelane(uint32_t old, uint32_t v, int lane) {
    return (int)(threadIdx.x & 63) == lane ? v : old;
}

// NPDU on one sector (Sec. III-C), one wave.
//   xyz   : the sector's first point in global memory
//   n, c  : points and samples (1 <= c <= n <= 64*64*Q)
//   k     : window parameter, 0 <= k <= 2n; the window of sample `cur` is
//           [cur - floor(k/2), cur + ceil(k/2)] cut to [0, n-1]
//   cur   : local start point
//   lds   : (XYZ_IN_LDS ? 4n : n) words of shared memory: x,y,z (row-major),
//           then D
// XYZ_IN_LDS = false reads window coordinates from global memory (L2) and
// keeps only D in LDS, for sectors too large for 16 bytes per point.
template <int Q, bool XYZ_IN_LDS>
__device__ __forceinline__ void sample_sector_npdu(const float* __restrict__ xyz, int n, int c,
                                                   int k, int cur, int base,
                                                   int32_t* __restrict__ out, uint32_t* lds) {
    constexpr int CH = 64 * Q;   // points per chunk
    const int lane = threadIdx.x & 63;
    float* sxyz = reinterpret_cast<float*>(lds);
    uint32_t* sd = lds + (XYZ_IN_LDS ? 3 * n : 0);

    if constexpr (XYZ_IN_LDS) {
        const int words = 3 * n;
        int e = lane;
        for (; e + 192 < words; e += 256) {
            const float a = xyz[e], b = xyz[e + 64], cc = xyz[e + 128], d = xyz[e + 192];
            sxyz[e] = a; sxyz[e + 64] = b; sxyz[e + 128] = cc; sxyz[e + 192] = d;
        }
        for (; e < words; e += 64) sxyz[e] = xyz[e];
    }
    for (int j = lane; j < n; j += 64) sd[j] = __float_as_uint(kInitialDistance);
    __syncthreads();

    // Chunk q = points [q*CH, q*CH + CH): lane q holds its maximum and the
    // lowest index reaching it.  Initially every distance is 1e10.
    const int nq = (n + CH - 1) / CH;
    uint32_t cm = lane < nq ? __float_as_uint(kInitialDistance) : 0u;
    uint32_t ci = lane < nq ? (uint32_t)(lane * CH) : 0xFFFFFFFFu;

    auto point = [&](int j, float& x, float& y, float& z) {
        if constexpr (XYZ_IN_LDS) { x = sxyz[3 * j]; y = sxyz[3 * j + 1]; z = sxyz[3 * j + 2]; }
        else { x = xyz[3 * j]; y = xyz[3 * j + 1]; z = xyz[3 * j + 2]; }
    };
    float px, py, pz;
    point(cur, px, py, pz);
    if (lane == 0) out[0] = base + cur;

    for (int i = 1; i < c; ++i) {
        const int lo = max(0, cur - (k >> 1));
        const int hi = min(n - 1, cur + (k - (k >> 1)));
        // Window update: one lane per point.
        for (int j0 = lo; j0 <= hi; j0 += 64) {
            const int j = j0 + lane;
            if (j <= hi) {
                float x, y, z;
                point(j, x, y, z);
                sd[j] = min(sd[j], sq_dist_bits(x, y, z, px, py, pz));
            }
        }
        // Re-reduce the chunks whose recorded maximum the window lowered.
        for (int q = lo / CH; q <= hi / CH; ++q) {
            const int at = (int)readlane(ci, q);
            if (at < lo || at > hi) continue;
            uint32_t m = 0;
            int rb = 0;
            bool valid = false;
#pragma unroll
            for (int r = 0; r < Q; ++r) {
                const int j = q * CH + 64 * r + lane;
                if (j < n) {
                    const uint32_t v = sd[j];
                    if (!valid || v > m) { m = v; rb = r; valid = true; }
                }
            }
            const uint32_t g = wave_max(m);
            const uint64_t top = __ballot(valid && m == g);
            uint32_t best;
            if (Q == 1 || !(top & (top - 1))) {
                const int l = (int)__builtin_ctzll(top);
                best = (uint32_t)(q * CH + 64 * (int)readlane((uint32_t)rb, l) + l);
            } else {
                const uint32_t key = (valid && m == g) ? (uint32_t)(64 * rb + lane) : 0xFFFFFFFFu;
                best = (uint32_t)(q * CH) + wave_min(key);
            }
            cm = writelane(cm, g, q);
            ci = writelane(ci, best, q);
        }
        // Max over chunks; chunk order is index order, so the lowest lane at
        // the maximum holds the lowest index.  Lanes past the last chunk hold
        // 0 and lie above every real chunk.
        const uint32_t g = wave_max(cm);
        const int qw = (int)__builtin_ctzll(__ballot(cm == g));
        cur = (int)readlane(ci, qw);
        point(cur, px, py, pz);
        if (lane == 0) out[i] = base + cur;
    }
}

}  // namespace afps
