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
//   One wave, sector in LDS (x, y, z and D, or D only for large sectors), cut
//   into blocks of 64 points whose maxima live one per lane; per iteration
//   one LDS round trip, the window update, and a re-reduction of the window's
//   blocks only (two at a time).
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

// Points per lane whose loads are in flight together when a sampler copies
// its sector into LDS (the NPDU samplers' LR): 32 for one wave alone on its
// SIMD; fewer keep the registers small enough for more waves per SIMD.
constexpr int kLoadRound = 32;

// Algorithm 1 initialises every distance to 1e10 (exact in fp32).
constexpr float kInitialDistance = 1e10f;

struct alignas(16) Candidate {
    uint32_t d;      // fp32 bits of the distance
    uint32_t idx;    // sector-local index
    float x, y, z;   // coordinates of the point
    uint32_t pad[3];
};

// Word 3 of a gfx9 buffer resource for raw (unswizzled, stride 0) 32-bit
// loads: data format 32, everything else zero.  Out-of-range reads return 0.
constexpr int kBufferWord3 = 0x00020000;
typedef uint32_t v3u32 __attribute__((ext_vector_type(3)));

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
// DPP with a row mask: rows outside `ROWS` receive 0 (the identity of an
// unsigned max), rows inside receive the permuted value.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_rows(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}

// Whole-wave max, returned wave-uniform: row maxima, then row_bcast:15 folds
// row 0 into row 1 and row 2 into row 3, row_bcast:31 folds lane 31 into rows
// 2 and 3; lane 63 ends with the maximum of all 64 lanes.
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    v = row_max(v);
    v = max(v, dpp_rows<0x142, 0xA>(v));   // row_bcast:15 into rows 1, 3
    v = max(v, dpp_rows<0x143, 0xC>(v));   // row_bcast:31 into rows 2, 3
    return readlane(v, 63);
}
// Two independent whole-wave maxima, step by step interleaved so that each
// chain's DPP hazard wait is filled by the other chain.
__device__ __forceinline__ void wave_max2(uint32_t a, uint32_t b, uint32_t& ma, uint32_t& mb) {
    a = max(a, dpp<0xB1>(a));
    b = max(b, dpp<0xB1>(b));
    a = max(a, dpp<0x4E>(a));
    b = max(b, dpp<0x4E>(b));
    a = max(a, dpp<0x141>(a));
    b = max(b, dpp<0x141>(b));
    a = max(a, dpp<0x140>(a));
    b = max(b, dpp<0x140>(b));
    a = max(a, dpp_rows<0x142, 0xA>(a));
    b = max(b, dpp_rows<0x142, 0xA>(b));
    a = max(a, dpp_rows<0x143, 0xC>(a));
    b = max(b, dpp_rows<0x143, 0xC>(b));
    ma = readlane(a, 63);
    mb = readlane(b, 63);
}
// v_writelane_b32 (clang declares no builtin for it): `old` with lane `lane`
// (wave-uniform) replaced by the wave-uniform `value`.
extern "C" __device__ int afps_llvm_writelane(int value, int lane, int old) __asm("llvm.amdgcn.writelane");
__device__ __forceinline__ uint32_t writelane(uint32_t old, uint32_t value, int lane) {
    return (uint32_t)afps_llvm_writelane((int)value, lane, (int)old);
}

// Whole-wave min, returned wave-uniform (rows outside the mask see UINT_MAX).
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = row_min(v);
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xA, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xC, 0xF, false));
    return readlane(v, 63);
}
// Lanes where pred holds, as a wave-uniform 64-bit mask.
__device__ __forceinline__ uint64_t ballot(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }

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
    // Slots are guarded in groups of four (one scalar branch per group);
    // slots past the sector inside a live group hold D = 0 and stay 0.
    constexpr int G = P < 4 ? P : 4;
#pragma unroll
    for (int g = 0; g < P; g += G) {
        if (g == 0 || g < ns) {
#pragma unroll
            for (int s = g; s < g + G; ++s) {
                const uint32_t d = min(D.get(s), sq_dist_bits(X[s], Y[s], Z[s], px, py, pz));
                D.set(s, d);
                // lane-local maximum, lowest slot on ties (ascending, strict >)
                if (s == 0 || d > m) { m = d; sl = s; }
            }
        }
    }
    Pick p;
    p.d = wave_max(m);
    const uint64_t at_max = ballot(m == p.d);
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
        const uint64_t tie = ballot(lane < W && ld == g);
        int win = (int)__builtin_ctzll(tie);
        if (tie & (tie - 1)) {
            const uint32_t key = ((tie >> lane) & 1) ? li : 0xFFFFFFFFu;
            const uint32_t lowest = readlane(row_min(key), 0);
            win = (int)__builtin_ctzll(ballot(key == lowest));
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
    // Picks go out 64 at a time (wave 0 writes); two steps per loop trip with
    // a scalar counter, as in the NPDU loop.
    uint32_t picks = (uint32_t)cur;   // sector-local pick of step s in lane s (every wave)
    auto step = [&](int s) {
        const Pick mine = update_and_pick<P, T, DL>(ns, w, lane, X, Y, Z, D, px, py, pz);
        const Pick p = combine_waves<W>(mine, lds, s & 1, w, lane);
        cur = (int)p.idx;
        px = p.x; py = p.y; pz = p.z;
        picks = writelane(picks, (uint32_t)cur, s);
    };
    for (int i0 = 0; i0 < c; i0 += 64) {
        const int s_end = min(64, c - i0);
        int s = i0 == 0 ? 1 : 0;
        for (; s + 1 < s_end; s = __builtin_amdgcn_readfirstlane(s + 2)) {
            step(s);
            step(s + 1);
        }
        if (s < s_end) step(s);
        if (w == 0 && lane < s_end) out[i0 + lane] = (int32_t)(picks + (uint32_t)base);
    }
}


// A sector of the NPDU samplers belongs to one wave: its LDS stores need only
// have completed before its own later loads, with no workgroup barrier (other
// waves of the workgroup may be sampling other sectors).
// The lane's index, opaque to the optimiser: what a sampler derives from it
// is computed inside the sampler instead of being hoisted out of a caller's
// work loop into registers held across every sampler inlined there.
__device__ __forceinline__ int sampler_lane() {
    int l = (int)(threadIdx.x & 63);
    asm volatile("" : "+v"(l));
    return l;
}

__device__ __forceinline__ void sector_lds_ready() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
}

// NPDU on one sector (Sec. III-C) for narrow windows, one wave:
//   n <= 4096 (at most 64 blocks of 64 points: one block maximum per lane)
//   k <= 64   (the window's at most k+1 points lie in two adjacent blocks)
// Arguments as for sample_sector_npdu below; lds holds npdu_padded_points(n)
// records of 16 bytes {D bits, x, y, z}, so a point is one 128-bit LDS read.
//
// Per iteration, in issue order (one wave issues one instruction at a time,
// so the loop is written for few instructions):
//   1. read the sample's record and the two blocks holding its window;
//   2. while the reads are in flight, the maximum over the other blocks;
//   3. update the window points of the two blocks, store their D;
//   4. re-reduce both blocks (two interleaved DPP chains), write their maxima
//      and first indices into their lanes;
//   5. the overall maximum is the larger of (2) and (4); the lowest lane
//      holding it is the lowest block, whose first index is the next sample.
// Ties therefore go to the lowest index, as in Algorithm 1.
template <bool SHIFT, int LR = kLoadRound>
__device__ __forceinline__ void sample_sector_npdu_narrow(const float* __restrict__ xyz, int n, int c,
                                                          int k, int cur, int base,
                                                          int32_t* __restrict__ out, uint32_t* lds,
                                                          bool first_full, uint64_t* t_loaded) {
    const int lane = sampler_lane();
    const int nb = (n + 63) >> 6;
    const int np = npdu_padded_points(n);
    uint32_t* rec = static_cast<uint32_t*>(__builtin_assume_aligned(lds, 16));
    // Records are read as whole 16-byte copies (char-typed, so they are
    // ordered with the 32-bit D stores of earlier iterations).
    auto read = [rec](int j) {
        uint4 r;
        __builtin_memcpy(&r, rec + 4 * j, 16);
        return r;
    };
    auto write = [rec](int j, uint32_t d, float x, float y, float z) {
        const uint4 r = make_uint4(d, __float_as_uint(x), __float_as_uint(y), __float_as_uint(z));
        __builtin_memcpy(rec + 4 * j, &r, 16);
    };
    const uint32_t init = __float_as_uint(kInitialDistance);
    // Full first update (kNpduFirstFull): the distances from the start point
    // are taken while the sector loads.
    float fx = 0.f, fy = 0.f, fz = 0.f;
    if (first_full) {
        fx = xyz[3 * cur];
        fy = xyz[3 * cur + 1];
        fz = xyz[3 * cur + 2];
    }

    // Load in rounds of LR points per lane, every load of a round in
    // flight at once (the rounds are latency bound).  Indices past n read
    // point n-1; records past n are padding (D = 0, never inside a window).
    for (int j0 = 0; j0 < np; j0 += LR * 64) {
        float v[3 * LR];
#pragma unroll
        for (int u = 0; u < LR; ++u) {
            const int jj = min(j0 + 64 * u + lane, n - 1);
            v[3 * u] = xyz[3 * jj];
            v[3 * u + 1] = xyz[3 * jj + 1];
            v[3 * u + 2] = xyz[3 * jj + 2];
        }
#pragma unroll
        for (int u = 0; u < LR; ++u) {
            const int jj = j0 + 64 * u + lane;
            uint32_t d = jj < n ? init : 0u;
            if (first_full && jj < n) d = min(init, sq_dist_bits(v[3 * u], v[3 * u + 1], v[3 * u + 2], fx, fy, fz));
            if (jj < np) write(jj, d, v[3 * u], v[3 * u + 1], v[3 * u + 2]);
        }
    }
    sector_lds_ready();
    if (t_loaded) *t_loaded = __builtin_amdgcn_s_memtime();

    // Lanes past the last block hold 0: a lower lane holds a value >= 0, so
    // they never win the lowest-lane search below.  bi holds, per block, the
    // position inside the block of its lowest-index maximum.
    uint32_t bm = lane < nb ? init : 0u;
    uint32_t bi = 0u;
    const int below = k >> 1, above = k - (k >> 1);
    uint32_t* const rec_lane = rec + 4 * lane;   // this lane's record in block 0
    uint32_t picks = (uint32_t)cur;               // sector-local pick of step s in lane s
    int s_first = 1;                              // step 0 of the sector is its start
    if (first_full) {
        // Every block's maximum after the full update, then its argmax: the
        // sector's pick of step 1.
        for (int b = 0; b < nb; ++b) {
            const uint32_t d = rec_lane[256 * b];
            const uint32_t g = wave_max(d);
            bm = writelane(bm, g, b);
            bi = writelane(bi, (uint32_t)__builtin_ctzll(ballot(d == g)), b);
        }
        if (c > 1) {
            const uint32_t g = wave_max(bm);
            const int wl = (int)__builtin_ctzll(ballot(bm == g));
            cur = 64 * wl + (int)readlane(bi, wl);
            picks = writelane(picks, (uint32_t)cur, 1);
            s_first = 2;
        }
    }

    // One iteration of the loop: the new sample's record, the two blocks
    // holding its window, their update and re-reduction, the next sample.
    auto step = [&](int s) {
        const uint4 P = read(cur);
        int lo, hi;
        if constexpr (SHIFT) {   // kNpduShiftEdges: keep the window's size inside the sector
            lo = cur - below;
            hi = cur + above;
            if (lo < 0) {
                hi -= lo;
                lo = 0;
            }
            if (hi > n - 1) {
                lo = max(0, lo - (hi - (n - 1)));
                hi = n - 1;
            }
        } else {
            lo = max(0, cur - below);
            hi = min(n - 1, cur + above);
        }
        const int blo = lo >> 6;
        uint32_t* const wb = rec_lane + 256 * blo;   // this lane's record in block blo
        uint4 A, B;
        __builtin_memcpy(&A, wb, 16);
        __builtin_memcpy(&B, wb + 256, 16);

        const uint32_t g_out = wave_max((uint32_t)(lane - blo) > 1u ? bm : 0u);

        // Window: A's point is in it iff 0 <= t <= hi - lo, B's iff
        // t + 64 <= hi - lo, with t = (64 blo + lane) - lo.
        const int t = lane - (lo & 63);
        const int span = hi - lo;
        const float px = __uint_as_float(P.y), py = __uint_as_float(P.z), pz = __uint_as_float(P.w);
        const uint32_t e0 = min(A.x, sq_dist_bits(__uint_as_float(A.y), __uint_as_float(A.z),
                                                  __uint_as_float(A.w), px, py, pz));
        const uint32_t e1 = min(B.x, sq_dist_bits(__uint_as_float(B.y), __uint_as_float(B.z),
                                                  __uint_as_float(B.w), px, py, pz));
        const uint32_t d0 = (uint32_t)t <= (uint32_t)span ? e0 : A.x;
        const uint32_t d1 = t <= span - 64 ? e1 : B.x;
        wb[0] = d0;
        wb[256] = d1;

        uint32_t g0, g1;
        wave_max2(d0, d1, g0, g1);
        const uint32_t i0 = (uint32_t)__builtin_ctzll(ballot(d0 == g0));
        const uint32_t i1 = (uint32_t)__builtin_ctzll(ballot(d1 == g1));
        // Block blo+1 may be the padding block (g1 = 0) or, for n = 4096,
        // lane 64, which does not exist: then it goes to lane 63 first and
        // block blo = 63 overwrites it.
        const int l1 = min(blo + 1, 63);
        bm = writelane(bm, g1, l1);
        bi = writelane(bi, i1, l1);
        bm = writelane(bm, g0, blo);
        bi = writelane(bi, i0, blo);

        const uint32_t g = max(g_out, max(g0, g1));
        const int wl = (int)__builtin_ctzll(ballot(bm == g));
        cur = 64 * wl + (int)readlane(bi, wl);
        picks = writelane(picks, (uint32_t)cur, s);
    };

    // Picks go out 64 at a time.  The loop is bound by instruction issue
    // (one wave): two steps per trip, and a loop counter kept scalar, save
    // the counter and branch work of every other step.
    for (int i0 = 0; i0 < c; i0 += 64) {
        const int s_end = min(64, c - i0);
        int s = i0 == 0 ? s_first : 0;
        for (; s + 1 < s_end; s = __builtin_amdgcn_readfirstlane(s + 2)) {
            step(s);
            step(s + 1);
        }
        if (s < s_end) step(s);
        if (lane < s_end) out[i0 + lane] = (int32_t)(picks + (uint32_t)base);
    }
}

// NPDU on one sector for narrow windows with the coordinates read from
// global memory (L2) and only D in LDS (npdu_lds_words(n, false) words):
//   n <= 4096, k <= 64.
// The loop of sample_sector_npdu_narrow with its three LDS record reads
// replaced by loads through a buffer resource bounded to the sector (points
// past it read as zeros): the sample's 12 bytes (one wave-uniform load) and
// the window's.  With WIN (windows of at most 64 points, k <= 63) lane l
// holds point lo + l: one 12-byte load per lane, the update of D written to
// LDS and the two blocks holding the window read back for their maxima; else
// (k = 64) the two blocks are loaded and updated in place, 128 lanes for at
// most 65 points.  The memory round trip is on every iteration's path, which
// many waves per SIMD hide; the sector takes a quarter of the LDS of 16-byte
// records.
template <bool SHIFT, bool WIN>
__device__ __forceinline__ void sample_sector_npdu_narrow_l2(const float* __restrict__ xyz, int n, int c, int k,
                                                             int cur, int base, int32_t* __restrict__ out,
                                                             uint32_t* lds, bool first_full, uint64_t* t_loaded) {
    const int lane = sampler_lane();
    const int nb = (n + 63) >> 6;
    const int np = npdu_padded_points(n);
    uint32_t* const rec = static_cast<uint32_t*>(__builtin_assume_aligned(lds, 16));
    const __amdgpu_buffer_rsrc_t xyz_rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(xyz), (short)0, 12 * n, kBufferWord3);
    const int lane12 = 12 * lane;
    const uint32_t init = __float_as_uint(kInitialDistance);
    // D of every point: the start point's distance for the full first
    // update (coordinates read once here), else 1e10; padding 0.
    float fx = 0.f, fy = 0.f, fz = 0.f;
    if (first_full) {
        fx = xyz[3 * cur];
        fy = xyz[3 * cur + 1];
        fz = xyz[3 * cur + 2];
    }
    for (int j = lane; j < np; j += 64) {
        uint32_t d = j < n ? init : 0u;
        if (first_full && j < n) d = min(init, sq_dist_bits(xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2], fx, fy, fz));
        rec[j] = d;
    }
    sector_lds_ready();
    if (t_loaded) *t_loaded = __builtin_amdgcn_s_memtime();

    uint32_t bm = lane < nb ? init : 0u;
    uint32_t bi = 0u;
    const int below = k >> 1, above = k - (k >> 1);
    uint32_t* const rec_lane = rec + lane;
    uint32_t picks = (uint32_t)cur;
    int s_first = 1;
    if (first_full) {
        for (int b = 0; b < nb; ++b) {
            const uint32_t d = rec_lane[64 * b];
            const uint32_t g = wave_max(d);
            bm = writelane(bm, g, b);
            bi = writelane(bi, (uint32_t)__builtin_ctzll(ballot(d == g)), b);
        }
        if (c > 1) {
            const uint32_t g = wave_max(bm);
            const int wl = (int)__builtin_ctzll(ballot(bm == g));
            cur = 64 * wl + (int)readlane(bi, wl);
            picks = writelane(picks, (uint32_t)cur, 1);
            s_first = 2;
        }
    }

    auto step = [&](int s) {
        // the sample's coordinates: scalar loads (the points are read-only
        // while the kernel runs, so the constant address space holds)
        typedef const __attribute__((address_space(4))) float* ConstPtr;
        typedef const __attribute__((address_space(4))) char* ConstBytes;
        const ConstPtr p = (ConstPtr)((ConstBytes)xyz + (uint32_t)(12 * cur));   // a 32-bit byte offset
        const float px = p[0], py = p[1], pz = p[2];
        int lo, hi;
        if constexpr (SHIFT) {   // kNpduShiftEdges: keep the window's size inside the sector
            lo = cur - below;
            hi = cur + above;
            if (lo < 0) {
                hi -= lo;
                lo = 0;
            }
            if (hi > n - 1) {
                lo = max(0, lo - (hi - (n - 1)));
                hi = n - 1;
            }
        } else {
            lo = max(0, cur - below);
            hi = min(n - 1, cur + above);
        }
        const int blo = lo >> 6;
        const int span = hi - lo;
        uint32_t* const wb = rec_lane + 64 * blo;
        uint32_t d0, d1, g_out;
        if constexpr (WIN) {
            // The window's own 64 lanes (point lo + lane; the window ends at
            // lane span <= 63): one load, one update, written to LDS, and the
            // two blocks holding it read back for their maxima.
            const v3u32 P = __builtin_amdgcn_raw_buffer_load_b96(xyz_rsrc, 12 * lo + lane12, 0, 0);
            uint32_t* const ww = rec_lane + lo;
            const uint32_t dw = ww[0];
            g_out = wave_max((uint32_t)(lane - blo) > 1u ? bm : 0u);
            const uint32_t ew = min(dw, sq_dist_bits(__uint_as_float(P.x), __uint_as_float(P.y),
                                                     __uint_as_float(P.z), px, py, pz));
            ww[0] = lane <= span ? ew : dw;
            d0 = wb[0];
            d1 = wb[64];
        } else {
            const int off = 768 * blo + lane12;   // block blo + 1 at 768 bytes further
            const v3u32 A = __builtin_amdgcn_raw_buffer_load_b96(xyz_rsrc, off, 0, 0);
            const v3u32 B = __builtin_amdgcn_raw_buffer_load_b96(xyz_rsrc, off + 768, 0, 0);
            const uint32_t da = wb[0], db = wb[64];

            g_out = wave_max((uint32_t)(lane - blo) > 1u ? bm : 0u);

            const int t = lane - (lo & 63);
            const uint32_t e0 = min(da, sq_dist_bits(__uint_as_float(A.x), __uint_as_float(A.y),
                                                     __uint_as_float(A.z), px, py, pz));
            const uint32_t e1 = min(db, sq_dist_bits(__uint_as_float(B.x), __uint_as_float(B.y),
                                                     __uint_as_float(B.z), px, py, pz));
            d0 = (uint32_t)t <= (uint32_t)span ? e0 : da;
            d1 = t <= span - 64 ? e1 : db;
            wb[0] = d0;
            wb[64] = d1;
        }

        uint32_t g0, g1;
        wave_max2(d0, d1, g0, g1);
        const uint32_t i0 = (uint32_t)__builtin_ctzll(ballot(d0 == g0));
        const uint32_t i1 = (uint32_t)__builtin_ctzll(ballot(d1 == g1));
        // Block blo+1 may be the padding block (g1 = 0) or, for n = 4096,
        // lane 64, which does not exist: then it goes to lane 63 first and
        // block blo = 63 overwrites it.
        const int l1 = min(blo + 1, 63);
        bm = writelane(bm, g1, l1);
        bi = writelane(bi, i1, l1);
        bm = writelane(bm, g0, blo);
        bi = writelane(bi, i0, blo);

        const uint32_t g = max(g_out, max(g0, g1));
        const int wl = (int)__builtin_ctzll(ballot(bm == g));
        cur = 64 * wl + (int)readlane(bi, wl);
        picks = writelane(picks, (uint32_t)cur, s);
    };

    for (int i0 = 0; i0 < c; i0 += 64) {
        const int s_end = min(64, c - i0);
        int s = i0 == 0 ? s_first : 0;
        for (; s + 1 < s_end; s = __builtin_amdgcn_readfirstlane(s + 2)) {
            step(s);
            step(s + 1);
        }
        if (s < s_end) step(s);
        if (lane < s_end) out[i0 + lane] = (int32_t)(picks + (uint32_t)base);
    }
}

// NPDU on one sector for narrow windows with the sector's coordinates held in
// vector registers instead of LDS:
//   n <= 4096 (at most 64 blocks of 64 points), k <= 64.
// Block b's coordinates sit in lane l (point 64 b + l) of element b >> 1 of
// the even (b even) or the odd (b odd) register set: three vectors of 32
// registers each, 192 VGPRs in all.  A wave-uniform element index reaches a
// vector by relative register addressing (one index per set), and the two
// adjacent blocks holding a window are always one even and one odd block.
// LDS holds only D (npdu_lds_words(n, false) words), so a CU holds as many
// of these sectors as it has waves, where 16-byte records in LDS would fit two
// of 4096 points into its 160 KB.  The iteration is that of
// sample_sector_npdu_narrow; the sample's coordinates come from the window
// block holding it by a lane read.  Needs about 220 VGPRs: at most two waves
// per SIMD.
typedef float f32x32 __attribute__((ext_vector_type(32)));

template <bool SHIFT>
__device__ __forceinline__ void sample_sector_npdu_regs(const float* __restrict__ xyz, int n, int c, int k,
                                                        int cur, int base, int32_t* __restrict__ out,
                                                        uint32_t* lds, bool first_full, uint64_t* t_loaded) {
    const int lane = sampler_lane();
    const int nb = (n + 63) >> 6;
    uint32_t* const rec = static_cast<uint32_t*>(__builtin_assume_aligned(lds, 16));
    // Loads through a buffer resource bounded to the sector's 12 n bytes:
    // points past the sector read as zeros.
    const __amdgpu_buffer_rsrc_t xyz_rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(xyz), (short)0, 12 * n, kBufferWord3);
    const int lane12 = 12 * lane;
    const uint32_t init = __float_as_uint(kInitialDistance);
    float fx = 0.f, fy = 0.f, fz = 0.f;   // start point, for the full first update
    if (first_full) {
        fx = xyz[3 * cur];
        fy = xyz[3 * cur + 1];
        fz = xyz[3 * cur + 2];
    }

    // Load eight blocks per test of the block count, every load of the
    // sector in flight at once.  Groups up to the one holding block nb (the
    // padding block, read as zeros) are loaded, so every element a window
    // can reach is defined.
    f32x32 xe, ye, ze, xo, yo, zo;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        if (8 * g <= nb) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = 8 * g + u;
                const v3u32 v = __builtin_amdgcn_raw_buffer_load_b96(xyz_rsrc, 768 * b + lane12, 0, 0);
                if (b & 1) {
                    xo[b >> 1] = __uint_as_float(v.x);
                    yo[b >> 1] = __uint_as_float(v.y);
                    zo[b >> 1] = __uint_as_float(v.z);
                } else {
                    xe[b >> 1] = __uint_as_float(v.x);
                    ye[b >> 1] = __uint_as_float(v.y);
                    ze[b >> 1] = __uint_as_float(v.z);
                }
            }
        }
    }
    // D of every point (the start point's distance for the full first
    // update, else 1e10) and of the padding block (0, never in a window).
    for (int b = 0; b <= nb; b = __builtin_amdgcn_readfirstlane(b + 1)) {
        const int j = 64 * b + lane;
        uint32_t d = j < n ? init : 0u;
        if (first_full && j < n) {
            const int i = b >> 1;   // b < nb <= 64 here
            const bool odd = (b & 1) != 0;
            d = min(init, sq_dist_bits(odd ? xo[i] : xe[i], odd ? yo[i] : ye[i], odd ? zo[i] : ze[i], fx, fy, fz));
        }
        rec[j] = d;
    }
    sector_lds_ready();
    if (t_loaded) *t_loaded = __builtin_amdgcn_s_memtime();

    uint32_t bm = lane < nb ? init : 0u;   // block maxima (0 past the last block)
    uint32_t bi = 0u;                      // position of each block's lowest-index maximum
    const int below = k >> 1, above = k - (k >> 1);
    uint32_t* const rec_lane = rec + lane;
    uint32_t picks = (uint32_t)cur;
    int s_first = 1;
    if (first_full) {
        for (int b = 0; b < nb; ++b) {
            const uint32_t d = rec_lane[64 * b];
            const uint32_t g = wave_max(d);
            bm = writelane(bm, g, b);
            bi = writelane(bi, (uint32_t)__builtin_ctzll(ballot(d == g)), b);
        }
        if (c > 1) {
            const uint32_t g = wave_max(bm);
            const int wl = (int)__builtin_ctzll(ballot(bm == g));
            cur = 64 * wl + (int)readlane(bi, wl);
            picks = writelane(picks, (uint32_t)cur, 1);
            s_first = 2;
        }
    }

    auto step = [&](int s) {
        int lo, hi;
        if constexpr (SHIFT) {   // kNpduShiftEdges: keep the window's size inside the sector
            lo = cur - below;
            hi = cur + above;
            if (lo < 0) {
                hi -= lo;
                lo = 0;
            }
            if (hi > n - 1) {
                lo = max(0, lo - (hi - (n - 1)));
                hi = n - 1;
            }
        } else {
            lo = max(0, cur - below);
            hi = min(n - 1, cur + above);
        }
        // The window lies in blocks blo and blo + 1: the odd one is 2h + 1,
        // the even one 2e.  For blo = 63 the second would be the padding block
        // 64, which holds no registers; block 62 (outside the window, so
        // re-reduced unchanged) takes its place.
        const int blo = lo >> 6;
        const int h = blo >> 1;
        const int e = min(h + (blo & 1), 31);
        const float ox = xo[h], oy = yo[h], oz = zo[h];
        const float ex = xe[e], ey = ye[e], ez = ze[e];
        const int lb = min(blo, 62);                 // the lower of the two blocks held
        uint32_t* const wb = rec_lane + 64 * lb;
        const uint32_t dl = wb[0], dh = wb[64];
        const bool lodd = (lb & 1) != 0;             // the lower block is the odd one
        const uint32_t de = lodd ? dh : dl, dod = lodd ? dl : dh;

        const uint32_t g_out = wave_max((uint32_t)(lane - lb) > 1u ? bm : 0u);

        // the sample: lane cur & 63 of whichever window block holds it
        const bool codd = ((cur >> 6) & 1) != 0;
        const int cl = cur & 63;
        const float px = readlane(codd ? ox : ex, cl);
        const float py = readlane(codd ? oy : ey, cl);
        const float pz = readlane(codd ? oz : ez, cl);

        const int span = hi - lo;
        const uint32_t fe = min(de, sq_dist_bits(ex, ey, ez, px, py, pz));
        const uint32_t fo = min(dod, sq_dist_bits(ox, oy, oz, px, py, pz));
        const uint32_t ne = (uint32_t)(128 * e + lane - lo) <= (uint32_t)span ? fe : de;
        const uint32_t no = (uint32_t)(128 * h + 64 + lane - lo) <= (uint32_t)span ? fo : dod;
        wb[0] = lodd ? no : ne;
        wb[64] = lodd ? ne : no;

        uint32_t ge, go;
        wave_max2(ne, no, ge, go);
        const uint32_t ie = (uint32_t)__builtin_ctzll(ballot(ne == ge));
        const uint32_t io = (uint32_t)__builtin_ctzll(ballot(no == go));
        bm = writelane(bm, ge, 2 * e);
        bi = writelane(bi, ie, 2 * e);
        bm = writelane(bm, go, 2 * h + 1);
        bi = writelane(bi, io, 2 * h + 1);

        const uint32_t g = max(g_out, max(ge, go));
        const int wl = (int)__builtin_ctzll(ballot(bm == g));
        cur = 64 * wl + (int)readlane(bi, wl);
        picks = writelane(picks, (uint32_t)cur, s);
    };

    for (int i0 = 0; i0 < c; i0 += 64) {
        const int s_end = min(64, c - i0);
        int s = i0 == 0 ? s_first : 0;
        for (; s + 1 < s_end; s = __builtin_amdgcn_readfirstlane(s + 2)) {
            step(s);
            step(s + 1);
        }
        if (s < s_end) step(s);
        if (lane < s_end) out[i0 + lane] = (int32_t)(picks + (uint32_t)base);
    }
}

// NPDU on sectors of up to 4096 R points, any window: the loop of
// sample_sector_npdu_narrow with R registers of block maxima (block 64 r + l
// in lane l of register r; a window block's maximum goes in by a lane select
// in every register and the block holding the new maximum is found by halving
// the register set, so every register index is a constant), the window's
// blocks re-reduced two at a time, and, for sectors too large for 16 bytes per point
// of LDS (XYZ_IN_LDS = false), only D in LDS and the coordinates read from
// global memory (L2).
template <int R, bool XYZ_IN_LDS, bool SHIFT, int LR = kLoadRound>
__device__ __forceinline__ void sample_sector_npdu_blocks(const float* __restrict__ xyz, int n, int c,
                                                          int k, int cur, int base,
                                                          int32_t* __restrict__ out, uint32_t* lds,
                                                          bool first_full, uint64_t* t_loaded) {
    static_assert(R >= 1 && R <= 8 && (R & (R - 1)) == 0, "R is 1, 2, 4 or 8 block registers");
    // Coordinates read from global memory (XYZ_IN_LDS = false) go through a
    // buffer resource bounded to the sector's 12 n bytes: a block's two loads
    // take one offset add on the fixed per-lane 12 lane, and a point past the
    // sector (in the padding block) reads as zeros instead of needing a clamp.
    // The whole offset is in the vector offset and the immediate, both covered
    // by the range check; a 12-byte record is either wholly inside or outside.
    const __amdgpu_buffer_rsrc_t xyz_rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(xyz), (short)0, 12 * n, kBufferWord3);
    const int lane = sampler_lane();
    const int lane12 = 12 * lane;
    constexpr int kWords = XYZ_IN_LDS ? 4 : 1;   // LDS words per point: {D, x, y, z} or D
    const int nb = (n + 63) >> 6;
    const int np = npdu_padded_points(n);
    uint32_t* rec = static_cast<uint32_t*>(__builtin_assume_aligned(lds, 16));
    const uint32_t init = __float_as_uint(kInitialDistance);
    float fx = 0.f, fy = 0.f, fz = 0.f;   // start point, for the full first update
    if (first_full) {
        fx = xyz[3 * cur];
        fy = xyz[3 * cur + 1];
        fz = xyz[3 * cur + 2];
    }

    // Load: rounds of LR points per lane with every load in flight
    // (coordinates are needed in LDS, or for the full first update).
    if (XYZ_IN_LDS || first_full) {
        for (int j0 = 0; j0 < np; j0 += LR * 64) {
            float v[3 * LR];
#pragma unroll
            for (int u = 0; u < LR; ++u) {
                const int jj = min(j0 + 64 * u + lane, n - 1);
                v[3 * u] = xyz[3 * jj];
                v[3 * u + 1] = xyz[3 * jj + 1];
                v[3 * u + 2] = xyz[3 * jj + 2];
            }
#pragma unroll
            for (int u = 0; u < LR; ++u) {
                const int jj = j0 + 64 * u + lane;
                uint32_t d = jj < n ? init : 0u;
                if (first_full && jj < n) d = min(init, sq_dist_bits(v[3 * u], v[3 * u + 1], v[3 * u + 2], fx, fy, fz));
                if (jj < np) {
                    if constexpr (XYZ_IN_LDS) {
                        const uint4 r4 = make_uint4(d, __float_as_uint(v[3 * u]), __float_as_uint(v[3 * u + 1]),
                                                    __float_as_uint(v[3 * u + 2]));
                        __builtin_memcpy(rec + 4 * jj, &r4, 16);
                    } else {
                        rec[jj] = d;
                    }
                }
            }
        }
    } else {
        for (int j = lane; j < np; j += 64) rec[j] = j < n ? init : 0u;
    }
    sector_lds_ready();
    if (t_loaded) *t_loaded = __builtin_amdgcn_s_memtime();

    uint32_t bm[R], bi[R];   // block maxima and their positions inside the block
#pragma unroll
    for (int r = 0; r < R; ++r) {
        bm[r] = 64 * r + lane < nb ? init : 0u;
        bi[r] = 0u;
    }
    auto set_block = [&](int blk, uint32_t g, uint32_t i) {
        with_slot<0, R - 1>(blk >> 6, [&](auto r) {
            bm[r] = writelane(bm[r], g, blk & 63);
            bi[r] = writelane(bi[r], i, blk & 63);
        });
    };
    // Blocks b0 and b0 + 1 (the latter dropped when past the registers)
    // take maxima g0, g1 and first positions i0, i1: in every register, the
    // lanes of the two blocks select the new values; no branch, no lane
    // write, so the register of a block need not be known.
    auto set_pair = [&](int b0, uint32_t g0, uint32_t i0, uint32_t g1, uint32_t i1) {
        const bool first = lane == (b0 & 63);
        const uint32_t gs = first ? g0 : g1, is = first ? i0 : i1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool mine = (uint32_t)(64 * r + lane - b0) < 2u;
            bm[r] = mine ? gs : bm[r];
            bi[r] = mine ? is : bi[r];
        }
    };
    // The lowest index holding distance g: the lowest block, then its position.
    // All R ballots are taken at once; the lowest register with a hit is found
    // by halving the register set with uniform selects, so one readlane fetches
    // the position (a branch per register measured 6-14% slower per iteration
    // at R >= 2).  At R = 4 the two halvings are written out: the loop form
    // compiles to a switch over the chosen register there.
    auto lowest_with = [&](uint32_t g) {
        if constexpr (R == 4) {
            const uint64_t h0 = ballot(bm[0] == g), h1 = ballot(bm[1] == g);
            const uint64_t h2 = ballot(bm[2] == g), h3 = ballot(bm[3] == g);
            const bool low = (h0 | h1) != 0;
            const uint64_t ha = low ? h0 : h2, hb = low ? h1 : h3;
            const uint32_t va = low ? bi[0] : bi[2], vb = low ? bi[1] : bi[3];
            const bool in_a = ha != 0;
            const uint32_t v = in_a ? va : vb;
            const int l = (int)__builtin_ctzll(in_a ? ha : (hb | (1ull << 63)));
            const int r = (low ? 0 : 2) + (in_a ? 0 : 1);
            return 64 * (64 * r + l) + (int)readlane(v, l);
        } else {
            uint64_t h[R];
            uint32_t v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                h[r] = ballot(bm[r] == g);
                v[r] = bi[r];
            }
            int r0 = 0;
#pragma unroll
            for (int len = R; len > 1; len >>= 1) {
                const int half = len >> 1;
                uint64_t any = 0;
#pragma unroll
                for (int r = 0; r < half; ++r) any |= h[r];
                const bool low = any != 0;
#pragma unroll
                for (int r = 0; r < half; ++r) {
                    h[r] = low ? h[r] : h[r + half];
                    v[r] = low ? v[r] : v[r + half];
                }
                r0 += low ? 0 : half;
            }
            // g is one of the block maxima, so h[0] has a bit set; bit 63 only
            // keeps the count defined.
            const int l = (int)__builtin_ctzll(h[0] | (1ull << 63));
            return 64 * (64 * r0 + l) + (int)readlane(v[0], l);
        }
    };
    const int below = k >> 1, above = k - (k >> 1);
    uint32_t picks = (uint32_t)cur;   // sector-local pick of step s in lane s
    int s_first = 1;
    if (first_full) {
        for (int b = 0; b < nb; ++b) {
            const uint32_t d = rec[kWords * (64 * b + lane)];
            const uint32_t g = wave_max(d);
            set_block(b, g, (uint32_t)__builtin_ctzll(ballot(d == g)));
        }
        if (c > 1) {
            uint32_t mx = 0u;
#pragma unroll
            for (int r = 0; r < R; ++r) mx = max(mx, bm[r]);
            cur = lowest_with(wave_max(mx));
            picks = writelane(picks, (uint32_t)cur, 1);
            s_first = 2;
        }
    }

    // The maxima of blocks b0, b0 + 1 holding d0, d1, recorded; returns the
    // larger.  Block b0+1 may be the padding block (maximum 0, never the
    // lowest holder of a maximum); past the registers it is not recorded.
    auto reduce_pair = [&](int b0, uint32_t d0, uint32_t d1) {
        uint32_t g0, g1;
        wave_max2(d0, d1, g0, g1);
        const uint32_t i0 = (uint32_t)__builtin_ctzll(ballot(d0 == g0));
        const uint32_t i1 = (uint32_t)__builtin_ctzll(ballot(d1 == g1));
        set_pair(b0, g0, i0, g1, i1);
        return max(g0, g1);
    };

    // Update and re-reduce the two blocks b0, b0 + 1 (window points [lo, hi]
    // only); returns the larger block maximum.
    auto update_pair = [&](int b0, int lo, int span, float px, float py, float pz) {
        const int j0 = 64 * b0 + lane, j1 = j0 + 64;
        uint32_t a_d, b_d;
        float ax, ay, az, bx, by, bz;
        if constexpr (XYZ_IN_LDS) {
            uint4 A, B;
            __builtin_memcpy(&A, rec + 4 * j0, 16);
            __builtin_memcpy(&B, rec + 4 * j1, 16);
            a_d = A.x; ax = __uint_as_float(A.y); ay = __uint_as_float(A.z); az = __uint_as_float(A.w);
            b_d = B.x; bx = __uint_as_float(B.y); by = __uint_as_float(B.z); bz = __uint_as_float(B.w);
        } else {
            a_d = rec[j0];
            b_d = rec[j1];
            // block b0 + 1 at immediate offset +768 bytes; padding points read zeros
            const int off = 768 * b0 + lane12;
            const v3u32 A = __builtin_amdgcn_raw_buffer_load_b96(xyz_rsrc, off, 0, 0);
            const v3u32 B = __builtin_amdgcn_raw_buffer_load_b96(xyz_rsrc, off + 768, 0, 0);
            ax = __uint_as_float(A.x); ay = __uint_as_float(A.y); az = __uint_as_float(A.z);
            bx = __uint_as_float(B.x); by = __uint_as_float(B.y); bz = __uint_as_float(B.z);
        }
        const uint32_t e0 = min(a_d, sq_dist_bits(ax, ay, az, px, py, pz));
        const uint32_t e1 = min(b_d, sq_dist_bits(bx, by, bz, px, py, pz));
        const uint32_t d0 = (uint32_t)(j0 - lo) <= (uint32_t)span ? e0 : a_d;
        const uint32_t d1 = (uint32_t)(j1 - lo) <= (uint32_t)span ? e1 : b_d;
        rec[kWords * j0] = d0;
        rec[kWords * j1] = d1;
        return reduce_pair(b0, d0, d1);
    };
    // Coordinates from L2 and a window of at most 64 points (k <= 63) in
    // blocks b0, b0 + 1 with b0 = lo >> 6: lane l takes point lo + l (one
    // load, one update, written to LDS) and the two blocks are read back.
    auto update_window = [&](int b0, int lo, int span, float px, float py, float pz) {
        const v3u32 P = __builtin_amdgcn_raw_buffer_load_b96(xyz_rsrc, 12 * lo + lane12, 0, 0);
        uint32_t* const ww = rec + lo + lane;   // inside the padded sector: lo + 63 < n + 64
        const uint32_t dw = ww[0];
        const uint32_t ew = min(dw, sq_dist_bits(__uint_as_float(P.x), __uint_as_float(P.y), __uint_as_float(P.z),
                                                 px, py, pz));
        ww[0] = lane <= span ? ew : dw;
        const int j0 = 64 * b0 + lane;
        return reduce_pair(b0, rec[j0], rec[j0 + 64]);
    };

    // One iteration; NARROW (k <= 64: the window lies in two adjacent blocks)
    // fixes the number of block pairs at one; its value 2 (coordinates from
    // L2, k <= 63) updates the window's own 64 lanes.
    auto step = [&](int s, auto narrow) {
        float px, py, pz;
        if constexpr (XYZ_IN_LDS) {
            px = __uint_as_float(rec[4 * cur + 1]);
            py = __uint_as_float(rec[4 * cur + 2]);
            pz = __uint_as_float(rec[4 * cur + 3]);
        } else {
            // scalar loads at a 32-bit byte offset (the points are read-only
            // while the kernel runs, so the constant address space holds)
            typedef const __attribute__((address_space(4))) float* ConstPtr;
            typedef const __attribute__((address_space(4))) char* ConstBytes;
            const ConstPtr p = (ConstPtr)((ConstBytes)xyz + (uint32_t)(12 * cur));
            px = p[0];
            py = p[1];
            pz = p[2];
        }
        int lo, hi;
        if constexpr (SHIFT) {   // kNpduShiftEdges: keep the window's size inside the sector
            lo = cur - below;
            hi = cur + above;
            if (lo < 0) {
                hi -= lo;
                lo = 0;
            }
            if (hi > n - 1) {
                lo = max(0, lo - (hi - (n - 1)));
                hi = n - 1;
            }
        } else {
            lo = max(0, cur - below);
            hi = min(n - 1, cur + above);
        }
        const int blo = lo >> 6;
        // the window's blocks [blo, hi >> 6], re-reduced in pairs
        const int pairs = decltype(narrow)::value ? 1 : ((hi >> 6) - blo + 2) >> 1;

        uint32_t mo = 0u;   // best of the blocks outside the re-reduced pairs
#pragma unroll
        for (int r = 0; r < R; ++r) mo = max(mo, (uint32_t)(64 * r + lane - blo) >= (uint32_t)(2 * pairs) ? bm[r] : 0u);
        uint32_t best = wave_max(mo);
        if constexpr (decltype(narrow)::value == 2)
            best = max(best, update_window(blo, lo, hi - lo, px, py, pz));
        else
            best = max(best, update_pair(blo, lo, hi - lo, px, py, pz));
        if constexpr (!decltype(narrow)::value)
            for (int p = 1; p < pairs; ++p) best = max(best, update_pair(blo + 2 * p, lo, hi - lo, px, py, pz));
        cur = lowest_with(best);
        picks = writelane(picks, (uint32_t)cur, s);
    };

    auto run = [&](auto narrow) {
        for (int i0 = 0; i0 < c; i0 += 64) {
            const int s_end = min(64, c - i0);
            int s = i0 == 0 ? s_first : 0;
            for (; s + 1 < s_end; s = __builtin_amdgcn_readfirstlane(s + 2)) {
                step(s, narrow);
                step(s + 1, narrow);
            }
            if (s < s_end) step(s, narrow);
            if (lane < s_end) out[i0 + lane] = (int32_t)(picks + (uint32_t)base);
        }
    };
    if constexpr (!XYZ_IN_LDS) {
        if (k <= 63) {
            run(std::integral_constant<int, 2>{});
            return;
        }
    }
    if (k <= 64) run(std::integral_constant<int, 1>{});
    else run(std::integral_constant<int, 0>{});
}

// NPDU on one sector (Sec. III-C), one wave.
//   xyz   : the sector's first point in global memory
//   n, c  : points and samples (1 <= c <= n <= 4096*R)
//   k     : window parameter, 0 <= k <= 2n; the window of sample `cur` is
//           [cur - floor(k/2), cur + ceil(k/2)] cut to [0, n-1] (or moved
//           inside it, kNpduShiftEdges)
//   cur   : local start point
//   lds   : npdu_lds_words(n, XYZ_IN_LDS) words of shared memory
//   flags : kNpduFirstFull, kNpduShiftEdges
//   t_loaded: if not null, receives the shader clock once the sector is in LDS
// The sector is cut into blocks of 64 consecutive points whose maxima (and
// the lowest index reaching them) live one block per lane.  Distances only
// decrease and only inside the window, so every other block keeps its
// maximum; per iteration the wave re-reduces the window's blocks and takes the
// lowest block holding the overall maximum.  LDS is padded with one empty
// block (D = 0, never a window point), so block reads need no bounds test.
// XYZ_IN_LDS = false reads coordinates from global memory (L2) and keeps only
// D in LDS, for sectors too large for 16 bytes per point.
template <int R, bool XYZ_IN_LDS, int LR = kLoadRound>
__device__ __forceinline__ void sample_sector_npdu(const float* __restrict__ xyz, int n, int c,
                                                   int k, int cur, int base,
                                                   int32_t* __restrict__ out, uint32_t* lds,
                                                   int flags, uint64_t* t_loaded = nullptr) {
    const bool first_full = (flags & kNpduFirstFull) != 0;
    const bool shift = (flags & kNpduShiftEdges) != 0;
    if constexpr (R == 1 && XYZ_IN_LDS) {
        if (k <= 64) {   // the window lies in two adjacent blocks
            if (shift) sample_sector_npdu_narrow<true, LR>(xyz, n, c, k, cur, base, out, lds, first_full, t_loaded);
            else sample_sector_npdu_narrow<false, LR>(xyz, n, c, k, cur, base, out, lds, first_full, t_loaded);
            return;
        }
    }
    if (shift)
        sample_sector_npdu_blocks<R, XYZ_IN_LDS, true, LR>(xyz, n, c, k, cur, base, out, lds, first_full, t_loaded);
    else
        sample_sector_npdu_blocks<R, XYZ_IN_LDS, false, LR>(xyz, n, c, k, cur, base, out, lds, first_full, t_loaded);
}

}  // namespace afps
