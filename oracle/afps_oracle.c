/*
 * CPU oracle for farthest point sampling (FPS), adjustable FPS (AFPS) and
 * nearest-point distance updating (NPDU) -- Li et al., "An Adjustable Farthest
 * Point Sampling Method for Approximately-sorted Point Cloud Data" -- and for
 * the grouping around the samples (ball query, at the end of this file).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  The GPU library
 * never links, calls or includes it, and it shares no code with the GPU path.
 *
 * The method is a heuristic (it does not reach the plain-FPS result by another
 * route), so this oracle takes the steps of the method in the paper's order:
 * plain FPS as Algorithm 1 defines it, the storage sectors of Sec. III-B, the
 * neighbourhood refresh of Sec. III-C.  It is deliberately slow and
 * unblocked: one sector after the other, one point after the other, a full
 * sequential scan for the farthest point after every pick.
 *
 * Readings of points the paper leaves open (each is used identically by the
 * GPU path; the numbering follows the design notes):
 *   - distance: squared Euclidean in fp32, ((dx*dx + dy*dy) + dz*dz) with
 *     dx = P[j].x - P[cur].x, every operation rounded to nearest, no fused
 *     multiply-add (the paper names a Euclidean distance; the farthest point
 *     does not change under sqrt, and skipping sqrt adds no rounding ties);
 *   - every running distance starts at 1e10, as in the paper, exact in fp32;
 *   - ties for the farthest point go to the lowest index (a sequential scan
 *     with strict '>');
 *   - start: sector s starts at its local point (start mod n_s);
 *   - sectors are contiguous storage ranges: the first N mod M sectors hold one
 *     extra point, the first C mod M sectors take one extra sample (Sec. III-B:
 *     C/M iterations per sector);
 *   - NPDU neighbourhood: the new sample plus floor(k/2) storage neighbours
 *     below and ceil(k/2) above, cut off at the sector's ends (Sec. III-C,
 *     Fig. 3); there is no refresh of the whole sector after the first pick;
 *   - the last pick refreshes no distance (the loop ends once it is stored).
 * The alternative readings of the three NPDU points are available as flags
 * (ORACLE_NPDU_* below), so that their effect can be measured.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math
 * (x86-64 SSE arithmetic: every fp32 operation is a single IEEE rounding).
 */
#include <stdint.h>
#include <stdlib.h>

#define ORACLE_OK 0
#define ORACLE_ERR_NULL (-1)
#define ORACLE_ERR_ARG (-2)
#define ORACLE_ERR_RANGE (-3)
#define ORACLE_ERR_NOMEM (-6)

/*
 * NPDU readings other than the default one (bit flags), for the points
 * Sec. III-C leaves open:
 *   FIRST_FULL : the first iteration updates every point of the sector (one
 *                full Algorithm-1 update from the start point); later
 *                iterations update only the window;
 *   SHIFT_EDGES: a window that would cross an edge of the sector is moved
 *                inward, keeping its size as far as the sector allows,
 *                instead of being truncated;
 *   K_WITH_SELF: the k updated points include the new sample: floor((k-1)/2)
 *                below it and ceil((k-1)/2) above (k >= 1), instead of the
 *                sample plus k neighbours.
 */
#define ORACLE_NPDU_FIRST_FULL 1
#define ORACLE_NPDU_SHIFT_EDGES 2
#define ORACLE_NPDU_K_WITH_SELF 4

/* Value every running distance starts from (exact in fp32). */
static const float INITIAL_DISTANCE = 1e10f;

/*
 * Sector s of M (Sec. III-B: the cloud is divided by storage location, and C
 * samples take C/M iterations).  Points: the first (n mod m) sectors get one
 * extra point; samples: the first (c mod m) sectors get one extra sample.
 */
void oracle_sector(int32_t n, int32_t c, int32_t m, int32_t s,
                   int32_t *first_point, int32_t *num_points,
                   int32_t *first_sample, int32_t *num_samples)
{
    int32_t qn = n / m, rn = n % m;
    int32_t qc = c / m, rc = c % m;
    *num_points = qn + (s < rn ? 1 : 0);
    *first_point = s * qn + (s < rn ? s : rn);
    *num_samples = qc + (s < rc ? 1 : 0);
    *first_sample = s * qc + (s < rc ? s : rc);
}

/* Squared Euclidean distance of p from q, in a fixed operation order. */
static float squared_distance(const float *p, const float *q)
{
    float dx = p[0] - q[0];
    float dy = p[1] - q[1];
    float dz = p[2] - q[2];
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float xy = xx + yy;
    return xy + zz;
}

/*
 * The storage range [*lo, *hi] (sector-local) whose distances a new sample at
 * local index cur refreshes.  The whole sector when `whole` is set (FPS and
 * AFPS, or the full first refresh of the FIRST_FULL reading); otherwise the
 * NPDU neighbourhood of Sec. III-C: the sample with `below` points under it
 * and `above` over it, cut off (or, SHIFT_EDGES, pushed back inside) at the
 * ends of the sector.
 */
static void refresh_range(int32_t n, int32_t k, int32_t flags, int whole, int32_t cur,
                          int32_t *lo, int32_t *hi)
{
    if (whole) {
        *lo = 0;
        *hi = n - 1;
        return;
    }
    int32_t below, above;
    if (flags & ORACLE_NPDU_K_WITH_SELF) {
        below = (k - 1) / 2;                           /* k >= 1 points counting the sample */
        above = (k - 1) - below;
    } else {
        below = k / 2;                                 /* the sample and k neighbours */
        above = k - k / 2;
    }
    int64_t from = (int64_t)cur - below, to = (int64_t)cur + above;
    if (flags & ORACLE_NPDU_SHIFT_EDGES) {
        if (from < 0) {                                /* slide up, off the bottom end */
            to -= from;
            from = 0;
        }
        if (to > n - 1) {                              /* slide down, off the top end */
            from -= to - (n - 1);
            to = n - 1;
        }
    }
    *lo = from < 0 ? 0 : (int32_t)from;                /* never outside the sector */
    *hi = to > n - 1 ? n - 1 : (int32_t)to;
}

/*
 * Lower the running distance of every point in [lo, hi] of the sector pts to
 * its squared distance from `sample` when that is smaller.  Returns the
 * number of distances computed.
 */
static int64_t relax(const float *pts, int32_t lo, int32_t hi, const float *sample, float *dist)
{
    for (int32_t j = lo; j <= hi; ++j) {
        float d = squared_distance(pts + 3 * (int64_t)j, sample);
        dist[j] = d < dist[j] ? d : dist[j];
    }
    return (int64_t)hi - lo + 1;
}

/* The lowest index whose running distance is the largest of the sector. */
static int32_t farthest(const float *dist, int32_t n)
{
    int32_t far = 0;
    for (int32_t j = 1; j < n; ++j)
        if (dist[j] > dist[far])
            far = j;
    return far;
}

/*
 * Farthest point sampling on one sector, the points P[first .. first+n):
 * c picks, the first at local index start mod n, each further one the point
 * farthest from the picks so far as the running distances see it.  After
 * each pick only refresh_range's points are refreshed (all of them without
 * NPDU, k < 0); the last pick refreshes nothing, since no pick follows it.
 * Writes the c global indices to out[0..c) and leaves the running distances
 * in dist[0..n).  Returns the number of distances computed.
 */
static int64_t sample_sector(const float *P, int32_t first, int32_t n, int32_t c,
                             int32_t k, int32_t flags, int32_t start, float *dist, int32_t *out)
{
    const float *pts = P + 3 * (int64_t)first;
    for (int32_t j = 0; j < n; ++j)
        dist[j] = INITIAL_DISTANCE;
    int64_t computed = 0;
    int32_t pick = start % n;
    out[0] = first + pick;
    for (int32_t t = 1; t < c; ++t) {
        const int whole = k < 0 || (t == 1 && (flags & ORACLE_NPDU_FIRST_FULL));
        int32_t lo, hi;
        refresh_range(n, k, flags, whole, pick, &lo, &hi);
        computed += relax(pts, lo, hi, pts + 3 * (int64_t)pick, dist);
        pick = farthest(dist, n);
        out[t] = first + pick;
    }
    return computed;
}

/*
 * AFPS with M sectors; k < 0 turns NPDU off; M = 1 and k < 0 is plain FPS;
 * flags selects NPDU readings (ORACLE_NPDU_*; 0 = the default reading).
 *   P      : n x 3 fp32, row-major (x, y, z per point)
 *   out    : c int32 global indices, sector-major, pick order inside a sector
 *   dist   : optional (may be NULL), n floats: the Distance arrays as the loop
 *            leaves them, sector after sector
 *   evals  : optional (may be NULL), total number of distance evaluations
 * Requires 1 <= m <= c <= n and 0 <= start < n.
 */
int oracle_afps_ex(const float *P, int32_t n, int32_t c, int32_t m, int32_t k, int32_t flags,
                   int32_t start, int32_t *out, float *dist, int64_t *evals)
{
    if (!P || !out)
        return ORACLE_ERR_NULL;
    if (m < 1 || c < m || n < c)
        return ORACLE_ERR_ARG;
    if (flags & ~(ORACLE_NPDU_FIRST_FULL | ORACLE_NPDU_SHIFT_EDGES | ORACLE_NPDU_K_WITH_SELF))
        return ORACLE_ERR_ARG;
    if (flags && k < 0)
        return ORACLE_ERR_ARG;                         /* the flags are NPDU readings */
    if ((flags & ORACLE_NPDU_K_WITH_SELF) && k < 1)
        return ORACLE_ERR_ARG;
    if (start < 0 || start >= n)
        return ORACLE_ERR_RANGE;

    float *work = dist;
    if (!work) {
        work = (float *)malloc(sizeof(float) * (size_t)n);
        if (!work)
            return ORACLE_ERR_NOMEM;
    }
    int64_t total = 0;
    for (int32_t s = 0; s < m; ++s) {                  /* sectors are independent */
        int32_t first, count, first_out, samples;
        oracle_sector(n, c, m, s, &first, &count, &first_out, &samples);
        total += sample_sector(P, first, count, samples, k, flags, start,
                               work + first, out + first_out);
    }
    if (work != dist)
        free(work);
    if (evals)
        *evals = total;
    return ORACLE_OK;
}

/* AFPS / NPDU with the default readings. */
int oracle_afps(const float *P, int32_t n, int32_t c, int32_t m, int32_t k,
                int32_t start, int32_t *out, float *dist, int64_t *evals)
{
    return oracle_afps_ex(P, n, c, m, k, 0, start, out, dist, evals);
}

/* Plain FPS: AFPS with one sector and no NPDU. */
int oracle_fps(const float *P, int32_t n, int32_t c, int32_t start, int32_t *out,
               float *dist, int64_t *evals)
{
    return oracle_afps(P, n, c, 1, -1, start, out, dist, evals);
}

/*
 * Grouping around the samples: the second half of a PointNet++ set
 * abstraction layer, which the paper names as the consumer of the samples
 * (Sec. I, Sec. II-A) without defining it.  Readings (design notes):
 *   - ball query: the neighbours of centre q are the points j with
 *     squared_distance(P[j], P[q]) < r2 (fp32, the distance above; r2 =
 *     radius * radius rounded to fp32), taken in increasing index order, at
 *     most K of them; slots past the found ones repeat the first found, or
 *     hold q when none was found (radius 0);
 *   - search window (Sec. III-A: with dimensional locality, storage
 *     neighbours approximate spatial neighbours): only j in
 *     [q - window, q + window] are candidates; window < 0 searches the whole
 *     cloud (the exact ball query).
 * out_idx gets K indices per centre (centre-major), out_cnt the number found
 * (at most K) per centre.
 */
int oracle_ball_query(const float *P, int32_t n, const int32_t *centers, int32_t c, float radius,
                      int32_t K, int32_t window, int32_t *out_idx, int32_t *out_cnt)
{
    if (!P || !centers || !out_idx || !out_cnt) return ORACLE_ERR_NULL;
    if (n < 1 || c < 0 || K < 1 || !(radius >= 0.0f)) return ORACLE_ERR_ARG;
    const float r2 = radius * radius;
    for (int32_t q = 0; q < c; ++q) {
        const int32_t ci = centers[q];
        if (ci < 0 || ci >= n) return ORACLE_ERR_RANGE;
        int32_t lo = 0, hi = n - 1;
        if (window >= 0) {
            lo = ci - window < 0 ? 0 : ci - window;
            hi = ci > n - 1 - window ? n - 1 : ci + window;
        }
        int32_t *row = out_idx + (int64_t)q * K;
        int32_t found = 0;
        for (int32_t j = lo; j <= hi && found < K; ++j)
            if (squared_distance(P + 3 * (int64_t)j, P + 3 * (int64_t)ci) < r2) row[found++] = j;
        const int32_t fill = found > 0 ? row[0] : ci;
        for (int32_t l = found; l < K; ++l) row[l] = fill;
        out_cnt[q] = found;
    }
    return ORACLE_OK;
}
