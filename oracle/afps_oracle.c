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
 * route), so this oracle follows the algorithm step by step in the paper's
 * order: Algorithm 1 (FPS), Sec. III-B (AFPS sectors), Sec. III-C (NPDU).  It is
 * deliberately slow and unblocked: one sector after the other, one point after
 * the other, a full sequential argmax scan every iteration.
 *
 * Readings of points the paper leaves open (each is used identically by the
 * GPU path; the numbering follows the design notes):
 *   - distance: squared Euclidean in fp32, ((dx*dx + dy*dy) + dz*dz) with
 *     dx = P[j].x - P[cur].x, every operation rounded to nearest, no fused
 *     multiply-add (Algorithm 1, geo_dist; the argmax does not change under
 *     sqrt, and skipping sqrt creates no extra rounding ties);
 *   - initial distance 1e10 (Algorithm 1 initialisation), exact in fp32;
 *   - argmax ties go to the lowest index (a sequential scan with strict '>');
 *   - start: sector s starts at its local point (start mod n_s);
 *   - sectors are contiguous storage ranges: the first N mod M sectors hold one
 *     extra point, the first C mod M sectors take one extra sample (Sec. III-B:
 *     C/M iterations per sector);
 *   - NPDU window: the new sample plus floor(k/2) storage neighbours below and
 *     ceil(k/2) above, truncated at the sector's edges (Sec. III-C, Fig. 3);
 *     there is no full distance pass on the first iteration;
 *   - the last sample's own distance update is never applied (Algorithm 1 ends
 *     after storing the last sample).
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

/* Algorithm 1: every distance starts at 1e10. */
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

/* Algorithm 1, geo_dist: squared Euclidean distance, fixed operation order. */
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
 * Local FPS on one sector (Algorithm 1 applied to P[first .. first+n)),
 * optionally with NPDU (k >= 0).  Writes c global indices to out[0..c).
 * dist is the sector's Distance array (n entries).  Returns the number of
 * distance evaluations.
 */
static int64_t sample_sector(const float *P, int32_t first, int32_t n, int32_t c,
                             int32_t k, int32_t flags, int32_t start, float *dist, int32_t *out)
{
    int64_t evaluations = 0;
    for (int32_t j = 0; j < n; ++j)
        dist[j] = INITIAL_DISTANCE;                    /* Algorithm 1: Distance = 1e10 */

    int32_t cur = start % n;                           /* first sample of the sector */
    out[0] = first + cur;

    for (int32_t i = 1; i < c; ++i) {                  /* Algorithm 1: i = 1 .. n_point-1 */
        /* Update set: the whole sector (FPS / AFPS), or the NPDU window. */
        int32_t lo = 0, hi = n - 1;
        if (k >= 0 && !(i == 1 && (flags & ORACLE_NPDU_FIRST_FULL))) {
            int32_t below, above;
            if (flags & ORACLE_NPDU_K_WITH_SELF) {
                below = (k - 1) / 2;                   /* k >= 1: k points with the sample */
                above = (k - 1) - below;
            } else {
                below = k / 2;                         /* the sample and k neighbours */
                above = k - k / 2;
            }
            int64_t l = (int64_t)cur - below, h = (int64_t)cur + above;
            if (flags & ORACLE_NPDU_SHIFT_EDGES) {
                if (l < 0) {                           /* move right, off the lower edge */
                    h -= l;
                    l = 0;
                }
                if (h > n - 1) {                       /* move left, off the upper edge */
                    l -= h - (n - 1);
                    h = n - 1;
                }
            }
            lo = l < 0 ? 0 : (int32_t)l;               /* truncate to the sector */
            hi = h > n - 1 ? n - 1 : (int32_t)h;
        }
        const float *sample = P + 3 * (int64_t)(first + cur);
        for (int32_t j = lo; j <= hi; ++j) {           /* Algorithm 1: distance update */
            float d = squared_distance(P + 3 * (int64_t)(first + j), sample);
            ++evaluations;
            if (d <= dist[j])
                dist[j] = d;
        }
        int32_t best = 0;                              /* Algorithm 1: argmax(Distance) */
        for (int32_t j = 1; j < n; ++j)
            if (dist[j] > dist[best])
                best = j;
        cur = best;
        out[i] = first + cur;                          /* Algorithm 1: Sampled[i] */
    }
    return evaluations;
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

/* Plain FPS (Algorithm 1): AFPS with one sector and no NPDU. */
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
