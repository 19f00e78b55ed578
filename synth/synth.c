/*
 * Seeded synthetic label-map rasterisers.
 *
 * This module only *draws input volumes*; it holds none of the SurfaceNets
 * arithmetic.  Both the HIP path and the CPU oracle receive the bytes written
 * here.  Random parameters (centres, radii, seed points, directions) are drawn
 * by the Python side with numpy's seeded generator and passed in explicitly,
 * so every function below is a deterministic function of its arguments and of
 * nothing else (no thread-count or scheduling dependence).
 *
 * Volumes are x-fastest: value(i,j,k) lives at i + M*(j + N*k).
 * `b` is the byte width of one label (1, 2 or 4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline void put_label(void *out, int b, int64_t idx, uint32_t v)
{
    if (b == 1)
        ((uint8_t *)out)[idx] = (uint8_t)v;
    else if (b == 2)
        ((uint16_t *)out)[idx] = (uint16_t)v;
    else
        ((uint32_t *)out)[idx] = v;
}

static inline uint32_t get_label(const void *in, int b, int64_t idx)
{
    if (b == 1)
        return ((const uint8_t *)in)[idx];
    if (b == 2)
        return ((const uint16_t *)in)[idx];
    return ((const uint32_t *)in)[idx];
}

/* Fill the whole volume with one value. */
void synth_fill(void *out, int b, int64_t M, int64_t N, int64_t O, uint32_t v)
{
    int64_t V = M * N * O;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < V; ++t)
        put_label(out, b, t, v);
}

/*
 * Overlapping balls, painted in order (a later ball overwrites an earlier one).
 * Voxel (i,j,k) belongs to ball s iff |(i,j,k) - c_s|^2 <= r_s^2 (index space).
 * The volume is first filled with `bg`.
 */
void synth_spheres(void *out, int b, int64_t M, int64_t N, int64_t O, int32_t n,
                   const double *centres, const double *radii, const uint32_t *labels,
                   uint32_t bg)
{
    synth_fill(out, b, M, N, O, bg);
    for (int32_t s = 0; s < n; ++s) {
        const double cx = centres[3 * s], cy = centres[3 * s + 1], cz = centres[3 * s + 2];
        const double r = radii[s], r2 = r * r;
        int64_t k0 = (int64_t)floor(cz - r), k1 = (int64_t)ceil(cz + r);
        int64_t j0 = (int64_t)floor(cy - r), j1 = (int64_t)ceil(cy + r);
        int64_t i0 = (int64_t)floor(cx - r), i1 = (int64_t)ceil(cx + r);
        if (k0 < 0) k0 = 0;
        if (j0 < 0) j0 = 0;
        if (i0 < 0) i0 = 0;
        if (k1 > O - 1) k1 = O - 1;
        if (j1 > N - 1) j1 = N - 1;
        if (i1 > M - 1) i1 = M - 1;
#pragma omp parallel for schedule(static)
        for (int64_t k = k0; k <= k1; ++k) {
            for (int64_t j = j0; j <= j1; ++j) {
                for (int64_t i = i0; i <= i1; ++i) {
                    double dx = (double)i - cx, dy = (double)j - cy, dz = (double)k - cz;
                    if (dx * dx + dy * dy + dz * dz <= r2)
                        put_label(out, b, i + M * (j + N * k), labels[s]);
                }
            }
        }
    }
}

/* ---- block-candidate helpers shared by the Voronoi rasterisers ----------- */

#define SYN_BLOCK 16

/* squared distance from point p to the axis-aligned box [lo, hi] */
static inline double box_min_d2(const double *p, const double *lo, const double *hi)
{
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d = 0.0;
        if (p[a] < lo[a])
            d = lo[a] - p[a];
        else if (p[a] > hi[a])
            d = p[a] - hi[a];
        d2 += d * d;
    }
    return d2;
}

static inline double box_max_d2(const double *p, const double *lo, const double *hi)
{
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d0 = fabs(p[a] - lo[a]), d1 = fabs(p[a] - hi[a]);
        double d = d0 > d1 ? d0 : d1;
        d2 += d * d;
    }
    return d2;
}

/*
 * Isotropic Voronoi partition in world space (world = index * spacing).
 * label(x) = labels[argmin_s |world(x) - seed_s|^2]; ties go to the lower s.
 * If ell != NULL and ell[3] > 0, voxels outside the index-space ellipsoid
 * ((i-cx)/ax)^2 + ((j-cy)/ay)^2 + ((k-cz)/az)^2 <= 1 get `bg`.
 * Candidates are pruned per 16^3 block with the exact bound
 * min_s maxdist(s, block) (a seed farther than that from the whole block can
 * never be the nearest), so the result equals the brute-force argmin.
 */
void synth_voronoi(void *out, int b, int64_t M, int64_t N, int64_t O, const double *spacing,
                   int32_t n, const double *seeds, const uint32_t *labels, const double *ell,
                   uint32_t bg)
{
    const int64_t BX = (M + SYN_BLOCK - 1) / SYN_BLOCK, BY = (N + SYN_BLOCK - 1) / SYN_BLOCK,
                  BZ = (O + SYN_BLOCK - 1) / SYN_BLOCK;
    const int use_mask = (ell != NULL && ell[3] > 0.0);
#pragma omp parallel
    {
        int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t blk = 0; blk < BX * BY * BZ; ++blk) {
            int64_t bx = blk % BX, by = (blk / BX) % BY, bz = blk / (BX * BY);
            int64_t i0 = bx * SYN_BLOCK, j0 = by * SYN_BLOCK, k0 = bz * SYN_BLOCK;
            int64_t i1 = i0 + SYN_BLOCK < M ? i0 + SYN_BLOCK : M;
            int64_t j1 = j0 + SYN_BLOCK < N ? j0 + SYN_BLOCK : N;
            int64_t k1 = k0 + SYN_BLOCK < O ? k0 + SYN_BLOCK : O;
            double lo[3] = {i0 * spacing[0], j0 * spacing[1], k0 * spacing[2]};
            double hi[3] = {(i1 - 1) * spacing[0], (j1 - 1) * spacing[1], (k1 - 1) * spacing[2]};
            double ub = INFINITY;
            for (int32_t s = 0; s < n; ++s) {
                double d = box_max_d2(seeds + 3 * s, lo, hi);
                if (d < ub) ub = d;
            }
            int32_t nc = 0;
            for (int32_t s = 0; s < n; ++s)
                if (box_min_d2(seeds + 3 * s, lo, hi) <= ub) cand[nc++] = s;
            for (int64_t k = k0; k < k1; ++k)
                for (int64_t j = j0; j < j1; ++j)
                    for (int64_t i = i0; i < i1; ++i) {
                        int64_t idx = i + M * (j + N * k);
                        if (use_mask) {
                            double u = ((double)i - ell[0]) / ell[3];
                            double v = ((double)j - ell[1]) / ell[4];
                            double w = ((double)k - ell[2]) / ell[5];
                            if (u * u + v * v + w * w > 1.0) {
                                put_label(out, b, idx, bg);
                                continue;
                            }
                        }
                        double x = i * spacing[0], y = j * spacing[1], z = k * spacing[2];
                        double best = INFINITY;
                        int32_t arg = -1;
                        for (int32_t c = 0; c < nc; ++c) {
                            const double *s = seeds + 3 * cand[c];
                            double dx = x - s[0], dy = y - s[1], dz = z - s[2];
                            double d = dx * dx + dy * dy + dz * dz;
                            if (d < best) { /* strict: ties keep the lower index */
                                best = d;
                                arg = cand[c];
                            }
                        }
                        put_label(out, b, idx, arg >= 0 ? labels[arg] : bg);
                    }
        }
        free(cand);
    }
}

/*
 * Stretched ("needle") Voronoi in index space.  Seed s has a unit direction
 * u_s; its distance is  d_s(x)^2 = |x-s|^2 - (1 - 1/alpha^2) ((x-s).u_s)^2,
 * which makes its cell alpha times longer along u_s.  Only seeds within
 * Euclidean distance R of x compete (a truncated partition; R is part of the
 * definition).  label(x) = labels[argmin d_s]; ties go to the lower s; no
 * candidate -> bg.  If tau > 0, voxels whose gap between the second-smallest
 * and smallest d_s is below tau become `bg` (a thin membrane along cell walls).
 * If gaps != NULL the function instead writes the gap of every `stride`-th
 * voxel (linear index 0, stride, 2*stride, ...) into gaps[] and writes no
 * labels; the caller picks tau as a quantile of those samples.
 */
void synth_stretched(void *out, int b, int64_t M, int64_t N, int64_t O, int32_t n,
                     const double *seeds, const double *dirs, const uint32_t *labels,
                     double alpha, double R, double tau, uint32_t bg, double *gaps,
                     int64_t stride)
{
    const int64_t BX = (M + SYN_BLOCK - 1) / SYN_BLOCK, BY = (N + SYN_BLOCK - 1) / SYN_BLOCK,
                  BZ = (O + SYN_BLOCK - 1) / SYN_BLOCK;
    const double shrink = 1.0 - 1.0 / (alpha * alpha);
    const double R2 = R * R;
    /* coarse bucket grid of seeds (bucket edge G voxels) for candidate lookup */
    const int64_t G = 32;
    const int64_t GX = (M + G - 1) / G, GY = (N + G - 1) / G, GZ = (O + G - 1) / G;
    const int64_t NG = GX * GY * GZ;
    int64_t *head = (int64_t *)calloc((size_t)NG + 1, sizeof(int64_t));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t s = 0; s < n; ++s) {
        int64_t gx = (int64_t)floor(seeds[3 * s] / G), gy = (int64_t)floor(seeds[3 * s + 1] / G),
                gz = (int64_t)floor(seeds[3 * s + 2] / G);
        if (gx < 0) gx = 0;
        if (gy < 0) gy = 0;
        if (gz < 0) gz = 0;
        if (gx >= GX) gx = GX - 1;
        if (gy >= GY) gy = GY - 1;
        if (gz >= GZ) gz = GZ - 1;
        head[gx + GX * (gy + GY * gz) + 1]++;
    }
    for (int64_t g = 0; g < NG; ++g) head[g + 1] += head[g];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)NG);
        memcpy(fill, head, sizeof(int64_t) * (size_t)NG);
        for (int32_t s = 0; s < n; ++s) { /* stable: seeds stay in index order per bucket */
            int64_t gx = (int64_t)floor(seeds[3 * s] / G), gy = (int64_t)floor(seeds[3 * s + 1] / G),
                    gz = (int64_t)floor(seeds[3 * s + 2] / G);
            if (gx < 0) gx = 0;
            if (gy < 0) gy = 0;
            if (gz < 0) gz = 0;
            if (gx >= GX) gx = GX - 1;
            if (gy >= GY) gy = GY - 1;
            if (gz >= GZ) gz = GZ - 1;
            order[fill[gx + GX * (gy + GY * gz)]++] = s;
        }
        free(fill);
    }
#pragma omp parallel
    {
        int32_t cap = 1024, *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
#pragma omp for schedule(dynamic, 1)
        for (int64_t blk = 0; blk < BX * BY * BZ; ++blk) {
            int64_t bx = blk % BX, by = (blk / BX) % BY, bz = blk / (BX * BY);
            int64_t i0 = bx * SYN_BLOCK, j0 = by * SYN_BLOCK, k0 = bz * SYN_BLOCK;
            int64_t i1 = i0 + SYN_BLOCK < M ? i0 + SYN_BLOCK : M;
            int64_t j1 = j0 + SYN_BLOCK < N ? j0 + SYN_BLOCK : N;
            int64_t k1 = k0 + SYN_BLOCK < O ? k0 + SYN_BLOCK : O;
            if (gaps) { /* skip blocks holding no sampled voxel */
                int any = 0;
                for (int64_t k = k0; k < k1 && !any; ++k)
                    for (int64_t j = j0; j < j1 && !any; ++j) {
                        int64_t a = i0 + M * (j + N * k), z = (i1 - 1) + M * (j + N * k);
                        int64_t first = ((a + stride - 1) / stride) * stride;
                        if (first <= z) any = 1;
                    }
                if (!any) continue;
            }
            double lo[3] = {(double)i0, (double)j0, (double)k0};
            double hi[3] = {(double)(i1 - 1), (double)(j1 - 1), (double)(k1 - 1)};
            /* candidate seeds: Euclidean distance to the block <= R, in index order */
            int64_t gx0 = (int64_t)floor((lo[0] - R) / G), gx1 = (int64_t)floor((hi[0] + R) / G);
            int64_t gy0 = (int64_t)floor((lo[1] - R) / G), gy1 = (int64_t)floor((hi[1] + R) / G);
            int64_t gz0 = (int64_t)floor((lo[2] - R) / G), gz1 = (int64_t)floor((hi[2] + R) / G);
            if (gx0 < 0) gx0 = 0;
            if (gy0 < 0) gy0 = 0;
            if (gz0 < 0) gz0 = 0;
            if (gx1 >= GX) gx1 = GX - 1;
            if (gy1 >= GY) gy1 = GY - 1;
            if (gz1 >= GZ) gz1 = GZ - 1;
            int32_t nc = 0;
            for (int64_t gz = gz0; gz <= gz1; ++gz)
                for (int64_t gy = gy0; gy <= gy1; ++gy)
                    for (int64_t gx = gx0; gx <= gx1; ++gx) {
                        int64_t g = gx + GX * (gy + GY * gz);
                        for (int64_t t = head[g]; t < head[g + 1]; ++t) {
                            int32_t s = order[t];
                            if (box_min_d2(seeds + 3 * s, lo, hi) <= R2) {
                                if (nc == cap) {
                                    cap *= 2;
                                    cand = (int32_t *)realloc(cand, sizeof(int32_t) * (size_t)cap);
                                }
                                cand[nc++] = s;
                            }
                        }
                    }
            /* index order so that the tie rule (lower s wins) does not depend on buckets */
            for (int32_t a = 1; a < nc; ++a) {
                int32_t v = cand[a], c = a - 1;
                while (c >= 0 && cand[c] > v) {
                    cand[c + 1] = cand[c];
                    --c;
                }
                cand[c + 1] = v;
            }
            for (int64_t k = k0; k < k1; ++k)
                for (int64_t j = j0; j < j1; ++j)
                    for (int64_t i = i0; i < i1; ++i) {
                        int64_t idx = i + M * (j + N * k);
                        if (gaps && (idx % stride) != 0) continue;
                        double best = INFINITY, second = INFINITY;
                        int32_t arg = -1;
                        for (int32_t c = 0; c < nc; ++c) {
                            const double *s = seeds + 3 * cand[c];
                            const double *u = dirs + 3 * cand[c];
                            double dx = (double)i - s[0], dy = (double)j - s[1], dz = (double)k - s[2];
                            double e2 = dx * dx + dy * dy + dz * dz;
                            if (e2 > R2) continue;
                            double t = dx * u[0] + dy * u[1] + dz * u[2];
                            double d = e2 - shrink * t * t;
                            if (d < best) {
                                second = best;
                                best = d;
                                arg = cand[c];
                            } else if (d < second) {
                                second = d;
                            }
                        }
                        double gap = sqrt(second > 0 ? second : 0) - sqrt(best > 0 ? best : 0);
                        if (gaps) {
                            gaps[idx / stride] = arg >= 0 ? gap : INFINITY;
                            continue;
                        }
                        uint32_t v = arg >= 0 ? labels[arg] : bg;
                        if (tau > 0 && arg >= 0 && gap < tau) v = bg;
                        put_label(out, b, idx, v);
                    }
        }
        free(cand);
    }
    free(head);
    free(order);
}

/* Remap every voxel through a lookup table of 2^(8b) entries (u8/u16 only). */
void synth_remap_lut(void *vol, int b, int64_t V, const uint32_t *lut)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < V; ++t)
        put_label(vol, b, t, lut[get_label(vol, b, t)]);
}
