/*
 * SurfaceNets oracle, all host cores -- TEST AND BENCHMARK INFRASTRUCTURE ONLY.
 *
 * The loops of the serial oracle (sn_oracle.c, included below unchanged)
 * spread over z-slices with OpenMP, for the benchmark's all-cores CPU
 * baseline.  Every output element is computed by the same definition and the
 * same FP64 operations in the same order as in the serial oracle:
 *
 *   classification    one value at a time (Sec. 2.1);
 *   points            per cell slice, a count, then ids from the exclusive
 *                     prefix of the slice counts, so ids still follow the cell
 *                     linear index (Sec. 2.2; the paper's Pass 3 prefix sum,
 *                     Sec. 2.3, taken over slices);
 *   quads             per lattice slice, a count, a prefix, then the quads of
 *                     each slice written at its offset, in the serial order;
 *   stencil           per cell slice, the same;
 *   smoothing         Eq. (1) with the box or sphere constraint, Jacobi: every
 *                     point of a sweep reads only the previous sweep's
 *                     positions, so points are independent within a sweep
 *                     (Sec. 2.4) and its per-point arithmetic is the serial one.
 *
 * So its results equal the serial oracle's bit for bit (a CPU test checks
 * this).  It is never the parity reference: the serial oracle is.  It shares
 * nothing with the GPU library.
 */
#include "sn_oracle.c"

#include <omp.h>

/* exclusive prefix of n counts into off[0..n]; serial (n is a slice count) */
static void prefix_counts(const int64_t *cnt, int64_t n, int64_t *off)
{
    off[0] = 0;
    for (int64_t t = 0; t < n; ++t)
        off[t + 1] = off[t] + cnt[t];
}

/* cells of the 4 quad vertices of the axis-a edge at (i,j,k), serial order */
static void quad_cells(int64_t i, int64_t j, int64_t k, int a, int64_t c4[4][3])
{
    if (a == 0) {
        int64_t t[4][3] = {{i, j - 1, k - 1}, {i, j - 1, k}, {i, j, k}, {i, j, k - 1}};
        memcpy(c4, t, sizeof t);
    } else if (a == 1) {
        int64_t t[4][3] = {{i - 1, j, k - 1}, {i, j, k - 1}, {i, j, k}, {i - 1, j, k}};
        memcpy(c4, t, sizeof t);
    } else {
        int64_t t[4][3] = {{i - 1, j - 1, k}, {i - 1, j, k}, {i, j, k}, {i, j - 1, k}};
        memcpy(c4, t, sizeof t);
    }
}

static int quad_emitted(const cvol *v, int64_t i, int64_t j, int64_t k, int a)
{
    if (!cut(v, i, j, k, a))
        return 0;
    int64_t c4[4][3];
    quad_cells(i, j, k, a, c4);
    for (int q = 0; q < 4; ++q)
        if (!cell_exists(v, c4[q][0], c4[q][1], c4[q][2]))
            return 0;
    return 1;
}

static int stencil_link(const cvol *v, int64_t i, int64_t j, int64_t k, int f, int64_t *n3)
{
    const int64_t d = (f % 2) ? 1 : -1;
    n3[0] = i + (f / 2 == 0) * d, n3[1] = j + (f / 2 == 1) * d, n3[2] = k + (f / 2 == 2) * d;
    return cell_exists(v, n3[0], n3[1], n3[2]) && face_has_cut(v, i, j, k, f);
}

/*
 * The 3D extraction on `threads` OpenMP threads (0: the runtime's default).
 * Same arguments and result as orc_extract.
 */
orc_mesh *orc_extract_par(const void *labels, int b, int64_t M, int64_t N, int64_t O,
                          const uint32_t *selected, int32_t n_sel, uint32_t background,
                          int32_t threads)
{
    if (M < 1 || N < 1 || O < 1 || (b != 1 && b != 2 && b != 4) || n_sel < 0 || threads < 0)
        return NULL;
    if (threads > 0)
        omp_set_num_threads(threads);
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    if (!m)
        return NULL;
    m->M = M, m->N = N, m->O = O;
    m->nv = 4;
    const int64_t V = M * N * O;
    uint32_t *sel = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n_sel > 0 ? n_sel : 1));
    uint32_t *cv = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)V);
    const int64_t CM = M - 1, CN = N - 1, CO = O - 1;
    const int64_t ncell = (CM > 0 && CN > 0 && CO > 0) ? CM * CN * CO : 0;
    const int64_t cslices = ncell > 0 ? CO : 0;
    int64_t *pid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    int64_t *cnt = (int64_t *)calloc((size_t)(O + 1), sizeof(int64_t));
    int64_t *off = (int64_t *)calloc((size_t)(O + 2), sizeof(int64_t));
    if (!sel || !cv || !pid || !cnt || !off) {
        free(sel), free(cv), free(pid), free(cnt), free(off), free(m);
        return NULL;
    }
    if (n_sel > 0)
        memcpy(sel, selected, sizeof(uint32_t) * (size_t)n_sel);
    qsort(sel, (size_t)n_sel, sizeof(uint32_t), cmp_u32);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < V; ++t)
        cv[t] = classify(raw_label(labels, b, t), sel, n_sel, background);
    free(sel);
    cvol v = {cv, M, N, O};

    /* points: flags and counts per cell slice, then ids in cell order */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < cslices; ++k) {
        int64_t n = 0;
        for (int64_t j = 0; j < CN; ++j)
            for (int64_t i = 0; i < CM; ++i) {
                const int pt = cell_has_point(&v, i, j, k);
                pid[i + CM * (j + CN * k)] = pt;
                n += pt;
            }
        cnt[k] = n;
    }
    prefix_counts(cnt, cslices, off);
    const int64_t P = off[cslices];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < cslices; ++k) {
        int64_t id = off[k];
        for (int64_t c = CM * CN * k; c < CM * CN * (k + 1); ++c)
            pid[c] = pid[c] ? id++ : -1;
    }
    m->P = P;
    m->cell_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P > 0 ? P : 1));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncell; ++c)
        if (pid[c] >= 0)
            m->cell_of[pid[c]] = c;
#define PID(i, j, k) pid[(i) + CM * ((j) + CN * (k))]

    /* quads: per lattice slice, counted, then written in the serial order */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < O; ++k) {
        int64_t n = 0;
        for (int64_t j = 0; j < N; ++j)
            for (int64_t i = 0; i < M; ++i)
                for (int a = 0; a < 3; ++a)
                    n += quad_emitted(&v, i, j, k, a);
        cnt[k] = n;
    }
    prefix_counts(cnt, O, off);
    const int64_t Q = off[O];
    m->Q = Q;
    m->quads = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(Q > 0 ? Q : 1));
    m->pairs = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (size_t)(Q > 0 ? Q : 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < O; ++k) {
        int64_t q = off[k];
        for (int64_t j = 0; j < N; ++j)
            for (int64_t i = 0; i < M; ++i)
                for (int a = 0; a < 3; ++a) {
                    if (!quad_emitted(&v, i, j, k, a))
                        continue;
                    int64_t c4[4][3];
                    quad_cells(i, j, k, a, c4);
                    for (int t = 0; t < 4; ++t)
                        m->quads[4 * q + t] = (int32_t)PID(c4[t][0], c4[t][1], c4[t][2]);
                    m->pairs[2 * q + 0] = C(&v, i, j, k);
                    m->pairs[2 * q + 1] = C(&v, i + (a == 0), j + (a == 1), k + (a == 2));
                    ++q;
                }
    }

    /* stencil: per cell slice, the points of the slice in id order */
    m->st_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P + 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < cslices; ++k) {
        int64_t n = 0;
        for (int64_t j = 0; j < CN; ++j)
            for (int64_t i = 0; i < CM; ++i) {
                if (PID(i, j, k) < 0)
                    continue;
                for (int f = 0; f < 6; ++f) {
                    int64_t n3[3];
                    n += stencil_link(&v, i, j, k, f, n3);
                }
            }
        cnt[k] = n;
    }
    prefix_counts(cnt, cslices, off);
    const int64_t S = off[cslices];
    m->S = S;
    m->st_ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(S > 0 ? S : 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < cslices; ++k) {
        int64_t s = off[k];
        for (int64_t j = 0; j < CN; ++j)
            for (int64_t i = 0; i < CM; ++i) {
                const int64_t p = PID(i, j, k);
                if (p < 0)
                    continue;
                m->st_off[p] = s;
                for (int f = 0; f < 6; ++f) {
                    int64_t n3[3];
                    if (stencil_link(&v, i, j, k, f, n3))
                        m->st_ids[s++] = (int32_t)PID(n3[0], n3[1], n3[2]);
                }
            }
    }
    m->st_off[P] = S;
#undef PID
    free(pid), free(cnt), free(off), free(cv);
    return m;
}

/*
 * Eq. (1) sweeps as orc_smooth_shape, points of a sweep spread over threads.
 */
int orc_smooth_par(const orc_mesh *m, int32_t iterations, double lambda, double d, int shape,
                   int32_t threads, double *out)
{
    if (threads < 0)
        return -1;
    if (threads > 0)
        omp_set_num_threads(threads);
    const int64_t P = m->P;
    double *centre = (double *)malloc(sizeof(double) * 3 * (size_t)(P > 0 ? P : 1));
    double *a = (double *)malloc(sizeof(double) * 3 * (size_t)(P > 0 ? P : 1));
    double *b = (double *)malloc(sizeof(double) * 3 * (size_t)(P > 0 ? P : 1));
    if (!centre || !a || !b) {
        free(centre), free(a), free(b);
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        cell_centre(m, p, centre + 3 * p);
        memcpy(a + 3 * p, centre + 3 * p, 3 * sizeof(double));
    }
    for (int32_t it = 0; it < iterations; ++it) {
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < P; ++p) {
            const int64_t n = m->st_off[p + 1] - m->st_off[p];
            double q[3];
            for (int ax = 0; ax < 3; ++ax) {
                q[ax] = a[3 * p + ax];
                if (n > 0) {
                    double sum = 0.0;
                    for (int64_t e = m->st_off[p]; e < m->st_off[p + 1]; ++e)
                        sum += a[3 * (int64_t)m->st_ids[e] + ax] - a[3 * p + ax];
                    q[ax] = a[3 * p + ax] + lambda * (sum / (double)n);
                }
            }
            const double *c = centre + 3 * p;
            if (shape == 1) {
                const double dx = q[0] - c[0], dy = q[1] - c[1], dz = q[2] - c[2];
                const double len = sqrt(dx * dx + dy * dy + dz * dz);
                if (len > d) {
                    q[0] = c[0] + dx * (d / len);
                    q[1] = c[1] + dy * (d / len);
                    q[2] = c[2] + dz * (d / len);
                }
            } else {
                for (int ax = 0; ax < 3; ++ax) {
                    if (q[ax] < c[ax] - d) q[ax] = c[ax] - d;
                    if (q[ax] > c[ax] + d) q[ax] = c[ax] + d;
                }
            }
            memcpy(b + 3 * p, q, sizeof q);
        }
        double *t = a;
        a = b;
        b = t;
    }
    memcpy(out, a, sizeof(double) * 3 * (size_t)P);
    free(centre), free(a), free(b);
    return 0;
}

/* threads an OpenMP parallel region of this library gets by default */
int32_t orc_par_max_threads(void) { return (int32_t)omp_get_max_threads(); }
