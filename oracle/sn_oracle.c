/*
 * SurfaceNets oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, deliberately slow CPU statement of what the SurfaceNets
 * method computes (Schroeder, Tsalikis, Halle, Frisken, "A High-Performance
 * SurfaceNets Discrete Isocontouring Algorithm").  It is used by the tests,
 * by the package smoke check and by the benchmark's CPU-baseline leg, and by
 * nothing else.  It shares no code, header, table or helper with the GPU
 * library.
 *
 * The extraction reaches an exact combinatorial result, so this file writes
 * that result's plain definition out directly, cell by cell and edge by edge,
 * with none of the paper's triads, trims, checkerboards or prefix sums:
 *
 *   classification    Sec. 2.1 (Notation): a value in the selected label set L
 *                     keeps its identity; any other value is background B.
 *   cut edge          Sec. 2.2: a lattice edge (s0,s1) is intersected iff
 *                     s0 != s1 and not both lie in B, i.e. C(s0) != C(s1).
 *   point             Sec. 2.2 / Sec. 3.5: a cell gets one point, at its
 *                     centre, iff any of its 12 edges is cut.
 *   quad              Sec. 2.2: one quad per cut edge, joining the points of
 *                     the four cells that share that edge; regions touching the
 *                     volume faces stay open (Sec. 4.2), so an edge on the
 *                     boundary of the cell grid emits no quad.
 *   label pair        Sec. 2.2: each quad carries the labels of the regions on
 *                     its two sides.
 *   stencil           Sec. 2.2 and Sec. 3.3: a point is linked to the point of a
 *                     face-neighbour cell iff the shared face holds a cut edge.
 *   smoothing         Eq. (1), Sec. 2.2, with the per-cell box constraint and
 *                     the double-buffered (Jacobi) update of Sec. 2.4.
 *   triangulation     Sec. 2.5: every quad becomes two triangles.
 *   2D                Sec. 5 (the method exists in 2D and 3D): the same
 *                     definitions on an image; see orc_extract2d.
 *
 * Readings of points the paper leaves open (all restated in the design notes):
 *   - point ids follow the cell linear index i + (M-1)(j + (N-1)k);
 *   - quads follow the lattice linear index i + M(j + Nk) of the edge origin
 *     s0, then axis x, y, z; vertex order, for the axis-a edge at (i,j,k):
 *       x: (i,j-1,k-1) (i,j-1,k) (i,j,k) (i,j,k-1)
 *       y: (i-1,j,k-1) (i,j,k-1) (i,j,k) (i-1,j,k)
 *       z: (i-1,j-1,k) (i-1,j,k) (i,j,k) (i,j-1,k)
 *     (right-hand normal along -a) and label pair (front, back) = (C(s0), C(s1));
 *   - stencil entries in face order -x, +x, -y, +y, -z, +z;
 *   - Eq. (1) is the mean over the N stencil neighbours; N = 0 means no motion;
 *   - the constraint is a box of half-width d (voxel units) per axis around
 *     the cell centre, or a sphere of radius d, applied after every sweep;
 *   - the triangles of quad (A,B,C,D) are (A,B,C) and (A,C,D);
 *   - the other tessellating diagonals Sec. 2.5 lists are read in
 *     orc_triangulate_rule below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t M, N, O;      /* lattice (sample) dimensions (O = 1: an image)       */
    int64_t P, Q, S;      /* points, quads (segments in 2D), directed stencil    */
    int32_t nv;           /* point ids per quad: 4, or 2 for the segments of 2D   */
    int64_t *cell_of;     /* [P]   linear cell index of each point               */
    int32_t *quads;       /* [Q*nv] point ids                                     */
    uint32_t *pairs;      /* [Q*2] (front, back) classified labels               */
    int64_t *st_off;      /* [P+1] CSR offsets                                    */
    int32_t *st_ids;      /* [S]   neighbour point ids                            */
} orc_mesh;

static uint32_t raw_label(const void *vol, int b, int64_t idx)
{
    if (b == 1)
        return ((const uint8_t *)vol)[idx];
    if (b == 2)
        return ((const uint16_t *)vol)[idx];
    return ((const uint32_t *)vol)[idx];
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Sec. 2.1: C(v) = v when v is a selected label, the background value
 * otherwise.  An empty selection selects every value except the background. */
static uint32_t classify(uint32_t v, const uint32_t *sorted_sel, int32_t n_sel, uint32_t bg)
{
    if (v == bg)
        return bg;
    if (n_sel == 0)
        return v;
    return bsearch(&v, sorted_sel, (size_t)n_sel, sizeof(uint32_t), cmp_u32) ? v : bg;
}

/* classified volume, filled once per extraction */
typedef struct {
    const uint32_t *c;
    int64_t M, N, O;
} cvol;

static uint32_t C(const cvol *v, int64_t i, int64_t j, int64_t k)
{
    return v->c[i + v->M * (j + v->N * k)];
}

/* Sec. 2.2: the lattice edge from (i,j,k) along axis a is cut iff the two
 * classified end values differ.  Edges leaving the lattice do not exist. */
static int cut(const cvol *v, int64_t i, int64_t j, int64_t k, int a)
{
    int64_t i1 = i + (a == 0), j1 = j + (a == 1), k1 = k + (a == 2);
    if (i < 0 || j < 0 || k < 0 || i1 >= v->M || j1 >= v->N || k1 >= v->O)
        return 0;
    return C(v, i, j, k) != C(v, i1, j1, k1);
}

static int cell_exists(const cvol *v, int64_t i, int64_t j, int64_t k)
{
    return i >= 0 && j >= 0 && k >= 0 && i <= v->M - 2 && j <= v->N - 2 && k <= v->O - 2;
}

/* Sec. 2.2: the twelve edges of cell (i,j,k): four along each axis. */
static int cell_has_point(const cvol *v, int64_t i, int64_t j, int64_t k)
{
    for (int64_t p = 0; p <= 1; ++p)
        for (int64_t q = 0; q <= 1; ++q) {
            if (cut(v, i, j + p, k + q, 0)) return 1; /* x-edges */
            if (cut(v, i + p, j, k + q, 1)) return 1; /* y-edges */
            if (cut(v, i + p, j + q, k, 2)) return 1; /* z-edges */
        }
    return 0;
}

/* Sec. 3.3: face f (0..5 = -x,+x,-y,+y,-z,+z) of cell (i,j,k) holds a cut
 * edge.  The face lies in the lattice plane x = i (or i+1, etc.) and is
 * bounded by two edges along each of the two other axes. */
static int face_has_cut(const cvol *v, int64_t i, int64_t j, int64_t k, int f)
{
    int axis = f / 2, plus = f % 2;
    if (axis == 0) {
        int64_t x = i + plus;
        return cut(v, x, j, k, 1) || cut(v, x, j, k + 1, 1) || cut(v, x, j, k, 2) ||
               cut(v, x, j + 1, k, 2);
    }
    if (axis == 1) {
        int64_t y = j + plus;
        return cut(v, i, y, k, 0) || cut(v, i, y, k + 1, 0) || cut(v, i, y, k, 2) ||
               cut(v, i + 1, y, k, 2);
    }
    int64_t z = k + plus;
    return cut(v, i, j, z, 0) || cut(v, i, j + 1, z, 0) || cut(v, i, j, z, 1) ||
           cut(v, i + 1, j, z, 1);
}

void orc_mesh_free(orc_mesh *m)
{
    if (!m)
        return;
    free(m->cell_of);
    free(m->quads);
    free(m->pairs);
    free(m->st_off);
    free(m->st_ids);
    free(m);
}

/*
 * Extraction.  `labels` is a host array of M*N*O values of b bytes (x fastest).
 * Returns NULL on allocation failure or bad arguments.
 */
orc_mesh *orc_extract(const void *labels, int b, int64_t M, int64_t N, int64_t O,
                      const uint32_t *selected, int32_t n_sel, uint32_t background)
{
    if (M < 1 || N < 1 || O < 1 || (b != 1 && b != 2 && b != 4) || n_sel < 0)
        return NULL;
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    if (!m)
        return NULL;
    m->M = M, m->N = N, m->O = O;
    m->nv = 4;
    const int64_t V = M * N * O;
    uint32_t *sel = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n_sel > 0 ? n_sel : 1));
    uint32_t *cv = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)V);
    if (!sel || !cv) {
        free(sel), free(cv), free(m);
        return NULL;
    }
    if (n_sel > 0)
        memcpy(sel, selected, sizeof(uint32_t) * (size_t)n_sel);
    qsort(sel, (size_t)n_sel, sizeof(uint32_t), cmp_u32);
    for (int64_t t = 0; t < V; ++t)
        cv[t] = classify(raw_label(labels, b, t), sel, n_sel, background);
    free(sel);
    cvol v = {cv, M, N, O};

    const int64_t CM = M - 1, CN = N - 1, CO = O - 1;
    const int64_t ncell = (CM > 0 && CN > 0 && CO > 0) ? CM * CN * CO : 0;
    int64_t *pid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));

    /* points: cells in ascending linear index */
    int64_t P = 0;
    for (int64_t k = 0; k < CO; ++k)
        for (int64_t j = 0; j < CN; ++j)
            for (int64_t i = 0; i < CM; ++i) {
                int64_t c = i + CM * (j + CN * k);
                pid[c] = cell_has_point(&v, i, j, k) ? P++ : -1;
            }
    m->P = P;
    m->cell_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P > 0 ? P : 1));
    for (int64_t c = 0; c < ncell; ++c)
        if (pid[c] >= 0)
            m->cell_of[pid[c]] = c;
#define PID(i, j, k) pid[(i) + CM * ((j) + CN * (k))]

    /* quads: lattice points in ascending linear index, then axis x, y, z */
    int64_t Q = 0, cap = 16;
    int32_t *qd = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)cap);
    uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (size_t)cap);
    for (int64_t k = 0; k < O; ++k)
        for (int64_t j = 0; j < N; ++j)
            for (int64_t i = 0; i < M; ++i)
                for (int a = 0; a < 3; ++a) {
                    if (!cut(&v, i, j, k, a))
                        continue;
                    int64_t c4[4][3];
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
                    int ok = 1;
                    for (int q = 0; q < 4; ++q)
                        ok &= cell_exists(&v, c4[q][0], c4[q][1], c4[q][2]);
                    if (!ok)
                        continue; /* open boundary: no quad on the cell-grid boundary */
                    if (Q == cap) {
                        cap *= 2;
                        qd = (int32_t *)realloc(qd, sizeof(int32_t) * 4 * (size_t)cap);
                        pr = (uint32_t *)realloc(pr, sizeof(uint32_t) * 2 * (size_t)cap);
                    }
                    for (int q = 0; q < 4; ++q)
                        qd[4 * Q + q] = (int32_t)PID(c4[q][0], c4[q][1], c4[q][2]);
                    pr[2 * Q + 0] = C(&v, i, j, k);
                    pr[2 * Q + 1] = C(&v, i + (a == 0), j + (a == 1), k + (a == 2));
                    ++Q;
                }
    m->Q = Q;
    m->quads = qd;
    m->pairs = pr;

    /* stencil: points in id order, faces -x,+x,-y,+y,-z,+z */
    m->st_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P + 1));
    int64_t S = 0, scap = 16;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)scap);
    for (int64_t p = 0; p < P; ++p) {
        m->st_off[p] = S;
        int64_t c = m->cell_of[p];
        int64_t i = c % CM, j = (c / CM) % CN, k = c / (CM * CN);
        for (int f = 0; f < 6; ++f) {
            int64_t d = (f % 2) ? 1 : -1;
            int64_t ni = i + (f / 2 == 0) * d, nj = j + (f / 2 == 1) * d, nk = k + (f / 2 == 2) * d;
            if (!cell_exists(&v, ni, nj, nk) || !face_has_cut(&v, i, j, k, f))
                continue;
            if (S == scap) {
                scap *= 2;
                ids = (int32_t *)realloc(ids, sizeof(int32_t) * (size_t)scap);
            }
            ids[S++] = (int32_t)PID(ni, nj, nk);
        }
    }
    m->st_off[P] = S;
    m->S = S;
    m->st_ids = ids;
#undef PID
    free(pid);
    free(cv);
    return m;
}

void orc_mesh_sizes(const orc_mesh *m, int64_t *out4)
{
    out4[0] = m->P, out4[1] = m->Q, out4[2] = m->S;
    out4[3] = 2 * m->Q;
}

/* Copy results out; any NULL destination is skipped. */
void orc_mesh_copy(const orc_mesh *m, int64_t *cell_of, int32_t *quads, uint32_t *pairs,
                   int64_t *st_off, int32_t *st_ids)
{
    if (cell_of) memcpy(cell_of, m->cell_of, sizeof(int64_t) * (size_t)m->P);
    if (quads) memcpy(quads, m->quads, sizeof(int32_t) * (size_t)m->nv * (size_t)m->Q);
    if (pairs) memcpy(pairs, m->pairs, sizeof(uint32_t) * 2 * (size_t)m->Q);
    if (st_off) memcpy(st_off, m->st_off, sizeof(int64_t) * (size_t)(m->P + 1));
    if (st_ids) memcpy(st_ids, m->st_ids, sizeof(int32_t) * (size_t)m->S);
}

/*
 * 2D.  An image of M x N samples, x fastest; cell (i,j), 0 <= i <= M-2,
 * 0 <= j <= N-2, spans samples (i..i+1, j..j+1).  The 3D definitions restated
 * in the plane:
 *   point    a cell gets one point, at its centre, iff any of its four edges
 *            (x-edges from (i,j) and (i,j+1), y-edges from (i,j) and (i+1,j))
 *            is cut;
 *   segment  one per cut edge, joining the points of the two cells that
 *            share it; an edge on the boundary of the cell grid emits none.
 *            Order: lattice linear index i + M j of the edge origin s0, then
 *            axis x, y.  Vertex order, with the right-hand normal facing s0 as
 *            for the quads: x-edge at (i,j): (i,j) (i,j-1); y-edge at (i,j):
 *            (i-1,j) (i,j).  Label pair (front, back) = (C(s0), C(s1));
 *   stencil  a point is linked to the point of an edge-neighbour cell iff
 *            their shared edge is cut; order -x, +x, -y, +y.
 * Points are cell centres as in 3D with k = 0; smoothing (orc_smooth_shape)
 * is unchanged and leaves the z coordinate alone (no point has a z neighbour).
 */
static int cell2_exists(int64_t M, int64_t N, int64_t i, int64_t j)
{
    return i >= 0 && j >= 0 && i <= M - 2 && j <= N - 2;
}

orc_mesh *orc_extract2d(const void *labels, int b, int64_t M, int64_t N, const uint32_t *selected,
                        int32_t n_sel, uint32_t background)
{
    if (M < 1 || N < 1 || (b != 1 && b != 2 && b != 4) || n_sel < 0)
        return NULL;
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    if (!m)
        return NULL;
    m->M = M, m->N = N, m->O = 1;
    m->nv = 2;
    const int64_t V = M * N;
    uint32_t *sel = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n_sel > 0 ? n_sel : 1));
    uint32_t *cv = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)V);
    if (!sel || !cv) {
        free(sel), free(cv), free(m);
        return NULL;
    }
    if (n_sel > 0)
        memcpy(sel, selected, sizeof(uint32_t) * (size_t)n_sel);
    qsort(sel, (size_t)n_sel, sizeof(uint32_t), cmp_u32);
    for (int64_t t = 0; t < V; ++t)
        cv[t] = classify(raw_label(labels, b, t), sel, n_sel, background);
    free(sel);
    cvol v = {cv, M, N, 1};

    const int64_t CM = M - 1, CN = N - 1;
    const int64_t ncell = (CM > 0 && CN > 0) ? CM * CN : 0;
    int64_t *pid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    int64_t P = 0;
    for (int64_t j = 0; j < CN; ++j)
        for (int64_t i = 0; i < CM; ++i) {
            const int pt = cut(&v, i, j, 0, 0) || cut(&v, i, j + 1, 0, 0) || cut(&v, i, j, 0, 1) ||
                           cut(&v, i + 1, j, 0, 1);
            pid[i + CM * j] = pt ? P++ : -1;
        }
    m->P = P;
    m->cell_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P > 0 ? P : 1));
    for (int64_t c = 0; c < ncell; ++c)
        if (pid[c] >= 0)
            m->cell_of[pid[c]] = c;

    int64_t Q = 0, cap = 16;
    int32_t *sg = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)cap);
    uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (size_t)cap);
    for (int64_t j = 0; j < N; ++j)
        for (int64_t i = 0; i < M; ++i)
            for (int a = 0; a < 2; ++a) {
                if (!cut(&v, i, j, 0, a))
                    continue;
                /* the two cells sharing the edge, in vertex order */
                const int64_t ai = a == 0 ? i : i - 1, aj = a == 0 ? j : j;
                const int64_t bi = a == 0 ? i : i, bj = a == 0 ? j - 1 : j;
                if (!cell2_exists(M, N, ai, aj) || !cell2_exists(M, N, bi, bj))
                    continue;
                if (Q == cap) {
                    cap *= 2;
                    sg = (int32_t *)realloc(sg, sizeof(int32_t) * 2 * (size_t)cap);
                    pr = (uint32_t *)realloc(pr, sizeof(uint32_t) * 2 * (size_t)cap);
                }
                sg[2 * Q + 0] = (int32_t)pid[ai + CM * aj];
                sg[2 * Q + 1] = (int32_t)pid[bi + CM * bj];
                pr[2 * Q + 0] = C(&v, i, j, 0);
                pr[2 * Q + 1] = C(&v, i + (a == 0), j + (a == 1), 0);
                ++Q;
            }
    m->Q = Q;
    m->quads = sg;
    m->pairs = pr;

    m->st_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P + 1));
    int64_t S = 0, scap = 16;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)scap);
    for (int64_t p = 0; p < P; ++p) {
        m->st_off[p] = S;
        const int64_t c = m->cell_of[p], i = c % CM, j = c / CM;
        /* neighbour cell and the edge the two cells share, per face */
        const int64_t ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
        const int shared[4] = {cut(&v, i, j, 0, 1), cut(&v, i + 1, j, 0, 1), cut(&v, i, j, 0, 0),
                               cut(&v, i, j + 1, 0, 0)};
        for (int f = 0; f < 4; ++f) {
            if (!cell2_exists(M, N, ni[f], nj[f]) || !shared[f])
                continue;
            if (S == scap) {
                scap *= 2;
                ids = (int32_t *)realloc(ids, sizeof(int32_t) * (size_t)scap);
            }
            ids[S++] = (int32_t)pid[ni[f] + CM * nj[f]];
        }
    }
    m->st_off[P] = S;
    m->S = S;
    m->st_ids = ids;
    free(pid);
    free(cv);
    return m;
}

/* Sec. 2.2: the generated point sits at the centre of its cell. */
static void cell_centre(const orc_mesh *m, int64_t p, double *x)
{
    int64_t CM = m->M - 1, CN = m->N - 1;
    int64_t c = m->cell_of[p];
    x[0] = (double)(c % CM) + 0.5;
    x[1] = (double)((c / CM) % CN) + 0.5;
    x[2] = (double)(c / (CM * CN)) + 0.5;
}

/*
 * Constrained Laplacian smoothing in index (voxel) space, FP64.
 * Eq. (1): p_i <- p_i + lambda * (1/N) * sum_j (p_j - p_i) over the N stencil
 * neighbours of p_i; the moved point is then held inside its constraint
 * region around its cell centre (Sec. 2.2, which names a fraction of the
 * voxel cell or a sphere): shape 0, the box of half-width d per axis
 * (clamped axis by axis); shape 1, the sphere of radius d (a point outside is
 * moved back along the ray from the centre onto the sphere).  All points are
 * updated from the previous sweep's positions (double buffering, Sec. 2.4).
 * out: [P*3] positions after `iterations` sweeps.  Returns 0 on success.
 */
int orc_smooth_shape(const orc_mesh *m, int32_t iterations, double lambda, double d, int shape,
                     double *out)
{
    const int64_t P = m->P;
    double *centre = (double *)malloc(sizeof(double) * 3 * (size_t)(P > 0 ? P : 1));
    double *a = (double *)malloc(sizeof(double) * 3 * (size_t)(P > 0 ? P : 1));
    double *b = (double *)malloc(sizeof(double) * 3 * (size_t)(P > 0 ? P : 1));
    if (!centre || !a || !b) {
        free(centre), free(a), free(b);
        return -1;
    }
    for (int64_t p = 0; p < P; ++p) {
        cell_centre(m, p, centre + 3 * p);
        memcpy(a + 3 * p, centre + 3 * p, 3 * sizeof(double));
    }
    for (int32_t it = 0; it < iterations; ++it) {
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

/* The box constraint (shape 0). */
int orc_smooth(const orc_mesh *m, int32_t iterations, double lambda, double d, double *out)
{
    return orc_smooth_shape(m, iterations, lambda, d, 0, out);
}

/* Index-space centres of all points (the unsmoothed positions). */
void orc_centres(const orc_mesh *m, double *out)
{
    for (int64_t p = 0; p < m->P; ++p)
        cell_centre(m, p, out + 3 * p);
}

/* World coordinates: origin + spacing * index-space position (per axis). */
void orc_world(int64_t P, const double *idx_pos, const double *origin, const double *spacing,
               double *out)
{
    for (int64_t p = 0; p < P; ++p)
        for (int ax = 0; ax < 3; ++ax)
            out[3 * p + ax] = origin[ax] + spacing[ax] * idx_pos[3 * p + ax];
}

/* Sec. 2.5: quad (A,B,C,D) -> triangles (A,B,C), (A,C,D); pairs repeated. */
void orc_triangulate(const orc_mesh *m, int32_t *tris, uint32_t *tri_pairs)
{
    for (int64_t q = 0; q < m->Q; ++q) {
        const int32_t *v = m->quads + 4 * q;
        int32_t *t0 = tris + 6 * q, *t1 = tris + 6 * q + 3;
        t0[0] = v[0], t0[1] = v[1], t0[2] = v[2];
        t1[0] = v[0], t1[1] = v[2], t1[2] = v[3];
        if (tri_pairs) {
            tri_pairs[4 * q + 0] = m->pairs[2 * q + 0];
            tri_pairs[4 * q + 1] = m->pairs[2 * q + 1];
            tri_pairs[4 * q + 2] = m->pairs[2 * q + 0];
            tri_pairs[4 * q + 3] = m->pairs[2 * q + 1];
        }
    }
}

/*
 * Sec. 2.5 lists ways to choose the tessellating diagonal of a (non-planar,
 * smoothed) quad without defining them; the readings, for quad (A,B,C,D) with
 * world points a, b, c, d:
 *   split AC: triangles (A,B,C), (A,C,D);  split BD: (A,B,D), (B,C,D)
 *   (both keep the quad's orientation);
 *   rule 0 fixed:        always AC;
 *   rule 1 shortest:     AC iff |c - a| <= |d - b|;
 *   rule 2 minimum area: AC iff area(ABC) + area(ACD) <= area(ABD) + area(BCD);
 *   rule 3 most planar:  AC iff the cosine of the angle between the normals of
 *                        its two triangles is >= that of the BD split (a split
 *                        with a degenerate triangle has cosine -2, never
 *                        preferred unless both are degenerate).
 * Ties go to AC.  pts: world points [P*3] (FP64); tris: [2Q*3].
 */
static void vsub(const double *x, const double *y, double *r)
{
    r[0] = x[0] - y[0], r[1] = x[1] - y[1], r[2] = x[2] - y[2];
}

static void vcross(const double *x, const double *y, double *r)
{
    r[0] = x[1] * y[2] - x[2] * y[1];
    r[1] = x[2] * y[0] - x[0] * y[2];
    r[2] = x[0] * y[1] - x[1] * y[0];
}

static double vdot(const double *x, const double *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; }

/* normal (y - x) x (z - x) of triangle (x, y, z) */
static void tri_normal(const double *x, const double *y, const double *z, double *n)
{
    double u[3], v[3];
    vsub(y, x, u);
    vsub(z, x, v);
    vcross(u, v, n);
}

static double tri_area(const double *x, const double *y, const double *z)
{
    double n[3];
    tri_normal(x, y, z, n);
    return 0.5 * sqrt(vdot(n, n));
}

static double normals_cos(const double *n1, const double *n2)
{
    const double l = sqrt(vdot(n1, n1) * vdot(n2, n2));
    return l > 0.0 ? vdot(n1, n2) / l : -2.0;
}

/* 1 if quad (a,b,c,d) is split along AC under `rule`, 0 for BD */
int orc_split_ac(const double *a, const double *b, const double *c, const double *d, int rule)
{
    if (rule == 1) {
        double ac[3], bd[3];
        vsub(c, a, ac);
        vsub(d, b, bd);
        return vdot(ac, ac) <= vdot(bd, bd);
    }
    if (rule == 2)
        return tri_area(a, b, c) + tri_area(a, c, d) <= tri_area(a, b, d) + tri_area(b, c, d);
    if (rule == 3) {
        double n1[3], n2[3], n3[3], n4[3];
        tri_normal(a, b, c, n1);
        tri_normal(a, c, d, n2);
        tri_normal(a, b, d, n3);
        tri_normal(b, c, d, n4);
        return normals_cos(n1, n2) >= normals_cos(n3, n4);
    }
    return 1;
}

void orc_triangulate_rule(int64_t Q, const int32_t *quads, const double *pts, int rule, int32_t *tris)
{
    for (int64_t q = 0; q < Q; ++q) {
        const int32_t *v = quads + 4 * q;
        const double *a = pts + 3 * (int64_t)v[0], *b = pts + 3 * (int64_t)v[1];
        const double *c = pts + 3 * (int64_t)v[2], *d = pts + 3 * (int64_t)v[3];
        int32_t *t0 = tris + 6 * q, *t1 = tris + 6 * q + 3;
        if (orc_split_ac(a, b, c, d, rule)) {
            t0[0] = v[0], t0[1] = v[1], t0[2] = v[2];
            t1[0] = v[0], t1[1] = v[2], t1[2] = v[3];
        } else {
            t0[0] = v[0], t0[1] = v[1], t0[2] = v[3];
            t1[0] = v[1], t1[1] = v[2], t1[2] = v[3];
        }
    }
}
