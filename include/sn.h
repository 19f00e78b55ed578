/*
 * sn.h -- C ABI of libsn.so: SurfaceNets surface extraction and constrained
 * smoothing of 3D integer label maps on an AMD Instinct MI355X (gfx950).
 *
 * The method is that of Schroeder, Tsalikis, Halle and Frisken, "A
 * High-Performance SurfaceNets Discrete Isocontouring Algorithm":
 *   - extraction (Sec. 2.2, 2.3): one point at the centre of every voxel cell
 *     with an intersected edge, one quad per intersected edge joining the four
 *     cells around it, a region-label pair per quad and a smoothing stencil
 *     linking face-neighbour cells;
 *   - smoothing (Eq. (1), Sec. 2.2, 2.4): double-buffered Laplacian relaxation
 *     of the points, each held inside a box or a sphere around its cell centre;
 *   - triangulation (Sec. 2.5): two triangles per quad.
 *
 * Conventions (all counts are int64; ids inside meshes are int32):
 *   - A label volume is x-fastest: value (i,j,k) at i + M*(j + N*k), where
 *     dims = {M, N, O} are the numbers of samples along x, y, z.
 *   - Classification (Sec. 2.1): a value is kept if it is selected and is not
 *     the background value; every other value becomes the background value.
 *     n_selected == 0 selects every value except the background.  An edge is
 *     intersected iff its two classified end values differ (Sec. 2.2).
 *   - Cell (i,j,k), 0 <= i < M-1 etc., spans samples (i..i+1, j..j+1, k..k+1).
 *     Point ids follow the cell linear index i + (M-1)*(j + (N-1)*k).
 *   - The quad of the intersected edge from sample s0=(i,j,k) to s1 = s0 + e_a
 *     exists iff all four cells around the edge exist (regions that touch the
 *     volume faces stay open, Sec. 4.2).  Quads are ordered by the sample
 *     linear index of s0, then by axis x, y, z.  Vertex order for the edge at
 *     (i,j,k) (right-hand normal along -e_a, i.e. facing s0):
 *        x: (i,j-1,k-1) (i,j-1,k) (i,j,k) (i,j,k-1)
 *        y: (i-1,j,k-1) (i,j,k-1) (i,j,k) (i-1,j,k)
 *        z: (i-1,j-1,k) (i-1,j,k) (i,j,k) (i,j-1,k)
 *     label_pairs[q] = (front, back) = (class(s0), class(s1)), stored in the
 *     input dtype.
 *   - Stencil (Sec. 2.2, 3.3): cell c links to face neighbour n iff n exists
 *     and the shared face holds an intersected edge; entries are in face
 *     order -x, +x, -y, +y, -z, +z, stored as CSR (offsets [P+1], ids [S]).
 *   - Points are world coordinates origin + spacing * (i+1/2+dx, j+1/2+dy,
 *     k+1/2+dz) in float32, xyz interleaved; d = (dx,dy,dz) are the
 *     cell-relative offsets ("offsets"), zero before smoothing.
 *   - Smoothing, per sweep: d <- clamp(d + lambda * mean_n(e_n + d_n - d),
 *     -c, c) per axis, where e_n is the unit step to neighbour n and c is the
 *     constraint distance in voxel units; no neighbours -> no motion.  With
 *     the sphere constraint the moved d is instead scaled back to length c
 *     when it is longer.
 *   - Triangles (SN_TRIS): quad (A,B,C,D) -> (A,B,C), (A,C,D); triangle 2q
 *     and 2q+1 come from quad q and repeat its label pair.
 *   - Images (SN_LINES, dims[2] == 1): the same definitions in the plane.
 *     Cell (i,j) spans samples (i..i+1, j..j+1) and has a point iff any of
 *     its four edges is intersected; one segment per intersected edge joins
 *     the points of the two cells sharing it (none on the cell-grid
 *     boundary), ordered by the sample linear index of s0, then axis x, y,
 *     with vertex order x: (i,j) (i,j-1), y: (i-1,j) (i,j) (right-hand
 *     normal facing s0) and label pair (class(s0), class(s1)).  The stencil
 *     links edge neighbours across an intersected edge (faces -x, +x, -y,
 *     +y).  Points are xyz with z = origin[2] and stay in that plane under
 *     smoothing (spacing[2] is not used).
 *
 * Memory: `labels` is a DEVICE pointer owned by the caller; every sn_mesh and
 * everything it points to is device memory owned by the library until
 * sn_mesh_free.  Host arrays passed in (selected labels, parameters) are
 * copied during the call.  Streams are passed as `void*` holding a
 * hipStream_t (NULL = the legacy default stream).
 *
 * Errors: every call returns an sn_status; out-parameters are written only on
 * SN_OK; nothing throws across the ABI.  sn_strerror() names a status.
 *
 * Threads: the plain, batched, tuning and profiling calls on one sn_ctx come
 * from one host thread at a time; a server's worker threads share its
 * context safely with that thread, and the sn_serve_* calls are thread-safe.
 */
#ifndef SN_H
#define SN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sn_status {
    SN_OK = 0,
    SN_EINVAL = -1,     /* a bad argument (message via sn_last_error)            */
    SN_ENOMEM = -2,     /* device memory (or the configured budget) exhausted    */
    SN_EDEVICE = -3,    /* a HIP runtime error                                   */
    SN_ETOOBIG = -4,    /* a point id, quad or stencil index exceeds int32       */
    SN_EAGAIN = -5,     /* serve: queue full, or the ticket is not finished yet  */
    SN_ENOTFOUND = -6,  /* serve: unknown ticket                                 */
    SN_ESHUTDOWN = -7,  /* serve: the server is stopping                         */
    SN_ETIMEDOUT = -8   /* serve: wait timed out                                 */
} sn_status;

typedef enum sn_dtype { SN_U8 = 1, SN_U16 = 2, SN_U32 = 4 } sn_dtype;
/* SN_LINES: the 2D method (Sec. 5: SurfaceNets exists in 2D and 3D) on an
 * image, dims = {M, N, 1}: contour segments instead of quads; see below. */
typedef enum sn_prim { SN_LINES = 2, SN_TRIS = 3, SN_QUADS = 4 } sn_prim;

typedef struct sn_ctx sn_ctx;
typedef struct sn_mesh sn_mesh;
typedef struct sn_server sn_server;

/* One label volume and its extraction parameters (Sec. 2.1, 2.2, 2.5). */
typedef struct sn_volume {
    const void *labels;        /* device, dims[0]*dims[1]*dims[2] values, x fastest,
                                  aligned to the dtype                                    */
    int32_t dtype;             /* sn_dtype: bytes per label                               */
    int64_t dims[3];           /* M, N, O >= 1; a dim below 2 gives an empty mesh (O = 1
                                  for SN_LINES)                                            */
    double spacing[3];         /* > 0 and finite                                          */
    double origin[3];          /* world position of sample (0,0,0)                        */
    const uint32_t *selected;  /* host; duplicates allowed                                */
    int32_t n_selected;        /* 0: every value except the background                    */
    uint32_t background;       /* must fit the dtype; must not be in `selected`           */
    int32_t prim;              /* sn_prim                                                 */
} sn_volume;

/* Region a smoothed point is held in, around its cell centre, in voxel units
 * (Sec. 2.2 names a fraction of the voxel cell, or a sphere). */
typedef enum sn_constraint_shape {
    SN_BOX = 0,    /* |delta_a| <= constraint on each axis (clamped per axis)    */
    SN_SPHERE = 1  /* |delta| <= constraint (scaled back onto the sphere)        */
} sn_constraint_shape;

/* Eq. (1) parameters: sweeps >= 0, 0 <= relaxation <= 1, constraint >= 0 (voxels),
 * shape an sn_constraint_shape (0 = box). */
typedef struct sn_smooth_params {
    int32_t iterations;
    float relaxation;
    float constraint;
    int32_t shape;
} sn_smooth_params;

/* Borrowed device pointers, valid until sn_mesh_free. */
typedef struct sn_mesh_view {
    int64_t n_points, n_quads, n_stencil, n_polys;
    int32_t prim, dtype;
    const float *points;        /* [n_points*3] world xyz                                 */
    const float *offsets;       /* [n_points*3] cell-relative offsets; NULL = all zero    */
    const int32_t *polys;       /* [n_polys*prim] point ids                               */
    const void *label_pairs;    /* [n_polys*2] (front, back), dtype bytes each            */
    const int32_t *stencil_off; /* [n_points+1]                                           */
    const int32_t *stencil_ids; /* [n_stencil]                                            */
    const int32_t *quads;       /* [n_quads*4] (same as polys for SN_QUADS; NULL for
                                   SN_LINES, whose polys are the segments [n_quads*2])   */
} sn_mesh_view;

/* ---- context -------------------------------------------------------------- */

/* Bind a context to HIP device `device`.  Reads SN_AUTOTUNE_CACHE (a JSON file
 * of schedule choices) from the environment, and four test knobs, none of
 * which changes results:
 *   SN_TEST_MEM_LIMIT          a byte cap on the library's device pool, to
 *                              force SN_ENOMEM;
 *   SN_TEST_COUNT_WIDE_WORDS   the number of cell words from which an
 *                              extraction counts four words per thread;
 *   SN_TEST_SWEEP_SMALL_POINTS the number of points above which a mesh takes
 *                              the large-mesh sweep form (non-temporal
 *                              accesses, slab-chunked block order; 2^24 by
 *                              default);
 *   SN_TEST_SWEEP_CHUNK        the blocks an XCD takes in turn in that block
 *                              order (default about a sixteenth of a slab). */
sn_status sn_ctx_create(int device, sn_ctx **out);
/* Device memory of the context's pool: the bytes handed out now (meshes and
 * the scratch of calls in progress) and the most ever handed out at once, each
 * block counted at the size asked for, rounded up to the pool's size classes
 * (512 B steps up to 1 MiB, 2 MiB steps above).  Cached free blocks are not
 * counted.  Either pointer may be NULL. */
sn_status sn_ctx_memory(sn_ctx *ctx, int64_t *in_use_bytes, int64_t *peak_bytes);
/* Release the caller's handle.  Meshes and servers made by the context hold
 * it alive: its device memory and streams go when the last of them is freed
 * (sn_mesh_free, sn_serve_stop), so meshes may be freed in any order. */
void sn_ctx_destroy(sn_ctx *ctx);
const char *sn_strerror(sn_status s);
/* Text of the last error raised on this host thread ("" if none). */
const char *sn_last_error(void);
/* Library build identification, e.g. "libsn gfx950 <date>". */
const char *sn_version(void);

/* ---- plain path ----------------------------------------------------------- */

/* Extract the SurfaceNets mesh of one volume (Sec. 2.3).  The call blocks until
 * the output sizes are known (the count pass writes three totals per volume
 * into host memory), then
 * enqueues generation on `stream` and returns; the mesh is complete once
 * `stream` reaches that point.  Points are cell centres; offsets are NULL. */
sn_status sn_extract(sn_ctx *ctx, const sn_volume *vol, void *stream, sn_mesh **out);

/* Smooth a mesh (Eq. (1), Sec. 2.4).  Always restarts from the unsmoothed
 * centres kept with the mesh (the smoothing cache of Sec. 3.7), so repeated
 * calls with different parameters are independent.  Enqueued on `stream`
 * (one launch per sweep).  iterations == 0 restores the centres. */
sn_status sn_smooth(sn_ctx *ctx, sn_mesh *mesh, const sn_smooth_params *p, void *stream);

/* Choice of the tessellating diagonal of a quad (Sec. 2.5 lists shortest
 * diagonal, minimum area and most co-planar without defining the measures). */
typedef enum sn_diag_rule {
    SN_DIAG_FIXED = 0,    /* always A-C: the split SN_TRIS makes at extraction     */
    SN_DIAG_SHORTEST = 1, /* A-C iff |C - A| <= |D - B|                            */
    SN_DIAG_MIN_AREA = 2, /* A-C iff area(ABC) + area(ACD) <= area(ABD) + area(BCD) */
    SN_DIAG_PLANAR = 3    /* A-C iff its two triangle normals are at least as
                             parallel (cosine) as those of the B-D split; a split
                             with a degenerate triangle has cosine -2            */
} sn_diag_rule;

/* Triangulate a mesh's quads from its current world points (Sec. 2.5: the
 * final step, after smoothing).  For quad (A,B,C,D) the A-C split gives
 * triangles (A,B,C), (A,C,D) and the B-D split (A,B,D), (B,C,D): both keep
 * the quad's orientation.  Measures are computed in FP64 from the FP32 world
 * points, in the order written above; ties go to A-C.  Triangles 2q and 2q+1
 * come from quad q.
 *   tris:       DEVICE [2*n_quads][3] int32, owned by the caller;
 *   tri_labels: DEVICE [2*n_quads][2] of the label type (the quad's label
 *               pair, repeated), owned by the caller, or NULL.
 * Works for meshes of either primitive (the quads are kept).  Enqueued on
 * `stream`, which must be ordered after the mesh's smoothing.  SN_EINVAL for
 * a NULL context or mesh, an unknown rule, an SN_LINES mesh (no quads), or
 * tris == NULL with n_quads > 0. */
sn_status sn_triangulate(sn_ctx *ctx, sn_mesh *mesh, sn_diag_rule rule, int32_t *tris,
                         void *tri_labels, void *stream);

sn_status sn_mesh_view_get(const sn_mesh *mesh, sn_mesh_view *out);

/* Synchronous copies of mesh arrays to host memory; a NULL destination skips
 * that array.  Sizes: points/offsets 3*P floats, polys n_polys*prim int32,
 * labels 2*n_polys*dtype bytes, stencil_off P+1, stencil_ids S int32. */
sn_status sn_mesh_copy_to_host(const sn_mesh *mesh, float *points, int32_t *polys, void *labels,
                               int32_t *stencil_off, int32_t *stencil_ids, float *offsets);
/* Releases the mesh without waiting: its device memory returns to the
 * context's pool and is handed out again only after the library's own work
 * on the mesh (on whatever stream it ran) has completed.  Device work of the
 * caller that still reads the mesh's arrays must be complete (or ordered
 * before the library's next use of the memory) when the mesh is freed. */
void sn_mesh_free(sn_mesh *mesh);

/* ---- no device allocation --------------------------------------------------- */

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc, processes that must not grow their device
 * memory after set-up): the
 * extraction of sn_extract written into caller-owned arrays, with every
 * scratch array (cut-edge planes, word metadata, scan status, totals, the
 * classification table) carved from one static device array of
 * SN_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on holds
 * until the process ends.  The call makes no device allocation of any kind.
 *
 * Every sn_extract_noalloc call on a GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other host threads, other streams of work still
 * running) race and give wrong results; calls on one stream, one after the
 * other, are safe.  The array keeps the last call's contents; what must start
 * at zero is cleared by the call's own first kernel.
 *
 * Arrays (DEVICE pointers owned by the caller; capacities in elements):
 *   points       [cap_points*3] float32 world cell centres, as sn_extract;
 *   stencil_off  [cap_points+1] int32 (required, also for an empty mesh);
 *   stencil_ids  [cap_stencil] int32;
 *   polys        [cap_polys*4] int32 quads (SN_QUADS) or [cap_polys*2]
 *                segments (SN_LINES); SN_TRIS is not supported (SN_EINVAL);
 *   label_pairs  [cap_polys*2] of the label type.
 * counts (host, 3 int64) receives (points, polys, stencil entries).
 *
 * The call blocks until the counts are known (Sec. 2.3: they size the
 * outputs), then enqueues generation on `stream` and returns; the arrays are
 * complete once `stream` reaches that point.  Returns SN_ETOOBIG when the
 * volume needs more scratch than SN_NOALLOC_SCRATCH_BYTES
 * (sn_noalloc_scratch_bytes tells how much it needs) or when ids exceed int32,
 * and SN_ENOMEM, with counts written, when the mesh does not fit the given
 * capacities (nothing is generated; call again with larger arrays).  Results
 * equal sn_extract's points, polys, label pairs and stencil bit for bit. */
#define SN_NOALLOC_SCRATCH_BYTES (64ll << 20)
typedef struct sn_extract_arrays {
    float *points;
    int32_t *polys;
    void *label_pairs;
    int32_t *stencil_off;
    int32_t *stencil_ids;
    int64_t cap_points, cap_polys, cap_stencil;
} sn_extract_arrays;
sn_status sn_extract_noalloc(sn_ctx *ctx, const sn_volume *vol, void *stream,
                             const sn_extract_arrays *out, int64_t *counts);
/* Scratch bytes sn_extract_noalloc needs for `vol`; -1 for an invalid volume. */
int64_t sn_noalloc_scratch_bytes(const sn_volume *vol);

/* ---- batched path ---------------------------------------------------------- */

/* Extract and smooth n independent volumes of any sizes together: one
 * counting launch, one readback of all totals, one generation launch and one
 * HIP-graph replay of the smoothing sweeps for the whole batch, with per-volume
 * sweep counts.  per_vol may be NULL (no smoothing).  Each out_meshes[v] equals
 * what sn_extract + sn_smooth give for volume v alone.  On failure no mesh is
 * returned.  The meshes of one call share one completion event; each can be
 * freed on its own at any time.  With SN_BATCH_SWEEPS=eager in the
 * environment when the context is created, the sweeps are launched one by one
 * instead of from a graph (same results). */
sn_status sn_batch_submit(sn_ctx *ctx, const sn_volume *vols, const sn_smooth_params *per_vol,
                          int32_t n, void *stream, sn_mesh **out_meshes);

/* ---- served path ----------------------------------------------------------- */

typedef struct sn_serve_config {
    int64_t hbm_budget_bytes; /* device bytes the server may hold for work and meshes    */
    int32_t max_inflight;     /* requests admitted but not yet finished (>= 1)           */
    int32_t n_streams;        /* concurrent device batches (>= 1)                        */
    int32_t max_batch;        /* requests fused into one batch (>= 1)                    */
    int32_t queue_capacity;   /* pending requests before sn_serve_submit says SN_EAGAIN */
} sn_serve_config;

typedef struct sn_serve_stats {
    int64_t n_submitted, n_done, n_rejected, n_batches;
    int64_t voxels_done, point_iters_done;
    double p50_us, p99_us, mean_us; /* completion - submission, finished requests     */
    double busy_s;                  /* wall time with at least one request in flight  */
    int64_t peak_reserved_bytes;    /* most device bytes reserved at once (see below) */
    int64_t n_split_batches;        /* fused batches that hit SN_ENOMEM and ran their
                                       requests one at a time                          */
    int64_t n_requeued;             /* requests queued again by the second admission
                                       phase (see sn_serve_start)                      */
} sn_serve_stats;

/* Start a request loop on ctx's device.  The server fuses the admitted
 * requests of a round into one batch (continuous batching: requests arriving
 * while batches run join the next free stream) and keeps result meshes
 * device-resident until claimed.  Admission reserves device bytes in two
 * phases, since a mesh's size is known only after its volume is counted
 * (Sec. 2.3):
 *   1. a pending request is admitted when its exact extraction scratch plus
 *      an estimate of its mesh (bytes per voxel of finished requests) fits
 *      the budget next to the reservations in flight;
 *   2. once the batch is counted, the exact mesh bytes (outputs, word
 *      metadata and smoothing buffers) replace the estimate; if they do not
 *      fit, the batch waits for reservations to be released, or, when every
 *      other batch in flight is waiting too, goes back to the head of the
 *      queue with its exact sizes (n_requeued).
 * Bytes are counted as sn_ctx_memory counts them; a request that alone
 * exceeds the budget runs when nothing else is in flight.  A fused batch that
 * still fails with SN_ENOMEM runs its requests one at a time
 * (n_split_batches). */
sn_status sn_serve_start(sn_ctx *ctx, const sn_serve_config *cfg, sn_server **out);
/* Queue a request.  The labels are read on the server's own streams after the
 * work enqueued on `stream` (a hipStream_t; NULL = the legacy default stream)
 * up to this call has completed, so they may still be being written there;
 * they must stay valid until the ticket is done. */
sn_status sn_serve_submit(sn_server *srv, const sn_volume *vol, const sn_smooth_params *p,
                          void *stream, uint64_t *ticket);
/* SN_OK and the mesh (ownership passes to the caller) once done; SN_EAGAIN
 * if not yet; the request's own error status if it failed. */
sn_status sn_serve_poll(sn_server *srv, uint64_t ticket, sn_mesh **out);
/* As poll, but blocks up to timeout_us (< 0: forever); SN_ETIMEDOUT on expiry. */
sn_status sn_serve_wait(sn_server *srv, uint64_t ticket, int64_t timeout_us, sn_mesh **out);
sn_status sn_serve_stats_get(sn_server *srv, sn_serve_stats *out);
/* Drain in-flight work, reject queued requests, stop the loop, free the server. */
sn_status sn_serve_stop(sn_server *srv);

/* ---- schedule tuning and profiling ----------------------------------------- */

/* Pick the schedule (sn_schedule below) for the volume's size class on this
 * device by timing: one knob at a time, with the others at their best so far,
 * over the k_edges segments per wave (1, 2, 4, 8), the k_count form (1 or 4
 * words per thread), the k_generate groups per wave (1, 2, 3, 4, 8), and, when
 * the volume's mesh takes the large-mesh sweep form, the block-order chunk
 * (half, once and twice the default; four sweeps timed each).  The choice is
 * remembered for the class (and written to SN_AUTOTUNE_CACHE if set).
 * `chosen`, if not NULL, receives the k_generate groups per wave (called
 * batches-per-wave in this interface). */
sn_status sn_autotune(sn_ctx *ctx, const sn_volume *vol, void *stream, int32_t *chosen);
/* A schedule of the kernels for one size class of volumes (the label type,
 * and the powers of two of the row length and of the number of cell rows).
 * Results never depend on it. */
typedef struct sn_schedule {
    int32_t gen_groups;    /* k_generate: groups of 32 cell words per wave, and k_emit:
                              batches of 4 words per wave (1..16; 1 untuned)            */
    int32_t count_words;   /* k_count: cell words per thread, 1 or 4 (0, untuned: 4 from
                              2^18 words in a launch, else 1)                          */
    int32_t edge_segments; /* k_edges: segments of four 64-sample words per wave
                              (1..16; 4 untuned)                                     */
    int32_t sweep_chunk;   /* the sweeps of a mesh of more than 2^24 points: blocks each
                              XCD takes in turn in the slab-chunked order (0, untuned:
                              about a sixteenth of a slab's blocks)                    */
} sn_schedule;
/* The schedule the context uses for volumes of vol's size class (tuned, set,
 * loaded from SN_AUTOTUNE_CACHE, or the untuned one). */
sn_status sn_schedule_get(sn_ctx *ctx, const sn_volume *vol, sn_schedule *out);
/* Use `in` for vol's size class from now on; SN_EINVAL for a value out of
 * range.  sn_autotune overwrites it. */
sn_status sn_schedule_set(sn_ctx *ctx, const sn_volume *vol, const sn_schedule *in);
/* Force the batches-per-wave schedule of the generation kernels (1..16) for
 * every later launch on this context; 0 returns to the tuned/default choice.
 * Results do not depend on the schedule. */
sn_status sn_set_batches_per_wave(sn_ctx *ctx, int32_t batches_per_wave);

/* Per-kernel timing: with on = 1 every library kernel launch is bracketed by
 * HIP events on the stream it runs on, and the sweeps of one smoothing call
 * (a mesh's run of launches, or a batch's sweep graph) are bracketed as a
 * whole (counted as `iterations` launches of k_jacobi: the count is of
 * sweeps, and a mesh's first two sweeps run in one launch); with on = 2 every
 * sweep launch has its own events (the fused first two counting as two); with
 * on = 3 only the sweeps are timed, as with on = 1 (the least added work
 * between kernels).  on = 0 turns
 * timing off.  sn_profile_read synchronises, folds the events into
 * per-kernel totals and fills up to `cap` records. */
typedef struct sn_kernel_stat {
    char name[48];
    int64_t launches;
    double total_ms;
} sn_kernel_stat;
sn_status sn_profile_enable(sn_ctx *ctx, int on);
sn_status sn_profile_reset(sn_ctx *ctx);
sn_status sn_profile_read(sn_ctx *ctx, sn_kernel_stat *out, int32_t cap, int32_t *n_out);

#ifdef __cplusplus
}
#endif
#endif /* SN_H */
