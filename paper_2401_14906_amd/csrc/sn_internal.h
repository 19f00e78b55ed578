// Internal declarations shared by the HIP kernels and the host runtime of
// libsn.so.  Not part of the public ABI (include/sn.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace sn {

// ---- classification (Sec. 2.1) ---------------------------------------------
// C(v) = v if v is selected and is not the background value, else background.
enum ClassMode : int32_t {
    CLS_IDENT = 0,   // every value selected: C is the identity
    CLS_BITMAP = 1,  // bit v of `table` (2048 words, 8 for u8) set <=> v selected (background
                     // bit clear): u8, u16, and u32 whose selected values are all below 65536
    CLS_SORTED = 2   // other u32: `table` holds n sorted, unique selected values (no background)
};

struct ClassSpec {
    int32_t mode;
    uint32_t bg;
    const uint32_t *table;
    int32_t n;
};

// Words and batches.  The cells of a volume are enumerated in their linear
// order i + CM*(j + CN*k); a "row" r = j + CN*k is the line of cells
// (0..CM-1, j, k), cut into W words of 64 cells (the last one ragged).  Word
// g = r*W + w holds cells 64w .. 64w+63 of row r.  A batch is up to kU
// consecutive words of one row (NB batches per row) and is the work item of
// one wavefront; a tile is 4*bpw consecutive batches, the work item of one
// workgroup and the unit of the device-wide scan.
constexpr int kU = 4;
// prim of an image (SN_LINES): 2D contours, one sample slice, segments [Q][2]
constexpr int32_t kPrimLines = 2;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;
constexpr int kMaxBatchesPerWave = 16;
// k_edges: a wave takes 1..kMaxSegmentsPerWave segments of four 64-sample
// words (the schedule's edge_segments), a tile kWavesPerBlock times that
constexpr int kMaxSegmentsPerWave = 16;
// A schedule of the kernels for one size class of volumes.  Results never
// depend on it; sn_autotune picks it by timing.
struct Schedule {
    int32_t gen_groups = 1;   // k_generate: groups of 32 words per wave; k_emit: batches per wave
    int32_t count_words = 0;  // k_count: words per thread, 1 or kCountWideV (0: by size)
    int32_t edge_segs = 4;    // k_edges: segments of four sample-row words per wave
    int32_t sweep_chunk = 0;  // a large single mesh's slab-chunked block order: blocks an
                              // XCD takes in turn (0: about a sixteenth of a slab)
};
inline int64_t edge_tiles(int64_t segments, int32_t spw)
{
    const int64_t t = (int64_t)kWavesPerBlock * spw;
    return (segments + t - 1) / t;
}
// k_generate: a wave takes groups of kGenWords consecutive words (any rows),
// bpw groups per wave
constexpr int kGenWords = 32;
constexpr int64_t kGenStagedPointsPerWord = 8;
// k_count: 1024 threads per workgroup, one or kCountWideV words per thread
// (the wide form for launches of at least kCountWideWords words: fewer scan
// tiles, and fewer of the ordered tile tickets every workgroup takes)
constexpr int kCountWaves = 16;
constexpr int kCountBlock = 64 * kCountWaves;
constexpr int kCountWideV = 4;
// (measured: 2.1 M words count in 48 us wide against 68 us narrow; 260 K
// words in 15.5 us narrow against 21 us wide)
constexpr int64_t kCountWideWords = int64_t(1) << 18;

// Division of 32-bit values by an invariant divisor d >= 1 (Granlund and
// Montgomery's method): with t = umulhi(n, m), n / d = (t + ((n - t) >> s1)) >> s2.
struct UDiv {
    uint32_t d, m, s1, s2;
};

inline UDiv make_udiv(uint32_t d)
{
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) ++l;  // l = ceil(log2 d)
    UDiv u;
    u.d = d;
    u.m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    u.s1 = l < 1 ? l : 1;
    u.s2 = l > 1 ? l - 1 : 0;
    return u;
}

__device__ __forceinline__ uint32_t udiv(uint32_t n, const UDiv &u)
{
    const uint32_t t = __umulhi(n, u.m);
    return (t + ((n - t) >> u.s1)) >> u.s2;
}

// Sample lattice M x N x O; cell grid CM x CN x CO = (M-1)(N-1)(O-1).
// Cut-edge planes (k_edges) hold one bit per sample, WS words per sample row;
// k_edges takes them four words at a time in (sample row, word) order.
struct Geom {
    int64_t M, N, O;
    int64_t CM, CN, CO;
    int64_t R;     // cell rows
    int32_t W;     // words per cell row
    int32_t NB;    // batches per cell row
    int64_t WS;    // words per sample row
    UDiv ws_div;   // division by WS (at least 1)
    UDiv n_div;    // division by N (at least 1)
};

// k_edges segments of a volume: four consecutive sample-row words each
__host__ __device__ inline int64_t edge_segments(const Geom &g)
{
    return (g.N * g.O * g.WS + 3) / 4;
}

// Everything the word kernels need for one volume.
struct VolDesc {
    const void *labels;
    int32_t dtype;  // 1, 2, 4
    int32_t prim;   // 3 or 4, or kPrimLines (an image)
    Geom g;
    ClassSpec cs;
    // cut-edge planes X, Y, Z: [3][O*N][WS]
    uint64_t *planes;
    // word metadata (kept with the mesh)
    uint64_t *pmask;  // [R*W] point bit per cell
    int32_t *wbP;     // [R*W] id of the first point of each word
    int32_t *wbQ;     // [R*W] index of the first quad owned by each word
    int32_t *wbS;     // [R*W] index of the first stencil entry of each word
    // outputs
    float *points;     // [P*3]
    uint8_t *faces;    // [P] stencil face mask, bit f = face f (-x,+x,-y,+y,-z,+z), or
                       // nullptr (k_generate then skips it: no smoothing follows)
    uint32_t *pcell;   // [P] cell linear index of each point, or nullptr (>= 2^32 cells)
    int32_t *st_off;   // [P+1]
    int32_t *st_ids;   // [S]
    int32_t *quads;    // [Q*4]
    void *pairs;       // [Q*2] dtype
    int32_t *tris;     // [2Q*3] (prim 3)
    void *tri_pairs;   // [2Q*2] dtype (prim 3)
    double origin[3], spacing[3];
    int64_t P, Q, S;
};

// One mesh's smoothing job.  Sweep 0 reads the CSR stencil (off, ids) and
// writes nbr: per point the ids of its -y, +y, -z, +z stencil neighbours
// (-1 where absent); later sweeps read nbr and take the -x / +x neighbours,
// which are always points p-1 / p+1, from the neighbouring lanes.
struct SmoothDesc {
    int64_t P;
    const uint8_t *faces;
    const int32_t *off;
    const int32_t *ids;
    int32_t *nbr;  // [P][4]
    float *da;
    float *db;
    int32_t iters;
    int32_t sphere;  // constraint: 0 box of half-width dist, 1 sphere of radius dist
    double lam;
    double dist;
    // the last sweep also writes world points when pcell is set:
    // origin + spacing * (cell centre + offset)
    const uint32_t *pcell;
    float *points;
    UDiv CM, CN;  // cells per row, rows per slice
    int32_t chunk;  // single large mesh: blocks an XCD takes in turn (about 1/16 of a slab)
    // 1: the sweep data is far beyond the last-level cache (more than
    // kSweepSmallPoints points in the mesh, or in all meshes of a launch over
    // many; or the context's test threshold): read-once streams and offset
    // stores take non-temporal hints, and a single mesh takes the
    // slab-chunked block order
    int32_t big;
    // neighbour-table form.  0: [P][4] int32 ids of the -y, +y, -z, +z
    // neighbours (-1 absent), read with the face byte.  Otherwise one 64-bit
    // word per point: bits 0-1 the -x / +x face bits, then the id distances
    // |p - q| of the -y and +y neighbours in pack_yb bits each and of the -z
    // and +z neighbours in pack_zb bits each (0 = absent; a neighbour is
    // never the point itself), 8 bytes per point instead of 17.  Used when
    // the largest distances fit: cells per row for y, cells per slice for z
    // (pack_yb + pack_zb <= 31, both >= 1).
    int32_t pack_yb, pack_zb;
    double origin[3], spacing[3];
};

// A smoothing block covers kSweepBlock * K consecutive points: each wave holds K
// chunks of 64 points.  K = 1 everywhere: two chunks per wave (K = 2, kept as a
// tuning option) need 91 registers against 40 and measure slower on every
// workload once large meshes take non-temporal accesses and the slab-chunked
// block order (connectome 1.45 ms per sweep against 1.15 ms, a batch of 64
// volumes 10.0 ms against 8.3 ms, torso 8.2 us against 7.1 us).  A mesh of more
// than kSweepSmallPoints points (sweep data of about 2.5 times the 256 MB
// last-level cache) reads its read-once streams and writes its offsets with
// non-temporal hints, and alone in a launch it takes the slab-chunked order;
// smaller meshes take XCD-contiguous blocks and ordinary accesses.  Measured:
// 3.5 M points 27 us per sweep against 34 us the other way, 7.1 M points 54 us
// against 61 us, and 140 M points the other way round, 1.14 ms against 1.23 ms.
constexpr int64_t kSweepSmallPoints = int64_t(1) << 24;
inline int sweep_chunks(int64_t /*points*/) { return 1; }
constexpr int kSweepBlock = 256;  // threads per smoothing workgroup
inline int64_t sweep_blocks_for(int64_t points, int K)
{
    return (points + (int64_t)kSweepBlock * K - 1) / ((int64_t)kSweepBlock * K);
}

// Scan tile status word: [63:62] flag, [61:0] value.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

// ---- launchers (sn_kernels.hip) ----------------------------------------------
// Each launch covers tiles tile_base .. tile_base + ntiles - 1 of a global
// tile numbering over the volumes of one extraction; tile_prefix[v] is the
// first tile of volume v and tile_prefix[nvol] the end.
//   k_edges   : a tile is 4*spw segments of four sample-row words; every volume of a launch has
//               the given label type (bytes), classification mode and `wide`
//               (rows 16-byte aligned and M % 4 == 0: one wide load per lane).
//               The launch also zeroes d_zero[0 .. nzero) (the count pass's scan
//               status), so the extraction needs no separate memset.
//   k_count   : a tile is kCountBlock or kCountWideV * kCountBlock cell words.
//   k_generate: a tile is 4*bpw groups of kGenWords words; label type and mode
//               as for k_edges.
hipError_t launch_edges(int32_t dtype, int32_t mode, bool wide, const VolDesc *d_descs,
                        const int64_t *d_tile_prefix, int32_t nvol, int64_t tile_base,
                        int64_t ntiles, uint64_t *d_zero, int64_t nzero, int32_t spw, hipStream_t s);
// Where k_count leaves each volume's totals (P, Q, S) for the host: the last
// tile of volume v writes totals[3v..3v+2] and then, after a system-scope
// fence, stamps[v] = seq (host-visible memory; seq differs between calls).
struct CountOut {
    int64_t *totals;
    int64_t *stamps;
    int64_t seq;
};
hipError_t launch_count(const VolDesc *d_descs, const int64_t *d_tile_prefix, int32_t nvol,
                        int64_t ntiles, int32_t words_per_thread, uint64_t *d_status,
                        uint32_t *d_ticket, const CountOut &out, hipStream_t s);
// staged: stencil ids, quads and pairs go through LDS (for meshes with at
// least kGenStagedPointsPerWord points per word on average)
hipError_t launch_generate(int32_t dtype, int32_t mode, bool staged, bool two_d, const VolDesc *d_descs,
                           const int64_t *d_tile_prefix, int32_t nvol, int64_t tile_base,
                           int64_t ntiles, int32_t bpw, hipStream_t s);
// k_emit: d_sds[v] (iterations, ping-pong buffers) names volume v's final offsets
hipError_t launch_emit(const VolDesc *d_descs, const SmoothDesc *d_sds, const int64_t *d_tile_prefix,
                       int32_t nvol, int64_t ntiles, int32_t bpw, hipStream_t s);
// block_prefix[v] = first block of volume v (kSweepBlock * K points per block, K
// from sweep_chunks of the launch's points); it = 0 runs the first sweep
// (zero input offsets, builds nbr)
// (big: every mesh's descriptor says big, and the launch takes the
// non-temporal form)
hipError_t launch_jacobi(const SmoothDesc *d_sd, const int64_t *d_block_prefix, int32_t nvol,
                         int64_t nblocks, int32_t it, int K, bool big, hipStream_t s);
// sweeps 0 and 1 over many meshes: fused over the leading grid1 blocks (the
// meshes of at least two sweeps), sweep 0 alone over blocks grid1 .. grid0
hipError_t launch_jacobi_first2(const SmoothDesc *d_sd, const int64_t *d_block_prefix, int32_t nvol,
                                int64_t grid0, int64_t grid1, int K, hipStream_t s);
// the same n sweeps as kernel nodes of `graph`, each depending on the one before
// (sweep `it` launches grid[it] blocks; sweeps 0 and 1 as launch_jacobi_first2)
hipError_t add_jacobi_nodes(hipGraph_t graph, const SmoothDesc *d_sd,
                            const int64_t *d_block_prefix, int32_t nvol, const int64_t *grid,
                            int32_t iters, int K, bool big);
// Copy `bytes` (rounded up to 8) from pinned host memory, given by its
// device-side mapping, to device memory `dst` with a kernel on `s`; both
// buffers 8-byte aligned and at least the rounded size.
hipError_t launch_stage(void *dst, const void *src_mapped, size_t bytes, hipStream_t s);
// Single-volume forms: the descriptor travels by value in the kernel
// arguments (no upload, no prefix array; tiles and blocks start at 0).
hipError_t launch_edges_one(const VolDesc &d, bool wide, int64_t ntiles, uint64_t *d_zero,
                            int64_t nzero, int32_t spw, hipStream_t s);
hipError_t launch_count_one(const VolDesc &d, int64_t ntiles, int32_t words_per_thread,
                            uint64_t *d_status, uint32_t *d_ticket, const CountOut &out, hipStream_t s);
hipError_t launch_generate_one(const VolDesc &d, bool staged, int64_t ntiles, int32_t bpw, hipStream_t s);
hipError_t launch_emit_one(const VolDesc &d, const SmoothDesc &sd, int64_t ntiles, int32_t bpw,
                           hipStream_t s);
hipError_t launch_jacobi_one(const SmoothDesc &sd, int64_t nblocks, int32_t it, int K, hipStream_t s);
// sweeps 0 and 1 of one mesh (iterations >= 2) in one launch, equal to two
// launch_jacobi_one calls bit for bit
hipError_t launch_jacobi_first2_one(const SmoothDesc &sd, int64_t nblocks, int K, hipStream_t s);
hipError_t launch_triangulate_one(const VolDesc &d, hipStream_t s);
// quads [Q][4] over world points -> tris [2Q][3] under diagonal rule 0..3;
// tri_pairs [2Q][2] of the label type (dtype bytes) when not null
hipError_t launch_tri_rule(int32_t rule, int32_t dtype, const int32_t *quads, const float *pts,
                           const void *pairs, int64_t Q, int32_t *tris, void *tri_pairs, hipStream_t s);
// quad blocks (256 quads per block) of the volumes with prim 3
hipError_t launch_triangulate(const VolDesc *d_descs, const int64_t *d_block_prefix, int32_t nvol,
                              int64_t nblocks, hipStream_t s);

}  // namespace sn
