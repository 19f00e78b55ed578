// SurfaceNets extraction and smoothing kernels for gfx950 (MI355X).
//
// Extraction works on bit planes and 64-cell words.  k_edges reads the label
// volume once, with wide coalesced row loads, and writes three cut-edge bit
// planes X, Y, Z (one bit per lattice sample and axis: the edge from the
// sample to its +x, +y or +z neighbour is cut).  Cells are enumerated in
// linear order and cut into 64-cell words (see sn_internal.h); every later
// step is mask algebra on 64-bit words of those planes: a cell's twelve edges
// are bits of four plane rows, its point bit is their OR, a face's cut test
// is the OR of four, and every rank inside a word is an mbcnt.  This replaces
// the paper's triad byte volume, trim intervals, checkerboarded point bits
// and 3x3 row iterator (Sec. 3.2-3.6) with bit planes, a 1-bit point plane
// and per-word prefix bases.
//
//   k_edges    : classification and cut-edge planes (Sec. 2.3 passes 1-2).
//   k_count    : per-word point / quad / stencil counts and the point-bit
//                plane, with a fused single-pass (decoupled look-back) scan
//                that gives every word its first point id, quad index and
//                stencil index (Sec. 2.3 pass 3 and the prefix sum).
//   k_generate : points, stencil CSR, quads and label pairs written at those
//                bases, without atomics (Sec. 2.3 pass 4).
//   k_jacobi_first, k_jacobi
//              : double-buffered sweeps of Eq. (1) with the box constraint
//                (Sec. 2.2, 2.4), on cell-relative offsets.
//   k_emit     : world coordinates of the points from the offsets.
//   k_tri      : two triangles per quad (Sec. 2.5).
//   k_tri_rule : two triangles per quad with a geometric diagonal choice.
#include "sn_internal.h"

#define SN_GLOBAL __attribute__((address_space(1)))
#define SN_CONST __attribute__((address_space(4)))

namespace sn {

// Pointers read out of descriptors are generic; these casts tell the compiler
// which memory they address (global for vector access; constant for data that
// is read-only during the kernel and read with wave-uniform addresses, which
// then go through the scalar unit).
template <typename T>
__device__ __forceinline__ SN_GLOBAL T *glb(T *p)
{
    return (SN_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const SN_GLOBAL T *glb(const T *p)
{
    return (const SN_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const SN_CONST T *cst(const T *p)
{
    return (const SN_CONST T *)p;
}

__device__ __forceinline__ uint32_t rank_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t lane_bit(uint64_t m, int lane)
{
    return (uint32_t)(m >> lane) & 1u;
}

__device__ __forceinline__ int find_seg(const int64_t *prefix, int n, int64_t t)
{
    const SN_CONST int64_t *p = cst(prefix);
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (p[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Where a launch finds its volume: an array of descriptors in device memory
// with a prefix of tiles (or blocks) per volume, for launches over many
// volumes; or a single descriptor passed by value in the kernel arguments,
// which needs no upload before the launch.  Kernels over many volumes take
// the array as __restrict__ parameters (so descriptor loads are known not to
// alias the kernel's stores) and wrap them in these structs for the shared
// bodies.
struct ManyVols {
    const VolDesc *descs;
    const int64_t *prefix;
    int32_t nvol;
};
struct OneVol {
    VolDesc d;
};
struct ManySmooth {
    const SmoothDesc *sds;
    const int64_t *prefix;
    int32_t nvol;
};
struct OneSmooth {
    SmoothDesc s;
};
struct ManyEmit {
    const VolDesc *descs;
    const SmoothDesc *sds;
    const int64_t *prefix;
    int32_t nvol;
};
struct OneEmit {
    VolDesc d;
    SmoothDesc s;
};

// Volume of global tile t, its index and its first tile.
__device__ __forceinline__ const VolDesc &vol_of(const ManyVols &a, int64_t t, int &v, int64_t &first)
{
    v = find_seg(a.prefix, a.nvol, t);
    first = cst(a.prefix)[v];
    return a.descs[v];
}
__device__ __forceinline__ const VolDesc &vol_of(const OneVol &a, int64_t, int &v, int64_t &first)
{
    v = 0, first = 0;
    return a.d;
}
__device__ __forceinline__ const SmoothDesc &smooth_of(const ManySmooth &a, int64_t b, int64_t &first)
{
    const int v = find_seg(a.prefix, a.nvol, b);
    first = cst(a.prefix)[v];
    return a.sds[v];
}
__device__ __forceinline__ const SmoothDesc &smooth_of(const OneSmooth &a, int64_t, int64_t &first)
{
    first = 0;
    return a.s;
}

template <int MODE>
__device__ __forceinline__ uint32_t classify(uint32_t v, const ClassSpec &cs)
{
    if constexpr (MODE == CLS_IDENT) {
        return v;
    } else if constexpr (MODE == CLS_BITMAP) {
        // the table covers values below 65536 (the whole range of u8 and
        // u16, for which this test folds away); larger u32 values are never
        // selected in this mode
        const bool in = v < 65536u;
        const uint32_t vi = in ? v : 0u;
        return (in && ((glb(cs.table)[vi >> 5] >> (vi & 31u)) & 1u)) ? v : cs.bg;
    } else {
        const SN_GLOBAL uint32_t *tab = glb(cs.table);
        int lo = 0, hi = cs.n;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (tab[mid] < v)
                lo = mid + 1;
            else
                hi = mid;
        }
        return (lo < cs.n && tab[lo] == v) ? v : cs.bg;
    }
}

// Where a batch sits.  Batch, row and word counts of a volume fit int32 (the
// host checks); the first batch of a wave is found with one 32-bit division
// and the following ones by stepping.
struct BatchPos {
    int32_t r, j, k;
    int32_t w0, nw;  // first word, number of words (1..kU)
    int64_t g0;      // linear index of the first word
};

__device__ __forceinline__ BatchPos batch_pos(const Geom &g, int64_t b)
{
    BatchPos p;
    const uint32_t NB = (uint32_t)g.NB, CN = (uint32_t)g.CN;
    p.r = (int32_t)((uint32_t)b / NB);
    p.w0 = ((int32_t)b - p.r * (int32_t)NB) * kU;
    p.j = (int32_t)((uint32_t)p.r % CN);
    p.k = (int32_t)((uint32_t)p.r / CN);
    p.nw = g.W - p.w0 < kU ? g.W - p.w0 : kU;
    p.g0 = (int64_t)p.r * g.W + p.w0;
    return p;
}

__device__ __forceinline__ void batch_next(const Geom &g, BatchPos &p)
{
    p.w0 += kU;
    if (p.w0 >= g.W) {
        p.w0 = 0;
        p.r += 1;
        p.j += 1;
        if (p.j == (int32_t)g.CN) p.j = 0, p.k += 1;
    }
    p.nw = g.W - p.w0 < kU ? g.W - p.w0 : kU;
    p.g0 = (int64_t)p.r * g.W + p.w0;
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

// One point's world coordinates (three consecutive floats).
__device__ __forceinline__ void store_point(SN_GLOBAL float *points, int32_t id, float x, float y,
                                            float z)
{
    SN_GLOBAL float *p = points + 3 * (int64_t)id;
    p[0] = x, p[1] = y, p[2] = z;
}

// Masks of one 64-cell word (bit L = cell 64w + L) from the cut-edge planes:
// a point where any of the twelve edges is cut (Sec. 2.2), a stencil face
// where one of its four edges is cut and the neighbour cell exists
// (Sec. 3.3), a quad per cut edge owned by the cell's origin sample whose
// four cells exist (Sec. 2.2, open boundary of Sec. 4.2).  The same algebra
// runs per lane (one word per lane, vector registers) in k_count and per wave
// (scalar registers) in k_generate.
struct WordMasks {
    uint64_t pt, qx, qy, qz;
    uint64_t f[6];  // -x, +x, -y, +y, -z, +z
};

// Plane words around cell word w of cell row (j,k): X of sample rows
// (j,k) (j+1,k) (j,k+1) (j+1,k+1); Y of (j,k), (j,k+1) and Z of (j,k), (j+1,k),
// each with the following word for the sample at i+1.
struct PlaneWords {
    uint64_t x00, x10, x01, x11;
    uint64_t y00, y00n, y01, y01n;
    uint64_t z00, z00n, z10, z10n;
};

template <typename P>
__device__ __forceinline__ PlaneWords plane_words(const P *planes, int64_t plane_stride, int64_t WS,
                                                  int64_t s00, int64_t N, int32_t w)
{
    const P *X = planes, *Y = planes + plane_stride, *Z = planes + 2 * plane_stride;
    const int64_t s10 = s00 + 1, s01 = s00 + N, s11 = s01 + 1;
    const bool nx = w + 1 < WS;
    PlaneWords p;
    p.x00 = X[s00 * WS + w], p.x10 = X[s10 * WS + w];
    p.x01 = X[s01 * WS + w], p.x11 = X[s11 * WS + w];
    p.y00 = Y[s00 * WS + w], p.y01 = Y[s01 * WS + w];
    p.z00 = Z[s00 * WS + w], p.z10 = Z[s10 * WS + w];
    p.y00n = nx ? Y[s00 * WS + w + 1] : 0ull, p.y01n = nx ? Y[s01 * WS + w + 1] : 0ull;
    p.z00n = nx ? Z[s00 * WS + w + 1] : 0ull, p.z10n = nx ? Z[s10 * WS + w + 1] : 0ull;
    return p;
}

// An image (one sample slice, the method in the plane): X of sample rows j
// and j+1 and Y of row j (with the following word); there are no z planes and
// no k+1 rows, and those words read as zero.
template <typename P>
__device__ __forceinline__ PlaneWords plane_words2d(const P *planes, int64_t plane_stride, int64_t WS,
                                                    int64_t s00, int32_t w)
{
    const P *X = planes, *Y = planes + plane_stride;
    PlaneWords p{};
    p.x00 = X[s00 * WS + w], p.x10 = X[(s00 + 1) * WS + w];
    p.y00 = Y[s00 * WS + w];
    p.y00n = w + 1 < WS ? Y[s00 * WS + w + 1] : 0ull;
    return p;
}

__device__ __forceinline__ uint64_t next_bit(uint64_t a, uint64_t an) { return (a >> 1) | (an << 63); }

// TWO_D: the same algebra on an image's words (z inputs zero, k = 0, one cell
// slice): a point where any of the cell's four edges is cut, faces -x, +x,
// -y, +y, and a segment per cut x- or y-edge owned by the cell (qx, qy) whose
// two cells exist.
template <bool TWO_D = false>
__device__ __forceinline__ WordMasks word_masks(const PlaneWords &p, int32_t w, int32_t j, int32_t k,
                                                const Geom &g)
{
    const uint64_t x0 = p.x00, x1 = p.x10, x2 = p.x01, x3 = p.x11;
    const uint64_t y0 = p.y00, y1 = next_bit(p.y00, p.y00n), y2 = p.y01, y3 = next_bit(p.y01, p.y01n);
    const uint64_t z0 = p.z00, z1 = next_bit(p.z00, p.z00n), z2 = p.z10, z3 = next_bit(p.z10, p.z10n);
    const int64_t rem = g.CM - 64 * (int64_t)w;       // cells of the row from this word on (>= 1)
    const uint64_t valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
    const uint64_t hasprev = w == 0 ? ~1ull : ~0ull;  // i >= 1
    const int64_t rem2 = rem - 1;                     // i + 1 <= CM - 1
    const uint64_t hasnext = rem2 >= 64 ? ~0ull : (rem2 <= 0 ? 0ull : ((1ull << rem2) - 1));
    const uint64_t ym = j >= 1 ? ~0ull : 0ull, yp = j + 1 <= g.CN - 1 ? ~0ull : 0ull;
    const uint64_t zm = k >= 1 ? ~0ull : 0ull, zp = k + 1 <= g.CO - 1 ? ~0ull : 0ull;
    WordMasks m;
    m.pt = (x0 | x1 | x2 | x3 | y0 | y1 | y2 | y3 | z0 | z1 | z2 | z3) & valid;
    m.f[0] = (y0 | y2 | z0 | z2) & valid & hasprev;
    m.f[1] = (y1 | y3 | z1 | z3) & hasnext;
    m.f[2] = (x0 | x2 | z0 | z1) & valid & ym;
    m.f[3] = (x1 | x3 | z2 | z3) & valid & yp;
    m.f[4] = (x0 | x1 | y0 | y1) & valid & zm;
    m.f[5] = (x2 | x3 | y2 | y3) & valid & zp;
    const uint64_t zq = TWO_D ? ~0ull : zm;  // an image's segments have no z neighbour cells
    m.qx = x0 & valid & ym & zq;
    m.qy = y0 & valid & hasprev & zq;
    m.qz = z0 & valid & hasprev & ym;
    return m;
}

__device__ __forceinline__ int64_t wave_sum(int64_t x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ int32_t wave_excl_scan32(int32_t x, int lane)
{
    int32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, (unsigned)o);
        if (lane >= o) inc += y;
    }
    return inc - x;
}

// Inclusive wave scan on DPP row shifts and row broadcasts (no LDS traffic).
__device__ __forceinline__ int32_t wave_incl_scan_dpp(int32_t v, int lane)
{
    const int rl = lane & 15;
    int32_t t;
    t = __builtin_amdgcn_mov_dpp(v, 0x111, 0xf, 0xf, false);  // row_shr:1
    if (rl >= 1) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x112, 0xf, 0xf, false);  // row_shr:2
    if (rl >= 2) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x114, 0xf, 0xf, false);  // row_shr:4
    if (rl >= 4) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x118, 0xf, 0xf, false);  // row_shr:8
    if (rl >= 8) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x142, 0xf, 0xf, false);  // row_bcast:15
    if ((lane & 31) >= 16) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x143, 0xf, 0xf, false);  // row_bcast:31
    if (lane >= 32) v += t;
    return v;
}

// ---------------------------------------------------------------------------
// k_edges: cut-edge planes X, Y, Z (Sec. 2.2): bit i of word m of sample row
// (j,k) of plane X is set iff C(i,j,k) != C(i+1,j,k) (Y: C(i,j+1,k), Z:
// C(i,j,k+1)).  A wave takes four 64-sample words (of one row or of two
// consecutive rows), four samples per lane, with one wide load per sample row
// (rows (j,k), (j+1,k), (j,k+1)); nibbles are merged into 64-bit words across
// 16 lanes.
// ---------------------------------------------------------------------------


typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

// dword vectors at 4-byte alignment (the narrow rows' windows)
typedef uint32_t v2u_a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t v3u_a4 __attribute__((ext_vector_type(3), aligned(4)));
typedef uint32_t v4u_a4 __attribute__((ext_vector_type(4), aligned(4)));

template <typename T, bool WIDE>
__device__ __forceinline__ void load_quad(const T *row_, int32_t i0, int32_t M1, const T *vol_end, T (&v)[4])
{
    const SN_GLOBAL T *row = glb(row_);
    if constexpr (WIDE) {
        // rows are 16-byte aligned and M % 4 == 0, so a quad never straddles the row end
        const int32_t ic = i0 <= M1 ? i0 : M1 - 3;
        if constexpr (sizeof(T) == 4) {
            const v4u q = *reinterpret_cast<const SN_GLOBAL v4u *>(row + ic);
            v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
        } else if constexpr (sizeof(T) == 2) {
            const v2u q = *reinterpret_cast<const SN_GLOBAL v2u *>(row + ic);
            v[0] = (T)(q.x & 0xffffu), v[1] = (T)(q.x >> 16), v[2] = (T)(q.y & 0xffffu),
            v[3] = (T)(q.y >> 16);
        } else {
            const uint32_t q = *reinterpret_cast<const SN_GLOBAL uint32_t *>(row + ic);
            v[0] = (T)(q & 0xffu), v[1] = (T)((q >> 8) & 0xffu), v[2] = (T)((q >> 16) & 0xffu),
            v[3] = (T)(q >> 24);
        }
    } else if constexpr (sizeof(T) == 4) {
        // rows of any alignment: the four samples as one 4-dword load (labels
        // are 4-byte aligned); only where it would pass the end of the volume
        // are they read one by one, clamped to the row
        if (i0 > M1) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = 0;
            return;
        }
        const uintptr_t a = reinterpret_cast<uintptr_t>(row_ + i0);
        if (a + 16 <= reinterpret_cast<uintptr_t>(vol_end)) {
            const v4u_a4 q = *reinterpret_cast<const SN_GLOBAL v4u_a4 *>(a);
            v[0] = (T)q.x, v[1] = (T)q.y, v[2] = (T)q.z, v[3] = (T)q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = row[(uint32_t)(i0 + e <= M1 ? i0 + e : M1)];
        }
    } else {
        // 1- and 2-byte labels in rows of any alignment: win_issue/win_finish
        static_assert(sizeof(T) == 4, "narrow 1- and 2-byte rows take the window loads");
    }
}

// Narrow rows of 1- and 2-byte labels: samples i0 .. i0+3 lie in the
// dword-aligned window of ND = 2 or 3 dwords at or below their address, and
// its last dword is the first of the next lane's window (the next four
// samples of the row: the lanes of one 16-lane group share a row and its
// activity).  A lane loads ND - 1 dwords and takes the last from the next
// lane; the group's last lane, and a lane whose next lane's window would pass
// the end of the volume, load it themselves.  Samples past the row end are
// loaded (the next row's) but never used.  Where a lane's own window would
// pass the end of the volume, its samples are read one by one, clamped to the
// row.  Two steps, so that the loads of all three rows are in flight before
// the exchange between lanes waits for them.
struct Win {
    uint32_t w0, w1, wl, sh;
    bool inb, own;
};

template <typename T>
__device__ __forceinline__ Win win_issue(const T *row_, int32_t i0, const T *vol_end, int lane, bool active)
{
    constexpr int ND = sizeof(T) == 1 ? 2 : 3;
    Win w{0u, 0u, 0u, 0u, false, false};
    const uintptr_t a = reinterpret_cast<uintptr_t>(row_ + i0);
    const uintptr_t ab = a & ~uintptr_t(3);
    const uintptr_t end = reinterpret_cast<uintptr_t>(vol_end);
    w.sh = (uint32_t)(a & 3u);
    w.inb = active && ab + 4 * ND <= end;
    w.own = (lane & 15) == 15 || ab + 4 * (ND - 1) + 4 * ND > end;
    if (w.inb) {
        const SN_GLOBAL uint32_t *wp = reinterpret_cast<const SN_GLOBAL uint32_t *>(ab);
        if constexpr (ND == 2) {
            w.w0 = wp[0];
        } else {
            const v2u_a4 q = *reinterpret_cast<const SN_GLOBAL v2u_a4 *>(wp);
            w.w0 = q.x, w.w1 = q.y;
        }
        if (w.own) w.wl = wp[ND - 1];
    }
    return w;
}

// every lane of the wave runs this (the exchange reads the next lane)
template <typename T>
__device__ __forceinline__ void win_finish(const Win &w, const T *row_, int32_t i0, int32_t M1, bool active,
                                           T (&v)[4])
{
    // the next lane's first dword (wave_shl:1; lane 63 is a group's last)
    const uint32_t nx = (uint32_t)__builtin_amdgcn_mov_dpp((int)w.w0, 0x130, 0xf, 0xf, false);
    if (w.inb) {
        const uint32_t wl = w.own ? w.wl : nx;
        if constexpr (sizeof(T) == 1) {
            const uint32_t x = __builtin_amdgcn_alignbyte(wl, w.w0, w.sh);
            v[0] = (T)(x & 0xffu), v[1] = (T)((x >> 8) & 0xffu), v[2] = (T)((x >> 16) & 0xffu),
            v[3] = (T)(x >> 24);
        } else {
            const uint32_t x0 = __builtin_amdgcn_alignbyte(w.w1, w.w0, w.sh);
            const uint32_t x1 = __builtin_amdgcn_alignbyte(wl, w.w1, w.sh);
            v[0] = (T)(x0 & 0xffffu), v[1] = (T)(x0 >> 16), v[2] = (T)(x1 & 0xffffu), v[3] = (T)(x1 >> 16);
        }
    } else if (active) {
        const SN_GLOBAL T *row = glb(row_);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = row[(uint32_t)(i0 + e <= M1 ? i0 + e : M1)];
    }
}

// OR of a 4-bit nibble per lane into the 64-bit word of each group of 16 lanes
// (lane 16g + l contributes bits 4l..4l+3); valid in lane 16g.
__device__ __forceinline__ uint64_t merge_nibbles(uint32_t nib, int lane)
{
    uint32_t v = nib << (4 * (lane & 7));
    v |= __shfl_xor(v, 1u);
    v |= __shfl_xor(v, 2u);
    v |= __shfl_xor(v, 4u);
    const uint32_t hi = __shfl_down(v, 8u);
    return (uint64_t)v | ((uint64_t)hi << 32);
}

template <typename T, int MODE, bool WIDE>
__device__ __forceinline__ void edges_segment(const VolDesc &d, int64_t seg, int lane)
{
    const Geom &g = d.g;
    // A segment is four consecutive words of the planes in (sample row, word)
    // order, one per 16 lanes: the words of one row, or the last words of a
    // row and the first of the next, so that rows of any length leave few
    // lanes idle.  Group lane l covers samples 64*wi + 4l .. 64*wi + 4l + 3.
    const uint32_t WS = (uint32_t)g.WS, N = (uint32_t)g.N;
    const uint32_t tw = N * (uint32_t)g.O * WS;  // < 2^31 (validated)
    const uint32_t fw = 4u * (uint32_t)seg + ((uint32_t)lane >> 4);
    const bool wok = fw < tw;
    const uint32_t srow = udiv(fw, g.ws_div);
    const uint32_t wi = fw - srow * WS;
    const uint32_t k = udiv(srow, g.n_div), j = srow - k * N;
    const int32_t M1 = (int32_t)(g.M - 1);
    const int32_t i0 = 64 * (int32_t)wi + 4 * (lane & 15);
    const T *ra = static_cast<const T *>(d.labels) + (int64_t)srow * g.M;
    const bool hasy = wok && j + 1 < N, hasz = wok && (int64_t)k + 1 < g.O;
    T a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
    const T *vend = static_cast<const T *>(d.labels) + g.M * g.N * g.O;
    if constexpr (!WIDE && sizeof(T) <= 2) {
        const Win wa = win_issue<T>(ra, i0, vend, lane, wok);
        const Win wb = win_issue<T>(ra + g.M, i0, vend, lane, hasy);
        const Win wc = win_issue<T>(ra + g.M * g.N, i0, vend, lane, hasz);
        win_finish<T>(wa, ra, i0, M1, wok, a);
        win_finish<T>(wb, ra + g.M, i0, M1, hasy, b);
        win_finish<T>(wc, ra + g.M * g.N, i0, M1, hasz, c);
    } else {
        if (wok) load_quad<T, WIDE>(ra, i0, M1, vend, a);
        if (hasy) load_quad<T, WIDE>(ra + g.M, i0, M1, vend, b);
        if (hasz) load_quad<T, WIDE>(ra + g.M * g.N, i0, M1, vend, c);
    }
    // the sample after the word (its last x edge), read by the group's last lane
    const bool last = (lane & 15) == 15;
    const int32_t inext = 64 * (int32_t)wi + 64;
    T an = 0;
    if (last && wok && inext <= M1) an = glb(ra)[(uint32_t)inext];
    uint32_t ca[5], cb[4], cc[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        ca[e] = classify<MODE>((uint32_t)a[e], d.cs);
        cb[e] = classify<MODE>((uint32_t)b[e], d.cs);
        cc[e] = classify<MODE>((uint32_t)c[e], d.cs);
    }
    ca[4] = __shfl_down(ca[0], 1u);
    if (last) ca[4] = classify<MODE>((uint32_t)an, d.cs);
    uint32_t xn = 0, yn = 0, zn = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int32_t i = i0 + e;
        xn |= ((ca[e] != ca[e + 1]) && i <= M1 - 1 ? 1u : 0u) << e;
        yn |= (hasy && (ca[e] != cb[e]) && i <= M1 ? 1u : 0u) << e;
        zn |= (hasz && (ca[e] != cc[e]) && i <= M1 ? 1u : 0u) << e;
    }
    const uint64_t X = merge_nibbles(xn, lane), Y = merge_nibbles(yn, lane), Z = merge_nibbles(zn, lane);
    if ((lane & 15) == 0 && wok) {
        SN_GLOBAL uint64_t *P = glb(d.planes);
        const int64_t ps = (int64_t)tw;
        P[fw] = X;  // word wi of sample row srow
        P[ps + fw] = Y;
        P[2 * ps + fw] = Z;
    }
}

// spw: segments of four words per wave (the schedule's edge_segments); a tile is
// kWavesPerBlock * spw segments
template <typename T, int MODE, bool WIDE, class Src>
__device__ __forceinline__ void edges_tile(const Src &a, int64_t tile_base, uint64_t *zero,
                                           int64_t nzero, int32_t spw)
{
    // clear the scan status words of the counting pass that follows
    for (int64_t z = (int64_t)blockIdx.x * kBlock + threadIdx.x; z < nzero;
         z += (int64_t)gridDim.x * kBlock)
        glb(zero)[z] = 0;
    const int64_t t = tile_base + blockIdx.x;
    int v;
    int64_t first;
    const VolDesc &d = vol_of(a, t, v, first);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t nseg = edge_segments(d.g);
    int64_t seg = (t - first) * (kWavesPerBlock * spw) + (int64_t)wave * spw;
    for (int q = 0; q < spw; ++q, ++seg) {
        if (seg >= nseg) break;
        edges_segment<T, MODE, WIDE>(d, seg, lane);
    }
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_edges_wide(const VolDesc *__restrict__ descs,
                                                       const int64_t *__restrict__ prefix,
                                                       int32_t nvol, int64_t tile_base,
                                                       uint64_t *zero, int64_t nzero, int32_t spw)
{
    edges_tile<T, MODE, true>(ManyVols{descs, prefix, nvol}, tile_base, zero, nzero, spw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_edges_narrow(const VolDesc *__restrict__ descs,
                                                         const int64_t *__restrict__ prefix,
                                                         int32_t nvol, int64_t tile_base,
                                                         uint64_t *zero, int64_t nzero, int32_t spw)
{
    edges_tile<T, MODE, false>(ManyVols{descs, prefix, nvol}, tile_base, zero, nzero, spw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_edges_wide_one(OneVol a, uint64_t *zero, int64_t nzero,
                                                           int32_t spw)
{
    edges_tile<T, MODE, true>(a, 0, zero, nzero, spw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_edges_narrow_one(OneVol a, uint64_t *zero, int64_t nzero,
                                                             int32_t spw)
{
    edges_tile<T, MODE, false>(a, 0, zero, nzero, spw);
}

// ---------------------------------------------------------------------------
// k_count: one lane per 64-cell word.  Point / quad / stencil counts of every
// word and the point-bit plane, then a fused single-pass (decoupled
// look-back) scan over words that gives every word its first point id, quad
// index and stencil index (Sec. 2.3 passes 1-3 and the prefix sum).
// ---------------------------------------------------------------------------

// Exclusive prefixes of tile t for the three counts, by one whole wave.  Each
// round inspects a window of 64 * kLookV tiles below `top`: window position
// q = L + 64 v (lane L, slot v) is tile top - q.  Tiles before `first` (the
// volume's first tile) read as an inclusive prefix of zero.  A count waits
// only while a tile closer than its nearest inclusive prefix has not yet
// published an aggregate; such a tile was handed out before t, so its
// workgroup is running and publishes without waiting on anything.
constexpr int kLookV = 1;

__device__ void look_back3(const uint64_t *status, int64_t t, int64_t first, int lane,
                           int64_t excl[3])
{
    int64_t top[3] = {t - 1, t - 1, t - 1};
    bool done[3] = {false, false, false};
    excl[0] = excl[1] = excl[2] = 0;
    while (!(done[0] && done[1] && done[2])) {
        uint64_t s[3][kLookV];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int v = 0; v < kLookV; ++v) {
                const int64_t p = top[c] - lane - 64 * v;
                s[c][v] = kFlagPrefix;
                if (!done[c] && p >= first)
                    s[c][v] = __hip_atomic_load(status + 3 * p + c, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            }
        bool stalled = false;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (done[c]) continue;
            // nearest inclusive prefix in the window (qp = 64 * kLookV: none)
            int qp = 64 * kLookV;
            bool waiting = false;
#pragma unroll
            for (int v = 0; v < kLookV; ++v) {
                const uint64_t flag = s[c][v] & ~kValMask;
                const uint64_t pm = __ballot(flag == kFlagPrefix);
                const uint64_t zm = __ballot(flag == 0);
                if (qp == 64 * kLookV) {
                    // slot v is reached: positions 64v .. up to its first prefix
                    const int lp = pm ? __builtin_ctzll(pm) : 64;
                    const uint64_t upto = lp >= 63 ? ~0ull : ((2ull << lp) - 1);
                    if (zm & upto) waiting = true;
                    if (pm) qp = 64 * v + lp;
                }
            }
            if (waiting) {
                stalled = true;
                continue;
            }
            int64_t part = 0;
#pragma unroll
            for (int v = 0; v < kLookV; ++v)
                if (64 * v + lane <= qp) part += (int64_t)(s[c][v] & kValMask);
            excl[c] += wave_sum(part);
            if (qp < 64 * kLookV)
                done[c] = true;
            else
                top[c] -= 64 * kLookV;
        }
        if (stalled) __builtin_amdgcn_s_sleep(1);
    }
}

// Last tile of volume v (a launch over one volume has exactly its tiles).
__device__ __forceinline__ int64_t last_tile(const ManyVols &a, int v)
{
    return cst(a.prefix)[v + 1] - 1;
}
__device__ __forceinline__ int64_t last_tile(const OneVol &, int)
{
    return (int64_t)gridDim.x - 1;
}

template <int V, class Src>
__device__ __forceinline__ void count_body(const Src &a, uint64_t *status, uint32_t *ticket,
                                           CountOut out)
{
    // a tile is V * kCountBlock words; word (v, thread) of the tile is
    // v * kCountBlock + thread, so each v is one coalesced pass
    __shared__ int64_t s_tile;
    __shared__ int32_t s_wtot[V][3][kCountWaves];
    __shared__ int64_t s_excl[3];
    if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t t = s_tile;  // tiles are handed out in order: predecessors are running
    int vol;
    int64_t first;
    const VolDesc &d = vol_of(a, t, vol, first);
    const Geom &g = d.g;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t words = g.R * g.W;
    const int64_t gw0 = (t - first) * (int64_t)(V * kCountBlock) + threadIdx.x;
    int32_t ex[V][3];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t gw = gw0 + v * kCountBlock;
        int32_t cnt[3] = {0, 0, 0};
        if (gw < words) {
            const uint32_t r = (uint32_t)gw / (uint32_t)g.W;
            const int32_t w = (int32_t)((uint32_t)gw - r * (uint32_t)g.W);
            const int32_t j = (int32_t)(r % (uint32_t)g.CN), k = (int32_t)(r / (uint32_t)g.CN);
            const int64_t ps = g.N * g.O * g.WS;
            WordMasks m;
            if (d.prim == kPrimLines) {  // an image: contour segments
                const PlaneWords p = plane_words2d(glb(d.planes), ps, g.WS, (int64_t)j, w);
                m = word_masks<true>(p, w, j, k, g);
            } else {
                const PlaneWords p = plane_words(glb(d.planes), ps, g.WS, j + g.N * (int64_t)k, g.N, w);
                m = word_masks(p, w, j, k, g);
            }
            glb(d.pmask)[gw] = m.pt;
            cnt[0] = __popcll(m.pt);
            cnt[1] = __popcll(m.qx) + __popcll(m.qy) + __popcll(m.qz);
            cnt[2] = __popcll(m.f[0]) + __popcll(m.f[1]) + __popcll(m.f[2]) + __popcll(m.f[3]) +
                     __popcll(m.f[4]) + __popcll(m.f[5]);
        }
        // wave-level exclusive scan of the three counts (a tile's counts fit 32 bits)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ex[v][c] = wave_excl_scan32(cnt[c], lane);
            if (lane == 63) s_wtot[v][c][wave] = ex[v][c] + cnt[c];
        }
    }
    __syncthreads();
    if (wave == 0) {
        int64_t agg[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            agg[c] = 0;
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int q = 0; q < kCountWaves; ++q) agg[c] += s_wtot[v][c][q];
            if (lane == 0)
                __hip_atomic_store(status + 3 * t + c,
                                   (t == first ? kFlagPrefix : kFlagAgg) | (uint64_t)agg[c],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        int64_t excl[3] = {0, 0, 0};
        if (t != first) {
            look_back3(status, t, first, lane, excl);
            if (lane == 0)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    __hip_atomic_store(status + 3 * t + c, kFlagPrefix | (uint64_t)(excl[c] + agg[c]),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s_excl[c] = excl[c];
                if (t == last_tile(a, vol)) out.totals[3 * vol + c] = excl[c] + agg[c];
            }
            if (t == last_tile(a, vol)) {
                // the host may read the totals as soon as it sees the stamp
                __threadfence_system();
                __hip_atomic_store(out.stamps + vol, out.seq, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
    __syncthreads();
    int32_t before[3] = {0, 0, 0};  // counts of the tile's words before (v, this wave)
#pragma unroll
    for (int v = 0; v < V; ++v) {
        int32_t b[3] = {before[0], before[1], before[2]};
#pragma unroll
        for (int q = 0; q < kCountWaves; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (q < wave) b[c] += s_wtot[v][c][q];
                before[c] += s_wtot[v][c][q];
            }
        const int64_t gw = gw0 + v * kCountBlock;
        if (gw < words) {
            glb(d.wbP)[gw] = (int32_t)(s_excl[0] + b[0] + ex[v][0]);
            glb(d.wbQ)[gw] = (int32_t)(s_excl[1] + b[1] + ex[v][1]);
            glb(d.wbS)[gw] = (int32_t)(s_excl[2] + b[2] + ex[v][2]);
        }
    }
}

template <int V>
__global__ __launch_bounds__(kCountBlock) void k_count(const VolDesc *__restrict__ descs,
                                                       const int64_t *__restrict__ prefix,
                                                       int32_t nvol, uint64_t *status,
                                                       uint32_t *ticket, CountOut out)
{
    count_body<V>(ManyVols{descs, prefix, nvol}, status, ticket, out);
}

template <int V>
__global__ __launch_bounds__(kCountBlock) void k_count_one(OneVol a, uint64_t *status,
                                                           uint32_t *ticket, CountOut out)
{
    count_body<V>(a, status, ticket, out);
}

// ---------------------------------------------------------------------------
// k_generate: points, stencil CSR, quads and label pairs (Sec. 2.3 pass 4).
// A wave takes groups of kGenWords consecutive words in cell order (a group
// may span several rows).
//   Phase 1, one lane per word: the word's masks from the cut-edge planes
//   (the algebra of k_count), the point bits and first point ids of the four
//   neighbouring cell rows, all stored in LDS as two 32-cell halves, and the
//   group's point list (word, bit) in id order, written by a per-lane loop
//   over the word's point bits.
//   Phase 2, one lane per point: 64 list entries per step.  A point's stencil
//   faces, owned quads and neighbour ids follow from its word's half at its
//   bit; the group's stencil entries and quads are contiguous and in point
//   order, so their positions come from a wave scan of per-point counts.
// Only cells with a point take a lane in phase 2, and each store of a step
// covers consecutive output addresses.
// ---------------------------------------------------------------------------

template <typename T> struct Pair;
template <> struct Pair<uint8_t> { using type = uint16_t; static constexpr int sh = 8; };
template <> struct Pair<uint16_t> { using type = uint32_t; static constexpr int sh = 16; };
template <> struct Pair<uint32_t> { using type = uint64_t; static constexpr int sh = 32; };

// One 32-cell half of a word.
struct GenHalf {
    uint32_t f[6];  // stencil faces -x, +x, -y, +y, -z, +z
    uint32_t q[3];  // quads owned along x, y, z
    uint32_t nm[5];  // point bits of the same cells in rows -y, +y, -z, +z, (-y,-z)
    int32_t nb[5];   // id of the first point of those rows in this half
    uint32_t pad;
};
struct GenWord {
    GenHalf h[2];
    int64_t soff;   // label index of sample (64w, j, k)
    int32_t ci0;    // 64w
    uint32_t cell0;  // linear index of the word's first cell (mod 2^32)
    float py, pz;   // world y and z of the row's cell centres
};
constexpr int kGenList = 64 * kGenWords;  // every cell of a group may hold a point
struct GenLdsBase {
    GenWord word[kGenWords];
    uint16_t list[kGenList];  // (word << 6) | bit, in point-id order
};
template <bool STAGE>
struct GenLds : GenLdsBase {};
// The staged form: one step's stencil ids (<= 6 per point), then its quads
// (<= 3 per point, 16 bytes), then its label pairs, in output order.
template <>
struct GenLds<true> : GenLdsBase {
    alignas(16) uint32_t stage[64 * 3 * 4];
};

__device__ __forceinline__ void wave_lds_sync()
{
    // LDS operations of one wave complete in order; this keeps the compiler
    // from moving LDS accesses of one phase across the other
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One phase-2 step of a lane: its point (list entry), stencil faces, owned
// quads, neighbour ids and the labels its quads need.
template <typename T>
struct GenStep {
    int32_t act;      // the lane holds a point this step
    int32_t R0;       // own point id
    int32_t R[5];     // ids of the cells -y, +y, -z, +z, (-y,-z)
    uint32_t ent;     // list entry
    uint32_t fm, qa;  // face and quad-axis bits (0: no point)
    uint32_t la, lx, ly, lz;  // labels at the sample and at +x, +y, +z
};

template <typename T, bool TWO_D>
__device__ __forceinline__ void generate_front(const VolDesc &d, const GenLdsBase &L, int32_t npg,
                                               int32_t pbase, int32_t base, int lane, int64_t sy,
                                               int64_t sz, GenStep<T> &x)
{
    const int32_t e = base + lane;
    const bool act = e < npg;
    x.act = act;
    x.ent = act ? (uint32_t)L.list[e] : 0u;
    const int u = (int)(x.ent >> 6), i = (int)(x.ent & 63u), ib = i & 31;
    const GenWord &W = L.word[u];
    const GenHalf &H = W.h[i >> 5];
    uint32_t fm = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) fm |= ((H.f[f] >> ib) & 1u) << f;
    const uint32_t qa =
        ((H.q[0] >> ib) & 1u) | (((H.q[1] >> ib) & 1u) << 1) | (((H.q[2] >> ib) & 1u) << 2);
    x.fm = act ? fm : 0u;
    x.qa = act ? qa : 0u;
    // loaded by every lane (a fixed number of loads per step, so waits for
    // them need not wait for the stores issued since): the sample of a lane
    // without a point is the first cell of the group's first word, whose +x,
    // +y and +z samples exist
    const SN_GLOBAL T *s0 = glb(static_cast<const T *>(d.labels)) + W.soff + (W.ci0 + i);
    x.la = s0[0], x.lx = s0[1], x.ly = s0[sy];
    x.lz = TWO_D ? 0u : (uint32_t)s0[sz];  // an image has no +z sample
    const uint32_t below = (1u << ib) - 1u;
#pragma unroll
    for (int n = 0; n < 5; ++n) x.R[n] = H.nb[n] + __popc(H.nm[n] & below);
    x.R0 = pbase + e;
}

// Copy n staged 4*V-byte elements to consecutive output addresses.
template <int V>
__device__ __forceinline__ void copy_staged(SN_GLOBAL uint32_t *out, const uint32_t *st, int32_t n,
                                            int lane)
{
    for (int32_t t = lane; t < n; t += 64) {
        if constexpr (V == 1) {
            out[t] = st[t];
        } else if constexpr (V == 2) {
            reinterpret_cast<SN_GLOBAL v2u *>(out)[t] = reinterpret_cast<const v2u *>(st)[t];
        } else {
            reinterpret_cast<SN_GLOBAL v4u *>(out)[t] = reinterpret_cast<const v4u *>(st)[t];
        }
    }
}

// Stores of one step.  Stencil ids, quads and label pairs are several per
// lane, so each store instruction for them covers the step's output range
// sparsely.  The staged form places them in LDS in output order first and
// copies them out with consecutive-address stores: one memory request per
// touched 64-byte line instead of one per instruction and line, which is what
// bounds meshes with many points per word.  The direct form saves the LDS
// round trip where steps are few.
template <typename T, int MODE, bool STAGE, bool TWO_D>
__device__ __forceinline__ void generate_back(const VolDesc &d, GenLds<STAGE> &L, const GenStep<T> &x,
                                              int32_t sbase, int32_t qbase, int32_t &scarry,
                                              int32_t &qcarry, int lane)
{
    using P = typename Pair<T>::type;
    const int32_t ns = __popc(x.fm), nq = __popc(x.qa);
    const int32_t inc = wave_incl_scan_dpp((ns << 16) | nq, lane);
    const int32_t tot = __builtin_amdgcn_readlane(inc, 63);
    const int32_t ex = inc - ((ns << 16) | nq);
    const int32_t so0 = sbase + scarry, qo0 = qbase + qcarry;  // first entry / quad of the step
    const int32_t nst = tot >> 16, nqt = tot & 0xffff;
    scarry += nst;
    qcarry += nqt;
    // the bounds hold by construction; checked so that no store can leave
    // the mesh's arrays
    const bool fits = so0 + nst <= d.S && qo0 + nqt <= d.Q;
    const bool act = x.act && x.R0 < d.P && fits;
    const int32_t R0 = x.R0, sr = ex >> 16, qr = ex & 0xffff;  // positions within the step
    const auto pack = [](uint32_t f, uint32_t bk) { return (P)(T)f | ((P)(T)bk << Pair<T>::sh); };
    if (act) {
        const int u = (int)(x.ent >> 6), i = (int)(x.ent & 63u);
        const GenWord &W = L.word[u];
        store_point(glb(d.points), R0,
                    (float)(d.origin[0] + d.spacing[0] * ((double)(W.ci0 + i) + 0.5)), W.py, W.pz);
        if (d.faces) glb(d.faces)[R0] = (uint8_t)x.fm;  // null: an extraction without smoothing state
        glb(d.st_off)[R0] = so0 + sr;
        if (d.pcell) glb(d.pcell)[R0] = W.cell0 + (uint32_t)i;
    }
    // ids in face order -x, +x, -y, +y, -z, +z; a point's quads along x, y, z
    auto put_ids = [&](auto *ids) {
        int32_t s = 0;
        if (x.fm & 1u) ids[s++] = R0 - 1;
        if (x.fm & 2u) ids[s++] = R0 + 1;
        if (x.fm & 4u) ids[s++] = x.R[0];
        if (x.fm & 8u) ids[s++] = x.R[1];
        if (x.fm & 16u) ids[s++] = x.R[2];
        if (x.fm & 32u) ids[s++] = x.R[3];
    };
    auto put_quads = [&](auto *qs) {
        int32_t k = 0;
        if (x.qa & 1u) qs[k++] = v4i{x.R[4], x.R[0], R0, x.R[2]};
        if (x.qa & 2u) qs[k++] = v4i{x.R[2] - 1, x.R[2], R0, R0 - 1};
        if (x.qa & 4u) qs[k] = v4i{x.R[0] - 1, R0 - 1, R0, x.R[0]};
    };
    // an image's segments: x-edge (i,j) joins cells (i,j), (i,j-1); y-edge
    // (i,j) joins (i-1,j), (i,j) (right-hand normal facing the edge origin)
    auto put_segs = [&](auto *qs) {
        int32_t k = 0;
        if (x.qa & 1u) qs[k++] = v2i{R0, x.R[0]};
        if (x.qa & 2u) qs[k] = v2i{R0 - 1, R0};
    };
    auto put_pairs = [&](auto *ps) {
        const uint32_t ca = classify<MODE>(x.la, d.cs);
        int32_t k = 0;
        if (x.qa & 1u) ps[k++] = pack(ca, classify<MODE>(x.lx, d.cs));
        if (x.qa & 2u) ps[k++] = pack(ca, classify<MODE>(x.ly, d.cs));
        if (x.qa & 4u) ps[k] = pack(ca, classify<MODE>(x.lz, d.cs));
    };
    if constexpr (!STAGE) {
        if (act) {
            put_ids(glb(d.st_ids) + so0 + sr);
            if (x.qa) {
                if constexpr (TWO_D)
                    put_segs(glb(reinterpret_cast<v2i *>(d.quads)) + qo0 + qr);
                else
                    put_quads(glb(reinterpret_cast<v4i *>(d.quads)) + qo0 + qr);
                put_pairs(glb(static_cast<P *>(d.pairs)) + qo0 + qr);
            }
        }
    } else {
        if (act) put_ids(reinterpret_cast<int32_t *>(L.stage) + sr);
        wave_lds_sync();
        if (fits)
            copy_staged<1>(reinterpret_cast<SN_GLOBAL uint32_t *>(glb(d.st_ids) + so0), L.stage, nst, lane);
        wave_lds_sync();
        if (nqt == 0) return;
        if constexpr (TWO_D) {
            if (act && x.qa) put_segs(reinterpret_cast<v2i *>(L.stage) + qr);
        } else {
            if (act && x.qa) put_quads(reinterpret_cast<v4i *>(L.stage) + qr);
        }
        wave_lds_sync();
        if (fits) {
            if constexpr (TWO_D)
                copy_staged<2>(reinterpret_cast<SN_GLOBAL uint32_t *>(glb(d.quads) + 2 * (int64_t)qo0),
                               L.stage, nqt, lane);
            else
                copy_staged<4>(reinterpret_cast<SN_GLOBAL uint32_t *>(glb(d.quads) + 4 * (int64_t)qo0),
                               L.stage, nqt, lane);
        }
        wave_lds_sync();
        if (act && x.qa) put_pairs(reinterpret_cast<P *>(L.stage) + qr);
        wave_lds_sync();
        if (fits) {
            SN_GLOBAL P *gp = glb(static_cast<P *>(d.pairs)) + qo0;
            const P *sp = reinterpret_cast<const P *>(L.stage);
            for (int32_t t = lane; t < nqt; t += 64) gp[t] = sp[t];
        }
        wave_lds_sync();
    }
}

template <typename T, int MODE, bool STAGE, bool TWO_D>
__device__ __forceinline__ void generate_group(const VolDesc &d, int64_t grp, int lane, GenLds<STAGE> &L)
{
    const Geom &g = d.g;
    const int64_t gw = grp * kGenWords + lane;
    const bool live = lane < kGenWords && gw < g.R * g.W;
    // ---- phase 1: one lane per word
    int32_t r = 0, w = 0, j = 0, k = 0;
    if (live) {
        r = (int32_t)((uint32_t)gw / (uint32_t)g.W);
        w = (int32_t)((uint32_t)gw - (uint32_t)r * (uint32_t)g.W);
        j = (int32_t)((uint32_t)r % (uint32_t)g.CN);
        k = (int32_t)((uint32_t)r / (uint32_t)g.CN);
    }
    bool need = live;
    if constexpr (!STAGE) {
        // sparse meshes: a word without points (the point bits k_count left)
        // has no outputs, so its plane words and neighbour rows are not read,
        // and a group without points ends here
        if (live) need = glb(d.pmask)[gw] != 0;
        if (__builtin_amdgcn_ballot_w64(need) == 0) return;
    }
    PlaneWords p{};
    uint64_t nm[5] = {0, 0, 0, 0, 0};
    int32_t nb[5] = {0, 0, 0, 0, 0};
    int32_t own_p = 0, own_q = 0, own_s = 0;
    if (live && lane == 0) own_p = glb(d.wbP)[gw], own_q = glb(d.wbQ)[gw], own_s = glb(d.wbS)[gw];
    if (need) {
        if constexpr (TWO_D)
            p = plane_words2d(glb(d.planes), g.N * g.O * g.WS, g.WS, (int64_t)j, w);
        else
            p = plane_words(glb(d.planes), g.N * g.O * g.WS, g.WS, j + g.N * (int64_t)k, g.N, w);
        const bool ex[5] = {j >= 1, j + 1 <= g.CN - 1, k >= 1, k + 1 <= g.CO - 1, j >= 1 && k >= 1};
        const int64_t dr[5] = {-1, 1, -g.CN, g.CN, -g.CN - 1};
#pragma unroll
        for (int n = 0; n < 5; ++n)
            if (ex[n]) {
                const int64_t nw = gw + dr[n] * g.W;
                nm[n] = glb(d.pmask)[nw];
                nb[n] = glb(d.wbP)[nw];
            }
    }
    const WordMasks m = word_masks<TWO_D>(p, w, j, k, g);  // all zero for lanes without a word
    const int32_t np = __popcll(m.pt);
    const int32_t npi = wave_incl_scan_dpp(np, lane);
    const int32_t start = npi - np;
    const int32_t npg = __builtin_amdgcn_readlane(npi, 63);
    const int32_t pbase = __builtin_amdgcn_readlane(own_p, 0);
    const int32_t qbase = __builtin_amdgcn_readlane(own_q, 0);
    const int32_t sbase = __builtin_amdgcn_readlane(own_s, 0);
    if (npg == 0) return;
    if (lane < kGenWords) {
        GenWord &W = L.word[lane];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            GenHalf &H = W.h[h];
#pragma unroll
            for (int f = 0; f < 6; ++f) H.f[f] = (uint32_t)(m.f[f] >> (32 * h));
            H.q[0] = (uint32_t)(m.qx >> (32 * h));
            H.q[1] = (uint32_t)(m.qy >> (32 * h));
            H.q[2] = (uint32_t)(m.qz >> (32 * h));
#pragma unroll
            for (int n = 0; n < 5; ++n) {
                H.nm[n] = (uint32_t)(nm[n] >> (32 * h));
                H.nb[n] = nb[n] + (h ? __popc((uint32_t)nm[n]) : 0);
            }
        }
        W.soff = g.M * ((int64_t)j + g.N * (int64_t)k);
        W.ci0 = 64 * w;
        W.cell0 = (uint32_t)(64 * w) + (uint32_t)g.CM * (uint32_t)r;
        W.py = (float)(d.origin[1] + d.spacing[1] * ((double)j + 0.5));
        W.pz = (float)(d.origin[2] + d.spacing[2] * ((double)k + 0.5));
    }
    {
        uint64_t mm = m.pt;
        int32_t pos = start;
        while (mm) {
            L.list[pos++] = (uint16_t)((lane << 6) | (int)__builtin_ctzll(mm));
            mm &= mm - 1;
        }
    }
    wave_lds_sync();
    // ---- phase 2: one lane per point, 64 list entries per step; the LDS
    // reads and label loads of step t+1 are issued before the stores of step t
    const int64_t sy = g.M, sz = g.M * g.N;
    int32_t scarry = 0, qcarry = 0;
    GenStep<T> A, B;  // two steps in flight, alternating
    generate_front<T, TWO_D>(d, L, npg, pbase, 0, lane, sy, sz, A);
    for (int32_t base = 0; base < npg; base += 128) {
        const bool more = base + 64 < npg;
        if (more) generate_front<T, TWO_D>(d, L, npg, pbase, base + 64, lane, sy, sz, B);
        generate_back<T, MODE, STAGE, TWO_D>(d, L, A, sbase, qbase, scarry, qcarry, lane);
        if (!more) break;
        if (base + 128 < npg) generate_front<T, TWO_D>(d, L, npg, pbase, base + 128, lane, sy, sz, A);
        generate_back<T, MODE, STAGE, TWO_D>(d, L, B, sbase, qbase, scarry, qcarry, lane);
    }
    wave_lds_sync();
}

template <typename T, int MODE, bool STAGE, bool TWO_D, class Src>
__device__ __forceinline__ void generate_body(const Src &a, int64_t tile_base, int32_t gpw)
{
    __shared__ GenLds<STAGE> lds[kWavesPerBlock];
    const int64_t t = tile_base + blockIdx.x;
    int v;
    int64_t first;
    const VolDesc &d = vol_of(a, t, v, first);
    const int64_t ngroups = (d.g.R * d.g.W + kGenWords - 1) / kGenWords;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (threadIdx.x == 0 && t == first) glb(d.st_off)[d.P] = (int32_t)d.S;
    const int64_t g0 = (t - first) * (kWavesPerBlock * gpw) + (int64_t)wave * gpw;
    for (int q = 0; q < gpw && g0 + q < ngroups; ++q)
        generate_group<T, MODE, STAGE, TWO_D>(d, g0 + q, lane, lds[wave]);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_generate(const VolDesc *__restrict__ descs,
                                                     const int64_t *__restrict__ prefix,
                                                     int32_t nvol, int64_t tile_base, int32_t gpw)
{
    generate_body<T, MODE, false, false>(ManyVols{descs, prefix, nvol}, tile_base, gpw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_generate_staged(const VolDesc *__restrict__ descs,
                                                            const int64_t *__restrict__ prefix,
                                                            int32_t nvol, int64_t tile_base,
                                                            int32_t gpw)
{
    generate_body<T, MODE, true, false>(ManyVols{descs, prefix, nvol}, tile_base, gpw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_generate_one(OneVol a, int32_t gpw)
{
    generate_body<T, MODE, false, false>(a, 0, gpw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_generate_staged_one(OneVol a, int32_t gpw)
{
    generate_body<T, MODE, true, false>(a, 0, gpw);
}

// The same passes on images (contour segments in the plane).
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_generate2d(const VolDesc *__restrict__ descs,
                                                       const int64_t *__restrict__ prefix,
                                                       int32_t nvol, int64_t tile_base, int32_t gpw)
{
    generate_body<T, MODE, false, true>(ManyVols{descs, prefix, nvol}, tile_base, gpw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_generate2d_staged(const VolDesc *__restrict__ descs,
                                                              const int64_t *__restrict__ prefix,
                                                              int32_t nvol, int64_t tile_base,
                                                              int32_t gpw)
{
    generate_body<T, MODE, true, true>(ManyVols{descs, prefix, nvol}, tile_base, gpw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_generate2d_one(OneVol a, int32_t gpw)
{
    generate_body<T, MODE, false, true>(a, 0, gpw);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_generate2d_staged_one(OneVol a, int32_t gpw)
{
    generate_body<T, MODE, true, true>(a, 0, gpw);
}

// ---------------------------------------------------------------------------
// k_emit: points = origin + spacing * (cell centre + offset)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Own-word data of one batch in lanes u < kU: point bits and first point id.
struct EmitAux {
    uint64_t pm;
    int32_t wbp;
};

__device__ __forceinline__ void issue_emit_aux(const VolDesc &d, const BatchPos &bp, int lane,
                                               EmitAux &A)
{
    A.pm = 0, A.wbp = 0;
    if (lane < bp.nw) {
        A.pm = glb(d.pmask)[bp.g0 + lane];
        A.wbp = glb(d.wbP)[bp.g0 + lane];
    }
}

__device__ __forceinline__ void emit_process(const VolDesc &d, const float *delta_, const BatchPos &bp,
                                             const EmitAux &A, int lane)
{
    const SN_GLOBAL float *delta = delta_ ? glb(delta_) : nullptr;
    const double y0 = (double)bp.j + 0.5, z0 = (double)bp.k + 0.5;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        if (u >= bp.nw) break;
        const uint64_t m = readlane64(A.pm, u);
        if (!lane_bit(m, lane)) continue;
        const int32_t id = __builtin_amdgcn_readlane(A.wbp, u) + (int32_t)rank_below(m);
        double dx = 0.0, dy = 0.0, dz = 0.0;
        if (delta) {
            dx = (double)delta[3 * (int64_t)id];
            dy = (double)delta[3 * (int64_t)id + 1];
            dz = (double)delta[3 * (int64_t)id + 2];
        }
        const double x0 = (double)(64 * (bp.w0 + u) + lane) + 0.5;
        store_point(glb(d.points), id, (float)(d.origin[0] + d.spacing[0] * (x0 + dx)),
                    (float)(d.origin[1] + d.spacing[1] * (y0 + dy)),
                    (float)(d.origin[2] + d.spacing[2] * (z0 + dz)));
    }
}

__device__ __forceinline__ const VolDesc &emit_of(const ManyEmit &a, int64_t t, const SmoothDesc *&sd,
                                                  int64_t &first)
{
    const int v = find_seg(a.prefix, a.nvol, t);
    first = cst(a.prefix)[v];
    sd = &a.sds[v];
    return a.descs[v];
}
__device__ __forceinline__ const VolDesc &emit_of(const OneEmit &a, int64_t, const SmoothDesc *&sd,
                                                  int64_t &first)
{
    first = 0;
    sd = &a.s;
    return a.d;
}

template <class Src>
__device__ __forceinline__ void emit_body(const Src &a, int32_t bpw)
{
    const int64_t t = blockIdx.x;
    const SmoothDesc *sdp;
    int64_t first;
    const VolDesc &d = emit_of(a, t, sdp, first);
    // the last of n sweeps wrote buffer ((n - 1) odd ? da : db); no sweep: centres
    const SmoothDesc &sd = *sdp;
    if (sd.iters > 0 && sd.pcell) return;  // the last sweep wrote the world points
    const float *delta = sd.iters <= 0 ? nullptr : (((sd.iters - 1) & 1) ? sd.da : sd.db);
    const int64_t nbv = d.g.R * d.g.NB;
    const int64_t bt0 = (t - first) * (kWavesPerBlock * bpw);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t b0 = bt0 + (int64_t)wave * bpw;
    const int64_t nb = nbv - b0 < bpw ? nbv - b0 : bpw;
    if (nb <= 0) return;
    EmitAux A0, A1;
    BatchPos P0 = batch_pos(d.g, b0), P1;
    issue_emit_aux(d, P0, lane, A0);
    for (int q = 0; q < nb; q += 2) {
        if (q + 1 < nb) {
            P1 = P0;
            batch_next(d.g, P1);
            issue_emit_aux(d, P1, lane, A1);
        }
        emit_process(d, delta, P0, A0, lane);
        if (q + 1 >= nb) break;
        if (q + 2 < nb) {
            P0 = P1;
            batch_next(d.g, P0);
            issue_emit_aux(d, P0, lane, A0);
        }
        emit_process(d, delta, P1, A1, lane);
    }
}

__global__ __launch_bounds__(kBlock) void k_emit(const VolDesc *__restrict__ descs,
                                                 const SmoothDesc *__restrict__ sds,
                                                 const int64_t *__restrict__ prefix, int32_t nvol,
                                                 int32_t bpw)
{
    emit_body(ManyEmit{descs, sds, prefix, nvol}, bpw);
}

__global__ __launch_bounds__(kBlock) void k_emit_one(OneEmit a, int32_t bpw)
{
    emit_body(a, bpw);
}

// ---------------------------------------------------------------------------
// k_jacobi: one sweep of Eq. (1) on the offsets, FP64 arithmetic, FP32 storage
// ---------------------------------------------------------------------------
// The offset of point p moves by lambda times the mean over its stencil
// neighbours q of (p_q - p_p) = (unit face step) + (delta_q - delta_p), then
// is clamped to the box [-d, d]^3 (Sec. 2.4, Eq. (1)).  Neighbours are summed
// in face order -x, +x, -y, +y, -z, +z.

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so that stencil neighbours (a row or a
// slice of points away) are mostly in its own L2.
__device__ __forceinline__ int64_t xcd_block(uint32_t b, uint32_t nb)
{
    const uint32_t x = b & 7u, i = b >> 3, q = nb >> 3, r = nb & 7u;
    return (int64_t)x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ double face_term(int face, int axis, double n, double own)
{
    // component `axis` of p_q - p_p for the neighbour across `face`
    const double step = (face & 1) ? 1.0 : -1.0;
    return (face >> 1) == axis ? step + n - own : n - own;
}

// Eq. (1) for one point with face mask fc: its offset (x, y, z) moves by
// lambda times the mean over its faces of (unit step + neighbour offset - own
// offset); nx, ny, nz hold the neighbour offsets in face order.  The first
// sweep and its table (first_offset) use this form; the later sweeps write the
// same arithmetic inline, which keeps their neighbour values out of arrays
// (40 registers instead of 60).
__device__ __forceinline__ void sweep_update(const SmoothDesc &s, uint32_t fc, const float (&nx)[6],
                                             const float (&ny)[6], const float (&nz)[6], double &x,
                                             double &y, double &z)
{
    const int n = __popc(fc);
    if (n == 0) return;
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int face = 0; face < 6; ++face) {
        if (!((fc >> face) & 1u)) continue;
        sx += face_term(face, 0, (double)nx[face], x);
        sy += face_term(face, 1, (double)ny[face], y);
        sz += face_term(face, 2, (double)nz[face], z);
    }
    const double inv = 1.0 / (double)n;
    x = x + s.lam * (sx * inv);
    y = y + s.lam * (sy * inv);
    z = z + s.lam * (sz * inv);
}



// Hold the offset in the constraint region (a box of half-width d per axis, or
// a sphere of radius d), store it, and in the mesh's last sweep also the
// world point origin + spacing * (cell centre + stored offset), from the
// point's cell index (the world-coordinate output, fused into the sweep).
// NT: streaming (non-temporal) stores, for meshes whose sweep data does not
// stay in the caches between sweeps anyway.
__device__ __forceinline__ void constrain(const SmoothDesc &s, double &x, double &y, double &z)
{
    const double c = s.dist;
    if (s.sphere) {
        // back onto the sphere of radius c around the cell centre
        const double l2 = x * x + y * y + z * z;
        if (l2 > c * c) {
            const double f = c / sqrt(l2);
            x *= f, y *= f, z *= f;
        }
    } else {
        x = fmin(fmax(x, -c), c);
        y = fmin(fmax(y, -c), c);
        z = fmin(fmax(z, -c), c);
    }
}

template <bool NT = false>
__device__ __forceinline__ void store_offset(const SmoothDesc &s, SN_GLOBAL float *dout, int64_t p,
                                             double x, double y, double z, bool last, uint32_t cell)
{
    constrain(s, x, y, z);
    const float fx = (float)x, fy = (float)y, fz = (float)z;
    if constexpr (NT) {
        __builtin_nontemporal_store(fx, dout + 3 * p);
        __builtin_nontemporal_store(fy, dout + 3 * p + 1);
        __builtin_nontemporal_store(fz, dout + 3 * p + 2);
    } else {
        dout[3 * p] = fx;
        dout[3 * p + 1] = fy;
        dout[3 * p + 2] = fz;
    }
    if (last) {
        const uint32_t r = udiv(cell, s.CM), i = cell - r * s.CM.d;
        const uint32_t k = udiv(r, s.CN), j = r - k * s.CN.d;
        SN_GLOBAL float *o = glb(s.points) + 3 * p;
        o[0] = (float)(s.origin[0] + s.spacing[0] * ((double)i + 0.5 + (double)fx));
        o[1] = (float)(s.origin[1] + s.spacing[1] * ((double)j + 0.5 + (double)fy));
        o[2] = (float)(s.origin[2] + s.spacing[2] * ((double)k + 0.5 + (double)fz));
    }
}

// The offset the first sweep gives a point with face mask f, as that sweep
// stores it: every input offset is zero, so it depends on f alone.
__device__ __forceinline__ void first_offset(const SmoothDesc &s, uint32_t f, float &fx, float &fy,
                                             float &fz)
{
    const float zero[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    double x = 0.0, y = 0.0, z = 0.0;
    sweep_update(s, f, zero, zero, zero, x, y, z);
    constrain(s, x, y, z);
    fx = (float)x, fy = (float)y, fz = (float)z;
}

// The y/z stencil neighbours of point p (face mask f) from the CSR stencil:
// ids of -y, +y, -z, +z, -1 where absent.
__device__ __forceinline__ v4i stencil_yz(const SmoothDesc &s, uint32_t f, int64_t p)
{
    int64_t e = glb(s.off)[p];
    v4i q = {-1, -1, -1, -1};
#pragma unroll
    for (int face = 0; face < 6; ++face) {
        if (!((f >> face) & 1u)) continue;
        const int32_t id = glb(s.ids)[e++];
        if (face == 2) q.x = id;
        if (face == 3) q.y = id;
        if (face == 4) q.z = id;
        if (face == 5) q.w = id;
    }
    return q;
}

// The packed neighbour word of point p (SmoothDesc::pack_yb > 0): face bits
// -x, +x and the id distances of the y/z neighbours q (ids of -y, +y, -z,
// +z, -1 where absent).
__device__ __forceinline__ uint64_t pack_nbr(const SmoothDesc &s, uint32_t f, int64_t p, v4i q)
{
    const uint32_t yb = (uint32_t)s.pack_yb, zb = (uint32_t)s.pack_zb;
    uint64_t w = f & 3u;
    w |= (uint64_t)(q.x >= 0 ? p - q.x : 0) << 2;
    w |= (uint64_t)(q.y >= 0 ? q.y - p : 0) << (2 + yb);
    w |= (uint64_t)(q.z >= 0 ? p - q.z : 0) << (2 + 2 * yb);
    w |= (uint64_t)(q.w >= 0 ? q.w - p : 0) << (2 + 2 * yb + zb);
    return w;
}

// Face mask and y/z neighbour ids of point p from its packed word.
__device__ __forceinline__ void unpack_nbr(const SmoothDesc &s, uint64_t w, int64_t p, uint32_t &f,
                                           v4i &q)
{
    const uint32_t yb = (uint32_t)s.pack_yb, zb = (uint32_t)s.pack_zb;
    const uint64_t ym = (1ull << yb) - 1, zm = (1ull << zb) - 1;
    const int32_t a = (int32_t)((w >> 2) & ym), b = (int32_t)((w >> (2 + yb)) & ym);
    const int32_t c = (int32_t)((w >> (2 + 2 * yb)) & zm), d = (int32_t)((w >> (2 + 2 * yb + zb)) & zm);
    const int32_t pi = (int32_t)p;
    f = ((uint32_t)w & 3u) | (a ? 4u : 0u) | (b ? 8u : 0u) | (c ? 16u : 0u) | (d ? 32u : 0u);
    q = v4i{a ? pi - a : -1, b ? pi + b : -1, c ? pi - c : -1, d ? pi + d : -1};
}

// Write point p's entry of the neighbour table in the mesh's form.
__device__ __forceinline__ void store_nbr(const SmoothDesc &s, uint32_t f, int64_t p, v4i q)
{
    if (s.pack_yb)
        glb(reinterpret_cast<uint64_t *>(s.nbr))[p] = pack_nbr(s, f, p, q);
    else
        glb(reinterpret_cast<v4i *>(s.nbr))[p] = q;
}

// Sweep 0: every input offset is zero, so p_q - p_p is the face step alone.
// Reads the CSR stencil once and writes the y/z neighbour table.
// Blocks of a sweep launch that carry points: a launch over many meshes has
// exactly those; for a single mesh they follow from its point count, so any
// blocks of a larger grid leave at once (and take no part in the XCD remap).
template <int K>
__device__ __forceinline__ uint32_t sweep_blocks(const ManySmooth &) { return gridDim.x; }
template <int K>
__device__ __forceinline__ uint32_t sweep_blocks(const OneSmooth &a)
{
    return (uint32_t)((a.s.P + kSweepBlock * K - 1) / (kSweepBlock * K));
}

// Blocks are handed to the 8 XCDs round robin (block b runs on XCD b % 8).
// Slab-chunked order: XCD x takes logical blocks x*C .. x*C + C - 1 of each
// run of 8*C, so that with C about a sixteenth of a slab's blocks, the y and z
// neighbours a block gathers were recently touched in the same L2.  A
// bijection on [0, nb): the tail that does not fill a run keeps its block.
__device__ __forceinline__ uint32_t slab_chunk_block(uint32_t b, uint32_t nb, uint32_t C)
{
    const uint32_t S = 8u * C;
    const uint32_t full = nb / S * S;
    if (C <= 1u || b >= full) return b;
    const uint32_t x = b & 7u, i = b >> 3;
    return (i / C) * S + x * C + (i % C);
}

// Logical block of a sweep.  Small meshes, whose sweep data fits the
// last-level cache, gain from XCD-contiguous blocks (stencil neighbours in
// the same L2), and so does a launch over many meshes whose sweep data
// together fits (with one chunk per wave; the hardware's order with two was
// 10.0 ms against 8.3 ms for a batch of 64 volumes).  A single large mesh
// streams from HBM and takes the slab-chunked order, and so does a launch
// over many meshes whose data together is beyond the caches, with runs of
// kManySweepChunk blocks (64-volume batch of 20.5 M points: 4.19-4.29 ms of
// sweeps for runs of 64 to 1024 blocks, 4.38 ms XCD-contiguous, 4.47 ms in
// hardware order).  BIG as for jacobi_body; a launch over many meshes gives
// all of them the same big.
constexpr uint32_t kManySweepChunk = 128;
template <int K, int BIG>
__device__ __forceinline__ int64_t sweep_block(const ManySmooth &a, uint32_t b, uint32_t nb)
{
    if (K != 1) return (int64_t)b;
    const bool big = BIG < 0 ? a.sds[0].big != 0 : BIG == 1;
    return big ? (int64_t)slab_chunk_block(b, nb, kManySweepChunk) : xcd_block(b, nb);
}
template <int K, int BIG>
__device__ __forceinline__ int64_t sweep_block(const OneSmooth &a, uint32_t b, uint32_t nb)
{
    return !a.s.big ? xcd_block(b, nb) : (int64_t)slab_chunk_block(b, nb, (uint32_t)a.s.chunk);
}

// block0: the launch covers logical blocks block0 .. (a launch over many
// meshes that runs the first sweep of its one-sweep meshes only)
template <int K, class Src>
__device__ __forceinline__ void jacobi_first_body(const Src &a, int64_t block0)
{
    const uint32_t nb = sweep_blocks<K>(a);
    if (blockIdx.x >= nb) return;
    const int64_t b = block0 + sweep_block<K, -1>(a, blockIdx.x, nb);
    int64_t first;
    const SmoothDesc &s = smooth_of(a, b, first);
    if (s.iters < 1) return;
    SN_GLOBAL float *dout = glb(s.db);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int64_t p = (b - first) * (kSweepBlock * K) + c * kSweepBlock + threadIdx.x;
        if (p >= s.P) break;
        const uint32_t f = glb(s.faces)[p];
        store_nbr(s, f, p, stencil_yz(s, f, p));
        const float zero[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        double x = 0.0, y = 0.0, z = 0.0;
        sweep_update(s, f, zero, zero, zero, x, y, z);
        const bool last = s.iters == 1 && s.pcell;
        store_offset(s, dout, p, x, y, z, last, last ? glb(s.pcell)[p] : 0u);
    }
}

template <int K>
__global__ __launch_bounds__(kSweepBlock) void k_jacobi_first(const SmoothDesc *__restrict__ sds,
                                                      const int64_t *__restrict__ prefix,
                                                      int32_t nvol, int64_t block0)
{
    jacobi_first_body<K>(ManySmooth{sds, prefix, nvol}, block0);
}

template <int K>
__global__ __launch_bounds__(kSweepBlock) void k_jacobi_first_one(OneSmooth a)
{
    jacobi_first_body<K>(a, 0);
}

// Whole-wave DPP shifts by one lane (no LDS traffic): lane l receives lane
// l - 1 (wave_shr:1) or lane l + 1 (wave_shl:1); the end lane that has no
// source is overwritten by the caller.
__device__ __forceinline__ float shfl_up1(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x138, 0xf, 0xf, false));
}

__device__ __forceinline__ float shfl_down1(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ float readlane_f(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Sweeps 1..n-1.  Each wave holds K chunks of 64 consecutive
// points, one point per lane and chunk; all loads of the wave are issued
// before any use.  The -x / +x neighbours of point p are points p - 1 / p + 1
// (consecutive cells of a row get consecutive ids), read from the adjacent
// lane; only the first and the last point of the wave load them.
//
// FUSED: sweeps 0 and 1 in one launch (it = 1).  The first sweep's offset of a
// point depends on its face mask alone (every input offset is zero), so the
// block tabulates it for all 64 masks in LDS, exactly as k_jacobi_first stores
// it, and sweep 1 reads its own and its neighbours' first-sweep offsets from
// the table through their face bytes instead of from an offset buffer; it
// also builds the neighbour table from the CSR stencil.  The result equals
// the two separate sweeps bit for bit.
// BIG: 1 for a single mesh whose sweep data is far beyond the caches (its
// read-once streams are loaded and its offsets stored with non-temporal
// hints), 0 for one that is not, -1 to decide per mesh at run time (a launch
// over many meshes).  A compile-time choice keeps the non-temporal loads from
// being merged with the ordinary ones of the other branch.
template <int K, bool FUSED, int BIG, class Src>
__device__ __forceinline__ void jacobi_body(const Src &a, int32_t it)
{
    const uint32_t nbl = sweep_blocks<K>(a);
    if (blockIdx.x >= nbl) return;
    const int64_t b = sweep_block<K, BIG>(a, blockIdx.x, nbl);
    int64_t first;
    const SmoothDesc &s = smooth_of(a, b, first);
    if (it >= s.iters) return;  // this mesh has finished its sweeps
    __shared__ float s_first[FUSED ? 64 * 3 : 1];
    if constexpr (FUSED) {
        // every wave of the block reaches this barrier (no exit before it
        // depends on the wave)
        if (threadIdx.x < 64)
            first_offset(s, threadIdx.x, s_first[3 * threadIdx.x], s_first[3 * threadIdx.x + 1],
                         s_first[3 * threadIdx.x + 2]);
        __syncthreads();
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t p0 = (b - first) * (kSweepBlock * K) + (int64_t)wave * (64 * K);
    const int64_t P = s.P;
    if (p0 >= P) return;
    const SN_GLOBAL float *din = glb((it & 1) ? s.db : s.da);
    SN_GLOBAL float *dout = glb((it & 1) ? s.da : s.db);
    const SN_GLOBAL v4i *nbr = glb(reinterpret_cast<const v4i *>(s.nbr));

    // the mesh's last sweep also writes world points from the cell indices
    const bool last = it == s.iters - 1 && s.pcell;
    const bool big = BIG < 0 ? s.big != 0 : BIG == 1;
    uint32_t f[K], cell[K];
    v4i nb[K];
    float ox[K], oy[K], oz[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int64_t p = p0 + 64 * c + lane;
        f[c] = 0, cell[c] = 0, nb[c] = v4i{-1, -1, -1, -1}, ox[c] = oy[c] = oz[c] = 0.f;
        if (p < P) {
            if constexpr (FUSED) {
                f[c] = glb(s.faces)[p];
                nb[c] = stencil_yz(s, f[c], p);
                store_nbr(s, f[c], p, nb[c]);
                ox[c] = s_first[3 * f[c]], oy[c] = s_first[3 * f[c] + 1], oz[c] = s_first[3 * f[c] + 2];
            } else {
                // own offset first: it is in flight while the table word is
                // awaited for the neighbour ids
                ox[c] = din[3 * p], oy[c] = din[3 * p + 1], oz[c] = din[3 * p + 2];
                if (s.pack_yb) {  // one 8-byte word: face bits and id distances
                    const SN_GLOBAL uint64_t *nw = glb(reinterpret_cast<const uint64_t *>(s.nbr));
                    uint64_t w;
                    if constexpr (BIG == 1)
                        w = __builtin_nontemporal_load(nw + p);
                    else if constexpr (BIG == 0)
                        w = nw[p];
                    else
                        w = big ? __builtin_nontemporal_load(nw + p) : nw[p];
                    unpack_nbr(s, w, p, f[c], nb[c]);
                } else if (big) {  // large meshes: read-once streams
                    f[c] = __builtin_nontemporal_load(glb(s.faces) + p);
                    nb[c] = __builtin_nontemporal_load(nbr + p);
                } else {
                    f[c] = glb(s.faces)[p];
                    nb[c] = nbr[p];
                }
            }
            if (last) cell[c] = glb(s.pcell)[p];
        }
    }
    // wave halo: -x of the first point, +x of the last one (p0 + 64K - 1)
    float hmx = 0.f, hmy = 0.f, hmz = 0.f, hpx = 0.f, hpy = 0.f, hpz = 0.f;
    if (lane == 0 && (f[0] & 1u)) {
        if constexpr (FUSED) {
            const uint32_t fq = glb(s.faces)[p0 - 1];
            hmx = s_first[3 * fq], hmy = s_first[3 * fq + 1], hmz = s_first[3 * fq + 2];
        } else {
            hmx = din[3 * (p0 - 1)], hmy = din[3 * (p0 - 1) + 1], hmz = din[3 * (p0 - 1) + 2];
        }
    }
    if (lane == 63 && (f[K - 1] & 2u)) {
        const int64_t q = p0 + 64 * K;
        if constexpr (FUSED) {
            const uint32_t fq = glb(s.faces)[q];
            hpx = s_first[3 * fq], hpy = s_first[3 * fq + 1], hpz = s_first[3 * fq + 2];
        } else {
            hpx = din[3 * q], hpy = din[3 * q + 1], hpz = din[3 * q + 2];
        }
    }
    // y / z neighbours
    float gx[K][4], gy[K][4], gz[K][4];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int32_t id[4] = {nb[c].x, nb[c].y, nb[c].z, nb[c].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            gx[c][e] = gy[c][e] = gz[c][e] = 0.f;
            if (id[e] >= 0) {
                const int64_t q = id[e];
                if constexpr (FUSED) {
                    const uint32_t fq = glb(s.faces)[q];
                    gx[c][e] = s_first[3 * fq], gy[c][e] = s_first[3 * fq + 1], gz[c][e] = s_first[3 * fq + 2];
                } else {
                    gx[c][e] = din[3 * q], gy[c][e] = din[3 * q + 1], gz[c][e] = din[3 * q + 2];
                }
            }
        }
    }
    // x neighbours, exchanged with every lane of the wave active:
    // -x from lane - 1 (lane 0: the previous chunk's lane 63, or the halo),
    // +x from lane + 1 (lane 63: the next chunk's lane 0, or the halo)
    float mx[K], my[K], mz[K], px[K], py[K], pz[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        mx[c] = shfl_up1(ox[c]), my[c] = shfl_up1(oy[c]), mz[c] = shfl_up1(oz[c]);
        px[c] = shfl_down1(ox[c]), py[c] = shfl_down1(oy[c]), pz[c] = shfl_down1(oz[c]);
        const float lmx = c > 0 ? readlane_f(ox[c > 0 ? c - 1 : 0], 63) : hmx;
        const float lmy = c > 0 ? readlane_f(oy[c > 0 ? c - 1 : 0], 63) : hmy;
        const float lmz = c > 0 ? readlane_f(oz[c > 0 ? c - 1 : 0], 63) : hmz;
        const float lpx = c + 1 < K ? readlane_f(ox[c + 1 < K ? c + 1 : 0], 0) : hpx;
        const float lpy = c + 1 < K ? readlane_f(oy[c + 1 < K ? c + 1 : 0], 0) : hpy;
        const float lpz = c + 1 < K ? readlane_f(oz[c + 1 < K ? c + 1 : 0], 0) : hpz;
        if (lane == 0) mx[c] = lmx, my[c] = lmy, mz[c] = lmz;
        if (lane == 63) px[c] = lpx, py[c] = lpy, pz[c] = lpz;
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int64_t p = p0 + 64 * c + lane;
        if (p >= P) continue;
        const uint32_t fc = f[c];
        double x = (double)ox[c], y = (double)oy[c], z = (double)oz[c];
        const int n = __popc(fc);
        if (n > 0) {
            const float nx[6] = {mx[c], px[c], gx[c][0], gx[c][1], gx[c][2], gx[c][3]};
            const float ny[6] = {my[c], py[c], gy[c][0], gy[c][1], gy[c][2], gy[c][3]};
            const float nz[6] = {mz[c], pz[c], gz[c][0], gz[c][1], gz[c][2], gz[c][3]};
            double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
            for (int face = 0; face < 6; ++face) {
                if (!((fc >> face) & 1u)) continue;
                sx += face_term(face, 0, (double)nx[face], x);
                sy += face_term(face, 1, (double)ny[face], y);
                sz += face_term(face, 2, (double)nz[face], z);
            }
            const double inv = 1.0 / (double)n;
            x = x + s.lam * (sx * inv);
            y = y + s.lam * (sy * inv);
            z = z + s.lam * (sz * inv);
        }
        if (big)  // large meshes: streaming stores
            store_offset<true>(s, dout, p, x, y, z, last, cell[c]);
        else
            store_offset<false>(s, dout, p, x, y, z, last, cell[c]);
    }
}

// BIG: 1 for a launch whose meshes' sweep data together is far beyond the
// caches (every mesh's descriptor then says big), else 0
template <int K, int BIG>
__global__ __launch_bounds__(kSweepBlock) void k_jacobi(const SmoothDesc *__restrict__ sds,
                                                const int64_t *__restrict__ prefix, int32_t nvol,
                                                int32_t it)
{
    jacobi_body<K, false, BIG>(ManySmooth{sds, prefix, nvol}, it);
}

template <int K, int BIG>
__global__ __launch_bounds__(kSweepBlock) void k_jacobi_one(OneSmooth a, int32_t it)
{
    jacobi_body<K, false, BIG>(a, it);
}

// Sweeps 0 and 1 in one launch (meshes of at least two sweeps; in a launch
// over many meshes these are the leading blocks, meshes being ordered by
// descending sweep count).
template <int K>
__global__ __launch_bounds__(kSweepBlock) void k_jacobi_first2_one(OneSmooth a)
{
    jacobi_body<K, true, -1>(a, 1);
}

template <int K>
__global__ __launch_bounds__(kSweepBlock) void k_jacobi_first2(const SmoothDesc *__restrict__ sds,
                                                       const int64_t *__restrict__ prefix,
                                                       int32_t nvol)
{
    jacobi_body<K, true, -1>(ManySmooth{sds, prefix, nvol}, 1);
}

// ---------------------------------------------------------------------------
// k_tri: quad (A,B,C,D) -> (A,B,C), (A,C,D)
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void tri_pairs(const VolDesc &d, int64_t q)
{
    const SN_GLOBAL T *src = glb(static_cast<const T *>(d.pairs));
    SN_GLOBAL T *dst = glb(static_cast<T *>(d.tri_pairs));
    const T f = src[2 * q], b = src[2 * q + 1];
    dst[4 * q] = f, dst[4 * q + 1] = b, dst[4 * q + 2] = f, dst[4 * q + 3] = b;
}

template <class Src>
__device__ __forceinline__ void tri_body(const Src &a)
{
    const int64_t b = blockIdx.x;
    int v;
    int64_t first;
    const VolDesc &d = vol_of(a, b, v, first);
    const int64_t q = (b - first) * 256 + threadIdx.x;
    if (q >= d.Q || d.prim != 3) return;
    const v4i s = glb(reinterpret_cast<const v4i *>(d.quads))[q];
    SN_GLOBAL int32_t *o = glb(d.tris) + 6 * q;
    o[0] = s.x, o[1] = s.y, o[2] = s.z, o[3] = s.x, o[4] = s.z, o[5] = s.w;
    if (d.dtype == 1) tri_pairs<uint8_t>(d, q);
    else if (d.dtype == 2) tri_pairs<uint16_t>(d, q);
    else tri_pairs<uint32_t>(d, q);
}

__global__ __launch_bounds__(256) void k_tri(const VolDesc *__restrict__ descs,
                                             const int64_t *__restrict__ prefix, int32_t nvol)
{
    tri_body(ManyVols{descs, prefix, nvol});
}

__global__ __launch_bounds__(256) void k_tri_one(OneVol a)
{
    tri_body(a);
}

// ---------------------------------------------------------------------------
// k_tri_rule: quads -> triangles with a geometric choice of diagonal (Sec. 2.5)
// ---------------------------------------------------------------------------
// Split AC gives (A,B,C), (A,C,D); split BD gives (A,B,D), (B,C,D); both keep
// the quad's orientation.  Measures, in FP64 on the mesh's FP32 world points,
// evaluated in the order written (no contraction), ties to AC:
//   shortest diagonal: |c - a|^2 <= |d - b|^2;
//   minimum area:      area(ABC) + area(ACD) <= area(ABD) + area(BCD);
//   most planar:       cos(normals of ABC, ACD) >= cos(normals of ABD, BCD),
//                      -2 for a split with a degenerate triangle.

struct D3 {
    double x, y, z;
};

__device__ __forceinline__ D3 load_point(const float *pts, int32_t id)
{
    const SN_GLOBAL float *p = glb(pts) + 3 * (int64_t)id;
    return D3{(double)p[0], (double)p[1], (double)p[2]};
}

#pragma clang fp contract(off)
__device__ __forceinline__ D3 d3_sub(const D3 &u, const D3 &v) { return D3{u.x - v.x, u.y - v.y, u.z - v.z}; }
__device__ __forceinline__ double d3_dot(const D3 &u, const D3 &v) { return u.x * v.x + u.y * v.y + u.z * v.z; }
__device__ __forceinline__ D3 d3_cross(const D3 &u, const D3 &v)
{
    return D3{u.y * v.z - u.z * v.y, u.z * v.x - u.x * v.z, u.x * v.y - u.y * v.x};
}
__device__ __forceinline__ D3 tri_normal3(const D3 &a, const D3 &b, const D3 &c)
{
    return d3_cross(d3_sub(b, a), d3_sub(c, a));
}
__device__ __forceinline__ double tri_area3(const D3 &a, const D3 &b, const D3 &c)
{
    const D3 n = tri_normal3(a, b, c);
    return 0.5 * sqrt(d3_dot(n, n));
}
__device__ __forceinline__ double normals_cos3(const D3 &n1, const D3 &n2)
{
    const double l = sqrt(d3_dot(n1, n1) * d3_dot(n2, n2));
    return l > 0.0 ? d3_dot(n1, n2) / l : -2.0;
}

template <int RULE>
__device__ __forceinline__ bool split_ac(const D3 &a, const D3 &b, const D3 &c, const D3 &d)
{
    if constexpr (RULE == 1) {
        const D3 ac = d3_sub(c, a), bd = d3_sub(d, b);
        return d3_dot(ac, ac) <= d3_dot(bd, bd);
    } else if constexpr (RULE == 2) {
        return tri_area3(a, b, c) + tri_area3(a, c, d) <= tri_area3(a, b, d) + tri_area3(b, c, d);
    } else {
        return normals_cos3(tri_normal3(a, b, c), tri_normal3(a, c, d)) >=
               normals_cos3(tri_normal3(a, b, d), tri_normal3(b, c, d));
    }
}
#pragma clang fp contract(on)

template <typename T, int RULE>
__global__ __launch_bounds__(256) void k_tri_rule(const int32_t *__restrict__ quads,
                                                  const float *__restrict__ pts,
                                                  const T *__restrict__ pairs, int64_t Q,
                                                  int32_t *__restrict__ tris,
                                                  T *__restrict__ tri_pairs)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= Q) return;
    const v4i v = glb(reinterpret_cast<const v4i *>(quads))[q];
    bool ac = true;
    if constexpr (RULE != 0)
        ac = split_ac<RULE>(load_point(pts, v.x), load_point(pts, v.y), load_point(pts, v.z),
                            load_point(pts, v.w));
    SN_GLOBAL int32_t *o = glb(tris) + 6 * q;
    if (ac) {
        o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.x, o[4] = v.z, o[5] = v.w;
    } else {
        o[0] = v.x, o[1] = v.y, o[2] = v.w, o[3] = v.y, o[4] = v.z, o[5] = v.w;
    }
    if (tri_pairs) {
        const T f = glb(pairs)[2 * q], bk = glb(pairs)[2 * q + 1];
        SN_GLOBAL T *tp = glb(tri_pairs) + 4 * q;
        tp[0] = f, tp[1] = bk, tp[2] = f, tp[3] = bk;
    }
}

hipError_t launch_tri_rule(int32_t rule, int32_t dtype, const int32_t *quads, const float *pts,
                           const void *pairs, int64_t Q, int32_t *tris, void *tri_pairs, hipStream_t s)
{
    if (Q <= 0) return hipSuccess;
    const dim3 grid((uint32_t)((Q + 255) / 256)), block(256);
#define SN_TRI_RULE(T)                                                                                \
    switch (rule) {                                                                                   \
    case 0: hipLaunchKernelGGL((k_tri_rule<T, 0>), grid, block, 0, s, quads, pts,                    \
                               static_cast<const T *>(pairs), Q, tris, static_cast<T *>(tri_pairs)); \
        break;                                                                                        \
    case 1: hipLaunchKernelGGL((k_tri_rule<T, 1>), grid, block, 0, s, quads, pts,                    \
                               static_cast<const T *>(pairs), Q, tris, static_cast<T *>(tri_pairs)); \
        break;                                                                                        \
    case 2: hipLaunchKernelGGL((k_tri_rule<T, 2>), grid, block, 0, s, quads, pts,                    \
                               static_cast<const T *>(pairs), Q, tris, static_cast<T *>(tri_pairs)); \
        break;                                                                                        \
    case 3: hipLaunchKernelGGL((k_tri_rule<T, 3>), grid, block, 0, s, quads, pts,                    \
                               static_cast<const T *>(pairs), Q, tris, static_cast<T *>(tri_pairs)); \
        break;                                                                                        \
    default: return hipErrorInvalidValue;                                                             \
    }
    if (dtype == 1) {
        SN_TRI_RULE(uint8_t)
    } else if (dtype == 2) {
        SN_TRI_RULE(uint16_t)
    } else if (dtype == 4) {
        SN_TRI_RULE(uint32_t)
    } else {
        return hipErrorInvalidValue;
    }
#undef SN_TRI_RULE
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// One instantiation per (label type, classification mode); every volume of a
// launch has that key.
#define SN_KEY_SWITCH(KERNEL, ...)                                                          \
    switch (dtype * 4 + mode) {                                                             \
    case 1 * 4 + CLS_IDENT: hipLaunchKernelGGL((KERNEL<uint8_t, CLS_IDENT>), __VA_ARGS__); break; \
    case 1 * 4 + CLS_BITMAP: hipLaunchKernelGGL((KERNEL<uint8_t, CLS_BITMAP>), __VA_ARGS__); break; \
    case 2 * 4 + CLS_IDENT: hipLaunchKernelGGL((KERNEL<uint16_t, CLS_IDENT>), __VA_ARGS__); break; \
    case 2 * 4 + CLS_BITMAP: hipLaunchKernelGGL((KERNEL<uint16_t, CLS_BITMAP>), __VA_ARGS__); break; \
    case 4 * 4 + CLS_IDENT: hipLaunchKernelGGL((KERNEL<uint32_t, CLS_IDENT>), __VA_ARGS__); break; \
    case 4 * 4 + CLS_BITMAP: hipLaunchKernelGGL((KERNEL<uint32_t, CLS_BITMAP>), __VA_ARGS__); break; \
    case 4 * 4 + CLS_SORTED: hipLaunchKernelGGL((KERNEL<uint32_t, CLS_SORTED>), __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                   \
    }

hipError_t launch_edges(int32_t dtype, int32_t mode, bool wide, const VolDesc *d_descs,
                        const int64_t *d_tile_prefix, int32_t nvol, int64_t tile_base,
                        int64_t ntiles, uint64_t *d_zero, int64_t nzero, int32_t spw, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (wide) {
        SN_KEY_SWITCH(k_edges_wide, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs,
                      d_tile_prefix, nvol, tile_base, d_zero, nzero, spw)
    } else {
        SN_KEY_SWITCH(k_edges_narrow, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs,
                      d_tile_prefix, nvol, tile_base, d_zero, nzero, spw)
    }
    return hipGetLastError();
}

hipError_t launch_edges_one(const VolDesc &d, bool wide, int64_t ntiles, uint64_t *d_zero,
                            int64_t nzero, int32_t spw, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const int32_t dtype = d.dtype, mode = d.cs.mode;
    if (wide) {
        SN_KEY_SWITCH(k_edges_wide_one, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, OneVol{d},
                      d_zero, nzero, spw)
    } else {
        SN_KEY_SWITCH(k_edges_narrow_one, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, OneVol{d},
                      d_zero, nzero, spw)
    }
    return hipGetLastError();
}

hipError_t launch_count(const VolDesc *d_descs, const int64_t *d_tile_prefix, int32_t nvol,
                        int64_t ntiles, int32_t words_per_thread, uint64_t *d_status,
                        uint32_t *d_ticket, const CountOut &out, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (words_per_thread == kCountWideV)
        hipLaunchKernelGGL(k_count<kCountWideV>, dim3((uint32_t)ntiles), dim3(kCountBlock), 0, s,
                           d_descs, d_tile_prefix, nvol, d_status, d_ticket, out);
    else
        hipLaunchKernelGGL(k_count<1>, dim3((uint32_t)ntiles), dim3(kCountBlock), 0, s, d_descs,
                           d_tile_prefix, nvol, d_status, d_ticket, out);
    return hipGetLastError();
}

hipError_t launch_count_one(const VolDesc &d, int64_t ntiles, int32_t words_per_thread,
                            uint64_t *d_status, uint32_t *d_ticket, const CountOut &out, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (words_per_thread == kCountWideV)
        hipLaunchKernelGGL(k_count_one<kCountWideV>, dim3((uint32_t)ntiles), dim3(kCountBlock), 0, s,
                           OneVol{d}, d_status, d_ticket, out);
    else
        hipLaunchKernelGGL(k_count_one<1>, dim3((uint32_t)ntiles), dim3(kCountBlock), 0, s, OneVol{d},
                           d_status, d_ticket, out);
    return hipGetLastError();
}

hipError_t launch_generate(int32_t dtype, int32_t mode, bool staged, bool two_d, const VolDesc *d_descs,
                           const int64_t *d_tile_prefix, int32_t nvol, int64_t tile_base,
                           int64_t ntiles, int32_t bpw, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (two_d && staged) {
        SN_KEY_SWITCH(k_generate2d_staged, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs,
                      d_tile_prefix, nvol, tile_base, bpw)
    } else if (two_d) {
        SN_KEY_SWITCH(k_generate2d, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs, d_tile_prefix,
                      nvol, tile_base, bpw)
    } else if (staged) {
        SN_KEY_SWITCH(k_generate_staged, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs,
                      d_tile_prefix, nvol, tile_base, bpw)
    } else {
        SN_KEY_SWITCH(k_generate, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs, d_tile_prefix,
                      nvol, tile_base, bpw)
    }
    return hipGetLastError();
}

hipError_t launch_generate_one(const VolDesc &d, bool staged, int64_t ntiles, int32_t bpw, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const int32_t dtype = d.dtype, mode = d.cs.mode;
    if (d.prim == kPrimLines && staged) {
        SN_KEY_SWITCH(k_generate2d_staged_one, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, OneVol{d}, bpw)
    } else if (d.prim == kPrimLines) {
        SN_KEY_SWITCH(k_generate2d_one, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, OneVol{d}, bpw)
    } else if (staged) {
        SN_KEY_SWITCH(k_generate_staged_one, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, OneVol{d}, bpw)
    } else {
        SN_KEY_SWITCH(k_generate_one, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, OneVol{d}, bpw)
    }
    return hipGetLastError();
}

hipError_t launch_emit(const VolDesc *d_descs, const SmoothDesc *d_sds, const int64_t *d_tile_prefix,
                       int32_t nvol, int64_t ntiles, int32_t bpw, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs, d_sds,
                       d_tile_prefix, nvol, bpw);
    return hipGetLastError();
}

hipError_t launch_emit_one(const VolDesc &d, const SmoothDesc &sd, int64_t ntiles, int32_t bpw,
                           hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit_one, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, OneEmit{d, sd}, bpw);
    return hipGetLastError();
}

template <int K>
static void jacobi_k(const SmoothDesc *d_sd, const int64_t *d_block_prefix, int32_t nvol,
                     int64_t nblocks, int32_t it, bool big, hipStream_t s)
{
    if (it == 0)
        hipLaunchKernelGGL(k_jacobi_first<K>, dim3((uint32_t)nblocks), dim3(kSweepBlock), 0, s, d_sd,
                           d_block_prefix, nvol, int64_t(0));
    else if (big)
        hipLaunchKernelGGL((k_jacobi<K, 1>), dim3((uint32_t)nblocks), dim3(kSweepBlock), 0, s, d_sd,
                           d_block_prefix, nvol, it);
    else
        hipLaunchKernelGGL((k_jacobi<K, 0>), dim3((uint32_t)nblocks), dim3(kSweepBlock), 0, s, d_sd,
                           d_block_prefix, nvol, it);
}

template <int K>
static void jacobi_one_k(const SmoothDesc &sd, int64_t nblocks, int32_t it, hipStream_t s)
{
    if (it == 0)
        hipLaunchKernelGGL(k_jacobi_first_one<K>, dim3((uint32_t)nblocks), dim3(kSweepBlock), 0, s,
                           OneSmooth{sd});
    else if (sd.big)
        hipLaunchKernelGGL((k_jacobi_one<K, 1>), dim3((uint32_t)nblocks), dim3(kSweepBlock), 0, s,
                           OneSmooth{sd}, it);
    else
        hipLaunchKernelGGL((k_jacobi_one<K, 0>), dim3((uint32_t)nblocks), dim3(kSweepBlock), 0, s,
                           OneSmooth{sd}, it);
}

hipError_t launch_jacobi(const SmoothDesc *d_sd, const int64_t *d_block_prefix, int32_t nvol,
                         int64_t nblocks, int32_t it, int K, bool big, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (K == 1)
        jacobi_k<1>(d_sd, d_block_prefix, nvol, nblocks, it, big, s);
    else
        jacobi_k<2>(d_sd, d_block_prefix, nvol, nblocks, it, big, s);
    return hipGetLastError();
}

hipError_t launch_jacobi_first2_one(const SmoothDesc &sd, int64_t nblocks, int K, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (K == 1)
        hipLaunchKernelGGL(k_jacobi_first2_one<1>, dim3((uint32_t)nblocks), dim3(kSweepBlock), 0, s,
                           OneSmooth{sd});
    else
        hipLaunchKernelGGL(k_jacobi_first2_one<2>, dim3((uint32_t)nblocks), dim3(kSweepBlock), 0, s,
                           OneSmooth{sd});
    return hipGetLastError();
}

hipError_t launch_jacobi_one(const SmoothDesc &sd, int64_t nblocks, int32_t it, int K, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (K == 1)
        jacobi_one_k<1>(sd, nblocks, it, s);
    else
        jacobi_one_k<2>(sd, nblocks, it, s);
    return hipGetLastError();
}

template <int K>
static void jacobi_first2_k(const SmoothDesc *d_sd, const int64_t *d_block_prefix, int32_t nvol,
                            int64_t grid0, int64_t grid1, hipStream_t s)
{
    hipLaunchKernelGGL(k_jacobi_first2<K>, dim3((uint32_t)grid1), dim3(kSweepBlock), 0, s, d_sd,
                       d_block_prefix, nvol);
    if (grid0 > grid1)
        hipLaunchKernelGGL(k_jacobi_first<K>, dim3((uint32_t)(grid0 - grid1)), dim3(kSweepBlock), 0, s,
                           d_sd, d_block_prefix, nvol, grid1);
}

hipError_t launch_jacobi_first2(const SmoothDesc *d_sd, const int64_t *d_block_prefix, int32_t nvol,
                                int64_t grid0, int64_t grid1, int K, hipStream_t s)
{
    if (grid1 <= 0) return hipErrorInvalidValue;
    if (K == 1)
        jacobi_first2_k<1>(d_sd, d_block_prefix, nvol, grid0, grid1, s);
    else
        jacobi_first2_k<2>(d_sd, d_block_prefix, nvol, grid0, grid1, s);
    return hipGetLastError();
}

// Kernel nodes of n sweeps over many meshes, each depending on the one before:
// sweeps 0 and 1 fused over the meshes of at least two sweeps (the leading
// grid[1] blocks) and sweep 0 alone over the rest, then sweeps 2 ...
hipError_t add_jacobi_nodes(hipGraph_t graph, const SmoothDesc *d_sd,
                            const int64_t *d_block_prefix, int32_t nvol, const int64_t *grid,
                            int32_t iters, int K, bool big)
{
    hipGraphNode_t prev = nullptr;
    auto add = [&](void *func, int64_t nblocks, void **args) -> hipError_t {
        hipKernelNodeParams kp{};
        kp.func = func;
        kp.gridDim = dim3((uint32_t)nblocks);
        kp.blockDim = dim3(kSweepBlock);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        const hipError_t e =
            hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (e == hipSuccess) prev = node;
        return e;
    };
    auto first = [K]() {
        return K == 1 ? reinterpret_cast<void *>(&k_jacobi_first<1>) : reinterpret_cast<void *>(&k_jacobi_first<2>);
    };
    int32_t it = 0;
    if (iters >= 2 && grid[1] > 0) {
        void *args_f2[] = {&d_sd, &d_block_prefix, &nvol};
        hipError_t e = add(K == 1 ? reinterpret_cast<void *>(&k_jacobi_first2<1>)
                                  : reinterpret_cast<void *>(&k_jacobi_first2<2>),
                           grid[1], args_f2);
        if (e != hipSuccess) return e;
        if (grid[0] > grid[1]) {
            int64_t block0 = grid[1];
            void *args_first[] = {&d_sd, &d_block_prefix, &nvol, &block0};
            e = add(first(), grid[0] - grid[1], args_first);
            if (e != hipSuccess) return e;
        }
        it = 2;
    }
    for (; it < iters && grid[it] > 0; ++it) {
        int64_t block0 = 0;
        void *args_first[] = {&d_sd, &d_block_prefix, &nvol, &block0};
        void *args[] = {&d_sd, &d_block_prefix, &nvol, &it};
        void *sweep = K == 1 ? (big ? reinterpret_cast<void *>(&k_jacobi<1, 1>)
                                    : reinterpret_cast<void *>(&k_jacobi<1, 0>))
                             : (big ? reinterpret_cast<void *>(&k_jacobi<2, 1>)
                                    : reinterpret_cast<void *>(&k_jacobi<2, 0>));
        const hipError_t e = it == 0 ? add(first(), grid[it], args_first) : add(sweep, grid[it], args);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}


// Descriptor staging: a copy of `n` 8-byte words from host-mapped pinned
// memory into device memory by the queue that runs the kernels, so that the
// kernel after it waits on no other engine.
__global__ __launch_bounds__(256) void k_stage(const uint64_t *__restrict__ src,
                                               uint64_t *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        glb(dst)[i] = src[i];
}

hipError_t launch_stage(void *dst, const void *src_mapped, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)((bytes + 7) / 8);
    if (n <= 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64);
    hipLaunchKernelGGL(k_stage, dim3(blocks), dim3(256), 0, s, static_cast<const uint64_t *>(src_mapped),
                       static_cast<uint64_t *>(dst), n);
    return hipGetLastError();
}

hipError_t launch_triangulate(const VolDesc *d_descs, const int64_t *d_block_prefix, int32_t nvol,
                              int64_t nblocks, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri, dim3((uint32_t)nblocks), dim3(256), 0, s, d_descs, d_block_prefix,
                       nvol);
    return hipGetLastError();
}

hipError_t launch_triangulate_one(const VolDesc &d, hipStream_t s)
{
    const int64_t nblocks = (d.Q + 255) / 256;
    if (nblocks <= 0 || d.prim != 3) return hipSuccess;
    hipLaunchKernelGGL(k_tri_one, dim3((uint32_t)nblocks), dim3(256), 0, s, OneVol{d});
    return hipGetLastError();
}

}  // namespace sn
