// SurfaceNets extraction and smoothing kernels for gfx950 (MI355X).
//
// Row kernels: one 64-lane wavefront walks one row of cells (fixed j, k) in
// 64-cell words; lane L of word w owns cell i = 64w + L and the sample (i,j,k).
// The four sample rows (j..j+1, k..k+1) around the cell row are read once per
// word; the +x corner comes from the next lane (cross-lane shuffle).  Every
// per-cell predicate becomes a 64-bit ballot, so in-row ranks of points,
// quads and stencil entries are mbcnt popcounts and row totals are scalar
// popcounts.  This replaces the paper's triad byte volume, trim intervals,
// checkerboarded PRODUCE_POINT bits and 3x3 row iterator (Sec. 3.2-3.6) with
// a 1-bit-per-cell point plane and per-row prefix bases.
//
//   k_count    : classify + cut edges + point/quad/stencil counts per row,
//                point-bit plane, fused decoupled-look-back exclusive scan of
//                the per-row counts (Sec. 2.3 passes 1-3 and the prefix sum).
//   k_generate : points, stencil CSR, quads and label pairs at the scanned
//                offsets, no atomics (Sec. 2.3 pass 4).
//   k_jacobi   : one double-buffered sweep of Eq. (1) with the box
//                constraint (Sec. 2.2, 2.4), on cell-relative offsets.
//   k_emit     : world coordinates of the points from the offsets.
//   k_tri      : two triangles per quad (Sec. 2.5).
#include "sn_internal.h"

namespace sn {

__device__ __forceinline__ uint32_t rank_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p ? 1 : 0); }

__device__ __forceinline__ int find_seg(const int64_t *prefix, int n, int64_t t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int MODE>
__device__ __forceinline__ uint32_t classify(uint32_t v, const ClassSpec &cs)
{
    if constexpr (MODE == CLS_IDENT) {
        return v;
    } else if constexpr (MODE == CLS_BITMAP) {
        return ((cs.table[v >> 5] >> (v & 31u)) & 1u) ? v : cs.bg;
    } else {
        int lo = 0, hi = cs.n;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (cs.table[mid] < v)
                lo = mid + 1;
            else
                hi = mid;
        }
        return (lo < cs.n && cs.table[lo] == v) ? v : cs.bg;
    }
}

// Classified values at the 8 corners of cell (i,j,k); index di + 2*dj + 4*dk.
template <typename T, int MODE>
__device__ __forceinline__ void load_corners(const T *__restrict__ vol, const Geom &g,
                                             const ClassSpec &cs, int64_t i, int64_t j, int64_t k,
                                             int lane, uint32_t c[8])
{
    const int64_t ic = i < g.M - 1 ? i : g.M - 1;
    const int64_t in = (i + 1) < g.M - 1 ? (i + 1) : g.M - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int dj = q & 1, dk = q >> 1;
        const T *row = vol + g.M * ((j + dj) + g.N * (k + dk));
        uint32_t a = classify<MODE>((uint32_t)row[ic], cs);
        uint32_t b = __shfl_down(a, 1u);
        if (lane == 63) b = classify<MODE>((uint32_t)row[in], cs);
        c[2 * dj + 4 * dk] = a;
        c[1 + 2 * dj + 4 * dk] = b;
    }
}

struct CellPred {
    bool point, qx, qy, qz;
    uint32_t fmask;
};

__device__ __forceinline__ bool nonuni4(uint32_t a, uint32_t b, uint32_t d, uint32_t e)
{
    return !((a == b) & (a == d) & (a == e));
}

// Sec. 2.2 / 3.3 predicates of one cell and of the edges owned by its origin sample.
__device__ __forceinline__ CellPred predicates(const uint32_t c[8], bool valid, int64_t i, int64_t j,
                                               int64_t k, const Geom &g)
{
    CellPred p;
    const uint32_t c000 = c[0], c100 = c[1], c010 = c[2], c110 = c[3];
    const uint32_t c001 = c[4], c101 = c[5], c011 = c[6], c111 = c[7];
    const bool all_eq = (c000 == c100) & (c000 == c010) & (c000 == c110) & (c000 == c001) &
                        (c000 == c101) & (c000 == c011) & (c000 == c111);
    p.point = valid && !all_eq;
    uint32_t fm = 0;
    fm |= (i >= 1 && nonuni4(c000, c010, c001, c011)) ? 1u : 0u;
    fm |= (i + 1 <= g.CM - 1 && nonuni4(c100, c110, c101, c111)) ? 2u : 0u;
    fm |= (j >= 1 && nonuni4(c000, c100, c001, c101)) ? 4u : 0u;
    fm |= (j + 1 <= g.CN - 1 && nonuni4(c010, c110, c011, c111)) ? 8u : 0u;
    fm |= (k >= 1 && nonuni4(c000, c100, c010, c110)) ? 16u : 0u;
    fm |= (k + 1 <= g.CO - 1 && nonuni4(c001, c101, c011, c111)) ? 32u : 0u;
    p.fmask = valid ? fm : 0u;
    p.qx = valid && (c000 != c100) && j >= 1 && k >= 1;
    p.qy = valid && (c000 != c010) && i >= 1 && k >= 1;
    p.qz = valid && (c000 != c001) && i >= 1 && j >= 1;
    return p;
}

// ---------------------------------------------------------------------------
// k_count
// ---------------------------------------------------------------------------

template <typename T, int MODE>
__device__ void count_row(const VolDesc &d, int64_t r, int lane, int64_t cnt[3])
{
    const Geom &g = d.g;
    const T *vol = static_cast<const T *>(d.labels);
    const int64_t j = r % g.CN, k = r / g.CN;
    int64_t nP = 0, nQ = 0, nS = 0;
    for (int32_t w = 0; w < g.W; ++w) {
        const int64_t i = 64 * (int64_t)w + lane;
        const bool valid = i < g.CM;
        uint32_t c[8];
        load_corners<T, MODE>(vol, g, d.cs, i, j, k, lane, c);
        const CellPred p = predicates(c, valid, i, j, k, g);
        const uint64_t bp = wave_ballot(p.point);
        if (lane == 0) d.pmask[r * g.W + w] = bp;
        nP += __popcll(bp);
        nQ += __popcll(wave_ballot(p.qx)) + __popcll(wave_ballot(p.qy)) +
              __popcll(wave_ballot(p.qz));
#pragma unroll
        for (int f = 0; f < 6; ++f) nS += __popcll(wave_ballot((p.fmask >> f) & 1u));
    }
    cnt[0] = nP, cnt[1] = nQ, cnt[2] = nS;
}

__device__ void count_row_dispatch(const VolDesc &d, int64_t r, int lane, int64_t cnt[3])
{
    const int m = d.cs.mode;
    if (d.dtype == 1) {
        if (m == CLS_IDENT) count_row<uint8_t, CLS_IDENT>(d, r, lane, cnt);
        else count_row<uint8_t, CLS_BITMAP>(d, r, lane, cnt);
    } else if (d.dtype == 2) {
        if (m == CLS_IDENT) count_row<uint16_t, CLS_IDENT>(d, r, lane, cnt);
        else count_row<uint16_t, CLS_BITMAP>(d, r, lane, cnt);
    } else {
        if (m == CLS_IDENT) count_row<uint32_t, CLS_IDENT>(d, r, lane, cnt);
        else count_row<uint32_t, CLS_SORTED>(d, r, lane, cnt);
    }
}

__global__ __launch_bounds__(kBlock) void k_count(const VolDesc *__restrict__ descs,
                                                  const int64_t *__restrict__ tile_prefix,
                                                  int32_t nvol, int32_t rpw, uint64_t *status,
                                                  uint32_t *ticket, int64_t *totals)
{
    __shared__ int64_t s_tile;
    __shared__ int64_t s_cnt[3][kWavesPerBlock * kMaxRowsPerWave];
    __shared__ int64_t s_excl[3];
    if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t t = s_tile;  // tiles are taken in launch order: predecessors are running
    const int v = find_seg(tile_prefix, nvol, t);
    const VolDesc &d = descs[v];
    const int TR = kWavesPerBlock * rpw;
    const int64_t r0 = (t - tile_prefix[v]) * TR;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = 0; q < rpw; ++q) {
        const int lr = wave + kWavesPerBlock * q;
        const int64_t r = r0 + lr;
        int64_t cnt[3] = {0, 0, 0};
        if (r < d.g.R) count_row_dispatch(d, r, lane, cnt);
        if (lane == 0) {
            s_cnt[0][lr] = cnt[0];
            s_cnt[1][lr] = cnt[1];
            s_cnt[2][lr] = cnt[2];
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        // single-pass scan with decoupled look-back, one lane per component
        const int comp = threadIdx.x;
        int64_t agg = 0;
        for (int lr = 0; lr < TR; ++lr) agg += s_cnt[comp][lr];
        uint64_t *mine = status + 3 * t + comp;
        int64_t excl = 0;
        if (t == tile_prefix[v]) {
            __hip_atomic_store(mine, kFlagPrefix | (uint64_t)agg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(mine, kFlagAgg | (uint64_t)agg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            int64_t p = t - 1;
            while (true) {
                const uint64_t s = __hip_atomic_load(status + 3 * p + comp, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t flag = s & ~kValMask;
                if (flag == 0) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += (int64_t)(s & kValMask);
                if (flag == kFlagPrefix) break;
                --p;
            }
            __hip_atomic_store(mine, kFlagPrefix | (uint64_t)(excl + agg), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_excl[comp] = excl;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int comp = threadIdx.x;
        int64_t *base = comp == 0 ? d.baseP : (comp == 1 ? d.baseQ : d.baseS);
        int64_t run = s_excl[comp];
        for (int lr = 0; lr < TR; ++lr) {
            const int64_t r = r0 + lr;
            if (r >= d.g.R) break;
            base[r] = run;
            run += s_cnt[comp][lr];
        }
        if (t == tile_prefix[v + 1] - 1) {
            base[d.g.R] = run;
            totals[3 * v + comp] = run;
        }
    }
}

// ---------------------------------------------------------------------------
// k_generate
// ---------------------------------------------------------------------------

template <typename T, int MODE>
__device__ void generate_row(const VolDesc &d, int64_t r, int lane)
{
    const Geom &g = d.g;
    const T *vol = static_cast<const T *>(d.labels);
    T *pairs = static_cast<T *>(d.pairs);
    const int64_t j = r % g.CN, k = r / g.CN;
    const int32_t W = g.W;
    const bool ym = j >= 1, yp = j + 1 <= g.CN - 1, zm = k >= 1, zp = k + 1 <= g.CO - 1;
    // running bases: point id of the next point in each of the six rows used
    int64_t b0 = d.baseP[r];
    int64_t bym = ym ? d.baseP[r - 1] : 0, byp = yp ? d.baseP[r + 1] : 0;
    int64_t bzm = zm ? d.baseP[r - g.CN] : 0, bzp = zp ? d.baseP[r + g.CN] : 0;
    int64_t bmm = (ym && zm) ? d.baseP[r - g.CN - 1] : 0;
    int64_t bq = d.baseQ[r], bs = d.baseS[r];
    const uint64_t *wym = d.pmask + (r - 1) * W, *wyp = d.pmask + (r + 1) * W;
    const uint64_t *wzm = d.pmask + (r - g.CN) * W, *wzp = d.pmask + (r + g.CN) * W;
    const uint64_t *wmm = d.pmask + (r - g.CN - 1) * W;
    const double ox = d.origin[0], oy = d.origin[1], oz = d.origin[2];
    const double hx = d.spacing[0], hy = d.spacing[1], hz = d.spacing[2];
    const float py = (float)(oy + hy * ((double)j + 0.5));
    const float pz = (float)(oz + hz * ((double)k + 0.5));
    for (int32_t w = 0; w < W; ++w) {
        const int64_t i = 64 * (int64_t)w + lane;
        const bool valid = i < g.CM;
        uint32_t c[8];
        load_corners<T, MODE>(vol, g, d.cs, i, j, k, lane, c);
        const CellPred p = predicates(c, valid, i, j, k, g);
        const uint64_t bp = wave_ballot(p.point);
        const uint64_t mym = ym ? wym[w] : 0ull, myp = yp ? wyp[w] : 0ull;
        const uint64_t mzm = zm ? wzm[w] : 0ull, mzp = zp ? wzp[w] : 0ull;
        const uint64_t mmm = (ym && zm) ? wmm[w] : 0ull;
        const int64_t R0 = b0 + rank_below(bp);
        const int64_t Rym = bym + rank_below(mym), Ryp = byp + rank_below(myp);
        const int64_t Rzm = bzm + rank_below(mzm), Rzp = bzp + rank_below(mzp);
        const int64_t Rmm = bmm + rank_below(mmm);
        uint64_t fb[6];
        uint32_t sp = 0;
        int64_t stot = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            fb[f] = wave_ballot((p.fmask >> f) & 1u);
            sp += rank_below(fb[f]);
            stot += __popcll(fb[f]);
        }
        const uint64_t bqx = wave_ballot(p.qx), bqy = wave_ballot(p.qy), bqz = wave_ballot(p.qz);
        if (p.point) {
            const int64_t id = R0;
            float *pt = d.points + 3 * id;
            pt[0] = (float)(ox + hx * ((double)i + 0.5));
            pt[1] = py;
            pt[2] = pz;
            d.faces[id] = (uint8_t)p.fmask;
            int64_t s = bs + sp;
            d.st_off[id] = (int32_t)s;
            int32_t *ids = d.st_ids;
            if (p.fmask & 1u) ids[s++] = (int32_t)(R0 - 1);
            if (p.fmask & 2u) ids[s++] = (int32_t)(R0 + 1);
            if (p.fmask & 4u) ids[s++] = (int32_t)Rym;
            if (p.fmask & 8u) ids[s++] = (int32_t)Ryp;
            if (p.fmask & 16u) ids[s++] = (int32_t)Rzm;
            if (p.fmask & 32u) ids[s++] = (int32_t)Rzp;
        }
        int64_t q = bq + rank_below(bqx) + rank_below(bqy) + rank_below(bqz);
        if (p.qx) {
            int32_t *o = d.quads + 4 * q;
            o[0] = (int32_t)Rmm, o[1] = (int32_t)Rym, o[2] = (int32_t)R0, o[3] = (int32_t)Rzm;
            pairs[2 * q] = (T)c[0], pairs[2 * q + 1] = (T)c[1];
            ++q;
        }
        if (p.qy) {
            int32_t *o = d.quads + 4 * q;
            o[0] = (int32_t)(Rzm - 1), o[1] = (int32_t)Rzm, o[2] = (int32_t)R0,
            o[3] = (int32_t)(R0 - 1);
            pairs[2 * q] = (T)c[0], pairs[2 * q + 1] = (T)c[2];
            ++q;
        }
        if (p.qz) {
            int32_t *o = d.quads + 4 * q;
            o[0] = (int32_t)(Rym - 1), o[1] = (int32_t)(R0 - 1), o[2] = (int32_t)R0,
            o[3] = (int32_t)Rym;
            pairs[2 * q] = (T)c[0], pairs[2 * q + 1] = (T)c[4];
        }
        b0 += __popcll(bp);
        bym += __popcll(mym), byp += __popcll(myp);
        bzm += __popcll(mzm), bzp += __popcll(mzp), bmm += __popcll(mmm);
        bq += __popcll(bqx) + __popcll(bqy) + __popcll(bqz);
        bs += stot;
    }
}

__device__ void generate_row_dispatch(const VolDesc &d, int64_t r, int lane)
{
    const int m = d.cs.mode;
    if (d.dtype == 1) {
        if (m == CLS_IDENT) generate_row<uint8_t, CLS_IDENT>(d, r, lane);
        else generate_row<uint8_t, CLS_BITMAP>(d, r, lane);
    } else if (d.dtype == 2) {
        if (m == CLS_IDENT) generate_row<uint16_t, CLS_IDENT>(d, r, lane);
        else generate_row<uint16_t, CLS_BITMAP>(d, r, lane);
    } else {
        if (m == CLS_IDENT) generate_row<uint32_t, CLS_IDENT>(d, r, lane);
        else generate_row<uint32_t, CLS_SORTED>(d, r, lane);
    }
}

__global__ __launch_bounds__(kBlock) void k_generate(const VolDesc *__restrict__ descs,
                                                     const int64_t *__restrict__ tile_prefix,
                                                     int32_t nvol, int32_t rpw)
{
    const int64_t t = blockIdx.x;
    const int v = find_seg(tile_prefix, nvol, t);
    const VolDesc &d = descs[v];
    const int64_t r0 = (t - tile_prefix[v]) * (kWavesPerBlock * rpw);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0 && t == tile_prefix[v]) d.st_off[d.P] = (int32_t)d.S;
    for (int q = 0; q < rpw; ++q) {
        const int64_t r = r0 + wave + kWavesPerBlock * q;
        if (r < d.g.R) generate_row_dispatch(d, r, lane);
    }
}

// ---------------------------------------------------------------------------
// k_emit: points = origin + spacing * (cell centre + offset)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_emit(const VolDesc *__restrict__ descs,
                                                 const int64_t *__restrict__ tile_prefix,
                                                 int32_t nvol, int32_t rpw)
{
    const int64_t t = blockIdx.x;
    const int v = find_seg(tile_prefix, nvol, t);
    const VolDesc &d = descs[v];
    const Geom &g = d.g;
    const int64_t r0 = (t - tile_prefix[v]) * (kWavesPerBlock * rpw);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float *delta = d.delta;
    for (int q = 0; q < rpw; ++q) {
        const int64_t r = r0 + wave + kWavesPerBlock * q;
        if (r >= g.R) break;
        const int64_t j = r % g.CN, k = r / g.CN;
        int64_t b = d.baseP[r];
        for (int32_t w = 0; w < g.W; ++w) {
            const uint64_t m = d.pmask[r * g.W + w];
            if (m == 0) continue;
            if ((m >> lane) & 1ull) {
                const int64_t id = b + rank_below(m);
                double dx = 0.0, dy = 0.0, dz = 0.0;
                if (delta) {
                    dx = (double)delta[3 * id], dy = (double)delta[3 * id + 1];
                    dz = (double)delta[3 * id + 2];
                }
                const int64_t i = 64 * (int64_t)w + lane;
                float *pt = d.points + 3 * id;
                pt[0] = (float)(d.origin[0] + d.spacing[0] * ((double)i + 0.5 + dx));
                pt[1] = (float)(d.origin[1] + d.spacing[1] * ((double)j + 0.5 + dy));
                pt[2] = (float)(d.origin[2] + d.spacing[2] * ((double)k + 0.5 + dz));
            }
            b += __popcll(m);
        }
    }
}

// ---------------------------------------------------------------------------
// k_jacobi: one sweep of Eq. (1) on the offsets, FP64 arithmetic, FP32 storage
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_jacobi(const SmoothDesc *__restrict__ sds,
                                                const int64_t *__restrict__ block_prefix,
                                                int32_t nvol, int32_t it)
{
    const int64_t b = blockIdx.x;
    const int v = find_seg(block_prefix, nvol, b);
    const SmoothDesc &s = sds[v];
    if (it >= s.iters) return;  // this mesh has finished its sweeps
    const int64_t p = (b - block_prefix[v]) * 256 + threadIdx.x;
    if (p >= s.P) return;
    const float *din = (it & 1) ? s.db : s.da;
    float *dout = (it & 1) ? s.da : s.db;
    const bool zero_in = (it == 0);
    const uint32_t f = s.faces[p];
    double x = 0.0, y = 0.0, z = 0.0;
    if (!zero_in) {
        x = (double)din[3 * p], y = (double)din[3 * p + 1], z = (double)din[3 * p + 2];
    }
    const int n = __popc(f);
    if (n > 0) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        int64_t e = s.off[p];
#pragma unroll
        for (int face = 0; face < 6; ++face) {
            if (!((f >> face) & 1u)) continue;
            const int64_t q = s.ids[e++];
            double nx = 0.0, ny = 0.0, nz = 0.0;
            if (!zero_in) {
                nx = (double)din[3 * q], ny = (double)din[3 * q + 1], nz = (double)din[3 * q + 2];
            }
            // p_q - p_p = unit face step + offset difference
            const double step = (face & 1) ? 1.0 : -1.0;
            sx += (face >> 1) == 0 ? step + nx - x : nx - x;
            sy += (face >> 1) == 1 ? step + ny - y : ny - y;
            sz += (face >> 1) == 2 ? step + nz - z : nz - z;
        }
        const double inv = 1.0 / (double)n;
        x = x + s.lam * (sx * inv);
        y = y + s.lam * (sy * inv);
        z = z + s.lam * (sz * inv);
    }
    const double c = s.dist;
    x = fmin(fmax(x, -c), c);
    y = fmin(fmax(y, -c), c);
    z = fmin(fmax(z, -c), c);
    dout[3 * p] = (float)x;
    dout[3 * p + 1] = (float)y;
    dout[3 * p + 2] = (float)z;
}

// ---------------------------------------------------------------------------
// k_tri: quad (A,B,C,D) -> (A,B,C), (A,C,D)
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void tri_pairs(const VolDesc &d, int64_t q)
{
    const T *src = static_cast<const T *>(d.pairs);
    T *dst = static_cast<T *>(d.tri_pairs);
    const T f = src[2 * q], b = src[2 * q + 1];
    dst[4 * q] = f, dst[4 * q + 1] = b, dst[4 * q + 2] = f, dst[4 * q + 3] = b;
}

__global__ __launch_bounds__(256) void k_tri(const VolDesc *__restrict__ descs,
                                             const int64_t *__restrict__ block_prefix,
                                             int32_t nvol)
{
    const int64_t b = blockIdx.x;
    const int v = find_seg(block_prefix, nvol, b);
    const VolDesc &d = descs[v];
    const int64_t q = (b - block_prefix[v]) * 256 + threadIdx.x;
    if (q >= d.Q || d.prim != 3) return;
    const int32_t *s = d.quads + 4 * q;
    const int32_t A = s[0], B = s[1], C = s[2], D = s[3];
    int32_t *o = d.tris + 6 * q;
    o[0] = A, o[1] = B, o[2] = C, o[3] = A, o[4] = C, o[5] = D;
    if (d.dtype == 1) tri_pairs<uint8_t>(d, q);
    else if (d.dtype == 2) tri_pairs<uint16_t>(d, q);
    else tri_pairs<uint32_t>(d, q);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_count(const VolDesc *d_descs, const int64_t *d_tile_prefix, int32_t nvol,
                        int64_t ntiles, int32_t rpw, uint64_t *d_status, uint32_t *d_ticket,
                        int64_t *d_totals, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs,
                       d_tile_prefix, nvol, rpw, d_status, d_ticket, d_totals);
    return hipGetLastError();
}

hipError_t launch_generate(const VolDesc *d_descs, const int64_t *d_tile_prefix, int32_t nvol,
                           int64_t ntiles, int32_t rpw, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_generate, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs,
                       d_tile_prefix, nvol, rpw);
    return hipGetLastError();
}

hipError_t launch_emit(const VolDesc *d_descs, const int64_t *d_tile_prefix, int32_t nvol,
                       int64_t ntiles, int32_t rpw, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit, dim3((uint32_t)ntiles), dim3(kBlock), 0, s, d_descs, d_tile_prefix,
                       nvol, rpw);
    return hipGetLastError();
}

hipError_t launch_jacobi(const SmoothDesc *d_sd, const int64_t *d_block_prefix, int32_t nvol,
                         int64_t nblocks, int32_t it, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jacobi, dim3((uint32_t)nblocks), dim3(256), 0, s, d_sd, d_block_prefix,
                       nvol, it);
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

}  // namespace sn
