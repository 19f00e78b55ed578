// The no-allocation extraction of libsn.so (sn_extract_noalloc): the passes
// of sn_extract (Sec. 2.3: classification and intersected edges, counting,
// prefix sum, generation) with every output in caller-owned arrays and all
// scratch (cut-edge planes, word metadata, scan status, totals and the
// classification table) in one static device array per GPU, so that the call
// makes no device allocation.  For callers that cannot allocate: tight
// serving loops, harnesses that forbid hipMalloc, processes that must not grow
// their device memory after set-up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sn.h"
#include "sn_internal.h"
#include "sn_runtime.h"

using namespace sn;

namespace {

// The scratch of every sn_extract_noalloc call on a GPU.  In host code the
// name stands for a host-side handle only: kernels get the device address
// resolved by noalloc_resolve, never the name.
constexpr size_t kScratchBytes = size_t(SN_NOALLOC_SCRATCH_BYTES);
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

size_t up256(size_t n) { return (n + 255) & ~size_t(255); }

// Carve of the scratch for one volume.  The scan status, the tile ticket and
// the totals come first: k_edges zeroes them (nzero words) before k_count
// reads them, so nothing of an earlier call survives there.
struct NoAllocLayout {
    size_t o_status, status_bytes, o_ticket, o_tot, nzero_bytes;
    size_t o_tab, o_planes, o_pmask, o_wbP, o_wbQ, o_wbS, bytes;
};

NoAllocLayout layout(const Geom &g, int64_t nctiles, size_t tab_words)
{
    NoAllocLayout l{};
    const int64_t words = std::max<int64_t>(g.R * g.W, 1);
    l.o_status = 0;
    l.status_bytes = 24 * (size_t)std::max<int64_t>(nctiles, 1);
    l.o_ticket = l.status_bytes;        // one uint32 ticket (256 bytes kept)
    l.o_tot = l.status_bytes + 256;     // totals (P, Q, S) and the stamp
    l.nzero_bytes = l.o_tot + 4 * 8;
    size_t at = up256(l.nzero_bytes);
    l.o_tab = at, at += up256(4 * std::max<size_t>(tab_words, 1));
    l.o_planes = at, at += up256(8 * (size_t)std::max<int64_t>(3 * g.N * g.O * g.WS, 1));
    l.o_pmask = at, at += up256(8 * (size_t)words);
    l.o_wbP = at, at += up256(4 * (size_t)words);
    l.o_wbQ = at, at += up256(4 * (size_t)words);
    l.o_wbS = at, at += up256(4 * (size_t)words);
    l.bytes = at;
    return l;
}

}  // namespace

sn_status sn::noalloc_resolve(int device, void **addr)
{
    if (device < 0 || device >= kMaxDevices) return fail(SN_EDEVICE, "noalloc: device index too large");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_addr[device]) {
        // the device is current (sn_ctx_create set it)
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(SN_EDEVICE, std::string("noalloc: hipGetSymbolAddress of the scratch array: ") +
                                        hipGetErrorString(e));
        }
        g_addr[device] = p;
    }
    *addr = g_addr[device];
    return SN_OK;
}

extern "C" int64_t sn_noalloc_scratch_bytes(const sn_volume *vol)
{
    if (!vol || validate_volume(vol) != SN_OK) return -1;
    const Geom g = make_geom(*vol);
    // narrow count tiles (one word per thread) are the most: an upper bound
    const int64_t nct = (g.R * g.W + kCountBlock - 1) / kCountBlock;
    int32_t mode = 0;
    std::vector<uint32_t> tab;
    class_table(*vol, &mode, &tab);
    return (int64_t)layout(g, nct, tab.size()).bytes;
}

extern "C" sn_status sn_extract_noalloc(sn_ctx *c, const sn_volume *vol, void *stream,
                                        const sn_extract_arrays *out, int64_t *counts)
{
    if (!c || !vol || !out || !counts) return fail(SN_EINVAL, "sn_extract_noalloc: NULL argument");
    sn_status st = validate_volume(vol);
    if (st != SN_OK) return st;
    if (vol->prim == SN_TRIS)
        return fail(SN_EINVAL, "sn_extract_noalloc: SN_TRIS is not supported (use SN_QUADS and "
                               "triangulate the caller's quads)");
    if (out->cap_points < 0 || out->cap_polys < 0 || out->cap_stencil < 0 || !out->stencil_off)
        return fail(SN_EINVAL, "sn_extract_noalloc: bad output arrays");
    if (!c->noalloc_scratch) return fail(SN_EDEVICE, "sn_extract_noalloc: scratch not resolved");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);

    VolDesc d;
    std::memset(&d, 0, sizeof d);
    d.labels = vol->labels;
    d.dtype = vol->dtype;
    d.prim = vol->prim;
    d.g = make_geom(*vol);
    for (int a = 0; a < 3; ++a) d.origin[a] = vol->origin[a], d.spacing[a] = vol->spacing[a];
    if (vol->prim == SN_LINES) d.spacing[2] = 0.0;  // an image's points lie in z = origin[2]
    std::vector<uint32_t> tab;
    int32_t mode = 0;
    class_table(*vol, &mode, &tab);
    d.cs.mode = mode;
    d.cs.bg = vol->background;
    d.cs.n = (int32_t)tab.size();

    const int64_t words = d.g.R * d.g.W;
    const Schedule sc = c->schedule(size_class(*vol));
    const int32_t cv = sc.count_words > 0 ? sc.count_words : (words >= c->count_wide_words ? kCountWideV : 1);
    const int64_t nctiles = (words + cv * kCountBlock - 1) / (cv * kCountBlock);
    const NoAllocLayout l = layout(d.g, nctiles, tab.size());
    if (l.bytes > kScratchBytes)
        return fail(SN_ETOOBIG, "sn_extract_noalloc: the volume needs " + std::to_string(l.bytes) +
                                    " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                                    " of the static array");
    uint8_t *base = static_cast<uint8_t *>(c->noalloc_scratch);
    uint64_t *status = reinterpret_cast<uint64_t *>(base + l.o_status);
    uint32_t *ticket = reinterpret_cast<uint32_t *>(base + l.o_ticket);
    int64_t *d_tot = reinterpret_cast<int64_t *>(base + l.o_tot);
    d.planes = reinterpret_cast<uint64_t *>(base + l.o_planes);
    d.pmask = reinterpret_cast<uint64_t *>(base + l.o_pmask);
    d.wbP = reinterpret_cast<int32_t *>(base + l.o_wbP);
    d.wbQ = reinterpret_cast<int32_t *>(base + l.o_wbQ);
    d.wbS = reinterpret_cast<int32_t *>(base + l.o_wbS);
    if (!tab.empty()) {
        d.cs.table = reinterpret_cast<const uint32_t *>(base + l.o_tab);
        // `tab` outlives the copy: the call waits on the stream below
        HIP_TRY(hipMemcpyAsync(base + l.o_tab, tab.data(), 4 * tab.size(), hipMemcpyHostToDevice, s));
    }

    int64_t tot[4] = {0, 0, 0, 0};
    const bool wide = vol->dims[0] % 4 == 0 && (reinterpret_cast<uintptr_t>(vol->labels) & 15) == 0;
    const int64_t nseg = edge_segments(d.g);
    const int64_t etiles = edge_tiles(nseg, sc.edge_segs);
    if (nctiles > 0) {
        {
            ProfScope ps(c, "k_edges", s);
            HIP_TRY(launch_edges_one(d, wide, etiles, status, (int64_t)(l.nzero_bytes / 8), sc.edge_segs, s));
        }
        static std::atomic<int64_t> g_seq{0};
        const int64_t seq = g_seq.fetch_add(1, std::memory_order_relaxed) + 1;
        {
            ProfScope ps(c, "k_count", s);
            HIP_TRY(launch_count_one(d, nctiles, cv, status, ticket, CountOut{d_tot, d_tot + 3, seq}, s));
        }
        HIP_TRY(hipMemcpyAsync(tot, d_tot, sizeof tot, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (tot[3] != seq) return fail(SN_EDEVICE, "sn_extract_noalloc: the count pass left no totals");
    } else if (!tab.empty()) {
        HIP_TRY(hipStreamSynchronize(s));
    }
    const int64_t P = tot[0], Q = tot[1], S = tot[2];
    if (P >= INT32_MAX || Q >= INT32_MAX / 2 || S >= INT32_MAX)
        return fail(SN_ETOOBIG, "sn_extract_noalloc: mesh indices exceed int32");
    counts[0] = P, counts[1] = Q, counts[2] = S;
    if (P > out->cap_points || Q > out->cap_polys || S > out->cap_stencil ||
        (P > 0 && !out->points) || (Q > 0 && (!out->polys || !out->label_pairs)) ||
        (S > 0 && !out->stencil_ids))
        return fail(SN_ENOMEM, "sn_extract_noalloc: output arrays too small for (" + std::to_string(P) +
                                   ", " + std::to_string(Q) + ", " + std::to_string(S) + ")");
    d.P = P, d.Q = Q, d.S = S;
    d.points = out->points;
    d.st_off = out->stencil_off;
    d.st_ids = out->stencil_ids;
    d.quads = out->polys;
    d.pairs = out->label_pairs;
    // no smoothing state: no face bytes, no cell index per point
    d.faces = nullptr;
    d.pcell = nullptr;
    const int32_t bpw = sc.gen_groups;
    const int64_t TB = kWavesPerBlock * bpw;
    const int64_t ngroups = (words + kGenWords - 1) / kGenWords;
    // at least one tile: the first writes stencil_off[P] = S
    const int64_t gtiles = std::max<int64_t>(1, (ngroups + TB - 1) / TB);
    const bool staged = P >= kGenStagedPointsPerWord * words;
    {
        ProfScope ps(c, "k_generate", s);
        HIP_TRY(launch_generate_one(d, staged, gtiles, bpw, s));
    }
    return SN_OK;
}
