// Host-side internals of libsn.so shared by sn_runtime.hip and sn_serve.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sn.h"
#include "sn_internal.h"

namespace sn {

sn_status fail(sn_status s, const std::string &msg);

// Size class of a pool block: 512-byte steps up to 1 MiB, 2 MiB steps above.
size_t round_size(size_t n);

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return ::sn::fail(SN_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// Recycled HIP events of one kind (timing or not).
class EventCache {
  public:
    explicit EventCache(unsigned flags) : flags_(flags) {}
    ~EventCache();
    hipEvent_t get();  // nullptr on failure
    void put(hipEvent_t e);

  private:
    unsigned flags_;
    std::mutex mu_;
    std::vector<hipEvent_t> free_;
};

class Pool;

// A completion event of the pool's cache that the meshes of one batch share
// (one marker on the stream instead of one per mesh); it goes back to the
// pool's cache when its last holder lets go.
struct SharedEvent {
    SharedEvent(hipEvent_t e, Pool *p) : ev(e), home(p) {}
    ~SharedEvent();
    SharedEvent(const SharedEvent &) = delete;
    SharedEvent &operator=(const SharedEvent &) = delete;
    hipEvent_t ev;
    Pool *home;
};
using EventRef = std::shared_ptr<SharedEvent>;

class Pool {
  public:
    static inline const hipStream_t kNoWait = reinterpret_cast<hipStream_t>(~uintptr_t(0));
    Pool(int device, bool pinned);
    ~Pool();
    // nullptr on failure (or over the test limit).  A cached block handed out
    // may be larger than asked for; in_use() and peak() count what was asked
    // for, rounded to the pool's size classes (round_size), so they do not
    // depend on the state of the cache.
    void *alloc(size_t bytes);
    // Return a block; with a stream, it is reused only after the stream's
    // current work has completed.
    void release(void *p, hipStream_t after);
    void release_all(const std::vector<void *> &ps, hipStream_t after);
    // As release_all, reused once `ev` has completed (the pending release
    // holds a reference to it until then).
    void release_all_after(const std::vector<void *> &ps, EventRef ev);
    // An event (timing disabled) of the pool's cache; nullptr on failure.
    EventRef shared_event();
    void put_event(hipEvent_t e) { events_.put(e); }
    int64_t in_use() const;
    int64_t peak() const;

  private:
    struct Pending {
        hipEvent_t ev;
        std::vector<void *> blocks;
        EventRef ref;  // set: ev is ref's (returned by dropping ref)
    };
    void reclaim_locked(bool wait);
    void raw_free(void *p);
    bool pinned_;
    mutable std::mutex mu_;
    std::multimap<size_t, void *> free_;
    std::map<void *, size_t> sizes_;    // block sizes
    std::map<void *, size_t> charged_;  // live blocks: bytes counted in in_use_
    std::deque<Pending> pending_;  // in release order
    EventCache events_{hipEventDisableTiming};
    int64_t in_use_ = 0, peak_ = 0, limit_ = -1;
};

}  // namespace sn

struct sn_ctx {
    explicit sn_ctx(int dev);
    ~sn_ctx();
    int device;
    // one reference for the caller's handle and one per live mesh or server
    std::atomic<int64_t> refs{1};
    sn::Pool pool;    // device blocks
    sn::Pool pinned;  // pinned host staging
    hipStream_t copy_stream = nullptr;  // non-blocking, for copies to the host
    sn::EventCache timing_events{hipEventDefault};
    sn::EventCache sync_events{hipEventDisableTiming};  // ordering only (served requests)
    // profiling
    bool profiling = false;
    bool profile_eager = false;        // every sweep bracketed by its own events
    bool profile_sweeps_only = false;  // only the sweeps are bracketed
    struct ProfEv {
        std::string name;
        hipEvent_t a, b;
        int64_t launches;
    };
    std::mutex prof_mu;
    std::vector<ProfEv> prof_pending;
    std::map<std::string, std::pair<int64_t, double>> prof_stats;
    // schedule table: size class -> schedule (sn_autotune, SN_AUTOTUNE_CACHE,
    // sn_schedule_set); forced_bpw overrides every class's gen_groups
    mutable std::mutex tune_mu;
    std::map<std::string, sn::Schedule> tune;
    std::string tune_path;
    int32_t forced_bpw = 0;
    int64_t count_wide_words = sn::kCountWideWords;  // SN_TEST_COUNT_WIDE_WORDS overrides
    // meshes of more than this many points take the large-mesh sweep form
    // (SN_TEST_SWEEP_SMALL_POINTS overrides); sweep_chunk > 0 replaces the
    // slab-chunk size of that form's block order (SN_TEST_SWEEP_CHUNK)
    int64_t sweep_small_points = sn::kSweepSmallPoints;
    int32_t sweep_chunk = 0;
    // SN_TEST_SWEEP_UNPACKED: every mesh keeps the 16-byte neighbour table
    // (the form of meshes whose id distances do not fit the packed word)
    bool sweep_unpacked = false;
    // test knob (SN_TEST_NO_PCELL): meshes keep no cell index per point, as
    // for volumes of 2^32 cells or more, so world points come from k_emit
    // after the sweeps
    bool no_pcell = false;
    // device address of the no-allocation extraction's static scratch array
    void *noalloc_scratch = nullptr;
    // the sweeps of a batch: one HIP graph per call (default), or the kernels
    // launched one by one (SN_BATCH_SWEEPS=eager)
    bool batch_eager = false;
    // sweep graphs launched and not yet known to be complete: destroyed once
    // their event has completed (destroying a graph in flight would hold the
    // host thread until it finishes)
    std::mutex graph_mu;
    std::vector<std::pair<hipGraphExec_t, hipEvent_t>> graph_retire;
    void reap_graphs(bool wait);
    sn::Schedule schedule(const std::string &cls) const;
    void load_tune_cache();
    void save_tune_cache() const;
};

struct sn_mesh {
    ~sn_mesh();
    sn_ctx *ctx = nullptr;
    sn::VolDesc d{};            // host copy (device pointers inside)
    int64_t P = 0, Q = 0, S = 0, voxels = 0, ntiles = 0;
    int32_t bpw = 2;
    sn::Schedule sched;  // the schedule of its extraction (and of its sweeps)
    std::vector<void *> blocks;  // every device block owned by the mesh
    float *da = nullptr, *db = nullptr;
    int32_t *nbr = nullptr;  // [P][4] y/z stencil neighbours, written by sweep 0
    const float *final_delta = nullptr;


    // recorded after the last library work on the mesh (shared by the meshes
    // of one batch call)
    sn::EventRef done;
};

namespace sn {

struct ProfScope {
    ProfScope(sn_ctx *c, const char *name, hipStream_t s, int64_t launches = 1);
    ~ProfScope();
    sn_ctx *c_;
    std::string name_;
    hipStream_t s_;
    int64_t launches_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

sn_status validate_volume(const sn_volume *v);
sn_status validate_smooth(const sn_smooth_params *p);
Geom make_geom(const sn_volume &v);
// classification mode of a volume and its table in host form (empty for the
// identity): the bitmap of selected values, or the sorted unique values
void class_table(const sn_volume &v, int32_t *mode, std::vector<uint32_t> *tab);
// The no-allocation extraction's static device scratch: resolves its address
// on the current device (once per device; sn_ctx_create calls it).
sn_status noalloc_resolve(int device, void **addr);
std::string size_class(const sn_volume &v);
// Called by extract_many once the totals of every volume are known and before
// any output is allocated: totals[3v .. 3v+2] = (P, Q, S) of vols[v].  A status
// other than SN_OK ends the extraction with that status (no mesh).
using AdmitFn = std::function<sn_status(const int64_t *totals)>;
// sched: the schedule to use, or nullptr for the context's choice for the
// largest volume's size class
sn_status extract_many(sn_ctx *c, const sn_volume *vols, int32_t n, hipStream_t s,
                       const Schedule *sched, sn_mesh **out, const AdmitFn *admit = nullptr);
// Device bytes, as the pool counts them (round_size per block), that an
// extraction of v holds for the call only (cut-edge planes, quad and stencil
// word bases, scan status, its share of the descriptor uploads), and that its
// mesh holds (word metadata, outputs, and the smoothing buffers when smoothed)
// for totals P, Q, S.
int64_t extract_scratch_bytes(const sn_volume &v);
int64_t mesh_bytes(const sn_volume &v, int64_t P, int64_t Q, int64_t S, bool smoothed);
sn_status smooth_many(sn_ctx *c, sn_mesh **ms, const sn_smooth_params *pv, int32_t n,
                      hipStream_t s);
// the plain path of one mesh (sweeps launched one by one, descriptor by value)
sn_status smooth_one(sn_ctx *c, sn_mesh *m, const sn_smooth_params *p, hipStream_t s);
sn_status ensure_smooth_buffers(sn_mesh *m);
// smoothing descriptor of a mesh for the given parameters
void fill_smooth_desc(const sn_mesh *m, const sn_smooth_params &p, SmoothDesc *sd);
// sweep `it` of grid.size() sweeps launches grid[it] blocks; big: the
// non-temporal form (every descriptor's big set)
sn_status run_sweeps(sn_ctx *c, const SmoothDesc *d_sd, const int64_t *d_bp, int32_t nvol,
                     const std::vector<int64_t> &grid, int K, bool big, hipStream_t s);
sn_status run_sweeps_one(sn_ctx *c, const SmoothDesc &sd, int64_t nblocks, int K, hipStream_t s);
sn_status mesh_mark(sn_mesh *m, hipStream_t s);
// mesh_mark for meshes[0..n) (null entries skipped) with one event recorded once
sn_status mesh_mark_all(sn_mesh *const *meshes, int32_t n, hipStream_t s);
void mesh_release(sn_mesh *m);
void ctx_retain(sn_ctx *c);
void ctx_release(sn_ctx *c);  // frees the context with its last reference

}  // namespace sn
