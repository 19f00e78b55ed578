// Host runtime of libsn.so: device memory pool, contexts, meshes, the plain
// and batched extraction/smoothing paths, the schedule tuner and profiling.
// The request server lives in sn_serve.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "sn.h"
#include "sn_internal.h"
#include "sn_runtime.h"

using namespace sn;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

sn_status sn::fail(sn_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

extern "C" const char *sn_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *sn_strerror(sn_status s)
{
    switch (s) {
    case SN_OK: return "ok";
    case SN_EINVAL: return "invalid argument";
    case SN_ENOMEM: return "out of device memory";
    case SN_EDEVICE: return "HIP runtime error";
    case SN_ETOOBIG: return "mesh index exceeds int32";
    case SN_EAGAIN: return "try again";
    case SN_ENOTFOUND: return "unknown ticket";
    case SN_ESHUTDOWN: return "server stopping";
    case SN_ETIMEDOUT: return "timed out";
    }
    return "unknown status";
}

extern "C" const char *sn_version(void) { return "libsn gfx950 " __DATE__; }

// ---------------------------------------------------------------------------
// Pool: caching allocator for device and pinned host blocks.  A released block
// may carry an event; it is reused only once that event has completed, so a
// block freed while a stream still uses it is never handed out early.
// ---------------------------------------------------------------------------

EventCache::~EventCache()
{
    for (auto e : free_) (void)hipEventDestroy(e);
}

hipEvent_t EventCache::get()
{
    {
        std::lock_guard<std::mutex> g(mu_);
        if (!free_.empty()) {
            hipEvent_t e = free_.back();
            free_.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, flags_) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Only events whose recorded work has completed come back here.
void EventCache::put(hipEvent_t e)
{
    if (!e) return;
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back(e);
}

size_t sn::round_size(size_t n)
{
    if (n == 0) n = 1;
    if (n <= (1u << 20)) return (n + 511) & ~size_t(511);
    const size_t g = size_t(2) << 20;
    return (n + g - 1) / g * g;
}

Pool::Pool(int /*device*/, bool pinned) : pinned_(pinned)
{
    if (!pinned) {
        const char *lim = std::getenv("SN_TEST_MEM_LIMIT");
        if (lim && *lim) limit_ = std::strtoll(lim, nullptr, 10);
    }
}

Pool::~Pool()
{
    std::lock_guard<std::mutex> g(mu_);
    reclaim_locked(true);
    for (auto &kv : free_) raw_free(kv.second);
    free_.clear();
}

void Pool::raw_free(void *p)
{
    if (pinned_)
        (void)hipHostFree(p);
    else
        (void)hipFree(p);
}

// Deferred blocks come back in release order; without `wait` the scan stops
// at the first release whose event has not completed.
void Pool::reclaim_locked(bool wait)
{
    while (!pending_.empty()) {
        Pending &pd = pending_.front();
        const hipError_t q = wait ? hipEventSynchronize(pd.ev) : hipEventQuery(pd.ev);
        if (q == hipErrorNotReady) break;
        for (void *p : pd.blocks) free_.emplace(sizes_[p], p);
        if (pd.ref)
            pd.ref.reset();  // the event returns to the cache with its last holder
        else if (q == hipSuccess)
            events_.put(pd.ev);
        else
            (void)hipEventDestroy(pd.ev);
        pending_.pop_front();
    }
}

void *Pool::alloc(size_t bytes)
{
    const size_t n = round_size(bytes);
    std::lock_guard<std::mutex> g(mu_);
    if (limit_ >= 0 && in_use_ + (int64_t)n > limit_) return nullptr;
    reclaim_locked(false);
    auto it = free_.lower_bound(n);
    if (it != free_.end() && it->first <= 2 * n + (size_t(4) << 20)) {
        void *p = it->second;
        free_.erase(it);
        charged_[p] = n;
        in_use_ += (int64_t)n;
        peak_ = std::max(peak_, in_use_);
        return p;
    }
    void *p = nullptr;
    // pinned host blocks are coherent: kernels may write results into them
    // (the count totals) that the host reads after the stream's completion
    hipError_t e = pinned_ ? hipHostMalloc(&p, n, hipHostMallocCoherent) : hipMalloc(&p, n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // drop every cached block (waiting for deferred ones) and retry once
        reclaim_locked(true);
        for (auto &kv : free_) raw_free(kv.second), sizes_.erase(kv.second), charged_.erase(kv.second);
        free_.clear();
        e = pinned_ ? hipHostMalloc(&p, n, hipHostMallocCoherent) : hipMalloc(&p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    sizes_[p] = n;
    charged_[p] = n;
    in_use_ += (int64_t)n;
    peak_ = std::max(peak_, in_use_);
    return p;
}

void Pool::release(void *p, hipStream_t after)
{
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = sizes_.find(p);
    if (it == sizes_.end()) return;
    in_use_ -= (int64_t)charged_[p];
    charged_.erase(p);
    if (after == kNoWait) {
        free_.emplace(it->second, p);
        return;
    }
    hipEvent_t ev = events_.get();
    if (!ev || hipEventRecord(ev, after) != hipSuccess) {
        (void)hipGetLastError();
        if (ev) (void)hipEventDestroy(ev);
        (void)hipStreamSynchronize(after);
        free_.emplace(it->second, p);
        return;
    }
    pending_.push_back(Pending{ev, {p}});
}

void Pool::release_all(const std::vector<void *> &ps, hipStream_t after)
{
    std::lock_guard<std::mutex> g(mu_);
    std::vector<void *> live;
    for (void *p : ps) {
        if (!p) continue;
        auto it = sizes_.find(p);
        if (it == sizes_.end()) continue;
        in_use_ -= (int64_t)charged_[p];
        charged_.erase(p);
        live.push_back(p);
    }
    if (live.empty()) return;
    hipEvent_t ev = after == kNoWait ? nullptr : events_.get();
    if (after == kNoWait || !ev || hipEventRecord(ev, after) != hipSuccess) {
        (void)hipGetLastError();
        if (ev) (void)hipEventDestroy(ev);
        if (after != kNoWait) (void)hipStreamSynchronize(after);
        for (void *p : live) free_.emplace(sizes_[p], p);
        return;
    }
    pending_.push_back(Pending{ev, std::move(live)});
}

SharedEvent::~SharedEvent()
{
    if (home) home->put_event(ev);
}

EventRef Pool::shared_event()
{
    hipEvent_t e = events_.get();
    if (!e) return nullptr;
    return std::make_shared<SharedEvent>(e, this);
}

void Pool::release_all_after(const std::vector<void *> &ps, EventRef ev)
{
    std::lock_guard<std::mutex> g(mu_);
    std::vector<void *> live;
    for (void *p : ps) {
        if (!p) continue;
        auto it = sizes_.find(p);
        if (it == sizes_.end()) continue;
        in_use_ -= (int64_t)charged_[p];
        charged_.erase(p);
        live.push_back(p);
    }
    if (live.empty()) return;
    hipEvent_t e = ev->ev;
    pending_.push_back(Pending{e, std::move(live), std::move(ev)});
}

int64_t Pool::in_use() const
{
    std::lock_guard<std::mutex> g(mu_);
    return in_use_;
}

int64_t Pool::peak() const
{
    std::lock_guard<std::mutex> g(mu_);
    return peak_;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

extern "C" sn_status sn_ctx_create(int device, sn_ctx **out)
{
    if (!out) return fail(SN_EINVAL, "sn_ctx_create: out is NULL");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return fail(SN_EDEVICE, "sn_ctx_create: no such HIP device");
    }
    HIP_TRY(hipSetDevice(device));
    sn_ctx *c = new sn_ctx(device);
    if (hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(SN_EDEVICE, "sn_ctx_create: stream creation failed");
    }
    if (sn_status st = noalloc_resolve(device, &c->noalloc_scratch); st != SN_OK) {
        (void)hipStreamDestroy(c->copy_stream);
        delete c;
        return st;
    }
    if (const char *cw = std::getenv("SN_TEST_COUNT_WIDE_WORDS"); cw && *cw)
        c->count_wide_words = std::strtoll(cw, nullptr, 10);
    if (const char *sp = std::getenv("SN_TEST_SWEEP_SMALL_POINTS"); sp && *sp)
        c->sweep_small_points = std::max<int64_t>(0, std::strtoll(sp, nullptr, 10));
    if (const char *be = std::getenv("SN_BATCH_SWEEPS"); be && *be)
        c->batch_eager = std::string(be) == "eager";
    if (const char *su = std::getenv("SN_TEST_SWEEP_UNPACKED"); su && *su)
        c->sweep_unpacked = std::strtoll(su, nullptr, 10) != 0;
    if (const char *np = std::getenv("SN_TEST_NO_PCELL"); np && *np)
        c->no_pcell = std::strtoll(np, nullptr, 10) != 0;
    if (const char *sc = std::getenv("SN_TEST_SWEEP_CHUNK"); sc && *sc)
        c->sweep_chunk = (int32_t)std::min<int64_t>(std::max<int64_t>(0, std::strtoll(sc, nullptr, 10)),
                                                    int64_t(1) << 20);
    const char *cache = std::getenv("SN_AUTOTUNE_CACHE");
    if (cache && *cache) {
        c->tune_path = cache;
        c->load_tune_cache();
    }
    *out = c;
    return SN_OK;
}

extern "C" sn_status sn_ctx_memory(sn_ctx *c, int64_t *in_use_bytes, int64_t *peak_bytes)
{
    if (!c) return fail(SN_EINVAL, "sn_ctx_memory: ctx is NULL");
    if (in_use_bytes) *in_use_bytes = c->pool.in_use();
    if (peak_bytes) *peak_bytes = c->pool.peak();
    return SN_OK;
}

void sn::ctx_retain(sn_ctx *c) { c->refs.fetch_add(1, std::memory_order_relaxed); }

void sn::ctx_release(sn_ctx *c)
{
    if (c->refs.fetch_sub(1, std::memory_order_acq_rel) != 1) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->copy_stream);
    (void)hipStreamDestroy(c->copy_stream);
    delete c;
}

extern "C" void sn_ctx_destroy(sn_ctx *c)
{
    if (c) ctx_release(c);
}

sn_ctx::sn_ctx(int dev) : device(dev), pool(dev, false), pinned(dev, true) {}

sn_ctx::~sn_ctx()
{
    reap_graphs(true);
    for (auto &p : prof_pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
}

void sn_ctx::reap_graphs(bool wait)
{
    std::lock_guard<std::mutex> g(graph_mu);
    size_t keep = 0;
    for (size_t k = 0; k < graph_retire.size(); ++k) {
        auto &gr = graph_retire[k];
        const hipError_t q = wait ? hipEventSynchronize(gr.second) : hipEventQuery(gr.second);
        if (q == hipErrorNotReady) {
            graph_retire[keep++] = gr;
            continue;
        }
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(gr.first);
        sync_events.put(gr.second);
    }
    graph_retire.resize(keep);
}

// ---- profiling -------------------------------------------------------------

ProfScope::ProfScope(sn_ctx *c, const char *name, hipStream_t s, int64_t launches)
    : c_(c), name_(name), s_(s), launches_(launches)
{
    if (!c_ || !c_->profiling || name_.empty()) return;  // an empty name: no events
    if (c_->profile_sweeps_only && name_ != "k_jacobi") return;
    a_ = c_->timing_events.get();
    b_ = c_->timing_events.get();
    if (!a_ || !b_) {
        c_->timing_events.put(a_);
        c_->timing_events.put(b_);
        a_ = b_ = nullptr;
        return;
    }
    (void)hipEventRecord(a_, s_);
}

ProfScope::~ProfScope()
{
    if (!a_) return;
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> g(c_->prof_mu);
    c_->prof_pending.push_back(sn_ctx::ProfEv{name_, a_, b_, launches_});
}

extern "C" sn_status sn_profile_enable(sn_ctx *c, int on)
{
    if (!c || on < 0 || on > 3) return fail(SN_EINVAL, "sn_profile_enable: bad arguments");
    c->profiling = on != 0;
    c->profile_eager = on == 2;
    c->profile_sweeps_only = on == 3;
    return SN_OK;
}

extern "C" sn_status sn_profile_reset(sn_ctx *c)
{
    if (!c) return fail(SN_EINVAL, "sn_profile_reset: ctx is NULL");
    std::lock_guard<std::mutex> g(c->prof_mu);
    for (auto &p : c->prof_pending) {
        (void)hipEventSynchronize(p.b);
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    c->prof_pending.clear();
    c->prof_stats.clear();
    return SN_OK;
}

extern "C" sn_status sn_profile_read(sn_ctx *c, sn_kernel_stat *out, int32_t cap, int32_t *n_out)
{
    if (!c || (cap > 0 && !out)) return fail(SN_EINVAL, "sn_profile_read: bad arguments");
    std::lock_guard<std::mutex> g(c->prof_mu);
    for (auto &p : c->prof_pending) {
        HIP_TRY(hipEventSynchronize(p.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
        auto &st = c->prof_stats[p.name];
        st.first += p.launches;
        st.second += ms;
        c->timing_events.put(p.a);
        c->timing_events.put(p.b);
    }
    c->prof_pending.clear();
    int32_t k = 0;
    for (auto &kv : c->prof_stats) {
        if (k < cap) {
            std::memset(&out[k], 0, sizeof(sn_kernel_stat));
            std::snprintf(out[k].name, sizeof(out[k].name), "%s", kv.first.c_str());
            out[k].launches = kv.second.first;
            out[k].total_ms = kv.second.second;
        }
        ++k;
    }
    if (n_out) *n_out = k;
    return SN_OK;
}

// ---- schedule table (size class -> batches per wave) ----------------------------------------------------------

std::string sn::size_class(const sn_volume &v)
{
    // the schedule matters through the number of rows and their length
    const int64_t M = v.dims[0], R = std::max<int64_t>(1, (v.dims[1] - 1) * (v.dims[2] - 1));
    int lm = 0, lr = 0;
    while ((int64_t(1) << (lm + 1)) <= M) ++lm;
    while ((int64_t(1) << (lr + 1)) <= R) ++lr;
    std::ostringstream os;
    os << "b" << v.dtype << "_m" << lm << "_r" << lr;
    return os.str();
}

Schedule sn_ctx::schedule(const std::string &cls) const
{
    std::lock_guard<std::mutex> g(tune_mu);
    // untuned: one k_generate group per wave, the fastest at every size
    // measured (torso 31 us against 43-80 us, connectome 3.23 ms against
    // 3.46-3.60 ms for 2 to 8 groups per wave), four k_edges segments per
    // wave, the k_count form by size, the default block order
    Schedule sc;
    auto it = tune.find(cls);
    if (it != tune.end()) sc = it->second;
    if (forced_bpw > 0) sc.gen_groups = forced_bpw;
    return sc;
}

static bool valid_schedule(const Schedule &s)
{
    return s.gen_groups >= 1 && s.gen_groups <= kMaxBatchesPerWave &&
           (s.count_words == 0 || s.count_words == 1 || s.count_words == kCountWideV) &&
           s.edge_segs >= 1 && s.edge_segs <= kMaxSegmentsPerWave && s.sweep_chunk >= 0 &&
           s.sweep_chunk <= (1 << 20);
}

void sn_ctx::load_tune_cache()
{
    std::ifstream f(tune_path);
    if (!f) return;
    // JSON object {"class": {"gen_groups": g, "count_words": c, "edge_segments": e,
    // "sweep_chunk": k}, ...}; an older flat {"class": g} gives gen_groups alone
    std::string s((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    auto field = [](const std::string &obj, const char *name, int32_t dflt) {
        const std::string key = std::string("\"") + name + "\"";
        const size_t p = obj.find(key);
        if (p == std::string::npos) return dflt;
        const size_t colon = obj.find(':', p + key.size());
        return colon == std::string::npos ? dflt : (int32_t)std::atoi(obj.c_str() + colon + 1);
    };
    size_t p = s.find('{');
    if (p == std::string::npos) return;
    ++p;
    while ((p = s.find('"', p)) != std::string::npos) {
        const size_t q = s.find('"', p + 1);
        if (q == std::string::npos) break;
        const std::string key = s.substr(p + 1, q - p - 1);
        size_t colon = s.find(':', q);
        if (colon == std::string::npos) break;
        size_t v = s.find_first_not_of(" \t\r\n", colon + 1);
        if (v == std::string::npos) break;
        Schedule sc;
        if (s[v] == '{') {
            const size_t e = s.find('}', v);
            if (e == std::string::npos) break;
            const std::string obj = s.substr(v, e - v + 1);
            sc.gen_groups = field(obj, "gen_groups", 1);
            sc.count_words = field(obj, "count_words", 0);
            sc.edge_segs = field(obj, "edge_segments", 4);
            sc.sweep_chunk = field(obj, "sweep_chunk", 0);
            p = e + 1;
        } else {
            sc.gen_groups = (int32_t)std::atoi(s.c_str() + v);
            p = v + 1;
        }
        if (valid_schedule(sc)) tune[key] = sc;
    }
}

void sn_ctx::save_tune_cache() const
{
    if (tune_path.empty()) return;
    std::ofstream f(tune_path);
    f << "{";
    bool first = true;
    for (auto &kv : tune) {
        const Schedule &sc = kv.second;
        f << (first ? "" : ",") << "\n \"" << kv.first << "\": {\"gen_groups\": " << sc.gen_groups
          << ", \"count_words\": " << sc.count_words << ", \"edge_segments\": " << sc.edge_segs
          << ", \"sweep_chunk\": " << sc.sweep_chunk << "}";
        first = false;
    }
    f << "\n}\n";
}

// ---------------------------------------------------------------------------
// validation and classification tables
// ---------------------------------------------------------------------------

sn_status sn::validate_volume(const sn_volume *v)
{
    if (!v) return fail(SN_EINVAL, "volume is NULL");
    if (v->dtype != 1 && v->dtype != 2 && v->dtype != 4)
        return fail(SN_EINVAL, "dtype must be SN_U8, SN_U16 or SN_U32");
    for (int a = 0; a < 3; ++a) {
        if (v->dims[a] < 1) return fail(SN_EINVAL, "dims must be >= 1");
        if (!(v->spacing[a] > 0) || !std::isfinite(v->spacing[a]))
            return fail(SN_EINVAL, "spacing must be positive and finite");
        if (!std::isfinite(v->origin[a])) return fail(SN_EINVAL, "origin must be finite");
    }
    if (v->dims[0] > (int64_t(1) << 30) || v->dims[1] > (int64_t(1) << 30) ||
        v->dims[2] > (int64_t(1) << 30))
        return fail(SN_ETOOBIG, "a dimension exceeds 2^30");
    if (v->prim != SN_QUADS && v->prim != SN_TRIS && v->prim != SN_LINES)
        return fail(SN_EINVAL, "prim must be SN_QUADS, SN_TRIS or SN_LINES");
    if (v->prim == SN_LINES && v->dims[2] != 1)
        return fail(SN_EINVAL, "SN_LINES contours an image: dims[2] must be 1");
    const uint64_t vmax = v->dtype == 4 ? 0xFFFFFFFFull : ((1ull << (8 * v->dtype)) - 1);
    if (v->background > vmax) return fail(SN_EINVAL, "background does not fit the dtype");
    if (v->n_selected < 0 || (v->n_selected > 0 && !v->selected))
        return fail(SN_EINVAL, "selected labels missing");
    for (int32_t s = 0; s < v->n_selected; ++s) {
        if (v->selected[s] > vmax) return fail(SN_EINVAL, "a selected label does not fit the dtype");
        if (v->selected[s] == v->background)
            return fail(SN_EINVAL, "the background value cannot be selected");
    }
    const bool empty = v->dims[0] < 2 || v->dims[1] < 2 || (v->prim != SN_LINES && v->dims[2] < 2);
    if (!v->labels && !empty) return fail(SN_EINVAL, "labels is NULL");
    if ((reinterpret_cast<uintptr_t>(v->labels) & (uintptr_t)(v->dtype - 1)) != 0)
        return fail(SN_EINVAL, "labels is not aligned to its dtype");
    {
        // the kernels index rows, words and batches of one volume with int32;
        // the factors are bounded first, so that no product overflows int64
        const Geom g = make_geom(*v);
        if (g.R >= INT32_MAX || g.N * g.O >= INT32_MAX || g.R * g.W >= INT32_MAX ||
            g.R * g.NB >= INT32_MAX || g.N * g.O * g.WS >= INT32_MAX)
            return fail(SN_ETOOBIG, "volume has more than 2^31 cell words or sample-row words");
    }
    return SN_OK;
}

Geom sn::make_geom(const sn_volume &v)
{
    Geom g;
    g.M = v.dims[0], g.N = v.dims[1], g.O = v.dims[2];
    // an image (SN_LINES, O = 1) has one slice of cells
    const bool image = v.prim == SN_LINES;
    const bool empty = g.M < 2 || g.N < 2 || (!image && g.O < 2);
    g.CM = empty ? 0 : g.M - 1;
    g.CN = empty ? 0 : g.N - 1;
    g.CO = empty ? 0 : (image ? 1 : g.O - 1);
    g.R = g.CN * g.CO;
    g.W = (int32_t)((g.CM + 63) / 64);
    g.NB = (g.W + kU - 1) / kU;
    g.WS = empty ? 0 : (g.M + 63) / 64;
    // (clamped: make_geom also serves the validation of oversized volumes)
    g.ws_div = make_udiv((uint32_t)std::max<int64_t>(std::min<int64_t>(g.WS, INT32_MAX), 1));
    g.n_div = make_udiv((uint32_t)std::max<int64_t>(std::min<int64_t>(g.N, INT32_MAX), 1));
    return g;
}

// host form of the classification table; empty vector for the identity
void sn::class_table(const sn_volume &v, int32_t *mode, std::vector<uint32_t> *tab)
{
    tab->clear();
    if (v.n_selected == 0) {
        *mode = CLS_IDENT;
        return;
    }
    // a bitmap over [0, 65536) serves u8 and u16, and u32 selections of small
    // values: one table load per sample instead of a binary search
    const uint32_t top = *std::max_element(v.selected, v.selected + v.n_selected);
    if (v.dtype <= 2 || top < 65536u) {
        *mode = CLS_BITMAP;
        tab->assign(v.dtype == 1 ? 8 : 2048, 0u);
        for (int32_t s = 0; s < v.n_selected; ++s) {
            const uint32_t x = v.selected[s];
            (*tab)[x >> 5] |= 1u << (x & 31u);
        }
        return;
    }
    *mode = CLS_SORTED;
    tab->assign(v.selected, v.selected + v.n_selected);
    std::sort(tab->begin(), tab->end());
    tab->erase(std::unique(tab->begin(), tab->end()), tab->end());
}

// ---------------------------------------------------------------------------
// meshes
// ---------------------------------------------------------------------------

sn_mesh::~sn_mesh() {}

void sn::mesh_release(sn_mesh *m)
{
    if (!m) return;
    sn_ctx *c = m->ctx;
    (void)hipSetDevice(c->device);
    // everything the library enqueued for this mesh precedes done_ev: the
    // blocks are reused once it has completed (the pool takes the event),
    // without blocking the host
    if (m->done)
        c->pool.release_all_after(m->blocks, std::move(m->done));
    else
        c->pool.release_all(m->blocks, Pool::kNoWait);
    delete m;
    ctx_release(c);
}

extern "C" void sn_mesh_free(sn_mesh *m) { mesh_release(m); }

sn_status sn::mesh_mark(sn_mesh *m, hipStream_t s)
{
    // an event shared with other meshes is not moved: this mesh takes its own
    if (!m->done || m->done.use_count() > 1) {
        m->done = m->ctx->pool.shared_event();
        if (!m->done) return fail(SN_EDEVICE, "mesh: no event");
    }
    HIP_TRY(hipEventRecord(m->done->ev, s));
    return SN_OK;
}

sn_status sn::mesh_mark_all(sn_mesh *const *meshes, int32_t n, hipStream_t s)
{
    sn_mesh *first = nullptr;
    for (int32_t k = 0; k < n && !first; ++k) first = meshes[k];
    if (!first) return SN_OK;
    EventRef e = first->ctx->pool.shared_event();
    if (!e) return fail(SN_EDEVICE, "mesh: no event");
    HIP_TRY(hipEventRecord(e->ev, s));
    for (int32_t k = 0; k < n; ++k)
        if (meshes[k]) meshes[k]->done = e;
    return SN_OK;
}

extern "C" sn_status sn_mesh_view_get(const sn_mesh *m, sn_mesh_view *out)
{
    if (!m || !out) return fail(SN_EINVAL, "sn_mesh_view_get: NULL argument");
    sn_mesh_view v;
    std::memset(&v, 0, sizeof v);
    v.n_points = m->P, v.n_quads = m->Q, v.n_stencil = m->S;
    v.prim = m->d.prim, v.dtype = m->d.dtype;
    v.points = m->d.points;
    v.offsets = m->final_delta;
    v.quads = m->d.quads;
    v.stencil_off = m->d.st_off;
    v.stencil_ids = m->d.st_ids;
    if (m->d.prim == SN_TRIS) {
        v.n_polys = 2 * m->Q;
        v.polys = m->d.tris;
        v.label_pairs = m->d.tri_pairs;
    } else if (m->d.prim == SN_LINES) {  // an image's contour segments
        v.n_polys = m->Q;
        v.polys = m->d.quads;
        v.label_pairs = m->d.pairs;
        v.quads = nullptr;
    } else {
        v.n_polys = m->Q;
        v.polys = m->d.quads;
        v.label_pairs = m->d.pairs;
    }
    *out = v;
    return SN_OK;
}

extern "C" sn_status sn_mesh_copy_to_host(const sn_mesh *m, float *points, int32_t *polys,
                                          void *labels, int32_t *st_off, int32_t *st_ids,
                                          float *offsets)
{
    if (!m) return fail(SN_EINVAL, "sn_mesh_copy_to_host: mesh is NULL");
    HIP_TRY(hipSetDevice(m->ctx->device));
    if (m->done) HIP_TRY(hipEventSynchronize(m->done->ev));
    sn_mesh_view v;
    sn_mesh_view_get(m, &v);
    // a non-blocking stream of the context: no implicit ordering with the
    // legacy stream or with other threads' streams (the mesh's own work is
    // complete after the event wait above)
    hipStream_t cs = m->ctx->copy_stream;
    auto cp = [cs](void *dst, const void *src, size_t n) -> hipError_t {
        if (!dst || n == 0) return hipSuccess;
        if (!src) return hipErrorInvalidValue;
        return hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, cs);
    };
    HIP_TRY(cp(points, v.points, sizeof(float) * 3 * v.n_points));
    HIP_TRY(cp(polys, v.polys, sizeof(int32_t) * v.prim * v.n_polys));
    HIP_TRY(cp(labels, v.label_pairs, (size_t)v.dtype * 2 * v.n_polys));
    HIP_TRY(cp(st_off, v.stencil_off, sizeof(int32_t) * (v.n_points + 1)));
    HIP_TRY(cp(st_ids, v.stencil_ids, sizeof(int32_t) * v.n_stencil));
    if (offsets) {
        if (v.offsets)
            HIP_TRY(cp(offsets, v.offsets, sizeof(float) * 3 * v.n_points));
        else
            std::memset(offsets, 0, sizeof(float) * 3 * v.n_points);
    }
    HIP_TRY(hipStreamSynchronize(cs));
    return SN_OK;
}

// ---------------------------------------------------------------------------
// extraction (plain = a batch of one)
// ---------------------------------------------------------------------------

namespace {

// Upload of a staging block from the pinned pool to a device block (both
// from the pools, so rounded to at least 512 bytes) by a kernel on `s`.
hipError_t stage_upload(void *d, void *h, size_t bytes, hipStream_t s)
{
    void *hm = nullptr;
    hipError_t e = hipHostGetDevicePointer(&hm, h, 0);
    if (e != hipSuccess) return e;
    return launch_stage(d, hm, bytes, s);
}

struct Scratch {
    sn_ctx *c;
    std::vector<void *> dev, host;
    explicit Scratch(sn_ctx *ctx) : c(ctx) {}
    void *d(size_t n)
    {
        void *p = c->pool.alloc(n);
        if (p) dev.push_back(p);
        return p;
    }
    void *h(size_t n)
    {
        void *p = c->pinned.alloc(n);
        if (p) host.push_back(p);
        return p;
    }
    void retire(hipStream_t s)
    {
        c->pool.release_all(dev, s);
        c->pinned.release_all(host, s);
        dev.clear();
        host.clear();
    }
};

// Sub-allocation of several arrays from one pool block: each array starts on
// a 256-byte boundary.
struct Carve {
    size_t bytes = 0;
    size_t add(int64_t n)
    {
        const size_t at = bytes;
        bytes += ((size_t)std::max<int64_t>(n, 1) + 255) & ~size_t(255);
        return at;
    }
};

// The mesh's word metadata block: point bits, then first point ids.
struct MetaLayout {
    size_t o_pm, o_wb, bytes;
};
MetaLayout meta_layout(int64_t words)
{
    Carve cv;
    MetaLayout l;
    l.o_pm = cv.add(8 * words);
    l.o_wb = cv.add(4 * words);
    l.bytes = cv.bytes;
    return l;
}

// Every output of a mesh in one block, sized exactly from the totals.
struct OutLayout {
    size_t o_pts, o_fc, o_off, o_ids, o_q, o_pr, o_t, o_tp, o_pc, bytes;
    bool tris, cells32;
};
OutLayout out_layout(const Geom &g, int32_t prim, int32_t dtype, int64_t P, int64_t Q, int64_t S)
{
    Carve cv;
    OutLayout l{};
    l.o_pts = cv.add(12 * P), l.o_fc = cv.add(P), l.o_off = cv.add(4 * (P + 1));
    const int64_t quad_bytes = prim == SN_LINES ? 8 : 16;  // segments [Q][2] or quads [Q][4]
    l.o_ids = cv.add(4 * S), l.o_q = cv.add(quad_bytes * Q), l.o_pr = cv.add(2 * Q * dtype);
    l.tris = prim == SN_TRIS;
    if (l.tris) l.o_t = cv.add(24 * Q), l.o_tp = cv.add(4 * Q * dtype);
    // cell index per point (for world points written by the last sweep),
    // when every cell index fits 32 bits
    l.cells32 = (uint64_t)g.R * (uint64_t)g.CM < (uint64_t(1) << 32);
    if (l.cells32) l.o_pc = cv.add(4 * P);
    l.bytes = cv.bytes;
    return l;
}

// The smoothing block: two offset buffers and the y/z neighbour table.
struct SmoothLayout {
    size_t o_a, o_b, o_n, bytes;
};
SmoothLayout smooth_layout(int64_t P)
{
    Carve cv;
    SmoothLayout l;
    l.o_a = cv.add(12 * P), l.o_b = cv.add(12 * P), l.o_n = cv.add(16 * P);
    l.bytes = cv.bytes;
    return l;
}

// Extraction scratch of one volume: quad and stencil word bases, cut-edge planes.
int64_t words_of(const Geom &g) { return g.R * g.W; }
int64_t plane_words_of(const Geom &g) { return 3 * g.N * g.O * g.WS; }

template <typename T>
T *dalloc(sn_mesh *m, int64_t count)
{
    void *p = m->ctx->pool.alloc(sizeof(T) * (size_t)std::max<int64_t>(count, 1));
    if (p) m->blocks.push_back(p);
    return static_cast<T *>(p);
}

}  // namespace

int64_t sn::extract_scratch_bytes(const sn_volume &v)
{
    const Geom g = make_geom(v);
    const int64_t words = words_of(g);
    const int64_t w1 = std::max<int64_t>(words, 1);
    // wbQ, wbS, planes; scan status (narrow tiles are the most) with the
    // ticket; descriptor, tile-map and table staging of a batch (three
    // uploads, each rounded on its own)
    const int64_t tiles = (words + kCountBlock - 1) / kCountBlock;
    const int64_t stage = 3 * (int64_t)sizeof(VolDesc) + (int64_t)sizeof(SmoothDesc) + 8 * 8 +
                          8 * (v.n_selected > 0 ? (v.dtype == 1 ? 4 : 1024) + v.n_selected : 0);
    return (int64_t)(2 * round_size(4 * w1) + round_size(8 * std::max<int64_t>(plane_words_of(g), 1)) +
                     round_size(24 * std::max<int64_t>(tiles, 1) + 256)) +
           stage + 3 * 512;
}

int64_t sn::mesh_bytes(const sn_volume &v, int64_t P, int64_t Q, int64_t S, bool smoothed)
{
    const Geom g = make_geom(v);
    int64_t b = (int64_t)round_size(meta_layout(words_of(g)).bytes) +
                (int64_t)round_size(out_layout(g, v.prim, v.dtype, P, Q, S).bytes);
    if (smoothed && P > 0) b += (int64_t)round_size(smooth_layout(P).bytes);
    return b;
}

// Host spin on the count stamps before blocking on the stream (longer than the
// edge and count passes of the largest single volumes measured, 0.75 ms).
constexpr int64_t kTotalsSpinUs = 3000;

// Wait until k_count has stamped the totals of every counted volume: spin on
// the host-visible stamps for a while (the count pass usually ends within
// that), then block on the stream.
static sn_status wait_totals(const int64_t *stamps, const std::vector<char> &counted, int64_t seq,
                             hipStream_t s)
{
    auto stamped = [&] {
        for (size_t k = 0; k < counted.size(); ++k)
            if (counted[k] && __atomic_load_n(stamps + k, __ATOMIC_ACQUIRE) != seq) return false;
        return true;
    };
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t spin = 1;; ++spin) {
        if (stamped()) return SN_OK;
        if ((spin & 255u) == 0 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kTotalsSpinUs))
            break;
        __builtin_ia32_pause();
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (!stamped()) return fail(SN_EDEVICE, "extract: the count pass left no totals");
    return SN_OK;
}

// As HIP_TRY, releasing the meshes of a failed extraction (the `cleanup`
// of extract_many) before returning.
#define HIP_TRY_CLEANUP(expr)                                                                      \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess)                                                                      \
            return cleanup(fail(SN_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)));   \
    } while (0)

sn_status sn::extract_many(sn_ctx *c, const sn_volume *vols, int32_t n, hipStream_t s,
                           const Schedule *sched, sn_mesh **out, const AdmitFn *admit)
{
    if (!c || !vols || !out || n < 1) return fail(SN_EINVAL, "extract: bad arguments");
    for (int32_t v = 0; v < n; ++v) {
        sn_status st = validate_volume(&vols[v]);
        if (st != SN_OK) return st;
    }
    HIP_TRY(hipSetDevice(c->device));
    std::vector<sn_mesh *> meshes(n, nullptr);
    Scratch scr(c);
    auto cleanup = [&](sn_status st) {
        scr.retire(s);
        for (auto *m : meshes)
            if (m) {
                m->ctx->pool.release_all(m->blocks, s);
                m->blocks.clear();
                delete m;
                ctx_release(c);
            }
        return st;
    };
    // one schedule for the launch: the one tuned for the largest volume
    int64_t big = 0;
    int32_t vb = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int64_t vox = vols[v].dims[0] * vols[v].dims[1] * vols[v].dims[2];
        if (vox > big) big = vox, vb = v;
    }
    const Schedule sc = sched ? *sched : c->schedule(size_class(vols[vb]));
    const int32_t bpw = sc.gen_groups;
    const int TB = kWavesPerBlock * bpw;

    // Volumes are processed grouped by (label type, classification mode): one
    // kernel instantiation per group.  Position k of the launch arrays holds
    // volume order[k].
    std::vector<int32_t> mode(n), order(n);
    std::vector<std::vector<uint32_t>> tabs(n);
    for (int32_t v = 0; v < n; ++v) {
        class_table(vols[v], &mode[v], &tabs[v]);
        order[v] = v;
    }
    // wide: rows start 16-byte aligned and hold a multiple of 4 samples
    auto wide = [&](int32_t v) {
        return vols[v].dims[0] % 4 == 0 && (reinterpret_cast<uintptr_t>(vols[v].labels) & 15) == 0;
    };
    auto key = [&](int32_t v) {
        return (vols[v].prim == SN_LINES ? 64 : 0) + vols[v].dtype * 8 + mode[v] * 2 + (wide(v) ? 1 : 0);
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });

    std::vector<int64_t> tile_prefix(n + 1, 0), etile_prefix(n + 1, 0), ctile_prefix(n + 1, 0);
    // A single volume travels to its kernels by value (kernel arguments); a
    // batch uploads its descriptor array and tile maps once.  Classification
    // tables are uploaded in the same block (read by k_edges and k_generate
    // only, so they live as long as this call's scratch).
    const bool one = (n == 1);
    size_t tab_words = 0;
    for (int32_t v = 0; v < n; ++v) tab_words += (tabs[v].size() + 1) / 2;
    const size_t arr_bytes = one ? 0 : sizeof(VolDesc) * n + sizeof(int64_t) * 3 * (n + 1);
    const size_t up_a = arr_bytes + 8 * tab_words;
    uint8_t *h_up = nullptr, *d_up = nullptr;
    if (up_a > 0) {
        h_up = static_cast<uint8_t *>(scr.h(up_a));
        d_up = static_cast<uint8_t *>(scr.d(up_a));
        if (!h_up || !d_up) return cleanup(fail(SN_ENOMEM, "extract: descriptor staging"));
    }
    std::vector<VolDesc> hd(n);  // host descriptors in launch order
    VolDesc *d_desc = one ? nullptr : reinterpret_cast<VolDesc *>(d_up);
    int64_t *d_tp = one ? nullptr : reinterpret_cast<int64_t *>(d_up + sizeof(VolDesc) * n);
    uint32_t *h_tab = h_up ? reinterpret_cast<uint32_t *>(h_up + arr_bytes) : nullptr;
    uint32_t *d_tab = d_up ? reinterpret_cast<uint32_t *>(d_up + arr_bytes) : nullptr;
    size_t tab_at = 0;  // in uint32 units, kept 8-byte aligned
    for (int32_t k = 0; k < n; ++k) {
        const int32_t v = order[k];
        const sn_volume &vol = vols[v];
        sn_mesh *m = new sn_mesh();
        meshes[v] = m;
        m->ctx = c;
        ctx_retain(c);
        m->bpw = bpw;
        m->sched = sc;
        VolDesc &d = m->d;
        std::memset(&d, 0, sizeof d);
        d.labels = vol.labels;
        d.dtype = vol.dtype;
        d.prim = vol.prim;
        d.g = make_geom(vol);
        for (int a = 0; a < 3; ++a) d.origin[a] = vol.origin[a], d.spacing[a] = vol.spacing[a];
        // an image's points lie in the plane z = origin[2]: with a zero z
        // spacing every kernel that writes world points puts them there
        if (vol.prim == SN_LINES) d.spacing[2] = 0.0;
        d.cs.mode = mode[v];
        d.cs.bg = vol.background;
        d.cs.n = (int32_t)tabs[v].size();
        if (!tabs[v].empty()) {
            std::memcpy(h_tab + tab_at, tabs[v].data(), sizeof(uint32_t) * tabs[v].size());
            d.cs.table = d_tab + tab_at;
            tab_at += 2 * ((tabs[v].size() + 1) / 2);
        }
        const int64_t words = words_of(d.g);
        {
            const MetaLayout ml = meta_layout(words);
            uint8_t *blk = dalloc<uint8_t>(m, (int64_t)ml.bytes);
            d.pmask = blk ? reinterpret_cast<uint64_t *>(blk + ml.o_pm) : nullptr;
            d.wbP = blk ? reinterpret_cast<int32_t *>(blk + ml.o_wb) : nullptr;
        }
        // extraction-only metadata: cut-edge planes and quad/stencil word bases
        d.wbQ = static_cast<int32_t *>(scr.d(sizeof(int32_t) * (size_t)std::max<int64_t>(words, 1)));
        d.wbS = static_cast<int32_t *>(scr.d(sizeof(int32_t) * (size_t)std::max<int64_t>(words, 1)));
        const int64_t pwords = plane_words_of(d.g);
        d.planes = static_cast<uint64_t *>(scr.d(sizeof(uint64_t) * (size_t)std::max<int64_t>(pwords, 1)));
        if (!d.pmask || !d.wbP || !d.wbQ || !d.wbS || !d.planes)
            return cleanup(fail(SN_ENOMEM, "extract: word metadata"));
        const int64_t nbatch = d.g.R * d.g.NB;
        // every volume has at least one generation tile: its first tile writes
        // st_off[P] = S (st_off[0] = 0 for an empty mesh)
        m->ntiles = std::max<int64_t>(1, (nbatch + TB - 1) / TB);  // k_emit
        const int64_t ngroups = (words + kGenWords - 1) / kGenWords;
        tile_prefix[k + 1] = tile_prefix[k] + std::max<int64_t>(1, (ngroups + TB - 1) / TB);
        const int64_t nseg = edge_segments(d.g);
        etile_prefix[k + 1] = etile_prefix[k] + edge_tiles(nseg, sc.edge_segs);
        ctile_prefix[k + 1] = words;  // words for now; tiles below
        m->voxels = vol.dims[0] * vol.dims[1] * vol.dims[2];
        hd[k] = d;
    }
    // count tiles: the wide form for launches of many words
    int64_t total_words = 0;
    for (int32_t k = 0; k < n; ++k) total_words += ctile_prefix[k + 1];
    const int32_t cv = sc.count_words > 0 ? sc.count_words
                                          : (total_words >= c->count_wide_words ? kCountWideV : 1);
    for (int32_t k = 0; k < n; ++k)
        ctile_prefix[k + 1] = ctile_prefix[k] + (ctile_prefix[k + 1] + cv * kCountBlock - 1) / (cv * kCountBlock);
    // groups: [gbeg[i], gbeg[i+1]) of the launch order share a key (k_edges);
    // k_generate does not depend on the row form, so its groups [ggbeg[i],
    // ggbeg[i+1]) join the wide and narrow volumes of a key (adjacent in the order)
    std::vector<int32_t> gbeg, ggbeg;
    for (int32_t k = 0; k < n; ++k) {
        if (k == 0 || key(order[k]) != key(order[k - 1])) gbeg.push_back(k);
        if (k == 0 || (key(order[k]) >> 1) != (key(order[k - 1]) >> 1)) ggbeg.push_back(k);
    }
    gbeg.push_back(n);
    ggbeg.push_back(n);
    const int32_t ngroups = (int32_t)gbeg.size() - 1, nggroups = (int32_t)ggbeg.size() - 1;

    const int64_t nctiles = ctile_prefix[n];
    // k_count writes the per-volume totals, then a stamp, straight into
    // coherent pinned host memory: no copy between the count pass and the
    // host's read of them, and the host sees them without waiting for the
    // whole pass to retire
    int64_t *h_tot = static_cast<int64_t *>(scr.h(sizeof(int64_t) * 4 * n));
    int64_t *d_tot = nullptr;
    if (h_tot && hipHostGetDevicePointer(reinterpret_cast<void **>(&d_tot), h_tot, 0) != hipSuccess)
        return cleanup(fail(SN_EDEVICE, "extract: totals buffer"));
    const size_t status_bytes = sizeof(uint64_t) * 3 * (size_t)std::max<int64_t>(nctiles, 1);
    uint8_t *d_status = static_cast<uint8_t *>(scr.d(status_bytes + 256));
    if (!h_tot || !d_tot || !d_status) return cleanup(fail(SN_ENOMEM, "extract: scratch"));
    uint64_t *status = reinterpret_cast<uint64_t *>(d_status);
    uint32_t *ticket = reinterpret_cast<uint32_t *>(d_status + status_bytes);
    if (!one) {
        // descriptors and the three tile maps: generation batches, edge segments, count words
        std::memcpy(h_up, hd.data(), sizeof(VolDesc) * n);
        int64_t *h_tp = reinterpret_cast<int64_t *>(h_up + sizeof(VolDesc) * n);
        std::memcpy(h_tp, tile_prefix.data(), sizeof(int64_t) * (n + 1));
        std::memcpy(h_tp + (n + 1), etile_prefix.data(), sizeof(int64_t) * (n + 1));
        std::memcpy(h_tp + 2 * (n + 1), ctile_prefix.data(), sizeof(int64_t) * (n + 1));
    }
    if (up_a > 0) HIP_TRY_CLEANUP(stage_upload(d_up, h_up, up_a, s));
    // the first edges launch clears the count pass's status words and ticket
    const int64_t nzero = (int64_t)((status_bytes + 256) / 8);
    {
        ProfScope ps(c, "k_edges", s);
        if (one) {
            HIP_TRY_CLEANUP(launch_edges_one(hd[0], wide(order[0]), etile_prefix[1], status, nzero,
                                             sc.edge_segs, s));
        } else {
            bool zeroed = false;
            for (int32_t gi = 0; gi < ngroups; ++gi) {
                const int32_t k0 = gbeg[gi], k1 = gbeg[gi + 1];
                const int64_t nt = etile_prefix[k1] - etile_prefix[k0];
                HIP_TRY_CLEANUP(launch_edges(hd[k0].dtype, hd[k0].cs.mode, wide(order[k0]), d_desc + k0,
                                     d_tp + (n + 1) + k0, k1 - k0, etile_prefix[k0], nt, status,
                                     (nt > 0 && !zeroed) ? nzero : 0, sc.edge_segs, s));
                zeroed = zeroed || nt > 0;
            }
        }
    }
    // Stamps: a value no earlier call in this process used (pinned blocks are
    // recycled, also between contexts), and the slots cleared by the host
    // before the count pass is enqueued, so a stale stamp in a recycled block
    // can never pass for this call's totals.
    static std::atomic<int64_t> g_count_seq{0};
    const int64_t seq = g_count_seq.fetch_add(1, std::memory_order_relaxed) + 1;
    for (int32_t k = 0; k < n; ++k) __atomic_store_n(h_tot + 3 * n + k, int64_t(0), __ATOMIC_RELAXED);
    std::atomic_thread_fence(std::memory_order_seq_cst);
    const CountOut cout{d_tot, d_tot + 3 * n, seq};
    {
        ProfScope ps(c, "k_count", s);
        if (one)
            HIP_TRY_CLEANUP(launch_count_one(hd[0], nctiles, cv, status, ticket, cout, s));
        else
            HIP_TRY_CLEANUP(launch_count(d_desc, d_tp + 2 * (n + 1), n, nctiles, cv, status, ticket, cout, s));
    }
    {
        std::vector<char> counted(n);
        for (int32_t k = 0; k < n; ++k) counted[k] = ctile_prefix[k + 1] > ctile_prefix[k];
        sn_status st = wait_totals(h_tot + 3 * n, counted, seq, s);
        if (st != SN_OK) return cleanup(st);
    }

    if (admit) {
        // the caller sees every volume's totals before any output is allocated
        std::vector<int64_t> tot(3 * (size_t)n, 0);
        for (int32_t k = 0; k < n; ++k)
            if (ctile_prefix[k + 1] > ctile_prefix[k])
                for (int q = 0; q < 3; ++q) tot[3 * order[k] + q] = h_tot[3 * k + q];
        sn_status st = (*admit)(tot.data());
        if (st != SN_OK) return cleanup(st);
    }
    // exact allocation of every output (Sec. 2.3: no incremental allocation)
    int64_t qblocks = 0;
    for (int32_t k = 0; k < n; ++k) {
        sn_mesh *m = meshes[order[k]];
        VolDesc &d = m->d;
        // a volume without cell words has no count tile and no totals written
        const bool counted = ctile_prefix[k + 1] > ctile_prefix[k];
        m->P = counted ? h_tot[3 * k] : 0;
        m->Q = counted ? h_tot[3 * k + 1] : 0;
        m->S = counted ? h_tot[3 * k + 2] : 0;
        if (m->P >= INT32_MAX || m->Q >= INT32_MAX / 2 || m->S >= INT32_MAX)
            return cleanup(fail(SN_ETOOBIG, "extract: mesh indices exceed int32"));
        d.P = m->P, d.Q = m->Q, d.S = m->S;
        // every output of the mesh in one block, sized exactly
        const OutLayout ol = out_layout(d.g, d.prim, d.dtype, m->P, m->Q, m->S);
        uint8_t *blk = dalloc<uint8_t>(m, (int64_t)ol.bytes);
        if (!blk) return cleanup(fail(SN_ENOMEM, "extract: outputs"));
        d.points = reinterpret_cast<float *>(blk + ol.o_pts);
        d.faces = blk + ol.o_fc;
        d.st_off = reinterpret_cast<int32_t *>(blk + ol.o_off);
        d.st_ids = reinterpret_cast<int32_t *>(blk + ol.o_ids);
        d.quads = reinterpret_cast<int32_t *>(blk + ol.o_q);
        d.pairs = blk + ol.o_pr;
        if (ol.tris) {
            d.tris = reinterpret_cast<int32_t *>(blk + ol.o_t);
            d.tri_pairs = blk + ol.o_tp;
            qblocks += (m->Q + 255) / 256;
        }
        d.pcell = ol.cells32 && !c->no_pcell ? reinterpret_cast<uint32_t *>(blk + ol.o_pc) : nullptr;
        hd[k] = d;
    }
    if (one) {
        {
            ProfScope ps(c, "k_generate", s);
            const bool staged = hd[0].P >= kGenStagedPointsPerWord * hd[0].g.R * hd[0].g.W;
            HIP_TRY_CLEANUP(launch_generate_one(hd[0], staged, tile_prefix[1], bpw, s));
        }
        if (qblocks > 0) {
            ProfScope ps(c, "k_tri", s);
            HIP_TRY_CLEANUP(launch_triangulate_one(hd[0], s));
        }
    } else {
        // second upload: descriptors with the output arrays, and the triangle
        // block map (volumes without triangles keep an empty range)
        const size_t up_b = sizeof(VolDesc) * n + sizeof(int64_t) * (n + 1);
        uint8_t *h_b = static_cast<uint8_t *>(scr.h(up_b));
        uint8_t *d_b = static_cast<uint8_t *>(scr.d(up_b));
        if (!h_b || !d_b) return cleanup(fail(SN_ENOMEM, "extract: descriptor staging"));
        std::memcpy(h_b, hd.data(), sizeof(VolDesc) * n);
        int64_t *h_qp = reinterpret_cast<int64_t *>(h_b + sizeof(VolDesc) * n);
        int64_t acc = 0;
        for (int32_t k = 0; k < n; ++k) {
            h_qp[k] = acc;
            if (hd[k].prim == SN_TRIS) acc += (hd[k].Q + 255) / 256;
        }
        h_qp[n] = acc;
        HIP_TRY_CLEANUP(stage_upload(d_b, h_b, up_b, s));
        VolDesc *d_desc2 = reinterpret_cast<VolDesc *>(d_b);
        {
            ProfScope ps(c, "k_generate", s);
            for (int32_t gi = 0; gi < nggroups; ++gi) {
                const int32_t k0 = ggbeg[gi], k1 = ggbeg[gi + 1];
                int64_t gp = 0, gw = 0;
                for (int32_t k = k0; k < k1; ++k) gp += hd[k].P, gw += hd[k].g.R * hd[k].g.W;
                const bool staged = gp >= kGenStagedPointsPerWord * gw;
                HIP_TRY_CLEANUP(launch_generate(hd[k0].dtype, hd[k0].cs.mode, staged, hd[k0].prim == SN_LINES,
                                                d_desc2 + k0, d_tp + k0, k1 - k0, tile_prefix[k0],
                                                tile_prefix[k1] - tile_prefix[k0], bpw, s));
            }
        }
        if (qblocks > 0) {
            ProfScope ps(c, "k_tri", s);
            HIP_TRY_CLEANUP(launch_triangulate(d_desc2, reinterpret_cast<int64_t *>(d_b + sizeof(VolDesc) * n),
                                       n, acc, s));
        }
    }
    if (sn_status st = mesh_mark_all(meshes.data(), n, s); st != SN_OK) return cleanup(st);
    scr.retire(s);
    for (int32_t v = 0; v < n; ++v) out[v] = meshes[v];
    return SN_OK;
}

#undef HIP_TRY_CLEANUP

extern "C" sn_status sn_extract(sn_ctx *c, const sn_volume *vol, void *stream, sn_mesh **out)
{
    if (!out) return fail(SN_EINVAL, "sn_extract: out is NULL");
    return extract_many(c, vol, 1, static_cast<hipStream_t>(stream), nullptr, out);
}

// ---------------------------------------------------------------------------
// smoothing
// ---------------------------------------------------------------------------

sn_status sn::validate_smooth(const sn_smooth_params *p)
{
    if (!p) return fail(SN_EINVAL, "smoothing parameters are NULL");
    if (p->iterations < 0) return fail(SN_EINVAL, "iterations must be >= 0");
    if (!(p->relaxation >= 0.f && p->relaxation <= 1.f))
        return fail(SN_EINVAL, "relaxation must be in [0, 1]");
    if (!(p->constraint >= 0.f) || !std::isfinite(p->constraint))
        return fail(SN_EINVAL, "constraint must be >= 0 and finite");
    if (p->shape != SN_BOX && p->shape != SN_SPHERE)
        return fail(SN_EINVAL, "constraint shape must be SN_BOX or SN_SPHERE");
    return SN_OK;
}

sn_status sn::ensure_smooth_buffers(sn_mesh *m)
{
    if (m->d.P == 0 || m->da) return SN_OK;
    const SmoothLayout sl = smooth_layout(m->P);
    uint8_t *blk = dalloc<uint8_t>(m, (int64_t)sl.bytes);
    if (!blk) return fail(SN_ENOMEM, "smooth: offset buffers");
    m->da = reinterpret_cast<float *>(blk + sl.o_a);
    m->db = reinterpret_cast<float *>(blk + sl.o_b);
    m->nbr = reinterpret_cast<int32_t *>(blk + sl.o_n);
    return SN_OK;
}

// Smoothing descriptor of a mesh for the given parameters.
void sn::fill_smooth_desc(const sn_mesh *m, const sn_smooth_params &p, SmoothDesc *sd)
{
    std::memset(sd, 0, sizeof *sd);
    sd->P = m->P, sd->faces = m->d.faces, sd->off = m->d.st_off, sd->ids = m->d.st_ids;
    sd->nbr = m->nbr, sd->da = m->da, sd->db = m->db, sd->iters = p.iterations;
    sd->lam = (double)p.relaxation, sd->dist = (double)p.constraint;
    sd->sphere = p.shape == SN_SPHERE ? 1 : 0;
    sd->pcell = m->d.pcell, sd->points = m->d.points;
    sd->CM = make_udiv((uint32_t)std::max<int64_t>(m->d.g.CM, 1));
    sd->CN = make_udiv((uint32_t)std::max<int64_t>(m->d.g.CN, 1));
    for (int a = 0; a < 3; ++a) sd->origin[a] = m->d.origin[a], sd->spacing[a] = m->d.spacing[a];
    // block order of a large single mesh: each XCD takes runs of about a
    // sixteenth of a slab's blocks in turn
    const int K = sweep_chunks(m->P);
    const int64_t per_slab = sweep_blocks_for(m->P, K) / std::max<int64_t>(1, m->d.g.CO);
    sd->chunk = (int32_t)std::max<int64_t>(1, (per_slab + 8) / 16);
    if (m->sched.sweep_chunk > 0) sd->chunk = m->sched.sweep_chunk;
    if (m->ctx->sweep_chunk > 0) sd->chunk = m->ctx->sweep_chunk;
    sd->big = m->P > m->ctx->sweep_small_points ? 1 : 0;
    // packed neighbour table when the id distances fit: at most a row of
    // cells for y neighbours, a slice for z (an image has no z neighbours)
    auto bits = [](int64_t v) {
        int32_t b = 0;
        while (b < 63 && (int64_t(1) << b) <= v) ++b;
        return std::max<int32_t>(b, 1);
    };
    const bool image = m->d.prim == SN_LINES;
    const int32_t yb = bits(m->d.g.CM), zb = image ? 1 : bits(m->d.g.CM * m->d.g.CN);
    if (yb + zb <= 31 && !m->ctx->sweep_unpacked) sd->pack_yb = yb, sd->pack_zb = zb;
}

// Sweeps over `nvol` meshes (descriptor array), replayed from a HIP graph of
// kernel nodes built for this call; sweep `it` launches grid[it] blocks
sn_status sn::run_sweeps(sn_ctx *c, const SmoothDesc *d_sd, const int64_t *d_bp, int32_t nvol,
                         const std::vector<int64_t> &grid, int K, bool big, hipStream_t s)
{
    const int32_t iters = (int32_t)grid.size();
    if (iters <= 0 || grid[0] <= 0) return SN_OK;
    if (c->profile_eager || c->batch_eager) {
        // eager launches (with profiling, each sweep bracketed by its own
        // events; sweeps 0 and 1 together, as in the graph)
        const bool each = c->profile_eager;
        ProfScope all(c, each ? "" : "k_jacobi", s, each ? 0 : iters);
        int32_t it0 = 0;
        if (iters >= 2 && grid[1] > 0) {
            ProfScope ps(c, each ? "k_jacobi" : "", s, each ? 2 : 0);
            HIP_TRY(launch_jacobi_first2(d_sd, d_bp, nvol, grid[0], grid[1], K, s));
            it0 = 2;
        }
        for (int32_t it = it0; it < iters && grid[it] > 0; ++it) {
            ProfScope ps(c, each ? "k_jacobi" : "", s, each ? 1 : 0);
            HIP_TRY(launch_jacobi(d_sd, d_bp, nvol, grid[it], it, K, big, s));
        }
        return SN_OK;
    }
    // one event pair around the whole graph replay: `iters` launches
    ProfScope ps(c, "k_jacobi", s, iters);
    // built node by node rather than by stream capture: no stream of the
    // process is ever in capture mode, so other threads' work on the legacy
    // stream cannot collide with it
    hipGraph_t graph;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipGraphCreate(&graph, 0));
    hipError_t e = add_jacobi_nodes(graph, d_sd, d_bp, nvol, grid.data(), iters, K, big);
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) {
        if (exec) (void)hipGraphExecDestroy(exec);
        return fail(SN_EDEVICE, std::string("smooth: sweep graph: ") + hipGetErrorString(e));
    }
    // destroyed once the replay has completed (destroying it now would hold
    // this thread until then, and the next call's work would start late)
    hipEvent_t done = c->sync_events.get();
    if (!done || hipEventRecord(done, s) != hipSuccess) {
        (void)hipGetLastError();
        if (done) c->sync_events.put(done);
        (void)hipGraphExecDestroy(exec);
        return SN_OK;
    }
    c->reap_graphs(false);
    std::lock_guard<std::mutex> g(c->graph_mu);
    c->graph_retire.emplace_back(exec, done);
    return SN_OK;
}

// n sweeps of one mesh, launched one by one (the first two fused): a single mesh's sweeps are
// launched from the calling thread (a graph launch holds that thread until
// the replay has nearly finished, so the next call's work would start late)
sn_status sn::run_sweeps_one(sn_ctx *c, const SmoothDesc &sd, int64_t nblocks, int K, hipStream_t s)
{
    const int32_t iters = sd.iters;
    if (iters <= 0 || nblocks <= 0) return SN_OK;
    // sweeps 0 and 1 go in one launch when there are two or more
    const int32_t it0 = iters >= 2 ? 2 : 0;
    if (c->profile_eager) {
        if (it0 == 2) {
            ProfScope ps(c, "k_jacobi", s, 2);
            HIP_TRY(launch_jacobi_first2_one(sd, nblocks, K, s));
        }
        for (int32_t it = it0; it < iters; ++it) {
            ProfScope ps(c, "k_jacobi", s);
            HIP_TRY(launch_jacobi_one(sd, nblocks, it, K, s));
        }
        return SN_OK;
    }
    // one event pair around the launches of the `iters` sweeps
    ProfScope ps(c, "k_jacobi", s, iters);
    if (it0 == 2) HIP_TRY(launch_jacobi_first2_one(sd, nblocks, K, s));
    for (int32_t it = it0; it < iters; ++it) HIP_TRY(launch_jacobi_one(sd, nblocks, it, K, s));
    return SN_OK;
}

extern "C" sn_status sn_triangulate(sn_ctx *c, sn_mesh *m, sn_diag_rule rule, int32_t *tris,
                                    void *tri_labels, void *stream)
{
    if (!c || !m) return fail(SN_EINVAL, "sn_triangulate: NULL argument");
    if (rule < SN_DIAG_FIXED || rule > SN_DIAG_PLANAR) return fail(SN_EINVAL, "sn_triangulate: unknown rule");
    if (m->d.prim == SN_LINES) return fail(SN_EINVAL, "sn_triangulate: an image's contour has no quads");
    if (m->Q > 0 && !tris) return fail(SN_EINVAL, "sn_triangulate: NULL triangle buffer");
    if (m->Q == 0) return SN_OK;
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        ProfScope ps(c, "k_tri_rule", s);
        HIP_TRY(launch_tri_rule((int32_t)rule, m->d.dtype, m->d.quads, m->d.points, m->d.pairs, m->Q,
                                tris, tri_labels, s));
    }
    return mesh_mark(m, s);
}

extern "C" sn_status sn_smooth(sn_ctx *c, sn_mesh *m, const sn_smooth_params *p, void *stream)
{
    if (!c || !m) return fail(SN_EINVAL, "sn_smooth: NULL argument");
    return smooth_one(c, m, p, static_cast<hipStream_t>(stream));
}

sn_status sn::smooth_one(sn_ctx *c, sn_mesh *m, const sn_smooth_params *p, hipStream_t s)
{
    sn_status st = validate_smooth(p);
    if (st != SN_OK) return st;
    HIP_TRY(hipSetDevice(c->device));
    if (m->P == 0) {
        m->final_delta = nullptr;
        return mesh_mark(m, s);
    }
    if (p->iterations > 0) {
        st = ensure_smooth_buffers(m);
        if (st != SN_OK) return st;
    }
    SmoothDesc sd;
    fill_smooth_desc(m, *p, &sd);
    const int K = sweep_chunks(m->P);
    st = run_sweeps_one(c, sd, sweep_blocks_for(m->P, K), K, s);
    if (st != SN_OK) return st;
    // the last sweep `it` wrote buffer (it odd ? da : db)
    m->final_delta = p->iterations == 0 ? nullptr : (((p->iterations - 1) & 1) ? m->da : m->db);
    if (p->iterations == 0 || !m->d.pcell) {  // else the last sweep wrote the points
        ProfScope ps(c, "k_emit", s);
        HIP_TRY(launch_emit_one(m->d, sd, m->ntiles, m->bpw, s));
    }
    return mesh_mark(m, s);
}

// ---------------------------------------------------------------------------
// batched path
// ---------------------------------------------------------------------------

sn_status sn::smooth_many(sn_ctx *c, sn_mesh **ms, const sn_smooth_params *pv, int32_t n,
                          hipStream_t s)
{
    Scratch scr(c);
    int64_t all_points = 0;
    for (int32_t v = 0; v < n; ++v) {
        sn_status st = validate_smooth(&pv[v]);
        if (st != SN_OK) return st;
        if (pv[v].iterations > 0 && ms[v]->P > 0) {
            st = ensure_smooth_buffers(ms[v]);
            if (st != SN_OK) return st;
        }
        all_points += ms[v]->P;
    }
    const int K = sweep_chunks(all_points);
    // meshes in order of descending sweep count: the blocks still sweeping at
    // sweep `it` are then a prefix of the block map, and each sweep launches
    // only those
    auto iters_of = [&](int32_t v) { return ms[v]->P > 0 ? pv[v].iterations : 0; };
    std::vector<int32_t> ord(n);
    for (int32_t v = 0; v < n; ++v) ord[v] = v;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int32_t a, int32_t b) { return iters_of(a) > iters_of(b); });
    std::vector<int64_t> bp(n + 1, 0), tp(n + 1, 0);
    for (int32_t k = 0; k < n; ++k) {
        bp[k + 1] = bp[k] + sweep_blocks_for(ms[ord[k]]->P, K);
        tp[k + 1] = tp[k] + ms[ord[k]]->ntiles;
    }
    const int32_t maxit = n > 0 ? iters_of(ord[0]) : 0;
    std::vector<int64_t> grid(maxit);
    for (int32_t it = 0, k = n; it < maxit; ++it) {
        while (k > 0 && iters_of(ord[k - 1]) <= it) --k;
        grid[it] = bp[k];
    }
    // one upload: smoothing and volume descriptors, sweep-block map, emit tile
    // map and per-mesh emit maps {0, ntiles}
    const size_t up = sizeof(SmoothDesc) * n + sizeof(VolDesc) * n + sizeof(int64_t) * (4 * n + 2);
    uint8_t *h_up = static_cast<uint8_t *>(scr.h(up));
    uint8_t *d_up = static_cast<uint8_t *>(scr.d(up));
    if (!h_up || !d_up) {
        scr.retire(s);
        return fail(SN_ENOMEM, "batch smooth: scratch");
    }
    SmoothDesc *h_sd = reinterpret_cast<SmoothDesc *>(h_up);
    VolDesc *h_vd = reinterpret_cast<VolDesc *>(h_up + sizeof(SmoothDesc) * n);
    int64_t *h_p = reinterpret_cast<int64_t *>(h_up + (sizeof(SmoothDesc) + sizeof(VolDesc)) * n);
    SmoothDesc *d_sd = reinterpret_cast<SmoothDesc *>(d_up);
    VolDesc *d_vd = reinterpret_cast<VolDesc *>(d_up + sizeof(SmoothDesc) * n);
    int64_t *d_p = reinterpret_cast<int64_t *>(d_up + (sizeof(SmoothDesc) + sizeof(VolDesc)) * n);
    bool need_emit = false;
    // the launch's sweep data together decides the non-temporal form
    const bool big = all_points > c->sweep_small_points;
    for (int32_t k = 0; k < n; ++k) {
        sn_mesh *m = ms[ord[k]];
        SmoothDesc &h = h_sd[k];
        fill_smooth_desc(m, pv[ord[k]], &h);
        h.big = big ? 1 : 0;
        h.iters = iters_of(ord[k]);
        need_emit = need_emit || h.iters == 0 || !h.pcell;
        m->final_delta =
            h.iters == 0 ? nullptr : (((h.iters - 1) & 1) ? m->da : m->db);
        h_vd[k] = m->d;
        h_p[2 * (n + 1) + 2 * k] = 0;
        h_p[2 * (n + 1) + 2 * k + 1] = m->ntiles;
    }
    std::memcpy(h_p, bp.data(), sizeof(int64_t) * (n + 1));
    std::memcpy(h_p + n + 1, tp.data(), sizeof(int64_t) * (n + 1));
    // the scratch blocks go back to the pool behind the stream's work, also on failure
    auto device_fail = [&](hipError_t e, const char *what) {
        (void)hipGetLastError();
        scr.retire(s);
        return fail(SN_EDEVICE, std::string("batch smooth: ") + what + ": " + hipGetErrorString(e));
    };
    if (hipError_t e = stage_upload(d_up, h_up, up, s); e != hipSuccess)
        return device_fail(e, "descriptor upload");
    sn_status st = run_sweeps(c, d_sd, d_p, n, grid, K, big, s);
    if (st != SN_OK) {
        scr.retire(s);
        return st;
    }
    bool same_bpw = true;
    for (int32_t v = 1; v < n; ++v) same_bpw &= ms[v]->bpw == ms[0]->bpw;
    if (need_emit) {  // meshes whose last sweep wrote the points skip inside k_emit
        ProfScope ps(c, "k_emit", s);
        if (same_bpw) {
            if (hipError_t e = launch_emit(d_vd, d_sd, d_p + n + 1, n, tp[n], ms[0]->bpw, s); e != hipSuccess)
                return device_fail(e, "k_emit");
        } else {
            for (int32_t k = 0; k < n; ++k)
                if (hipError_t e = launch_emit(d_vd + k, d_sd + k, d_p + 2 * (n + 1) + 2 * k, 1,
                                               ms[ord[k]]->ntiles, ms[ord[k]]->bpw, s);
                    e != hipSuccess)
                    return device_fail(e, "k_emit");
        }
    }
    scr.retire(s);
    return mesh_mark_all(ms, n, s);
}

extern "C" sn_status sn_batch_submit(sn_ctx *c, const sn_volume *vols,
                                     const sn_smooth_params *per_vol, int32_t n, void *stream,
                                     sn_mesh **out)
{
    if (!c || !vols || !out || n < 1) return fail(SN_EINVAL, "sn_batch_submit: bad arguments");
    if (per_vol)
        for (int32_t v = 0; v < n; ++v) {
            sn_status st = validate_smooth(&per_vol[v]);
            if (st != SN_OK) return st;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<sn_mesh *> ms(n, nullptr);
    sn_status st = extract_many(c, vols, n, s, nullptr, ms.data());
    if (st != SN_OK) return st;
    if (per_vol) {
        st = smooth_many(c, ms.data(), per_vol, n, s);
        if (st != SN_OK) {
            for (auto *m : ms) mesh_release(m);
            return st;
        }
    }
    for (int32_t v = 0; v < n; ++v) out[v] = ms[v];
    return SN_OK;
}

// ---------------------------------------------------------------------------
// schedule tuner: time k_count + k_generate for each batches-per-wave candidate
// ---------------------------------------------------------------------------

// Time one extraction of `vol` under schedule `sc`: the best of three after a
// warm-up, wall clock around the call and its completion.
static sn_status time_extract(sn_ctx *c, const sn_volume *vol, hipStream_t s, const Schedule &sc,
                              double *out)
{
    double best = 1e30;
    for (int rep = 0; rep < 4; ++rep) {
        HIP_TRY(hipStreamSynchronize(s));
        const auto t0 = std::chrono::steady_clock::now();
        sn_mesh *m = nullptr;
        const sn_status st = extract_many(c, vol, 1, s, &sc, &m);
        if (st != SN_OK) return st;
        const hipError_t e = hipStreamSynchronize(s);
        const auto t1 = std::chrono::steady_clock::now();
        mesh_release(m);
        if (e != hipSuccess) return fail(SN_EDEVICE, std::string("sn_autotune: ") + hipGetErrorString(e));
        if (rep > 0) best = std::min(best, std::chrono::duration<double>(t1 - t0).count());
    }
    *out = best;
    return SN_OK;
}

// Coordinate descent over the schedule, one knob at a time in the order of
// the passes, each knob's candidates timed with the others at their best so
// far: k_edges segments per wave, the k_count form, k_generate groups per
// wave, and, for a mesh that takes the large-mesh sweep form, the chunk of its
// block order (four sweeps timed per candidate).
extern "C" sn_status sn_autotune(sn_ctx *c, const sn_volume *vol, void *stream, int32_t *chosen)
{
    if (!c || !vol) return fail(SN_EINVAL, "sn_autotune: NULL argument");
    sn_status st = validate_volume(vol);
    if (st != SN_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(c->device));
    // the timed runs record no profiling events; the setting is restored on every return
    struct ProfilingOff {
        sn_ctx *c;
        bool was;
        ~ProfilingOff() { c->profiling = was; }
    } off{c, c->profiling};
    c->profiling = false;
    const std::string cls = size_class(*vol);
    Schedule best;
    {
        std::lock_guard<std::mutex> g(c->tune_mu);
        auto it = c->tune.find(cls);
        if (it != c->tune.end()) best = it->second;
    }
    double tbest = 1e30;
    st = time_extract(c, vol, s, best, &tbest);
    if (st != SN_OK) return st;
    auto knob = [&](int32_t Schedule::*field, std::initializer_list<int32_t> cands) -> sn_status {
        for (int32_t v : cands) {
            if (best.*field == v) continue;
            Schedule sc = best;
            sc.*field = v;
            double t = 0;
            const sn_status e = time_extract(c, vol, s, sc, &t);
            if (e != SN_OK) return e;
            if (t < tbest) tbest = t, best = sc;
        }
        return SN_OK;
    };
    if ((st = knob(&Schedule::edge_segs, {1, 2, 4, 8})) != SN_OK) return st;
    if ((st = knob(&Schedule::count_words, {1, kCountWideV})) != SN_OK) return st;
    if ((st = knob(&Schedule::gen_groups, {1, 2, 3, 4, 8})) != SN_OK) return st;
    // the sweeps' block order, for a mesh in the large-mesh form
    {
        sn_mesh *m = nullptr;
        st = extract_many(c, vol, 1, s, &best, &m);
        if (st != SN_OK) return st;
        if (m->P > c->sweep_small_points && c->sweep_chunk == 0 && m->d.prim != SN_LINES) {
            const sn_smooth_params p{4, 0.5f, 1.0f, SN_BOX};
            SmoothDesc sd;
            fill_smooth_desc(m, p, &sd);
            const int32_t d0 = sd.chunk;  // the default (or the tuned) chunk
            double cbest = 1e30;
            int32_t carg = best.sweep_chunk;
            for (int32_t ch : {d0 / 2, d0, 2 * d0}) {
                if (ch < 1) continue;
                m->sched.sweep_chunk = ch;
                double t = 1e30;
                for (int rep = 0; rep < 3 && st == SN_OK; ++rep) {
                    HIP_TRY(hipStreamSynchronize(s));
                    const auto t0 = std::chrono::steady_clock::now();
                    st = smooth_one(c, m, &p, s);
                    const hipError_t e = hipStreamSynchronize(s);
                    const auto t1 = std::chrono::steady_clock::now();
                    if (st == SN_OK && e != hipSuccess)
                        st = fail(SN_EDEVICE, std::string("sn_autotune: ") + hipGetErrorString(e));
                    if (rep > 0) t = std::min(t, std::chrono::duration<double>(t1 - t0).count());
                }
                if (st != SN_OK) break;
                if (t < cbest) cbest = t, carg = ch == d0 && best.sweep_chunk == 0 ? 0 : ch;
            }
            best.sweep_chunk = carg;
        }
        mesh_release(m);
        if (st != SN_OK) return st;
    }
    {
        std::lock_guard<std::mutex> g(c->tune_mu);
        c->tune[cls] = best;
        c->save_tune_cache();
    }
    if (chosen) *chosen = best.gen_groups;
    return SN_OK;
}

extern "C" sn_status sn_schedule_get(sn_ctx *c, const sn_volume *vol, sn_schedule *out)
{
    if (!c || !vol || !out) return fail(SN_EINVAL, "sn_schedule_get: NULL argument");
    sn_status st = validate_volume(vol);
    if (st != SN_OK) return st;
    const Schedule sc = c->schedule(size_class(*vol));
    out->gen_groups = sc.gen_groups;
    out->count_words = sc.count_words;
    out->edge_segments = sc.edge_segs;
    out->sweep_chunk = sc.sweep_chunk;
    return SN_OK;
}

extern "C" sn_status sn_schedule_set(sn_ctx *c, const sn_volume *vol, const sn_schedule *in)
{
    if (!c || !vol || !in) return fail(SN_EINVAL, "sn_schedule_set: NULL argument");
    sn_status st = validate_volume(vol);
    if (st != SN_OK) return st;
    Schedule sc;
    sc.gen_groups = in->gen_groups;
    sc.count_words = in->count_words;
    sc.edge_segs = in->edge_segments;
    sc.sweep_chunk = in->sweep_chunk;
    if (!valid_schedule(sc)) return fail(SN_EINVAL, "sn_schedule_set: value out of range");
    std::lock_guard<std::mutex> g(c->tune_mu);
    c->tune[size_class(*vol)] = sc;
    return SN_OK;
}

extern "C" sn_status sn_set_batches_per_wave(sn_ctx *c, int32_t bpw)
{
    if (!c || bpw < 0 || bpw > kMaxBatchesPerWave)
        return fail(SN_EINVAL, "sn_set_batches_per_wave: bad arguments");
    std::lock_guard<std::mutex> g(c->tune_mu);
    c->forced_bpw = bpw;
    return SN_OK;
}
