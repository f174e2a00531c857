// Serving loop with continuous batching for the deform-then-splat render.
//
// A request is (scene, camera, t, output image).  Scenes (canonical
// Gaussians, HexPlane planes, decoder weights) are copied once into
// server-owned HBM and stay resident.  Per request the server needs a
// buffer set: the deformed Gaussians and a render workspace sized for the
// scene, the frame size and an instance capacity learned per (scene, frame
// size).  Buffer sets are kept after use and handed to the next request of
// the same class, so the render graph captured on a set is replayed with
// only the frame descriptor changed.
//
// Scheduling (one executor thread):
//   - requests wait in a FIFO; the head is admitted when a slot is free and
//     its buffer set can be had within the memory budget (a kept set of the
//     same class, or a new one, evicting kept sets of other classes); a head
//     that does not fit blocks the ones behind it, so nothing starves;
//   - the requests admitted in one round are deformed together: one batched
//     launch per shape class (up to G4D_MAX_BATCH_JOBS jobs) on a deform
//     stream, followed on each request's slot stream (after an event wait)
//     by its render, as a graph replay when its set has been captured;
//   - completion is observed by polling per-slot events; the device status
//     copied behind the render says whether the instance capacity sufficed,
//     otherwise the class capacity grows and the request re-enters the head
//     of the queue with a larger set.
// Requests that arrive while others run are admitted as slots and memory
// free up; their work overlaps on the device through the slot streams.
#include "g4d_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

namespace g4d {
namespace serve {

double wall_now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Percentile by linear interpolation between order statistics.
double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q / 100.0 * (double)(v.size() - 1);
    const size_t lo = (size_t)pos;
    const size_t hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

// ------------------------------------------------------------------ core

using ClassKey = std::tuple<int, int, int>;   // (scene / class id, width, height)

struct BufferSet {
    ClassKey key{};
    int64_t capacity = 0;
    size_t bytes = 0;
    double last_use = 0.0;
    // device part (unused by the simulator)
    void *mem = nullptr;
    g4d_workspace ws{};
    g4d_splats splats{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t frame_node = nullptr;
};

struct Req {
    uint64_t ticket = 0;
    int index = 0;              // simulator: trace index
    ClassKey key{};
    int shape = 0;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    bool done = false;
    int status = G4D_OK;
    int slot = -1;
    BufferSet *bufs = nullptr;
    int retries = 0;
    // device payload
    g4d_camera cam{};
    float t = 0.0f;
    float *out = nullptr;
    // simulator payload
    double remaining = 0.0;
    size_t sim_bytes = 0;
};

// Memory accounting of buffer sets against the budget: in use + kept <= budget.
class Pool {
  public:
    template <typename AllocFn, typename FreeFn>
    BufferSet *acquire(const ClassKey &key, int64_t capacity, size_t bytes, double now, AllocFn alloc,
                       FreeFn free_fn, bool *reused) {
        *reused = false;
        for (size_t i = 0; i < kept_.size(); ++i) {
            BufferSet *b = kept_[i];
            if (b->key == key && b->capacity >= capacity) {
                kept_.erase(kept_.begin() + (long)i);
                b->last_use = now;
                *reused = true;
                return b;
            }
        }
        // evict kept sets (least recently used first) until the new one fits
        while (held_ + bytes > budget_ && !kept_.empty()) {
            auto it = std::min_element(kept_.begin(), kept_.end(),
                                       [](BufferSet *a, BufferSet *b) { return a->last_use < b->last_use; });
            BufferSet *v = *it;
            kept_.erase(it);
            held_ -= v->bytes;
            free_fn(v);
            delete v;
        }
        if (held_ + bytes > budget_) return nullptr;
        auto *b = new BufferSet();
        b->key = key;
        b->capacity = capacity;
        b->bytes = bytes;
        b->last_use = now;
        if (!alloc(b)) {
            delete b;
            return nullptr;
        }
        held_ += bytes;
        peak_ = std::max(peak_, held_);
        return b;
    }
    void release(BufferSet *b, double now) {
        b->last_use = now;
        kept_.push_back(b);
    }
    template <typename FreeFn>
    void drop(BufferSet *b, FreeFn free_fn) {
        held_ -= b->bytes;
        free_fn(b);
        delete b;
    }
    template <typename FreeFn>
    void clear(FreeFn free_fn) {
        for (BufferSet *b : kept_) {
            held_ -= b->bytes;
            free_fn(b);
            delete b;
        }
        kept_.clear();
    }
    size_t budget_ = 0, held_ = 0, peak_ = 0;
    std::vector<BufferSet *> kept_;
};

struct Stats {
    std::vector<double> lat_ms;
    double first_submit = -1.0, last_done = 0.0;
    int64_t submitted = 0, completed = 0, rejected = 0, batched_launches = 0, graph_replays = 0,
            eager_renders = 0, overflow_retries = 0, buffer_reuses = 0;
    void reset() { *this = Stats(); }
};

// ------------------------------------------------------------- device server

struct Scene {
    int n = 0, sh_degree = 0;
    g4d_gaussians G{};
    g4d_planes P{};
    g4d_mlp M{};
    std::vector<void *> allocs;
};

}  // namespace serve
}  // namespace g4d

struct g4d_server {
    g4d_server_config cfg{};
    std::vector<std::unique_ptr<g4d::serve::Scene>> scenes;
    std::map<g4d::serve::ClassKey, int64_t> class_capacity;
    g4d::serve::Pool pool;
    g4d::serve::Stats stats;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<g4d::serve::Req *> pending;
    std::vector<g4d::serve::Req *> inflight;
    std::map<uint64_t, std::unique_ptr<g4d::serve::Req>> reqs;
    std::vector<int> free_slots;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::atomic<uint64_t> submit_count{0};   // requests submitted (read by the idle worker's poll)
    std::atomic<bool> stop_flag{false};
    std::thread worker;
    // device objects
    int device = 0;
    std::vector<hipStream_t> slot_stream;
    std::vector<hipEvent_t> slot_done;
    std::vector<hipEvent_t> round_events;
    size_t round_event_next = 0;
    g4d::DevStatus *status_host = nullptr;   // pinned, one per slot
    int hip_error = 0;
};

namespace g4d {
namespace serve {

namespace {

// Per-frame Gaussians of a scene: means, scales, quats, opacity, and the
// deformed SH coefficients when the decoder has a colour head.
int colour_rows(const Scene &sc) { return sc.M.wc ? 3 * (sc.sh_degree + 1) * (sc.sh_degree + 1) : 0; }
size_t splat_bytes(const Scene &sc) {
    return align_up((size_t)sc.n * (11 + colour_rows(sc)) * sizeof(float), 256);
}

int64_t initial_capacity(const g4d_server *S, int scene, int w, int h) {
    const int n = S->scenes[scene]->n;
    const double f = S->cfg.instance_factor > 0 ? S->cfg.instance_factor : 64.0;
    const int tiles = ((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile);
    int64_t c = (int64_t)(f * n) + 4096;
    c = std::min<int64_t>(c, (int64_t)n * tiles + 4096);
    return std::min<int64_t>(c, (int64_t(1) << 30) - 1);
}

size_t set_bytes(const g4d_server *S, int scene, int w, int h, int64_t cap) {
    const int n = S->scenes[scene]->n;
    return splat_bytes(*S->scenes[scene]) + g4d_render_workspace_bytes(std::max(n, 1), w, h, cap) + 256;
}

bool dev_alloc(g4d_server *S, BufferSet *b) {
    const int scene = std::get<0>(b->key), w = std::get<1>(b->key), h = std::get<2>(b->key);
    const Scene &sc = *S->scenes[scene];
    if (hipMalloc(&b->mem, b->bytes) != hipSuccess) {
        (void)hipGetLastError();
        b->mem = nullptr;
        return false;
    }
    char *base = static_cast<char *>(b->mem);
    float *f = reinterpret_cast<float *>(base);
    const int n = sc.n;
    b->splats.n = n;
    b->splats.sh_degree = sc.sh_degree;
    b->splats.means = f;
    b->splats.scales = f + 3 * (size_t)n;
    b->splats.quats = f + 6 * (size_t)n;
    b->splats.opacity = f + 10 * (size_t)n;
    b->splats.sh = colour_rows(sc) ? f + 11 * (size_t)n : const_cast<float *>(sc.G.sh);
    char *wsp = base + splat_bytes(sc);
    wsp = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(wsp), 256));
    b->ws.ptr = wsp;
    b->ws.bytes = g4d_render_workspace_bytes(std::max(n, 1), w, h, b->capacity);
    b->ws.n_max = std::max(n, 1);
    b->ws.width_max = w;
    b->ws.height_max = h;
    b->ws.instance_capacity = b->capacity;
    return true;
}

void dev_free(BufferSet *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->mem) (void)hipFree(b->mem);
    b->exec = nullptr;
    b->graph = nullptr;
    b->mem = nullptr;
}

hipEvent_t next_round_event(g4d_server *S) {
    if (S->round_events.empty()) {
        S->round_events.resize(64);
        for (auto &e : S->round_events) (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    }
    hipEvent_t e = S->round_events[S->round_event_next % S->round_events.size()];
    ++S->round_event_next;
    return e;
}

// Launch deform + render for the requests admitted in one round.  A request
// that has the device to itself (nothing else in flight or queued) renders
// with direct launches, which start the device soonest; requests that
// overlap others replay their captured graphs, which take the worker thread
// one call per render instead of one per kernel.
void launch_round(g4d_server *S, std::vector<Req *> &batch, bool busy) {
    const bool batched = S->cfg.batch_deform != 0;
    if (batched) {
        // one batched launch per shape class, chunks of G4D_MAX_BATCH_JOBS,
        // on the slot stream of the chunk's first request (no stream hop for
        // it: a lone request runs deform and render back to back on its
        // stream); the chunk's other requests wait for it with an event
        std::map<int, std::vector<Req *>> by_shape;
        for (Req *r : batch) by_shape[r->shape].push_back(r);
        for (auto &kv : by_shape) {
            auto &v = kv.second;
            for (size_t i = 0; i < v.size(); i += G4D_MAX_BATCH_JOBS) {
                const size_t m = std::min<size_t>(G4D_MAX_BATCH_JOBS, v.size() - i);
                g4d_deform_job jobs[G4D_MAX_BATCH_JOBS];
                for (size_t q = 0; q < m; ++q) {
                    Req *r = v[i + q];
                    const Scene &sc = *S->scenes[std::get<0>(r->key)];
                    jobs[q] = g4d_deform_job{&sc.G, &sc.P, &sc.M, r->t, &r->bufs->splats};
                }
                hipStream_t ds = S->slot_stream[v[i]->slot];
                const g4d_status st = deform_batched(jobs, (int)m, ds);
                if (st != G4D_OK) {
                    for (size_t q = 0; q < m; ++q) v[i + q]->status = st;
                }
                ++S->stats.batched_launches;
                if (m > 1) {
                    hipEvent_t ev = next_round_event(S);
                    (void)hipEventRecord(ev, ds);
                    for (size_t q = 1; q < m; ++q) (void)hipStreamWaitEvent(S->slot_stream[v[i + q]->slot], ev, 0);
                }
            }
        }
    }
    for (Req *r : batch) {
        hipStream_t s = S->slot_stream[r->slot];
        const Scene &sc = *S->scenes[std::get<0>(r->key)];
        BufferSet *b = r->bufs;
        if (!batched) {
            g4d_deform_job job{&sc.G, &sc.P, &sc.M, r->t, &b->splats};
            const g4d_status st = deform_batched(&job, 1, s);
            if (st != G4D_OK) r->status = st;
        }
        if (r->status == G4D_OK) {
            g4d_status st = G4D_OK;
            if (S->cfg.use_graphs && busy) {
                if (!b->exec) {
                    hipGraph_t g = nullptr;
                    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
                        st = G4D_EHIP;
                    } else {
                        st = render(&b->splats, &r->cam, &b->ws, r->out, nullptr, nullptr, s);
                        if (hipStreamEndCapture(s, &g) != hipSuccess) st = G4D_EHIP;
                        if (st == G4D_OK && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
                            st = G4D_EHIP;
                        if (st == G4D_OK) st = graph_find_camera_node(g, &b->frame_node);
                        b->graph = g;
                    }
                } else {
                    st = graph_set_frame(b->exec, b->frame_node, &b->ws, &r->cam, r->out, nullptr, nullptr);
                }
                if (st == G4D_OK && hipGraphLaunch(b->exec, s) != hipSuccess) st = G4D_EHIP;
                if (st == G4D_OK) ++S->stats.graph_replays;
            } else {
                st = render(&b->splats, &r->cam, &b->ws, r->out, nullptr, nullptr, s);
                ++S->stats.eager_renders;
            }
            if (st != G4D_OK) {
                (void)hipGetLastError();
                r->status = st;
            }
        }
        const size_t off = status_offset(&b->ws);
        (void)hipMemcpyAsync(&S->status_host[r->slot], static_cast<char *>(b->ws.ptr) + off, sizeof(DevStatus),
                             hipMemcpyDeviceToHost, s);
        (void)hipEventRecord(S->slot_done[r->slot], s);
    }
}

constexpr int kIdleSpinUs = 2000;   // idle worker: polling window before it sleeps

void worker_loop(g4d_server *S) {
    (void)hipSetDevice(S->device);
    std::vector<Req *> batch;
    while (true) {
        batch.clear();
        bool idle = false, busy = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // completions
            for (size_t i = 0; i < S->inflight.size();) {
                Req *r = S->inflight[i];
                if (hipEventQuery(S->slot_done[r->slot]) != hipSuccess) {
                    ++i;
                    continue;
                }
                const DevStatus &ds = S->status_host[r->slot];
                const double now = wall_now();
                S->inflight.erase(S->inflight.begin() + (long)i);
                S->free_slots.push_back(r->slot);
                r->slot = -1;
                if (r->status == G4D_OK && ds.overflow) {
                    // grow the class capacity and retry at the head of the queue
                    int64_t &cap = S->class_capacity[r->key];
                    cap = std::max<int64_t>(cap, (int64_t)((double)ds.k_total * 1.25) + 4096);
                    cap = std::min<int64_t>(cap, (int64_t(1) << 30) - 1);
                    S->pool.drop(r->bufs, dev_free);
                    r->bufs = nullptr;
                    ++r->retries;
                    ++S->stats.overflow_retries;
                    S->pending.push_front(r);
                    continue;
                }
                if (r->status == G4D_OK && ds.sort_error) r->status = G4D_EDEVICE;
                if (r->status == G4D_OK) {
                    // remember what the class needed, with headroom
                    int64_t &cap = S->class_capacity[r->key];
                    const int64_t want = (int64_t)((double)ds.k_total * 1.15) + 4096;
                    if (want > cap) cap = std::min<int64_t>(want, (int64_t(1) << 30) - 1);
                }
                S->pool.release(r->bufs, now);
                r->bufs = nullptr;
                r->t_done = now;
                r->done = true;
                if (r->status == G4D_OK) {
                    S->stats.lat_ms.push_back(1e3 * (r->t_done - r->t_submit));
                    S->stats.last_done = std::max(S->stats.last_done, now);
                    ++S->stats.completed;
                }
                S->cv_done.notify_all();
            }
            // admission (FIFO; the head blocks the queue when it does not fit)
            while (!S->pending.empty() && !S->free_slots.empty()) {
                Req *r = S->pending.front();
                const int scene = std::get<0>(r->key), w = std::get<1>(r->key), h = std::get<2>(r->key);
                int64_t &cap = S->class_capacity[r->key];
                if (cap == 0) cap = initial_capacity(S, scene, w, h);
                const size_t bytes = set_bytes(S, scene, w, h, cap);
                if (bytes > S->cfg.hbm_budget) {
                    S->pending.pop_front();
                    r->status = G4D_ENOMEM;
                    r->done = true;
                    ++S->stats.rejected;
                    S->cv_done.notify_all();
                    continue;
                }
                bool reused = false;
                BufferSet *b = S->pool.acquire(
                    r->key, cap, bytes, wall_now(), [&](BufferSet *x) { return dev_alloc(S, x); }, dev_free,
                    &reused);
                if (!b) break;
                if (reused) ++S->stats.buffer_reuses;
                S->pending.pop_front();
                r->bufs = b;
                r->slot = S->free_slots.back();
                S->free_slots.pop_back();
                r->t_admit = wall_now();
                S->inflight.push_back(r);
                batch.push_back(r);
            }
            busy = batch.size() > 1 || S->inflight.size() > batch.size() || !S->pending.empty();
            if (S->stop && S->pending.empty() && S->inflight.empty() && batch.empty()) break;
            idle = batch.empty() && S->inflight.empty() && S->pending.empty();
            if (idle) {
                // poll for a new request for a while before sleeping: a thread
                // woken from a condition variable starts tens of microseconds
                // late, which an arrival at an idle device would pay in full
                const uint64_t seen = S->submit_count.load(std::memory_order_acquire);
                const auto spin_end = std::chrono::steady_clock::now() + std::chrono::microseconds(kIdleSpinUs);
                lk.unlock();
                while (S->submit_count.load(std::memory_order_acquire) == seen && !S->stop_flag.load() &&
                       std::chrono::steady_clock::now() < spin_end)
                    std::this_thread::yield();
                lk.lock();
                if (S->pending.empty() && !S->stop) S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
        }
        if (!batch.empty()) launch_round(S, batch, busy);
        else std::this_thread::yield();
    }
}

g4d_status copy_dev(Scene &sc, const void *src, size_t bytes, void **dst) {
    *dst = nullptr;
    if (bytes == 0) return G4D_OK;
    if (!src) return G4D_EINVAL;
    G4D_HIP_CHECK(hipMalloc(dst, bytes));
    sc.allocs.push_back(*dst);
    G4D_HIP_CHECK(hipMemcpy(*dst, src, bytes, hipMemcpyDeviceToDevice));
    return G4D_OK;
}

}  // namespace
}  // namespace serve
}  // namespace g4d

using namespace g4d::serve;

extern "C" g4d_status g4d_server_create(const g4d_server_config *cfg, g4d_server **out) {
    if (!cfg || !out || cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->hbm_budget == 0) return G4D_EINVAL;
    auto *S = new g4d_server();
    S->cfg = *cfg;
    S->pool.budget_ = cfg->hbm_budget;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return G4D_EHIP;
    }
    hipError_t e = hipSuccess;
    S->slot_stream.resize(cfg->max_slots);
    S->slot_done.resize(cfg->max_slots);
    for (int i = 0; i < cfg->max_slots && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&S->slot_stream[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->slot_done[i], hipEventDisableTiming);
        S->free_slots.push_back(cfg->max_slots - 1 - i);
    }
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&S->status_host), sizeof(g4d::DevStatus) * cfg->max_slots,
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        g4d::set_hip_error(e);
        delete S;
        return G4D_EHIP;
    }
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return G4D_OK;
}

extern "C" g4d_status g4d_server_add_scene(g4d_server *S, const g4d_gaussians *G, const g4d_planes *P,
                                           const g4d_mlp *M, int32_t *scene_id) {
    if (!S || !G || !P || !M || !scene_id || G->n < 1 || G->sh_degree < 0 || G->sh_degree > 3) return G4D_EINVAL;
    if (M->in_dim != P->feat * P->n_scales || P->n_scales < 1 || P->n_scales > 3) return G4D_EINVAL;
    if ((M->wc == nullptr) != (M->bc == nullptr) || (M->wa == nullptr) != (M->ba == nullptr)) return G4D_EINVAL;
    auto sc = std::make_unique<Scene>();
    sc->n = G->n;
    sc->sh_degree = G->sh_degree;
    const size_t n = (size_t)G->n;
    const size_t nsh = (size_t)(G->sh_degree + 1) * (G->sh_degree + 1) * 3 * n;
    void *p = nullptr;
    sc->G.n = G->n;
    sc->G.sh_degree = G->sh_degree;
    g4d_status st;
#define G4D_COPY(dst, src, bytes)                                      \
    st = copy_dev(*sc, src, bytes, &p);                                \
    if (st != G4D_OK) {                                                \
        for (void *a : sc->allocs) (void)hipFree(a);                   \
        return st;                                                     \
    }                                                                  \
    dst = static_cast<typename std::remove_reference<decltype(dst)>::type>(p);
    G4D_COPY(sc->G.means, G->means, 3 * n * 4);
    G4D_COPY(sc->G.log_scales, G->log_scales, 3 * n * 4);
    G4D_COPY(sc->G.quats, G->quats, 4 * n * 4);
    G4D_COPY(sc->G.opacity_logits, G->opacity_logits, n * 4);
    G4D_COPY(sc->G.sh, G->sh, nsh * 4);
    sc->P = *P;
    for (int l = 0; l < P->n_scales; ++l)
        for (int q = 0; q < 6; ++q) {
            static const int ax[6][2] = {{0, 1}, {0, 2}, {1, 2}, {0, 3}, {1, 3}, {2, 3}};
            const size_t elems = (size_t)P->res[l][ax[q][0]] * P->res[l][ax[q][1]] * P->feat;
            G4D_COPY(sc->P.plane[l][q], P->plane[l][q], elems * 4);
        }
    sc->M = *M;
    const size_t hd = (size_t)M->hidden, in = (size_t)M->in_dim;
    G4D_COPY(sc->M.w1, M->w1, hd * in * 4);
    G4D_COPY(sc->M.b1, M->b1, hd * 4);
    G4D_COPY(sc->M.wx, M->wx, 3 * hd * 4);
    G4D_COPY(sc->M.bx, M->bx, 3 * 4);
    G4D_COPY(sc->M.wr, M->wr, 4 * hd * 4);
    G4D_COPY(sc->M.br, M->br, 4 * 4);
    G4D_COPY(sc->M.ws, M->ws, 3 * hd * 4);
    G4D_COPY(sc->M.bs, M->bs, 3 * 4);
    if (M->wc) {
        const size_t rows = 3 * (size_t)(G->sh_degree + 1) * (G->sh_degree + 1);
        G4D_COPY(sc->M.wc, M->wc, rows * hd * 4);
        G4D_COPY(sc->M.bc, M->bc, rows * 4);
    }
    if (M->wa) {
        G4D_COPY(sc->M.wa, M->wa, hd * 4);
        G4D_COPY(sc->M.ba, M->ba, 4);
    }
#undef G4D_COPY
    std::lock_guard<std::mutex> lk(S->mu);
    *scene_id = (int32_t)S->scenes.size();
    S->scenes.push_back(std::move(sc));
    return G4D_OK;
}

extern "C" g4d_status g4d_server_submit(g4d_server *S, int32_t scene_id, const g4d_camera *cam, float t,
                                        float *out_image, uint64_t *ticket) {
    if (!S || !cam || !out_image || !ticket) return G4D_EINVAL;
    if (!(t >= 0.0f && t <= 1.0f)) return G4D_EINVAL;
    if (cam->width < 1 || cam->height < 1 || cam->width > S->cfg.max_width || cam->height > S->cfg.max_height)
        return G4D_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (scene_id < 0 || scene_id >= (int32_t)S->scenes.size()) return G4D_ENOTFOUND;
    auto r = std::make_unique<Req>();
    r->ticket = S->next_ticket++;
    r->key = ClassKey{scene_id, cam->width, cam->height};
    const Scene &sc = *S->scenes[scene_id];
    // deform shape class: the kernel variant (head tiles: 1 for up to 16 head rows, else 4)
    const int head_tiles = 10 + colour_rows(sc) + (sc.M.wa ? 1 : 0) <= 16 ? 1 : 4;
    r->shape = sc.P.feat * 1000000 + sc.P.n_scales * 10000 + sc.M.hidden * 10 + sc.M.precision + 2 * head_tiles;
    r->cam = *cam;
    r->t = t;
    r->out = out_image;
    r->t_submit = wall_now();
    if (S->stats.first_submit < 0) S->stats.first_submit = r->t_submit;
    ++S->stats.submitted;
    *ticket = r->ticket;
    S->pending.push_back(r.get());
    S->submit_count.fetch_add(1, std::memory_order_release);
    S->reqs[r->ticket] = std::move(r);
    S->cv_work.notify_one();
    return G4D_OK;
}

extern "C" g4d_status g4d_server_wait(g4d_server *S, uint64_t ticket, double *latency_ms) {
    if (!S) return G4D_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return G4D_ENOTFOUND;
    Req *r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->done; });
    const int st = r->status;
    if (latency_ms) *latency_ms = 1e3 * (r->t_done - r->t_submit);
    S->reqs.erase(it);
    return (g4d_status)st;
}

extern "C" g4d_status g4d_server_drain(g4d_server *S) {
    if (!S) return G4D_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->pending.empty() && S->inflight.empty(); });
    return G4D_OK;
}

extern "C" g4d_status g4d_server_stats_get(g4d_server *S, g4d_server_stats *out) {
    if (!S || !out) return G4D_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    const Stats &st = S->stats;
    *out = g4d_server_stats{};
    out->submitted = st.submitted;
    out->completed = st.completed;
    out->rejected = st.rejected;
    out->p50_ms = percentile(st.lat_ms, 50.0);
    out->p99_ms = percentile(st.lat_ms, 99.0);
    double sum = 0.0, mx = 0.0;
    for (double v : st.lat_ms) {
        sum += v;
        mx = std::max(mx, v);
    }
    out->mean_ms = st.lat_ms.empty() ? 0.0 : sum / (double)st.lat_ms.size();
    out->max_ms = mx;
    out->wall_s = st.first_submit >= 0 && st.last_done > st.first_submit ? st.last_done - st.first_submit : 0.0;
    out->frames_per_s = out->wall_s > 0 ? (double)st.completed / out->wall_s : 0.0;
    out->batched_launches = st.batched_launches;
    out->graph_replays = st.graph_replays;
    out->eager_renders = st.eager_renders;
    out->overflow_retries = st.overflow_retries;
    out->peak_bytes = S->pool.peak_;
    return G4D_OK;
}

extern "C" g4d_status g4d_server_reset_stats(g4d_server *S) {
    if (!S) return G4D_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.reset();
    S->pool.peak_ = S->pool.held_;
    return G4D_OK;
}

extern "C" g4d_status g4d_server_destroy(g4d_server *S) {
    if (!S) return G4D_EINVAL;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->pending.empty() && S->inflight.empty(); });
        S->stop = true;
        S->stop_flag.store(true);
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    (void)hipDeviceSynchronize();
    S->pool.clear(dev_free);
    for (auto &sc : S->scenes)
        for (void *a : sc->allocs) (void)hipFree(a);
    for (auto &e : S->round_events) (void)hipEventDestroy(e);
    for (size_t i = 0; i < S->slot_stream.size(); ++i) {
        if (S->slot_done[i]) (void)hipEventDestroy(S->slot_done[i]);
        if (S->slot_stream[i]) (void)hipStreamDestroy(S->slot_stream[i]);
    }
    if (S->status_host) (void)hipHostFree(S->status_host);
    delete S;
    return G4D_OK;
}

// ------------------------------------------------------------- simulation

extern "C" g4d_status g4d_server_simulate(const g4d_sim_config *cfg, g4d_sim_result *out) {
    if (!cfg || !out || cfg->n_requests < 0 || cfg->max_slots < 1 || cfg->hbm_budget == 0) return G4D_EINVAL;
    const int n = cfg->n_requests;
    if (n > 0 && (!cfg->arrival_s || !cfg->service_s || !cfg->bytes || !cfg->class_id || !cfg->shape_class))
        return G4D_EINVAL;
    for (int i = 1; i < n; ++i)
        if (cfg->arrival_s[i] < cfg->arrival_s[i - 1]) return G4D_EINVAL;
    const double ov = std::min(1.0, std::max(0.0, cfg->overlap));
    Pool pool;
    pool.budget_ = cfg->hbm_budget;
    std::vector<Req> reqs(n);
    std::deque<Req *> pending;
    std::vector<Req *> inflight;
    int free_slots = cfg->max_slots, max_in_flight = 0, admitted_count = 0;
    int64_t launches = 0, reuses = 0;
    int32_t rejected = 0;
    double now = 0.0;
    int next = 0;
    std::vector<double> lat;
    auto no_alloc = [](BufferSet *) { return true; };
    auto no_free = [](BufferSet *) {};
    while (next < n || !pending.empty() || !inflight.empty()) {
        // admission round at the current time
        std::map<int, int> round_shapes;
        while (!pending.empty() && free_slots > 0) {
            Req *r = pending.front();
            if (r->sim_bytes > cfg->hbm_budget) {
                pending.pop_front();
                r->done = true;
                r->status = G4D_ENOMEM;
                ++rejected;
                continue;
            }
            bool reused = false;
            BufferSet *b = pool.acquire(ClassKey{cfg->class_id[r->index], 0, 0}, 0, r->sim_bytes, now, no_alloc,
                                        no_free, &reused);
            if (!b) break;
            if (reused) ++reuses;
            pending.pop_front();
            r->bufs = b;
            r->t_admit = now;
            --free_slots;
            inflight.push_back(r);
            if (out->admit_order) out->admit_order[admitted_count] = r->index;
            ++admitted_count;
            round_shapes[cfg->shape_class[r->index]]++;
        }
        for (auto &kv : round_shapes)
            launches += cfg->batch_deform ? (kv.second + G4D_MAX_BATCH_JOBS - 1) / G4D_MAX_BATCH_JOBS : kv.second;
        max_in_flight = std::max(max_in_flight, (int)inflight.size());
        // next event: an arrival or the earliest completion under processor sharing
        const int m = (int)inflight.size();
        const double rate = m > 0 ? (1.0 + ov * (m - 1)) / m : 0.0;
        double t_comp = 1e300;
        Req *first = nullptr;
        for (Req *r : inflight) {
            const double tc = now + r->remaining / rate;
            if (tc < t_comp) {
                t_comp = tc;
                first = r;
            }
        }
        const double t_arr = next < n ? cfg->arrival_s[next] : 1e300;
        const double t_next = std::min(t_comp, t_arr);
        if (t_next >= 1e299) break;   // nothing can progress (cannot happen with a positive budget)
        for (Req *r : inflight) r->remaining -= rate * (t_next - now);
        now = t_next;
        if (t_comp <= t_arr && first) {
            first->remaining = 0.0;
            first->done = true;
            first->t_done = now;
            inflight.erase(std::find(inflight.begin(), inflight.end(), first));
            pool.release(first->bufs, now);
            first->bufs = nullptr;
            ++free_slots;
        } else {
            // every request that has arrived by now joins the queue before the
            // next admission round
            while (next < n && cfg->arrival_s[next] <= now) {
                Req &r = reqs[next];
                r.index = next;
                r.t_submit = cfg->arrival_s[next];
                r.remaining = std::max(0.0, cfg->service_s[next]);
                r.sim_bytes = cfg->bytes[next];
                pending.push_back(&r);
                ++next;
            }
        }
    }
    pool.clear(no_free);
    double sum = 0.0, mx = 0.0, makespan = 0.0;
    for (int i = 0; i < n; ++i) {
        const Req &r = reqs[i];
        const double l = (r.done && r.status == G4D_OK) ? 1e3 * (r.t_done - r.t_submit) : -1.0;
        if (out->latency_ms) out->latency_ms[i] = l;
        if (l >= 0) {
            lat.push_back(l);
            sum += l;
            mx = std::max(mx, l);
            makespan = std::max(makespan, r.t_done);
        }
    }
    out->p50_ms = percentile(lat, 50.0);
    out->p99_ms = percentile(lat, 99.0);
    out->mean_ms = lat.empty() ? 0.0 : sum / (double)lat.size();
    out->max_ms = mx;
    out->makespan_s = makespan;
    out->peak_bytes = pool.peak_;
    out->max_in_flight = max_in_flight;
    out->rejected = rejected;
    out->batched_launches = launches;
    out->buffer_reuses = reuses;
    return G4D_OK;
}
