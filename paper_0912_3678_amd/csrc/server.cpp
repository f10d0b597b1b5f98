// Request scheduler for serving: continuous batching of factor-and-solve
// requests of uneven size under a device-memory budget, with a cache of
// resident factors for requests that bring a new right-hand side for a
// matrix already factored.
//
// Admission is continuous: at every submit / poll / wait the scheduler
// retires the requests whose completion event has fired (their memory goes
// back to the budget unless the factor is kept), then admits waiting
// requests in arrival order while the budget and the in-flight limit allow,
// evicting least recently used resident factors that no queued or running
// request needs.  Admitted requests run on a small set of streams, so the
// work of requests that arrived while others were running overlaps on the
// device.  All requests on one resident factor run on that factor's stream
// (they share its workspace).  Nothing here waits on the host for device
// work except pf_server_wait.
//
// Request memory comes from one device allocation made at start-up
// (pf_server_reserve), carved by a sub-allocator of the server's own, so no
// request's allocation reaches the driver; what does not fit there comes
// from a memory pool of the server's own whose release threshold is the
// budget (what retired requests give back stays mapped for the next ones).
#include "pf.h"
#include "pf_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <vector>

using namespace pf;

namespace {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Ticket {
    pf_request req{};
    size_t bytes = 0;          // budget charged while running
    int stream = -1;
    int state = 0;             // 0 queued, 1 running, 2 done
    pf_info info{};
    double t_submit = 0, t_start = -1, t_done = -1;   // ms, server clock
    hipEvent_t ev_start = nullptr, ev_done = nullptr;
    hipEvent_t ev_ready = nullptr;   // inputs ready (recorded on req.after at submission)
    pf_factor_t F = nullptr;   // the factor this request ran on
    // PF_FP32_IR: refinement driven from the scheduler's polling -- each
    // step's residual norms arrive in pinned host words (ev_norms), and the
    // next step is queued only when they say so; no host wait
    bool ir = false;
    int iters = 0, slow = 0;
    double eta = INFINITY, prev = INFINITY;
    unsigned long long *hnorms = nullptr;   // 3 nrhs + 1 pinned words (a server slot)
    size_t hcap = 0;                        // the slot's words
    hipEvent_t ev_norms = nullptr;
};

struct Resident {
    pf_factor_t F = nullptr;   // null until the request that factors it starts
    size_t bytes = 0;
    int stream = 0;
    int users = 0;             // queued or running requests on it (its own included)
    double last_use = 0;
    bool released = false;
    int failed = 0;            // status of a factoring request that could not start
    bool refining = false;     // a request on it is between refinement steps: the
                               // residual and correction workspace is taken
};

}  // namespace

// One device allocation carved for the requests (pf_server_reserve): free
// ranges by offset, coalesced; a range freed on a stream is pending until an
// event recorded behind the free has fired, and is handed out before that
// only to a stream told to wait for the event -- nothing here waits on the
// host, and no request's allocation reaches the driver.
struct Slab {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free;   // offset -> bytes
    struct Pending {
        size_t off, bytes;
        hipEvent_t ev;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;   // events to record frees with
};

struct pf_server_s {
    size_t budget = 0, used = 0;
    Slab slab;                       // reserved memory (pf_server_reserve)
    hipMemPool_t pool = nullptr;     // other factor memory (release threshold = budget)
    Allocator al;                    // hands the pool to new handles
    double setup_ms_max = 0, setup_ms_total = 0;     // host: handle set-up + allocation
    double launch_ms_max = 0, launch_ms_total = 0;   // host: a request's whole launch
    pf_opts opts{};
    int max_inflight = 8;
    std::vector<hipStream_t> streams;
    std::vector<int> load;                 // running requests per stream
    hipEvent_t epoch = nullptr;
    double epoch_ms = 0;
    int64_t next = 0;
    std::map<int64_t, Ticket> tickets;
    std::deque<int64_t> queue;
    int inflight = 0;
    std::map<int64_t, Resident> resident;  // keyed by the ticket that factored it
    int64_t evictions = 0, completed = 0;
    // pinned host slots for the residual norms of refined requests: taken
    // and given back per request, allocated only when none is large enough
    // (pinning and unpinning host memory can wait for the whole device)
    std::vector<std::pair<unsigned long long *, size_t>> pin_free;
    std::vector<unsigned long long *> pin_all;
};

namespace {

constexpr size_t kSlabAlign = 256;

size_t slab_round(size_t bytes) { return (bytes + kSlabAlign - 1) / kSlabAlign * kSlabAlign; }

void slab_insert(Slab &B, size_t off, size_t bytes)
{
    auto next = B.free.lower_bound(off);
    if (next != B.free.end() && off + bytes == next->first) {
        bytes += next->second;
        next = B.free.erase(next);
    }
    if (next != B.free.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += bytes;
            return;
        }
    }
    B.free.emplace(off, bytes);
}

// ranges whose free has completed on the device become free
void slab_reclaim(Slab &B)
{
    for (size_t i = 0; i < B.pending.size();) {
        if (hipEventQuery(B.pending[i].ev) == hipSuccess) {
            slab_insert(B, B.pending[i].off, B.pending[i].bytes);
            B.spare.push_back(B.pending[i].ev);
            B.pending[i] = B.pending.back();
            B.pending.pop_back();
        } else {
            ++i;
        }
    }
}

// the smallest free range of at least `bytes` (best fit), split from its start
void *slab_alloc(Slab &B, size_t bytes, hipStream_t s)
{
    if (!B.base) return nullptr;
    bytes = slab_round(bytes);
    slab_reclaim(B);
    auto best = B.free.end();
    for (auto it = B.free.begin(); it != B.free.end(); ++it)
        if (it->second >= bytes && (best == B.free.end() || it->second < best->second)) best = it;
    if (best != B.free.end()) {
        const size_t off = best->first, have = best->second;
        B.free.erase(best);
        if (have > bytes) B.free.emplace(off + bytes, have - bytes);
        return B.base + off;
    }
    // a range whose free is still in flight: this stream waits for it
    size_t pick = B.pending.size();
    for (size_t i = 0; i < B.pending.size(); ++i)
        if (B.pending[i].bytes >= bytes &&
            (pick == B.pending.size() || B.pending[i].bytes < B.pending[pick].bytes))
            pick = i;
    if (pick == B.pending.size()) return nullptr;
    Slab::Pending P = B.pending[pick];
    if (hipStreamWaitEvent(s, P.ev, 0) != hipSuccess) return nullptr;
    if (P.bytes > bytes) {   // the rest stays pending behind the same event
        B.pending[pick].off = P.off + bytes;
        B.pending[pick].bytes = P.bytes - bytes;
    } else {
        B.spare.push_back(P.ev);
        B.pending[pick] = B.pending.back();
        B.pending.pop_back();
    }
    return B.base + P.off;
}

bool slab_free(Slab &B, void *p, size_t bytes, hipStream_t s)
{
    char *c = (char *)p;
    if (!B.base || c < B.base || c >= B.base + B.size) return false;
    hipEvent_t ev = nullptr;
    if (!B.spare.empty()) {
        ev = B.spare.back();
        B.spare.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
    }
    const size_t off = (size_t)(c - B.base);
    if (!ev || hipEventRecord(ev, s) != hipSuccess) {
        // no event: the range comes back once the stream has drained
        if (hipStreamSynchronize(s) == hipSuccess) slab_insert(B, off, slab_round(bytes));
        if (ev) B.spare.push_back(ev);
        return true;
    }
    B.pending.push_back({off, slab_round(bytes), ev});
    return true;
}

// the reserved slab first, the server's pool for what does not fit in it
void *pool_alloc(size_t bytes, void *stream, void *ctx)
{
    pf_server_s *S = (pf_server_s *)ctx;
    if (void *q = slab_alloc(S->slab, bytes, (hipStream_t)stream)) return q;
    void *p = nullptr;
    if (hipMallocFromPoolAsync(&p, bytes, S->pool, (hipStream_t)stream) != hipSuccess)
        return nullptr;
    return p;
}
void pool_free(void *p, size_t bytes, void *stream, void *ctx)
{
    pf_server_s *S = (pf_server_s *)ctx;
    if (slab_free(S->slab, p, bytes, (hipStream_t)stream)) return;
    (void)hipFreeAsync(p, (hipStream_t)stream);
}

size_t request_bytes(const pf_server_s *S, const pf_request &r)
{
    const size_t per = pf_solve_bytes_per_rhs(&r.A, &S->opts);
    if (r.factor >= 0) return per * (size_t)std::max(r.nrhs, 1);
    return pf_factor_bytes(&r.A, &S->opts) + per * (size_t)std::max(r.nrhs, 1);
}

// evict least recently used resident factors nobody needs until `need`
// bytes fit
bool make_room(pf_server_s *S, size_t need)
{
    while (S->used + need > S->budget) {
        int64_t victim = -1;
        double oldest = 0;
        for (auto &kv : S->resident) {
            const Resident &R = kv.second;
            if (R.users > 0 || !R.F) continue;
            if (victim < 0 || R.last_use < oldest) {
                victim = kv.first;
                oldest = R.last_use;
            }
        }
        if (victim < 0) return false;
        Resident &R = S->resident[victim];
        destroy_async(R.F);   // stream-ordered frees after the factor's last work
        S->used -= R.bytes;
        S->resident.erase(victim);
        ++S->evictions;
    }
    return true;
}

// a pinned slot of at least `words` words (smallest free one that fits)
bool pin_take(pf_server_s *S, size_t words, unsigned long long **p, size_t *cap)
{
    size_t best = S->pin_free.size();
    for (size_t i = 0; i < S->pin_free.size(); ++i)
        if (S->pin_free[i].second >= words &&
            (best == S->pin_free.size() || S->pin_free[i].second < S->pin_free[best].second))
            best = i;
    if (best < S->pin_free.size()) {
        *p = S->pin_free[best].first;
        *cap = S->pin_free[best].second;
        S->pin_free.erase(S->pin_free.begin() + (long)best);
        return true;
    }
    const size_t c = std::max<size_t>(words, 512);
    void *q = nullptr;
    if (hipHostMalloc(&q, c * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
        return false;
    S->pin_all.push_back((unsigned long long *)q);
    *p = (unsigned long long *)q;
    *cap = c;
    return true;
}
void pin_give(pf_server_s *S, Ticket &T)
{
    if (T.hnorms) S->pin_free.emplace_back(T.hnorms, T.hcap);
    T.hnorms = nullptr;
    T.hcap = 0;
}

// One refinement decision for a request whose residual norms have arrived:
// done (ev_done recorded behind the work so far), or the next correction
// and residual queued.  The same test and order as pf_solve's loop.
void refine_step(pf_server_s *S, int64_t id, Ticket &T)
{
    hipStream_t s = S->streams[T.stream];
    const pf_request &r = T.req;
    const pf_opts &o = handle_opts(T.F);
    T.eta = ir_eta(T.hnorms, r.nrhs);
    int status = PF_OK;
    bool done = true;
    if (T.eta <= o.tol) {
    } else if (T.iters >= o.max_refine || !std::isfinite(T.eta)) {
        status = PF_ENOCONV;
    } else {
        T.slow = (T.eta > 0.5 * T.prev) ? T.slow + 1 : 0;
        if (T.slow >= 2) status = PF_ENOCONV;
        else done = false;
    }
    if (!done) {
        T.prev = T.eta;
        int rc = ir_queue_correction(T.F, r.nrhs, r.x, r.ldx, s);
        if (!rc) rc = ir_queue_residual(T.F, r.nrhs, r.f, r.ldf, r.x, r.ldx, s, T.hnorms);
        if (!rc && hipEventRecord(T.ev_norms, s) != hipSuccess) rc = PF_EHIP;
        ++T.iters;
        if (!rc) return;
        status = rc;
    }
    T.ir = false;
    T.info.status = status;   // kept; the device status word is read at retirement
    if (hipEventRecord(T.ev_done, s) != hipSuccess) T.info.status = PF_EHIP;
    const int64_t home = r.factor >= 0 ? r.factor : (r.keep ? id : -1);
    if (home >= 0) S->resident[home].refining = false;
}

void retire(pf_server_s *S)
{
    for (auto &kv : S->tickets) {
        Ticket &T = kv.second;
        if (T.state != 1) continue;
        if (T.ir) {
            if (hipEventQuery(T.ev_norms) != hipSuccess) continue;
            refine_step(S, kv.first, T);
            continue;   // retired once ev_done has fired, at a later poll
        }
        if (hipEventQuery(T.ev_done) != hipSuccess) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, S->epoch, T.ev_done) == hipSuccess) T.t_done = S->epoch_ms + ms;
        if (hipEventElapsedTime(&ms, S->epoch, T.ev_start) == hipSuccess) T.t_start = S->epoch_ms + ms;
        {
            const int ir_status = T.info.status;
            status_nosync(T.F, &T.info);
            if (T.hnorms) {   // a refined request: its iterations, eta and outcome
                T.info.refine_iters = T.iters;
                T.info.eta = T.eta;
                if (T.info.status == PF_OK) T.info.status = ir_status;
                pin_give(S, T);
            }
        }
        T.state = 2;
        --S->inflight;
        --S->load[T.stream];
        ++S->completed;
        S->used -= T.bytes;
        if (T.req.factor >= 0) {
            auto it = S->resident.find(T.req.factor);
            if (it != S->resident.end()) {
                --it->second.users;
                it->second.last_use = now_ms();
                if (it->second.released && it->second.users == 0) {
                    if (it->second.F) destroy_async(it->second.F);
                    S->used -= it->second.bytes;
                    S->resident.erase(it);
                }
            }
        } else if (T.req.keep) {
            auto it = S->resident.find(kv.first);
            if (it != S->resident.end()) {
                --it->second.users;
                it->second.last_use = now_ms();
                if (it->second.released && it->second.users == 0) {
                    destroy_async(it->second.F);
                    S->used -= it->second.bytes;
                    S->resident.erase(it);
                }
            }
        } else {
            destroy_async(T.F);
        }
        hipEventDestroy(T.ev_start);
        hipEventDestroy(T.ev_done);
        if (T.ev_ready) hipEventDestroy(T.ev_ready);
        if (T.ev_norms) hipEventDestroy(T.ev_norms);
        T.ev_start = T.ev_done = T.ev_ready = T.ev_norms = nullptr;
    }
}

// PF_FP32_IR: queue the first residual behind the FP32 solve; the
// refinement continues from the polling (refine_step)
int start_refinement(pf_server_s *S, int64_t id, Ticket &T, hipStream_t s)
{
    const pf_request &r = T.req;
    if (!pin_take(S, 3 * (size_t)r.nrhs + 1, &T.hnorms, &T.hcap)) return PF_EHIP;
    if (hipEventCreateWithFlags(&T.ev_norms, hipEventDisableTiming) != hipSuccess) return PF_EHIP;
    const int rc = ir_queue_residual(T.F, r.nrhs, r.f, r.ldf, r.x, r.ldx, s, T.hnorms);
    if (rc) return rc;
    if (hipEventRecord(T.ev_norms, s) != hipSuccess) return PF_EHIP;
    T.ir = true;
    if (r.factor >= 0) S->resident[r.factor].refining = true;
    else if (r.keep) S->resident[id].refining = true;
    return 0;
}

int launch(pf_server_s *S, int64_t id, Ticket &T)
{
    const pf_request &r = T.req;
    if (hipEventCreateWithFlags(&T.ev_start, 0) != hipSuccess ||
        hipEventCreateWithFlags(&T.ev_done, 0) != hipSuccess)
        return PF_EHIP;
    int si;
    if (r.factor >= 0) {
        si = S->resident[r.factor].stream;
    } else {
        si = (int)(std::min_element(S->load.begin(), S->load.end()) - S->load.begin());
    }
    hipStream_t s = S->streams[si];
    const double t0 = now_ms();
    if (T.ev_ready && hipStreamWaitEvent(s, T.ev_ready, 0) != hipSuccess) return PF_EHIP;
    hipEventRecord(T.ev_start, s);
    int rc;
    if (r.factor >= 0) {
        T.F = S->resident[r.factor].F;
        rc = solve_queued(T.F, r.nrhs, r.f, r.ldf, r.x, r.ldx, s);
    } else {
        double setup = 0;
        rc = factor_new_solve(&r.A, &S->opts, s, r.nrhs, r.f, r.ldf, r.x, r.ldx, &T.F, &S->al,
                              &setup);
        S->setup_ms_max = std::max(S->setup_ms_max, setup);
        S->setup_ms_total += setup;
    }
    if (rc) return rc;
    if (S->opts.prec == PF_FP32_IR && (rc = start_refinement(S, id, T, s))) {
        if (r.factor < 0) {
            destroy_async(T.F);
            T.F = nullptr;
        }
        return rc;
    }
    const double dt = now_ms() - t0;
    S->launch_ms_max = std::max(S->launch_ms_max, dt);
    S->launch_ms_total += dt;
    if (!T.ir) hipEventRecord(T.ev_done, s);
    T.stream = si;
    T.state = 1;
    ++S->inflight;
    ++S->load[si];
    if (r.factor < 0 && r.keep) {
        // the entry was registered at submission; the factor's memory stays
        // charged after this request: move it from the request to the entry
        Resident &R = S->resident[id];
        R.F = T.F;
        R.bytes = T.bytes;
        R.stream = si;
        R.last_use = now_ms();
        T.bytes = 0;
    }
    return 0;
}

// a request that cannot run any more (its factor's request failed)
void fail(pf_server_s *S, Ticket &T, int rc)
{
    T.state = 2;
    T.info = pf_info{};
    T.info.status = rc;
    T.info.eta = -1.0;
    T.info.bad_block = -1;
    T.t_done = now_ms();
    if (T.ev_start) hipEventDestroy(T.ev_start);
    if (T.ev_done) hipEventDestroy(T.ev_done);
    if (T.ev_ready) hipEventDestroy(T.ev_ready);
    if (T.ev_norms) hipEventDestroy(T.ev_norms);
    pin_give(S, T);
    T.ev_start = T.ev_done = T.ev_ready = T.ev_norms = nullptr;
    T.ir = false;
}

// Admit queued requests in arrival order; one that does not fit yet stays
// queued while later ones that fit go ahead (a request for a resident factor
// needs only solve workspace).
void admit(pf_server_s *S)
{
    for (auto q = S->queue.begin(); q != S->queue.end() && S->inflight < S->max_inflight;) {
        const int64_t id = *q;
        Ticket &T = S->tickets[id];
        if (T.req.factor >= 0) {
            Resident &R = S->resident[T.req.factor];
            if (R.failed) {                  // its factor never came to exist
                q = S->queue.erase(q);
                --R.users;
                fail(S, T, R.failed);
                continue;
            }
            if (!R.F || R.refining) {        // its factor's request has not started, or
                ++q;                         // another request is refining on its workspace
                continue;
            }
        }
        const size_t need = request_bytes(S, T.req);
        if (!make_room(S, need)) {
            ++q;
            continue;
        }
        q = S->queue.erase(q);
        S->used += need;
        T.bytes = need;
        const int rc = launch(S, id, T);
        if (rc) {
            S->used -= need;
            if (T.req.factor >= 0) --S->resident[T.req.factor].users;
            if (T.req.factor < 0 && T.req.keep) {
                Resident &R = S->resident[id];
                R.failed = rc;
                --R.users;
            }
            fail(S, T, rc);
        }
    }
}

void progress(pf_server_s *S)
{
    retire(S);
    admit(S);
}

}  // namespace

extern "C" {

int pf_server_create(size_t budget_bytes, const pf_opts *opts, int32_t max_inflight,
                     int32_t nstreams, pf_server_t *out)
{
    if (!out) return -5;
    *out = nullptr;
    if (budget_bytes == 0) return -1;
    if (max_inflight < 0) return -3;
    if (nstreams < 0) return -4;
    pf_server_s *S = new pf_server_s();
    S->budget = budget_bytes;
    if (opts) S->opts = *opts;
    S->opts.flags &= ~PF_FLAG_AUTOTUNE;
    if (S->opts.prec != PF_FP64 && S->opts.prec != PF_FP32_IR) {
        delete S;
        return -2;
    }
    S->max_inflight = max_inflight ? max_inflight : 8;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) {
            pf_server_destroy(S);
            return PF_EHIP;
        }
        hipMemPoolProps pp{};
        pp.allocType = hipMemAllocationTypePinned;
        pp.handleTypes = hipMemHandleTypeNone;
        pp.location.type = hipMemLocationTypeDevice;
        pp.location.id = dev;
        uint64_t keep = budget_bytes;
        if (hipMemPoolCreate(&S->pool, &pp) != hipSuccess ||
            hipMemPoolSetAttribute(S->pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
            pf_server_destroy(S);
            return PF_EHIP;
        }
        S->al.alloc = pool_alloc;
        S->al.free = pool_free;
        S->al.ctx = (void *)S;
    }
    const int ns = nstreams ? nstreams : 4;
    for (int i = 0; i < ns; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            pf_server_destroy(S);
            return PF_EHIP;
        }
        S->streams.push_back(s);
        S->load.push_back(0);
    }
    if (hipEventCreate(&S->epoch) != hipSuccess || hipEventRecord(S->epoch, S->streams[0]) != hipSuccess ||
        hipEventSynchronize(S->epoch) != hipSuccess) {
        pf_server_destroy(S);
        return PF_EHIP;
    }
    S->epoch_ms = now_ms();
    *out = S;
    return 0;
}

int pf_server_submit(pf_server_t S, const pf_request *req, int64_t *ticket)
{
    if (!S) return -1;
    if (!req) return -2;
    if (!ticket) return -3;
    const pf_request &r = *req;
    if (r.nrhs < 1 || !r.f || !r.x) return -2;
    const int64_t n = r.A.nb * r.A.m;
    if (pf_factor_bytes(&r.A, &S->opts) == 0 || r.ldf < n || r.ldx < n) return -2;
    if (r.factor >= 0) {
        auto it = S->resident.find(r.factor);
        if (it == S->resident.end() || it->second.released || it->second.failed) return -2;
    }
    if (request_bytes(S, r) > S->budget) return PF_ENOMEM;
    const int64_t id = S->next++;
    Ticket &T = S->tickets[id];
    T.req = r;
    T.t_submit = now_ms();
    if (hipEventCreateWithFlags(&T.ev_ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(T.ev_ready, (hipStream_t)r.after) != hipSuccess) {
        if (T.ev_ready) hipEventDestroy(T.ev_ready);
        S->tickets.erase(id);
        return PF_EHIP;
    }
    if (r.factor >= 0) ++S->resident[r.factor].users;
    if (r.factor < 0 && r.keep) {      // later requests may name it at once
        Resident R;
        R.users = 1;
        R.last_use = T.t_submit;
        S->resident[id] = R;
    }
    S->queue.push_back(id);
    *ticket = id;
    progress(S);
    return 0;
}

int pf_server_poll(pf_server_t S, int64_t ticket, pf_info *info)
{
    if (!S) return -1;
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return -2;
    progress(S);
    if (it->second.state != 2) return 0;
    if (info) *info = it->second.info;
    return 1;
}

int pf_server_wait(pf_server_t S, int64_t ticket, pf_info *info)
{
    if (!S) return -1;
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return -2;
    for (;;) {
        progress(S);
        Ticket &T = it->second;
        if (T.state == 2) break;
        if (T.state == 1) {
            if (hipEventSynchronize(T.ir ? T.ev_norms : T.ev_done) != hipSuccess) return PF_EHIP;
        } else {
            // queued: wait for the oldest running request to make room
            hipEvent_t ev = nullptr;
            for (auto &kv : S->tickets)
                if (kv.second.state == 1) {
                    ev = kv.second.ir ? kv.second.ev_norms : kv.second.ev_done;
                    break;
                }
            if (!ev) return PF_ENOMEM;    // nothing running and still not admitted
            if (hipEventSynchronize(ev) != hipSuccess) return PF_EHIP;
        }
    }
    if (info) *info = it->second.info;
    return it->second.info.status;
}

int pf_server_times(pf_server_t S, int64_t ticket, double *submit_ms, double *start_ms,
                    double *done_ms)
{
    if (!S) return -1;
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return -2;
    const Ticket &T = it->second;
    if (submit_ms) *submit_ms = T.t_submit - S->epoch_ms;
    if (start_ms) *start_ms = T.t_start < 0 ? -1.0 : T.t_start - S->epoch_ms;
    if (done_ms) *done_ms = T.t_done < 0 ? -1.0 : T.t_done - S->epoch_ms;
    return T.state == 2 ? 1 : 0;
}

int pf_server_release(pf_server_t S, int64_t factor)
{
    if (!S) return -1;
    auto it = S->resident.find(factor);
    if (it == S->resident.end()) return -2;
    it->second.released = true;
    if (it->second.users == 0) {
        if (it->second.F) destroy_async(it->second.F);
        S->used -= it->second.bytes;
        S->resident.erase(it);
    }
    return 0;
}

int pf_server_stats(pf_server_t S, pf_server_info *st)
{
    if (!S) return -1;
    if (!st) return -2;
    progress(S);
    std::memset(st, 0, sizeof *st);
    st->budget = S->budget;
    st->used = S->used;
    st->queued = (int64_t)S->queue.size();
    st->inflight = S->inflight;
    st->resident = (int64_t)S->resident.size();
    st->completed = S->completed;
    st->evictions = S->evictions;
    st->setup_ms_max = S->setup_ms_max;
    st->setup_ms_total = S->setup_ms_total;
    st->launch_ms_max = S->launch_ms_max;
    st->launch_ms_total = S->launch_ms_total;
    return 0;
}

int pf_server_reserve(pf_server_t S, size_t bytes)
{
    if (!S) return -1;
    if (bytes > S->budget) return -2;
    if (bytes == 0) return 0;
    if (S->slab.base) return -3;   // once per server
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, slab_round(bytes));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? PF_ENOMEM : PF_EHIP;
    S->slab.base = (char *)p;
    S->slab.size = slab_round(bytes);
    S->slab.free.emplace(0, S->slab.size);
    return 0;
}

void pf_server_destroy(pf_server_t S)
{
    if (!S) return;
    for (hipStream_t s : S->streams) hipStreamSynchronize(s);
    for (auto &kv : S->tickets) {
        Ticket &T = kv.second;
        if (T.ev_start) hipEventDestroy(T.ev_start);
        if (T.ev_done) hipEventDestroy(T.ev_done);
        if (T.ev_ready) hipEventDestroy(T.ev_ready);
        if (T.ev_norms) hipEventDestroy(T.ev_norms);
        if (T.state == 2 && T.req.factor < 0 && !T.req.keep) continue;   // freed at retire
        if (T.state == 1 && T.req.factor < 0 && !T.req.keep) destroy_async(T.F);
    }
    for (auto &kv : S->resident)
        if (kv.second.F) destroy_async(kv.second.F);
    for (hipStream_t s : S->streams) {
        hipStreamSynchronize(s);
        hipStreamDestroy(s);
    }
    if (S->epoch) hipEventDestroy(S->epoch);
    for (auto &P : S->slab.pending) hipEventDestroy(P.ev);
    for (hipEvent_t ev : S->slab.spare) hipEventDestroy(ev);
    if (S->slab.base) hipFree(S->slab.base);
    if (S->pool) hipMemPoolDestroy(S->pool);
    for (unsigned long long *p : S->pin_all) hipHostFree(p);
    delete S;
}

}  // extern "C"
