// Continuous-batching request loop (serving): requests for resident lenses
// and maps are admitted in arrival order while their accounted memory fits a
// budget, split into chunks, and the chunks are launched on a small pool of
// HIP streams as streams free up, round-robin over the admitted requests, so
// short requests are not stuck behind long ones and requests that arrive
// while others run overlap with them on the device.
//
// The loop is driven by the caller's lt_server_poll calls (no thread of its
// own): each call reaps finished chunks (event queries), admits, launches and
// reports completed requests.  Completion times are device times (events
// against the server's start event), so the host's polling rate does not
// enter the latencies it reports.
#include <algorithm>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "lt_internal.h"
#include "lt_map.h"

namespace lt {

namespace {

constexpr int kMaxStreams = 16;

struct Request {
    int64_t tag = 0;
    bool is_map = true;
    lt_map map = nullptr;
    int32_t dtype = LT_BF16;
    lt_lens lens = nullptr;
    lt_path path{};
    lt_rays rays{};
    lt_map_out mout{};
    lt_exit eout{};
    int64_t n = 0;
    int64_t chunk = 0;        // rays per launch for this request
    int64_t next = 0;         // first ray not yet launched
    int64_t in_flight = 0;    // launched chunks not yet reaped
    int64_t mem = 0;          // accounted bytes
    double done_s = 0.0;      // latest chunk completion so far
    int32_t status = LT_OK;
};

struct Server {
    lt_server_cfg cfg{};
    int dev = 0;
    hipStream_t streams[kMaxStreams] = {};
    hipEvent_t events[kMaxStreams] = {};
    Request *slot_req[kMaxStreams] = {};
    hipEvent_t t0 = nullptr;
    std::deque<Request *> waiting;
    std::vector<Request *> active;
    std::deque<lt_server_done> ready;
    int64_t in_use = 0, max_in_use = 0, launches = 0, open = 0;
    uint64_t rr = 0;
};

Server *as_server(lt_server h) { return reinterpret_cast<Server *>(h); }

template <class T>
T *at(T *p, int64_t k)
{
    return p ? p + k : p;
}

bool rays_set(const lt_rays &r)
{
    return r.x && r.y && r.dx && r.dy && r.dz && r.lambda_nm;
}

bool packed_current(const Map &M, int32_t dtype)
{
    if (dtype == LT_F32)
        return M.packed_f32 == M.version;
    if (dtype == LT_FP8)
        return M.packed_fp8 == M.version;
    return M.packed_bf16 == M.version;
}

lt_status queue(Server *S, Request *r)
{
    if (r->mem > S->cfg.mem_budget) {
        delete r;
        return fail(LT_ERR_ARG, "request needs more memory than the server's budget");
    }
    S->waiting.push_back(r);
    ++S->open;
    return LT_OK;
}

void finish(Server *S, Request *r)
{
    S->in_use -= r->mem;
    S->active.erase(std::find(S->active.begin(), S->active.end(), r));
    S->ready.push_back(lt_server_done{r->tag, r->done_s, r->status});
    delete r;
}

lt_status launch(Server *S, int slot, Request *r)
{
    const int64_t lo = r->next, hi = std::min(r->n, lo + r->chunk);
    r->next = hi;
    hipStream_t s = S->streams[slot];
    const lt_rays rays{at(r->rays.x, lo), at(r->rays.y, lo), at(r->rays.dx, lo),
                       at(r->rays.dy, lo), at(r->rays.dz, lo), at(r->rays.lambda_nm, lo)};
    lt_status st;
    if (r->is_map) {
        const lt_map_out o{at(r->mout.logit, lo), at(r->mout.mask, lo), at(r->mout.x, lo),
                           at(r->mout.y, lo), at(r->mout.dx, lo), at(r->mout.dy, lo),
                           at(r->mout.dz, lo), at(r->mout.throughput, lo)};
        st = lt_map_eval(r->map, r->dtype, &rays, &o, hi - lo, s);
    } else {
        const lt_exit e{at(r->eout.mask, lo), at(r->eout.x, lo), at(r->eout.y, lo), at(r->eout.dx, lo),
                        at(r->eout.dy, lo), at(r->eout.dz, lo), at(r->eout.throughput, lo)};
        st = lt_trace(r->lens, &r->path, &rays, &e, hi - lo, s);
    }
    if (st != LT_OK && r->status == LT_OK)
        r->status = st;
    lt_status ev = check_hip(hipEventRecord(S->events[slot], s), "hipEventRecord");
    if (ev != LT_OK)
        return ev;
    S->slot_req[slot] = r;
    ++r->in_flight;
    ++S->launches;
    return LT_OK;
}

lt_status reap(Server *S)
{
    for (int k = 0; k < S->cfg.n_streams; ++k) {
        Request *r = S->slot_req[k];
        if (!r)
            continue;
        const hipError_t q = hipEventQuery(S->events[k]);
        if (q == hipErrorNotReady)
            continue;
        if (q != hipSuccess)
            return check_hip(q, "hipEventQuery");
        float ms = 0.0f;
        lt_status st = check_hip(hipEventElapsedTime(&ms, S->t0, S->events[k]), "hipEventElapsedTime");
        if (st != LT_OK)
            return st;
        S->slot_req[k] = nullptr;
        r->done_s = std::max(r->done_s, 1e-3 * static_cast<double>(ms));
        if (--r->in_flight == 0 && r->next >= r->n)
            finish(S, r);
    }
    return LT_OK;
}

void admit(Server *S)
{
    while (!S->waiting.empty() && S->in_use + S->waiting.front()->mem <= S->cfg.mem_budget) {
        Request *r = S->waiting.front();
        S->waiting.pop_front();
        S->in_use += r->mem;
        S->max_in_use = std::max(S->max_in_use, S->in_use);
        S->active.push_back(r);
        if (r->n == 0)
            finish(S, r);   // nothing to launch; completes at its admission
    }
}

lt_status launch_free(Server *S)
{
    std::vector<Request *> cands;
    for (int k = 0; k < S->cfg.n_streams; ++k) {
        if (S->slot_req[k])
            continue;
        cands.clear();
        for (Request *r : S->active)
            if (r->next < r->n)
                cands.push_back(r);
        if (cands.empty())
            break;
        Request *r = cands[S->rr++ % cands.size()];
        lt_status st = launch(S, k, r);
        if (st != LT_OK)
            return st;
    }
    return LT_OK;
}

}  // namespace
}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_server_create(const lt_server_cfg *cfg, lt_server *out)
{
    if (!cfg || !out)
        return fail(LT_ERR_ARG, "NULL cfg or out");
    if (cfg->n_streams < 1 || cfg->n_streams > kMaxStreams)
        return fail(LT_ERR_ARG, "n_streams must be in 1..16");
    if (cfg->chunk < 1 || cfg->mem_budget < 1 || cfg->bytes_per_ray < 0)
        return fail(LT_ERR_ARG, "chunk and mem_budget must be positive, bytes_per_ray non-negative");
    Server *S = new (std::nothrow) Server;
    if (!S)
        return fail(LT_ERR_OOM, "host allocation");
    S->cfg = *cfg;
    lt_status st = check_hip(hipGetDevice(&S->dev), "hipGetDevice");
    for (int k = 0; st == LT_OK && k < cfg->n_streams; ++k) {
        st = check_hip(hipStreamCreateWithFlags(&S->streams[k], hipStreamNonBlocking), "hipStreamCreate");
        if (st == LT_OK)
            st = check_hip(hipEventCreate(&S->events[k]), "hipEventCreate");
    }
    if (st == LT_OK)
        st = check_hip(hipEventCreate(&S->t0), "hipEventCreate");
    if (st == LT_OK)
        st = check_hip(hipEventRecord(S->t0, S->streams[0]), "hipEventRecord");
    if (st == LT_OK)
        st = check_hip(hipEventSynchronize(S->t0), "hipEventSynchronize");
    if (st != LT_OK) {
        lt_server_destroy(reinterpret_cast<lt_server>(S));
        return st;
    }
    *out = reinterpret_cast<lt_server>(S);
    return LT_OK;
}

lt_status lt_server_destroy(lt_server server)
{
    Server *S = as_server(server);
    if (!S)
        return LT_OK;
    lt_status st = LT_OK;
    for (int k = 0; k < kMaxStreams; ++k) {
        if (S->streams[k]) {
            lt_status s2 = check_hip(hipStreamSynchronize(S->streams[k]), "hipStreamSynchronize");
            if (st == LT_OK)
                st = s2;
            (void)hipStreamDestroy(S->streams[k]);
        }
        if (S->events[k])
            (void)hipEventDestroy(S->events[k]);
    }
    if (S->t0)
        (void)hipEventDestroy(S->t0);
    for (Request *r : S->waiting)
        delete r;
    for (Request *r : S->active)
        delete r;
    delete S;
    return st;
}

lt_status lt_server_submit_map(lt_server server, lt_map map, int32_t dtype, const lt_rays *rays,
                               const lt_map_out *out, int64_t n, int64_t tag)
{
    Server *S = as_server(server);
    Map *M = as_map(map);
    if (!S || !M || !rays || !out)
        return fail(LT_ERR_ARG, "NULL server, map, rays or out");
    if (n < 0)
        return fail(LT_ERR_ARG, "negative ray count");
    if (dtype != LT_BF16 && dtype != LT_FP8 && dtype != LT_F32)
        return fail(LT_ERR_DTYPE, "precision not available (LT_F32, LT_BF16, LT_FP8)");
    if (n > 0 && (!rays_set(*rays) || !out->logit || !out->mask || !out->x || !out->y || !out->dx ||
                  !out->dy || !out->dz || !out->throughput))
        return fail(LT_ERR_ARG, "NULL ray or output field");
    if (n > 0 && !packed_current(*M, dtype))
        return fail(LT_ERR_STATE, "run lt_map_quantize for this precision before submitting");
    Request *r = new (std::nothrow) Request;
    if (!r)
        return fail(LT_ERR_OOM, "host allocation");
    r->tag = tag;
    r->is_map = true;
    r->map = map;
    r->dtype = dtype;
    r->rays = *rays;
    r->mout = *out;
    r->n = n;
    // head-major outputs keep the request's own stride only when it runs whole
    r->chunk = M->lay.P == 1 ? S->cfg.chunk : std::max<int64_t>(n, 1);
    r->mem = n * S->cfg.bytes_per_ray;
    return queue(S, r);
}

lt_status lt_server_submit_trace(lt_server server, lt_lens lens, const lt_path *path,
                                 const lt_rays *rays, const lt_exit *out, int64_t n, int64_t tag)
{
    Server *S = as_server(server);
    Lens *L = as_lens(lens);
    if (!S || !L || !path || !rays || !out)
        return fail(LT_ERR_ARG, "NULL server, lens, path, rays or out");
    if (n < 0)
        return fail(LT_ERR_ARG, "negative ray count");
    if (n > 0 && (!rays_set(*rays) || !out->mask || !out->x || !out->y || !out->dx || !out->dy ||
                  !out->dz || !out->throughput))
        return fail(LT_ERR_ARG, "NULL ray or output field");
    TraceTable table;
    lt_status st = build_trace_table(*L, *path, false, &table);
    if (st != LT_OK)
        return st;
    Request *r = new (std::nothrow) Request;
    if (!r)
        return fail(LT_ERR_OOM, "host allocation");
    r->tag = tag;
    r->is_map = false;
    r->lens = lens;
    r->path = *path;
    r->rays = *rays;
    r->eout = *out;
    r->n = n;
    r->chunk = S->cfg.chunk;
    r->mem = n * S->cfg.bytes_per_ray;
    return queue(S, r);
}

lt_status lt_server_poll(lt_server server, lt_server_done *done, int32_t cap, int32_t *n_done,
                         int64_t *n_open)
{
    Server *S = as_server(server);
    if (!S || !n_done || cap < 0 || (cap > 0 && !done))
        return fail(LT_ERR_ARG, "NULL server or n_done, or bad done/cap");
    int prev = S->dev;
    lt_status st = check_hip(hipGetDevice(&prev), "hipGetDevice");
    if (st == LT_OK && prev != S->dev)
        st = check_hip(hipSetDevice(S->dev), "hipSetDevice");
    if (st == LT_OK)
        st = reap(S);
    if (st == LT_OK) {
        admit(S);
        st = launch_free(S);
    }
    if (prev != S->dev)
        (void)hipSetDevice(prev);
    int32_t k = 0;
    while (k < cap && !S->ready.empty()) {
        done[k++] = S->ready.front();
        S->ready.pop_front();
    }
    S->open -= k;
    *n_done = k;
    if (n_open)
        *n_open = S->open;
    return st;
}

lt_status lt_server_stats(lt_server server, int64_t *max_in_use_bytes, int64_t *launches)
{
    Server *S = as_server(server);
    if (!S)
        return fail(LT_ERR_ARG, "NULL server");
    if (max_in_use_bytes)
        *max_in_use_bytes = S->max_in_use;
    if (launches)
        *launches = S->launches;
    return LT_OK;
}

}  // extern "C"
