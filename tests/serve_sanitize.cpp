// The serving loop's host bookkeeping (lt_serve.cpp: admission by memory,
// chunking, round-robin launch over a stream pool, reaping by event query,
// completion reports, teardown with requests in flight) under
// AddressSanitizer and UndefinedBehaviorSanitizer on the CPU.  The device is
// replaced by a fake HIP runtime (streams and events whose completion is
// reported after a random number of queries) and fake lt_map_eval / lt_trace
// launches that write every output element of their chunk, so a chunk that
// strays outside its request's buffers is an ASan report and a ray covered
// twice or never is a failed check.  Built and run by
// tests/test_serve_sanitize.py; any sanitizer report aborts the run.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "lt.h"
#include "lt_internal.h"
#include "lt_map.h"

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed, line %d: %s\n", __LINE__, #c); \
            std::abort();                                                    \
        }                                                                    \
    } while (0)

namespace {
std::mt19937_64 rng(20261204);
int pick(int a, int b) { return std::uniform_int_distribution<int>(a, b)(rng); }
double clock_ms = 0.0;
}  // namespace

// ------------------------------------------------------------ fake HIP --
struct ihipStream_t {
    std::vector<ihipEvent_t *> events;
};
struct ihipEvent_t {
    ihipStream_t *stream = nullptr;
    int pending = 0;     // queries that still report "not ready"
    double t_ms = 0.0;   // completion time
    bool recorded = false;
};

namespace {
std::set<ihipStream_t *> live_streams;
std::set<ihipEvent_t *> live_events;
int current_device = 0;
}  // namespace

extern "C" {
hipError_t hipGetDevice(int *d)
{
    *d = current_device;
    return hipSuccess;
}
hipError_t hipSetDevice(int d)
{
    current_device = d;
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    auto *p = new ihipStream_t;
    live_streams.insert(p);
    *s = p;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    CHECK(live_streams.count(s));
    for (ihipEvent_t *e : s->events)
        if (live_events.count(e))
            e->pending = 0;
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    CHECK(live_streams.erase(s) == 1);
    delete s;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    auto *p = new ihipEvent_t;
    live_events.insert(p);
    *e = p;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    CHECK(live_events.count(e) && live_streams.count(s));
    e->stream = s;
    e->pending = pick(0, 3);
    clock_ms += 0.01 * pick(1, 50);
    e->t_ms = clock_ms;
    e->recorded = true;
    s->events.push_back(e);
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e)
{
    CHECK(live_events.count(e) && e->recorded);
    if (e->pending > 0) {
        --e->pending;
        return hipErrorNotReady;
    }
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    CHECK(live_events.count(e) && e->recorded);
    e->pending = 0;
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    CHECK(live_events.count(a) && live_events.count(b) && a->recorded && b->recorded);
    CHECK(a->pending == 0 && b->pending == 0);   // only completed events are timed
    *ms = static_cast<float>(b->t_ms - a->t_ms);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e)
{
    CHECK(live_events.erase(e) == 1);
    for (ihipStream_t *s : live_streams)
        s->events.erase(std::remove(s->events.begin(), s->events.end(), e), s->events.end());
    delete e;
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "fake HIP error"; }
}  // extern "C"

// ------------------------------------------------- fake device launches --
namespace {
struct Buffers {
    int64_t n = 0;
    int P = 1;
    std::vector<float> x, y, dx, dy, dz, lam;  // rays
    std::vector<float> o[7];                   // outputs (float fields)
    std::vector<uint8_t> mask;
    std::vector<int> covered;                  // launches that wrote each ray
    bool fail = false;                         // the fake launch reports an error
};
std::map<const float *, Buffers *> by_first;   // rays.x -> buffers
int64_t fake_launches = 0;

Buffers *find_chunk(const float *x, int64_t n, int64_t *lo)
{
    for (auto &kv : by_first) {
        Buffers *b = kv.second;
        if (x >= b->x.data() && x + n <= b->x.data() + b->n) {
            *lo = x - b->x.data();
            return b;
        }
    }
    return nullptr;
}
}  // namespace

namespace lt {
Map *as_map(lt_map h) { return reinterpret_cast<Map *>(h); }
}  // namespace lt

extern "C" lt_status lt_map_eval(lt_map map, int32_t, const lt_rays *rays, const lt_map_out *out, int64_t n,
                                 void *stream)
{
    CHECK(map && rays && out && n > 0 && live_streams.count(static_cast<hipStream_t>(stream)));
    ++fake_launches;
    int64_t lo = 0;
    Buffers *b = find_chunk(static_cast<const float *>(rays->x), n, &lo);
    CHECK(b != nullptr);
    // head-major outputs: every head's row of the chunk (the request runs
    // whole when it has several heads)
    for (int h = 0; h < b->P; ++h) {
        float *fields[] = {out->logit, out->x, out->y, out->dx, out->dy, out->dz, out->throughput};
        for (float *f : fields)
            for (int64_t k = 0; k < n; ++k)
                f[static_cast<int64_t>(h) * n + k] = static_cast<float>(lo + k);
        for (int64_t k = 0; k < n; ++k)
            out->mask[static_cast<int64_t>(h) * n + k] = 1;
    }
    for (int64_t k = 0; k < n; ++k)
        ++b->covered[lo + k];
    return b->fail ? LT_ERR_DEVICE : LT_OK;
}

extern "C" lt_status lt_trace(lt_lens lens, const lt_path *path, const lt_rays *rays, const lt_exit *out,
                              int64_t n, void *stream)
{
    CHECK(lens && path && rays && out && n > 0 && live_streams.count(static_cast<hipStream_t>(stream)));
    ++fake_launches;
    int64_t lo = 0;
    Buffers *b = find_chunk(static_cast<const float *>(rays->x), n, &lo);
    CHECK(b != nullptr);
    float *fields[] = {out->x, out->y, out->dx, out->dy, out->dz, out->throughput};
    for (float *f : fields)
        for (int64_t k = 0; k < n; ++k)
            f[k] = static_cast<float>(lo + k);
    for (int64_t k = 0; k < n; ++k) {
        out->mask[k] = 1;
        ++b->covered[lo + k];
    }
    return b->fail ? LT_ERR_DEVICE : LT_OK;
}

// ------------------------------------------------------------- scenarios --
namespace {

Buffers *make_buffers(int64_t n, int P)
{
    auto *b = new Buffers;
    b->n = n;
    b->P = P;
    for (auto *v : {&b->x, &b->y, &b->dx, &b->dy, &b->dz, &b->lam})
        v->assign(static_cast<size_t>(std::max<int64_t>(n, 0)), 0.5f);
    for (auto &v : b->o)
        v.assign(static_cast<size_t>(n * P), NAN);
    b->mask.assign(static_cast<size_t>(n * P), 0);
    b->covered.assign(static_cast<size_t>(n), 0);
    return b;
}

lt_rays rays_of(Buffers *b)
{
    return lt_rays{b->x.data(), b->y.data(), b->dx.data(), b->dy.data(), b->dz.data(), b->lam.data()};
}

int n_scenarios = 0, n_requests = 0, n_rejected = 0;

void scenario(lt_lens lens, lt::Map *maps[2])
{
    ++n_scenarios;
    lt_server_cfg cfg{};
    cfg.n_streams = pick(1, 16);
    cfg.chunk = pick(1, 3000);
    cfg.bytes_per_ray = pick(0, 32);
    cfg.mem_budget = static_cast<int64_t>(pick(1, 2000000));
    lt_server S = nullptr;
    CHECK(lt_server_create(&cfg, &S) == LT_OK && S);
    std::map<int64_t, Buffers *> open;     // tag -> buffers
    std::map<int64_t, lt_status> expect;   // tag -> expected status
    std::set<int64_t> reported;
    const int n_req = pick(0, 60);
    int64_t tag = 1000 * n_scenarios;
    auto poll = [&](int cap) {
        std::vector<lt_server_done> done(static_cast<size_t>(std::max(cap, 1)));
        int32_t nd = 0;
        int64_t nopen = 0;
        CHECK(lt_server_poll(S, cap ? done.data() : nullptr, cap, &nd, &nopen) == LT_OK);
        CHECK(nd >= 0 && nd <= cap && nopen >= 0);
        for (int k = 0; k < nd; ++k) {
            const lt_server_done &d = done[static_cast<size_t>(k)];
            CHECK(open.count(d.tag) && !reported.count(d.tag));
            CHECK(d.status == expect[d.tag]);
            CHECK(d.done_s >= 0.0);
            Buffers *b = open[d.tag];
            for (int64_t r = 0; r < b->n; ++r)
                CHECK(b->covered[r] == 1);   // every ray of the request exactly once
            reported.insert(d.tag);
        }
    };
    for (int q = 0; q < n_req; ++q) {
        const bool is_map = pick(0, 1) == 1;
        const int P = is_map ? (pick(0, 3) == 0 ? 3 : 1) : 1;
        const int64_t n = pick(0, 9) == 0 ? 0 : pick(1, 20000);
        Buffers *b = make_buffers(n, P);
        b->fail = pick(0, 15) == 0 && n > 0;
        by_first[b->x.data()] = b;
        const lt_rays r = rays_of(b);
        ++tag;
        lt_status st;
        if (is_map) {
            lt_map_out o{b->o[0].data(), b->mask.data(), b->o[1].data(), b->o[2].data(),
                         b->o[3].data(), b->o[4].data(), b->o[5].data(), b->o[6].data()};
            lt::Map *M = maps[P == 3 ? 1 : 0];
            st = lt_server_submit_map(S, reinterpret_cast<lt_map>(M), LT_BF16, &r, &o, n, tag);
        } else {
            lt_exit e{b->mask.data(), b->o[1].data(), b->o[2].data(), b->o[3].data(),
                      b->o[4].data(), b->o[5].data(), b->o[6].data()};
            const bool ghost = pick(0, 1) == 1;
            lt_path p{ghost ? 1 : 0, ghost ? 1 : 0, ghost ? 2 : 0};
            st = lt_server_submit_trace(S, lens, &p, &r, &e, n, tag);
        }
        const bool too_big = n * cfg.bytes_per_ray > cfg.mem_budget;
        CHECK((st == LT_OK) != too_big);
        ++n_requests;
        if (st != LT_OK) {
            ++n_rejected;
            by_first.erase(b->x.data());
            delete b;
            continue;
        }
        open[tag] = b;
        expect[tag] = b->fail ? LT_ERR_DEVICE : LT_OK;
        if (pick(0, 2) == 0)
            poll(pick(0, 8));
    }
    // drain most scenarios; leave some with requests in flight for teardown
    const bool drain = pick(0, 4) != 0;
    for (int it = 0; drain && reported.size() < open.size(); ++it) {
        CHECK(it < 1000000);
        poll(pick(1, 64));
    }
    if (drain)
        CHECK(reported.size() == open.size());
    int64_t max_in_use = -1, launches = -1;
    CHECK(lt_server_stats(S, &max_in_use, &launches) == LT_OK);
    CHECK(max_in_use >= 0 && max_in_use <= cfg.mem_budget);
    CHECK(launches >= 0);
    CHECK(lt_server_destroy(S) == LT_OK);
    for (auto &kv : open) {
        by_first.erase(kv.second->x.data());
        delete kv.second;
    }
}

void misuse(lt_lens lens, lt::Map *maps[2])
{
    lt_server_cfg cfg{};
    cfg.n_streams = 2;
    cfg.chunk = 100;
    cfg.mem_budget = 1 << 20;
    cfg.bytes_per_ray = 4;
    lt_server S = nullptr;
    CHECK(lt_server_create(nullptr, &S) == LT_ERR_ARG);
    for (int ns : {0, 17, -1}) {
        lt_server_cfg c = cfg;
        c.n_streams = ns;
        CHECK(lt_server_create(&c, &S) == LT_ERR_ARG);
    }
    {
        lt_server_cfg c = cfg;
        c.chunk = 0;
        CHECK(lt_server_create(&c, &S) == LT_ERR_ARG);
    }
    CHECK(lt_server_create(&cfg, &S) == LT_OK);
    Buffers *b = make_buffers(10, 1);
    by_first[b->x.data()] = b;
    lt_rays r = rays_of(b);
    lt_map_out o{b->o[0].data(), b->mask.data(), b->o[1].data(), b->o[2].data(),
                 b->o[3].data(), b->o[4].data(), b->o[5].data(), b->o[6].data()};
    lt_exit e{b->mask.data(), b->o[1].data(), b->o[2].data(), b->o[3].data(),
              b->o[4].data(), b->o[5].data(), b->o[6].data()};
    lt_map M0 = reinterpret_cast<lt_map>(maps[0]);
    CHECK(lt_server_submit_map(nullptr, M0, LT_BF16, &r, &o, 10, 1) == LT_ERR_ARG);
    CHECK(lt_server_submit_map(S, nullptr, LT_BF16, &r, &o, 10, 1) == LT_ERR_ARG);
    CHECK(lt_server_submit_map(S, M0, LT_BF16, &r, &o, -1, 1) == LT_ERR_ARG);
    CHECK(lt_server_submit_map(S, M0, 7, &r, &o, 10, 1) == LT_ERR_DTYPE);
    lt_rays rn = r;
    rn.dz = nullptr;
    CHECK(lt_server_submit_map(S, M0, LT_BF16, &rn, &o, 10, 1) == LT_ERR_ARG);
    maps[0]->version += 1;   // parameters changed, not repacked
    CHECK(lt_server_submit_map(S, M0, LT_BF16, &r, &o, 10, 1) == LT_ERR_STATE);
    maps[0]->version -= 1;
    lt_path bad{1, 3, 2};
    CHECK(lt_server_submit_trace(S, lens, &bad, &r, &e, 10, 1) == LT_ERR_PATH);
    CHECK(lt_server_submit_trace(S, lens, nullptr, &r, &e, 10, 1) == LT_ERR_ARG);
    int32_t nd = 0;
    CHECK(lt_server_poll(nullptr, nullptr, 0, &nd, nullptr) == LT_ERR_ARG);
    CHECK(lt_server_poll(S, nullptr, 3, &nd, nullptr) == LT_ERR_ARG);
    CHECK(lt_server_poll(S, nullptr, 0, nullptr, nullptr) == LT_ERR_ARG);
    CHECK(lt_server_stats(nullptr, nullptr, nullptr) == LT_ERR_ARG);
    CHECK(lt_server_destroy(nullptr) == LT_OK);
    CHECK(lt_server_destroy(S) == LT_OK);
    by_first.erase(b->x.data());
    delete b;
}

}  // namespace

int main()
{
    // a 4-surface lens for the trace requests (its trace tables are built on
    // submission)
    lt_surface s[4] = {{40.0, 5.0, 12.0, 1, 0}, {-30.0, 2.0, 12.0, 0, 0}, {0.0, 3.0, 8.0, 0, 1},
                       {-60.0, 30.0, 12.0, 0, 0}};
    lt_glass g[2] = {{0, 0, {0, 0, 0, 0, 0, 0}}, {1, 0, {1.5168, 0.0042, 0.0, 0, 0, 0}}};
    lt_lens lens = nullptr;
    CHECK(lt_lens_create(s, 4, g, 2, &lens) == LT_OK);
    lt::Map *maps[2];
    for (int k = 0; k < 2; ++k) {
        maps[k] = new lt::Map;
        maps[k]->lay.P = k == 0 ? 1 : 3;
        maps[k]->version = 5;
        maps[k]->packed_bf16 = maps[k]->packed_fp8 = maps[k]->packed_f32 = 5;
    }
    misuse(lens, maps);
    for (int k = 0; k < 400; ++k)
        scenario(lens, maps);
    CHECK(live_streams.empty() && live_events.empty());
    for (lt::Map *m : maps)
        delete m;
    CHECK(lt_lens_destroy(lens) == LT_OK);
    std::printf("serving loop under sanitizers: %d scenarios, %d requests (%d over budget), %lld launches\n",
                n_scenarios, n_requests, n_rejected, static_cast<long long>(fake_launches));
    return n_scenarios == 400 && fake_launches > 1000 ? 0 : 1;
}
