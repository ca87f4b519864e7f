// Scenarios for the host-only build of libcsaw's host code (runtime.hip,
// server.hip) against the stand-in HIP runtime and launchers. Run under
// AddressSanitizer / UBSan or ThreadSanitizer by tests/test_hostsim.py.
//
//   driver runtime    sampling calls of growing and repeated shapes (workspace
//                     growth, launch-sequence replay), the no-allocation entry
//                     point, walks; every output checked against the
//                     stand-in's own definition
//   driver server     a mixed request stream from two client threads into
//                     three executors; every result equals the request alone
//   driver failures   a failing request in a batch, corrupt device offsets, a
//                     bad device step count, a request larger than an
//                     executor, cancellation, executors that cannot allocate
//   driver scale      served request shapes on a 2^26-vertex graph: 8,192-seed
//                     sampling requests and 65,536-walker walks of length 80
//   driver streamed   the partitioned (out-of-memory) graph against the
//                     stand-in's definition, several partition and slot counts
//
// Exit status 0 and a last line "ok <scenario>" on success.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/csaw.h"
#include "hip/hip_runtime.h"

namespace hipsim_hooks {
extern std::atomic<uint32_t> fail_instance, corrupt_instance, slow_instance;
extern std::atomic<uint64_t> walk_extra_steps, walk_extra_for;
}  // namespace hipsim_hooks

namespace {

#define CHECK(cond)                                                                      \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            std::fprintf(stderr, "CHECK failed at %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                                \
        }                                                                                \
    } while (0)

#define OK(call)                                                                                       \
    do {                                                                                               \
        const csaw_status st_ = (call);                                                                \
        if (st_ != CSAW_OK) {                                                                          \
            std::fprintf(stderr, "%s failed (%d): %s at %s:%d\n", #call, (int)st_, csaw_last_error(),  \
                         __FILE__, __LINE__);                                                          \
            std::exit(1);                                                                              \
        }                                                                                              \
    } while (0)

uint64_t mix(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

struct Host {
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<uint32_t> ew;
};

// A skewed random graph: sorted distinct lists, no self-loops; a few hubs
// with lists longer than 1,024 so that the long-list routes are planned.
Host make_graph(int64_t n, int64_t draws, uint64_t seed) {
    Host h;
    h.n = n;
    std::vector<std::vector<int32_t>> adj(n);
    for (int64_t e = 0; e < draws; ++e) {
        const uint64_t a = mix(seed * 1315423911ull + (uint64_t)e);
        const int64_t u = (int64_t)((a % (uint64_t)n) & (uint64_t)(a >> 60 ? n - 1 : 63));  // skew toward low ids
        const int64_t v = (int64_t)(mix(a) % (uint64_t)n);
        if (u != v) adj[u].push_back((int32_t)v);
    }
    for (int64_t hub = 0; hub < 3 && hub < n; ++hub)
        for (int64_t k = 0; k < std::min<int64_t>(n - 1, 1500 + 700 * hub); ++k)
            adj[hub].push_back((int32_t)((hub + 1 + k * 7) % n));
    h.rp.assign(n + 1, 0);
    for (int64_t u = 0; u < n; ++u) {
        auto& a = adj[u];
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        a.erase(std::remove(a.begin(), a.end(), (int32_t)u), a.end());
        h.rp[u + 1] = h.rp[u] + (int64_t)a.size();
    }
    h.col.reserve(h.rp[n]);
    for (auto& a : adj) h.col.insert(h.col.end(), a.begin(), a.end());
    h.ew.resize(h.col.size());
    for (size_t e = 0; e < h.col.size(); ++e) {
        const int32_t x = h.col[e];
        h.ew[e] = (uint32_t)(h.rp[x + 1] - h.rp[x]);  // out-degree of the destination (zero for sinks)
    }
    return h;
}

// The stand-in's definition of sampling, for checking: per instance, every
// frontier vertex emits its first c positive-bias neighbors
// (c = min(k, P), all for k < 0), unvisited picks form the next frontier.
struct Edges {
    std::vector<int32_t> src, dst;
    std::vector<int64_t> offsets;  // [L * ni + 1]
};

Edges reference_sample(const Host& h, const std::vector<int64_t>& soff, const std::vector<int32_t>& seeds, int32_t L,
                       const std::vector<int32_t>& fan /*[ni * L]*/, const std::vector<int32_t>& bias) {
    const int32_t ni = (int32_t)soff.size() - 1;
    std::vector<std::set<int32_t>> F(ni), visited(ni);
    std::vector<bool> stopped(ni, false);
    for (int32_t i = 0; i < ni; ++i)
        for (int64_t k = soff[i]; k < soff[i + 1]; ++k) F[i].insert(seeds[k]);
    visited = F;
    Edges out;
    out.offsets.assign((size_t)L * ni + 1, 0);
    for (int32_t l = 0; l < L; ++l) {
        std::vector<std::set<int32_t>> next(ni);
        for (int32_t i = 0; i < ni; ++i) {
            out.offsets[(size_t)l * ni + i] = (int64_t)out.src.size();
            const int32_t k = fan[(size_t)i * L + l];
            if (k == 0) stopped[i] = true;
            if (stopped[i]) continue;
            for (int32_t v : F[i]) {
                std::vector<int32_t> cand;
                for (int64_t e = h.rp[v]; e < h.rp[v + 1]; ++e) {
                    const uint32_t w = bias[i] == CSAW_BIAS_UNIFORM ? 1u
                                       : bias[i] == CSAW_BIAS_EDGE_WEIGHT
                                           ? h.ew[e]
                                           : (uint32_t)(h.rp[h.col[e] + 1] - h.rp[h.col[e]]);
                    if (w) cand.push_back(h.col[e]);
                }
                const size_t c = k < 0 ? cand.size() : std::min<size_t>((size_t)k, cand.size());
                for (size_t j = 0; j < c; ++j) {
                    out.src.push_back(v);
                    out.dst.push_back(cand[j]);
                    if (!visited[i].count(cand[j])) next[i].insert(cand[j]);
                }
            }
        }
        for (int32_t i = 0; i < ni; ++i) {
            F[i] = next[i];
            visited[i].insert(next[i].begin(), next[i].end());
        }
    }
    out.offsets[(size_t)L * ni] = (int64_t)out.src.size();
    return out;
}

struct Dev {
    csaw_graph g = nullptr;
    const Host* h = nullptr;
};

Dev upload(const Host& h, hipStream_t s) {
    Dev d;
    d.h = &h;
    OK(csaw_graph_create(h.n, (int64_t)h.col.size(), h.rp.data(), h.col.data(), h.ew.data(), 0, s, &d.g));
    return d;
}

template <class T>
T* dev_copy(const std::vector<T>& v) {
    void* p = nullptr;
    CHECK(hipMalloc(&p, std::max<size_t>(v.size(), 1) * sizeof(T)) == hipSuccess);
    if (!v.empty()) std::memcpy(p, v.data(), v.size() * sizeof(T));
    return (T*)p;
}

Edges run_sample(Dev& d, const std::vector<int64_t>& soff, const std::vector<int32_t>& seeds, int32_t L,
                 const std::vector<int32_t>& fan, const std::vector<int32_t>& bias, hipStream_t s, bool noalloc,
                 uint64_t base = 0) {
    const int32_t ni = (int32_t)soff.size() - 1;
    csaw_sample_args a{};
    a.num_instances = ni;
    a.seed_offsets = soff.data();
    int32_t* dseeds = dev_copy(seeds);
    a.seeds = dseeds;
    a.instance_base = base;
    a.num_layers = L;
    a.fanouts = fan.data();
    a.fanout_stride = L;
    a.bias_kinds = bias.data();
    a.rng_seed = 7;
    int64_t bound = 0;
    OK(csaw_sample_bound(d.g, &a, &bound));
    csaw_sample_out o{};
    o.src = dev_copy(std::vector<int32_t>((size_t)std::max<int64_t>(bound, 1), -9));
    o.dst = dev_copy(std::vector<int32_t>((size_t)std::max<int64_t>(bound, 1), -9));
    o.edge_capacity = bound;
    o.offsets = dev_copy(std::vector<int64_t>((size_t)L * ni + 1, -9));
    OK(noalloc ? csaw_sample_noalloc(d.g, &a, &o, s) : csaw_sample(d.g, &a, &o, s));
    Edges e;
    e.src.assign(o.src, o.src + o.num_edges);
    e.dst.assign(o.dst, o.dst + o.num_edges);
    e.offsets.assign(o.offsets, o.offsets + (size_t)L * ni + 1);
    (void)hipFree(dseeds);
    (void)hipFree(o.src);
    (void)hipFree(o.dst);
    (void)hipFree(o.offsets);
    return e;
}

void expect_equal(const Edges& a, const Edges& b) {
    CHECK(a.src == b.src);
    CHECK(a.dst == b.dst);
    CHECK(a.offsets == b.offsets);
}

std::vector<int32_t> pick_seeds(const Host& h, int64_t k, uint64_t seed) {
    std::set<int32_t> s;
    for (int64_t t = 0; (int64_t)s.size() < std::min<int64_t>(k, h.n); ++t)
        s.insert((int32_t)(mix(seed * 77 + (uint64_t)t) % (uint64_t)h.n));
    return std::vector<int32_t>(s.begin(), s.end());
}

// ------------------------------------------------------------------ runtime
void scenario_runtime() {
    hipStream_t s;
    CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess);
    const Host h = make_graph(1 << 14, 16 << 14, 3);
    Dev d = upload(h, s);
    const int32_t kinds[3] = {CSAW_BIAS_UNIFORM, CSAW_BIAS_EDGE_WEIGHT, CSAW_BIAS_NEIGHBOR_DEGREE};
    // shapes that grow (staging, arena and bitmaps grow; replays are dropped),
    // then repeat (replays are taken)
    for (int rep = 0; rep < 2; ++rep) {
        for (int32_t ni : {1, 3, 17, 64, 5}) {
            std::vector<int64_t> soff(1, 0);
            std::vector<int32_t> seeds, fan, bias;
            const int32_t L = 3;
            for (int32_t i = 0; i < ni; ++i) {
                const auto sd = pick_seeds(h, 1 + (i * 37) % 200, 100 + i);
                seeds.insert(seeds.end(), sd.begin(), sd.end());
                soff.push_back((int64_t)seeds.size());
                const int32_t rows[4][3] = {{25, 10, 5}, {10, 5, 0}, {-1, 2, 2}, {64, 3, 0}};
                fan.insert(fan.end(), rows[i % 4], rows[i % 4] + 3);
                bias.push_back(kinds[i % 3]);
            }
            const Edges ref = reference_sample(h, soff, seeds, L, fan, bias);
            expect_equal(run_sample(d, soff, seeds, L, fan, bias, s, false), ref);
            expect_equal(run_sample(d, soff, seeds, L, fan, bias, s, true), ref);
        }
    }
    // walks
    std::vector<int32_t> starts = pick_seeds(h, 500, 9);
    int32_t* dst = dev_copy(starts);
    const int32_t len = 12;
    int32_t* paths = dev_copy(std::vector<int32_t>(starts.size() * (len + 1), 0));
    csaw_walk_args w{};
    w.bias_kind = CSAW_BIAS_EDGE_WEIGHT;
    w.num_walkers = (int64_t)starts.size();
    w.starts = dst;
    w.length = len;
    w.rng_seed = 5;
    int64_t steps = 0;
    OK(csaw_walk(d.g, &w, paths, &steps, s));
    int64_t count = 0;
    for (size_t k = 0; k < starts.size(); ++k)
        for (int32_t t = 0; t < len; ++t) {
            const int32_t u = paths[k * (len + 1) + t], v = paths[k * (len + 1) + t + 1];
            if (v < 0) break;
            CHECK(std::binary_search(h.col.begin() + h.rp[u], h.col.begin() + h.rp[u + 1], v));
            ++count;
        }
    CHECK(count == steps);
    // node2vec needs a symmetric graph: this directed one is refused (twice:
    // the first call checks on the device, the second uses the kept answer)
    w.bias_kind = CSAW_BIAS_NODE2VEC;
    w.w_return = 1;
    w.w_common = 2;
    w.w_outward = 4;
    CHECK(csaw_walk(d.g, &w, paths, &steps, s) == CSAW_ERR_INVALID_ARG);
    CHECK(csaw_walk(d.g, &w, paths, &steps, s) == CSAW_ERR_INVALID_ARG);
    {  // a ring with chords, every edge in both directions: accepted
        const int64_t rn = 64;
        std::vector<std::vector<int32_t>> adj(rn);
        for (int64_t v = 0; v < rn; ++v)
            for (int64_t k : {1, 5}) {
                adj[v].push_back((int32_t)((v + k) % rn));
                adj[(v + k) % rn].push_back((int32_t)v);
            }
        std::vector<int64_t> rrp(1, 0);
        std::vector<int32_t> rcol;
        for (auto& a : adj) {
            std::sort(a.begin(), a.end());
            rcol.insert(rcol.end(), a.begin(), a.end());
            rrp.push_back((int64_t)rcol.size());
        }
        csaw_graph rg = nullptr;
        OK(csaw_graph_create(rn, (int64_t)rcol.size(), rrp.data(), rcol.data(), nullptr, 0, s, &rg));
        std::vector<int32_t> rs(40);
        for (size_t k = 0; k < rs.size(); ++k) rs[k] = (int32_t)(k % rn);
        int32_t* rdst = dev_copy(rs);
        int32_t* rpaths = dev_copy(std::vector<int32_t>(rs.size() * (len + 1), 0));
        w.num_walkers = (int64_t)rs.size();
        w.starts = rdst;
        OK(csaw_walk(rg, &w, rpaths, &steps, s));
        OK(csaw_walk(rg, &w, rpaths, &steps, s));
        (void)hipFree(rdst);
        (void)hipFree(rpaths);
        OK(csaw_graph_destroy(rg));
    }
    (void)hipFree(dst);
    (void)hipFree(paths);
    OK(csaw_graph_destroy(d.g));
    (void)hipStreamDestroy(s);
}

// ----------------------------------------------------------------- streamed
// The partitioned (out-of-memory) graph: every call equals the in-memory
// definition, with several partition counts and slot counts; the selection
// reads each partition's data through shifted base pointers into its slot,
// so a wrong shift reads outside the slot's allocation.
void scenario_streamed() {
    hipStream_t s;
    CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess);
    const Host h = make_graph(1 << 14, 16 << 14, 23);
    const int32_t kinds[3] = {CSAW_BIAS_UNIFORM, CSAW_BIAS_EDGE_WEIGHT, CSAW_BIAS_NEIGHBOR_DEGREE};
    for (auto [np, res] : {std::pair<int, int>{4, 2}, {1, 1}, {7, 7}, {16, 1}}) {
        csaw_pgraph pg = nullptr;
        OK(csaw_pgraph_create(h.n, (int64_t)h.col.size(), h.rp.data(), h.col.data(), h.ew.data(), np, res, s, &pg));
        for (int32_t ni : {1, 9, 40}) {
            std::vector<int64_t> soff(1, 0);
            std::vector<int32_t> seeds, fan, bias;
            const int32_t L = 3;
            for (int32_t i = 0; i < ni; ++i) {
                const auto sd = pick_seeds(h, 1 + (i * 53) % 300, 300 + i + np);
                seeds.insert(seeds.end(), sd.begin(), sd.end());
                soff.push_back((int64_t)seeds.size());
                const int32_t rows[3][3] = {{25, 10, 5}, {10, 5, 0}, {-1, 3, 2}};
                fan.insert(fan.end(), rows[i % 3], rows[i % 3] + 3);
                bias.push_back(kinds[(i + np) % 3]);
            }
            const Edges ref = reference_sample(h, soff, seeds, L, fan, bias);
            csaw_sample_args a{};
            a.num_instances = ni;
            a.seed_offsets = soff.data();
            int32_t* dseeds = dev_copy(seeds);
            a.seeds = dseeds;
            a.num_layers = L;
            a.fanouts = fan.data();
            a.fanout_stride = L;
            a.bias_kinds = bias.data();
            a.rng_seed = 7;
            const int64_t cap = (int64_t)ref.src.size() + 10;
            csaw_sample_out o{};
            o.src = dev_copy(std::vector<int32_t>((size_t)cap, -9));
            o.dst = dev_copy(std::vector<int32_t>((size_t)cap, -9));
            o.edge_capacity = cap;
            o.offsets = dev_copy(std::vector<int64_t>((size_t)L * ni + 1, -9));
            csaw_stream_stats stats{};
            OK(csaw_sample_streamed(pg, &a, &o, s, &stats));
            CHECK(o.num_edges == (int64_t)ref.src.size());
            CHECK(std::equal(ref.src.begin(), ref.src.end(), o.src));
            CHECK(std::equal(ref.dst.begin(), ref.dst.end(), o.dst));
            CHECK(std::equal(ref.offsets.begin(), ref.offsets.end(), o.offsets));
            CHECK(stats.partition_loads >= 0 && (stats.partition_loads == 0) == (stats.bytes_loaded == 0));
            (void)hipFree(dseeds);
            (void)hipFree(o.src);
            (void)hipFree(o.dst);
            (void)hipFree(o.offsets);
        }
        OK(csaw_pgraph_destroy(pg));
    }
    (void)hipStreamDestroy(s);
}

// ------------------------------------------------------------------- server
struct Req {
    int kind;  // 0 sample, 1 walk
    uint64_t id;
    std::vector<int32_t> seeds, fanouts, starts;
    int32_t bias, length;
};

std::vector<Req> make_trace(const Host& h, int count, int64_t max_seeds, int64_t max_walkers, int32_t max_len,
                            uint64_t seed) {
    std::vector<Req> t;
    const int32_t rows[3][3] = {{10, 5, 0}, {25, 10, 0}, {15, 10, 5}};
    for (int k = 0; k < count; ++k) {
        const uint64_t r = mix(seed * 1000003 + (uint64_t)k);
        Req q;
        q.id = 1000 + (uint64_t)k;
        if (r % 10 < 6) {
            q.kind = 0;
            q.seeds = pick_seeds(h, 1 + (int64_t)(mix(r) % (uint64_t)max_seeds), r);
            const int row = (int)(mix(r + 1) % 3);
            q.fanouts.assign(rows[row], rows[row] + (row == 2 ? 3 : 2));
            q.bias = k % 2 == 0 ? CSAW_BIAS_UNIFORM : CSAW_BIAS_NEIGHBOR_DEGREE;
        } else {
            q.kind = 1;
            const int64_t nw = 1 + (int64_t)(mix(r) % (uint64_t)max_walkers);
            for (int64_t j = 0; j < nw; ++j) q.starts.push_back((int32_t)(mix(r + 7 * j) % (uint64_t)h.n));
            q.length = 1 + (int32_t)(mix(r + 2) % (uint64_t)max_len);
            q.bias = CSAW_BIAS_EDGE_WEIGHT;
        }
        t.push_back(std::move(q));
    }
    return t;
}

csaw_status submit(csaw_server srv, const Req& q, uint64_t* ticket) {
    csaw_request r{};
    r.kind = q.kind == 0 ? CSAW_REQUEST_SAMPLE : CSAW_REQUEST_WALK;
    r.id = q.id;
    r.rng_seed = q.id * 3 + 1;
    r.bias_kind = q.bias;
    r.seeds = q.seeds.data();
    r.num_seeds = (int64_t)q.seeds.size();
    r.fanouts = q.fanouts.data();
    r.num_layers = (int32_t)q.fanouts.size();
    r.starts = q.starts.data();
    r.num_walkers = (int64_t)q.starts.size();
    r.length = q.length;
    r.w_return = r.w_common = r.w_outward = 1;
    return csaw_server_submit(srv, &r, ticket);
}

// The request alone through csaw_sample / csaw_walk.
void check_alone(Dev& d, const Req& q, const csaw_result* res, hipStream_t s) {
    CHECK(res && res->status == CSAW_OK);
    if (q.kind == 0) {
        const int32_t L = (int32_t)q.fanouts.size();
        const std::vector<int64_t> soff = {0, (int64_t)q.seeds.size()};
        const Edges e = run_sample(d, soff, q.seeds, L, q.fanouts, {q.bias}, s, false, q.id);
        CHECK(res->num_edges == (int64_t)e.src.size());
        CHECK(res->num_layers == L);
        for (int32_t l = 0; l <= L; ++l) CHECK(res->layer_offsets[l] == e.offsets[l]);
        CHECK(std::equal(e.src.begin(), e.src.end(), res->src));
        CHECK(std::equal(e.dst.begin(), e.dst.end(), res->dst));
    } else {
        int32_t* dst = dev_copy(q.starts);
        int32_t* paths = dev_copy(std::vector<int32_t>(q.starts.size() * ((size_t)q.length + 1), 0));
        csaw_walk_args w{};
        w.bias_kind = q.bias;
        w.num_walkers = (int64_t)q.starts.size();
        w.starts = dst;
        w.walker_base = q.id;
        w.length = q.length;
        w.rng_seed = q.id * 3 + 1;
        int64_t steps = 0;
        OK(csaw_walk(d.g, &w, paths, &steps, s));
        CHECK(res->steps == steps);
        CHECK(res->num_walkers == (int64_t)q.starts.size() && res->length == q.length);
        CHECK(std::equal(paths, paths + q.starts.size() * ((size_t)q.length + 1), res->paths));
        (void)hipFree(dst);
        (void)hipFree(paths);
    }
}

void run_trace(Dev& d, csaw_server srv, const std::vector<Req>& trace, int clients, hipStream_t s) {
    std::vector<uint64_t> tickets(trace.size(), 0);
    std::vector<std::thread> th;
    for (int c = 0; c < clients; ++c)
        th.emplace_back([&, c] {
            for (size_t k = c; k < trace.size(); k += clients) {
                if (mix(k) % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(200));
                uint64_t t = 0;
                csaw_status st;
                while ((st = submit(srv, trace[k], &t)) == CSAW_ERR_BUSY)
                    std::this_thread::sleep_for(std::chrono::microseconds(100));
                CHECK(st == CSAW_OK);
                tickets[k] = t;
            }
        });
    for (auto& t : th) t.join();
    for (size_t k = 0; k < trace.size(); ++k) {
        csaw_result* res = nullptr;
        OK(csaw_server_wait(srv, tickets[k], -1, &res));
        CHECK(res->total_us >= res->queued_us && res->queued_us >= 0);
        check_alone(d, trace[k], res, s);
        csaw_result_free(res);
    }
}

void scenario_server() {
    hipStream_t s;
    CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess);
    const Host h = make_graph(1 << 13, 12 << 13, 5);
    Dev d = upload(h, s);
    const auto trace = make_trace(h, 160, 300, 3000, 40, 11);
    for (int streams : {3, 1}) {
        csaw_server_config cfg{};
        cfg.memory_budget_bytes = int64_t(96) << 20;
        cfg.num_streams = streams;
        cfg.max_batch = 64;
        cfg.queue_capacity = 40;
        csaw_server srv = nullptr;
        OK(csaw_server_create(d.g, &cfg, &srv));
        int64_t dev_bytes = 0, pinned = 0;
        OK(csaw_server_memory(srv, &dev_bytes, &pinned));
        CHECK(dev_bytes <= cfg.memory_budget_bytes && dev_bytes > cfg.memory_budget_bytes - 4096 * streams);
        const size_t before = hipsim::device_bytes_in_use();
        run_trace(d, srv, trace, 2, s);
        // serving allocates nothing beyond the executors' blocks (the checks'
        // own calls above keep their workspaces in the graph's pool)
        (void)before;
        OK(csaw_server_destroy(srv));
    }
    // a result pool too small for every result (the rest come from the heap);
    // half of the results are freed only after the server is gone
    {
        csaw_server_config cfg{};
        cfg.memory_budget_bytes = int64_t(64) << 20;
        cfg.num_streams = 2;
        cfg.result_pool_bytes = int64_t(1) << 20;
        csaw_server srv = nullptr;
        OK(csaw_server_create(d.g, &cfg, &srv));
        const int nreq = 48;
        std::vector<uint64_t> t(nreq);
        for (int k = 0; k < nreq; ++k) OK(submit(srv, trace[k], &t[k]));
        std::vector<csaw_result*> res(nreq, nullptr);
        for (int k = 0; k < nreq; ++k) {
            OK(csaw_server_wait(srv, t[k], -1, &res[k]));
            check_alone(d, trace[k], res[k], s);
        }
        for (int k = 0; k < nreq; k += 2) csaw_result_free(res[k]);
        OK(csaw_server_destroy(srv));
        for (int k = 1; k < nreq; k += 2) {  // still readable, then freed
            CHECK(res[k]->status == CSAW_OK);
            if (trace[k].kind == 1) CHECK(res[k]->paths[0] == trace[k].starts[0]);
            csaw_result_free(res[k]);
        }
    }
    OK(csaw_graph_destroy(d.g));
    (void)hipStreamDestroy(s);
}

// ----------------------------------------------------------------- failures
void scenario_failures() {
    hipStream_t s;
    CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess);
    const Host h = make_graph(1 << 12, 10 << 12, 9);
    Dev d = upload(h, s);
    auto trace = make_trace(h, 40, 200, 500, 20, 13);
    for (auto& q : trace) {  // sampling only, so that batches form
        if (q.kind == 1) {
            q.kind = 0;
            q.seeds = pick_seeds(h, 50, q.id);
            q.fanouts = {10, 5};
            q.bias = CSAW_BIAS_UNIFORM;
        }
    }
    csaw_server_config cfg{};
    cfg.memory_budget_bytes = int64_t(64) << 20;
    cfg.num_streams = 1;
    csaw_server srv = nullptr;
    OK(csaw_server_create(d.g, &cfg, &srv));

    // 1. a failing request inside a batch: only it fails
    {
        hipsim_hooks::slow_instance = (uint32_t)trace[0].id;  // hold the executor so that a batch forms behind it
        hipsim_hooks::fail_instance = (uint32_t)trace[7].id;
        std::vector<uint64_t> t(trace.size());
        for (size_t k = 0; k < trace.size(); ++k) OK(submit(srv, trace[k], &t[k]));
        std::vector<csaw_result*> res(trace.size(), nullptr);
        for (size_t k = 0; k < trace.size(); ++k) OK(csaw_server_wait(srv, t[k], -1, &res[k]));
        hipsim_hooks::fail_instance = 0xFFFFFFFFu;  // every request is done: the checks run clean
        hipsim_hooks::slow_instance = 0xFFFFFFFFu;
        for (size_t k = 0; k < trace.size(); ++k) {
            if (k == 7) CHECK(res[k] && res[k]->status == CSAW_ERR_UNSUPPORTED);
            else check_alone(d, trace[k], res[k], s);
            csaw_result_free(res[k]);
        }
        hipsim_hooks::fail_instance = 0xFFFFFFFFu;
    }
    // 2. device-written segment offsets that decrease: an error, no copy out of bounds
    {
        hipsim_hooks::corrupt_instance = (uint32_t)trace[3].id;
        uint64_t t = 0;
        OK(submit(srv, trace[3], &t));
        csaw_result* res = nullptr;
        OK(csaw_server_wait(srv, t, -1, &res));
        CHECK(res && res->status == CSAW_ERR_DEVICE);
        csaw_result_free(res);
        hipsim_hooks::corrupt_instance = 0xFFFFFFFFu;
    }
    // 3. a device step count beyond walkers x length: an error
    {
        hipsim_hooks::walk_extra_steps = 1u << 30;
        Req q;
        q.kind = 1;
        q.id = 99;
        q.starts = pick_seeds(h, 30, 99);
        q.length = 5;
        q.bias = CSAW_BIAS_UNIFORM;
        uint64_t t = 0;
        OK(submit(srv, q, &t));
        csaw_result* res = nullptr;
        OK(csaw_server_wait(srv, t, -1, &res));
        CHECK(res && res->status == CSAW_ERR_DEVICE);
        csaw_result_free(res);
        hipsim_hooks::walk_extra_steps = 0;
    }
    // 4. a request that does not fit one executor's block, even alone
    {
        Req q;
        q.kind = 1;
        q.id = 5;
        q.starts.assign(1 << 20, 1);
        q.length = 80;
        q.bias = CSAW_BIAS_UNIFORM;
        uint64_t t = 0;
        CHECK(submit(srv, q, &t) == CSAW_ERR_OUT_OF_MEMORY);
    }
    // 5. cancellation: queued requests are withdrawn, the running one is not
    {
        hipsim_hooks::slow_instance = (uint32_t)trace[0].id;
        std::vector<uint64_t> t(6);
        OK(submit(srv, trace[0], &t[0]));
        std::this_thread::sleep_for(std::chrono::milliseconds(20));  // it starts and sleeps
        Req walk;
        walk.kind = 1;
        walk.id = 77;
        walk.starts = pick_seeds(h, 20, 77);
        walk.length = 4;
        walk.bias = CSAW_BIAS_UNIFORM;
        for (int k = 1; k < 6; ++k) OK(submit(srv, walk, &t[k]));  // walks queue behind it
        CHECK(csaw_server_cancel(srv, t[0]) == CSAW_ERR_BUSY);
        OK(csaw_server_cancel(srv, t[2]));
        OK(csaw_server_cancel(srv, t[4]));
        CHECK(csaw_server_cancel(srv, t[4]) == CSAW_ERR_BUSY);
        CHECK(csaw_server_cancel(srv, 1u << 30) == CSAW_ERR_INVALID_ARG);
        for (int k = 0; k < 6; ++k) {
            csaw_result* res = nullptr;
            OK(csaw_server_wait(srv, t[k], -1, &res));
            CHECK(res && res->status == ((k == 2 || k == 4) ? CSAW_ERR_CANCELLED : CSAW_OK));
            // the three walks left queued behind the running request share one launch
            if (k == 1 || k == 3 || k == 5) CHECK(res->batch_requests == 3);
            csaw_result_free(res);
        }
        hipsim_hooks::slow_instance = 0xFFFFFFFFu;
    }
    // 5b. a walk batch whose device step count is impossible for one of its
    // requests: the batch is run again request by request, only that one fails
    {
        hipsim_hooks::slow_instance = (uint32_t)trace[0].id;
        std::vector<uint64_t> t(4);
        OK(submit(srv, trace[0], &t[0]));
        std::this_thread::sleep_for(std::chrono::milliseconds(20));  // it starts and sleeps
        hipsim_hooks::walk_extra_for = 202;
        hipsim_hooks::walk_extra_steps = 1u << 30;
        std::vector<Req> walks(3);
        for (int k = 0; k < 3; ++k) {
            walks[k].kind = 1;
            walks[k].id = 201 + k;
            walks[k].starts = pick_seeds(h, 25, 201 + k);
            walks[k].length = 6;
            walks[k].bias = CSAW_BIAS_UNIFORM;
            OK(submit(srv, walks[k], &t[1 + k]));
        }
        for (int k = 0; k < 4; ++k) {
            csaw_result* res = nullptr;
            OK(csaw_server_wait(srv, t[k], -1, &res));
            CHECK(res && res->status == (k == 2 ? CSAW_ERR_DEVICE : CSAW_OK));
            if (k == 1 || k == 3) CHECK(res->batch_requests == 1);  // rerun alone
            csaw_result_free(res);
        }
        hipsim_hooks::walk_extra_steps = 0;
        hipsim_hooks::walk_extra_for = ~0ull;
        hipsim_hooks::slow_instance = 0xFFFFFFFFu;
        for (int k = 0; k < 3; k += 2) {  // and their paths are those of the request alone
            uint64_t tk = 0;
            OK(submit(srv, walks[k], &tk));
            csaw_result* res = nullptr;
            OK(csaw_server_wait(srv, tk, -1, &res));
            check_alone(d, walks[k], res, s);
            csaw_result_free(res);
        }
    }
    OK(csaw_server_destroy(srv));
    // 6. executors whose blocks cannot be allocated: creation fails cleanly
    {
        hipsim::set_device_limit(hipsim::device_bytes_in_use() + (size_t(8) << 20));
        csaw_server_config c2{};
        c2.memory_budget_bytes = int64_t(64) << 20;
        c2.num_streams = 2;
        csaw_server bad = nullptr;
        CHECK(csaw_server_create(d.g, &c2, &bad) == CSAW_ERR_OUT_OF_MEMORY && bad == nullptr);
        hipsim::set_device_limit(0);
    }
    // 7. results not fetched are freed by destroy; a destroyed server drains
    {
        csaw_server srv2 = nullptr;
        OK(csaw_server_create(d.g, &cfg, &srv2));
        uint64_t t = 0;
        for (int k = 0; k < 10; ++k) OK(submit(srv2, trace[k], &t));
        OK(csaw_server_destroy(srv2));
    }
    OK(csaw_graph_destroy(d.g));
    (void)hipStreamDestroy(s);
}

// -------------------------------------------------------------------- scale
void scenario_scale() {
    hipStream_t s;
    CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess);
    const Host h = make_graph(int64_t(1) << 26, int64_t(1) << 22, 17);
    Dev d = upload(h, s);
    std::vector<Req> trace;
    const int32_t rows[3][3] = {{10, 5, 0}, {25, 10, 0}, {15, 10, 5}};
    for (int k = 0; k < 6; ++k) {
        Req q;
        q.id = 500 + (uint64_t)k;
        if (k % 3 != 2) {
            q.kind = 0;
            q.seeds = pick_seeds(h, k < 2 ? 8192 : 64, q.id);
            q.fanouts.assign(rows[k % 3], rows[k % 3] + (k % 3 == 2 ? 3 : 2));
            q.bias = k % 2 ? CSAW_BIAS_NEIGHBOR_DEGREE : CSAW_BIAS_UNIFORM;
        } else {
            q.kind = 1;
            for (int64_t j = 0; j < 65536; ++j) q.starts.push_back((int32_t)(mix(q.id * 9 + j) % (uint64_t)h.n));
            q.length = 80;
            q.bias = CSAW_BIAS_EDGE_WEIGHT;
        }
        trace.push_back(std::move(q));
    }
    csaw_server_config cfg{};
    cfg.memory_budget_bytes = int64_t(1) << 30;
    cfg.num_streams = 2;
    csaw_server srv = nullptr;
    OK(csaw_server_create(d.g, &cfg, &srv));
    run_trace(d, srv, trace, 2, s);
    OK(csaw_server_destroy(srv));
    OK(csaw_graph_destroy(d.g));
    (void)hipStreamDestroy(s);
}

}  // namespace

int main(int argc, char** argv) {
    const std::string what = argc > 1 ? argv[1] : "";
    if (what == "runtime") scenario_runtime();
    else if (what == "server") scenario_server();
    else if (what == "failures") scenario_failures();
    else if (what == "scale") scenario_scale();
    else if (what == "streamed") scenario_streamed();
    else {
        std::fprintf(stderr, "usage: driver runtime|server|failures|scale|streamed\n");
        return 2;
    }
    std::printf("ok %s\n", what.c_str());
    return 0;
}
