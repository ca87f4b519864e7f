// server.hip -- request server over one resident graph (csaw_server_* in
// include/csaw.h): admission by device-memory budget, continuous batching of
// sampling requests into multi-instance calls, executor threads with their
// own streams so that batches overlap on the device, per-request latency.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/csaw.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int32_t kind = 0;
    uint64_t id = 0, rng_seed = 0;
    int32_t bias = 0;
    std::vector<int32_t> seeds, fanouts, starts;
    int32_t length = 0;
    uint32_t wr = 1, wc = 1, wo = 1;
    int64_t mem = 0;
    Clock::time_point t_submit;
};

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;
    bool ensure(size_t n) {
        if (cap >= n) return true;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        const size_t c = std::max<size_t>(n + n / 4, 1024);
        if (hipMalloc((void**)&p, c * sizeof(T)) != hipSuccess) return false;
        cap = c;
        return true;
    }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

template <class T>
struct HostBuf {
    T* p = nullptr;
    size_t cap = 0;
    bool ensure(size_t n) {
        if (cap >= n) return true;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        const size_t c = std::max<size_t>(n + n / 4, 1024);
        if (hipHostMalloc((void**)&p, c * sizeof(T), hipHostMallocDefault) != hipSuccess) return false;
        cap = c;
        return true;
    }
    ~HostBuf() {
        if (p) (void)hipHostFree(p);
    }
};

double us_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::micro>(b - a).count();
}

}  // namespace

// Buffers of one executor, kept across batches.
struct Exec {
    hipStream_t st = nullptr;
    DevBuf<int32_t> d_seeds, d_src, d_dst, d_starts, d_paths;
    DevBuf<int64_t> d_off;
    HostBuf<int32_t> h_src, h_dst, h_seeds;
    HostBuf<int64_t> h_off;
};

struct csaw_server_s {
    csaw_graph g = nullptr;
    csaw_server_config cfg{};
    int device = 0;
    int64_t n = 0, m = 0, max_deg = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, csaw_result*> done;
    std::unordered_map<uint64_t, bool> known;  // ticket -> not yet handed over
    int64_t inflight_mem = 0;
    int inflight_batches = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;

    void worker();
    void run_sample_batch(std::vector<Request*>& batch, Exec& x, Clock::time_point t0);
    void run_walk(Request* r, Exec& x, Clock::time_point t0);
    void finish(Request* r, csaw_result* res);

};

namespace {

thread_local std::string t_srv_err;

csaw_result* new_result(int32_t kind, csaw_status st) {
    csaw_result* r = (csaw_result*)std::calloc(1, sizeof(csaw_result));
    if (r) {
        r->status = st;
        r->kind = kind;
    }
    return r;
}

int64_t sample_request_mem(const csaw_server_s* s, const Request& r) {
    // edges out (8 B), frontier entries (~36 B), per-instance bitmaps, seeds
    int64_t B = std::min<int64_t>((int64_t)r.seeds.size(), s->n), edges = 0, fr = B;
    for (int32_t f : r.fanouts) {
        if (f == 0) break;
        const int64_t per = f < 0 ? s->max_deg : std::min<int64_t>(f, s->max_deg);
        const int64_t e = std::min<int64_t>(B * per, s->m);
        edges += e;
        B = std::min<int64_t>(e, s->n);
        fr += B;
    }
    const int64_t nwp = ((s->n + 31) / 32 + 3) / 4 * 4;
    return edges * 8 + fr * 36 + nwp * 8 + (int64_t)r.seeds.size() * 4 + 4096;
}

}  // namespace

void csaw_server_s::finish(Request* r, csaw_result* res) {
    std::lock_guard<std::mutex> lk(mu);
    done[r->ticket] = res;
    cv_done.notify_all();
}

void csaw_server_s::run_walk(Request* r, Exec& x, Clock::time_point t0) {
    hipStream_t st = x.st;
    const int64_t nw = (int64_t)r->starts.size();
    const int64_t L1 = (int64_t)r->length + 1;
    csaw_result* res = new_result(CSAW_REQUEST_WALK, CSAW_OK);
    if (!res) return finish(r, nullptr);
    res->num_walkers = nw;
    res->length = r->length;
    res->paths = (int32_t*)std::malloc(std::max<int64_t>(nw * L1, 1) * sizeof(int32_t));
    res->queued_us = us_between(r->t_submit, t0);
    DevBuf<int32_t>& d_starts = x.d_starts;
    DevBuf<int32_t>& d_paths = x.d_paths;
    csaw_status stt = CSAW_OK;
    if (!res->paths || !d_starts.ensure(std::max<int64_t>(nw, 1)) || !d_paths.ensure(std::max<int64_t>(nw * L1, 1)))
        stt = CSAW_ERR_OUT_OF_MEMORY;
    if (stt == CSAW_OK && nw > 0 &&
        hipMemcpyAsync(d_starts.p, r->starts.data(), nw * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess)
        stt = CSAW_ERR_DEVICE;
    if (stt == CSAW_OK) {
        csaw_walk_args a{};
        a.bias_kind = r->bias;
        a.w_return = r->wr;
        a.w_common = r->wc;
        a.w_outward = r->wo;
        a.num_walkers = nw;
        a.starts = d_starts.p;
        a.walker_base = r->id;
        a.length = r->length;
        a.rng_seed = r->rng_seed;
        a.walker_ids = nullptr;
        int64_t steps = 0;
        stt = csaw_walk(g, &a, d_paths.p, &steps, st);
        res->steps = steps;
    }
    if (stt == CSAW_OK && nw > 0 &&
        (hipMemcpyAsync(res->paths, d_paths.p, nw * L1 * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
        stt = CSAW_ERR_DEVICE;
    res->status = stt;
    res->total_us = us_between(r->t_submit, Clock::now());
    finish(r, res);
}

void csaw_server_s::run_sample_batch(std::vector<Request*>& batch, Exec& x, Clock::time_point t0) {
    hipStream_t st = x.st;
    const int32_t ni = (int32_t)batch.size();
    int32_t L = 0;
    for (Request* r : batch) L = std::max<int32_t>(L, (int32_t)r->fanouts.size());
    std::vector<int64_t> offs(ni + 1, 0);
    for (int32_t i = 0; i < ni; ++i) offs[i + 1] = offs[i] + (int64_t)batch[i]->seeds.size();
    std::vector<int32_t> fan((size_t)ni * std::max(L, 1), 0), bias(ni);
    std::vector<uint64_t> ids(ni), keys(ni);
    for (int32_t i = 0; i < ni; ++i) {
        std::copy(batch[i]->fanouts.begin(), batch[i]->fanouts.end(), fan.begin() + (size_t)i * L);
        bias[i] = batch[i]->bias;
        ids[i] = batch[i]->id;
        keys[i] = batch[i]->rng_seed;
    }
    csaw_sample_args a{};
    a.num_instances = ni;
    a.seed_offsets = offs.data();
    a.num_layers = L;
    a.fanouts = fan.data();
    a.fanout_stride = L;
    a.bias_kinds = bias.data();
    a.instance_ids = ids.data();
    a.rng_seeds = keys.data();
    int64_t bound = 0;
    csaw_status stt = csaw_sample_bound(g, &a, &bound);
    DevBuf<int32_t>& d_seeds = x.d_seeds;
    DevBuf<int32_t>& d_src = x.d_src;
    DevBuf<int32_t>& d_dst = x.d_dst;
    DevBuf<int64_t>& d_off = x.d_off;
    HostBuf<int32_t>& h_src = x.h_src;
    HostBuf<int32_t>& h_dst = x.h_dst;
    HostBuf<int64_t>& h_off = x.h_off;
    const size_t noff = (size_t)L * ni + 1;
    if (stt == CSAW_OK &&
        (!d_seeds.ensure(std::max<int64_t>(offs[ni], 1)) || !d_src.ensure(std::max<int64_t>(bound, 1)) ||
         !d_dst.ensure(std::max<int64_t>(bound, 1)) || !d_off.ensure(noff) || !h_off.ensure(noff)))
        stt = CSAW_ERR_OUT_OF_MEMORY;
    if (stt == CSAW_OK && !x.h_seeds.ensure(std::max<int64_t>(offs[ni], 1))) stt = CSAW_ERR_OUT_OF_MEMORY;
    if (stt == CSAW_OK) {
        for (int32_t i = 0; i < ni; ++i)
            std::copy(batch[i]->seeds.begin(), batch[i]->seeds.end(), x.h_seeds.p + offs[i]);
        if (offs[ni] > 0 &&
            hipMemcpyAsync(d_seeds.p, x.h_seeds.p, offs[ni] * sizeof(int32_t), hipMemcpyHostToDevice, st) !=
                hipSuccess)
            stt = CSAW_ERR_DEVICE;
    }
    csaw_sample_out out{};
    if (stt == CSAW_OK) {
        a.seeds = d_seeds.p;
        out.src = d_src.p;
        out.dst = d_dst.p;
        out.edge_capacity = bound;
        out.offsets = d_off.p;
        stt = csaw_sample(g, &a, &out, st);
    }
    if (stt != CSAW_OK) {
        if (ni > 1) {  // isolate: every request on its own, so only a faulty one fails
            for (Request* r : batch) {
                std::vector<Request*> one{r};
                run_sample_batch(one, x, t0);
            }
            return;
        }
        csaw_result* res = new_result(CSAW_REQUEST_SAMPLE, stt);
        if (res) {
            res->queued_us = us_between(batch[0]->t_submit, t0);
            res->total_us = us_between(batch[0]->t_submit, Clock::now());
        }
        return finish(batch[0], res);
    }
    const int64_t ne = out.num_edges;
    if (!h_src.ensure(std::max<int64_t>(ne, 1)) || !h_dst.ensure(std::max<int64_t>(ne, 1)) ||
        (ne > 0 && (hipMemcpyAsync(h_src.p, d_src.p, ne * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipMemcpyAsync(h_dst.p, d_dst.p, ne * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess)) ||
        hipMemcpyAsync(h_off.p, d_off.p, noff * sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        for (Request* r : batch) finish(r, new_result(CSAW_REQUEST_SAMPLE, CSAW_ERR_DEVICE));
        return;
    }
    // the segment offsets come from device memory: check them before they size
    // host copies (monotone, inside [0, ne])
    bool offsets_ok = h_off.p[0] >= 0 && h_off.p[noff - 1] == ne;
    for (size_t j = 1; offsets_ok && j < noff; ++j) offsets_ok = h_off.p[j] >= h_off.p[j - 1];
    if (!offsets_ok) {
        for (Request* r : batch) finish(r, new_result(CSAW_REQUEST_SAMPLE, CSAW_ERR_DEVICE));
        return;
    }
    const Clock::time_point t_end = Clock::now();
    for (int32_t i = 0; i < ni; ++i) {
        Request* r = batch[i];
        const int32_t Li = (int32_t)r->fanouts.size();
        csaw_result* res = new_result(CSAW_REQUEST_SAMPLE, CSAW_OK);
        if (!res) {
            finish(r, nullptr);
            continue;
        }
        int64_t cnt = 0;
        for (int32_t l = 0; l < Li; ++l) cnt += h_off.p[(size_t)l * ni + i + 1] - h_off.p[(size_t)l * ni + i];
        res->num_edges = cnt;
        res->num_layers = Li;
        res->src = (int32_t*)std::malloc(std::max<int64_t>(cnt, 1) * sizeof(int32_t));
        res->dst = (int32_t*)std::malloc(std::max<int64_t>(cnt, 1) * sizeof(int32_t));
        res->layer_offsets = (int64_t*)std::malloc(((size_t)Li + 1) * sizeof(int64_t));
        if (!res->src || !res->dst || !res->layer_offsets) {
            res->status = CSAW_ERR_OUT_OF_MEMORY;
        } else {
            int64_t w = 0;
            for (int32_t l = 0; l < Li; ++l) {
                const int64_t b = h_off.p[(size_t)l * ni + i], e = h_off.p[(size_t)l * ni + i + 1];
                res->layer_offsets[l] = w;
                std::memcpy(res->src + w, h_src.p + b, (e - b) * sizeof(int32_t));
                std::memcpy(res->dst + w, h_dst.p + b, (e - b) * sizeof(int32_t));
                w += e - b;
            }
            res->layer_offsets[Li] = w;
        }
        res->queued_us = us_between(r->t_submit, t0);
        res->total_us = us_between(r->t_submit, t_end);
        finish(r, res);
    }
}

void csaw_server_s::worker() {
    (void)hipSetDevice(device);
    Exec x;
    if (hipStreamCreateWithFlags(&x.st, hipStreamNonBlocking) != hipSuccess) x.st = nullptr;
    for (;;) {
        std::vector<Request*> batch;
        int64_t mem = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (!queue.empty()) {
                    Request* head = queue.front();
                    const bool fits = inflight_mem + head->mem <= cfg.memory_budget_bytes || inflight_batches == 0;
                    if (fits) break;
                } else if (stop) {
                    break;
                }
                cv_work.wait(lk);
            }
            if (queue.empty()) break;  // stop requested and drained
            Request* head = queue.front();
            queue.pop_front();
            batch.push_back(head);
            mem = head->mem;
            if (head->kind == CSAW_REQUEST_SAMPLE) {
                // every sampling request waiting now that still fits joins the batch
                for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < cfg.max_batch;) {
                    Request* r = *it;
                    if (r->kind == CSAW_REQUEST_SAMPLE && inflight_mem + mem + r->mem <= cfg.memory_budget_bytes) {
                        batch.push_back(r);
                        mem += r->mem;
                        it = queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            inflight_mem += mem;
            ++inflight_batches;
        }
        const Clock::time_point t0 = Clock::now();
        if (batch[0]->kind == CSAW_REQUEST_SAMPLE) run_sample_batch(batch, x, t0);
        else run_walk(batch[0], x, t0);
        for (Request* r : batch) delete r;
        {
            std::lock_guard<std::mutex> lk(mu);
            inflight_mem -= mem;
            --inflight_batches;
        }
        cv_work.notify_all();
    }
    if (x.st) (void)hipStreamDestroy(x.st);
}

extern "C" {

csaw_status csaw_server_create(csaw_graph g, const csaw_server_config* cfg, csaw_server* out) {
    if (!g || !out) return CSAW_ERR_INVALID_ARG;
    *out = nullptr;
    csaw_server s = new csaw_server_s();
    s->g = g;
    if (cfg) s->cfg = *cfg;
    if (s->cfg.memory_budget_bytes <= 0) s->cfg.memory_budget_bytes = int64_t(32) << 30;
    if (s->cfg.max_batch <= 0) s->cfg.max_batch = 512;
    if (s->cfg.queue_capacity <= 0) s->cfg.queue_capacity = 65536;
    if (s->cfg.num_streams <= 0) s->cfg.num_streams = 2;
    if (s->cfg.num_streams > 16 || s->cfg.max_batch > (1 << 20)) {
        delete s;
        return CSAW_ERR_INVALID_ARG;
    }
    int32_t sorted = 0;
    csaw_graph_info(g, &s->n, &s->m, &s->max_deg, &sorted);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return CSAW_ERR_DEVICE;
    }
    for (int i = 0; i < s->cfg.num_streams; ++i) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return CSAW_OK;
}

csaw_status csaw_server_submit(csaw_server s, const csaw_request* q, uint64_t* ticket) {
    if (!s || !q || !ticket) return CSAW_ERR_INVALID_ARG;
    Request* r = new Request();
    r->kind = q->kind;
    r->id = q->id;
    r->rng_seed = q->rng_seed;
    r->bias = q->bias_kind;
    if (q->kind == CSAW_REQUEST_SAMPLE) {
        if (q->num_seeds < 0 || (q->num_seeds > 0 && !q->seeds) || q->num_layers < 0 ||
            q->num_layers > CSAW_MAX_LAYERS || (q->num_layers > 0 && !q->fanouts) || q->bias_kind < 0 ||
            q->bias_kind > CSAW_BIAS_NEIGHBOR_DEGREE) {
            delete r;
            return CSAW_ERR_INVALID_ARG;
        }
        r->seeds.assign(q->seeds, q->seeds + q->num_seeds);
        r->fanouts.assign(q->fanouts, q->fanouts + q->num_layers);
        for (int32_t v : r->seeds)
            if (v < 0 || (int64_t)v >= s->n) {
                delete r;
                return CSAW_ERR_INVALID_ARG;
            }
        for (int32_t f : r->fanouts)
            if (f < -1 || f > 0xFFFF) {
                delete r;
                return CSAW_ERR_INVALID_ARG;
            }
        r->mem = sample_request_mem(s, *r);
    } else if (q->kind == CSAW_REQUEST_WALK) {
        if (q->num_walkers < 0 || (q->num_walkers > 0 && !q->starts) || q->length < 0 || q->bias_kind < 0 ||
            q->bias_kind > CSAW_BIAS_METROPOLIS_HASTINGS) {
            delete r;
            return CSAW_ERR_INVALID_ARG;
        }
        r->starts.assign(q->starts, q->starts + q->num_walkers);
        for (int32_t v : r->starts)
            if (v < 0 || (int64_t)v >= s->n) {
                delete r;
                return CSAW_ERR_INVALID_ARG;
            }
        r->length = q->length;
        r->wr = q->w_return;
        r->wc = q->w_common;
        r->wo = q->w_outward;
        r->mem = q->num_walkers * ((int64_t)q->length + 2) * 4 + 4096;
    } else {
        delete r;
        return CSAW_ERR_INVALID_ARG;
    }
    if (r->mem > s->cfg.memory_budget_bytes) {
        delete r;
        return CSAW_ERR_OUT_OF_MEMORY;
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->queue.size() >= s->cfg.queue_capacity || s->stop) {
            delete r;
            return CSAW_ERR_BUSY;
        }
        r->ticket = s->next_ticket++;
        s->known[r->ticket] = true;
        *ticket = r->ticket;
        s->queue.push_back(r);
    }
    s->cv_work.notify_one();
    return CSAW_OK;
}

static csaw_status take_result(csaw_server s, uint64_t ticket, csaw_result** result) {
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return CSAW_ERR_NOT_READY;
    *result = it->second;
    s->done.erase(it);
    s->known.erase(ticket);
    return *result ? CSAW_OK : CSAW_ERR_OUT_OF_MEMORY;
}

csaw_status csaw_server_poll(csaw_server s, uint64_t ticket, csaw_result** result) {
    if (!s || !result) return CSAW_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return CSAW_ERR_INVALID_ARG;
    return take_result(s, ticket, result);
}

csaw_status csaw_server_wait(csaw_server s, uint64_t ticket, int64_t timeout_us, csaw_result** result) {
    if (!s || !result) return CSAW_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return CSAW_ERR_INVALID_ARG;
    auto ready = [&] { return s->done.count(ticket) > 0; };
    if (timeout_us < 0) s->cv_done.wait(lk, ready);
    else s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    return take_result(s, ticket, result);
}

void csaw_result_free(csaw_result* r) {
    if (!r) return;
    std::free(r->src);
    std::free(r->dst);
    std::free(r->layer_offsets);
    std::free(r->paths);
    std::free(r);
}

csaw_status csaw_server_destroy(csaw_server s) {
    if (!s) return CSAW_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->done) csaw_result_free(kv.second);
    delete s;
    return CSAW_OK;
}

}  // extern "C"
