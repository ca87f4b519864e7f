// Stand-in launchers for the host-only build of libcsaw's host code (see
// hip/hip_runtime.h). Test infrastructure only.
//
// Each launcher enqueues a host function on the stream that produces outputs
// of the real kernels' shape and bookkeeping -- frontier entries with their
// counts, offsets and routes, control-block totals, segment offsets, claimed
// picks, walk paths -- so that the runtime's and the server's sizing,
// staging, replay and result handling run on real sizes. The selection itself
// is a deterministic placeholder (the first positive-bias neighbors of a
// list; a hashed neighbor per walk step), not the sampling method: these
// tests are about the host code, and a result depends only on its own
// request, as the real one does.
#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "../../paper_2009_09103_amd/csrc/kernels.h"

namespace hipsim_hooks {
// Failure and delay injection (set by the driver before the calls it affects).
std::atomic<uint32_t> fail_instance{0xFFFFFFFFu};    // a call holding this instance id reports UNSUPPORTED
std::atomic<uint32_t> corrupt_instance{0xFFFFFFFFu}; // ... writes decreasing segment offsets
std::atomic<uint32_t> slow_instance{0xFFFFFFFFu};    // ... takes 50 ms
std::atomic<uint64_t> walk_extra_steps{0};           // walks report this many steps too many ...
std::atomic<uint64_t> walk_extra_for{~0ull};         // ... only the request with this walker base (all: ~0)
}  // namespace hipsim_hooks

namespace csaw {

namespace {

int32_t positive_count(const GraphDev& g, int32_t kind, int32_t v, int64_t d, bool& wide) {
    wide = false;
    if (kind == kUniform) return (int32_t)d;
    const int32_t p = kind == kEdgeWeight ? g.ppos_ew[v] : g.ppos_deg[v];
    wide = (p & kWideList) != 0;
    return p & ~kWideList;
}

const uint32_t* weights(const GraphDev& g, int32_t kind) {
    return kind == kEdgeWeight ? g.ew : kind == kNeighborDegree ? g.degw : nullptr;
}

uint64_t mix(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

void launch_partition_work(const int32_t* fv, const int32_t* cnt, const SampleCtl* ctl, int32_t layer, int64_t,
                           const int64_t* bounds, int32_t np, unsigned long long* work, hipStream_t s) {
    hipsim::enqueue(s, [=] {
        for (int64_t e = 0; e < ctl->fcount[layer]; ++e) {
            int32_t q = 0;
            while (q + 1 < np && bounds[q + 1] <= fv[e]) ++q;
            work[2 * q] += 1;
            work[2 * q + 1] += (unsigned long long)cnt[e];
        }
    });
}

void launch_scatter_segments(const int32_t* src, const int32_t* dst, const int64_t* off, int64_t nseg,
                             int64_t total, int32_t* const* to_src, int32_t* const* to_dst, hipStream_t s) {
    if (nseg <= 0 || total <= 0) return;
    hipsim::enqueue(s, [=] {
        if (total != off[nseg]) abort();  // the launcher's grid is sized by total
        for (int64_t j = 0; j < nseg; ++j) {
            if (!to_src[j] || !to_dst[j]) continue;
            for (int64_t k = off[j]; k < off[j + 1]; ++k) {
                to_src[j][k - off[j]] = src[k];
                to_dst[j][k - off[j]] = dst[k];
            }
        }
    });
}

void launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    hipsim::enqueue(s, [=] { std::fill(p, p + count, value); });
}

void launch_degree_weights(RowPtr rowptr, const int32_t* col, int64_t m, uint32_t* degw, hipStream_t s) {
    hipsim::enqueue(s, [=] {
        for (int64_t e = 0; e < m; ++e) degw[e] = (uint32_t)(rowptr[col[e] + 1] - rowptr[col[e]]);
    });
}

void launch_positive_counts(RowPtr rowptr, const uint32_t* w, int64_t n, int32_t* ppos, uint64_t* wtot,
                            hipStream_t s) {
    hipsim::enqueue(s, [=] {
        for (int64_t v = 0; v < n; ++v) {
            int64_t c = 0;
            uint64_t t = 0;
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                c += w[e] > 0;
                t += w[e];
            }
            ppos[v] = (int32_t)c | ((t >> 32) ? kWideList : 0);
            wtot[v] = t;
        }
    });
}

int64_t chunk_table_rows(int64_t m) { return (m >> kTabShift) + 1; }

void launch_chunk_table(RowPtr rowptr, const uint32_t* w, int64_t n, uint64_t* tab, uint64_t* ctab,
                        hipStream_t s) {
    hipsim::enqueue(s, [=] {
        for (int64_t v = 0; v < n; ++v) {
            const int64_t b = rowptr[v], d = rowptr[v + 1] - b;
            if (d <= kWaveMaxD) continue;
            uint64_t* row = tab + (b >> kTabShift) * kChunkGroups;
            uint64_t run = 0;
            for (int64_t j = 0; j * kChunk < d; ++j) {
                uint64_t acc = 0;
                for (int q = 0; q < kChunkGroups; ++q) {
                    for (int i = 0; i < 16; ++i) {
                        const int64_t e = j * kChunk + q * 16 + i;
                        if (e < d) acc += w[b + e];
                    }
                    row[j * kChunkGroups + q] = acc;
                }
                run += acc;
                if (ctab) ctab[(b >> kTabShift) + j] = run;
            }
        }
    });
}

void launch_mark_seeds(const int32_t* seeds, int64_t num_seeds, const int64_t* seed_off, int32_t ni, int64_t n,
                       uint32_t* next, int64_t nwp, uint32_t* summ, int64_t nsw, SampleCtl* ctl, hipStream_t s) {
    if (num_seeds <= 0) return;
    hipsim::enqueue(s, [=] {
        int32_t i = 0;
        for (int64_t k = 0; k < num_seeds; ++k) {
            while (i + 1 < ni && seed_off[i + 1] <= k) ++i;
            const int32_t v = seeds[k];
            if (v < 0 || v >= n) {
                ctl->bad_seed = 1;
                continue;
            }
            next[(int64_t)i * nwp + (v >> 5)] |= 1u << (v & 31);
            if (summ) summ[(int64_t)i * nsw + (v >> 10)] |= 1u << ((v >> 5) & 31);
        }
    });
}

int64_t sparse_build_blocks(int64_t capacity) { return capacity > 0 ? (capacity + 255) / 256 : 1; }
int64_t dirty_compact_blocks(int64_t summary_words) { return summary_words > 0 ? (summary_words + 1023) / 1024 : 1; }

int64_t frontier_build_blocks(int64_t words) {
    const int64_t per = 256 * (words > (int64_t(1) << 20) ? 16 : 1);
    const int64_t nb = (words + per - 1) / per;
    return nb > 0 ? nb : 1;
}

void launch_frontier_build(const FrontierBuild& fb, hipStream_t s, LaunchEvents) {
    hipsim::enqueue(s, [fb] {
        SampleCtl* ctl = fb.ctl;
        const int64_t out_base = ctl->out_base[fb.layer];
        int64_t pos = 0, eoff = 0, nbig = 0, ndirty = 0;
        if (fb.summ) {  // sparse: the dirty list from the summary, which is cleared
            for (int64_t i = 0; i < (int64_t)fb.num_instances * fb.nsw; ++i) {
                const int64_t inst = i / fb.nsw;
                for (uint32_t bits = fb.summ[i]; bits; bits &= bits - 1)
                    fb.dirty[ndirty++] = inst * fb.nwp + (i - inst * fb.nsw) * 32 + __builtin_ctz(bits);
                fb.summ[i] = 0;
            }
            ctl->ndirty[fb.layer] = ndirty;
        }
        for (int64_t iw = 0; iw < fb.nwords; ++iw) {
            const int64_t inst = iw / fb.nwp, local = iw - inst * fb.nwp;
            if (local == 0 && fb.offsets && fb.layer < fb.num_layers)
                fb.offsets[(int64_t)fb.layer * fb.num_instances + inst] = out_base + eoff;
            const uint32_t w = fb.next[iw] & ~fb.visited[iw];
            fb.visited[iw] |= w;
            fb.next[iw] = 0;
            for (uint32_t bits = w; bits; bits &= bits - 1) {
                const int32_t v = (int32_t)(local * 32 + __builtin_ctz(bits));
                const int32_t k = fb.fanout[inst], kind = fb.bias[inst];
                const int64_t beg = fb.g.rowptr[v], d = fb.g.rowptr[v + 1] - beg;
                bool wide;
                const int32_t P = positive_count(fb.g, kind, v, d, wide);
                int32_t c = (k == 0 || P == 0) ? 0 : (k < 0 || k >= P) ? P : k;
                if (k > kMaxDrawFanout && k < P) {
                    ctl->unsupported = 1;
                    c = 0;
                }
                const bool big = kind != kUniform && c > 0 && k > 0 && k < P && (d > kWaveMaxD || wide);
                fb.fv[pos] = v;
                fb.fi[pos] = (int32_t)inst;
                fb.cnt[pos] = c;
                fb.off[pos] = eoff;
                fb.fbeg[pos] = beg;
                fb.fdeg[pos] = (int32_t)d;
                fb.fpos[pos] = P | (wide ? kWideList : 0);
                if (big) fb.bigs[nbig++] = (int32_t)pos;
                ++pos;
                eoff += c;
                if (fb.inst_id[inst] == hipsim_hooks::fail_instance.load()) ctl->unsupported = 1;
            }
        }
        ctl->fcount[fb.layer] = pos;
        ctl->total[fb.layer] = eoff;
        ctl->nbig[fb.layer] = (unsigned long long)nbig;
        const int64_t ob = out_base + eoff;
        for (int j = fb.layer + 1; j <= fb.num_layers; ++j) ctl->out_base[j] = ob;
        if (fb.offsets) {
            const int64_t ni = fb.num_instances;
            for (int64_t j = fb.layer + 1; j < fb.num_layers; ++j)
                for (int64_t i = 0; i < ni; ++i) fb.offsets[j * ni + i] = ob;
            fb.offsets[(int64_t)fb.num_layers * ni] = ob;
            for (int64_t i = 0; i < ni; ++i)
                if (fb.inst_id[i] == hipsim_hooks::corrupt_instance.load() && fb.layer < fb.num_layers)
                    fb.offsets[(int64_t)fb.layer * ni + i] = out_base + eoff + 1000;
        }
    });
}

// Every entry of the layer: the first c positive-bias neighbors in list
// order; picks not visited join the instance's next bitmap.
void launch_select(const SampleLayer& p, int, hipStream_t s, LaunchEvents) {
    hipsim::enqueue(s, [p] {
        SampleCtl* ctl = p.ctl;
        const int64_t fcount = ctl->fcount[p.layer], out_base = ctl->out_base[p.layer];
        for (int32_t i = 0; i < p.num_instances; ++i)
            if (p.inst_id[i] == hipsim_hooks::slow_instance.load())
                std::this_thread::sleep_for(std::chrono::milliseconds(50));
        for (int64_t e = 0; e < fcount; ++e) {
            const int32_t c = p.cnt[e];
            if (c == 0) continue;
            const int64_t o = out_base + p.off[e];
            if (o + c > p.capacity) {
                ctl->overflow = 1;
                continue;
            }
            const int32_t v = p.fv[e], inst = p.fi[e], kind = p.bias[inst];
            if (v < p.vlo || v >= p.vhi) continue;
            const uint32_t* w = weights(p.g, kind);
            const int64_t beg = p.fbeg[e], d = p.fdeg[e];
            const bool claim = p.fanout_next[inst] != 0;
            int32_t j = 0;
            for (int64_t i = 0; i < d && j < c; ++i) {
                if (w && w[beg + i] == 0) continue;
                const int32_t x = p.g.col[beg + i];
                p.src[o + j] = v;
                p.dst[o + j] = x;
                ++j;
                const int64_t wd = (int64_t)inst * p.nwp + (x >> 5);
                const uint32_t bit = 1u << (x & 31);
                if (claim && !(p.visited[wd] & bit)) {
                    if (p.summ && p.next[wd] == 0) p.summ[(int64_t)inst * p.nsw + ((x >> 5) >> 5)] |= 1u << ((x >> 5) & 31);
                    p.next[wd] |= bit;
                }
            }
        }
    });
}

void launch_select_small(const SampleLayer&, int, hipStream_t, LaunchEvents) {}
void launch_select_big(const SampleLayer&, int, hipStream_t, LaunchEvents) {}

void launch_clear_visited(const ClearVisited& c, hipStream_t s, LaunchEvents) {
    hipsim::enqueue(s, [c] {
        std::memcpy(c.host_ctl, c.ctl, sizeof(SampleCtl));
        for (int l = 0; l < c.num_layers; ++l)
            for (int64_t e = 0; e < c.fcount[l]; ++e) c.visited[(int64_t)c.fi[l][e] * c.nwp + (c.fv[l][e] >> 5)] = 0;
    });
}

void launch_call_setup(uint32_t* ctl, int64_t nctl, const uint32_t* host_tab, uint32_t* tab, int64_t ntab,
                       hipStream_t s) {
    hipsim::enqueue(s, [=] {
        std::fill(ctl, ctl + nctl, 0u);
        if (ntab > 0) std::memcpy(tab, host_tab, (size_t)ntab * 4);
    });
}

// A walk step from v moves to neighbor hash(walker id, step) mod deg(v).
void launch_walk(const WalkParams& p, int, hipStream_t s, LaunchEvents) {
    hipsim::enqueue(s, [p] {
        // walker w's key, length, id, path row and counter, as the kernels
        // resolve them (from the call, or from its request in a batch)
        if (!p.batch.req) *p.steps = 0;
        for (int64_t w = 0; w < p.num_walkers; ++w) {
            uint64_t key = p.k0, id;
            int32_t len = p.length;
            int32_t* path;
            unsigned long long* counter = p.steps;
            if (p.batch.req) {
                const int32_t q = p.batch.req[w];
                key = (uint32_t)p.batch.key[q];
                len = p.batch.length[q];
                const int64_t i = w - p.batch.first[q];
                id = (uint32_t)(p.batch.base[q] + (uint64_t)i);
                path = p.paths + p.batch.path[q] + i * ((int64_t)len + 1);
                counter = p.batch.steps + q;
            } else {
                id = (uint32_t)(p.walker_ids ? p.walker_ids[w] : p.walker_base + (uint64_t)w);
                path = p.paths + w * ((int64_t)len + 1);
            }
            int32_t v = p.starts[w];
            if (v < 0 || v >= p.g.n) {
                *p.bad_start = 1;
                continue;
            }
            path[0] = v;
            for (int32_t t = 0; t < len; ++t) {
                const int64_t b = p.g.rowptr[v], d = p.g.rowptr[v + 1] - b;
                if (d == 0) {
                    for (int32_t r = t; r < len; ++r) path[r + 1] = -1;
                    break;
                }
                v = p.g.col[b + (int64_t)(mix(id * 131 + (uint64_t)t + (key << 32)) % (uint64_t)d)];
                path[t + 1] = v;
                ++*counter;
            }
        }
        const uint64_t extra = hipsim_hooks::walk_extra_steps.load(), only = hipsim_hooks::walk_extra_for.load();
        if (!p.batch.req) {
            if (only == ~0ull || only == p.walker_base) *p.steps += extra;
        } else {
            for (int32_t q = 0; p.num_walkers > 0 && q <= p.batch.req[p.num_walkers - 1]; ++q)
                if (only == ~0ull || only == p.batch.base[q]) p.batch.steps[q] += extra;
        }
    });
}

void launch_symmetric_check(RowPtr rowptr, const int32_t* col, int64_t n, int32_t* flag, hipStream_t s) {
    hipsim::enqueue(s, [=] {
        for (int64_t u = 0; u < n; ++u)
            for (int64_t i = rowptr[u]; i < rowptr[u + 1]; ++i) {
                const int32_t x = col[i];
                if (!std::binary_search(col + rowptr[x], col + rowptr[x + 1], (int32_t)u)) *flag = 1;
            }
    });
}

void launch_walk_guides(RowPtr rowptr, const int32_t* col, const uint32_t* w, const uint64_t* wtot, int64_t n,
                        WalkEdge* rec, WalkVertex* vtx, WalkBucket* gd, hipStream_t s) {
    hipsim::enqueue(s, [=] {
        for (int64_t v = 0; v < n; ++v) {
            const int64_t b = rowptr[v], d = rowptr[v + 1] - b;
            const uint64_t W = wtot[v];
            if (vtx) vtx[v] = WalkVertex{W, (uint32_t)b, (uint32_t)d};
            if (W == 0) continue;
            const int sh = guide_shift(W, d);
            const uint64_t K = ((W - 1) >> sh) + 1;
            if (K > (uint64_t)(kGuideBucketsPerEdge * d)) abort();  // the list's slots hold its buckets
            WalkBucket* G = gd + guide_base(b, v);
            uint64_t run = 0, k = 0;
            for (int64_t i = 0; i < d; ++i) {
                run += w[b + i];
                rec[b + i] = WalkEdge{run, col[b + i], w[b + i]};
                for (; k < K && (k << sh) < run; ++k) G[k] = WalkBucket{run, (uint32_t)i, col[b + i]};
            }
        }
    });
}

void launch_layer_sample(const LayerParams& p, hipStream_t s, LaunchEvents) {
    hipsim::enqueue(s, [p] {
        for (int64_t i = 0; i < (int64_t)p.num_instances * p.L; ++i) p.counts[i] = 0;
    });
}

void launch_mdrw(const MdrwParams& p, hipStream_t s, LaunchEvents) {
    hipsim::enqueue(s, [p] { *p.total = 0; });
}

}  // namespace csaw
