// kernels.h -- host-side launchers of the gfx950 kernels (internal to libcsaw).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csaw {

constexpr int kMaxLayers = 16;
constexpr int kMaxDrawFanout = 64;   // slots of one wave
constexpr int kRounds = 8;           // repeated-sampling rounds
constexpr int kScanItems = 1024;     // items per scan block (256 threads x 4)

enum BiasKind : int32_t { kUniform = 0, kEdgeWeight = 1, kNeighborDegree = 2, kNode2vec = 3 };

// Graph resident in HBM.
struct GraphDev {
    int64_t n, m;
    const int64_t* rowptr;     // n+1
    const int32_t* col;        // m
    const uint32_t* ew;        // m or null (EDGE_WEIGHT)
    const uint32_t* degw;      // m or null (NEIGHBOR_DEGREE, materialised)
    const int32_t* ppos_ew;    // n: #positive weights per list, or null
    const int32_t* ppos_deg;   // n
};

// Device-resident control block of one sampling call.
struct SampleCtl {
    int64_t fcount[kMaxLayers + 1];    // frontier sizes
    int64_t total[kMaxLayers];         // edges per layer
    int64_t out_base[kMaxLayers + 1];  // first edge of each layer
    unsigned long long nmid[kMaxLayers];  // mid-kernel entries per layer
    unsigned long long nhub[kMaxLayers];  // hub-kernel entries per layer
    int32_t bad_seed;
    int32_t overflow;
    int32_t unsupported;
    int32_t pad;
};

struct SampleLayer {
    GraphDev g;
    int32_t layer;
    int32_t num_instances;
    uint32_t k0, k1;                 // Philox key
    uint64_t instance_base;
    const int32_t* fanout;           // [ni] fanout of this layer per instance
    const int32_t* fanout_next;      // [ni] fanout of the next layer (0 = none)
    const int32_t* bias;             // [ni]
    const int32_t* fv;               // frontier vertices
    const int32_t* fi;               // frontier instance indices
    const int32_t* cnt;              // per-entry edge count
    const int64_t* off;              // per-entry exclusive offset
    int32_t* mids;                   // entries routed to the mid kernel
    int32_t* hubs;                   // entries routed to the hub kernel
    SampleCtl* ctl;
    int32_t* src;
    int32_t* dst;
    int64_t capacity;
    const uint32_t* visited;         // [ni * nwp]
    uint32_t* next;                  // [ni * nwp]
    int64_t nwp;                     // bitmap words per instance (multiple of 4)
};

// --- sampling (sample_kernels.hip)
void launch_mark_seeds(const int32_t* seeds, int64_t num_seeds, const int64_t* seed_offsets,
                       int32_t ni, int64_t n, uint32_t* next, int64_t nwp, SampleCtl* ctl,
                       hipStream_t s);
void launch_bitmap_compact(uint32_t* next, uint32_t* visited, int64_t words, int64_t nwp,
                           int64_t* blocksum, int64_t* fcount_out, int32_t* fv, int32_t* fi,
                           int64_t* fstart, int32_t ni, hipStream_t s);
void launch_count(const SampleLayer& p, int32_t* cnt, int64_t cap_entries, hipStream_t s);
void launch_scan_counts(const int32_t* cnt, const int64_t* fcount, int64_t cap_entries,
                        int64_t* blocksum, int64_t* off, int64_t* total_out, hipStream_t s);
void launch_select(const SampleLayer& p, int grid, hipStream_t s);
void launch_select_mid(const SampleLayer& p, int grid, hipStream_t s);
void launch_select_hub(const SampleLayer& p, int grid, hipStream_t s);
void launch_segments(const SampleLayer& p, const int64_t* fstart, int64_t* offsets, hipStream_t s);
void launch_clear_visited(const int32_t* fv, const int32_t* fi, const int64_t* fcount,
                          int64_t cap_entries, uint32_t* visited, int64_t nwp, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);

// --- graph preparation (sample_kernels.hip)
void launch_degree_weights(const int64_t* rowptr, const int32_t* col, int64_t m, uint32_t* degw,
                           hipStream_t s);
void launch_positive_counts(const int64_t* rowptr, const uint32_t* w, int64_t n, int32_t* ppos,
                            hipStream_t s);

// --- walks (walk_kernels.hip)
struct WalkParams {
    GraphDev g;
    int32_t bias;
    uint32_t w_return, w_common, w_outward;
    int64_t num_walkers;
    const int32_t* starts;
    uint64_t walker_base;
    int32_t length;
    uint32_t k0, k1;
    int32_t* paths;
    unsigned long long* steps;       // device counter
    int32_t* bad_start;              // device flag
};
void launch_walk(const WalkParams& p, int grid, hipStream_t s);

}  // namespace csaw
