// internal.h -- calls of libcsaw shared by its C-ABI entry points and the
// request server (not exported).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/csaw.h"

namespace csaw {

// Device bytes of a walk call's counters in caller scratch.
constexpr size_t kWalkScratch = 512;

// Frontier capacity per layer ([num_layers + 1]) and the edge bound of a
// sampling call, as the call itself plans them (host only).
csaw_status sample_plan_caps(csaw_graph g, const csaw_sample_args* a, std::vector<int64_t>& fcap,
                             int64_t* max_edges);

// Device scratch of a sampling call of num_instances instances, num_layers
// layers and per-layer frontier capacities fcap (summed over instances) that
// runs in caller memory: arena, both instance bitmaps, control block copy.
size_t sample_scratch_bytes(csaw_graph g, int32_t num_instances, int32_t num_layers,
                            const std::vector<int64_t>& fcap);

// csaw_sample / csaw_walk with every device byte in `scratch` (no
// allocation, no capture, every kernel on `stream`).
csaw_status sample_in_scratch(csaw_graph g, const csaw_sample_args* a, csaw_sample_out* out, hipStream_t stream,
                              char* scratch, size_t scratch_bytes);
csaw_status walk_in_scratch(csaw_graph g, const csaw_walk_args* a, int32_t* paths, int64_t* total_steps,
                            hipStream_t stream, char* scratch);

// Several walk requests of one bias kind, node2vec weights and move
// thresholds in one launch (request server). Device tables of a batch: per
// walker its request; per request its Philox key, length, first walker,
// walker id of that walker, first path entry and step counter; then a flag
// for a start vertex outside [0, n).
struct WalkBatchReq {
    int64_t num_walkers;
    int32_t length;
    uint64_t rng_seed;
    uint64_t walker_base;
};
struct WalkBatchLayout {
    size_t o_req, o_key, o_len, o_first, o_base, o_path, o_steps, o_bad, bytes;
};
WalkBatchLayout walk_batch_layout(int32_t nreq, int64_t nw);
// Host image of the tables (walk_batch_layout(...).bytes, counters and flag
// zero); request q's walkers follow those of requests 0..q-1 and its paths
// start at entry path_offset[q] of the batch's path array.
void walk_batch_image(const WalkBatchReq* reqs, int32_t nreq, const int64_t* path_offset, char* image);
// Runs a batch whose tables (the uploaded image) are at d_tables and whose
// starts are at d_starts (request by request); common gives the bias kind,
// node2vec weights and thresholds. steps[q] gets request q's step count.
// Allocates nothing; the bias kind's tables must exist (NOT_READY otherwise).
csaw_status walk_batch_in_scratch(csaw_graph g, const csaw_walk_args* common, const WalkBatchReq* reqs,
                                  int32_t nreq, const int32_t* d_starts, int32_t* d_paths, char* d_tables,
                                  int64_t* steps, hipStream_t stream);

// Builds the tables of a bias kind now, with its walk guide tables, if they
// do not exist yet (their first use otherwise builds them).
csaw_status prepare_bias_tables(csaw_graph g, int32_t bias_kind, hipStream_t stream);

}  // namespace csaw
