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

// Builds the tables of a bias kind now, if they do not exist yet (their
// first use otherwise builds them).
csaw_status prepare_bias_tables(csaw_graph g, int32_t bias_kind, hipStream_t stream);

}  // namespace csaw
