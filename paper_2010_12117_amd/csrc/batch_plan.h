// Host planning of a batched solve (batch.h): which matrices go together, where their
// intermediates live in the workspace, and the launches with their descriptor tables.
#pragma once

#include <string>
#include <vector>

#include "batch.h"
#include "plan.h"

namespace pd {

struct BatchPlan {
  std::vector<BLaunch> launches;   // in stream order, chunk after chunk
  std::vector<uint8_t> desc_blob;  // every launch's descriptors (uploaded once)
  std::vector<int> singles;        // matrices solved one by one after the chunks
  int chunks = 0;
  bool halves = false;             // chunk c in half c mod 2 of the workspace
  size_t ws_bytes = 0;             // workspace the solve needs
};

// Whether a matrix can run in the batched launches (fused elimination, at most kBatchMaxM
// coefficients per variable in the evaluation passes).
bool batchable(const MatPlan& P);

// Workspace bytes of one matrix in a chunk.
size_t batch_footprint(const MatPlan& P);

// Plans the batched solve of `mats` (device tables already uploaded) with chunks of at most
// `budget` workspace bytes in all; with `halves`, chunks of half the budget that alternate
// between the two halves of the workspace (consecutive chunks share no memory and can run
// on two streams). Returns an error message or "".
std::string build_batch(const std::vector<MatPlan>& mats, size_t budget, bool halves,
                        BatchPlan* out);

}  // namespace pd
