// Batched assembly (batch.hip): internal interface used by the C ABI.
#pragma once

#include <vector>

#include "assemble_items.h"

struct nlfem_batch;

namespace nlfem {

// tune_mode: 0 default shapes, 1 cached or tuned (cache written), 2 always tuned
// handles: the problems' pair handles (checked again before every run: a
// plain rebuild of one since the creation makes the batch stale)
int batch_create(const std::vector<items::AssemblePlan> &plans, const std::vector<nlfem_pairs *> &handles,
                 const char *tune_cache, int tune_mode, nlfem_batch **out, hipStream_t s);
int batch_run(nlfem_batch *b, hipStream_t s);
int batch_graph_launch(nlfem_batch *b, hipStream_t s);
int batch_info(const nlfem_batch *b, int32_t *groups, int32_t *shape);
void batch_free(nlfem_batch *b);
// the same assembly with its tables and counters in a static device array
// (no allocation; one synchronisation for the table copy); E_OVERFLOW when
// the tables exceed batch_scratch_bytes()
int batch_assemble_noalloc(const std::vector<items::AssemblePlan> &plans, hipStream_t s);
size_t batch_scratch_bytes();

}  // namespace nlfem
