// rvea_internal.h -- host-side launchers of the library's kernels (one per
// kernel group; each enqueues on the given stream and returns the launch
// error, if any).
#pragma once

#include <hip/hip_runtime.h>

#include "rvea_dev.h"

namespace rvea {

// records the HIP error of a call that has no run handle; read back with
// rvea_last_error(NULL) on the same thread
void note_thread_error(const char *what, hipError_t e);
void note_thread_message(const char *msg);

constexpr int kOffBlock = 64;  // threads per workgroup of the offspring kernels
// template class of a batched offspring launch: the segment width, plus
// kDefaultIndices when the run has the default distribution indices
constexpr int kSegMask = 0xff, kDefaultIndices = 0x100;

int pick_segment(int d);                 // lanes per individual (initialization)
int offspring_segment(int d, int64_t N);  // lanes per parent pair
int offspring_splits(int d, int64_t N);   // segments per parent pair
int assoc_rows_per_block();
int rerank_rows_per_wave();      // batched launch
int default_rerank_rows(int64_t rows);  // single-run default for this many rows

hipError_t launch_lattice(const RunView &R, hipStream_t s, int H);
hipError_t launch_vec_aux(const RunView &R, hipStream_t s);
hipError_t launch_gamma(const RunView &R, hipStream_t s, int force);
hipError_t launch_init(const RunView &R, hipStream_t s);
hipError_t launch_prepare(const RunView &R, hipStream_t s);
// row stamps and per-block valid counts of the current population (after
// initialization or a host-set state)
hipError_t launch_stamp(const RunView &R, hipStream_t s);
// reproduction and evaluation of the run's operator (the genetic kernels,
// or launch_operator for the others)
hipError_t launch_offspring(const RunView &R, hipStream_t s);
hipError_t launch_operator(const RunView &R, hipStream_t s);  // DE, PSO, CSO, random
// batched reproduction of the runs with another operator: their template
// class (kOperatorClass, the operator, the segment width), block count and
// launch
constexpr int kOperatorClass = 0x10000;
int operator_class(const RunView &R);
int64_t operator_blocks(const RunView &R);
hipError_t launch_batch_operator(int cls, const RunView *runs, const Span *spans, int n,
                                 int64_t blocks, hipStream_t s);
hipError_t launch_assoc(const RunView &R, hipStream_t s);
// indexed association (two and three objectives): the index of V, rebuilt
// when V changes (force, or the adaptation's changed flag), and the
// association
int grid_side(int m, int64_t K);  // cells per side (0: not indexed)
int grid_slot();                  // list records per cell
hipError_t launch_grid_build(const RunView &R, hipStream_t s, int force);
// the rebuild after an adaptation, which has already counted each vector
// into its cell (runs only when the vectors changed)
hipError_t launch_grid_rebuild(const RunView &R, hipStream_t s);
hipError_t launch_assoc_grid(const RunView &R, hipStream_t s);
hipError_t launch_rerank(const RunView &R, hipStream_t s);
hipError_t launch_select_back(const RunView &R, hipStream_t s);
hipError_t launch_adapt(const RunView &R, hipStream_t s);
hipError_t launch_init_gauss(const RunView &R, hipStream_t s);
// objectives of the N initial slots (offspring = false) or of the offspring
hipError_t launch_rollout(const RunView &R, hipStream_t s, bool offspring);

// Batched phases: one launch advances one phase of every run listed in the
// span table (runs of the same template class: segment width for the
// offspring, objective count for the association phases).
enum BatchPhase {
    BP_PREP, BP_OFFSPRING, BP_OFFSPRING_FIN, BP_ASSOC, BP_RERANK,
    BP_NEWPOP, BP_ADAPT, BP_GRID_RANGES, BP_GRID_FILL, BP_GRID_CELLS,
    BP_GAMMA_ASSOC, BP_GAMMA_RERANK, BP_COUNT
};
// blocks per workgroup of the batched phases that most generations skip
// (span_blocks), used by launches of at least kSkipBlocks * kFillBlocks
// blocks; kFillBlocks workgroups fill the device several times over
constexpr int kSkipBlocks = 8;
constexpr int64_t kFillBlocks = 2048;
// class of the indexed association launches (runs with an index of V), with
// the objective count; the full-scan association classes are the counts alone
constexpr int kIndexedClass = 0x100;
// the gamma passes run over a view with the gamma pass's own vector chunks
inline bool batch_phase_gamma(int phase)
{
    return phase == BP_GAMMA_ASSOC || phase == BP_GAMMA_RERANK;
}
int batch_phase_class(int phase, const RunView &R);       // template class of a run
int64_t batch_phase_blocks(int phase, const RunView &R);  // its block count
int64_t batch_phase_nbx(int phase, const RunView &R);     // row blocks of 2-D phases
hipError_t launch_batch(int phase, int cls, const RunView *runs, const Span *spans, int n,
                        int64_t blocks, hipStream_t s);
hipError_t launch_batch_gen(int phase, int cls, const RunView *runs, const Span *spans, int n,
                            int64_t blocks, hipStream_t s);
hipError_t launch_batch_select(int phase, int cls, const RunView *runs, const Span *spans,
                               int n, int64_t blocks, hipStream_t s);
// the index's phases (association of indexed runs, the three build phases
// after the adaptation's counting):
// blocks of a run (0 without an index) and the launch
int64_t grid_phase_blocks(int phase, const RunView &R);
hipError_t launch_batch_grid(int phase, int cls, const RunView *runs, const Span *spans, int n,
                             int64_t blocks, hipStream_t s);
hipError_t launch_batch_vectors(int phase, int cls, const RunView *runs, const Span *spans,
                                int n, int64_t blocks, hipStream_t s);

}  // namespace rvea
