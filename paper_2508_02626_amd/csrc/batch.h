// Pieces of the batched evaluation shared by the entry points in api.hip and
// noalloc.hip (internal, not part of the ABI).  None of them allocates memory.
#pragma once
#include <string>
#include "fmm.h"
#include "common.h"

namespace fmm {
// records msg as the calling thread's last error and returns code
int set_error(int code, const std::string &msg);
// validates a batch, makes `stream` wait for the plans' builds and fills
// idx[0..count) with the plans ordered by (order, FP32 M2L, position)
int batch_prepare(fmm_plan_t const *plans, const double *const *q_dev, double *const *phi_dev, int32_t count,
                  hipStream_t stream, int *idx);
// evaluates plans idx[c0..c1) (at most kMaxBatch) with their views staged in
// the device array Vd (c1 - c0 entries), stream-ordered on `stream`
int batch_chunk(fmm_plan_t const *plans, const int *idx, int c0, int c1, const double *const *q_dev,
                double *const *phi_dev, double *const *field_dev, hipStream_t stream, PlanView *Vd);
// records the evaluation on `stream` for fmm_plan_destroy
int batch_note_use(fmm_plan_t const *plans, int32_t count, hipStream_t stream);
int plan_device(fmm_plan_t plan);
} // namespace fmm
