// Internal entry points of the ForceAtlas2 driver (fl_fa2.hip) used by the
// layout pipeline and the layout server.
#pragma once

#include "fl_common.h"

namespace fl {

// Validate FA2 parameters and a CSR graph (synchronises; throws fl::Error).
void fa2_validate(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *deg,
                  const fl_fa2_params *prm);
// `iters` iterations on a validated graph, enqueued on the context stream
// without host synchronisation.  flags: zeroed device int (non-finite bits).
void fa2_run_internal(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *deg, float *x,
                      float *y, fl_fa2_state *st, const fl_fa2_params *prm, int iters, int32_t *flags);

int32_t components(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *label);
void kk_layout_subset(fl_ctx *c, int n_all, const int32_t *off, const std::vector<int32_t> &ids,
                      const int32_t *row_ptr, const int32_t *col, float *x, float *y, double l, int steps);

}  // namespace fl
