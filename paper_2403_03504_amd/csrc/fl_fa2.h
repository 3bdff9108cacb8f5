// Internal entry points of the ForceAtlas2 driver (fl_fa2.hip) used by the
// layout pipeline and the layout server.
#pragma once

#include <vector>

#include "fl_common.h"

namespace fl {

// Validate FA2 parameters and a CSR graph (synchronises; throws fl::Error).
void fa2_validate(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *deg,
                  const fl_fa2_params *prm);

// Exact O(n^2) repulsion of n points with masses deg + 1 (no validation).
void exact_repulsion(fl_ctx *c, int32_t n, const float *x, const float *y, const int32_t *deg, float kr, float *frx,
                     float *fry);

// An independent system for fa2_run_many (device arrays; ids local to it).
struct FA2System {
    int32_t n;
    int64_t nnz;  // row_ptr[n], known on the host
    const int32_t *row_ptr, *col, *deg;
    float *x, *y;
};
// `iters` iterations of every system from a zero state, concurrently: the
// systems are dealt to up to 8 branch contexts (own streams), one captured
// graph holds one iteration of all of them and is replayed iters-1 times.
// Ordered after earlier, and before later, work on the context's stream;
// throws if an FMM capacity guard tripped.
void fa2_run_many(fl_ctx *c, const std::vector<FA2System> &sys, const fl_fa2_params *prm, int iters,
                  int32_t fmm_min_nodes, int32_t *flags);

int32_t components(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *label);
void kk_layout_subset(fl_ctx *c, int n_all, const int32_t *off, const std::vector<int32_t> &ids,
                      const int32_t *row_ptr, const int32_t *col, float *x, float *y, double l, int steps);

}  // namespace fl
