// Internal entry points of the ForceAtlas2 driver (fl_fa2.hip) used by the
// layout pipeline and the layout server.
#pragma once

#include <vector>

#include "fl_tree.h"

namespace fl {

// Validate FA2 parameters and a CSR graph (synchronises; throws fl::Error).
void fa2_validate(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *deg,
                  const fl_fa2_params *prm);

// Exact O(n^2) repulsion within every system of `sg`, masses deg + 1 (no
// validation).
void exact_repulsion(fl_ctx *c, const Segs &sg, const float *x, const float *y, const int32_t *deg, float kr,
                     float2 *fr);

// A batch of independent systems sharing one set of parameters: system k owns
// nodes [coff[k], coff[k+1]) of the arrays, whose CSR ids are local to the
// batch.  prm.repulsion is FL_REP_EXACT or FL_REP_FMM.
struct FA2Batch {
    std::vector<int32_t> coff;  // host, K + 1 entries
    int64_t nnz;                // row_ptr[n], known on the host
    const int32_t *row_ptr, *col, *deg;
    float *x, *y;
    fl_fa2_params prm;
};
// `iters` iterations of every batch from a zero state.  With graphs on, each
// batch runs on its own branch context (own stream) as one replayed graph,
// concurrently with the others; otherwise one after the other, eagerly, on
// the context's stream.  Ordered after earlier, and before later, work on the
// context's stream; throws if an FMM capacity guard tripped.  Every system
// has its own status word (a system whose forces turn non-finite stops moving;
// the others go on); at the end the words are OR-ed into *flags on the
// context's stream (bit 0: a non-finite force, bit 1: a non-finite position).
void fa2_run_batches(fl_ctx *c, const std::vector<FA2Batch> &b, int iters, int32_t *flags);

int32_t components(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *label);

// Nodes stably sorted by label (labels in [0, n)): perm[r] = node at sorted
// position r; flag[r] = 1 where a new label starts; pos = exclusive scan of
// flag; d_off[k] = first position of the k-th smallest label, d_off[K] = n;
// off = the same offsets on the host.  Throws FL_EINVAL unless there are
// exactly n_labels distinct labels.  Synchronises.
struct LabelSort {
    const int32_t *perm = nullptr, *flag = nullptr, *pos = nullptr;
    int32_t *d_off = nullptr;
    std::vector<int32_t> off;
};
LabelSort sort_by_label(fl_ctx *c, int32_t n, const int32_t *label, int32_t n_labels);
void kk_layout_subset(fl_ctx *c, int n_all, const int32_t *off, const std::vector<int32_t> &ids,
                      const int32_t *row_ptr, const int32_t *col, float *x, float *y, const fl_kk_params &prm);
// Throws FL_EINVAL unless the Kamada-Kawai parameters are valid.
void check_kk_params(const fl_kk_params *p);

}  // namespace fl

// fl_fa2_step / fl_fa2_run behind their C entry points (argument checks,
// errors mapped to fl_status and the context's last-error text).
fl_status fa2_run_impl(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *deg,
                       float *x, float *y, fl_fa2_state *st, const fl_fa2_params *prm, int32_t iters,
                       fl_step_stats *per_iter, bool always_sync);
