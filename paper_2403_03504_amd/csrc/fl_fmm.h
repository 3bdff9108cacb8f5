// FMM repulsion driver (fl_fmm.hip) over the tree and lists of fl_tree.h.
#pragma once

#include <functional>

#include "fl_tree.h"

namespace fl {

bool fmm_order_supported(int p);

// F_r of every node in original order into fr (FP32 (x, y) pairs), on the
// context stream, without host synchronisation.  deg supplies the masses
// deg + 1.  Every system of `s` is its own particle set: no force crosses
// systems.  lanes: lanes per cell of the list kernels (1 or 8).  When
// `on_lists` is given it is called once the list build has been enqueued,
// with an event recorded on the context stream just after it: work that
// should overlap the near field (and not the latency-bound tree build) is
// forked from there, on a branch stream that joins the context stream later.
// The hook enqueues `tail` on that branch ahead of its join (the FMM puts the
// list statistics there, off the upward/M2L branch that the far field waits
// for).  xy_out (optional, n float2) receives the (x, y) pairs from the tree
// build; bb: the positions' tile extrema when already known.
using BranchTail = std::function<void(hipStream_t)>;
using ListsHook = std::function<void(hipEvent_t lists, const BranchTail &tail)>;
void fmm_repulsion(fl_ctx *c, const Segs &s, const float *x, const float *y, const int32_t *deg, int p, int leaf,
                   int bits, int lanes, float kr, float2 *fr, const ListsHook *on_lists = nullptr,
                   float2 *xy_out = nullptr, BBoxIn bb = {});

}  // namespace fl
