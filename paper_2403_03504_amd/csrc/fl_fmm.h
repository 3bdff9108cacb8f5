// FMM repulsion driver (fl_fmm.hip) over the tree and lists of fl_tree.h.
#pragma once

#include "fl_tree.h"

namespace fl {

bool fmm_order_supported(int p);

// F_r of every node in original order into frx/fry (FP32), on the context
// stream, without host synchronisation.  deg supplies the masses deg + 1.
void fmm_repulsion(fl_ctx *c, int32_t n, const float *x, const float *y, const int32_t *deg, int p, int leaf,
                   int bits, float kr, float *frx, float *fry);

}  // namespace fl
