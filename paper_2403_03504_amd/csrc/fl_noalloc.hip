// One ForceAtlas2 iteration that allocates nothing: the workspace the
// iteration needs (sort buffers, tree, hash table, lists, expansions, force
// and reduction buffers) is carved from a fixed device array instead of the
// context's grow-only workspace.  For callers that cannot allocate device
// memory while they run (graph capture, tight serving loops).
//
// The array is one per GPU (each device the library runs on holds its own
// copy until the process ends); its device address is looked up once per
// device and kept.  Every call on a GPU uses that GPU's array from its start,
// so calls that overlap on one GPU (on different streams, or from different
// threads) race; buffers that must start at zero are cleared by fill kernels
// in every call.
#include <mutex>

#include "fl_fa2.h"

namespace {

static __device__ __align__(256) char scratch[FL_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
char *g_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up on the first
// call on the device, with that device current).
char *scratch_ptr(int device)
{
    if (device < 0 || device >= MAX_DEVICES)
        throw fl::Error(FL_EUNSUPPORTED, "fl_fa2_step_noalloc: device id past the supported range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        FL_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw fl::Error(FL_EHIP, "fl_fa2_step_noalloc: no device address for the scratch array");
        g_ptr[device] = static_cast<char *>(p);
    }
    return g_ptr[device];
}

// Switches a context to the fixed arena for one call and back: its own
// workspace map, caches and launch modes are set aside and restored.
struct ArenaScope {
    fl_ctx *c;
    std::map<std::string, fl::DevBuf> bufs;
    int32_t seg1_n;
    int tree_cbits;
    bool branches, timing, use_graphs;
    ArenaScope(fl_ctx *ctx, char *base, size_t cap) : c(ctx)
    {
        bufs.swap(c->bufs);
        seg1_n = c->seg1_n;
        tree_cbits = c->tree_cbits;
        branches = c->branches;
        timing = c->timing;
        use_graphs = c->use_graphs;
        c->seg1_n = -1;       // the one-system descriptor is rebuilt in the arena
        c->tree_cbits = -1;   // the hash table is new: restart its epoch (clears it)
        c->branches = false;  // every launch on the caller's stream: no events or private streams
        c->timing = false;
        c->use_graphs = false;
        c->arena = base;
        c->arena_cap = cap;
        c->arena_used = 0;
    }
    ~ArenaScope()
    {
        c->arena = nullptr;
        c->arena_cap = c->arena_used = 0;
        c->bufs.swap(bufs);
        c->seg1_n = seg1_n;
        c->tree_cbits = tree_cbits;
        c->branches = branches;
        c->timing = timing;
        c->use_graphs = use_graphs;
    }
};

}  // namespace

extern "C" {

fl_status fl_fa2_step_noalloc(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                              const int32_t *deg, float *x, float *y, fl_fa2_state *st, const fl_fa2_params *prm,
                              fl_step_stats *stats)
{
    if (!c) return FL_EINVAL;
    char *base = nullptr;
    try {
        FL_CHECK_HIP(hipSetDevice(c->device));
        base = scratch_ptr(c->device);
    } catch (const fl::Error &e) {
        c->err = e.what();
        return e.code;
    }
    if (c->arena) {
        c->err = "fl_fa2_step_noalloc: the context is already inside an allocation-free call";
        return FL_EBUSY;
    }
    ArenaScope scope(c, base, (size_t)FL_NOALLOC_SCRATCH_BYTES);
    return fa2_run_impl(c, n, row_ptr, col_idx, deg, x, y, st, prm, 1, stats, true);
}

}  // extern "C"
