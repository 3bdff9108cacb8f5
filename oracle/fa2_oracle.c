/*
 * fa2_oracle.c -- plain, slow, FP64 CPU oracle for the FMM-ForceAtlas2 /
 * Kamada-Kawai layout method of "Graph Visualization for Blockchain Data".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code, header,
 * table or helper with the HIP library; neither includes the other.
 *
 * Every routine follows the paper's text (section numbers below) in the
 * paper's order, in double precision, with no blocking, fusion or reordering
 * beyond what the cited definition states.  Where the paper is silent the
 * reading taken is stated at the routine.
 *
 *   orc_repulsion_exact  sec. 3.2: pairwise repulsion, proportional to one
 *                        over the distance, degree-weighted as in ForceAtlas2
 *                        (Jacomy et al. 2014): kr (deg_i+1)(deg_j+1) / d.
 *   orc_components       sec. 4: split into components ignoring directions.
 *   orc_bfs_hops         sec. 3.1: d_ij = length of the shortest path (unit
 *                        edge weights, so breadth-first search is exact).
 *   orc_morton/orc_tree  sec. 3.2.1: quadtree over a square covering all
 *                        particles; a square with more than a given number of
 *                        particles is divided into four.
 *   orc_fmm_repulsion    sec. 3.2.1: outgoing expansions of leaves, shifted up
 *                        to parents; incoming expansions from the parent's
 *                        shift plus converted outgoing expansions of
 *                        interacting cells; evaluation at nodes plus the direct
 *                        near field.  Operators of Greengard & Rokhlin (1987).
 *   orc_kk_*             sec. 3.1: the Kamada-Kawai energy and its
 *                        minimisation: localized stress majorization, and
 *                        the paper's Newton-Raphson (orc_kk_newton).
 *   orc_bh_repulsion     sec. 3.2.1: Barnes-Hut, the O(N log N) method the
 *                        FMM improves on (comparator), on the same quadtree.
 *   orc_stress,          sec. 4: Kamada-Kawai on the graph whose nodes are
 *   orc_kk_sweeps        the components, with real edge lengths (sequential
 *                        localized stress majorization).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Repulsion: the plain definition (sec. 3.2, all node pairs).                */
/* F_i = kr * m_i * sum_{j != i, p_j != p_i} m_j (p_i - p_j) / |p_i - p_j|^2 */
/* j runs in ascending order with an FP64 accumulator.  A coincident pair     */
/* (d = 0) contributes nothing (the paper is silent on d = 0).                */
/* ------------------------------------------------------------------------ */
void orc_repulsion_exact(int64_t n, const double *x, const double *y, const double *m, double kr,
                         int64_t nt, const int64_t *targets, double *fx, double *fy)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets ? targets[t] : t;
        double ax = 0.0, ay = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j];
            double d2 = dx * dx + dy * dy;
            if (d2 == 0.0) continue;
            ax += m[j] * dx / d2;
            ay += m[j] * dy / d2;
        }
        fx[t] = kr * m[i] * ax;
        fy[t] = kr * m[i] * ay;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Components (sec. 4).  label[v] = smallest node id of v's component: nodes */
/* are scanned in ascending order and each unlabelled node starts a search.  */
/* ------------------------------------------------------------------------ */
int64_t orc_components(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *label)
{
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t ncomp = 0;
    for (int64_t v = 0; v < n; ++v) label[v] = -1;
    for (int64_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        ++ncomp;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = (int32_t)s;
        while (head < tail) {
            int64_t v = queue[head++];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t w = col[e];
                if (label[w] < 0) { label[w] = (int32_t)s; queue[tail++] = w; }
            }
        }
    }
    free(queue);
    return ncomp;
}

/* ------------------------------------------------------------------------ */
/* Hop distances (sec. 3.1): one breadth-first search per source on a graph  */
/* with local ids 0..n-1.  dist[s*n + v]; -1 where v is unreachable.         */
/* ------------------------------------------------------------------------ */
void orc_bfs_hops(int32_t n, const int64_t *row_ptr, const int32_t *col, int32_t *dist)
{
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t s = 0; s < n; ++s) {
        int32_t *d = dist + (int64_t)s * n;
        for (int32_t v = 0; v < n; ++v) d[v] = -1;
        int32_t head = 0, tail = 0;
        d[s] = 0;
        queue[tail++] = s;
        while (head < tail) {
            int32_t v = queue[head++];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t w = col[e];
                if (d[w] < 0) { d[w] = d[v] + 1; queue[tail++] = w; }
            }
        }
    }
    free(queue);
}

/* ------------------------------------------------------------------------ */
/* Quadtree (sec. 3.2.1).                                                     */
/* Root square: lower-left (xmin, ymin), side L = max extent (1 if zero).    */
/* A particle's cell coordinates at depth `bits`:                             */
/*   q = min(floor((x - xmin) * S), 2^bits - 1),  S = 2^bits / L  (FP64).    */
/* The Morton key interleaves q_x into the even bits and q_y into the odd    */
/* bits, so a cell at level l is the set of keys sharing the top 2l bits.    */
/* ------------------------------------------------------------------------ */
typedef struct { double xmin, ymin, L, S; } oroot;

static oroot root_square(int64_t n, const double *x, const double *y, int bits)
{
    oroot r;
    double x0 = x[0], x1 = x[0], y0 = y[0], y1 = y[0];
    for (int64_t i = 1; i < n; ++i) {
        if (x[i] < x0) x0 = x[i];
        if (x[i] > x1) x1 = x[i];
        if (y[i] < y0) y0 = y[i];
        if (y[i] > y1) y1 = y[i];
    }
    double L = (x1 - x0) > (y1 - y0) ? (x1 - x0) : (y1 - y0);
    if (!(L > 0.0)) L = 1.0;
    r.xmin = x0; r.ymin = y0; r.L = L;
    r.S = ldexp(1.0, bits) / L;
    return r;
}

static uint32_t quantize(double v, double vmin, double S, int bits)
{
    double t = floor((v - vmin) * S);
    double top = ldexp(1.0, bits) - 1.0;
    if (t > top) t = top;
    if (t < 0.0) t = 0.0;
    return (uint32_t)t;
}

static uint64_t interleave(uint32_t qx, uint32_t qy, int bits)
{
    uint64_t k = 0;
    for (int b = 0; b < bits; ++b) {
        k |= (uint64_t)((qx >> b) & 1u) << (2 * b);
        k |= (uint64_t)((qy >> b) & 1u) << (2 * b + 1);
    }
    return k;
}

void orc_root(int64_t n, const double *x, const double *y, int bits, double *out4)
{
    oroot r = root_square(n, x, y, bits);
    out4[0] = r.xmin; out4[1] = r.ymin; out4[2] = r.L; out4[3] = r.S;
}

void orc_morton(int64_t n, const double *x, const double *y, int bits, uint64_t *key)
{
    oroot r = root_square(n, x, y, bits);
    for (int64_t i = 0; i < n; ++i)
        key[i] = interleave(quantize(x[i], r.xmin, r.S, bits), quantize(y[i], r.ymin, r.S, bits), bits);
}

/* stable sort of node indices by key (ties by node index) */
static const uint64_t *g_sort_keys;
static int cmp_key_idx(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    uint64_t ki = g_sort_keys[i], kj = g_sort_keys[j];
    if (ki < kj) return -1;
    if (ki > kj) return 1;
    return (i < j) ? -1 : (i > j);
}

void orc_sort_by_key(int64_t n, const uint64_t *key, int64_t *perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    g_sort_keys = key;
    qsort(perm, (size_t)n, sizeof(int64_t), cmp_key_idx);
}

/* Cells: level, (ix, iy) at that level, particle range [begin, end) of the  */
/* sorted order, parent, child[4] (-1 = empty quadrant).  Child q covers      */
/* ix' = 2ix + (q & 1), iy' = 2iy + (q >> 1).  Cells are produced in          */
/* breadth-first order, i.e. sorted by (level, Morton prefix).                */
typedef struct { int32_t level, ix, iy, begin, end, parent, child[4]; } ocell;

typedef struct {
    ocell *c;
    int64_t n, cap;
} otree;

static void tree_push(otree *t, ocell c)
{
    if (t->n == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 1024;
        t->c = (ocell *)realloc(t->c, sizeof(ocell) * (size_t)t->cap);
    }
    t->c[t->n++] = c;
}

/* first index in [lo, hi) whose key is >= v */
static int64_t lower_bound_u64(const uint64_t *k, int64_t lo, int64_t hi, uint64_t v)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (k[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static otree build_tree(int64_t n, const uint64_t *skey, int bits, int leaf_size)
{
    otree t = {0, 0, 0};
    ocell root = {0, 0, 0, 0, (int32_t)n, -1, {-1, -1, -1, -1}};
    tree_push(&t, root);
    for (int64_t ci = 0; ci < t.n; ++ci) {
        ocell c = t.c[ci];
        int32_t cnt = c.end - c.begin;
        if (cnt <= leaf_size || c.level >= bits) continue; /* leaf */
        int sh = 2 * (bits - c.level - 1);
        uint64_t prefix = skey[c.begin] >> (sh + 2);
        int64_t b[5];
        b[0] = c.begin; b[4] = c.end;
        for (int q = 1; q < 4; ++q)
            b[q] = lower_bound_u64(skey, c.begin, c.end, ((prefix << 2) | (uint64_t)q) << sh);
        for (int q = 0; q < 4; ++q) {
            if (b[q + 1] == b[q]) continue;
            ocell ch = {c.level + 1, 2 * c.ix + (q & 1), 2 * c.iy + (q >> 1), (int32_t)b[q], (int32_t)b[q + 1],
                        (int32_t)ci, {-1, -1, -1, -1}};
            t.c[ci].child[q] = (int32_t)t.n;
            tree_push(&t, ch);
        }
    }
    return t;
}

static int is_leaf(const ocell *c) { return c->child[0] < 0 && c->child[1] < 0 && c->child[2] < 0 && c->child[3] < 0; }

/* orc_tree: keys must be sorted ascending.  out holds 10 int32 per cell:    */
/* level, ix, iy, begin, end, parent, child0..3.  Returns the cell count, or */
/* -(count) when `cap` is too small (nothing written then).                  */
int64_t orc_tree(int64_t n, const uint64_t *skey, int bits, int leaf_size, int64_t cap, int32_t *out)
{
    otree t = build_tree(n, skey, bits, leaf_size);
    int64_t cnt = t.n;
    if (cnt > cap) { free(t.c); return -cnt; }
    for (int64_t i = 0; i < cnt; ++i) {
        const ocell *c = &t.c[i];
        int32_t *o = out + 10 * i;
        o[0] = c->level; o[1] = c->ix; o[2] = c->iy; o[3] = c->begin; o[4] = c->end; o[5] = c->parent;
        for (int q = 0; q < 4; ++q) o[6 + q] = c->child[q];
    }
    free(t.c);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Neighbour and interaction lists (sec. 3.2.1).                              */
/*                                                                            */
/* The paper: the neighbours of a cell are the adjacent cells of minimal size */
/* not smaller than the cell; its interacting cells are the minimal cells     */
/* that neighbour its parent or are children of the parent's neighbours,      */
/* less its own neighbours ("far away" = not in a neighbouring cell).  On an  */
/* adaptive tree this is read as the lists of Carrier, Greengard & Rokhlin    */
/* (1988), which coincide with the paper's on a uniform tree:                 */
/*   U(b), leaf b:  b and every leaf adjacent to it (any size) -> direct sum  */
/*   V(c):          children of the parent's same-level neighbours that are   */
/*                  not adjacent to c                    -> outgoing->incoming */
/*   W(b), leaf b:  descendants of b's same-level neighbours whose parent is   */
/*                  adjacent to b but which are not      -> outgoing at nodes  */
/*   X(c):          leaves adjacent to c's parent, not adjacent to c, coarser */
/*                  than c                               -> nodes->incoming   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t *ptr; /* [ncell+1] */
    int32_t *idx;
    int64_t n, cap;
} olist;

static void list_push(olist *l, int32_t v)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 4096;
        l->idx = (int32_t *)realloc(l->idx, sizeof(int32_t) * (size_t)l->cap);
    }
    l->idx[l->n++] = v;
}

/* Deepest existing cell on the path to region (level, ix, iy): returns that  */
/* region's own cell, or the leaf covering it if the path ends in a leaf     */
/* above `level`, or -1 when the region is empty.                            */
static int32_t lookup(const otree *t, int level, int32_t ix, int32_t iy)
{
    int32_t cur = 0;
    for (int l = 0; l < level; ++l) {
        const ocell *c = &t->c[cur];
        if (is_leaf(c)) return cur;
        int sh = level - l - 1;
        int q = (int)(((ix >> sh) & 1) | (((iy >> sh) & 1) << 1));
        int32_t nx = c->child[q];
        if (nx < 0) return -1;
        cur = nx;
    }
    return cur;
}

/* closed squares of two distinct, non-nested cells touch */
static int adjacent(const ocell *a, const ocell *b)
{
    int L = a->level > b->level ? a->level : b->level;
    int64_t sa = (int64_t)1 << (L - a->level), sb = (int64_t)1 << (L - b->level);
    int64_t ax0 = (int64_t)a->ix * sa, ax1 = ax0 + sa, ay0 = (int64_t)a->iy * sa, ay1 = ay0 + sa;
    int64_t bx0 = (int64_t)b->ix * sb, bx1 = bx0 + sb, by0 = (int64_t)b->iy * sb, by1 = by0 + sb;
    return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
}

static int contains(const int32_t *a, int n, int32_t v)
{
    for (int i = 0; i < n; ++i) if (a[i] == v) return 1;
    return 0;
}

typedef struct { olist U, V, W, X; } olists;

static void collect_uw(const otree *t, int32_t b, int32_t d, olist *U, olist *W)
{
    const ocell *cd = &t->c[d];
    for (int q = 0; q < 4; ++q) {
        int32_t ch = cd->child[q];
        if (ch < 0) continue;
        if (adjacent(&t->c[ch], &t->c[b])) {
            if (is_leaf(&t->c[ch])) list_push(U, ch);
            else collect_uw(t, b, ch, U, W);
        } else {
            list_push(W, ch);
        }
    }
}

static olists build_lists(const otree *t)
{
    olists L;
    memset(&L, 0, sizeof(L));
    int64_t nc = t->n;
    L.U.ptr = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    L.V.ptr = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    L.W.ptr = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    L.X.ptr = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    for (int64_t ci = 0; ci < nc; ++ci) {
        const ocell *c = &t->c[ci];
        int lv = c->level;
        int32_t side = (int32_t)1 << lv;
        /* V and X from the parent's ring */
        if (c->parent >= 0) {
            const ocell *P = &t->c[c->parent];
            int32_t pside = (int32_t)1 << (lv - 1);
            int32_t seenx[8];
            int nseenx = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    int32_t rx = P->ix + dx, ry = P->iy + dy;
                    if (rx < 0 || ry < 0 || rx >= pside || ry >= pside) continue;
                    int32_t N = lookup(t, lv - 1, rx, ry);
                    if (N < 0) continue;
                    const ocell *cn = &t->c[N];
                    if (cn->level == lv - 1 && !is_leaf(cn)) {
                        for (int q = 0; q < 4; ++q) {
                            int32_t ch = cn->child[q];
                            if (ch >= 0 && !adjacent(&t->c[ch], c)) list_push(&L.V, ch);
                        }
                    } else if (is_leaf(cn)) {
                        if (!adjacent(cn, c) && !contains(seenx, nseenx, N)) {
                            seenx[nseenx++] = N;
                            list_push(&L.X, N);
                        }
                    }
                }
        }
        L.V.ptr[ci + 1] = L.V.n;
        L.X.ptr[ci + 1] = L.X.n;
        /* U and W for leaves */
        if (is_leaf(c)) {
            list_push(&L.U, (int32_t)ci);
            int32_t seen[8];
            int nseen = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    int32_t rx = c->ix + dx, ry = c->iy + dy;
                    if (rx < 0 || ry < 0 || rx >= side || ry >= side) continue;
                    int32_t N = lookup(t, lv, rx, ry);
                    if (N < 0) continue;
                    const ocell *cn = &t->c[N];
                    if (is_leaf(cn)) {
                        if (!contains(seen, nseen, N)) { seen[nseen++] = N; list_push(&L.U, N); }
                    } else {
                        collect_uw(t, (int32_t)ci, N, &L.U, &L.W);
                    }
                }
        }
        L.U.ptr[ci + 1] = L.U.n;
        L.W.ptr[ci + 1] = L.W.n;
    }
    return L;
}

static void free_lists(olists *L)
{
    free(L->U.ptr); free(L->U.idx); free(L->V.ptr); free(L->V.idx);
    free(L->W.ptr); free(L->W.idx); free(L->X.ptr); free(L->X.idx);
}

/* ------------------------------------------------------------------------ */
/* Expansion operators (Greengard & Rokhlin 1987), potential                  */
/*   phi(z) = sum_j q_j log(z - z_j),   F_i = kr m_i conj(phi'(z_i)),         */
/* with q_j = m_j.  Outgoing (multipole) expansion about z_c:                 */
/*   phi(z) = Q log(z - z_c) + sum_{k=1..p} a_k / (z - z_c)^k                 */
/* incoming (local) expansion about z_c: phi(z) = sum_{l=0..p} b_l (z-z_c)^l. */
/* Coefficient arrays hold p+1 entries; entry 0 is Q (outgoing) or b_0        */
/* (incoming, never needed since only phi' is evaluated).                     */
/* ------------------------------------------------------------------------ */
static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

/* P2M: Q = sum q_j, a_k = -sum q_j (z_j - z_c)^k / k */
static void op_p2m(int64_t cnt, const cplx *z, const double *q, cplx zc, int p, cplx *a)
{
    for (int k = 0; k <= p; ++k) a[k] = 0.0;
    for (int64_t j = 0; j < cnt; ++j) {
        cplx d = z[j] - zc, pw = 1.0;
        a[0] += q[j];
        for (int k = 1; k <= p; ++k) {
            pw *= d;
            a[k] += -q[j] * pw / (double)k;
        }
    }
}

/* M2M: outgoing expansion about z_c + z0 re-centred at z_c (GR87 Lemma 2.3) */
static void op_m2m(const cplx *a, cplx z0, int p, cplx *b /* accumulated */)
{
    cplx Q = a[0];
    b[0] += Q;
    for (int l = 1; l <= p; ++l) {
        cplx s = -Q * cpow(z0, l) / (double)l;
        for (int k = 1; k <= l; ++k) s += a[k] * cpow(z0, l - k) * binom(l - 1, k - 1);
        b[l] += s;
    }
}

/* M2L: outgoing expansion about z_t + z0 converted to an incoming expansion */
/* about z_t (GR87 Lemma 2.4), l >= 1 only                                   */
static void op_m2l(const cplx *a, cplx z0, int p, cplx *b /* accumulated */)
{
    cplx Q = a[0];
    for (int l = 1; l <= p; ++l) {
        cplx s = 0.0;
        for (int k = 1; k <= p; ++k) {
            double sg = (k & 1) ? -1.0 : 1.0;
            s += a[k] / cpow(z0, k) * binom(l + k - 1, k - 1) * sg;
        }
        b[l] += -Q / ((double)l * cpow(z0, l)) + s / cpow(z0, l);
    }
}

/* P2L: a point mass q at z_t + z0 as an incoming expansion about z_t        */
static void op_p2l(double q, cplx z0, int p, cplx *b)
{
    for (int l = 1; l <= p; ++l) b[l] += -q / ((double)l * cpow(z0, l));
}

/* L2L: incoming expansion about z_p re-centred at z_p + z0 (GR87 Lemma 2.5) */
static void op_l2l(const cplx *b, cplx z0, int p, cplx *c /* accumulated */)
{
    for (int m = 0; m <= p; ++m) {
        cplx s = 0.0;
        for (int l = m; l <= p; ++l) s += b[l] * binom(l, m) * cpow(z0, l - m);
        c[m] += s;
    }
}

/* L2P: phi'(z) = sum_{l=1..p} l b_l (z - z_c)^{l-1} */
static cplx op_l2p(const cplx *b, cplx d, int p)
{
    cplx s = 0.0, pw = 1.0;
    for (int l = 1; l <= p; ++l) {
        s += (double)l * b[l] * pw;
        pw *= d;
    }
    return s;
}

/* M2P: phi'(z) of an outgoing expansion, d = z - z_c:                        */
/* Q/d - sum_k k a_k / d^{k+1}                                                */
static cplx op_m2p(const cplx *a, cplx d, int p)
{
    cplx s = a[0] / d;
    for (int k = 1; k <= p; ++k) s -= (double)k * a[k] / cpow(d, k + 1);
    return s;
}

/* exported thin wrappers (test access to the operators, FP64 split re/im)  */
static void to_c(int n, const double *re, const double *im, cplx *o) { for (int i = 0; i < n; ++i) o[i] = re[i] + I * im[i]; }
static void from_c(int n, const cplx *c, double *re, double *im) { for (int i = 0; i < n; ++i) { re[i] = creal(c[i]); im[i] = cimag(c[i]); } }

void orc_op_p2m(int64_t cnt, const double *zx, const double *zy, const double *q, double cx, double cy, int p,
                double *are, double *aim)
{
    cplx *z = (cplx *)malloc(sizeof(cplx) * (size_t)(cnt > 0 ? cnt : 1));
    cplx a[64];
    for (int64_t j = 0; j < cnt; ++j) z[j] = zx[j] + I * zy[j];
    op_p2m(cnt, z, q, cx + I * cy, p, a);
    from_c(p + 1, a, are, aim);
    free(z);
}

void orc_op_m2m(const double *are, const double *aim, double z0x, double z0y, int p, double *bre, double *bim)
{
    cplx a[64], b[64];
    to_c(p + 1, are, aim, a);
    to_c(p + 1, bre, bim, b);
    op_m2m(a, z0x + I * z0y, p, b);
    from_c(p + 1, b, bre, bim);
}

void orc_op_m2l(const double *are, const double *aim, double z0x, double z0y, int p, double *bre, double *bim)
{
    cplx a[64], b[64];
    to_c(p + 1, are, aim, a);
    to_c(p + 1, bre, bim, b);
    op_m2l(a, z0x + I * z0y, p, b);
    from_c(p + 1, b, bre, bim);
}

void orc_op_l2l(const double *bre, const double *bim, double z0x, double z0y, int p, double *cre, double *cim)
{
    cplx b[64], c[64];
    to_c(p + 1, bre, bim, b);
    to_c(p + 1, cre, cim, c);
    op_l2l(b, z0x + I * z0y, p, c);
    from_c(p + 1, c, cre, cim);
}

void orc_op_l2p(const double *bre, const double *bim, double dx, double dy, int p, double *out2)
{
    cplx b[64];
    to_c(p + 1, bre, bim, b);
    cplx v = op_l2p(b, dx + I * dy, p);
    out2[0] = creal(v); out2[1] = cimag(v);
}

void orc_op_m2p(const double *are, const double *aim, double dx, double dy, int p, double *out2)
{
    cplx a[64];
    to_c(p + 1, are, aim, a);
    cplx v = op_m2p(a, dx + I * dy, p);
    out2[0] = creal(v); out2[1] = cimag(v);
}

void orc_op_p2l(double q, double z0x, double z0y, int p, double *bre, double *bim)
{
    cplx b[64];
    to_c(p + 1, bre, bim, b);
    op_p2l(q, z0x + I * z0y, p, b);
    from_c(p + 1, b, bre, bim);
}

/* ------------------------------------------------------------------------ */
/* The FMM repulsion (sec. 3.2.1), FP64.                                      */
/* stats (optional, 12 entries): cells, leaves, max level, |U| pairs (near    */
/* field particle pairs incl. self), |V|, |W| (cell-leaf), |X| (leaf-cell),   */
/* min coverage, max coverage, U entries, W entries, X entries.               */
/* Coverage of a leaf = particles reached through U, W and the V and X lists  */
/* of the leaf and its ancestors; it equals n when the lists are complete.    */
/* ------------------------------------------------------------------------ */
static cplx cell_center(const oroot *r, const ocell *c)
{
    double w = r->L / (double)((int64_t)1 << c->level);
    return (r->xmin + ((double)c->ix + 0.5) * w) + I * (r->ymin + ((double)c->iy + 0.5) * w);
}

int orc_fmm_repulsion(int64_t n, const double *x, const double *y, const double *m, double kr, int p,
                      int leaf_size, int bits, double *fx, double *fy, int64_t *stats)
{
    if (n <= 0 || p < 1 || p > 60 || leaf_size < 1 || bits < 1 || bits > 31) return -1;
    oroot r = root_square(n, x, y, bits);
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        key[i] = interleave(quantize(x[i], r.xmin, r.S, bits), quantize(y[i], r.ymin, r.S, bits), bits);
    orc_sort_by_key(n, key, perm);
    uint64_t *skey = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    cplx *z = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        skey[k] = key[perm[k]];
        z[k] = x[perm[k]] + I * y[perm[k]];
        q[k] = m[perm[k]];
    }
    otree t = build_tree(n, skey, bits, leaf_size);
    olists Ls = build_lists(&t);
    int64_t nc = t.n;
    int P1 = p + 1;
    cplx *M = (cplx *)calloc((size_t)(nc * P1), sizeof(cplx));
    cplx *Lc = (cplx *)calloc((size_t)(nc * P1), sizeof(cplx));
    int maxlev = 0;
    for (int64_t c = 0; c < nc; ++c) if (t.c[c].level > maxlev) maxlev = t.c[c].level;

    /* upward pass: outgoing expansions of leaves, then shifted to parents */
    for (int64_t c = 0; c < nc; ++c) {
        const ocell *cc = &t.c[c];
        if (is_leaf(cc)) op_p2m(cc->end - cc->begin, z + cc->begin, q + cc->begin, cell_center(&r, cc), p, M + c * P1);
    }
    for (int lev = maxlev; lev >= 1; --lev)
        for (int64_t c = 0; c < nc; ++c) {
            const ocell *cc = &t.c[c];
            if (cc->level != lev) continue;
            cplx z0 = cell_center(&r, cc) - cell_center(&r, &t.c[cc->parent]);
            op_m2m(M + c * P1, z0, p, M + (int64_t)cc->parent * P1);
        }
    /* downward pass: parent's incoming shifted down, plus the interacting    */
    /* cells' outgoing expansions converted to incoming ones                 */
    for (int lev = 0; lev <= maxlev; ++lev)
        for (int64_t c = 0; c < nc; ++c) {
            const ocell *cc = &t.c[c];
            if (cc->level != lev) continue;
            cplx zc = cell_center(&r, cc);
            if (cc->parent >= 0) op_l2l(Lc + (int64_t)cc->parent * P1, zc - cell_center(&r, &t.c[cc->parent]), p, Lc + c * P1);
            for (int64_t e = Ls.V.ptr[c]; e < Ls.V.ptr[c + 1]; ++e) {
                int32_t s = Ls.V.idx[e];
                op_m2l(M + (int64_t)s * P1, cell_center(&r, &t.c[s]) - zc, p, Lc + c * P1);
            }
            for (int64_t e = Ls.X.ptr[c]; e < Ls.X.ptr[c + 1]; ++e) {
                const ocell *cs = &t.c[Ls.X.idx[e]];
                for (int32_t j = cs->begin; j < cs->end; ++j) op_p2l(q[j], z[j] - zc, p, Lc + c * P1);
            }
        }
    /* evaluation: incoming expansion of the leaf, plus direct forces from   */
    /* the leaf itself and its neighbouring cells                            */
    double *gx = (double *)malloc(sizeof(double) * (size_t)n);
    double *gy = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t npairs = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : npairs)
    for (int64_t c = 0; c < nc; ++c) {
        const ocell *cc = &t.c[c];
        if (!is_leaf(cc)) continue;
        cplx zc = cell_center(&r, cc);
        for (int32_t i = cc->begin; i < cc->end; ++i) {
            cplx g = op_l2p(Lc + c * P1, z[i] - zc, p);
            for (int64_t e = Ls.W.ptr[c]; e < Ls.W.ptr[c + 1]; ++e) {
                const ocell *cs = &t.c[Ls.W.idx[e]];
                g += op_m2p(M + (int64_t)Ls.W.idx[e] * P1, z[i] - cell_center(&r, cs), p);
            }
            for (int64_t e = Ls.U.ptr[c]; e < Ls.U.ptr[c + 1]; ++e) {
                const ocell *cs = &t.c[Ls.U.idx[e]];
                npairs += cs->end - cs->begin;
                for (int32_t j = cs->begin; j < cs->end; ++j) {
                    if (j == i) continue;
                    cplx d = z[i] - z[j];
                    if (creal(d) == 0.0 && cimag(d) == 0.0) continue;
                    g += q[j] / d;
                }
            }
            /* F = kr m_i conj(phi') */
            gx[i] = kr * q[i] * creal(g);
            gy[i] = -kr * q[i] * cimag(g);
        }
    }
    for (int64_t k = 0; k < n; ++k) { fx[perm[k]] = gx[k]; fy[perm[k]] = gy[k]; }

    if (stats) {
        int64_t leaves = 0, nv = Ls.V.n, nw = 0, nx = 0, cmin = INT64_MAX, cmax = 0;
        for (int64_t c = 0; c < nc; ++c) {
            const ocell *cc = &t.c[c];
            if (!is_leaf(cc)) continue;
            ++leaves;
            int64_t cov = 0;
            for (int64_t e = Ls.U.ptr[c]; e < Ls.U.ptr[c + 1]; ++e) cov += t.c[Ls.U.idx[e]].end - t.c[Ls.U.idx[e]].begin;
            for (int64_t e = Ls.W.ptr[c]; e < Ls.W.ptr[c + 1]; ++e) cov += t.c[Ls.W.idx[e]].end - t.c[Ls.W.idx[e]].begin;
            nw += Ls.W.ptr[c + 1] - Ls.W.ptr[c];
            for (int64_t a = c; a >= 0; a = t.c[a].parent) {
                for (int64_t e = Ls.V.ptr[a]; e < Ls.V.ptr[a + 1]; ++e) cov += t.c[Ls.V.idx[e]].end - t.c[Ls.V.idx[e]].begin;
                for (int64_t e = Ls.X.ptr[a]; e < Ls.X.ptr[a + 1]; ++e) cov += t.c[Ls.X.idx[e]].end - t.c[Ls.X.idx[e]].begin;
            }
            if (cov < cmin) cmin = cov;
            if (cov > cmax) cmax = cov;
        }
        for (int64_t c = 0; c < nc; ++c) nx += Ls.X.ptr[c + 1] - Ls.X.ptr[c];
        stats[0] = nc; stats[1] = leaves; stats[2] = maxlev; stats[3] = npairs; stats[4] = nv;
        stats[5] = nw; stats[6] = nx; stats[7] = cmin; stats[8] = cmax; stats[9] = Ls.U.n; stats[10] = Ls.W.n;
        stats[11] = Ls.X.n;
    }
    free(gx); free(gy); free(M); free(Lc); free_lists(&Ls); free(t.c);
    free(key); free(perm); free(skey); free(z); free(q);
    return 0;
}

/* Lists for the tree of the given positions, flattened for comparison:       */
/* per list kind (U, V, W, X) a CSR pair over cells.  Returns the cell count,  */
/* or -(needed) if a capacity is too small.  caps/lens: [5] = cells, U, V, W, X */
int64_t orc_fmm_lists(int64_t n, const double *x, const double *y, int leaf_size, int bits,
                      const int64_t *caps, int32_t *cells10, int64_t *ptrs /* 4*(cells+1) */,
                      int32_t *uidx, int32_t *vidx, int32_t *widx, int32_t *xidx, int64_t *lens)
{
    oroot r = root_square(n, x, y, bits);
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        key[i] = interleave(quantize(x[i], r.xmin, r.S, bits), quantize(y[i], r.ymin, r.S, bits), bits);
    orc_sort_by_key(n, key, perm);
    uint64_t *skey = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    for (int64_t k = 0; k < n; ++k) skey[k] = key[perm[k]];
    otree t = build_tree(n, skey, bits, leaf_size);
    olists Ls = build_lists(&t);
    lens[0] = t.n; lens[1] = Ls.U.n; lens[2] = Ls.V.n; lens[3] = Ls.W.n; lens[4] = Ls.X.n;
    int64_t ret = t.n;
    if (t.n > caps[0] || Ls.U.n > caps[1] || Ls.V.n > caps[2] || Ls.W.n > caps[3] || Ls.X.n > caps[4]) {
        ret = -1;
    } else {
        for (int64_t i = 0; i < t.n; ++i) {
            const ocell *c = &t.c[i];
            int32_t *o = cells10 + 10 * i;
            o[0] = c->level; o[1] = c->ix; o[2] = c->iy; o[3] = c->begin; o[4] = c->end; o[5] = c->parent;
            for (int qq = 0; qq < 4; ++qq) o[6 + qq] = c->child[qq];
        }
        memcpy(ptrs, Ls.U.ptr, sizeof(int64_t) * (size_t)(t.n + 1));
        memcpy(ptrs + (t.n + 1), Ls.V.ptr, sizeof(int64_t) * (size_t)(t.n + 1));
        memcpy(ptrs + 2 * (t.n + 1), Ls.W.ptr, sizeof(int64_t) * (size_t)(t.n + 1));
        memcpy(ptrs + 3 * (t.n + 1), Ls.X.ptr, sizeof(int64_t) * (size_t)(t.n + 1));
        if (Ls.U.n) memcpy(uidx, Ls.U.idx, sizeof(int32_t) * (size_t)Ls.U.n);
        if (Ls.V.n) memcpy(vidx, Ls.V.idx, sizeof(int32_t) * (size_t)Ls.V.n);
        if (Ls.W.n) memcpy(widx, Ls.W.idx, sizeof(int32_t) * (size_t)Ls.W.n);
        if (Ls.X.n) memcpy(xidx, Ls.X.idx, sizeof(int32_t) * (size_t)Ls.X.n);
    }
    free_lists(&Ls); free(t.c); free(key); free(perm); free(skey);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* Kamada-Kawai (sec. 3.1).  Energy                                           */
/*   E = sum_{i<j} d_ij^-2 (|p_i - p_j| - l d_ij)^2                           */
/* minimised by localized stress majorization, all nodes updated together    */
/* from the previous positions:                                               */
/*   p_i' = sum_{j!=i} w_ij (p_j + l_ij u_ij) / sum_{j!=i} w_ij,               */
/*   w_ij = d_ij^-2, l_ij = l d_ij, u_ij = (p_i - p_j)/|p_i - p_j| (0 if       */
/*   coincident).  dist is the n*n hop matrix of one connected component.     */
/*   For n = 2 the update maps the pair's distance r to |2l - r| (a           */
/*   reflection that never settles when r < 2l), so there each node moves    */
/*   half way: the pair lands at distance l about its midpoint in one step.   */
/* ------------------------------------------------------------------------ */
double orc_kk_energy(int32_t n, const int32_t *dist, double l, const double *x, const double *y)
{
    double e = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) {
            double d = (double)dist[(int64_t)i * n + j];
            double dx = x[i] - x[j], dy = y[i] - y[j];
            double r = sqrt(dx * dx + dy * dy) - l * d;
            e += r * r / (d * d);
        }
    return e;
}

void orc_kk_steps(int32_t n, const int32_t *dist, double l, int32_t steps, double *x, double *y)
{
    double *nx = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *ny = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t s = 0; s < steps; ++s) {
        for (int32_t i = 0; i < n; ++i) {
            double sw = 0.0, ax = 0.0, ay = 0.0;
            for (int32_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double d = (double)dist[(int64_t)i * n + j];
                double w = 1.0 / (d * d);
                double dx = x[i] - x[j], dy = y[i] - y[j];
                double r = sqrt(dx * dx + dy * dy);
                double ux = r > 0.0 ? dx / r : 0.0, uy = r > 0.0 ? dy / r : 0.0;
                sw += w;
                ax += w * (x[j] + l * d * ux);
                ay += w * (y[j] + l * d * uy);
            }
            nx[i] = sw > 0.0 ? ax / sw : x[i];
            ny[i] = sw > 0.0 ? ay / sw : y[i];
            if (n == 2) { /* the update reflects a pair's distance r to |2l - r|: relax it by 1/2 */
                nx[i] = 0.5 * (x[i] + nx[i]);
                ny[i] = 0.5 * (y[i] + ny[i]);
            }
        }
        memcpy(x, nx, sizeof(double) * (size_t)n);
        memcpy(y, ny, sizeof(double) * (size_t)n);
    }
    free(nx); free(ny);
}

/* ------------------------------------------------------------------------ */
/* Kamada-Kawai on the graph of components (sec. 4).  The meta-graph has     */
/* real edge lengths, so d_ij here is the length of the shortest path and     */
/* the energy is E = sum_{i<j} d_ij^-2 (|p_i - p_j| - d_ij)^2 (no extra       */
/* length scale).  It is minimised by localized stress majorization in its   */
/* sequential form: in one sweep, nodes 0, 1, ..., n-1 in turn move to       */
/*   p_i' = sum_{j!=i} w_ij (p_j + d_ij u_ij) / sum_{j!=i} w_ij               */
/* using the positions current at that moment (already moved nodes included).*/
/* Each move minimises a majorizing function of E in p_i alone, so E never   */
/* increases.  dist is the n*n matrix (row-major, FP64), > 0 off the         */
/* diagonal.                                                                  */
/* ------------------------------------------------------------------------ */
double orc_stress(int32_t n, const double *dist, const double *x, const double *y)
{
    double e = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) {
            double d = dist[(int64_t)i * n + j];
            double dx = x[i] - x[j], dy = y[i] - y[j];
            double r = sqrt(dx * dx + dy * dy) - d;
            e += r * r / (d * d);
        }
    return e;
}

void orc_kk_sweeps(int32_t n, const double *dist, int32_t sweeps, double *x, double *y)
{
    for (int32_t s = 0; s < sweeps; ++s) {
        for (int32_t i = 0; i < n; ++i) {
            double sw = 0.0, ax = 0.0, ay = 0.0;
            for (int32_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double d = dist[(int64_t)i * n + j];
                double w = 1.0 / (d * d);
                double dx = x[i] - x[j], dy = y[i] - y[j];
                double r = sqrt(dx * dx + dy * dy);
                double ux = r > 0.0 ? dx / r : 0.0, uy = r > 0.0 ? dy / r : 0.0;
                sw += w;
                ax += w * (x[j] + d * ux);
                ay += w * (y[j] + d * uy);
            }
            if (sw > 0.0) {
                x[i] = ax / sw;
                y[i] = ay / sw;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Barnes-Hut repulsion (sec. 3.2.1 names it as the O(N log N) approach the  */
/* FMM improves on; Barnes & Hut 1986).  The same quadtree as the FMM.  Every */
/* cell carries its total mass and centre of mass.  For a target, the tree is */
/* walked from the root, children in quadrant order: a cell that does not     */
/* hold the target and whose side s and distance d from the target to its     */
/* centre of mass satisfy s < theta d acts as one particle (its mass at its   */
/* centre of mass); otherwise its children are visited, and a leaf that is    */
/* visited contributes its particles directly.  Same force law and masses as  */
/* orc_repulsion_exact; theta = 0 gives the exact sum.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    const otree *t;
    const double *cx, *cy, *cm, *side;  /* per cell */
    const double *px, *py, *pq;         /* sorted particles */
    double theta;
} obh;

static void bh_visit(const obh *b, int64_t c, int64_t k, double tx, double ty, double *ax, double *ay)
{
    const ocell *cc = &b->t->c[c];
    int holds = k >= cc->begin && k < cc->end;
    if (!holds) {
        double dx = tx - b->cx[c], dy = ty - b->cy[c];
        double d2 = dx * dx + dy * dy;
        if (b->side[c] * b->side[c] < b->theta * b->theta * d2) {
            *ax += b->cm[c] * dx / d2;
            *ay += b->cm[c] * dy / d2;
            return;
        }
    }
    if (is_leaf(cc)) {
        for (int64_t j = cc->begin; j < cc->end; ++j) {
            if (j == k) continue;
            double dx = tx - b->px[j], dy = ty - b->py[j];
            double d2 = dx * dx + dy * dy;
            if (d2 == 0.0) continue;
            *ax += b->pq[j] * dx / d2;
            *ay += b->pq[j] * dy / d2;
        }
        return;
    }
    for (int q = 0; q < 4; ++q)
        if (cc->child[q] >= 0) bh_visit(b, cc->child[q], k, tx, ty, ax, ay);
}

int orc_bh_repulsion(int64_t n, const double *x, const double *y, const double *m, double kr, double theta,
                     int leaf_size, int bits, int64_t nt, const int64_t *targets, double *fx, double *fy)
{
    if (n <= 0 || theta < 0.0 || leaf_size < 1 || bits < 1 || bits > 31) return -1;
    oroot r = root_square(n, x, y, bits);
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        key[i] = interleave(quantize(x[i], r.xmin, r.S, bits), quantize(y[i], r.ymin, r.S, bits), bits);
    orc_sort_by_key(n, key, perm);
    uint64_t *skey = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    double *px = (double *)malloc(sizeof(double) * (size_t)n);
    double *py = (double *)malloc(sizeof(double) * (size_t)n);
    double *pq = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        skey[k] = key[perm[k]];
        px[k] = x[perm[k]];
        py[k] = y[perm[k]];
        pq[k] = m[perm[k]];
        rank[perm[k]] = k;
    }
    otree t = build_tree(n, skey, bits, leaf_size);
    int64_t nc = t.n;
    double *cx = (double *)malloc(sizeof(double) * (size_t)nc);
    double *cy = (double *)malloc(sizeof(double) * (size_t)nc);
    double *cm = (double *)malloc(sizeof(double) * (size_t)nc);
    double *side = (double *)malloc(sizeof(double) * (size_t)nc);
    for (int64_t c = 0; c < nc; ++c) {
        double sm = 0.0, sx = 0.0, sy = 0.0;
        for (int64_t j = t.c[c].begin; j < t.c[c].end; ++j) {
            sm += pq[j];
            sx += pq[j] * px[j];
            sy += pq[j] * py[j];
        }
        cm[c] = sm;
        cx[c] = sx / sm;
        cy[c] = sy / sm;
        side[c] = r.L / (double)((int64_t)1 << t.c[c].level);
    }
    obh b = {&t, cx, cy, cm, side, px, py, pq, theta};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < nt; ++s) {
        int64_t i = targets ? targets[s] : s;
        int64_t k = rank[i];
        double ax = 0.0, ay = 0.0;
        bh_visit(&b, 0, k, px[k], py[k], &ax, &ay);
        fx[s] = kr * m[i] * ax;
        fy[s] = kr * m[i] * ay;
    }
    free(cx); free(cy); free(cm); free(side); free(t.c);
    free(key); free(perm); free(rank); free(skey); free(px); free(py); free(pq);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Kamada-Kawai's own minimiser (sec. 3.1: Newton-Raphson).  With           */
/* E = sum_{i<j} w_ij (r_ij - L_ij)^2, w_ij = d_ij^-2, L_ij = l d_ij and      */
/* r_ij = |p_i - p_j|, the derivatives of E in the position of one node m,    */
/* over the other nodes i (pairs at r = 0 contribute nothing), are            */
/*   dE/dx_m        = sum 2 w (dx - L dx / r)                                 */
/*   d2E/dx_m^2     = sum 2 w (1 - L dy^2 / r^3)                              */
/*   d2E/dx_m dy_m  = sum 2 w L dx dy / r^3                                   */
/*   d2E/dy_m^2     = sum 2 w (1 - L dx^2 / r^3)        with dx = x_m - x_i,  */
/* and the part of E that depends on p_m is E_m = sum w (r - L)^2.            */
/* A move takes the node with the largest gradient norm Delta_m (the lowest   */
/* index on a tie) and makes Newton-Raphson steps on p_m alone until Delta_m  */
/* < eps l or `inner` steps were made.  A step solves the 2x2 system when the */
/* Hessian is positive definite; otherwise it is the gradient step            */
/* -g / (2 sum w).  It is halved (at most 30 times) until E_m decreases; a    */
/* step that finds no decrease ends the move.  Moves repeat until every       */
/* Delta < eps l or `moves` moves were made.  Every quantity is computed from */
/* the current positions, from scratch.  Returns the number of moves made.    */
/* ------------------------------------------------------------------------ */
void orc_kk_grad_hess(int32_t n, const int32_t *dist, double l, int32_t m, const double *x, const double *y,
                      double *out5)
{
    double gx = 0.0, gy = 0.0, hxx = 0.0, hxy = 0.0, hyy = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (i == m) continue;
        double d = (double)dist[(int64_t)m * n + i];
        double w = 1.0 / (d * d), L = l * d;
        double dx = x[m] - x[i], dy = y[m] - y[i];
        double r = sqrt(dx * dx + dy * dy);
        if (r == 0.0) continue;
        double r3 = r * r * r;
        gx += 2.0 * w * (dx - L * dx / r);
        gy += 2.0 * w * (dy - L * dy / r);
        hxx += 2.0 * w * (1.0 - L * dy * dy / r3);
        hxy += 2.0 * w * L * dx * dy / r3;
        hyy += 2.0 * w * (1.0 - L * dx * dx / r3);
    }
    out5[0] = gx; out5[1] = gy; out5[2] = hxx; out5[3] = hxy; out5[4] = hyy;
}

static double kk_node_energy(int32_t n, const int32_t *dist, double l, int32_t m, double px, double py,
                             const double *x, const double *y)
{
    double e = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (i == m) continue;
        double d = (double)dist[(int64_t)m * n + i];
        double dx = px - x[i], dy = py - y[i];
        double r = sqrt(dx * dx + dy * dy) - l * d;
        e += r * r / (d * d);
    }
    return e;
}

int32_t orc_kk_newton(int32_t n, const int32_t *dist, double l, double eps, int32_t moves, int32_t inner,
                      double *x, double *y)
{
    double gh[5];
    const double tol = eps * l;
    int32_t done = 0;
    for (; done < moves; ++done) {
        int32_t m = -1;
        double best = -1.0;
        for (int32_t i = 0; i < n; ++i) {
            orc_kk_grad_hess(n, dist, l, i, x, y, gh);
            double dlt = sqrt(gh[0] * gh[0] + gh[1] * gh[1]);
            if (dlt > best) { best = dlt; m = i; }
        }
        if (m < 0 || best < tol) break;
        double sw = 0.0;
        for (int32_t i = 0; i < n; ++i)
            if (i != m) sw += 1.0 / ((double)dist[(int64_t)m * n + i] * (double)dist[(int64_t)m * n + i]);
        for (int32_t s = 0; s < inner; ++s) {
            orc_kk_grad_hess(n, dist, l, m, x, y, gh);
            if (sqrt(gh[0] * gh[0] + gh[1] * gh[1]) < tol) break;
            double det = gh[2] * gh[4] - gh[3] * gh[3];
            double sx, sy;
            if (gh[2] > 0.0 && det > 0.0) {
                sx = -(gh[4] * gh[0] - gh[3] * gh[1]) / det;
                sy = -(gh[2] * gh[1] - gh[3] * gh[0]) / det;
            } else {
                sx = -gh[0] / (2.0 * sw);
                sy = -gh[1] / (2.0 * sw);
            }
            double e0 = kk_node_energy(n, dist, l, m, x[m], y[m], x, y);
            int moved = 0;
            for (int h = 0; h <= 30; ++h) {
                double nx = x[m] + sx, ny = y[m] + sy;
                if (kk_node_energy(n, dist, l, m, nx, ny, x, y) < e0) {
                    x[m] = nx;
                    y[m] = ny;
                    moved = 1;
                    break;
                }
                sx *= 0.5;
                sy *= 0.5;
            }
            if (!moved) break;
        }
    }
    return done;
}
