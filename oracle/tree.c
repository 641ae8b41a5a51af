/*
 * Reference octree and interaction lists.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper fixes only the principle (Sec. 1: recursive subdivision into
 * boxes, a full tree for uniform data and a partially overlapping tree
 * otherwise; Sec. 3.5: a box with more than s particles is subdivided; Sec. 3.4:
 * at most 189 boxes in an interaction list; Sec. 3.1: P2L when a box lies in
 * the near region of a childless box).  Everything else is a stated reading:
 *
 *   root      lo_k = min_i x_ik, W = max_k (max_i x_ik - lo_k) (W = 1 if 0),
 *             unless the caller passes {lo, W};
 *   keys      g_k = clamp(floor((x_k - lo_k) * (2^D / W)), 0, 2^D - 1) in FP64,
 *             bit b of g_x, g_y, g_z at key bits 3b+2, 3b+1, 3b; D is the
 *             uniform depth or the adaptive depth cap;
 *   order     particles by (key, original index); boxes by (level, Morton code);
 *   uniform   every box of every level 0..D exists, empty or not;
 *   adaptive  split iff count > s and level < D; empty children are not made;
 *   lists     Carrier-Greengard-Rokhlin: U (adjacent leaves, self included),
 *             V (children of the parent's colleagues not adjacent to the box,
 *             levels >= 2), W (descendants of colleagues not adjacent to the
 *             leaf whose parent is adjacent), X (transpose of W); "adjacent"
 *             means the closed cubes touch, tested in integer finest-grid
 *             coordinates; every list sorted by source box number.
 *
 * The construction is the plain one: breadth-first subdivision by scanning
 * the sorted keys, and lists by walking colleagues and descendants.
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { int32_t *v; int64_t n, cap; } ivec;
static void ivec_push(ivec *a, int32_t x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 64;
        a->v = realloc(a->v, sizeof(int32_t) * (size_t)a->cap);
    }
    a->v[a->n++] = x;
}

struct oracle_tree {
    int64_t n;
    int D, depth;
    double lo[3], W;
    int64_t *perm;
    uint64_t *key;
    int64_t nboxes, cap;
    int32_t *level, *parent, *child_begin, *nchild;
    uint64_t *morton;
    int64_t *first, *count;
    int64_t level_begin[24];
    int64_t *off[4];   /* U V W X */
    int32_t *src[4];
    int64_t nlist[4];
};

typedef struct { uint64_t key; int64_t idx; } kv;
static int kv_cmp(const void *a, const void *b)
{
    const kv *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static void coords(uint64_t code, int l, int64_t c[3])
{
    c[0] = c[1] = c[2] = 0;
    for (int b = 0; b < l; ++b) {
        c[0] |= (int64_t)((code >> (3 * b + 2)) & 1) << b;
        c[1] |= (int64_t)((code >> (3 * b + 1)) & 1) << b;
        c[2] |= (int64_t)((code >> (3 * b)) & 1) << b;
    }
}

static uint64_t interleave(const int64_t c[3], int l)
{
    uint64_t k = 0;
    for (int b = 0; b < l; ++b) {
        k |= (uint64_t)((c[0] >> b) & 1) << (3 * b + 2);
        k |= (uint64_t)((c[1] >> b) & 1) << (3 * b + 1);
        k |= (uint64_t)((c[2] >> b) & 1) << (3 * b);
    }
    return k;
}

static void add_box(oracle_tree *t, int l, uint64_t code, int64_t first, int64_t count,
                    int32_t parent)
{
    if (t->nboxes == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 1024;
        t->level = realloc(t->level, sizeof(int32_t) * (size_t)t->cap);
        t->parent = realloc(t->parent, sizeof(int32_t) * (size_t)t->cap);
        t->child_begin = realloc(t->child_begin, sizeof(int32_t) * (size_t)t->cap);
        t->nchild = realloc(t->nchild, sizeof(int32_t) * (size_t)t->cap);
        t->morton = realloc(t->morton, sizeof(uint64_t) * (size_t)t->cap);
        t->first = realloc(t->first, sizeof(int64_t) * (size_t)t->cap);
        t->count = realloc(t->count, sizeof(int64_t) * (size_t)t->cap);
    }
    int64_t b = t->nboxes++;
    t->level[b] = l; t->morton[b] = code; t->first[b] = first; t->count[b] = count;
    t->parent[b] = parent; t->child_begin[b] = -1; t->nchild[b] = 0;
}

/* box number of (level, code), or -1 */
static int32_t find_box(const oracle_tree *t, int l, uint64_t code)
{
    int64_t lo = t->level_begin[l], hi = t->level_begin[l + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (t->morton[mid] < code) lo = mid + 1; else hi = mid;
    }
    return (lo < t->level_begin[l + 1] && t->morton[lo] == code) ? (int32_t)lo : -1;
}

static int adjacent(const oracle_tree *t, int32_t a, int32_t b)
{
    int64_t ca[3], cb[3];
    coords(t->morton[a], t->level[a], ca);
    coords(t->morton[b], t->level[b], cb);
    int64_t sa = (int64_t)1 << (t->D - t->level[a]), sb = (int64_t)1 << (t->D - t->level[b]);
    for (int k = 0; k < 3; ++k) {
        int64_t la = ca[k] * sa, lb = cb[k] * sb;
        if (la > lb + sb || lb > la + sa) return 0;
    }
    return 1;
}

static int is_leaf(const oracle_tree *t, int32_t b) { return t->nchild[b] == 0; }

/* colleagues: same-level adjacent boxes, the box itself included */
static int colleagues(const oracle_tree *t, int32_t b, int32_t out[27])
{
    int l = t->level[b], m = 0;
    int64_t c[3], nb[3], side = (int64_t)1 << l;
    coords(t->morton[b], l, c);
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                nb[0] = c[0] + dx; nb[1] = c[1] + dy; nb[2] = c[2] + dz;
                if (nb[0] < 0 || nb[1] < 0 || nb[2] < 0 || nb[0] >= side || nb[1] >= side ||
                    nb[2] >= side)
                    continue;
                int32_t f = find_box(t, l, interleave(nb, l));
                if (f >= 0) out[m++] = f;
            }
    return m;
}

static void u_descend(const oracle_tree *t, int32_t c, int32_t b, ivec *out)
{
    if (is_leaf(t, c)) { ivec_push(out, c); return; }
    for (int k = 0; k < t->nchild[c]; ++k) {
        int32_t d = t->child_begin[c] + k;
        if (adjacent(t, d, b)) u_descend(t, d, b, out);
    }
}

static void w_descend(const oracle_tree *t, int32_t c, int32_t b, ivec *out)
{
    for (int k = 0; k < t->nchild[c]; ++k) {
        int32_t d = t->child_begin[c] + k;
        if (!adjacent(t, d, b)) ivec_push(out, d);
        else if (!is_leaf(t, d)) w_descend(t, d, b, out);
    }
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void to_csr(oracle_tree *t, int which, ivec *lists)
{
    int64_t tot = 0;
    t->off[which] = malloc(sizeof(int64_t) * (size_t)(t->nboxes + 1));
    for (int64_t b = 0; b < t->nboxes; ++b) {
        t->off[which][b] = tot;
        tot += lists[b].n;
    }
    t->off[which][t->nboxes] = tot;
    t->src[which] = malloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
    for (int64_t b = 0; b < t->nboxes; ++b) {
        qsort(lists[b].v, (size_t)lists[b].n, sizeof(int32_t), cmp_i32);
        if (lists[b].n) memcpy(t->src[which] + t->off[which][b], lists[b].v,
                               sizeof(int32_t) * (size_t)lists[b].n);
        free(lists[b].v);
        lists[b].v = NULL; lists[b].n = lists[b].cap = 0;
    }
    t->nlist[which] = tot;
}

oracle_tree *oracle_tree_build(int64_t n, const double *xyz, const double *root,
                               int uniform_depth, int max_depth, int leaf_size)
{
    if (n < 1 || !xyz) return NULL;
    int D = uniform_depth >= 0 ? uniform_depth : max_depth;
    if (D < 0 || D > 21 || (uniform_depth < 0 && leaf_size < 1)) return NULL;
    oracle_tree *t = calloc(1, sizeof(*t));
    t->n = n; t->D = D;
    if (root) {
        t->lo[0] = root[0]; t->lo[1] = root[1]; t->lo[2] = root[2]; t->W = root[3];
    } else {
        double hi[3];
        for (int k = 0; k < 3; ++k) { t->lo[k] = xyz[k]; hi[k] = xyz[k]; }
        for (int64_t i = 1; i < n; ++i)
            for (int k = 0; k < 3; ++k) {
                if (xyz[3 * i + k] < t->lo[k]) t->lo[k] = xyz[3 * i + k];
                if (xyz[3 * i + k] > hi[k]) hi[k] = xyz[3 * i + k];
            }
        t->W = 0.0;
        for (int k = 0; k < 3; ++k)
            if (hi[k] - t->lo[k] > t->W) t->W = hi[k] - t->lo[k];
        if (t->W == 0.0) t->W = 1.0;
    }
    /* quantisation and keys */
    double scale = ldexp(1.0, D) / t->W;
    int64_t gmax = ((int64_t)1 << D) - 1;
    kv *a = malloc(sizeof(kv) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t g[3];
        for (int k = 0; k < 3; ++k) {
            double s = (xyz[3 * i + k] - t->lo[k]) * scale;
            double f = floor(s);
            if (!(f >= 0.0)) f = 0.0;
            if (f > (double)gmax) f = (double)gmax;
            g[k] = (int64_t)f;
        }
        a[i].key = interleave(g, D);
        a[i].idx = i;
    }
    qsort(a, (size_t)n, sizeof(kv), kv_cmp);
    t->perm = malloc(sizeof(int64_t) * (size_t)n);
    t->key = malloc(sizeof(uint64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) { t->perm[i] = a[i].idx; t->key[i] = a[i].key; }
    free(a);

    /* breadth-first subdivision: parents are visited in Morton order, so the
     * children of one level come out in Morton order as well */
    add_box(t, 0, 0, 0, n, -1);
    t->level_begin[0] = 0;
    int l = 0;
    int64_t lb = 0, le = 1;
    for (;;) {
        t->level_begin[l + 1] = le;
        if (l == D) break;
        for (int64_t b = lb; b < le; ++b) {
            int split = uniform_depth >= 0 ? 1 : (t->count[b] > leaf_size);
            if (!split) continue;
            int shift = 3 * (D - l - 1);
            int64_t s = t->first[b], e = s + t->count[b];
            t->child_begin[b] = (int32_t)t->nboxes;
            for (int o = 0; o < 8; ++o) {
                uint64_t code = t->morton[b] * 8 + (uint64_t)o;
                int64_t f = s;
                while (s < e && (t->key[s] >> shift) == code) ++s;
                if (s > f || uniform_depth >= 0) {
                    add_box(t, l + 1, code, f, s - f, (int32_t)b);
                    t->nchild[b]++;
                }
            }
        }
        if (t->nboxes == le) break;
        lb = le; le = t->nboxes; ++l;
    }
    t->depth = l;
    for (int k = l + 1; k < 24; ++k) t->level_begin[k] = t->nboxes;
    for (int64_t b = 0; b < t->nboxes; ++b)
        if (t->nchild[b] == 0) t->child_begin[b] = -1;

    /* interaction lists */
    ivec *L[4];
    for (int w = 0; w < 4; ++w) L[w] = calloc((size_t)t->nboxes, sizeof(ivec));
    for (int64_t b = 0; b < t->nboxes; ++b) {
        int32_t col[27];
        int nc = colleagues(t, (int32_t)b, col);
        int lvl = t->level[b];
        if (lvl >= 2) { /* V */
            int32_t pc[27];
            int np = colleagues(t, t->parent[b], pc);
            for (int i = 0; i < np; ++i)
                for (int k = 0; k < t->nchild[pc[i]]; ++k) {
                    int32_t d = t->child_begin[pc[i]] + k;
                    if (!adjacent(t, d, (int32_t)b)) ivec_push(&L[1][b], d);
                }
        }
        if (!is_leaf(t, (int32_t)b)) continue;
        for (int i = 0; i < nc; ++i) { /* U (same or finer) and W */
            u_descend(t, col[i], (int32_t)b, &L[0][b]);
            if (col[i] != b) w_descend(t, col[i], (int32_t)b, &L[2][b]);
        }
        for (int32_t anc = t->parent[b]; anc >= 0; anc = t->parent[anc]) { /* U, coarser */
            int32_t ac[27];
            int na = colleagues(t, anc, ac);
            for (int i = 0; i < na; ++i)
                if (ac[i] != anc && is_leaf(t, ac[i]) && adjacent(t, ac[i], (int32_t)b))
                    ivec_push(&L[0][b], ac[i]);
        }
    }
    for (int64_t b = 0; b < t->nboxes; ++b) /* X = transpose of W */
        for (int64_t k = 0; k < L[2][b].n; ++k) ivec_push(&L[3][L[2][b].v[k]], (int32_t)b);
    for (int w = 0; w < 4; ++w) { to_csr(t, w, L[w]); free(L[w]); }
    return t;
}

void oracle_tree_free(oracle_tree *t)
{
    if (!t) return;
    free(t->perm); free(t->key); free(t->level); free(t->parent); free(t->child_begin);
    free(t->nchild); free(t->morton); free(t->first); free(t->count);
    for (int w = 0; w < 4; ++w) { free(t->off[w]); free(t->src[w]); }
    free(t);
}

void oracle_tree_sizes(const oracle_tree *t, int64_t s[7])
{
    s[0] = t->nboxes; s[1] = t->nlist[0]; s[2] = t->nlist[1]; s[3] = t->nlist[2];
    s[4] = t->nlist[3]; s[5] = t->depth; s[6] = t->D;
}

void oracle_tree_root(const oracle_tree *t, double r[4])
{
    r[0] = t->lo[0]; r[1] = t->lo[1]; r[2] = t->lo[2]; r[3] = t->W;
}

#define CP(dst, srcp, cnt) do { if (dst) memcpy(dst, srcp, sizeof(*(dst)) * (size_t)(cnt)); } while (0)
void oracle_tree_export(const oracle_tree *t, int64_t *perm, int32_t *level, uint64_t *morton,
                        int64_t *first, int64_t *count, int32_t *parent, int32_t *child_begin,
                        int32_t *nchild, int64_t *U_off, int32_t *U_src, int64_t *V_off,
                        int32_t *V_src, int64_t *W_off, int32_t *W_src, int64_t *X_off,
                        int32_t *X_src)
{
    CP(perm, t->perm, t->n);
    CP(level, t->level, t->nboxes); CP(morton, t->morton, t->nboxes);
    CP(first, t->first, t->nboxes); CP(count, t->count, t->nboxes);
    CP(parent, t->parent, t->nboxes); CP(child_begin, t->child_begin, t->nboxes);
    CP(nchild, t->nchild, t->nboxes);
    CP(U_off, t->off[0], t->nboxes + 1); CP(U_src, t->src[0], t->nlist[0]);
    CP(V_off, t->off[1], t->nboxes + 1); CP(V_src, t->src[1], t->nlist[1]);
    CP(W_off, t->off[2], t->nboxes + 1); CP(W_src, t->src[2], t->nlist[2]);
    CP(X_off, t->off[3], t->nboxes + 1); CP(X_src, t->src[3], t->nlist[3]);
}

/* accessors for the FMM driver in the same library */
int64_t oracle_tree_n(const oracle_tree *t) { return t->n; }
int64_t oracle_tree_nboxes(const oracle_tree *t) { return t->nboxes; }
int oracle_tree_depth(const oracle_tree *t) { return t->depth; }
const int64_t *oracle_tree_perm(const oracle_tree *t) { return t->perm; }
const int32_t *oracle_tree_level(const oracle_tree *t) { return t->level; }
const int32_t *oracle_tree_parent(const oracle_tree *t) { return t->parent; }
const int32_t *oracle_tree_child_begin(const oracle_tree *t) { return t->child_begin; }
const int32_t *oracle_tree_nchild(const oracle_tree *t) { return t->nchild; }
const int64_t *oracle_tree_first(const oracle_tree *t) { return t->first; }
const int64_t *oracle_tree_count(const oracle_tree *t) { return t->count; }
const int64_t *oracle_tree_off(const oracle_tree *t, int w) { return t->off[w]; }
const int32_t *oracle_tree_src(const oracle_tree *t, int w) { return t->src[w]; }
const int64_t *oracle_tree_level_begin(const oracle_tree *t) { return t->level_begin; }
void oracle_tree_center(const oracle_tree *t, int32_t b, double c[3])
{
    int64_t g[3];
    coords(t->morton[b], t->level[b], g);
    double h = t->W / ldexp(1.0, t->level[b]);
    for (int k = 0; k < 3; ++k) c[k] = t->lo[k] + ((double)g[k] + 0.5) * h;
}
double oracle_tree_width(const oracle_tree *t, int l) { return t->W / ldexp(1.0, l); }
void oracle_tree_coords(const oracle_tree *t, int32_t b, int64_t g[3])
{
    coords(t->morton[b], t->level[b], g);
}
