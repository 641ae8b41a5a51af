// Octree / interaction-list kernels (see tree_kernels.hip).
#pragma once
#include <cmath>
#include "common.h"

namespace fmm {

constexpr int kBBoxBlocks = 1024;

struct BoxArrays {
    int32_t *level, *first, *count, *parent, *child_begin, *nchild;
    uint64_t *morton;
};

struct TreeArgs {
    BoxArrays bx;
    const int32_t *lvl_begin; // device [kMaxDepth + 2]
    int D, nboxes;
    int uniform; // every level full: no coarser adjacent leaves, no W lists
    const int32_t *leafcol; // per box: a colleague (other than itself) is a leaf; NULL = unknown
};

void plan_init(const double *given_root, double *root_dev, int *bad, hipStream_t s);
// uniform trees: U counts (W and X set empty) or U contents, without colleagues
void ulist_uniform(const TreeArgs &a, int which, int64_t *ucnt, int64_t *wcnt, int64_t *xcnt, const int64_t *uoff,
                   int32_t *usrc, hipStream_t s);
// uniform trees: V counts and complete M2L slot rows (no fill needed)
void vslot_uniform(const TreeArgs &a, int64_t *cnt, int32_t *vslot, hipStream_t s);
void bbox(const double *xyz, int n, double *part, double *root, hipStream_t s);
void morton_keys(const double *xyz, int n, const double *root_dev, int D, uint64_t *keys,
                 int32_t *idx, int *bad, hipStream_t s);
void gather_sorted(const double *xyz, const int32_t *perm, int n, double *xs, double *ys,
                   double *zs, hipStream_t s);
void uniform_boxes(const uint64_t *keys, int n, int D, int nboxes, BoxArrays bx, int32_t *lvl_begin,
                   hipStream_t s);
// adaptive tree: boxes emitted per particle (count, then fill after a scan)
void emit_count(const uint64_t *keys, int n, int D, int leaf_size, int64_t *cnt, hipStream_t s);
void adaptive_boxes(const uint64_t *keys, int n, int D, int leaf_size, const int64_t *off, int nb,
                    uint64_t *elevel, int32_t *eidx, uint64_t *tk, int32_t *tv, int32_t *efirst,
                    int32_t *ecount, uint64_t *emorton, int32_t *sort_scratch, BoxArrays bx,
                    int32_t *lvl_begin, hipStream_t s);
void colleagues(const TreeArgs &a, int32_t *coll, int64_t *zero, int32_t *leafcol, hipStream_t s);
void vlist(const TreeArgs &a, const int32_t *coll, int which, int64_t *cnt, const int64_t *off,
           int32_t *src, int32_t *vslot, hipStream_t s);
void uwlist(const TreeArgs &a, const int32_t *coll, int which, int64_t *ucnt, const int64_t *uoff,
            int32_t *usrc, int64_t *wcnt, const int64_t *woff, int32_t *wsrc, int64_t *xcnt, hipStream_t s);
void w_pairs(const int64_t *woff, const int32_t *wsrc, int nboxes, uint64_t *key, int32_t *val, hipStream_t s);
void flags(const BoxArrays &bx, int nboxes, const int64_t *xcnt, const int64_t *vcnt, int64_t *fleaf,
           int64_t *fnon, int64_t *fx, int64_t *fv, hipStream_t s);
void compact(const int64_t *flag, const int64_t *pos, int nboxes, int32_t *out, hipStream_t s);
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void mark(const int32_t *idx, int64_t n, int32_t *flag, hipStream_t s); // flag[idx[i]] = 1
void m2l_tiles(const BoxArrays &bx, const int32_t *tg, int nt, int uniform, uint64_t *key, int32_t *val,
               uint64_t *tk, int32_t *tv, int32_t *sort_scratch, int *octoff, int32_t *slots,
               int64_t slot_cap, hipStream_t s);

} // namespace fmm
