// Octree and interaction-list kernels.
//
// The paper fixes only the principle of the tree (Sec. 1: recursive
// subdivision, a full tree for uniform data, a partially overlapping tree
// otherwise; Sec. 3.5: a box with more than s particles is subdivided) and
// the size of the interaction list (at most 189 boxes, Sec. 3.4).  This code
// implements these readings:
//   root   bounding cube lo_k = min x_k, W = max_k (max x_k - lo_k) (1 if 0),
//          unless given;
//   keys   g_k = clamp(floor((x_k - lo_k) * (2^D / W)), 0, 2^D - 1) in FP64
//          (subtract, then multiply: no fused operation), interleaved with x
//          in the highest bit of each triple; particles ordered by (key, index);
//   boxes  ordered by (level, Morton code); uniform: every box of levels 0..D;
//          adaptive: split iff count > s and level < D, empty children omitted;
//   lists  Carrier-Greengard-Rokhlin U, V, W, X with "adjacent" = closed cubes
//          touch (integer finest-grid test), each list ascending in box number.
#include "tree_kernels.h"
#include "sort.h"

namespace fmm {

// ---------------- root, keys, sorted particles ----------------
__global__ __launch_bounds__(256) void k_bbox_partial(const double *xyz, int n, double *part)
{
    __shared__ double sh[6][256];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        for (int k = 0; k < 3; ++k) {
            double v = xyz[3 * i + k];
            mn[k] = fmin(mn[k], v);
            mx[k] = fmax(mx[k], v);
        }
    for (int k = 0; k < 3; ++k) { sh[k][threadIdx.x] = mn[k]; sh[3 + k][threadIdx.x] = mx[k]; }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 3; ++k) {
                sh[k][threadIdx.x] = fmin(sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
                sh[3 + k][threadIdx.x] = fmax(sh[3 + k][threadIdx.x], sh[3 + k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_bbox_final(const double *part, int nb, double *root)
{
    if (threadIdx.x != 0) return;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < 3; ++k) {
            mn[k] = fmin(mn[k], part[6 * b + k]);
            mx[k] = fmax(mx[k], part[6 * b + 3 + k]);
        }
    double W = 0.0;
    for (int k = 0; k < 3; ++k) {
        root[k] = mn[k];
        double e = mx[k] - mn[k];
        if (e > W) W = e;
    }
    root[3] = W == 0.0 ? 1.0 : W;
}

void bbox(const double *xyz, int n, double *part, double *root, hipStream_t s)
{
    int nb = (int)ceil_div(n, 256);
    if (nb > kBBoxBlocks) nb = kBBoxBlocks;
    k_bbox_partial<<<nb, 256, 0, s>>>(xyz, n, part);
    k_bbox_final<<<1, 64, 0, s>>>(part, nb, root);
}

__global__ __launch_bounds__(256) void k_keys(const double *xyz, int n, double lo0, double lo1,
                                              double lo2, double scale, int D, uint64_t *keys,
                                              int32_t *idx, int *bad)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double lo[3] = {lo0, lo1, lo2};
    double gmax = (double)((1ll << D) - 1);
    int g[3];
    bool finite = true;
    for (int k = 0; k < 3; ++k) {
        double x = xyz[3 * i + k];
        finite = finite && isfinite(x);
        double t = __dsub_rn(x, lo[k]);
        double f = floor(__dmul_rn(t, scale));
        if (!(f >= 0.0)) f = 0.0;
        if (f > gmax) f = gmax;
        g[k] = (int)f;
    }
    if (!finite) atomicOr(bad, 1);
    keys[i] = interleave(g, D);
    idx[i] = i;
}

void morton_keys(const double *xyz, int n, const double root[4], int D, uint64_t *keys,
                 int32_t *idx, int *bad, hipStream_t s)
{
    double scale = std::ldexp(1.0, D) / root[3];
    k_keys<<<ceil_div(n, 256), 256, 0, s>>>(xyz, n, root[0], root[1], root[2], scale, D, keys, idx, bad);
}

__global__ __launch_bounds__(256) void k_gather_sorted(const double *xyz, const int32_t *perm, int n,
                                                       double *xs, double *ys, double *zs)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int j = perm[i];
    xs[i] = xyz[3 * j];
    ys[i] = xyz[3 * j + 1];
    zs[i] = xyz[3 * j + 2];
}

void gather_sorted(const double *xyz, const int32_t *perm, int n, double *xs, double *ys,
                   double *zs, hipStream_t s)
{
    k_gather_sorted<<<ceil_div(n, 256), 256, 0, s>>>(xyz, perm, n, xs, ys, zs);
}

// ---------------- boxes ----------------
__device__ inline int lower_bound_key(const uint64_t *keys, int lo, int hi, uint64_t v)
{
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Uniform tree: box b of level l has Morton code b - level_begin[l].
__global__ __launch_bounds__(256) void k_uniform_boxes(const uint64_t *keys, int n, int D, int nboxes,
                                                       BoxArrays bx)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nboxes) return;
    int l = 0;
    long long beg = 0, size = 1;
    while (b >= beg + size) { beg += size; size *= 8; ++l; }
    uint64_t m = (uint64_t)(b - beg);
    int sh = 3 * (D - l);
    int f = lower_bound_key(keys, 0, n, m << sh);
    int e = lower_bound_key(keys, f, n, (m + 1) << sh);
    bx.level[b] = l;
    bx.morton[b] = m;
    bx.first[b] = f;
    bx.count[b] = e - f;
    bx.parent[b] = l == 0 ? -1 : (int)((beg - size / 8) + (long long)(m >> 3));
    if (l < D) {
        bx.child_begin[b] = (int)(beg + size + (long long)m * 8);
        bx.nchild[b] = 8;
    } else {
        bx.child_begin[b] = -1;
        bx.nchild[b] = 0;
    }
}

void uniform_boxes(const uint64_t *keys, int n, int D, int nboxes, BoxArrays bx, hipStream_t s)
{
    k_uniform_boxes<<<ceil_div(nboxes, 256), 256, 0, s>>>(keys, n, D, nboxes, bx);
}

__global__ void k_root_box(int n, BoxArrays bx)
{
    bx.level[0] = 0; bx.morton[0] = 0; bx.first[0] = 0; bx.count[0] = n;
    bx.parent[0] = -1; bx.child_begin[0] = -1; bx.nchild[0] = 0;
}

// adaptive: number of non-empty children of each box of [lb, le) that splits
__global__ __launch_bounds__(256) void k_count_children(const uint64_t *keys, int D, int l, int lb,
                                                        int le, int leaf_size, BoxArrays bx,
                                                        int64_t *nch)
{
    int b = lb + blockIdx.x * 256 + threadIdx.x;
    if (b >= le) return;
    int c = 0;
    if (bx.count[b] > leaf_size && l < D) {
        int f = bx.first[b], e = f + bx.count[b];
        int sh = 3 * (D - l - 1);
        uint64_t m = bx.morton[b];
        int s = f;
        for (int o = 0; o < 8; ++o) {
            uint64_t code = m * 8 + (uint64_t)o;
            int t = lower_bound_key(keys, s, e, (code + 1) << sh);
            if (t > s) ++c;
            s = t;
        }
    }
    nch[b - lb] = c;
}

__global__ __launch_bounds__(256) void k_fill_children(const uint64_t *keys, int D, int l, int lb,
                                                       int le, const int64_t *off, BoxArrays bx)
{
    int b = lb + blockIdx.x * 256 + threadIdx.x;
    if (b >= le) return;
    int cnt = (int)(off[b - lb + 1] - off[b - lb]);
    if (cnt == 0) { bx.child_begin[b] = -1; bx.nchild[b] = 0; return; }
    int cb = le + (int)off[b - lb];
    bx.child_begin[b] = cb;
    bx.nchild[b] = cnt;
    int f = bx.first[b], e = f + bx.count[b];
    int sh = 3 * (D - l - 1);
    uint64_t m = bx.morton[b];
    int s = f, k = 0;
    for (int o = 0; o < 8; ++o) {
        uint64_t code = m * 8 + (uint64_t)o;
        int t = lower_bound_key(keys, s, e, (code + 1) << sh);
        if (t > s) {
            int c = cb + k++;
            bx.level[c] = l + 1; bx.morton[c] = code; bx.first[c] = s; bx.count[c] = t - s;
            bx.parent[c] = b; bx.child_begin[c] = -1; bx.nchild[c] = 0;
        }
        s = t;
    }
}

void root_box(int n, BoxArrays bx, hipStream_t s) { k_root_box<<<1, 1, 0, s>>>(n, bx); }

void count_children(const uint64_t *keys, int D, int l, int lb, int le, int leaf_size,
                    BoxArrays bx, int64_t *nch, hipStream_t s)
{
    k_count_children<<<ceil_div(le - lb, 256), 256, 0, s>>>(keys, D, l, lb, le, leaf_size, bx, nch);
}

void fill_children(const uint64_t *keys, int D, int l, int lb, int le, const int64_t *off,
                   BoxArrays bx, hipStream_t s)
{
    k_fill_children<<<ceil_div(le - lb, 256), 256, 0, s>>>(keys, D, l, lb, le, off, bx);
}

// ---------------- lists ----------------
struct TreeView {
    BoxArrays bx;
    const int32_t *lvl_begin; // [kMaxDepth + 2]
    int D, nboxes;
};

__device__ inline int find_box(const TreeView &t, int l, uint64_t code)
{
    int lo = t.lvl_begin[l], hi = t.lvl_begin[l + 1];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (t.bx.morton[mid] < code) lo = mid + 1; else hi = mid;
    }
    return (lo < t.lvl_begin[l + 1] && t.bx.morton[lo] == code) ? lo : -1;
}

__device__ inline bool adjacent(const TreeView &t, int a, int b)
{
    int ca[3], cb[3];
    int la = t.bx.level[a], lb = t.bx.level[b];
    deinterleave(t.bx.morton[a], la, ca);
    deinterleave(t.bx.morton[b], lb, cb);
    long long sa = 1ll << (t.D - la), sb = 1ll << (t.D - lb);
    for (int k = 0; k < 3; ++k) {
        long long xa = ca[k] * sa, xb = cb[k] * sb;
        if (xa > xb + sb || xb > xa + sa) return false;
    }
    return true;
}

__global__ __launch_bounds__(256) void k_colleagues(TreeView t, int32_t *coll)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= t.nboxes) return;
    int l = t.bx.level[b], c[3], nb[3], side = 1 << l, m = 0;
    deinterleave(t.bx.morton[b], l, c);
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                nb[0] = c[0] + dx; nb[1] = c[1] + dy; nb[2] = c[2] + dz;
                int f = -1;
                if (nb[0] >= 0 && nb[1] >= 0 && nb[2] >= 0 && nb[0] < side && nb[1] < side && nb[2] < side)
                    f = find_box(t, l, interleave(nb, l));
                if (f >= 0) { // insert keeping ascending box numbers
                    int j = m++;
                    while (j > 0 && coll[27 * b + j - 1] > f) { coll[27 * b + j] = coll[27 * b + j - 1]; --j; }
                    coll[27 * b + j] = f;
                }
            }
    for (; m < 27; ++m) coll[27 * b + m] = -1;
}

// which: 0 count, 1 fill.  V for boxes of level >= 2: children of the
// parent's colleagues that are not adjacent (same level, so adjacency is
// max |delta| <= 1 in cell coordinates).  Colleagues are sorted and children
// are consecutive, so the list comes out ascending.  The fill pass also
// records each source in the box's M2L slot row (offset slot, Sec. 3.4).
__global__ __launch_bounds__(256) void k_vlist(TreeView t, const int32_t *coll, int which,
                                               int64_t *cnt, const int64_t *off, int32_t *src,
                                               int32_t *vslot)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= t.nboxes) return;
    int n = 0;
    int64_t o = which ? off[b] : 0;
    const int l = t.bx.level[b];
    if (l >= 2) {
        int cb[3], cc[3];
        deinterleave(t.bx.morton[b], l, cb);
        const int oct = (int)(t.bx.morton[b] & 7);
        const int pb = t.bx.parent[b];
        for (int i = 0; i < 27; ++i) {
            int c = coll[27 * pb + i];
            if (c < 0) break;
            deinterleave(t.bx.morton[c], l - 1, cc);
            for (int k = 0; k < t.bx.nchild[c]; ++k) {
                int d = t.bx.child_begin[c] + k;
                int od = (int)(t.bx.morton[d] & 7);
                int dx = 2 * cc[0] + ((od >> 2) & 1) - cb[0];
                int dy = 2 * cc[1] + ((od >> 1) & 1) - cb[1];
                int dz = 2 * cc[2] + (od & 1) - cb[2];
                if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) continue;
                if (which) {
                    src[o + n] = d;
                    int sl = vslot_of(oct, -dx, -dy, -dz); // offset = target - source
                    if (sl >= 0) vslot[(int64_t)b * kVSlots + sl] = d;
                }
                ++n;
            }
        }
    }
    if (!which) cnt[b] = n;
}

// U (P2P) and W (M2P) for leaves, by walking colleagues and their descendants.
constexpr int kStack = 8 * (kMaxDepth + 1) + 8;

__global__ __launch_bounds__(128) void k_uwlist(TreeView t, const int32_t *coll, int which,
                                                int64_t *ucnt, const int64_t *uoff, int32_t *usrc,
                                                int64_t *wcnt, const int64_t *woff, int32_t *wsrc)
{
    int b = blockIdx.x * 128 + threadIdx.x;
    if (b >= t.nboxes) return;
    int nu = 0, nw = 0;
    if (t.bx.nchild[b] == 0) {
        int64_t uo = which ? uoff[b] : 0, wo = which ? woff[b] : 0;
        int stack[kStack];
        for (int i = 0; i < 27; ++i) {
            int c = coll[27 * b + i];
            if (c < 0) break;
            // U: descend through adjacent boxes down to leaves
            int sp = 0;
            stack[sp++] = c;
            while (sp > 0) {
                int x = stack[--sp];
                if (t.bx.nchild[x] == 0) {
                    if (which) usrc[uo + nu] = x;
                    ++nu;
                    continue;
                }
                for (int k = t.bx.nchild[x] - 1; k >= 0; --k) {
                    int d = t.bx.child_begin[x] + k;
                    if (adjacent(t, d, b)) stack[sp++] = d;
                }
            }
            // W: descendants not adjacent whose parent is adjacent
            if (c == b) continue;
            sp = 0;
            if (t.bx.nchild[c] > 0) stack[sp++] = c;
            while (sp > 0) {
                int x = stack[--sp];
                for (int k = t.bx.nchild[x] - 1; k >= 0; --k) {
                    int d = t.bx.child_begin[x] + k;
                    if (!adjacent(t, d, b)) {
                        if (which) wsrc[wo + nw] = d;
                        ++nw;
                    } else if (t.bx.nchild[d] > 0) {
                        stack[sp++] = d;
                    }
                }
            }
        }
        // U, coarser leaves: colleagues of ancestors that are leaves and adjacent
        for (int a = t.bx.parent[b]; a >= 0; a = t.bx.parent[a])
            for (int i = 0; i < 27; ++i) {
                int c = coll[27 * a + i];
                if (c < 0) break;
                if (c != a && t.bx.nchild[c] == 0 && adjacent(t, c, b)) {
                    if (which) usrc[uo + nu] = c;
                    ++nu;
                }
            }
    }
    if (!which) { ucnt[b] = nu; wcnt[b] = nw; }
}

// ascending order inside every CSR segment (insertion sort, segments are short)
__global__ __launch_bounds__(256) void k_sort_segments(const int64_t *off, int nseg, int32_t *v)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nseg) return;
    int64_t s = off[b], e = off[b + 1];
    for (int64_t i = s + 1; i < e; ++i) {
        int32_t x = v[i];
        int64_t j = i - 1;
        while (j >= s && v[j] > x) { v[j + 1] = v[j]; --j; }
        v[j + 1] = x;
    }
}

void colleagues(const TreeArgs &a, int32_t *coll, hipStream_t s)
{
    TreeView t{a.bx, a.lvl_begin, a.D, a.nboxes};
    k_colleagues<<<ceil_div(a.nboxes, 256), 256, 0, s>>>(t, coll);
}

void vlist(const TreeArgs &a, const int32_t *coll, int which, int64_t *cnt, const int64_t *off,
           int32_t *src, int32_t *vslot, hipStream_t s)
{
    TreeView t{a.bx, a.lvl_begin, a.D, a.nboxes};
    k_vlist<<<ceil_div(a.nboxes, 256), 256, 0, s>>>(t, coll, which, cnt, off, src, vslot);
}

void uwlist(const TreeArgs &a, const int32_t *coll, int which, int64_t *ucnt, const int64_t *uoff,
            int32_t *usrc, int64_t *wcnt, const int64_t *woff, int32_t *wsrc, hipStream_t s)
{
    TreeView t{a.bx, a.lvl_begin, a.D, a.nboxes};
    k_uwlist<<<ceil_div(a.nboxes, 128), 128, 0, s>>>(t, coll, which, ucnt, uoff, usrc, wcnt, woff, wsrc);
}

void sort_segments(const int64_t *off, int nseg, int32_t *v, hipStream_t s)
{
    k_sort_segments<<<ceil_div(nseg, 256), 256, 0, s>>>(off, nseg, v);
}

// X = transpose of W: pairs (key = source box, value = target box), stably
// sorted by source; targets arrive in ascending order.
__global__ __launch_bounds__(256) void k_w_pairs(const int64_t *woff, const int32_t *wsrc, int nboxes,
                                                 uint64_t *key, int32_t *val, int64_t *xcnt)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nboxes) return;
    for (int64_t e = woff[b]; e < woff[b + 1]; ++e) {
        key[e] = (uint64_t)wsrc[e];
        val[e] = b;
        atomicAdd((unsigned long long *)&xcnt[wsrc[e]], 1ull);
    }
}

void w_pairs(const int64_t *woff, const int32_t *wsrc, int nboxes, uint64_t *key, int32_t *val,
             int64_t *xcnt, hipStream_t s)
{
    k_w_pairs<<<ceil_div(nboxes, 256), 256, 0, s>>>(woff, wsrc, nboxes, key, val, xcnt);
}

// ---------------- work lists ----------------
// flag[b] = predicate; compaction via exclusive scan of the flags
__global__ __launch_bounds__(256) void k_flags(const BoxArrays bx, int nboxes, int what,
                                               const int64_t *off, int64_t *flag)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nboxes) return;
    int64_t f = 0;
    if (what == 0) f = bx.nchild[b] == 0;               // leaves
    else if (what == 1) f = bx.nchild[b] > 0;           // non-leaves
    else f = off[b + 1] > off[b];                       // non-empty list
    flag[b] = f;
}

__global__ __launch_bounds__(256) void k_compact(const int64_t *flag, const int64_t *pos, int nboxes,
                                                 int32_t *out)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nboxes) return;
    if (flag[b]) out[pos[b]] = b;
}

void flags(const BoxArrays &bx, int nboxes, int what, const int64_t *off, int64_t *flag, hipStream_t s)
{
    k_flags<<<ceil_div(nboxes, 256), 256, 0, s>>>(bx, nboxes, what, off, flag);
}

void compact(const int64_t *flag, const int64_t *pos, int nboxes, int32_t *out, hipStream_t s)
{
    k_compact<<<ceil_div(nboxes, 256), 256, 0, s>>>(flag, pos, nboxes, out);
}

// leaf of every sorted particle
__global__ __launch_bounds__(256) void k_leaf_of(const BoxArrays bx, const int32_t *leaves, int nleaves,
                                                 int32_t *leaf_of)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nleaves) return;
    int b = leaves[i];
    for (int k = bx.first[b]; k < bx.first[b] + bx.count[b]; ++k) leaf_of[k] = b;
}

void leaf_of(const BoxArrays &bx, const int32_t *leaves, int nleaves, int32_t *lo, hipStream_t s)
{
    k_leaf_of<<<ceil_div(nleaves, 256), 256, 0, s>>>(bx, leaves, nleaves, lo);
}

// ---------------- M2L target tiles ----------------
// Targets (boxes with a V list, ascending) are stably sorted by octant, then
// each octant group is placed at a multiple of 64 so that the 64 targets of
// one M2L block share one set of 189 offsets.
__global__ __launch_bounds__(256) void k_oct_keys(const BoxArrays bx, const int32_t *tg, int nt,
                                                  uint64_t *key, int32_t *val)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nt) return;
    key[i] = bx.morton[tg[i]] & 7;
    val[i] = tg[i];
}

// start of every octant in the sorted keys, and the padded output offsets
__global__ void k_oct_offsets(const uint64_t *key, int nt, int *octoff)
{
    __shared__ int st[9];
    int o = threadIdx.x;
    if (o <= 8) {
        int lo = 0, hi = nt;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (key[mid] < (uint64_t)o) lo = mid + 1; else hi = mid;
        }
        st[o] = o == 8 ? nt : lo;
    }
    __syncthreads();
    if (o == 0) {
        int s = 0;
        for (int k = 0; k < 8; ++k) {
            octoff[k] = s;              // padded start
            octoff[9 + k] = st[k];      // unpadded start
            s += (st[k + 1] - st[k] + 63) & ~63;
        }
        octoff[8] = s;
        octoff[17] = nt;
    }
}

__global__ __launch_bounds__(256) void k_oct_place(const uint64_t *key, const int32_t *val, int nt,
                                                   const int *octoff, int32_t *slots)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nt) return;
    int o = (int)key[i];
    slots[octoff[o] + (i - octoff[9 + o])] = val[i];
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n > 0) k_fill_i32<<<ceil_div(n, 256), 256, 0, s>>>(p, n, v);
}

void m2l_tiles(const BoxArrays &bx, const int32_t *tg, int nt, uint64_t *key, int32_t *val,
               uint64_t *tk, int32_t *tv, int32_t *sort_scratch, int *octoff, int32_t *slots,
               int64_t slot_cap, hipStream_t s)
{
    fill_i32(slots, slot_cap, -1, s);
    if (nt == 0) return;
    k_oct_keys<<<ceil_div(nt, 256), 256, 0, s>>>(bx, tg, nt, key, val);
    radix_sort_pairs(key, val, tk, tv, nt, 3, sort_scratch, s);
    k_oct_offsets<<<1, 64, 0, s>>>(key, nt, octoff);
    k_oct_place<<<ceil_div(nt, 256), 256, 0, s>>>(key, val, nt, octoff, slots);
}

// ---------------- mixed precision particle data ----------------
// leaf-local offsets x - c_leaf split into an FP32 head and an FP32 tail
__global__ __launch_bounds__(256) void k_local_split(const double *xs, const double *ys, const double *zs,
                                                     const int32_t *leaf_of, const BoxArrays bx, int n,
                                                     double lo0, double lo1, double lo2, double W,
                                                     float *ux, float *uy, float *uz, float *vx,
                                                     float *vy, float *vz)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int b = leaf_of[i];
    int l = bx.level[b], c[3];
    deinterleave(bx.morton[b], l, c);
    double h = W / (double)(1ll << l);
    double lo[3] = {lo0, lo1, lo2}, x[3] = {xs[i], ys[i], zs[i]};
    float hi[3], lw[3];
    for (int k = 0; k < 3; ++k) {
        double cen = lo[k] + ((double)c[k] + 0.5) * h;
        double d = x[k] - cen;
        hi[k] = (float)d;
        lw[k] = (float)(d - (double)hi[k]);
    }
    ux[i] = hi[0]; uy[i] = hi[1]; uz[i] = hi[2];
    vx[i] = lw[0]; vy[i] = lw[1]; vz[i] = lw[2];
}

void local_split(const double *xs, const double *ys, const double *zs, const int32_t *leaf_of,
                 const BoxArrays &bx, int n, const double root[4], float *ux, float *uy, float *uz,
                 float *vx, float *vy, float *vz, hipStream_t s)
{
    k_local_split<<<ceil_div(n, 256), 256, 0, s>>>(xs, ys, zs, leaf_of, bx, n, root[0], root[1], root[2],
                                                  root[3], ux, uy, uz, vx, vy, vz);
}

} // namespace fmm
