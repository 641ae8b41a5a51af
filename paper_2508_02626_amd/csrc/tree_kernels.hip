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
            double v = xyz[3 * (int64_t)i + k];
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

__global__ __launch_bounds__(64) void k_bbox_final(const double *part, int nb, double *root)
{
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += 64)
        for (int k = 0; k < 3; ++k) {
            mn[k] = fmin(mn[k], part[6 * b + k]);
            mx[k] = fmax(mx[k], part[6 * b + 3 + k]);
        }
    for (int o = 32; o > 0; o >>= 1)
        for (int k = 0; k < 3; ++k) {
            mn[k] = fmin(mn[k], __shfl_xor(mn[k], o));
            mx[k] = fmax(mx[k], __shfl_xor(mx[k], o));
        }
    if (threadIdx.x != 0) return;
    double W = 0.0;
    for (int k = 0; k < 3; ++k) {
        root[k] = mn[k];
        double e = mx[k] - mn[k];
        if (e > W) W = e;
    }
    root[3] = W == 0.0 ? 1.0 : W;
}

// clears the non-finite flag and, when the root cube is given, stores it
__global__ void k_plan_init(int given, double r0, double r1, double r2, double r3, double *root, int *bad)
{
    if (threadIdx.x != 0) return;
    *bad = 0;
    if (given) { root[0] = r0; root[1] = r1; root[2] = r2; root[3] = r3; }
}

void plan_init(const double *given_root, double *root_dev, int *bad, hipStream_t s)
{
    if (given_root)
        k_plan_init<<<1, 64, 0, s>>>(1, given_root[0], given_root[1], given_root[2], given_root[3], root_dev, bad);
    else
        k_plan_init<<<1, 64, 0, s>>>(0, 0, 0, 0, 0, root_dev, bad);
}

void bbox(const double *xyz, int n, double *part, double *root, hipStream_t s)
{
    int nb = (int)ceil_div(n, 256);
    if (nb > kBBoxBlocks) nb = kBBoxBlocks;
    k_bbox_partial<<<nb, 256, 0, s>>>(xyz, n, part);
    k_bbox_final<<<1, 64, 0, s>>>(part, nb, root);
}

__global__ __launch_bounds__(256) void k_keys(const double *xyz, int n, const double *root, int D,
                                              uint64_t *keys, int32_t *idx, int *bad)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {root[0], root[1], root[2]};
    const double scale = (double)(1ll << D) / root[3]; // correctly rounded, as on the host
    double gmax = (double)((1ll << D) - 1);
    int g[3];
    bool finite = true;
    for (int k = 0; k < 3; ++k) {
        double x = xyz[3 * (int64_t)i + k];
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

void morton_keys(const double *xyz, int n, const double *root_dev, int D, uint64_t *keys,
                 int32_t *idx, int *bad, hipStream_t s)
{
    k_keys<<<ceil_div(n, 256), 256, 0, s>>>(xyz, n, root_dev, D, keys, idx, bad);
}

__global__ __launch_bounds__(256) void k_gather_sorted(const double *xyz, const int32_t *perm, int n,
                                                       double *xs, double *ys, double *zs)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int j = perm[i];
    xs[i] = xyz[3 * (int64_t)j];
    ys[i] = xyz[3 * (int64_t)j + 1];
    zs[i] = xyz[3 * (int64_t)j + 2];
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
                                                       BoxArrays bx, int32_t *lvl_begin)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b == 0) { // level starts: 0, 1, 9, 73, ... then nboxes
        long long beg = 0, size = 1;
        for (int l = 0; l <= kMaxDepth + 1; ++l) {
            lvl_begin[l] = l <= D ? (int)beg : nboxes;
            beg += size;
            size *= 8;
            if (beg > nboxes) beg = nboxes;
        }
    }
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

void uniform_boxes(const uint64_t *keys, int n, int D, int nboxes, BoxArrays bx, int32_t *lvl_begin,
                   hipStream_t s)
{
    k_uniform_boxes<<<ceil_div(nboxes, 256), 256, 0, s>>>(keys, n, D, nboxes, bx, lvl_begin);
}

// Adaptive tree straight from the sorted keys, with no host round trip per
// level.  The boxes of level l are the runs of equal level-l key prefixes
// inside boxes of level l-1 that split; a box of level l exists iff the run
// of level l-1 around it holds more than s particles (counts only shrink
// down the tree, so this also covers every older ancestor).  Particle i
// starts a run at every level from first_new_level(i) down, so it emits the
// boxes of those levels whose parent run exceeds s, down to the first run
// that holds at most s particles (or level D).
__device__ inline int first_new_level(uint64_t prev, uint64_t cur, int D)
{
    uint64_t x = prev ^ cur;
    if (x == 0) return D + 1;
    return D - (63 - __clzll((long long)x)) / 3;
}

// true iff the level-l run containing particle i holds more than s particles
// (both searches are clamped to s elements on either side of i)
__device__ inline bool run_exceeds(const uint64_t *keys, int n, int i, int l, int D, int s)
{
    const int sh = 3 * (D - l);
    const uint64_t pre = keys[i] >> sh;
    int a = lower_bound_key(keys, i - s > 0 ? i - s : 0, i, pre << sh);
    int b = lower_bound_key(keys, i + 1, i + s + 1 < n ? i + s + 1 : n, (pre + 1) << sh);
    return b - a > s;
}

template <bool FILL>
__device__ int emit_boxes(const uint64_t *keys, int n, int D, int s, int i, int64_t pos,
                          uint64_t *elevel, int32_t *eidx, int32_t *efirst, int32_t *ecount,
                          uint64_t *emorton)
{
    int l = i == 0 ? 0 : first_new_level(keys[i - 1], keys[i], D);
    if (l > D) return 0;
    if (l > 0 && !run_exceeds(keys, n, i, l - 1, D, s)) return 0;
    int cnt = 0, hi = n;
    for (;; ++l) {
        const int sh = 3 * (D - l);
        const uint64_t pre = keys[i] >> sh, lim = (pre + 1) << sh;
        const int w = i + s + 1 < hi ? i + s + 1 : hi;
        int e = lower_bound_key(keys, i + 1, w, lim);
        if (e == w && w < hi) e = lower_bound_key(keys, w, hi, lim);
        if (FILL) {
            int64_t k = pos + cnt;
            elevel[k] = (uint64_t)l;
            eidx[k] = (int32_t)k;
            efirst[k] = i;
            ecount[k] = e - i;
            emorton[k] = pre;
        }
        ++cnt;
        if (e - i <= s || l == D) break;
        hi = e;
    }
    return cnt;
}

__global__ __launch_bounds__(256) void k_emit_count(const uint64_t *keys, int n, int D, int s, int64_t *cnt)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    cnt[i] = emit_boxes<false>(keys, n, D, s, i, 0, nullptr, nullptr, nullptr, nullptr, nullptr);
}

__global__ __launch_bounds__(256) void k_emit_fill(const uint64_t *keys, int n, int D, int s,
                                                   const int64_t *off, uint64_t *elevel, int32_t *eidx,
                                                   int32_t *efirst, int32_t *ecount, uint64_t *emorton)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    emit_boxes<true>(keys, n, D, s, i, off[i], elevel, eidx, efirst, ecount, emorton);
}

// boxes in (level, Morton) order: the emitted boxes stably sorted by level
// (within a level they were emitted in particle order, i.e. Morton order)
__global__ __launch_bounds__(256) void k_box_place(const uint64_t *elevel, const int32_t *eidx, int nb,
                                                   const int32_t *efirst, const int32_t *ecount,
                                                   const uint64_t *emorton, BoxArrays bx)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    int e = eidx[b];
    bx.level[b] = (int32_t)elevel[b];
    bx.first[b] = efirst[e];
    bx.count[b] = ecount[e];
    bx.morton[b] = emorton[e];
}

// lvl_begin[l] = first box of level l (nb for levels below the deepest)
__global__ __launch_bounds__(256) void k_level_bounds(const int32_t *level, int nb, int32_t *lvl_begin)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    int l = level[b];
    int from = b == 0 ? 0 : level[b - 1] + 1;
    for (int k = from; k <= l; ++k) lvl_begin[k] = b;
    if (b == nb - 1)
        for (int k = l + 1; k <= kMaxDepth + 1; ++k) lvl_begin[k] = nb;
}

__device__ inline int lower_bound_first(const int32_t *first, int lo, int hi, int v)
{
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (first[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// parent: the box of the level above whose particle range contains this
// box's first particle; children: the boxes of the level below that start
// inside this box's range (contiguous)
__global__ __launch_bounds__(256) void k_box_links(BoxArrays bx, int nb, const int32_t *lvl_begin)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    const int l = bx.level[b], f = bx.first[b], c = bx.count[b];
    if (l == 0) {
        bx.parent[b] = -1;
    } else {
        int lo = lvl_begin[l - 1], hi = lvl_begin[l];
        bx.parent[b] = lower_bound_first(bx.first, lo, hi, f + 1) - 1;
    }
    int c0 = 0, c1 = 0;
    if (l < kMaxDepth) {
        int lo = lvl_begin[l + 1], hi = lvl_begin[l + 2];
        c0 = lower_bound_first(bx.first, lo, hi, f);
        c1 = lower_bound_first(bx.first, c0, hi, f + c);
    }
    bx.child_begin[b] = c1 > c0 ? c0 : -1;
    bx.nchild[b] = c1 - c0;
}

void emit_count(const uint64_t *keys, int n, int D, int leaf_size, int64_t *cnt, hipStream_t s)
{
    k_emit_count<<<ceil_div(n, 256), 256, 0, s>>>(keys, n, D, leaf_size, cnt);
}

void adaptive_boxes(const uint64_t *keys, int n, int D, int leaf_size, const int64_t *off, int nb,
                    uint64_t *elevel, int32_t *eidx, uint64_t *tk, int32_t *tv, int32_t *efirst,
                    int32_t *ecount, uint64_t *emorton, int32_t *sort_scratch, BoxArrays bx,
                    int32_t *lvl_begin, hipStream_t s)
{
    k_emit_fill<<<ceil_div(n, 256), 256, 0, s>>>(keys, n, D, leaf_size, off, elevel, eidx, efirst, ecount,
                                                 emorton);
    radix_sort_pairs(elevel, eidx, tk, tv, nb, 5, sort_scratch, s);
    k_box_place<<<ceil_div(nb, 256), 256, 0, s>>>(elevel, eidx, nb, efirst, ecount, emorton, bx);
    k_level_bounds<<<ceil_div(nb, 256), 256, 0, s>>>(bx.level, nb, lvl_begin);
    k_box_links<<<ceil_div(nb, 256), 256, 0, s>>>(bx, nb, lvl_begin);
}

// ---------------- lists ----------------
struct TreeView {
    BoxArrays bx;
    const int32_t *lvl_begin; // [kMaxDepth + 2]
    int D, nboxes;
    int uniform; // every level full: all leaves on the last level
    const int32_t *leafcol; // per box: a colleague (other than itself) is a leaf, or NULL
};

__device__ inline int find_box(const TreeView &t, int l, uint64_t code)
{
    int lo = t.lvl_begin[l], hi = t.lvl_begin[l + 1];
    // a level that holds all 8^l cells (every level of a uniform tree) is
    // sorted by code with no gaps: the box is the level's start plus the code
    if (l <= 10 && hi - lo == (1 << (3 * l))) return lo + (int)code;
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

// The list kernels give one wavefront to each box (four boxes per block).

// Colleagues: the up to 27 same-level boxes adjacent to b (b included),
// ascending, padded with -1.  Lane j < 27 looks up neighbour cell j.
__global__ __launch_bounds__(256) void k_colleagues(TreeView t, int32_t *coll, int64_t *zero, int32_t *leafcol)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= t.nboxes) return;
    if (zero && lane == 0) zero[b] = 0; // counters the later list passes accumulate into
    const int l = t.bx.level[b], side = 1 << l;
    int c[3];
    deinterleave(t.bx.morton[b], l, c);
    int f = INT_MAX;
    if (lane < 27) {
        int nb[3] = {c[0] + lane / 9 - 1, c[1] + (lane / 3) % 3 - 1, c[2] + lane % 3 - 1};
        if (nb[0] >= 0 && nb[1] >= 0 && nb[2] >= 0 && nb[0] < side && nb[1] < side && nb[2] < side) {
            int g = find_box(t, l, interleave(nb, l));
            if (g >= 0) f = g;
        }
    }
    int rank = 0;
    for (int k = 0; k < 27; ++k) rank += __shfl(f, k) < f;
    const int found = __popcll(__ballot(f != INT_MAX));
    if (f != INT_MAX) coll[27 * b + rank] = f;    // ranks fill [0, found)
    if (lane >= found && lane < 27) coll[27 * b + lane] = -1;
    if (leafcol) { // does the U/W walk of a descendant leaf need this box's colleagues?
        const bool lf = f != INT_MAX && f != b && t.bx.nchild[f] == 0;
        const uint64_t m = __ballot(lf);
        if (lane == 0) leafcol[b] = m != 0;
    }
}

// which: 0 count, 1 fill.  V for boxes of level >= 2: children of the
// parent's colleagues that are not adjacent (same level, so adjacency is
// max |delta| <= 1 in cell coordinates).  Lane j of a round looks at child
// j % 8 of colleague j / 8; colleagues are ascending and children
// consecutive, so compaction in lane order gives an ascending list.  Either
// pass records each source in the box's M2L slot row (Sec. 3.4) if given one.
__global__ __launch_bounds__(256) void k_vlist(TreeView t, const int32_t *coll, int which,
                                               int64_t *cnt, const int64_t *off, int32_t *src,
                                               int32_t *vslot)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= t.nboxes) return;
    int n = 0;
    const int l = t.bx.level[b];
    if (l >= 2) {
        const int64_t o = which ? off[b] : 0;
        int cb[3];
        deinterleave(t.bx.morton[b], l, cb);
        const int oct = (int)(t.bx.morton[b] & 7);
        const int pb = t.bx.parent[b];
        // the four rounds' loads are issued together, one dependent level at
        // a time (colleague, its children, their codes)
        constexpr int R = (27 * 8 + 63) / 64;
        int cc[R], ch[R], nc[R];
        uint64_t md[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = (64 * r + lane) >> 3;
            cc[r] = coll[27 * pb + (i < 27 ? i : 26)];
            if (i >= 27) cc[r] = -1;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int c = cc[r] >= 0 ? cc[r] : 0;
            nc[r] = t.bx.nchild[c];
            ch[r] = t.bx.child_begin[c];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = (64 * r + lane) & 7;
            ch[r] = (cc[r] >= 0 && k < nc[r]) ? ch[r] + k : -1;
            md[r] = t.bx.morton[ch[r] >= 0 ? ch[r] : 0];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bool sel = false;
            const int d = ch[r];
            int dx = 0, dy = 0, dz = 0;
            if (d >= 0) {
                int cd[3];
                deinterleave(md[r], l, cd);
                dx = cd[0] - cb[0]; dy = cd[1] - cb[1]; dz = cd[2] - cb[2];
                sel = dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1;
            }
            const uint64_t m = __ballot(sel);
            if (sel && which) src[o + n + __popcll(m & lanes_below(lane))] = d;
            if (sel && vslot) {
                int sl = vslot_of(oct, -dx, -dy, -dz); // offset = target - source
                if (sl >= 0) vslot[(int64_t)b * kVSlots + sl] = d;
            }
            n += __popcll(m);
        }
    }
    if (!which && lane == 0) cnt[b] = n;
}

// Uniform trees: V counts and M2L slot rows without the colleague walk.  In a
// full level the V source at slot offset k (target - source) is the box of
// cell (target cell - k) whenever that cell lies in the grid; every row is
// written whole (-1 where there is no source, all of it below level 2).
__global__ __launch_bounds__(256) void k_vslot_uniform(TreeView t, int64_t *cnt, int32_t *vslot)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= t.nboxes) return;
    const int l = t.bx.level[b];
    int32_t *row = vslot + (int64_t)b * kVSlots;
    int n = 0;
    if (l < 2) {
        for (int j = lane; j < kVSlots; j += 64) row[j] = -1;
    } else {
        const int side = 1 << l, base = t.lvl_begin[l];
        const uint64_t code = t.bx.morton[b];
        int cb[3];
        deinterleave(code, l, cb);
        const int oct = (int)(code & 7);
        const int s[3] = {((oct >> 2) & 1) ? -2 : -3, ((oct >> 1) & 1) ? -2 : -3, (oct & 1) ? -2 : -3};
        for (int j = lane; j < 216; j += 64) { // the 6 x 6 x 6 block of offsets, near cube excluded
            const int k[3] = {j / 36 + s[0], (j / 6) % 6 + s[1], j % 6 + s[2]};
            const int sl = vslot_of(oct, k[0], k[1], k[2]);
            if (sl < 0) continue;
            int c[3] = {cb[0] - k[0], cb[1] - k[1], cb[2] - k[2]};
            const bool in = c[0] >= 0 && c[1] >= 0 && c[2] >= 0 && c[0] < side && c[1] < side && c[2] < side;
            row[sl] = in ? base + (int)interleave(c, l) : -1;
            n += in;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) n += __shfl_xor(n, o);
    }
    if (lane == 0) cnt[b] = n;
}

// Uniform trees: U lists without the colleague walk.  A leaf's U list is the
// leaves of its 3 x 3 x 3 cell neighbourhood (itself included), in box order;
// W and X lists are empty.  Counts: one thread per box; fill: one wavefront
// per leaf, the neighbours ranked by box index.
__global__ __launch_bounds__(256) void k_ucount_uniform(TreeView t, int64_t *ucnt, int64_t *wcnt, int64_t *xcnt)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= t.nboxes) return;
    const int l = t.bx.level[b];
    int n = 0;
    if (l == t.D) {
        const int side = 1 << l;
        int c[3];
        deinterleave(t.bx.morton[b], l, c);
        n = 1;
        for (int k = 0; k < 3; ++k) n *= (c[k] + 1 < side - 1 ? c[k] + 1 : side - 1) - (c[k] > 0 ? c[k] - 1 : 0) + 1;
    }
    ucnt[b] = n;
    wcnt[b] = 0;
    xcnt[b] = 0;
}

__global__ __launch_bounds__(256) void k_ufill_uniform(TreeView t, const int64_t *uoff, int32_t *usrc)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= t.nboxes) return;
    const int l = t.bx.level[b];
    if (l != t.D) return;
    const int side = 1 << l, base = t.lvl_begin[l];
    int c[3];
    deinterleave(t.bx.morton[b], l, c);
    int f = INT_MAX;
    if (lane < 27) {
        int nb[3] = {c[0] + lane / 9 - 1, c[1] + (lane / 3) % 3 - 1, c[2] + lane % 3 - 1};
        if (nb[0] >= 0 && nb[1] >= 0 && nb[2] >= 0 && nb[0] < side && nb[1] < side && nb[2] < side)
            f = base + (int)interleave(nb, l);
    }
    int rank = 0;
    for (int k = 0; k < 27; ++k) rank += __shfl(f, k) < f;
    if (f != INT_MAX) usrc[uoff[b] + rank] = f;
}

// U (P2P) and W (M2P) for leaves.  U(b): the leaves adjacent to b (b
// included); W(b): boxes not adjacent to b whose parent is adjacent to b and
// that descend from a colleague of b.  A wavefront walks the adjacent
// descendants of b's colleagues breadth-first through an LDS stack (64
// entries per step), then adds the coarser adjacent leaves (colleagues of
// b's ancestors); both lists are collected in LDS and written ascending.  A
// walk that would overflow the LDS buffers is redone by one lane with a
// private depth-first stack.  The count pass also counts the X lists
// (X = transpose of W).
constexpr int kUWStack = 512, kUWBuf = 512;
constexpr int kSerialStack = 8 * (kMaxDepth + 1) + 8;

struct Cell { long long x[3], side; };

__device__ inline Cell cell_of(const TreeView &t, int a)
{
    Cell c;
    int ca[3], la = t.bx.level[a];
    deinterleave(t.bx.morton[a], la, ca);
    c.side = 1ll << (t.D - la);
    for (int k = 0; k < 3; ++k) c.x[k] = ca[k] * c.side;
    return c;
}

__device__ inline bool touches(const Cell &a, const Cell &b)
{
    for (int k = 0; k < 3; ++k)
        if (a.x[k] > b.x[k] + b.side || b.x[k] > a.x[k] + a.side) return false;
    return true;
}

__device__ inline void sort_serial(int32_t *v, int64_t m)
{
    for (int64_t i = 1; i < m; ++i) {
        int32_t x = v[i];
        int64_t j = i - 1;
        while (j >= 0 && v[j] > x) { v[j + 1] = v[j]; --j; }
        v[j + 1] = x;
    }
}

// one lane: depth-first walk writing straight to the lists, then sorting them
__device__ void uw_serial(const TreeView &t, const int32_t *coll, int b, int which, int32_t *usrc,
                          int32_t *wsrc, int64_t *xcnt, int &nu_out, int &nw_out)
{
    const Cell cb = cell_of(t, b);
    int stack[kSerialStack];
    int nu = 0, nw = 0;
    for (int i = 0; i < 27; ++i) {
        int c = coll[27 * b + i];
        if (c < 0) break;
        int sp = 0;
        stack[sp++] = c;
        while (sp > 0) {
            int x = stack[--sp];
            const int nch = t.bx.nchild[x];
            if (nch == 0) {
                if (which) usrc[nu] = x;
                ++nu;
                continue;
            }
            for (int k = nch - 1; k >= 0; --k) {
                int d = t.bx.child_begin[x] + k;
                if (touches(cell_of(t, d), cb)) {
                    stack[sp++] = d;
                } else {
                    if (which) wsrc[nw] = d;
                    else atomicAdd((unsigned long long *)&xcnt[d], 1ull);
                    ++nw;
                }
            }
        }
    }
    for (int a = t.bx.parent[b]; a >= 0; a = t.bx.parent[a])
        for (int i = 0; i < 27; ++i) {
            int c = coll[27 * a + i];
            if (c < 0) break;
            if (c != a && t.bx.nchild[c] == 0 && touches(cell_of(t, c), cb)) {
                if (which) usrc[nu] = c;
                ++nu;
            }
        }
    if (which) { sort_serial(usrc, nu); sort_serial(wsrc, nw); }
    nu_out = nu;
    nw_out = nw;
}

// ascending copy of buf[0..m) (distinct values) to out, by ranks
__device__ inline void write_ranked(const int32_t *buf, int m, int32_t *out, int lane)
{
    for (int j = lane; j < m; j += 64) {
        int v = buf[j], r = 0;
        for (int k = 0; k < m; ++k) r += buf[k] < v;
        out[r] = v;
    }
}

__global__ __launch_bounds__(256) void k_uwlist(TreeView t, const int32_t *coll, int which,
                                                int64_t *ucnt, const int64_t *uoff, int32_t *usrc,
                                                int64_t *wcnt, const int64_t *woff, int32_t *wsrc,
                                                int64_t *xcnt)
{
    __shared__ int32_t sstk[4][kUWStack];
    __shared__ int32_t sbu[4][kUWBuf];
    __shared__ int32_t sbw[4][kUWBuf];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = blockIdx.x * 4 + wv;
    if (b >= t.nboxes) return;
    if (t.bx.nchild[b] != 0) {
        if (!which && lane == 0) { ucnt[b] = 0; wcnt[b] = 0; }
        return;
    }
    int32_t *stk = sstk[wv], *bu = sbu[wv], *bw = sbw[wv];
    const uint64_t below = lanes_below(lane);
    const Cell cb = cell_of(t, b);
    int nu = 0, nw = 0;
    bool ok = true;
    {
        int c = lane < 27 ? coll[27 * b + lane] : -1;
        uint64_t m = __ballot(c >= 0);
        if (c >= 0) stk[__popcll(m & below)] = c;
        int sp = __popcll(m);
        wave_sync();
        while (sp > 0) {
            // pop as many as fit: the stack grows by at most 7 per popped box,
            // each popped box adds at most 1 U and 8 W entries
            int take = sp < 64 ? sp : 64;
            take = min(take, (kUWStack - sp) / 7);
            take = min(take, kUWBuf - nu);
            take = min(take, (kUWBuf - nw) / 8);
            if (take <= 0) {
                ok = false;
                break;
            }
            const int x = lane < take ? stk[sp - take + lane] : -1;
            sp -= take;
            wave_sync();
            const int nch = x >= 0 ? t.bx.nchild[x] : 0;
            const bool isu = x >= 0 && nch == 0;
            uint64_t mu = __ballot(isu);
            if (isu) bu[nu + __popcll(mu & below)] = x;
            nu += __popcll(mu);
            const int cfirst = nch > 0 ? t.bx.child_begin[x] : 0;
            for (int k = 0; k < 8; ++k) {
                const bool has = k < nch;
                const int d = cfirst + k;
                const bool adj = has && touches(cell_of(t, d), cb);
                const bool isw = has && !adj;
                const uint64_t mp = __ballot(adj), mw = __ballot(isw);
                if (adj) stk[sp + __popcll(mp & below)] = d;
                if (isw) bw[nw + __popcll(mw & below)] = d;
                sp += __popcll(mp);
                nw += __popcll(mw);
            }
            wave_sync();
        }
    }
    if (ok && !t.uniform) { // (a uniform tree has all its leaves on one level)
        for (int a = t.bx.parent[b]; a >= 0; a = t.bx.parent[a]) {
            if (t.leafcol && !t.leafcol[a]) continue; // no leaf among a's colleagues
            const int c = lane < 27 ? coll[27 * a + lane] : -1;
            const bool hit = c >= 0 && c != a && t.bx.nchild[c] == 0 && touches(cell_of(t, c), cb);
            const uint64_t m = __ballot(hit);
            if (nu + __popcll(m) > kUWBuf) { ok = false; break; }
            if (hit) bu[nu + __popcll(m & below)] = c;
            nu += __popcll(m);
        }
    }
    wave_sync();
    if (!ok) {
        int su = 0, sw = 0;
        if (lane == 0)
            uw_serial(t, coll, b, which, which ? usrc + uoff[b] : nullptr, which ? wsrc + woff[b] : nullptr,
                      xcnt, su, sw);
        if (!which && lane == 0) { ucnt[b] = su; wcnt[b] = sw; }
        return;
    }
    if (!which) {
        for (int j = lane; j < nw; j += 64) atomicAdd((unsigned long long *)&xcnt[bw[j]], 1ull);
        if (lane == 0) { ucnt[b] = nu; wcnt[b] = nw; }
        return;
    }
    write_ranked(bu, nu, usrc + uoff[b], lane);
    write_ranked(bw, nw, wsrc + woff[b], lane);
}

void colleagues(const TreeArgs &a, int32_t *coll, int64_t *zero, int32_t *leafcol, hipStream_t s)
{
    TreeView t{a.bx, a.lvl_begin, a.D, a.nboxes, a.uniform, a.leafcol};
    k_colleagues<<<ceil_div(a.nboxes, 4), 256, 0, s>>>(t, coll, zero, leafcol);
}

void vlist(const TreeArgs &a, const int32_t *coll, int which, int64_t *cnt, const int64_t *off,
           int32_t *src, int32_t *vslot, hipStream_t s)
{
    TreeView t{a.bx, a.lvl_begin, a.D, a.nboxes, a.uniform, a.leafcol};
    k_vlist<<<ceil_div(a.nboxes, 4), 256, 0, s>>>(t, coll, which, cnt, off, src, vslot);
}

void ulist_uniform(const TreeArgs &a, int which, int64_t *ucnt, int64_t *wcnt, int64_t *xcnt, const int64_t *uoff,
                   int32_t *usrc, hipStream_t s)
{
    TreeView t{a.bx, a.lvl_begin, a.D, a.nboxes, a.uniform, a.leafcol};
    if (!which) k_ucount_uniform<<<ceil_div(a.nboxes, 256), 256, 0, s>>>(t, ucnt, wcnt, xcnt);
    else k_ufill_uniform<<<ceil_div(a.nboxes, 4), 256, 0, s>>>(t, uoff, usrc);
}

void vslot_uniform(const TreeArgs &a, int64_t *cnt, int32_t *vslot, hipStream_t s)
{
    TreeView t{a.bx, a.lvl_begin, a.D, a.nboxes, a.uniform, a.leafcol};
    k_vslot_uniform<<<ceil_div(a.nboxes, 4), 256, 0, s>>>(t, cnt, vslot);
}

void uwlist(const TreeArgs &a, const int32_t *coll, int which, int64_t *ucnt, const int64_t *uoff,
            int32_t *usrc, int64_t *wcnt, const int64_t *woff, int32_t *wsrc, int64_t *xcnt, hipStream_t s)
{
    TreeView t{a.bx, a.lvl_begin, a.D, a.nboxes, a.uniform, a.leafcol};
    k_uwlist<<<ceil_div(a.nboxes, 4), 256, 0, s>>>(t, coll, which, ucnt, uoff, usrc, wcnt, woff, wsrc, xcnt);
}

// X = transpose of W: pairs (key = source box, value = target box), stably
// sorted by source; targets arrive in ascending order.
__global__ __launch_bounds__(256) void k_w_pairs(const int64_t *woff, const int32_t *wsrc, int nboxes,
                                                 uint64_t *key, int32_t *val)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nboxes) return;
    for (int64_t e = woff[b]; e < woff[b + 1]; ++e) {
        key[e] = (uint64_t)wsrc[e];
        val[e] = b;
    }
}

void w_pairs(const int64_t *woff, const int32_t *wsrc, int nboxes, uint64_t *key, int32_t *val, hipStream_t s)
{
    k_w_pairs<<<ceil_div(nboxes, 256), 256, 0, s>>>(woff, wsrc, nboxes, key, val);
}

// ---------------- work lists ----------------
// Work-list membership of every box: leaves, non-leaves, boxes with an X
// list, boxes with a V list; compaction via exclusive scans of the flags.
__global__ __launch_bounds__(256) void k_flags(const BoxArrays bx, int nboxes, const int64_t *xcnt,
                                               const int64_t *vcnt, int64_t *fleaf, int64_t *fnon,
                                               int64_t *fx, int64_t *fv)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nboxes) return;
    const bool leaf = bx.nchild[b] == 0;
    fleaf[b] = leaf;
    fnon[b] = !leaf;
    fx[b] = xcnt[b] > 0;
    fv[b] = vcnt[b] > 0;
}

void flags(const BoxArrays &bx, int nboxes, const int64_t *xcnt, const int64_t *vcnt, int64_t *fleaf,
           int64_t *fnon, int64_t *fx, int64_t *fv, hipStream_t s)
{
    k_flags<<<ceil_div(nboxes, 256), 256, 0, s>>>(bx, nboxes, xcnt, vcnt, fleaf, fnon, fx, fv);
}

__global__ __launch_bounds__(256) void k_compact(const int64_t *flag, const int64_t *pos, int nboxes,
                                                 int32_t *out)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nboxes) return;
    if (flag[b]) out[pos[b]] = b;
}

void compact(const int64_t *flag, const int64_t *pos, int nboxes, int32_t *out, hipStream_t s)
{
    k_compact<<<ceil_div(nboxes, 256), 256, 0, s>>>(flag, pos, nboxes, out);
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

__global__ void k_mark(const int32_t *idx, int64_t n, int32_t *flag)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) flag[idx[i]] = 1;
}

void mark(const int32_t *idx, int64_t n, int32_t *flag, hipStream_t s)
{
    if (n > 0) k_mark<<<ceil_div(n, 256), 256, 0, s>>>(idx, n, flag);
}

} // namespace fmm
