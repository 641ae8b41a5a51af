// C ABI of the library (include/fmm.h): plan construction, evaluation, batched
// evaluation, exports and lifetime.  See fmm.h for the contract of each call.
#include "fmm.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "ops.h"
#include "sort.h"
#include "tables.h"
#include "tree_kernels.h"

using namespace fmm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(FMM_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxUniformDepth = 8;

} // namespace

struct fmm_plan_s {
    int device = 0;
    hipStream_t stream = 0;
    fmm_allocator_t alloc{};
    bool user_alloc = false;
    std::vector<std::pair<void *, size_t>> bufs;  // owned, freed by destroy
    std::vector<std::pair<void *, size_t>> temps; // freed at the end of the build
    size_t footprint = 0;
    double root[4] = {0, 0, 0, 1};
    int p = 0, nc = 0, nh = 0, ldm = 0, ldh = 0, D = 0, depth = 0, leaf_size = 0;
    int uniform = 0, precision = 0, mixed_m2l = 0;
    int n = 0, nboxes = 0, nleaves = 0, nxtgt = 0, nslots = 0;
    int64_t nlist[4] = {0, 0, 0, 0};
    std::vector<int> lvl_begin;       // boxes per level (host)
    std::vector<int> lvl_nonleaf_off; // non-leaf boxes per level (host)
    const OrderTables *tab = nullptr;
    PlanView view{};
    PlanView *view_dev = nullptr;
    BoxArrays bx{};
    int64_t *off[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *src[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *perm = nullptr;
    // stage timing
    bool timing = false;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;      // recorded, not yet read
    std::vector<Rec> pool;      // reusable event pairs

    void *raw_alloc(size_t bytes)
    {
        if (bytes == 0) bytes = 8;
        bytes = (bytes + 255) & ~(size_t)255;
        void *p = nullptr;
        if (user_alloc) p = alloc.alloc(bytes, stream, alloc.ctx);
        else if (hipMallocAsync(&p, bytes, stream) != hipSuccess) p = nullptr;
        return p;
    }
    void raw_free(void *p)
    {
        if (!p) return;
        if (user_alloc) alloc.free(p, stream, alloc.ctx);
        else (void)hipFreeAsync(p, stream);
    }
    template <typename T> T *own(size_t count)
    {
        void *p = raw_alloc(sizeof(T) * count);
        if (p) { bufs.push_back({p, sizeof(T) * count}); footprint += sizeof(T) * count; }
        return (T *)p;
    }
    template <typename T> T *temp(size_t count)
    {
        void *p = raw_alloc(sizeof(T) * count);
        if (p) temps.push_back({p, sizeof(T) * count});
        return (T *)p;
    }
    void release_temps()
    {
        for (auto &t : temps) raw_free(t.first);
        temps.clear();
    }
    void release_all()
    {
        release_temps();
        for (auto &b : bufs) raw_free(b.first);
        bufs.clear();
        footprint = 0;
    }
};

extern "C" void fmm_default_options(fmm_options_t *opt)
{
    if (!opt) return;
    opt->uniform_depth = -1;
    opt->max_depth = kMaxDepth;
    opt->precision = FMM_FP64;
    opt->want_field = 1;
    opt->root = nullptr;
}

extern "C" const char *fmm_last_error(void) { return g_err.c_str(); }

namespace {

template <typename T> int copy_to_host(T *dst, const T *src, size_t n, hipStream_t s)
{
    if (n == 0) return 0;
    HIPCHK(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyDeviceToHost, s));
    return 0;
}

#define NOMEM(ptr)                                                                         \
    do {                                                                                   \
        if (!(ptr)) return fail(FMM_ENOMEM, "device allocation failed (" #ptr ")");       \
    } while (0)

// Adaptive boxes, level by level (one host synchronisation per level to learn
// how many children the level produced).
int build_adaptive(fmm_plan_s *P, const uint64_t *keys)
{
    hipStream_t s = P->stream;
    int cap = std::max(64, (int)std::min<int64_t>(2 + 16LL * P->n / (P->leaf_size + 1), 1LL << 30));
    auto alloc_boxes = [&](int c, BoxArrays &b) {
        b.level = P->temp<int32_t>(c); b.first = P->temp<int32_t>(c); b.count = P->temp<int32_t>(c);
        b.parent = P->temp<int32_t>(c); b.child_begin = P->temp<int32_t>(c); b.nchild = P->temp<int32_t>(c);
        b.morton = P->temp<uint64_t>(c);
        return b.level && b.first && b.count && b.parent && b.child_begin && b.nchild && b.morton;
    };
    BoxArrays bx{};
    if (!alloc_boxes(cap, bx)) return fail(FMM_ENOMEM, "device allocation failed (boxes)");
    root_box(P->n, bx, s);
    P->lvl_begin = {0, 1};
    int64_t *nch = P->temp<int64_t>(cap + 1), *off = P->temp<int64_t>(cap + 2);
    int64_t *scr = P->temp<int64_t>(scan_scratch_bytes(cap) / 8 + 1);
    NOMEM(nch); NOMEM(off); NOMEM(scr);
    int ncap_scan = cap;
    for (int l = 0; l < P->D; ++l) {
        int lb = P->lvl_begin[l], le = P->lvl_begin[l + 1], m = le - lb;
        if (m > ncap_scan) {
            ncap_scan = 2 * m;
            nch = P->temp<int64_t>(ncap_scan + 1); off = P->temp<int64_t>(ncap_scan + 2);
            scr = P->temp<int64_t>(scan_scratch_bytes(ncap_scan) / 8 + 1);
            NOMEM(nch); NOMEM(off); NOMEM(scr);
        }
        count_children(keys, P->D, l, lb, le, P->leaf_size, bx, nch, s);
        scan_exclusive(nch, off, m, scr, s);
        int64_t total = 0;
        if (copy_to_host(&total, off + m, 1, s)) return FMM_EDEVICE;
        HIPCHK(hipStreamSynchronize(s));
        if (total == 0) break;
        if (le + total > cap) { // grow, keep contents
            int ncap = (int)std::max<int64_t>(2LL * cap, le + total + 1);
            BoxArrays nb{};
            if (!alloc_boxes(ncap, nb)) return fail(FMM_ENOMEM, "device allocation failed (boxes)");
            HIPCHK(hipMemcpyAsync(nb.level, bx.level, 4ull * le, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(nb.first, bx.first, 4ull * le, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(nb.count, bx.count, 4ull * le, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(nb.parent, bx.parent, 4ull * le, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(nb.child_begin, bx.child_begin, 4ull * le, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(nb.nchild, bx.nchild, 4ull * le, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(nb.morton, bx.morton, 8ull * le, hipMemcpyDeviceToDevice, s));
            bx = nb;
            cap = ncap;
        }
        fill_children(keys, P->D, l, lb, le, off, bx, s);
        P->lvl_begin.push_back(le + (int)total);
    }
    P->nboxes = P->lvl_begin.back();
    // move into owned arrays of the exact size
    int nb = P->nboxes;
    BoxArrays o{};
    o.level = P->own<int32_t>(nb); o.first = P->own<int32_t>(nb); o.count = P->own<int32_t>(nb);
    o.parent = P->own<int32_t>(nb); o.child_begin = P->own<int32_t>(nb); o.nchild = P->own<int32_t>(nb);
    o.morton = P->own<uint64_t>(nb);
    if (!(o.level && o.first && o.count && o.parent && o.child_begin && o.nchild && o.morton))
        return fail(FMM_ENOMEM, "device allocation failed (boxes)");
    HIPCHK(hipMemcpyAsync(o.level, bx.level, 4ull * nb, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(o.first, bx.first, 4ull * nb, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(o.count, bx.count, 4ull * nb, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(o.parent, bx.parent, 4ull * nb, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(o.child_begin, bx.child_begin, 4ull * nb, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(o.nchild, bx.nchild, 4ull * nb, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(o.morton, bx.morton, 8ull * nb, hipMemcpyDeviceToDevice, s));
    P->bx = o;
    return 0;
}

int build_plan(fmm_plan_s *P, const double *xyz)
{
    hipStream_t s = P->stream;
    const int n = P->n;
    // root cube
    double *root_dev = P->temp<double>(4), *part = P->temp<double>(6 * kBBoxBlocks);
    int *bad = P->temp<int>(1);
    NOMEM(root_dev); NOMEM(part); NOMEM(bad);
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
    if (P->root[3] <= 0) { // bounding cube
        bbox(xyz, n, part, root_dev, s);
        if (copy_to_host(P->root, root_dev, 4, s)) return FMM_EDEVICE;
        HIPCHK(hipStreamSynchronize(s));
        if (!std::isfinite(P->root[0]) || !std::isfinite(P->root[1]) || !std::isfinite(P->root[2]) ||
            !std::isfinite(P->root[3]))
            return fail(FMM_EINVAL, "non-finite coordinates");
    }
    // keys and sorted order
    uint64_t *keys = P->temp<uint64_t>(n), *tk = P->temp<uint64_t>(n);
    int32_t *tv = P->temp<int32_t>(n), *sscr = P->temp<int32_t>(sort_scratch_bytes(n) / 4 + 1);
    P->perm = P->own<int32_t>(n);
    NOMEM(keys); NOMEM(tk); NOMEM(tv); NOMEM(sscr); NOMEM(P->perm);
    morton_keys(xyz, n, P->root, P->D, keys, P->perm, bad, s);
    radix_sort_pairs(keys, P->perm, tk, tv, n, 3 * P->D, sscr, s);
    double *xs = P->own<double>(n), *ys = P->own<double>(n), *zs = P->own<double>(n);
    NOMEM(xs); NOMEM(ys); NOMEM(zs);
    gather_sorted(xyz, P->perm, n, xs, ys, zs, s);
    // boxes
    if (P->uniform) {
        P->lvl_begin.assign(1, 0);
        long long tot = 0, sz = 1;
        for (int l = 0; l <= P->D; ++l) { tot += sz; sz *= 8; P->lvl_begin.push_back((int)tot); }
        P->nboxes = (int)tot;
        int nb = P->nboxes;
        BoxArrays o{};
        o.level = P->own<int32_t>(nb); o.first = P->own<int32_t>(nb); o.count = P->own<int32_t>(nb);
        o.parent = P->own<int32_t>(nb); o.child_begin = P->own<int32_t>(nb); o.nchild = P->own<int32_t>(nb);
        o.morton = P->own<uint64_t>(nb);
        if (!(o.level && o.first && o.count && o.parent && o.child_begin && o.nchild && o.morton))
            return fail(FMM_ENOMEM, "device allocation failed (boxes)");
        uniform_boxes(keys, n, P->D, nb, o, s);
        P->bx = o;
    } else {
        int rc = build_adaptive(P, keys);
        if (rc) return rc;
    }
    P->depth = (int)P->lvl_begin.size() - 2;
    const int nb = P->nboxes;
    int32_t *lvl_dev = P->own<int32_t>(kMaxDepth + 2);
    NOMEM(lvl_dev);
    {
        std::vector<int32_t> lb(kMaxDepth + 2, nb);
        for (size_t i = 0; i < P->lvl_begin.size() && i < lb.size(); ++i) lb[i] = P->lvl_begin[i];
        HIPCHK(hipMemcpyAsync(lvl_dev, lb.data(), sizeof(int32_t) * lb.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s)); // lb is a host temporary
    }
    TreeArgs ta{P->bx, lvl_dev, P->D, nb};
    // lists: count, scan, sizes
    int32_t *coll = P->temp<int32_t>(27ull * nb);
    int64_t *cntV = P->temp<int64_t>(nb), *cntU = P->temp<int64_t>(nb), *cntW = P->temp<int64_t>(nb);
    int64_t *cntX = P->temp<int64_t>(nb);
    int64_t *scr = P->temp<int64_t>(scan_scratch_bytes(nb) / 8 + 1);
    for (int w = 0; w < 4; ++w) P->off[w] = P->own<int64_t>(nb + 1);
    NOMEM(coll); NOMEM(cntV); NOMEM(cntU); NOMEM(cntW); NOMEM(cntX); NOMEM(scr);
    NOMEM(P->off[0]); NOMEM(P->off[1]); NOMEM(P->off[2]); NOMEM(P->off[3]);
    int32_t *vslot = P->own<int32_t>((size_t)nb * kVSlots);
    NOMEM(vslot);
    fill_i32(vslot, (int64_t)nb * kVSlots, -1, s);
    colleagues(ta, coll, s);
    vlist(ta, coll, 0, cntV, nullptr, nullptr, nullptr, s);
    uwlist(ta, coll, 0, cntU, nullptr, nullptr, cntW, nullptr, nullptr, s);
    scan_exclusive(cntU, P->off[0], nb, scr, s);
    scan_exclusive(cntV, P->off[1], nb, scr, s);
    scan_exclusive(cntW, P->off[2], nb, scr, s);
    int64_t tot[3];
    if (copy_to_host(&tot[0], P->off[0] + nb, 1, s) || copy_to_host(&tot[1], P->off[1] + nb, 1, s) ||
        copy_to_host(&tot[2], P->off[2] + nb, 1, s))
        return FMM_EDEVICE;
    int badh = 0;
    if (copy_to_host(&badh, bad, 1, s)) return FMM_EDEVICE;
    HIPCHK(hipStreamSynchronize(s));
    if (badh) return fail(FMM_EINVAL, "non-finite coordinates");
    P->nlist[0] = tot[0]; P->nlist[1] = tot[1]; P->nlist[2] = tot[2]; P->nlist[3] = tot[2];
    for (int w = 0; w < 4; ++w) { P->src[w] = P->own<int32_t>(P->nlist[w] ? P->nlist[w] : 1); NOMEM(P->src[w]); }
    vlist(ta, coll, 1, nullptr, P->off[1], P->src[1], vslot, s); // ascending by construction
    uwlist(ta, coll, 1, nullptr, P->off[0], P->src[0], nullptr, P->off[2], P->src[2], s);
    sort_segments(P->off[0], nb, P->src[0], s);
    sort_segments(P->off[2], nb, P->src[2], s);
    // X = transpose of W
    HIPCHK(hipMemsetAsync(cntX, 0, sizeof(int64_t) * nb, s));
    if (P->nlist[2] > 0) {
        int64_t m = P->nlist[2];
        uint64_t *wk = P->temp<uint64_t>(m), *wk2 = P->temp<uint64_t>(m);
        int32_t *wv2 = P->temp<int32_t>(m), *wscr = P->temp<int32_t>(sort_scratch_bytes((int)m) / 4 + 1);
        NOMEM(wk); NOMEM(wk2); NOMEM(wv2); NOMEM(wscr);
        w_pairs(P->off[2], P->src[2], nb, wk, P->src[3], cntX, s);
        int bits = 1;
        while ((1LL << bits) < nb) ++bits;
        radix_sort_pairs(wk, P->src[3], wk2, wv2, (int)m, bits, wscr, s);
    }
    scan_exclusive(cntX, P->off[3], nb, scr, s);
    // work lists: leaves, non-leaves, X targets, M2L targets
    int64_t *flag = P->temp<int64_t>(nb), *pos = P->temp<int64_t>(nb + 1);
    int64_t *flag2 = P->temp<int64_t>(nb), *pos2 = P->temp<int64_t>(nb + 1);
    int64_t *flag3 = P->temp<int64_t>(nb), *pos3 = P->temp<int64_t>(nb + 1);
    int64_t *flag4 = P->temp<int64_t>(nb), *pos4 = P->temp<int64_t>(nb + 1);
    int32_t *leaves = P->own<int32_t>(nb), *nonleaf = P->own<int32_t>(nb), *xtgt = P->own<int32_t>(nb);
    int32_t *mtg = P->temp<int32_t>(nb);
    NOMEM(flag); NOMEM(pos); NOMEM(flag2); NOMEM(pos2); NOMEM(flag3); NOMEM(pos3); NOMEM(flag4); NOMEM(pos4);
    NOMEM(leaves); NOMEM(nonleaf); NOMEM(xtgt); NOMEM(mtg);
    flags(P->bx, nb, 0, nullptr, flag, s);
    scan_exclusive(flag, pos, nb, scr, s);
    compact(flag, pos, nb, leaves, s);
    flags(P->bx, nb, 1, nullptr, flag2, s);
    scan_exclusive(flag2, pos2, nb, scr, s);
    compact(flag2, pos2, nb, nonleaf, s);
    flags(P->bx, nb, 2, P->off[3], flag3, s);
    scan_exclusive(flag3, pos3, nb, scr, s);
    compact(flag3, pos3, nb, xtgt, s);
    flags(P->bx, nb, 2, P->off[1], flag4, s);
    scan_exclusive(flag4, pos4, nb, scr, s);
    compact(flag4, pos4, nb, mtg, s);
    std::vector<int64_t> posh(nb + 1);
    int64_t cnts[3], xt = 0;
    if (copy_to_host(posh.data(), pos2, nb + 1, s) || copy_to_host(&cnts[0], pos + nb, 1, s) ||
        copy_to_host(&cnts[1], pos3 + nb, 1, s) || copy_to_host(&cnts[2], pos4 + nb, 1, s) ||
        copy_to_host(&xt, P->off[3] + nb, 1, s))
        return FMM_EDEVICE;
    HIPCHK(hipStreamSynchronize(s));
    P->nleaves = (int)cnts[0];
    P->nxtgt = (int)cnts[1];
    const int nt = (int)cnts[2];
    if (xt != P->nlist[3]) return fail(FMM_EDEVICE, "X list size mismatch");
    P->lvl_nonleaf_off.assign(P->depth + 2, 0);
    for (int l = 0; l <= P->depth + 1; ++l) {
        int b = l < (int)P->lvl_begin.size() ? P->lvl_begin[l] : nb;
        P->lvl_nonleaf_off[l] = (int)posh[std::min(b, nb)];
    }
    int32_t *lnl_off = P->own<int32_t>(P->depth + 2);
    NOMEM(lnl_off);
    HIPCHK(hipMemcpyAsync(lnl_off, P->lvl_nonleaf_off.data(), sizeof(int32_t) * (P->depth + 2),
                          hipMemcpyHostToDevice, s));
    // M2L target slots
    int64_t slot_cap = ((int64_t)nt + 8 * (kM2LSlots - 1) + kM2LSlots - 1) / kM2LSlots * kM2LSlots;
    if (slot_cap < kM2LSlots) slot_cap = kM2LSlots;
    int32_t *slots = P->own<int32_t>(slot_cap);
    int *octoff = P->temp<int>(32);
    uint64_t *okey = P->temp<uint64_t>(nt + 1), *otk = P->temp<uint64_t>(nt + 1);
    int32_t *oval = P->temp<int32_t>(nt + 1), *otv = P->temp<int32_t>(nt + 1);
    int32_t *oscr = P->temp<int32_t>(sort_scratch_bytes(nt + 1) / 4 + 1);
    NOMEM(slots); NOMEM(octoff); NOMEM(okey); NOMEM(otk); NOMEM(oval); NOMEM(otv); NOMEM(oscr);
    m2l_tiles(P->bx, mtg, nt, okey, oval, otk, otv, oscr, octoff, slots, slot_cap, s);
    P->nslots = (int)slot_cap;
    // evaluation buffers
    double *qs = P->own<double>(n), *pf = P->own<double>(n), *ff = P->own<double>(3ull * n);
    double *M = P->own<double>((size_t)nb * P->ldm), *L = P->own<double>((size_t)nb * P->ldm);
    double *Mh = P->own<double>((size_t)nb * P->ldh), *Lh = P->own<double>((size_t)nb * P->ldh);
    float *Mhf = P->mixed_m2l ? P->own<float>((size_t)nb * P->ldh) : nullptr;
    NOMEM(qs); NOMEM(pf); NOMEM(ff); NOMEM(M); NOMEM(L); NOMEM(Mh); NOMEM(Lh);
    if (P->mixed_m2l) NOMEM(Mhf);
    P->view_dev = P->own<PlanView>(1);
    NOMEM(P->view_dev);

    PlanView &v = P->view;
    v.p = P->p; v.nc = P->nc; v.nh = P->nh; v.ldm = P->ldm; v.ldh = P->ldh;
    v.precision = P->precision; v.mixed_m2l = P->mixed_m2l; v.depth = P->depth; v.D = P->D;
    v.n = n; v.nboxes = nb; v.nleaves = P->nleaves; v.nxtgt = P->nxtgt; v.nslots = P->nslots;
    for (int k = 0; k < 3; ++k) v.lo[k] = P->root[k];
    v.W = P->root[3];
    v.level = P->bx.level; v.parent = P->bx.parent; v.child_begin = P->bx.child_begin;
    v.nchild = P->bx.nchild; v.first = P->bx.first; v.count = P->bx.count; v.morton = P->bx.morton;
    v.perm = P->perm; v.xs = xs; v.ys = ys; v.zs = zs;
    v.U_off = P->off[0]; v.V_off = P->off[1]; v.W_off = P->off[2]; v.X_off = P->off[3];
    v.U_src = P->src[0]; v.W_src = P->src[2]; v.X_src = P->src[3];
    v.m2l_tgt = slots; v.vslot = vslot; v.leaves = leaves; v.xtgt = xtgt;
    v.lvl_nonleaf = nonleaf; v.lvl_nonleaf_off = lnl_off; v.tab = P->tab;
    v.qs = qs; v.M = M; v.Mh = Mh; v.Lh = Lh; v.L = L; v.Mhf = Mhf; v.phi_far = pf; v.fld_far = ff;
    HIPCHK(hipMemcpyAsync(P->view_dev, &v, sizeof(PlanView), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    P->release_temps();
    HIPCHK(hipStreamSynchronize(s));
    return 0;
}

int check_options(const fmm_options_t &o, int order, int leaf_size)
{
    if (o.uniform_depth < -1 || o.uniform_depth > kMaxUniformDepth)
        return fail(FMM_EINVAL, "uniform_depth must be -1 or 0..8");
    if (o.uniform_depth < 0 && (o.max_depth < 1 || o.max_depth > kMaxDepth))
        return fail(FMM_EINVAL, "max_depth must be 1..21");
    if (o.precision != FMM_FP64 && o.precision != FMM_MIXED) return fail(FMM_EINVAL, "bad precision");
    if (o.uniform_depth < 0 && leaf_size < 1) return fail(FMM_EINVAL, "leaf_size must be >= 1");
    if (order < 0 || order > kMaxOrder) return fail(FMM_EINVAL, "order must be 0..12");
    if (o.root) {
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(o.root[k])) return fail(FMM_EINVAL, "non-finite root");
        if (!(o.root[3] > 0)) return fail(FMM_EINVAL, "root width must be > 0");
    }
    return 0;
}

} // namespace

extern "C" int fmm_plan(const double *xyz_dev, int64_t n, int32_t order, int32_t leaf_size,
                        const fmm_options_t *opt, const fmm_allocator_t *alloc, hipStream_t stream,
                        fmm_plan_t *out)
{
    g_err.clear();
    if (!xyz_dev || !out) return fail(FMM_EINVAL, "null pointer argument");
    if (n < 1 || n >= (1LL << 31)) return fail(FMM_EINVAL, "n must be in [1, 2^31)");
    fmm_options_t o;
    fmm_default_options(&o);
    if (opt) o = *opt;
    int rc = check_options(o, order, leaf_size);
    if (rc) return rc;
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(FMM_EINVAL, "allocator without functions");
    static thread_local int pool_dev = -1;
    {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess && dev != pool_dev) {
            hipMemPool_t pool;
            if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
                uint64_t thr = UINT64_MAX; // keep freed memory for reuse by later plans
                (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
            }
            pool_dev = dev;
        }
    }
    std::string err;
    const OrderTables *host_tab = nullptr;
    const OrderTables *tab = get_order_tables(order, &host_tab, err);
    if (!tab) return fail(FMM_EDEVICE, err);
    fmm_plan_s *P = new (std::nothrow) fmm_plan_s();
    if (!P) return fail(FMM_ENOMEM, "host allocation failed");
    if (hipGetDevice(&P->device) != hipSuccess) { delete P; return fail(FMM_EDEVICE, "hipGetDevice failed"); }
    P->stream = stream;
    if (alloc) { P->alloc = *alloc; P->user_alloc = true; }
    P->p = order; P->nc = ncoef(order); P->nh = nharm(order);
    P->ldm = pad16(P->nc); P->ldh = pad16(P->nh);
    P->uniform = o.uniform_depth >= 0;
    P->D = P->uniform ? o.uniform_depth : o.max_depth;
    P->leaf_size = leaf_size;
    P->precision = o.precision;
    P->mixed_m2l = (o.precision == FMM_MIXED && order <= 8) ? 1 : 0;
    P->n = (int)n;
    P->tab = tab;
    if (o.root) for (int k = 0; k < 4; ++k) P->root[k] = o.root[k];
    else P->root[3] = -1.0;
    rc = build_plan(P, xyz_dev);
    if (rc) {
        std::string msg = g_err;
        (void)hipStreamSynchronize(stream);
        P->release_all();
        (void)hipStreamSynchronize(stream);
        delete P;
        g_err = msg;
        return rc;
    }
    *out = P;
    return FMM_OK;
}

namespace {

struct StagePlan {
    // per-stage block counts of one plan
    int permute, p2m, fold, m2l, p2l, unfold, far, p2p;
};

StagePlan stage_blocks(const fmm_plan_s *P)
{
    StagePlan sp;
    sp.permute = (int)ceil_div(P->n, 256);
    sp.p2m = P->nleaves;
    sp.fold = (int)ceil_div(P->nboxes, 4);
    sp.m2l = P->nslots / kM2LSlots;
    sp.p2l = P->nxtgt;
    sp.unfold = sp.fold;
    sp.far = P->nleaves;
    sp.p2p = (int)ceil_div(P->nleaves, 4);
    return sp;
}

int nonleaf_groups(const fmm_plan_s *P, int level)
{
    if (level < 0 || level > P->depth) return 0;
    int c = P->lvl_nonleaf_off[level + 1] - P->lvl_nonleaf_off[level];
    return (int)ceil_div(c, 16);
}

// Brackets a stage with events when the (single) plan has timing on.
struct StageTimer {
    fmm_plan_s *P;
    hipStream_t s;
    fmm_plan_s::Rec cur{};
    bool on = false;
    StageTimer(fmm_plan_s *p, hipStream_t st) : P(p), s(st) {}
    void begin(int stage)
    {
        on = P && P->timing;
        if (!on) return;
        if (!P->pool.empty()) { cur = P->pool.back(); P->pool.pop_back(); }
        else if (hipEventCreate(&cur.a) != hipSuccess || hipEventCreate(&cur.b) != hipSuccess) { on = false; return; }
        cur.stage = stage;
        (void)hipEventRecord(cur.a, s);
    }
    void end()
    {
        if (!on) return;
        (void)hipEventRecord(cur.b, s);
        P->recs.push_back(cur);
        on = false;
    }
};

// Runs the whole evaluation pipeline for `count` plans whose views are in V.
// Plans with different orders get separate launches of the order-templated
// kernels; everything else is one launch per stage for all plans.
int run_pipeline(fmm_plan_s *const *P, int count, const PlanView *V, hipStream_t s)
{
    StageTimer T(count == 1 ? P[0] : nullptr, s);
    auto make = [&](auto fn, const std::vector<int> &sel) {
        Bases B{};
        B.n = (int)sel.size();
        B.b[0] = 0;
        for (size_t i = 0; i < sel.size(); ++i) B.b[i + 1] = B.b[i] + fn(P[sel[i]]);
        return B;
    };
    // all plans are addressed by their index in V; a launch over a subset uses
    // a view array offset, so subsets must be contiguous runs of equal order
    std::vector<int> all(count);
    for (int i = 0; i < count; ++i) all[i] = i;
    Bases Bp = make([](const fmm_plan_s *p) { return stage_blocks(p).permute; }, all);
    T.begin(0);
    launch_permute_q(V, Bp, s);
    T.end();
    // runs of equal order (callers sort batches by order)
    std::vector<std::pair<int, int>> runs;
    for (int i = 0; i < count;) {
        int j = i;
        while (j < count && P[j]->p == P[i]->p && P[j]->mixed_m2l == P[i]->mixed_m2l) ++j;
        runs.push_back({i, j});
        i = j;
    }
    auto sub = [&](int a, int b, auto fn) {
        std::vector<int> idx;
        for (int i = a; i < b; ++i) idx.push_back(i);
        Bases B{};
        B.n = b - a;
        B.b[0] = 0;
        for (int i = 0; i < b - a; ++i) B.b[i + 1] = B.b[i] + fn(P[a + i]);
        return B;
    };
    T.begin(1);
    for (auto &r : runs)
        launch_p2m(P[r.first]->p, V + r.first,
                   sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).p2m; }), s);
    for (auto &r : runs)
        launch_p2m_transform(V + r.first, sub(r.first, r.second, [](const fmm_plan_s *p) {
            return (int)ceil_div(p->nleaves, 16) * (p->ldm / 16); }), s);
    T.end();
    int maxdepth = 0;
    for (int i = 0; i < count; ++i) maxdepth = std::max(maxdepth, P[i]->depth);
    T.begin(2);
    // Multipoles of levels 0 and 1 are never read by M2L (V lists start at
    // level 2) nor by M2P (W lists hold boxes of level >= 2), so the upward
    // pass stops at level 2; fmm_plan_export_expansions completes it on demand.
    for (auto &r : runs)
        for (int l = maxdepth - 1; l >= 2; --l)
            launch_m2m(V + r.first,
                       sub(r.first, r.second, [l](const fmm_plan_s *p) { return nonleaf_groups(p, l) * (p->ldm / 16); }), l, s);
    T.end();
    T.begin(3);
    launch_fold(V, make([](const fmm_plan_s *p) { return stage_blocks(p).fold; }, all), s);
    T.end();
    T.begin(4);
    for (auto &r : runs)
        launch_m2l(P[r.first]->p, P[r.first]->mixed_m2l, V + r.first,
                   sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).m2l; }), s);
    T.end();
    T.begin(5);
    for (auto &r : runs)
        launch_p2l(P[r.first]->p, V + r.first,
                   sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).p2l; }), s);
    for (auto &r : runs)
        launch_p2l_transform(V + r.first, sub(r.first, r.second, [](const fmm_plan_s *p) {
            return (int)ceil_div(p->nxtgt, 16) * (p->ldh / 16); }), s);
    T.end();
    T.begin(6);
    launch_unfold(V, make([](const fmm_plan_s *p) { return stage_blocks(p).unfold; }, all), s);
    T.end();
    T.begin(7);
    for (auto &r : runs)
        for (int l = 2; l < maxdepth; ++l)
            launch_l2l(V + r.first,
                       sub(r.first, r.second, [l](const fmm_plan_s *p) { return nonleaf_groups(p, l) * (p->ldm / 16); }), l, s);
    T.end();
    T.begin(8);
    for (auto &r : runs)
        launch_far(P[r.first]->p, V + r.first,
                   sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).far; }), s);
    T.end();
    T.begin(9);
    // P2P: FP64 and mixed plans in separate launches
    for (int mixed = 0; mixed <= 1; ++mixed) {
        for (int i = 0; i < count;) {
            if ((P[i]->precision == FMM_MIXED) != (mixed == 1)) { ++i; continue; }
            int j = i;
            while (j < count && (P[j]->precision == FMM_MIXED) == (mixed == 1)) ++j;
            launch_p2p(mixed, V + i, sub(i, j, [](const fmm_plan_s *p) { return stage_blocks(p).p2p; }), s);
            i = j;
        }
    }
    T.end();
    HIPCHK(hipGetLastError());
    return 0;
}

} // namespace

extern "C" int fmm_evaluate(fmm_plan_t plan, const double *q_dev, double *phi_dev, double *field_dev,
                            hipStream_t stream)
{
    g_err.clear();
    if (!plan || !q_dev || !phi_dev) return fail(FMM_EINVAL, "null pointer argument");
    fmm_plan_s *P = plan;
    PlanView v = P->view;
    v.q_in = q_dev;
    v.phi_out = phi_dev;
    v.fld_out = field_dev;
    HIPCHK(hipMemcpyAsync(P->view_dev, &v, sizeof(PlanView), hipMemcpyHostToDevice, stream));
    fmm_plan_s *arr[1] = {P};
    return run_pipeline(arr, 1, P->view_dev, stream);
}

extern "C" int fmm_evaluate_batch(fmm_plan_t const *plans, const double *const *q_dev,
                                  double *const *phi_dev, double *const *field_dev, int32_t count,
                                  hipStream_t stream)
{
    g_err.clear();
    if (count < 0 || (count > 0 && (!plans || !q_dev || !phi_dev)))
        return fail(FMM_EINVAL, "bad batch arguments");
    if (count == 0) return FMM_OK;
    for (int i = 0; i < count; ++i)
        if (!plans[i] || !q_dev[i] || !phi_dev[i]) return fail(FMM_EINVAL, "null entry in batch");
    // order the plans by (order, mixed M2L) so that equal orders are contiguous
    std::vector<int> idx(count);
    for (int i = 0; i < count; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (plans[a]->p != plans[b]->p) return plans[a]->p < plans[b]->p;
        return plans[a]->mixed_m2l < plans[b]->mixed_m2l;
    });
    for (int c0 = 0; c0 < count; c0 += kMaxBatch) {
        int c1 = std::min(count, c0 + kMaxBatch);
        std::vector<fmm_plan_s *> P;
        std::vector<PlanView> views;
        for (int t = c0; t < c1; ++t) {
            int i = idx[t];
            P.push_back(plans[i]);
            PlanView v = plans[i]->view;
            v.q_in = q_dev[i];
            v.phi_out = phi_dev[i];
            v.fld_out = field_dev ? field_dev[i] : nullptr;
            views.push_back(v);
        }
        PlanView *Vd = nullptr;
        HIPCHK(hipMallocAsync((void **)&Vd, sizeof(PlanView) * views.size(), stream));
        HIPCHK(hipMemcpyAsync(Vd, views.data(), sizeof(PlanView) * views.size(), hipMemcpyHostToDevice, stream));
        int rc = run_pipeline(P.data(), (int)P.size(), Vd, stream);
        (void)hipFreeAsync(Vd, stream);
        if (rc) return rc;
    }
    return FMM_OK;
}

extern "C" int fmm_plan_footprint(fmm_plan_t plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(FMM_EINVAL, "null pointer argument");
    *bytes = plan->footprint;
    return FMM_OK;
}

extern "C" int fmm_plan_estimate(int64_t n, int32_t order, int32_t leaf_size, const fmm_options_t *opt,
                                 size_t *bytes)
{
    if (!bytes || n < 1 || order < 0 || order > kMaxOrder) return fail(FMM_EINVAL, "bad arguments");
    fmm_options_t o;
    fmm_default_options(&o);
    if (opt) o = *opt;
    double boxes;
    if (o.uniform_depth >= 0) {
        boxes = 0;
        for (int l = 0, s = 1; l <= o.uniform_depth; ++l, s *= 8) boxes += s;
    } else {
        boxes = 1 + 8.0 * 2.0 * n / (leaf_size + 1);
    }
    double ldm = pad16(ncoef(order)), ldh = pad16(nharm(order));
    double per_box = 8 * (2 * ldm + 2 * ldh) + 4 * (ldh) + 4 * 200 + 64; // expansions, slots, lists
    double per_particle = 8 * 3 + 4 + 8 * 5 + 8 * 2;
    double total = boxes * per_box + n * per_particle + 8 * 27 * boxes;
    *bytes = (size_t)(total * 1.25);
    return FMM_OK;
}

extern "C" int fmm_plan_sizes(fmm_plan_t plan, int64_t out[10])
{
    if (!plan || !out) return fail(FMM_EINVAL, "null pointer argument");
    out[0] = plan->nboxes; out[1] = plan->nlist[0]; out[2] = plan->nlist[1];
    out[3] = plan->nlist[2]; out[4] = plan->nlist[3]; out[5] = plan->depth; out[6] = plan->D;
    out[7] = plan->n; out[8] = plan->p; out[9] = plan->nc;
    return FMM_OK;
}

extern "C" int fmm_plan_export_tree(fmm_plan_t plan, hipStream_t stream, double *root_host,
                                    int64_t *perm_host, int32_t *level_host, uint64_t *morton_host,
                                    int64_t *first_host, int64_t *count_host, int32_t *parent_host,
                                    int32_t *child_begin_host, int32_t *nchild_host, int64_t *U_off_host,
                                    int32_t *U_src_host, int64_t *V_off_host, int32_t *V_src_host,
                                    int64_t *W_off_host, int32_t *W_src_host, int64_t *X_off_host,
                                    int32_t *X_src_host)
{
    if (!plan) return fail(FMM_EINVAL, "null plan");
    fmm_plan_s *P = plan;
    HIPCHK(hipStreamSynchronize(stream));
    const int nb = P->nboxes, n = P->n;
    if (root_host) std::memcpy(root_host, P->root, sizeof(P->root));
    std::vector<int32_t> t32;
    auto widen = [&](int64_t *dst, const int32_t *src, int cnt) -> int {
        if (!dst) return 0;
        t32.resize(cnt);
        if (cnt) HIPCHK(hipMemcpy(t32.data(), src, 4ull * cnt, hipMemcpyDeviceToHost));
        for (int i = 0; i < cnt; ++i) dst[i] = t32[i];
        return 0;
    };
    auto copy32 = [&](int32_t *dst, const int32_t *src, int64_t cnt) -> int {
        if (dst && cnt) HIPCHK(hipMemcpy(dst, src, 4ull * cnt, hipMemcpyDeviceToHost));
        return 0;
    };
    auto copy64 = [&](void *dst, const void *src, int64_t cnt) -> int {
        if (dst && cnt) HIPCHK(hipMemcpy(dst, src, 8ull * cnt, hipMemcpyDeviceToHost));
        return 0;
    };
    int rc = widen(perm_host, P->perm, n) | widen(first_host, P->bx.first, nb) |
             widen(count_host, P->bx.count, nb) | copy32(level_host, P->bx.level, nb) |
             copy64(morton_host, P->bx.morton, nb) | copy32(parent_host, P->bx.parent, nb) |
             copy32(child_begin_host, P->bx.child_begin, nb) | copy32(nchild_host, P->bx.nchild, nb) |
             copy64(U_off_host, P->off[0], nb + 1) | copy32(U_src_host, P->src[0], P->nlist[0]) |
             copy64(V_off_host, P->off[1], nb + 1) | copy32(V_src_host, P->src[1], P->nlist[1]) |
             copy64(W_off_host, P->off[2], nb + 1) | copy32(W_src_host, P->src[2], P->nlist[2]) |
             copy64(X_off_host, P->off[3], nb + 1) | copy32(X_src_host, P->src[3], P->nlist[3]);
    return rc ? FMM_EDEVICE : FMM_OK;
}

extern "C" int fmm_plan_export_expansions(fmm_plan_t plan, hipStream_t stream, double *M_host,
                                          double *L_host)
{
    if (!plan) return fail(FMM_EINVAL, "null plan");
    fmm_plan_s *P = plan;
    HIPCHK(hipStreamSynchronize(stream));
    const int nb = P->nboxes, nc = P->nc, ldm = P->ldm;
    std::vector<int32_t> lev(nb);
    HIPCHK(hipMemcpy(lev.data(), P->bx.level, 4ull * nb, hipMemcpyDeviceToHost));
    std::vector<int> deg(nc);
    std::vector<double> fct(nc);
    for (int d = 0; d <= P->p; ++d)
        for (int i = d; i >= 0; --i)
            for (int j = d - i; j >= 0; --j) {
                int k = d - i - j, id = mono_index(i, j, k);
                deg[id] = d;
                double f = 1;
                for (int t = 2; t <= i; ++t) f *= t;
                for (int t = 2; t <= j; ++t) f *= t;
                for (int t = 2; t <= k; ++t) f *= t;
                fct[id] = f;
            }
    std::vector<double> inv_w(P->p + 1);
    for (int d = 0; d <= P->p; ++d) {
        double df = 1;
        for (int t = 2 * d - 1; t > 1; t -= 2) df *= t;
        inv_w[d] = (d & 1) ? -df : df;
    }
    std::vector<double> buf((size_t)nb * ldm);
    if (M_host) {
        // finish the upward pass into levels 1 and 0 (not needed by the evaluation)
        Bases B{};
        B.n = 1;
        B.b[0] = 0;
        for (int l = std::min(1, P->depth - 1); l >= 0; --l) {
            B.b[1] = nonleaf_groups(P, l) * (P->ldm / 16);
            launch_m2m(P->view_dev, B, l, stream);
        }
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(hipMemcpy(buf.data(), P->view.M, 8ull * nb * ldm, hipMemcpyDeviceToHost));
        for (int b = 0; b < nb; ++b) {
            double h = P->root[3] / std::ldexp(1.0, lev[b]);
            for (int a = 0; a < nc; ++a)
                M_host[(size_t)b * nc + a] = buf[(size_t)b * ldm + a] * inv_w[deg[a]] * std::pow(h, deg[a]);
        }
    }
    if (L_host) {
        HIPCHK(hipMemcpy(buf.data(), P->view.L, 8ull * nb * ldm, hipMemcpyDeviceToHost));
        for (int b = 0; b < nb; ++b) {
            double h = P->root[3] / std::ldexp(1.0, lev[b]);
            for (int a = 0; a < nc; ++a)
                L_host[(size_t)b * nc + a] =
                    lev[b] >= 2 ? buf[(size_t)b * ldm + a] / (fct[a] * std::pow(h, deg[a] + 1)) : 0.0;
        }
    }
    return FMM_OK;
}

extern "C" int fmm_plan_set_timing(fmm_plan_t plan, int on)
{
    if (!plan) return fail(FMM_EINVAL, "null plan");
    plan->timing = on != 0;
    return FMM_OK;
}

extern "C" int fmm_plan_read_timing(fmm_plan_t plan, double ms[16], int64_t calls[16])
{
    if (!plan || !ms || !calls) return fail(FMM_EINVAL, "null pointer argument");
    for (auto &r : plan->recs) {
        HIPCHK(hipEventSynchronize(r.b));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.stage] += t;
        calls[r.stage] += 1;
        plan->pool.push_back(r);
    }
    plan->recs.clear();
    return FMM_OK;
}

extern "C" int fmm_plan_destroy(fmm_plan_t plan)
{
    if (!plan) return fail(FMM_EINVAL, "null plan");
    for (auto &r : plan->recs) { (void)hipEventSynchronize(r.b); plan->pool.push_back(r); }
    for (auto &r : plan->pool) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    plan->recs.clear();
    plan->pool.clear();
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev != plan->device) (void)hipSetDevice(plan->device);
    plan->release_all();
    if (dev != plan->device) (void)hipSetDevice(dev);
    delete plan;
    return FMM_OK;
}
