// C ABI of the library (include/fmm.h): plan construction, evaluation, batched
// evaluation, exports and lifetime.  See fmm.h for the contract of each call.
#include "fmm.h"

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "ops.h"
#include "soft.h"
#include "sort.h"
#include "tables.h"
#include "tree_kernels.h"
#include "batch.h"

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

// Everything the host needs to know about a tree before it sizes the list
// arrays, gathered on the device and fetched with one copy.
struct PlanSizes {
    int64_t tot[4];                  // U, V, W, X list lengths
    int64_t nleaves, nnonleaf, nxtgt, nmtg;
    int64_t lnl[kMaxDepth + 2];      // non-leaf boxes before each level
    int32_t lvl_begin[kMaxDepth + 2];
    double root[4];
    int32_t bad;
};

__global__ void k_collect_sizes(const int64_t *uoff, const int64_t *voff, const int64_t *woff,
                                const int64_t *xoff, const int64_t *pleaf, const int64_t *pnon,
                                const int64_t *px, const int64_t *pv, const int32_t *lvl_begin,
                                const double *root, const int *bad, int nb, PlanSizes *out,
                                int32_t *lnl_off)
{
    const int t = threadIdx.x;
    if (t == 0) {
        out->tot[0] = uoff[nb]; out->tot[1] = voff[nb]; out->tot[2] = woff[nb]; out->tot[3] = xoff[nb];
        out->nleaves = pleaf[nb]; out->nnonleaf = pnon[nb]; out->nxtgt = px[nb]; out->nmtg = pv[nb];
        out->bad = *bad;
    }
    if (t < 4) out->root[t] = root[t];
    if (t < kMaxDepth + 2) {
        int b = lvl_begin[t];
        out->lvl_begin[t] = b;
        out->lnl[t] = pnon[b < nb ? b : nb];
        lnl_off[t] = (int32_t)pnon[b < nb ? b : nb]; // non-leaf boxes before level t
    }
}

// Device memory cache.  Plans are built and destroyed per solve, and every
// build takes a few large chunks (owned and temporary), so hipMallocAsync /
// hipFreeAsync calls would dominate small solves.  A freed chunk is kept,
// with an event recorded on the stream that freed it, in a per-device list
// (up to kCacheBytes); an allocation of at most the chunk's size and at least
// half of it takes it back after making its own stream wait for that event,
// so the memory is reused in stream order without blocking the host.
namespace {
constexpr size_t kCacheBytes = (size_t)8 << 30;
struct Cached { void *p; size_t bytes; hipEvent_t ready; };
std::mutex g_cache_mu;
std::map<int, std::multimap<size_t, Cached>> g_mem_cache;
std::map<int, size_t> g_cache_total;
std::map<int, std::vector<hipEvent_t>> g_event_pool;
} // namespace

// *got receives the size of the chunk handed out (>= bytes)
static void *cache_alloc(int dev, size_t bytes, hipStream_t s, size_t *got)
{
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto &m = g_mem_cache[dev];
        auto it = m.lower_bound(bytes);
        if (it != m.end() && it->first <= 2 * bytes) {
            Cached c = it->second;
            m.erase(it);
            g_cache_total[dev] -= c.bytes;
            if (hipStreamWaitEvent(s, c.ready, 0) == hipSuccess) {
                g_event_pool[dev].push_back(c.ready);
                *got = c.bytes;
                return c.p;
            }
            (void)hipEventSynchronize(c.ready);
            (void)hipEventDestroy(c.ready);
            (void)hipFree(c.p);
        }
    }
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
        // out of memory: hand the cached chunks back to the device and retry
        (void)hipGetLastError();
        std::multimap<size_t, Cached> all;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            all.swap(g_mem_cache[dev]);
            g_cache_total[dev] = 0;
        }
        if (all.empty()) return nullptr;
        for (auto &e : all) {
            (void)hipEventSynchronize(e.second.ready);
            (void)hipEventDestroy(e.second.ready);
            (void)hipFree(e.second.p);
        }
        if (hipMallocAsync(&p, bytes, s) != hipSuccess) return nullptr;
    }
    *got = bytes;
    return p;
}

static void cache_free(int dev, void *p, size_t bytes, hipStream_t s)
{
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (g_cache_total[dev] + bytes > kCacheBytes) {
            (void)hipFreeAsync(p, s);
            return;
        }
        auto &ep = g_event_pool[dev];
        if (!ep.empty()) { ev = ep.back(); ep.pop_back(); }
    }
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipFreeAsync(p, s);
        return;
    }
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipEventDestroy(ev);
        (void)hipFreeAsync(p, s);
        return;
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_mem_cache[dev].insert({bytes, Cached{p, bytes, ev}});
    g_cache_total[dev] += bytes;
}

// Side streams (with their fork and join events) are kept in a per-device
// pool: creating a stream costs far more than an evaluation's launches, and a
// plan built per solve would otherwise create one every time.  A released
// stream may still be running its last P2P; work queued on it later simply
// follows.
namespace {
struct SideSet { hipStream_t s; hipEvent_t fork, join; };
std::mutex g_side_mu;
std::map<int, std::vector<SideSet>> g_side_pool;
} // namespace

static int side_acquire(int dev, hipStream_t &s, hipEvent_t &fork, hipEvent_t &join)
{
    {
        std::lock_guard<std::mutex> lk(g_side_mu);
        auto &v = g_side_pool[dev];
        if (!v.empty()) {
            s = v.back().s; fork = v.back().fork; join = v.back().join;
            v.pop_back();
            return 0;
        }
    }
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) { s = nullptr; return -1; }
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(s);
        s = nullptr;
        return -1;
    }
    return 0;
}

static void side_release(int dev, hipStream_t s, hipEvent_t fork, hipEvent_t join)
{
    std::lock_guard<std::mutex> lk(g_side_mu);
    g_side_pool[dev].push_back({s, fork, join});
}

struct fmm_plan_s {
    int device = 0;
    hipStream_t stream = 0;
    fmm_allocator_t alloc{};
    bool user_alloc = false;
    std::vector<std::pair<void *, size_t>> bufs;  // owned, freed by destroy
    std::vector<std::pair<void *, size_t>> temps; // freed at the end of the build
    size_t footprint = 0;
    double root[4] = {0, 0, 0, 1};
    int p = 0, nc = 0, nh = 0, ldm = 0, ldh = 0, ldmh = 0, D = 0, depth = 0, leaf_size = 0;
    int uniform = 0, precision = 0, mixed_m2l = 0, m2l_rot = 0;
    const RotTables *rot = nullptr; // rotation-based M2L factors (device)
    int kernel = FMM_KERNEL_COULOMB;  // softened kernel: full expansions, tables per level
    double eps = 0.0;
    int n = 0, nboxes = 0, nleaves = 0, nxtgt = 0, nslots = 0, m2l_parts = 1;
    int64_t nlist[4] = {0, 0, 0, 0};
    std::vector<int> lvl_begin;       // boxes per level (host)
    std::vector<int> lvl_nonleaf_off; // non-leaf boxes per level (host)
    const OrderTables *tab = nullptr;
    PlanView view{};
    PlanView *view_dev = nullptr;
    // recorded on the build stream after the last build step: work on other
    // streams (evaluations, exports) waits for it
    hipEvent_t built = nullptr;
    BoxArrays bx{};
    int64_t *off[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *src[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *perm = nullptr;
    // stage timing
    bool timing = false;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;      // recorded, not yet read
    std::vector<Rec> pool;      // reusable event pairs

    // streams other than the build stream that evaluated this plan, each with
    // an event after its latest evaluation; destroy waits for them
    std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
    int note_use(hipStream_t s)
    {
        if (s == stream) return 0;
        hipEvent_t ev = nullptr;
        for (auto &u : uses)
            if (u.first == s) ev = u.second;
        if (!ev) {
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return -1;
            uses.push_back({s, ev});
        }
        return hipEventRecord(ev, s) == hipSuccess ? 0 : -1;
    }
    // P2P runs on a stream of the plan's own, concurrently with the far-field
    // stages; two events fork it after the charge permutation and join it
    // before the output
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int ensure_side()
    {
        if (side) return 0;
        return side_acquire(device, side, ev_fork, ev_join);
    }
    void release_side()
    {
        if (side) side_release(device, side, ev_fork, ev_join);
        side = nullptr; ev_fork = ev_join = nullptr;
    }
    PlanSizes sizes{};         // host copy of the device size record
    int32_t *lvl_dev = nullptr; // first box of every level (device)
    int32_t *wsrc = nullptr;    // W-list source flags (plans with W lists)

    static size_t rounded(size_t bytes) { return ((bytes ? bytes : 8) + 255) & ~(size_t)255; }
    // returns the chunk and, in *got, its size
    void *raw_alloc(size_t bytes, size_t *got)
    {
        bytes = rounded(bytes);
        *got = bytes;
        if (user_alloc) return alloc.alloc(bytes, stream, alloc.ctx);
        return cache_alloc(device, bytes, stream, got);
    }
    void raw_free(void *p, size_t bytes)
    {
        if (!p) return;
        if (user_alloc) alloc.free(p, stream, alloc.ctx);
        else cache_free(device, p, bytes, stream);
    }
    // Buffers are carved from a few large chunks (reserve_*), one per build
    // phase; a request that does not fit the current chunk gets its own
    // allocation.  Owned buffers live until destroy, temporaries until the end
    // of the build.
    struct Chunk { char *base = nullptr; size_t cap = 0, used = 0; };
    Chunk own_chunk, temp_chunk;
    void *carve(Chunk &c, size_t bytes)
    {
        bytes = rounded(bytes);
        if (!c.base || c.used + bytes > c.cap) return nullptr;
        void *p = c.base + c.used;
        c.used += bytes;
        return p;
    }
    bool reserve(bool owned, size_t bytes)
    {
        bytes = rounded(bytes);
        size_t got = 0;
        void *p = raw_alloc(bytes, &got);
        if (!p) return false;
        if (owned) { bufs.push_back({p, got}); footprint += got; own_chunk = {(char *)p, bytes, 0}; }
        else { temps.push_back({p, got}); temp_chunk = {(char *)p, bytes, 0}; }
        return true;
    }
    template <typename T> T *own(size_t count)
    {
        size_t b = sizeof(T) * count, got = 0;
        void *p = carve(own_chunk, b);
        if (p) return (T *)p;
        p = raw_alloc(b, &got);
        if (p) { bufs.push_back({p, got}); footprint += got; }
        return (T *)p;
    }
    template <typename T> T *temp(size_t count)
    {
        size_t b = sizeof(T) * count, got = 0;
        void *p = carve(temp_chunk, b);
        if (p) return (T *)p;
        p = raw_alloc(b, &got);
        if (p) temps.push_back({p, got});
        return (T *)p;
    }
    void release_temps()
    {
        for (auto &t : temps) raw_free(t.first, t.second);
        temps.clear();
        temp_chunk = Chunk{};
    }
    void release_all()
    {
        release_temps();
        for (auto &b : bufs) raw_free(b.first, b.second);
        bufs.clear();
        own_chunk = Chunk{};
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
    opt->m2l_method = FMM_M2L_SIGN_CLASS;
    opt->kernel = FMM_KERNEL_COULOMB;
    opt->softening = 0.0;
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

// Byte total of a list of buffers carved from one chunk.
struct Sizer {
    size_t total = 0;
    template <typename T> Sizer &add(size_t count) { total += fmm_plan_s::rounded(sizeof(T) * count); return *this; }
};

// Plan construction, stream-ordered on the plan's stream with three host
// synchronisations (two for a uniform tree): the box count of an adaptive
// tree, the list and work-list sizes, and the end of the build.
int build_plan(fmm_plan_s *P, const double *xyz)
{
    hipStream_t s = P->stream;
    const int n = P->n;
    const bool adaptive = !P->uniform;
    // ---- phase A: particles (sizes known from n)
    {
        Sizer o;
        o.add<int32_t>(n).add<double>(n).add<double>(n).add<double>(n).add<double>(n).add<double>(n).add<double>(3ull * n);
        if (!P->reserve(true, o.total)) return fail(FMM_ENOMEM, "device allocation failed (particles)");
        Sizer t;
        t.add<double>(4).add<double>(6 * kBBoxBlocks).add<int>(1).add<uint64_t>(n).add<uint64_t>(n).add<int32_t>(n)
         .add<int32_t>(sort_scratch_bytes(n) / 4 + 1);
        if (adaptive) t.add<int64_t>(n + 1).add<int64_t>(n + 2).add<int64_t>(scan_scratch_bytes(n + 1) / 8 + 1);
        if (!P->reserve(false, t.total)) return fail(FMM_ENOMEM, "device allocation failed (keys)");
    }
    P->perm = P->own<int32_t>(n);
    double *xs = P->own<double>(n), *ys = P->own<double>(n), *zs = P->own<double>(n);
    double *qs = P->own<double>(n), *pf = P->own<double>(n), *ff = P->own<double>(3ull * n);
    double *root_dev = P->temp<double>(4), *part = P->temp<double>(6 * kBBoxBlocks);
    int *bad = P->temp<int>(1);
    uint64_t *keys = P->temp<uint64_t>(n), *tk = P->temp<uint64_t>(n);
    int32_t *tv = P->temp<int32_t>(n), *sscr = P->temp<int32_t>(sort_scratch_bytes(n) / 4 + 1);
    NOMEM(P->perm); NOMEM(xs); NOMEM(ys); NOMEM(zs); NOMEM(qs); NOMEM(pf); NOMEM(ff);
    NOMEM(root_dev); NOMEM(part); NOMEM(bad); NOMEM(keys); NOMEM(tk); NOMEM(tv); NOMEM(sscr);
    const bool given = P->root[3] > 0;
    plan_init(given ? P->root : nullptr, root_dev, bad, s);
    if (!given) bbox(xyz, n, part, root_dev, s); // bounding cube, stays on the device
    morton_keys(xyz, n, root_dev, P->D, keys, P->perm, bad, s);
    radix_sort_pairs(keys, P->perm, tk, tv, n, 3 * P->D, sscr, s);
    gather_sorted(xyz, P->perm, n, xs, ys, zs, s);
    // ---- box count
    int64_t *ecnt = nullptr, *eoff = nullptr;
    if (adaptive) {
        ecnt = P->temp<int64_t>(n + 1);
        eoff = P->temp<int64_t>(n + 2);
        int64_t *escr = P->temp<int64_t>(scan_scratch_bytes(n + 1) / 8 + 1);
        NOMEM(ecnt); NOMEM(eoff); NOMEM(escr);
        emit_count(keys, n, P->D, P->leaf_size, ecnt, s);
        scan_exclusive(ecnt, eoff, n, escr, s);
        int64_t total = 0;
        if (copy_to_host(&total, eoff + n, 1, s)) return FMM_EDEVICE;
        HIPCHK(hipStreamSynchronize(s));
        if (total < 1 || total >= (1LL << 31)) return fail(FMM_EDEVICE, "bad box count");
        P->nboxes = (int)total;
    } else {
        long long tot = 0, sz = 1;
        for (int l = 0; l <= P->D; ++l) { tot += sz; sz *= 8; }
        P->nboxes = (int)tot;
    }
    const int nb = P->nboxes;
    const bool soft = P->kernel == FMM_KERNEL_SOFTENED;
    P->m2l_parts = (P->m2l_rot || soft) ? 1 : sym_m2l_parts(P->p);
    // the sign-class M2L addresses the folded multipoles with 32-bit byte offsets
    if (!soft && m2l_sym(P->p) && (unsigned long long)(nb + 1) * (unsigned long long)P->ldmh * 8ULL >= (1ULL << 32))
        return fail(FMM_EUNSUPPORTED, "too many boxes for this order (folded multipoles reach 4 GiB)");
    // (and the softened kernel's class-ordered moments)
    const int ldms = soft && P->p >= kSoftSymOrder && P->p <= kSoftSymMaxOrder ? soft_sym_ld(P->p) : 0;
    if ((unsigned long long)(nb + 1) * (unsigned long long)ldms * 8ULL >= (1ULL << 32))
        return fail(FMM_EUNSUPPORTED, "too many boxes for this order (class-ordered moments reach 4 GiB)");
    // ---- phase B: boxes, list counts, work lists (sizes known from nb)
    {
        Sizer o;
        o.add<int32_t>(nb).add<int32_t>(nb).add<int32_t>(nb).add<int32_t>(nb).add<int32_t>(nb).add<int32_t>(nb)
         .add<uint64_t>(nb).add<int32_t>(kMaxDepth + 2);
        for (int w = 0; w < 4; ++w) o.add<int64_t>(nb + 1);
        o.add<int32_t>((size_t)nb * kVSlots).add<int32_t>(nb).add<int32_t>(nb).add<int32_t>(nb)
         .add<int32_t>(kMaxDepth + 2).add<PlanView>(1)
         .add<double>((size_t)nb * P->ldm).add<double>((size_t)nb * P->ldm);
        if (soft) {
            o.add<int>(soft_table_ldc(P->p)).add<double>(P->ldm);
            if (ldms) o.add<double>((size_t)(nb + 1) * ldms);
        } else {
            o.add<double>((size_t)(nb + 1) * P->ldmh).add<double>((size_t)nb * P->ldh);
            if (P->m2l_parts > 1 && !sym_parts_add(P->p)) o.add<double>((size_t)(P->m2l_parts - 1) * nb * P->ldh);
            if (P->mixed_m2l && m2l_f32_operands(P->p)) o.add<float>((size_t)(nb + 1) * P->ldmh);
        }
        if (!P->reserve(true, o.total)) return fail(FMM_ENOMEM, "device allocation failed (boxes)");
        Sizer t;
        if (adaptive)
            t.add<uint64_t>(nb).add<int32_t>(nb).add<uint64_t>(nb).add<int32_t>(nb).add<int32_t>(nb).add<int32_t>(nb)
             .add<uint64_t>(nb).add<int32_t>(sort_scratch_bytes(nb) / 4 + 1);
        t.add<int32_t>(27ull * nb).add<int32_t>(nb);
        for (int w = 0; w < 8; ++w) t.add<int64_t>(nb + 1);
        for (int w = 0; w < 4; ++w) t.add<int64_t>(nb + 1);
        t.add<int64_t>(scan_multi_scratch_bytes(nb, 8) / 8 + 1).add<int32_t>(nb).add<PlanSizes>(1);
        if (!P->reserve(false, t.total)) return fail(FMM_ENOMEM, "device allocation failed (lists)");
    }
    BoxArrays bx{};
    bx.level = P->own<int32_t>(nb); bx.first = P->own<int32_t>(nb); bx.count = P->own<int32_t>(nb);
    bx.parent = P->own<int32_t>(nb); bx.child_begin = P->own<int32_t>(nb); bx.nchild = P->own<int32_t>(nb);
    bx.morton = P->own<uint64_t>(nb);
    int32_t *lvl_dev = P->lvl_dev = P->own<int32_t>(kMaxDepth + 2);
    if (!(bx.level && bx.first && bx.count && bx.parent && bx.child_begin && bx.nchild && bx.morton && lvl_dev))
        return fail(FMM_ENOMEM, "device allocation failed (boxes)");
    P->bx = bx;
    for (int w = 0; w < 4; ++w) { P->off[w] = P->own<int64_t>(nb + 1); NOMEM(P->off[w]); }
    int32_t *vslot = P->own<int32_t>((size_t)nb * kVSlots);
    int32_t *leaves = P->own<int32_t>(nb), *nonleaf = P->own<int32_t>(nb), *xtgt = P->own<int32_t>(nb);
    int32_t *lnl_off = P->own<int32_t>(kMaxDepth + 2);
    P->view_dev = P->own<PlanView>(1);
    double *M = P->own<double>((size_t)nb * P->ldm), *L = P->own<double>((size_t)nb * P->ldm);
    // folded multipoles: one row per box and an all-zero row after them
    // (Coulomb kernel; the softened kernel has its tables instead)
    double *Mh = soft ? nullptr : P->own<double>((size_t)(nb + 1) * P->ldmh);
    double *Lh = soft ? nullptr : P->own<double>((size_t)nb * P->ldh);
    float *Mhf = P->mixed_m2l && m2l_f32_operands(P->p) ? P->own<float>((size_t)(nb + 1) * P->ldmh) : nullptr;
    // orders >= 12: partial sums of the M2L class parts after the first
    const bool lh2 = P->m2l_parts > 1 && !sym_parts_add(P->p);
    double *Lh2 = lh2 ? P->own<double>((size_t)(P->m2l_parts - 1) * nb * P->ldh) : nullptr;
    if (lh2) NOMEM(Lh2);
    double *Dsoft = nullptr, *zrow = nullptr;
    int *soft_map = nullptr;
    if (soft) {
        soft_map = P->own<int>(soft_table_ldc(P->p));
        zrow = P->own<double>(P->ldm);
        NOMEM(soft_map); NOMEM(zrow);
        if (ldms) { // class-ordered moments of the sign-class M2L (in the folded multipoles' place)
            Mh = P->own<double>((size_t)(nb + 1) * ldms);
            NOMEM(Mh);
        }
    } else {
        NOMEM(Mh); NOMEM(Lh);
    }
    NOMEM(vslot); NOMEM(leaves); NOMEM(nonleaf); NOMEM(xtgt); NOMEM(lnl_off); NOMEM(P->view_dev);
    NOMEM(M); NOMEM(L);
    if (P->mixed_m2l && m2l_f32_operands(P->p)) NOMEM(Mhf);
    if (adaptive) {
        uint64_t *elevel = P->temp<uint64_t>(nb), *etk = P->temp<uint64_t>(nb), *emorton = P->temp<uint64_t>(nb);
        int32_t *eidx = P->temp<int32_t>(nb), *etv = P->temp<int32_t>(nb);
        int32_t *efirst = P->temp<int32_t>(nb), *ecount = P->temp<int32_t>(nb);
        int32_t *escr = P->temp<int32_t>(sort_scratch_bytes(nb) / 4 + 1);
        NOMEM(elevel); NOMEM(etk); NOMEM(emorton); NOMEM(eidx); NOMEM(etv); NOMEM(efirst); NOMEM(ecount); NOMEM(escr);
        adaptive_boxes(keys, n, P->D, P->leaf_size, eoff, nb, elevel, eidx, etk, etv, efirst, ecount, emorton,
                       escr, bx, lvl_dev, s);
    } else {
        uniform_boxes(keys, n, P->D, nb, bx, lvl_dev, s);
    }
    int32_t *leafcol = P->uniform ? nullptr : P->temp<int32_t>(nb);
    TreeArgs ta{bx, lvl_dev, P->D, nb, P->uniform, leafcol};
    int32_t *coll = P->temp<int32_t>(27ull * nb);
    int64_t *cnt[4], *flg[4], *pos[4];
    for (int w = 0; w < 4; ++w) { cnt[w] = P->temp<int64_t>(nb + 1); NOMEM(cnt[w]); }
    for (int w = 0; w < 4; ++w) { flg[w] = P->temp<int64_t>(nb + 1); pos[w] = P->temp<int64_t>(nb + 1); NOMEM(flg[w]); NOMEM(pos[w]); }
    int64_t *mscr = P->temp<int64_t>(scan_multi_scratch_bytes(nb, 8) / 8 + 1);
    int32_t *mtg = P->temp<int32_t>(nb);
    PlanSizes *sizes_dev = P->temp<PlanSizes>(1);
    NOMEM(coll); NOMEM(mscr); NOMEM(mtg); NOMEM(sizes_dev);
    if (P->uniform) { // lists straight from the cell coordinates
        ulist_uniform(ta, 0, cnt[0], cnt[2], cnt[3], nullptr, nullptr, s); // U counts, empty W and X
        vslot_uniform(ta, cnt[1], vslot, s); // V counts and whole M2L slot rows
    } else {
        NOMEM(leafcol);
        colleagues(ta, coll, cnt[3], leafcol, s); // also clears the X counts
        fill_i32(vslot, (int64_t)nb * kVSlots, -1, s);
        vlist(ta, coll, 0, cnt[1], nullptr, nullptr, vslot, s); // V counts and M2L slot rows
        uwlist(ta, coll, 0, cnt[0], nullptr, nullptr, cnt[2], nullptr, nullptr, cnt[3], s);
    }
    flags(bx, nb, cnt[3], cnt[1], flg[0], flg[1], flg[2], flg[3], s);
    {
        const int64_t *in[8] = {cnt[0], cnt[1], cnt[2], cnt[3], flg[0], flg[1], flg[2], flg[3]};
        int64_t *out[8] = {P->off[0], P->off[1], P->off[2], P->off[3], pos[0], pos[1], pos[2], pos[3]};
        scan_exclusive_multi(in, out, 8, nb, mscr, s);
    }
    compact(flg[0], pos[0], nb, leaves, s);
    compact(flg[1], pos[1], nb, nonleaf, s);
    compact(flg[2], pos[2], nb, xtgt, s);
    compact(flg[3], pos[3], nb, mtg, s);
    k_collect_sizes<<<1, 64, 0, s>>>(P->off[0], P->off[1], P->off[2], P->off[3], pos[0], pos[1], pos[2], pos[3],
                                     lvl_dev, root_dev, bad, nb, sizes_dev, lnl_off);
    HIPCHK(hipGetLastError());
    if (copy_to_host(&P->sizes, sizes_dev, 1, s)) return FMM_EDEVICE;
    HIPCHK(hipStreamSynchronize(s));
    const PlanSizes &Z = P->sizes;
    if (Z.bad) return fail(FMM_EINVAL, "non-finite coordinates");
    for (int k = 0; k < 4; ++k) P->root[k] = Z.root[k];
    int depth = 0;
    while (depth + 1 <= kMaxDepth && Z.lvl_begin[depth + 1] < nb) ++depth;
    P->depth = depth;
    P->lvl_begin.assign(Z.lvl_begin, Z.lvl_begin + depth + 2);
    P->lvl_nonleaf_off.assign(depth + 2, 0);
    for (int l = 0; l <= depth + 1; ++l) P->lvl_nonleaf_off[l] = (int)Z.lnl[l];
    for (int w = 0; w < 4; ++w) P->nlist[w] = Z.tot[w];
    if (Z.tot[2] != Z.tot[3]) return fail(FMM_EDEVICE, "X list size mismatch");
    P->nleaves = (int)Z.nleaves;
    P->nxtgt = (int)Z.nxtgt;
    const int nt = (int)Z.nmtg;
    // ---- phase C: list contents and M2L tiles (sizes known)
    int64_t slot_cap = ((int64_t)nt + 8 * (kM2LSlots - 1) + kM2LSlots - 1) / kM2LSlots * kM2LSlots;
    if (slot_cap < kM2LSlots) slot_cap = kM2LSlots;
    const int64_t mw = P->nlist[2];
    {
        Sizer o;
        for (int w = 0; w < 4; ++w)
            if (w != 1) o.add<int32_t>(P->nlist[w] ? P->nlist[w] : 1);
        o.add<int32_t>(slot_cap);
        if (!P->reserve(true, o.total)) return fail(FMM_ENOMEM, "device allocation failed (list arrays)");
        Sizer t;
        if (mw > 0) t.add<uint64_t>(mw).add<uint64_t>(mw).add<int32_t>(mw).add<int32_t>(sort_scratch_bytes((int)mw) / 4 + 1);
        t.add<int>(32).add<uint64_t>(nt + 1).add<uint64_t>(nt + 1).add<int32_t>(nt + 1).add<int32_t>(nt + 1)
         .add<int32_t>(sort_scratch_bytes(nt + 1) / 4 + 1);
        if (!P->reserve(false, t.total)) return fail(FMM_ENOMEM, "device allocation failed (list temporaries)");
    }
    for (int w = 0; w < 4; ++w) { // the V list itself is built on demand (export); M2L uses the slot rows
        if (w == 1) continue;
        P->src[w] = P->own<int32_t>(P->nlist[w] ? P->nlist[w] : 1);
        NOMEM(P->src[w]);
    }
    int32_t *slots = P->own<int32_t>(slot_cap);
    NOMEM(slots);
    if (P->uniform) ulist_uniform(ta, 1, nullptr, nullptr, nullptr, P->off[0], P->src[0], s);
    else uwlist(ta, coll, 1, nullptr, P->off[0], P->src[0], nullptr, P->off[2], P->src[2], nullptr, s);
    if (mw > 0) { // X = transpose of W
        uint64_t *wk = P->temp<uint64_t>(mw), *wk2 = P->temp<uint64_t>(mw);
        int32_t *wv2 = P->temp<int32_t>(mw), *wscr = P->temp<int32_t>(sort_scratch_bytes((int)mw) / 4 + 1);
        NOMEM(wk); NOMEM(wk2); NOMEM(wv2); NOMEM(wscr);
        w_pairs(P->off[2], P->src[2], nb, wk, P->src[3], s);
        int bits = 1;
        while ((1LL << bits) < nb) ++bits;
        radix_sort_pairs(wk, P->src[3], wk2, wv2, (int)mw, bits, wscr, s);
        // M2P sources: their full multipoles are rebuilt from the folded ones
        P->wsrc = P->own<int32_t>(nb);
        NOMEM(P->wsrc);
        fill_i32(P->wsrc, nb, 0, s);
        mark(P->src[2], mw, P->wsrc, s);
    }
    int *octoff = P->temp<int>(128);
    uint64_t *okey = P->temp<uint64_t>(nt + 1), *otk = P->temp<uint64_t>(nt + 1);
    int32_t *oval = P->temp<int32_t>(nt + 1), *otv = P->temp<int32_t>(nt + 1);
    int32_t *oscr = P->temp<int32_t>(sort_scratch_bytes(nt + 1) / 4 + 1);
    NOMEM(octoff); NOMEM(okey); NOMEM(otk); NOMEM(oval); NOMEM(otv); NOMEM(oscr);
    m2l_tiles(bx, mtg, nt, P->uniform, okey, oval, otk, otv, oscr, octoff, slots, slot_cap, s);
    P->nslots = (int)slot_cap;

    PlanView &v = P->view;
    v.p = P->p; v.nc = P->nc; v.nh = P->nh; v.ldm = P->ldm; v.ldh = P->ldh; v.ldmh = P->ldmh;
    v.precision = P->precision; v.mixed_m2l = P->mixed_m2l; v.depth = P->depth; v.D = P->D;
    v.n = n; v.nboxes = nb; v.nleaves = P->nleaves; v.nxtgt = P->nxtgt; v.nslots = P->nslots;
    for (int k = 0; k < 3; ++k) v.lo[k] = P->root[k];
    v.W = P->root[3];
    v.level = bx.level; v.parent = bx.parent; v.child_begin = bx.child_begin;
    v.nchild = bx.nchild; v.first = bx.first; v.count = bx.count; v.morton = bx.morton;
    v.perm = P->perm; v.xs = xs; v.ys = ys; v.zs = zs;
    v.U_off = P->off[0]; v.V_off = P->off[1]; v.W_off = P->off[2]; v.X_off = P->off[3];
    v.U_src = P->src[0]; v.W_src = P->src[2]; v.X_src = P->src[3]; v.wsrc = P->wsrc;
    v.m2l_tgt = slots; v.vslot = vslot; v.leaves = leaves; v.xtgt = xtgt;
    v.lvl_nonleaf = nonleaf; v.lvl_nonleaf_off = lnl_off; v.tab = P->tab; v.rot = P->rot;
    // row `nb` of the folded multipoles is the all-zero operand of absent M2L
    // sources; it is never written by an evaluation
    if (Mh) launch_zero(Mh + (size_t)nb * P->ldmh, P->ldmh, s);
    if (Mhf) launch_zero_f32(Mhf + (size_t)nb * P->ldmh, P->ldmh, s);
    v.kernel = P->kernel;
    v.eps2 = P->eps * P->eps;
    if (soft) {
        // derivative tables of the levels 2..depth that have boxes
        const int soft_nlev = std::max(P->depth - 1, 0);
        Dsoft = P->own<double>((size_t)std::max(soft_nlev, 1) * 343 * soft_table_ldc(P->p));
        NOMEM(Dsoft);
        launch_zero(zrow, P->ldm, s);
        launch_soft_tables(P->p, soft_nlev, Dsoft, soft_map, P->root[3], P->eps, s);
    }
    v.Dsoft = Dsoft; v.soft_map = soft_map; v.zrow = zrow;
    v.qs = qs; v.M = M; v.Mh = Mh; v.Lh = Lh; v.Lh2 = Lh2; v.m2l_parts = P->m2l_parts; v.L = L; v.Mhf = Mhf; v.phi_near = pf; v.fld_near = ff;
    HIPCHK(hipMemcpyAsync(P->view_dev, &v, sizeof(PlanView), hipMemcpyHostToDevice, s));
    HIPCHK(hipGetLastError());
    P->release_temps();
    // no wait for the rest of the build: later work on this stream follows it,
    // work on other streams waits for this event
    HIPCHK(hipEventCreateWithFlags(&P->built, hipEventDisableTiming));
    HIPCHK(hipEventRecord(P->built, s));
    return 0;
}

int check_options(const fmm_options_t &o, int order, int leaf_size)
{
    if (o.uniform_depth < -1 || o.uniform_depth > kMaxUniformDepth)
        return fail(FMM_EINVAL, "uniform_depth must be -1 or 0..8");
    if (o.uniform_depth < 0 && (o.max_depth < 1 || o.max_depth > kMaxDepth))
        return fail(FMM_EINVAL, "max_depth must be 1..21");
    if (o.precision & ~FMM_MIXED) return fail(FMM_EINVAL, "bad precision");
    if (o.m2l_method != FMM_M2L_SIGN_CLASS && o.m2l_method != FMM_M2L_ROTATION)
        return fail(FMM_EINVAL, "bad m2l_method");
    if (o.kernel != FMM_KERNEL_COULOMB && o.kernel != FMM_KERNEL_SOFTENED) return fail(FMM_EINVAL, "bad kernel");
    if (o.kernel == FMM_KERNEL_SOFTENED) {
        if (!std::isfinite(o.softening) || o.softening < 0) return fail(FMM_EINVAL, "softening must be finite and >= 0");
        if (o.precision != FMM_FP64) return fail(FMM_EINVAL, "the softened kernel runs in FMM_FP64 only");
        if (o.m2l_method != FMM_M2L_SIGN_CLASS) return fail(FMM_EINVAL, "the softened kernel has one M2L method");
        if (order > kSoftMaxOrder) return fail(FMM_EINVAL, "the softened kernel supports orders 0..10");
    }
    if (o.uniform_depth < 0 && leaf_size < 1) return fail(FMM_EINVAL, "leaf_size must be >= 1");
    if (order < 0 || order > kMaxOrder) return fail(FMM_EINVAL, "order must be 0..16");
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
    P->ldm = pad16(P->nc); P->ldh = pad16(P->nh); P->ldmh = folded_ld(order);
    P->uniform = o.uniform_depth >= 0;
    P->D = P->uniform ? o.uniform_depth : o.max_depth;
    P->leaf_size = leaf_size;
    P->precision = o.precision;
    P->m2l_rot = o.m2l_method == FMM_M2L_ROTATION;
    P->kernel = o.kernel;
    P->eps = o.kernel == FMM_KERNEL_SOFTENED ? o.softening : 0.0;
    P->mixed_m2l = (!P->m2l_rot && (o.precision & FMM_M2L_F32) && (order <= 8 || order >= 12)) ? 1 : 0;
    if (P->m2l_rot) {
        P->rot = get_rotation_tables(order, err);
        if (!P->rot) { delete P; return fail(FMM_EDEVICE, err); }
    }
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
        if (P->built) (void)hipEventDestroy(P->built);
        delete P;
        g_err = msg;
        return rc;
    }
    *out = P;
    return FMM_OK;
}

extern "C" int fmm_plan_batch(int32_t count, const double *const *xyz_dev, const int64_t *n,
                              const int32_t *order, const int32_t *leaf_size, const fmm_options_t *opts,
                              const fmm_allocator_t *alloc, hipStream_t stream, int32_t threads,
                              fmm_plan_t *out)
{
    g_err.clear();
    if (count < 0 || (count > 0 && (!xyz_dev || !n || !order || !leaf_size || !out)))
        return fail(FMM_EINVAL, "bad batch arguments");
    if (count == 0) return FMM_OK;
    for (int i = 0; i < count; ++i) out[i] = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(FMM_EINVAL, "allocator without functions");
    for (int i = 0; i < count; ++i) { // everything checkable on the host, before any device call
        fmm_options_t o;
        fmm_default_options(&o);
        if (opts) o = opts[i];
        if (!xyz_dev[i]) return fail(FMM_EINVAL, "plan " + std::to_string(i) + ": null pointer argument");
        if (n[i] < 1 || n[i] >= (1LL << 31)) return fail(FMM_EINVAL, "plan " + std::to_string(i) + ": bad n");
        if (int rc = check_options(o, order[i], leaf_size[i])) {
            g_err = "plan " + std::to_string(i) + ": " + g_err;
            return rc;
        }
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    // work enqueued on the caller's stream before this call precedes the builds
    hipEvent_t ready = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ready, stream));
    int nthr = alloc ? 1 : std::max(1, std::min<int>(threads, count));
    std::atomic<int> next{0}, first_bad{count};
    std::vector<int> rcs(count, FMM_OK);
    std::vector<std::string> msgs(count);
    auto worker = [&](bool own_stream) {
        if (hipSetDevice(dev) != hipSuccess) return;
        hipStream_t ws = stream;
        hipEvent_t e1 = nullptr, e2 = nullptr; // (unused events of the pooled stream set)
        if (own_stream && side_acquire(dev, ws, e1, e2)) ws = stream;
        if (ws != stream) (void)hipStreamWaitEvent(ws, ready, 0);
        for (int i; (i = next.fetch_add(1)) < count;) {
            if (first_bad.load() < count) break;
            int rc = fmm_plan(xyz_dev[i], n[i], order[i], leaf_size[i], opts ? &opts[i] : nullptr, alloc, ws, &out[i]);
            if (rc) {
                rcs[i] = rc;
                msgs[i] = g_err;
                int cur = first_bad.load();
                while (i < cur && !first_bad.compare_exchange_weak(cur, i)) {}
                break;
            }
            // complete before it changes streams: later frees are ordered on the caller's stream
            if (ws != stream && hipStreamSynchronize(ws) != hipSuccess) {
                rcs[i] = FMM_EDEVICE;
                msgs[i] = "stream synchronisation failed";
                int cur = first_bad.load();
                while (i < cur && !first_bad.compare_exchange_weak(cur, i)) {}
                break;
            }
            out[i]->stream = stream;
        }
        if (ws != stream) side_release(dev, ws, e1, e2);
    };
    if (nthr == 1) {
        worker(false);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nthr; ++t) pool.emplace_back(worker, true);
        for (auto &t : pool) t.join();
    }
    (void)hipEventDestroy(ready);
    if (nthr == 1) HIPCHK(hipStreamSynchronize(stream)); // every plan complete on return
    int bad = first_bad.load();
    if (bad < count) {
        for (int i = 0; i < count; ++i)
            if (out[i]) { fmm_plan_destroy(out[i]); out[i] = nullptr; }
        return fail(rcs[bad] ? rcs[bad] : FMM_EDEVICE, "plan " + std::to_string(bad) + ": " + msgs[bad]);
    }
    return FMM_OK;
}

namespace {

struct StagePlan {
    // per-stage block counts of one plan
    int permute, p2m, fold, m2l, p2l, unfold, far, p2p[2];
};

StagePlan stage_blocks(const fmm_plan_s *P)
{
    StagePlan sp;
    sp.permute = (int)ceil_div(P->n, 256);
    sp.p2m = P->nleaves;
    sp.fold = (int)ceil_div(P->nleaves, 64);
    sp.m2l = P->nslots / kM2LSlots * (P->m2l_rot ? m2l_rot_blocks_per_tile(P->p) : P->m2l_parts);
    sp.p2l = P->nxtgt;
    sp.unfold = (int)ceil_div(P->nboxes, kRemapBoxes);
    sp.far = (int)ceil_div(P->nleaves, 2); // two leaves per block
    const int split = p2p_split(P->nleaves);
    sp.p2p[0] = (int)ceil_div(split, 4);
    sp.p2p[1] = (int)ceil_div(P->nleaves - split, 4);
    return sp;
}

int nonleaf_groups(const fmm_plan_s *P, int level)
{
    if (level < 0 || level > P->depth) return 0;
    int c = P->lvl_nonleaf_off[level + 1] - P->lvl_nonleaf_off[level];
    return (int)ceil_div(c, 16);
}
// blocks of the folded M2M at a level (16-parent groups x row-tile groups)
int m2m_blocks(const fmm_plan_s *P, int level)
{
    const int g = nonleaf_groups(P, level);
    return g * m2m_row_split(P->ldmh / 16, g);
}

// Brackets a stage with events when the (single) plan has timing on.
struct StageTimer {
    fmm_plan_s *P;
    hipStream_t s;
    fmm_plan_s::Rec cur{};
    bool on = false;
    StageTimer(fmm_plan_s *p, hipStream_t st) : P(p), s(st) {}
    void begin(int stage, hipStream_t on_stream)
    {
        s = on_stream;
        begin(stage);
    }
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
    // (no heap allocation here: the batched entry point without allocation
    // runs this too)
    StageTimer T(count == 1 ? P[0] : nullptr, s);
    // all plans are addressed by their index in V; a launch over a subset uses
    // a view array offset, so subsets must be contiguous runs of equal order
    auto sub = [&](int a, int b, auto fn) {
        Bases B{};
        B.n = b - a;
        B.b[0] = 0;
        for (int i = 0; i < b - a; ++i) B.b[i + 1] = B.b[i] + fn(P[a + i]);
        return B;
    };
    Bases Bp = sub(0, count, [](const fmm_plan_s *p) { return stage_blocks(p).permute; });
    T.begin(0);
    launch_permute_q(V, Bp, s);
    T.end();
    // P2P needs only the sorted charges.  Its first part runs on the side
    // stream next to P2M, M2M and fold; its second part next to the
    // downward pass (unfold, L2L).  M2L, which fills the GPU by itself, runs
    // alone: overlapping it with P2P slows it by about as much as it hides.
    fmm_plan_s *F = P[0];
    if (F->ensure_side()) return fail(FMM_EDEVICE, "side stream creation failed");
    StageTimer T2(count == 1 ? P[0] : nullptr, F->side);
    auto p2p_part = [&](int part) {
        T2.begin(9 + part);
        for (int mixed = 0; mixed <= 1; ++mixed) { // FP64 and mixed plans in separate launches
            for (int i = 0; i < count;) {
                if (((P[i]->precision & FMM_P2P_F32) != 0) != (mixed == 1)) { ++i; continue; }
                int j = i;
                while (j < count && ((P[j]->precision & FMM_P2P_F32) != 0) == (mixed == 1)) ++j;
                Bases Bq{};
                Bq.n = j - i;
                Bq.b[0] = 0;
                for (int t = 0; t < j - i; ++t) Bq.b[t + 1] = Bq.b[t] + stage_blocks(P[i + t]).p2p[part];
                launch_p2p(mixed, part, V + i, Bq, F->side);
                i = j;
            }
        }
        T2.end();
    };
    HIPCHK(hipEventRecord(F->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(F->side, F->ev_fork, 0));
    // Lh rows zeroed for the M2L class parts to add into (orders 6-11; the
    // M2L waits for the side stream's first part)
    launch_lh_zero(V, sub(0, count, [](const fmm_plan_s *p) {
        return p->m2l_parts > 1 && sym_parts_add(p->p) ? (int)ceil_div((int64_t)p->nboxes * p->ldh, 512) : 0; }), F->side);
    p2p_part(0);
    HIPCHK(hipEventRecord(F->ev_join, F->side));
    // runs of equal order (callers sort batches by order)
    struct Run { int first, second; };
    Run runs_buf[kMaxBatch];
    int nruns = 0;
    for (int i = 0; i < count;) {
        int j = i;
        while (j < count && P[j]->p == P[i]->p && P[j]->mixed_m2l == P[i]->mixed_m2l &&
               P[j]->m2l_rot == P[i]->m2l_rot)
            ++j;
        runs_buf[nruns++] = {i, j};
        i = j;
    }
    struct Runs {
        const Run *b, *e;
        const Run *begin() const { return b; }
        const Run *end() const { return e; }
    } runs{runs_buf, runs_buf + nruns};
    // raw moments of the leaves, then their folded multipoles (P2M and fold
    // in one map); the parents' folded multipoles follow from the M2M on the
    // folded components.  Full multipoles only for leaves M2P reads.
    T.begin(1);
    for (auto &r : runs)
        launch_p2m(P[r.first]->p, V + r.first,
                   sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).p2m; }), s);
    T.end();
    T.begin(3);
    for (auto &r : runs)
        launch_p2m_fold(P[r.first]->p, V + r.first,
                        sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).fold; }), s);
    T.end();
    int maxdepth = 0;
    for (int i = 0; i < count; ++i) maxdepth = std::max(maxdepth, P[i]->depth);
    T.begin(2);
    // Multipoles of levels 0 and 1 are never read by M2L (V lists start at
    // level 2) nor by M2P (W lists hold boxes of level >= 2), so the upward
    // pass stops at level 2; fmm_plan_export_expansions completes it on demand.
    for (auto &r : runs)
        for (int l = maxdepth - 1; l >= 2; --l)
            launch_m2mh(P[r.first]->p, V + r.first,
                        sub(r.first, r.second, [l](const fmm_plan_s *p) { return m2m_blocks(p, l); }), l, s);
    // parents' FP32 operands (mixed M2L) and full multipoles (M2P sources)
    for (auto &r : runs) {
        int mixed = 0, wl = 0;
        for (int i = r.first; i < r.second; ++i) { mixed |= P[i]->view.Mhf != nullptr; wl |= P[i]->nlist[2] > 0; }
        if (mixed || wl)
            launch_parent_mh(V + r.first,
                             sub(r.first, r.second, [](const fmm_plan_s *p) { return (int)ceil_div(p->nboxes, 4); }), wl, s);
    }
    T.end();
    // The M2L runs alone at every order: running P2L's moments, the second
    // P2P part and M2P beside it at p = 14 (where it keeps one wavefront per
    // SIMD) slowed it from 26.4 to 34.6 ms, more than they take.
    HIPCHK(hipStreamWaitEvent(s, F->ev_join, 0)); // first part of P2P done
    T.begin(4);
    for (auto &r : runs)
        if (P[r.first]->m2l_rot)
            launch_m2l_rot(P[r.first]->p, V + r.first,
                           sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).m2l; }), s);
        else
            launch_m2l(P[r.first]->p, P[r.first]->mixed_m2l, V + r.first,
                       sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).m2l; }), s);
    T.end();
    HIPCHK(hipEventRecord(F->ev_fork, s)); // second part of P2P next to the downward pass
    HIPCHK(hipStreamWaitEvent(F->side, F->ev_fork, 0));
    p2p_part(1);
    // M2P (W lists) adds into the near-field sums after P2P, next to the
    // downward pass; plans without W lists skip it
    {
        T2.begin(11);
        for (auto &r : runs) {
            int w = 0;
            for (int i = r.first; i < r.second; ++i) w += P[i]->nlist[2] > 0;
            if (w)
                launch_m2p(P[r.first]->p, V + r.first,
                           sub(r.first, r.second, [](const fmm_plan_s *p) { return p->nlist[2] > 0 ? p->nleaves : 0; }), F->side);
        }
        T2.end();
    }
    HIPCHK(hipEventRecord(F->ev_join, F->side));
    T.begin(5);
    for (auto &r : runs)
        launch_p2l(P[r.first]->p, V + r.first,
                   sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).p2l; }), s);
    for (auto &r : runs)
        launch_p2l_transform(V + r.first, sub(r.first, r.second, [](const fmm_plan_s *p) {
            return (int)ceil_div(p->nxtgt, 16) * (p->ldh / 16); }), s);
    // complete Lh rows of plans whose M2L stores them (zero where nothing
    // arrived, plus the second part of the sign classes from order 12)
    launch_lh_init(V, sub(0, count, [](const fmm_plan_s *p) {
        return p->m2l_parts > 1 && sym_parts_add(p->p) ? 0 : (int)ceil_div(p->nboxes, 4); }), s);
    T.end();
    // L2L on the harmonic components, then full local expansions at the leaves
    T.begin(7);
    for (auto &r : runs)
        for (int l = 2; l < maxdepth; ++l)
            launch_l2lh(P[r.first]->p, V + r.first,
                        sub(r.first, r.second, [l](const fmm_plan_s *p) { return nonleaf_groups(p, l) * (p->ldh / 16); }), l, s);
    T.end();
    T.begin(6);
    for (auto &r : runs)
        launch_unfold(P[r.first]->p, V + r.first,
                      sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).unfold; }), 1, s);
    T.end();
    // far field (L2P) plus the near field (P2P, M2P), written in the caller's order
    HIPCHK(hipStreamWaitEvent(s, F->ev_join, 0));
    T.begin(8);
    for (auto &r : runs)
        launch_far(P[r.first]->p, V + r.first,
                   sub(r.first, r.second, [](const fmm_plan_s *p) { return stage_blocks(p).far; }), s);
    T.end();
    HIPCHK(hipGetLastError());
    return 0;
}

// The softened kernel's pipeline (one plan).  P2P's first part runs on the
// side stream beside P2M and M2M, the M2L alone (it holds two wavefronts per
// SIMD and slows down by more than P2P takes when they share the GPU), the
// second part and M2P (W lists) beside P2L (X lists) and the L2L.  P2M raw
// moments -> moments, M2M by one-axis shifts, M2L on the full components with
// the level's tables, L2L by one-axis shifts, then L2P with the near field.
int run_soft(fmm_plan_s *P, hipStream_t s)
{
    const PlanView *V = P->view_dev;
    StageTimer T(P, s);
    auto one = [](int nblocks) {
        Bases B{};
        B.n = 1;
        B.b[0] = 0;
        B.b[1] = nblocks;
        return B;
    };
    const StagePlan sp = stage_blocks(P);
    T.begin(0);
    launch_permute_q(V, one(sp.permute), s);
    T.end();
    if (P->ensure_side()) return fail(FMM_EDEVICE, "side stream creation failed");
    StageTimer T2(P, P->side);
    auto p2p_part = [&](int part) {
        HIPCHK(hipEventRecord(P->ev_fork, s));
        HIPCHK(hipStreamWaitEvent(P->side, P->ev_fork, 0));
        T2.begin(9 + part);
        launch_p2p(2, part, V, one(sp.p2p[part]), P->side);
        T2.end();
        if (part == 1 && P->nlist[2] > 0) { // M2P adds into the near-field sums
            T2.begin(11);
            launch_soft_m2p(P->p, V, P->nleaves, P->side);
            T2.end();
        }
        HIPCHK(hipEventRecord(P->ev_join, P->side));
        return 0;
    };
    if (p2p_part(0)) return FMM_EDEVICE;
    const int depth = P->depth;
    auto lb = [&](int l) { return P->lvl_begin[l]; };
    T.begin(1);
    launch_p2m(P->p, V, one(sp.p2m), s);
    launch_soft_p2m(P->p, V, P->nleaves, P->ldm, s);
    // M2L writes the rows of its targets, P2L and L2L add: start from zero
    launch_zero(P->view.L, (int64_t)P->nboxes * P->ldm, s);
    T.end();
    T.begin(2);
    for (int l = depth - 1; l >= 2; --l) launch_soft_m2m(P->p, V, lb(l), lb(l + 1) - lb(l), s);
    T.end();
    HIPCHK(hipStreamWaitEvent(s, P->ev_join, 0)); // first P2P part done
    T.begin(4);
    {
        SoftGrid G{};
        if (P->uniform) {
            G.nlev = std::max(depth - 1, 0);
            for (int i = 0; i < G.nlev; ++i) {
                const int l = i + 2;
                const long long cells = 1ll << (3 * (l - 1));
                G.tiles[i] = (int)((cells + 63) / 64);
                G.start[i] = G.nblocks;
                G.lvl_first[i] = lb(l);
                G.nblocks += 8 * G.tiles[i];
            }
        } else {
            G.adaptive = 1;
            G.nblocks = P->nslots / kM2LSlots;
        }
        launch_m2l_soft(P->p, V, G, P->view.Mh, P->nboxes, s);
    }
    T.end();
    if (p2p_part(1)) return FMM_EDEVICE;
    T.begin(5);
    launch_soft_p2l(P->p, V, P->nxtgt, s);
    T.end();
    T.begin(7);
    for (int l = 2; l < depth; ++l) launch_soft_l2l(P->p, V, lb(l + 1), lb(l + 2) - lb(l + 1), s);
    T.end();
    HIPCHK(hipStreamWaitEvent(s, P->ev_join, 0));
    T.begin(8);
    launch_far(P->p, V, one(sp.far), s);
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
    if (stream != P->stream) HIPCHK(hipStreamWaitEvent(stream, P->built, 0));
    PlanView v = P->view;
    v.q_in = q_dev;
    v.phi_out = phi_dev;
    v.fld_out = field_dev;
    HIPCHK(hipMemcpyAsync(P->view_dev, &v, sizeof(PlanView), hipMemcpyHostToDevice, stream));
    fmm_plan_s *arr[1] = {P};
    int rc = P->kernel == FMM_KERNEL_SOFTENED ? run_soft(P, stream) : run_pipeline(arr, 1, P->view_dev, stream);
    if (rc) return rc;
    if (P->note_use(stream)) return fail(FMM_EDEVICE, "event record failed");
    return FMM_OK;
}

namespace fmm {

int set_error(int code, const std::string &msg) { return fail(code, msg); }

// Checks a batch, makes `stream` wait for the plans' builds and fills idx[]
// with the plans ordered by (order, FP32 M2L, position), so that equal orders
// are contiguous.  No heap allocation.
int batch_prepare(fmm_plan_t const *plans, const double *const *q_dev, double *const *phi_dev, int32_t count,
                  hipStream_t stream, int *idx)
{
    if (count < 0 || (count > 0 && (!plans || !q_dev || !phi_dev)))
        return fail(FMM_EINVAL, "bad batch arguments");
    for (int i = 0; i < count; ++i)
        if (!plans[i] || !q_dev[i] || !phi_dev[i]) return fail(FMM_EINVAL, "null entry in batch");
    for (int i = 0; i < count; ++i)
        if (plans[i]->kernel != FMM_KERNEL_COULOMB)
            return fail(FMM_EINVAL, "batched evaluation runs Coulomb-kernel plans only (softened plans: fmm_evaluate)");
    for (int i = 0; i < count; ++i)
        if (stream != plans[i]->stream) HIPCHK(hipStreamWaitEvent(stream, plans[i]->built, 0));
    for (int i = 0; i < count; ++i) idx[i] = i;
    std::sort(idx, idx + count, [&](int a, int b) {
        if (plans[a]->p != plans[b]->p) return plans[a]->p < plans[b]->p;
        if (plans[a]->mixed_m2l != plans[b]->mixed_m2l) return plans[a]->mixed_m2l < plans[b]->mixed_m2l;
        if (plans[a]->m2l_rot != plans[b]->m2l_rot) return plans[a]->m2l_rot < plans[b]->m2l_rot;
        return a < b;
    });
    return 0;
}

// Runs the plans idx[c0..c1) (c1 - c0 <= kMaxBatch) with their views staged in
// the device array Vd.  No heap allocation (the views are built on the stack
// and copied on `stream`).
int batch_chunk(fmm_plan_t const *plans, const int *idx, int c0, int c1, const double *const *q_dev,
                double *const *phi_dev, double *const *field_dev, hipStream_t stream, PlanView *Vd)
{
    fmm_plan_s *P[kMaxBatch];
    PlanView views[kMaxBatch];
    const int m = c1 - c0;
    for (int t = 0; t < m; ++t) {
        const int i = idx[c0 + t];
        P[t] = plans[i];
        views[t] = plans[i]->view;
        views[t].q_in = q_dev[i];
        views[t].phi_out = phi_dev[i];
        views[t].fld_out = field_dev ? field_dev[i] : nullptr;
    }
    HIPCHK(hipMemcpyAsync(Vd, views, sizeof(PlanView) * m, hipMemcpyHostToDevice, stream));
    return run_pipeline(P, m, Vd, stream);
}

int batch_note_use(fmm_plan_t const *plans, int32_t count, hipStream_t stream)
{
    for (int i = 0; i < count; ++i)
        if (plans[i]->note_use(stream)) return fail(FMM_EDEVICE, "event record failed");
    return FMM_OK;
}

int plan_device(fmm_plan_t plan) { return plan->device; }

} // namespace fmm

extern "C" int fmm_evaluate_batch(fmm_plan_t const *plans, const double *const *q_dev,
                                  double *const *phi_dev, double *const *field_dev, int32_t count,
                                  hipStream_t stream)
{
    g_err.clear();
    if (count == 0) return FMM_OK;
    std::vector<int> idx(count > 0 ? count : 0);
    if (int rc = batch_prepare(plans, q_dev, phi_dev, count, stream, idx.data())) return rc;
    for (int c0 = 0; c0 < count; c0 += kMaxBatch) {
        const int c1 = std::min(count, c0 + kMaxBatch);
        PlanView *Vd = nullptr;
        HIPCHK(hipMallocAsync((void **)&Vd, sizeof(PlanView) * (c1 - c0), stream));
        int rc = batch_chunk(plans, idx.data(), c0, c1, q_dev, phi_dev, field_dev, stream, Vd);
        (void)hipFreeAsync(Vd, stream);
        if (rc) return rc;
    }
    return batch_note_use(plans, count, stream);
}

extern "C" int fmm_plan_footprint(fmm_plan_t plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(FMM_EINVAL, "null pointer argument");
    *bytes = plan->footprint;
    return FMM_OK;
}

extern "C" int fmm_cached_bytes(int device, size_t *bytes)
{
    if (!bytes) return fail(FMM_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache_total.find(device);
    *bytes = it == g_cache_total.end() ? 0 : it->second;
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
    double ldm = pad16(ncoef(order)), ldh = pad16(nharm(order)), ldmh = folded_ld(order);
    const int parts = sym_parts_add(order) ? 1 : sym_m2l_parts(order);
    double per_box = 8 * (2 * ldm + parts * ldh + ldmh) + 4 * ldmh + 4 * 200 + 64; // expansions, slots, lists
    double per_particle = 8 * 3 + 4 + 8 * 5 + 8 * 2;
    double total = boxes * per_box + n * per_particle + 8 * 27 * boxes;
    const int depth = o.uniform_depth >= 0 ? o.uniform_depth : o.max_depth;
    if (o.kernel == FMM_KERNEL_SOFTENED && depth >= 2 && order <= kSoftMaxOrder)
        total += 8.0 * (depth - 1) * 343 * soft_table_ldc(order); // derivative tables per level (at most)
    if (o.kernel == FMM_KERNEL_SOFTENED && order >= kSoftSymOrder && order <= kSoftSymMaxOrder)
        total += boxes * 8.0 * (soft_sym_ld(order) - ldmh); // class-ordered moments instead of folded ones
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
    HIPCHK(hipEventSynchronize(P->built));
    HIPCHK(hipStreamSynchronize(stream));
    const int nb = P->nboxes, n = P->n;
    if (!P->src[1]) { // the V list proper is built on first request (evaluation reads the slot rows)
        TreeArgs ta{P->bx, P->lvl_dev, P->D, nb, P->uniform};
        int32_t *coll = nullptr;
        HIPCHK(hipMalloc((void **)&coll, sizeof(int32_t) * 27 * (size_t)nb));
        int32_t *v1 = P->own<int32_t>(P->nlist[1] ? P->nlist[1] : 1);
        if (!v1) { (void)hipFree(coll); return fail(FMM_ENOMEM, "device allocation failed (V list)"); }
        colleagues(ta, coll, nullptr, nullptr, P->stream);
        vlist(ta, coll, 1, nullptr, P->off[1], v1, nullptr, P->stream);
        hipError_t e1 = hipStreamSynchronize(P->stream);
        (void)hipFree(coll);
        if (e1 != hipSuccess) return fail(FMM_EDEVICE, std::string("V list: ") + hipGetErrorString(e1));
        P->src[1] = v1;
    }
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
    HIPCHK(hipEventSynchronize(P->built));
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
        // The evaluation keeps the multipoles folded (leaves: written by the
        // folded P2M, parents: by the folded M2M) and stops at level 2.
        // Levels 1 and 0 are completed with the same folded M2M, then every
        // box's full multipole is rebuilt from its folded one by the
        // per-degree harmonic reconstruction, which is exact for harmonic
        // expansions: the exported multipoles are the evaluation's own P2M and
        // M2M results, not a separate computation.
        const bool soft = P->kernel == FMM_KERNEL_SOFTENED;
        Bases B{};
        B.n = 1;
        B.b[0] = 0;
        for (int l = std::min(P->depth - 1, 1); l >= 0; --l) {
            if (soft) {
                launch_soft_m2m(P->p, P->view_dev, P->lvl_begin[l], P->lvl_begin[l + 1] - P->lvl_begin[l], stream);
                continue;
            }
            B.b[1] = m2m_blocks(P, l);
            launch_m2mh(P->p, P->view_dev, B, l, stream);
        }
        if (!soft) {
            B.b[1] = (int)ceil_div(P->nboxes, 4);
            launch_parent_mh(P->view_dev, B, 2, stream); // leaves too: from the folded P2M
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(hipMemcpy(buf.data(), P->view.M, 8ull * nb * ldm, hipMemcpyDeviceToHost));
        // Coulomb: Mhat_a = w_|a| M_a / h^|a|; softened: moments Mhat_a = M_a / h^|a|
        for (int b = 0; b < nb; ++b) {
            double h = P->root[3] / std::ldexp(1.0, lev[b]);
            for (int a = 0; a < nc; ++a)
                M_host[(size_t)b * nc + a] = buf[(size_t)b * ldm + a] * (soft ? 1.0 : inv_w[deg[a]]) * std::pow(h, deg[a]);
        }
    }
    if (L_host) {
        // the evaluation unfolds leaves only: complete the full expansions of
        // every box (softened kernel: L holds the full expansions already)
        if (P->kernel == FMM_KERNEL_COULOMB) {
            Bases B{};
            B.n = 1;
            B.b[0] = 0;
            B.b[1] = stage_blocks(P).unfold;
            launch_unfold(P->p, P->view_dev, B, 0, stream);
        }
        HIPCHK(hipStreamSynchronize(stream));
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
    for (auto &u : plan->uses) {
        (void)hipStreamWaitEvent(plan->stream, u.second, 0);
        (void)hipEventDestroy(u.second);
    }
    plan->uses.clear();
    plan->release_all();
    plan->release_side();
    if (plan->built) (void)hipEventDestroy(plan->built);
    if (dev != plan->device) (void)hipSetDevice(dev);
    delete plan;
    return FMM_OK;
}
