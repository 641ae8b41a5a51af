// M2L target tiles: which 64 targets each M2L block takes, and in which
// order the blocks are laid out over the XCDs.  Kept apart from the tree and
// list kernels because the M2L kernels' memory traffic depends on it.
#include "tree_kernels.h"
#include "sort.h"

namespace fmm {

// ---------------- M2L target tiles ----------------
// Targets (boxes with a V list, ascending) are stably sorted by octant, then
// each octant group is placed at a multiple of 64 so that the 64 targets of
// one M2L block share one set of 189 offsets.  In a uniform tree the offsets a
// box actually has depend only on its octant and on its distance (0, 1, 2 or
// more cells) to each face of the root, so there the targets are also grouped
// by these distances (Morton order inside a group): the blocks near the faces
// then skip the offsets none of their targets has.  The tiles are then laid
// out region by region: the x-th eighth of every octant's tiles (a spatial
// region, as the tiles follow Morton order) forms the x-th eighth of the
// sequence, which the M2L launch hands to XCD x, so each XCD's L2 holds the
// multipoles of one region instead of those of the whole domain.  Inside a
// region the eight octants' tiles are dealt round-robin, so the blocks that
// run at the same time hold the children of the same parents, whose V lists
// draw on the same source boxes.
constexpr int kCatBits = 12;

__global__ __launch_bounds__(256) void k_oct_keys(const BoxArrays bx, const int32_t *tg, int nt, int uniform,
                                                  uint64_t *key, int32_t *val)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nt) return;
    const int b = tg[i];
    uint64_t cat = 0;
    if (uniform) {
        const int l = bx.level[b], side = 1 << l;
        int c[3];
        deinterleave(bx.morton[b], l, c);
        for (int k = 0; k < 3; ++k) {
            const int lo = c[k] < 3 ? c[k] : 3, hi = side - 1 - c[k] < 3 ? side - 1 - c[k] : 3;
            cat |= (uint64_t)(lo * 4 + hi) << (4 * k);
        }
    }
    key[i] = ((bx.morton[b] & 7) << kCatBits) | cat;
    val[i] = b;
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
            if ((key[mid] >> kCatBits) < (uint64_t)o) lo = mid + 1; else hi = mid;
        }
        st[o] = o == 8 ? nt : lo;
    }
    __syncthreads();
    if (o == 0) {
        int s = 0;
        for (int k = 0; k < 8; ++k) {
            octoff[k] = s;              // padded start
            octoff[9 + k] = st[k];      // unpadded start
            octoff[96 + k] = (st[k + 1] - st[k] + 63) / 64; // tiles of the octant
            s += (st[k + 1] - st[k] + 63) & ~63;
        }
        octoff[8] = s;
        octoff[17] = nt;
        // first tile of (region x, octant k) in the region-major sequence
        int t = 0;
        for (int x = 0; x < 8; ++x)
            for (int k = 0; k < 8; ++k) {
                const int T = octoff[96 + k];
                octoff[32 + 8 * x + k] = t;
                t += (x + 1) * T / 8 - x * T / 8;
            }
    }
}

__global__ __launch_bounds__(256) void k_oct_place(const uint64_t *key, const int32_t *val, int nt,
                                                   const int *octoff, int32_t *slots)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nt) return;
    const int o = (int)(key[i] >> kCatBits), j = i - octoff[9 + o], t = j >> 6, T = octoff[96 + o];
    int x = 0;
    while (x < 7 && t >= (x + 1) * T / 8) ++x;
    // within region x the octants' tiles are dealt round-robin: tile u of
    // octant o follows tile u of octants < o and precedes tile u + 1 of all
    const int u = t - x * T / 8;
    int pos = 0;
    for (int k = 0; k < 8; ++k) {
        const int n = (x + 1) * octoff[96 + k] / 8 - x * octoff[96 + k] / 8; // tiles of octant k in region x
        pos += min(n, u + (k < o ? 1 : 0));
    }
    const int tile = octoff[32 + 8 * x] + pos;
    slots[(int64_t)tile * 64 + (j & 63)] = val[i];
}

void m2l_tiles(const BoxArrays &bx, const int32_t *tg, int nt, int uniform, uint64_t *key, int32_t *val,
               uint64_t *tk, int32_t *tv, int32_t *sort_scratch, int *octoff, int32_t *slots,
               int64_t slot_cap, hipStream_t s)
{
    fill_i32(slots, slot_cap, -1, s);
    if (nt == 0) return;
    k_oct_keys<<<ceil_div(nt, 256), 256, 0, s>>>(bx, tg, nt, uniform, key, val);
    radix_sort_pairs(key, val, tk, tv, nt, kCatBits + 3, sort_scratch, s);
    k_oct_offsets<<<1, 64, 0, s>>>(key, nt, octoff);
    k_oct_place<<<ceil_div(nt, 256), 256, 0, s>>>(key, val, nt, octoff, slots);
}

} // namespace fmm
