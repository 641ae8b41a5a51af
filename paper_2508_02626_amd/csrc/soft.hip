// The softened Coulomb kernel K(x) = 1/sqrt(|x|^2 + eps^2): a second
// non-oscillatory kernel through the same tree, lists and pipeline (the DA
// formulation is not tied to 1/r; closing remark of Sec. 3.4).
//
// K is not harmonic, so there is no fold: the expansions are the full
// Cartesian Taylor ones.  In scaled units (h = box width, u = (x - c)/h):
//   Mhat_a = M_a / h^|a| = sum_i q_i (-u_i)^a / a!          (P2M: moments)
//   Lhat_b = b! h^(|b|+1) L_b,  phi(c + h u) = (1/h) sum_b Lhat_b u^b / b!
//   M2L  Lhat_b(B) = sum_a D_(a+b)(k) Mhat_a(C),  D_g(k) = d^g K_eta(k),
//        eta = eps / h: unlike 1/r the kernel is not homogeneous, so the
//        derivative tables depend on the level (one set per level)
//   M2M  Mhat_a(P) = sum_{b <= a} 2^-|b| Mhat_b(C) (-tau)^(a-b) / (a-b)!
//   L2L  Lhat_b(C) += 2^(-|b|-1) sum_{g >= b} Lhat_g(P) tau^(g-b) / (g-b)!
//        tau = (c_C - c_P) / h_P = (+-1/4, +-1/4, +-1/4)
// The shifts factor over the axes, so M2M and L2L run as three one-axis
// shifts (O(n_p p) per box instead of n_p^2).  K is even in every coordinate,
// so the M2L shares one contraction among the offsets that differ only in
// sign (orders 4-8).  P2L and M2P (adaptive trees) need K's Taylor
// coefficients at particles, one particle per lane.  The tables come from the
// Taylor recurrence of rho^(-1/2), rho = |x|^2 + eta^2:
//   n rho a_g + (2n - 1) sum_k x_k a_(g - e_k) + (n - 1) sum_k a_(g - 2e_k) = 0,
// a_g = d^g K / g! (degree n = |g|; eta = 0 gives the 1/r recurrence).
#include "ops.h"
#include "soft.h"

namespace fmm {

typedef double double4_t __attribute__((ext_vector_type(4)));
template <typename T> __device__ inline T gload(const T *p) { return *gptr(p); }

// exponents of the monomial at DA index e of degree n (mono_index inverse)
__device__ inline void mono_exps(int e, int n, int &i, int &j, int &k)
{
    int r = e - below(n), a = 0;
    while ((a + 1) * (a + 2) / 2 <= r) ++a;
    k = r - a * (a + 1) / 2;
    j = a - k;
    i = n - a;
}
__device__ inline double fact_d(int n)
{
    double r = 1.0;
    for (int t = 2; t <= n; ++t) r *= t;
    return r;
}

// LDS layout of one derivative table in the M2L: entry g at addr(g) = g_x SA +
// g_y SB + g_z, linear (so addr(a) + addr(b) = addr(a + b) and a product's
// operand is one gather) and one-to-one on the degrees |g| <= 2p the table
// holds; the padding entry of the compact rows goes to the slot after the
// largest address (2p SA).  Orders 0-3: the dense cube (SB = 2p + 1,
// SA = SB^2); orders 4-10: strides picked by a search over the sign-class tiles so
// that the 16 rows of a tile (with one column each) and the 32 lanes of two
// columns fall on as few common LDS banks as possible (with the cube's
// strides, both = 1 mod 16, the bank follows |a + b| mod 16 and a tile's rows
// share two or three banks).
template <int P> struct SoftCube {
    static constexpr int S = 2 * P + 1;
    static constexpr int SA = P == 4 ? 92 : P == 5 ? 100 : P == 6 ? 190 : P == 7 ? 267 : P == 8 ? 315
                            : P == 9 ? 395 : P == 10 ? 455 : S * S;
    static constexpr int SB = P == 4 ? 11 : P == 5 ? 22 : P == 6 ? 23 : P == 7 ? 18 : P == 8 ? 18
                            : P == 9 ? 26 : P == 10 ? 22 : S;
    static constexpr int SIZE = 2 * P * SA + 1, LDD = SIZE + 1; // addresses, and the padding slot
    __host__ __device__ static constexpr int addr(int i, int j, int k) { return i * SA + j * SB + k; }
    __device__ static int addr(int x) { return addr(x & 255, (x >> 8) & 255, x >> 16); }
    static constexpr bool one_to_one()
    {
        bool used[SIZE] = {};
        for (int i = 0; i <= 2 * P; ++i)
            for (int j = 0; i + j <= 2 * P; ++j)
                for (int k = 0; i + j + k <= 2 * P; ++k) {
                    const int a = addr(i, j, k);
                    if (a < 0 || a >= SIZE || used[a]) return false;
                    used[a] = true;
                }
        return true;
    }
    static_assert(P == 0 || (SB > 2 * P && SA > SB), "strides");
    static_assert(one_to_one(), "addresses one-to-one on the table's degrees");
};

// ---------------- derivative tables, one block per (level, offset) ----------------
template <int P>
__global__ __launch_bounds__(256) void k_soft_tables(double *D, int *map, int ldc, double W, double eps)
{
    constexpr int Q = 2 * P, NQ = ncoef(Q);
    __shared__ double a[NQ];
    const int lev = blockIdx.x / 343 + 2, off = blockIdx.x % 343;
    const int kx = off / 49 - 3, ky = (off / 7) % 7 - 3, kz = off % 7 - 3;
    double *out = D + (int64_t)blockIdx.x * ldc;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0)
        for (int e = tid; e < ldc; e += 256) {
            int n = 0, i = 0, j = 0, k = 0;
            if (e < NQ) {
                while (below(n + 1) <= e) ++n;
                mono_exps(e, n, i, j, k);
                map[e] = SoftCube<P>::addr(i, j, k);
            } else {
                map[e] = SoftCube<P>::SIZE; // the padding slot, never read
            }
        }
    // only V-list offsets (some |k_i| >= 2) are ever read
    if (max(abs(kx), max(abs(ky), abs(kz))) <= 1) {
        for (int e = tid; e < ldc; e += 256) out[e] = 0.0;
        return;
    }
    const double eta = eps * (double)(1ll << lev) / W;
    const double x[3] = {(double)kx, (double)ky, (double)kz};
    const double rho = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + eta * eta;
    if (tid == 0) a[0] = 1.0 / sqrt(rho);
    for (int n = 1; n <= Q; ++n) {
        __syncthreads();
        for (int e = below(n) + tid; e < below(n + 1); e += 256) {
            int g[3];
            mono_exps(e, n, g[0], g[1], g[2]);
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (g[d] >= 1) {
                    int h[3] = {g[0], g[1], g[2]};
                    h[d] -= 1;
                    s1 += x[d] * a[mono_index(h[0], h[1], h[2])];
                }
                if (g[d] >= 2) {
                    int h[3] = {g[0], g[1], g[2]};
                    h[d] -= 2;
                    s2 += a[mono_index(h[0], h[1], h[2])];
                }
            }
            a[e] = -((2 * n - 1) * s1 + (n - 1) * s2) / (n * rho);
        }
    }
    __syncthreads();
    for (int e = tid; e < ldc; e += 256) {
        double v = 0.0;
        if (e < NQ) {
            int n = 0, i, j, k;
            while (below(n + 1) <= e) ++n;
            mono_exps(e, n, i, j, k);
            v = a[e] * fact_d(i) * fact_d(j) * fact_d(k); // d^g K = g! a_g
        }
        out[e] = v;
    }
}

// ---------------- P2M: moments from the raw moments ----------------
// Raw moments Q_g = sum q u^g (k_p2m, in the leaf's L row) -> Mhat_a =
// (-1)^|a| Q_a / a! in its M row (padding columns zero).
template <int P>
__global__ __launch_bounds__(256) void k_soft_p2m(const PlanView *V)
{
    constexpr int NC = ncoef(P);
    const PlanView &v = V[0];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int ldm = v.ldm;
    if (e >= (int64_t)v.nleaves * ldm) return;
    const int li = (int)(e / ldm), a = (int)(e - (int64_t)li * ldm);
    const int box = v.leaves[li];
    double m = 0.0;
    if (a < NC) {
        int n = 0, i, j, k;
        while (below(n + 1) <= a) ++n;
        mono_exps(a, n, i, j, k);
        const double q = v.L[(int64_t)box * ldm + a] * v.tab->inv_fact[a];
        m = (n & 1) ? -q : q;
    }
    v.M[(int64_t)box * ldm + a] = m;
}

// Exponents of the coefficients a lane handles in the one-axis shifts
// (entries lane, lane + 64, ...): degree n, a = j + k and (i, j, k).
template <int P> struct ShiftLane {
    static constexpr int NC = ncoef(P), RC = (NC + 63) / 64;
    int n[RC], a[RC], e[RC][3];
    __device__ void init(int lane)
    {
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int g = lane + 64 * r;
            int nn = 0, i = 0, j = 0, k = 0;
            if (g < NC) {
                while (below(nn + 1) <= g) ++nn;
                mono_exps(g, nn, i, j, k);
            }
            n[r] = nn;
            a[r] = j + k;
            e[r][0] = i;
            e[r][1] = j;
            e[r][2] = k;
        }
    }
};

// one-axis shift of a vector of NC coefficients in LDS: out[g] = sum_m c[m] in[g -+ m e_D]
// (DIR = -1: lower indices, the moment shift, m <= g_D; DIR = +1: higher, the
// Taylor shift, m <= p - |g|).  The index of g -+ m e_D in the DA order is
// below(n') + a'(a' + 1)/2 + k' with n' = n -+ m and a', k' moved only on the
// axes they contain.
template <int P, int D, int DIR>
__device__ inline void axis_shift(const double *in, double *out, const double *c, const ShiftLane<P> &sl, int lane)
{
    constexpr int NC = ncoef(P), RC = ShiftLane<P>::RC;
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const int g = lane + 64 * r;
        if (g >= NC) continue;
        const int n = sl.n[r], a = sl.a[r], k = sl.e[r][2];
        const int top = DIR < 0 ? sl.e[r][D] : P - n;
        double s = 0.0;
        for (int m = 0; m <= top; ++m) {
            const int nm = n + DIR * m, am = D == 0 ? a : a + DIR * m, km = D == 2 ? k + DIR * m : k;
            s += c[m] * in[below(nm) + am * (am + 1) / 2 + km];
        }
        out[g] = s;
    }
}

// ---------------- M2M: one block per parent of `level`, one wavefront per child ----------------
// Each wavefront shifts one child (its own LDS vectors, three one-axis
// shifts); the parent's moments are the sum over the children in child order.
template <int P>
__global__ __launch_bounds__(512) void k_soft_m2m(const PlanView *V, int first_box)
{
    constexpr int NC = ncoef(P);
    __shared__ double s0[8][NC], s1[8][NC];
    __shared__ double cf[8][3][P + 1];
    const PlanView &v = V[0];
    const int box = first_box + blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63, ldm = v.ldm;
    const int nch = v.nchild[box], c0 = v.child_begin[box];
    if (nch == 0) return; // a leaf keeps its P2M multipole
    if (w < nch) {
        ShiftLane<P> sl;
        sl.init(lane);
        const int ch = c0 + w, o = (int)(v.morton[ch] & 7);
#pragma unroll
        for (int r = 0; r < ShiftLane<P>::RC; ++r) {
            const int g = lane + 64 * r;
            if (g < NC) s0[w][g] = v.M[(int64_t)ch * ldm + g] * ldexp(1.0, -sl.n[r]);
        }
        if (lane < 3 * (P + 1)) { // (-tau_d)^m / m!, tau_d = (2 o_d - 1) / 4
            const int d = lane / (P + 1), m = lane - d * (P + 1);
            const double t = -(2.0 * ((o >> (2 - d)) & 1) - 1.0) * 0.25;
            double pw = 1.0;
            for (int u = 0; u < m; ++u) pw *= t;
            cf[w][d][m] = pw / fact_d(m);
        }
        wave_sync();
        axis_shift<P, 0, -1>(s0[w], s1[w], cf[w][0], sl, lane);
        wave_sync();
        axis_shift<P, 1, -1>(s1[w], s0[w], cf[w][1], sl, lane);
        wave_sync();
        axis_shift<P, 2, -1>(s0[w], s1[w], cf[w][2], sl, lane);
    }
    __syncthreads();
    for (int g = tid; g < ldm; g += 512) {
        double val = 0.0;
        if (g < NC)
            for (int c = 0; c < nch; ++c) val += s1[c][g];
        v.M[(int64_t)box * ldm + g] = val;
    }
}

// ---------------- L2L: one block (one wavefront) per child of a box of `level` ----------------
template <int P>
__global__ __launch_bounds__(64) void k_soft_l2l(const PlanView *V, int first_child)
{
    constexpr int NC = ncoef(P), RC = ShiftLane<P>::RC;
    __shared__ double s0[NC], s1[NC];
    __shared__ double cf[3][P + 1];
    const PlanView &v = V[0];
    const int ch = first_child + blockIdx.x, lane = threadIdx.x, ldm = v.ldm;
    const int par = v.parent[ch], o = (int)(v.morton[ch] & 7);
    ShiftLane<P> sl;
    sl.init(lane);
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const int g = lane + 64 * r;
        if (g < NC) s0[g] = v.L[(int64_t)par * ldm + g];
    }
    if (lane < 3 * (P + 1)) { // tau_d^m / m!
        const int d = lane / (P + 1), m = lane - d * (P + 1);
        const double t = (2.0 * ((o >> (2 - d)) & 1) - 1.0) * 0.25;
        double pw = 1.0;
        for (int u = 0; u < m; ++u) pw *= t;
        cf[d][m] = pw / fact_d(m);
    }
    wave_sync();
    axis_shift<P, 0, 1>(s0, s1, cf[0], sl, lane);
    wave_sync();
    axis_shift<P, 1, 1>(s1, s0, cf[1], sl, lane);
    wave_sync();
    axis_shift<P, 2, 1>(s0, s1, cf[2], sl, lane);
    wave_sync();
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const int g = lane + 64 * r;
        if (g < NC) v.L[(int64_t)ch * ldm + g] += ldexp(s1[g], -sl.n[r] - 1);
    }
}

// The 64 targets of M2L tile `item` (-1 for an empty place): in a uniform
// tree boxes 8 (64 t + i) + o of one level (item -> level, octant, tile); in
// an adaptive tree the plan's target tile.  Blocks map to items through
// xcd_remap, each XCD taking a contiguous range.
__device__ inline void soft_tile_targets(const PlanView &v, const SoftGrid &G, int item, int tid, int *sTg)
{
    if (G.adaptive) {
        if (tid < 64) sTg[tid] = v.m2l_tgt[(int64_t)item * kM2LSlots + tid];
    } else {
        int li = 0;
        while (li + 1 < G.nlev && item >= G.start[li + 1]) ++li;
        item -= G.start[li];
        const int lev = li + 2, per = G.tiles[li], o = item / per, t = item - o * per;
        const int64_t cells = 1ll << (3 * (lev - 1)); // boxes of one octant at this level
        if (tid < 64) {
            const int64_t m = (int64_t)t * 64 + tid;
            sTg[tid] = m < cells ? G.lvl_first[li] + (int)(8 * m + o) : -1;
        }
    }
}

// Levels of the targets (sLv, -1 for empty places) and, in info, their level
// range and octant (info[1] < 0: no target).  sTg must be visible to the block.
__device__ inline void soft_tile_levels(const PlanView &v, int tid, const int *sTg, int *sLv, int *info)
{
    if (tid < 64) sLv[tid] = sTg[tid] >= 0 ? v.level[sTg[tid]] : -1;
    __syncthreads();
    if (tid == 0) {
        int lo = 1 << 30, hi = -1, oc = 0;
        for (int q = 0; q < 64; ++q)
            if (sTg[q] >= 0) {
                lo = min(lo, sLv[q]);
                hi = max(hi, sLv[q]);
                oc = (int)(v.morton[sTg[q]] & 7);
            }
        info[0] = lo;
        info[1] = hi;
        info[2] = oc;
    }
    __syncthreads();
}

// ---------------- M2L on the full components (FP64 MFMA) ----------------
// Per used offset slot each wavefront runs an n_p x n_p by 16 product with
// 16x16x4 MFMAs, as the slot-by-slot Coulomb M2L: A[b][a] = D(addr(b) +
// addr(a)) gathered from the slot's table in LDS (SoftCube: addr(a) + addr(b)
// = addr(a + b)); B the 16
// targets' source multipoles, one 16-byte vector (two k-steps) per lane, one
// vector ahead.  Tables are double-buffered in LDS (one barrier per slot).
// The 64 targets of a block share the 189 offsets of one octant: in a uniform
// tree 64 boxes of one level and octant (Morton index 8 (64 t + i) + o); in an
// adaptive tree the plan's M2L target tiles, whose targets are in level order
// within their octant, so that only the tiles at a level boundary hold two
// levels.  A block runs its levels one after the other with that level's
// tables; a target's operands are zero in the other levels' products.
template <int P> struct SoftM2L {
    static constexpr int NP = ncoef(P), MT = (NP + 15) / 16, KS = ((NP + 3) / 4 + 1) & ~1, KSV = KS / 2;
    static constexpr int LDD = SoftCube<P>::LDD, LDC = (ncoef(2 * P) + 1) & ~1;
};

template <int P>
__global__ __launch_bounds__(256) void k_m2l_soft(const PlanView *V, SoftGrid G)
{
    using SH = SoftM2L<P>;
    constexpr int NP = SH::NP, MT = SH::MT, KS = SH::KS, KSV = SH::KSV, LDD = SH::LDD, LDC = SH::LDC;
    constexpr int DV = (LDC / 2 + 255) / 256;
    static_assert(8 * KSV <= pad16(NP), "operand vectors stay inside a padded row");
    typedef double vec_t __attribute__((ext_vector_type(2)));
    __shared__ double sD[2][LDD];
    __shared__ int sHo[4][KS];
    __shared__ int sTg[64], sLv[64];
    __shared__ int sList[kVSlots];
    __shared__ int sN, sInfo[3];
    const PlanView &v = V[0];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
    const OrderTables &tb = *v.tab;
    soft_tile_targets(v, G, xcd_remap(blockIdx.x, G.nblocks), tid, sTg);
    for (int e = tid; e < 4 * KS; e += 256) {
        const int g = e / KS, ks = e - g * KS, a = 8 * (ks / 2) + 2 * g + (ks & 1);
        sHo[g][ks] = a < NP ? SoftCube<P>::addr(gptr(tb.exps)[a]) : 0;
    }
    int hb[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int b = 16 * mt + col;
        hb[mt] = b < NP ? SoftCube<P>::addr(gptr(tb.exps)[b]) : 0;
    }
    __syncthreads();
    soft_tile_levels(v, tid, sTg, sLv, sInfo);
    const int lmin = sInfo[0], lmax = sInfo[1], oct = sInfo[2];
    if (lmax < 0) return; // (block-uniform)
    const auto vs = gptr(v.vslot);
    const auto offs = gptr(tb.offs) + oct * kVSlots;
    const int tgt = sTg[wave * 16 + col], tlev = sLv[wave * 16 + col];
    typedef double dvec_t __attribute__((ext_vector_type(2)));
    dvec_t pd[DV];
    int dm[DV][2];
#pragma unroll
    for (int r = 0; r < DV; ++r)
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int e = (tid + 256 * r) * 2 + w;
            dm[r][w] = e < LDC ? gptr(v.soft_map)[e] : LDD - 1;
        }
    const int ldm = v.ldm;
    double4_t acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = double4_t{0, 0, 0, 0};
    for (int L = lmin; L <= lmax; ++L) {
        // slots used by the block's targets of level L, in increasing order
        if (tid < kVSlots) {
            int any = 0;
            for (int q = 0; q < 64; ++q) any |= sLv[q] == L && vs[(int64_t)sTg[q] * kVSlots + tid] >= 0;
            sList[tid] = any;
        }
        __syncthreads();
        if (tid == 0) {
            int n = 0;
            for (int j = 0; j < kVSlots; ++j)
                if (sList[j]) sList[n++] = j;
            sN = n;
        }
        __syncthreads();
        const int nslot = sN;
        const double *Dl = v.Dsoft + (int64_t)(L - 2) * 343 * LDC;
        auto load_d = [&](int j) {
            const dvec_t *Dk = (const dvec_t *)(Dl + (int64_t)offs[j] * LDC);
#pragma unroll
            for (int r = 0; r < DV; ++r) {
                const int e = tid + 256 * r;
                pd[r] = e < LDC / 2 ? gload(Dk + e) : dvec_t{0, 0};
            }
        };
        auto store_d = [&](int buf) {
#pragma unroll
            for (int r = 0; r < DV; ++r)
                if (tid + 256 * r < LDC / 2)
#pragma unroll
                    for (int w = 0; w < 2; ++w) sD[buf][dm[r][w]] = pd[r][w];
        };
        auto row_of = [&](int j) -> const double * {
            const int src = tgt >= 0 && tlev == L ? vs[(int64_t)tgt * kVSlots + j] : -1;
            return (src >= 0 ? v.M + (int64_t)src * ldm : v.zrow) + 2 * kq;
        };
        const double *rc = v.zrow, *rn = v.zrow;
        vec_t cur{0, 0}, nxt{0, 0};
        if (nslot > 0) {
            load_d(sList[0]);
            store_d(0);
            rc = row_of(sList[0]);
            cur = gload((const vec_t *)rc);
            __syncthreads();
        }
        for (int q = 0; q < nslot; ++q) {
            const int buf = q & 1;
            const bool more = q + 1 < nslot;
            if (more) {
                load_d(sList[q + 1]);
                rn = row_of(sList[q + 1]);
            }
            // the wavefront skips a slot none of its targets has
            const bool has = rc != v.zrow + 2 * kq;
            if (__ballot(has)) {
                const double *D = sD[buf];
#pragma unroll 1
                for (int jv = 0; jv < KSV; ++jv) {
                    nxt = jv + 1 < KSV ? gload((const vec_t *)(rc + 8 * (jv + 1))) : gload((const vec_t *)rn);
#pragma unroll
                    for (int w = 0; w < 2; ++w) {
                        const int ha = sHo[kq][2 * jv + w];
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
                            acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(D[hb[mt] + ha], cur[w], acc[mt], 0, 0, 0);
                    }
                    cur = nxt;
                }
            } else {
                cur = gload((const vec_t *)rn);
            }
            rc = rn;
            if (more) store_d(buf ^ 1);
            __syncthreads();
        }
    }
    if (tgt < 0) return;
    double *L = v.L + (int64_t)tgt * ldm;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = 16 * mt + 4 * r + kq;
            if (b < NP) L[b] = acc[mt][r];
        }
}

// ---------------- sign-class M2L (orders kSoftSymOrder .. kSoftSymMaxOrder) ----------------
// K_eta is even in every coordinate, so d^g K_eta(s o k) = s^g d^g K_eta(k)
// for a vector s of signs: the offsets that differ from a representative k
// only by signs (the members of its class) share k's table.  With rows b and
// columns a grouped by the parities pi(g) of their exponents (3 bits: x, y, z),
//   Lhat_b = sum_a D_(a+b)(k) H_(pi(a) ^ pi(b))[a],
//   H_s[a] = sum_m (-1)^|m & s| Mhat_a(source of member m),
// the Walsh-Hadamard transform over the members (m: the axes a member
// negates): one contraction per class instead of one per member.  Where k is
// zero on an axis the class has no member negating it and the derivatives odd
// in it vanish (those products are skipped).  The class tables are the
// Coulomb sign-class ones (56 classes per octant).
//
// Layout: each parity class is padded to whole 16-row tiles (rows) and 4-index
// k-steps (columns); the moments are copied into that column order (k_soft_msort,
// a row per box and an all-zero row after them), k-steps 2j, 2j + 1 of lane
// group g at 8 j + 2 g + {0, 1}, so a lane reads two k-steps with one 16-byte load.
template <int P> struct SoftSym {
    static constexpr int csize(int c)
    {
        int n = 0;
        for (int i = 0; i <= P; ++i)
            for (int j = 0; i + j <= P; ++j)
                for (int k = 0; i + j + k <= P; ++k) n += ((i & 1) << 2 | (j & 1) << 1 | (k & 1)) == c;
        return n;
    }
    static constexpr int sum_tiles(int q)
    {
        int t = 0;
        for (int c = 0; c < 8; ++c) t += (csize(c) + q - 1) / q;
        return t;
    }
    static constexpr int NP = ncoef(P), MT = sum_tiles(16), KS = sum_tiles(4), KSV = (KS + 1) / 2, LDMS = 8 * KSV;
    static constexpr int CMAX = csize(0); // the all-even class is the largest
    int csz[8] = {}, rc[MT] = {}, kc[KS] = {}, rfirst[9] = {}, kfirst[9] = {};
    constexpr SoftSym()
    {
        int t = 0, u = 0;
        for (int c = 0; c < 8; ++c) {
            csz[c] = csize(c);
            rfirst[c] = t;
            kfirst[c] = u;
            for (int q = 0; q < (csz[c] + 15) / 16; ++q) rc[t++] = c;
            for (int q = 0; q < (csz[c] + 3) / 4; ++q) kc[u++] = c;
        }
        rfirst[8] = t;
        kfirst[8] = u;
    }
};
int soft_sym_ld(int p)
{
    switch (p) {
    case 4: return SoftSym<4>::LDMS; case 5: return SoftSym<5>::LDMS; case 6: return SoftSym<6>::LDMS;
    case 7: return SoftSym<7>::LDMS; case 8: return SoftSym<8>::LDMS;
    default: return 0;
    }
}

// pos[c][t]: DA index of the t-th monomial (in DA order) of parity class c
template <int P, int CMAX, typename IP> __device__ inline void soft_class_positions(IP exps, int tid, int nt, int (*pos)[CMAX])
{
    auto cls = [](int x) { return (x & 1) << 2 | ((x >> 8) & 1) << 1 | ((x >> 16) & 1); };
    for (int e = tid; e < ncoef(P); e += nt) {
        const int c = cls(exps[e]);
        int r = 0;
        for (int f = 0; f < e; ++f) r += cls(exps[f]) == c;
        pos[c][r] = e;
    }
}

// the moments in the sign-class column order; row nrows - 1 is all zero
template <int P>
__global__ __launch_bounds__(256) void k_soft_msort(const PlanView *V, double *Ms, int nrows)
{
    using SS = SoftSym<P>;
    static constexpr SS S{};
    constexpr int LDMS = SS::LDMS;
    __shared__ int sPos[8][SS::CMAX];
    __shared__ int sCol[LDMS];
    const PlanView &v = V[0];
    const int tid = threadIdx.x;
    soft_class_positions<P, SS::CMAX>(gptr(v.tab->exps), tid, 256, sPos);
    __syncthreads();
    for (int q = tid; q < LDMS; q += 256) {
        const int ks = 2 * (q / 8) + (q & 1), g = (q & 7) >> 1;
        int a = -1;
        if (ks < SS::KS) {
            const int c = S.kc[ks], t = 4 * (ks - S.kfirst[c]) + g;
            if (t < S.csz[c]) a = sPos[c][t];
        }
        sCol[q] = a;
    }
    __syncthreads();
    const int64_t total = (int64_t)nrows * LDMS, ldm = v.ldm;
    for (int64_t e = (int64_t)blockIdx.x * 256 + tid; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t row = e / LDMS;
        const int a = sCol[e - row * LDMS];
        Ms[e] = row < nrows - 1 && a >= 0 ? v.M[row * ldm + a] : 0.0;
    }
}

// Two blocks of 4 wavefronts per target tile (each block every other class of
// the tile's used ones), each wavefront 16 targets with all row tiles; per
// level the classes used by the level's targets, one after the other (in
// zero-mask order, so Z is a compile-time constant of the loop that runs
// them; a wavefront skips a class none of its targets has): the
// representative's table staged in
// LDS (SoftCube layout, double-buffered), per k-step the 8 members' operands
// (one 16-byte vector of two k-steps per member, one vector ahead), their
// transform, then one MFMA per compatible row tile with the output of the
// transform that the row and column parities select.
template <int P>
__global__ __launch_bounds__(256) void k_m2l_soft_sym(const PlanView *V, SoftGrid G)
{
    using SS = SoftSym<P>;
    static constexpr SS S{};
    constexpr int MT = SS::MT, KS = SS::KS, KSV = SS::KSV, LDMS = SS::LDMS, CMAX = SS::CMAX;
    constexpr int LDD = SoftCube<P>::LDD, LDC = (ncoef(2 * P) + 1) & ~1;
    constexpr int DV = (LDC / 2 + 255) / 256;
    static_assert(8 * CMAX * sizeof(int) <= LDD * sizeof(double), "class positions fit in a table buffer");
    typedef double dvec_t __attribute__((ext_vector_type(2)));
    __shared__ double sD[2][LDD];
    __shared__ int sHo[4][KS];
    __shared__ int sTg[64], sLv[64];
    __shared__ int sRep[kSymClasses];
    __shared__ unsigned char sMem[kSymClasses][8]; // member slots (255: none)
    __shared__ unsigned char sSl[kVSlots];         // class of each V slot
    __shared__ unsigned char sList[kSymClasses];
    __shared__ int sZend[8];
    __shared__ unsigned long long sUsed;
    __shared__ int sN, sInfo[3];
    int(*sPos)[CMAX] = (int(*)[CMAX]) & sD[1][0]; // (set-up and output only)
    const PlanView &v = V[0];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
    const OrderTables &tb = *v.tab;
    const auto exps = gptr(tb.exps);
    // two blocks per tile (consecutive, so on one XCD), each taking every
    // other class of the tile's used ones; both add into L, which is zero
    // before the M2L (two terms added to zero in either order: deterministic)
    const int item = xcd_remap(blockIdx.x, 2 * G.nblocks), part = item & 1;
    soft_tile_targets(v, G, item >> 1, tid, sTg);
    soft_class_positions<P, CMAX>(exps, tid, 256, sPos);
    __syncthreads();
    soft_tile_levels(v, tid, sTg, sLv, sInfo);
    const int lmin = sInfo[0], lmax = sInfo[1], oct = sInfo[2];
    if (lmax < 0) return; // (block-uniform)
    {
        const auto rep = gptr(tb.srep) + oct * kSymClasses, mem = gptr(tb.smem) + oct * kSymClasses * 8;
        const auto ssl = gptr(tb.sslot) + oct * kVSlots;
        for (int e = tid; e < kSymClasses * 8; e += 256) {
            const int j = mem[e];
            sMem[e >> 3][e & 7] = (unsigned char)(j >= 0 ? j : 255);
        }
        if (tid < kSymClasses) sRep[tid] = rep[tid];
        if (tid < kVSlots) sSl[tid] = (unsigned char)ssl[tid];
        for (int e = tid; e < 4 * KS; e += 256) {
            const int g = e / KS, ks = e - g * KS, c = S.kc[ks], t = 4 * (ks - S.kfirst[c]) + g;
            sHo[g][ks] = t < S.csz[c] ? SoftCube<P>::addr(exps[sPos[c][t]]) : 0;
        }
    }
    int hb[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int c = S.rc[mt], t = 16 * (mt - S.rfirst[c]) + col;
        hb[mt] = t < S.csz[c] ? SoftCube<P>::addr(exps[sPos[c][t]]) : 0;
    }
    const int tgt = sTg[wave * 16 + col], tlev = sLv[wave * 16 + col];
    const auto vs = gptr(v.vslot);
    const uint32_t zoff = (uint32_t)v.nboxes * (uint32_t)LDMS * 8u; // the all-zero row
    const auto Mg = gptr((const char *)v.Mh);
    dvec_t pd[DV];
    int dm[DV][2];
#pragma unroll
    for (int r = 0; r < DV; ++r)
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int e = (tid + 256 * r) * 2 + w;
            dm[r][w] = e < LDC ? gptr(v.soft_map)[e] : LDD - 1;
        }
    double4_t acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = double4_t{0, 0, 0, 0};
    __syncthreads(); // sPos is overwritten by the tables from here on

    for (int L = lmin; L <= lmax; ++L) {
        // classes used by the targets of level L
        if (tid == 0) sUsed = 0;
        __syncthreads();
        {
            unsigned long long used = 0;
            for (int e = tid; e < 64 * kVSlots; e += 256) {
                const int q = e / kVSlots, j = e - q * kVSlots;
                if (sLv[q] == L && vs[(int64_t)sTg[q] * kVSlots + j] >= 0) used |= 1ull << sSl[j];
            }
            if (used) atomicOr(&sUsed, used);
        }
        __syncthreads();
        if (tid < 64) { // this part's classes in table order; where each zero mask's classes end
            const unsigned long long below = lanes_below(lane);
            const int c = lane;
            const unsigned long long used =
                __ballot(c < kSymClasses && ((sUsed >> c) & 1) && (__popcll(sUsed & below) & 1) == part);
            if (c < kSymClasses && ((used >> c) & 1)) sList[__popcll(used & below)] = (unsigned char)c;
            const int z = c < kSymClasses ? sRep[c] >> 16 : 0, zn = c + 1 < kSymClasses ? sRep[c + 1] >> 16 : 8;
            if (c < kSymClasses && zn != z) sZend[z] = __popcll(used & (below | (1ull << c)));
            if (lane == 0) sN = __popcll(used);
        }
        __syncthreads();
        const int nq = sN;
        if (nq == 0) continue; // (block-uniform)
        const double *Dl = v.Dsoft + (int64_t)(L - 2) * 343 * LDC;
        auto load_d = [&](int c) {
            const dvec_t *Dk = (const dvec_t *)(Dl + (int64_t)(sRep[c] & 0xffff) * LDC);
#pragma unroll
            for (int r = 0; r < DV; ++r) {
                const int e = tid + 256 * r;
                pd[r] = e < LDC / 2 ? gload(Dk + e) : dvec_t{0, 0};
            }
        };
        auto store_d = [&](int buf) {
#pragma unroll
            for (int r = 0; r < DV; ++r)
                if (tid + 256 * r < LDC / 2)
#pragma unroll
                    for (int w = 0; w < 2; ++w) sD[buf][dm[r][w]] = pd[r][w];
        };
        // byte offsets of the members' sorted rows (lane group kq's vector 0)
        auto class_src = [&](int q, uint32_t (&src)[8]) {
            const int c = sList[q];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int j = sMem[c][m];
                const int b = j != 255 && tlev == L ? vs[(int64_t)tgt * kVSlots + j] : -1;
                src[m] = b >= 0 ? ((uint32_t)b * (uint32_t)LDMS + 2u * (uint32_t)kq) * 8u : zoff + 16u * (uint32_t)kq;
            }
        };
        dvec_t cur[8], nxt[8];
        auto load_v = [&](dvec_t (&dst)[8], const uint32_t (&src)[8], int j, auto zc) {
            constexpr int Z = decltype(zc)::value;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                if (m & Z) continue;
                uint32_t o = src[m];
                asm volatile("" : "+v"(o)); // (keeps base + 32-bit offset addressing)
                dst[m] = *(const __attribute__((address_space(1))) dvec_t *)(Mg + (uint64_t)o + 64u * (uint32_t)j);
            }
        };
        uint32_t srcc[8], srcn[8];
        load_d(sList[0]);
        store_d(0);
        class_src(0, srcc);
        load_v(cur, srcc, 0, std::integral_constant<int, 0>{});
        __syncthreads();
        int q = 0;
        auto run_mask = [&](auto zc) {
            constexpr int Z = decltype(zc)::value;
            const int qend = sZend[Z] < nq ? sZend[Z] : nq;
            for (; q < qend; ++q) {
                const int buf = q & 1;
                const bool more = q + 1 < nq;
                if (more) {
                    load_d(sList[q + 1]);
                    class_src(q + 1, srcn);
                } else {
#pragma unroll
                    for (int m = 0; m < 8; ++m) srcn[m] = zoff + 16u * (uint32_t)kq;
                }
                // the wavefront skips a class none of its targets has
                bool has = false;
#pragma unroll
                for (int m = 0; m < 8; ++m) has |= srcc[m] != zoff + 16u * (uint32_t)kq;
                if (__ballot(has)) {
                    const double *D = sD[buf];
                    const int *Ho = sHo[kq];
#pragma unroll
                    for (int jv = 0; jv < KSV; ++jv) {
                        if (jv + 1 < KSV) load_v(nxt, srcc, jv + 1, zc);
                        else load_v(nxt, srcn, 0, std::integral_constant<int, 0>{});
#pragma unroll
                        for (int w = 0; w < 2; ++w) {
                            const int ks = 2 * jv + w;
                            if (ks < KS) {
                                const int ha = Ho[ks];
                                double h[8];
#pragma unroll
                                for (int m = 0; m < 8; ++m) h[m] = (m & Z) ? 0.0 : cur[m][w];
                                wht8z<Z>(h);
#pragma unroll
                                for (int mt = 0; mt < MT; ++mt)
                                    if (!((S.rc[mt] ^ S.kc[ks]) & Z))
                                        acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(D[hb[mt] + ha], h[S.rc[mt] ^ S.kc[ks]],
                                                                                       acc[mt], 0, 0, 0);
                            }
                        }
#pragma unroll
                        for (int m = 0; m < 8; ++m) cur[m] = nxt[m];
                    }
                } else {
                    load_v(cur, srcn, 0, std::integral_constant<int, 0>{});
                }
#pragma unroll
                for (int m = 0; m < 8; ++m) srcc[m] = srcn[m];
                if (more) store_d(buf ^ 1);
                __syncthreads();
            }
        };
        run_mask(std::integral_constant<int, 0>{});
        run_mask(std::integral_constant<int, 1>{});
        run_mask(std::integral_constant<int, 2>{});
        run_mask(std::integral_constant<int, 3>{});
        run_mask(std::integral_constant<int, 4>{});
        run_mask(std::integral_constant<int, 5>{});
        run_mask(std::integral_constant<int, 6>{}); // at most two zero axes
    }
    // outputs: row 4 r + kq of each tile, back in DA order
    __syncthreads();
    soft_class_positions<P, CMAX>(exps, tid, 256, sPos);
    __syncthreads();
    if (tgt < 0) return;
    double *Lt = v.L + (int64_t)tgt * v.ldm;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int c = S.rc[mt];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = 16 * (mt - S.rfirst[c]) + 4 * r + kq;
            if (t < S.csz[c]) atomicAdd(Lt + sPos[c][t], acc[mt][r]);
        }
    }
}

// ---------------- P2L and M2P (adaptive trees) ----------------
__device__ inline void soft_box_geom(const PlanView &v, int b, double cen[3], double &h)
{
    const int l = v.level[b];
    int c[3];
    deinterleave(v.morton[b], l, c);
    h = v.W / (double)(1ll << l);
    for (int k = 0; k < 3; ++k) cen[k] = v.lo[k] + ((double)c[k] + 0.5) * h;
}

// ---- Taylor coefficients per lane ----
// One particle per lane: a_g (|g| <= Q) of (|x + z|^2 + eta^2)^(-1/2) in z by
// the recurrence above, unrolled at compile time so that every a_g lives in a
// register (a shell is needed only by the next two), each handed to a
// consumer as soon as it exists.
namespace lane_taylor {
constexpr int cx_ncoef(int n) { return (n + 1) * (n + 2) * (n + 3) / 6; }
constexpr int cx_below(int n) { return n * (n + 1) * (n + 2) / 6; }
constexpr int cx_deg(int e)
{
    int n = 0;
    while (cx_ncoef(n) <= e) ++n;
    return n;
}
constexpr int cx_jk(int e) // j + k of the monomial at DA index e
{
    const int r = e - cx_below(cx_deg(e));
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= r) ++a;
    return a;
}
constexpr int cx_k(int e) { return e - cx_below(cx_deg(e)) - cx_jk(e) * (cx_jk(e) + 1) / 2; }
constexpr int cx_j(int e) { return cx_jk(e) - cx_k(e); }
constexpr int cx_i(int e) { return cx_deg(e) - cx_jk(e); }
constexpr int cx_index(int i, int j, int k) { return cx_below(i + j + k) + (j + k) * (j + k + 1) / 2 + k; }
constexpr double cx_fact(int n) { return n <= 1 ? 1.0 : n * cx_fact(n - 1); }
constexpr double cx_gfact(int e) { return cx_fact(cx_i(e)) * cx_fact(cx_j(e)) * cx_fact(cx_k(e)); }

// per-shell multipliers: a_g = sum_d w_d a_(g - e_d) + z sum_d a_(g - 2e_d),
// w_d = -(2n - 1) x_d / (n rho), z = -(n - 1) / (n rho)
struct Shell {
    double w0, w1, w2, z;
};

template <int E, int NQ> struct Run {
    template <class F>
    static __device__ __forceinline__ void go(double *a, Shell &sh, const double x[3], double ir, F &f)
    {
        constexpr int n = cx_deg(E), i = cx_i(E), j = cx_j(E), k = cx_k(E);
        if constexpr (E == cx_below(n)) {
            const double c1 = -(2.0 * n - 1.0) / n * ir;
            sh.w0 = c1 * x[0];
            sh.w1 = c1 * x[1];
            sh.w2 = c1 * x[2];
            sh.z = -(n - 1.0) / n * ir;
        }
        double s1 = 0.0, s2 = 0.0;
        if constexpr (i >= 1) s1 = sh.w0 * a[cx_index(i - 1, j, k)];
        if constexpr (j >= 1) s1 = fma(sh.w1, a[cx_index(i, j - 1, k)], s1);
        if constexpr (k >= 1) s1 = fma(sh.w2, a[cx_index(i, j, k - 1)], s1);
        if constexpr (i >= 2) s2 = a[cx_index(i - 2, j, k)];
        if constexpr (j >= 2) s2 += a[cx_index(i, j - 2, k)];
        if constexpr (k >= 2) s2 += a[cx_index(i, j, k - 2)];
        if constexpr (n >= 2)
            a[E] = fma(sh.z, s2, s1);
        else
            a[E] = s1;
        f.template on<E>(a[E]);
        // keep the scheduler from hoisting every consumer load to the top
        if constexpr (E % 16 == 15) __builtin_amdgcn_sched_barrier(0);
        Run<E + 1, NQ>::go(a, sh, x, ir, f);
    }
};
template <int NQ> struct Run<NQ, NQ> {
    template <class F> static __device__ __forceinline__ void go(double *, Shell &, const double *, double, F &) {}
};

// a_g(x) for |g| <= Q into the consumer f (f.on<E>(a_E) in DA order)
template <int Q, class F> __device__ __forceinline__ void taylor(const double x[3], double eta2, F &f)
{
    constexpr int NQ = cx_ncoef(Q);
    double a[NQ];
    const double rho = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + eta2;
    const double ir = 1.0 / rho;
    a[0] = 1.0 / sqrt(rho);
    f.template on<0>(a[0]);
    Shell sh;
    Run<1, NQ>::go(a, sh, x, ir, f);
}
} // namespace lane_taylor

// P2L: Lhat_b(B) += q b! a_b((c_B - x_j) / h_B; eta = eps / h_B) for every
// particle j of the boxes of B's X list.  One wavefront per X target; the
// source particles of the list, 64 at a time, one per lane; the sums over the
// lanes run through an LDS transpose, 32 coefficients at a time, as the
// coefficients are produced (lane r < 32 keeps coefficient 32 G + r of group G).
namespace p2l_detail {
template <int P> struct Acc {
    static constexpr int NC = ncoef(P), NG = (NC + 31) / 32;
    double (*T)[65];
    double q, acc[NG];
    int lane;
    template <int E> __device__ __forceinline__ void on(double v)
    {
        T[E % 32][lane] = q * v;
        if constexpr (E % 32 == 31 || E == NC - 1) {
            constexpr int rows = E % 32 + 1;
            wave_sync();
            const int r = lane & 31, c0 = (lane >> 5) * 32;
            double s = 0.0;
            if (r < rows) {
#pragma unroll 8
                for (int c = 0; c < 32; ++c) s += T[r][c0 + c];
            }
            s += __shfl_xor(s, 32);
            acc[E / 32] += s;
            wave_sync();
        }
    }
};
} // namespace p2l_detail

template <int P>
__global__ __launch_bounds__(64) void k_soft_p2l(const PlanView *V)
{
    using A = p2l_detail::Acc<P>;
    constexpr int NC = A::NC, NG = A::NG;
    __shared__ double T[32][65];
    __shared__ int pre[65], pf[64];
    const PlanView &v = V[0];
    const int box = v.xtgt[blockIdx.x], lane = threadIdx.x;
    double cen[3], h;
    soft_box_geom(v, box, cen, h);
    const double ih = 1.0 / h, eta2 = v.eps2 * ih * ih;
    A acc;
    acc.T = T;
    acc.lane = lane;
#pragma unroll
    for (int g = 0; g < NG; ++g) acc.acc[g] = 0.0;
    const int64_t x0 = v.X_off[box], x1 = v.X_off[box + 1];
    for (int64_t xb = x0; xb < x1; xb += 64) {
        // the next 64 entries of the list: exclusive prefix of their counts
        const int ne = x1 - xb < 64 ? (int)(x1 - xb) : 64;
        int c = 0, f = 0;
        if (lane < ne) {
            const int src = v.X_src[xb + lane];
            c = v.count[src];
            f = v.first[src];
        }
        int incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        wave_sync();
        pre[lane + 1] = incl;
        pf[lane] = f;
        if (lane == 0) pre[0] = 0;
        wave_sync();
        const int total = pre[ne];
        for (int t0 = 0; t0 < total; t0 += 64) {
            const int t = t0 + lane < total ? t0 + lane : total - 1;
            int lo = 0, hi = ne - 1; // the entry s with pre[s] <= t < pre[s + 1]
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int i = pf[lo] + (t - pre[lo]);
            const double x[3] = {(cen[0] - v.xs[i]) * ih, (cen[1] - v.ys[i]) * ih, (cen[2] - v.zs[i]) * ih};
            acc.q = t0 + lane < total ? v.qs[i] : 0.0;
            lane_taylor::taylor<P>(x, eta2, acc);
        }
        wave_sync(); // pre and pf are rewritten for the next piece
    }
    if (lane < 32) {
        double *L = v.L + (int64_t)box * v.ldm;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int e = 32 * g + lane;
            if (e < NC) {
                int n = 0, i, j, k;
                while (below(n + 1) <= e) ++n;
                mono_exps(e, n, i, j, k);
                L[e] += acc.acc[g] * (fact_d(i) * fact_d(j) * fact_d(k));
            }
        }
    }
}

// M2P: phi(x) += (1/h) sum_a Mhat_a a! a_a(u), u = (x - c_C)/h_C, eta = eps/h_C,
// and its gradient (1/h^2) sum_g g! a_g(u) sum_k e_k Mhat_(g - e_k), for every
// box C of the leaf's W list, added to the near-field sums (after P2P).  One
// wavefront per leaf, one particle per lane (64 at a time); the moments of the
// W box are read from LDS (the same address on every lane), the next box's
// prefetched into registers meanwhile.
namespace m2p_detail {
template <int P> struct Acc {
    const double *m; // Mhat of the W box, m[NC] = 0
    double ph, g0, g1, g2;
    template <int E> __device__ __forceinline__ void on(double v)
    {
        using namespace lane_taylor;
        constexpr int n = cx_deg(E), i = cx_i(E), j = cx_j(E), k = cx_k(E);
        constexpr double gf = cx_gfact(E); // (a constant: no factorial at run time)
        const double b = v * gf;
        if constexpr (n <= P) ph = fma(m[E], b, ph);
        if constexpr (i >= 1) g0 = fma(m[cx_index(i - 1, j, k)], b, g0);
        if constexpr (j >= 1) g1 = fma(m[cx_index(i, j - 1, k)], b, g1);
        if constexpr (k >= 1) g2 = fma(m[cx_index(i, j, k - 1)], b, g2);
    }
};
} // namespace m2p_detail

template <int P>
__global__ __launch_bounds__(64) void k_soft_m2p(const PlanView *V)
{
    constexpr int NC = ncoef(P), RC = (NC + 63) / 64;
    __shared__ double cm[2][NC];
    const PlanView &v = V[0];
    const int box = v.leaves[blockIdx.x], lane = threadIdx.x;
    const int64_t w0 = v.W_off[box], w1 = v.W_off[box + 1];
    if (w0 == w1) return;
    const int f = v.first[box], cnt = v.count[box];
    for (int s0 = 0; s0 < cnt; s0 += 64) {
        const bool act = s0 + lane < cnt;
        const int i = act ? f + s0 + lane : f;
        const double px = v.xs[i], py = v.ys[i], pz = v.zs[i];
        double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        // W entries 64 at a time, lane l holding entry wb + l
        int64_t wb = w0;
        int wl = wb + lane < w1 ? v.W_src[wb + lane] : 0;
        double nxt[RC];
        auto fetch = [&](int64_t e) {
            if (e - wb >= 64) {
                wb += 64;
                wl = wb + lane < w1 ? v.W_src[wb + lane] : 0;
            }
            const int src = __builtin_amdgcn_readlane(wl, (int)(e - wb));
            const double *Ms = v.M + (int64_t)src * v.ldm;
#pragma unroll
            for (int r = 0; r < RC; ++r) nxt[r] = lane + 64 * r < NC ? Ms[lane + 64 * r] : 0.0;
            return src;
        };
        int src = fetch(w0);
        for (int64_t e = w0; e < w1; ++e) {
            const int buf = (int)((e - w0) & 1);
#pragma unroll
            for (int r = 0; r < RC; ++r)
                if (lane + 64 * r < NC) cm[buf][lane + 64 * r] = nxt[r];
            wave_sync();
            double cs[3], hs;
            soft_box_geom(v, src, cs, hs);
            if (e + 1 < w1) src = fetch(e + 1);
            const double ih = 1.0 / hs, eta2 = v.eps2 * ih * ih;
            const double u[3] = {(px - cs[0]) * ih, (py - cs[1]) * ih, (pz - cs[2]) * ih};
            m2p_detail::Acc<P> acc{cm[buf], 0.0, 0.0, 0.0, 0.0};
            lane_taylor::taylor<P + 1>(u, eta2, acc);
            phi = fma(acc.ph, ih, phi);
            const double ih2 = ih * ih;
            gx = fma(acc.g0, ih2, gx);
            gy = fma(acc.g1, ih2, gy);
            gz = fma(acc.g2, ih2, gz);
        }
        if (act) { // E = -grad phi
            v.phi_near[i] += phi;
            v.fld_near[3 * (int64_t)i] -= gx;
            v.fld_near[3 * (int64_t)i + 1] -= gy;
            v.fld_near[3 * (int64_t)i + 2] -= gz;
        }
        wave_sync();
    }
}

// ---------------- launchers ----------------
#define SOFT_SWITCH(p, CALL)                                                                   \
    switch (p) {                                                                               \
    case 0: CALL(0); break; case 1: CALL(1); break; case 2: CALL(2); break; case 3: CALL(3); break; \
    case 4: CALL(4); break; case 5: CALL(5); break; case 6: CALL(6); break; case 7: CALL(7); break; \
    case 8: CALL(8); break; case 9: CALL(9); break; default: CALL(10); break;                 \
    }

int soft_table_ldc(int p) { return (ncoef(2 * p) + 1) & ~1; }

void launch_soft_tables(int p, int nlev, double *D, int *map, double W, double eps, hipStream_t s)
{
    if (nlev <= 0) return;
    const int ldc = soft_table_ldc(p);
#define T_(PP) k_soft_tables<PP><<<nlev * 343, 256, 0, s>>>(D, map, ldc, W, eps)
    SOFT_SWITCH(p, T_)
#undef T_
}

void launch_soft_p2m(int p, const PlanView *V, int nleaves, int ldm, hipStream_t s)
{
    const int64_t tot = (int64_t)nleaves * ldm;
    if (!tot) return;
    const unsigned nb = (unsigned)((tot + 255) / 256);
#define T_(PP) k_soft_p2m<PP><<<nb, 256, 0, s>>>(V)
    SOFT_SWITCH(p, T_)
#undef T_
}

void launch_soft_m2m(int p, const PlanView *V, int first_box, int nbox, hipStream_t s)
{
    if (nbox <= 0) return;
#define T_(PP) k_soft_m2m<PP><<<nbox, 512, 0, s>>>(V, first_box)
    SOFT_SWITCH(p, T_)
#undef T_
}

void launch_soft_l2l(int p, const PlanView *V, int first_child, int nchild, hipStream_t s)
{
    if (nchild <= 0) return;
#define T_(PP) k_soft_l2l<PP><<<nchild, 64, 0, s>>>(V, first_child)
    SOFT_SWITCH(p, T_)
#undef T_
}

void launch_soft_p2l(int p, const PlanView *V, int nxtgt, hipStream_t s)
{
    if (nxtgt <= 0) return;
#define T_(PP) k_soft_p2l<PP><<<nxtgt, 64, 0, s>>>(V)
    SOFT_SWITCH(p, T_)
#undef T_
}

void launch_soft_m2p(int p, const PlanView *V, int nleaves, hipStream_t s)
{
    if (nleaves <= 0) return;
#define T_(PP) k_soft_m2p<PP><<<nleaves, 64, 0, s>>>(V)
    SOFT_SWITCH(p, T_)
#undef T_
}

void launch_m2l_soft(int p, const PlanView *V, const SoftGrid &G, double *Ms, int nboxes, hipStream_t s)
{
    if (G.nblocks <= 0) return;
    if (p >= kSoftSymOrder && p <= kSoftSymMaxOrder) {
        const int64_t tot = (int64_t)(nboxes + 1) * soft_sym_ld(p);
        const unsigned nb = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
        switch (p) {
#define T_(PP)                                                                   \
    case PP:                                                                     \
        k_soft_msort<PP><<<nb, 256, 0, s>>>(V, Ms, nboxes + 1);                  \
        k_m2l_soft_sym<PP><<<2 * G.nblocks, 256, 0, s>>>(V, G);                  \
        break;
            T_(4) T_(5) T_(6) T_(7) T_(8)
#undef T_
        default: break;
        }
        return;
    }
#define T_(PP) k_m2l_soft<PP><<<G.nblocks, 256, 0, s>>>(V, G)
    SOFT_SWITCH(p, T_)
#undef T_
}

} // namespace fmm
