// M2L (Sec. 2.3) on the matrix cores.
//
// In scaled units the DA M2L is the contraction
//     Lhat_b(B) = sum_{C in V(B)} sum_a D_(a+b)(k_BC) Mhat_a(C),
// D_g(k) the derivative tensor of 1/|x| at the integer box offset k.  Because
// 1/|x| is harmonic, D_(g+2e_z) = -D_(g+2e_x) - D_(g+2e_y): the contraction is
// carried out on the (p+1)^2 components with a_z, b_z <= 1 after folding Mhat
// onto them, and the other components of Lhat are recovered afterwards (unfold).
//
// Work decomposition.  A block holds 64 targets (4 wavefronts x 16) of one
// octant, so they share the same 189 source offsets (Sec. 3.4: at most 189
// boxes per interaction list); slots that no target of the block uses are
// skipped, and so are the products of a wavefront none of whose targets uses
// the slot.  For every offset slot each wavefront runs a (p+1)^2 x (p+1)^2 by
// 16 product with 16x16x4 MFMAs: A[b][a] = D(addr(b) + addr(a)) is gathered
// from the slot's derivative table in LDS with the additive address
// addr(i,j,k) = k s2 + i s1 + j, which turns the Hankel structure of the
// matrix into a single add per operand (the strides s1, s2 are chosen per
// order to spread one operand load over the LDS banks); B, the 16 source vectors, is
// loaded from memory straight into the lanes that feed it to the MFMA, one
// slot ahead (each k-step's operand register is refilled for the next slot
// once its MFMAs are issued).  The derivative tables are double-buffered in
// LDS, so a slot costs one workgroup barrier.  When (p+1)^2 exceeds a
// multiple of 16 by one or two rows (p = 6, 8), those rows are computed with
// FMAs on the vector unit from the same operands instead of a mostly empty
// MFMA row tile.  Accumulators stay in registers across all 189 slots, so
// every target is written once; the FP32 variant adds each slot's FP32 partial
// into FP64 accumulators, so only the per-slot products carry FP32 rounding.  Operand layouts (verified on gfx950):
// A: lane l holds A[l%16][l/16]; B: lane l holds B[l/16][l%16];
// D: f64 lane l reg r -> D[4r + l/16][l%16], f32 lane l reg r -> D[4(l/16)+r][l%16].
#include "ops.h"

#include <type_traits>

namespace fmm {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef double4_t acc_t;
    __device__ static acc_t run(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
    __device__ static const double *D(const OrderTables &t) { return t.D; }
    __device__ static const double *M(const PlanView &v) { return v.Mh; }
};
template <> struct Mfma<float> {
    typedef float4_t acc_t;
    __device__ static acc_t run(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static const float *D(const OrderTables &t) { return t.Df; }
    __device__ static const float *M(const PlanView &v) { return v.Mhf; }
};

// k-steps of 4 indices needed to cover nh indices with groups of vw steps
// (index 4 vw (s / vw) + vw g + s % vw for step s and lane group g)
__host__ __device__ constexpr int m2l_ksteps(int nh, int vw)
{
    const int q = nh / (4 * vw), r = nh - 4 * vw * q;
    return vw * q + (r == 0 ? 0 : (r <= vw ? r : vw));
}

// Loads through global address-space pointers: generic (flat) loads would also
// count against the LDS wait counter and stall the operand reads behind them.
template <typename T> __device__ inline T gload(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

// (orders 0-5; orders from 6 on run on sign classes)
template <int P, typename T>
__global__ __launch_bounds__(256) void k_m2l(const PlanView *V, Bases B)
{
    static_assert(P <= 5, "slot-by-slot M2L serves orders 0-5");
    constexpr int RS = 1; // row tiles per wavefront group: all of them
    constexpr int NT = 256 * RS; // threads per block
    constexpr int NH = (P + 1) * (P + 1);
    constexpr int MF = NH / 16, XR0 = NH - 16 * MF;
    constexpr bool XV = MF >= 1 && XR0 <= 2;     // leftover rows go to the VALU
    constexpr int MT = XV ? MF : (NH + 15) / 16; // MFMA row tiles
    constexpr int XR = XV ? XR0 : 0;             // VALU rows
    constexpr int MTW = (MT + RS - 1) / RS;      // row tiles per wavefront
    // K order: with groups of VW k-steps, step ks gives lane group kq the index
    // a = 4 VW (ks / VW) + VW kq + ks % VW, so that the VW steps of a group read
    // VW consecutive components of the lane's source: B operands come as one
    // aligned vector per group.  A last, partial group needs only as many
    // steps as the components left over, up to VW.  VW = 4 (16-byte FP32
    // loads) where that costs no step over (p+1)^2 / 4 rounded up, else 2.
    constexpr int KS0 = (NH + 3) / 4;
    constexpr int VW = (sizeof(T) == 4 && m2l_ksteps(NH, 4) == KS0) ? 4 : 2;
    constexpr int KS = m2l_ksteps(NH, VW);
    constexpr int NV = (KS + VW - 1) / VW; // vector loads per lane and slot
    static_assert(4 * VW * NV <= ((NH + 15) & ~15), "vectors must stay inside a padded row");
    constexpr int LDD = dlayout_ldd(P); // table size in the additive LDS layout
    constexpr int LDC = dlayout_ldc(P); // compact table in memory (only the entries read)
    constexpr int DW = 16 / (int)sizeof(T); // compact tables move in 16-byte vectors
    static_assert(LDC % DW == 0, "compact rows must be whole vectors");
    constexpr int DV = (LDC / DW + NT - 1) / NT; // table vectors per thread
    typedef typename Mfma<T>::acc_t acc_t;
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    typedef T dvec_t __attribute__((ext_vector_type(16 / sizeof(T))));
    __shared__ T sD[2][LDD];
    __shared__ int sHo[4][KS]; // additive address of the K index of (ks, kq) (0 if padding)
    __shared__ int sTg[64];
    __shared__ int sList[kVSlots];
    __shared__ int sSrc[64][kVSlots]; // slot rows of the block's targets
    __shared__ int sDoff[kVSlots];     // derivative table of each slot of this octant
    __shared__ int sN, soct;

    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int tile = xcd_remap(blockIdx.x - B.b[k], B.b[k + 1] - B.b[k]);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
    const int tw = RS > 1 ? wave & 3 : wave, half = RS > 1 ? wave >> 2 : 0; // target group, row share
    // lanes col, col+16, col+32, col+48 serve target tw*16+col (one B column)
    const int tgt = v.m2l_tgt[tile * kM2LSlots + tw * 16 + col];
    if (!__syncthreads_or(tgt >= 0)) return;
    if (tgt >= 0) soct = (int)(v.morton[tgt] & 7); // every target of the block has this octant
    if (tid < 64) sTg[tid] = v.m2l_tgt[tile * kM2LSlots + tid];
    const OrderTables &tb = *v.tab;
    for (int e = tid; e < 4 * KS; e += NT) {
        const int g = e / KS, ks = e - g * KS, a = 4 * VW * (ks / VW) + VW * g + ks % VW;
        sHo[g][ks] = a < NH ? tb.hoff[a] : 0;
    }
    int hb[MTW], hx[XR > 0 ? XR : 1];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
        int b = (half * MTW + mt) * 16 + col;
        hb[mt] = b < NH ? tb.hoff[b] : 0;
    }
#pragma unroll
    for (int x = 0; x < XR; ++x) hx[x] = tb.hoff[16 * MT + x];
    __syncthreads();
    // the targets' slot rows, then the slots used by at least one target of
    // the block, in increasing order
    {
        const auto vs = gptr(v.vslot);
        for (int e = tid; e < 64 * kVSlots; e += NT) {
            const int t = e / kVSlots, j = e - t * kVSlots, g = sTg[t];
            sSrc[t][j] = g >= 0 ? vs[(int64_t)g * kVSlots + j] : -1;
        }
    }
    __syncthreads();
    if (tid < kVSlots) {
        int any = 0;
        for (int t = 0; t < 64; ++t) any |= sSrc[t][tid] >= 0;
        sList[tid] = any;
        sDoff[tid] = gptr(tb.offs)[soct * kVSlots + tid] * LDC;
    }
    __syncthreads();
    if (tid == 0) {
        int n = 0;
        for (int j = 0; j < kVSlots; ++j)
            if (sList[j]) sList[n++] = j;
        sN = n;
    }
    __syncthreads();
    const int nvalid = sN, ldh = v.ldmh;
    const T *Dt = Mfma<T>::D(tb);
    const T *Mh = Mfma<T>::M(v);
    const int *vsl = sSrc[tw * 16 + col];

    acc_t acc[MTW];
    double4_t acc64[MTW]; // FP32 path: per-offset partials are summed in FP64
    T xacc[XR > 0 ? XR : 1];
    double xacc64[XR > 0 ? XR : 1];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) { acc[mt] = acc_t{0, 0, 0, 0}; acc64[mt] = double4_t{0, 0, 0, 0}; }
#pragma unroll
    for (int x = 0; x < XR; ++x) { xacc[x] = (T)0; xacc64[x] = 0.0; }

    // B operands of k-steps VW t .. VW t + VW - 1 (vector t of a slot):
    // components 4 VW t + VW kq (+0 .. VW-1).  FP64 keeps a window of NW
    // vectors in flight: vector t of the current slot lives in pb[t % NW], and
    // once it is used, vector t + NW is loaded into the same register (taken
    // from the next slot when t + NW runs past the end of this one).  At these
    // orders the window is the whole slot.
    constexpr bool DB = sizeof(T) == 4;
    constexpr int NW = NV;
    vec_t pb[NW];
    dvec_t pd[DV];
    int dm[DV][DW]; // LDS address of each compact table entry this thread moves
#pragma unroll
    for (int r = 0; r < DV; ++r)
#pragma unroll
        for (int w = 0; w < DW; ++w) {
            const int e = (tid + NT * r) * DW + w;
            dm[r][w] = e < LDC ? gptr(tb.dmap)[e] : LDD - 1;
        }
    auto load_d = [&](int j) {
        const dvec_t *Dk = (const dvec_t *)(Dt + sDoff[j]);
#pragma unroll
        for (int r = 0; r < DV; ++r) {
            int e = tid + NT * r;
            pd[r] = e < LDC / DW ? gload(Dk + e) : dvec_t{};
        }
    };
    auto store_d = [&](int buf) { // scatter into the additive layout
#pragma unroll
        for (int r = 0; r < DV; ++r)
            if (tid + NT * r < LDC / DW)
#pragma unroll
                for (int w = 0; w < DW; ++w) sD[buf][dm[r][w]] = pd[r][w];
    };
    // Loads are always issued (a clamped row for absent sources), so that the
    // waits can count them; operands of absent sources and padding components
    // are zeroed at use.  FP32: the next slot's operands go to a second
    // register set loaded at the top of the slot.
    vec_t pbn[DB ? NV : 1];
    const int64_t kofs = VW * kq;
    auto load_b = [&](int buf, int t, int src) {
        const vec_t val = gload((const vec_t *)(Mh + (int64_t)(src >= 0 ? src : 0) * ldh + kofs) + 4 * t);
        if constexpr (DB) pbn[buf] = val;
        else pb[buf] = val;
    };
    int src = -1;
    if (nvalid > 0) {
        load_d(sList[0]);
        store_d(0);
        src = vsl[sList[0]];
#pragma unroll
        for (int t = 0; t < NW; ++t) load_b(t, t, src);
        if constexpr (DB) {
#pragma unroll
            for (int t = 0; t < NV; ++t) pb[t] = pbn[t];
        }
        __syncthreads();
    }
    for (int q = 0; q < nvalid; ++q) {
        const int cur = q & 1;
        const bool more = q + 1 < nvalid;
        const int jn = more ? sList[q + 1] : 0;
        if (more) load_d(jn); // in flight during the products
        const int nsrc = more ? vsl[jn] : -1;
        const T *D = sD[cur];
        const int *Ho = sHo[kq];
        if constexpr (DB) {
#pragma unroll
            for (int t = 0; t < NV; ++t) load_b(t, t, nsrc);
            __builtin_amdgcn_sched_barrier(0); // keep the loads ahead of the products
        }
        {
            // A operands of step ks+1 are read from LDS while the MFMAs of step ks run
            T ac[MTW], an[MTW];
            {
                const int ha = Ho[0];
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt) ac[mt] = D[hb[mt] + ha];
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int ha = Ho[ks];
                if (ks + 1 < KS) {
                    const int hn = Ho[ks + 1];
#pragma unroll
                    for (int mt = 0; mt < MTW; ++mt) an[mt] = D[hb[mt] + hn];
                }
                const T bv = (src >= 0 && 4 * VW * (ks / VW) + VW * kq + ks % VW < NH)
                                 ? pb[(ks / VW) % NW][ks % VW] : (T)0;
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt)
                    if (RS == 1 || half * MTW + mt < MT) acc[mt] = Mfma<T>::run(ac[mt], bv, acc[mt]);
                if (half == RS - 1)
#pragma unroll
                    for (int x = 0; x < XR; ++x) xacc[x] += D[hx[x] + ha] * bv;
                if constexpr (!DB) // refill once this vector is used up
                    if (ks % VW == VW - 1 || ks == KS - 1) {
                        const int t = ks / VW;
                        if (t + NW < NV) load_b((t + NW) % NW, t + NW, src);
                        else load_b(t % NW, t % NW, nsrc);
                    }
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt) ac[mt] = an[mt];
            }
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[mt][r] += (double)acc[mt][r];
                    acc[mt] = acc_t{0, 0, 0, 0};
                }
#pragma unroll
                for (int x = 0; x < XR; ++x) { xacc64[x] += (double)xacc[x]; xacc[x] = (T)0; }
            }
        }
        if constexpr (DB) {
#pragma unroll
            for (int t = 0; t < NV; ++t) pb[t] = pbn[t];
        }
        if (more) store_d(cur ^ 1);
        src = nsrc;
        __syncthreads(); // next table written; everyone is done with this one
    }
    // VALU rows: each lane holds the terms a = kq (mod 4); sum the four lanes
    double xs[XR > 0 ? XR : 1];
#pragma unroll
    for (int x = 0; x < XR; ++x) {
        double t = sizeof(T) == 4 ? xacc64[x] : (double)xacc[x];
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        xs[x] = t;
    }
    if (tgt < 0) return;
    double *Lh = v.Lh + (int64_t)tgt * ldh;
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int b = (half * MTW + mt) * 16 + Mfma<T>::row(lane, r);
            if (b < NH && (RS == 1 || half * MTW + mt < MT))
                Lh[b] = sizeof(T) == 4 ? acc64[mt][r] : (double)acc[mt][r];
        }
    if (kq == 0 && half == RS - 1) {
#pragma unroll
        for (int x = 0; x < XR; ++x) Lh[16 * MT + x] = xs[x];
    }
}

// ---------------- M2L on sign classes (orders with m2l_sym) ----------------
// Same block decomposition (64 targets of one octant, 4 wavefronts x 16), but
// the loop runs over the octant's 56 sign classes instead of its 189 slots.
// For class c with representative offset k (components >= 0 on the axes
// where the class has a pair of members) and members s o k, s negating the
// axes in the 3-bit mask m:
//     sum_m sum_a D_(a+b)(s o k) Mhat_a(m) = sum_a D_(a+b)(k) H_a[par(a+b)],
//     H[r] = sum_m (-1)^|m & r| Mhat(m),
// a Walsh-Hadamard transform of the members' multipoles (absent members
// count as zero).  Rows and columns are in parity-sorted order, so the
// parity of a + b is the same for a whole 16-row tile and k-step: each MFMA
// takes its B operand from one transform output fixed at compile time.  Where
// k has a zero component, D_g(k) vanishes for odd g on that axis, and the
// row-tile / k-step pairs of opposite parity on it are skipped, and so are
// the members that would negate it (they do not exist) with their loads and
// butterflies.  Each k-step loads the members' operands (one component per
// lane and member; a member missing on a nonzero axis reads the zero row, so
// that the loads of one zero mask are fixed at compile time and the waits
// count them) two vectors ahead, across class boundaries (all eight members
// for the next class, whose mask is not known there).  m2l_parts blocks share
// a tile, each running a contiguous part of its classes (the first with
// kSymFirstPart % of the matrix-core work, dispatched before the others),
// and adds its sums into the target rows of Lh, zeroed before the launch, with
// FP64 atomics: with two parts each entry receives 0 + a + b in either order,
// which is exact-order independent (a + b = b + a), so the result does not
// depend on which part finishes first.  (k_m2l_symh, orders >= 12: part i > 0
// writes its partial sums to slice i - 1 of Lh2, which the pass before the L2L
// adds in part order.)
template <int P> struct SymShape {
    static constexpr int RT = sym_row_tiles(P), KS = sym_ksteps(P);
    int rc[RT], kc[KS]; // parity class of each row tile and k-step
    int kb[9];          // first k-step of each column class
    constexpr SymShape() : rc(), kc(), kb()
    {
        for (int r = 0; r < RT; ++r) rc[r] = sym_tile_class(P, r, true);
        int k = 0;
        for (int c = 0; c < 8; ++c) {
            kb[c] = k;
            for (int t = 0; t < sym_class_ksteps(P, c); ++t) kc[k++] = c;
        }
        kb[8] = k;
    }
};

template <typename T> __device__ inline void wht8(T (&h)[8])
{
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!(i & bit)) {
                const T u = h[i], w = h[i | bit];
                h[i] = u + w;
                h[i | bit] = u - w;
            }
}

// Run by one whole wavefront: from the mask of classes used by a tile's
// targets, list them in class order (sList), note where each zero mask's
// classes end in the list (sZend; the table orders classes by zero mask) and
// pick the range [sQa, sQb) of part `part` when the list is split into
// `parts` contiguous ranges of matrix-core work (a class with z zero axes
// runs 1 / 2^z of the row-tile / k-step products), the first holding
// kSymFirstPart % of it and the others equal shares of the rest: a class
// belongs to the part that holds the midpoint of its weight.  Lane c handles
// class c.
__device__ inline void sym_select_classes(unsigned long long used, const int *rep, int parts, int part, int lane,
                                          int *list, int *zend, int *qa, int *qb)
{
    const int c = lane;
    const bool u = c < kSymClasses && ((used >> c) & 1);
    const int z = c < kSymClasses ? rep[c] >> 16 : 0, zn = c + 1 < kSymClasses ? rep[c + 1] >> 16 : 8;
    const unsigned long long below = lanes_below(c);
    if (u) list[__popcll(used & below)] = c;
    if (c < kSymClasses && zn != z) zend[z] = __popcll(used & (below | (1ull << c)));
    const int pz = __popc(z), w = 4 >> pz;
    const unsigned long long b0 = __ballot(u && pz == 0), b1 = __ballot(u && pz == 1), b2 = __ballot(u && pz == 2);
    const int W = 4 * __popcll(b0) + 2 * __popcll(b1) + __popcll(b2);
    const int cw = 4 * __popcll(b0 & below) + 2 * __popcll(b1 & below) + __popcll(b2 & below);
    // part 0 ends at kSymFirstPart % of the weight, the others share the rest
    int pt = 0;
    for (int q = 0; q + 1 < parts; ++q)
        pt += (int64_t)(2 * cw + w) * 100 * (parts - 1) >=
              (int64_t)2 * W * (kSymFirstPart * (parts - 1) + q * (100 - kSymFirstPart));
    const unsigned long long lo = __ballot(u && pt < part), hi = __ballot(u && pt <= part);
    if (lane == 0) {
        *qa = __popcll(lo);
        *qb = __popcll(hi);
    }
}

// Block set-up shared by the sign-class kernels.  The loads are issued in
// batches (row and column indices, then their D addresses and the octant), so
// that the set-up costs a few memory round trips rather than one per entry.
// Returns the thread's target (-1 for an empty slot), or kNoTargets when the
// tile has none (the whole block then returns).  Fills hb (D address of the
// lane's row in each of the MTW row tiles from R0 on), sTg, sHo (D address of each
// column), soct and clears sUsed.
constexpr int kNoTargets = -2;

// Tile and part of block i of n = tiles x parts: each XCD gets a contiguous
// range of (tile, part) items (as xcd_remap) and runs the range's first parts
// (the longest) before its other parts, so that the end of the launch is made
// of the shorter blocks.
__device__ inline void sym_block(int i, int n, int parts, int &tile, int &part)
{
    const int x = i % kXCDs, y = i / kXCDs, q = n / kXCDs, r = n % kXCDs;
    const int b0 = x * q + (x < r ? x : r), cnt = q + (x < r ? 1 : 0);
    int yy = y, rb = b0;
    for (int p = 0; p < parts; ++p) {
        const int fp = b0 + ((p - b0 % parts) + parts) % parts;
        const int np = fp < b0 + cnt ? (b0 + cnt - 1 - fp) / parts + 1 : 0;
        if (yy < np) { rb = fp + parts * yy; break; }
        yy -= np;
    }
    tile = rb / parts;
    part = rb - tile * parts;
}
template <int MTW, int KS, int R0 = 0>
__device__ inline int sym_setup_tile(const PlanView &v, const OrderTables &tb, int tile, int tid, int col, int (&hb)[MTW],
                                     int *sTg, int (*sHo)[KS], int *soct, unsigned long long *sUsed)
{
    constexpr int NT = 256, NHO = (4 * KS + NT - 1) / NT;
    const auto t_hoff = gptr(tb.hoff), t_srow = gptr(tb.srow), t_scol = gptr(tb.scol);
    const auto mtg = gptr(v.m2l_tgt) + (int64_t)tile * kM2LSlots;
    const int wave = tid >> 6;
    const int tgt = mtg[wave * 16 + col], tg64 = mtg[tid & 63];
    int rowi[MTW], coli[NHO];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) rowi[mt] = t_srow[16 * (R0 + mt) + col];
#pragma unroll
    for (int i = 0; i < NHO; ++i) {
        const int e = tid + NT * i < 4 * KS ? tid + NT * i : 0, g = e / KS, ks = e - g * KS;
        coli[i] = t_scol[4 * ks + g];
    }
    if (!__syncthreads_or(tgt >= 0)) return kNoTargets;
    const int oct = (int)(gptr(v.morton)[max(tgt, 0)] & 7);
    int hov[NHO];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) hb[mt] = t_hoff[max(rowi[mt], 0)];
#pragma unroll
    for (int i = 0; i < NHO; ++i) hov[i] = t_hoff[max(coli[i], 0)];
    if (tid < 64) sTg[tid] = tg64;
    if (tid == 0) *sUsed = 0;
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) hb[mt] = rowi[mt] >= 0 ? hb[mt] : 0;
#pragma unroll
    for (int i = 0; i < NHO; ++i) {
        const int e = tid + NT * i, g = e / KS, ks = e - g * KS;
        if (e < 4 * KS) sHo[g][ks] = coli[i] >= 0 ? hov[i] : 0;
    }
    if (tgt >= 0) *soct = oct;
    __syncthreads();
    return tgt;
}

// The octant's class table: members, representative | zero mask, and the
// class of each V slot.
__device__ inline void sym_stage_classes(const OrderTables &tb, int oct, int tid, int (*sMem)[8], int *sRep, int *sSl)
{
    constexpr int NT = 256, NM = (kSymClasses * 8 + NT - 1) / NT;
    const auto t_smem = gptr(tb.smem) + oct * kSymClasses * 8;
    int mv[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) mv[i] = t_smem[tid + NT * i < kSymClasses * 8 ? tid + NT * i : 0];
    const int rv = gptr(tb.srep)[oct * kSymClasses + (tid < kSymClasses ? tid : 0)];
    const int sv = gptr(tb.sslot)[oct * kVSlots + (tid < kVSlots ? tid : 0)];
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        const int e = tid + NT * i;
        if (e < kSymClasses * 8) sMem[e >> 3][e & 7] = mv[i];
    }
    if (tid < kSymClasses) sRep[tid] = rv;
    if (tid < kVSlots) sSl[tid] = sv;
}

template <int P, typename T>
__global__ __launch_bounds__(256, 2) void k_m2l_sym(const PlanView *V, Bases B)
{
    static constexpr SymShape<P> S{};
    constexpr int RT = SymShape<P>::RT, KS = SymShape<P>::KS;
    constexpr int NT = 256, MTW = RT; // one wavefront holds all row tiles of its 16 targets
    static_assert(RT <= 12, "accumulators of at most 12 row tiles per wavefront");
    // operands move in vectors of VW k-steps (sym_pos layout); a class has KSV
    // vectors, rounded up to an even count KSVW (a virtual last one)
    constexpr int VW = 16 / (int)sizeof(T), KSV = (KS + VW - 1) / VW, KSVW = (KSV + 1) / 2 * 2;
    static_assert(4 * VW * KSV <= folded_ld(P), "vectors inside the folded row");
    constexpr int LDD = dlayout_ldd(P), LDC = dlayout_ldc(P);
    constexpr int DW = 16 / (int)sizeof(T);
    static_assert(LDC % DW == 0, "compact rows must be whole vectors");
    constexpr int DV = (LDC / DW + NT - 1) / NT;
    typedef typename Mfma<T>::acc_t acc_t;
    typedef T dvec_t __attribute__((ext_vector_type(16 / sizeof(T))));
    __shared__ T sD[2][LDD];
    __shared__ int sHo[4][KS];              // D address of column (ks, kq) (0 for padding)
    __shared__ int sTg[64];
    __shared__ int sList[kSymClasses];      // classes the block uses
    __shared__ int sRep[kSymClasses];       // representative | zero mask << 16
    __shared__ int sMem[kSymClasses][8];    // member slots
    __shared__ int sZend[8];                // end of each zero mask's classes in sList
    __shared__ int sSrc[64][kVSlots];
    __shared__ int sSl[kVSlots];            // class of each V slot
    __shared__ unsigned long long sUsed;
    __shared__ int sQa, sQb, soct;

    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    // m2l_parts blocks per tile, each taking a part of the tile's classes
    // (more, shorter blocks: less idle time at the end of the launch)
    const int parts = v.m2l_parts;
    int tile, part;
    sym_block(blockIdx.x - B.b[k], B.b[k + 1] - B.b[k], parts, tile, part);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
    const OrderTables &tb = *v.tab;
    int hb[MTW];
    const int tgt = sym_setup_tile<MTW, KS>(v, tb, tile, tid, col, hb, sTg, sHo, &soct, &sUsed);
    if (tgt == kNoTargets) return;
    {
        // the targets' slot rows: every load issued before the first is used
        const auto vs = gptr(v.vslot);
        constexpr int NE = 64 * kVSlots, PER = (NE + NT - 1) / NT;
        int val[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + NT * i < NE ? tid + NT * i : NE - 1, t = e / kVSlots, j = e - t * kVSlots;
            val[i] = vs[(int64_t)max(sTg[t], 0) * kVSlots + j];
        }
        sym_stage_classes(tb, soct, tid, sMem, sRep, sSl);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + NT * i, t = e / kVSlots, j = e - t * kVSlots;
            if (e < NE) sSrc[t][j] = sTg[t] >= 0 ? val[i] : -1;
        }
    }
    __syncthreads();
    { // classes used by the block: four threads scan each target's slots
        const int *row = sSrc[tid >> 2];
        unsigned long long used = 0;
        for (int j = tid & 3; j < kVSlots; j += 4)
            if (row[j] >= 0) used |= 1ull << sSl[j];
        if (used) atomicOr(&sUsed, used);
    }
    __syncthreads();
    if (tid < 64) sym_select_classes(sUsed, sRep, parts, part, lane, sList, sZend, &sQa, &sQb);
    __syncthreads();
    const int qa = sQa, qb = sQb; // this block's classes
    const int64_t ldmh = v.ldmh;
    const T *Dt = Mfma<T>::D(tb);
    const T *Mh = Mfma<T>::M(v);
    const int *vsl = sSrc[wave * 16 + col];

    acc_t acc[MTW];
    double4_t acc64[MTW];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) { acc[mt] = acc_t{0, 0, 0, 0}; acc64[mt] = double4_t{0, 0, 0, 0}; }

    dvec_t pd[DV];
    int dm[DV][DW];
#pragma unroll
    for (int r = 0; r < DV; ++r)
#pragma unroll
        for (int w = 0; w < DW; ++w) {
            const int e = (tid + NT * r) * DW + w;
            dm[r][w] = e < LDC ? gptr(tb.dmap)[e] : LDD - 1;
        }
    auto load_d = [&](int c) {
        const dvec_t *Dk = (const dvec_t *)(Dt + (int64_t)(sRep[c] & 0xffff) * LDC);
#pragma unroll
        for (int r = 0; r < DV; ++r) {
            const int e = tid + NT * r;
            pd[r] = e < LDC / DW ? gload(Dk + e) : dvec_t{};
        }
    };
    auto store_d = [&](int buf) {
#pragma unroll
        for (int r = 0; r < DV; ++r)
            if (tid + NT * r < LDC / DW)
#pragma unroll
                for (int w = 0; w < DW; ++w) sD[buf][dm[r][w]] = pd[r][w];
    };
    // member sources of the lane's target for class list entry q; absent
    // members read the all-zero row after the boxes
    const int zrow = v.nboxes;
    // (as 32-bit byte offsets from Mh: plans check that the array is below 4 GiB)
    auto class_src = [&](int q, uint32_t (&src)[8]) {
        const int c = sList[q];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int j = sMem[c][m];
            const int b = j >= 0 ? vsl[j] : -1;
            src[m] = ((uint32_t)(b >= 0 ? b : zrow) * (uint32_t)ldmh + (uint32_t)(VW * kq)) * (uint32_t)sizeof(T);
        }
    };
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    vec_t pb[2][8]; // vector j of a class lives in pb[j % 2]
    const auto Mg = gptr((const char *)Mh);
    // (the empty asm keeps each 32-bit offset in its register at the load, so
    // the address stays base + offset instead of a 64-bit pointer per member
    // hoisted out of the class loop)
    // (zc: the class's zero axes, whose negating members are absent and not
    // loaded; 0 for loads of a class whose mask is not known here)
    auto load_b = [&](int slot, int j, const uint32_t (&src)[8], auto zc) {
        constexpr int Z = decltype(zc)::value;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            if (m & Z) continue;
            uint32_t o = src[m];
            asm volatile("" : "+v"(o));
            pb[slot][m] = *(gp<const vec_t>)(Mg + (uint64_t)o + 16 * (4 * j));
        }
    };
    uint32_t srcc[8], srcn[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) srcc[m] = srcn[m] = (uint32_t)zrow * (uint32_t)ldmh * (uint32_t)sizeof(T);
    // one class: KS k-steps; Z (zero-axis mask) decides at compile time which
    // row-tile / k-step products exist
    auto run_class = [&](auto zc, const T *D) {
        constexpr int Z = decltype(zc)::value;
        const int *Ho = sHo[kq];
#pragma unroll
        for (int ks = 0; ks < VW * KSVW; ++ks) {
            if (ks < KS) {
                const int ha = Ho[ks];
                T ac[MTW];
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt) {
                    if (!((S.rc[mt] ^ S.kc[ks]) & Z)) ac[mt] = D[hb[mt] + ha];
                }
                T h[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) h[m] = (m & Z) ? T(0) : pb[(ks / VW) % 2][m][ks % VW];
                wht8z<Z>(h);
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt) {
                    if (!((S.rc[mt] ^ S.kc[ks]) & Z))
                        acc[mt] = Mfma<T>::run(ac[mt], h[S.rc[mt] ^ S.kc[ks]], acc[mt]);
                }
            }
            if (ks % VW == VW - 1) { // vector j used up: refill its registers with vector j + 2
                const int j = ks / VW, jn = j + 2;
                if (jn < KSV) load_b(j % 2, jn, srcc, zc);
                else if (jn >= KSVW && jn - KSVW < KSV) load_b(j % 2, jn - KSVW, srcn, std::integral_constant<int, 0>{});
            }
        }
    };
    if (qb > qa) {
        load_d(sList[qa]);
        store_d(0);
        class_src(qa, srcc);
        load_b(0, 0, srcc, std::integral_constant<int, 0>{});
        if (KSV > 1) load_b(1, 1, srcc, std::integral_constant<int, 0>{});
        __syncthreads();
    }
    // the classes of one zero mask follow each other: one loop per mask
    int q = qa;
    auto run_mask = [&](auto zc) {
        const int qend = min(sZend[decltype(zc)::value], qb);
        for (; q < qend; ++q) {
            const int cur = (q - qa) & 1;
            const bool more = q + 1 < qb;
            if (more) {
                load_d(sList[q + 1]);
                class_src(q + 1, srcn);
            }
            run_class(zc, sD[cur]);
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[mt][r] += (double)acc[mt][r];
                    acc[mt] = acc_t{0, 0, 0, 0};
                }
            }
#pragma unroll
            for (int m = 0; m < 8; ++m) srcc[m] = srcn[m];
            if (more) store_d(cur ^ 1);
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
    if (tgt < 0) return;
    static_assert(sym_parts_add(P), "parts add into the zeroed rows");
    double *Lh = v.Lh + (int64_t)tgt * v.ldh;
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = gptr(tb.srow)[16 * mt + Mfma<T>::row(lane, r)];
            if (b >= 0) atomicAdd(Lh + b, sizeof(T) == 4 ? acc64[mt][r] : (double)acc[mt][r]);
        }
    }
}

// ---------------- sign-class M2L for orders >= 12 ----------------
// The same decomposition as k_m2l_sym (classes in zero-mask order, m2l_parts
// blocks per tile over parts of the classes, transform of the members, one
// MFMA per row tile and k-step with a compile-time transform output),
// organised so that the code stays small at high order: within a class the
// eight column classes are unrolled while each one's k-steps run in a loop
// over 16-byte operand vectors (two k-steps; columns are padded to 8 per
// class so that no vector straddles two classes).  Operands move one vector
// ahead through a current / next register pair, the next class's first vector
// loaded during the last one.  The targets' slot rows are read from memory
// (the classes a block uses come from a 64-bit mask built by all threads),
// which leaves LDS to the derivative tables.  All row tiles of the 16
// targets stay in one wavefront (one wavefront per SIMD, the accumulators in
// the accumulation registers), so that every member operand and transform
// serves every row.  Row tiles from F32T on (the higher degrees: rows are in
// sym_tile_class order) run on FP32 MFMA from the same FP64 operands and
// transform outputs rounded to FP32, each class's FP32 sums added into FP64
// after the class; a local coefficient of degree n carries about rho^n of the
// far field (rho < 1 the convergence ratio), which scales their rounding down.
template <int P, int F32T>
__global__ __launch_bounds__(256, 1) void k_m2l_symh(const PlanView *V, Bases B)
{
    typedef double T;
    static constexpr SymShape<P> S{};
    constexpr int RT = SymShape<P>::RT, KS = SymShape<P>::KS;
    constexpr int MTW = RT, R0 = 0;
    static_assert(MTW <= 24 && F32T >= 1 && F32T <= RT, "row tiles");
    constexpr int N32 = RT - F32T; // FP32 row tiles
    constexpr int KSV = (KS + 1) / 2; // operand vectors per class
    static_assert(8 * KSV <= folded_ld(P), "two-k-step vectors inside the folded row");
    constexpr int NT = 256;
    constexpr int LDD = dlayout_ldd(P), LDC = dlayout_ldc(P);
    constexpr int DW = 2; // compact tables move in 16-byte vectors
    static_assert(LDC % DW == 0, "compact rows must be whole vectors");
    constexpr int DV = (LDC / DW + NT - 1) / NT;
    typedef typename Mfma<T>::acc_t acc_t;
    typedef typename Mfma<float>::acc_t acc32_t;
    typedef T vec_t __attribute__((ext_vector_type(2)));
    __shared__ T sD[2][LDD];
    __shared__ int sHo[4][KS];
    __shared__ int sTg[64];
    __shared__ int sList[kSymClasses];
    __shared__ int sRep[kSymClasses];
    __shared__ int sMem[kSymClasses][8];
    __shared__ int sZend[8];
    __shared__ int sSl[kVSlots];
    __shared__ unsigned long long sUsed;
    __shared__ int sQa, sQb, soct;

    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int parts = v.m2l_parts;
    int tile, part;
    sym_block(blockIdx.x - B.b[k], B.b[k + 1] - B.b[k], parts, tile, part);
    const int tid = threadIdx.x, lane = tid & 63, col = lane & 15, kq = lane >> 4;
    const OrderTables &tb = *v.tab;
    int hb[MTW];
    const int tgt = sym_setup_tile<MTW, KS, R0>(v, tb, tile, tid, col, hb, sTg, sHo, &soct, &sUsed);
    if (tgt == kNoTargets) return;
    const auto vs = gptr(v.vslot);
    {
        // classes used by the block: four threads scan each target's slots
        // (all loads issued before the first is used)
        constexpr int PER = (kVSlots + 3) / 4;
        const int g = sTg[tid >> 2];
        int sv[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = (tid & 3) + 4 * i < kVSlots ? (tid & 3) + 4 * i : kVSlots - 1;
            sv[i] = vs[(int64_t)max(g, 0) * kVSlots + j];
        }
        sym_stage_classes(tb, soct, tid, sMem, sRep, sSl);
        __syncthreads();
        unsigned long long used = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = (tid & 3) + 4 * i;
            if (g >= 0 && j < kVSlots && sv[i] >= 0) used |= 1ull << sSl[j];
        }
        if (used) atomicOr(&sUsed, used);
    }
    __syncthreads();
    if (tid < 64) sym_select_classes(sUsed, sRep, parts, part, lane, sList, sZend, &sQa, &sQb);
    __syncthreads();
    const int qa = sQa, qb = sQb;
    const int64_t ldmh = v.ldmh;
    const T *Dt = tb.D;
    const T *Mh = v.Mh;

    acc_t acc[F32T];
#pragma unroll
    for (int mt = 0; mt < F32T; ++mt) acc[mt] = acc_t{0, 0, 0, 0};
    acc32_t acc32[N32 > 0 ? N32 : 1];
    double4_t acc64[N32 > 0 ? N32 : 1]; // FP32 tiles: per-class sums added here
#pragma unroll
    for (int mt = 0; mt < N32; ++mt) { acc32[mt] = acc32_t{0, 0, 0, 0}; acc64[mt] = double4_t{0, 0, 0, 0}; }

    typedef T dvec_t __attribute__((ext_vector_type(DW)));
    dvec_t pd[DV];
    int dm[DV][DW];
#pragma unroll
    for (int r = 0; r < DV; ++r)
#pragma unroll
        for (int w = 0; w < DW; ++w) {
            const int e = (tid + NT * r) * DW + w;
            dm[r][w] = e < LDC ? gptr(tb.dmap)[e] : LDD - 1;
        }
    auto load_d = [&](int c) {
        const dvec_t *Dk = (const dvec_t *)(Dt + (int64_t)(sRep[c] & 0xffff) * LDC);
#pragma unroll
        for (int r = 0; r < DV; ++r) {
            const int e = tid + NT * r;
            pd[r] = e < LDC / DW ? gload(Dk + e) : dvec_t{};
        }
    };
    auto store_d = [&](int buf) {
#pragma unroll
        for (int r = 0; r < DV; ++r)
            if (tid + NT * r < LDC / DW)
#pragma unroll
                for (int w = 0; w < DW; ++w) sD[buf][dm[r][w]] = pd[r][w];
    };
    // member operand rows as 32-bit byte offsets (plans check the 4 GiB bound);
    // absent members read the zero row after the boxes
    const uint32_t zoff = (uint32_t)v.nboxes * (uint32_t)ldmh * 8u;
    const uint32_t vrow = (uint32_t)(tgt >= 0 ? tgt : 0) * (uint32_t)kVSlots;
    auto class_src = [&](int q, uint32_t (&src)[8]) {
        const int c = sList[q];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int j = sMem[c][m];
            const int b = j >= 0 && tgt >= 0 ? vs[vrow + (uint32_t)j] : -1;
            src[m] = (b >= 0 ? (uint32_t)b * (uint32_t)ldmh * 8u : zoff) + 16u * (uint32_t)kq;
        }
    };
    const auto Mg = gptr((const char *)Mh);
    auto load_v = [&](vec_t (&dst)[8], int j, const uint32_t (&src)[8]) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            uint32_t o = src[m];
            asm volatile("" : "+v"(o));
            dst[m] = *(gp<const vec_t>)(Mg + (uint64_t)o + 64 * j);
        }
    };
    uint32_t srcc[8], srcn[8];
    vec_t cur[8], nxt[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) srcc[m] = srcn[m] = zoff;
    if (qb > qa) {
        load_d(sList[qa]);
        store_d(0);
        class_src(qa, srcc);
        load_v(cur, 0, srcc);
        __syncthreads();
    }
    // one class: column classes unrolled, their vectors in a loop.  A column
    // class may start on the second k-step of a vector (the previous class
    // ran its first) and end on the first k-step of one (the next class runs
    // its second): the vector moves on, and the one after it is requested,
    // where its first k-step is taken.
    auto run_class = [&](auto zc, const T *D) {
        constexpr int Z = decltype(zc)::value;
        const int *Ho = sHo[kq];
        auto column_class = [&](auto tc) {
            constexpr int TAU = decltype(tc)::value;
            constexpr int K0 = S.kb[TAU], K1 = S.kb[TAU + 1];
            auto kstep = [&](int ks, auto wc) {
                constexpr int w = decltype(wc)::value;
                const int ha = Ho[ks];
                T ac[MTW];
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt)
                    if (!((S.rc[mt] ^ TAU) & Z)) ac[mt] = D[hb[mt] + ha];
                T h[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) h[m] = cur[m][w];
                wht8(h);
#pragma unroll
                for (int mt = 0; mt < F32T; ++mt)
                    if (!((S.rc[mt] ^ TAU) & Z))
                        acc[mt] = Mfma<T>::run(ac[mt], h[S.rc[mt] ^ TAU], acc[mt]);
                if constexpr (N32 > 0) {
                    float hf[8];
#pragma unroll
                    for (int m = 0; m < 8; ++m) hf[m] = (float)h[m];
#pragma unroll
                    for (int mt = F32T; mt < MTW; ++mt)
                        if (!((S.rc[mt] ^ TAU) & Z))
                            acc32[mt - F32T] = Mfma<float>::run((float)ac[mt], hf[S.rc[mt] ^ TAU], acc32[mt - F32T]);
                }
            };
            auto request = [&](int j) { // the vector after vector j
                if (j + 1 < KSV) load_v(nxt, j + 1, srcc);
                else load_v(nxt, 0, srcn);
            };
            auto move_on = [&]() {
#pragma unroll
                for (int m = 0; m < 8; ++m) cur[m] = nxt[m];
            };
            using W0 = std::integral_constant<int, 0>;
            using W1 = std::integral_constant<int, 1>;
            if constexpr (K1 > K0) {
                if constexpr (K0 % 2 == 1) { // second half of a vector the previous class began
                    kstep(K0, W1{});
                    move_on();
                }
#pragma unroll 1
                for (int j = (K0 + 1) / 2; j < K1 / 2; ++j) {
                    request(j);
                    kstep(2 * j, W0{});
                    kstep(2 * j + 1, W1{});
                    move_on();
                }
                if constexpr (K1 % 2 == 1) { // first half of a vector
                    request(K1 / 2);
                    kstep(K1 - 1, W0{});
                    if constexpr (K1 == KS) move_on(); // its second half is padding
                }
            }
        };
        column_class(std::integral_constant<int, 0>{});
        column_class(std::integral_constant<int, 1>{});
        column_class(std::integral_constant<int, 2>{});
        column_class(std::integral_constant<int, 3>{});
        column_class(std::integral_constant<int, 4>{});
        column_class(std::integral_constant<int, 5>{});
        column_class(std::integral_constant<int, 6>{});
        column_class(std::integral_constant<int, 7>{});
    };
    int q = qa;
    auto run_mask = [&](auto zc) {
        const int qend = min(sZend[decltype(zc)::value], qb);
        for (; q < qend; ++q) {
            const int curb = (q - qa) & 1;
            const bool more = q + 1 < qb;
            if (more) {
                load_d(sList[q + 1]);
                class_src(q + 1, srcn);
            }
            run_class(zc, sD[curb]);
            if constexpr (N32 > 0) {
#pragma unroll
                for (int mt = 0; mt < N32; ++mt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[mt][r] += (double)acc32[mt][r];
                    acc32[mt] = acc32_t{0, 0, 0, 0};
                }
            }
#pragma unroll
            for (int m = 0; m < 8; ++m) srcc[m] = srcn[m];
            if (more) store_d(curb ^ 1);
            __syncthreads();
        }
    };
    run_mask(std::integral_constant<int, 0>{});
    run_mask(std::integral_constant<int, 1>{});
    run_mask(std::integral_constant<int, 2>{});
    run_mask(std::integral_constant<int, 3>{});
    run_mask(std::integral_constant<int, 4>{});
    run_mask(std::integral_constant<int, 5>{});
    run_mask(std::integral_constant<int, 6>{});
    if (tgt < 0) return;
    static_assert(!sym_parts_add(P), "parts store their sums");
    double *Lh = (part ? v.Lh2 + (int64_t)(part - 1) * v.nboxes * v.ldh : v.Lh) + (int64_t)tgt * v.ldh;
#pragma unroll
    for (int mt = 0; mt < F32T; ++mt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = gptr(tb.srow)[16 * mt + Mfma<T>::row(lane, r)];
            if (b >= 0) Lh[b] = acc[mt][r];
        }
    }
#pragma unroll
    for (int mt = F32T; mt < MTW; ++mt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = gptr(tb.srow)[16 * mt + Mfma<float>::row(lane, r)];
            if (b >= 0) Lh[b] = acc64[mt - F32T][r];
        }
    }
}

#define M2L_CASE(PP)                                                               \
    case PP:                                                                       \
        if (f32) k_m2l<PP, float><<<nb, 256, 0, s>>>(V, B);                        \
        else k_m2l<PP, double><<<nb, 256, 0, s>>>(V, B);                           \
        break;

// FP32 sign-class M2L with all rows in FP32: orders 6-8 (9-11 stay FP64)
#define M2L_SYM(PP)                                                                \
    case PP:                                                                       \
        if (f32) k_m2l_sym<PP, float><<<nb, 256, 0, s>>>(V, B);                    \
        else k_m2l_sym<PP, double><<<nb, 256, 0, s>>>(V, B);                       \
        break;
#define M2L_SYM64(PP)                                                              \
    case PP: k_m2l_sym<PP, double><<<nb, 256, 0, s>>>(V, B); break;

// Orders >= 12: one launch with every row tile; with f32 the row tiles after
// the first eight (the first 16 rows, lowest degrees, of each parity class
// stay FP64; rows are in sym_tile_class order) run on FP32 MFMA.
template <int P> void launch_symh(unsigned nb, const PlanView *V, const Bases &B, int f32, hipStream_t s)
{
    constexpr int RT = sym_row_tiles(P);
    static_assert(RT > 8 && sym_tile_class(P, 7, false) == 0 && sym_tile_class(P, 8, false) == 1, "tile order");
    if (f32) k_m2l_symh<P, 8><<<nb, 256, 0, s>>>(V, B);
    else k_m2l_symh<P, RT><<<nb, 256, 0, s>>>(V, B);
}
#define M2L_SYMH(PP) \
    case PP: launch_symh<PP>(nb, V, B, f32, s); break;

// FP32 M2L: all of it up to p = 8, the row parts after the first from
// p = 12 (orders 9-11 keep M2L in FP64); orders from 6 on run on sign
// classes (m2l_sym), from 12 on in k_m2l_symh
void launch_m2l(int p, int f32, const PlanView *V, const Bases &B, hipStream_t s)
{
    unsigned nb = (unsigned)B.b[B.n];
    if (!nb) return;
    static_assert(m2l_sym(6) && !m2l_sym(5), "dispatch below");
    switch (p) {
        M2L_CASE(0) M2L_CASE(1) M2L_CASE(2) M2L_CASE(3) M2L_CASE(4) M2L_CASE(5)
        M2L_SYM(6) M2L_SYM(7) M2L_SYM(8) M2L_SYM64(9) M2L_SYM64(10) M2L_SYM64(11)
        M2L_SYMH(12) M2L_SYMH(13) M2L_SYMH(14) M2L_SYMH(15)
    default: launch_symh<16>(nb, V, B, f32, s);
    }
}

} // namespace fmm
