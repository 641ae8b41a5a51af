// Internal declarations of the MI355X DA-FMM library (not part of the ABI).
//
// Expansion storage.  The paper's DA vectors (Sec. 2) hold Taylor
// coefficients M_a of phi_M in d = r/r^2 (multipole, Eq. P2M) and L_b of phi_L
// in d' = r - c (local, Eq. P2L), monomials ordered by degree and descending
// exponents (Table 1).  On the device every box keeps them in scaled units
// that make the translation operators independent of the level:
//     Mhat_a = w_|a| M_a / h^|a|,   w_n = (-1)^n / (2n-1)!!,
//     Lhat_b = b! L_b h^(|b|+1),
// h being the box width.  With these, the DA M2L of Sec. 2.3 becomes
//     Lhat_b += sum_a D_(a+b)(k) Mhat_a,   D_g(k) = d^g (1/|x|) at x = k,
// k the integer offset of the two boxes (the harmonic degrees of phi_M turn the
// composition into a derivative-tensor contraction), and M2M, L2L are fixed
// matrices per child octant.  The export path converts back to the DA
// convention.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace fmm {

constexpr int kMaxOrder = 16;
constexpr int kMaxDepth = 21;
constexpr int kVSlots = 189;   // M2L sources per box, one slot per offset (Sec. 3.4)
constexpr int kMaxBatch = 256; // plans per batched launch

__host__ __device__ constexpr int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ constexpr int nharm(int p) { return (p + 1) * (p + 1); }
__host__ __device__ inline int below(int n) { return n * (n + 1) * (n + 2) / 6; }
// position of d1^i d2^j d3^k in the DA order of Table 1
__host__ __device__ inline int mono_index(int i, int j, int k)
{
    int n = i + j + k, a = j + k;
    return below(n) + a * (a + 1) / 2 + k;
}
// Harmonic (compressed) order used by M2L: exponents (i, j, kz) with kz in {0,1};
// degree n holds (i, n-i, 0) for i = n..0, then (i, n-1-i, 1) for i = n-1..0.
__host__ __device__ inline int harm_index(int i, int j, int kz)
{
    int n = i + j + kz;
    return n * n + (kz == 0 ? (n - i) : (n + 1) + (n - 1 - i));
}
__host__ __device__ constexpr int pad16(int n) { return (n + 15) & ~15; }
__host__ __device__ constexpr int pad4(int n) { return (n + 3) & ~3; }
// terms of the fold (and of the unfold): harmonic (I, J, kz) collects the full
// components (I - 2a, J - 2(m - a), kz + 2m)
__host__ __device__ constexpr int fold_terms(int p)
{
    int t = 0;
    for (int n = 0; n <= p; ++n)
        for (int kz = 0; kz <= 1 && kz <= n; ++kz)
            for (int i = n - kz; i >= 0; --i) {
                const int j = n - kz - i;
                for (int m = 0; kz + 2 * m <= p; ++m)
                    for (int a = 0; a <= m; ++a)
                        if (i - 2 * a >= 0 && j - 2 * (m - a) >= 0) ++t;
            }
    return t;
}
// Additive layout of one offset's derivative table: addr(i,j,k) = k*s2 + i*s1 + j
// for x, y exponents up to 2p and z exponent up to 2 (any s1 > 2p and
// s2 > 2p (s1 + 1) keep it one-to-one).  The strides are chosen per order to
// minimise LDS bank conflicts of the M2L operand gather (64 lanes reading
// D(addr(b) + addr(a)) for 16 rows b and 4 columns a at once), within about
// 10% of the smallest table.
__host__ __device__ constexpr int dlayout_s1(int p)
{
    constexpr int t[17] = {1, 3, 6, 7, 10, 11, 13, 15, 19, 19, 24, 24, 28, 28, 30, 34, 38};
    return t[p];
}
__host__ __device__ constexpr int dlayout_s2(int p)
{
    constexpr int t[17] = {1, 11, 30, 49, 91, 125, 184, 252, 328, 392, 516, 580, 719, 773, 887, 1066, 1252};
    return t[p];
}
__host__ __device__ constexpr int dlayout_ldd(int p) { return (3 * dlayout_s2(p) + 3) & ~3; } // 16-byte rows
// entries d^g with g_z <= 2, |g| <= 2p (the ones M2L reads), rounded up to 4
__host__ __device__ constexpr int dlayout_ldc(int p)
{
    return ((2 * p + 1) * (2 * p + 2) / 2 + (2 * p) * (2 * p + 1) / 2 + (2 * p - 1) * (2 * p) / 2 + 3) & ~3;
}

// Sign classes of M2L offsets.  1/|x| is even in every coordinate, so
// D_g(s o k) = s^g D_g(k) for a sign vector s (s^g = prod s_i^g_i).  The V
// list offsets of one octant fall into 56 classes of offsets that differ only
// in sign (|k_x|, |k_y|, |k_z| fixed); with the multipoles of a class's members
// combined by a Walsh-Hadamard transform over the signs, one contraction with
// the derivative table of a single representative serves the whole class,
// output rows taking the combination that matches their parity.  The M2L
// operands are kept in parity-sorted order for this: the harmonic components
// of each parity class c (x, y, z exponent parities as bits 2, 1, 0), in
// increasing harmonic index, padded to 16 rows (output) or 4 columns (input).
constexpr int kSymClasses = 56;
__host__ __device__ constexpr int sym_class_count(int p, int c)
{
    int n = 0;
    for (int i = (c >> 2) & 1; i + (c & 1) <= p; i += 2)
        for (int j = (c >> 1) & 1; i + j + (c & 1) <= p; j += 2) ++n;
    return n;
}
__host__ __device__ constexpr int sym_row_tiles(int p)
{
    int n = 0;
    for (int c = 0; c < 8; ++c) n += (sym_class_count(p, c) + 15) / 16;
    return n;
}
// columns of a parity class are padded to a multiple of sym_colpad: 4 (one
// k-step) at every order; from p = 12 the kernel's 16-byte operand vectors
// (two k-steps) may hold the last k-step of one class and the first of the
// next
__host__ __device__ constexpr int sym_colpad(int) { return 4; }
__host__ __device__ constexpr int sym_class_ksteps(int p, int c)
{
    return (sym_class_count(p, c) + sym_colpad(p) - 1) / sym_colpad(p) * (sym_colpad(p) / 4);
}
__host__ __device__ constexpr int sym_ksteps(int p)
{
    int n = 0;
    for (int c = 0; c < 8; ++c) n += sym_class_ksteps(p, c);
    return n;
}
// orders whose M2L runs on sign classes (fewer matrix-core products from p = 6 on)
__host__ __device__ constexpr bool m2l_sym(int p) { return p >= 6; }
// blocks per M2L tile of 64 targets at sign-class orders: the tile's classes
// are split into this many contiguous parts by matrix-core work, each block
// writing its own partial sums.  Two: more, shorter blocks did not shorten the
// launch's tail as much as their per-block set-up cost (uniform 10^6 points,
// p = 8, equal parts: 0.97 ms with two, 0.96 with three, 1.07 with four; on a
// Plummer tree three were slower than two).
__host__ __device__ constexpr int sym_m2l_parts(int p) { return m2l_sym(p) ? 2 : 1; }
// Orders 6-11: the parts add their sums into Lh rows zeroed before the M2L,
// with FP64 atomics (two addends onto zero give the same sum in either order,
// more would not), so no pass over partial sums follows the launch (uniform
// 10^6 points, p = 8: 2.36 against 2.56 ms per step).  From order 12 the
// second part stores its sums to a slice of its own and the pass before the
// L2L adds them (the atomics slowed the p = 14 launch by 3%, more than that
// pass takes).
__host__ __device__ constexpr bool sym_parts_add(int p) { return m2l_sym(p) && p <= 11; }
static_assert(sym_m2l_parts(6) <= 2 && sym_m2l_parts(11) <= 2, "M2L parts add into Lh in any order");
// share (percent) of a tile's matrix-core work in its first part; the launch
// runs the first parts before the others (longest first), so that its end is
// made of the shorter blocks (uniform 10^6 points, p = 8, FP64: about 6%
// faster at 68-74 than at 50-56, slower again from 78)
constexpr int kSymFirstPart = 72;
// Order of the row tiles: by parity class, then tile within the class, up to
// p = 11; from p = 12 by tile within the class first (the first 16 rows of
// every class, then the next 16, ...): rows of a class are in increasing
// degree, so the first eight tiles hold the lowest degrees (the FP32 M2L of
// these orders keeps them in FP64).  Class and tile-in-class of row tile r:
__host__ __device__ constexpr int sym_tile_class(int p, int r, bool want_class)
{
    if (p < 12) {
        for (int c = 0; c < 8; ++c) {
            const int n = (sym_class_count(p, c) + 15) / 16;
            if (r < n) return want_class ? c : r;
            r -= n;
        }
        return -1;
    }
    for (int t = 0; t < 8; ++t)
        for (int c = 0; c < 8; ++c)
            if (16 * t < sym_class_count(p, c)) {
                if (r == 0) return want_class ? c : t;
                --r;
            }
    return -1;
}
// Folded multipoles of sign-class orders are stored so that a lane's
// operands of vw consecutive k-steps are adjacent (one 16-byte load): sorted
// column 4 ks + g (k-step ks, lane group g) sits at 4 vw (ks / vw) + vw g +
// ks % vw, vw = 2 for FP64 and 4 for FP32.
__host__ __device__ constexpr int sym_pos(int ks, int g, int vw) { return 4 * vw * (ks / vw) + vw * g + ks % vw; }
// row stride of the folded multipoles (both precisions' layouts fit)
// orders whose FP32 M2L reads an FP32 copy of the folded multipoles (above
// them the FP32 row tiles round the FP64 operands in registers)
__host__ __device__ constexpr bool m2l_f32_operands(int p) { return p <= 8; }
__host__ __device__ constexpr int folded_ld(int p)
{
    return m2l_sym(p) ? 16 * ((sym_ksteps(p) + 3) / 4) : (((p + 1) * (p + 1) + 15) & ~15);
}

// LDS exchange between the lanes of one wavefront (no workgroup barrier: the
// wavefronts of a block run independent loops)
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline uint64_t lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Walsh-Hadamard transform of the 8 members of a sign class of M2L offsets,
// h[s] <- sum_m (-1)^|m & s| h[m] (bit 2, 1, 0 of m: the member negates x, y,
// z).  For a class with zero axes Z: members that negate a zero axis
// do not exist, and only outputs r with r & Z == 0 are used, so the butterflies
// run over the other axes on the entries with no bit of Z (h[m], m & Z != 0,
// is neither read nor written).
template <int Z, typename T> __device__ inline void wht8z(T (&h)[8])
{
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!(bit & Z) && !(i & bit) && !(i & Z)) {
                const T u = h[i], w = h[i | bit];
                h[i] = u + w;
                h[i | bit] = u - w;
            }
}

// Global address-space views of device pointers.  Loads and stores through
// them compile to global_* instructions, counted by the vector-memory counter
// only; the generic (flat_*) form also counts against the LDS counter, so an
// LDS read that waits would wait for every memory load in flight as well.
template <typename T> using gp = __attribute__((address_space(1))) T *;
template <typename T> __device__ inline gp<const T> gptr(const T *p) { return (gp<const T>)p; }
template <typename T> __device__ inline gp<T> gptr(T *p) { return (gp<T>)p; }

// Morton codes: bit b of the x, y, z cell index sits at code bits 3b+2, 3b+1, 3b
// (levels up to 21).  The bits are spread and gathered with the usual shift-
// and-mask steps (5 each); only the low l bits of a cell index take part.
__host__ __device__ inline uint64_t spread3(uint64_t v) // bit b -> bit 3b
{
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}
__host__ __device__ inline uint32_t gather3(uint64_t v) // bit 3b -> bit b
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}
__host__ __device__ inline void deinterleave(uint64_t code, int l, int c[3])
{
    const uint32_t m = (1u << l) - 1;
    c[0] = (int)(gather3(code >> 2) & m);
    c[1] = (int)(gather3(code >> 1) & m);
    c[2] = (int)(gather3(code) & m);
}
__host__ __device__ inline uint64_t interleave(const int c[3], int l)
{
    const uint32_t m = (1u << l) - 1;
    return spread3((uint32_t)c[0] & m) << 2 | spread3((uint32_t)c[1] & m) << 1 | spread3((uint32_t)c[2] & m);
}

// V-list slots.  A box whose octant within its parent is o (bits ox, oy, oz)
// sees sources at offsets k = target - source with k_x in [-3,2] if ox = 0 and
// [-2,3] if ox = 1 (likewise y, z), excluding the 27 near offsets: 189 slots,
// numbered in lexicographic order of (k_x, k_y, k_z).
__host__ __device__ inline int vslot_of(int oct, int kx, int ky, int kz)
{
    int s[3] = {((oct >> 2) & 1) ? -2 : -3, ((oct >> 1) & 1) ? -2 : -3, (oct & 1) ? -2 : -3};
    int a[3] = {kx - s[0], ky - s[1], kz - s[2]};
    for (int t = 0; t < 3; ++t)
        if (a[t] < 0 || a[t] > 5) return -1;
    int nx = -1 - s[0], ny = -1 - s[1], nz = -1 - s[2]; // start of the near cube
    bool inx = a[0] >= nx && a[0] < nx + 3, iny = a[1] >= ny && a[1] < ny + 3,
         inz = a[2] >= nz && a[2] < nz + 3;
    if (inx && iny && inz) return -1;
    int clx = a[0] - nx < 0 ? 0 : (a[0] - nx > 3 ? 3 : a[0] - nx);
    int cly = a[1] - ny < 0 ? 0 : (a[1] - ny > 3 ? 3 : a[1] - ny);
    int clz = a[2] - nz < 0 ? 0 : (a[2] - nz > 3 ? 3 : a[2] - nz);
    int skipped = clx * 9 + (inx ? (cly * 3 + (iny ? clz : 0)) : 0);
    return a[0] * 36 + a[1] * 6 + a[2] - skipped;
}

// Per-order constant tables (device pointers), built once per order and device.
struct OrderTables {
    int p, nc, nh, ldm, ldh, ldd;   // ldd: size of one offset's table in the additive (LDS) layout
    int ldc;                        // stride of one offset's compact table
    int d3;                         // x stride of the additive D layout
    int ldmh;                       // row stride of the folded multipoles
    const int *mpos;    // [ldmh] harmonic index of each folded position (-1 padding)
    const int *mposf;   // same for the FP32 copy
    const double *D;    // [343][ldc] derivative tensors d^g(1/|x|) at integer x, compact
    const float *Df;    // same in FP32
    const int *dmap;    // [ldc] additive-layout address of each compact entry
    const int *offs;    // [8][189] packed offsets (kx+3)*49 + (ky+3)*7 + (kz+3)
    const int *hoff;    // [ldh] additive D address of each harmonic index (-1 padding)
    const double *GH;   // [8][nh][nh] L2L on the harmonic components, GH[o][a][c] = d Lh'_c / d Lh_a
    const double *TM;   // [8][ldmh][ldmh] M2M on the folded positions, TM[o][a][c] = d Mh'_c / d Mh_a
    const double *HR;   // [nh][nc] full harmonic Mhat from the folded (harmonic-order) components, HR[c][b]
    const int *hpos;    // [nh] folded position of each harmonic component
    const int *hposf;   // [nh] same in the FP32 copy
    const double *FP2M; // [nc][ldh] raw moments -> folded components in harmonic order (P2M, then fold)
    const double *P2L;  // [nc][ldh] inverse moments -> harmonic Lhat
    const int *fold_off; const int *fold_idx; const double *fold_c;     // Mhat -> folded
    const int *unfold_off; const int *unfold_idx; const double *unfold_c; // Lh -> Lhat
    // sign classes (orders with m2l_sym): rows and columns in parity order,
    // and per octant the 56 classes: representative offset (packed as in offs)
    // | zero-axis mask << 16, and the V slot of each member, indexed by the
    // axes it negates (bits 2, 1, 0 = x, y, z; -1 where there is none)
    const int *srow;    // [16 row tiles] harmonic index of each sorted row (-1 padding)
    const int *scol;    // [4 k-steps] harmonic index of each sorted column (-1 padding)
    const int *srep;    // [8][56]
    const int *smem;    // [8][56][8]
    const int *sslot;   // [8][189] class of each V slot
    const double *inv_fact;     // [nc] 1/b!
    const double *inv_w;        // [p+1] 1/w_n = (-1)^n (2n-1)!!
    const int *exps;            // [nc] packed exponents i | j<<8 | k<<16
};

// Rotation-based M2L factors of one order (device pointers): per class of
// offsets (|k_x|, |k_y|, |k_z|) the multipole map F and local map B (per
// degree, [input][output]), the axial blocks A per distinct |k|^2 and the
// block of each class (rotation.hip).
struct RotTables {
    const double *F, *B, *A;
    const int *aidx;
};

// Everything a kernel needs to know about one plan (lives in device memory).
struct PlanView {
    int p, nc, nh, ldm, ldh, ldmh;
    int precision;          // FMM_FP64 / FMM_MIXED
    int mixed_m2l;          // FP32 MFMA M2L
    int depth, D;
    int32_t n, nboxes, nleaves, nxtgt, nslots;
    double lo[3], W;
    const int32_t *level, *parent, *child_begin, *nchild, *first, *count;
    const uint64_t *morton;
    const int32_t *perm;                // sorted position -> original index
    const double *xs, *ys, *zs;         // sorted positions (SoA)
    const int64_t *U_off, *V_off, *W_off, *X_off;
    const int32_t *U_src, *W_src, *X_src;
    const int32_t *wsrc;                // [boxes] 1 for boxes in some W list (M2P sources), or null
    const int32_t *m2l_tgt;             // M2L targets, octant-grouped, groups padded to 64
    const int32_t *vslot;               // [boxes][189] M2L source per offset slot, or -1
    const int32_t *leaves;              // leaf boxes
    const int32_t *xtgt;                // boxes with a non-empty X list
    const int32_t *lvl_nonleaf;         // non-leaf boxes grouped by level
    const int32_t *lvl_nonleaf_off;     // [depth+2] ranges into lvl_nonleaf
    const OrderTables *tab;             // device copy of the order tables
    const RotTables *rot;               // rotation-based M2L factors (device), or null
    // evaluation buffers
    double *qs;                         // sorted charges
    double *M, *Mh, *Lh, *L;            // [boxes][ldm] / [boxes][ldmh] / [boxes][ldh]
    double *Lh2;                        // orders >= 12: [m2l_parts - 1][boxes][ldh] partial sums
                                        // of the M2L class parts after the first (else null)
    int m2l_parts;                      // blocks per M2L tile (1 below the sign-class orders)
    float *Mhf;                         // FP32 folded multipoles (mixed M2L)
    // softened kernel 1/sqrt(|x|^2 + eps^2) (kernel == 1): full Cartesian
    // expansions in M and L, derivative tables per level
    int kernel;
    double eps2;                        // eps^2 (P2P)
    const double *Dsoft;                // [depth - 1][343][soft_ldc] d^g K at the offsets of levels 2..depth
    const int *soft_map;                // [soft_ldc] LDS address of each compact entry (dense cube)
    const double *zrow;                 // [ldm] zeros: operand of absent M2L sources
    double *phi_near, *fld_near;        // near-field (P2P) part, sorted order
    // caller's arrays for this evaluation
    const double *q_in;
    double *phi_out, *fld_out;
};

// Work split of a batched launch: plan k owns items [b[k], b[k+1]).
struct Bases {
    int n;
    int b[kMaxBatch + 1];
};

__device__ inline int find_plan(const Bases &B, int item)
{
    int lo = 0, hi = B.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (B.b[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

inline unsigned ceil_div(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// Work groups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Maps the i-th block (of n) so that every XCD receives one contiguous range of
// items: neighbouring items (Morton-adjacent boxes sharing interaction-list
// sources) then share an L2.  Bijective on [0, n).
constexpr int kXCDs = 8;
__device__ inline int xcd_remap(int i, int n)
{
    const int x = i % kXCDs, y = i / kXCDs, q = n / kXCDs, r = n % kXCDs;
    return x * q + (x < r ? x : r) + y;
}

} // namespace fmm
