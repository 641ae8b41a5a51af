// Evaluation kernels other than M2L.  Every kernel serves a batch of plans:
// block b belongs to the plan k with Bases.b[k] <= b < Bases.b[k+1].
//
// Scaled units (h = box width): Mhat_a = w_|a| M_a / h^|a|, Lhat_b = b! L_b h^(|b|+1).
//   P2M  (Sec. 2.1) Mhat_a = sum_g P[g][a] Q_g with raw moments Q_g = sum q u^g,
//        u = (x - c)/h; one wavefront per leaf, one lane per moment, so the
//        per-box reduction is an in-lane sequential sum (deterministic); the
//        fixed matrix P is then applied to 16 leaves at a time on MFMA.
//   M2M  (Sec. 2.2) parent Mhat = sum over children of S_octant * child Mhat,
//        applied during evaluation to the folded components (TM_octant) and
//        in full only to complete the expansions for export.
//   L2L  (Sec. 2.5) child Lhat += G_octant * parent Lhat, applied to the
//        harmonic components (GH_octant) before the leaves are unfolded.
//   L2P / M2P (Sec. 3.2) share one evaluation routine (nested Horner with the
//        gradient); M2P evaluates phi = |d| phi_M(d), d = y/|y|^2 (Eq. P2M_phi).
//   P2L  (Sec. 2.4) Lhat_b += q d^b(1/|x|) at x = (c - x_i)/h, through inverse
//        moments and a fixed harmonic map.
//   P2P  (Sec. 1) pairwise sum over the U list, skipping j == i and r == 0.
#include "ops.h"

#include <type_traits>

namespace fmm {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ inline void box_geom(const PlanView &v, int b, double cen[3], double &h)
{
    int l = v.level[b], c[3];
    deinterleave(v.morton[b], l, c);
    h = v.W / (double)(1ll << l);
    for (int k = 0; k < 3; ++k) cen[k] = v.lo[k] + ((double)c[k] + 0.5) * h;
}

__device__ inline int degree_of(int idx)
{
    int d = 0;
    while (below(d + 1) <= idx) ++d;
    return d;
}

// ---------------- charges in sorted order ----------------
__global__ __launch_bounds__(256) void k_permute_q(const PlanView *V, Bases B)
{
    int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    int i = (blockIdx.x - B.b[k]) * 256 + threadIdx.x;
    if (i < v.n) v.qs[i] = v.q_in[v.perm[i]];
}

// ---------------- moments by columns (P2M, P2L) ----------------
// Both P2M and P2L sum moments W_g = sum_t w_t u_t^g over all monomials g of
// degree <= P of a set of particles (P2M: u = (x - c)/h, w = q; P2L: the
// inverted u = x'/|x'|^2, w = q/|x'|).  Lane l owns the columns (b, c) =
// (g_y, g_z) numbered l, l + 64, ... by degree b + c and sums every a = g_x of
// them: per particle a lane forms one product u_y^b u_z^c from the powers
// staged in LDS and adds it times w u_x^a, formed in registers, to its
// P + 1 - (b + c) sums (p = 10: 12 mults, 12 FMAs and 5 LDS reads, where a lane
// per moment reads three staged powers for each of its moments).
__host__ __device__ constexpr int col_degree(int j) // degree b + c of column j
{
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= j) ++s;
    return s;
}
template <int P>
struct Cols {
    static constexpr int NCOL = (P + 1) * (P + 2) / 2, RC = (NCOL + 63) / 64;
    static constexpr int CH = 32; // particles per LDS chunk
    typedef double Pow[P + 1][CH + 1];
};
template <int P>
__device__ inline void col_setup(int lane, int (&cb)[Cols<P>::RC], int (&cc)[Cols<P>::RC],
                                 double (&acc)[Cols<P>::RC][P + 1])
{
#pragma unroll
    for (int r = 0; r < Cols<P>::RC; ++r) {
        const int j = lane + 64 * r, d = j < Cols<P>::NCOL ? col_degree(j) : 0;
        cc[r] = j < Cols<P>::NCOL ? j - d * (d + 1) / 2 : 0;
        cb[r] = d - cc[r];
#pragma unroll
        for (int a = 0; a <= P; ++a) acc[r][a] = 0.0;
    }
}
// stage particle `slot` of a chunk: powers of u_y, u_z and the pair (u_x, w)
template <int P>
__device__ inline void col_stage(typename Cols<P>::Pow &py, typename Cols<P>::Pow &pz, double2 *xw, int slot,
                                 double ux, double uy, double uz, double w)
{
    double a = 1.0, c = 1.0;
#pragma unroll
    for (int t = 0; t <= P; ++t) {
        py[t][slot] = a; pz[t][slot] = c;
        a *= uy; c *= uz;
    }
    xw[slot] = make_double2(ux, w);
}
// add the m staged particles to the lane's column sums
template <int P>
__device__ inline void col_add(const typename Cols<P>::Pow &py, const typename Cols<P>::Pow &pz, const double2 *xw,
                               int m, const int (&cb)[Cols<P>::RC], const int (&cc)[Cols<P>::RC],
                               double (&acc)[Cols<P>::RC][P + 1])
{
#pragma unroll 1
    for (int t = 0; t < m; ++t) {
        const double2 u = xw[t];
        double xp[P + 1];
        xp[0] = u.y;
#pragma unroll
        for (int a = 1; a <= P; ++a) xp[a] = xp[a - 1] * u.x;
#pragma unroll
        for (int r = 0; r < Cols<P>::RC; ++r) {
            const double yz = py[cb[r]][t] * pz[cc[r]][t];
            // columns of slot r have degree >= col_degree(64 r)
#pragma unroll
            for (int a = 0; a <= P - col_degree(64 * r); ++a) acc[r][a] = fma(xp[a], yz, acc[r][a]);
        }
    }
}
// W[mono_index(a, b, c)] for every monomial of degree <= P
template <int P>
__device__ inline void col_store(double *W, int lane, const int (&cb)[Cols<P>::RC], const int (&cc)[Cols<P>::RC],
                                 const double (&acc)[Cols<P>::RC][P + 1])
{
#pragma unroll
    for (int r = 0; r < Cols<P>::RC; ++r) {
        if (lane + 64 * r >= Cols<P>::NCOL) continue;
#pragma unroll
        for (int a = 0; a <= P; ++a)
            if (a <= P - cb[r] - cc[r]) W[mono_index(a, cb[r], cc[r])] = acc[r][a];
    }
}

// ---------------- P2M ----------------
// Raw moments Q_g = sum_i q_i ((x_i - c)/h)^g of a leaf (Eq. P2M in scaled
// units), one wavefront per leaf, by columns.
template <int P>
__global__ __launch_bounds__(64) void k_p2m(const PlanView *V, Bases B)
{
    using C = Cols<P>;
    __shared__ typename C::Pow py, pz;
    __shared__ double2 xw[C::CH];
    int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int box = v.leaves[blockIdx.x - B.b[k]];
    const int lane = threadIdx.x;
    double cen[3], h;
    box_geom(v, box, cen, h);
    const double ih = 1.0 / h;
    int cb[C::RC], cc[C::RC];
    double acc[C::RC][P + 1];
    col_setup<P>(lane, cb, cc, acc);
    const int f = v.first[box], cnt = v.count[box];
    for (int s0 = 0; s0 < cnt; s0 += C::CH) {
        const int m = cnt - s0 < C::CH ? cnt - s0 : C::CH;
        __syncthreads(); // the previous chunk is consumed
        if (lane < m) {
            const int i = f + s0 + lane;
            col_stage<P>(py, pz, xw, lane, (v.xs[i] - cen[0]) * ih, (v.ys[i] - cen[1]) * ih,
                         (v.zs[i] - cen[2]) * ih, v.qs[i]);
        }
        __syncthreads();
        col_add<P>(py, pz, xw, m, cb, cc, acc);
    }
    // raw moments go to the (not yet used) local-expansion row of the leaf;
    // k_p2m_fold turns them into the folded (and, for M2P sources, full) Mhat
    col_store<P>(v.L + (int64_t)box * v.ldm, lane, cb, cc, acc);
}

// Folded multipoles of the leaves straight from their raw moments:
// Mh = FP2M^t Q (P2M followed by the fold, one matrix; both keep the degree).
// A wavefront takes 16 leaves and walks the degrees: it loads the 16 leaves'
// moments of degree n once (the B operands of every k-step), then runs the
// 16-row tiles of that degree's 2n+1 folded components on FP64 MFMA.  A
// wavefront holding a leaf that M2P reads (a W-list source) also rebuilds the
// full multipoles of degree n from the folded ones, Mhat_n = HR_n^t Mh_n
// (exact: each degree part of a multipole is harmonic): the MFMA result of a
// folded 16-row tile, register r of lane (kq, col) holding row 4r + kq of
// leaf col, is exactly the B operand of the tile's four k-steps, so the
// reconstruction reads it from registers.
// Results go to the components' folded positions (and the FP32 copy for the
// FP32 M2L); the padding positions of the rows are written as zeros (the M2L
// reads them as operands of padded columns).
template <int P>
__global__ __launch_bounds__(256) void k_p2m_fold(const PlanView *V, Bases B)
{
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
    const int li = (blockIdx.x - B.b[k]) * 64 + wave * 16 + col;
    const int leaf = li < v.nleaves ? v.leaves[li] : -1;
    if (!__any(leaf >= 0)) return;
    constexpr int NC = ncoef(P), NH = nharm(P), LDM = pad16(NC), LDH = pad16(NH);
    const int ldmh = v.ldmh;
    const OrderTables &t = *v.tab;
    const auto Q = gptr(v.L + (int64_t)(leaf >= 0 ? leaf : 0) * LDM);
    const auto FT = gptr(t.FP2M), HR = gptr(t.HR);
    const auto Mh = gptr(v.Mh + (int64_t)(leaf >= 0 ? leaf : 0) * ldmh);
    const bool full = v.wsrc && __any(leaf >= 0 && v.wsrc[leaf]);
    const bool mine = full && leaf >= 0 && v.wsrc[leaf];
    const auto Mf = gptr(v.M + (int64_t)(leaf >= 0 ? leaf : 0) * LDM);
    const bool f32 = v.Mhf != nullptr; // FP32 copy for the FP32 M2L
#pragma unroll
    for (int n = 0; n <= P; ++n) {
        const int g0 = below(n), mn = (n + 1) * (n + 2) / 2, KS = (mn + 3) / 4;
        double q[(P + 1) * (P + 2) / 8 + 1];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int g = 4 * s + kq;
            q[s] = leaf >= 0 && g < mn ? Q[g0 + g] : 0.0;
        }
        // folded components n^2 .. (n+1)^2 - 1
        double4_t fo[(2 * P + 16) / 16];
#pragma unroll
        for (int t0 = 0; t0 < 2 * n + 1; t0 += 16) {
            const int c = n * n + t0 + col, cend = (n + 1) * (n + 1);
            double4_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int g = 4 * s + kq;
                const double a = c < cend && g < mn ? FT[(int64_t)(g0 + g) * LDH + c] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, q[s], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) { // f64 layout: lane l reg r -> row 4r + l/16
                const int cr = n * n + t0 + 4 * r + kq;
                if (leaf >= 0 && cr < cend) {
                    Mh[t.hpos[cr]] = acc[r];
                    if (f32) gptr(v.Mhf)[(int64_t)leaf * ldmh + t.hposf[cr]] = (float)acc[r];
                }
            }
            fo[t0 / 16] = acc; // rows >= (n+1)^2 are zero
        }
        if (!full) continue;
        // full multipole of degree n, monomials g0 .. g0 + mn - 1
        const int cend = (n + 1) * (n + 1), KF = (2 * n + 4) / 4;
#pragma unroll
        for (int m0 = 0; m0 < mn; m0 += 16) {
            double4_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KF; ++s) {
                const int c = n * n + 4 * s + kq;
                const double a = c < cend && m0 + col < mn ? HR[(int64_t)c * NC + g0 + m0 + col] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, fo[s / 4][s % 4], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int g = m0 + 4 * r + kq;
                if (mine && g < mn) Mf[g0 + g] = acc[r];
            }
        }
    }
    if (leaf < 0) return;
    for (int pos = kq; pos < ldmh; pos += 4) { // padding of the folded rows
        if (t.mpos[pos] < 0) Mh[pos] = 0.0;
        if (f32 && t.mposf[pos] < 0) gptr(v.Mhf)[(int64_t)leaf * ldmh + pos] = 0.f;
    }
    if (mine)
        for (int b = NC + kq; b < LDM; b += 4) Mf[b] = 0.0;
}

constexpr int kPG = 16; // parents per translation block

// Child of `parent` in octant o, or -1: the children are consecutive and their
// Morton codes are loaded together (a non-leaf has at least one child).
__device__ inline int child_in_octant(const PlanView &v, int parent, int o)
{
    if (parent < 0) return -1;
    const int cb = gptr(v.child_begin)[parent], ncd = gptr(v.nchild)[parent];
    uint64_t mk[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) mk[i] = gptr(v.morton)[cb + (i < ncd ? i : ncd - 1)];
    int ch = -1;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (i < ncd && (int)(mk[i] & 7) == o) ch = cb + i;
    return ch;
}

// acc += A^t x for one 16-row tile: A [K][lda] in memory (rows a, column
// bA), x the lane's source vector; k-steps of four in batches of 16 whose
// loads are all issued before the first product.  Entries a >= K and
// lanes without a source (xok false) contribute zero; k-steps below s_lo
// (whose entries of A are zero for the tile's rows) are skipped.
template <int K>
__device__ inline void mfma_rows(const double *A, int lda, int bA, bool aok, const double *x, bool xok, int kq,
                                 double4_t &acc, int s_lo = 0)
{
    constexpr int KS = (K + 3) / 4, CHK = 16;
#pragma unroll
    for (int s0 = 0; s0 < KS; s0 += CHK) {
        if (s0 + CHK <= s_lo) continue; // (block-uniform)
        double av[CHK], bv[CHK];
#pragma unroll
        for (int t = 0; t < CHK; ++t) {
            if (s0 + t >= KS) break;
            const int a = 4 * (s0 + t) + kq, ac = a < K ? a : K - 1;
            const double ta = gptr(A)[(int64_t)ac * lda + bA], tx = gptr(x)[ac];
            av[t] = aok && a < K ? ta : 0.0;
            bv[t] = xok && a < K ? tx : 0.0;
        }
#pragma unroll
        for (int t = 0; t < CHK; ++t) {
            if (s0 + t >= KS) break;
            if (s0 + t >= s_lo) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], acc, 0, 0, 0);
        }
    }
}

// ---------------- M2M on the folded components ----------------
// The far field of a multipole, hence its translation truncated at degree p,
// depends only on its folded vector: Mh(parent) = sum_o TM_o^t Mh(child_o),
// TM_o a (folded positions)^2 matrix.  A block takes 16 parents of one level,
// one wavefront per child octant (16x16x4 FP64 MFMA): the wavefront loads its
// children's folded vectors once (the B operands of every k-step) and runs
// the row tiles of the parents' vectors (all of them, or at levels with few
// parents a share, m2m_row_split); the eight octants' partial tiles are
// summed in octant order through LDS.
template <int P>
__global__ __launch_bounds__(512) void k_m2mh(const PlanView *V, Bases B, int level)
{
    __shared__ double4_t red[8][64];
    constexpr int LD = folded_ld(P), MT = LD / 16, KS = LD / 4;
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int o = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, col = lane & 15, kq = lane >> 4;
    const int lb = v.lvl_nonleaf_off[level], le = v.lvl_nonleaf_off[level + 1];
    const int rs = m2m_row_split(MT, (le - lb + kPG - 1) / kPG);
    const int g = (blockIdx.x - B.b[k]) / rs, rg = (blockIdx.x - B.b[k]) - g * rs;
    const int pidx = lb + g * kPG + col;
    const int parent = pidx < le ? v.lvl_nonleaf[pidx] : -1;
    const int ch = child_in_octant(v, parent, o); // child of this lane's parent in octant o
    const bool any = __any(ch >= 0);
    const auto X = gptr(v.Mh + (int64_t)(ch >= 0 ? ch : 0) * LD);
    double b[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st) b[st] = ch >= 0 ? X[4 * st + kq] : 0.0;
    const auto T = gptr(v.tab->TM + (int64_t)o * LD * LD);
    for (int mt = rg * (MT / rs); mt < (rg + 1) * (MT / rs); ++mt) {
        double4_t acc = {0, 0, 0, 0};
        if (any) {
#pragma unroll
            for (int s0 = 0; s0 < KS; s0 += 16) { // A operands in batches of 16 k-steps
                double a[16];
#pragma unroll
                for (int st = 0; st < 16 && s0 + st < KS; ++st)
                    a[st] = T[(int64_t)(4 * (s0 + st) + kq) * LD + mt * 16 + col];
#pragma unroll
                for (int st = 0; st < 16 && s0 + st < KS; ++st)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[s0 + st], acc, 0, 0, 0);
            }
        }
        red[o][lane] = acc;
        __syncthreads();
        if (o == 0 && parent >= 0) {
            double4_t sum = red[0][lane];
#pragma unroll
            for (int w = 1; w < 8; ++w) sum += red[w][lane]; // fixed order
#pragma unroll
            for (int r = 0; r < 4; ++r) // f64 layout: lane l reg r -> row 4r + l/16
                gptr(v.Mh)[(int64_t)parent * LD + mt * 16 + 4 * r + kq] = sum[r];
        }
        __syncthreads();
    }
}

// Parents' FP32 operand copy (mixed M2L) and, for plans with W lists, their
// full multipoles for M2P, from the folded ones: one wavefront per non-leaf
// box of level >= 2 (full = 0: FP32 copy only, 1: also the full multipoles
// of M2P sources; the fold writes those of the leaves).  full = 2 (export):
// the full multipoles of every box, leaf or not, of any level, and nothing
// else.
__global__ __launch_bounds__(256) void k_parent_mh(const PlanView *V, Bases B, int full)
{
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int box = (blockIdx.x - B.b[k]) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (box >= v.nboxes || (full != 2 && (v.nchild[box] == 0 || v.level[box] < 2))) return;
    const OrderTables &t = *v.tab;
    const auto Mh = gptr(v.Mh + (int64_t)box * v.ldmh);
    if (v.Mhf && full != 2)
        for (int c = lane; c < v.ldmh; c += 64) {
            const int h = t.mposf[c];
            gptr(v.Mhf)[(int64_t)box * v.ldmh + c] = h >= 0 ? (float)Mh[t.hpos[h]] : 0.f;
        }
    if (!full || (full == 1 && (!v.wsrc || !v.wsrc[box]))) return; // only M2P sources need it
    // the reconstruction keeps the degree: coefficient b of degree n comes
    // from the 2n + 1 folded components n^2 .. (n + 1)^2 - 1 alone
    const auto HR = gptr(t.HR);
    for (int b = lane; b < v.ldm; b += 64) {
        double s = 0.0;
        if (b < v.nc) {
            int n = 0;
            while (below(n + 1) <= b) ++n;
            for (int c = n * n; c < (n + 1) * (n + 1); ++c) s += HR[(int64_t)c * v.nc + b] * Mh[t.hpos[c]];
        }
        gptr(v.M)[(int64_t)box * v.ldm + b] = s;
    }
}

// ---------------- L2L on the harmonic components ----------------
// Lh(child) += GH_o^t Lh(parent): a block computes 16 rows of 16 parents of
// one level, one wavefront per child octant (16x16x4 FP64 MFMA), and adds the
// product of octant o to the octant-o children.
template <int P>
__global__ __launch_bounds__(512) void k_l2lh(const PlanView *V, Bases B, int level)
{
    constexpr int NH = nharm(P), LDH = pad16(NH), MT = LDH / 16;
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int item = blockIdx.x - B.b[k];
    const int nh = NH, ldh = LDH, g = item / MT, mt = item - g * MT;
    const int o = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, col = lane & 15, kq = lane >> 4;
    const int lb = v.lvl_nonleaf_off[level], le = v.lvl_nonleaf_off[level + 1];
    const int pidx = lb + g * kPG + col;
    const int parent = pidx < le ? v.lvl_nonleaf[pidx] : -1;
    const int ch = child_in_octant(v, parent, o); // child of this lane's parent in octant o
    if (!__any(ch >= 0)) return;
    const int bA = mt * 16 + col;
    // the shift keeps or lowers the degree: rows of degree >= d (the tile's
    // lowest) take nothing from inputs of degree < d, the first d^2 harmonic
    // components
    int d = 0;
    while ((d + 1) * (d + 1) <= mt * 16) ++d;
    double4_t acc = {0, 0, 0, 0};
    mfma_rows<NH>(v.tab->GH + (int64_t)o * nh * nh, nh, bA < nh ? bA : nh - 1, bA < nh,
                  v.Lh + (int64_t)(parent >= 0 ? parent : 0) * ldh, parent >= 0, kq, acc, d * d / 4);
    if (ch < 0) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int b = mt * 16 + 4 * r + kq; // f64 layout: lane l reg r -> row 4r + l/16
        if (b < nh) gptr(v.Lh)[(int64_t)ch * ldh + b] += acc[r];
    }
}

// Before the L2L, plans whose M2L stores its rows (orders below 6 and from 12
// on): Lh rows of boxes (level >= 2) without M2L or P2L contributions are set
// to zero, and from order 12 the partial sums of the other M2L class parts
// (Lh2 slices) are added in part order.
__global__ __launch_bounds__(256) void k_lh_init(const PlanView *V, Bases B)
{
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int box = (blockIdx.x - B.b[k]) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (box >= v.nboxes || v.level[box] < 2) return;
    const bool has_v = v.V_off[box + 1] > v.V_off[box], has_x = v.X_off[box + 1] > v.X_off[box];
    const auto Lh = gptr(v.Lh + (int64_t)box * v.ldh);
    if (!has_v && !has_x) {
        for (int a = lane; a < v.ldh; a += 64) Lh[a] = 0.0;
    } else if (has_v && v.Lh2) {
        const int64_t slice = (int64_t)v.nboxes * v.ldh;
        const auto Lh2 = gptr(v.Lh2 + (int64_t)box * v.ldh);
        for (int a = lane; a < v.ldh; a += 64) {
            double s = Lh[a];
            for (int i = 0; i < v.m2l_parts - 1; ++i) s += Lh2[i * slice + a];
            Lh[a] = s;
        }
    }
}

// Plans whose M2L parts add into Lh (orders 6-11): every row zeroed before
// the M2L (two doubles per thread).
__global__ __launch_bounds__(256) void k_lh_zero(const PlanView *V, Bases B)
{
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int64_t i = 2 * ((int64_t)(blockIdx.x - B.b[k]) * 256 + threadIdx.x), n = (int64_t)v.nboxes * v.ldh;
    typedef double d2 __attribute__((ext_vector_type(2)));
    if (i < n) *(d2 *)(v.Lh + i) = d2{0.0, 0.0}; // ldh is a multiple of 16
}

// ---------------- unfold the M2L result to full local expansions ----------------
// Same layout as the fold: 16 boxes per block, tables and the box's Lhat row
// in LDS.
template <int P>
__global__ __launch_bounds__(256) void k_unfold(const PlanView *V, Bases B, int leaves_only)
{
    constexpr int NC = ncoef(P), NT = fold_terms(P), LDM = pad16(NC), LDH = pad16(nharm(P));
    __shared__ int sOff[NC + 1], sIdx[NT];
    __shared__ double sC[NT];
    __shared__ double sRow[4][LDH];
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const OrderTables &t = *v.tab;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int e = tid; e < NT; e += 256) { sIdx[e] = gptr(t.unfold_idx)[e]; sC[e] = gptr(t.unfold_c)[e]; }
    for (int e = tid; e <= NC; e += 256) sOff[e] = gptr(t.unfold_off)[e];
    __syncthreads();
    const int first = (blockIdx.x - B.b[k]) * kRemapBoxes + 4 * w;
    for (int i = 0; i < 4; ++i) {
        const int box = first + i;
        if (box >= v.nboxes) break;
        if (leaves_only && v.nchild[box] > 0) continue;
        // local expansions exist from level 2 on (Lh complete after the L2L)
        double *L = v.L + (int64_t)box * LDM;
        if (v.level[box] < 2) {
            for (int b = lane; b < LDM; b += 64) gptr(L)[b] = 0.0;
            continue;
        }
        const auto Lh = gptr(v.Lh + (int64_t)box * LDH);
        for (int a = lane; a < LDH; a += 64) sRow[w][a] = Lh[a];
        wave_sync();
        for (int b = lane; b < LDM; b += 64) {
            double s = 0.0;
            if (b < NC)
                for (int e = sOff[b]; e < sOff[b + 1]; ++e) s += sC[e] * sRow[w][sIdx[e]];
            gptr(L)[b] = s;
        }
        wave_sync();
    }
}

// ---------------- P2L (X list) ----------------
// Lhat_b(B) += sum_i q_i d^b(1/|x|) at x_i' = (c_B - x_i)/h_B (Sec. 2.4 in
// scaled units).  With d^b(1/|x|) = (-1)^n (2n-1)!! pi(x^b)/|x|^(2n+1), the
// harmonic components are a fixed map (table P2L) of the inverse moments
// W_g = sum_i q_i x'^g / |x'|^(2|g|+1) = sum_i w_i u_i^g, with u = x'/|x'|^2
// and w = q/|x'| (the Kelvin inversion of the particle about the centre).
// One wavefront per target box accumulates W by columns over the particles of
// its X list; k_p2l_transform then applies the map on MFMA for 16 boxes at a
// time.
template <int P>
__global__ __launch_bounds__(64) void k_p2l(const PlanView *V, Bases B)
{
    using C = Cols<P>;
    __shared__ typename C::Pow py, pz;
    __shared__ double2 xw[C::CH];
    int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int box = v.xtgt[blockIdx.x - B.b[k]];
    const int lane = threadIdx.x;
    double cen[3], h;
    box_geom(v, box, cen, h);
    const double ih = 1.0 / h;
    int cb[C::RC], cc[C::RC];
    double acc[C::RC][P + 1];
    col_setup<P>(lane, cb, cc, acc);
    // the X list's source leaves, 64 at a time, lane l holding entry xb + l
    const int64_t x0 = v.X_off[box], x1 = v.X_off[box + 1];
    for (int64_t xb = x0; xb < x1; xb += 64) {
        int lf = 0, lc = 0;
        if (xb + lane < x1) { const int src = v.X_src[xb + lane]; lf = v.first[src]; lc = v.count[src]; }
        const int ne = x1 - xb < 64 ? (int)(x1 - xb) : 64;
        for (int e = 0; e < ne; ++e) {
            const int f = __builtin_amdgcn_readlane(lf, e), cnt = __builtin_amdgcn_readlane(lc, e);
            for (int s0 = 0; s0 < cnt; s0 += C::CH) {
                const int m = cnt - s0 < C::CH ? cnt - s0 : C::CH;
                __syncthreads(); // the previous chunk is consumed
                if (lane < m) {
                    const int i = f + s0 + lane;
                    const double x = (cen[0] - v.xs[i]) * ih, y = (cen[1] - v.ys[i]) * ih, z = (cen[2] - v.zs[i]) * ih;
                    const double ir2 = 1.0 / (x * x + y * y + z * z);
                    col_stage<P>(py, pz, xw, lane, x * ir2, y * ir2, z * ir2, v.qs[i] * sqrt(ir2));
                }
                __syncthreads();
                col_add<P>(py, pz, xw, m, cb, cc, acc);
            }
        }
    }
    col_store<P>(v.L + (int64_t)box * v.ldm, lane, cb, cc, acc); // L is free until the unfold stage
}

__device__ inline int harm_degree(int c)
{
    int n = 0;
    while ((n + 1) * (n + 1) <= c) ++n;
    return n;
}

__global__ __launch_bounds__(64) void k_p2l_transform(const PlanView *V, Bases B)
{
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int item = blockIdx.x - B.b[k];
    const int MT = v.ldh / 16, g = item / MT, mt = item - g * MT;
    const int lane = threadIdx.x, col = lane & 15, kq = lane >> 4;
    const int bi = g * 16 + col;
    const int box = bi < v.nxtgt ? v.xtgt[bi] : -1;
    const int nc = v.nc, nh = v.nh, ldh = v.ldh;
    const int cA = mt * 16 + col;
    const double *T = v.tab->P2L;
    const int dlo = harm_degree(mt * 16 < nh ? mt * 16 : nh - 1);
    const int dhi = harm_degree(mt * 16 + 15 < nh ? mt * 16 + 15 : nh - 1);
    const int k0 = below(dlo) & ~3, k1 = below(dhi + 1);
    const double *W = box >= 0 ? v.L + (int64_t)box * v.ldm : nullptr;
    double4_t acc = {0, 0, 0, 0};
#pragma unroll 4
    for (int kk = k0; kk < k1; kk += 4) {
        const int a = kk + kq;
        const double av = (cA < nh && a < nc) ? T[(int64_t)a * ldh + cA] : 0.0;
        const double bv = (W && a < nc) ? W[a] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    if (box < 0) return;
    const bool has_v = v.V_off[box + 1] > v.V_off[box]; // M2L wrote this row?
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int c = mt * 16 + 4 * r + kq;
        if (c < nh) {
            double *dst = v.Lh + (int64_t)box * ldh + c;
            *dst = (has_v ? *dst : 0.0) + acc[r];
        }
    }
}

// ---------------- far field at the targets: L2P + M2P ----------------
// Position of the coefficient of x^i y^j z^k in the order the nested Horner
// below visits them (i, then j, then k descending), so that its reads are
// consecutive and can be merged into wide LDS reads.
template <int P>
__device__ constexpr int horner_pos(int i, int j, int k)
{
    // the (P - i)(P - i + 1)(P - i + 2)/6 coefficients of larger x exponents,
    // then the (P - i - j)(P - i - j + 1)/2 of this one with larger y exponents
    const int a = P - i, b = P - i - j;
    return a * (a + 1) * (a + 2) / 6 + b * (b + 1) / 2 + (b - k);
}
// position of DA coefficient a (exponents packed i | j << 8 | k << 16)
template <int P>
__device__ inline int horner_pos_of(int packed)
{
    return horner_pos<P>(packed & 255, (packed >> 8) & 255, (packed >> 16) & 255);
}

// f = sum_a c_a x^a y^b z^c and its gradient, nested Horner in z, y, x; c in
// horner_pos order
template <int P>
__device__ inline void eval_poly(const double *c, double x, double y, double z, double &f,
                                 double &fx, double &fy, double &fz)
{
    f = fx = fy = fz = 0.0;
    int h = 0;
#pragma unroll
    for (int i = P; i >= 0; --i) {
        double S = 0.0, Sy = 0.0, Sz = 0.0;
#pragma unroll
        for (int j = P - i; j >= 0; --j) {
            double T = 0.0, Tz = 0.0;
#pragma unroll
            for (int kk = P - i - j; kk >= 0; --kk) {
                Tz = Tz * z + T;
                T = T * z + c[h++];
            }
            Sy = Sy * y + S;
            S = S * y + T;
            Sz = Sz * y + Tz;
        }
        fx = fx * x + f;
        f = f * x + S;
        fy = fy * x + Sy;
        fz = fz * x + Sz;
    }
}

// Two leaves per wavefront, one per 32-lane half (leaves hold a few tens of
// particles: one leaf per wavefront left most lanes idle), each half with its
// leaf's coefficients in LDS.
template <int P>
__global__ __launch_bounds__(64) void k_far(const PlanView *V, Bases B)
{
    constexpr int NC = (P + 1) * (P + 2) * (P + 3) / 6;
    __shared__ double cl[2][NC];
    int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int lane = threadIdx.x, half = lane >> 5, hl = lane & 31;
    const int l0 = 2 * (blockIdx.x - B.b[k]);
    const int li = l0 + half;
    const bool valid = li < v.nleaves;
    const int box = v.leaves[valid ? li : l0];
    const OrderTables &t = *v.tab;
    double cen[3], h;
    box_geom(v, box, cen, h);
    const bool loc = valid && v.level[box] >= 2;
    if (loc)
        for (int a = hl; a < NC; a += 32)
            cl[half][horner_pos_of<P>(t.exps[a])] = v.L[(int64_t)box * v.ldm + a] * t.inv_fact[a];
    __syncthreads();
    const int f = v.first[box], cnt = valid ? v.count[box] : 0;
    const int cmax = max(cnt, __shfl_xor(cnt, 32)); // both halves run the longer leaf's chunks
    for (int s = 0; s < cmax; s += 32) {
        int i = f + s + hl;
        bool act = s + hl < cnt;
        double x = act ? v.xs[i] : cen[0], y = act ? v.ys[i] : cen[1], z = act ? v.zs[i] : cen[2];
        double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        if (loc) {
            double ih = 1.0 / h, f0, fx, fy, fz;
            eval_poly<P>(cl[half], (x - cen[0]) * ih, (y - cen[1]) * ih, (z - cen[2]) * ih, f0, fx, fy, fz);
            phi = f0 * ih;
            double ih2 = ih * ih;
            gx = fx * ih2; gy = fy * ih2; gz = fz * ih2;
        }
        if (act) { // far part plus the near part (P2P, M2P), in the caller's order
            const int o = v.perm[i];
            v.phi_out[o] = phi + v.phi_near[i];
            if (v.fld_out) {
                v.fld_out[3 * (int64_t)o] = -gx + v.fld_near[3 * (int64_t)i];
                v.fld_out[3 * (int64_t)o + 1] = -gy + v.fld_near[3 * (int64_t)i + 1];
                v.fld_out[3 * (int64_t)o + 2] = -gz + v.fld_near[3 * (int64_t)i + 2];
            }
        }
    }
}

// ---------------- M2P (W list) ----------------
// phi_i += |d| sum_a M_a d^a, d = (x_i - c_C)/|x_i - c_C|^2 (Eq. P2M_phi at a
// target, the M2P of Sec. 3.2), and its gradient, for every box C of the
// leaf's W list, added to the near-field sums.  It needs only multipoles and
// the near field, so it runs after the second P2P part on the side stream,
// next to the downward pass.  One wavefront per leaf.
template <int P>
__global__ __launch_bounds__(64) void k_m2p(const PlanView *V, Bases B)
{
    constexpr int NC = (P + 1) * (P + 2) * (P + 3) / 6;
    __shared__ double cm[NC];
    int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int box = v.leaves[blockIdx.x - B.b[k]];
    const int64_t w0 = v.W_off[box], w1 = v.W_off[box + 1];
    if (w0 == w1) return;
    const int lane = threadIdx.x;
    const OrderTables &t = *v.tab;
    double cen[3], h;
    box_geom(v, box, cen, h);
    const int f = v.first[box], cnt = v.count[box];
    // the coefficients of the next W box are loaded into registers (a slice
    // per lane) while the current box is evaluated
    constexpr int R = (NC + 63) / 64;
    double wsc[R], nxt[R];
    int hp[R]; // LDS position of the lane's coefficients (Horner order)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int a = lane + 64 * r, ea = a < NC ? t.exps[a] : 0;
        wsc[r] = a < NC ? t.inv_w[(ea & 255) + ((ea >> 8) & 255) + ((ea >> 16) & 255)] : 0.0;
        hp[r] = horner_pos_of<P>(ea);
    }
    // W entries are read 64 at a time, lane l holding entry wb + l
    int64_t wb = w0;
    int wl = 0;
    auto load_entries = [&]() { wl = wb + lane < w1 ? v.W_src[wb + lane] : 0; };
    int nlev = 0;
    uint64_t nmor = 0;
    auto fetch = [&](int64_t e) { // raw coefficients and cell of entry e
        if (e - wb >= 64) { wb += 64; load_entries(); }
        const int src = __builtin_amdgcn_readlane(wl, (int)(e - wb));
        const double *Ms = v.M + (int64_t)src * v.ldm;
#pragma unroll
        for (int r = 0; r < R; ++r) nxt[r] = lane + 64 * r < NC ? Ms[lane + 64 * r] : 0.0;
        nlev = v.level[src];
        nmor = v.morton[src];
    };
    for (int s = 0; s < cnt; s += 64) {
        int i = f + s + lane;
        bool act = s + lane < cnt;
        double x = act ? v.xs[i] : cen[0], y = act ? v.ys[i] : cen[1], z = act ? v.zs[i] : cen[2];
        double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        wb = w0;
        load_entries();
        fetch(w0);
        for (int64_t e = w0; e < w1; ++e) {
            __syncthreads(); // the previous box's coefficients are consumed
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (lane + 64 * r < NC) cm[hp[r]] = nxt[r] * wsc[r];
            const int lev = nlev;
            const uint64_t mor = nmor;
            __syncthreads();
            if (e + 1 < w1) fetch(e + 1);
            double sc[3];
            int cc[3];
            deinterleave(mor, lev, cc);
            const double hs = v.W / (double)(1ll << lev);
#pragma unroll
            for (int d = 0; d < 3; ++d) sc[d] = v.lo[d] + ((double)cc[d] + 0.5) * hs;
            double y0 = x - sc[0], y1 = y - sc[1], y2 = z - sc[2];
            double s2 = 1.0 / (y0 * y0 + y1 * y1 + y2 * y2), sr = sqrt(s2);
            double f0, fx, fy, fz;
            eval_poly<P>(cm, y0 * s2 * hs, y1 * s2 * hs, y2 * s2 * hs, f0, fx, fy, fz);
            double yf = y0 * fx + y1 * fy + y2 * fz;
            phi += sr * f0;
            gx += sr * (-y0 * s2 * f0 + hs * s2 * fx - 2.0 * hs * s2 * s2 * y0 * yf);
            gy += sr * (-y1 * s2 * f0 + hs * s2 * fy - 2.0 * hs * s2 * s2 * y1 * yf);
            gz += sr * (-y2 * s2 * f0 + hs * s2 * fz - 2.0 * hs * s2 * s2 * y2 * yf);
        }
        if (act) { // E = -grad phi
            v.phi_near[i] += phi;
            v.fld_near[3 * (int64_t)i] -= gx;
            v.fld_near[3 * (int64_t)i + 1] -= gy;
            v.fld_near[3 * (int64_t)i + 2] -= gz;
        }
    }
}

// ---------------- P2P ----------------
// The near-field part goes to phi_near / fld_near (sorted order); the far-field
// kernel adds it and writes the caller's order.
// Four wavefronts per block, one target leaf each.  A pass takes up to 64
// targets of the leaf; every lane holds two of them (targets t and t + TPG,
// TPG = ceil(c/2) for the c targets of the pass), and the 64 / TPG lane groups
// split every source chunk into contiguous ranges, so that each source read
// from LDS serves two pairs and few lanes idle.  The group partial sums are
// combined in a fixed order at the end.  Source chunks (up to 64 particles,
// taken from consecutive U-list boxes) are staged in LDS as 32-byte records;
// the next chunk is loaded into registers while the current one is summed.
// FP64: plain sums.  FP32 (mixed precision): pair offsets are formed in FP64
// and rounded to FP32, the pair terms are FP32 (hardware rsq), and each
// lane's sums over all its sources are compensated FP32 sums (Kahan: the
// rounding error of every addition is carried in a second FP32 register and
// subtracted at the end), taken to FP64 for the combination of the groups.
struct SrcRec {
    double x, y, z, q;
};
// softened kernel: the source's sorted index too (j == i is skipped by index,
// since distinct coincident points interact through q / eps)
struct SrcRecS {
    double x, y, z, q;
    int j;
};
template <int KIND> using SrcT = typename std::conditional<KIND == 2, SrcRecS, SrcRec>::type;

struct Tgt {
    double x, y, z;
    int i;
    double phi, ex, ey, ez;
    float s[4], c[4]; // FP32 path: compensated sums (phi, ex, ey, ez) and their errors
};

// s + t with the rounding error kept in c (the true sum is s - c)
__device__ inline void kahan_add(float &s, float &c, float t)
{
    const float y = t - c;
    const float u = s + y;
    c = (u - s) - y;
    s = u;
}

// 1/sqrt(x) for finite x > 0: the hardware estimate (relative error about
// 2^-24) refined by one third-order Householder step,
// y' = y (1 + e/2 + 3e^2/8) with e = 1 - x y^2, which leaves an error at the
// level of the final rounding.  x = 0 gives NaN (callers select it away).
__device__ inline double rsqrt_refined(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(y, e * fma(e, 0.375, 0.5), y);
}

// KIND 0 (FP64) and 1 (FP32 terms): a pair contributes iff r^2 > 0, which
// skips j == i (same coordinates) and coincident points alike.  KIND 2 (the
// softened kernel, FP64): every j != i with r^2 + eps^2 > 0.
template <int MIXED>
__device__ inline void p2p_range(const SrcT<MIXED> *S, int lo, int hi, Tgt &a, Tgt &b, double eps2)
{
    if constexpr (MIXED == 2) {
        auto term = [eps2](const SrcRecS &s, Tgt &t) {
            const double dx = t.x - s.x, dy = t.y - s.y, dz = t.z - s.z;
            const double r2 = dx * dx + dy * dy + dz * dz + eps2;
            const double ri = (s.j != t.i && r2 > 0.0) ? rsqrt_refined(r2) : 0.0;
            const double qr = s.q * ri;
            const double qr3 = qr * ri * ri;
            t.phi += qr;
            t.ex += qr3 * dx; t.ey += qr3 * dy; t.ez += qr3 * dz;
        };
        for (int jj = lo; jj < hi; ++jj) {
            const SrcRecS s0 = S[jj];
            term(s0, a);
            term(s0, b);
        }
    } else if constexpr (MIXED == 1) {
        auto term = [](const SrcRec &s, Tgt &t) {
            const float dx = (float)(t.x - s.x), dy = (float)(t.y - s.y), dz = (float)(t.z - s.z);
            const float r2 = dx * dx + dy * dy + dz * dz;
            float ri = __builtin_amdgcn_rsqf(r2);
            ri = r2 > 0.f ? ri : 0.f;
            const float qr = (float)s.q * ri;
            const float qr3 = qr * ri * ri;
            kahan_add(t.s[0], t.c[0], qr);
            kahan_add(t.s[1], t.c[1], qr3 * dx);
            kahan_add(t.s[2], t.c[2], qr3 * dy);
            kahan_add(t.s[3], t.c[3], qr3 * dz);
        };
        for (int jj = lo; jj < hi; ++jj) {
            const SrcRec s0 = S[jj];
            term(s0, a);
            term(s0, b);
        }
    } else {
        auto term = [](const SrcRec &s, Tgt &t) {
            const double dx = t.x - s.x, dy = t.y - s.y, dz = t.z - s.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ri = r2 > 0.0 ? rsqrt_refined(r2) : 0.0;
            const double qr = s.q * ri;
            const double qr3 = qr * ri * ri;
            t.phi += qr;
            t.ex += qr3 * dx; t.ey += qr3 * dy; t.ez += qr3 * dz;
        };
        for (int jj = lo; jj < hi; ++jj) {
            const SrcRec s0 = S[jj];
            term(s0, a);
            term(s0, b);
        }
    }
}

// five waves per SIMD (at most 102 VGPRs): the kernel waits on its source
// loads more than on arithmetic, and the few values this spills are read
// once per target pass, outside the pair loop
template <int MIXED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_p2p(const PlanView *V, Bases B, int part)
{
    __shared__ SrcT<MIXED> sS[4][64];
    __shared__ double sR[4][8][64]; // group partials for the final combination
    int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // part 0: leaves [0, split), part 1: leaves [split, nleaves)
    const int split = p2p_split(v.nleaves);
    const int lo = part ? split : 0, hi = part ? v.nleaves : split;
    const int li = lo + xcd_remap(blockIdx.x - B.b[k], B.b[k + 1] - B.b[k]) * 4 + wave;
    if (li >= hi) return;
    const auto first = gptr(v.first), count = gptr(v.count), usrc = gptr(v.U_src);
    const auto xs = gptr(v.xs), ys = gptr(v.ys), zs = gptr(v.zs);
    const auto qs = gptr(v.qs);
    const int box = v.leaves[li];
    const int f = first[box], cnt = count[box];
    const int64_t u0 = v.U_off[box], u1 = v.U_off[box + 1];
    SrcT<MIXED> *S = sS[wave];
    double(*R)[64] = sR[wave];
    for (int ts = 0; ts < cnt; ts += 64) {
        const int c = cnt - ts < 64 ? cnt - ts : 64;
        const int TPG = (c + 1) >> 1, G = 64 / TPG, grp = lane / TPG, tl = lane - grp * TPG;
        const bool inG = grp < G;
        const bool acta = inG && tl < c, actb = inG && tl + TPG < c;
        Tgt ta, tb;
        ta.i = f + ts + (acta ? tl : 0);
        tb.i = actb ? f + ts + tl + TPG : -1;
        {
            const int ib = actb ? tb.i : ta.i;
            ta.x = xs[ta.i]; ta.y = ys[ta.i]; ta.z = zs[ta.i];
            tb.x = xs[ib]; tb.y = ys[ib]; tb.z = zs[ib];
        }
        ta.phi = ta.ex = ta.ey = ta.ez = 0.0;
        tb.phi = tb.ex = tb.ey = tb.ez = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) ta.s[r] = ta.c[r] = tb.s[r] = tb.c[r] = 0.f;
        // the U list's particles as one stream, in chunks of up to CH (a chunk
        // spans several source boxes), the next chunk prefetched into registers
        constexpr int CH = 64;
        // the U list's boxes are read 64 at a time, lane l holding the first
        // particle and the count of entry ub + l, so that walking the list
        // waits on one chain of dependent loads per 64 boxes, not one per box
        int64_t ub = u0;
        int bfirst = 0, bcount = 0;
        auto load_boxes = [&]() {
            const int64_t ee = ub + lane;
            bfirst = 0;
            bcount = 0;
            if (ee < u1) { const int src = usrc[ee]; bfirst = first[src]; bcount = count[src]; }
        };
        int64_t e = u0;
        int s = 0, sf = 0, sc = 0;
        auto box_at = [&]() { // sf, sc of entry e (u0 <= e < u1, e - ub <= 64)
            if (e - ub >= 64) { ub += 64; load_boxes(); }
            const int l = (int)(e - ub);
            sf = __builtin_amdgcn_readlane(bfirst, l);
            sc = __builtin_amdgcn_readlane(bcount, l);
        };
        load_boxes();
        if (e < u1) box_at();
        SrcT<MIXED> nx{};
        auto fill = [&]() { // next chunk into nx; returns its size
            int m = 0;
            while (m < CH && e < u1) {
                const int take = sc - s < CH - m ? sc - s : CH - m;
                if (lane >= m && lane < m + take) {
                    const int j = sf + s + (lane - m);
                    nx.x = xs[j]; nx.y = ys[j]; nx.z = zs[j]; nx.q = qs[j];
                    if constexpr (MIXED == 2) nx.j = j;
                }
                m += take;
                s += take;
                if (s >= sc) {
                    s = 0;
                    if (++e < u1) box_at();
                }
            }
            return m;
        };
        int m = fill();
        while (m > 0) {
            wave_sync();
            S[lane] = nx;
            wave_sync();
            const int mn = fill(); // in flight during this chunk's pairs
            const int per = (m + G - 1) / G;
            const int lo = inG ? grp * per : m, hi = lo + per < m ? lo + per : m;
            p2p_range<MIXED>(S, lo, hi, ta, tb, v.eps2);
            m = mn;
        }
        if (MIXED == 1) { // compensated FP32 sums -> FP64
            ta.phi = (double)ta.s[0] - (double)ta.c[0]; ta.ex = (double)ta.s[1] - (double)ta.c[1];
            ta.ey = (double)ta.s[2] - (double)ta.c[2]; ta.ez = (double)ta.s[3] - (double)ta.c[3];
            tb.phi = (double)tb.s[0] - (double)tb.c[0]; tb.ex = (double)tb.s[1] - (double)tb.c[1];
            tb.ey = (double)tb.s[2] - (double)tb.c[2]; tb.ez = (double)tb.s[3] - (double)tb.c[3];
        }
        // combine the lane groups in a fixed order
        wave_sync();
        R[0][lane] = ta.phi; R[1][lane] = ta.ex; R[2][lane] = ta.ey; R[3][lane] = ta.ez;
        R[4][lane] = tb.phi; R[5][lane] = tb.ex; R[6][lane] = tb.ey; R[7][lane] = tb.ez;
        wave_sync();
        if (lane < TPG) {
            double acc[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) acc[r] = R[r][lane];
            for (int g = 1; g < G; ++g)
#pragma unroll
                for (int r = 0; r < 8; ++r) acc[r] += R[r][g * TPG + lane];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = lane + h * TPG;
                if (t >= c) continue;
                const int i = f + ts + t;
                v.phi_near[i] = acc[4 * h];
                v.fld_near[3 * (int64_t)i] = acc[4 * h + 1];
                v.fld_near[3 * (int64_t)i + 1] = acc[4 * h + 2];
                v.fld_near[3 * (int64_t)i + 2] = acc[4 * h + 3];
            }
        }
    }
}

template <typename T> __global__ void k_zero(T *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = T(0);
}

// ---------------- launchers ----------------
#define DISPATCH_P(p, KERNEL, ...)                                                     \
    switch (p) {                                                                       \
    case 0: KERNEL<0> __VA_ARGS__; break;  case 1: KERNEL<1> __VA_ARGS__; break;     \
    case 2: KERNEL<2> __VA_ARGS__; break;  case 3: KERNEL<3> __VA_ARGS__; break;     \
    case 4: KERNEL<4> __VA_ARGS__; break;  case 5: KERNEL<5> __VA_ARGS__; break;     \
    case 6: KERNEL<6> __VA_ARGS__; break;  case 7: KERNEL<7> __VA_ARGS__; break;     \
    case 8: KERNEL<8> __VA_ARGS__; break;  case 9: KERNEL<9> __VA_ARGS__; break;     \
    case 10: KERNEL<10> __VA_ARGS__; break; case 11: KERNEL<11> __VA_ARGS__; break;  \
    case 12: KERNEL<12> __VA_ARGS__; break; case 13: KERNEL<13> __VA_ARGS__; break;  \
    case 14: KERNEL<14> __VA_ARGS__; break; case 15: KERNEL<15> __VA_ARGS__; break;  \
    default: KERNEL<16> __VA_ARGS__; break;                                            \
    }

static inline unsigned nblk(const Bases &B) { return (unsigned)B.b[B.n]; }

void launch_permute_q(const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) k_permute_q<<<nblk(B), 256, 0, s>>>(V, B);
}
void launch_p2m(int p, const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) DISPATCH_P(p, k_p2m, <<<nblk(B), 64, 0, s>>>(V, B));
}
void launch_p2m_fold(int p, const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) DISPATCH_P(p, k_p2m_fold, <<<nblk(B), 256, 0, s>>>(V, B));
}
void launch_unfold(int p, const PlanView *V, const Bases &B, int leaves_only, hipStream_t s)
{
    if (nblk(B)) DISPATCH_P(p, k_unfold, <<<nblk(B), 256, 0, s>>>(V, B, leaves_only));
}
void launch_m2mh(int p, const PlanView *V, const Bases &B, int level, hipStream_t s)
{
    if (nblk(B)) DISPATCH_P(p, k_m2mh, <<<nblk(B), 512, 0, s>>>(V, B, level));
}
void launch_parent_mh(const PlanView *V, const Bases &B, int full, hipStream_t s)
{
    if (nblk(B)) k_parent_mh<<<nblk(B), 256, 0, s>>>(V, B, full);
}
void launch_lh_zero(const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) k_lh_zero<<<nblk(B), 256, 0, s>>>(V, B);
}
void launch_lh_init(const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) k_lh_init<<<nblk(B), 256, 0, s>>>(V, B);
}
void launch_l2lh(int p, const PlanView *V, const Bases &B, int level, hipStream_t s)
{
    if (nblk(B)) DISPATCH_P(p, k_l2lh, <<<nblk(B), 512, 0, s>>>(V, B, level));
}
void launch_p2l(int p, const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) DISPATCH_P(p, k_p2l, <<<nblk(B), 64, 0, s>>>(V, B));
}
void launch_p2l_transform(const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) k_p2l_transform<<<nblk(B), 64, 0, s>>>(V, B);
}
void launch_m2p(int p, const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) DISPATCH_P(p, k_m2p, <<<nblk(B), 64, 0, s>>>(V, B));
}
void launch_far(int p, const PlanView *V, const Bases &B, hipStream_t s)
{
    if (nblk(B)) DISPATCH_P(p, k_far, <<<nblk(B), 64, 0, s>>>(V, B));
}
void launch_p2p(int mixed, int part, const PlanView *V, const Bases &B, hipStream_t s)
{
    if (!nblk(B)) return;
    if (mixed == 2) k_p2p<2><<<nblk(B), 256, 0, s>>>(V, B, part);
    else if (mixed) k_p2p<1><<<nblk(B), 256, 0, s>>>(V, B, part);
    else k_p2p<0><<<nblk(B), 256, 0, s>>>(V, B, part);
}
void launch_zero(double *p, int64_t n, hipStream_t s)
{
    if (n > 0) k_zero<double><<<ceil_div(n, 256), 256, 0, s>>>(p, n);
}
void launch_zero_f32(float *p, int64_t n, hipStream_t s)
{
    if (n > 0) k_zero<float><<<ceil_div(n, 256), 256, 0, s>>>(p, n);
}

} // namespace fmm
