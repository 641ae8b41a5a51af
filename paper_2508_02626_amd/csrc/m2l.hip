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
// skipped.  For every offset slot the block stages the offset's derivative
// table and the 16 source vectors of each wavefront in LDS (loaded into
// registers while the previous slot is being multiplied), then each wavefront
// runs a (p+1)^2 x (p+1)^2 by 16 product with
// 16x16x4 MFMAs: A[b][a] = D(addr(b) + addr(a)) is gathered from LDS with the
// additive address addr(i,j,k) = k s2 + i (2p+2) + j, which turns the
// Hankel structure of the matrix into a single add per operand (the x stride
// 2p+2 keeps the 16 rows of one operand load in different LDS banks); B holds the
// gathered sources.  Accumulators stay in registers across all 189 slots, so
// every target is written once; the FP32 variant adds each slot's FP32 partial
// into FP64 accumulators, so only the per-slot products carry FP32 rounding.  Operand layouts (verified on gfx950):
// A: lane l holds A[l%16][l/16]; B: lane l holds B[l/16][l%16];
// D: f64 lane l reg r -> D[4r + l/16][l%16], f32 lane l reg r -> D[4(l/16)+r][l%16].
#include "ops.h"

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

template <int P, typename T>
__global__ __launch_bounds__(256) void k_m2l(const PlanView *V, Bases B)
{
    constexpr int NH = (P + 1) * (P + 1);
    constexpr int LDH = (NH + 15) & ~15;
    constexpr int MT = LDH / 16;
    constexpr int NK = (NH + 3) & ~3;
    constexpr int KS = NK / 4;
    constexpr int LDD = dlayout_ldd(P);
    constexpr int BST = NK + 1;
    constexpr int DR = (LDD + 255) / 256; // derivative-table words per thread
    constexpr int BR = (16 * NK) / 64;    // source-tile words per lane (16 rows of NK)
    typedef typename Mfma<T>::acc_t acc_t;
    __shared__ T sD[LDD];
    __shared__ T sB[4][16][BST];
    __shared__ int sHo[NK];
    __shared__ int sTg[64];
    __shared__ int sList[kVSlots];
    __shared__ int sN, soct;

    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const int tile = xcd_remap(blockIdx.x - B.b[k], B.b[k + 1] - B.b[k]);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
    const int slot = tile * kM2LSlots + wave * 16 + col;
    const int tgt = v.m2l_tgt[slot];
    if (!__syncthreads_or(tgt >= 0)) return;
    if (tgt >= 0) soct = (int)(v.morton[tgt] & 7); // every target of the block has this octant
    if (tid < 64) sTg[tid] = v.m2l_tgt[tile * kM2LSlots + tid];
    const OrderTables &tb = *v.tab;
    for (int a = tid; a < NK; a += 256) sHo[a] = a < NH ? tb.hoff[a] : 0;
    int hb[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        int b = mt * 16 + col;
        hb[mt] = b < NH ? tb.hoff[b] : 0;
    }
    __syncthreads();
    // slots used by at least one target of the block, in increasing order
    const int32_t *vs = v.vslot;
    if (tid < kVSlots) {
        bool any = false;
        for (int t = 0; t < 64 && !any; ++t) {
            int g = sTg[t];
            any = g >= 0 && vs[(int64_t)g * kVSlots + tid] >= 0;
        }
        sList[tid] = any ? 1 : 0;
    }
    __syncthreads();
    if (tid == 0) {
        int n = 0;
        for (int j = 0; j < kVSlots; ++j)
            if (sList[j]) sList[n++] = j;
        sN = n;
    }
    __syncthreads();
    const int nvalid = sN, oct = soct, ldh = v.ldh;
    const T *Dt = Mfma<T>::D(tb);
    const T *Mh = Mfma<T>::M(v);
    const int32_t *vsl = vs + (int64_t)(tgt >= 0 ? tgt : 0) * kVSlots;

    acc_t acc[MT];
    double4_t acc64[MT]; // FP32 path: per-offset partials are summed in FP64
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) { acc[mt] = acc_t{0, 0, 0, 0}; acc64[mt] = double4_t{0, 0, 0, 0}; }

    T pD[DR], pB[BR];
    auto prefetch = [&](int j) {
        const T *Dk = Dt + (int64_t)tb.offs[oct * kVSlots + j] * LDD;
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            int e = tid + 256 * r;
            pD[r] = e < LDD ? Dk[e] : (T)0;
        }
        const int src = tgt >= 0 ? vsl[j] : -1;
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const int f = lane + 64 * r, t = f / NK, e = f - t * NK;
            const int st = __shfl(src, t);
            pB[r] = st >= 0 ? Mh[(int64_t)st * ldh + e] : (T)0;
        }
    };
    if (nvalid > 0) prefetch(sList[0]);
    for (int q = 0; q < nvalid; ++q) {
        __syncthreads(); // the previous slot's products are done with sD / sB
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            int e = tid + 256 * r;
            if (e < LDD) sD[e] = pD[r];
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const int f = lane + 64 * r, t = f / NK, e = f - t * NK;
            sB[wave][t][e] = pB[r];
        }
        __syncthreads();
        if (q + 1 < nvalid) prefetch(sList[q + 1]); // in flight during the products
        // operands of step ks+1 are read from LDS while the MFMAs of step ks run
        T ac[MT], an[MT], bc, bn = (T)0;
        {
            const int ha = sHo[kq];
            bc = sB[wave][col][kq];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) ac[mt] = sD[hb[mt] + ha];
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (ks + 1 < KS) {
                const int a = (ks + 1) * 4 + kq;
                const int ha = sHo[a];
                bn = sB[wave][col][a];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) an[mt] = sD[hb[mt] + ha];
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = Mfma<T>::run(ac[mt], bc, acc[mt]);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) ac[mt] = an[mt];
            bc = bn;
        }
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[mt][r] += (double)acc[mt][r];
                acc[mt] = acc_t{0, 0, 0, 0};
            }
        }
    }
    if (tgt < 0) return;
    double *Lh = v.Lh + (int64_t)tgt * ldh;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int b = mt * 16 + Mfma<T>::row(lane, r);
            if (b < NH) Lh[b] = sizeof(T) == 4 ? acc64[mt][r] : (double)acc[mt][r];
        }
}

#define M2L_CASE(PP)                                                               \
    case PP:                                                                       \
        if (f32) k_m2l<PP, float><<<nb, 256, 0, s>>>(V, B);                        \
        else k_m2l<PP, double><<<nb, 256, 0, s>>>(V, B);                           \
        break;

void launch_m2l(int p, int f32, const PlanView *V, const Bases &B, hipStream_t s)
{
    unsigned nb = (unsigned)B.b[B.n];
    if (!nb) return;
    switch (p) {
        M2L_CASE(0) M2L_CASE(1) M2L_CASE(2) M2L_CASE(3) M2L_CASE(4) M2L_CASE(5) M2L_CASE(6)
        M2L_CASE(7) M2L_CASE(8) M2L_CASE(9) M2L_CASE(10) M2L_CASE(11)
    default:
        if (f32) k_m2l<12, float><<<nb, 256, 0, s>>>(V, B);
        else k_m2l<12, double><<<nb, 256, 0, s>>>(V, B);
    }
}

} // namespace fmm
