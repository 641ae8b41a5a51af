// Rotation-based M2L (Sec. 3.4): the transfer between two boxes depends only
// on their offset k, and in a frame whose axis is along k it reduces to a
// one-variable (axial) map.  Per V pair the folded multipole is rotated into
// that frame and expressed in azimuthal modes about the axis (F_k), the axial
// map couples only equal modes (A_|k|), and the result is expressed back in
// the original frame's folded local components (B_k):
//     T(k) = B_k A_|k| F_k,   T(k)[b][a] = D_(a+b)(k)  (the M2L contraction).
// Each factor keeps the degree (F, B) or the mode (A), so a pair costs
// sum_n 2 (2n+1)^2 + sum_m (p+1-|m|)^2 multiply-adds instead of (p+1)^4:
// O(p^3) against O(p^4).
//
// Construction (host, long double, per order):
//  * Q_k, the rotation taking k to the z axis: as in Sec. 3.4, a rotation
//    about x by theta = atan2(k_z, k_y) brings k into the x-y plane, one about
//    z by phi = atan2(sqrt(k_y^2 + k_z^2), k_x) onto the x axis, and the
//    cyclic relabelling (x, y, z) -> (y, z, x) takes the x axis to z (the
//    mode basis below uses z as its axis).
//  * Rotations of the folded components: with x' = Q x, d/dx_i =
//    sum_j Q_ji d/dx'_j, so the derivative d^a of degree n is the product of
//    the linear forms l_i = sum_j Q_ji d'_j, expanded over the degree-n
//    monomials of d' (E[a][a']).  Multipoles: Mh' = fold(E^t Mh) (the fold
//    uses Laplace's equation on 1/r); locals: Lh = E unfold(Lh').
//  * Mode basis V (per degree n): the folded symbols
//    Re, Im (x + iy)^m (x^2 + y^2)^s z^kz, kz = (n - m) mod 2, which a
//    rotation about z only mixes within m.  Multipole mode coordinates are
//    V^-1 Mh, local ones V^t Lh (the pairing of symbols with derivatives),
//    and A = V^t T(|k| e_z) V is block diagonal in m (equal for cos and sin).
//  * Reflections: for a sign vector s, T(s o k) = R_s T(k) R_s with R_s the
//    diagonal +-1 of the components' exponent parities, so the factors are
//    stored for the 56 offsets with non-negative components only.
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "fmm.h"
#include "common.h"
#include "tables.h"
#include "ops.h"

namespace fmm {

namespace {
typedef long double ld;

ld binom_ld(int m, int a)
{
    ld r = 1;
    for (int i = 1; i <= a; ++i) r = r * (m - a + i) / i;
    return r;
}
ld fact_ld(int n) { ld r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }

// folded components of degree n in harmonic order
struct Comp { int i, j, k; };
std::vector<Comp> folded(int n)
{
    std::vector<Comp> c;
    for (int i = n; i >= 0; --i) c.push_back({i, n - i, 0});
    for (int i = n - 1; i >= 0; --i) c.push_back({i, n - 1 - i, 1});
    return c;
}
// dense index of a degree-n monomial (i, j, k = n - i - j)
inline int midx(int n, int i, int j) { return i * (n + 1) + j; }

// Gauss-Jordan inverse with partial pivoting (n x n, row-major)
std::vector<ld> invert(std::vector<ld> A, int n)
{
    std::vector<ld> I((size_t)n * n, 0.0L);
    for (int r = 0; r < n; ++r) I[(size_t)r * n + r] = 1.0L;
    for (int c = 0; c < n; ++c) {
        int pv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)pv * n + c])) pv = r;
        if (A[(size_t)pv * n + c] == 0.0L) throw std::logic_error("rotation tables: singular mode basis");
        for (int t = 0; t < n; ++t) {
            std::swap(A[(size_t)c * n + t], A[(size_t)pv * n + t]);
            std::swap(I[(size_t)c * n + t], I[(size_t)pv * n + t]);
        }
        const ld d = A[(size_t)c * n + c];
        for (int t = 0; t < n; ++t) { A[(size_t)c * n + t] /= d; I[(size_t)c * n + t] /= d; }
        for (int r = 0; r < n; ++r)
            if (r != c && A[(size_t)r * n + c] != 0.0L) {
                const ld f = A[(size_t)r * n + c];
                for (int t = 0; t < n; ++t) {
                    A[(size_t)r * n + t] -= f * A[(size_t)c * n + t];
                    I[(size_t)r * n + t] -= f * I[(size_t)c * n + t];
                }
            }
    }
    return I;
}

// mode index within a degree: m = 0 -> 0, else 2m - 1 + type (0 cos, 1 sin)
inline int mode_idx(int m, int t) { return m == 0 ? 0 : 2 * m - 1 + t; }

// V_n: column mode_idx(m, t) holds the folded coefficients of the symbol
// Re/Im (x + iy)^m (x^2 + y^2)^s z^kz
std::vector<ld> mode_basis(int n)
{
    const int w = 2 * n + 1;
    std::vector<Comp> c = folded(n);
    std::vector<ld> V((size_t)w * w, 0.0L);
    for (int m = 0; m <= n; ++m)
        for (int t = 0; t < (m ? 2 : 1); ++t) {
            const int kz = (n - m) & 1, d = n - kz, s = (d - m) / 2;
            // (x + iy)^m: real part t even powers of y, imaginary odd
            std::vector<ld> xy(d + 1, 0.0L); // coefficient of x^(d - q) y^q
            for (int q = t; q <= m; q += 2) {
                const ld sg = ((q - t) / 2) & 1 ? -1.0L : 1.0L;
                const ld cm = sg * binom_ld(m, q);
                for (int u = 0; u <= s; ++u) // (x^2 + y^2)^s
                    xy[q + 2 * (s - u)] += cm * binom_ld(s, u);
            }
            for (int col = 0; col < w; ++col)
                if (c[col].k == kz) V[(size_t)col * w + mode_idx(m, t)] = xy[c[col].j];
        }
    return V;
}

struct Rot {
    int p;
    std::vector<double> F, B, A; // see fmm_order_table, tables 5-7
    std::vector<int> aidx;       // [64] index of |k|^2 among the A blocks
};

// D_g(x) = g! a_g(x) for folded a, b of degrees l, n: T[b][a] = D_(a+b)
void transfer(const ld x[3], int p, std::vector<std::vector<ld>> &T)
{
    std::vector<ld> a;
    inv_r_taylor(x, 2 * p, 2, a);
    T.assign((size_t)(p + 1) * (p + 1), {});
    for (int l = 0; l <= p; ++l)
        for (int n = 0; n <= p; ++n) {
            std::vector<Comp> cb = folded(l), ca = folded(n);
            std::vector<ld> &t = T[(size_t)l * (p + 1) + n];
            t.assign(cb.size() * ca.size(), 0.0L);
            for (size_t r = 0; r < cb.size(); ++r)
                for (size_t q = 0; q < ca.size(); ++q) {
                    const int gi = cb[r].i + ca[q].i, gj = cb[r].j + ca[q].j, gk = cb[r].k + ca[q].k;
                    t[r * ca.size() + q] = a[mono_index(gi, gj, gk)] * fact_ld(gi) * fact_ld(gj) * fact_ld(gk);
                }
        }
}

void build(int p, Rot &R)
{
    R.p = p;
    const int S = (p + 1) * (2 * p + 1) * (2 * p + 3) / 3; // sum_n (2n+1)^2
    int SA = 0;
    for (int m = 0; m <= p; ++m) SA += (p + 1 - m) * (p + 1 - m);
    std::vector<std::vector<ld>> Vn(p + 1), Vi(p + 1);
    for (int n = 0; n <= p; ++n) { Vn[n] = mode_basis(n); Vi[n] = invert(Vn[n], 2 * n + 1); }
    // axial blocks, one per |k|^2
    std::map<int, int> r2idx;
    for (int ax = 0; ax <= 3; ++ax)
        for (int ay = 0; ay <= 3; ++ay)
            for (int az = 0; az <= 3; ++az)
                if (ax > 1 || ay > 1 || az > 1) r2idx.emplace(ax * ax + ay * ay + az * az, 0);
    int nr = 0;
    for (auto &e : r2idx) e.second = nr++;
    R.A.assign((size_t)nr * SA, 0.0);
    for (auto &e : r2idx) {
        const ld x[3] = {0.0L, 0.0L, std::sqrt((ld)e.first)};
        std::vector<std::vector<ld>> T;
        transfer(x, p, T);
        int off = 0;
        for (int m = 0; m <= p; ++m) {
            const int w = p + 1 - m;
            for (int l = m; l <= p; ++l)
                for (int n = m; n <= p; ++n) {
                    // (V_l^t T V_n)[(l, m, cos)][(n, m, cos)]
                    const int wl = 2 * l + 1, wn = 2 * n + 1, jl = mode_idx(m, 0), jn = mode_idx(m, 0);
                    const std::vector<ld> &t = T[(size_t)l * (p + 1) + n];
                    ld s = 0.0L;
                    for (int r = 0; r < wl; ++r) {
                        const ld vl = Vn[l][(size_t)r * wl + jl];
                        if (vl == 0.0L) continue;
                        for (int q = 0; q < wn; ++q) s += vl * t[(size_t)r * wn + q] * Vn[n][(size_t)q * wn + jn];
                    }
                    // stored transposed: [n - m][l - m]
                    R.A[(size_t)e.second * SA + off + (size_t)(n - m) * w + (l - m)] = (double)s;
                }
            off += w * w;
        }
    }
    // rotations per class (|k_x|, |k_y|, |k_z|)
    R.F.assign((size_t)64 * S, 0.0);
    R.B.assign((size_t)64 * S, 0.0);
    R.aidx.assign(64, -1);
    for (int ax = 0; ax <= 3; ++ax)
        for (int ay = 0; ay <= 3; ++ay)
            for (int az = 0; az <= 3; ++az) {
                if (ax <= 1 && ay <= 1 && az <= 1) continue;
                const int cls = ax * 16 + ay * 4 + az;
                R.aidx[cls] = r2idx[ax * ax + ay * ay + az * az];
                // Q: about x by theta, about z by phi, then (x, y, z) -> (y, z, x)
                const ld kx = ax, ky = ay, kz = az, rho = std::sqrt(ky * ky + kz * kz);
                const ld th = std::atan2(kz, ky), ph = std::atan2(rho, kx);
                const ld Rx[3][3] = {{1, 0, 0}, {0, std::cos(th), std::sin(th)}, {0, -std::sin(th), std::cos(th)}};
                const ld Rz[3][3] = {{std::cos(ph), std::sin(ph), 0}, {-std::sin(ph), std::cos(ph), 0}, {0, 0, 1}};
                const ld Pc[3][3] = {{0, 1, 0}, {0, 0, 1}, {1, 0, 0}};
                ld M1[3][3] = {}, Q[3][3] = {};
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        for (int t = 0; t < 3; ++t) M1[i][j] += Rz[i][t] * Rx[t][j];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        for (int t = 0; t < 3; ++t) Q[i][j] += Pc[i][t] * M1[t][j];
                const ld kk[3] = {kx, ky, kz}, kn = std::sqrt(kx * kx + ky * ky + kz * kz);
                for (int i = 0; i < 3; ++i) {
                    ld s = 0.0L;
                    for (int j = 0; j < 3; ++j) s += Q[i][j] * kk[j];
                    if (std::fabs(s - (i == 2 ? kn : 0.0L)) > 1e-15L * kn) throw std::logic_error("rotation does not align the offset");
                }
                int off = 0;
                for (int n = 0; n <= p; ++n) {
                    const int w = 2 * n + 1;
                    std::vector<Comp> c = folded(n);
                    // E[a][a']: product of l_i^(a_i), l_i = sum_j Q_ji d'_j, over degree-n monomials
                    std::vector<std::vector<ld>> E(w);
                    for (int q = 0; q < w; ++q) {
                        std::vector<ld> cur(1, 1.0L); // degree 0
                        int deg = 0;
                        const int ex[3] = {c[q].i, c[q].j, c[q].k};
                        for (int ivar = 0; ivar < 3; ++ivar)
                            for (int rep = 0; rep < ex[ivar]; ++rep) {
                                std::vector<ld> nx((size_t)(deg + 2) * (deg + 2), 0.0L);
                                for (int i = 0; i <= deg; ++i)
                                    for (int j = 0; i + j <= deg; ++j) {
                                        const ld v = cur[midx(deg, i, j)];
                                        if (v == 0.0L) continue;
                                        nx[midx(deg + 1, i + 1, j)] += Q[0][ivar] * v;
                                        nx[midx(deg + 1, i, j + 1)] += Q[1][ivar] * v;
                                        nx[midx(deg + 1, i, j)] += Q[2][ivar] * v;
                                    }
                                cur.swap(nx);
                                ++deg;
                            }
                        E[q] = cur; // degree n, midx(n, i, j)
                    }
                    // RM[c][a] = sum over the fold terms of c of coefficient * E[a][term]
                    std::vector<ld> RM((size_t)w * w, 0.0L), RL((size_t)w * w, 0.0L);
                    for (int r = 0; r < w; ++r) {
                        const int I = c[r].i, J = c[r].j, K = c[r].k;
                        for (int mm = 0; K + 2 * mm <= n; ++mm)
                            for (int aa = 0; aa <= mm; ++aa) {
                                const int i = I - 2 * aa, j = J - 2 * (mm - aa);
                                if (i < 0 || j < 0) continue;
                                const ld cf = ((mm & 1) ? -1.0L : 1.0L) * binom_ld(mm, aa);
                                for (int q = 0; q < w; ++q) RM[(size_t)r * w + q] += cf * E[q][midx(n, i, j)];
                            }
                    }
                    // RL[b][c'] = sum_{b' full} E[b][b'] unfold(b' <- c'), unfold:
                    // (i, j, k) <- sum_a (-1)^m C(m, a) Lh(i + 2a, j + 2(m - a), k mod 2), m = k / 2
                    for (int r = 0; r < w; ++r)
                        for (int i = 0; i <= n; ++i)
                            for (int j = 0; i + j <= n; ++j) {
                                const ld e = E[r][midx(n, i, j)];
                                if (e == 0.0L) continue;
                                const int k = n - i - j, mm = k / 2;
                                for (int aa = 0; aa <= mm; ++aa) {
                                    const int hi = i + 2 * aa, hj = j + 2 * (mm - aa), hk = k & 1;
                                    // position of (hi, hj, hk) among the folded components of degree n
                                    const int pos = hk == 0 ? n - hi : (n + 1) + (n - 1 - hi);
                                    (void)hj;
                                    RL[(size_t)r * w + pos] += e * ((mm & 1) ? -1.0L : 1.0L) * binom_ld(mm, aa);
                                }
                            }
                    // F = V^-1 RM (modes <- folded), B = RL V^-t (folded <- modes)
                    for (int row = 0; row < w; ++row)
                        for (int col = 0; col < w; ++col) {
                            ld f = 0.0L, b = 0.0L;
                            for (int t = 0; t < w; ++t) {
                                f += Vi[n][(size_t)row * w + t] * RM[(size_t)t * w + col];
                                b += RL[(size_t)row * w + t] * Vi[n][(size_t)col * w + t];
                            }
                            // stored transposed ([input][output]): F[n][folded a][mode], B[n][mode][folded b]
                            R.F[(size_t)cls * S + off + (size_t)col * w + row] = (double)f;
                            R.B[(size_t)cls * S + off + (size_t)col * w + row] = (double)b;
                        }
                    off += w * w;
                }
            }
}
} // namespace


// ---------------- device tables ----------------
namespace {
std::mutex g_rot_mu;
std::map<std::pair<int, int>, const RotTables *> g_rot_cache;

template <typename T>
int upload_rot(const std::vector<T> &v, const T **out, std::string &err)
{
    void *d = nullptr;
    const size_t bytes = sizeof(T) * (v.empty() ? 1 : v.size());
    if (hipMalloc(&d, bytes) != hipSuccess) { err = "hipMalloc failed for rotation tables"; return -1; }
    if (!v.empty() && hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
        err = "hipMemcpy failed for rotation tables";
        return -1;
    }
    *out = (const T *)d;
    return 0;
}
} // namespace

const RotTables *get_rotation_tables(int p, std::string &err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { err = "hipGetDevice failed"; return nullptr; }
    std::lock_guard<std::mutex> lk(g_rot_mu);
    auto key = std::make_pair(dev, p);
    auto it = g_rot_cache.find(key);
    if (it != g_rot_cache.end()) return it->second;
    Rot R;
    try {
        build(p, R);
    } catch (const std::exception &e) {
        err = e.what();
        return nullptr;
    }
    RotTables t{};
    if (upload_rot(R.F, &t.F, err) || upload_rot(R.B, &t.B, err) || upload_rot(R.A, &t.A, err) ||
        upload_rot(R.aidx, &t.aidx, err))
        return nullptr;
    void *d = nullptr;
    if (hipMalloc(&d, sizeof(RotTables)) != hipSuccess ||
        hipMemcpy(d, &t, sizeof(RotTables), hipMemcpyHostToDevice) != hipSuccess) {
        err = "hipMalloc/hipMemcpy failed for rotation tables";
        return nullptr;
    }
    auto &slot = g_rot_cache[key];
    slot = (const RotTables *)d;
    return slot;
}

// ---------------- the kernel ----------------
// A block takes TG targets of one M2L tile (one octant) and runs every V
// pair of them, class of offsets by class: the class's factors F, B (for
// |k|) and its axial block A go to LDS, then for each member offset s o |k|
// the TG sources' folded multipoles (signs R_s applied) are staged as
// X[component][target] and the three products run on the vector unit, one
// thread per output component: y = F x (per degree), z = A y (per mode, the
// same block for cos and sin), acc += R_s B z (per degree).  Every product
// reads one table entry for TG multiply-adds; y and z overwrite X after a
// barrier.  The targets' accumulators stay in registers over all classes.
template <int P> struct RotShape {
    static constexpr int NH = (P + 1) * (P + 1);
    static constexpr int S = (P + 1) * (2 * P + 1) * (2 * P + 3) / 3;
    static constexpr int SA = (P + 1) * (P + 2) * (2 * P + 3) / 6;
    static constexpr int TG = P >= 15 ? 16 : 32;   // targets per block (LDS)
    static constexpr int CPT = (NH + 255) / 256;   // components per thread
};

template <int P>
__global__ __launch_bounds__(256, 1) void k_m2l_rot(const PlanView *V, Bases B)
{
    using SH = RotShape<P>;
    constexpr int NH = SH::NH, S = SH::S, SA = SH::SA, TG = SH::TG, CPT = SH::CPT;
    constexpr int TPB = kM2LSlots / TG; // blocks per tile
    __shared__ double sF[S], sB[S], sA[SA];
    __shared__ double X[NH][TG];
    __shared__ int sTg[TG];
    __shared__ int sMem[kSymClasses][8], sRep[kSymClasses], sSl[kVSlots];
    __shared__ unsigned long long sUsed;
    __shared__ int sHas[kVSlots], soct;
    const int k = find_plan(B, blockIdx.x);
    const PlanView &v = V[k];
    const OrderTables &tb = *v.tab;
    const RotTables &rt = *v.rot;
    const int item = xcd_remap(blockIdx.x - B.b[k], B.b[k + 1] - B.b[k]);
    const int tile = item / TPB, sub = item - tile * TPB;
    const int tid = threadIdx.x;
    if (tid < TG) sTg[tid] = v.m2l_tgt[tile * kM2LSlots + sub * TG + tid];
    if (tid == 0) sUsed = 0;
    __syncthreads();
    int anyt = -1;
    for (int t = 0; t < TG; ++t) anyt = anyt >= 0 ? anyt : sTg[t];
    if (anyt < 0) return; // (uniform: every thread read the same sTg)
    if (tid == 0) soct = (int)(v.morton[anyt] & 7);
    __syncthreads();
    // the octant's classes: members' slots, representative offset, class of each slot
    const int oct = soct;
    for (int e = tid; e < kSymClasses * 8; e += 256) sMem[e >> 3][e & 7] = tb.smem[oct * kSymClasses * 8 + e];
    if (tid < kSymClasses) sRep[tid] = tb.srep[oct * kSymClasses + tid];
    if (tid < kVSlots) sSl[tid] = tb.sslot[oct * kVSlots + tid];
    __syncthreads();
    // slots with a source for some target, and the classes they belong to
    const auto vs = gptr(v.vslot);
    for (int j = tid; j < kVSlots; j += 256) {
        int h = 0;
        for (int t = 0; t < TG; ++t) h |= sTg[t] >= 0 && vs[(int64_t)sTg[t] * kVSlots + j] >= 0;
        sHas[j] = h;
        if (h) atomicOr(&sUsed, 1ull << sSl[j]);
    }
    __syncthreads();
    const unsigned long long used = sUsed;
    // the thread's components: c = tid + 256 i (folded harmonic index for the
    // input and output, global mode index n^2 + mode for the intermediates)
    int cdeg[CPT], cpos[CPT], cpar[CPT], cm[CPT], ctyp[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = tid + 256 * i < NH ? tid + 256 * i : 0;
        int n = 0;
        while ((n + 1) * (n + 1) <= c) ++n;
        cdeg[i] = n;
        cpos[i] = c - n * n; // position within the degree (folded or mode)
        // folded component (i, j, k) at that position: parities for R_s
        const int q = cpos[i];
        const int fi = q <= n ? n - q : (n - 1) - (q - n - 1), fk = q <= n ? 0 : 1, fj = n - fk - fi;
        cpar[i] = (fi & 1) << 2 | (fj & 1) << 1 | fk;
        cm[i] = q == 0 ? 0 : (q + 1) / 2; // mode m and type of mode index q
        ctyp[i] = q == 0 ? 0 : (q + 1) & 1;
    }
    double acc[CPT][TG];
#pragma unroll
    for (int i = 0; i < CPT; ++i)
#pragma unroll
        for (int t = 0; t < TG; ++t) acc[i][t] = 0.0;
    const auto Mh = gptr(v.Mh);
    const int ldmh = v.ldmh;
    for (int c = 0; c < kSymClasses; ++c) {
        if (!((used >> c) & 1)) continue;
        // factors of |k| for this class
        const int rep = sRep[c] & 0xffff;
        const int kx = rep / 49 - 3, ky = (rep / 7) % 7 - 3, kz = rep % 7 - 3;
        const int cls = abs(kx) * 16 + abs(ky) * 4 + abs(kz);
        const int ai = rt.aidx[cls];
        __syncthreads(); // previous class done with the tables
        for (int e = tid; e < S; e += 256) {
            sF[e] = rt.F[(int64_t)cls * S + e];
            sB[e] = rt.B[(int64_t)cls * S + e];
        }
        for (int e = tid; e < SA; e += 256) sA[e] = rt.A[(int64_t)ai * SA + e];
        for (int m = 0; m < 8; ++m) {
            const int j = sMem[c][m];
            if (j < 0 || !sHas[j]) continue;
            // negated axes of this member relative to |k|
            const int mx = ((m >> 2) & 1) ^ (kx < 0), my = ((m >> 1) & 1) ^ (ky < 0), mz = (m & 1) ^ (kz < 0);
            const int neg = mx << 2 | my << 1 | mz;
            __syncthreads(); // tables staged / previous member's X consumed
            for (int e = tid; e < NH * TG; e += 256) {
                const int cc = e % NH, t = e / NH;
                const int src = sTg[t] >= 0 ? vs[(int64_t)sTg[t] * kVSlots + j] : -1;
                double x = 0.0;
                if (src >= 0) {
                    int n = 0;
                    while ((n + 1) * (n + 1) <= cc) ++n;
                    const int q = cc - n * n;
                    const int fi = q <= n ? n - q : (n - 1) - (q - n - 1), fk = q <= n ? 0 : 1, fj = n - fk - fi;
                    const int par = (fi & 1) << 2 | (fj & 1) << 1 | fk;
                    x = Mh[(int64_t)src * ldmh + tb.hpos[cc]];
                    if (__popc(par & neg) & 1) x = -x;
                }
                X[cc][t] = x;
            }
            __syncthreads();
            // y = F x: mode (n, q) <- folded components of degree n
            double y[CPT][TG];
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int n = cdeg[i], w = 2 * n + 1, off = n * (2 * n - 1) * (2 * n + 1) / 3;
#pragma unroll
                for (int t = 0; t < TG; ++t) y[i][t] = 0.0;
                if (tid + 256 * i >= NH) continue;
                for (int a = 0; a < w; ++a) {
                    const double f = sF[off + a * w + cpos[i]];
                    const double *xr = X[n * n + a];
#pragma unroll
                    for (int t = 0; t < TG; ++t) y[i][t] = fma(f, xr[t], y[i][t]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < CPT; ++i)
                if (tid + 256 * i < NH)
#pragma unroll
                    for (int t = 0; t < TG; ++t) X[tid + 256 * i][t] = y[i][t];
            __syncthreads();
            // z = A y: mode (l, m, type) <- modes (n, m, type), n = m..P
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int l = cdeg[i], mm = cm[i], ty = ctyp[i], w = P + 1 - mm;
                int aoff = 0; // blocks of the modes below mm
                for (int q = 0; q < mm; ++q) aoff += (P + 1 - q) * (P + 1 - q);
#pragma unroll
                for (int t = 0; t < TG; ++t) y[i][t] = 0.0;
                if (tid + 256 * i >= NH) continue;
                const int qm = mm == 0 ? 0 : 2 * mm - 1 + ty;
                for (int n = mm; n <= P; ++n) {
                    const double a = sA[aoff + (n - mm) * w + (l - mm)];
                    const double *yr = X[n * n + qm];
#pragma unroll
                    for (int t = 0; t < TG; ++t) y[i][t] = fma(a, yr[t], y[i][t]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < CPT; ++i)
                if (tid + 256 * i < NH)
#pragma unroll
                    for (int t = 0; t < TG; ++t) X[tid + 256 * i][t] = y[i][t];
            __syncthreads();
            // acc += R_s B z: folded (l, q) <- modes of degree l
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                if (tid + 256 * i >= NH) continue;
                const int l = cdeg[i], w = 2 * l + 1, off = l * (2 * l - 1) * (2 * l + 1) / 3;
                const double sg = (__popc(cpar[i] & neg) & 1) ? -1.0 : 1.0;
                double z[TG];
#pragma unroll
                for (int t = 0; t < TG; ++t) z[t] = 0.0;
                for (int u = 0; u < w; ++u) {
                    const double b = sB[off + u * w + cpos[i]];
                    const double *zr = X[l * l + u];
#pragma unroll
                    for (int t = 0; t < TG; ++t) z[t] = fma(b, zr[t], z[t]);
                }
#pragma unroll
                for (int t = 0; t < TG; ++t) acc[i][t] = fma(sg, z[t], acc[i][t]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = tid + 256 * i;
        if (c >= NH) continue;
#pragma unroll
        for (int t = 0; t < TG; ++t)
            if (sTg[t] >= 0) gptr(v.Lh)[(int64_t)sTg[t] * v.ldh + c] = acc[i][t];
    }
}

#define ROT_CASE(PP) \
    case PP: k_m2l_rot<PP><<<nb, 256, 0, s>>>(V, B); break;

int m2l_rot_blocks_per_tile(int p) { return p >= 15 ? kM2LSlots / 16 : kM2LSlots / 32; }

void launch_m2l_rot(int p, const PlanView *V, const Bases &B, hipStream_t s)
{
    const unsigned nb = (unsigned)B.b[B.n];
    if (!nb) return;
    switch (p) {
        ROT_CASE(0) ROT_CASE(1) ROT_CASE(2) ROT_CASE(3) ROT_CASE(4) ROT_CASE(5) ROT_CASE(6) ROT_CASE(7)
        ROT_CASE(8) ROT_CASE(9) ROT_CASE(10) ROT_CASE(11) ROT_CASE(12) ROT_CASE(13) ROT_CASE(14) ROT_CASE(15)
    default: k_m2l_rot<16><<<nb, 256, 0, s>>>(V, B); break;
    }
}

int host_rotation_tables(int p, int which, std::vector<double> &out)
{
    Rot R;
    build(p, R);
    const int S = (p + 1) * (2 * p + 1) * (2 * p + 3) / 3;
    int SA = 0;
    for (int m = 0; m <= p; ++m) SA += (p + 1 - m) * (p + 1 - m);
    switch (which) {
    case 0: out = R.F; return S;
    case 1: out = R.B; return S;
    case 2: out = R.A; return SA;
    case 3: out.assign(R.aidx.begin(), R.aidx.end()); return 64;
    default: return -1;
    }
}

} // namespace fmm
