// Per-order constant tables, derived on the host in long double from closed
// forms (not from a DA composition), then rounded to FP64 / FP32 and uploaded
// once per (device, order).
//
//  P2M     The multipole of one charge at offset y is (1 - 2 y.d + y^2 d^2)^-1/2
//          (Eq. P2M, sign reading), the Legendre generating function; its
//          degree-n coefficients c_a(y) obey
//              n c_a = (2n-1) sum_k y_k c_(a-e_k) - (n-1) |y|^2 sum_k c_(a-2e_k).
//          Each c_a is a homogeneous polynomial in y, so the expansion of a box
//          is a fixed linear map of its raw moments Q_g = sum q u^g (u = y/h).
//  M2L     With harmonic degrees, phi = sum_a w_|a| M_a d^a(1/|x|), so the
//          local coefficients are derivatives of 1/|x| at the offset:
//          Lhat_b = sum_a D_(a+b)(k) Mhat_a (see common.h).  D_g(k) = g! a_g(k)
//          from the recurrence of the Taylor coefficients a_g of 1/|x|:
//              n |x|^2 a_g + (2n-1) sum_k x_k a_(g-e_k) + (n-1) sum_k a_(g-2e_k) = 0.
//          Since d^2/dz^2 (1/r) = -(d^2/dx^2 + d^2/dy^2)(1/r), only components
//          with a_z, b_z <= 1 are contracted: Mhat is first folded onto them,
//          and the result unfolded by the same identity.
//  M2M     The child's field sum_a W_a d^a(1/|x - c|) (W = w M) re-expanded at
//          the parent centre by Taylor in the source position, then projected
//          onto harmonic polynomials per degree (which leaves the field
//          unchanged and gives the DA representative):
//              pi_n(P) = sum_k (-1)^k (2n-2k-1)!! / ((2n-1)!! (2k)!!) r^(2k) Lap^k P.
//  L2L     Taylor shift of a polynomial (map M3 of Sec. 2.5).
#include "tables.h"
#include "fmm.h"

#include <stdexcept>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace fmm {

typedef long double ld;

namespace {

struct Mono {
    int p, n;
    std::vector<int> e; // 3 per monomial
    Mono(int p_) : p(p_), n(ncoef(p_)), e(3 * ncoef(p_))
    {
        for (int d = 0; d <= p; ++d)
            for (int i = d; i >= 0; --i)
                for (int j = d - i; j >= 0; --j) {
                    int k = d - i - j, id = mono_index(i, j, k);
                    e[3 * id] = i; e[3 * id + 1] = j; e[3 * id + 2] = k;
                }
    }
    int deg(int id) const { return e[3 * id] + e[3 * id + 1] + e[3 * id + 2]; }
};

ld fact(int n) { ld r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }
ld dfact(int n) { ld r = 1; for (int i = n; i > 1; i -= 2) r *= i; return r; } // n!!, (-1)!! = 1
ld binom(int m, int a) { return fact(m) / (fact(a) * fact(m - a)); }
ld ipow(ld x, int k) { ld r = 1; for (int i = 0; i < k; ++i) r *= x; return r; }

} // namespace

// Taylor coefficients a_g(x) of 1/|x| for |g| <= maxdeg and g_z <= maxz,
// stored by mono_index (order maxdeg); entries with g_z > maxz left 0.
void inv_r_taylor(const ld x[3], int maxdeg, int maxz, std::vector<ld> &a)
{
    Mono m(maxdeg);
    a.assign(m.n, 0.0L);
    ld r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    a[0] = 1.0L / std::sqrt(r2);
    for (int id = 1; id < m.n; ++id) {
        int g[3] = {m.e[3 * id], m.e[3 * id + 1], m.e[3 * id + 2]};
        if (g[2] > maxz) continue;
        int n = g[0] + g[1] + g[2];
        ld s1 = 0, s2 = 0;
        for (int k = 0; k < 3; ++k) {
            if (g[k] >= 1) {
                int h[3] = {g[0], g[1], g[2]}; h[k] -= 1;
                s1 += x[k] * a[mono_index(h[0], h[1], h[2])];
            }
            if (g[k] >= 2) {
                int h[3] = {g[0], g[1], g[2]}; h[k] -= 2;
                s2 += a[mono_index(h[0], h[1], h[2])];
            }
        }
        a[id] = -((2 * n - 1) * s1 + (n - 1) * s2) / (n * r2);
    }
}

namespace {

// P2M: coefficients of the polynomials c_a(u) (degree |a|) over monomials u^g.
// Returns C[a][g] (n x n, block diagonal by degree).
std::vector<ld> p2m_polys(const Mono &m)
{
    int n = m.n;
    std::vector<ld> C((size_t)n * n, 0.0L);
    C[0] = 1.0L;
    for (int id = 1; id < n; ++id) {
        int a[3] = {m.e[3 * id], m.e[3 * id + 1], m.e[3 * id + 2]};
        int d = a[0] + a[1] + a[2];
        std::vector<ld> out(n, 0.0L);
        for (int k = 0; k < 3; ++k) {
            if (a[k] >= 1) { // (2d-1) u_k c_(a-e_k)
                int h[3] = {a[0], a[1], a[2]}; h[k] -= 1;
                const ld *src = &C[(size_t)mono_index(h[0], h[1], h[2]) * n];
                for (int g = 0; g < n; ++g)
                    if (src[g] != 0) {
                        int t[3] = {m.e[3 * g], m.e[3 * g + 1], m.e[3 * g + 2]}; t[k] += 1;
                        out[mono_index(t[0], t[1], t[2])] += (2 * d - 1) * src[g];
                    }
            }
            if (a[k] >= 2) { // -(d-1) |u|^2 c_(a-2e_k)
                int h[3] = {a[0], a[1], a[2]}; h[k] -= 2;
                const ld *src = &C[(size_t)mono_index(h[0], h[1], h[2]) * n];
                for (int g = 0; g < n; ++g)
                    if (src[g] != 0)
                        for (int j = 0; j < 3; ++j) {
                            int t[3] = {m.e[3 * g], m.e[3 * g + 1], m.e[3 * g + 2]}; t[j] += 2;
                            out[mono_index(t[0], t[1], t[2])] -= (d - 1) * src[g];
                        }
            }
        }
        for (int g = 0; g < n; ++g) C[(size_t)id * n + g] = out[g] / d;
    }
    return C;
}

// harmonic projection of the homogeneous polynomial with coefficient vector v
// (over all monomials of order p; only degree `deg` entries nonzero)
std::vector<ld> harmonic_projection(const Mono &m, const std::vector<ld> &v, int deg)
{
    int n = m.n;
    std::vector<ld> out(n, 0.0L), lap = v;
    for (int k = 0; 2 * k <= deg; ++k) {
        ld c = ((k & 1) ? -1.0L : 1.0L) * dfact(2 * deg - 2 * k - 1) /
               (dfact(2 * deg - 1) * dfact(2 * k));
        // r^(2k) * lap
        std::vector<ld> t = lap;
        for (int s = 0; s < k; ++s) {
            std::vector<ld> u(n, 0.0L);
            for (int g = 0; g < n; ++g)
                if (t[g] != 0)
                    for (int j = 0; j < 3; ++j) {
                        int e[3] = {m.e[3 * g], m.e[3 * g + 1], m.e[3 * g + 2]}; e[j] += 2;
                        int d = e[0] + e[1] + e[2];
                        if (d <= m.p) u[mono_index(e[0], e[1], e[2])] += t[g];
                    }
            t.swap(u);
        }
        for (int g = 0; g < n; ++g) out[g] += c * t[g];
        // next Laplacian
        std::vector<ld> u(n, 0.0L);
        for (int g = 0; g < n; ++g)
            if (lap[g] != 0)
                for (int j = 0; j < 3; ++j) {
                    int e[3] = {m.e[3 * g], m.e[3 * g + 1], m.e[3 * g + 2]};
                    if (e[j] < 2) continue;
                    ld f = (ld)e[j] * (e[j] - 1);
                    e[j] -= 2;
                    u[mono_index(e[0], e[1], e[2])] += f * lap[g];
                }
        lap.swap(u);
    }
    return out;
}

struct Built {
    std::vector<double> D, S, G, GH, TM, HR, P2M, FP2M, P2L, fold_c, unfold_c, inv_fact, inv_w;
    std::vector<float> Df;
    std::vector<int> offs, hoff, fold_off, fold_idx, unfold_off, unfold_idx, exps, dmap;
    std::vector<int> mpos, mposf, hpos, hposf, srow, scol, srep, smem, sslot;
    int ldd = 0, ldc = 0;
};

void build_tables(int p, Built &B)
{
    Mono m(p);
    const int nc = m.n, nh = nharm(p), ldh = pad16(nh);
    // additive layout addr(i,j,k) = k*s2 + i*s1 + j of the derivative tables
    // (strides per order, chosen for the M2L operand gather)
    const int s1 = dlayout_s1(p), s2 = dlayout_s2(p);
    // exponent packing, factorial tables
    B.exps.resize(nc);
    B.inv_fact.resize(nc);
    for (int id = 0; id < nc; ++id) {
        int i = m.e[3 * id], j = m.e[3 * id + 1], k = m.e[3 * id + 2];
        B.exps[id] = i | (j << 8) | (k << 16);
        B.inv_fact[id] = (double)(1.0L / (fact(i) * fact(j) * fact(k)));
    }
    B.inv_w.resize(p + 1);
    for (int n = 0; n <= p; ++n) B.inv_w[n] = (double)(((n & 1) ? -1.0L : 1.0L) * dfact(2 * n - 1));

    // harmonic index -> exponents, additive D addresses
    std::vector<int> hx(nh), hy(nh), hz(nh);
    for (int n = 0; n <= p; ++n) {
        for (int i = n; i >= 0; --i) { int c = harm_index(i, n - i, 0); hx[c] = i; hy[c] = n - i; hz[c] = 0; }
        for (int i = n - 1; i >= 0; --i) { int c = harm_index(i, n - 1 - i, 1); hx[c] = i; hy[c] = n - 1 - i; hz[c] = 1; }
    }
    B.hoff.assign(ldh, 0);
    for (int c = 0; c < nh; ++c) B.hoff[c] = hz[c] * s2 + hx[c] * s1 + hy[c];

    // derivative tensors at the 343 integer offsets (near ones left zero),
    // stored compactly: only the entries d^g with g_z <= 2, |g| <= 2p that the
    // M2L reads, in (z, x, y) order; dmap[e] is the additive LDS address of
    // entry e (row padding -> ldd - 1, an address the layout never uses)
    B.ldd = dlayout_ldd(p);
    B.dmap.clear();
    for (int z = 0; z <= 2; ++z)
        for (int i = 0; i + z <= 2 * p; ++i)
            for (int j = 0; i + j + z <= 2 * p; ++j) B.dmap.push_back(z * s2 + i * s1 + j);
    B.ldc = pad4((int)B.dmap.size());
    if (B.ldc != dlayout_ldc(p)) throw std::logic_error("compact derivative table size");
    B.dmap.resize(B.ldc, B.ldd - 1);
    B.D.assign((size_t)343 * B.ldc, 0.0);
    B.Df.assign((size_t)343 * B.ldc, 0.0f);
    std::vector<ld> a;
    for (int kx = -3; kx <= 3; ++kx)
        for (int ky = -3; ky <= 3; ++ky)
            for (int kz = -3; kz <= 3; ++kz) {
                if (std::abs(kx) <= 1 && std::abs(ky) <= 1 && std::abs(kz) <= 1) continue;
                ld x[3] = {(ld)kx, (ld)ky, (ld)kz};
                inv_r_taylor(x, 2 * p, 2, a);
                size_t e = (size_t)((kx + 3) * 49 + (ky + 3) * 7 + (kz + 3)) * B.ldc;
                for (int z = 0; z <= 2; ++z)
                    for (int i = 0; i + z <= 2 * p; ++i)
                        for (int j = 0; i + j + z <= 2 * p; ++j, ++e) {
                            ld v = a[mono_index(i, j, z)] * fact(i) * fact(j) * fact(z);
                            B.D[e] = (double)v;
                            B.Df[e] = (float)v;
                        }
            }
    // V-list slot -> offset
    B.offs.assign(8 * kVSlots, 0);
    for (int o = 0; o < 8; ++o)
        for (int kx = -3; kx <= 3; ++kx)
            for (int ky = -3; ky <= 3; ++ky)
                for (int kz = -3; kz <= 3; ++kz) {
                    int s = vslot_of(o, kx, ky, kz);
                    if (s >= 0) B.offs[o * kVSlots + s] = (kx + 3) * 49 + (ky + 3) * 7 + (kz + 3);
                }

    // sign classes: parity-sorted rows (16-row tiles in the order of
    // sym_tile_class) and columns (padded to sym_colpad per class)
    B.srow.clear();
    B.scol.clear();
    std::vector<int> cls[8];
    for (int c = 0; c < 8; ++c) {
        for (int h = 0; h < nh; ++h)
            if ((hx[h] & 1) == ((c >> 2) & 1) && (hy[h] & 1) == ((c >> 1) & 1) && hz[h] == (c & 1)) {
                cls[c].push_back(h);
                B.scol.push_back(h);
            }
        const int cp = sym_colpad(p);
        B.scol.resize(((int)B.scol.size() + cp - 1) / cp * cp, -1);
    }
    for (int r = 0; r < sym_row_tiles(p); ++r) {
        const int c = sym_tile_class(p, r, true), t = sym_tile_class(p, r, false);
        for (int i = 0; i < 16; ++i)
            B.srow.push_back(16 * t + i < (int)cls[c].size() ? cls[c][16 * t + i] : -1);
    }
    if ((int)B.srow.size() != 16 * sym_row_tiles(p) || (int)B.scol.size() != 4 * sym_ksteps(p))
        throw std::logic_error("sign-class layout");
    // folded multipoles: parity-sorted in load order for sign-class orders,
    // else harmonic order
    B.mpos.assign(folded_ld(p), -1);
    B.mposf.assign(folded_ld(p), -1);
    if (m2l_sym(p)) {
        for (int ks = 0; ks < sym_ksteps(p); ++ks)
            for (int g = 0; g < 4; ++g) {
                B.mpos[sym_pos(ks, g, 2)] = B.scol[4 * ks + g];
                B.mposf[sym_pos(ks, g, 4)] = B.scol[4 * ks + g];
            }
    } else {
        for (int c = 0; c < nh; ++c) B.mpos[c] = B.mposf[c] = c;
    }
    // the classes of each octant: per axis, |k| in {1, 2} gives a pair of
    // members (+, -), 0 and 3 a single one (the octant admits only one of +-3)
    // (listed by zero-axis mask, so that a block runs the classes of one mask
    // one after the other)
    B.srep.assign(8 * kSymClasses, 0);
    B.smem.assign(8 * kSymClasses * 8, -1);
    for (int o = 0; o < 8; ++o) {
        int c = 0;
        for (int zsel = 0; zsel < 8; ++zsel)
            for (int ax = 0; ax <= 3; ++ax)
                for (int ay = 0; ay <= 3; ++ay)
                    for (int az = 0; az <= 3; ++az) {
                        if (ax <= 1 && ay <= 1 && az <= 1) continue;
                        const int a[3] = {ax, ay, az};
                        int rep[3], zero = 0, pair = 0;
                        for (int d = 0; d < 3; ++d) {
                            const int hi = (o >> (2 - d)) & 1; // octant bit: range [-3, 2] or [-2, 3]
                            rep[d] = a[d] == 3 ? (hi ? 3 : -3) : a[d];
                            if (a[d] == 0) zero |= 4 >> d;
                            if (a[d] == 1 || a[d] == 2) pair |= 4 >> d;
                        }
                        if (zero != zsel) continue;
                        B.srep[o * kSymClasses + c] = ((rep[0] + 3) * 49 + (rep[1] + 3) * 7 + (rep[2] + 3)) | (zero << 16);
                        for (int m = 0; m < 8; ++m) {
                            if (m & ~pair) continue;
                            int k[3];
                            for (int d = 0; d < 3; ++d) k[d] = (m & (4 >> d)) ? -rep[d] : rep[d];
                            const int slot = vslot_of(o, k[0], k[1], k[2]);
                            if (slot < 0) throw std::logic_error("sign class member outside the V slots");
                            B.smem[(o * kSymClasses + c) * 8 + m] = slot;
                        }
                        ++c;
                    }
        if (c != kSymClasses) throw std::logic_error("sign class count");
    }
    B.sslot.assign(8 * kVSlots, -1);
    for (int o = 0; o < 8; ++o) {
        for (int c = 0; c < kSymClasses; ++c)
            for (int m = 0; m < 8; ++m) {
                const int j = B.smem[(o * kSymClasses + c) * 8 + m];
                if (j >= 0) B.sslot[o * kVSlots + j] = c;
            }
        for (int j = 0; j < kVSlots; ++j)
            if (B.sslot[o * kVSlots + j] < 0) throw std::logic_error("V slot without a sign class");
    }

    // P2M: moments -> Mhat, table[g][a] = w_|a| C[a][g]
    std::vector<ld> C = p2m_polys(m);
    B.P2M.assign((size_t)nc * nc, 0.0);
    for (int id = 0; id < nc; ++id) {
        int d = m.deg(id);
        ld w = ((d & 1) ? -1.0L : 1.0L) / dfact(2 * d - 1);
        for (int g = 0; g < nc; ++g) B.P2M[(size_t)g * nc + id] = (double)(w * C[(size_t)id * nc + g]);
    }

    // M2M: S[o][a][b] = d Mhat'_b / d Mhat_a.  tau = (child - parent) / h_child.
    // The harmonic projection is linear: tabulate it on the monomial basis.
    std::vector<ld> Pi((size_t)nc * nc, 0.0L); // Pi[g][b]: projection of u^g, coefficient b
    for (int g = 0; g < nc; ++g) {
        std::vector<ld> unit(nc, 0.0L);
        unit[g] = 1.0L;
        std::vector<ld> h = harmonic_projection(m, unit, m.deg(g));
        for (int be = 0; be < nc; ++be) Pi[(size_t)g * nc + be] = h[be];
    }
    // P2L: d^b(1/|x|) = (-1)^n (2n-1)!! pi(x^b)(x) / |x|^(2n+1) (n = |b|), since
    // the non-harmonic part of x^b, a multiple of |x|^2, turns into a Laplacian
    // of 1/|x|.  So the harmonic components of Lhat are a fixed map of the
    // inverse moments W_g = sum q x^g / |x|^(2|g|+1):
    // P2L[g][c] = (-1)^n (2n-1)!! * (coefficient of x^g in pi(x^b(c))).
    B.P2L.assign((size_t)nc * ldh, 0.0);
    for (int g = 0; g < nc; ++g) {
        int n = m.deg(g);
        ld f = ((n & 1) ? -1.0L : 1.0L) * dfact(2 * n - 1);
        for (int c = 0; c < nh; ++c) {
            int be = mono_index(hx[c], hy[c], hz[c]);
            if (m.deg(be) != n) continue;
            B.P2L[(size_t)g * ldh + c] = (double)(f * Pi[(size_t)be * nc + g]);
        }
    }
    B.S.assign((size_t)8 * nc * nc, 0.0);
    for (int o = 0; o < 8; ++o) {
        ld tau[3] = {((o >> 2) & 1) ? 0.5L : -0.5L, ((o >> 1) & 1) ? 0.5L : -0.5L,
                     (o & 1) ? 0.5L : -0.5L};
        for (int al = 0; al < nc; ++al) {
            int ea[3] = {m.e[3 * al], m.e[3 * al + 1], m.e[3 * al + 2]};
            // shifted (non-harmonic) coefficients N_g = 2^-|g| (-tau)^(g-a)/(g-a)!
            std::vector<ld> out(nc, 0.0L);
            for (int g = 0; g < nc; ++g) {
                int eg[3] = {m.e[3 * g], m.e[3 * g + 1], m.e[3 * g + 2]};
                if (eg[0] < ea[0] || eg[1] < ea[1] || eg[2] < ea[2]) continue;
                ld v = std::ldexp(1.0L, -(eg[0] + eg[1] + eg[2]));
                for (int k = 0; k < 3; ++k) v *= ipow(-tau[k], eg[k] - ea[k]) / fact(eg[k] - ea[k]);
                // the projection keeps the degree: only that degree's block of Pi
                const int n = m.deg(g);
                for (int be = below(n); be < below(n + 1); ++be) out[be] += Pi[(size_t)g * nc + be] * v;
            }
            for (int be = 0; be < nc; ++be) B.S[((size_t)o * nc + al) * nc + be] = (double)out[be];
        }
    }
    // L2L: G[o][g][b] = tau^(g-b)/(g-b)! 2^-(|g|+1) for g >= b
    B.G.assign((size_t)8 * nc * nc, 0.0);
    for (int o = 0; o < 8; ++o) {
        ld tau[3] = {((o >> 2) & 1) ? 0.5L : -0.5L, ((o >> 1) & 1) ? 0.5L : -0.5L,
                     (o & 1) ? 0.5L : -0.5L};
        for (int g = 0; g < nc; ++g) {
            int eg[3] = {m.e[3 * g], m.e[3 * g + 1], m.e[3 * g + 2]};
            for (int be = 0; be < nc; ++be) {
                int eb[3] = {m.e[3 * be], m.e[3 * be + 1], m.e[3 * be + 2]};
                if (eg[0] < eb[0] || eg[1] < eb[1] || eg[2] < eb[2]) continue;
                ld v = std::ldexp(1.0L, -(eg[0] + eg[1] + eg[2] + 1));
                for (int k = 0; k < 3; ++k) v *= ipow(tau[k], eg[k] - eb[k]) / fact(eg[k] - eb[k]);
                B.G[((size_t)o * nc + g) * nc + be] = (double)v;
            }
        }
    }
    // fold: harmonic c = (I,J,kz) <- full (I-2a, J-2(m-a), kz+2m), coefficient (-1)^m C(m,a)
    B.fold_off.assign(ldh + 1, 0);
    for (int c = 0; c < ldh; ++c) {
        B.fold_off[c] = (int)B.fold_idx.size();
        if (c >= nh) continue;
        for (int mm = 0; hz[c] + 2 * mm <= p; ++mm)
            for (int aa = 0; aa <= mm; ++aa) {
                int i = hx[c] - 2 * aa, j = hy[c] - 2 * (mm - aa), k = hz[c] + 2 * mm;
                if (i < 0 || j < 0) continue;
                B.fold_idx.push_back(mono_index(i, j, k));
                B.fold_c.push_back((double)(((mm & 1) ? -1.0L : 1.0L) * binom(mm, aa)));
            }
    }
    B.fold_off[ldh] = (int)B.fold_idx.size();
    if ((int)B.fold_idx.size() != fold_terms(p)) throw std::logic_error("fold term count");
    // unfold: full b = (i,j,k) <- harmonic (i+2a, j+2(m-a), k mod 2), m = k/2
    B.unfold_off.assign(nc + 1, 0);
    for (int be = 0; be < nc; ++be) {
        B.unfold_off[be] = (int)B.unfold_idx.size();
        int i = m.e[3 * be], j = m.e[3 * be + 1], k = m.e[3 * be + 2], mm = k / 2;
        for (int aa = 0; aa <= mm; ++aa) {
            B.unfold_idx.push_back(harm_index(i + 2 * aa, j + 2 * (mm - aa), k & 1));
            B.unfold_c.push_back((double)(((mm & 1) ? -1.0L : 1.0L) * binom(mm, aa)));
        }
    }
    B.unfold_off[nc] = (int)B.unfold_idx.size();
    if ((int)B.unfold_idx.size() != fold_terms(p)) throw std::logic_error("unfold term count");
    // L2L on the harmonic components: a local expansion is harmonic, so the
    // full Lhat is the unfold of its (p+1)^2 components and the child's
    // components follow from the parent's ones:
    // GH[o][a][c] = sum_g unfold(g <- a) G[o][g][full index of c]
    B.GH.assign((size_t)8 * nh * nh, 0.0);
    for (int o = 0; o < 8; ++o)
        for (int g = 0; g < nc; ++g)
            for (int e = B.unfold_off[g]; e < B.unfold_off[g + 1]; ++e) {
                const int a = B.unfold_idx[e];
                const double w = B.unfold_c[e];
                for (int c = 0; c < nh; ++c)
                    B.GH[((size_t)o * nh + a) * nh + c] += w * B.G[((size_t)o * nc + g) * nc + mono_index(hx[c], hy[c], hz[c])];
            }
    // M2M on the folded components: the far field of a multipole, hence its
    // translation truncated at degree p, depends only on the folded vector, so
    // TMh[o][a][c] = sum over the fold terms (j, w) of c of w S[o][full a][j],
    // a taken as the full component with the same exponents; stored on the
    // folded positions (mpos) of the M2L operand layout
    const int ldmh = (int)B.mpos.size();
    std::vector<ld> TMh((size_t)8 * nh * nh, 0.0L);
    for (int o = 0; o < 8; ++o)
        for (int c = 0; c < nh; ++c)
            for (int e = B.fold_off[c]; e < B.fold_off[c + 1]; ++e) {
                const int j = B.fold_idx[e];
                const ld w = B.fold_c[e];
                for (int a = 0; a < nh; ++a)
                    TMh[((size_t)o * nh + a) * nh + c] +=
                        w * (ld)B.S[((size_t)o * nc + mono_index(hx[a], hy[a], hz[a])) * nc + j];
            }
    B.TM.assign((size_t)8 * ldmh * ldmh, 0.0);
    for (int o = 0; o < 8; ++o)
        for (int pa = 0; pa < ldmh; ++pa)
            for (int pb = 0; pb < ldmh; ++pb) {
                const int a = B.mpos[pa], c = B.mpos[pb];
                if (a >= 0 && c >= 0) B.TM[((size_t)o * ldmh + pa) * ldmh + pb] = (double)TMh[((size_t)o * nh + a) * nh + c];
            }
    B.hpos.assign(nh, -1);
    B.hposf.assign(nh, -1);
    for (int pa = 0; pa < ldmh; ++pa) {
        if (B.mpos[pa] >= 0) B.hpos[B.mpos[pa]] = pa;
        if (B.mposf[pa] >= 0) B.hposf[B.mposf[pa]] = pa;
    }
    // P2M followed by the fold: raw moments -> folded components (harmonic
    // order), FP2M[g][c] = sum over the fold terms (j, w) of c of w P2M[g][j];
    // both keep the degree, so column c only has entries of its degree's moments
    {
        std::vector<ld> F((size_t)nc * ldh, 0.0L);
        for (int c = 0; c < nh; ++c)
            for (int e = B.fold_off[c]; e < B.fold_off[c + 1]; ++e) {
                const int j = B.fold_idx[e], d = m.deg(j);
                const ld wf = (ld)B.fold_c[e] * (((d & 1) ? -1.0L : 1.0L) / dfact(2 * d - 1));
                for (int g = below(d); g < below(d + 1); ++g) F[(size_t)g * ldh + c] += wf * C[(size_t)j * nc + g];
            }
        B.FP2M.assign(F.begin(), F.end());
    }
    // full harmonic Mhat from the folded components (for M2P sources that are
    // not leaves): per degree n, the projections of the monomials with z
    // exponent <= 1 span the harmonic polynomials; with F the fold,
    // HR_n = Bn (F Bn)^-1, stored transposed ([nh][nc])
    B.HR.assign((size_t)nc * nh, 0.0);
    for (int n = 0; n <= p; ++n) {
        std::vector<int> hc; // harmonic components of degree n
        for (int c = 0; c < nh; ++c)
            if (hx[c] + hy[c] + hz[c] == n) hc.push_back(c);
        const int k = (int)hc.size();
        std::vector<ld> A((size_t)k * k, 0.0L); // A[r][s] = (F Bn)[hc r][hc s]
        for (int r = 0; r < k; ++r)
            for (int e = B.fold_off[hc[r]]; e < B.fold_off[hc[r] + 1]; ++e)
                for (int t = 0; t < k; ++t) {
                    const int g = mono_index(hx[hc[t]], hy[hc[t]], hz[hc[t]]);
                    A[(size_t)r * k + t] += (ld)B.fold_c[e] * Pi[(size_t)g * nc + B.fold_idx[e]];
                }
        // invert A (Gauss-Jordan with partial pivoting, long double)
        std::vector<ld> Ai((size_t)k * k, 0.0L);
        for (int r = 0; r < k; ++r) Ai[(size_t)r * k + r] = 1.0L;
        for (int col = 0; col < k; ++col) {
            int piv = col;
            for (int r = col + 1; r < k; ++r)
                if (std::fabs(A[(size_t)r * k + col]) > std::fabs(A[(size_t)piv * k + col])) piv = r;
            if (A[(size_t)piv * k + col] == 0.0L) throw std::logic_error("harmonic reconstruction: singular");
            for (int t = 0; t < k; ++t) {
                std::swap(A[(size_t)col * k + t], A[(size_t)piv * k + t]);
                std::swap(Ai[(size_t)col * k + t], Ai[(size_t)piv * k + t]);
            }
            const ld d = A[(size_t)col * k + col];
            for (int t = 0; t < k; ++t) { A[(size_t)col * k + t] /= d; Ai[(size_t)col * k + t] /= d; }
            for (int r = 0; r < k; ++r)
                if (r != col) {
                    const ld f = A[(size_t)r * k + col];
                    if (f == 0.0L) continue;
                    for (int t = 0; t < k; ++t) {
                        A[(size_t)r * k + t] -= f * A[(size_t)col * k + t];
                        Ai[(size_t)r * k + t] -= f * Ai[(size_t)col * k + t];
                    }
                }
        }
        // HR[be][hc s] = sum_t Bn[be][t] Ai[t][s], Bn[be][t] = Pi[mono(hc t)][be]
        for (int be = 0; be < nc; ++be) {
            if (m.deg(be) != n) continue;
            for (int sI = 0; sI < k; ++sI) {
                ld acc = 0.0L;
                for (int t = 0; t < k; ++t)
                    acc += Pi[(size_t)mono_index(hx[hc[t]], hy[hc[t]], hz[hc[t]]) * nc + be] * Ai[(size_t)t * k + sI];
                B.HR[(size_t)hc[sI] * nc + be] = (double)acc;
            }
        }
    }
}

struct Entry {
    OrderTables host;       // device pointers
    OrderTables *dev = nullptr;
};

std::mutex g_mu;
std::map<std::pair<int, int>, Entry> g_cache;

template <typename T>
int upload(const std::vector<T> &v, const T **out, std::string &err)
{
    void *d = nullptr;
    size_t bytes = sizeof(T) * (v.empty() ? 1 : v.size());
    if (hipMalloc(&d, bytes) != hipSuccess) { err = "hipMalloc failed for order tables"; return -1; }
    if (!v.empty() && hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
        err = "hipMemcpy failed for order tables";
        return -1;
    }
    *out = (const T *)d;
    return 0;
}

} // namespace

const OrderTables *get_order_tables(int p, const OrderTables **host_copy, std::string &err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { err = "hipGetDevice failed"; return nullptr; }
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, p);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        if (host_copy) *host_copy = &it->second.host;
        return it->second.dev;
    }
    Built B;
    build_tables(p, B);
    Entry e;
    OrderTables &t = e.host;
    t.p = p; t.nc = ncoef(p); t.nh = nharm(p); t.ldm = pad16(t.nc); t.ldh = pad16(t.nh);
    t.ldd = B.ldd; t.ldc = B.ldc; t.d3 = dlayout_s1(p); t.ldmh = folded_ld(p);
    if (upload(B.D, &t.D, err) || upload(B.Df, &t.Df, err) || upload(B.dmap, &t.dmap, err) ||
        upload(B.offs, &t.offs, err) ||
        upload(B.hoff, &t.hoff, err) || upload(B.GH, &t.GH, err) || upload(B.TM, &t.TM, err) ||
        upload(B.HR, &t.HR, err) || upload(B.hpos, &t.hpos, err) || upload(B.hposf, &t.hposf, err) ||
        upload(B.FP2M, &t.FP2M, err) ||
        upload(B.P2L, &t.P2L, err) || upload(B.fold_off, &t.fold_off, err) ||
        upload(B.fold_idx, &t.fold_idx, err) || upload(B.fold_c, &t.fold_c, err) ||
        upload(B.unfold_off, &t.unfold_off, err) || upload(B.unfold_idx, &t.unfold_idx, err) ||
        upload(B.unfold_c, &t.unfold_c, err) || upload(B.inv_fact, &t.inv_fact, err) ||
        upload(B.inv_w, &t.inv_w, err) || upload(B.exps, &t.exps, err) || upload(B.mpos, &t.mpos, err) || upload(B.mposf, &t.mposf, err) ||
        upload(B.srow, &t.srow, err) || upload(B.scol, &t.scol, err) || upload(B.srep, &t.srep, err) ||
        upload(B.smem, &t.smem, err) || upload(B.sslot, &t.sslot, err))
        return nullptr;
    void *d = nullptr;
    if (hipMalloc(&d, sizeof(OrderTables)) != hipSuccess ||
        hipMemcpy(d, &t, sizeof(OrderTables), hipMemcpyHostToDevice) != hipSuccess) {
        err = "hipMalloc/hipMemcpy failed for order tables";
        return nullptr;
    }
    e.dev = (OrderTables *)d;
    auto &slot = g_cache[key];
    slot = e;
    if (host_copy) *host_copy = &slot.host;
    return slot.dev;
}

// Host-side copies for tests of the closed forms (same construction).
int host_order_tables(int p, int which, std::vector<double> &out)
{
    Built B;
    build_tables(p, B);
    switch (which) {
    case 0: out = B.D; return B.ldc;
    case 1: out = B.S; return ncoef(p);
    case 2: out = B.G; return ncoef(p);
    case 3: out = B.P2M; return ncoef(p);
    case 4: out = B.HR; return ncoef(p);
    case 9: out.assign(B.mpos.begin(), B.mpos.end()); return folded_ld(p);
    default: return -1;
    }
}

} // namespace fmm

extern "C" int fmm_order_table(int32_t order, int32_t which, double *out_host, int64_t capacity,
                               int64_t *count, int32_t *ld)
{
    if (order < 0 || order > fmm::kMaxOrder || which < 0 || which > 9 || !count || !ld) return FMM_EINVAL;
    std::vector<double> t;
    try {
        *ld = which <= 4 || which == 9 ? fmm::host_order_tables(order, which, t)
                                       : fmm::host_rotation_tables(order, which - 5, t);
    } catch (...) {
        return FMM_EUNSUPPORTED;
    }
    *count = (int64_t)t.size();
    if (out_host) {
        if (capacity < (int64_t)t.size()) return FMM_EINVAL;
        std::memcpy(out_host, t.data(), sizeof(double) * t.size());
    }
    return FMM_OK;
}
