/*
 * The DA-FMM for a second non-oscillatory kernel: the Plummer-softened
 * Coulomb potential K(x) = 1 / sqrt(|x|^2 + eps^2) (eps = 0 is 1/|x|).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper notes that the DA-based formulation, like the Cartesian tensor
 * one, extends to any non-oscillatory kernel (closing remark of Sec. 3.4 on
 * the M2L, and the comparison with other FMMs in Sec. 3.5).  Without the
 * inversion d = r / r^2 that Eq. P2M uses for 1/r, the expansions are the
 * plain Cartesian Taylor ones, and the one kernel-specific ingredient is the
 * Taylor series of K about a point x0, computed in the DA algebra the way
 * Table 1 computes it for 1/r (Sec. 3: the polynomial |x0 + z|^2 + eps^2 in
 * z, then its square root, then the inverse), to order 2p for the M2L and
 * p + 1 for the M2P and its gradient.  With T(x0) those coefficients, so that
 * d^g K(x0) = g! T_g(x0), and y_i = x_i - c the charge offsets:
 *   P2M  M_a = sum_i q_i (-y_i)^a / a!,  so that  phi(x) = sum_a M_a d^a K(x - c)
 *   M2M  M_a(P) = sum_{b <= a} M_b(C) (-t)^(a-b) / (a-b)!,  t = c_C - c_P
 *   M2L  L_b(B) += sum_a M_a(C) (a+b)! / b! T_(a+b)(c_B - c_C)
 *   P2L  L_b(B) += q_j T_b(c_B - x_j)
 *   L2L  L_b(C) += sum_{g >= b} L_g(P) C(g, b) t^(g-b),  t = c_C - c_P
 *   L2P  phi(c + z) = sum_b L_b z^b   (field: minus its gradient)
 *   M2P  phi(x) = sum_a M_a a! T_a(x - c),  grad_k = sum_a M_a (a + e_k)! T_(a+e_k)
 *   P2P  q_j K(x_i - x_j) for j != i; a pair with |x|^2 + eps^2 = 0 (coincident
 *        points at eps = 0) contributes nothing, as for the Coulomb kernel.
 * Multi-index factorials and binomials are products over the three axes.
 * The tree, the lists and the order of the passes are those of oracle_fmm.
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* accessors defined in tree.c */
int64_t oracle_tree_n(const oracle_tree *t);
int64_t oracle_tree_nboxes(const oracle_tree *t);
int oracle_tree_depth(const oracle_tree *t);
const int64_t *oracle_tree_perm(const oracle_tree *t);
const int32_t *oracle_tree_level(const oracle_tree *t);
const int32_t *oracle_tree_parent(const oracle_tree *t);
const int32_t *oracle_tree_child_begin(const oracle_tree *t);
const int32_t *oracle_tree_nchild(const oracle_tree *t);
const int64_t *oracle_tree_first(const oracle_tree *t);
const int64_t *oracle_tree_count(const oracle_tree *t);
const int64_t *oracle_tree_off(const oracle_tree *t, int w);
const int32_t *oracle_tree_src(const oracle_tree *t, int w);
const int64_t *oracle_tree_level_begin(const oracle_tree *t);
void oracle_tree_center(const oracle_tree *t, int32_t b, double c[3]);
double oracle_tree_width(const oracle_tree *t, int l);
void oracle_tree_coords(const oracle_tree *t, int32_t b, int64_t g[3]);

/* n! for n <= 22 (exact in double) */
static const double FACT[23] = {
    1.0, 1.0, 2.0, 6.0,
    24.0, 120.0, 720.0, 5040.0,
    40320.0, 362880.0, 3628800.0, 39916800.0,
    479001600.0, 6227020800.0, 87178291200.0, 1307674368000.0,
    20922789888000.0, 355687428096000.0, 6402373705728000.0, 121645100408832000.0,
    2432902008176640000.0, 51090942171709440000.0, 1124000727777607680000.0};
static double fact(int n) { return FACT[n]; }
static double mfact(const int e[3]) { return fact(e[0]) * fact(e[1]) * fact(e[2]); }
static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }
static double ipow(double x, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

/* Taylor coefficients of K(x0 + z) in z to the context's order, by the DA
 * algebra: v = (|x0|^2 + eps^2) + 2 x0.z + |z|^2, then sqrt, then inverse. */
static void soft_taylor_ctx(const da_ctx *c, const double x0[3], double eps, double *out)
{
    double *v = calloc((size_t)c->n, sizeof(double)), *s = calloc((size_t)c->n, sizeof(double));
    v[0] = x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2] + eps * eps;
    if (c->p >= 1) {
        v[da_index(1, 0, 0)] = 2.0 * x0[0];
        v[da_index(0, 1, 0)] = 2.0 * x0[1];
        v[da_index(0, 0, 1)] = 2.0 * x0[2];
    }
    if (c->p >= 2) {
        v[da_index(2, 0, 0)] = 1.0;
        v[da_index(0, 2, 0)] = 1.0;
        v[da_index(0, 0, 2)] = 1.0;
    }
    da_sqrt(c, v, s);
    da_inv(c, s, out);
    free(v); free(s);
}

int oracle_soft_taylor(int p, const double x0[3], double eps, double *out)
{
    if (p < 0 || eps < 0.0) return -1;
    if (x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2] + eps * eps <= 0.0) return -1;
    da_ctx c;
    if (da_ctx_init(&c, p)) return -1;
    soft_taylor_ctx(&c, x0, eps, out);
    da_ctx_free(&c);
    return 0;
}

/* ---- the operators on one box or pair ---- */
static void s_p2m(const da_ctx *c, const double y[3], double q, double *M)
{
    for (int a = 0; a < c->n; ++a) {
        const int *e = c->e[a];
        M[a] += q * ipow(-y[0], e[0]) * ipow(-y[1], e[1]) * ipow(-y[2], e[2]) / mfact(e);
    }
}

static void s_m2m(const da_ctx *c, const double t[3], const double *Mc, double *Mp)
{
    for (int a = 0; a < c->n; ++a) {
        const int *ea = c->e[a];
        double s = 0.0;
        for (int b = 0; b < c->n; ++b) {
            const int *eb = c->e[b];
            if (eb[0] > ea[0] || eb[1] > ea[1] || eb[2] > ea[2]) continue;
            const int d[3] = {ea[0] - eb[0], ea[1] - eb[1], ea[2] - eb[2]};
            s += Mc[b] * ipow(-t[0], d[0]) * ipow(-t[1], d[1]) * ipow(-t[2], d[2]) / mfact(d);
        }
        Mp[a] += s;
    }
}

/* The M2L's fixed structure: for output b and input a, the position of
 * a + b among the order-2p coefficients and the factor (a+b)! / b!. */
typedef struct { int *ix; double *cf; } m2l_index;
static void m2l_index_init(const da_ctx *c, m2l_index *m)
{
    const size_t n = (size_t)c->n;
    m->ix = malloc(sizeof(int) * n * n);
    m->cf = malloc(sizeof(double) * n * n);
    for (int b = 0; b < c->n; ++b) {
        const int *eb = c->e[b];
        for (int a = 0; a < c->n; ++a) {
            const int *ea = c->e[a];
            const int g[3] = {ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2]};
            m->ix[(size_t)b * n + a] = da_index(g[0], g[1], g[2]);
            m->cf[(size_t)b * n + a] = mfact(g) / mfact(eb);
        }
    }
}
static void m2l_index_free(m2l_index *m) { free(m->ix); free(m->cf); }

/* L_b += sum_a M_a (a+b)!/b! T_(a+b); T: coefficients of order 2p */
static void s_m2l(const da_ctx *c, const m2l_index *mi, const double *T, const double *M, double *L)
{
    const size_t n = (size_t)c->n;
    for (int b = 0; b < c->n; ++b) {
        const int *ix = mi->ix + (size_t)b * n;
        const double *cf = mi->cf + (size_t)b * n;
        double s = 0.0;
        for (int a = 0; a < c->n; ++a) s += M[a] * cf[a] * T[ix[a]];
        L[b] += s;
    }
}

static void s_l2l(const da_ctx *c, const double t[3], const double *Lp, double *Lc)
{
    for (int b = 0; b < c->n; ++b) {
        const int *eb = c->e[b];
        double s = 0.0;
        for (int g = 0; g < c->n; ++g) {
            const int *eg = c->e[g];
            if (eg[0] < eb[0] || eg[1] < eb[1] || eg[2] < eb[2]) continue;
            double w = Lp[g];
            for (int k = 0; k < 3; ++k) w *= binom(eg[k], eb[k]) * ipow(t[k], eg[k] - eb[k]);
            s += w;
        }
        Lc[b] += s;
    }
}

static void s_l2p(const da_ctx *c, const double *L, const double z[3], double *phi, double g[3])
{
    double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int b = 0; b < c->n; ++b) {
        const int *e = c->e[b];
        const double px = ipow(z[0], e[0]), py = ipow(z[1], e[1]), pz = ipow(z[2], e[2]);
        f += L[b] * px * py * pz;
        if (e[0]) gx += L[b] * e[0] * ipow(z[0], e[0] - 1) * py * pz;
        if (e[1]) gy += L[b] * e[1] * px * ipow(z[1], e[1] - 1) * pz;
        if (e[2]) gz += L[b] * e[2] * px * py * ipow(z[2], e[2] - 1);
    }
    *phi = f;
    g[0] = gx; g[1] = gy; g[2] = gz;
}

/* M of order p (context c), T of order p + 1 (context c1) at x - c_s */
static void s_m2p(const da_ctx *c, const double *M, const double *T, double *phi, double g[3])
{
    double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int a = 0; a < c->n; ++a) {
        const int *e = c->e[a];
        f += M[a] * mfact(e) * T[da_index(e[0], e[1], e[2])];
        const int ex[3] = {e[0] + 1, e[1], e[2]}, ey[3] = {e[0], e[1] + 1, e[2]}, ez[3] = {e[0], e[1], e[2] + 1};
        gx += M[a] * mfact(ex) * T[da_index(ex[0], ex[1], ex[2])];
        gy += M[a] * mfact(ey) * T[da_index(ey[0], ey[1], ey[2])];
        gz += M[a] * mfact(ez) * T[da_index(ez[0], ez[1], ez[2])];
    }
    *phi = f;
    g[0] = gx; g[1] = gy; g[2] = gz;
}

/* ---- direct sum ---- */
int oracle_direct_soft(int64_t n, const double *xyz, const double *q, double eps, int64_t nt,
                       const int64_t *targets, double *phi, double *field)
{
    if (n < 0 || nt < 0 || eps < 0.0 || (!targets && nt != n)) return -1;
    const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        double ph = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
                         dz = xyz[3 * i + 2] - xyz[3 * j + 2];
            const double s2 = dx * dx + dy * dy + dz * dz + e2;
            if (s2 == 0.0) continue;
            const double s = sqrt(s2);
            ph += q[j] / s;
            const double f = q[j] / (s2 * s);
            ex += f * dx; ey += f * dy; ez += f * dz;
        }
        phi[t] = ph;
        if (field) { field[3 * t] = ex; field[3 * t + 1] = ey; field[3 * t + 2] = ez; }
    }
    return 0;
}

/* ---- single operators, for the tests ---- */
int oracle_soft_op(int op, int p, double eps, const double *a3, const double *b3, const double *in, double *out)
{
    da_ctx c, c2;
    if (p < 0 || eps < 0.0 || da_ctx_init(&c, p)) return -1;
    if (da_ctx_init(&c2, 2 * p)) { da_ctx_free(&c); return -1; }
    int rc = 0;
    memset(out, 0, sizeof(double) * (size_t)c.n);
    if (op == 0) { /* M2M: a3 child centre, b3 parent centre */
        const double t[3] = {a3[0] - b3[0], a3[1] - b3[1], a3[2] - b3[2]};
        s_m2m(&c, t, in, out);
    } else if (op == 1) { /* M2L: a3 source centre, b3 target centre */
        const double k[3] = {b3[0] - a3[0], b3[1] - a3[1], b3[2] - a3[2]};
        double *T = calloc((size_t)c2.n, sizeof(double));
        if (k[0] * k[0] + k[1] * k[1] + k[2] * k[2] + eps * eps > 0.0) {
            m2l_index mi;
            m2l_index_init(&c, &mi);
            soft_taylor_ctx(&c2, k, eps, T);
            s_m2l(&c, &mi, T, in, out);
            m2l_index_free(&mi);
        } else rc = -1;
        free(T);
    } else if (op == 2) { /* L2L: a3 parent centre, b3 child centre */
        const double t[3] = {b3[0] - a3[0], b3[1] - a3[1], b3[2] - a3[2]};
        s_l2l(&c, t, in, out);
    } else rc = -1;
    da_ctx_free(&c); da_ctx_free(&c2);
    return rc;
}

int oracle_soft_p2m(int p, int64_t n, const double *xyz, const double *q, const double center[3], double *M)
{
    da_ctx c;
    if (p < 0 || n < 0 || da_ctx_init(&c, p)) return -1;
    memset(M, 0, sizeof(double) * (size_t)c.n);
    for (int64_t i = 0; i < n; ++i) {
        const double y[3] = {xyz[3 * i] - center[0], xyz[3 * i + 1] - center[1], xyz[3 * i + 2] - center[2]};
        s_p2m(&c, y, q[i], M);
    }
    da_ctx_free(&c);
    return 0;
}

int oracle_soft_p2l(int p, double eps, int64_t n, const double *xyz, const double *q, const double center[3],
                    double *L)
{
    da_ctx c;
    if (p < 0 || n < 0 || eps < 0.0 || da_ctx_init(&c, p)) return -1;
    memset(L, 0, sizeof(double) * (size_t)c.n);
    double *T = calloc((size_t)c.n, sizeof(double));
    int rc = 0;
    for (int64_t i = 0; i < n && !rc; ++i) {
        const double x0[3] = {center[0] - xyz[3 * i], center[1] - xyz[3 * i + 1], center[2] - xyz[3 * i + 2]};
        if (x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2] + eps * eps <= 0.0) { rc = -1; break; }
        soft_taylor_ctx(&c, x0, eps, T);
        for (int b = 0; b < c.n; ++b) L[b] += q[i] * T[b];
    }
    free(T);
    da_ctx_free(&c);
    return rc;
}

/* ---- the FMM (Sec. 1 recipe on the reference tree, operators above) ---- */
int oracle_fmm_soft(const oracle_tree *t, int p, double eps, const double *xyz, const double *q,
                    double *phi_out, double *field_out, double *M_out, double *L_out)
{
    if (!t || p < 0 || eps < 0.0) return -1;
    da_ctx c, c1, c2;
    if (da_ctx_init(&c, p)) return -1;
    if (da_ctx_init(&c1, p + 1)) { da_ctx_free(&c); return -1; }
    if (da_ctx_init(&c2, 2 * p)) { da_ctx_free(&c); da_ctx_free(&c1); return -1; }
    const int n = c.n;
    const int64_t N = oracle_tree_n(t), nb = oracle_tree_nboxes(t);
    const int depth = oracle_tree_depth(t);
    const int64_t *perm = oracle_tree_perm(t), *first = oracle_tree_first(t), *count = oracle_tree_count(t);
    const int32_t *level = oracle_tree_level(t), *parent = oracle_tree_parent(t);
    const int32_t *cbeg = oracle_tree_child_begin(t), *nch = oracle_tree_nchild(t);
    const int64_t *lbeg = oracle_tree_level_begin(t);
    const int64_t *Uo = oracle_tree_off(t, 0), *Vo = oracle_tree_off(t, 1), *Wo = oracle_tree_off(t, 2),
                  *Xo = oracle_tree_off(t, 3);
    const int32_t *Us = oracle_tree_src(t, 0), *Vs = oracle_tree_src(t, 1), *Ws = oracle_tree_src(t, 2),
                  *Xs = oracle_tree_src(t, 3);
    double *xs = malloc(sizeof(double) * 3 * (size_t)(N ? N : 1)), *qs = malloc(sizeof(double) * (size_t)(N ? N : 1));
    for (int64_t i = 0; i < N; ++i) {
        for (int k = 0; k < 3; ++k) xs[3 * i + k] = xyz[3 * perm[i] + k];
        qs[i] = q[perm[i]];
    }
    double *M = calloc((size_t)(nb * n), sizeof(double));
    double *L = calloc((size_t)(nb * n), sizeof(double));
    double *cen = malloc(sizeof(double) * 3 * (size_t)nb);
    for (int64_t b = 0; b < nb; ++b) oracle_tree_center(t, (int32_t)b, cen + 3 * b);

    /* P2M at the leaves */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
        if (nch[b] != 0) continue;
        for (int64_t i = first[b]; i < first[b] + count[b]; ++i) {
            const double y[3] = {xs[3 * i] - cen[3 * b], xs[3 * i + 1] - cen[3 * b + 1], xs[3 * i + 2] - cen[3 * b + 2]};
            s_p2m(&c, y, qs[i], M + b * n);
        }
    }
    /* upward pass, finest level first */
    for (int l = depth; l >= 1; --l) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = lbeg[l - 1]; b < lbeg[l]; ++b)
            for (int k = 0; k < nch[b]; ++k) {
                const int32_t ch = cbeg[b] + k;
                const double tt[3] = {cen[3 * ch] - cen[3 * b], cen[3 * ch + 1] - cen[3 * b + 1],
                                      cen[3 * ch + 2] - cen[3 * b + 2]};
                s_m2m(&c, tt, M + (int64_t)ch * n, M + b * n);
            }
    }
    /* downward pass level by level: M2L (V) + P2L (X), then L2L.  The
     * kernel's coefficients at an offset depend on the level (eps does not
     * scale with the boxes), so they are kept per level and offset. */
    double *T343 = malloc(sizeof(double) * 343 * (size_t)c2.n);
    int have[343];
    m2l_index mi;
    m2l_index_init(&c, &mi);
    for (int l = 2; l <= depth; ++l) {
        const double h = oracle_tree_width(t, l);
        memset(have, 0, sizeof(have));
        for (int64_t b = lbeg[l]; b < lbeg[l + 1]; ++b)
            for (int64_t e = Vo[b]; e < Vo[b + 1]; ++e) {
                int64_t gb[3], gs[3];
                oracle_tree_coords(t, (int32_t)b, gb);
                oracle_tree_coords(t, Vs[e], gs);
                have[(gb[0] - gs[0] + 3) * 49 + (gb[1] - gs[1] + 3) * 7 + (gb[2] - gs[2] + 3)] = 1;
            }
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k < 343; ++k) {
            if (!have[k]) continue;
            const double k0[3] = {(k / 49 - 3) * h, ((k / 7) % 7 - 3) * h, (k % 7 - 3) * h};
            soft_taylor_ctx(&c2, k0, eps, T343 + (size_t)k * c2.n);
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = lbeg[l]; b < lbeg[l + 1]; ++b) {
            double *T = malloc(sizeof(double) * (size_t)n);
            for (int64_t e = Vo[b]; e < Vo[b + 1]; ++e) {
                int64_t gb[3], gs[3];
                oracle_tree_coords(t, (int32_t)b, gb);
                oracle_tree_coords(t, Vs[e], gs);
                const int k = (int)((gb[0] - gs[0] + 3) * 49 + (gb[1] - gs[1] + 3) * 7 + (gb[2] - gs[2] + 3));
                s_m2l(&c, &mi, T343 + (size_t)k * c2.n, M + (int64_t)Vs[e] * n, L + b * n);
            }
            for (int64_t e = Xo[b]; e < Xo[b + 1]; ++e) {
                const int32_t s = Xs[e];
                for (int64_t i = first[s]; i < first[s] + count[s]; ++i) {
                    const double x0[3] = {cen[3 * b] - xs[3 * i], cen[3 * b + 1] - xs[3 * i + 1],
                                          cen[3 * b + 2] - xs[3 * i + 2]};
                    soft_taylor_ctx(&c, x0, eps, T);
                    for (int a = 0; a < n; ++a) L[b * n + a] += qs[i] * T[a];
                }
            }
            free(T);
        }
        if (l == depth) break;
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t ch = lbeg[l + 1]; ch < lbeg[l + 2]; ++ch) {
            const int32_t b = parent[ch];
            const double tt[3] = {cen[3 * ch] - cen[3 * b], cen[3 * ch + 1] - cen[3 * b + 1],
                                  cen[3 * ch + 2] - cen[3 * b + 2]};
            s_l2l(&c, tt, L + (int64_t)b * n, L + ch * n);
        }
    }
    free(T343);
    m2l_index_free(&mi);

    /* evaluation at the leaves: L2P + M2P (W list) + P2P (U list) */
    double *phs = calloc((size_t)(N ? N : 1), sizeof(double)), *fs = calloc(3 * (size_t)(N ? N : 1), sizeof(double));
    const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
        if (nch[b] != 0) continue;
        double *T = malloc(sizeof(double) * (size_t)c1.n);
        for (int64_t i = first[b]; i < first[b] + count[b]; ++i) {
            double ph = 0.0, g[3] = {0, 0, 0}, pv, gv[3];
            if (level[b] >= 2) {
                const double z[3] = {xs[3 * i] - cen[3 * b], xs[3 * i + 1] - cen[3 * b + 1], xs[3 * i + 2] - cen[3 * b + 2]};
                s_l2p(&c, L + b * n, z, &pv, gv);
                ph += pv; g[0] += gv[0]; g[1] += gv[1]; g[2] += gv[2];
            }
            for (int64_t e = Wo[b]; e < Wo[b + 1]; ++e) {
                const int32_t s = Ws[e];
                const double x0[3] = {xs[3 * i] - cen[3 * s], xs[3 * i + 1] - cen[3 * s + 1], xs[3 * i + 2] - cen[3 * s + 2]};
                soft_taylor_ctx(&c1, x0, eps, T);
                s_m2p(&c, M + (int64_t)s * n, T, &pv, gv);
                ph += pv; g[0] += gv[0]; g[1] += gv[1]; g[2] += gv[2];
            }
            double ex = -g[0], ey = -g[1], ez = -g[2];
            for (int64_t e = Uo[b]; e < Uo[b + 1]; ++e) {
                const int32_t s = Us[e];
                for (int64_t j = first[s]; j < first[s] + count[s]; ++j) {
                    if (j == i) continue;
                    const double dx = xs[3 * i] - xs[3 * j], dy = xs[3 * i + 1] - xs[3 * j + 1],
                                 dz = xs[3 * i + 2] - xs[3 * j + 2];
                    const double s2 = dx * dx + dy * dy + dz * dz + e2;
                    if (s2 == 0.0) continue;
                    const double sq = sqrt(s2);
                    ph += qs[j] / sq;
                    const double f = qs[j] / (s2 * sq);
                    ex += f * dx; ey += f * dy; ez += f * dz;
                }
            }
            phs[i] = ph;
            fs[3 * i] = ex; fs[3 * i + 1] = ey; fs[3 * i + 2] = ez;
        }
        free(T);
    }
    for (int64_t i = 0; i < N; ++i) {
        if (phi_out) phi_out[perm[i]] = phs[i];
        if (field_out)
            for (int k = 0; k < 3; ++k) field_out[3 * perm[i] + k] = fs[3 * i + k];
    }
    if (M_out) memcpy(M_out, M, sizeof(double) * (size_t)(nb * n));
    if (L_out) memcpy(L_out, L, sizeof(double) * (size_t)(nb * n));
    free(phs); free(fs); free(xs); free(qs); free(M); free(L); free(cen);
    da_ctx_free(&c); da_ctx_free(&c1); da_ctx_free(&c2);
    return 0;
}
