/*
 * The DA-based FMM operators of Sec. 2 and the FMM recipe of Sec. 1, built
 * from the truncated power series algebra in tpsa.c.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Notation of Sec. 2: a multipole expansion phi_M is a DA vector in the
 * inverted variable d = r / r^2 about the box centre, with phi = |d| phi_M(d)
 * (Eq. P2M_phi); a local expansion phi_L is a DA vector in d' = r - r0 about
 * the box centre.  Readings of garbled passages (restated where used):
 *   - Eq. P2M prints 2 r.d inside the root; the expansion of 1/|r_i - r| needs
 *     1 + r_i^2 d^2 - 2 r_i.d with r_i the charge offset from the box centre;
 *   - Sec. 2.3 prints R = 1/|r0 + r'| but Eq. m2l multiplies by sqrt(R) to get
 *     the 1/r factor and divides r0 + r' by R to get d, so R = 1/|r0 + r'|^2;
 *   - fields are E = -grad(phi), obtained by running the evaluation in an
 *     order-1 DA in the target offset (the paper computes potentials only).
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

static double *da_new(const da_ctx *c) { return calloc((size_t)c->n, sizeof(double)); }

/* a[i] += val for the monomial x^e, dropped when its degree exceeds the order */
static void da_add_mono(const da_ctx *c, double *a, int i, int j, int k, double val)
{
    if (i + j + k <= c->p) a[da_index(i, j, k)] += val;
}

/* the DA vector c0 + d_v */
static void da_var(const da_ctx *c, double *a, int v, double c0)
{
    da_zero(c, a);
    a[0] = c0;
    da_add_mono(c, a, v == 0, v == 1, v == 2, 1.0);
}

/* |d|^2 = d1^2 + d2^2 + d3^2 as a DA vector */
static void da_norm2_vars(const da_ctx *c, double *out)
{
    da_zero(c, out);
    da_add_mono(c, out, 2, 0, 0, 1.0);
    da_add_mono(c, out, 0, 2, 0, 1.0);
    da_add_mono(c, out, 0, 0, 2, 1.0);
}

/* ---- P2M (Sec. 2.1, Eq. P2M; Sec. 3.1: a square root and an inverse) ---- */
static void p2m_add(const da_ctx *c, const double y[3], double q, double *M)
{
    double *v = da_new(c), *s = da_new(c), *t = da_new(c);
    double y2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    da_norm2_vars(c, v);
    for (int i = 0; i < c->n; ++i) v[i] *= y2;       /* r_i^2 d^2 */
    v[0] += 1.0;                                      /* 1 + ...   */
    for (int k = 0; k < 3; ++k)                       /* - 2 r_i.d */
        da_add_mono(c, v, k == 0, k == 1, k == 2, -2.0 * y[k]);
    da_sqrt(c, v, s);
    da_inv(c, s, t);
    for (int i = 0; i < c->n; ++i) M[i] += q * t[i];
    free(v); free(s); free(t);
}

int oracle_p2m(int p, int64_t n, const double *xyz, const double *q, const double cen[3],
               double *M)
{
    da_ctx c;
    if (da_ctx_init(&c, p)) return -1;
    da_zero(&c, M);
    for (int64_t i = 0; i < n; ++i) {
        double y[3] = {xyz[3 * i] - cen[0], xyz[3 * i + 1] - cen[1], xyz[3 * i + 2] - cen[2]};
        p2m_add(&c, y, q[i], M);
    }
    da_ctx_free(&c);
    return 0;
}

/* ---- translation maps: DA images of the basis monomials ----
 * Each translation is linear in the expansion it acts on: out = pre *
 * (in o args) = sum_J in_J * (pre * args^J).  cols[J*n + m] holds pre*args^J. */

/* M2M (Sec. 2.2, Eq. m2m): child centre at the origin, parent at r0.
 * M1: d = (d' + d'^2 r0) R, R = 1/(1 + r0^2 d'^2 + 2 r0.d'); pre = sqrt(R). */
static void m2m_map(const da_ctx *c, const double r0[3], double *args[3], double *pre)
{
    double *dd = da_new(c), *den = da_new(c), *R = da_new(c), *t = da_new(c);
    double r02 = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
    da_norm2_vars(c, dd);
    for (int i = 0; i < c->n; ++i) den[i] = r02 * dd[i];
    den[0] += 1.0;
    for (int k = 0; k < 3; ++k) da_add_mono(c, den, k == 0, k == 1, k == 2, 2.0 * r0[k]);
    da_inv(c, den, R);
    for (int k = 0; k < 3; ++k) {
        da_var(c, t, k, 0.0);
        for (int i = 0; i < c->n; ++i) t[i] += dd[i] * r0[k];
        da_mul(c, t, R, args[k]);
    }
    da_sqrt(c, R, pre);
    free(dd); free(den); free(R); free(t);
}

/* M2L (Sec. 2.3, Eq. m2l): source centre at the origin, target at r0.
 * M2: d = (r0 + r') R with R = 1/|r0 + r'|^2 (reading); pre = sqrt(R). */
static void m2l_map(const da_ctx *c, const double r0[3], double *args[3], double *pre)
{
    double *s = da_new(c), *R = da_new(c), *t = da_new(c);
    for (int k = 0; k < 3; ++k) {
        da_var(c, t, k, r0[k]);
        da_mul(c, t, t, t);
        for (int i = 0; i < c->n; ++i) s[i] += t[i];
    }
    da_inv(c, s, R);
    for (int k = 0; k < 3; ++k) {
        da_var(c, t, k, r0[k]);
        da_mul(c, t, R, args[k]);
    }
    da_sqrt(c, R, pre);
    free(s); free(R); free(t);
}

/* L2L (Sec. 2.5, Eq. l2l): parent centre at the origin, child at r0.
 * M3: d = r0 + d' (a linear shift); no prefactor. */
static void l2l_map(const da_ctx *c, const double r0[3], double *args[3], double *pre)
{
    for (int k = 0; k < 3; ++k) da_var(c, args[k], k, r0[k]);
    da_zero(c, pre);
    pre[0] = 1.0;
}

typedef void (*map_fn)(const da_ctx *, const double *, double **, double *);

static void translation_matrix(const da_ctx *c, map_fn f, const double r0[3], double *cols)
{
    double *args[3] = {da_new(c), da_new(c), da_new(c)}, *pre = da_new(c);
    f(c, r0, args, pre);
    da_monomials(c, c, (const double *const *)args, cols);
    for (int J = 0; J < c->n; ++J) da_mul(c, cols + (size_t)J * c->n, pre, cols + (size_t)J * c->n);
    for (int k = 0; k < 3; ++k) free(args[k]);
    free(pre);
}

static void apply_matrix(const da_ctx *c, const double *cols, const double *in, double *out)
{
    for (int J = 0; J < c->n; ++J) {
        double a = in[J];
        if (a == 0.0) continue;
        const double *col = cols + (size_t)J * c->n;
        for (int m = 0; m < c->n; ++m) out[m] += a * col[m];
    }
}

/* translation by full DA composition: out += pre * (in o args) */
static void translate(const da_ctx *c, map_fn f, const double r0[3], const double *in,
                      double *out)
{
    double *args[3] = {da_new(c), da_new(c), da_new(c)}, *pre = da_new(c), *t = da_new(c);
    f(c, r0, args, pre);
    da_compose(c, in, c, (const double *const *)args, t);
    da_mul(c, t, pre, t);
    for (int m = 0; m < c->n; ++m) out[m] += t[m];
    for (int k = 0; k < 3; ++k) free(args[k]);
    free(pre); free(t);
}

int oracle_m2m(int p, const double cc[3], const double pc[3], const double *M, double *Mout)
{
    da_ctx c;
    if (da_ctx_init(&c, p)) return -1;
    double r0[3] = {pc[0] - cc[0], pc[1] - cc[1], pc[2] - cc[2]};
    da_zero(&c, Mout);
    translate(&c, m2m_map, r0, M, Mout);
    da_ctx_free(&c);
    return 0;
}

int oracle_m2l(int p, const double sc[3], const double tc[3], const double *M, double *L)
{
    da_ctx c;
    if (da_ctx_init(&c, p)) return -1;
    double r0[3] = {tc[0] - sc[0], tc[1] - sc[1], tc[2] - sc[2]};
    da_zero(&c, L);
    translate(&c, m2l_map, r0, M, L);
    da_ctx_free(&c);
    return 0;
}

int oracle_l2l(int p, const double pc[3], const double cc[3], const double *L, double *Lout)
{
    da_ctx c;
    if (da_ctx_init(&c, p)) return -1;
    double r0[3] = {cc[0] - pc[0], cc[1] - pc[1], cc[2] - pc[2]};
    da_zero(&c, Lout);
    translate(&c, l2l_map, r0, L, Lout);
    da_ctx_free(&c);
    return 0;
}

/* ---- P2L (Sec. 2.4, Eq. P2L): L += q / |r0 - r_i + d'| ---- */
static void p2l_add(const da_ctx *c, const double cen[3], const double x[3], double q, double *L)
{
    double *s = da_new(c), *t = da_new(c), *u = da_new(c);
    for (int k = 0; k < 3; ++k) {
        da_var(c, t, k, cen[k] - x[k]);
        da_mul(c, t, t, t);
        for (int i = 0; i < c->n; ++i) s[i] += t[i];
    }
    da_sqrt(c, s, t);
    da_inv(c, t, u);
    for (int i = 0; i < c->n; ++i) L[i] += q * u[i];
    free(s); free(t); free(u);
}

int oracle_p2l(int p, int64_t n, const double *xyz, const double *q, const double cen[3],
               double *L)
{
    da_ctx c;
    if (da_ctx_init(&c, p)) return -1;
    da_zero(&c, L);
    for (int64_t i = 0; i < n; ++i) p2l_add(&c, cen, xyz + 3 * i, q[i], L);
    da_ctx_free(&c);
    return 0;
}

/* ---- L2P and M2P (Sec. 3.2) ----
 * Both evaluate a DA vector at the target.  To get E = -grad(phi) as well, the
 * evaluation runs in an order-1 DA of the target offset (y + delta). */
static void l2p_one(const da_ctx *c, const da_ctx *c1, const double *L, const double y[3],
                    double *phi, double *grad)
{
    double a0[4], a1[4], a2[4], r[4];
    da_var(c1, a0, 0, y[0]); da_var(c1, a1, 1, y[1]); da_var(c1, a2, 2, y[2]);
    const double *args[3] = {a0, a1, a2};
    da_compose(c, L, c1, args, r);
    *phi = r[0];
    grad[0] = r[1]; grad[1] = r[2]; grad[2] = r[3];
}

/* M2P: d = y / |y|^2, phi = |d| phi_M(d) (Eq. P2M_phi); in the order-1 DA,
 * R = 1/(Y.Y), D = Y R and |d| = sqrt(R). */
static void m2p_one(const da_ctx *c, const da_ctx *c1, const double *M, const double y[3],
                    double *phi, double *grad)
{
    double Y[3][4], s[4] = {0, 0, 0, 0}, t[4], R[4], D[3][4], sR[4], r[4];
    for (int k = 0; k < 3; ++k) {
        da_var(c1, Y[k], k, y[k]);
        da_mul(c1, Y[k], Y[k], t);
        for (int i = 0; i < 4; ++i) s[i] += t[i];
    }
    da_inv(c1, s, R);
    for (int k = 0; k < 3; ++k) da_mul(c1, Y[k], R, D[k]);
    da_sqrt(c1, R, sR);
    const double *args[3] = {D[0], D[1], D[2]};
    da_compose(c, M, c1, args, r);
    da_mul(c1, r, sR, r);
    *phi = r[0];
    grad[0] = r[1]; grad[1] = r[2]; grad[2] = r[3];
}

int oracle_l2p(int p, const double cen[3], const double *L, int64_t n, const double *xyz,
               double *phi, double *field)
{
    da_ctx c, c1;
    if (da_ctx_init(&c, p) || da_ctx_init(&c1, 1)) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double y[3] = {xyz[3 * i] - cen[0], xyz[3 * i + 1] - cen[1], xyz[3 * i + 2] - cen[2]}, g[3];
        l2p_one(&c, &c1, L, y, &phi[i], g);
        if (field) for (int k = 0; k < 3; ++k) field[3 * i + k] = -g[k];
    }
    da_ctx_free(&c); da_ctx_free(&c1);
    return 0;
}

int oracle_m2p(int p, const double cen[3], const double *M, int64_t n, const double *xyz,
               double *phi, double *field)
{
    da_ctx c, c1;
    if (da_ctx_init(&c, p) || da_ctx_init(&c1, 1)) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double y[3] = {xyz[3 * i] - cen[0], xyz[3 * i + 1] - cen[1], xyz[3 * i + 2] - cen[2]}, g[3];
        m2p_one(&c, &c1, M, y, &phi[i], g);
        if (field) for (int k = 0; k < 3; ++k) field[3 * i + k] = -g[k];
    }
    da_ctx_free(&c); da_ctx_free(&c1);
    return 0;
}

/* ---- the FMM recipe (Sec. 1) ---- */
static int octant(const oracle_tree *t, int32_t b, int k)
{
    int64_t g[3];
    oracle_tree_coords(t, b, g);
    return (int)(g[k] & 1);
}

int oracle_fmm(const oracle_tree *t, int p, const double *xyz, const double *q, int memo,
               double *phi_out, double *field_out, double *M_out, double *L_out)
{
    da_ctx c, c1;
    if (da_ctx_init(&c, p) || da_ctx_init(&c1, 1)) return -1;
    const int n = c.n;
    const int64_t N = oracle_tree_n(t), nb = oracle_tree_nboxes(t);
    const int depth = oracle_tree_depth(t);
    const int64_t *perm = oracle_tree_perm(t), *first = oracle_tree_first(t),
                  *count = oracle_tree_count(t), *lbeg = oracle_tree_level_begin(t);
    const int32_t *level = oracle_tree_level(t), *parent = oracle_tree_parent(t),
                  *cbeg = oracle_tree_child_begin(t), *nch = oracle_tree_nchild(t);
    const int64_t *Uo = oracle_tree_off(t, 0), *Vo = oracle_tree_off(t, 1),
                  *Wo = oracle_tree_off(t, 2), *Xo = oracle_tree_off(t, 3);
    const int32_t *Us = oracle_tree_src(t, 0), *Vs = oracle_tree_src(t, 1),
                  *Ws = oracle_tree_src(t, 2), *Xs = oracle_tree_src(t, 3);

    double *xs = malloc(sizeof(double) * 3 * (size_t)N), *qs = malloc(sizeof(double) * (size_t)N);
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
            double y[3] = {xs[3 * i] - cen[3 * b], xs[3 * i + 1] - cen[3 * b + 1],
                           xs[3 * i + 2] - cen[3 * b + 2]};
            p2m_add(&c, y, qs[i], M + b * n);
        }
    }

    /* upward pass: M2M, finest level first */
    double *oct = memo ? malloc(sizeof(double) * 8 * (size_t)n * n) : NULL;
    for (int l = depth; l >= 1; --l) {
        double h = oracle_tree_width(t, l);
        if (memo) {
#pragma omp parallel for
            for (int o = 0; o < 8; ++o) {
                /* parent centre minus child centre: (1 - 2 o_k) h / 2 */
                double r0[3] = {(1 - 2 * ((o >> 2) & 1)) * 0.5 * h, (1 - 2 * ((o >> 1) & 1)) * 0.5 * h,
                                (1 - 2 * (o & 1)) * 0.5 * h};
                translation_matrix(&c, m2m_map, r0, oct + (size_t)o * n * n);
            }
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = lbeg[l - 1]; b < lbeg[l]; ++b) {
            for (int k = 0; k < nch[b]; ++k) {
                int32_t ch = cbeg[b] + k;
                if (memo) {
                    int o = (octant(t, ch, 0) << 2) | (octant(t, ch, 1) << 1) | octant(t, ch, 2);
                    apply_matrix(&c, oct + (size_t)o * n * n, M + (int64_t)ch * n, M + b * n);
                } else {
                    double r0[3] = {cen[3 * b] - cen[3 * ch], cen[3 * b + 1] - cen[3 * ch + 1],
                                    cen[3 * b + 2] - cen[3 * ch + 2]};
                    translate(&c, m2m_map, r0, M + (int64_t)ch * n, M + b * n);
                }
            }
        }
    }

    /* downward pass, level by level: M2L (V list) + P2L (X list), then L2L to
     * the children of this level */
    double *m2l = memo ? malloc(sizeof(double) * 343 * (size_t)n * n) : NULL;
    int have[343];
    for (int l = 2; l <= depth; ++l) {
        double h = oracle_tree_width(t, l);
        if (memo) {
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
                double r0[3] = {(k / 49 - 3) * h, ((k / 7) % 7 - 3) * h, (k % 7 - 3) * h};
                translation_matrix(&c, m2l_map, r0, m2l + (size_t)k * n * n);
            }
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = lbeg[l]; b < lbeg[l + 1]; ++b) {
            for (int64_t e = Vo[b]; e < Vo[b + 1]; ++e) {
                int32_t s = Vs[e];
                if (memo) {
                    int64_t gb[3], gs[3];
                    oracle_tree_coords(t, (int32_t)b, gb);
                    oracle_tree_coords(t, s, gs);
                    int k = (int)((gb[0] - gs[0] + 3) * 49 + (gb[1] - gs[1] + 3) * 7 + (gb[2] - gs[2] + 3));
                    apply_matrix(&c, m2l + (size_t)k * n * n, M + (int64_t)s * n, L + b * n);
                } else {
                    double r0[3] = {cen[3 * b] - cen[3 * s], cen[3 * b + 1] - cen[3 * s + 1],
                                    cen[3 * b + 2] - cen[3 * s + 2]};
                    translate(&c, m2l_map, r0, M + (int64_t)s * n, L + b * n);
                }
            }
            for (int64_t e = Xo[b]; e < Xo[b + 1]; ++e) {
                int32_t s = Xs[e];
                for (int64_t i = first[s]; i < first[s] + count[s]; ++i)
                    p2l_add(&c, cen + 3 * b, xs + 3 * i, qs[i], L + b * n);
            }
        }
        if (l == depth) break;
        double hc = oracle_tree_width(t, l + 1);
        if (memo) {
#pragma omp parallel for
            for (int o = 0; o < 8; ++o) {
                /* child centre minus parent centre: (2 o_k - 1) h_child / 2 */
                double r0[3] = {(2 * ((o >> 2) & 1) - 1) * 0.5 * hc, (2 * ((o >> 1) & 1) - 1) * 0.5 * hc,
                                (2 * (o & 1) - 1) * 0.5 * hc};
                translation_matrix(&c, l2l_map, r0, oct + (size_t)o * n * n);
            }
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t ch = lbeg[l + 1]; ch < lbeg[l + 2]; ++ch) {
            int32_t b = parent[ch];
            if (memo) {
                int o = (octant(t, (int32_t)ch, 0) << 2) | (octant(t, (int32_t)ch, 1) << 1) |
                        octant(t, (int32_t)ch, 2);
                apply_matrix(&c, oct + (size_t)o * n * n, L + (int64_t)b * n, L + ch * n);
            } else {
                double r0[3] = {cen[3 * ch] - cen[3 * b], cen[3 * ch + 1] - cen[3 * b + 1],
                                cen[3 * ch + 2] - cen[3 * b + 2]};
                translate(&c, l2l_map, r0, L + (int64_t)b * n, L + ch * n);
            }
        }
    }
    free(m2l); free(oct);

    /* evaluation at the leaves: L2P + M2P (W list) + P2P (U list) */
    double *phs = calloc((size_t)N, sizeof(double)), *fs = calloc(3 * (size_t)N, sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
        if (nch[b] != 0) continue;
        for (int64_t i = first[b]; i < first[b] + count[b]; ++i) {
            double ph = 0.0, g[3] = {0, 0, 0}, pv, gv[3];
            if (level[b] >= 2) {
                double y[3] = {xs[3 * i] - cen[3 * b], xs[3 * i + 1] - cen[3 * b + 1],
                               xs[3 * i + 2] - cen[3 * b + 2]};
                l2p_one(&c, &c1, L + b * n, y, &pv, gv);
                ph += pv; g[0] += gv[0]; g[1] += gv[1]; g[2] += gv[2];
            }
            for (int64_t e = Wo[b]; e < Wo[b + 1]; ++e) {
                int32_t s = Ws[e];
                double y[3] = {xs[3 * i] - cen[3 * s], xs[3 * i + 1] - cen[3 * s + 1],
                               xs[3 * i + 2] - cen[3 * s + 2]};
                m2p_one(&c, &c1, M + (int64_t)s * n, y, &pv, gv);
                ph += pv; g[0] += gv[0]; g[1] += gv[1]; g[2] += gv[2];
            }
            double ex = -g[0], ey = -g[1], ez = -g[2];
            for (int64_t e = Uo[b]; e < Uo[b + 1]; ++e) {
                int32_t s = Us[e];
                for (int64_t j = first[s]; j < first[s] + count[s]; ++j) {
                    if (j == i) continue;
                    double dx = xs[3 * i] - xs[3 * j], dy = xs[3 * i + 1] - xs[3 * j + 1],
                           dz = xs[3 * i + 2] - xs[3 * j + 2];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 == 0.0) continue;
                    double r = sqrt(r2);
                    ph += qs[j] / r;
                    double f = qs[j] / (r2 * r);
                    ex += f * dx; ey += f * dy; ez += f * dz;
                }
            }
            phs[i] = ph;
            fs[3 * i] = ex; fs[3 * i + 1] = ey; fs[3 * i + 2] = ez;
        }
    }
    for (int64_t i = 0; i < N; ++i) {
        if (phi_out) phi_out[perm[i]] = phs[i];
        if (field_out)
            for (int k = 0; k < 3; ++k) field_out[3 * perm[i] + k] = fs[3 * i + k];
    }
    if (M_out) memcpy(M_out, M, sizeof(double) * (size_t)(nb * n));
    if (L_out) memcpy(L_out, L, sizeof(double) * (size_t)(nb * n));
    free(phs); free(fs); free(xs); free(qs); free(M); free(L); free(cen);
    da_ctx_free(&c); da_ctx_free(&c1);
    return 0;
}
