/*
 * Truncated power series algebra nD_v with v = 3 variables (App. A).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * A DA vector of order p holds the Taylor coefficients of all monomials
 * d1^J1 d2^J2 d3^J3 with J1+J2+J3 <= p (Eq. poly).  The coefficients are
 * Taylor coefficients, i.e. the 1/J! factor is included, which is what the
 * printed values of Table 1 show.  Monomials are ordered by total degree and,
 * inside one degree, by descending exponent of d1, then of d2 (Table 1:
 * 000, 100, 010, 001, 200, 110, 101, 020, 011, 002).
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* number of monomials of total degree < n in three variables */
static int below(int n) { return n * (n + 1) * (n + 2) / 6; }

int da_index(int i, int j, int k)
{
    int n = i + j + k;
    int a = j + k; /* monomials of degree n with a larger d1 exponent come first */
    return below(n) + a * (a + 1) / 2 + k;
}

int da_ctx_init(da_ctx *c, int p)
{
    memset(c, 0, sizeof(*c));
    if (p < 0) return -1;
    c->p = p;
    c->n = below(p + 1);
    c->e = malloc(sizeof(int[3]) * (size_t)c->n);
    c->deg = malloc(sizeof(int) * (size_t)c->n);
    if (!c->e || !c->deg) return -1;
    for (int n = 0; n <= p; ++n)
        for (int i = n; i >= 0; --i)
            for (int j = n - i; j >= 0; --j) {
                int k = n - i - j;
                int id = da_index(i, j, k);
                c->e[id][0] = i; c->e[id][1] = j; c->e[id][2] = k;
                c->deg[id] = n;
            }
    /* product table of Eq. addmlt: keep only pairs whose product survives the
     * truncation at order p */
    int cnt = 0;
    for (int a = 0; a < c->n; ++a)
        for (int b = 0; b < c->n; ++b)
            if (c->deg[a] + c->deg[b] <= p) ++cnt;
    c->npairs = cnt;
    c->pa = malloc(sizeof(int) * (size_t)cnt);
    c->pb = malloc(sizeof(int) * (size_t)cnt);
    c->pc = malloc(sizeof(int) * (size_t)cnt);
    if (!c->pa || !c->pb || !c->pc) return -1;
    cnt = 0;
    for (int a = 0; a < c->n; ++a)
        for (int b = 0; b < c->n; ++b)
            if (c->deg[a] + c->deg[b] <= p) {
                c->pa[cnt] = a; c->pb[cnt] = b;
                c->pc[cnt] = da_index(c->e[a][0] + c->e[b][0], c->e[a][1] + c->e[b][1],
                                      c->e[a][2] + c->e[b][2]);
                ++cnt;
            }
    return 0;
}

void da_ctx_free(da_ctx *c)
{
    free(c->e); free(c->deg); free(c->pa); free(c->pb); free(c->pc);
    memset(c, 0, sizeof(*c));
}

void da_zero(const da_ctx *c, double *a) { memset(a, 0, sizeof(double) * (size_t)c->n); }

void da_copy(const da_ctx *c, const double *a, double *out)
{
    memmove(out, a, sizeof(double) * (size_t)c->n);
}

/* [a]*[b] truncated at order p (App. A, Eq. addmlt). out may alias a or b. */
void da_mul(const da_ctx *c, const double *a, const double *b, double *out)
{
    double *t = calloc((size_t)c->n, sizeof(double));
    for (int k = 0; k < c->npairs; ++k)
        t[c->pc[k]] += a[c->pa[k]] * b[c->pb[k]];
    memcpy(out, t, sizeof(double) * (size_t)c->n);
    free(t);
}

/* Split a = a0 (1 + abar) with abar infinitely small (no constant part). */
static void split(const da_ctx *c, const double *a, double *abar, double *a0)
{
    *a0 = a[0];
    for (int i = 0; i < c->n; ++i) abar[i] = a[i] / a[0];
    abar[0] = 0.0;
}

/* Inverse of a non-infinitely-small element (App. A; Sec. 3 "order-by-order").
 * 1/a = (1/a0) sum_{k=0..p} (-abar)^k.  Every multiplication by abar raises the
 * lowest order by one, so p steps of s <- 1 - abar*s fix the result to order p. */
void da_inv(const da_ctx *c, const double *a, double *out)
{
    double a0, *abar = malloc(sizeof(double) * (size_t)c->n);
    double *s = calloc((size_t)c->n, sizeof(double));
    split(c, a, abar, &a0);
    s[0] = 1.0;
    for (int k = 0; k < c->p; ++k) {
        da_mul(c, abar, s, s);
        for (int i = 0; i < c->n; ++i) s[i] = -s[i];
        s[0] += 1.0;
    }
    for (int i = 0; i < c->n; ++i) out[i] = s[i] / a0;
    free(abar); free(s);
}

/* Square root (App. A: roots of non-infinitely-small elements exist):
 * sqrt(a) = sqrt(a0) sum_{k=0..p} binom(1/2, k) abar^k, summed by Horner. */
void da_sqrt(const da_ctx *c, const double *a, double *out)
{
    double a0, *abar = malloc(sizeof(double) * (size_t)c->n);
    double *s = calloc((size_t)c->n, sizeof(double));
    double *coef = malloc(sizeof(double) * (size_t)(c->p + 1));
    split(c, a, abar, &a0);
    coef[0] = 1.0;
    for (int k = 1; k <= c->p; ++k) coef[k] = coef[k - 1] * (0.5 - (k - 1)) / k;
    s[0] = coef[c->p];
    for (int k = c->p - 1; k >= 0; --k) {
        da_mul(c, abar, s, s);
        s[0] += coef[k];
    }
    double r = sqrt(a0);
    for (int i = 0; i < c->n; ++i) out[i] = s[i] * r;
    free(abar); free(s); free(coef);
}

/* Derivation d/dx_v (App. A, Eq. dev): the result is meaningful to order p-1. */
void da_deriv(const da_ctx *c, const double *a, int v, double *out)
{
    double *t = calloc((size_t)c->n, sizeof(double));
    for (int id = 0; id < c->n; ++id) {
        int e[3] = {c->e[id][0], c->e[id][1], c->e[id][2]};
        if (e[v] == 0) continue;
        double f = e[v];
        e[v] -= 1;
        t[da_index(e[0], e[1], e[2])] += f * a[id];
    }
    memcpy(out, t, sizeof(double) * (size_t)c->n);
    free(t);
}

/* All monomials args^J, |J| <= outer->p, as DA vectors of the inner algebra:
 * cols[J * inner->n + m]. */
void da_monomials(const da_ctx *outer, const da_ctx *inner, const double *const args[3],
                  double *cols)
{
    int p = outer->p, ni = inner->n;
    double *pw = malloc(sizeof(double) * (size_t)(3 * (p + 1) * ni));
    for (int v = 0; v < 3; ++v) {
        double *base = pw + (size_t)v * (p + 1) * ni;
        da_zero(inner, base);
        base[0] = 1.0;
        for (int k = 1; k <= p; ++k)
            da_mul(inner, base + (size_t)(k - 1) * ni, args[v], base + (size_t)k * ni);
    }
    double *tij = malloc(sizeof(double) * (size_t)ni);
    for (int id = 0; id < outer->n; ++id) {
        const int *e = outer->e[id];
        da_mul(inner, pw + (size_t)(0 * (p + 1) + e[0]) * ni,
               pw + (size_t)(1 * (p + 1) + e[1]) * ni, tij);
        da_mul(inner, tij, pw + (size_t)(2 * (p + 1) + e[2]) * ni, cols + (size_t)id * ni);
    }
    free(tij); free(pw);
}

/* Composition f o (args): substitute three DA vectors of the inner algebra for
 * the variables of f (the DA "composition" used by Eq. m2m, m2l and l2l). */
void da_compose(const da_ctx *outer, const double *f, const da_ctx *inner,
                const double *const args[3], double *out)
{
    int ni = inner->n;
    double *cols = malloc(sizeof(double) * (size_t)outer->n * ni);
    da_monomials(outer, inner, args, cols);
    double *t = calloc((size_t)ni, sizeof(double));
    for (int id = 0; id < outer->n; ++id)
        for (int m = 0; m < ni; ++m) t[m] += f[id] * cols[(size_t)id * ni + m];
    memcpy(out, t, sizeof(double) * (size_t)ni);
    free(t); free(cols);
}

/* Table 1: f = 1/|x0 + d|.  Following Sec. 3, first v = sum_k (x0_k + d_k)^2,
 * then the square root, then the inverse. */
int oracle_da_inv_r(int p, const double x0[3], double *out)
{
    da_ctx c;
    if (da_ctx_init(&c, p)) return -1;
    double *v = calloc((size_t)c.n, sizeof(double));
    double *t = calloc((size_t)c.n, sizeof(double));
    for (int k = 0; k < 3; ++k) {
        da_zero(&c, t);
        t[0] = x0[k];
        if (p >= 1) t[da_index(k == 0, k == 1, k == 2)] = 1.0;
        da_mul(&c, t, t, t);
        for (int i = 0; i < c.n; ++i) v[i] += t[i];
    }
    da_sqrt(&c, v, t);
    da_inv(&c, t, out);
    free(v); free(t);
    da_ctx_free(&c);
    return 0;
}

/* Test entry points over the algebra.  op: 0 product a*b, 1 inverse of a,
 * 2 square root of a, 3/4/5 derivation of a in d1/d2/d3. */
int oracle_da_op(int op, int p, const double *a, const double *b, double *out)
{
    da_ctx c;
    if (da_ctx_init(&c, p)) return -1;
    int rc = 0;
    switch (op) {
    case 0: da_mul(&c, a, b, out); break;
    case 1: da_inv(&c, a, out); break;
    case 2: da_sqrt(&c, a, out); break;
    case 3: case 4: case 5: da_deriv(&c, a, op - 3, out); break;
    default: rc = -1;
    }
    da_ctx_free(&c);
    return rc;
}

/* f (order p) composed with three order-q DA vectors args[3*nq]. */
int oracle_da_compose(int p, const double *f, int q, const double *args, double *out)
{
    da_ctx co, ci;
    if (da_ctx_init(&co, p) || da_ctx_init(&ci, q)) return -1;
    const double *a[3] = {args, args + ci.n, args + 2 * ci.n};
    da_compose(&co, f, &ci, a, out);
    da_ctx_free(&co); da_ctx_free(&ci);
    return 0;
}
