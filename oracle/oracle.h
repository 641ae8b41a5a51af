/*
 * CPU oracle for the differential-algebra (DA / TPSA) fast multipole method
 * for the 3-D Coulomb potential (Zhang, "Boosting the Efficiency of the
 * Differential Algebra-based Fast Multipole Method Using Symbolic Differential
 * Algebra", arXiv 2508.02626).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, FP64 reference
 * that the GPU path is checked against.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product path never
 * calls it and shares no code, header, table or helper with it.
 *
 * Pieces (each function cites the passage it follows):
 *   - a truncated power series algebra in three variables (App. A, Eq. addmlt,
 *     Eq. dev, Eq. poly; inverse and roots by the order-by-order fixed point of
 *     Sec. 3 / App. A), with composition (Sec. 1-2);
 *   - the seven DA-FMM operators exactly as written in Sec. 2.1-2.5
 *     (Eq. P2M_phi, P2M, m2m_phi, m2m, m2l, P2L, l2l), built from that algebra;
 *   - the O(N^2) direct sum of Eq. P2M_phi (left-hand side);
 *   - a reference octree and Carrier-Greengard-Rokhlin interaction lists
 *     (uniform full tree or adaptive tree with leaf size s, Sec. 1 and 3.5);
 *   - the FMM driver of Sec. 1 (upward pass, M2L/P2L, downward pass, L2P,
 *     M2P, P2P);
 *   - the same driver for a second non-oscillatory kernel, the softened
 *     Coulomb potential (soft.c).
 *
 * Readings of passages that are garbled or silent are listed in the design
 * notes; the ones that change arithmetic are restated at the function.
 */
#ifndef FMM_ORACLE_H
#define FMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- truncated power series algebra (App. A) ---------------- */

typedef struct {
    int p;          /* truncation order n of nD_v in App. A */
    int n;          /* number of coefficients, (p+1)(p+2)(p+3)/6 */
    int (*e)[3];    /* exponents (J1,J2,J3) of each basis monomial, Eq. poly */
    int *deg;       /* total degree of each monomial */
    int npairs;     /* number of (a,b) with deg a + deg b <= p */
    int *pa, *pb, *pc; /* product table: monomial pa*pb = monomial pc */
} da_ctx;

int  da_ctx_init(da_ctx *c, int p);
void da_ctx_free(da_ctx *c);
int  da_index(int i, int j, int k);            /* position of x^i y^j z^k */
void da_zero(const da_ctx *c, double *a);
void da_copy(const da_ctx *c, const double *a, double *out);
void da_mul(const da_ctx *c, const double *a, const double *b, double *out);
void da_inv(const da_ctx *c, const double *a, double *out);
void da_sqrt(const da_ctx *c, const double *a, double *out);
void da_deriv(const da_ctx *c, const double *a, int v, double *out);
void da_monomials(const da_ctx *outer, const da_ctx *inner, const double *const args[3],
                  double *cols);
void da_compose(const da_ctx *outer, const double *f,
                const da_ctx *inner, const double *const args[3], double *out);

/* Taylor coefficients of 1/|x0 + d| about x0 (Table 1): built with the DA
 * algebra exactly as Sec. 3 describes (v, then square root, then inverse). */
int oracle_da_inv_r(int p, const double x0[3], double *out);
int oracle_da_op(int op, int p, const double *a, const double *b, double *out);
int oracle_da_compose(int p, const double *f, int q, const double *args, double *out);

/* ---------------- single operators (Sec. 2) ---------------- */
int oracle_p2m(int p, int64_t n, const double *xyz, const double *q,
               const double center[3], double *M);
int oracle_m2m(int p, const double child_center[3], const double parent_center[3],
               const double *M, double *Mout);
int oracle_m2l(int p, const double src_center[3], const double tgt_center[3],
               const double *M, double *L);
int oracle_p2l(int p, int64_t n, const double *xyz, const double *q,
               const double center[3], double *L);
int oracle_l2l(int p, const double parent_center[3], const double child_center[3],
               const double *L, double *Lout);
int oracle_l2p(int p, const double center[3], const double *L, int64_t n,
               const double *xyz, double *phi, double *field);
int oracle_m2p(int p, const double center[3], const double *M, int64_t n,
               const double *xyz, double *phi, double *field);

/* ---------------- direct sum ---------------- */
/* phi_i = sum_{j != i, r_ij > 0} q_j / r_ij and E_i = sum q_j (x_i-x_j)/r_ij^3
 * for the listed targets (all if targets == NULL; then nt must equal n). */
int oracle_direct(int64_t n, const double *xyz, const double *q,
                  int64_t nt, const int64_t *targets, double *phi, double *field);

/* ---------------- reference tree and lists ---------------- */
typedef struct oracle_tree oracle_tree;

/* root: NULL for the bounding cube, else {lo_x, lo_y, lo_z, W}.
 * uniform_depth >= 0: full tree of that depth (leaf_size ignored);
 * uniform_depth < 0: adaptive, split iff count > leaf_size and level < max_depth. */
oracle_tree *oracle_tree_build(int64_t n, const double *xyz, const double *root,
                               int uniform_depth, int max_depth, int leaf_size);
void oracle_tree_free(oracle_tree *t);
/* sizes[0]=nboxes sizes[1]=nU sizes[2]=nV sizes[3]=nW sizes[4]=nX
 * sizes[5]=depth (deepest level) sizes[6]=key depth D */
void oracle_tree_sizes(const oracle_tree *t, int64_t sizes[7]);
void oracle_tree_root(const oracle_tree *t, double root[4]);
/* Any pointer may be NULL.  perm[n]: sorted position -> original index.
 * Per box: level, morton, first, count, parent, child_begin, nchild.
 * Lists as CSR over boxes: X_off[nboxes+1], X_src[nX]. */
void oracle_tree_export(const oracle_tree *t, int64_t *perm, int32_t *level,
                        uint64_t *morton, int64_t *first, int64_t *count,
                        int32_t *parent, int32_t *child_begin, int32_t *nchild,
                        int64_t *U_off, int32_t *U_src, int64_t *V_off, int32_t *V_src,
                        int64_t *W_off, int32_t *W_src, int64_t *X_off, int32_t *X_src);

/* ---------------- the DA-FMM (Sec. 1 recipe, Sec. 2 operators) ---------------- */
/* memo != 0: the translation operators, which are linear in the expansion,
 * are tabulated once per (level, offset) as the DA images of the basis
 * monomials and applied as such; memo == 0 recomputes every translation by
 * full DA composition.  field may be NULL.  Optional outputs M, L
 * (nboxes * n coefficients, box order of the tree) may be NULL. */
int oracle_fmm(const oracle_tree *t, int p, const double *xyz, const double *q,
               int memo, double *phi, double *field, double *M, double *L);

/* ---------------- the softened Coulomb kernel (soft.c) ---------------- */
/* K(x) = 1/sqrt(|x|^2 + eps^2): the same recipe with Cartesian Taylor
 * expansions (multipole moments, local Taylor coefficients in physical
 * units) and the kernel's Taylor coefficients from the DA algebra. */
int oracle_soft_taylor(int p, const double x0[3], double eps, double *out);
int oracle_direct_soft(int64_t n, const double *xyz, const double *q, double eps, int64_t nt,
                       const int64_t *targets, double *phi, double *field);
/* op 0: M2M (a3 child centre, b3 parent centre); 1: M2L (a3 source centre,
 * b3 target centre); 2: L2L (a3 parent centre, b3 child centre) */
int oracle_soft_op(int op, int p, double eps, const double *a3, const double *b3, const double *in,
                   double *out);
int oracle_soft_p2m(int p, int64_t n, const double *xyz, const double *q, const double center[3],
                    double *M);
int oracle_soft_p2l(int p, double eps, int64_t n, const double *xyz, const double *q,
                    const double center[3], double *L);
int oracle_fmm_soft(const oracle_tree *t, int p, double eps, const double *xyz, const double *q,
                    double *phi, double *field, double *M, double *L);

/* thread count used by OpenMP regions */
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
