// Softened Coulomb kernel 1/sqrt(|x|^2 + eps^2) (soft.hip).
#pragma once
#include "common.h"

namespace fmm {
// M2L launch over nblocks target tiles (one block per tile; the sign-class
// kernel runs two per tile).  Adaptive trees: the plan's M2L target tiles.
// Uniform trees, levels 2..depth: level 2 + i has tiles[i] tiles of 64 boxes
// per octant, its tiles start at start[i], its first box is lvl_first[i].
constexpr int kSoftMaxLevels = 8;
struct SoftGrid {
    int nblocks, nlev, adaptive;
    int start[kSoftMaxLevels], tiles[kSoftMaxLevels], lvl_first[kSoftMaxLevels];
};
constexpr int kSoftMaxOrder = 10; // the double-buffered table (2p SA + 2 doubles) fills the LDS at p = 10
int soft_table_ldc(int p);        // doubles per (level, offset) table
void launch_soft_tables(int p, int nlev, double *D, int *map, double W, double eps, hipStream_t s);
void launch_soft_p2m(int p, const PlanView *V, int nleaves, int ldm, hipStream_t s);
void launch_soft_m2m(int p, const PlanView *V, int first_box, int nbox, hipStream_t s);
void launch_soft_l2l(int p, const PlanView *V, int first_child, int nchild, hipStream_t s);
// orders kSoftSymOrder .. kSoftSymMaxOrder: sign-class M2L over the moments
// copied into the class order (Ms: (nboxes + 1) rows of soft_sym_ld(p)
// doubles); other orders one contraction per offset (the sign-class kernel's
// unrolled k-steps exceed the unroller's limit beyond order 8)
constexpr int kSoftSymOrder = 4, kSoftSymMaxOrder = 8;
int soft_sym_ld(int p);
void launch_m2l_soft(int p, const PlanView *V, const SoftGrid &G, double *Ms, int nboxes, hipStream_t s);
void launch_soft_p2l(int p, const PlanView *V, int nxtgt, hipStream_t s);   // 1 X target/block
void launch_soft_m2p(int p, const PlanView *V, int nleaves, hipStream_t s); // 1 leaf/block (W lists)
} // namespace fmm
