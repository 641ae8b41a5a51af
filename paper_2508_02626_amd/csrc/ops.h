// Launchers of the evaluation kernels (see ops.hip and m2l.hip).  Every
// launcher takes the device array of plan views and the block split.
#pragma once
#include <string>
#include "common.h"

namespace fmm {
void launch_permute_q(const PlanView *V, const Bases &B, hipStream_t s);   // 256 particles/block
void launch_p2m(int p, const PlanView *V, const Bases &B, hipStream_t s);  // 1 leaf/block
void launch_p2m_fold(int p, const PlanView *V, const Bases &B, hipStream_t s); // 64 leaves/block
void launch_l2lh(int p, const PlanView *V, const Bases &B, int level, hipStream_t s); // 16 parents x 16 rows/block (harmonic rows)
void launch_lh_init(const PlanView *V, const Bases &B, hipStream_t s);        // 4 boxes/block
void launch_lh_zero(const PlanView *V, const Bases &B, hipStream_t s);        // 512 doubles/block
void launch_m2mh(int p, const PlanView *V, const Bases &B, int level, hipStream_t s); // 16 parents/block
// Row-tile groups per 16-parent M2M group: levels with few parents spread the
// mt row tiles of each group over up to mt blocks (powers of two dividing mt)
// until the level has about 512 blocks.
__host__ __device__ inline int m2m_row_split(int mt, int groups)
{
    int r = 1;
    while (2 * r <= mt && mt % (2 * r) == 0 && groups * r < 512) r *= 2;
    return r;
}
void launch_parent_mh(const PlanView *V, const Bases &B, int full, hipStream_t s); // 4 boxes/block
void launch_unfold(int p, const PlanView *V, const Bases &B, int leaves_only, hipStream_t s); // kRemapBoxes boxes/block
void launch_p2l(int p, const PlanView *V, const Bases &B, hipStream_t s);  // 1 X target/block
void launch_p2l_transform(const PlanView *V, const Bases &B, hipStream_t s); // 16 X targets x 16 rows/block
void launch_far(int p, const PlanView *V, const Bases &B, hipStream_t s);  // 2 leaves/block (L2P + output)
void launch_m2p(int p, const PlanView *V, const Bases &B, hipStream_t s);  // 1 leaf/block (W lists)
// P2P runs in two parts (leaves [0, split) and [split, nleaves)), each
// overlapping a latency-bound phase of the far field
__host__ __device__ inline int p2p_split(int nleaves) { return (int)((int64_t)nleaves * 5 / 8) & ~3; }
// mixed: 0 FP64, 1 FP32 terms, 2 softened kernel (FP64)
void launch_p2p(int mixed, int part, const PlanView *V, const Bases &B, hipStream_t s); // 4 leaves/block
void launch_zero(double *p, int64_t n, hipStream_t s);
void launch_zero_f32(float *p, int64_t n, hipStream_t s);
void launch_m2l(int p, int f32, const PlanView *V, const Bases &B, hipStream_t s); // 64 slots/block
constexpr int kM2LSlots = 64;
// rotation-based M2L (rotation.hip): device factors of order p (built on
// first use, kept for the process), blocks per 64-target tile, launcher
const RotTables *get_rotation_tables(int p, std::string &err);
int m2l_rot_blocks_per_tile(int p);
void launch_m2l_rot(int p, const PlanView *V, const Bases &B, hipStream_t s);
constexpr int kRemapBoxes = 16; // boxes per block of the unfold
} // namespace fmm
