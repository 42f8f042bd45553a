// ot_coarse.h -- device side of the coarse substitute for missing neighbours
// (a reading of an FMM at a refinement boundary; the paper gives no FMM
// formulas): for a target whose fine neighbour in slot s is missing and is
// covered by octant o of a parent-level node P, each of the 4^3 coarse cells
// J of that octant stands in for its 2x2x2 fine children when all of them
// would be in the target cell's stencil. Included by ot_fmm.hip after
// ot_interact.h (uses its derivatives, trace-reduced contraction and staging
// scales).
#pragma once

#include "ot_interact.h"

namespace {

struct CoarseParams {
    const double* pos;      // fine centres [3][pos_stride] (targets)
    long pos_stride;
    const double* mom_c;    // coarse moments [20][c_stride]
    const double* pos_c;    // coarse centres [3][c_stride]
    long c_stride;
    const int* list;        // work list: target index, most substitute slots first
    const int2* coarse;     // [T][27] {coarse node P, octant o}, P = -1: none
    const int4* rel;        // forward relations (.z: packed periodic shift)
    const int* own_blk;     // target -> store block
    double* out;            // L [20][out_stride], accumulated
    long out_stride;
    double period[3];
};

// One work-group (8 wavefronts, lane = target cell x + 8 y of plane z =
// wavefront) per target with substitutes; the 64 coarse cells of each
// substitute slot are staged in LDS in turn. Inclusion is decided per lane
// from integer cell coordinates: every child j = 8 s + 2 J + {0,1}^3 of J
// must satisfy |j - i|^2 > 16, and the common parent criterion
// |J + 4 s - floor(i/2)|^2 <= 16 must hold.
__global__ void __launch_bounds__(512) k_coarse_fine(const CoarseParams p)
{
    constexpr int kNc = 3 + kNRed;  // staged values per coarse cell
    __shared__ double s_src[64][kNc + 1];
    const int tid = threadIdx.x;
    const int t = p.list[blockIdx.x];
    const int xt = tid & 7, yt = (tid >> 3) & 7, zt = tid >> 6;
    const int hi[3] = {8 + xt, 8 + yt, 8 + zt};
    const int pi[3] = {hi[0] >> 1, hi[1] >> 1, hi[2] >> 1};
    const long own = (long)p.own_blk[t] * kSub3 + tid;
    const double xi = p.pos[own], yi = p.pos[p.pos_stride + own], zi = p.pos[2 * p.pos_stride + own];
    double acc[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) acc[a] = 0.0;

    for (int slot = 0; slot < 27; ++slot) {
        const int2 cs = p.coarse[t * 27 + slot];  // uniform
        if (cs.x < 0) continue;
        const int o = cs.y;
        const int so[3] = {slot % 3, (slot / 3) % 3, slot / 9};
        const int packed = p.rel[t * 27 + slot].z;
        __syncthreads();  // the previous slot's sources are no longer read
        for (int v = tid; v < 64 * kNc; v += 512) {
            const int J = v / kNc, k = v - J * kNc;
            const int cx = J & 3, cy = (J >> 2) & 3, cz = J >> 4;
            const int pc = (cx + 4 * (o & 1)) + 8 * (cy + 4 * ((o >> 1) & 1)) + 64 * (cz + 4 * (o >> 2));
            const long jj = (long)cs.x * kSub3 + pc;
            double val;
            if (k < 3) {
                const double sh = (double)(int)(int8_t)((packed >> (8 * k)) & 0xff) * p.period[k];
                val = p.pos_c[k * p.c_stride + jj] + sh;
            } else {
                const int cP = c_red_src[k - 3][0], cS = c_red_src[k - 3][1];
                val = c_scale_fwd[cP] * p.mom_c[cP * p.c_stride + jj];
                if (cS >= 0) val -= c_scale_fwd[cS] * p.mom_c[cS * p.c_stride + jj];
            }
            s_src[J][k] = val;
        }
        __syncthreads();
        for (int J = 0; J < 64; ++J) {
            const int cj[3] = {J & 3, (J >> 2) & 3, J >> 4};
            // parent-level criterion, common to the 8 children
            int dp2 = 0, near2 = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int dpk = 4 * so[k] + cj[k] - pi[k];
                dp2 += dpk * dpk;
                // closest of the two child coordinates along axis k
                const int d0 = 8 * so[k] + 2 * cj[k] - hi[k], d1 = d0 + 1;
                const int m = (d0 <= 0 && d1 >= 0) ? 0 : ((d0 > 0) ? d0 : -d1);
                near2 += m * m;
            }
            if (dp2 > 16 || near2 <= 16) continue;  // not all 8 children are in S(i)
            double f[kNc];
#pragma unroll
            for (int k = 0; k < kNc; ++k) f[k] = s_src[J][k];
            double G[20];
            green<3>(xi - f[0], yi - f[1], zi - f[2], G);
            contract_red<0, TRUNC3>(acc, f + 3, G, std::make_integer_sequence<int, 20>{});
        }
    }
    double L[20];
    expand<0>(acc, L, std::make_integer_sequence<int, 20>{});
    const long ob = (long)t * kSub3 + tid;
#pragma unroll
    for (int a = 0; a < 20; ++a) p.out[a * p.out_stride + ob] += L[a];
}

}  // namespace
