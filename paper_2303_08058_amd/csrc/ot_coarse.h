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
    const int* list;        // work list: target index, most work first
    const int2* coarse;     // [T][27] {coarse node P, octant o}, P = -1: none
    const int4* rel;        // forward relations (.z: packed periodic shift)
    const int* own_blk;     // target -> store block
    const int* lane_cell;   // [27][512] target cell of each lane, per slot
    const unsigned long long* lane_mask;  // [27][512] bit J: coarse cell J included
    double* out;            // L [20][out_stride], accumulated
    long out_stride;
    double period[3];
};

// One work-group (8 wavefronts) per target with substitutes. For each
// substituted slot the 64 coarse cells of the octant are staged in LDS; lane
// l then takes target cell lane_cell[slot][l] -- per slot the cells are
// ordered by their number of included coarse cells, so that the lanes of a
// wavefront run loops of similar length -- and walks the set bits of its
// inclusion mask (every child j = 8 s + 2 J + {0,1}^3 of J satisfies
// |j - i|^2 > 16 and the common parent criterion |J + 4 s - floor(i/2)|^2
// <= 16 holds). The partial sums of a slot are added to the cell's
// trace-reduced accumulators in LDS, one lane per cell and slot, slots in
// order: deterministic. The last phase expands them and adds L.
__global__ void __launch_bounds__(512) k_coarse_fine(const CoarseParams p)
{
    constexpr int kNc = 3 + kNRed;                        // staged values per coarse cell
    constexpr int kNa = ModeTraits<MODE_FWD_STORE>::nacc;  // kept L_a of the reduced form
    __shared__ double s_acc[kNa][kSub3];
    __shared__ double s_src[kNc][64];  // value-major: lanes gather distinct J
    const int tid = threadIdx.x;
    const int t = p.list[blockIdx.x];
    const long own0 = (long)p.own_blk[t] * kSub3;
#pragma unroll
    for (int a = 0; a < kNa; ++a) s_acc[a][tid] = 0.0;

    for (int slot = 0; slot < 27; ++slot) {
        const int2 cs = p.coarse[t * 27 + slot];  // uniform
        if (cs.x < 0) continue;
        const int o = cs.y;
        const int packed = p.rel[t * 27 + slot].z;
        __syncthreads();  // the previous slot's sources and accumulators are done
        for (int v = tid; v < 64 * kNc; v += 512) {
            const int k = v >> 6, J = v & 63;
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
            s_src[k][J] = val;
        }
        __syncthreads();
        unsigned long long mask = p.lane_mask[slot * kSub3 + tid];
        if (mask) {
            const int cell = p.lane_cell[slot * kSub3 + tid];
            const long own = own0 + cell;
            const double xi = p.pos[own], yi = p.pos[p.pos_stride + own], zi = p.pos[2 * p.pos_stride + own];
            double acc[kNa];
#pragma unroll
            for (int a = 0; a < kNa; ++a) acc[a] = 0.0;
            do {
                const int J = __builtin_ctzll(mask);
                mask &= mask - 1;
                double f[kNc];
#pragma unroll
                for (int k = 0; k < kNc; ++k) f[k] = s_src[k][J];
                double G[20];
                green<3>(xi - f[0], yi - f[1], zi - f[2], G);
                contract_red<0, TRUNC3>(acc, f + 3, G, std::make_integer_sequence<int, 20>{});
            } while (mask);
#pragma unroll
            for (int a = 0; a < kNa; ++a) s_acc[a][cell] += acc[a];
        }
    }
    __syncthreads();
    double acc[kNa];
#pragma unroll
    for (int a = 0; a < kNa; ++a) acc[a] = s_acc[a][tid];
    double L[20];
    expand<0>(acc, L, std::make_integer_sequence<int, 20>{});
    const long ob = (long)t * kSub3 + tid;
#pragma unroll
    for (int a = 0; a < 20; ++a) p.out[a * p.out_stride + ob] += L[a];
}

}  // namespace
