// ot_coarse.h -- device side of the coarse substitute for missing neighbours
// (Sec. 2.1 names the octree FMM without formulas; this is a reading of the
// interaction across a refinement boundary): for a target whose fine
// neighbour in slot s is missing and is covered by octant o of a
// parent-level node P, each of the 4^3 coarse cells J of that octant stands
// in for its 2x2x2 fine children when all of them would be in the target
// cell's stencil. Included by ot_fmm.hip after ot_interact.h (uses its
// derivatives, trace-reduced contraction and staging scales).
#pragma once

#include "ot_interact.h"

namespace {

struct CoarseParams {
    const double* pos;      // fine centres [3][pos_stride] (targets)
    long pos_stride;
    const double* mom_c;    // coarse moments [20][c_stride]
    const double* pos_c;    // coarse centres [3][c_stride]
    long c_stride;
    const int4* items;      // work items {target, lane order, first entry, entries}, most work first
    const int4* entries;    // substituted slots {slot, coarse node P, octant o, 0}
    const int* lane_cell;   // [orders][512] target cell of each lane
    const unsigned long long* cell_mask;  // [27][512] bit J: coarse cell J included for cell c
    const int4* rel;        // forward relations (.z: packed periodic shift)
    const int* own_blk;     // target -> store block
    double* out;            // L [20][out_stride], accumulated
    long out_stride;
    double period[3];
};

// One target's 512 cells, ranked by their total number of included coarse
// cells for its pattern of substituted slots, form 8 blocks of 64 ranks. A
// work-group of NW wavefronts takes the blocks part, part + 8/NW, ... of one
// target (8/NW work items per target): smaller work-groups release their
// registers and LDS as soon as their own blocks are done.
template <int NW>
struct CoarseShape {
    static constexpr int parts = 8 / NW;
    static constexpr int batch = NW;  // substituted slots staged together (LDS: NW x 9.5 KiB)
};

// The coarse cells of up to `batch` substituted slots are staged in LDS at
// once, value-major (one row of 64 coarse cells per value; measured faster
// than a cell-major layout read with 16-byte loads). Each lane takes one
// ranked target cell, so that the lanes of a wavefront run loops of similar
// length, and walks, in one loop over the batch, the set bits of its cell's
// inclusion mask of each slot (every child j = 8 s + 2 J + {0,1}^3 of coarse
// cell J satisfies |j - i|^2 > 16, and the common parent criterion
// |J + 4 s - floor(i/2)|^2 <= 16 holds), with its accumulators in registers;
// the order of the sums is fixed (slots, then J ascending): deterministic.
// With 8 wavefronts (a whole target) the accumulators go through LDS at the
// end so that L is read and written in cell order; smaller work-groups add
// into their cells directly. FULL: the full truncation (every |b| <= 3 for
// every |a| <= 3, derivatives of G to order 6), with the same staged values
// and kept outputs as the total order; its derivatives need up to 256
// registers, so it runs at half the waves per SIMD.
template <int NW, bool FULL>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(FULL ? 2 : 4)))
k_coarse_fine(const CoarseParams p)
{
    using Sh = CoarseShape<NW>;
    constexpr int kNc = 3 + kNRed;                        // staged values per coarse cell
    constexpr int kNa = ModeTraits<MODE_FWD_STORE>::nacc;  // kept L_a of the reduced form (either truncation)
    static_assert(ModeTraits<MODE_FULL_STORE>::nacc == kNa, "both truncations keep the same outputs");
    constexpr int kSlotVals = kNc * 64;
    __shared__ double s_src[Sh::batch * kSlotVals];
    __shared__ int s_slot[Sh::batch];
    __shared__ int4 s_ent[Sh::batch];        // the batch's entries {slot, coarse node, octant, -}
    __shared__ double s_shift[Sh::batch][3];  // and the periodic shift of each slot
    static_assert(NW != 8 || kNa * kSub3 <= Sh::batch * kSlotVals, "epilogue reuses the staging buffer");
    const int tid = threadIdx.x;
    const int4 it = p.items[blockIdx.x];  // uniform
    const int t = it.x;
    const int order = it.y >> 3, part = it.y & 7;
    const int rank = 64 * (part + Sh::parts * (tid >> 6)) + (tid & 63);
    const int cell = p.lane_cell[(long)order * kSub3 + rank];
    const long own = (long)p.own_blk[t] * kSub3 + cell;
    const double xi = p.pos[own], yi = p.pos[p.pos_stride + own], zi = p.pos[2 * p.pos_stride + own];
    double acc[kNa];
#pragma unroll
    for (int a = 0; a < kNa; ++a) acc[a] = 0.0;

    for (int b0 = 0; b0 < it.w; b0 += Sh::batch) {
        const int nb = (it.w - b0 < Sh::batch) ? it.w - b0 : Sh::batch;
        const int4* ent = p.entries + it.z + b0;
        __syncthreads();  // the previous batch is no longer read
        if (tid < nb) {
            // the batch's entries and shifts, read once
            const int4 e = ent[tid];
            const int packed = p.rel[(long)t * 27 + e.x].z;
            s_ent[tid] = e;
            s_slot[tid] = e.x;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                s_shift[tid][k] = (double)(int)(int8_t)((packed >> (8 * k)) & 0xff) * p.period[k];
        }
        __syncthreads();
        // a thread's values four at a time (their loads in flight together;
        // no load depends on another)
        constexpr int kIter = (Sh::batch * kSlotVals + NW * 64 - 1) / (NW * 64);
#pragma unroll 4
        for (int i = 0; i < kIter; ++i) {
            const int v = tid + i * NW * 64;
            if (v < nb * kSlotVals) {
                const int b = v / kSlotVals, r = v - b * kSlotVals;
                const int k = r >> 6, J = r & 63;
                const int4 e = s_ent[b];
                const int o = e.z;
                const int cx = J & 3, cy = (J >> 2) & 3, cz = J >> 4;
                const int pc = (cx + 4 * (o & 1)) + 8 * (cy + 4 * ((o >> 1) & 1)) + 64 * (cz + 4 * (o >> 2));
                const long jj = (long)e.y * kSub3 + pc;
                double val;
                if (k < 3) {
                    val = p.pos_c[k * p.c_stride + jj] + s_shift[b][k];
                } else {
                    const int cP = c_red_src[k - 3][0], cS = c_red_src[k - 3][1];
                    val = c_scale_fwd[cP] * p.mom_c[cP * p.c_stride + jj];
                    if (cS >= 0) val -= c_scale_fwd[cS] * p.mom_c[cS * p.c_stride + jj];
                }
                s_src[v] = val;
            }
        }
        __syncthreads();
        // one loop over the lane's (slot, coarse cell) pairs of the batch, so
        // that a wavefront runs as many trips as its busiest lane has pairs;
        // the next slot's mask is loaded while the current one is worked on
        int b = 0;
        unsigned long long cur = p.cell_mask[s_slot[0] * kSub3 + cell];
        unsigned long long nxt = nb > 1 ? p.cell_mask[s_slot[1] * kSub3 + cell] : 0ull;
        for (;;) {
            while (cur == 0ull && b + 1 < nb) {
                ++b;
                cur = nxt;
                nxt = b + 1 < nb ? p.cell_mask[s_slot[b + 1] * kSub3 + cell] : 0ull;
            }
            if (cur == 0ull) break;
            const int J = __builtin_ctzll(cur);
            cur &= cur - 1;
            const double* src = s_src + b * kSlotVals + J;
            double f[kNc];
#pragma unroll
            for (int k = 0; k < kNc; ++k) f[k] = src[k * 64];
            if constexpr (FULL) {
                double D[7];
                const double rr[3] = {xi - f[0], yi - f[1], zi - f[2]};
                radial<6>(rr[0], rr[1], rr[2], D);
                contract_full<0>(acc, f + 3, rr, D, std::make_integer_sequence<int, 20>{});
            } else {
                double G[20];
                green<3>(xi - f[0], yi - f[1], zi - f[2], G);
                contract_red<0, TRUNC3>(acc, f + 3, G, std::make_integer_sequence<int, 20>{});
            }
        }
    }
    int oc = cell;
    if constexpr (NW == 8) {
        // back to cell order through LDS
        __syncthreads();
#pragma unroll
        for (int a = 0; a < kNa; ++a) s_src[a * kSub3 + cell] = acc[a];
        __syncthreads();
#pragma unroll
        for (int a = 0; a < kNa; ++a) acc[a] = s_src[a * kSub3 + tid];
        oc = tid;
    }
    double L[20];
    expand<0>(acc, L, std::make_integer_sequence<int, 20>{});
    const long ob = (long)t * kSub3 + oc;
#pragma unroll
    for (int a = 0; a < 20; ++a) p.out[a * p.out_stride + ob] += L[a];
}

}  // namespace
