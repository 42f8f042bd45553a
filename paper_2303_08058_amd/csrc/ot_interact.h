// ot_interact.h -- device side of the interaction kernels: sub-grid geometry,
// the compile-time stencil table, per-pair arithmetic, LDS staging and the
// k_interact kernel template. Included once, by ot_fmm.hip (host side and
// C ABI). The design notes are at the top of ot_fmm.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "ot_common.h"
#include "ot_fmm.h"

using namespace otfmm;

namespace {

// Staging scale of the source components: forward sources carry
// s_beta = (-1)^{|beta|}/beta!, adjoint sources carry (-1)^{|alpha|}.
__constant__ double c_scale_fwd[20] = {
    parity_sign(0) * inv_multi_factorial(0),   parity_sign(1) * inv_multi_factorial(1),
    parity_sign(2) * inv_multi_factorial(2),   parity_sign(3) * inv_multi_factorial(3),
    parity_sign(4) * inv_multi_factorial(4),   parity_sign(5) * inv_multi_factorial(5),
    parity_sign(6) * inv_multi_factorial(6),   parity_sign(7) * inv_multi_factorial(7),
    parity_sign(8) * inv_multi_factorial(8),   parity_sign(9) * inv_multi_factorial(9),
    parity_sign(10) * inv_multi_factorial(10), parity_sign(11) * inv_multi_factorial(11),
    parity_sign(12) * inv_multi_factorial(12), parity_sign(13) * inv_multi_factorial(13),
    parity_sign(14) * inv_multi_factorial(14), parity_sign(15) * inv_multi_factorial(15),
    parity_sign(16) * inv_multi_factorial(16), parity_sign(17) * inv_multi_factorial(17),
    parity_sign(18) * inv_multi_factorial(18), parity_sign(19) * inv_multi_factorial(19)};
__constant__ double c_scale_rev[20] = {
    parity_sign(0),  parity_sign(1),  parity_sign(2),  parity_sign(3),  parity_sign(4),
    parity_sign(5),  parity_sign(6),  parity_sign(7),  parity_sign(8),  parity_sign(9),
    parity_sign(10), parity_sign(11), parity_sign(12), parity_sign(13), parity_sign(14),
    parity_sign(15), parity_sign(16), parity_sign(17), parity_sign(18), parity_sign(19)};

// ---------------------------------------------------------------------------
// Stencil: for target parity (0, 0, pz), the offsets d = j - i grouped into
// rows (dz, dy, [dx0, dx0 + n)). Built at compile time from the criterion.
// Targets of x (y) parity 1 use the same rows with dx (dy) negated.
// ---------------------------------------------------------------------------
constexpr int floor_half(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }

constexpr bool criterion(int ix, int iy, int iz, int jx, int jy, int jz)
{
    const int dx = jx - ix, dy = jy - iy, dz = jz - iz;
    const int px = floor_half(jx) - floor_half(ix), py = floor_half(jy) - floor_half(iy),
              pz = floor_half(jz) - floor_half(iz);
    return dx * dx + dy * dy + dz * dz > 16 && px * px + py * py + pz * pz <= 16;
}

struct StencilTable {
    uint32_t rows[2][kMaxRows];           // packed: dy | dx0 << 8 | n << 16
    int range[2][2 * kReach + 1][3];      // per (pz, dz+9): first row, split row, end row
    int count[2];                         // offsets per parity (1799)
};

constexpr uint32_t pack_row(int dy, int dx0, int n)
{
    return (uint32_t)(dy & 0xff) | ((uint32_t)(dx0 & 0xff) << 8) | ((uint32_t)n << 16);
}

constexpr StencilTable build_stencil()
{
    StencilTable t{};
    for (int pz = 0; pz < 2; ++pz) {
        const int ix = 8, iy = 8, iz = 8 + pz;
        int nr = 0, total = 0;
        for (int dz = -kReach; dz <= kReach; ++dz) {
            const int first = nr;
            int offs = 0;
            for (int dy = -kReach; dy <= kReach; ++dy) {
                int dx = -kReach;
                while (dx <= kReach) {
                    if (!criterion(ix, iy, iz, ix + dx, iy + dy, iz + dz)) {
                        ++dx;
                        continue;
                    }
                    int n = 0;
                    while (dx + n <= kReach && criterion(ix, iy, iz, ix + dx + n, iy + dy, iz + dz))
                        ++n;
                    t.rows[pz][nr++] = pack_row(dy, dx, n);
                    offs += n;
                    dx += n;
                }
            }
            // split point: first row at which the running count reaches half
            int split = first, run = 0;
            while (split < nr && 2 * run < offs) {
                run += (int)(t.rows[pz][split] >> 16);
                ++split;
            }
            if (split > first && 2 * run - offs > offs - 2 * (run - (int)(t.rows[pz][split - 1] >> 16)))
                --split;
            t.range[pz][dz + kReach][0] = first;
            t.range[pz][dz + kReach][1] = split;
            t.range[pz][dz + kReach][2] = nr;
            total += offs;
        }
        t.count[pz] = total;
    }
    return t;
}

constexpr StencilTable kStencilHost = build_stencil();
static_assert(kStencilHost.count[0] == 1799 && kStencilHost.count[1] == 1799, "stencil size");
__constant__ StencilTable c_stencil = build_stencil();

// Exact number of pairs between the 8^3 target cells and the neighbour block
// at each slot, plus a check that the mirrored table reproduces the stencil
// of every parity. Computed once on the host.
struct SlotCounts {
    int64_t pairs[27];
    bool mirror_ok;
};

SlotCounts compute_slot_counts()
{
    SlotCounts sc{};
    for (int slot = 0; slot < 27; ++slot) {
        const int ox = 8 * (slot % 3), oy = 8 * ((slot / 3) % 3), oz = 8 * (slot / 9);
        int64_t n = 0;
        for (int i = 0; i < kSub3; ++i) {
            const int ix = 8 + i % 8, iy = 8 + (i / 8) % 8, iz = 8 + i / 64;
            for (int j = 0; j < kSub3; ++j)
                n += criterion(ix, iy, iz, ox + j % 8, oy + (j / 8) % 8, oz + j / 64);
        }
        sc.pairs[slot] = n;
    }
    // every parity's brute-force stencil == mirrored rows of its z-parity
    bool ok = true;
    for (int p = 0; p < 8 && ok; ++p) {
        const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
        const int ix = 8 + px, iy = 8 + py, iz = 8 + pz;
        static bool mark[19][19][19];
        std::memset(mark, 0, sizeof(mark));
        int n_table = 0;
        for (int dz = -kReach; dz <= kReach; ++dz) {
            const int* rg = kStencilHost.range[pz][dz + kReach];
            for (int r = rg[0]; r < rg[2]; ++r) {
                const uint32_t w = kStencilHost.rows[pz][r];
                const int dy = (int8_t)(w & 0xff), dx0 = (int8_t)((w >> 8) & 0xff), n = (int)(w >> 16);
                for (int k = 0; k < n; ++k) {
                    const int dx = (px ? -1 : 1) * (dx0 + k), dyy = (py ? -1 : 1) * dy;
                    if (!criterion(ix, iy, iz, ix + dx, iy + dyy, iz + dz)) ok = false;
                    mark[dz + 9][dyy + 9][dx + 9] = true;
                    ++n_table;
                }
            }
        }
        int n_brute = 0;
        for (int dz = -kReach; dz <= kReach; ++dz)
            for (int dy = -kReach; dy <= kReach; ++dy)
                for (int dx = -kReach; dx <= kReach; ++dx)
                    if (criterion(ix, iy, iz, ix + dx, iy + dy, iz + dz)) {
                        ++n_brute;
                        if (!mark[dz + 9][dy + 9][dx + 9]) ok = false;
                    }
        if (n_brute != n_table) ok = false;
    }
    sc.mirror_ok = ok;
    return sc;
}

const SlotCounts& slot_counts()
{
    static const SlotCounts sc = compute_slot_counts();
    return sc;
}

// ---------------------------------------------------------------------------
// Per-pair arithmetic
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_fp64(double a)
{
    // hardware estimate, then y (1 + e/2 + 3e^2/8) with e = 1 - a y^2
    double y = __builtin_amdgcn_rsq(a);
    const double e = __builtin_fma(-a * y, y, 1.0);
    y = __builtin_fma(y * e, __builtin_fma(0.375, e, 0.5), y);
    return y;
}

// G_gamma(r), |gamma| <= ORD (3 or 4), graded-lex order, from the radial
// factors D0 = -1/r, D1 = 1/r^3, D2 = -3/r^5, D3 = 15/r^7, D4 = -105/r^9:
//   G_a = r_a D1, G_ab = r_a r_b D2 + d_ab D1,
//   G_abc = r_a r_b r_c D3 + (d_ab r_c + d_ac r_b + d_bc r_a) D2,
//   G_abcd = r_a r_b r_c r_d D4 + (sum of 6 d r r) D3 + (sum of 3 d d) D2.
template <int ORD>
__device__ __forceinline__ void green(double x, double y, double z, double* G)
{
    const double r2 = __builtin_fma(x, x, __builtin_fma(y, y, z * z));
    const double ri = rsqrt_fp64(r2);
    const double ri2 = ri * ri;
    const double D1 = ri * ri2;
    const double D2 = -3.0 * D1 * ri2;
    const double D3 = -5.0 * D2 * ri2;
    G[0] = -ri;
    G[1] = x * D1;
    G[2] = y * D1;
    G[3] = z * D1;
    const double xD2 = x * D2, yD2 = y * D2, zD2 = z * D2;
    G[4] = __builtin_fma(x, xD2, D1);
    G[5] = x * yD2;
    G[6] = x * zD2;
    G[7] = __builtin_fma(y, yD2, D1);
    G[8] = y * zD2;
    const double xD3 = x * D3, yD3 = y * D3, zD3 = z * D3;
    const double xx3 = x * xD3, xy3 = x * yD3, xz3 = x * zD3;
    const double yy3 = y * yD3, yz3 = y * zD3;
    G[10] = __builtin_fma(x, xx3, 3.0 * xD2);  // xxx
    G[11] = __builtin_fma(y, xx3, yD2);        // xxy
    G[12] = __builtin_fma(z, xx3, zD2);        // xxz
    G[13] = __builtin_fma(x, yy3, xD2);        // xyy
    G[14] = z * xy3;                           // xyz
    G[16] = __builtin_fma(y, yy3, 3.0 * yD2);  // yyy
    G[17] = __builtin_fma(z, yy3, zD2);        // yyz
    // components with z^2 from the trace (Laplace: G_{g+xx} + G_{g+yy} + G_{g+zz} = 0)
    G[9] = -(G[4] + G[7]);     // zz
    G[15] = -(G[10] + G[13]);  // xzz
    G[18] = -(G[11] + G[16]);  // yzz
    G[19] = -(G[12] + G[17]);  // zzz
    if constexpr (ORD >= 4) {
        const double D4 = -7.0 * D3 * ri2;
        const double xD4 = x * D4, yD4 = y * D4;
        const double xx4 = x * xD4, yy4 = y * yD4;
        G[20] = __builtin_fma(x * x, xx4, __builtin_fma(6.0, xx3, 3.0 * D2));  // xxxx
        G[21] = __builtin_fma(x * y, xx4, 3.0 * xy3);                         // xxxy
        G[22] = __builtin_fma(x * z, xx4, 3.0 * xz3);                         // xxxz
        G[23] = __builtin_fma(y * y, xx4, __builtin_fma(1.0, xx3 + yy3, D2)); // xxyy
        G[24] = __builtin_fma(y * z, xx4, yz3);                               // xxyz
        G[26] = __builtin_fma(x * y, yy4, 3.0 * xy3);                         // xyyy
        G[27] = __builtin_fma(x * z, yy4, xz3);                               // xyyz
        G[30] = __builtin_fma(y * y, yy4, __builtin_fma(6.0, yy3, 3.0 * D2)); // yyyy
        G[31] = __builtin_fma(y * z, yy4, 3.0 * yz3);                         // yyyz
        G[25] = -(G[20] + G[23]);  // xxzz
        G[28] = -(G[21] + G[26]);  // xyzz
        G[29] = -(G[22] + G[27]);  // xzzz
        G[32] = -(G[23] + G[30]);  // yyzz
        G[33] = -(G[24] + G[31]);  // yzzz
        G[34] = -(G[25] + G[32]);  // zzzz
    }
}

// ---------------------------------------------------------------------------
// Trace-reduced contractions. Every derivative of 1/r of order >= 2 is
// trace-free (Laplace's equation): G_{g+xx} + G_{g+yy} + G_{g+zz} = 0. So
//  * source side: a complete order-2 or order-3 shell of source components
//    contracts through 16 combinations instead of 20 -- q_xx - q_zz and
//    q_yy - q_zz (paired with G_{.+xx}, G_{.+yy}); q_xxx - q_xzz,
//    q_xyy - q_xzz, q_xxy - q_yzz, q_yyy - q_yzz, q_xxz - q_zzz,
//    q_yyz - q_zzz and q_xyz for order 3;
//  * output side: within a group of outputs of one order and one truncation,
//    every output whose z exponent is >= 2 follows from two others,
//    L_{g+zz} = -(L_{g+xx} + L_{g+yy}), and is rebuilt after the sum.
// The results equal the plain contraction up to rounding.
// ---------------------------------------------------------------------------
constexpr int kNRed = 16;
// reduced component b = q[kRedP[b]] - q[kRedS[b]] (kRedS = -1: q[kRedP[b]]);
// it pairs with G_{g + kRedP[b]}
constexpr int kRedP[kNRed] = {0, 1, 2, 3, 4, 7, 5, 6, 8, 10, 13, 11, 16, 12, 17, 14};
constexpr int kRedS[kNRed] = {-1, -1, -1, -1, 9, 9, -1, -1, -1, 15, 15, 18, 18, 19, 19, -1};
__constant__ int c_red_src[kNRed][2] = {
    {kRedP[0], kRedS[0]},   {kRedP[1], kRedS[1]},   {kRedP[2], kRedS[2]},   {kRedP[3], kRedS[3]},
    {kRedP[4], kRedS[4]},   {kRedP[5], kRedS[5]},   {kRedP[6], kRedS[6]},   {kRedP[7], kRedS[7]},
    {kRedP[8], kRedS[8]},   {kRedP[9], kRedS[9]},   {kRedP[10], kRedS[10]}, {kRedP[11], kRedS[11]},
    {kRedP[12], kRedS[12]}, {kRedP[13], kRedS[13]}, {kRedP[14], kRedS[14]}, {kRedP[15], kRedS[15]}};

__host__ __device__ constexpr bool kept(int g) { return exp_of(g).c < 2; }

// position of a kept multi-index among the kept ones of [lo, g)
__host__ __device__ constexpr int kept_slot(int lo, int g)
{
    int n = 0;
    for (int h = lo; h < g; ++h) n += kept(h) ? 1 : 0;
    return n;
}

constexpr bool check_reduction()
{
    for (int b = 0; b < kNRed; ++b) {
        if (kRedS[b] < 0) continue;
        // the eliminated component is the primary one with an xx (or yy) traded for zz
        const Exp3 p = exp_of(kRedP[b]), q = exp_of(kRedS[b]);
        const bool via_x = p.a >= 2 && q.a == p.a - 2 && q.b == p.b && q.c == p.c + 2;
        const bool via_y = p.b >= 2 && q.b == p.b - 2 && q.a == p.a && q.c == p.c + 2;
        if (!via_x && !via_y) return false;
    }
    return kept_slot(0, 20) == 16 && kept_slot(1, 35) == 24;
}
static_assert(check_reduction(), "trace reduction tables");

// truncation rules: acc over outputs g (range [LO, LO + N)) and reduced sources b
enum Trunc : int { TRUNC3 = 0, TRUNC4 = 1, EXACT4 = 2 };

__host__ __device__ constexpr bool allowed(int rule, int og, int ob)
{
    return rule == TRUNC3 ? og + ob <= 3 : (rule == TRUNC4 ? og + ob <= 4 : og + ob == 4);
}

template <int LO, int RULE, int G_, int B>
__device__ __forceinline__ void term_red(double* acc, const double* r, const double* G)
{
    if constexpr (kept(G_) && allowed(RULE, ord_of(G_), ord_of(kRedP[B]))) {
        constexpr int slot = kept_slot(LO, G_);
        constexpr int S = sum_idx(G_, kRedP[B]);
        acc[slot] = __builtin_fma(r[B], G[S], acc[slot]);
    }
}
template <int LO, int RULE, int G_, int... B>
__device__ __forceinline__ void row_red(double* acc, const double* r, const double* G,
                                        std::integer_sequence<int, B...>)
{
    (term_red<LO, RULE, G_, B>(acc, r, G), ...);
}
// acc[kept slot of g] += sum_b r[b] G[g + kRedP[b]] for g in [LO, LO + sizeof...(I))
template <int LO, int RULE, int... I>
__device__ __forceinline__ void contract_red(double* acc, const double* r, const double* G,
                                             std::integer_sequence<int, I...>)
{
    (row_red<LO, RULE, LO + I>(acc, r, G, std::make_integer_sequence<int, kNRed>{}), ...);
}

// full[g - LO] for g in [LO, LO + sizeof...(I)) from the kept accumulators;
// outputs with z exponent >= 2 are rebuilt in index order (their two
// partners always come earlier in graded-lex order).
template <int LO, int G_>
__device__ __forceinline__ void expand_one(const double* acc, double* full)
{
    if constexpr (kept(G_)) {
        constexpr int slot = kept_slot(LO, G_);
        full[G_ - LO] = acc[slot];
    } else {
        constexpr Exp3 e = exp_of(G_);
        constexpr int gx = idx_of(e.a + 2, e.b, e.c - 2);
        constexpr int gy = idx_of(e.a, e.b + 2, e.c - 2);
        full[G_ - LO] = -(full[gx - LO] + full[gy - LO]);
    }
}
template <int LO, int... I>
__device__ __forceinline__ void expand(const double* acc, double* full, std::integer_sequence<int, I...>)
{
    (expand_one<LO, LO + I>(acc, full), ...);
}

// ---------------------------------------------------------------------------
// Full truncation: every output |a| <= 3 keeps every source moment |b| <= 3,
// so derivatives of G are needed up to order 6. With the radial factors D_p
// (D_0 = G = -1/r, D_{p+1} = -(2p+1) D_p / r^2, i.e. D_p = d^p G / d(r^2/2)^p)
// and Phi^(p)_g = d^g D_p, the chain rule d_k D_p = r_k D_{p+1} gives
//   Phi^(p)_{g+e_k} = r_k Phi^(p+1)_g + g_k Phi^(p+1)_{g-e_k},   G_g = Phi^(0)_g
// (the same factors give the order <= 4 forms above). The recursion is
// unrolled at compile time, reducing z first, then x, then y; the compiler
// merges the repeated subexpressions, so each needed Phi is evaluated once.
// The trace reduction of sources and outputs holds unchanged: every output
// keeps complete source shells of orders 2 and 3, and the three outputs
// L_{g+xx}, L_{g+yy}, L_{g+zz} keep the same sources.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void radial(double x, double y, double z, double* D)
{
    const double r2 = __builtin_fma(x, x, __builtin_fma(y, y, z * z));
    const double ri = rsqrt_fp64(r2);
    const double ri2 = ri * ri;
    D[0] = -ri;
    D[1] = ri * ri2;
#pragma unroll
    for (int p = 1; p < N; ++p) D[p + 1] = (-(2.0 * p + 1.0)) * D[p] * ri2;
}

template <int P, int A, int B, int C>
__device__ __forceinline__ double phi(const double* r, const double* D)
{
    if constexpr (A + B + C == 0) {
        return D[P];
    } else if constexpr (C > 0) {
        const double t = r[2] * phi<P + 1, A, B, C - 1>(r, D);
        if constexpr (C >= 2) return __builtin_fma((double)(C - 1), phi<P + 1, A, B, C - 2>(r, D), t);
        else return t;
    } else if constexpr (A > 0) {
        const double t = r[0] * phi<P + 1, A - 1, B, C>(r, D);
        if constexpr (A >= 2) return __builtin_fma((double)(A - 1), phi<P + 1, A - 2, B, C>(r, D), t);
        else return t;
    } else {
        const double t = r[1] * phi<P + 1, A, B - 1, C>(r, D);
        if constexpr (B >= 2) return __builtin_fma((double)(B - 1), phi<P + 1, A, B - 2, C>(r, D), t);
        else return t;
    }
}

// acc[kept slot of g in [LO, ...)] += sum_b q[b] G_{g + kRedP[b]} over all 16
// reduced sources
template <int LO, int G_, int B>
__device__ __forceinline__ void term_full(double* acc, const double* q, const double* r, const double* D)
{
    if constexpr (kept(G_)) {
        constexpr int slot = kept_slot(LO, G_);
        constexpr Exp3 e = exp_of(G_);
        constexpr Exp3 f = exp_of(kRedP[B]);
        acc[slot] = __builtin_fma(q[B], phi<0, e.a + f.a, e.b + f.b, e.c + f.c>(r, D), acc[slot]);
    }
}
template <int LO, int G_, int... B>
__device__ __forceinline__ void row_full(double* acc, const double* q, const double* r, const double* D,
                                         std::integer_sequence<int, B...>)
{
    (term_full<LO, G_, B>(acc, q, r, D), ...);
}
template <int LO, int... I>
__device__ __forceinline__ void contract_full(double* acc, const double* q, const double* r, const double* D,
                                              std::integer_sequence<int, I...>)
{
    (row_full<LO, LO + I>(acc, q, r, D, std::make_integer_sequence<int, kNRed>{}), ...);
}

// Adjoint epilogue: with C_g (g = 1..34, stored at C[g - 1]) the derivative
// sums of orders 1..4 -- L'_g for the target role, F_g + E_g (E_g alone for
// |g| = 4) for the source role -- the position gradient is
// gX_k = sum_a c_a C_{a+e_k}, where c_a is the target's weight w_a (target
// role) or M_a / a! (source role).
template <int A, int K>
__device__ __forceinline__ double c_term(const double* C)
{
    constexpr int g = sum_idx(A, K);
    return C[g - 1];
}
template <int... A>
__device__ __forceinline__ void grad_x(const double* c, const double* C, double* gx,
                                       std::integer_sequence<int, A...>)
{
    ((gx[0] = __builtin_fma(c[A], c_term<A, 1>(C), gx[0]),
      gx[1] = __builtin_fma(c[A], c_term<A, 2>(C), gx[1]),
      gx[2] = __builtin_fma(c[A], c_term<A, 3>(C), gx[2])),
     ...);
}
// C_g = F_g + E_g for 1 <= |g| <= 3, E_g for |g| = 4 (g = I + 1)
template <int... I>
__device__ __forceinline__ void combine_fe(const double* F, const double* E, double* C,
                                           std::integer_sequence<int, I...>)
{
    ((C[I] = (I + 1 < 20) ? F[(I + 1) % 20] + E[I] : E[I]), ...);
}
template <int A>
__device__ __forceinline__ double inv_fact_c()
{
    constexpr double f = inv_multi_factorial(A);
    return f;
}
template <int... A>
__device__ __forceinline__ void scale_inv_fact(double* c, std::integer_sequence<int, A...>)
{
    ((c[A] *= inv_fact_c<A>()), ...);
}

// ---------------------------------------------------------------------------
// Kernel
// ---------------------------------------------------------------------------
enum Mode : int {
    MODE_MONO_HALO = 0,  // single block, mass only -> L
    MODE_FWD_HALO = 1,   // single block, moments -> L
    MODE_FWD_STORE = 2,  // batched forward -> L
    MODE_B2_STORE = 3,   // adjoint, source role per store sub-grid -> gM, gX (overwrite)
    MODE_B1_STORE = 4,   // adjoint, target role per target -> gX (accumulate)
    MODE_FULL_STORE = 5,  // batched forward, full truncation -> L
    MODE_B2F_STORE = 6,   // adjoint of the full truncation, source role -> gM, gX (overwrite)
    MODE_B1F_STORE = 7,   // adjoint of the full truncation, target role -> gX (accumulate)
    MODE_FS_STORE = 8,    // batched forward -> L, plus the target-role sums the adjoint needs
    MODE_B2S_STORE = 9,   // adjoint from those sums: source role per store sub-grid, plus the
                          // target role of its cells from the saved sums -> gM, gX (overwrite)
    MODE_AMC_STORE = 10,  // batched forward -> L, plus the angular-momentum correction of the
                          // force of each target cell -> dF
    MODE_FSF_STORE = 11,  // full truncation: forward -> L, plus the target-role sums of its adjoint
    MODE_B2SF_STORE = 12  // full truncation: one-pass adjoint from those sums -> gM, gX (overwrite)
};

constexpr int kMaxPieces = 16;  // work-list pieces (one per XCD) of a persistent launch

struct KParams {
    const double* mom;   // source moments / masses / weights, [ncomp][mom_stride]
    const double* pos;   // centres of mass, [3][pos_stride] (halo or store)
    long mom_stride;
    long pos_stride;
    const int4* rel;       // [owners][27]: {moment block, position block, packed shift, 0}
    const int* own_blk;    // owner -> store block of its own cells (NULL: identity)
    const int* order;      // work-group -> owner (NULL: identity)
    const double* aux;     // epilogue input: gL (B1) or M (B2), [20][aux_stride]
    long aux_stride;
    // B2S epilogue, the target role of the owner's cells: store sub-grid ->
    // target index (-1: none), that target's gL [20][aux_stride2] and its
    // saved sums [24][aux_stride2]
    const int* store_tgt;
    const double* aux2;
    const double* save;
    long aux_stride2;
    double* out0;          // L, or gM (B2), or gX (B1)
    double* out1;          // gX (B2), the saved target-role sums (FS) or the force correction (AMC)
    long out_stride;
    const int* out_blk;    // owner -> output block (NULL: identity)
    double period[3];
    int* counter;          // persistent launch: work counter(s), zeroed before the launch
    int n_items;           // persistent launch: number of work-list entries
    // persistent launch in pieces (npieces > 0): the work list is cut into
    // npieces consecutive pieces, [piece_off[k], piece_off[k + 1]), one per
    // XCD, each with its own counter counter[k]
    int npieces;
    int piece_off[kMaxPieces + 1];
};

template <int MODE>
struct ModeTraits {
    static constexpr bool halo = (MODE == MODE_MONO_HALO || MODE == MODE_FWD_HALO);
    // staged source components: the mass, or the 16 trace-reduced moments
    static constexpr int nq = (MODE == MODE_MONO_HALO) ? 1 : kNRed;
    static constexpr int nc = nq + 3;  // + centre of mass
    static constexpr bool adjoint = (MODE == MODE_B1_STORE || MODE == MODE_B2_STORE || MODE == MODE_B1F_STORE ||
                                     MODE == MODE_B2F_STORE || MODE == MODE_B2S_STORE || MODE == MODE_B2SF_STORE);
    static constexpr bool source_role = (MODE == MODE_B2_STORE || MODE == MODE_B2F_STORE ||
                                         MODE == MODE_B2S_STORE || MODE == MODE_B2SF_STORE);
    // one set of sums of orders 0..4 under the full truncation (every |b| <= 3)
    static constexpr bool full4 = (MODE == MODE_B2F_STORE || MODE == MODE_B2SF_STORE || MODE == MODE_FSF_STORE);
    // the target role added from saved sums in the source-role pass's epilogue
    static constexpr bool saved_target = (MODE == MODE_B2S_STORE || MODE == MODE_B2SF_STORE);
    // the F + E sums (total order 3, and the order-4 terms of orders 1..4)
    static constexpr bool fe = (MODE == MODE_B2_STORE || MODE == MODE_B2S_STORE || MODE == MODE_FS_STORE ||
                                MODE == MODE_AMC_STORE);
    // accumulators: monopole 20; forward 16 kept of 20; target-role adjoint
    // 24 kept of the 34 orders 1..4; source-role adjoint and the forward
    // with saved sums 16 + 24; with the full truncation the source role keeps
    // one set for orders 0..4 (25)
    static constexpr int nacc = (MODE == MODE_MONO_HALO)                             ? 20
                                : (MODE == MODE_B1_STORE || MODE == MODE_B1F_STORE) ? 24
                                : fe                                                ? 40
                                : full4                                             ? 25
                                                                                    : 16;
};

// LDS plane layout: cell-major, Layout::stride doubles per cell -- the
// centre (x, y, z), then the nq scaled source components, then padding. A
// pair is read with 16-byte loads from one base address (immediate offsets).
// The cell stride in 16-byte units is odd, so the 8 lanes served per LDS
// cycle by a 16-byte read -- 8 different cells modulo 8 in the mirrored lane
// pattern -- fall on disjoint banks.
template <int MODE>
struct Layout {
    static constexpr int nc = ModeTraits<MODE>::nc;
    static constexpr int nvec = (nc + 1) / 2;                               // 16-byte reads per cell
    static constexpr int stride = (nvec % 2 == 1) ? 2 * nvec : 2 * nvec + 2;  // doubles per cell
};

template <int MODE, int NW, bool SPLIT, int NP>
constexpr int lds_doubles()
{
    constexpr int plane = Layout<MODE>::stride * kPlane;
    constexpr int merge =
        SPLIT ? NW * ModeTraits<MODE>::nacc * 64 : ((NW == 16 || NP == 2) ? 20 * kSub3 : 0);
    return plane > merge ? plane : merge;
}

// Staging of one source z-plane (the 24 x 24 cells of the 3 x 3 neighbour
// blocks), one cell per thread: thread v takes cell v & 63 of block v >> 6
// (the block is wavefront-uniform, so its relation is a scalar load), loads
// the cell's centre and each of its moments once (a load of a wavefront reads
// 512 contiguous bytes in the batched forms, 8 rows of 64 bytes in the
// single-block form), forms the scaled trace-reduced sources with
// compile-time factors, and writes the cell's record with 16-byte LDS
// stores. A missing neighbour block is staged far away with zero sources.
template <int MODE, int B>
__device__ __forceinline__ double staged_source(const double* raw)
{
    constexpr bool rev = ModeTraits<MODE>::source_role;
    constexpr int cP = kRedP[B], cS = kRedS[B];
    constexpr double aP = rev ? parity_sign(cP) : parity_sign(cP) * inv_multi_factorial(cP);
    if constexpr (cS < 0) {
        return raw[cP] * aP;
    } else {
        constexpr double aS = rev ? parity_sign(cS) : parity_sign(cS) * inv_multi_factorial(cS);
        return __builtin_fma(raw[cS], -aS, raw[cP] * aP);
    }
}
template <int MODE, int... B>
__device__ __forceinline__ void staged_sources(const double* raw, double* val, std::integer_sequence<int, B...>)
{
    ((val[3 + B] = staged_source<MODE, B>(raw)), ...);
}

template <int MODE, int NW>
__device__ __forceinline__ void stage_plane(const KParams& p, const int4* rel, int zs, int tid, double* lds)
{
    using T = ModeTraits<MODE>;
    using Lay = Layout<MODE>;
    constexpr int nm = (T::nq == 1) ? 1 : 20;  // moments read per cell
    for (int v = tid; v < 9 * 64; v += NW * 64) {
        const int bxy = __builtin_amdgcn_readfirstlane(v >> 6);
        const int lane = v & 63;
        const int by = bxy / 3, bx = bxy - 3 * by;
        const double* pm;
        const double* px;
        long sm, sx;
        double sh[3] = {0.0, 0.0, 0.0};
        bool present = true;
        if constexpr (T::halo) {
            const long off = (long)zs * kPlane + (by * 8 + (lane >> 3)) * kHalo + bx * 8 + (lane & 7);
            pm = p.mom + off;
            px = p.pos + off;
            sm = sx = kHalo3;
        } else {
            const int4 rr = rel[9 * (zs >> 3) + bxy];  // uniform address: scalar load
            present = rr.x >= 0;
            const long o = 64 * (zs & 7) + lane;
            pm = p.mom + (present ? (long)rr.x * kSub3 : 0) + o;
            px = p.pos + (present ? (long)rr.y * kSub3 : 0) + o;
            sm = p.mom_stride;
            sx = p.pos_stride;
#pragma unroll
            for (int k = 0; k < 3; ++k) sh[k] = (double)(int)(int8_t)((rr.z >> (8 * k)) & 0xff) * p.period[k];
        }
        double val[2 * Lay::nvec];
#pragma unroll
        for (int c = 0; c < 2 * Lay::nvec; ++c) val[c] = 0.0;
        if (present) {
            double raw[nm];
#pragma unroll
            for (int c = 0; c < nm; ++c) raw[c] = pm[c * sm];
#pragma unroll
            for (int k = 0; k < 3; ++k) val[k] = px[k * sx] + sh[k];
            staged_sources<MODE>(raw, val, std::make_integer_sequence<int, T::nq>{});
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) val[k] = kFar;
        }
        double2* dst = reinterpret_cast<double2*>(
            lds + ((by * 8 + (lane >> 3)) * kHalo + bx * 8 + (lane & 7)) * Lay::stride);
#pragma unroll
        for (int j = 0; j < Lay::nvec; ++j) dst[j] = make_double2(val[2 * j], val[2 * j + 1]);
    }
}

// SPLIT (single-block forms only): one work-group per target z-plane of the
// block; its NW wavefronts share the plane's 64 cells and take the stencil
// rows round-robin; only the 19 source planes within reach are staged, and the
// partial sums are added in a fixed order at the end.
// NP = 2 (8 wavefronts): two passes over the source planes, target planes
// 0-3 then 4-7, two wavefronts per target plane with its stencil rows split
// in halves as with 16 wavefronts. Each pass stages the 21 source planes in
// its reach (42 instead of 24), and in exchange the work per staged plane is
// spread evenly over the 4 SIMDs (about 95% against 86% for one pass with a
// wavefront per target plane).
template <int MODE, int NW, bool SPLIT, int NP, bool PERSIST>
__global__ void __launch_bounds__(NW * 64) k_interact(const KParams p)
{
    using T = ModeTraits<MODE>;
    using Lay = Layout<MODE>;
    static_assert(NW == 8 || NW == 16, "8 or 16 wavefronts");
    static_assert(!SPLIT || (T::halo && NW == 8 && NP == 1), "plane split: single-block forms, 8 wavefronts");
    static_assert(NP == 1 || (NP == 2 && NW == 8), "two passes: 8 wavefronts");
    constexpr bool HALVES = !SPLIT && (NW == 16 || NP == 2);  // two wavefronts per target plane
    __shared__ double lds[lds_doubles<MODE, NW, SPLIT, NP>()];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int half = HALVES ? (wave & 1) : 0;
    // Persistent launch (counter != NULL): the work-group takes work-list
    // entries from a global counter until the list is exhausted; otherwise it
    // does the one entry of its index.
    __shared__ int s_item;
    static_assert(!PERSIST || !T::halo, "persistent launches: batched forms");
    constexpr bool persistent = PERSIST;
    int item = (int)blockIdx.x;
    // in pieces: the work-group starts on the piece of its XCD (work-group b
    // runs on XCD b mod npieces) and moves on to the next piece when that is
    // exhausted, until every piece is (s_step: pieces left behind)
    __shared__ int s_step;
    if (persistent && tid == 0) s_step = 0;
#pragma unroll 1
    for (;;) {
    if (persistent) {
        __syncthreads();  // the previous entry is finished by every wavefront
        if (tid == 0) {
            int it = p.n_items;
            if (p.npieces > 0) {
                for (int step = s_step; step < p.npieces; ++step) {
                    const int k = ((int)blockIdx.x + step) % p.npieces;
                    const int i = atomicAdd(p.counter + k, 1);
                    if (i < p.piece_off[k + 1] - p.piece_off[k]) {
                        it = p.piece_off[k] + i;
                        s_step = step;
                        break;
                    }
                }
            } else {
                it = atomicAdd(p.counter, 1);
            }
            s_item = it;
        }
        __syncthreads();
        item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= p.n_items) break;
    }
    const int owner = SPLIT ? 0 : (p.order ? p.order[item] : item);
    const int4* s_rel = T::halo ? nullptr : p.rel + (long)owner * 27;  // this owner's relations
#pragma unroll 1
    for (int pass = 0; pass < NP; ++pass) {
    // With 8 wavefronts and one pass (wave w on SIMD w % 4) the target planes
    // are paired per SIMD as (0,4) (1,6) (2,5) (3,7): the pairing whose summed
    // per-plane work varies least from one staged plane to the next.
    const int zt = SPLIT ? (int)blockIdx.x
                 : (NW == 16) ? (wave >> 1)
                 : (NP == 2) ? 4 * pass + (wave >> 1)
                             : (wave == 5 ? 6 : (wave == 6 ? 5 : wave));
    const int xt = lane & 7, yt = lane >> 3;
    const int pz = zt & 1;
    const int cell = xt + 8 * yt + 64 * zt;
    const int sgx = (xt & 1) ? -1 : 1;
    const int sgy = (yt & 1) ? -1 : 1;

    double xi, yi, zi;
    if constexpr (T::halo) {
        const int h = (8 + xt) + kHalo * (8 + yt) + kPlane * (8 + zt);
        xi = p.pos[h];
        yi = p.pos[kHalo3 + h];
        zi = p.pos[2 * kHalo3 + h];
    } else {
        const long b = p.own_blk ? p.own_blk[owner] : owner;
        const long o = b * kSub3 + cell;
        xi = p.pos[o];
        yi = p.pos[p.pos_stride + o];
        zi = p.pos[2 * p.pos_stride + o];
    }

    double acc[T::nacc];
#pragma unroll
    for (int a = 0; a < T::nacc; ++a) acc[a] = 0.0;

    // addresses in 16-byte units of the LDS plane
    constexpr int cs = Lay::stride / 2;
    const int lane_off = ((8 + yt) * kHalo + 8 + xt) * cs;
    const int step_x = sgx * cs;
    const int step_y = sgy * kHalo * cs;
    const double2* lds2 = reinterpret_cast<const double2*>(lds);

    const int zs_begin = SPLIT ? (8 + zt - kReach > 0 ? 8 + zt - kReach : 0)
                       : (NP == 2 ? (pass == 0 ? 0 : 8 + 4 - kReach) : 0);
    const int zs_end = SPLIT ? (8 + zt + kReach + 1 < kHalo ? 8 + zt + kReach + 1 : kHalo)
                     : (NP == 2 ? (pass == 0 ? 8 + 3 + kReach + 1 : kHalo) : kHalo);
    for (int zs = zs_begin; zs < zs_end; ++zs) {
        __syncthreads();
        stage_plane<MODE, NW>(p, s_rel, zs, tid, lds);
        __syncthreads();
        const int dz = zs - (8 + zt);
        if (dz >= -kReach && dz <= kReach) {
            const int* rg = c_stencil.range[pz][dz + kReach];
            int r0 = rg[0], r1 = rg[2], rstep = 1;
            if (SPLIT) {
                r0 += wave;
                rstep = NW;
            } else if (HALVES) {
                if (half == 0)
                    r1 = rg[1];
                else
                    r0 = rg[1];
            }
            for (int r = r0; r < r1; r += rstep) {
                const uint32_t w = c_stencil.rows[pz][r];
                const int dy = (int)(int8_t)(w & 0xff);
                const int dx0 = (int)(int8_t)((w >> 8) & 0xff);
                const int n = (int)(w >> 16);
                int off = lane_off + dy * step_y + dx0 * step_x;
                for (int k = 0; k < n; ++k, off += step_x) {
                    double f[2 * Lay::nvec];
#pragma unroll
                    for (int j = 0; j < Lay::nvec; ++j) {
                        const double2 v = lds2[off + j];
                        f[2 * j] = v.x;
                        f[2 * j + 1] = v.y;
                    }
                    const double rx = xi - f[0];
                    const double ry = yi - f[1];
                    const double rz = zi - f[2];
                    const double* q = f + 3;
                    if constexpr (MODE == MODE_MONO_HALO) {
                        double G[20];
                        green<3>(rx, ry, rz, G);
#pragma unroll
                        for (int a = 0; a < 20; ++a) acc[a] = __builtin_fma(q[0], G[a], acc[a]);
                    } else if constexpr (MODE == MODE_FULL_STORE) {
                        // L_a, |a| <= 3 and |b| <= 3
                        double D[7];
                        radial<6>(rx, ry, rz, D);
                        const double rr[3] = {rx, ry, rz};
                        contract_full<0>(acc, q, rr, D, std::make_integer_sequence<int, 20>{});
                    } else if constexpr (MODE == MODE_B1F_STORE) {
                        // L'_g, 1 <= |g| <= 4, every |b| <= 3
                        double D[8];
                        radial<7>(rx, ry, rz, D);
                        const double rr[3] = {rx, ry, rz};
                        contract_full<1>(acc, q, rr, D, std::make_integer_sequence<int, 34>{});
                    } else if constexpr (T::full4) {
                        // C_d, 0 <= |d| <= 4, every source moment (|a| <= 3 or |b| <= 3)
                        double D[8];
                        radial<7>(rx, ry, rz, D);
                        const double rr[3] = {rx, ry, rz};
                        contract_full<0>(acc, q, rr, D, std::make_integer_sequence<int, 35>{});
                    } else if constexpr (!T::adjoint && !T::fe) {
                        // L_a, |a| + |b| <= 3
                        double G[20];
                        green<3>(rx, ry, rz, G);
                        contract_red<0, TRUNC3>(acc, q, G, std::make_integer_sequence<int, 20>{});
                    } else if constexpr (MODE == MODE_B1_STORE) {
                        // L'_g, 1 <= |g| <= 4, |g| + |b| <= 4
                        double G[35];
                        green<4>(rx, ry, rz, G);
                        contract_red<1, TRUNC4>(acc, q, G, std::make_integer_sequence<int, 34>{});
                    } else {
                        // F_d (|d| + |a| <= 3) and E_d (|d| + |a| = 4, |d| >= 1)
                        double G[35];
                        green<4>(rx, ry, rz, G);
                        contract_red<0, TRUNC3>(acc, q, G, std::make_integer_sequence<int, 20>{});
                        contract_red<1, EXACT4>(acc + 16, q, G, std::make_integer_sequence<int, 34>{});
                    }
                }
            }
        }
    }

    // ---------------- epilogues ----------------
    if constexpr (SPLIT) {
        // partial sums of the plane's wavefronts, added by wavefront 0 in order
        __syncthreads();
#pragma unroll
        for (int a = 0; a < T::nacc; ++a) lds[(wave * T::nacc + a) * 64 + lane] = acc[a];
        __syncthreads();
        if (wave != 0) return;
#pragma unroll
        for (int a = 0; a < T::nacc; ++a) {
            double v = lds[a * 64 + lane];
            for (int w = 1; w < NW; ++w) v += lds[(w * T::nacc + a) * 64 + lane];
            acc[a] = v;
        }
    } else if constexpr (HALVES) {
        // the two wavefronts of a target plane add their partial sums, through
        // LDS in rounds of at most 20 components
#pragma unroll
        for (int a0 = 0; a0 < T::nacc; a0 += 20) {
            __syncthreads();
            if (half == 1) {
#pragma unroll
                for (int a = a0; a < T::nacc && a < a0 + 20; ++a) lds[(a - a0) * kSub3 + cell] = acc[a];
            }
            __syncthreads();
            if (half == 0) {
#pragma unroll
                for (int a = a0; a < T::nacc && a < a0 + 20; ++a) acc[a] += lds[(a - a0) * kSub3 + cell];
            }
        }
        if (half == 1) continue;  // the next pass (none after the last)
    }
    if constexpr (MODE == MODE_FSF_STORE) {
        // full truncation: L is the sums of orders 0..3 (kept slots 0..15);
        // the target-role sums C'_g, 1 <= |g| <= 4, are the kept slots 1..24
        double L[20];
        expand<0>(acc, L, std::make_integer_sequence<int, 20>{});
        const long b = p.out_blk ? p.out_blk[owner] : owner;
        const long ob = b * kSub3 + cell;
#pragma unroll
        for (int a = 0; a < 20; ++a) p.out0[a * p.out_stride + ob] = L[a];
#pragma unroll
        for (int k = 0; k < 24; ++k) p.out1[k * p.out_stride + ob] = acc[k + 1];
    } else if constexpr (MODE == MODE_FS_STORE) {
        // L from F; the saved sums C'_g (1 <= |g| <= 4, total order 4) =
        // F_g + E_g for |g| <= 3, E_g for |g| = 4, in kept slots (F's kept
        // slot k + 1 and C's kept slot k are the same multi-index)
        double L[20];
        expand<0>(acc, L, std::make_integer_sequence<int, 20>{});
        const long b = p.out_blk ? p.out_blk[owner] : owner;
        const long ob = b * kSub3 + cell;
#pragma unroll
        for (int a = 0; a < 20; ++a) p.out0[a * p.out_stride + ob] = L[a];
#pragma unroll
        for (int k = 0; k < 24; ++k) p.out1[k * p.out_stride + ob] = k < 15 ? acc[k + 1] + acc[16 + k] : acc[16 + k];
    } else if constexpr (MODE == MODE_AMC_STORE) {
        // L from F; the force correction dF_k = -sum_{|a| <= 3} (M_a/a!) E_{a+e_k}
        // (E: the sums of exact total order 4), with the target cell's own moments
        double L[20];
        expand<0>(acc, L, std::make_integer_sequence<int, 20>{});
        const long b = p.out_blk ? p.out_blk[owner] : owner;
        const long ob = b * kSub3 + cell;
#pragma unroll
        for (int a = 0; a < 20; ++a) p.out0[a * p.out_stride + ob] = L[a];
        double E[34];
        expand<1>(acc + 16, E, std::make_integer_sequence<int, 34>{});
        const long mb = (p.own_blk ? p.own_blk[owner] : owner) * (long)kSub3 + cell;
        double c[20];
#pragma unroll
        for (int a = 0; a < 20; ++a) c[a] = p.aux[a * p.aux_stride + mb];
        scale_inv_fact(c, std::make_integer_sequence<int, 20>{});
        double gx[3] = {0.0, 0.0, 0.0};
        grad_x(c, E, gx, std::make_integer_sequence<int, 20>{});
#pragma unroll
        for (int k = 0; k < 3; ++k) p.out1[k * p.out_stride + ob] = -gx[k];
    } else if constexpr (!T::adjoint) {
        double L[20];
        if constexpr (MODE == MODE_MONO_HALO) {
#pragma unroll
            for (int a = 0; a < 20; ++a) L[a] = acc[a];
        } else {
            expand<0>(acc, L, std::make_integer_sequence<int, 20>{});
        }
        if constexpr (T::halo) {
#pragma unroll
            for (int a = 0; a < 20; ++a) p.out0[a * kSub3 + cell] = L[a];
        } else {
            const long b = p.out_blk ? p.out_blk[owner] : owner;
#pragma unroll
            for (int a = 0; a < 20; ++a) p.out0[a * p.out_stride + b * kSub3 + cell] = L[a];
        }
    } else {
        double C[34];
        double F[20];
        if constexpr (MODE == MODE_B1_STORE || MODE == MODE_B1F_STORE) {
            expand<1>(acc, C, std::make_integer_sequence<int, 34>{});
        } else if constexpr (T::full4) {
            // one set of sums for orders 0..4: F (orders 0..3) and C (1..4)
            expand<0>(acc, F, std::make_integer_sequence<int, 20>{});
            expand<1>(acc + 1, C, std::make_integer_sequence<int, 34>{});
        } else {
            double E[34];
            expand<0>(acc, F, std::make_integer_sequence<int, 20>{});
            expand<1>(acc + 16, E, std::make_integer_sequence<int, 34>{});
            combine_fe(F, E, C, std::make_integer_sequence<int, 34>{});
        }
        const long ab = (long)owner * kSub3 + cell;
        double c[20];
#pragma unroll
        for (int a = 0; a < 20; ++a) c[a] = p.aux[a * p.aux_stride + ab];
        if constexpr (T::source_role)
            scale_inv_fact(c, std::make_integer_sequence<int, 20>{});  // M_b / b!
        double gx[3] = {0.0, 0.0, 0.0};
        grad_x(c, C, gx, std::make_integer_sequence<int, 20>{});
        const long b = p.out_blk ? p.out_blk[owner] : owner;
        const long ob = b * kSub3 + cell;
        if constexpr (T::source_role) {
            scale_inv_fact(F, std::make_integer_sequence<int, 20>{});  // gM_b = F_b / b!
#pragma unroll
            for (int a = 0; a < 20; ++a) p.out0[a * p.out_stride + ob] = F[a];
            if constexpr (T::saved_target) {
                // the target role of the owner's cells, from the sums the
                // forward saved: gX_k += sum_a w_a C'_{a+e_k}
                const int t = p.store_tgt[owner];
                if (t >= 0) {
                    const long tb = (long)t * kSub3 + cell;
                    double Ck[24], Cf[34], w[20];
#pragma unroll
                    for (int k = 0; k < 24; ++k) Ck[k] = p.save[k * p.aux_stride2 + tb];
                    expand<1>(Ck, Cf, std::make_integer_sequence<int, 34>{});
#pragma unroll
                    for (int a = 0; a < 20; ++a) w[a] = p.aux2[a * p.aux_stride2 + tb];
                    double gt[3] = {0.0, 0.0, 0.0};
                    grad_x(w, Cf, gt, std::make_integer_sequence<int, 20>{});
#pragma unroll
                    for (int k = 0; k < 3; ++k) gx[k] += gt[k];
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) p.out1[k * p.out_stride + ob] = gx[k];
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) p.out0[k * p.out_stride + ob] += gx[k];
        }
    }
    }  // pass
    if (!persistent) break;
    }  // work-list entries
}

// zeroes the kMaxPieces counters of a persistent launch (one per lane)
__global__ void k_zero_counter(int* c) { c[threadIdx.x] = 0; }

}  // namespace
