// ot_tree.hip -- tree passes around the interaction kernels: the upward pass
// (M2M), the downward pass (L2L) and the local evaluation of force and
// energy, behind the C ABI declared in include/ot_fmm.h. All three are
// streaming kernels bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <new>
#include <utility>
#include <vector>

#include "ot_common.h"
#include "ot_host.h"
#include "ot_fmm.h"

using namespace otfmm;

namespace {

// ---------------------------------------------------------------------------
// Tree passes around the interaction (paper Sec. 2.1 / 2.3: the FMM gravity
// solver works on the octree of sub-grids). A parent node p has 8 child nodes
// children[p][o], o = ox + 2 oy + 4 oz; parent cell (X, Y, Z) covers the 2x2x2
// child cells (2 (X % 4) + a, 2 (Y % 4) + b, 2 (Z % 4) + c) of child o =
// (X / 4, Y / 4, Z / 4). These kernels are bound by HBM bandwidth.
// ---------------------------------------------------------------------------
template <int B, int G>
__device__ __forceinline__ void shift_term(double* acc, const double* m, const double* mono)
{
    // acc_B += C(B, G) m_G d^(B - G) for G <= B componentwise
    constexpr Exp3 b = exp_of(B), g = exp_of(G);
    if constexpr (g.a <= b.a && g.b <= b.b && g.c <= b.c) {
        constexpr double c = factorial(b.a) / (factorial(g.a) * factorial(b.a - g.a)) *
                             factorial(b.b) / (factorial(g.b) * factorial(b.b - g.b)) *
                             factorial(b.c) / (factorial(g.c) * factorial(b.c - g.c));
        constexpr int e = idx_of(b.a - g.a, b.b - g.b, b.c - g.c);
        if constexpr (c == 1.0)
            acc[B] = __builtin_fma(m[G], mono[e], acc[B]);
        else
            acc[B] = __builtin_fma(c * m[G], mono[e], acc[B]);
    }
}
template <int B, int... G>
__device__ __forceinline__ void shift_row(double* acc, const double* m, const double* mono,
                                          std::integer_sequence<int, G...>)
{
    (shift_term<B, G>(acc, m, mono), ...);
}
template <int... B>
__device__ __forceinline__ void moment_shift(double* acc, const double* m, const double* mono,
                                             std::integer_sequence<int, B...>)
{
    (shift_row<B>(acc, m, mono, std::make_integer_sequence<int, 20>{}), ...);
}

// the 20 monomials d^e, |e| <= 3, graded-lex order
__device__ __forceinline__ void monomials(double x, double y, double z, double* t)
{
    t[0] = 1.0;
    t[1] = x;
    t[2] = y;
    t[3] = z;
    t[4] = x * x;
    t[5] = x * y;
    t[6] = x * z;
    t[7] = y * y;
    t[8] = y * z;
    t[9] = z * z;
    t[10] = t[4] * x;
    t[11] = t[4] * y;
    t[12] = t[4] * z;
    t[13] = x * t[7];
    t[14] = t[5] * z;
    t[15] = x * t[9];
    t[16] = t[7] * y;
    t[17] = t[7] * z;
    t[18] = y * t[9];
    t[19] = t[9] * z;
}

struct TreeParams {
    const int* children;  // [Sp][8]
    const double* m_in;   // M2M: child moments; L2L: parent coefficients
    const double* x_in;   // M2M: child centres; L2L: parent centres
    const double* x_in2;  // L2L: child centres
    double* m_out;        // M2M: parent moments; L2L: child coefficients (accumulated)
    double* x_out;        // M2M: parent centres
    long n_child, n_parent;  // cells per component in child / parent stores
    int Sp;
};

// Cross-lane exchange inside a wavefront through DPP (no LDS traffic): the
// value held by lane ^ 1 (quad permutation [1, 0, 3, 2]) or by lane ^ 8
// (rotation by 8 inside each row of 16 lanes).
constexpr int kDppXor1 = 0xB1;
constexpr int kDppXor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ double dpp_get(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// Sum over the lanes {l, l^1, l^8, l^9}; every one of them gets the same bits
// (each step adds the same two values, in either order).
__device__ __forceinline__ double quad_sum(double v)
{
    v += dpp_get<kDppXor1>(v);
    return v + dpp_get<kDppXor8>(v);
}

// Upward pass. A wavefront covers one z-pair of the cells of one child node
// (lane = x + 8 y; cells (x, y, 2Z) and (x, y, 2Z + 1)), so every load is one
// contiguous 512-byte row. The 8 children of a parent cell are the two cells
// of lanes l, l^1, l^8 and l^9, summed by cross-lane exchange; each of those
// four lanes then puts 5 of the 20 parent moments into LDS, where the four
// wavefronts of the work-group assemble one full 8x8 parent plane that is
// stored as 512-byte rows (directly from the lanes, the stores were 32-byte
// pieces and the pass 20% slower).
__global__ void __launch_bounds__(256) k_m2m(const TreeParams p)
{
    // work-group = one z-plane of a parent node (8 per node): its 4 wavefronts
    // are the 4 child octants below that plane (one z-pair of cells each); the
    // indices are wave-uniform (scalar registers, scalar child lookup)
    const long blk = blockIdx.x;
    if (blk >= (long)p.Sp * 8) return;  // whole work-groups
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int node = (int)(blk >> 3), oz = (int)((blk >> 2) & 1), Z = (int)(blk & 3);
    const int o = wave + 4 * oz;
    const long j0 = (long)p.children[node * 8 + o] * kSub3 + 128 * Z + lane;
    const long j1 = j0 + 64;
    const long nc = p.n_child;

    // every load of the wavefront is issued before the first use
    double m0[20], m1[20], x0[3], x1[3], c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        x0[k] = p.x_in[k * nc + j0];
        x1[k] = p.x_in[k * nc + j1];
    }
#pragma unroll
    for (int b = 0; b < 20; ++b) {
        m0[b] = p.m_in[b * nc + j0];
        m1[b] = p.m_in[b * nc + j1];
    }
    const double m = quad_sum(m0[0] + m1[0]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double mx = quad_sum(__builtin_fma(m0[0], x0[k], m1[0] * x1[k]));
        const double gx = quad_sum(x0[k] + x1[k]);
        c[k] = m > 0.0 ? mx / m : gx * 0.125;  // plain mean of the centres if massless
    }

    double acc[20], mono[20];
#pragma unroll
    for (int b = 0; b < 20; ++b) acc[b] = 0.0;
    monomials(x0[0] - c[0], x0[1] - c[1], x0[2] - c[2], mono);
    moment_shift(acc, m0, mono, std::make_integer_sequence<int, 20>{});
    monomials(x1[0] - c[0], x1[1] - c[1], x1[2] - c[2], mono);
    moment_shift(acc, m1, mono, std::make_integer_sequence<int, 20>{});
#pragma unroll
    for (int b = 0; b < 20; ++b) acc[b] = quad_sum(acc[b]);

    // the 8x8 parent cells of the plane gather in LDS, so that every store
    // is one contiguous 512-byte row
    __shared__ double s_out[23][64];
    const int x = lane & 7, y = lane >> 3;
    const int q = (x & 1) + 2 * (y & 1);
    const int cp = (x >> 1) + 4 * (o & 1) + 8 * ((y >> 1) + 4 * ((o >> 1) & 1));  // cell in the plane
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const double v = q == 0 ? acc[4 * i] : q == 1 ? acc[4 * i + 1] : q == 2 ? acc[4 * i + 2]
                                                                                  : acc[4 * i + 3];
        s_out[4 * i + q][cp] = v;
    }
    if (q < 3) s_out[20 + q][cp] = q == 0 ? c[0] : q == 1 ? c[1] : c[2];
    __syncthreads();
    const long np = p.n_parent;
    const long base = (long)node * kSub3 + 64 * (Z + 4 * oz) + lane;
    for (int comp = wave; comp < 23; comp += 4) {
        if (comp < 20)
            p.m_out[comp * np + base] = s_out[comp][lane];
        else
            p.x_out[(comp - 20) * np + base] = s_out[comp][lane];
    }
}

// L_A(child) += sum_{|G| <= 3 - |A|} L_{A+G}(parent) d^G / G!
template <int A, int G>
__device__ __forceinline__ void l2l_term(double& acc, const double* lp, const double* mono)
{
    if constexpr (ord_of(A) + ord_of(G) <= 3) {
        constexpr int S = sum_idx(A, G);
        constexpr double f = inv_multi_factorial(G);
        if constexpr (f == 1.0)
            acc = __builtin_fma(lp[S], mono[G], acc);
        else
            acc = __builtin_fma(lp[S] * f, mono[G], acc);
    }
}
template <int A, int... G>
__device__ __forceinline__ void l2l_row(double* out, const double* lp, const double* mono,
                                        std::integer_sequence<int, G...>)
{
    double acc = 0.0;
    (l2l_term<A, G>(acc, lp, mono), ...);
    out[A] += acc;
}
template <int... A>
__device__ __forceinline__ void l2l_shift(double* out, const double* lp, const double* mono,
                                          std::integer_sequence<int, A...>)
{
    (l2l_row<A>(out, lp, mono, std::make_integer_sequence<int, 20>{}), ...);
}

// Downward pass: one thread per child cell (the child node of parent `node`
// at octant o, cell c); each child node has one parent, so writes never race.
// (Read per thread from global memory, the parent values took 5% longer.)
__global__ void __launch_bounds__(256) k_l2l(const TreeParams p)
{
    // work-group = 4 child z-planes (256 cells) of one child node; its 32
    // parent cells (2 planes x 4 x 4) are read once into LDS and shared by
    // the 8 children of each (instead of 8 loads per value)
    const long blk = blockIdx.x;
    if (blk >= (long)p.Sp * 16) return;  // whole work-groups
    const int tid = threadIdx.x;
    const int node = (int)(blk >> 4), o = (int)((blk >> 1) & 7), zh = (int)(blk & 1);
    __shared__ double s_lp[23][32];
    for (int i = tid; i < 23 * 32; i += 256) {
        const int comp = i >> 5, r = i & 31;
        const int xl = r & 3, yl = (r >> 2) & 3, zl = r >> 4;
        const int pc = xl + 4 * (o & 1) + 8 * (yl + 4 * ((o >> 1) & 1)) + 64 * (2 * zh + zl + 4 * (o >> 2));
        const long ip = (long)node * kSub3 + pc;
        s_lp[comp][r] = comp < 20 ? p.m_in[comp * p.n_parent + ip] : p.x_in[(comp - 20) * p.n_parent + ip];
    }
    __syncthreads();
    const int c = 256 * zh + tid;
    const int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
    const int r = (x >> 1) + 4 * (y >> 1) + 16 * ((z >> 1) - 2 * zh);
    const long j = (long)p.children[node * 8 + o] * kSub3 + c;
    double lp[20], mono[20], out[20];
#pragma unroll
    for (int a = 0; a < 20; ++a) lp[a] = s_lp[a][r];
#pragma unroll
    for (int a = 0; a < 20; ++a) out[a] = p.m_out[a * p.n_child + j];
    monomials(p.x_in2[j] - s_lp[20][r], p.x_in2[p.n_child + j] - s_lp[21][r],
              p.x_in2[2 * p.n_child + j] - s_lp[22][r], mono);
    l2l_shift(out, lp, mono, std::make_integer_sequence<int, 20>{});
#pragma unroll
    for (int a = 0; a < 20; ++a) p.m_out[a * p.n_child + j] = out[a];
}

// F_k = - sum_{|a| <= 2} M_a / a! L_{a+e_k},  W = 1/2 sum_{|a| <= 3} M_a / a! L_a
template <int A>
__device__ __forceinline__ void eval_term(const double* m, const double* l, double* f, double& w)
{
    constexpr double inv = inv_multi_factorial(A);
    const double ma = (inv == 1.0) ? m[A] : m[A] * inv;
    w = __builtin_fma(ma, l[A], w);
    if constexpr (ord_of(A) <= 2) {
        f[0] = __builtin_fma(-ma, l[sum_idx(A, 1)], f[0]);
        f[1] = __builtin_fma(-ma, l[sum_idx(A, 2)], f[1]);
        f[2] = __builtin_fma(-ma, l[sum_idx(A, 3)], f[2]);
    }
}
template <int... A>
__device__ __forceinline__ void eval_all(const double* m, const double* l, double* f, double& w,
                                         std::integer_sequence<int, A...>)
{
    (eval_term<A>(m, l, f, w), ...);
}

__global__ void __launch_bounds__(256) k_evaluate(const double* M, const double* L, double* F,
                                                  double* W, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double m[20], l[20], f[3] = {0.0, 0.0, 0.0}, w = 0.0;
#pragma unroll
    for (int a = 0; a < 20; ++a) {
        m[a] = M[a * n + i];
        l[a] = L[a * n + i];
    }
    eval_all(m, l, f, w, std::make_integer_sequence<int, 20>{});
    F[i] = f[0];
    F[n + i] = f[1];
    F[2 * n + i] = f[2];
    W[i] = 0.5 * w;
}

}  // namespace

struct ot_fmm_tree_s {
    int device = 0;
    int32_t Sp = 0, Sc = 0;
    int* d_children = nullptr;  // [Sp][8]
};

// a pass of a tree runs on the device the tree was created on
static int check_tree(ot_fmm_tree tree)
{
    if (!tree) return fail(OT_FMM_EINVAL, "null tree");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != tree->device) return fail(OT_FMM_EINVAL, "tree belongs to another device");
    return OT_FMM_OK;
}

extern "C" {

int ot_fmm_tree_create(int32_t Sp, int32_t Sc, const int32_t* children, ot_fmm_tree* out)
{
    g_last_error.clear();
    if (!out) return fail(OT_FMM_EINVAL, "null output pointer");
    *out = nullptr;
    if (Sp <= 0 || Sc <= 0 || !children) return fail(OT_FMM_EINVAL, "Sp, Sc > 0 and children required");
    // keeps every launch grid (one thread per child cell) below 2^27 work-groups
    if ((int64_t)Sp * 8 > ((int64_t)1 << 26)) return fail(OT_FMM_EINVAL, "tree too large");
    std::vector<char> used(Sc, 0);
    for (int64_t i = 0; i < (int64_t)Sp * 8; ++i) {
        const int32_t c = children[i];
        if (c < 0 || c >= Sc) return fail(OT_FMM_EINVAL, "child id out of range");
        if (used[c]) return fail(OT_FMM_EINVAL, "a child node appears under two parents");
        used[c] = 1;
    }
    int rc = ensure_device();
    if (rc) return rc;
    ot_fmm_tree t = new (std::nothrow) ot_fmm_tree_s();
    if (!t) return fail(OT_FMM_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&t->device);
    if (e != hipSuccess) {
        delete t;
        return hip_fail(e, "hipGetDevice");
    }
    t->Sp = Sp;
    t->Sc = Sc;
    std::vector<int> ch(children, children + (int64_t)Sp * 8);
    if ((rc = upload(&t->d_children, ch))) {
        (void)hipFree(t->d_children);
        delete t;
        return rc;
    }
    *out = t;
    return OT_FMM_OK;
}

int ot_fmm_tree_destroy(ot_fmm_tree tree)
{
    g_last_error.clear();
    if (!tree) return OT_FMM_OK;
    (void)hipFree(tree->d_children);
    delete tree;
    return OT_FMM_OK;
}

int ot_fmm_m2m(ot_fmm_tree tree, const double* Mc, const double* comc, double* Mp, double* comp,
               void* stream)
{
    g_last_error.clear();
    int rc = check_tree(tree);
    if (rc) return rc;
    if (!aligned8(Mc) || !aligned8(comc) || !aligned8(Mp) || !aligned8(comp))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    {
        const int64_t nc = (int64_t)tree->Sc * kSub3, np = (int64_t)tree->Sp * kSub3;
        if (overlap(Mp, 20 * np, Mc, 20 * nc) || overlap(Mp, 20 * np, comc, 3 * nc) ||
            overlap(comp, 3 * np, Mc, 20 * nc) || overlap(comp, 3 * np, comc, 3 * nc) ||
            overlap(Mp, 20 * np, comp, 3 * np))
            return fail(OT_FMM_EINVAL, "outputs overlap inputs or each other");
    }
    TreeParams tp{};
    tp.children = tree->d_children;
    tp.m_in = Mc;
    tp.x_in = comc;
    tp.m_out = Mp;
    tp.x_out = comp;
    tp.n_child = (long)tree->Sc * kSub3;
    tp.n_parent = (long)tree->Sp * kSub3;
    tp.Sp = tree->Sp;
    // 8 work-groups of 4 wavefronts per parent node
    hipLaunchKernelGGL(k_m2m, dim3((unsigned)tree->Sp * 8), dim3(256), 0, (hipStream_t)stream, tp);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? OT_FMM_OK : hip_fail(e, "kernel launch");
}

int ot_fmm_l2l(ot_fmm_tree tree, const double* Lp, const double* comp, const double* comc,
               double* Lc, void* stream)
{
    g_last_error.clear();
    int rc = check_tree(tree);
    if (rc) return rc;
    if (!aligned8(Lp) || !aligned8(comp) || !aligned8(comc) || !aligned8(Lc))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    {
        const int64_t nc = (int64_t)tree->Sc * kSub3, np = (int64_t)tree->Sp * kSub3;
        if (overlap(Lc, 20 * nc, Lp, 20 * np) || overlap(Lc, 20 * nc, comp, 3 * np) ||
            overlap(Lc, 20 * nc, comc, 3 * nc))
            return fail(OT_FMM_EINVAL, "Lc overlaps an input");
    }
    TreeParams tp{};
    tp.children = tree->d_children;
    tp.m_in = Lp;
    tp.x_in = comp;
    tp.x_in2 = comc;
    tp.m_out = Lc;
    tp.n_child = (long)tree->Sc * kSub3;
    tp.n_parent = (long)tree->Sp * kSub3;
    tp.Sp = tree->Sp;
    const long n = (long)tree->Sp * 8 * kSub3;
    // 16 work-groups of 256 child cells per parent node
    hipLaunchKernelGGL(k_l2l, dim3((unsigned)(n / 256)), dim3(256), 0, (hipStream_t)stream, tp);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? OT_FMM_OK : hip_fail(e, "kernel launch");
}

int ot_fmm_evaluate(int64_t ncells, const double* M, const double* L, double* F, double* W,
                    void* stream)
{
    g_last_error.clear();
    if (ncells <= 0 || ncells > ((int64_t)1 << 38)) return fail(OT_FMM_EINVAL, "ncells out of range");
    if (!aligned8(M) || !aligned8(L) || !aligned8(F) || !aligned8(W))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    if (overlap(F, 3 * ncells, M, 20 * ncells) || overlap(F, 3 * ncells, L, 20 * ncells) ||
        overlap(W, ncells, M, 20 * ncells) || overlap(W, ncells, L, 20 * ncells) || overlap(F, 3 * ncells, W, ncells))
        return fail(OT_FMM_EINVAL, "outputs overlap inputs or each other");
    int rc = ensure_device();
    if (rc) return rc;
    hipLaunchKernelGGL(k_evaluate, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, M, L, F, W, (long)ncells);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? OT_FMM_OK : hip_fail(e, "kernel launch");
}

}  // extern "C"
