/*
 * ot_oracle.c -- plain FP64 CPU oracle for the FMM cell-to-cell gravity
 * interaction kernels. TEST INFRASTRUCTURE ONLY: it is called by the tests,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by
 * the library. It shares no code, header, table or generator with the HIP
 * path.
 *
 * What it computes (paper Sec. 2.1: Octo-Tiger's gravity solver is a fast
 * multipole method on an octree of 8x8x8 sub-grids; Sec. 2.2.1 / 2.3: each
 * compute kernel works on one sub-grid plus its ghost layers; Sec. 2.2.4:
 * kernels for many sub-grids may be aggregated into one launch):
 *
 *   For every target cell i of a target sub-grid and every alpha, |alpha|<=3,
 *     L_alpha(i) = sum_{j in S(i)} sum_{|beta| <= 3-|alpha|}
 *                        s_beta M_beta(j) G_{alpha+beta}(X_i - X_j)
 *   G(r) = -1/|r|, G_gamma = d^gamma G, s_beta = (-1)^{|beta|}/beta!,
 *   M_beta(j) = raw Cartesian moments of cell j about its centre of mass X_j,
 *   S(i) = cells j of the 3x3x3 sub-grid neighbourhood (24^3 halo block) with
 *          |j - i|_2 > 4  and  |floor(j/2) - floor(i/2)|_2 <= 4  (integer
 *          cell coordinates), whose sub-grid is available.
 *
 * The method reaches exactly this sum (no approximation beyond the stated
 * truncation), so the oracle is that sum written out: a loop over target
 * cells, a brute-force test of the criterion for every candidate source, and
 * the plain double sum over (alpha, beta). The adjoint is the chain rule
 * applied to the same definition, pair by pair.
 *
 * Component order of every 20- or 35-vector: graded lexicographic with x most
 * significant (1; x,y,z; xx,xy,xz,yy,yz,zz; xxx,xxy,...,zzz; xxxx,...).
 *
 * A second truncation is available beside it (the "full" one: every output
 * order keeps every moment |beta| <= 3, derivatives to order 6), with the
 * derivatives from the general closed form of d^gamma(1/r).
 *
 * Pins (tests/test_oracle_*.py): closed forms of G against symbolic
 * differentiation, Laplace trace identities, the lattice-point count of the
 * stencil, single-source closed forms, direct summation over point masses
 * with the error shrinking at the rate of the omitted order, eight symmetric
 * children = monopole, Newton's third law, translation and reflection
 * symmetry, 30-digit evaluation, and for the adjoint: dot-product test,
 * complex-step derivatives and translation invariance.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NM 20  /* moments / outputs, |beta| <= 3 */
#define NG3 20 /* derivatives up to order 3 */
#define NG 35  /* derivatives up to order 4 */
#define SUB 8
#define SUB3 512
#define HALO 24
#define HALO3 13824

/* ---------------------------------------------------------------------------
 * Multi-index bookkeeping (enumerated at start-up, graded lexicographic)
 * ------------------------------------------------------------------------- */
static int g_exp[NG][3];
static int g_ord[NG];
static int g_nax[NG], g_ax[NG][4];
static int g_sum[NG][NG];    /* index of gamma + delta, -1 if the order exceeds 4 */
static double g_tsign[NG];   /* s_beta = (-1)^{|beta|} / beta! */
static int g_ready = 0;

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

static int find_index(int a, int b, int c)
{
    for (int g = 0; g < NG; ++g)
        if (g_exp[g][0] == a && g_exp[g][1] == b && g_exp[g][2] == c) return g;
    return -1;
}

static void init_tables(void)
{
    if (g_ready) return;
    int k = 0;
    for (int n = 0; n <= 4; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                g_exp[k][0] = a;
                g_exp[k][1] = b;
                g_exp[k][2] = n - a - b;
                ++k;
            }
    for (int g = 0; g < NG; ++g) {
        g_ord[g] = g_exp[g][0] + g_exp[g][1] + g_exp[g][2];
        /* axis list, e.g. xxy -> {0,0,1} */
        int m = 0;
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e < g_exp[g][d]; ++e) g_ax[g][m++] = d;
        g_nax[g] = m;
        double bf = factorial(g_exp[g][0]) * factorial(g_exp[g][1]) * factorial(g_exp[g][2]);
        g_tsign[g] = ((g_ord[g] % 2) ? -1.0 : 1.0) / bf;
    }
    for (int g = 0; g < NG; ++g)
        for (int h = 0; h < NG; ++h)
            g_sum[g][h] = find_index(g_exp[g][0] + g_exp[h][0], g_exp[g][1] + g_exp[h][1],
                                     g_exp[g][2] + g_exp[h][2]);
    g_ready = 1;
}

static int ncomp(int order) { return (order + 1) * (order + 2) * (order + 3) / 6; }
static int order_of(int g) { return g_ord[g]; }
static int index_of(int a, int b, int c) { return find_index(a, b, c); }
static int sum_index(int g, int h) { return g_sum[g][h]; }
static double taylor_sign(int g) { return g_tsign[g]; }

/* axis list of component g; returns its length */
static int axes_of(int g, int ax[4])
{
    for (int m = 0; m < g_nax[g]; ++m) ax[m] = g_ax[g][m];
    return g_nax[g];
}

static double delta(int a, int b) { return a == b ? 1.0 : 0.0; }

/* ---------------------------------------------------------------------------
 * Opening criterion on integer halo-block coordinates (all >= 0)
 * ------------------------------------------------------------------------- */
static int in_stencil(const int hi[3], const int hj[3])
{
    int d2 = 0, p2 = 0;
    for (int k = 0; k < 3; ++k) {
        int d = hj[k] - hi[k];
        int p = hj[k] / 2 - hi[k] / 2;
        d2 += d * d;
        p2 += p * p;
    }
    return d2 > 16 && p2 <= 16;
}

/* slot = sx + 3 sy + 9 sz, s in {0,1,2} <-> neighbour offset -1, 0, +1 */
static void slot_coords(int slot, int s[3])
{
    s[0] = slot % 3;
    s[1] = (slot / 3) % 3;
    s[2] = slot / 9;
}

static void local_coords(int c, int l[3])
{
    l[0] = c % SUB;
    l[1] = (c / SUB) % SUB;
    l[2] = c / (SUB * SUB);
}

/* ---------------------------------------------------------------------------
 * "Full" truncation, the variant beside the total-order one: every output
 * order |alpha| <= 3 keeps every source moment |beta| <= 3, so derivatives of
 * G are needed to order 6:
 *   L_alpha(i) = sum_{j in S(i)} sum_{|beta| <= 3} s_beta M_beta(j) G_{alpha+beta}(X_i - X_j)
 * Derivatives of any order come from the general closed form of d^gamma (1/r)
 * (Hobson's formula), independent of the Kronecker-delta forms above: for
 * gamma = (a, b, c), n = a + b + c,
 *   d^gamma (1/r) = sum_{i <= a/2, j <= b/2, k <= c/2}
 *       (-1)^(n-m) (2n-2m-1)!! r^-(2n-2m+1) h(a,i) h(b,j) h(c,k) x^(a-2i) y^(b-2j) z^(c-2k),
 *   m = i + j + k,  h(a,i) = a! / (2^i i! (a-2i)!),  (-1)!! = 1,
 * and G_gamma = -d^gamma (1/r).
 * ------------------------------------------------------------------------- */
#define NGA 120 /* derivatives up to order 7 (the full truncation and its adjoint) */
static int g6_exp[NGA][3];
static int g6_sum[NM][NM]; /* index of alpha + beta among the NGA */
/* the terms of the closed form of each derivative, tabulated once:
 * coefficient, power of 1/r, powers of x, y, z (in the order i, j, k) */
#define MAXTERMS 16
static int g6_nterm[NGA];
static double g6_coef[NGA][MAXTERMS];
static int g6_pow[NGA][MAXTERMS][4];
static int g6_ready = 0;
static double double_factorial(int n);
static double hobson_h(int a, int i);

static void init_tables6(void)
{
    if (g6_ready) return;
    init_tables();
    int k = 0;
    for (int n = 0; n <= 7; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                g6_exp[k][0] = a;
                g6_exp[k][1] = b;
                g6_exp[k][2] = n - a - b;
                ++k;
            }
    for (int g = 0; g < NM; ++g)
        for (int h = 0; h < NM; ++h) {
            int e[3] = {g_exp[g][0] + g_exp[h][0], g_exp[g][1] + g_exp[h][1], g_exp[g][2] + g_exp[h][2]};
            g6_sum[g][h] = -1;
            for (int q = 0; q < NGA; ++q)
                if (g6_exp[q][0] == e[0] && g6_exp[q][1] == e[1] && g6_exp[q][2] == e[2]) g6_sum[g][h] = q;
        }
    for (int g = 0; g < NGA; ++g) {
        int a = g6_exp[g][0], b = g6_exp[g][1], c = g6_exp[g][2], n = a + b + c, t = 0;
        for (int i = 0; 2 * i <= a; ++i)
            for (int j = 0; 2 * j <= b; ++j)
                for (int k = 0; 2 * k <= c; ++k) {
                    int m = i + j + k;
                    g6_coef[g][t] = (((n - m) & 1) ? -1.0 : 1.0) * double_factorial(2 * n - 2 * m - 1) *
                                    hobson_h(a, i) * hobson_h(b, j) * hobson_h(c, k);
                    g6_pow[g][t][0] = 2 * n - 2 * m + 1;
                    g6_pow[g][t][1] = a - 2 * i;
                    g6_pow[g][t][2] = b - 2 * j;
                    g6_pow[g][t][3] = c - 2 * k;
                    ++t;
                }
        g6_nterm[g] = t;
    }
    g6_ready = 1;
}

static double double_factorial(int n)
{
    double f = 1.0;
    for (int k = n; k > 1; k -= 2) f *= k;
    return f;
}

static double hobson_h(int a, int i) { return factorial(a) / (ldexp(1.0, i) * factorial(i) * factorial(a - 2 * i)); }

/* index of the exponent (a, b, c) in the graded-lex enumeration */
static int gidx(int a, int b, int c)
{
    int n = a + b + c, k = n > 0 ? ncomp(n - 1) : 0;
    for (int ap = n; ap > a; --ap) k += n - ap + 1;
    return k + (n - a) - b;
}

/* ---------------------------------------------------------------------------
 * Scalar-generic core: real and complex instantiations
 * ------------------------------------------------------------------------- */
#define SC double
#define SQRT sqrt
#define FN(x) x##_re
#define cabs_generic(v) fabs(v)
#include "core.inc"
#undef SC
#undef SQRT
#undef FN
#undef cabs_generic

#define SC double _Complex
#define SQRT csqrt
#define FN(x) x##_cx
#define cabs_generic(v) cabs(v)
#include "core.inc"
#undef SC
#undef SQRT
#undef FN
#undef cabs_generic

static void pair_forward_any(int full, const double Xi[3], const double Xj[3], const double *Mj, int nm,
                             int mmax, double *L, double *Aabs)
{
    if (full)
        pair_forward_full_re(Xi, Xj, Mj, nm, mmax, L, Aabs);
    else
        pair_forward_re(Xi, Xj, Mj, nm, mmax, L, Aabs);
}

/* nthreads > 0: that many threads for this call; 0: the process default
 * (OMP_NUM_THREADS or all cores), also after a call that asked for fewer. */
static int g_default_threads = 0;

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (g_default_threads == 0) g_default_threads = omp_get_max_threads();
    omp_set_num_threads(nthreads > 0 ? nthreads : g_default_threads);
#else
    (void)nthreads;
#endif
}

/* ---------------------------------------------------------------------------
 * Exported helpers (for the pins)
 * ------------------------------------------------------------------------- */
void orc_multi_index(int g, int out[3])
{
    init_tables();
    out[0] = g_exp[g][0];
    out[1] = g_exp[g][1];
    out[2] = g_exp[g][2];
}

void orc_green(const double r[3], int order, double *G)
{
    init_tables();
    green_re(r, order, G);
}

int orc_in_stencil(const int hi[3], const int hj[3]) { return in_stencil(hi, hj); }

/* G_gamma for |gamma| <= order (order <= 7) from the general closed form. */
int orc_green_general(const double r[3], int order, double *G)
{
    if (order < 0 || order > 7) return -1;
    init_tables6();
    green_general_re(r, order, G);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return g_default_threads ? g_default_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Single sub-grid form: 24^3 halo block, SoA, cell index x + 24 y + 576 z.
 * M[nm][13824] raw moments (nm = 1: monopole masses, nm = 20: moments up to
 * order 3), X[3][13824] centres of mass; L[20][512] for the central 8^3
 * (index x + 8 y + 64 z). All halo cells are available.
 * ------------------------------------------------------------------------- */
static int block_forward(int full, const double *M, int nm, const double *X, int mmax, double *L,
                         double *Aabs, int nthreads)
{
    init_tables();
    init_tables6();
    if (nm != 1 && nm != NM) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
    for (int ci = 0; ci < SUB3; ++ci) {
        int li[3];
        local_coords(ci, li);
        int hi[3] = {li[0] + 8, li[1] + 8, li[2] + 8};
        int iidx = hi[0] + HALO * hi[1] + HALO * HALO * hi[2];
        double Xi[3] = {X[iidx], X[HALO3 + iidx], X[2 * HALO3 + iidx]};
        double acc[NM] = {0};
        double aabs[NM] = {0};
        for (int jz = 0; jz < HALO; ++jz)
            for (int jy = 0; jy < HALO; ++jy)
                for (int jx = 0; jx < HALO; ++jx) {
                    int hj[3] = {jx, jy, jz};
                    if (!in_stencil(hi, hj)) continue;
                    int jidx = jx + HALO * jy + HALO * HALO * jz;
                    double Xj[3] = {X[jidx], X[HALO3 + jidx], X[2 * HALO3 + jidx]};
                    double Mj[NM];
                    for (int b = 0; b < nm; ++b) Mj[b] = M[(size_t)b * HALO3 + jidx];
                    pair_forward_any(full, Xi, Xj, Mj, nm, mmax, acc, Aabs ? aabs : NULL);
                }
        for (int a = 0; a < NM; ++a) {
            L[a * SUB3 + ci] = acc[a];
            if (Aabs) Aabs[a * SUB3 + ci] = aabs[a];
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Batched form (store of S sub-grids, T targets).
 *   M[20][S*512], X[3][S*512]: cell c of store sub-grid s at s*512 + c.
 *   tgt[T]: store id of each target; nbr[T][27]: store id of the sub-grid in
 *   each neighbour slot (slot 13 = the target itself), -1 = not available
 *   (pairs with sources there are dropped).
 *   shift[T][27][3] (may be NULL): periodic image shift of the neighbour, in
 *   units of period[3]; the source centre used is X_j + shift * period.
 * Outputs are compact over a selection tsel[nsel] of target indices:
 *   L[20][nsel*512].
 * ------------------------------------------------------------------------- */
static int check_batch(int S, int T, const int32_t *tgt, const int32_t *nbr)
{
    if (S <= 0 || T <= 0 || !tgt || !nbr) return -1;
    for (int t = 0; t < T; ++t) {
        if (tgt[t] < 0 || tgt[t] >= S) return -1;
        for (int s = 0; s < 27; ++s)
            if (nbr[t * 27 + s] < -1 || nbr[t * 27 + s] >= S) return -1;
        if (nbr[t * 27 + 13] != tgt[t]) return -1;
    }
    return 0;
}

static void neighbour_shift(const int8_t *shift, const double *period, int t, int slot,
                            double sh[3])
{
    for (int k = 0; k < 3; ++k)
        sh[k] = (shift && period) ? (double)shift[((size_t)t * 27 + slot) * 3 + k] * period[k]
                                  : 0.0;
}

static int batched_forward(int full, int S, int T, const int32_t *tgt, const int32_t *nbr,
                           const int8_t *shift, const double *period, const double *M,
                           const double *X, const int32_t *tsel, int nsel, double *L,
                           double *Aabs, int nthreads)
{
    init_tables();
    init_tables6();
    if (check_batch(S, T, tgt, nbr)) return -1;
    for (int q = 0; q < nsel; ++q)
        if (tsel[q] < 0 || tsel[q] >= T) return -1;
    const size_t NS = (size_t)S * SUB3;
    const size_t NO = (size_t)nsel * SUB3;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int q = 0; q < nsel; ++q)
        for (int ci = 0; ci < SUB3; ++ci) {
            int t = tsel[q];
            int li[3];
            local_coords(ci, li);
            int hi[3] = {li[0] + 8, li[1] + 8, li[2] + 8};
            size_t iidx = (size_t)tgt[t] * SUB3 + ci;
            double Xi[3] = {X[iidx], X[NS + iidx], X[2 * NS + iidx]};
            double acc[NM] = {0}, aabs[NM] = {0};
            for (int slot = 0; slot < 27; ++slot) {
                int blk = nbr[t * 27 + slot];
                if (blk < 0) continue;
                int so[3];
                slot_coords(slot, so);
                double sh[3];
                neighbour_shift(shift, period, t, slot, sh);
                for (int cj = 0; cj < SUB3; ++cj) {
                    int lj[3];
                    local_coords(cj, lj);
                    int hj[3] = {8 * so[0] + lj[0], 8 * so[1] + lj[1], 8 * so[2] + lj[2]};
                    if (!in_stencil(hi, hj)) continue;
                    size_t jidx = (size_t)blk * SUB3 + cj;
                    double Xj[3] = {X[jidx] + sh[0], X[NS + jidx] + sh[1],
                                    X[2 * NS + jidx] + sh[2]};
                    double Mj[NM];
                    for (int b = 0; b < NM; ++b) Mj[b] = M[b * NS + jidx];
                    pair_forward_any(full, Xi, Xj, Mj, NM, 3, acc, Aabs ? aabs : NULL);
                }
            }
            for (int a = 0; a < NM; ++a) {
                L[a * NO + (size_t)q * SUB3 + ci] = acc[a];
                if (Aabs) Aabs[a * NO + (size_t)q * SUB3 + ci] = aabs[a];
            }
        }
    return 0;
}

int orc_block_forward(const double *M, int nm, const double *X, int mmax, double *L,
                      double *Aabs, int nthreads)
{
    return block_forward(0, M, nm, X, mmax, L, Aabs, nthreads);
}

int orc_block_forward_full(const double *M, int nm, const double *X, int mmax, double *L,
                           double *Aabs, int nthreads)
{
    return block_forward(1, M, nm, X, mmax, L, Aabs, nthreads);
}

int orc_batched_forward(int S, int T, const int32_t *tgt, const int32_t *nbr,
                        const int8_t *shift, const double *period, const double *M,
                        const double *X, const int32_t *tsel, int nsel, double *L,
                        double *Aabs, int nthreads)
{
    return batched_forward(0, S, T, tgt, nbr, shift, period, M, X, tsel, nsel, L, Aabs, nthreads);
}

int orc_batched_forward_full(int S, int T, const int32_t *tgt, const int32_t *nbr,
                             const int8_t *shift, const double *period, const double *M,
                             const double *X, const int32_t *tsel, int nsel, double *L,
                             double *Aabs, int nthreads)
{
    return batched_forward(1, S, T, tgt, nbr, shift, period, M, X, tsel, nsel, L, Aabs, nthreads);
}

/* Target-side derivatives of the forward: the chain rule applied to the
 * definition of L_alpha(i) with respect to the target's own centre X_i only
 * (the sources' centres held fixed); d/dX_i,k of G_{alpha+beta}(X_i - X_j) is
 * G_{alpha+beta+e_k}(X_i - X_j), so
 *   D_{alpha,k}(i) = sum_{j in S(i)} sum_{|beta| <= 3-|alpha|}
 *                        s_beta M_beta(j) G_{alpha+beta+e_k}(X_i - X_j).
 * (Cell i is never one of its own sources, so this is the whole derivative of
 * L(i) with respect to X_i whenever i's sub-grid appears only in slot 13.)
 * Output D[20][3][nsel*512] for targets tsel; Aabs (may be NULL): the sums of
 * the magnitudes of the terms.
 * full != 0: the same derivatives of the full truncation's L (every
 * |beta| <= 3 for every |alpha| <= 3; derivatives of G to order 7). */
static void pair_tgrad(const double Xi[3], const double Xj[3], const double *Mj, double *D, double *Aabs)
{
    double r[3] = {Xi[0] - Xj[0], Xi[1] - Xj[1], Xi[2] - Xj[2]};
    double G[NG];
    green_re(r, 4, G);
    for (int a = 0; a < NM; ++a)
        for (int k = 0; k < 3; ++k)
            for (int b = 0; b < NM; ++b) {
                if (order_of(a) + order_of(b) > 3) continue;
                double term = taylor_sign(b) * Mj[b] * G[sum_index(sum_index(a, b), 1 + k)];
                D[a * 3 + k] += term;
                if (Aabs) Aabs[a * 3 + k] += fabs(term);
            }
}

static void pair_tgrad_full(const double Xi[3], const double Xj[3], const double *Mj, double *D, double *Aabs)
{
    double r[3] = {Xi[0] - Xj[0], Xi[1] - Xj[1], Xi[2] - Xj[2]};
    double G[NGA];
    green_general_re(r, 7, G);
    for (int a = 0; a < NM; ++a)
        for (int k = 0; k < 3; ++k)
            for (int b = 0; b < NM; ++b) {
                int e[3] = {g_exp[a][0] + g_exp[b][0], g_exp[a][1] + g_exp[b][1], g_exp[a][2] + g_exp[b][2]};
                e[k] += 1;
                double term = taylor_sign(b) * Mj[b] * G[gidx(e[0], e[1], e[2])];
                D[a * 3 + k] += term;
                if (Aabs) Aabs[a * 3 + k] += fabs(term);
            }
}

static int batched_forward_tgrad(int full, int S, int T, const int32_t *tgt, const int32_t *nbr,
                                 const int8_t *shift, const double *period, const double *M, const double *X,
                                 const int32_t *tsel, int nsel, double *D, double *Aabs, int nthreads)
{
    init_tables();
    init_tables6();
    if (check_batch(S, T, tgt, nbr)) return -1;
    for (int q = 0; q < nsel; ++q)
        if (tsel[q] < 0 || tsel[q] >= T) return -1;
    const size_t NS = (size_t)S * SUB3;
    const size_t NO = (size_t)nsel * SUB3;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int q = 0; q < nsel; ++q)
        for (int ci = 0; ci < SUB3; ++ci) {
            int t = tsel[q];
            int li[3];
            local_coords(ci, li);
            int hi[3] = {li[0] + 8, li[1] + 8, li[2] + 8};
            size_t iidx = (size_t)tgt[t] * SUB3 + ci;
            double Xi[3] = {X[iidx], X[NS + iidx], X[2 * NS + iidx]};
            double acc[NM * 3] = {0}, aabs[NM * 3] = {0};
            for (int slot = 0; slot < 27; ++slot) {
                int blk = nbr[t * 27 + slot];
                if (blk < 0) continue;
                int so[3];
                slot_coords(slot, so);
                double sh[3];
                neighbour_shift(shift, period, t, slot, sh);
                for (int cj = 0; cj < SUB3; ++cj) {
                    int lj[3];
                    local_coords(cj, lj);
                    int hj[3] = {8 * so[0] + lj[0], 8 * so[1] + lj[1], 8 * so[2] + lj[2]};
                    if (!in_stencil(hi, hj)) continue;
                    size_t jidx = (size_t)blk * SUB3 + cj;
                    double Xj[3] = {X[jidx] + sh[0], X[NS + jidx] + sh[1], X[2 * NS + jidx] + sh[2]};
                    double Mj[NM];
                    for (int b = 0; b < NM; ++b) Mj[b] = M[b * NS + jidx];
                    if (full)
                        pair_tgrad_full(Xi, Xj, Mj, acc, Aabs ? aabs : NULL);
                    else
                        pair_tgrad(Xi, Xj, Mj, acc, Aabs ? aabs : NULL);
                }
            }
            for (int a = 0; a < NM * 3; ++a) {
                D[a * NO + (size_t)q * SUB3 + ci] = acc[a];
                if (Aabs) Aabs[a * NO + (size_t)q * SUB3 + ci] = aabs[a];
            }
        }
    return 0;
}

int orc_batched_forward_tgrad(int S, int T, const int32_t *tgt, const int32_t *nbr, const int8_t *shift,
                              const double *period, const double *M, const double *X, const int32_t *tsel,
                              int nsel, double *D, double *Aabs, int nthreads)
{
    return batched_forward_tgrad(0, S, T, tgt, nbr, shift, period, M, X, tsel, nsel, D, Aabs, nthreads);
}

int orc_batched_forward_tgrad_full(int S, int T, const int32_t *tgt, const int32_t *nbr, const int8_t *shift,
                                   const double *period, const double *M, const double *X, const int32_t *tsel,
                                   int nsel, double *D, double *Aabs, int nthreads)
{
    return batched_forward_tgrad(1, S, T, tgt, nbr, shift, period, M, X, tsel, nsel, D, Aabs, nthreads);
}

/* Angular-momentum correction of the force (a reading; Sec. 2.1 cites the
 * FMM without its formulas). With the total-order truncation the pair energy
 *   e_ij = sum_{|a|+|b| <= 3} (M_a(i)/a!) s_b M_b(j) G_{a+b}(X_i - X_j)
 * is invariant under rotations of positions and moments together, so the
 * forces F_i = -dE/dX_i and the spin torques of the cells,
 *   tau_i,m = -sum_{|g| <= 2} eps_mnl (M_{g+e_n}(i)/g!) L_{g+e_l}(i),
 * balance: sum_i (X_i x F_i + tau_i) = 0, as sum_i F_i = 0. The force
 * evaluated from L alone, -sum_{|a| <= 2} (M_a/a!) L_{a+e_k}, is the gradient
 * of the energy truncated one order lower and misses the terms of
 * -dE/dX_i with |a| + |b| = 3; the correction adds them:
 *   dF_k(i) = -sum_{j in S(i)} sum_{|a|+|b| = 3} (M_a(i)/a!) s_b M_b(j) G_{a+b+e_k}(X_i - X_j).
 * Output dF[3][nsel*512] for targets tsel; Aabs (may be NULL): the sums of the
 * magnitudes of the terms. */
static double multi_factorial(int g) { return factorial(g_exp[g][0]) * factorial(g_exp[g][1]) * factorial(g_exp[g][2]); }

static void pair_amc(const double Xi[3], const double *Mi, const double Xj[3], const double *Mj, double *dF,
                     double *Aabs)
{
    double r[3] = {Xi[0] - Xj[0], Xi[1] - Xj[1], Xi[2] - Xj[2]};
    double G[NG];
    green_re(r, 4, G);
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < NM; ++a)
            for (int b = 0; b < NM; ++b) {
                if (order_of(a) + order_of(b) != 3) continue;
                double ma = Mi[a] / multi_factorial(a); /* M_a / a! */
                double term = -ma * taylor_sign(b) * Mj[b] * G[sum_index(sum_index(a, b), 1 + k)];
                dF[k] += term;
                if (Aabs) Aabs[k] += fabs(term);
            }
}

int orc_batched_forward_amc(int S, int T, const int32_t *tgt, const int32_t *nbr, const int8_t *shift,
                            const double *period, const double *M, const double *X, const int32_t *tsel,
                            int nsel, double *dF, double *Aabs, int nthreads)
{
    init_tables();
    if (check_batch(S, T, tgt, nbr)) return -1;
    for (int q = 0; q < nsel; ++q)
        if (tsel[q] < 0 || tsel[q] >= T) return -1;
    const size_t NS = (size_t)S * SUB3;
    const size_t NO = (size_t)nsel * SUB3;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int q = 0; q < nsel; ++q)
        for (int ci = 0; ci < SUB3; ++ci) {
            int t = tsel[q];
            int li[3];
            local_coords(ci, li);
            int hi[3] = {li[0] + 8, li[1] + 8, li[2] + 8};
            size_t iidx = (size_t)tgt[t] * SUB3 + ci;
            double Xi[3] = {X[iidx], X[NS + iidx], X[2 * NS + iidx]};
            double Mi[NM];
            for (int a = 0; a < NM; ++a) Mi[a] = M[a * NS + iidx];
            double acc[3] = {0}, aabs[3] = {0};
            for (int slot = 0; slot < 27; ++slot) {
                int blk = nbr[t * 27 + slot];
                if (blk < 0) continue;
                int so[3];
                slot_coords(slot, so);
                double sh[3];
                neighbour_shift(shift, period, t, slot, sh);
                for (int cj = 0; cj < SUB3; ++cj) {
                    int lj[3];
                    local_coords(cj, lj);
                    int hj[3] = {8 * so[0] + lj[0], 8 * so[1] + lj[1], 8 * so[2] + lj[2]};
                    if (!in_stencil(hi, hj)) continue;
                    size_t jidx = (size_t)blk * SUB3 + cj;
                    double Xj[3] = {X[jidx] + sh[0], X[NS + jidx] + sh[1], X[2 * NS + jidx] + sh[2]};
                    double Mj[NM];
                    for (int b = 0; b < NM; ++b) Mj[b] = M[b * NS + jidx];
                    pair_amc(Xi, Mi, Xj, Mj, acc, Aabs ? aabs : NULL);
                }
            }
            for (int k = 0; k < 3; ++k) {
                dF[k * NO + (size_t)q * SUB3 + ci] = acc[k];
                if (Aabs) Aabs[k * NO + (size_t)q * SUB3 + ci] = aabs[k];
            }
        }
    return 0;
}

/* Coarse substitute for missing neighbours -- a reading: the paper gives no
 * FMM formulas; at a refinement boundary an FMM lets fine cells interact with
 * the coarser cells that cover a region holding no fine cells.
 * For target t and a slot s whose fine sub-grid is missing, coarse[t][s] is
 * the parent-level node P and octant[t][s] = o the octant of P that covers
 * the missing block (halo cells 8 s_k .. 8 s_k + 7 per axis). Its 4^3 coarse
 * cells J are the parents of the 2x2x2 fine cells j = 8 s_k + 2 J_k + {0, 1}.
 * Target cell i interacts with J iff all 8 of those fine cells are in S(i);
 * J then stands in for them, with its own moments about its own centre:
 *   L_a(i) += sum_{|b| <= 3-|a|} s_b M_b(J) G_{a+b}(X_i - X_J - shift(t, s)).
 * A J with some child near i is left out, like every near pair.
 * Mp[20][Sp*512], Xp[3][Sp*512]: coarse store; coarse cell (cx, cy, cz) of
 * octant o is cell (cx + 4 o_x) + 8 (cy + 4 o_y) + 64 (cz + 4 o_z) of P.
 * Returns the coarse contributions only, L (20, nsel*512), for targets tsel.
 * full != 0: the same substitute under the full truncation (every |b| <= 3
 * for every |a| <= 3), as in the full batched forward. */
static int coarse_fine(int full, int S, int T, const int32_t *tgt, const int32_t *nbr,
                       const int8_t *shift, const double *period, const double *X, int Sp,
                       const int32_t *coarse, const int8_t *octant, const double *Mp,
                       const double *Xp, const int32_t *tsel, int nsel, double *L,
                       double *Aabs, int nthreads)
{
    init_tables();
    init_tables6();
    if (check_batch(S, T, tgt, nbr) || Sp <= 0 || !coarse || !octant) return -1;
    for (int t = 0; t < T; ++t)
        for (int s = 0; s < 27; ++s) {
            int c = coarse[t * 27 + s];
            if (c < -1 || c >= Sp) return -1;
            if (c >= 0 && (s == 13 || nbr[t * 27 + s] >= 0)) return -1;
            if (c >= 0 && (octant[t * 27 + s] < 0 || octant[t * 27 + s] > 7)) return -1;
        }
    for (int q = 0; q < nsel; ++q)
        if (tsel[q] < 0 || tsel[q] >= T) return -1;
    const size_t NS = (size_t)S * SUB3, NP = (size_t)Sp * SUB3, NO = (size_t)nsel * SUB3;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int q = 0; q < nsel; ++q)
        for (int ci = 0; ci < SUB3; ++ci) {
            int t = tsel[q];
            int li[3];
            local_coords(ci, li);
            int hi[3] = {li[0] + 8, li[1] + 8, li[2] + 8};
            size_t iidx = (size_t)tgt[t] * SUB3 + ci;
            double Xi[3] = {X[iidx], X[NS + iidx], X[2 * NS + iidx]};
            double acc[NM] = {0}, aabs[NM] = {0};
            for (int slot = 0; slot < 27; ++slot) {
                int P = coarse[t * 27 + slot];
                if (P < 0) continue;
                int o = octant[t * 27 + slot], so[3];
                slot_coords(slot, so);
                double sh[3];
                neighbour_shift(shift, period, t, slot, sh);
                for (int J = 0; J < 64; ++J) {
                    int cj[3] = {J % 4, (J / 4) % 4, J / 16};
                    int all_in = 1;
                    for (int n = 0; n < 8 && all_in; ++n) {
                        int hj[3] = {8 * so[0] + 2 * cj[0] + (n & 1), 8 * so[1] + 2 * cj[1] + ((n >> 1) & 1),
                                     8 * so[2] + 2 * cj[2] + (n >> 2)};
                        all_in = in_stencil(hi, hj);
                    }
                    if (!all_in) continue;
                    int pc = (cj[0] + 4 * (o & 1)) + SUB * (cj[1] + 4 * ((o >> 1) & 1)) +
                             SUB * SUB * (cj[2] + 4 * (o >> 2));
                    size_t jidx = (size_t)P * SUB3 + pc;
                    double Xj[3] = {Xp[jidx] + sh[0], Xp[NP + jidx] + sh[1], Xp[2 * NP + jidx] + sh[2]};
                    double Mj[NM];
                    for (int b = 0; b < NM; ++b) Mj[b] = Mp[b * NP + jidx];
                    pair_forward_any(full, Xi, Xj, Mj, NM, 3, acc, Aabs ? aabs : NULL);
                }
            }
            for (int a = 0; a < NM; ++a) {
                L[a * NO + (size_t)q * SUB3 + ci] = acc[a];
                if (Aabs) Aabs[a * NO + (size_t)q * SUB3 + ci] = aabs[a];
            }
        }
    return 0;
}

int orc_coarse_fine(int S, int T, const int32_t *tgt, const int32_t *nbr, const int8_t *shift,
                    const double *period, const double *X, int Sp, const int32_t *coarse,
                    const int8_t *octant, const double *Mp, const double *Xp,
                    const int32_t *tsel, int nsel, double *L, double *Aabs, int nthreads)
{
    return coarse_fine(0, S, T, tgt, nbr, shift, period, X, Sp, coarse, octant, Mp, Xp, tsel, nsel,
                       L, Aabs, nthreads);
}

int orc_coarse_fine_full(int S, int T, const int32_t *tgt, const int32_t *nbr,
                         const int8_t *shift, const double *period, const double *X, int Sp,
                         const int32_t *coarse, const int8_t *octant, const double *Mp,
                         const double *Xp, const int32_t *tsel, int nsel, double *L,
                         double *Aabs, int nthreads)
{
    return coarse_fine(1, S, T, tgt, nbr, shift, period, X, Sp, coarse, octant, Mp, Xp, tsel, nsel,
                       L, Aabs, nthreads);
}

/* Same sum with complex centres of mass X = Xre + i Xim (moments real), for
 * complex-step differentiation: d(sum w L)/dX_c,k = Im(sum w L(X + i h e_ck))/h. */
static int batched_forward_cs(int full, int S, int T, const int32_t *tgt, const int32_t *nbr,
                              const int8_t *shift, const double *period, const double *M,
                              const double *Xre, const double *Xim, const int32_t *tsel,
                              int nsel, double *Lre, double *Lim, int nthreads)
{
    init_tables();
    init_tables6();
    if (check_batch(S, T, tgt, nbr)) return -1;
    for (int q = 0; q < nsel; ++q)
        if (tsel[q] < 0 || tsel[q] >= T) return -1;
    const size_t NS = (size_t)S * SUB3;
    const size_t NO = (size_t)nsel * SUB3;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int q = 0; q < nsel; ++q)
        for (int ci = 0; ci < SUB3; ++ci) {
            int t = tsel[q];
            int li[3];
            local_coords(ci, li);
            int hi[3] = {li[0] + 8, li[1] + 8, li[2] + 8};
            size_t iidx = (size_t)tgt[t] * SUB3 + ci;
            double _Complex Xi[3];
            for (int k = 0; k < 3; ++k) Xi[k] = Xre[k * NS + iidx] + I * Xim[k * NS + iidx];
            double _Complex acc[NM];
            for (int a = 0; a < NM; ++a) acc[a] = 0;
            for (int slot = 0; slot < 27; ++slot) {
                int blk = nbr[t * 27 + slot];
                if (blk < 0) continue;
                int so[3];
                slot_coords(slot, so);
                double sh[3];
                neighbour_shift(shift, period, t, slot, sh);
                for (int cj = 0; cj < SUB3; ++cj) {
                    int lj[3];
                    local_coords(cj, lj);
                    int hj[3] = {8 * so[0] + lj[0], 8 * so[1] + lj[1], 8 * so[2] + lj[2]};
                    if (!in_stencil(hi, hj)) continue;
                    size_t jidx = (size_t)blk * SUB3 + cj;
                    double _Complex Xj[3];
                    for (int k = 0; k < 3; ++k)
                        Xj[k] = (Xre[k * NS + jidx] + sh[k]) + I * Xim[k * NS + jidx];
                    double Mj[NM];
                    for (int b = 0; b < NM; ++b) Mj[b] = M[b * NS + jidx];
                    if (full)
                        pair_forward_full_cx(Xi, Xj, Mj, NM, 3, acc, NULL);
                    else
                        pair_forward_cx(Xi, Xj, Mj, NM, 3, acc, NULL);
                }
            }
            for (int a = 0; a < NM; ++a) {
                Lre[a * NO + (size_t)q * SUB3 + ci] = creal(acc[a]);
                Lim[a * NO + (size_t)q * SUB3 + ci] = cimag(acc[a]);
            }
        }
    return 0;
}

int orc_batched_forward_cs(int S, int T, const int32_t *tgt, const int32_t *nbr,
                           const int8_t *shift, const double *period, const double *M,
                           const double *Xre, const double *Xim, const int32_t *tsel,
                           int nsel, double *Lre, double *Lim, int nthreads)
{
    return batched_forward_cs(0, S, T, tgt, nbr, shift, period, M, Xre, Xim, tsel, nsel, Lre, Lim, nthreads);
}

int orc_batched_forward_cs_full(int S, int T, const int32_t *tgt, const int32_t *nbr,
                                const int8_t *shift, const double *period, const double *M,
                                const double *Xre, const double *Xim, const int32_t *tsel,
                                int nsel, double *Lre, double *Lim, int nthreads)
{
    return batched_forward_cs(1, S, T, tgt, nbr, shift, period, M, Xre, Xim, tsel, nsel, Lre, Lim, nthreads);
}

/* ---------------------------------------------------------------------------
 * Adjoint of the batched form for the loss  l = sum_t sum_i sum_alpha
 * gL_alpha(t, i) L_alpha(t, i)  (gL[20][T*512] = dl/dL).
 *
 * For one pair (target i of target t, source j) with r = X_i - (X_j + shift):
 *   P = sum_{|a|+|b|<=3} w_a(i) s_b M_b(j) G_{a+b}(r)
 *   dP/dM_b(j) = s_b sum_{|a|<=3-|b|} w_a(i) G_{a+b}(r)
 *   dP/dX_i,k  = + sum_{a,b} w_a(i) s_b M_b(j) G_{a+b+e_k}(r)
 *   dP/dX_j,k  = - (same sum)
 * The gradients of a store cell c are the sums over every pair in which c is
 * the source and every pair in which c is the target. The loops below visit
 * those pairs from c's side (so that any subset of store sub-grids can be
 * evaluated on its own); the summand of each pair is the chain rule above.
 * Outputs are compact over a selection ssel[nsel] of store sub-grids:
 *   gM[20][nsel*512], gX[3][nsel*512].
 * ------------------------------------------------------------------------- */
static void pair_gradients(const double Xi[3], const double Xj[3], const double *w,
                           const double *Mj, double dM[NM], double dX[3])
{
    double r[3] = {Xi[0] - Xj[0], Xi[1] - Xj[1], Xi[2] - Xj[2]};
    double G[NG];
    green_re(r, 4, G);
    int ek[3] = {index_of(1, 0, 0), index_of(0, 1, 0), index_of(0, 0, 1)};
    for (int b = 0; b < NM; ++b) dM[b] = 0.0;
    dX[0] = dX[1] = dX[2] = 0.0;
    for (int a = 0; a < NM; ++a)
        for (int b = 0; b < NM; ++b) {
            if (order_of(a) + order_of(b) > 3) continue;
            int ab = sum_index(a, b);
            dM[b] += taylor_sign(b) * w[a] * G[ab];
            for (int k = 0; k < 3; ++k)
                dX[k] += w[a] * taylor_sign(b) * Mj[b] * G[sum_index(ab, ek[k])];
        }
}

/* The same with the full truncation (all |a|, |b| <= 3; G to order 7). */
static void pair_gradients_full(const double Xi[3], const double Xj[3], const double *w,
                                const double *Mj, double dM[NM], double dX[3])
{
    double r[3] = {Xi[0] - Xj[0], Xi[1] - Xj[1], Xi[2] - Xj[2]};
    double G[NGA];
    green_general_re(r, 7, G);
    for (int b = 0; b < NM; ++b) dM[b] = 0.0;
    dX[0] = dX[1] = dX[2] = 0.0;
    for (int a = 0; a < NM; ++a)
        for (int b = 0; b < NM; ++b) {
            int e[3] = {g_exp[a][0] + g_exp[b][0], g_exp[a][1] + g_exp[b][1], g_exp[a][2] + g_exp[b][2]};
            dM[b] += taylor_sign(b) * w[a] * G[gidx(e[0], e[1], e[2])];
            for (int k = 0; k < 3; ++k)
                dX[k] += w[a] * taylor_sign(b) * Mj[b] *
                         G[gidx(e[0] + (k == 0), e[1] + (k == 1), e[2] + (k == 2))];
        }
}

static int batched_backward(int full, int S, int T, const int32_t *tgt, const int32_t *nbr,
                            const int8_t *shift, const double *period, const double *M,
                            const double *X, const double *gL, const int32_t *ssel, int nsel,
                            double *gM, double *gX, int nthreads)
{
    init_tables();
    init_tables6();
    if (check_batch(S, T, tgt, nbr)) return -1;
    for (int q = 0; q < nsel; ++q)
        if (ssel[q] < 0 || ssel[q] >= S) return -1;
    const size_t NS = (size_t)S * SUB3;
    const size_t NT = (size_t)T * SUB3;
    const size_t NO = (size_t)nsel * SUB3;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < nsel; ++q) {
        int s = ssel[q];
        /* every (target, slot) that sees sub-grid s as a source, and every
         * target whose own sub-grid is s -- found by plain search */
        int nrel = 0, cap = 64;
        int *rel_t = malloc(sizeof(int) * cap), *rel_slot = malloc(sizeof(int) * cap);
        for (int t = 0; t < T; ++t)
            for (int slot = 0; slot < 27; ++slot)
                if (nbr[t * 27 + slot] == s) {
                    if (nrel == cap) {
                        cap *= 2;
                        rel_t = realloc(rel_t, sizeof(int) * cap);
                        rel_slot = realloc(rel_slot, sizeof(int) * cap);
                    }
                    rel_t[nrel] = t;
                    rel_slot[nrel] = slot;
                    ++nrel;
                }
        for (int cc = 0; cc < SUB3; ++cc) {
            int lc[3];
            local_coords(cc, lc);
            size_t cidx = (size_t)s * SUB3 + cc;
            double Xc[3] = {X[cidx], X[NS + cidx], X[2 * NS + cidx]};
            double Mc[NM];
            for (int b = 0; b < NM; ++b) Mc[b] = M[b * NS + cidx];
            double accM[NM] = {0}, accX[3] = {0, 0, 0};
            double dM[NM], dX[3], w[NM];
            /* (a) c as a source of target cells of target t, seen at `slot` */
            for (int e = 0; e < nrel; ++e) {
                int t = rel_t[e], slot = rel_slot[e];
                int so[3];
                slot_coords(slot, so);
                int hj[3] = {8 * so[0] + lc[0], 8 * so[1] + lc[1], 8 * so[2] + lc[2]};
                double sh[3];
                neighbour_shift(shift, period, t, slot, sh);
                double Xj[3] = {Xc[0] + sh[0], Xc[1] + sh[1], Xc[2] + sh[2]};
                for (int ci = 0; ci < SUB3; ++ci) {
                    int li[3];
                    local_coords(ci, li);
                    int hi[3] = {li[0] + 8, li[1] + 8, li[2] + 8};
                    if (!in_stencil(hi, hj)) continue;
                    size_t iidx = (size_t)tgt[t] * SUB3 + ci;
                    double Xi[3] = {X[iidx], X[NS + iidx], X[2 * NS + iidx]};
                    for (int a = 0; a < NM; ++a) w[a] = gL[a * NT + (size_t)t * SUB3 + ci];
                    if (full)
                        pair_gradients_full(Xi, Xj, w, Mc, dM, dX);
                    else
                        pair_gradients(Xi, Xj, w, Mc, dM, dX);
                    for (int b = 0; b < NM; ++b) accM[b] += dM[b];
                    for (int k = 0; k < 3; ++k) accX[k] -= dX[k];
                }
            }
            /* (b) c as a target cell of every target t whose sub-grid is s */
            for (int t = 0; t < T; ++t) {
                if (tgt[t] != s) continue;
                int hi[3] = {lc[0] + 8, lc[1] + 8, lc[2] + 8};
                for (int a = 0; a < NM; ++a) w[a] = gL[a * NT + (size_t)t * SUB3 + cc];
                for (int slot = 0; slot < 27; ++slot) {
                    int blk = nbr[t * 27 + slot];
                    if (blk < 0) continue;
                    int so[3];
                    slot_coords(slot, so);
                    double sh[3];
                    neighbour_shift(shift, period, t, slot, sh);
                    for (int cj = 0; cj < SUB3; ++cj) {
                        int lj[3];
                        local_coords(cj, lj);
                        int hj[3] = {8 * so[0] + lj[0], 8 * so[1] + lj[1], 8 * so[2] + lj[2]};
                        if (!in_stencil(hi, hj)) continue;
                        size_t jidx = (size_t)blk * SUB3 + cj;
                        double Xj[3] = {X[jidx] + sh[0], X[NS + jidx] + sh[1],
                                        X[2 * NS + jidx] + sh[2]};
                        double Mj[NM];
                        for (int b = 0; b < NM; ++b) Mj[b] = M[b * NS + jidx];
                        if (full)
                            pair_gradients_full(Xc, Xj, w, Mj, dM, dX);
                        else
                            pair_gradients(Xc, Xj, w, Mj, dM, dX);
                        for (int k = 0; k < 3; ++k) accX[k] += dX[k];
                    }
                }
            }
            for (int b = 0; b < NM; ++b) gM[b * NO + (size_t)q * SUB3 + cc] = accM[b];
            for (int k = 0; k < 3; ++k) gX[k * NO + (size_t)q * SUB3 + cc] = accX[k];
        }
        free(rel_t);
        free(rel_slot);
    }
    return 0;
}

int orc_batched_backward(int S, int T, const int32_t *tgt, const int32_t *nbr,
                         const int8_t *shift, const double *period, const double *M,
                         const double *X, const double *gL, const int32_t *ssel, int nsel,
                         double *gM, double *gX, int nthreads)
{
    return batched_backward(0, S, T, tgt, nbr, shift, period, M, X, gL, ssel, nsel, gM, gX, nthreads);
}

int orc_batched_backward_full(int S, int T, const int32_t *tgt, const int32_t *nbr,
                              const int8_t *shift, const double *period, const double *M,
                              const double *X, const double *gL, const int32_t *ssel, int nsel,
                              double *gM, double *gX, int nthreads)
{
    return batched_backward(1, S, T, tgt, nbr, shift, period, M, X, gL, ssel, nsel, gM, gX, nthreads);
}

/* ---------------------------------------------------------------------------
 * Tree passes around the interaction (paper Sec. 2.1: the FMM works on the
 * octree; Sec. 2.3: the gravity solver traverses the tree of sub-grids).
 * A parent node p and its 8 child nodes children[p][o] (o = ox + 2 oy + 4 oz)
 * hold 8^3 cells each; parent cell (X, Y, Z) covers the 2x2x2 child cells
 * (2 (X % 4) + a, 2 (Y % 4) + b, 2 (Z % 4) + c) of child node o = (X/4, Y/4, Z/4).
 * ------------------------------------------------------------------------- */
static double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

/* d^e = d_x^e_x d_y^e_y d_z^e_z */
static double mono(const double d[3], const int e[3])
{
    double v = 1.0;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < e[k]; ++i) v *= d[k];
    return v;
}

static void parent_children_cells(int pc, int child_local[8], int *octant)
{
    int lp[3];
    local_coords(pc, lp);
    *octant = lp[0] / 4 + 2 * (lp[1] / 4) + 4 * (lp[2] / 4);
    int n = 0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                int l[3] = {2 * (lp[0] % 4) + a, 2 * (lp[1] % 4) + b, 2 * (lp[2] % 4) + c};
                child_local[n++] = l[0] + SUB * l[1] + SUB * SUB * l[2];
            }
}

/* Upward pass (M2M; P2M when the children are point masses): the parent
 * cell's mass is the children's total, its centre the mass-weighted mean of
 * the children's centres (their plain mean if the total mass is 0), and its
 * raw moments about that centre follow from the children's by the binomial
 * expansion of (x - X_p)^b = ((x - X_c) + (X_c - X_p))^b:
 *   M_b(p) = sum_c sum_{g <= b} C(b, g) M_g(c) (X_c - X_p)^(b - g),
 * C(b, g) = prod_k binom(b_k, g_k). Exact for |b| <= 3 (no truncation).
 * Mc[20][Sc*512], Xc[3][Sc*512] -> Mp[20][nsel*512], Xp[3][nsel*512] over the
 * selected parent nodes psel. */
int orc_m2m(int Sp, int Sc, const int32_t *children, const double *Mc, const double *Xc,
            const int32_t *psel, int nsel, double *Mp, double *Xp, int nthreads)
{
    init_tables();
    if (Sp <= 0 || Sc <= 0 || !children) return -1;
    for (int i = 0; i < Sp * 8; ++i)
        if (children[i] < 0 || children[i] >= Sc) return -1;
    for (int q = 0; q < nsel; ++q)
        if (psel[q] < 0 || psel[q] >= Sp) return -1;
    const size_t NC = (size_t)Sc * SUB3, NO = (size_t)nsel * SUB3;
    set_threads(nthreads);
#pragma omp parallel for schedule(static) collapse(2)
    for (int q = 0; q < nsel; ++q)
        for (int pc = 0; pc < SUB3; ++pc) {
            int p = psel[q], cl[8], o;
            parent_children_cells(pc, cl, &o);
            int blk = children[p * 8 + o];
            double m = 0.0, mx[3] = {0, 0, 0}, gx[3] = {0, 0, 0};
            for (int n = 0; n < 8; ++n) {
                size_t j = (size_t)blk * SUB3 + cl[n];
                m += Mc[j];
                for (int k = 0; k < 3; ++k) {
                    mx[k] += Mc[j] * Xc[k * NC + j];
                    gx[k] += Xc[k * NC + j];
                }
            }
            double X[3];
            for (int k = 0; k < 3; ++k) X[k] = m > 0.0 ? mx[k] / m : gx[k] / 8.0;
            double acc[NM] = {0};
            for (int n = 0; n < 8; ++n) {
                size_t j = (size_t)blk * SUB3 + cl[n];
                double d[3] = {Xc[j] - X[0], Xc[NC + j] - X[1], Xc[2 * NC + j] - X[2]};
                for (int b = 0; b < NM; ++b)
                    for (int g = 0; g < NM; ++g) {
                        int ok = 1, e[3];
                        double c = 1.0;
                        for (int k = 0; k < 3; ++k) {
                            e[k] = g_exp[b][k] - g_exp[g][k];
                            if (e[k] < 0) ok = 0;
                            else c *= binom(g_exp[b][k], g_exp[g][k]);
                        }
                        if (!ok) continue;
                        acc[b] += c * Mc[g * NC + j] * mono(d, e);
                    }
            }
            for (int b = 0; b < NM; ++b) Mp[b * NO + (size_t)q * SUB3 + pc] = acc[b];
            for (int k = 0; k < 3; ++k) Xp[k * NO + (size_t)q * SUB3 + pc] = X[k];
        }
    return 0;
}

/* Downward pass (L2L): the parent cell's local expansion
 *   phi(x) = sum_a L_a(p) (x - X_p)^a / a!
 * is re-expanded about each child cell's centre and kept to order 3:
 *   L_a(c) += sum_{|g| <= 3 - |a|} L_{a+g}(p) (X_c - X_p)^g / g!
 * (exact for the cubic phi). Lp[20][Sp*512], Xp[3][Sp*512], Xc[3][Sc*512];
 * Lc[20][Sc*512] is accumulated into for every child node of a parent. */
int orc_l2l(int Sp, int Sc, const int32_t *children, const double *Lp, const double *Xp,
            const double *Xc, double *Lc, int nthreads)
{
    init_tables();
    if (Sp <= 0 || Sc <= 0 || !children) return -1;
    for (int i = 0; i < Sp * 8; ++i)
        if (children[i] < 0 || children[i] >= Sc) return -1;
    const size_t NC = (size_t)Sc * SUB3, NP = (size_t)Sp * SUB3;
    set_threads(nthreads);
#pragma omp parallel for schedule(static) collapse(2)
    for (int p = 0; p < Sp; ++p)
        for (int pc = 0; pc < SUB3; ++pc) {
            int cl[8], o;
            parent_children_cells(pc, cl, &o);
            int blk = children[p * 8 + o];
            size_t ip = (size_t)p * SUB3 + pc;
            for (int n = 0; n < 8; ++n) {
                size_t j = (size_t)blk * SUB3 + cl[n];
                double d[3] = {Xc[j] - Xp[ip], Xc[NC + j] - Xp[NP + ip], Xc[2 * NC + j] - Xp[2 * NP + ip]};
                for (int a = 0; a < NM; ++a) {
                    double s = 0.0;
                    for (int g = 0; g < NM; ++g) {
                        if (order_of(a) + order_of(g) > 3) continue;
                        s += Lp[sum_index(a, g) * NP + ip] * mono(d, g_exp[g]) /
                             (factorial(g_exp[g][0]) * factorial(g_exp[g][1]) * factorial(g_exp[g][2]));
                    }
                    Lc[a * NC + j] += s;
                }
            }
        }
    return 0;
}

/* Local evaluation of a cell from its moments M (about its centre) and its
 * local expansion L (about the same centre):
 *   force      F_k = - sum_{|a| <= 2} M_a / a! L_{a+e_k}
 *   energy     W   = 1/2 sum_{|a| <= 3} M_a / a! L_a
 * (the integrals of -rho grad(phi) and rho phi / 2 over the cell's mass, with
 * phi truncated at order 3). M, L [20][N] -> F[3][N], W[N]. */
int orc_evaluate(long N, const double *M, const double *L, double *F, double *W, int nthreads)
{
    init_tables();
    if (N <= 0) return -1;
    int ek[3] = {index_of(1, 0, 0), index_of(0, 1, 0), index_of(0, 0, 1)};
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        double f[3] = {0, 0, 0}, w = 0.0;
        for (int a = 0; a < NM; ++a) {
            double ma = M[a * N + i] /
                        (factorial(g_exp[a][0]) * factorial(g_exp[a][1]) * factorial(g_exp[a][2]));
            w += 0.5 * ma * L[a * N + i];
            if (order_of(a) <= 2)
                for (int k = 0; k < 3; ++k) f[k] -= ma * L[sum_index(a, ek[k]) * N + i];
        }
        for (int k = 0; k < 3; ++k) F[k * N + i] = f[k];
        W[i] = w;
    }
    return 0;
}
