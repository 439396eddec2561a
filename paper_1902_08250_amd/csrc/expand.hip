// FMM passes on the uniform interface-split quadtree (Algorithm 1, Steps 2-4).
//
//  * P2M  (source-to-multipole, Definition "Multipole Expansion"): per source
//    leaf, M_q = sum_j q_j J_q(k1 r_j) e^{-i q theta_j}, stored scaled.
//  * M2M  (Lemma M2M): free-space Helmholtz shift with k1, 4 children -> parent.
//  * M2L (Lemma M2L): at every level in one launch, each target box in the
//    two rows nearest the interface (every row at the coarsest level) gathers
//    its interaction list through the Sommerfeld translation tables.
//  * L2L (Lemma L2L): level by level, every target box receives its parent's
//    local expansion shifted with the free-space operator for k2, plus its own
//    M2L result.
//  * L2P + S2T (Definition "Local Expansion"; direct interactions): per
//    target leaf, the leaf's L2L shift, then the local expansion evaluated at
//    the targets, plus the direct interactions of the adjacent source leaves
//    across the interface (contour quadrature of g_2^t, by sweeps or pairs).
//
// Expansions are stored scaled: Mhat_q = s_q M_q and Lhat_p = L_p / s_p with
// s_q = |q|! (2/(k R))^|q|, R the box half-diagonal, which keeps FP32 in
// range.  Layout: [box][rhs][2P+1] complex, box = row * ncol + column.
#include "lmfmm_internal.h"
#include "cexp_tab.h"

#include <atomic>

namespace lmfmm {

namespace {

// ---------------------------------------------------------------------------
// P2M: a block takes G consecutive source leaves, whose points are contiguous
// in the grouped order (as are their densities, qs), and walks those points in
// chunks of CH: a thread per point evaluates the point's scaled basis into
// LDS, then threads over (leaf, right-hand side, coefficient) add the points
// of their leaf in the chunk, in index order.  The output block of the G leaves is contiguous, and
// so are the threads' stores.  Leaves without points get zeros.
// ---------------------------------------------------------------------------
constexpr int P2M_THREADS = 256;
constexpr int P2M_CHMAX = 320;  // points per chunk (a thread evaluates up to two)
constexpr int LEAF_GMAX = 32;  // leaves per block (P2M and L2P)
template <typename T, int PMAX>
__global__ void __launch_bounds__(P2M_THREADS) k_p2m(const int32_t *__restrict__ start,
                                                     const int32_t *__restrict__ end, const double *__restrict__ xs,
                                                     const double *__restrict__ ys, const cx<T> *__restrict__ qs,
                                                     int64_t ns, int nrhs, int P, int nbox, int ncol, int col_lo,
                                                     double x_lo, double w, cx<T> k1, T invR, int G, int CH,
                                                     cx<T> *__restrict__ M)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ int bnd[LEAF_GMAX + 1];
    const int nc = 2 * P + 1;
    cx<T> *B = reinterpret_cast<cx<T> *>(smem_raw);  // [CH][nc]
    cx<T> *Q = B + CH * nc;                          // [CH][nrhs]
    const int t = threadIdx.x;
    const int b0 = blockIdx.x * G;
    const int ng = nbox - b0 < G ? nbox - b0 : G;
    if (t <= ng) bnd[t] = t < ng ? start[b0 + t] : end[b0 + ng - 1];
    __syncthreads();
    const int S = bnd[0], E = bnd[ng];
    const int nout = nc * nrhs, nitem = ng * nout;
    cx<T> *Mb = M + (int64_t)b0 * nout;
    for (int c0 = S; c0 < E || c0 == S; c0 += CH) {
        for (int jl = t; jl < CH; jl += P2M_THREADS) {
            const int j = c0 + jl;
            if (j >= E) break;
            int g = 0;
            while (j >= bnd[g + 1]) ++g;
            const int box = b0 + g;
            const int row = box / ncol, col = col_lo + box % ncol;
            const double cxp = x_lo + (col + 0.5) * w, cyp = (row + 0.5) * w;
            const T X = (T)(xs[j] - cxp), Y = (T)(ys[j] - cyp);
            bessel_basis<T, PMAX>(k1, X, Y, invR, P, -1, B + jl * nc, 1);
            for (int r = 0; r < nrhs; ++r) Q[jl * nrhs + r] = qs[(int64_t)r * ns + j];
        }
        __syncthreads();
        const int cend = E - c0 < CH ? E : c0 + CH;
        for (int it = t; it < nitem; it += P2M_THREADS) {
            const int g = it / nout, o = it - g * nout;
            const int r = o / nc, c = o - r * nc;
            const int j0 = bnd[g] > c0 ? bnd[g] : c0, j1 = bnd[g + 1] < cend ? bnd[g + 1] : cend;
            // in increasing point order; four points' LDS reads issued together
            const cx<T> *bp = B + (j0 - c0) * nc + c, *qp = Q + (j0 - c0) * nrhs + r;
            const int np = j1 - j0;
            cx<T> acc = mk<T>(0, 0);
            int jj = 0;
            for (; jj + 4 <= np; jj += 4) {
                const cx<T> b0 = bp[jj * nc], b1 = bp[(jj + 1) * nc], b2 = bp[(jj + 2) * nc], b3 = bp[(jj + 3) * nc];
                const cx<T> q0 = qp[jj * nrhs], q1 = qp[(jj + 1) * nrhs], q2 = qp[(jj + 2) * nrhs],
                            q3 = qp[(jj + 3) * nrhs];
                cfma(acc, b0, q0);
                cfma(acc, b1, q1);
                cfma(acc, b2, q2);
                cfma(acc, b3, q3);
            }
            for (; jj < np; ++jj) cfma(acc, bp[jj * nc], qp[jj * nrhs]);
            if (c0 == S)
                Mb[it] = acc;
            else if (j1 > j0)
                Mb[it] += acc;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Translations (Lemma M2M, Lemma M2L, Lemma L2L) as one matrix-vector product
// per (table, vector) item: out[p] += sum_k A[k][p] x[k], A a per-level table
// (M2M and L2L: one per child position; M2L: one per translation class) and
// x the expansion being translated.  A wave evaluates one item with lanes over
// the output coefficients p: it stages x in LDS and issues the loads of a
// whole K chunk of its table column at once, so an item costs about one
// memory round trip.  The waves of a block take the items of one output box
// in turn; their sums are added in wave order through LDS, so the result does
// not depend on scheduling.
// ---------------------------------------------------------------------------
template <typename T>
struct Tr {
    static constexpr int R = sizeof(T) == 4 ? 4 : 2;    // right-hand sides per pass
    static constexpr int KC = sizeof(T) == 4 ? 48 : 24;  // table rows loaded per round trip
};

// Per-wave LDS: x chunk [R][KC] and the wave's partial sums [R][64].
template <typename T>
struct WaveLds {
    cx<T> x[Tr<T>::R][Tr<T>::KC];
    cx<T> out[Tr<T>::R][64];
};

// acc[r] += sum_{k < nk} A[k * nout + p] x[r * xstride + k], p = p0 + lane,
// r < nr.  Every lane of the wave calls this with the same arguments.
template <typename T>
__device__ inline void item_matvec(const cx<T> *__restrict__ A, int nk, int nout, int p0,
                                   const cx<T> *__restrict__ x, int64_t xstride, int nr, WaveLds<T> &lds,
                                   cx<T> (&acc)[Tr<T>::R])
{
    constexpr int R = Tr<T>::R, KC = Tr<T>::KC;
    const int lane = threadIdx.x & 63;
    const int p = p0 + lane;
    const int pc = p < nout ? p : nout - 1;
    for (int k0 = 0; k0 < nk; k0 += KC) {
        const int kc = nk - k0 < KC ? nk - k0 : KC;
        // the table loads first, then the vector's: both round trips overlap
        cx<T> av[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int k = k0 + (j < kc ? j : kc - 1);
            av[j] = A[(int64_t)k * nout + pc];
        }
        cx<T> xv[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            xv[r] = (lane < kc && r < nr) ? x[r * xstride + k0 + lane] : mk<T>(0, 0);
        __builtin_amdgcn_wave_barrier();
        if (lane < KC)
#pragma unroll
            for (int r = 0; r < R; ++r) lds.x[r][lane] = xv[r];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j0 = 0; j0 < KC; j0 += 8) {
            if (j0 < kc) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (r < nr)
#pragma unroll
                        for (int j = j0; j < j0 + 8; ++j) cfma(acc[r], av[j], lds.x[r][j]);
            }
        }
    }
}

// Sum of the waves' partials in wave order by wave 0; writes out[r * ostride + p].
template <typename T, int NW>
__device__ inline void block_reduce_store(WaveLds<T> *lds, const cx<T> (&acc)[Tr<T>::R], int nr, int p0, int nout,
                                          cx<T> *__restrict__ out, int64_t ostride)
{
    constexpr int R = Tr<T>::R;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < R; ++r) lds[w].out[r][lane] = acc[r];
    __syncthreads();
    if (w == 0 && p0 + lane < nout)
        for (int r = 0; r < nr; ++r) {
            cx<T> v = lds[0].out[r][lane];
#pragma unroll
            for (int i = 1; i < NW; ++i) v += lds[i].out[r][lane];
            out[r * ostride + p0 + lane] = v;
        }
    __syncthreads();
}

// Upward pass of one level (Lemma M2M): one block per parent box at level
// lc - 1; wave w translates the child at position w (dx = w & 1, dy = w >> 1).
template <typename T>
__global__ void __launch_bounds__(256) k_up(const cx<T> *__restrict__ Mc, cx<T> *__restrict__ Mp,
                                            const cx<T> *__restrict__ tab, int nrhs, int ncc, int ncp, int ncol_c,
                                            int col_lo_c, int rows_c, int ncol_p, int col_lo_p)
{
    constexpr int R = Tr<T>::R;
    __shared__ WaveLds<T> lds[4];
    const int b = blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int prow = b / ncol_p, pcol = col_lo_p + b % ncol_p;
    const int crow = 2 * prow + (w >> 1), ccl = 2 * pcol + (w & 1) - col_lo_c;
    const bool ok = crow < rows_c && ccl >= 0 && ccl < ncol_c;
    const cx<T> *x = Mc + ((int64_t)crow * ncol_c + ccl) * nrhs * ncc;
    const cx<T> *A = tab + (int64_t)w * ncc * ncp;
    for (int r0 = 0; r0 < nrhs; r0 += R) {
        const int nr = nrhs - r0 < R ? nrhs - r0 : R;
        for (int p0 = 0; p0 < ncp; p0 += 64) {
            cx<T> acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = mk<T>(0, 0);
            if (ok) item_matvec<T>(A, ncc, ncp, p0, x + (int64_t)r0 * ncc, ncc, nr, lds[w], acc);
            block_reduce_store<T, 4>(lds, acc, nr, p0, ncp, Mp + ((int64_t)b * nrhs + r0) * ncp, ncp);
        }
    }
}

struct DownArgs {
    // level l
    int nc, ncol, col_lo, rows_s, rows_t;
    int top;     // 1 at the coarsest expansion level: every non-adjacent pair, no parent test
    int nrt;     // target rows with M2L classes (their slots: row_off[row] .. row_off[row + 1])
    int nb_m2l;  // blocks with one box each: rows < nrt
    // level l - 1
    int ncp, ncol_p, col_lo_p, rows_t_p;
    int has_l2l;
    int add_rows;  // rows whose stored local expansion (M2L of an earlier launch) is added to the L2L shift
};

// Downward pass of one level: L_box = L2L(parent's L) + sum over the box's
// interaction list of M2L (Lemma L2L, Lemma M2L).  Blocks below nb_m2l take
// one box of the M2L rows each (items: the L2L shift, then the row's class
// slots, dealt to the waves in turn; the waves' sums are added in order);
// the remaining blocks take DW boxes, one per wave, whose only item is the
// L2L shift, plus the stored value in rows below add_rows.  The apply runs
// the M2L of all levels first (k_m2l_all) and then this kernel level by level
// in its L2L form (nb_m2l = 0, add_rows = the interface rows).
constexpr int DW = 8;
template <typename T>
__global__ void __launch_bounds__(64 * DW) k_down(DownArgs a, int nrhs, const cx<T> *__restrict__ Lp,
                                                  const cx<T> *__restrict__ l2l, cx<T> *__restrict__ Lc,
                                                  const cx<T> *__restrict__ Ms, const cx<T> *__restrict__ atab,
                                                  const int *__restrict__ cls3, const int *__restrict__ row_off)
{
    constexpr int R = Tr<T>::R;
    __shared__ WaveLds<T> lds[DW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool m2l_block = (int)blockIdx.x < a.nb_m2l;
    int64_t box;
    int first, step, nitems, s0 = 0;
    if (m2l_block) {
        box = blockIdx.x;
        const int row = (int)(box / a.ncol);
        s0 = row_off[row];
        nitems = a.has_l2l + row_off[row + 1] - s0;
        first = w;
        step = DW;
    } else {
        box = (int64_t)a.nrt * a.ncol + (int64_t)(blockIdx.x - a.nb_m2l) * DW + w;
        if (box >= (int64_t)a.rows_t * a.ncol) return;  // whole wave; no block barrier on this path
        nitems = a.has_l2l;
        first = 0;
        step = 1;
    }
    const int row = (int)(box / a.ncol), col = a.col_lo + (int)(box % a.ncol);
    const int prow = row >> 1, pcl = (col >> 1) - a.col_lo_p, pos = (col & 1) + 2 * (row & 1);
    const bool pok = prow < a.rows_t_p && pcl >= 0 && pcl < a.ncol_p;
    for (int r0 = 0; r0 < nrhs; r0 += R) {
        const int nr = nrhs - r0 < R ? nrhs - r0 : R;
        for (int p0 = 0; p0 < a.nc; p0 += 64) {
            cx<T> acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = mk<T>(0, 0);
            cx<T> *out = Lc + (box * nrhs + r0) * a.nc;
            // the stored value to add, loaded before the shift's own loads
            const int pp = p0 + (threadIdx.x & 63);
            const bool addp = !m2l_block && row < a.add_rows && pp < a.nc;
            cx<T> prev[R];
#pragma unroll
            for (int r = 0; r < R; ++r) prev[r] = (addp && r < nr) ? out[r * a.nc + pp] : mk<T>(0, 0);
            for (int i = first; i < nitems; i += step) {
                const cx<T> *A, *x;
                int nk;
                bool ok;
                if (i < a.has_l2l) {
                    A = l2l + (int64_t)pos * a.ncp * a.nc;
                    x = Lp + (((int64_t)prow * a.ncol_p + pcl) * nrhs + r0) * a.ncp;
                    nk = a.ncp;
                    ok = pok;
                } else {
                    const int slot = s0 + i - a.has_l2l;
                    const int rs = cls3[3 * slot + 1], dc = cls3[3 * slot + 2];
                    const int cs = col + dc, csl = cs - a.col_lo, dp = (cs >> 1) - (col >> 1);
                    A = atab + (int64_t)slot * a.nc * a.nc;
                    x = Ms + (((int64_t)rs * a.ncol + csl) * nrhs + r0) * a.nc;
                    nk = a.nc;
                    ok = rs < a.rows_s && csl >= 0 && csl < a.ncol && (a.top || (dp <= 1 && dp >= -1));
                }
                if (ok) item_matvec<T>(A, nk, a.nc, p0, x, nk, nr, lds[w], acc);
            }
            if (m2l_block) {
                block_reduce_store<T, DW>(lds, acc, nr, p0, a.nc, out, a.nc);
            } else if (pp < a.nc) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (r < nr) out[r * a.nc + pp] = addp ? acc[r] + prev[r] : acc[r];
            }
        }
    }
}

// M2L of every expansion level in one launch (Lemma M2L): one block per
// target box of a level's interface rows (all rows at the coarsest level);
// the box's class slots are dealt to the waves in turn and the waves' sums
// added in order.  The result is stored as the box's local expansion, which
// the level's L2L launch then adds to the shifted parent expansion.
constexpr int M2L_MAXLEV = 26;
template <typename T>
struct M2LLevels {
    int n;
    int blk0[M2L_MAXLEV + 1];  // first block of each listed level; blk0[n] = total
    int nc[M2L_MAXLEV], ncol[M2L_MAXLEV], col_lo[M2L_MAXLEV], rows_s[M2L_MAXLEV], top[M2L_MAXLEV];
    int64_t off_s[M2L_MAXLEV], off_t[M2L_MAXLEV];
    const cx<T> *atab[M2L_MAXLEV];
    const int *cls3[M2L_MAXLEV];
    const int *row_off[M2L_MAXLEV];
};

constexpr int M2L_DW = 8;  // waves per target box in the M2L launch
template <typename T>
__global__ void __launch_bounds__(64 * M2L_DW) k_m2l_all(M2LLevels<T> a, int nrhs, const cx<T> *__restrict__ M,
                                                     cx<T> *__restrict__ Lc)
{
    constexpr int R = Tr<T>::R;
    __shared__ WaveLds<T> lds[M2L_DW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int li = 0;
    while (li + 1 < a.n && (int)blockIdx.x >= a.blk0[li + 1]) ++li;
    const int box = blockIdx.x - a.blk0[li];
    const int nc = a.nc[li], ncol = a.ncol[li], col_lo = a.col_lo[li];
    const int row = box / ncol, col = col_lo + box % ncol;
    const int *row_off = a.row_off[li], *cls3 = a.cls3[li];
    const int s0 = row_off[row], nitems = row_off[row + 1] - s0;
    const cx<T> *Ms = M + a.off_s[li];
    for (int r0 = 0; r0 < nrhs; r0 += R) {
        const int nr = nrhs - r0 < R ? nrhs - r0 : R;
        for (int p0 = 0; p0 < nc; p0 += 64) {
            cx<T> acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = mk<T>(0, 0);
            for (int i = w; i < nitems; i += M2L_DW) {
                const int slot = s0 + i;
                const int rs = cls3[3 * slot + 1], dc = cls3[3 * slot + 2];
                const int cs = col + dc, csl = cs - col_lo, dp = (cs >> 1) - (col >> 1);
                if (rs < a.rows_s[li] && csl >= 0 && csl < ncol && (a.top[li] || (dp <= 1 && dp >= -1)))
                    item_matvec<T>(a.atab[li] + (int64_t)slot * nc * nc, nc, nc, p0,
                                   Ms + (((int64_t)rs * ncol + csl) * nrhs + r0) * nc, nc, nr, lds[w], acc);
            }
            block_reduce_store<T, M2L_DW>(lds, acc, nr, p0, nc, Lc + a.off_t[li] + ((int64_t)box * nrhs + r0) * nc, nc);
        }
    }
}

// ---------------------------------------------------------------------------
// Near-field pair sum: G = sum over nodes of D_n exp(s2_n y1 - s1_n y0 + i lam_n dx).
// Nodes: nmid on the finite piece, then panels of 2*NGL nodes (right and left
// ray) of geometrically growing length; panel m starts at t0 2^(m-1).
// ---------------------------------------------------------------------------
__device__ inline cx<double> node_term(const Node &nd, double y1, double y0, double dx)
{
    double er = nd.str * y1 - nd.ssr * y0 - nd.li * dx;
    double ei = nd.sti * y1 - nd.ssi * y0 + nd.lr * dx;
    double m = exp(er), sn, cs;
    sincos(ei, &sn, &cs);
    double vr = m * cs, vi = m * sn;
    return {nd.dr * vr - nd.di * vi, nd.dr * vi + nd.di * vr};
}

__device__ inline int panels_needed(double a, double dx, double t0, int npan)
{
    // ray node t: |integrand| ~ exp(-t (a + dx)/sqrt(2)); keep panels whose
    // start t_s satisfies t_s (a + dx)/sqrt(2) < 40
    double r = (a + dx) * 0.70710678118654752;
    double lim = 40.0 / (r * t0);
    int m = 1;
    if (lim > 1.0) m = 2 + (int)floor(log2(lim));
    return m < npan ? m : npan;
}

__device__ inline int wave_max_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ inline cx<double> pair_kernel(const Node *__restrict__ nodes, int nmid, int npan, double t0, double y1,
                                         double y0, double dx, bool act)
{
    int need = act ? panels_needed(y0 - y1, dx, t0, npan) : 0;
    int wneed = wave_max_i(need);
    cx<double> G = {0.0, 0.0};
    for (int n = 0; n < nmid; ++n) G += node_term(nodes[n], y1, y0, dx);
    for (int m = 0; m < wneed; ++m) {
        const Node *pn = nodes + nmid + m * 2 * NGL;
        cx<double> Gp = {0.0, 0.0};
        for (int n = 0; n < 2 * NGL; ++n) Gp += node_term(pn[n], y1, y0, dx);
        if (m < need) G += Gp;
    }
    return G;
}

// ---------------------------------------------------------------------------
// L2P (Definition "Local Expansion"): res[r] = sum_p Lhat_p J_p(k2 r)
// e^{i p theta} at the point (X, Y) relative to the leaf centre, from the
// scaled expansion Ls[r][2P+1], r < nr.
// ---------------------------------------------------------------------------
template <typename T, int PMAX, int RMAX>
__device__ inline void eval_local(cx<T> k2, T X, T Y, T invR, int P, const cx<T> *Ls, int nr, cx<double> (&res)[RMAX])
{
    const int nc = 2 * P + 1;
    cx<T> tm[PMAX + 1];
    cx<T> J0;
    bessel_ratios<T, PMAX>(k2, X, Y, P, tm, J0);
    cx<T> up = mk<T>(X * invR, Y * invR), dn = mk<T>(-X * invR, Y * invR);
    cx<T> acc[RMAX];
    for (int r = 0; r < RMAX; ++r) acc[r] = (r < nr) ? J0 * Ls[r * nc + P] : mk<T>(0, 0);
    cx<T> vp = J0, vm = J0;
#pragma unroll
    for (int p = 1; p <= PMAX; ++p) {
        if (p <= P) {
            cx<T> f = T(2 * p) * tm[p];
            vp = vp * (f * up);
            vm = vm * (f * dn);
            for (int r = 0; r < RMAX; ++r)
                if (r < nr) {
                    cfma(acc[r], vp, Ls[r * nc + P + p]);
                    cfma(acc[r], vm, Ls[r * nc + P - p]);
                }
        }
    }
    for (int r = 0; r < RMAX; ++r) res[r] = {(double)acc[r].re, (double)acc[r].im};
}

// ---------------------------------------------------------------------------
// L2P over G consecutive target leaves per block (points contiguous in the
// sorted order); the near field, if any, comes from the sweep kernel's parts.
// First the leaves' local expansions go to LDS: by the leaf-level L2L shift of
// the parent's (Lemma L2L, one leaf per wave at a time), plus the stored M2L
// result in the interface rows, or copied from the stored expansions.  Then
// a thread per target evaluates its leaf's expansion and adds the near-field
// parts in order.  Writes u[r][original index].
// ---------------------------------------------------------------------------
constexpr int L2P_THREADS = 512;
template <typename T, int PMAX, int RMAX>
__global__ void __launch_bounds__(L2P_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_l2p(const int32_t *__restrict__ start,
                                                     const int32_t *__restrict__ end, const int32_t *__restrict__ idx,
                                                     const double *__restrict__ xs, const double *__restrict__ ys,
                                                     int64_t ns, int64_t nt, int nrhs, int P, int nbox, int ncol,
                                                     int col_lo, double x_lo, double w, cx<T> k2, T invR,
                                                     const cx<T> *__restrict__ Lc, LeafShift<T> sh, int64_t key_t0,
                                                     int G, int do_far, const cx<double> *__restrict__ unear,
                                                     int nparts, cx<T> *__restrict__ u)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ WaveLds<T> wl[L2P_THREADS / 64];
    __shared__ int bnd[LEAF_GMAX + 1];
    constexpr int R = Tr<T>::R;
    const int nc = 2 * P + 1;
    cx<T> *Ls = reinterpret_cast<cx<T> *>(smem_raw);  // [G][RMAX][nc]
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int b0 = blockIdx.x * G;
    const int ng = nbox - b0 < G ? nbox - b0 : G;
    const int r0 = blockIdx.y * RMAX;
    const int nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    if (t <= ng) bnd[t] = t < ng ? start[key_t0 + b0 + t] : end[key_t0 + b0 + ng - 1];
    __syncthreads();
    const int S = bnd[0], E = bnd[ng];
    if (E <= S) return;
    // the first chunk's points: their loads are in flight while the leaf
    // expansions are formed
    double px = 0.0, py = 0.0;
    int32_t pid = 0;
    if (S + t < E) {
        px = xs[S + t];
        py = ys[S + t];
        pid = idx[S + t];
    }
    if (do_far && sh.tab) {
        for (int g = wv; g < ng; g += L2P_THREADS / 64) {
            if (bnd[g + 1] <= bnd[g]) continue;  // no targets in this leaf
            const int box = b0 + g, row = box / ncol, col = col_lo + box % ncol;
            const int prow = row >> 1, pcl = (col >> 1) - sh.col_lo_p, pos = (col & 1) + 2 * (row & 1);
            const bool pok = prow < sh.rows_p && pcl >= 0 && pcl < sh.ncol_p;
            const cx<T> *x = sh.Lp + ((int64_t)prow * sh.ncol_p + pcl) * nrhs * sh.ncp;
            const bool add = row < sh.add_rows;
            for (int rr = 0; rr < nr; rr += R) {
                const int nrr = nr - rr < R ? nr - rr : R;
                for (int p0 = 0; p0 < nc; p0 += 64) {
                    cx<T> acc[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] = mk<T>(0, 0);
                    const int p = p0 + lane;
                    // the stored M2L value, loaded before the shift's own loads
                    cx<T> prev[R];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        prev[r] = (add && p < nc && r < nrr) ? Lc[((int64_t)box * nrhs + r0 + rr + r) * nc + p]
                                                             : mk<T>(0, 0);
                    if (pok)
                        item_matvec<T>(sh.tab + (int64_t)pos * sh.ncp * nc, sh.ncp, nc, p0,
                                       x + (int64_t)(r0 + rr) * sh.ncp, sh.ncp, nrr, wl[wv], acc);
                    if (p < nc)
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            if (r < nrr) Ls[(g * RMAX + rr + r) * nc + p] = add ? acc[r] + prev[r] : acc[r];
                }
            }
        }
    } else if (do_far) {
        const int per = nr * nc;
        for (int e = t; e < ng * per; e += L2P_THREADS) {
            const int g = e / per, o = e - g * per, r = o / nc, c = o - r * nc;
            Ls[(g * RMAX + r) * nc + c] = Lc[((int64_t)(b0 + g) * nrhs + r0 + r) * nc + c];
        }
    }
    __syncthreads();
    for (int c0 = S; c0 < E; c0 += L2P_THREADS) {
        const int i = c0 + t;
        if (i >= E) break;
        if (c0 != S) {
            px = xs[i];
            py = ys[i];
            pid = idx[i];
        }
        int g = 0;
        while (i >= bnd[g + 1]) ++g;
        const int box = b0 + g, row = box / ncol, col = col_lo + box % ncol;
        cx<double> res[RMAX];
        for (int r = 0; r < RMAX; ++r) res[r] = {0.0, 0.0};
        if (do_far) {
            const double cxp = x_lo + (col + 0.5) * w, cyp = -(row + 0.5) * w;
            eval_local<T, PMAX, RMAX>(k2, (T)(px - cxp), (T)(py - cyp), invR, P, Ls + g * RMAX * nc, nr, res);
        }
        const int64_t o = pid - ns;
        if (unear && row == 0)
            for (int pp = 0; pp < nparts; ++pp)
                for (int r = 0; r < RMAX; ++r)
                    if (r < nr) res[r] += unear[((int64_t)pp * nrhs + r0 + r) * nt + o];
        for (int r = 0; r < RMAX; ++r)
            if (r < nr) u[(int64_t)(r0 + r) * nt + o] = mk<T>((T)res[r].re, (T)res[r].im);
    }
}

// ---------------------------------------------------------------------------
// Fused L2P + S2T per target leaf, the near field by pairs (the alternative
// to the sweep); lanes over targets (chunks of 64).
// Writes u[r][original index] (no accumulation across kernels).
// ---------------------------------------------------------------------------
template <typename T, int PMAX, int RMAX>
__global__ void __launch_bounds__(64) k_l2p_near(const int32_t *__restrict__ start, const int32_t *__restrict__ end,
                                                 const int32_t *__restrict__ idx, const double *__restrict__ xs,
                                                 const double *__restrict__ ys, const cx<T> *__restrict__ q,
                                                 int64_t ns, int64_t nt, int nrhs, int P, int ncol, int col_lo,
                                                 int rows_s, double x_lo, double w, cx<T> k2, T invR,
                                                 const cx<T> *__restrict__ Lc, LeafShift<T> sh,
                                                 const Node *__restrict__ nodes, int nmid, int npan, double t0,
                                                 int do_far, int do_near, int64_t key_t0,
                                                 const cx<double> *__restrict__ unear, int nparts,
                                                 cx<T> *__restrict__ u)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ WaveLds<T> wl;
    const int nc = 2 * P + 1;
    cx<T> *Ls = reinterpret_cast<cx<T> *>(smem_raw);  // [RMAX][nc]
    const int box = blockIdx.x, lane = threadIdx.x;
    const int r0 = blockIdx.y * RMAX;
    const int nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    const int row = box / ncol, cl = box % ncol, col = col_lo + cl;
    const double cxp = x_lo + (col + 0.5) * w, cyp = -(row + 0.5) * w;
    const int s = start[key_t0 + box], e = end[key_t0 + box];
    if (e <= s) return;
    if (do_far && sh.tab) {
        // the leaf's local expansion: L2L shift of the parent's (Lemma L2L),
        // plus the stored M2L result in the interface rows
        constexpr int R = Tr<T>::R;
        const int prow = row >> 1, pcl = (col >> 1) - sh.col_lo_p, pos = (col & 1) + 2 * (row & 1);
        const bool pok = prow < sh.rows_p && pcl >= 0 && pcl < sh.ncol_p;
        const cx<T> *x = sh.Lp + ((int64_t)prow * sh.ncol_p + pcl) * nrhs * sh.ncp;
        const bool add = row < sh.add_rows;
        for (int rr = 0; rr < nr; rr += R) {
            const int nrr = nr - rr < R ? nr - rr : R;
            for (int p0 = 0; p0 < nc; p0 += 64) {
                cx<T> acc[R];
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] = mk<T>(0, 0);
                if (pok)
                    item_matvec<T>(sh.tab + (int64_t)pos * sh.ncp * nc, sh.ncp, nc, p0,
                                   x + (int64_t)(r0 + rr) * sh.ncp, sh.ncp, nrr, wl, acc);
                const int p = p0 + lane;
                if (p < nc)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (r < nrr) {
                            cx<T> v = acc[r];
                            if (add) v += Lc[(((int64_t)row * ncol + cl) * nrhs + r0 + rr + r) * nc + p];
                            Ls[(rr + r) * nc + p] = v;
                        }
            }
        }
        __syncthreads();
    } else if (do_far) {
        for (int r = 0; r < nr; ++r)
            for (int t = lane; t < nc; t += 64)
                Ls[r * nc + t] = Lc[(((int64_t)row * ncol + cl) * nrhs + r0 + r) * nc + t];
        __syncthreads();
    }
    for (int c0 = s; c0 < e; c0 += 64) {
        int i = c0 + lane;
        bool act = i < e;
        int ii = act ? i : s;
        double x1 = xs[ii], y1 = ys[ii];
        cx<double> res[RMAX];
        for (int r = 0; r < RMAX; ++r) res[r] = {0.0, 0.0};
        if (do_far) eval_local<T, PMAX, RMAX>(k2, (T)(x1 - cxp), (T)(y1 - cyp), invR, P, Ls, nr, res);
        if (do_near && row == 0 && rows_s > 0) {
            if (unear) {
                // near field computed by the sweep kernel: add its parts in order
                if (act) {
                    int64_t o = idx[i] - ns;
                    for (int pp = 0; pp < nparts; ++pp)
                        for (int r = 0; r < RMAX; ++r)
                            if (r < nr) res[r] += unear[((int64_t)pp * nrhs + r0 + r) * nt + o];
                }
            } else {
                for (int dc = -1; dc <= 1; ++dc) {
                    int cs = cl + dc;
                    if (cs < 0 || cs >= ncol) continue;
                    int js = start[cs], je = end[cs];  // row-0 source leaf
                    for (int j = js; j < je; ++j) {
                        double x0 = xs[j], y0 = ys[j];
                        cx<double> G = pair_kernel(nodes, nmid, npan, t0, y1, y0, fabs(x1 - x0), act);
                        int64_t o = idx[j];
                        for (int r = 0; r < RMAX; ++r)
                            if (r < nr) {
                                cx<T> qq = q[(int64_t)(r0 + r) * ns + o];
                                cfma(res[r], G, cx<double>{(double)qq.re, (double)qq.im});
                            }
                    }
                }
            }
        }
        if (act) {
            int64_t o = idx[i] - ns;
            for (int r = 0; r < RMAX; ++r)
                if (r < nr) u[(int64_t)(r0 + r) * nt + o] = mk<T>((T)res[r].re, (T)res[r].im);
        }
    }
}

// ---------------------------------------------------------------------------
// Near field by x-ordered sweeps (S2T over adjacent leaves across the
// interface).  For a fixed node lam_n of the pair-independent contour, the
// pair term of source j and target i with x_j <= x_i is
//   D_n e^{s_t y_i} * e^{i lam_n (x_i - x_j)} * e^{-s_s y_j} q_j.
// Writing x_i - x_j = (x_i - b) - (x_j - b) for a base point b <= x_j splits
// the x factor between the two points, so sweeping the points in increasing x
// while carrying
//   V_n = sum of e^{-i lam_n (x_j - b) - s_s y_j} q_j over the sources passed
// gives sum_{j: x_j <= x_i} at a target as D_n e^{i lam_n (x_i - b) + s_t y_i} V_n:
// one complex exponential per point and node.  The source factor grows like
// e^{Im lam_n (x_j - b)}; before that exceeds e^{SW_RESCALE} for any node of
// the wave, the base moves to the current point (V_n <- e^{i lam_n (x - b)} V_n,
// a decaying factor).  A sweep in decreasing x (base to the right) gives the
// sources with x_j > x_i (|x_i - x_j| enters by evenness).  Every pair's
// product equals its term in the pairwise sum.
//
// Row-0 leaves are x-intervals, so one sweep runs along a segment of
// consecutive leaf columns.  It keeps two sums: Vp, the complete sum of the
// previous leaf's sources, and Vc, the running sum of the current leaf's; a
// target of leaf c takes Vp + Vc, which is exactly its sources in leaves c - 1
// and c on the sweep's side.  Entering a leaf, Vp <- Vc and Vc <- 0.  The
// sweep starts one leaf before the segment (sources only), so each source is
// visited once per direction and segment instead of once per adjacent target
// leaf.  Lanes are nodes; a wave carries SweepCap::G groups of 64 nodes
// (independent chains) and adds their terms per lane before one wave
// reduction in fixed order.  Each wave keeps its target sums in LDS (and
// clears them itself); they are added in wave order when a piece of
// SweepCap::T targets or an x-slab is complete.  The increasing-x sweep stores
// the sum and the decreasing-x sweep adds its own (the same thread handles a
// target in both).
// One block per (segment, rhs chunk, node part); results go to
// unear[part][rhs][target] and the leaf evaluation adds the parts in order.
// ---------------------------------------------------------------------------
// points of one leaf column (sources and targets) held in LDS with their
// densities, targets per accumulator piece, node groups per wave; a larger
// leaf column is swept in x-slabs, and a segment with a slab that still does
// not fit takes the pairwise sum
template <int RMAX>
struct SweepCap {
    static constexpr int N = RMAX == 1 ? 512 : 256;
    static constexpr int T = RMAX == 1 ? 96 : 64;
    static constexpr int G = RMAX == 1 ? 2 : 1;  // node groups per wave (independent chains)
};
constexpr int SW_W = 4;               // waves per block
constexpr double SW_RESCALE = 300.0;  // largest exponent of a source factor

__device__ inline double wave_max_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// One DPP lane move of a double (both halves); lanes of rows outside ROWMASK
// read 0.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_d(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Sum over the wave in a fixed order, complete in lane 63: pairs, quads,
// half rows and rows by lane permutations within each row of 16, then row 0
// into row 1, row 2 into row 3, and rows 0-1 into row 3.
__device__ inline double wave_total_d(double v)
{
    v += dpp_d<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_d<0x141, 0xf>(v);  // row_half_mirror
    v += dpp_d<0x140, 0xf>(v);  // row_mirror
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

constexpr int SW_KMAX = 32;  // x-slabs per leaf column at most

// Fill the tables of cexp_tab (2^{j/64}, sin and cos of j pi/32).
__device__ inline void cexp_tab_init(CexpTab &tb, int t, int nthreads)
{
    for (int j = t; j < 64; j += nthreads) {
        tb.t2[j] = exp2(j / 64.0);
        double sv, cv;
        sincospi(j / 32.0, &sv, &cv);
        tb.sn[j] = sv;
        tb.cs[j] = cv;
    }
}

__device__ inline int leaf_count(const int32_t *start, const int32_t *end, int64_t k)
{
    const int a = start[k], b = end[k];
    return b > a ? b - a : 0;
}

template <typename T, int RMAX>
__global__ void __launch_bounds__(64 * SW_W) __attribute__((amdgpu_waves_per_eu(4))) k_near_sweep(const int32_t *__restrict__ start,
                                                          const int32_t *__restrict__ end,
                                                          const int32_t *__restrict__ idx, const double *__restrict__ xs,
                                                          const double *__restrict__ ys, const cx<T> *__restrict__ q,
                                                          int64_t ns, int64_t nt, int nrhs, int ncol, int64_t key_t0,
                                                          int seglen, double xl0, double w,
                                                          const Node *__restrict__ nodes, int nnodes,
                                                          int nmid, int npan, double t0, int nparts,
                                                          cx<double> *__restrict__ unear)
{
    constexpr int NMAX = SweepCap<RMAX>::N, TCAP = SweepCap<RMAX>::T, NT = 64 * SW_W;
    static_assert(TCAP <= NT, "a piece's targets map to distinct threads");
    __shared__ double sx[NMAX], sy[NMAX];
    __shared__ double ox[NMAX], oy[NMAX];  // positions in increasing-x order
    __shared__ int oi[NMAX];               // staging index in increasing-x order (targets: -1 - index)
    __shared__ int tk[NMAX];               // staging index of the slab's target of each rank
    __shared__ int lid[NMAX];              // leaf index of each staged point (targets after sources)
    __shared__ int s_cnt[2];               // staged points, of them targets
    __shared__ int hist[SW_KMAX];
    __shared__ CexpTab ctab;
    __shared__ cx<double> sq[NMAX][RMAX];  // the sources' densities
    __shared__ double accr[SW_W][TCAP][RMAX], acci[SW_W][TCAP][RMAX];  // per wave
    __shared__ int s_big;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int r0 = blockIdx.y * RMAX, nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    const int part = blockIdx.z;
    const int c0 = blockIdx.x * seglen, c1 = c0 + seglen < ncol ? c0 + seglen : ncol;
    cx<double> *un = unear + (int64_t)part * nrhs * nt;

    // no targets: nothing to write; no sources: the targets' sums are zero
    int ntot = 0, nsrc = 0;
    for (int c = c0 > 0 ? c0 - 1 : 0; c < (c1 < ncol ? c1 + 1 : ncol); ++c) {
        nsrc += leaf_count(start, end, c);
        if (c >= c0 && c < c1) ntot += leaf_count(start, end, key_t0 + c);
    }
    if (ntot == 0) return;
    if (nsrc == 0) {
        for (int c = c0; c < c1; ++c) {
            const int ts = start[key_t0 + c], nT = leaf_count(start, end, key_t0 + c);
            for (int k = t; k < nT * nr; k += NT)
                un[(int64_t)(r0 + k % nr) * nt + (idx[ts + k / nr] - ns)] = cx<double>{0.0, 0.0};
        }
        return;
    }

    // a leaf column of the segment's range whose x-slabs do not fit in LDS
    // sends the whole segment to the pairwise sum
    if (t == 0) s_big = 0;
    cexp_tab_init(ctab, t, NT);
    for (int c = (c0 > 0 ? c0 - 1 : 0); c < (c1 < ncol ? c1 + 1 : ncol); ++c) {
        const int nS = leaf_count(start, end, c), nT = c >= c0 && c < c1 ? leaf_count(start, end, key_t0 + c) : 0;
        const int n = nS + nT, K = sweep_slabs(n, NMAX);
        if (K == 1) continue;
        if (K > SW_KMAX) {
            if (t == 0) s_big = 1;
            continue;
        }
        const double xl = xl0 + c * w, sc = K / w;
        __syncthreads();
        for (int k = t; k < K; k += NT) hist[k] = 0;
        __syncthreads();
        for (int k = t; k < n; k += NT) {
            const double x = xs[k < nS ? start[c] + k : start[key_t0 + c] + k - nS];
            atomicAdd(&hist[slab_of(x, xl, sc, K)], 1);
        }
        __syncthreads();
        for (int k = t; k < K; k += NT)
            if (hist[k] > NMAX) s_big = 1;
    }
    __syncthreads();
    if (s_big) {
        // pairwise sum per target leaf, lanes over targets (part 0 only)
        for (int cl = c0; cl < c1; ++cl) {
            const int ts = start[key_t0 + cl], te = end[key_t0 + cl];
            int js = 0, je = 0;
            bool any = false;
            for (int dc = -1; dc <= 1; ++dc) {
                const int cs = cl + dc;
                if (cs < 0 || cs >= ncol) continue;
                const int a = start[cs], b = end[cs];
                if (b <= a) continue;
                if (!any) js = a;
                je = b;
                any = true;
            }
            for (int i0 = ts; i0 < te; i0 += NT) {
                const int i = i0 + t;
                const bool act = i < te;
                const int ii = act ? i : ts;
                const double x1 = xs[ii], y1 = ys[ii];
                cx<double> res[RMAX];
                for (int r = 0; r < RMAX; ++r) res[r] = {0.0, 0.0};
                if (part == 0 && any)
                    for (int j = js; j < je; ++j) {
                        const cx<double> G = pair_kernel(nodes, nmid, npan, t0, y1, ys[j], fabs(x1 - xs[j]), act);
                        const int64_t o = idx[j];
                        for (int r = 0; r < nr; ++r) {
                            const cx<T> qq = q[(int64_t)(r0 + r) * ns + o];
                            cfma(res[r], G, cx<double>{(double)qq.re, (double)qq.im});
                        }
                    }
                if (act)
                    for (int r = 0; r < nr; ++r) un[(int64_t)(r0 + r) * nt + (idx[i] - ns)] = res[r];
            }
        }
        return;
    }

    constexpr int G = SweepCap<RMAX>::G;
    const int ngroups = (nnodes + 63) / 64, nunits = (ngroups + G - 1) / G;  // a unit: G groups of 64 nodes
    const int slots = nparts * SW_W, slot = part * SW_W + wv;
    const int gpw = nunits > 0 ? (nunits + slots - 1) / slots : 1;  // at least one pass writes the targets
    for (int k = lane; k < TCAP * RMAX; k += 64) {
        (&accr[wv][0][0])[k] = 0.0;
        (&acci[wv][0][0])[k] = 0.0;
    }
    for (int gi = 0; gi < gpw; ++gi) {
        const int unit = gi * slots + slot;
        const bool has = unit < nunits;  // this wave has node groups
        Node nd[G];
        double limax[G];
        for (int g = 0; g < G; ++g) {
            const int nn = (unit * G + g) * 64 + lane;
            const bool act = has && nn < nnodes;
            nd[g] = nodes[act ? nn : 0];
            if (!act) nd[g].dr = nd[g].di = 0.0;  // contributes nothing
            limax[g] = wave_max_d(act ? fabs(nd[g].li) : 0.0);
        }
        for (int dir = 0; dir < 2; ++dir) {
            cx<double> Vp[G][RMAX], Vc[G][RMAX];
            double xb[G];
            for (int g = 0; g < G; ++g) {
                xb[g] = 0.0;
                for (int r = 0; r < RMAX; ++r) Vp[g][r] = Vc[g][r] = {0.0, 0.0};
            }
            bool based = false;
            for (int lc = 0; lc <= c1 - c0; ++lc) {
                const int c = dir == 0 ? c0 - 1 + lc : c1 - lc;
                if (c < 0 || c >= ncol) continue;
                const bool warm = dir == 0 ? c < c0 : c >= c1;  // sources only
                const int ss = start[c], nS = leaf_count(start, end, c);
                const int ts = start[key_t0 + c], nT = warm ? 0 : leaf_count(start, end, key_t0 + c);
                const int n = nS + nT;
                for (int g = 0; g < G; ++g)
                    for (int r = 0; r < RMAX; ++r) {
                        Vp[g][r] = Vc[g][r];
                        Vc[g][r] = {0.0, 0.0};
                    }
                // the leaf in x-slabs that fit in LDS, visited in sweep order
                const int K = sweep_slabs(n, NMAX);
                const double xl = xl0 + c * w, sc = K / w;
                int pbase = 0, pcnt = 0;  // targets flushed so far (sweep order); open piece size
                int tdone = 0;            // targets of the slabs already visited
                for (int sl = 0; sl < K; ++sl) {
                    const int sidx = dir == 0 ? sl : K - 1 - sl;
                    __syncthreads();  // the previous slab's LDS contents are no longer read
                    if (t == 0) s_cnt[0] = s_cnt[1] = 0;
                    __syncthreads();
                    for (int k = t; k < n; k += NT) {
                        const bool src = k < nS;
                        const int64_t gp = src ? ss + k : ts + k - nS;
                        const double x = xs[gp];
                        int pos = k;
                        if (K > 1) {
                            if (slab_of(x, xl, sc, K) != sidx) continue;
                            pos = atomicAdd(&s_cnt[0], 1);
                            if (!src) atomicAdd(&s_cnt[1], 1);
                        }
                        sx[pos] = x;
                        sy[pos] = ys[gp];
                        lid[pos] = k;
                        if (src) {
                            const int64_t o = idx[gp];
                            for (int r = 0; r < RMAX; ++r) {
                                const cx<T> qq = r < nr ? q[(int64_t)(r0 + r) * ns + o] : mk<T>(0, 0);
                                sq[pos][r] = cx<double>{(double)qq.re, (double)qq.im};
                            }
                        }
                    }
                    __syncthreads();
                    const int m = K > 1 ? s_cnt[0] : n, mt = K > 1 ? s_cnt[1] : nT;
                    // order by (x, sources before targets, leaf index): rank by
                    // counting; targets also get their rank among the slab's targets
                    for (int a = t; a < m; a += NT) {
                        const double xa = sx[a];
                        const int la = lid[a], ta = la >= nS;
                        int rank = 0, trank = 0;
                        for (int b = 0; b < m; ++b) {
                            const double xq = sx[b];
                            const int lb = lid[b], tb = lb >= nS;
                            const bool less = xq < xa || (xq == xa && (tb < ta || (tb == ta && lb < la)));
                            rank += less ? 1 : 0;
                            trank += less && tb ? 1 : 0;
                        }
                        ox[rank] = xa;
                        oy[rank] = sy[a];
                        oi[rank] = ta ? -1 - a : a;
                        if (ta) tk[trank] = a;
                    }
                    __syncthreads();
                    for (int step = 0; step < m; ++step) {
                        const int k = dir == 0 ? step : m - 1 - step;
                        const int it = oi[k];
                        if (has) {
                            const double x = ox[k], y = oy[k];
                            if (!based) {
                                for (int g = 0; g < G; ++g) xb[g] = x;
                                based = true;
                            }
                            cx<double> e[G];
                            for (int g = 0; g < G; ++g) {
                                const Node &ng = nd[g];
                                double u = dir == 0 ? x - xb[g] : xb[g] - x;  // >= 0
                                if (limax[g] * u > SW_RESCALE) {
                                    // move the base to x: V <- e^{i lam u} V
                                    const cx<double> f = cexp_tab(-ng.li * u, ng.lr * u, ctab);
                                    for (int r = 0; r < RMAX; ++r)
                                        if (r < nr) {
                                            Vp[g][r] = Vp[g][r] * f;
                                            Vc[g][r] = Vc[g][r] * f;
                                        }
                                    xb[g] = x;
                                    u = 0.0;
                                }
                                // source: e^{-i lam u - s_s y}; target: D e^{i lam u + s_t y}
                                e[g] = it >= 0 ? cexp_tab(fma(ng.li, u, -ng.ssr * y), fma(-ng.lr, u, -ng.ssi * y), ctab)
                                               : cexp_tab(fma(-ng.li, u, ng.str * y), fma(ng.lr, u, ng.sti * y), ctab) *
                                                     cx<double>{ng.dr, ng.di};
                            }
                            if (it >= 0) {
                                // source: Vc += e q
                                for (int g = 0; g < G; ++g)
                                    for (int r = 0; r < RMAX; ++r)
                                        if (r < nr) cfma(Vc[g][r], e[g], sq[it][r]);
                            } else {
                                // target: add e (Vp + Vc) summed over the wave's nodes
                                for (int r = 0; r < RMAX; ++r)
                                    if (r < nr) {
                                        cx<double> cc = e[0] * (Vp[0][r] + Vc[0][r]);
                                        for (int g = 1; g < G; ++g) cfma(cc, e[g], Vp[g][r] + Vc[g][r]);
                                        const double cr = wave_total_d(cc.re), ci = wave_total_d(cc.im);
                                        if (lane == 63) {
                                            accr[wv][pcnt][r] += cr;
                                            acci[wv][pcnt][r] += ci;
                                        }
                                    }
                            }
                        }
                        if (it < 0) ++pcnt;
                        if (pcnt > 0 && (pcnt == TCAP || step == m - 1)) {
                            // the piece is complete: add the waves' sums in wave
                            // order; target of x-rank tr goes to thread tr mod NT
                            __syncthreads();
                            const int j = dir == 0 ? ((t - pbase) % NT + NT) % NT
                                                   : ((nT - 1 - pbase - t) % NT + NT) % NT;
                            if (j < pcnt) {
                                const int tr = dir == 0 ? pbase + j : nT - 1 - (pbase + j);
                                const int tlo = dir == 0 ? tdone : nT - tdone - mt;  // x-rank of the slab's first target
                                const int64_t o = idx[ts + lid[tk[tr - tlo]] - nS] - ns;
                                for (int r = 0; r < nr; ++r) {
                                    double sr = accr[0][j][r], si = acci[0][j][r];
                                    for (int w2 = 1; w2 < SW_W; ++w2) {
                                        sr += accr[w2][j][r];
                                        si += acci[w2][j][r];
                                    }
                                    cx<double> &dst = un[(int64_t)(r0 + r) * nt + o];
                                    if (dir == 0 && gi == 0)
                                        dst = cx<double>{sr, si};
                                    else
                                        dst = dst + cx<double>{sr, si};
                                }
                            }
                            __syncthreads();
                            // each wave clears its own sums: its next additions
                            // follow in its own program order
                            for (int kk = lane; kk < TCAP * RMAX; kk += 64) {
                                (&accr[wv][0][0])[kk] = 0.0;
                                (&acci[wv][0][0])[kk] = 0.0;
                            }
                            pbase += pcnt;
                            pcnt = 0;
                        }
                    }
                    tdone += mt;
                }
            }
        }
    }
}

// Near-field derivative sums for the gradient: returns (sum D e^E lam, sum D e^E s_t)
// so that d/dx1 = i sgn(x1 - x0) * first and d/dy1 = second.
__device__ inline void pair_kernel_grad(const Node *__restrict__ nodes, int nmid, int npan, double t0, double y1,
                                        double y0, double dx, bool act, cx<double> &GL, cx<double> &GS)
{
    int need = act ? panels_needed(y0 - y1, dx, t0, npan) : 0;
    int wneed = wave_max_i(need);
    GL = {0.0, 0.0};
    GS = {0.0, 0.0};
    auto add = [&](const Node &nd, cx<double> &al, cx<double> &as) {
        cx<double> v = node_term(nd, y1, y0, dx);
        al += v * cx<double>{nd.lr, nd.li};
        as += v * cx<double>{nd.str, nd.sti};
    };
    for (int n = 0; n < nmid; ++n) add(nodes[n], GL, GS);
    for (int m = 0; m < wneed; ++m) {
        const Node *pn = nodes + nmid + m * 2 * NGL;
        cx<double> al = {0.0, 0.0}, as = {0.0, 0.0};
        for (int n = 0; n < 2 * NGL; ++n) add(pn[n], al, as);
        if (m < need) {
            GL += al;
            GS += as;
        }
    }
}

// Coordinate gradient at the targets: gout[0][i] = Re sum_r c[r][i] du_r/dx(x_i),
// gout[1][i] = ysign * Re sum_r c[r][i] du_r/dy(x_i), u = the field of densities q.
// Far part: the local expansion's gradient is a local expansion of order P+1,
//   d/dx (J_p e^{ip th}) = (k/2)(J_{p-1} e^{i(p-1)th} - J_{p+1} e^{i(p+1)th}),
//   d/dy (J_p e^{ip th}) = (ik/2)(J_{p-1} e^{i(p-1)th} + J_{p+1} e^{i(p+1)th}),
// rewritten for the scaled coefficients.  Near part: the integrand times
// i lam sgn(x1 - x0) (x) or s_t (y).
template <typename T, int PMAX>
__global__ void __launch_bounds__(64) k_l2p_grad(const int32_t *__restrict__ start, const int32_t *__restrict__ end,
                                                 const int32_t *__restrict__ idx, const double *__restrict__ xs,
                                                 const double *__restrict__ ys, const cx<T> *__restrict__ q,
                                                 const cx<T> *__restrict__ cw, int64_t ns, int64_t nt, int nrhs,
                                                 int r0, int nr, int accumulate,
                                                 int P, int ncol, int col_lo, int rows_s, double x_lo, double w,
                                                 cx<T> kt, T invR, const cx<T> *__restrict__ Lc,
                                                 const Node *__restrict__ nodes, int nmid, int npan, double t0,
                                                 int do_far, int do_near, int64_t key_t0, double ysign,
                                                 double *__restrict__ gout)
{
    extern __shared__ unsigned char smem_raw[];
    const int ncg = 2 * (P + 1) + 1;           // gradient expansions have order P + 1
    cx<T> *Gx = reinterpret_cast<cx<T> *>(smem_raw);  // [nr][ncg], right-hand sides r0 .. r0+nr-1
    cx<T> *Gy = Gx + (size_t)nr * ncg;
    const int box = blockIdx.x, lane = threadIdx.x;
    const int row = box / ncol, cl = box % ncol, col = col_lo + cl;
    const double cxp = x_lo + (col + 0.5) * w, cyp = -(row + 0.5) * w;
    const int s = start[key_t0 + box], e = end[key_t0 + box];
    if (e <= s) return;
    const int nc = 2 * P + 1;
    if (do_far) {
        const T R = T(1) / invR;
        const cx<T> hk2R = T(0.25) * R * (kt * kt);  // k^2 R / 4
        for (int t = lane; t < nr * ncg; t += 64) {
            int r = r0 + t / ncg, n = t % ncg - (P + 1);
            auto Lh = [&](int m) {
                return (m >= -P && m <= P) ? Lc[(((int64_t)row * ncol + cl) * nrhs + r) * nc + m + P] : mk<T>(0, 0);
            };
            cx<T> up = Lh(n + 1), dn = Lh(n - 1);
            // (k/2) s_{n+1}/s_n and (k/2) s_{n-1}/s_n
            cx<T> fp = n >= 0 ? mk<T>(T(n + 1) * invR, T(0)) : hk2R * (T(1) / T(-n));
            cx<T> fm = n > 0 ? hk2R * (T(1) / T(n)) : mk<T>(T(1 - n) * invR, T(0));
            cx<T> a = fp * up, b = fm * dn;
            Gx[t] = a - b;
            cx<T> sum = a + b;
            Gy[t] = mk<T>(-sum.im, sum.re);
        }
        __syncthreads();
    }
    for (int c0 = s; c0 < e; c0 += 64) {
        int i = c0 + lane;
        bool act = i < e;
        int ii = act ? i : s;
        double x1 = xs[ii], y1 = ys[ii];
        int64_t oi = idx[ii] - ns;
        double gx = 0.0, gy = 0.0;
        if (do_far) {
            cx<T> tm[PMAX + 1];
            cx<T> J0;
            T X = (T)(x1 - cxp), Y = (T)(y1 - cyp);
            const int Pg = P + 1;
            bessel_ratios<T, PMAX>(kt, X, Y, Pg, tm, J0);
            cx<T> up = mk<T>(X * invR, Y * invR), dn = mk<T>(-X * invR, Y * invR);
            for (int rr = 0; rr < nr; ++rr) {
                const int r = r0 + rr;
                const cx<T> *gxr = Gx + rr * ncg, *gyr = Gy + rr * ncg;
                cx<T> ax = J0 * gxr[Pg], ay = J0 * gyr[Pg];
                cx<T> vp = J0, vm = J0;
#pragma unroll
                for (int p = 1; p <= PMAX; ++p) {
                    if (p <= Pg) {
                        cx<T> f = T(2 * p) * tm[p];
                        vp = vp * (f * up);
                        vm = vm * (f * dn);
                        cfma(ax, vp, gxr[Pg + p]);
                        cfma(ax, vm, gxr[Pg - p]);
                        cfma(ay, vp, gyr[Pg + p]);
                        cfma(ay, vm, gyr[Pg - p]);
                    }
                }
                cx<T> cr = act ? cw[(int64_t)r * nt + oi] : mk<T>(0, 0);
                gx += (double)(cr.re * ax.re - cr.im * ax.im);
                gy += (double)(cr.re * ay.re - cr.im * ay.im);
            }
        }
        if (do_near && row == 0 && rows_s > 0) {
            for (int dc = -1; dc <= 1; ++dc) {
                int cs = cl + dc;
                if (cs < 0 || cs >= ncol) continue;
                int js = start[cs], je = end[cs];
                for (int j = js; j < je; ++j) {
                    double x0 = xs[j], y0 = ys[j];
                    cx<double> GL, GS;
                    pair_kernel_grad(nodes, nmid, npan, t0, y1, y0, fabs(x1 - x0), act, GL, GS);
                    double sg = x1 > x0 ? 1.0 : (x1 < x0 ? -1.0 : 0.0);
                    cx<double> GX = {-GL.im * sg, GL.re * sg};  // i sgn * GL
                    int64_t o = idx[j];
                    for (int r = r0; r < r0 + nr; ++r) {
                        cx<T> qq = q[(int64_t)r * ns + o];
                        cx<T> cr = act ? cw[(int64_t)r * nt + oi] : mk<T>(0, 0);
                        cx<double> cq = cx<double>{(double)cr.re, (double)cr.im} * cx<double>{(double)qq.re, (double)qq.im};
                        gx += cq.re * GX.re - cq.im * GX.im;
                        gy += cq.re * GS.re - cq.im * GS.im;
                    }
                }
            }
        }
        if (act) {
            gout[oi] = accumulate ? gout[oi] + gx : gx;
            gout[nt + oi] = accumulate ? gout[nt + oi] + ysign * gy : ysign * gy;
        }
    }
}

// Direct all-pairs sum (no tree): lanes over targets, loop over all sources.
// Direct sum over all pairs: block (target tile of 64, rhs chunk of 8,
// source chunk z) sums sources [z cs, (z + 1) cs) for its targets.  With one
// chunk it writes u; otherwise FP64 partials part[z][rhs][target], added in
// chunk order by k_direct_reduce.
template <typename T>
__global__ void __launch_bounds__(64) k_direct(const double *__restrict__ src, int64_t ns, const cx<T> *__restrict__ q,
                                               const double *__restrict__ tgt, int64_t nt, int nrhs,
                                               const Node *__restrict__ nodes, int nmid, int npan, double t0,
                                               int64_t cs, cx<double> *__restrict__ part, cx<T> *__restrict__ u)
{
    constexpr int RMAX = 8;
    int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int r0 = blockIdx.y * RMAX;
    const int nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    const int64_t j0 = (int64_t)blockIdx.z * cs, j1 = j0 + cs < ns ? j0 + cs : ns;
    bool act = i < nt;
    double x1 = act ? tgt[i] : tgt[0], y1 = act ? tgt[nt + i] : tgt[nt];
    cx<double> res[RMAX];
    for (int r = 0; r < RMAX; ++r) res[r] = {0.0, 0.0};
    for (int64_t j = j0; j < j1; ++j) {
        double x0 = src[j], y0 = src[ns + j];
        cx<double> G = pair_kernel(nodes, nmid, npan, t0, y1, y0, fabs(x1 - x0), act);
        for (int r = 0; r < RMAX; ++r)
            if (r < nr) {
                cx<T> qq = q[(int64_t)(r0 + r) * ns + j];
                cfma(res[r], G, cx<double>{(double)qq.re, (double)qq.im});
            }
    }
    if (!act) return;
    if (part) {
        for (int r = 0; r < RMAX; ++r)
            if (r < nr) part[((int64_t)blockIdx.z * nrhs + r0 + r) * nt + i] = res[r];
    } else {
        for (int r = 0; r < RMAX; ++r)
            if (r < nr) u[(int64_t)(r0 + r) * nt + i] = mk<T>((T)res[r].re, (T)res[r].im);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_direct_reduce(const cx<double> *__restrict__ part, int nchunk, int64_t m,
                                                       cx<T> *__restrict__ u)
{
    int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= m) return;
    cx<double> v = {0.0, 0.0};
    for (int z = 0; z < nchunk; ++z) v += part[(int64_t)z * m + o];
    u[o] = mk<T>((T)v.re, (T)v.im);
}


// Compute units and LDS bytes per compute unit of the current device.
struct DeviceShape {
    int cus = 256;
    int lds = 160 * 1024;
};
DeviceShape device_shape()
{
    static std::atomic<int> cus_cache[64], lds_cache[64];
    DeviceShape d;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return d;
    if (!cus_cache[dev].load()) {
        int v = 0, m = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = d.cus;
        if (hipDeviceGetAttribute(&m, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            m <= 0)
            m = d.lds;
        lds_cache[dev].store(m);
        cus_cache[dev].store(v);
    }
    d.cus = cus_cache[dev].load();
    d.lds = lds_cache[dev].load();
    return d;
}

// Leaves per block for a kernel of `threads` threads per block over nbox leaves
// holding npts points: the fewest blocks per compute unit (at most max_per_cu)
// that keep a block's points within 4/5 of its threads, then as many leaves
// per block as fill that many blocks on every compute unit.  A grid just
// under a multiple of the compute units balances the blocks per unit.
inline int leaves_per_block(int64_t nbox, int64_t npts, int threads, int max_per_cu)
{
    const DeviceShape dv = device_shape();
    int64_t k = (int64_t)std::ceil((double)npts / (0.8 * threads * dv.cus));
    k = k < 1 ? 1 : (k > max_per_cu ? max_per_cu : k);
    int64_t G = (nbox + k * dv.cus - 1) / (k * dv.cus);
    return (int)(G < 1 ? 1 : (G > LEAF_GMAX ? LEAF_GMAX : G));
}

template <typename T, int PMAX>
void p2m_dispatch(const int32_t *start, const int32_t *end, const double *xs, const double *ys, const void *qs,
                  int64_t ns, int nrhs, const Geometry &g, Medium med, cx<T> *M, hipStream_t st)
{
    const Level &lv = g.lev[g.L];
    int nbox = lv.rows_s * lv.ncol;
    if (nbox == 0) return;
    // points per chunk: as many as 78 KB of LDS hold (two blocks per compute
    // unit), at most P2M_CHMAX
    const size_t per = (size_t)(lv.nc + nrhs) * sizeof(cx<T>);
    int CH = (int)((78 * 1024) / per);
    CH = CH > P2M_CHMAX ? P2M_CHMAX : (CH < 1 ? 1 : CH);
    const size_t sh = (size_t)CH * per;
    int per_cu = (int)(device_shape().lds / (sh > 0 ? sh : 1));
    per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
    const int G = leaves_per_block(nbox, ns, CH < P2M_THREADS ? CH : P2M_THREADS, per_cu);
    cx<double> kd = k_src(med);
    cx<T> k1 = mk<T>((T)kd.re, (T)kd.im);
    T invR = (T)(M_SQRT2 / lv.w);
    LMFMM_LAUNCH((k_p2m<T, PMAX>), dim3((nbox + G - 1) / G), dim3(P2M_THREADS), sh, st, start, end, xs, ys,
                 reinterpret_cast<const cx<T> *>(qs), ns, nrhs, lv.P, nbox, lv.ncol, lv.col_lo, g.x_lo, lv.w, k1,
                 invR, G, CH, M + lv.off_s);
}

template <typename T, int PMAX>
void l2p_dispatch(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs, const double *ys,
                  const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g, Medium med, const cx<T> *Lc,
                  const LeafShift<T> &shift, const Node *nodes, int nmid, int npan, double t0, int do_far,
                  int do_near, const cx<double> *unear, int nparts, void *u, hipStream_t st)
{
    const Level &lv = g.lev[g.L];
    int nbox = lv.rows_t * lv.ncol;
    if (nbox == 0) return;
    size_t sh = (size_t)lv.nc * 8 * sizeof(cx<T>);
    cx<double> kd = k_tgt(med);
    cx<T> k2 = mk<T>((T)kd.re, (T)kd.im);
    T invR = (T)(M_SQRT2 / lv.w);
    int64_t key_t0 = (int64_t)lv.rows_s * lv.ncol;
    if (!(do_near && lv.rows_s > 0)) unear = nullptr;
    if (!do_near || unear || lv.rows_s == 0) {
        // far field plus, if any, the sweep's near-field parts: G leaves per block
        const int RM = nrhs == 1 ? 1 : 8;
        const size_t per_leaf = (size_t)RM * lv.nc * sizeof(cx<T>);
        // about 0.8 x 256 points per block, two blocks per compute unit: one
        // leaf per wave in the shift phase
        int G = leaves_per_block(nbox, nt, 256, 2);
        G = G > L2P_THREADS / 64 ? L2P_THREADS / 64 : G;
        const int gmax = (int)((48 * 1024) / per_leaf);
        G = G > gmax ? gmax : G;
        G = G < 1 ? 1 : G;
        const dim3 grid((nbox + G - 1) / G, (nrhs + RM - 1) / RM);
#define LMFMM_L2P_PACKED(RMC)                                                                                      \
    LMFMM_LAUNCH((k_l2p<T, PMAX, RMC>), grid, dim3(L2P_THREADS), G * per_leaf, st, start, end, idx, xs, ys, ns, nt, \
                 nrhs, lv.P, nbox, lv.ncol, lv.col_lo, g.x_lo, lv.w, k2, invR, Lc + lv.off_t, shift, key_t0, G,    \
                 do_far, unear, unear ? nparts : 0, reinterpret_cast<cx<T> *>(u))
        if (nrhs == 1)
            LMFMM_L2P_PACKED(1);
        else
            LMFMM_L2P_PACKED(8);
#undef LMFMM_L2P_PACKED
        return;
    }
    // near field by pairs: one leaf per block
#define LMFMM_L2P_LAUNCH(RM)                                                                                      \
    LMFMM_LAUNCH((k_l2p_near<T, PMAX, RM>), dim3(nbox, (nrhs + RM - 1) / RM), dim3(64), sh, st, start, end, idx, xs, \
                 ys, reinterpret_cast<const cx<T> *>(q), ns, nt, nrhs, lv.P, lv.ncol, lv.col_lo, lv.rows_s, g.x_lo,  \
                 lv.w, k2, invR, Lc + lv.off_t, shift, nodes, nmid, npan, t0, do_far, do_near, key_t0, unear, nparts,\
                 reinterpret_cast<cx<T> *>(u))
    if (nrhs == 1)
        LMFMM_L2P_LAUNCH(1);
    else
        LMFMM_L2P_LAUNCH(8);
#undef LMFMM_L2P_LAUNCH
}

template <typename T, int PMAX>
void grad_dispatch(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs, const double *ys,
                   const void *q, const void *cw, int64_t ns, int64_t nt, int nrhs, const Geometry &g, Medium med,
                   const cx<T> *Lc, const Node *nodes, int nmid, int npan, double t0, int do_far, int do_near,
                   double ysign, double *gout, hipStream_t st)
{
    const Level &lv = g.lev[g.L];
    int nbox = lv.rows_t * lv.ncol;
    if (nbox == 0) return;
    cx<double> kd = k_tgt(med);
    cx<T> kt = mk<T>((T)kd.re, (T)kd.im);
    T invR = (T)(M_SQRT2 / lv.w);
    int64_t key_t0 = (int64_t)lv.rows_s * lv.ncol;
    for (int r0 = 0; r0 < nrhs; r0 += 8) {
        int nr = nrhs - r0 < 8 ? nrhs - r0 : 8;
        size_t sh = (size_t)2 * nr * (2 * (lv.P + 1) + 1) * sizeof(cx<T>);
        LMFMM_LAUNCH((k_l2p_grad<T, PMAX>), dim3(nbox), dim3(64), sh, st, start, end, idx, xs, ys,
                           reinterpret_cast<const cx<T> *>(q), reinterpret_cast<const cx<T> *>(cw), ns, nt, nrhs, r0,
                           nr, r0 > 0 ? 1 : 0, lv.P, lv.ncol, lv.col_lo, lv.rows_s, g.x_lo, lv.w, kt, invR,
                           Lc + lv.off_t, nodes, nmid, npan, t0, do_far, do_near, key_t0, ysign, gout);
    }
}

}  // namespace

template <typename T>
void launch_p2m(const int32_t *start, const int32_t *end, const double *xs, const double *ys, const void *qs,
                int64_t ns, int nrhs, const Geometry &g, Medium med, cx<T> *M, hipStream_t st)
{
    int P = g.lev[g.L].P;
    if (P <= 16)
        p2m_dispatch<T, 16>(start, end, xs, ys, qs, ns, nrhs, g, med, M, st);
    else if (P <= 32)
        p2m_dispatch<T, 32>(start, end, xs, ys, qs, ns, nrhs, g, med, M, st);
    else if (P <= 64)
        p2m_dispatch<T, 64>(start, end, xs, ys, qs, ns, nrhs, g, med, M, st);
    else
        p2m_dispatch<T, 256>(start, end, xs, ys, qs, ns, nrhs, g, med, M, st);
}

template <typename T>
void launch_m2m(const Geometry &g, int lc, const cx<T> *tab, cx<T> *M, int nrhs, hipStream_t st)
{
    const Level &c = g.lev[lc], &p = g.lev[lc - 1];
    int nbox = p.rows_s * p.ncol;
    if (nbox == 0) return;
    LMFMM_LAUNCH((k_up<T>), dim3(nbox), dim3(256), 0, st, M + c.off_s, M + p.off_s, tab, nrhs, c.nc, p.nc,
                       c.ncol, c.col_lo, c.rows_s, p.ncol, p.col_lo);
}

template <typename T>
void launch_down(const Geometry &g, int l, const cx<T> *atab, const int *cls3, const int *row_off, int nrt,
                 const cx<T> *M, cx<T> *Lc, int nrhs, const cx<T> *l2l_tab, bool top, int add_rows, hipStream_t st)
{
    const Level &lv = g.lev[l], &pv = g.lev[l - 1];
    DownArgs a;
    a.nc = lv.nc;
    a.ncol = lv.ncol;
    a.col_lo = lv.col_lo;
    a.rows_s = lv.rows_s;
    a.rows_t = lv.rows_t;
    a.top = top ? 1 : 0;
    a.nrt = atab ? (nrt < lv.rows_t ? nrt : lv.rows_t) : 0;
    a.nb_m2l = a.nrt * lv.ncol;
    a.ncp = pv.nc;
    a.ncol_p = pv.ncol;
    a.col_lo_p = pv.col_lo;
    a.rows_t_p = pv.rows_t;
    a.has_l2l = l2l_tab != nullptr;
    a.add_rows = add_rows;
    int64_t rest = (int64_t)(lv.rows_t - a.nrt) * lv.ncol;
    int64_t nblk = a.nb_m2l + (a.has_l2l ? (rest + DW - 1) / DW : 0);
    if (nblk == 0) return;
    LMFMM_LAUNCH((k_down<T>), dim3((unsigned)nblk), dim3(64 * DW), 0, st, a, nrhs, Lc + pv.off_t, l2l_tab,
                       Lc + lv.off_t, M + lv.off_s, atab, cls3, row_off);
}

template <typename T>
void launch_m2l_all(const Geometry &g, int l0, int l1, const cx<T> *const *atab, const int *const *cls3,
                    const int *const *row_off, const int *nrt, const cx<T> *M, cx<T> *Lc, int nrhs, hipStream_t st)
{
    M2LLevels<T> a;
    a.n = 0;
    int blk = 0;
    for (int l = l0; l <= l1 && a.n < M2L_MAXLEV; ++l) {
        const Level &lv = g.lev[l];
        const int rows = nrt[l - l0] < lv.rows_t ? nrt[l - l0] : lv.rows_t;
        if (!atab[l - l0] || rows <= 0 || lv.ncol <= 0) continue;
        const int i = a.n++;
        a.blk0[i] = blk;
        a.nc[i] = lv.nc;
        a.ncol[i] = lv.ncol;
        a.col_lo[i] = lv.col_lo;
        a.rows_s[i] = lv.rows_s;
        a.top[i] = l == g.ltop;
        a.off_s[i] = lv.off_s;
        a.off_t[i] = lv.off_t;
        a.atab[i] = atab[l - l0];
        a.cls3[i] = cls3[l - l0];
        a.row_off[i] = row_off[l - l0];
        blk += rows * lv.ncol;
    }
    a.blk0[a.n] = blk;
    if (blk == 0) return;
    LMFMM_LAUNCH((k_m2l_all<T>), dim3(blk), dim3(64 * M2L_DW), 0, st, a, nrhs, M, Lc);
}

template <typename T>
int launch_near_sweep(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs,
                      const double *ys, const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g,
                      const Node *nodes, int nmid, int npan, double t0, cx<double> *unear, hipStream_t st)
{
    const Level &lv = g.lev[g.L];
    if (lv.rows_t == 0 || lv.rows_s == 0 || lv.ncol == 0) return 0;
    const int nnodes = nmid + 2 * NGL * npan;
    // node groups of 64 over up to 4 parts of SW_W waves; segments of leaf
    // columns long enough to share the sources, short enough for about two
    // thousand blocks
    const int RM = nrhs == 1 ? 1 : 8;
    const int G = RM == 1 ? SweepCap<1>::G : SweepCap<8>::G;
    const int nunits = ((nnodes + 63) / 64 + G - 1) / G;
    int nparts = (nunits + SW_W - 1) / SW_W;
    nparts = nparts < 1 ? 1 : (nparts > 4 ? 4 : nparts);
    const int nrc = (nrhs + RM - 1) / RM;
    int64_t seg = (int64_t)lv.ncol * nrc * nparts / 2048;
    const int seglen = seg < 1 ? 1 : (seg > 16 ? 16 : (int)seg);
    const int nseg = (lv.ncol + seglen - 1) / seglen;
#define LMFMM_SWEEP_LAUNCH(R)                                                                                     \
    LMFMM_LAUNCH((k_near_sweep<T, R>), dim3(nseg, nrc, nparts), dim3(64 * SW_W), 0, st, start, end, idx, xs, ys,  \
                 reinterpret_cast<const cx<T> *>(q), ns, nt, nrhs, lv.ncol, (int64_t)lv.rows_s * lv.ncol, seglen, \
                 g.x_lo + lv.col_lo * lv.w, lv.w,                                                                  \
                 nodes, nnodes, nmid, npan, t0, nparts, unear)
    if (RM == 1)
        LMFMM_SWEEP_LAUNCH(1);
    else
        LMFMM_SWEEP_LAUNCH(8);
#undef LMFMM_SWEEP_LAUNCH
    return nparts;
}

template <typename T>
void launch_l2p_near(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs,
                     const double *ys, const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g,
                     Medium med, const cx<T> *Lc, const LeafShift<T> &shift, const Node *nodes, int nmid, int npan,
                     double t0, int do_far, int do_near, const cx<double> *unear, int nparts, void *u, hipStream_t st)
{
    int P = g.lev[g.L].P;
    if (!unear) nparts = 0;
#define LMFMM_L2P(PM)                                                                                          \
    l2p_dispatch<T, PM>(start, end, idx, xs, ys, q, ns, nt, nrhs, g, med, Lc, shift, nodes, nmid, npan, t0, \
                        do_far, do_near, unear, nparts, u, st)
    if (P <= 16)
        LMFMM_L2P(16);
    else if (P <= 32)
        LMFMM_L2P(32);
    else if (P <= 64)
        LMFMM_L2P(64);
    else
        LMFMM_L2P(256);
#undef LMFMM_L2P
}

template <typename T>
void launch_l2p_grad(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs,
                     const double *ys, const void *q, const void *cw, int64_t ns, int64_t nt, int nrhs,
                     const Geometry &g, Medium med, const cx<T> *Lc, const Node *nodes, int nmid, int npan, double t0,
                     int do_far, int do_near, double ysign, double *gout, hipStream_t st)
{
    int P = g.lev[g.L].P + 1;
#define LMFMM_GR(PM)                                                                                             \
    grad_dispatch<T, PM>(start, end, idx, xs, ys, q, cw, ns, nt, nrhs, g, med, Lc, nodes, nmid, npan, t0, do_far, \
                         do_near, ysign, gout, st)
    if (P <= 16)
        LMFMM_GR(16);
    else if (P <= 32)
        LMFMM_GR(32);
    else if (P <= 64)
        LMFMM_GR(64);
    else
        LMFMM_GR(256);
#undef LMFMM_GR
}

int direct_chunks(int64_t ns, int64_t nt, int nrhs)
{
    // enough blocks to fill the GPU, at least 256 sources per chunk, and at
    // most 256 MiB of partials
    int64_t tiles = ((nt + 63) / 64) * ((nrhs + 7) / 8);
    int64_t z = (2048 + tiles - 1) / tiles;
    int64_t zmax = (ns + 255) / 256;
    int64_t zmem = ((int64_t)256 << 20) / std::max<int64_t>(1, nt * nrhs * 16);
    z = std::min(z, std::min(zmax, zmem));
    return (int)std::max<int64_t>(1, z);
}

void launch_direct(const double *src, int64_t ns, const void *q, const double *tgt, int64_t nt, int nrhs, int prec,
                   const Node *nodes, int nmid, int npan, double t0, int nchunk, cx<double> *part, void *u,
                   hipStream_t st)
{
    if (nt == 0) return;
    int64_t cs = (ns + nchunk - 1) / nchunk;
    dim3 grid((unsigned)((nt + 63) / 64), (unsigned)((nrhs + 7) / 8), (unsigned)nchunk);
    cx<double> *pp = nchunk > 1 ? part : nullptr;
    const int64_t m = nt * nrhs;
    if (prec == 0) {
        hipLaunchKernelGGL((k_direct<double>), grid, dim3(64), 0, st, src, ns,
                           reinterpret_cast<const cx<double> *>(q), tgt, nt, nrhs, nodes, nmid, npan, t0, cs, pp,
                           reinterpret_cast<cx<double> *>(u));
        if (pp)
            hipLaunchKernelGGL((k_direct_reduce<double>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, pp,
                               nchunk, m, reinterpret_cast<cx<double> *>(u));
    } else {
        hipLaunchKernelGGL((k_direct<float>), grid, dim3(64), 0, st, src, ns, reinterpret_cast<const cx<float> *>(q),
                           tgt, nt, nrhs, nodes, nmid, npan, t0, cs, pp, reinterpret_cast<cx<float> *>(u));
        if (pp)
            hipLaunchKernelGGL((k_direct_reduce<float>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, pp,
                               nchunk, m, reinterpret_cast<cx<float> *>(u));
    }
}

#define LMFMM_INST(T)                                                                                               \
    template void launch_p2m<T>(const int32_t *, const int32_t *, const double *, const double *, const void *,      \
                                int64_t, int, const Geometry &, Medium, cx<T> *, hipStream_t);                      \
    template void launch_m2m<T>(const Geometry &, int, const cx<T> *, cx<T> *, int, hipStream_t);                   \
    template void launch_down<T>(const Geometry &, int, const cx<T> *, const int *, const int *, int, const cx<T> *, \
                                 cx<T> *, int, const cx<T> *, bool, int, hipStream_t);                              \
    template void launch_m2l_all<T>(const Geometry &, int, int, const cx<T> *const *, const int *const *,           \
                                    const int *const *, const int *, const cx<T> *, cx<T> *, int, hipStream_t);     \
    template int launch_near_sweep<T>(const int32_t *, const int32_t *, const int32_t *, const double *,            \
                                      const double *, const void *, int64_t, int64_t, int, const Geometry &,        \
                                      const Node *, int, int, double, cx<double> *, hipStream_t);                   \
    template void launch_l2p_near<T>(const int32_t *, const int32_t *, const int32_t *, const double *,             \
                                     const double *, const void *, int64_t, int64_t, int, const Geometry &, Medium, \
                                     const cx<T> *, const LeafShift<T> &, const Node *, int, int, double, int, int, \
                                     const cx<double> *, int, void *, hipStream_t);                                 \
    template void launch_l2p_grad<T>(const int32_t *, const int32_t *, const int32_t *, const double *,             \
                                     const double *, const void *, const void *, int64_t, int64_t, int,             \
                                     const Geometry &, Medium, const cx<T> *, const Node *, int, int, double, int,  \
                                     int, double, double *, hipStream_t);
LMFMM_INST(double)
LMFMM_INST(float)

}  // namespace lmfmm
