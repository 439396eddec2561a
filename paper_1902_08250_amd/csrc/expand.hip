// FMM passes on the uniform interface-split quadtree (Algorithm 1, Steps 2-4).
//
//  * P2M  (source-to-multipole, Definition "Multipole Expansion"): per source
//    leaf, M_q = sum_j q_j J_q(k1 r_j) e^{-i q theta_j}, stored scaled.
//  * M2M  (Lemma M2M): free-space Helmholtz shift with k1, 4 children -> parent.
//  * M2L + L2L (Lemma M2L, Lemma L2L): at each level, every target box in the
//    two rows nearest the interface gathers its interaction list through the
//    Sommerfeld translation tables; every target box also receives its
//    parent's local expansion shifted with the free-space operator for k2.
//  * L2P + S2T (Definition "Local Expansion"; direct interactions): per
//    target leaf, the local expansion is evaluated at the targets and the
//    adjacent source leaves across the interface are summed by contour
//    quadrature of g_2^t.
//
// Expansions are stored scaled: Mhat_q = s_q M_q and Lhat_p = L_p / s_p with
// s_q = |q|! (2/(k R))^|q|, R the box half-diagonal, which keeps FP32 in
// range.  Layout: [box][rhs][2P+1] complex, box = row * ncol + column.
#include "lmfmm_internal.h"

namespace lmfmm {

namespace {

// ---------------------------------------------------------------------------
// P2M: one wave per source leaf; lanes over points, then lanes over outputs.
// ---------------------------------------------------------------------------
template <typename T, int PMAX>
__global__ void __launch_bounds__(64) k_p2m(const int32_t *__restrict__ start, const int32_t *__restrict__ end,
                                            const int32_t *__restrict__ idx, const double *__restrict__ xs,
                                            const double *__restrict__ ys, const cx<T> *__restrict__ q, int64_t ns,
                                            int nrhs, int P, int ncol, int col_lo, double x_lo, double w, cx<T> k1,
                                            T invR, int CH, cx<T> *__restrict__ M)
{
    extern __shared__ unsigned char smem_raw[];
    const int nc = 2 * P + 1;
    cx<T> *B = reinterpret_cast<cx<T> *>(smem_raw);  // [CH][nc]
    cx<T> *Q = B + CH * nc;                          // [CH][nrhs]
    const int box = blockIdx.x, lane = threadIdx.x;
    const int row = box / ncol, col = col_lo + box % ncol;
    const double cxp = x_lo + (col + 0.5) * w, cyp = (row + 0.5) * w;
    const int s = start[box], e = end[box];
    const int nout = nc * nrhs;
    cx<T> *Mb = M + (int64_t)box * nout;
    bool first = true;
    for (int c0 = s; c0 < e || first; c0 += CH) {
        int j = c0 + lane;
        bool act = lane < CH && j < e;
        if (act) {
            T X = (T)(xs[j] - cxp), Y = (T)(ys[j] - cyp);
            bessel_basis<T, PMAX>(k1, X, Y, invR, P, -1, B + lane * nc, 1);
            int64_t o = idx[j];
            for (int r = 0; r < nrhs; ++r) Q[lane * nrhs + r] = q[(int64_t)r * ns + o];
        }
        __syncthreads();
        int cnt = e - c0 < CH ? e - c0 : CH;
        if (cnt < 0) cnt = 0;
        for (int o = lane; o < nout; o += 64) {
            int t = o % nc, r = o / nc;
            cx<T> acc = mk<T>(0, 0);
            for (int jj = 0; jj < cnt; ++jj) cfma(acc, B[jj * nc + t], Q[jj * nrhs + r]);
            Mb[r * nc + t] = first ? acc : Mb[r * nc + t] + acc;
        }
        __syncthreads();
        first = false;
    }
}

// ---------------------------------------------------------------------------
// M2M: one wave per parent box at level lp = lc - 1.
// tab: [4 children][nc_child][nc_parent] (transposed for coalesced reads).
// Child position c = 2*dy + dx (dx: column parity, dy: row parity).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) k_m2m(const cx<T> *__restrict__ Mc, cx<T> *__restrict__ Mp,
                                            const cx<T> *__restrict__ tab, int nrhs, int ncc, int ncp, int ncol_c,
                                            int col_lo_c, int rows_c, int ncol_p, int col_lo_p)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *C = reinterpret_cast<cx<T> *>(smem_raw);  // [4][ncc]
    const int box = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
    const int prow = box / ncol_p, pcol = col_lo_p + box % ncol_p;
    for (int c = 0; c < 4; ++c) {
        int dx = c & 1, dy = c >> 1;
        int crow = 2 * prow + dy, ccol = 2 * pcol + dx - col_lo_c;
        bool ok = crow < rows_c && ccol >= 0 && ccol < ncol_c;
        const cx<T> *src = Mc + (((int64_t)crow * ncol_c + ccol) * nrhs + r) * ncc;
        for (int t = lane; t < ncc; t += 64) C[c * ncc + t] = ok ? src[t] : mk<T>(0, 0);
    }
    __syncthreads();
    for (int n = lane; n < ncp; n += 64) {
        cx<T> acc = mk<T>(0, 0);
        for (int c = 0; c < 4; ++c) {
            const cx<T> *tc = tab + (int64_t)c * ncc * ncp;
            const cx<T> *mc = C + c * ncc;
            for (int k = 0; k < ncc; ++k) cfma(acc, tc[(int64_t)k * ncp + n], mc[k]);
        }
        Mp[((int64_t)box * nrhs + r) * ncp + n] = acc;
    }
}

// ---------------------------------------------------------------------------
// Fused L2L + M2L at level l: one wave per target box.
// l2l: [4 child positions][nc_parent][nc] or null at the top level.
// atab: M2L tables, [class][nc (q)][nc (p)]; cls_index[(rt*2+rs)*7 + dcol+3]
// gives the class slot or -1.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) k_m2l_l2l(const cx<T> *__restrict__ Ms, const cx<T> *__restrict__ Lp,
                                                cx<T> *__restrict__ Lc, const cx<T> *__restrict__ atab,
                                                const int *__restrict__ cls_index, const cx<T> *__restrict__ l2l,
                                                int nrhs, int nc, int ncp, int ncol, int col_lo, int rows_s,
                                                int ncol_p, int col_lo_p, int do_m2l)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *S = reinterpret_cast<cx<T> *>(smem_raw);  // [max(nc, ncp)]
    const int box = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
    const int row = box / ncol, cl = box % ncol, col = col_lo + cl;
    constexpr int MAXACC = 16;  // nc <= 1024
    cx<T> acc[MAXACC];
    for (int a = 0; a < MAXACC; ++a) acc[a] = mk<T>(0, 0);
    // L2L from the parent
    if (l2l) {
        int prow = row >> 1, pcol = (col >> 1) - col_lo_p;
        int c = ((row & 1) << 1) | (col & 1);
        const cx<T> *src = Lp + (((int64_t)prow * ncol_p + pcol) * nrhs + r) * ncp;
        for (int t = lane; t < ncp; t += 64) S[t] = src[t];
        __syncthreads();
        const cx<T> *tc = l2l + (int64_t)c * ncp * nc;
#pragma unroll
        for (int a = 0; a < MAXACC; ++a) {
            int p = lane + 64 * a;
            if (p < nc)
                for (int k = 0; k < ncp; ++k) cfma(acc[a], tc[(int64_t)k * nc + p], S[k]);
        }
        __syncthreads();
    }
    // M2L from the interaction list (only the two rows next to the interface)
    if (do_m2l && row < 2) {
        for (int rs = 0; rs < 2 && rs < rows_s; ++rs) {
            for (int dc = -3; dc <= 3; ++dc) {
                int slot = cls_index[(row * 2 + rs) * 7 + dc + 3];
                if (slot < 0) continue;
                int cs = col + dc;
                int dp = (cs >> 1) - (col >> 1);
                if (dp > 1 || dp < -1) continue;
                int csl = cs - col_lo;
                if (csl < 0 || csl >= ncol) continue;
                const cx<T> *src = Ms + (((int64_t)rs * ncol + csl) * nrhs + r) * nc;
                for (int t = lane; t < nc; t += 64) S[t] = src[t];
                __syncthreads();
                const cx<T> *A = atab + (int64_t)slot * nc * nc;
#pragma unroll
                for (int a = 0; a < MAXACC; ++a) {
                    int p = lane + 64 * a;
                    if (p < nc)
                        for (int k = 0; k < nc; ++k) cfma(acc[a], A[(int64_t)k * nc + p], S[k]);
                }
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int a = 0; a < MAXACC; ++a) {
        int p = lane + 64 * a;
        if (p < nc) Lc[((int64_t)box * nrhs + r) * nc + p] = acc[a];
    }
}

// ---------------------------------------------------------------------------
// Near-field pair sum: G = sum over nodes of D_n exp(s2_n y1 - s1_n y0 + i lam_n dx).
// Nodes: nmid on the finite piece, then panels of 2*NGL nodes (right and left
// ray) of geometrically growing length; panel m starts at t0 2^(m-1).
// ---------------------------------------------------------------------------
__device__ inline cx<double> node_term(const Node &nd, double y1, double y0, double dx)
{
    double er = nd.s2r * y1 - nd.s1r * y0 - nd.li * dx;
    double ei = nd.s2i * y1 - nd.s1i * y0 + nd.lr * dx;
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
// Fused L2P + S2T per target leaf; lanes over targets (chunks of 64).
// Writes u[r][original index] (no accumulation across kernels).
// ---------------------------------------------------------------------------
template <typename T, int PMAX>
__global__ void __launch_bounds__(64) k_l2p_near(const int32_t *__restrict__ start, const int32_t *__restrict__ end,
                                                 const int32_t *__restrict__ idx, const double *__restrict__ xs,
                                                 const double *__restrict__ ys, const cx<T> *__restrict__ q,
                                                 int64_t ns, int64_t nt, int nrhs, int P, int ncol, int col_lo,
                                                 int rows_s, double x_lo, double w, cx<T> k2, T invR,
                                                 const cx<T> *__restrict__ Lc, const Node *__restrict__ nodes,
                                                 int nmid, int npan, double t0, int do_far, int do_near,
                                                 int64_t key_t0, cx<T> *__restrict__ u)
{
    constexpr int RMAX = 8;
    extern __shared__ unsigned char smem_raw[];
    const int nc = 2 * P + 1;
    cx<T> *Ls = reinterpret_cast<cx<T> *>(smem_raw);  // [RMAX][nc]
    const int box = blockIdx.x, lane = threadIdx.x;
    const int r0 = blockIdx.y * RMAX;
    const int nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    const int row = box / ncol, cl = box % ncol, col = col_lo + cl;
    const double cxp = x_lo + (col + 0.5) * w, cyp = -(row + 0.5) * w;
    const int s = start[key_t0 + box], e = end[key_t0 + box];
    if (e <= s) return;
    if (do_far) {
        for (int r = 0; r < nr; ++r)
            for (int t = lane; t < nc; t += 64) Ls[r * nc + t] = Lc[((int64_t)box * nrhs + r0 + r) * nc + t];
        __syncthreads();
    }
    for (int c0 = s; c0 < e; c0 += 64) {
        int i = c0 + lane;
        bool act = i < e;
        int ii = act ? i : s;
        double x1 = xs[ii], y1 = ys[ii];
        cx<double> res[RMAX];
        for (int r = 0; r < RMAX; ++r) res[r] = {0.0, 0.0};
        if (do_far) {
            cx<T> tm[PMAX + 1];
            cx<T> J0;
            T X = (T)(x1 - cxp), Y = (T)(y1 - cyp);
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
        if (do_near && row == 0 && rows_s > 0) {
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
        if (act) {
            int64_t o = idx[i] - ns;
            for (int r = 0; r < RMAX; ++r)
                if (r < nr) u[(int64_t)(r0 + r) * nt + o] = mk<T>((T)res[r].re, (T)res[r].im);
        }
    }
}

// Direct all-pairs sum (no tree): lanes over targets, loop over all sources.
template <typename T>
__global__ void __launch_bounds__(64) k_direct(const double *__restrict__ src, int64_t ns, const cx<T> *__restrict__ q,
                                               const double *__restrict__ tgt, int64_t nt, int nrhs,
                                               const Node *__restrict__ nodes, int nmid, int npan, double t0,
                                               cx<T> *__restrict__ u)
{
    constexpr int RMAX = 8;
    int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int r0 = blockIdx.y * RMAX;
    const int nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    bool act = i < nt;
    double x1 = act ? tgt[i] : tgt[0], y1 = act ? tgt[nt + i] : tgt[nt];
    cx<double> res[RMAX];
    for (int r = 0; r < RMAX; ++r) res[r] = {0.0, 0.0};
    for (int64_t j = 0; j < ns; ++j) {
        double x0 = src[j], y0 = src[ns + j];
        cx<double> G = pair_kernel(nodes, nmid, npan, t0, y1, y0, fabs(x1 - x0), act);
        for (int r = 0; r < RMAX; ++r)
            if (r < nr) {
                cx<T> qq = q[(int64_t)(r0 + r) * ns + j];
                cfma(res[r], G, cx<double>{(double)qq.re, (double)qq.im});
            }
    }
    if (act)
        for (int r = 0; r < RMAX; ++r)
            if (r < nr) u[(int64_t)(r0 + r) * nt + i] = mk<T>((T)res[r].re, (T)res[r].im);
}

template <typename T, int PMAX>
void p2m_dispatch(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs, const double *ys,
                  const void *q, int64_t ns, int nrhs, const Geometry &g, Medium med, cx<T> *M, hipStream_t st)
{
    const Level &lv = g.lev[g.L];
    int nbox = lv.rows_s * lv.ncol;
    if (nbox == 0) return;
    int CH = (int)((60 * 1024) / ((size_t)(lv.nc + nrhs) * sizeof(cx<T>)));
    CH = CH > 64 ? 64 : (CH < 1 ? 1 : CH);
    size_t sh = (size_t)CH * (lv.nc + nrhs) * sizeof(cx<T>);
    cx<T> k1 = mk<T>((T)med.k1.re, (T)med.k1.im);
    T invR = (T)(M_SQRT2 / lv.w);
    hipLaunchKernelGGL((k_p2m<T, PMAX>), dim3(nbox), dim3(64), sh, st, start, end, idx, xs, ys,
                       reinterpret_cast<const cx<T> *>(q), ns, nrhs, lv.P, lv.ncol, lv.col_lo, g.x_lo, lv.w, k1, invR,
                       CH, M + lv.off_s);
}

template <typename T, int PMAX>
void l2p_dispatch(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs, const double *ys,
                  const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g, Medium med, const cx<T> *Lc,
                  const Node *nodes, int nmid, int npan, double t0, int do_far, int do_near, void *u, hipStream_t st)
{
    const Level &lv = g.lev[g.L];
    int nbox = lv.rows_t * lv.ncol;
    if (nbox == 0) return;
    size_t sh = (size_t)lv.nc * 8 * sizeof(cx<T>);
    cx<T> k2 = mk<T>((T)med.k2.re, (T)med.k2.im);
    T invR = (T)(M_SQRT2 / lv.w);
    int64_t key_t0 = (int64_t)lv.rows_s * lv.ncol;
    hipLaunchKernelGGL((k_l2p_near<T, PMAX>), dim3(nbox, (nrhs + 7) / 8), dim3(64), sh, st, start, end, idx, xs, ys,
                       reinterpret_cast<const cx<T> *>(q), ns, nt, nrhs, lv.P, lv.ncol, lv.col_lo, lv.rows_s, g.x_lo,
                       lv.w, k2, invR, Lc + lv.off_t, nodes, nmid, npan, t0, do_far, do_near, key_t0,
                       reinterpret_cast<cx<T> *>(u));
}

}  // namespace

template <typename T>
void launch_p2m(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs, const double *ys,
                const void *q, int64_t ns, int nrhs, const Geometry &g, Medium med, cx<T> *M, hipStream_t st)
{
    int P = g.lev[g.L].P;
    if (P <= 16)
        p2m_dispatch<T, 16>(start, end, idx, xs, ys, q, ns, nrhs, g, med, M, st);
    else if (P <= 32)
        p2m_dispatch<T, 32>(start, end, idx, xs, ys, q, ns, nrhs, g, med, M, st);
    else if (P <= 64)
        p2m_dispatch<T, 64>(start, end, idx, xs, ys, q, ns, nrhs, g, med, M, st);
    else
        p2m_dispatch<T, 256>(start, end, idx, xs, ys, q, ns, nrhs, g, med, M, st);
}

template <typename T>
void launch_m2m(const Geometry &g, int lc, const cx<T> *tab, cx<T> *M, int nrhs, hipStream_t st)
{
    const Level &c = g.lev[lc], &p = g.lev[lc - 1];
    int nbox = p.rows_s * p.ncol;
    if (nbox == 0) return;
    size_t sh = (size_t)4 * c.nc * sizeof(cx<T>);
    hipLaunchKernelGGL((k_m2m<T>), dim3(nbox, nrhs), dim3(64), sh, st, M + c.off_s, M + p.off_s, tab, nrhs, c.nc, p.nc,
                       c.ncol, c.col_lo, c.rows_s, p.ncol, p.col_lo);
}

template <typename T>
void launch_m2l(const Geometry &g, int l, const cx<T> *atab, const int *cls_index, const cx<T> *M, cx<T> *Lc,
                int nrhs, const cx<T> *l2l_tab, int do_m2l, hipStream_t st)
{
    const Level &lv = g.lev[l], &pv = g.lev[l - 1];
    int nbox = lv.rows_t * lv.ncol;
    if (nbox == 0) return;
    int ncmax = lv.nc > pv.nc ? lv.nc : pv.nc;
    size_t sh = (size_t)ncmax * sizeof(cx<T>);
    hipLaunchKernelGGL((k_m2l_l2l<T>), dim3(nbox, nrhs), dim3(64), sh, st, M + lv.off_s, Lc + pv.off_t, Lc + lv.off_t, atab,
                       cls_index, l2l_tab, nrhs, lv.nc, pv.nc, lv.ncol, lv.col_lo, lv.rows_s, pv.ncol, pv.col_lo,
                       do_m2l);
}

template <typename T>
void launch_l2p_near(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs,
                     const double *ys, const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g,
                     Medium med, const cx<T> *Lc, const Node *nodes, int nmid, int npan, double t0, int do_far,
                     int do_near, void *u, hipStream_t st)
{
    int P = g.lev[g.L].P;
    if (P <= 16)
        l2p_dispatch<T, 16>(start, end, idx, xs, ys, q, ns, nt, nrhs, g, med, Lc, nodes, nmid, npan, t0, do_far,
                            do_near, u, st);
    else if (P <= 32)
        l2p_dispatch<T, 32>(start, end, idx, xs, ys, q, ns, nt, nrhs, g, med, Lc, nodes, nmid, npan, t0, do_far,
                            do_near, u, st);
    else if (P <= 64)
        l2p_dispatch<T, 64>(start, end, idx, xs, ys, q, ns, nt, nrhs, g, med, Lc, nodes, nmid, npan, t0, do_far,
                            do_near, u, st);
    else
        l2p_dispatch<T, 256>(start, end, idx, xs, ys, q, ns, nt, nrhs, g, med, Lc, nodes, nmid, npan, t0, do_far,
                             do_near, u, st);
}

void launch_direct(const double *src, int64_t ns, const void *q, const double *tgt, int64_t nt, int nrhs, int prec,
                   const Node *nodes, int nmid, int npan, double t0, void *u, hipStream_t st)
{
    if (nt == 0) return;
    dim3 grid((unsigned)((nt + 63) / 64), (unsigned)((nrhs + 7) / 8));
    if (prec == 0)
        hipLaunchKernelGGL((k_direct<double>), grid, dim3(64), 0, st, src, ns,
                           reinterpret_cast<const cx<double> *>(q), tgt, nt, nrhs, nodes, nmid, npan, t0,
                           reinterpret_cast<cx<double> *>(u));
    else
        hipLaunchKernelGGL((k_direct<float>), grid, dim3(64), 0, st, src, ns, reinterpret_cast<const cx<float> *>(q),
                           tgt, nt, nrhs, nodes, nmid, npan, t0, reinterpret_cast<cx<float> *>(u));
}

#define LMFMM_INST(T)                                                                                               \
    template void launch_p2m<T>(const int32_t *, const int32_t *, const int32_t *, const double *, const double *,   \
                                const void *, int64_t, int, const Geometry &, Medium, cx<T> *, hipStream_t);        \
    template void launch_m2m<T>(const Geometry &, int, const cx<T> *, cx<T> *, int, hipStream_t);                   \
    template void launch_m2l<T>(const Geometry &, int, const cx<T> *, const int *, const cx<T> *, cx<T> *, int,     \
                                const cx<T> *, int, hipStream_t);                                                   \
    template void launch_l2p_near<T>(const int32_t *, const int32_t *, const int32_t *, const double *,             \
                                     const double *, const void *, int64_t, int64_t, int, const Geometry &, Medium, \
                                     const cx<T> *, const Node *, int, int, double, int, int, void *, hipStream_t);
LMFMM_INST(double)
LMFMM_INST(float)

}  // namespace lmfmm
