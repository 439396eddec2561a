// Quadrature-node tables (Algorithm 1, Step 1: "precompute necessary tables").
//
//  * Near-field table: on a contour fixed per plan and tree, the FP64 values
//    lambda_n, s1(lambda_n), s2(lambda_n) and D_n = weight_n sigma / (4 pi s2)
//    (sigma and s2 = the target layer's root of the plan's field component;
//    sigma_2^t and the middle layer's root by default).
//  * M2L translation matrices (Lemma M2L, the remark on precomputing A per
//    level): for a translation class with target centre (x_t, y_t) and source
//    centre (x_s, y_s),
//      Ahat_{p,q} = Int That_p(lam) Shat_q(lam) e^{s2 y_t - s1 y_s + i lam (x_t - x_s)}
//                       sigma_2^t / (4 pi s2) d lam,
//      That_p = (i (lam - s2) R/2)^p / p!,   That_{-m} = (-i (lam + s2) R/2)^m / m!,
//      Shat_q = (-i (lam + s1) R/2)^q / q!,  Shat_{-m} = ( i (lam - s1) R/2)^m / m!,
//    i.e. A_{p,q} of the lemma with the expansion scalings folded in.  The
//    integral is a sum over the class's contour nodes, so the table is the
//    contraction That * diag(D) * Shat over nodes.
#include "lmfmm_internal.h"

namespace lmfmm {

namespace {

__global__ void __launch_bounds__(256) k_node_table(const double *__restrict__ lamw, int n, Medium med,
                                                    Node *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cx<double> lam = {lamw[4 * i], lamw[4 * i + 1]};
    cx<double> wt = {lamw[4 * i + 2], lamw[4 * i + 3]};
    cx<double> s1 = sroot_d(lam, med.k1), s2 = sroot_d(lam, k_target_layer(med));
    cx<double> sg = sigma_d(lam, med, s1);
    cx<double> D = cdiv(wt * sg, (4.0 * M_PI) * s2);
    cx<double> ss = med.adj ? s2 : s1, stt = med.adj ? s1 : s2;
    Node nd;
    nd.lr = lam.re;
    nd.li = lam.im;
    nd.ssr = ss.re;
    nd.ssi = ss.im;
    nd.str = stt.re;
    nd.sti = stt.im;
    nd.dr = D.re;
    nd.di = D.im;
    out[i] = nd;
}

// lam +- s without cancellation: the larger of the two is formed directly and
// the other from (lam + s)(lam - s) = k^2.
__device__ inline void plus_minus(cx<double> lam, cx<double> s, cx<double> k, cx<double> &a, cx<double> &b)
{
    a = lam + s;
    b = lam - s;
    if (cabs2(a) >= cabs2(b))
        b = cdiv(k * k, a);
    else
        a = cdiv(k * k, b);
}

// One thread per node of any class.  cls_geo[c] = {dx_c, y_t, y_s, R}.
__global__ void __launch_bounds__(256) k_m2l_factors(const double *__restrict__ lamw,
                                                     const int *__restrict__ node_cls,
                                                     const int *__restrict__ node_local, int ntot,
                                                     const double *__restrict__ cls_geo, Medium med,
                                                     const int *__restrict__ cls_P, const int *__restrict__ cls_Q,
                                                     const int64_t *__restrict__ cls_toff,
                                                     cx<double> *__restrict__ Tm, cx<double> *__restrict__ Sm)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    int c = node_cls[i], n = node_local[i];
    int P = cls_P[c], Q = cls_Q[c], nc = 2 * P + 1;
    double dxc = cls_geo[4 * c], yt = cls_geo[4 * c + 1], ys = cls_geo[4 * c + 2], R = cls_geo[4 * c + 3];
    cx<double> lam = {lamw[4 * i], lamw[4 * i + 1]};
    cx<double> wt = {lamw[4 * i + 2], lamw[4 * i + 3]};
    cx<double> s1 = sroot_d(lam, med.k1), s2 = sroot_d(lam, k_target_layer(med));
    cx<double> sg = sigma_d(lam, med, s1);
    // source side (multipole, Shat) and target side (local, That); s2 is the
    // target layer's root (k2 for the middle layer)
    cx<double> ss = med.adj ? s2 : s1, stt = med.adj ? s1 : s2;
    cx<double> E = cexp_d(stt * yt - ss * ys + mk(-lam.im * dxc, lam.re * dxc));
    cx<double> D = cdiv(wt * E * sg, (4.0 * M_PI) * s2);
    cx<double> a1, b1, a2, b2;
    plus_minus(lam, ss, k_src(med), a1, b1);
    plus_minus(lam, stt, k_tgt(med), a2, b2);
    double hR = 0.5 * R;
    cx<double> I1 = {0.0, 1.0};
    cx<double> tp = (I1 * b2) * hR, tn = (-I1 * a2) * hR;  // That ratios
    cx<double> sp = (-I1 * a1) * hR, sn = (I1 * b1) * hR;  // Shat ratios
    cx<double> *T = Tm + cls_toff[c];                      // [nc][Q]
    cx<double> *S = Sm + cls_toff[c];                      // [Q][nc]
    T[(int64_t)P * Q + n] = mk(1.0, 0.0);
    S[(int64_t)n * nc + P] = D;
    cx<double> vtp = mk(1.0, 0.0), vtn = mk(1.0, 0.0), vsp = D, vsn = D;
    for (int m = 1; m <= P; ++m) {
        double im = 1.0 / m;
        vtp = vtp * (tp * im);
        vtn = vtn * (tn * im);
        vsp = vsp * (sp * im);
        vsn = vsn * (sn * im);
        T[(int64_t)(P + m) * Q + n] = vtp;
        T[(int64_t)(P - m) * Q + n] = vtn;
        S[(int64_t)n * nc + P + m] = vsp;
        S[(int64_t)n * nc + P - m] = vsn;
    }
}

// Ahat[c][q][p] = sum_n T[c][p][n] S[c][n][q] (the contraction over the
// class's quadrature nodes in Lemma M2L) on the FP64 matrix cores: a block of
// CW waves per 16 x 16 output tile, wave w taking the steps of four nodes
// w, w + CW, ... (CU steps' operands loaded together), v_mfma_f64_16x16x4f64
// with the complex product as four real products into two accumulators; the
// waves' sums are added in wave order through LDS.  Operand layout of that
// instruction: lane l supplies row l % 16, column l / 16 of the 16 x 4 left
// factor and row l / 16, column l % 16 of the 4 x 16 right factor; its register
// v returns entry (l / 16 + 4 v, l % 16) of the product.  Writes FP64 and FP32
// copies.
//
// Blocks are numbered so that all tiles of a class go to the same XCD (the
// dispatcher deals consecutive blocks to the eight XCDs in turn): block b
// takes class ((b / 8) / tiles^2) * 8 + b % 8 and tile (b / 8) % tiles^2, so
// the class's factor columns come from HBM into one L2 once.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int CT = 16, CW = 4, CU = 8, NXCD = 8;
__global__ void __launch_bounds__(64 * CW) k_m2l_contract(const int *__restrict__ cls_P,
                                                          const int *__restrict__ cls_Q,
                                                          const int64_t *__restrict__ cls_toff,
                                                          const int64_t *__restrict__ cls_aoff,
                                                          const cx<double> *__restrict__ Tm,
                                                          const cx<double> *__restrict__ Sm,
                                                          cx<double> *__restrict__ A, cx<float> *__restrict__ A32,
                                                          int ncls, int tiles)
{
    __shared__ f64x4 part[CW][2][64];
    const int b = blockIdx.x, nt2 = tiles * tiles;
    const int c = ((b / NXCD) / nt2) * NXCD + b % NXCD, tile = (b / NXCD) % nt2;
    if (c >= ncls) return;  // the whole block
    const int P = cls_P[c], Q = cls_Q[c], nc = 2 * P + 1;
    const int p0 = (tile % tiles) * CT, q0 = (tile / tiles) * CT;
    if (p0 >= nc || q0 >= nc) return;  // the whole block
    const cx<double> *T = Tm + cls_toff[c];  // [nc][Q]
    const cx<double> *S = Sm + cls_toff[c];  // [Q][nc]
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l % 16, lk = l / 16;
    const int p = p0 + li, q = q0 + li;
    f64x4 dr = {0.0, 0.0, 0.0, 0.0}, di = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = w * CU; 4 * s0 < Q; s0 += CW * CU) {
        cx<double> a[CU], b[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int k = 4 * (s0 + u) + lk;
            a[u] = (p < nc && k < Q) ? T[(int64_t)p * Q + k] : mk(0.0, 0.0);
            b[u] = (q < nc && k < Q) ? S[(int64_t)k * nc + q] : mk(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            dr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].re, b[u].re, dr, 0, 0, 0);
            dr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].im, b[u].im, dr, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].re, b[u].im, di, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].im, b[u].re, di, 0, 0, 0);
        }
    }
    part[w][0][l] = dr;
    part[w][1][l] = di;
    __syncthreads();
    if (w != 0) return;
    for (int x = 1; x < CW; ++x) {
        dr += part[x][0][l];
        di += part[x][1][l];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int pp = p0 + lk + 4 * v, qq = q0 + li;
        if (pp < nc && qq < nc) {
            const int64_t o = cls_aoff[c] + (int64_t)qq * nc + pp;
            A[o] = mk(dr[v], di[v]);
            A32[o] = mk((float)dr[v], (float)di[v]);
        }
    }
}

}  // namespace

void launch_node_table(const double *lamw, int n, Medium med, Node *out, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_node_table, dim3((n + 255) / 256), dim3(256), 0, st, lamw, n, med, out);
}

void launch_m2l_tables(const double *lamw, const int *node_cls, const int *node_local, int ntot,
                       const double *cls_geo, Medium med, const int *cls_P, const int *cls_Q,
                       const int64_t *cls_toff, const int64_t *cls_aoff, int ncls, int ncmax, cx<double> *Tm,
                       cx<double> *Sm, cx<double> *A, cx<float> *A32, hipStream_t st)
{
    if (ntot <= 0 || ncls <= 0) return;
    hipLaunchKernelGGL(k_m2l_factors, dim3((ntot + 255) / 256), dim3(256), 0, st, lamw, node_cls, node_local, ntot,
                       cls_geo, med, cls_P, cls_Q, cls_toff, Tm, Sm);
    const int tiles = (ncmax + CT - 1) / CT;
    const int64_t nblk = (int64_t)((ncls + NXCD - 1) / NXCD) * NXCD * tiles * tiles;
    hipLaunchKernelGGL(k_m2l_contract, dim3((unsigned)nblk), dim3(64 * CW), 0, st, cls_P, cls_Q, cls_toff, cls_aoff,
                       Tm, Sm, A, A32, ncls, tiles);
}

}  // namespace lmfmm
