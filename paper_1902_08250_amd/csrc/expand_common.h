// Device helpers shared by the FMM passes: the per-item matrix-vector product
// of the translations (and of the leaf-level shift in the local evaluation),
// and the pairwise near-field quadrature sum.
#pragma once
#include "lmfmm_internal.h"

namespace lmfmm {

namespace {

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

// Sum over each aligned group of S adjacent lanes (S = 1, 2, 4, ..., 64), in
// a fixed order, complete in the group's last lane: pairs, quads, half rows
// and rows of 16 by lane permutations (then the sum is in every lane of the
// row), then row 0 into row 1 and row 2 into row 3, then rows 0-1 into row 3.
// Every lane of the wave must be active.
__device__ inline double group_sum_d(double v, int S)
{
    if (S >= 2) v += dpp_d<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    if (S >= 4) v += dpp_d<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    if (S >= 8) v += dpp_d<0x141, 0xf>(v);  // row_half_mirror
    if (S >= 16) v += dpp_d<0x140, 0xf>(v); // row_mirror
    if (S >= 32) v += dpp_d<0x142, 0xa>(v); // row_bcast:15 into rows 1 and 3
    if (S >= 64) v += dpp_d<0x143, 0xc>(v); // row_bcast:31 into rows 2 and 3
    return v;
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
struct WaveX {
    cx<T> x[Tr<T>::R][Tr<T>::KC];
};
template <typename T>
struct WaveLds : WaveX<T> {
    cx<T> out[Tr<T>::R][64];
};

// acc[r] += sum_{k < nk} A[k * nout + p] x[r * xstride + k], p = p0 + lane,
// r < nr.  Every lane of the wave calls this with the same arguments.
template <typename T>
__device__ inline void item_matvec(const cx<T> *__restrict__ A, int nk, int nout, int p0,
                                   const cx<T> *__restrict__ x, int64_t xstride, int nr, WaveX<T> &lds,
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

}  // namespace

}  // namespace lmfmm
