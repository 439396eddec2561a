// Direct interactions (S2T) of the FMM: the near field of adjacent leaves
// across the interface by x-ordered sweeps over one pair-independent node
// table, and the brute-force direct sum over all pairs (contour quadrature of
// g_2^t, Section 1; Section 4.2 contours).
#include "lmfmm_internal.h"
#include "expand_common.h"
#include "cexp_tab.h"

namespace lmfmm {

namespace {

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

template <typename T>
struct SweepArgs {
    const int32_t *start, *end, *idx;
    const double *xs, *ys;
    const cx<T> *q;
    int64_t ns, nt;
    int nrhs, ncol;
    int64_t key_t0;
    int seglen;
    double xl0, w;
    const Node *nodes;
    int nnodes, nmid, npan;
    double t0;
    int nparts;
    cx<double> *unear;
};
template <typename T, int RMAX>
__device__ __forceinline__ void near_sweep_body(const int32_t *__restrict__ start, const int32_t *__restrict__ end,
                                                const int32_t *__restrict__ idx, const double *__restrict__ xs,
                                                const double *__restrict__ ys, const cx<T> *__restrict__ q,
                                                int64_t ns, int64_t nt, int nrhs, int ncol, int64_t key_t0,
                                                int seglen, double xl0, double w, const Node *__restrict__ nodes,
                                                int nnodes, int nmid, int npan, double t0, int nparts,
                                                cx<double> *__restrict__ unear, const int bx, const int by,
                                                const int bz)
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
    const int r0 = by * RMAX, nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    const int part = bz;
    const int c0 = bx * seglen, c1 = c0 + seglen < ncol ? c0 + seglen : ncol;
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

// (the body takes the fields one by one: its register use then matches a
// kernel with those parameters)
#define LMFMM_SWEEP_FIELDS(a)                                                                                      \
    a.start, a.end, a.idx, a.xs, a.ys, a.q, a.ns, a.nt, a.nrhs, a.ncol, a.key_t0, a.seglen, a.xl0, a.w, a.nodes, \
        a.nnodes, a.nmid, a.npan, a.t0, a.nparts, a.unear
// the one-instance kernel takes the fields as separate arguments (fewer
// registers spilled than with the struct argument)
template <typename T, int RMAX>
__global__ void __launch_bounds__(64 * SW_W) __attribute__((amdgpu_waves_per_eu(4)))
k_near_sweep(const int32_t *__restrict__ start, const int32_t *__restrict__ end, const int32_t *__restrict__ idx,
             const double *__restrict__ xs, const double *__restrict__ ys, const cx<T> *__restrict__ q, int64_t ns,
             int64_t nt, int nrhs, int ncol, int64_t key_t0, int seglen, double xl0, double w,
             const Node *__restrict__ nodes, int nnodes, int nmid, int npan, double t0, int nparts,
             cx<double> *__restrict__ unear)
{
    near_sweep_body<T, RMAX>(start, end, idx, xs, ys, q, ns, nt, nrhs, ncol, key_t0, seglen, xl0, w, nodes, nnodes,
                             nmid, npan, t0, nparts, unear, blockIdx.x, blockIdx.y, blockIdx.z);
}
template <typename T, int RMAX>
__global__ void __launch_bounds__(64 * SW_W) __attribute__((amdgpu_waves_per_eu(4))) k_near_sweep_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    const SweepArgs<T> &a = static_cast<const SweepArgs<T> *>(m.args)[i];
    near_sweep_body<T, RMAX>(LMFMM_SWEEP_FIELDS(a), bx, by, bz);
}
#undef LMFMM_SWEEP_FIELDS

// Direct all-pairs sum (no tree): lanes over targets, loop over all sources.
// Direct sum over all pairs: block (target tile of 64, rhs chunk of 8,
// source chunk z) sums sources [z cs, (z + 1) cs) for its targets.  With one
// chunk it writes u; otherwise FP64 partials part[z][rhs][target], added in
// chunk order by k_direct_reduce.
template <typename T>
__global__ void __launch_bounds__(64) k_direct(const double *__restrict__ src, int64_t ns, const cx<T> *__restrict__ q,
                                               const double *__restrict__ tgt, int64_t nt, double ty_a, double ty_b,
                                               int nrhs,
                                               const Node *__restrict__ nodes, int nmid, int npan, double t0,
                                               int64_t cs, cx<double> *__restrict__ part, cx<T> *__restrict__ u)
{
    constexpr int RMAX = 8;
    int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int r0 = blockIdx.y * RMAX;
    const int nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    const int64_t j0 = (int64_t)blockIdx.z * cs, j1 = j0 + cs < ns ? j0 + cs : ns;
    bool act = i < nt;
    double x1 = act ? tgt[i] : tgt[0], y1 = fma(ty_a, act ? tgt[nt + i] : tgt[nt], ty_b);
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


}  // namespace

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
    const int RM = nrhs == 1 ? 1 : (nrhs <= 4 ? 4 : 8);
    const int G = RM == 1 ? SweepCap<1>::G : (RM == 4 ? SweepCap<4>::G : SweepCap<8>::G);
    const int nunits = ((nnodes + 63) / 64 + G - 1) / G;
    int nparts = (nunits + SW_W - 1) / SW_W;
    nparts = nparts < 1 ? 1 : (nparts > 4 ? 4 : nparts);
    const int nrc = (nrhs + RM - 1) / RM;
    int64_t seg = (int64_t)lv.ncol * nrc * nparts / 2048;
    const int seglen = seg < 1 ? 1 : (seg > 16 ? 16 : (int)seg);
    const int nseg = (lv.ncol + seglen - 1) / seglen;
    const SweepArgs<T> a{start, end, idx, xs, ys, reinterpret_cast<const cx<T> *>(q), ns, nt, nrhs, lv.ncol,
                         (int64_t)lv.rows_s * lv.ncol, seglen, g.x_lo + lv.col_lo * lv.w, lv.w, nodes, nnodes, nmid,
                         npan, t0, nparts, unear};
#define LMFMM_SWEEP_LAUNCH(R)                                                                                     \
    do {                                                                                                           \
        if (launch_recorder())                                                                                     \
            emit((const void *)nullptr, (const void *)k_near_sweep_multi<T, R>, 0, dim3(nseg, nrc, nparts),        \
                 dim3(64 * SW_W), 0, st, a);                                                                       \
        else                                                                                                       \
            LMFMM_LAUNCH((k_near_sweep<T, R>), dim3(nseg, nrc, nparts), dim3(64 * SW_W), 0, st, a.start, a.end,    \
                         a.idx, a.xs, a.ys, a.q, a.ns, a.nt, a.nrhs, a.ncol, a.key_t0, a.seglen, a.xl0, a.w, a.nodes, \
                         a.nnodes, a.nmid, a.npan, a.t0, a.nparts, a.unear);                                       \
    } while (0)
    if (RM == 1)
        LMFMM_SWEEP_LAUNCH(1);
    else if (RM == 4)
        LMFMM_SWEEP_LAUNCH(4);
    else
        LMFMM_SWEEP_LAUNCH(8);
#undef LMFMM_SWEEP_LAUNCH
    return nparts;
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

void launch_direct(const double *src, int64_t ns, const void *q, const double *tgt, int64_t nt, double ty_a,
                   double ty_b, int nrhs, int prec, const Node *nodes, int nmid, int npan, double t0, int nchunk,
                   cx<double> *part, void *u, hipStream_t st)
{
    if (nt == 0) return;
    int64_t cs = (ns + nchunk - 1) / nchunk;
    dim3 grid((unsigned)((nt + 63) / 64), (unsigned)((nrhs + 7) / 8), (unsigned)nchunk);
    cx<double> *pp = nchunk > 1 ? part : nullptr;
    const int64_t m = nt * nrhs;
    if (prec == 0) {
        hipLaunchKernelGGL((k_direct<double>), grid, dim3(64), 0, st, src, ns,
                           reinterpret_cast<const cx<double> *>(q), tgt, nt, ty_a, ty_b, nrhs, nodes, nmid, npan, t0, cs, pp,
                           reinterpret_cast<cx<double> *>(u));
        if (pp)
            hipLaunchKernelGGL((k_direct_reduce<double>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, pp,
                               nchunk, m, reinterpret_cast<cx<double> *>(u));
    } else {
        hipLaunchKernelGGL((k_direct<float>), grid, dim3(64), 0, st, src, ns, reinterpret_cast<const cx<float> *>(q),
                           tgt, nt, ty_a, ty_b, nrhs, nodes, nmid, npan, t0, cs, pp, reinterpret_cast<cx<float> *>(u));
        if (pp)
            hipLaunchKernelGGL((k_direct_reduce<float>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, pp,
                               nchunk, m, reinterpret_cast<cx<float> *>(u));
    }
}

#define LMFMM_INST(T)                                                                                               \
    template int launch_near_sweep<T>(const int32_t *, const int32_t *, const int32_t *, const double *,            \
                                      const double *, const void *, int64_t, int64_t, int, const Geometry &,        \
                                      const Node *, int, int, double, cx<double> *, hipStream_t);
LMFMM_INST(double)
LMFMM_INST(float)

}  // namespace lmfmm
