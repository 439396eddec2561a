// Leaf passes of the FMM on the uniform interface-split quadtree (Algorithm 1,
// Steps 2 and 4):
//
//  * P2M  (source-to-multipole, Definition "Multipole Expansion"): per source
//    leaf, M_q = sum_j q_j J_q(k1 r_j) e^{-i q theta_j}, stored scaled.
//  * L2P + S2T (Definition "Local Expansion"; direct interactions): per
//    target leaf, the leaf's L2L shift, then the local expansion evaluated at
//    the targets, plus the direct interactions of the adjacent source leaves
//    across the interface (from the sweep's results, or by pairs).
//  * The coordinate gradient of the local evaluation and of the direct
//    interactions.
//
// Expansions are stored scaled: Mhat_q = s_q M_q and Lhat_p = L_p / s_p with
// s_q = |q|! (2/(k R))^|q|, R the box half-diagonal, which keeps FP32 in
// range.  Layout: [box][rhs][2P+1] complex, box = row * ncol + column.
#include "lmfmm_internal.h"
#include "expand_common.h"

#include <atomic>

namespace lmfmm {

namespace {

// ---------------------------------------------------------------------------
// P2M by the recurrence form: a block takes G consecutive source leaves, whose
// points are contiguous in the grouped order (as are their densities, qs),
// and walks those points in chunks of CH: a thread per point evaluates the
// point's scaled basis into LDS, with the point's densities padded with zeros
// to a multiple of R4 right-hand sides (1, 2 or 4, from nrhs), then threads
// over (leaf, chunk of R4 right-hand sides, coefficient) add the points of
// their leaf in the chunk, in index order; the padding keeps that loop free
// of per-lane branches.  The output block of the G leaves is contiguous, and so are the
// threads' stores.  Leaves without points get zeros.
// ---------------------------------------------------------------------------
constexpr int P2M_THREADS = 256;
constexpr int P2M_CHMAX = 320;  // points per chunk (a thread evaluates up to two)
constexpr int LEAF_GMAX = 32;   // leaves per block (P2M and L2P)
template <typename T>
struct P2MArgs {
    const int32_t *start, *end;
    const double *xs, *ys;
    const cx<T> *qs;
    int64_t ns;
    int nrhs, P, nbox, ncol, col_lo;
    double x_lo, w;
    cx<T> k1;
    T invR;
    int G, CH;
    cx<T> *M;
    int32_t *occ;  // the leaves' occupancy flags
};
template <typename T, int R4>
__device__ __forceinline__ void p2m_body(const P2MArgs<T> &A, const int bx)
{
    const int32_t *__restrict__ start = A.start;
    const int32_t *__restrict__ end = A.end;
    const double *__restrict__ xs = A.xs;
    const double *__restrict__ ys = A.ys;
    const cx<T> *__restrict__ qs = A.qs;
    cx<T> *__restrict__ M = A.M;
    const int64_t ns = A.ns;
    const int nrhs = A.nrhs, P = A.P, nbox = A.nbox, ncol = A.ncol, col_lo = A.col_lo, G = A.G, CH = A.CH;
    const double x_lo = A.x_lo, w = A.w;
    const cx<T> k1 = A.k1;
    const T invR = A.invR;
    extern __shared__ unsigned char smem_raw[];
    __shared__ int bnd[LEAF_GMAX + 1];
    const int nc = 2 * P + 1;
    const int nrc = (nrhs + R4 - 1) / R4, nq = R4 * nrc;
    cx<T> *B = reinterpret_cast<cx<T> *>(smem_raw);  // [CH][nc]
    cx<T> *Q = B + CH * nc;                          // [CH][nq]
    const int t = threadIdx.x;
    const int b0 = bx * G;
    const int ng = nbox - b0 < G ? nbox - b0 : G;
    if (t <= ng) bnd[t] = t < ng ? start[b0 + t] : end[b0 + ng - 1];
    __syncthreads();
    if (t < ng) A.occ[b0 + t] = bnd[t + 1] > bnd[t] ? 1 : 0;
    const int S = bnd[0], E = bnd[ng];
    const int nout = nc * nrhs;
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
            bessel_basis<T>(k1, X, Y, invR, P, -1, B + jl * nc, 1);
            for (int r = 0; r < nq; ++r) Q[jl * nq + r] = r < nrhs ? qs[(int64_t)r * ns + j] : mk<T>(0, 0);
        }
        __syncthreads();
        const int cend = E - c0 < CH ? E : c0 + CH;
        // the chunk's leaves: those ending after c0 or starting at or after
        // it, up to the last starting before cend (every remaining leaf for
        // the last chunk); a leaf starting in the chunk (empty leaves
        // included) is written, one continuing into it is added to
        int glo = 0;
        while (glo < ng && bnd[glo + 1] <= c0 && bnd[glo] < c0) ++glo;
        int ghi = ng - 1;
        if (cend < E)
            while (ghi >= glo && bnd[ghi] >= cend) --ghi;
        // items (leaf, chunk of up to four right-hand sides, coefficient):
        // one basis value read per point serves every right-hand side of the
        // chunk
        const int nout4 = nrc * nc;
        const int nit = (ghi - glo + 1) * nout4;
        for (int it0 = t; it0 < nit; it0 += P2M_THREADS) {
            const int it = glo * nout4 + it0;
            const int g = it / nout4, o = it - g * nout4;
            const int rc = o / nc, c = o - rc * nc;
            const int r0 = rc * R4, nr = nrhs - r0 < R4 ? nrhs - r0 : R4;
            const int j0 = bnd[g] > c0 ? bnd[g] : c0, j1 = bnd[g + 1] < cend ? bnd[g + 1] : cend;
            // in increasing point order; four points' LDS reads issued together
            const cx<T> *bp = B + (j0 - c0) * nc + c, *qp = Q + (j0 - c0) * nq + r0;
            const int np = j1 - j0;
            // groups of four points summed plainly, the groups' sums added
            // with compensation (FP32: the error does not grow with the
            // leaf's point count)
            CAcc<T> acc[R4];
#pragma unroll
            for (int r = 0; r < R4; ++r) acc[r].zero();
            int jj = 0;
            for (; jj + 4 <= np; jj += 4) {
                cx<T> b[4], qv[4][R4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    b[i] = bp[(jj + i) * nc];
#pragma unroll
                    for (int r = 0; r < R4; ++r) qv[i][r] = qp[(jj + i) * nq + r];
                }
#pragma unroll
                for (int r = 0; r < R4; ++r) {
                    cx<T> g4 = b[0] * qv[0][r];
                    cfma(g4, b[1], qv[1][r]);
                    cfma(g4, b[2], qv[2][r]);
                    cfma(g4, b[3], qv[3][r]);
                    acc[r].add(g4);
                }
            }
            cx<T> g4[R4];
#pragma unroll
            for (int r = 0; r < R4; ++r) g4[r] = mk<T>(0, 0);
            for (; jj < np; ++jj) {
                const cx<T> bj = bp[jj * nc];
#pragma unroll
                for (int r = 0; r < R4; ++r) cfma(g4[r], bj, qp[jj * nq + r]);
            }
#pragma unroll
            for (int r = 0; r < R4; ++r)
                if (r < nr) {
                    acc[r].add(g4[r]);
                    cx<T> &dst = Mb[(int64_t)g * nout + (r0 + r) * nc + c];
                    if (bnd[g] >= c0)
                        dst = acc[r].value();
                    else if (j1 > j0)
                        dst += acc[r].value();
                }
        }
        __syncthreads();
    }
}

template <typename T, int R4>
__global__ void __launch_bounds__(P2M_THREADS) k_p2m(P2MArgs<T> a) { p2m_body<T, R4>(a, blockIdx.x); }
template <typename T, int R4>
__global__ void __launch_bounds__(P2M_THREADS) k_p2m_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    p2m_body<T, R4>(static_cast<const P2MArgs<T> *>(m.args)[i], bx);
}

// ---------------------------------------------------------------------------
// P2M by the ascending series of J (DLMF 10.2.2), for leaves whose k1 R is
// small.  With z = k1 r, the scaled basis value of order +-a is
//     s_a J_a(z) e^{-+ i a theta} = S_a(zeta) up^a   and   S_a(zeta) dn^a,
//     S_a(zeta) = sum_m a! zeta^m / (m! (m + a)!),   zeta = -z^2 / 4,
// with up = (X - iY)/R and dn = -conj(up), so that no recurrence over the
// order and no division is needed.  S_a is summed by Horner's rule from the
// term ratios zeta / (m (m + a)); the reciprocals 1/(m (m + a)) come from a
// constant table.  A wave owns two magnitudes a, a + 1 (four coefficients)
// of 64 / S leaves, a lane one leaf and a slice of its points (offsets s,
// s + S, ...); the slices are added by lane permutations at the end, into the
// group's last lane, which stores the sums.  No LDS,
// no barrier: every wave is independent.  Everything is computed in FP64
// (FP64 and FP32 issue at the same rate on the vector units) and stored in
// the expansion's precision.
// ---------------------------------------------------------------------------
constexpr int P2MS_MMAX = 24;   // series terms at most
constexpr int P2M_SERIES_MIN_PER_LEAF = 40;  // FP32: mean points per leaf for the series form
constexpr int P2MS_AMAX = 258;  // magnitudes 0..257 (orders up to 256, and one more)
struct P2MSeriesTable {
    double v[P2MS_AMAX][P2MS_MMAX];  // v[a][m-1] = 1 / (m (m + a))
    constexpr P2MSeriesTable() : v()
    {
        for (int a = 0; a < P2MS_AMAX; ++a)
            for (int m = 1; m <= P2MS_MMAX; ++m) v[a][m - 1] = 1.0 / ((double)m * (double)(m + a));
    }
};
__constant__ const P2MSeriesTable p2ms_tab = P2MSeriesTable();

template <typename T>
struct P2MSArgs {
    const int32_t *start, *end;
    const double *xs, *ys;
    const cx<T> *qs;
    int64_t ns;
    int nrhs, P, nbox, ncol, col_lo;
    double x_lo, w;
    cx<double> kappa;  // -k1^2 / 4
    double invR;
    int S, LB;         // slices per leaf (adjacent lanes), leaves per wave
    int npair, ncpg;   // magnitude pairs, groups of four pairs (one per block)
    int nterm;         // series terms
    cx<T> *M;
    int32_t *occ;
};
template <typename T>
__device__ __forceinline__ void p2ms_body(const P2MSArgs<T> &A, const int bx, const int rc)
{
    const int lg = bx / A.ncpg, cpg = bx - lg * A.ncpg;
    const int cp = __builtin_amdgcn_readfirstlane(cpg * 4 + (int)(threadIdx.x >> 6));
    if (cp >= A.npair) return;  // the whole wave: no barrier follows
    const int lane = threadIdx.x & 63, S = A.S, P = A.P, nc = 2 * P + 1;
    const int leaf = lg * A.LB + lane / S, s = lane & (S - 1);
    const bool act = leaf < A.nbox;
    int j0 = 0, j1 = 0;
    if (act) {
        j0 = A.start[leaf];
        j1 = A.end[leaf];
    }
    const int row = leaf / A.ncol, col = A.col_lo + leaf % A.ncol;
    const double cxp = A.x_lo + (col + 0.5) * A.w, cyp = (row + 0.5) * A.w;
    const int a = 2 * cp;
    const bool two = a + 1 <= P;
    const int r0 = 4 * rc, nr = A.nrhs - r0 < 4 ? A.nrhs - r0 : 4;
    const cx<double> kappa = A.kappa;
    const double invR = A.invR;
    const double *__restrict__ ta = p2ms_tab.v[a];
    const double *__restrict__ tb = p2ms_tab.v[a + 1];
    cx<double> acc[4][4];  // coefficients +a, -a, +(a+1), -(a+1); right-hand sides
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][r] = mk<double>(0, 0);
    // FP32 densities: the next point's coordinates and densities are loaded
    // while the current one is summed (with FP64 densities the extra
    // registers cost a wave per SIMD, and the prefetch then loses)
    constexpr bool PF = sizeof(T) == 4;
    double xn = 0.0, yn = 0.0;
    cx<T> qn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) qn[r] = mk<T>(0, 0);
    auto load = [&](int j) {
        xn = A.xs[j];
        yn = A.ys[j];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r < nr) qn[r] = A.qs[(int64_t)(r0 + r) * A.ns + j];
    };
    if (PF && j0 + s < j1) load(j0 + s);
    for (int j = j0 + s; j < j1; j += S) {
        if (!PF) load(j);
        const double X = xn - cxp, Y = yn - cyp;
        cx<double> qv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) qv[r] = mk<double>(qn[r].re, qn[r].im);
        if (PF && j + S < j1) load(j + S);
        const cx<double> zeta = kappa * (X * X + Y * Y);
        const cx<double> up = mk<double>(X * invR, -Y * invR);
        cx<double> pa = mk<double>(1, 0), bb = up;
        for (int e = a; e; e >>= 1) {
            if (e & 1) pa = pa * bb;
            bb = bb * bb;
        }
        cx<double> Sa = mk<double>(1, 0), Sb = mk<double>(1, 0);
        for (int m = A.nterm; m >= 1; --m) {
            const cx<double> za = zeta * Sa, zb = zeta * Sb;
            Sa = mk<double>(fma(za.re, ta[m - 1], 1.0), za.im * ta[m - 1]);
            Sb = mk<double>(fma(zb.re, tb[m - 1], 1.0), zb.im * tb[m - 1]);
        }
        const cx<double> pb = pa * up;
        const double sa = (a & 1) ? -1.0 : 1.0;
        const cx<double> B0 = pa * Sa;
        const cx<double> B1 = mk<double>(sa * pa.re, -sa * pa.im) * Sa;
        const cx<double> B2 = pb * Sb;
        const cx<double> B3 = mk<double>(-sa * pb.re, sa * pb.im) * Sb;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cfma(acc[0][r], B0, qv[r]);
            cfma(acc[1][r], B1, qv[r]);
            cfma(acc[2][r], B2, qv[r]);
            cfma(acc[3][r], B3, qv[r]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            acc[i][r].re = group_sum_d(acc[i][r].re, S);
            acc[i][r].im = group_sum_d(acc[i][r].im, S);
        }
    if (!act || s != S - 1) return;
    cx<T> *Mb = A.M + (int64_t)leaf * nc * A.nrhs;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r >= nr) break;
        cx<T> *m = Mb + (int64_t)(r0 + r) * nc + P;
        m[a] = mk<T>((T)acc[0][r].re, (T)acc[0][r].im);
        if (a > 0) m[-a] = mk<T>((T)acc[1][r].re, (T)acc[1][r].im);
        if (two) {
            m[a + 1] = mk<T>((T)acc[2][r].re, (T)acc[2][r].im);
            m[-a - 1] = mk<T>((T)acc[3][r].re, (T)acc[3][r].im);
        }
    }
    if (cp == 0 && rc == 0) A.occ[leaf] = j1 > j0 ? 1 : 0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_p2m_series(P2MSArgs<T> a) { p2ms_body<T>(a, blockIdx.x, blockIdx.y); }
template <typename T>
__global__ void __launch_bounds__(256) k_p2m_series_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    p2ms_body<T>(static_cast<const P2MSArgs<T> *>(m.args)[i], bx, by);
}

// ---------------------------------------------------------------------------
// L2P (Definition "Local Expansion"): res[r] = sum_p Lhat_p J_p(k2 r)
// e^{i p theta} at the point (X, Y) relative to the leaf centre, from the
// scaled expansion Ls[r][2P+1], r < nr.
// ---------------------------------------------------------------------------
// The local expansion of order P at offset (X, Y) from its centre, for nr
// right-hand sides (Ls[r * (2P + 1) + P + p], p = -P..P): sum_p Lhat_p B_p.
// The basis ratios g_p = B_p / B_{p-1} come out of the backward recurrence in
// decreasing p, so the sums are formed there by Horner's rule,
// sum_{p >= 1} Lhat_p B_p = B_0 g_1 (Lhat_1 + g_2 (Lhat_2 + ...)), and no
// table of ratios is kept (B_0 = J_0 is known only at the end).
template <typename T, int RMAX>
__device__ inline void eval_local(cx<T> k2, T X, T Y, T invR, int P, const cx<T> *Ls, int nr, cx<double> (&res)[RMAX])
{
    const int nc = 2 * P + 1;
    const cx<T> z2 = (k2 * k2) * (X * X + Y * Y);
    const int N = miller_start<T>(z2, P);
    cx<T> t = mk<T>(0, 0), tprev = mk<T>(0, 0), U = mk<T>(0, 0);
    for (int m = N; m > P; --m) miller_step<T>(z2, m, t, tprev, U);
    const cx<T> up = mk<T>(X * invR, Y * invR), dn = mk<T>(-X * invR, Y * invR);
    cx<T> hp[RMAX], hm[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) hp[r] = hm[r] = mk<T>(0, 0);
    for (int m = P; m >= 1; --m) {
        miller_step<T>(z2, m, t, tprev, U);
        const cx<T> f = T(2 * m) * t;
        const cx<T> gp = f * up, gm = f * dn;
#pragma unroll
        for (int r = 0; r < RMAX; ++r)
            if (r < nr) {
                hp[r] = gp * (Ls[r * nc + P + m] + hp[r]);
                hm[r] = gm * (Ls[r * nc + P - m] + hm[r]);
            }
    }
    const cx<T> J0 = cinv(mk<T>(T(1), T(0)) + U);
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        const cx<T> v = r < nr ? J0 * (Ls[r * nc + P] + hp[r] + hm[r]) : mk<T>(0, 0);
        res[r] = {(double)v.re, (double)v.im};
    }
}

// ---------------------------------------------------------------------------
// L2P over consecutive target leaves (points contiguous in the sorted order);
// the near field, if any, comes from the sweep kernel's parts.  Blocks below
// nb_if take G_if leaves each from the first n_if leaves (the interface rows),
// the others G leaves each from the rest.  Each leaf evaluates one local
// expansion (EvalLevels): its own, or its ancestor's at the level where the
// far field was complete.  Leaves with the same expansion share a slot in LDS.
// Slots are filled first: by the leaf-level L2L shift of the parent's
// expansion (Lemma L2L, one slot per wave at a time) plus the stored M2L
// result in the interface rows, or copied from the stored expansions.  Then a
// thread per target evaluates its slot's expansion and adds the near-field
// parts in order.  Writes u[r][original index].
// ---------------------------------------------------------------------------
constexpr int L2P_THREADS = 512;
constexpr int L2P_GMAX = 64;  // leaves per block (at most one wave's lanes)
template <typename T>
struct L2PArgs {
    const int32_t *start, *end, *idx;
    const double *xs, *ys;
    int64_t ns, nt;
    int nrhs, P, nbox, ncol, col_lo;
    double x_lo, w;
    cx<T> k2;
    T invR;
    const cx<T> *Lc;  // local expansions of every level (ev.off[l]: level l)
    LeafShift<T> sh;
    int64_t key_t0;
    int G, G_if, n_if, nb_if, ncmax, do_far;
    const cx<double> *unear;
    int nparts;
    cx<T> *u;
    EvalLevels ev;
};
template <typename T, int RMAX>
__device__ __forceinline__ void l2p_body(const L2PArgs<T> &A, const int bx, const int by)
{
    const int32_t *__restrict__ start = A.start;
    const int32_t *__restrict__ end = A.end;
    const int32_t *__restrict__ idx = A.idx;
    const double *__restrict__ xs = A.xs;
    const double *__restrict__ ys = A.ys;
    const cx<double> *__restrict__ unear = A.unear;
    cx<T> *__restrict__ u = A.u;
    const LeafShift<T> &sh = A.sh;
    const EvalLevels &ev = A.ev;
    const int64_t ns = A.ns, nt = A.nt, key_t0 = A.key_t0;
    const int nrhs = A.nrhs, P = A.P, nbox = A.nbox, ncol = A.ncol, col_lo = A.col_lo, do_far = A.do_far,
              nparts = A.nparts, ncmax = A.ncmax, L = ev.L;
    const double x_lo = A.x_lo, w = A.w;
    const cx<T> k2 = A.k2;
    const T invR = A.invR;
    const cx<T> *__restrict__ LcL = A.Lc + ev.off[L];
    extern __shared__ unsigned char smem_raw[];
    __shared__ WaveX<T> wl[L2P_THREADS / 64];
    __shared__ int bnd[L2P_GMAX + 1];
    __shared__ int s_slot[L2P_GMAX], s_leaf[L2P_GMAX + 1], s_lev[L2P_GMAX], s_P[L2P_GMAX];
    __shared__ int s_nslot;
    constexpr int R = Tr<T>::R;
    const int nc = 2 * P + 1;
    cx<T> *Ls = reinterpret_cast<cx<T> *>(smem_raw);  // [slot][RMAX][nc of the slot's level]
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int b0 = bx < A.nb_if ? bx * A.G_if : A.n_if + (bx - A.nb_if) * A.G;
    const int Gb = bx < A.nb_if ? A.G_if : A.G;
    const int lim = bx < A.nb_if ? A.n_if : nbox;
    const int ng = lim - b0 < Gb ? lim - b0 : Gb;
    const int r0 = by * RMAX;
    const int nr = nrhs - r0 < RMAX ? nrhs - r0 : RMAX;
    if (t <= ng) bnd[t] = t < ng ? start[key_t0 + b0 + t] : end[key_t0 + b0 + ng - 1];
    if (wv == 0) {
        // the expansion each leaf evaluates: consecutive leaves with the same
        // (level, ancestor box) share a slot
        int e = L, khi = -1, klo = -1;
        if (lane < ng) {
            const int box = b0 + lane, row = box / ncol, col = col_lo + box % ncol;
            e = eval_level(ev, row);
            khi = (e << 24) | (row >> (L - e));
            klo = col >> (L - e);
        }
        const int phi = __shfl_up(khi, 1), plo = __shfl_up(klo, 1);
        const bool isnew = lane < ng && (lane == 0 || khi != phi || klo != plo);
        const unsigned long long m = __ballot(isnew);
        const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const int slot = __popcll(m & le) - 1;
        if (lane < ng) s_slot[lane] = slot;
        if (isnew) {
            s_leaf[slot] = lane;
            s_lev[slot] = e;
            s_P[slot] = ev.on ? ev.P[e] : P;
        }
        if (lane == 0) {
            s_nslot = __popcll(m);
            s_leaf[__popcll(m)] = ng;
        }
    }
    __syncthreads();
    const int S = bnd[0], E = bnd[ng];
    if (E <= S) return;
    // the first chunk's points: their loads are in flight while the slots
    // are filled
    double px = 0.0, py = 0.0;
    int32_t pid = 0;
    if (S + t < E) {
        px = xs[S + t];
        py = ys[S + t];
        pid = idx[S + t];
    }
    const int nslot = s_nslot;
    if (do_far) {
        for (int s = wv; s < nslot; s += L2P_THREADS / 64) {
            const int g = s_leaf[s], e = s_lev[s];
            if (bnd[s_leaf[s + 1]] <= bnd[g]) continue;  // no targets in the slot's leaves
            const int box = b0 + g, row = box / ncol, col = col_lo + box % ncol;
            cx<T> *Lslot = Ls + (int64_t)s * RMAX * ncmax;
            if (sh.tab && e == L) {
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
                            prev[r] = (add && p < nc && r < nrr)
                                          ? LcL[((int64_t)box * nrhs + r0 + rr + r) * nc + p]
                                          : mk<T>(0, 0);
                        if (pok)
                            item_matvec<T>(sh.tab + (int64_t)pos * sh.ncp * nc, sh.ncp, nc, p0,
                                           x + (int64_t)(r0 + rr) * sh.ncp, sh.ncp, nrr, wl[wv], acc);
                        if (p < nc)
#pragma unroll
                            for (int r = 0; r < R; ++r)
                                if (r < nrr) Lslot[(rr + r) * nc + p] = add ? acc[r] + prev[r] : acc[r];
                    }
                }
            } else {
                // the stored expansion of the slot's box at level e
                const int she = L - e, nce = 2 * s_P[s] + 1;
                const int64_t be = (int64_t)(row >> she) * (ev.on ? ev.ncol[e] : ncol) + (col >> she) -
                                   (col_lo >> she);
                // nr rows of nce coefficients, contiguous in both: every load of
                // the copy is issued before the first store
                const cx<T> *src = A.Lc + ev.off[e] + (be * nrhs + r0) * nce;
                const int ntot = nr * nce;
                for (int e0 = 0; e0 < ntot; e0 += 8 * 64) {
                    cx<T> v[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int ee = e0 + k * 64 + lane;
                        v[k] = ee < ntot ? src[ee] : mk<T>(0, 0);
                    }
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int ee = e0 + k * 64 + lane;
                        if (ee < ntot) Lslot[ee] = v[k];
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int c0 = S; c0 < E; c0 += L2P_THREADS) {
        const int i = c0 + t;
        if (i >= E) break;
        const double px0 = px, py0 = py;
        const int32_t pid0 = pid;
        if (i + L2P_THREADS < E) {  // the next chunk's point, loaded during this one
            px = xs[i + L2P_THREADS];
            py = ys[i + L2P_THREADS];
            pid = idx[i + L2P_THREADS];
        }
        int g = 0;
        while (i >= bnd[g + 1]) ++g;
        const int box = b0 + g, row = box / ncol, col = col_lo + box % ncol;
        cx<double> res[RMAX];
        for (int r = 0; r < RMAX; ++r) res[r] = {0.0, 0.0};
        if (do_far) {
            const int s = s_slot[g], she = L - s_lev[s];
            const double we = ldexp(w, she);
            const double cxp = x_lo + ((col >> she) + 0.5) * we, cyp = -((row >> she) + 0.5) * we;
            eval_local<T, RMAX>(k2, (T)(px0 - cxp), (T)(py0 - cyp), invR / (T)(1 << she), s_P[s],
                                      Ls + (int64_t)s * RMAX * ncmax, nr, res);
        }
        const int64_t o = pid0 - ns;
        if (unear && row == 0)
            for (int pp = 0; pp < nparts; ++pp)
                for (int r = 0; r < RMAX; ++r)
                    if (r < nr) res[r] += unear[((int64_t)pp * nrhs + r0 + r) * nt + o];
        for (int r = 0; r < RMAX; ++r)
            if (r < nr) u[(int64_t)(r0 + r) * nt + o] = mk<T>((T)res[r].re, (T)res[r].im);
    }
}

template <typename T, int RMAX>
__global__ void __launch_bounds__(L2P_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_l2p(L2PArgs<T> a)
{
    l2p_body<T, RMAX>(a, blockIdx.x, blockIdx.y);
}
template <typename T, int RMAX>
__global__ void __launch_bounds__(L2P_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_l2p_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    l2p_body<T, RMAX>(static_cast<const L2PArgs<T> *>(m.args)[i], bx, by);
}

// ---------------------------------------------------------------------------
// Fused L2P + S2T per target leaf, the near field by pairs (the alternative
// to the sweep); lanes over targets (chunks of 64).
// Writes u[r][original index] (no accumulation across kernels).
// ---------------------------------------------------------------------------
template <typename T>
struct L2PNearArgs {
    const int32_t *start, *end, *idx;
    const double *xs, *ys;
    const cx<T> *q;
    int64_t ns, nt;
    int nrhs, P, ncol, col_lo, rows_s;
    double x_lo, w;
    cx<T> k2;
    T invR;
    const cx<T> *Lc;
    LeafShift<T> sh;
    const Node *nodes;
    int nmid, npan;
    double t0;
    int do_far, do_near;
    int64_t key_t0;
    const cx<double> *unear;
    int nparts;
    cx<T> *u;
};
template <typename T, int RMAX>
__device__ __forceinline__ void l2p_near_body(const L2PNearArgs<T> &A, const int bx, const int by)
{
    const int32_t *__restrict__ start = A.start;
    const int32_t *__restrict__ end = A.end;
    const int32_t *__restrict__ idx = A.idx;
    const double *__restrict__ xs = A.xs;
    const double *__restrict__ ys = A.ys;
    const cx<T> *__restrict__ q = A.q;
    const cx<T> *__restrict__ Lc = A.Lc;
    const Node *__restrict__ nodes = A.nodes;
    const cx<double> *__restrict__ unear = A.unear;
    cx<T> *__restrict__ u = A.u;
    const LeafShift<T> &sh = A.sh;
    const int64_t ns = A.ns, nt = A.nt, key_t0 = A.key_t0;
    const int nrhs = A.nrhs, P = A.P, ncol = A.ncol, col_lo = A.col_lo, rows_s = A.rows_s, nmid = A.nmid,
              npan = A.npan, do_far = A.do_far, do_near = A.do_near, nparts = A.nparts;
    const double x_lo = A.x_lo, w = A.w, t0 = A.t0;
    const cx<T> k2 = A.k2;
    const T invR = A.invR;
    extern __shared__ unsigned char smem_raw[];
    __shared__ WaveLds<T> wl;
    const int nc = 2 * P + 1;
    cx<T> *Ls = reinterpret_cast<cx<T> *>(smem_raw);  // [RMAX][nc]
    const int box = bx, lane = threadIdx.x;
    const int r0 = by * RMAX;
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
        if (do_far) eval_local<T, RMAX>(k2, (T)(x1 - cxp), (T)(y1 - cyp), invR, P, Ls, nr, res);
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

template <typename T, int RMAX>
__global__ void __launch_bounds__(64) k_l2p_near(L2PNearArgs<T> a) { l2p_near_body<T, RMAX>(a, blockIdx.x, blockIdx.y); }
template <typename T, int RMAX>
__global__ void __launch_bounds__(64) k_l2p_near_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    l2p_near_body<T, RMAX>(static_cast<const L2PNearArgs<T> *>(m.args)[i], bx, by);
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
#pragma unroll PUnroll<PMAX>::n
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

template <typename T>
void p2m_dispatch(const int32_t *start, const int32_t *end, const double *xs, const double *ys, const void *qs,
                  int64_t ns, int nrhs, const Geometry &g, Medium med, cx<T> *M, int32_t *occ, hipStream_t st)
{
    const Level &lv = g.lev[g.L];
    int nbox = lv.rows_s * lv.ncol;
    if (nbox == 0) return;
    // points per chunk: as many as the LDS share of a block holds, at most
    // P2M_CHMAX; the share is 78 KB (two blocks per compute unit) up to about
    // 0.8 x 256 points per block and compute unit, else 38 KB (four blocks)
    // right-hand sides per item: the densities are padded to a multiple of it
    const int R4 = nrhs == 1 ? 1 : (nrhs == 2 ? 2 : 4);
    const size_t per = (size_t)(lv.nc + R4 * ((nrhs + R4 - 1) / R4)) * sizeof(cx<T>);
    const int64_t load = std::max<int64_t>(ns, launch_batch_points());
    const size_t share = load > (int64_t)(2 * 0.8 * P2M_THREADS * device_shape().cus) ? 38 * 1024 : 78 * 1024;
    int CH = (int)(share / per);
    CH = CH > P2M_CHMAX ? P2M_CHMAX : (CH < 1 ? 1 : CH);
    const size_t sh = (size_t)CH * per;
    int per_cu = (int)(device_shape().lds / (sh > 0 ? sh : 1));
    per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
    int G = leaves_per_block(nbox, ns, CH < P2M_THREADS ? CH : P2M_THREADS, per_cu);
    // in a merged launch of several instances the others fill the compute
    // units too: take enough leaves for about 0.8 x 256 points per block
    if (launch_batch_points() > ns) {
        const double per_leaf = (double)ns / nbox;
        const int64_t gf =
            (int64_t)std::ceil(0.8 * (CH < P2M_THREADS ? CH : P2M_THREADS) / std::max(per_leaf, 1.0 / LEAF_GMAX));
        G = (int)std::max<int64_t>(G, std::min<int64_t>(gf, LEAF_GMAX));
    }
    cx<double> kd = k_src(med);
    cx<T> k1 = mk<T>((T)kd.re, (T)kd.im);
    T invR = (T)(M_SQRT2 / lv.w);
    const P2MArgs<T> a{start, end, xs, ys, reinterpret_cast<const cx<T> *>(qs), ns, nrhs, lv.P, nbox, lv.ncol,
                       lv.col_lo, g.x_lo, lv.w, k1, invR, G, CH, M + lv.off_s, occ + lv.off_occ};
    if (R4 == 1)
        emit((const void *)k_p2m<T, 1>, (const void *)k_p2m_multi<T, 1>, 0, dim3((nbox + G - 1) / G),
             dim3(P2M_THREADS), sh, st, a);
    else if (R4 == 2)
        emit((const void *)k_p2m<T, 2>, (const void *)k_p2m_multi<T, 2>, 0, dim3((nbox + G - 1) / G),
             dim3(P2M_THREADS), sh, st, a);
    else
        emit((const void *)k_p2m<T, 4>, (const void *)k_p2m_multi<T, 4>, 0, dim3((nbox + G - 1) / G),
             dim3(P2M_THREADS), sh, st, a);
}

// Terms of the series P2M for the leaf level, or 0 where its k1 R is too
// large for the series (then the recurrence form is used).  The terms left
// out are below 1e-18 (FP64) or 1e-10 (FP32 expansions) of the leading one:
// |zeta| <= (|k1| R)^2 / 4 and the m-th term is at most |zeta|^m / (m!)^2.
// Up to k1 R = 3 the terms' sum exceeds the result by a factor I_0(3) < 5 at
// most, which bounds the rounding error.
int p2m_series_terms(const Geometry &g, Medium med, bool fp64)
{
    const Level &lv = g.lev[g.L];
    const cx<double> k = k_src(med);
    const double kr = std::sqrt(k.re * k.re + k.im * k.im) * lv.w * M_SQRT1_2;
    if (!(kr <= 3.0) || lv.P + 1 >= P2MS_AMAX) return 0;
    const double z = kr * kr / 4, eps = fp64 ? 1e-18 : 1e-10;
    double term = 1.0;
    for (int m = 1; m <= P2MS_MMAX; ++m) {
        term *= z / ((double)m * m);
        if (term < eps) return m;
    }
    return 0;
}

template <typename T>
void p2m_series_dispatch(const int32_t *start, const int32_t *end, const double *xs, const double *ys,
                         const void *qs, int64_t ns, int nrhs, const Geometry &g, Medium med, cx<T> *M,
                         int32_t *occ, int nterm, hipStream_t st)
{
    const Level &lv = g.lev[g.L];
    const int nbox = lv.rows_s * lv.ncol;
    if (nbox == 0) return;
    // slices per leaf: a power of two up to 64, about an eighth of the mean
    // points per leaf
    const double per_leaf = (double)ns / nbox;
    int S = 1;
    while (S < 64 && 8.0 * S <= per_leaf) S <<= 1;
    const int LB = 64 / S;
    const int npair = (lv.P + 2) / 2;
    const int ncpg = (npair + 3) / 4;
    const int nlg = (nbox + LB - 1) / LB;
    const cx<double> k = k_src(med);
    const cx<double> kappa = mk<double>(-(k.re * k.re - k.im * k.im) / 4, -(2 * k.re * k.im) / 4);
    const P2MSArgs<T> a{start, end, xs, ys, reinterpret_cast<const cx<T> *>(qs), ns, nrhs, lv.P, nbox, lv.ncol,
                        lv.col_lo, g.x_lo, lv.w, kappa, M_SQRT2 / lv.w, S, LB, npair, ncpg, nterm,
                        M + lv.off_s, occ + lv.off_occ};
    emit((const void *)k_p2m_series<T>, (const void *)k_p2m_series_multi<T>, 1, dim3(nlg * ncpg, (nrhs + 3) / 4),
         dim3(256), 0, st, a);
}

template <typename T, int PMAX>
void l2p_dispatch(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs, const double *ys,
                  const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g, Medium med, const cx<T> *Lc,
                  const LeafShift<T> &shift, const EvalLevels &ev_in, const Node *nodes, int nmid, int npan,
                  double t0, int do_far, int do_near, const cx<double> *unear, int nparts, void *u, hipStream_t st)
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
        // far field plus, if any, the sweep's near-field parts
        EvalLevels ev = ev_in;
        ev.L = g.L;
        ev.P[g.L] = lv.P;
        ev.ncol[g.L] = lv.ncol;
        ev.off[g.L] = lv.off_t;
        int ncmax = lv.nc;
        if (ev.on)
            for (int l = ev.lc; l < g.L; ++l) ncmax = std::max(ncmax, 2 * ev.P[l] + 1);
        const int RM = nrhs == 1 ? 1 : (nrhs <= 4 ? 4 : 8);
        const size_t per_leaf = (size_t)RM * ncmax * sizeof(cx<T>);
        // Leaves that shift (evaluation at the leaf level): about 0.8 x 256
        // points per block, two blocks per compute unit, one leaf per wave
        // (larger blocks, whose waves shift several leaves in turn, were
        // slower).  The other leaves only copy a stored expansion, shared by
        // neighbouring leaves: up to L2P_GMAX leaves and about 0.8 x 512
        // points per block.  Without evaluation levels every leaf shifts.
        const int gmax = std::max(1, (int)((48 * 1024) / per_leaf));
        const int gmax_deep = gmax;
        int n_if = nbox;
        if (ev.on && ev.lc < g.L) n_if = std::min(nbox, shift.tab ? shift.add_rows * lv.ncol : 0);
        int G_if = leaves_per_block(nbox, nt, 256, 2);
        G_if = std::max(1, std::min(std::min(G_if, L2P_THREADS / 64), gmax));
        int G = G_if;
        if (n_if < nbox) {
            const DeviceShape dv = device_shape();
            int64_t k = (int64_t)std::ceil((double)nt / (0.8 * L2P_THREADS * dv.cus));
            k = k < 1 ? 1 : (k > 2 ? 2 : k);
            const int64_t gd = ((int64_t)(nbox - n_if) + k * dv.cus - 1) / (k * dv.cus);
            G = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(gd, L2P_GMAX), gmax_deep));
            // in a merged launch of several instances the others fill the
            // compute units too: take enough leaves for about 0.8 x 512
            // targets per block instead of spreading this instance's few
            // targets over nearly empty blocks
            if (launch_batch_points() > nt && nbox > n_if) {
                const double per_leaf = (double)nt / nbox;
                const int64_t gf = (int64_t)std::ceil(0.8 * L2P_THREADS / std::max(per_leaf, 1.0 / L2P_GMAX));
                G = (int)std::max<int64_t>(G, std::min<int64_t>(std::min<int64_t>(gf, L2P_GMAX), gmax_deep));
            }
        }
        const int nb_if = (n_if + G_if - 1) / G_if;
        const int nblk = nb_if + (nbox - n_if + G - 1) / G;
        const dim3 grid(nblk, (nrhs + RM - 1) / RM);
        L2PArgs<T> a{start, end, idx, xs, ys, ns, nt, nrhs, lv.P, nbox, lv.ncol, lv.col_lo, g.x_lo, lv.w, k2,
                     invR, Lc, shift, key_t0, G, G_if, n_if, nb_if, ncmax, do_far, unear, unear ? nparts : 0,
                     reinterpret_cast<cx<T> *>(u), ev};
        const size_t shmem = (size_t)std::max(G, G_if) * per_leaf;
#define LMFMM_L2P_PACKED(RMC)                                                                              \
    emit((const void *)k_l2p<T, RMC>, (const void *)k_l2p_multi<T, RMC>, 0, grid, dim3(L2P_THREADS), \
         shmem, st, a)
        if (RM == 1)
            LMFMM_L2P_PACKED(1);
        else if (RM == 4)
            LMFMM_L2P_PACKED(4);
        else
            LMFMM_L2P_PACKED(8);
#undef LMFMM_L2P_PACKED
        return;
    }
    // near field by pairs: one leaf per block
    const L2PNearArgs<T> a{start, end, idx, xs, ys, reinterpret_cast<const cx<T> *>(q), ns, nt, nrhs, lv.P,
                           lv.ncol, lv.col_lo, lv.rows_s, g.x_lo, lv.w, k2, invR, Lc + lv.off_t, shift, nodes, nmid,
                           npan, t0, do_far, do_near, key_t0, unear, nparts, reinterpret_cast<cx<T> *>(u)};
#define LMFMM_L2P_LAUNCH(RM)                                                                                 \
    emit((const void *)k_l2p_near<T, RM>, (const void *)k_l2p_near_multi<T, RM>, 0,             \
         dim3(nbox, (nrhs + RM - 1) / RM), dim3(64), sh, st, a)
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
                int64_t ns, int nrhs, const Geometry &g, Medium med, cx<T> *M, int32_t *occ, bool series,
                hipStream_t st)
{
    // the series form wherever its terms allow, except for FP32 expansions of
    // leaves with few points, where evaluating each point's basis once (the
    // recurrence form) costs less than the series' per-point work, which is
    // repeated for every pair of orders
    const Level &lv = g.lev[g.L];
    const int64_t nbox = (int64_t)lv.rows_s * lv.ncol;
    // (in a recorded batch the series launch runs for the other instances
    // anyway, and one merged launch fewer saves more than the form costs)
    const bool few =
        sizeof(T) == 4 && nbox > 0 && ns < P2M_SERIES_MIN_PER_LEAF * nbox && launch_batch_points() <= ns;
    const int nterm = series && !few ? p2m_series_terms(g, med, sizeof(T) == 8) : 0;
    if (nterm > 0)
        p2m_series_dispatch<T>(start, end, xs, ys, qs, ns, nrhs, g, med, M, occ, nterm, st);
    else
        p2m_dispatch<T>(start, end, xs, ys, qs, ns, nrhs, g, med, M, occ, st);
}

template <typename T>
void launch_l2p_near(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs,
                     const double *ys, const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g,
                     Medium med, const cx<T> *Lc, const LeafShift<T> &shift, const EvalLevels &ev, const Node *nodes,
                     int nmid, int npan, double t0, int do_far, int do_near, const cx<double> *unear, int nparts,
                     void *u, hipStream_t st)
{
    int P = g.lev[g.L].P;
    if (ev.on)
        for (int l = ev.lc; l < g.L; ++l) P = std::max(P, ev.P[l]);
    if (!unear) nparts = 0;
#define LMFMM_L2P(PM)                                                                                               \
    l2p_dispatch<T, PM>(start, end, idx, xs, ys, q, ns, nt, nrhs, g, med, Lc, shift, ev, nodes, nmid, npan, t0, \
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

#define LMFMM_INST(T)                                                                                               \
    template void launch_p2m<T>(const int32_t *, const int32_t *, const double *, const double *, const void *,      \
                                int64_t, int, const Geometry &, Medium, cx<T> *, int32_t *, bool, hipStream_t);     \
    template void launch_l2p_near<T>(const int32_t *, const int32_t *, const int32_t *, const double *,             \
                                     const double *, const void *, int64_t, int64_t, int, const Geometry &, Medium, \
                                     const cx<T> *, const LeafShift<T> &, const EvalLevels &, const Node *, int,    \
                                     int, double, int, int, const cx<double> *, int, void *, hipStream_t);          \
    template void launch_l2p_grad<T>(const int32_t *, const int32_t *, const int32_t *, const double *,             \
                                     const double *, const void *, const void *, int64_t, int64_t, int,             \
                                     const Geometry &, Medium, const cx<T> *, const Node *, int, int, double, int,  \
                                     int, double, double *, hipStream_t);
LMFMM_INST(double)
LMFMM_INST(float)

}  // namespace lmfmm
