// Translations on the uniform interface-split quadtree (Algorithm 1, Steps 2
// and 3):
//
//  * M2M (Lemma M2M): free-space Helmholtz shift with k1, 4 children -> parent.
//  * M2L (Lemma M2L): at every level in one launch, each target box in the
//    two rows nearest the interface (every row at the coarsest level) gathers
//    its interaction list through the Sommerfeld translation tables.
//  * L2L (Lemma L2L): level by level, every target box receives its parent's
//    local expansion shifted with the free-space operator for k2, plus its own
//    M2L result.
//
// Expansions are stored scaled: Mhat_q = s_q M_q and Lhat_p = L_p / s_p with
// s_q = |q|! (2/(k R))^|q|, R the box half-diagonal, which keeps FP32 in
// range.  Layout: [box][rhs][2P+1] complex, box = row * ncol + column.
#include "lmfmm_internal.h"
#include "expand_common.h"

namespace lmfmm {

namespace {

// Upward pass of one level (Lemma M2M): one block per parent box at level
// lc - 1; wave w translates the child at position w (dx = w & 1, dy = w >> 1).
template <typename T>
struct UpArgs {
    const cx<T> *Mc;
    cx<T> *Mp;
    const cx<T> *tab;
    int nrhs, ncc, ncp, ncol_c, col_lo_c, rows_c, ncol_p, col_lo_p;
    const int32_t *occ_c;  // occupancy flags of the children's level
    int32_t *occ_p;        // ... of the parents' level (written: any child occupied)
};
template <typename T>
__device__ __forceinline__ void up_body(const UpArgs<T> &ua, int b)
{
    const cx<T> *__restrict__ Mc = ua.Mc;
    cx<T> *__restrict__ Mp = ua.Mp;
    const cx<T> *__restrict__ tab = ua.tab;
    const int nrhs = ua.nrhs, ncc = ua.ncc, ncp = ua.ncp, ncol_c = ua.ncol_c, col_lo_c = ua.col_lo_c,
              rows_c = ua.rows_c, ncol_p = ua.ncol_p, col_lo_p = ua.col_lo_p;
    constexpr int R = Tr<T>::R;
    __shared__ WaveLds<T> lds[4];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int prow = b / ncol_p, pcol = col_lo_p + b % ncol_p;
    const int crow = 2 * prow + (w >> 1), ccl = 2 * pcol + (w & 1) - col_lo_c;
    const bool ok = crow < rows_c && ccl >= 0 && ccl < ncol_c;
    const cx<T> *x = Mc + ((int64_t)crow * ncol_c + ccl) * nrhs * ncc;
    const cx<T> *A = tab + (int64_t)w * ncc * ncp;
    if (threadIdx.x == 0) {
        int any = 0;
        for (int c = 0; c < 4; ++c) {
            const int cr = 2 * prow + (c >> 1), cc = 2 * pcol + (c & 1) - col_lo_c;
            if (cr < rows_c && cc >= 0 && cc < ncol_c) any |= ua.occ_c[(int64_t)cr * ncol_c + cc];
        }
        ua.occ_p[b] = any;
    }
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
template <typename T>
__global__ void __launch_bounds__(256) k_up(UpArgs<T> a) { up_body<T>(a, blockIdx.x); }
template <typename T>
__global__ void __launch_bounds__(256) k_up_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    up_body<T>(static_cast<const UpArgs<T> *>(m.args)[i], bx);
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
    int rows_l2l;  // the L2L shift covers rows below this one (the rest are never read)
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
struct DownK {
    DownArgs a;
    int nrhs;
    const cx<T> *Lp, *l2l;
    cx<T> *Lc;
    const cx<T> *Ms, *atab;
    const int *cls3, *row_off;
};
template <typename T>
__device__ __forceinline__ void down_body(const DownK<T> &k, const int bx)
{
    const DownArgs &a = k.a;
    const int nrhs = k.nrhs;
    const cx<T> *__restrict__ Lp = k.Lp;
    const cx<T> *__restrict__ l2l = k.l2l;
    cx<T> *__restrict__ Lc = k.Lc;
    const cx<T> *__restrict__ Ms = k.Ms;
    const cx<T> *__restrict__ atab = k.atab;
    const int *__restrict__ cls3 = k.cls3;
    const int *__restrict__ row_off = k.row_off;
    constexpr int R = Tr<T>::R;
    __shared__ WaveLds<T> lds[DW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool m2l_block = bx < a.nb_m2l;
    int64_t box;
    int first, step, nitems, s0 = 0;
    if (m2l_block) {
        box = bx;
        const int row = (int)(box / a.ncol);
        s0 = row_off[row];
        nitems = a.has_l2l + row_off[row + 1] - s0;
        first = w;
        step = DW;
    } else {
        box = (int64_t)a.nrt * a.ncol + (int64_t)(bx - a.nb_m2l) * DW + w;
        if (box >= (int64_t)a.rows_l2l * a.ncol) return;  // whole wave; no block barrier on this path
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

template <typename T>
__global__ void __launch_bounds__(64 * DW) k_down(DownK<T> a) { down_body<T>(a, blockIdx.x); }
template <typename T>
__global__ void __launch_bounds__(64 * DW) k_down_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    down_body<T>(static_cast<const DownK<T> *>(m.args)[i], bx);
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
    int nrow[M2L_MAXLEV];  // target rows of the launch at each level
    int64_t off_s[M2L_MAXLEV], off_t[M2L_MAXLEV];
    const int32_t *occ[M2L_MAXLEV];  // source-box occupancy flags (null: not used)
    const cx<T> *atab[M2L_MAXLEV];
    const int *cls3[M2L_MAXLEV];
    const int *row_off[M2L_MAXLEV];
};

constexpr int M2L_DW = 8;  // waves per target box in the M2L launch
template <typename T>
struct M2LK {
    M2LLevels<T> a;
    int nrhs;
    const cx<T> *M;
    cx<T> *Lc;
};
template <typename T>
__device__ __forceinline__ void m2l_all_body(const M2LK<T> &k, const int bx)
{
    const M2LLevels<T> &a = k.a;
    const int nrhs = k.nrhs;
    const cx<T> *__restrict__ M = k.M;
    cx<T> *__restrict__ Lc = k.Lc;
    constexpr int R = Tr<T>::R;
    __shared__ WaveLds<T> lds[M2L_DW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int li = 0;
    while (li + 1 < a.n && bx >= a.blk0[li + 1]) ++li;
    const int box = bx - a.blk0[li];
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

template <typename T>
__global__ void __launch_bounds__(64 * M2L_DW) k_m2l_all(M2LK<T> a) { m2l_all_body<T>(a, blockIdx.x); }
template <typename T>
__global__ void __launch_bounds__(64 * M2L_DW) k_m2l_all_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    m2l_all_body<T>(static_cast<const M2LK<T> *>(m.args)[i], bx);
}

// ---------------------------------------------------------------------------
// M2L on the matrix cores (Lemma M2L written as products of matrices).  A
// translation class (target row, source row, column offset) has one table
// A_s for every box of its rows, so the local expansions of a tile of
// neighbouring target boxes in a row are
//   L[p][(box, rhs)] = sum over the row's class slots s of
//                      sum_q A_s[q][p] M[source box of (box, s)][rhs][q],
// a sum of (2P+1) x (2P+1) by (2P+1) x 16 products: 16 columns = NB boxes x
// RC right-hand sides.  A block of MW waves takes one (level, row, column
// tile, right-hand-side chunk, 16-row tile of p); its waves take the slots in
// turn and run each slot's product on v_mfma_f32_16x16x4f32 (FP32 path) or
// v_mfma_f64_16x16x4f64 (FP64 path), the complex product as four real ones.
// FP32: every slot's product starts from zero and is added to the wave's sum
// with compensation (Kahan), so the sum's rounding error does not grow with
// the number of slots; the waves' sums are then added in wave order (again
// compensated).  Operand layout of both instructions (checked on the GPU):
// lane l supplies row l % 16, column l / 16 of the 16 x 4 left factor and row
// l / 16, column l % 16 of the 4 x 16 right factor; register v of the FP32
// result holds entry (4 (l / 16) + v, l % 16), of the FP64 result entry
// (l / 16 + 4 v, l % 16).
// ---------------------------------------------------------------------------
constexpr int MW = 4;       // waves per block
// waves per block at the coarsest level (every non-adjacent pair: long slot
// lists); measured on the batched workload, 8 beat 4 and 16 in FP32, and the
// FP64 operand prefetch needs more registers than a 16-wave block allows
template <typename T>
constexpr int mw_top() { return 8; }
constexpr int MKS = 8;      // k-steps (4 coefficients each) whose operands are loaded together
template <typename T>
struct M2LMK {
    M2LLevels<T> a;  // blk0: first block of each level
    int nrhs, RC, NB;
    const cx<T> *M;
    cx<T> *Lc;
};
typedef float mf32x4 __attribute__((ext_vector_type(4)));
typedef double mf64x4 __attribute__((ext_vector_type(4)));

__device__ inline void mfma_c(mf32x4 &dr, mf32x4 &di, cx<float> x, cx<float> y)
{
    dr = __builtin_amdgcn_mfma_f32_16x16x4f32(x.re, y.re, dr, 0, 0, 0);
    dr = __builtin_amdgcn_mfma_f32_16x16x4f32(-x.im, y.im, dr, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_16x16x4f32(x.re, y.im, di, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_16x16x4f32(x.im, y.re, di, 0, 0, 0);
}
// FP64 complex product as three real ones (Gauss): with t1 = (xr + xi) yr,
// t2 = xr (yi - yr) and t3 = xi (yr + yi), the real part is t1 - t3 and the
// imaginary part t1 + t2.  The extra rounding is a few units in the last
// place of FP64.
__device__ inline void mfma_c3(mf64x4 &t1, mf64x4 &t2, mf64x4 &t3, cx<double> x, cx<double> y)
{
    t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x.re + x.im, y.re, t1, 0, 0, 0);
    t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x.re, y.im - y.re, t2, 0, 0, 0);
    t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(x.im, y.re + y.im, t3, 0, 0, 0);
}
__device__ inline void mfma_c(mf64x4 &dr, mf64x4 &di, cx<double> x, cx<double> y)
{
    dr = __builtin_amdgcn_mfma_f64_16x16x4f64(x.re, y.re, dr, 0, 0, 0);
    dr = __builtin_amdgcn_mfma_f64_16x16x4f64(-x.im, y.im, dr, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f64_16x16x4f64(x.re, y.im, di, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f64_16x16x4f64(x.im, y.re, di, 0, 0, 0);
}

template <typename T, int NW>
__device__ __forceinline__ void m2l_mfma_body(const M2LMK<T> &k, const int bx)
{
    typedef typename std::conditional<sizeof(T) == 4, mf32x4, mf64x4>::type vx4;
    constexpr bool F32 = sizeof(T) == 4;
    const M2LLevels<T> &a = k.a;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    int li = 0;
    while (li + 1 < a.n && bx >= a.blk0[li + 1]) ++li;
    int loc = bx - a.blk0[li];
    const int nc = a.nc[li], ncol = a.ncol[li], col_lo = a.col_lo[li];
    const int npt = (nc + 15) >> 4, ntile = (ncol + k.NB - 1) / k.NB, nrc = (k.nrhs + k.RC - 1) / k.RC;
    // block index within the level: coefficient tile fastest, then the
    // right-hand-side chunk, the column tile and the target row
    const int pt = loc % npt;
    loc /= npt;
    const int rcn = loc % nrc;
    loc /= nrc;
    const int tile = loc % ntile, row = loc / ntile;
    const int n = l & 15, kk = l >> 4;
    const int j = n / k.RC, r = rcn * k.RC + n % k.RC;
    const int colL = tile * k.NB + j, col = col_lo + colL;
    const bool nvalid = colL < ncol && r < k.nrhs;
    const int p = pt * 16 + n;  // output coefficient of this lane's row of the left factor
    const int *__restrict__ cls3 = a.cls3[li];
    const int s0 = a.row_off[li][row], s1 = a.row_off[li][row + 1];
    const cx<T> *__restrict__ Ms = k.M + a.off_s[li];
    const cx<T> *__restrict__ At = a.atab[li];
    const int nks = (nc + 3) >> 2;
    vx4 sr = {0, 0, 0, 0}, si = {0, 0, 0, 0}, cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    const int rows_s = a.rows_s[li];
    const bool top = a.top[li];
    const int32_t *__restrict__ occ = a.occ[li];
    // a slot's source box for this lane's column, and whether it is in range
    // (adjacent parents at the levels below the coarsest); an empty source box
    // has a zero expansion, so its flag is read too and the slot skipped when
    // no lane has a source.  The next slot's entry, flag and first MKS steps of
    // operands are read while the current slot computes (operands of boxes in
    // range; those of empty boxes are dropped when used).
    auto probe = [&](int ss, int &rs_, int &csl_, bool &in_, int &flag_) {
        rs_ = cls3[3 * ss + 1];
        const int cs = col + cls3[3 * ss + 2];
        csl_ = cs - col_lo;
        const int dp = (cs >> 1) - (col >> 1);
        in_ = nvalid && rs_ < rows_s && csl_ >= 0 && csl_ < ncol && (top || (dp >= -1 && dp <= 1));
        flag_ = in_ ? (occ ? occ[(int64_t)rs_ * ncol + csl_] : 1) : 0;
    };
    auto load_steps = [&](int ss, int rs_, int csl_, bool in_, int k0, cx<T> (&av)[MKS], cx<T> (&bv)[MKS]) {
        const cx<T> *__restrict__ As = At + (int64_t)ss * nc * nc;
        const cx<T> *__restrict__ xb = Ms + (((int64_t)(in_ ? rs_ : 0) * ncol + (in_ ? csl_ : 0)) * k.nrhs + (in_ ? r : 0)) * nc;
#pragma unroll
        for (int u = 0; u < MKS; ++u) {
            const int kq = 4 * (k0 + u) + kk;
            const bool kin = kq < nc;
            av[u] = (kin && p < nc) ? As[(int64_t)kq * nc + p] : mk<T>(0, 0);
            bv[u] = (kin && in_) ? xb[kq] : mk<T>(0, 0);
        }
    };
    if constexpr (F32) {
        // FP32: the next slot's entry and flag only (a prefetch of operands was
        // slower: more registers, fewer waves)
        int rsN = 0, cslN = 0, flagN = 0;
        bool inN = false;
        if (s0 + w < s1) probe(s0 + w, rsN, cslN, inN, flagN);
        for (int s = s0 + w; s < s1; s += NW) {
            const int rs = rsN, csl = cslN;
            const bool ok = flagN != 0;
            if (s + NW < s1) probe(s + NW, rsN, cslN, inN, flagN);
            if (!__any(ok)) continue;
            const cx<T> *__restrict__ As = At + (int64_t)s * nc * nc;
            const cx<T> *__restrict__ xb = Ms + (((int64_t)rs * ncol + (ok ? csl : 0)) * k.nrhs + (ok ? r : 0)) * nc;
            vx4 dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
            // the 4-wave launch (levels below the coarsest) has registers for
            // ten steps in flight, a whole column up to order 19
            constexpr int MK = NW == 4 ? 10 : MKS;
            for (int k0 = 0; k0 < nks; k0 += MK) {
                cx<T> av[MK], bv[MK];
#pragma unroll
                for (int u = 0; u < MK; ++u) {
                    const int kq = 4 * (k0 + u) + kk;
                    const bool kin = kq < nc;
                    av[u] = (kin && p < nc) ? As[(int64_t)kq * nc + p] : mk<T>(0, 0);
                    bv[u] = (kin && ok) ? xb[kq] : mk<T>(0, 0);
                }
#pragma unroll
                for (int u = 0; u < MK; ++u)
                    if (k0 + u < nks) mfma_c(dr, di, av[u], bv[u]);
            }
            // compensated addition of the slot's product to the wave's sum
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T yr = dr[v] - cr[v], yi = di[v] - ci[v];
                const T tr = sr[v] + yr, ti = si[v] + yi;
                cr[v] = (tr - sr[v]) - yr;
                ci[v] = (ti - si[v]) - yi;
                sr[v] = tr;
                si[v] = ti;
            }
        }
    } else {
        int rsN = 0, cslN = 0, flagN = 0;
        bool inN = false;
        cx<T> avN[MKS], bvN[MKS];
        if (s0 + w < s1) {
            probe(s0 + w, rsN, cslN, inN, flagN);
            load_steps(s0 + w, rsN, cslN, inN, 0, avN, bvN);
        }
        for (int s = s0 + w; s < s1; s += NW) {
            const int rs = rsN, csl = cslN;
            const bool in = inN, ok = flagN != 0;
            cx<T> av0[MKS], bv0[MKS];
#pragma unroll
            for (int u = 0; u < MKS; ++u) {
                av0[u] = avN[u];
                bv0[u] = ok ? bvN[u] : mk<T>(0, 0);
            }
            if (s + NW < s1) {
                probe(s + NW, rsN, cslN, inN, flagN);
                load_steps(s + NW, rsN, cslN, inN, 0, avN, bvN);
            }
            if (!__any(ok)) continue;
            vx4 t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < MKS; ++u)
                if (u < nks) mfma_c3(t1, t2, t3, av0[u], bv0[u]);
            for (int k0 = MKS; k0 < nks; k0 += MKS) {
                cx<T> av[MKS], bv[MKS];
                load_steps(s, rs, csl, in, k0, av, bv);
#pragma unroll
                for (int u = 0; u < MKS; ++u)
                    if (k0 + u < nks) mfma_c3(t1, t2, t3, av[u], ok ? bv[u] : mk<T>(0, 0));
            }
            const vx4 dr = t1 - t3, di = t1 + t2;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                sr[v] += dr[v];
                si[v] += di[v];
            }
        }
    }
    // the waves' sums added in wave order by wave 0, four waves per round
    __shared__ T red[4][4][4][64];  // wave of the round, (sr, si, cr, ci), v, lane
    CAcc<T> are[4], aim[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        are[v].zero();
        aim[v].zero();
    }
    for (int r0 = 0; r0 < NW; r0 += 4) {
        if (w >= r0 && w < r0 + 4) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                red[w - r0][0][v][l] = sr[v];
                red[w - r0][1][v][l] = si[v];
                red[w - r0][2][v][l] = cr[v];
                red[w - r0][3][v][l] = ci[v];
            }
        }
        __syncthreads();
        if (w == 0)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                for (int x = 0; x < 4; ++x) {
                    are[v].add({red[x][0][v][l], -red[x][2][v][l]});
                    aim[v].add({red[x][1][v][l], -red[x][3][v][l]});
                }
        __syncthreads();
    }
    if (w != 0 || !nvalid) return;
    const int64_t obase = a.off_t[li] + (((int64_t)row * ncol + colL) * k.nrhs + r) * nc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int prow = F32 ? 4 * kk + v : kk + 4 * v;
        const int pp = pt * 16 + prow;
        const cx<T> vr = are[v].value(), vi = aim[v].value();
        if (pp < nc) k.Lc[obase + pp] = mk<T>(vr.re + vr.im, vi.re + vi.im);
    }
}
template <typename T, int NW>
__global__ void __launch_bounds__(64 * NW) k_m2l_mfma(M2LMK<T> a) { m2l_mfma_body<T, NW>(a, blockIdx.x); }
template <typename T, int NW>
__global__ void __launch_bounds__(64 * NW) k_m2l_mfma_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    m2l_mfma_body<T, NW>(static_cast<const M2LMK<T> *>(m.args)[i], bx);
}

// ---------------------------------------------------------------------------
// M2M and L2L on the matrix cores (Lemma M2M, Lemma L2L): per child position
// the shift table (in x out) times the expansions of a tile of NB output
// boxes x RC right-hand sides, v_mfma_f32_16x16x4f32 (FP64: ..._f64_...) with
// the lane layouts of the M2L kernel above.
//   M2M (UP = true): a block takes one tile of parent boxes and one tile of 16
//   output coefficients; wave w takes child position w; the four products
//   are added in wave order through LDS.  It also writes the parents'
//   occupancy flags.
//   L2L (UP = false): a block takes one tile of child boxes of one column
//   parity (so that they share the position and the table) and four tiles of
//   output coefficients, one per wave; rows below add_rows add their stored
//   M2L result.
// ---------------------------------------------------------------------------
template <typename T>
struct ShiftMK {
    const cx<T> *X;  // input expansions (children for M2M, parents for L2L)
    cx<T> *Y;        // output expansions
    const cx<T> *tab;  // [4][nc_in][nc_out]
    int nc_in, ncol_in, col_lo_in, rows_in;
    int nc_out, ncol_out, col_lo_out, rows_out;  // rows_out: output rows computed
    int nrhs, RC, NB, add_rows;
    const int32_t *occ_in;  // M2M: children's occupancy flags
    int32_t *occ_out;       // M2M: parents'
};
template <typename T, bool UP>
__device__ __forceinline__ void shift_mfma_body(const ShiftMK<T> &k, const int bx)
{
    // operand steps in flight: with FP32, a whole column up to order 23 at
    // once (with FP64 the registers would cost a wave per SIMD)
    constexpr int MKS_SH = sizeof(T) == 4 ? 12 : MKS;
    typedef typename std::conditional<sizeof(T) == 4, mf32x4, mf64x4>::type vx4;
    constexpr bool F32 = sizeof(T) == 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const int nin = k.nc_in, nout = k.nc_out;
    const int npt = (nout + 15) >> 4, npb = UP ? npt : (npt + 3) >> 2;  // p-tile blocks
    // L2L: tiles of boxes of one column parity: half-tiles 0 .. nth-1 take
    // the columns colL = c0 + 2 m (c0 = 0 or 1), m in the tile
    const int nhalf = (k.ncol_out + 1) >> 1, nth = (nhalf + k.NB - 1) / k.NB;
    const int ntile = UP ? (k.ncol_out + k.NB - 1) / k.NB : 2 * nth, nrc = (k.nrhs + k.RC - 1) / k.RC;
    int loc = bx;
    const int ptb = loc % npb;
    loc /= npb;
    const int rcn = loc % nrc;
    loc /= nrc;
    const int tile = loc % ntile, row = loc / ntile;
    const int pt = UP ? ptb : 4 * ptb + w;  // this wave's tile of output coefficients
    const int n = l & 15, kk = l >> 4;
    const int j = n / k.RC, r = rcn * k.RC + n % k.RC;
    const int colL = UP ? tile * k.NB + j : (tile & 1) + 2 * ((tile >> 1) * k.NB + j);
    const int col = k.col_lo_out + colL;
    const bool nvalid = colL < k.ncol_out && r < k.nrhs && row < k.rows_out;
    const int p = pt * 16 + n;  // this lane's row of the left factor (output coefficient)
    // the input box and the child position
    int irow, icl, pos;
    if (UP) {
        pos = w;
        irow = 2 * row + (w >> 1);
        icl = 2 * col + (w & 1) - k.col_lo_in;
    } else {
        pos = (col & 1) + 2 * (row & 1);
        irow = row >> 1;
        icl = (col >> 1) - k.col_lo_in;
    }
    bool ok = nvalid && irow < k.rows_in && icl >= 0 && icl < k.ncol_in;
    if (UP && ok && k.occ_in) ok = k.occ_in[(int64_t)irow * k.ncol_in + icl] != 0;
    if (UP && rcn == 0 && ptb == 0 && threadIdx.x < k.NB) {
        // parents' occupancy: any child holds sources
        const int cL = tile * k.NB + threadIdx.x, pc = k.col_lo_out + cL;
        if (cL < k.ncol_out && row < k.rows_out) {
            int any = 0;
            for (int c = 0; c < 4; ++c) {
                const int cr = 2 * row + (c >> 1), cc = 2 * pc + (c & 1) - k.col_lo_in;
                if (cr < k.rows_in && cc >= 0 && cc < k.ncol_in) any |= k.occ_in[(int64_t)cr * k.ncol_in + cc];
            }
            k.occ_out[(int64_t)row * k.ncol_out + cL] = any;
        }
    }
    vx4 dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
    if (__any(ok) && (UP || pt < npt)) {
        const cx<T> *__restrict__ A = k.tab + (int64_t)pos * nin * nout;
        const cx<T> *__restrict__ xb =
            k.X + (((int64_t)(ok ? irow : 0) * k.ncol_in + (ok ? icl : 0)) * k.nrhs + (ok ? r : 0)) * nin;
        const int nks = (nin + 3) >> 2;
        for (int k0 = 0; k0 < nks; k0 += MKS_SH) {
            cx<T> av[MKS_SH], bv[MKS_SH];
#pragma unroll
            for (int u = 0; u < MKS_SH; ++u) {
                const int kq = 4 * (k0 + u) + kk;
                const bool kin = kq < nin;
                av[u] = (kin && p < nout) ? A[(int64_t)kq * nout + p] : mk<T>(0, 0);
                bv[u] = (kin && ok) ? xb[kq] : mk<T>(0, 0);
            }
#pragma unroll
            for (int u = 0; u < MKS_SH; ++u)
                if (k0 + u < nks) mfma_c(dr, di, av[u], bv[u]);
        }
    }
    if (UP) {
        // the four positions' products added in wave order by wave 0
        __shared__ T red[4][2][4][64];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            red[w][0][v][l] = dr[v];
            red[w][1][v][l] = di[v];
        }
        __syncthreads();
        if (w != 0 || !nvalid) return;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            dr[v] = red[0][0][v][l] + red[1][0][v][l] + red[2][0][v][l] + red[3][0][v][l];
            di[v] = red[0][1][v][l] + red[1][1][v][l] + red[2][1][v][l] + red[3][1][v][l];
        }
    }
    if (!nvalid || pt >= npt) return;
    cx<T> *__restrict__ out = k.Y + (((int64_t)row * k.ncol_out + colL) * k.nrhs + r) * nout;
    const bool add = !UP && row < k.add_rows;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int prow = F32 ? 4 * kk + v : kk + 4 * v;
        const int pp = pt * 16 + prow;
        if (pp < nout) {
            cx<T> val = mk<T>(dr[v], di[v]);
            if (add) val += out[pp];
            out[pp] = val;
        }
    }
}
template <typename T, bool UP>
__global__ void __launch_bounds__(256) k_shift_mfma(ShiftMK<T> a) { shift_mfma_body<T, UP>(a, blockIdx.x); }
template <typename T, bool UP>
__global__ void __launch_bounds__(256) k_shift_mfma_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    shift_mfma_body<T, UP>(static_cast<const ShiftMK<T> *>(m.args)[i], bx);
}

}  // namespace

template <typename T>
void launch_m2m(const Geometry &g, int lc, const cx<T> *tab, cx<T> *M, int32_t *occ, int nrhs, bool mfma,
                hipStream_t st)
{
    const Level &c = g.lev[lc], &p = g.lev[lc - 1];
    int nbox = p.rows_s * p.ncol;
    if (nbox == 0) return;
    if (mfma) {
        const int RC = nrhs >= 16 ? 16 : (nrhs > 8 ? 16 : (nrhs > 4 ? 8 : (nrhs > 2 ? 4 : nrhs))), NB = 16 / RC;
        const ShiftMK<T> a{M + c.off_s, M + p.off_s, tab, c.nc, c.ncol, c.col_lo, c.rows_s, p.nc, p.ncol, p.col_lo,
                           p.rows_s, nrhs, RC, NB, 0, occ + c.off_occ, occ + p.off_occ};
        const int64_t nblk = (int64_t)p.rows_s * ((p.ncol + NB - 1) / NB) * ((nrhs + RC - 1) / RC) * ((p.nc + 15) / 16);
        emit((const void *)k_shift_mfma<T, true>, (const void *)k_shift_mfma_multi<T, true>, 0, dim3((unsigned)nblk),
             dim3(256), 0, st, a);
        return;
    }
    const UpArgs<T> a{M + c.off_s, M + p.off_s, tab, nrhs, c.nc, p.nc, c.ncol, c.col_lo, c.rows_s, p.ncol, p.col_lo,
                      occ + c.off_occ, occ + p.off_occ};
    emit((const void *)k_up<T>, (const void *)k_up_multi<T>, 0, dim3(nbox), dim3(256), 0, st, a);
}

template <typename T>
void launch_down(const Geometry &g, int l, const cx<T> *atab, const int *cls3, const int *row_off, int nrt,
                 const cx<T> *M, cx<T> *Lc, int nrhs, const cx<T> *l2l_tab, bool top, int add_rows, hipStream_t st,
                 int rows_l2l, bool mfma)
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
    a.rows_l2l = rows_l2l < 0 || rows_l2l > lv.rows_t ? lv.rows_t : rows_l2l;
    if (mfma && !atab && l2l_tab) {
        // the L2L form on the matrix cores
        const int RC = nrhs >= 16 ? 16 : (nrhs > 8 ? 16 : (nrhs > 4 ? 8 : (nrhs > 2 ? 4 : nrhs))), NB = 16 / RC;
        const ShiftMK<T> s{Lc + pv.off_t, Lc + lv.off_t, l2l_tab, pv.nc, pv.ncol, pv.col_lo, pv.rows_t, lv.nc, lv.ncol,
                           lv.col_lo, a.rows_l2l, nrhs, RC, NB, add_rows, nullptr, nullptr};
        const int nth = (((lv.ncol + 1) >> 1) + NB - 1) / NB;
        const int64_t nblk =
            (int64_t)a.rows_l2l * 2 * nth * ((nrhs + RC - 1) / RC) * ((((lv.nc + 15) / 16) + 3) / 4);
        if (nblk == 0) return;
        emit((const void *)k_shift_mfma<T, false>, (const void *)k_shift_mfma_multi<T, false>, 0,
             dim3((unsigned)nblk), dim3(256), 0, st, s);
        return;
    }
    int64_t rest = (int64_t)(a.rows_l2l > a.nrt ? a.rows_l2l - a.nrt : 0) * lv.ncol;
    int64_t nblk = a.nb_m2l + (a.has_l2l ? (rest + DW - 1) / DW : 0);
    if (nblk == 0) return;
    const DownK<T> k{a, nrhs, Lc + pv.off_t, l2l_tab, Lc + lv.off_t, M + lv.off_s, atab, cls3, row_off};
    emit((const void *)k_down<T>, (const void *)k_down_multi<T>, 0, dim3((unsigned)nblk), dim3(64 * DW), 0, st, k);
}

template <typename T>
void launch_m2l_all(const Geometry &g, int l0, int l1, const cx<T> *const *atab, const int *const *cls3,
                    const int *const *row_off, const int *nrt, const cx<T> *M, cx<T> *Lc, int nrhs, bool mfma,
                    const int32_t *occ, int part, hipStream_t st)
{
    // matrix-core form: columns of 16 = NB boxes x RC right-hand sides
    const int RC = nrhs >= 16 ? 16 : (nrhs > 8 ? 16 : (nrhs > 4 ? 8 : (nrhs > 2 ? 4 : nrhs))), NB = 16 / RC;
    // the levels of one launch: the coarsest level alone (its rows list every
    // non-adjacent pair, so its blocks take more waves) or all the others
    auto levels = [&](bool top, M2LLevels<T> &a) {
        a.n = 0;
        int blk = 0;
        for (int l = l0; l <= l1 && a.n < M2L_MAXLEV; ++l) {
            if (mfma && (l == g.ltop) != top) continue;
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
            a.occ[i] = occ ? occ + lv.off_occ : nullptr;
            a.atab[i] = atab[l - l0];
            a.cls3[i] = cls3[l - l0];
            a.row_off[i] = row_off[l - l0];
            a.nrow[i] = rows;
            if (mfma)
                blk += rows * ((lv.ncol + NB - 1) / NB) * ((nrhs + RC - 1) / RC) * ((lv.nc + 15) / 16);
            else
                blk += rows * lv.ncol;
        }
        a.blk0[a.n] = blk;
        return blk;
    };
    M2LLevels<T> a;
    if (mfma) {
        if (part != 2 && levels(true, a) > 0) {
            const M2LMK<T> k{a, nrhs, RC, NB, M, Lc};
            // a block's slots run over every source box of the level, each a
            // product of about nc^2 / 4 steps
            const Level &lt = g.lev[g.ltop];
            launch_cost() = (double)lt.rows_s * lt.ncol * lt.nc * lt.nc;
            emit((const void *)k_m2l_mfma<T, mw_top<T>()>, (const void *)k_m2l_mfma_multi<T, mw_top<T>()>, 0,
                 dim3(a.blk0[a.n]), dim3(64 * mw_top<T>()), 0, st, k);
            launch_cost() = 0;
        }
        if (part != 1 && levels(false, a) > 0) {
            const M2LMK<T> k{a, nrhs, RC, NB, M, Lc};
            emit((const void *)k_m2l_mfma<T, MW>, (const void *)k_m2l_mfma_multi<T, MW>, 0, dim3(a.blk0[a.n]),
                 dim3(64 * MW), 0, st, k);
        }
        return;
    }
    if (part == 2 || levels(false, a) == 0) return;
    const M2LK<T> k{a, nrhs, M, Lc};
    emit((const void *)k_m2l_all<T>, (const void *)k_m2l_all_multi<T>, 0, dim3(a.blk0[a.n]), dim3(64 * M2L_DW), 0, st,
         k);
}


#define LMFMM_INST(T)                                                                                               \
    template void launch_m2m<T>(const Geometry &, int, const cx<T> *, cx<T> *, int32_t *, int, bool, hipStream_t);  \
    template void launch_down<T>(const Geometry &, int, const cx<T> *, const int *, const int *, int, const cx<T> *, \
                                 cx<T> *, int, const cx<T> *, bool, int, hipStream_t, int, bool);                   \
    template void launch_m2l_all<T>(const Geometry &, int, int, const cx<T> *const *, const int *const *,           \
                                    const int *const *, const int *, const cx<T> *, cx<T> *, int, bool,             \
                                    const int32_t *, int, hipStream_t);
LMFMM_INST(double)
LMFMM_INST(float)

}  // namespace lmfmm
