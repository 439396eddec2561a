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
    int64_t off_s[M2L_MAXLEV], off_t[M2L_MAXLEV];
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

}  // namespace

template <typename T>
void launch_m2m(const Geometry &g, int lc, const cx<T> *tab, cx<T> *M, int nrhs, hipStream_t st)
{
    const Level &c = g.lev[lc], &p = g.lev[lc - 1];
    int nbox = p.rows_s * p.ncol;
    if (nbox == 0) return;
    const UpArgs<T> a{M + c.off_s, M + p.off_s, tab, nrhs, c.nc, p.nc, c.ncol, c.col_lo, c.rows_s, p.ncol, p.col_lo};
    emit((const void *)k_up<T>, (const void *)k_up_multi<T>, 0, dim3(nbox), dim3(256), 0, st, a);
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
    const DownK<T> k{a, nrhs, Lc + pv.off_t, l2l_tab, Lc + lv.off_t, M + lv.off_s, atab, cls3, row_off};
    emit((const void *)k_down<T>, (const void *)k_down_multi<T>, 0, dim3((unsigned)nblk), dim3(64 * DW), 0, st, k);
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
    const M2LK<T> k{a, nrhs, M, Lc};
    emit((const void *)k_m2l_all<T>, (const void *)k_m2l_all_multi<T>, 0, dim3(blk), dim3(64 * M2L_DW), 0, st, k);
}


#define LMFMM_INST(T)                                                                                               \
    template void launch_m2m<T>(const Geometry &, int, const cx<T> *, cx<T> *, int, hipStream_t);                   \
    template void launch_down<T>(const Geometry &, int, const cx<T> *, const int *, const int *, int, const cx<T> *, \
                                 cx<T> *, int, const cx<T> *, bool, int, hipStream_t);                              \
    template void launch_m2l_all<T>(const Geometry &, int, int, const cx<T> *const *, const int *const *,           \
                                    const int *const *, const int *, const cx<T> *, cx<T> *, int, hipStream_t);
LMFMM_INST(double)
LMFMM_INST(float)

}  // namespace lmfmm
