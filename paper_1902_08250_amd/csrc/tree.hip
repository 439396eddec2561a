// Quadtree construction (Algorithm 1, Step 1): bounding box and layer checks,
// leaf keys, and the points grouped by leaf.
//
// The tree is uniform with its root square split at the interface y = 0, so
// every box holds either sources (above) or targets (below).  A leaf key is
// (row, column) of the level-L box; target keys follow all source keys, so one
// grouping orders both point sets and the grouped array holds sources first.
// Grouping is a counting sort: per-leaf counts (atomics, whose old values are
// the points' slots), one exclusive scan for the leaf ranges, a scatter to the
// slots, and a per-leaf sort of the scattered original indices, so that every
// leaf lists its points in increasing original index whatever order the
// atomics took.
#include "lmfmm_internal.h"

namespace lmfmm {

namespace {

constexpr int BB_THREADS = 256;

__device__ inline double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Per-block partial bounding box: xmin, xmax over all points; source y min/max;
// target y min/max; count of points outside their layer or not finite.  The
// points are taken as one sequence, sources then targets, in chunks of
// BB_PER * BB_THREADS per block; a thread issues the loads of its BB_PER points
// before using any of them.
constexpr int BB_PER = 4;
__global__ void __launch_bounds__(BB_THREADS) k_bbox_partial(const double *__restrict__ src, int64_t ns,
                                                             const double *__restrict__ tgt, int64_t nt, Layers ly,
                                                             double *__restrict__ partial)
{
    double v[7] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    const int64_t n = ns + nt, chunk = (int64_t)BB_PER * BB_THREADS;
    for (int64_t base = (int64_t)blockIdx.x * chunk; base < n; base += (int64_t)gridDim.x * chunk) {
        double x[BB_PER], y[BB_PER];
#pragma unroll
        for (int k = 0; k < BB_PER; ++k) {
            const int64_t i = base + k * BB_THREADS + threadIdx.x;
            x[k] = 0.0;
            y[k] = 0.0;
            if (i < ns) {
                x[k] = src[i];
                y[k] = src[ns + i];
            } else if (i < n) {
                x[k] = tgt[i - ns];
                y[k] = fma(ly.ty_a, tgt[nt + i - ns], ly.ty_b);
            }
        }
#pragma unroll
        for (int k = 0; k < BB_PER; ++k) {
            const int64_t i = base + k * BB_THREADS + threadIdx.x;
            if (i >= n) continue;
            const bool tg = i >= ns;
            const bool ok = isfinite(x[k]) && isfinite(y[k]) && (tg ? (y[k] < ly.yt_hi && y[k] > ly.yt_lo)
                                                                    : (y[k] > ly.ys_lo && y[k] < ly.ys_hi));
            if (!ok) {
                v[6] += 1.0;
                continue;
            }
            v[0] = fmin(v[0], x[k]);
            v[1] = fmax(v[1], x[k]);
            if (tg) {
                v[4] = fmin(v[4], y[k]);
                v[5] = fmax(v[5], y[k]);
            } else {
                v[2] = fmin(v[2], y[k]);
                v[3] = fmax(v[3], y[k]);
            }
        }
    }
    __shared__ double red[BB_THREADS / 64][7];
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double r[7];
    r[0] = wave_min(v[0]);
    r[1] = wave_max(v[1]);
    r[2] = wave_min(v[2]);
    r[3] = wave_max(v[3]);
    r[4] = wave_min(v[4]);
    r[5] = wave_max(v[5]);
    r[6] = wave_sum(v[6]);
    if (lane == 0)
        for (int j = 0; j < 7; ++j) red[wv][j] = r[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BB_THREADS / 64; ++w) {
            r[0] = fmin(r[0], red[w][0]);
            r[1] = fmax(r[1], red[w][1]);
            r[2] = fmin(r[2], red[w][2]);
            r[3] = fmax(r[3], red[w][3]);
            r[4] = fmin(r[4], red[w][4]);
            r[5] = fmax(r[5], red[w][5]);
            r[6] += red[w][6];
        }
        for (int j = 0; j < 7; ++j) partial[blockIdx.x * 8 + j] = r[j];
    }
}

// One wave reduces the nblk partials and writes the box to host-visible
// memory, then its sequence number: one more than the previous launch's, kept
// in device memory (*dseq), so that launches replayed from a graph still
// number their results.
__global__ void __launch_bounds__(64) k_bbox_final(const double *__restrict__ partial, int nblk,
                                                   uint64_t *__restrict__ dseq, double *out)
{
    double v2[7] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    for (int b = threadIdx.x; b < nblk; b += 64) {
        double q[7];
        for (int j = 0; j < 7; ++j) q[j] = partial[b * 8 + j];
        v2[0] = fmin(v2[0], q[0]);
        v2[1] = fmax(v2[1], q[1]);
        v2[2] = fmin(v2[2], q[2]);
        v2[3] = fmax(v2[3], q[3]);
        v2[4] = fmin(v2[4], q[4]);
        v2[5] = fmax(v2[5], q[5]);
        v2[6] += q[6];
    }
    v2[0] = wave_min(v2[0]);
    v2[1] = wave_max(v2[1]);
    v2[2] = wave_min(v2[2]);
    v2[3] = wave_max(v2[3]);
    v2[4] = wave_min(v2[4]);
    v2[5] = wave_max(v2[5]);
    v2[6] = wave_sum(v2[6]);
    if (threadIdx.x == 0) {
        const uint64_t seq = *dseq + 1;
        *dseq = seq;
        for (int j = 0; j < 7; ++j) __hip_atomic_store(&out[j], v2[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(reinterpret_cast<uint64_t *>(out + 8), seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}


// Leaf key of every point.  Sources (y > 0) take row floor(y/w) above the
// interface, targets row floor(-y/w) below it; columns are relative to
// col_lo.  Out-of-range rows/columns (points outside a fixed domain) and
// points in the wrong layer raise the error flag and are clamped.  The
// counter's old value is the point's slot within its leaf (in arrival order;
// the leaf pass sorts each leaf by original index).  The counters start at
// zero: the scan of the previous build cleared them.
struct TreeCountArgs {
    const double *src;
    int64_t ns;
    const double *tgt;
    int64_t nt;
    double x_lo, invw;
    int col_lo, ncol, rows_s, rows_t;
    Layers ly;
    uint32_t *key;
    int32_t *rank, *cnt, *err;
};
constexpr int TC_THREADS = 1024;  // threads per block of the count (1024 finished a few microseconds sooner than 256)
__device__ __forceinline__ void tree_count_body(const TreeCountArgs &a, int bx)
{
    int64_t i = (int64_t)bx * TC_THREADS + threadIdx.x;
    if (i >= a.ns + a.nt) return;
    bool tg = i >= a.ns;
    double x = tg ? a.tgt[i - a.ns] : a.src[i];
    double y = tg ? fma(a.ly.ty_a, a.tgt[a.nt + i - a.ns], a.ly.ty_b) : a.src[a.ns + i];
    bool bad = !(isfinite(x) && isfinite(y)) ||
               (tg ? !(y < a.ly.yt_hi && y > a.ly.yt_lo) : !(y > a.ly.ys_lo && y < a.ly.ys_hi));
    double fc = floor((x - a.x_lo) * a.invw) - (double)a.col_lo;
    double fr = floor((tg ? -y : y) * a.invw);
    int rows = tg ? a.rows_t : a.rows_s;
    if (!(fc >= 0.0 && fc < (double)a.ncol && fr >= 0.0 && fr < (double)rows)) bad = true;
    int c = (int)fmin(fmax(fc, 0.0), (double)(a.ncol - 1));
    int r = (int)fmin(fmax(fr, 0.0), (double)(rows - 1));
    if (bad) atomicOr(a.err, 1);
    uint32_t k = (uint32_t)r * (uint32_t)a.ncol + (uint32_t)c;
    if (tg) k += (uint32_t)a.rows_s * (uint32_t)a.ncol;
    a.key[i] = k;
    a.rank[i] = atomicAdd(&a.cnt[k], 1);
}
__global__ void __launch_bounds__(TC_THREADS) k_tree_count(TreeCountArgs a) { tree_count_body(a, blockIdx.x); }
__global__ void __launch_bounds__(TC_THREADS) k_tree_count_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_count_body(static_cast<const TreeCountArgs *>(m.args)[i], bx);
}

// Exclusive scan of the leaf counts by one block, in LDS tiles of SC_TILE
// counts (loaded and stored coalesced): start[b], end[b].  The counters are
// cleared for the next build, and the error flag of this build is moved to
// err[1], where the host reads it (err[0] is cleared).  Counts that do not add
// up to the number of points (counters not zero at the start) leave every
// leaf empty and set bit 1 of err[1], so that no later kernel indexes with
// them.
constexpr int SC_THREADS = 1024, SC_PER = 8, SC_TILE = SC_THREADS * SC_PER;
struct TreeScanArgs {
    int32_t *cnt;
    int64_t nbox, n;
    int32_t *start, *end, *err;
};
__device__ __forceinline__ void tree_scan_body(const TreeScanArgs &A)
{
    int32_t *__restrict__ cnt = A.cnt;
    int32_t *__restrict__ start = A.start;
    int32_t *__restrict__ end = A.end;
    int32_t *__restrict__ err = A.err;
    const int64_t nbox = A.nbox, n = A.n;
    __shared__ int32_t tile[SC_TILE];
    __shared__ int32_t wsum[SC_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) {
        err[1] = err[0];
        err[0] = 0;
    }
    int32_t carry = 0;
    for (int64_t t0 = 0; t0 < nbox; t0 += SC_TILE) {
#pragma unroll
        for (int k = 0; k < SC_PER; ++k) {
            int64_t b = t0 + k * SC_THREADS + t;
            tile[k * SC_THREADS + t] = b < nbox ? cnt[b] : 0;
        }
        __syncthreads();
        int32_t c[SC_PER], s = 0;
#pragma unroll
        for (int k = 0; k < SC_PER; ++k) {
            c[k] = tile[t * SC_PER + k];
            s += c[k];
        }
        int32_t v = s;  // inclusive scan over the wave, then over the waves
        for (int o = 1; o < 64; o <<= 1) {
            int32_t u = __shfl_up(v, o);
            if (lane >= o) v += u;
        }
        if (lane == 63) wsum[wv] = v;
        __syncthreads();
        if (wv == 0) {
            int32_t w = lane < SC_THREADS / 64 ? wsum[lane] : 0;
            for (int o = 1; o < SC_THREADS / 64; o <<= 1) {
                int32_t u = __shfl_up(w, o);
                if (lane >= o) w += u;
            }
            if (lane < SC_THREADS / 64) wsum[lane] = w;
        }
        __syncthreads();
        int32_t run = carry + v - s + (wv > 0 ? wsum[wv - 1] : 0);
#pragma unroll
        for (int k = 0; k < SC_PER; ++k) {
            tile[t * SC_PER + k] = run;
            run += c[k];
        }
        carry += wsum[SC_THREADS / 64 - 1];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SC_PER; ++k) {
            int64_t b = t0 + k * SC_THREADS + t;
            if (b < nbox) {
                int32_t st = tile[k * SC_THREADS + t];
                int32_t n_b = cnt[b];
                start[b] = st;
                end[b] = st + n_b;
                cnt[b] = 0;
            }
        }
        __syncthreads();
    }
    if ((int64_t)carry != n) {
        for (int64_t b = t; b < nbox; b += SC_THREADS) {
            start[b] = 0;
            end[b] = 0;
        }
        if (t == 0) err[1] |= 2;
    }
}

__global__ void __launch_bounds__(SC_THREADS) k_tree_scan(TreeScanArgs a) { tree_scan_body(a); }
__global__ void __launch_bounds__(SC_THREADS) k_tree_scan_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_scan_body(static_cast<const TreeScanArgs *>(m.args)[i]);
}

struct TreeScatterArgs {
    const uint32_t *key;
    const int32_t *rank;
    int64_t n;
    const int32_t *start;
    int32_t *perm;
};
__device__ __forceinline__ void tree_scatter_body(const TreeScatterArgs &a, int bx)
{
    int64_t i = (int64_t)bx * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int64_t pos = (int64_t)a.start[a.key[i]] + a.rank[i];
    if (pos >= 0 && pos < a.n) a.perm[pos] = (int32_t)i;
}
__global__ void __launch_bounds__(256) k_tree_scatter(TreeScatterArgs a) { tree_scatter_body(a, blockIdx.x); }
__global__ void __launch_bounds__(256) k_tree_scatter_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_scatter_body(static_cast<const TreeScatterArgs *>(m.args)[i], bx);
}

__device__ inline void cswap(int32_t &a, int32_t &b, bool up)
{
    if ((a > b) == up) {
        int32_t t = a;
        a = b;
        b = t;
    }
}

// One wave per leaf: sort the leaf's scattered original indices (bitonic; in
// registers up to 64 points, in LDS up to LF_LDS, else in the leaf's own
// slice of the scratch array), then write idx and gather the coordinates.
constexpr int LF_LDS = 1024;  // small, so that many one-wave blocks fit on a CU
struct TreeLeafArgs {
    const int32_t *start, *end, *perm;
    int32_t *scratch, *idx;
    const double *src;
    int64_t ns;
    const double *tgt;
    int64_t nt;
    double *xs, *ys;
    const uint64_t *q;
    uint64_t *qs;
    int nrhs, qw;
    double ty_a, ty_b;  // tree coordinate of a target: ty_a y + ty_b
};
__device__ __forceinline__ void tree_leaf_body(const TreeLeafArgs &A, int b)
{
    const int32_t *__restrict__ start = A.start;
    const int32_t *__restrict__ end = A.end;
    const int32_t *__restrict__ perm = A.perm;
    int32_t *__restrict__ scratch = A.scratch;
    int32_t *__restrict__ idx = A.idx;
    const double *__restrict__ src = A.src;
    const double *__restrict__ tgt = A.tgt;
    double *__restrict__ xs = A.xs;
    double *__restrict__ ys = A.ys;
    const uint64_t *__restrict__ q = A.q;
    uint64_t *__restrict__ qs = A.qs;
    const int64_t ns = A.ns, nt = A.nt;
    const int nrhs = A.nrhs, qw = A.qw;
    __shared__ int32_t sh[LF_LDS];
    const int lane = threadIdx.x;
    const int s = start[b], nb = end[b] - s;
    if (nb <= 0) return;
    auto emit = [&](int k, int32_t o) {
        idx[s + k] = o;
        if (o < ns) {
            xs[s + k] = src[o];
            ys[s + k] = src[ns + o];
            if (q)
                for (int r = 0; r < nrhs; ++r)
                    for (int w = 0; w < qw; ++w)
                        qs[((int64_t)r * ns + s + k) * qw + w] = q[((int64_t)r * ns + o) * qw + w];
        } else {
            xs[s + k] = tgt[o - ns];
            ys[s + k] = fma(A.ty_a, tgt[nt + o - ns], A.ty_b);
        }
    };
    if (nb <= 64) {
        int32_t v = lane < nb ? perm[s + lane] : INT32_MAX;
        for (int k = 2; k <= 64; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                int32_t w = __shfl_xor(v, j);
                bool up = (lane & k) == 0, low = (lane & j) == 0;
                v = (low == up) ? min(v, w) : max(v, w);
            }
        if (lane < nb) emit(lane, v);
        return;
    }
    int m = 128;
    while (m < nb) m <<= 1;
    // the array being sorted: LDS, or the slice [2 s, 2 s + m) of scratch (m <= 2 nb)
    int32_t *a = m <= LF_LDS ? sh : scratch + 2 * (int64_t)s;
    for (int i = lane; i < m; i += 64) a[i] = i < nb ? perm[s + i] : INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < m; i += 64) {
                int p = i ^ j;
                if (p > i) {
                    int32_t x = a[i], y = a[p];
                    cswap(x, y, (i & k) == 0);
                    a[i] = x;
                    a[p] = y;
                }
            }
            __syncthreads();
        }
    for (int i = lane; i < nb; i += 64) emit(i, a[i]);
}

__global__ void __launch_bounds__(64) k_tree_leaf(TreeLeafArgs a) { tree_leaf_body(a, blockIdx.x); }
__global__ void __launch_bounds__(64) k_tree_leaf_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_leaf_body(static_cast<const TreeLeafArgs *>(m.args)[i], bx);
}

struct ZeroArgs {
    uint32_t *p;
    int64_t n;
};
__device__ __forceinline__ void zero_body(const ZeroArgs &a, int bx)
{
    int64_t i = (int64_t)bx * 256 + threadIdx.x;
    if (i < a.n) a.p[i] = 0u;
}
__global__ void __launch_bounds__(256) k_zero_u32(ZeroArgs a) { zero_body(a, blockIdx.x); }
__global__ void __launch_bounds__(256) k_zero_u32_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    zero_body(static_cast<const ZeroArgs *>(m.args)[i], bx);
}

}  // namespace

int bbox_blocks(int64_t n)
{
    // about 1024 points per block, at most 256 blocks (partials of 8 doubles)
    int64_t b = (n + 1023) / 1024;
    if (b < 1) b = 1;
    if (b > 256) b = 256;
    return (int)b;
}

void launch_bbox(const double *src, int64_t ns, const double *tgt, int64_t nt, const Layers &ly, double *partial,
                 uint64_t *dseq, int nblk, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_bbox_partial, dim3(nblk), dim3(BB_THREADS), 0, st, src, ns, tgt, nt, ly, partial);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, partial, nblk, dseq, out);
}


__global__ void k_mirror(const double *__restrict__ xy, int64_t n, double a, double b, double *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        out[i] = xy[i];
        out[n + i] = -fma(a, xy[n + i], b);
    }
}

void launch_mirror(const double *xy, int64_t n, double a, double b, double *out, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mirror, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xy, n, a, b, out);
}


void launch_zero_bytes(void *p, size_t nbytes, hipStream_t st)
{
    int64_t n = (int64_t)(nbytes / 4);
    if (n <= 0) return;
    const ZeroArgs a{(uint32_t *)p, n};
    emit((const void *)k_zero_u32, (const void *)k_zero_u32_multi, 0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
         st, a);
}

void launch_tree(const double *src, int64_t ns, const double *tgt, int64_t nt, double x_lo, double w, int col_lo,
                 int ncol, int rows_s, int rows_t, const Layers &ly, const TreeBufs &b, int32_t *err,
                 hipStream_t st)
{
    const int64_t n = ns + nt;
    const int64_t nbox = (int64_t)(rows_s + rows_t) * ncol;
    if (n == 0 || nbox == 0) return;
    const unsigned g = (unsigned)((n + 255) / 256);
    const TreeCountArgs ca{src, ns, tgt, nt, x_lo, 1.0 / w, col_lo, ncol, rows_s, rows_t, ly, b.key, b.rank, b.cnt, err};
    emit((const void *)k_tree_count, (const void *)k_tree_count_multi, 0,
         dim3((unsigned)((n + TC_THREADS - 1) / TC_THREADS)), dim3(TC_THREADS), 0, st, ca);
    const TreeScanArgs sa{b.cnt, nbox, n, b.start, b.end, err};
    emit((const void *)k_tree_scan, (const void *)k_tree_scan_multi, 1, dim3(1), dim3(SC_THREADS), 0, st, sa);
    const TreeScatterArgs xa{b.key, b.rank, n, b.start, b.perm};
    emit((const void *)k_tree_scatter, (const void *)k_tree_scatter_multi, 2, dim3(g), dim3(256), 0, st, xa);
    const TreeLeafArgs la{b.start, b.end, b.perm, b.scratch, b.idx, src, ns, tgt, nt, b.xs, b.ys, b.q, b.qs, b.nrhs,
                          b.qw, ly.ty_a, ly.ty_b};
    emit((const void *)k_tree_leaf, (const void *)k_tree_leaf_multi, 3, dim3((unsigned)nbox), dim3(64), 0, st, la);
}

}  // namespace lmfmm
