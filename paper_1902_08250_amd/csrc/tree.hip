// Quadtree construction (Algorithm 1, Step 1): bounding box and layer checks,
// leaf keys, and the points grouped by leaf.
//
// The tree is uniform with its root square split at the interface y = 0, so
// every box holds either sources (above) or targets (below).  A leaf key is
// (row, column) of the level-L box; target keys follow all source keys, so one
// grouping orders both point sets and the grouped array holds sources first.
// Grouping has two forms with the same result, every leaf listing its points
// in increasing original index: a stable radix sort of the leaf keys (LDS
// counting only; large trees) and a counting sort by atomics (small trees).
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


// Grouping by leaf is a stable least-significant-digit radix sort of the leaf
// keys: one to four passes over digits of at most 8 bits, each a per-block
// digit histogram, one exclusive scan of the (digit, block) table and a
// stable scatter.  All counting happens in LDS, so no global atomics are
// taken per point.  A last element-parallel pass gathers the coordinates and
// source densities into grouped order and writes the leaf ranges.  Every leaf
// lists its points in increasing original index.
constexpr int RS_THREADS = 256, RS_PER = 8, RS_TILE = RS_THREADS * RS_PER;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_MAXBITS = 8;

// Leaf key of every point.  Sources (y > 0) take row floor(y/w) above the
// interface, targets row floor(-y/w) below it; columns are relative to
// col_lo.  Out-of-range rows/columns (points outside a fixed domain) and
// points in the wrong layer raise the error flag and are clamped.  The same
// kernel counts the first pass's digits and clears the leaf ranges (a leaf
// the last pass does not reach stays empty).
struct TreeKeyArgs {
    const double *src;
    int64_t ns;
    const double *tgt;
    int64_t nt;
    double x_lo, invw;
    int col_lo, ncol, rows_s, rows_t;
    Layers ly;
    uint32_t *key;
    int32_t *tab;  // (digit, block) counts, digit-major
    int32_t *start, *end;
    int64_t nbox;
    int nb, bits;
    int32_t *err;
};
__device__ __forceinline__ void tree_key_body(const TreeKeyArgs &a, int b)
{
    __shared__ int32_t h[1 << RS_MAXBITS];
    const int t = threadIdx.x;
    const uint32_t dmask = (1u << a.bits) - 1u;
    const int64_t n = a.ns + a.nt;
    h[t] = 0;
    for (int64_t k = (int64_t)b * RS_THREADS + t; k < a.nbox; k += (int64_t)a.nb * RS_THREADS) {
        a.start[k] = 0;
        a.end[k] = 0;
    }
    double xv[RS_PER], yv[RS_PER];
#pragma unroll
    for (int r = 0; r < RS_PER; ++r) {
        const int64_t i = (int64_t)b * RS_TILE + r * RS_THREADS + t;
        xv[r] = yv[r] = 0.0;
        if (i < a.ns) {
            xv[r] = a.src[i];
            yv[r] = a.src[a.ns + i];
        } else if (i < n) {
            xv[r] = a.tgt[i - a.ns];
            yv[r] = a.tgt[a.nt + i - a.ns];
        }
    }
    __syncthreads();
    bool bad_any = false;
#pragma unroll
    for (int r = 0; r < RS_PER; ++r) {
        const int64_t i = (int64_t)b * RS_TILE + r * RS_THREADS + t;
        if (i >= n) continue;
        const bool tg = i >= a.ns;
        const double x = xv[r];
        const double y = tg ? fma(a.ly.ty_a, yv[r], a.ly.ty_b) : yv[r];
        bool bad = !(isfinite(x) && isfinite(y)) ||
                   (tg ? !(y < a.ly.yt_hi && y > a.ly.yt_lo) : !(y > a.ly.ys_lo && y < a.ly.ys_hi));
        const double fc = floor((x - a.x_lo) * a.invw) - (double)a.col_lo;
        const double fr = floor((tg ? -y : y) * a.invw);
        const int rows = tg ? a.rows_t : a.rows_s;
        if (!(fc >= 0.0 && fc < (double)a.ncol && fr >= 0.0 && fr < (double)rows)) bad = true;
        const int c = (int)fmin(fmax(fc, 0.0), (double)(a.ncol - 1));
        const int rr = (int)fmin(fmax(fr, 0.0), (double)(rows - 1));
        bad_any |= bad;
        uint32_t k = (uint32_t)rr * (uint32_t)a.ncol + (uint32_t)c;
        if (tg) k += (uint32_t)a.rows_s * (uint32_t)a.ncol;
        a.key[i] = k;
        atomicAdd(&h[k & dmask], 1);
    }
    if (bad_any) atomicOr(a.err, 1);
    __syncthreads();
    if (t <= (int)dmask) a.tab[(int64_t)t * a.nb + b] = h[t];
}
__global__ void __launch_bounds__(RS_THREADS) k_tree_key(TreeKeyArgs a) { tree_key_body(a, blockIdx.x); }
__global__ void __launch_bounds__(RS_THREADS) k_tree_key_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_key_body(static_cast<const TreeKeyArgs *>(m.args)[i], bx);
}

// Digit histogram of a later pass, over the same blocks as its scatter.
struct TreeHistArgs {
    const uint32_t *key;
    int64_t n;
    int32_t *tab;
    int nb, shift, bits;
};
__device__ __forceinline__ void tree_hist_body(const TreeHistArgs &a, int b)
{
    __shared__ int32_t h[1 << RS_MAXBITS];
    const int t = threadIdx.x;
    const uint32_t dmask = (1u << a.bits) - 1u;
    h[t] = 0;
    uint32_t kv[RS_PER];
#pragma unroll
    for (int r = 0; r < RS_PER; ++r) {
        const int64_t i = (int64_t)b * RS_TILE + r * RS_THREADS + t;
        kv[r] = i < a.n ? a.key[i] : 0xffffffffu;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_PER; ++r) {
        const int64_t i = (int64_t)b * RS_TILE + r * RS_THREADS + t;
        if (i < a.n) atomicAdd(&h[(kv[r] >> a.shift) & dmask], 1);
    }
    __syncthreads();
    if (t <= (int)dmask) a.tab[(int64_t)t * a.nb + b] = h[t];
}
__global__ void __launch_bounds__(RS_THREADS) k_tree_hist(TreeHistArgs a) { tree_hist_body(a, blockIdx.x); }
__global__ void __launch_bounds__(RS_THREADS) k_tree_hist_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_hist_body(static_cast<const TreeHistArgs *>(m.args)[i], bx);
}

// Exclusive scan, in place, of a pass's (digit, block) table by one block:
// each thread takes SC_PER consecutive counts (four 16-byte loads), so a
// table of up to SC_TILE counts costs one round trip.  The first pass's scan
// also moves the build's error flag to err[1], where the host reads it
// (err[0] is cleared for the next build).
constexpr int SC_THREADS = 1024, SC_PER = 16, SC_TILE = SC_THREADS * SC_PER;
struct TreeScanArgs {
    int32_t *tab;  // 16-byte aligned
    int64_t len;
    int32_t *err;  // null after the first pass
};
__device__ __forceinline__ void tree_scan_body(const TreeScanArgs &A)
{
    int32_t *__restrict__ tab = A.tab;
    const int64_t len = A.len;
    __shared__ int32_t wsum[SC_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (A.err && t == 0) {
        A.err[1] = A.err[0];
        A.err[0] = 0;
    }
    int32_t carry = 0;
    for (int64_t t0 = 0; t0 < len; t0 += SC_TILE) {
        const int64_t e0 = t0 + (int64_t)t * SC_PER;
        const bool full = e0 + SC_PER <= len;
        int32_t c[SC_PER];
        if (full) {
#pragma unroll
            for (int k = 0; k < SC_PER / 4; ++k) {
                const int4 v4 = reinterpret_cast<const int4 *>(tab + e0)[k];
                c[4 * k] = v4.x;
                c[4 * k + 1] = v4.y;
                c[4 * k + 2] = v4.z;
                c[4 * k + 3] = v4.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < SC_PER; ++k) c[k] = e0 + k < len ? tab[e0 + k] : 0;
        }
        int32_t s = 0;
#pragma unroll
        for (int k = 0; k < SC_PER; ++k) s += c[k];
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
            const int32_t x = c[k];
            c[k] = run;
            run += x;
        }
        if (full) {
#pragma unroll
            for (int k = 0; k < SC_PER / 4; ++k)
                reinterpret_cast<int4 *>(tab + e0)[k] = make_int4(c[4 * k], c[4 * k + 1], c[4 * k + 2], c[4 * k + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < SC_PER; ++k)
                if (e0 + k < len) tab[e0 + k] = c[k];
        }
        carry += wsum[SC_THREADS / 64 - 1];
        __syncthreads();
    }
}
__global__ void __launch_bounds__(SC_THREADS) k_tree_scan(TreeScanArgs a) { tree_scan_body(a); }
__global__ void __launch_bounds__(SC_THREADS) k_tree_scan_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_scan_body(static_cast<const TreeScanArgs *>(m.args)[i]);
}

// Stable scatter of one pass.  Wave w of block b takes the RS_PER * 64
// consecutive elements from b * RS_TILE + w * 64 * RS_PER, 64 at a time, so
// (wave, round, lane) is the input order.  A lane's rank among the equal
// digits of its round comes from ballots over the digit bits; a per-wave LDS
// counter per digit carries the ranks across rounds; the scanned table and
// the counts of the lower waves give the block's base for each digit.
struct TreeScatterArgs {
    const uint32_t *kin;
    const int32_t *iin;  // null in the first pass: the index is the position
    uint32_t *kout;
    int32_t *iout;
    const int32_t *tab;  // scanned
    int64_t n;
    int nb, shift, bits;
};
__device__ __forceinline__ void tree_scatter_body(const TreeScatterArgs &a, int b)
{
    __shared__ int32_t wc[RS_WAVES][1 << RS_MAXBITS];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t dmask = (1u << a.bits) - 1u;
    for (int k = t; k < RS_WAVES * (1 << RS_MAXBITS); k += RS_THREADS) (&wc[0][0])[k] = 0;
    const int64_t base = (int64_t)b * RS_TILE + (int64_t)w * 64 * RS_PER;
    uint32_t kv[RS_PER];
    int32_t iv[RS_PER];
#pragma unroll
    for (int r = 0; r < RS_PER; ++r) {
        const int64_t pos = base + r * 64 + lane;
        const bool v = pos < a.n;
        kv[r] = v ? a.kin[pos] : 0u;
        iv[r] = v ? (a.iin ? a.iin[pos] : (int32_t)pos) : -1;
    }
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int32_t rk[RS_PER];
#pragma unroll
    for (int r = 0; r < RS_PER; ++r) {
        const bool v = iv[r] >= 0;
        const uint32_t d = (kv[r] >> a.shift) & dmask;
        uint64_t m = __ballot(v);
        for (int bit = 0; bit < a.bits; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bb = __ballot(on);
            m &= on ? bb : ~bb;
        }
        const int before = __popcll(m & below);
        const int old = v ? wc[w][d] : 0;
        if (v && before == 0) wc[w][d] = old + __popcll(m);
        rk[r] = v ? old + before : -1;
    }
    __syncthreads();
    if (t <= (int)dmask) {
        int32_t run = a.tab[(int64_t)t * a.nb + b];
#pragma unroll
        for (int u = 0; u < RS_WAVES; ++u) {
            const int32_t c = wc[u][t];
            wc[u][t] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_PER; ++r) {
        if (rk[r] < 0) continue;
        const int64_t p = (int64_t)wc[w][(kv[r] >> a.shift) & dmask] + rk[r];
        if (p >= 0 && p < a.n) {
            a.kout[p] = kv[r];
            a.iout[p] = iv[r];
        }
    }
}
__global__ void __launch_bounds__(RS_THREADS) k_tree_scatter(TreeScatterArgs a) { tree_scatter_body(a, blockIdx.x); }
__global__ void __launch_bounds__(RS_THREADS) k_tree_scatter_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_scatter_body(static_cast<const TreeScatterArgs *>(m.args)[i], bx);
}

// Last pass, one thread per grouped position j in [0, n]: the leaf ranges
// from the sorted keys (leaves between the keys at j - 1 and j start and end
// at j; a wave fills long runs of empty leaves together), the original index
// and the gathered coordinates and source densities.  Keys out of order (not
// produced by a correct sort) set bit 1 of err[1].
constexpr int GA_THREADS = 256, GA_RUN = 16;
struct TreeGatherArgs {
    const uint32_t *skey;
    const int32_t *perm;
    int64_t nbox;
    int32_t *start, *end, *idx;
    const double *src;
    int64_t ns;
    const double *tgt;
    int64_t nt;
    double *xs, *ys;
    const uint64_t *q;
    uint64_t *qs;
    int nrhs, qw;
    double ty_a, ty_b;  // tree coordinate of a target: ty_a y + ty_b
    int32_t *err;
};
__device__ __forceinline__ void tree_gather_body(const TreeGatherArgs &a, int b)
{
    const int64_t ns = a.ns, nt = a.nt, n = ns + nt;
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)b * GA_THREADS + threadIdx.x;
    const bool act = j <= n;
    const uint32_t last = (uint32_t)(a.nbox - 1);
    int prev = -1, cur = (int)a.nbox;
    if (act && j > 0) prev = (int)min(a.skey[j - 1], last);
    if (act && j < n) cur = (int)min(a.skey[j], last);
    if (prev > cur) {
        atomicOr(a.err + 1, 2);
        cur = prev;
    }
    if (act && cur - prev <= GA_RUN) {
        for (int k = prev + 1; k <= cur && k <= (int)last; ++k) a.start[k] = (int32_t)j;
        for (int k = max(prev, 0); k < cur; ++k) a.end[k] = (int32_t)j;
    }
    uint64_t big = __ballot(act && cur - prev > GA_RUN);
    while (big) {
        const int l = __ffsll((unsigned long long)big) - 1;
        big &= big - 1;
        const int p0 = __shfl(prev, l), c0 = __shfl(cur, l), jj = __shfl((int)j, l);
        for (int k = p0 + 1 + lane; k <= c0 && k <= (int)last; k += 64) a.start[k] = jj;
        for (int k = max(p0, 0) + lane; k < c0; k += 64) a.end[k] = jj;
    }
    if (j >= n) return;
    const int32_t o = a.perm[j];
    if (o < 0 || (int64_t)o >= n) {
        atomicOr(a.err + 1, 2);
        return;
    }
    a.idx[j] = o;
    if (o < ns) {
        a.xs[j] = a.src[o];
        a.ys[j] = a.src[ns + o];
        if (a.q && j < ns)
            for (int r = 0; r < a.nrhs; ++r)
                for (int w = 0; w < a.qw; ++w)
                    a.qs[((int64_t)r * ns + j) * a.qw + w] = a.q[((int64_t)r * ns + o) * a.qw + w];
    } else {
        a.xs[j] = a.tgt[o - ns];
        a.ys[j] = fma(a.ty_a, a.tgt[nt + o - ns], a.ty_b);
    }
}
__global__ void __launch_bounds__(GA_THREADS) k_tree_gather(TreeGatherArgs a) { tree_gather_body(a, blockIdx.x); }
__global__ void __launch_bounds__(GA_THREADS) k_tree_gather_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_gather_body(static_cast<const TreeGatherArgs *>(m.args)[i], bx);
}

// The counting-sort form of the grouping, for small trees, where the
// radix passes cost more than they save: per-leaf counts by atomics (whose
// old values are the points' slots in arrival order), one exclusive scan for
// the leaf ranges, a scatter to the slots, and a per-leaf sort of the
// scattered original indices, so that every leaf again lists its points in
// increasing original index.
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

// Exclusive scan of the leaf counts by one block, in LDS tiles of CS_TILE
// counts (loaded and stored coalesced): start[b], end[b].  The counters are
// cleared for the next build, and the error flag of this build is moved to
// err[1], where the host reads it (err[0] is cleared).  Counts that do not add
// up to the number of points (counters not zero at the start) leave every
// leaf empty and set bit 1 of err[1], so that no later kernel indexes with
// them.
constexpr int CS_THREADS = 1024, CS_PER = 8, CS_TILE = CS_THREADS * CS_PER;
struct TreeRangeArgs {
    int32_t *cnt;
    int64_t nbox, n;
    int32_t *start, *end, *err;
};
__device__ __forceinline__ void tree_range_body(const TreeRangeArgs &A)
{
    int32_t *__restrict__ cnt = A.cnt;
    int32_t *__restrict__ start = A.start;
    int32_t *__restrict__ end = A.end;
    int32_t *__restrict__ err = A.err;
    const int64_t nbox = A.nbox, n = A.n;
    __shared__ int32_t tile[CS_TILE];
    __shared__ int32_t wsum[CS_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) {
        err[1] = err[0];
        err[0] = 0;
    }
    int32_t carry = 0;
    for (int64_t t0 = 0; t0 < nbox; t0 += CS_TILE) {
#pragma unroll
        for (int k = 0; k < CS_PER; ++k) {
            int64_t b = t0 + k * CS_THREADS + t;
            tile[k * CS_THREADS + t] = b < nbox ? cnt[b] : 0;
        }
        __syncthreads();
        int32_t c[CS_PER], s = 0;
#pragma unroll
        for (int k = 0; k < CS_PER; ++k) {
            c[k] = tile[t * CS_PER + k];
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
            int32_t w = lane < CS_THREADS / 64 ? wsum[lane] : 0;
            for (int o = 1; o < CS_THREADS / 64; o <<= 1) {
                int32_t u = __shfl_up(w, o);
                if (lane >= o) w += u;
            }
            if (lane < CS_THREADS / 64) wsum[lane] = w;
        }
        __syncthreads();
        int32_t run = carry + v - s + (wv > 0 ? wsum[wv - 1] : 0);
#pragma unroll
        for (int k = 0; k < CS_PER; ++k) {
            tile[t * CS_PER + k] = run;
            run += c[k];
        }
        carry += wsum[CS_THREADS / 64 - 1];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CS_PER; ++k) {
            int64_t b = t0 + k * CS_THREADS + t;
            if (b < nbox) {
                int32_t st = tile[k * CS_THREADS + t];
                int32_t n_b = cnt[b];
                start[b] = st;
                end[b] = st + n_b;
                cnt[b] = 0;
            }
        }
        __syncthreads();
    }
    if ((int64_t)carry != n) {
        for (int64_t b = t; b < nbox; b += CS_THREADS) {
            start[b] = 0;
            end[b] = 0;
        }
        if (t == 0) err[1] |= 2;
    }
}

__global__ void __launch_bounds__(CS_THREADS) k_tree_ranges(TreeRangeArgs a) { tree_range_body(a); }
__global__ void __launch_bounds__(CS_THREADS) k_tree_ranges_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_range_body(static_cast<const TreeRangeArgs *>(m.args)[i]);
}

struct TreeSlotArgs {
    const uint32_t *key;
    const int32_t *rank;
    int64_t n;
    const int32_t *start;
    int32_t *perm;
};
__device__ __forceinline__ void tree_slot_body(const TreeSlotArgs &a, int bx)
{
    int64_t i = (int64_t)bx * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int64_t pos = (int64_t)a.start[a.key[i]] + a.rank[i];
    if (pos >= 0 && pos < a.n) a.perm[pos] = (int32_t)i;
}
__global__ void __launch_bounds__(256) k_tree_slots(TreeSlotArgs a) { tree_slot_body(a, blockIdx.x); }
__global__ void __launch_bounds__(256) k_tree_slots_multi(MultiArgs m)
{
    int i, bx, by, bz;
    multi_locate(m, i, bx, by, bz);
    tree_slot_body(static_cast<const TreeSlotArgs *>(m.args)[i], bx);
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

int tree_sort_bits(int64_t nbox, int &passes)
{
    int b = 0;
    while (b < 32 && ((int64_t)1 << b) < nbox) ++b;
    passes = b <= RS_MAXBITS ? 1 : (b + RS_MAXBITS - 1) / RS_MAXBITS;
    return (b + passes - 1) / passes;
}

bool tree_radix(int64_t n, int form)
{
    const int64_t all = launch_batch_all_points() > 0 ? launch_batch_all_points() : n;
    return form < 0 ? all >= TREE_RADIX_MIN_POINTS : form != 0;
}

int tree_launch_count(int64_t nbox, bool radix)
{
    if (!radix) return 4;
    int passes;
    tree_sort_bits(nbox, passes);
    return 3 * passes + 1;
}

int64_t tree_table_len(int64_t n) { return (n + RS_TILE - 1) / RS_TILE * ((int64_t)1 << RS_MAXBITS); }

void launch_tree(const double *src, int64_t ns, const double *tgt, int64_t nt, double x_lo, double w, int col_lo,
                 int ncol, int rows_s, int rows_t, const Layers &ly, const TreeBufs &b, int32_t *err, bool radix,
                 hipStream_t st)
{
    const int64_t n = ns + nt;
    const int64_t nbox = (int64_t)(rows_s + rows_t) * ncol;
    if (n == 0 || nbox == 0) return;
    if (!radix) {
        const TreeCountArgs ca{src,  ns,     tgt,    nt, x_lo,  1.0 / w, col_lo, ncol,
                               rows_s, rows_t, ly, b.key, b.rank, b.cnt,  err};
        emit((const void *)k_tree_count, (const void *)k_tree_count_multi, 0,
             dim3((unsigned)((n + TC_THREADS - 1) / TC_THREADS)), dim3(TC_THREADS), 0, st, ca);
        const TreeRangeArgs ra{b.cnt, nbox, n, b.start, b.end, err};
        emit((const void *)k_tree_ranges, (const void *)k_tree_ranges_multi, 1, dim3(1), dim3(CS_THREADS), 0, st, ra);
        const TreeSlotArgs xa{b.key, b.rank, n, b.start, b.perm};
        emit((const void *)k_tree_slots, (const void *)k_tree_slots_multi, 2, dim3((unsigned)((n + 255) / 256)),
             dim3(256), 0, st, xa);
        const TreeLeafArgs la{b.start, b.end, b.perm, b.scratch, b.idx, src,  ns,     tgt,   nt,
                              b.xs,    b.ys,  b.q,    b.qs,      b.nrhs, b.qw, ly.ty_a, ly.ty_b};
        emit((const void *)k_tree_leaf, (const void *)k_tree_leaf_multi, 3, dim3((unsigned)nbox), dim3(64), 0, st,
             la);
        return;
    }
    int passes;
    const int bits = tree_sort_bits(nbox, passes);
    const int nb = (int)((n + RS_TILE - 1) / RS_TILE);
    const int64_t tlen = (int64_t)nb << bits;
    // ping-pong buffers: (key, rank) and the two halves of scratch
    uint32_t *kA = b.key, *kB = reinterpret_cast<uint32_t *>(b.scratch);
    int32_t *iA = b.rank, *iB = b.scratch + n;
    const TreeKeyArgs ka{src,   ns,   tgt,     nt,  x_lo, 1.0 / w, col_lo, ncol, rows_s, rows_t, ly,
                         kA,    b.tab, b.start, b.end, nbox, nb,     bits,   err};
    emit((const void *)k_tree_key, (const void *)k_tree_key_multi, 0, dim3(nb), dim3(RS_THREADS), 0, st, ka);
    for (int p = 0; p < passes; ++p) {
        const bool fwd = (p & 1) == 0;  // A -> B on even passes
        const uint32_t *kin = fwd ? kA : kB;
        const int32_t *iin = p == 0 ? nullptr : (fwd ? iA : iB);
        uint32_t *kout = fwd ? kB : kA;
        int32_t *iout = fwd ? iB : iA;
        if (p > 0) {
            const TreeHistArgs ha{kin, n, b.tab, nb, p * bits, bits};
            emit((const void *)k_tree_hist, (const void *)k_tree_hist_multi, 3 * p, dim3(nb), dim3(RS_THREADS), 0, st,
                 ha);
        }
        const TreeScanArgs sa{b.tab, tlen, p == 0 ? err : nullptr};
        emit((const void *)k_tree_scan, (const void *)k_tree_scan_multi, 3 * p + 1, dim3(1), dim3(SC_THREADS), 0, st,
             sa);
        const TreeScatterArgs xa{kin, iin, kout, iout, b.tab, n, nb, p * bits, bits};
        emit((const void *)k_tree_scatter, (const void *)k_tree_scatter_multi, 3 * p + 2, dim3(nb), dim3(RS_THREADS),
             0, st, xa);
    }
    const bool inB = (passes & 1) != 0;
    const TreeGatherArgs ga{inB ? kB : kA, inB ? iB : iA, nbox, b.start, b.end, b.idx, src, ns, tgt, nt, b.xs, b.ys,
                            b.q, b.qs, b.nrhs, b.qw, ly.ty_a, ly.ty_b, err};
    emit((const void *)k_tree_gather, (const void *)k_tree_gather_multi, 12,
         dim3((unsigned)((n + GA_THREADS) / GA_THREADS)), dim3(GA_THREADS), 0, st, ga);
}

}  // namespace lmfmm
