// Quadtree construction (Algorithm 1, Step 1): bounding box and layer checks,
// leaf keys, a stable LSD radix sort of the keys, and leaf ranges.
//
// The tree is uniform with its root square split at the interface y = 0, so
// every box holds either sources (above) or targets (below).  A leaf key is
// (row, column) of the level-L box; target keys follow all source keys, so one
// sort orders both point sets and the sorted array holds sources first.
#include "lmfmm_internal.h"

namespace lmfmm {

namespace {

constexpr int BB_THREADS = 256;
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

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
// target y min/max; count of points outside their layer or not finite.
__global__ void __launch_bounds__(BB_THREADS) k_bbox_partial(const double *__restrict__ src, int64_t ns,
                                                             const double *__restrict__ tgt, int64_t nt,
                                                             double ys_lim, double yt_lim, double *partial,
                                                             unsigned *counter, double *out, uint64_t seq)
{
    double v[7] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += stride) {
        double x = src[i], y = src[ns + i];
        bool ok = isfinite(x) && isfinite(y) && y > 0.0 && y < ys_lim;
        if (ok) {
            v[0] = fmin(v[0], x);
            v[1] = fmax(v[1], x);
            v[2] = fmin(v[2], y);
            v[3] = fmax(v[3], y);
        } else {
            v[6] += 1.0;
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += stride) {
        double x = tgt[i], y = tgt[nt + i];
        bool ok = isfinite(x) && isfinite(y) && y < 0.0 && y > yt_lim;
        if (ok) {
            v[0] = fmin(v[0], x);
            v[1] = fmax(v[1], x);
            v[4] = fmin(v[4], y);
            v[5] = fmax(v[5], y);
        } else {
            v[6] += 1.0;
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
    __shared__ int last;
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
        for (int j = 0; j < 7; ++j)
            __hip_atomic_store(&partial[blockIdx.x * 8 + j], r[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = t == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x >= 64) return;
    // the last block to finish: reduce the partials of all blocks
    double v2[7] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    for (int b = threadIdx.x; b < (int)gridDim.x; b += 64) {
        double q[7];
        for (int j = 0; j < 7; ++j) q[j] = __hip_atomic_load(&partial[b * 8 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
        // result, then its sequence number, in host-visible memory; rearm the counter
        for (int j = 0; j < 7; ++j) __hip_atomic_store(&out[j], v2[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(reinterpret_cast<uint64_t *>(out + 8), seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}


// Leaf key of every point.  Sources (y > 0) take row floor(y/w) above the
// interface, targets row floor(-y/w) below it; columns are relative to
// col_lo.  Out-of-range rows/columns (points outside a fixed domain) and
// points in the wrong layer raise the error flag and are clamped.
__global__ void __launch_bounds__(256) k_keys(const double *__restrict__ src, int64_t ns,
                                              const double *__restrict__ tgt, int64_t nt, double x_lo, double invw,
                                              int col_lo, int ncol, int rows_s, int rows_t, double ys_lim,
                                              double yt_lim, uint32_t *__restrict__ key,
                                              int32_t *__restrict__ idx, int32_t *__restrict__ err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns + nt) return;
    bool tg = i >= ns;
    double x = tg ? tgt[i - ns] : src[i];
    double y = tg ? tgt[nt + i - ns] : src[ns + i];
    bool bad = !(isfinite(x) && isfinite(y)) || (tg ? !(y < 0.0 && y > yt_lim) : !(y > 0.0 && y < ys_lim));
    double fc = floor((x - x_lo) * invw) - (double)col_lo;
    double fr = floor((tg ? -y : y) * invw);
    int rows = tg ? rows_t : rows_s;
    if (!(fc >= 0.0 && fc < (double)ncol && fr >= 0.0 && fr < (double)rows)) bad = true;
    int c = (int)fmin(fmax(fc, 0.0), (double)(ncol - 1));
    int r = (int)fmin(fmax(fr, 0.0), (double)(rows - 1));
    if (bad) atomicOr(err, 1);
    uint32_t k = (uint32_t)r * (uint32_t)ncol + (uint32_t)c;
    if (tg) k += (uint32_t)rows_s * (uint32_t)ncol;
    key[i] = k;
    idx[i] = (int32_t)i;
}

// Radix sort pass, step 1: per-tile digit histogram, stored digit-major.
__global__ void __launch_bounds__(RS_THREADS) k_rs_upsweep(const uint32_t *__restrict__ key, int64_t n, int shift,
                                                           uint32_t *__restrict__ hist, int nblk)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int j = threadIdx.x; j < RS_TILE; j += RS_THREADS) {
        int64_t g = base + j;
        if (g < n) atomicAdd(&cnt[(key[g] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)blockIdx.x * 256 + threadIdx.x] = cnt[threadIdx.x];
}

// Step 2: exclusive scan in digit-major order of the block-major histogram
// hist[block][digit] (one block; thread d owns digit d, loads are coalesced
// across threads).
__global__ void __launch_bounds__(256) k_rs_scan(uint32_t *__restrict__ hist, int nblk)
{
    __shared__ uint32_t tot[256];
    const int d = threadIdx.x;
    uint32_t s = 0;
#pragma unroll 8
    for (int b = 0; b < nblk; ++b) s += hist[(int64_t)b * 256 + d];
    tot[d] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t v = d >= o ? tot[d - o] : 0u;
        __syncthreads();
        tot[d] += v;
        __syncthreads();
    }
    uint32_t run = tot[d] - s;
#pragma unroll 8
    for (int b = 0; b < nblk; ++b) {
        uint32_t c = hist[(int64_t)b * 256 + d];
        hist[(int64_t)b * 256 + d] = run;
        run += c;
    }
}

// Step 3: stable scatter.  Each tile is processed in rounds of 256 elements in
// index order; within a round an element's rank among equal digits comes from
// wave ballots over the 8 digit bits plus the counts of earlier waves.
__global__ void __launch_bounds__(RS_THREADS) k_rs_downsweep(const uint32_t *__restrict__ kin,
                                                             const int32_t *__restrict__ iin,
                                                             uint32_t *__restrict__ kout, int32_t *__restrict__ iout,
                                                             int64_t n, int shift, const uint32_t *__restrict__ hist,
                                                             int nblk)
{
    constexpr int NW = RS_THREADS / 64;
    __shared__ uint32_t offs[256];
    __shared__ uint32_t wcnt[NW][256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    offs[tid] = hist[(int64_t)blockIdx.x * 256 + tid];
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t g = base + (int64_t)r * RS_THREADS + tid;
        bool act = g < n;
        uint32_t k = act ? kin[g] : 0u;
        uint32_t dg = (k >> shift) & 255u;
        for (int w = 0; w < NW; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        uint64_t m = __ballot(act);
        for (int b = 0; b < 8; ++b) {
            bool bit = (dg >> b) & 1u;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(m & lt);
        if (act && rank == 0) wcnt[wv][dg] = (uint32_t)__popcll(m);
        __syncthreads();
        {
            uint32_t acc = offs[tid];
            for (int w = 0; w < NW; ++w) {
                uint32_t c = wcnt[w][tid];
                wcnt[w][tid] = acc;
                acc += c;
            }
            offs[tid] = acc;
        }
        __syncthreads();
        if (act) {
            uint32_t pos = wcnt[wv][dg] + rank;
            kout[pos] = k;
            iout[pos] = iin[g];
        }
        __syncthreads();
    }
}

__global__ void k_zero_u32(uint32_t *__restrict__ p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Leaf ranges [start, end) per key and the sorted coordinates.
__global__ void __launch_bounds__(256) k_leaf_ranges(const uint32_t *__restrict__ key,
                                                     const int32_t *__restrict__ idx, int64_t n,
                                                     int32_t *__restrict__ start, int32_t *__restrict__ end,
                                                     const double *__restrict__ src, int64_t ns,
                                                     const double *__restrict__ tgt, int64_t nt,
                                                     double *__restrict__ xs, double *__restrict__ ys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t k = key[i];
    if (i == 0 || key[i - 1] != k) start[k] = (int32_t)i;
    if (i == n - 1 || key[i + 1] != k) end[k] = (int32_t)(i + 1);
    int64_t o = idx[i];
    if (o < ns) {
        xs[i] = src[o];
        ys[i] = src[ns + o];
    } else {
        xs[i] = tgt[o - ns];
        ys[i] = tgt[nt + o - ns];
    }
}

}  // namespace

int bbox_blocks(int64_t n)
{
    int64_t b = (n + 1023) / 1024;
    if (b < 1) b = 1;
    if (b > 512) b = 512;
    return (int)b;
}

void launch_bbox(const double *src, int64_t ns, const double *tgt, int64_t nt, double ys_lim, double yt_lim,
                 double *partial, unsigned *counter, int nblk, double *out, uint64_t seq, hipStream_t st)
{
    hipLaunchKernelGGL(k_bbox_partial, dim3(nblk), dim3(BB_THREADS), 0, st, src, ns, tgt, nt, ys_lim, yt_lim,
                       partial, counter, out, seq);
}

void launch_keys(const double *src, int64_t ns, const double *tgt, int64_t nt, double x_lo, double w, int col_lo,
                 int ncol, int rows_s, int rows_t, double ys_lim, double yt_lim, uint32_t *key, int32_t *idx,
                 int32_t *err, hipStream_t st)
{
    int64_t n = ns + nt;
    if (n == 0) return;
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, ns, tgt, nt, x_lo, 1.0 / w,
                       col_lo, ncol, rows_s, rows_t, ys_lim, yt_lim, key, idx, err);
}

__global__ void k_mirror(const double *__restrict__ xy, int64_t n, double *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        out[i] = xy[i];
        out[n + i] = -xy[n + i];
    }
}

void launch_mirror(const double *xy, int64_t n, double *out, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mirror, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xy, n, out);
}

int sort_blocks(int64_t n) { return (int)((n + RS_TILE - 1) / RS_TILE); }

int launch_radix_sort(SortBufs &b, int64_t n, int bits, hipStream_t st)
{
    int passes = (bits + 7) / 8;
    int nblk = sort_blocks(n);
    uint32_t *kin = b.key_a, *kout = b.key_b;
    int32_t *iin = b.idx_a, *iout = b.idx_b;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_upsweep, dim3(nblk), dim3(RS_THREADS), 0, st, kin, n, shift, b.hist, nblk);
        hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(256), 0, st, b.hist, nblk);
        hipLaunchKernelGGL(k_rs_downsweep, dim3(nblk), dim3(RS_THREADS), 0, st, kin, iin, kout, iout, n, shift,
                           b.hist, nblk);
        uint32_t *tk = kin;
        kin = kout;
        kout = tk;
        int32_t *ti = iin;
        iin = iout;
        iout = ti;
    }
    return (passes & 1) ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_zero3(int32_t *__restrict__ a, int64_t na, int32_t *__restrict__ b,
                                               int64_t nb, int32_t *__restrict__ c, int64_t nc)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < na)
        a[i] = 0;
    else if (i < na + nb)
        b[i - na] = 0;
    else if (i < na + nb + nc)
        c[i - na - nb] = 0;
}

void launch_zero3(int32_t *a, int64_t na, int32_t *b, int64_t nb, int32_t *c, int64_t nc, hipStream_t st)
{
    int64_t n = na + nb + nc;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, na, b, nb, c, nc);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

void launch_zero_bytes(void *p, size_t nbytes, hipStream_t st)
{
    int64_t n = (int64_t)(nbytes / 4);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t *)p, n);
}

void launch_leaf_ranges(const uint32_t *key, const int32_t *idx, int64_t n, int64_t nbox, int32_t *start,
                        int32_t *end, const double *src, int64_t ns, const double *tgt, int64_t nt, double *xs,
                        double *ys, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_leaf_ranges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, key, idx, n, start, end,
                       src, ns, tgt, nt, xs, ys);
}

}  // namespace lmfmm
