// Internal declarations of the MI355X layered-media FMM library.
//
// Shared by the host plan code and the HIP kernels: a small complex type,
// the principal-branch square root, sigma_2^t, the scaled Bessel bases of the
// multipole and local expansions, and the launch wrappers of every kernel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>
#include <vector>

namespace lmfmm {

// Start/stop events for the next timed kernel launch of this host thread
// (set by a plan in timing mode, consumed by LMFMM_LAUNCH): the runtime
// stamps them at the kernel's own start and end.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
inline LaunchTiming &launch_timing()
{
    static thread_local LaunchTiming t;
    return t;
}

#define LMFMM_LAUNCH(K, grid, block, sh, st, ...)                                    \
    do {                                                                             \
        ::lmfmm::LaunchTiming &lt_ = ::lmfmm::launch_timing();                       \
        if (lt_.start) {                                                             \
            hipEvent_t a_ = lt_.start, b_ = lt_.stop;                                \
            lt_.start = lt_.stop = nullptr;                                          \
            hipExtLaunchKernelGGL(K, grid, block, sh, st, a_, b_, 0, __VA_ARGS__);   \
        } else {                                                                     \
            hipLaunchKernelGGL(K, grid, block, sh, st, __VA_ARGS__);                 \
        }                                                                            \
    } while (0)


// ---------------------------------------------------------------------------
// Launches through a recorder.
//
// Every kernel of the apply takes one argument struct by value.  Its launch
// wrapper calls emit(), which launches the kernel at once (with the start and
// stop events of launch_timing, if set) or, while a recorder is set for this
// host thread, appends the launch to it.  The batched apply records every
// instance's launch sequence and merges the launches of one stage into one
// launch of the kernel's multi-instance form (MultiArgs below).
// ---------------------------------------------------------------------------
enum Stage { S_ZERO = 1, S_TREE, S_P2M, S_M2M, S_ZTOP, S_M2L, S_L2L, S_SWEEP, S_L2P };

struct RecLaunch {
    int key;             // launch_stage() + sub: position in the merged launch sequence
    const void *single;  // the kernel, taking the argument struct by value
    const void *multi;   // its multi-instance form (one MultiArgs argument), or null
    dim3 grid, block;
    size_t shmem;
    size_t align;             // alignment of the argument struct
    std::vector<char> args;  // the argument struct's bytes
    double cost = 0;         // estimated work per block (merged launches start the costliest instances first)
};
struct Recorder {
    std::vector<RecLaunch> v;
};
// Estimated work per block of the next recorded launches (0: none).
inline double &launch_cost()
{
    static thread_local double c = 0;
    return c;
}
inline Recorder *&launch_recorder()
{
    static thread_local Recorder *r = nullptr;
    return r;
}
// key of the launches that follow: stage * 64 + j, j the launch's index among
// the instance's launches of that stage (the level of a per-level pass); a
// launcher issuing several kernels adds 0, 1, ... to it
inline int &launch_stage()
{
    static thread_local int s = 0;
    return s;
}
inline void set_stage(Stage s, int j = 0) { launch_stage() = (int)s * 64 + j; }
// While a batch is recorded: the sources of all its instances.  A launcher
// that sizes its blocks' LDS for occupancy sizes them for this many points
// (a merged launch runs with the largest LDS size of its instances).
inline int64_t &launch_batch_points()
{
    static thread_local int64_t n = 0;
    return n;
}
// While a batch is recorded: the sources and targets of all its instances.
inline int64_t &launch_batch_all_points()
{
    static thread_local int64_t n = 0;
    return n;
}

// Argument of a multi-instance launch: instance i takes the blocks
// [blk0[i], blk0[i + 1]) of the flat grid, its own grid is grid[3i .. 3i + 2]
// (x, y, z), and its argument struct is element i of args.
struct MultiArgs {
    const int *blk0;
    const int *grid;
    const void *args;
    int n;
};

template <class A>
inline void emit(const void *single, const void *multi, int sub, dim3 grid, dim3 block, size_t sh, hipStream_t st,
                 const A &a)
{
    static_assert(std::is_trivially_copyable<A>::value, "kernel arguments are copied as bytes");
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return;
    if (Recorder *r = launch_recorder()) {
        RecLaunch L;
        L.key = launch_stage() + sub;
        L.single = single;
        L.multi = multi;
        L.grid = grid;
        L.block = block;
        L.shmem = sh;
        L.align = alignof(A);
        L.cost = launch_cost();
        L.args.assign(reinterpret_cast<const char *>(&a), reinterpret_cast<const char *>(&a) + sizeof(A));
        r->v.push_back(std::move(L));
        return;
    }
    void *args[] = {const_cast<A *>(&a)};
    LaunchTiming &lt = launch_timing();
    if (lt.start) {
        hipEvent_t a_ = lt.start, b_ = lt.stop;
        lt.start = lt.stop = nullptr;
        (void)hipExtLaunchKernel(single, grid, block, args, sh, st, a_, b_, 0);
    } else {
        (void)hipLaunchKernel(single, grid, block, args, sh, st);
    }
}

// Block of a multi-instance launch: its instance and its block index in the
// instance's own grid.
__device__ inline void multi_locate(const MultiArgs &m, int &i, int &bx, int &by, int &bz)
{
    const int b = blockIdx.x;
    int lo = 0, hi = m.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m.blk0[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    i = lo;
    const int loc = b - m.blk0[lo], gx = m.grid[3 * lo], gy = m.grid[3 * lo + 1];
    bx = loc % gx;
    by = (loc / gx) % gy;
    bz = loc / (gx * gy);
}

// ---------------------------------------------------------------------------
// Complex arithmetic (device and host)
// ---------------------------------------------------------------------------
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ inline cx<T> operator*(cx<T> a, T s) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ inline cx<T> &operator+=(cx<T> &a, cx<T> b)
{
    a.re += b.re;
    a.im += b.im;
    return a;
}
// a += b * c
template <typename T>
__host__ __device__ inline void cfma(cx<T> &a, cx<T> b, cx<T> c)
{
    a.re = fma(b.re, c.re, fma(-b.im, c.im, a.re));
    a.im = fma(b.re, c.im, fma(b.im, c.re, a.im));
}
// Compensated complex accumulator (Kahan summation): in FP32 the rounding
// error of each addition is kept in c and taken off the next addend, so the
// error of a long sum does not grow with the number of terms; FP64 adds
// plainly.
template <typename T>
struct CAcc {
    cx<T> s, c;
    __host__ __device__ void zero()
    {
        s = {T(0), T(0)};
        c = {T(0), T(0)};
    }
    __host__ __device__ void add(cx<T> x)
    {
        if (sizeof(T) == 8) {
            s.re += x.re;
            s.im += x.im;
            return;
        }
        const T yr = x.re - c.re, yi = x.im - c.im;
        const T tr = s.re + yr, ti = s.im + yi;
        c.re = (tr - s.re) - yr;
        c.im = (ti - s.im) - yi;
        s.re = tr;
        s.im = ti;
    }
    __host__ __device__ cx<T> value() const { return {s.re - c.re, s.im - c.im}; }
};

template <typename T>
__host__ __device__ inline cx<T> cinv(cx<T> a)
{
    T s = T(1) / (a.re * a.re + a.im * a.im);
    return {a.re * s, -a.im * s};
}
// FP32 on the device: the hardware reciprocal of |a|^2 refined by one Newton
// step, within about one unit in the last place of the division, in far fewer
// instructions than the IEEE division sequence.
__device__ inline cx<float> cinv(cx<float> a)
{
    const float d = a.re * a.re + a.im * a.im;
    const float r = __builtin_amdgcn_rcpf(d);
    const float s = fmaf(fmaf(-d, r, 1.0f), r, r);
    return {a.re * s, -a.im * s};
}
// FP64: on the device the hardware reciprocal refined by two Newton steps
// (each about doubles the correct bits), without the IEEE division's scaling
// and fix-up steps (|a|^2 here stays far from the overflow and underflow
// thresholds); on the host the division.
__host__ __device__ inline cx<double> cinv(cx<double> a)
{
    const double d = a.re * a.re + a.im * a.im;
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
#else
    const double r = 1.0 / d;
#endif
    return {a.re * r, -a.im * r};
}
template <typename T>
__host__ __device__ inline cx<T> cdiv(cx<T> a, cx<T> b) { return a * cinv(b); }
template <typename T>
__host__ __device__ inline T cabs2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// exp(z) in FP64
__host__ __device__ inline cx<double> cexp_d(cx<double> z)
{
    double e = exp(z.re), s, c;
    sincos(z.im, &s, &c);
    return {e * c, e * s};
}

// Principal square root: branch cut on the negative real axis, Re >= 0.
__host__ __device__ inline cx<double> csqrt_d(cx<double> z)
{
    double r = hypot(z.re, z.im);
    if (r == 0.0) return {0.0, 0.0};
    if (z.re >= 0.0) {
        double t = sqrt(0.5 * (r + z.re));
        return {t, z.im / (2.0 * t)};
    }
    double t = sqrt(0.5 * (r - z.re));
    return {fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// s_m(lam) = sqrt(lam^2 - k^2), principal branch.
__host__ __device__ inline cx<double> sroot_d(cx<double> lam, cx<double> k) { return csqrt_d(lam * lam - k * k); }

// Field components (Section 3): the part of the scattered field applied,
// with its target factor and density.  In the tree's coordinates every one is
// the same kind of integral,
//   Int e^{s_t y'} e^{-s_s y0} e^{i lam (x - x0)} sigma(lam) / (4 pi s_t) d lam,
// with the target's image coordinate y' = a y + b:
//   COMP_2T  g_2^t (Example 4, middle layer):  y' = y,        s_t = s2
//   COMP_2B  g_2^b (middle layer):             y' = -y - 2d,  s_t = s2
//   COMP_1S  g_1^s (top layer):                y' = -y,       s_t = s1
//   COMP_3S  g_3^s (bottom layer):             y' = y,        s_t = s3
//   COMP_IMP the impedance half-space (Example 3, wave number k1, impedance
//            alpha; source and target above y = 0): y' = -y,  s_t = s_s = s1.
// The source factor is e^{-s1 y0} in every case.
enum { COMP_2T = 0, COMP_2B = 1, COMP_1S = 2, COMP_3S = 3, COMP_IMP = 4 };

// The medium and the orientation of the operator.  adj = 0: the forward
// operator (sources in the top layer carry k1, targets the component's wave
// number).  adj = 1: the transposed operator in mirrored coordinates (x, -y'):
// substituting lam -> -lam in the Sommerfeld integral shows that G^T acting
// on target densities is the same kind of operator with the roles of the
// source and target sides exchanged and the same density sigma / (4 pi s_t).
struct Medium {
    cx<double> k1, k2, k3;
    double d;
    int adj;
    int comp = COMP_2T;
    double alpha = 0.0;  // impedance (COMP_IMP)
};
// the physical target's wave number
__host__ __device__ inline cx<double> k_target_layer(const Medium &m)
{
    return (m.comp == COMP_1S || m.comp == COMP_IMP) ? m.k1 : (m.comp == COMP_3S ? m.k3 : m.k2);
}
// wave number of the multipole (source) side and of the local (target) side
__host__ __device__ inline cx<double> k_src(const Medium &m) { return m.adj ? k_target_layer(m) : m.k1; }
__host__ __device__ inline cx<double> k_tgt(const Medium &m) { return m.adj ? m.k1 : k_target_layer(m); }

// The densities of Section 3 Example 4 from the paper's closed forms, with
// numerator and denominator divided by exp(d s2) so that every factor stays
// bounded (Re s2 >= 0); the common denominator is that of sigma_2^t:
//   sigma_2^t = e^{d s2} (lam^2 + s2 s3 - k2^2) / D,
//   sigma_2^b = -e^{d s2} (-lam^2 + s2 s3 + k2^2) / D,
//   sigma_1   = [sinh(d s2)(-lam^2 + s1 s3 + k2^2) + s2 (s1 - s3) cosh(d s2)] / D,
//   sigma_3   = 2 s2 s3 e^{d s3} / D,
//   D = sinh(d s2)(lam^2 + s1 s3 - k2^2) + s2 (s1 + s3) cosh(d s2);
// and the image term of Example 3, (s + i k alpha) / (s - i k alpha).
__host__ __device__ inline cx<double> sigma_d(cx<double> lam, const Medium &m, cx<double> s1)
{
    const cx<double> one = mk(1.0, 0.0);
    if (m.comp == COMP_IMP) {
        const cx<double> ika = mk(-m.k1.im * m.alpha, m.k1.re * m.alpha);
        return cdiv(s1 + ika, s1 - ika);
    }
    const cx<double> s2 = sroot_d(lam, m.k2), s3 = sroot_d(lam, m.k3);
    const cx<double> e = cexp_d(mk(-2.0 * m.d * s2.re, -2.0 * m.d * s2.im));
    const cx<double> l2 = lam * lam, kk = m.k2 * m.k2;
    const cx<double> den = 0.5 * ((one - e) * (l2 + s1 * s3 - kk)) + 0.5 * (s2 * (s1 + s3) * (one + e));
    switch (m.comp) {
    case COMP_2B: return cdiv(-(s2 * s3 + kk - l2), den);
    case COMP_1S: return cdiv(0.5 * ((one - e) * (s1 * s3 + kk - l2)) + 0.5 * (s2 * (s1 - s3) * (one + e)), den);
    case COMP_3S: {
        const cx<double> g = s3 - s2;
        return cdiv(2.0 * (s2 * s3) * cexp_d(mk(m.d * g.re, m.d * g.im)), den);
    }
    default: return cdiv(l2 + s2 * s3 - kk, den);
    }
}

// The layers in the tree's coordinates: sources need ys_lo < y < ys_hi; a
// target's tree coordinate is ty_a y + ty_b (the component's image map) and
// needs yt_lo < . < yt_hi.
struct Layers {
    double ys_lo, ys_hi, yt_lo, yt_hi, ty_a, ty_b;
};

// ---------------------------------------------------------------------------
// Scaled Bessel bases of the expansions.
//
// Multipole basis (sign = -1) at offset (X, Y) from the box centre, wave
// number k, scale radius R:   B_q = s_q J_q(k r) e^{-i q theta},
// local basis (sign = +1):    B_p = s_p J_p(k r) e^{+i p theta},
// with s_q = |q|! (2/(kR))^|q| so that |B_q| <= ~(r/R)^|q| at low frequency.
// J_{-q} = (-1)^q J_q.  Computed by Miller's backward recurrence on the ratios
// t_m = J_m / (z J_{m-1}) = 1/(2m - z^2 t_{m+1}), z = k r, which needs only
// z^2 = k^2 (X^2 + Y^2) (no square root or angle), and the normalisation
// 1 = J_0 + 2 sum_m J_{2m}.  Then J_q e^{i sign q theta} s_q / (J_{q-1} ...) =
// 2 q t_q (X + i sign Y) / R.
// ---------------------------------------------------------------------------
// Loops over the orders are unrolled up to order 64 (their arrays then stay
// in registers); the largest-order variants keep the loops.
template <int PMAX>
struct PUnroll {
    static constexpr int n = PMAX <= 64 ? PMAX : 1;
};

// Start of the backward recurrence: starting at N with t_{N+1} = 0 perturbs
// t_m by about prod_{j=m+1}^{N} |z|^2 / (4 j^2); take N so that this is below
// the working precision at m = P.
template <typename T>
__host__ __device__ inline int miller_start(cx<T> z2, int P)
{
    const T a2 = sqrt(cabs2(z2)) * T(0.25);
    const T eps = sizeof(T) == 8 ? T(1e-17) : T(1e-8);
    int N = P;
    T prod = T(1);
    while (N < P + 200 && (prod > eps || T(N * N) < a2)) {
        ++N;
        T f = a2 / T(N * N);
        prod *= f < T(1) ? f : T(1);
    }
    return N;
}
// One step m of the recurrence: t <- t_m, and U = 2 sum_{even j >= max(m,2)}
// J_j / J_m updated at every odd m: U_{m-1} = 2 [m-1 >= 2] + U_{m+1} z^2
// t_{m+1} t_m.  J_0 = 1 / (1 + U) after the step m = 1.
template <typename T>
__host__ __device__ inline void miller_step(cx<T> z2, int m, cx<T> &t, cx<T> &tprev, cx<T> &U)
{
    t = cinv(mk<T>(T(2 * m), T(0)) - z2 * t);
    if (m & 1) {
        U = U * (z2 * (tprev * t));
        if (m - 1 >= 2) U.re += T(2);
    }
    tprev = t;
}

template <typename T, int PMAX>
__host__ __device__ inline void bessel_ratios(cx<T> k, T X, T Y, int P, cx<T> *tm, cx<T> &J0)
{
    cx<T> z2 = (k * k) * (X * X + Y * Y);
    const int N = miller_start<T>(z2, P);
    cx<T> t = mk<T>(0, 0), tprev = mk<T>(0, 0), U = mk<T>(0, 0);
    for (int m = N; m > P; --m) miller_step<T>(z2, m, t, tprev, U);
#pragma unroll PUnroll<PMAX>::n
    for (int m = PMAX; m >= 1; --m) {
        if (m <= P) {
            miller_step<T>(z2, m, t, tprev, U);
            tm[m] = t;
        }
    }
    J0 = cinv(mk<T>(T(1), T(0)) + U);
}

// Scaled basis values written to out[(P+q)*stride], q = -P..P.  The ratios
// t_m = J_m / J_{m-1} of the downward recurrence are parked in the slots of
// q = m and turned into basis values in increasing q, so that no per-thread
// array of P values is needed.
template <typename T>
__host__ __device__ inline void bessel_basis(cx<T> k, T X, T Y, T invR, int P, int sign, cx<T> *out, int stride)
{
    const cx<T> z2 = (k * k) * (X * X + Y * Y);
    const int N = miller_start<T>(z2, P);
    cx<T> t = mk<T>(0, 0), tprev = mk<T>(0, 0), U = mk<T>(0, 0);
    for (int m = N; m > P; --m) miller_step<T>(z2, m, t, tprev, U);
    for (int m = P; m >= 1; --m) {
        miller_step<T>(z2, m, t, tprev, U);
        out[(P + m) * stride] = t;
    }
    const cx<T> J0 = cinv(mk<T>(T(1), T(0)) + U);
    out[P * stride] = J0;
    const cx<T> up = mk<T>(X * invR, T(sign) * Y * invR);   // (X + i sign Y)/R
    const cx<T> dn = mk<T>(-X * invR, T(sign) * Y * invR);  // -(X - i sign Y)/R
    cx<T> vp = J0, vm = J0;
    for (int q = 1; q <= P; ++q) {
        const cx<T> f = T(2 * q) * out[(P + q) * stride];
        vp = vp * (f * up);
        vm = vm * (f * dn);
        out[(P + q) * stride] = vp;
        out[(P - q) * stride] = vm;
    }
}

// ---------------------------------------------------------------------------
// Tree geometry
// ---------------------------------------------------------------------------
constexpr int MAXLEV = 24;

struct Level {
    int P;           // expansion order at this level
    int nc;          // 2P + 1
    int col_lo;      // first column (global index) covered at this level
    int ncol;        // columns covered
    int rows_s;      // rows of source boxes (above y = 0)
    int rows_t;      // rows of target boxes (below y = 0)
    double w;        // box width
    int64_t off_s;   // offset (in complex elements) of this level's multipole block
    int64_t off_t;   // offset of this level's local block
    int64_t off_occ; // offset of this level's source-box occupancy flags
};

struct Geometry {
    double x_lo, W;
    int L;
    int ltop;  // coarsest level carrying expansions (M2L among all its non-adjacent boxes)
    Level lev[MAXLEV + 1];
    int64_t ncoef_s, ncoef_t;  // total complex coefficients (times nrhs)
    int64_t nocc_s;            // source boxes over all levels (one occupancy flag each)
};

// Near-field node record (FP64): lambda, the source-side and target-side
// square roots s_s = sqrt(lam^2 - k_src^2), s_t = sqrt(lam^2 - k_tgt^2), and the
// weighted density D = dlam-weight * sigma_2^t / (4 pi s2).
struct Node {
    double lr, li, ssr, ssi, str, sti, dr, di;
};

constexpr int NGL = 16;  // Gauss-Legendre points per panel

// ---------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files)
// ---------------------------------------------------------------------------
// tree.hip
// bounding box (targets in their tree coordinates) and the count of points
// outside their layers (ly) of both point sets: nblk = bbox_blocks(n)
// blocks write partials (partial[nblk][8]), one wave reduces them and writes
// out[0..6] and then the 64-bit sequence number at out + 8 (host-mapped
// memory).  The sequence number is *dseq + 1, stored back to *dseq (device
// memory, zero at first), so that launches replayed from a graph still
// number their results.
void launch_bbox(const double *src, int64_t ns, const double *tgt, int64_t nt, const Layers &ly,
                 double *partial, uint64_t *dseq, int nblk, double *out, hipStream_t st);
// out = (x, -(a y + b)) of every point
void launch_mirror(const double *xy, int64_t n, double a, double b, double *out, hipStream_t st);
int bbox_blocks(int64_t n);
// Points grouped by leaf (counting sort; every leaf in increasing original
// index).  cnt: nbox counts, zero on entry.  Results: start/end[nbox] (leaf
// ranges in the grouped order), idx[n] (original index, targets offset by
// n_src), xs/ys[n] (grouped coordinates).  key, perm: n; scratch: 2n.
// Tree-build buffers.  cnt (one counter per leaf) must be zero when a build
// starts; each build leaves it zero.  err[0] collects the build's error flag,
// err[1] receives it at the scan (err[0] is then cleared).  The densities q
// ([nrhs][ns] elements of qw 64-bit words) are copied in the sources' grouped
// order to qs (same layout), unless q is null.
struct TreeBufs {
    uint32_t *key;
    int32_t *rank, *cnt, *tab, *start, *end, *perm, *scratch, *idx;  // scratch: 2n; tab: tree_table_len(n)
    double *xs, *ys;
    const uint64_t *q = nullptr;
    uint64_t *qs = nullptr;
    int nrhs = 0, qw = 0;
};
void launch_tree(const double *src, int64_t ns, const double *tgt, int64_t nt, double x_lo, double w, int col_lo,
                 int ncol, int rows_s, int rows_t, const Layers &ly, const TreeBufs &b, int32_t *err, bool radix,
                 hipStream_t st);
void launch_zero_bytes(void *p, size_t nbytes, hipStream_t st);
// Grouping form of a tree of n points (form: -1 by size, 0 counting sort, 1
// radix sort; a recorded batch decides by all its points), the kernels
// launch_tree issues for nbox leaves, and the ints of TreeBufs::tab.
constexpr int64_t TREE_RADIX_MIN_POINTS = 300000;
bool tree_radix(int64_t n, int form);
int tree_launch_count(int64_t nbox, bool radix);
int64_t tree_table_len(int64_t n);


// leaf.hip and translate.hip (T = double or float)
// (occ: the source-box occupancy flags of every level, Level::off_occ; P2M
// writes the leaves', M2M the parents; series: P2M by the ascending series
// where the leaves' k1 R allows it)
template <typename T>
void launch_p2m(const int32_t *start, const int32_t *end, const double *xs, const double *ys, const void *qs,
                int64_t ns, int nrhs, const Geometry &g, Medium med, cx<T> *M, int32_t *occ, bool series,
                hipStream_t st);
template <typename T>
// (mfma: on the matrix cores)
void launch_m2m(const Geometry &g, int lchild, const cx<T> *tab, cx<T> *M, int32_t *occ, int nrhs, bool mfma,
                hipStream_t st);
// downward pass of level l: M2L (atab non-null; class slots of target row r:
// row_off[r] .. row_off[r + 1], rows < nrt) and/or L2L from level l - 1
// (l2l_tab non-null); add_rows: rows whose stored local expansion (M2L of an
// earlier launch) is added to the L2L shift; rows_l2l: the L2L shift covers
// rows below it only (-1: every row); mfma: the L2L form on the matrix cores
template <typename T>
void launch_down(const Geometry &g, int l, const cx<T> *atab, const int *cls3, const int *row_off, int nrt,
                 const cx<T> *M, cx<T> *Lc, int nrhs, const cx<T> *l2l_tab, bool top, int add_rows,
                 hipStream_t st, int rows_l2l = -1, bool mfma = false);
// M2L of levels l0 .. l1 (entry l - l0 of each array: class tables, class
// codes, row slot offsets, number of rows with classes; a null table skips
// the level); the result is stored as the local expansion.  mfma: products of
// the class tables with tiles of boxes on the matrix cores, the coarsest level
// (part 1) and the others (part 2) in a launch each (part 0: both); else
// per-box matrix-vector products on the vector units, every level in one
// launch (part 1 launches nothing).  occ: source-box occupancy flags.
template <typename T>
void launch_m2l_all(const Geometry &g, int l0, int l1, const cx<T> *const *atab, const int *const *cls3,
                    const int *const *row_off, const int *nrt, const cx<T> *M, cx<T> *Lc, int nrhs, bool mfma,
                    const int32_t *occ, int part, hipStream_t st);
// returns the number of node parts written to unear ([part][rhs][target])
template <typename T>
int launch_near_sweep(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs,
                      const double *ys, const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g,
                      const Node *nodes, int nmid, int npan, double t0, cx<double> *unear, hipStream_t st);
// The leaf level's L2L shift done by the leaf evaluation itself: tab (null:
// read the stored leaf expansions instead), parent expansions Lp of level
// L - 1 (ncp coefficients, ncol_p columns from col_lo_p, rows_p rows), and
// add_rows: leaf rows whose stored M2L result is added.
template <typename T>
struct LeafShift {
    const cx<T> *tab = nullptr;
    const cx<T> *Lp = nullptr;
    int ncp = 0, ncol_p = 0, col_lo_p = 0, rows_p = 0, add_rows = 0;
};
// The local expansions that the leaf evaluation reads.  on = 0: every leaf
// evaluates its own expansion (level L).  on = 1: the downward pass shifts
// every row down to level lc and, below it, only the rows with M2L classes
// (row < nrt[l]) and their ancestors; a leaf evaluates the expansion of its
// ancestor at the finest level e >= lc at which that ancestor has M2L
// classes, else at lc.  Below e the downward pass adds nothing to the leaf's
// ancestors, so that expansion holds the leaf's whole far field, and the L2L
// shifts of the other rows are not needed.  Per level: the order, the columns
// and the offset of its block of local expansions.
struct EvalLevels {
    int on = 0, lc = 0, L = 0;
    int nrt[MAXLEV + 1] = {};
    int P[MAXLEV + 1] = {};
    int ncol[MAXLEV + 1] = {};
    int64_t off[MAXLEV + 1] = {};
};
__host__ __device__ inline int eval_level(const EvalLevels &ev, int row)
{
    if (!ev.on) return ev.L;
    for (int l = ev.L; l > ev.lc; --l)
        if ((row >> (ev.L - l)) < ev.nrt[l]) return l;
    return ev.lc;
}
// Lc: the local expansions of every level (ev.off[l] is level l's block)
template <typename T>
void launch_l2p_near(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs,
                     const double *ys, const void *q, int64_t ns, int64_t nt, int nrhs, const Geometry &g,
                     Medium med, const cx<T> *Lc, const LeafShift<T> &shift, const EvalLevels &ev, const Node *nodes,
                     int nmid, int npan, double t0, int do_far, int do_near, const cx<double> *unear, int nparts,
                     void *u, hipStream_t st);
template <typename T>
void launch_l2p_grad(const int32_t *start, const int32_t *end, const int32_t *idx, const double *xs,
                     const double *ys, const void *q, const void *cw, int64_t ns, int64_t nt, int nrhs,
                     const Geometry &g, Medium med, const cx<T> *Lc, const Node *nodes, int nmid, int npan, double t0,
                     int do_far, int do_near, double ysign, double *gout, hipStream_t st);
// direct sum over all pairs, split into nchunk source chunks (partials in
// part: nchunk * nrhs * nt, needed when nchunk > 1); direct_chunks picks nchunk
int direct_chunks(int64_t ns, int64_t nt, int nrhs);
// (a target's tree coordinate is ty_a y + ty_b)
void launch_direct(const double *src, int64_t ns, const void *q, const double *tgt, int64_t nt, double ty_a,
                   double ty_b, int nrhs, int prec, const Node *nodes, int nmid, int npan, double t0, int nchunk,
                   cx<double> *part, void *u, hipStream_t st);

// noalloc.hip: the fixed device array of lmfmm_apply_noalloc (its size is
// LMFMM_NOALLOC_MAX_BYTES of lmfmm.h).  init resolves the address on device
// dev (which must be current); ptr returns it, or null before init.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
hipError_t noalloc_scratch_init(int dev);
void *noalloc_scratch_ptr(int dev);

// tables.hip
void launch_node_table(const double *lamw, int n, Medium med, Node *out, hipStream_t st);
void launch_m2l_tables(const double *lamw, const int *node_cls, const int *node_local, int ntot,
                       const double *cls_geo, Medium med, const int *cls_P, const int *cls_Q,
                       const int64_t *cls_toff, const int64_t *cls_aoff, int ncls, int ncmax, cx<double> *Tm,
                       cx<double> *Sm, cx<double> *A, cx<float> *A32, hipStream_t st);

}  // namespace lmfmm
