// Host side of the library: plan state, tree geometry, table construction and
// the apply sequence of Algorithm 1, behind the C ABI of include/lmfmm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <immintrin.h>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <map>
#include <string>
#include <vector>

#include "lmfmm.h"
#include "lmfmm_internal.h"

using namespace lmfmm;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define HIPCHK(x)                                                                                            \
    do {                                                                                                     \
        hipError_t e_ = (x);                                                                                 \
        if (e_ != hipSuccess) return fail(LMFMM_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));    \
    } while (0)

// ---------------------------------------------------------------------------
// Device buffer
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
    uint64_t gen = 0;  // allocations so far (a new allocation may reuse the old address)
    int ensure(size_t bytes)
    {
        if (bytes <= n && p) return LMFMM_OK;
        if (p) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
            p = nullptr;
            n = 0;
        }
        size_t want = bytes < 256 ? 256 : bytes;
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            return fail(LMFMM_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
        }
        n = want;
        ++gen;
        return LMFMM_OK;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// Bump allocator over one device arena.
struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *r = reinterpret_cast<T *>(base + off);
        off += count * sizeof(T);
        return r;
    }
};

// ---------------------------------------------------------------------------
// Gauss-Legendre rule (Newton on the Legendre polynomial, three-term recurrence)
// ---------------------------------------------------------------------------
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
            double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        pp = n * (z * p1 - p2) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

typedef std::complex<double> zc;

// Nodes of one contour piece: appends (lam, weight) pairs.
struct NodeList {
    std::vector<double> lw;  // [n][4]: lam re, lam im, w re, w im
    int count() const { return (int)(lw.size() / 4); }
    void add(zc lam, zc w)
    {
        lw.push_back(lam.real());
        lw.push_back(lam.imag());
        lw.push_back(w.real());
        lw.push_back(w.imag());
    }
};

static const std::vector<double> &gl_x()
{
    static std::vector<double> x, w;
    if (x.empty()) gauss_legendre(NGL, x, w);
    return x;
}
static const std::vector<double> &gl_w()
{
    static std::vector<double> x, w;
    if (w.empty()) gauss_legendre(NGL, x, w);
    return w;
}

// Finite piece of the contour: lam(t) = t - i h sin(pi t / c), t in [-c, c],
// below the real axis for Re lam > 0 and above it for Re lam < 0, where the
// integrand has no singularity (Section 4.2, Fig. 1 argument).
static void add_bump(NodeList &nl, double c, double h, int npan)
{
    const auto &X = gl_x();
    const auto &W = gl_w();
    for (int p = 0; p < npan; ++p) {
        double a = -c + 2.0 * c * p / npan, b = -c + 2.0 * c * (p + 1) / npan;
        double hw = 0.5 * (b - a), m = 0.5 * (a + b);
        for (int i = 0; i < NGL; ++i) {
            double t = m + hw * X[i];
            zc lam(t, -h * std::sin(M_PI * t / c));
            zc dl(1.0, -h * M_PI / c * std::cos(M_PI * t / c));
            nl.add(lam, W[i] * hw * dl);
        }
    }
}

// Ray panel [ta, tb] of both rays: right lam = c + t e^{i s psi}, left
// lam = -c - t e^{-i s psi} (traversed towards -c); weights include dlam/dt.
static void add_ray_panel(NodeList &nl, double c, double psi, double sgn, double ta, double tb)
{
    const auto &X = gl_x();
    const auto &W = gl_w();
    zc er = std::polar(1.0, sgn * psi), el = std::polar(1.0, -sgn * psi);
    double hw = 0.5 * (tb - ta), m = 0.5 * (ta + tb);
    for (int i = 0; i < NGL; ++i) {
        double t = m + hw * X[i];
        nl.add(zc(c, 0) + t * er, W[i] * hw * er);
    }
    for (int i = 0; i < NGL; ++i) {
        double t = m + hw * X[i];
        nl.add(zc(-c, 0) - t * el, W[i] * hw * el);
    }
}

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct LevelTables {
    int P = 0, Pp = 0;
    DevBuf m2m64, m2m32, l2l64, l2l32;  // [4][nc_in][nc_out]
    DevBuf a64, a32;                    // M2L tables [slot][nc][nc]
    DevBuf clsof;                       // int[3 * nslots]: target row, source row, column offset
    std::vector<int> clsof_host;
    DevBuf rowoff;                      // slots of target row r are [rowoff[r], rowoff[r+1])
    int nslots = 0;
    int nrt = 0;  // target rows with classes (row_off has nrt + 1 entries)
    int64_t nodes = 0;
};

struct VarTables {
    // far-field tables
    int t_L = -1, t_top = -1;
    double t_W = -1;
    int t_P[MAXLEV + 1] = {0};
    std::vector<int> t_shape;  // row and column counts the class sets were built for
    uint64_t version = 0;      // bumped on every rebuild of any table
    LevelTables lt[MAXLEV + 1];
    double table_seconds = 0;
    // near-field node table
    DevBuf near_nodes;
    double n_c = 0, n_h = -1, n_t0 = 0;
    int n_nmid = 0, n_npan = 0;
    void release()
    {
        near_nodes.release();
        for (auto &t : lt) {
            t.m2m64.release();
            t.m2m32.release();
            t.l2l64.release();
            t.l2l32.release();
            t.a64.release();
            t.a32.release();
            t.clsof.release();
            t.rowoff.release();
        }
    }
};

struct lmfmm_plan_s {
    int device = 0;  // the device current at creation
    Medium med;
    int order = 16;
    double tol = 1e-6;
    int levels_opt = 0;
    int fixed_order = 0;
    double kr_max = 8.0;
    bool have_domain = false;
    bool have_box = false;        // pinned bounding box (set by the batch driver)
    double box[6] = {0, 0, 0, 0, 0, 0};
    double dom[4] = {0, 0, 0, 0};  // xmin, xmax, ys_max, yt_min
    bool do_near = true, do_far = true;
    bool near_sweep = true;  // near field by x-ordered sweeps (else pairwise)
    int tree_sort = -1;      // grouping by radix sort (1), by counting sort (0), or chosen by the point count (-1)
    int m2l_mfma = -1;       // M2L on the matrix cores (1), as vector matrix-vector products (0), or chosen by nrhs (-1)
    bool eval_levels = true; // leaves evaluate the expansion of the level where their far field is complete
    bool shift_mfma = true;  // M2M and L2L on the matrix cores (else vector matrix-vector products)
    bool p2m_series = true;  // P2M by the ascending series where k1 R is small (else the recurrence form)

    DevBuf ws;
    double *h_bbox = nullptr;  // pinned, host-coherent: [0..6] box, [8] sequence number, [12] error copy
    double *d_bbox = nullptr;  // its device address
    uint64_t bbox_seq = 0;
    DevBuf bbox_dev;           // per-block partials [512][8], then the sequence counter (at [512][1])

    // cached tables of the forward (0) and transposed (1) operator
    VarTables vt[2];
    DevBuf mirror;  // mirrored coordinates for the transposed operator

    // direct-sum node table and source-chunk partials
    DevBuf dir_nodes, dir_part;
    double d_h = -1;
    int d_nmid = 0, d_npan = 0;
    double d_t0 = 0;

    Geometry geo;
    lmfmm_stats stats;
    // Work counts that depend on how the points fall into the leaves (the
    // leaf evaluation at its levels, the near-field sweep over the row-0
    // leaves): the last apply's leaf ranges are read back when the
    // statistics are asked for.
    struct DeferredWork {
        bool pending = false, far = false, grad = false, sweep = false;
        const int32_t *start = nullptr, *end = nullptr;  // leaf ranges (source keys, then target keys)
        Geometry g;
        std::vector<std::vector<int>> cls;  // class codes per level
        EvalLevels ev;
        int rows_l2l[MAXLEV + 1] = {};
        int nrhs = 0, nodes = 0;
    } dw;
    EvalLevels last_ev;           // evaluation levels of the last launch sequence
    int last_rows_l2l[MAXLEV + 1] = {};
    int32_t *d_err = nullptr;  // device error flags of the last apply (in the workspace)
    bool err_valid = false;    // the last apply built a tree (and so wrote d_err[1])
    // the workspace prefix holding the error flags and leaf counters, zeroed
    // once per allocation (every tree build leaves it zero again)
    uint64_t tz_gen = 0;
    size_t tz_bytes = 0;

    // per-kernel timing: an event before each timed kernel (or kernel group)
    // and one after the last; interval j is attributed to ev_tag[j]
    // timing entries j: events ev[2j] (start) and ev[2j + 1] (stop), either
    // stamped by the runtime at a kernel's start and end or recorded around
    // a group of kernels (bounding box and tree build)
    static constexpr int NEV = 96;
    bool timing = false;
    bool ev_pending = false;
    hipEvent_t ev[NEV] = {};
    int ev_tag[NEV / 2] = {0};
    int ev_nl[NEV / 2] = {0};
    int ev_n = 0;

    // replay of the apply's launch sequence as a HIP graph: captured on the
    // second consecutive apply with the same key (geometry, pointers, sizes,
    // tables, flags), replayed while the key stays the same
    bool use_graph = true;
    std::vector<uint64_t> gkey, last_key;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // With the bounding box computed on the device, the graph starts with the
    // bounding-box kernel.  An apply whose arguments, options, tables and
    // workspace are those the graph was captured with (g_prekey) launches it
    // at once and then checks the box it computed against g_bb; on a mismatch
    // the replay's results are discarded (recomputed for the new box).
    bool g_bbox = false;
    double g_bb[7] = {0, 0, 0, 0, 0, 0, 0};
    std::vector<uint64_t> g_prekey;
    size_t g_zero_bytes = 0;   // the workspace prefix its tree build needs zeroed
    uint64_t cfg_version = 0;  // bumped by every set_option call

    // cached M2L pair counts per level for the last geometry
};

// Fold the events of the previous timed apply into the statistics.
static void collect_timing(lmfmm_plan_s *p)
{
    if (!p->ev_pending) {
        p->ev_n = 0;  // an apply that failed part-way leaves no timing
        return;
    }
    const int n = p->ev_n;
    (void)hipEventSynchronize(p->ev[2 * n - 1]);
    for (int j = 0; j < n; ++j) {
        float ms = 0.f;
        int t = p->ev_tag[j];
        if (hipEventElapsedTime(&ms, p->ev[2 * j], p->ev[2 * j + 1]) == hipSuccess) p->stats.kernel_ms[t] += ms;
        p->stats.kernel_launches[t] += p->ev_nl[j];
    }
    p->stats.timed_applies += 1;
    p->ev_pending = false;
    p->ev_n = 0;
}

// largest real part of the wave numbers the density depends on (the
// impedance half-space has only k1)
static double kmax_re(const Medium &m)
{
    return m.comp == COMP_IMP ? m.k1.re : std::max(m.k1.re, std::max(m.k2.re, m.k3.re));
}
static double contour_c(const Medium &m) { return std::max(1.0, 1.25 * kmax_re(m)); }

// Smallest n with |J_n(z)| <= eps for real z > 0 (n >= z): Miller ratios.
static int bessel_cutoff(double z, double eps)
{
    if (!(z > 0)) return 0;
    int M = (int)std::ceil(z) + 80;
    if (M > 1000) M = 1000;
    std::vector<cx<double>> tm(1025);
    cx<double> J0;
    bessel_ratios<double, 1024>(cx<double>{z, 0.0}, 1.0, 0.0, M, tm.data(), J0);
    double v = std::fabs(J0.re);
    for (int n = 1; n <= M; ++n) {
        v *= std::fabs(z * tm[n].re);  // |J_n / J_{n-1}| = |z t_n| (real argument)
        if (n >= z && v <= eps) return n;
    }
    return M;
}

// Low-frequency limit for the expansions: a level carries multipole and
// local expansions only if k R <= kr_max (R the box half-diagonal; plan
// option "kr_max", default 8: above it the translation tables lose digits
// to cancellation on the finite contour piece).

static double kabs_max(const Medium &m)
{
    const cx<double> kt = k_target_layer(m);
    return std::max(std::abs(zc(m.k1.re, m.k1.im)), std::abs(zc(kt.re, kt.im)));
}

// Expansion order at a level: max(order, the order the tolerance needs for the
// worst one-box-separated pair (ratio ~0.4 per term, Theorem 1), the order at
// which |J_P(|k| R)| falls below 1e-4 tol for the level's box radius R).  The
// Bessel margin covers the slow decay of the expansions' terms for lambda just
// above the branch point at the high-frequency levels (k R near kr_max): with
// tol/100 there, an FP64 apply at tol 1e-10 measured 1.7e-10 against the
// oracle.
static int order_for_level(const lmfmm_plan_s *p, double w)
{
    if (p->fixed_order) return p->order;
    double R = w / std::sqrt(2.0);
    int ptol = (int)std::ceil(std::log(p->tol) / std::log(0.4));
    int pj = bessel_cutoff(kabs_max(p->med) * R, 1e-4 * p->tol);
    int P = std::max(p->order, std::max(ptol, pj));
    return std::min(P, 480);
}

// Build the geometry from a bounding box {xmin, xmax, ys_min, ys_max, yt_min, yt_max}.
static int make_geometry(lmfmm_plan_s *p, const double *bb, int64_t ns, int nrhs, Geometry &g)
{
    double xmin = bb[0], xmax = bb[1], ysmax = bb[3], ytmin = bb[4];
    if (!(xmax >= xmin)) xmin = xmax = 0.0;
    if (!(ysmax > 0)) ysmax = 0.0;
    if (!(ytmin < 0)) ytmin = 0.0;
    double ext = std::max(xmax - xmin, 2.0 * std::max(ysmax, -ytmin));
    if (!(ext > 0)) ext = 1.0;
    double W = ext * (1.0 + 1e-9) + 1e-300;
    g.W = W;
    g.x_lo = 0.5 * (xmin + xmax) - 0.5 * W;
    int L = p->levels_opt;
    if (L <= 0) {
        L = 1;
        for (int l = 2; l <= 20; ++l) {
            double w = W / std::ldexp(1.0, l);
            double ncol = std::floor((xmax - g.x_lo) / w) - std::floor((xmin - g.x_lo) / w) + 1;
            double rows = std::floor(std::max(ysmax, 0.0) / w) + 1;
            rows = std::min(rows, std::ldexp(1.0, l - 1));
            if ((double)ns / (ncol * rows) >= 24.0)
                L = l;
            else
                break;
        }
    }
    if (L > MAXLEV) return fail(LMFMM_EINVAL, "too many levels");
    g.L = L;
    double wL = W / std::ldexp(1.0, L);
    long maxcol = (1L << L) - 1, maxrow = (1L << (L - 1)) - 1;
    long clo = (long)std::floor((xmin - g.x_lo) / wL), chi = (long)std::floor((xmax - g.x_lo) / wL);
    clo = std::max(0L, std::min(clo, maxcol));
    chi = std::max(clo, std::min(chi, maxcol));
    long rs = std::min((long)std::floor(ysmax / wL), maxrow) + 1;
    long rt = std::min((long)std::floor(-ytmin / wL), maxrow) + 1;
    int64_t offs = 0, offt = 0;
    for (int l = L; l >= 1; --l) {
        Level &lv = g.lev[l];
        int sh = L - l;
        lv.w = W / std::ldexp(1.0, l);
        lv.col_lo = (int)(clo >> sh);
        lv.ncol = (int)((chi >> sh) - (clo >> sh) + 1);
        lv.rows_s = (int)(((rs - 1) >> sh) + 1);
        lv.rows_t = (int)(((rt - 1) >> sh) + 1);
        lv.P = order_for_level(p, lv.w);
        lv.nc = 2 * lv.P + 1;
    }
    g.lev[0] = g.lev[1];
    g.ltop = L;
    for (int l = 2; l <= L; ++l)
        if (kabs_max(p->med) * g.lev[l].w / std::sqrt(2.0) <= p->kr_max) {
            g.ltop = l;
            break;
        }
    for (int l = 1; l <= L; ++l) {
        Level &lv = g.lev[l];
        lv.off_s = offs;
        lv.off_t = offt;
        offs += (int64_t)lv.rows_s * lv.ncol * lv.nc * nrhs;
        offt += (int64_t)lv.rows_t * lv.ncol * lv.nc * nrhs;
    }
    g.ncoef_s = offs;
    g.ncoef_t = offt;
    int64_t nocc = 0;
    for (int l = 1; l <= L; ++l) {
        g.lev[l].off_occ = nocc;
        nocc += (int64_t)g.lev[l].rows_s * g.lev[l].ncol;
    }
    g.lev[0].off_occ = 0;
    g.nocc_s = nocc;
    return LMFMM_OK;
}

// Free-space shift tables (Lemma M2M with k1, Lemma L2L with k2), scaled.
// g_m = J_m(k rho) e^{sign i m phi} for |m| <= M, from the Bessel ratios.
static void shift_coeffs(zc k, double X, double Y, int M, int sign, std::vector<zc> &g)
{
    std::vector<cx<double>> tm(M + 1);
    cx<double> J0;
    cx<double> kk = {k.real(), k.imag()};
    // bessel_ratios is instantiated with a large static bound on the host
    std::vector<cx<double>> buf(1025);
    bessel_ratios<double, 1024>(kk, X, Y, M, buf.data(), J0);
    g.assign(2 * M + 1, zc(0, 0));
    zc j0(J0.re, J0.im);
    g[M] = j0;
    zc up = k * zc(X, sign * Y), dn = -k * zc(X, -sign * Y);
    zc vp = j0, vm = j0;
    for (int m = 1; m <= M; ++m) {
        zc t(buf[m].re, buf[m].im);
        vp *= t * up;
        vm *= t * dn;
        g[M + m] = vp;
        g[M - m] = vm;
    }
}

// log of the scale factor s_n = |n|! (2/(kR))^|n| as a complex number
static zc log_scale(int n, zc k, double R)
{
    int a = std::abs(n);
    return zc(std::lgamma(a + 1.0), 0.0) + (double)a * std::log(zc(2.0, 0.0) / (k * R));
}

static int upload(DevBuf &b, const void *h, size_t bytes)
{
    int rc = b.ensure(bytes);
    if (rc) return rc;
    HIPCHK(hipMemcpy(b.p, h, bytes, hipMemcpyHostToDevice));
    return LMFMM_OK;
}

static int build_shift_tables(VarTables &vt, const Medium &med, const Geometry &g, int l)
{
    // children at level l, parents at level l - 1
    LevelTables &T = vt.lt[l];
    const Level &c = g.lev[l], &pa = g.lev[l - 1];
    int ncc = c.nc, ncp = pa.nc, Pc = c.P, Pp = pa.P;
    double Rc = c.w / std::sqrt(2.0), Rp = pa.w / std::sqrt(2.0);
    // multipole side (M2M) and local side (L2L) wave numbers
    cx<double> kS = k_src(med), kT = k_tgt(med);
    zc k1(kS.re, kS.im), k2(kT.re, kT.im);
    std::vector<cx<double>> m2m((size_t)4 * ncc * ncp), l2l((size_t)4 * ncp * ncc);
    std::vector<zc> gm;
    for (int pos = 0; pos < 4; ++pos) {
        int dx = pos & 1, dy = pos >> 1;
        double X = (dx - 0.5) * c.w;
        // sources: child centre minus parent centre, multipole shift with k1
        double Ys = (dy - 0.5) * c.w;
        shift_coeffs(k1, X, Ys, Pc + Pp, -1, gm);
        for (int a = 0; a < ncc; ++a)
            for (int b = 0; b < ncp; ++b) {
                int np_ = b - Pp, nc_ = a - Pc;  // parent index n, child index n'
                zc sc = std::exp(log_scale(np_, k1, Rp) - log_scale(nc_, k1, Rc));
                zc v = sc * gm[(Pc + Pp) + (np_ - nc_)];
                m2m[((size_t)pos * ncc + a) * ncp + b] = {v.real(), v.imag()};
            }
        // targets: child centre minus parent centre (rows grow downwards), local shift with k2
        double Yt = -(dy - 0.5) * c.w;
        shift_coeffs(k2, X, Yt, Pc + Pp, +1, gm);
        for (int a = 0; a < ncp; ++a)
            for (int b = 0; b < ncc; ++b) {
                int npp = a - Pp, nch = b - Pc;  // parent index n'', child index n
                zc sc = std::exp(log_scale(npp, k2, Rp) - log_scale(nch, k2, Rc));
                zc v = sc * gm[(Pc + Pp) + (npp - nch)];
                l2l[((size_t)pos * ncp + a) * ncc + b] = {v.real(), v.imag()};
            }
    }
    std::vector<cx<float>> m2m32(m2m.size()), l2l32(l2l.size());
    for (size_t i = 0; i < m2m.size(); ++i) m2m32[i] = {(float)m2m[i].re, (float)m2m[i].im};
    for (size_t i = 0; i < l2l.size(); ++i) l2l32[i] = {(float)l2l[i].re, (float)l2l[i].im};
    int rc;
    if ((rc = upload(T.m2m64, m2m.data(), m2m.size() * sizeof(cx<double>)))) return rc;
    if ((rc = upload(T.m2m32, m2m32.data(), m2m32.size() * sizeof(cx<float>)))) return rc;
    if ((rc = upload(T.l2l64, l2l.data(), l2l.size() * sizeof(cx<double>)))) return rc;
    if ((rc = upload(T.l2l32, l2l32.data(), l2l32.size() * sizeof(cx<float>)))) return rc;
    return LMFMM_OK;
}

// M2L tables of one level: one class per (target row, source row, column offset).
static int build_m2l_tables(VarTables &vt, const Medium &med, const Geometry &g, int l, bool full)
{
    LevelTables &T = vt.lt[l];
    const Level &lv = g.lev[l];
    int P = lv.P, nc = lv.nc;
    double w = lv.w, R = w / std::sqrt(2.0), c = contour_c(med);
    std::vector<int> cls_of, row_off;
    NodeList nl;
    std::vector<int> node_cls, node_local, cP, cQ;
    std::vector<int64_t> toff, aoff;
    std::vector<double> geo;
    int64_t tsum = 0;
    int slot = 0;
    // Classes (target row rt, source row rs, column offset dc = source - target
    // column).  Standard level: rows 0/1 and |dc| <= 3 (children of adjacent
    // parents); top level: every non-adjacent pair of its boxes.
    const int nrt = full ? lv.rows_t : std::min(2, lv.rows_t);
    const int nrs = full ? lv.rows_s : std::min(2, lv.rows_s);
    const int dmax = full ? lv.ncol - 1 : 3;
    if (full && (int64_t)nrt * nrs * (2 * dmax + 1) > 4096)
        return fail(LMFMM_ETOL, "too many translation classes at the coarsest low-frequency level "
                                "(wave number too large for the domain)");
    for (int rt = 0; rt < nrt; ++rt) {
        row_off.push_back(slot);
        for (int rs = 0; rs < nrs; ++rs)
            for (int dc = -dmax; dc <= dmax; ++dc) {
                if (rt == 0 && rs == 0 && std::abs(dc) <= 1) continue;
                double dxc = -dc * w;  // x_t - x_s with source column = target column + dc
                double yt = -(rt + 0.5) * w, ys = (rs + 0.5) * w;
                double a = ys - yt;
                double psi = std::atan2(std::fabs(dxc), a), sgn = dxc >= 0 ? 1.0 : -1.0;
                double rho = std::hypot(dxc, a);
                double h = std::fabs(dxc) > 0 ? std::min(0.25 * c, 3.0 / std::fabs(dxc)) : 0.25 * c;
                int nmp = std::max(16, (int)std::ceil(4.0 * c / h));
                int start = nl.count();
                add_bump(nl, c, h, nmp);
                double umax = 2.0 * P + 60.0;
                double e0 = std::min(c, 2.0 / rho);
                for (int k = 0; k < 4; ++k) add_ray_panel(nl, c, psi, sgn, e0 * k / 4, e0 * (k + 1) / 4);
                // Panels of length 2/rho (two e-folds of the ray's decay), but
                // no longer than their distance from the ray's start: the
                // branch points +-k and the 1/s2 factor sit within ~c of the
                // start, and a panel many times longer than that distance
                // resolves them poorly (for small boxes 2/rho >> c; a 16-node
                // panel of length 2/rho there left 4e-9 relative error at
                // k = 20, leaf width 2e-3, and 4e-6 for the impedance density).
                for (double t = e0; t * rho < umax;) {
                    double len = std::min(2.0 / rho, std::max(t, c));
                    add_ray_panel(nl, c, psi, sgn, t, t + len);
                    t += len;
                }
                int Q = nl.count() - start;
                for (int i = 0; i < Q; ++i) {
                    node_cls.push_back(slot);
                    node_local.push_back(i);
                }
                cls_of.push_back(rt);
                cls_of.push_back(rs);
                cls_of.push_back(dc);
                cP.push_back(P);
                cQ.push_back(Q);
                toff.push_back(tsum);
                aoff.push_back((int64_t)slot * nc * nc);
                tsum += (int64_t)Q * nc;
                geo.push_back(dxc);
                geo.push_back(yt);
                geo.push_back(ys);
                geo.push_back(R);
                ++slot;
            }
    }
    row_off.push_back(slot);
    T.nslots = slot;
    T.nrt = slot > 0 ? nrt : 0;
    T.nodes = nl.count();
    int rc;
    if (slot == 0) return LMFMM_OK;
    if ((rc = upload(T.clsof, cls_of.data(), cls_of.size() * sizeof(int)))) return rc;
    if ((rc = upload(T.rowoff, row_off.data(), row_off.size() * sizeof(int)))) return rc;
    T.clsof_host = cls_of;
    DevBuf d_lw, d_ncls, d_nloc, d_geo, d_P, d_Q, d_toff, d_aoff, d_T, d_S;
    if ((rc = upload(d_lw, nl.lw.data(), nl.lw.size() * sizeof(double)))) return rc;
    if ((rc = upload(d_ncls, node_cls.data(), node_cls.size() * sizeof(int)))) return rc;
    if ((rc = upload(d_nloc, node_local.data(), node_local.size() * sizeof(int)))) return rc;
    if ((rc = upload(d_geo, geo.data(), geo.size() * sizeof(double)))) return rc;
    if ((rc = upload(d_P, cP.data(), cP.size() * sizeof(int)))) return rc;
    if ((rc = upload(d_Q, cQ.data(), cQ.size() * sizeof(int)))) return rc;
    if ((rc = upload(d_toff, toff.data(), toff.size() * sizeof(int64_t)))) return rc;
    if ((rc = upload(d_aoff, aoff.data(), aoff.size() * sizeof(int64_t)))) return rc;
    if ((rc = d_T.ensure((size_t)tsum * sizeof(cx<double>)))) return rc;
    if ((rc = d_S.ensure((size_t)tsum * sizeof(cx<double>)))) return rc;
    if ((rc = T.a64.ensure((size_t)slot * nc * nc * sizeof(cx<double>)))) return rc;
    if ((rc = T.a32.ensure((size_t)slot * nc * nc * sizeof(cx<float>)))) return rc;
    launch_m2l_tables((const double *)d_lw.p, (const int *)d_ncls.p, (const int *)d_nloc.p, nl.count(),
                      (const double *)d_geo.p, med, (const int *)d_P.p, (const int *)d_Q.p,
                      (const int64_t *)d_toff.p, (const int64_t *)d_aoff.p, slot, nc, (cx<double> *)d_T.p,
                      (cx<double> *)d_S.p, (cx<double> *)T.a64.p, (cx<float> *)T.a32.p, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    d_lw.release();
    d_ncls.release();
    d_nloc.release();
    d_geo.release();
    d_P.release();
    d_Q.release();
    d_toff.release();
    d_aoff.release();
    d_T.release();
    d_S.release();
    return LMFMM_OK;
}

// Length of the first ray panel of a pair-independent table: the ray
// integrand decays like exp(-t (a + dx)/sqrt 2), so the first panel must be
// short against 1/dx_max as well as against c.
static double ray_t0(double c, double dxmax) { return std::min(c / 8.0, 0.5 / std::max(dxmax, 1e-300)); }

// Near-field node table on the contour: bump over [-c, c] plus the two rays at
// 45 degrees (valid for x1 - x0 >= 0; |x1 - x0| is used by evenness).  The
// panel count covers pairs down to a vertical gap a_min.
static int build_near_table(DevBuf &buf, const Medium &med, double dxmax, double amin, double &c_out, double &h_out,
                            double &t0_out, int &nmid_out, int &npan_out)
{
    double c = contour_c(med);
    double h = std::min(0.25 * c, 3.0 / std::max(dxmax, 1e-300));
    int nmp = std::max(16, (int)std::ceil(4.0 * c / h));
    double t0 = ray_t0(c, dxmax);
    double ar = std::max(amin, 1e-12) / std::sqrt(2.0);
    int npan = 2 + (int)std::ceil(std::log2(std::max(2.0, 40.0 / (ar * t0))));
    npan = std::min(npan, 64);
    NodeList nl;
    add_bump(nl, c, h, nmp);
    int nmid = nl.count();
    for (int m = 0; m < npan; ++m) {
        double ta = m == 0 ? 0.0 : t0 * std::ldexp(1.0, m - 1), tb = t0 * std::ldexp(1.0, m);
        add_ray_panel(nl, c, M_PI / 4, 1.0, ta, tb);
    }
    DevBuf lw;
    int rc;
    if ((rc = upload(lw, nl.lw.data(), nl.lw.size() * sizeof(double)))) return rc;
    if ((rc = buf.ensure((size_t)nl.count() * sizeof(Node)))) return rc;
    launch_node_table((const double *)lw.p, nl.count(), med, (Node *)buf.p, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    lw.release();
    c_out = c;
    h_out = h;
    t0_out = t0;
    nmid_out = nmid;
    npan_out = npan;
    return LMFMM_OK;
}

// The translation classes of a level depend on the rows next to the interface
// (at most two per side) and, at the coarsest expansion level, on all its rows
// and columns.
static std::vector<int> class_shape(const Geometry &g)
{
    std::vector<int> k;
    for (int l = g.ltop; l <= g.L; ++l) {
        const Level &lv = g.lev[l];
        if (l == g.ltop)
            k.insert(k.end(), {lv.rows_t, lv.rows_s, lv.ncol});
        else
            k.insert(k.end(), {std::min(2, lv.rows_t), std::min(2, lv.rows_s)});
    }
    return k;
}

// build = false: report LMFMM_EINVAL instead of building (allocation-free apply)
static int ensure_far_tables(VarTables &vt, const Medium &med, const Geometry &g, bool build = true)
{
    bool same = vt.t_L == g.L && vt.t_W == g.W && vt.t_top == g.ltop;
    for (int l = 1; same && l <= g.L; ++l) same = vt.t_P[l] == g.lev[l].P;
    std::vector<int> shape = class_shape(g);
    if (same) same = shape == vt.t_shape;
    if (same) return LMFMM_OK;
    if (!build)
        return fail(LMFMM_EINVAL, "the plan has no translation tables for this geometry (an lmfmm_apply with the "
                                  "same geometry builds them)");
    double t_start = (double)clock() / CLOCKS_PER_SEC;
    int rc;
    vt.t_L = -1;
    for (int l = g.ltop; l <= g.L; ++l)
        if ((rc = build_m2l_tables(vt, med, g, l, l == g.ltop))) return rc;
    for (int l = g.ltop + 1; l <= g.L; ++l)
        if ((rc = build_shift_tables(vt, med, g, l))) return rc;
    vt.t_L = g.L;
    vt.t_W = g.W;
    vt.t_top = g.ltop;
    vt.t_shape = shape;
    vt.version++;
    for (int l = 0; l <= MAXLEV; ++l) vt.t_P[l] = l <= g.L ? g.lev[l].P : 0;
    vt.table_seconds = (double)clock() / CLOCKS_PER_SEC - t_start;
    return LMFMM_OK;
}

static int ensure_near_table(VarTables &vt, const Medium &med, const Geometry &g, double amin, bool build = true)
{
    double dxmax = 2.0 * g.lev[g.L].w;
    double c = contour_c(med);
    double h = std::min(0.25 * c, 3.0 / dxmax);
    double t0 = ray_t0(c, dxmax);
    double ar = std::max(amin, 1e-12) / std::sqrt(2.0);
    int npan = std::min(64, 2 + (int)std::ceil(std::log2(std::max(2.0, 40.0 / (ar * t0)))));
    if (vt.near_nodes.p && vt.n_h == h && vt.n_t0 == t0 && vt.n_npan >= npan) return LMFMM_OK;
    if (!build)
        return fail(LMFMM_EINVAL, "the plan has no near-field table for this geometry (an lmfmm_apply with the "
                                  "same geometry builds it)");
    vt.version++;
    return build_near_table(vt.near_nodes, med, dxmax, amin, vt.n_c, vt.n_h, vt.n_t0, vt.n_nmid, vt.n_npan);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
static void resolve_work(lmfmm_plan_s *p);

extern "C" {

const char *lmfmm_status_string(int s)
{
    switch (s) {
    case LMFMM_OK: return "ok";
    case LMFMM_EINVAL: return "invalid argument";
    case LMFMM_EDOMAIN: return "point outside its layer or domain";
    case LMFMM_ENOMEM: return "out of memory";
    case LMFMM_EHIP: return "HIP runtime error";
    case LMFMM_ETOL: return "tolerance cannot be met";
    case LMFMM_ENODEV: return "no GPU";
    default: return "unknown status";
    }
}

const char *lmfmm_last_error(void) { return g_last_error.c_str(); }

int lmfmm_create(const double k[6], double d, int order, double tol, lmfmm_plan *out)
{
    if (!out) return fail(LMFMM_EINVAL, "out is null");
    *out = nullptr;
    if (!k) return fail(LMFMM_EINVAL, "k is null");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(k[i])) return fail(LMFMM_EINVAL, "wave numbers must be finite");
    if (!(k[0] > 0 && k[2] > 0 && k[4] > 0)) return fail(LMFMM_EINVAL, "Re k must be positive");
    if (k[1] < 0 || k[3] < 0 || k[5] < 0) return fail(LMFMM_EINVAL, "Im k must be >= 0");
    if (!(d > 0) || !std::isfinite(d)) return fail(LMFMM_EINVAL, "d must be positive");
    if (order < 1 || order > 256) return fail(LMFMM_EINVAL, "order must be in [1, 256]");
    if (!(tol > 0 && tol < 1)) return fail(LMFMM_EINVAL, "tol must be in (0, 1)");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(LMFMM_ENODEV, "no HIP device available");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LMFMM_ENODEV, "no current HIP device");
    // resolve this device's copy of the allocation-free apply's array (a
    // failure is reported by that entry point, not here)
    (void)noalloc_scratch_init(dev);
    (void)hipGetLastError();
    lmfmm_plan_s *p = new (std::nothrow) lmfmm_plan_s();
    if (!p) return fail(LMFMM_ENOMEM, "plan allocation failed");
    p->device = dev;
    p->med.k1 = {k[0], k[1]};
    p->med.k2 = {k[2], k[3]};
    p->med.k3 = {k[4], k[5]};
    p->med.d = d;
    p->med.adj = 0;
    p->order = order;
    p->tol = tol;
    std::memset(&p->stats, 0, sizeof(p->stats));
    if (hipHostMalloc((void **)&p->h_bbox, 16 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&p->d_bbox, p->h_bbox, 0) != hipSuccess) {
        if (p->h_bbox) (void)hipHostFree(p->h_bbox);
        delete p;
        return fail(LMFMM_ENOMEM, "pinned allocation failed");
    }
    std::memset(p->h_bbox, 0, 16 * sizeof(double));
    if (p->bbox_dev.ensure(8 * 520 * sizeof(double)) ||
        hipMemset(p->bbox_dev.p, 0, 8 * 520 * sizeof(double)) != hipSuccess) {
        (void)hipHostFree(p->h_bbox);
        delete p;
        return fail(LMFMM_ENOMEM, "device allocation failed");
    }
    *out = p;
    return LMFMM_OK;
}

int lmfmm_destroy(lmfmm_plan p)
{
    if (!p) return fail(LMFMM_EINVAL, "plan is null");
    (void)hipDeviceSynchronize();
    p->ws.release();
    p->bbox_dev.release();
    p->dir_nodes.release();
    p->dir_part.release();
    p->mirror.release();
    p->vt[0].release();
    p->vt[1].release();
    if (p->h_bbox) (void)hipHostFree(p->h_bbox);
    for (int i = 0; i < lmfmm_plan_s::NEV; ++i)
        if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    delete p;
    return LMFMM_OK;
}

int lmfmm_set_option(lmfmm_plan p, const char *key, const char *value)
{
    if (!p || !key || !value) return fail(LMFMM_EINVAL, "null argument");
    p->cfg_version++;
    std::string k(key), v(value);
    if (k == "levels") {
        if (v == "auto") {
            p->levels_opt = 0;
            return LMFMM_OK;
        }
        int L = std::atoi(value);
        if (L < 1 || L > MAXLEV) return fail(LMFMM_EINVAL, "levels must be in [1, 24] or auto");
        p->levels_opt = L;
        return LMFMM_OK;
    }
    if (k == "fixed_order") {
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "fixed_order must be 0 or 1");
        p->fixed_order = v == "1";
        return LMFMM_OK;
    }
    if (k == "graph") {
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "graph must be 0 or 1");
        p->use_graph = v == "1";
        p->last_key.clear();
        return LMFMM_OK;
    }
    if (k == "near_sweep") {
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "near_sweep must be 0 or 1");
        p->near_sweep = v == "1";
        return LMFMM_OK;
    }
    if (k == "component" || k == "alpha") {
        Medium m = p->med;
        if (k == "alpha") {
            char *e = nullptr;
            const double a = std::strtod(value, &e);
            if (!e || *e || !std::isfinite(a)) return fail(LMFMM_EINVAL, "alpha must be a finite number");
            m.alpha = a;
        } else if (v == "2t") {
            m.comp = COMP_2T;
        } else if (v == "2b") {
            m.comp = COMP_2B;
        } else if (v == "1s") {
            m.comp = COMP_1S;
        } else if (v == "3s") {
            m.comp = COMP_3S;
        } else if (v == "impedance") {
            m.comp = COMP_IMP;
        } else {
            return fail(LMFMM_EINVAL, "component must be 2t, 2b, 1s, 3s or impedance");
        }
        p->med = m;
        // every table depends on the component: build them again
        for (auto &vt : p->vt) {
            vt.t_L = -1;
            vt.n_h = -1;
            vt.version++;
        }
        p->d_h = -1;
        p->last_key.clear();
        p->g_prekey.clear();
        return LMFMM_OK;
    }
    if (k == "tree_sort") {
        if (v != "radix" && v != "count" && v != "auto")
            return fail(LMFMM_EINVAL, "tree_sort must be radix, count or auto");
        p->tree_sort = v == "auto" ? -1 : (v == "radix" ? 1 : 0);
        return LMFMM_OK;
    }
    if (k == "m2l_mfma") {
        if (v != "0" && v != "1" && v != "auto") return fail(LMFMM_EINVAL, "m2l_mfma must be 0, 1 or auto");
        p->m2l_mfma = v == "auto" ? -1 : (v == "1" ? 1 : 0);
        return LMFMM_OK;
    }
    if (k == "shift_mfma") {
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "shift_mfma must be 0 or 1");
        p->shift_mfma = v == "1";
        return LMFMM_OK;
    }
    if (k == "p2m_series") {
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "p2m_series must be 0 or 1");
        p->p2m_series = v == "1";
        return LMFMM_OK;
    }
    if (k == "eval_levels") {
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "eval_levels must be 0 or 1");
        p->eval_levels = v == "1";
        return LMFMM_OK;
    }
    if (k == "near" || k == "far") {
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "near/far must be 0 or 1");
        (k == "near" ? p->do_near : p->do_far) = v == "1";
        return LMFMM_OK;
    }
    if (k == "kr_max") {
        double v2 = std::atof(value);
        if (!(v2 >= 1.0 && v2 <= 200.0)) return fail(LMFMM_EINVAL, "kr_max must be in [1, 200]");
        p->kr_max = v2;
        return LMFMM_OK;
    }
    if (k == "timing") {
        if (v == "reset") {
            collect_timing(p);
            for (int i = 0; i < 8; ++i) {
                p->stats.kernel_ms[i] = 0;
                p->stats.kernel_launches[i] = 0;
            }
            p->stats.timed_applies = 0;
            return LMFMM_OK;
        }
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "timing must be 0, 1 or reset");
        if (v == "1" && !p->ev[0])
            for (int i = 0; i < lmfmm_plan_s::NEV; ++i)
                if (hipEventCreate(&p->ev[i]) != hipSuccess) return fail(LMFMM_EHIP, "hipEventCreate failed");
        collect_timing(p);
        p->timing = v == "1";
        return LMFMM_OK;
    }
    if (k == "domain") {
        if (v == "auto") {
            p->have_domain = false;
            return LMFMM_OK;
        }
        double a[4];
        if (std::sscanf(value, "%lf,%lf,%lf,%lf", &a[0], &a[1], &a[2], &a[3]) != 4)
            return fail(LMFMM_EINVAL, "domain must be 'xmin,xmax,ys_max,yt_min' or auto");
        if (!(a[1] >= a[0]) || !(a[2] > 0) || !(a[3] < 0)) return fail(LMFMM_EINVAL, "bad domain");
        std::memcpy(p->dom, a, sizeof a);
        p->have_domain = true;
        return LMFMM_OK;
    }
    return fail(LMFMM_EINVAL, "unknown option '" + k + "'");
}

int lmfmm_get_stats(lmfmm_plan p, lmfmm_stats *s)
{
    if (!p || !s) return fail(LMFMM_EINVAL, "null argument");
    collect_timing(p);
    resolve_work(p);
    *s = p->stats;
    return LMFMM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Apply
// ---------------------------------------------------------------------------
static int check_common(lmfmm_plan p, int64_t ns, const double *src, int64_t nt, const double *tgt, const void *in,
                        const void *out, int nrhs, int prec)
{
    if (!p) return fail(LMFMM_EINVAL, "plan is null");
    if (ns < 0 || nt < 0) return fail(LMFMM_EINVAL, "negative size");
    if (ns > (int64_t)1 << 30 || nt > (int64_t)1 << 30) return fail(LMFMM_EINVAL, "too many points");
    if (nrhs < 1 || nrhs > 64) return fail(LMFMM_EINVAL, "nrhs must be in [1, 64]");
    if (prec != LMFMM_C128 && prec != LMFMM_C64_MIXED) return fail(LMFMM_EINVAL, "unknown precision");
    if ((ns > 0 && !src) || (nt > 0 && !tgt)) return fail(LMFMM_EINVAL, "null coordinates");
    if ((ns > 0 && !in) || (nt > 0 && !out)) return fail(LMFMM_EINVAL, "null density or output");
    return LMFMM_OK;
}

// The image map of the plan's field component (a target's tree coordinate
// is a y + b) and its layer in tree coordinates.
static void image_map(const Medium &m, double &a, double &b)
{
    a = 1.0;
    b = 0.0;
    if (m.comp == COMP_2B) {
        a = -1.0;
        b = -2.0 * m.d;
    } else if (m.comp == COMP_1S || m.comp == COMP_IMP) {
        a = -1.0;
    }
}
static void target_layer(const Medium &m, double &lo, double &hi)
{
    switch (m.comp) {
    case COMP_2B: lo = -2.0 * m.d; hi = -m.d; break;  // -d < y < 0
    case COMP_1S:
    case COMP_IMP: lo = -INFINITY; hi = 0.0; break;  // y > 0
    case COMP_3S: lo = -INFINITY; hi = -m.d; break;  // y < -d
    default: lo = -m.d; hi = 0.0;                    // -d < y < 0
    }
}
// Layers of both point sets in tree coordinates: forward, sources y > 0 and
// the targets' image layer; transposed (mirrored coordinates), the sources are
// the mirrored image targets and the targets the mirrored sources (y < 0).
static Layers layers_of(const Medium &m)
{
    double lo, hi, a, b;
    target_layer(m, lo, hi);
    image_map(m, a, b);
    if (m.adj) return Layers{-hi, -lo, -INFINITY, 0.0, 1.0, 0.0};
    return Layers{0.0, INFINITY, lo, hi, a, b};
}

// Bounding box of the points (host readback) or the fixed domain.
// Bounding box on the device: the kernel writes the result into host-coherent
// memory with a sequence number one above the previous launch's.
static void bbox_launch(lmfmm_plan p, const Medium &med, int64_t ns, const double *src, int64_t nt,
                        const double *tgt, hipStream_t st)
{
    double *part = (double *)p->bbox_dev.p;
    uint64_t *dseq = (uint64_t *)(part + 8 * 512 + 1);
    launch_bbox(src, ns, tgt, nt, layers_of(med), part, dseq, bbox_blocks(ns + nt), p->d_bbox, st);
}

// Wait for the result of the bbox_seq-th launch: spin on its sequence number
// (a short wait in the usual case), else synchronize the stream.
static int bbox_wait(lmfmm_plan p, hipStream_t st, double *bb)
{
    const uint64_t seq = p->bbox_seq;
    volatile uint64_t *flag = reinterpret_cast<volatile uint64_t *>(p->h_bbox + 8);
    const auto t0 = std::chrono::steady_clock::now();
    while (*flag != seq) {
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
            HIPCHK(hipStreamSynchronize(st));
            break;
        }
        _mm_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    if (*flag != seq) {
        p->bbox_seq = *flag;  // resynchronise with the device's count
        return fail(LMFMM_EHIP, "bounding-box result did not arrive");
    }
    std::memcpy(bb, p->h_bbox, 7 * sizeof(double));
    bb[7] = 0.0;
    if (bb[6] > 0) return fail(LMFMM_EDOMAIN, std::to_string((long long)bb[6]) + " point(s) outside their layer");
    return LMFMM_OK;
}

static int get_bbox(lmfmm_plan p, const Medium &med, int64_t ns, const double *src, int64_t nt, const double *tgt,
                    hipStream_t st, double *bb)
{
    if (p->have_box && !med.adj) {
        for (int i = 0; i < 6; ++i) bb[i] = p->box[i];
        bb[6] = 0.0;
        return LMFMM_OK;
    }
    if (p->have_domain) {
        bb[0] = p->dom[0];
        bb[1] = p->dom[1];
        bb[2] = 0.0;
        bb[3] = p->dom[2];
        bb[4] = p->dom[3];
        bb[5] = 0.0;
        bb[6] = 0.0;
        return LMFMM_OK;
    }
    bbox_launch(p, med, ns, src, nt, tgt, st);
    HIPCHK(hipGetLastError());
    ++p->bbox_seq;
    return bbox_wait(p, st, bb);
}

// Algorithmic floating-point work of one apply per kernel (complex
// multiply-add = 8 real operations; Bessel/exponential basis of order P at
// 60 P per point; the near-field sweep at 32 per complex exponential plus 8
// per right-hand side, for every point of the row-0 leaves, node and
// direction).  Translations count only boxes that hold points (source boxes
// with sources, target boxes with targets): the statistics call completes
// the counts from the leaf populations of the apply (resolve_work).
static void count_flops(lmfmm_plan_s *p, const VarTables &vt, const Geometry &g, bool far, int64_t ns, int64_t nt,
                        int nrhs, bool grad, bool sweep, const int32_t *start, const int32_t *end)
{
    double *f = p->stats.kernel_flops;
    for (int i = 0; i < 8; ++i) f[i] = 0;
    p->stats.m2l_pairs = 0;
    auto &dw = p->dw;
    dw = lmfmm_plan_s::DeferredWork();
    const Level &lf = g.lev[g.L];
    dw.start = start;
    dw.end = end;
    dw.g = g;
    dw.far = far;
    dw.grad = grad;
    dw.nrhs = nrhs;
    dw.sweep = sweep && !grad;
    dw.nodes = vt.n_nmid + 2 * NGL * vt.n_npan;
    dw.pending = dw.sweep || far;
    if (!far) return;
    f[LMFMM_K_P2M] = (double)ns * (60.0 * lf.P + 8.0 * lf.nc * nrhs);
    if (grad) f[LMFMM_K_L2P] = (double)nt * (60.0 * (lf.P + 1) + 3.0 * 8.0 * (lf.nc + 2) * nrhs);
    dw.cls.assign(MAXLEV + 1, std::vector<int>());
    for (int l = g.ltop; l <= g.L; ++l) dw.cls[l] = vt.lt[l].clsof_host;
    dw.ev = p->last_ev;
    if (!dw.ev.on || grad) {
        dw.ev = EvalLevels();
        dw.ev.L = g.L;
        dw.ev.P[g.L] = lf.P;
    }
    for (int l = 0; l <= MAXLEV; ++l) dw.rows_l2l[l] = p->last_ev.on && !grad ? p->last_rows_l2l[l] : -1;
}

// Completes the work counts of the last apply from its leaf populations
// (reads the leaf ranges back; synchronizes the device).
static void resolve_work(lmfmm_plan_s *p)
{
    auto &dw = p->dw;
    if (!dw.pending) return;
    dw.pending = false;
    const Geometry &g = dw.g;
    const int L = g.L, ltop = g.ltop;
    const Level &lf = g.lev[L];
    const int64_t nbs = (int64_t)lf.rows_s * lf.ncol, nbt = (int64_t)lf.rows_t * lf.ncol;
    if (nbs + nbt <= 0 || !dw.start || !dw.end) return;
    std::vector<int32_t> st(nbs + nbt), en(nbs + nbt);
    if (hipDeviceSynchronize() != hipSuccess) return;
    if (hipMemcpy(st.data(), dw.start, (nbs + nbt) * 4, hipMemcpyDeviceToHost) != hipSuccess) return;
    if (hipMemcpy(en.data(), dw.end, (nbs + nbt) * 4, hipMemcpyDeviceToHost) != hipSuccess) return;
    auto cnt_s = [&](int64_t b) { return (int64_t)en[b] - st[b]; };
    auto cnt_t = [&](int64_t b) { return (int64_t)en[nbs + b] - st[nbs + b]; };
    double *f = p->stats.kernel_flops;
    const double R = dw.nrhs;
    if (dw.sweep && lf.ncol > 0) {
        // points of the row-0 leaves of both sides
        int64_t n0 = 0;
        for (int c = 0; c < lf.ncol; ++c) {
            if (lf.rows_s > 0) n0 += cnt_s(c);
            if (lf.rows_t > 0) n0 += cnt_t(c);
        }
        f[LMFMM_K_SWEEP] = (double)n0 * dw.nodes * 2.0 * (32.0 + 8.0 * R);
    }
    if (!dw.far) return;
    // occupancy of every box of the expansion levels (row-major, rows from
    // the interface; a parent holds points if any child does)
    std::vector<std::vector<char>> os(MAXLEV + 1), ot(MAXLEV + 1);
    os[L].resize(nbs);
    ot[L].resize(nbt);
    for (int64_t b = 0; b < nbs; ++b) os[L][b] = cnt_s(b) > 0;
    for (int64_t b = 0; b < nbt; ++b) ot[L][b] = cnt_t(b) > 0;
    for (int l = L - 1; l >= ltop; --l) {
        const Level &c = g.lev[l + 1], &pa = g.lev[l];
        os[l].assign((size_t)pa.rows_s * pa.ncol, 0);
        ot[l].assign((size_t)pa.rows_t * pa.ncol, 0);
        for (int r = 0; r < c.rows_s; ++r)
            for (int b = 0; b < c.ncol; ++b)
                if (os[l + 1][(size_t)r * c.ncol + b]) os[l][(size_t)(r >> 1) * pa.ncol + ((c.col_lo + b) >> 1) - pa.col_lo] = 1;
        for (int r = 0; r < c.rows_t; ++r)
            for (int b = 0; b < c.ncol; ++b)
                if (ot[l + 1][(size_t)r * c.ncol + b]) ot[l][(size_t)(r >> 1) * pa.ncol + ((c.col_lo + b) >> 1) - pa.col_lo] = 1;
    }
    f[LMFMM_K_M2M] = 0;
    for (int l = L; l >= ltop + 1; --l) {
        const Level &c = g.lev[l], &pa = g.lev[l - 1];
        int64_t n = 0;
        for (char v : os[l]) n += v;
        f[LMFMM_K_M2M] += 8.0 * R * (double)n * c.nc * pa.nc;
    }
    f[LMFMM_K_DOWN] = 0;
    int64_t pairs = 0;
    for (int l = ltop; l <= L; ++l) {
        const Level &lv = g.lev[l];
        const std::vector<int> &c3 = dw.cls[l];
        int64_t cnt = 0;
        for (size_t sl = 0; sl + 2 < c3.size(); sl += 3) {
            const int rt = c3[sl], rs = c3[sl + 1], dc = c3[sl + 2];
            if (rt >= lv.rows_t || rs >= lv.rows_s) continue;
            for (int b = 0; b < lv.ncol; ++b) {
                const int col = lv.col_lo + b, cs = col + dc, csl = cs - lv.col_lo;
                if (csl < 0 || csl >= lv.ncol) continue;
                const int dp = (cs >> 1) - (col >> 1);
                if (l != ltop && (dp < -1 || dp > 1)) continue;
                if (ot[l][(size_t)rt * lv.ncol + b] && os[l][(size_t)rs * lv.ncol + csl]) ++cnt;
            }
        }
        pairs += cnt;
        f[LMFMM_K_DOWN] += 8.0 * R * (double)cnt * lv.nc * lv.nc;
    }
    p->stats.m2l_pairs = pairs;
    // L2L: the target boxes shifted (levels below ltop; the leaf level's
    // shift is counted with the leaf evaluation, except in the gradient form)
    f[LMFMM_K_L2L] = 0;
    for (int l = ltop + 1; l <= L; ++l) {
        if (l == L && !dw.grad) break;
        const Level &lv = g.lev[l], &pa = g.lev[l - 1];
        const int rows = dw.rows_l2l[l] >= 0 ? std::min(dw.rows_l2l[l], lv.rows_t) : lv.rows_t;
        int64_t n = 0;
        for (int64_t b = 0; b < (int64_t)rows * lv.ncol; ++b) n += ot[l][b];
        f[LMFMM_K_L2L] += 8.0 * R * (double)n * pa.nc * lv.nc;
    }
    if (dw.grad) return;
    // the leaf evaluation: per target, the basis and contraction of the
    // expansion it evaluates, plus the shift of each occupied leaf that
    // evaluates its own expansion
    const EvalLevels &ev = dw.ev;
    const int ncs = L > ltop ? g.lev[L - 1].nc : 0;
    double fl = 0.0;
    for (int r = 0; r < lf.rows_t; ++r) {
        const int e = eval_level(ev, r), P = ev.P[e];
        for (int c = 0; c < lf.ncol; ++c) {
            const int64_t n = cnt_t((int64_t)r * lf.ncol + c);
            if (n <= 0) continue;
            fl += (double)n * (60.0 * P + 8.0 * (2 * P + 1) * R);
            if (e == L && ncs) fl += 8.0 * R * ncs * lf.nc;
        }
    }
    f[LMFMM_K_L2P] = fl;
}

// One pass of Algorithm 1 for the operator of orientation adj (0: forward,
// 1: transposed in mirrored coordinates).  With gw == nullptr the field of the
// densities q is written to u; otherwise the target-side coordinate gradient of
// Re sum gw * field is written to gout ([2][nt], y component times ysign).
template <typename T>
// fixed_ws: the allocation-free form (lmfmm_apply_noalloc): the workspace is
// that fixed array of NOALLOC_SCRATCH_BYTES, the tables must already exist,
// every kernel is launched directly, and the statistics are not updated.
static int apply_impl(lmfmm_plan p, int adj, int64_t ns, const double *src, const void *q, int64_t nt,
                      const double *tgt, void *u, int nrhs, hipStream_t st, const void *gw = nullptr,
                      double *gout = nullptr, double ysign = 1.0, void *fixed_ws = nullptr)
{
    if (nt == 0) return LMFMM_OK;
    int rc;
    if (ns == 0) {
        if (gw)
            launch_zero_bytes(gout, (size_t)2 * nt * sizeof(double), st);
        else
            launch_zero_bytes(u, (size_t)nt * nrhs * sizeof(cx<T>), st);
        HIPCHK(hipGetLastError());
        return LMFMM_OK;
    }
    Medium med = p->med;
    med.adj = adj;
    VarTables &vt = p->vt[adj];
    collect_timing(p);
    // event before each timed kernel (group); tag -1 closes the last interval
    // timed kernel: its start/stop events ride on its own launch; a group
    // (bounding box and tree build) is bracketed by recorded events
    auto timed = [&](int tag, int nl) {
        if (!p->timing || p->ev_n >= lmfmm_plan_s::NEV / 2) return;
        const int j = p->ev_n;
        p->ev_tag[j] = tag;
        p->ev_nl[j] = nl;
        launch_timing() = {p->ev[2 * j], p->ev[2 * j + 1]};
    };
    auto timed_done = [&]() {  // after the launcher: keep the entry only if a kernel took the events
        LaunchTiming &lt = launch_timing();
        if (!p->timing || p->ev_n >= lmfmm_plan_s::NEV / 2) return;
        if (lt.start)
            lt = LaunchTiming{};
        else
            ++p->ev_n;
    };
    auto group_begin = [&](int tag, hipStream_t sx) {
        if (!p->timing || p->ev_n >= lmfmm_plan_s::NEV / 2) return;
        p->ev_tag[p->ev_n] = tag;
        p->ev_nl[p->ev_n] = 0;
        (void)hipEventRecord(p->ev[2 * p->ev_n], sx);
    };
    auto group_end = [&](int nl, hipStream_t sx) {
        if (!p->timing || p->ev_n >= lmfmm_plan_s::NEV / 2) return;
        p->ev_nl[p->ev_n] = nl;
        (void)hipEventRecord(p->ev[2 * p->ev_n + 1], sx);
        ++p->ev_n;
    };
    const bool have_bb = p->have_domain || (p->have_box && !adj);
    // arguments, options, tables and workspace that a captured graph bakes in
    // besides the geometry
    const bool graph_ok = p->use_graph && !p->timing && !fixed_ws;
    // (built for every apply but the allocation-free one, which uses no key:
    // the key code below writes entries 12-14)
    std::vector<uint64_t> prekey;
    if (!fixed_ws) {
        auto put = [&](uint64_t v) { prekey.push_back(v); };
        auto putp = [&](const void *ptr) { put((uint64_t)(uintptr_t)ptr); };
        uint64_t ys_bits;
        std::memcpy(&ys_bits, &ysign, 8);
        put(sizeof(T));
        put((uint64_t)adj);
        putp(src);
        putp(q);
        putp(tgt);
        putp(u);
        putp(gw);
        putp(gout);
        put(ys_bits);
        put((uint64_t)ns);
        put((uint64_t)nt);
        put((uint64_t)nrhs);
        putp(p->ws.p);
        put(p->ws.gen);
        put(vt.version);
        put(p->cfg_version);
    }
    double bb[8];
    bool bb_known = false;
    if (!have_bb && graph_ok && p->gexec && p->g_bbox && prekey == p->g_prekey && p->tz_gen == p->ws.gen &&
        p->tz_bytes >= p->g_zero_bytes) {
        // speculative replay: launch, then compare the box it computed
        HIPCHK(hipGraphLaunch(p->gexec, st));
        ++p->bbox_seq;
        if ((rc = bbox_wait(p, st, bb))) return rc;
        if (std::memcmp(bb, p->g_bb, sizeof p->g_bb) == 0) {
            p->stats.graph_applies++;
            return LMFMM_OK;  // same box, same geometry: the statistics stand
        }
        bb_known = true;  // another box: compute again below (the replay's results are overwritten)
        p->g_prekey.clear();  // and no more speculation until a graph is captured or matched again
    }
    group_begin(LMFMM_K_TREE, st);
    if (!bb_known && (rc = get_bbox(p, med, ns, src, nt, tgt, st, bb))) return rc;
    Geometry &g = p->geo;
    if ((rc = make_geometry(p, bb, ns, nrhs, g))) return rc;
    const int L = g.L;
    if (g.lev[L].P > 255) return fail(LMFMM_EINVAL, "leaf-level expansion order above 255: use more levels");
    bool far = p->do_far && L >= 2;
    if (far && (rc = ensure_far_tables(vt, med, g, !fixed_ws))) return rc;
    double amin = std::max(bb[2], 0.0) + std::max(-bb[5], 0.0);
    if (!(amin > 0)) amin = 1e-9 * g.W;
    if ((rc = ensure_near_table(vt, med, g, amin, !fixed_ws))) return rc;

    // workspace
    const Level &lv = g.lev[L];
    int64_t n = ns + nt;
    int64_t nbox = (int64_t)(lv.rows_s + lv.rows_t) * lv.ncol;
    size_t need = 0;
    need += 6 * (size_t)n * 4 + (size_t)tree_table_len(n) * 4 + 3 * (size_t)nbox * 4 + 2 * (size_t)n * 8 + 2 * 256;
    need += (size_t)ns * nrhs * sizeof(cx<T>) + 256;  // densities in grouped order
    need += ((size_t)g.ncoef_s + (size_t)g.ncoef_t) * sizeof(cx<T>) + 64 + 20 * 256;
    need += (size_t)g.nocc_s * 4 + 256;
    const int ltop = g.ltop;
    // near-field sweep results: up to 4 node parts x nrhs x targets (FP64)
    // direct interactions exist only between row-0 leaves on both sides
    const bool near_on = p->do_near && !(bb[2] >= lv.w) && !(bb[5] <= -lv.w);
    const bool sweep = near_on && p->near_sweep && !gw;
    int64_t nun = sweep ? (int64_t)4 * nrhs * nt : 0;
    need += (size_t)nun * sizeof(cx<double>) + 256;
    if (fixed_ws) {
        if (need > NOALLOC_SCRATCH_BYTES)
            return fail(LMFMM_EINVAL, "this apply needs " + std::to_string(need) +
                                          " bytes of workspace; the allocation-free apply has " +
                                          std::to_string(NOALLOC_SCRATCH_BYTES));
    } else if ((rc = p->ws.ensure(need))) {
        return rc;
    }
    Carve cv{fixed_ws ? (char *)fixed_ws : (char *)p->ws.p};
    TreeBufs tb;
    // error flags and the counting sort's leaf counters first: this prefix
    // must hold zeros when a tree build starts (every build leaves it so)
    int32_t *err = cv.take<int32_t>(2);
    tb.cnt = cv.take<int32_t>(nbox);
    const size_t zero_bytes = cv.off;
    tb.tab = cv.take<int32_t>(tree_table_len(n));
    tb.key = cv.take<uint32_t>(n);
    tb.rank = cv.take<int32_t>(n);
    tb.perm = cv.take<int32_t>(n);
    tb.scratch = cv.take<int32_t>(2 * n);
    tb.idx = cv.take<int32_t>(n);
    tb.start = cv.take<int32_t>(nbox);
    tb.end = cv.take<int32_t>(nbox);
    tb.xs = cv.take<double>(n);
    tb.ys = cv.take<double>(n);
    tb.q = reinterpret_cast<const uint64_t *>(q);
    tb.qs = cv.take<uint64_t>((size_t)ns * nrhs * (sizeof(cx<T>) / 8));
    tb.nrhs = nrhs;
    tb.qw = (int)(sizeof(cx<T>) / 8);
    int32_t *start = tb.start, *end = tb.end, *idx = tb.idx;
    double *xs = tb.xs, *ys = tb.ys;
    cx<T> *M = cv.take<cx<T>>(g.ncoef_s > 0 ? g.ncoef_s : 1);
    cx<T> *Lc = cv.take<cx<T>>(g.ncoef_t > 0 ? g.ncoef_t : 1);
    int32_t *occ = cv.take<int32_t>(g.nocc_s > 0 ? g.nocc_s : 1);
    p->d_err = err;
    p->err_valid = n > 0 && nbox > 0;
    cx<double> *unear = sweep ? cv.take<cx<double>>(nun) : nullptr;
    const bool radix = tree_radix(n, p->tree_sort);
    int tree_launches = (have_bb ? 0 : 2) + tree_launch_count(nbox, radix);
    if (fixed_ws) {
        // the fixed array is shared by every plan on this device: clear the
        // counters every time
        set_stage(S_ZERO);
        launch_zero_bytes(fixed_ws, zero_bytes, st);
        ++tree_launches;
    } else {
        if (p->tz_gen != p->ws.gen || zero_bytes > p->tz_bytes) {
            set_stage(S_ZERO);
            launch_zero_bytes(p->ws.p, zero_bytes, st);
            ++tree_launches;
            p->tz_gen = p->ws.gen;
        }
        // past this apply's counters its other buffers begin: only its own
        // counter range is known to be zero afterwards
        p->tz_bytes = zero_bytes;
    }

    // the launch sequence (Steps 1-4) on stream sx
    auto launch_all = [&](hipStream_t sx, bool with_bbox) {
        // Step 1: tree (in a graph of the device-computed box, the box first)
        if (with_bbox) bbox_launch(p, med, ns, src, nt, tgt, sx);
        set_stage(S_TREE);
        launch_tree(src, ns, tgt, nt, g.x_lo, lv.w, lv.col_lo, lv.ncol, lv.rows_s, lv.rows_t, layers_of(med), tb,
                    err, radix, sx);
        group_end(tree_launches, sx);

        // Step 2: upward pass
        LeafShift<T> shift;
        // The leaf evaluation reads each leaf's expansion at the level where
        // its far field is complete (the sweep or no near field: the packed
        // evaluation kernel); the gradient and pairwise forms read the leaves'
        // own expansions.
        EvalLevels ev;
        int rows_l2l[MAXLEV + 1] = {};
        const bool eval_on = far && !gw && (sweep || !near_on || lv.rows_s == 0) && p->eval_levels;
        if (far) {
            timed(LMFMM_K_P2M, 1);
            set_stage(S_P2M);
            launch_p2m<T>(start, end, xs, ys, tb.qs, ns, nrhs, g, med, M, occ, p->p2m_series, sx);
            timed_done();
            for (int l = L; l >= ltop + 1; --l) {
                const LevelTables &tb = vt.lt[l];
                const cx<T> *tab = (const cx<T> *)(sizeof(T) == 8 ? tb.m2m64.p : tb.m2m32.p);
                timed(LMFMM_K_M2M, 1);
                set_stage(S_M2M, L - l);
                launch_m2m<T>(g, l, tab, M, occ, nrhs, p->shift_mfma, sx);
                timed_done();
            }
            // Step 3: downward pass.  M2L of every level in one launch (the
            // coarsest level between all its non-adjacent boxes), stored as the
            // local expansions of the interface rows; then level by level the
            // L2L shift of the parent's expansion, adding the stored M2L.
            const cx<T> *atab[MAXLEV + 1] = {};
            const int *cls3[MAXLEV + 1] = {}, *roff[MAXLEV + 1] = {};
            int nrt[MAXLEV + 1] = {0};
            for (int l = ltop; l <= L; ++l) {
                const LevelTables &tl = vt.lt[l];
                if (tl.nslots == 0) continue;
                atab[l - ltop] = (const cx<T> *)(sizeof(T) == 8 ? tl.a64.p : tl.a32.p);
                cls3[l - ltop] = (const int *)tl.clsof.p;
                roff[l - ltop] = (const int *)tl.rowoff.p;
                nrt[l - ltop] = std::min(tl.nrt, g.lev[l].rows_t);
            }
            if (!atab[0]) {
                // coarsest level without translation classes: no far field reaches it
                const Level &lt = g.lev[ltop];
                set_stage(S_ZTOP);
                launch_zero_bytes(Lc + lt.off_t, (size_t)lt.rows_t * lt.ncol * nrhs * lt.nc * sizeof(cx<T>), sx);
            }
            for (int part = 1; part <= 2; ++part) {
                timed(LMFMM_K_DOWN, 1);
                set_stage(S_M2L, part);
                // the matrix-core form pays from 4 right-hand sides (FP32) or 3
                // (FP64) on; with fewer its 16-column tiles are mostly boxes
                // whose tables differ little in cost from the vector form's
                const bool mf = p->m2l_mfma < 0 ? nrhs >= (sizeof(T) == 8 ? 3 : 4) : p->m2l_mfma != 0;
                launch_m2l_all<T>(g, ltop, L, atab, cls3, roff, nrt, M, Lc, nrhs, mf, occ, part, sx);
                timed_done();
            }
            // the leaf level's shift is done by the leaf evaluation (forward apply)
            const int l2l_last = (!gw && L > ltop) ? L - 1 : L;
            if (eval_on) {
                // Levels down to lc (the coarsest whose order is within two of
                // the leaves') are shifted in every row; below it only the
                // rows whose expansion is read: those with M2L classes, and
                // the parents of the rows shifted one level finer.  A leaf
                // evaluates at lc or at the finest level where its ancestor
                // has M2L classes, if finer.
                int lc = L;
                for (int l = ltop; l <= L; ++l)
                    if (g.lev[l].P <= g.lev[L].P + 2) {
                        lc = l;
                        break;
                    }
                ev.on = 1;
                ev.lc = lc;
                ev.L = L;
                int need = L > ltop ? nrt[L - ltop] : 0;
                for (int l = L; l >= ltop; --l) {
                    const Level &lv2 = g.lev[l];
                    ev.nrt[l] = l <= lc ? lv2.rows_t : nrt[l - ltop];
                    ev.P[l] = lv2.P;
                    ev.ncol[l] = lv2.ncol;
                    ev.off[l] = lv2.off_t;
                    if (l < L) need = std::max(ev.nrt[l], (need + 1) >> 1);
                    rows_l2l[l] = l <= lc ? -1 : (l == L ? nrt[L - ltop] : need);
                }
            }
            if (l2l_last < L) {
                const LevelTables &tl = vt.lt[L];
                const Level &pv = g.lev[L - 1];
                shift.tab = (const cx<T> *)(sizeof(T) == 8 ? tl.l2l64.p : tl.l2l32.p);
                shift.Lp = Lc + pv.off_t;
                shift.ncp = pv.nc;
                shift.ncol_p = pv.ncol;
                shift.col_lo_p = pv.col_lo;
                shift.rows_p = pv.rows_t;
                shift.add_rows = nrt[L - ltop];
            }
            for (int l = ltop + 1; l <= l2l_last; ++l) {
                const LevelTables &tl = vt.lt[l];
                const cx<T> *l2l = (const cx<T> *)(sizeof(T) == 8 ? tl.l2l64.p : tl.l2l32.p);
                timed(LMFMM_K_L2L, 1);
                set_stage(S_L2L, l - ltop - 1);
                launch_down<T>(g, l, (const cx<T> *)nullptr, nullptr, nullptr, 0, M, Lc, nrhs, l2l, false,
                               nrt[l - ltop], sx, eval_on ? rows_l2l[l] : -1, p->shift_mfma);
                timed_done();
            }
        }
        p->last_ev = ev;
        for (int l = 0; l <= MAXLEV; ++l) p->last_rows_l2l[l] = rows_l2l[l];
        // Step 4: local evaluation and direct interactions
        const Node *nnodes = (const Node *)vt.near_nodes.p;
        int nparts = 0;
        if (!gw) {
            if (sweep) {
                timed(LMFMM_K_SWEEP, 1);
                set_stage(S_SWEEP);
                nparts = launch_near_sweep<T>(start, end, idx, xs, ys, q, ns, nt, nrhs, g, nnodes, vt.n_nmid, vt.n_npan,
                                              vt.n_t0, unear, sx);
                timed_done();
            }
            timed(LMFMM_K_L2P, 1);
            set_stage(S_L2P);
            launch_l2p_near<T>(start, end, idx, xs, ys, q, ns, nt, nrhs, g, med, Lc, shift, ev, nnodes, vt.n_nmid,
                               vt.n_npan, vt.n_t0, far ? 1 : 0, near_on ? 1 : 0, nparts ? unear : nullptr, nparts, u,
                               sx);
            timed_done();
        } else {
            timed(LMFMM_K_L2P, 1);  // the first right-hand-side chunk
            launch_l2p_grad<T>(start, end, idx, xs, ys, q, gw, ns, nt, nrhs, g, med, Lc, nnodes, vt.n_nmid, vt.n_npan,
                               vt.n_t0, far ? 1 : 0, near_on ? 1 : 0, ysign, gout, sx);
            timed_done();
        }
    };
    if (fixed_ws) {
        launch_all(st, false);
        HIPCHK(hipGetLastError());
        if (p->ev_n > 0 && p->timing) p->ev_pending = true;
        return LMFMM_OK;
    }
    // key of everything the launch sequence bakes into its kernel arguments
    // (the workspace and tables as they are now)
    prekey[12] = (uint64_t)(uintptr_t)p->ws.p;
    prekey[13] = p->ws.gen;
    prekey[14] = vt.version;
    std::vector<uint64_t> key = prekey;
    {
        key.push_back((uint64_t)far | (uint64_t)near_on << 1 | (uint64_t)sweep << 2);
        std::vector<uint64_t> gb((sizeof(Geometry) + 7) / 8, 0);
        std::memcpy(gb.data(), &g, sizeof(Geometry));
        key.insert(key.end(), gb.begin(), gb.end());
    }
    // (timing mode launches kernel by kernel: the events ride on the launches)
    if (graph_ok && p->gexec && key == p->gkey) {
        // replay (the bounding-box kernel inside runs again)
        HIPCHK(hipGraphLaunch(p->gexec, st));
        if (p->g_bbox) {
            ++p->bbox_seq;
            std::memcpy(p->g_bb, bb, sizeof p->g_bb);
            p->g_prekey = prekey;
        }
        p->stats.graph_applies++;
    } else if (graph_ok && key == p->last_key) {
        // second apply with this key: capture it on the plan's stream and replay
        if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->gexec = nullptr;
        p->graph = nullptr;
        p->gkey.clear();
        p->g_bbox = false;
        if (!p->cap) HIPCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
        bool ok = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            launch_all(p->cap, !have_bb);
            hipGraph_t gr = nullptr;
            ok = hipStreamEndCapture(p->cap, &gr) == hipSuccess && gr;
            if (ok) ok = hipGraphInstantiate(&p->gexec, gr, nullptr, nullptr, 0) == hipSuccess;
            if (ok) {
                p->graph = gr;
                p->gkey = key;
                p->g_bbox = !have_bb;
                std::memcpy(p->g_bb, bb, sizeof p->g_bb);
                p->g_prekey = prekey;
                p->g_zero_bytes = zero_bytes;
            } else {
                if (gr) (void)hipGraphDestroy(gr);
                p->gexec = nullptr;
            }
        }
        (void)hipGetLastError();
        if (ok) {
            HIPCHK(hipGraphLaunch(p->gexec, st));
            if (p->g_bbox) ++p->bbox_seq;
            p->stats.graph_applies++;
        } else {
            // capture is not available here: stay with direct launches for this key
            p->use_graph = false;
            launch_all(st, false);
        }
    } else {
        p->last_key = key;
        launch_all(st, false);
    }
    if (hipPeekAtLastError() != hipSuccess) p->tz_bytes = 0;  // counters in an unknown state: zero them again
    HIPCHK(hipGetLastError());
    if (p->ev_n > 0 && p->timing) p->ev_pending = true;

    // statistics (host-side counts)
    lmfmm_stats &s = p->stats;
    s.levels = L;
    for (int l = 0; l < 32; ++l) s.order[l] = l <= L ? g.lev[l].P : 0;
    s.root_x_lo = g.x_lo;
    s.root_width = g.W;
    s.leaves_src = (int64_t)lv.rows_s * lv.ncol;
    s.leaves_tgt = (int64_t)lv.rows_t * lv.ncol;
    s.near_nodes_mid = vt.n_nmid;
    s.near_nodes_ray = vt.n_npan * NGL;
    int ncls = 0;
    int64_t nn = 0;
    for (int l = ltop; l <= L && far; ++l) {
        ncls += vt.lt[l].nslots;
        nn += vt.lt[l].nodes;
    }
    s.m2l_classes = ncls;
    s.m2l_nodes = nn;
    s.table_seconds = vt.table_seconds;
    count_flops(p, vt, g, far, ns, nt, nrhs, gw != nullptr, sweep, start, end);
    return LMFMM_OK;
}

// Mirrored copies (x, -y) of both point sets for the transposed operator:
// the targets become its sources and the sources its targets.
static int mirror_points(lmfmm_plan p, int64_t ns, const double *src, int64_t nt, const double *tgt,
                         hipStream_t st, double *&msrc, double *&mtgt)
{
    int rc = p->mirror.ensure((size_t)2 * (ns + nt) * sizeof(double) + 512);
    if (rc) return rc;
    mtgt = (double *)p->mirror.p;             // mirrored original sources: targets of G^T
    msrc = mtgt + 2 * ns;                     // mirrored image targets: sources of G^T
    double a, b;
    image_map(p->med, a, b);
    launch_mirror(src, ns, 1.0, 0.0, mtgt, st);
    launch_mirror(tgt, nt, a, b, msrc, st);
    HIPCHK(hipGetLastError());
    return LMFMM_OK;
}

extern "C" {

int lmfmm_apply(lmfmm_plan p, int64_t ns, const double *src, const void *q, int64_t nt, const double *tgt, void *u,
                int nrhs, int prec, void *stream)
{
    int rc = check_common(p, ns, src, nt, tgt, q, u, nrhs, prec);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    return prec == LMFMM_C128 ? apply_impl<double>(p, 0, ns, src, q, nt, tgt, u, nrhs, st)
                              : apply_impl<float>(p, 0, ns, src, q, nt, tgt, u, nrhs, st);
}

int lmfmm_apply_noalloc(lmfmm_plan p, int64_t ns, const double *src, const void *q, int64_t nt, const double *tgt,
                        void *u, int nrhs, int prec, void *stream)
{
    int rc = check_common(p, ns, src, nt, tgt, q, u, nrhs, prec);
    if (rc) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(LMFMM_EINVAL, "the plan's device must be current");
    void *ws = noalloc_scratch_ptr(dev);
    if (!ws) return fail(LMFMM_EHIP, "the device address of the allocation-free apply's array is not resolved");
    hipStream_t st = (hipStream_t)stream;
    return prec == LMFMM_C128 ? apply_impl<double>(p, 0, ns, src, q, nt, tgt, u, nrhs, st, nullptr, nullptr, 1.0, ws)
                              : apply_impl<float>(p, 0, ns, src, q, nt, tgt, u, nrhs, st, nullptr, nullptr, 1.0, ws);
}

int lmfmm_direct(lmfmm_plan p, int64_t ns, const double *src, const void *q, int64_t nt, const double *tgt, void *u,
                 int nrhs, int prec, void *stream)
{
    int rc = check_common(p, ns, src, nt, tgt, q, u, nrhs, prec);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nt == 0) return LMFMM_OK;
    if (ns == 0) {
        launch_zero_bytes(u, (size_t)nt * nrhs * (prec == LMFMM_C128 ? 16 : 8), st);
        return LMFMM_OK;
    }
    bool saved = p->have_domain;
    p->have_domain = false;
    double bb[8];
    rc = get_bbox(p, p->med, ns, src, nt, tgt, st, bb);
    p->have_domain = saved;
    if (rc) return rc;
    double dxmax = std::max(bb[1] - bb[0], 1e-12);
    double amin = std::max(bb[2], 0.0) + std::max(-bb[5], 0.0);
    double c = contour_c(p->med), h = std::min(0.25 * c, 3.0 / dxmax), t0 = ray_t0(c, dxmax);
    double ar = std::max(amin, 1e-12) / std::sqrt(2.0);
    int npan = std::min(64, 2 + (int)std::ceil(std::log2(std::max(2.0, 40.0 / (ar * t0)))));
    if (!p->dir_nodes.p || p->d_h != h || p->d_t0 != t0 || p->d_npan < npan) {
        double cc, hh, tt;
        int nm, np;
        if ((rc = build_near_table(p->dir_nodes, p->med, dxmax, amin, cc, hh, tt, nm, np))) return rc;
        p->d_h = hh;
        p->d_nmid = nm;
        p->d_npan = np;
        p->d_t0 = tt;
    }
    const int nchunk = direct_chunks(ns, nt, nrhs);
    if (nchunk > 1 && (rc = p->dir_part.ensure((size_t)nchunk * nt * nrhs * sizeof(cx<double>)))) return rc;
    double ty_a, ty_b;
    image_map(p->med, ty_a, ty_b);
    launch_direct(src, ns, q, tgt, nt, ty_a, ty_b, nrhs, prec, (const Node *)p->dir_nodes.p, p->d_nmid, p->d_npan,
                  p->d_t0, nchunk, (cx<double> *)p->dir_part.p, u, st);
    HIPCHK(hipGetLastError());
    return LMFMM_OK;
}

int lmfmm_apply_adjoint(lmfmm_plan p, int64_t ns, const double *src, int64_t nt, const double *tgt, const void *w,
                        void *v, int nrhs, int prec, void *stream)
{
    // v has n_src entries per right-hand side and w has n_tgt
    int rc = check_common(p, nt, tgt, ns, src, w, v, nrhs, prec);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (ns == 0) return LMFMM_OK;
    double *msrc = nullptr, *mtgt = nullptr;
    if ((rc = mirror_points(p, ns, src, nt, tgt, st, msrc, mtgt))) return rc;
    return prec == LMFMM_C128 ? apply_impl<double>(p, 1, nt, msrc, w, ns, mtgt, v, nrhs, st)
                              : apply_impl<float>(p, 1, nt, msrc, w, ns, mtgt, v, nrhs, st);
}

int lmfmm_grad_coords(lmfmm_plan p, int64_t ns, const double *src, const void *q, int64_t nt, const double *tgt,
                      const void *w, double *dsrc, double *dtgt, int nrhs, int prec, void *stream)
{
    int rc = check_common(p, ns, src, nt, tgt, q, w, nrhs, prec);
    if (rc) return rc;
    if ((ns > 0 && !dsrc) || (nt > 0 && !dtgt)) return fail(LMFMM_EINVAL, "null gradient output");
    hipStream_t st = (hipStream_t)stream;
    // target coordinates: gradient of the field of q contracted with w (the
    // y derivative in tree coordinates times the image map's slope)
    double ty_a, ty_b;
    image_map(p->med, ty_a, ty_b);
    rc = prec == LMFMM_C128 ? apply_impl<double>(p, 0, ns, src, q, nt, tgt, nullptr, nrhs, st, w, dtgt, ty_a)
                            : apply_impl<float>(p, 0, ns, src, q, nt, tgt, nullptr, nrhs, st, w, dtgt, ty_a);
    if (rc) return rc;
    if (ns == 0) return LMFMM_OK;
    // source coordinates: gradient of the transposed field of w contracted with q,
    // in mirrored coordinates (d/dy0 = -d/dy')
    double *msrc = nullptr, *mtgt = nullptr;
    if ((rc = mirror_points(p, ns, src, nt, tgt, st, msrc, mtgt))) return rc;
    return prec == LMFMM_C128 ? apply_impl<double>(p, 1, nt, msrc, w, ns, mtgt, nullptr, nrhs, st, q, dsrc, -1.0)
                              : apply_impl<float>(p, 1, nt, msrc, w, ns, mtgt, nullptr, nrhs, st, q, dsrc, -1.0);
}

int lmfmm_sync_status(lmfmm_plan p, void *stream)
{
    if (!p) return fail(LMFMM_EINVAL, "plan is null");
    hipStream_t st = (hipStream_t)stream;
    if (p->d_err && p->err_valid) {
        HIPCHK(hipMemcpyAsync(p->h_bbox + 12, p->d_err + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int32_t e;
        std::memcpy(&e, p->h_bbox + 12, sizeof e);
        if (e & 2) return fail(LMFMM_EHIP, "inconsistent grouping in the tree build (results invalid)");
        if (e) return fail(LMFMM_EDOMAIN, "a point lies outside the domain or its layer");
        return LMFMM_OK;
    }
    HIPCHK(hipStreamSynchronize(st));
    return LMFMM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched apply: many independent problems, one launch per stage.
//
// Preparation (first call, or when the instance descriptors change):
//   1. each instance's bounding box is read once and pinned in its plan, so
//      later applies queue no host synchronisation;
//   2. each instance's (order floor, levels) comes from the tuning cache when
//      it holds the instance's key, else the autotuner times every candidate
//      (order floors of the set x levels around the automatic choice) with HIP
//      events and keeps the fastest; the tolerance is met by every candidate
//      (the order rule of the plan enforces it).  New choices are written to
//      the cache;
//   3. one apply per instance builds its tables and workspace; then every
//      instance's launch sequence is recorded instead of launched, and the
//      launches of one stage (zeroing, the four tree passes, P2M, the M2M of
//      each level counted from the leaves, M2L, the L2L of each level counted
//      from the top, near field, local evaluation) become one launch of the
//      kernel's multi-instance form over all instances (instances whose
//      kernels differ in template arguments take separate launches of the
//      stage).  The per-instance arguments go to device memory once;
//   4. the merged sequence is captured in a HIP graph on one stream.
// Every later call with the same descriptors is one hipGraphLaunch.
// ---------------------------------------------------------------------------
struct BatchLaunch {
    const void *fn;  // multi-instance kernel
    dim3 block;
    size_t shmem;
    unsigned nblk;
    int n;
    int cls;  // LMFMM_K_* class of its stage
    size_t off_blk0, off_grid, off_args;
    MultiArgs m;
};

struct TuneEntry {
    int order = 0, levels = 0, sweep = 1;
    double us = 0;
};

struct lmfmm_batch_s {
    int n = 0;
    std::vector<lmfmm_plan_s *> plans;
    std::vector<int> order_set;
    double tol = 1e-6;
    bool tune = true, graph = true;
    bool tune_near = true;  // the tuner also picks the near-field form (cleared when the caller sets it)
    std::string cache_path;  // tuning cache (one JSON object per line); empty: none
    // prepared state
    bool prepared = false;
    std::vector<lmfmm_instance> desc;
    int nrhs = 0, prec = -1;
    std::vector<BatchLaunch> seq;
    DevBuf meta;  // blk0, grid and argument arrays of every merged launch
    hipStream_t cap_stream = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    std::vector<int> chosen_order, chosen_levels, from_cache;
    std::vector<double> chosen_us;
    lmfmm_batch_stats stats;
    // per-launch timing
    bool timing = false, ev_pending = false;
    std::vector<hipEvent_t> ev;
};

static void batch_drop_graph(lmfmm_batch_s *b)
{
    if (b->ge) (void)hipGraphExecDestroy(b->ge);
    if (b->g) (void)hipGraphDestroy(b->g);
    b->ge = nullptr;
    b->g = nullptr;
    b->prepared = false;
}

static void batch_collect_timing(lmfmm_batch_s *b)
{
    if (!b->ev_pending) return;
    b->ev_pending = false;
    const size_t n = b->seq.size();
    if (b->ev.size() < 2 * n || n == 0) return;
    (void)hipEventSynchronize(b->ev[2 * n - 1]);
    for (size_t j = 0; j < n; ++j) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b->ev[2 * j], b->ev[2 * j + 1]) == hipSuccess)
            b->stats.kernel_ms[b->seq[j].cls] += ms;
        b->stats.kernel_launches[b->seq[j].cls] += 1;
    }
    b->stats.timed_applies += 1;
}

// the merged sequence on stream s (with start/stop events per launch when timed)
static int batch_launch_seq(lmfmm_batch_s *b, hipStream_t s, bool timed)
{
    for (size_t j = 0; j < b->seq.size(); ++j) {
        BatchLaunch &L = b->seq[j];
        void *args[] = {&L.m};
        hipError_t e = timed ? hipExtLaunchKernel(L.fn, dim3(L.nblk), L.block, args, L.shmem, s, b->ev[2 * j],
                                                  b->ev[2 * j + 1], 0)
                             : hipLaunchKernel(L.fn, dim3(L.nblk), L.block, args, L.shmem, s);
        if (e != hipSuccess) return fail(LMFMM_EHIP, std::string("batched launch: ") + hipGetErrorString(e));
    }
    return LMFMM_OK;
}

static int plan_apply_any(lmfmm_plan_s *p, const lmfmm_instance &in, int nrhs, int prec, hipStream_t st)
{
    return prec == LMFMM_C128 ? apply_impl<double>(p, 0, in.n_src, in.src_xy, in.q, in.n_tgt, in.tgt_xy, in.u, nrhs, st)
                              : apply_impl<float>(p, 0, in.n_src, in.src_xy, in.q, in.n_tgt, in.tgt_xy, in.u, nrhs, st);
}

static bool same_desc(const lmfmm_instance &a, const lmfmm_instance &b)
{
    return a.n_src == b.n_src && a.src_xy == b.src_xy && a.q == b.q && a.n_tgt == b.n_tgt && a.tgt_xy == b.tgt_xy &&
           a.u == b.u;
}

// Tuning-cache key of an instance: medium, sizes (in half-octave buckets),
// tolerance, right-hand sides, precision and the candidate order set.
static std::string tune_key(const lmfmm_batch_s *b, const lmfmm_plan_s *p, const lmfmm_instance &in, int nrhs,
                            int prec)
{
    char buf[512];
    auto bucket = [](int64_t n) { return (int)std::floor(2.0 * std::log2((double)std::max<int64_t>(n, 1))); };
    std::snprintf(buf, sizeof buf, "k=%.9g,%.9g,%.9g,%.9g,%.9g,%.9g d=%.9g ns=%d nt=%d tol=%.3g nrhs=%d prec=%d o=",
                  p->med.k1.re, p->med.k1.im, p->med.k2.re, p->med.k2.im, p->med.k3.re, p->med.k3.im, p->med.d,
                  bucket(in.n_src), bucket(in.n_tgt), b->tol, nrhs, prec);
    std::string k(buf);
    for (int o : b->order_set) k += std::to_string(o) + ":";
    return k;
}

static void read_tune_cache(const std::string &path, std::map<std::string, TuneEntry> &out)
{
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        // {"key": "<key>", "order": o, "levels": L, "us": t, "sweep": 0/1 (optional, default 1)}
        const char *k0 = std::strstr(line, "\"key\": \"");
        if (!k0) continue;
        k0 += 8;
        const char *k1 = std::strchr(k0, '"');
        if (!k1) continue;
        TuneEntry e;
        // the text after a field's name (null if the field is absent)
        auto field = [&](const char *name) -> const char * {
            const char *f = std::strstr(k1, name);
            return f ? f + std::strlen(name) : nullptr;
        };
        const char *o = field("\"order\": "), *l = field("\"levels\": "), *u = field("\"us\": ");
        if (!o || !l || !u) continue;
        e.order = std::atoi(o);
        e.levels = std::atoi(l);
        e.us = std::atof(u);
        if (const char *sw = field("\"sweep\": ")) e.sweep = std::atoi(sw) != 0;
        if (e.order < 1 || e.order > 256 || e.levels < 1 || e.levels > MAXLEV) continue;
        out[std::string(k0, k1)] = e;
    }
    std::fclose(f);
}

static void write_tune_cache(const std::string &path, const std::map<std::string, TuneEntry> &m)
{
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto &kv : m)
        std::fprintf(f, "{\"key\": \"%s\", \"order\": %d, \"levels\": %d, \"us\": %.3f, \"sweep\": %d}\n",
                     kv.first.c_str(), kv.second.order, kv.second.levels, kv.second.us, kv.second.sweep);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path.c_str());
}

static int stage_class(int key)
{
    switch (key / 64) {
    case S_ZERO:
    case S_TREE: return LMFMM_K_TREE;
    case S_P2M: return LMFMM_K_P2M;
    case S_M2M: return LMFMM_K_M2M;
    case S_ZTOP:
    case S_M2L: return LMFMM_K_DOWN;
    case S_L2L: return LMFMM_K_L2L;
    case S_SWEEP: return LMFMM_K_SWEEP;
    case S_L2P: return LMFMM_K_L2P;
    default: return LMFMM_K_OTHER;
    }
}

// Record every instance's launch sequence and merge it by stage (see above).
static int batch_record_merge(lmfmm_batch_s *b, const lmfmm_instance *inst, int nrhs, int prec, hipStream_t st)
{
    struct Rec {
        int inst;
        RecLaunch L;
    };
    std::vector<Rec> all;
    int64_t tot_src = 0, tot_all = 0;
    for (int i = 0; i < b->n; ++i) {
        tot_src += inst[i].n_src;
        tot_all += inst[i].n_src + inst[i].n_tgt;
    }
    launch_batch_points() = tot_src;
    launch_batch_all_points() = tot_all;
    for (int i = 0; i < b->n; ++i) {
        lmfmm_plan_s *p = b->plans[i];
        if (inst[i].n_tgt == 0 || inst[i].n_src == 0) continue;  // (no sources: zeroed by the apply)
        Recorder rec;
        const bool timing = p->timing;
        p->timing = false;
        // (no clearing launch is recorded while the plan's counters are known to
        // be zero: the warm apply of the preparation left them so, and every
        // tree build, replays included, leaves them zero)
        launch_recorder() = &rec;
        int rc = plan_apply_any(p, inst[i], nrhs, prec, st);
        launch_recorder() = nullptr;
        p->timing = timing;
        if (rc) {
            launch_batch_points() = 0;
            launch_batch_all_points() = 0;
            return rc;
        }
        for (auto &L : rec.v) all.push_back(Rec{i, std::move(L)});
    }
    launch_batch_points() = 0;
    launch_batch_all_points() = 0;
    std::stable_sort(all.begin(), all.end(), [](const Rec &a, const Rec &c) {
        if (a.L.key != c.L.key) return a.L.key < c.L.key;
        return std::less<const void *>()(a.L.multi, c.L.multi);
    });
    b->seq.clear();
    std::vector<char> host;
    auto put = [&](const void *src, size_t bytes) {
        size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + bytes);
        std::memcpy(host.data() + off, src, bytes);
        return off;
    };
    for (size_t s = 0; s < all.size();) {
        size_t e = s + 1;
        const RecLaunch &f = all[s].L;
        while (e < all.size() && all[e].L.key == f.key && all[e].L.multi == f.multi &&
               all[e].L.block.x == f.block.x && all[e].L.block.y == f.block.y && all[e].L.block.z == f.block.z)
            ++e;
        if (!f.multi) return fail(LMFMM_EINVAL, "a kernel of this apply has no batched form");
        // instances with the costliest blocks first: the dispatcher hands out
        // blocks in index order, so their long blocks do not start last
        std::stable_sort(all.begin() + s, all.begin() + e,
                         [](const Rec &a, const Rec &c) { return a.L.cost > c.L.cost; });
        BatchLaunch BL;
        BL.fn = f.multi;
        BL.block = f.block;
        BL.shmem = 0;
        BL.n = (int)(e - s);
        BL.cls = stage_class(f.key);
        std::vector<int> blk0(BL.n + 1), grid(3 * BL.n);
        const size_t asz = f.args.size(), stride = (asz + f.align - 1) / f.align * f.align;
        std::vector<char> args(stride * BL.n, 0);
        int64_t tot = 0;
        for (int k = 0; k < BL.n; ++k) {
            const RecLaunch &L = all[s + k].L;
            if (L.args.size() != asz) return fail(LMFMM_EINVAL, "batched launch with mixed argument layouts");
            blk0[k] = (int)tot;
            tot += (int64_t)L.grid.x * L.grid.y * L.grid.z;
            grid[3 * k] = (int)L.grid.x;
            grid[3 * k + 1] = (int)L.grid.y;
            grid[3 * k + 2] = (int)L.grid.z;
            std::memcpy(args.data() + stride * k, L.args.data(), asz);
            BL.shmem = std::max(BL.shmem, L.shmem);
        }
        if (tot > INT32_MAX) return fail(LMFMM_EINVAL, "batched launch too large");
        blk0[BL.n] = (int)tot;
        BL.nblk = (unsigned)tot;
        BL.off_blk0 = put(blk0.data(), blk0.size() * sizeof(int));
        BL.off_grid = put(grid.data(), grid.size() * sizeof(int));
        BL.off_args = put(args.data(), args.size());
        b->seq.push_back(BL);
        s = e;
    }
    int rc;
    if ((rc = upload(b->meta, host.data(), std::max<size_t>(host.size(), 256)))) return rc;
    char *base = (char *)b->meta.p;
    for (auto &BL : b->seq)
        BL.m = MultiArgs{(const int *)(base + BL.off_blk0), (const int *)(base + BL.off_grid),
                         (const void *)(base + BL.off_args), BL.n};
    return LMFMM_OK;
}

static int batch_prepare(lmfmm_batch_s *b, const lmfmm_instance *inst, int nrhs, int prec, hipStream_t st)
{
    batch_drop_graph(b);
    batch_collect_timing(b);
    const auto t_start = std::chrono::steady_clock::now();
    int rc;
    b->chosen_order.assign(b->n, 0);
    b->chosen_levels.assign(b->n, 0);
    b->chosen_us.assign(b->n, 0.0);
    b->from_cache.assign(b->n, 0);
    std::map<std::string, TuneEntry> cache;
    if (b->tune && !b->cache_path.empty()) read_tune_cache(b->cache_path, cache);
    bool cache_dirty = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct EvGuard {
        hipEvent_t &a, &c;
        ~EvGuard()
        {
            if (a) (void)hipEventDestroy(a);
            if (c) (void)hipEventDestroy(c);
        }
    } guard{e0, e1};
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // every timed (order, levels, us) of the instances tuned here, and their
    // cache keys and near-field forms
    std::vector<std::vector<std::array<double, 3>>> cands(b->n);
    std::vector<std::string> keys(b->n);
    std::vector<int> sweeps(b->n, 1);
    for (int i = 0; i < b->n; ++i) {
        lmfmm_plan_s *p = b->plans[i];
        const lmfmm_instance &in = inst[i];
        p->have_box = false;
        if (in.n_src == 0 || in.n_tgt == 0) continue;
        // 1. pin the bounding box
        double bb[8];
        if ((rc = get_bbox(p, p->med, in.n_src, in.src_xy, in.n_tgt, in.tgt_xy, st, bb))) return rc;
        for (int j = 0; j < 6; ++j) p->box[j] = bb[j];
        p->have_box = true;
        // 2. order floor and levels: the cache, else timed candidates
        p->levels_opt = 0;
        Geometry g0;
        if ((rc = make_geometry(p, bb, in.n_src, nrhs, g0))) return rc;
        const std::string key = tune_key(b, p, in, nrhs, prec);
        auto hit = cache.find(key);
        int bo = b->order_set.front(), bl = g0.L, bs = p->near_sweep ? 1 : 0;
        double best = 0.0;
        if (b->tune && hit != cache.end()) {
            bo = hit->second.order;
            bl = hit->second.levels;
            if (b->tune_near) bs = hit->second.sweep;
            best = hit->second.us;
            b->from_cache[i] = 1;
        } else if (b->tune) {
            // time one candidate: a first apply builds its tables, a second
            // captures its launch sequence, then the replays are timed in
            // three windows of three, of which the fastest counts
            auto time_candidate = [&](double &us) -> int {
                int r = plan_apply_any(p, in, nrhs, prec, st);
                if (r) return r;
                if ((r = plan_apply_any(p, in, nrhs, prec, st))) return r;
                const int reps = 3;
                us = 1e300;
                for (int win = 0; win < 3; ++win) {
                    HIPCHK(hipEventRecord(e0, st));
                    for (int k = 0; k < reps && r == LMFMM_OK; ++k) r = plan_apply_any(p, in, nrhs, prec, st);
                    if (r) return r;
                    HIPCHK(hipEventRecord(e1, st));
                    HIPCHK(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                    us = std::min(us, 1e3 * ms / reps);
                }
                return LMFMM_OK;
            };
            // per order floor, the depth by descent from the automatic one:
            // deeper while that is faster, else shallower while faster
            best = 1e300;
            for (int o : b->order_set) {
                p->order = o;
                std::map<int, double> seen;
                auto at = [&](int L, double &us) -> int {
                    auto it = seen.find(L);
                    if (it != seen.end()) {
                        us = it->second;
                        return LMFMM_OK;
                    }
                    p->levels_opt = L;
                    int r = time_candidate(us);
                    if (r == LMFMM_ETOL) us = 1e300, r = LMFMM_OK;
                    if (!r) seen[L] = us;
                    return r;
                };
                int Lb = g0.L;
                double ub = 0.0;
                if ((rc = at(Lb, ub))) return rc;
                for (int dir = 1; dir >= -1; dir -= 2) {
                    bool moved = false;
                    while (Lb + dir >= 1 && Lb + dir <= std::min(MAXLEV, g0.L + 6)) {
                        double un = 0.0;
                        if ((rc = at(Lb + dir, un))) return rc;
                        if (!(un < ub)) break;
                        Lb += dir;
                        ub = un;
                        moved = true;
                    }
                    if (moved) break;
                }
                if (ub < best) {
                    best = ub;
                    bo = o;
                    bl = Lb;
                }
                for (const auto &kv : seen)
                    if (kv.second < 1e300) cands[i].push_back({(double)o, (double)kv.first, kv.second});
            }
            if (best >= 1e300) return fail(LMFMM_ETOL, "no candidate order meets the tolerance");
            if (b->tune_near) {
                // the other near-field form at the chosen order and depth
                p->order = bo;
                p->levels_opt = bl;
                p->near_sweep = !bs;
                double us = 0.0;
                if ((rc = time_candidate(us))) return rc;
                if (us < best) {
                    best = us;
                    bs = !bs;
                }
            }
            cache[key] = TuneEntry{bo, bl, bs, best};
            cache_dirty = true;
            keys[i] = key;
            sweeps[i] = bs;
        }
        p->order = bo;
        p->levels_opt = b->tune ? bl : 0;
        p->near_sweep = bs != 0;
        b->chosen_order[i] = bo;
        b->chosen_levels[i] = bl;
        b->chosen_us[i] = best;
        // 3. warm the chosen configuration (tables, workspace)
        if ((rc = plan_apply_any(p, in, nrhs, prec, st))) return rc;
        b->chosen_levels[i] = p->geo.L;
    }
    // 4. The merged launches of one stage run together, so the deepest
    // instance sets how many per-level launches the batch has.  Cap the depth
    // of the instances tuned here at one and two levels below the deepest
    // (each deeper one takes its fastest timed candidate within the cap, else
    // its order at the cap's depth if the near field stays empty there), time
    // the merged sequence, and keep the cap that saves most (by more than
    // 1 %).  A cap some instance cannot meet (its order or tolerance out of
    // reach at that depth) is skipped.
    int deepest = 0;
    for (int i = 0; i < b->n; ++i)
        if (!cands[i].empty()) deepest = std::max(deepest, b->chosen_levels[i]);
    if (deepest > 2 && b->n > 1) {
        auto time_merged = [&](double &us) -> int {
            int r = batch_record_merge(b, inst, nrhs, prec, st);
            if (r || (r = batch_launch_seq(b, st, false))) return r;
            us = 1e300;
            for (int win = 0; win < 3; ++win) {
                HIPCHK(hipEventRecord(e0, st));
                for (int k = 0; k < 3; ++k)
                    if ((r = batch_launch_seq(b, st, false))) return r;
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                us = std::min(us, 1e3 * ms / 3);
            }
            return LMFMM_OK;
        };
        auto set_choice = [&](const std::vector<int> &o, const std::vector<int> &l) -> int {
            for (int i = 0; i < b->n; ++i) {
                lmfmm_plan_s *p = b->plans[i];
                if (cands[i].empty() || (p->order == o[i] && p->levels_opt == l[i] && p->geo.L == l[i])) continue;
                p->order = o[i];
                p->levels_opt = l[i];
                int r = plan_apply_any(p, inst[i], nrhs, prec, st);
                if (r) return r;
            }
            return LMFMM_OK;
        };
        const std::vector<int> o0 = b->chosen_order, l0 = b->chosen_levels;
        std::vector<int> bo = o0, bl = l0;
        double best_us = 0.0;
        if ((rc = time_merged(best_us))) return rc;
        for (int cap = deepest - 1; cap >= std::max(2, deepest - 2); --cap) {
            std::vector<int> o = o0, l = l0;
            bool changed = false;
            for (int i = 0; i < b->n; ++i) {
                if (cands[i].empty() || l0[i] <= cap) continue;
                double bu = 1e300;
                for (const auto &c : cands[i])
                    if ((int)c[1] <= cap && c[2] < bu) {
                        bu = c[2];
                        o[i] = (int)c[0];
                        l[i] = (int)c[1];
                    }
                if (bu >= 1e300) {
                    // not timed alone: allowed where the cap's leaves leave the
                    // near field empty (else its cost can grow many times over)
                    lmfmm_plan_s *p = b->plans[i];
                    const int keep = p->levels_opt;
                    Geometry gc;
                    p->levels_opt = cap;
                    const int grc = make_geometry(p, p->box, inst[i].n_src, nrhs, gc);
                    p->levels_opt = keep;
                    const double wl = gc.lev[gc.L].w;
                    if (grc || gc.L != cap || !(p->box[2] >= wl || p->box[5] <= -wl)) continue;
                    l[i] = cap;
                }
                changed = true;
            }
            if (!changed) break;
            double us = 0.0;
            rc = set_choice(o, l);
            if (rc == LMFMM_ETOL || rc == LMFMM_EINVAL) continue;
            if (rc || (rc = time_merged(us))) return rc;
            if (us < 0.99 * best_us) {
                best_us = us;
                bo = o;
                bl = l;
            }
        }
        if ((rc = set_choice(bo, bl))) return rc;
        for (int i = 0; i < b->n; ++i) {
            if (cands[i].empty()) continue;
            if (bo[i] != o0[i] || bl[i] != l0[i]) {
                for (const auto &c : cands[i])
                    if ((int)c[0] == bo[i] && (int)c[1] == bl[i]) b->chosen_us[i] = c[2];
                cache[keys[i]] = TuneEntry{bo[i], bl[i], sweeps[i], b->chosen_us[i]};
            }
            b->chosen_order[i] = bo[i];
            b->chosen_levels[i] = b->plans[i]->geo.L;
        }
    }
    if (cache_dirty && !b->cache_path.empty()) write_tune_cache(b->cache_path, cache);
    HIPCHK(hipStreamSynchronize(st));
    if ((rc = batch_record_merge(b, inst, nrhs, prec, st))) return rc;
    b->desc.assign(inst, inst + b->n);
    b->nrhs = nrhs;
    b->prec = prec;
    // statistics: algorithmic work of every instance's apply (the recording
    // pass counted it), merged launches per apply
    for (int k = 0; k < 8; ++k) b->stats.kernel_flops[k] = 0.0;
    for (int i = 0; i < b->n; ++i)
        if (inst[i].n_tgt > 0 && inst[i].n_src > 0) {
            resolve_work(b->plans[i]);  // the leaf ranges of the warm apply (the recording launched nothing)
            for (int k = 0; k < 8; ++k) b->stats.kernel_flops[k] += b->plans[i]->stats.kernel_flops[k];
        }
    b->stats.launches = (int)b->seq.size();
    b->stats.instances = b->n;
    int ncache = 0;
    for (int v : b->from_cache) ncache += v;
    b->stats.tuned_from_cache = ncache;
    if (b->timing && b->ev.size() < 2 * b->seq.size()) {
        const size_t old = b->ev.size();
        b->ev.resize(2 * b->seq.size(), nullptr);
        for (size_t j = old; j < b->ev.size(); ++j) HIPCHK(hipEventCreate(&b->ev[j]));
    }
    if (b->graph) {
        if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        const int lrc = batch_launch_seq(b, b->cap_stream, false);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(b->cap_stream, &g);  // the capture always ends here
        if (lrc || ce != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            if (lrc) return lrc;
            return fail(LMFMM_EHIP, std::string("graph capture failed: ") + hipGetErrorString(ce));
        }
        b->g = g;
        HIPCHK(hipGraphInstantiate(&b->ge, g, nullptr, nullptr, 0));
    }
    b->stats.prepare_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    b->prepared = true;
    return LMFMM_OK;
}

extern "C" {

int lmfmm_batch_create(int n_inst, const double *k, const double *d, const int *order_set, int n_orders, double tol,
                       lmfmm_batch *out)
{
    if (!out) return fail(LMFMM_EINVAL, "out is null");
    *out = nullptr;
    if (n_inst < 1 || n_inst > 4096 || !k || !d) return fail(LMFMM_EINVAL, "bad instance count or media");
    if (!order_set || n_orders < 1 || n_orders > 16) return fail(LMFMM_EINVAL, "bad order set");
    for (int i = 0; i < n_orders; ++i)
        if (order_set[i] < 1 || order_set[i] > 256) return fail(LMFMM_EINVAL, "orders must be in [1, 256]");
    lmfmm_batch_s *b = new (std::nothrow) lmfmm_batch_s();
    if (!b) return fail(LMFMM_ENOMEM, "batch allocation failed");
    std::memset(&b->stats, 0, sizeof b->stats);
    b->n = n_inst;
    b->tol = tol;
    b->order_set.assign(order_set, order_set + n_orders);
    std::sort(b->order_set.begin(), b->order_set.end());
    if (const char *env = std::getenv("LMFMM_TUNE_CACHE")) b->cache_path = env;
    for (int i = 0; i < n_inst; ++i) {
        lmfmm_plan p = nullptr;
        int rc = lmfmm_create(k + 6 * i, d[i], b->order_set.front(), tol, &p);
        if (rc) {
            for (auto q : b->plans) lmfmm_destroy(q);
            delete b;
            return rc;
        }
        p->use_graph = false;  // the batch launches its instances' kernels itself
        b->plans.push_back(p);
    }
    *out = b;
    return LMFMM_OK;
}

int lmfmm_batch_destroy(lmfmm_batch b)
{
    if (!b) return fail(LMFMM_EINVAL, "batch is null");
    (void)hipDeviceSynchronize();
    batch_drop_graph(b);
    b->meta.release();
    for (auto p : b->plans) lmfmm_destroy(p);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (auto e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
    return LMFMM_OK;
}

int lmfmm_batch_set_option(lmfmm_batch b, const char *key, const char *value)
{
    if (!b || !key || !value) return fail(LMFMM_EINVAL, "null argument");
    std::string k(key), v(value);
    if (k == "tune" || k == "graph") {
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "tune/graph must be 0 or 1");
        (k == "tune" ? b->tune : b->graph) = v == "1";
        batch_drop_graph(b);
        return LMFMM_OK;
    }
    if (k == "tune_cache") {
        b->cache_path = v;
        return LMFMM_OK;
    }
    if (k == "timing") {
        if (v == "reset") {
            batch_collect_timing(b);
            for (int i = 0; i < 8; ++i) {
                b->stats.kernel_ms[i] = 0;
                b->stats.kernel_launches[i] = 0;
            }
            b->stats.timed_applies = 0;
            return LMFMM_OK;
        }
        if (v != "0" && v != "1") return fail(LMFMM_EINVAL, "timing must be 0, 1 or reset");
        batch_collect_timing(b);
        b->timing = v == "1";
        if (b->timing && b->ev.size() < 2 * b->seq.size()) {
            const size_t old = b->ev.size();
            b->ev.resize(2 * b->seq.size(), nullptr);
            for (size_t j = old; j < b->ev.size(); ++j)
                if (hipEventCreate(&b->ev[j]) != hipSuccess) return fail(LMFMM_EHIP, "hipEventCreate failed");
        }
        return LMFMM_OK;
    }
    // any other key is forwarded to every instance's plan
    if (k == "near_sweep") b->tune_near = false;
    for (auto p : b->plans) {
        int rc = lmfmm_set_option(p, key, value);
        if (rc) return rc;
    }
    batch_drop_graph(b);
    return LMFMM_OK;
}

int lmfmm_batch_apply(lmfmm_batch b, const lmfmm_instance *inst, int nrhs, int prec, void *stream)
{
    if (!b || !inst) return fail(LMFMM_EINVAL, "null argument");
    for (int i = 0; i < b->n; ++i) {
        int rc = check_common(b->plans[i], inst[i].n_src, inst[i].src_xy, inst[i].n_tgt, inst[i].tgt_xy, inst[i].q,
                              inst[i].u, nrhs, prec);
        if (rc) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    bool same = b->prepared && nrhs == b->nrhs && prec == b->prec;
    for (int i = 0; same && i < b->n; ++i) same = same_desc(inst[i], b->desc[i]);
    if (!same) {
        int rc = batch_prepare(b, inst, nrhs, prec, st);
        if (rc) {
            batch_drop_graph(b);
            return rc;
        }
    }
    // instances without sources have no recorded launches: zero their outputs
    for (int i = 0; i < b->n; ++i)
        if (inst[i].n_src == 0 && inst[i].n_tgt > 0)
            launch_zero_bytes(inst[i].u, (size_t)inst[i].n_tgt * nrhs * (prec == LMFMM_C128 ? 16 : 8), st);
    batch_collect_timing(b);
    if (b->timing && b->ev.size() >= 2 * b->seq.size()) {
        int rc = batch_launch_seq(b, st, true);
        if (rc) return rc;
        b->ev_pending = !b->seq.empty();
        return LMFMM_OK;
    }
    if (b->ge) {
        HIPCHK(hipGraphLaunch(b->ge, st));
        b->stats.graph_applies++;
        return LMFMM_OK;
    }
    return batch_launch_seq(b, st, false);
}

int lmfmm_batch_get_choice(lmfmm_batch b, int i, int *order, int *levels, double *us, int *near_sweep)
{
    if (!b || i < 0 || i >= b->n) return fail(LMFMM_EINVAL, "bad batch or index");
    if (!b->prepared) return fail(LMFMM_EINVAL, "batch not prepared yet");
    if (order) *order = b->chosen_order[i];
    if (levels) *levels = b->chosen_levels[i];
    if (us) *us = b->chosen_us[i];
    if (near_sweep) *near_sweep = b->plans[i]->near_sweep ? 1 : 0;
    return LMFMM_OK;
}

int lmfmm_batch_get_stats(lmfmm_batch b, lmfmm_batch_stats *s)
{
    if (!b || !s) return fail(LMFMM_EINVAL, "null argument");
    batch_collect_timing(b);
    *s = b->stats;
    return LMFMM_OK;
}

int lmfmm_batch_sync_status(lmfmm_batch b, void *stream)
{
    if (!b) return fail(LMFMM_EINVAL, "batch is null");
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    if (!b->prepared) return LMFMM_OK;
    std::string bad;
    for (int i = 0; i < b->n; ++i) {
        lmfmm_plan_s *p = b->plans[i];
        if (!p->d_err || !p->err_valid) continue;
        int32_t e = 0;
        HIPCHK(hipMemcpy(&e, p->d_err + 1, sizeof e, hipMemcpyDeviceToHost));
        if (e) bad += (bad.empty() ? "" : ", ") + std::to_string(i);
    }
    if (!bad.empty()) {
        batch_drop_graph(b);  // the next apply reads the bounding boxes again
        return fail(LMFMM_EDOMAIN, "instance(s) " + bad +
                                       ": points outside the bounding box the batch was prepared for, or outside "
                                       "their layer (their results are invalid)");
    }
    return LMFMM_OK;
}

}  // extern "C"
