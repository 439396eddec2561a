/*
 * lmfmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 CPU reference for the reflected field g_2^t of the
 * two-dimensional three-layer Helmholtz medium (Cho & Huang, arXiv 1902.08250,
 * Section 1 and Section 3 Example 4), applied to densities by an O(N*M) direct
 * sum.  Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load this library; the GPU library never links or calls it, and it
 * shares no source, header or table with the GPU library.
 *
 * What is computed (Section 1, eq. for g_2^t; Section 3, Example 4):
 *
 *   g(x1,y1; x0,y0) = Int_R exp(s2*y1 + i*lam*x1) exp(-s1*y0 - i*lam*x0)
 *                            * sigma_2^t(lam) / (4*pi*s2)  d lam,
 *   s_m = sqrt(lam^2 - k_m^2)  (principal branch, Re s_m >= 0),
 *
 * for a source in the top layer (y0 > 0) and a target in the middle layer
 * (-d < y1 < 0).  The other components of the scattered field of Example 4
 * (g_1^s in the top layer, g_2^b in the middle layer, g_3^s in the bottom
 * layer) and the impedance half-space of Example 3 are the same kind of
 * integral with another target factor and density (sigma_comp and
 * target_exponent below).  sigma_2^t is the closed form the paper gives (Section 1,
 * repeated in Section 3 Example 4 and Section 5); numerator and denominator
 * are both divided by exp(d*s2), which leaves the value unchanged and keeps
 * every factor bounded.
 *
 * How the integral is evaluated.  With Im k_m > 0 the integrand is analytic on
 * the real axis; its singularities (branch points +-k_m, guided-mode poles of
 * sigma) lie in the first and third quadrants.  Following the paper's
 * contour-integration argument (Section 4.2, Fig. 1 and the "first contour" of
 * Section 5, Fig. 2), the real-axis integral is split at +-c with c beyond
 * every singularity:
 *   - the finite piece [-c, c] is moved off the axis onto the polyline
 *     -c -> -c + i h -> c - i h -> c (above the axis for Re lam < 0, below it
 *     for Re lam > 0, where the integrand has no singularity);
 *   - "north" representation (|x1-x0| <= eta*(y0-y1)): the two tails stay on
 *     the real axis, where they decay like exp(-|lam|(y0-y1));
 *   - "east" representation, the alternative direction (|x1-x0| > eta*(y0-y1)):
 *     each tail is turned onto the vertical ray +-c + i tau, tau >= 0, where
 *     exp(i lam |x1-x0|) decays like exp(-tau |x1-x0|).
 * The integrand depends on x1 - x0 only through exp(i lam (x1-x0)) and is
 * otherwise even in lam, so g is even in x1 - x0 and |x1 - x0| is used.
 *
 * Every piece is integrated with adaptive bisection of 16-point Gauss-Legendre
 * panels (nodes found by Newton's method on the Legendre polynomial), and the
 * direct sums use Neumaier compensated summation.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EDOMAIN (-2)

/* ------------------------------------------------------------------------ */
/* Medium and options                                                        */
/* ------------------------------------------------------------------------ */
/* The field component (which layer the target is in, and which part):
 *   COMP_2T: middle layer, part from the top interface, g_2^t (the default);
 *   COMP_2B: middle layer, part from the bottom interface, g_2^b;
 *   COMP_1S: top layer (reflected field), g_1^s;
 *   COMP_3S: bottom layer (transmitted field), g_3^s;
 *   COMP_IMP: the impedance half-space of Section 3 Example 3 (source and
 *   target above y = 0, wave number k = k1, impedance alpha). */
enum { COMP_2T = 0, COMP_2B = 1, COMP_1S = 2, COMP_3S = 3, COMP_IMP = 4 };

typedef struct {
    cplx k1, k2, k3;
    double d;
    int sigma_unity; /* 1: replace sigma by 1 (free-space closed-form check) */
    int comp;        /* COMP_*                                              */
    double alpha;    /* impedance (COMP_IMP)                                */
} medium_t;

typedef struct {
    double eta;      /* north if |dx| <= eta*(y0-y1), else east            */
    double c_factor; /* c = c_factor * max Re k_m                          */
    int rep;         /* 0 automatic, 1 force north, 2 force east           */
    double eps;      /* relative accuracy goal per piece                   */
} opts_t;

static void read_medium(const double *med, int flags, medium_t *m)
{
    m->k1 = med[0] + I * med[1];
    m->k2 = med[2] + I * med[3];
    m->k3 = med[4] + I * med[5];
    m->d = med[6];
    m->sigma_unity = flags & 1;
    m->comp = (flags >> 1) & 7;
    m->alpha = med[7];
}

static void read_opts(const double *opt, opts_t *o)
{
    o->eta = 1.0;
    o->c_factor = 1.5;
    o->rep = 0;
    o->eps = 1e-15;
    if (opt) {
        if (opt[0] > 0) o->eta = opt[0];
        if (opt[1] > 0) o->c_factor = opt[1];
        o->rep = (int)opt[2];
        if (opt[3] > 0) o->eps = opt[3];
    }
}

/* ------------------------------------------------------------------------ */
/* Kernel pieces                                                             */
/* ------------------------------------------------------------------------ */
/* s_m = sqrt(lam^2 - k^2), principal branch (csqrt has Re >= 0). */
static cplx sroot(cplx lam, cplx k) { return csqrt(lam * lam - k * k); }

/* sigma_2^t(lam): the paper's closed form (Section 1; Section 3 Example 4,
 * second component of the solution of the 4x4 interface system) with
 * numerator and denominator divided by exp(d*s2):
 *   sinh(d s2)/e^{d s2} = (1 - e^{-2 d s2})/2,  cosh(d s2)/e^{d s2} = (1 + e^{-2 d s2})/2. */
static cplx sigma2t(cplx lam, const medium_t *m)
{
    if (m->sigma_unity) return 1.0;
    cplx s1 = sroot(lam, m->k1), s2 = sroot(lam, m->k2), s3 = sroot(lam, m->k3);
    cplx e = cexp(-2.0 * m->d * s2);
    cplx l2 = lam * lam, kk2 = m->k2 * m->k2;
    cplx num = l2 + s2 * s3 - kk2;
    cplx den = 0.5 * (1.0 - e) * (l2 + s1 * s3 - kk2) + 0.5 * s2 * (s1 + s3) * (1.0 + e);
    return num / den;
}

/* The other densities of Section 3 Example 4, from the paper's closed forms
 * with numerator and denominator divided by exp(d*s2) as for sigma_2^t (the
 * common denominator D below is that of sigma_2^t):
 *   sigma_1   = [sinh(d s2)(-l^2 + s1 s3 + k2^2) + s2 (s1 - s3) cosh(d s2)] / D,
 *   sigma_2^b = -e^{d s2} (-l^2 + s2 s3 + k2^2) / D,
 *   sigma_3   = 2 s2 s3 e^{d s3} / D.
 * (The 4x4 interface system's unknowns are sigma_1, sigma_2^t,
 * e^{-d s2} sigma_2^b and e^{-d s3} sigma_3 of these closed forms.) */
static cplx sigma_comp(cplx lam, const medium_t *m)
{
    if (m->sigma_unity) return 1.0;
    if (m->comp == COMP_2T) return sigma2t(lam, m);
    if (m->comp == COMP_IMP) {
        /* Section 3 Example 3: (s + i k alpha) / (s - i k alpha), s = sqrt(lam^2 - k^2) */
        cplx s = sroot(lam, m->k1);
        return (s + I * m->k1 * m->alpha) / (s - I * m->k1 * m->alpha);
    }
    cplx s1 = sroot(lam, m->k1), s2 = sroot(lam, m->k2), s3 = sroot(lam, m->k3);
    cplx e = cexp(-2.0 * m->d * s2);
    cplx l2 = lam * lam, kk2 = m->k2 * m->k2;
    cplx den = 0.5 * (1.0 - e) * (l2 + s1 * s3 - kk2) + 0.5 * s2 * (s1 + s3) * (1.0 + e);
    if (m->comp == COMP_1S) return (0.5 * (1.0 - e) * (-l2 + s1 * s3 + kk2) + 0.5 * s2 * (s1 - s3) * (1.0 + e)) / den;
    if (m->comp == COMP_2B) return -(-l2 + s2 * s3 + kk2) / den;
    return 2.0 * s2 * s3 * cexp(m->d * (s3 - s2)) / den; /* COMP_3S */
}

/* The target factor of each component: exp(tgt_exp(s_t) ...) with the
 * target-side root s_t, and the density sigma / (4 pi s_t):
 *   g_2^t: e^{ s2 y},          g_2^b: e^{-s2 (y + 2d)},   g_1^s: e^{-s1 y},
 *   g_3^s: e^{ s3 y} (read: the printed e^{-s3 (y + 2d)} grows as y -> -inf
 *          and contradicts the interface system; e^{s3 y} with sigma_3 as
 *          above satisfies it and gives the free field in a homogeneous
 *          medium),
 *   impedance: e^{-s y}.
 * The source factor is e^{-s1 y0} (e^{-s y0} for the impedance case). */
static cplx target_root(cplx lam, const medium_t *m)
{
    switch (m->comp) {
    case COMP_1S:
    case COMP_IMP: return sroot(lam, m->k1);
    case COMP_3S: return sroot(lam, m->k3);
    default: return sroot(lam, m->k2);
    }
}
/* exponent of the target factor and its derivative in y */
static cplx target_exponent(cplx st, double y, const medium_t *m, cplx *dy)
{
    switch (m->comp) {
    case COMP_2B: *dy = -st; return -st * (y + 2.0 * m->d);
    case COMP_1S:
    case COMP_IMP: *dy = -st; return -st * y;
    default: *dy = st; return st * y; /* COMP_2T, COMP_3S */
    }
}

/* One pair: geometry and the derivative factor to apply. */
typedef struct {
    double y1, y0, adx; /* target y, source y, |x1 - x0|            */
    double sgn;         /* sign of x1 - x0 (0 when equal)          */
    const medium_t *m;
    int nder;           /* number of outputs: 1 (g) or 5 (g and 4 derivatives) */
} pair_t;

/* Integrand values at lam: out[0] = f, out[1..4] = f times the factor that
 * differentiates with respect to x1, y1, x0, y0 respectively. */
static void integrand(cplx lam, const pair_t *p, cplx *out)
{
    const medium_t *m = p->m;
    cplx s1 = sroot(lam, m->k1), st = target_root(lam, m), dy1;
    cplx f = cexp(target_exponent(st, p->y1, m, &dy1) - s1 * p->y0 + I * lam * p->adx) * sigma_comp(lam, m) /
             (4.0 * M_PI * st);
    out[0] = f;
    if (p->nder > 1) {
        out[1] = f * (I * lam * p->sgn);  /* d/dx1 */
        out[2] = f * dy1;                 /* d/dy1 */
        out[3] = -out[1];                 /* d/dx0 */
        out[4] = f * (-s1);               /* d/dy0 */
    }
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre 16-point rule on [-1, 1]                                   */
/* ------------------------------------------------------------------------ */
#define NGL 16
static double gl_x[NGL], gl_w[NGL];
static int gl_ready = 0;

/* Nodes are the roots of P_16, found by Newton's method from the standard
 * cosine initial guesses; P_n and P_n' come from the three-term recurrence
 * (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}.  Weights are 2/((1-x^2) P'(x)^2). */
static void gl_init(void)
{
    if (gl_ready) return;
    for (int i = 0; i < NGL; ++i) {
        double x = cos(M_PI * (i + 0.75) / (NGL + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int n = 1; n < NGL; ++n) {
                double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
                p0 = p1;
                p1 = p2;
            }
            double dp = NGL * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        double p0 = 1.0, p1 = x;
        for (int n = 1; n < NGL; ++n) {
            double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
            p0 = p1;
            p1 = p2;
        }
        double dp = NGL * (x * p1 - p0) / (x * x - 1.0);
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

#define MAXOUT 5

/* Gauss-Legendre on the straight complex segment A -> B. */
static void gl_segment(cplx A, cplx B, const pair_t *p, cplx *res)
{
    cplx half = 0.5 * (B - A), mid = 0.5 * (A + B);
    cplx v[MAXOUT];
    for (int k = 0; k < p->nder; ++k) res[k] = 0;
    for (int i = 0; i < NGL; ++i) {
        integrand(mid + half * gl_x[i], p, v);
        for (int k = 0; k < p->nder; ++k) res[k] += gl_w[i] * v[k];
    }
    for (int k = 0; k < p->nder; ++k) res[k] *= half;
}

static double vmax_abs(const cplx *v, int n)
{
    double m = 0;
    for (int k = 0; k < n; ++k)
        if (cabs(v[k]) > m) m = cabs(v[k]);
    return m;
}

/* Adaptive bisection: accept the two halves once they agree with the whole. */
static void adapt(cplx A, cplx B, const cplx *whole, double tol, int depth, const pair_t *p, cplx *res)
{
    cplx M = 0.5 * (A + B), l[MAXOUT], r[MAXOUT], diff[MAXOUT];
    gl_segment(A, M, p, l);
    gl_segment(M, B, p, r);
    for (int k = 0; k < p->nder; ++k) diff[k] = whole[k] - (l[k] + r[k]);
    if (vmax_abs(diff, p->nder) <= tol || depth >= 48) {
        for (int k = 0; k < p->nder; ++k) res[k] = l[k] + r[k];
        return;
    }
    cplx rl[MAXOUT], rr[MAXOUT];
    adapt(A, M, l, tol, depth + 1, p, rl);
    adapt(M, B, r, tol, depth + 1, p, rr);
    for (int k = 0; k < p->nder; ++k) res[k] = rl[k] + rr[k];
}

/* A contour piece given as a chain of straight segments. */
#define MAXSEG 96
typedef struct {
    int n;
    cplx a[MAXSEG], b[MAXSEG];
    double sign; /* +1 or -1: orientation factor applied to the piece's integral */
} piece_t;

static void piece_add(piece_t *pc, cplx a, cplx b)
{
    if (pc->n < MAXSEG) {
        pc->a[pc->n] = a;
        pc->b[pc->n] = b;
        pc->n++;
    }
}

/* Geometrically graded segments of a ray start + dir*t, t in [0, T]. */
static void piece_ray(piece_t *pc, cplx start, cplx dir, double t0, double T)
{
    double a = 0.0, b = t0;
    if (b > T) b = T;
    while (a < T) {
        piece_add(pc, start + dir * a, start + dir * b);
        a = b;
        b = (2.0 * b < T) ? 2.0 * b : T;
    }
}

/* Integrate a set of pieces: a coarse pass sets the absolute scale, then every
 * segment is refined adaptively against eps * scale. */
static void integrate_pieces(piece_t *pcs, int npc, const pair_t *p, double eps, cplx *out)
{
    static const int MAXTOT = 3 * MAXSEG;
    cplx coarse[3 * MAXSEG][MAXOUT];
    double scale = 0;
    int idx = 0;
    for (int q = 0; q < npc; ++q)
        for (int s = 0; s < pcs[q].n && idx < MAXTOT; ++s, ++idx) {
            gl_segment(pcs[q].a[s], pcs[q].b[s], p, coarse[idx]);
            double m = vmax_abs(coarse[idx], p->nder);
            if (m > scale) scale = m;
        }
    if (scale == 0) scale = 1e-300;
    double tol = eps * scale;
    for (int k = 0; k < p->nder; ++k) out[k] = 0;
    idx = 0;
    for (int q = 0; q < npc; ++q) {
        for (int s = 0; s < pcs[q].n && idx < MAXTOT; ++s, ++idx) {
            cplx r[MAXOUT];
            adapt(pcs[q].a[s], pcs[q].b[s], coarse[idx], tol, 0, p, r);
            for (int k = 0; k < p->nder; ++k) out[k] += pcs[q].sign * r[k];
        }
    }
}

static double max3(double a, double b, double c)
{
    double m = a > b ? a : b;
    return m > c ? m : c;
}

/* One kernel entry (and optionally its four coordinate derivatives).
 * rep_used reports 1 (north) or 2 (east). */
static int entry(double x1, double y1, double x0, double y0, const medium_t *m, const opts_t *o, int nder,
                 cplx *out, int *rep_used)
{
    pair_t p;
    p.y1 = y1;
    p.y0 = y0;
    p.adx = fabs(x1 - x0);
    p.sgn = (x1 > x0) ? 1.0 : ((x1 < x0) ? -1.0 : 0.0);
    p.m = m;
    p.nder = nder;
    /* vertical decay length of the integrand along the real axis */
    double a = y0 - y1; /* g_2^t, g_3^s */
    if (m->comp == COMP_2B) a = y0 + y1 + 2.0 * m->d;
    if (m->comp == COMP_1S || m->comp == COMP_IMP) a = y0 + y1;
    double kmax = max3(creal(m->k1), creal(m->k2), creal(m->k3));
    double c = o->c_factor * kmax;
    if (c < 1.0) c = 1.0;
    double h = 0.25 * c;
    if (p.adx > 0 && 2.0 / p.adx < h) h = 2.0 / p.adx;

    int rep = o->rep;
    if (rep == 0) rep = (p.adx <= o->eta * a) ? 1 : 2;
    if (rep_used) *rep_used = rep;

    piece_t pcs[3];
    memset(pcs, 0, sizeof(pcs));
    /* finite piece: polyline -c -> -c + ih -> c - ih -> c, split into short segments */
    pcs[0].sign = 1.0;
    piece_add(&pcs[0], -c, -c + I * h);
    {
        int nseg = 8;
        cplx A = -c + I * h, B = c - I * h;
        for (int s = 0; s < nseg; ++s) piece_add(&pcs[0], A + (B - A) * ((double)s / nseg), A + (B - A) * ((double)(s + 1) / nseg));
    }
    piece_add(&pcs[0], c - I * h, c);

    if (rep == 1) {
        /* north: real-axis tails, truncated where exp(-(lam - c) a) < e^-60 */
        double T = 60.0 / a;
        pcs[1].sign = 1.0;
        piece_ray(&pcs[1], c, 1.0, 0.25 * c, T);
        pcs[2].sign = -1.0; /* -c -> -c - T traversed backwards */
        piece_ray(&pcs[2], -c, -1.0, 0.25 * c, T);
    } else {
        /* east (alternative direction): Int_c^inf f = i Int_0^inf f(c + i tau) d tau,
         * Int_{-inf}^{-c} f = -i Int_0^inf f(-c + i tau) d tau */
        if (p.adx <= 0) return ORC_EINVAL;
        double T = 60.0 / p.adx;
        pcs[1].sign = 1.0;
        piece_ray(&pcs[1], c, I, 0.25 * c, T);
        pcs[2].sign = -1.0;
        piece_ray(&pcs[2], -c, I, 0.25 * c, T);
    }
    integrate_pieces(pcs, 3, &p, o->eps, out);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Neumaier compensated complex accumulator                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double sr, cr, si, ci;
} nsum_t;

static void nadd1(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

static void nadd(nsum_t *a, cplx v)
{
    nadd1(&a->sr, &a->cr, creal(v));
    nadd1(&a->si, &a->ci, cimag(v));
}

static cplx nval(const nsum_t *a) { return (a->sr + a->cr) + I * (a->si + a->ci); }

/* ------------------------------------------------------------------------ */
/* Exported API                                                              */
/* ------------------------------------------------------------------------ */
/* the target's layer of each component */
static int target_in_layer(double y, const medium_t *m)
{
    switch (m->comp) {
    case COMP_1S:
    case COMP_IMP: return y > 0;
    case COMP_3S: return y < -m->d;
    default: return y < 0 && y > -m->d;
    }
}

static int check_layers(long n_src, const double *src, long n_tgt, const double *tgt, const medium_t *m)
{
    for (long j = 0; j < n_src; ++j)
        if (!(src[n_src + j] > 0) || !isfinite(src[j]) || !isfinite(src[n_src + j])) return ORC_EDOMAIN;
    for (long i = 0; i < n_tgt; ++i)
        if (!target_in_layer(tgt[n_tgt + i], m) || !isfinite(tgt[i]) || !isfinite(tgt[n_tgt + i])) return ORC_EDOMAIN;
    return ORC_OK;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* sigma_2^t at n complex points lam (interleaved re,im) -> out (interleaved). */
int orc_sigma2t(const double *med, int flags, long n, const double *lam, double *out)
{
    medium_t m;
    read_medium(med, flags, &m);
    for (long i = 0; i < n; ++i) {
        cplx v = sigma2t(lam[2 * i] + I * lam[2 * i + 1], &m);
        out[2 * i] = creal(v);
        out[2 * i + 1] = cimag(v);
    }
    return ORC_OK;
}

/* sigma of the medium's component (flags bits 1-3) at n complex points. */
int orc_sigma(const double *med, int flags, long n, const double *lam, double *out)
{
    medium_t m;
    read_medium(med, flags, &m);
    for (long i = 0; i < n; ++i) {
        cplx v = sigma_comp(lam[2 * i] + I * lam[2 * i + 1], &m);
        out[2 * i] = creal(v);
        out[2 * i + 1] = cimag(v);
    }
    return ORC_OK;
}

/* One entry g(x1,y1;x0,y0) (nder=1) or g and its derivatives d/dx1, d/dy1,
 * d/dx0, d/dy0 (nder=5); out holds nder interleaved complex values. */
int orc_entry(const double *med, int flags, const double *opt, double x1, double y1, double x0, double y0, int nder,
              double *out, int *rep_used)
{
    if (nder != 1 && nder != 5) return ORC_EINVAL;
    medium_t m;
    opts_t o;
    read_medium(med, flags, &m);
    read_opts(opt, &o);
    if (!(y0 > 0) || !target_in_layer(y1, &m)) return ORC_EDOMAIN;
    gl_init();
    cplx v[MAXOUT];
    int rc = entry(x1, y1, x0, y0, &m, &o, nder, v, rep_used);
    for (int k = 0; k < nder; ++k) {
        out[2 * k] = creal(v[k]);
        out[2 * k + 1] = cimag(v[k]);
    }
    return rc;
}

/* u[r][i] = sum_j g(tgt_i, src_j) q[r][j].  src, tgt: SoA [2][n] (x then y);
 * q: [nrhs][n_src] interleaved complex; u: [nrhs][n_tgt] interleaved complex.
 * The (target, source-chunk) tasks run in parallel; each chunk's sum is
 * compensated and the chunks of a target are added in chunk order. */
int orc_apply(const double *med, int flags, const double *opt, long n_src, const double *src, const double *q,
              long n_tgt, const double *tgt, double *u, int nrhs, int nthreads)
{
    if (n_src < 0 || n_tgt < 0 || nrhs < 1 || nrhs > 64) return ORC_EINVAL;
    medium_t m;
    opts_t o;
    read_medium(med, flags, &m);
    read_opts(opt, &o);
    int rc = check_layers(n_src, src, n_tgt, tgt, &m);
    if (rc) return rc;
    gl_init();
    set_threads(nthreads);
    /* split the sources so that there are at least ~4 tasks per thread */
    long nth = orc_max_threads();
    long nchunk = 1;
    if (n_tgt > 0 && n_tgt < 4 * nth) nchunk = (4 * nth + n_tgt - 1) / n_tgt;
    if (nchunk > n_src) nchunk = n_src > 0 ? n_src : 1;
    long clen = n_src > 0 ? (n_src + nchunk - 1) / nchunk : 0;
    nsum_t *part = (nsum_t *)calloc((size_t)n_tgt * nchunk * nrhs + 1, sizeof(nsum_t));
    if (!part) return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (long task = 0; task < n_tgt * nchunk; ++task) {
        long i = task / nchunk, c = task % nchunk;
        long j0 = c * clen, j1 = j0 + clen < n_src ? j0 + clen : n_src;
        nsum_t *acc = part + (size_t)task * nrhs;
        for (long j = j0; j < j1; ++j) {
            cplx g;
            if (entry(tgt[i], tgt[n_tgt + i], src[j], src[n_src + j], &m, &o, 1, &g, NULL)) bad = 1;
            for (int r = 0; r < nrhs; ++r) {
                const double *qr = q + 2 * (size_t)r * n_src;
                nadd(&acc[r], g * (qr[2 * j] + I * qr[2 * j + 1]));
            }
        }
    }
    for (long i = 0; i < n_tgt; ++i)
        for (int r = 0; r < nrhs; ++r) {
            nsum_t tot;
            memset(&tot, 0, sizeof tot);
            for (long c = 0; c < nchunk; ++c) nadd(&tot, nval(&part[((size_t)i * nchunk + c) * nrhs + r]));
            cplx v = nval(&tot);
            u[2 * ((size_t)r * n_tgt + i)] = creal(v);
            u[2 * ((size_t)r * n_tgt + i) + 1] = cimag(v);
        }
    free(part);
    return bad ? ORC_EINVAL : ORC_OK;
}

/* Transposed operator, no conjugation: v[r][j] = sum_i g(tgt_i, src_j) w[r][i].
 * The outer loop runs over sources. */
int orc_apply_adjoint(const double *med, int flags, const double *opt, long n_src, const double *src, long n_tgt,
                      const double *tgt, const double *w, double *v, int nrhs, int nthreads)
{
    if (n_src < 0 || n_tgt < 0 || nrhs < 1 || nrhs > 64) return ORC_EINVAL;
    medium_t m;
    opts_t o;
    read_medium(med, flags, &m);
    read_opts(opt, &o);
    int rc = check_layers(n_src, src, n_tgt, tgt, &m);
    if (rc) return rc;
    gl_init();
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (long j = 0; j < n_src; ++j) {
        nsum_t acc[64];
        memset(acc, 0, sizeof(nsum_t) * nrhs);
        for (long i = 0; i < n_tgt; ++i) {
            cplx g;
            if (entry(tgt[i], tgt[n_tgt + i], src[j], src[n_src + j], &m, &o, 1, &g, NULL)) bad = 1;
            for (int r = 0; r < nrhs; ++r) {
                const double *wr = w + 2 * (size_t)r * n_tgt;
                nadd(&acc[r], g * (wr[2 * i] + I * wr[2 * i + 1]));
            }
        }
        for (int r = 0; r < nrhs; ++r) {
            cplx val = nval(&acc[r]);
            v[2 * ((size_t)r * n_src + j)] = creal(val);
            v[2 * ((size_t)r * n_src + j) + 1] = cimag(val);
        }
    }
    return bad ? ORC_EINVAL : ORC_OK;
}

/* Gradients of L = Re sum_r sum_i w[r][i] u[r][i], u = G q, with respect to
 * the coordinates.  dsrc: [2][n_src] (d/dx0, d/dy0), dtgt: [2][n_tgt]
 * (d/dx1, d/dy1).  Derivatives of the kernel are integrals of the same form
 * with the factor i*lam (x1), s2 (y1), -i*lam (x0), -s1 (y0). */
int orc_grad_coords(const double *med, int flags, const double *opt, long n_src, const double *src, const double *q,
                    long n_tgt, const double *tgt, const double *w, int nrhs, double *dsrc, double *dtgt,
                    int nthreads)
{
    if (n_src < 0 || n_tgt < 0 || nrhs < 1 || nrhs > 64) return ORC_EINVAL;
    medium_t m;
    opts_t o;
    read_medium(med, flags, &m);
    read_opts(opt, &o);
    int rc = check_layers(n_src, src, n_tgt, tgt, &m);
    if (rc) return rc;
    gl_init();
    set_threads(nthreads);
    int bad = 0;
    /* target-side derivatives: loop over targets */
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n_tgt; ++i) {
        nsum_t ax, ay;
        memset(&ax, 0, sizeof ax);
        memset(&ay, 0, sizeof ay);
        for (long j = 0; j < n_src; ++j) {
            cplx e[5];
            if (entry(tgt[i], tgt[n_tgt + i], src[j], src[n_src + j], &m, &o, 5, e, NULL)) bad = 1;
            for (int r = 0; r < nrhs; ++r) {
                const double *qr = q + 2 * (size_t)r * n_src;
                const double *wr = w + 2 * (size_t)r * n_tgt;
                cplx wq = (wr[2 * i] + I * wr[2 * i + 1]) * (qr[2 * j] + I * qr[2 * j + 1]);
                nadd(&ax, e[1] * wq);
                nadd(&ay, e[2] * wq);
            }
        }
        dtgt[i] = creal(nval(&ax));
        dtgt[n_tgt + i] = creal(nval(&ay));
    }
    /* source-side derivatives: loop over sources */
#pragma omp parallel for schedule(dynamic, 1)
    for (long j = 0; j < n_src; ++j) {
        nsum_t ax, ay;
        memset(&ax, 0, sizeof ax);
        memset(&ay, 0, sizeof ay);
        for (long i = 0; i < n_tgt; ++i) {
            cplx e[5];
            if (entry(tgt[i], tgt[n_tgt + i], src[j], src[n_src + j], &m, &o, 5, e, NULL)) bad = 1;
            for (int r = 0; r < nrhs; ++r) {
                const double *qr = q + 2 * (size_t)r * n_src;
                const double *wr = w + 2 * (size_t)r * n_tgt;
                cplx wq = (wr[2 * i] + I * wr[2 * i + 1]) * (qr[2 * j] + I * qr[2 * j + 1]);
                nadd(&ax, e[3] * wq);
                nadd(&ay, e[4] * wq);
            }
        }
        dsrc[j] = creal(nval(&ax));
        dsrc[n_src + j] = creal(nval(&ay));
    }
    return bad ? ORC_EINVAL : ORC_OK;
}
