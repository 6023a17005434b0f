/*
 * rc_oracle.c -- plain FP64 CPU reference of the forest-of-octrees raycasting
 * hot path (Burstedde, "Distributed-Memory Forest-of-Octrees Raycasting").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  It shares no code,
 * header, table or helper with the HIP library, and it computes everything in
 * double precision with straightforward loops.
 *
 * What it computes, per pixel p of a camera (the classic back-to-front result
 * written with the segment group operation of Sec. 2.4):
 *   1. every leaf whose projected pixel rectangle (Sec. 2.2, camera-aligned
 *      AABB projected to the image) contains p is intersected with p's ray;
 *   2. every hit gives a segment [s_in, s_out] and its (A, B) from the ODE
 *      I' = gamma - beta I (eq. Iode .. ABgeneral), either in closed form for
 *      constant coefficients (eq. ABconstant) or by explicit RK4 stages
 *      (eq. RKresultAB) over equal substeps combined with (+) (Sec. 2.4);
 *   3. the segments of p are SORTED by entry depth (allowed here: this is the
 *      definition the sort-free GPU fold must reproduce) and folded front to
 *      back with (A2,B2) (+) (A1,B1) = (A2 A1, B2 + A2 B1) (eq. aggregate);
 *   4. I = A * I_b + B (Sec. 2.4, final intensity).
 * Gradients use forward-mode dual numbers through step 2 and the product
 * structure of the fold in step 3.
 *
 * Readings of the paper that the text leaves open are fixed identically on
 * both implementations: the canonical rectangle and slab predicates below,
 * the orthographic ray, the corner numbering and the RK4 point placement.
 *
 * Parity: every function here is pinned by CPU tests against closed forms,
 * group identities, brute-force marching and finite differences.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_QMAX 19
#define OR_NPMAX 16
#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* group operations on segments (Sec. 2.4 - 2.6)                            */
/* ------------------------------------------------------------------------ */

/* (A2,B2) (+) (A1,B1): segment 2 is the one nearer to the camera (eq. aggregate). */
void or_combine(const double *near2, const double *far1, double *out)
{
    double A = near2[0] * far1[0];
    double B = near2[1] + near2[0] * far1[1];
    out[0] = A;
    out[1] = B;
}

/* (-)(A,B) = (1/A, -B/A) (eq. identityinverse). */
void or_inverse(const double *s, double *out)
{
    out[0] = 1.0 / s[0];
    out[1] = -s[1] / s[0];
}

/* Split (A,B) of length dx into pieces of length dx1 and dx - dx1 (eq. segsplit).
 * out1 is the piece of length dx1. */
void or_split(const double *s, double frac1, double *out1, double *out2)
{
    double A = s[0], B = s[1];
    double fr[2] = {frac1, 1.0 - frac1};
    double *o[2] = {out1, out2};
    for (int i = 0; i < 2; i++) {
        double Ai = pow(A, fr[i]);
        double Bi = (A == 1.0) ? B * fr[i] : B * (1.0 - Ai) / (1.0 - A);
        o[i][0] = Ai;
        o[i][1] = Bi;
    }
}

/* Average of two segments over the same interval (eq. segaverage). */
void or_average(const double *s1, const double *s2, double *out)
{
    out[0] = sqrt(s1[0] * s2[0]);
    out[1] = 0.5 * (s1[1] + s2[1]);
}

/* Constant coefficients equivalent to (A,B) over length dx (eq. betagammafromAB). */
void or_physical(const double *s, double dx, double *beta_gamma)
{
    double beta = -log(s[0]) / dx;
    double gamma = (s[0] == 1.0) ? s[1] / dx : beta * s[1] / (1.0 - s[0]);
    beta_gamma[0] = beta;
    beta_gamma[1] = gamma;
}

/* ------------------------------------------------------------------------ */
/* dual numbers: value plus np partial derivatives                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double v;
    double d[OR_NPMAX];
} dn;

static dn dn_c(double v, int np)
{
    dn r;
    r.v = v;
    for (int k = 0; k < np; k++) r.d[k] = 0.0;
    return r;
}
static dn dn_add(dn a, dn b, int np)
{
    dn r;
    r.v = a.v + b.v;
    for (int k = 0; k < np; k++) r.d[k] = a.d[k] + b.d[k];
    return r;
}
static dn dn_sub(dn a, dn b, int np)
{
    dn r;
    r.v = a.v - b.v;
    for (int k = 0; k < np; k++) r.d[k] = a.d[k] - b.d[k];
    return r;
}
static dn dn_mul(dn a, dn b, int np)
{
    dn r;
    r.v = a.v * b.v;
    for (int k = 0; k < np; k++) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
static dn dn_scale(dn a, double s, int np)
{
    dn r;
    r.v = a.v * s;
    for (int k = 0; k < np; k++) r.d[k] = a.d[k] * s;
    return r;
}
static dn dn_exp(dn a, int np)
{
    dn r;
    r.v = exp(a.v);
    for (int k = 0; k < np; k++) r.d[k] = r.v * a.d[k];
    return r;
}
static dn dn_div(dn a, dn b, int np)
{
    dn r;
    r.v = a.v / b.v;
    for (int k = 0; k < np; k++) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
static dn dn_sqrt(dn a, int np)
{
    dn r;
    r.v = sqrt(a.v);
    for (int k = 0; k < np; k++) r.d[k] = a.d[k] / (2.0 * r.v);
    return r;
}
/* phi(x) = (1 - e^{-x}) / x with phi(0) = 1, and its derivative. */
static dn dn_phi(dn x, int np)
{
    dn r;
    double v = x.v, f, df;
    if (fabs(v) < 1e-4) {
        /* Taylor: 1 - x/2 + x^2/6 - x^3/24 + x^4/120 */
        f = 1.0 - v / 2.0 + v * v / 6.0 - v * v * v / 24.0 + v * v * v * v / 120.0;
        df = -0.5 + v / 3.0 - v * v / 8.0 + v * v * v / 30.0;
    } else {
        double em = -expm1(-v); /* 1 - e^{-x} */
        f = em / v;
        df = (exp(-v) * v - em) / (v * v);
    }
    r.v = f;
    for (int k = 0; k < np; k++) r.d[k] = df * x.d[k];
    return r;
}

/* ------------------------------------------------------------------------ */
/* segment evaluation (Sec. 2.3 and 2.7)                                    */
/* ------------------------------------------------------------------------ */

/* Constant coefficients (eq. ABconstant): A = exp(-beta dx), B = gamma dx phi(beta dx). */
static void seg_const_dn(dn beta, dn gamma, double dx, int np, dn *A, dn *B)
{
    dn x = dn_scale(beta, dx, np);
    *A = dn_exp(dn_scale(x, -1.0, np), np);
    *B = dn_mul(dn_scale(gamma, dx, np), dn_phi(x, np), np);
}

/* One explicit RK step for the two ODEs of eq. ODEsAB from (A,B) = (1,0), with
 * the stage values of eq. RKresultAB for the classical RK4 tableau:
 * c = (0, 1/2, 1/2, 1), a10 = a21 = 1/2, a32 = 1, b = (1/6, 1/3, 1/3, 1/6).
 * beta[i], gamma[i] are the coefficients at xi_i = x1 + c_i h (x1 = far end). */
static void rk4_step_dn(const dn *beta, const dn *gamma, double h, int np, dn *Aout, dn *Bout)
{
    static const double a[5][4] = {
        {0.0, 0.0, 0.0, 0.0},
        {0.5, 0.0, 0.0, 0.0},
        {0.0, 0.5, 0.0, 0.0},
        {0.0, 0.0, 1.0, 0.0},
        {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}, /* final row a_Mj = b_j */
    };
    dn Ab[5], Bb[5];
    for (int i = 0; i <= 4; i++) {
        dn sa = dn_c(0.0, np), sb = dn_c(0.0, np);
        for (int j = 0; j < i; j++) {
            if (a[i][j] == 0.0) continue;
            dn fa = dn_scale(dn_mul(beta[j], Ab[j], np), -1.0, np);       /* -beta A */
            dn fb = dn_sub(gamma[j], dn_mul(beta[j], Bb[j], np), np);     /* gamma - beta B */
            sa = dn_add(sa, dn_scale(fa, a[i][j], np), np);
            sb = dn_add(sb, dn_scale(fb, a[i][j], np), np);
        }
        Ab[i] = dn_add(dn_c(1.0, np), dn_scale(sa, h, np), np);
        Bb[i] = dn_scale(sb, h, np);
    }
    *Aout = Ab[4];
    *Bout = Bb[4];
}

void or_rk4_step(const double *beta4, const double *gamma4, double h, double *AB)
{
    dn b[4], g[4], A, B;
    for (int i = 0; i < 4; i++) {
        b[i] = dn_c(beta4[i], 0);
        g[i] = dn_c(gamma4[i], 0);
    }
    rk4_step_dn(b, g, h, 0, &A, &B);
    AB[0] = A.v;
    AB[1] = B.v;
}

/* Trilinear interpolation of 8 corner values (corner c = bx + 2 by + 4 bz) at
 * reference coordinates xi in [0,1]^3; the corner values are the parameters
 * p0 .. p0+7 of the dual numbers when np > 0. */
static dn trilin_dn(const double *cv, const double *xi, int np, int p0)
{
    dn r = dn_c(0.0, np);
    for (int c = 0; c < 8; c++) {
        double w = 1.0;
        for (int k = 0; k < 3; k++) w *= ((c >> k) & 1) ? xi[k] : 1.0 - xi[k];
        r.v += cv[c] * w;
        if (np > 0) r.d[p0 + c] += w;
    }
    return r;
}

/* Leaf geometry in the unit cube. */
typedef struct {
    double lo[3], hi[3], hlen;
} leafbox;

static leafbox leaf_box(uint8_t level, uint32_t x, uint32_t y, uint32_t z)
{
    leafbox b;
    double q = ldexp(1.0, -OR_QMAX);
    uint32_t len = (uint32_t)1 << (OR_QMAX - level);
    uint32_t a[3] = {x, y, z};
    for (int k = 0; k < 3; k++) {
        b.lo[k] = (double)a[k] * q;
        b.hi[k] = (double)(a[k] + len) * q;
    }
    b.hlen = ldexp(1.0, -(int)level);
    return b;
}

/* Field evaluation context for one leaf. */
typedef struct {
    int kind;          /* 0: constant per leaf, 1: trilinear corners */
    double kap[8], eps[8];
} leaffield;

/* Leaf reference coordinates of a real-space point. */
typedef void (*ref_fn)(const void *ctx, const double *x, double *xi);

static void cube_ref(const void *ctx, const double *x, double *xi)
{
    const leafbox *bx = (const leafbox *)ctx;
    for (int k = 0; k < 3; k++) xi[k] = (x[k] - bx->lo[k]) / bx->hlen;
}

/* Segment [s_in, s_out] of ray x(s) = rho + s r inside a leaf, integrated from
 * the far end s_out toward the camera.  Returns (A,B) as dual numbers over the
 * leaf's parameters: kappa corners 0..nc-1 then eps corners nc..2nc-1. */
static void segment_dn_ref(const leaffield *F, ref_fn ref, const void *ctx, const double *rho, const double *r,
                           double rnorm, double s_in, double s_out, int method, int substeps, double c_rk, int np,
                           dn *Aout, dn *Bout);

static void segment_dn(const leaffield *F, const leafbox *bx, const double *rho, const double *r,
                       double rnorm, double s_in, double s_out, int method, int substeps, double c_rk, int np,
                       dn *Aout, dn *Bout)
{
    segment_dn_ref(F, cube_ref, bx, rho, r, rnorm, s_in, s_out, method, substeps, c_rk, np, Aout, Bout);
}

/* Coefficients at ray parameter s (Sec. 2.3): trilinear in the leaf's reference
 * coordinates (kind 1) or constant per leaf; kind 2 holds the equilibrium
 * intensity I = gamma / beta of eq. BIrelation in place of gamma, so that
 * gamma = beta I.  Dual parts: kappa parameters first, then eps (or I). */
static void field_dn(const leaffield *F, ref_fn ref, const void *ctx, const double *rho, const double *r, double s,
                     int np, dn *beta, dn *gamma)
{
    int nc = F->kind == 1 ? 8 : 1;
    if (F->kind == 1) {
        double xi[3], pt[3];
        for (int k = 0; k < 3; k++) pt[k] = rho[k] + s * r[k];
        ref(ctx, pt, xi);
        *beta = trilin_dn(F->kap, xi, np, 0);
        *gamma = trilin_dn(F->eps, xi, np, nc);
        return;
    }
    dn e = dn_c(F->eps[0], np);
    *beta = dn_c(F->kap[0], np);
    if (np > 0) {
        beta->d[0] = 1.0;
        e.d[nc] = 1.0;
    }
    *gamma = F->kind == 2 ? dn_mul(*beta, e, np) : e;
}

/* ------------------------------------------------------------------------ */
/* integrators over dyadic pieces of a segment (Sec. 2.7)                   */
/* ------------------------------------------------------------------------ */

#define OR_ADAPT_MAXDEPTH 16

typedef struct {
    const leaffield *F;
    ref_fn ref;
    const void *ctx;
    const double *rho, *r;
    double rnorm, s_in, s_out, c_rk;
    int method, np;
} segjob;

/* Stage positions c_i of each method, measured from the far end x1 of a piece
 * (xi_i = x1 + c_i dx): RK4 (0, 1/2, 1/2, 1), Gauss (1/2 -+ sqrt(3)/6),
 * Simpson (0, 1/2, 1). */
static int stage_c(int method, double *c)
{
    if (method == 1) {
        c[0] = 0.0; c[1] = 0.5; c[2] = 0.5; c[3] = 1.0;
        return 4;
    }
    if (method == 2) {
        c[0] = 0.5 - sqrt(3.0) / 6.0;
        c[1] = 0.5 + sqrt(3.0) / 6.0;
        return 2;
    }
    c[0] = 0.0; c[1] = 0.5; c[2] = 1.0;
    return 3;
}

/* Piece k of depth d covers the fraction [k, k+1] / 2^d of the segment,
 * counted from its near end; s(u) = s_in + u (s_out - s_in). */
static double piece_s(const segjob *J, int64_t k, int d, double c)
{
    double u = ((double)(k + 1) - c) * ldexp(1.0, -d);
    return J->s_in + u * (J->s_out - J->s_in);
}

static double piece_dx(const segjob *J, int64_t k, int d)
{
    return (piece_s(J, k, d, 0.0) - piece_s(J, k, d, 1.0)) * J->rnorm;
}

/* One step of the method over piece (k, d), from (A, B) = (1, 0). */
static void piece_step(const segjob *J, int64_t k, int d, dn *A, dn *B)
{
    int np = J->np;
    double c[4], dx = piece_dx(J, k, d);
    int m = stage_c(J->method, c);
    dn be[4], ga[4];
    for (int i = 0; i < m; i++) field_dn(J->F, J->ref, J->ctx, J->rho, J->r, piece_s(J, k, d, c[i]), np, &be[i], &ga[i]);
    if (J->method == 1) {
        rk4_step_dn(be, ga, dx, np, A, B);
    } else if (J->method == 2) {
        /* implicit Gauss, 2 stages (eq. gaussAB, eq. gaussABab) */
        dn a1 = dn_scale(dn_add(be[0], be[1], np), dx / 4.0, np);
        dn a2 = dn_scale(dn_mul(be[0], be[1], np), dx * dx / 12.0, np);
        dn b1 = dn_scale(dn_add(ga[0], ga[1], np), dx / 2.0, np);
        dn b2 = dn_scale(dn_sub(dn_mul(be[0], ga[1], np), dn_mul(be[1], ga[0], np), np), dx * dx * sqrt(3.0) / 12.0,
                         np);
        dn den = dn_add(dn_add(dn_c(1.0, np), a1, np), a2, np);
        *A = dn_div(dn_add(dn_sub(dn_c(1.0, np), a1, np), a2, np), den, np);
        *B = dn_div(dn_add(b1, b2, np), den, np);
    } else {
        /* Simpson quadrature of the closed form (eq. simpson), weights 1/6, 4/6, 1/6 */
        dn sb = dn_add(dn_add(be[0], dn_scale(be[1], 4.0, np), np), be[2], np);
        *A = dn_exp(dn_scale(sb, -dx / 6.0, np), np);
        dn t0 = dn_mul(*A, ga[0], np);
        dn t1 = dn_scale(dn_mul(dn_sqrt(*A, np), ga[1], np), 4.0, np);
        *B = dn_scale(dn_add(dn_add(t0, t1, np), ga[2], np), dx / 6.0, np);
    }
}

/* Alg. adaptiverk: a piece whose stage coefficients give dx beta(xi_i) > c_RK
 * is replaced by its two halves, the nearer one on the left of (+). */
static void piece_eval(const segjob *J, int64_t k, int d, dn *A, dn *B)
{
    if (J->c_rk > 0.0 && d < OR_ADAPT_MAXDEPTH) {
        double c[4], dx = piece_dx(J, k, d);
        int m = stage_c(J->method, c), split = 0;
        for (int i = 0; i < m && !split; i++) {
            dn be, ga;
            field_dn(J->F, J->ref, J->ctx, J->rho, J->r, piece_s(J, k, d, c[i]), 0, &be, &ga);
            if (dx * be.v > J->c_rk) split = 1;
        }
        if (split) {
            int np = J->np;
            dn An, Bn, Af, Bf;
            piece_eval(J, 2 * k, d + 1, &An, &Bn);
            piece_eval(J, 2 * k + 1, d + 1, &Af, &Bf);
            *A = dn_mul(An, Af, np);
            *B = dn_add(Bn, dn_mul(An, Bf, np), np);
            return;
        }
    }
    piece_step(J, k, d, A, B);
}

static void segment_dn_ref(const leaffield *F, ref_fn ref, const void *ctx, const double *rho, const double *r,
                           double rnorm, double s_in, double s_out, int method, int substeps, double c_rk, int np,
                           dn *Aout, dn *Bout)
{
    int nc = F->kind == 1 ? 8 : 1;
    if (method == 0) {
        /* analytic: constant coefficients, eq. ABconstant (kind 2: gamma = beta I) */
        dn beta, gamma;
        field_dn(F, ref, ctx, rho, r, s_in, np, &beta, &gamma);
        seg_const_dn(beta, gamma, (s_out - s_in) * rnorm, np, Aout, Bout);
        return;
    }
    if (method == 1 && c_rk <= 0.0) {
        /* RK4 over `substeps` equal substeps, farthest first, combined with (+). */
        double ds = (s_out - s_in) / substeps;
        double h = ds * rnorm;
        dn A = dn_c(1.0, np), B = dn_c(0.0, np);
        for (int q = 0; q < substeps; q++) {
            double s_far = s_out - q * ds;
            double sp[4] = {s_far, s_far - 0.5 * ds, s_far - 0.5 * ds, s_far - ds};
            dn beta[4], gamma[4];
            for (int i = 0; i < 4; i++) field_dn(F, ref, ctx, rho, r, sp[i], np, &beta[i], &gamma[i]);
            dn a, b;
            rk4_step_dn(beta, gamma, h, np, &a, &b);
            /* (A,B) <- (a,b) (+) (A,B): the new substep is nearer to the camera */
            dn nA = dn_mul(a, A, np);
            dn nB = dn_add(b, dn_mul(a, B, np), np);
            A = nA;
            B = nB;
        }
        *Aout = A;
        *Bout = B;
        return;
    }
    /* RK4 with recursion, Gauss or Simpson: `substeps` = 2^d0 equal pieces, each
     * evaluated by piece_eval, combined nearest first. */
    (void)nc;
    segjob J = {F, ref, ctx, rho, r, rnorm, s_in, s_out, c_rk, method, np};
    int d0 = 0;
    while ((1 << d0) < substeps) d0++;
    dn A = dn_c(1.0, np), B = dn_c(0.0, np);
    for (int64_t k = 0; k < ((int64_t)1 << d0); k++) {
        dn a, b;
        piece_eval(&J, k, d0, &a, &b);
        dn nA = dn_mul(A, a, np);
        dn nB = dn_add(B, dn_mul(A, b, np), np);
        A = nA;
        B = nB;
    }
    *Aout = A;
    *Bout = B;
}

/* ------------------------------------------------------------------------ */
/* camera (Sec. 2.2) and the canonical visibility / pairing predicates      */
/* ------------------------------------------------------------------------ */

typedef struct {
    double o[3], v[3], t[3], u[3], ell, zfar, bg;
    int w, h, ortho;
    /* derived */
    double n, vh[3], sc, cx, cy, smin, smax;
} orcam;

static void cam_parse(const double *raw, orcam *c)
{
    for (int k = 0; k < 3; k++) {
        c->o[k] = raw[k];
        c->v[k] = raw[3 + k];
        c->t[k] = raw[6 + k];
        c->u[k] = raw[9 + k];
    }
    c->ell = raw[12];
    c->zfar = raw[13];
    c->w = (int)raw[14];
    c->h = (int)raw[15];
    c->ortho = raw[16] != 0.0;
    c->bg = raw[17];
    c->n = sqrt((c->v[0] * c->v[0] + c->v[1] * c->v[1]) + c->v[2] * c->v[2]);
    for (int k = 0; k < 3; k++) c->vh[k] = c->v[k] / c->n;
    c->sc = c->n / c->ell;
    c->cx = (c->w - 1) / 2.0;
    c->cy = (c->h - 1) / 2.0;
    c->smin = c->ortho ? c->n : 1.0;
    c->smax = c->ortho ? c->zfar : c->zfar / c->n;
}

/* extremes of a . (x - o) over the box [lo, hi] */
static double box_dot_min(const double *a, const double *lo, const double *hi, const double *o)
{
    double s0 = a[0] * ((a[0] >= 0.0 ? lo[0] : hi[0]) - o[0]);
    double s1 = a[1] * ((a[1] >= 0.0 ? lo[1] : hi[1]) - o[1]);
    double s2 = a[2] * ((a[2] >= 0.0 ? lo[2] : hi[2]) - o[2]);
    return (s0 + s1) + s2;
}
static double box_dot_max(const double *a, const double *lo, const double *hi, const double *o)
{
    double s0 = a[0] * ((a[0] >= 0.0 ? hi[0] : lo[0]) - o[0]);
    double s1 = a[1] * ((a[1] >= 0.0 ? hi[1] : lo[1]) - o[1]);
    double s2 = a[2] * ((a[2] >= 0.0 ? hi[2] : lo[2]) - o[2]);
    return (s0 + s1) + s2;
}

/* Pixel interval [k0, k1] covered by camera-space extent [X0, X1] at clipped
 * depths [Z0, Z1] (perspective) or directly (orthographic). */
static void pixel_range(const orcam *c, double X0, double X1, double Z0, double Z1, double center,
                        int npx, int *k0, int *k1)
{
    double p0, p1;
    if (c->ortho) {
        p0 = X0 / c->ell + center;
        p1 = X1 / c->ell + center;
    } else {
        double q0 = (X0 >= 0.0) ? X0 / Z1 : X0 / Z0;
        double q1 = (X1 >= 0.0) ? X1 / Z0 : X1 / Z1;
        p0 = q0 * c->sc + center;
        p1 = q1 * c->sc + center;
    }
    double a = ceil(p0), b = floor(p1);
    if (a < 0.0) a = 0.0;
    if (b > (double)(npx - 1)) b = (double)(npx - 1);
    if (a > b) {
        *k0 = 1;
        *k1 = 0;
    } else {
        *k0 = (int)a;
        *k1 = (int)b;
    }
}

/* Pixel rectangle of a box: camera-aligned AABB (eq. camerageometry applied to
 * the box), clipped to depth [n, f], projected to the image.  Returns 1 if the
 * rectangle holds at least one pixel centre. */
static int box_rect(const orcam *c, const double *lo, const double *hi, int *rect)
{
    double Z0 = box_dot_min(c->vh, lo, hi, c->o), Z1 = box_dot_max(c->vh, lo, hi, c->o);
    rect[0] = 1;
    rect[1] = 0;
    rect[2] = 1;
    rect[3] = 0;
    if (Z1 < c->n || Z0 > c->zfar) return 0;
    double Zc0 = Z0 < c->n ? c->n : Z0;
    double Zc1 = Z1 > c->zfar ? c->zfar : Z1;
    double X0 = box_dot_min(c->t, lo, hi, c->o), X1 = box_dot_max(c->t, lo, hi, c->o);
    double Y0 = box_dot_min(c->u, lo, hi, c->o), Y1 = box_dot_max(c->u, lo, hi, c->o);
    int i0, i1, j0, j1;
    pixel_range(c, X0, X1, Zc0, Zc1, c->cx, c->w, &i0, &i1);
    pixel_range(c, Y0, Y1, Zc0, Zc1, c->cy, c->h, &j0, &j1);
    if (i0 > i1 || j0 > j1) return 0;
    rect[0] = i0;
    rect[1] = i1;
    rect[2] = j0;
    rect[3] = j1;
    return 1;
}

/* Ray of pixel (i, j): x(s) = rho + s r (eq. ray; orthographic variant shifts the origin). */
static void pixel_ray(const orcam *c, int i, int j, double *rho, double *r)
{
    double a = c->ell * ((double)i - c->cx);
    double b = c->ell * ((double)j - c->cy);
    for (int k = 0; k < 3; k++) {
        double off = a * c->t[k] + b * c->u[k];
        if (c->ortho) {
            rho[k] = c->o[k] + off;
            r[k] = c->vh[k];
        } else {
            rho[k] = c->o[k];
            r[k] = c->v[k] + off;
        }
    }
}

/* Slab test of a ray against a box, clipped to [smin, smax].  Returns 1 on a
 * hit of positive length.  Each face value enters through (face - rho) * inv,
 * so boxes sharing a face share the crossing parameter bit for bit. */
static int slab(const orcam *c, const double *rho, const double *r, const double *lo, const double *hi,
                double *s_in, double *s_out)
{
    double a = c->smin, b = c->smax;
    for (int k = 0; k < 3; k++) {
        if (r[k] != 0.0) {
            double inv = 1.0 / r[k];
            double t0 = (lo[k] - rho[k]) * inv;
            double t1 = (hi[k] - rho[k]) * inv;
            double tmin = t0 < t1 ? t0 : t1, tmax = t0 < t1 ? t1 : t0;
            if (tmin > a) a = tmin;
            if (tmax < b) b = tmax;
        } else if (!(rho[k] >= lo[k] && rho[k] < hi[k])) {
            return 0;
        }
    }
    *s_in = a;
    *s_out = b;
    return b > a;
}

static double ray_norm(const double *r)
{
    return sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
}

/* ------------------------------------------------------------------------ */
/* exported: visibility                                                     */
/* ------------------------------------------------------------------------ */

/* Pixel rectangle of every leaf for every camera: rect[cam][leaf][4] =
 * (i0, i1, j0, j1), empty as (1, 0, 1, 0).  Returns the number of visible pairs. */
int64_t or_prune(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
                 int ncams, const double *cams, int32_t *rect)
{
    int64_t nvis = 0;
    for (int ci = 0; ci < ncams; ci++) {
        orcam c;
        cam_parse(cams + 20 * ci, &c);
        for (int64_t l = 0; l < n; l++) {
            leafbox b = leaf_box(level[l], x[l], y[l], z[l]);
            int rr[4];
            nvis += box_rect(&c, b.lo, b.hi, rr);
            for (int k = 0; k < 4; k++) rect[((int64_t)ci * n + l) * 4 + k] = rr[k];
        }
    }
    return nvis;
}

/* Rectangle of an arbitrary node (level, anchor): used to pin nesting. */
int or_node_rect(int level, uint32_t x, uint32_t y, uint32_t z, const double *cam, int32_t *rect)
{
    orcam c;
    cam_parse(cam, &c);
    leafbox b = leaf_box((uint8_t)level, x, y, z);
    int rr[4];
    int vis = box_rect(&c, b.lo, b.hi, rr);
    for (int k = 0; k < 4; k++) rect[k] = rr[k];
    return vis;
}

/* Pairing of the candidates of the listed leaves: for leaf list[m] and each
 * pixel of its rectangle in row-major order, hit[q] in {0,1} and the interval
 * (sio[2q], sio[2q+1]) (zeros on a miss).  Returns the number of candidates. */
int64_t or_pairs(int64_t nlist, const int64_t *list, const uint8_t *level, const uint32_t *x,
                 const uint32_t *y, const uint32_t *z, const double *cam, uint8_t *hit, double *sio,
                 int64_t cap)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t q = 0;
    for (int64_t m = 0; m < nlist; m++) {
        int64_t l = list[m];
        leafbox b = leaf_box(level[l], x[l], y[l], z[l]);
        int rr[4];
        if (!box_rect(&c, b.lo, b.hi, rr)) continue;
        for (int j = rr[2]; j <= rr[3]; j++)
            for (int i = rr[0]; i <= rr[1]; i++) {
                if (q < cap) {
                    double rho[3], r[3], a = 0, bb = 0;
                    pixel_ray(&c, i, j, rho, r);
                    int h = slab(&c, rho, r, b.lo, b.hi, &a, &bb);
                    hit[q] = (uint8_t)h;
                    sio[2 * q] = h ? a : 0.0;
                    sio[2 * q + 1] = h ? bb : 0.0;
                }
                q++;
            }
    }
    return q;
}

/* ------------------------------------------------------------------------ */
/* exported: rendering and gradients                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t pix;   /* selected-pixel index */
    double s_in, s_out;
    int64_t leaf;
    double A, B;
} orseg;

static int seg_cmp(const void *pa, const void *pb)
{
    const orseg *a = (const orseg *)pa, *b = (const orseg *)pb;
    if (a->pix != b->pix) return a->pix < b->pix ? -1 : 1;
    if (a->s_in != b->s_in) return a->s_in < b->s_in ? -1 : 1;
    if (a->s_out != b->s_out) return a->s_out < b->s_out ? -1 : 1;
    return 0;
}

static void leaf_field(int kind, int64_t n, int64_t l, const double *kap, const double *eps, leaffield *F)
{
    F->kind = kind;
    int nc = kind == 1 ? 8 : 1;
    for (int c = 0; c < nc; c++) {
        F->kap[c] = kap[(int64_t)c * n + l];
        F->eps[c] = eps[(int64_t)c * n + l];
    }
}

/* Gather all segments of the selected pixels (all pixels when npix_sel < 0). */
static orseg *gather(const orcam *c, int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y,
                     const uint32_t *z, int64_t npix_sel, const int64_t *pix_sel, int64_t *nseg_out)
{
    int64_t W = c->w, H = c->h, P = W * H;
    int64_t *selmap = NULL;
    if (npix_sel >= 0) {
        selmap = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);
        for (int64_t p = 0; p < P; p++) selmap[p] = -1;
        for (int64_t q = 0; q < npix_sel; q++) selmap[pix_sel[q]] = q;
    }
    int64_t cap = 1 << 16, ns = 0;
    orseg *segs = (orseg *)malloc(sizeof(orseg) * (size_t)cap);
    for (int64_t l = 0; l < n; l++) {
        leafbox b = leaf_box(level[l], x[l], y[l], z[l]);
        int rr[4];
        if (!box_rect(c, b.lo, b.hi, rr)) continue;
        for (int j = rr[2]; j <= rr[3]; j++)
            for (int i = rr[0]; i <= rr[1]; i++) {
                int64_t p = (int64_t)j * W + i, ps = p;
                if (selmap) {
                    ps = selmap[p];
                    if (ps < 0) continue;
                }
                double rho[3], r[3], a, bb;
                pixel_ray(c, i, j, rho, r);
                if (!slab(c, rho, r, b.lo, b.hi, &a, &bb)) continue;
                if (ns == cap) {
                    cap *= 2;
                    segs = (orseg *)realloc(segs, sizeof(orseg) * (size_t)cap);
                }
                segs[ns].pix = ps;
                segs[ns].s_in = a;
                segs[ns].s_out = bb;
                segs[ns].leaf = l;
                ns++;
            }
    }
    free(selmap);
    qsort(segs, (size_t)ns, sizeof(orseg), seg_cmp);
    *nseg_out = ns;
    return segs;
}

static void selected_ij(const orcam *c, int64_t npix_sel, const int64_t *pix_sel, int64_t q, int *i, int *j)
{
    int64_t p = (npix_sel >= 0) ? pix_sel[q] : q;
    *i = (int)(p % c->w);
    *j = (int)(p / c->w);
}

/*
 * Render one camera.  kap/eps: [nc][n] doubles (nc = 8 for kind 1, else 1; kind 2
 * holds the equilibrium intensity I in eps).  method 0 = analytic (constant),
 * 1 = RK4, 2 = implicit Gauss (2 stages), 3 = Simpson, over `substeps` equal
 * substeps (a power of two for methods 2, 3 and for c_rk > 0); c_rk > 0 turns
 * on the recursion of Alg. adaptiverk with that stability parameter.
 * Pixels: all (npix_sel < 0, outputs have w*h entries, row j = 0 at the bottom)
 * or the listed pixel indices p = j*w + i (outputs have npix_sel entries).
 * stats[0] = segments, stats[1] = overlaps beyond 1e-12 relative,
 * stats[2] = candidates tested.  Returns 0.
 */
int or_render(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
              int kind, const double *kap, const double *eps, int method, int substeps, double c_rk,
              const double *cam, int64_t npix_sel, const int64_t *pix_sel, double *Aout, double *Bout, double *Iout,
              int32_t *nseg_pix, int64_t *stats)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t npo = (npix_sel >= 0) ? npix_sel : (int64_t)c.w * c.h;
    int64_t ns = 0;
    orseg *segs = gather(&c, n, level, x, y, z, npix_sel, pix_sel, &ns);

#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < ns; k++) {
        orseg *s = &segs[k];
        int i, j;
        selected_ij(&c, npix_sel, pix_sel, s->pix, &i, &j);
        double rho[3], r[3];
        pixel_ray(&c, i, j, rho, r);
        leafbox b = leaf_box(level[s->leaf], x[s->leaf], y[s->leaf], z[s->leaf]);
        leaffield F;
        leaf_field(kind, n, s->leaf, kap, eps, &F);
        dn A, B;
        segment_dn(&F, &b, rho, r, ray_norm(r), s->s_in, s->s_out, method, substeps, c_rk, 0, &A, &B);
        s->A = A.v;
        s->B = B.v;
    }

    int64_t overlaps = 0;
    for (int64_t q = 0; q < npo; q++) {
        Aout[q] = 1.0;
        Bout[q] = 0.0;
        if (nseg_pix) nseg_pix[q] = 0;
    }
    int64_t k = 0;
    while (k < ns) {
        int64_t q = segs[k].pix;
        double acc[2] = {1.0, 0.0};
        double prev_out = -INFINITY;
        int cnt = 0;
        for (; k < ns && segs[k].pix == q; k++) {
            if (segs[k].s_in < prev_out - 1e-12 * fabs(prev_out)) overlaps++;
            prev_out = segs[k].s_out;
            double sg[2] = {segs[k].A, segs[k].B}, t[2];
            or_combine(acc, sg, t); /* acc is nearer: acc (+) next */
            acc[0] = t[0];
            acc[1] = t[1];
            cnt++;
        }
        Aout[q] = acc[0];
        Bout[q] = acc[1];
        if (nseg_pix) nseg_pix[q] = cnt;
    }
    for (int64_t q = 0; q < npo; q++) Iout[q] = Aout[q] * c.bg + Bout[q];
    if (stats) {
        stats[0] = ns;
        stats[1] = overlaps;
    }
    free(segs);
    return 0;
}

/*
 * Gradient of a pixel loss: given g[p] = dL/dI_p for the selected pixels,
 * accumulate dL/dkappa and dL/deps ([nc][n], overwritten) through
 *   I = sum_k T_k B_k + T_{m+1} I_b,   T_k = prod_{j<k} A_j (front to back),
 * so dI/dB_k = T_k and dI/dA_k = T_k J_k with J_k the intensity entering
 * segment k from behind; segment derivatives come from dual numbers.
 */
static int grad_sum(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
                    int kind, const double *kap, const double *eps, int method, int substeps, double c_rk,
                    const double *cam, int64_t npix_sel, const int64_t *pix_sel, const double *g, double *gk,
                    double *ge, int absolute);

int or_grad(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
            int kind, const double *kap, const double *eps, int method, int substeps, double c_rk,
            const double *cam, int64_t npix_sel, const int64_t *pix_sel, const double *g, double *gk, double *ge)
{
    return grad_sum(n, level, x, y, z, kind, kap, eps, method, substeps, c_rk, cam, npix_sel, pix_sel, g, gk, ge, 0);
}

/*
 * Weighted absolute sensitivities: for weights g[p] >= 0, gk and ge receive
 * sum_p g[p] |dI_p / dtheta| for every coefficient theta, with the same
 * segments, fold factors and dual numbers as or_grad.  A leaf meets a pixel's
 * ray in at most one segment, so each term is one segment's contribution.
 * This bounds |sum_p dg_p dI_p/dtheta| for any per-pixel perturbation with
 * |dg_p| <= g[p] (the triangle inequality).  Returns -1 on a negative weight.
 */
int or_grad_abs(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
                int kind, const double *kap, const double *eps, int method, int substeps, double c_rk,
                const double *cam, int64_t npix_sel, const int64_t *pix_sel, const double *g, double *gk,
                double *ge)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t m = npix_sel >= 0 ? npix_sel : (int64_t)c.w * c.h;
    for (int64_t q = 0; q < m; q++)
        if (!(g[q] >= 0.0)) return -1;
    return grad_sum(n, level, x, y, z, kind, kap, eps, method, substeps, c_rk, cam, npix_sel, pix_sel, g, gk, ge, 1);
}

static int grad_sum(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
                    int kind, const double *kap, const double *eps, int method, int substeps, double c_rk,
                    const double *cam, int64_t npix_sel, const int64_t *pix_sel, const double *g, double *gk,
                    double *ge, int absolute)
{
    orcam c;
    cam_parse(cam, &c);
    int nc = kind == 1 ? 8 : 1, np = 2 * nc;
    int64_t ns = 0;
    orseg *segs = gather(&c, n, level, x, y, z, npix_sel, pix_sel, &ns);
    for (int64_t q = 0; q < (int64_t)nc * n; q++) {
        gk[q] = 0.0;
        ge[q] = 0.0;
    }
    /* values */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < ns; k++) {
        orseg *s = &segs[k];
        int i, j;
        selected_ij(&c, npix_sel, pix_sel, s->pix, &i, &j);
        double rho[3], r[3];
        pixel_ray(&c, i, j, rho, r);
        leafbox b = leaf_box(level[s->leaf], x[s->leaf], y[s->leaf], z[s->leaf]);
        leaffield F;
        leaf_field(kind, n, s->leaf, kap, eps, &F);
        dn A, B;
        segment_dn(&F, &b, rho, r, ray_norm(r), s->s_in, s->s_out, method, substeps, c_rk, 0, &A, &B);
        s->A = A.v;
        s->B = B.v;
    }
    /* per pixel: T (front product) and J (intensity from behind) per segment */
    double *dIdA = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1));
    double *dIdB = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1));
    int64_t k = 0;
    while (k < ns) {
        int64_t k0 = k, q = segs[k].pix;
        while (k < ns && segs[k].pix == q) k++;
        double J = c.bg;
        for (int64_t m = k - 1; m >= k0; m--) { /* back to front: J_m */
            dIdA[m] = J;                        /* temporarily J_m */
            J = segs[m].B + segs[m].A * J;
        }
        double T = 1.0;
        for (int64_t m = k0; m < k; m++) {
            double gp = g[q];
            dIdA[m] = gp * T * dIdA[m];
            dIdB[m] = gp * T;
            T *= segs[m].A;
        }
    }
    /* chain rule through each segment's dual numbers (serial accumulation) */
    for (int64_t m = 0; m < ns; m++) {
        orseg *s = &segs[m];
        int i, j;
        selected_ij(&c, npix_sel, pix_sel, s->pix, &i, &j);
        double rho[3], r[3];
        pixel_ray(&c, i, j, rho, r);
        leafbox b = leaf_box(level[s->leaf], x[s->leaf], y[s->leaf], z[s->leaf]);
        leaffield F;
        leaf_field(kind, n, s->leaf, kap, eps, &F);
        dn A, B;
        segment_dn(&F, &b, rho, r, ray_norm(r), s->s_in, s->s_out, method, substeps, c_rk, np, &A, &B);
        for (int p = 0; p < nc; p++) {
            double tk = dIdA[m] * A.d[p] + dIdB[m] * B.d[p];
            double te = dIdA[m] * A.d[nc + p] + dIdB[m] * B.d[nc + p];
            gk[(int64_t)p * n + s->leaf] += absolute ? fabs(tk) : tk;
            ge[(int64_t)p * n + s->leaf] += absolute ? fabs(te) : te;
        }
    }
    free(dIdA);
    free(dIdB);
    free(segs);
    return 0;
}

/* Value and gradient of one segment for a single leaf (exposed for pins):
 * AB[2] and dAB[2][np] with np = 2 * nc. */
int or_segment(int kind, const double *kap, const double *eps, uint8_t level, uint32_t x, uint32_t y,
               uint32_t z, const double *rho, const double *r, double s_in, double s_out, int method,
               int substeps, double c_rk, double *AB, double *dAB)
{
    leafbox b = leaf_box(level, x, y, z);
    leaffield F;
    F.kind = kind;
    int nc = kind == 1 ? 8 : 1, np = 2 * nc;
    for (int cc = 0; cc < nc; cc++) {
        F.kap[cc] = kap[cc];
        F.eps[cc] = eps[cc];
    }
    dn A, B;
    segment_dn(&F, &b, rho, r, ray_norm(r), s_in, s_out, method, substeps, c_rk, np, &A, &B);
    AB[0] = A.v;
    AB[1] = B.v;
    if (dAB)
        for (int p = 0; p < np; p++) {
            dAB[p] = A.d[p];
            dAB[np + p] = B.d[p];
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* exported: brute-force marcher (independent of pairing and the fold)      */
/* ------------------------------------------------------------------------ */

/* Point location by scanning every leaf (tiny meshes only). */
static int64_t locate(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
                      const double *p, leafbox *out)
{
    for (int64_t l = 0; l < n; l++) {
        leafbox b = leaf_box(level[l], x[l], y[l], z[l]);
        if (p[0] >= b.lo[0] && p[0] < b.hi[0] && p[1] >= b.lo[1] && p[1] < b.hi[1] && p[2] >= b.lo[2] &&
            p[2] < b.hi[2]) {
            *out = b;
            return l;
        }
    }
    return -1;
}

/*
 * March every pixel's ray through the unit cube in M equal steps (midpoint
 * rule): each step takes the coefficients at its midpoint as constant, uses
 * eq. ABconstant, and is folded front to back.  Converges to the exact
 * integral as M grows; shares neither pairing nor tree order with or_render.
 */
/* ------------------------------------------------------------------------ */
/* one process's share: maximal complete subtrees and per-pixel lists       */
/* (Sec. 3.3 coarsening to the share's maximal subtrees, Sec. 3.5 lists,    */
/* Sec. 2.5 cutting and averaging overlapping segments)                     */
/* ------------------------------------------------------------------------ */

static uint64_t key_of(uint32_t x, uint32_t y, uint32_t z)
{
    uint64_t k = 0;
    for (int b = 0; b < OR_QMAX; b++) {
        k |= (uint64_t)((x >> b) & 1u) << (3 * b);
        k |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        k |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
    }
    return k;
}

static void anchor_of(uint64_t k, uint32_t *x, uint32_t *y, uint32_t *z)
{
    *x = *y = *z = 0;
    for (int b = 0; b < OR_QMAX; b++) {
        *x |= (uint32_t)((k >> (3 * b)) & 1u) << b;
        *y |= (uint32_t)((k >> (3 * b + 1)) & 1u) << b;
        *z |= (uint32_t)((k >> (3 * b + 2)) & 1u) << b;
    }
}

/* The share's leaves tile the curve interval [S, E) of the finest-level keys;
 * its maximal complete subtrees are the largest aligned blocks of that
 * interval, taken greedily from S.  Returns their number (written when
 * ulevel != NULL, up to cap). */
int64_t or_share_units(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
                       uint8_t *ulevel, uint32_t *ux, uint32_t *uy, uint32_t *uz, int64_t cap)
{
    if (n <= 0) return 0;
    uint64_t S = key_of(x[0], y[0], z[0]);
    uint64_t E = key_of(x[n - 1], y[n - 1], z[n - 1]) + ((uint64_t)1 << (3 * (OR_QMAX - level[n - 1])));
    int64_t m = 0;
    uint64_t p = S;
    while (p < E) {
        int l = 0;
        for (; l <= OR_QMAX; l++) {
            uint64_t size = (uint64_t)1 << (3 * (OR_QMAX - l));
            if (p % size == 0 && p + size <= E) break;
        }
        if (ulevel && m < cap) {
            ulevel[m] = (uint8_t)l;
            anchor_of(p, &ux[m], &uy[m], &uz[m]);
        }
        m++;
        p += (uint64_t)1 << (3 * (OR_QMAX - l));
    }
    return m;
}

/* Per-pixel lists of one share for one camera: for every pixel, one entry per
 * maximal subtree that its ray meets, (s_in, s_out) the canonical slab interval
 * of the subtree's box and (A, B) the nearest-first fold of the share's
 * segments inside it; entries in depth order.  offsets[P + 1]; entries[4 per
 * entry] written when entries != NULL (up to cap).  Returns the entry count. */
int64_t or_share_lists(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
                       int kind, const double *kap, const double *eps, int method, int substeps, double c_rk,
                       const double *cam, int64_t *offsets, double *entries, int64_t cap)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t P = (int64_t)c.w * c.h;
    int64_t nu = or_share_units(n, level, x, y, z, NULL, NULL, NULL, NULL, 0);
    uint8_t *ul = (uint8_t *)malloc((size_t)(nu > 0 ? nu : 1));
    uint32_t *ux = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nu > 0 ? nu : 1));
    uint32_t *uy = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nu > 0 ? nu : 1));
    uint32_t *uz = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nu > 0 ? nu : 1));
    or_share_units(n, level, x, y, z, ul, ux, uy, uz, nu);
    /* unit of every leaf: units and leaves are both in curve order */
    int64_t *lunit = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t u = 0;
    for (int64_t l = 0; l < n; l++) {
        uint64_t k = key_of(x[l], y[l], z[l]);
        while (u + 1 < nu && key_of(ux[u + 1], uy[u + 1], uz[u + 1]) <= k) u++;
        lunit[l] = u;
    }
    int64_t ns = 0;
    orseg *segs = gather(&c, n, level, x, y, z, -1, NULL, &ns);
    for (int64_t k = 0; k < ns; k++) {
        orseg *sg = &segs[k];
        int i = (int)(sg->pix % c.w), j = (int)(sg->pix / c.w);
        double rho[3], r[3];
        pixel_ray(&c, i, j, rho, r);
        leafbox b = leaf_box(level[sg->leaf], x[sg->leaf], y[sg->leaf], z[sg->leaf]);
        leaffield F;
        leaf_field(kind, n, sg->leaf, kap, eps, &F);
        dn A, B;
        segment_dn(&F, &b, rho, r, ray_norm(r), sg->s_in, sg->s_out, method, substeps, c_rk, 0, &A, &B);
        sg->A = A.v;
        sg->B = B.v;
    }
    for (int64_t q = 0; q <= P; q++) offsets[q] = 0;
    int64_t m = 0, k = 0;
    while (k < ns) {
        int64_t pix = segs[k].pix;
        while (k < ns && segs[k].pix == pix) {
            int64_t un = lunit[segs[k].leaf];
            double acc[2] = {1.0, 0.0};
            for (; k < ns && segs[k].pix == pix && lunit[segs[k].leaf] == un; k++) {
                double sgab[2] = {segs[k].A, segs[k].B}, t[2];
                or_combine(acc, sgab, t);
                acc[0] = t[0];
                acc[1] = t[1];
            }
            leafbox ub = leaf_box(ul[un], ux[un], uy[un], uz[un]);
            double rho[3], r[3], a, bb;
            pixel_ray(&c, (int)(pix % c.w), (int)(pix / c.w), rho, r);
            if (!slab(&c, rho, r, ub.lo, ub.hi, &a, &bb)) continue; /* cannot happen for a tiled unit */
            if (entries && m < cap) {
                entries[4 * m] = a;
                entries[4 * m + 1] = bb;
                entries[4 * m + 2] = acc[0];
                entries[4 * m + 3] = acc[1];
            }
            offsets[pix + 1]++;
            m++;
        }
    }
    for (int64_t q = 0; q < P; q++) offsets[q + 1] += offsets[q];
    free(segs);
    free(lunit);
    free(ul);
    free(ux);
    free(uy);
    free(uz);
    return m;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* One pixel's entries of all shares, sorted by (s_in, s_out).  The depths where
 * an entry starts or ends cut the ray into elementary intervals; over each,
 * every entry covering it contributes the piece of its own length fraction
 * (eq. segsplit), and where several cover it their pieces are averaged: the
 * geometric mean of the A and the arithmetic mean of the B (eq. segaverage,
 * taken over all covering entries).  The intervals are folded nearest first;
 * a zero-length entry is folded whole at its depth.  Returns the number of
 * overlaps: entries starting before the end of an entry that started earlier. */
int64_t or_merge_pixel(int64_t m, const double *e, double *AB)
{
    double acc[2] = {1.0, 0.0}, t[2];
    int64_t overlaps = 0;
    for (int64_t q = 0; q < m; q++) {
        if (!(e[4 * q + 1] > e[4 * q])) continue;
        for (int64_t r = 0; r < q; r++)
            if (e[4 * r + 1] > e[4 * r] && e[4 * r] <= e[4 * q] && e[4 * q] < e[4 * r + 1]) {
                overlaps++;
                break;
            }
    }
    double *bp = (double *)malloc(sizeof(double) * (size_t)(2 * m > 0 ? 2 * m : 1));
    int64_t nb = 0;
    for (int64_t q = 0; q < m; q++) {
        bp[nb++] = e[4 * q];
        bp[nb++] = e[4 * q + 1];
    }
    qsort(bp, (size_t)nb, sizeof(double), cmp_double);
    int64_t u = 0;
    for (int64_t k = 0; k < nb; k++)
        if (u == 0 || bp[k] != bp[u - 1]) bp[u++] = bp[k];
    for (int64_t k = 0; k < u; k++) {
        for (int64_t q = 0; q < m; q++) /* zero-length entries at this depth */
            if (!(e[4 * q + 1] > e[4 * q]) && e[4 * q] == bp[k]) {
                or_combine(acc, e + 4 * q + 2, t);
                acc[0] = t[0];
                acc[1] = t[1];
            }
        if (k + 1 == u) break;
        double lo = bp[k], hi = bp[k + 1], logA = 0.0, sumB = 0.0, one[2] = {1.0, 0.0};
        int n = 0;
        for (int64_t q = 0; q < m; q++) {
            const double *x = e + 4 * q;
            if (!(x[1] > x[0]) || x[0] > lo || x[1] < hi) continue;
            double piece[2], rest[2];
            or_split(x + 2, (hi - lo) / (x[1] - x[0]), piece, rest);
            logA += log(piece[0]);
            sumB += piece[1];
            one[0] = piece[0];
            one[1] = piece[1];
            n++;
        }
        if (n == 0) continue;
        double avg[2] = {n == 1 ? one[0] : exp(logA / n), n == 1 ? one[1] : sumB / n};
        or_combine(acc, avg, t);
        acc[0] = t[0];
        acc[1] = t[1];
    }
    free(bp);
    AB[0] = acc[0];
    AB[1] = acc[1];
    return overlaps;
}

/* or_merge_pixel over every pixel: off[P + 1] into entries sorted by s_in within
 * each pixel; AB[2 P]; returns the total number of overlaps. */
int64_t or_merge_sorted(int64_t P, const int64_t *off, const double *e, double *AB)
{
    int64_t ov = 0;
    for (int64_t p = 0; p < P; p++) ov += or_merge_pixel(off[p + 1] - off[p], e + 4 * off[p], AB + 2 * p);
    return ov;
}

int or_march(int64_t n, const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z, int kind,
             const double *kap, const double *eps, const double *cam, int M, double *Aout, double *Bout,
             double *Iout)
{
    orcam c;
    cam_parse(cam, &c);
    double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    int64_t P = (int64_t)c.w * c.h;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < P; p++) {
        int i = (int)(p % c.w), j = (int)(p / c.w);
        double rho[3], r[3], a, b;
        pixel_ray(&c, i, j, rho, r);
        double acc[2] = {1.0, 0.0};
        if (slab(&c, rho, r, lo, hi, &a, &b)) {
            double rn = ray_norm(r), ds = (b - a) / M;
            for (int m = 0; m < M; m++) {
                double sm = a + (m + 0.5) * ds, pt[3];
                for (int k = 0; k < 3; k++) pt[k] = rho[k] + sm * r[k];
                leafbox bx;
                int64_t l = locate(n, level, x, y, z, pt, &bx);
                if (l < 0) continue;
                double kv, ev;
                if (kind == 1) {
                    double xi[3], kc[8], ec[8];
                    for (int k = 0; k < 3; k++) xi[k] = (pt[k] - bx.lo[k]) / bx.hlen;
                    for (int cc = 0; cc < 8; cc++) {
                        kc[cc] = kap[(int64_t)cc * n + l];
                        ec[cc] = eps[(int64_t)cc * n + l];
                    }
                    kv = trilin_dn(kc, xi, 0, 0).v;
                    ev = trilin_dn(ec, xi, 0, 0).v;
                } else {
                    kv = kap[l];
                    ev = kind == 2 ? kap[l] * eps[l] : eps[l];
                }
                dn A, B;
                seg_const_dn(dn_c(kv, 0), dn_c(ev, 0), ds * rn, 0, &A, &B);
                double sg[2] = {A.v, B.v}, t[2];
                or_combine(acc, sg, t);
                acc[0] = t[0];
                acc[1] = t[1];
            }
        }
        Aout[p] = acc[0];
        Bout[p] = acc[1];
        Iout[p] = acc[0] * c.bg + acc[1];
    }
    return 0;
}

/* ======================================================================== */
/* six-tree spherical shell (equiangular cubed sphere, Sec. 2.1 eq.          */
/* geometrytrafo with a smooth per-tree map)                                 */
/* ======================================================================== */
/*
 * Tree k: axis m = k / 2, sign sg = +1 (k even) or -1; frame e1 = unit(m+1),
 * e2 = unit(m+2), e3 = sg unit(m).  Reference t in [0,1]^3 maps to
 *   x = r (a e1 + b e2 + e3) / sqrt(1 + a^2 + b^2),
 *   a = tan(pi/4 (2 t1 - 1)), b = tan(pi/4 (2 t2 - 1)), r = r0 + (r1 - r0) t3.
 * geom = [r0, r1, L, tan(pi/4 (2 i / 2^L - 1)) for i = 0 .. 2^L]: the tan values
 * at dyadic parameters are an input table, so no library call enters a
 * predicate.  An element is bounded by four planes through the origin
 * (constant t1, t2) and two spheres (constant t3); a ray meets it in at most
 * two intervals.
 */

typedef struct {
    int k, m, m1, m2;
    double sg;
    double alo, ahi, blo, bhi, rlo, rhi;
    double tlo[3];
    double hlen;
    double r0, r1;
} shellelem;

static shellelem shell_elem(const double *geom, int k, uint8_t level, uint32_t x, uint32_t y, uint32_t z)
{
    shellelem e;
    e.k = k;
    e.m = k / 2;
    e.sg = (k % 2 == 0) ? 1.0 : -1.0;
    e.m1 = (e.m + 1) % 3;
    e.m2 = (e.m + 2) % 3;
    e.r0 = geom[0];
    e.r1 = geom[1];
    int L = (int)geom[2];
    const double *tab = geom + 3;
    uint32_t len = (uint32_t)1 << (OR_QMAX - level);
    int sh = OR_QMAX - L;
    e.alo = tab[x >> sh];
    e.ahi = tab[(x + len) >> sh];
    e.blo = tab[y >> sh];
    e.bhi = tab[(y + len) >> sh];
    double q = ldexp(1.0, -OR_QMAX);
    double dr = e.r1 - e.r0;
    e.rlo = e.r0 + dr * ((double)z * q);
    e.rhi = e.r0 + dr * ((double)(z + len) * q);
    e.tlo[0] = (double)x * q;
    e.tlo[1] = (double)y * q;
    e.tlo[2] = (double)z * q;
    e.hlen = ldexp(1.0, -(int)level);
    return e;
}

/* Reference coordinates of a point by the closed-form inverse of the map. */
static void shell_ref(const void *ctx, const double *x, double *xi)
{
    const shellelem *e = (const shellelem *)ctx;
    double w = e->sg * x[e->m];
    double a = x[e->m1] / w, b = x[e->m2] / w;
    double t[3];
    t[0] = (atan(a) / (OR_PI / 4.0) + 1.0) / 2.0;
    t[1] = (atan(b) / (OR_PI / 4.0) + 1.0) / 2.0;
    double rr = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    t[2] = (rr - e->r0) / (e->r1 - e->r0);
    for (int c = 0; c < 3; c++) xi[c] = (t[c] - e->tlo[c]) / e->hlen;
}

/* Plane of constant a (tangent axis mt) through the origin: P(v) = v[mt] - a (sg v[m]).
 * lower != 0: the element keeps P >= 0, else P < 0.  Clips [*sa, *sb]. */
static int shell_plane(const shellelem *e, int mt, double a, int lower, const double *rho, const double *r,
                       double *sa, double *sb)
{
    double Pr = r[mt] - a * (e->sg * r[e->m]);
    double Pp = rho[mt] - a * (e->sg * rho[e->m]);
    if (Pr != 0.0) {
        double sx = -(Pp / Pr);
        int ge = lower ? (Pr > 0.0) : (Pr < 0.0); /* keep s >= sx */
        if (ge) {
            if (sx > *sa) *sa = sx;
        } else {
            if (sx < *sb) *sb = sx;
        }
        return 1;
    }
    return lower ? (Pp >= 0.0) : (Pp < 0.0);
}

/* Parameters where |rho + s r| = R: |.|^2 = A s^2 + 2 B s + C. */
static int shell_sphere(double A, double B, double C, double R, double *lo, double *hi)
{
    double c = C - R * R;
    double D = B * B - A * c;
    if (!(D > 0.0)) return 0;
    double sq = sqrt(D);
    double q = (B >= 0.0) ? -(B + sq) : (sq - B);
    double s1 = q / A, s2 = c / q;
    *lo = s1 < s2 ? s1 : s2;
    *hi = s1 < s2 ? s2 : s1;
    return 1;
}

/* Hit intervals of a ray with a shell element, clipped to [smin, smax]. */
static int shell_pair(const orcam *c, const shellelem *e, const double *rho, const double *r, double *iv)
{
    double sa = c->smin, sb = c->smax;
    if (!shell_plane(e, e->m1, e->alo, 1, rho, r, &sa, &sb)) return 0;
    if (!shell_plane(e, e->m1, e->ahi, 0, rho, r, &sa, &sb)) return 0;
    if (!shell_plane(e, e->m2, e->blo, 1, rho, r, &sa, &sb)) return 0;
    if (!shell_plane(e, e->m2, e->bhi, 0, rho, r, &sa, &sb)) return 0;
    if (!(sb > sa)) return 0;
    double A = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    double B = (rho[0] * r[0] + rho[1] * r[1]) + rho[2] * r[2];
    double C = (rho[0] * rho[0] + rho[1] * rho[1]) + rho[2] * rho[2];
    double o0, o1, i0, i1;
    if (!shell_sphere(A, B, C, e->rhi, &o0, &o1)) return 0;
    if (o0 > sa) sa = o0;
    if (o1 < sb) sb = o1;
    if (!(sb > sa)) return 0;
    int n = 0;
    if (!shell_sphere(A, B, C, e->rlo, &i0, &i1)) {
        iv[0] = sa;
        iv[1] = sb;
        return 1;
    }
    double b0 = i0 < sb ? i0 : sb;
    if (b0 > sa) {
        iv[2 * n] = sa;
        iv[2 * n + 1] = b0;
        n++;
    }
    double a1 = i1 > sa ? i1 : sa;
    if (sb > a1) {
        iv[2 * n] = a1;
        iv[2 * n + 1] = sb;
        n++;
    }
    return n;
}

/* Lenient camera-space box of a shell element: the element lies in the convex
 * hull of rlo c_i and (rhi / mu) c_i, c_i the unit corner directions and mu the
 * smallest cosine between them and their normalized mean. */
static int shell_rect(const orcam *c, const shellelem *e, int *rect)
{
    double cd[4][3];
    double av[2] = {e->alo, e->ahi}, bv[2] = {e->blo, e->bhi};
    for (int q = 0; q < 4; q++) {
        double a = av[q & 1], b = bv[q >> 1];
        double nrm = sqrt((1.0 + a * a) + b * b);
        cd[q][e->m1] = a / nrm;
        cd[q][e->m2] = b / nrm;
        cd[q][e->m] = e->sg / nrm;
    }
    double mean[3];
    for (int k = 0; k < 3; k++) mean[k] = ((cd[0][k] + cd[1][k]) + cd[2][k]) + cd[3][k];
    double ml = sqrt((mean[0] * mean[0] + mean[1] * mean[1]) + mean[2] * mean[2]);
    for (int k = 0; k < 3; k++) mean[k] = mean[k] / ml;
    double mu = 1.0;
    for (int q = 0; q < 4; q++) {
        double d = (cd[q][0] * mean[0] + cd[q][1] * mean[1]) + cd[q][2] * mean[2];
        if (d < mu) mu = d;
    }
    double sin_ = e->rlo * (1.0 - 1e-12), sout = e->rhi * (1.0 + 1e-12) / mu;
    double ext[3][2];
    const double *axes[3] = {c->t, c->u, c->vh};
    for (int ax = 0; ax < 3; ax++) {
        ext[ax][0] = INFINITY;
        ext[ax][1] = -INFINITY;
    }
    for (int q = 0; q < 8; q++) {
        double sc = (q < 4) ? sin_ : sout;
        double p[3];
        for (int k = 0; k < 3; k++) p[k] = sc * cd[q & 3][k] - c->o[k];
        for (int ax = 0; ax < 3; ax++) {
            const double *a = axes[ax];
            double v = (a[0] * p[0] + a[1] * p[1]) + a[2] * p[2];
            if (v < ext[ax][0]) ext[ax][0] = v;
            if (v > ext[ax][1]) ext[ax][1] = v;
        }
    }
    rect[0] = 1;
    rect[1] = 0;
    rect[2] = 1;
    rect[3] = 0;
    double Z0 = ext[2][0], Z1 = ext[2][1];
    if (Z1 < c->n || Z0 > c->zfar) return 0;
    double Zc0 = Z0 < c->n ? c->n : Z0;
    double Zc1 = Z1 > c->zfar ? c->zfar : Z1;
    int i0, i1, j0, j1;
    pixel_range(c, ext[0][0], ext[0][1], Zc0, Zc1, c->cx, c->w, &i0, &i1);
    pixel_range(c, ext[1][0], ext[1][1], Zc0, Zc1, c->cy, c->h, &j0, &j1);
    if (i0 > i1 || j0 > j1) return 0;
    rect[0] = i0;
    rect[1] = i1;
    rect[2] = j0;
    rect[3] = j1;
    return 1;
}

static int tree_of(int64_t l, int ntrees, const int64_t *tree_begin)
{
    int k = 0;
    while (k + 1 < ntrees && l >= tree_begin[k + 1]) k++;
    return k;
}

int64_t or_shell_prune(int64_t n, int ntrees, const int64_t *tree_begin, const double *geom, const uint8_t *level,
                       const uint32_t *x, const uint32_t *y, const uint32_t *z, const double *cam, int32_t *rect)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t nvis = 0;
    for (int64_t l = 0; l < n; l++) {
        shellelem e = shell_elem(geom, tree_of(l, ntrees, tree_begin), level[l], x[l], y[l], z[l]);
        int rr[4];
        nvis += shell_rect(&c, &e, rr);
        for (int k = 0; k < 4; k++) rect[l * 4 + k] = rr[k];
    }
    return nvis;
}

/* Pairing of the listed leaves' candidates: nseg[q] in {0,1,2} and up to two
 * intervals (sio[4q .. 4q+3], zeros where absent).  Returns the candidate count. */
int64_t or_shell_pairs(int64_t nlist, const int64_t *list, int ntrees, const int64_t *tree_begin, const double *geom,
                       const uint8_t *level, const uint32_t *x, const uint32_t *y, const uint32_t *z,
                       const double *cam, uint8_t *nseg, double *sio, int64_t cap)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t q = 0;
    for (int64_t m = 0; m < nlist; m++) {
        int64_t l = list[m];
        shellelem e = shell_elem(geom, tree_of(l, ntrees, tree_begin), level[l], x[l], y[l], z[l]);
        int rr[4];
        if (!shell_rect(&c, &e, rr)) continue;
        for (int j = rr[2]; j <= rr[3]; j++)
            for (int i = rr[0]; i <= rr[1]; i++) {
                if (q < cap) {
                    double rho[3], r[3], iv[4] = {0, 0, 0, 0};
                    pixel_ray(&c, i, j, rho, r);
                    int ns = shell_pair(&c, &e, rho, r, iv);
                    nseg[q] = (uint8_t)ns;
                    for (int k = 0; k < 4; k++) sio[4 * q + k] = (k < 2 * ns) ? iv[k] : 0.0;
                }
                q++;
            }
    }
    return q;
}

/* Render one camera of a shell forest (trilinear or constant fields in
 * reference coordinates): same definition as or_render, with the closed-form
 * inverse map for the field points.  Arguments as or_render plus the tree
 * layout and the geometry table. */
int or_shell_render(int64_t n, int ntrees, const int64_t *tree_begin, const double *geom, const uint8_t *level,
                    const uint32_t *x, const uint32_t *y, const uint32_t *z, int kind, const double *kap,
                    const double *eps, int method, int substeps, double c_rk, const double *cam, int64_t npix_sel,
                    const int64_t *pix_sel, double *Aout, double *Bout, double *Iout, int32_t *nseg_pix,
                    int64_t *stats)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t W = c.w, H = c.h, P = W * H;
    int64_t npo = (npix_sel >= 0) ? npix_sel : P;
    int64_t *selmap = NULL;
    if (npix_sel >= 0) {
        selmap = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);
        for (int64_t p = 0; p < P; p++) selmap[p] = -1;
        for (int64_t q = 0; q < npix_sel; q++) selmap[pix_sel[q]] = q;
    }
    int64_t cap = 1 << 16, ns = 0;
    orseg *segs = (orseg *)malloc(sizeof(orseg) * (size_t)cap);
    for (int64_t l = 0; l < n; l++) {
        shellelem e = shell_elem(geom, tree_of(l, ntrees, tree_begin), level[l], x[l], y[l], z[l]);
        int rr[4];
        if (!shell_rect(&c, &e, rr)) continue;
        for (int j = rr[2]; j <= rr[3]; j++)
            for (int i = rr[0]; i <= rr[1]; i++) {
                int64_t p = (int64_t)j * W + i, ps = p;
                if (selmap) {
                    ps = selmap[p];
                    if (ps < 0) continue;
                }
                double rho[3], r[3], iv[4];
                pixel_ray(&c, i, j, rho, r);
                int nh = shell_pair(&c, &e, rho, r, iv);
                for (int h = 0; h < nh; h++) {
                    if (ns == cap) {
                        cap *= 2;
                        segs = (orseg *)realloc(segs, sizeof(orseg) * (size_t)cap);
                    }
                    segs[ns].pix = ps;
                    segs[ns].s_in = iv[2 * h];
                    segs[ns].s_out = iv[2 * h + 1];
                    segs[ns].leaf = l;
                    ns++;
                }
            }
    }
    free(selmap);
    qsort(segs, (size_t)ns, sizeof(orseg), seg_cmp);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < ns; k++) {
        orseg *s = &segs[k];
        int64_t p = (npix_sel >= 0) ? pix_sel[s->pix] : s->pix;
        int i = (int)(p % W), j = (int)(p / W);
        double rho[3], r[3];
        pixel_ray(&c, i, j, rho, r);
        int64_t l = s->leaf;
        shellelem e = shell_elem(geom, tree_of(l, ntrees, tree_begin), level[l], x[l], y[l], z[l]);
        leaffield F;
        leaf_field(kind, n, l, kap, eps, &F);
        dn A, B;
        segment_dn_ref(&F, shell_ref, &e, rho, r, ray_norm(r), s->s_in, s->s_out, method, substeps, c_rk, 0, &A, &B);
        s->A = A.v;
        s->B = B.v;
    }
    int64_t overlaps = 0;
    for (int64_t q = 0; q < npo; q++) {
        Aout[q] = 1.0;
        Bout[q] = 0.0;
        if (nseg_pix) nseg_pix[q] = 0;
    }
    int64_t k = 0;
    while (k < ns) {
        int64_t q = segs[k].pix;
        double acc[2] = {1.0, 0.0};
        double prev_out = -INFINITY;
        int cnt = 0;
        for (; k < ns && segs[k].pix == q; k++) {
            if (segs[k].s_in < prev_out - 1e-12 * fabs(prev_out)) overlaps++;
            prev_out = segs[k].s_out;
            double sg[2] = {segs[k].A, segs[k].B}, t[2];
            or_combine(acc, sg, t);
            acc[0] = t[0];
            acc[1] = t[1];
            cnt++;
        }
        Aout[q] = acc[0];
        Bout[q] = acc[1];
        if (nseg_pix) nseg_pix[q] = cnt;
    }
    for (int64_t q = 0; q < npo; q++) Iout[q] = Aout[q] * c.bg + Bout[q];
    if (stats) {
        stats[0] = ns;
        stats[1] = overlaps;
    }
    free(segs);
    return 0;
}

/* Forward map of tree k (for pins): reference t -> real x, using the library tan. */
void or_shell_map(const double *geom, int k, const double *t, double *x)
{
    shellelem e = shell_elem(geom, k, 0, 0, 0, 0);
    double a = tan(OR_PI / 4.0 * (2.0 * t[0] - 1.0)), b = tan(OR_PI / 4.0 * (2.0 * t[1] - 1.0));
    double r = e.r0 + (e.r1 - e.r0) * t[2];
    double nrm = sqrt(1.0 + a * a + b * b);
    x[e.m1] = r * a / nrm;
    x[e.m2] = r * b / nrm;
    x[e.m] = r * e.sg / nrm;
}

/* Closed-form inverse of tree k's map (for pins). */
void or_shell_inverse(const double *geom, int k, const double *x, double *t)
{
    shellelem e = shell_elem(geom, k, 0, 0, 0, 0);
    shell_ref(&e, x, t);
}

/* Brute-force march through the shell: M equal steps over the ray's chord of
 * the outer sphere; each step's midpoint is located by its dominant axis
 * (tree), the closed-form inverse map and a scan of the tree's leaves; the
 * step uses eq. ABconstant with the coefficients at the midpoint. */
int or_shell_march(int64_t n, int ntrees, const int64_t *tree_begin, const double *geom, const uint8_t *level,
                   const uint32_t *x, const uint32_t *y, const uint32_t *z, int kind, const double *kap,
                   const double *eps, const double *cam, int M, double *Aout, double *Bout, double *Iout)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t P = (int64_t)c.w * c.h;
    double r0 = geom[0], r1 = geom[1];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < P; p++) {
        int i = (int)(p % c.w), j = (int)(p / c.w);
        double rho[3], r[3];
        pixel_ray(&c, i, j, rho, r);
        double acc[2] = {1.0, 0.0};
        double A = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        double B = (rho[0] * r[0] + rho[1] * r[1]) + rho[2] * r[2];
        double C = (rho[0] * rho[0] + rho[1] * rho[1]) + rho[2] * rho[2];
        double a, b;
        if (shell_sphere(A, B, C, r1, &a, &b)) {
            if (a < c.smin) a = c.smin;
            if (b > c.smax) b = c.smax;
            double rn = ray_norm(r), ds = (b - a) / M;
            for (int m = 0; m < M && b > a; m++) {
                double sm = a + (m + 0.5) * ds, pt[3];
                for (int k = 0; k < 3; k++) pt[k] = rho[k] + sm * r[k];
                double rad = sqrt(pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2]);
                if (rad < r0 || rad >= r1) continue;
                int ax = 0;
                for (int k = 1; k < 3; k++)
                    if (fabs(pt[k]) > fabs(pt[ax])) ax = k;
                int tree = 2 * ax + (pt[ax] < 0.0 ? 1 : 0);
                if (tree >= ntrees) continue;
                shellelem e0 = shell_elem(geom, tree, 0, 0, 0, 0);
                double t[3];
                shell_ref(&e0, pt, t);
                int64_t found = -1;
                for (int64_t l = tree_begin[tree]; l < tree_begin[tree + 1]; l++) {
                    double q = ldexp(1.0, -OR_QMAX), hl = ldexp(1.0, -(int)level[l]);
                    double lo[3] = {(double)x[l] * q, (double)y[l] * q, (double)z[l] * q};
                    if (t[0] >= lo[0] && t[0] < lo[0] + hl && t[1] >= lo[1] && t[1] < lo[1] + hl && t[2] >= lo[2] &&
                        t[2] < lo[2] + hl) {
                        found = l;
                        break;
                    }
                }
                if (found < 0) continue;
                shellelem e = shell_elem(geom, tree, level[found], x[found], y[found], z[found]);
                double xi[3];
                shell_ref(&e, pt, xi);
                double kv, ev;
                if (kind == 1) {
                    double kc[8], ec[8];
                    for (int cc = 0; cc < 8; cc++) {
                        kc[cc] = kap[(int64_t)cc * n + found];
                        ec[cc] = eps[(int64_t)cc * n + found];
                    }
                    kv = trilin_dn(kc, xi, 0, 0).v;
                    ev = trilin_dn(ec, xi, 0, 0).v;
                } else {
                    kv = kap[found];
                    ev = kind == 2 ? kap[found] * eps[found] : eps[found];
                }
                dn Ad, Bd;
                seg_const_dn(dn_c(kv, 0), dn_c(ev, 0), ds * rn, 0, &Ad, &Bd);
                double sg[2] = {Ad.v, Bd.v}, tt[2];
                or_combine(acc, sg, tt);
                acc[0] = tt[0];
                acc[1] = tt[1];
            }
        }
        Aout[p] = acc[0];
        Bout[p] = acc[1];
        Iout[p] = acc[0] * c.bg + acc[1];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* surfaces: quadtree leaves on bilinear tree patches                       */
/* (Sec. 2.8 thin and opaque surfaces, eq. ABphi; App. A.1 ray against a    */
/* tensor-product surface, the bilinear case by a quadratic)                */
/* ------------------------------------------------------------------------ */

/* Tree k's patch J(t1, t2) = a + b t1 + c t2 + d t1 t2 from its corners
 * P00, P10, P01, P11 (12 doubles per tree: corner q at t = (q & 1, q >> 1)). */
typedef struct {
    double a[3], b[3], c[3], d[3];
} orpatch;

static orpatch patch_of(const double *P)
{
    orpatch S;
    for (int k = 0; k < 3; k++) {
        S.a[k] = P[k];
        S.b[k] = P[3 + k] - P[k];
        S.c[k] = P[6 + k] - P[k];
        S.d[k] = (P[9 + k] - P[3 + k]) - (P[6 + k] - P[k]);
    }
    return S;
}

static double dot3(const double *u, const double *w) { return (u[0] * w[0] + u[1] * w[1]) + u[2] * w[2]; }

static void cross3(const double *u, const double *w, double *o)
{
    o[0] = u[1] * w[2] - u[2] * w[1];
    o[1] = u[2] * w[0] - u[0] * w[2];
    o[2] = u[0] * w[1] - u[1] * w[0];
}

/* Hits of the ray rho + s r with the patch for (t1, t2) in [0, 1]^2 and s in
 * the clip range, nearest first (at most two).  App. A.1: with d1, d2 normal
 * to r, the two projections d_j . (J(t1, t2) - rho) = 0 are bilinear in
 * (t1, t2); eliminating t1 leaves a quadratic in t2, and t1 follows from the
 * projection with the larger coefficient of t1.  d1 = r x e_k for the axis k
 * of smallest |r_k|, d2 = r x d1.  A double root counts once. */
static int surface_hits(const orcam *cm, const orpatch *S, const double *rho, const double *r, double *hs,
                        double *ht1, double *ht2)
{
    int k = 0;
    if (fabs(r[1]) < fabs(r[k])) k = 1;
    if (fabs(r[2]) < fabs(r[k])) k = 2;
    double ek[3] = {0.0, 0.0, 0.0}, d1[3], d2[3], e[3];
    ek[k] = 1.0;
    cross3(r, ek, d1);
    cross3(r, d1, d2);
    for (int q = 0; q < 3; q++) e[q] = S->a[q] - rho[q];
    double A1 = dot3(d1, S->d), B1 = dot3(d1, S->b), C1 = dot3(d1, S->c), D1 = dot3(d1, e);
    double A2 = dot3(d2, S->d), B2 = dot3(d2, S->b), C2 = dot3(d2, S->c), D2 = dot3(d2, e);
    /* (A_j t2 + B_j) t1 + (C_j t2 + D_j) = 0 for j = 1, 2; the determinant in t1 vanishes */
    double qa = A1 * C2 - A2 * C1;
    double qb = (A1 * D2 - A2 * D1) + (B1 * C2 - B2 * C1);
    double qc = B1 * D2 - B2 * D1;
    double roots[2];
    int nr = 0;
    if (qa == 0.0) {
        if (qb != 0.0) roots[nr++] = -qc / qb;
    } else {
        double disc = qb * qb - (4.0 * qa) * qc;
        if (disc == 0.0) {
            roots[nr++] = -qb / (2.0 * qa);
        } else if (disc > 0.0) {
            double sq = sqrt(disc);
            double q = -0.5 * (qb + (qb >= 0.0 ? sq : -sq));
            roots[nr++] = q / qa;
            roots[nr++] = qc / q;
        }
    }
    double rr = dot3(r, r);
    int nh = 0;
    for (int m = 0; m < nr; m++) {
        double t2 = roots[m];
        double den1 = A1 * t2 + B1, den2 = A2 * t2 + B2, t1;
        if (fabs(den1) >= fabs(den2)) {
            if (den1 == 0.0) continue;
            t1 = -(C1 * t2 + D1) / den1;
        } else {
            t1 = -(C2 * t2 + D2) / den2;
        }
        if (!(t1 >= 0.0 && t1 <= 1.0 && t2 >= 0.0 && t2 <= 1.0)) continue;
        double pr[3];
        for (int q = 0; q < 3; q++) pr[q] = (((S->a[q] + S->b[q] * t1) + S->c[q] * t2) + S->d[q] * (t1 * t2)) - rho[q];
        double s = dot3(pr, r) / rr;
        if (!(s >= cm->smin && s <= cm->smax)) continue;
        hs[nh] = s;
        ht1[nh] = t1;
        ht2[nh] = t2;
        nh++;
    }
    if (nh == 2 && hs[1] < hs[0]) {
        double t;
        t = hs[0]; hs[0] = hs[1]; hs[1] = t;
        t = ht1[0]; ht1[0] = ht1[1]; ht1[1] = t;
        t = ht2[0]; ht2[0] = ht2[1]; ht2[1] = t;
    }
    return nh;
}

/* The leaf of tree [b, e) whose square holds (t1, t2): half-open squares on
 * the finest grid, the tree's far edges closed.  -1 where no leaf covers it. */
static int64_t surface_leaf(const uint8_t *level, const uint32_t *x, const uint32_t *y, int64_t b, int64_t e,
                            double t1, double t2)
{
    double X = t1 * (double)(1u << OR_QMAX), Y = t2 * (double)(1u << OR_QMAX);
    uint32_t top = (1u << OR_QMAX) - 1u;
    uint32_t ix = X >= (double)top ? top : (uint32_t)X, iy = Y >= (double)top ? top : (uint32_t)Y;
    uint64_t kp = key_of(ix, iy, 0);
    int64_t lo = b, hi = e; /* last leaf with key <= kp */
    if (b >= e || key_of(x[b], y[b], 0) > kp) return -1;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (key_of(x[mid], y[mid], 0) <= kp)
            lo = mid;
        else
            hi = mid;
    }
    uint64_t span = (uint64_t)1 << (3 * (OR_QMAX - level[lo]));
    return kp < key_of(x[lo], y[lo], 0) + span ? lo : -1;
}

/* Surface model at a hit (Sec. 2.8, eq. ABphi with eq. BIrelation): the
 * transparency A_s and intensity I_s interpolated bilinearly from the leaf's
 * corners at its local coordinates, A = A_s^(1 / cos phi) with phi the angle
 * between the ray and the patch normal, B = I_s (1 - A). */
static void surface_value(int64_t n, int64_t leaf, const uint8_t *level, const uint32_t *x, const uint32_t *y,
                          const double *As, const double *Is, const orpatch *S, const double *r, double t1, double t2,
                          double *A, double *B)
{
    double len = (double)(1u << (OR_QMAX - level[leaf]));
    double u = (t1 * (double)(1u << OR_QMAX) - (double)x[leaf]) / len;
    double v = (t2 * (double)(1u << OR_QMAX) - (double)y[leaf]) / len;
    double w[4] = {(1.0 - u) * (1.0 - v), u * (1.0 - v), (1.0 - u) * v, u * v};
    double as = 0.0, is = 0.0;
    for (int q = 0; q < 4; q++) {
        as += w[q] * As[(int64_t)q * n + leaf];
        is += w[q] * Is[(int64_t)q * n + leaf];
    }
    double j1[3], j2[3], nr[3];
    for (int q = 0; q < 3; q++) {
        j1[q] = S->b[q] + S->d[q] * t2;
        j2[q] = S->c[q] + S->d[q] * t1;
    }
    cross3(j1, j2, nr);
    double cosphi = fabs(dot3(nr, r)) / sqrt(dot3(nr, nr) * dot3(r, r));
    *A = pow(as, 1.0 / cosphi);
    *B = is * (1.0 - *A);
}

/* Render a surface forest: per pixel, every tree's hits, each given to the
 * leaf whose square holds it, folded front to back with the background.
 * As, Is: [4][n] corner values.  nsel >= 0: only the pixels pix[0..nsel).
 * hit_leaf, hit_s (optional, [npix][2 * ntrees]): the hits in depth order,
 * leaf -1 past the last. */
int or_surface_render(int64_t n, int ntrees, const int64_t *tree_begin, const double *corners, const uint8_t *level,
                      const uint32_t *x, const uint32_t *y, const double *As, const double *Is, const double *cam,
                      int64_t nsel, const int64_t *pix, double *Aout, double *Bout, double *Iout, int32_t *hit_leaf,
                      double *hit_s)
{
    orcam c;
    cam_parse(cam, &c);
    int64_t P = nsel >= 0 ? nsel : (int64_t)c.w * c.h;
    int H = 2 * ntrees;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < P; q++) {
        int64_t p = nsel >= 0 ? pix[q] : q;
        int i = (int)(p % c.w), j = (int)(p / c.w);
        double rho[3], r[3];
        pixel_ray(&c, i, j, rho, r);
        double hs[2 * 64], hA[2 * 64], hB[2 * 64];
        int64_t hl[2 * 64];
        int nh = 0;
        for (int k = 0; k < ntrees; k++) {
            orpatch S = patch_of(corners + 12 * k);
            double s[2], t1[2], t2[2];
            int m = surface_hits(&c, &S, rho, r, s, t1, t2);
            for (int a = 0; a < m; a++) {
                int64_t leaf = surface_leaf(level, x, y, tree_begin[k], tree_begin[k + 1], t1[a], t2[a]);
                if (leaf < 0) continue;
                surface_value(n, leaf, level, x, y, As, Is, &S, r, t1[a], t2[a], &hA[nh], &hB[nh]);
                hs[nh] = s[a];
                hl[nh] = leaf;
                /* insertion in depth order; equal depths keep tree order */
                for (int b = nh; b > 0 && hs[b] < hs[b - 1]; b--) {
                    double t;
                    int64_t tl;
                    t = hs[b]; hs[b] = hs[b - 1]; hs[b - 1] = t;
                    t = hA[b]; hA[b] = hA[b - 1]; hA[b - 1] = t;
                    t = hB[b]; hB[b] = hB[b - 1]; hB[b - 1] = t;
                    tl = hl[b]; hl[b] = hl[b - 1]; hl[b - 1] = tl;
                }
                nh++;
            }
        }
        double acc[2] = {1.0, 0.0}, t[2];
        for (int b = 0; b < nh; b++) {
            double sg[2] = {hA[b], hB[b]};
            or_combine(acc, sg, t);
            acc[0] = t[0];
            acc[1] = t[1];
        }
        Aout[q] = acc[0];
        Bout[q] = acc[1];
        Iout[q] = acc[0] * c.bg + acc[1];
        if (hit_leaf) {
            for (int b = 0; b < H; b++) {
                hit_leaf[q * H + b] = b < nh ? (int32_t)hl[b] : -1;
                hit_s[q * H + b] = b < nh ? hs[b] : 0.0;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* high-order surfaces: degree-R tensor Lagrange maps on Gauss-Lobatto      */
/* nodes (eq. nodal, eq. tensorgeom), hits by subdivision with Bernstein    */
/* convex-hull exclusion and Newton's method (App. A.1)                     */
/* ------------------------------------------------------------------------ */

#define OR_HO_MAXR 3
#define OR_HO_DEPTH 10    /* subdivision of the tree square before Newton */
#define OR_HO_MAXDEPTH 24 /* squares where Newton leaves the square are split further, down to this */

typedef struct {
    int R;
    double eta[OR_HO_MAXR + 1];
    double einv[(OR_HO_MAXR + 1) * (OR_HO_MAXR + 1)]; /* equispaced values -> Bernstein coefficients */
    const double *z;                                 /* (R+1)^2 control points, m1 fastest */
} orho;

static double binom(int n, int k)
{
    double b = 1.0;
    for (int i = 1; i <= k; i++) b = b * (n - k + i) / i;
    return b;
}

/* Gauss-Lobatto nodes on [0, 1]: the ends and the roots of P_R' mapped there. */
static void ho_init(orho *H, int R, const double *z)
{
    H->R = R;
    H->z = z;
    H->eta[0] = 0.0;
    H->eta[R] = 1.0;
    if (R == 2) H->eta[1] = 0.5;
    if (R == 3) {
        H->eta[1] = 0.5 * (1.0 - 1.0 / sqrt(5.0));
        H->eta[2] = 0.5 * (1.0 + 1.0 / sqrt(5.0));
    }
    /* E[j][k] = B_k(j / R); einv = E^-1 by Gauss-Jordan elimination */
    int n = R + 1;
    double a[OR_HO_MAXR + 1][2 * (OR_HO_MAXR + 1)];
    for (int j = 0; j < n; j++)
        for (int k = 0; k < n; k++) {
            double u = (double)j / R;
            a[j][k] = binom(R, k) * pow(u, k) * pow(1.0 - u, R - k);
            a[j][n + k] = j == k ? 1.0 : 0.0;
        }
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        for (int k = 0; k < 2 * n; k++) {
            double t = a[c][k];
            a[c][k] = a[piv][k];
            a[piv][k] = t;
        }
        double d = a[c][c];
        for (int k = 0; k < 2 * n; k++) a[c][k] /= d;
        for (int r = 0; r < n; r++)
            if (r != c) {
                double f = a[r][c];
                for (int k = 0; k < 2 * n; k++) a[r][k] -= f * a[c][k];
            }
    }
    for (int j = 0; j < n; j++)
        for (int k = 0; k < n; k++) H->einv[j * n + k] = a[j][n + k];
}

/* Lagrange basis psi_m(t) on the nodes and its derivative (eq. nodal). */
static void ho_basis(const orho *H, double t, double *psi, double *dpsi)
{
    for (int m = 0; m <= H->R; m++) {
        double p = 1.0, dp = 0.0;
        for (int l = 0; l <= H->R; l++) {
            if (l == m) continue;
            double den = H->eta[m] - H->eta[l];
            dp = dp * ((t - H->eta[l]) / den) + p / den;
            p *= (t - H->eta[l]) / den;
        }
        psi[m] = p;
        dpsi[m] = dp;
    }
}

/* J(t1, t2) (eq. tensorgeom) and its partial derivatives. */
static void ho_eval(const orho *H, double t1, double t2, double *J, double *J1, double *J2)
{
    double p1[OR_HO_MAXR + 1], d1[OR_HO_MAXR + 1], p2[OR_HO_MAXR + 1], d2[OR_HO_MAXR + 1];
    ho_basis(H, t1, p1, d1);
    ho_basis(H, t2, p2, d2);
    int n = H->R + 1;
    for (int k = 0; k < 3; k++) {
        double v = 0.0, v1 = 0.0, v2 = 0.0;
        for (int m2 = 0; m2 < n; m2++)
            for (int m1 = 0; m1 < n; m1++) {
                double zc = H->z[3 * (m1 + n * m2) + k];
                v += zc * p1[m1] * p2[m2];
                v1 += zc * d1[m1] * p2[m2];
                v2 += zc * p1[m1] * d2[m2];
            }
        J[k] = v;
        if (J1) J1[k] = v1;
        if (J2) J2[k] = v2;
    }
}

/* Does the patch over the square [a1, a1 + h] x [a2, a2 + h] possibly meet the
 * planes d1 . (x - rho) = 0 and d2 . (x - rho) = 0?  The Bernstein coefficients
 * of each projection over the square (from the values on an equispaced grid)
 * bound it; a square whose coefficients of one projection share a strict sign,
 * beyond a relative 1e-10 for rounding, holds no hit. */
static int ho_square_may_hit(const orho *H, const double *rho, const double *d1, const double *d2, double a1,
                             double a2, double h)
{
    int n = H->R + 1;
    double g[2][(OR_HO_MAXR + 1) * (OR_HO_MAXR + 1)], tmp[(OR_HO_MAXR + 1) * (OR_HO_MAXR + 1)];
    for (int j2 = 0; j2 < n; j2++)
        for (int j1 = 0; j1 < n; j1++) {
            double J[3], e[3];
            ho_eval(H, a1 + h * j1 / H->R, a2 + h * j2 / H->R, J, NULL, NULL);
            for (int k = 0; k < 3; k++) e[k] = J[k] - rho[k];
            g[0][j1 + n * j2] = dot3(d1, e);
            g[1][j1 + n * j2] = dot3(d2, e);
        }
    for (int f = 0; f < 2; f++) {
        /* values -> Bernstein coefficients along t1, then along t2 */
        for (int j2 = 0; j2 < n; j2++)
            for (int k = 0; k < n; k++) {
                double s = 0.0;
                for (int j = 0; j < n; j++) s += H->einv[k * n + j] * g[f][j + n * j2];
                tmp[k + n * j2] = s;
            }
        /* a coefficient within rounding of zero counts for both signs */
        double c[(OR_HO_MAXR + 1) * (OR_HO_MAXR + 1)], big = 0.0;
        for (int k1 = 0; k1 < n; k1++)
            for (int k = 0; k < n; k++) {
                double s = 0.0;
                for (int j = 0; j < n; j++) s += H->einv[k * n + j] * tmp[k1 + n * j];
                c[k1 + n * k] = s;
                big = fmax(big, fabs(s));
            }
        double tol = 1e-10 * big;
        int pos = 0, neg = 0;
        for (int q = 0; q < n * n; q++) {
            pos |= c[q] >= -tol;
            neg |= c[q] <= tol;
        }
        if (!(pos && neg)) return 0;
    }
    return 1;
}

/* One Newton step on d_j . (J(t1, t2) - rho) = 0, j = 1, 2; the step in (s1, s2).
 * Returns 0 at a singular Jacobian. */
static int ho_newton(const orho *H, const double *rho, const double *d1, const double *d2, double *t1, double *t2,
                     double *s1, double *s2)
{
    double J[3], J1[3], J2[3], e[3];
    ho_eval(H, *t1, *t2, J, J1, J2);
    for (int q = 0; q < 3; q++) e[q] = J[q] - rho[q];
    double f1 = dot3(d1, e), f2 = dot3(d2, e);
    double a = dot3(d1, J1), b = dot3(d1, J2), c = dot3(d2, J1), dd = dot3(d2, J2);
    double det = a * dd - b * c;
    if (det == 0.0) return 0;
    *s1 = (dd * f1 - b * f2) / det;
    *s2 = (a * f2 - c * f1) / det;
    *t1 -= *s1;
    *t2 -= *s2;
    return 1;
}

/* Hits of the ray with a degree-R tree patch for (t1, t2) in [0, 1]^2 and s in
 * the clip range, nearest first (up to cap): the tree square is subdivided
 * OR_HO_DEPTH times, discarding squares that cannot hold a hit, and Newton's
 * method runs from the centre of each square left; a root counts in the
 * square whose half-open extent holds it rounded to the 2^-40 grid of the
 * canonical polish (far tree edges closed), and ht1, ht2 return it so rounded
 * (the leaf holding it is found from them).  A square
 * whose Newton iteration does not end inside it is split again, down to
 * OR_HO_MAXDEPTH, so that close roots near a tangency are separated.  Newton has
 * converged when its step falls below tol. */
static int ho_hits(const orcam *cm, const orho *H, const double *rho, const double *r, double *hs, double *ht1,
                   double *ht2, int cap, double tol)
{
    int k = 0;
    if (fabs(r[1]) < fabs(r[k])) k = 1;
    if (fabs(r[2]) < fabs(r[k])) k = 2;
    double ek[3] = {0.0, 0.0, 0.0}, d1[3], d2[3];
    ek[k] = 1.0;
    cross3(r, ek, d1);
    cross3(r, d1, d2);
    double rr = dot3(r, r);
    int nh = 0;
    /* depth-first over squares (index i1, i2 at depth d) */
    int st_i1[4 * OR_HO_MAXDEPTH + 4], st_i2[4 * OR_HO_MAXDEPTH + 4], st_d[4 * OR_HO_MAXDEPTH + 4], sp = 0;
    st_i1[0] = st_i2[0] = st_d[0] = 0;
    sp = 1;
    /* a ray lying in the surface leaves every square undecided: bounded work */
    for (long visits = 0; sp > 0 && visits < 1000000; visits++) {
        sp--;
        int i1 = st_i1[sp], i2 = st_i2[sp], d = st_d[sp];
        double h = ldexp(1.0, -d), a1 = i1 * h, a2 = i2 * h;
        if (!ho_square_may_hit(H, rho, d1, d2, a1, a2, h)) continue;
        if (d < OR_HO_DEPTH) {
            for (int c = 3; c >= 0; c--) {
                st_i1[sp] = 2 * i1 + (c & 1);
                st_i2[sp] = 2 * i2 + (c >> 1);
                st_d[sp] = d + 1;
                sp++;
            }
            continue;
        }
        double t1 = a1 + 0.5 * h, t2 = a2 + 0.5 * h, J[3], e[3];
        int ok = 0;
        for (int it = 0; it < 40; it++) {
            double s1, s2;
            if (!ho_newton(H, rho, d1, d2, &t1, &t2, &s1, &s2)) break;
            if (fabs(s1) + fabs(s2) < tol) {
                ok = 1;
                break;
            }
        }
        /* canonical polish: the same start for every square that converged to this
         * root, so that exactly one square holds the result */
        const double g = 1099511627776.0; /* 2^40 */
        double q1 = t1, q2 = t2;
        if (ok) {
            t1 = nearbyint(t1 * g) / g;
            t2 = nearbyint(t2 * g) / g;
            double s1, s2;
            for (int it = 0; it < 2; it++) ok = ok && ho_newton(H, rho, d1, d2, &t1, &t2, &s1, &s2);
            /* the square and the leaf that hold the root are decided on the root
             * rounded to the same grid, which holds every leaf edge: a root within
             * rounding of an edge goes to the leaf starting there, whatever the
             * last bits of the polish */
            q1 = nearbyint(t1 * g) / g;
            q2 = nearbyint(t2 * g) / g;
        }
        int in1 = (q1 >= a1 && q1 < a1 + h) || (q1 == 1.0 && a1 + h == 1.0);
        int in2 = (q2 >= a2 && q2 < a2 + h) || (q2 == 1.0 && a2 + h == 1.0);
        if (!(ok && in1 && in2)) {
            if (d < OR_HO_MAXDEPTH) {
                for (int c = 3; c >= 0; c--) {
                    st_i1[sp] = 2 * i1 + (c & 1);
                    st_i2[sp] = 2 * i2 + (c >> 1);
                    st_d[sp] = d + 1;
                    sp++;
                }
            }
            continue;
        }
        ho_eval(H, t1, t2, J, NULL, NULL);
        for (int q = 0; q < 3; q++) e[q] = J[q] - rho[q];
        double s = dot3(e, r) / rr;
        if (!(s >= cm->smin && s <= cm->smax) || nh >= cap) continue;
        /* insertion in depth order */
        int b = nh++;
        for (; b > 0 && hs[b - 1] > s; b--) {
            hs[b] = hs[b - 1];
            ht1[b] = ht1[b - 1];
            ht2[b] = ht2[b - 1];
        }
        hs[b] = s;
        ht1[b] = q1;
        ht2[b] = q2;
    }
    return nh;
}

/* Render a degree-R surface forest (geom: [R, then (R+1)^2 control points of 3
 * doubles per tree on the Gauss-Lobatto grid, m1 fastest]); arguments and
 * outputs as or_surface_render, with up to 2 R^2 hits per tree. */
int or_ho_surface_render(int64_t n, int ntrees, const int64_t *tree_begin, const double *geom, const uint8_t *level,
                         const uint32_t *x, const uint32_t *y, const double *As, const double *Is, const double *cam,
                         int64_t nsel, const int64_t *pix, double *Aout, double *Bout, double *Iout, int32_t *hit_leaf,
                         double *hit_s, int hcap)
{
    orcam c;
    cam_parse(cam, &c);
    int R = (int)geom[0];
    if (R < 2 || R > OR_HO_MAXR) return -1;
    int npt = (R + 1) * (R + 1);
    int64_t P = nsel >= 0 ? nsel : (int64_t)c.w * c.h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < P; q++) {
        int64_t p = nsel >= 0 ? pix[q] : q;
        int i = (int)(p % c.w), j = (int)(p / c.w);
        double rho[3], r[3];
        pixel_ray(&c, i, j, rho, r);
        double hs[64], hA[64], hB[64];
        int64_t hl[64];
        int nh = 0;
        for (int k = 0; k < ntrees; k++) {
            orho H;
            ho_init(&H, R, geom + 1 + 3 * npt * k);
            double s[2 * OR_HO_MAXR * OR_HO_MAXR], t1[2 * OR_HO_MAXR * OR_HO_MAXR], t2[2 * OR_HO_MAXR * OR_HO_MAXR];
            int m = ho_hits(&c, &H, rho, r, s, t1, t2, 2 * R * R, 1e-15);
            for (int a = 0; a < m && nh < 64; a++) {
                int64_t leaf = surface_leaf(level, x, y, tree_begin[k], tree_begin[k + 1], t1[a], t2[a]);
                if (leaf < 0) continue;
                /* the surface model with the normal of the degree-R map */
                double len = (double)(1u << (OR_QMAX - level[leaf]));
                double u = (t1[a] * (double)(1u << OR_QMAX) - (double)x[leaf]) / len;
                double v = (t2[a] * (double)(1u << OR_QMAX) - (double)y[leaf]) / len;
                double w[4] = {(1.0 - u) * (1.0 - v), u * (1.0 - v), (1.0 - u) * v, u * v};
                double as = 0.0, is = 0.0;
                for (int qq = 0; qq < 4; qq++) {
                    as += w[qq] * As[(int64_t)qq * n + leaf];
                    is += w[qq] * Is[(int64_t)qq * n + leaf];
                }
                double J[3], J1[3], J2[3], nr[3];
                ho_eval(&H, t1[a], t2[a], J, J1, J2);
                cross3(J1, J2, nr);
                double cosphi = fabs(dot3(nr, r)) / sqrt(dot3(nr, nr) * dot3(r, r));
                double Av = pow(as, 1.0 / cosphi);
                int b = nh++;
                for (; b > 0 && hs[b - 1] > s[a]; b--) {
                    hs[b] = hs[b - 1];
                    hA[b] = hA[b - 1];
                    hB[b] = hB[b - 1];
                    hl[b] = hl[b - 1];
                }
                hs[b] = s[a];
                hA[b] = Av;
                hB[b] = is * (1.0 - Av);
                hl[b] = leaf;
            }
        }
        double acc[2] = {1.0, 0.0}, t[2];
        for (int b = 0; b < nh; b++) {
            double sg[2] = {hA[b], hB[b]};
            or_combine(acc, sg, t);
            acc[0] = t[0];
            acc[1] = t[1];
        }
        Aout[q] = acc[0];
        Bout[q] = acc[1];
        Iout[q] = acc[0] * c.bg + acc[1];
        if (hit_leaf) {
            for (int b = 0; b < hcap; b++) {
                hit_leaf[q * hcap + b] = b < nh ? (int32_t)hl[b] : -1;
                hit_s[q * hcap + b] = b < nh ? hs[b] : 0.0;
            }
        }
    }
    return 0;
}

/* J of a degree-R tree at parameter points (for tests and generators' checks). */
void or_ho_map(const double *geom, int tree, int64_t m, const double *t, double *out)
{
    int R = (int)geom[0];
    orho H;
    ho_init(&H, R, geom + 1 + 3 * (R + 1) * (R + 1) * tree);
    for (int64_t i = 0; i < m; i++) ho_eval(&H, t[2 * i], t[2 * i + 1], out + 3 * i, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* degree-R volume trees: each tree maps its reference cube by a tensor     */
/* product of degree-R Lagrange polynomials on the Gauss-Lobatto nodes       */
/* (eq. nodal, eq. tensorgeom).  A ray meets a leaf (a sub-cube of the       */
/* reference cube) where it crosses the leaf's six curved faces (App. A.1:   */
/* each face is a degree-R patch, searched as the surfaces above); the       */
/* crossings cut the clip range into pieces, and the pieces whose midpoint   */
/* maps back into the leaf's cube are the ray's path through the leaf        */
/* (Sec. 2.1), adjacent ones joined.                                         */
/* ------------------------------------------------------------------------ */

#define OR_VOL_MAXCROSS 64 /* face crossings kept per (leaf, ray) */

typedef struct {
    orho B;        /* degree, nodes and the node basis (its z unused) */
    const double *z; /* (R+1)^3 control points of 3 doubles, m1 fastest, then m2, then m3 */
} orvol;

static void vol_init(orvol *V, int R, const double *z)
{
    ho_init(&V->B, R, NULL);
    V->z = z;
}

/* X(xi) and its Jacobian J[k][a] = dX_k / dxi_a. */
static void vol_eval(const orvol *V, const double *xi, double *X, double J[3][3])
{
    int n = V->B.R + 1;
    double p[3][OR_HO_MAXR + 1], d[3][OR_HO_MAXR + 1];
    for (int a = 0; a < 3; a++) ho_basis(&V->B, xi[a], p[a], d[a]);
    for (int k = 0; k < 3; k++) {
        double v = 0.0, v0 = 0.0, v1 = 0.0, v2 = 0.0;
        for (int m3 = 0; m3 < n; m3++)
            for (int m2 = 0; m2 < n; m2++)
                for (int m1 = 0; m1 < n; m1++) {
                    double zc = V->z[3 * (m1 + n * (m2 + n * m3)) + k];
                    v += zc * p[0][m1] * p[1][m2] * p[2][m3];
                    v0 += zc * d[0][m1] * p[1][m2] * p[2][m3];
                    v1 += zc * p[0][m1] * d[1][m2] * p[2][m3];
                    v2 += zc * p[0][m1] * p[1][m2] * d[2][m3];
                }
        X[k] = v;
        if (J) {
            J[k][0] = v0;
            J[k][1] = v1;
            J[k][2] = v2;
        }
    }
}

/* Reference coordinates of the point x: Newton's method on X(xi) = x from the
 * start xi (replaced by the result).  Returns 1 when the step falls below
 * 1e-14 within 60 iterations, 0 otherwise. */
static int vol_inverse(const orvol *V, const double *x, double *xi)
{
    for (int it = 0; it < 60; it++) {
        double X[3], J[3][3], e[3];
        vol_eval(V, xi, X, J);
        for (int k = 0; k < 3; k++) e[k] = X[k] - x[k];
        /* solve J s = e by Cramer's rule */
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det != 0.0) || !isfinite(det)) return 0;
        double s[3];
        for (int c = 0; c < 3; c++) {
            double M[3][3];
            for (int k = 0; k < 3; k++)
                for (int a = 0; a < 3; a++) M[k][a] = a == c ? e[k] : J[k][a];
            s[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                    M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) /
                   det;
        }
        double step = 0.0;
        for (int a = 0; a < 3; a++) {
            xi[a] -= s[a];
            step += fabs(s[a]);
        }
        if (!(fabs(xi[0]) < 4.0 && fabs(xi[1]) < 4.0 && fabs(xi[2]) < 4.0)) return 0;
        if (step < 1e-14) return 1;
    }
    return 0;
}

typedef struct {
    const orvol *V;
    double lo[3], len; /* the leaf's cube in the tree's reference coordinates */
} orvleaf;

static orvleaf vol_leaf(const orvol *V, uint8_t level, uint32_t x, uint32_t y, uint32_t z)
{
    orvleaf L;
    L.V = V;
    double q = ldexp(1.0, -OR_QMAX);
    L.lo[0] = (double)x * q;
    L.lo[1] = (double)y * q;
    L.lo[2] = (double)z * q;
    L.len = ldexp(1.0, -(int)level);
    return L;
}

/* Leaf reference coordinates of a real-space point (the field's argument). */
static void vol_ref(const void *ctx, const double *x, double *xil)
{
    const orvleaf *L = (const orvleaf *)ctx;
    double xi[3];
    for (int a = 0; a < 3; a++) xi[a] = L->lo[a] + 0.5 * L->len;
    vol_inverse(L->V, x, xi);
    for (int a = 0; a < 3; a++) xil[a] = (xi[a] - L->lo[a]) / L->len;
}

static int vol_inside(const orvleaf *L, const double *x)
{
    double xi[3];
    for (int a = 0; a < 3; a++) xi[a] = L->lo[a] + 0.5 * L->len;
    if (!vol_inverse(L->V, x, xi)) return 0;
    for (int a = 0; a < 3; a++)
        if (!(xi[a] >= L->lo[a] && xi[a] <= L->lo[a] + L->len)) return 0;
    return 1;
}

/* Face f of the leaf (axis f / 2 at its low (f even) or high end) as a
 * degree-R surface patch over [0, 1]^2: its control points are the map's
 * values on the face's node grid, which the patch interpolates exactly. */
static void vol_face(const orvleaf *L, int f, double *zf)
{
    int R = L->V->B.R, n = R + 1;
    int k = f / 2, a = (k + 1) % 3, b = (k + 2) % 3;
    for (int m2 = 0; m2 < n; m2++)
        for (int m1 = 0; m1 < n; m1++) {
            double xi[3];
            xi[k] = L->lo[k] + ((f & 1) ? L->len : 0.0);
            xi[a] = L->lo[a] + L->len * L->V->B.eta[m1];
            xi[b] = L->lo[b] + L->len * L->V->B.eta[m2];
            vol_eval(L->V, xi, zf + 3 * (m1 + n * m2), NULL);
        }
}

static int cmp_dbl(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* The ray's intervals inside the leaf, clipped to the camera's range: up to
 * cap intervals (s_in, s_out) into iv, nearest first; returns their number. */
static int vol_pair(const orcam *cm, const orvleaf *L, const double *rho, const double *r, double *iv, int cap)
{
    int R = L->V->B.R, n = R + 1;
    double ev[OR_VOL_MAXCROSS + 2];
    int ne = 0;
    ev[ne++] = cm->smin;
    ev[ne++] = cm->smax;
    for (int f = 0; f < 6; f++) {
        double zf[3 * (OR_HO_MAXR + 1) * (OR_HO_MAXR + 1)];
        vol_face(L, f, zf);
        orho H;
        ho_init(&H, R, zf);
        double hs[2 * OR_HO_MAXR * OR_HO_MAXR], t1[2 * OR_HO_MAXR * OR_HO_MAXR], t2[2 * OR_HO_MAXR * OR_HO_MAXR];
        /* a leaf's face is small: Newton's step stalls near 1e-15 there, so the
         * convergence test is looser; the canonical polish follows anyway */
        int m = ho_hits(cm, &H, rho, r, hs, t1, t2, 2 * R * R, 1e-12);
        for (int q = 0; q < m && ne < OR_VOL_MAXCROSS + 2; q++) ev[ne++] = hs[q];
        (void)n;
    }
    qsort(ev, (size_t)ne, sizeof(double), cmp_dbl);
    int ni = 0;
    double cur_in = 0.0, cur_out = -1.0;
    int open = 0;
    for (int q = 0; q + 1 < ne; q++) {
        double a = ev[q], b = ev[q + 1];
        if (!(b > a)) continue;
        double sm = 0.5 * (a + b), x[3];
        for (int k = 0; k < 3; k++) x[k] = rho[k] + sm * r[k];
        int in = vol_inside(L, x);
        if (in && open && a == cur_out) {
            cur_out = b; /* adjacent pieces inside: one interval */
        } else if (in) {
            if (open) {
                if (ni < cap) {
                    iv[2 * ni] = cur_in;
                    iv[2 * ni + 1] = cur_out;
                }
                ni++;
            }
            open = 1;
            cur_in = a;
            cur_out = b;
        }
    }
    if (open) {
        if (ni < cap) {
            iv[2 * ni] = cur_in;
            iv[2 * ni + 1] = cur_out;
        }
        ni++;
    }
    return ni;
}

/* Conservative pixel rectangle of a leaf: the camera-space box of the
 * Bernstein coefficients of the map over the leaf's cube (convex hull
 * property), from the map's values on an equispaced grid of the cube, widened
 * by a relative 1e-9. */
static int vol_rect(const orcam *c, const orvleaf *L, int *rect)
{
    int R = L->V->B.R, n = R + 1;
    double vals[3][(OR_HO_MAXR + 1) * (OR_HO_MAXR + 1) * (OR_HO_MAXR + 1)];
    for (int j3 = 0; j3 < n; j3++)
        for (int j2 = 0; j2 < n; j2++)
            for (int j1 = 0; j1 < n; j1++) {
                double xi[3] = {L->lo[0] + L->len * j1 / R, L->lo[1] + L->len * j2 / R, L->lo[2] + L->len * j3 / R};
                double X[3];
                vol_eval(L->V, xi, X, NULL);
                const double *ax[3] = {c->t, c->u, c->vh};
                for (int k = 0; k < 3; k++) {
                    double e[3] = {X[0] - c->o[0], X[1] - c->o[1], X[2] - c->o[2]};
                    vals[k][j1 + n * (j2 + n * j3)] = dot3(ax[k], e);
                }
            }
    double lo[3], hi[3], mag = 0.0;
    for (int k = 0; k < 3; k++) {
        /* equispaced values -> Bernstein coefficients along each axis in turn */
        double *v = vals[k], t[(OR_HO_MAXR + 1) * (OR_HO_MAXR + 1) * (OR_HO_MAXR + 1)];
        for (int ax = 0; ax < 3; ax++) {
            int st = ax == 0 ? 1 : (ax == 1 ? n : n * n);
            for (int q = 0; q < n * n * n; q++) {
                int jj = (q / st) % n;
                double s = 0.0;
                for (int j = 0; j < n; j++) s += L->V->B.einv[jj * n + j] * v[q + (j - jj) * st];
                t[q] = s;
            }
            for (int q = 0; q < n * n * n; q++) v[q] = t[q];
        }
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
        for (int q = 0; q < n * n * n; q++) {
            lo[k] = fmin(lo[k], v[q]);
            hi[k] = fmax(hi[k], v[q]);
        }
        mag = fmax(mag, fmax(fabs(lo[k]), fabs(hi[k])));
    }
    double m = 1e-9 * (1.0 + mag);
    for (int k = 0; k < 3; k++) {
        lo[k] -= m;
        hi[k] += m;
    }
    rect[0] = rect[2] = 1;
    rect[1] = rect[3] = 0;
    if (hi[2] < c->n || lo[2] > c->zfar) return 0;
    double Z0 = lo[2] < c->n ? c->n : lo[2], Z1 = hi[2] > c->zfar ? c->zfar : hi[2];
    pixel_range(c, lo[0], hi[0], Z0, Z1, c->cx, c->w, &rect[0], &rect[1]);
    pixel_range(c, lo[1], hi[1], Z0, Z1, c->cy, c->h, &rect[2], &rect[3]);
    return rect[0] <= rect[1] && rect[2] <= rect[3];
}

/* Intervals of explicit candidates: leaf[q] at pixel (pi[q], pj[q]) of camera
 * cam; nseg[q] = the number of intervals, iv[4 q .. 4 q + 3] the first two
 * (s_in, s_out) pairs, zeros where absent.  geom: [R, then (R+1)^3 control
 * points of 3 doubles per tree]. */
int or_vol_cands(int64_t m, const int64_t *leaf, const int32_t *pi, const int32_t *pj, int ntrees,
                 const int64_t *tree_begin, const double *geom, const uint8_t *level, const uint32_t *x,
                 const uint32_t *y, const uint32_t *z, const double *cam, int32_t *nseg, double *iv)
{
    orcam c;
    cam_parse(cam, &c);
    int R = (int)geom[0];
    if (R < 2 || R > OR_HO_MAXR) return -1;
    int npt = (R + 1) * (R + 1) * (R + 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < m; q++) {
        int64_t l = leaf[q];
        orvol V;
        vol_init(&V, R, geom + 1 + 3 * npt * tree_of(l, ntrees, tree_begin));
        orvleaf L = vol_leaf(&V, level[l], x[l], y[l], z[l]);
        double rho[3], r[3], w[2 * OR_VOL_MAXCROSS];
        pixel_ray(&c, pi[q], pj[q], rho, r);
        int k = vol_pair(&c, &L, rho, r, w, OR_VOL_MAXCROSS);
        nseg[q] = k;
        for (int h = 0; h < 4; h++) iv[4 * q + h] = 0.0;
        for (int h = 0; h < k && h < 2; h++) {
            iv[4 * q + 2 * h] = w[2 * h];
            iv[4 * q + 2 * h + 1] = w[2 * h + 1];
        }
    }
    return 0;
}

/* Render one camera of a volume forest: every leaf whose conservative
 * rectangle holds the pixel contributes its intervals, integrated with the
 * field at reference coordinates from the inverse map (Newton), then all of a
 * pixel's segments are folded nearest first.  Arguments and outputs as
 * or_shell_render; stats[0] = segments, stats[1] = overlaps. */
int or_vol_render(int64_t n, int ntrees, const int64_t *tree_begin, const double *geom, const uint8_t *level,
                  const uint32_t *x, const uint32_t *y, const uint32_t *z, int kind, const double *kap,
                  const double *eps, int method, int substeps, const double *cam, int64_t npix_sel,
                  const int64_t *pix_sel, double *Aout, double *Bout, double *Iout, int32_t *nseg_pix, int64_t *stats)
{
    orcam c;
    cam_parse(cam, &c);
    int R = (int)geom[0];
    if (R < 2 || R > OR_HO_MAXR) return -1;
    int npt = (R + 1) * (R + 1) * (R + 1);
    int64_t W = c.w, H = c.h, P = W * H;
    int64_t npo = (npix_sel >= 0) ? npix_sel : P;
    int64_t *selmap = NULL;
    if (npix_sel >= 0) {
        selmap = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);
        for (int64_t p = 0; p < P; p++) selmap[p] = -1;
        for (int64_t q = 0; q < npix_sel; q++) selmap[pix_sel[q]] = q;
    }
    /* candidates (leaf, pixel) of every leaf's rectangle */
    int64_t cap = 1 << 16, nc = 0;
    int64_t *cl = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap), *cp = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    for (int64_t l = 0; l < n; l++) {
        orvol V;
        vol_init(&V, R, geom + 1 + 3 * npt * tree_of(l, ntrees, tree_begin));
        orvleaf L = vol_leaf(&V, level[l], x[l], y[l], z[l]);
        int rr[4];
        if (!vol_rect(&c, &L, rr)) continue;
        for (int j = rr[2]; j <= rr[3]; j++)
            for (int i = rr[0]; i <= rr[1]; i++) {
                int64_t p = (int64_t)j * W + i;
                if (selmap && selmap[p] < 0) continue;
                if (nc == cap) {
                    cap *= 2;
                    cl = (int64_t *)realloc(cl, sizeof(int64_t) * (size_t)cap);
                    cp = (int64_t *)realloc(cp, sizeof(int64_t) * (size_t)cap);
                }
                cl[nc] = l;
                cp[nc] = p;
                nc++;
            }
    }
    /* intervals per candidate (up to 4), then the segments */
    double *civ = (double *)malloc(sizeof(double) * 8 * (size_t)(nc > 0 ? nc : 1));
    int *cn = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nc; q++) {
        int64_t l = cl[q];
        orvol V;
        vol_init(&V, R, geom + 1 + 3 * npt * tree_of(l, ntrees, tree_begin));
        orvleaf L = vol_leaf(&V, level[l], x[l], y[l], z[l]);
        double rho[3], r[3], w[2 * OR_VOL_MAXCROSS];
        pixel_ray(&c, (int)(cp[q] % W), (int)(cp[q] / W), rho, r);
        int k = vol_pair(&c, &L, rho, r, w, OR_VOL_MAXCROSS);
        cn[q] = k < 4 ? k : 4;
        for (int h = 0; h < cn[q]; h++) {
            civ[8 * q + 2 * h] = w[2 * h];
            civ[8 * q + 2 * h + 1] = w[2 * h + 1];
        }
    }
    int64_t ns = 0;
    for (int64_t q = 0; q < nc; q++) ns += cn[q];
    orseg *segs = (orseg *)malloc(sizeof(orseg) * (size_t)(ns > 0 ? ns : 1));
    ns = 0;
    for (int64_t q = 0; q < nc; q++)
        for (int h = 0; h < cn[q]; h++) {
            segs[ns].pix = selmap ? selmap[cp[q]] : cp[q];
            segs[ns].s_in = civ[8 * q + 2 * h];
            segs[ns].s_out = civ[8 * q + 2 * h + 1];
            segs[ns].leaf = cl[q];
            ns++;
        }
    free(cl);
    free(cp);
    free(civ);
    free(cn);
    free(selmap);
    qsort(segs, (size_t)ns, sizeof(orseg), seg_cmp);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < ns; k++) {
        orseg *s = &segs[k];
        int64_t p = (npix_sel >= 0) ? pix_sel[s->pix] : s->pix;
        double rho[3], r[3];
        pixel_ray(&c, (int)(p % W), (int)(p / W), rho, r);
        int64_t l = s->leaf;
        orvol V;
        vol_init(&V, R, geom + 1 + 3 * npt * tree_of(l, ntrees, tree_begin));
        orvleaf L = vol_leaf(&V, level[l], x[l], y[l], z[l]);
        leaffield F;
        leaf_field(kind, n, l, kap, eps, &F);
        dn A, B;
        segment_dn_ref(&F, vol_ref, &L, rho, r, ray_norm(r), s->s_in, s->s_out, method, substeps, 0.0, 0, &A, &B);
        s->A = A.v;
        s->B = B.v;
    }
    int64_t overlaps = 0;
    for (int64_t q = 0; q < npo; q++) {
        Aout[q] = 1.0;
        Bout[q] = 0.0;
        if (nseg_pix) nseg_pix[q] = 0;
    }
    int64_t k = 0;
    while (k < ns) {
        int64_t q = segs[k].pix;
        double acc[2] = {1.0, 0.0};
        double prev_out = -INFINITY;
        int cnt = 0;
        for (; k < ns && segs[k].pix == q; k++) {
            if (segs[k].s_in < prev_out - 1e-12 * fabs(prev_out)) overlaps++;
            prev_out = segs[k].s_out;
            double sg[2] = {segs[k].A, segs[k].B}, t[2];
            or_combine(acc, sg, t);
            acc[0] = t[0];
            acc[1] = t[1];
            cnt++;
        }
        Aout[q] = acc[0];
        Bout[q] = acc[1];
        if (nseg_pix) nseg_pix[q] = cnt;
    }
    for (int64_t q = 0; q < npo; q++) Iout[q] = Aout[q] * c.bg + Bout[q];
    if (stats) {
        stats[0] = ns;
        stats[1] = overlaps;
    }
    free(segs);
    return 0;
}

/* X of tree `tree` at m reference points, and its inverse by Newton's method
 * from the cube's centre (for tests). */
void or_vol_map(const double *geom, int tree, int64_t m, const double *xi, double *out)
{
    int R = (int)geom[0];
    orvol V;
    vol_init(&V, R, geom + 1 + 3 * (R + 1) * (R + 1) * (R + 1) * tree);
    for (int64_t i = 0; i < m; i++) vol_eval(&V, xi + 3 * i, out + 3 * i, NULL);
}

int or_vol_inverse(const double *geom, int tree, int64_t m, const double *x, double *xi)
{
    int R = (int)geom[0];
    orvol V;
    vol_init(&V, R, geom + 1 + 3 * (R + 1) * (R + 1) * (R + 1) * tree);
    int ok = 1;
    for (int64_t i = 0; i < m; i++) {
        double t[3] = {0.5, 0.5, 0.5};
        ok &= vol_inverse(&V, x + 3 * i, t);
        for (int a = 0; a < 3; a++) xi[3 * i + a] = t[a];
    }
    return ok;
}
