/*
 * oracle.c -- plain, slow, double-precision reference of the tile-based
 * 3D Gaussian Splatting rasterizer that Local-GS accelerates.
 *
 * TEST INFRASTRUCTURE ONLY.  It is built into liboracle.so and called from the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg.  The
 * product library never links, loads or calls it, and the two share no code.
 *
 * What it computes, and where the paper defines it (Local-GS, arXiv 2606.16566):
 *
 *  - projection ("preprocessing"): each 3D Gaussian (mean, scale, rotation,
 *    opacity, SH colour) is projected to a 2D mean, a 2D conic and a colour;
 *    the Gaussian's screen footprint decides which 16x16 tiles it touches
 *    (Sec. II-A, pipeline description and Fig. 2).  The paper inherits the
 *    details from 3DGS and does not restate them; the readings used here
 *    (EWA Jacobian, 0.3 px low-pass, near plane, SH basis, exact footprint of
 *    the alpha >= 1/255 ellipse) are listed in the design notes.
 *  - per-pixel blending: alpha = min(0.99, o * exp(-q/2)) with the conic
 *    quadratic q (Sec. III-B, Eqs. for alpha and the conic matrix), Gaussians
 *    with alpha < 1/255 skipped, front-to-back accumulation that stops before
 *    the first Gaussian that would take T below 1e-4 (Alg. 1, baseline column).
 *  - binning: per-tile lists ordered by (depth, index) (Sec. II-A).
 *  - gradients: the derivative of the blended colour and final transmittance
 *    with respect to every projected attribute, written out directly from the
 *    blending sum (no recurrence), and the projection Jacobian obtained by
 *    forward-mode dual numbers through the same projection code.  The paper
 *    has no backward pass; this is the plain definition of the derivative.
 *
 * Every quantity is IEEE double unless stated.  The only single-precision
 * step is the depth key, which is defined as the float rounding of the
 * camera-space z computed in double with a fixed fused-multiply-add order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* camera block: 27 doubles                                                  */
/* ------------------------------------------------------------------------ */
enum {
    CAM_VIEW = 0,   /* 12: world->camera [R|t], row-major 3x4 */
    CAM_POS = 12,   /* 3: camera centre in world space */
    CAM_FX = 15, CAM_FY = 16, CAM_CX = 17, CAM_CY = 18,
    CAM_TANX = 19, CAM_TANY = 20,  /* tan of half field of view */
    CAM_W = 21, CAM_H = 22, CAM_ZNEAR = 23,
    CAM_BG = 24,    /* 3: background colour */
    CAM_LEN = 27
};

#define TILE 16
#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_MIN 1e-4
#define LOWPASS 0.3
#define FRUSTUM_GUARD 1.3
/* footprint slack: the rectangle of touched pixel centres is taken for the
   ellipse q <= tau * (1 + FOOT_REL) + FOOT_ABS, widened by FOOT_PX pixels */
#define FOOT_REL 1e-5
#define FOOT_ABS 1e-5
#define FOOT_PX 1e-2

/* ------------------------------------------------------------------------ */
/* forward-mode dual numbers: value + derivative w.r.t. the 11 geometric raw */
/* parameters of one Gaussian: mean (0..2), log-scale (3..5),                */
/* quaternion w,x,y,z (6..9), opacity logit (10)                             */
/* ------------------------------------------------------------------------ */
#define NT 11
typedef struct { double v; double t[NT]; } dual;

static dual dconst(double v) { dual r; r.v = v; memset(r.t, 0, sizeof r.t); return r; }
static dual dvar(double v, int k) { dual r = dconst(v); r.t[k] = 1.0; return r; }
static dual dadd(dual a, dual b) { a.v += b.v; for (int i = 0; i < NT; ++i) a.t[i] += b.t[i]; return a; }
static dual dsub(dual a, dual b) { a.v -= b.v; for (int i = 0; i < NT; ++i) a.t[i] -= b.t[i]; return a; }
static dual dscale(dual a, double s) { a.v *= s; for (int i = 0; i < NT; ++i) a.t[i] *= s; return a; }
static dual daddc(dual a, double c) { a.v += c; return a; }
static dual dmul(dual a, dual b)
{
    dual r; r.v = a.v * b.v;
    for (int i = 0; i < NT; ++i) r.t[i] = a.t[i] * b.v + a.v * b.t[i];
    return r;
}
static dual ddiv(dual a, dual b)
{
    dual r; r.v = a.v / b.v;
    for (int i = 0; i < NT; ++i) r.t[i] = (a.t[i] * b.v - a.v * b.t[i]) / (b.v * b.v);
    return r;
}
static dual dsqrt(dual a)
{
    dual r; r.v = sqrt(a.v);
    for (int i = 0; i < NT; ++i) r.t[i] = a.t[i] / (2.0 * r.v);
    return r;
}
static dual dexp(dual a)
{
    dual r; r.v = exp(a.v);
    for (int i = 0; i < NT; ++i) r.t[i] = a.t[i] * r.v;
    return r;
}

/* ------------------------------------------------------------------------ */
/* real spherical harmonics, degree <= 3, Condon-Shortley phase included.    */
/* Y_l^0 = K_l^0 P_l^0(z);  Y_l^{+m} = sqrt2 K_l^m P_l^m(z) cos(m phi);      */
/* Y_l^{-m} = sqrt2 K_l^m P_l^m(z) sin(m phi), index l*l + l + m.            */
/* Evaluated without angles: P_l^m(z) = Q_l^m(z) sin^m(theta) with Q from    */
/* the associated-Legendre recurrence, and sin^m(theta) e^{i m phi} =        */
/* (x + i y)^m for a unit direction.  Duals carry d/d(raw params).           */
/* ------------------------------------------------------------------------ */
static double factorial(int k) { double f = 1; for (int i = 2; i <= k; ++i) f *= i; return f; }

static void sh_basis_dual(int deg, dual x, dual y, dual z, dual *Y /* (deg+1)^2 */)
{
    /* Re/Im of (x + i y)^m */
    dual cr[4], ci[4];
    cr[0] = dconst(1.0); ci[0] = dconst(0.0);
    for (int m = 1; m <= deg; ++m) {
        cr[m] = dsub(dmul(cr[m - 1], x), dmul(ci[m - 1], y));
        ci[m] = dadd(dmul(cr[m - 1], y), dmul(ci[m - 1], x));
    }
    for (int m = 0; m <= deg; ++m) {
        /* Q_m^m = (-1)^m (2m-1)!! */
        double dfact = 1.0;
        for (int k = 2 * m - 1; k > 0; k -= 2) dfact *= k;
        dual q_lm2 = dconst(0.0);
        dual q_lm1 = dconst((m & 1) ? -dfact : dfact);
        for (int l = m; l <= deg; ++l) {
            dual q;
            if (l == m) q = q_lm1;
            else if (l == m + 1) q = dscale(dmul(z, q_lm1), 2.0 * m + 1.0);
            else q = dscale(dsub(dscale(dmul(z, q_lm1), 2.0 * l - 1.0), dscale(q_lm2, l + m - 1.0)),
                            1.0 / (l - m));
            if (l > m) { q_lm2 = q_lm1; q_lm1 = q; }
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
            if (m == 0) {
                Y[l * l + l] = dscale(q, K);
            } else {
                Y[l * l + l + m] = dscale(dmul(q, cr[m]), sqrt(2.0) * K);
                Y[l * l + l - m] = dscale(dmul(q, ci[m]), sqrt(2.0) * K);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* projection of one Gaussian                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int visible;
    dual mx, my;            /* projected mean (pixels) */
    dual ka, kb, kc;        /* conic: q = ka dx^2 + 2 kb dx dy + kc dy^2 */
    dual op;                /* opacity */
    dual col[3];            /* colour after the clamp at 0 */
    int col_clamped[3];
    double Y[16];           /* SH basis values (for d colour / d sh) */
    float depth;            /* depth key */
    int rect[4];            /* touched tiles [tx0, ty0, tx1, ty1), empty if invisible */
} proj_t;

static int finite_all(const double *p, int k) { for (int i = 0; i < k; ++i) if (!isfinite(p[i])) return 0; return 1; }

static void project_one(const double *cam, int deg, const double *m3, const double *ls, const double *qt,
                        double logit, const double *sh, proj_t *P)
{
    memset(P, 0, sizeof *P);
    P->depth = INFINITY;
    int K = (deg + 1) * (deg + 1);
    if (!finite_all(m3, 3) || !finite_all(ls, 3) || !finite_all(qt, 4) || !isfinite(logit)
        || !finite_all(sh, 3 * K))
        return;
    const double *V = cam + CAM_VIEW;
    dual mu[3] = { dvar(m3[0], 0), dvar(m3[1], 1), dvar(m3[2], 2) };
    dual s[3] = { dexp(dvar(ls[0], 3)), dexp(dvar(ls[1], 4)), dexp(dvar(ls[2], 5)) };
    dual q[4] = { dvar(qt[0], 6), dvar(qt[1], 7), dvar(qt[2], 8), dvar(qt[3], 9) };
    dual o = ddiv(dconst(1.0), daddc(dexp(dscale(dvar(logit, 10), -1.0)), 1.0));

    /* camera-space position, value with the fixed FMA order of the depth key */
    dual t[3];
    for (int k = 0; k < 3; ++k) {
        t[k] = dconst(fma(V[4 * k + 2], m3[2], fma(V[4 * k + 1], m3[1], fma(V[4 * k + 0], m3[0], V[4 * k + 3]))));
        for (int j = 0; j < 3; ++j) t[k].t[j] = V[4 * k + j];
    }
    if (!(t[2].v > cam[CAM_ZNEAR])) return;

    double qn2 = qt[0] * qt[0] + qt[1] * qt[1] + qt[2] * qt[2] + qt[3] * qt[3];
    if (!(qn2 > 0.0)) return;
    dual n2 = dadd(dadd(dmul(q[0], q[0]), dmul(q[1], q[1])), dadd(dmul(q[2], q[2]), dmul(q[3], q[3])));
    dual inv = ddiv(dconst(1.0), dsqrt(n2));
    dual w = dmul(q[0], inv), x = dmul(q[1], inv), y = dmul(q[2], inv), z = dmul(q[3], inv);

    /* rotation matrix of the unit quaternion (w, x, y, z) */
    dual R[3][3];
    R[0][0] = dsub(dconst(1.0), dscale(dadd(dmul(y, y), dmul(z, z)), 2.0));
    R[0][1] = dscale(dsub(dmul(x, y), dmul(w, z)), 2.0);
    R[0][2] = dscale(dadd(dmul(x, z), dmul(w, y)), 2.0);
    R[1][0] = dscale(dadd(dmul(x, y), dmul(w, z)), 2.0);
    R[1][1] = dsub(dconst(1.0), dscale(dadd(dmul(x, x), dmul(z, z)), 2.0));
    R[1][2] = dscale(dsub(dmul(y, z), dmul(w, x)), 2.0);
    R[2][0] = dscale(dsub(dmul(x, z), dmul(w, y)), 2.0);
    R[2][1] = dscale(dadd(dmul(y, z), dmul(w, x)), 2.0);
    R[2][2] = dsub(dconst(1.0), dscale(dadd(dmul(x, x), dmul(y, y)), 2.0));

    /* world covariance Sigma3 = (R S)(R S)^T */
    dual M[3][3], S3[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) M[i][j] = dmul(R[i][j], s[j]);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
        dual acc = dconst(0.0);
        for (int k = 0; k < 3; ++k) acc = dadd(acc, dmul(M[i][k], M[j][k]));
        S3[i][j] = acc;
    }

    /* EWA: Jacobian of the perspective map at the (guard-band clamped) point */
    double fx = cam[CAM_FX], fy = cam[CAM_FY];
    double limx = FRUSTUM_GUARD * cam[CAM_TANX], limy = FRUSTUM_GUARD * cam[CAM_TANY];
    dual u = ddiv(t[0], t[2]), v = ddiv(t[1], t[2]);
    if (u.v < -limx) u = dconst(-limx); else if (u.v > limx) u = dconst(limx);
    if (v.v < -limy) v = dconst(-limy); else if (v.v > limy) v = dconst(limy);
    dual rz = ddiv(dconst(1.0), t[2]);
    dual J[2][3];
    J[0][0] = dscale(rz, fx); J[0][1] = dconst(0.0); J[0][2] = dscale(dmul(u, rz), -fx);
    J[1][0] = dconst(0.0); J[1][1] = dscale(rz, fy); J[1][2] = dscale(dmul(v, rz), -fy);
    /* T = J W (W = rotation part of the view matrix) */
    dual T[2][3];
    for (int i = 0; i < 2; ++i) for (int j = 0; j < 3; ++j) {
        dual acc = dconst(0.0);
        for (int k = 0; k < 3; ++k) acc = dadd(acc, dscale(J[i][k], V[4 * k + j]));
        T[i][j] = acc;
    }
    /* Sigma2 = T Sigma3 T^T + 0.3 I */
    dual S2[2][2];
    for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) {
        dual acc = dconst(0.0);
        for (int k = 0; k < 3; ++k) for (int l = 0; l < 3; ++l)
            acc = dadd(acc, dmul(dmul(T[i][k], S3[k][l]), T[j][l]));
        S2[i][j] = acc;
    }
    S2[0][0] = daddc(S2[0][0], LOWPASS);
    S2[1][1] = daddc(S2[1][1], LOWPASS);
    dual det = dsub(dmul(S2[0][0], S2[1][1]), dmul(S2[0][1], S2[1][0]));
    if (!(det.v > 0.0)) return;
    P->ka = ddiv(S2[1][1], det);
    P->kb = dscale(ddiv(S2[0][1], det), -1.0);
    P->kc = ddiv(S2[0][0], det);

    /* projected mean: pinhole at the unclamped point */
    P->mx = daddc(dscale(ddiv(t[0], t[2]), fx), cam[CAM_CX]);
    P->my = daddc(dscale(ddiv(t[1], t[2]), fy), cam[CAM_CY]);
    P->op = o;

    /* view-dependent colour */
    dual dir[3];
    for (int k = 0; k < 3; ++k) dir[k] = daddc(mu[k], -cam[CAM_POS + k]);
    dual dn = dsqrt(dadd(dadd(dmul(dir[0], dir[0]), dmul(dir[1], dir[1])), dmul(dir[2], dir[2])));
    dual Yd[16];
    if (dn.v > 0.0) {
        for (int k = 0; k < 3; ++k) dir[k] = ddiv(dir[k], dn);
        sh_basis_dual(deg, dir[0], dir[1], dir[2], Yd);
    } else {
        sh_basis_dual(deg, dconst(0.0), dconst(0.0), dconst(1.0), Yd);
        for (int k = 0; k < K; ++k) Yd[k] = dconst(Yd[k].v);
    }
    for (int k = 0; k < K; ++k) P->Y[k] = Yd[k].v;
    for (int ch = 0; ch < 3; ++ch) {
        dual acc = dconst(0.5);
        for (int k = 0; k < K; ++k) acc = dadd(acc, dscale(Yd[k], sh[3 * k + ch]));
        if (acc.v < 0.0) { P->col[ch] = dconst(0.0); P->col_clamped[ch] = 1; }
        else P->col[ch] = acc;
    }

    /* footprint: alpha >= 1/255  <=>  q <= tau = 2 ln(255 o) */
    double tau = 2.0 * log(255.0 * o.v);
    if (!(tau > 0.0)) return;
    double tau_m = tau * (1.0 + FOOT_REL) + FOOT_ABS;
    double rx = sqrt(tau_m * S2[0][0].v) + FOOT_PX, ry = sqrt(tau_m * S2[1][1].v) + FOOT_PX;
    double W = cam[CAM_W], H = cam[CAM_H];
    double x0 = ceil(P->mx.v - rx), x1 = floor(P->mx.v + rx);
    double y0 = ceil(P->my.v - ry), y1 = floor(P->my.v + ry);
    if (!(isfinite(x0) && isfinite(x1) && isfinite(y0) && isfinite(y1))) return;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > W - 1) x1 = W - 1;
    if (y1 > H - 1) y1 = H - 1;
    if (x0 > x1 || y0 > y1) return;
    P->rect[0] = (int)x0 / TILE; P->rect[1] = (int)y0 / TILE;
    P->rect[2] = (int)x1 / TILE + 1; P->rect[3] = (int)y1 / TILE + 1;
    P->depth = (float)t[2].v;
    P->visible = 1;
}

/*
 * oracle_project: projection of n Gaussians.
 * Outputs (all length n or n x k, double unless stated): visible (int32),
 * means2d [n,2], conic [n,3] (a, b, c), opacity [n], rgb [n,3],
 * depth (float32, +inf when invisible), rect [n,4] int32 tile rectangle
 * [tx0, ty0, tx1, ty1) (zeros when invisible), rgb_clamped [n,3] int32.
 */
void oracle_project(const double *cam, int64_t n, int deg, const double *means3d, const double *log_scales,
                    const double *quats, const double *logits, const double *sh,
                    int32_t *visible, double *means2d, double *conic, double *opacity, double *rgb,
                    float *depth, int32_t *rect, int32_t *rgb_clamped)
{
    int K = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < n; ++i) {
        proj_t P;
        project_one(cam, deg, means3d + 3 * i, log_scales + 3 * i, quats + 4 * i, logits[i], sh + 3 * K * i, &P);
        visible[i] = P.visible;
        means2d[2 * i] = P.mx.v; means2d[2 * i + 1] = P.my.v;
        conic[3 * i] = P.ka.v; conic[3 * i + 1] = P.kb.v; conic[3 * i + 2] = P.kc.v;
        opacity[i] = P.op.v;
        for (int c = 0; c < 3; ++c) { rgb[3 * i + c] = P.col[c].v; rgb_clamped[3 * i + c] = P.col_clamped[c]; }
        depth[i] = P.depth;
        for (int c = 0; c < 4; ++c) rect[4 * i + c] = P.rect[c];
    }
}

/*
 * oracle_project_backward: chain rule from the projected attributes to the raw
 * parameters.  g_means2d [n,2], g_conic [n,3], g_opacity [n], g_rgb [n,3] are
 * dL/d(projected attribute); writes dL/d means3d [n,3], log_scales [n,3],
 * quats [n,4], logits [n], sh [n,K,3].  Invisible Gaussians get zero.
 */
void oracle_project_backward(const double *cam, int64_t n, int deg, const double *means3d,
                             const double *log_scales, const double *quats, const double *logits,
                             const double *sh, const double *g_means2d, const double *g_conic,
                             const double *g_opacity, const double *g_rgb,
                             double *d_means3d, double *d_log_scales, double *d_quats,
                             double *d_logits, double *d_sh)
{
    int K = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < n; ++i) {
        proj_t P;
        project_one(cam, deg, means3d + 3 * i, log_scales + 3 * i, quats + 4 * i, logits[i], sh + 3 * K * i, &P);
        double g[NT];
        memset(g, 0, sizeof g);
        double *dsh = d_sh + 3 * K * i;
        memset(dsh, 0, sizeof(double) * 3 * K);
        if (P.visible) {
            const dual *outs[9] = { &P.mx, &P.my, &P.ka, &P.kb, &P.kc, &P.op, &P.col[0], &P.col[1], &P.col[2] };
            double go[9] = { g_means2d[2 * i], g_means2d[2 * i + 1], g_conic[3 * i], g_conic[3 * i + 1],
                             g_conic[3 * i + 2], g_opacity[i], g_rgb[3 * i], g_rgb[3 * i + 1], g_rgb[3 * i + 2] };
            for (int o = 0; o < 9; ++o)
                for (int k = 0; k < NT; ++k) g[k] += go[o] * outs[o]->t[k];
            for (int k = 0; k < K; ++k)
                for (int c = 0; c < 3; ++c)
                    dsh[3 * k + c] = P.col_clamped[c] ? 0.0 : g_rgb[3 * i + c] * P.Y[k];
        }
        for (int k = 0; k < 3; ++k) d_means3d[3 * i + k] = g[k];
        for (int k = 0; k < 3; ++k) d_log_scales[3 * i + k] = g[3 + k];
        for (int k = 0; k < 4; ++k) d_quats[4 * i + k] = g[6 + k];
        d_logits[i] = g[10];
    }
}

/* evaluate the SH basis for one direction (used by tests to pin it) */
void oracle_sh_basis(int deg, double x, double y, double z, double *out)
{
    dual Y[16];
    sh_basis_dual(deg, dconst(x), dconst(y), dconst(z), Y);
    for (int k = 0; k < (deg + 1) * (deg + 1); ++k) out[k] = Y[k].v;
}

/* ------------------------------------------------------------------------ */
/* ordering: ascending (depth key, index)                                    */
/* ------------------------------------------------------------------------ */
typedef struct { float d; int32_t id; } dkey;
static int cmp_dkey(const void *a, const void *b)
{
    const dkey *x = (const dkey *)a, *y = (const dkey *)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/*
 * oracle_tile_lists: for every tile, the ids of the Gaussians whose tile
 * rectangle contains it, in ascending (depth, id) order.  offsets has
 * num_tiles+1 entries; ids must hold sum of rectangle areas (see
 * oracle_count_pairs).  Returns the pair count.
 */
int64_t oracle_count_pairs(int64_t n, const int32_t *visible, const int32_t *rect)
{
    int64_t p = 0;
    for (int64_t i = 0; i < n; ++i)
        if (visible[i]) p += (int64_t)(rect[4 * i + 2] - rect[4 * i]) * (rect[4 * i + 3] - rect[4 * i + 1]);
    return p;
}

int64_t oracle_tile_lists(int64_t n, const int32_t *visible, const float *depth, const int32_t *rect,
                          int tiles_x, int tiles_y, int64_t *offsets, int32_t *ids)
{
    int64_t nt = (int64_t)tiles_x * tiles_y;
    for (int64_t t = 0; t <= nt; ++t) offsets[t] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!visible[i]) continue;
        for (int ty = rect[4 * i + 1]; ty < rect[4 * i + 3]; ++ty)
            for (int tx = rect[4 * i]; tx < rect[4 * i + 2]; ++tx) offsets[(int64_t)ty * tiles_x + tx + 1]++;
    }
    for (int64_t t = 0; t < nt; ++t) offsets[t + 1] += offsets[t];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (nt > 0 ? nt : 1));
    for (int64_t t = 0; t < nt; ++t) fill[t] = offsets[t];
    for (int64_t i = 0; i < n; ++i) {
        if (!visible[i]) continue;
        for (int ty = rect[4 * i + 1]; ty < rect[4 * i + 3]; ++ty)
            for (int tx = rect[4 * i]; tx < rect[4 * i + 2]; ++tx) ids[fill[(int64_t)ty * tiles_x + tx]++] = (int32_t)i;
    }
    free(fill);
    int64_t maxlen = 0;
    for (int64_t t = 0; t < nt; ++t) if (offsets[t + 1] - offsets[t] > maxlen) maxlen = offsets[t + 1] - offsets[t];
    dkey *buf = (dkey *)malloc(sizeof(dkey) * (maxlen > 0 ? maxlen : 1));
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = offsets[t], b = offsets[t + 1];
        for (int64_t k = a; k < b; ++k) { buf[k - a].d = depth[ids[k]]; buf[k - a].id = ids[k]; }
        qsort(buf, (size_t)(b - a), sizeof(dkey), cmp_dkey);
        for (int64_t k = a; k < b; ++k) ids[k] = buf[k - a].id;
    }
    free(buf);
    return offsets[nt];
}

/*
 * Minimum of the quadratic q(d) = a dx^2 + 2 b dx dy + c dy^2 (positive
 * definite) over the rectangle [x0, x1] x [y0, y1]: 0 if the rectangle holds
 * the origin, else the minimum lies on its boundary, and along each edge q is
 * a convex parabola, smallest at its stationary point clamped to the edge.
 */
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

double oracle_rect_min_q(double a, double b, double c, double x0, double x1, double y0, double y1)
{
    if (x0 <= 0.0 && 0.0 <= x1 && y0 <= 0.0 && 0.0 <= y1) return 0.0;
    double best = INFINITY;
    const double xs[2] = { x0, x1 }, ys[2] = { y0, y1 };
    for (int k = 0; k < 2; ++k) {
        double X = xs[k], Y = clampd(-b * X / c, y0, y1);        /* edge x = X */
        double v = a * X * X + 2.0 * b * X * Y + c * Y * Y;
        if (v < best) best = v;
        Y = ys[k];
        X = clampd(-b * Y / a, x0, x1);                          /* edge y = Y */
        v = a * X * X + 2.0 * b * X * Y + c * Y * Y;
        if (v < best) best = v;
    }
    return best;
}

/*
 * oracle_tile_lists_exact: per-tile lists as oracle_tile_lists, but a
 * Gaussian is listed in a tile of its rectangle only where its alpha >= 1/255
 * ellipse, q <= tau (1 + tau_rel) + tau_abs with tau = 2 ln(255 o), meets the
 * rectangle spanned by the tile's pixel centres (clip != 0: the in-image ones;
 * else all 16 x 16) widened by `pad` pixels on every side: the exact
 * tile-ellipse intersection of the footprint (Sec. II-A's tile assignment
 * made exact, as in the block-level culling the paper builds on).  Returns
 * the pair count; with ids == NULL only counts (offsets still filled).
 */
int64_t oracle_tile_lists_exact(int64_t n, const int32_t *visible, const float *depth, const int32_t *rect,
                                const double *means2d, const double *conic, const double *opacity, int W, int H,
                                double tau_rel, double tau_abs, double pad, int clip, int64_t *offsets,
                                int32_t *ids)
{
    int tiles_x = (W + TILE - 1) / TILE, tiles_y = (H + TILE - 1) / TILE;
    int64_t nt = (int64_t)tiles_x * tiles_y;
    for (int64_t t = 0; t <= nt; ++t) offsets[t] = 0;
    int64_t *fill = ids ? (int64_t *)malloc(sizeof(int64_t) * (nt > 0 ? nt : 1)) : NULL;
    for (int pass = 0; pass < (ids ? 2 : 1); ++pass) {
        if (pass == 1) {
            for (int64_t t = 0; t < nt; ++t) offsets[t + 1] += offsets[t];
            for (int64_t t = 0; t < nt; ++t) fill[t] = offsets[t];
        }
        for (int64_t i = 0; i < n; ++i) {
            if (!visible[i]) continue;
            double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
            double tau = 2.0 * log(255.0 * opacity[i]);
            double tm = tau * (1.0 + tau_rel) + tau_abs;
            for (int ty = rect[4 * i + 1]; ty < rect[4 * i + 3]; ++ty)
                for (int tx = rect[4 * i]; tx < rect[4 * i + 2]; ++tx) {
                    double px0 = TILE * tx, px1 = TILE * tx + TILE - 1;
                    double py0 = TILE * ty, py1 = TILE * ty + TILE - 1;
                    if (clip) {
                        if (px1 > W - 1) px1 = W - 1;
                        if (py1 > H - 1) py1 = H - 1;
                    }
                    double qm = oracle_rect_min_q(a, b, c, px0 - pad - means2d[2 * i], px1 + pad - means2d[2 * i],
                                                  py0 - pad - means2d[2 * i + 1], py1 + pad - means2d[2 * i + 1]);
                    if (!(qm <= tm)) continue;
                    int64_t t = (int64_t)ty * tiles_x + tx;
                    if (pass == 0) offsets[t + 1]++;
                    else ids[fill[t]++] = (int32_t)i;
                }
        }
    }
    if (!ids) {
        int64_t p = 0;
        for (int64_t t = 0; t < nt; ++t) p += offsets[t + 1];
        return p;
    }
    free(fill);
    int64_t maxlen = 0;
    for (int64_t t = 0; t < nt; ++t) if (offsets[t + 1] - offsets[t] > maxlen) maxlen = offsets[t + 1] - offsets[t];
    dkey *buf = (dkey *)malloc(sizeof(dkey) * (maxlen > 0 ? maxlen : 1));
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a0 = offsets[t], b0 = offsets[t + 1];
        for (int64_t k = a0; k < b0; ++k) { buf[k - a0].d = depth[ids[k]]; buf[k - a0].id = ids[k]; }
        qsort(buf, (size_t)(b0 - a0), sizeof(dkey), cmp_dkey);
        for (int64_t k = a0; k < b0; ++k) ids[k] = buf[k - a0].id;
    }
    free(buf);
    return offsets[nt];
}

/* ------------------------------------------------------------------------ */
/* per-pixel blending (Alg. 1, baseline column)                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *mean, *conic, *opac, *rgb;
    double bg[3];
} splats_t;

/* quadratic form of the conic at displacement d = pixel - mean */
static double conic_q(const double *K, double dx, double dy)
{
    return K[0] * dx * dx + 2.0 * K[1] * dx * dy + K[2] * dy * dy;
}

/*
 * Blend one pixel over `list` (ids in front-to-back order).  Writes colour,
 * final T, the 1-based list position and the id of the last blended
 * Gaussian (0 / -1 if none), the number blended, the smallest decision
 * margin in log space over all alpha-floor and termination tests (the
 * forward's only discrete decisions), and the smallest log-space distance of
 * a blended Gaussian's unclamped alpha from the 0.99 clamp (where only the
 * derivative switches).
 */
static void blend_pixel(const splats_t *S, const int32_t *list, int64_t len, double px, double py,
                        double *C, double *Tout, int32_t *last_pos, int32_t *last_id, int32_t *count,
                        double *margin, double *cmargin)
{
    double T = 1.0, acc[3] = { 0, 0, 0 }, mmin = INFINITY, cmin = INFINITY;
    int32_t lp = 0, lid = -1, cnt = 0;
    for (int64_t k = 0; k < len; ++k) {
        int32_t g = list[k];
        const double *K = S->conic + 3 * g;
        double dx = px - S->mean[2 * g], dy = py - S->mean[2 * g + 1];
        double q = conic_q(K, dx, dy);
        double a_raw = S->opac[g] * exp(-0.5 * q);
        double la = log(S->opac[g]) - 0.5 * q;           /* ln of the unclamped alpha */
        double m1 = fabs(la - log(ALPHA_MIN));
        if (m1 < mmin) mmin = m1;
        double alpha = a_raw < ALPHA_MAX ? a_raw : ALPHA_MAX;
        if (alpha < ALPHA_MIN) continue;
        /* min(0.99, .) is continuous, so the clamp decides nothing in the
           forward; only the derivative switches there (gradient tests) */
        double m3 = fabs(la - log(ALPHA_MAX));
        if (m3 < cmin) cmin = m3;
        double test = T * (1.0 - alpha);
        double m2 = fabs(log(test) - log(T_MIN));
        if (m2 < mmin) mmin = m2;
        if (test < T_MIN) break;
        for (int c = 0; c < 3; ++c) acc[c] += S->rgb[3 * g + c] * alpha * T;
        T = test;
        lp = (int32_t)(k + 1); lid = g; cnt++;
    }
    for (int c = 0; c < 3; ++c) C[c] = acc[c] + T * S->bg[c];
    *Tout = T; *last_pos = lp; *last_id = lid; *count = cnt; *margin = mmin;
    if (cmargin) *cmargin = cmin;
}

/*
 * Alternatives of one pixel's blend (reading of the several-correct-results
 * remark, Sec. IV-B): every decision of the blend (the 1/255 floor of a
 * Gaussian, the 1e-4 stop) whose log-space margin is below `guard` may go
 * either way under rounding, so the blend is explored along both outcomes of
 * each such decision, depth first, front to back.  Writes up to max_alts
 * outcomes (colour + T bg, final T, id of the last blended Gaussian or -1) and
 * returns their number, or -1 if there were more (then the first max_alts).
 */
typedef struct {
    const splats_t *S;
    const int32_t *list;
    int64_t len;
    double px, py, guard;
    int max_alts, n;
    double *img, *T;
    int32_t *lid;
    int overflow;
} alt_ctx;

static void alt_explore(alt_ctx *c, int64_t k0, double T, double a0, double a1, double a2, int32_t lid)
{
    if (c->overflow) return;
    const splats_t *S = c->S;
    for (int64_t k = k0; k < c->len; ++k) {
        int32_t g = c->list[k];
        const double *K = S->conic + 3 * g;
        double dx = c->px - S->mean[2 * g], dy = c->py - S->mean[2 * g + 1];
        double q = conic_q(K, dx, dy);
        double a_raw = S->opac[g] * exp(-0.5 * q);
        double la = log(S->opac[g]) - 0.5 * q;
        double alpha = a_raw < ALPHA_MAX ? a_raw : ALPHA_MAX;
        int keep = !(alpha < ALPHA_MIN);
        if (fabs(la - log(ALPHA_MIN)) < c->guard) {
            /* the other outcome of the floor, explored first */
            if (keep) {
                alt_explore(c, k + 1, T, a0, a1, a2, lid);
            } else {
                double test = T * (1.0 - alpha);
                if (!(test < T_MIN))
                    alt_explore(c, k + 1, test, a0 + S->rgb[3 * g] * alpha * T, a1 + S->rgb[3 * g + 1] * alpha * T,
                                a2 + S->rgb[3 * g + 2] * alpha * T, g);
            }
            if (c->overflow) return;
        }
        if (!keep) continue;
        double test = T * (1.0 - alpha);
        int stop = test < T_MIN;
        if (T > 0.0 && fabs(log(test) - log(T_MIN)) < c->guard) {
            if (stop) {
                alt_explore(c, k + 1, test, a0 + S->rgb[3 * g] * alpha * T, a1 + S->rgb[3 * g + 1] * alpha * T,
                            a2 + S->rgb[3 * g + 2] * alpha * T, g);
            } else {
                /* stopping here instead */
                if (c->n >= c->max_alts) { c->overflow = 1; return; }
                c->img[3 * c->n] = a0 + T * S->bg[0];
                c->img[3 * c->n + 1] = a1 + T * S->bg[1];
                c->img[3 * c->n + 2] = a2 + T * S->bg[2];
                c->T[c->n] = T;
                c->lid[c->n] = lid;
                c->n++;
            }
            if (c->overflow) return;
        }
        if (stop) break;
        a0 += S->rgb[3 * g] * alpha * T;
        a1 += S->rgb[3 * g + 1] * alpha * T;
        a2 += S->rgb[3 * g + 2] * alpha * T;
        T = test;
        lid = g;
    }
    if (c->n >= c->max_alts) { c->overflow = 1; return; }
    c->img[3 * c->n] = a0 + T * S->bg[0];
    c->img[3 * c->n + 1] = a1 + T * S->bg[1];
    c->img[3 * c->n + 2] = a2 + T * S->bg[2];
    c->T[c->n] = T;
    c->lid[c->n] = lid;
    c->n++;
}

int oracle_blend_alternatives(int W, int H, const int64_t *offsets, const int32_t *ids, const double *means2d,
                              const double *conic, const double *opacity, const double *rgb, const double *bg,
                              int x, int y, double guard, int max_alts, double *img, double *T, int32_t *last_id)
{
    splats_t S = { means2d, conic, opacity, rgb, { bg[0], bg[1], bg[2] } };
    int tiles_x = (W + TILE - 1) / TILE;
    int64_t t = (int64_t)(y / TILE) * tiles_x + x / TILE;
    (void)H;
    alt_ctx c = { &S, ids + offsets[t], offsets[t + 1] - offsets[t], (double)x, (double)y, guard, max_alts, 0,
                  img, T, last_id, 0 };
    alt_explore(&c, 0, 1.0, 0.0, 0.0, 0.0, -1);
    return c.overflow ? -1 : c.n;
}

/*
 * oracle_render_untiled: the plain definition -- every pixel blends every
 * visible Gaussian in ascending (depth, id) order.  Outputs image [3,H,W],
 * T [H,W], last contributing id [H,W], contributor count [H,W], decision
 * margin [H,W] and clamp margin [H,W] (NULL: not written).
 */
void oracle_render_untiled(int W, int H, int64_t n, const int32_t *visible, const float *depth,
                           const double *means2d, const double *conic, const double *opacity,
                           const double *rgb, const double *bg, double *image, double *T_out,
                           int32_t *last_id, int32_t *count, double *margin, double *cmargin)
{
    splats_t S = { means2d, conic, opacity, rgb, { bg[0], bg[1], bg[2] } };
    dkey *order = (dkey *)malloc(sizeof(dkey) * (n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) if (visible[i]) { order[m].d = depth[i]; order[m].id = (int32_t)i; m++; }
    qsort(order, (size_t)m, sizeof(dkey), cmp_dkey);
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (m > 0 ? m : 1));
    for (int64_t k = 0; k < m; ++k) list[k] = order[k].id;
    free(order);
    int64_t HW = (int64_t)W * H;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            double C[3]; int32_t lp;
            blend_pixel(&S, list, m, x, y, C, &T_out[p], &lp, &last_id[p], &count[p], &margin[p],
                        cmargin ? &cmargin[p] : NULL);
            for (int c = 0; c < 3; ++c) image[c * HW + p] = C[c];
        }
    free(list);
}

/*
 * oracle_render_tiled: the same blend, each pixel over its tile's list
 * (offsets/ids from oracle_tile_lists).  If pix (length npix, pairs of
 * x, y) is non-NULL only those pixels are rendered and outputs are
 * per-sample [3,npix] / [npix]; otherwise the full image.  last_pos is the
 * 1-based position in the tile list of the last blended Gaussian.
 */
void oracle_render_tiled(int W, int H, const int64_t *offsets, const int32_t *ids,
                         const double *means2d, const double *conic, const double *opacity,
                         const double *rgb, const double *bg, const int32_t *pix, int64_t npix,
                         double *image, double *T_out, int32_t *last_pos, int32_t *last_id,
                         int32_t *count, double *margin, double *cmargin)
{
    splats_t S = { means2d, conic, opacity, rgb, { bg[0], bg[1], bg[2] } };
    int tiles_x = (W + TILE - 1) / TILE;
    int64_t total = pix ? npix : (int64_t)W * H;
    for (int64_t s = 0; s < total; ++s) {
        int x = pix ? pix[2 * s] : (int)(s % W);
        int y = pix ? pix[2 * s + 1] : (int)(s / W);
        int64_t t = (int64_t)(y / TILE) * tiles_x + x / TILE;
        double C[3];
        blend_pixel(&S, ids + offsets[t], offsets[t + 1] - offsets[t], x, y, C, &T_out[s], &last_pos[s],
                    &last_id[s], &count[s], &margin[s], cmargin ? &cmargin[s] : NULL);
        for (int c = 0; c < 3; ++c) image[c * total + s] = C[c];
    }
}

/*
 * oracle_render_backward: gradients of L = sum(gC * C) + sum(gT * T_final)
 * with respect to each Gaussian's projected mean, conic (a, b, c), opacity and
 * colour, accumulated over all pixels (tile lists as in oracle_render_tiled).
 *
 * For pixel p with contributors k = 1..m (alpha_k, T_k = prod_{j<k}(1-alpha_j)):
 *   C = sum_k c_k alpha_k T_k + T_m+1 bg
 *   dC/dc_k     = alpha_k T_k
 *   dC/dalpha_k = c_k T_k - (sum_{i>k} c_i alpha_i T_i + T_final bg) / (1 - alpha_k)
 *   dT_final/dalpha_k = -T_final / (1 - alpha_k)
 * and where alpha_k = o_k exp(-q_k/2) is not clamped at 0.99:
 *   dalpha/do = exp(-q/2), dalpha/dq = -alpha/2,
 *   dq/dmean = -2 K d, dq/da = dx^2, dq/db = 2 dx dy, dq/dc = dy^2.
 * Decisions (alpha floor, termination, clamp) are held fixed.
 */
void oracle_render_backward(int W, int H, const int64_t *offsets, const int32_t *ids, int64_t n,
                            const double *means2d, const double *conic, const double *opacity,
                            const double *rgb, const double *bg, const double *gC /*[3,H,W]*/,
                            const double *gT /*[H,W] or NULL*/, double *g_means2d, double *g_conic,
                            double *g_opacity, double *g_rgb)
{
    memset(g_means2d, 0, sizeof(double) * 2 * n);
    memset(g_conic, 0, sizeof(double) * 3 * n);
    memset(g_opacity, 0, sizeof(double) * n);
    memset(g_rgb, 0, sizeof(double) * 3 * n);
    int tiles_x = (W + TILE - 1) / TILE;
    int64_t HW = (int64_t)W * H;
    int64_t maxlen = 0, nt = (int64_t)tiles_x * ((H + TILE - 1) / TILE);
    for (int64_t t = 0; t < nt; ++t) if (offsets[t + 1] - offsets[t] > maxlen) maxlen = offsets[t + 1] - offsets[t];
    int32_t *cid = (int32_t *)malloc(sizeof(int32_t) * (maxlen + 1));
    double *ca = (double *)malloc(sizeof(double) * (maxlen + 1));
    double *cT = (double *)malloc(sizeof(double) * (maxlen + 1));
    double *cq = (double *)malloc(sizeof(double) * (maxlen + 1));
    int *cclamp = (int *)malloc(sizeof(int) * (maxlen + 1));
    double *suffix = (double *)malloc(sizeof(double) * 3 * (maxlen + 2));
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            int64_t t = (int64_t)(y / TILE) * tiles_x + x / TILE;
            const int32_t *list = ids + offsets[t];
            int64_t len = offsets[t + 1] - offsets[t];
            /* forward: collect contributors */
            double T = 1.0;
            int64_t m = 0;
            for (int64_t k = 0; k < len; ++k) {
                int32_t g = list[k];
                double dx = x - means2d[2 * g], dy = y - means2d[2 * g + 1];
                double q = conic_q(conic + 3 * g, dx, dy);
                double a_raw = opacity[g] * exp(-0.5 * q);
                int clamped = !(a_raw < ALPHA_MAX);
                double alpha = clamped ? ALPHA_MAX : a_raw;
                if (alpha < ALPHA_MIN) continue;
                double test = T * (1.0 - alpha);
                if (test < T_MIN) break;
                cid[m] = g; ca[m] = alpha; cT[m] = T; cq[m] = q; cclamp[m] = clamped; m++;
                T = test;
            }
            double Tf = T;
            double g3[3] = { gC[p], gC[HW + p], gC[2 * HW + p] };
            double gt = gT ? gT[p] : 0.0;
            /* suffix sums of c_i alpha_i T_i */
            for (int c = 0; c < 3; ++c) suffix[3 * m + c] = 0.0;
            for (int64_t k = m - 1; k >= 0; --k)
                for (int c = 0; c < 3; ++c)
                    suffix[3 * k + c] = suffix[3 * (k + 1) + c] + rgb[3 * cid[k] + c] * ca[k] * cT[k];
            for (int64_t k = 0; k < m; ++k) {
                int32_t g = cid[k];
                double dLda = 0.0;
                for (int c = 0; c < 3; ++c) {
                    g_rgb[3 * g + c] += g3[c] * ca[k] * cT[k];
                    double dCda = rgb[3 * g + c] * cT[k] - (suffix[3 * (k + 1) + c] + Tf * bg[c]) / (1.0 - ca[k]);
                    dLda += g3[c] * dCda;
                }
                dLda += gt * (-Tf / (1.0 - ca[k]));
                if (cclamp[k]) continue;
                double G = exp(-0.5 * cq[k]);
                g_opacity[g] += dLda * G;
                double dLdq = dLda * (-0.5 * ca[k]);
                double dx = x - means2d[2 * g], dy = y - means2d[2 * g + 1];
                const double *K = conic + 3 * g;
                g_means2d[2 * g] += dLdq * (-2.0) * (K[0] * dx + K[1] * dy);
                g_means2d[2 * g + 1] += dLdq * (-2.0) * (K[1] * dx + K[2] * dy);
                g_conic[3 * g] += dLdq * dx * dx;
                g_conic[3 * g + 1] += dLdq * 2.0 * dx * dy;
                g_conic[3 * g + 2] += dLdq * dy * dy;
            }
        }
    free(cid); free(ca); free(cT); free(cq); free(cclamp); free(suffix);
}

/*
 * oracle_footprint: tile rectangle of splats given directly in screen space
 * (mean, conic, opacity), with the same footprint rule as oracle_project:
 * pixel centres of the ellipse q <= tau = 2 ln(255 o), clipped to the image.
 */
void oracle_footprint(int W, int H, int64_t n, const double *means2d, const double *conic, const double *opacity,
                      int32_t *visible, int32_t *rect)
{
    for (int64_t i = 0; i < n; ++i) {
        visible[i] = 0;
        for (int c = 0; c < 4; ++c) rect[4 * i + c] = 0;
        double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
        double det = a * c - b * b;
        double tau = 2.0 * log(255.0 * opacity[i]);
        if (!(det > 0.0) || !(tau > 0.0) || !(a > 0.0)) continue;
        double sxx = c / det, syy = a / det;            /* covariance = inverse of the conic */
        double tau_m = tau * (1.0 + FOOT_REL) + FOOT_ABS;
        double rx = sqrt(tau_m * sxx) + FOOT_PX, ry = sqrt(tau_m * syy) + FOOT_PX;
        double x0 = ceil(means2d[2 * i] - rx), x1 = floor(means2d[2 * i] + rx);
        double y0 = ceil(means2d[2 * i + 1] - ry), y1 = floor(means2d[2 * i + 1] + ry);
        if (!(isfinite(x0) && isfinite(x1) && isfinite(y0) && isfinite(y1))) continue;
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > W - 1) x1 = W - 1;
        if (y1 > H - 1) y1 = H - 1;
        if (x0 > x1 || y0 > y1) continue;
        rect[4 * i] = (int)x0 / TILE; rect[4 * i + 1] = (int)y0 / TILE;
        rect[4 * i + 2] = (int)x1 / TILE + 1; rect[4 * i + 3] = (int)y1 / TILE + 1;
        visible[i] = 1;
    }
}
