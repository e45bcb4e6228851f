/*
 * gvo_raster.c -- FP64 reference ("oracle") for 3D Gaussian splatting image
 * formation and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP kernels.
 *
 * What it computes (paper Sec. 3.1: the footprints of Gaussians with mean mu,
 * covariance Sigma = (RS)(RS)^T, colour c and opacity o are splatted onto the
 * image plane, and the parameters are fitted by comparing the images with the
 * video; the rasterizer itself is the one of 3D Gaussian Splatting, which the
 * paper cites).  The plain,
 * tile-free definition is written out, per pixel, with no binning:
 *
 *   1. Time evaluation (Sec. 3.2, Eq. 2-3).  Either
 *      mu(t) = mu0 + a1 t + a2 t^2 + a3 t^3 when cubic coefficients are given
 *      (the polynomial motion basis of Fig. 3 / Tab. 2), or, when M control
 *      points P_0..P_{M-1} are given, the clamped cubic B-spline
 *      mu(t) = sum_i N_{i,3}(t) P_i of Eq. 2 (knots: four at 0, four at 1,
 *      the M-4 interior ones evenly spaced; N_{i,p} by the Cox-de Boor
 *      recursion).  Log-scales and quaternions may be cubic polynomials in t
 *      (Eq. 3): l(t) = l0 + b1 t + b2 t^2 + b3 t^3, q(t) likewise before
 *      normalisation.
 *   2. s = exp(log_scale), qhat = q/|q|, R = R(qhat) (w first),
 *      o = 1/(1+exp(-eta)), Sigma = R diag(s)^2 R^T          (Sec. 3.1)
 *      colour: the stored RGB plus, with spherical-harmonics coefficients of
 *      degree D (1..3, Sec. 3.1), sum over 1 <= l <= D, -l <= m <= l of
 *      k_lm Y_lm(d), d the unit vector from the camera centre to the mean
 *      (the RGB term plays the part of the l = 0 function).
 *   3. camera: world->camera rotation Rc = R(qc/|qc|), translation tc;
 *      m = Rc mu + tc; the Gaussian is dropped if m_z <= near_plane.
 *   4. (u,v) = (fx m_x/m_z + cx, fy m_y/m_z + cy);  J = d(u,v)/dm;
 *      Sigma' = J Rc Sigma Rc^T J^T + dilation * I2  (EWA local affine
 *      approximation of the perspective map, plus a low-pass term);
 *      dropped if det(Sigma') <= 0;  A = Sigma'^{-1} (the conic).
 *   5. order = ascending (fp32 rounding of m_z, Gaussian index).
 *   6. per pixel centre p = (x + 1/2, y + 1/2): T = 1, C = 0; for each
 *      Gaussian in order: d = p - (u,v); q = d^T A d; skip if q > 9;
 *      alpha = min(0.99, o exp(-q/2)); skip if alpha < 1/255;
 *      stop (without blending it) if T (1 - alpha) < 1e-4;
 *      C += c alpha T; T *= 1 - alpha.   Finally C += T * bg.
 *
 * Adjoint: given dL/dC at some pixels, the contributor list of each pixel is
 * walked back to front with the stored transmittances (no division), then
 * the chain rule is taken through step 4..1 in closed matrix form.  Skip and
 * stop decisions and the alpha clamp are piecewise constants (their
 * derivative is zero).  Gradients are with respect to the stored parameters:
 * means (or mu0 and a1..a3, or the control points), log-scales (and b1..b3),
 * unnormalised quaternions (and r1..r3), opacity logits, colours (and SH
 * coefficients), the 7-vector pose (qc unnormalised, tc) and the intrinsics
 * (fx, fy, cx, cy).
 *
 * Per pixel the oracle also reports how close each discrete decision came to
 * its threshold (relative margins), so that comparisons against an FP32
 * implementation can set aside pixels whose outcome is decided by rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n;
    const double *means;          /* [3][n] (mu0 when cubic; unused with control points) */
    const double *log_scales;     /* [3][n] */
    const double *quats;          /* [4][n] w,x,y,z */
    const double *opacity_logits; /* [n] */
    const double *colors;         /* [3][n] */
    const double *mean_coeffs;    /* NULL or [3 coeff][3 xyz][n] */
    int32_t width, height;
    double fx, fy, cx, cy, near_plane, dilation;
    double bg[3];
    double pose[7];               /* world->camera qw qx qy qz tx ty tz */
    double t;                     /* frame time in [0, 1] */
    int32_t n_ctrl;               /* M >= 4 control points of the B-spline mean, or 0 */
    const double *ctrl;           /* NULL or [M][3][n] */
    const double *scale_coeffs;   /* NULL or [3 coeff][3][n]: b1..b3 of the log-scales */
    const double *quat_coeffs;    /* NULL or [3 coeff][4][n]: r1..r3 of the quaternion */
    int32_t sh_degree;            /* 0 (RGB only) .. 3 */
    const double *sh;             /* NULL or [(D+1)^2 - 1][3][n]: k_lm for l >= 1, (l, m) ascending */
} gvo_frame;

typedef struct {
    double *means, *log_scales, *quats, *opacity_logits, *colors, *mean_coeffs, *pose;
    double *ctrl, *scale_coeffs, *quat_coeffs, *sh;
    double *intrinsics;           /* NULL or [4]: fx, fy, cx, cy (shared by all frames, Sec. 3.4) */
} gvo_grads;

typedef struct {
    int valid;
    double mu[3], s[3], qhat[4], qnorm;
    double R[3][3], M[3][3], Sigma[3][3];
    double m[3], J[2][3], T[2][3];
    double cov[2][2], A[2][2];
    double u, v, o;
    float key;
    double col[3];                /* colour seen from this frame's camera */
    double dir[3], vnorm;         /* unit direction camera centre -> mean, and the distance */
    double Y[15];                 /* real SH basis at dir, l = 1..3 */
} proj_t;

typedef struct {
    double Rc[3][3], qc_hat[4], qc_norm, tc[3];
    double C[3];                  /* camera centre in the world, -Rc^T tc */
} cam_t;

/* ------------------------------------------------------------------ */
/* small dense helpers                                                 */
/* ------------------------------------------------------------------ */

/* Rotation matrix of a unit quaternion (w, x, y, z). */
static void quat_to_rot(const double q[4], double R[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

/* dR/dq_k of the map above, for k = w, x, y, z. */
static void quat_to_rot_partials(const double q[4], double D[4][3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    memset(D, 0, sizeof(double) * 36);
    /* d/dw */
    D[0][0][1] = -2 * z; D[0][0][2] = 2 * y;
    D[0][1][0] = 2 * z;  D[0][1][2] = -2 * x;
    D[0][2][0] = -2 * y; D[0][2][1] = 2 * x;
    /* d/dx */
    D[1][0][1] = 2 * y;  D[1][0][2] = 2 * z;
    D[1][1][0] = 2 * y;  D[1][1][1] = -4 * x; D[1][1][2] = -2 * w;
    D[1][2][0] = 2 * z;  D[1][2][1] = 2 * w;  D[1][2][2] = -4 * x;
    /* d/dy */
    D[2][0][0] = -4 * y; D[2][0][1] = 2 * x;  D[2][0][2] = 2 * w;
    D[2][1][0] = 2 * x;  D[2][1][2] = 2 * z;
    D[2][2][0] = -2 * w; D[2][2][1] = 2 * z;  D[2][2][2] = -4 * y;
    /* d/dz */
    D[3][0][0] = -4 * z; D[3][0][1] = -2 * w; D[3][0][2] = 2 * x;
    D[3][1][0] = 2 * w;  D[3][1][1] = -4 * z; D[3][1][2] = 2 * y;
    D[3][2][0] = 2 * x;  D[3][2][1] = 2 * y;
}

/* Gradient of a loss w.r.t. an unnormalised quaternion q, given the gradient
 * dR w.r.t. R(q/|q|). */
static void rot_grad_to_quat(const double qhat[4], double qnorm, const double dR[3][3], double dq[4])
{
    double D[4][3][3], dqh[4], dot = 0.0;
    quat_to_rot_partials(qhat, D);
    for (int k = 0; k < 4; ++k) {
        double acc = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc += D[k][i][j] * dR[i][j];
        dqh[k] = acc;
    }
    for (int k = 0; k < 4; ++k) dot += qhat[k] * dqh[k];
    for (int k = 0; k < 4; ++k) dq[k] = (dqh[k] - qhat[k] * dot) / qnorm;
}

/* Clamped cubic B-spline basis of Eq. 2 on [0, 1] with M >= 4 control
 * points: knot u_j = 0 for j <= 3, 1 for j >= M, (j - 3)/(M - 3) between.
 * Cox-de Boor: N_{j,0}(t) = 1 on [u_j, u_{j+1}) (the last non-empty span is
 * closed at t = 1), N_{j,p} = (t - u_j)/(u_{j+p} - u_j) N_{j,p-1}
 * + (u_{j+p+1} - t)/(u_{j+p+1} - u_{j+1}) N_{j+1,p-1}, a term with a zero
 * denominator being 0.  out[i] = N_{i,3}(t), i < M. */
#define SPLINE_MAX_CTRL 64
static double knot(int j, int M)
{
    if (j <= 3) return 0.0;
    if (j >= M) return 1.0;
    return (double)(j - 3) / (double)(M - 3);
}

int gvo_bspline_basis(int32_t M, double t, double *out)
{
    if (M < 4 || M > SPLINE_MAX_CTRL || !(t >= 0.0 && t <= 1.0)) return -1;
    double N[SPLINE_MAX_CTRL + 3];
    const int nk = M + 4;
    for (int j = 0; j < nk - 1; ++j) {
        double a = knot(j, M), b = knot(j + 1, M);
        N[j] = (a <= t && t < b) ? 1.0 : 0.0;
        if (t == 1.0 && j == M - 1) N[j] = 1.0; /* close the last span */
    }
    for (int p = 1; p <= 3; ++p)
        for (int j = 0; j < nk - 1 - p; ++j) {
            double v = 0.0;
            double d1 = knot(j + p, M) - knot(j, M);
            double d2 = knot(j + p + 1, M) - knot(j + 1, M);
            if (d1 > 0.0) v += (t - knot(j, M)) / d1 * N[j];
            if (d2 > 0.0) v += (knot(j + p + 1, M) - t) / d2 * N[j + 1];
            N[j] = v;
        }
    for (int i = 0; i < M; ++i) out[i] = N[i];
    return 0;
}

/* Real spherical harmonics Y_lm, 1 <= l <= 3, at the unit vector (x, y, z),
 * out[l*l + l + m - 1]: the l-th degree harmonic polynomials with the
 * orthonormal normalisation sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times
 * sqrt 2 for m != 0) and the Condon-Shortley sign (-1)^m for m > 0, which the
 * real forms carry as a sign on the odd-m terms.  grad (optional) receives
 * the partial derivatives of each polynomial w.r.t. x, y, z. */
int gvo_sh_basis(int32_t degree, const double d[3], double *out, double *grad)
{
    if (degree < 0 || degree > 3) return -1;
    const double x = d[0], y = d[1], z = d[2];
    const double pi = 3.14159265358979323846;
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = sqrt(15.0 / (4.0 * pi)), c2b = sqrt(5.0 / (16.0 * pi)), c2c = sqrt(15.0 / (16.0 * pi));
    const double c3a = -sqrt(35.0 / (32.0 * pi)), c3b = sqrt(105.0 / (4.0 * pi));
    const double c3c = -sqrt(21.0 / (32.0 * pi)), c3d = sqrt(7.0 / (16.0 * pi));
    const double c3e = sqrt(105.0 / (16.0 * pi));
    double Y[15], G[15][3];
    /* l = 1 */
    Y[0] = -c1 * y;                    G[0][0] = 0;        G[0][1] = -c1;      G[0][2] = 0;
    Y[1] = c1 * z;                     G[1][0] = 0;        G[1][1] = 0;        G[1][2] = c1;
    Y[2] = -c1 * x;                    G[2][0] = -c1;      G[2][1] = 0;        G[2][2] = 0;
    /* l = 2 */
    Y[3] = c2a * x * y;                G[3][0] = c2a * y;  G[3][1] = c2a * x;  G[3][2] = 0;
    Y[4] = -c2a * y * z;               G[4][0] = 0;        G[4][1] = -c2a * z; G[4][2] = -c2a * y;
    Y[5] = c2b * (2 * z * z - x * x - y * y);
    G[5][0] = -2 * c2b * x;  G[5][1] = -2 * c2b * y;  G[5][2] = 4 * c2b * z;
    Y[6] = -c2a * x * z;               G[6][0] = -c2a * z; G[6][1] = 0;        G[6][2] = -c2a * x;
    Y[7] = c2c * (x * x - y * y);      G[7][0] = 2 * c2c * x; G[7][1] = -2 * c2c * y; G[7][2] = 0;
    /* l = 3 */
    Y[8] = c3a * y * (3 * x * x - y * y);
    G[8][0] = c3a * 6 * x * y;  G[8][1] = c3a * (3 * x * x - 3 * y * y);  G[8][2] = 0;
    Y[9] = c3b * x * y * z;
    G[9][0] = c3b * y * z;  G[9][1] = c3b * x * z;  G[9][2] = c3b * x * y;
    Y[10] = c3c * y * (4 * z * z - x * x - y * y);
    G[10][0] = c3c * (-2 * x * y);  G[10][1] = c3c * (4 * z * z - x * x - 3 * y * y);  G[10][2] = c3c * 8 * y * z;
    Y[11] = c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
    G[11][0] = c3d * (-6 * x * z);  G[11][1] = c3d * (-6 * y * z);  G[11][2] = c3d * (6 * z * z - 3 * x * x - 3 * y * y);
    Y[12] = c3c * x * (4 * z * z - x * x - y * y);
    G[12][0] = c3c * (4 * z * z - 3 * x * x - y * y);  G[12][1] = c3c * (-2 * x * y);  G[12][2] = c3c * 8 * x * z;
    Y[13] = c3e * z * (x * x - y * y);
    G[13][0] = c3e * 2 * x * z;  G[13][1] = c3e * (-2 * y * z);  G[13][2] = c3e * (x * x - y * y);
    Y[14] = c3a * x * (x * x - 3 * y * y);
    G[14][0] = c3a * (3 * x * x - 3 * y * y);  G[14][1] = c3a * (-6 * x * y);  G[14][2] = 0;
    const int nb = (degree + 1) * (degree + 1) - 1;
    for (int k = 0; k < nb; ++k) {
        out[k] = Y[k];
        if (grad)
            for (int j = 0; j < 3; ++j) grad[k * 3 + j] = G[k][j];
    }
    return 0;
}

static int all_finite(const double *v, int k)
{
    for (int i = 0; i < k; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static void setup_camera(const gvo_frame *fr, cam_t *c, int *ok)
{
    double qn = sqrt(fr->pose[0] * fr->pose[0] + fr->pose[1] * fr->pose[1] +
                     fr->pose[2] * fr->pose[2] + fr->pose[3] * fr->pose[3]);
    *ok = (qn > 0.0 && isfinite(qn) && all_finite(fr->pose, 7));
    if (!*ok) return;
    c->qc_norm = qn;
    for (int k = 0; k < 4; ++k) c->qc_hat[k] = fr->pose[k] / qn;
    quat_to_rot(c->qc_hat, c->Rc);
    for (int k = 0; k < 3; ++k) c->tc[k] = fr->pose[4 + k];
    for (int i = 0; i < 3; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 3; ++j) acc -= c->Rc[j][i] * c->tc[j];
        c->C[i] = acc;
    }
}

/* Steps 1-4 for Gaussian g. */
static void project_one(const gvo_frame *fr, const cam_t *c, int64_t g, proj_t *P)
{
    const int64_t n = fr->n;
    const double t = fr->t;
    double raw[14];
    memset(P, 0, sizeof(*P));
    for (int k = 0; k < 3; ++k) raw[k] = fr->n_ctrl > 0 ? 0.0 : fr->means[k * n + g];
    for (int k = 0; k < 3; ++k) raw[3 + k] = fr->log_scales[k * n + g];
    for (int k = 0; k < 4; ++k) raw[6 + k] = fr->quats[k * n + g];
    raw[10] = fr->opacity_logits[g];
    for (int k = 0; k < 3; ++k) raw[11 + k] = fr->colors[k * n + g];
    if (!all_finite(raw, 14)) return;

    /* 1. time evaluation: mean, log-scales and quaternion at t */
    if (fr->n_ctrl > 0) {
        double B[SPLINE_MAX_CTRL];
        if (gvo_bspline_basis(fr->n_ctrl, t, B)) return;
        /* local support: a control point with zero weight at t takes no part
         * (not even through a non-finite value) */
        for (int k = 0; k < 3; ++k) {
            double mu = 0.0;
            for (int i = 0; i < fr->n_ctrl; ++i) {
                if (B[i] == 0.0) continue;
                double c = fr->ctrl[((int64_t)i * 3 + k) * n + g];
                if (!isfinite(c)) return;
                mu += B[i] * c;
            }
            P->mu[k] = mu;
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            double mu = raw[k];
            if (fr->mean_coeffs) {
                double a1 = fr->mean_coeffs[(0 * 3 + k) * n + g];
                double a2 = fr->mean_coeffs[(1 * 3 + k) * n + g];
                double a3 = fr->mean_coeffs[(2 * 3 + k) * n + g];
                if (!isfinite(a1) || !isfinite(a2) || !isfinite(a3)) return;
                mu = mu + a1 * t + a2 * t * t + a3 * t * t * t;
            }
            P->mu[k] = mu;
        }
    }
    if (fr->scale_coeffs)
        for (int k = 0; k < 3; ++k) {
            double b1 = fr->scale_coeffs[(0 * 3 + k) * n + g];
            double b2 = fr->scale_coeffs[(1 * 3 + k) * n + g];
            double b3 = fr->scale_coeffs[(2 * 3 + k) * n + g];
            if (!isfinite(b1) || !isfinite(b2) || !isfinite(b3)) return;
            raw[3 + k] = raw[3 + k] + b1 * t + b2 * t * t + b3 * t * t * t;
        }
    if (fr->quat_coeffs)
        for (int k = 0; k < 4; ++k) {
            double r1 = fr->quat_coeffs[(0 * 4 + k) * n + g];
            double r2 = fr->quat_coeffs[(1 * 4 + k) * n + g];
            double r3 = fr->quat_coeffs[(2 * 4 + k) * n + g];
            if (!isfinite(r1) || !isfinite(r2) || !isfinite(r3)) return;
            raw[6 + k] = raw[6 + k] + r1 * t + r2 * t * t + r3 * t * t * t;
        }
    /* colour, view-dependent with SH coefficients */
    for (int ch = 0; ch < 3; ++ch) P->col[ch] = raw[11 + ch];
    if (fr->sh_degree > 0) {
        double v[3], vn = 0.0;
        for (int k = 0; k < 3; ++k) { v[k] = P->mu[k] - c->C[k]; vn += v[k] * v[k]; }
        vn = sqrt(vn);
        if (!(vn > 0.0)) return;
        P->vnorm = vn;
        for (int k = 0; k < 3; ++k) P->dir[k] = v[k] / vn;
        gvo_sh_basis(fr->sh_degree, P->dir, P->Y, NULL);
        const int nb = (fr->sh_degree + 1) * (fr->sh_degree + 1) - 1;
        for (int ch = 0; ch < 3; ++ch) {
            double acc = P->col[ch];
            for (int k = 0; k < nb; ++k) {
                double kc = fr->sh[((int64_t)k * 3 + ch) * n + g];
                if (!isfinite(kc)) return;
                acc += P->Y[k] * kc;
            }
            P->col[ch] = acc;
        }
    }
    /* 2. activations and world covariance */
    P->qnorm = sqrt(raw[6] * raw[6] + raw[7] * raw[7] + raw[8] * raw[8] + raw[9] * raw[9]);
    if (!(P->qnorm > 0.0)) return;
    for (int k = 0; k < 4; ++k) P->qhat[k] = raw[6 + k] / P->qnorm;
    for (int k = 0; k < 3; ++k) P->s[k] = exp(raw[3 + k]);
    P->o = 1.0 / (1.0 + exp(-raw[10]));
    quat_to_rot(P->qhat, P->R);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P->M[i][j] = P->R[i][j] * P->s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += P->M[i][k] * P->M[j][k];
            P->Sigma[i][j] = acc;
        }
    /* 3. camera space */
    for (int i = 0; i < 3; ++i) {
        double acc = c->tc[i];
        for (int k = 0; k < 3; ++k) acc += c->Rc[i][k] * P->mu[k];
        P->m[i] = acc;
    }
    if (!(P->m[2] > fr->near_plane)) return;
    /* 4. perspective projection of the mean and EWA covariance */
    double mx = P->m[0], my = P->m[1], mz = P->m[2];
    P->u = fr->fx * mx / mz + fr->cx;
    P->v = fr->fy * my / mz + fr->cy;
    P->J[0][0] = fr->fx / mz; P->J[0][1] = 0.0;        P->J[0][2] = -fr->fx * mx / (mz * mz);
    P->J[1][0] = 0.0;        P->J[1][1] = fr->fy / mz; P->J[1][2] = -fr->fy * my / (mz * mz);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += P->J[i][k] * c->Rc[k][j];
            P->T[i][j] = acc;
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) acc += P->T[i][a] * P->Sigma[a][b] * P->T[j][b];
            P->cov[i][j] = acc + (i == j ? fr->dilation : 0.0);
        }
    double det = P->cov[0][0] * P->cov[1][1] - P->cov[0][1] * P->cov[1][0];
    if (!(det > 0.0) || !isfinite(det)) return;
    P->A[0][0] = P->cov[1][1] / det;
    P->A[0][1] = -P->cov[0][1] / det;
    P->A[1][0] = -P->cov[1][0] / det;
    P->A[1][1] = P->cov[0][0] / det;
    P->key = (float)mz;
    P->valid = 1;
}

/* ------------------------------------------------------------------ */
/* depth order                                                         */
/* ------------------------------------------------------------------ */

static const proj_t *g_sort_proj; /* comparator context (sorting is serial) */

static int cmp_order(const void *a, const void *b)
{
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    float ka = g_sort_proj[ia].key, kb = g_sort_proj[ib].key;
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (ia < ib) ? -1 : (ia > ib);
}

/* ------------------------------------------------------------------ */
/* per-pixel compositing                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t g;
    double alpha, T, G, dx, dy;
    int clamped;
} contrib_t;

typedef struct {
    contrib_t *v;
    int64_t len, cap;
} clist_t;

static int clist_push(clist_t *L, contrib_t c)
{
    if (L->len == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 256;
        contrib_t *nv = (contrib_t *)realloc(L->v, (size_t)nc * sizeof(contrib_t));
        if (!nv) return -1;
        L->v = nv;
        L->cap = nc;
    }
    L->v[L->len++] = c;
    return 0;
}

#define ALPHA_MAX 0.99
#define ALPHA_MIN (1.0 / 255.0)
#define T_MIN 1e-4
#define Q_MAX 9.0

static void upd(double *m, double v) { if (v < *m) *m = v; }

/* Step 6 at one pixel centre.  margins: [0] |q-9|/9 where the cut-off decides,
 * [1] |255 alpha - 1|, [2] |T(1-alpha) - 1e-4|/1e-4, [3] |o G - 0.99|/0.99.
 *
 * Optional stake (when stake_tol != NULL): an upper bound on the blending
 * weight that the pixel's set-aside decisions control, i.e. how much of the
 * composite could change if an implementation with slightly different
 * rounding took one of them the other way.  An entry whose 3-sigma or
 * 1/255 decision lies within stake_tol[0] / stake_tol[1] of its threshold
 * puts its weight alpha T at stake (included or not, it moves the colour by
 * at most alpha T times the colour range).  Those entries also scale the
 * transmittance of every later entry by up to a factor 1 - alpha, so a stop
 * decision within stake_tol[2] plus that accumulated factor puts the whole
 * remaining transmittance T at stake (everything from that entry on is
 * bounded by it), and nothing after it is added. */
static int composite_pixel(const gvo_frame *fr, const proj_t *P, const int64_t *order, int64_t nv,
                           double px, double py, double C[3], double *Tout, int64_t *ncontrib,
                           double margins[4], clist_t *L, const double *stake_tol, double *stake)
{
    double T = 1.0;
    int64_t nc = 0;
    double st = 0.0, slack = 0.0;
    int tail_at_stake = 0;
    C[0] = C[1] = C[2] = 0.0;
    for (int k = 0; k < 4; ++k) margins[k] = INFINITY;
    const double alpha_at_cut_factor = exp(-0.5 * Q_MAX);
    for (int64_t i = 0; i < nv; ++i) {
        int64_t g = order[i];
        const proj_t *p = &P[g];
        double dx = px - p->u, dy = py - p->v;
        double q = p->A[0][0] * dx * dx + (p->A[0][1] + p->A[1][0]) * dx * dy + p->A[1][1] * dy * dy;
        const double mq = fabs(q - Q_MAX) / Q_MAX;
        if (p->o * alpha_at_cut_factor >= ALPHA_MIN) upd(&margins[0], mq);
        if (stake_tol && !tail_at_stake && mq < stake_tol[0] && p->o * alpha_at_cut_factor >= ALPHA_MIN) {
            /* the weight this entry would have just inside the cut */
            double w = p->o * exp(-0.5 * q);
            w = (w < ALPHA_MAX ? w : ALPHA_MAX);
            st += w * T;
            slack += w;
        }
        if (q > Q_MAX) continue;
        double G = exp(-0.5 * q);
        double a = p->o * G;
        double alpha = a < ALPHA_MAX ? a : ALPHA_MAX;
        const double ma = fabs(alpha / ALPHA_MIN - 1.0);
        upd(&margins[1], ma);
        if (stake_tol && !tail_at_stake && ma < stake_tol[1]) {
            st += alpha * T;
            slack += alpha;
        }
        if (alpha < ALPHA_MIN) continue;
        double Tn = T * (1.0 - alpha);
        const double ms = fabs(Tn - T_MIN) / T_MIN;
        upd(&margins[2], ms);
        if (stake_tol && !tail_at_stake && ms < stake_tol[2] + 1.02 * slack) {
            st += T;
            tail_at_stake = 1;
        }
        if (Tn < T_MIN) break;
        upd(&margins[3], fabs(a - ALPHA_MAX) / ALPHA_MAX);
        for (int ch = 0; ch < 3; ++ch) C[ch] += p->col[ch] * alpha * T;
        if (L) {
            contrib_t c = {g, alpha, T, G, dx, dy, a >= ALPHA_MAX};
            if (clist_push(L, c)) return -1;
        }
        T = Tn;
        ++nc;
    }
    for (int ch = 0; ch < 3; ++ch) C[ch] += T * fr->bg[ch];
    *Tout = T;
    *ncontrib = nc;
    if (stake) *stake = st;
    return 0;
}

/* Adjoint of step 6 for one pixel: accumulate dL/d(u, v, A00, A01, A11, o, c)
 * into acc[g*9 + .] (A01 is the single off-diagonal parameter, which enters q
 * twice).  Walks the contributor list back to front; S is the colour
 * composited behind the current entry, starting with T_final * bg. */
static void composite_pixel_adjoint(const gvo_frame *fr, const proj_t *P, const clist_t *L,
                                    double T_final, const double dC[3], double *acc)
{
    double S[3];
    for (int ch = 0; ch < 3; ++ch) S[ch] = T_final * fr->bg[ch];
    for (int64_t k = L->len - 1; k >= 0; --k) {
        const contrib_t *e = &L->v[k];
        const int64_t g = e->g;
        const proj_t *p = &P[g];
        double *d = acc + g * 9;
        double c[3], dalpha = 0.0;
        for (int ch = 0; ch < 3; ++ch) c[ch] = p->col[ch];
        for (int ch = 0; ch < 3; ++ch) {
            d[6 + ch] += e->alpha * e->T * dC[ch];
            dalpha += dC[ch] * (c[ch] * e->T - S[ch] / (1.0 - e->alpha));
        }
        for (int ch = 0; ch < 3; ++ch) S[ch] += c[ch] * e->alpha * e->T;
        if (e->clamped) continue;  /* alpha = 0.99 is constant in o and q */
        /* alpha = o G, G = exp(-q/2) */
        double dq = dalpha * p->o * e->G * (-0.5);
        d[5] += dalpha * e->G;
        /* q = A00 dx^2 + 2 A01 dx dy + A11 dy^2 with d = p - (u, v) */
        d[2] += dq * e->dx * e->dx;
        d[3] += dq * 2.0 * e->dx * e->dy;
        d[4] += dq * e->dy * e->dy;
        d[0] += dq * (-2.0) * (p->A[0][0] * e->dx + p->A[0][1] * e->dy);
        d[1] += dq * (-2.0) * (p->A[1][0] * e->dx + p->A[1][1] * e->dy);
    }
}

/* Adjoint of steps 1-4 for one Gaussian: from d = dL/d(u, v, A00, A01, A11,
 * o, c) to the stored parameters; the pose contribution is added to
 * dRc (3x3) and dtc (3). */
static void project_adjoint(const gvo_frame *fr, const cam_t *c, int64_t g, const proj_t *P,
                            const double d[9], gvo_grads *gr, double dRc[3][3], double dtc[3])
{
    const int64_t n = fr->n;
    /* gradient w.r.t. the symmetric conic matrix: A01 appears at (0,1) and (1,0) */
    double GA[2][2] = {{d[2], 0.5 * d[3]}, {0.5 * d[3], d[4]}};
    /* A = cov^{-1}  =>  dcov = -A GA A */
    double AG[2][2], Gc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) AG[i][j] = P->A[i][0] * GA[0][j] + P->A[i][1] * GA[1][j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) Gc[i][j] = -(AG[i][0] * P->A[0][j] + AG[i][1] * P->A[1][j]);
    /* cov = T Sigma T^T + dil I,  T = J Rc (2x3) */
    double GS[3][3], dT[2][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) acc += P->T[i][a] * Gc[i][j] * P->T[j][b];
            GS[a][b] = acc;
        }
    for (int i = 0; i < 2; ++i)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int j = 0; j < 2; ++j)
                for (int a = 0; a < 3; ++a) acc += Gc[i][j] * P->T[j][a] * P->Sigma[a][b];
            dT[i][b] = 2.0 * acc;
        }
    double dJ[2][3];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int j = 0; j < 3; ++j) acc += dT[i][j] * c->Rc[k][j];
            dJ[i][k] = acc;
        }
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int i = 0; i < 2; ++i) acc += P->J[i][k] * dT[i][j];
            dRc[k][j] += acc;
        }
    /* J(m) and (u, v)(m) */
    double mx = P->m[0], my = P->m[1], mz = P->m[2];
    double fx = fr->fx, fy = fr->fy;
    /* intrinsics: u = fx mx/mz + cx, v = fy my/mz + cy, J00 = fx/mz,
     * J02 = -fx mx/mz^2, J11 = fy/mz, J12 = -fy my/mz^2 */
    if (gr->intrinsics) {
        gr->intrinsics[0] += d[0] * mx / mz + dJ[0][0] / mz - dJ[0][2] * mx / (mz * mz);
        gr->intrinsics[1] += d[1] * my / mz + dJ[1][1] / mz - dJ[1][2] * my / (mz * mz);
        gr->intrinsics[2] += d[0];
        gr->intrinsics[3] += d[1];
    }
    double dm[3];
    dm[0] = dJ[0][2] * (-fx / (mz * mz)) + d[0] * fx / mz;
    dm[1] = dJ[1][2] * (-fy / (mz * mz)) + d[1] * fy / mz;
    dm[2] = dJ[0][0] * (-fx / (mz * mz)) + dJ[0][2] * (2.0 * fx * mx / (mz * mz * mz))
          + dJ[1][1] * (-fy / (mz * mz)) + dJ[1][2] * (2.0 * fy * my / (mz * mz * mz))
          - d[0] * fx * mx / (mz * mz) - d[1] * fy * my / (mz * mz);
    /* m = Rc mu + tc */
    double dmu[3];
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int i = 0; i < 3; ++i) acc += c->Rc[i][k] * dm[i];
        dmu[k] = acc;
        dtc[k] += dm[k];
    }
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) dRc[i][k] += dm[i] * P->mu[k];
    /* Sigma = M M^T, M = R diag(s) */
    double dM[3][3], dR[3][3], ds[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += GS[i][k] * P->M[k][j];
            dM[i][j] = 2.0 * acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            dR[i][j] = dM[i][j] * P->s[j];
            ds[j] += dM[i][j] * P->R[i][j];
        }
    double dq[4];
    rot_grad_to_quat(P->qhat, P->qnorm, dR, dq);
    /* view-dependent colour: d[6..8] is dL/d(colour); the direction
     * v / |v|, v = mu - C, passes a gradient to the mean and, through the
     * camera centre C = -Rc^T tc, to the pose */
    if (fr->sh_degree > 0) {
        const int nb = (fr->sh_degree + 1) * (fr->sh_degree + 1) - 1;
        double Yb[15], Gb[45], ddir[3] = {0, 0, 0};
        gvo_sh_basis(fr->sh_degree, P->dir, Yb, Gb);
        for (int k = 0; k < nb; ++k)
            for (int ch = 0; ch < 3; ++ch) {
                double kc = fr->sh[((int64_t)k * 3 + ch) * n + g];
                if (gr->sh) gr->sh[((int64_t)k * 3 + ch) * n + g] += Yb[k] * d[6 + ch];
                for (int j = 0; j < 3; ++j) ddir[j] += d[6 + ch] * kc * Gb[k * 3 + j];
            }
        double dot = P->dir[0] * ddir[0] + P->dir[1] * ddir[1] + P->dir[2] * ddir[2];
        double dv[3];
        for (int j = 0; j < 3; ++j) dv[j] = (ddir[j] - P->dir[j] * dot) / P->vnorm;
        for (int j = 0; j < 3; ++j) dmu[j] += dv[j];
        /* dL/dC = -dv; C_i = -sum_j Rc[j][i] tc[j] */
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int i = 0; i < 3; ++i) acc += c->Rc[j][i] * dv[i];
            dtc[j] += acc;
            for (int i = 0; i < 3; ++i) dRc[j][i] += c->tc[j] * dv[i];
        }
    }
    /* write (accumulate); the time evaluation of step 1 is linear in every
     * coefficient, so each gets the gradient of its value times its basis
     * function (N_i(t) or t^k) */
    const double t = fr->t;
    double B[SPLINE_MAX_CTRL];
    if (fr->n_ctrl > 0) gvo_bspline_basis(fr->n_ctrl, t, B);
    for (int k = 0; k < 3; ++k) {
        if (fr->n_ctrl > 0) {
            if (gr->ctrl)
                for (int i = 0; i < fr->n_ctrl; ++i) gr->ctrl[((int64_t)i * 3 + k) * n + g] += B[i] * dmu[k];
        } else {
            gr->means[k * n + g] += dmu[k];
        }
        if (gr->mean_coeffs && fr->mean_coeffs) {
            gr->mean_coeffs[(0 * 3 + k) * n + g] += dmu[k] * t;
            gr->mean_coeffs[(1 * 3 + k) * n + g] += dmu[k] * t * t;
            gr->mean_coeffs[(2 * 3 + k) * n + g] += dmu[k] * t * t * t;
        }
        double dl = ds[k] * P->s[k];
        gr->log_scales[k * n + g] += dl;
        if (gr->scale_coeffs && fr->scale_coeffs) {
            gr->scale_coeffs[(0 * 3 + k) * n + g] += dl * t;
            gr->scale_coeffs[(1 * 3 + k) * n + g] += dl * t * t;
            gr->scale_coeffs[(2 * 3 + k) * n + g] += dl * t * t * t;
        }
        gr->colors[k * n + g] += d[6 + k];
    }
    for (int k = 0; k < 4; ++k) {
        gr->quats[k * n + g] += dq[k];
        if (gr->quat_coeffs && fr->quat_coeffs) {
            gr->quat_coeffs[(0 * 4 + k) * n + g] += dq[k] * t;
            gr->quat_coeffs[(1 * 4 + k) * n + g] += dq[k] * t * t;
            gr->quat_coeffs[(2 * 4 + k) * n + g] += dq[k] * t * t * t;
        }
    }
    gr->opacity_logits[g] += d[5] * P->o * (1.0 - P->o);
}

/* ------------------------------------------------------------------ */
/* exported entry points                                               */
/* ------------------------------------------------------------------ */

/* Per-Gaussian projection (steps 1-4).  out: [n][24] with
 * valid, u, v, cov00, cov01, cov11, A00, A01, A11, m_z, key(float),
 * o, Sigma xx xy xz yy yz zz, m_x, m_y, (pad x4). */
int gvo_project(const gvo_frame *fr, double *out)
{
    cam_t c;
    int ok;
    setup_camera(fr, &c, &ok);
    for (int64_t g = 0; g < fr->n; ++g) {
        double *o = out + g * 24;
        memset(o, 0, 24 * sizeof(double));
        if (!ok) continue;
        proj_t P;
        project_one(fr, &c, g, &P);
        if (!P.valid) continue;
        o[0] = 1; o[1] = P.u; o[2] = P.v;
        o[3] = P.cov[0][0]; o[4] = P.cov[0][1]; o[5] = P.cov[1][1];
        o[6] = P.A[0][0]; o[7] = P.A[0][1]; o[8] = P.A[1][1];
        o[9] = P.m[2]; o[10] = (double)P.key; o[11] = P.o;
        o[12] = P.Sigma[0][0]; o[13] = P.Sigma[0][1]; o[14] = P.Sigma[0][2];
        o[15] = P.Sigma[1][1]; o[16] = P.Sigma[1][2]; o[17] = P.Sigma[2][2];
        o[18] = P.m[0]; o[19] = P.m[1];
    }
    return 0;
}

/* Render the listed pixels (linear index y*W + x; pix == NULL means all
 * pixels in raster order) and, if dL_dC is given, accumulate (+=) the
 * gradient of sum_p dL_dC[p] . C[p] into grads.  With stake_tol (3 relative
 * margins) and stake given, stake[i] is the weight at stake in pixel i (see
 * composite_pixel).  Returns 0, or -1 when out of memory, -2 for an invalid
 * pose. */
/* Tiled form: the candidates of a pixel are the Gaussians whose footprint
 * box (half-extents 3 sqrt(Sigma'_00) and 3 sqrt(Sigma'_11), widened by 0.05 %
 * and one hundredth of a pixel) meets the pixel-centre box of its tile,
 * listed in the global depth order.  Every Gaussian that a pixel of the tile
 * reaches (q <= 9) is a candidate, and so is every one whose q lies within
 * 1e-3 of the cut there, so colours, transmittances, contributor counts, the
 * margins below 1e-3, the stakes and the gradients (same pixel loop, same
 * order of accumulation) equal those of the per-pixel definition exactly.
 * Only the cost differs: a pixel visits its tile's list instead of every
 * Gaussian. */
typedef struct {
    int tile, tiles_x, tiles_y;
    int64_t *off;   /* [tiles + 1] list offsets */
    int64_t *ids;   /* concatenated lists, each in the global order */
} tiles_t;

static int build_tiles(const gvo_frame *fr, const proj_t *P, const int64_t *order, int64_t nv, int tile,
                       tiles_t *T)
{
    T->tile = tile;
    T->tiles_x = (fr->width + tile - 1) / tile;
    T->tiles_y = (fr->height + tile - 1) / tile;
    const int64_t nt = (int64_t)T->tiles_x * T->tiles_y;
    T->off = (int64_t *)calloc((size_t)(nt + 1), sizeof(int64_t));
    int64_t *rect = (int64_t *)malloc((size_t)(nv > 0 ? nv : 1) * 4 * sizeof(int64_t));
    if (!T->off || !rect) { free(T->off); free(rect); T->off = NULL; return -1; }
    /* tile range of each candidate: tiles whose centre box [t tile + 1/2,
     * t tile + tile - 1/2] meets [u - hx, u + hx] (clipped to the image) */
    for (int64_t k = 0; k < nv; ++k) {
        const proj_t *p = &P[order[k]];
        const double hx = 3.0 * sqrt(p->cov[0][0]) * 1.0005 + 0.01, hy = 3.0 * sqrt(p->cov[1][1]) * 1.0005 + 0.01;
        /* clamped in double before the conversion (huge footprints) */
        const double d[4] = {fmax(ceil((p->u - hx - (tile - 0.5)) / tile), 0.0),
                             fmin(floor((p->u + hx - 0.5) / tile), T->tiles_x - 1.0),
                             fmax(ceil((p->v - hy - (tile - 0.5)) / tile), 0.0),
                             fmin(floor((p->v + hy - 0.5) / tile), T->tiles_y - 1.0)};
        int64_t r[4] = {0, -1, 0, -1};  /* empty unless both ranges are */
        if (d[0] <= d[1] && d[2] <= d[3])
            for (int j = 0; j < 4; ++j) r[j] = (int64_t)d[j];
        memcpy(rect + 4 * k, r, sizeof(r));
        for (int64_t ty = r[2]; ty <= r[3]; ++ty)
            for (int64_t tx = r[0]; tx <= r[1]; ++tx) T->off[ty * T->tiles_x + tx + 1] += 1;
    }
    for (int64_t t = 0; t < nt; ++t) T->off[t + 1] += T->off[t];
    T->ids = (int64_t *)malloc((size_t)(T->off[nt] > 0 ? T->off[nt] : 1) * sizeof(int64_t));
    int64_t *cur = (int64_t *)malloc((size_t)nt * sizeof(int64_t));
    if (!T->ids || !cur) { free(T->off); free(T->ids); free(cur); free(rect); T->off = NULL; return -1; }
    memcpy(cur, T->off, (size_t)nt * sizeof(int64_t));
    for (int64_t k = 0; k < nv; ++k) {
        const int64_t *r = rect + 4 * k;
        for (int64_t ty = r[2]; ty <= r[3]; ++ty)
            for (int64_t tx = r[0]; tx <= r[1]; ++tx) T->ids[cur[ty * T->tiles_x + tx]++] = order[k];
    }
    free(cur);
    free(rect);
    return 0;
}

static int render_impl(const gvo_frame *fr, int64_t n_pix, const int64_t *pix, double *color,
                       double *T_final, int64_t *n_contrib, double *margins, const double *dL_dC,
                       gvo_grads *grads, int n_threads, const double *stake_tol, double *stake, int tile)
{
    cam_t cam;
    int ok;
    setup_camera(fr, &cam, &ok);
    if (!ok) return -2;
    const int64_t n = fr->n;
    proj_t *P = (proj_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(proj_t));
    int64_t *order = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!P || !order) { free(P); free(order); return -1; }
    int64_t nv = 0;
    for (int64_t g = 0; g < n; ++g) {
        project_one(fr, &cam, g, &P[g]);
        if (P[g].valid) order[nv++] = g;
    }
    g_sort_proj = P;
    qsort(order, (size_t)nv, sizeof(int64_t), cmp_order);
    tiles_t TL = {0, 0, 0, NULL, NULL};
    if (tile > 0 && build_tiles(fr, P, order, nv, tile, &TL)) { free(P); free(order); return -1; }

    const int bwd = (dL_dC != NULL && grads != NULL);
    int nt = 1;
#ifdef _OPENMP
    nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    double *acc = NULL;
    if (bwd) {
        acc = (double *)calloc((size_t)nt * (size_t)(n > 0 ? n : 1) * 9, sizeof(double));
        if (!acc) { free(P); free(order); return -1; }
    }
    int err = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        clist_t L = {0, 0, 0};
        double *my_acc = bwd ? acc + (size_t)tid * (size_t)n * 9 : NULL;
#ifdef _OPENMP
#pragma omp for schedule(static, 8)
#endif
        for (int64_t i = 0; i < n_pix; ++i) {
            int64_t lin = pix ? pix[i] : i;
            int64_t x = lin % fr->width, y = lin / fr->width;
            double mg[4], C[3], T;
            int64_t nc;
            L.len = 0;
            const int64_t *cand = order;
            int64_t ncand = nv;
            if (tile > 0) {
                const int64_t t = (y / tile) * TL.tiles_x + x / tile;
                cand = TL.ids + TL.off[t];
                ncand = TL.off[t + 1] - TL.off[t];
            }
            if (composite_pixel(fr, P, cand, ncand, (double)x + 0.5, (double)y + 0.5, C, &T, &nc, mg,
                                bwd ? &L : NULL, stake ? stake_tol : NULL, stake ? &stake[i] : NULL)) {
                err = -1;
                continue;
            }
            for (int ch = 0; ch < 3; ++ch) color[i * 3 + ch] = C[ch];
            if (T_final) T_final[i] = T;
            if (n_contrib) n_contrib[i] = nc;
            if (margins)
                for (int k = 0; k < 4; ++k) margins[i * 4 + k] = mg[k];
            if (bwd) composite_pixel_adjoint(fr, P, &L, T, dL_dC + i * 3, my_acc);
        }
        free(L.v);
    }
    if (bwd && !err) {
        double dRc[3][3] = {{0}}, dtc[3] = {0, 0, 0};
        for (int64_t g = 0; g < n; ++g) {
            if (!P[g].valid) continue;
            double d[9] = {0};
            int any = 0;
            for (int t = 0; t < nt; ++t)
                for (int k = 0; k < 9; ++k) d[k] += acc[((size_t)t * n + g) * 9 + k];
            for (int k = 0; k < 9; ++k) any |= (d[k] != 0.0);
            if (any) project_adjoint(fr, &cam, g, &P[g], d, grads, dRc, dtc);
        }
        if (grads->pose) {
            double dq[4];
            rot_grad_to_quat(cam.qc_hat, cam.qc_norm, dRc, dq);
            for (int k = 0; k < 4; ++k) grads->pose[k] += dq[k];
            for (int k = 0; k < 3; ++k) grads->pose[4 + k] += dtc[k];
        }
    }
    free(acc);
    free(TL.off);
    free(TL.ids);
    free(P);
    free(order);
    return err;
}

int gvo_render(const gvo_frame *fr, int64_t n_pix, const int64_t *pix, double *color,
               double *T_final, int64_t *n_contrib, double *margins, const double *dL_dC,
               gvo_grads *grads, int n_threads, const double *stake_tol, double *stake)
{
    return render_impl(fr, n_pix, pix, color, T_final, n_contrib, margins, dL_dC, grads, n_threads, stake_tol,
                       stake, 0);
}

/* gvo_render in its tiled form (see build_tiles), tile >= 1 pixels. */
int gvo_render_tiled(const gvo_frame *fr, int64_t n_pix, const int64_t *pix, double *color,
                     double *T_final, int64_t *n_contrib, double *margins, const double *dL_dC,
                     gvo_grads *grads, int n_threads, const double *stake_tol, double *stake, int tile)
{
    if (tile < 1) return -3;
    return render_impl(fr, n_pix, pix, color, T_final, n_contrib, margins, dL_dC, grads, n_threads, stake_tol,
                       stake, tile);
}

/* Flags (0/1) of the Gaussians that contribute to at least one pixel of the
 * frame (alpha >= 1/255 inside the 3-sigma cut, before the pixel stopped):
 * the "appears in this frame" test behind warping unseen Gaussians (Sec. 4.1).
 * Returns 0, -1 when out of memory, -2 for an invalid pose. */
int gvo_contributors(const gvo_frame *fr, uint8_t *flags, int n_threads)
{
    cam_t cam;
    int ok;
    setup_camera(fr, &cam, &ok);
    const int64_t n = fr->n;
    memset(flags, 0, (size_t)(n > 0 ? n : 0));
    if (!ok) return -2;
    proj_t *P = (proj_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(proj_t));
    int64_t *order = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!P || !order) { free(P); free(order); return -1; }
    int64_t nv = 0;
    for (int64_t g = 0; g < n; ++g) {
        project_one(fr, &cam, g, &P[g]);
        if (P[g].valid) order[nv++] = g;
    }
    g_sort_proj = P;
    qsort(order, (size_t)nv, sizeof(int64_t), cmp_order);
    int nt = 1;
#ifdef _OPENMP
    nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    uint8_t *local = (uint8_t *)calloc((size_t)nt * (size_t)(n > 0 ? n : 1), 1);
    int err = local ? 0 : -1;
    const int64_t npix = (int64_t)fr->width * fr->height;
    if (!err) {
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            clist_t L = {0, 0, 0};
            uint8_t *mine = local + (size_t)tid * (size_t)n;
#ifdef _OPENMP
#pragma omp for schedule(static, 8)
#endif
            for (int64_t i = 0; i < npix; ++i) {
                double mg[4], C[3], T;
                int64_t nc;
                L.len = 0;
                if (composite_pixel(fr, P, order, nv, (double)(i % fr->width) + 0.5, (double)(i / fr->width) + 0.5,
                                    C, &T, &nc, mg, &L, NULL, NULL)) {
                    err = -1;
                    continue;
                }
                for (int64_t k = 0; k < L.len; ++k) mine[L.v[k].g] = 1;
            }
            free(L.v);
        }
        for (int t = 0; t < nt; ++t)
            for (int64_t g = 0; g < n; ++g) flags[g] |= local[(size_t)t * (size_t)n + g];
    }
    free(local);
    free(P);
    free(order);
    return err;
}

int gvo_abi_version(void) { return 7; }
