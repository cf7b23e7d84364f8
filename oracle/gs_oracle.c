/*
 * gs_oracle.c -- plain FP64 CPU oracle for the differentiable tile-splatting
 * step of 3D Gaussian Splatting (BalanceGS, arXiv 2510.14564, Sec. II-A).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header,
 * table or constant with the HIP path; the two meet only through the seeded
 * input arrays.  It is deliberately plain: one Gaussian or one pixel at a time,
 * no blocking and no fusion; OpenMP only spreads independent items over cores.
 *
 * What it computes (each function cites the passage it follows):
 *   - the Gaussian kernel G(x) = exp(-1/2 (x-mu)^T Sigma^-1 (x-mu))   (Sec. II-A)
 *   - EWA projection Sigma' = J W Sigma W^T J^T                        (Sec. II-A)
 *   - colour from SH coefficients                                      (Sec. I, Sec. II-A)
 *   - 16x16 pixel tiles sharing one Gaussian list                      (Sec. IV-C.1)
 *   - Gaussians sorted by depth per tile                               (Sec. II-A)
 *   - front-to-back blending C = sum c_i a_i prod_{j<i}(1 - a_j)       (Sec. II-A)
 *   - the exact analytic derivative of all of the above (training).
 * The paper is silent on the parameterisation, the Jacobian's form, the
 * low-pass dilation, the radius rule, the tile rectangle, tie-breaks, the
 * alpha thresholds and the SH basis; the readings used are spelled out next to
 * the code that applies them.
 *
 * Camera array (double[22]):
 *   0 fx, 1 fy, 2 cx, 3 cy, 4 near_z, 5 tan_half_fov_x, 6 tan_half_fov_y,
 *   7..15 R_cw row-major, 16..18 t_cw, 19..21 bg.
 * Record array (double[n][9]): u, v, A, B, C, opacity, r, g, b.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_TILE 16
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_ALPHA_MAX 0.99
#define OR_T_MIN 1e-4
#define OR_DILATION 0.3
#define OR_SLOPE_LIMIT 1.3
#define OR_RADIUS_MAX 4194304.0 /* 2^22 px: larger footprints are culled */

/* ------------------------------------------------------------------ helpers */

static int64_t floor_div(int64_t a, int64_t b) { /* b > 0, rounds toward -inf */
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* d R / d q_k for a quaternion q (no normalisation), row-major 3x3 each. */
static void quat_rot_jac(const double q[4], double dR[4][9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    /* d/dw */
    double a[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    /* d/dx */
    double b[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    /* d/dy */
    double c[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    /* d/dz */
    double d[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    memcpy(dR[0], a, sizeof a); memcpy(dR[1], b, sizeof b);
    memcpy(dR[2], c, sizeof c); memcpy(dR[3], d, sizeof d);
}

/* ------------------------------------------------------------- SH basis ---
 * Real spherical harmonics with the Condon-Shortley phase kept, ordered by l
 * then m = -l..l (reading of "SH coefficients", Sec. I / Sec. II-A):
 *   m = 0 : N_l^0 P_l(z)
 *   m > 0 : sqrt2 N_l^m (-1)^m P_l^(m)(z) Re((x + i y)^m)
 *   m < 0 : sqrt2 N_l^|m| (-1)^|m| P_l^(|m|)(z) Im((x + i y)^|m|)
 * with N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^(k) the k-th
 * derivative of the Legendre polynomial, from Rodrigues' formula
 * P_l = 1/(2^l l!) d^l/dz^l (z^2 - 1)^l.  For a unit direction (x, y, z),
 * (1 - z^2)^(m/2) e^{i m phi} = (x + i y)^m, which gives the polynomial form.
 * Every constant is derived here at run time; none is typed in.
 */
#define OR_MAXL 3
static double g_legendre[OR_MAXL + 1][2 * OR_MAXL + 2]; /* coefficients of P_l in z^k */
static double g_norm[OR_MAXL + 1][OR_MAXL + 1];          /* N_l^m */
static int g_sh_ready = 0;

static double factorial(int k) { double f = 1; for (int i = 2; i <= k; ++i) f *= i; return f; }

static void sh_init(void) {
    if (g_sh_ready) return;
    for (int l = 0; l <= OR_MAXL; ++l) {
        /* (z^2 - 1)^l = sum_j C(l,j) (-1)^(l-j) z^(2j) */
        double poly[2 * OR_MAXL + 2];
        memset(poly, 0, sizeof poly);
        for (int j = 0; j <= l; ++j)
            poly[2 * j] = factorial(l) / (factorial(j) * factorial(l - j)) * (((l - j) & 1) ? -1.0 : 1.0);
        /* differentiate l times */
        for (int t = 0; t < l; ++t)
            for (int k = 0; k < 2 * OR_MAXL + 1; ++k) poly[k] = (k + 1) * poly[k + 1];
        double s = 1.0 / (pow(2.0, l) * factorial(l));
        for (int k = 0; k < 2 * OR_MAXL + 2; ++k) g_legendre[l][k] = poly[k] * s;
        for (int m = 0; m <= l; ++m)
            g_norm[l][m] = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
    }
    g_sh_ready = 1;
}

/* k-th derivative of P_l at z */
static double legendre_deriv(int l, int k, double z) {
    double acc = 0.0;
    for (int p = 2 * OR_MAXL + 1; p >= k; --p) {
        double c = g_legendre[l][p];
        for (int t = 0; t < k; ++t) c *= (double)(p - t);
        acc = acc * z + c;   /* Horner in z over powers p-k */
    }
    return acc;
}

/* (x + i y)^m and its partial derivatives in x and y */
static void cpow_xy(double x, double y, int m, double* re, double* im) {
    double r = 1.0, i = 0.0;
    for (int k = 0; k < m; ++k) { double nr = r * x - i * y; double ni = r * y + i * x; r = nr; i = ni; }
    *re = r; *im = i;
}

/* Y_j(d) for j < (deg+1)^2 and, if grad != NULL, dY_j/dd (3 per j). */
static void sh_eval(int deg, const double d[3], double* Y, double* grad) {
    sh_init();
    double x = d[0], y = d[1], z = d[2];
    int j = 0;
    for (int l = 0; l <= deg; ++l) {
        for (int m = -l; m <= l; ++m, ++j) {
            int am = m < 0 ? -m : m;
            double K = (am == 0 ? 1.0 : sqrt(2.0)) * g_norm[l][am] * ((am & 1) ? -1.0 : 1.0);
            double P = legendre_deriv(l, am, z);
            double dP = legendre_deriv(l, am + 1, z);
            double re, im, re1 = 0, im1 = 0;
            cpow_xy(x, y, am, &re, &im);
            if (am > 0) cpow_xy(x, y, am - 1, &re1, &im1);
            double ang, dang_dx, dang_dy;
            if (m >= 0) { ang = re; dang_dx = am * re1; dang_dy = -am * im1; }
            else        { ang = im; dang_dx = am * im1; dang_dy = am * re1; }
            Y[j] = K * P * ang;
            if (grad) {
                grad[3 * j + 0] = K * P * dang_dx;
                grad[3 * j + 1] = K * P * dang_dy;
                grad[3 * j + 2] = K * dP * ang;
            }
        }
    }
}

/* exported for the basis pins */
void or_sh_basis(int deg, const double* d, double* Y, double* grad) { sh_eval(deg, d, Y, grad); }

/* -------------------------------------------------------- tile rectangle ---
 * Reading of "16x16 pixel blocks that share the same set of Gaussians"
 * (Sec. IV-C.1): a Gaussian belongs to every tile that meets the closed square
 * [u-r, u+r] x [v-r, v+r]; tile (tx, ty) covers pixels [16tx, 16tx+16) x
 * [16ty, 16ty+16).  With r an integer, floor((u +- r)/16) equals
 * floor((floor(u) +- r)/16), which is evaluated in integers.  Returns the
 * number of tiles and writes x0, x1, y0, y1.
 */
static int64_t tile_rect(double u, double v, int64_t r, int W, int H, int32_t rect[4]) {
    int64_t tx = (W + OR_TILE - 1) / OR_TILE, ty = (H + OR_TILE - 1) / OR_TILE;
    rect[0] = 0; rect[1] = -1; rect[2] = 0; rect[3] = -1;
    if (r <= 0 || !isfinite(u) || !isfinite(v)) return 0;
    if (u < -(double)r || u >= (double)(OR_TILE * tx + r)) return 0;
    if (v < -(double)r || v >= (double)(OR_TILE * ty + r)) return 0;
    int64_t fu = (int64_t)floor(u), fv = (int64_t)floor(v);
    int64_t x0 = floor_div(fu - r, OR_TILE), x1 = floor_div(fu + r, OR_TILE);
    int64_t y0 = floor_div(fv - r, OR_TILE), y1 = floor_div(fv + r, OR_TILE);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > tx - 1) x1 = tx - 1;
    if (y1 > ty - 1) y1 = ty - 1;
    if (x0 > x1 || y0 > y1) return 0;
    rect[0] = (int32_t)x0; rect[1] = (int32_t)x1; rect[2] = (int32_t)y0; rect[3] = (int32_t)y1;
    return (x1 - x0 + 1) * (y1 - y0 + 1);
}

int64_t or_tile_rect(double u, double v, int64_t r, int W, int H, int32_t* rect) {
    return tile_rect(u, v, r, W, H, rect);
}

/* ---------------------------------------------------------- projection ----
 * Per Gaussian (Sec. II-A):
 *   opacity o = sigmoid(logit); q^ = q/|q|; Sigma = R(q^) diag(e^s)^2 R(q^)^T
 *   t = W mu + t_cw with W = R_cw (viewing transform)
 *   J = [[fx/tz, 0, -fx sx/tz], [0, fy/tz, -fy sy/tz]] with slopes
 *       s = clamp(t_xy/tz, +-1.3 tan_half_fov) (first-order pinhole Jacobian)
 *   Sigma' = J W Sigma W^T J^T + 0.3 I  (low-pass dilation, a reading)
 *   conic = Sigma'^-1 (A, B, C) = (S11, -S01, S00)/det, culled if det <= 0
 *   r = ceil(3 sqrt(lambda_max)), lambda_max = m + sqrt(max(0.1, m^2 - det))
 *   (u, v) = (fx tx/tz + cx, fy ty/tz + cy)
 *   colour_k = max(0, sum_j Y_j(d) f_jk + 1/2), d = unit(mu - camera centre)
 * Culled (radius 0, no tiles): tz <= near_z, non-finite values, det <= 0,
 * radius above 2^22 px.
 * flags bit0: 3 sqrt(lambda_max) lies within a relative 2e-5 of an integer
 * (an FP32 evaluation may round the radius the other way);
 * flags bit1: tz within a relative 1e-5 of near_z; bit2: a slope within 1e-5 of
 * its clamp; bit3: an SH colour within 1e-6 of its clamp at 0.
 */
typedef struct {
    double o, qn[4], qnorm, R[9], S[3], Sigma[9];
    double t[3], sx, sy, clampx, clampy, J[6], T[6], Sp[3] /*a b c*/, det;
    double d[3], dirlen, Y[16], raw[3];
    int culled, radius;
} or_gauss_state;

static int project_one(int deg, const double* p_mean, const double* p_ls, const double* p_q, double logit,
                       const double* p_sh /* [nc][3] gathered */, const double* cam,
                       or_gauss_state* st, double rec[9], double* depth, uint8_t* flag) {
    const double fx = cam[0], fy = cam[1], cx = cam[2], cy = cam[3], near_z = cam[4];
    const double* W = cam + 7; const double* tcw = cam + 16;
    memset(st, 0, sizeof *st);
    *flag = 0;
    for (int k = 0; k < 9; ++k) rec[k] = 0.0;
    *depth = 0.0;
    st->culled = 1;

    st->o = 1.0 / (1.0 + exp(-logit));
    double qn2 = p_q[0] * p_q[0] + p_q[1] * p_q[1] + p_q[2] * p_q[2] + p_q[3] * p_q[3];
    st->qnorm = sqrt(qn2);
    for (int k = 0; k < 4; ++k) st->qn[k] = p_q[k] / st->qnorm;
    quat_to_rot(st->qn, st->R);
    for (int k = 0; k < 3; ++k) st->S[k] = exp(p_ls[k]);
    /* Sigma = R S S^T R^T */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += st->R[3 * i + k] * st->S[k] * st->S[k] * st->R[3 * j + k];
            st->Sigma[3 * i + j] = s;
        }
    for (int i = 0; i < 3; ++i)
        st->t[i] = W[3 * i] * p_mean[0] + W[3 * i + 1] * p_mean[1] + W[3 * i + 2] * p_mean[2] + tcw[i];
    double tz = st->t[2];
    if (!(tz > near_z) || !isfinite(tz)) {
        if (isfinite(tz) && fabs(tz - near_z) <= 1e-5 * near_z) *flag |= 2;
        return 0;
    }
    if (fabs(tz - near_z) <= 1e-5 * near_z) *flag |= 2;
    double limx = OR_SLOPE_LIMIT * cam[5], limy = OR_SLOPE_LIMIT * cam[6];
    double rx = st->t[0] / tz, ry = st->t[1] / tz;
    st->sx = rx; st->sy = ry; st->clampx = 0; st->clampy = 0;
    if (rx > limx) { st->sx = limx; st->clampx = 1; }
    if (rx < -limx) { st->sx = -limx; st->clampx = 1; }
    if (ry > limy) { st->sy = limy; st->clampy = 1; }
    if (ry < -limy) { st->sy = -limy; st->clampy = 1; }
    if (fabs(fabs(rx) - limx) <= 1e-5 * limx || fabs(fabs(ry) - limy) <= 1e-5 * limy) *flag |= 4;
    st->J[0] = fx / tz; st->J[1] = 0; st->J[2] = -fx * st->sx / tz;
    st->J[3] = 0; st->J[4] = fy / tz; st->J[5] = -fy * st->sy / tz;
    /* T = J W (2x3) */
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            st->T[3 * i + j] = st->J[3 * i] * W[j] + st->J[3 * i + 1] * W[3 + j] + st->J[3 * i + 2] * W[6 + j];
    /* Sigma' = T Sigma T^T */
    double Sp[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) s += st->T[3 * i + k] * st->Sigma[3 * k + l] * st->T[3 * j + l];
            Sp[2 * i + j] = s;
        }
    double a = Sp[0] + OR_DILATION, b = Sp[1], c = Sp[3] + OR_DILATION;
    st->Sp[0] = a; st->Sp[1] = b; st->Sp[2] = c;
    double det = a * c - b * b;
    st->det = det;
    if (!(det > 0.0) || !isfinite(det)) return 0;
    double A = c / det, B = -b / det, C = a / det;
    double mid = 0.5 * (a + c);
    double lam = mid + sqrt(fmax(0.1, mid * mid - det));
    double r3 = 3.0 * sqrt(lam);
    if (!isfinite(r3) || r3 > OR_RADIUS_MAX) return 0;
    double rr = ceil(r3);
    if (fabs(r3 - nearbyint(r3)) <= 2e-5 * fmax(1.0, r3)) *flag |= 1;
    double u = fx * st->t[0] / tz + cx, v = fy * st->t[1] / tz + cy;
    /* colour */
    double cc[3];
    for (int i = 0; i < 3; ++i) cc[i] = -(W[i] * tcw[0] + W[3 + i] * tcw[1] + W[6 + i] * tcw[2]);
    double dir[3] = {p_mean[0] - cc[0], p_mean[1] - cc[1], p_mean[2] - cc[2]};
    st->dirlen = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    for (int k = 0; k < 3; ++k) st->d[k] = dir[k] / st->dirlen;
    int nc = (deg + 1) * (deg + 1);
    sh_eval(deg, st->d, st->Y, NULL);
    double rgb[3];
    for (int ch = 0; ch < 3; ++ch) {
        double s = 0.0;
        for (int j = 0; j < nc; ++j) s += st->Y[j] * p_sh[3 * j + ch];
        st->raw[ch] = s + 0.5;
        rgb[ch] = st->raw[ch] > 0.0 ? st->raw[ch] : 0.0;
        if (fabs(st->raw[ch]) <= 1e-6) *flag |= 8;
    }
    rec[0] = u; rec[1] = v; rec[2] = A; rec[3] = B; rec[4] = C; rec[5] = st->o;
    rec[6] = rgb[0]; rec[7] = rgb[1]; rec[8] = rgb[2];
    for (int k = 0; k < 9; ++k)
        if (!isfinite(rec[k])) { for (int q = 0; q < 9; ++q) rec[q] = 0.0; return 0; }
    *depth = tz;
    st->culled = 0;
    st->radius = (int)rr;
    return (int)rr;
}

static void gather_params(int64_t n, int64_t i, int deg, const double* means, const double* ls,
                          const double* quats, const double* sh,
                          double m[3], double s[3], double q[4], double* shg) {
    for (int k = 0; k < 3; ++k) { m[k] = means[k * n + i]; s[k] = ls[k * n + i]; }
    for (int k = 0; k < 4; ++k) q[k] = quats[k * n + i];
    int nc = (deg + 1) * (deg + 1);
    for (int j = 0; j < nc; ++j)
        for (int ch = 0; ch < 3; ++ch) shg[3 * j + ch] = sh[(3 * j + ch) * n + i];
}

/* Project every Gaussian.  rect is [n][4] (x0, x1, y0, y1); tiles_touched[n]. */
int or_project(int64_t n, int deg, const double* means, const double* log_scales, const double* quats,
               const double* logits, const double* sh, const double* cam, int W, int H,
               double* rec, double* depth, int32_t* radius, int32_t* rect, int64_t* tiles_touched,
               uint8_t* flags) {
    if (n < 0 || deg < 0 || deg > OR_MAXL || W <= 0 || H <= 0) return -1;
    sh_init();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double m[3], s[3], q[4], shg[48];
        or_gauss_state st;
        gather_params(n, i, deg, means, log_scales, quats, sh, m, s, q, shg);
        uint8_t fl;
        int r = project_one(deg, m, s, q, logits[i], shg, cam, &st, rec + 9 * i, depth + i, &fl);
        radius[i] = r;
        flags[i] = fl;
        tiles_touched[i] = tile_rect(rec[9 * i], rec[9 * i + 1], r, W, H, rect + 4 * i);
        if (tiles_touched[i] == 0) radius[i] = r; /* radius kept; no tiles */
    }
    return 0;
}

/* ------------------------------------------------------------ bin + sort ---
 * Sec. II-A: the Gaussians contributing to a pixel are taken in depth order;
 * Sec. IV-C.1: 16x16 tiles share one list.  Readings: entries are emitted in
 * index order (rows y0..y1, columns x0..x1 within a row) at the exclusive
 * prefix sum of tiles_touched, then sorted by (tile, FP32 depth bits, index),
 * which is a total order; empty tiles get (S_t, S_t).
 */
typedef struct { uint32_t tile, key, idx; } or_entry;

static int entry_cmp(const void* pa, const void* pb) {
    const or_entry* a = (const or_entry*)pa;
    const or_entry* b = (const or_entry*)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Number of (tile, Gaussian) pairs for the given FP32-valued projection. */
int64_t or_bin_count(int64_t n, const double* u, const double* v, const int32_t* radius, int W, int H,
                     int64_t* tiles_touched, int64_t* offsets) {
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t rect[4];
        tiles_touched[i] = tile_rect(u[i], v[i], radius[i], W, H, rect);
        offsets[i] = total;
        total += tiles_touched[i];
    }
    return total;
}

/* Every Gaussian's tile rectangle rect[i] = (x0, x1, y0, y1), inclusive
 * (x1 < x0 when it touches no tile), and the per-tile entry counts
 * counts[ty * tiles_x + tx] (a Gaussian counts once in every tile of its
 * rectangle).  Returns K, the total. */
int64_t or_bin_rects(int64_t n, const double* u, const double* v, const int32_t* radius, int W, int H,
                     int32_t* rect, int64_t* counts) {
    int64_t tx = (W + OR_TILE - 1) / OR_TILE, ty = (H + OR_TILE - 1) / OR_TILE;
    int64_t total = 0;
    for (int64_t t = 0; t < tx * ty; ++t) counts[t] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t* r = rect + 4 * i;
        total += tile_rect(u[i], v[i], radius[i], W, H, r);
        for (int y = r[2]; y <= r[3]; ++y)
            for (int x = r[0]; x <= r[1]; ++x) ++counts[y * tx + x];
    }
    return total;
}

/* point_list[K], ranges[T][2]; depth_bits are the FP32 bit patterns of depth.
 * tile_mask (optional): only the tiles with a non-zero byte get their lists
 * (the others get empty ranges); K is then the entry count of those tiles. */
int or_bin_sort(int64_t n, const double* u, const double* v, const int32_t* radius,
                const uint32_t* depth_bits, int W, int H, const uint8_t* tile_mask, int64_t K,
                uint32_t* point_list, uint32_t* ranges) {
    int64_t tx = (W + OR_TILE - 1) / OR_TILE, ty = (H + OR_TILE - 1) / OR_TILE;
    int64_t ntiles = tx * ty;
    or_entry* e = (or_entry*)malloc(sizeof(or_entry) * (size_t)(K > 0 ? K : 1));
    if (!e) return -2;
    int64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t rect[4];
        int64_t cnt = tile_rect(u[i], v[i], radius[i], W, H, rect);
        if (cnt == 0) continue;
        for (int y = rect[2]; y <= rect[3]; ++y)
            for (int x = rect[0]; x <= rect[1]; ++x) {
                if (tile_mask && !tile_mask[y * tx + x]) continue;
                if (off >= K) { free(e); return -3; }
                e[off].tile = (uint32_t)(y * tx + x);
                e[off].key = depth_bits[i];
                e[off].idx = (uint32_t)i;
                ++off;
            }
    }
    if (off != K) { free(e); return -3; }
    qsort(e, (size_t)K, sizeof(or_entry), entry_cmp);
    for (int64_t m = 0; m < K; ++m) point_list[m] = e[m].idx;
    /* ranges by linear scan */
    int64_t m = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        ranges[2 * t] = (uint32_t)m;
        while (m < K && e[m].tile == (uint32_t)t) ++m;
        ranges[2 * t + 1] = (uint32_t)m;
    }
    free(e);
    return 0;
}

/* ------------------------------------------------------- forward render ---
 * Sec. II-A blending, per pixel, over the tile's depth-sorted list:
 *   power = -1/2 (A dx^2 + C dy^2) - B dx dy, (dx, dy) = (u, v) - pixel centre,
 *   with the pixel centre at (x + 0.5, y + 0.5) (reading);
 *   alpha = min(0.99, o e^power); entries with power > 0 or alpha < 1/255 are
 *   skipped; if T (1 - alpha) < 1e-4 the walk stops before blending (reading);
 *   otherwise C += c alpha T, T *= (1 - alpha), n_contrib = position + 1.
 *   out = C + T bg.
 *
 * Near-threshold decisions.  An FP32 evaluation of the same walk may take a
 * decision the other way when the FP64 value lies close to its threshold.  The
 * walk counts such "near" decisions in the order it meets them (k = 0, 1, ...)
 * and sets a pixel flag for each kind:
 *   bit0  alpha within a relative ma of 1/255            (skip or blend),
 *   bit1  T' within a relative mT of 1e-4                (stop or blend),
 *   bit2  o e^power within a relative mc of 0.99          (clamp or not).
 * The pair's alpha margins are ma = margins[0] + margins[3] Q and
 * mc = margins[2] + margins[3] Q with Q = (|A| dx^2 + 2 |B dx dy| + |C| dy^2)/2,
 * the magnitude of the power's terms: a power evaluated in FP32 errs by a few
 * units of 2^-24 of Q, which exceeds the fixed margin for elongated footprints
 * whose terms cancel (margins[3] = 0: fixed margins only).
 * mT starts at margins[1] and grows by alpha/(1 - alpha) ma + 2^-22 for
 * every blended entry (clamped entries add 1e-6 instead): the relative error
 * that a product of (1 - alpha) factors carries when each alpha is known to
 * ma relative and each product is rounded once.
 * Bit k of `flips` (a per-pixel mask; 0 = none) makes the walk take the other
 * branch of near decision k; with flips = 0 this is the plain definition.
 * The walk stops counting at 8 near decisions (flips has 8 bits).
 */
typedef struct {
    uint32_t* idx;
    double *alpha, *T, *eg, *dx, *dy;
    uint8_t* clamped;
    int cap;
} or_blend_buf;

static void blend_buf_grow(or_blend_buf* b, int need) {
    if (need <= b->cap) return;
    int cap = b->cap ? b->cap : 256;
    while (cap < need) cap *= 2;
    b->idx = (uint32_t*)realloc(b->idx, sizeof(uint32_t) * cap);
    b->alpha = (double*)realloc(b->alpha, sizeof(double) * cap);
    b->T = (double*)realloc(b->T, sizeof(double) * cap);
    b->eg = (double*)realloc(b->eg, sizeof(double) * cap);
    b->dx = (double*)realloc(b->dx, sizeof(double) * cap);
    b->dy = (double*)realloc(b->dy, sizeof(double) * cap);
    b->clamped = (uint8_t*)realloc(b->clamped, cap);
    b->cap = cap;
}

static void blend_buf_free(or_blend_buf* b) {
    free(b->idx); free(b->alpha); free(b->T); free(b->eg); free(b->dx); free(b->dy); free(b->clamped);
}

typedef struct {
    double acc[3], T;
    int32_t nc;
    uint8_t flags, n_near;
    int nb; /* blended entries recorded in the buffer */
} or_pixel;

/* One pixel's front-to-back walk over list entries [s, e).  If bl is not NULL
 * the blended entries are recorded in walk order (for the backward). */
static void walk_pixel(const double* rec, const uint32_t* point_list, uint32_t s, uint32_t e, double cxp,
                       double cyp, const double* margins, uint32_t flips, or_blend_buf* bl, or_pixel* out) {
    double T = 1.0, acc[3] = {0, 0, 0};
    double mT = margins[1];
    int32_t nc = 0;
    uint8_t fl = 0;
    int k = 0, nb = 0;
    for (uint32_t m = s; m < e; ++m) {
        const double* g = rec + 9 * (int64_t)point_list[m];
        double dx = g[0] - cxp, dy = g[1] - cyp;
        double power = -0.5 * (g[2] * dx * dx + g[4] * dy * dy) - g[3] * dx * dy;
        if (power > 0.0) continue; /* only an FP guard: Sigma' is positive definite */
        double eg = exp(power);
        double og = g[5] * eg;
        double qm = margins[3] > 0.0
                        ? margins[3] * 0.5 * (fabs(g[2]) * dx * dx + 2.0 * fabs(g[3] * dx * dy) + fabs(g[4]) * dy * dy)
                        : 0.0;
        double ma = margins[0] + qm;
        int clamp = !(og < OR_ALPHA_MAX);
        if (fabs(og - OR_ALPHA_MAX) <= (margins[2] + qm) * OR_ALPHA_MAX && k < 8) {
            fl |= 4;
            if ((flips >> k) & 1u) clamp = !clamp;
            ++k;
        }
        double alpha = clamp ? OR_ALPHA_MAX : og;
        int skip = alpha < OR_ALPHA_MIN;
        if (fabs(alpha - OR_ALPHA_MIN) <= ma * OR_ALPHA_MIN && k < 8) {
            fl |= 1;
            if ((flips >> k) & 1u) skip = !skip;
            ++k;
        }
        if (skip) continue;
        double Tn = T * (1.0 - alpha);
        int stop = Tn < OR_T_MIN;
        if (fabs(Tn - OR_T_MIN) <= mT * OR_T_MIN && k < 8) {
            fl |= 2;
            if ((flips >> k) & 1u) stop = !stop;
            ++k;
        }
        if (stop) break;
        if (bl) {
            blend_buf_grow(bl, nb + 1);
            bl->idx[nb] = point_list[m]; bl->alpha[nb] = alpha; bl->T[nb] = T; bl->eg[nb] = eg;
            bl->dx[nb] = dx; bl->dy[nb] = dy; bl->clamped[nb] = (uint8_t)clamp;
        }
        ++nb;
        for (int ch = 0; ch < 3; ++ch) acc[ch] += g[6 + ch] * alpha * T;
        T = Tn;
        nc = (int32_t)(m - s + 1);
        mT += (clamp ? 1e-6 : alpha / (1.0 - alpha) * ma) + 0x1p-22;
    }
    for (int ch = 0; ch < 3; ++ch) out->acc[ch] = acc[ch];
    out->T = T;
    out->nc = nc;
    out->flags = fl;
    out->n_near = (uint8_t)k;
    out->nb = nb;
}

/* Forward render of every pixel (of the tiles selected by tile_mask, if not
 * NULL).  flips: per-pixel near-decision masks (NULL = none).  pix_flags and
 * n_near (per pixel, may be NULL) receive the walk's flags and near count. */
int or_render_fwd(int W, int H, const double* rec, const uint32_t* point_list, const uint32_t* ranges,
                  const double* bg, const double* margins, const uint8_t* tile_mask, const uint8_t* flips,
                  double* image, double* final_T, int32_t* n_contrib, uint8_t* pix_flags, uint8_t* n_near) {
    int64_t tx = (W + OR_TILE - 1) / OR_TILE, ty = (H + OR_TILE - 1) / OR_TILE;
    int64_t HW = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < tx * ty; ++t) {
        if (tile_mask && !tile_mask[t]) continue;
        int64_t x0 = (t % tx) * OR_TILE, y0 = (t / tx) * OR_TILE;
        uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
        for (int64_t py = y0; py < y0 + OR_TILE && py < H; ++py)
            for (int64_t px = x0; px < x0 + OR_TILE && px < W; ++px) {
                int64_t p = py * W + px;
                or_pixel o;
                walk_pixel(rec, point_list, s, e, px + 0.5, py + 0.5, margins, flips ? flips[p] : 0u, NULL, &o);
                for (int ch = 0; ch < 3; ++ch) image[ch * HW + p] = o.acc[ch] + o.T * bg[ch];
                final_T[p] = o.T;
                n_contrib[p] = o.nc;
                if (pix_flags) pix_flags[p] = o.flags;
                if (n_near) n_near[p] = o.n_near;
            }
    }
    return 0;
}

/* The same walk for a list of (pixel, flips) pairs: pixel index pix[j] =
 * y W + x with mask flips[j].  Outputs per pair: colour out[j][3] (with bg),
 * final_T, n_contrib, flags and near count.  Used to enumerate the outcomes a
 * flagged pixel may legitimately have. */
int or_render_pixels(int W, int H, const double* rec, const uint32_t* point_list, const uint32_t* ranges,
                     const double* bg, const double* margins, int64_t npairs, const int64_t* pix,
                     const uint8_t* flips, double* out, double* final_T, int32_t* n_contrib, uint8_t* pix_flags,
                     uint8_t* n_near) {
    int64_t tx = (W + OR_TILE - 1) / OR_TILE;
    for (int64_t j = 0; j < npairs; ++j)
        if (pix[j] < 0 || pix[j] >= (int64_t)W * H) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < npairs; ++j) {
        int64_t px = pix[j] % W, py = pix[j] / W;
        int64_t t = (py / OR_TILE) * tx + px / OR_TILE;
        or_pixel o;
        walk_pixel(rec, point_list, ranges[2 * t], ranges[2 * t + 1], px + 0.5, py + 0.5, margins, flips[j], NULL,
                   &o);
        for (int ch = 0; ch < 3; ++ch) out[3 * j + ch] = o.acc[ch] + o.T * bg[ch];
        final_T[j] = o.T;
        n_contrib[j] = o.nc;
        pix_flags[j] = o.flags;
        n_near[j] = o.n_near;
    }
    return 0;
}

/* ------------------------------------------------------ backward render ---
 * Exact derivative of the blending above with the set of blended entries held
 * fixed (skips and the stop are piecewise-constant decisions; `flips` selects
 * the branches exactly as in the forward).  For blended entry m of a pixel
 * with upstream gradient G:
 *   dL/dc_m   = alpha_m T_m G
 *   dL/dalpha = sum_k G_k (c_mk T_m - S_mk/(1 - alpha_m)),
 *               S_m = sum_{j>m, blended} c_j alpha_j T_j + T_final bg
 *   alpha = o e^power (unclamped branch): dL/do = e^power dL/dalpha,
 *   dL/dpower = alpha dL/dalpha; on the clamped branch both are 0.
 *   dL/du = dL/dpower (-A dx - B dy), dL/dv = dL/dpower (-B dx - C dy)
 *   dL/dA = -1/2 dx^2 dL/dpower, dL/dB = -dx dy dL/dpower,
 *   dL/dC = -1/2 dy^2 dL/dpower  (B enters the power once, as -B dx dy).
 * The oracle recomputes the forward per pixel itself, keeps the blended list,
 * and forms S_m as an explicit suffix sum.  g2d is [n][9] in record order
 * (u, v, A, B, C, o, r, g, b), summed over pixels, and is overwritten.
 * Optional outputs, scales for judging any other summation order (its
 * rounding error is proportional to them, not to the sum):
 *   g2d_mass[n][9]  sum over pixels of |per-pixel term| of each g2d entry;
 *   cov_mass[n][3]  the same for the per-pixel conic gradient carried to the
 *                   2D covariance Sigma' = K^-1 = [[a, b], [b, c]] before the
 *                   sum, dL/dSigma' = -K (dL/dK) K, as (a, b, c) with b
 *                   counted in both off-diagonal places.
 */
int or_render_bwd(int W, int H, int64_t n, const double* rec, const uint32_t* point_list,
                  const uint32_t* ranges, const double* bg, const double* dL_dimage,
                  const uint8_t* tile_mask, const double* margins, const uint8_t* flips, double* g2d,
                  double* g2d_mass, double* cov_mass) {
    int64_t tx = (W + OR_TILE - 1) / OR_TILE, ty = (H + OR_TILE - 1) / OR_TILE;
    int64_t HW = (int64_t)W * H;
    memset(g2d, 0, sizeof(double) * 9 * (size_t)n);
    if (g2d_mass) memset(g2d_mass, 0, sizeof(double) * 9 * (size_t)n);
    if (cov_mass) memset(cov_mass, 0, sizeof(double) * 3 * (size_t)n);
#pragma omp parallel
    {
        or_blend_buf bl;
        memset(&bl, 0, sizeof bl);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < tx * ty; ++t) {
            if (tile_mask && !tile_mask[t]) continue;
            int64_t x0 = (t % tx) * OR_TILE, y0 = (t / tx) * OR_TILE;
            uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
            for (int64_t py = y0; py < y0 + OR_TILE && py < H; ++py)
                for (int64_t px = x0; px < x0 + OR_TILE && px < W; ++px) {
                    int64_t p = py * W + px;
                    double G[3] = {dL_dimage[p], dL_dimage[HW + p], dL_dimage[2 * HW + p]};
                    /* forward walk, remembering the blended entries */
                    or_pixel o;
                    walk_pixel(rec, point_list, s, e, px + 0.5, py + 0.5, margins, flips ? flips[p] : 0u, &bl, &o);
                    /* suffix sums S_m, walking back */
                    double S[3] = {o.T * bg[0], o.T * bg[1], o.T * bg[2]};
                    for (int k = o.nb - 1; k >= 0; --k) {
                        const double* g = rec + 9 * (int64_t)bl.idx[k];
                        double a = bl.alpha[k], Tm = bl.T[k];
                        double dc[3], dalpha = 0.0;
                        for (int ch = 0; ch < 3; ++ch) {
                            dc[ch] = a * Tm * G[ch];
                            dalpha += G[ch] * (g[6 + ch] * Tm - S[ch] / (1.0 - a));
                        }
                        double dpow = 0.0, dop = 0.0;
                        if (!bl.clamped[k]) { dop = bl.eg[k] * dalpha; dpow = a * dalpha; }
                        double dx = bl.dx[k], dy = bl.dy[k];
                        double gr[9];
                        gr[0] = dpow * (-g[2] * dx - g[3] * dy);
                        gr[1] = dpow * (-g[3] * dx - g[4] * dy);
                        gr[2] = -0.5 * dx * dx * dpow;
                        gr[3] = -dx * dy * dpow;
                        gr[4] = -0.5 * dy * dy * dpow;
                        gr[5] = dop;
                        gr[6] = dc[0]; gr[7] = dc[1]; gr[8] = dc[2];
                        double* out = g2d + 9 * (int64_t)bl.idx[k];
                        for (int q = 0; q < 9; ++q) {
#pragma omp atomic
                            out[q] += gr[q];
                        }
                        if (g2d_mass) {
                            double* mo = g2d_mass + 9 * (int64_t)bl.idx[k];
                            for (int q = 0; q < 9; ++q) {
#pragma omp atomic
                                mo[q] += fabs(gr[q]);
                            }
                        }
                        if (cov_mass) {
                            /* -K Gc K with Gc = [[gA, gB/2], [gB/2, gC]] */
                            double K[4] = {g[2], g[3], g[3], g[4]};
                            double Gc[4] = {gr[2], 0.5 * gr[3], 0.5 * gr[3], gr[4]};
                            double KG[4], GS[4];
                            for (int i = 0; i < 2; ++i)
                                for (int j = 0; j < 2; ++j) KG[2 * i + j] = K[2 * i] * Gc[j] + K[2 * i + 1] * Gc[2 + j];
                            for (int i = 0; i < 2; ++i)
                                for (int j = 0; j < 2; ++j)
                                    GS[2 * i + j] = -(KG[2 * i] * K[j] + KG[2 * i + 1] * K[2 + j]);
                            double cm[3] = {fabs(GS[0]), fabs(GS[1] + GS[2]), fabs(GS[3])};
                            double* co = cov_mass + 3 * (int64_t)bl.idx[k];
                            for (int q = 0; q < 3; ++q) {
#pragma omp atomic
                                co[q] += cm[q];
                            }
                        }
                        for (int ch = 0; ch < 3; ++ch) S[ch] += g[6 + ch] * a * Tm;
                    }
                }
        }
        blend_buf_free(&bl);
    }
    return 0;
}

/* ----------------------------------------------------- projection backward --
 * Exact chain rule through the projection above, per Gaussian, from the
 * record gradient g2d[9] to the raw parameters.  Steps:
 *   colour: clamp mask, dL/df_jk = Y_j(d) dL/dc_k, dL/dd = sum f_jk grad Y_j,
 *           then mu via (I - d d^T)/|mu - c|;
 *   opacity: dL/dlogit = dL/do o (1 - o);
 *   conic: K = Sigma'^-1, d(K) = -K d(Sigma') K, so the symmetric conic
 *          gradient Gc = [[gA, gB/2], [gB/2, gC]] gives dL/dSigma' = -K Gc K;
 *   Sigma' = T Sigma T^T (T = J W): dL/dSigma = T^T G T, dL/dT = 2 G T Sigma;
 *   dL/dJ = dL/dT W^T; J(t) with the clamp mask on the slopes; u, v -> t;
 *   t = W mu + t_cw -> dL/dmu += W^T dL/dt;
 *   Sigma = M M^T, M = R S: dL/dM = 2 dL/dSigma M, dL/ds_i = (R^T dL/dM)_ii S_i,
 *   dL/dR = dL/dM S, dL/dq^ through R(q^), dL/dq = (I - q^ q^^T) dL/dq^ / |q|.
 * Culled Gaussians get zero gradients.  Outputs use the parameter layouts.
 */
int or_project_bwd(int64_t n, int deg, const double* means, const double* log_scales, const double* quats,
                   const double* logits, const double* sh, const double* cam, const double* g2d,
                   double* g_means, double* g_log_scales, double* g_quats, double* g_logits, double* g_sh) {
    if (n < 0 || deg < 0 || deg > OR_MAXL) return -1;
    sh_init();
    const double fx = cam[0], fy = cam[1];
    const double* W = cam + 7;
    int nc = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double m[3], s[3], q[4], shg[48], rec[9], depth;
        uint8_t fl;
        or_gauss_state st;
        gather_params(n, i, deg, means, log_scales, quats, sh, m, s, q, shg);
        project_one(deg, m, s, q, logits[i], shg, cam, &st, rec, &depth, &fl);
        double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gl = 0;
        double gsh[48];
        memset(gsh, 0, sizeof gsh);
        if (!st.culled) {
            const double* g = g2d + 9 * i;
            /* colour */
            double Y[16], dY[48];
            sh_eval(deg, st.d, Y, dY);
            double gd[3] = {0, 0, 0};
            for (int ch = 0; ch < 3; ++ch) {
                double gc = st.raw[ch] >= 0.0 ? g[6 + ch] : 0.0;
                for (int j = 0; j < nc; ++j) {
                    gsh[3 * j + ch] = Y[j] * gc;
                    for (int k = 0; k < 3; ++k) gd[k] += gc * shg[3 * j + ch] * dY[3 * j + k];
                }
            }
            double dd = st.d[0] * gd[0] + st.d[1] * gd[1] + st.d[2] * gd[2];
            for (int k = 0; k < 3; ++k) gm[k] += (gd[k] - st.d[k] * dd) / st.dirlen;
            /* opacity */
            gl = g[5] * st.o * (1.0 - st.o);
            /* conic -> Sigma': dL/dSigma' = -K Gc K */
            double K[4] = {rec[2], rec[3], rec[3], rec[4]};
            double Gc[4] = {g[2], 0.5 * g[3], 0.5 * g[3], g[4]};
            double KG[4], GS[4];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) KG[2 * a + b] = K[2 * a] * Gc[b] + K[2 * a + 1] * Gc[2 + b];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) GS[2 * a + b] = -(KG[2 * a] * K[b] + KG[2 * a + 1] * K[2 + b]);
            /* dL/dSigma = T^T GS T ; dL/dT = 2 GS T Sigma */
            double gSig[9], gT[6];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double acc = 0;
                    for (int k = 0; k < 2; ++k)
                        for (int l = 0; l < 2; ++l) acc += st.T[3 * k + a] * GS[2 * k + l] * st.T[3 * l + b];
                    gSig[3 * a + b] = acc;
                }
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 3; ++b) {
                    double acc = 0;
                    for (int k = 0; k < 2; ++k)
                        for (int l = 0; l < 3; ++l) acc += GS[2 * a + k] * st.T[3 * k + l] * st.Sigma[3 * l + b];
                    gT[3 * a + b] = 2.0 * acc;
                }
            /* dL/dJ = dL/dT W^T */
            double gJ[6];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 3; ++b)
                    gJ[3 * a + b] = gT[3 * a] * W[3 * b] + gT[3 * a + 1] * W[3 * b + 1] + gT[3 * a + 2] * W[3 * b + 2];
            /* J(t): J00 = fx/tz, J02 = -fx sx/tz, J11 = fy/tz, J12 = -fy sy/tz */
            double tz = st.t[2];
            double gt[3] = {0, 0, 0};
            gt[2] += gJ[0] * (-fx / (tz * tz)) + gJ[4] * (-fy / (tz * tz));
            gt[2] += gJ[2] * (fx * st.sx / (tz * tz)) + gJ[5] * (fy * st.sy / (tz * tz));
            double gsx = gJ[2] * (-fx / tz), gsy = gJ[5] * (-fy / tz);
            if (!st.clampx) { gt[0] += gsx / tz; gt[2] += gsx * (-st.t[0] / (tz * tz)); }
            if (!st.clampy) { gt[1] += gsy / tz; gt[2] += gsy * (-st.t[1] / (tz * tz)); }
            /* u, v */
            gt[0] += g[0] * fx / tz;
            gt[1] += g[1] * fy / tz;
            gt[2] += -g[0] * fx * st.t[0] / (tz * tz) - g[1] * fy * st.t[1] / (tz * tz);
            for (int k = 0; k < 3; ++k) gm[k] += W[k] * gt[0] + W[3 + k] * gt[1] + W[6 + k] * gt[2];
            /* Sigma = M M^T, M = R S */
            double M[9], gM[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) M[3 * a + b] = st.R[3 * a + b] * st.S[b];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double acc = 0;
                    for (int k = 0; k < 3; ++k) acc += (gSig[3 * a + k] + gSig[3 * k + a]) * M[3 * k + b];
                    gM[3 * a + b] = acc; /* (G + G^T) M, = 2 G M for symmetric G */
                }
            for (int k = 0; k < 3; ++k) {
                double acc = 0;
                for (int a = 0; a < 3; ++a) acc += st.R[3 * a + k] * gM[3 * a + k];
                gs[k] = acc * st.S[k];
            }
            double gR[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) gR[3 * a + b] = gM[3 * a + b] * st.S[b];
            double dR[4][9];
            quat_rot_jac(st.qn, dR);
            double gqn[4];
            for (int k = 0; k < 4; ++k) {
                double acc = 0;
                for (int e = 0; e < 9; ++e) acc += gR[e] * dR[k][e];
                gqn[k] = acc;
            }
            double qd = 0;
            for (int k = 0; k < 4; ++k) qd += st.qn[k] * gqn[k];
            for (int k = 0; k < 4; ++k) gq[k] = (gqn[k] - st.qn[k] * qd) / st.qnorm;
        }
        for (int k = 0; k < 3; ++k) { g_means[k * n + i] = gm[k]; g_log_scales[k * n + i] = gs[k]; }
        for (int k = 0; k < 4; ++k) g_quats[k * n + i] = gq[k];
        g_logits[i] = gl;
        for (int j = 0; j < nc; ++j)
            for (int ch = 0; ch < 3; ++ch) g_sh[(3 * j + ch) * n + i] = gsh[3 * j + ch];
    }
    return 0;
}

int or_num_threads(void) {
    int t = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
#endif
    return t;
}

/* ======================================================= learned colour ===
 * Learned colour decoder (not in the paper; the build's optional replacement
 * of the SH colour read).  Per sample: x = [z (16 latent values); Y_0..15(d)]
 * (the 16 real SH values of the view direction), then
 *   h1 = ReLU(W1 x + b1) (64),  h2 = ReLU(W2 h1 + b2) (64),
 *   c  = sigmoid(W3 h2 + b3) (3).
 * Parameter vector (6467 values): W1[64][32], b1[64], W2[64][64], b2[64],
 * W3[3][64], b3[3], row-major.  Plain matrix-vector products, one sample at a
 * time; the caller widens the decoder's BF16 values exactly to FP64.
 */
#define OR_MLP_IN 32
#define OR_MLP_H 64
#define OR_MLP_OUT 3
#define OR_W1 0
#define OR_B1 (OR_W1 + OR_MLP_H * OR_MLP_IN)
#define OR_W2 (OR_B1 + OR_MLP_H)
#define OR_B2 (OR_W2 + OR_MLP_H * OR_MLP_H)
#define OR_W3 (OR_B2 + OR_MLP_H)
#define OR_B3 (OR_W3 + OR_MLP_OUT * OR_MLP_H)
#define OR_MLP_NPARAM (OR_B3 + OR_MLP_OUT)

static void mlp_forward_one(const double* x, const double* P, double* h1, double* h2, double* c) {
    for (int o = 0; o < OR_MLP_H; ++o) {
        double s = P[OR_B1 + o];
        for (int i = 0; i < OR_MLP_IN; ++i) s += P[OR_W1 + o * OR_MLP_IN + i] * x[i];
        h1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < OR_MLP_H; ++o) {
        double s = P[OR_B2 + o];
        for (int i = 0; i < OR_MLP_H; ++i) s += P[OR_W2 + o * OR_MLP_H + i] * h1[i];
        h2[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < OR_MLP_OUT; ++o) {
        double s = P[OR_B3 + o];
        for (int i = 0; i < OR_MLP_H; ++i) s += P[OR_W3 + o * OR_MLP_H + i] * h2[i];
        c[o] = 1.0 / (1.0 + exp(-s));
    }
}

int or_mlp_num_params(void) { return OR_MLP_NPARAM; }

/* out[S][3]; h1, h2 ([S][64]) optional. */
int or_mlp_fwd(int64_t S, const double* x, const double* P, double* out, double* h1o, double* h2o) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s) {
        double h1[OR_MLP_H], h2[OR_MLP_H];
        mlp_forward_one(x + OR_MLP_IN * s, P, h1, h2, out + OR_MLP_OUT * s);
        if (h1o) memcpy(h1o + OR_MLP_H * s, h1, sizeof h1);
        if (h2o) memcpy(h2o + OR_MLP_H * s, h2, sizeof h2);
    }
    return 0;
}

/* Gradient of sum_s dL_dc[s] . c(x_s) with respect to the parameters
 * (dP[6467], overwritten, summed over samples) and, if dx != NULL, the inputs
 * (dx[S][32]).  Textbook backpropagation: sigmoid' = c (1 - c), ReLU' = [h > 0]. */
int or_mlp_bwd(int64_t S, const double* x, const double* P, const double* dL_dc, double* dP, double* dx) {
    memset(dP, 0, sizeof(double) * OR_MLP_NPARAM);
#pragma omp parallel
    {
        double* acc = (double*)calloc(OR_MLP_NPARAM, sizeof(double));
#pragma omp for schedule(static)
        for (int64_t s = 0; s < S; ++s) {
            const double* xs = x + OR_MLP_IN * s;
            double h1[OR_MLP_H], h2[OR_MLP_H], c[OR_MLP_OUT];
            mlp_forward_one(xs, P, h1, h2, c);
            double g3[OR_MLP_OUT], g2[OR_MLP_H], g1[OR_MLP_H];
            for (int o = 0; o < OR_MLP_OUT; ++o) g3[o] = dL_dc[OR_MLP_OUT * s + o] * c[o] * (1.0 - c[o]);
            for (int o = 0; o < OR_MLP_OUT; ++o) {
                acc[OR_B3 + o] += g3[o];
                for (int i = 0; i < OR_MLP_H; ++i) acc[OR_W3 + o * OR_MLP_H + i] += g3[o] * h2[i];
            }
            for (int i = 0; i < OR_MLP_H; ++i) {
                double t = 0.0;
                for (int o = 0; o < OR_MLP_OUT; ++o) t += P[OR_W3 + o * OR_MLP_H + i] * g3[o];
                g2[i] = h2[i] > 0.0 ? t : 0.0;
            }
            for (int o = 0; o < OR_MLP_H; ++o) {
                acc[OR_B2 + o] += g2[o];
                for (int i = 0; i < OR_MLP_H; ++i) acc[OR_W2 + o * OR_MLP_H + i] += g2[o] * h1[i];
            }
            for (int i = 0; i < OR_MLP_H; ++i) {
                double t = 0.0;
                for (int o = 0; o < OR_MLP_H; ++o) t += P[OR_W2 + o * OR_MLP_H + i] * g2[o];
                g1[i] = h1[i] > 0.0 ? t : 0.0;
            }
            for (int o = 0; o < OR_MLP_H; ++o) {
                acc[OR_B1 + o] += g1[o];
                for (int i = 0; i < OR_MLP_IN; ++i) acc[OR_W1 + o * OR_MLP_IN + i] += g1[o] * xs[i];
            }
            if (dx) {
                for (int i = 0; i < OR_MLP_IN; ++i) {
                    double t = 0.0;
                    for (int o = 0; o < OR_MLP_H; ++o) t += P[OR_W1 + o * OR_MLP_IN + i] * g1[o];
                    dx[OR_MLP_IN * s + i] = t;
                }
            }
        }
#pragma omp critical
        for (int k = 0; k < OR_MLP_NPARAM; ++k) dP[k] += acc[k];
        free(acc);
    }
    return 0;
}

/* SH colour max(0, sum_j Y_j(d) f_j + 1/2) of Gaussian i at `per` given unit
 * directions dirs[n][per][3] -> out[n][per][3] (the distillation target before
 * clamping to [0, 1]). */
int or_sh_colour(int64_t n, int deg, const double* sh, const double* dirs, int per, double* out) {
    if (deg < 0 || deg > OR_MAXL) return -1;
    sh_init();
    int nc = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double Y[16];
        for (int k = 0; k < per; ++k) {
            sh_eval(deg, dirs + 3 * (per * i + k), Y, NULL);
            for (int ch = 0; ch < 3; ++ch) {
                double s = 0.0;
                for (int j = 0; j < nc; ++j) s += Y[j] * sh[(3 * j + ch) * n + i];
                s += 0.5;
                out[3 * (per * i + k) + ch] = s > 0.0 ? s : 0.0;
            }
        }
    }
    return 0;
}

/* Decoder inputs x[n*per][32] = [z_i (16); Y_0..15(d_ik)] for Gaussian i and
 * its k-th unit direction. */
int or_mlp_inputs(int64_t n, int per, const double* z, const double* dirs, double* x) {
    sh_init();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < per; ++k) {
            double* xs = x + OR_MLP_IN * (per * i + k);
            for (int j = 0; j < 16; ++j) xs[j] = z[16 * i + j];
            sh_eval(3, dirs + 3 * (per * i + k), xs + 16, NULL);
        }
    return 0;
}

/* ------------------------------------------------- colour-hash sampling ---
 * Similarity-based sampling with colour hashing (Sec. IV-C.1), an optional
 * approximate mode of the forward and backward compositing.  Readings (the
 * paper gives the quantisation and hash formulas and the aggregation rule,
 * not where the aggregation happens or what a merged Gaussian looks like):
 *   - Colour quantisation: each channel's 8-bit value is
 *     v8 = floor(255 clamp(c, 0, 1) + 1/2), evaluated in FP32 (two rounded
 *     operations, product then sum; a NaN channel counts as 0), and its level
 *     is c_q = floor(v8 / 256 * 16) = v8 >> 4 (16 levels per channel).
 *   - Hash: h = R_q * 256 + G_q * 16 + B_q, one of 4096 buckets.
 *   - Grouping: the 16x16 tile is the block that shares one Gaussian list;
 *     the list is taken in windows of `window` consecutive entries starting
 *     at the tile's first entry.  Inside a window, the entries whose Gaussians
 *     fall into the same bucket form one group.
 *   - Aggregation: a group of two or more is composited as one entry, its
 *     front-most member (the representative), whose colour becomes the mean
 *     of the members' colours and whose opacity becomes the accumulated
 *     opacity 1 - prod_j (1 - o_j) (what members with one footprint and one
 *     colour would composite to at the footprint's centre).  The other
 *     members are not composited.  A group of one keeps its record as it is,
 *     so window = 1 is the exact method.
 *   - Bucket table: over all list entries of the frame, per bucket, the
 *     entry count and the sums of colour and opacity (the representative
 *     colour of a bucket is its colour sum over its count).
 * The compositing itself is the plain walk above, run over per-entry records.
 */

/* 4-bit level of one colour channel (FP32, as stated above). */
static uint32_t chs_level(float c) {
    float cc = c > 0.0f ? (c < 1.0f ? c : 1.0f) : 0.0f; /* NaN -> 0 */
    float t = cc * 255.0f;
    t = t + 0.5f;
    uint32_t v8 = (uint32_t)floorf(t);
    return v8 >> 4;
}

/* Bucket of each of n FP32 colours rgb[n][3]. */
int or_colour_hash(int64_t n, const float* rgb, uint16_t* hash) {
    for (int64_t i = 0; i < n; ++i)
        hash[i] = (uint16_t)(chs_level(rgb[3 * i]) * 256u + chs_level(rgb[3 * i + 1]) * 16u +
                             chs_level(rgb[3 * i + 2]));
    return 0;
}

/* Per-entry records of the approximate mode.  For list position m (tile t,
 * window w) with Gaussian i = point_list[m]:
 *   rep[m]    = list position of the group's representative (m itself for a
 *               representative),
 *   size[m]   = number of members of m's group,
 *   rec_e[m]  = rec[i] with, for a representative, colour = the members'
 *               mean colour and opacity = 1 - prod (1 - o_j), and for every
 *               other member opacity 0 (never composited: alpha = 0 < 1/255).
 * Compositing rec_e with point list 0, 1, ..., K-1 and the same ranges is the
 * approximate render.  tab_count[4096] and tab_sum[4096][4] (r, g, b,
 * opacity) receive the bucket table (may be NULL).  Returns 0, or -1 for a
 * window outside [1, 2^20]. */
int or_chs_aggregate(int64_t ntiles, const uint32_t* ranges, const uint32_t* point_list, const double* rec,
                     const uint16_t* hash, int window, double* rec_e, int64_t* rep, int32_t* size,
                     uint32_t* tab_count, double* tab_sum) {
    if (window < 1 || window > (1 << 20)) return -1;
    if (tab_count) memset(tab_count, 0, sizeof(uint32_t) * 4096);
    if (tab_sum) memset(tab_sum, 0, sizeof(double) * 4096 * 4);
    int64_t first[4096];
    for (int b = 0; b < 4096; ++b) first[b] = -1;
    for (int64_t t = 0; t < ntiles; ++t) {
        int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        for (int64_t w0 = s; w0 < e; w0 += window) {
            int64_t w1 = w0 + window < e ? w0 + window : e;
            /* members: each entry joins the group of its bucket's first entry */
            for (int64_t m = w0; m < w1; ++m) {
                uint32_t h = hash[point_list[m]];
                if (first[h] < 0) first[h] = m;
                rep[m] = first[h];
            }
            /* group sizes, then each representative's mean colour and
             * accumulated opacity (members in list order) */
            for (int64_t m = w0; m < w1; ++m) {
                const double* g = rec + 9 * (int64_t)point_list[m];
                memcpy(rec_e + 9 * m, g, 9 * sizeof(double));
                size[m] = 0;
            }
            for (int64_t m = w0; m < w1; ++m) size[rep[m]] += 1;
            for (int64_t m = w0; m < w1; ++m) {
                if (rep[m] != m || size[m] == 1) continue; /* a group of one is its Gaussian */
                double csum[3] = {0, 0, 0}, keep = 1.0;
                for (int64_t j = m; j < w1; ++j) {
                    if (rep[j] != m) continue;
                    const double* g = rec + 9 * (int64_t)point_list[j];
                    for (int ch = 0; ch < 3; ++ch) csum[ch] += g[6 + ch];
                    keep *= 1.0 - g[5];
                }
                for (int ch = 0; ch < 3; ++ch) rec_e[9 * m + 6 + ch] = csum[ch] / size[m];
                rec_e[9 * m + 5] = 1.0 - keep;
            }
            for (int64_t m = w0; m < w1; ++m) {
                if (rep[m] != m) {
                    rec_e[9 * m + 5] = 0.0;
                    size[m] = size[rep[m]];
                }
                first[hash[point_list[m]]] = -1;
            }
        }
    }
    if (tab_count || tab_sum) {
        for (int64_t t = 0; t < ntiles; ++t)
            for (int64_t m = ranges[2 * t]; m < (int64_t)ranges[2 * t + 1]; ++m) {
                uint32_t i = point_list[m], h = hash[i];
                if (tab_count) tab_count[h] += 1;
                if (tab_sum)
                    for (int q = 0; q < 4; ++q) tab_sum[4 * h + q] += rec[9 * (int64_t)i + (q < 3 ? 6 + q : 5)];
            }
    }
    return 0;
}

/* Chain rule of the aggregation: from the gradients g_e[K][9] of the per-entry
 * records (the backward render of rec_e over point list 0..K-1) to the
 * Gaussians' record gradients g2d[n][9] (overwritten).  Per group with
 * representative m and members j (list positions):
 *   geometry (u, v, A, B, C): all of g_e[m] goes to the representative;
 *   colour: c_m = mean_j c_j, so each member gets g_e[m][colour] / size;
 *   opacity: o_m = 1 - prod_j (1 - o_j), so member j gets
 *            g_e[m][o] prod_{i != j} (1 - o_i).
 * Members other than the representative carry no geometry gradient of their
 * own (they are not composited). */
int or_chs_route(int64_t n, int64_t ntiles, const uint32_t* ranges, const uint32_t* point_list, const double* rec,
                 int window, const int64_t* rep, const int32_t* size, const double* g_e, double* g2d) {
    if (window < 1 || window > (1 << 20)) return -1;
    memset(g2d, 0, sizeof(double) * 9 * (size_t)n);
    for (int64_t t = 0; t < ntiles; ++t) {
        int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        for (int64_t w0 = s; w0 < e; w0 += window) {
            int64_t w1 = w0 + window < e ? w0 + window : e;
            for (int64_t m = w0; m < w1; ++m) {
                int64_t r = rep[m];
                if (r < w0 || r > m) return -2;
                const double* ge = g_e + 9 * r;
                double* out = g2d + 9 * (int64_t)point_list[m];
                if (r == m)
                    for (int q = 0; q < 5; ++q) out[q] += ge[q];
                for (int ch = 0; ch < 3; ++ch) out[6 + ch] += ge[6 + ch] / size[m];
                double others = 1.0;
                for (int64_t j = r; j < w1; ++j)
                    if (rep[j] == r && j != m) others *= 1.0 - rec[9 * (int64_t)point_list[j] + 5];
                out[5] += ge[5] * others;
            }
        }
    }
    return 0;
}

/* --------------------------------------------------- density control (T1) ---
 * Workload-sensitive density control (Sec. III-C): statistical thresholds on
 * the local density, densification of sparse points next to themselves with
 * Gaussian spread and a uniform perturbation, and merging of dense points.
 * Readings (the paper names the quantities, not every detail):
 *   - local density rho_i = number of other points within the radius r
 *     (Sec. III-C.1); the distance decision is taken in FP32, as the kernels
 *     take it: dx = x_i - x_j per axis, d2 = (dx^2 + dy^2) + dz^2, each
 *     operation rounded, compared with r2 = r r rounded (d2 <= r2);
 *   - thresholds rho_low = mu - alpha sigma, rho_high = mu + beta sigma over
 *     all points (Sec. III-C.1; population standard deviation), in FP64 from
 *     the exact integer sums S1 = sum rho, S2 = sum rho^2:
 *     mu = S1/n, sigma = sqrt(max(S2/n - mu^2, 0)); low: rho < rho_low,
 *     high: rho > rho_high;
 *   - the mean distance to the k nearest other points (Sec. III-C.2), nearest
 *     by (FP32 d2, index), sqrt and sum in FP32 in that order, over k;
 *   - densification: each low point spawns one new point
 *     p_new = p + (a d_bar) z + delta e with z ~ N(0, I3) and e ~ U(-1, 1)^3
 *     given per point as inputs (Sec. III-C.2: sigma_p = a d_bar, a > 1, and
 *     the uniform perturbation); the rest of its parameters are the
 *     parent's; one round per call (the caller repeats rounds);
 *   - merging (Sec. III-C.3): d_merge = mu_d + gamma sigma_d over every
 *     point's nearest-neighbour distance (FP64 statistics); a high point whose
 *     nearest neighbour is high, has it as its own nearest neighbour (mutual),
 *     and lies within d_merge merges with it into the lower index:
 *     position and SH colour opacity-weighted means, scale the mean scale
 *     (log of the mean of exp(log-scale) per axis), opacity accumulated
 *     1 - (1 - o_i)(1 - o_j), rotation of the more opaque (lower index on a
 *     tie); the higher index is removed;
 *   - output: the kept points in index order, then the new points in the
 *     order of their parents.
 */

/* FP32 squared distance between points i and j of means[3][n] (rounded as stated). */
static float dc_d2(const float* m, int64_t n, int64_t i, int64_t j) {
    float dx = m[i] - m[j];
    float dy = m[n + i] - m[n + j];
    float dz = m[2 * n + i] - m[2 * n + j];
    float s = dx * dx;
    s = s + dy * dy;
    s = s + dz * dz;
    return s;
}

/* rho of the queried points q[0..nq) (brute force over all n points). */
int or_density(int64_t n, const float* means, float r, int64_t nq, const int64_t* q, int32_t* rho) {
    float r2 = r * r;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < nq; ++a) {
        int64_t i = q[a];
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && dc_d2(means, n, i, j) <= r2) ++c;
        rho[a] = c;
    }
    return 0;
}

/* The k nearest other points of each queried point, by (FP32 d2, index):
 * idx[nq][k] (-1 past n - 1 points) and d2[nq][k]. */
int or_knn(int64_t n, const float* means, int k, int64_t nq, const int64_t* q, int64_t* idx, float* d2) {
    if (k < 1 || k > 64) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < nq; ++a) {
        int64_t i = q[a];
        int64_t* bi = idx + a * k;
        float* bd = d2 + a * k;
        int cnt = 0;
        for (int m = 0; m < k; ++m) { bi[m] = -1; bd[m] = INFINITY; }
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            float d = dc_d2(means, n, i, j);
            /* insert (d, j) if it precedes the current k-th */
            if (cnt == k && !(d < bd[k - 1] || (d == bd[k - 1] && j < bi[k - 1]))) continue;
            int pos = cnt < k ? cnt : k - 1;
            while (pos > 0 && (d < bd[pos - 1] || (d == bd[pos - 1] && j < bi[pos - 1]))) {
                bd[pos] = bd[pos - 1];
                bi[pos] = bi[pos - 1];
                --pos;
            }
            bd[pos] = d;
            bi[pos] = j;
            if (cnt < k) ++cnt;
        }
    }
    return 0;
}

static double dc_sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }
static double dc_softplus(double x) { return x > 0 ? x + log1p(exp(-x)) : log1p(exp(x)); }

/* One round of density control over n points (brute force, for small n).
 * prm[7] = r, alpha, beta, k, a, delta, gamma.  noise[6][n] = z (3 rows), e (3 rows).
 * Outputs (capacity 2n each, SoA with stride 2n): out_means[3], out_ls[3],
 * out_q[4], out_logit, out_sh[nc*3]; per input point: rho, cls (1 low, 2 high,
 * 0 neither), nn (nearest other point), dbar (mean k-NN distance, FP32), fate
 * (-1 removed, else output index); stats[8] = mu, sigma, rho_low, rho_high,
 * mu_d, sigma_d, d_merge, n_out.  Returns 0. */
int or_density_control(int64_t n, int deg, const float* means, const float* ls, const float* quats,
                       const float* logits, const float* sh, const double* prm, const float* noise,
                       double* out_means, double* out_ls, double* out_q, double* out_logit, double* out_sh,
                       int32_t* rho, int8_t* cls, int64_t* nn, float* dbar, int64_t* fate, double* stats) {
    const int nc = (deg + 1) * (deg + 1);
    const float r = (float)prm[0];
    const double alpha = prm[1], beta = prm[2];
    const int k = (int)prm[3];
    const float a = (float)prm[4], delta = (float)prm[5];
    const double gamma = prm[6];
    const int64_t cap = 2 * n;
    int64_t* q = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    q[0] = 0;
    for (int64_t i = 0; i < n; ++i) q[i] = i;
    or_density(n, means, r, n, q, rho);
    int64_t S1 = 0, S2 = 0;
    for (int64_t i = 0; i < n; ++i) { S1 += rho[i]; S2 += (int64_t)rho[i] * rho[i]; }
    double mu = n > 0 ? (double)S1 / (double)n : 0.0;
    double var = n > 0 ? (double)S2 / (double)n - mu * mu : 0.0;
    double sigma = sqrt(var > 0.0 ? var : 0.0);
    double lo = mu - alpha * sigma, hi = mu + beta * sigma;
    for (int64_t i = 0; i < n; ++i) cls[i] = rho[i] < lo ? 1 : (rho[i] > hi ? 2 : 0);
    /* k nearest neighbours of every point */
    int kk = k < 1 ? 1 : k;
    int64_t* ki = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1) * kk);
    float* kd = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1) * kk);
    or_knn(n, means, kk, n, q, ki, kd);
    double sd = 0.0, sd2 = 0.0;
    int64_t nd = 0;
    float* dnn = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        nn[i] = ki[i * kk];
        float s = 0.0f;
        int cnt = 0;
        for (int m = 0; m < kk; ++m)
            if (ki[i * kk + m] >= 0) { s = s + sqrtf(kd[i * kk + m]); ++cnt; }
        dbar[i] = cnt ? s / (float)cnt : 0.0f;
        dnn[i] = nn[i] >= 0 ? sqrtf(kd[i * kk]) : 0.0f;
        if (nn[i] >= 0) { sd += dnn[i]; sd2 += (double)dnn[i] * dnn[i]; ++nd; }
    }
    double mu_d = nd ? sd / (double)nd : 0.0;
    double var_d = nd ? sd2 / (double)nd - mu_d * mu_d : 0.0;
    double sigma_d = sqrt(var_d > 0.0 ? var_d : 0.0);
    double dmerge = mu_d + gamma * sigma_d;
    /* mutual nearest-neighbour merges among high points */
    int64_t* partner = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = nn[i];
        partner[i] = (cls[i] == 2 && j >= 0 && cls[j] == 2 && nn[j] == i && (double)dnn[i] <= dmerge) ? j : -1;
    }
    int64_t o = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = partner[i];
        if (j >= 0 && j < i) { fate[i] = -1; continue; }
        fate[i] = o;
        if (j < 0) {
            for (int c = 0; c < 3; ++c) { out_means[c * cap + o] = means[c * n + i]; out_ls[c * cap + o] = ls[c * n + i]; }
            for (int c = 0; c < 4; ++c) out_q[c * cap + o] = quats[c * n + i];
            out_logit[o] = logits[i];
            for (int c = 0; c < 3 * nc; ++c) out_sh[(int64_t)c * cap + o] = sh[(int64_t)c * n + i];
        } else {
            double oi = dc_sigmoid(logits[i]), oj = dc_sigmoid(logits[j]);
            double w = oi + oj;
            for (int c = 0; c < 3; ++c) {
                out_means[c * cap + o] = (oi * means[c * n + i] + oj * means[c * n + j]) / w;
                out_ls[c * cap + o] = log(0.5 * (exp((double)ls[c * n + i]) + exp((double)ls[c * n + j])));
            }
            int64_t qsrc = oj > oi ? j : i;
            for (int c = 0; c < 4; ++c) out_q[c * cap + o] = quats[c * n + qsrc];
            double om = oi + oj - oi * oj;
            out_logit[o] = log(om) + dc_softplus(logits[i]) + dc_softplus(logits[j]);
            for (int c = 0; c < 3 * nc; ++c)
                out_sh[(int64_t)c * cap + o] = (oi * sh[(int64_t)c * n + i] + oj * sh[(int64_t)c * n + j]) / w;
        }
        ++o;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (cls[i] != 1) continue;
        float t = a * dbar[i];
        for (int c = 0; c < 3; ++c) {
            float p = means[c * n + i] + t * noise[c * n + i];
            p = p + delta * noise[(3 + c) * n + i];
            out_means[c * cap + o] = p;
            out_ls[c * cap + o] = ls[c * n + i];
        }
        for (int c = 0; c < 4; ++c) out_q[c * cap + o] = quats[c * n + i];
        out_logit[o] = logits[i];
        for (int c = 0; c < 3 * nc; ++c) out_sh[(int64_t)c * cap + o] = sh[(int64_t)c * n + i];
        ++o;
    }
    stats[0] = mu; stats[1] = sigma; stats[2] = lo; stats[3] = hi;
    stats[4] = mu_d; stats[5] = sigma_d; stats[6] = dmerge; stats[7] = (double)o;
    free(q); free(ki); free(kd); free(dnn); free(partner);
    return 0;
}
