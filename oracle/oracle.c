/*
 * oracle.c -- plain FP64 CPU oracle of the matched-filter trajectory search
 * (Ganapathi, "Maximum Likelihood Systematic Effect Modeling and Matched
 * Filtering to Detect Trans-Neptunian Objects with TESS", arXiv:2209.09848).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (Sec. 3.2, eq. 4, and Sec. 3.3):
 *   The matched filter for one constant-velocity trajectory is the trajectory
 *   line convolved with the pixel response function (Sec. 3.2); applying it
 *   is the dot product of filter and data at every start pixel (eq. 4), and
 *   the result estimates the object's flux (Sec. 3.2).  With a per-pixel
 *   Gaussian noise sigma (Sec. 3.2 noise model) the maximum-likelihood form
 *   weights each residual by its inverse variance:
 *
 *     ivar(y,x)   = 1/sigma(y,x)^2 if sigma finite and > 0, else 0
 *                   (masked / clipped pixels, Sec. 3.2), 0 off the image
 *     D_k         = v * (t_k - t_ref) + theta_k           (per axis, FP64;
 *                   theta_k = pointing jitter of frame k, Sec. 2.1 / 3.1,
 *                   folded into the filter as Sec. 3.2 says; 0 if absent)
 *     i_k         = floor(D_k + 1/2),  f_k = D_k - i_k    (anchor, phase)
 *   Gaussian PRF (separable):
 *     g(b; f)     = exp(-(b - f)^2 / (2 sp^2))            (sampled Gaussian)
 *              or = Phi((b+1/2-f)/sp) - Phi((b-1/2-f)/sp) (pixel-integrated)
 *     ghat        = g / sum_b g                           b = -h..h, S = 2h+1
 *     W_k(a,b)    = ghat(a; f_y,k) * ghat(b; f_x,k)       a = row, b = column
 *   Tabulated PRF (Sec. 2: the PRF gives the share of a point source's
 *   flux that each pixel records; not separable in general):
 *     P(u_y, u_x) = the share recorded by a pixel whose centre lies at offset
 *                   (u_y, u_x) from the source, tabulated on the grid
 *                   u = -(h+1) + i/q, i = 0 .. (S+1)q, and read between grid
 *                   points by bilinear interpolation
 *     W_k(a,b)    = P(a - f_y,k, b - f_x,k)               (used as given)
 *     nu(y0,x0)   = sum_k sum_ab W_k(a,b) R_k(Y,X) ivar(Y,X)
 *     Lam(y0,x0)  = sum_k sum_ab W_k(a,b)^2 ivar(Y,X)
 *                   with Y = y0 + i_y,k + a, X = x0 + i_x,k + b
 *     SNR = nu / sqrt(Lam),  flux = nu / Lam   (both 0 where Lam = 0)
 *
 * Everything is evaluated literally in FP64, in the order written above,
 * with no blocking, fusion or reordering beyond the loop nest.  Compile with
 * -ffp-contract=off so that v*dt + 1/2 is not fused into one rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PRF_SAMPLED 0
#define ORACLE_PRF_INTEGRATED 1
#define ORACLE_PRF_TABLE 2
#define ORACLE_MAX_S 31

/* Standard normal CDF difference Phi(hi) - Phi(lo), with erfc in the tails
 * so that the far taps of wide stamps keep their relative accuracy. */
static double phi_diff(double lo, double hi)
{
    const double r2 = 0.70710678118654752440; /* 1/sqrt(2) */
    if (lo >= 0.0)
        return 0.5 * (erfc(lo * r2) - erfc(hi * r2));
    if (hi <= 0.0)
        return 0.5 * (erfc(-hi * r2) - erfc(-lo * r2));
    return 0.5 * (erf(hi * r2) - erf(lo * r2));
}

/* Integer anchor and sub-pixel phase of displacement v*dt + th (reading:
 * pixel centres sit at integers, the anchor rounds half up, phase in
 * [-1/2, 1/2)). */
void oracle_offset(double v, double dt, double th, int32_t *i_out, double *f_out)
{
    double d = v * dt + th;
    double a = floor(d + 0.5);
    *i_out = (int32_t)a;
    *f_out = d - a;
}

/* Unit-sum 1-D PRF profile at phase f, taps b = -h..h (S = 2h+1). */
void oracle_profile(int kind, double sp, int S, double f, double *g)
{
    int h = S / 2;
    double sum = 0.0;
    for (int b = -h; b <= h; ++b) {
        double v;
        if (kind == ORACLE_PRF_INTEGRATED) {
            v = phi_diff(((double)b - 0.5 - f) / sp, ((double)b + 0.5 - f) / sp);
        } else {
            double u = (double)b - f;
            v = exp(-(u * u) / (2.0 * sp * sp));
        }
        g[b + h] = v;
        sum += v;
    }
    for (int b = 0; b < S; ++b)
        g[b] = g[b] / sum;
}

/* Tabulated PRF at offset (uy, ux) by bilinear interpolation of the grid
 * tab[(S+1)q+1][(S+1)q+1], row-major, rows along y.  For |u| <= h + 1/2 the
 * cell index stays inside the grid. */
static double table_value(const double *tab, int S, int q, double uy, double ux)
{
    const int n = (S + 1) * q + 1;
    const double r = (double)(S / 2 + 1);
    double gy = (uy + r) * (double)q;
    double gx = (ux + r) * (double)q;
    double cy = floor(gy), cx = floor(gx);
    double ty = gy - cy, tx = gx - cx;
    int i = (int)cy, m = (int)cx;
    const double *r0 = tab + (size_t)i * n;
    const double *r1 = r0 + n;
    double top = (1.0 - tx) * r0[m] + tx * r0[m + 1];
    double bot = (1.0 - tx) * r1[m] + tx * r1[m + 1];
    return (1.0 - ty) * top + ty * bot;
}

/* Stamp weights W(a, b) at phase (fy, fx): w[(a+h)*S + (b+h)]. */
void oracle_weights(int kind, double sp, int S, const double *tab, int q, double fy,
                    double fx, double *w)
{
    int h = S / 2;
    if (kind == ORACLE_PRF_TABLE) {
        for (int a = -h; a <= h; ++a)
            for (int b = -h; b <= h; ++b)
                w[(a + h) * S + (b + h)] = table_value(tab, S, q, (double)a - fy, (double)b - fx);
        return;
    }
    double gy[ORACLE_MAX_S], gx[ORACLE_MAX_S];
    oracle_profile(kind, sp, S, fy, gy);
    oracle_profile(kind, sp, S, fx, gx);
    for (int a = 0; a < S; ++a)
        for (int b = 0; b < S; ++b)
            w[a * S + b] = gy[a] * gx[b];
}

/* Offsets and phases of every (trajectory j, frame k):
 * iy, ix [J][T] int32 ; fy, fx [J][T] double.  vel is [J][2] = (vx, vy);
 * jit is [T][2] = (theta_x, theta_y) or NULL. */
void oracle_offsets(int T, const double *times, double t_ref, int J,
                    const double *vel, const double *jit, int32_t *iy, int32_t *ix,
                    double *fy, double *fx)
{
    for (int j = 0; j < J; ++j)
        for (int k = 0; k < T; ++k) {
            double dt = times[k] - t_ref;
            double thx = jit ? jit[2 * k + 0] : 0.0, thy = jit ? jit[2 * k + 1] : 0.0;
            oracle_offset(vel[2 * j + 0], dt, thx, &ix[(size_t)j * T + k], &fx[(size_t)j * T + k]);
            oracle_offset(vel[2 * j + 1], dt, thy, &iy[(size_t)j * T + k], &fy[(size_t)j * T + k]);
        }
}

static int prf_ok(int kind, double sp, int S, const double *tab, int q)
{
    if (S < 1 || S > ORACLE_MAX_S || (S % 2) == 0)
        return 0;
    if (kind == ORACLE_PRF_TABLE)
        return tab != NULL && q >= 1 && q <= 256;
    return (kind == ORACLE_PRF_SAMPLED || kind == ORACLE_PRF_INTEGRATED) && sp > 0.0;
}

static double *make_ivar(int H, int W, const float *sigma)
{
    double *iv = (double *)malloc(sizeof(double) * (size_t)H * W);
    if (!iv)
        return NULL;
    for (size_t p = 0; p < (size_t)H * W; ++p) {
        double s = (double)sigma[p];
        iv[p] = (isfinite(s) && s > 0.0) ? 1.0 / (s * s) : 0.0;
    }
    return iv;
}

/* Full search over the start-pixel rectangle [y_lo,y_hi) x [x_lo,x_hi).
 * R is the residual stack [T][H][W] (FP32, widened on the fly), sigma [H][W].
 * nu, lam are [J][y_hi-y_lo][x_hi-x_lo] FP64.  Returns 0, or -1 on bad
 * arguments / allocation failure. */
int oracle_search(int H, int W, int T, const float *R, const float *sigma,
                  const double *times, double t_ref, int J, const double *vel,
                  const double *jit, int kind, double sp, int S, const double *tab, int q,
                  int y_lo, int y_hi, int x_lo, int x_hi,
                  double *nu, double *lam)
{
    if (H <= 0 || W <= 0 || T <= 0 || J < 0 || !prf_ok(kind, sp, S, tab, q))
        return -1;
    if (y_lo < 0 || y_hi > H || y_lo > y_hi || x_lo < 0 || x_hi > W || x_lo > x_hi)
        return -1;
    const int h = S / 2;
    const int ny = y_hi - y_lo, nx = x_hi - x_lo;
    double *iv = make_ivar(H, W, sigma);
    if (!iv)
        return -1;
    memset(nu, 0, sizeof(double) * (size_t)J * ny * nx);
    memset(lam, 0, sizeof(double) * (size_t)J * ny * nx);

#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < J; ++j) {
        double wt[ORACLE_MAX_S * ORACLE_MAX_S];
        double *nuj = nu + (size_t)j * ny * nx;
        double *lamj = lam + (size_t)j * ny * nx;
        for (int k = 0; k < T; ++k) {
            int32_t iy, ix;
            double fy, fx;
            double dt = times[k] - t_ref;
            double thx = jit ? jit[2 * k + 0] : 0.0, thy = jit ? jit[2 * k + 1] : 0.0;
            oracle_offset(vel[2 * j + 0], dt, thx, &ix, &fx);
            oracle_offset(vel[2 * j + 1], dt, thy, &iy, &fy);
            oracle_weights(kind, sp, S, tab, q, fy, fx, wt);
            const float *Rk = R + (size_t)k * H * W;
            for (int a = -h; a <= h; ++a) {
                for (int y0 = y_lo; y0 < y_hi; ++y0) {
                    long Y = (long)y0 + iy + a;
                    if (Y < 0 || Y >= H)
                        continue;
                    for (int b = -h; b <= h; ++b) {
                        double w = wt[(a + h) * S + (b + h)];
                        double w2 = w * w;
                        for (int x0 = x_lo; x0 < x_hi; ++x0) {
                            long X = (long)x0 + ix + b;
                            if (X < 0 || X >= W)
                                continue;
                            size_t p = (size_t)Y * W + (size_t)X;
                            size_t o = (size_t)(y0 - y_lo) * nx + (size_t)(x0 - x_lo);
                            nuj[o] += w * ((double)Rk[p] * iv[p]);
                            lamj[o] += w2 * iv[p];
                        }
                    }
                }
            }
        }
    }
    free(iv);
    return 0;
}

/* The same sums for an explicit list of n hypotheses (j, y0, x0). */
int oracle_hypotheses(int H, int W, int T, const float *R, const float *sigma,
                      const double *times, double t_ref, int J, const double *vel,
                      const double *jit, int kind, double sp, int S, const double *tab,
                      int q, int n, const int32_t *hj, const int32_t *hy, const int32_t *hx,
                      double *nu, double *lam)
{
    if (H <= 0 || W <= 0 || T <= 0 || !prf_ok(kind, sp, S, tab, q))
        return -1;
    for (int e = 0; e < n; ++e)
        if (hj[e] < 0 || hj[e] >= J || hy[e] < 0 || hy[e] >= H || hx[e] < 0 || hx[e] >= W)
            return -1;
    const int h = S / 2;
#pragma omp parallel for schedule(dynamic, 4)
    for (int e = 0; e < n; ++e) {
        double wt[ORACLE_MAX_S * ORACLE_MAX_S];
        int j = hj[e];
        double snu = 0.0, slam = 0.0;
        for (int k = 0; k < T; ++k) {
            int32_t iy, ix;
            double fy, fx;
            double dt = times[k] - t_ref;
            double thx = jit ? jit[2 * k + 0] : 0.0, thy = jit ? jit[2 * k + 1] : 0.0;
            oracle_offset(vel[2 * j + 0], dt, thx, &ix, &fx);
            oracle_offset(vel[2 * j + 1], dt, thy, &iy, &fy);
            oracle_weights(kind, sp, S, tab, q, fy, fx, wt);
            const float *Rk = R + (size_t)k * H * W;
            for (int a = -h; a <= h; ++a) {
                long Y = (long)hy[e] + iy + a;
                if (Y < 0 || Y >= H)
                    continue;
                for (int b = -h; b <= h; ++b) {
                    long X = (long)hx[e] + ix + b;
                    if (X < 0 || X >= W)
                        continue;
                    size_t p = (size_t)Y * W + (size_t)X;
                    double s = (double)sigma[p];
                    double iv = (isfinite(s) && s > 0.0) ? 1.0 / (s * s) : 0.0;
                    double w = wt[(a + h) * S + (b + h)];
                    snu += w * ((double)Rk[p] * iv);
                    slam += (w * w) * iv;
                }
            }
        }
        nu[e] = snu;
        lam[e] = slam;
    }
    return 0;
}

/* Number of threads OpenMP will use (reported beside the CPU timing). */
int oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing on one core and on all of them). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
