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
 *     D_k         = v * (t_k - t_ref)                     (per axis, FP64)
 *     i_k         = floor(D_k + 1/2),  f_k = D_k - i_k    (anchor, phase)
 *     g(b; f)     = exp(-(b - f)^2 / (2 sp^2))            (sampled Gaussian)
 *              or = Phi((b+1/2-f)/sp) - Phi((b-1/2-f)/sp) (pixel-integrated)
 *     ghat        = g / sum_b g                           b = -h..h, S = 2h+1
 *     W_k(a,b)    = ghat(a; f_y,k) * ghat(b; f_x,k)       a = row, b = column
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

/* Integer anchor and sub-pixel phase of displacement v*dt (reading: pixel
 * centres sit at integers, the anchor rounds half up, phase in [-1/2, 1/2)). */
void oracle_offset(double v, double dt, int32_t *i_out, double *f_out)
{
    double d = v * dt;
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

/* Offsets and phases of every (trajectory j, frame k):
 * iy, ix [J][T] int32 ; fy, fx [J][T] double.  vel is [J][2] = (vx, vy). */
void oracle_offsets(int T, const double *times, double t_ref, int J,
                    const double *vel, int32_t *iy, int32_t *ix,
                    double *fy, double *fx)
{
    for (int j = 0; j < J; ++j)
        for (int k = 0; k < T; ++k) {
            double dt = times[k] - t_ref;
            oracle_offset(vel[2 * j + 0], dt, &ix[(size_t)j * T + k], &fx[(size_t)j * T + k]);
            oracle_offset(vel[2 * j + 1], dt, &iy[(size_t)j * T + k], &fy[(size_t)j * T + k]);
        }
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
                  int kind, double sp, int S,
                  int y_lo, int y_hi, int x_lo, int x_hi,
                  double *nu, double *lam)
{
    if (H <= 0 || W <= 0 || T <= 0 || J < 0 || S < 1 || S > 31 || (S % 2) == 0)
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
        double gy[31], gx[31];
        double *nuj = nu + (size_t)j * ny * nx;
        double *lamj = lam + (size_t)j * ny * nx;
        for (int k = 0; k < T; ++k) {
            int32_t iy, ix;
            double fy, fx;
            double dt = times[k] - t_ref;
            oracle_offset(vel[2 * j + 0], dt, &ix, &fx);
            oracle_offset(vel[2 * j + 1], dt, &iy, &fy);
            oracle_profile(kind, sp, S, fy, gy);
            oracle_profile(kind, sp, S, fx, gx);
            const float *Rk = R + (size_t)k * H * W;
            for (int a = -h; a <= h; ++a) {
                for (int y0 = y_lo; y0 < y_hi; ++y0) {
                    long Y = (long)y0 + iy + a;
                    if (Y < 0 || Y >= H)
                        continue;
                    for (int b = -h; b <= h; ++b) {
                        double w = gy[a + h] * gx[b + h];
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
                      int kind, double sp, int S, int n,
                      const int32_t *hj, const int32_t *hy, const int32_t *hx,
                      double *nu, double *lam)
{
    if (H <= 0 || W <= 0 || T <= 0 || S < 1 || S > 31 || (S % 2) == 0)
        return -1;
    for (int q = 0; q < n; ++q)
        if (hj[q] < 0 || hj[q] >= J || hy[q] < 0 || hy[q] >= H || hx[q] < 0 || hx[q] >= W)
            return -1;
    const int h = S / 2;
#pragma omp parallel for schedule(dynamic, 4)
    for (int q = 0; q < n; ++q) {
        double gy[31], gx[31];
        int j = hj[q];
        double snu = 0.0, slam = 0.0;
        for (int k = 0; k < T; ++k) {
            int32_t iy, ix;
            double fy, fx;
            double dt = times[k] - t_ref;
            oracle_offset(vel[2 * j + 0], dt, &ix, &fx);
            oracle_offset(vel[2 * j + 1], dt, &iy, &fy);
            oracle_profile(kind, sp, S, fy, gy);
            oracle_profile(kind, sp, S, fx, gx);
            const float *Rk = R + (size_t)k * H * W;
            for (int a = -h; a <= h; ++a) {
                long Y = (long)hy[q] + iy + a;
                if (Y < 0 || Y >= H)
                    continue;
                for (int b = -h; b <= h; ++b) {
                    long X = (long)hx[q] + ix + b;
                    if (X < 0 || X >= W)
                        continue;
                    size_t p = (size_t)Y * W + (size_t)X;
                    double s = (double)sigma[p];
                    double iv = (isfinite(s) && s > 0.0) ? 1.0 / (s * s) : 0.0;
                    double w = gy[a + h] * gx[b + h];
                    snu += w * ((double)Rk[p] * iv);
                    slam += (w * w) * iv;
                }
            }
        }
        nu[q] = snu;
        lam[q] = slam;
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
