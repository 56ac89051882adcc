// tno_refit.hip -- per-pixel background re-fit that produces the residual
// stack and noise map of the matched-filter search (arXiv:2209.09848,
// Sec. 3.1 eq. 1-3 and Sec. 3.2).
//
// Pipeline (one stream, FP64 arithmetic):
//   k_gram         one block: basis rows x_t = (1, tx, ty, tx^2, ty^2, tx ty),
//                  the shared Gram matrix G = X^T X, its inverse, and the
//                  projection rows p_t = G^-1 x_t (so beta = sum_t p_t y_t)
//   k_refit_fit    one thread per pixel: y_t = D_t - U(S_t) streamed from HBM,
//                  least-squares start, then rounds beta += sum_t p_t clip(r_t)
//                  (the least-squares fit to X beta + clip(r) in one pass)
//   k_refit_sigma  one pass per estimate of the common sigma: sums of r^2
//                  and counts over unmasked samples within kappa * previous
//   k_refit_write  residual stack (0 at masked pixels and clipped samples),
//                  sigma map, clip and mask counts
// Every reduction runs in a fixed order (block tree, then one block over the
// block partials), so results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cmath>

#include "tno_internal.h"
#include "../../include/tno_search.h"

namespace tno {
namespace {

constexpr int NB = 6;        // basis functions
constexpr int RB = 256;      // threads per block of the per-pixel kernels
constexpr int FB = 1024;     // threads of the final reductions

typedef __attribute__((address_space(4))) double cdouble_t;   // constant address space
// Word 3 of a raw (unformatted, stride 0) buffer resource on gfx9-family GPUs.
constexpr int BUF_DWORD3 = 0x00020000;

// ------------------------------------------------------------------ k_gram

// One block.  err |= 1: a jitter value is not finite; err |= 2: the basis does
// not have full rank (a Gauss-Jordan pivot below 1e-12 of the largest diagonal
// entry of G).
__global__ __launch_bounds__(RB) void k_gram(int T, const double *__restrict__ jit,
                                            double *__restrict__ X, double *__restrict__ P,
                                            int32_t *__restrict__ err)
{
    __shared__ double red[RB];
    __shared__ double G[NB][2 * NB];
    const int tid = threadIdx.x;
    // basis rows, and this thread's share of the 21 distinct Gram entries
    double g[21];
    for (int e = 0; e < 21; ++e)
        g[e] = 0.0;
    int bad = 0;
    for (int t = tid; t < T; t += RB) {
        const double tx = jit[2 * t], ty = jit[2 * t + 1];
        if (!isfinite(tx) || !isfinite(ty))
            bad = 1;
        const double x[NB] = {1.0, tx, ty, tx * tx, ty * ty, tx * ty};
        int e = 0;
        for (int i = 0; i < NB; ++i) {
            X[(size_t)t * NB + i] = x[i];
            for (int j = i; j < NB; ++j)
                g[e++] += x[i] * x[j];
        }
    }
    if (bad)
        atomicOr(err, 1);
    // tree reductions, one entry at a time
    int e = 0;
    for (int i = 0; i < NB; ++i)
        for (int j = i; j < NB; ++j, ++e) {
            red[tid] = g[e];
            __syncthreads();
            for (int s = RB / 2; s > 0; s >>= 1) {
                if (tid < s)
                    red[tid] += red[tid + s];
                __syncthreads();
            }
            if (tid == 0) {
                G[i][j] = red[0];
                G[j][i] = red[0];
            }
            __syncthreads();
        }
    if (tid == 0) {
        // Gauss-Jordan on [G | I] with partial pivoting
        double dmax = 0.0;
        for (int i = 0; i < NB; ++i) {
            dmax = fmax(dmax, fabs(G[i][i]));
            for (int j = 0; j < NB; ++j)
                G[i][NB + j] = (i == j) ? 1.0 : 0.0;
        }
        bool singular = !(dmax > 0.0);
        for (int c = 0; c < NB && !singular; ++c) {
            int piv = c;
            for (int r = c + 1; r < NB; ++r)
                if (fabs(G[r][c]) > fabs(G[piv][c]))
                    piv = r;
            if (!(fabs(G[piv][c]) > 1e-12 * dmax)) {
                singular = true;
                break;
            }
            if (piv != c)
                for (int j = 0; j < 2 * NB; ++j) {
                    double tmp = G[c][j];
                    G[c][j] = G[piv][j];
                    G[piv][j] = tmp;
                }
            const double inv = 1.0 / G[c][c];
            for (int j = 0; j < 2 * NB; ++j)
                G[c][j] *= inv;
            for (int r = 0; r < NB; ++r)
                if (r != c) {
                    const double f = G[r][c];
                    for (int j = 0; j < 2 * NB; ++j)
                        G[r][j] -= f * G[c][j];
                }
        }
        if (singular)
            atomicOr(err, 2);
    }
    __syncthreads();
    // projection rows p_t = G^-1 x_t
    for (int t = tid; t < T; t += RB) {
        const double *x = X + (size_t)t * NB;
        for (int m = 0; m < NB; ++m) {
            double s = 0.0;
            for (int n = 0; n < NB; ++n)
                s += G[m][NB + n] * x[n];
            P[(size_t)t * NB + m] = s;
        }
    }
}

// ------------------------------------------------------------------ per-pixel passes

struct PixelArgs {
    int H, W, T, ny, nx;           // ny == 0: no scattered-light term
    const float *D;                // [T][H][W]
    const float *S;                // [T][ny][nx]
    const double *X, *P;           // [T][6]
    double *beta;                  // [6][H][W]
};

// Bilinear read positions of output index i along one axis (grid cells tile
// the axis; positions beyond the outermost grid points take the edge value).
__device__ void axis_weights(int n_in, int n_out, int i, int &i0, int &i1, double &w0, double &w1)
{
    double src = ((double)i + 0.5) * ((double)n_in / (double)n_out) - 0.5;
    src = fmax(src, 0.0);
    i0 = min((int)floor(src), n_in - 1);
    i1 = min(i0 + 1, n_in - 1);
    w1 = (i1 == i0) ? 0.0 : src - (double)i0;
    w0 = 1.0 - w1;
}

// y_t = D_t - U(S_t) at one pixel.  Frame bases are wave-uniform (scalar
// registers); each lane adds 32-bit element offsets.
struct PixelData {
    const float *D, *S;
    size_t hw, snn;
    uint32_t p;                    // pixel index y*W + x
    uint32_t o00, o01, o10, o11;   // grid offsets of the four scattered-light points
    double wy0, wy1, wx0, wx1;
};

__device__ PixelData pixel_data(const PixelArgs &a, int p)
{
    PixelData q;
    const int yy = p / a.W, xx = p - yy * a.W;
    q.D = a.D;
    q.S = a.S;
    q.hw = (size_t)a.H * a.W;
    q.snn = (size_t)a.ny * a.nx;
    q.p = (uint32_t)p;
    q.o00 = q.o01 = q.o10 = q.o11 = 0;
    q.wy0 = q.wy1 = q.wx0 = q.wx1 = 0.0;
    if (a.ny > 0) {
        int y0, y1, x0, x1;
        axis_weights(a.ny, a.H, yy, y0, y1, q.wy0, q.wy1);
        axis_weights(a.nx, a.W, xx, x0, x1, q.wx0, q.wx1);
        q.o00 = (uint32_t)(y0 * a.nx + x0);
        q.o01 = (uint32_t)(y0 * a.nx + x1);
        q.o10 = (uint32_t)(y1 * a.nx + x0);
        q.o11 = (uint32_t)(y1 * a.nx + x1);
    }
    return q;
}

// Calls f(t, y_t) for t = 0..T-1 in order.  The frames are read in groups of
// YG, every load of a group issued before any is used, so that each thread
// keeps several HBM reads in flight.  SL: with the scattered-light term.
constexpr int YG = 8;
template <bool SL, class F>
__device__ __forceinline__ void for_each_y(const PixelData &q, int T, F &&f)
{
    auto y_of = [&](float d, float a, float b, float c, float e) -> double {
        double v = (double)d;
        if constexpr (SL) {
            const double top = (double)a * q.wx0 + (double)b * q.wx1;
            const double bot = (double)c * q.wx0 + (double)e * q.wx1;
            v -= top * q.wy0 + bot * q.wy1;
        }
        return v;
    };
    // buffer loads (raw 32-bit words, reinterpreted as float): a per-frame
    // resource (scalar) plus the lane's byte offset, which stays below 2^32
    // (H*W <= 2^30)
    auto load = [&](int t, float &d, float &a, float &b, float &c, float &e) {
        const __amdgpu_buffer_rsrc_t rd =
            __builtin_amdgcn_make_buffer_rsrc((void *)(q.D + (size_t)t * q.hw), (short)0, -1, BUF_DWORD3);
        d = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rd, q.p * 4u, 0, 0));
        if constexpr (SL) {
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void *)(q.S + (size_t)t * q.snn), (short)0, -1, BUF_DWORD3);
            a = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, q.o00 * 4u, 0, 0));
            b = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, q.o01 * 4u, 0, 0));
            c = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, q.o10 * 4u, 0, 0));
            e = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, q.o11 * 4u, 0, 0));
        }
    };
    int t = 0;
    for (; t + YG <= T; t += YG) {
        float dv[YG], s0[YG], s1[YG], s2[YG], s3[YG];
#pragma unroll
        for (int u = 0; u < YG; ++u)
            load(t + u, dv[u], s0[u], s1[u], s2[u], s3[u]);
#pragma unroll
        for (int u = 0; u < YG; ++u)
            f(t + u, y_of(dv[u], s0[u], s1[u], s2[u], s3[u]));
    }
    for (; t < T; ++t) {
        float d, a = 0.f, b = 0.f, c = 0.f, e = 0.f;
        load(t, d, a, b, c, e);
        f(t, y_of(d, a, b, c, e));
    }
}

__device__ double residual(const cdouble_t *x, const double (&b)[NB], double y)
{
    double fit = 0.0;
#pragma unroll
    for (int m = 0; m < NB; ++m)
        fit += x[m] * b[m];
    return y - fit;
}

// Least-squares start and `iters` clip-and-solve rounds; beta to HBM.
template <bool SL>
__global__ __launch_bounds__(RB) void k_refit_fit(PixelArgs a, double delta, int iters)
{
    const int p = blockIdx.x * RB + threadIdx.x;
    if (p >= a.H * a.W)
        return;
    const PixelData q = pixel_data(a, p);
    const cdouble_t *Xc = (const cdouble_t *)a.X;
    const cdouble_t *Pc = (const cdouble_t *)a.P;
    double b[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m)
        b[m] = 0.0;
    for_each_y<SL>(q, a.T, [&](int t, double y) {
        const cdouble_t *pt = Pc + (size_t)t * NB;
#pragma unroll
        for (int m = 0; m < NB; ++m)
            b[m] += pt[m] * y;
    });
    for (int it = 0; it < iters; ++it) {
        double acc[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m)
            acc[m] = 0.0;
        for_each_y<SL>(q, a.T, [&](int t, double y) {
            const double r = residual(Xc + (size_t)t * NB, b, y);
            const double c = fmin(fmax(r, -delta), delta);
            const cdouble_t *pt = Pc + (size_t)t * NB;
#pragma unroll
            for (int m = 0; m < NB; ++m)
                acc[m] += pt[m] * c;
        });
#pragma unroll
        for (int m = 0; m < NB; ++m)
            b[m] += acc[m];
    }
    const size_t HW = (size_t)a.H * a.W;
#pragma unroll
    for (int m = 0; m < NB; ++m)
        a.beta[(size_t)m * HW + p] = b[m];
}

__device__ void load_beta(const PixelArgs &a, int p, double (&b)[NB])
{
    const size_t HW = (size_t)a.H * a.W;
#pragma unroll
    for (int m = 0; m < NB; ++m)
        b[m] = a.beta[(size_t)m * HW + p];
}

// Block sums of (value, count) into partial[blockIdx] (fixed-order tree).
__device__ void block_sum2(double v, double c, double2 *partial)
{
    __shared__ double rv[RB], rc[RB];
    const int tid = threadIdx.x;
    rv[tid] = v;
    rc[tid] = c;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (tid < s) {
            rv[tid] += rv[tid + s];
            rc[tid] += rc[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0)
        partial[blockIdx.x] = make_double2(rv[0], rc[0]);
}

// One sigma estimate: sums of r^2 and counts over unmasked pixels' samples
// with |r| <= kappa * sig[round - 1] (every sample in round 0).
template <bool SL>
__global__ __launch_bounds__(RB) void k_refit_sigma(PixelArgs a, double bright, double kappa,
                                                   const double *__restrict__ sig, int round,
                                                   double2 *__restrict__ partial)
{
    const int p = blockIdx.x * RB + threadIdx.x;
    double s = 0.0, c = 0.0;
    if (p < a.H * a.W) {
        double b[NB];
        load_beta(a, p, b);
        if (!(b[0] > bright)) {
            const PixelData q = pixel_data(a, p);
            const cdouble_t *Xc = (const cdouble_t *)a.X;
            const double lim = round == 0 ? INFINITY : kappa * sig[round - 1];
            for_each_y<SL>(q, a.T, [&](int t, double y) {
                const double r = residual(Xc + (size_t)t * NB, b, y);
                if (fabs(r) <= lim) {
                    s += r * r;
                    c += 1.0;
                }
            });
        }
    }
    block_sum2(s, c, partial);
}

// sig[round] = sqrt(sum / count) over the block partials (0 if no samples).
__global__ __launch_bounds__(FB) void k_sigma_final(const double2 *__restrict__ partial, int n,
                                                   double *__restrict__ sig, int round)
{
    __shared__ double rv[FB], rc[FB];
    const int tid = threadIdx.x;
    double v = 0.0, c = 0.0;
    for (int i = tid; i < n; i += FB) {
        v += partial[i].x;
        c += partial[i].y;
    }
    rv[tid] = v;
    rc[tid] = c;
    __syncthreads();
    for (int s = FB / 2; s > 0; s >>= 1) {
        if (tid < s) {
            rv[tid] += rv[tid + s];
            rc[tid] += rc[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0)
        sig[round] = rc[0] > 0.0 ? sqrt(rv[0] / rc[0]) : 0.0;
}

// Residual stack, sigma map and (clipped, masked) counts per block.
template <bool SL>
__global__ __launch_bounds__(RB) void k_refit_write(PixelArgs a, double bright, double kappa,
                                                   const double *__restrict__ sig, int round,
                                                   float *__restrict__ R, float *__restrict__ sigma_map,
                                                   double2 *__restrict__ partial)
{
    const int p = blockIdx.x * RB + threadIdx.x;
    double nclip = 0.0, nmask = 0.0;
    if (p < a.H * a.W) {
        double b[NB];
        load_beta(a, p, b);
        const double s0 = sig[round];
        const size_t HW = (size_t)a.H * a.W;
        const bool masked = b[0] > bright;
        sigma_map[p] = masked ? 0.0f : (float)s0;
        if (masked) {
            nmask = 1.0;
            for (int t = 0; t < a.T; ++t)
                R[(size_t)t * HW + p] = 0.0f;
        } else {
            const PixelData q = pixel_data(a, p);
            const cdouble_t *Xc = (const cdouble_t *)a.X;
            const double lim = kappa * s0;
            for_each_y<SL>(q, a.T, [&](int t, double y) {
                const double r = residual(Xc + (size_t)t * NB, b, y);
                const bool big = fabs(r) > lim;
                nclip += big ? 1.0 : 0.0;
                R[(size_t)t * HW + p] = big ? 0.0f : (float)r;
            });
        }
    }
    block_sum2(nclip, nmask, partial);
}

// (sum of x, sum of y) over the block partials into out[0], out[1].
__global__ __launch_bounds__(FB) void k_count_final(const double2 *__restrict__ partial, int n,
                                                   double *__restrict__ out)
{
    __shared__ double rv[FB], rc[FB];
    const int tid = threadIdx.x;
    double v = 0.0, c = 0.0;
    for (int i = tid; i < n; i += FB) {
        v += partial[i].x;
        c += partial[i].y;
    }
    rv[tid] = v;
    rc[tid] = c;
    __syncthreads();
    for (int s = FB / 2; s > 0; s >>= 1) {
        if (tid < s) {
            rv[tid] += rv[tid + s];
            rc[tid] += rc[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = rv[0];
        out[1] = rc[0];
    }
}

int refuse(int code, const char *msg)
{
    record_error("tno_refit: %s", msg);
    return code;
}

}  // namespace
}  // namespace tno

extern "C" int tno_refit(const tno_refit_request *req, tno_refit_outputs *out, void *stream)
{
    using namespace tno;
    if (!req || !out)
        return refuse(TNO_E_INVAL, "request or outputs is NULL");
    const tno_refit_request &r = *req;
    if (r.flags != 0 || r.reserved != 0)
        return refuse(TNO_E_INVAL, "flags and reserved must be 0");
    if (r.height <= 0 || r.width <= 0 || r.height > 32768 || r.width > 32768)
        return refuse(TNO_E_INVAL, "height and width must be in 1..32768");
    if ((int64_t)r.height * r.width > 1073741824LL)
        return refuse(TNO_E_INVAL, "height*width must be <= 2^30");
    if (r.n_frames < NB || r.n_frames > 65535)
        return refuse(TNO_E_INVAL, "n_frames must be in 6..65535");
    if (!r.data || !r.jitter || !out->residuals || !out->sigma)
        return refuse(TNO_E_INVAL, "data, jitter, residuals and sigma must be non-NULL");
    if (r.scattered && (r.sl_height < 1 || r.sl_width < 1 || r.sl_height > 32768 || r.sl_width > 32768))
        return refuse(TNO_E_INVAL, "scattered-light grid must be 1..32768 on each side");
    if (!(r.delta > 0.0))
        return refuse(TNO_E_INVAL, "delta must be > 0");
    if (std::isnan(r.bright_threshold))
        return refuse(TNO_E_INVAL, "bright_threshold must not be NaN");
    if (!(r.clip_sigma > 0.0))
        return refuse(TNO_E_INVAL, "clip_sigma must be > 0");
    if (r.iterations < 0 || r.iterations > 1000)
        return refuse(TNO_E_INVAL, "iterations must be in 0..1000");
    if (r.sigma_rounds < 0 || r.sigma_rounds > 100)
        return refuse(TNO_E_INVAL, "sigma_rounds must be in 0..100");

    hipStream_t st = (hipStream_t)stream;
    const int T = r.n_frames, H = r.height, W = r.width;
    const size_t HW = (size_t)H * W;
    const int nblk = (int)((HW + RB - 1) / RB);
    const int nsig = r.sigma_rounds + 1;
    // scratch: X, P, err, sigma estimates, counts, partials, beta (unless the caller's)
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = (off + bytes + 255) / 256 * 256;
        return at;
    };
    const size_t oX = take((size_t)T * NB * 8), oP = take((size_t)T * NB * 8), oErr = take(4),
                 oSig = take((size_t)nsig * 8), oCnt = take(16), oPart = take((size_t)nblk * 16),
                 oBeta = out->coeffs ? 0 : take((size_t)NB * HW * 8);
    char *scratch = nullptr;
    hipError_t e = hipMalloc((void **)&scratch, off);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        record_error("tno_refit: device allocation of %zu bytes failed", off);
        return TNO_E_NOMEM;
    }
    double *X = (double *)(scratch + oX), *P = (double *)(scratch + oP);
    int32_t *err = (int32_t *)(scratch + oErr);
    double *sig = (double *)(scratch + oSig), *cnt = (double *)(scratch + oCnt);
    double2 *part = (double2 *)(scratch + oPart);
    PixelArgs a;
    a.H = H;
    a.W = W;
    a.T = T;
    a.ny = r.scattered ? r.sl_height : 0;
    a.nx = r.scattered ? r.sl_width : 0;
    a.D = r.data;
    a.S = r.scattered;
    a.X = X;
    a.P = P;
    a.beta = out->coeffs ? out->coeffs : (double *)(scratch + oBeta);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int32_t herr = 0;
    double hsig = 0.0, hcnt[2] = {0.0, 0.0};
    float ms = 0.0f;
    auto run = [&]() -> hipError_t {
        hipError_t x;
        if ((x = hipEventCreate(&ev0)) != hipSuccess || (x = hipEventCreate(&ev1)) != hipSuccess)
            return x;
        if ((x = hipEventRecord(ev0, st)) != hipSuccess)
            return x;
        if ((x = launch_zero(st, err, 1)) != hipSuccess)
            return x;
        const bool sl = a.ny > 0;
        hipLaunchKernelGGL(k_gram, dim3(1), dim3(RB), 0, st, T, r.jitter, X, P, err);
        if (sl)
            hipLaunchKernelGGL(k_refit_fit<true>, dim3(nblk), dim3(RB), 0, st, a, r.delta, r.iterations);
        else
            hipLaunchKernelGGL(k_refit_fit<false>, dim3(nblk), dim3(RB), 0, st, a, r.delta, r.iterations);
        for (int k = 0; k < nsig; ++k) {
            if (sl)
                hipLaunchKernelGGL(k_refit_sigma<true>, dim3(nblk), dim3(RB), 0, st, a, r.bright_threshold,
                                   r.clip_sigma, (const double *)sig, k, part);
            else
                hipLaunchKernelGGL(k_refit_sigma<false>, dim3(nblk), dim3(RB), 0, st, a, r.bright_threshold,
                                   r.clip_sigma, (const double *)sig, k, part);
            hipLaunchKernelGGL(k_sigma_final, dim3(1), dim3(FB), 0, st, (const double2 *)part, nblk, sig, k);
        }
        if (sl)
            hipLaunchKernelGGL(k_refit_write<true>, dim3(nblk), dim3(RB), 0, st, a, r.bright_threshold,
                               r.clip_sigma, (const double *)sig, nsig - 1, out->residuals, out->sigma, part);
        else
            hipLaunchKernelGGL(k_refit_write<false>, dim3(nblk), dim3(RB), 0, st, a, r.bright_threshold,
                               r.clip_sigma, (const double *)sig, nsig - 1, out->residuals, out->sigma, part);
        hipLaunchKernelGGL(k_count_final, dim3(1), dim3(FB), 0, st, (const double2 *)part, nblk, cnt);
        if ((x = hipGetLastError()) != hipSuccess || (x = hipEventRecord(ev1, st)) != hipSuccess)
            return x;
        if ((x = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (x = hipMemcpyAsync(&hsig, sig + (nsig - 1), 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (x = hipMemcpyAsync(hcnt, cnt, 16, hipMemcpyDeviceToHost, st)) != hipSuccess)
            return x;
        if ((x = hipStreamSynchronize(st)) != hipSuccess)
            return x;
        return hipEventElapsedTime(&ms, ev0, ev1);
    };
    e = run();
    (void)hipStreamSynchronize(st);
    if (ev0)
        (void)hipEventDestroy(ev0);
    if (ev1)
        (void)hipEventDestroy(ev1);
    (void)hipFree(scratch);
    if (e != hipSuccess) {
        record_error("tno_refit: %s", hipGetErrorString(e));
        return TNO_E_DEVICE;
    }
    if (herr & 1)
        return refuse(TNO_E_INVAL, "jitter has a non-finite value");
    if (herr & 2)
        return refuse(TNO_E_INVAL, "the jitter basis is singular (degenerate jitter series)");
    out->sigma0 = hsig;
    out->n_clipped = (int64_t)hcnt[0];
    out->n_masked = (int64_t)hcnt[1];
    out->device_ms = ms;
    return TNO_OK;
}
