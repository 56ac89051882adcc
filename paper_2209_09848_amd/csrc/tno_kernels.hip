// tno_kernels.hip -- gfx950 kernels of the matched-filter trajectory search
// (arXiv:2209.09848, Sec. 3.2 eq. 4 and Sec. 3.3).
//
// Pipeline of one request (all on one HIP stream):
//   k_ivar      ivar = 1/sigma^2 (FP64, also rounded to FP32); 0 for masked pixels
//   k_prep_z    Z = decode(R) * ivar into a zero-padded FP32 stack (float4 rows)
//   k_table     per (trajectory, frame): FP64 anchor/phase (pointing jitter
//               included) and the stamp weights (Gaussian profiles or the
//               tabulated PRF read at the phase)
//   k_trail     per trajectory: collapsed trail kernel K_j(q) = sum_k W_jk^2 at q (FP64)
//   k_lambda    Lam_j = ivar (x) K_j, a sparse FP64 correlation
//   k_search    nu_j = sum_k W_jk (x) Z_k at the frame's shift; LDS-staged window,
//               separable (2S taps) or general (S*S taps) stamp, FP32 frame
//               chunks into FP64 totals; epilogue
//               SNR = nu/sqrt(Lam), flux = nu/Lam, per-tile maximum key
//   k_trajmax / k_best / top-k   the reductions of Sec. 3.2-3.3
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <limits.h>
#include <type_traits>
#include <algorithm>

#include "tno_internal.h"
#include "tno_device.h"
#include "../../include/tno_search.h"

namespace tno {

// ------------------------------------------------------------------ helpers

// ------------------------------------------------------------------ k_zero

// Clears small device counters with a kernel (no memset nodes in the stream).
__global__ void k_zero(int32_t *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_zero(hipStream_t st, int32_t *p, int n)
{
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_ivar

__global__ void k_ivar(int W, const float *__restrict__ sigma, float *__restrict__ ivar32,
                       double *__restrict__ ivar64, int64_t HWq, int Wq, int H, int Pyt, int Pxl, int tr,
                       int32_t *__restrict__ err)
{
    // one thread per element of the zero-bordered FP64 map; with tr its rows
    // are the image's columns
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < HWq; q += (int64_t)gridDim.x * blockDim.x) {
        const int yq = (int)(q / Wq), xq = (int)(q - (int64_t)yq * Wq);
        const int y = tr ? xq - Pxl : yq - Pyt, x = tr ? yq - Pyt : xq - Pxl;
        double iv = 0.0;
        if ((unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W) {
            const size_t p = (size_t)y * W + x;
            const double s = (double)sigma[p];
            iv = (__builtin_isfinite(s) && s > 0.0) ? 1.0 / (s * s) : 0.0;
            if (ivar32) {
                const float iv32 = (float)iv;
                if (!__builtin_isfinite(iv32))
                    atomicOr(err, 2);     // 1/sigma^2 beyond single precision: rejected
                ivar32[p] = iv32;
            }
        }
        ivar64[q] = iv;
    }
}

hipError_t launch_ivar(hipStream_t st, int H, int W, const float *sigma, float *ivar32, double *ivar64,
                       int Hq, int Wq, int Pyt, int Pxl, int tr, int32_t *err)
{
    const int64_t n = (int64_t)Hq * Wq;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_ivar, dim3((unsigned)blocks), dim3(256), 0, st, W, sigma, ivar32, ivar64, n, Wq, H,
                       Pyt, Pxl, tr, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------ decode + k_prep_z


template <int DT>
__device__ __forceinline__ float load_residual(const void *R, const float *scales, size_t idx,
                                               int k, int y, int x, int nqy, int nqx)
{
    if constexpr (DT == TNO_F32) {
        return ((const float *)R)[idx];
    } else {
        float s = scales[((size_t)k * nqy + (y >> 6)) * nqx + (x >> 6)];
        if constexpr (DT == TNO_BF16) {
            uint32_t b = ((const uint16_t *)R)[idx];
            return __uint_as_float(b << 16) * s;
        } else if constexpr (DT == TNO_F16) {
            _Float16 hv = ((const _Float16 *)R)[idx];
            return (float)hv * s;
        } else {
            uint32_t c = ((const uint8_t *)R)[idx];
            return decode_e4m3(c) * (s * 256.0f);
        }
    }
}

// One thread per float4 group of the padded stack; grid (groups/256, Hp, T).
// A group holds image columns 4g..4g+3 in the order (4g, 4g+2, 4g+1, 4g+3):
// even columns first, so that k_search can stage a row's even and odd columns
// into separate halves with whole 8-byte stores.
template <int DT>
__global__ void k_prep_z(const void *__restrict__ R, const float *__restrict__ scales,
                         const float *__restrict__ ivar32, float4 *__restrict__ Z4, int H, int W,
                         int Hp, int Wp4, int Pt, int Pl)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Wp4)
        return;
    int yp = blockIdx.y;
    int k = blockIdx.z;
    int y = yp - Pt;
    int nqy = (H + TNO_QTILE - 1) / TNO_QTILE, nqx = (W + TNO_QTILE - 1) / TNO_QTILE;
    const int x0 = 4 * g - Pl;        // Pl is a multiple of 4
    float v[4];
    if ((W & 3) == 0 && y >= 0 && y < H && x0 >= 0 && x0 + 3 < W) {
        // whole group inside the image and 4-aligned: vector loads
        const size_t p = (size_t)y * W + x0;
        const size_t i = (size_t)k * H * W + p;
        const float4 iv = *reinterpret_cast<const float4 *>(ivar32 + p);
        float r[4];
        if constexpr (DT == TNO_F32) {
            const float4 rv = *reinterpret_cast<const float4 *>((const float *)R + i);
            r[0] = rv.x; r[1] = rv.y; r[2] = rv.z; r[3] = rv.w;
        } else {
            const float s = scales[((size_t)k * nqy + (y >> 6)) * nqx + (x0 >> 6)];
            if constexpr (DT == TNO_FP8_E4M3) {
                const uint32_t c4 = *reinterpret_cast<const uint32_t *>((const uint8_t *)R + i);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    r[e] = decode_e4m3((c4 >> (8 * e)) & 0xFFu) * (s * 256.0f);
            } else {
                const uint2 c2 = *reinterpret_cast<const uint2 *>((const uint16_t *)R + i);
                const uint32_t c[4] = {c2.x & 0xFFFFu, c2.x >> 16, c2.y & 0xFFFFu, c2.y >> 16};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if constexpr (DT == TNO_BF16) {
                        r[e] = __uint_as_float(c[e] << 16) * s;
                    } else {
                        uint16_t hb = (uint16_t)c[e];
                        _Float16 hv;
                        __builtin_memcpy(&hv, &hb, 2);
                        r[e] = (float)hv * s;
                    }
                }
            }
        }
        Z4[((size_t)k * Hp + yp) * Wp4 + g] = make_float4(r[0] * iv.x, r[2] * iv.z, r[1] * iv.y, r[3] * iv.w);
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        int x = 4 * g + e - Pl;
        v[e] = 0.0f;
        if (y >= 0 && y < H && x >= 0 && x < W) {
            size_t p = (size_t)y * W + x;
            float r = load_residual<DT>(R, scales, (size_t)k * H * W + p, k, y, x, nqy, nqx);
            v[e] = r * ivar32[p];
        }
    }
    Z4[((size_t)k * Hp + yp) * Wp4 + g] = make_float4(v[0], v[2], v[1], v[3]);
}

hipError_t launch_prep_z(hipStream_t st, int dtype, const void *R, const float *scales,
                         const float *ivar32, float4 *Z4, int T, int H, int W, int Hp, int Wp4,
                         int Pt, int Pl)
{
    dim3 grid((Wp4 + 255) / 256, Hp, T);
    switch (dtype) {
    case TNO_F32:
        hipLaunchKernelGGL(k_prep_z<TNO_F32>, grid, dim3(256), 0, st, R, scales, ivar32, Z4, H, W, Hp, Wp4, Pt, Pl);
        break;
    case TNO_BF16:
        hipLaunchKernelGGL(k_prep_z<TNO_BF16>, grid, dim3(256), 0, st, R, scales, ivar32, Z4, H, W, Hp, Wp4, Pt, Pl);
        break;
    case TNO_F16:
        hipLaunchKernelGGL(k_prep_z<TNO_F16>, grid, dim3(256), 0, st, R, scales, ivar32, Z4, H, W, Hp, Wp4, Pt, Pl);
        break;
    default:
        hipLaunchKernelGGL(k_prep_z<TNO_FP8_E4M3>, grid, dim3(256), 0, st, R, scales, ivar32, Z4, H, W, Hp, Wp4, Pt, Pl);
        break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_table (FP64)

// Phi(hi) - Phi(lo) of the standard normal, using erfc in the tails.
__device__ double normal_mass(double lo, double hi)
{
    const double r2 = 0.70710678118654752440;
    if (lo >= 0.0)
        return 0.5 * (erfc(lo * r2) - erfc(hi * r2));
    if (hi <= 0.0)
        return 0.5 * (erfc(-hi * r2) - erfc(-lo * r2));
    return 0.5 * (erf(hi * r2) - erf(lo * r2));
}

// Unit-sum profile of the Gaussian PRF at phase f over taps -h..h.
__device__ void prf_profile(int kind, double sp, int S, double f, double *g)
{
#pragma clang fp contract(off)
    int h = S / 2;
    double sum = 0.0;
    for (int b = -h; b <= h; ++b) {
        double v;
        if (kind == TNO_PRF_GAUSS_INTEGRATED) {
            v = normal_mass(((double)b - 0.5 - f) / sp, ((double)b + 0.5 - f) / sp);
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

// Tabulated PRF at offset (uy, ux) by bilinear interpolation of the grid
// tab[n][n], n = (S+1)q+1, samples at u = -(h+1) + i/q.  |u| <= h + 1/2 keeps
// the cell inside the grid.
__device__ double prf_table_value(const double *__restrict__ tab, int S, int q, double uy,
                                  double ux)
{
#pragma clang fp contract(off)
    const int n = (S + 1) * q + 1;
    const double r = (double)(S / 2 + 1);
    const double gy = (uy + r) * (double)q, gx = (ux + r) * (double)q;
    const double cy = floor(gy), cx = floor(gx);
    const double ty = gy - cy, tx = gx - cx;
    const int i = min(max((int)cy, 0), n - 2), m = min(max((int)cx, 0), n - 2);
    const double *r0 = tab + (size_t)i * n;
    const double *r1 = r0 + n;
    const double top = (1.0 - tx) * r0[m] + tx * r0[m + 1];
    const double bot = (1.0 - tx) * r1[m] + tx * r1[m + 1];
    return (1.0 - ty) * top + ty * bot;
}

// One thread per (trajectory j, frame k): displacement D = v*dt + theta_k,
// anchor i = floor(D + 1/2) and phase f = D - i per axis in FP64 without
// fused multiply-add (the anchor must flip exactly where the definition
// flips), then the stamp weights: both Gaussian profiles, or the S x S
// tabulated weights P(a - f_y, b - f_x).
__global__ void k_table(int J, int T, const double *__restrict__ times, double t_ref,
                        const double *__restrict__ vel, const double *__restrict__ jitter,
                        PrfSpec prf, int32_t *__restrict__ tab32, double *__restrict__ tab64)
{
#pragma clang fp contract(off)
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= J * T)
        return;
    const int S = prf.S;
    int j = e / T, k = e - j * T;
    double dt = times[k] - t_ref;
    const double thx = jitter ? jitter[2 * k + 0] : 0.0;
    const double thy = jitter ? jitter[2 * k + 1] : 0.0;
    double dx = vel[2 * j + 0] * dt + thx;
    double dy = vel[2 * j + 1] * dt + thy;
    double ax = floor(dx + 0.5), ay = floor(dy + 0.5);
    double fx = dx - ax, fy = dy - ay;
    const bool sep = prf_separable(prf.kind);
    const int TS = table_stride(S, sep);
    const int T64 = table64_stride(S, sep);
    int32_t *t = tab32 + (size_t)e * TS;
    double *t64 = tab64 + (size_t)e * T64;
    t[0] = (int32_t)ay;
    t[1] = (int32_t)ax;
    if (sep) {
        double gy[TNO_MAX_STAMP], gx[TNO_MAX_STAMP];
        prf_profile(prf.kind, prf.sigma_px, S, fy, gy);
        prf_profile(prf.kind, prf.sigma_px, S, fx, gx);
        // FP32 form for the search: the centre column tap (the largest of a
        // unimodal unit-sum profile, so at least 1/S) is moved into the row
        // weights, gy[a] gx[h] and gx[b] / gx[h], so that a horizontal pass
        // starts from the centre value with no multiply; W = gy gx is unchanged
        const int h = S / 2;
        for (int s = 0; s < S; ++s) {
            t[2 + s] = __float_as_int((float)(gy[s] * gx[h]));
            t[2 + S + s] = __float_as_int(s == h ? 1.0f : (float)(gx[s] / gx[h]));
            t64[s] = gy[s];
            t64[S + s] = gx[s];
        }
    } else {
        const int h = S / 2;
        for (int a = 0; a < S; ++a)
            for (int b = 0; b < S; ++b) {
                const double w = prf_table_value(prf.table, S, prf.q, (double)(a - h) - fy,
                                                 (double)(b - h) - fx);
                t[2 + a * S + b] = __float_as_int((float)w);
                t64[a * S + b] = w;
            }
    }
    for (int s = 2 + T64; s < TS; ++s)
        t[s] = 0;
}

hipError_t launch_table(hipStream_t st, int J, int T, const double *times, double t_ref,
                        const double *vel, const double *jitter, const PrfSpec &prf,
                        int32_t *tab32, double *tab64)
{
    int n = J * T;
    hipLaunchKernelGGL(k_table, dim3((n + 127) / 128), dim3(128), 0, st, J, T, times, t_ref, vel,
                       jitter, prf, tab32, tab64);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_trail (FP64)

// One block per trajectory, one thread per major offset of the trail box
// (a column offset qx, or a row offset qy for a box stored transposed).
// K_j(qy, qx) = sum_k W_jk(qy - iy_k, qx - ix_k)^2 over the frames whose
// stamp covers (qy, qx); each major line is one contiguous run along the
// minor axis, summed frame by frame in frame order (deterministic).  W is
// gy*gx for a separable PRF, the tabulated weight otherwise.
__global__ void k_trail(int T, int S, int sep, const int32_t *__restrict__ tab32,
                        const double *__restrict__ tab64, const TrailInfo *__restrict__ info,
                        int2 *__restrict__ colmeta, double *__restrict__ kvals,
                        int32_t *__restrict__ err)
{
    const int j = blockIdx.x;
    const TrailInfo ti = info[j];
    const int h = S / 2;
    const int TS = table_stride(S, sep);
    const int T64 = table64_stride(S, sep);
    const int32_t *tj = tab32 + (size_t)j * T * TS;
    const double *t64 = tab64 + (size_t)j * T * T64;
    // major axis: x (tr = 0) or y (tr = 1); table entries hold (iy, ix)
    const int mj = ti.tr ? 0 : 1, mn = 1 - mj;
    for (int c = threadIdx.x; c < ti.ncols; c += blockDim.x) {
        const int qm = ti.qx0 + c;
        int lo = INT_MAX, hi = INT_MIN;
        for (int k = 0; k < T; ++k) {
            int im = tj[(size_t)k * TS + mj];
            int dmo = qm - im;
            if (dmo >= -h && dmo <= h) {
                int in = tj[(size_t)k * TS + mn];
                lo = min(lo, in - h);
                hi = max(hi, in + h);
            }
        }
        lo = max(lo, ti.qy_lo);
        hi = min(hi, ti.qy_hi);
        int len = hi >= lo ? hi - lo + 1 : 0;
        if (len > ti.cap) {
            atomicOr(err, 1);
            len = 0;
        }
        colmeta[ti.col_off + c] = make_int2(lo, len);
        double *kv = kvals + ti.val_off + (int64_t)c * ti.cap;
        for (int i = 0; i < ti.cap; ++i)   // the zero tail pads runs to whole chunks
            kv[i] = 0.0;
        if (len == 0)
            continue;
        for (int k = 0; k < T; ++k) {
            int im = tj[(size_t)k * TS + mj];
            int dmo = qm - im;
            if (dmo < -h || dmo > h)
                continue;
            int in = tj[(size_t)k * TS + mn];
            const double *wk = t64 + (size_t)k * T64;
            // tap (a along y, b along x) of the stamp: the major tap is fixed
            // (dmo + h), the minor one runs
            if (sep) {
                double wm = ti.tr ? wk[dmo + h] : wk[S + dmo + h];
                double wm2 = wm * wm;
                for (int t = 0; t < S; ++t) {
                    int r = in - h + t - lo;
                    if (r < 0 || r >= len)
                        continue;
                    double wn = ti.tr ? wk[S + t] : wk[t];
                    kv[r] += wm2 * (wn * wn);
                }
            } else {
                for (int t = 0; t < S; ++t) {
                    int r = in - h + t - lo;
                    if (r < 0 || r >= len)
                        continue;
                    double w = ti.tr ? wk[(dmo + h) * S + t] : wk[t * S + dmo + h];
                    kv[r] += w * w;
                }
            }
        }
    }
}

hipError_t launch_trail(hipStream_t st, int J, int T, int S, bool sep, const int32_t *tab32,
                        const double *tab64, const TrailInfo *info, int2 *colmeta,
                        double *kvals, int32_t *err)
{
    hipLaunchKernelGGL(k_trail, dim3(J), dim3(256), 0, st, T, S, (int)sep, tab32, tab64, info,
                       colmeta, kvals, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_lambda (FP64)

// Lam_j(y, x) = sum over trail columns qx, rows qy of K_j(qy, qx) ivar(y+qy, x+qx).
// (Boxes wider than tall run in the transposed image: the same computation
// with rows and columns exchanged, the result written back untransposed.)
// A lane owns one image column x and R = 32 consecutive rows.  Each trail
// column's run is zero-padded to whole chunks of C = LAMBDA_CHUNK values; per
// chunk the C K values are wave-uniform (scalar loads) and a sliding window of
// R + C - 1 ivar values down the image column feeds R C FP64 FMAs, each ivar
// load serving up to R outputs.
// ivar is read from a copy with a zero border wide enough for every read of
// the launch, so no load is clamped or masked: a wave's loads of one chunk are
// buffer loads from a scalar base (the chunk's first row at the wave's first
// column) with the lane's 8-byte column offset and a scalar row offset.
// One launch serves both storage orientations: items below a0.n_items are
// those of a0 (trails stored by columns), the rest those of a1 (by rows).
__global__ __launch_bounds__(256) void k_lambda(LambdaArgs a0, LambdaArgs a1)
{
    constexpr int R = LAMBDA_TY / 4;   // outputs per lane (4 waves stacked)
    constexpr int C = LAMBDA_CHUNK;    // K values per chunk
    int item = xcd_item(blockIdx.x, gridDim.x);
    const bool second = item >= a0.n_items;
    const LambdaArgs &a = second ? a1 : a0;
    if (second)
        item -= a0.n_items;
    if (item >= a.n_items)
        return;
    const int j = a.jlist[item % a.nj];
    const int tile = item / a.nj;
    const int tyi = tile / a.ntx, txi = tile - tyi * a.ntx;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xw = txi * LAMBDA_TX;            // the wave's first column
    const int y0 = tyi * LAMBDA_TY + wv * R;   // the wave's first row
    const int x = xw + lane;
    const TrailInfo ti = a.info[j];
    const uint32_t rowb = (uint32_t)a.Wq * 8u;
    const int voff = lane * 8;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        acc[r] = 0.0;
    for (int c = 0; c < ti.ncols; ++c) {
        const int2 m = a.colmeta[ti.col_off + c];
        const int len = m.y;
        if (len == 0)
            continue;
        // the run's first row for this wave, at the wave's first column
        const double *base = a.ivar64 + (size_t)(a.Pyt + y0 + m.x) * a.Wq + (a.Pxl + xw + ti.qx0 + c);
        auto ld = [&](const __amdgpu_buffer_rsrc_t &rs, int i) -> double {
            const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, (int)(i * rowb), 0);
            return __builtin_bit_cast(double, w);
        };
        const double *kv = a.kvals + ti.val_off + (int64_t)c * ti.cap;
        // the run's rows sit in a circular window, row i in slot i % NS, with
        // the chunk loop unrolled over NS / C chunks so that every slot index
        // is a constant and the window never moves
        constexpr int NS = (R + C - 1 + C - 1) / C * C;
        double v[NS];
        {
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, 0x7FFFFFFF, BUF_DWORD3);
#pragma unroll
            for (int i = 0; i < R - 1; ++i)
                v[i] = ld(rs, i);
        }
        for (int q0 = 0; q0 < len; q0 += NS) {
#pragma unroll
            for (int u = 0; u < NS / C; ++u) {
                const int qq = q0 + u * C;
                if (qq >= len)
                    break;
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(base + (size_t)(qq + R - 1) * a.Wq), (short)0, 0x7FFFFFFF, BUF_DWORD3);
#pragma unroll
                for (int t = 0; t < C; ++t)
                    v[(u * C + R - 1 + t) % NS] = ld(rs, t);
                double kc[C];
#pragma unroll
                for (int t = 0; t < C; ++t)
                    kc[t] = kv[qq + t];
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int t = 0; t < C; ++t)
                        acc[r] = fma(kc[t], v[(u * C + t + r) % NS], acc[r]);
            }
        }
    }
    const int jr = a.jrow[j];   // the trajectory's row of the slab's map
    if (x < a.W) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int y = y0 + r;
            if (y < a.H) {
                // (y, x) of the launch's frame; transposed: image row x, column y
                const size_t o = a.tr ? ((size_t)jr * a.H0 + x) * a.W0 + y : ((size_t)jr * a.H0 + y) * a.W0 + x;
                a.lam[o] = acc[r];
            }
        }
    }
}

hipError_t launch_lambda(hipStream_t st, const LambdaArgs &a0, const LambdaArgs &a1)
{
    const int n = a0.n_items + a1.n_items;
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_lambda, dim3(xcd_grid(n)), dim3(256), 0, st, a0, a1);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_search

// One block = one (tile of (64 CPL) x (RPL NWAVE) start pixels, trajectory);
// a lane owns CPL columns x RPL rows.  Per frame k the block needs the window
// of Z its stamps cover at the frame's integer shift: (TY+S-1) rows x
// (TX+S-1) columns, fetched as aligned float4 groups (buffer loads, the
// sub-float4 offset d applied when reading) and staged de-interleaved into
// LDS.  The window of frame k+1 is fetched into registers before frame k is
// computed and stored into LDS afterwards, so global latency overlaps the
// arithmetic.  SEP: the separable stamp, a horizontal pass of S taps per
// window row streamed into a vertical pass of S taps; otherwise the general
// S x S stamp.  XCH (separable stamps): every horizontal row is computed once
// per block and the S-1 halo rows below each wave's strip come from the wave
// that owns them through a small LDS exchange buffer; the window is single
// buffered and refilled between two barriers per frame.  Otherwise each wave
// computes its own halo rows and a double-buffered window needs one barrier
// per frame.  The table entry (shift, weights) is wave-uniform (scalar loads).
// Frame partials accumulate in FP32 over FRAME_CHUNK frames, then into FP64;
// every form adds the terms of an output in the same order.
// SRC: the window's source, the staged stack Z (SRC_Z) or a reduced-precision
// stack read in place (its dtype): codes, tile scale and ivar are fetched and
// decode x scale x ivar is stored, the very products the staging of Z forms,
// so both sources give the same bits.
template <int S, int NWAVE, int CPL, int RPL, bool SEP, bool XCH, int SRC = SRC_Z>
__device__ __forceinline__ void search_item(const SearchArgs &a, int item)
{
    constexpr int h = S / 2;
    constexpr int NT = 64 * NWAVE;
    constexpr int TX = 64 * CPL, TY = RPL * NWAVE;
    constexpr int WY = TY + S - 1;
    constexpr int NG = (TX + S - 1 + 3 + 3) / 4;
    constexpr int LS = NG * 4;
    constexpr int NWIN = WY * NG;
    constexpr int NLD = (NWIN + NT - 1) / NT;
    constexpr int TS = table_stride(S, SEP);
    constexpr int NW = table64_stride(S, SEP);   // FP32 weights per table entry
    constexpr int NV = CPL + S - 1;
    // XCH: one window buffer plus the exchange rows of the horizontal pass
    // ((NWAVE+1) x (S-1) rows of TX values); otherwise two window buffers
    static_assert(!XCH || (SEP && CPL % 2 == 0 && S > 1 && S - 1 <= RPL),
                  "the exchange form needs a separable stamp wider than 1, even CPL and S-1 <= RPL");
    constexpr int NXR = XCH ? (NWAVE + 1) * (S - 1) : 0;
    __shared__ __align__(16) float win[XCH ? 1 : 2][NWIN * 4];
    __shared__ __align__(16) float xch[XCH ? 2 * NXR * TX : 1];

    // work order: blocks of `tblock` velocity-sorted trajectories; within a
    // block the trajectory index runs fastest, then the tile
    const int ntiles = a.ntx * a.nty;
    const int per_blk = ntiles * a.tblock;
    const int jb = item / per_blk;
    const int rem = item - jb * per_blk;
    const int bcur = min(a.tblock, a.J - jb * a.tblock);
    const int tile = rem / bcur;
    const int j = a.perm[jb * a.tblock + (rem - tile * bcur)];
    const int tyi = tile / a.ntx, txi = tile - tyi * a.ntx;
    const int ty0 = tyi * TY, tx0 = txi * TX;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;

    // This thread's staging slots: window group idx = tid + NT*it at (row r,
    // group g): Z's byte offset (r * Wp4 + g) * 16 from the window origin
    // (below 2^32: WY * Wp4 * 16 is); read in place, the element offset
    // r * W + 4g (every pixel offset fits: H * W * 4 < 2^31)
    uint32_t soff[NLD];
#pragma unroll
    for (int it = 0; it < NLD; ++it) {
        const int idx = tid + NT * it;
        const int r = idx / NG;
        if constexpr (SRC == SRC_Z)
            soff[it] = (uint32_t)(r * a.Wp4 + (idx - r * NG)) * 16u;
        else
            soff[it] = (uint32_t)(r * a.W + 4 * (idx - r * NG));
    }
    // only the last slot can fall past the window; such a lane's buffer
    // offset is set past every resource, so it reads 0 and touches no memory
    const bool last_ok = tid + NT * (NLD - 1) < NWIN;
    if (!last_ok)
        soff[NLD - 1] = 0x80000000u;

    // the table is read-only for the whole launch: read it through the
    // constant address space so its wave-uniform entries stay scalar loads
    const cint32_t *tabj = (const cint32_t *)(a.tab32) + (size_t)j * a.T * TS;
    const size_t frame4 = (size_t)a.Hp * a.Wp4;

    // Fetch the window of frame k into registers; returns its sub-float4 offset.
    // Read in place, ivar is fetched only when the window covers other pixels
    // than at the previous fetch (the slots are not written between the store
    // of one window and the fetch of the next, so they still hold it).
    int f_oy = INT_MIN, f_ox = INT_MIN;
    auto fetch = [&](int k, Raw<SRC> (&pre)[NLD]) -> int {
        k *= a.kstride;
        const cint32_t *e = tabj + (size_t)k * TS;
        if constexpr (SRC != SRC_Z) {
            constexpr int EB = src_bytes<SRC>();
            constexpr uint32_t OOB = 0x80000000u;
            const size_t HW = (size_t)a.H * a.W;
            const int W4 = a.W >> 2;
            const int oy = ty0 + e[0] - h;
            const int ox = tx0 + e[1] - h;
            const int ag = ox >> 2;   // floor
            const bool inside = oy >= 0 && oy + WY <= a.H && ag >= 0 && ag + NG <= W4;
            // resources at the window origin (inside the image) or at the
            // frame start; OOB lies past every resource
            const size_t e0 = inside ? (size_t)oy * a.W + 4 * (size_t)ag : 0;
            const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
                (void *)((const char *)a.R + ((size_t)k * HW + e0) * EB), (short)0, (int)((HW - e0) * EB),
                BUF_DWORD3);
            const __amdgpu_buffer_rsrc_t ri = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.ivar32 + e0), (short)0, (int)((HW - e0) * 4), BUF_DWORD3);
            const __amdgpu_buffer_rsrc_t rsc = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.scales + (size_t)k * a.nqy * a.nqx), (short)0, a.nqy * a.nqx * 4, BUF_DWORD3);
            const bool moved = oy != f_oy || ox != f_ox;   // wave-uniform
            f_oy = oy;
            f_ox = ox;
#pragma unroll
            for (int it = 0; it < NLD; ++it) {
                const int idx = tid + NT * it;
                const int r = idx / NG, g = idx - r * NG;
                const int y = oy + r, gi = ag + g;
                const bool ok = (it < NLD - 1 || last_ok) &&
                                (inside || ((unsigned)y < (unsigned)a.H && (unsigned)gi < (unsigned)W4));
                const uint32_t eo = inside ? soff[it] : (uint32_t)(y * a.W + 4 * gi);
                const int ro = (int)(ok ? eo * (uint32_t)EB : OOB), io = (int)(ok ? eo * 4u : OOB);
                if (moved)
                    pre[it].iv = as_f4(__builtin_amdgcn_raw_buffer_load_b128(ri, io, 0, 0));
                if constexpr (SRC == TNO_FP8_E4M3) {
                    pre[it].c = __builtin_amdgcn_raw_buffer_load_b32(rr, ro, 0, 0);
                } else {
                    const auto c = __builtin_amdgcn_raw_buffer_load_b64(rr, ro, 0, 0);
                    pre[it].c = make_uint2(c[0], c[1]);
                }
                // the frame's scale of the 64 x 64 tile holding (y, 4gi)
                const int so = (int)(ok ? (uint32_t)(((y >> 6) * a.nqx + (gi >> 4)) * 4) : OOB);
                pre[it].s = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsc, so, 0, 0));
            }
            return ox & 3;
        } else {
            const int oy = ty0 + e[0] - h + a.Pt;
            const int ox = tx0 + e[1] - h + a.Pl;
            const int ag = ox >> 2;      // floor division (arithmetic shift)
            const float4 *Zk = a.Z4 + (size_t)k * frame4;
            if (oy >= 0 && oy + WY <= a.Hp && ag >= 0 && ag + NG <= a.Wp4) {
                // buffer loads from a resource at the window origin (scalar
                // registers) plus 32-bit lane offsets; the resource ends with the
                // frame (at most 2^31 - 1 bytes on), so no load reaches past it
                const size_t o0 = (size_t)oy * a.Wp4 + ag;
                const size_t rem = (frame4 - o0) * 16;
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(Zk + o0), (short)0, (int)(rem < 0x7FFFFFFFu ? rem : 0x7FFFFFFFu), BUF_DWORD3);
#pragma unroll
                for (int it = 0; it < NLD; ++it)
                    pre[it].z = as_f4(__builtin_amdgcn_raw_buffer_load_b128(rs, (int)soff[it], 0, 0));
            } else {
#pragma unroll
                for (int it = 0; it < NLD; ++it) {
                    const int idx = tid + NT * it;
                    const int r = idx / NG;
                    const int yp = oy + r, gp = ag + (idx - r * NG);
                    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (idx < NWIN && (unsigned)yp < (unsigned)a.Hp && (unsigned)gp < (unsigned)a.Wp4)
                        v = Zk[(size_t)yp * a.Wp4 + gp];
                    pre[it].z = v;
                }
            }
            return ox - (ag << 2);
        }
    };
    // LDS window, de-interleaved: the even columns of all WY rows, then the
    // odd columns (rows of LH floats each).  A staged group arrives as (even,
    // even, odd, odd), so each half takes one 8-byte store.  With an even
    // number of columns per lane, a lane's run of window columns splits into
    // one run in each half whose order does not depend on the parity of the
    // frame's sub-float4 offset: one code path serves every frame.  The short
    // rows keep four rows of a half within one LDS instruction's offset range.
    constexpr bool SPLIT = CPL % 2 == 0;
    constexpr int LH = LS / 2;
    constexpr int HALF = WY * LH;
    auto store = [&](int buf, const Raw<SRC> (&pre)[NLD]) {
#pragma unroll
        for (int it = 0; it < NLD; ++it)
            if (it < NLD - 1 || last_ok) {
                const int idx = tid + NT * it;
                const int r = idx / NG, g = idx - r * NG;
                float2 ev, od;
                if constexpr (SRC == SRC_Z) {
                    ev = make_float2(pre[it].z.x, pre[it].z.y);
                    od = make_float2(pre[it].z.z, pre[it].z.w);
                } else {
                    const float4 v = decode_group<SRC>(pre[it]);   // image column order
                    ev = make_float2(v.x, v.z);
                    od = make_float2(v.y, v.w);
                }
                reinterpret_cast<float2 *>(&win[buf][r * LH])[g] = ev;
                reinterpret_cast<float2 *>(&win[buf][HALF + r * LH])[g] = od;
            }
    };

    float part[RPL][CPL];
    double acc[RPL][CPL];
#pragma unroll
    for (int o = 0; o < RPL; ++o)
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            part[o][c] = 0.0f;
            acc[o][c] = 0.0;
        }

    // XCH: the halo rows of frame k are added at the start of frame k+1 (or
    // at the end of the frame chunk), from the exchange buffer of frame k's
    // parity and with frame k's vertical weights, in the same order as
    // without the exchange
    float wyp[S];
    auto halo = [&](int kp) {
        if constexpr (XCH) {
            const int wvu = __builtin_amdgcn_readfirstlane(wv);
#pragma unroll
            for (int i = 0; i < S - 1; ++i) {
                const float *xr = xch + (kp & 1) * NXR * TX + ((wvu + 1) * (S - 1) + i) * TX + CPL * lane;
                float hs[CPL];
#pragma unroll
                for (int c = 0; c < CPL; c += 2) {
                    const float2 q = *reinterpret_cast<const float2 *>(xr + c);
                    hs[c] = q.x;
                    hs[c + 1] = q.y;
                }
#pragma unroll
                for (int aa = 0; aa < S; ++aa) {
                    const int o = RPL + i - aa;
                    if (o >= 0 && o < RPL) {
#pragma unroll
                        for (int c = 0; c < CPL; ++c)
                            part[o][c] = fmaf(wyp[aa], hs[c], part[o][c]);
                    }
                }
            }
        }
    };

    Raw<SRC> pre[NLD];
    int d_cur = fetch(0, pre);
    store(0, pre);
    __syncthreads();
    for (int k0 = 0; k0 < a.nframes; k0 += FRAME_CHUNK) {
        const int k1 = min(k0 + FRAME_CHUNK, a.nframes);
        // one frame; the first frame of a chunk has no pending halo rows (the
        // previous chunk added them), so it is peeled off and the loop body
        // adds them unconditionally
        auto frame = [&](int k, bool do_halo) __attribute__((always_inline)) {
            const int buf = XCH ? 0 : (k & 1);
            // the last iteration re-fetches frame T-1 into the idle buffer: no
            // branch around the prefetch, so its store stays behind the arithmetic
            const int d_next = fetch(min(k + 1, a.nframes - 1), pre);

            const cint32_t *e = tabj + (size_t)k * a.kstride * TS;
            if constexpr (XCH) {
                if (do_halo)
                    halo(k - 1);
            }
            float wt[NW];     // gy[S] gx[h], gx[S] / gx[h] (separable) or W[S][S]
#pragma unroll
            for (int s = 0; s < NW; ++s)
                wt[s] = __int_as_float(e[2 + s]);
            // this wave's first window row in the even half
            const float *wrow = win[buf] + (wv * RPL) * LH;
            // SPLIT: first column s = d + CPL*lane has the parity of d; values
            // v[0], v[2], .. come from the half of that parity starting at s/2,
            // v[1], v[3], .. from the other half starting at (s+1)/2
            // (odd CPL: column s + t sits at half (s+t)&1, index (s+t)>>1)
            const int par = d_cur & 1;
            // SPLIT: LDS byte addresses of the two runs, one base per group of
            // RG window rows, so that every read of a group is an immediate
            // offset of its base (paired reads reach 255 words): the bases are
            // made opaque to keep the compiler from re-deriving one per row
            constexpr int NR = RPL + S - 1;
            constexpr int RG = (255 - (NV - 1) / 2) / LH + 1;
            constexpr int NGR = (NR + RG - 1) / RG;
            uint32_t ga[NGR], gb[NGR];
            uint32_t a0 = 0, b0 = 0;
            if constexpr (SPLIT) {
                a0 = (uint32_t)(uintptr_t)(const lfloat_t *)(wrow + par * HALF + (d_cur >> 1) + (CPL / 2) * lane);
                b0 = (uint32_t)(uintptr_t)(const lfloat_t *)(wrow + (1 - par) * HALF + ((d_cur + 1) >> 1) +
                                                             (CPL / 2) * lane);
#pragma unroll
                for (int g = 0; g < NGR; ++g) {
                    ga[g] = a0 + (uint32_t)(g * RG * LH * 4);
                    gb[g] = b0 + (uint32_t)(g * RG * LH * 4);
                    asm volatile("" : "+v"(ga[g]), "+v"(gb[g]));
                }
            }
            const float *pt[SPLIT ? 1 : NV];
            if constexpr (!SPLIT) {
                const int s0 = d_cur + CPL * lane;
#pragma unroll
                for (int t = 0; t < NV; ++t)
                    pt[t] = wrow + ((s0 + t) & 1) * HALF + ((s0 + t) >> 1);
            }
            auto row = [&](int rr, float (&v)[NV]) {
#pragma unroll
                for (int t = 0; t < NV; ++t) {
                    if constexpr (SPLIT) {
                        const int g = rr / RG, rl = rr - g * RG;
                        const lfloat_t *q = (const lfloat_t *)(uintptr_t)((t & 1) ? gb[g] : ga[g]);
                        v[t] = q[rl * LH + (t >> 1)];
                    } else {
                        v[t] = pt[t][rr * LH];
                    }
                }
            };
            // horizontal pass of one window row (separable stamp)
            // (the table holds the column taps relative to the centre tap, whose
            // weight is folded into the row taps)
            auto horiz = [&](const float (&v)[NV], float (&hs)[CPL]) {
                if constexpr (SEP) {
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        float sum = v[c + h];
#pragma unroll
                        for (int b = 0; b < S; ++b)
                            if (b != h)
                                sum = fmaf(wt[S + b], v[c + b], sum);
                        hs[c] = sum;
                    }
                }
            };
            // vertical pass: horizontal row rr (relative to the wave's first
            // row) is stamp row aa of output row rr - aa
            auto vert = [&](int rr, const float (&hs)[CPL]) {
#pragma unroll
                for (int aa = 0; aa < S; ++aa) {
                    const int o = rr - aa;
                    if (o >= 0 && o < RPL) {
#pragma unroll
                        for (int c = 0; c < CPL; ++c)
                            part[o][c] = fmaf(wt[aa], hs[c], part[o][c]);
                    }
                }
            };
            if constexpr (XCH) {
                // Each horizontal row is computed once per block: wave v does
                // its RPL own rows and leaves the first S-1 of them in xch rows
                // v(S-1) ... for the wave above (wave 0's copy is not read);
                // the S-1 rows below the tile are spread over the waves and
                // land in xch rows NWAVE(S-1) ...; wave w then reads its halo
                // rows from xch rows (w+1)(S-1) ... after the frame's second
                // barrier (two exchange buffers, by frame parity).  One window
                // buffer: it is refilled between the two barriers, after every
                // wave has read it.
                const int wvu = __builtin_amdgcn_readfirstlane(wv);
                auto put = [&](int xrow, const float (&hs)[CPL]) {
                    float *xr = xch + (k & 1) * NXR * TX + xrow * TX + CPL * lane;
#pragma unroll
                    for (int c = 0; c < CPL; c += 2)
                        *reinterpret_cast<float2 *>(xr + c) = make_float2(hs[c], hs[c + 1]);
                };
                float vbuf[2][NV];
                row(0, vbuf[0]);
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    if (rr + 1 < RPL)
                        row(rr + 1, vbuf[(rr + 1) & 1]);
                    float hs[CPL];
                    horiz(vbuf[rr & 1], hs);
                    vert(rr, hs);
                    if (rr < S - 1)
                        put(wvu * (S - 1) + rr, hs);
                }
                constexpr int NB = (S - 1 + NWAVE - 1) / NWAVE;   // rows below the tile per wave
#pragma unroll
                for (int m = 0; m < NB; ++m) {
                    const int i = wvu + m * NWAVE;
                    if ((S - 1) % NWAVE == 0 || i < S - 1) {
                        const uint32_t off = (uint32_t)((TY + i - wvu * RPL) * LH * 4);
                        const lfloat_t *qa = (const lfloat_t *)(uintptr_t)(a0 + off);
                        const lfloat_t *qb = (const lfloat_t *)(uintptr_t)(b0 + off);
                        float v[NV];
#pragma unroll
                        for (int t = 0; t < NV; ++t)
                            v[t] = (t & 1) ? qb[t >> 1] : qa[t >> 1];
                        float hs[CPL];
                        horiz(v, hs);
                        put(NWAVE * (S - 1) + i, hs);
                    }
                }
                // keep the own-row arithmetic ahead of the barrier
#pragma unroll
                for (int o = 0; o < RPL; ++o)
#pragma unroll
                    for (int c = 0; c < CPL; ++c)
                        asm volatile("" : "+v"(part[o][c]));
                __builtin_amdgcn_sched_barrier(0);
                __syncthreads();
                store(0, pre);
#pragma unroll
                for (int aa = 0; aa < S; ++aa)
                    wyp[aa] = wt[aa];
                __syncthreads();
                d_cur = d_next;
                return;
            }
            // window rows are read one row ahead of their use (the loop is
            // unrolled, so the two buffers are register renames)
            float vbuf[2][NV];
            row(0, vbuf[0]);
#pragma unroll
            for (int rr = 0; rr < RPL + S - 1; ++rr) {
                if (rr + 1 < RPL + S - 1)
                    row(rr + 1, vbuf[(rr + 1) & 1]);
                const float (&v)[NV] = vbuf[rr & 1];
                if constexpr (SEP) {
                    // horizontal pass of the row, streamed into the vertical pass
                    float hs[CPL];
                    horiz(v, hs);
                    vert(rr, hs);
                } else {
                    // general stamp: window row rr is stamp row aa of output row rr - aa
#pragma unroll
                    for (int aa = 0; aa < S; ++aa) {
                        const int o = rr - aa;
                        if (o >= 0 && o < RPL) {
#pragma unroll
                            for (int c = 0; c < CPL; ++c) {
                                float sum = part[o][c];
#pragma unroll
                                for (int b = 0; b < S; ++b)
                                    sum = fmaf(wt[aa * S + b], v[c + b], sum);
                                part[o][c] = sum;
                            }
                        }
                    }
                }
            }
            // keep the store (and its wait on the prefetch loads) after the
            // arithmetic, so the loads' latency hides behind it: the empty
            // volatile asm statements consume every accumulator, and the store
            // (a side effect) is not moved above them
#pragma unroll
            for (int o = 0; o < RPL; ++o)
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    asm volatile("" : "+v"(part[o][c]));
            __builtin_amdgcn_sched_barrier(0);
            store(buf ^ 1, pre);
            __syncthreads();
            d_cur = d_next;
        };
        frame(k0, false);
        for (int k = k0 + 1; k < k1; ++k)
            frame(k, true);
        if constexpr (XCH)
            halo(k1 - 1);
        // frame chunk done: into the FP64 totals
#pragma unroll
        for (int o = 0; o < RPL; ++o)
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                acc[o][c] += (double)part[o][c];
                part[o][c] = 0.0f;
            }
    }

    // epilogue: SNR and flux (into the trajectory's row of the slab's
    // maps), and the tile's largest (SNR, -pixel) key
    const int jr = a.jrow[j];
    uint64_t best = 0;
    const size_t HW = (size_t)a.H * a.W;
#pragma unroll
    for (int o = 0; o < RPL; ++o) {
        const int y = ty0 + wv * RPL + o;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int x = tx0 + CPL * lane + c;
            if (y < a.H && x < a.W) {
                const double nu = acc[o][c] + (double)part[o][c];
                const size_t p = (size_t)y * a.W + x;
                const size_t mp = (size_t)jr * HW + p;
                const double L = a.lam[mp];
                float snr = 0.0f, flux = 0.0f;
                if (L > 0.0) {
                    snr = (float)(nu / sqrt(L));
                    flux = (float)(nu / L);
                }
                snr = snr + 0.0f;    // -0 -> +0 so equal scores compare equal as keys
                flux = flux + 0.0f;
                if (a.snr)
                    a.snr[mp] = snr;
                if (a.flux)
                    a.flux[mp] = flux;
                uint64_t key = ((uint64_t)ordered_key(snr) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)p);
                best = key > best ? key : best;
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t o = __shfl_xor(best, off, 64);
        best = o > best ? o : best;
    }
    __shared__ uint64_t wbest[NWAVE];
    if (lane == 0)
        wbest[wv] = best;
    __syncthreads();
    if (tid == 0) {
        uint64_t m = wbest[0];
        for (int w = 1; w < NWAVE; ++w)
            m = wbest[w] > m ? wbest[w] : m;
        a.tile_keys[(size_t)j * ntiles + tile] = m;
    }
}

// One request: block b takes work item xcd_item(b) of the request.
// (4 waves per SIMD: a stack read in place holds more registers per staged
// group, and the allocation is held at 128 VGPRs rather than lose a wave.)
template <int S, int NWAVE, int CPL, int RPL, bool SEP, bool XCH, int SRC>
__global__ __launch_bounds__(64 * NWAVE) __attribute__((amdgpu_waves_per_eu(SRC == SRC_Z ? 1 : 4)))
void k_search(SearchArgs a)
{
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item < a.n_items)
        search_item<S, NWAVE, CPL, RPL, SEP, XCH, SRC>(a, item);
}

// A step of the serving loop: consecutive block ranges take work items of
// different requests (step_item maps a block to its request and item).
template <int S, int NWAVE, int CPL, int RPL, bool SEP, bool XCH, int SRC>
__global__ __launch_bounds__(64 * NWAVE) __attribute__((amdgpu_waves_per_eu(SRC == SRC_Z ? 1 : 4)))
void k_search_step(StepArgs s)
{
    int r, item;
    if (step_item(s, r, item))
        search_item<S, NWAVE, CPL, RPL, SEP, XCH, SRC>(step_args(s, r), item);
}

template <int S, int NWAVE, int CPL, int RPL = 8, bool SEP = true, int SRC = SRC_Z>
static void launch_search_t(hipStream_t st, const SearchArgs &a, const StepArgs *step = nullptr,
                            int nblocks = 0)
{
    // the shared-row form wherever it applies, its LDS (one window, two
    // exchange buffers) keeps as many blocks per CU as two windows do, and the
    // block has at most 4 waves (with 8 its registers cost a wave per SIMD)
    constexpr int NWIN = (RPL * NWAVE + S - 1) * ((64 * CPL + S - 1 + 6) / 4);
    constexpr int LDS_X = NWIN * 16 + 2 * (NWAVE + 1) * (S - 1) * 64 * CPL * 4;
    constexpr int LDS_2 = 2 * NWIN * 16;
    constexpr bool XCH = SEP && CPL % 2 == 0 && S > 1 && S - 1 <= RPL && NWAVE > 1 && NWAVE <= 4 &&
                         LDS_PER_CU / LDS_X >= LDS_PER_CU / LDS_2;
    if (step)
        hipLaunchKernelGGL((k_search_step<S, NWAVE, CPL, RPL, SEP, XCH, SRC>), dim3(nblocks), dim3(64 * NWAVE), 0,
                           st, *step);
    else
        hipLaunchKernelGGL((k_search<S, NWAVE, CPL, RPL, SEP, XCH, SRC>), dim3(xcd_grid(a.n_items)),
                           dim3(64 * NWAVE), 0, st, a);
}

// The default tile shape for a stack of `dtype` read in place (stamp 5).
template <bool SEP>
static hipError_t launch_search_direct(hipStream_t st, int dtype, const SearchArgs &a, const StepArgs *step,
                                       int nblocks)
{
    switch (dtype) {
    case TNO_BF16: launch_search_t<5, 4, 2, 8, SEP, TNO_BF16>(st, a, step, nblocks); break;
    case TNO_F16: launch_search_t<5, 4, 2, 8, SEP, TNO_F16>(st, a, step, nblocks); break;
    case TNO_FP8_E4M3: launch_search_t<5, 4, 2, 8, SEP, TNO_FP8_E4M3>(st, a, step, nblocks); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t launch_search_any(hipStream_t st, int S, bool sep, int variant, const SearchArgs &a,
                                    const StepArgs *step, int nblocks)
{
    if (variant == SEARCH_WS || variant == SEARCH_WS4)
        return ws_stamp(S) ? launch_search_ws(st, S, sep, variant, a, step, nblocks) : hipErrorInvalidValue;
    if (!a.Z4) {
        // a reduced-precision stack read in place: the default shape, stamp 5
        if (variant != 0 || S != 5)
            return hipErrorInvalidValue;
        return sep ? launch_search_direct<true>(st, a.dtype, a, step, nblocks)
                   : launch_search_direct<false>(st, a.dtype, a, step, nblocks);
    }
    if (S == 5 && sep) {
        switch (variant) {
        case 0: launch_search_t<5, 4, 2>(st, a, step, nblocks); break;
        case 1: launch_search_t<5, 8, 2>(st, a, step, nblocks); break;
        case 2: launch_search_t<5, 2, 2>(st, a, step, nblocks); break;
        case 3: launch_search_t<5, 4, 1>(st, a, step, nblocks); break;
        case 4: launch_search_t<5, 8, 1>(st, a, step, nblocks); break;
        case 5: launch_search_t<5, 4, 4>(st, a, step, nblocks); break;
        case 6: launch_search_t<5, 2, 2, 16>(st, a, step, nblocks); break;
        case 7: launch_search_t<5, 4, 2, 16>(st, a, step, nblocks); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (S == 5) {   // the general 5 x 5 stamp (tabulated PRF)
        switch (variant) {
        case 0: launch_search_t<5, 4, 2, 8, false>(st, a, step, nblocks); break;
        case 1: launch_search_t<5, 8, 2, 8, false>(st, a, step, nblocks); break;
        case 2: launch_search_t<5, 2, 2, 8, false>(st, a, step, nblocks); break;
        case 3: launch_search_t<5, 4, 1, 8, false>(st, a, step, nblocks); break;
        case 4: launch_search_t<5, 8, 1, 8, false>(st, a, step, nblocks); break;
        case 5: launch_search_t<5, 4, 4, 8, false>(st, a, step, nblocks); break;
        case 6: launch_search_t<5, 2, 2, 16, false>(st, a, step, nblocks); break;
        case 7: launch_search_t<5, 4, 2, 16, false>(st, a, step, nblocks); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (variant != 0)
        return hipErrorInvalidValue;
    if (sep) {
        switch (S) {
        case 1: launch_search_t<1, 4, 2>(st, a, step, nblocks); break;
        case 3: launch_search_t<3, 4, 2>(st, a, step, nblocks); break;
        case 7: launch_search_t<7, 4, 2>(st, a, step, nblocks); break;
        case 9: launch_search_t<9, 4, 2>(st, a, step, nblocks); break;
        case 11: launch_search_t<11, 4, 2>(st, a, step, nblocks); break;
        case 13: launch_search_t<13, 4, 2>(st, a, step, nblocks); break;
        case 15: launch_search_t<15, 4, 2>(st, a, step, nblocks); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (S) {
        case 1: launch_search_t<1, 4, 2, 8, false>(st, a, step, nblocks); break;
        case 3: launch_search_t<3, 4, 2, 8, false>(st, a, step, nblocks); break;
        case 7: launch_search_t<7, 4, 2, 8, false>(st, a, step, nblocks); break;
        case 9: launch_search_t<9, 4, 2, 8, false>(st, a, step, nblocks); break;
        case 11: launch_search_t<11, 4, 2, 8, false>(st, a, step, nblocks); break;
        case 13: launch_search_t<13, 4, 2, 8, false>(st, a, step, nblocks); break;
        case 15: launch_search_t<15, 4, 2, 8, false>(st, a, step, nblocks); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_search(hipStream_t st, int S, bool sep, int variant, const SearchArgs &a)
{
    return launch_search_any(st, S, sep, variant, a, nullptr, 0);
}

hipError_t launch_search_step(hipStream_t st, int S, bool sep, int variant, const SearchArgs &proto,
                              const StepArgs &step, int nblocks)
{
    if (nblocks <= 0 || step.n <= 0)
        return hipErrorInvalidValue;
    return launch_search_any(st, S, sep, variant, proto, &step, nblocks);
}

// ------------------------------------------------------------------ reductions

// Per trajectory of a slab (block r: trajectory rows[r], row r of the slab's
// maps): the largest tile key; ties in SNR go to the smallest pixel index
// because the key stores 0xFFFFFFFF - (y*W + x) in its low half.
__global__ void k_trajmax(int ntiles, int W, int HW, const int32_t *__restrict__ rows,
                          const uint64_t *__restrict__ tile_keys, const float *__restrict__ snr,
                          const float *__restrict__ flux, tno_peak *__restrict__ out)
{
    const int r = blockIdx.x;
    const int j = rows[r];
    uint64_t m = 0;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        uint64_t v = tile_keys[(size_t)j * ntiles + t];
        m = v > m ? v : m;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    __shared__ uint64_t wm[4];
    if ((threadIdx.x & 63) == 0)
        wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            m = wm[w] > m ? wm[w] : m;
        m = wm[0] > m ? wm[0] : m;
        uint32_t p = 0xFFFFFFFFu - (uint32_t)(m & 0xFFFFFFFFu);
        size_t mp = (size_t)r * HW + p;
        tno_peak pk;
        pk.snr = snr[mp];
        pk.flux = flux[mp];
        pk.y = (int32_t)(p / (uint32_t)W);
        pk.x = (int32_t)(p % (uint32_t)W);
        out[j] = pk;
    }
}

hipError_t launch_trajmax(hipStream_t st, int J, int ntiles, int W, int HW, const int32_t *rows,
                          const uint64_t *tile_keys, const float *snr, const float *flux,
                          void *traj_max_out)
{
    hipLaunchKernelGGL(k_trajmax, dim3(J), dim3(256), 0, st, ntiles, W, HW, rows, tile_keys, snr, flux,
                       (tno_peak *)traj_max_out);
    return hipGetLastError();
}

// Per start pixel: the bank maximum (Sec. 3.2) over the trajectories searched
// so far, merged with one more slab (row r of `snr` and `flux` holds
// trajectory rows[r]); among equal scores the lowest trajectory number wins.
// best_flux is the flux of the maximising trajectory.  first: the slab
// starts the maximum.
__global__ void k_best(int J, int64_t HW, const int32_t *__restrict__ rows, int first,
                       const float *__restrict__ snr, const float *__restrict__ flux,
                       float *__restrict__ best_snr, int32_t *__restrict__ best_traj,
                       float *__restrict__ best_flux)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < HW;
         p += (int64_t)gridDim.x * blockDim.x) {
        float b;
        int bj, m0;
        int64_t bm;   // slab row of the maximum, or -1: kept from earlier slabs
        if (first) {
            b = snr[p];
            bj = rows[0];
            bm = 0;
            m0 = 1;
        } else {
            b = best_snr[p];
            bj = best_traj[p];
            bm = -1;
            m0 = 0;
        }
        for (int m = m0; m < J; ++m) {
            const float s = snr[(int64_t)m * HW + p];
            const int j = rows[m];
            if (s > b || (s == b && j < bj)) {
                b = s;
                bj = j;
                bm = m;
            }
        }
        if (bm >= 0) {
            best_snr[p] = b;
            best_traj[p] = bj;
            best_flux[p] = flux[bm * HW + p];
        }
    }
}

hipError_t launch_best(hipStream_t st, int J, int64_t HW, const int32_t *rows, bool first, const float *snr,
                       const float *flux, float *best_snr, int32_t *best_traj, float *best_flux)
{
    int64_t blocks = (HW + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_best, dim3((unsigned)blocks), dim3(256), 0, st, J, HW, rows, (int)first, snr, flux,
                       best_snr, best_traj, best_flux);
    return hipGetLastError();
}

// Row r of a slab's map into row rows[r] of the map with a row per trajectory.
__global__ void k_rows_out(int64_t HW, const int32_t *__restrict__ rows, const float *__restrict__ src,
                           float *__restrict__ dst)
{
    const int r = blockIdx.y;
    const float *s = src + (int64_t)r * HW;
    float *d = dst + (int64_t)rows[r] * HW;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

hipError_t launch_rows_out(hipStream_t st, int J, int64_t HW, const int32_t *rows, const float *slab_map,
                           float *full_map)
{
    const int64_t bx = std::min<int64_t>((HW + 255) / 256, 1024);
    hipLaunchKernelGGL(k_rows_out, dim3((unsigned)bx, (unsigned)J), dim3(256), 0, st, HW, rows, slab_map,
                       full_map);
    return hipGetLastError();
}

// ------------------------------------------------------------------ exact top-k
//
// Order: SNR descending, then flat index j*H*W + y*W + x ascending (the map's
// linear index).  Keys are the order-preserving uint32 images of the SNRs.
// 1) four 8-bit radix passes find the k-th largest key K* and how many of the
//    K*-valued elements are needed; 2) one pass appends every key > K*;
// 3) chunk counts + a scan give each K*-valued element its rank in index
//    order, and the first `need` are appended; 4) one block sorts the k.

// honor: return at once when the pruned selection already produced the top k.
__global__ void k_topk_init(TopkState *st, int k, uint64_t *cand, int honor)
{
    if (honor && st->skip)
        return;
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->k_rem = k;
        st->n_gt = 0;
    }
    for (int i = threadIdx.x; i < 256; i += blockDim.x)
        st->hist[i] = 0;
    for (int i = threadIdx.x; i < 2 * TNO_MAX_TOPK; i += blockDim.x)
        cand[i] = 0;
}

__global__ void k_topk_hist(const float *__restrict__ snr, int64_t N, TopkState *st, int shift, int honor)
{
    if (honor && st->skip)
        return;
    __shared__ uint32_t hl[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x)
        hl[i] = 0;
    __syncthreads();
    const uint32_t prefix = st->prefix, mask = st->mask;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t key = ordered_key(snr[i]);
        if ((key & mask) == prefix)
            atomicAdd(&hl[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += blockDim.x)
        if (hl[i])
            atomicAdd(&st->hist[i], hl[i]);
}

__global__ void k_topk_select(TopkState *st, int shift, int honor)
{
    if (honor && st->skip)
        return;
    if (threadIdx.x == 0) {
        int32_t krem = st->k_rem;
        uint32_t above = 0;
        int b = 255;
        for (; b > 0; --b) {
            uint32_t c = st->hist[b];
            if ((int64_t)above + c >= (int64_t)krem)
                break;
            above += c;
        }
        st->prefix |= (uint32_t)b << shift;
        st->mask |= 255u << shift;
        st->k_rem = krem - (int32_t)above;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += blockDim.x)
        st->hist[i] = 0;
}

// Append keys > K*; count K*-valued keys per chunk of TOPK_CHUNK elements.
__global__ void k_topk_gt(const float *__restrict__ snr, int64_t N, int k, TopkState *st,
                          uint32_t *__restrict__ chunk_cnt, uint64_t *__restrict__ cand, int honor)
{
    if (honor && st->skip)
        return;
    const uint32_t kstar = st->prefix;
    const int64_t c0 = (int64_t)blockIdx.x * TOPK_CHUNK;
    uint32_t ties = 0;
    for (int64_t i = c0 + threadIdx.x; i < N && i < c0 + TOPK_CHUNK; i += blockDim.x) {
        uint32_t key = ordered_key(snr[i]);
        if (key > kstar) {
            uint32_t pos = atomicAdd(&st->n_gt, 1u);
            if (pos < (uint32_t)k) {      // at most k-1 keys exceed the k-th
                cand[2 * pos] = key;
                cand[2 * pos + 1] = (uint64_t)i;
            }
        } else if (key == kstar) {
            ++ties;
        }
    }
    for (int off = 32; off >= 1; off >>= 1)
        ties += __shfl_xor(ties, off, 64);
    __shared__ uint32_t wt[4];
    if ((threadIdx.x & 63) == 0)
        wt[threadIdx.x >> 6] = ties;
    __syncthreads();
    if (threadIdx.x == 0)
        chunk_cnt[blockIdx.x] = wt[0] + wt[1] + wt[2] + wt[3];
}

// Exclusive scan of the chunk counts (one block).
__global__ void k_topk_scan(uint32_t *cnt, int64_t n, const TopkState *st, int honor)
{
    if (honor && st->skip)
        return;
    __shared__ uint32_t carry;
    __shared__ uint32_t buf[256];
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < n; b += 256) {
        int64_t i = b + threadIdx.x;
        uint32_t v = i < n ? cnt[i] : 0u;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            uint32_t t = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0u;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        uint32_t incl = buf[threadIdx.x];
        if (i < n)
            cnt[i] = carry + incl - v;
        __syncthreads();
        if (threadIdx.x == 255)
            carry += incl;
        __syncthreads();
    }
}

// Append the first `need` K*-valued elements in index order.
__global__ void k_topk_ties(const float *__restrict__ snr, int64_t N, int k,
                            const TopkState *__restrict__ st,
                            const uint32_t *__restrict__ chunk_off, uint64_t *__restrict__ cand, int honor)
{
    if (honor && st->skip)
        return;
    const uint32_t kstar = st->prefix;
    const uint32_t need = (uint32_t)st->k_rem;
    const uint32_t n_gt = (uint32_t)k - need;
    const uint32_t start = chunk_off[blockIdx.x];
    if (start >= need)
        return;
    const int64_t c0 = (int64_t)blockIdx.x * TOPK_CHUNK;
    __shared__ uint32_t buf[256];
    uint32_t running = start;
    for (int64_t b = c0; b < N && b < c0 + TOPK_CHUNK; b += 256) {
        int64_t i = b + threadIdx.x;
        uint32_t f = (i < N && ordered_key(snr[i]) == kstar) ? 1u : 0u;
        buf[threadIdx.x] = f;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            uint32_t t = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0u;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        uint32_t rank = running + buf[threadIdx.x] - f;
        if (f && rank < need) {
            cand[2 * (n_gt + rank)] = kstar;
            cand[2 * (n_gt + rank) + 1] = (uint64_t)i;
        }
        uint32_t tot = buf[255];
        __syncthreads();
        running += tot;
        if (running >= need)
            break;
    }
}

// Bitonic sort of up to TNO_MAX_TOPK (key, index) pairs in LDS into
// (key descending, index ascending); one thread per slot, slots >= k padded.
__device__ void sort_candidates(uint64_t *sk, uint64_t *si, const uint64_t *cand, int k)
{
    const int t = threadIdx.x;
    // pad with the smallest key and the largest index
    sk[t] = t < k ? cand[2 * t] : 0u;
    si[t] = t < k ? cand[2 * t + 1] : ~0ull;
    __syncthreads();
    for (int size = 2; size <= TNO_MAX_TOPK; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            int p = t ^ stride;
            if (p > t) {
                // "before" = larger key, or equal key and smaller index
                bool t_before_p = sk[t] > sk[p] || (sk[t] == sk[p] && si[t] < si[p]);
                bool ascending = (t & size) == 0;   // ascending in "before" order
                if (ascending != t_before_p) {
                    uint64_t a = sk[t]; sk[t] = sk[p]; sk[p] = a;
                    uint64_t b = si[t]; si[t] = si[p]; si[p] = b;
                }
            }
            __syncthreads();
        }
    }
}

// Merge the k_new candidates of one slab (unsorted (key, index into the
// slab's map) pairs in cand, row r of the map holding trajectory rows[r];
// flux from the slab's map) into the k_run
// candidates kept from earlier slabs (sorted, in out) and write back the first
// k_out of the union in the top-k order as (snr, flux, traj, y, x).  The
// order is total (SNR descending, then flat index j*H*W + y*W + x ascending),
// so the top k of all slabs is the top k of the slabs' top k.
constexpr int MERGE_N = 2 * TNO_MAX_TOPK;
__global__ __launch_bounds__(1024) void k_topk_merge(int k_new, int k_run, int k_out, int64_t N, int64_t HW,
                                                     int W, const int32_t *__restrict__ rows,
                                                     const uint64_t *__restrict__ cand,
                                                     const float *__restrict__ flux,
                                                     tno_candidate *__restrict__ out)
{
    __shared__ uint64_t sk[MERGE_N];
    __shared__ uint64_t si[MERGE_N];
    __shared__ float sf[MERGE_N];
    for (int t = threadIdx.x; t < MERGE_N; t += blockDim.x) {
        if (t < k_run) {
            const tno_candidate c = out[t];
            sk[t] = ordered_key(c.snr);
            si[t] = ((uint64_t)c.traj * (uint64_t)HW) + (uint64_t)c.y * (uint64_t)W + (uint64_t)c.x;
            sf[t] = c.flux;
        } else if (t < k_run + k_new) {
            const uint64_t c = cand[2 * (t - k_run) + 1];
            const uint64_t li = c < (uint64_t)N ? c : 0;   // (always below N)
            sk[t] = cand[2 * (t - k_run)];
            si[t] = (uint64_t)rows[li / (uint64_t)HW] * (uint64_t)HW + li % (uint64_t)HW;
            sf[t] = flux[li];
        } else {
            sk[t] = 0u;      // padding: the smallest key and the largest index
            si[t] = ~0ull;
            sf[t] = 0.0f;
        }
    }
    __syncthreads();
    // bitonic sort into (key descending, index ascending); the thread owning
    // slot t compares it with its partner t ^ stride when that is larger
    for (int size = 2; size <= MERGE_N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < MERGE_N; t += blockDim.x) {
                const int p = t ^ stride;
                if (p > t) {
                    const bool t_before_p = sk[t] > sk[p] || (sk[t] == sk[p] && si[t] < si[p]);
                    const bool ascending = (t & size) == 0;
                    if (ascending != t_before_p) {
                        const uint64_t a = sk[t]; sk[t] = sk[p]; sk[p] = a;
                        const uint64_t b = si[t]; si[t] = si[p]; si[p] = b;
                        const float c = sf[t]; sf[t] = sf[p]; sf[p] = c;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < k_out; t += blockDim.x) {
        tno_candidate c;
        c.snr = key_to_float((uint32_t)sk[t]);
        c.flux = sf[t];
        c.traj = (int32_t)(si[t] / (uint64_t)HW);
        const uint64_t p = si[t] % (uint64_t)HW;
        c.y = (int32_t)(p / (uint64_t)W);
        c.x = (int32_t)(p % (uint64_t)W);
        out[t] = c;
    }
}

// Radix select + tie resolution of the k largest keys of `vals` (N values);
// leaves the k (key, index) pairs, unsorted, in cand.
// honor: every pass returns at once if the pruned selection set state->skip.
static void topk_select(hipStream_t st, const float *vals, int64_t N, int k, TopkState *state,
                        uint32_t *chunk_cnt, int64_t n_chunks, uint64_t *cand, int honor)
{
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, st, state, k, cand, honor);
    int64_t blocks = (N + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    for (int pass = 0; pass < 4; ++pass) {
        int shift = 24 - 8 * pass;
        hipLaunchKernelGGL(k_topk_hist, dim3((unsigned)blocks), dim3(256), 0, st, vals, N, state, shift, honor);
        hipLaunchKernelGGL(k_topk_select, dim3(1), dim3(256), 0, st, state, shift, honor);
    }
    hipLaunchKernelGGL(k_topk_gt, dim3((unsigned)n_chunks), dim3(256), 0, st, vals, N, k, state, chunk_cnt, cand,
                       honor);
    hipLaunchKernelGGL(k_topk_scan, dim3(1), dim3(256), 0, st, chunk_cnt, n_chunks, state, honor);
    hipLaunchKernelGGL(k_topk_ties, dim3((unsigned)n_chunks), dim3(256), 0, st, vals, N, k, state, chunk_cnt, cand,
                       honor);
}

// Pruned selection of one slab's top k.  The tile keys hold each (tile,
// trajectory) maximum, and k of them are elements of the slab, so the k-th
// largest tile maximum T* is at most the slab's k-th largest score: every
// entry of the top k has a key of at least T* and lies in a tile whose
// maximum reaches T*.  Those entries are gathered and, if there are few
// enough, sorted in one block; otherwise the full selection runs.

// One block: T* by four 8-bit radix passes over the slab's tile keys (rows
// of the slab, all tiles); resets the gather count and the skip flag.
__global__ __launch_bounds__(1024) void k_tile_threshold(const int32_t *__restrict__ rows, int nj, int ntiles,
                                                         const uint64_t *__restrict__ tile_keys, int k,
                                                         TopkState *st)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_prefix, s_mask;
    __shared__ int32_t s_krem;
    const int64_t n = (int64_t)nj * ntiles;
    if (threadIdx.x == 0) {
        s_prefix = 0;
        s_mask = 0;
        s_krem = k;
    }
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int i = threadIdx.x; i < 256; i += blockDim.x)
            hist[i] = 0;
        __syncthreads();
        const uint32_t prefix = s_prefix, mask = s_mask;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            const int64_t r = i / ntiles;
            const uint32_t key = (uint32_t)(tile_keys[(int64_t)rows[r] * ntiles + (i - r * ntiles)] >> 32);
            if ((key & mask) == prefix)
                atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t above = 0;
            int b = 255;
            for (; b > 0; --b) {
                const uint32_t c = hist[b];
                if ((int64_t)above + c >= (int64_t)s_krem)
                    break;
                above += c;
            }
            s_prefix |= (uint32_t)b << shift;
            s_mask |= 255u << shift;
            s_krem -= (int32_t)above;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->tstar = n >= k ? s_prefix : 0u;   // fewer tiles than k: every entry qualifies
        st->n_cand = 0;
        st->skip = 0;
    }
}

// One block per (slab row, tile): a tile whose maximum reaches T* appends
// every entry with a key of at least T* as (key, index in the slab's map).
__global__ void k_tile_gather(const int32_t *__restrict__ rows, int ntiles, int ntx, int tx, int ty, int H, int W,
                              int64_t HW, const uint64_t *__restrict__ tile_keys, const float *__restrict__ snr,
                              TopkState *st, uint64_t *__restrict__ buf)
{
    const int r = blockIdx.x / ntiles, t = blockIdx.x - r * ntiles;
    const uint32_t tstar = st->tstar;
    if ((uint32_t)(tile_keys[(int64_t)rows[r] * ntiles + t] >> 32) < tstar)
        return;
    const int tyi = t / ntx, txi = t - tyi * ntx;
    const int y0 = tyi * ty, x0 = txi * tx;
    const int th = min(ty, H - y0), tw = min(tx, W - x0);
    for (int i = threadIdx.x; i < th * tw; i += blockDim.x) {
        const int yy = i / tw;
        const int64_t li = (int64_t)r * HW + (int64_t)(y0 + yy) * W + (x0 + i - yy * tw);
        const uint32_t key = ordered_key(snr[li]);
        if (key >= tstar) {
            const uint32_t pos = atomicAdd(&st->n_cand, 1u);
            if (pos < (uint32_t)TOPK_GATHER_CAP) {
                buf[2 * pos] = key;
                buf[2 * pos + 1] = (uint64_t)li;
            }
        }
    }
}

// One block: if at most TOPK_GATHER_CAP entries were gathered, sort them
// (key descending, index ascending), write the first k to cand and set
// skip; otherwise leave skip 0 for the full selection.
__global__ __launch_bounds__(1024) void k_topk_small(const uint64_t *__restrict__ buf, int k, TopkState *st,
                                                     uint64_t *__restrict__ cand)
{
    __shared__ uint32_t sk[TOPK_GATHER_CAP];
    __shared__ uint64_t si[TOPK_GATHER_CAP];
    const uint32_t n = st->n_cand;
    if (n > (uint32_t)TOPK_GATHER_CAP || n < (uint32_t)k)
        return;
    int np = 1;
    while (np < (int)n)
        np <<= 1;
    for (int t = threadIdx.x; t < np; t += blockDim.x) {
        const bool in = t < (int)n;
        sk[t] = in ? (uint32_t)buf[2 * t] : 0u;     // padding: the smallest key, the largest index
        si[t] = in ? buf[2 * t + 1] : ~0ull;
    }
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < np; t += blockDim.x) {
                const int p = t ^ stride;
                if (p > t) {
                    const bool t_before_p = sk[t] > sk[p] || (sk[t] == sk[p] && si[t] < si[p]);
                    const bool ascending = (t & size) == 0;
                    if (ascending != t_before_p) {
                        const uint32_t a = sk[t]; sk[t] = sk[p]; sk[p] = a;
                        const uint64_t b = si[t]; si[t] = si[p]; si[p] = b;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        cand[2 * t] = sk[t];
        cand[2 * t + 1] = si[t];
    }
    if (threadIdx.x == 0)
        st->skip = 1;
}

hipError_t launch_topk(hipStream_t st, const float *snr, const float *flux, int64_t N, int64_t HW,
                       int H, int W, const int32_t *rows, int k, int k_run, const uint64_t *tile_keys,
                       int ntiles, int ntx, int tx, int ty, uint64_t *gbuf, TopkState *state,
                       uint32_t *chunk_cnt, int64_t n_chunks, uint64_t *cand, void *topk_out)
{
    const int k_new = (int)std::min<int64_t>(k, N);
    const int nj = (int)(N / HW);
    hipLaunchKernelGGL(k_tile_threshold, dim3(1), dim3(1024), 0, st, rows, nj, ntiles, tile_keys, k_new, state);
    hipLaunchKernelGGL(k_tile_gather, dim3((unsigned)(nj * ntiles)), dim3(256), 0, st, rows, ntiles, ntx, tx, ty, H,
                       W, HW, tile_keys, snr, state, gbuf);
    hipLaunchKernelGGL(k_topk_small, dim3(1), dim3(1024), 0, st, gbuf, k_new, state, cand);
    topk_select(st, snr, N, k_new, state, chunk_cnt, n_chunks, cand, 1);
    hipLaunchKernelGGL(k_topk_merge, dim3(1), dim3(1024), 0, st, k_new, k_run, std::min(k, k_run + k_new), N,
                       HW, W, rows, cand, flux, (tno_candidate *)topk_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ significance (Sec. 3.3)
//
// The paper expresses each pixel's best score in units of the standard
// deviation of the scores in the box x box square centred on it.  Windows are
// clipped at the image edges; the std is the population std of the scores
// inside, from FP64 window sums of s and s^2 along rows, then columns; a
// variance below 1e-12 of the window's mean square counts as 0.

constexpr int BOX_BLK = 16;   // aligned block of the window sums

// Window sums never slide: a window's sum is its loose ends plus the sums of
// the aligned blocks of BOX_BLK values it covers, so it depends only on the
// values inside the window (a constant window gives the exact square of its
// mean, and a one-pixel window a variance of exactly 0).

// Block sums along each row of the best map: (sum v, sum v^2) per block.
__global__ void k_box_rblk(int H, int W, const float *__restrict__ s, double *__restrict__ b1,
                           double *__restrict__ b2)
{
    const int nb = (W + BOX_BLK - 1) / BOX_BLK;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= H * nb)
        return;
    const int y = gid / nb, b = gid - y * nb;
    const float *row = s + (size_t)y * W;
    double a1 = 0.0, a2 = 0.0;
    for (int x = b * BOX_BLK; x < min(W, (b + 1) * BOX_BLK); ++x) {
        const double v = row[x];
        a1 += v;
        a2 += v * v;
    }
    b1[gid] = a1;
    b2[gid] = a2;
}

// Row window sums over [x-hb, x+hb] clipped to the row.
__global__ void k_box_rows(int H, int W, int hb, const float *__restrict__ s,
                           const double *__restrict__ b1, const double *__restrict__ b2,
                           double *__restrict__ r1, double *__restrict__ r2)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)H * W)
        return;
    const int y = (int)(gid / W), x = (int)(gid - (int64_t)y * W);
    const int nb = (W + BOX_BLK - 1) / BOX_BLK;
    const float *row = s + (size_t)y * W;
    const int lo = max(0, x - hb), hi = min(W - 1, x + hb);
    const int bl = (lo + BOX_BLK - 1) / BOX_BLK, bh = (hi + 1) / BOX_BLK;   // whole blocks [bl, bh)
    double a1 = 0.0, a2 = 0.0;
    auto one = [&](int xx) {
        const double v = row[xx];
        a1 += v;
        a2 += v * v;
    };
    if (bl < bh) {
        for (int xx = lo; xx < bl * BOX_BLK; ++xx)
            one(xx);
        for (int b = bl; b < bh; ++b) {
            a1 += b1[(size_t)y * nb + b];
            a2 += b2[(size_t)y * nb + b];
        }
        for (int xx = bh * BOX_BLK; xx <= hi; ++xx)
            one(xx);
    } else {
        for (int xx = lo; xx <= hi; ++xx)
            one(xx);
    }
    r1[gid] = a1;
    r2[gid] = a2;
}

// Block sums down each column of the row window sums.
__global__ void k_box_cblk(int H, int W, const double *__restrict__ r1,
                           const double *__restrict__ r2, double *__restrict__ b1,
                           double *__restrict__ b2)
{
    const int nb = (H + BOX_BLK - 1) / BOX_BLK;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)nb * W)
        return;
    const int b = (int)(gid / W), x = (int)(gid - (int64_t)b * W);   // adjacent threads: adjacent columns
    double a1 = 0.0, a2 = 0.0;
    for (int y = b * BOX_BLK; y < min(H, (b + 1) * BOX_BLK); ++y) {
        a1 += r1[(size_t)y * W + x];
        a2 += r2[(size_t)y * W + x];
    }
    b1[gid] = a1;
    b2[gid] = a2;
}

// Column window sums, the clipped window's count, the population standard
// deviation and significance = best / std (0 where std is 0).
__global__ void k_box_cols(int H, int W, int hb, const double *__restrict__ r1,
                           const double *__restrict__ r2, const double *__restrict__ b1,
                           const double *__restrict__ b2, const float *__restrict__ s,
                           float *__restrict__ sig)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)H * W)
        return;
    const int y = (int)(gid / W), x = (int)(gid - (int64_t)y * W);
    const int lo = max(0, y - hb), hi = min(H - 1, y + hb);
    const int bl = (lo + BOX_BLK - 1) / BOX_BLK, bh = (hi + 1) / BOX_BLK;
    double a1 = 0.0, a2 = 0.0;
    auto one = [&](int yy) {
        a1 += r1[(size_t)yy * W + x];
        a2 += r2[(size_t)yy * W + x];
    };
    if (bl < bh) {
        for (int yy = lo; yy < bl * BOX_BLK; ++yy)
            one(yy);
        for (int b = bl; b < bh; ++b) {
            a1 += b1[(size_t)b * W + x];
            a2 += b2[(size_t)b * W + x];
        }
        for (int yy = bh * BOX_BLK; yy <= hi; ++yy)
            one(yy);
    } else {
        for (int yy = lo; yy <= hi; ++yy)
            one(yy);
    }
    const double nx = (double)(min(W - 1, x + hb) - max(0, x - hb) + 1);
    const double n = nx * (double)(hi - lo + 1);
    const double mean = a1 / n;
    const double var = a2 / n - mean * mean;
    // rounding of the sums leaves a residue of order n * 1e-16 of the mean
    // square where the window is constant: treat such a variance as 0
    const double sd = var > 1e-12 * (a2 / n) ? sqrt(var) : 0.0;
    float g = sd > 0.0 ? (float)((double)s[gid] / sd) : 0.0f;
    sig[gid] = g + 0.0f;
}

__global__ void k_count_above(int64_t N, const float *__restrict__ sig, float thr, int32_t *count)
{
    uint32_t c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        c += sig[i] >= thr ? 1u : 0u;
    for (int off = 32; off >= 1; off >>= 1)
        c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c)
        atomicAdd(count, (int32_t)c);
}

// Sort the k most significant pixels and keep those at or above the threshold.
__global__ __launch_bounds__(1024) void k_detect_final(
    int64_t HW, int W, int k, float thr, const uint64_t *__restrict__ cand,
    const float *__restrict__ best_snr, const int32_t *__restrict__ best_traj,
    const float *__restrict__ best_flux, tno_detection *__restrict__ out, int32_t *n_out)
{
    __shared__ uint64_t sk[TNO_MAX_TOPK];
    __shared__ uint64_t si[TNO_MAX_TOPK];
    __shared__ int32_t n_keep;
    const int t = threadIdx.x;
    if (t == 0)
        n_keep = 0;
    sort_candidates(sk, si, cand, k);
    if (t < k) {
        const float g = key_to_float((uint32_t)sk[t]);
        if (g >= thr) {
            const uint64_t p = si[t] < (uint64_t)HW ? si[t] : 0;
            const int32_t j = best_traj[p];
            tno_detection d;
            d.significance = g;
            d.snr = best_snr[p];
            d.flux = best_flux[p];
            d.traj = j;
            d.y = (int32_t)(p / (uint64_t)W);
            d.x = (int32_t)(p % (uint64_t)W);
            out[t] = d;
            atomicAdd(&n_keep, 1);
        }
    }
    __syncthreads();
    if (t == 0)
        *n_out = n_keep;
}

int64_t significance_block_values(int H, int W)
{
    return std::max<int64_t>((int64_t)H * ((W + BOX_BLK - 1) / BOX_BLK),
                             (int64_t)W * ((H + BOX_BLK - 1) / BOX_BLK));
}

hipError_t launch_significance(hipStream_t st, int H, int W, int box, float thr, int k,
                               const float *best_snr, const int32_t *best_traj, const float *best_flux,
                               double *r1, double *r2, double *b1, double *b2, float *sig,
                               TopkState *state, uint32_t *chunk_cnt, int64_t n_chunks,
                               uint64_t *cand, tno_detection *det, int32_t *counts)
{
    const int hb = box / 2;
    const int64_t HW = (int64_t)H * W;
    const int64_t nrb = (int64_t)H * ((W + BOX_BLK - 1) / BOX_BLK);
    const int64_t ncb = (int64_t)W * ((H + BOX_BLK - 1) / BOX_BLK);
    auto grid = [](int64_t n) { return dim3((unsigned)((n + 255) / 256)); };
    hipLaunchKernelGGL(k_box_rblk, grid(nrb), dim3(256), 0, st, H, W, best_snr, b1, b2);
    hipLaunchKernelGGL(k_box_rows, grid(HW), dim3(256), 0, st, H, W, hb, best_snr, b1, b2, r1, r2);
    hipLaunchKernelGGL(k_box_cblk, grid(ncb), dim3(256), 0, st, H, W, r1, r2, b1, b2);
    hipLaunchKernelGGL(k_box_cols, grid(HW), dim3(256), 0, st, H, W, hb, r1, r2, b1, b2, best_snr, sig);
    int blocks = (int)std::min<int64_t>((HW + 255) / 256, 4096);
    hipLaunchKernelGGL(k_count_above, dim3(blocks), dim3(256), 0, st, HW, sig, thr, counts);
    if (k > 0) {
        topk_select(st, sig, HW, k, state, chunk_cnt, n_chunks, cand, 0);
        hipLaunchKernelGGL(k_detect_final, dim3(1), dim3(TNO_MAX_TOPK), 0, st, HW, W, k, thr, cand,
                           best_snr, best_traj, best_flux, det, counts + 1);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ quantize (precision form)

__device__ __forceinline__ uint32_t encode_e4m3(float x)
{
    // round to nearest even, saturating at 448; zero keeps no sign
    uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
    float a = fminf(fabsf(x), 448.0f);
    uint32_t mag;
    if (a < 0.015625f) {                          // below 2^-6: subnormal step 2^-9
        mag = (uint32_t)rintf(a * 512.0f);        // 0..8 (8 is the smallest normal)
    } else {
        uint32_t u = __float_as_uint(a);
        int E = (int)((u >> 23) & 0xFF) - 127;    // -6..8
        uint32_t m = u & 0x7FFFFFu;
        uint32_t r = m >> 20, rem = m & 0xFFFFFu;
        if (rem > 0x80000u || (rem == 0x80000u && (r & 1u)))
            ++r;
        if (r == 8u) {
            r = 0;
            ++E;
        }
        mag = ((uint32_t)(E + 7) << 3) | r;
        if (mag > 0x7Eu)
            mag = 0x7Eu;
    }
    return mag ? (sign | mag) : 0u;
}

__device__ __forceinline__ uint32_t encode_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// One block per (frame, 64x64 tile): amax, power-of-two scale, encode.
template <int DT>
__global__ __launch_bounds__(256) void k_quantize(const float *__restrict__ R, int H, int W,
                                                  void *__restrict__ codes,
                                                  float *__restrict__ scales)
{
    const int nqx = gridDim.x, nqy = gridDim.y;
    const int tx = blockIdx.x, ty = blockIdx.y, k = blockIdx.z;
    const size_t fo = (size_t)k * H * W;
    float am = 0.0f;
    for (int e = threadIdx.x; e < TNO_QTILE * TNO_QTILE; e += 256) {
        int y = ty * TNO_QTILE + (e >> 6), x = tx * TNO_QTILE + (e & 63);
        if (y < H && x < W)
            am = fmaxf(am, fabsf(R[fo + (size_t)y * W + x]));
    }
    for (int off = 32; off >= 1; off >>= 1)
        am = fmaxf(am, __shfl_xor(am, off, 64));
    __shared__ float wa[4];
    if ((threadIdx.x & 63) == 0)
        wa[threadIdx.x >> 6] = am;
    __syncthreads();
    am = fmaxf(fmaxf(wa[0], wa[1]), fmaxf(wa[2], wa[3]));
    constexpr int E = DT == TNO_FP8_E4M3 ? 8 : 15;
    int c = 0;
    float s = 1.0f;
    if (am > 0.0f) {
        int e2;
        float m = frexpf(am, &e2);     // am = m * 2^e2, m in [0.5, 1)
        c = (m == 0.5f) ? e2 - 1 : e2;
        s = ldexpf(1.0f, c - E);
    }
    if (threadIdx.x == 0)
        scales[((size_t)k * nqy + ty) * nqx + tx] = s;
    for (int e = threadIdx.x; e < TNO_QTILE * TNO_QTILE; e += 256) {
        int y = ty * TNO_QTILE + (e >> 6), x = tx * TNO_QTILE + (e & 63);
        if (y >= H || x >= W)
            continue;
        size_t i = fo + (size_t)y * W + x;
        float v = am > 0.0f ? ldexpf(R[i], E - c) : R[i];
        if constexpr (DT == TNO_FP8_E4M3) {
            ((uint8_t *)codes)[i] = (uint8_t)encode_e4m3(v);
        } else if constexpr (DT == TNO_BF16) {
            ((uint16_t *)codes)[i] = (uint16_t)encode_bf16(v);
        } else {
            _Float16 hv = (_Float16)v;
            ((_Float16 *)codes)[i] = hv;
        }
    }
}

hipError_t launch_quantize(hipStream_t st, int dtype, const float *R, int T, int H, int W,
                           void *codes, float *scales)
{
    dim3 grid((W + TNO_QTILE - 1) / TNO_QTILE, (H + TNO_QTILE - 1) / TNO_QTILE, T);
    switch (dtype) {
    case TNO_BF16: hipLaunchKernelGGL(k_quantize<TNO_BF16>, grid, dim3(256), 0, st, R, H, W, codes, scales); break;
    case TNO_F16: hipLaunchKernelGGL(k_quantize<TNO_F16>, grid, dim3(256), 0, st, R, H, W, codes, scales); break;
    case TNO_FP8_E4M3: hipLaunchKernelGGL(k_quantize<TNO_FP8_E4M3>, grid, dim3(256), 0, st, R, H, W, codes, scales); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tno
