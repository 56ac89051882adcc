// tno_search_ws.hip -- numerator search (arXiv:2209.09848, Sec. 3.2 eq. 4) for
// stamps of side 1, 3 and 5, with the neighbour columns of each lane taken from
// the adjacent lanes by wave shifts instead of re-reading them from LDS.
//
//   nu_j(y0, x0) = sum_k sum_ab W_jk(a, b) Z_k(y0 + iy_jk + a - h, x0 + ix_jk + b - h)
//   Z_k = R_k * ivar (0 off the image and at masked pixels)
//
// Block = one (tile of 124 x 32 start pixels, trajectory); 4 waves stacked
// vertically, 8 rows each.  Lane L of a wave holds window columns 2L and 2L+1
// of each window row it reads (one 8-byte LDS read per row); the stamp taps
// at columns 2L-2 .. 2L+3 come from lanes L-1, L and L+1, so the window is 128
// columns wide and lanes 1..62 produce the 124 start columns of the tile
// (lanes 0 and 63 have no outer neighbour).  Reading one column pair per row
// instead of the CPL + S - 1 columns a lane's stamps cover cuts the LDS read
// traffic of the horizontal pass threefold; the LDS bandwidth, not only the
// vector ALU, bounds the earlier form of the search.
//
// Per frame the window ((32 + S - 1) rows x 128 columns at the frame's
// integer shift) is staged into LDS once for the block; the next frame's
// window is fetched into registers before the current frame is computed.  The
// stack comes either staged (Z: FP32, zero-padded, weighted by ivar) or
// straight from the caller's residuals of any storage type (decoded, scaled
// by the frame's tile scale and weighted by ivar while the window is staged).
// Separable stamps: a horizontal pass per window row (centre tap weight 1,
// the others u_b = gx_b / gx_h) streamed into a vertical pass (row weights
// gy_a gx_h); every horizontal row is computed once per block and the S - 1
// rows below a wave's strip come from the wave beneath through a small LDS
// exchange buffer.  General (tabulated) stamps: S x S taps per output.
// Frame partials accumulate in FP32 over FRAME_CHUNK frames, then in FP64.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "tno_internal.h"
#include "tno_device.h"
#include "../../include/tno_search.h"

namespace tno {

namespace {

constexpr int WS_NWAVE = 4;
constexpr int WS_TX = 124;            // start columns per tile (lanes 1..62, two each)
constexpr int WS_NG = 33;             // staged float4 groups per row: offset 0..3 + 128 columns
constexpr int WS_LS = 136;            // LDS floats per window row (a multiple of 4)
#ifndef TNO_WS_AHEAD
#define TNO_WS_AHEAD 1
#endif
constexpr int WS_AHEAD = TNO_WS_AHEAD;   // window rows read ahead of their use


static_assert(WS_TX == SEARCH_VARIANTS[SEARCH_WS].tx && SEARCH_VARIANTS[SEARCH_WS].rpl == 8 &&
              SEARCH_VARIANTS[SEARCH_WS4].tx == WS_TX && SEARCH_VARIANTS[SEARCH_WS4].rpl == 4,
              "variant table out of step");

// Lane i receives lane i-1's value (prev) or lane i+1's (next); the lane at
// the end of the wave with no such neighbour receives 0.
__device__ __forceinline__ float lane_prev(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_next(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

// Horizontal pass of one window row of a separable stamp for the lane's two
// columns: ve at window column 2L (output column 2L - 2 of the tile), vo at
// 2L + 1.  The centre tap has weight 1; u[b] = gx[b] / gx[h] for the others.
// Taps held by the neighbour lanes enter through FMAs whose first operand is
// read wave-shifted (v_fmac_f32_dpp with wave_shr:1 = lane i-1, wave_shl:1 =
// lane i+1); the compiler does not fold the shift intrinsics into FMAs, so
// these are written out.  The leading s_nop provides the 5 wait states a DPP
// read needs after a vector-ALU write of its source register or of EXEC;
// inside the block only h0 and h1 are written and neither is read shifted.
// Order of the terms: centre, the lane's own other column, then the shifted
// taps by increasing offset.
template <int S>
__device__ __forceinline__ void horiz_ws(float ve, float vo, const float (&u)[S], float &h0, float &h1);

template <>
__device__ __forceinline__ void horiz_ws<5>(float ve, float vo, const float (&u)[5], float &h0, float &h1)
{
    // column 2L: taps (-2..2) = prev(ve), prev(vo), ve, vo, next(ve)
    // column 2L+1:              prev(vo), ve, vo, next(ve), next(vo)
    asm("s_nop 4\n\t"
        "v_fma_f32 %0, %3, %6, %2\n\t"
        "v_fma_f32 %1, %2, %5, %3\n\t"
        "v_fmac_f32_dpp %0, %2, %4 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %0, %3, %5 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %0, %2, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %3, %4 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %2, %6 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %3, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(h0), "=&v"(h1)
        : "v"(ve), "v"(vo), "v"(u[0]), "v"(u[1]), "v"(u[3]), "v"(u[4]));
}

template <>
__device__ __forceinline__ void horiz_ws<3>(float ve, float vo, const float (&u)[3], float &h0, float &h1)
{
    // column 2L: taps (-1..1) = prev(vo), ve, vo;  column 2L+1: ve, vo, next(ve)
    asm("s_nop 4\n\t"
        "v_fma_f32 %0, %3, %5, %2\n\t"
        "v_fma_f32 %1, %2, %4, %3\n\t"
        "v_fmac_f32_dpp %0, %3, %4 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %2, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(h0), "=&v"(h1)
        : "v"(ve), "v"(vo), "v"(u[0]), "v"(u[2]));
}

template <>
__device__ __forceinline__ void horiz_ws<1>(float ve, float vo, const float (&)[1], float &h0, float &h1)
{
    h0 = ve;
    h1 = vo;
}

}  // namespace

template <int S, bool SEP, int SRC, int RPL>
__device__ __forceinline__ void search_ws_item(const SearchArgs &a, int item)
{
    constexpr int h = S / 2;
    constexpr int NWAVE = WS_NWAVE, NT = 64 * NWAVE;
    constexpr int TX = WS_TX, TY = NWAVE * RPL;
    constexpr int WY = TY + S - 1;             // window rows
    constexpr int NG = WS_NG, LS = WS_LS;
    constexpr int NWIN = WY * NG;              // staged groups per frame
    constexpr int NLD = (NWIN + NT - 1) / NT;  // per thread
    constexpr int TS = table_stride(S, SEP);
    constexpr bool XCH = SEP && S > 1;         // halo rows through the exchange buffer
    constexpr int NXR = NWAVE * (S - 1);       // exchange rows (128 values each)
    // XCH: one window buffer and the exchange rows, both refilled and read
    // between the two barriers of a frame; otherwise two window buffers
    __shared__ __align__(16) float win[XCH ? 1 : 2][WY * LS];
    __shared__ __align__(16) float xch[XCH ? NXR * 128 : 2];

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
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);

    // This thread's staging slots: group idx = tid + NT*it of the window, at
    // window row r = idx / NG and group g = idx % NG; ldx = its LDS float
    // index r*LS + 4g; soff = its offset from the window origin in the
    // source: bytes in Z (rows of Wp4 groups), elements in the caller's stack
    // (rows of W values).  Only the last slot can fall past the window: such
    // a lane reads nothing (its offsets lie past every buffer resource, so
    // the loads return 0 and touch no memory) and stores nothing.  Where a
    // fetch needs (r, g) again they are recovered from ldx behind an empty
    // asm statement, so that the compiler does not keep them in registers
    // for the whole kernel.
    constexpr int EB = src_bytes<SRC>();
    constexpr uint32_t OOB = 0x80000000u;
    int ldx[NLD];
    uint32_t soff[NLD];
#pragma unroll
    for (int it = 0; it < NLD; ++it) {
        const int idx = tid + NT * it;
        const int r = idx / NG, g = idx - r * NG;
        ldx[it] = r * LS + 4 * g;
        if constexpr (SRC == SRC_Z)
            soff[it] = (uint32_t)(r * a.Wp4 + g) * 16u;
        else
            soff[it] = (uint32_t)(r * a.W + 4 * g);
    }
    auto slot_rg = [&](int it, int &r, int &g) {
        int l = ldx[it];
        asm volatile("" : "+v"(l));
        r = l / LS;
        g = (l - r * LS) >> 2;
    };
    const bool last_ok = tid + NT * (NLD - 1) < NWIN;
    if (!last_ok)
        soff[NLD - 1] = OOB;

    const cint32_t *tabj = (const cint32_t *)(a.tab32) + (size_t)j * a.T * TS;
    const size_t frame4 = (size_t)a.Hp * a.Wp4;
    const size_t HW = (size_t)a.H * a.W;
    const int W4 = a.W >> 2;

    // Fetch the window of frame k into registers; returns its column offset d
    // within the first staged group (the window starts at image column
    // ox = tx0 + ix - 2 and row oy = ty0 + iy - h).  Read in place, ivar is
    // fetched only when the window covers other pixels than at the previous
    // fetch (the frame's integer shift moved): otherwise the registers still
    // hold it (the slots are not written between the store of one window and
    // the fetch of the next).
    int f_oy = INT_MIN, f_ox = INT_MIN;
    auto fetch = [&](int k, Raw<SRC> (&pre)[NLD]) -> int {
        k *= a.kstride;
        const cint32_t *e = tabj + (size_t)k * TS;
        const int oy = ty0 + e[0] - h;
        const int ox = tx0 + e[1] - 2;
        if constexpr (SRC == SRC_Z) {
            const int oyp = oy + a.Pt, oxp = ox + a.Pl;   // Pl is a multiple of 4
            const int ag = oxp >> 2;
            const float4 *Zk = a.Z4 + (size_t)k * frame4;
            if (oyp >= 0 && oyp + WY <= a.Hp && ag >= 0 && ag + NG <= a.Wp4) {
                const size_t o0 = (size_t)oyp * a.Wp4 + ag;
                const size_t rb = (frame4 - o0) * 16;
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(Zk + o0), (short)0, (int)(rb < 0x7FFFFFFFu ? rb : 0x7FFFFFFFu), BUF_DWORD3);
#pragma unroll
                for (int it = 0; it < NLD; ++it)
                    pre[it].z = as_f4(__builtin_amdgcn_raw_buffer_load_b128(rs, (int)soff[it], 0, 0));
            } else {
#pragma unroll
                for (int it = 0; it < NLD; ++it) {
                    int r, g;
                    slot_rg(it, r, g);
                    const int yp = oyp + r, gp = ag + g;
                    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if ((it < NLD - 1 || last_ok) && (unsigned)yp < (unsigned)a.Hp && (unsigned)gp < (unsigned)a.Wp4)
                        v = Zk[(size_t)yp * a.Wp4 + gp];
                    pre[it].z = v;
                }
            }
            return oxp & 3;
        } else {
            const int ag = ox >> 2;   // floor
            const bool inside = oy >= 0 && oy + WY <= a.H && ag >= 0 && ag + NG <= W4;
            // resources at the window origin (inside the image) or at the
            // frame start; the plan keeps H*W*4 below 2^31, so every offset of
            // a pixel fits and OOB lies past every resource
            const size_t e0 = inside ? (size_t)oy * a.W + 4 * (size_t)ag : 0;
            const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
                (void *)((const char *)a.R + ((size_t)k * HW + e0) * EB), (short)0, (int)((HW - e0) * EB),
                BUF_DWORD3);
            const __amdgpu_buffer_rsrc_t ri = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.ivar32 + e0), (short)0, (int)((HW - e0) * 4), BUF_DWORD3);
            // (F32: no scales; the resource is built but never read)
            const __amdgpu_buffer_rsrc_t rsc = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(SRC == TNO_F32 ? a.ivar32 : a.scales + (size_t)k * a.nqy * a.nqx), (short)0,
                SRC == TNO_F32 ? 0 : a.nqy * a.nqx * 4, BUF_DWORD3);
            const bool moved = oy != f_oy || ox != f_ox;   // wave-uniform
            f_oy = oy;
            f_ox = ox;
#pragma unroll
            for (int it = 0; it < NLD; ++it) {
                int r, g;
                slot_rg(it, r, g);
                const int y = oy + r, gi = ag + g;
                const bool ok = (it < NLD - 1 || last_ok) &&
                                (inside || ((unsigned)y < (unsigned)a.H && (unsigned)gi < (unsigned)W4));
                const uint32_t eo = inside ? soff[it] : (uint32_t)(y * a.W + 4 * gi);
                const int ro = (int)(ok ? eo * (uint32_t)EB : OOB), io = (int)(ok ? eo * 4u : OOB);
                if (moved)
                    pre[it].iv = as_f4(__builtin_amdgcn_raw_buffer_load_b128(ri, io, 0, 0));
                if constexpr (SRC == TNO_F32) {
                    pre[it].r = as_f4(__builtin_amdgcn_raw_buffer_load_b128(rr, ro, 0, 0));
                } else {
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
            }
            return ox & 3;
        }
    };
    // Stage a fetched window into LDS buffer `buf`.  Window column q (0..127)
    // of row r is staged column d + q; the row is stored shifted by p = d & 1
    // floats, at LDS float r*LS + p + d + q, so that every lane's column pair
    // (2L, 2L+1) starts at an even index and is one 8-byte read.  p = 0: one
    // 16-byte store per group; p = 1: a 4-byte, an 8-byte and a 4-byte store.
    auto store = [&](int buf, int d, const Raw<SRC> (&pre)[NLD]) {
        if ((d & 1) == 0) {
#pragma unroll
            for (int it = 0; it < NLD; ++it)
                if (it < NLD - 1 || last_ok)
                    *reinterpret_cast<float4 *>(&win[buf][ldx[it]]) = decode_group<SRC>(pre[it]);
        } else {
#pragma unroll
            for (int it = 0; it < NLD; ++it)
                if (it < NLD - 1 || last_ok) {
                    const float4 z = decode_group<SRC>(pre[it]);
                    float *q = &win[buf][ldx[it]];
                    q[1] = z.x;
                    *reinterpret_cast<float2 *>(q + 2) = make_float2(z.y, z.z);
                    q[4] = z.w;
                }
        }
    };

    float part[RPL][2];
    double acc[RPL][2];
#pragma unroll
    for (int o = 0; o < RPL; ++o)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            part[o][c] = 0.0f;
            acc[o][c] = 0.0;
        }

    // vertical pass: horizontal row rr (relative to the wave's first row) is
    // stamp row aa of output row rr - aa
    auto vert = [&](int rr, const float (&wy)[S], float h0, float h1) {
#pragma unroll
        for (int aa = 0; aa < S; ++aa) {
            const int o = rr - aa;
            if (o >= 0 && o < RPL) {
                part[o][0] = fmaf(wy[aa], h0, part[o][0]);
                part[o][1] = fmaf(wy[aa], h1, part[o][1]);
            }
        }
    };
    // XCH: the halo rows of frame k (the S-1 rows below the wave's strip),
    // left in the exchange buffer by the wave beneath, are added after the
    // frame's first barrier, with frame k's row weights
    auto halo = [&](const float (&wy)[S]) {
        if constexpr (XCH) {
            // the lane's slot in this wave's first halo row
            const float *xr = xch + wv * (S - 1) * 128 + 2 * lane;
#pragma unroll
            for (int i = 0; i < S - 1; ++i) {
                const float2 q = *reinterpret_cast<const float2 *>(xr + i * 128);
                vert(RPL + i, wy, q.x, q.y);
            }
        }
    };

    Raw<SRC> pre[NLD];
    int d_cur = fetch(0, pre);
    store(0, d_cur, pre);
    __syncthreads();
    for (int k0 = 0; k0 < a.nframes; k0 += FRAME_CHUNK) {
        const int k1 = min(k0 + FRAME_CHUNK, a.nframes);
        auto frame = [&](int k) __attribute__((always_inline)) {
            const int buf = XCH ? 0 : (k & 1);
            // the last frame re-fetches itself: no branch around the prefetch
            const int d_next = fetch(min(k + 1, a.nframes - 1), pre);
            const cint32_t *e = tabj + (size_t)k * a.kstride * TS;
            // the lane's column pair of window row rr of this wave: LDS floats
            // (wv*RPL + rr)*LS + p + d + 2L and the next (8-byte aligned)
            const float *wrow = win[buf] + (wv * RPL) * LS + (d_cur + (d_cur & 1)) + 2 * lane;
            auto row = [&](int rr) -> float2 { return *reinterpret_cast<const float2 *>(wrow + rr * LS); };
            float wy[S];
            if constexpr (SEP) {
                float u[S];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    wy[s] = __int_as_float(e[2 + s]);
                    u[s] = __int_as_float(e[2 + S + s]);
                    // every weight goes into a VGPR once per frame: the
                    // shifted-tap FMAs take their weight from one, and an FMA
                    // with a scalar operand issues at half the rate of one
                    // whose operands are all vector registers
                    asm volatile("" : "+v"(u[s]), "+v"(wy[s]));
                }
                // the lane's slot in exchange row (wv-1)(S-1): the first of
                // the rows this wave leaves for the wave above
                float *xw = xch + (wv - 1) * (S - 1) * 128 + 2 * lane;
                auto put = [&](int xrel, float h0, float h1) {
                    *reinterpret_cast<float2 *>(xw + xrel * 128) = make_float2(h0, h1);
                };
                // rows are read AH ahead of their use (a ring of AH+1)
                constexpr int AH = WS_AHEAD < RPL ? WS_AHEAD : RPL;
                float2 vr[AH + 1];
#pragma unroll
                for (int i = 0; i < AH; ++i)
                    vr[i] = row(i);
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    if (rr + AH < RPL)
                        vr[(rr + AH) % (AH + 1)] = row(rr + AH);
                    const float2 v = vr[rr % (AH + 1)];
                    float h0, h1;
                    horiz_ws<S>(v.x, v.y, u, h0, h1);
                    vert(rr, wy, h0, h1);
                    // this wave's first S-1 rows are the halo of the wave above
                    if constexpr (XCH) {
                        if (rr < S - 1 && wv > 0)
                            put(rr, h0, h1);
                    }
                }
                if constexpr (XCH) {
                    // the S-1 rows below the tile, one per wave
                    if (wv < S - 1) {
                        const float2 v = row(TY + wv - wv * RPL);
                        float h0, h1;
                        horiz_ws<S>(v.x, v.y, u, h0, h1);
                        put((NWAVE - 1) * (S - 1) + wv - (wv - 1) * (S - 1), h0, h1);
                    }
                }
            } else {
                // general stamp: window row rr is stamp row aa of output row
                // rr - aa; tap b of column c is the value at offset c + b - h
                float wt[S * S];
#pragma unroll
                for (int s = 0; s < S * S; ++s)
                    wt[s] = __int_as_float(e[2 + s]);
#pragma unroll
                for (int rr = 0; rr < RPL + S - 1; ++rr) {
                    const float2 v = row(rr);
                    // values at offsets -2..3 from column 2L
                    float val[6];
                    val[0] = (h >= 2) ? lane_prev(v.x) : 0.0f;
                    val[1] = (h >= 1) ? lane_prev(v.y) : 0.0f;
                    val[2] = v.x;
                    val[3] = v.y;
                    val[4] = (h >= 1) ? lane_next(v.x) : 0.0f;
                    val[5] = (h >= 2) ? lane_next(v.y) : 0.0f;
#pragma unroll
                    for (int aa = 0; aa < S; ++aa) {
                        const int o = rr - aa;
                        if (o >= 0 && o < RPL) {
#pragma unroll
                            for (int c = 0; c < 2; ++c) {
                                float sum = part[o][c];
#pragma unroll
                                for (int b = 0; b < S; ++b)
                                    sum = fmaf(wt[aa * S + b], val[c + b - h + 2], sum);
                                part[o][c] = sum;
                            }
                        }
                    }
                }
            }
            // keep the window store (and its wait on the prefetch loads) behind
            // the arithmetic
#pragma unroll
            for (int o = 0; o < RPL; ++o)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    asm volatile("" : "+v"(part[o][c]));
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (XCH) {
                __syncthreads();
                halo(wy);
                store(0, d_next, pre);
                __syncthreads();
            } else {
                store(buf ^ 1, d_next, pre);
                __syncthreads();
            }
            d_cur = d_next;
        };
        for (int k = k0; k < k1; ++k)
            frame(k);
        // frame chunk done: into the FP64 totals
#pragma unroll
        for (int o = 0; o < RPL; ++o)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                acc[o][c] += (double)part[o][c];
                part[o][c] = 0.0f;
            }
    }

    // epilogue: SNR and flux (into the trajectory's row of the slab's
    // maps), and the tile's largest (SNR, -pixel) key
    const int jr = a.jrow[j];
    uint64_t best = 0;
    const bool lane_out = lane >= 1 && lane <= 62;
#pragma unroll
    for (int o = 0; o < RPL; ++o) {
        const int y = ty0 + wv * RPL + o;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int x = tx0 + 2 * lane + c - 2;
            if (lane_out && y < a.H && x < a.W) {
                const double nu = acc[o][c];
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
                const uint64_t key = ((uint64_t)ordered_key(snr) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)p);
                best = key > best ? key : best;
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t o = __shfl_xor(best, off, 64);
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
template <int S, bool SEP, int SRC, int RPL>
__global__ __launch_bounds__(64 * WS_NWAVE) __attribute__((amdgpu_waves_per_eu(4))) void k_search_ws(SearchArgs a)
{
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item < a.n_items)
        search_ws_item<S, SEP, SRC, RPL>(a, item);
}

// A step of the serving loop: block ranges for the work items of several requests.
template <int S, bool SEP, int SRC, int RPL>
__global__ __launch_bounds__(64 * WS_NWAVE) __attribute__((amdgpu_waves_per_eu(4))) void k_search_ws_step(StepArgs s)
{
    int r, item;
    if (step_item(s, r, item))
        search_ws_item<S, SEP, SRC, RPL>(step_args(s, r), item);
}

namespace {

template <int S, bool SEP, int SRC, int RPL>
void launch_ws_kernel(hipStream_t st, const SearchArgs &a, const StepArgs *step, int nblocks)
{
    const dim3 block(64 * WS_NWAVE);
    if (step)
        hipLaunchKernelGGL((k_search_ws_step<S, SEP, SRC, RPL>), dim3(nblocks), block, 0, st, *step);
    else
        hipLaunchKernelGGL((k_search_ws<S, SEP, SRC, RPL>), dim3(xcd_grid(a.n_items)), block, 0, st, a);
}

template <int S, bool SEP, int RPL>
hipError_t launch_ws_src(hipStream_t st, const SearchArgs &a, const StepArgs *step, int nblocks)
{
    if (a.Z4) {
        launch_ws_kernel<S, SEP, SRC_Z, RPL>(st, a, step, nblocks);
    } else {
        switch (a.dtype) {
        case TNO_F32: launch_ws_kernel<S, SEP, TNO_F32, RPL>(st, a, step, nblocks); break;
        case TNO_BF16: launch_ws_kernel<S, SEP, TNO_BF16, RPL>(st, a, step, nblocks); break;
        case TNO_F16: launch_ws_kernel<S, SEP, TNO_F16, RPL>(st, a, step, nblocks); break;
        case TNO_FP8_E4M3: launch_ws_kernel<S, SEP, TNO_FP8_E4M3, RPL>(st, a, step, nblocks); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <int RPL>
hipError_t launch_ws_rpl(hipStream_t st, int S, bool sep, const SearchArgs &a, const StepArgs *step, int nblocks)
{
    switch (S * 2 + (sep ? 1 : 0)) {
    case 3: return launch_ws_src<1, true, RPL>(st, a, step, nblocks);
    case 2: return launch_ws_src<1, false, RPL>(st, a, step, nblocks);
    case 7: return launch_ws_src<3, true, RPL>(st, a, step, nblocks);
    case 6: return launch_ws_src<3, false, RPL>(st, a, step, nblocks);
    case 11: return launch_ws_src<5, true, RPL>(st, a, step, nblocks);
    case 10: return launch_ws_src<5, false, RPL>(st, a, step, nblocks);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_search_ws(hipStream_t st, int S, bool sep, int variant, const SearchArgs &a,
                            const StepArgs *step, int nblocks)
{
    if (!a.Z4 && (a.W % 4 != 0 || !a.R || !a.ivar32 || (a.dtype != TNO_F32 && !a.scales)))
        return hipErrorInvalidValue;
    if (variant == SEARCH_WS)
        return launch_ws_rpl<8>(st, S, sep, a, step, nblocks);
    if (variant == SEARCH_WS4)
        return launch_ws_rpl<4>(st, S, sep, a, step, nblocks);
    return hipErrorInvalidValue;
}

}  // namespace tno
