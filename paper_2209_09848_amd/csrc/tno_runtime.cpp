// tno_runtime.cpp -- host side of the C ABI declared in include/tno_search.h.
//
// Responsibilities: argument validation; the per-request plan (shift bounds,
// padding of the staged stack, trail-kernel layout, tiling, footprint);
// admission against an HBM budget and an in-flight limit; resident residual
// stacks keyed by stack_key with LRU eviction; one device arena per request
// from a block cache; a pool of HIP streams so that concurrently admitted
// requests overlap on the device; the kernel sequence of a request on its
// stream; ticketed completion with HIP events.  Validation and planning touch
// no GPU and back the host-only helpers tno_search_validate / footprint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <numeric>
#include <sstream>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tno_search.h"
#include "tno_internal.h"

namespace {

thread_local char g_last_error[256] = {0};

void set_msg(char *dst, size_t n, const char *fmt, va_list ap)
{
    if (dst && n)
        vsnprintf(dst, n, fmt, ap);
}

struct Fail {
    int code;
    char msg[160];
};

Fail fail(int code, const char *fmt, ...)
{
    Fail f;
    f.code = code;
    va_list ap;
    va_start(ap, fmt);
    set_msg(f.msg, sizeof f.msg, fmt, ap);
    va_end(ap);
    return f;
}

constexpr int PAD_CAP = 512;      // largest zero border of the staged stack, per side
constexpr size_t ALIGN = 256;
// Device bytes of a trajectory slab's normaliser and maps (a slab holds at
// least one trajectory).
constexpr size_t SLAB_BYTES = 4ull << 30;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int dtype)
{
    switch (dtype) {
    case TNO_F32: return 4;
    case TNO_BF16:
    case TNO_F16: return 2;
    case TNO_FP8_E4M3: return 1;
    default: return 0;
    }
}

// Everything derived from a request before any device work.
struct Plan {
    int H = 0, W = 0, T = 0, J = 0, S = 0, h = 0, kind = 0, dtype = 0, k = 0;
    double sigma_px = 0, t_ref = 0;
    bool sep = true;                  // separable (Gaussian) PRF; else the tabulated one
    int table_q = 0, table_n = 0;     // tabulated PRF: samples per pixel, grid side
    bool jitter = false;
    bool dev = false;
    int Pt = 0, Pb = 0, Pl = 0, Pr = 0, Hp = 0, Wp4 = 0;
    // the search reads the caller's stack directly (decode x scale x ivar
    // while staging) instead of a staged FP32 copy Z: reduced-precision
    // storage, stamps 1/3/5, W a multiple of 4, one frame below 2^31 bytes
    bool direct = false;
    std::vector<tno::TrailInfo> trail;
    int64_t n_colmeta = 0, n_kvals = 0;
    int ntx = 0, nty = 0, ntiles = 0;
    int variant = 0, tblock = 1;      // search tile shape and trajectory block of the work order
    int ntiles_max = 0;               // tiles of the smallest shape (sizes the tile-key buffer)
    std::vector<int32_t> perm;        // search order (velocity-sorted)
    // normaliser launches: [0] trails stored by columns, [1] by rows (run in
    // the transposed image); each with its zero-bordered FP64 ivar map
    struct LamLaunch {
        int nj = 0;                    // trajectories (all slabs)
        int Hf = 0, Wf = 0;            // image in the launch's frame
        int ntx = 0, nty = 0;
        int Pyt = 0, Pxl = 0, Hq = 0, Wq = 0;
        size_t o_map = 0;
    } lam[2];
    // Trajectory slabs: consecutive runs of the search order.  The normaliser
    // and the SNR and flux maps exist for one slab at a time, a row per
    // trajectory of the slab in increasing trajectory number; the reductions
    // merge slab after slab, and maps the caller asked for receive each
    // slab's rows.
    struct Slab {
        int a0 = 0, a1 = 0;            // search positions a0 .. a1-1 (perm, rows)
        int joff[2] = {0, 0}, nj[2] = {0, 0};   // its normaliser launches in `jlist`
    };
    std::vector<Slab> slabs;
    int jslab = 0;                    // trajectories of the largest slab
    std::vector<int32_t> rows;        // per slab: its trajectories in increasing order (map rows)
    std::vector<int32_t> jrow;        // [J] row of each trajectory in its slab's maps
    std::vector<int32_t> jlist;       // per slab: trajectories of launch 0, then of launch 1
    int64_t N = 0, n_chunks = 0;
    bool full_snr = false, full_flux = false;   // maps with every trajectory's row (asked for)
    bool own_snr = false, own_flux = false;     // ... held in the arena (host outputs)
    int box = 0, kdet = 0;            // significance window side; detections wanted
    float thr = 0.0f;
    bool stack_in_arena = false;      // host residuals copied into the arena (no stack_key)
    size_t stack_bytes = 0;           // bytes of a resident stack holding these residuals
    // arena layout (byte offsets)
    size_t o_R = 0, o_scales = 0, o_sigma = 0, o_times = 0, o_vel = 0, o_Z = 0, o_iv32 = 0,
           o_iv64 = 0, o_tab32 = 0, o_tab64 = 0, o_trail = 0, o_colmeta = 0, o_kvals = 0,
           o_err = 0, o_lam = 0, o_snr = 0, o_flux = 0, o_tkeys = 0, o_tstate = 0, o_chunks = 0,
           o_cand = 0, o_tmax = 0, o_topk = 0, o_best = 0, o_bestj = 0, o_bestf = 0, o_perm = 0, o_rows = 0,
           o_jrow = 0, o_snr_full = 0, o_flux_full = 0, o_gbuf = 0, o_r1 = 0,
           o_r2 = 0, o_b1 = 0, o_b2 = 0, o_sig = 0, o_det = 0, o_counts = 0, o_prf = 0, o_jit = 0,
           o_jl = 0, bytes = 0;
};

bool finite(double v) { return std::isfinite(v); }

// Checks that need no input values.  Returns code 0 on success.
Fail check_shape(const tno_request *r, const tno_outputs *o)
{
    if (!r)
        return fail(TNO_E_INVAL, "request is NULL");
    if (!o)
        return fail(TNO_E_INVAL, "outputs is NULL");
    if (r->reserved != 0)
        return fail(TNO_E_INVAL, "request.reserved must be 0");
    if (r->height <= 0 || r->width <= 0 || r->n_frames <= 0)
        return fail(TNO_E_INVAL, "height, width and n_frames must be positive");
    if (r->height > 32768 || r->width > 32768)
        return fail(TNO_E_INVAL, "height and width must be <= 32768");
    if (r->n_frames > 65535)
        return fail(TNO_E_INVAL, "n_frames must be <= 65535");
    if (r->n_traj <= 0)
        return fail(TNO_E_INVAL, "n_traj must be >= 1");
    if (r->dtype < TNO_F32 || r->dtype > TNO_FP8_E4M3)
        return fail(TNO_E_INVAL, "unknown dtype %d", r->dtype);
    if (!r->residuals && r->stack_key == 0)
        return fail(TNO_E_INVAL, "residuals is NULL and no stack_key given");
    // residuals, scales and sigma of a resident stack come from its copy
    if (r->residuals && r->dtype != TNO_F32 && !r->tile_scales)
        return fail(TNO_E_INVAL, "tile_scales required for reduced-precision residuals");
    if (r->residuals && !r->sigma)
        return fail(TNO_E_INVAL, "sigma must be non-NULL");
    if (!r->times || !r->velocities)
        return fail(TNO_E_INVAL, "times and velocities must be non-NULL");
    if (r->prf.kind != TNO_PRF_GAUSS_SAMPLED && r->prf.kind != TNO_PRF_GAUSS_INTEGRATED &&
        r->prf.kind != TNO_PRF_TABLE)
        return fail(TNO_E_INVAL, "unknown PRF kind %d", r->prf.kind);
    if (r->prf.stamp < 1 || r->prf.stamp > TNO_MAX_STAMP || (r->prf.stamp % 2) == 0)
        return fail(TNO_E_INVAL, "stamp must be odd and in 1..%d", TNO_MAX_STAMP);
    if (r->prf.reserved != 0)
        return fail(TNO_E_INVAL, "prf.reserved must be 0");
    if (r->prf.kind == TNO_PRF_TABLE) {
        if (!r->prf.table)
            return fail(TNO_E_INVAL, "TNO_PRF_TABLE needs prf.table");
        if (r->prf.table_q < 1 || r->prf.table_q > TNO_MAX_TABLE_Q)
            return fail(TNO_E_INVAL, "prf.table_q must be in 1..%d", TNO_MAX_TABLE_Q);
    } else if (!(r->prf.sigma_px > 0.0) || !finite(r->prf.sigma_px)) {
        return fail(TNO_E_INVAL, "prf.sigma_px must be finite and > 0");
    }
    if (r->top_k < 0 || r->top_k > TNO_MAX_TOPK)
        return fail(TNO_E_INVAL, "top_k must be in 0..%d", TNO_MAX_TOPK);
    if (r->top_k > 0 && !o->topk)
        return fail(TNO_E_INVAL, "top_k > 0 needs outputs.topk");
    if (o->reserved != 0)
        return fail(TNO_E_INVAL, "outputs.reserved must be 0");
    if (r->sig_box < 0 || r->sig_box > 65535 || (r->sig_box > 0 && r->sig_box % 2 == 0))
        return fail(TNO_E_INVAL, "sig_box must be 0 or odd and <= 65535");
    if (r->sig_box > 0 && !std::isfinite(r->sig_threshold))
        return fail(TNO_E_INVAL, "sig_threshold must be finite");
    if (o->max_detections < 0 || o->max_detections > TNO_MAX_DETECTIONS)
        return fail(TNO_E_INVAL, "max_detections must be in 0..%d", TNO_MAX_DETECTIONS);
    if (o->max_detections > 0 && !o->detections)
        return fail(TNO_E_INVAL, "max_detections > 0 needs outputs.detections");
    if ((o->significance || o->max_detections > 0) && r->sig_box == 0)
        return fail(TNO_E_INVAL, "significance outputs need sig_box > 0");
    if ((r->flags & ~(TNO_REQ_DEVICE_PTRS | TNO_REQ_VALIDATE | TNO_REQ_STAGE_FP32)) != 0)
        return fail(TNO_E_INVAL, "unknown request flags 0x%x", r->flags);
    if (!finite(r->t_ref) && !std::isnan(r->t_ref))
        return fail(TNO_E_INVAL, "t_ref must be finite or NaN");
    if ((double)r->n_traj * r->n_frames > 2.0e8)
        return fail(TNO_E_INVAL, "n_traj*n_frames too large");
    const double jhw = (double)r->n_traj * r->height * r->width;
    if (jhw > 4.0e12)
        return fail(TNO_E_INVAL, "n_traj*height*width too large");
    const double items = (double)r->n_traj * ((r->height + 15) / 16) * ((r->width + 63) / 64);
    if (items > 2.0e9)
        return fail(TNO_E_INVAL, "too many (tile, trajectory) work items");
    return fail(TNO_OK, "");
}

// Tile shape of search variant v and trajectory-block size of the work order.
constexpr int DEFAULT_TBLOCK = 16;

// Whether search variant v is built for the plan's stamp: variant 0 serves
// every stamp, the other k_search shapes the stamp of side 5 (separable or
// tabulated), the wave-shift variants stamps 1, 3 and 5 of either kind; a
// stack read in place: the wave-shift variants, and variant 0 for stamp 5.
bool variant_serves(const Plan &p, int v)
{
    if (v == tno::SEARCH_WS || v == tno::SEARCH_WS4)
        return tno::ws_stamp(p.S);
    if (p.direct)
        return v == 0 && p.S == 5;   // the default k_search shape reads stamp-5 stacks in place
    return v == 0 || (v > 0 && v < tno::SEARCH_WS && p.S == 5);
}

bool direct_ok(const Plan &p)
{
    return tno::ws_stamp(p.S) && p.W % 4 == 0 && (double)p.H * p.W * 4.0 < 2147483647.0;
}

int default_variant(const Plan &p)
{
    if (!p.direct)
        return 0;
    return p.S == 5 ? 0 : tno::SEARCH_WS;
}

void set_search_shape(Plan &p, int v, int tblock)
{
    p.variant = v;
    p.ntx = (p.W + tno::search_tx(v) - 1) / tno::search_tx(v);
    p.nty = (p.H + tno::search_ty(v) - 1) / tno::search_ty(v);
    p.ntiles = p.ntx * p.nty;
    p.tblock = std::max(1, std::min(tblock, p.J));
}

// Build the plan from host copies of times, velocities and jitter (NULL: none).
Fail make_plan(const tno_request *r, const tno_outputs *o, const double *times,
               const double *vel, const double *jit, Plan &p, size_t slab_bytes = SLAB_BYTES)
{
    Fail f = check_shape(r, o);
    if (f.code)
        return f;
    p.H = r->height;
    p.W = r->width;
    p.T = r->n_frames;
    p.J = r->n_traj;
    p.S = r->prf.stamp;
    p.h = p.S / 2;
    p.kind = r->prf.kind;
    p.sigma_px = r->prf.sigma_px;
    p.sep = tno::prf_separable(p.kind);
    p.table_q = p.sep ? 0 : r->prf.table_q;
    p.table_n = p.sep ? 0 : (p.S + 1) * p.table_q + 1;
    p.jitter = jit != nullptr;
    // jitter extremes per axis (0 when absent)
    double jxmin = 0, jxmax = 0, jymin = 0, jymax = 0;
    if (jit) {
        for (int k = 0; k < r->n_frames; ++k) {
            const double tx = jit[2 * k], ty = jit[2 * k + 1];
            if (!finite(tx) || !finite(ty) || std::fabs(tx) > 256.0 || std::fabs(ty) > 256.0)
                return fail(TNO_E_INVAL, "jitter[%d] must be finite with |theta| <= 256", k);
            if (k == 0) {
                jxmin = jxmax = tx;
                jymin = jymax = ty;
            }
            jxmin = std::min(jxmin, tx);
            jxmax = std::max(jxmax, tx);
            jymin = std::min(jymin, ty);
            jymax = std::max(jymax, ty);
        }
    }
    p.dtype = r->dtype;
    p.dev = (r->flags & TNO_REQ_DEVICE_PTRS) != 0;
    for (int k = 0; k < p.T; ++k)
        if (!finite(times[k]))
            return fail(TNO_E_INVAL, "times[%d] is not finite", k);
    p.t_ref = std::isnan(r->t_ref) ? times[0] : r->t_ref;
    double dtmin = INFINITY, dtmax = -INFINITY;
    for (int k = 0; k < p.T; ++k) {
        double dt = times[k] - p.t_ref;
        dtmin = std::min(dtmin, dt);
        dtmax = std::max(dtmax, dt);
    }
    if (!finite(dtmin) || !finite(dtmax))
        return fail(TNO_E_INVAL, "time baseline overflows");
    // Shift bounds per trajectory: v*dt is monotone in dt, so its extremes sit
    // at the extreme times; the jitter adds its own extremes; one pixel of
    // margin each side covers the rounding of the sums.
    int gymin = 0, gymax = 0, gxmin = 0, gxmax = 0;
    const int H = p.H, W = p.W, h = p.h, S = p.S;
    p.trail.resize(p.J);
    int64_t coff = 0, voff = 0;
    for (int j = 0; j < p.J; ++j) {
        double vx = vel[2 * j], vy = vel[2 * j + 1];
        if (!finite(vx) || !finite(vy))
            return fail(TNO_E_INVAL, "velocity %d is not finite", j);
        double e[4] = {vx * dtmin, vx * dtmax, vy * dtmin, vy * dtmax};
        for (double d : e)
            if (!(std::fabs(d) < 1.0e9))
                return fail(TNO_E_INVAL, "trajectory %d moves more than 1e9 px", j);
        double x1 = std::floor(std::min(e[0], e[1]) + jxmin + 0.5);
        double x2 = std::floor(std::max(e[0], e[1]) + jxmax + 0.5);
        double y1 = std::floor(std::min(e[2], e[3]) + jymin + 0.5);
        double y2 = std::floor(std::max(e[2], e[3]) + jymax + 0.5);
        int xlo = (int)std::min(x1, x2) - 1, xhi = (int)std::max(x1, x2) + 1;
        int ylo = (int)std::min(y1, y2) - 1, yhi = (int)std::max(y1, y2) + 1;
        gxmin = std::min(gxmin, xlo);
        gxmax = std::max(gxmax, xhi);
        gymin = std::min(gymin, ylo);
        gymax = std::max(gymax, yhi);
        tno::TrailInfo ti{};
        const int qx0 = std::max(xlo - h, -(W - 1)), qx1 = std::min(xhi + h, W - 1);
        const int qy0 = std::max(ylo - h, -(H - 1)), qy1 = std::min(yhi + h, H - 1);
        const int ncols = std::max(0, qx1 - qx0 + 1), nrows = std::max(0, qy1 - qy0 + 1);
        // a box wider than tall is stored by rows: its runs along x are the
        // long ones, and the normaliser reloads ivar once per run
        ti.tr = ncols > nrows ? 1 : 0;
        // frames whose stamp covers one major line have |v_m dt + theta_m - q| <= h + 1/2:
        // a time span of (S + jitter range along it) / |v_m|, over which the
        // minor anchor moves by |v_n| times that plus its jitter range
        const double vm = ti.tr ? vy : vx, vn = ti.tr ? vx : vy;
        const double jm = ti.tr ? jymax - jymin : jxmax - jxmin, jn = ti.tr ? jxmax - jxmin : jymax - jymin;
        ti.qx0 = ti.tr ? qy0 : qx0;
        ti.ncols = ti.tr ? nrows : ncols;
        ti.qy_lo = ti.tr ? qx0 : qy0;
        ti.qy_hi = ti.tr ? qx1 : qy1;
        int cap = ti.tr ? ncols : nrows;
        if (vm != 0.0) {
            double c = std::ceil((double)S + ((double)S + jm) * std::fabs(vn) / std::fabs(vm) + jn) + 3.0;
            if (c < (double)cap)
                cap = (int)c;
        }
        ti.cap = (int)align_up((size_t)std::max(cap, 1), tno::LAMBDA_CHUNK);   // whole chunks
        ti.col_off = coff;
        ti.val_off = voff;
        coff += ti.ncols;
        voff += (int64_t)ti.ncols * ti.cap;
        p.trail[j] = ti;
    }
    p.n_colmeta = std::max<int64_t>(coff, 1);
    p.n_kvals = std::max<int64_t>(voff, 1);
    p.Pt = std::min(PAD_CAP, std::max(0, -gymin) + h);
    p.Pb = std::min(PAD_CAP, std::max(0, gymax) + h + tno::SEARCH_MAX_TY);
    p.Pl = (int)align_up((size_t)std::min(PAD_CAP, std::max(0, -gxmin) + h + 3), 4);
    p.Pr = std::min(PAD_CAP, std::max(0, gxmax) + h + tno::SEARCH_MAX_TX + 4);
    p.Hp = H + p.Pt + p.Pb;
    p.Wp4 = (int)(align_up((size_t)W + p.Pl + p.Pr, 4) / 4);
    // reduced-precision stacks are searched in place (no FP32 copy) where
    // the wave-shift search serves the stamp, unless the caller asks for the
    // staged copy
    p.direct = p.dtype != TNO_F32 && (r->flags & TNO_REQ_STAGE_FP32) == 0 && direct_ok(p);
    // untuned default: the first tile shape, also for a stack read in place
    // with stamp 5 (other stamps: the wave-shift shape).  Its tiles are 128
    // columns wide against the wave-shift kernel's 124, which wastes 45 % of
    // a 256-px cutout (3 tiles), and it reads FP8 faster: on the serving mix
    // BF16 p99 242-261 against 283-298 ms, on the FFI workload FP8 238
    // against 272 ms (BF16 261 against 255).  Trajectories in blocks of 16
    // (on the 100-trajectory FFI bank 2.7 % faster than one block of all, and
    // blocks of 8 are 25 % slower: fewer trajectories of a tile run together
    // and share its windows in L2)
    set_search_shape(p, default_variant(p), DEFAULT_TBLOCK);
    p.ntiles_max = ((W + 63) / 64) * ((H + 15) / 16);
    // search order: trajectories adjacent in the work order should have nearby
    // shifts, so that the windows of a tile's co-resident blocks share cache
    // lines.  Two candidate orders: the Morton (Z-order) code of the quantised
    // velocity, and direction then speed.  Each is scored by the summed
    // bounding box of the windows of every trajectory block at 8 times over
    // the span (the footprint its blocks read together); the direction order
    // is taken only when its footprint is smaller.  (Morton suits banks of
    // many close speeds such as nested shells; a polar grid of few speeds over
    // wide directions does better by direction.)
    {
        double vxmin = INFINITY, vxmax = -INFINITY, vymin = INFINITY, vymax = -INFINITY;
        for (int j = 0; j < p.J; ++j) {
            vxmin = std::min(vxmin, vel[2 * j]);
            vxmax = std::max(vxmax, vel[2 * j]);
            vymin = std::min(vymin, vel[2 * j + 1]);
            vymax = std::max(vymax, vel[2 * j + 1]);
        }
        std::vector<uint32_t> code(p.J);
        for (int j = 0; j < p.J; ++j) {
            auto q = [](double v, double lo, double hi) -> uint32_t {
                return hi > lo ? (uint32_t)std::min(65535.0, std::floor((v - lo) / (hi - lo) * 65535.0)) : 0u;
            };
            uint32_t a = q(vel[2 * j], vxmin, vxmax), b = q(vel[2 * j + 1], vymin, vymax), c = 0;
            for (int bit = 0; bit < 16; ++bit)
                c |= (((a >> bit) & 1u) << (2 * bit)) | (((b >> bit) & 1u) << (2 * bit + 1));
            code[j] = c;
        }
        p.perm.resize(p.J);
        std::iota(p.perm.begin(), p.perm.end(), 0);
        std::stable_sort(p.perm.begin(), p.perm.end(), [&](int32_t x, int32_t y) { return code[x] < code[y]; });
        std::vector<int32_t> dir(p.J);
        std::vector<double> ang(p.J), spd(p.J);
        for (int j = 0; j < p.J; ++j) {
            ang[j] = std::atan2(vel[2 * j + 1], vel[2 * j]);
            spd[j] = std::hypot(vel[2 * j], vel[2 * j + 1]);
        }
        std::iota(dir.begin(), dir.end(), 0);
        std::stable_sort(dir.begin(), dir.end(), [&](int32_t x, int32_t y) {
            return ang[x] < ang[y] || (ang[x] == ang[y] && spd[x] < spd[y]);
        });
        const double wx = tno::search_tx(p.variant) + p.S - 1, wy = tno::search_ty(p.variant) + p.S - 1;
        auto footprint = [&](const std::vector<int32_t> &ord) {
            double area = 0.0;
            for (int b0 = 0; b0 < p.J; b0 += p.tblock) {
                const int b1 = std::min(p.J, b0 + p.tblock);
                for (int i = 0; i < 8; ++i) {
                    const double t = dtmin + (dtmax - dtmin) * i / 7.0;
                    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
                    for (int m = b0; m < b1; ++m) {
                        const double sx = vel[2 * ord[m]] * t, sy = vel[2 * ord[m] + 1] * t;
                        x0 = std::min(x0, sx);
                        x1 = std::max(x1, sx);
                        y0 = std::min(y0, sy);
                        y1 = std::max(y1, sy);
                    }
                    area += (wx + x1 - x0) * (wy + y1 - y0);
                }
            }
            return area;
        };
        if (footprint(dir) < footprint(p.perm))
            p.perm = dir;
    }
    for (int o = 0; o < 2; ++o) {
        auto &L = p.lam[o];
        L.nj = 0;
        L.Hf = o ? W : H;
        L.Wf = o ? H : W;
        L.ntx = (L.Wf + tno::LAMBDA_TX - 1) / tno::LAMBDA_TX;
        L.nty = (L.Hf + tno::LAMBDA_TY - 1) / tno::LAMBDA_TY;
        // In the launch's frame the normaliser reads ivar at x + q (x below
        // ntx * TX, q a major offset of a box) and, along a run [lo, lo +
        // len) of minor offsets inside [qy_lo, qy_hi], rows y0 + lo ... y0 +
        // lo + roundC(len) + R - 2 (C = LAMBDA_CHUNK) for a wave whose first
        // row y0 is at most nty * TY - R, i.e. at most nty * TY + qy_hi + C -
        // 2.  The border covers them all (every slab's launches).
        int qxmin = 0, qxmax = 0, qymin = 0, qymax = 0;
        for (int j = 0; j < p.J; ++j) {
            const auto &ti = p.trail[j];
            if (ti.tr != o)
                continue;
            ++L.nj;
            if (ti.ncols <= 0)
                continue;
            qxmin = std::min(qxmin, ti.qx0);
            qxmax = std::max(qxmax, ti.qx0 + ti.ncols - 1);
            qymin = std::min(qymin, ti.qy_lo);
            qymax = std::max(qymax, ti.qy_hi);
        }
        if ((double)L.ntx * L.nty * L.nj > 2.0e9)
            return fail(TNO_E_INVAL, "too many normaliser work items");
        L.Pxl = -qxmin;
        const int pxr = std::max(0, L.ntx * tno::LAMBDA_TX + qxmax - L.Wf);
        L.Pyt = -qymin;
        const int pyb = std::max(0, L.nty * tno::LAMBDA_TY + qymax + tno::LAMBDA_CHUNK - 1 - L.Hf);
        L.Wq = L.Wf + L.Pxl + pxr;
        L.Hq = L.Hf + L.Pyt + pyb;
    }
    p.box = r->sig_box;
    p.thr = r->sig_threshold;
    p.kdet = (int)std::min<int64_t>(o->max_detections, (int64_t)p.H * p.W);
    p.full_snr = o->snr != nullptr;
    p.full_flux = o->flux != nullptr;
    p.own_snr = p.full_snr && !p.dev;
    p.own_flux = p.full_flux && !p.dev;
    // trajectory slabs: runs of the search order, as many trajectories per
    // slab as keep Lam and the slab's maps within slab_bytes, in whole
    // trajectory blocks of the work order where a slab holds one or more
    // (each block of a launch reads the stack once: a slab cut through a
    // block would make one more pass over it)
    {
        const size_t per = (size_t)H * W * 16;
        int js = (int)std::max<size_t>(1, std::min<size_t>((size_t)p.J, slab_bytes / per));
        if (js < p.J && js >= DEFAULT_TBLOCK)
            js = js / DEFAULT_TBLOCK * DEFAULT_TBLOCK;
        const int ns = (p.J + js - 1) / js;
        p.jslab = js;
        p.slabs.assign(ns, Plan::Slab{});
        p.rows.assign(p.perm.begin(), p.perm.end());
        p.jrow.assign(p.J, 0);
        p.jlist.clear();
        for (int s = 0; s < ns; ++s) {
            auto &sl = p.slabs[s];
            sl.a0 = s * p.jslab;
            sl.a1 = std::min(p.J, sl.a0 + p.jslab);
            std::sort(p.rows.begin() + sl.a0, p.rows.begin() + sl.a1);
            for (int a = sl.a0; a < sl.a1; ++a)
                p.jrow[p.rows[a]] = a - sl.a0;
            for (int o2 = 0; o2 < 2; ++o2) {
                sl.joff[o2] = (int)p.jlist.size();
                for (int a = sl.a0; a < sl.a1; ++a)
                    if (p.trail[p.rows[a]].tr == o2)
                        p.jlist.push_back(p.rows[a]);
                sl.nj[o2] = (int)p.jlist.size() - sl.joff[o2];
                // the normaliser's work items run tile by tile with these
                // trajectories fastest: the costliest trail kernels (major
                // lines x run capacity) first, so that the items dispatched
                // last are the short ones and the launch ends with a short tail
                auto cost = [&](int32_t j) { return (int64_t)p.trail[j].ncols * (p.trail[j].cap + 31); };
                std::stable_sort(p.jlist.begin() + sl.joff[o2], p.jlist.end(),
                                 [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
            }
        }
    }
    p.N = (int64_t)p.J * H * W;
    p.k = (int)std::min<int64_t>(r->top_k, p.N);
    p.n_chunks = ((int64_t)p.jslab * H * W + tno::TOPK_CHUNK - 1) / tno::TOPK_CHUNK;

    // arena layout
    const size_t HW = (size_t)H * W, T = (size_t)p.T, J = (size_t)p.J;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + std::max<size_t>(bytes, 1), ALIGN);
        return at;
    };
    const size_t scale_bytes = p.dtype == TNO_F32 ? 0 : T * ((H + 63) / 64) * ((W + 63) / 64) * 4;
    p.stack_bytes = align_up(T * HW * elem_bytes(p.dtype), ALIGN) + align_up(scale_bytes, ALIGN) +
                    align_up(HW * 4, ALIGN);
    p.stack_in_arena = !p.dev && r->stack_key == 0;
    if (p.stack_in_arena) {
        p.o_R = take(T * HW * elem_bytes(p.dtype));
        if (scale_bytes)
            p.o_scales = take(scale_bytes);
        p.o_sigma = take(HW * 4);
    }
    if (!p.dev) {
        p.o_times = take(T * 8);
        p.o_vel = take(J * 16);
        if (p.jitter)
            p.o_jit = take(T * 16);
        if (!p.sep)
            p.o_prf = take((size_t)p.table_n * p.table_n * 8);
    }
    if (!p.direct)
        p.o_Z = take(T * (size_t)p.Hp * p.Wp4 * 16);
    p.o_iv32 = take(HW * 4);
    for (auto &L : p.lam)
        L.o_map = L.nj > 0 || &L == &p.lam[0] ? take((size_t)L.Hq * L.Wq * 8) : 0;
    p.o_jl = take(J * 4);
    p.o_tab32 = take(J * T * tno::table_stride(S, p.sep) * 4);
    p.o_tab64 = take(J * T * tno::table64_stride(S, p.sep) * 8);
    p.o_trail = take(J * sizeof(tno::TrailInfo));
    p.o_colmeta = take((size_t)p.n_colmeta * 8);
    p.o_kvals = take((size_t)p.n_kvals * 8);
    p.o_err = take(4);
    const size_t JS = (size_t)p.jslab;
    p.o_lam = take(JS * HW * 8);
    p.o_snr = take(JS * HW * 4);
    p.o_flux = take(JS * HW * 4);
    if (p.own_snr)
        p.o_snr_full = take(J * HW * 4);
    if (p.own_flux)
        p.o_flux_full = take(J * HW * 4);
    p.o_tkeys = take(J * p.ntiles_max * 8);
    p.o_perm = take(J * 4);
    p.o_rows = take(J * 4);
    p.o_jrow = take(J * 4);
    p.o_tstate = take(sizeof(tno::TopkState));
    p.o_chunks = take((size_t)p.n_chunks * 4);
    p.o_cand = take((size_t)TNO_MAX_TOPK * 16);
    p.o_gbuf = take((size_t)tno::TOPK_GATHER_CAP * 16);
    p.o_tmax = take(J * sizeof(tno_peak));
    p.o_topk = take((size_t)TNO_MAX_TOPK * sizeof(tno_candidate));
    p.o_best = take(HW * 4);
    p.o_bestj = take(HW * 4);
    p.o_bestf = take(HW * 4);
    p.o_counts = take(16);
    if (p.box > 0) {
        p.o_r1 = take(HW * 8);
        p.o_r2 = take(HW * 8);
        p.o_b1 = take((size_t)tno::significance_block_values(H, W) * 8);
        p.o_b2 = take((size_t)tno::significance_block_values(H, W) * 8);
        p.o_sig = take(HW * 4);
        p.o_det = take((size_t)TNO_MAX_DETECTIONS * sizeof(tno_detection));
    }
    p.bytes = off;
    return fail(TNO_OK, "");
}

// A residual stack kept on the device under a caller's stack_key: codes or
// FP32 residuals, tile scales, sigma.  Requests reference it while in flight.
struct Stack {
    uint64_t key = 0;
    int H = 0, W = 0, T = 0, dtype = 0;
    void *block = nullptr;
    size_t block_bytes = 0;
    size_t bytes = 0;          // bytes counted against the budget
    size_t o_R = 0, o_scales = 0, o_sigma = 0;
    int refs = 0;
    uint64_t last_use = 0;
    hipEvent_t ready = nullptr;
};

struct Request {
    uint64_t ticket = 0;
    Plan plan;
    tno_outputs out{};
    void *arena = nullptr;
    size_t arena_bytes = 0;
    Stack *stack = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev[6] = {};   // ev[0] start, ev[1] weighting done, ev[2] table and trail done, ev[5] end
    // per slab s: sev[3s] normaliser start, sev[3s+1] its end (search start),
    // sev[3s+2] search end
    std::vector<hipEvent_t> sev;
    std::chrono::steady_clock::time_point t_submit;
    uint64_t updates = 0;
    hipGraphExec_t exec = nullptr;   // graph mode: the executable graph this request ran
    std::string exec_key;
    bool cancelled = false;          // tno_search_cancel: no outputs copied, poll gives CANCELLED
    const void *src_R = nullptr;     // the residual stack on the device (set when enqueued)
    const float *src_scales = nullptr;
    // TNO_CFG_BATCH: end of the preparation on `stream`, and the next search
    // work item not yet handed to a step
    hipEvent_t prep_done = nullptr;
    int slab = 0;                    // the slab being searched
    int next_item = 0;               // (of that slab)
    bool end_recorded = false;       // ev[5] recorded (a batched request records it late)
};

// Device arenas of finished requests, kept for reuse: a later request takes
// the smallest cached block that fits, so steady-state serving and repeated
// searches of one shape allocate nothing.  Blocks are freed when the cached
// total would exceed the handle's budget, on allocation failure, and at
// destroy.
struct ArenaCache {
    std::multimap<size_t, void *> blocks;
    size_t held = 0;
    void *take(size_t bytes, size_t *got)
    {
        // a cached block is already counted against the budget (as cached),
        // so taking a larger one than asked for moves bytes from `held` to
        // the taker's count without raising the total
        auto it = blocks.lower_bound(bytes);
        if (it == blocks.end() || it->first > 2 * bytes + (64u << 20))
            return nullptr;
        void *p = it->second;
        *got = it->first;
        held -= it->first;
        blocks.erase(it);
        return p;
    }
    void put(void *p, size_t bytes)
    {
        blocks.emplace(bytes, p);
        held += bytes;
    }
    void trim(size_t keep)
    {
        while (held > keep && !blocks.empty()) {
            auto it = blocks.begin();      // drop the smallest first
            (void)hipFree(it->second);
            held -= it->first;
            blocks.erase(it);
        }
    }
};

}  // namespace

constexpr int STREAM_POOL = 4;   // at the default priority
// TNO_CFG_BATCH: step size (blocks), requests per step, step descriptor slots
#ifndef TNO_STEP_BLOCKS
#define TNO_STEP_BLOCKS 8192
#endif
#ifndef TNO_STEP_CHUNK_MIN
#define TNO_STEP_CHUNK_MIN 1024
#endif
constexpr int STEP_BLOCKS = TNO_STEP_BLOCKS;
constexpr int STEP_ENTRIES = 32;
constexpr int STEP_SLOTS = 4;
constexpr int STEP_CHUNK_MIN = TNO_STEP_CHUNK_MIN;   // smallest chunk a request gets in a shared step
constexpr int STEP_OLDEST_QUARTERS = 2;               // quarters of a shared step for the oldest request

struct tno_search {
    int device = 0;
    std::vector<hipStream_t> streams;
    bool own_streams = false;
    // TNO_CFG_RESERVE: the budget as one device block, arenas and resident
    // stacks carved from it (no device allocation or free after create)
    void *pool_base = nullptr;
    tno::OffsetPool pool;
    unsigned next_stream = 0;
    uint64_t budget = 0;
    uint64_t in_use = 0;               // device blocks held by live requests and resident stacks
                                       // (their actual sizes, so in_use + cache.held is what
                                       // the handle holds on the device)
    int max_inflight = 64;
    size_t slab_bytes = SLAB_BYTES;    // device bytes of a request's trajectory slab
    uint64_t next_ticket = 1;
    uint64_t tick = 0;
    std::mutex mu;
    std::map<uint64_t, Request *> live;
    std::map<uint64_t, Stack *> stacks;
    ArenaCache cache;
    // tuning table: shape class -> (variant, trajectory block, probe updates/s)
    struct Tuned {
        int variant, tblock;
        double rate;
    };
    bool autotune = false;
    bool graphs = false;
    // executable graphs not in flight, by request structure (graph_key)
    std::multimap<std::string, hipGraphExec_t> free_execs;
    std::string arch;
    std::string tune_path;
    std::map<std::string, Tuned> tuned;
    uint64_t n_alloc = 0;              // fresh device allocations attempted by get_block
    uint64_t fault_alloc = 0;          // TNO_FAULT=alloc:N: the N-th attempt fails (0: never)
    // TNO_CFG_BATCH: requests whose search items are not all launched (FIFO),
    // the two search streams, and the step descriptor slots (device table +
    // pinned host staging, busy until the step's event completes)
    bool batch = false;
    std::deque<Request *> ready;
    hipStream_t sstream[2] = {nullptr, nullptr};
    unsigned next_sstream = 0;
    struct StepSlot {
        void *dev = nullptr;
        void *host = nullptr;
        hipEvent_t done = nullptr;
        bool busy = false;
    } slots[STEP_SLOTS];
    uint64_t n_steps = 0, n_step_items = 0, n_shared = 0;

    void load_tuning()
    {
        std::ifstream f(tune_path);
        std::string line;
        while (std::getline(f, line)) {
            if (line.empty() || line[0] == '#')
                continue;
            std::istringstream ss(line);
            std::string a, cls, vname;
            int tb = 0;
            double rate = 0;
            if (!(ss >> a >> cls >> vname >> tb >> rate) || a != arch)
                continue;
            for (int v = 0; v < tno::N_SEARCH_VARIANTS; ++v)
                if (vname == tno::SEARCH_VARIANTS[v].name)
                    tuned[cls] = {v, tb, rate};
        }
    }
    void save_tuning() const
    {
        if (tune_path.empty())
            return;
        std::ofstream f(tune_path, std::ios::trunc);
        f << "# tno_search tuning cache: arch shape-class variant trajectory-block probe-updates/s\n";
        for (auto &kv : tuned)
            f << arch << " " << kv.first << " " << tno::SEARCH_VARIANTS[kv.second.variant].name << " "
              << kv.second.tblock << " " << kv.second.rate << "\n";
    }
};

namespace {

void set_last(const Fail &f) { snprintf(g_last_error, sizeof g_last_error, "%s", f.msg); }

int hip_fail(hipError_t e, const char *what, char *msg, size_t n)
{
    if (msg)
        snprintf(msg, n, "%s: %s", what, hipGetErrorString(e));
    snprintf(g_last_error, sizeof g_last_error, "%s: %s", what, hipGetErrorString(e));
    return TNO_E_DEVICE;
}

template <class T> T *at(void *arena, size_t off) { return (T *)((char *)arena + off); }

// A block no longer held: back to the reserved block's free ranges, or to
// the cache of blocks kept for reuse.
void keep_block(tno_search *h, void *p, size_t bytes)
{
    if (h->pool_base)
        h->pool.give((size_t)((char *)p - (char *)h->pool_base), bytes);
    else
        h->cache.put(p, bytes);
}

// Make `need` bytes of budget available: evict idle resident stacks (least
// recently used first), then shrink the block cache so that live memory plus
// cached blocks stay within the budget.  Returns false if it cannot.
bool make_room(tno_search *h, size_t need)
{
    while (h->in_use + need > h->budget) {
        Stack *victim = nullptr;
        for (auto &kv : h->stacks)
            if (kv.second->refs == 0 && (!victim || kv.second->last_use < victim->last_use))
                victim = kv.second;
        if (!victim)
            return false;
        h->stacks.erase(victim->key);
        keep_block(h, victim->block, victim->block_bytes);
        h->in_use -= victim->bytes;
        if (victim->ready)
            (void)hipEventDestroy(victim->ready);
        delete victim;
    }
    h->cache.trim(h->budget - h->in_use - need);
    return true;
}

// Drop the least recently used idle resident stack (its block is freed).
// Returns false if every resident stack is in use.
bool evict_one(tno_search *h)
{
    Stack *victim = nullptr;
    for (auto &kv : h->stacks)
        if (kv.second->refs == 0 && (!victim || kv.second->last_use < victim->last_use))
            victim = kv.second;
    if (!victim)
        return false;
    h->stacks.erase(victim->key);
    if (h->pool_base)
        keep_block(h, victim->block, victim->block_bytes);
    else
        (void)hipFree(victim->block);
    h->in_use -= victim->bytes;
    if (victim->ready)
        (void)hipEventDestroy(victim->ready);
    delete victim;
    return true;
}

// A device block of at least `bytes` from the cache, else hipMalloc.  The
// device can be short of memory inside the budget (other users of the GPU):
// then the cached blocks are freed, then idle resident stacks one at a time,
// before the allocation is given up.
void *get_block(tno_search *h, size_t bytes, size_t *got)
{
    if (h->pool_base) {
        // reserved: a range of the handle's block (idle resident stacks give
        // theirs back, least recently used first, when none fits)
        if (++h->n_alloc == h->fault_alloc)
            return nullptr;           // injected failure (TNO_FAULT=alloc:N)
        for (;;) {
            const size_t off = h->pool.take(bytes, got);
            if (off != tno::OffsetPool::NONE)
                return (char *)h->pool_base + off;
            if (!evict_one(h))
                return nullptr;
        }
    }
    void *p = h->cache.take(bytes, got);
    if (p)
        return p;
    if (++h->n_alloc == h->fault_alloc)
        return nullptr;               // injected failure (TNO_FAULT=alloc:N)
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        h->cache.trim(0);
        while (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (!evict_one(h))
                return nullptr;
        }
    }
    *got = bytes;
    return p;
}

struct Inputs {
    const void *R;
    const float *scales;
    const float *sigma;
    const double *times;
    const double *vel;
    const double *jit;       // NULL: no jitter
    const double *prf_tab;   // tabulated PRF grid, or NULL
};

Inputs inputs_of(const Request *q, const tno_request *r)
{
    const Plan &p = q->plan;
    void *A = q->arena;
    Inputs in;
    if (q->stack) {
        void *B = q->stack->block;
        in.R = at<void>(B, q->stack->o_R);
        in.scales = p.dtype == TNO_F32 ? nullptr : at<float>(B, q->stack->o_scales);
        in.sigma = at<float>(B, q->stack->o_sigma);
    } else if (p.stack_in_arena) {
        in.R = at<void>(A, p.o_R);
        in.scales = p.dtype == TNO_F32 ? nullptr : at<float>(A, p.o_scales);
        in.sigma = at<float>(A, p.o_sigma);
    } else {
        in.R = r->residuals;
        in.scales = p.dtype == TNO_F32 ? nullptr : r->tile_scales;
        in.sigma = r->sigma;
    }
    in.times = p.dev ? r->times : at<double>(A, p.o_times);
    in.vel = p.dev ? r->velocities : at<double>(A, p.o_vel);
    in.jit = !p.jitter ? nullptr : p.dev ? r->jitter : at<double>(A, p.o_jit);
    in.prf_tab = p.sep ? nullptr : p.dev ? r->prf.table : at<double>(A, p.o_prf);
    return in;
}

#define TRY(x)                  \
    do {                        \
        e = (x);                \
        if (e != hipSuccess)    \
            return e;           \
    } while (0)

// The maps of the slab being searched (a row per trajectory of the slab),
// and the maps with a row per trajectory that the caller asked for (the
// caller's device maps, or the arena's copies of host maps), or NULL.
float *snr_rows(const Request *q) { return at<float>(q->arena, q->plan.o_snr); }
float *flux_rows(const Request *q) { return at<float>(q->arena, q->plan.o_flux); }
float *snr_full(const Request *q)
{
    const Plan &p = q->plan;
    return !p.full_snr ? nullptr : p.own_snr ? at<float>(q->arena, p.o_snr_full) : q->out.snr;
}
float *flux_full(const Request *q)
{
    const Plan &p = q->plan;
    return !p.full_flux ? nullptr : p.own_flux ? at<float>(q->arena, p.o_flux_full) : q->out.flux;
}

// Search arguments of slab s (its first nframes frames, every kstride-th).
tno::SearchArgs search_args(const Request *q, int s, int nframes, int kstride = 1)
{
    const Plan &p = q->plan;
    const Plan::Slab &sl = p.slabs[s];
    void *A = q->arena;
    tno::SearchArgs sa;
    sa.Z4 = p.direct ? nullptr : at<float4>(A, p.o_Z);
    sa.R = q->src_R;
    sa.scales = q->src_scales;
    sa.ivar32 = at<float>(A, p.o_iv32);
    sa.dtype = p.dtype;
    sa.nqy = (p.H + TNO_QTILE - 1) / TNO_QTILE;
    sa.nqx = (p.W + TNO_QTILE - 1) / TNO_QTILE;
    sa.tab32 = at<int32_t>(A, p.o_tab32);
    sa.lam = at<double>(A, p.o_lam);
    sa.snr = snr_rows(q);
    sa.flux = flux_rows(q);
    sa.tile_keys = at<uint64_t>(A, p.o_tkeys);
    sa.perm = at<int32_t>(A, p.o_perm) + sl.a0;
    sa.jrow = at<int32_t>(A, p.o_jrow);
    sa.H = p.H;
    sa.W = p.W;
    sa.T = p.T;
    sa.J = sl.a1 - sl.a0;
    sa.Hp = p.Hp;
    sa.Wp4 = p.Wp4;
    sa.Pt = p.Pt;
    sa.Pl = p.Pl;
    sa.ntx = p.ntx;
    sa.nty = p.nty;
    sa.n_items = p.ntiles * sa.J;
    sa.tblock = std::min(p.tblock, sa.J);
    sa.nframes = nframes;
    sa.kstride = kstride;
    return sa;
}

// Enqueue what precedes the kernels: the wait on a resident stack's upload,
// the start event, and the host-side trail layout and search order.  (Kept
// out of a captured graph: host-to-device copies and cross-stream waits.)
hipError_t enqueue_pre(Request *q)
{
    const Plan &p = q->plan;
    hipStream_t st = q->stream;
    void *A = q->arena;
    hipError_t e;
    if (q->stack && q->stack->ready)
        TRY(hipStreamWaitEvent(st, q->stack->ready, 0));
    TRY(hipEventRecord(q->ev[0], st));
    TRY(hipMemcpyAsync(at<void>(A, p.o_trail), p.trail.data(), p.trail.size() * sizeof(tno::TrailInfo),
                       hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync(at<void>(A, p.o_perm), p.perm.data(), p.perm.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync(at<void>(A, p.o_jl), p.jlist.data(), p.jlist.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync(at<void>(A, p.o_rows), p.rows.data(), p.rows.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync(at<void>(A, p.o_jrow), p.jrow.data(), p.jrow.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, st));
    return hipSuccess;
}

hipError_t enqueue_lambda(Request *q, int s, bool events);

// Enqueue the kernels before the numerator search: weighting, table, trail,
// the first slab's Lam; `events`: record the phase boundaries (not inside a
// captured graph).
hipError_t enqueue_front(Request *q, const tno_request *r, bool events)
{
    const Plan &p = q->plan;
    hipStream_t st = q->stream;
    void *A = q->arena;
    const Inputs in = inputs_of(q, r);
    hipError_t e;
    q->src_R = in.R;
    q->src_scales = in.scales;
    TRY(tno::launch_zero(st, at<int32_t>(A, p.o_err), 1));
    for (int o = 0; o < 2; ++o) {
        const auto &L = p.lam[o];
        if (o == 0 || L.nj > 0)
            TRY(tno::launch_ivar(st, p.H, p.W, in.sigma, o == 0 ? at<float>(A, p.o_iv32) : nullptr,
                                 at<double>(A, L.o_map), L.Hq, L.Wq, L.Pyt, L.Pxl, o, at<int32_t>(A, p.o_err)));
    }
    if (!p.direct)
        TRY(tno::launch_prep_z(st, p.dtype, in.R, in.scales, at<float>(A, p.o_iv32), at<float4>(A, p.o_Z),
                               p.T, p.H, p.W, p.Hp, p.Wp4, p.Pt, p.Pl));
    if (events)
        TRY(hipEventRecord(q->ev[1], st));
    const tno::PrfSpec prf{p.kind, p.S, p.sigma_px, in.prf_tab, p.table_q};
    TRY(tno::launch_table(st, p.J, p.T, in.times, p.t_ref, in.vel, in.jit, prf,
                          at<int32_t>(A, p.o_tab32), at<double>(A, p.o_tab64)));
    TRY(tno::launch_trail(st, p.J, p.T, p.S, p.sep, at<int32_t>(A, p.o_tab32), at<double>(A, p.o_tab64),
                          at<tno::TrailInfo>(A, p.o_trail), at<int2>(A, p.o_colmeta),
                          at<double>(A, p.o_kvals), at<int32_t>(A, p.o_err)));
    if (events)
        TRY(hipEventRecord(q->ev[2], st));
    return enqueue_lambda(q, 0, events);
}

// The normaliser of slab s (into the slab's Lam rows); `events`: record its
// start and end.
hipError_t enqueue_lambda(Request *q, int s, bool events)
{
    const Plan &p = q->plan;
    const Plan::Slab &sl = p.slabs[s];
    hipStream_t st = q->stream;
    void *A = q->arena;
    hipError_t e;
    if (events)
        TRY(hipEventRecord(q->sev[3 * s], st));
    tno::LambdaArgs las[2];
    for (int o = 0; o < 2; ++o) {
        const auto &L = p.lam[o];
        tno::LambdaArgs &la = las[o];
        la.info = at<tno::TrailInfo>(A, p.o_trail);
        la.colmeta = at<int2>(A, p.o_colmeta);
        la.kvals = at<double>(A, p.o_kvals);
        la.ivar64 = at<double>(A, L.o_map);
        la.lam = at<double>(A, p.o_lam);
        la.jrow = at<int32_t>(A, p.o_jrow);
        la.jlist = at<int32_t>(A, p.o_jl) + sl.joff[o];
        la.H = L.Hf;
        la.W = L.Wf;
        la.H0 = p.H;
        la.W0 = p.W;
        la.nj = sl.nj[o];
        la.ntx = L.ntx;
        la.nty = L.nty;
        la.n_items = L.ntx * L.nty * sl.nj[o];
        la.Pyt = L.Pyt;
        la.Pxl = L.Pxl;
        la.Wq = L.Wq;
        la.tr = o;
    }
    TRY(tno::launch_lambda(st, las[0], las[1]));
    if (events)
        TRY(hipEventRecord(q->sev[3 * s + 1], st));
    return hipSuccess;
}

// Enqueue the search of every slab with its reductions (the first slab's
// Lam is already enqueued), then the significance pass and output copies;
// `events`: record the phase boundaries and the end event.
hipError_t enqueue_slab_reduce(Request *q, int s);
hipError_t enqueue_final(Request *q, bool events);

hipError_t enqueue_back(Request *q, bool events)
{
    const Plan &p = q->plan;
    hipError_t e;
    for (int s = 0; s < (int)p.slabs.size(); ++s) {
        if (s > 0)
            TRY(enqueue_lambda(q, s, events));
        TRY(tno::launch_search(q->stream, p.S, p.sep, p.variant, search_args(q, s, p.T)));
        if (events)
            TRY(hipEventRecord(q->sev[3 * s + 2], q->stream));
        TRY(enqueue_slab_reduce(q, s));
    }
    return enqueue_final(q, events);
}

// After slab s's search (on the request's stream): its rows into the maps
// the caller asked for, its trajectories' peaks, and the bank maximum and
// top-k merged with the slab's maps.
hipError_t enqueue_slab_reduce(Request *q, int s)
{
    const Plan &p = q->plan;
    const Plan::Slab &sl = p.slabs[s];
    hipStream_t st = q->stream;
    void *A = q->arena;
    const int nj = sl.a1 - sl.a0;
    const int64_t HW = (int64_t)p.H * p.W;
    const int32_t *rows = at<int32_t>(A, p.o_rows) + sl.a0;
    const float *snr = snr_rows(q);
    const float *flux = flux_rows(q);
    hipError_t e;
    if (p.full_snr)
        TRY(tno::launch_rows_out(st, nj, HW, rows, snr, snr_full(q)));
    if (p.full_flux)
        TRY(tno::launch_rows_out(st, nj, HW, rows, flux, flux_full(q)));
    TRY(tno::launch_trajmax(st, nj, p.ntiles, p.W, (int)HW, rows, at<uint64_t>(A, p.o_tkeys), snr, flux,
                            at<void>(A, p.o_tmax)));
    TRY(tno::launch_best(st, nj, HW, rows, s == 0, snr, flux, at<float>(A, p.o_best),
                         at<int32_t>(A, p.o_bestj), at<float>(A, p.o_bestf)));
    if (p.k > 0) {
        const int k_run = (int)std::min<int64_t>(p.k, (int64_t)sl.a0 * HW);   // kept from earlier slabs
        TRY(tno::launch_topk(st, snr, flux, (int64_t)nj * HW, HW, p.H, p.W, rows, p.k, k_run,
                             at<uint64_t>(A, p.o_tkeys), p.ntiles, p.ntx, tno::search_tx(p.variant),
                             tno::search_ty(p.variant), at<uint64_t>(A, p.o_gbuf),
                             at<tno::TopkState>(A, p.o_tstate), at<uint32_t>(A, p.o_chunks), p.n_chunks,
                             at<uint64_t>(A, p.o_cand), at<void>(A, p.o_topk)));
    }
    return hipSuccess;
}

// The significance pass and the output copies after the last slab;
// `events`: record the end event.
hipError_t enqueue_final(Request *q, bool events)
{
    const Plan &p = q->plan;
    hipStream_t st = q->stream;
    void *A = q->arena;
    const int HW = p.H * p.W;
    hipError_t e;
    TRY(tno::launch_zero(st, at<int32_t>(A, p.o_counts), 4));
    if (p.box > 0)
        TRY(tno::launch_significance(st, p.H, p.W, p.box, p.thr, p.kdet, at<float>(A, p.o_best),
                                     at<int32_t>(A, p.o_bestj), at<float>(A, p.o_bestf), at<double>(A, p.o_r1),
                                     at<double>(A, p.o_r2), at<double>(A, p.o_b1),
                                     at<double>(A, p.o_b2), at<float>(A, p.o_sig),
                                     at<tno::TopkState>(A, p.o_tstate), at<uint32_t>(A, p.o_chunks),
                                     p.n_chunks, at<uint64_t>(A, p.o_cand),
                                     at<tno_detection>(A, p.o_det), at<int32_t>(A, p.o_counts)));
    if (p.dev) {
        const tno_outputs &o = q->out;
        if (o.significance && p.box > 0)
            TRY(hipMemcpyAsync(o.significance, at<void>(A, p.o_sig), (size_t)HW * 4, hipMemcpyDeviceToDevice, st));
        if (o.detections && p.kdet > 0)
            TRY(hipMemcpyAsync(o.detections, at<void>(A, p.o_det), (size_t)p.kdet * sizeof(tno_detection),
                               hipMemcpyDeviceToDevice, st));
        if (o.traj_max)
            TRY(hipMemcpyAsync(o.traj_max, at<void>(A, p.o_tmax), (size_t)p.J * sizeof(tno_peak),
                               hipMemcpyDeviceToDevice, st));
        if (o.topk && p.k > 0)
            TRY(hipMemcpyAsync(o.topk, at<void>(A, p.o_topk), (size_t)p.k * sizeof(tno_candidate),
                               hipMemcpyDeviceToDevice, st));
        if (o.best_snr)
            TRY(hipMemcpyAsync(o.best_snr, at<void>(A, p.o_best), (size_t)HW * 4, hipMemcpyDeviceToDevice, st));
        if (o.best_traj)
            TRY(hipMemcpyAsync(o.best_traj, at<void>(A, p.o_bestj), (size_t)HW * 4, hipMemcpyDeviceToDevice, st));
    }
    if (events)
        TRY(hipEventRecord(q->ev[5], st));
    q->end_recorded = q->end_recorded || events;
    return hipSuccess;
}

// Shape class of a request for the tuning table: stamp and the binary
// orders of magnitude of H, W, J and T.
std::string shape_class(const Plan &p)
{
    auto lg = [](int v) { int b = 0; while ((1 << b) < v) ++b; return b; };
    char buf[64];
    snprintf(buf, sizeof buf, "%s%s%d_H%d_W%d_J%d_T%d", p.direct ? "D" : "", p.sep ? "S" : "P", p.S, lg(p.H),
             lg(p.W), lg(p.J), lg(p.T));
    return buf;
}

// Time every (tile shape, trajectory block) candidate on the first frames of
// this request (its weighting, table and normaliser are already enqueued) and
// keep the fastest for the request's shape class.  Synchronises the stream.
hipError_t autotune(tno_search *h, Request *q)
{
    Plan &p = q->plan;
    struct Cand {
        int v, tb;
        float ms;
    };
    std::vector<Cand> cands;
    const int js = p.slabs[0].a1 - p.slabs[0].a0;
    std::vector<int> tbs = {js};
    for (int tb : {64, 16})
        if (tb < js)
            tbs.push_back(tb);
    for (int v = 0; v < tno::N_SEARCH_VARIANTS; ++v)
        if (variant_serves(p, v))
            for (int tb : tbs)
                cands.push_back({v, tb, 0.0f});
    // the probe's frames are spread over the sequence (every kstride-th), so
    // that the trajectories' shifts spread as they do over the whole search
    const int probe = std::min(p.T, 48);
    const int kstride = std::max(1, p.T / probe);
    std::vector<hipEvent_t> ev(2 * cands.size(), nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess)
            e = hipEventCreate(&x);
    for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) {
        set_search_shape(p, cands[i].v, cands[i].tb);
        const tno::SearchArgs sa = search_args(q, 0, probe, kstride);   // the first slab
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // second run is timed
            if (rep == 1)
                e = hipEventRecord(ev[2 * i], q->stream);
            if (e == hipSuccess)
                e = tno::launch_search(q->stream, p.S, p.sep, p.variant, sa);
        }
        if (e == hipSuccess)
            e = hipEventRecord(ev[2 * i + 1], q->stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(q->stream);
    int best = 0;
    for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) {
        e = hipEventElapsedTime(&cands[i].ms, ev[2 * i], ev[2 * i + 1]);
        if (cands[i].ms < cands[best].ms)
            best = (int)i;
    }
    for (auto &x : ev)
        if (x)
            (void)hipEventDestroy(x);
    if (e != hipSuccess)
        return e;
    // the untuned default (its tile shape, blocks of 16) stays unless a
    // candidate's probe beats it by more than 2 %: a short probe does not
    // rank candidates that close reliably over the whole sequence
    int def = 0;
    const int def_v = default_variant(p);
    for (size_t i = 0; i < cands.size(); ++i)
        if (cands[i].v == def_v && cands[i].tb == std::min(DEFAULT_TBLOCK, p.J))
            def = (int)i;
    if (cands[best].ms > 0.98f * cands[def].ms)
        best = def;
    set_search_shape(p, cands[best].v, cands[best].tb);
    const double rate = (double)js * p.H * p.W * probe / (cands[best].ms * 1e-3);
    h->tuned[shape_class(p)] = {cands[best].v, cands[best].tb, rate};
    h->save_tuning();
    return hipSuccess;
}

// Everything that fixes the node structure of a request's graph: sizes,
// kernel shapes and which optional kernels and copies run.  Pointers and
// scalar arguments are free (an executable graph is updated to them).
std::string graph_key(const Request *q)
{
    const Plan &p = q->plan;
    const tno_outputs &o = q->out;
    const unsigned copies = p.dev ? ((o.significance && p.box > 0) << 0 | (o.detections && p.kdet > 0) << 1 |
                                     (o.traj_max != nullptr) << 2 | (o.topk && p.k > 0) << 3 |
                                     (o.best_snr != nullptr) << 4 | (o.best_traj != nullptr) << 5)
                                  : 0u;
    char buf[256];
    snprintf(buf, sizeof buf, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %u", p.H, p.W,
             p.T, p.J, p.S, (int)p.sep, p.kind, p.variant, p.tblock, p.dtype, p.k, p.box, p.kdet,
             (int)p.full_snr, (int)p.full_flux, (int)p.dev, (int)p.jitter, (int)p.direct, p.Hp, p.Wp4,
             p.lam[0].nj > 0, p.lam[1].nj > 0, copies);
    std::string key = buf;
    for (const auto &sl : p.slabs) {       // the slabs' launches
        snprintf(buf, sizeof buf, " %d:%d:%d", sl.a1 - sl.a0, sl.nj[0], sl.nj[1]);
        key += buf;
    }
    return key;
}

// Graph mode: the request's kernels and device copies are captured into a
// graph, which updates an executable graph of the same structure left by an
// earlier request (or is instantiated), and launched.  Uploads, the wait on a
// resident stack and the start/end events stay outside the graph; phase
// times are not recorded.
hipError_t run_graphed(tno_search *h, Request *q, const tno_request *req)
{
    hipError_t e = enqueue_pre(q);
    if (e != hipSuccess)
        return e;
    if ((e = hipStreamBeginCapture(q->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return e;
    hipError_t ek = enqueue_front(q, req, false);
    if (ek == hipSuccess)
        ek = enqueue_back(q, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(q->stream, &g);
    if (ek != hipSuccess || e != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return ek != hipSuccess ? ek : e;
    }
    const std::string key = graph_key(q);
    hipGraphExec_t x = nullptr;
    auto it = h->free_execs.find(key);
    if (it != h->free_execs.end()) {
        x = it->second;
        h->free_execs.erase(it);
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult ur = hipGraphExecUpdateSuccess;
        if (hipGraphExecUpdate(x, g, &bad, &ur) != hipSuccess || ur != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(x);
            x = nullptr;
        }
    }
    if (!x)
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return e;
    q->exec = x;
    q->exec_key = key;
    if ((e = hipGraphLaunch(x, q->stream)) != hipSuccess)
        return e;
    q->end_recorded = true;
    return hipEventRecord(q->ev[5], q->stream);
}
#undef TRY

// TNO_CFG_BATCH: form and launch search steps while fewer than two are
// queued.  A step takes the oldest ready request (preparation finished)
// with search items left and every other ready request of the same kernel
// (stamp, separability, tile shape, source kind), gives each a chunk of its
// items in request order (an equal share of STEP_BLOCKS, at least
// STEP_CHUNK_MIN), copies the requests' arguments and chunk table into a free
// descriptor slot and launches once on the next search stream.  The stream
// of every request in the step waits for the step; a request whose slab's
// last items were launched gets the slab's reductions queued there, then the
// next slab's normaliser (the request is ready again when it is done) or the
// final pass.  Cancelled requests
// leave the queue with their end event recorded after their launched steps.
// Called with the handle's lock held.
hipError_t pump(tno_search *h)
{
    hipError_t e = hipSuccess;
    for (;;) {
        int nbusy = 0, slot = -1;
        for (int i = 0; i < STEP_SLOTS; ++i) {
            auto &sl = h->slots[i];
            if (sl.busy && hipEventQuery(sl.done) == hipSuccess)
                sl.busy = false;
            if (sl.busy)
                ++nbusy;
            else if (slot < 0)
                slot = i;
        }
        // drop cancelled requests from the queue
        for (auto it = h->ready.begin(); it != h->ready.end();) {
            Request *q = *it;
            if (!q->cancelled) {
                ++it;
                continue;
            }
            if ((e = hipEventRecord(q->ev[5], q->stream)) != hipSuccess)
                return e;
            q->end_recorded = true;
            it = h->ready.erase(it);
        }
        if (nbusy >= 2 || slot < 0 || h->ready.empty())
            return hipSuccess;
        // the requests this step serves
        std::vector<Request *> take;
        const Plan *cls = nullptr;
        for (Request *q : h->ready) {
            if (hipEventQuery(q->prep_done) != hipSuccess)
                continue;
            const Plan &p = q->plan;
            if (cls && (p.S != cls->S || p.sep != cls->sep || p.variant != cls->variant ||
                        p.direct != cls->direct || (p.direct && p.dtype != cls->dtype)))
                continue;
            if (!cls)
                cls = &p;
            take.push_back(q);
            if ((int)take.size() == STEP_ENTRIES)
                break;
        }
        if (take.empty())
            return hipSuccess;
        // the oldest request takes half of the step and the rest share the
        // other half (equal shares throughout slowed the largest requests:
        // p99 ≈ 325 against ≈ 280 ms on the serving mix of the bench)
        constexpr int OQ = STEP_OLDEST_QUARTERS;
        const int nt = (int)take.size();
        const int share = OQ && nt > 1 ? std::max(STEP_CHUNK_MIN, (STEP_BLOCKS * (4 - OQ) / 4 / (nt - 1) + 7) / 8 * 8)
                                       : std::max(STEP_CHUNK_MIN, (STEP_BLOCKS / nt + 7) / 8 * 8);
        const int share0 = OQ && nt > 1 ? STEP_BLOCKS * OQ / 4 : share;
        auto &sl = h->slots[slot];
        tno::SearchArgs *args = (tno::SearchArgs *)sl.host;
        tno::StepEntry *ent = (tno::StepEntry *)((char *)sl.host + STEP_ENTRIES * sizeof(tno::SearchArgs));
        int n = 0, nblocks = 0;
        for (Request *q : take) {
            const Plan &p = q->plan;
            const int n_items = p.ntiles * (p.slabs[q->slab].a1 - p.slabs[q->slab].a0);
            const int cnt = std::min(n == 0 ? share0 : share, n_items - q->next_item);
            args[n] = search_args(q, q->slab, p.T);
            ent[n] = {nblocks, (cnt + 7) / 8 * 8, q->next_item, cnt};
            nblocks += ent[n].nblk;
            ++n;
        }
        hipStream_t ss = h->sstream[h->next_sstream++ & 1];
        tno::StepArgs sa;
        sa.reqs = (const tno::SearchArgs *)sl.dev;
        sa.ent = (const tno::StepEntry *)((char *)sl.dev + STEP_ENTRIES * sizeof(tno::SearchArgs));
        sa.n = n;
        const size_t bytes = STEP_ENTRIES * (sizeof(tno::SearchArgs) + sizeof(tno::StepEntry));
        const Plan &p0 = take[0]->plan;
        if ((e = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, ss)) != hipSuccess ||
            (e = tno::launch_search_step(ss, p0.S, p0.sep, p0.variant, args[0], sa, nblocks)) != hipSuccess ||
            (e = hipEventRecord(sl.done, ss)) != hipSuccess)
            return e;
        sl.busy = true;
        h->n_steps += 1;
        h->n_shared += n > 1;
        for (int i = 0; i < n; ++i) {
            Request *q = take[i];
            q->next_item += ent[i].count;
            h->n_step_items += ent[i].count;
            if ((e = hipStreamWaitEvent(q->stream, sl.done, 0)) != hipSuccess)
                return e;
            const Plan &p = q->plan;
            const int s = q->slab;
            if (q->next_item < p.ntiles * (p.slabs[s].a1 - p.slabs[s].a0))
                continue;
            // the slab's last items: its reductions, then the next slab's
            // normaliser (its items are ready when that is done) or the end
            if ((e = hipEventRecord(q->sev[3 * s + 2], q->stream)) != hipSuccess ||
                (e = enqueue_slab_reduce(q, s)) != hipSuccess)
                return e;
            if (s + 1 < (int)p.slabs.size()) {
                q->slab = s + 1;
                q->next_item = 0;
                if ((e = enqueue_lambda(q, s + 1, true)) != hipSuccess ||
                    (e = hipEventRecord(q->prep_done, q->stream)) != hipSuccess)
                    return e;
            } else {
                h->ready.erase(std::find(h->ready.begin(), h->ready.end(), q));
                if ((e = enqueue_final(q, true)) != hipSuccess)
                    return e;
            }
        }
    }
}

void release(tno_search *hd, Request *q)
{
    if (q->exec)
        hd->free_execs.emplace(q->exec_key, q->exec);
    if (q->arena) {
        keep_block(hd, q->arena, q->arena_bytes);
        hd->in_use -= q->arena_bytes;
    }
    if (q->stack) {
        q->stack->refs -= 1;
        q->stack->last_use = ++hd->tick;
    }
    for (hipEvent_t &e : q->ev)
        if (e)
            (void)hipEventDestroy(e);
    for (hipEvent_t &e : q->sev)
        if (e)
            (void)hipEventDestroy(e);
    if (q->prep_done)
        (void)hipEventDestroy(q->prep_done);
    delete q;
}

// Copy host-side outputs back after completion (the stream work is done).
hipError_t finish_outputs(Request *q)
{
    const Plan &p = q->plan;
    if (p.dev)
        return hipSuccess;
    const tno_outputs &o = q->out;
    void *A = q->arena;
    const size_t HW = (size_t)p.H * p.W, J = (size_t)p.J;
    hipError_t e = hipSuccess;
    auto cp = [&](void *dst, size_t off, size_t bytes) {
        if (dst && e == hipSuccess)
            e = hipMemcpy(dst, at<void>(A, off), bytes, hipMemcpyDeviceToHost);
    };
    cp(o.snr, p.o_snr_full, J * HW * 4);
    cp(o.flux, p.o_flux_full, J * HW * 4);
    cp(o.best_snr, p.o_best, HW * 4);
    cp(o.best_traj, p.o_bestj, HW * 4);
    cp(o.traj_max, p.o_tmax, J * sizeof(tno_peak));
    if (p.k > 0)
        cp(o.topk, p.o_topk, (size_t)p.k * sizeof(tno_candidate));
    if (p.box > 0) {
        cp(o.significance, p.o_sig, HW * 4);
        if (p.kdet > 0)
            cp(o.detections, p.o_det, (size_t)p.kdet * sizeof(tno_detection));
    }
    return e;
}

}  // namespace

extern "C" {

int tno_search_validate(const tno_request *req, const tno_outputs *out, char *msg, int32_t len)
{
    Fail f = check_shape(req, out);
    if (f.code == TNO_OK && !(req->flags & TNO_REQ_DEVICE_PTRS)) {
        Plan p;
        f = make_plan(req, out, req->times, req->velocities, req->jitter, p);
    }
    if (msg && len > 0)
        snprintf(msg, (size_t)len, "%s", f.msg);
    return f.code;
}

uint64_t tno_search_footprint(const tno_request *req, const tno_outputs *out)
{
    if (!req || !out || (req->flags & TNO_REQ_DEVICE_PTRS))
        return 0;
    Plan p;
    Fail f = make_plan(req, out, req->times, req->velocities, req->jitter, p);
    if (f.code != TNO_OK)
        return 0;
    return (uint64_t)p.bytes + (req->stack_key ? p.stack_bytes : 0);
}

const char *tno_search_last_error(void) { return g_last_error; }

}  // extern "C"

// The message of a refusal by another part of the library (same thread-local slot).
void tno::record_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
}

extern "C" {

int tno_search_create(const tno_config *cfg, tno_search **out_handle)
{
    if (!cfg || !out_handle) {
        set_last(fail(TNO_E_INVAL, "config or out_handle is NULL"));
        return TNO_E_INVAL;
    }
    if (cfg->reserved != 0) {
        set_last(fail(TNO_E_INVAL, "config.reserved must be 0"));
        return TNO_E_INVAL;
    }
    if ((cfg->flags & ~(TNO_CFG_GRAPHS | TNO_CFG_AUTOTUNE | TNO_CFG_BATCH | TNO_CFG_RESERVE)) != 0) {
        set_last(fail(TNO_E_INVAL, "unknown config flags 0x%x", cfg->flags));
        return TNO_E_INVAL;
    }
    if ((cfg->flags & TNO_CFG_BATCH) && (cfg->stream || (cfg->flags & TNO_CFG_GRAPHS))) {
        set_last(fail(TNO_E_INVAL, "TNO_CFG_BATCH needs the own stream pool and excludes TNO_CFG_GRAPHS"));
        return TNO_E_INVAL;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || cfg->device < 0 || cfg->device >= ndev) {
        set_last(fail(TNO_E_DEVICE, "device %d not available (%d devices)", cfg->device, ndev));
        return TNO_E_DEVICE;
    }
    if ((e = hipSetDevice(cfg->device)) != hipSuccess)
        return hip_fail(e, "hipSetDevice", nullptr, 0);
    tno_search *h = new (std::nothrow) tno_search();
    if (!h) {
        set_last(fail(TNO_E_NOMEM, "out of host memory"));
        return TNO_E_NOMEM;
    }
    h->device = cfg->device;
    h->max_inflight = cfg->max_inflight > 0 ? cfg->max_inflight : 64;
    h->slab_bytes = cfg->slab_bytes ? (size_t)cfg->slab_bytes : SLAB_BYTES;
    if (cfg->stream) {
        h->streams.push_back((hipStream_t)cfg->stream);
    } else {
        h->own_streams = true;
        for (int i = 0; i < STREAM_POOL; ++i) {
            hipStream_t s = nullptr;
            if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) {
                for (hipStream_t t : h->streams)
                    (void)hipStreamDestroy(t);
                delete h;
                return hip_fail(e, "hipStreamCreate", nullptr, 0);
            }
            h->streams.push_back(s);
        }
    }
    size_t fr = 0, tot = 0;
    if ((e = hipMemGetInfo(&fr, &tot)) != hipSuccess) {
        if (h->own_streams)
            for (hipStream_t t : h->streams)
                (void)hipStreamDestroy(t);
        delete h;
        return hip_fail(e, "hipMemGetInfo", nullptr, 0);
    }
    h->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (uint64_t)(0.9 * (double)fr);
    if (cfg->flags & TNO_CFG_RESERVE) {
        // the whole budget now, as one block: a large hipMalloc or hipFree can
        // hold the host for hundreds of ms (seconds, measured), which a
        // serving loop cannot afford between its polls
        h->pool.reset(h->budget);
        h->budget = h->pool.total();
        if (h->budget == 0 || (e = hipMalloc(&h->pool_base, h->budget)) != hipSuccess) {
            (void)hipGetLastError();
            h->pool_base = nullptr;
            set_last(fail(TNO_E_NOMEM, "reserving the HBM budget of %.3g GB failed", h->budget / 1e9));
            tno_search_destroy(h);
            return TNO_E_NOMEM;
        }
    }
    if (const char *fe = getenv("TNO_FAULT")) {
        // test hook: "alloc:N" makes the N-th fresh device allocation of this
        // handle fail as if the device were out of memory
        unsigned long long n = 0;
        if (sscanf(fe, "alloc:%llu", &n) == 1)
            h->fault_alloc = n;
    }
    h->autotune = (cfg->flags & TNO_CFG_AUTOTUNE) != 0;
    h->graphs = (cfg->flags & TNO_CFG_GRAPHS) != 0;
    h->batch = (cfg->flags & TNO_CFG_BATCH) != 0;
    if (h->batch) {
        const size_t bytes = STEP_ENTRIES * (sizeof(tno::SearchArgs) + sizeof(tno::StepEntry));
        for (int i = 0; i < 2 && e == hipSuccess; ++i)
            e = hipStreamCreateWithFlags(&h->sstream[i], hipStreamNonBlocking);
        for (int i = 0; i < STEP_SLOTS && e == hipSuccess; ++i) {
            auto &sl = h->slots[i];
            if ((e = hipMalloc(&sl.dev, bytes)) == hipSuccess && (e = hipHostMalloc(&sl.host, bytes, 0)) == hipSuccess)
                e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            const int rc = hip_fail(e, "creating the batching streams and step slots", nullptr, 0);
            tno_search_destroy(h);
            return rc;
        }
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) == hipSuccess) {
        h->arch = prop.gcnArchName;
        size_t colon = h->arch.find(':');
        if (colon != std::string::npos)
            h->arch.resize(colon);
    }
    if (cfg->tune_cache_path) {
        h->tune_path = cfg->tune_cache_path;
        h->load_tuning();
    }
    *out_handle = h;
    return TNO_OK;
}

int tno_search_submit(tno_search *h, const tno_request *req, const tno_outputs *out,
                      uint64_t *out_ticket)
{
    if (!h || !out_ticket) {
        set_last(fail(TNO_E_INVAL, "handle or out_ticket is NULL"));
        return TNO_E_INVAL;
    }
    Fail f = check_shape(req, out);
    if (f.code) {
        set_last(f);
        return f.code;
    }
    std::lock_guard<std::mutex> lock(h->mu);
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice", nullptr, 0);
    const bool dev = (req->flags & TNO_REQ_DEVICE_PTRS) != 0;

    // resident stack lookup
    Stack *st = nullptr;
    if (req->stack_key) {
        auto it = h->stacks.find(req->stack_key);
        if (it != h->stacks.end()) {
            st = it->second;
            if (st->H != req->height || st->W != req->width || st->T != req->n_frames ||
                st->dtype != req->dtype) {
                set_last(fail(TNO_E_INVAL, "stack_key %llu is resident with another shape or dtype",
                              (unsigned long long)req->stack_key));
                return TNO_E_INVAL;
            }
        }
    }
    if (!st && !req->residuals) {
        set_last(fail(TNO_E_INVAL, "stack_key %llu is not resident", (unsigned long long)req->stack_key));
        return TNO_E_INVAL;
    }

    std::vector<double> times_h, vel_h, jit_h;
    const double *times = req->times, *vel = req->velocities, *jit = req->jitter;
    if (dev) {
        times_h.resize(req->n_frames);
        vel_h.resize((size_t)2 * req->n_traj);
        if ((e = hipMemcpy(times_h.data(), req->times, times_h.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(vel_h.data(), req->velocities, vel_h.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(e, "reading times/velocities", nullptr, 0);
        times = times_h.data();
        vel = vel_h.data();
        if (req->jitter) {
            jit_h.resize((size_t)2 * req->n_frames);
            if ((e = hipMemcpy(jit_h.data(), req->jitter, jit_h.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess)
                return hip_fail(e, "reading jitter", nullptr, 0);
            jit = jit_h.data();
        }
    }
    Request *q = new (std::nothrow) Request();
    if (!q) {
        set_last(fail(TNO_E_NOMEM, "out of host memory"));
        return TNO_E_NOMEM;
    }
    f = make_plan(req, out, times, vel, jit, q->plan, h->slab_bytes);
    if (f.code) {
        delete q;
        set_last(f);
        return f.code;
    }
    const Plan &p = q->plan;
    const bool new_stack = req->stack_key && !st;
    const size_t need = p.bytes + (new_stack ? p.stack_bytes : 0);
    if (need > h->budget) {
        delete q;
        set_last(fail(TNO_E_NOMEM, "request needs %.3g GB, budget is %.3g GB", need / 1e9, h->budget / 1e9));
        return TNO_E_NOMEM;
    }
    if (st)
        st->refs += 1;   // pin before making room so it cannot be evicted
    if ((int)h->live.size() >= h->max_inflight || !make_room(h, need)) {
        if (st)
            st->refs -= 1;
        delete q;
        set_last(fail(TNO_E_BUSY, "in-flight limit or HBM budget reached"));
        return TNO_E_BUSY;
    }
    if ((req->flags & TNO_REQ_VALIDATE) && !dev && req->dtype == TNO_F32 && req->residuals) {
        const float *Rh = (const float *)req->residuals;
        size_t n = (size_t)p.T * p.H * p.W;
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(Rh[i])) {
                if (st)
                    st->refs -= 1;
                delete q;
                set_last(fail(TNO_E_INVAL, "residual %zu is not finite", i));
                return TNO_E_INVAL;
            }
    }
    q->out = *out;
    q->t_submit = std::chrono::steady_clock::now();
    q->updates = (uint64_t)p.J * p.H * p.W * p.T;
    q->stream = h->streams[h->next_stream++ % h->streams.size()];
    q->stack = st;
    q->arena = get_block(h, p.bytes, &q->arena_bytes);
    if (!q->arena) {
        if (st)
            st->refs -= 1;
        delete q;
        // with requests in flight their memory comes back: retry later
        const int code = h->live.empty() ? TNO_E_NOMEM : TNO_E_BUSY;
        set_last(fail(code, "device allocation of %.3g GB failed%s", p.bytes / 1e9,
                      code == TNO_E_BUSY ? " while requests are in flight" : ""));
        return code;
    }
    h->in_use += q->arena_bytes;
    q->sev.assign(3 * p.slabs.size(), nullptr);
    for (hipEvent_t *ev : {q->ev, q->sev.data()})
        for (size_t i = 0, n = ev == q->ev ? 6 : q->sev.size(); i < n; ++i)
            if ((e = hipEventCreate(&ev[i])) != hipSuccess) {
                release(h, q);
                return hip_fail(e, "hipEventCreate", nullptr, 0);
            }
    const size_t HW = (size_t)p.H * p.W;
    const size_t rbytes = (size_t)p.T * HW * elem_bytes(p.dtype);
    const size_t sbytes = p.dtype == TNO_F32 ? 0 : (size_t)p.T * ((p.H + 63) / 64) * ((p.W + 63) / 64) * 4;
    if (new_stack) {
        // keep these residuals on the device under the caller's key
        Stack *ns = new (std::nothrow) Stack();
        size_t got = 0;
        void *blk = ns ? get_block(h, p.stack_bytes, &got) : nullptr;
        if (!blk) {
            delete ns;
            release(h, q);
            const int code = h->live.empty() ? TNO_E_NOMEM : TNO_E_BUSY;
            set_last(fail(code, "device allocation of a %.3g GB stack failed%s", p.stack_bytes / 1e9,
                          code == TNO_E_BUSY ? " while requests are in flight" : ""));
            return code;
        }
        ns->key = req->stack_key;
        ns->H = p.H;
        ns->W = p.W;
        ns->T = p.T;
        ns->dtype = p.dtype;
        ns->block = blk;
        ns->block_bytes = got;
        ns->bytes = got;
        ns->o_R = 0;
        ns->o_scales = align_up(rbytes, ALIGN);
        ns->o_sigma = ns->o_scales + align_up(sbytes, ALIGN);
        const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        if ((e = hipEventCreate(&ns->ready)) == hipSuccess &&
            (e = hipMemcpyAsync(at<void>(blk, ns->o_R), req->residuals, rbytes, kind, q->stream)) == hipSuccess &&
            (!sbytes || (e = hipMemcpyAsync(at<void>(blk, ns->o_scales), req->tile_scales, sbytes, kind,
                                            q->stream)) == hipSuccess) &&
            (e = hipMemcpyAsync(at<void>(blk, ns->o_sigma), req->sigma, HW * 4, kind, q->stream)) == hipSuccess &&
            (e = hipEventRecord(ns->ready, q->stream)) == hipSuccess) {
            if (!dev)
                e = hipStreamSynchronize(q->stream);   // host inputs are read before submit returns
        }
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(q->stream);
            if (ns->ready)
                (void)hipEventDestroy(ns->ready);
            keep_block(h, blk, got);
            delete ns;
            release(h, q);
            return hip_fail(e, "staging a resident stack", nullptr, 0);
        }
        ns->refs = 1;
        ns->last_use = ++h->tick;
        h->stacks[ns->key] = ns;
        h->in_use += ns->bytes;
        q->stack = ns;
    }
    if (!dev) {
        // host inputs are copied before submit returns
        void *A = q->arena;
        struct {
            size_t off;
            const void *src;
            size_t bytes;
        } cps[] = {
            {p.o_R, req->residuals, p.stack_in_arena ? rbytes : 0},
            {p.o_scales, req->tile_scales, p.stack_in_arena ? sbytes : 0},
            {p.o_sigma, req->sigma, p.stack_in_arena ? HW * 4 : 0},
            {p.o_times, req->times, (size_t)p.T * 8},
            {p.o_vel, req->velocities, (size_t)p.J * 16},
            {p.o_jit, req->jitter, p.jitter ? (size_t)p.T * 16 : 0},
            {p.o_prf, req->prf.table, p.sep ? 0 : (size_t)p.table_n * p.table_n * 8},
        };
        for (auto &c : cps)
            if (c.bytes && (e = hipMemcpy(at<void>(A, c.off), c.src, c.bytes, hipMemcpyHostToDevice)) != hipSuccess) {
                release(h, q);
                return hip_fail(e, "copying inputs", nullptr, 0);
            }
    }
    bool tune_now = false;
    {
        auto it = h->tuned.find(shape_class(q->plan));
        if (it != h->tuned.end() && variant_serves(q->plan, it->second.variant))
            set_search_shape(q->plan, it->second.variant, it->second.tblock);
        else
            tune_now = h->autotune;
    }
    if (h->graphs && !tune_now) {
        e = run_graphed(h, q, req);
    } else if (h->batch && !tune_now) {
        // the preparation now; the search joins the next steps (pump)
        if ((e = enqueue_pre(q)) == hipSuccess && (e = enqueue_front(q, req, true)) == hipSuccess &&
            (e = hipEventCreateWithFlags(&q->prep_done, hipEventDisableTiming)) == hipSuccess &&
            (e = hipEventRecord(q->prep_done, q->stream)) == hipSuccess) {
            q->next_item = 0;
            h->ready.push_back(q);
            e = pump(h);
            if (e != hipSuccess)
                h->ready.erase(std::find(h->ready.begin(), h->ready.end(), q));
        }
    } else if ((e = enqueue_pre(q)) == hipSuccess && (e = enqueue_front(q, req, true)) == hipSuccess &&
               (!tune_now || (e = autotune(h, q)) == hipSuccess)) {
        e = enqueue_back(q, true);
    }
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(q->stream);
        release(h, q);
        return hip_fail(e, "enqueue", nullptr, 0);
    }
    q->ticket = h->next_ticket++;
    h->live[q->ticket] = q;
    *out_ticket = q->ticket;
    return TNO_OK;
}

int tno_search_poll(tno_search *h, uint64_t ticket, int32_t timeout_ms, tno_result *out_result)
{
    if (!h || !out_result) {
        set_last(fail(TNO_E_INVAL, "handle or out_result is NULL"));
        return TNO_E_INVAL;
    }
    auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        {
            std::lock_guard<std::mutex> lock(h->mu);
            auto it = h->live.find(ticket);
            if (it == h->live.end()) {
                set_last(fail(TNO_E_TICKET, "unknown or collected ticket %llu", (unsigned long long)ticket));
                return TNO_E_TICKET;
            }
            Request *q = it->second;
            (void)hipSetDevice(h->device);
            if (h->batch) {
                hipError_t ep = pump(h);
                if (ep != hipSuccess) {
                    set_last(fail(TNO_E_DEVICE, "search step: %s", hipGetErrorString(ep)));
                    return TNO_E_DEVICE;
                }
            }
            // (a batched request's end event is recorded once its last
            // search step is launched: pending until then)
            hipError_t e = q->end_recorded ? hipEventQuery(q->ev[5]) : hipErrorNotReady;
            if (e == hipSuccess && q->cancelled) {
                // the enqueued work has drained; nothing is copied back
                tno_result res;
                memset(&res, 0, sizeof res);
                res.status = TNO_E_CANCELLED;
                snprintf(res.message, sizeof res.message, "request cancelled");
                res.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                         q->t_submit).count();
                h->live.erase(it);
                release(h, q);
                *out_result = res;
                return TNO_E_CANCELLED;
            }
            if (e == hipSuccess) {
                tno_result res;
                memset(&res, 0, sizeof res);
                res.status = TNO_OK;
                res.updates = q->updates;
                res.n_topk = q->plan.k;
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, q->ev[0], q->ev[5]) == hipSuccess)
                    res.device_ms = ms;
                if (!q->exec) {      // (graph mode records no phases)
                    auto span = [&](hipEvent_t a, hipEvent_t b) {
                        float t = 0.0f;
                        return hipEventElapsedTime(&t, a, b) == hipSuccess ? (double)t : 0.0;
                    };
                    res.prep_ms = span(q->ev[0], q->ev[1]);
                    res.table_ms = span(q->ev[1], q->ev[2]);
                    for (size_t s = 0; s < q->plan.slabs.size(); ++s) {
                        res.lambda_ms += span(q->sev[3 * s], q->sev[3 * s + 1]);
                        res.search_ms += span(q->sev[3 * s + 1], q->sev[3 * s + 2]);
                    }
                    // the slabs' reductions and the final pass
                    res.reduce_ms = std::max(0.0, res.device_ms - res.prep_ms - res.table_ms -
                                                      res.lambda_ms - res.search_ms);
                }
                int32_t err = 0, counts[4] = {0, 0, 0, 0};
                hipError_t e2 = hipMemcpy(&err, at<void>(q->arena, q->plan.o_err), 4, hipMemcpyDeviceToHost);
                if (e2 == hipSuccess)
                    e2 = hipMemcpy(counts, at<void>(q->arena, q->plan.o_counts), 16, hipMemcpyDeviceToHost);
                res.n_above = counts[0];
                res.n_detections = counts[1];
                if (e2 == hipSuccess && !err)
                    e2 = finish_outputs(q);
                if (e2 != hipSuccess) {
                    res.status = TNO_E_DEVICE;
                    snprintf(res.message, sizeof res.message, "%s", hipGetErrorString(e2));
                } else if (err & 1) {
                    res.status = TNO_E_INTERNAL;
                    snprintf(res.message, sizeof res.message, "trail run exceeded its planned capacity");
                } else if (err & 2) {
                    res.status = TNO_E_INVAL;
                    snprintf(res.message, sizeof res.message,
                             "sigma so small that 1/sigma^2 overflows single precision");
                }
                auto t1 = std::chrono::steady_clock::now();
                res.total_ms = std::chrono::duration<double, std::milli>(t1 - q->t_submit).count();
                res.queue_ms = std::max(0.0, res.total_ms - res.device_ms);
                h->live.erase(it);
                release(h, q);
                *out_result = res;
                return res.status;
            }
            if (e != hipErrorNotReady) {
                tno_result res;
                memset(&res, 0, sizeof res);
                res.status = TNO_E_DEVICE;
                snprintf(res.message, sizeof res.message, "%s", hipGetErrorString(e));
                (void)hipStreamSynchronize(q->stream);
                h->live.erase(it);
                release(h, q);
                *out_result = res;
                return TNO_E_DEVICE;
            }
        }
        if (timeout_ms == 0)
            return TNO_PENDING;
        auto el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (timeout_ms > 0 && el >= timeout_ms)
            return TNO_PENDING;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

int tno_search_cancel(tno_search *h, uint64_t ticket)
{
    if (!h) {
        set_last(fail(TNO_E_INVAL, "handle is NULL"));
        return TNO_E_INVAL;
    }
    std::lock_guard<std::mutex> lock(h->mu);
    auto it = h->live.find(ticket);
    if (it == h->live.end()) {
        set_last(fail(TNO_E_TICKET, "unknown or collected ticket %llu", (unsigned long long)ticket));
        return TNO_E_TICKET;
    }
    it->second->cancelled = true;
    return TNO_OK;
}

int tno_search_stats(tno_search *h, tno_stats *out)
{
    if (!h || !out) {
        set_last(fail(TNO_E_INVAL, "handle or out is NULL"));
        return TNO_E_INVAL;
    }
    std::lock_guard<std::mutex> lock(h->mu);
    memset(out, 0, sizeof *out);
    out->budget_bytes = h->budget;
    out->in_use_bytes = h->in_use;
    out->cached_bytes = h->cache.held;
    uint64_t held = 0;
    for (auto &kv : h->live)
        held += kv.second->arena_bytes;
    for (auto &kv : h->stacks)
        held += kv.second->block_bytes;
    out->held_bytes = held;
    out->inflight = (int32_t)h->live.size();
    out->resident_stacks = (int32_t)h->stacks.size();
    out->device_allocs = h->n_alloc;
    out->batch_steps = h->n_steps;
    out->batch_items = h->n_step_items;
    out->batch_shared = h->n_shared;
    return TNO_OK;
}

int tno_quantize(int32_t n_frames, int32_t height, int32_t width, int32_t dtype,
                 const float *residuals, void *codes, float *tile_scales, void *stream)
{
    if (n_frames <= 0 || height <= 0 || width <= 0 || n_frames > 65535 || height > 32768 ||
        width > 32768 || !residuals || !codes || !tile_scales ||
        (dtype != TNO_BF16 && dtype != TNO_F16 && dtype != TNO_FP8_E4M3)) {
        set_last(fail(TNO_E_INVAL, "tno_quantize: bad arguments"));
        return TNO_E_INVAL;
    }
    hipError_t e = tno::launch_quantize((hipStream_t)stream, dtype, residuals, n_frames, height, width,
                                        codes, tile_scales);
    if (e != hipSuccess)
        return hip_fail(e, "tno_quantize", nullptr, 0);
    return TNO_OK;
}

void tno_search_destroy(tno_search *h)
{
    if (!h)
        return;
    {
        std::lock_guard<std::mutex> lock(h->mu);
        (void)hipSetDevice(h->device);
        for (hipStream_t s : h->sstream)
            if (s)
                (void)hipStreamSynchronize(s);
        for (hipStream_t s : h->streams)
            (void)hipStreamSynchronize(s);
        h->ready.clear();
        for (auto &kv : h->live)
            release(h, kv.second);
        h->live.clear();
        for (auto &kv : h->free_execs)
            (void)hipGraphExecDestroy(kv.second);
        h->free_execs.clear();
        for (auto &kv : h->stacks) {
            keep_block(h, kv.second->block, kv.second->block_bytes);
            if (kv.second->ready)
                (void)hipEventDestroy(kv.second->ready);
            delete kv.second;
        }
        h->stacks.clear();
        h->cache.trim(0);
        if (h->pool_base)
            (void)hipFree(h->pool_base);
        if (h->own_streams)
            for (hipStream_t s : h->streams)
                (void)hipStreamDestroy(s);
        for (hipStream_t s : h->sstream)
            if (s)
                (void)hipStreamDestroy(s);
        for (auto &sl : h->slots) {
            if (sl.dev)
                (void)hipFree(sl.dev);
            if (sl.host)
                (void)hipHostFree(sl.host);
            if (sl.done)
                (void)hipEventDestroy(sl.done);
        }
    }
    delete h;
}

}  // extern "C"

// ---------------------------------------------------------------- search without allocation
//
// tno_search_run_scratch: one synchronous search whose device working memory
// (the plan's arena: staged stack, ivar maps, offset/weight table, trail
// kernels, normaliser, maps the caller did not ask for, tile keys, top-k
// state) is a fixed array in the library's code object instead of memory
// allocated per request.  Requests whose arena exceeds it are refused.

namespace {
constexpr size_t SCRATCH_BYTES = TNO_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;
}  // namespace

// The array in device memory (one per GPU the library runs on).  In host code
// its name is only a stand-in: the kernels get the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

struct ScratchSlot {
    std::mutex mu;           // held for a whole call: calls on one GPU do not overlap
    void *ptr = nullptr;     // the array's device address on this GPU
};
ScratchSlot g_scratch[MAX_DEVICES];

// This device's address of `scratch` (looked up once per device, with the
// device current); call with g_scratch[dev].mu held.
hipError_t scratch_address(int dev, void **out)
{
    ScratchSlot &s = g_scratch[dev];
    if (!s.ptr) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        s.ptr = p;
    }
    *out = s.ptr;
    return hipSuccess;
}

}  // namespace

int tno_search_run_scratch(const tno_request *req, const tno_outputs *out, void *stream, tno_result *out_result)
{
    if (!out_result) {
        set_last(fail(TNO_E_INVAL, "out_result is NULL"));
        return TNO_E_INVAL;
    }
    auto t0 = std::chrono::steady_clock::now();
    tno_result res;
    memset(&res, 0, sizeof res);
    auto refuse = [&](const Fail &f) {
        set_last(f);
        res.status = f.code;
        snprintf(res.message, sizeof res.message, "%s", f.msg);
        *out_result = res;
        return f.code;
    };
    Fail f = check_shape(req, out);
    if (f.code)
        return refuse(f);
    if ((req->flags & TNO_REQ_DEVICE_PTRS) == 0)
        return refuse(fail(TNO_E_INVAL, "tno_search_run_scratch needs TNO_REQ_DEVICE_PTRS"));
    if (!req->residuals || req->stack_key != 0)
        return refuse(fail(TNO_E_INVAL, "tno_search_run_scratch needs residuals and no stack_key"));
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return refuse(fail(TNO_E_DEVICE, "no usable current device (%s)", hipGetErrorString(e)));
    // host copies of the small inputs the plan reads
    std::vector<double> times_h((size_t)req->n_frames), vel_h((size_t)2 * req->n_traj), jit_h;
    if ((e = hipMemcpy(times_h.data(), req->times, times_h.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(vel_h.data(), req->velocities, vel_h.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return refuse(fail(TNO_E_DEVICE, "reading times/velocities: %s", hipGetErrorString(e)));
    if (req->jitter) {
        jit_h.resize((size_t)2 * req->n_frames);
        if ((e = hipMemcpy(jit_h.data(), req->jitter, jit_h.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess)
            return refuse(fail(TNO_E_DEVICE, "reading jitter: %s", hipGetErrorString(e)));
    }
    Request q;
    // slabs of at most a quarter of the array, so that the normaliser and
    // unrequested maps of many trajectories fit by taking them a few at a time
    f = make_plan(req, out, times_h.data(), vel_h.data(), req->jitter ? jit_h.data() : nullptr, q.plan,
                  SCRATCH_BYTES / 4);
    if (f.code)
        return refuse(f);
    const Plan &p = q.plan;
    if (p.bytes > SCRATCH_BYTES)
        return refuse(fail(TNO_E_NOMEM, "the request needs %zu bytes of working memory; "
                                        "tno_search_run_scratch has %zu", p.bytes, SCRATCH_BYTES));
    std::lock_guard<std::mutex> lock(g_scratch[dev].mu);
    void *arena = nullptr;
    if ((e = scratch_address(dev, &arena)) != hipSuccess)
        return refuse(fail(TNO_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e)));
    q.out = *out;
    q.arena = arena;
    q.arena_bytes = p.bytes;
    q.stream = (hipStream_t)stream;
    q.updates = (uint64_t)p.J * p.H * p.W * p.T;
    // the host-side trail layout, search order and normaliser lists (the
    // call waits for the stream before it returns, so the host vectors
    // outlive the copies), then the request's kernels
    hipStream_t st = q.stream;
    if ((e = hipMemcpyAsync(at<void>(arena, p.o_trail), p.trail.data(), p.trail.size() * sizeof(tno::TrailInfo),
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(at<void>(arena, p.o_perm), p.perm.data(), p.perm.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(at<void>(arena, p.o_jl), p.jlist.data(), p.jlist.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(at<void>(arena, p.o_rows), p.rows.data(), p.rows.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(at<void>(arena, p.o_jrow), p.jrow.data(), p.jrow.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = enqueue_front(&q, req, false)) != hipSuccess || (e = enqueue_back(&q, false)) != hipSuccess) {
        (void)hipStreamSynchronize(st);
        return refuse(fail(TNO_E_DEVICE, "enqueue: %s", hipGetErrorString(e)));
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return refuse(fail(TNO_E_DEVICE, "search: %s", hipGetErrorString(e)));
    int32_t err = 0, counts[4] = {0, 0, 0, 0};
    if ((e = hipMemcpy(&err, at<void>(arena, p.o_err), 4, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(counts, at<void>(arena, p.o_counts), 16, hipMemcpyDeviceToHost)) != hipSuccess)
        return refuse(fail(TNO_E_DEVICE, "reading status: %s", hipGetErrorString(e)));
    if (err & 1)
        return refuse(fail(TNO_E_INTERNAL, "trail run exceeded its planned capacity"));
    if (err & 2)
        return refuse(fail(TNO_E_INVAL, "sigma so small that 1/sigma^2 overflows single precision"));
    res.status = TNO_OK;
    res.updates = q.updates;
    res.n_topk = p.k;
    res.n_above = counts[0];
    res.n_detections = counts[1];
    res.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out_result = res;
    return TNO_OK;
}
