// tno_internal.h -- shared declarations of the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tno_search.h"

#include <cstddef>
#include <iterator>
#include <map>

namespace tno {

// Search tile shapes.  A lane owns CPL adjacent columns x RPL rows; a block
// stacks NWAVE waves vertically; the tile is TX start columns wide.
// Variants 0-7 (k_search) read every window column a lane needs from LDS; a
// wave spans 64*CPL columns.  Variant 8 (k_search_ws, stamps 1, 3 and 5)
// reads only the lane's own two columns and takes its neighbours' columns
// from the adjacent lanes by wave shifts, so the first and last lane of a
// wave produce no output: 124 start columns per 128-column window.
struct SearchVariant {
    int nwave, cpl, rpl, tx;
    const char *name;
};
inline constexpr SearchVariant SEARCH_VARIANTS[] = {
    {4, 2, 8, 128, "w4c2"}, {8, 2, 8, 128, "w8c2"}, {2, 2, 8, 128, "w2c2"}, {4, 1, 8, 64, "w4c1"},
    {8, 1, 8, 64, "w8c1"}, {4, 4, 8, 256, "w4c4"}, {2, 2, 16, 128, "w2c2r16"}, {4, 2, 16, 128, "w4c2r16"},
    {4, 2, 8, 124, "ws"}, {4, 2, 4, 124, "ws4"},
};
constexpr int N_SEARCH_VARIANTS = 10;
constexpr int SEARCH_WS = 8;             // the wave-shift variants: 8 and 4 rows per lane
constexpr int SEARCH_WS4 = 9;
constexpr int SEARCH_MAX_TX = 256;
constexpr int SEARCH_MAX_TY = 64;
__host__ __device__ constexpr int search_tx(int v) { return SEARCH_VARIANTS[v].tx; }
__host__ __device__ constexpr int search_ty(int v) { return SEARCH_VARIANTS[v].rpl * SEARCH_VARIANTS[v].nwave; }
// Stamps the wave-shift variant serves (a lane's neighbours reach 2 columns).
__host__ __device__ constexpr bool ws_stamp(int S) { return S == 1 || S == 3 || S == 5; }
// Normaliser tile: 64 columns (1 per lane) x 128 rows (32 per lane, 4 waves).
constexpr int LAMBDA_TX = 64;
constexpr int LAMBDA_TY = 128;
// K values per normaliser chunk: every trail column run is zero-padded to a
// whole number of chunks.
constexpr int LAMBDA_CHUNK = 2;
// Frames summed in FP32 before each FP64 accumulation of the numerator.
constexpr int FRAME_CHUNK = 8;
constexpr int LDS_PER_CU = 160 * 1024;   // gfx950 LDS bytes per compute unit

// Dwords per offset/weight table entry, padded to 16 bytes: iy, ix and the
// FP32 weights, gy[S] gx[h] and gx[S] / gx[h] (the centre column tap folded
// into the row taps) for a separable (Gaussian) PRF or W[S][S] (row-major)
// for a tabulated one.  The FP64 weights of the trail kernel are gy[S],
// gx[S] or W[S][S] without the shifts: 2S or S*S doubles per entry.
__host__ __device__ constexpr int table_stride(int S, bool sep) { return (2 + (sep ? 2 * S : S * S) + 3) & ~3; }
__host__ __device__ constexpr int table64_stride(int S, bool sep) { return sep ? 2 * S : S * S; }

// Per-trajectory layout of the collapsed trail kernel K_j (column runs).
struct TrailInfo {
    // tr = 0: the box's columns are the major axis and each column's run goes
    // down the rows.  tr = 1 (boxes wider than tall): stored transposed, the
    // box's rows are the major axis (qx0, ncols = first row offset, rows) and
    // each row's run goes along the columns (qy_lo, qy_hi = column offsets).
    int32_t qx0;       // first major offset of the trail box
    int32_t ncols;     // major lines in the box (clipped to |q| below the image side)
    int32_t qy_lo;     // smallest minor offset kept (clipped likewise)
    int32_t qy_hi;     // largest minor offset kept
    int32_t cap;       // stride of one run: a multiple of LAMBDA_CHUNK, zero-padded
    int32_t tr;        // 1: stored transposed
    int64_t col_off;   // index of this trajectory's first run record
    int64_t val_off;   // index of this trajectory's first K value
};

// Radix-select state of the exact top-k.
struct TopkState {
    uint32_t prefix;   // key bits fixed so far
    uint32_t mask;     // which bits are fixed
    int32_t k_rem;     // rank still to find among keys matching prefix
    uint32_t n_gt;     // candidates strictly above the threshold written
    uint32_t hist[256];
    // the pruned selection of a slab: the k-th largest tile maximum, the
    // entries gathered from the tiles that reach it, and whether it produced
    // the slab's top k (the full selection's passes then return at once)
    uint32_t tstar, n_cand, skip, pad;
};
// Entries the pruned selection sorts in one block.
constexpr int TOPK_GATHER_CAP = 4096;

struct SearchArgs {
    const float4 *Z4;        // padded inverse-variance-weighted stack [T][Hp][Wp4] float4
                             // (each group's columns in the order 4g, 4g+2, 4g+1, 4g+3);
                             // NULL: read the caller's stack directly (R, scales,
                             // ivar32 below; k_search_ws only)
    const void *R;           // direct source: residuals [T][H][W] of `dtype`, W % 4 == 0
    const float *scales;     // direct source: tile scales [T][nqy][nqx] (not F32)
    const float *ivar32;     // direct source: ivar [H][W]
    int dtype, nqy, nqx;
    const int32_t *tab32;    // [J][T][table_stride(S, sep)]
    // One launch searches a slab of J trajectories; its maps hold one row of
    // H*W values per trajectory of the slab, trajectory j in row jrow[j].
    const double *lam;       // [J][H][W]
    float *snr;              // [J][H][W]
    float *flux;             // [J][H][W]
    uint64_t *tile_keys;     // [all trajectories][ntiles], by trajectory number
    const int32_t *perm;     // [J] the slab's trajectories in search order (velocity-sorted)
    const int32_t *jrow;     // [all trajectories] row of each in its slab's maps
    int H, W, T, J;
    int Hp, Wp4, Pt, Pl;
    int ntx, nty, n_items;
    int tblock;              // trajectories per block of the work order
    int nframes;             // frames to accumulate (T, or fewer for a tuning probe)
    int kstride;             // frame k of the launch is frame k * kstride of the stack (1; a
                             // tuning probe spreads its frames over the whole sequence)
};

// A step of the serving loop's search: one launch whose consecutive block
// ranges work for different requests.  Entry r takes work items item0 ..
// item0+count-1 of request r with blocks begin .. begin+nblk-1 (nblk a
// multiple of 8, so that each entry's items are dealt to the XCDs in
// contiguous ranges as a single-request launch deals them).
struct StepEntry {
    int32_t begin, nblk, item0, count;
};
struct StepArgs {
    const SearchArgs *reqs;  // [n] the requests' search arguments (device memory)
    const StepEntry *ent;    // [n] (device memory), by increasing begin
    int n;
};

// One launch of the normaliser covers the trajectories of one storage
// orientation; a transposed launch works in the transposed image (rows <->
// columns) and writes Lam back in the image's own layout.
struct LambdaArgs {
    const TrailInfo *info;
    const int2 *colmeta;     // per major line: (minor offset of run start, run length)
    const double *kvals;
    const double *ivar64;    // [Hq][Wq] in the launch's frame: ivar at (Pyt + y, Pxl + x), zero around it
    double *lam;             // [slab][H0][W0]: trajectory j in row jrow[j]
    const int32_t *jrow;
    const int32_t *jlist;    // [nj] trajectories of this launch
    int H, W;                // image in the launch's frame (W0, H0 when transposed)
    int H0, W0;              // image
    int nj, ntx, nty, n_items;
    int Pyt, Pxl, Wq;
    int tr;                  // 1: transposed launch
};

// ---- launch wrappers (all on `st`; return hipError_t of the launch)
hipError_t launch_zero(hipStream_t st, int32_t *p, int n);
// ivar32 [H][W] (when not NULL) and the zero-bordered FP64 map [Hq][Wq] of
// the image (tr = 0) or of its transpose (tr = 1).
hipError_t launch_ivar(hipStream_t st, int H, int W, const float *sigma, float *ivar32, double *ivar64,
                       int Hq, int Wq, int Pyt, int Pxl, int tr, int32_t *err);
hipError_t launch_prep_z(hipStream_t st, int dtype, const void *R, const float *scales,
                         const float *ivar32, float4 *Z4, int T, int H, int W, int Hp, int Wp4,
                         int Pt, int Pl);
// The PRF of one request: kind, stamp, Gaussian sigma or the tabulated grid.
struct PrfSpec {
    int kind;
    int S;
    double sigma_px;
    const double *table;     // device [(S+1)q+1]^2 for TNO_PRF_TABLE, else unused
    int q;
};
__host__ __device__ constexpr bool prf_separable(int kind) { return kind != TNO_PRF_TABLE; }

hipError_t launch_table(hipStream_t st, int J, int T, const double *times, double t_ref,
                        const double *vel, const double *jitter, const PrfSpec &prf,
                        int32_t *tab32, double *tab64);
hipError_t launch_trail(hipStream_t st, int J, int T, int S, bool sep, const int32_t *tab32,
                        const double *tab64, const TrailInfo *info, int2 *colmeta,
                        double *kvals, int32_t *err);
// Both orientations' normaliser work in one launch (either may have no items).
hipError_t launch_lambda(hipStream_t st, const LambdaArgs &a0, const LambdaArgs &a1);
// Variants 0..N_SEARCH_VARIANTS-1 for stamps of side 5 (separable or not);
// variant 0 and the wave-shift variants (sides 1 and 3) for the others.
hipError_t launch_search(hipStream_t st, int S, bool sep, int variant, const SearchArgs &a);
// One step of the serving loop over `nblocks` blocks; every request of the
// step has the stamp, separability, variant and source kind (staged stack, or
// the dtype read in place) of `proto`.
hipError_t launch_search_step(hipStream_t st, int S, bool sep, int variant, const SearchArgs &proto,
                              const StepArgs &step, int nblocks);
// The wave-shift search (variants SEARCH_WS/SEARCH_WS4) for stamps 1, 3 and 5,
// separable or general, from Z or (Z4 NULL) directly from the caller's stack;
// with `step`, the serving loop's multi-request launch.
hipError_t launch_search_ws(hipStream_t st, int S, bool sep, int variant, const SearchArgs &a,
                            const StepArgs *step = nullptr, int nblocks = 0);
// Slab reductions: a slab's maps have J rows, row r holding trajectory
// rows[r] (increasing with r).
// Peaks of the slab's trajectories: traj_max_out[rows[r]] from row r.
hipError_t launch_trajmax(hipStream_t st, int J, int ntiles, int W, int HW, const int32_t *rows,
                          const uint64_t *tile_keys, const float *snr, const float *flux,
                          void *traj_max_out);
// The bank maximum merged with one slab; first: the slab starts it.
hipError_t launch_best(hipStream_t st, int J, int64_t HW, const int32_t *rows, bool first, const float *snr,
                       const float *flux, float *best_snr, int32_t *best_traj, float *best_flux);
// The exact top k of one slab's N = J*HW scores merged into the k_run
// candidates kept in topk_out from earlier slabs (0: none).
// (Pruned by the slab's tile maxima: tiles of tx x ty start pixels, ntx per
// row, their keys in tile_keys [trajectory][ntiles]; gbuf holds
// TOPK_GATHER_CAP (key, index) pairs.)
hipError_t launch_topk(hipStream_t st, const float *snr, const float *flux, int64_t N, int64_t HW,
                       int H, int W, const int32_t *rows, int k, int k_run, const uint64_t *tile_keys,
                       int ntiles, int ntx, int tx, int ty, uint64_t *gbuf, TopkState *state,
                       uint32_t *chunk_cnt, int64_t n_chunks, uint64_t *cand, void *topk_out);
// Row r of a slab's map (J rows of HW values) into row rows[r] of a map with
// a row per trajectory.
hipError_t launch_rows_out(hipStream_t st, int J, int64_t HW, const int32_t *rows, const float *slab_map,
                           float *full_map);
// Doubles in each of the two block-sum buffers of the significance pass.
int64_t significance_block_values(int H, int W);
hipError_t launch_significance(hipStream_t st, int H, int W, int box, float thr, int k,
                               const float *best_snr, const int32_t *best_traj, const float *best_flux,
                               double *r1, double *r2, double *b1, double *b2, float *sig,
                               TopkState *state, uint32_t *chunk_cnt, int64_t n_chunks,
                               uint64_t *cand, tno_detection *det, int32_t *counts);
hipError_t launch_quantize(hipStream_t st, int dtype, const float *R, int T, int H, int W,
                           void *codes, float *scales);

constexpr int TOPK_CHUNK = 8192;

// Set the thread's last-error message (read by tno_search_last_error).
void record_error(const char *fmt, ...);

// Byte ranges of one device block reserved at handle creation
// (TNO_CFG_RESERVE): best fit over the free ranges, which are kept by offset
// and merged with their neighbours when a range comes back, so that every
// request's arena and every resident stack is carved from the block without a
// device allocation.  Sizes are rounded up to GRAIN (a multiple of the
// arenas' 256-byte alignment).  Host logic only.
class OffsetPool {
  public:
    static constexpr size_t GRAIN = size_t(2) << 20;
    static constexpr size_t NONE = ~size_t(0);

    void reset(size_t bytes)
    {
        free_.clear();
        total_ = bytes / GRAIN * GRAIN;
        if (total_)
            free_[0] = total_;
    }
    size_t total() const { return total_; }
    size_t free_bytes() const
    {
        size_t n = 0;
        for (const auto &kv : free_)
            n += kv.second;
        return n;
    }
    size_t ranges() const { return free_.size(); }
    // Offset of a range of at least `bytes` (its size in *got), or NONE.
    size_t take(size_t bytes, size_t *got)
    {
        const size_t need = (bytes + GRAIN - 1) / GRAIN * GRAIN;
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= need && (best == free_.end() || it->second < best->second))
                best = it;
        if (need == 0 || best == free_.end())
            return NONE;
        const size_t off = best->first, size = best->second;
        free_.erase(best);
        if (size > need)
            free_[off + need] = size - need;
        *got = need;
        return off;
    }
    // Return a range that take() handed out.
    void give(size_t off, size_t bytes)
    {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

  private:
    std::map<size_t, size_t> free_;   // offset -> size of each free range
    size_t total_ = 0;
};

}  // namespace tno
