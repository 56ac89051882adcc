// Host-only driver for a sanitizer build of the runtime (tno_runtime.cpp):
// exercises request validation, planning and the footprint estimate -- the
// host code every submit runs before any device work -- over hand-made edge
// cases and seeded random requests.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitize.py; never touches a
// GPU.  The device launch wrappers the runtime links against are stubs here.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2209_09848_amd/csrc/tno_internal.h"

namespace tno {
// stubs of the device side (never reached: the driver calls host-only entries)
hipError_t launch_zero(hipStream_t, int32_t *, int) { return hipErrorNotSupported; }
hipError_t launch_ivar(hipStream_t, int, int, const float *, float *, double *, int, int, int, int, int,
                       int32_t *) { return hipErrorNotSupported; }
hipError_t launch_prep_z(hipStream_t, int, const void *, const float *, const float *, float4 *, int, int,
                         int, int, int, int, int) { return hipErrorNotSupported; }
hipError_t launch_table(hipStream_t, int, int, const double *, double, const double *, const double *,
                        const PrfSpec &, int32_t *, double *) { return hipErrorNotSupported; }
hipError_t launch_trail(hipStream_t, int, int, int, bool, const int32_t *, const double *, const TrailInfo *,
                        int2 *, double *, int32_t *) { return hipErrorNotSupported; }
hipError_t launch_lambda(hipStream_t, const LambdaArgs &, const LambdaArgs &) { return hipErrorNotSupported; }
hipError_t launch_search(hipStream_t, int, bool, int, const SearchArgs &) { return hipErrorNotSupported; }
hipError_t launch_search_step(hipStream_t, int, bool, int, const SearchArgs &, const StepArgs &, int)
{
    return hipErrorNotSupported;
}
hipError_t launch_trajmax(hipStream_t, int, int, int, int, const int32_t *, const uint64_t *, const float *,
                          const float *, void *) { return hipErrorNotSupported; }
hipError_t launch_best(hipStream_t, int, int64_t, const int32_t *, bool, const float *, const float *, float *,
                       int32_t *, float *) { return hipErrorNotSupported; }
hipError_t launch_topk(hipStream_t, const float *, const float *, int64_t, int64_t, int, int, const int32_t *, int,
                       int, const uint64_t *, int, int, int, int, uint64_t *, TopkState *, uint32_t *, int64_t,
                       uint64_t *, void *) { return hipErrorNotSupported; }
hipError_t launch_rows_out(hipStream_t, int, int64_t, const int32_t *, const float *, float *)
{
    return hipErrorNotSupported;
}
int64_t significance_block_values(int H, int W) { return (int64_t)H * W; }
hipError_t launch_significance(hipStream_t, int, int, int, float, int, const float *, const int32_t *,
                               const float *, double *, double *, double *, double *, float *, TopkState *,
                               uint32_t *, int64_t, uint64_t *, tno_detection *, int32_t *)
{
    return hipErrorNotSupported;
}
hipError_t launch_quantize(hipStream_t, int, const float *, int, int, int, void *, float *)
{
    return hipErrorNotSupported;
}
}  // namespace tno

struct Case {
    std::vector<float> R, sigma;
    std::vector<double> times, vel, jit, tab;
    tno_request req{};
    tno_outputs out{};
};

static void fill(Case &c, int H, int W, int T, int J, std::mt19937_64 &g)
{
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    c.R.assign((size_t)T * H * W, 0.0f);
    c.sigma.assign((size_t)H * W, 1.0f);
    c.times.resize(T);
    for (int k = 0; k < T; ++k)
        c.times[k] = 2000.0 + k / 48.0 + (k >= T / 2 ? 1.0 : 0.0);
    c.vel.resize(2 * (size_t)J);
    for (auto &v : c.vel)
        v = 20.0 * u(g);
    memset(&c.req, 0, sizeof c.req);
    memset(&c.out, 0, sizeof c.out);
    c.req.height = H;
    c.req.width = W;
    c.req.n_frames = T;
    c.req.dtype = TNO_F32;
    c.req.residuals = c.R.data();
    c.req.sigma = c.sigma.data();
    c.req.times = c.times.data();
    c.req.t_ref = NAN;
    c.req.prf.kind = TNO_PRF_GAUSS_SAMPLED;
    c.req.prf.stamp = 5;
    c.req.prf.sigma_px = 0.7;
    c.req.n_traj = J;
    c.req.velocities = c.vel.data();
}

// The reserved-block allocator: random takes and gives never hand out
// overlapping ranges, keep the byte count, refuse what does not fit, and
// merge every range back into one when all are given back.
static int check_offset_pool(std::mt19937_64 &g)
{
    const size_t G = tno::OffsetPool::GRAIN;
    tno::OffsetPool pool;
    pool.reset(1000 * G + 123);
    if (pool.total() != 1000 * G || pool.free_bytes() != pool.total() || pool.ranges() != 1)
        return 20;
    struct Held { size_t off, size; };
    std::vector<Held> held;
    size_t got = 0;
    if (pool.take(1001 * G, &got) != tno::OffsetPool::NONE || pool.take(0, &got) != tno::OffsetPool::NONE)
        return 21;
    for (int it = 0; it < 20000; ++it) {
        if (held.empty() || g() % 3 != 0) {
            const size_t want = 1 + g() % (40 * G);
            const size_t off = pool.take(want, &got);
            if (off == tno::OffsetPool::NONE)
                continue;
            if (got < want || got % G != 0 || off % G != 0 || off + got > pool.total())
                return 22;
            for (const Held &h : held)
                if (off < h.off + h.size && h.off < off + got)
                    return 23;
            held.push_back({off, got});
        } else {
            const size_t i = g() % held.size();
            pool.give(held[i].off, held[i].size);
            held[i] = held.back();
            held.pop_back();
        }
        size_t in_use = 0;
        for (const Held &h : held)
            in_use += h.size;
        if (in_use + pool.free_bytes() != pool.total())
            return 24;
    }
    for (const Held &h : held)
        pool.give(h.off, h.size);
    if (pool.free_bytes() != pool.total() || pool.ranges() != 1)
        return 25;
    return 0;
}

int main()
{
    std::mt19937_64 g(2209);
    std::uniform_int_distribution<int> side(1, 300), frames(1, 60), traj(1, 40), pick(0, 15);
    int ok = 0, refused = 0;
    char msg[256];
    for (int it = 0; it < 4000; ++it) {
        Case c;
        fill(c, side(g), side(g), frames(g), traj(g), g);
        tno_request &r = c.req;
        switch (pick(g)) {   // one perturbation per case, valid or not
        case 0: r.prf.stamp = 1 + 2 * (int)(g() % 8); break;
        case 1: r.prf.stamp = 2 * (int)(g() % 9); break;                       // even: refused
        case 2: r.prf.kind = TNO_PRF_GAUSS_INTEGRATED; break;
        case 3: {
            r.prf.kind = TNO_PRF_TABLE;
            r.prf.table_q = 1 + (int)(g() % 9);
            const int n = (r.prf.stamp + 1) * r.prf.table_q + 1;
            c.tab.assign((size_t)n * n, 0.01);
            r.prf.table = c.tab.data();
            break;
        }
        case 4: c.jit.assign(2 * (size_t)r.n_frames, 0.1); r.jitter = c.jit.data(); break;
        case 5: c.jit.assign(2 * (size_t)r.n_frames, 300.0); r.jitter = c.jit.data(); break;  // refused
        case 6: c.vel[0] = NAN; break;                                       // refused
        case 7: c.times[r.n_frames - 1] = INFINITY; break;                   // refused
        case 8: r.top_k = 1 + (int)(g() % 50); break;                        // no topk buffer: refused
        case 9: r.sig_box = 2 * (int)(g() % 200) + 1; r.sig_threshold = 5.0f; break;
        case 10: r.t_ref = 1999.0; break;
        case 11: c.vel[1] = 1.0e12; break;                                   // refused
        case 12: r.dtype = TNO_BF16; break;                                  // no scales: refused
        case 13: r.height = -r.height; break;                                // refused
        case 14: r.n_traj = 0; break;                                        // refused
        default: break;
        }
        const int rc = tno_search_validate(&r, &c.out, msg, sizeof msg);
        const uint64_t fp = tno_search_footprint(&r, &c.out);
        if (rc == TNO_OK) {
            ++ok;
            if (fp == 0) {
                fprintf(stderr, "case %d: valid request with zero footprint\n", it);
                return 2;
            }
        } else {
            ++refused;
            if (fp != 0) {
                fprintf(stderr, "case %d: refused request (%s) with a footprint\n", it, msg);
                return 3;
            }
        }
    }
    // a message longer than the caller's buffer is cut, not overrun
    Case c;
    fill(c, 8, 8, 3, 1, g);
    c.req.prf.stamp = 4;
    char tiny[5];
    if (tno_search_validate(&c.req, &c.out, tiny, sizeof tiny) != TNO_E_INVAL || strlen(tiny) != 4)
        return 4;
    if (tno_search_validate(nullptr, &c.out, msg, sizeof msg) != TNO_E_INVAL)
        return 5;
    if (tno_search_footprint(nullptr, nullptr) != 0)
        return 6;
    if (int rc = check_offset_pool(g))
        return rc;
    printf("host sanitizer driver: %d valid, %d refused; offset pool checked\n", ok, refused);
    return 0;
}
