// hpmc_api.hip -- C-ABI of the implicit-depletant hard-particle Monte Carlo
// library (declared in include/hpmc.h).  Host-side validation, derived
// parameters, workspace layout and the launch sequence of one sweep:
//   grid shift + colour order, cell list (Sec. III.E)
//   8 phase launches, one per colour in random order (Sec. III.E)
//   scatter of the cell-ordered records back to the caller's SoA state
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "hpmc.h"
#include "kernels.hpp"

using namespace hpmc;

// Static scratch of the allocation-free entry point (hpmc_sweep_static): a
// file-scope device array, one copy per device, held until the process ends.
// Host code never passes the array's name to a kernel: it uses the address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct hpmc_sim {
    int64_t N = 0;
    double L = 0, halfL = 0;
    uint64_t seed = 0;
    uint32_t replica = 0;
    int precision = HPMC_FP64;
    hipStream_t stream = nullptr;
    // shape
    int have_shape = 0;
    int kind = 0;
    double par[2] = {0, 0};
    Shape S{};
    double vol_p = 0;
    // depletants and moves
    double z_p = 0, d_dep = 0;
    int n_trial = 0;
    double d_trans = 0.1, a_rot = 0, p_rot = 0;
    int n_select = 1;
    int region = HPMC_V0_BALL;
    // launch shape (results do not depend on it): 0 = default
    int tune_chunk = 0, tune_wpb = 0, tune_waves = 0;
    // derived
    int n = 0;
    double w = 0, inv_w = 0, R0 = 0, lambda = 0, lambda_c = 0, s_ball = 0;
    double r_inner = 0, span = 0;  // shell region: inner radius, R0 - r_inner
    int n_chunks = 1;
    double F[kPoissonC];  // compact inverse-CDF table of the chunk mean (see kernels.hpp)
    int G[kGuide];        // guide: first compact index with F >= i / kGuide
    int pk_min = 0, pk_n = 1;
    int table_set = 0;    // F and G hold the table of the current parameters
    int F_dirty = 1;
    // state and workspace
    double* pos = nullptr;
    double* quat = nullptr;
    uint64_t sweep = 0;
    int have_state = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    Work W{};
    int trace = 0;
    int trace_valid = 0;
    std::vector<hipEvent_t> events;  // timing of phase launches (counters requested)
    int sweep_dev_stale = 0;         // the workspace's sweep counter lags (hpmc_sweep_static ran)
    Desc static_desc{};              // host copy of the descriptor in the static scratch
    hipGraphExec_t graph = nullptr;  // one captured sweep, replayed for untimed multi-sweep calls
    std::vector<unsigned char> graph_key;
    // side streams (default priority) that let the shape groups of a batched
    // sweep run concurrently; created on first use
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
    Desc desc{};                     // host copy of the device descriptor
    Desc* d_desc = nullptr;          // device descriptor (in the workspace)
    // pinned staging buffers of the descriptors of batched sweeps led by this
    // handle, used in turn, each with the event after its last upload (a
    // buffer is rewritten only once its copy is done)
    static constexpr int kStages = 4;
    unsigned char* batch_stage[kStages] = {};
    size_t batch_stage_cap[kStages] = {};  // bytes
    hipEvent_t batch_up[kStages] = {};
    int batch_next = 0;
    unsigned long long* d_gather = nullptr;
    int desc_dirty = 1;
    std::string err;
    ~hpmc_sim()
    {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        if (graph) (void)hipGraphExecDestroy(graph);
        for (int i = 0; i < 3; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
        }
        if (fork) (void)hipEventDestroy(fork);
        for (int i = 0; i < kStages; ++i) {
            if (batch_up[i]) {
                (void)hipEventSynchronize(batch_up[i]);
                (void)hipEventDestroy(batch_up[i]);
            }
            if (batch_stage[i]) (void)hipHostFree(batch_stage[i]);
        }
    }
};

namespace {

int fail(hpmc_sim* s, int code, const std::string& msg)
{
    if (s) s->err = msg;
    return code;
}

int hip_fail(hpmc_sim* s, hipError_t e, const char* where)
{
    return fail(s, HPMC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// derived parameters, in the order of the determinism contract
int derive(hpmc_sim* s)
{
    if (!s->have_shape) return HPMC_OK;
    double rcirc = s->S.rcirc;
    double r_dep = 0.5 * s->d_dep;
    s->R0 = rcirc + r_dep;
    double wmin = 2.0 * rcirc + s->d_dep;
    int n = static_cast<int>(floor(s->L / wmin));
    if (n % 2) n -= 1;
    if (n < 2) return fail(s, HPMC_EBOX, "box smaller than two cells of width 2 R_circ + d_dep");
    // (this also keeps every cell coordinate below 1024: the sphere kernel packs them in 10 bits)
    if (static_cast<int64_t>(n) * n * n > 0x3FFFFFFF) return fail(s, HPMC_EBOX, "too many cells");
    s->n = n;
    s->w = s->L / static_cast<double>(n);
    s->inv_w = 1.0 / s->w;
    s->s_ball = s->R0 * 0x1p-21;
    double vol0 = 4.0 / 3.0 * M_PI * s->R0 * s->R0 * s->R0;
    s->r_inner = 0.0;
    s->span = s->R0;
    if (s->region == HPMC_V0_SHELL) {
        // the core ball stays inside the old pose for translations up to sqrt(3) d_trans
        double ri = (s->S.rin + r_dep) - sqrt(3.0) * s->d_trans;
        if (ri < 0.0) ri = 0.0;
        s->r_inner = ri;
        s->span = s->R0 - ri;
        vol0 = 4.0 / 3.0 * M_PI * (s->R0 * s->R0 * s->R0 - ri * ri * ri);
    }
    s->lambda = s->z_p * vol0;
    int m = static_cast<int>(ceil(s->lambda / 256.0));
    if (m < 1) m = 1;
    s->n_chunks = m;
    s->lambda_c = s->lambda / static_cast<double>(m);
    // the full table F[k] = P(N <= k) by forward recursion, sentinel last
    std::vector<double> full(kPoissonK);
    double P = exp(-s->lambda_c);
    full[0] = P;
    for (int k = 1; k < kPoissonK - 1; ++k) {
        P = P * (s->lambda_c / static_cast<double>(k));
        full[k] = full[k - 1] + P;
    }
    full[kPoissonK - 1] = 2.0;
    // the entries a 52-bit uniform can stop at (kernels.hpp), then the sentinel
    const double umin = ldexp(1.0, -53), umax = 1.0 - ldexp(1.0, -53);
    int kmin = 0;
    while (full[static_cast<size_t>(kmin)] < umin) ++kmin;
    int kend = kmin;
    while (kend < kPoissonK - 2 && full[static_cast<size_t>(kend)] < umax &&
           full[static_cast<size_t>(kend) + 1] != full[static_cast<size_t>(kend)])
        ++kend;
    const int nc = kend - kmin + 1;
    if (nc + 1 > kPoissonC) return fail(s, HPMC_EINVAL, "Poisson table of the chunk mean exceeds its capacity");
    for (int i = 0; i < kPoissonC; ++i) s->F[i] = i < nc ? full[static_cast<size_t>(kmin + i)] : 2.0;
    s->pk_min = kmin;
    s->pk_n = nc;
    s->table_set = 1;
    for (int i = 0, k = 0; i < kGuide; ++i) {
        double lev = static_cast<double>(i) / static_cast<double>(kGuide);
        while (s->F[k] < lev) ++k;
        s->G[i] = k;
    }
    s->F_dirty = 1;
    Shape& S = s->S;
    S.r_dep = r_dep;
    S.R0sq = s->R0 * s->R0;
    S.rdsq = r_dep * r_dep;
    S.rsd_sq = (S.rs + r_dep) * (S.rs + r_dep);
    return HPMC_OK;
}

struct Layout {
    size_t cell_count, cell_start, scan_tmp, pcell, prank, order, rpos, rquat, F, grid, perm, counters, flags, obs,
        desc, sweep, gather, trace, total;
};

constexpr int kObsWords = 8192;

Layout layout(const hpmc_sim* s)
{
    Layout l{};
    size_t ncells = static_cast<size_t>(s->n) * s->n * s->n;
    size_t N = static_cast<size_t>(s->N);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    l.cell_count = take(ncells * 4);
    l.cell_start = take((ncells + 1) * 4);
    l.scan_tmp = take(((ncells + 1023) / 1024 + 1) * 4);
    l.pcell = take(N * 4);
    l.prank = take(N * 4);
    l.order = take(N * 4);
    l.rpos = take(N * 32);
    l.rquat = take(s->S.oriented ? N * 32 : 0);
    l.F = take(kPoissonC * 8 + kGuide * 4);
    l.grid = take(4 * 8);
    l.perm = take(8 * 4);
    l.counters = take(static_cast<size_t>(kCounterCopies) * kCounterStride * 8);
    l.flags = take(4 * 4);
    l.obs = take(static_cast<size_t>(kObsWords) * 8);
    l.desc = take(sizeof(Desc));
    l.sweep = take(4);
    l.gather = take(kCounterStride * 8);
    l.trace = take(s->trace ? N * static_cast<size_t>(s->n_select) * sizeof(hpmc_move_record) : 0);
    l.total = off;
    return l;
}

// the workspace regions of handle s carved out of the buffer at b
Work carve(const hpmc_sim* s, unsigned char* b, Desc** d_desc, unsigned long long** d_gather)
{
    Layout l = layout(s);
    Work W{};
    W.cell_count = reinterpret_cast<int*>(b + l.cell_count);
    W.cell_start = reinterpret_cast<int*>(b + l.cell_start);
    W.scan_tmp = reinterpret_cast<int*>(b + l.scan_tmp);
    W.pcell = reinterpret_cast<int*>(b + l.pcell);
    W.prank = reinterpret_cast<int*>(b + l.prank);
    W.order = reinterpret_cast<int*>(b + l.order);
    W.rpos = reinterpret_cast<double4*>(b + l.rpos);
    W.rquat = s->S.oriented ? reinterpret_cast<double4*>(b + l.rquat) : nullptr;
    W.F = reinterpret_cast<double*>(b + l.F);
    W.grid = reinterpret_cast<double*>(b + l.grid);
    W.perm = reinterpret_cast<int*>(b + l.perm);
    W.counters = reinterpret_cast<unsigned long long*>(b + l.counters);
    W.flags = reinterpret_cast<int*>(b + l.flags);
    W.obs = reinterpret_cast<unsigned long long*>(b + l.obs);
    W.trace = s->trace ? static_cast<void*>(b + l.trace) : nullptr;
    W.sweep_dev = reinterpret_cast<uint32_t*>(b + l.sweep);
    W.pos = s->pos;
    W.quat = s->quat;
    *d_desc = reinterpret_cast<Desc*>(b + l.desc);
    *d_gather = reinterpret_cast<unsigned long long*>(b + l.gather);
    return W;
}

void bind_work(hpmc_sim* s)
{
    s->W = carve(s, static_cast<unsigned char*>(s->ws), &s->d_desc, &s->d_gather);
    s->desc_dirty = 1;
}

int64_t packing_bound(const hpmc_sim* s, double side)
{
    double v = side * side * side / s->vol_p;
    if (v > 1e9) v = 1e9;
    int64_t b = static_cast<int64_t>(floor(v)) + 1;
    return std::min<int64_t>(b, s->N);
}

Params make_params(const hpmc_sim* s)
{
    Params P{};
    P.S = s->S;
    P.N = static_cast<int>(s->N);
    P.n = s->n;
    P.h = s->n / 2;
    P.ncells = s->n * s->n * s->n;
    P.active_cells = P.h * P.h * P.h;
    P.n_select = s->n_select;
    P.n_trial = s->n_trial;
    P.n_chunks = s->n_chunks;
    P.pk_min = s->pk_min;
    P.pk_n = s->pk_n;
    P.has_dep = s->z_p > 0.0 ? 1 : 0;
    P.trace = s->trace;
    P.precision = s->precision;
    P.key0 = static_cast<uint32_t>(s->seed & 0xFFFFFFFFu);
    P.key1 = static_cast<uint32_t>(s->seed >> 32) ^ s->replica;
    P.sweep = 0;  // kernels read the sweep index from the workspace's device counter
    P.L = s->L;
    P.halfL = s->halfL;
    P.w = s->w;
    P.inv_w = s->inv_w;
    P.d_trans = s->d_trans;
    P.a_rot = s->a_rot;
    P.p_rot = s->S.oriented ? s->p_rot : 0.0;
    P.s_ball = s->s_ball;
    P.shell = s->region == HPMC_V0_SHELL;
    P.r_inner = s->r_inner;
    P.span = s->span;
    {
        // sigma = the colloid's circumdiameter
        double eps = 1e-5 * (2.0 * s->S.rcirc);
        // spheres: band of |v|^2 around R0^2; oriented shapes: band of the
        // distance to the core around r_dep (hemisphere) or r_s + r_dep (swept disk)
        double thr = s->S.kind == HPMC_DISCOID ? s->S.rs + 0.5 * s->d_dep : 0.5 * s->d_dep;
        double lo = (s->R0 - eps) * (s->R0 - eps), hi = (s->R0 + eps) * (s->R0 + eps);
        if (s->S.oriented) {
            lo = thr - eps;
            hi = thr + eps;
        }
        P.g_lo = nextafterf(static_cast<float>(lo), 0.0f);
        P.g_hi = nextafterf(static_cast<float>(hi), INFINITY);
    }
    // per-wave LDS of the phase kernel: a rigorous packing bound (hard bodies
    // are disjoint) for the stencil list
    double rc2 = 2.0 * s->S.rcirc;
    int64_t list_cap = (s->n == 2) ? s->N : packing_bound(s, 3.0 * s->w + rc2);
    int gs = s->S.oriented ? 12 : 3;
    // Oriented shapes cache the stencil's positions and rotation matrices in
    // LDS: 64 entries, which keeps two waves per SIMD resident; entries past the
    // cache are read from HBM.  In a box of two cells per axis every colloid is
    // in every stencil and a phase is one cell's serial chain of trials, so
    // the whole box is cached (up to 512 colloids).
    int64_t geo_cap = std::min<int64_t>(list_cap, 512);
    if (s->S.oriented) geo_cap = std::min<int64_t>(list_cap, s->n == 2 ? 512 : 64);
    const size_t lds_max = lds_limit();
    // A depletant point of B(x', R0) or a CB trial point of B(x, R0) can only
    // overlap a colloid whose reference point lies within reach of x'.
    const double reach = s->R0 + s->S.rcirc + 0.5 * s->d_dep + 1.7320508075688772 * s->d_trans * (1.0 + 1e-12) + 1e-9;
    P.reach_sq = reach * reach;
    if (!s->S.oriented) {
        // spheres: two stage buffers, each the stencil list + staged records (x, y) and (z, index)
        size_t o = align256(static_cast<size_t>(list_cap) * 4);
        P.off_rec_a = static_cast<int>(o);
        o = align256(o + 64 * 16);
        P.off_rec_b = static_cast<int>(o);
        o = align256(o + 64 * 16);
        P.off_geo = 0;
        P.off_cnt = static_cast<int>(2 * o);  // after the two stage buffers: the wave's counters
        P.wave_lds = static_cast<int>(2 * o + kNumCounters * 8);
        P.list_cap = static_cast<int>(list_cap);
        P.geo_cap = static_cast<int>(geo_cap);
        int wpb = s->tune_wpb ? s->tune_wpb : kSphereWpb;
        while (wpb > 1 && kTableLds + static_cast<size_t>(wpb) * P.wave_lds > lds_max) wpb >>= 1;
        P.waves_per_block = wpb;
        P.chunk = s->tune_chunk ? s->tune_chunk : kChunk;
        P.blk0 = 0;
        P.nblk = phase_blocks(kSphere, P.active_cells, P.chunk, wpb, 0);
        return P;
    }
    // oriented shapes: the stencil list, the geometry cache and the per-trial
    // close and reach lists (the cell's own records stay in HBM); a cache that
    // would not fit one wave's share of the LDS is halved
    // A colloid whose reference point lies within 2 r_circ of the proposed one
    // has its body inside the cube of side 6 r_circ around it; one in reach,
    // inside the cube of side 2 reach + 2 r_circ.  Hard bodies are disjoint,
    // so both counts obey the packing bound.
    const double rc = s->S.rcirc;
    P.close_cap = static_cast<int>(std::min<int64_t>(list_cap, packing_bound(s, 6.0 * rc)));
    P.reach_cap = static_cast<int>(std::min<int64_t>(list_cap, packing_bound(s, 2.0 * reach + 2.0 * rc)));
    size_t off = 0;
    for (;;) {
        off = align256(static_cast<size_t>(list_cap) * 4);
        P.off_geo = static_cast<int>(off);
        off = align256(off + static_cast<size_t>(geo_cap) * 8 * gs);
        P.off_close = static_cast<int>(off);
        off = align256(off + static_cast<size_t>(P.close_cap) * 4);
        P.off_reach = static_cast<int>(off);
        off = align256(off + static_cast<size_t>(P.reach_cap) * 4);
        if (kTableLds + off <= lds_max || geo_cap <= 64) break;
        geo_cap = std::max<int64_t>(64, geo_cap / 2);
    }
    P.list_cap = static_cast<int>(list_cap);
    P.geo_cap = static_cast<int>(geo_cap);
    P.wave_lds = static_cast<int>(off);
    // a large cache (dense boxes: few active cells, long serial chains) runs
    // one wave per workgroup, so it holds a CU's LDS only as long as that wave
    int wpb = s->tune_wpb ? s->tune_wpb : (geo_cap > 64 ? 1 : 4);
    while (wpb > 1 && kTableLds + static_cast<size_t>(wpb) * off > lds_max) wpb >>= 1;
    P.waves_per_block = wpb;
    P.chunk = kChunk;
    P.blk0 = 0;
    P.nblk = phase_blocks(s->S.kind, P.active_cells, P.chunk, wpb, s->tune_waves ? s->tune_waves : kMaxWaves);
    return P;
}

// launch shape of a group of replicas (descriptors already on the device)
// pars: the members' make_params results, or null to compute them here
Group make_group(const Desc* d, const hpmc_sim* const* sims, int n, const Params* pars = nullptr)
{
    Group g{};
    g.d = d;
    g.nrep = n;
    g.kind = sims[0]->S.kind;
    g.precision = sims[0]->precision;
    g.shell = sims[0]->region == HPMC_V0_SHELL;
    g.wpb = 4;
    g.chunk = sims[0]->tune_chunk ? sims[0]->tune_chunk : kChunk;
    g.max_waves = sims[0]->tune_waves ? sims[0]->tune_waves : kMaxWaves;
    size_t wave_lds = 0;
    for (int i = 0; i < n; ++i) {
        const Params P = pars ? pars[i] : make_params(sims[i]);
        g.maxN = std::max(g.maxN, P.N);
        g.maxCells = std::max(g.maxCells, P.ncells);
        g.maxActive = std::max(g.maxActive, P.active_cells);
        g.wpb = std::min(g.wpb, P.waves_per_block);
        wave_lds = std::max(wave_lds, static_cast<size_t>(P.wave_lds));
    }
    g.lds = kTableLds + static_cast<size_t>(g.wpb) * wave_lds;
    // small sphere boxes sweep in one workgroup per replica, many sweeps per launch
    g.lds_small = kTableLds + static_cast<size_t>(kSmallWaves) * wave_lds;
    g.small = g.kind == kSphere && g.maxActive <= kSmallMaxActive && g.maxN <= kSmallMaxN &&
              g.lds_small + kSmallStaticLds <= lds_limit();
    // a group of one replica owns every block of its phase launches
    g.brep = nullptr;
    g.nblocks = phase_blocks(g.kind, g.maxActive, g.chunk, g.wpb, g.max_waves);
    return g;
}

// Launch group of a replica in a batched sweep: replicas of one shape kind,
// precision and insertion region share the phase launches, except that small
// sphere boxes (one workgroup sweeps each) and oriented boxes with a large
// geometry cache (few active cells, long serial chains; their LDS would lower
// everyone's occupancy) form groups of their own.
int batch_class(const hpmc_sim* s, const Params& P)
{
    const int small = (s->S.kind == HPMC_SPHERE && P.active_cells <= kSmallMaxActive && P.N <= kSmallMaxN &&
                       kTableLds + static_cast<size_t>(kSmallWaves) * P.wave_lds + kSmallStaticLds <= lds_limit())
                          ? 1
                          : 0;
    const int dense = s->S.oriented && P.geo_cap > 64 ? 1 : 0;
    return 16 * s->S.kind + 8 * dense + 4 * small + 2 * s->precision + s->region;
}
constexpr int kBatchClasses = 48;
int class_is_small(int cl) { return (cl >> 2) & 1; }

// launch shapes the autotuners time; the first is the default
std::vector<hpmc_tuning> tuning_candidates(bool oriented)
{
    std::vector<hpmc_tuning> cand;
    if (!oriented) {
        for (int c : {kChunk, 4, 6, 10, 12, 16, 32, 64})
            for (int w : {kSphereWpb, 2, 4}) cand.push_back(hpmc_tuning{c, w, 0, 0, 0.0, 0.0});
    } else {
        for (int m : {kMaxWaves, 1024, 2048, 4096, 16384, 32768})
            for (int w : {4, 2, 1}) cand.push_back(hpmc_tuning{0, w, m, 0, 0.0, 0.0});
    }
    return cand;
}

// descriptor of a handle whose make_params result is P, at a launch shape
Desc make_desc(const hpmc_sim* s, const Params& P, int wpb, int chunk)
{
    Desc d{};
    d.P = P;
    d.P.waves_per_block = wpb;
    d.P.chunk = chunk;
    d.P.blk0 = 0;
    d.P.nblk = phase_blocks(s->S.kind, d.P.active_cells, chunk, wpb, s->tune_waves ? s->tune_waves : kMaxWaves);
    d.W = s->W;
    return d;
}

// refresh the device descriptor of a single handle when its host copy changed
int sync_desc(hpmc_sim* s)
{
    Params P = make_params(s);
    Desc d = make_desc(s, P, P.waves_per_block, P.chunk);
    if (!s->desc_dirty && memcmp(&d, &s->desc, sizeof(Desc)) == 0) return HPMC_OK;
    s->desc = d;
    hipError_t e = hipMemcpyAsync(s->d_desc, &s->desc, sizeof(Desc), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "hipMemcpyAsync(descriptor)");
    s->desc_dirty = 0;
    return HPMC_OK;
}

Group single_group(hpmc_sim* s)
{
    const hpmc_sim* one[1] = {s};
    return make_group(s->d_desc, one, 1);
}

int set_sweep_dev(hpmc_sim* s)
{
    hipError_t e = launch_fill_int(reinterpret_cast<int*>(s->W.sweep_dev), 1,
                                   static_cast<int>(static_cast<uint32_t>(s->sweep)), s->stream);
    return e == hipSuccess ? HPMC_OK : hip_fail(s, e, "sweep counter");
}

// Handles created without a stream share one library stream per device: a
// blocking stream, so it is ordered with work on the null stream, and a real
// stream, so untimed multi-sweep calls can be captured into a graph.
hipStream_t library_stream()
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreate(&streams[dev]) != hipSuccess) streams[dev] = nullptr;
    return streams[dev];
}

// P_out: if not null, receives the handle's make_params result
int check_ready(hpmc_sim* s, bool need_state, Params* P_out = nullptr)
{
    if (!s->stream) s->stream = library_stream();
    if (!s->have_shape) return fail(s, HPMC_ESTATE, "shape not set");
    if (!s->ws) return fail(s, HPMC_ESTATE, "workspace not set");
    if (s->ws_bytes < layout(s).total) return fail(s, HPMC_ENOMEM, "workspace too small for the current settings");
    if (need_state && !s->have_state) return fail(s, HPMC_ESTATE, "state not set");
    Params P = make_params(s);
    if (kTableLds + static_cast<size_t>(P.waves_per_block) * P.wave_lds > lds_limit())
        return fail(s, HPMC_ECAPACITY, "stencil too large for the LDS of one workgroup");
    if (s->sweep_dev_stale && s->have_state) {
        int r = set_sweep_dev(s);
        if (r != HPMC_OK) return r;
        s->sweep_dev_stale = 0;
    }
    if (P_out) *P_out = P;
    return HPMC_OK;
}

int upload_table(hpmc_sim* s)
{
    if (!s->F_dirty) return HPMC_OK;
    hipError_t e = hipMemcpyAsync(s->W.F, s->F, sizeof(s->F), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->W.F + kPoissonC, s->G, sizeof(s->G), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "hipMemcpyAsync(table)");
    s->F_dirty = 0;
    return HPMC_OK;
}

// Capacity flags are sticky: a kernel that had to skip work sets them, and
// they stay set until a synchronising call reports them (ECAPACITY) and
// clears them, so untimed and graph-replayed sweeps cannot lose one.
int report_flags(hpmc_sim* s, int flags)
{
    if (!flags) return HPMC_OK;
    hipError_t e = launch_fill_int(s->W.flags, 4, 0, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "clear flags");
    return fail(s, HPMC_ECAPACITY, "a cell's stencil exceeded its capacity in an earlier sweep; its trials were "
                                   "skipped (flags " + std::to_string(flags) + ")");
}

// Address of the static scratch on each device (set up once per device, with
// that device current).
std::mutex g_scratch_mu;
void* g_scratch[64] = {};

int static_scratch(hpmc_sim* s, unsigned char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(s, e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(s, HPMC_EINVAL, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(s, e, "hipGetSymbolAddress(static scratch)");
        if (!p) return fail(s, HPMC_EHIP, "hipGetSymbolAddress(static scratch) returned a null address");
        g_scratch[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch[dev]);
    return HPMC_OK;
}

// Lay the handle's workspace out in the static scratch of the current device
// and enqueue its descriptor, Poisson table, sweep counter and cleared flags
// there.  Whatever an earlier call left in the scratch is overwritten.
int bind_static(hpmc_sim* s, Group& g, Work& W, unsigned long long** gather)
{
    const size_t need = layout(s).total;
    if (need > kStaticScratchBytes)
        return fail(s, HPMC_ENOMEM, "this handle needs " + std::to_string(need) + " bytes of scratch; the static "
                                    "scratch holds " + std::to_string(kStaticScratchBytes));
    Params P = make_params(s);
    if (kTableLds + static_cast<size_t>(P.waves_per_block) * P.wave_lds > lds_limit())
        return fail(s, HPMC_ECAPACITY, "stencil too large for the LDS of one workgroup");
    unsigned char* base = nullptr;
    int r = static_scratch(s, &base);
    if (r != HPMC_OK) return r;
    Desc* d_desc = nullptr;
    W = carve(s, base, &d_desc, gather);
    s->static_desc = make_desc(s, P, P.waves_per_block, P.chunk);
    s->static_desc.W = W;
    hipError_t e = hipMemcpyAsync(d_desc, &s->static_desc, sizeof(Desc), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(W.F, s->F, sizeof(s->F), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(W.F + kPoissonC, s->G, sizeof(s->G), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = launch_fill_int(reinterpret_cast<int*>(W.sweep_dev), 1, static_cast<int>(static_cast<uint32_t>(s->sweep)),
                            s->stream);
    if (e == hipSuccess) e = launch_fill_int(W.flags, 4, 0, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "static scratch set-up");
    const hpmc_sim* one[1] = {s};
    g = make_group(d_desc, one, 1);
    return HPMC_OK;
}

int check_flags(hpmc_sim* s)
{
    int flags = 0;
    hipError_t e = hipMemcpyAsync(&flags, s->W.flags, sizeof(int), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "read flags");
    return report_flags(s, flags);
}

}  // namespace

extern "C" {

int hpmc_create(hpmc_sim** out, int64_t n, double box_L, uint64_t seed, uint32_t replica_id, int precision,
                void* hip_stream)
{
    if (!out) return HPMC_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 0x3FFFFFFF || !(box_L > 0.0) || !isfinite(box_L)) return HPMC_EINVAL;
    if (precision != HPMC_FP64 && precision != HPMC_FP32_GUARDED) return HPMC_EINVAL;
    hpmc_sim* s = new hpmc_sim();
    s->N = n;
    s->L = box_L;
    s->halfL = 0.5 * box_L;
    s->seed = seed;
    s->replica = replica_id;
    s->precision = precision;
    s->stream = static_cast<hipStream_t>(hip_stream);
    *out = s;
    return HPMC_OK;
}

void hpmc_destroy(hpmc_sim* sim) { delete sim; }

const char* hpmc_last_error(const hpmc_sim* sim) { return sim ? sim->err.c_str() : "null handle"; }

int hpmc_set_shape(hpmc_sim* s, int kind, const double* p, int np)
{
    if (!s) return HPMC_EINVAL;
    if (!p) return fail(s, HPMC_EINVAL, "null shape parameters");
    Shape S{};
    S.kind = kind;
    double vol;
    if (kind == HPMC_SPHERE || kind == HPMC_HEMISPHERE) {
        if (np < 1 || !(p[0] > 0.0) || !isfinite(p[0])) return fail(s, HPMC_EINVAL, "diameter must be positive");
        S.a = 0.5 * p[0];
        S.rcirc = 0.5 * p[0];
        S.rin = (kind == HPMC_SPHERE) ? 0.5 * p[0] : 0.0;  // hemisphere: the face centre is on the boundary
        S.dsq = p[0] * p[0];
        S.oriented = kind == HPMC_HEMISPHERE;
        vol = (kind == HPMC_SPHERE) ? M_PI * p[0] * p[0] * p[0] / 6.0 : M_PI * p[0] * p[0] * p[0] / 12.0;
    } else if (kind == HPMC_DISCOID) {
        if (np < 2 || !(p[0] > 0.0) || !(p[1] > 0.0)) return fail(s, HPMC_EINVAL, "disk and sweep radii must be positive");
        S.a = p[0];
        S.rs = p[1];
        S.rcirc = p[0] + p[1];
        S.rin = p[1];
        S.dsq = 4.0 * S.rcirc * S.rcirc;
        S.oriented = 1;
        vol = 2.0 * M_PI * p[0] * p[0] * p[1] + M_PI * M_PI * p[0] * p[1] * p[1] + 4.0 / 3.0 * M_PI * p[1] * p[1] * p[1];
    } else {
        return fail(s, HPMC_EINVAL, "unknown shape");
    }
    S.asq = S.a * S.a;
    S.lim_sq = (2.0 * S.rcirc) * (2.0 * S.rcirc);
    hpmc_sim saved = *s;
    s->S = S;
    s->kind = kind;
    s->par[0] = p[0];
    s->par[1] = np > 1 ? p[1] : 0.0;
    s->vol_p = vol;
    s->have_shape = 1;
    int r = derive(s);
    if (r != HPMC_OK) {
        std::string e = s->err;
        *s = saved;
        s->err = e;
        return r;
    }
    if (s->ws) bind_work(s);
    return HPMC_OK;
}

int hpmc_set_fugacity(hpmc_sim* s, double z_p, double d_dep, int n_trial)
{
    if (!s) return HPMC_EINVAL;
    if (!(z_p >= 0.0) || !isfinite(z_p) || !(d_dep >= 0.0) || !isfinite(d_dep) || n_trial < 0 || n_trial > 255)
        return fail(s, HPMC_EINVAL, "invalid depletant parameters");
    double oz = s->z_p, od = s->d_dep;
    int ot = s->n_trial;
    s->z_p = z_p;
    s->d_dep = d_dep;
    s->n_trial = n_trial;
    int r = derive(s);
    if (r == HPMC_OK && s->lambda > 60000.0) r = fail(s, HPMC_EINVAL, "mean depletant number per move too large");
    if (r != HPMC_OK) {
        s->z_p = oz;
        s->d_dep = od;
        s->n_trial = ot;
        derive(s);
        return r;
    }
    if (s->ws) bind_work(s);
    return HPMC_OK;
}

int hpmc_set_moves(hpmc_sim* s, double d_trans, double a_rot, double p_rot, int n_select)
{
    if (!s) return HPMC_EINVAL;
    if (!(d_trans >= 0.0) || !isfinite(d_trans) || !(a_rot >= 0.0) || !isfinite(a_rot) || !(p_rot >= 0.0 && p_rot <= 1.0) ||
        n_select < 1 || n_select > 1024)
        return fail(s, HPMC_EINVAL, "invalid move parameters");
    double od = s->d_trans;
    s->d_trans = d_trans;
    int r = derive(s);  // the shell region depends on d_trans
    if (r != HPMC_OK) {
        s->d_trans = od;
        derive(s);
        return r;
    }
    s->a_rot = a_rot;
    s->p_rot = p_rot;
    s->n_select = n_select;
    if (s->ws) bind_work(s);
    return HPMC_OK;
}

int hpmc_set_insertion(hpmc_sim* s, int region)
{
    if (!s) return HPMC_EINVAL;
    if (region != HPMC_V0_BALL && region != HPMC_V0_SHELL) return fail(s, HPMC_EINVAL, "unknown insertion region");
    int o = s->region;
    s->region = region;
    int r = derive(s);
    if (r != HPMC_OK) {
        s->region = o;
        derive(s);
        return r;
    }
    if (s->ws) bind_work(s);
    return HPMC_OK;
}

int hpmc_workspace_bytes(const hpmc_sim* s, size_t* bytes)
{
    if (!s || !bytes) return HPMC_EINVAL;
    if (!s->have_shape) return HPMC_ESTATE;
    *bytes = layout(s).total;
    return HPMC_OK;
}

int hpmc_set_workspace(hpmc_sim* s, void* dev_ptr, size_t bytes)
{
    if (!s) return HPMC_EINVAL;
    if (!dev_ptr) return fail(s, HPMC_EINVAL, "null workspace");
    if (!s->have_shape) return fail(s, HPMC_ESTATE, "shape not set");
    if (bytes < layout(s).total) return fail(s, HPMC_ENOMEM, "workspace too small");
    const bool fresh = dev_ptr != s->ws;
    s->ws = dev_ptr;
    s->ws_bytes = bytes;
    s->F_dirty = 1;
    bind_work(s);
    if (!s->stream) s->stream = library_stream();
    if (fresh) {
        // new memory: no capacity flag raised yet (the same buffer keeps a pending one)
        hipError_t e = launch_fill_int(s->W.flags, 4, 0, s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "clear flags");
    }
    // the device-side sweep counter lives in the workspace: carry it over
    if (s->have_state) return set_sweep_dev(s);
    return HPMC_OK;
}

int hpmc_set_trace(hpmc_sim* s, int enable)
{
    if (!s) return HPMC_EINVAL;
    s->trace = enable ? 1 : 0;
    s->trace_valid = 0;
    // a larger workspace may now be needed; device calls refuse (ENOMEM) until it is set
    if (s->ws && s->ws_bytes >= layout(s).total) bind_work(s);
    return HPMC_OK;
}

namespace {

// hpmc_set_state on a handle without a workspace: the state is taken and its
// hard-core check runs in the static scratch of the current device
int set_state_static(hpmc_sim* s, double* pos, double* quat, uint64_t sweep_index)
{
    if (!s->stream) s->stream = library_stream();
    s->pos = pos;
    s->quat = s->S.oriented ? quat : nullptr;
    s->W.pos = s->pos;
    s->W.quat = s->quat;
    s->sweep = sweep_index;
    s->trace_valid = 0;
    s->have_state = 0;
    Group g{};
    Work W{};
    unsigned long long* gather = nullptr;
    int r = bind_static(s, g, W, &gather);
    if (r != HPMC_OK) return r;
    hipError_t e = launch_build_cells(g, false, s->stream);
    if (e == hipSuccess) e = launch_fill_u64(W.obs, 1, s->stream);
    if (e == hipSuccess) e = launch_overlap_count(g, s->stream);
    unsigned long long cnt = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, W.obs, 8, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "set_state");
    if (cnt > 0) return fail(s, HPMC_EOVERLAP, std::to_string(cnt) + " overlapping colloid pairs");
    s->have_state = 1;
    s->sweep_dev_stale = 1;  // a workspace set later gets the sweep counter
    return HPMC_OK;
}

}  // namespace

int hpmc_set_state(hpmc_sim* s, double* pos, double* quat, uint64_t sweep_index)
{
    if (!s) return HPMC_EINVAL;
    if (!pos) return fail(s, HPMC_EINVAL, "null positions");
    if (s->have_shape && s->S.oriented && !quat) return fail(s, HPMC_EINVAL, "oriented shape needs quaternions");
    if (s->have_shape && !s->ws) return set_state_static(s, pos, quat, sweep_index);
    int r = check_ready(s, false);
    if (r != HPMC_OK) return r;
    s->pos = pos;
    s->quat = s->S.oriented ? quat : nullptr;
    s->W.pos = s->pos;
    s->W.quat = s->quat;
    s->sweep = sweep_index;
    s->have_state = 1;
    s->trace_valid = 0;
    r = sync_desc(s);
    if (r == HPMC_OK) r = set_sweep_dev(s);
    if (r != HPMC_OK) {
        s->have_state = 0;
        return r;
    }
    // hard-core check on a cell list with zero shift
    Group g = single_group(s);
    hipError_t e = launch_build_cells(g, false, s->stream);
    if (e == hipSuccess) e = launch_fill_u64(s->W.obs, 1, s->stream);
    if (e == hipSuccess) e = launch_overlap_count(g, s->stream);
    unsigned long long cnt = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, s->W.obs, 8, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        s->have_state = 0;
        return hip_fail(s, e, "set_state");
    }
    if (cnt > 0) {
        s->have_state = 0;
        return fail(s, HPMC_EOVERLAP, std::to_string(cnt) + " overlapping colloid pairs");
    }
    return HPMC_OK;
}

int hpmc_get_state(hpmc_sim* s, uint64_t* sweep_index)
{
    if (!s || !sweep_index) return HPMC_EINVAL;
    if (!s->have_state) return HPMC_ESTATE;
    *sweep_index = s->sweep;
    // the state is final once the stream has drained; a capacity flag raised
    // by the sweeps since the last report is reported here
    return s->ws ? check_flags(s) : HPMC_OK;
}

namespace {

// Untimed sweeps of a fixed launch shape replay one captured sweep (a hipGraph
// of its ~20 kernels): the kernels read descriptors and the sweep counter from
// device memory, so the graph stays valid while the groups' shapes do.
// one sweep of every group: group 0 on st, groups 1 to 3 on the owner's side
// streams (forked from and joined back into st by events), any further group
// on st, so groups of different kinds and sizes overlap on the device
hipError_t sweep_groups(hpmc_sim* owner, const std::vector<Group>& groups, hipStream_t st)
{
    if (groups.size() == 1) return launch_sweep(groups[0], nullptr, nullptr, st);
    hipError_t e = hipSuccess;
    if (!owner->fork) e = hipEventCreateWithFlags(&owner->fork, hipEventDisableTiming);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        if (!owner->side[i]) e = hipStreamCreateWithFlags(&owner->side[i], hipStreamNonBlocking);
        if (e == hipSuccess && !owner->join[i]) e = hipEventCreateWithFlags(&owner->join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventRecord(owner->fork, st);
    const size_t nside = std::min<size_t>(groups.size() - 1, 3);
    for (size_t i = 0; i < nside && e == hipSuccess; ++i) {
        e = hipStreamWaitEvent(owner->side[i], owner->fork, 0);
        if (e == hipSuccess) e = launch_sweep(groups[i + 1], nullptr, nullptr, owner->side[i]);
        if (e == hipSuccess) e = hipEventRecord(owner->join[i], owner->side[i]);
    }
    if (e == hipSuccess) e = launch_sweep(groups[0], nullptr, nullptr, st);
    for (size_t i = nside + 1; i < groups.size() && e == hipSuccess; ++i)
        e = launch_sweep(groups[i], nullptr, nullptr, st);
    for (size_t i = 0; i < nside && e == hipSuccess; ++i) e = hipStreamWaitEvent(st, owner->join[i], 0);
    return e;
}

hipError_t run_sweeps(hpmc_sim* owner, const std::vector<Group>& groups, int n, hipStream_t st)
{
    bool all_small = !groups.empty();
    for (const Group& g : groups) all_small = all_small && g.small;
    if (all_small) {
        // every group sweeps in one launch of n sweeps: no graph needed
        hipError_t e = hipSuccess;
        for (const Group& g : groups)
            if (e == hipSuccess && n > 0) e = launch_sweep_small(g, n, st);
        return e;
    }
    std::vector<unsigned char> key(groups.size() * sizeof(Group));
    if (!groups.empty()) memcpy(key.data(), groups.data(), key.size());
    hipError_t e = hipSuccess;
    if (n >= 2 && st != nullptr) {
        if (!owner->graph || owner->graph_key != key) {
            if (owner->graph) {
                (void)hipGraphExecDestroy(owner->graph);
                owner->graph = nullptr;
            }
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) e = sweep_groups(owner, groups, st);
            hipError_t e2 = hipStreamEndCapture(st, &graph);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&owner->graph, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                owner->graph = nullptr;
                return e;
            }
            owner->graph_key = key;
        }
        for (int i = 0; i < n && e == hipSuccess; ++i) e = hipGraphLaunch(owner->graph, st);
        return e;
    }
    for (int i = 0; i < n && e == hipSuccess; ++i) e = sweep_groups(owner, groups, st);
    return e;
}

// events: [0] call start, [1] call end, then (phases begin, phases end) per sweep
int ensure_events(hpmc_sim* s, size_t need)
{
    while (s->events.size() < need) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return hip_fail(s, e, "hipEventCreate");
        s->events.push_back(ev);
    }
    return HPMC_OK;
}

void unpack_counters(const unsigned long long* host, hpmc_counters* out)
{
    memset(out, 0, sizeof(*out));
    uint64_t* o = reinterpret_cast<uint64_t*>(out);
    for (int k = 0; k < kNumCounters; ++k) o[k] = host[k];
}

}  // namespace

int hpmc_sweep(hpmc_sim* s, int n_sweeps, hpmc_counters* out)
{
    if (!s) return HPMC_EINVAL;
    if (n_sweeps < 0) return fail(s, HPMC_EINVAL, "negative sweep count");
    int r = check_ready(s, true);
    if (r == HPMC_OK) r = upload_table(s);
    if (r == HPMC_OK) r = sync_desc(s);
    const bool timed = out != nullptr;
    if (r == HPMC_OK && timed) r = ensure_events(s, 2 * static_cast<size_t>(n_sweeps) + 2);
    if (r != HPMC_OK) return r;
    Group g = single_group(s);
    hipError_t e = timed ? hipEventRecord(s->events[0], s->stream) : hipSuccess;
    if (e == hipSuccess) e = launch_clear_counters(g, s->stream);
    if (timed) {
        for (int i = 0; i < n_sweeps && e == hipSuccess; ++i)
            e = launch_sweep(g, s->events[2 + 2 * i], s->events[3 + 2 * i], s->stream);
    } else if (e == hipSuccess) {
        e = run_sweeps(s, std::vector<Group>{g}, n_sweeps, s->stream);
    }
    if (e != hipSuccess) return hip_fail(s, e, "sweep launch");
    s->sweep += static_cast<uint64_t>(n_sweeps);
    s->trace_valid = s->trace && n_sweeps > 0;
    if (out) {
        unsigned long long host[kCounterStride];
        e = launch_reduce_counters(g, s->d_gather, s->stream);
        if (e == hipSuccess) e = hipEventRecord(s->events[1], s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(host, s->d_gather, sizeof(host), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "sweep counters");
        unpack_counters(host, out);
        double phase_ms = 0.0;
        for (int i = 0; i < n_sweeps; ++i) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, s->events[2 + 2 * i], s->events[3 + 2 * i]);
            if (e != hipSuccess) return hip_fail(s, e, "hipEventElapsedTime");
            phase_ms += ms;
        }
        float all = 0.0f;
        e = hipEventElapsedTime(&all, s->events[0], s->events[1]);
        if (e != hipSuccess) return hip_fail(s, e, "hipEventElapsedTime");
        out->phase_kernel_ms = phase_ms;
        out->sweep_ms = all;
        return report_flags(s, static_cast<int>(host[kNumCounters]));
    }
    return HPMC_OK;
}

int hpmc_sweep_static(hpmc_sim* s, int n_sweeps, hpmc_counters* out)
{
    if (!s) return HPMC_EINVAL;
    if (n_sweeps < 0) return fail(s, HPMC_EINVAL, "negative sweep count");
    if (!s->stream) s->stream = library_stream();
    if (!s->have_shape) return fail(s, HPMC_ESTATE, "shape not set");
    if (!s->have_state) return fail(s, HPMC_ESTATE, "state not set");
    if (s->trace) return fail(s, HPMC_EINVAL, "tracing writes into the caller's workspace; use hpmc_sweep");
    Group g{};
    Work W{};
    unsigned long long* gather = nullptr;
    int r = bind_static(s, g, W, &gather);
    if (r != HPMC_OK) return r;
    hipError_t e = launch_clear_counters(g, s->stream);
    if (g.small) {
        if (e == hipSuccess && n_sweeps > 0) e = launch_sweep_small(g, n_sweeps, s->stream);
    } else {
        for (int i = 0; i < n_sweeps && e == hipSuccess; ++i) e = launch_sweep(g, nullptr, nullptr, s->stream);
    }
    if (e != hipSuccess) return hip_fail(s, e, "static sweep launch");
    s->sweep += static_cast<uint64_t>(n_sweeps);
    s->sweep_dev_stale = 1;  // the caller's workspace, if any, still holds the old sweep index
    s->trace_valid = 0;
    if (out) {
        unsigned long long host[kCounterStride];
        e = launch_reduce_counters(g, gather, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(host, gather, sizeof(host), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "static sweep counters");
        unpack_counters(host, out);
        if (host[kNumCounters])
            return fail(s, HPMC_ECAPACITY, "a cell's stencil exceeded its capacity; its trials were skipped");
    }
    return HPMC_OK;
}

int hpmc_set_tuning(hpmc_sim* s, const hpmc_tuning* t)
{
    if (!s) return HPMC_EINVAL;
    if (!t) return fail(s, HPMC_EINVAL, "null tuning");
    if (t->cells_per_wave < 0 || t->cells_per_wave > 64 || t->max_waves < 0 ||
        !(t->waves_per_block == 0 || t->waves_per_block == 1 || t->waves_per_block == 2 || t->waves_per_block == 4))
        return fail(s, HPMC_EINVAL, "launch shape out of range");
    s->tune_chunk = t->cells_per_wave;
    s->tune_wpb = t->waves_per_block;
    s->tune_waves = t->max_waves;
    s->desc_dirty = 1;
    return HPMC_OK;
}

int hpmc_autotune(hpmc_sim* s, void* scratch, size_t bytes, int sweeps, hpmc_tuning* out)
{
    if (!s) return HPMC_EINVAL;
    if (!scratch || sweeps < 1 || sweeps > 64) return fail(s, HPMC_EINVAL, "autotune needs scratch and 1..64 sweeps");
    int r = check_ready(s, true);
    if (r != HPMC_OK) return r;
    const size_t N = static_cast<size_t>(s->N);
    const size_t need = N * 3 * sizeof(double) + (s->S.oriented ? N * 4 * sizeof(double) : 0);
    if (bytes < need) return fail(s, HPMC_ENOMEM, "autotune scratch smaller than the state");
    const std::vector<hpmc_tuning> cand = tuning_candidates(s->S.oriented != 0);
    // run on a copy of the state; restore everything afterwards
    double* pos0 = s->pos;
    double* quat0 = s->quat;
    const uint64_t sweep0 = s->sweep;
    const int trace0 = s->trace;
    const int c0 = s->tune_chunk, w0 = s->tune_wpb, m0 = s->tune_waves;
    double* spos = static_cast<double*>(scratch);
    double* squat = s->S.oriented ? spos + 3 * N : nullptr;
    hipError_t e = hipMemcpyAsync(spos, pos0, N * 3 * sizeof(double), hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && squat)
        e = hipMemcpyAsync(squat, quat0, N * 4 * sizeof(double), hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "autotune copy");
    s->pos = spos;
    s->quat = squat;
    s->W.pos = spos;
    s->W.quat = squat;
    s->trace = 0;
    s->desc_dirty = 1;
    int best = -1;
    double best_ms = 0.0, default_ms = 0.0;
    for (size_t i = 0; i < cand.size() && r == HPMC_OK; ++i) {
        s->tune_chunk = cand[i].cells_per_wave;
        s->tune_wpb = cand[i].waves_per_block;
        s->tune_waves = cand[i].max_waves;
        s->desc_dirty = 1;
        hpmc_counters c{};
        r = hpmc_sweep(s, 1, &c);
        if (r == HPMC_OK) r = hpmc_sweep(s, sweeps, &c);
        if (r != HPMC_OK) break;
        double ms = c.phase_kernel_ms / sweeps;
        if (i == 0) default_ms = ms;
        if (best < 0 || ms < best_ms) {
            best = static_cast<int>(i);
            best_ms = ms;
        }
    }
    // restore the state pointers, the sweep index and its device copy
    s->pos = pos0;
    s->quat = quat0;
    s->W.pos = pos0;
    s->W.quat = quat0;
    s->trace = trace0;
    s->trace_valid = 0;
    s->sweep = sweep0;
    s->desc_dirty = 1;
    int r2 = set_sweep_dev(s);
    if (r == HPMC_OK && r2 != HPMC_OK) r = r2;
    e = hipStreamSynchronize(s->stream);
    if (r == HPMC_OK && e != hipSuccess) r = hip_fail(s, e, "autotune");
    if (r != HPMC_OK) {
        s->tune_chunk = c0;
        s->tune_wpb = w0;
        s->tune_waves = m0;
        return r;
    }
    s->tune_chunk = cand[best].cells_per_wave;
    s->tune_wpb = cand[best].waves_per_block;
    s->tune_waves = cand[best].max_waves;
    if (out) {
        *out = cand[best];
        out->candidates = static_cast<int32_t>(cand.size());
        out->best_ms = best_ms;
        out->default_ms = default_ms;
    }
    return HPMC_OK;
}

namespace {

// Descriptors of a batched sweep go to the batch workspace from one of the
// leader's pinned staging buffers, with no host synchronisation: the copy is
// ordered on the stream after the previous call's kernels, and a staging
// buffer is rewritten only once its previous copy completed (with four in
// turn, the host may enqueue that many calls ahead of the device).
int upload_batch(hpmc_sim* lead, void* dst, const std::vector<unsigned char>& host, hipStream_t st)
{
    const size_t bytes = host.size();
    const int k = lead->batch_next;
    lead->batch_next = (k + 1) % hpmc_sim::kStages;
    hipError_t e = hipSuccess;
    if (lead->batch_up[k]) e = hipEventSynchronize(lead->batch_up[k]);
    if (e == hipSuccess && lead->batch_stage_cap[k] < bytes) {
        if (lead->batch_stage[k]) e = hipHostFree(lead->batch_stage[k]);
        lead->batch_stage[k] = nullptr;
        lead->batch_stage_cap[k] = 0;
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&lead->batch_stage[k]), bytes, hipHostMallocDefault);
        if (e == hipSuccess) lead->batch_stage_cap[k] = bytes;
    }
    if (e == hipSuccess && !lead->batch_up[k]) e = hipEventCreateWithFlags(&lead->batch_up[k], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(lead, e, "batch descriptor staging");
    memcpy(lead->batch_stage[k], host.data(), bytes);
    e = hipMemcpyAsync(dst, lead->batch_stage[k], bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(lead->batch_up[k], st);
    if (e != hipSuccess) return hip_fail(lead, e, "batch descriptor upload");
    return HPMC_OK;
}

// batch workspace: descriptors, then the block-to-replica map of the phase
// launches (at most kMaxReplicaBlocks blocks per replica), then counters
struct BatchLayout {
    size_t desc, brep, gather, total;
};

BatchLayout batch_layout(int n_sims)
{
    BatchLayout l{};
    const size_t n = static_cast<size_t>(n_sims);
    l.desc = 0;
    l.brep = align256(n * sizeof(Desc));
    l.gather = l.brep + align256(n * kMaxReplicaBlocks * sizeof(int));
    l.total = l.gather + align256(n * kCounterStride * 8);
    return l;
}

}  // namespace

int hpmc_batch_workspace_bytes(int n_sims, size_t* bytes)
{
    if (n_sims < 1 || !bytes) return HPMC_EINVAL;
    *bytes = batch_layout(n_sims).total;
    return HPMC_OK;
}

int hpmc_sweep_batch(hpmc_sim* const* sims, int n_sims, void* batch_ws, size_t bytes, int n_sweeps,
                     hpmc_counters* out)
{
    if (!sims || n_sims < 1 || n_sweeps < 0) return HPMC_EINVAL;
    size_t need = 0;
    hpmc_batch_workspace_bytes(n_sims, &need);
    if (!batch_ws || bytes < need) {
        if (sims[0]) fail(sims[0], HPMC_ENOMEM, "batch workspace missing or too small");
        return HPMC_ENOMEM;
    }
    // every replica's derived parameters, once per call
    std::vector<Params> par(static_cast<size_t>(n_sims));
    for (int i = 0; i < n_sims; ++i) {
        if (!sims[i]) return HPMC_EINVAL;
        int r = check_ready(sims[i], true, &par[static_cast<size_t>(i)]);
        // a member's own uploads (its table, below) go on its stream: the batch
        // runs on the first member's, so one stream for all keeps them ordered
        if (r == HPMC_OK && sims[i]->stream != sims[0]->stream)
            r = fail(sims[0], HPMC_EINVAL, "every handle of a batch must use the stream of the first");
        if (r == HPMC_OK) r = upload_table(sims[i]);
        if (r != HPMC_OK) return r;
        if (sims[i]->trace) return fail(sims[i], HPMC_EINVAL, "tracing is per handle; disable it for batched sweeps");
    }
    hipStream_t st = sims[0]->stream;
    // replicas that share a shape kind, precision and insertion region share each launch
    const BatchLayout bl = batch_layout(n_sims);
    unsigned char* base = static_cast<unsigned char*>(batch_ws);
    Desc* d_all = reinterpret_cast<Desc*>(base + bl.desc);
    int* d_brep = reinterpret_cast<int*>(base + bl.brep);
    unsigned long long* d_gather = reinterpret_cast<unsigned long long*>(base + bl.gather);
    std::vector<int> cl(static_cast<size_t>(n_sims));
    for (int i = 0; i < n_sims; ++i) cl[static_cast<size_t>(i)] = batch_class(sims[i], par[static_cast<size_t>(i)]);
    auto cls = [&](int i) { return cl[static_cast<size_t>(i)]; };
    // within a group, the most crowded cells first: their blocks are dispatched
    // first, since their serial chains of trials set the length of a phase
    auto crowd = [&](int i) {
        const Params& Pi = par[static_cast<size_t>(i)];
        return static_cast<double>(Pi.N) / static_cast<double>(Pi.ncells);
    };
    std::vector<int> order;
    for (int k = 0; k < kBatchClasses; ++k) {
        const size_t first = order.size();
        for (int i = 0; i < n_sims; ++i)
            if (cls(i) == k) order.push_back(i);
        std::stable_sort(order.begin() + static_cast<std::ptrdiff_t>(first), order.end(),
                         [&](int a, int b) { return crowd(a) > crowd(b); });
    }
    std::vector<Desc> host(static_cast<size_t>(n_sims));
    std::vector<int> brep;
    std::vector<Group> groups;
    for (size_t b = 0; b < order.size();) {
        size_t e = b;
        while (e < order.size() && cls(order[e]) == cls(order[b])) ++e;
        std::vector<const hpmc_sim*> members;
        std::vector<Params> mpar;
        for (size_t q = b; q < e; ++q) {
            members.push_back(sims[order[q]]);
            mpar.push_back(par[static_cast<size_t>(order[q])]);
        }
        Group g = make_group(d_all + b, members.data(), static_cast<int>(members.size()), mpar.data());
        // flat phase launch: each replica's own blocks, one after another
        const size_t first_block = brep.size();
        for (size_t q = b; q < e; ++q) {
            Desc d = make_desc(sims[order[q]], par[static_cast<size_t>(order[q])], g.wpb, g.chunk);
            if (g.kind == kSphere) {
                // a wave takes one chunk of cells: a large box takes larger chunks
                while (d.P.nblk > kMaxReplicaBlocks && d.P.chunk < 64) {
                    d.P.chunk = std::min(64, 2 * d.P.chunk);
                    d.P.nblk = phase_blocks(kSphere, d.P.active_cells, d.P.chunk, g.wpb, 0);
                }
                if (d.P.nblk > kMaxReplicaBlocks)
                    return fail(sims[0], HPMC_ECAPACITY, "replica " + std::to_string(order[q]) +
                                                              " is too large for a batched sweep; sweep it alone");
            }
            // oriented shapes: the waves of a capped replica take several cells in turn
            int nb = std::min(d.P.nblk, kMaxReplicaBlocks);
            d.P.blk0 = static_cast<int>(brep.size() - first_block);
            d.P.nblk = nb;
            brep.insert(brep.end(), static_cast<size_t>(nb), static_cast<int>(q - b));
            host[q] = d;
        }
        g.brep = d_brep + first_block;
        g.nblocks = static_cast<int>(brep.size() - first_block);
        groups.push_back(g);
        b = e;
    }
    {
        // descriptors and block map in one copy (they are adjacent)
        std::vector<unsigned char> up(bl.brep + brep.size() * sizeof(int));
        memcpy(up.data(), host.data(), host.size() * sizeof(Desc));
        if (!brep.empty()) memcpy(up.data() + bl.brep, brep.data(), brep.size() * sizeof(int));
        int ru = upload_batch(sims[0], base, up, st);
        if (ru != HPMC_OK) return ru;
    }
    hipError_t e = hipSuccess;
    if (out) {
        int re = ensure_events(sims[0], 2);
        if (re != HPMC_OK) return re;
    }
    for (const Group& g : groups)
        if (e == hipSuccess) e = launch_clear_counters(g, st);
    // with counters: the device time of the sweeps of every group, on the lead stream
    if (e == hipSuccess && out) e = hipEventRecord(sims[0]->events[0], st);
    if (e == hipSuccess) e = run_sweeps(sims[0], groups, n_sweeps, st);
    if (e == hipSuccess && out) e = hipEventRecord(sims[0]->events[1], st);
    if (e != hipSuccess) return hip_fail(sims[0], e, "batched sweep launch");
    for (int i = 0; i < n_sims; ++i) sims[i]->sweep += static_cast<uint64_t>(n_sweeps);
    if (out) {
        std::vector<unsigned long long> hc(static_cast<size_t>(n_sims) * kCounterStride);
        size_t off = 0;
        for (const Group& g : groups) {
            if (e == hipSuccess) e = launch_reduce_counters(g, d_gather + off * kCounterStride, st);
            off += static_cast<size_t>(g.nrep);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(hc.data(), d_gather, hc.size() * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(sims[0], e, "batched counters");
        float all = 0.0f;
        e = hipEventElapsedTime(&all, sims[0]->events[0], sims[0]->events[1]);
        if (e != hipSuccess) return hip_fail(sims[0], e, "hipEventElapsedTime");
        int r = HPMC_OK;
        for (size_t q = 0; q < order.size(); ++q) {
            unpack_counters(&hc[q * kCounterStride], &out[order[q]]);
            out[order[q]].sweep_ms = all;  // the whole batch's sweeps (phase launches not timed apart)
            const int f = static_cast<int>(hc[q * kCounterStride + kNumCounters]);
            if (f) {
                hpmc_sim* x = sims[order[q]];
                int rq = report_flags(x, f);
                if (r == HPMC_OK) {
                    r = rq;
                    if (x != sims[0]) fail(sims[0], rq, "replica " + std::to_string(order[q]) + ": " + x->err);
                }
            }
        }
        return r;
    }
    return HPMC_OK;
}

int hpmc_autotune_batch(hpmc_sim* const* sims, int n_sims, void* batch_ws, size_t ws_bytes, void* scratch,
                        size_t scratch_bytes, int sweeps, hpmc_tuning* out)
{
    if (!sims || n_sims < 1) return HPMC_EINVAL;
    for (int i = 0; i < n_sims; ++i)
        if (!sims[i]) return HPMC_EINVAL;
    hpmc_sim* s0 = sims[0];
    if (!scratch || sweeps < 1 || sweeps > 64) return fail(s0, HPMC_EINVAL, "autotune needs scratch and 1..64 sweeps");
    std::vector<const hpmc_sim*> sorted(sims, sims + n_sims);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(s0, HPMC_EINVAL, "a handle appears twice in the batch");
    std::vector<int> cl(static_cast<size_t>(n_sims));
    std::vector<size_t> off(static_cast<size_t>(n_sims));
    size_t need = 0;
    for (int i = 0; i < n_sims; ++i) {
        hpmc_sim* x = sims[i];
        Params Px;
        int r = check_ready(x, true, &Px);
        if (r != HPMC_OK) return r;
        // the copies below and the synchronisation at the end use this stream,
        // and each group's sweeps that of its first member
        if (x->stream != s0->stream) return fail(s0, HPMC_EINVAL, "every handle of a batch must use the stream of the first");
        if (x->trace) return fail(x, HPMC_EINVAL, "tracing is per handle; disable it for batched sweeps");
        cl[static_cast<size_t>(i)] = batch_class(x, Px);
        off[static_cast<size_t>(i)] = need;
        const size_t N = static_cast<size_t>(x->N);
        need += (N * 3 * sizeof(double) + (x->S.oriented ? N * 4 * sizeof(double) : 0) + 255) / 256 * 256;
    }
    if (scratch_bytes < need) return fail(s0, HPMC_ENOMEM, "autotune scratch smaller than the states of the batch");
    // every member sweeps a copy of its state; pointers, sweep index and
    // launch shape are restored afterwards
    struct Saved {
        double* pos;
        double* quat;
        uint64_t sweep;
        int chunk, wpb, waves;
    };
    std::vector<Saved> sv(static_cast<size_t>(n_sims));
    hipStream_t st = s0->stream;
    hipError_t e = hipSuccess;
    for (int i = 0; i < n_sims && e == hipSuccess; ++i) {
        hpmc_sim* x = sims[i];
        const size_t N = static_cast<size_t>(x->N);
        sv[static_cast<size_t>(i)] = Saved{x->pos, x->quat, x->sweep, x->tune_chunk, x->tune_wpb, x->tune_waves};
        double* cp = reinterpret_cast<double*>(static_cast<unsigned char*>(scratch) + off[static_cast<size_t>(i)]);
        double* cq = x->S.oriented ? cp + 3 * N : nullptr;
        e = hipMemcpyAsync(cp, x->pos, N * 3 * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && cq) e = hipMemcpyAsync(cq, x->quat, N * 4 * sizeof(double), hipMemcpyDeviceToDevice, st);
        x->pos = cp;
        x->quat = cq;
        x->W.pos = cp;
        x->W.quat = cq;
        x->desc_dirty = 1;
    }
    int r = e == hipSuccess ? HPMC_OK : hip_fail(s0, e, "autotune copy");
    std::vector<hpmc_tuning> chosen(static_cast<size_t>(n_sims));
    for (int i = 0; i < n_sims; ++i)
        chosen[static_cast<size_t>(i)] = hpmc_tuning{sims[i]->tune_chunk, sims[i]->tune_wpb, sims[i]->tune_waves, 0, 0.0, 0.0};
    // each launch group alone: the candidate shapes on all its members at once
    for (int k = 0; k < kBatchClasses && r == HPMC_OK; ++k) {
        std::vector<hpmc_sim*> mem;
        for (int i = 0; i < n_sims; ++i)
            if (cl[static_cast<size_t>(i)] == k) mem.push_back(sims[i]);
        if (mem.empty() || class_is_small(k)) continue;  // one workgroup per small replica: no shape to tune
        const std::vector<hpmc_tuning> cand = tuning_candidates(mem[0]->S.oriented != 0);
        std::vector<hpmc_counters> cnt(mem.size());
        int best = -1;
        double best_ms = 0.0, default_ms = 0.0;
        for (size_t c = 0; c < cand.size() && r == HPMC_OK; ++c) {
            for (hpmc_sim* x : mem) {
                x->tune_chunk = cand[c].cells_per_wave;
                x->tune_wpb = cand[c].waves_per_block;
                x->tune_waves = cand[c].max_waves;
                x->desc_dirty = 1;
            }
            const int nm = static_cast<int>(mem.size());
            r = hpmc_sweep_batch(mem.data(), nm, batch_ws, ws_bytes, 1, nullptr);
            if (r == HPMC_OK) r = hpmc_sweep_batch(mem.data(), nm, batch_ws, ws_bytes, sweeps, cnt.data());
            if (r != HPMC_OK) break;
            const double ms = cnt[0].sweep_ms / sweeps;
            if (c == 0) default_ms = ms;
            if (best < 0 || ms < best_ms) {
                best = static_cast<int>(c);
                best_ms = ms;
            }
        }
        if (r != HPMC_OK) break;
        for (int i = 0; i < n_sims; ++i)
            if (cl[static_cast<size_t>(i)] == k) {
                chosen[static_cast<size_t>(i)] = cand[static_cast<size_t>(best)];
                chosen[static_cast<size_t>(i)].candidates = static_cast<int32_t>(cand.size());
                chosen[static_cast<size_t>(i)].best_ms = best_ms;
                chosen[static_cast<size_t>(i)].default_ms = default_ms;
            }
    }
    // restore every member (also after an error), then hand out the shapes
    for (int i = 0; i < n_sims; ++i) {
        hpmc_sim* x = sims[i];
        const Saved& v = sv[static_cast<size_t>(i)];
        if (!v.pos) continue;  // not reached by the copy loop
        x->pos = v.pos;
        x->quat = v.quat;
        x->W.pos = v.pos;
        x->W.quat = v.quat;
        x->sweep = v.sweep;
        x->trace_valid = 0;
        x->tune_chunk = v.chunk;
        x->tune_wpb = v.wpb;
        x->tune_waves = v.waves;
        x->desc_dirty = 1;
        int r2 = set_sweep_dev(x);
        if (r == HPMC_OK && r2 != HPMC_OK) r = r2;
    }
    e = hipStreamSynchronize(st);
    if (r == HPMC_OK && e != hipSuccess) r = hip_fail(s0, e, "autotune");
    if (r != HPMC_OK) return r;
    for (int i = 0; i < n_sims; ++i) {
        sims[i]->tune_chunk = chosen[static_cast<size_t>(i)].cells_per_wave;
        sims[i]->tune_wpb = chosen[static_cast<size_t>(i)].waves_per_block;
        sims[i]->tune_waves = chosen[static_cast<size_t>(i)].max_waves;
        if (out) out[i] = chosen[static_cast<size_t>(i)];
    }
    return HPMC_OK;
}

int hpmc_poisson_draw(const hpmc_sim* s, double u, int32_t* k)
{
    if (!s || !k) return HPMC_EINVAL;
    if (!(u > 0.0 && u < 1.0)) return HPMC_EINVAL;
    if (!s->table_set) return HPMC_ESTATE;
    *k = poisson_compact_draw(s->F, s->G, u, s->pk_min, s->pk_n);
    return HPMC_OK;
}

int hpmc_trace(hpmc_sim* s, hpmc_move_record* buf, int64_t cap, int64_t* n_written)
{
    if (!s || !n_written || (cap > 0 && !buf)) return HPMC_EINVAL;
    *n_written = 0;
    if (!s->trace || !s->trace_valid) return fail(s, HPMC_ESTATE, "no traced sweep");
    int rf = check_flags(s);
    if (rf != HPMC_OK) return rf;
    int64_t n = s->N * s->n_select;
    if (n > cap) n = cap;
    if (n > 0) {
        hipError_t e = hipMemcpyAsync(buf, s->W.trace, static_cast<size_t>(n) * sizeof(hpmc_move_record),
                                      hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "trace copy");
    }
    *n_written = n;
    return HPMC_OK;
}

int hpmc_observables(hpmc_sim* s, int kind, const hpmc_obs_params* p, double* out, int64_t out_len)
{
    if (!s) return HPMC_EINVAL;
    if (!p || !out) return fail(s, HPMC_EINVAL, "null observable arguments");
    int r = check_ready(s, true);
    if (r == HPMC_OK) r = sync_desc(s);
    if (r == HPMC_OK) r = check_flags(s);
    if (r != HPMC_OK) return r;
    Params P = make_params(s);
    Group g = single_group(s);
    const double V = s->L * s->L * s->L;
    auto run_cells = [&]() { return launch_build_cells(g, false, s->stream); };
    auto fetch = [&](int n, std::vector<unsigned long long>& h, int first) {
        h.assign(static_cast<size_t>(n), 0ull);
        hipError_t e = hipMemcpyAsync(h.data(), s->W.obs + first, static_cast<size_t>(n) * 8, hipMemcpyDeviceToHost,
                                      s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        return e;
    };
    std::vector<unsigned long long> h;
    if (kind == HPMC_OBS_GR) {
        int nb = p->n_bins;
        if (nb < 1 || nb > kObsWords || out_len < nb || !(p->r_max > 0.0) || p->r_max > s->halfL)
            return fail(s, HPMC_EINVAL, "bad g(r) parameters");
        hipError_t e = run_cells();
        if (e == hipSuccess) e = launch_gr(g, P, s->W, nb, p->r_max, s->stream);
        if (e == hipSuccess) e = fetch(nb, h, 0);
        if (e != hipSuccess) return hip_fail(s, e, "g(r)");
        double npair = 0.5 * static_cast<double>(s->N) * static_cast<double>(s->N - 1);
        double dr = p->r_max / static_cast<double>(nb);
        for (int b = 0; b < nb; ++b) {
            double r0 = static_cast<double>(b) * dr, r1 = static_cast<double>(b + 1) * dr;
            double shell = 4.0 / 3.0 * M_PI * (r1 * r1 * r1 - r0 * r0 * r0);
            out[b] = static_cast<double>(h[static_cast<size_t>(b)]) / (npair * shell / V);
        }
        return HPMC_OK;
    }
    auto probes = [&](double scale, int slot) {
        hipError_t e = launch_free_volume(g, p->n_probe, p->obs_seq, scale, slot, s->stream);
        return e;
    };
    if (kind == HPMC_OBS_FREE_VOLUME) {
        if (out_len < 3 || p->n_probe < 1 || p->n_probe > 0xFFFFFFFFll)
            return fail(s, HPMC_EINVAL, "bad free-volume parameters");
        hipError_t e = run_cells();
        if (e == hipSuccess) e = launch_fill_u64(s->W.obs, 1, s->stream);
        if (e == hipSuccess) e = probes(1.0, 0);
        if (e == hipSuccess) e = fetch(1, h, 0);
        if (e != hipSuccess) return hip_fail(s, e, "free volume");
        double alpha = static_cast<double>(h[0]) / static_cast<double>(p->n_probe);
        double phi_r = M_PI / 6.0 * s->d_dep * s->d_dep * s->d_dep * s->z_p;
        out[0] = alpha;
        out[1] = phi_r * alpha;
        out[2] = static_cast<double>(h[0]);
        return HPMC_OK;
    }
    if (kind == HPMC_OBS_SDF) {
        int nb = p->n_bins;
        if (nb < 2 || nb > kObsWords - 2 || out_len < 4 + nb || !(p->x_max > 0.0) || p->x_max >= 1.0 || p->n_fit < 2 ||
            p->n_fit > nb || p->n_probe < 0 || p->n_probe > 0xFFFFFFFFll)
            return fail(s, HPMC_EINVAL, "bad SDF parameters");
        hipError_t e = run_cells();
        if (e == hipSuccess) e = launch_sdf(g, P, s->W, nb, p->x_max, s->stream);
        if (e == hipSuccess) e = fetch(nb, h, 0);
        if (e != hipSuccess) return hip_fail(s, e, "SDF");
        double* hist = out + 4;
        double dx = p->x_max / static_cast<double>(nb);
        for (int b = 0; b < nb; ++b)
            hist[b] = static_cast<double>(h[static_cast<size_t>(b)]) / (static_cast<double>(s->N) * dx);
        double sx = 0, sy = 0, sxx = 0, sxy = 0;
        int nf = p->n_fit;
        for (int b = 0; b < nf; ++b) {
            double xb = (static_cast<double>(b) + 0.5) * dx;
            sx += xb;
            sy += hist[b];
            sxx += xb * xb;
            sxy += xb * hist[b];
        }
        double den = static_cast<double>(nf) * sxx - sx * sx;
        double slope = (static_cast<double>(nf) * sxy - sx * sy) / den;
        double s0 = (sy - slope * sx) / static_cast<double>(nf);
        double rho = static_cast<double>(s->N) / V;
        double bp_hard = rho * (1.0 + s0 / 6.0);
        double bp_dep = 0.0;
        if (s->z_p > 0.0 && p->n_probe > 0) {
            const int s0slot = kObsWords - 2, s1slot = kObsWords - 1;
            double sc = 1.0 + p->eps;
            e = launch_fill_u64(s->W.obs + s0slot, 2, s->stream);
            if (e == hipSuccess) e = probes(1.0, s0slot);
            if (e == hipSuccess) e = probes(sc, s1slot);
            if (e == hipSuccess) e = fetch(2, h, s0slot);
            if (e != hipSuccess) return hip_fail(s, e, "SDF probes");
            double g3 = sc * sc * sc;
            double a0 = static_cast<double>(h[0]) / static_cast<double>(p->n_probe);
            double a1 = static_cast<double>(h[1]) / static_cast<double>(p->n_probe);
            bp_dep = s->z_p * ((g3 * a1 - a0) / (g3 - 1.0));
        }
        out[0] = bp_hard + bp_dep;
        out[1] = bp_hard;
        out[2] = bp_dep;
        out[3] = s0;
        return HPMC_OK;
    }
    return fail(s, HPMC_EINVAL, "unknown observable");
}

}  // extern "C"

static_assert(sizeof(hpmc_move_record) == 40, "record layout");
static_assert(sizeof(hpmc_counters) == kNumCounters * 8 + 16, "counter layout");
