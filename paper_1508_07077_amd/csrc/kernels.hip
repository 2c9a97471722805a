// kernels.hip -- HIP kernels of one implicit-depletant hard-particle Monte
// Carlo sweep on CDNA4 (gfx950).
//
// Method: Glaser, Karas & Glotzer, arXiv:1508.07077.
//   grid_kernel ............ random colour order and grid shift (Sec. III.E)
//   bin / scan / scatter /
//   rank / gather .......... cell list under the shifted checkerboard (Sec. III.E)
//   phase_kernel ........... trial moves of one colour: proposal, hard overlap
//                            (Eq. pacc), Poisson depletants in the circumsphere
//                            (Sec. III.B step 2, Sec. III.C), classification and
//                            early exit (Sec. III.B step 3, Fig. 2, App. A),
//                            configurational bias (Sec. III.D, Eq. pacc_cb)
//   scatter_back ........... cell-ordered records back to the caller's SoA state
//
// Mapping: one wavefront runs the active cells of a chunk one after another
// (spheres: 8 cells by default, one wave per workgroup; oriented shapes: one
// cell at a time).  The draws of a cell's trials that depend on the random
// streams alone come from one Philox pass for several trials.  In a
// depletant pass, lanes draw one Philox block each (two ball candidates);
// accepted candidates get their depletant index from a ballot + popcount
// prefix, so the wave resolves ~67 depletants per pass in exactly the serial
// order.  Depletants that survive the cheap old-pose test (a few per move) are
// tested against the cell stencil lane-per-neighbour, and CB re-insertions of
// a blocking depletant run lane-per-trial.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"
#include "rng.hpp"

namespace hpmc {

namespace {

// Address spaces of the phase kernels' memory: LDS and global.  Pointers
// typed with them compile to ds_* and global_* instructions instead of flat
// ones, whose completion the wave could only await together (an LDS read
// would then also wait for the next cell's records still streaming in).
#define LAS __attribute__((address_space(3)))
#define GAS __attribute__((address_space(1)))

// the phase kernels' view of a replica's workspace, with global pointers
struct WorkG {
    const GAS int* cell_start;
    GAS double4* rpos;
    GAS double4* rquat;
    const GAS double* F;
    const GAS double* grid;
    const GAS int* perm;
    GAS unsigned long long* counters;
    GAS int* flags;
    GAS unsigned char* trace;
    const GAS uint32_t* sweep_dev;
};

__device__ inline WorkG gview(const Work& W)
{
    WorkG g;
    g.cell_start = (const GAS int*)W.cell_start;
    g.rpos = (GAS double4*)W.rpos;
    g.rquat = (GAS double4*)W.rquat;
    g.F = (const GAS double*)W.F;
    g.grid = (const GAS double*)W.grid;
    g.perm = (const GAS int*)W.perm;
    g.counters = (GAS unsigned long long*)W.counters;
    g.flags = (GAS int*)W.flags;
    g.trace = (GAS unsigned char*)W.trace;
    g.sweep_dev = (const GAS uint32_t*)W.sweep_dev;
    return g;
}

// 32-byte records in global memory (the vector types take no address-space
// qualified references, so the four words are moved one by one; the compiler
// merges them into wide loads and stores)
__device__ inline double4 rd4(const GAS double4* p, size_t i)
{
    const GAS double* q = (const GAS double*)(p + i);
    return make_double4(q[0], q[1], q[2], q[3]);
}

__device__ inline void wr4(GAS double4* p, size_t i, double4 v)
{
    GAS double* q = (GAS double*)(p + i);
    q[0] = v.x;
    q[1] = v.y;
    q[2] = v.z;
    q[3] = v.w;
}

// the same through plain (generic) pointers, for the kernels that use them
__device__ inline double4 rd4(const double4* p, size_t i) { return p[i]; }
__device__ inline void wr4(double4* p, size_t i, double4 v) { p[i] = v; }

// LDS base of the dynamic shared memory
__device__ inline LAS unsigned char* lds_base()
{
    extern __shared__ __align__(16) unsigned char smem[];
    return (LAS unsigned char*)smem;
}

constexpr double kFar = 1.0e30;

__device__ inline double mi(const Params& P, double d)
{
    if (d > P.halfL)
        d -= P.L;
    else if (d < -P.halfL)
        d += P.L;
    return d;
}

__device__ inline int cell_coord(const Params& P, double x, double g)
{
    double y = x - g;
    if (y < 0.0) y += P.L;
    int c = static_cast<int>(floor(y * P.inv_w));
    if (c > P.n - 1) c = P.n - 1;
    if (c < 0) c = 0;
    return c;
}

__device__ inline int cell_of(const Params& P, double x, double y, double z, double g0, double g1, double g2)
{
    int cx = cell_coord(P, x, g0), cy = cell_coord(P, y, g1), cz = cell_coord(P, z, g2);
    return cx + P.n * (cy + P.n * cz);
}

__device__ inline int lane_id() { return __lane_id(); }

// periodic wrap of a cell coordinate that is at most one cell outside [0, n)
__device__ inline int wrap1(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }
// cell id of packed coordinates cx | cy << 10 | cz << 20 (at most 1024 cells per axis)
__device__ inline int cell_id(const Params& P, int X) { return (X & 1023) + P.n * (((X >> 10) & 1023) + P.n * (X >> 20)); }

// this lane's offset in the de-duplicated cell stencil: 27 lanes over
// {0, -1, +1}^3 (n > 2) or 8 lanes over {0, +1}^3 (n = 2); lane 0 is the cell
// itself (divisions by the constant 3 only)
struct NbOff {
    int dx, dy, dz;
    bool on;
};
__device__ inline NbOff nb_offset(int n)
{
    int l = lane_id();
    // opaque to the optimiser: the offsets are recomputed where they are used
    // (a few integer operations) instead of held in registers across loops
    asm volatile("" : "+v"(l));
    NbOff o;
    if (n == 2) {
        o.on = l < 8;
        o.dx = l & 1;
        o.dy = (l >> 1) & 1;
        o.dz = (l >> 2) & 1;
    } else {
        o.on = l < 27;
        int ix = l % 3, iy = (l / 3) % 3, iz = l / 9;
        o.dx = ix == 1 ? -1 : (ix == 2 ? 1 : 0);
        o.dy = iy == 1 ? -1 : (iy == 2 ? 1 : 0);
        o.dz = iz == 1 ? -1 : (iz == 2 ? 1 : 0);
    }
    return o;
}

// number of set bits of `mask` in lanes below this one
__device__ inline int bits_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ inline int ffs64(unsigned long long m) { return __builtin_ctzll(m); }

__device__ inline uint32_t rdlane_u(uint32_t v, int l) { return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l)); }

__device__ inline double rdlane_d(double v, int l)
{
    unsigned long long b = __double_as_longlong(v);
    uint32_t lo = rdlane_u(static_cast<uint32_t>(b), l);
    uint32_t hi = rdlane_u(static_cast<uint32_t>(b >> 32), l);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b mod 8, each XCD with its own L2).  This hands the XCDs runs of kXcdRun
// consecutive logical blocks in turn, so neighbouring chunks of cells, whose
// stencils overlap, are read through the same L2 while every XCD still gets
// work from all over the box.  A bijection on [0, nb): the blocks past the
// last whole round of runs keep their index.
constexpr int kXcdRun = 16;
__device__ inline int xcd_block(int b, int nb)
{
    const int main = nb / (8 * kXcdRun) * (8 * kXcdRun);
    if (b >= main) return b;
    const int x = b & 7, i = b >> 3;
    return ((i / kXcdRun) * 8 + x) * kXcdRun + i % kXcdRun;
}

__device__ inline int wave_excl_scan(int v, int& total)
{
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane_id() >= d) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

// sum of v over lanes first .. first + n - 1 (n wave-uniform and small):
// scalar reads of the lanes instead of a cross-lane reduction tree
__device__ inline int lanes_sum(int v, int first, int n)
{
    int s = 0;
    for (int i = 0; i < n; ++i) s += __builtin_amdgcn_readlane(v, first + i);
    return s;
}

__device__ inline int wave_sum(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ inline Words draw(const Params& P, uint32_t cell, uint32_t t, uint32_t purpose, uint32_t index)
{
    return philox(P.sweep, cell, (t << 8) | purpose, index, P.key0, P.key1);
}

// 4-ball candidate: 25-bit fields, odd m in (-2^25, 2^25), accepted iff sum m^2 < 2^50
// depletant candidates of block `blk` of a trial's insertion stream: two ball
// candidates (V_0 = B(x', R0)) or one shell candidate (V_0 = the shell)
template <bool SHELL>
__device__ inline void depl_candidates_t(const Params& P, uint32_t cell, uint32_t t, uint32_t blk, bool& acc0,
                                         bool& acc1, Vec3& e0, Vec3& e1)
{
    if constexpr (SHELL) {
        Words dw = draw(P, cell, t, kDeplShell, blk);
        double x, y, z;
        acc0 = shell3(dw, P.r_inner, P.span, P.S.R0sq, x, y, z);
        acc1 = false;
        e0 = v3(x, y, z);
        e1 = e0;
    } else {
        Words dw = draw(P, cell, t, kDepl, blk);
        double a0, a1, a2, b0, b1, b2;
        acc0 = ball3(dw.w0, dw.w1, a0, a1, a2);
        acc1 = ball3(dw.w2, dw.w3, b0, b1, b2);
        e0 = v3(P.s_ball * a0, P.s_ball * a1, P.s_ball * a2);
        e1 = v3(P.s_ball * b0, P.s_ball * b1, P.s_ball * b2);
    }
}

__device__ inline void depl_candidates(const Params& P, uint32_t cell, uint32_t t, uint32_t blk, bool& acc0, bool& acc1,
                                       Vec3& e0, Vec3& e1)
{
    if (P.shell)
        depl_candidates_t<true>(P, cell, t, blk, acc0, acc1, e0, e1);
    else
        depl_candidates_t<false>(P, cell, t, blk, acc0, acc1, e0, e1);
}

__device__ inline bool ball4(Words w, double m[4])
{
    uint32_t ws[4] = {w.w0, w.w1, w.w2, w.w3};
#pragma unroll
    for (int a = 0; a < 4; ++a) m[a] = static_cast<double>(static_cast<int32_t>(2u * (ws[a] >> 7) + 1u) - (1 << 25));
    double s = ((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2]) + m[3] * m[3];
    return s < 0x1p50;
}

// per-wave working set of the phase kernel.  The cell's own records are
// updated in place in the cell-ordered arrays: during a phase only the wave
// that runs a cell reads or writes its members (neighbouring cells of the same
// colour are two cells apart), so no other wave sees them change.
struct WaveCtx {
    LAS int* list;      // stencil slots
    LAS double* geo;    // per-cell geometry cache: position (3) [+ R (9)] per entry
    LAS int* close;     // per trial: entries whose circumsphere meets the proposed pose's
    LAS int* reach;     // per trial: entries a depletant or CB trial point can overlap
    int start, nc, nst;
    int jslot;
    int jl;             // list index of the moved colloid (own members come first)
    int nr;             // entries in reach (all nst of them when rl is null)
    const LAS int* rl;  // reach, or null when the list overflowed its bound
    Vec3 xn;
};

__device__ inline int reach_entry(const WaveCtx& c, int k) { return c.rl ? c.rl[k] : k; }

template <int KIND>
struct Traits {
    static constexpr bool oriented = (KIND != kSphere);
    static constexpr int geo_stride = oriented ? 12 : 3;
};

// stencil entry i's reference point relative to the proposed position (the
// moved colloid's own entry reads as far away)
template <int KIND>
__device__ inline Vec3 get_offset(const Params& P, const WorkG& W, const WaveCtx& c, int i)
{
    double4 p;
    if (i == c.jl) return v3(kFar, kFar, kFar);
    if (i < P.geo_cap) {
        const LAS double* g = c.geo + static_cast<size_t>(i) * Traits<KIND>::geo_stride;
        p = make_double4(g[0], g[1], g[2], 0.0);
    } else {
        p = rd4(W.rpos, c.list[i]);
    }
    return v3(mi(P, p.x - c.xn.x), mi(P, p.y - c.xn.y), mi(P, p.z - c.xn.z));
}

// geometry of stencil entry i relative to the proposed position
template <int KIND>
__device__ inline void load_entry(const Params& P, const WorkG& W, const WaveCtx& c, int i, Vec3& D, Mat3& R)
{
    const int slot = c.list[i];
    const double4 p = rd4(W.rpos, slot);
    if (slot == c.jslot) {
        D = v3(kFar, kFar, kFar);
    } else {
        D = v3(mi(P, p.x - c.xn.x), mi(P, p.y - c.xn.y), mi(P, p.z - c.xn.z));
    }
    if constexpr (Traits<KIND>::oriented) {
        const double4 q = rd4(W.rquat, slot);
        R = quat_to_mat(q.x, q.y, q.z, q.w);
    }
}

template <int KIND>
__device__ inline void get_entry(const Params& P, const WorkG& W, const WaveCtx& c, int i, Vec3& D, Mat3& R)
{
    if (i < P.geo_cap) {
        const LAS double* g = c.geo + static_cast<size_t>(i) * Traits<KIND>::geo_stride;
        D = (i == c.jl) ? v3(kFar, kFar, kFar) : v3(mi(P, g[0] - c.xn.x), mi(P, g[1] - c.xn.y), mi(P, g[2] - c.xn.z));
        if constexpr (Traits<KIND>::oriented) {
#pragma unroll
            for (int k = 0; k < 9; ++k) R.m[k] = g[3 + k];
        }
    } else {
        load_entry<KIND>(P, W, c, i, D, R);
    }
}

// --- FP32 with an FP64 guard band for the oriented depletant predicates ----
struct Mat3f {
    float m[9];
};

__device__ inline Mat3f to_f32(const Mat3& R)
{
    Mat3f r;
#pragma unroll
    for (int k = 0; k < 9; ++k) r.m[k] = static_cast<float>(R.m[k]);
    return r;
}

// distance from the body-frame point p to the shape's core (hemisphere: the
// half ball, <= 0 inside it; swept disk: the bare disk), in FP32.  The
// depletant overlaps exactly when this distance is below r_dep (hemisphere)
// or r_s + r_dep (swept disk); the branch formulas agree on the branch
// boundaries, so an FP32 branch choice off by rounding changes the value only
// by about the rounding.
template <int KIND>
__device__ inline float core_dist32(const Shape& S, float px, float py, float pz)
{
    const float a = static_cast<float>(S.a);
    const float rho2 = px * px + py * py;
    if constexpr (KIND == kHemisphere) {
        if (pz >= 0.0f) return sqrtf(rho2 + pz * pz) - a;
        if (rho2 <= a * a) return -pz;
    } else {
        if (rho2 <= a * a) return fabsf(pz);
    }
    const float t = sqrtf(rho2) - a;
    return sqrtf(t * t + pz * pz);
}

// Depletant at world offset v from a colloid with rotation R: FP64 (the
// contract) or FP32 decided outside a band of 1e-5 sigma around the threshold
// (the FP32 error of the distance is below 1e-6 for |v| < 4), FP64 inside it
// (counted in fb).
template <int KIND, bool F32>
__device__ inline bool dep_ov_g(const Params& P, Vec3 v, const Mat3& R, const Mat3f& Rf, unsigned& fb,
                                bool counted = true)
{
    if constexpr (!F32) {
        return dep_ov<KIND>(P.S, v, R);
    } else {
        const float vx = static_cast<float>(v.x), vy = static_cast<float>(v.y), vz = static_cast<float>(v.z);
        const float px = (Rf.m[0] * vx + Rf.m[3] * vy) + Rf.m[6] * vz;
        const float py = (Rf.m[1] * vx + Rf.m[4] * vy) + Rf.m[7] * vz;
        const float pz = (Rf.m[2] * vx + Rf.m[5] * vy) + Rf.m[8] * vz;
        const float d = core_dist32<KIND>(P.S, px, py, pz);
        if (d < P.g_lo) return true;
        if (d > P.g_hi) return false;
        if (counted) ++fb;
        return dep_ov<KIND>(P.S, v, R);
    }
}

// wave-cooperative: does a depletant at offset e overlap any stencil colloid
// (those in reach: no other can)?
template <int KIND, bool F32 = false>
__device__ inline bool stencil_hit_coop(const Params& P, const WorkG& W, const WaveCtx& c, Vec3 e, unsigned& fb)
{
    bool hit = false;
    for (int k = lane_id(); k < c.nr; k += 64) {
        Vec3 D;
        Mat3 R;
        get_entry<KIND>(P, W, c, reach_entry(c, k), D, R);
        Mat3f Rf{};
        if constexpr (F32) Rf = to_f32(R);
        hit = hit || dep_ov_g<KIND, F32>(P, e - D, R, Rf, fb);
    }
    return __ballot(hit) != 0ull;
}

// per-lane: does the point p overlap any stencil colloid in reach?  (all lanes
// read the same entry at the same time: LDS broadcast)
template <int KIND>
__device__ inline bool stencil_hit_lane(const Params& P, const WorkG& W, const WaveCtx& c, Vec3 p, bool active)
{
    bool hit = !active;
    for (int k = 0; k < c.nr; ++k) {
        if (__ballot(!hit) == 0ull) break;
        Vec3 D;
        Mat3 R;
        get_entry<KIND>(P, W, c, reach_entry(c, k), D, R);
        if (!hit) hit = dep_ov<KIND>(P.S, p - D, R);
    }
    return hit && active;
}

// CB trial insertions of blocking depletant ks (Sec. III.D): forward trial i is
// the i-th accepted ball candidate of the CB_FWD stream of ks (uniform in
// B(x, R0)), reverse trial i the i-th of the CB_REV stream (uniform in
// B(x', R0)).  Lanes 0-31 draw forward blocks, lanes 32-63 reverse blocks; a
// ballot rank inside each half assigns the trial index, so one Philox pass
// usually yields every trial.  Returns the valid counts W'_k and W_k.
template <int KIND>
__device__ inline void cb_weights(const Params& P, const WorkG& W, const WaveCtx& c, uint32_t C, uint32_t t,
                                  uint32_t ks, Vec3 Dold, const Mat3& Rn, const Mat3& Ro, uint32_t& Wf, uint32_t& Wr)
{
    const int lane = lane_id();
    const bool fwd = lane < 32;
    const unsigned long long lo_half = 0x00000000FFFFFFFFull;
    const unsigned long long half = fwd ? lo_half : ~lo_half;
    const int need_f = P.n_trial, need_r = P.n_trial - 1;
    int have_f = 0, have_r = 0;
    Wf = 0;
    Wr = 0;
    for (uint32_t blk = 0; (have_f < need_f || have_r < need_r) && blk < 65536u; blk += 32) {
        const int have = fwd ? have_f : have_r;
        const int need = fwd ? need_f : need_r;
        Words w = draw(P, C, t, fwd ? kCbFwd : kCbRev, (ks << 16) | (blk + static_cast<uint32_t>(lane & 31)));
        double a0, a1, a2, b0, b1, b2;
        bool c0 = ball3(w.w0, w.w1, a0, a1, a2) && have < need;
        bool c1 = ball3(w.w2, w.w3, b0, b1, b2) && have < need;
        const unsigned long long M0 = __ballot(c0), M1 = __ballot(c1);
        int r0 = have + bits_below(M0 & half) + bits_below(M1 & half);
        int r1 = r0 + (c0 ? 1 : 0);
        bool v0 = c0 && r0 < need, v1 = c1 && r1 < need;
        Vec3 f0 = v3(P.s_ball * a0, P.s_ball * a1, P.s_ball * a2);
        Vec3 f1 = v3(P.s_ball * b0, P.s_ball * b1, P.s_ball * b2);
        // forward: overlaps the old pose (implied for spheres), misses the new pose;
        // reverse: overlaps the new pose (implied for spheres), misses the old pose
        Vec3 p0 = fwd ? (Dold + f0) : f0, p1 = fwd ? (Dold + f1) : f1;
        if (v0) {
            if constexpr (Traits<KIND>::oriented) v0 = dep_ov<KIND>(P.S, f0, fwd ? Ro : Rn);
            if (v0) v0 = fwd ? !dep_ov<KIND>(P.S, p0, Rn) : !dep_ov<KIND>(P.S, f0 - Dold, Ro);
        }
        if (v1) {
            if constexpr (Traits<KIND>::oriented) v1 = dep_ov<KIND>(P.S, f1, fwd ? Ro : Rn);
            if (v1) v1 = fwd ? !dep_ov<KIND>(P.S, p1, Rn) : !dep_ov<KIND>(P.S, f1 - Dold, Ro);
        }
        // and miss every other colloid of the stencil
        v0 = v0 && !stencil_hit_lane<KIND>(P, W, c, p0, v0);
        v1 = v1 && !stencil_hit_lane<KIND>(P, W, c, p1, v1);
        const unsigned long long V0 = __ballot(v0), V1 = __ballot(v1);
        Wf += static_cast<uint32_t>(__popcll(V0 & lo_half) + __popcll(V1 & lo_half));
        Wr += static_cast<uint32_t>(__popcll(V0 & ~lo_half) + __popcll(V1 & ~lo_half));
        have_f += __popcll(M0 & lo_half) + __popcll(M1 & lo_half);
        have_r += __popcll(M0 & ~lo_half) + __popcll(M1 & ~lo_half);
    }
}

template <typename FP, typename GP>
__device__ inline int poisson_guided(FP F, GP G, double u, const Params& P)
{
    return poisson_compact_draw(F, G, u, P.pk_min, P.pk_n);
}

struct TrialOut {
    uint32_t n_dep, resolved, nblk, wf, wr, cbt;
    int reason;
    bool near;
};

}  // namespace

// Every kernel serves a group of independent replicas: blockIdx.y selects the
// replica's descriptor (its constants and workspace); one handle is a group of one.
#define HPMC_REPLICA(D)                     \
    const Params P = (D)[blockIdx.y].P;     \
    const Work W = (D)[blockIdx.y].W

// ---------------------------------------------------------------------------
// grid, cells
// ---------------------------------------------------------------------------
__device__ inline void grid_setup(const Params& P, const Work& W);

__global__ void grid_kernel(const Desc* __restrict__ D, int with_grid)
{
    Params P = D[blockIdx.y].P;
    const Work W = D[blockIdx.y].W;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    P.sweep = *W.sweep_dev;
    if (!with_grid) {
        for (int a = 0; a < 3; ++a) W.grid[a] = 0.0;
        for (int i = 0; i < 8; ++i) W.perm[i] = i;
        return;
    }
    grid_setup(P, W);
}

__global__ void clear_counters_kernel(const Desc* __restrict__ D)
{
    const Work W = D[blockIdx.y].W;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kCounterCopies * kCounterStride) W.counters[i] = 0ull;
}

__global__ void clear_cells_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.ncells) W.cell_count[i] = 0;
}

// counters (13 per replica, after the reduction) and flags gathered for one copy
__global__ void gather_counters_kernel(const Desc* __restrict__ D, int nrep, unsigned long long* out)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    const Work W = D[r].W;
    for (int k = 0; k < kNumCounters; ++k) out[static_cast<size_t>(r) * kCounterStride + k] = W.counters[k];
    out[static_cast<size_t>(r) * kCounterStride + kNumCounters] = static_cast<unsigned long long>(W.flags[0]);
}

__global__ void fill_int_kernel(int* p, int n, int value)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ void fill_u64_kernel(unsigned long long* p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void bin_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    const double* __restrict__ pos = W.pos;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.N) return;
    int c = cell_of(P, pos[i], pos[P.N + i], pos[2 * P.N + i], W.grid[0], W.grid[1], W.grid[2]);
    W.pcell[i] = c;
    W.prank[i] = atomicAdd(&W.cell_count[c], 1);
}

// exclusive scan, 1024 elements per block of 256 threads
__global__ __launch_bounds__(256) void scan_local_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    const int* __restrict__ in = W.cell_count;
    int* __restrict__ out = W.cell_start;
    int* __restrict__ totals = W.scan_tmp;
    const int n = P.ncells;
    if (static_cast<int>(blockIdx.x) * 1024 >= n) return;
    __shared__ int wsum[4];
    int base = blockIdx.x * 1024 + threadIdx.x * 4;
    int v[4];
    int s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int ex = wave_excl_scan(s, tot);
    int wv = threadIdx.x >> 6;
    if (lane_id() == 0) wsum[wv] = tot;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < wv; ++k) woff += wsum[k];
    int run = woff + ex;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) totals[blockIdx.x] = woff + ex + s;
}

__global__ __launch_bounds__(256) void scan_top_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    int* totals = W.scan_tmp;
    const int nblocks = (P.ncells + 1023) / 1024;
    (void)P;
    __shared__ int wsum[4];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblocks; base += 256) {
        int i = base + threadIdx.x;
        int v = (i < nblocks) ? totals[i] : 0;
        int tot;
        int ex = wave_excl_scan(v, tot);
        int wv = threadIdx.x >> 6;
        if (lane_id() == 0) wsum[wv] = tot;
        __syncthreads();
        int woff = 0, all = 0;
        for (int k = 0; k < 4; ++k) {
            if (k < wv) woff += wsum[k];
            all += wsum[k];
        }
        if (i < nblocks) totals[i] = carry + woff + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += all;
        __syncthreads();
    }
}

__global__ void scan_add_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    int* out = W.cell_start;
    const int* totals = W.scan_tmp;
    const int n = P.ncells, total_all = P.N;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += totals[i / 1024];
    if (i == 0) out[n] = total_all;
}

__global__ void scatter_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.N) return;
    W.order[W.cell_start[W.pcell[i]] + W.prank[i]] = i;
}

// Members of each cell in ascending particle index, the order trials select
// from.  The scatter placed them in the order of their atomic ranks; each
// particle's rank among its cell's members is the number of smaller indices
// there, and a second scatter by these ranks sorts every cell at once (one
// thread per particle, no serial pass over a cell).
__global__ void rank_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.N) return;
    const int c = W.pcell[i];
    const int s = W.cell_start[c], e = W.cell_start[c + 1];
    int r = 0;
    for (int k = s; k < e; ++k) r += W.order[k] < i ? 1 : 0;
    W.prank[i] = r;
}

__global__ void gather_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    const double* __restrict__ pos = W.pos;
    const double* __restrict__ quat = W.quat;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.N) return;
    int i = W.order[s];
    wr4(W.rpos, s, make_double4(pos[i], pos[P.N + i], pos[2 * P.N + i], static_cast<double>(i)));
    if (P.S.oriented)
        wr4(W.rquat, s, make_double4(quat[i], quat[P.N + i], quat[2 * P.N + i], quat[3 * P.N + i]));
}

// cell-ordered records back to the SoA state; the sweep counter advances here
__global__ void scatter_back_kernel(const Desc* __restrict__ D, int advance)
{
    HPMC_REPLICA(D);
    double* __restrict__ pos = W.pos;
    double* __restrict__ quat = W.quat;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (advance && s == 0) *W.sweep_dev = *W.sweep_dev + 1u;
    if (s >= P.N) return;
    double4 r = rd4(W.rpos, s);
    int i = static_cast<int>(r.w);
    pos[i] = r.x;
    pos[P.N + i] = r.y;
    pos[2 * P.N + i] = r.z;
    if (P.S.oriented) {
        double4 q = rd4(W.rquat, s);
        quat[i] = q.x;
        quat[P.N + i] = q.y;
        quat[2 * P.N + i] = q.z;
        quat[3 * P.N + i] = q.w;
    }
}

// ---------------------------------------------------------------------------
// one colour of the checkerboard: every active cell runs its trials
// ---------------------------------------------------------------------------
template <int KIND, bool F32>
__device__ __forceinline__ void phase_body(const Params& P, const WorkG& W, int phase, int lb, int nblk)
{
    unsigned fb = 0;  // FP64 fallbacks of the guarded FP32 depletant tests (this lane)
    LAS unsigned char* smem = lds_base();
    LAS double* sF = (LAS double*)smem;
    LAS int* sG = (LAS int*)(smem + kPoissonC * sizeof(double));
    const GAS int* gG = (const GAS int*)(W.F + kPoissonC);
    for (int i = threadIdx.x; i < kPoissonC; i += blockDim.x) sF[i] = W.F[i];
    for (int i = threadIdx.x; i < kGuide; i += blockDim.x) sG[i] = gG[i];
    __syncthreads();

    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));  // wave-uniform
    LAS unsigned char* wbase = smem + kTableLds + static_cast<size_t>(wv) * P.wave_lds;
    WaveCtx c;
    c.list = (LAS int*)wbase;
    c.geo = (LAS double*)(wbase + P.off_geo);
    c.close = (LAS int*)(wbase + P.off_close);
    c.reach = (LAS int*)(wbase + P.off_reach);
    constexpr int GS = Traits<KIND>::geo_stride;
    constexpr bool ORI = Traits<KIND>::oriented;
    static_assert(ORI, "spheres run phase_sphere_body");

    unsigned long long cnt[kNumCounters];
#pragma unroll
    for (int k = 0; k < kNumCounters; ++k) cnt[k] = 0ull;

    const int colour = W.perm[phase];
    const int gw = lb * P.waves_per_block + wv;
    const int nwaves = nblk * P.waves_per_block;
    const double g0 = W.grid[0], g1 = W.grid[1], g2 = W.grid[2];
    const NbOff nb = nb_offset(P.n);

    for (int a = gw; a < P.active_cells; a += nwaves) {
        const int ax = a % P.h, ay = (a / P.h) % P.h, az = a / (P.h * P.h);
        const int cx = 2 * ax + (colour & 1), cy = 2 * ay + ((colour >> 1) & 1), cz = 2 * az + ((colour >> 2) & 1);
        const int C = cx + P.n * (cy + P.n * cz);
        c.start = W.cell_start[C];
        c.nc = W.cell_start[C + 1] - c.start;
        if (c.nc == 0) continue;
        // stencil: the de-duplicated 27 (n > 2) or 8 (n = 2) cells around C
        int es = 0, ec = 0;
        if (nb.on) {
            int ex = wrap1(cx + nb.dx, P.n), ey = wrap1(cy + nb.dy, P.n), ez = wrap1(cz + nb.dz, P.n);
            int e = ex + P.n * (ey + P.n * ez);
            es = W.cell_start[e];
            ec = W.cell_start[e + 1] - es;
        }
        int nst;
        int off = wave_excl_scan(ec, nst);
        if (nst > P.list_cap) {
            if (lane == 0) __hip_atomic_fetch_or(W.flags, kFlagListOverflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        for (int k = 0; k < ec; ++k) c.list[off + k] = es + k;
        c.nst = nst;
        wave_sync();
        // geometry cache of the stencil, once per cell: positions and rotation
        // matrices (the moved colloid's entry is updated when a move is accepted)
        {
            const int ng = c.nst < P.geo_cap ? c.nst : P.geo_cap;
            for (int i = lane; i < ng; i += 64) {
                const int slot = c.list[i];
                const double4 pp = rd4(W.rpos, slot);
                LAS double* g = c.geo + static_cast<size_t>(i) * GS;
                g[0] = pp.x;
                g[1] = pp.y;
                g[2] = pp.z;
                if constexpr (ORI) {
                    const double4 qq = rd4(W.rquat, slot);
                    Mat3 R = quat_to_mat(qq.x, qq.y, qq.z, qq.w);
#pragma unroll
                    for (int k = 0; k < 9; ++k) g[3 + k] = R.m[k];
                }
            }
            wave_sync();
        }

        // A trial's own draws (selection, translation, acceptance and its
        // Poisson chunks: B Philox blocks) depend on the random streams alone,
        // not on the state, so those of T = 64 / B consecutive trials of the
        // cell are drawn at once, one block per lane (the Poisson chunks
        // resolved there), and read across lanes when each trial runs.
        // Rotation candidates are drawn by the trials that rotate.
        const int ntr = P.n_select * c.nc;
        const int B = 3 + P.n_chunks < 64 ? 3 + P.n_chunks : 64;
        const int T = 64 / B;
        int tb = -64;  // first trial of the batch in the lanes (none yet)
        Words wb{0u, 0u, 0u, 0u};
        int kcb = 0;
        for (int t = 0; t < ntr; ++t) {
            if (t >= tb + T) {
                tb = t;
                const int tl = lane / B, q = lane - tl * B;
                const bool valid = tl < T && tb + tl < ntr;
                const uint32_t purpose = q == 0 ? kSelect : (q == 1 ? kTrans : (q == 2 ? kAccept : kPoisson));
                const uint32_t index = q >= 3 ? static_cast<uint32_t>(q - 3) : 0u;
                wb = draw(P, static_cast<uint32_t>(C), static_cast<uint32_t>(tb + tl), purpose, index);
                kcb = 0;
                if (valid && P.has_dep && q >= 3 && q - 3 < P.n_chunks) kcb = poisson_guided(sF, sG, u52(wb.w0, wb.w1), P);
            }
            const int base = (t - tb) * B;
            const uint32_t sel0 = rdlane_u(wb.w0, base), sel1 = rdlane_u(wb.w1, base);
            const int jl = static_cast<int>(pick(sel0, static_cast<uint32_t>(c.nc)));
            const bool rotate = ORI && P.p_rot > 0.0 && u01(sel1) < P.p_rot;
            c.jslot = c.start + jl;
            c.jl = jl;
            const double4 pj = rd4(W.rpos, c.jslot);
            double4 qj = make_double4(1.0, 0.0, 0.0, 0.0);
            if constexpr (ORI) qj = rd4(W.rquat, c.jslot);
            Vec3 xn = v3(pj.x, pj.y, pj.z);
            double qn[4] = {qj.x, qj.y, qj.z, qj.w};
            if (!rotate) {
                double xs[3] = {pj.x, pj.y, pj.z};
                uint32_t tw[3] = {rdlane_u(wb.w0, base + 1), rdlane_u(wb.w1, base + 1), rdlane_u(wb.w2, base + 1)};
                double xo[3];
#pragma unroll
                for (int ax3 = 0; ax3 < 3; ++ax3) {
                    double v = xs[ax3] + P.d_trans * sym01(tw[ax3]);
                    if (v >= P.L)
                        v -= P.L;
                    else if (v < 0.0)
                        v += P.L;
                    xo[ax3] = v;
                }
                xn = v3(xo[0], xo[1], xo[2]);
            } else {
                // the first accepted 4-ball candidate of the trial's ROT stream
                // (indices 0 .. 255, 64 per pass, in index order)
                double m[4];
                int src = -1;
                uint32_t vw[4] = {0, 0, 0, 0};
                for (uint32_t rb = 0; rb < 256u && src < 0; rb += 64) {
                    Words r = draw(P, static_cast<uint32_t>(C), static_cast<uint32_t>(t), kRot, rb + lane);
                    unsigned long long om = __ballot(ball4(r, m));
                    if (om) {
                        src = ffs64(om);
                        vw[0] = rdlane_u(r.w0, src);
                        vw[1] = rdlane_u(r.w1, src);
                        vw[2] = rdlane_u(r.w2, src);
                        vw[3] = rdlane_u(r.w3, src);
                    }
                }
                if (src >= 0) {
                    Words vv{vw[0], vw[1], vw[2], vw[3]};
                    ball4(vv, m);
                    double qq[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) qq[k] = qn[k] + P.a_rot * (m[k] * 0x1p-25);
                    double nrm = sqrt(((qq[0] * qq[0] + qq[1] * qq[1]) + qq[2] * qq[2]) + qq[3] * qq[3]);
#pragma unroll
                    for (int k = 0; k < 4; ++k) qn[k] = qq[k] / nrm;
                }
            }
            c.xn = xn;

            TrialOut o{0, 0, 0, 0, 0, 0, 0, false};
            // --- cell exit (particles may not leave their cell, Sec. III.E) ----
            if (cell_of(P, xn.x, xn.y, xn.z, g0, g1, g2) != C) {
                o.reason = 1;
            } else {
                // A stencil of more than one entry per lane: one pass over it builds
                // the close list (circumspheres of the proposed pose and the entry
                // meet, so the pair needs the narrow phase) and the reach list (a
                // depletant of V_0 or a CB trial point can overlap the entry), both
                // in ascending entry order, so that the narrow phase and the
                // depletant tests take one round instead of one per 64 entries.
                // A smaller stencil is taken whole: it is one round either way.
                int ncl = 0, nrc = 0;
                const int nlist = c.nst > 64 ? c.nst : 0;
                for (int i0 = 0; i0 < nlist; i0 += 64) {
                    const int i = i0 + lane;
                    bool cl = false, rc = false;
                    if (i < c.nst) {
                        const Vec3 D = get_offset<KIND>(P, W, c, i);
                        const double dd = dot(D, D);
                        cl = dd < P.S.lim_sq;
                        rc = dd < P.reach_sq;
                    }
                    const unsigned long long mc = __ballot(cl), mr = __ballot(rc);
                    const int kc = ncl + bits_below(mc), kr = nrc + bits_below(mr);
                    if (cl && kc < P.close_cap) c.close[kc] = i;
                    if (rc && kr < P.reach_cap) c.reach[kr] = i;
                    ncl += __popcll(mc);
                    nrc += __popcll(mr);
                }
                if (nlist) wave_sync();
                // a list beyond its packing bound (impossible for disjoint bodies) falls back to every entry
                const LAS int* cl_list = (nlist && ncl <= P.close_cap) ? c.close : nullptr;
                const int n_close = cl_list ? ncl : c.nst;
                c.rl = (nlist && nrc <= P.reach_cap) ? c.reach : nullptr;
                c.nr = c.rl ? nrc : c.nst;
                Mat3 Rn, Ro;
                if constexpr (ORI) {
                    Rn = quat_to_mat(qn[0], qn[1], qn[2], qn[3]);
                    Ro = quat_to_mat(qj.x, qj.y, qj.z, qj.w);
                }
                Mat3f Rn32{}, Ro32{};
                if constexpr (F32) {
                    Rn32 = to_f32(Rn);
                    Ro32 = to_f32(Ro);
                }
                // --- hard colloid overlap: min(1, exp(-beta dH_cc)) ---------------
                bool hit = false, nearc = false;
                int checks = 0;
                for (int k = lane; k < n_close; k += 64) {
                    Vec3 D;
                    Mat3 R;
                    get_entry<KIND>(P, W, c, cl_list ? cl_list[k] : k, D, R);
                    PairResult pr = pair_ov<KIND>(P.S, D, Rn, R);
                    hit = hit || pr.overlap;
                    nearc = nearc || pr.near;
                    checks++;
                }
                o.near = __ballot(nearc) != 0ull;
                cnt[cOverlapChecks] += static_cast<unsigned long long>(wave_sum(checks));
                if (__ballot(hit) != 0ull) {
                    o.reason = 2;
                } else if (P.has_dep) {
                    // --- Poisson number of depletants in V_0 ------------------------
                    // chunk counts sit in lanes base + 3 .. base + 2 + n_chunks; chunks past
                    // lane 63 (more than 61 of them: then one trial per batch) are drawn here
                    int kx = (lane >= base + 3 && lane < base + 3 + P.n_chunks) ? kcb : 0;
                    for (int cbase = 61; cbase < P.n_chunks; cbase += 64) {
                        int ci = cbase + lane;
                        if (ci < P.n_chunks) {
                            Words pw = draw(P, static_cast<uint32_t>(C), static_cast<uint32_t>(t), kPoisson,
                                            static_cast<uint32_t>(ci));
                            kx += poisson_guided(sF, sG, u52(pw.w0, pw.w1), P);
                        }
                    }
                    const uint32_t Np =
                        static_cast<uint32_t>(P.n_chunks <= 8 ? lanes_sum(kcb, base + 3, P.n_chunks) : wave_sum(kx));
                    o.n_dep = Np;
                    const double au = u52(rdlane_u(wb.w0, base + 2), rdlane_u(wb.w1, base + 2));
                    const Vec3 Dold = v3(mi(P, pj.x - xn.x), mi(P, pj.y - xn.y), mi(P, pj.z - xn.z));
                    const Vec3 zero3 = v3(0.0, 0.0, 0.0);
                    double ratio = 1.0;
                    bool done = false;
                    uint32_t kbase = 0, blk = 0;
                    while (!done && kbase < Np && blk < (1u << 30)) {
                        bool acc0, acc1;
                        Vec3 e0, e1;
                        depl_candidates(P, static_cast<uint32_t>(C), static_cast<uint32_t>(t), blk + lane, acc0, acc1,
                                        e0, e1);
                        unsigned long long m0 = __ballot(acc0), m1 = __ballot(acc1);
                        uint32_t k0 = kbase + static_cast<uint32_t>(bits_below(m0) + bits_below(m1));
                        uint32_t k1 = k0 + (acc0 ? 1u : 0u);
                        bool v0 = acc0 && k0 < Np, v1 = acc1 && k1 < Np;
                        // irrelevant (misses M') or ignored by the old pose
                        {
                            // evaluated in every lane (no branch); a fallback is counted only
                            // where the test decides: valid candidate, and for the old pose
                            // one that overlaps the new pose
                            const bool n0 = dep_ov_g<KIND, F32>(P, e0, Rn, Rn32, fb, v0);
                            const bool n1 = dep_ov_g<KIND, F32>(P, e1, Rn, Rn32, fb, v1);
                            const bool o0 = dep_ov_g<KIND, F32>(P, e0 - Dold, Ro, Ro32, fb, v0 && n0);
                            const bool o1 = dep_ov_g<KIND, F32>(P, e1 - Dold, Ro, Ro32, fb, v1 && n1);
                            v0 = v0 && n0 && !o0;
                            v1 = v1 && n1 && !o1;
                        }
                        unsigned long long r0 = __ballot(v0), r1 = __ballot(v1);
                        // survivors in ascending depletant index: lane order, candidate 0 before 1
                        while ((r0 | r1) && !done) {
                            int l0 = r0 ? ffs64(r0) : 64, l1 = r1 ? ffs64(r1) : 64;
                            int src, cand;
                            if (l0 <= l1) {
                                src = l0;
                                cand = 0;
                                r0 &= ~(1ull << l0);
                            } else {
                                src = l1;
                                cand = 1;
                                r1 &= ~(1ull << l1);
                            }
                            src = __builtin_amdgcn_readfirstlane(src);
                            Vec3 es = cand ? e1 : e0;
                            es = v3(rdlane_d(es.x, src), rdlane_d(es.y, src), rdlane_d(es.z, src));
                            uint32_t ks = rdlane_u(cand ? k1 : k0, src);
                            if (stencil_hit_coop<KIND, F32>(P, W, c, es, fb)) continue;  // ignored
                            // blocking: free in M, overlapping M'
                            o.nblk++;
                            if (P.n_trial == 0) {
                                o.reason = 3;
                                o.resolved = ks + 1;
                                done = true;
                                break;
                            }
                            // configurational bias: n_trial forward + (n_trial - 1) reverse insertions
                            const int ntot = 2 * P.n_trial - 1;
                            uint32_t Wf, Wr;
                            cb_weights<KIND>(P, W, c, static_cast<uint32_t>(C), static_cast<uint32_t>(t), ks, Dold, Rn,
                                             Ro, Wf, Wr);
                            o.wf += Wf;
                            if (Wf == 0) {
                                o.reason = 4;
                                o.resolved = ks + 1 + o.cbt + static_cast<uint32_t>(P.n_trial);
                                o.cbt += static_cast<uint32_t>(P.n_trial);
                                done = true;
                                break;
                            }
                            o.wr += Wr;
                            ratio = ratio * (static_cast<double>(Wf) / static_cast<double>(1 + Wr));
                            o.cbt += static_cast<uint32_t>(ntot);
                        }
                        kbase += static_cast<uint32_t>(__popcll(m0) + __popcll(m1));
                        blk += 64;
                    }
                    (void)zero3;
                    if (!done) {
                        o.resolved = Np + o.cbt;
                        if (o.nblk > 0 && !(au < ratio)) o.reason = 5;
                    }
                }
            }
            // --- accept / commit / record ---------------------------------------
            if (o.reason == 0 && lane == 0) {
                wr4(W.rpos, c.jslot, make_double4(xn.x, xn.y, xn.z, pj.w));
                if constexpr (ORI) wr4(W.rquat, c.jslot, make_double4(qn[0], qn[1], qn[2], qn[3]));
                if (jl < P.geo_cap) {
                    LAS double* g = c.geo + static_cast<size_t>(jl) * GS;
                    g[0] = xn.x;
                    g[1] = xn.y;
                    g[2] = xn.z;
                    if constexpr (ORI) {
                        Mat3 R = quat_to_mat(qn[0], qn[1], qn[2], qn[3]);
#pragma unroll
                        for (int k = 0; k < 9; ++k) g[3 + k] = R.m[k];
                    }
                }
            }
            wave_sync();
            cnt[cTrials] += 1;
            // one compare per reason, no branch and no indexed select over the counters
            cnt[cAccepts] += o.reason == 0 ? 1ull : 0ull;
            cnt[cRejCellExit] += o.reason == 1 ? 1ull : 0ull;
            cnt[cRejOverlap] += o.reason == 2 ? 1ull : 0ull;
            cnt[cRejDepletant] += o.reason == 3 ? 1ull : 0ull;
            cnt[cRejCbZero] += o.reason == 4 ? 1ull : 0ull;
            cnt[cRejCbMetro] += o.reason == 5 ? 1ull : 0ull;
            cnt[cDrawn] += o.n_dep;
            cnt[cResolved] += o.resolved;
            cnt[cCbTrials] += o.cbt;
            cnt[cNearContact] += o.near ? 1 : 0;
            if (P.trace && lane == 0) {
                GAS uint32_t* r = (GAS uint32_t*)(W.trace + (static_cast<size_t>(P.n_select) * c.start + t) * 40);
                r[0] = P.sweep;
                r[1] = static_cast<uint32_t>(C);
                r[2] = static_cast<uint32_t>(t);
                r[3] = static_cast<uint32_t>(pj.w);
                r[4] = o.n_dep;
                r[5] = o.resolved;
                r[6] = o.nblk;
                r[7] = o.wf;
                r[8] = o.wr;
                r[9] = static_cast<uint32_t>(phase) | (static_cast<uint32_t>(o.reason) << 8) |
                       (static_cast<uint32_t>(rotate ? 1 : 0) << 16) | (static_cast<uint32_t>(o.near ? 1 : 0) << 24);
            }
        }
    }
    cnt[cFp64Fallbacks] += static_cast<unsigned long long>(wave_sum(static_cast<int>(fb)));
    if (lane == 0) {
        GAS unsigned long long* dst = W.counters + static_cast<size_t>(gw % kCounterCopies) * kCounterStride;
#pragma unroll
        for (int k = 0; k < kNumCounters; ++k)
            if (cnt[k]) __hip_atomic_fetch_add(dst + k, cnt[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Spheres: one wave per chunk of P.chunk active cells.  The stencil records of
// a cell (its own members first, then the 26 neighbour cells) are staged in
// LDS by direct global->LDS loads issued while the previous non-empty cell of
// the chunk runs its trials; neighbour ranges two cells ahead are loaded into
// registers at the same time.  Trials then read only LDS and registers.
// ---------------------------------------------------------------------------
constexpr int kStage = 64;  // staged stencil entries per cell (more are read from HBM)

// Is the point at offset a - b within R0 of the centre?  FP64 (the contract)
// or, in the guarded mode, FP32 with a band of 1e-5 sigma around R0: outside
// the band the FP32 decision equals the FP64 one (its rounding error is below
// 1e-6 where |a - b| is near R0, the band is 1.1e-5 wide in |a - b|^2), inside it
// the FP64 test decides and the fallback is counted.
template <bool F32>
__device__ inline bool sphere_in(const Params& P, Vec3 a, Vec3 b, bool active, unsigned& fallbacks)
{
    if constexpr (!F32) return dot(a - b, a - b) < P.S.R0sq;
    float vx = static_cast<float>(a.x) - static_cast<float>(b.x);
    float vy = static_cast<float>(a.y) - static_cast<float>(b.y);
    float vz = static_cast<float>(a.z) - static_cast<float>(b.z);
    float q = (vx * vx + vy * vy) + vz * vz;
    bool in = q < P.g_lo;
    bool amb = active && !in && !(q > P.g_hi);
    if (__ballot(amb)) {
        if (amb) {
            ++fallbacks;  // this lane's count: callers may run with some lanes off
            in = dot(a - b, a - b) < P.S.R0sq;
        }
    }
    return in;
}

struct SphereStage {
    LAS int* list;     // stencil slots (list_cap)
    LAS double* recA;  // entry i: (x, y) at [2i, 2i + 1]
    LAS double* recB;  // entry i: (z, particle index) at [2i, 2i + 1]
};

__device__ inline double4 stage_rec(const SphereStage& sb, int i)
{
    return make_double4(sb.recA[2 * i], sb.recA[2 * i + 1], sb.recB[2 * i], sb.recB[2 * i + 1]);
}

// neighbour-cell ranges of cell C at (cx, cy, cz): a lane with nb.on holds
// the range of its neighbour (lane 0: C itself)
__device__ inline void stencil_ranges(const Params& P, const WorkG& W, const NbOff& nb, int C, int cx, int cy, int cz,
                                      int& es, int& ec)
{
    es = 0;
    ec = 0;
    if (C >= 0 && nb.on) {
        int e = wrap1(cx + nb.dx, P.n) + P.n * (wrap1(cy + nb.dy, P.n) + P.n * wrap1(cz + nb.dz, P.n));
        es = W.cell_start[e];
        ec = W.cell_start[e + 1] - es;
    }
}

// write the stencil list of a cell and start the direct loads of its first
// kStage records into LDS; returns the stencil size (or -1 on overflow)
__device__ inline int stage_issue(const Params& P, const WorkG& W, const SphereStage& sb, int es, int ec)
{
    const int lane = lane_id();
    int nst;
    int off = wave_excl_scan(ec, nst);
    if (nst > P.list_cap) return -1;
    for (int k = 0; k < ec; ++k) sb.list[off + k] = es + k;
    wave_sync();
    if (lane < nst && lane < kStage) {
        const GAS char* g = (const GAS char*)(W.rpos + sb.list[lane]);
        __builtin_amdgcn_global_load_lds((const GAS void*)g, (LAS void*)sb.recA, 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const GAS void*)(g + 16), (LAS void*)sb.recB, 16, 0, 0);
    }
    return nst;
}

// does a point at offset p (from x') overlap any stencil colloid?  per lane.
// The staged entries (lane i of Dreg holds entry i's offset) are taken from
// rmask, the entries in reach of the CB regions, read across lanes; entries
// beyond the stage from the records.
__device__ inline bool sphere_hit_lane(const Params& P, const WorkG& W, const SphereStage& sb, int nst, int jent,
                                       Vec3 xn, unsigned long long rmask, Vec3 Dreg, Vec3 p, bool active)
{
    bool hit = !active;
    for (unsigned long long m = rmask; m; m &= m - 1ull) {
        const int i = ffs64(m);
        const Vec3 D = v3(rdlane_d(Dreg.x, i), rdlane_d(Dreg.y, i), rdlane_d(Dreg.z, i));
        hit = hit || dot(p - D, p - D) < P.S.R0sq;
    }
    for (int i = kStage; i < nst; ++i) {
        if (__ballot(!hit) == 0ull) break;
        if (i == jent) continue;
        double4 r = rd4(W.rpos, sb.list[i]);
        Vec3 D = v3(mi(P, r.x - xn.x), mi(P, r.y - xn.y), mi(P, r.z - xn.z));
        if (!hit) hit = dot(p - D, p - D) < P.S.R0sq;
    }
    return hit && active;
}

// Poisson table and its guide into the workgroup's LDS (before any phase body)
__device__ inline void load_table(const WorkG& W, LAS unsigned char* smem)
{
    LAS double* sF = (LAS double*)smem;
    LAS int* sG = (LAS int*)(smem + kPoissonC * sizeof(double));
    const GAS int* gG = (const GAS int*)(W.F + kPoissonC);
    for (int i = threadIdx.x; i < kPoissonC; i += blockDim.x) sF[i] = W.F[i];
    for (int i = threadIdx.x; i < kGuide; i += blockDim.x) sG[i] = gG[i];
}

// a wave's LDS counters added to one of the HBM counter copies (lane 0)
__device__ inline void flush_wave_counters(const WorkG& W, LAS unsigned long long* wcnt, int gw)
{
    wave_sync();
    if (lane_id() == 0) {
        GAS unsigned long long* dst = W.counters + static_cast<size_t>(gw % kCounterCopies) * kCounterStride;
#pragma unroll
        for (int k = 0; k < kNumCounters; ++k) {
            const unsigned long long v = wcnt[k];
            if (v) __hip_atomic_fetch_add(dst + k, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// One wave's share of a phase: the chunk gw of active cells (P.chunk cells).
// OWN_COUNTERS: the wave's LDS counters start at zero here and go to HBM at
// the end; otherwise the caller clears and flushes them (a launch of many
// phases keeps adding to them).
template <bool F32, bool SHELL, bool OWN_COUNTERS = true>
__device__ __forceinline__ void phase_sphere_body(const Params& P, const WorkG& W, int phase, int gw)
{
    LAS unsigned char* smem = lds_base();
    LAS double* sF = (LAS double*)smem;
    LAS int* sG = (LAS int*)(smem + kPoissonC * sizeof(double));

    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));  // wave-uniform
    LAS unsigned char* wbase = smem + kTableLds + static_cast<size_t>(wv) * P.wave_lds;
    auto stage_buf = [&](int b) {
        LAS unsigned char* q = wbase + static_cast<size_t>(b) * (P.off_cnt / 2);
        return SphereStage{(LAS int*)q, (LAS double*)(q + P.off_rec_a), (LAS double*)(q + P.off_rec_b)};
    };

    // the wave's counters live in its LDS (uniform values, no registers); lane
    // 0 adds to them without waiting for the result
    LAS unsigned long long* wcnt = (LAS unsigned long long*)(wbase + P.off_cnt);
    auto wadd = [&](int k, unsigned long long v) {
        __hip_atomic_fetch_add(wcnt + k, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    if (OWN_COUNTERS && lane < kNumCounters) wcnt[lane] = 0ull;
    unsigned fallbacks = 0;  // FP64 fallbacks of the guarded FP32 tests (this lane)

    const int colour = W.perm[phase];
    const double g0 = W.grid[0], g1 = W.grid[1], g2 = W.grid[2];
    const Mat3 Rnone{};

    // the chunk: lane k < P.chunk holds active cell gw * P.chunk + k
    int Xk = 0, startk = 0, nck = 0;  // Xk: the cell's coordinates, cx | cy << 10 | cz << 20
    {
        int a = gw * P.chunk + lane;
        if (lane < P.chunk && a < P.active_cells) {
            int ax = a % P.h, ay = (a / P.h) % P.h, az = a / (P.h * P.h);
            const int cxk = 2 * ax + (colour & 1);
            const int cyk = 2 * ay + ((colour >> 1) & 1);
            const int czk = 2 * az + ((colour >> 2) & 1);
            Xk = cxk | (cyk << 10) | (czk << 20);
            const int Ck = cxk + P.n * (cyk + P.n * czk);
            startk = W.cell_start[Ck];
            nck = W.cell_start[Ck + 1] - startk;
        }
    }
    unsigned long long todo = __ballot(nck > 0);

    // Trial slots of the chunk: cell k's n_select * n_c trials take slots
    // offk .. offk + ntrk - 1, in cell order.  A trial's own draws (selection,
    // translation, acceptance and its Poisson chunks: B Philox blocks) depend
    // on the random streams alone, not on the state, so those of T = 64 / B
    // trials are drawn at once, one block per lane (and the Poisson chunks
    // resolved there), and read across lanes when each trial runs.
    const int ntrk = P.n_select * nck;
    int nslots;
    const int offk = wave_excl_scan(ntrk, nslots);
    const int B = 3 + P.n_chunks < 64 ? 3 + P.n_chunks : 64;
    const int T = 64 / B;
    int sb = -64;  // first slot of the batch in the lanes (none yet)
    Words wb{0u, 0u, 0u, 0u};
    int jlb = 0, kcb = 0;
    auto draw_batch = [&](int s0) {
        const int tl = lane / B, q = lane - tl * B;
        const int sl = s0 + tl;
        // the cell of slot sl (slots of a cell are contiguous, cells in order)
        int k = 0;
        for (int kk = 1; kk < P.chunk; ++kk)
            if (static_cast<int>(rdlane_u(static_cast<uint32_t>(offk), kk)) <= sl) k = kk;
        const int o = __shfl(offk, k, 64), nk = __shfl(nck, k, 64), Cs = cell_id(P, __shfl(Xk, k, 64));
        const bool valid = tl < T && sl < nslots;
        const uint32_t purpose = q == 0 ? kSelect : (q == 1 ? kTrans : (q == 2 ? kAccept : kPoisson));
        const uint32_t index = q >= 3 ? static_cast<uint32_t>(q - 3) : 0u;
        wb = draw(P, static_cast<uint32_t>(Cs), static_cast<uint32_t>(sl - o), purpose, index);
        jlb = static_cast<int>(pick(wb.w0, static_cast<uint32_t>(nk > 0 ? nk : 1)));
        kcb = 0;
        if (valid && P.has_dep && q >= 3 && q - 3 < P.n_chunks) kcb = poisson_guided(sF, sG, u52(wb.w0, wb.w1), P);
    };
    // ranges of the stencil of chunk cell k (k < 0: none)
    auto ranges_of = [&](int k, int& es, int& ec) {
        const NbOff nb = nb_offset(P.n);
        if (k < 0) {
            stencil_ranges(P, W, nb, -1, 0, 0, 0, es, ec);
            return;
        }
        const int X = static_cast<int>(rdlane_u(static_cast<uint32_t>(Xk), k));
        stencil_ranges(P, W, nb, cell_id(P, X), X & 1023, (X >> 10) & 1023, X >> 20, es, ec);
    };
    // pipeline: ranges two cells ahead, records one cell ahead
    auto next_cell = [&](unsigned long long& m) -> int {
        if (!m) return -1;
        int k = ffs64(m);
        m &= m - 1ull;
        return k;
    };
    unsigned long long rem = todo;
    int kc = next_cell(rem);   // cell being processed
    int kn = next_cell(rem);   // next
    int es, ec;
    ranges_of(kc, es, ec);
    int nst_cur = (kc >= 0) ? stage_issue(P, W, stage_buf(0), es, ec) : 0;
    ranges_of(kn, es, ec);
    int buf = 0;

    while (kc >= 0) {
        __builtin_amdgcn_s_waitcnt(0);
        wave_sync();
        const SphereStage S0 = stage_buf(buf);
        const int C = cell_id(P, static_cast<int>(rdlane_u(static_cast<uint32_t>(Xk), kc)));
        const int start = static_cast<int>(rdlane_u(static_cast<uint32_t>(startk), kc));
        const int nc = static_cast<int>(rdlane_u(static_cast<uint32_t>(nck), kc));
        const int nst = nst_cur;
        const int slot0 = static_cast<int>(rdlane_u(static_cast<uint32_t>(offk), kc));
        // start staging the next cell while this one runs
        int kn2 = next_cell(rem);
        int nst_next = 0;
        if (kn >= 0) {
            nst_next = stage_issue(P, W, stage_buf(buf ^ 1), es, ec);
            ranges_of(kn2, es, ec);
        }
        if (nst < 0) {
            if (lane == 0) __hip_atomic_fetch_or(W.flags, kFlagListOverflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const int ntr = P.n_select * nc;
            for (int t = 0; t < ntr; ++t) {
                // --- this trial's draws, from the batch in the lanes -------------
                const int slot = slot0 + t;
                if (slot >= sb + T) {
                    sb = slot;
                    draw_batch(sb);
                }
                const int base = (slot - sb) * B;
                const int jl = static_cast<int>(rdlane_u(static_cast<uint32_t>(jlb), base));
                // own members are entries 0 .. nc-1: staged, or (past the stage) in HBM
                const double4 pj = jl < kStage ? stage_rec(S0, jl) : rd4(W.rpos, start + jl);
                Vec3 xn;
                {
                    uint32_t tw0 = rdlane_u(wb.w0, base + 1), tw1 = rdlane_u(wb.w1, base + 1), tw2 = rdlane_u(wb.w2, base + 1);
                    auto wrapL = [&](double v) {
                        const double a = v - P.L, b = v + P.L;
                        return v >= P.L ? a : (v < 0.0 ? b : v);
                    };
                    xn.x = wrapL(pj.x + P.d_trans * sym01(tw0));
                    xn.y = wrapL(pj.y + P.d_trans * sym01(tw1));
                    xn.z = wrapL(pj.z + P.d_trans * sym01(tw2));
                }
                TrialOut o{0, 0, 0, 0, 0, 0, 0, false};
                if (cell_of(P, xn.x, xn.y, xn.z, g0, g1, g2) != C) {
                    o.reason = 1;
                } else {
                    // stencil geometry relative to x': lane i holds entry i
                    Vec3 Dreg = v3(kFar, kFar, kFar);
                    if (lane < nst && lane < kStage && lane != jl) {
                        double4 r = stage_rec(S0, lane);
                        Dreg = v3(mi(P, r.x - xn.x), mi(P, r.y - xn.y), mi(P, r.z - xn.z));
                    }
                    // hard overlap with another colloid
                    bool hit = dot(Dreg, Dreg) < P.S.dsq;
                    for (int i = kStage + lane; i < nst; i += 64) {
                        if (i == jl) continue;  // the moved colloid itself (a member past the stage)
                        double4 r = rd4(W.rpos, S0.list[i]);
                        Vec3 D = v3(mi(P, r.x - xn.x), mi(P, r.y - xn.y), mi(P, r.z - xn.z));
                        hit = hit || dot(D, D) < P.S.dsq;
                    }
                    if (lane == 0) wadd(cOverlapChecks, static_cast<unsigned long long>(nst - 1));
                    // staged entries a CB trial point can reach (the moved colloid's lane holds kFar)
                    const unsigned long long rmask = __ballot(dot(Dreg, Dreg) < P.reach_sq);
                    if (__ballot(hit) != 0ull) {
                        o.reason = 2;
                    } else if (P.has_dep) {
                        // chunk counts sit in lanes base + 3 .. base + 2 + n_chunks; chunks past
                        // lane 63 (more than 61 of them: then one trial per batch) are drawn here
                        int kx = (lane >= base + 3 && lane < base + 3 + P.n_chunks) ? kcb : 0;
                        for (int cbase = 61; cbase < P.n_chunks; cbase += 64) {
                            int ci = cbase + lane;
                            if (ci < P.n_chunks) {
                                Words pw = draw(P, static_cast<uint32_t>(C), static_cast<uint32_t>(t), kPoisson,
                                                static_cast<uint32_t>(ci));
                                kx += poisson_guided(sF, sG, u52(pw.w0, pw.w1), P);
                            }
                        }
                        const uint32_t Np = static_cast<uint32_t>(P.n_chunks <= 8 ? lanes_sum(kcb, base + 3, P.n_chunks)
                                                                                  : wave_sum(kx));
                        o.n_dep = Np;
                        const double au = u52(rdlane_u(wb.w0, base + 2), rdlane_u(wb.w1, base + 2));
                        const Vec3 Dold = v3(mi(P, pj.x - xn.x), mi(P, pj.y - xn.y), mi(P, pj.z - xn.z));
                        double ratio = 1.0;
                        bool done = false;
                        uint32_t kbase = 0, blk = 0;
                        while (!done && kbase < Np && blk < (1u << 30)) {
                            bool acc0, acc1;
                            Vec3 e0, e1;
                            depl_candidates_t<SHELL>(P, static_cast<uint32_t>(C), static_cast<uint32_t>(t), blk + lane, acc0,
                                            acc1, e0, e1);
                            unsigned long long m0 = __ballot(acc0), m1 = __ballot(acc1);
                            uint32_t k0 = kbase + static_cast<uint32_t>(bits_below(m0) + bits_below(m1));
                            uint32_t k1 = k0 + (acc0 ? 1u : 0u);
                            // ignored by the old pose (every ball point overlaps the new pose)
                            bool v0 = acc0 && k0 < Np, v1 = acc1 && k1 < Np;
                            // evaluated in every lane (no branch; a lane's value counts only where valid)
                            const bool in0 = sphere_in<F32>(P, e0, Dold, v0, fallbacks);
                            const bool in1 = sphere_in<F32>(P, e1, Dold, v1, fallbacks);
                            v0 = v0 && !in0;
                            v1 = v1 && !in1;
                            unsigned long long r0 = __ballot(v0), r1 = __ballot(v1);
                            while ((r0 | r1) && !done) {
                                int l0 = r0 ? ffs64(r0) : 64, l1 = r1 ? ffs64(r1) : 64;
                                int src, cand;
                                if (l0 <= l1) {
                                    src = l0;
                                    cand = 0;
                                    r0 &= ~(1ull << l0);
                                } else {
                                    src = l1;
                                    cand = 1;
                                    r1 &= ~(1ull << l1);
                                }
                                src = __builtin_amdgcn_readfirstlane(src);
                                Vec3 es3 = cand ? e1 : e0;
                                es3 = v3(rdlane_d(es3.x, src), rdlane_d(es3.y, src), rdlane_d(es3.z, src));
                                uint32_t ks = rdlane_u(cand ? k1 : k0, src);
                                bool h = sphere_in<F32>(P, es3, Dreg, true, fallbacks);
                                for (int i = kStage + lane; i < nst; i += 64) {
                                    if (i == jl) continue;
                                    double4 r = rd4(W.rpos, S0.list[i]);
                                    Vec3 D = v3(mi(P, r.x - xn.x), mi(P, r.y - xn.y), mi(P, r.z - xn.z));
                                    h = h || dot(es3 - D, es3 - D) < P.S.R0sq;
                                }
                                if (__ballot(h) != 0ull) continue;  // ignored
                                o.nblk++;
                                if (P.n_trial == 0) {
                                    o.reason = 3;
                                    o.resolved = ks + 1;
                                    done = true;
                                    break;
                                }
                                // configurational bias: one ballot-compacted pass per depletant
                                const unsigned long long lo_half = 0x00000000FFFFFFFFull;
                                const bool fwd = lane < 32;
                                const unsigned long long half = fwd ? lo_half : ~lo_half;
                                const int need_f = P.n_trial, need_r = P.n_trial - 1;
                                int have_f = 0, have_r = 0;
                                uint32_t Wf = 0, Wr = 0;
                                for (uint32_t cb = 0; (have_f < need_f || have_r < need_r) && cb < 65536u; cb += 32) {
                                    const int have = fwd ? have_f : have_r;
                                    const int need = fwd ? need_f : need_r;
                                    Words cw = draw(P, static_cast<uint32_t>(C), static_cast<uint32_t>(t),
                                                    fwd ? kCbFwd : kCbRev,
                                                    (ks << 16) | (cb + static_cast<uint32_t>(lane & 31)));
                                    double c0x, c0y, c0z, c1x, c1y, c1z;
                                    bool q0 = ball3(cw.w0, cw.w1, c0x, c0y, c0z) && have < need;
                                    bool q1 = ball3(cw.w2, cw.w3, c1x, c1y, c1z) && have < need;
                                    const unsigned long long M0 = __ballot(q0), M1 = __ballot(q1);
                                    int rk0 = have + bits_below(M0 & half) + bits_below(M1 & half);
                                    int rk1 = rk0 + (q0 ? 1 : 0);
                                    bool u0 = q0 && rk0 < need, u1 = q1 && rk1 < need;
                                    Vec3 f0 = v3(P.s_ball * c0x, P.s_ball * c0y, P.s_ball * c0z);
                                    Vec3 f1 = v3(P.s_ball * c1x, P.s_ball * c1y, P.s_ball * c1z);
                                    Vec3 p0 = fwd ? (Dold + f0) : f0, p1 = fwd ? (Dold + f1) : f1;
                                    // forward: misses the new pose; reverse: misses the old pose
                                    if (u0) u0 = fwd ? !(dot(p0, p0) < P.S.R0sq) : !(dot(f0 - Dold, f0 - Dold) < P.S.R0sq);
                                    if (u1) u1 = fwd ? !(dot(p1, p1) < P.S.R0sq) : !(dot(f1 - Dold, f1 - Dold) < P.S.R0sq);
                                    u0 = u0 && !sphere_hit_lane(P, W, S0, nst, jl, xn, rmask, Dreg, p0, u0);
                                    u1 = u1 && !sphere_hit_lane(P, W, S0, nst, jl, xn, rmask, Dreg, p1, u1);
                                    const unsigned long long V0 = __ballot(u0), V1 = __ballot(u1);
                                    Wf += static_cast<uint32_t>(__popcll(V0 & lo_half) + __popcll(V1 & lo_half));
                                    Wr += static_cast<uint32_t>(__popcll(V0 & ~lo_half) + __popcll(V1 & ~lo_half));
                                    have_f += __popcll(M0 & lo_half) + __popcll(M1 & lo_half);
                                    have_r += __popcll(M0 & ~lo_half) + __popcll(M1 & ~lo_half);
                                }
                                o.wf += Wf;
                                if (Wf == 0) {
                                    o.reason = 4;
                                    o.resolved = ks + 1 + o.cbt + static_cast<uint32_t>(P.n_trial);
                                    o.cbt += static_cast<uint32_t>(P.n_trial);
                                    done = true;
                                    break;
                                }
                                o.wr += Wr;
                                ratio = ratio * (static_cast<double>(Wf) / static_cast<double>(1 + Wr));
                                o.cbt += static_cast<uint32_t>(2 * P.n_trial - 1);
                            }
                            kbase += static_cast<uint32_t>(__popcll(m0) + __popcll(m1));
                            blk += 64;
                        }
                        if (!done) {
                            o.resolved = Np + o.cbt;
                            if (o.nblk > 0 && !(au < ratio)) o.reason = 5;
                        }
                    }
                }
                // --- accept / commit / record -----------------------------------
                if (o.reason == 0 && lane == 0) {
                    if (jl < kStage) {
                        S0.recA[2 * jl] = xn.x;
                        S0.recA[2 * jl + 1] = xn.y;
                        S0.recB[2 * jl] = xn.z;
                    } else {
                        // a member past the stage: its record is updated in place (only this
                        // wave reads the cell's members during the phase)
                        wr4(W.rpos, start + jl, make_double4(xn.x, xn.y, xn.z, pj.w));
                    }
                }
                wave_sync();
                if (lane == 0) {
                    wadd(cTrials, 1ull);
                    wadd(cAccepts + o.reason, 1ull);  // reasons 0..5 in counter order
                    if (o.n_dep) wadd(cDrawn, static_cast<unsigned long long>(o.n_dep));
                    if (o.resolved) wadd(cResolved, static_cast<unsigned long long>(o.resolved));
                    if (o.cbt) wadd(cCbTrials, static_cast<unsigned long long>(o.cbt));
                }
                if (P.trace && lane == 0) {
                    GAS uint32_t* r = (GAS uint32_t*)(W.trace + (static_cast<size_t>(P.n_select) * start + t) * 40);
                    r[0] = P.sweep;
                    r[1] = static_cast<uint32_t>(C);
                    r[2] = static_cast<uint32_t>(t);
                    r[3] = static_cast<uint32_t>(pj.w);
                    r[4] = o.n_dep;
                    r[5] = o.resolved;
                    r[6] = o.nblk;
                    r[7] = o.wf;
                    r[8] = o.wr;
                    r[9] = static_cast<uint32_t>(phase) | (static_cast<uint32_t>(o.reason) << 8);
                }
            }
            // staged own-cell records back to HBM
            for (int i = lane; i < nc && i < kStage; i += 64) wr4(W.rpos, start + i, stage_rec(S0, i));
        }
        kc = kn;
        kn = kn2;
        nst_cur = nst_next;
        buf ^= 1;
    }
    (void)Rnone;
    if constexpr (F32) {
        const int fb = wave_sum(static_cast<int>(fallbacks));
        if (lane == 0 && fb) wadd(cFp64Fallbacks, static_cast<unsigned long long>(fb));
    }
    if constexpr (OWN_COUNTERS) flush_wave_counters(W, wcnt, gw);
}

#ifndef HPMC_SPHERE_WAVES_PER_EU
#define HPMC_SPHERE_WAVES_PER_EU 4
#endif
// F32: depletant tests in FP32 with the FP64 guard band (precision HPMC_FP32_GUARDED);
// SHELL: depletants in the shell region
// Phase launches are flat: the blocks of every replica of a group follow each
// other (brep[b] names block b's replica; null for a launch of one replica),
// so a launch holds only blocks with work, and every block serves one replica
// (its Poisson table and LDS layout).
#define HPMC_PHASE_REPLICA(D, brep)                                             \
    const int rep_ = (brep) ? (brep)[blockIdx.x] : 0;                           \
    Params P = (D)[rep_].P;                                                     \
    const WorkG W = gview((D)[rep_].W);                                         \
    const int lb = static_cast<int>(blockIdx.x) - P.blk0; /* block in the replica */ \
    const int nb = P.nblk

template <bool F32, bool SHELL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HPMC_SPHERE_WAVES_PER_EU, 8))) void
phase_sphere_kernel(const Desc* __restrict__ D, const int* __restrict__ brep, int phase)
{
    HPMC_PHASE_REPLICA(D, brep);
    P.sweep = *W.sweep_dev;
    load_table(W, lds_base());
    __syncthreads();
    // one box: XCD-aware chunk order; a batch keeps the dispatch order.  Every
    // wave takes one chunk of P.chunk active cells (the launch covers them all).
    const int b = brep ? lb : xcd_block(lb, nb);
    phase_sphere_body<F32, SHELL>(P, W, phase,
                                  b * P.waves_per_block +
                                      __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6)));
}

// Small sphere boxes: one workgroup of kSmallWaves waves sweeps a whole
// replica, n_sweeps sweeps in one launch (grid shift and colour order, cell
// list, the 8 phases, scatter back), with workgroup barriers between the
// steps instead of kernel boundaries.  The same arithmetic as the multi-kernel
// sweep, so the same trajectory.
__device__ inline void grid_setup(const Params& P, const Work& W)
{
    Words a = draw(P, kNoCell, 0, kGrid, 0);
    W.grid[0] = P.w * u01(a.w0);
    W.grid[1] = P.w * u01(a.w1);
    W.grid[2] = P.w * u01(a.w2);
    Words b = draw(P, kNoCell, 0, kGrid, 1);
    Words c = draw(P, kNoCell, 0, kGrid, 2);
    const uint32_t fy[7] = {b.w0, b.w1, b.w2, b.w3, c.w0, c.w1, c.w2};
    // Fisher-Yates over the 8 colours; the permutation is packed four bits
    // per entry into one register (entry i in bits 4i .. 4i + 3)
    uint32_t perm = 0x76543210u;
#pragma unroll
    for (int i = 7; i >= 1; --i) {
        const uint32_t j = pick(fy[7 - i], static_cast<uint32_t>(i + 1));
        const uint32_t si = 4u * static_cast<uint32_t>(i), sj = 4u * j;
        const uint32_t pi = (perm >> si) & 15u, pj = (perm >> sj) & 15u;
        perm &= ~((15u << si) | (15u << sj));
        perm |= (pj << si) | (pi << sj);
    }
    for (int i = 0; i < 8; ++i) W.perm[i] = static_cast<int>((perm >> (4 * i)) & 15u);
}

template <bool F32, bool SHELL>
__global__ __launch_bounds__(64 * kSmallWaves) void sweep_small_kernel(const Desc* __restrict__ D, int n_sweeps)
{
    Params P = D[blockIdx.y].P;
    const Work W = D[blockIdx.y].W;
    const WorkG WG = gview(W);
    __shared__ int s_wsum[kSmallWaves];
    __shared__ int s_carry;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int wv = tid >> 6;
    const uint32_t sweep0 = *W.sweep_dev;
    // spread the active cells of a phase over the waves (trials of one cell are serial)
    P.chunk = (P.active_cells + kSmallWaves - 1) / kSmallWaves;
    if (P.chunk > 64) P.chunk = 64;
    load_table(WG, lds_base());
    // each wave's LDS counters add up over every phase and sweep of the launch
    LAS unsigned long long* wcnt =
        (LAS unsigned long long*)(lds_base() + kTableLds + static_cast<size_t>(wv) * P.wave_lds + P.off_cnt);
    if (lane_id() < kNumCounters) wcnt[lane_id()] = 0ull;
    for (int sw = 0; sw < n_sweeps; ++sw) {
        P.sweep = sweep0 + static_cast<uint32_t>(sw);
        if (tid == 0) grid_setup(P, W);
        for (int i = tid; i < P.ncells; i += nt) W.cell_count[i] = 0;
        __syncthreads();
        for (int i = tid; i < P.N; i += nt) {
            int c = cell_of(P, W.pos[i], W.pos[P.N + i], W.pos[2 * P.N + i], W.grid[0], W.grid[1], W.grid[2]);
            W.pcell[i] = c;
            W.prank[i] = atomicAdd(&W.cell_count[c], 1);
        }
        if (tid == 0) s_carry = 0;
        __syncthreads();
        // exclusive scan of the cell counts, one thread per cell, tile by tile
        for (int base = 0; base < P.ncells; base += nt) {
            int i = base + tid;
            int v = i < P.ncells ? W.cell_count[i] : 0;
            int tot;
            int ex = wave_excl_scan(v, tot);
            if (lane_id() == 0) s_wsum[wv] = tot;
            __syncthreads();
            int woff = 0, all = 0;
            for (int k = 0; k < kSmallWaves; ++k) {
                if (k < wv) woff += s_wsum[k];
                all += s_wsum[k];
            }
            if (i < P.ncells) W.cell_start[i] = s_carry + woff + ex;
            __syncthreads();
            if (tid == 0) s_carry += all;
            __syncthreads();
        }
        if (tid == 0) W.cell_start[P.ncells] = P.N;
        __syncthreads();
        for (int i = tid; i < P.N; i += nt) W.order[W.cell_start[W.pcell[i]] + W.prank[i]] = i;
        __syncthreads();
        // each cell's members in ascending index: ranks among the cell, then scatter again
        for (int i = tid; i < P.N; i += nt) {
            const int c = W.pcell[i];
            int r = 0;
            for (int k = W.cell_start[c]; k < W.cell_start[c + 1]; ++k) r += W.order[k] < i ? 1 : 0;
            W.prank[i] = r;
        }
        __syncthreads();
        for (int i = tid; i < P.N; i += nt) W.order[W.cell_start[W.pcell[i]] + W.prank[i]] = i;
        __syncthreads();
        for (int q = tid; q < P.N; q += nt) {
            int i = W.order[q];
            wr4(W.rpos, q, make_double4(W.pos[i], W.pos[P.N + i], W.pos[2 * P.N + i], static_cast<double>(i)));
        }
        __syncthreads();
        for (int phase = 0; phase < 8; ++phase) {
            for (int gw = wv; gw * P.chunk < P.active_cells; gw += kSmallWaves)
                phase_sphere_body<F32, SHELL, false>(P, WG, phase, gw);
            __syncthreads();
        }
        for (int q = tid; q < P.N; q += nt) {
            double4 r = rd4(W.rpos, q);
            int i = static_cast<int>(r.w);
            W.pos[i] = r.x;
            W.pos[P.N + i] = r.y;
            W.pos[2 * P.N + i] = r.z;
        }
        __syncthreads();
    }
    flush_wave_counters(WG, wcnt, wv);
    if (tid == 0) *W.sweep_dev = sweep0 + static_cast<uint32_t>(n_sweeps);
}

// F32: depletant predicates in FP32 with the FP64 guard band
template <int KIND, bool F32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(F32 ? 2 : 1, 8))) void phase_oriented_kernel(
    const Desc* __restrict__ D, const int* __restrict__ brep, int phase)
{
    HPMC_PHASE_REPLICA(D, brep);
    P.sweep = *W.sweep_dev;
    phase_body<KIND, F32>(P, W, phase, lb, nb);
}

__global__ void reduce_counters_kernel(const Desc* __restrict__ D)
{
    const Work W = D[blockIdx.y].W;
    int k = threadIdx.x;
    if (k >= kNumCounters) return;
    unsigned long long s = 0;
    for (int c = 1; c < kCounterCopies; ++c) s += W.counters[static_cast<size_t>(c) * kCounterStride + k];
    W.counters[k] += s;
}

// hard-core check of a state: pairs (slot order) that overlap
__global__ void overlap_count_kernel(const Desc* __restrict__ D)
{
    HPMC_REPLICA(D);
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.N) return;
    double4 a = rd4(W.rpos, s);
    int ia = static_cast<int>(a.w);
    Mat3 RA, RB;
    if (P.S.oriented) {
        double4 q = rd4(W.rquat, s);
        RA = quat_to_mat(q.x, q.y, q.z, q.w);
    }
    int cx = cell_coord(P, a.x, 0.0), cy = cell_coord(P, a.y, 0.0), cz = cell_coord(P, a.z, 0.0);
    const int noff = (P.n == 2) ? 2 : 3;
    unsigned long long cntv = 0;
    for (int l = 0; l < noff * noff * noff; ++l) {
        int dx = l % noff, dy = (l / noff) % noff, dz = l / (noff * noff);
        if (noff == 3) {
            dx -= 1;
            dy -= 1;
            dz -= 1;
        }
        int e = (cx + dx + P.n) % P.n + P.n * ((cy + dy + P.n) % P.n + P.n * ((cz + dz + P.n) % P.n));
        for (int q = W.cell_start[e]; q < W.cell_start[e + 1]; ++q) {
            double4 b = rd4(W.rpos, q);
            int ib = static_cast<int>(b.w);
            if (ib <= ia) continue;
            Vec3 d = v3(mi(P, b.x - a.x), mi(P, b.y - a.y), mi(P, b.z - a.z));
            if (P.S.oriented) {
                double4 qb = rd4(W.rquat, q);
                RB = quat_to_mat(qb.x, qb.y, qb.z, qb.w);
            }
            if (pair_overlap(P.S, d, RA, RB).overlap) cntv++;
        }
    }
    if (cntv) atomicAdd(W.obs, cntv);
}

// ---------------------------------------------------------------------------
// observables of the current state (cell list built with zero shift)
// ---------------------------------------------------------------------------
namespace {

// cells within +-k of c along one axis, de-duplicated when 2k+1 >= n
__device__ inline int axis_span(int n, int k, int& first)
{
    if (2 * k + 1 >= n) {
        first = 0;
        return n;
    }
    first = -k;
    return 2 * k + 1;
}

__device__ inline int wrap_cell(int c, int n) { return ((c % n) + n) % n; }

}  // namespace

// pair-distance histogram (pairs i < j), W.obs[0..n_bins)
__global__ __launch_bounds__(256) void gr_kernel(const Desc* __restrict__ D, int n_bins, double r_max, int k)
{
    HPMC_REPLICA(D);
    extern __shared__ unsigned long long hist[];
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x) hist[b] = 0ull;
    __syncthreads();
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < P.N) {
        double4 a = rd4(W.rpos, s);
        int ia = static_cast<int>(a.w);
        int cx = cell_coord(P, a.x, 0.0), cy = cell_coord(P, a.y, 0.0), cz = cell_coord(P, a.z, 0.0);
        double inv_dr = static_cast<double>(n_bins) / r_max;
        double rm2 = r_max * r_max;
        int fx, fy, fz;
        int nx = axis_span(P.n, k, fx), ny = axis_span(P.n, k, fy), nz = axis_span(P.n, k, fz);
        for (int dz = 0; dz < nz; ++dz)
            for (int dy = 0; dy < ny; ++dy)
                for (int dx = 0; dx < nx; ++dx) {
                    int ex = (nx == P.n) ? dx : wrap_cell(cx + fx + dx, P.n);
                    int ey = (ny == P.n) ? dy : wrap_cell(cy + fy + dy, P.n);
                    int ez = (nz == P.n) ? dz : wrap_cell(cz + fz + dz, P.n);
                    int e = ex + P.n * (ey + P.n * ez);
                    for (int q = W.cell_start[e]; q < W.cell_start[e + 1]; ++q) {
                        double4 b = rd4(W.rpos, q);
                        if (static_cast<int>(b.w) <= ia) continue;
                        Vec3 d = v3(mi(P, b.x - a.x), mi(P, b.y - a.y), mi(P, b.z - a.z));
                        double r2 = dot(d, d);
                        if (r2 >= rm2) continue;
                        double r = sqrt(r2);
                        if (r < r_max) {
                            int bin = static_cast<int>(floor(r * inv_dr));
                            if (bin < n_bins) atomicAdd(&hist[bin], 1ull);
                        }
                    }
                }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
        if (hist[b]) atomicAdd(&W.obs[b], hist[b]);
}

// uniform probes that overlap no colloid (displacements scaled by `scale`)
__global__ __launch_bounds__(256) void free_volume_kernel(const Desc* __restrict__ D, int64_t n_probe, uint32_t seq,
                                                          double scale, int slot)
{
    HPMC_REPLICA(D);
    int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int free_ = 0;
    if (p < n_probe) {
        Words w = philox(seq, kNoCell, kObsFv, static_cast<uint32_t>(p), P.key0, P.key1);
        double X = P.L * u01(w.w0), Y = P.L * u01(w.w1), Z = P.L * u01(w.w2);
        int cx = cell_coord(P, X, 0.0), cy = cell_coord(P, Y, 0.0), cz = cell_coord(P, Z, 0.0);
        const int noff = (P.n == 2) ? 2 : 3;
        bool hit = false;
        for (int l = 0; l < noff * noff * noff && !hit; ++l) {
            int dx = l % noff, dy = (l / noff) % noff, dz = l / (noff * noff);
            if (noff == 3) {
                dx -= 1;
                dy -= 1;
                dz -= 1;
            }
            int e = wrap_cell(cx + dx, P.n) + P.n * (wrap_cell(cy + dy, P.n) + P.n * wrap_cell(cz + dz, P.n));
            for (int q = W.cell_start[e]; q < W.cell_start[e + 1] && !hit; ++q) {
                double4 b = rd4(W.rpos, q);
                Vec3 v = v3(mi(P, X - b.x), mi(P, Y - b.y), mi(P, Z - b.z));
                if (scale != 1.0) v = v3(v.x * scale, v.y * scale, v.z * scale);
                Mat3 R;
                if (P.S.oriented) {
                    double4 qq = rd4(W.rquat, q);
                    R = quat_to_mat(qq.x, qq.y, qq.z, qq.w);
                }
                hit = dep_overlap(P.S, v, R);
            }
        }
        free_ = hit ? 0 : 1;
    }
    int tot = wave_sum(free_);
    if (lane_id() == 0 && tot) atomicAdd(&W.obs[slot], static_cast<unsigned long long>(tot));
}

// Scale-distribution function (per-particle smallest compression at which a
// neighbour pair overlaps, histogram in W.obs).
// Scale factor at which the pair (A at the origin, B at offset d) first
// overlaps when the centre distance is compressed by (1 - x): bisection of
// [0, x_max] in 40 steps (overlap grows monotonically with x).
__device__ inline double sdf_bisect(const Shape& S, Vec3 d, const Mat3& RA, const Mat3& RB, double x_max, double lim)
{
    double lo = 0.0, hi = x_max;
    for (int it = 0; it < 40; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = 1.0 - mid;
        Vec3 dx3 = v3(d.x * fm, d.y * fm, d.z * fm);
        bool ov = dot(dx3, dx3) < lim * lim && !sat_disjoint(S, dx3, RA, RB) && mpr_overlap(S, dx3, RA, RB).overlap;
        if (ov)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

constexpr int kSdfCand = 16;  // candidate pairs per particle held for the bisection pass

// Per particle (thread) the minimum compression factor over its neighbours,
// histogrammed.  Spheres: closed form.  Convex shapes: a scan over the
// neighbours keeps the pairs that overlap at the largest compression x_max,
// then the lanes of a wave bisect their candidates together, so bisections
// of different particles do not run one after another.
__global__ __launch_bounds__(128) void sdf_kernel(const Desc* __restrict__ D, int n_bins, double x_max, int k)
{
    HPMC_REPLICA(D);
    __shared__ int cand_lds[128 * kSdfCand];
    int* cand = cand_lds + threadIdx.x * kSdfCand;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = s < P.N;
    double4 a = live ? rd4(W.rpos, s) : make_double4(0.0, 0.0, 0.0, -1.0);
    int ia = static_cast<int>(a.w);
    Mat3 RA, RB;
    if (P.S.oriented && live) {
        double4 q = rd4(W.rquat, s);
        RA = quat_to_mat(q.x, q.y, q.z, q.w);
    }
    int cx = cell_coord(P, a.x, 0.0), cy = cell_coord(P, a.y, 0.0), cz = cell_coord(P, a.z, 0.0);
    double lim_s = 2.0 * P.S.rcirc / (1.0 - x_max);
    double lim = 2.0 * P.S.rcirc;
    double xmin = x_max;
    int ncand = 0;
    bool overflow = false;
    int fx, fy, fz;
    int nx = axis_span(P.n, k, fx), ny = axis_span(P.n, k, fy), nz = axis_span(P.n, k, fz);
    for (int dz = 0; dz < nz && live; ++dz)
        for (int dy = 0; dy < ny; ++dy)
            for (int dx = 0; dx < nx; ++dx) {
                int ex = (nx == P.n) ? dx : wrap_cell(cx + fx + dx, P.n);
                int ey = (ny == P.n) ? dy : wrap_cell(cy + fy + dy, P.n);
                int ez = (nz == P.n) ? dz : wrap_cell(cz + fz + dz, P.n);
                int e = ex + P.n * (ey + P.n * ez);
                for (int q = W.cell_start[e]; q < W.cell_start[e + 1]; ++q) {
                    double4 b = rd4(W.rpos, q);
                    if (static_cast<int>(b.w) == ia) continue;
                    Vec3 d = v3(mi(P, b.x - a.x), mi(P, b.y - a.y), mi(P, b.z - a.z));
                    double dd = dot(d, d);
                    if (dd >= lim_s * lim_s) continue;
                    if (P.S.kind == kSphere) {
                        double r = sqrt(dd);
                        double x = 1.0 - P.S.a * 2.0 / r;
                        if (x > x_max) x = x_max;
                        if (x < xmin) xmin = x;
                        continue;
                    }
                    // keep the pair if it overlaps at the largest compression
                    double4 qb = rd4(W.rquat, q);
                    RB = quat_to_mat(qb.x, qb.y, qb.z, qb.w);
                    double f = 1.0 - x_max;
                    Vec3 dm = v3(d.x * f, d.y * f, d.z * f);
                    if (dot(dm, dm) >= lim * lim || sat_disjoint(P.S, dm, RA, RB) ||
                        !mpr_overlap(P.S, dm, RA, RB).overlap)
                        continue;
                    if (ncand < kSdfCand) {
                        cand[ncand++] = q;
                    } else {
                        overflow = true;  // rare: bisect in place
                        double x = sdf_bisect(P.S, d, RA, RB, x_max, lim);
                        if (x < xmin) xmin = x;
                    }
                }
            }
    (void)overflow;
    // bisection pass: candidate c of every lane at the same time.  A pair that
    // does not overlap at the current minimum cannot lower it (monotonicity).
    for (int c = 0; c < ncand; ++c) {
        int q = cand[c];
        double4 b = rd4(W.rpos, q);
        Vec3 d = v3(mi(P, b.x - a.x), mi(P, b.y - a.y), mi(P, b.z - a.z));
        double4 qb = rd4(W.rquat, q);
        RB = quat_to_mat(qb.x, qb.y, qb.z, qb.w);
        if (xmin < x_max) {
            double f = 1.0 - xmin;
            Vec3 dm = v3(d.x * f, d.y * f, d.z * f);
            if (dot(dm, dm) >= lim * lim || sat_disjoint(P.S, dm, RA, RB) || !mpr_overlap(P.S, dm, RA, RB).overlap)
                continue;
        }
        double x = sdf_bisect(P.S, d, RA, RB, x_max, lim);
        if (x < xmin) xmin = x;
    }
    if (live && xmin < x_max) {
        int bin = static_cast<int>(floor(xmin * (static_cast<double>(n_bins) / x_max)));
        if (bin < n_bins) atomicAdd(&W.obs[bin], 1ull);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int blocks_for(int n, int bs) { return (n + bs - 1) / bs; }

hipError_t launch_fill_int(int* p, int n, int value, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p, n, value);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_build_cells(const Group& g, bool with_grid, hipStream_t stream)
{
    const int R = g.nrep;
    hipLaunchKernelGGL(grid_kernel, dim3(1, R), dim3(64), 0, stream, g.d, with_grid ? 1 : 0);
    hipLaunchKernelGGL(clear_cells_kernel, dim3(blocks_for(g.maxCells, 256), R), dim3(256), 0, stream, g.d);
    hipLaunchKernelGGL(bin_kernel, dim3(blocks_for(g.maxN, 256), R), dim3(256), 0, stream, g.d);
    int nb = blocks_for(g.maxCells, 1024);
    hipLaunchKernelGGL(scan_local_kernel, dim3(nb, R), dim3(256), 0, stream, g.d);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1, R), dim3(256), 0, stream, g.d);
    hipLaunchKernelGGL(scan_add_kernel, dim3(blocks_for(g.maxCells, 256), R), dim3(256), 0, stream, g.d);
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(g.maxN, 256), R), dim3(256), 0, stream, g.d);
    hipLaunchKernelGGL(rank_kernel, dim3(blocks_for(g.maxN, 256), R), dim3(256), 0, stream, g.d);
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(g.maxN, 256), R), dim3(256), 0, stream, g.d);
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(g.maxN, 256), R), dim3(256), 0, stream, g.d);
    return hipGetLastError();
}

int phase_blocks(int kind, int active, int chunk, int wpb, int max_waves)
{
    int waves = kind == kSphere ? blocks_for(active, chunk) : (active < max_waves ? active : max_waves);
    return blocks_for(waves, wpb);
}

namespace {
// The phase kernels may use every byte of LDS the device gives a workgroup
// (less their static LDS).  A refusal leaves the default limit; the error it
// leaves behind is cleared so that no later launch check reports it.
template <typename K>
void raise_lds(K kernel, size_t bytes)
{
    hipFuncAttributes a{};
    const void* f = reinterpret_cast<const void*>(kernel);
    if (hipFuncGetAttributes(&a, f) == hipSuccess && a.sharedSizeBytes < bytes)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(bytes - a.sharedSizeBytes));
    (void)hipGetLastError();
}
}  // namespace

size_t lds_limit()
{
    static std::once_flag once[64];
    static size_t limit[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
    std::call_once(once[dev], [dev]() {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v < 65536)
            v = 65536;
        limit[dev] = static_cast<size_t>(v);
        raise_lds(phase_sphere_kernel<false, false>, limit[dev]);
        raise_lds(phase_sphere_kernel<false, true>, limit[dev]);
        raise_lds(phase_sphere_kernel<true, false>, limit[dev]);
        raise_lds(phase_sphere_kernel<true, true>, limit[dev]);
        raise_lds(phase_oriented_kernel<kHemisphere, false>, limit[dev]);
        raise_lds(phase_oriented_kernel<kHemisphere, true>, limit[dev]);
        raise_lds(phase_oriented_kernel<kDiscoid, false>, limit[dev]);
        raise_lds(phase_oriented_kernel<kDiscoid, true>, limit[dev]);
        raise_lds(sweep_small_kernel<false, false>, limit[dev]);
        raise_lds(sweep_small_kernel<false, true>, limit[dev]);
        raise_lds(sweep_small_kernel<true, false>, limit[dev]);
        raise_lds(sweep_small_kernel<true, true>, limit[dev]);
    });
    return limit[dev];
}

hipError_t launch_phase(const Group& g, int phase, hipStream_t stream)
{
    dim3 bs(64 * g.wpb), grid(g.nblocks);
    if (g.kind == kSphere) {
        if (g.precision == 1 && g.shell)
            hipLaunchKernelGGL((phase_sphere_kernel<true, true>), grid, bs, g.lds, stream, g.d, g.brep, phase);
        else if (g.precision == 1)
            hipLaunchKernelGGL((phase_sphere_kernel<true, false>), grid, bs, g.lds, stream, g.d, g.brep, phase);
        else if (g.shell)
            hipLaunchKernelGGL((phase_sphere_kernel<false, true>), grid, bs, g.lds, stream, g.d, g.brep, phase);
        else
            hipLaunchKernelGGL((phase_sphere_kernel<false, false>), grid, bs, g.lds, stream, g.d, g.brep, phase);
    } else {
        if (g.kind == kHemisphere && g.precision == 1)
            hipLaunchKernelGGL((phase_oriented_kernel<kHemisphere, true>), grid, bs, g.lds, stream, g.d, g.brep, phase);
        else if (g.kind == kHemisphere)
            hipLaunchKernelGGL((phase_oriented_kernel<kHemisphere, false>), grid, bs, g.lds, stream, g.d, g.brep,
                               phase);
        else if (g.precision == 1)
            hipLaunchKernelGGL((phase_oriented_kernel<kDiscoid, true>), grid, bs, g.lds, stream, g.d, g.brep, phase);
        else
            hipLaunchKernelGGL((phase_oriented_kernel<kDiscoid, false>), grid, bs, g.lds, stream, g.d, g.brep, phase);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_small(const Group& g, int n_sweeps, hipStream_t stream)
{
    dim3 grid(1, g.nrep), bs(64 * kSmallWaves);
    if (g.precision == 1 && g.shell)
        hipLaunchKernelGGL((sweep_small_kernel<true, true>), grid, bs, g.lds_small, stream, g.d, n_sweeps);
    else if (g.precision == 1)
        hipLaunchKernelGGL((sweep_small_kernel<true, false>), grid, bs, g.lds_small, stream, g.d, n_sweeps);
    else if (g.shell)
        hipLaunchKernelGGL((sweep_small_kernel<false, true>), grid, bs, g.lds_small, stream, g.d, n_sweeps);
    else
        hipLaunchKernelGGL((sweep_small_kernel<false, false>), grid, bs, g.lds_small, stream, g.d, n_sweeps);
    return hipGetLastError();
}

hipError_t launch_sweep(const Group& g, hipEvent_t phases_begin, hipEvent_t phases_end, hipStream_t stream)
{
    if (g.small) {
        hipError_t e = phases_begin ? hipEventRecord(phases_begin, stream) : hipSuccess;
        if (e == hipSuccess) e = launch_sweep_small(g, 1, stream);
        if (e == hipSuccess && phases_end) e = hipEventRecord(phases_end, stream);
        return e;
    }
    hipError_t e = launch_build_cells(g, true, stream);
    if (e == hipSuccess && phases_begin) e = hipEventRecord(phases_begin, stream);
    for (int p = 0; p < 8 && e == hipSuccess; ++p) e = launch_phase(g, p, stream);
    if (e == hipSuccess && phases_end) e = hipEventRecord(phases_end, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scatter_back_kernel, dim3(blocks_for(g.maxN, 256), g.nrep), dim3(256), 0, stream, g.d, 1);
    return hipGetLastError();
}

hipError_t launch_clear_counters(const Group& g, hipStream_t stream)
{
    hipLaunchKernelGGL(clear_counters_kernel, dim3(blocks_for(kCounterCopies * kCounterStride, 256), g.nrep),
                       dim3(256), 0, stream, g.d);
    return hipGetLastError();
}

hipError_t launch_overlap_count(const Group& g, hipStream_t stream)
{
    hipLaunchKernelGGL(overlap_count_kernel, dim3(blocks_for(g.maxN, 128), g.nrep), dim3(128), 0, stream, g.d);
    return hipGetLastError();
}

hipError_t launch_reduce_counters(const Group& g, unsigned long long* gather_out, hipStream_t stream)
{
    hipLaunchKernelGGL(reduce_counters_kernel, dim3(1, g.nrep), dim3(64), 0, stream, g.d);
    hipLaunchKernelGGL(gather_counters_kernel, dim3(blocks_for(g.nrep, 64)), dim3(64), 0, stream, g.d, g.nrep,
                       gather_out);
    return hipGetLastError();
}

}  // namespace hpmc

namespace hpmc {

hipError_t launch_gr(const Group& g, const Params& P, const Work& W, int n_bins, double r_max, hipStream_t stream)
{
    hipError_t e = launch_fill_u64(W.obs, n_bins, stream);
    if (e != hipSuccess) return e;
    int k = static_cast<int>(ceil(r_max * P.inv_w));
    hipLaunchKernelGGL(gr_kernel, dim3(blocks_for(P.N, 256), 1), dim3(256), n_bins * sizeof(unsigned long long), stream,
                       g.d, n_bins, r_max, k);
    return hipGetLastError();
}

hipError_t launch_free_volume(const Group& g, int64_t n_probe, uint32_t seq, double scale, int slot,
                              hipStream_t stream)
{
    int64_t blocks = (n_probe + 255) / 256;
    hipLaunchKernelGGL(free_volume_kernel, dim3(static_cast<unsigned>(blocks), 1), dim3(256), 0, stream, g.d, n_probe,
                       seq, scale, slot);
    return hipGetLastError();
}

hipError_t launch_sdf(const Group& g, const Params& P, const Work& W, int n_bins, double x_max, hipStream_t stream)
{
    hipError_t e = launch_fill_u64(W.obs, n_bins, stream);
    if (e != hipSuccess) return e;
    double lim_s = 2.0 * P.S.rcirc / (1.0 - x_max);
    int k = static_cast<int>(ceil(lim_s * P.inv_w));
    hipLaunchKernelGGL(sdf_kernel, dim3(blocks_for(P.N, 128), 1), dim3(128), 0, stream, g.d, n_bins, x_max, k);
    return hipGetLastError();
}

}  // namespace hpmc
