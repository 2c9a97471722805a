// kernels.hpp -- launch interface between the C-ABI host code and the HIP
// kernels of one implicit-depletant sweep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.hpp"

namespace hpmc {

// Poisson chunk counts: the inverse CDF F[k] = P(N <= k) of the chunk mean,
// k < kPoissonK, whose last entry is a sentinel (a draw returns 0 .. K - 1).
// Only k_min .. k_end can be returned for a 52-bit uniform u in
// [2^-53, 1 - 2^-53]: F[k] < 2^-53 below k_min, and k_end is the first entry
// >= 1 - 2^-53 or the start of the plateau where the running sum stops
// growing (past it only the sentinel is reached).  The device keeps these
// entries (at most 263 for chunk means up to 256) and a sentinel that stands
// for K - 1: the same doubles, so the same draws, in a third of the LDS.
constexpr int kPoissonK = 1024;
constexpr int kPoissonC = 272;       // compact table capacity, sentinel included
constexpr int kGuide = 256;          // guide table: first compact index with F >= i / 256
constexpr int kTableLds = kPoissonC * 8 + kGuide * 4;

// The chunk count of a 52-bit uniform u in (0, 1): the smallest k with
// F[k] >= u, scanned from the guide entry G[floor(256 u)] of the compact table
// (pk_n entries from k = pk_min, then the sentinel, which stands for K - 1).
template <typename FP, typename GP>
__host__ __device__ inline int poisson_compact_draw(FP F, GP G, double u, int pk_min, int pk_n)
{
    int k = G[static_cast<int>(u * 256.0)];
    while (F[k] < u) ++k;
    return k < pk_n ? pk_min + k : kPoissonK - 1;
}
constexpr int kCounterCopies = 256;  // spread copies of the counters (atomic contention)
constexpr int kNumCounters = 13;
constexpr int kCounterStride = 16;

enum CounterIdx : int {
    cTrials = 0,
    cAccepts,
    cRejCellExit,
    cRejOverlap,
    cRejDepletant,
    cRejCbZero,
    cRejCbMetro,
    cDrawn,
    cResolved,
    cCbTrials,
    cOverlapChecks,
    cNearContact,
    cFp64Fallbacks,
};

enum Flags : int { kFlagListOverflow = 1 };

// constants of one state point, passed by value to every kernel
struct Params {
    Shape S;
    int N;
    int n;      // cells per axis (even)
    int h;      // n / 2
    int ncells; // n^3
    int n_select;
    int n_trial;
    int n_chunks;
    int has_dep;
    int trace;
    int precision;
    uint32_t key0, key1;
    uint32_t sweep;
    double L, halfL, w, inv_w;
    double d_trans, a_rot, p_rot;
    double s_ball;  // R0 * 2^-21
    int shell;      // depletants in the shell r_inner <= |e| < R0 instead of the ball
    double r_inner, span;  // span = R0 - r_inner
    float g_lo, g_hi;      // FP32 guard band (eps = 1e-5 sigma): spheres (R0 -+ eps)^2, oriented shapes thr -+ eps, rounded outward
    // per-wave LDS layout of the phase kernel
    int list_cap, geo_cap;
    int wave_lds;       // bytes per wave
    int off_rec_a, off_rec_b;  // spheres: staged (x, y) and (z, index) pairs within a stage buffer
    int off_geo;        // oriented shapes: the geometry cache
    int off_cnt;        // spheres: the wave's counters (the two stage buffers come before it)
    // oriented shapes, per trial: stencil entries whose circumsphere meets the
    // proposed pose's (close list) and entries a depletant or CB trial can reach
    int close_cap, reach_cap, off_close, off_reach;
    double reach_sq;    // (R0 + r_circ + r_dep + sqrt(3) d_trans)^2 plus a margin (spheres: the CB reach mask)
    int waves_per_block;
    int chunk;          // spheres: active cells per wave (1..64)
    int active_cells;   // h^3
    // the phase launch: this replica's blocks are blk0 .. blk0 + nblk - 1 of the grid
    int blk0, nblk;
    // compact Poisson table: entry i < pk_n is F[pk_min + i]; entry pk_n is the sentinel
    int pk_min, pk_n;
};

// device workspace carved from the caller's buffer
struct Work {
    int* cell_count;   // ncells
    int* cell_start;   // ncells + 1
    int* scan_tmp;     // scan block totals
    int* pcell;        // N
    int* prank;        // N
    int* order;        // N: sorted slot -> particle
    double4* rpos;     // N: cell-ordered (x, y, z, particle index)
    double4* rquat;    // N: cell-ordered (w, x, y, z) (oriented shapes)
    double* F;         // the compact Poisson table (kPoissonC doubles), then kGuide ints
    double* grid;      // shift g[3]
    int* perm;         // colour order [8]
    unsigned long long* counters;  // kCounterCopies x kCounterStride
    void* trace;       // hpmc_move_record[N * n_select] or null
    int* flags;
    unsigned long long* obs;  // observables scratch
    uint32_t* sweep_dev;      // sweep index of the random streams, advanced on the device
    double* pos;              // caller's state [3][N]
    double* quat;             // caller's orientations [4][N] or null
};

// per-replica descriptor in device memory
struct Desc {
    Params P;
    Work W;
};

// host-side launch shape of a group of replicas of one shape kind
struct Group {
    const Desc* d;  // device array of nrep descriptors
    const int* brep;  // phase launches: replica of each block (null: one replica owns every block)
    int nblocks;      // phase launches: blocks of the grid
    int nrep;
    int kind;
    int precision;  // 0 FP64, 1 FP32 depletant tests with the FP64 guard band
    int shell;      // insertion region: 0 ball, 1 shell (common to the group)
    int maxN, maxCells, maxActive;
    int wpb;        // waves per block of the phase kernel (common to the group)
    int chunk;      // spheres: active cells per wave (common to the group)
    int max_waves;  // oriented shapes: waves of the grid-stride phase launch
    size_t lds;     // dynamic LDS bytes of the phase kernel (common to the group)
    int small;      // spheres in small boxes: one workgroup sweeps each replica (sweep_small_kernel)
    size_t lds_small;
};

// host-side launchers (enqueue on `stream`)
hipError_t launch_fill_int(int* p, int n, int value, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long* p, int n, hipStream_t stream);
hipError_t launch_build_cells(const Group& g, bool with_grid, hipStream_t stream);
hipError_t launch_phase(const Group& g, int phase, hipStream_t stream);
hipError_t launch_sweep(const Group& g, hipEvent_t phases_begin, hipEvent_t phases_end, hipStream_t stream);
hipError_t launch_sweep_small(const Group& g, int n_sweeps, hipStream_t stream);
hipError_t launch_clear_counters(const Group& g, hipStream_t stream);
hipError_t launch_overlap_count(const Group& g, hipStream_t stream);
hipError_t launch_reduce_counters(const Group& g, unsigned long long* gather_out, hipStream_t stream);
hipError_t launch_gr(const Group& g, const Params& P, const Work& W, int n_bins, double r_max, hipStream_t stream);
hipError_t launch_free_volume(const Group& g, int64_t n_probe, uint32_t seq, double scale, int slot,
                              hipStream_t stream);
hipError_t launch_sdf(const Group& g, const Params& P, const Work& W, int n_bins, double x_max, hipStream_t stream);
// largest dynamic LDS of one workgroup on the current device (bytes); raises
// the phase kernels' LDS limit to it on first use
size_t lds_limit();
// phase blocks one replica needs: spheres, chunks of `chunk` active cells per
// wave; oriented shapes, one wave per active cell up to max_waves
int phase_blocks(int kind, int active, int chunk, int wpb, int max_waves);

constexpr int kChunk = 8;      // default active cells per wave of the sphere phase kernel
constexpr int kSphereWpb = 1;  // default waves per workgroup of the sphere phase kernel: a wave's
                               // slot and LDS are freed as soon as it ends
constexpr int kMaxReplicaBlocks = 1024;  // phase blocks of one replica in a batched launch (waves loop over more)
constexpr int kMaxWaves = 256 * 32;  // default wave count of the oriented phase launch
constexpr int kSmallMaxActive = 32;  // spheres with at most this many active cells per phase and
constexpr int kSmallMaxN = 8192;     // at most this many particles sweep in one workgroup
constexpr int kSmallWaves = 8;       // waves of that workgroup
constexpr size_t kSmallStaticLds = 256;  // that workgroup's static LDS (scan partials), rounded up

}  // namespace hpmc
