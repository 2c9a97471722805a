/*
 * hpmc.h -- C-ABI of the MI355X implicit-depletant hard-particle Monte Carlo
 * library (libhpmc.so).
 *
 * Method: J. Glaser, A. S. Karas, S. C. Glotzer, "A parallel algorithm for
 * implicit depletant simulations" (arXiv:1508.07077).  A sweep samples the
 * semigrand ensemble exp(z_p V_f - beta H_cc) (Sec. III.A, Eq. gc_ensemble) of N
 * hard colloids in a periodic cubic box with ideal penetrable depletants of
 * diameter d_dep and fugacity z_p:
 *   - trial moves on a shifted checkerboard of cells, 8 colours in random
 *     order, particles confined to their cell (Sec. III.E);
 *   - per move, a Poisson number of depletants uniform in the circumsphere of
 *     the moved colloid (Sec. III.B step 2, Sec. III.C);
 *   - rejection when a depletant free in the old configuration overlaps the
 *     moved colloid (Sec. III.B step 3, Eq. pacc, Fig. 2);
 *   - configurational-bias re-insertion for n_trial > 0 (Sec. III.D,
 *     Eq. pacc_cb, multiple-try reading).
 *
 * Conventions
 *   - Every function returns HPMC_OK (0) or a negative HPMC_E* code; nothing
 *     aborts.  hpmc_last_error() returns a message for the last failure.
 *   - Pointers documented "device" are HIP device allocations owned by the
 *     caller; the library owns no device memory.  "host" pointers are read or
 *     written synchronously.
 *   - All device work is enqueued on the stream given to hpmc_create (NULL =
 *     the library's own blocking stream for the device, see hpmc_create).  A
 *     handle is not thread-safe; handles are independent of each other.
 *   - Positions are SoA [3][n] doubles (x row, y row, z row) in [0, L];
 *     orientations are SoA [4][n] unit quaternions (w, x, y, z rows).
 */
#ifndef HPMC_H
#define HPMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define HPMC_OK 0
#define HPMC_EINVAL (-1)    /* invalid argument */
#define HPMC_EBOX (-2)      /* box holds fewer than 2 cells of width 2 R_circ + d_dep per axis */
#define HPMC_EOVERLAP (-3)  /* the state has overlapping colloids */
#define HPMC_ENOMEM (-4)    /* workspace missing or too small */
#define HPMC_ESTATE (-5)    /* called out of order (shape / state / workspace not set) */
#define HPMC_EHIP (-6)      /* a HIP runtime call failed; see hpmc_last_error */
#define HPMC_ECAPACITY (-7) /* a device-side capacity was exceeded during a sweep */

/* shapes (hpmc_set_shape) */
#define HPMC_SPHERE 0     /* params {d} */
#define HPMC_HEMISPHERE 1 /* params {d}: half of a ball of diameter d; reference point = face centre,
                             dome toward the body +z axis (Sec. V.A) */
#define HPMC_DISCOID 2    /* params {a, r_s}: disk of radius a in the body xy plane swept by a ball of
                             radius r_s */

/* precision (hpmc_create) */
#define HPMC_FP64 0          /* all geometry in FP64 */
#define HPMC_FP32_GUARDED 1  /* FP32 depletant geometry, FP64 recomputation inside a guard band */

/* depletant insertion region V_0 (hpmc_set_insertion) */
#define HPMC_V0_BALL 0   /* the circumsphere B(x', R0) of the new pose, R0 = R_circ + d_dep/2 */
#define HPMC_V0_SHELL 1  /* B(x', R0) less the core B(x', r_in + d_dep/2 - sqrt(3) d_trans) */

/* trial outcomes (hpmc_move_record.reason) */
#define HPMC_ACCEPT 0
#define HPMC_REJ_CELL_EXIT 1
#define HPMC_REJ_OVERLAP 2
#define HPMC_REJ_DEPLETANT 3
#define HPMC_REJ_CB_ZERO 4
#define HPMC_REJ_CB_METROPOLIS 5

/* observables (hpmc_observables) */
#define HPMC_OBS_GR 0
#define HPMC_OBS_FREE_VOLUME 1
#define HPMC_OBS_SDF 2

typedef struct hpmc_sim hpmc_sim;

/* Counters accumulated over one hpmc_sweep call. */
typedef struct hpmc_counters {
    uint64_t trials;              /* trial moves (a particle was selected) */
    uint64_t accepts;
    uint64_t rej_cell_exit;
    uint64_t rej_overlap;
    uint64_t rej_depletant;
    uint64_t rej_cb_zero;
    uint64_t rej_cb_metropolis;
    uint64_t depletants_drawn;    /* sum of N_p over trials that drew depletants */
    uint64_t depletants_resolved; /* depletant checks in serial order up to each decision, + CB insertions */
    uint64_t cb_trials;           /* CB trial insertions performed (serial semantics) */
    uint64_t overlap_checks;      /* narrow-phase colloid-pair tests executed (implementation-specific) */
    uint64_t near_contact;        /* colloid pairs decided within 1e-9 of contact */
    uint64_t fp64_fallbacks;      /* FP64 recomputations of guarded FP32 decisions */
    double phase_kernel_ms;       /* summed device time of the 8 phase launches of every sweep, from HIP
                                     events recorded on the handle's stream around them */
    double sweep_ms;              /* device time from the first to the last kernel of the call */
} hpmc_counters;

/* One record per trial, in cell order: index n_select * (first sorted slot of
 * the cell) + t. */
typedef struct hpmc_move_record {
    uint32_t sweep;        /* low 32 bits of the sweep index */
    uint32_t cell;         /* cell id cx + n (cy + n cz) */
    uint32_t t;            /* round within the cell */
    uint32_t particle;     /* selected particle */
    uint32_t n_depletants; /* Poisson number drawn (0 if the trial ended before) */
    uint32_t resolved;     /* depletant checks resolved in serial order, + CB insertions */
    uint32_t n_blocking;   /* blocking depletants processed */
    uint32_t w_fwd;        /* sum of forward CB weights W'_k */
    uint32_t w_rev;        /* sum of reverse CB weights W_k */
    uint8_t phase;         /* 0..7 */
    uint8_t reason;        /* HPMC_ACCEPT or HPMC_REJ_* */
    uint8_t rotation;      /* 1 if the proposal was a rotation */
    uint8_t near_contact;  /* a colloid pair of this trial was decided within 1e-9 of contact */
} hpmc_move_record;

typedef struct hpmc_obs_params {
    int32_t n_bins;   /* GR and SDF histogram bins */
    int32_t n_fit;    /* SDF: leading bins of the linear extrapolation to zero compression */
    double r_max;     /* GR: upper edge, <= L/2 */
    double x_max;     /* SDF: upper edge of the compression histogram, in (0, 1) */
    int64_t n_probe;  /* FREE_VOLUME and the SDF depletant term: uniform probes */
    uint32_t obs_seq; /* selects the probe stream */
    uint32_t pad;
    double eps;       /* SDF depletant term: relative virtual expansion */
} hpmc_obs_params;

/* Create a handle for n colloids in a cubic periodic box of side box_L.
 * seed and replica_id key the counter-based random streams (Philox4x32-10);
 * precision is HPMC_FP64 or HPMC_FP32_GUARDED; hip_stream is the hipStream_t
 * every call of this handle is enqueued on, or NULL: then the library's own
 * stream for the current device (created on first device work, shared by all
 * such handles, blocking, so ordered with work on the null stream).
 * Allocates host metadata only.  Errors: EINVAL. */
int hpmc_create(hpmc_sim** out, int64_t n, double box_L, uint64_t seed, uint32_t replica_id, int precision,
                void* hip_stream);

/* Release the handle (device buffers stay with the caller). */
void hpmc_destroy(hpmc_sim* sim);

/* Message of the last failure on this handle (valid until the next call). */
const char* hpmc_last_error(const hpmc_sim* sim);

/* Colloid shape (Sec. V: spheres, hemispheres, discoids).  params as listed at
 * HPMC_SPHERE / HPMC_HEMISPHERE / HPMC_DISCOID.  Errors: EINVAL, EBOX. */
int hpmc_set_shape(hpmc_sim* sim, int kind, const double* params, int nparams);

/* Depletants (Sec. III.A, III.D): z_p is the depletant fugacity (reservoir
 * number density, phi_p^r = (pi/6) d_dep^3 z_p); z_p = 0 disables them.
 * n_trial = 0 is the plain scheme of Sec. III.B/C; n_trial in 1..255 enables
 * configurational bias.  Errors: EINVAL, EBOX. */
int hpmc_set_fugacity(hpmc_sim* sim, double z_p, double d_dep, int n_trial);

/* Proposals (Sec. III.B step 1; symmetric): translation uniform in the cube
 * [-d_trans, d_trans]^3 or, with probability p_rot (oriented shapes only),
 * rotation q' = (q + a_rot v)/|q + a_rot v| with v uniform in the unit 4-ball.
 * n_select trials per cell member and sweep.  Errors: EINVAL. */
int hpmc_set_moves(hpmc_sim* sim, double d_trans, double a_rot, double p_rot, int n_select);

/* Depletant insertion region (Sec. III.C: V_0 may be any region that holds
 * every depletant able to block the move).  HPMC_V0_BALL (default): the
 * circumsphere of the new pose.  HPMC_V0_SHELL: that ball less a core ball of
 * radius r_in + d_dep/2 - sqrt(3) d_trans (clamped at 0), r_in being the
 * largest ball about the reference point inside the shape (sphere d/2,
 * hemisphere 0, swept disk r_s); a depletant in the core overlaps the old pose
 * for every translation of at most sqrt(3) d_trans and so is never free.  The
 * shell mode draws its depletants from its own random stream (one candidate
 * per Philox block), so its trajectories differ from the ball mode's while
 * sampling the same ensemble.  Errors: EINVAL (unknown region). */
int hpmc_set_insertion(hpmc_sim* sim, int region);

/* Bytes of device workspace this handle needs with the current shape,
 * fugacity, moves and trace setting. */
int hpmc_workspace_bytes(const hpmc_sim* sim, size_t* bytes);

/* Hand the library a device workspace of at least hpmc_workspace_bytes bytes
 * (kept until replaced; the caller frees it after hpmc_destroy).  Errors:
 * ENOMEM if too small, EINVAL if NULL. */
int hpmc_set_workspace(hpmc_sim* sim, void* dev_ptr, size_t bytes);

/* Borrow the caller's device state: pos_soa [3][n] doubles, quat_soa [4][n]
 * doubles (required for oriented shapes, ignored for spheres), both kept for
 * the lifetime of the handle; sweeps update them in place.  sweep_index sets
 * the sweep counter of the random streams.  Synchronises the stream and checks
 * that no two colloids overlap (in the caller's workspace, or, when none is
 * set, in the static scratch of hpmc_sweep_static).  Errors: EINVAL, ESTATE,
 * EOVERLAP, EHIP, ENOMEM (no workspace and more than the static scratch). */
int hpmc_set_state(hpmc_sim* sim, double* pos_soa, double* quat_soa, uint64_t sweep_index);

/* Current sweep index (the state itself is in the caller's buffers).
 * Synchronises the handle's stream, so the state buffers hold the result of
 * every sweep enqueued so far.  Errors: EINVAL, ESTATE, EHIP, ECAPACITY (a
 * sweep since the last report skipped a cell whose stencil exceeded its
 * capacity; reported once, by this or the next synchronising call). */
int hpmc_get_state(hpmc_sim* sim, uint64_t* sweep_index);

/* Record one hpmc_move_record per trial of the most recent sweep (parity
 * mode).  Enabling it grows hpmc_workspace_bytes; device calls return ENOMEM
 * until a large enough workspace is set.  Errors: EINVAL. */
int hpmc_set_trace(hpmc_sim* sim, int enable);

/* Run n_sweeps sweeps, enqueued on the stream.  If out is non-NULL the call
 * synchronises and fills the counters summed over these sweeps (host).
 * Errors: ESTATE, ENOMEM, EHIP, ECAPACITY.  ECAPACITY means that a cell's
 * stencil exceeded the packing bound its lists are sized by, which disjoint
 * bodies cannot reach; its trials were skipped.  The device flag behind it is
 * sticky: it is reported once, by the first synchronising call after the
 * sweep that raised it (this call with out non-NULL, hpmc_get_state,
 * hpmc_observables, hpmc_trace), and cleared by that report. */
int hpmc_sweep(hpmc_sim* sim, int n_sweeps, hpmc_counters* out);

/* Allocation-free variant of hpmc_sweep, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  It runs the same kernels as hpmc_sweep, with the
 * handle's workspace laid out in the library's static scratch instead of the
 * caller's buffer: a file-scope device array of 64 MiB (one copy per device,
 * held until the process ends) on the current device.  The call allocates
 * nothing; the caller still owns the state (hpmc_set_state; without a
 * workspace, its one-time hard-core check also runs in the static scratch).
 * Needs shape and state; tracing off.  Each call writes the descriptor,
 * Poisson table, sweep counter and cleared flags into the scratch before its
 * sweeps, so a call does not depend on what an earlier one left there; calls
 * on one device share the one array, so calls that overlap on a device (two
 * streams, two threads) race and must be serialised by the caller.  The
 * handle's own workspace, if set, is not touched; its sweep counter is brought
 * up to date by the next call that uses it.  out: as for hpmc_sweep, except
 * that phase_kernel_ms and sweep_ms are 0 (no events are recorded).  Errors:
 * EINVAL, ESTATE, ENOMEM (the handle needs more than 64 MiB of scratch; about
 * 76 bytes per sphere, 108 per oriented body, plus 8 per cell), EHIP,
 * ECAPACITY (reported only when out is non-NULL). */
int hpmc_sweep_static(hpmc_sim* sim, int n_sweeps, hpmc_counters* out);

/* Launch shape of the phase kernels.  It never changes a result (every
 * random draw is keyed by sweep, cell, round and purpose, not by thread), only
 * the speed.  Zero fields mean the default. */
typedef struct hpmc_tuning {
    int32_t cells_per_wave;  /* spheres: active cells per wave, 1..64 (default 8) */
    int32_t waves_per_block; /* 1, 2 or 4 (default 1 for spheres, 4 for oriented shapes; lowered to what the LDS holds) */
    int32_t max_waves;       /* oriented shapes: waves of the grid-stride launch, >= 1 (default 8192) */
    int32_t candidates;      /* hpmc_autotune: configurations timed */
    double best_ms;          /* hpmc_autotune: phase-kernel ms per sweep of the chosen shape */
    double default_ms;       /* hpmc_autotune: the same for the default shape */
} hpmc_tuning;

/* Set the launch shape explicitly (the last three fields are ignored).
 * Batched sweeps use the shape of the most crowded handle of each group
 * (hpmc_autotune_batch gives a group's handles one shape).
 * Errors: EINVAL (a field out of range). */
int hpmc_set_tuning(hpmc_sim* sim, const hpmc_tuning* tuning);

/* Autotuner: time candidate launch shapes (spheres: cells per wave in
 * {4, 6, 8, 10, 12, 16, 32, 64} x waves per block in {1, 2, 4}; oriented shapes: waves
 * per block x wave count in {1024 .. 32768}) on a copy of the current state,
 * `sweeps` timed sweeps each after one untimed, keep the fastest, and report
 * it in *out (may be NULL).  The handle's state and sweep index are left as
 * they were.  scratch: device memory of at least 8 N (3 + 4 if oriented)
 * bytes, used only during the call.  Synchronises.  Errors: EINVAL, ESTATE,
 * ENOMEM (scratch too small), EHIP, ECAPACITY. */
int hpmc_autotune(hpmc_sim* sim, void* scratch, size_t scratch_bytes, int sweeps, hpmc_tuning* out);

/* Device scratch needed by hpmc_sweep_batch for n_sims handles. */
int hpmc_batch_workspace_bytes(int n_sims, size_t* bytes);

/* Run n_sweeps sweeps of n_sims independent handles (replicas of uneven size,
 * density and fugacity; growth path of the paper's parallel scheme,
 * Sec. III.E) in shared launches.  Replicas of one shape kind, precision,
 * insertion region and box class form a launch group (groups run on up to
 * four streams); a group's cell-list kernels index its replicas by the grid's
 * second dimension, and each of its phase launches holds only blocks with
 * work, every replica's blocks one after another (at most 1024 per replica;
 * past that an oriented replica's waves take several cells in turn and a
 * sphere replica takes larger chunks of cells, up to 64 per wave, else
 * ECAPACITY).  Each handle keeps its own state, workspace and random streams,
 * so every replica's trajectory is identical to what hpmc_sweep gives it
 * alone.  All handles must be ready
 * (shape, workspace, state) and use the stream of sims[0] (EINVAL
 * otherwise); tracing must be off.  batch_ws: device scratch of hpmc_batch_workspace_bytes(n_sims); the
 * descriptors are copied into it on the stream from pinned host staging
 * buffers of sims[0], so the call does not wait for the device unless out is
 * given.  out: NULL or n_sims counter records (synchronises); their
 * sweep_ms is the device time of the whole batched call, the same in every
 * record, and phase_kernel_ms is 0.  Errors: EINVAL,
 * ESTATE, ENOMEM, EHIP, ECAPACITY (as for hpmc_sweep, per replica). */
int hpmc_sweep_batch(hpmc_sim* const* sims, int n_sims, void* batch_ws, size_t bytes, int n_sweeps,
                     hpmc_counters* out);

/* Autotuner of a batch (run-time tuning of launch shapes, App. A, applied to
 * the batched sweeps of Sec. III.E): for each launch group of
 * hpmc_sweep_batch (replicas of one shape kind, precision and insertion
 * region; small sphere boxes, which sweep in one workgroup each, and oriented
 * boxes of two cells per axis apart), time the candidate shapes of
 * hpmc_autotune with that group's members swept together, and give every
 * member of the group the fastest.  The sweeps run on copies of the states:
 * states, sweep indices and traces are as before the call, and trajectories
 * do not depend on the shape.  Same conditions as hpmc_sweep_batch (ready
 * handles, tracing off, the stream of sims[0], batch_ws of
 * hpmc_batch_workspace_bytes(n_sims)); each handle at most once.
 * scratch: device memory for every member's state, members in order, each
 * N*24 bytes (+ N*32 for oriented shapes) rounded up to 256 bytes.
 * sweeps: 1..64 timed per candidate (after one untimed).  out: NULL or n_sims
 * records (best_ms / default_ms: device ms per batched sweep of the member's
 * group; candidates is 0 for a small sphere box).  Synchronous.
 * Errors: EINVAL, ESTATE, ENOMEM, EHIP, ECAPACITY; on error every handle keeps
 * its state and its previous launch shape. */
int hpmc_autotune_batch(hpmc_sim* const* sims, int n_sims, void* batch_ws, size_t ws_bytes, void* scratch,
                        size_t scratch_bytes, int sweeps, hpmc_tuning* out);

/* The Poisson count of one depletant chunk (Sec. III.B, step 2: the number of
 * depletants in V_0 is a sum of chunk counts) that the sweeps draw for the
 * 52-bit uniform u in (0, 1), evaluated on the host from the table the device
 * uses: the smallest k with P(N <= k) >= u for the chunk mean of the current
 * fugacity, or 1023 when the running sum of the table stays below u.  For
 * inspection and tests; no device work.  Errors: EINVAL (u outside (0, 1)),
 * ESTATE (no shape set yet, so no table). */
int hpmc_poisson_draw(const hpmc_sim* sim, double u, int32_t* k);

/* Observables of the current state (host out, synchronous):
 *   HPMC_OBS_GR: out[0..n_bins) = g(r) of reference-point distances on
 *     [0, r_max), minimum image;
 *   HPMC_OBS_FREE_VOLUME: out[0] = free-volume fraction alpha (probes that
 *     overlap no colloid), out[1] = phi_p = phi_p^r alpha (Sec. IV.A),
 *     out[2] = number of free probes;
 *   HPMC_OBS_SDF: out[0] = beta P total, out[1] = rho (1 + s(0+)/6),
 *     out[2] = z_p dV_f/dV (virtual expansion of the probe set), out[3] = s(0+),
 *     out[4..4+n_bins) = s(x) histogram of the per-particle minimum compression.
 * Errors: EINVAL, ESTATE, ENOMEM, EHIP, ECAPACITY (a pending capacity flag of
 * an earlier sweep, see hpmc_sweep). */
int hpmc_observables(hpmc_sim* sim, int kind, const hpmc_obs_params* params, double* out, int64_t out_len);

/* Copy the trace of the most recent sweep (host buf, cap records); requires
 * hpmc_set_trace(sim, 1) before that sweep.  Errors: ESTATE, EHIP, ECAPACITY
 * (a pending capacity flag, see hpmc_sweep). */
int hpmc_trace(hpmc_sim* sim, hpmc_move_record* buf, int64_t cap, int64_t* n_written);

#ifdef __cplusplus
}
#endif
#endif
