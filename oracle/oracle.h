/*
 * oracle.h -- plain, single-threaded FP64 CPU oracle of the implicit-depletant
 * hard-particle Monte Carlo trial move (Glaser, Karas & Glotzer, "A parallel
 * algorithm for implicit depletant simulations", arXiv:1508.07077).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library: both follow the
 * same written determinism contract (random-number stream layout, arithmetic
 * order), each in its own code.
 *
 * What it computes, by paper passage:
 *   - target distribution exp(z_p V_f - beta H_cc)            Sec. III.A, Eq. (gc_ensemble)
 *   - trial move + Poisson depletants + reject if a depletant
 *     that was free in M overlaps M'                           Sec. III.B, Eqs. (move_gen), (pacc)
 *   - sampling region V_0 = circumsphere of the new pose, or
 *     that ball less a core inside the old pose (shell)       Sec. III.C, Eq. (transition_prob_final)
 *   - configurational-bias re-insertion                        Sec. III.D, Eq. (pacc_cb), Fig. 3
 *   - checkerboard cells, random colour order, random shift   Sec. III.E
 */
#ifndef HPMC_ORACLE_H
#define HPMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_SPHERE = 0,     /* params {d}                                   */
    ORC_HEMISPHERE = 1, /* params {d}; reference point = face centre    */
    ORC_DISCOID = 2     /* params {a, r_s}: disk of radius a swept by a ball of radius r_s */
};

enum {
    ORC_ACCEPT = 0,
    ORC_REJ_CELL_EXIT = 1,
    ORC_REJ_OVERLAP = 2,
    ORC_REJ_DEPLETANT = 3,
    ORC_REJ_CB_ZERO = 4,
    ORC_REJ_CB_METROPOLIS = 5
};

enum { ORC_OBS_GR = 0, ORC_OBS_FREE_VOLUME = 1, ORC_OBS_SDF = 2 };

/* depletant insertion region V_0 (Sec. III.C) */
enum {
    ORC_V0_BALL = 0,  /* circumsphere B(x', R0) of the new pose */
    ORC_V0_SHELL = 1  /* B(x', R0) minus B(x', r_in + r_dep - sqrt(3) d_trans) */
};

/* One record per trial, laid out exactly like the GPU library's record. */
typedef struct orc_record {
    uint32_t sweep;
    uint32_t cell;
    uint32_t t;
    uint32_t particle;
    uint32_t n_depletants;
    uint32_t resolved;
    uint32_t n_blocking;
    uint32_t w_fwd;      /* sum of forward CB weights W'_k over processed blocking depletants */
    uint32_t w_rev;      /* sum of reverse CB weights W_k */
    uint8_t phase;
    uint8_t reason;
    uint8_t rotation;
    uint8_t near_contact;
} orc_record;

typedef struct orc_counters {
    uint64_t trials;
    uint64_t accepts;
    uint64_t rej_cell_exit;
    uint64_t rej_overlap;
    uint64_t rej_depletant;
    uint64_t rej_cb_zero;
    uint64_t rej_cb_metropolis;
    uint64_t depletants_drawn;
    uint64_t depletants_resolved;
    uint64_t cb_trials;
    uint64_t overlap_checks;
    uint64_t near_contact;
    uint64_t fp64_fallbacks;
} orc_counters;

typedef struct orc_obs_params {
    int32_t n_bins;       /* GR, SDF histogram bins */
    int32_t n_fit;        /* SDF: bins used for the linear extrapolation to x = 0 */
    double r_max;         /* GR upper edge */
    double x_max;         /* SDF histogram upper edge (scale factor) */
    int64_t n_probe;      /* FREE_VOLUME, SDF depletant term: number of probes */
    uint32_t obs_seq;     /* random-stream selector for probes */
    uint32_t pad;
    double eps;           /* SDF depletant term: relative virtual expansion */
} orc_obs_params;

typedef struct orc_sim orc_sim;

/* lifecycle and parameters (mirrors the GPU C-ABI; all buffers are host) */
orc_sim* orc_create(int64_t n, double box_L, uint64_t seed, uint32_t replica_id);
void orc_destroy(orc_sim* s);
const char* orc_last_error(const orc_sim* s);
int orc_set_shape(orc_sim* s, int kind, const double* params, int nparams);
int orc_set_fugacity(orc_sim* s, double z_p, double d_dep, int n_trial);
int orc_set_moves(orc_sim* s, double d_trans, double a_rot, double p_rot, int n_select);
int orc_set_insertion(orc_sim* s, int region);
int orc_set_state(orc_sim* s, const double* pos_soa, const double* quat_soa, uint64_t sweep_index);
int orc_get_state(const orc_sim* s, double* pos_soa, double* quat_soa, uint64_t* sweep_index);
int orc_set_trace(orc_sim* s, int enable);
/* OpenMP threads over the active cells of a phase (default 1: the serial
 * loop).  The cells of a phase are independent, so the result is that of one
 * thread, bit for bit. */
int orc_set_threads(orc_sim* s, int threads);
int orc_sweep(orc_sim* s, int n_sweeps, orc_counters* out);
int orc_sweep_cone(orc_sim* s, int64_t target_cell, orc_counters* out);
int orc_trace(const orc_sim* s, orc_record* buf, int64_t cap, int64_t* n_written);
int orc_observables(orc_sim* s, int kind, const orc_obs_params* p, double* out, int64_t out_len);
int orc_count_overlaps(orc_sim* s, int64_t* n_pairs);
int orc_derived(const orc_sim* s, double* out, int out_len);

/* One trial with an explicit proposal (x', q') for particle j and explicit
 * stream coordinates (sweep, cell, t).  The stencil is every other particle.
 * Does not commit; returns the reason code, fills *rec if non-NULL. */
int orc_try_move(orc_sim* s, int64_t j, const double* xnew, const double* qnew,
                 uint32_t sweep, uint32_t cell, uint32_t t, orc_record* rec);

int orc_try_move_many(orc_sim* s, int64_t j, const double* xnew, const double* qnew, uint32_t sweep0,
                      int64_t count, uint8_t* reasons, uint32_t* n_depletants);

/* building blocks, exported for the pins */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int orc_poisson_table(double lambda_c, double* F, int K);
int orc_poisson_draw(const double* F, int K, double u);
int orc_ball_candidate(uint32_t wa, uint32_t wb, int32_t m[3]);
int orc_shell_candidate(const uint32_t w[4], double r_i, double span, double R0sq, double e[3]);
int orc_depletant_overlap(int kind, const double* params, double r_dep,
                          const double* v_world, const double* quat);
int orc_pair_overlap(int kind, const double* params, const double* d_world,
                     const double* qa, const double* qb, int* near_contact);

#ifdef __cplusplus
}
#endif
#endif
