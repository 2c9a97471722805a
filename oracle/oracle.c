/*
 * oracle.c -- plain FP64 CPU oracle of the implicit-depletant hard-particle
 * Monte Carlo sweep (Glaser, Karas & Glotzer, arXiv:1508.07077).  Single
 * threaded unless orc_set_threads asks for OpenMP threads over the active
 * cells of a phase (the same result, bit for bit).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no code
 * with the HIP library.  Both sides follow the same written determinism
 * contract (stream layout of the counter-based generator, order of every
 * floating-point operation that decides an outcome), each in its own code, so
 * that the two reach the same accept/reject decision for every trial.
 *
 * The steps below follow the paper in its order and notation:
 *   Sec. III.A  ensemble weight exp(z_p V_f - beta H_cc)           (Eq. gc_ensemble)
 *   Sec. III.B  move, Poisson depletant number, reject on overlap  (Eqs. move_gen, pacc; Fig. 2)
 *   Sec. III.C  V_0 = circumsphere around the new pose, or that   (Eq. transition_prob_final)
 *               ball less a core ball inside the old pose (shell)
 *   Sec. III.D  configurational-bias re-insertion                  (Eq. pacc_cb; Fig. 3)
 *   Sec. III.E  checkerboard: inactive layer of width d_c + d_dep,
 *               particles may not leave their cell, random colour
 *               order, randomly shifted grid
 * Where the paper is silent (random numbers, Poisson sampler, point sampler,
 * overlap algorithm, sweep definition) the contract fixes a reading; each is
 * listed with its reason in the design notes.
 *
 * Parity status per function:
 *   philox, conversions, Poisson table, ball sampler     pinned (known-answer vectors, chi-square)
 *   depletant/shape predicates                            pinned (dense point clouds)
 *   convex pair test (GJK)                                pinned (brute force on random pairs)
 *   trial move, CB weights, sweep                         pinned (closed forms P1/P2/P3/P6, explicit depletants)
 *   shell insertion region and its sampler                pinned (radial CDF, isotropy, closed forms,
 *                                                         forward/backward ratio, ball/shell invariance)
 *   g(r), free volume                                     pinned (brute force / analytic limits)
 *   SDF pressure                                          pinned only in its limits (z_p = 0 spheres vs
 *                                                         Carnahan-Starling, dilute limit); otherwise
 *                                                         parity unpinned
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Counter-based generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror,
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).               */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* stream purposes: third counter word is (t << 8) | purpose */
enum {
    P_GRID = 1,
    P_SELECT = 2,
    P_TRANS = 3,
    P_ROT = 4,
    P_POISSON = 5,
    P_DEPL = 6,
    P_CB_FWD = 7,
    P_CB_REV = 8,
    P_ACCEPT = 9,
    P_DEPL_SHELL = 10,
    P_OBS_FV = 16
};
#define NO_CELL 0xFFFFFFFFu

typedef struct {
    uint32_t key[2];
    uint32_t sweep;
    uint32_t cell;
    uint32_t t;
} stream_t;

static void draw(const stream_t* st, uint32_t purpose, uint32_t index, uint32_t w[4])
{
    uint32_t ctr[4] = {st->sweep, st->cell, (st->t << 8) | purpose, index};
    orc_philox4x32_10(ctr, st->key, w);
}

/* u32 -> (0,1): (w + 1/2) 2^-32, exact */
static double u01(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* two words -> 52-bit uniform in (0,1): (k + 1/2) 2^-52, exact */
static double u52(uint32_t w0, uint32_t w1)
{
    uint64_t k = ((uint64_t)w1 << 20) | (uint64_t)(w0 >> 12);
    return ((double)k + 0.5) * 0x1p-52;
}

/* u32 -> symmetric (-1,1): (2w + 1 - 2^32) 2^-32, exact */
static double sym01(uint32_t w)
{
    double odd = (double)(2.0 * (double)w + 1.0) - 4294967296.0;
    return odd * 0x1p-32;
}

/* multiply-shift choice in [0, n) */
static uint32_t pick(uint32_t w, uint32_t n) { return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32); }

/* Uniform point in the open unit ball on the grid of odd multiples of 2^-21:
 * 63 bits of (wa, wb) give three 21-bit fields f_i; m_i = 2 f_i + 1 - 2^21;
 * accepted iff m0^2 + m1^2 + m2^2 < 2^42 (exact integer test). */
int orc_ball_candidate(uint32_t wa, uint32_t wb, int32_t m[3])
{
    uint64_t v = (uint64_t)wa | ((uint64_t)wb << 32);
    int64_t s = 0;
    for (int i = 0; i < 3; ++i) {
        int64_t f = (int64_t)((v >> (21 * i)) & 0x1FFFFFu);
        int64_t mi = 2 * f + 1 - (1 << 21);
        m[i] = (int32_t)mi;
        s += mi * mi;
    }
    return s < ((int64_t)1 << 42);
}

/* Uniform point in the spherical shell r_i <= |e| < R0 (Sec. III.C: any
 * region V_0 that holds every depletant that can block the move may be used;
 * the inner ball lies inside the old pose for every allowed move, so a
 * depletant there is never free in M).  One candidate per Philox block:
 * direction by Marsaglia's method (1972) from two symmetric uniforms, radius
 * uniform in [r_i, R0) accepted with probability r^2 / R0^2, so the density
 * is proportional to r^2 on the shell.  IEEE + - * sqrt only, in this order. */
int orc_shell_candidate(const uint32_t w[4], double r_i, double span, double R0sq, double e[3])
{
    double x1 = sym01(w[0]), x2 = sym01(w[1]);
    double s = x1 * x1 + x2 * x2;
    if (!(s < 1.0)) return 0;
    double r = r_i + span * u01(w[2]);
    if (!(u01(w[3]) * R0sq < r * r)) return 0;
    double h = 2.0 * sqrt(1.0 - s);
    e[0] = r * (x1 * h);
    e[1] = r * (x2 * h);
    e[2] = r * (1.0 - 2.0 * s);
    return 1;
}

/* k-th accepted candidate of a ball stream; candidates are taken in the order
 * (block 0: words 0,1), (block 0: words 2,3), (block 1: words 0,1), ... */
typedef struct {
    const stream_t* st;
    uint32_t purpose;
    uint32_t index_base;
    uint32_t block;
    int half;
    uint32_t w[4];
    int have;
} ball_stream_t;

static void ball_stream_init(ball_stream_t* b, const stream_t* st, uint32_t purpose, uint32_t index_base)
{
    b->st = st;
    b->purpose = purpose;
    b->index_base = index_base;
    b->block = 0;
    b->half = 0;
    b->have = 0;
}

/* next accepted candidate; returns 0 only if max_blocks blocks were spent */
static int ball_stream_next(ball_stream_t* b, int32_t m[3], uint32_t max_blocks)
{
    for (;;) {
        if (!b->have) {
            if (b->block >= max_blocks) return 0;
            draw(b->st, b->purpose, b->index_base + b->block, b->w);
            b->have = 1;
            b->half = 0;
        }
        int ok = orc_ball_candidate(b->w[2 * b->half], b->w[2 * b->half + 1], m);
        if (b->half == 0) {
            b->half = 1;
        } else {
            b->have = 0;
            b->block += 1;
        }
        if (ok) return 1;
    }
}

/* ------------------------------------------------------------------------ */
/* Poisson number of depletants (Sec. III.B, step 2): inverse-CDF table.      */
/* F[k] = P(N <= k) by forward recursion; F[K-1] = 2 is a sentinel.          */
/* ------------------------------------------------------------------------ */
#define POISSON_K 1024
#define POISSON_CHUNK 256.0

int orc_poisson_table(double lambda_c, double* F, int K)
{
    if (K < 2) return -1;
    double P = exp(-lambda_c);
    F[0] = P;
    for (int k = 1; k < K - 1; ++k) {
        P = P * (lambda_c / (double)k);
        F[k] = F[k - 1] + P;
    }
    F[K - 1] = 2.0;
    return 0;
}

/* smallest k with F[k] >= u, by plain linear scan */
int orc_poisson_draw(const double* F, int K, double u)
{
    int k = 0;
    while (k < K - 1 && F[k] < u) ++k;
    return k;
}

/* ------------------------------------------------------------------------ */
/* Shapes                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind;
    double d;     /* sphere / hemisphere diameter */
    double a;     /* hemisphere radius d/2; discoid disk radius */
    double rs;    /* discoid sweep radius */
    double rcirc; /* circumradius about the reference point */
    double rin;   /* radius of the largest ball about the reference point inside the shape */
    double vol;
    int oriented;
} shape_t;

static int shape_setup(shape_t* sh, int kind, const double* p, int np)
{
    memset(sh, 0, sizeof(*sh));
    sh->kind = kind;
    if (kind == ORC_SPHERE) {
        if (np < 1 || !(p[0] > 0.0)) return -1;
        sh->d = p[0];
        sh->a = 0.5 * p[0];
        sh->rcirc = 0.5 * p[0];
        sh->rin = 0.5 * p[0];
        sh->vol = M_PI * p[0] * p[0] * p[0] / 6.0;
        sh->oriented = 0;
    } else if (kind == ORC_HEMISPHERE) {
        if (np < 1 || !(p[0] > 0.0)) return -1;
        sh->d = p[0];
        sh->a = 0.5 * p[0];
        sh->rcirc = 0.5 * p[0];
        sh->rin = 0.0; /* the face centre lies on the boundary */
        sh->vol = M_PI * p[0] * p[0] * p[0] / 12.0;
        sh->oriented = 1;
    } else if (kind == ORC_DISCOID) {
        if (np < 2 || !(p[0] > 0.0) || !(p[1] > 0.0)) return -1;
        sh->a = p[0];
        sh->rs = p[1];
        sh->d = 2.0 * (p[0] + p[1]);
        sh->rcirc = p[0] + p[1];
        sh->rin = p[1];
        sh->vol = 2.0 * M_PI * p[0] * p[0] * p[1] + M_PI * M_PI * p[0] * p[1] * p[1] +
                  4.0 / 3.0 * M_PI * p[1] * p[1] * p[1];
        sh->oriented = 1;
    } else {
        return -1;
    }
    return 0;
}

/* rotation matrix (body -> world) of the quaternion (w, x, y, z) */
static void quat_to_mat(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double xx = x * x, yy = y * y, zz = z * z;
    double xy = x * y, xz = x * z, yz = y * z;
    double wx = w * x, wy = w * y, wz = w * z;
    R[0] = 1.0 - 2.0 * (yy + zz);
    R[1] = 2.0 * (xy - wz);
    R[2] = 2.0 * (xz + wy);
    R[3] = 2.0 * (xy + wz);
    R[4] = 1.0 - 2.0 * (xx + zz);
    R[5] = 2.0 * (yz - wx);
    R[6] = 2.0 * (xz - wy);
    R[7] = 2.0 * (yz + wx);
    R[8] = 1.0 - 2.0 * (xx + yy);
}

/* body = R^T v */
static void to_body(const double R[9], const double v[3], double p[3])
{
    p[0] = (R[0] * v[0] + R[3] * v[1]) + R[6] * v[2];
    p[1] = (R[1] * v[0] + R[4] * v[1]) + R[7] * v[2];
    p[2] = (R[2] * v[0] + R[5] * v[1]) + R[8] * v[2];
}

/* world = R b */
static void to_world(const double R[9], const double b[3], double v[3])
{
    v[0] = (R[0] * b[0] + R[1] * b[1]) + R[2] * b[2];
    v[1] = (R[3] * b[0] + R[4] * b[1]) + R[5] * b[2];
    v[2] = (R[6] * b[0] + R[7] * b[1]) + R[8] * b[2];
}

/* Does a depletant sphere of radius r_dep centred at body-frame point p
 * overlap the shape?  Strict: touching is not overlapping. */
static int dep_overlap_body(const shape_t* sh, double r_dep, const double p[3])
{
    if (sh->kind == ORC_HEMISPHERE) {
        double a = sh->a;
        double rho2 = p[0] * p[0] + p[1] * p[1];
        if (p[2] >= 0.0) {
            double R = a + r_dep;
            return rho2 + p[2] * p[2] < R * R;
        }
        if (rho2 <= a * a) return -p[2] < r_dep;
        double t = sqrt(rho2) - a;
        return t * t + p[2] * p[2] < r_dep * r_dep;
    } else { /* discoid */
        double a = sh->a;
        double R = sh->rs + r_dep;
        double rho2 = p[0] * p[0] + p[1] * p[1];
        if (rho2 <= a * a) return p[2] * p[2] < R * R;
        double t = sqrt(rho2) - a;
        return t * t + p[2] * p[2] < R * R;
    }
}

/* depletant at world offset v from the shape's reference point */
static int dep_overlap(const shape_t* sh, double r_dep, const double v[3], const double* R)
{
    if (sh->kind == ORC_SPHERE) {
        double Rs = sh->rcirc + r_dep;
        return (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2] < Rs * Rs;
    }
    double p[3];
    to_body(R, v, p);
    return dep_overlap_body(sh, r_dep, p);
}

int orc_depletant_overlap(int kind, const double* params, double r_dep, const double* v_world, const double* quat)
{
    shape_t sh;
    int np = (kind == ORC_DISCOID) ? 2 : 1;
    if (shape_setup(&sh, kind, params, np)) return -1;
    double R[9];
    double qi[4] = {1.0, 0.0, 0.0, 0.0};
    quat_to_mat(quat ? quat : qi, R);
    return dep_overlap(&sh, r_dep, v_world, R);
}

/* ---------------- convex colloid pairs: GJK distance with bounds -------- */
/* Support point of the body-frame core: hemisphere -> the half ball itself;
 * discoid -> the bare disk (the sweep radius enters through the threshold). */
static void core_support_body(const shape_t* sh, const double n[3], double out[3])
{
    double rho = sqrt(n[0] * n[0] + n[1] * n[1]);
    if (sh->kind == ORC_HEMISPHERE && n[2] > 0.0) {
        double nn = sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
        out[0] = sh->a * n[0] / nn;
        out[1] = sh->a * n[1] / nn;
        out[2] = sh->a * n[2] / nn;
        return;
    }
    if (rho > 0.0) {
        out[0] = sh->a * n[0] / rho;
        out[1] = sh->a * n[1] / rho;
    } else {
        out[0] = 0.0;
        out[1] = 0.0;
    }
    out[2] = 0.0;
}

static void core_support_world(const shape_t* sh, const double R[9], const double c[3], const double n[3],
                               double out[3])
{
    double nb[3], sb[3], sw[3];
    to_body(R, n, nb);
    core_support_body(sh, nb, sb);
    to_world(R, sb, sw);
    out[0] = c[0] + sw[0];
    out[1] = c[1] + sw[1];
    out[2] = c[2] + sw[2];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Closest point to the origin of the convex hull of k <= 4 points, by trying
 * every non-empty subset: the minimiser over each subset's affine hull is
 * kept when all its barycentric weights are >= 0; the smallest such point is
 * the closest point of the hull.  Returns the subset mask used. */
static int hull_closest(const double P[4][3], int k, double v[3], double* vv)
{
    double best = INFINITY;
    int best_mask = 0;
    double bv[3] = {0, 0, 0};
    for (int mask = 1; mask < (1 << k); ++mask) {
        int idx[4], m = 0;
        for (int i = 0; i < k; ++i)
            if (mask & (1 << i)) idx[m++] = i;
        double lam[4];
        if (m == 1) {
            lam[0] = 1.0;
        } else {
            /* minimise |p0 + sum_i mu_i (p_i - p0)|^2 : G mu = -b */
            double E[3][3], G[3][4];
            for (int i = 1; i < m; ++i)
                for (int c = 0; c < 3; ++c) E[i - 1][c] = P[idx[i]][c] - P[idx[0]][c];
            int n = m - 1;
            for (int r = 0; r < n; ++r) {
                for (int c = 0; c < n; ++c) G[r][c] = dot3(E[r], E[c]);
                G[r][n] = -dot3(E[r], P[idx[0]]);
            }
            /* Gaussian elimination with partial pivoting */
            double scale = 0.0;
            for (int r = 0; r < n; ++r) scale = fmax(scale, fabs(G[r][r]));
            int singular = 0;
            for (int c = 0; c < n && !singular; ++c) {
                int piv = c;
                for (int r = c + 1; r < n; ++r)
                    if (fabs(G[r][c]) > fabs(G[piv][c])) piv = r;
                if (!(fabs(G[piv][c]) > 1e-14 * scale)) {
                    singular = 1;
                    break;
                }
                if (piv != c)
                    for (int cc = 0; cc <= n; ++cc) {
                        double tmp = G[c][cc];
                        G[c][cc] = G[piv][cc];
                        G[piv][cc] = tmp;
                    }
                for (int r = c + 1; r < n; ++r) {
                    double f = G[r][c] / G[c][c];
                    for (int cc = c; cc <= n; ++cc) G[r][cc] -= f * G[c][cc];
                }
            }
            if (singular) continue;
            double mu[3];
            for (int r = n - 1; r >= 0; --r) {
                double s = G[r][n];
                for (int cc = r + 1; cc < n; ++cc) s -= G[r][cc] * mu[cc];
                mu[r] = s / G[r][r];
            }
            double s0 = 1.0;
            for (int r = 0; r < n; ++r) {
                lam[r + 1] = mu[r];
                s0 -= mu[r];
            }
            lam[0] = s0;
        }
        int ok = 1;
        for (int i = 0; i < m; ++i)
            if (lam[i] < 0.0) ok = 0;
        if (!ok) continue;
        double y[3] = {0, 0, 0};
        for (int i = 0; i < m; ++i)
            for (int c = 0; c < 3; ++c) y[c] += lam[i] * P[idx[i]][c];
        double yy = dot3(y, y);
        if (yy < best) {
            best = yy;
            best_mask = mask;
            bv[0] = y[0];
            bv[1] = y[1];
            bv[2] = y[2];
        }
    }
    v[0] = bv[0];
    v[1] = bv[1];
    v[2] = bv[2];
    *vv = best;
    return best_mask;
}

#define NEAR_BAND 1e-9

/* Overlap of shape B (reference point at offset d from A's, orientation RB)
 * with shape A (at the origin, orientation RA).  The distance between the
 * cores is bracketed [lo, hi] by GJK (Gilbert, Johnson, Keerthi 1988):
 * hi = |v| for the closest point v of the current simplex (a point of the
 * Minkowski difference B - A), lo = max over iterations of (v . w)/|v| with w
 * the support point of B - A in direction -v.  Overlap iff the core distance
 * is below thr (2 r_s for swept disks, 0 for hemispheres). */
static int convex_pair(const shape_t* sh, const double d[3], const double RA[9], const double RB[9], int* near)
{
    static const double zero[3] = {0, 0, 0};
    double thr = (sh->kind == ORC_DISCOID) ? 2.0 * sh->rs : 0.0;
    /* interior reference points: hemisphere centroid (0,0,3a/8), disk centre */
    double cb[3] = {0, 0, (sh->kind == ORC_HEMISPHERE) ? 0.375 * sh->a : 0.0};
    double ca_w[3], cb_w[3];
    to_world(RA, cb, ca_w);
    to_world(RB, cb, cb_w);
    double v[3] = {d[0] + cb_w[0] - ca_w[0], d[1] + cb_w[1] - ca_w[1], d[2] + cb_w[2] - ca_w[2]};
    double W[4][3];
    int k = 0;
    double lo = -INFINITY;
    *near = 0;
    double vv = dot3(v, v);
    if (vv == 0.0) return 1;
    for (int it = 0; it < 128; ++it) {
        double hi = sqrt(vv);
        double nd[3] = {-v[0], -v[1], -v[2]};
        double sb[3], sa[3];
        core_support_world(sh, RB, d, nd, sb);
        core_support_world(sh, RA, zero, v, sa);
        double w[3] = {sb[0] - sa[0], sb[1] - sa[1], sb[2] - sa[2]};
        double l = dot3(v, w) / hi;
        if (l > lo) lo = l;
        if (lo > thr) {
            *near = (lo < thr + NEAR_BAND);
            return 0;
        }
        if (hi - lo <= 1e-13) break;
        /* add w (skip if it duplicates a vertex) */
        int dup = 0;
        for (int i = 0; i < k; ++i)
            if (W[i][0] == w[0] && W[i][1] == w[1] && W[i][2] == w[2]) dup = 1;
        if (dup) break;
        W[k][0] = w[0];
        W[k][1] = w[1];
        W[k][2] = w[2];
        ++k;
        int mask = hull_closest(W, k, v, &vv);
        /* keep only the vertices supporting the closest point */
        double Wn[4][3];
        int kn = 0;
        for (int i = 0; i < k; ++i)
            if (mask & (1 << i)) {
                Wn[kn][0] = W[i][0];
                Wn[kn][1] = W[i][1];
                Wn[kn][2] = W[i][2];
                ++kn;
            }
        memcpy(W, Wn, sizeof(W));
        k = kn;
        if (k == 4 || vv == 0.0) return 1; /* origin inside the simplex */
        double hn = sqrt(vv);
        if (hn < thr) {
            *near = (hn > thr - NEAR_BAND);
            return 1;
        }
    }
    /* bracket too tight to decide with certainty: contact within rounding */
    double hi = sqrt(vv);
    *near = 1;
    return 0.5 * (hi + lo) < thr;
}

int orc_pair_overlap(int kind, const double* params, const double* d_world, const double* qa, const double* qb,
                     int* near_contact)
{
    shape_t sh;
    int np = (kind == ORC_DISCOID) ? 2 : 1;
    if (shape_setup(&sh, kind, params, np)) return -1;
    int nc = 0;
    int r;
    double dd = dot3(d_world, d_world);
    if (kind == ORC_SPHERE) {
        r = (d_world[0] * d_world[0] + d_world[1] * d_world[1]) + d_world[2] * d_world[2] < sh.d * sh.d;
    } else {
        double lim = 2.0 * sh.rcirc;
        if (dd >= lim * lim) {
            r = 0;
        } else {
            double RA[9], RB[9];
            quat_to_mat(qa, RA);
            quat_to_mat(qb, RB);
            r = convex_pair(&sh, d_world, RA, RB, &nc);
        }
    }
    if (near_contact) *near_contact = nc;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Simulation state                                                           */
/* ------------------------------------------------------------------------ */
struct orc_sim {
    int64_t N;
    double L, halfL;
    uint64_t seed;
    uint32_t replica;
    uint32_t key[2];
    shape_t sh;
    int have_shape;
    /* depletants */
    double z_p, d_dep, r_dep;
    int n_trial;
    /* moves */
    double d_trans, a_rot, p_rot;
    int n_select;
    /* derived */
    int n;
    double w, inv_w, R0, R0sq, lambda, lambda_c, s_ball;
    int region;            /* ORC_V0_BALL or ORC_V0_SHELL */
    double r_inner, span;  /* shell: inner radius and R0 - r_inner */
    int n_chunks;
    double F[POISSON_K];
    /* state */
    double* x[3];
    double* q[4];
    uint64_t sweep;
    int have_state;
    /* cells */
    int* cell_of;
    int* cell_start; /* n^3 + 1 */
    int* members;
    int64_t ncells;
    /* trace */
    int trace_on;
    orc_record* trace;
    int64_t trace_n;
    /* threads over the active cells of a phase (1: the plain serial loop) */
    int threads;
    char err[256];
};

static int fail(orc_sim* s, int code, const char* msg)
{
    snprintf(s->err, sizeof(s->err), "%s", msg);
    return code;
}

orc_sim* orc_create(int64_t n, double box_L, uint64_t seed, uint32_t replica_id)
{
    if (n < 1 || !(box_L > 0.0)) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->N = n;
    s->L = box_L;
    s->halfL = 0.5 * box_L;
    s->seed = seed;
    s->replica = replica_id;
    s->key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    s->key[1] = (uint32_t)(seed >> 32) ^ replica_id;
    for (int a = 0; a < 3; ++a) s->x[a] = (double*)calloc((size_t)n, sizeof(double));
    for (int a = 0; a < 4; ++a) s->q[a] = (double*)calloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i < n; ++i) s->q[0][i] = 1.0;
    s->cell_of = (int*)calloc((size_t)n, sizeof(int));
    s->members = (int*)calloc((size_t)n, sizeof(int));
    s->n_select = 1;
    s->threads = 1;
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    for (int a = 0; a < 3; ++a) free(s->x[a]);
    for (int a = 0; a < 4; ++a) free(s->q[a]);
    free(s->cell_of);
    free(s->members);
    free(s->cell_start);
    free(s->trace);
    free(s);
}

const char* orc_last_error(const orc_sim* s) { return s ? s->err : "null handle"; }

/* derived parameters, in the contract's order of operations */
static int derive(orc_sim* s)
{
    if (!s->have_shape) return 0;
    s->r_dep = 0.5 * s->d_dep;
    s->R0 = s->sh.rcirc + s->r_dep;
    s->R0sq = s->R0 * s->R0;
    double wmin = 2.0 * s->sh.rcirc + s->d_dep;
    int n = (int)floor(s->L / wmin);
    if (n % 2) n -= 1;
    if (n < 2) return fail(s, -2, "box smaller than two cells of the minimum width");
    if ((int64_t)n * n * n > 0x7FFFFFFF) return fail(s, -2, "too many cells");
    s->n = n;
    s->w = s->L / (double)n;
    s->inv_w = 1.0 / s->w;
    s->s_ball = s->R0 * 0x1p-21;
    double vol0 = 4.0 / 3.0 * M_PI * s->R0 * s->R0 * s->R0;
    s->r_inner = 0.0;
    s->span = s->R0;
    if (s->region == ORC_V0_SHELL) {
        /* a translation moves the centre by at most sqrt(3) d_trans */
        double ri = (s->sh.rin + s->r_dep) - sqrt(3.0) * s->d_trans;
        if (ri < 0.0) ri = 0.0;
        s->r_inner = ri;
        s->span = s->R0 - ri;
        vol0 = 4.0 / 3.0 * M_PI * (s->R0 * s->R0 * s->R0 - ri * ri * ri);
    }
    s->lambda = s->z_p * vol0;
    int m = (int)ceil(s->lambda / POISSON_CHUNK);
    if (m < 1) m = 1;
    s->n_chunks = m;
    s->lambda_c = s->lambda / (double)m;
    orc_poisson_table(s->lambda_c, s->F, POISSON_K);
    int64_t nc = (int64_t)n * n * n;
    if (nc != s->ncells) {
        free(s->cell_start);
        s->cell_start = (int*)calloc((size_t)nc + 1, sizeof(int));
        s->ncells = nc;
    }
    return 0;
}

int orc_set_shape(orc_sim* s, int kind, const double* params, int nparams)
{
    if (shape_setup(&s->sh, kind, params, nparams)) return fail(s, -1, "invalid shape");
    s->have_shape = 1;
    if (!s->sh.oriented) s->p_rot = 0.0;
    return derive(s);
}

int orc_set_fugacity(orc_sim* s, double z_p, double d_dep, int n_trial)
{
    if (!(z_p >= 0.0) || !(d_dep >= 0.0) || n_trial < 0 || n_trial > 255)
        return fail(s, -1, "invalid depletant parameters");
    s->z_p = z_p;
    s->d_dep = d_dep;
    s->n_trial = n_trial;
    int r = derive(s);
    if (r) return r;
    if (s->lambda > 60000.0) return fail(s, -1, "depletant mean per move too large");
    return 0;
}

int orc_set_moves(orc_sim* s, double d_trans, double a_rot, double p_rot, int n_select)
{
    if (!(d_trans >= 0.0) || !(a_rot >= 0.0) || !(p_rot >= 0.0 && p_rot <= 1.0) || n_select < 1)
        return fail(s, -1, "invalid move parameters");
    s->d_trans = d_trans;
    s->a_rot = a_rot;
    s->p_rot = (s->have_shape && !s->sh.oriented) ? 0.0 : p_rot;
    s->n_select = n_select;
    return derive(s);
}

int orc_set_insertion(orc_sim* s, int region)
{
    if (region != ORC_V0_BALL && region != ORC_V0_SHELL) return fail(s, -1, "invalid insertion region");
    s->region = region;
    return derive(s);
}

int orc_set_state(orc_sim* s, const double* pos, const double* quat, uint64_t sweep_index)
{
    for (int a = 0; a < 3; ++a) memcpy(s->x[a], pos + (size_t)a * s->N, (size_t)s->N * sizeof(double));
    if (quat)
        for (int a = 0; a < 4; ++a) memcpy(s->q[a], quat + (size_t)a * s->N, (size_t)s->N * sizeof(double));
    s->sweep = sweep_index;
    s->have_state = 1;
    return 0;
}

int orc_get_state(const orc_sim* s, double* pos, double* quat, uint64_t* sweep_index)
{
    if (pos)
        for (int a = 0; a < 3; ++a) memcpy(pos + (size_t)a * s->N, s->x[a], (size_t)s->N * sizeof(double));
    if (quat)
        for (int a = 0; a < 4; ++a) memcpy(quat + (size_t)a * s->N, s->q[a], (size_t)s->N * sizeof(double));
    if (sweep_index) *sweep_index = s->sweep;
    return 0;
}

int orc_set_threads(orc_sim* s, int threads)
{
    if (threads < 1) return fail(s, -1, "threads must be >= 1");
    s->threads = threads;
    return 0;
}

int orc_set_trace(orc_sim* s, int enable)
{
    s->trace_on = enable ? 1 : 0;
    if (s->trace_on && !s->trace) s->trace = (orc_record*)calloc((size_t)s->N * (size_t)s->n_select, sizeof(orc_record));
    return 0;
}

int orc_derived(const orc_sim* s, double* out, int out_len)
{
    double v[14] = {(double)s->n, s->w,         s->inv_w,    s->R0,     s->lambda,
                    (double)s->n_chunks, s->lambda_c, s->s_ball, s->r_dep, s->sh.rcirc,
                    s->sh.vol,   s->halfL,     s->r_inner,  s->span};
    for (int i = 0; i < out_len && i < 14; ++i) out[i] = v[i];
    return 0;
}

/* minimum-image difference along one axis */
static double mi(const orc_sim* s, double d)
{
    if (d > s->halfL)
        d -= s->L;
    else if (d < -s->halfL)
        d += s->L;
    return d;
}

/* cell coordinate of x along one axis under shift g */
static int cell_coord(const orc_sim* s, double xa, double g)
{
    double y = xa - g;
    if (y < 0.0) y += s->L;
    int c = (int)floor(y * s->inv_w);
    if (c > s->n - 1) c = s->n - 1;
    if (c < 0) c = 0;
    return c;
}

static int cell_of_point(const orc_sim* s, const double x[3], const double g[3])
{
    int cx = cell_coord(s, x[0], g[0]);
    int cy = cell_coord(s, x[1], g[1]);
    int cz = cell_coord(s, x[2], g[2]);
    return cx + s->n * (cy + s->n * cz);
}

/* ------------------------------------------------------------------------ */
/* One trial (Sec. III.B-D): returns reason code, fills the record.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    const int* idx; /* stencil particle indices (excluding j) */
    int n;
} stencil_t;

/* overlap of a depletant at offset e (relative to x') with any stencil colloid */
static int dep_hits_stencil(const orc_sim* s, const double e[3], const double (*D)[3], const double (*Rn)[9],
                            int nst)
{
    for (int i = 0; i < nst; ++i) {
        double v[3] = {e[0] - D[i][0], e[1] - D[i][1], e[2] - D[i][2]};
        if (dep_overlap(&s->sh, s->r_dep, v, Rn ? Rn[i] : NULL)) return 1;
    }
    return 0;
}

static int trial(orc_sim* s, int64_t j, const double xn[3], const double qn[4], const stream_t* st,
                 const stencil_t* stc, orc_record* rec, orc_counters* cnt)
{
    const shape_t* sh = &s->sh;
    int nst = stc->n;
    double xo[3] = {s->x[0][j], s->x[1][j], s->x[2][j]};
    double qo[4] = {s->q[0][j], s->q[1][j], s->q[2][j], s->q[3][j]};
    double Rold[9], Rnew[9];
    if (sh->oriented) {
        quat_to_mat(qo, Rold);
        quat_to_mat(qn, Rnew);
    }

    /* displacements (minimum image) of stencil colloids from the new position */
    double (*D)[3] = (double (*)[3])malloc(sizeof(double[3]) * (size_t)(nst > 0 ? nst : 1));
    double (*Rn)[9] = NULL;
    if (sh->oriented) Rn = (double (*)[9])malloc(sizeof(double[9]) * (size_t)(nst > 0 ? nst : 1));
    for (int i = 0; i < nst; ++i) {
        int64_t p = stc->idx[i];
        for (int a = 0; a < 3; ++a) D[i][a] = mi(s, s->x[a][p] - xn[a]);
        if (sh->oriented) {
            double qq[4] = {s->q[0][p], s->q[1][p], s->q[2][p], s->q[3][p]};
            quat_to_mat(qq, Rn[i]);
        }
    }
    int reason = ORC_ACCEPT;

    /* colloid-colloid hard overlap: min(1, exp(-beta dH_cc)) in {0,1} (Eq. pacc) */
    for (int i = 0; i < nst; ++i) {
        cnt->overlap_checks++;
        int ov;
        if (sh->kind == ORC_SPHERE) {
            ov = (D[i][0] * D[i][0] + D[i][1] * D[i][1]) + D[i][2] * D[i][2] < sh->d * sh->d;
        } else {
            double dd = (D[i][0] * D[i][0] + D[i][1] * D[i][1]) + D[i][2] * D[i][2];
            double lim = 2.0 * sh->rcirc;
            if (dd >= lim * lim) {
                ov = 0;
            } else {
                int nc = 0;
                ov = convex_pair(sh, D[i], Rnew, Rn[i], &nc);
                if (nc) {
                    rec->near_contact = 1;
                    cnt->near_contact++;
                }
            }
        }
        if (ov) {
            reason = ORC_REJ_OVERLAP;
            break;
        }
    }

    if (reason == ORC_ACCEPT && s->z_p > 0.0) {
        /* Poisson number of depletants in V_0 = B(x', R0) (Sec. III.B step 2, Sec. III.C) */
        uint32_t Np = 0;
        for (int c = 0; c < s->n_chunks; ++c) {
            uint32_t w[4];
            draw(st, P_POISSON, (uint32_t)c, w);
            Np += (uint32_t)orc_poisson_draw(s->F, POISSON_K, u52(w[0], w[1]));
        }
        rec->n_depletants = Np;
        cnt->depletants_drawn += Np;
        double Dold[3];
        for (int a = 0; a < 3; ++a) Dold[a] = mi(s, xo[a] - xn[a]);
        const double zero3[3] = {0, 0, 0};
        (void)zero3;

        ball_stream_t bs;
        ball_stream_init(&bs, st, P_DEPL, 0);
        uint32_t shell_block = 0;
        uint64_t resolved = 0, cbt = 0;
        uint32_t nblk = 0, wf = 0, wr = 0;
        double ratio = 1.0;
        for (uint32_t k = 0; k < Np && reason == ORC_ACCEPT; ++k) {
            double e[3];
            if (s->region == ORC_V0_SHELL) {
                /* k-th accepted block of the shell stream */
                for (;;) {
                    uint32_t w[4];
                    draw(st, P_DEPL_SHELL, shell_block++, w);
                    if (orc_shell_candidate(w, s->r_inner, s->span, s->R0sq, e)) break;
                }
            } else {
                int32_t m[3];
                ball_stream_next(&bs, m, 0xFFFFFFFFu);
                e[0] = s->s_ball * (double)m[0];
                e[1] = s->s_ball * (double)m[1];
                e[2] = s->s_ball * (double)m[2];
            }
            resolved++;
            /* irrelevant: does not overlap the moved colloid in M' (always overlaps for spheres) */
            if (sh->kind != ORC_SPHERE && !dep_overlap(sh, s->r_dep, e, Rnew)) continue;
            /* ignored: overlaps the colloid in M, or any other colloid (rejection sampling of V_f) */
            double vo[3] = {e[0] - Dold[0], e[1] - Dold[1], e[2] - Dold[2]};
            if (dep_overlap(sh, s->r_dep, vo, Rold)) continue;
            if (dep_hits_stencil(s, e, (const double (*)[3])D, (const double (*)[9])Rn, nst)) continue;
            /* blocking: free in M, overlapping in M' */
            nblk++;
            if (s->n_trial == 0) {
                reason = ORC_REJ_DEPLETANT;
                break;
            }
            /* configurational bias (Sec. III.D): forward re-insertions into B(x, R0)
             * that are valid in M' and overlap the old pose */
            /* trial i is the i-th accepted candidate of the stream of depletant k */
            uint32_t Wf = 0;
            ball_stream_t fs;
            ball_stream_init(&fs, st, P_CB_FWD, k << 16);
            for (int i = 0; i < s->n_trial; ++i) {
                int32_t mf[3];
                double f[3] = {0, 0, 0}, p[3];
                if (ball_stream_next(&fs, mf, 65536)) {
                    f[0] = s->s_ball * (double)mf[0];
                    f[1] = s->s_ball * (double)mf[1];
                    f[2] = s->s_ball * (double)mf[2];
                }
                /* f is the offset from the old centre; p the offset from the new one */
                for (int a = 0; a < 3; ++a) p[a] = Dold[a] + f[a];
                cbt++;
                int ok = 1;
                if (sh->kind != ORC_SPHERE) ok = dep_overlap(sh, s->r_dep, f, Rold);
                if (ok && dep_overlap(sh, s->r_dep, p, Rnew)) ok = 0;
                if (ok && dep_hits_stencil(s, p, (const double (*)[3])D, (const double (*)[9])Rn, nst)) ok = 0;
                Wf += (uint32_t)ok;
            }
            wf += Wf;
            if (Wf == 0) {
                reason = ORC_REJ_CB_ZERO;
                break;
            }
            /* reverse: n_trial - 1 insertions into B(x', R0), valid in M, overlapping the new pose */
            uint32_t Wr = 0;
            ball_stream_t rs;
            ball_stream_init(&rs, st, P_CB_REV, k << 16);
            for (int i = 0; i < s->n_trial - 1; ++i) {
                int32_t mr[3];
                double r[3] = {0, 0, 0};
                if (ball_stream_next(&rs, mr, 65536)) {
                    r[0] = s->s_ball * (double)mr[0];
                    r[1] = s->s_ball * (double)mr[1];
                    r[2] = s->s_ball * (double)mr[2];
                }
                cbt++;
                int ok = 1;
                if (sh->kind != ORC_SPHERE) ok = dep_overlap(sh, s->r_dep, r, Rnew);
                if (ok) {
                    double vq[3] = {r[0] - Dold[0], r[1] - Dold[1], r[2] - Dold[2]};
                    if (dep_overlap(sh, s->r_dep, vq, Rold)) ok = 0;
                }
                if (ok && dep_hits_stencil(s, r, (const double (*)[3])D, (const double (*)[9])Rn, nst)) ok = 0;
                Wr += (uint32_t)ok;
            }
            wr += Wr;
            ratio = ratio * ((double)Wf / (double)(1 + Wr));
        }
        if (reason == ORC_ACCEPT && nblk > 0) {
            uint32_t w[4];
            draw(st, P_ACCEPT, 0, w);
            if (!(u52(w[0], w[1]) < ratio)) reason = ORC_REJ_CB_METROPOLIS;
        }
        rec->resolved = (uint32_t)(resolved + cbt);
        rec->n_blocking = nblk;
        rec->w_fwd = wf;
        rec->w_rev = wr;
        cnt->depletants_resolved += resolved + cbt;
        cnt->cb_trials += cbt;
    }
    free(D);
    free(Rn);
    return reason;
}

static void count_reason(orc_counters* c, int reason)
{
    c->trials++;
    switch (reason) {
    case ORC_ACCEPT: c->accepts++; break;
    case ORC_REJ_CELL_EXIT: c->rej_cell_exit++; break;
    case ORC_REJ_OVERLAP: c->rej_overlap++; break;
    case ORC_REJ_DEPLETANT: c->rej_depletant++; break;
    case ORC_REJ_CB_ZERO: c->rej_cb_zero++; break;
    case ORC_REJ_CB_METROPOLIS: c->rej_cb_metropolis++; break;
    }
}

/* proposal (Sec. III.B step 1): translation uniform in the cube [-d, d]^3, or a
 * rotation q' = (q + a v)/|q + a v| with v uniform in the unit 4-ball */
static int propose(const orc_sim* s, int64_t j, const stream_t* st, int rotate, double xn[3], double qn[4])
{
    for (int a = 0; a < 3; ++a) xn[a] = s->x[a][j];
    for (int a = 0; a < 4; ++a) qn[a] = s->q[a][j];
    if (!rotate) {
        uint32_t w[4];
        draw(st, P_TRANS, 0, w);
        for (int a = 0; a < 3; ++a) {
            double xa = s->x[a][j] + s->d_trans * sym01(w[a]);
            if (xa >= s->L)
                xa -= s->L;
            else if (xa < 0.0)
                xa += s->L;
            xn[a] = xa;
        }
        return 0;
    }
    for (uint32_t b = 0; b < 256; ++b) {
        uint32_t w[4];
        draw(st, P_ROT, b, w);
        int64_t m[4], ss = 0;
        for (int a = 0; a < 4; ++a) {
            m[a] = 2 * (int64_t)(w[a] >> 7) + 1 - ((int64_t)1 << 25);
            ss += m[a] * m[a];
        }
        if (ss < ((int64_t)1 << 50)) {
            double qq[4];
            for (int a = 0; a < 4; ++a) qq[a] = s->q[a][j] + s->a_rot * ((double)m[a] * 0x1p-25);
            double nrm = sqrt(((qq[0] * qq[0] + qq[1] * qq[1]) + qq[2] * qq[2]) + qq[3] * qq[3]);
            for (int a = 0; a < 4; ++a) qn[a] = qq[a] / nrm;
            return 1;
        }
    }
    return 1;
}

int orc_try_move(orc_sim* s, int64_t j, const double* xnew, const double* qnew, uint32_t sweep, uint32_t cell,
                 uint32_t t, orc_record* rec)
{
    if (!s->have_shape) return fail(s, -5, "shape not set");
    stream_t st = {{s->key[0], s->key[1]}, sweep, cell, t};
    int* idx = (int*)malloc(sizeof(int) * (size_t)s->N);
    int nst = 0;
    for (int64_t i = 0; i < s->N; ++i)
        if (i != j) idx[nst++] = (int)i;
    stencil_t stc = {idx, nst};
    orc_record r;
    memset(&r, 0, sizeof(r));
    orc_counters c;
    memset(&c, 0, sizeof(c));
    double qi[4] = {1, 0, 0, 0};
    int reason = trial(s, j, xnew, qnew ? qnew : qi, &st, &stc, &r, &c);
    r.particle = (uint32_t)j;
    r.reason = (uint8_t)reason;
    r.sweep = sweep;
    r.cell = cell;
    r.t = t;
    if (rec) *rec = r;
    free(idx);
    return reason;
}

/* the same fixed proposal tried on `count` independent streams (sweep index
 * sweep0 + i); reasons[i] receives each outcome (statistical pins) */
int orc_try_move_many(orc_sim* s, int64_t j, const double* xnew, const double* qnew, uint32_t sweep0,
                      int64_t count, uint8_t* reasons, uint32_t* n_depletants)
{
    if (!s->have_shape) return fail(s, -5, "shape not set");
    int* idx = (int*)malloc(sizeof(int) * (size_t)s->N);
    int nst = 0;
    for (int64_t i = 0; i < s->N; ++i)
        if (i != j) idx[nst++] = (int)i;
    stencil_t stc = {idx, nst};
    double qi[4] = {1, 0, 0, 0};
    for (int64_t i = 0; i < count; ++i) {
        stream_t st = {{s->key[0], s->key[1]}, sweep0 + (uint32_t)i, 0, 0};
        orc_record r;
        memset(&r, 0, sizeof(r));
        orc_counters c;
        memset(&c, 0, sizeof(c));
        int reason = trial(s, j, xnew, qnew ? qnew : qi, &st, &stc, &r, &c);
        reasons[i] = (uint8_t)reason;
        if (n_depletants) n_depletants[i] = r.n_depletants;
    }
    free(idx);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sweep (Sec. III.E): shifted checkerboard, 8 colours in random order.       */
/* ------------------------------------------------------------------------ */
static int cheb(int a, int b, int n)
{
    int d = a > b ? a - b : b - a;
    return d < n - d ? d : n - d;
}

/* The trials of one active cell c in phase p, in round order (Sec. III.E:
 * n_select n_c rounds, each selecting a member uniformly). */
static void run_cell(orc_sim* s, int64_t c, int p, const double g[3], int* stidx, orc_counters* cnt)
{
    int n = s->n;
    uint32_t sw = (uint32_t)s->sweep;
    uint32_t w[4];
    int offs[3], noff;
    if (n == 2) {
        offs[0] = 0;
        offs[1] = 1;
        noff = 2;
    } else {
        offs[0] = -1;
        offs[1] = 0;
        offs[2] = 1;
        noff = 3;
    }
    int cx = (int)(c % n), cy = (int)((c / n) % n), cz = (int)(c / ((int64_t)n * n));
    int nmem = s->cell_start[c + 1] - s->cell_start[c];
    if (nmem == 0) return;
    int ntr = s->n_select * nmem;
    for (int t = 0; t < ntr; ++t) {
        stream_t st = {{s->key[0], s->key[1]}, sw, (uint32_t)c, (uint32_t)t};
        orc_record rec;
        memset(&rec, 0, sizeof(rec));
        draw(&st, P_SELECT, 0, w);
        int jl = (int)pick(w[0], (uint32_t)nmem);
        int64_t j = s->members[s->cell_start[c] + jl];
        int rotate = s->sh.oriented && s->p_rot > 0.0 && u01(w[1]) < s->p_rot;
        double xn[3], qn[4];
        propose(s, j, &st, rotate, xn, qn);
        int reason;
        if (cell_of_point(s, xn, g) != (int)c) {
            reason = ORC_REJ_CELL_EXIT;
        } else {
            /* stencil: de-duplicated neighbour cells, minus j */
            int nst = 0;
            for (int a = 0; a < noff; ++a)
                for (int b = 0; b < noff; ++b)
                    for (int d = 0; d < noff; ++d) {
                        int ex = (cx + offs[d] + n) % n;
                        int ey = (cy + offs[b] + n) % n;
                        int ez = (cz + offs[a] + n) % n;
                        int e = ex + n * (ey + n * ez);
                        for (int q = s->cell_start[e]; q < s->cell_start[e + 1]; ++q)
                            if (s->members[q] != j) stidx[nst++] = s->members[q];
                    }
            stencil_t stc = {stidx, nst};
            reason = trial(s, j, xn, qn, &st, &stc, &rec, cnt);
        }
        if (reason == ORC_ACCEPT) {
            for (int a = 0; a < 3; ++a) s->x[a][j] = xn[a];
            for (int a = 0; a < 4; ++a) s->q[a][j] = qn[a];
        }
        count_reason(cnt, reason);
        if (s->trace_on) {
            rec.sweep = sw;
            rec.cell = (uint32_t)c;
            rec.t = (uint32_t)t;
            rec.particle = (uint32_t)j;
            rec.phase = (uint8_t)p;
            rec.reason = (uint8_t)reason;
            rec.rotation = (uint8_t)rotate;
            s->trace[(int64_t)s->n_select * s->cell_start[c] + t] = rec;
        }
    }
}

/* One sweep.  target < 0: every cell.  target >= 0: only the cells whose
 * outcome can reach that cell's trials -- in phase q, the cells within
 * (periodic Chebyshev) distance p* - q of it, p* being its own phase -- so a
 * single cell of a large box is reproduced exactly without the whole sweep. */
static void sweep_once(orc_sim* s, orc_counters* cnt, int64_t target)
{
    int n = s->n;
    uint32_t sw = (uint32_t)s->sweep;
    stream_t gs = {{s->key[0], s->key[1]}, sw, NO_CELL, 0};
    uint32_t w[4];
    /* random grid shift in [0, w)^3 */
    draw(&gs, P_GRID, 0, w);
    double g[3];
    for (int a = 0; a < 3; ++a) g[a] = s->w * u01(w[a]);
    /* random colour order: Fisher-Yates over {0..7} */
    int perm[8];
    for (int i = 0; i < 8; ++i) perm[i] = i;
    uint32_t fy[7];
    draw(&gs, P_GRID, 1, w);
    fy[0] = w[0];
    fy[1] = w[1];
    fy[2] = w[2];
    fy[3] = w[3];
    draw(&gs, P_GRID, 2, w);
    fy[4] = w[0];
    fy[5] = w[1];
    fy[6] = w[2];
    for (int i = 7, f = 0; i >= 1; --i, ++f) {
        int jx = (int)pick(fy[f], (uint32_t)(i + 1));
        int tmp = perm[i];
        perm[i] = perm[jx];
        perm[jx] = tmp;
    }
    /* bin: members of each cell in ascending particle index */
    int64_t nc = s->ncells;
    memset(s->cell_start, 0, sizeof(int) * (size_t)(nc + 1));
    for (int64_t i = 0; i < s->N; ++i) {
        double xi[3] = {s->x[0][i], s->x[1][i], s->x[2][i]};
        int c = cell_of_point(s, xi, g);
        s->cell_of[i] = c;
        s->cell_start[c + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) s->cell_start[c + 1] += s->cell_start[c];
    int* fill = (int*)calloc(nc > 0 ? (size_t)nc : 1u, sizeof(int));
    for (int64_t i = 0; i < s->N; ++i) {
        int c = s->cell_of[i];
        s->members[s->cell_start[c] + fill[c]++] = (int)i;
    }
    free(fill);

    int tx = 0, ty = 0, tz = 0, tphase = 7;
    if (target >= 0) {
        tx = (int)(target % n);
        ty = (int)((target / n) % n);
        tz = (int)(target / ((int64_t)n * n));
        int tcol = (tx & 1) | ((ty & 1) << 1) | ((tz & 1) << 2);
        for (int p = 0; p < 8; ++p)
            if (perm[p] == tcol) tphase = p;
    }
    int64_t* act = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nc > 0 ? nc : 1));
    for (int p = 0; p < 8; ++p) {
        int col = perm[p];
        if (target >= 0 && p > tphase) break;
        /* the active cells of this phase, in ascending cell id */
        int64_t nact = 0;
        for (int64_t c = 0; c < nc; ++c) {
            int cx = (int)(c % n), cy = (int)((c / n) % n), cz = (int)(c / ((int64_t)n * n));
            int ccol = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
            if (ccol != col) continue;
            if (target >= 0) {
                int reach = tphase - p;
                if (cheb(cx, tx, n) > reach || cheb(cy, ty, n) > reach || cheb(cz, tz, n) > reach) continue;
            }
            act[nact++] = c;
        }
        /* Cells of one colour share no stencil cell and each trial moves only a
         * member of its own cell, so the cells of a phase may run in any order
         * or at once (Sec. III.E); with threads > 1 they are spread over
         * OpenMP threads, each with its own counters, summed afterwards
         * (integer sums: the result is that of the serial loop). */
#pragma omp parallel num_threads(s->threads) if (s->threads > 1)
        {
            int* stidx = (int*)malloc(sizeof(int) * (size_t)s->N);
            orc_counters lc;
            memset(&lc, 0, sizeof(lc));
#pragma omp for schedule(dynamic, 16)
            for (int64_t i = 0; i < nact; ++i) run_cell(s, act[i], p, g, stidx, &lc);
#pragma omp critical
            {
                uint64_t* dst = (uint64_t*)cnt;
                const uint64_t* src = (const uint64_t*)&lc;
                for (size_t k = 0; k < sizeof(orc_counters) / sizeof(uint64_t); ++k) dst[k] += src[k];
            }
            free(stidx);
        }
    }
    free(act);
    if (s->trace_on) s->trace_n = (int64_t)s->n_select * s->N;
    s->sweep++;
}

int orc_sweep(orc_sim* s, int n_sweeps, orc_counters* out)
{
    if (!s->have_shape || !s->have_state) return fail(s, -5, "shape or state not set");
    if (s->n < 2) return fail(s, -2, "invalid box");
    orc_counters c;
    memset(&c, 0, sizeof(c));
    if (s->trace_on) {
        free(s->trace);
        s->trace = (orc_record*)calloc((size_t)s->N * (size_t)s->n_select, sizeof(orc_record));
    }
    for (int i = 0; i < n_sweeps; ++i) sweep_once(s, &c, -1);
    if (out) *out = c;
    return 0;
}

int orc_sweep_cone(orc_sim* s, int64_t target_cell, orc_counters* out)
{
    if (!s->have_shape || !s->have_state) return fail(s, -5, "shape or state not set");
    if (target_cell < 0 || target_cell >= s->ncells) return fail(s, -1, "target cell out of range");
    orc_counters c;
    memset(&c, 0, sizeof(c));
    if (s->trace_on) {
        free(s->trace);
        s->trace = (orc_record*)calloc((size_t)s->N * (size_t)s->n_select, sizeof(orc_record));
    }
    sweep_once(s, &c, target_cell);
    if (out) *out = c;
    return 0;
}

int orc_trace(const orc_sim* s, orc_record* buf, int64_t cap, int64_t* n_written)
{
    int64_t n = s->trace_on ? s->trace_n : 0;
    if (n > cap) n = cap;
    if (n > 0) memcpy(buf, s->trace, sizeof(orc_record) * (size_t)n);
    if (n_written) *n_written = n;
    return 0;
}

/* all pairs i<j that overlap (hard-core invariant) */
int orc_count_overlaps(orc_sim* s, int64_t* n_pairs)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < s->N; ++i) {
        double qa[4] = {s->q[0][i], s->q[1][i], s->q[2][i], s->q[3][i]};
        double RA[9];
        quat_to_mat(qa, RA);
        for (int64_t j = i + 1; j < s->N; ++j) {
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = mi(s, s->x[a][j] - s->x[a][i]);
            double dd = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            int ov;
            if (s->sh.kind == ORC_SPHERE) {
                ov = dd < s->sh.d * s->sh.d;
            } else {
                double lim = 2.0 * s->sh.rcirc;
                if (dd >= lim * lim) {
                    ov = 0;
                } else {
                    double qb[4] = {s->q[0][j], s->q[1][j], s->q[2][j], s->q[3][j]};
                    double RB[9];
                    quat_to_mat(qb, RB);
                    int nc;
                    ov = convex_pair(&s->sh, d, RA, RB, &nc);
                }
            }
            cnt += ov;
        }
    }
    *n_pairs = cnt;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Observables: g(r), free-volume fraction (Sec. IV.A), SDF pressure          */
/* ------------------------------------------------------------------------ */
static int probe_free(const orc_sim* s, const double P[3], double scale)
{
    for (int64_t i = 0; i < s->N; ++i) {
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = mi(s, P[a] - s->x[a][i]);
        if (scale != 1.0)
            for (int a = 0; a < 3; ++a) v[a] = v[a] * scale;
        double R[9];
        if (s->sh.oriented) {
            double q[4] = {s->q[0][i], s->q[1][i], s->q[2][i], s->q[3][i]};
            quat_to_mat(q, R);
        }
        if (dep_overlap(&s->sh, s->r_dep, v, R)) return 0;
    }
    return 1;
}

static void probe_point(const orc_sim* s, uint32_t seq, int64_t p, double P[3])
{
    stream_t st = {{s->key[0], s->key[1]}, seq, NO_CELL, 0};
    uint32_t w[4];
    draw(&st, P_OBS_FV, (uint32_t)p, w);
    for (int a = 0; a < 3; ++a) P[a] = s->L * u01(w[a]);
}

/* smallest compression x in [0, x_max) of the pair separation at which the
 * pair overlaps; returns x_max when it does not overlap at x_max */
static double pair_scale(const orc_sim* s, const double d[3], const double RA[9], const double RB[9], double x_max)
{
    if (s->sh.kind == ORC_SPHERE) {
        double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
        double x = 1.0 - s->sh.d / r;
        return x < x_max ? x : x_max;
    }
    int nc;
    double f = 1.0 - x_max;
    double dm[3] = {d[0] * f, d[1] * f, d[2] * f};
    double dd = (dm[0] * dm[0] + dm[1] * dm[1]) + dm[2] * dm[2];
    double lim = 2.0 * s->sh.rcirc;
    if (dd >= lim * lim || !convex_pair(&s->sh, dm, RA, RB, &nc)) return x_max;
    double lo = 0.0, hi = x_max;
    for (int it = 0; it < 40; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = 1.0 - mid;
        double dx[3] = {d[0] * fm, d[1] * fm, d[2] * fm};
        double d2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
        int ov = (d2 < lim * lim) && convex_pair(&s->sh, dx, RA, RB, &nc);
        if (ov)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

int orc_observables(orc_sim* s, int kind, const orc_obs_params* p, double* out, int64_t out_len)
{
    if (!s->have_shape || !s->have_state) return fail(s, -5, "shape or state not set");
    double V = s->L * s->L * s->L;
    if (kind == ORC_OBS_GR) {
        int nb = p->n_bins;
        if (nb < 1 || out_len < nb || !(p->r_max > 0.0) || p->r_max > s->halfL) return fail(s, -1, "bad g(r) params");
        double* cnt = (double*)calloc((size_t)nb, sizeof(double));
        double inv_dr = (double)nb / p->r_max;
        for (int64_t i = 0; i < s->N; ++i)
            for (int64_t j = i + 1; j < s->N; ++j) {
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = mi(s, s->x[a][j] - s->x[a][i]);
                double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
                if (r < p->r_max) {
                    int b = (int)floor(r * inv_dr);
                    if (b < nb) cnt[b] += 1.0;
                }
            }
        double npair = 0.5 * (double)s->N * (double)(s->N - 1);
        double dr = p->r_max / (double)nb;
        for (int b = 0; b < nb; ++b) {
            double r0 = (double)b * dr, r1 = (double)(b + 1) * dr;
            double shell = 4.0 / 3.0 * M_PI * (r1 * r1 * r1 - r0 * r0 * r0);
            out[b] = cnt[b] / (npair * shell / V);
        }
        free(cnt);
        return 0;
    }
    if (kind == ORC_OBS_FREE_VOLUME) {
        if (out_len < 3 || p->n_probe < 1) return fail(s, -1, "bad free-volume params");
        int64_t nfree = 0;
        for (int64_t k = 0; k < p->n_probe; ++k) {
            double P[3];
            probe_point(s, p->obs_seq, k, P);
            nfree += probe_free(s, P, 1.0);
        }
        double alpha = (double)nfree / (double)p->n_probe;
        double phi_r = M_PI / 6.0 * s->d_dep * s->d_dep * s->d_dep * s->z_p;
        out[0] = alpha;
        out[1] = phi_r * alpha;
        out[2] = (double)nfree;
        return 0;
    }
    if (kind == ORC_OBS_SDF) {
        int nb = p->n_bins;
        if (nb < 2 || out_len < 4 + nb || !(p->x_max > 0.0) || p->x_max >= 1.0 || p->n_fit < 2 || p->n_fit > nb)
            return fail(s, -1, "bad SDF params");
        double* hist = out + 4;
        for (int b = 0; b < nb; ++b) hist[b] = 0.0;
        double inv_dx = (double)nb / p->x_max;
        for (int64_t i = 0; i < s->N; ++i) {
            double qa[4] = {s->q[0][i], s->q[1][i], s->q[2][i], s->q[3][i]};
            double RA[9];
            quat_to_mat(qa, RA);
            double xmin = p->x_max;
            for (int64_t j = 0; j < s->N; ++j) {
                if (j == i) continue;
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = mi(s, s->x[a][j] - s->x[a][i]);
                double dd = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                /* pairs that cannot touch even after compression by x_max */
                double lim = 2.0 * s->sh.rcirc / (1.0 - p->x_max);
                if (dd >= lim * lim) continue;
                double qb[4] = {s->q[0][j], s->q[1][j], s->q[2][j], s->q[3][j]};
                double RB[9];
                quat_to_mat(qb, RB);
                double x = pair_scale(s, d, RA, RB, p->x_max);
                if (x < xmin) xmin = x;
            }
            if (xmin < p->x_max) {
                int b = (int)floor(xmin * inv_dx);
                if (b < nb) hist[b] += 1.0;
            }
        }
        double dx = p->x_max / (double)nb;
        for (int b = 0; b < nb; ++b) hist[b] = hist[b] / ((double)s->N * dx);
        /* s(0+) by a least-squares line through the first n_fit bin centres */
        double sx = 0, sy = 0, sxx = 0, sxy = 0;
        int nf = p->n_fit;
        for (int b = 0; b < nf; ++b) {
            double xb = ((double)b + 0.5) * dx;
            sx += xb;
            sy += hist[b];
            sxx += xb * xb;
            sxy += xb * hist[b];
        }
        double den = (double)nf * sxx - sx * sx;
        double slope = ((double)nf * sxy - sx * sy) / den;
        double s0 = (sy - slope * sx) / (double)nf;
        double rho = (double)s->N / V;
        double bp_hard = rho * (1.0 + s0 / 6.0);
        /* depletant term z_p dV_f/dV by a virtual expansion of the probe set */
        double bp_dep = 0.0;
        if (s->z_p > 0.0 && p->n_probe > 0) {
            int64_t f0 = 0, f1 = 0;
            double sc = 1.0 + p->eps;
            for (int64_t k = 0; k < p->n_probe; ++k) {
                double P[3];
                probe_point(s, p->obs_seq, k, P);
                f0 += probe_free(s, P, 1.0);
                f1 += probe_free(s, P, sc);
            }
            double g3 = sc * sc * sc;
            double a0 = (double)f0 / (double)p->n_probe, a1 = (double)f1 / (double)p->n_probe;
            bp_dep = s->z_p * ((g3 * a1 - a0) / (g3 - 1.0));
        }
        out[0] = bp_hard + bp_dep;
        out[1] = bp_hard;
        out[2] = bp_dep;
        out[3] = s0;
        return 0;
    }
    return fail(s, -1, "unknown observable");
}
