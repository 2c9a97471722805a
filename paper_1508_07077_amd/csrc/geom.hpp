// geom.hpp -- shape predicates on the device (FP64, IEEE operations in a fixed
// order; compiled without floating-point contraction).
//
// The paper (arXiv:1508.07077) uses hard spheres (Sec. IV), hemispheres
// (Sec. V.A) and discoids (Sec. V.B) with penetrable spherical depletants but
// gives no overlap algorithm.  Depletant-colloid tests here are exact distance
// tests; colloid-colloid tests of convex shapes use Minkowski portal refinement
// (MPR, "XenoCollide", G. Snethen, Game Programming Gems 7, 2008) on support
// functions.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace hpmc {

enum ShapeKind : int { kSphere = 0, kHemisphere = 1, kDiscoid = 2 };

struct Vec3 {
    double x, y, z;
};

__host__ __device__ inline Vec3 v3(double x, double y, double z) { return Vec3{x, y, z}; }
__host__ __device__ inline Vec3 operator-(Vec3 a, Vec3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline Vec3 operator+(Vec3 a, Vec3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline Vec3 operator*(double s, Vec3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__host__ __device__ inline Vec3 neg(Vec3 a) { return v3(-a.x, -a.y, -a.z); }
__host__ __device__ inline double dot(Vec3 a, Vec3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__host__ __device__ inline Vec3 cross(Vec3 a, Vec3 b)
{
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// body -> world rotation of the unit quaternion (w, x, y, z)
struct Mat3 {
    double m[9];
};

__host__ __device__ inline Mat3 quat_to_mat(double w, double x, double y, double z)
{
    double xx = x * x, yy = y * y, zz = z * z;
    double xy = x * y, xz = x * z, yz = y * z;
    double wx = w * x, wy = w * y, wz = w * z;
    Mat3 R;
    R.m[0] = 1.0 - 2.0 * (yy + zz);
    R.m[1] = 2.0 * (xy - wz);
    R.m[2] = 2.0 * (xz + wy);
    R.m[3] = 2.0 * (xy + wz);
    R.m[4] = 1.0 - 2.0 * (xx + zz);
    R.m[5] = 2.0 * (yz - wx);
    R.m[6] = 2.0 * (xz - wy);
    R.m[7] = 2.0 * (yz + wx);
    R.m[8] = 1.0 - 2.0 * (xx + yy);
    return R;
}

// R^T v
__host__ __device__ inline Vec3 to_body(const Mat3& R, Vec3 v)
{
    return v3((R.m[0] * v.x + R.m[3] * v.y) + R.m[6] * v.z, (R.m[1] * v.x + R.m[4] * v.y) + R.m[7] * v.z,
              (R.m[2] * v.x + R.m[5] * v.y) + R.m[8] * v.z);
}

// R b
__host__ __device__ inline Vec3 to_world(const Mat3& R, Vec3 b)
{
    return v3((R.m[0] * b.x + R.m[1] * b.y) + R.m[2] * b.z, (R.m[3] * b.x + R.m[4] * b.y) + R.m[5] * b.z,
              (R.m[6] * b.x + R.m[7] * b.y) + R.m[8] * b.z);
}

// per-state-point shape constants (host-computed)
struct Shape {
    int kind;
    int oriented;
    double a;        // hemisphere radius d/2; discoid disk radius
    double rs;       // discoid sweep radius
    double rcirc;    // circumradius about the reference point
    double rin;      // radius of the largest ball about the reference point inside the shape
    double dsq;      // sphere: d^2
    double r_dep;    // depletant radius
    double R0sq;     // (rcirc + r_dep)^2 : sphere and hemisphere dome threshold
    double asq;      // a^2
    double rdsq;     // r_dep^2
    double rsd_sq;   // (r_s + r_dep)^2
    double lim_sq;   // (2 rcirc)^2 : colloid circumsphere pre-test
};

// depletant of radius r_dep at body-frame point p overlaps the shape (strict)
__host__ __device__ inline bool dep_overlap_body(const Shape& S, Vec3 p)
{
    double rho2 = p.x * p.x + p.y * p.y;
    if (S.kind == kHemisphere) {
        if (p.z >= 0.0) return rho2 + p.z * p.z < S.R0sq;
        if (rho2 <= S.asq) return -p.z < S.r_dep;
        double t = sqrt(rho2) - S.a;
        return t * t + p.z * p.z < S.rdsq;
    }
    // discoid
    if (rho2 <= S.asq) return p.z * p.z < S.rsd_sq;
    double t = sqrt(rho2) - S.a;
    return t * t + p.z * p.z < S.rsd_sq;
}

__host__ __device__ inline bool dep_overlap_sphere(const Shape& S, Vec3 v) { return dot(v, v) < S.R0sq; }

__host__ __device__ inline bool dep_overlap(const Shape& S, Vec3 v, const Mat3& R)
{
    if (S.kind == kSphere) return dep_overlap_sphere(S, v);
    return dep_overlap_body(S, to_body(R, v));
}

// ---------------------------------------------------------------------------
// Support functions of the full shapes (body frame), direction n != 0.
// ---------------------------------------------------------------------------
__host__ __device__ inline Vec3 support_body(const Shape& S, Vec3 n)
{
    // unit directions by reciprocal square roots: no divisions in the MPR loop
    double rho2 = n.x * n.x + n.y * n.y;
    if (S.kind == kHemisphere) {
        if (n.z > 0.0) {
            double inv = S.a * rsqrt(dot(n, n));
            return v3(n.x * inv, n.y * inv, n.z * inv);
        }
        if (rho2 > 0.0) {
            double inv = S.a * rsqrt(rho2);
            return v3(n.x * inv, n.y * inv, 0.0);
        }
        return v3(0.0, 0.0, 0.0);
    }
    // discoid: disk support + ball support
    double inv_n = S.rs * rsqrt(dot(n, n));
    Vec3 s = v3(n.x * inv_n, n.y * inv_n, n.z * inv_n);
    if (rho2 > 0.0) {
        double inv_r = S.a * rsqrt(rho2);
        s.x = s.x + n.x * inv_r;
        s.y = s.y + n.y * inv_r;
    }
    return s;
}

__host__ __device__ inline Vec3 support_world(const Shape& S, const Mat3& R, Vec3 c, Vec3 n)
{
    return c + to_world(R, support_body(S, to_body(R, n)));
}

struct PairResult {
    bool overlap;
    bool near;
};

// Minkowski portal refinement on the difference B - A (B at offset d with
// rotation RB, A at the origin with rotation RA).  The origin lies inside the
// difference iff the shapes overlap.  It runs in A's body frame, where A's
// support needs no rotation and B sits at RA^T d with rotation RA^T RB.
// Interior seed: difference of the shapes' interior points (hemisphere
// centroid (0,0,3a/8), disk centre).
__host__ __device__ inline PairResult mpr_overlap(const Shape& S, Vec3 d, const Mat3& RA, const Mat3& RB)
{
    const double tol = 1e-13;
    PairResult res{false, false};
    const Vec3 dA = to_body(RA, d);
    Mat3 RAB;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            RAB.m[3 * i + j] = (RA.m[i] * RB.m[j] + RA.m[3 + i] * RB.m[3 + j]) + RA.m[6 + i] * RB.m[6 + j];
    Vec3 cin = v3(0.0, 0.0, S.kind == kHemisphere ? 0.375 * S.a : 0.0);
    Vec3 v0 = (dA + to_world(RAB, cin)) - cin;
    if (dot(v0, v0) < 1e-30) v0 = v3(1e-12, 0.0, 0.0);
    // support of B - A in direction n
#define HPMC_SUP(n) (support_world(S, RAB, dA, (n)) - support_body(S, neg(n)))
    Vec3 n = neg(v0);
    Vec3 v1 = HPMC_SUP(n);
    if (dot(v1, n) <= 0.0) return res;
    n = cross(v1, v0);
    if (dot(n, n) < 1e-30) {
        res.overlap = true;
        return res;
    }
    Vec3 v2 = HPMC_SUP(n);
    if (dot(v2, n) <= 0.0) return res;
    n = cross(v1 - v0, v2 - v0);
    if (dot(n, v0) > 0.0) {
        Vec3 t = v1;
        v1 = v2;
        v2 = t;
        n = neg(n);
    }
    Vec3 v3p = v0;
    // portal discovery: a triangle (v1, v2, v3) whose cone from v0 holds the origin ray
    int it = 0;
    for (; it < 64; ++it) {
        v3p = HPMC_SUP(n);
        if (dot(v3p, n) <= 0.0) return res;
        if (dot(cross(v1, v3p), v0) < 0.0) {
            v2 = v3p;
            n = cross(v1 - v0, v3p - v0);
            continue;
        }
        if (dot(cross(v3p, v2), v0) < 0.0) {
            v1 = v3p;
            n = cross(v3p - v0, v2 - v0);
            continue;
        }
        break;
    }
    if (it == 64) {
        res.near = true;
        return res;
    }
    // portal refinement
    for (int k = 0; k < 96; ++k) {
        n = cross(v2 - v1, v3p - v1);
        if (dot(n, v1) >= 0.0) {
            res.overlap = true;
            return res;
        }
        Vec3 v4 = HPMC_SUP(n);
        // tolerances relative to |n|, compared in squares (no square root per step)
        const double n2 = dot(n, n);
        const double s4 = dot(v4, n);
        if (s4 <= 0.0) {
            res.near = s4 * s4 < 1e-18 * n2;
            return res;
        }
        auto within = [&](double t) { return t <= 0.0 || t * t <= (tol * tol) * n2; };
        if (within(dot(v4 - v3p, n)) || within(dot(v4 - v1, n)) || within(dot(v4 - v2, n))) {
            // support plane within tolerance of the portal: contact within rounding
            res.near = true;
            res.overlap = false;
            return res;
        }
        Vec3 dd = cross(v4, v0);
        if (dot(v1, dd) > 0.0) {
            if (dot(v2, dd) > 0.0)
                v1 = v4;
            else
                v3p = v4;
        } else {
            if (dot(v3p, dd) > 0.0)
                v2 = v4;
            else
                v1 = v4;
        }
    }
#undef HPMC_SUP
    res.near = true;
    return res;
}

// 1/sqrt(x) for a normal x > 0: the hardware estimate refined by one Newton
// step, relative error far below 1e-12.  Enough for the separating-axis
// filter, whose verdicts carry a 2e-9 margin; the correctly rounded square
// root and division take several times as many dependent operations.
__device__ inline double rsq_newton(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    return r * (1.5 - (0.5 * x) * (r * r));
}

// Support value max_{x in shape} u.x of a body (reference point at the
// origin, body z axis nz in world coordinates) along the unit vector u.
__host__ __device__ inline double support_value(const Shape& S, Vec3 nz, Vec3 u)
{
    double c = dot(nz, u);
    double s2 = 1.0 - c * c;
    double rim = s2 > 0.0 ? S.a * (s2 * rsq_newton(s2)) : 0.0;
    if (S.kind == kHemisphere) return c >= 0.0 ? S.a : rim;
    return rim + S.rs;
}

// Separating-axis test of two oriented bodies (A at the origin, B at offset d)
// along the centre line, both body axes and their cross product.  True only
// when one axis separates them by more than 2e-9, so the bodies are then
// disjoint and farther apart than any contact tolerance: every exact test
// (MPR here, GJK in the oracle) reports no overlap for them.
__host__ __device__ inline bool sat_axis_separates(const Shape& S, Vec3 na, Vec3 nb, Vec3 d, Vec3 u)
{
    const double margin = 2e-9;
    Vec3 mu = neg(u);
    double sd = dot(u, d);
    // B beyond A along u, or along -u
    return support_value(S, na, u) + support_value(S, nb, mu) + margin < sd ||
           support_value(S, na, mu) + support_value(S, nb, u) + margin < -sd;
}

__host__ __device__ inline bool sat_disjoint(const Shape& S, Vec3 d, const Mat3& RA, const Mat3& RB)
{
    Vec3 na = v3(RA.m[2], RA.m[5], RA.m[8]);
    Vec3 nb = v3(RB.m[2], RB.m[5], RB.m[8]);
    double dd = dot(d, d);
    if (dd > 1e-200) {
        double inv = rsq_newton(dd);
        if (sat_axis_separates(S, na, nb, d, v3(d.x * inv, d.y * inv, d.z * inv))) return true;
    }
    if (sat_axis_separates(S, na, nb, d, na) || sat_axis_separates(S, na, nb, d, nb)) return true;
    Vec3 cr = cross(na, nb);
    double cc = dot(cr, cr);
    if (cc > 1e-12) {
        double inv = rsq_newton(cc);
        if (sat_axis_separates(S, na, nb, d, v3(cr.x * inv, cr.y * inv, cr.z * inv))) return true;
    }
    return false;
}

// compile-time shape dispatch for the hot loops
template <int KIND>
__host__ __device__ inline bool dep_ov(const Shape& S, Vec3 v, const Mat3& R)
{
    if constexpr (KIND == kSphere) {
        return dot(v, v) < S.R0sq;
    } else {
        Vec3 p = to_body(R, v);
        double rho2 = p.x * p.x + p.y * p.y;
        if constexpr (KIND == kHemisphere) {
            if (p.z >= 0.0) return rho2 + p.z * p.z < S.R0sq;
            if (rho2 <= S.asq) return -p.z < S.r_dep;
            double t = sqrt(rho2) - S.a;
            return t * t + p.z * p.z < S.rdsq;
        } else {
            if (rho2 <= S.asq) return p.z * p.z < S.rsd_sq;
            double t = sqrt(rho2) - S.a;
            return t * t + p.z * p.z < S.rsd_sq;
        }
    }
}

// colloid-colloid overlap: B at offset d from A
__host__ __device__ inline PairResult pair_overlap(const Shape& S, Vec3 d, const Mat3& RA, const Mat3& RB)
{
    double dd = dot(d, d);
    if (S.kind == kSphere) return PairResult{dd < S.dsq, false};
    if (dd >= S.lim_sq) return PairResult{false, false};
    if (sat_disjoint(S, d, RA, RB)) return PairResult{false, false};
    return mpr_overlap(S, d, RA, RB);
}

template <int KIND>
__host__ __device__ inline PairResult pair_ov(const Shape& S, Vec3 d, const Mat3& RA, const Mat3& RB)
{
    double dd = dot(d, d);
    if constexpr (KIND == kSphere) {
        return PairResult{dd < S.dsq, false};
    } else {
        if (dd >= S.lim_sq) return PairResult{false, false};
        if (sat_disjoint(S, d, RA, RB)) return PairResult{false, false};
        return mpr_overlap(S, d, RA, RB);
    }
}

}  // namespace hpmc
