// rng.hpp -- counter-based random numbers on the device.
//
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): a pure function of a 128-bit counter
// and a 64-bit key, so every draw of a trial is fixed by (seed, replica, sweep,
// cell, round, purpose, index) and independent of the thread mapping.
// The paper (arXiv:1508.07077) names no generator; this layout is the
// library's determinism contract.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpmc {

enum Purpose : uint32_t {
    kGrid = 1,
    kSelect = 2,
    kTrans = 3,
    kRot = 4,
    kPoisson = 5,
    kDepl = 6,
    kCbFwd = 7,
    kCbRev = 8,
    kAccept = 9,
    kDeplShell = 10,
    kObsFv = 16,
};

constexpr uint32_t kNoCell = 0xFFFFFFFFu;

struct Words {
    uint32_t w0, w1, w2, w3;
};

// one 32x32 -> 64 multiply gives both halves (v_mad_u64_u32)
__device__ inline void mulhilo(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo)
{
    uint64_t p = static_cast<uint64_t>(a) * static_cast<uint64_t>(b);
    hi = static_cast<uint32_t>(p >> 32);
    lo = static_cast<uint32_t>(p);
}

// a ^ b ^ k in one VALU instruction (three-input bit operation, truth table
// 0x96 = odd parity); the round key k is wave-uniform
__device__ inline uint32_t xor3(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// Philox4x32-10 (Salmon et al., SC'11): per round two 32x32->64 multiplies
// and two three-way XORs; the key schedule runs on the scalar unit
__device__ inline Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, c0, hi0, lo0);
        mulhilo(0xCD9E8D57u, c2, hi1, lo1);
        c0 = xor3(hi1, c1, k0);
        c1 = lo1;
        c2 = xor3(hi0, c3, k1);
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        // the next round key is derived here, two scalar adds, rather than all
        // twenty kept live across the kernel (which spills scalar registers)
        asm volatile("" : "+s"(k0), "+s"(k1));
    }
    return Words{c0, c1, c2, c3};
}

// (w + 1/2) 2^-32, exact
__host__ __device__ inline double u01(uint32_t w) { return (static_cast<double>(w) + 0.5) * 0x1p-32; }

// 52-bit uniform (k + 1/2) 2^-52 with k = (w1 << 20) | (w0 >> 12), exact
__host__ __device__ inline double u52(uint32_t w0, uint32_t w1)
{
    uint64_t k = (static_cast<uint64_t>(w1) << 20) | static_cast<uint64_t>(w0 >> 12);
    return (static_cast<double>(k) + 0.5) * 0x1p-52;
}

// (2w + 1 - 2^32) 2^-32 in (-1, 1): (w + 1/2) 2^-31 - 1, every step exact
__host__ __device__ inline double sym01(uint32_t w) { return (static_cast<double>(w) + 0.5) * 0x1p-31 - 1.0; }

// multiply-shift choice in [0, n)
__host__ __device__ inline uint32_t pick(uint32_t w, uint32_t n)
{
    return static_cast<uint32_t>((static_cast<uint64_t>(w) * n) >> 32);
}

// Ball candidate from two words: three 21-bit fields, odd m in (-2^21, 2^21),
// accepted iff m0^2 + m1^2 + m2^2 < 2^42 (exact in FP64: each square < 2^42,
// the sum < 2^44).  Returns the odd integers as doubles.
__host__ __device__ inline bool ball3(uint32_t wa, uint32_t wb, double& m0, double& m1, double& m2)
{
    uint32_t f0 = wa & 0x1FFFFFu;
    uint32_t f1 = (wa >> 21) | ((wb & 0x3FFu) << 11);
    uint32_t f2 = (wb >> 10) & 0x1FFFFFu;
    m0 = static_cast<double>(static_cast<int32_t>(2u * f0 + 1u) - (1 << 21));
    m1 = static_cast<double>(static_cast<int32_t>(2u * f1 + 1u) - (1 << 21));
    m2 = static_cast<double>(static_cast<int32_t>(2u * f2 + 1u) - (1 << 21));
    // every partial sum is an integer below 2^44: the fused form is exact
    double s = fma(m0, m0, fma(m1, m1, m2 * m2));
    return s < 0x1p42;
}

// Point uniform in the shell r_i <= |e| < R0 from one block: direction by
// Marsaglia's method (two symmetric uniforms inside the unit disk), radius
// uniform in [r_i, R0) kept with probability r^2 / R0^2.  Plain IEEE
// + - * sqrt in a fixed order (compiled without contraction).
__host__ __device__ inline bool shell3(const Words& w, double r_i, double span, double R0sq, double& e0, double& e1,
                                       double& e2)
{
    double x1 = sym01(w.w0), x2 = sym01(w.w1);
    double s = x1 * x1 + x2 * x2;
    double r = r_i + span * u01(w.w2);
    bool ok = (s < 1.0) && (u01(w.w3) * R0sq < r * r);
    double h = 2.0 * sqrt(ok ? 1.0 - s : 1.0);
    e0 = r * (x1 * h);
    e1 = r * (x2 * h);
    e2 = r * (1.0 - 2.0 * s);
    return ok;
}

}  // namespace hpmc
