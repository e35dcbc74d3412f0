// lbm_device.h -- device-side lattice algebra of the TRT-R D2Q9 step (gfx950).
//
// Everything here works in lattice units: velocities are e_i / c (components in {-1, 0, 1}), u is
// stored as u dt / dx, c_s^2 = 1/3, and the relaxation is parameterised by k = tau1 - 1/2 =
// kappa / (c_s^2 dt) (Sec. 2.4).  In these units one step of Sec. 2.2, Eq. (14) is
//
//   P_i = w_i [ a0 + 3 e_i . a1 + 9/2 (e_ia e_ib - delta_ab / 3) a2_ab
//               + 27/2 (H_i,xxy a3_xxy + H_i,xyy a3_xyy) ]
//
// with the post-collision Hermite coefficients
//   a0    = phi + s                       (s = dt S + dt^2/2 dS/dt, Eq. (3) and its derivative)
//   a1    = phi u + w1 B + beta (A + u s)  (B = j - phi u: first-order neq moment, Eq. (8);
//                                           A = phi u.grad u: auxiliary term, Eq. (16))
//   a2_ab = phi u_a u_b + w2 N_ab         (N_ab = Pi_ab - phi delta_ab/3 - phi u_a u_b, Eq. (13))
//   a3    = phi u_x^2 u_y, phi u_x u_y^2  (third-order equilibrium; the only non-zero third-order
//                                           Hermite components on D2Q9, Eq. (6))
// where w1 = 1 - 1/tau1, w2 = 1 - 1/tau2 and beta = 1 - 1/(2 tau1).  This is Eq. (12) written in
// moment space: Hermite orthogonality turns the projections of Eqs. (8) and (13) into the raw
// moments j and Pi, and the relaxed neq content above second order is zero.  Opposite velocities
// share the even part and flip the odd part, which is the symmetric/antisymmetric (TRT) split.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// D2Q9 velocity order of the population planes.
constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};  // e_kOpp[i] = -e_i
constexpr double kW[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// w3 = 1 - 1/tau3 relaxes the third-order non-equilibrium moments (MRT-R, Eq. (11)); 0 is TRT-R.
template <class M>
struct Relax {
    M w1, w2, beta, w3;
};

// k = tau1 - 1/2 (lattice diffusivity), lambda = magic parameter.
template <class M>
__device__ __forceinline__ Relax<M> relax_from_k(M k, M lambda, M w3)
{
    const M tau1 = M(0.5) + k;
    const M tau2 = M(0.5) + lambda / k;
    Relax<M> r;
    r.w1 = M(1) - M(1) / tau1;
    r.w2 = M(1) - M(1) / tau2;
    r.beta = M(1) - M(0.5) / tau1;
    r.w3 = w3;
    return r;
}

// P_i from the Hermite coefficients (see the header comment).
template <class M>
__device__ __forceinline__ void reconstruct(M a0, M a1x, M a1y, M a2xx, M a2yy, M a2xy, M a3xxy,
                                            M a3xyy, M (&P)[9])
{
    const M w0 = M(4.0 / 9.0), wa = M(1.0 / 9.0), wd = M(1.0 / 36.0);
    P[0] = w0 * (a0 - M(1.5) * (a2xx + a2yy));
    const M ex = a0 + M(3) * a2xx - M(1.5) * a2yy;
    const M ox = M(3) * a1x - M(4.5) * a3xyy;
    P[1] = wa * (ex + ox);
    P[3] = wa * (ex - ox);
    const M ey = a0 + M(3) * a2yy - M(1.5) * a2xx;
    const M oy = M(3) * a1y - M(4.5) * a3xxy;
    P[2] = wa * (ey + oy);
    P[4] = wa * (ey - oy);
    const M ed = a0 + M(3) * (a2xx + a2yy);
    const M e57 = ed + M(9) * a2xy;
    const M o57 = M(3) * (a1x + a1y) + M(9) * (a3xxy + a3xyy);
    P[5] = wd * (e57 + o57);
    P[7] = wd * (e57 - o57);
    const M e68 = ed - M(9) * a2xy;
    const M o68 = M(3) * (a1y - a1x) + M(9) * (a3xxy - a3xyy);
    P[6] = wd * (e68 + o68);
    P[8] = wd * (e68 - o68);
}

// Third-order Hermite equilibrium (Eq. (6)) in lattice units.
template <class M>
__device__ __forceinline__ void equilibrium(M phi, M ux, M uy, M (&P)[9])
{
    const M pux = phi * ux, puy = phi * uy;
    reconstruct<M>(phi, pux, puy, pux * ux, puy * uy, pux * uy, pux * ux * uy, pux * uy * uy, P);
}

// TRT-R collision + source + auxiliary term for one node (Eq. (14) without the streaming).
//   g: pre-collision populations; (ux, uy): lattice velocity; r: relaxation; (Ax, Ay): auxiliary
//   vector A (already multiplied by phi); s: dt S + dt^2/2 dS/dt (0 without a source).
template <class M, bool MRT = false>
__device__ __forceinline__ void collide(const M (&g)[9], M ux, M uy, const Relax<M> &r, M Ax, M Ay,
                                        M s, M (&P)[9])
{
    const M phi = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
    const M jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const M jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const M sd = (g[5] + g[6]) + (g[7] + g[8]);
    const M pxx = g[1] + g[3] + sd;
    const M pyy = g[2] + g[4] + sd;
    const M pxy = (g[5] + g[7]) - (g[6] + g[8]);
    const M pux = phi * ux, puy = phi * uy;
    const M euxx = pux * ux, euyy = puy * uy, euxy = pux * uy;  // phi u_a u_b
    const M third = phi * M(1.0 / 3.0);
    const M a1x = pux + r.w1 * (jx - pux) + r.beta * (Ax + ux * s);
    const M a1y = puy + r.w1 * (jy - puy) + r.beta * (Ay + uy * s);
    const M a2xx = euxx + r.w2 * (pxx - third - euxx);
    const M a2yy = euyy + r.w2 * (pyy - third - euyy);
    const M a2xy = euxy + r.w2 * (pxy - euxy);
    // third Hermite moments: the equilibrium's phi u_x^2 u_y, phi u_x u_y^2 (TRT-R), plus for MRT-R
    // w3 times the non-equilibrium part sum_i H_i,xxy g_i - phi u_x^2 u_y, H_xxy = e_y (e_x^2 - 1/3)
    M a3xxy = euxx * uy, a3xyy = euxy * uy;
    if constexpr (MRT) {
        const M qxxy = (g[5] + g[6]) - (g[7] + g[8]);
        const M qxyy = (g[5] - g[6]) - (g[7] - g[8]);
        a3xxy += r.w3 * (qxxy - jy * M(1.0 / 3.0) - a3xxy);
        a3xyy += r.w3 * (qxyy - jx * M(1.0 / 3.0) - a3xyy);
    }
    reconstruct<M>(phi + s, a1x, a1y, a2xx, a2yy, a2xy, a3xxy, a3xyy, P);
}

// ---- population storage codecs --------------------------------------------------------------

struct StoreF64 {
    using T = double;
};
struct StoreF32 {
    using T = float;
};
struct StoreF16S {
    using T = _Float16;
};
struct StoreF16SR {  // the F16S code, written with stochastic rounding
    using T = _Float16;
};

// F16S codec constants: h = f16((g - w_i phi_ref) * 2^k); g = h * 2^-k + w_i phi_ref.
struct F16Params {
    float scale, inv_scale;
    float wref[27];  // w_i phi_ref per velocity (9, 19 or 27 used)
    uint64_t seed;   // F16SR: start state of the rounding stream
    int64_t nodes;   // F16SR: nodes of the lattice (the stream's stride per time level)
};

// ---- random bits of the stochastic rounding (F16SR) ------------------------------------------
//
// Stochastic rounding (Croci & Giles 2020 studied it for low-precision time stepping of the heat
// equation) rounds a value to one of its two FP16 neighbours with probability proportional to its
// distance from the other, so the rounding error has zero mean and small updates are not lost on
// average.  The random bits are a pure function of (time level, node): every launch shape, tile
// order and kernel gives the same codes.  Node j of a lattice of n nodes at time level t takes
// outputs 2(t n + j) and 2(t n + j) + 1 of SplitMix64 (Steele, Lea & Flood 2014: output k of the
// generator started at state s is mix(s + (k + 1) gamma)), 128 bits hi:lo, and population i uses bits
// 13 i .. 13 i + 12 (117 bits for the nine) as its integer r.  Thirteen bits are what FP32 carries
// below the FP16 unit in the last place (24 - 11 significand bits), so the rounding of a normal FP16
// value is exactly unbiased for its FP32 input.

constexpr uint64_t kSplitMixGamma = 0x9e3779b97f4a7c15ull;

__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

struct NoBits {};  // what the deterministic codecs take in place of random bits
struct NodeBits {
    uint64_t lo, hi;  // stream outputs 2(t n + j) and 2(t n + j) + 1
};

// The random operand of the conversion below for population i: its bits 19..31 are the complement of
// bits 13 i .. 13 i + 12 of hi:lo (i.e. 2^13 - 1 - r); the conversion reads no other bits.  i is a
// compile-time constant once the callers' loops unroll, so this is one shift or funnel shift.
__device__ __forceinline__ uint32_t sr_operand(const NodeBits &b, int i)
{
    const int sh = 13 * i - 19;
    const uint64_t lo = ~b.lo, hi = ~b.hi;
    if (sh < 0) return (uint32_t)(lo << -sh);
    if (sh + 32 <= 64) return (uint32_t)(lo >> sh);
    if (sh >= 64) return (uint32_t)(hi >> (sh - 64));
    return (uint32_t)((lo >> sh) | (hi << (64 - sh)));
}

// FP32 -> FP16 with stochastic rounding, by gfx950's v_cvt_sr_f16_f32: with lo <= |s| < lo + ulp the
// FP16 neighbours of |s| and m the 13 bits of |s| just below the FP16 spacing (m = floor(2^13 (|s| -
// lo) / ulp); bits further down, which exist only in the FP16 subnormal range, are dropped), the
// conversion adds the top 13 bits R of its random operand to m and keeps the carry: |s| goes up iff
// m + R >= 2^13.  With R = 2^13 - 1 - r that is r < m: probability m / 2^13, exactly (|s| - lo) / ulp
// for FP16 normal values.  Rounding up from 65504, or any |s| from 65536 on, gives infinity; NaN, the
// infinities and signed zeros are kept.  (Measured on the device over 2^17 value/operand pairs and the
// special values; the tests hold every stored code to this rule, bitwise.)
__device__ __forceinline__ _Float16 sr_half(float s, uint32_t operand)
{
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const half2_t z = {(_Float16)0.0f, (_Float16)0.0f};
    return __builtin_amdgcn_cvt_sr_f16_f32(z, s, operand, false)[0];
}

// A codec decodes a stored element to the math type and encodes one back.  `bits(f, level, row_node, x)`
// gives what enc needs besides the value: the random bits of node row_node + x (row_node = y nx) at time
// level `level` (the step count of the state being written) for F16SR, nothing for the others;
// kStochastic says whether a kernel has to track the time level.
template <class St, class M>
struct Codec;

template <class M>
struct DetCodecBase {
    static constexpr bool kStochastic = false;
    using Bits = NoBits;
    __device__ __forceinline__ static NoBits bits(const F16Params &, int64_t, int64_t, unsigned) { return {}; }
};

template <>
struct Codec<StoreF64, double> : DetCodecBase<double> {
    __device__ __forceinline__ static double dec(double v, int, const F16Params &) { return v; }
    __device__ __forceinline__ static double enc(double v, int, const F16Params &, NoBits = {}) { return v; }
};
template <>
struct Codec<StoreF64, float> : DetCodecBase<float> {
    __device__ __forceinline__ static float dec(double v, int, const F16Params &) { return (float)v; }
    __device__ __forceinline__ static double enc(float v, int, const F16Params &, NoBits = {}) { return (double)v; }
};
template <>
struct Codec<StoreF32, float> : DetCodecBase<float> {
    __device__ __forceinline__ static float dec(float v, int, const F16Params &) { return v; }
    __device__ __forceinline__ static float enc(float v, int, const F16Params &, NoBits = {}) { return v; }
};
template <>
struct Codec<StoreF16S, float> : DetCodecBase<float> {
    __device__ __forceinline__ static float dec(_Float16 v, int i, const F16Params &c)
    {
        return (float)v * c.inv_scale + c.wref[i];
    }
    __device__ __forceinline__ static _Float16 enc(float v, int i, const F16Params &c, NoBits = {})
    {
        // The shift is a plain FP32 subtraction of the rounded value v (never fused with the product
        // that formed v), so the stored code does not depend on how the caller's arithmetic is
        // contracted; the power-of-two scale is exact; v_cvt_f16_f32 rounds to nearest even.
#pragma clang fp contract(off)
        return (_Float16)((v - c.wref[i]) * c.scale);
    }
};
template <>
struct Codec<StoreF16SR, float> {
    static constexpr bool kStochastic = true;
    using Bits = NodeBits;
    // Node j = row_node + x: the generator state of output 2(level n + j) is seed + (2(level n + j) + 1)
    // gamma, split into a part uniform over the row and 2 gamma x, which stays in registers along a walk.
    __device__ __forceinline__ static NodeBits bits(const F16Params &c, int64_t level, int64_t row_node, unsigned x)
    {
        const uint64_t s0 = c.seed + kSplitMixGamma * (2u * ((uint64_t)level * (uint64_t)c.nodes + (uint64_t)row_node) + 1u) +
                            (2u * kSplitMixGamma) * (uint64_t)x;
        return {splitmix64_mix(s0), splitmix64_mix(s0 + kSplitMixGamma)};
    }
    __device__ __forceinline__ static float dec(_Float16 v, int i, const F16Params &c)
    {
        return (float)v * c.inv_scale + c.wref[i];
    }
    __device__ __forceinline__ static _Float16 enc(float v, int i, const F16Params &c, const NodeBits &b)
    {
        // the same FP32 value as F16S encodes (shift not fused, exact scale), rounded stochastically
        float t;
        {
#pragma clang fp contract(off)
            t = (v - c.wref[i]) * c.scale;
        }
        return sr_half(t, sr_operand(b, i));
    }
};

// ---- compensated FP64 accumulation (Neumaier / TwoSum) ------------------------------------

struct CSum {
    double s, c;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}
__device__ __forceinline__ void csum_add(CSum &x, double v)
{
    double s, e;
    two_sum(x.s, v, s, e);
    x.s = s;
    x.c += e;
}
__device__ __forceinline__ CSum csum_merge(CSum a, CSum b)
{
    double s, e;
    two_sum(a.s, b.s, s, e);
    CSum r;
    r.s = s;
    r.c = a.c + b.c + e;
    return r;
}

}  // namespace lbm
