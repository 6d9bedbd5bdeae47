// fpt_device.h -- device-side arithmetic of one Euler-Maruyama step of the
// biased slow-roll Langevin equation, for gfx950.
//
// Method: arXiv:2206.11234, Sec. 2.1-2.3.  Every binary32 operation below is
// part of the step semantics shared with the CPU checker: the step count of a
// run is decided in binary32, so the order of operations and the places where
// fma is used are fixed (the library is built with -ffp-contract=off and no
// fast-math).  Reciprocals and square roots are fma-only Newton sequences:
// cheaper on gfx950 than the IEEE division/sqrt expansions and reproducible
// operation for operation on any IEEE binary32 machine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpt {

enum : int { POT_QUADRATIC = 0, POT_QUADRATIC_BUMP = 1, POT_FLAT = 2 };
enum : int { BIAS_NONE = 0, BIAS_NOISE_SCALED = 1, BIAS_POWER = 2, BIAS_MLP = 3 };
enum : int { ST_RUNNING = 0, ST_ENDED = 1, ST_CENSORED = 2, ST_ESCAPED = 3 };

// ---------------------------------------------------------------------------
// Counter-based noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// Ten rounds of two 32x32->64 multiplies; the key advances by the Weyl
// constants between rounds.  The key (the seed) is wave-uniform.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32->64 multiply per word gives both halves (v_mad_u64_u32)
        const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t lo_a = static_cast<uint32_t>(pa);
        const uint32_t hi_a = static_cast<uint32_t>(pa >> 32);
        const uint32_t lo_b = static_cast<uint32_t>(pb);
        const uint32_t hi_b = static_cast<uint32_t>(pb >> 32);
        // three-input xor in one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi_b, c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi_a, c3, k1, 0x96);
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
    }
    return U4{c0, c1, c2, c3};
}

// u = (2 (x >> 9) + 1) 2^-24: odd multiples of 2^-24 in (0, 1), exact in binary32.
// Formed as (1 + (x >> 9) 2^-23) + (2^-24 - 1): the first term is the float with exponent
// bits of 1.0 and mantissa x >> 9, the constant is exact, and the sum, a multiple of 2^-24
// below 1, is exact too.
__device__ __forceinline__ float uniform24(uint32_t x) {
    return __uint_as_float(0x3F800000u | (x >> 9)) + (0x1p-24f - 1.0f);
}

// 1/x for positive normal x: Newton-Raphson y <- fma(y, fma(-x, y, 1), y), three
// steps from the seed bits(0x7EF311C3 - bits(x)) (relative error < 5.1%); the result
// is within 0.51 ulp.  Division-free: only fma and integer subtract.  The seed negates the
// exponent by subtracting the float's bits from a constant (J. Blinn, "Floating-point
// tricks", IEEE CG&A 17(4), 1997); 0x7EF311C3 is a published tuning of that constant.
__device__ __forceinline__ float recip_f32(float x) {
    float y = __uint_as_float(0x7EF311C3u - __float_as_uint(x));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float e = __builtin_fmaf(-x, y, 1.0f);
        y = __builtin_fmaf(y, e, y);
    }
    return y;
}

// sqrt x for positive normal x: reciprocal square root by Newton-Raphson
// y <- fma(y, fma(-x/2, y*y, 1/2), y), three steps from bits(0x5F3759DF - (bits(x) >> 1)),
// then x*y; within 2 ulp.  The seed constant is the one of the Quake III Arena source (1999),
// analysed by C. Lomont, "Fast inverse square root" (2003).
__device__ __forceinline__ float sqrt_f32(float x) {
    float y = __uint_as_float(0x5F3759DFu - (__float_as_uint(x) >> 1));
    const float hx = 0.5f * x;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float yy = y * y;
        const float e = __builtin_fmaf(-hx, yy, 0.5f);
        y = __builtin_fmaf(y, e, y);
    }
    return x * y;
}

// ln x for positive normal x: x = 2^e f with f in (sqrt(1/2), sqrt 2], bit patterns
// (0x3F3504F3, 0x3FB504F3]; ln f = 2 atanh(s), s = (f-1)/(f+1), as the odd series to s^9;
// ln x = e ln2_hi + (e ln2_lo + ln f).  The split is done on the bits: b - 0x3F3504F4 has e
// in its arithmetic-shifted top bits and f - 0x3F3504F4 in its low 23.
__device__ __forceinline__ float log_f32(float x) {
    const int32_t ix = static_cast<int32_t>(__float_as_uint(x) - 0x3F3504F4u);
    const int e = ix >> 23;
    const float f = __uint_as_float((static_cast<uint32_t>(ix) & 0x007FFFFFu) + 0x3F3504F4u);
    const float s = (f - 1.0f) * recip_f32(f + 1.0f);
    const float z = s * s;
    float p = 1.0f / 9.0f;
    p = __builtin_fmaf(p, z, 1.0f / 7.0f);
    p = __builtin_fmaf(p, z, 1.0f / 5.0f);
    p = __builtin_fmaf(p, z, 1.0f / 3.0f);
    const float t = s + s;
    const float tz = t * z;
    const float lf = __builtin_fmaf(tz, p, t);
    const float ef = static_cast<float>(e);
    const float ln2_hi = 0.693145751953125f;
    const float ln2_lo = 1.42860682030941723212e-6f;
    return __builtin_fmaf(ef, ln2_hi, __builtin_fmaf(ef, ln2_lo, lf));
}

// cos(2 pi u), sin(2 pi u) for the uniform u = uniform24(x): nearest quarter q = rint(4u),
// r = u - q/4 in [-1/8, 1/8], Taylor polynomials of sin(2 pi r) to r^9 and cos(2 pi r) to r^10
// with coefficients (+-)(2 pi)^n/n!, then a quarter-turn rotation by q.
// q and r come from the bits of x: with y = x + 2^29 (mod 2^32), q = y >> 30 (mod 4) and
// r = (2 a + 1 - 2^21) 2^-24 for a = bits 9..29 of y, formed exactly as
// (0.5 + (2a + 1) 2^-24) - 0.625 -- the same values as the float reduction of u, for every x.
__device__ __forceinline__ void sincos2pi_bits(uint32_t x, float &c_out, float &s_out) {
    const uint32_t y = x + 0x20000000u;
    const uint32_t a = (y >> 9) & 0x1FFFFFu;
    const float r = __uint_as_float(0x3F000001u | (a << 1)) - 0.625f;
    const float r2 = r * r;
    float ps = __builtin_fmaf(42.058693944897653145f, r2, -76.7058597530613858416f);
    ps = __builtin_fmaf(ps, r2, 81.6052492760750542034f);
    ps = __builtin_fmaf(ps, r2, -41.341702240399760234f);
    ps = __builtin_fmaf(ps, r2, 6.28318530717958647692f);
    const float sn = ps * r;
    float pc = __builtin_fmaf(-26.4262567833743974529f, r2, 60.2446413718766603627f);
    pc = __builtin_fmaf(pc, r2, -85.456817206693727736f);
    pc = __builtin_fmaf(pc, r2, 64.939394022668291491f);
    pc = __builtin_fmaf(pc, r2, -19.7392088021787172377f);
    const float cs = __builtin_fmaf(pc, r2, 1.0f);
    // quarter-turn rotation by q = y >> 30, branch-free: odd q swaps (cos, sin); cos changes
    // sign for q = 1, 2 (bit 31 of y + 2^30) and sin for q = 2, 3 (bit 31 of y); IEEE negation
    // is the sign bit
    const bool swap = (y & 0x40000000u) != 0u;
    const float c0 = swap ? sn : cs;
    const float s0 = swap ? cs : sn;
    const uint32_t sign_c = (y + 0x40000000u) & 0x80000000u;
    const uint32_t sign_s = y & 0x80000000u;
    c_out = __uint_as_float(__float_as_uint(c0) ^ sign_c);
    s_out = __uint_as_float(__float_as_uint(s0) ^ sign_s);
}

// e^x for x <= 0 (x < -80 gives 0): n = rint(x / ln 2), r = x - n ln2 (two-part),
// Taylor series of e^r to r^7, times 2^n assembled in the exponent field.
__device__ __forceinline__ float exp_f32(float x) {
    const bool under = x < -80.0f;
    if (x > 0.0f) x = 0.0f;
    if (under) x = -80.0f;
    const float n = __builtin_rintf(x * 1.44269504088896340736f);
    float r = __builtin_fmaf(-n, 0.693145751953125f, x);
    r = __builtin_fmaf(-n, 1.42860682030941723212e-6f, r);
    float p = 1.0f / 5040.0f;
    p = __builtin_fmaf(p, r, 1.0f / 720.0f);
    p = __builtin_fmaf(p, r, 1.0f / 120.0f);
    p = __builtin_fmaf(p, r, 1.0f / 24.0f);
    p = __builtin_fmaf(p, r, 1.0f / 6.0f);
    p = __builtin_fmaf(p, r, 0.5f);
    p = __builtin_fmaf(p, r, 1.0f);
    p = __builtin_fmaf(p, r, 1.0f);
    const int ni = static_cast<int>(n);
    const float scale = __uint_as_float(static_cast<uint32_t>(ni + 127) << 23);
    const float y = p * scale;
    return under ? 0.0f : y;
}

// Four standard normals for steps 4j .. 4j+3 of run t: Box-Muller on (u0,u1), (u2,u3).
struct F4 {
    float a, b, c, d;
};

__device__ __forceinline__ F4 normals4(uint32_t j, uint64_t t, uint32_t stream, uint32_t key0, uint32_t key1) {
    // the key schedule is recomputed by scalar adds at each call: left to itself the compiler
    // hoists all twenty round keys into scalar registers and spills them to vector lanes
    asm volatile("" : "+s"(key0), "+s"(key1));
    const U4 x = philox4x32_10(j, static_cast<uint32_t>(t), static_cast<uint32_t>(t >> 32), stream, key0, key1);
    F4 out;
    {
        const float ua = uniform24(x.x);
        const float rho = sqrt_f32(-2.0f * log_f32(ua));
        float c, s;
        sincos2pi_bits(x.y, c, s);
        out.a = rho * c;
        out.b = rho * s;
    }
    {
        const float ua = uniform24(x.z);
        const float rho = sqrt_f32(-2.0f * log_f32(ua));
        float c, s;
        sincos2pi_bits(x.w, c, s);
        out.c = rho * c;
        out.d = rho * s;
    }
    return out;
}

// ---------------------------------------------------------------------------
// Per-instance binary32 step constants (rounded once on the host from the
// binary64 inputs).
// ---------------------------------------------------------------------------
struct StepConsts {
    float dN, sq, hdN, cm;        // dN, sqrt dN, dN/2, m/(2 pi sqrt 6) (flat: S)
    float a, phi0, inv_w2, inv_2w2;
    float A, phi_end, phi_uv, two_uv;
    float phi_esc, phi_in;
    int32_t p;
    uint32_t k_max;
};

// D = -V'/V and S = sqrt(V/3)/(2 pi) at phi (Sec. 2.3).
template <int POT>
__device__ __forceinline__ void drift_noise(const StepConsts &C, float phi, float &D, float &S) {
    if constexpr (POT == POT_QUADRATIC) {
        const float y = recip_f32(phi);
        const float d = y + y;          // 2/phi
        D = -d;
        S = C.cm * phi;
    } else if constexpr (POT == POT_QUADRATIC_BUMP) {
        const float dphi = phi - C.phi0;
        const float e2 = dphi * dphi;
        const float x = -(e2 * C.inv_2w2);
        const float g = exp_f32(x);
        const float ag = C.a * g;
        const float one_ag = 1.0f + ag;
        const float num = (dphi * C.inv_w2) * ag;
        const float corr = num * recip_f32(one_ag);
        const float y = recip_f32(phi);
        const float d = y + y;
        D = corr - d;
        S = (C.cm * phi) * sqrt_f32(one_ag);
    } else {
        D = 0.0f;
        S = C.cm;
    }
}

// r = B/S in noise units (Sec. 2.3 eq. eq_importance_sampling_amplitude_general
// with f = S, and the power law of Sec. 3.4).
template <int BIAS>
__device__ __forceinline__ float bias_ratio(const StepConsts &C, float phi, float S) {
    if constexpr (BIAS == BIAS_NOISE_SCALED) {
        return C.A;
    } else if constexpr (BIAS == BIAS_POWER) {
        float pw = 1.0f;
        for (int i = 0; i < C.p; ++i) pw = pw * phi;
        return (C.A * pw) * recip_f32(S);
    } else {
        return 0.0f;
    }
}

// Status of a run that has stopped, from where it stopped: the end surface takes precedence
// over the step cap, the cap over escape (Sec. 2.1, Sec. 3).
__device__ __forceinline__ int final_status(const StepConsts &C, float phi, uint32_t k) {
    if (phi <= C.phi_end) return ST_ENDED;
    if (k >= C.k_max) return ST_CENSORED;
    return (phi > C.phi_esc) ? ST_ESCAPED : ST_RUNNING;
}

// One Euler-Maruyama step of the biased Langevin equation (Sec. 2.2 eq. eq_euler_maruyam_modified,
// drift, noise and bias at the pre-step point), the weight increment
// -r (r dN/2 + sqrt(dN) xi) accumulated in binary64, reflection above phi_UV, and the end /
// cap / escape tests (Sec. 2.1, Sec. 3).  run stays true while none of the three tests fires;
// final_status() names the one that did.  r_net is the bias when it comes from the learned
// network.  Returns r and writes sqrt(dN) xi, which the training replay reuses.
template <int POT, int BIAS>
__device__ __forceinline__ float em_step(const StepConsts &C, float &phi, uint32_t &k, double &lw, bool &run, float xi,
                                         float r_net, float &sxi) {
    float D, S;
    drift_noise<POT>(C, phi, D, S);
    float drift, r = 0.0f;
    if constexpr (BIAS == BIAS_NONE) {
        drift = D;
    } else {
        if constexpr (BIAS == BIAS_MLP) r = r_net;
        else r = bias_ratio<BIAS>(C, phi, S);
        const float B = r * S;
        drift = D + B;
    }
    // The whole increment (D + B) dN + S sqrt(dN) xi is formed first and rounded onto phi once.
    // Adding the deterministic part to phi on its own would round it to phi's grid every step:
    // at small dN it spans only tens of ulps of phi, and its fraction of an ulp changes so slowly
    // with phi that the rounding error repeats from step to step instead of averaging out.
    sxi = C.sq * xi;
    const float inc_phi = __builtin_fmaf(S, sxi, drift * C.dN);
    float nphi = phi + inc_phi;
    if constexpr (BIAS != BIAS_NONE) {
        const float inc = __builtin_fmaf(r, C.hdN, sxi);
        const float dlw = -(r * inc);
        lw += static_cast<double>(dlw);
    }
    // Reflection x -> 2 phi_UV - x above the wall, as a minimum: 2 phi_UV is exact and rounding
    // is monotone, so fl(2 phi_UV - x) <= phi_UV < x exactly when x > phi_UV (and >= x otherwise);
    // with no wall 2 phi_UV is +inf and the minimum is x.
    phi = __builtin_fminf(nphi, C.two_uv - nphi);
    k += 1;
    run = !(phi <= C.phi_end) && (k < C.k_max) && !(phi > C.phi_esc);
    return r;
}

}  // namespace fpt
