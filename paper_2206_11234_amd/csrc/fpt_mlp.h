// fpt_mlp.h -- the learned drift bias r_theta(phi, N, N*) inside the step loop, on MFMA.
//
// Network (the learned proposal): inputs x = ((phi, k dN, N*) - mean) * inv_scale,
// h1 = tanh(W1 x + b1) in R^64, h2 = tanh(W2 h1 + b2) in R^64, r = out_scale (w3 . h2 + b3).
// Weights and biases are bfloat16 (4481 values, row-major W[out][in]); products are exact in
// binary32 and accumulate in binary32 on the matrix cores; activations (tanh_act, accurate to
// the bfloat16 they are rounded to) enter the next layer as bfloat16.
//
// Mapping onto v_mfma_f32_32x32x16_bf16 (A 32x16, B 16x32, D 32x32): the 64 lanes of a wave
// are 64 trajectories and form the N dimension (two N-blocks of 32 columns); hidden units are
// the M dimension.  Each layer computes H^T = W X^T, so the accumulator lane l holds column
// l % 32 (one trajectory of N-block nb) and rows (v%4) + 8(v/4) + 4(l/32), v = 0..15.  The next
// layer's B operand needs, in the same lane, 8 K-slots of that same column: a register-only
// repacking if the K index of layer 2 (and 3) enumerates hidden units in the order the
// accumulator holds them; W2 and w3 are loaded with their columns permuted to that order.
// Biases ride on a fifth K-block whose B operand is 1 in one slot.  Layer 1 has K = 3 inputs
// plus a constant 1 (bias); lanes 0-31 feed N-block 0 from K-slots 0..3 and lanes 32-63 feed
// N-block 1 from K-slots 8..11 (the A tile carries W1 in both), so no lane reads another's state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MLP_H = 64;
// offsets (in bfloat16 elements) of the parameter block
constexpr int MLP_W1 = 0, MLP_B1 = 192, MLP_W2 = 256, MLP_B2 = 4352, MLP_W3 = 4416, MLP_B3 = 4480;
constexpr int MLP_N_PARAMS = 4481;

struct MlpConsts {
    float in_mean[3], in_inv[3];
    float out_scale;
    float target_N;
};

// hidden unit held at K-slot (kb, half h, s) of a layer fed by an accumulator pair (mb = kb/2):
// register v = 8 (kb % 2) + s of block mb, row (v%4) + 8 (v/4) + 4 h.
__device__ __forceinline__ int unit_of_slot(int kb, int h, int s) {
    const int v = 8 * (kb & 1) + s;
    return 32 * (kb >> 1) + (v & 3) + 8 * (v >> 2) + 4 * h;
}

__device__ __forceinline__ __bf16 bf_at(const uint16_t *p, int i) {
    return __builtin_bit_cast(__bf16, p[i]);
}

struct MlpTiles {
    bf16x8 a1[2];      // layer 1, M-blocks 0/1 (K: inputs 0..2, bias at 3; copied at 8..11)
    bf16x8 a2[2][5];   // layer 2, M-blocks x K-blocks (K-block 4: bias)
    bf16x8 a3[5];      // layer 3, row 0 only (K-block 4: bias)
};

// Each lane loads the A-operand values it holds (done once per wave).
__device__ __forceinline__ void mlp_load_tiles(const uint16_t *__restrict__ P, MlpTiles &T) {
    const int l = __lane_id();
    const int h = l >> 5, i = l & 31;
    const __bf16 z = __builtin_bit_cast(__bf16, (uint16_t)0);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const int u = 32 * mb + i;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            __bf16 v = z;
            if (s < 3) v = bf_at(P, MLP_W1 + u * 3 + s);
            else if (s == 3) v = bf_at(P, MLP_B1 + u);
            T.a1[mb][s] = v;
        }
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int s = 0; s < 8; ++s) T.a2[mb][kb][s] = bf_at(P, MLP_W2 + u * 64 + unit_of_slot(kb, h, s));
#pragma unroll
        for (int s = 0; s < 8; ++s) T.a2[mb][4][s] = (h == 0 && s == 0) ? bf_at(P, MLP_B2 + u) : z;
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int s = 0; s < 8; ++s) T.a3[kb][s] = (i == 0) ? bf_at(P, MLP_W3 + unit_of_slot(kb, h, s)) : z;
#pragma unroll
    for (int s = 0; s < 8; ++s) T.a3[4][s] = (i == 0 && h == 0 && s == 0) ? bf_at(P, MLP_B3) : z;
}

// tanh x = 1 - 2 / (1 + e^{2x}) with the hardware base-2 exponential and reciprocal (binary32
// accuracy; the training kernels use it).
__device__ __forceinline__ float tanh_hw(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
    return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
}

// The sampler's activation, whose result is rounded to bfloat16: tanh to within 0.31 of a
// bfloat16 ulp of tanh x (before that rounding), from seven binary32 operations and no
// transcendental.  x is clamped to [-3.4, 3.4] (beyond it tanh rounds to +-1 in bfloat16) and
// tanh x = x q(|x|) with q of degree 5, the minimax fit of the error in bfloat16 ulps over
// [0, 3.4] and the clamped tail, evaluated by Horner's rule with fused multiply-adds.  The
// rounded activation equals the correctly rounded tanh in about 85 % of cases and is never
// more than one bfloat16 ulp from it.  The exponential form above needs two transcendentals
// at four times the cost of a fused multiply-add.
__device__ __forceinline__ float tanh_act(float x) {
    const float xc = __builtin_amdgcn_fmed3f(x, -3.4f, 3.4f);
    const float t = __builtin_fabsf(xc);
    float q = 0.005465357564389706f;
    q = __builtin_fmaf(q, t, -0.06311261653900146f);
    q = __builtin_fmaf(q, t, 0.27104586362838745f);
    q = __builtin_fmaf(q, t, -0.47482094168663025f);
    q = __builtin_fmaf(q, t, 0.02362865023314953f);
    q = __builtin_fmaf(q, t, 0.9999812841415405f);
    return q * xc;
}

// B operands of the next layer from an accumulator pair: tanh, round to bfloat16, repack.
__device__ __forceinline__ void act_to_operands(const f32x16 &d0, const f32x16 &d1, bf16x8 b[5]) {
    const int h = __lane_id() >> 5;
    const __bf16 z = __builtin_bit_cast(__bf16, (uint16_t)0);
    const __bf16 one = (__bf16)1.0f;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        b[0][s] = (__bf16)tanh_act(d0[s]);
        b[1][s] = (__bf16)tanh_act(d0[8 + s]);
        b[2][s] = (__bf16)tanh_act(d1[s]);
        b[3][s] = (__bf16)tanh_act(d1[8 + s]);
        b[4][s] = (h == 0 && s == 0) ? one : z;
    }
}

// r_theta for this lane's trajectory at (phi, N).  Every lane of the wave must call it
// together (the matrix instructions use all 64 lanes).
__device__ __forceinline__ float mlp_forward(const MlpTiles &T, const MlpConsts &M, float phi, float N) {
    const int l = __lane_id();
    const int h = l >> 5;
    const __bf16 z = __builtin_bit_cast(__bf16, (uint16_t)0);
    const float x0 = (phi - M.in_mean[0]) * M.in_inv[0];
    const float x1 = (N - M.in_mean[1]) * M.in_inv[1];
    const float x2 = (M.target_N - M.in_mean[2]) * M.in_inv[2];
    bf16x8 xin;
    xin[0] = (__bf16)x0;
    xin[1] = (__bf16)x1;
    xin[2] = (__bf16)x2;
    xin[3] = (__bf16)1.0f;
#pragma unroll
    for (int s = 4; s < 8; ++s) xin[s] = z;
    bf16x8 zero8;
#pragma unroll
    for (int s = 0; s < 8; ++s) zero8[s] = z;
    const bf16x8 bx0 = (h == 0) ? xin : zero8;    // N-block 0 columns come from lanes 0-31
    const bf16x8 bx1 = (h == 1) ? xin : zero8;    // N-block 1 columns from lanes 32-63
    const f32x16 zacc = {};
    // layer 1
    f32x16 d[2][2];
    d[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(T.a1[0], bx0, zacc, 0, 0, 0);
    d[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(T.a1[1], bx0, zacc, 0, 0, 0);
    d[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(T.a1[0], bx1, zacc, 0, 0, 0);
    d[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(T.a1[1], bx1, zacc, 0, 0, 0);
    // layer 2
    bf16x8 b[2][5];
    act_to_operands(d[0][0], d[1][0], b[0]);
    act_to_operands(d[0][1], d[1][1], b[1]);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            f32x16 acc = zacc;
#pragma unroll
            for (int kb = 0; kb < 5; ++kb) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(T.a2[mb][kb], b[nb][kb], acc, 0, 0, 0);
            d[mb][nb] = acc;
        }
    // layer 3: row 0 of the output holds w3 . h2 + b3 for the 32 columns of each N-block
    act_to_operands(d[0][0], d[1][0], b[0]);
    act_to_operands(d[0][1], d[1][1], b[1]);
    f32x16 o0 = zacc, o1 = zacc;
#pragma unroll
    for (int kb = 0; kb < 5; ++kb) {
        o0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(T.a3[kb], b[0][kb], o0, 0, 0, 0);
        o1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(T.a3[kb], b[1][kb], o1, 0, 0, 0);
    }
    // row 0 lives in lanes 0-31 (register 0): lane l < 32 has its own trajectory in o0,
    // lane l >= 32 reads o1 from lane l - 32
    const float other = __shfl(o1[0], l ^ 32, 64);
    const float o = (h == 0) ? o0[0] : other;
    return M.out_scale * o;
}

// The single-instance sampler keeps the operand tiles in LDS instead (17 fragments x 64 lanes x
// 16 B = 17 KiB per workgroup, one copy shared by its waves, read at each use) and evaluates the
// two N-blocks one after the other, so that its registers fit three waves per SIMD: the step
// loop is latency-bound and the third wave hides more of it than the register tiles save.  The
// matrix instructions and their operands are those of mlp_forward, so the result is the same bit
// for bit.
constexpr int MLP_N_FRAG = 17;
constexpr size_t MLP_TILE_LDS_BYTES = static_cast<size_t>(MLP_N_FRAG) * 64 * sizeof(bf16x8);

__device__ __forceinline__ void mlp_store_tiles_lds(const MlpTiles &T, bf16x8 *L) {
    const int l = __lane_id();
    L[0 * 64 + l] = T.a1[0];
    L[1 * 64 + l] = T.a1[1];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int kb = 0; kb < 5; ++kb) L[(2 + 5 * mb + kb) * 64 + l] = T.a2[mb][kb];
#pragma unroll
    for (int kb = 0; kb < 5; ++kb) L[(12 + kb) * 64 + l] = T.a3[kb];
}

__device__ __forceinline__ float mlp_forward_lds(const bf16x8 *L, const MlpConsts &M, float phi, float N) {
    const int l = __lane_id();
    const int h = l >> 5;
    const __bf16 z = __builtin_bit_cast(__bf16, (uint16_t)0);
    const float x0 = (phi - M.in_mean[0]) * M.in_inv[0];
    const float x1 = (N - M.in_mean[1]) * M.in_inv[1];
    const float x2 = (M.target_N - M.in_mean[2]) * M.in_inv[2];
    bf16x8 xin;
    xin[0] = (__bf16)x0;
    xin[1] = (__bf16)x1;
    xin[2] = (__bf16)x2;
    xin[3] = (__bf16)1.0f;
#pragma unroll
    for (int s = 4; s < 8; ++s) xin[s] = z;
    bf16x8 zero8;
#pragma unroll
    for (int s = 0; s < 8; ++s) zero8[s] = z;
    const f32x16 zacc = {};
    float out[2];
#pragma unroll 1
    for (int nb = 0; nb < 2; ++nb) {
        // N-block nb: the trajectories of lanes 32 nb .. 32 nb + 31
        const bf16x8 bx = (h == nb) ? xin : zero8;
        f32x16 d0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L[0 * 64 + l], bx, zacc, 0, 0, 0);
        f32x16 d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L[1 * 64 + l], bx, zacc, 0, 0, 0);
        bf16x8 b[5];
        act_to_operands(d0, d1, b);
        // keep each layer's LDS reads next to their use: hoisted together they would hold all
        // 17 tiles in registers again
        __builtin_amdgcn_sched_barrier(0);
        d0 = zacc;
        d1 = zacc;
#pragma unroll
        for (int kb = 0; kb < 5; ++kb) {
            d0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L[(2 + kb) * 64 + l], b[kb], d0, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L[(7 + kb) * 64 + l], b[kb], d1, 0, 0, 0);
        }
        act_to_operands(d0, d1, b);
        __builtin_amdgcn_sched_barrier(0);
        f32x16 o = zacc;
#pragma unroll
        for (int kb = 0; kb < 5; ++kb) o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L[(12 + kb) * 64 + l], b[kb], o, 0, 0, 0);
        out[nb] = o[0];
    }
    // row 0 lives in lanes 0-31: lane l < 32 has its own trajectory in N-block 0, lane l >= 32
    // reads N-block 1's from lane l - 32
    const float other = __shfl(out[1], l ^ 32, 64);
    const float o = (h == 0) ? out[0] : other;
    return M.out_scale * o;
}

}  // namespace fpt
