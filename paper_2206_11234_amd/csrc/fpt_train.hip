// fpt_train.hip -- training kernels of the learned proposal.
//
// The paper leaves the choice of the best bias open (Sec. 3.4); the learned proposal is trained
// to minimise the second moment of the importance weights of runs that end in a target window
// B*:  M2(theta) = E_0[w_0 w_theta 1_B*], estimated on paths drawn once from the current
// proposal theta_0 (Sec. 2.2: the weight is the ratio of the target and sample path densities).
// On a fixed path, step k's target-measure noise increment is eta_k = r_0,k dN + sqrt(dN) xi_k,
// and the weight the same path would have under a candidate bias held over groups of E steps
// is  ln w_theta = sum_e [ -r_theta(x_e) H_e + r_theta(x_e)^2 n_e dN/2 ],  H_e = sum of eta over
// group e, n_e its length.  So a path reduces to records (phi_e, k_e, H_e, n_e):
//
//   fpt_record_kernel    replays paths under theta_0 (the sampler's own step and network code,
//                        so the replay reproduces the sampled runs) and writes their records
//                        (every group's, or every stride-th group's, each then standing for
//                        stride groups: an unbiased estimate of the sums over a path);
//   fpt_train_fwd_kernel r_theta per record (binary32 network on the master weights), per-path
//                        sum of ln w_theta in binary64 (one workgroup per path, fixed order);
//   fpt_train_softmax_kernel  c_i = w_0,i w_theta,i / sum_j w_0,j w_theta,j and log M2, or for
//                        the cross-entropy objective c_i = w_0,i / sum_j w_0,j and
//                        sum_i c_i ln w_theta,i (the KL divergence of the proposal from the
//                        target restricted to the window, up to a constant); w_0 may be
//                        tempered to w_0^beta;
//   fpt_train_bwd_kernel gradient of the objective: per record (forward recomputed in place) the
//                        coefficient
//                        c_i (r n dN - H) out_scale multiplies d(w3.h2 + b3)/d theta; each lane
//                        back-propagates one record, and the weight gradient of the 64x64 layer,
//                        a contraction over the 64 records of a wave, runs on
//                        v_mfma_f32_32x32x2f32 from LDS tiles;
//   fpt_train_reduce_kernel  per-workgroup partial gradients summed in a fixed order (binary64);
//   fpt_adam_kernel      Adam (Kingma & Ba) on the binary32 master weights, then the bfloat16
//                        copy that the sampler reads.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fpt_kernels.h"
#include "fpt_train.h"

namespace fpt {

// ---------------------------------------------------------------------------
// replay into records
// ---------------------------------------------------------------------------
template <int POT, int BIAS>
__global__ __launch_bounds__(256) void fpt_record_kernel(RecordArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool have = i < a.n_paths;
    const StepConsts C = a.inst.c;
    MlpTiles tiles;
    if constexpr (BIAS == BIAS_MLP) mlp_load_tiles(a.mlp_params, tiles);
    const MlpConsts mc = a.inst.mlp;
    const uint64_t t = have ? a.t_ids[i] : 0;
    const uint64_t base = have ? a.rec_off[i] : 0;
    const uint64_t cap = have ? a.rec_off[i + 1] - base : 0;
    const uint32_t emask = static_cast<uint32_t>(a.group - 1);
    float phi = C.phi_in;
    uint32_t k = 0;
    double lw = 0.0;
    bool run = have;
    float H = 0.0f, phi_e = phi;
    uint32_t k_e = 0, n_e = 0;
    uint64_t n_rec = 0;
    // the sampling network (if any) is evaluated every E steps, wave-wide: a pass covers
    // max(4, E) steps, so every lane is at a multiple of the pass length at its start
    const int E = (BIAS == BIAS_MLP) ? a.mlp_every : 4;
    const int n_q = E > 4 ? E >> 2 : 1;
    while (__any(run)) {
        float r_mlp = 0.0f;
        for (int q = 0; q < n_q; ++q) {
            if constexpr (BIAS == BIAS_MLP) {
                if (q * 4 % E == 0) r_mlp = mlp_forward(tiles, mc, phi, static_cast<float>(k) * C.dN);
            }
            F4 z{};
            if (run) z = normals4(k >> 2, t, a.inst.stream, a.key0, a.key1);
            const float zs[4] = {z.a, z.b, z.c, z.d};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if constexpr (BIAS == BIAS_MLP) {
                    if (s > 0 && E == 1) r_mlp = mlp_forward(tiles, mc, phi, static_cast<float>(k) * C.dN);
                }
                if (run) {
                    if ((k & emask) == 0) {
                        phi_e = phi;
                        k_e = k;
                        H = 0.0f;
                        n_e = 0;
                    }
                    float sxi;
                    const float r = em_step<POT, BIAS>(C, phi, k, lw, run, zs[s], r_mlp, sxi);
                    H = H + __builtin_fmaf(r, C.dN, sxi);
                    n_e += 1;
                    if ((k & emask) == 0 || !run) {
                        const uint32_t grp = k_e / static_cast<uint32_t>(a.group);
                        if (grp % static_cast<uint32_t>(a.stride) == 0 && n_rec < cap) {
                            TrainRec R;
                            R.phi = phi_e;
                            R.k = k_e;
                            R.H = H;
                            R.pn = (i << 5) | n_e;
                            a.rec[base + n_rec] = R;
                        }
                        if (grp % static_cast<uint32_t>(a.stride) == 0) n_rec += 1;
                    }
                }
            }
        }
    }
    if (have) {
        a.k_out[i] = k;
        a.lw_out[i] = lw;
        a.st_out[i] = final_status(C, phi, k);
        a.n_rec_out[i] = n_rec;
    }
}

// ---------------------------------------------------------------------------
// the network being trained (binary32, master weights, no roundings)
// ---------------------------------------------------------------------------
// The weights are loop-invariant in the record loops; reading them through a pointer offset
// by a zero the compiler cannot see through keeps it from hoisting thousands of them out of
// the loop into registers (they stay uniform, scalar loads).
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

__device__ __forceinline__ void net_inputs(const MlpConsts &M, float phi, uint32_t k, float dN, float x[3]) {
    const float N = static_cast<float>(k) * dN;
    x[0] = (phi - M.in_mean[0]) * M.in_inv[0];
    x[1] = (N - M.in_mean[1]) * M.in_inv[1];
    x[2] = (M.target_N - M.in_mean[2]) * M.in_inv[2];
}

__device__ __forceinline__ void net_layer1(const float *__restrict__ th, const float x[3], float h1[64]) {
#pragma unroll
    for (int u = 0; u < 64; ++u) {
        float s = th[NET_B1 + u];
        s = __builtin_fmaf(th[NET_W1 + 3 * u + 0], x[0], s);
        s = __builtin_fmaf(th[NET_W1 + 3 * u + 1], x[1], s);
        s = __builtin_fmaf(th[NET_W1 + 3 * u + 2], x[2], s);
        h1[u] = tanh_hw(s);
    }
}

__device__ __forceinline__ float net_unit2(const float *__restrict__ th, int u, const float h1[64]) {
    float s = th[NET_B2 + u];
#pragma unroll
    for (int v = 0; v < 64; ++v) s = __builtin_fmaf(th[NET_W2 + 64 * u + v], h1[v], s);
    return tanh_hw(s);
}

// ---------------------------------------------------------------------------
// forward: r per record, ln w_theta per path
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fpt_train_fwd_kernel(TrainArgs a, const float *__restrict__ th0) {
    __shared__ double red[256];
    const int i = blockIdx.x;
    const uint64_t e0 = a.rec_off[i], e1 = a.rec_off[i + 1];
    const double hdN = 0.5 * static_cast<double>(a.dN);
    double s = 0.0;
    for (uint64_t b = e0; b < e1; b += blockDim.x) {
        const uint64_t e = b + threadIdx.x;
        if (e >= e1) break;
        const float *th = th0 + opaque_zero();
        const TrainRec R = a.rec[e];
        float x[3], h1[64];
        net_inputs(a.mc, R.phi, R.k, a.dN, x);
        net_layer1(th, x, h1);
        float o = 0.0f;
#pragma unroll 1
        for (int u = 0; u < 64; ++u) o = __builtin_fmaf(th[NET_W3 + u], net_unit2(th, u, h1), o);
        const float r = a.mc.out_scale * (o + th0[NET_B3]);
        const double rd = static_cast<double>(r);
        const double n = static_cast<double>(R.pn & 31u);
        s += (-rd * static_cast<double>(R.H) + rd * rd * n * hdN) * static_cast<double>(a.rec_weight);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.lw_theta[i] = red[0];
}

// ---------------------------------------------------------------------------
// softmax over paths and log M2
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void fpt_train_softmax_kernel(TrainArgs a) {
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    const double use_t = a.objective == 0 ? 1.0 : 0.0;
    double m = -INFINITY;
    const double beta = static_cast<double>(a.temper);
    for (int i = tid; i < a.n_paths; i += 1024) m = fmax(m, beta * a.lw0[i] + use_t * a.lw_theta[i]);
    red[tid] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
        __syncthreads();
    }
    const double M = red[0];
    __syncthreads();
    double s = 0.0;
    for (int i = tid; i < a.n_paths; i += 1024) s += exp(beta * a.lw0[i] + use_t * a.lw_theta[i] - M);
    red[tid] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double S = red[0];
    __syncthreads();
    double ce = 0.0;
    for (int i = tid; i < a.n_paths; i += 1024) {
        const double c = exp(beta * a.lw0[i] + use_t * a.lw_theta[i] - M) / S;
        a.c[i] = c;
        ce += c * a.lw_theta[i];
    }
    red[tid] = ce;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) a.loss[0] = a.objective == 0 ? M + log(S) - log(a.n_total) : red[0];
}

// ---------------------------------------------------------------------------
// backward: one wave per workgroup, 64 records per tile
// ---------------------------------------------------------------------------
constexpr int TS = 65;  // padded row stride of the [sample][unit] LDS tiles

typedef float f32x16v __attribute__((ext_vector_type(16)));

// The three 64x64x64 contractions of a tile run on v_mfma_f32_32x32x2f32 (binary32 products and
// sums, like the rest of the training network).  Operand layout of that instruction, per lane l
// and k-step: A[m = l & 31][k = l >> 5], B[k = l >> 5][n = l & 31]; accumulator element q of lane l
// is D[m = (q & 3) + 8 (q >> 2) + 4 (l >> 5)][n = l & 31] of its 32x32 block.
__device__ __forceinline__ int acc_row(int q, int lane) { return (q & 3) + 8 * (q >> 2) + 4 * (lane >> 5); }

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void fpt_train_bwd_kernel(TrainArgs a,
                                                                                          const float *__restrict__ th0) {
    // two [sample][unit] tiles: HA holds h1, then delta1; HB holds h2, then delta2 (34 KB with the
    // inputs and coefficients, so four single-wave workgroups share a CU, one per SIMD)
    __shared__ float HA[64 * TS];
    __shared__ float HB[64 * TS];
    __shared__ float XS[64 * 4];
    __shared__ float GS[64];
    const int lane = threadIdx.x;
    const int col = lane & 31, kh = lane >> 5;
    const double dNd = static_cast<double>(a.dN);
    // this lane's B fragments of W2 for the whole kernel: WT for h1 W2^T (k = input v, n = unit u),
    // WN for delta2 W2 (k = unit u, n = input v); and its units' b2
    float WT[2][32], WN[2][32], b2v[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
        for (int ks = 0; ks < 32; ++ks) {
            WT[nb][ks] = th0[NET_W2 + 64 * (32 * nb + col) + 2 * ks + kh];
            WN[nb][ks] = th0[NET_W2 + 64 * (2 * ks + kh) + 32 * nb + col];
        }
        b2v[nb] = th0[NET_B2 + 32 * nb + col];
    }
    f32x16v acc[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[mb][nb][q] = 0.0f;
    float g_w3 = 0.0f, g_b2 = 0.0f, g_b1 = 0.0f, g_w1[3] = {0.0f, 0.0f, 0.0f}, g_b3 = 0.0f;
    const uint64_t n_tiles = (a.n_rec + 63) / 64;
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const float *th = th0 + opaque_zero();
        const uint64_t e = tile * 64 + lane;
        const bool valid = e < a.n_rec;
        TrainRec R{};
        if (valid) R = a.rec[e];
        else R.phi = a.mc.in_mean[0];
        // forward: h1 into HA (this lane's record), h2 = tanh(W2 h1 + b2) into HB on the matrix
        // cores (M = record, N = unit, K = input), then r from this lane's row of HB
        float g = 0.0f;
        {
            float x[3], h1[64];
            net_inputs(a.mc, R.phi, R.k, a.dN, x);
            net_layer1(th, x, h1);
#pragma unroll
            for (int u = 0; u < 64; ++u) HA[lane * TS + u] = h1[u];
            XS[lane * 4 + 0] = x[0];
            XS[lane * 4 + 1] = x[1];
            XS[lane * 4 + 2] = x[2];
            XS[lane * 4 + 3] = 1.0f;
        }
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            f32x16v z[2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int q = 0; q < 16; ++q) z[nb][q] = 0.0f;
#pragma unroll
            for (int ks = 0; ks < 32; ++ks) {
                const float av = HA[(32 * mb + col) * TS + 2 * ks + kh];
                z[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, WT[0][ks], z[0], 0, 0, 0);
                z[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, WT[1][ks], z[1], 0, 0, 0);
            }
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    HB[(32 * mb + acc_row(q, lane)) * TS + 32 * nb + col] = tanh_hw(z[nb][q] + b2v[nb]);
        }
        __syncthreads();
        {
            float o = 0.0f;
#pragma unroll 8
            for (int u = 0; u < 64; ++u) o = __builtin_fmaf(th[NET_W3 + u], HB[lane * TS + u], o);
            if (valid) {
                const double r = static_cast<double>(a.mc.out_scale * (o + th[NET_B3]));
                const uint32_t path = R.pn >> 5;
                const double n = static_cast<double>(R.pn & 31u);
                g = static_cast<float>(a.c[path] * (r * n * dNd - static_cast<double>(R.H)) *
                                       static_cast<double>(a.mc.out_scale) * static_cast<double>(a.rec_weight));
            }
            GS[lane] = g;
        }
        __syncthreads();
        // lane = unit: w3 and b3 from h2
        {
            float sw3 = 0.0f, sb3 = 0.0f;
#pragma unroll 4
            for (int s = 0; s < 64; ++s) {
                const float gs = GS[s];
                sw3 = __builtin_fmaf(gs, HB[s * TS + lane], sw3);
                sb3 += gs;
            }
            g_w3 += sw3;
            g_b3 += sb3;
        }
        __syncthreads();
        // delta2 = g w3 (1 - h2^2), in place over this lane's h2
#pragma unroll 4
        for (int u = 0; u < 64; ++u) {
            const float h = HB[lane * TS + u];
            HB[lane * TS + u] = (g * th[NET_W3 + u]) * __builtin_fmaf(-h, h, 1.0f);
        }
        __syncthreads();
        // lane = unit: b2 from delta2
        {
            float sb2 = 0.0f;
#pragma unroll 4
            for (int s = 0; s < 64; ++s) sb2 += HB[s * TS + lane];
            g_b2 += sb2;
        }
        // dW2[u][v] += sum_s delta2[s][u] h1[s][v]: M = u, N = v, K = the tile's samples
        {
            const int row = lane & 31, kh = lane >> 5;
#pragma unroll 4
            for (int ks = 0; ks < 32; ++ks) {
                const int s = 2 * ks + kh;
                const float a0 = HB[s * TS + row], a1 = HB[s * TS + 32 + row];
                const float b0 = HA[s * TS + row], b1 = HA[s * TS + 32 + row];
                acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
            }
        }
        __syncthreads();
        // delta1 = (delta2 W2) (1 - h1^2) on the matrix cores (M = record, N = input, K = unit); each
        // accumulator element overwrites the h1 it was scaled by (one lane owns each element)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            f32x16v z[2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int q = 0; q < 16; ++q) z[nb][q] = 0.0f;
#pragma unroll
            for (int ks = 0; ks < 32; ++ks) {
                const float av = HB[(32 * mb + col) * TS + 2 * ks + kh];
                z[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, WN[0][ks], z[0], 0, 0, 0);
                z[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, WN[1][ks], z[1], 0, 0, 0);
            }
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int idx = (32 * mb + acc_row(q, lane)) * TS + 32 * nb + col;
                    const float h = HA[idx];
                    HA[idx] = z[nb][q] * __builtin_fmaf(-h, h, 1.0f);
                }
        }
        __syncthreads();
        // lane = unit: W1, b1 from delta1
        {
            float sb1 = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll 4
            for (int s = 0; s < 64; ++s) {
                const float d = HA[s * TS + lane];
                sb1 += d;
                s0 = __builtin_fmaf(d, XS[s * 4 + 0], s0);
                s1 = __builtin_fmaf(d, XS[s * 4 + 1], s1);
                s2 = __builtin_fmaf(d, XS[s * 4 + 2], s2);
            }
            g_b1 += sb1;
            g_w1[0] += s0;
            g_w1[1] += s1;
            g_w1[2] += s2;
        }
        __syncthreads();
    }
    // partial gradient of this workgroup
    float *P = a.part + static_cast<size_t>(blockIdx.x) * NET_N_PARAMS;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int u = 32 * mb + (q & 3) + 8 * (q >> 2) + 4 * (lane >> 5);
                const int v = 32 * nb + (lane & 31);
                P[NET_W2 + 64 * u + v] = acc[mb][nb][q];
            }
    P[NET_W1 + 3 * lane + 0] = g_w1[0];
    P[NET_W1 + 3 * lane + 1] = g_w1[1];
    P[NET_W1 + 3 * lane + 2] = g_w1[2];
    P[NET_B1 + lane] = g_b1;
    P[NET_B2 + lane] = g_b2;
    P[NET_W3 + lane] = g_w3;
    if (lane == 0) P[NET_B3] = g_b3;
}

__global__ __launch_bounds__(256) void fpt_train_reduce_kernel(const float *part, int n_part, double *grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NET_N_PARAMS) return;
    double s = 0.0;
    for (int w = 0; w < n_part; ++w) s += static_cast<double>(part[static_cast<size_t>(w) * NET_N_PARAMS + j]);
    grad[j] = s;
}

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return static_cast<uint16_t>(b >> 16);
}

__global__ __launch_bounds__(256) void fpt_adam_kernel(AdamArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NET_N_PARAMS) return;
    const float g = static_cast<float>(a.grad[j]);
    const float m = a.beta1 * a.m[j] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.v[j] + (1.0f - a.beta2) * g * g;
    a.m[j] = m;
    a.v[j] = v;
    const float mh = m / a.bc1;
    const float vh = v / a.bc2;
    const float th = a.theta[j] - a.lr * mh / (sqrtf(vh) + a.eps);
    a.theta[j] = th;
    a.bf16[j] = bf16_bits(th);
}

__global__ __launch_bounds__(256) void fpt_to_bf16_kernel(const float *theta, uint16_t *bf) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < NET_N_PARAMS) bf[j] = bf16_bits(theta[j]);
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
template <int POT, int BIAS>
static hipError_t launch_record_t(const RecordArgs &a, hipStream_t s) {
    const unsigned blocks = (a.n_paths + 255) / 256;
    hipLaunchKernelGGL((fpt_record_kernel<POT, BIAS>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int POT>
static hipError_t launch_record_b(int bias, const RecordArgs &a, hipStream_t s) {
    switch (bias) {
    case BIAS_NONE: return launch_record_t<POT, BIAS_NONE>(a, s);
    case BIAS_NOISE_SCALED: return launch_record_t<POT, BIAS_NOISE_SCALED>(a, s);
    case BIAS_POWER: return launch_record_t<POT, BIAS_POWER>(a, s);
    case BIAS_MLP: return launch_record_t<POT, BIAS_MLP>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_records(int pot, int bias, const RecordArgs &a, hipStream_t s) {
    if (a.n_paths == 0) return hipSuccess;
    switch (pot) {
    case POT_QUADRATIC: return launch_record_b<POT_QUADRATIC>(bias, a, s);
    case POT_QUADRATIC_BUMP: return launch_record_b<POT_QUADRATIC_BUMP>(bias, a, s);
    case POT_FLAT: return launch_record_b<POT_FLAT>(bias, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_train_loss(const TrainArgs &a, hipStream_t s) {
    if (a.n_paths <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fpt_train_fwd_kernel, dim3(a.n_paths), dim3(256), 0, s, a, a.theta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fpt_train_softmax_kernel, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_train_grad(const TrainArgs &a, hipStream_t s) {
    if (a.n_part <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fpt_train_bwd_kernel, dim3(a.n_part), dim3(64), 0, s, a, a.theta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fpt_train_reduce_kernel, dim3((NET_N_PARAMS + 255) / 256), dim3(256), 0, s, a.part, a.n_part,
                       a.grad);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(fpt_adam_kernel, dim3((NET_N_PARAMS + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *theta, uint16_t *bf, hipStream_t s) {
    hipLaunchKernelGGL(fpt_to_bf16_kernel, dim3((NET_N_PARAMS + 255) / 256), dim3(256), 0, s, theta, bf);
    return hipGetLastError();
}

}  // namespace fpt
