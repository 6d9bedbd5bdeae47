// fpt_kernels.hip -- persistent first-passage kernels for gfx950 (CDNA4).
//
// fpt_step: one lane per trajectory.  Each lane repeats groups of four
// Euler-Maruyama steps of the biased Langevin equation (arXiv:2206.11234,
// Sec. 2.2 eq. eq_euler_maruyam_modified) from one Philox call, updates the
// binary64 log-weight (Sec. 2.2 eq. eq_importance_sampling_bias_w, with the
// minus sign of the likelihood ratio), and stops at first passage
// (Sec. 2.1).  Finished lanes are retired at group boundaries: a wave ballot
// finds them, one atomic per wave claims new trajectory ids from the shared
// queue (mbcnt-style prefix ranks hand them out) and the lanes restart.  The
// kernel is persistent: it runs until the queue is drained.
//
// Each retiring run is binned in N = k dN (right-closed bins, Sec. 2.1) and
// accumulated into its workgroup's table: counts per (jackknife subset, row),
// log-sum-exp of w per (subset, row) and of w^2 per row (the weighted
// estimator of Sec. 2.2 and its jackknife, Sec. 2.1), and power sums of ln w
// about a per-row shift (the moments used by the lognormal estimator of
// Sec. 2.4).  The table sits in LDS when it fits and is copied to the
// workgroup's global slice at the end; otherwise it lives in that slice.
//
// fpt_merge / fpt_finalize: fold the per-workgroup slices in workgroup order
// (binary64 log-sum-exp for the weight sums, integer sums for counts,
// binomial re-basing for the moments) and evaluate the per-bin estimators.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "fpt_kernels.h"

namespace fpt {

#define FPT_NAN_BITS 0x7FF8000000000000ull
#define FPT_NEG_INF_BITS 0xFFF0000000000000ull

__device__ __forceinline__ double lse2(double a, double b) {
    if (__builtin_isinf(a) && a < 0) return b;
    if (__builtin_isinf(b) && b < 0) return a;
    const double m = fmax(a, b);
    return m + log1p(exp(-fabs(a - b)));
}

template <typename T>
__device__ __forceinline__ void atomic_lse(T *p, double x) {
    unsigned long long *a = reinterpret_cast<unsigned long long *>(p);
    unsigned long long old = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (true) {
        const double cur = __longlong_as_double(static_cast<long long>(old));
        const double nv = lse2(cur, x);
        const unsigned long long want = static_cast<unsigned long long>(__double_as_longlong(nv));
        if (want == old) return;
        const unsigned long long prev = atomicCAS(a, old, want);
        if (prev == old) return;
        old = prev;
    }
}

__device__ __forceinline__ void atomic_add_f64(double *p, double x) {
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

struct Tab {
    double *scal, *jk_lse, *lse_w2, *shift, *s1, *s2, *s3, *s4;
    uint32_t *cnt;
};

__device__ __forceinline__ Tab make_tab(unsigned char *base, const TableLayout &L) {
    Tab T;
    T.scal = reinterpret_cast<double *>(base + L.off_scal);
    T.jk_lse = reinterpret_cast<double *>(base + L.off_jk_lse);
    T.lse_w2 = reinterpret_cast<double *>(base + L.off_lse_w2);
    T.shift = reinterpret_cast<double *>(base + L.off_shift);
    T.s1 = reinterpret_cast<double *>(base + L.off_s1);
    T.s2 = reinterpret_cast<double *>(base + L.off_s2);
    T.s3 = reinterpret_cast<double *>(base + L.off_s3);
    T.s4 = reinterpret_cast<double *>(base + L.off_s4);
    T.cnt = reinterpret_cast<uint32_t *>(base + L.off_cnt);
    return T;
}

// Initial contents: -inf for log-sums, NaN ("no shift yet") for shifts, 0 elsewhere.
__device__ __forceinline__ void init_table(unsigned char *base, const TableLayout &L) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(base);
    const uint32_t n_words = L.slice_bytes / 8;
    for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x) {
        const uint32_t off = i * 8;
        unsigned long long v = 0ull;
        if (off < L.off_jk_lse) {
            const uint32_t f = ((off - L.off_scal) / 8) & 15u;
            v = (f < 4) ? FPT_NEG_INF_BITS : 0ull;
        } else if (off < L.off_shift) {
            v = FPT_NEG_INF_BITS;           // jk_lse, lse_w2
        } else if (off < L.off_s1) {
            v = FPT_NAN_BITS;               // shift
        }
        w[i] = v;
    }
}

// Wave-wide log-sum-exp / sum over lanes (all 64 lanes take part).
__device__ __forceinline__ double wave_lse(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = lse2(x, __shfl_xor(x, m, 64));
    return x;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

struct LaneAcc {
    int inst;
    double w, w2, wk, wk2, k2;
    double steps;   // exact: integer-valued, < 2^53 per lane
};

__device__ __forceinline__ void acc_reset(LaneAcc &a, int inst) {
    a.inst = inst;
    a.w = a.w2 = a.wk = a.wk2 = -INFINITY;
    a.k2 = 0.0;
    a.steps = 0.0;
}

__device__ __forceinline__ void acc_commit_direct(const Tab &T, const LaneAcc &a) {
    double *s = T.scal + static_cast<size_t>(a.inst) * 16;
    atomic_lse(s + 0, a.w);
    atomic_lse(s + 1, a.w2);
    atomic_lse(s + 2, a.wk);
    atomic_lse(s + 3, a.wk2);
    atomic_add_f64(s + 4, a.k2);
    atomic_add_f64(s + 5, a.steps);
}

extern __shared__ __align__(16) unsigned char fpt_lds[];

// SINGLE: one instance of the batch has runs, so its constants are uniform across the workgroup
// (the compiler keeps them in scalar registers) and queue ids are its trajectory ids.
template <int POT, int BIAS, bool LDS, bool SINGLE = false>
__device__ __forceinline__ void fpt_step_body(const StepArgs &a) {
    unsigned char *lds = fpt_lds;
    unsigned char *gslice = a.slices + static_cast<size_t>(blockIdx.x) * a.lay.slice_bytes;
    unsigned char *base = LDS ? lds : gslice;
    init_table(base, a.lay);
    __syncthreads();
    const Tab T = make_tab(base, a.lay);
    const uint32_t RT = a.lay.n_rows;
    const uint32_t J = a.lay.n_sub;

    const uint32_t lane = __lane_id();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // lane state
    StepConsts C{};
    uint32_t stream = 0, n_bins = 0, row_base = 0, thr_base = 0, dump_slot = 0, k_center = 0;
    uint64_t t0 = 0;            // the current instance's first run id
    int cur_inst = -1;
    float phi = 0.0f;
    uint32_t k = 0;
    double lw = 0.0;
    uint64_t t = 0;
    bool run = false;
    bool active = false;
    bool need = true;
    LaneAcc acc;
    acc_reset(acc, -1);
    // this wave's reserved queue range
    uint64_t res_lo = 0, res_hi = 0;
    // learned proposal: this wave's share of the network's A operands
    MlpTiles tiles;
    if constexpr (BIAS == BIAS_MLP) mlp_load_tiles(a.mlp_params, tiles);
    // the single-instance learned sampler reads its operand tiles from one LDS copy
    constexpr bool TILES_LDS = BIAS == BIAS_MLP && SINGLE;
    __shared__ bf16x8 tile_lds[TILES_LDS ? MLP_N_FRAG * 64 : 1];
    if constexpr (TILES_LDS) {
        if (threadIdx.x < 64) mlp_store_tiles_lds(tiles, tile_lds);
        __syncthreads();
    }
    MlpConsts mc{};
    auto network = [&](float phi_, float N_) {
        if constexpr (TILES_LDS) return mlp_forward_lds(tile_lds, mc, phi_, N_);
        else return mlp_forward(tiles, mc, phi_, N_);
    };
    int single_inst = 0;
    if constexpr (SINGLE) {
        // the one instance with runs (others in the batch, if any, have none)
        single_inst = static_cast<int>(a.order[0]);
        const InstDev &I = a.inst[single_inst];
        C = I.c;
        stream = I.stream;
        n_bins = I.n_bins;
        row_base = I.row_base;
        thr_base = I.thr_base;
        dump_slot = I.dump_slot;
        k_center = I.k_center;
        t0 = I.t_first;
        if constexpr (BIAS == BIAS_MLP) mc = I.mlp;
        cur_inst = single_inst;
    }

    while (true) {
        // ---- refill: hand new trajectory ids to lanes that need one
        const uint64_t need_mask = __ballot(need);
        if (need_mask) {
            const uint32_t n_need = __popcll(need_mask);
            const uint32_t rank = __popcll(need_mask & lt_mask);
            const uint64_t avail = res_hi - res_lo;
            uint64_t v;
            if (avail >= n_need) {
                v = res_lo + rank;
                res_lo += n_need;
            } else {
                const uint64_t short_by = n_need - avail;
                const uint64_t amt = short_by * a.chunk;
                const int leader = __ffsll(static_cast<unsigned long long>(need_mask)) - 1;
                unsigned long long b = 0;
                if (static_cast<int>(lane) == leader) b = atomicAdd(a.queue, static_cast<unsigned long long>(amt));
                b = __shfl(b, leader, 64);
                v = (rank < avail) ? res_lo + rank : b + (rank - avail);
                res_lo = b + short_by;
                res_hi = b + amt;
            }
            if (need) {
                need = false;
                if (v < a.v_total) {
                    int ii = single_inst;
                    if constexpr (SINGLE) {
                        t = v;                 // the only instance with runs starts the queue
                    } else {
                        int lo = 0, hi = a.n_inst;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (a.vbeg_sorted[mid] <= v) lo = mid; else hi = mid;
                        }
                        ii = static_cast<int>(a.order[lo]);
                        t = v - a.vbeg_sorted[lo];
                    }
                    if (!SINGLE && ii != cur_inst) {
                        const InstDev &I = a.inst[ii];
                        C = I.c;
                        stream = I.stream;
                        n_bins = I.n_bins;
                        row_base = I.row_base;
                        thr_base = I.thr_base;
                        dump_slot = I.dump_slot;
                        k_center = I.k_center;
                        t0 = I.t_first;
                        if constexpr (BIAS == BIAS_MLP) mc = I.mlp;
                        cur_inst = ii;
                    }
                    t += t0;                   // the run's id: Philox counter and jackknife subset
                    if (acc.inst != ii) {
                        if (acc.inst >= 0) acc_commit_direct(T, acc);
                        acc_reset(acc, ii);
                    }
                    phi = C.phi_in;
                    k = 0;
                    lw = 0.0;
                    run = true;
                    active = true;
                } else {
                    active = false;
                }
            }
        }
        if (!__any(active)) break;

        // ---- four Euler-Maruyama steps from one Philox call
        float sxi;
        auto step = [&](float xi, float r_net) { (void)em_step<POT, BIAS>(C, phi, k, lw, run, xi, r_net, sxi); };
        if constexpr (BIAS != BIAS_MLP) {
            if (active) {
                const F4 z = normals4(k >> 2, t, stream, a.key0, a.key1);
                const float zs[4] = {z.a, z.b, z.c, z.d};
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    if (run) step(zs[s], 0.0f);
                }
            }
        } else {
            // the network is evaluated by all 64 lanes together, outside divergent code.  One
            // pass covers max(4, E) steps for the evaluation interval E (1, 4, 8 or 16): runs
            // start at k = 0 and refill only between passes, so every lane of the wave is at a
            // multiple of the pass length here and the evaluation points of all lanes coincide.
            const int E = a.mlp_every;
            // One evaluation per pass of E = 4, 8 or 16 steps.  The pass's normals do not depend
            // on the network, so they are drawn before it and the scheduler interleaves their
            // vector work with the evaluation's matrix-core chains (they are the normals of
            // counters k/4 .. k/4 + E/4 - 1, the ones the steps would draw; a lane whose run ends
            // early leaves the rest unused).  The evaluation runs at a raised wave priority, so
            // that it finishes sooner while the SIMD's other waves fill the gaps with steps.
            auto pass = [&](auto nq_tag) {
                constexpr int NQ = decltype(nq_tag)::value;
                F4 zz[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) zz[q] = normals4((k >> 2) + q, t, stream, a.key0, a.key1);
                __builtin_amdgcn_s_setprio(2);
                const float r_mlp = network(phi, static_cast<float>(k) * C.dN);
                __builtin_amdgcn_s_setprio(0);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const float zs[4] = {zz[q].a, zz[q].b, zz[q].c, zz[q].d};
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        if (active && run) step(zs[s], r_mlp);
                }
            };
            if (E == 16) {
                pass(std::integral_constant<int, 4>{});
            } else if (E == 8) {
                pass(std::integral_constant<int, 2>{});
            } else if (E == 4) {
                pass(std::integral_constant<int, 1>{});
            } else {
                // E = 1: an evaluation before every step
                F4 z{};
                if (active && run) z = normals4(k >> 2, t, stream, a.key0, a.key1);
                const float zs[4] = {z.a, z.b, z.c, z.d};
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const float r_mlp = network(phi, static_cast<float>(k) * C.dN);
                    if (active && run) step(zs[s], r_mlp);
                }
            }
        }

        // ---- retire finished runs into the workgroup table
        const bool fin = active && !run;
        if (fin) {
            const int st = final_status(C, phi, k);
            uint32_t rl;
            if (st == ST_ENDED) {
                const uint32_t *K = a.thr + thr_base;
                uint32_t lo = 0, hi = n_bins + 1;   // first index with K >= k
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (K[mid] < k) lo = mid + 1; else hi = mid;
                }
                rl = (lo == 0) ? n_bins : ((lo == n_bins + 1) ? n_bins + 1 : lo - 1);
            } else {
                rl = (st == ST_CENSORED) ? n_bins + 2 : n_bins + 3;
            }
            const uint32_t row = row_base + rl;
            const uint32_t sub = static_cast<uint32_t>(t % J);
            atomicAdd(&T.cnt[sub * RT + row], 1u);
            atomic_lse(&T.jk_lse[sub * RT + row], lw);
            atomic_lse(&T.lse_w2[row], 2.0 * lw);
            unsigned long long *sp = reinterpret_cast<unsigned long long *>(&T.shift[row]);
            unsigned long long cb = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const unsigned long long lwb = static_cast<unsigned long long>(__double_as_longlong(lw));
            if (cb == FPT_NAN_BITS) {
                const unsigned long long prev = atomicCAS(sp, FPT_NAN_BITS, lwb);
                cb = (prev == FPT_NAN_BITS) ? lwb : prev;
            }
            const double d = lw - __longlong_as_double(static_cast<long long>(cb));
            const double d2 = d * d;
            atomic_add_f64(&T.s1[row], d);
            atomic_add_f64(&T.s2[row], d2);
            atomic_add_f64(&T.s3[row], d2 * d);
            atomic_add_f64(&T.s4[row], d2 * d2);
            if (st == ST_ENDED) {
                // correlation of ln w with N over the ended runs (Sec. 3.4)
                double *sc = T.scal + static_cast<size_t>(cur_inst) * 16;
                const double y = static_cast<double>(static_cast<int64_t>(k) - static_cast<int64_t>(k_center));
                atomic_add_f64(sc + 6, 1.0);
                atomic_add_f64(sc + 7, lw);
                atomic_add_f64(sc + 8, lw * lw);
                atomic_add_f64(sc + 9, y);
                atomic_add_f64(sc + 10, y * y);
                atomic_add_f64(sc + 11, lw * y);
            }
            // instance-wide sums in lane registers
            const double kd = static_cast<double>(k);
            const double lk = log(kd);
            acc.w = lse2(acc.w, lw);
            acc.w2 = lse2(acc.w2, 2.0 * lw);
            acc.wk = lse2(acc.wk, lw + lk);
            acc.wk2 = lse2(acc.wk2, lw + 2.0 * lk);
            acc.k2 += kd * kd;
            acc.steps += kd;
            if (a.dump.n != 0 && ((t - t0) % a.dump.stride) == 0) {
                const uint64_t idx = (t - t0) / a.dump.stride;
                if (idx < a.dump.n) {
                    const uint64_t pos = static_cast<uint64_t>(dump_slot) * a.dump.n + idx;
                    a.dump.k[pos] = k;
                    a.dump.lw[pos] = lw;
                    a.dump.phi[pos] = phi;
                    a.dump.status[pos] = st;
                }
            }
            active = false;
            need = true;
        }
    }

    // ---- flush lane accumulators: one wave reduction per distinct instance
    bool pending = acc.inst >= 0;
    while (true) {
        const uint64_t pm = __ballot(pending);
        if (!pm) break;
        const int leader = __ffsll(static_cast<unsigned long long>(pm)) - 1;
        const int inst_l = __shfl(acc.inst, leader, 64);
        const bool mine = pending && acc.inst == inst_l;
        const double w = wave_lse(mine ? acc.w : -INFINITY);
        const double w2 = wave_lse(mine ? acc.w2 : -INFINITY);
        const double wk = wave_lse(mine ? acc.wk : -INFINITY);
        const double wk2 = wave_lse(mine ? acc.wk2 : -INFINITY);
        const double k2 = wave_sum(mine ? acc.k2 : 0.0);
        const double steps = wave_sum(mine ? acc.steps : 0.0);
        if (static_cast<int>(lane) == leader) {
            LaneAcc r;
            r.inst = inst_l;
            r.w = w; r.w2 = w2; r.wk = wk; r.wk2 = wk2; r.k2 = k2; r.steps = steps;
            acc_commit_direct(T, r);
        }
        if (mine) pending = false;
    }
    __syncthreads();
    if constexpr (LDS) {
        const unsigned long long *src = reinterpret_cast<const unsigned long long *>(lds);
        unsigned long long *dst = reinterpret_cast<unsigned long long *>(gslice);
        const uint32_t n_words = a.lay.slice_bytes / 8;
        for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x) dst[i] = src[i];
    }
}

// Workgroups of up to 1024 threads for the closed-form biases; the learned bias holds the
// network's operands in registers and runs with up to 256 threads (one wave per SIMD can use
// the whole register file).
template <int POT, int BIAS, bool LDS>
__global__ __launch_bounds__(1024) void fpt_step_kernel(StepArgs a) {
    fpt_step_body<POT, BIAS, LDS>(a);
}

template <int POT, bool LDS>
__global__ __launch_bounds__(256) void fpt_step_mlp_kernel(StepArgs a) {
    fpt_step_body<POT, BIAS_MLP, LDS>(a);
}

// One instance: uniform constants in scalar registers and the network's operand tiles in LDS,
// fitted to three waves per SIMD so that one wave's matrix-core work and latency overlap the
// others' vector work.
template <int POT, bool LDS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void fpt_step_mlp1_kernel(StepArgs a) {
    fpt_step_body<POT, BIAS_MLP, LDS, true>(a);
}

__global__ void fpt_init_queue_kernel(unsigned long long *q) {
    if (threadIdx.x == 0) q[0] = 0ull;
}

// Instance owning global row r (rows are assigned in instance order).
__device__ __forceinline__ int inst_of_row(const MergeInst *mi, int n_inst, uint32_t r) {
    int lo = 0, hi = n_inst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (mi[mid].row_base <= r) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void fpt_merge_kernel(MergeArgs a) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const TableLayout &L = a.lay;
    const uint32_t RT = L.n_rows, J = L.n_sub;
    if (tid < J * RT) {
        const uint32_t s = tid / RT, r = tid % RT;
        uint64_t cnt = 0;
        double l = -INFINITY;
        for (int w = 0; w < a.n_wg; ++w) {
            const unsigned char *sl = a.slices + static_cast<size_t>(w) * L.slice_bytes;
            cnt += reinterpret_cast<const uint32_t *>(sl + L.off_cnt)[s * RT + r];
            l = lse2(l, reinterpret_cast<const double *>(sl + L.off_jk_lse)[s * RT + r]);
        }
        const int i = inst_of_row(a.mi, a.n_inst, r);
        const MergeInst m = a.mi[i];
        const uint32_t lr = r - m.row_base;
        const ResultLayout RL = result_layout(m.n_bins, J);
        a.counts[m.counts_off + RL.jk_count + static_cast<uint64_t>(s) * m.n_rows + lr] = cnt;
        a.values[m.values_off + RL.jk_lse_w + static_cast<uint64_t>(s) * m.n_rows + lr] = l;
    } else if (tid < J * RT + RT) {
        const uint32_t r = tid - J * RT;
        double l2 = -INFINITY;
        double c = NAN;
        double n = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0;
        for (int w = 0; w < a.n_wg; ++w) {
            const unsigned char *sl = a.slices + static_cast<size_t>(w) * L.slice_bytes;
            l2 = lse2(l2, reinterpret_cast<const double *>(sl + L.off_lse_w2)[r]);
            const double cw = reinterpret_cast<const double *>(sl + L.off_shift)[r];
            if (isnan(cw)) continue;
            double nw = 0.0;
            for (uint32_t s = 0; s < J; ++s)
                nw += static_cast<double>(reinterpret_cast<const uint32_t *>(sl + L.off_cnt)[s * RT + r]);
            if (nw == 0.0) continue;
            if (isnan(c)) c = cw;
            const double d = cw - c;
            const double s1 = reinterpret_cast<const double *>(sl + L.off_s1)[r];
            const double s2 = reinterpret_cast<const double *>(sl + L.off_s2)[r];
            const double s3 = reinterpret_cast<const double *>(sl + L.off_s3)[r];
            const double s4 = reinterpret_cast<const double *>(sl + L.off_s4)[r];
            // sum (x - c)^j = sum ((x - cw) + d)^j
            S4 += s4 + 4.0 * d * s3 + 6.0 * d * d * s2 + 4.0 * d * d * d * s1 + nw * d * d * d * d;
            S3 += s3 + 3.0 * d * s2 + 3.0 * d * d * s1 + nw * d * d * d;
            S2 += s2 + 2.0 * d * s1 + nw * d * d;
            S1 += s1 + nw * d;
            n += nw;
        }
        const int i = inst_of_row(a.mi, a.n_inst, r);
        const MergeInst m = a.mi[i];
        const uint32_t lr = r - m.row_base;
        const ResultLayout RL = result_layout(m.n_bins, J);
        double* V = a.values + m.values_off;
        V[RL.lse_w2 + lr] = l2;
        if (n > 0.0) {
            const double mu = S1 / n;
            const double e2 = S2 / n, e3 = S3 / n, e4 = S4 / n;
            V[RL.mean_lnw + lr] = c + mu;
            V[RL.m2_lnw + lr] = e2 - mu * mu;
            V[RL.m3_lnw + lr] = e3 - 3.0 * mu * e2 + 2.0 * mu * mu * mu;
            V[RL.m4_lnw + lr] = e4 - 4.0 * mu * e3 + 6.0 * mu * mu * e2 - 3.0 * mu * mu * mu * mu;
        } else {
            V[RL.mean_lnw + lr] = NAN;
            V[RL.m2_lnw + lr] = NAN;
            V[RL.m3_lnw + lr] = NAN;
            V[RL.m4_lnw + lr] = NAN;
        }
    } else if (tid < J * RT + RT + static_cast<uint32_t>(a.n_inst)) {
        const int i = static_cast<int>(tid - J * RT - RT);
        double f[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
        double k2 = 0.0, steps = 0.0, ps[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int w = 0; w < a.n_wg; ++w) {
            const double *sc = reinterpret_cast<const double *>(a.slices + static_cast<size_t>(w) * L.slice_bytes + L.off_scal) + static_cast<size_t>(i) * 16;
            for (int q = 0; q < 4; ++q) f[q] = lse2(f[q], sc[q]);
            k2 += sc[4];
            steps += sc[5];
            for (int q = 0; q < 6; ++q) ps[q] += sc[6 + q];
        }
        const MergeInst m = a.mi[i];
        const ResultLayout RL = result_layout(m.n_bins, J);
        double *V = a.values + m.values_off;
        V[RL.lse_w_all] = f[0];
        V[RL.lse_w2_all] = f[1];
        V[RL.lse_wk] = f[2];
        V[RL.lse_wk2] = f[3];
        V[RL.sum_k2] = k2;
        {
            // Pearson's r of ln w with N over the ended runs (equal to that of log10 w with N)
            const double n = ps[0];
            const double mx = ps[1] / n, my = ps[3] / n;
            const double cxy = ps[5] / n - mx * my;
            const double vx = ps[2] / n - mx * mx, vy = ps[4] / n - my * my;
            V[RL.pearson_r] = (n >= 2.0 && vx > 0.0 && vy > 0.0) ? cxy / sqrt(vx * vy) : NAN;
        }
        a.counts[m.counts_off + RL.n_traj] = m.n_traj;
        a.counts[m.counts_off + RL.total_steps] = static_cast<uint64_t>(steps);
        V[RL.lognormal_gate] = 1.0;     // cleared by the finalize kernel where a bin fails
    }
}

// D'Agostino and Pearson's omnibus K^2 test of normality from the sample skewness g1 = m3/m2^1.5
// and kurtosis b2 = m4/m2^2 (population central moments) of n values: the skewness is mapped to a
// standard normal by D'Agostino's (1970) Johnson S_U transformation, the kurtosis by Anscombe and
// Glynn's (1983) Wilson-Hilferty-type transformation, and K^2 = Z1^2 + Z2^2 is chi^2 with two
// degrees of freedom, so p = exp(-K^2/2).
__device__ double dagostino_pearson_p(double n, double g1, double b2) {
    // skewness
    const double y = g1 * sqrt((n + 1.0) * (n + 3.0) / (6.0 * (n - 2.0)));
    const double beta2 = 3.0 * (n * n + 27.0 * n - 70.0) * (n + 1.0) * (n + 3.0) /
                         ((n - 2.0) * (n + 5.0) * (n + 7.0) * (n + 9.0));
    const double w2 = -1.0 + sqrt(2.0 * (beta2 - 1.0));
    const double delta = 1.0 / sqrt(0.5 * log(w2));
    const double alpha = sqrt(2.0 / (w2 - 1.0));
    const double z1 = delta * asinh(y / alpha);
    // kurtosis
    const double e = 3.0 * (n - 1.0) / (n + 1.0);
    const double var = 24.0 * n * (n - 2.0) * (n - 3.0) / ((n + 1.0) * (n + 1.0) * (n + 3.0) * (n + 5.0));
    const double x = (b2 - e) / sqrt(var);
    const double sb1 = 6.0 * (n * n - 5.0 * n + 2.0) / ((n + 7.0) * (n + 9.0)) *
                       sqrt(6.0 * (n + 3.0) * (n + 5.0) / (n * (n - 2.0) * (n - 3.0)));
    const double A = 6.0 + 8.0 / sb1 * (2.0 / sb1 + sqrt(1.0 + 4.0 / (sb1 * sb1)));
    const double den = 1.0 + x * sqrt(2.0 / (A - 4.0));
    if (den == 0.0) return NAN;
    const double z2 = ((1.0 - 2.0 / (9.0 * A)) - cbrt((1.0 - 2.0 / A) / den)) / sqrt(2.0 / (9.0 * A));
    return exp(-0.5 * (z1 * z1 + z2 * z2));
}

// Lognormal estimator of one bin (Sec. 2.4): <w> = exp(<ln w> + s^2/2) with s^2 the unbiased
// sample variance of ln w; P_hat = n_j <w> / (n_traj width); its Cox interval
// P_hat exp(+-u), u = sqrt(s^2/n + s^4/(2n - 2)); and the normality p-value of ln w.
// log_norm = log(width) + log(n_traj).
__device__ void lognormal_bin(double *V, const ResultLayout &RL, uint32_t lr, uint64_t cnt, double log_norm) {
    double lp = NAN, lo = NAN, hi = NAN, pv = NAN;
    if (cnt >= 2) {
        const double n = static_cast<double>(cnt);
        const double c2 = V[RL.m2_lnw + lr];
        const double s2 = c2 * n / (n - 1.0);
        lp = log(n) + V[RL.mean_lnw + lr] + 0.5 * s2 - log_norm;
        const double u = sqrt(s2 / n + s2 * s2 / (2.0 * n - 2.0));
        hi = expm1(u);
        lo = -expm1(-u);
        if (cnt >= 8 && c2 > 0.0) {
            const double g1 = V[RL.m3_lnw + lr] / (c2 * sqrt(c2));
            const double b2 = V[RL.m4_lnw + lr] / (c2 * c2);
            pv = dagostino_pearson_p(n, g1, b2);
        }
    }
    V[RL.log_p_ln + lr] = lp;
    V[RL.rel_err_ln_lo + lr] = lo;
    V[RL.rel_err_ln_hi + lr] = hi;
    V[RL.normal_p + lr] = pv;
}

__global__ __launch_bounds__(256) void fpt_finalize_kernel(MergeArgs a) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t RT = a.lay.n_rows, J = a.lay.n_sub;
    if (r >= RT) return;
    const int i = inst_of_row(a.mi, a.n_inst, r);
    const MergeInst m = a.mi[i];
    const uint32_t lr = r - m.row_base;
    const ResultLayout RL = result_layout(m.n_bins, J);
    uint64_t *Cn = a.counts + m.counts_off;
    double *V = a.values + m.values_off;
    uint64_t cnt = 0;
    double l = -INFINITY;
    for (uint32_t s = 0; s < J; ++s) {
        cnt += Cn[RL.jk_count + static_cast<uint64_t>(s) * m.n_rows + lr];
        l = lse2(l, V[RL.jk_lse_w + static_cast<uint64_t>(s) * m.n_rows + lr]);
    }
    Cn[RL.count + lr] = cnt;
    V[RL.lse_w + lr] = l;
    if (lr < m.n_bins) {
        const double width = a.edges[m.edge_base + lr + 1] - a.edges[m.edge_base + lr];
        const double nt = static_cast<double>(m.n_traj);
        V[RL.log_p + lr] = l - log(width) - log(nt);
        // jackknife: P_s / P = exp(lse_s - lse) * n_traj / n_s; spread over subsets / sqrt(J)
        double mean = 0.0, m2 = 0.0;
        for (uint32_t s = 0; s < J; ++s) {
            // runs of subset s: ids t = s mod J in [t_first, t_first + n_traj), as the number below
            // the end minus the number below the start (ids below x in subset s: x/J + (x mod J > s))
            const uint64_t x1 = m.t_first + m.n_traj, x0 = m.t_first;
            const double ns = static_cast<double>((x1 / J + ((x1 % J) > s ? 1 : 0)) - (x0 / J + ((x0 % J) > s ? 1 : 0)));
            const double rel = exp(V[RL.jk_lse_w + static_cast<uint64_t>(s) * m.n_rows + lr] - l) * (nt / ns);
            const double dlt = rel - mean;
            mean += dlt / static_cast<double>(s + 1);
            m2 += dlt * (rel - mean);
        }
        V[RL.rel_err_jk + lr] = sqrt(m2 / static_cast<double>(J - 1)) / sqrt(static_cast<double>(J));
        const double k2 = exp(V[RL.lse_w2 + lr] - 2.0 * l) - 1.0 / nt;
        V[RL.rel_err_kish + lr] = (cnt == 0) ? NAN : sqrt(fmax(k2, 0.0));
        if (cnt == 0) V[RL.rel_err_jk + lr] = NAN;
        // Kish's effective sample size of the bin, (sum w)^2 / sum w^2
        V[RL.ess + lr] = (cnt == 0) ? 0.0 : exp(2.0 * l - V[RL.lse_w2 + lr]);
        lognormal_bin(V, RL, lr, cnt, log(width) + log(nt));
        // the paper's gate (Sec. 2.4): the lognormal estimator holds for the result when no bin
        // with a normality p-value (n_j >= 8) falls below 0.5 %; every failing bin writes 0
        const double pv = V[RL.normal_p + lr];
        if (cnt >= 8 && pv == pv && pv < 0.005) V[RL.lognormal_gate] = 0.0;
    }
}

// The learned bias on its own: r_theta at n given (phi, N) points (waves run full; lanes past
// n compute on a copy of the last point and do not write).
__global__ __launch_bounds__(256) void fpt_mlp_forward_kernel(const uint16_t *params, MlpConsts c, const float *phi,
                                                             const float *N, float *r, uint64_t n) {
    MlpTiles tiles;
    mlp_load_tiles(params, tiles);
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t j = i < n ? i : n - 1;
    const float out = mlp_forward(tiles, c, phi[j], N[j]);
    if (i < n) r[i] = out;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
template <int POT, int BIAS, bool LDS>
static hipError_t launch_step_t(int n_wg, int block, size_t lds_bytes, const StepArgs &args, hipStream_t stream) {
    void (*kern)(StepArgs);
    if constexpr (BIAS == BIAS_MLP) {
        if (block > 256) return hipErrorInvalidConfiguration;
        kern = args.n_inst == 1 ? fpt_step_mlp1_kernel<POT, LDS> : fpt_step_mlp_kernel<POT, LDS>;
    } else {
        kern = fpt_step_kernel<POT, BIAS, LDS>;
    }
    if (LDS && lds_bytes > 0) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(n_wg), dim3(block), LDS ? lds_bytes : 0, stream, args);
    return hipGetLastError();
}

template <int POT, bool LDS>
static hipError_t launch_step_b(int bias, int n_wg, int block, size_t lds, const StepArgs &a, hipStream_t s) {
    switch (bias) {
    case BIAS_NONE: return launch_step_t<POT, BIAS_NONE, LDS>(n_wg, block, lds, a, s);
    case BIAS_NOISE_SCALED: return launch_step_t<POT, BIAS_NOISE_SCALED, LDS>(n_wg, block, lds, a, s);
    case BIAS_POWER: return launch_step_t<POT, BIAS_POWER, LDS>(n_wg, block, lds, a, s);
    case BIAS_MLP: return launch_step_t<POT, BIAS_MLP, LDS>(n_wg, block, lds, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool LDS>
static hipError_t launch_step_p(int pot, int bias, int n_wg, int block, size_t lds, const StepArgs &a, hipStream_t s) {
    switch (pot) {
    case POT_QUADRATIC: return launch_step_b<POT_QUADRATIC, LDS>(bias, n_wg, block, lds, a, s);
    case POT_QUADRATIC_BUMP: return launch_step_b<POT_QUADRATIC_BUMP, LDS>(bias, n_wg, block, lds, a, s);
    case POT_FLAT: return launch_step_b<POT_FLAT, LDS>(bias, n_wg, block, lds, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(int pot, int bias, bool tables_in_lds, int n_wg, int block, size_t lds_bytes,
                       const StepArgs &args, hipStream_t stream) {
    if (tables_in_lds) return launch_step_p<true>(pot, bias, n_wg, block, lds_bytes, args, stream);
    return launch_step_p<false>(pot, bias, n_wg, block, 0, args, stream);
}

hipError_t launch_init_queue(unsigned long long *queue, hipStream_t stream) {
    hipLaunchKernelGGL(fpt_init_queue_kernel, dim3(1), dim3(64), 0, stream, queue);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint16_t *params, MlpConsts c, const float *phi, const float *N, float *r,
                              uint64_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(fpt_mlp_forward_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, params, c,
                       phi, N, r, n);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs &args, int total_rows, int n_sub, hipStream_t stream) {
    const int n1 = n_sub * total_rows + total_rows + args.n_inst;
    hipLaunchKernelGGL(fpt_merge_kernel, dim3((n1 + 255) / 256), dim3(256), 0, stream, args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fpt_finalize_kernel, dim3((total_rows + 255) / 256), dim3(256), 0, stream, args);
    return hipGetLastError();
}

}  // namespace fpt
