// fpt_kernels.h -- host-visible launch interface of the first-passage kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fpt_device.h"
#include "fpt_mlp.h"

namespace fpt {

// One instance as the step kernel sees it (uploaded per call).
struct InstDev {
    StepConsts c;
    MlpConsts mlp;        // learned proposal: input normalisation, output scale, N*
    uint32_t stream;      // Philox counter word 3
    uint32_t n_bins;
    uint32_t row_base;    // first row of this instance in the per-workgroup table
    uint32_t thr_base;    // first integer bin threshold of this instance
    uint32_t dump_slot;   // caller's instance index
    uint32_t k_center;    // expected step count: centre of k in the correlation sums
    uint64_t n_traj;
    uint64_t v_begin;     // first id of this instance in the shared queue
    uint64_t t_first;     // run id of the instance's first run
};

// Per-workgroup table: byte offsets inside one workgroup's slice.
// Rows: all instances' rows concatenated (R_i = n_bins_i + 4).
struct TableLayout {
    uint32_t n_rows;      // total rows over instances
    uint32_t n_sub;       // J, jackknife subsets
    uint32_t n_inst;
    uint32_t slice_bytes;
    // binary64 arrays
    uint32_t off_scal;    // [n_inst][16]: lse_w_all, lse_w2_all, lse_wk, lse_wk2, sum_k2, steps, then over the
                          // ended runs: n, sum x, sum x^2, sum y, sum y^2, sum xy (x = ln w, y = k - k_center), pad
    uint32_t off_jk_lse;  // [J][n_rows]
    uint32_t off_lse_w2;  // [n_rows]
    uint32_t off_shift;   // [n_rows]
    uint32_t off_s1, off_s2, off_s3, off_s4;  // [n_rows] each
    // uint32 arrays
    uint32_t off_cnt;     // [J][n_rows]
};

struct DumpDev {
    uint64_t n, stride;
    uint32_t *k;
    double *lw;
    float *phi;
    int32_t *status;
};

struct StepArgs {
    const InstDev *inst;
    const uint32_t *order;        // instance indices sorted by v_begin
    const uint64_t *vbeg_sorted;  // v_begin in queue order
    int32_t n_inst;
    const uint32_t *thr;          // integer bin thresholds K_j (all instances)
    unsigned long long *queue;    // shared id counter
    uint64_t v_total;
    uint32_t key0, key1;          // Philox key = seed
    unsigned char *slices;        // n_wg slices of layout.slice_bytes
    TableLayout lay;
    DumpDev dump;
    uint32_t chunk;
    const uint16_t *mlp_params;   // bfloat16 network shared by the batch (learned proposal)
    int32_t mlp_every;            // evaluate the network every 1, 4, 8 or 16 steps
};

// Per-instance merge metadata.
struct MergeInst {
    uint32_t row_base, n_rows, n_bins, edge_base;
    uint64_t counts_off, values_off;  // into the staging result arrays
    uint64_t n_traj;
    uint64_t t_first;                 // runs t_first .. t_first + n_traj - 1 (jackknife subset t mod J)
};

struct MergeArgs {
    const unsigned char *slices;
    int32_t n_wg;
    TableLayout lay;
    const MergeInst *mi;
    int32_t n_inst;
    const double *edges;
    uint64_t *counts;   // staging
    double *values;     // staging
};

// Result layout offsets for one instance (elements).
struct ResultLayout {
    uint64_t n_counts, n_values;
    uint64_t count, jk_count, n_traj, total_steps;
    uint64_t lse_w, lse_w2, jk_lse_w, mean_lnw, m2_lnw, m3_lnw, m4_lnw;
    uint64_t log_p, rel_err_jk, rel_err_kish;
    uint64_t log_p_ln, rel_err_ln_lo, rel_err_ln_hi, normal_p;
    uint64_t lse_w_all, lse_w2_all, lse_wk, lse_wk2, sum_k2;
    uint64_t pearson_r;
    uint64_t ess, lognormal_gate;
};

__host__ __device__ inline ResultLayout result_layout(uint32_t n_bins, uint32_t n_sub) {
    const uint64_t R = n_bins + 4, J = n_sub, B = n_bins;
    ResultLayout L{};
    uint64_t c = 0;
    L.count = c; c += R;
    L.jk_count = c; c += J * R;
    L.n_traj = c; c += 1;
    L.total_steps = c; c += 1;
    L.n_counts = c;
    uint64_t v = 0;
    L.lse_w = v; v += R;
    L.lse_w2 = v; v += R;
    L.jk_lse_w = v; v += J * R;
    L.mean_lnw = v; v += R;
    L.m2_lnw = v; v += R;
    L.m3_lnw = v; v += R;
    L.m4_lnw = v; v += R;
    L.log_p = v; v += B;
    L.rel_err_jk = v; v += B;
    L.rel_err_kish = v; v += B;
    L.log_p_ln = v; v += B;
    L.rel_err_ln_lo = v; v += B;
    L.rel_err_ln_hi = v; v += B;
    L.normal_p = v; v += B;
    L.lse_w_all = v++;
    L.lse_w2_all = v++;
    L.lse_wk = v++;
    L.lse_wk2 = v++;
    L.sum_k2 = v++;
    L.pearson_r = v++;
    L.ess = v; v += B;
    L.lognormal_gate = v++;
    L.n_values = v;
    return L;
}

// Launches (defined in fpt_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_init_queue(unsigned long long *queue, hipStream_t stream);
hipError_t launch_step(int pot, int bias, bool tables_in_lds, int n_wg, int block, size_t lds_bytes,
                       const StepArgs &args, hipStream_t stream);
hipError_t launch_merge(const MergeArgs &args, int total_rows, int n_sub, hipStream_t stream);
hipError_t launch_mlp_forward(const uint16_t *params, MlpConsts c, const float *phi, const float *N, float *r,
                              uint64_t n, hipStream_t stream);
size_t max_lds_bytes();

}  // namespace fpt
