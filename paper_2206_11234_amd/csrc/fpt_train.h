// fpt_train.h -- host-visible interface of the proposal-training kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fpt_kernels.h"

namespace fpt {

// parameter offsets of the 3-64-64-1 network (same order as the bfloat16 block)
constexpr int NET_W1 = 0, NET_B1 = 192, NET_W2 = 256, NET_B2 = 4352, NET_W3 = 4416, NET_B3 = 4480;
constexpr int NET_N_PARAMS = 4481;

// One record: the network input at an evaluation point and the group's noise sum.
struct TrainRec {
    float phi;      // field before the group's first step
    uint32_t k;     // step index of the evaluation point
    float H;        // sum over the group of fma(r_0, dN, sqrt(dN) xi)
    uint32_t pn;    // path index << 5 | steps in the group (1 .. 16)
};
static_assert(sizeof(TrainRec) == 16, "record layout");

struct RecordArgs {
    InstDev inst;               // the sampling proposal (step constants, network normalisation)
    const uint64_t *t_ids;      // run ids to replay
    uint32_t n_paths;
    uint32_t key0, key1;        // Philox key = seed of the sampling run
    int32_t group;              // one record per group of 1, 4, 8 or 16 steps
    int32_t stride;             // keep the record of every stride-th group (g % stride == 0)
    int32_t mlp_every;
    const uint16_t *mlp_params; // bfloat16 network of the sampling proposal
    const uint64_t *rec_off;    // n_paths + 1 record offsets
    TrainRec *rec;
    uint32_t *k_out;
    double *lw_out;
    int32_t *st_out;
    uint64_t *n_rec_out;        // records the replay produced (equals the slot when it matches)
};

struct TrainArgs {
    const TrainRec *rec;
    uint64_t n_rec;
    const uint64_t *rec_off;    // n_paths + 1
    int32_t n_paths;
    int32_t n_part;             // workgroups of the backward pass
    int32_t objective;          // 0: log M2 (c ~ w_0 w_theta); 1: cross entropy (c ~ w_0)
    float temper;               // w_0 enters the path weights as w_0^temper
    float rec_weight;           // each record stands for this many groups (the record stride)
    const float *theta;         // binary32 master parameters
    MlpConsts mc;               // input normalisation, output scale, N*
    float dN;                   // binary32 dN
    double *lw_theta;           // ln w_theta per path
    const double *lw0;          // ln w_0 per path (sampled)
    double n_total;             // runs drawn
    double *c;                  // softmax weights per path
    double *loss;               // log M2
    float *part;                // n_part x NET_N_PARAMS
    double *grad;               // NET_N_PARAMS
};

struct AdamArgs {
    float *theta, *m, *v;
    const double *grad;
    uint16_t *bf16;
    float lr, beta1, beta2, eps;
    float bc1, bc2;             // 1 - beta1^t, 1 - beta2^t
};

hipError_t launch_records(int pot, int bias, const RecordArgs &a, hipStream_t s);
hipError_t launch_train_loss(const TrainArgs &a, hipStream_t s);
hipError_t launch_train_grad(const TrainArgs &a, hipStream_t s);
hipError_t launch_adam(const AdamArgs &a, hipStream_t s);
hipError_t launch_to_bf16(const float *theta, uint16_t *bf, hipStream_t s);

}  // namespace fpt
