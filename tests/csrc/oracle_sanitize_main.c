/* Runs every entry point of the C oracle once on small inputs, so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc) checks its memory accesses
 * and arithmetic: the binary32 and binary64 simulations (all four modes) of every potential and
 * bias kind the oracle knows, the learned bias, the training replay into records and the loss
 * with its gradient.  Exits 0 and prints a summary line when nothing is reported (the
 * sanitizers abort on the first error). */
#include "../../oracle/fpt_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static oracle_params base(void)
{
    oracle_params P;
    memset(&P, 0, sizeof P);
    P.pot_kind = 0;
    P.m = 1.0;
    P.phi_in = 6.0;
    P.phi_end = sqrt(2.0);
    P.phi_uv = 8.0;
    P.phi_esc = INFINITY;
    P.dN = 1e-3;
    P.k_max = 200000;
    P.seed = 0;
    P.eval_every = 4;
    P.out_scale = 1.0f;
    return P;
}

int main(void)
{
    enum { N = 64 };
    uint64_t k[N];
    double lw[N], phi[N];
    int32_t st[N];
    long total = 0;
    oracle_params cases[5];
    cases[0] = base();                                               /* quadratic, noise-scaled bias */
    cases[0].bias_kind = 1;
    cases[0].A = 1.0;
    cases[1] = base();                                               /* bump, no wall, escape */
    cases[1].pot_kind = 1; cases[1].m = 0.05; cases[1].a = 0.02; cases[1].phi0 = 4.0; cases[1].w = 0.1;
    cases[1].phi_in = 4.5; cases[1].phi_uv = INFINITY; cases[1].phi_esc = 450.0; cases[1].dN = 1e-3;
    cases[2] = base();                                               /* flat well */
    cases[2].pot_kind = 2; cases[2].V0 = 1.0; cases[2].phi_in = 1.0; cases[2].phi_end = 0.0; cases[2].phi_uv = 1.5;
    cases[3] = base();                                               /* power-law bias, capped runs */
    cases[3].m = 0.01; cases[3].phi_in = 5.0; cases[3].phi_uv = INFINITY; cases[3].phi_esc = 500.0;
    cases[3].bias_kind = 2; cases[3].A = 2e-5; cases[3].p = 3; cases[3].k_max = 3000;
    static float theta_f[4481];
    for (int i = 0; i < 4481; ++i) theta_f[i] = bf16_round(0.01f * (float)((i * 37) % 17 - 8));
    theta_f[4480] = 1.0f;
    cases[4] = base();                                               /* learned bias */
    cases[4].bias_kind = 3; cases[4].mlp = theta_f; cases[4].target_N = 20.0;
    cases[4].in_mean[0] = 5.0f; cases[4].in_mean[1] = 20.0f; cases[4].in_mean[2] = 20.0f;
    cases[4].in_inv[0] = 0.4f; cases[4].in_inv[1] = 0.05f; cases[4].in_inv[2] = 0.05f;
    cases[4].k_max = 20000;
    for (int c = 0; c < 5; ++c)
        for (int mode = 0; mode < 4; ++mode) {
            oracle_simulate(&cases[c], 0, 1, N, mode, k, lw, phi, st, 2);
            for (int i = 0; i < N; ++i) total += (long)k[i];
        }
    float pv[8], nv[8];
    double r[8];
    for (int i = 0; i < 8; ++i) { pv[i] = 1.5f + 0.8f * (float)i; nv[i] = 3.0f * (float)i; }
    oracle_mlp_r_batch(&cases[4], pv, nv, r, 8);
    /* training replay of the learned-bias runs, then the loss and gradient */
    uint64_t ids[N], off[N + 1];
    off[0] = 0;
    for (int i = 0; i < N; ++i) {
        ids[i] = (uint64_t)i;
        off[i + 1] = off[i] + (k[i] + 3) / 4;        /* k from the last simulation of case 4 */
    }
    oracle_record *rec = (oracle_record *)malloc(sizeof(oracle_record) * (off[N] + 1));
    uint64_t k2[N];
    double lw2[N], lw0[N], lwt[N];
    int32_t st2[N];
    int64_t bad = oracle_records(&cases[4], ids, N, 4, 1, off, rec, k2, lw2, st2);
    static double theta[4481], grad[4481];
    for (int i = 0; i < 4481; ++i) theta[i] = theta_f[i];
    double *gp = (double *)malloc(sizeof(double) * 4481 * N);
    double loss = 0.0;
    for (int i = 0; i < N; ++i) lw0[i] = lw2[i];
    for (int obj = 0; obj < 2; ++obj)
        oracle_loss_grad(&cases[4], theta, rec, off, N, lw0, (double)N, obj, 0.5, 1.0, &loss, grad, lwt, gp);
    free(rec);
    free(gp);
    printf("sanitized oracle run: %ld steps, %lld mismatched record slots, loss %.6g\n", total, (long long)bad, loss);
    return bad == 0 ? 0 : 1;
}
