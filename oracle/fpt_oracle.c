/*
 * fpt_oracle.c -- plain CPU oracle for the importance-sampled first-passage
 * simulation of stochastic inflation (Jackson, Assadullahi, Koyama, Vennin,
 * Wands, "Numerical simulations of stochastic inflation using importance
 * sampling", arXiv:2206.11234).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the GPU path.
 *
 * What it computes, one trajectory at a time, in the paper's order:
 *   - the Euler-Maruyama step of the biased Langevin equation
 *     (Sec. 2.2, eq. eq_euler_maruyam_modified), with drift D = -V'/V and
 *     noise amplitude S = sqrt(V/3)/(2 pi) in Planck units (Sec. 2.3,
 *     eq. eq_sr_diffusion with H^2 = V/3);
 *   - the running exponent of the importance weight (Sec. 2.2,
 *     eq. eq_importance_sampling_bias_w).  The exponent is accumulated with
 *     a MINUS sign: substituting the two Gaussian path densities
 *     (eqs. eq_importance_sampling_probability_of_target_path and
 *     eq_importance_sampling_probability_of_sample_path) into the weight
 *     ratio gives ln w = -sum (B/S^2)[B dt/2 + S xi sqrt(dt)]; the printed
 *     equation drops that sign.  E_S[w] = 1 (tested) fixes it;
 *   - repetition until the end surface phi_end is reached, recording the
 *     elapsed number of steps k, so that N = k dN exactly (Sec. 2.1);
 *   - a reflecting wall at phi_UV (Sec. 2.3, eq. eq:meanN:S:gen and the
 *     discussion of the UV boundary in Sec. 3).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - drift, noise amplitude and bias are evaluated at the pre-step point
 *     (Ito, Sec. 2.1);
 *   - the weight includes the crossing step (product over m = 0..M-1);
 *   - the end test phi <= phi_end is applied after the reflection;
 *   - a step cap k_max and (without a wall) an escape level phi_esc stop
 *     runs that would not terminate; such runs are reported, not dropped.
 *
 * Two arithmetic modes over the SAME noise stream:
 *   MODE_F32 -- every step in IEEE binary32, written operation by operation
 *               with explicit fmaf, no contraction (build with
 *               -ffp-contract=off), with the transcendental functions of the
 *               normal transform, the reciprocal and the square root written
 *               out below as fma sequences (so that the integer step count is
 *               decided in binary32 by a fixed sequence of operations);
 *   MODE_F64 -- the same semantics in binary64 with libm transcendentals,
 *               used to state the binary32 error of every result.
 *
 * Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11), counter (k/4, t_lo, t_hi, stream), key
 * (seed_lo, seed_hi); each 32-bit word x gives the uniform
 * u = (2*(x>>9)+1) * 2^-24 in (0,1), and the Box-Muller transform maps
 * (u0,u1) and (u2,u3) to four standard normals for steps 4j .. 4j+3:
 * rho = sqrt(-2 ln u_a), z = rho cos(2 pi u_b), z' = rho sin(2 pi u_b).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): multipliers and Weyl key increments.          */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u = (2*(x>>9)+1) * 2^-24: an odd multiple of 2^-24, exact in binary32. */
float oracle_uniform24(uint32_t x)
{
    uint32_t odd = ((x >> 9) << 1) | 1u;
    return (float)odd * 0x1p-24f;
}

static float bits_to_f32(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t f32_to_bits(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

/* ------------------------------------------------------------------ */
/* binary32 reciprocal of a positive normal x: Newton-Raphson           */
/* y <- y (2 - x y), written y <- fma(y, fma(-x, y, 1), y), three times */
/* from the exponent-negating seed bits(0x7EF311C3 - bits(x)) (relative */
/* error below 5.1%, so 3 steps reach the binary32 rounding level).     */
/* The bit-subtraction seed is J. Blinn's ("Floating-point tricks",     */
/* IEEE CG&A 17(4), 1997); 0x7EF311C3 is a published tuning of it.      */
/* ------------------------------------------------------------------ */
float oracle_recip_f32(float x)
{
    float y = bits_to_f32(0x7EF311C3u - f32_to_bits(x));
    for (int i = 0; i < 3; ++i) {
        float e = fmaf(-x, y, 1.0f);
        y = fmaf(y, e, y);
    }
    return y;
}

/* ------------------------------------------------------------------ */
/* binary32 square root of a positive normal x: reciprocal square root  */
/* by Newton-Raphson y <- y (3 - x y^2)/2, written                      */
/* y <- fma(y, fma(-x/2, y*y, 1/2), y), three times from the seed       */
/* bits(0x5F3759DF - (bits(x) >> 1)) (relative error below 3.5%), then  */
/* sqrt x = x y.  The seed constant is the Quake III Arena one (1999),   */
/* analysed by C. Lomont, "Fast inverse square root" (2003).            */
/* ------------------------------------------------------------------ */
float oracle_sqrt_f32(float x)
{
    float y = bits_to_f32(0x5F3759DFu - (f32_to_bits(x) >> 1));
    float hx = 0.5f * x;
    for (int i = 0; i < 3; ++i) {
        float yy = y * y;
        float e = fmaf(-hx, yy, 0.5f);
        y = fmaf(y, e, y);
    }
    return x * y;
}

/* ------------------------------------------------------------------ */
/* binary32 natural logarithm for positive normal inputs.               */
/* Method: x = 2^e f with f in [sqrt(1/2), sqrt(2)); s = (f-1)/(f+1)    */
/* (the quotient as (f-1) * recip(f+1));                                 */
/* ln f = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + s^7/7 + s^9/9 + ...);     */
/* ln x = e ln2 + ln f with ln2 split in a 16-bit head and a tail.      */
/* |s| <= 0.1716, so the first omitted term is below 1e-9 relative.    */
/* ------------------------------------------------------------------ */
float oracle_log_f32(float x)
{
    uint32_t b = f32_to_bits(x);
    int e = (int)(b >> 23) - 127;
    float f = bits_to_f32((b & 0x007FFFFFu) | 0x3F800000u); /* [1,2) */
    if (f > 1.41421354f) {                                    /* fl32(sqrt 2) */
        f = bits_to_f32((b & 0x007FFFFFu) | 0x3F000000u);     /* f/2, exact */
        e += 1;
    }
    float s = (f - 1.0f) * oracle_recip_f32(f + 1.0f);
    float z = s * s;
    float p = 1.0f / 9.0f;
    p = fmaf(p, z, 1.0f / 7.0f);
    p = fmaf(p, z, 1.0f / 5.0f);
    p = fmaf(p, z, 1.0f / 3.0f);
    float t = s + s;           /* 2s, exact */
    float tz = t * z;
    float lf = fmaf(tz, p, t); /* 2s + 2s z P(z) */
    float ef = (float)e;
    const float ln2_hi = 0.693145751953125f;       /* 16 significant bits */
    const float ln2_lo = 1.42860682030941723212e-6f; /* ln 2 - ln2_hi */
    return fmaf(ef, ln2_hi, fmaf(ef, ln2_lo, lf));
}

/* ------------------------------------------------------------------ */
/* binary32 cos(2 pi u) and sin(2 pi u) for u in [0,1], u a multiple of */
/* 2^-24.  q = nearest quarter, r = u - q/4 in [-1/8,1/8] (exact);      */
/* Taylor series of sin(2 pi r) to r^9 and cos(2 pi r) to r^10 with     */
/* coefficients (+-)(2 pi)^n / n!; the quadrant q rotates the pair.     */
/* ------------------------------------------------------------------ */
void oracle_sincos2pi_f32(float u, float *c_out, float *s_out)
{
    float q = rintf(u * 4.0f);
    float r = u - q * 0.25f;
    float r2 = r * r;
    /* sin(2 pi r) = r (S1 + r2 (S3 + r2 (S5 + r2 (S7 + r2 S9)))) */
    const float S1 = 6.28318530717958647692f;      /*  (2pi)^1/1!  */
    const float S3 = -41.341702240399760234f;     /* -(2pi)^3/3!  */
    const float S5 = 81.6052492760750542034f;      /*  (2pi)^5/5!  */
    const float S7 = -76.7058597530613858416f;     /* -(2pi)^7/7!  */
    const float S9 = 42.058693944897653145f;      /*  (2pi)^9/9!  */
    const float C2 = -19.7392088021787172377f;     /* -(2pi)^2/2!  */
    const float C4 = 64.939394022668291491f;      /*  (2pi)^4/4!  */
    const float C6 = -85.456817206693727736f;     /* -(2pi)^6/6!  */
    const float C8 = 60.2446413718766603627f;      /*  (2pi)^8/8!  */
    const float C10 = -26.4262567833743974529f;    /* -(2pi)^10/10! */
    float ps = fmaf(S9, r2, S7);
    ps = fmaf(ps, r2, S5);
    ps = fmaf(ps, r2, S3);
    ps = fmaf(ps, r2, S1);
    float sn = ps * r;
    float pc = fmaf(C10, r2, C8);
    pc = fmaf(pc, r2, C6);
    pc = fmaf(pc, r2, C4);
    pc = fmaf(pc, r2, C2);
    float cs = fmaf(pc, r2, 1.0f);
    int iq = ((int)q) & 3;
    float c, s;
    switch (iq) {
    case 0: c = cs;  s = sn;  break;
    case 1: c = -sn; s = cs;  break;
    case 2: c = -cs; s = -sn; break;
    default: c = sn; s = -cs; break;
    }
    *c_out = c;
    *s_out = s;
}

/* ------------------------------------------------------------------ */
/* binary32 exp(x) for x <= 0 (used by the Gaussian-bump potential).    */
/* x < -80 gives 0.  n = rint(x/ln2); r = x - n ln2 (two-part ln2);     */
/* Taylor series of e^r to r^7 (|r| <= 0.347: omitted term < 6e-9);     */
/* result = P(r) * 2^n built from the exponent field.                   */
/* ------------------------------------------------------------------ */
float oracle_exp_f32(float x)
{
    if (x < -80.0f) return 0.0f;
    if (x > 0.0f) x = 0.0f;
    const float inv_ln2 = 1.44269504088896340736f;
    const float ln2_hi = 0.693145751953125f;
    const float ln2_lo = 1.42860682030941723212e-6f;
    float n = rintf(x * inv_ln2);
    float r = fmaf(-n, ln2_hi, x);
    r = fmaf(-n, ln2_lo, r);
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    int ni = (int)n;
    float scale = bits_to_f32((uint32_t)(ni + 127) << 23);
    return p * scale;
}

/* Four normals for steps 4j .. 4j+3 of trajectory t in stream `stream`. */
void oracle_normals_f32(uint64_t seed, uint32_t stream, uint64_t t, uint32_t j, float out[4])
{
    uint32_t ctr[4] = { j, (uint32_t)t, (uint32_t)(t >> 32), stream };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    for (int pair = 0; pair < 2; ++pair) {
        float ua = oracle_uniform24(x[2 * pair]);
        float ub = oracle_uniform24(x[2 * pair + 1]);
        float L = oracle_log_f32(ua);
        float rho = oracle_sqrt_f32(-2.0f * L);
        float c, s;
        oracle_sincos2pi_f32(ub, &c, &s);
        out[2 * pair] = rho * c;
        out[2 * pair + 1] = rho * s;
    }
}

/* The same four normals in binary64 with libm (reference mode). */
void oracle_normals_f64(uint64_t seed, uint32_t stream, uint64_t t, uint32_t j, double out[4])
{
    uint32_t ctr[4] = { j, (uint32_t)t, (uint32_t)(t >> 32), stream };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    const double two_pi = 6.283185307179586476925;
    for (int pair = 0; pair < 2; ++pair) {
        double ua = (double)oracle_uniform24(x[2 * pair]);
        double ub = (double)oracle_uniform24(x[2 * pair + 1]);
        double rho = sqrt(-2.0 * log(ua));
        out[2 * pair] = rho * cos(two_pi * ub);
        out[2 * pair + 1] = rho * sin(two_pi * ub);
    }
}

/* ------------------------------------------------------------------ */
/* Model description.                                                   */
/* ------------------------------------------------------------------ */
enum { POT_QUADRATIC = 0, POT_QUADRATIC_BUMP = 1, POT_FLAT = 2 };
enum { BIAS_NONE = 0, BIAS_NOISE_SCALED = 1, BIAS_POWER = 2, BIAS_MLP = 3 };
enum { ST_RUNNING = 0, ST_ENDED = 1, ST_CENSORED = 2, ST_ESCAPED = 3 };
/* MODE_F32_KAHAN and MODE_F32_SUM: the binary32 step of MODE_F32 (same k, phi, increments) with
 * ln w summed in binary32, with Kahan's compensation or plainly, to measure what the binary64
 * sum buys (the step's k and phi do not depend on ln w). */
enum { MODE_F32 = 0, MODE_F64 = 1, MODE_F32_KAHAN = 2, MODE_F32_SUM = 3 };

/* All fields are the user's binary64 values; MODE_F32 rounds each of the
 * derived constants below to binary32 once, MODE_F64 keeps them. */
typedef struct {
    int pot_kind;
    double m, a, phi0, w, V0;   /* V = m^2 phi^2/2 [1 + a exp(-(phi-phi0)^2/(2w^2))], or V0 */
    int bias_kind;
    double A;                   /* B = A S (noise-scaled) or B = A phi^p (power law) */
    int p;
    double phi_in, phi_end, phi_uv, phi_esc, dN;
    uint64_t k_max;
    uint64_t seed;
    uint32_t stream;
    /* learned bias: 4481 parameters (bfloat16 values stored as float) in the order
     * W1[64][3], b1[64], W2[64][64], b2[64], w3[64], b3; inputs (phi, k dN, N*) */
    const float *mlp;
    float in_mean[3], in_inv[3];
    float out_scale;
    double target_N;
    int eval_every;
} oracle_params;

/* round a binary32 value to the nearest bfloat16 (ties to even), returned as binary32 */
static float bf16_round(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7F800000u) == 0x7F800000u) return x;     /* inf / nan unchanged */
    b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
    float y;
    memcpy(&y, &b, 4);
    return y;
}

/* The network's activation in the sampler: tanh to within a third of a bfloat16 ulp (the
 * precision its result is rounded to), as a clamped polynomial in binary32: x is clamped to
 * [-3.4, 3.4], beyond which tanh rounds to +-1 in bfloat16, and tanh x ~ x q(|x|), with q of
 * degree 5 fitted to minimise the largest error in bfloat16 ulps of tanh over [0, 3.4] and the
 * clamped tail.  q is evaluated by Horner's rule with correctly rounded fused multiply-adds
 * (fmaf) and the last product is a binary32 multiplication: the sequence the sampler executes,
 * so that given the same pre-activation the two agree bit for bit.  The pins bound its
 * distance to tanh; the training tools below use tanh itself. */
static float tanh_act_f32(float x)
{
    const float xc = fminf(fmaxf(x, -3.4f), 3.4f);
    const float t = fabsf(xc);
    float q = 0.005465357564389706f;
    q = fmaf(q, t, -0.06311261653900146f);
    q = fmaf(q, t, 0.27104586362838745f);
    q = fmaf(q, t, -0.47482094168663025f);
    q = fmaf(q, t, 0.02362865023314953f);
    q = fmaf(q, t, 0.9999812841415405f);
    return q * xc;
}

/* The learned bias r = out_scale (w3 . h2 + b3), h2 = tanh(W2 h1 + b2), h1 = tanh(W1 x + b1),
 * with the sampler's roundings: inputs and both hidden activations are rounded to bfloat16
 * before they multiply the next layer's weights; each layer's sum of products (exact for
 * bfloat16 operands) is formed in binary64 and rounded once to binary32, the activation is
 * tanh_act_f32, and the output is out_scale times the binary32 sum, in binary32. */
double oracle_mlp_r(const oracle_params *P, float phi, float N)
{
    const float *W1 = P->mlp, *b1 = P->mlp + 192, *W2 = P->mlp + 256, *b2 = P->mlp + 4352;
    const float *w3 = P->mlp + 4416, b3 = P->mlp[4480];
    float x[3];
    x[0] = bf16_round((phi - P->in_mean[0]) * P->in_inv[0]);
    x[1] = bf16_round((N - P->in_mean[1]) * P->in_inv[1]);
    x[2] = bf16_round(((float)P->target_N - P->in_mean[2]) * P->in_inv[2]);
    double h1[64], h2[64];
    for (int u = 0; u < 64; ++u) {
        double a = (double)b1[u];
        for (int s = 0; s < 3; ++s) a += (double)W1[u * 3 + s] * (double)x[s];
        h1[u] = (double)bf16_round(tanh_act_f32((float)a));
    }
    for (int u = 0; u < 64; ++u) {
        double a = (double)b2[u];
        for (int v = 0; v < 64; ++v) a += (double)W2[u * 64 + v] * h1[v];
        h2[u] = (double)bf16_round(tanh_act_f32((float)a));
    }
    double o = (double)b3;
    for (int u = 0; u < 64; ++u) o += (double)w3[u] * h2[u];
    return (double)(P->out_scale * (float)o);
}

void oracle_mlp_r_batch(const oracle_params *P, const float *phi, const float *N, double *r, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) r[i] = oracle_mlp_r(P, phi[i], N[i]);
}

/* The activation alone, for its pins. */
void oracle_tanh_act(const float *x, float *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = tanh_act_f32(x[i]);
}

/* Derived constants (Planck units):
 *   quadratic:  D = -2/phi,  S = c_m phi,  c_m = m/(2 pi sqrt 6)
 *   bump:       V'/V = 2/phi - ((phi-phi0)/w^2) a g/(1 + a g),
 *               g = exp(-(phi-phi0)^2/(2 w^2)),  S = c_m phi sqrt(1 + a g)
 *   flat:       D = 0,  S = sqrt(V0/3)/(2 pi)                           */
static double cm_of(double m) { return m / (2.0 * M_PI * sqrt(6.0)); }
static double s_flat_of(double V0) { return sqrt(V0 / 3.0) / (2.0 * M_PI); }

typedef struct {
    float dN, sq, hdN, cm, s_flat, a, phi0, inv_w2, inv_2w2, A, phi_end, phi_uv, two_uv, phi_esc, phi_in;
} consts_f32;

static void make_consts_f32(const oracle_params *P, consts_f32 *c)
{
    c->dN = (float)P->dN;
    c->sq = (float)sqrt(P->dN);
    c->hdN = (float)(0.5 * P->dN);
    c->cm = (float)cm_of(P->m);
    c->s_flat = (float)s_flat_of(P->V0);
    c->a = (float)P->a;
    c->phi0 = (float)P->phi0;
    c->inv_w2 = (float)(1.0 / (P->w * P->w));
    c->inv_2w2 = (float)(0.5 / (P->w * P->w));
    c->A = (float)P->A;
    c->phi_end = (float)P->phi_end;
    c->phi_uv = (float)P->phi_uv;
    c->two_uv = c->phi_uv + c->phi_uv;
    c->phi_esc = (float)P->phi_esc;
    c->phi_in = (float)P->phi_in;
}

/* D and S at phi, binary32, operation by operation. */
static void drift_noise_f32(const oracle_params *P, const consts_f32 *c, float phi, float *D, float *S)
{
    if (P->pot_kind == POT_QUADRATIC) {
        float y = oracle_recip_f32(phi);
        float d = y + y;               /* 2/phi */
        *D = -d;
        *S = c->cm * phi;
    } else if (P->pot_kind == POT_QUADRATIC_BUMP) {
        float dphi = phi - c->phi0;
        float e2 = dphi * dphi;
        float x = -(e2 * c->inv_2w2);
        float g = oracle_exp_f32(x);
        float ag = c->a * g;
        float one_ag = 1.0f + ag;
        float num = (dphi * c->inv_w2) * ag;
        float corr = num * oracle_recip_f32(one_ag);
        float y = oracle_recip_f32(phi);
        float d = y + y;
        *D = corr - d;
        *S = (c->cm * phi) * oracle_sqrt_f32(one_ag);
    } else {
        *D = 0.0f;
        *S = c->s_flat;
    }
}

/* r = B/S in noise units, binary32. */
static float bias_ratio_f32(const oracle_params *P, const consts_f32 *c, float phi, float S)
{
    if (P->bias_kind == BIAS_NOISE_SCALED) return c->A;
    if (P->bias_kind == BIAS_POWER) {
        float pw = 1.0f;
        for (int i = 0; i < P->p; ++i) pw = pw * phi;
        return (c->A * pw) * oracle_recip_f32(S);
    }
    return 0.0f;
}

static void drift_noise_f64(const oracle_params *P, double phi, double *D, double *S)
{
    if (P->pot_kind == POT_QUADRATIC) {
        *D = -2.0 / phi;
        *S = cm_of(P->m) * phi;
    } else if (P->pot_kind == POT_QUADRATIC_BUMP) {
        double dphi = phi - P->phi0;
        double g = exp(-dphi * dphi / (2.0 * P->w * P->w));
        double ag = P->a * g;
        *D = (dphi / (P->w * P->w)) * ag / (1.0 + ag) - 2.0 / phi;
        *S = cm_of(P->m) * phi * sqrt(1.0 + ag);
    } else {
        *D = 0.0;
        *S = s_flat_of(P->V0);
    }
}

static double bias_ratio_f64(const oracle_params *P, double phi, double S)
{
    if (P->bias_kind == BIAS_NOISE_SCALED) return P->A;
    if (P->bias_kind == BIAS_POWER) return P->A * pow(phi, (double)P->p) / S;
    return 0.0;
}

/* One trajectory, binary32 mirror.  Returns the status; writes k, ln w and
 * the final field value. */
static int simulate_f32(const oracle_params *P, const consts_f32 *c, uint64_t t, int mode,
                        uint64_t *k_out, double *lw_out, double *phi_out)
{
    float phi = c->phi_in;
    double lw = 0.0;
    float lw32 = 0.0f, comp = 0.0f;   /* binary32 sum and Kahan's running compensation */
    uint64_t k = 0;
    float xi4[4];
    float r_mlp = 0.0f;
    int status = ST_RUNNING;
    while (status == ST_RUNNING) {
        if ((k & 3u) == 0) oracle_normals_f32(P->seed, P->stream, t, (uint32_t)(k >> 2), xi4);
        float xi = xi4[k & 3u];
        float D, S;
        drift_noise_f32(P, c, phi, &D, &S);
        float r;
        if (P->bias_kind == BIAS_MLP) {
            /* evaluated at the first step of each group of eval_every steps (1, 4, 8 or 16) */
            if (k % (uint64_t)P->eval_every == 0) r_mlp = (float)oracle_mlp_r(P, phi, (float)k * c->dN);
            r = r_mlp;
        } else {
            r = bias_ratio_f32(P, c, phi, S);
        }
        float B = r * S;
        float drift = D + B;
        /* increment first, then one rounding onto phi */
        float sxi = c->sq * xi;
        float dphi = fmaf(S, sxi, drift * c->dN);
        float nphi = phi + dphi;
        float inc = fmaf(r, c->hdN, sxi);
        float dlw = -(r * inc);
        if (mode == MODE_F32_KAHAN) {
            float y = dlw - comp;
            float tsum = lw32 + y;
            comp = (tsum - lw32) - y;
            lw32 = tsum;
        } else if (mode == MODE_F32_SUM) {
            lw32 += dlw;
        } else {
            lw += (double)dlw;
        }
        if (nphi > c->phi_uv) nphi = c->two_uv - nphi;
        phi = nphi;
        k += 1;
        if (phi <= c->phi_end) status = ST_ENDED;
        else if (k >= P->k_max) status = ST_CENSORED;
        else if (phi > c->phi_esc) status = ST_ESCAPED;
    }
    *k_out = k;
    if (mode == MODE_F32_KAHAN) *lw_out = (double)lw32 - (double)comp;
    else if (mode == MODE_F32_SUM) *lw_out = (double)lw32;
    else *lw_out = lw;
    *phi_out = (double)phi;
    return status;
}

/* One trajectory, binary64 reference on the same uniforms. */
static int simulate_f64(const oracle_params *P, uint64_t t, uint64_t *k_out, double *lw_out, double *phi_out)
{
    double phi = P->phi_in;
    double lw = 0.0;
    uint64_t k = 0;
    double xi4[4];
    const double sq = sqrt(P->dN);
    double r_mlp = 0.0;
    int status = ST_RUNNING;
    while (status == ST_RUNNING) {
        if ((k & 3u) == 0) oracle_normals_f64(P->seed, P->stream, t, (uint32_t)(k >> 2), xi4);
        double xi = xi4[k & 3u];
        double D, S;
        drift_noise_f64(P, phi, &D, &S);
        double r;
        if (P->bias_kind == BIAS_MLP) {
            if (k % (uint64_t)P->eval_every == 0) r_mlp = oracle_mlp_r(P, (float)phi, (float)((double)k * P->dN));
            r = r_mlp;
        } else {
            r = bias_ratio_f64(P, phi, S);
        }
        double nphi = phi + (D + r * S) * P->dN + S * sq * xi;
        lw += -r * (0.5 * r * P->dN + sq * xi);
        if (nphi > P->phi_uv) nphi = 2.0 * P->phi_uv - nphi;
        phi = nphi;
        k += 1;
        if (phi <= P->phi_end) status = ST_ENDED;
        else if (k >= P->k_max) status = ST_CENSORED;
        else if (phi > P->phi_esc) status = ST_ESCAPED;
    }
    *k_out = k;
    *lw_out = lw;
    *phi_out = phi;
    return status;
}

/* Simulate trajectories t0 .. t0+n-1 (every one of them, or every
 * `stride`-th id when stride > 1: t = t0 + i*stride).  Outputs are indexed
 * by i.  Returns the number of threads used. */
int oracle_simulate(const oracle_params *P, uint64_t t0, uint64_t stride, uint64_t n, int mode,
                    uint64_t *k_out, double *lw_out, double *phi_out, int32_t *status_out,
                    int n_threads)
{
    consts_f32 c;
    make_consts_f32(P, &c);
    if (stride == 0) stride = 1;
    int used = 1;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
    used = n_threads;
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
#endif
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t t = t0 + (uint64_t)i * stride;
        int st;
        if (mode == MODE_F64)
            st = simulate_f64(P, t, &k_out[i], &lw_out[i], &phi_out[i]);
        else
            st = simulate_f32(P, &c, t, mode, &k_out[i], &lw_out[i], &phi_out[i]);
        status_out[i] = st;
    }
    return used;
}

/* Exposed for the pins: binary32 D, S and r at one field value. */
void oracle_drift_noise_bias_f32(const oracle_params *P, float phi, float out[3])
{
    consts_f32 c;
    make_consts_f32(P, &c);
    float D, S;
    drift_noise_f32(P, &c, phi, &D, &S);
    out[0] = D;
    out[1] = S;
    out[2] = bias_ratio_f32(P, &c, phi, S);
}

/* Batch helpers for the exhaustive accuracy pins. */
void oracle_log_f32_batch(const float *x, float *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = oracle_log_f32(x[i]);
}

void oracle_sincos2pi_f32_batch(const float *u, float *c, float *s, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) oracle_sincos2pi_f32(u[i], &c[i], &s[i]);
}

void oracle_recip_f32_batch(const float *x, float *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = oracle_recip_f32(x[i]);
}

void oracle_sqrt_f32_batch(const float *x, float *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = oracle_sqrt_f32(x[i]);
}

void oracle_exp_f32_batch(const float *x, float *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = oracle_exp_f32(x[i]);
}

void oracle_normals_f32_batch(uint64_t seed, uint32_t stream, uint64_t t, uint32_t j0, uint32_t nj, float *out)
{
    for (uint32_t j = 0; j < nj; ++j) oracle_normals_f32(seed, stream, t, j0 + j, out + 4 * (size_t)j);
}

void oracle_normals_f64_batch(uint64_t seed, uint32_t stream, uint64_t t, uint32_t j0, uint32_t nj, double *out)
{
    for (uint32_t j = 0; j < nj; ++j) oracle_normals_f64(seed, stream, t, j0 + j, out + 4 * (size_t)j);
}

/* ------------------------------------------------------------------ */
/* Training of the learned proposal.                                    */
/*                                                                      */
/* Sec. 2.2 writes the weight of a path as the ratio of its target and  */
/* sample densities; Sec. 3.4 leaves the choice of the best bias open.  */
/* The proposal is tuned by minimising the second moment of the weights */
/* of the runs that end in a target window B*,                          */
/*     M2(theta) = E_theta[w_theta^2 1_B*] = E_0[w_0 w_theta 1_B*],      */
/* estimated on paths drawn once from the current proposal theta_0.    */
/* On a fixed path the target-measure noise increment of step k is      */
/* eta_k = r_0,k dN + sqrt(dN) xi_k (the sample-path increment with the */
/* bias drift taken out), so the weight the same path would have under  */
/* a candidate bias r_theta is                                         */
/*     ln w_theta = sum_k [ -r_theta,k eta_k + r_theta,k^2 dN/2 ].       */
/* The candidate network is held over groups of E steps (its evaluation */
/* schedule), so a path reduces to records at its evaluation points:    */
/* the network input (phi, k), H = sum of eta over the group and the    */
/* group's length n, and ln w_theta = sum_e [-r_e H_e + r_e^2 n_e dN/2]. */
/* ------------------------------------------------------------------ */
typedef struct {
    float phi;      /* field at the evaluation point (before the step)       */
    uint32_t k;     /* step index of the evaluation point                    */
    float H;        /* sum over the group of eta = fma(r_0, dN, sqrt(dN) xi) */
    uint32_t pn;    /* path index << 5 | steps in the group (1 .. 16)        */
} oracle_record;

/* Replay one path under the model's own proposal (binary32 mirror, identical to simulate_f32)
 * and cut it into records at multiples of E steps; at most cap records are written. */
static int64_t records_f32(const oracle_params *P, const consts_f32 *c, uint64_t t, uint32_t path, int E, int stride,
                           oracle_record *rec, int64_t cap, uint64_t *k_out, double *lw_out, int *st_out)
{
    float phi = c->phi_in;
    double lw = 0.0;
    uint64_t k = 0;
    float xi4[4];
    float r_mlp = 0.0f;
    int status = ST_RUNNING;
    int64_t n_rec = 0;
    float H = 0.0f, phi_e = phi;
    uint32_t k_e = 0, n_e = 0;
    while (status == ST_RUNNING) {
        if ((k & 3u) == 0) oracle_normals_f32(P->seed, P->stream, t, (uint32_t)(k >> 2), xi4);
        if (k % (uint64_t)E == 0) {
            phi_e = phi;
            k_e = (uint32_t)k;
            H = 0.0f;
            n_e = 0;
        }
        float xi = xi4[k & 3u];
        float D, S;
        drift_noise_f32(P, c, phi, &D, &S);
        float r;
        if (P->bias_kind == BIAS_MLP) {
            if (k % (uint64_t)P->eval_every == 0) r_mlp = (float)oracle_mlp_r(P, phi, (float)k * c->dN);
            r = r_mlp;
        } else {
            r = bias_ratio_f32(P, c, phi, S);
        }
        float B = r * S;
        float drift = D + B;
        float sxi = c->sq * xi;
        float dphi = fmaf(S, sxi, drift * c->dN);
        float nphi = phi + dphi;
        float inc = fmaf(r, c->hdN, sxi);
        float dlw = -(r * inc);
        lw += (double)dlw;
        H = H + fmaf(r, c->dN, sxi);
        n_e += 1;
        if (nphi > c->phi_uv) nphi = c->two_uv - nphi;
        phi = nphi;
        k += 1;
        if (phi <= c->phi_end) status = ST_ENDED;
        else if (k >= P->k_max) status = ST_CENSORED;
        else if (phi > c->phi_esc) status = ST_ESCAPED;
        if (k % (uint64_t)E == 0 || status != ST_RUNNING) {
            /* keep the groups g = 0, stride, 2 stride, ... */
            if ((k_e / (uint32_t)E) % (uint32_t)stride == 0) {
                if (n_rec < cap) {
                    rec[n_rec].phi = phi_e;
                    rec[n_rec].k = k_e;
                    rec[n_rec].H = H;
                    rec[n_rec].pn = (path << 5) | n_e;
                }
                n_rec += 1;
            }
        }
    }
    *k_out = k;
    *lw_out = lw;
    *st_out = status;
    return n_rec;
}

/* Records of the paths t_ids[0..n): path i owns rec[rec_off[i] .. rec_off[i+1]); with stride s only
 * the groups g = 0, s, 2s, ... are kept, each record then standing for s groups.  Returns the
 * number of paths whose record count did not match their slot (0 when the offsets came from
 * the same paths' step counts). */
int64_t oracle_records(const oracle_params *P, const uint64_t *t_ids, int64_t n, int E, int stride,
                       const uint64_t *rec_off, oracle_record *rec, uint64_t *k_out, double *lw_out, int32_t *st_out)
{
    consts_f32 c;
    make_consts_f32(P, &c);
    int64_t bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : bad)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int st;
        const int64_t cap = (int64_t)(rec_off[i + 1] - rec_off[i]);
        const int64_t got = records_f32(P, &c, t_ids[i], (uint32_t)i, E, stride, rec + rec_off[i], cap, &k_out[i],
                                        &lw_out[i], &st);
        st_out[i] = st;
        if (got != cap) bad += 1;
    }
    return bad;
}

/* The network being trained, in binary64 without roundings (its parameters theta are the
 * binary32 master copy; inference rounds them and the activations to bfloat16). */
static double net_f64(const oracle_params *P, const double *th, float phi, uint32_t k, float dN_f, double x[3],
                      double h1[64], double h2[64])
{
    const double *W1 = th, *b1 = th + 192, *W2 = th + 256, *b2 = th + 4352, *w3 = th + 4416, b3 = th[4480];
    const float N = (float)k * dN_f;
    x[0] = ((double)phi - (double)P->in_mean[0]) * (double)P->in_inv[0];
    x[1] = ((double)N - (double)P->in_mean[1]) * (double)P->in_inv[1];
    x[2] = ((double)(float)P->target_N - (double)P->in_mean[2]) * (double)P->in_inv[2];
    for (int u = 0; u < 64; ++u) {
        double a = b1[u];
        for (int s = 0; s < 3; ++s) a += W1[u * 3 + s] * x[s];
        h1[u] = tanh(a);
    }
    double o = b3;
    for (int u = 0; u < 64; ++u) {
        double a = b2[u];
        for (int v = 0; v < 64; ++v) a += W2[u * 64 + v] * h1[v];
        h2[u] = tanh(a);
        o += w3[u] * h2[u];
    }
    return (double)P->out_scale * o;
}

/* Two objectives over the window paths given by their records and sampled weights lw0:
 *   objective 0, the second moment:  L = log M2(theta) = log( sum_i w_0,i w_theta,i / n_total ),
 *       dL/dtheta = sum_i c_i d ln w_theta,i / dtheta,  c_i = w_0,i w_theta,i / sum_j w_0,j w_theta,j;
 *   objective 1, the cross entropy of the proposal against the target restricted to the
 *       window, KL(p_T 1_B / P(B) || q_theta) up to a constant:  L = sum_i c_i ln w_theta,i,
 *       c_i = w_0,i / sum_j w_0,j (the weights do not depend on theta),
 *       dL/dtheta = sum_i c_i d ln w_theta,i / dtheta.
 * In both, d ln w_theta / dtheta = sum_e (r_e n_e dN - H_e) d r_e / dtheta.
 * temper = beta in (0, 1] replaces w_0 by w_0^beta in the path weights c_i (beta = 1: the
 * objectives as written; smaller beta trades the bias of a tempered target for a gradient less
 * dominated by the few heaviest runs while the proposal is still poor).  rec_weight: each record
 * stands for that many groups (records kept at a stride: unbiased estimates of the path sums).
 * grad_path (n_paths x 4481 scratch) keeps the per-path sums so the total is summed in path
 * order. */
void oracle_loss_grad(const oracle_params *P, const double *theta, const oracle_record *rec, const uint64_t *rec_off,
                      int64_t n_paths, const double *lw0, double n_total, int objective, double temper,
                      double rec_weight, double *loss, double *grad, double *lw_theta, double *grad_path)
{
    const float dN_f = (float)P->dN;
    const double dN = (double)dN_f;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < n_paths; ++i) {
        double x[3], h1[64], h2[64], s = 0.0;
        for (uint64_t e = rec_off[i]; e < rec_off[i + 1]; ++e) {
            const double r = net_f64(P, theta, rec[e].phi, rec[e].k, dN_f, x, h1, h2);
            const double n = (double)(rec[e].pn & 31u);
            s += (-r * (double)rec[e].H + r * r * n * dN * 0.5) * rec_weight;
        }
        lw_theta[i] = s;
    }
    const double use_t = objective == 0 ? 1.0 : 0.0;
    double M = -INFINITY;
    for (int64_t i = 0; i < n_paths; ++i) M = fmax(M, temper * lw0[i] + use_t * lw_theta[i]);
    double S = 0.0;
    for (int64_t i = 0; i < n_paths; ++i) S += exp(temper * lw0[i] + use_t * lw_theta[i] - M);
    if (objective == 0) {
        *loss = M + log(S) - log(n_total);
    } else {
        double L = 0.0;
        for (int64_t i = 0; i < n_paths; ++i) L += exp(temper * lw0[i] - M) / S * lw_theta[i];
        *loss = L;
    }
    const double *W2 = theta + 256, *w3 = theta + 4416;
    const double osc = (double)P->out_scale;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < n_paths; ++i) {
        double *g = grad_path + (size_t)i * 4481;
        for (int j = 0; j < 4481; ++j) g[j] = 0.0;
        const double ci = exp(temper * lw0[i] + use_t * lw_theta[i] - M) / S;
        double x[3], h1[64], h2[64], d2[64];
        for (uint64_t e = rec_off[i]; e < rec_off[i + 1]; ++e) {
            const double r = net_f64(P, theta, rec[e].phi, rec[e].k, dN_f, x, h1, h2);
            const double n = (double)(rec[e].pn & 31u);
            const double go = ci * (r * n * dN - (double)rec[e].H) * osc * rec_weight;   /* d loss / d o */
            g[4480] += go;
            for (int u = 0; u < 64; ++u) {
                g[4416 + u] += go * h2[u];
                d2[u] = go * w3[u] * (1.0 - h2[u] * h2[u]);
                g[4352 + u] += d2[u];
            }
            for (int u = 0; u < 64; ++u)
                for (int v = 0; v < 64; ++v) g[256 + u * 64 + v] += d2[u] * h1[v];
            for (int v = 0; v < 64; ++v) {
                double a = 0.0;
                for (int u = 0; u < 64; ++u) a += W2[u * 64 + v] * d2[u];
                const double d1 = a * (1.0 - h1[v] * h1[v]);
                g[192 + v] += d1;
                for (int s = 0; s < 3; ++s) g[v * 3 + s] += d1 * x[s];
            }
        }
    }
    for (int j = 0; j < 4481; ++j) grad[j] = 0.0;
    for (int64_t i = 0; i < n_paths; ++i)
        for (int j = 0; j < 4481; ++j) grad[j] += grad_path[(size_t)i * 4481 + j];
}
