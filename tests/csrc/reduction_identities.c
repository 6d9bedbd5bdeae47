/* Exhaustive CPU check of two integer range reductions used by the step kernel's normal
 * generator, against the float reductions they replace.  Exit status 0 when every input
 * agrees.
 *
 *  1. Quarter-turn reduction of the Box-Muller angle 2 pi u, u = (2 (x >> 9) + 1) 2^-24:
 *     float form  q = rint(4u), r = u - q/4, quadrant q mod 4;
 *     word form   y = x + 2^29 (mod 2^32), quadrant y >> 30,
 *                 r = bits(0x3F000001 | (((y >> 9) & 0x1FFFFF) << 1)) - 0.625.
 *     All 2^32 words x.
 *  2. Exponent / mantissa split of ln x, f in (sqrt(1/2), sqrt 2]:
 *     float form  e = biased exponent - 127, f = 1.mant, halved (e + 1) when f > 1.41421354;
 *     bit form    i = bits(x) - 0x3F3504F4 (signed), e = i >> 23,
 *                 f = bits((i & 0x7FFFFF) + 0x3F3504F4).
 *     All positive normal binary32 x.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

static float as_f(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t as_u(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

int main(void) {
    unsigned long long bad_turn = 0, bad_log = 0;
    for (uint64_t xx = 0; xx < (1ull << 32); ++xx) {
        const uint32_t x = (uint32_t)xx;
        const float u = (float)(((x >> 9) << 1) | 1u) * 0x1p-24f;
        const float q = rintf(u * 4.0f);
        const float r = u - q * 0.25f;
        const uint32_t iq = ((uint32_t)(int)q) & 3u;
        const uint32_t y = x + 0x20000000u;
        const float r2 = as_f(0x3F000001u | (((y >> 9) & 0x1FFFFFu) << 1)) - 0.625f;
        if (as_u(r) != as_u(r2) || iq != (y >> 30)) ++bad_turn;
    }
    for (uint32_t b = 0x00800000u; b < 0x7F800000u; ++b) {
        int e = (int)(b >> 23) - 127;
        const uint32_t mant = b & 0x7FFFFFu;
        float f = as_f(mant | 0x3F800000u);
        if (f > 1.41421354f) {
            f = as_f(mant | 0x3F000000u);
            e += 1;
        }
        const int32_t i = (int32_t)(b - 0x3F3504F4u);
        const uint32_t fb = ((uint32_t)i & 0x7FFFFFu) + 0x3F3504F4u;
        if ((i >> 23) != e || fb != as_u(f)) ++bad_log;
    }
    printf("quarter-turn mismatches %llu, log-split mismatches %llu\n", bad_turn, bad_log);
    return (bad_turn == 0 && bad_log == 0) ? 0 : 1;
}
