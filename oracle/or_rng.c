/*
 * Counter-based random numbers for the oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * The paper draws every newly created piece of crystal from its statistical
 * description (Sec. 2, "Second": new material "correctly represents the
 * desired statistical structure"), and clones must diverge only through
 * material created after the cloning (Sec. 2, cloning paragraph).  A
 * counter-based generator keyed by (track key, cell, basis atom) gives both
 * properties without any stored stream state.
 *
 * Generator: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
 * published definition: per round two 64x64->128 products of counter words
 * with fixed odd multipliers, the high halves xor-ed with the other counter
 * words and the round key; the key is bumped by two Weyl constants between
 * rounds.
 */
#include <math.h>
#include "or_internal.h"

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
    *lo = (uint64_t)prod;
    *hi = (uint64_t)(prod >> 64);
}

void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t mult0 = 0xD2E7470EE14C6C93ULL, mult1 = 0xCA5A826395121157ULL;
    const uint64_t weyl0 = 0x9E3779B97F4A7C15ULL, weyl1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(mult0, c0, &hi0, &lo0);
        mulhilo64(mult1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in the open interval (0,1): the top 52 bits plus one half, times
 * 2^-52.  Every value is an exact double; neither 0 nor 1 can occur. */
double or_u01(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * (1.0 / 4503599627370496.0);
}

/* Three independent standard normal deviates for basis atom b of cell
 * (cx,cy,cz) of the crystal realisation `key` (Box-Muller on two pairs of
 * uniforms; the fourth deviate is not used). */
void or_gauss3(uint64_t key, uint64_t seed, int64_t cx, int64_t cy, int64_t cz, int b, double g[3])
{
    uint64_t ctr[4] = {(uint64_t)OR_TAG_THERMAL | ((uint64_t)b << 8), (uint64_t)cx,
                       (uint64_t)cy, (uint64_t)cz};
    uint64_t k[2] = {key, seed};
    uint64_t r[4];
    or_philox4x64(ctr, k, r);
    double u0 = or_u01(r[0]), u1 = or_u01(r[1]), u2 = or_u01(r[2]), u3 = or_u01(r[3]);
    double rad0 = sqrt(-2.0 * log(u0));
    double rad1 = sqrt(-2.0 * log(u2));
    g[0] = rad0 * cos(2.0 * OR_PI * u1);
    g[1] = rad0 * sin(2.0 * OR_PI * u1);
    g[2] = rad1 * cos(2.0 * OR_PI * u3);
}

/* Key of clone i made when a track with key `key` crosses threshold k. */
uint64_t or_child_key(uint64_t key, uint64_t seed, int32_t k, int32_t i)
{
    uint64_t ctr[4] = {OR_TAG_CHILD_KEY, (uint64_t)(int64_t)k, (uint64_t)(int64_t)i, 0};
    uint64_t kk[2] = {key, seed};
    uint64_t r[4];
    or_philox4x64(ctr, kk, r);
    return r[0];
}

/* Keys of the next cloning level: out[j * n_clones + i] = key of copy i made
 * when a track with key in[j] crosses cloning depth k. */
void or_child_keys(const uint64_t* in, int64_t n, uint64_t seed, int32_t k, int32_t n_clones, uint64_t* out)
{
    for (int64_t j = 0; j < n; ++j)
        for (int32_t i = 0; i < n_clones; ++i) out[j * n_clones + i] = or_child_key(in[j], seed, k, i);
}

/* Crystal-realisation key of primary `id`. */
uint64_t or_primary_key(uint64_t seed, int64_t id)
{
    uint64_t ctr[4] = {OR_TAG_PRIMARY_KEY, (uint64_t)id, 0, 0};
    uint64_t kk[2] = {seed, 0};
    uint64_t r[4];
    or_philox4x64(ctr, kk, r);
    return r[0];
}
