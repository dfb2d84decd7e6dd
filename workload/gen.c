/*
 * Fast form of the SplitMix64 counter-based generator of workload/__init__.py
 * (Steele, Lea and Flood, OOPSLA 2014). Input data only: no sorting
 * arithmetic. The numpy implementation is the definition; tests check that
 * both produce identical words.
 */
#include <stddef.h>
#include <stdint.h>

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* out[i] = mix64(base + (start + i + 1) * gamma) */
void gen_words(uint64_t base, uint64_t start, size_t n, uint64_t *out)
{
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    for (size_t i = 0; i < n; i++) out[i] = mix64(base + (start + i + 1) * gamma);
}

/* AND of streams: out[i] &= word (in place), for AND-of-q keys */
void gen_and_words(uint64_t base, uint64_t start, size_t n, uint64_t *inout)
{
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    for (size_t i = 0; i < n; i++) inout[i] &= mix64(base + (start + i + 1) * gamma);
}

/* High halves of words as 32-bit keys. */
void gen_words_hi32(uint64_t base, uint64_t start, size_t n, uint32_t *out)
{
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    for (size_t i = 0; i < n; i++) out[i] = (uint32_t)(mix64(base + (start + i + 1) * gamma) >> 32);
}

void gen_and_words_hi32(uint64_t base, uint64_t start, size_t n, uint32_t *inout)
{
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    for (size_t i = 0; i < n; i++)
        inout[i] &= (uint32_t)(mix64(base + (start + i + 1) * gamma) >> 32);
}
