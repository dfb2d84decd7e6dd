/*
 * Multithreaded LSD radix sort on the host: the secondary CPU baseline of the
 * benchmark (the primary one is the single-threaded oracle). Benchmark
 * infrastructure only; the HIP library never uses it.
 *
 * Stable LSD sort over 8-bit digit places (Section 1 of the paper: p = k / 8
 * passes of a stable counting scatter), run with OpenMP on all host cores.
 * A place whose keys all share one digit is skipped (its permutation is the
 * identity); the digit counts of a place do not depend on the order of the
 * keys, so they are taken from the input once, for every place. Each executed
 * pass cuts its source into one contiguous chunk per thread; each thread
 * counts its chunk's digits; the counts are scanned digit-major, then
 * chunk-major (bin v of chunk t starts after every key of a smaller digit
 * and after bin v of the chunks before t, which keeps the scatter stable);
 * each thread then scatters its chunk in input order.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RADIX 256
#define MAX_THREADS 256

/* Returns 0 on success, 1 on bad arguments, 2 when memory runs out.
 * keys_out receives the keys sorted ascending as unsigned integers of the
 * whole key width; vals_out (when vals_in is not NULL) the values in the same
 * order. threads <= 0 uses every core OpenMP reports. */
int cpu_lsd_sort(const void *keys_in, void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                 int key_bits, size_t n, int threads) {
  if (key_bits != 32 && key_bits != 64) return 1;
  if (n == 0) return 0;
  if (!keys_in || !keys_out || (vals_in && !vals_out)) return 1;
  if (threads <= 0) threads = omp_get_max_threads();
  if (threads > MAX_THREADS) threads = MAX_THREADS;
  const size_t kb = (size_t)key_bits / 8;
  const int places = key_bits / 8;
  size_t(*cnt)[RADIX] = calloc((size_t)threads * (size_t)places, sizeof *cnt);
  if (!cnt) return 2;

  /* Digit counts of every place, from the input (one read). */
#pragma omp parallel num_threads(threads)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
    const size_t lo = n * (size_t)t / (size_t)nt, hi = n * (size_t)(t + 1) / (size_t)nt;
    size_t(*c)[RADIX] = cnt + (size_t)t * places;
    for (size_t i = lo; i < hi; ++i) {
      const uint64_t k = key_bits == 32 ? ((const uint32_t *)keys_in)[i]
                                        : ((const uint64_t *)keys_in)[i];
      for (int j = 0; j < places; ++j) c[j][(k >> (8 * j)) & 0xFFu]++;
    }
  }
  int runs[8], nruns = 0;
  for (int j = 0; j < places; ++j) {
    int trivial = 0;
    for (int v = 0; v < RADIX && !trivial; ++v) {
      size_t total = 0;
      for (int t = 0; t < threads; ++t) total += cnt[(size_t)t * places + j][v];
      trivial = total == n;
    }
    if (!trivial) runs[nruns++] = j;
  }
  if (nruns == 0) {
    if (keys_out != keys_in) memmove(keys_out, keys_in, n * kb);
    if (vals_in && vals_out != vals_in) memmove(vals_out, vals_in, n * sizeof(uint32_t));
    free(cnt);
    return 0;
  }

  void *tmp_k = malloc(n * kb);
  uint32_t *tmp_v = vals_in ? malloc(n * sizeof(uint32_t)) : NULL;
  if (!tmp_k || (vals_in && !tmp_v)) {
    free(tmp_k);
    free(tmp_v);
    free(cnt);
    return 2;
  }
  const void *src_k = keys_in;
  const uint32_t *src_v = vals_in;
  for (int r = 0; r < nruns; ++r) {
    const int shift = 8 * runs[r];
    /* The last executed pass writes keys_out; earlier ones alternate back
     * from it, so no final copy is needed. */
    const int to_out = (nruns - 1 - r) % 2 == 0;
    void *dst_k = to_out ? keys_out : tmp_k;
    uint32_t *dst_v = vals_in ? (to_out ? vals_out : tmp_v) : NULL;
#pragma omp parallel num_threads(threads)
    {
      const int t = omp_get_thread_num(), nt = omp_get_num_threads();
      const size_t lo = n * (size_t)t / (size_t)nt, hi = n * (size_t)(t + 1) / (size_t)nt;
      size_t *c = cnt[t];
      memset(c, 0, RADIX * sizeof(size_t));
      if (key_bits == 32)
        for (size_t i = lo; i < hi; ++i) c[(((const uint32_t *)src_k)[i] >> shift) & 0xFFu]++;
      else
        for (size_t i = lo; i < hi; ++i) c[(((const uint64_t *)src_k)[i] >> shift) & 0xFFu]++;
#pragma omp barrier
#pragma omp single
      {
        size_t run = 0;
        for (int v = 0; v < RADIX; ++v)
          for (int u = 0; u < nt; ++u) {
            const size_t here = cnt[u][v];
            cnt[u][v] = run;
            run += here;
          }
      }
      if (key_bits == 32) {
        const uint32_t *s = src_k;
        uint32_t *d = dst_k;
        for (size_t i = lo; i < hi; ++i) {
          const size_t p = c[(s[i] >> shift) & 0xFFu]++;
          d[p] = s[i];
          if (dst_v) dst_v[p] = src_v[i];
        }
      } else {
        const uint64_t *s = src_k;
        uint64_t *d = dst_k;
        for (size_t i = lo; i < hi; ++i) {
          const size_t p = c[(s[i] >> shift) & 0xFFu]++;
          d[p] = s[i];
          if (dst_v) dst_v[p] = src_v[i];
        }
      }
    }
    src_k = dst_k;
    src_v = dst_v;
  }
  free(tmp_k);
  free(tmp_v);
  free(cnt);
  return 0;
}

/* Threads a call with threads <= 0 runs on. */
int cpu_lsd_default_threads(void) { return omp_get_max_threads(); }
