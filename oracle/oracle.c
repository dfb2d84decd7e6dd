/*
 * CPU oracle for the Onesweep LSD radix sort (Adinets and Merrill,
 * "Onesweep: A Faster Least Significant Digit Radix Sort for GPUs", 2022).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it. It shares no code with the GPU library.
 *
 * Plain, single-threaded, deliberately unoptimised C. Every function cites the
 * passage of the paper it follows. Counts are 64-bit so that no size limit of
 * the GPU design (30-bit status values, 32-bit shared-memory counters) leaks
 * into the checker.
 *
 * Problem statement (Section 1): for each d-bit digit place of a k-bit key a
 * radix-r sort, r = 2^d, partitions the keys into r bins by their digit at
 * that place; an LSD sort visits the p = ceil(k/d) places from least to most
 * significant, and each iteration is stable. Here the "key" is the bit field
 * [begin_bit, end_bit) of a 32- or 64-bit unsigned word, the full word is
 * carried along, and an optional 32-bit value travels with each key.
 *
 * Digit place j covers bits [begin + j*d, min(begin + (j+1)*d, end)); the last
 * place is narrower when d does not divide end - begin.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 2

/* Status word layout of the chained scan (Section 3, Figure 6): the two high
 * bits hold the status, the low 30 bits the value. */
#define STATUS_N 0u /* value not ready */
#define STATUS_L 1u /* value is the tile's local digit count */
#define STATUS_G 2u /* value is the inclusive prefix over this and all earlier tiles */

static int check_args(int key_bits, int begin_bit, int end_bit, int d)
{
    if (key_bits != 32 && key_bits != 64) return ORACLE_EINVAL;
    if (begin_bit < 0 || begin_bit > end_bit || end_bit > key_bits) return ORACLE_EINVAL;
    if (d < 1 || d > 16) return ORACLE_EINVAL;
    return ORACLE_OK;
}

static uint64_t load_key(const void *keys, int key_bits, size_t i)
{
    if (key_bits == 32) return ((const uint32_t *)keys)[i];
    return ((const uint64_t *)keys)[i];
}

static void store_key(void *keys, int key_bits, size_t i, uint64_t k)
{
    if (key_bits == 32) ((uint32_t *)keys)[i] = (uint32_t)k;
    else ((uint64_t *)keys)[i] = k;
}

/* Number of digit places p = ceil((end - begin) / d)  (Section 1). */
int oracle_num_places(int begin_bit, int end_bit, int d)
{
    if (d < 1 || end_bit < begin_bit) return -1;
    return (end_bit - begin_bit + d - 1) / d;
}

/* Bit offset and width of digit place j. */
static void place_bits(int begin_bit, int end_bit, int d, int j, int *lo, int *width)
{
    int a = begin_bit + j * d;
    int b = a + d;
    if (b > end_bit) b = end_bit;
    *lo = a;
    *width = b - a;
}

static uint64_t digit_at(uint64_t key, int lo, int width)
{
    return (key >> lo) & ((1ull << width) - 1ull);
}

/* Digit of key i at place j: exposed for tests of the decoding rule. */
uint64_t oracle_digit(uint64_t key, int begin_bit, int end_bit, int d, int j)
{
    int lo, width;
    place_bits(begin_bit, end_bit, d, j, &lo, &width);
    return digit_at(key, lo, width);
}

/*
 * Histograms of global digit counts for all places (Section 3, phase 1 and
 * Figure 5): hist[j * 2^d + v] = number of keys whose digit at place j is v.
 * The counts depend only on the multiset of keys, never on their order.
 */
int oracle_histograms(const void *keys, int key_bits, size_t n, int begin_bit,
                      int end_bit, int d, uint64_t *hist)
{
    int rc = check_args(key_bits, begin_bit, end_bit, d);
    if (rc) return rc;
    int p = oracle_num_places(begin_bit, end_bit, d);
    size_t r = (size_t)1 << d;
    memset(hist, 0, sizeof(uint64_t) * r * (size_t)p);
    for (size_t i = 0; i < n; i++) {
        uint64_t k = load_key(keys, key_bits, i);
        for (int j = 0; j < p; j++) {
            int lo, width;
            place_bits(begin_bit, end_bit, d, j, &lo, &width);
            hist[(size_t)j * r + digit_at(k, lo, width)] += 1;
        }
    }
    return ORACLE_OK;
}

/*
 * Exclusive prefix sum of each place's histogram (Section 3, phase 2;
 * Section 2 defines the exclusive prefix sum: output i is the sum of the
 * inputs before i). off[j][v] is the global bin offset of digit v at place j.
 */
void oracle_exclusive_sums(const uint64_t *hist, int p, int d, uint64_t *off)
{
    size_t r = (size_t)1 << d;
    for (int j = 0; j < p; j++) {
        uint64_t running = 0;
        for (size_t v = 0; v < r; v++) {
            off[(size_t)j * r + v] = running;
            running += hist[(size_t)j * r + v];
        }
    }
}

/* Inclusive prefix sum: what the chained scan over tiles computes for one
 * digit (Section 2, chained scan; Figure 7's final state). */
void oracle_inclusive_scan(const uint64_t *in, size_t count, uint64_t *out)
{
    uint64_t running = 0;
    for (size_t i = 0; i < count; i++) {
        running += in[i];
        out[i] = running;
    }
}

/*
 * One digit-binning iteration at place j (Section 3, phase 3 and Figure 8):
 * element i goes to global bin offset + (number of earlier elements with the
 * same digit). Walking the input in order and bumping a per-digit cursor that
 * starts at the global bin offset computes exactly that sum, so the pass is
 * stable. `off_j` holds the 2^width global bin offsets of this place.
 */
int oracle_binning_pass(const void *src_keys, const uint32_t *src_vals, void *dst_keys,
                        uint32_t *dst_vals, int key_bits, size_t n, int lo, int width,
                        const uint64_t *off_j)
{
    if (key_bits != 32 && key_bits != 64) return ORACLE_EINVAL;
    if (width < 0 || width > 16 || lo < 0 || lo + width > key_bits) return ORACLE_EINVAL;
    size_t r = (size_t)1 << width;
    uint64_t *cursor = (uint64_t *)malloc(sizeof(uint64_t) * r);
    if (!cursor) return ORACLE_ENOMEM;
    memcpy(cursor, off_j, sizeof(uint64_t) * r);
    for (size_t i = 0; i < n; i++) {
        uint64_t k = load_key(src_keys, key_bits, i);
        uint64_t v = digit_at(k, lo, width);
        uint64_t dst = cursor[v]++;
        store_key(dst_keys, key_bits, dst, k);
        if (src_vals) dst_vals[dst] = src_vals[i];
    }
    free(cursor);
    return ORACLE_OK;
}

/*
 * Complete LSD sort (Section 3, the three phases): histogram every place in
 * one pass, exclusive-sum each histogram, then bin place 0, 1, ..., p-1 in
 * turn. No pass is skipped and there is no per-tile shortcut: the checker
 * always does all the work. p = 0 (begin == end) copies the input.
 *
 * `pass_keys`, when not NULL, receives the output of every pass back to back
 * (p * n keys) so that tests can check each iteration on its own.
 * `vals_in` may be NULL (keys only).
 */
int oracle_sort(const void *keys_in, const uint32_t *vals_in, void *keys_out,
                uint32_t *vals_out, int key_bits, size_t n, int begin_bit, int end_bit,
                int d, void *pass_keys)
{
    int rc = check_args(key_bits, begin_bit, end_bit, d);
    if (rc) return rc;
    size_t kb = (size_t)key_bits / 8;
    int p = oracle_num_places(begin_bit, end_bit, d);
    size_t r = (size_t)1 << d;
    if (n == 0) return ORACLE_OK;

    uint64_t *hist = (uint64_t *)malloc(sizeof(uint64_t) * r * (size_t)(p > 0 ? p : 1));
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * r * (size_t)(p > 0 ? p : 1));
    void *src_k = malloc(kb * n), *dst_k = malloc(kb * n);
    uint32_t *src_v = NULL, *dst_v = NULL;
    if (vals_in) {
        src_v = (uint32_t *)malloc(4 * n);
        dst_v = (uint32_t *)malloc(4 * n);
    }
    if (!hist || !off || !src_k || !dst_k || (vals_in && (!src_v || !dst_v))) {
        free(hist); free(off); free(src_k); free(dst_k); free(src_v); free(dst_v);
        return ORACLE_ENOMEM;
    }
    memcpy(src_k, keys_in, kb * n);
    if (vals_in) memcpy(src_v, vals_in, 4 * n);

    oracle_histograms(src_k, key_bits, n, begin_bit, end_bit, d, hist);
    oracle_exclusive_sums(hist, p, d, off);
    for (int j = 0; j < p; j++) {
        int lo, width;
        place_bits(begin_bit, end_bit, d, j, &lo, &width);
        /* A narrower last place uses only its first 2^width offsets: the
         * digits above 2^width - 1 never occur there, so their bins are empty. */
        oracle_binning_pass(src_k, src_v, dst_k, dst_v, key_bits, n, lo, width,
                            off + (size_t)j * r);
        if (pass_keys) memcpy((char *)pass_keys + (size_t)j * n * kb, dst_k, kb * n);
        void *tk = src_k; src_k = dst_k; dst_k = tk;
        uint32_t *tv = src_v; src_v = dst_v; dst_v = tv;
    }
    memcpy(keys_out, src_k, kb * n);
    if (vals_in && vals_out) memcpy(vals_out, src_v, 4 * n);
    free(hist); free(off); free(src_k); free(dst_k); free(src_v); free(dst_v);
    return ORACLE_OK;
}

/*
 * Key order (Section 3, binning kernel: signed and floating-point keys are
 * ranked after a magnitude-preserving conversion to unsigned integers).
 * key_type 0: unsigned, unchanged. 1: two's complement; adding 2^(w-1)
 * modulo 2^w maps [-2^(w-1), 2^(w-1)) onto [0, 2^w) in order, which is
 * flipping the sign bit. 2: IEEE 754; a value with the sign bit clear moves
 * above every value with it set (sign bit flipped), and among negative values
 * a larger magnitude must come first, so all bits are flipped. descending:
 * the result is complemented, reversing the order.
 */
uint64_t oracle_ordered_bits(uint64_t key, int key_bits, int key_type, int descending)
{
    uint64_t all = key_bits == 64 ? ~(uint64_t)0 : (uint64_t)0xFFFFFFFFu;
    uint64_t top = (uint64_t)1 << (key_bits - 1);
    uint64_t k = key & all;
    if (key_type == 1) {
        k ^= top;
    } else if (key_type == 2) {
        if (k & top) k = ~k & all;
        else k ^= top;
    }
    if (descending) k = ~k & all;
    return k;
}

int oracle_ordered_keys(const void *keys, int key_bits, size_t n, int key_type, int descending,
                        void *out)
{
    if (key_bits != 32 && key_bits != 64) return ORACLE_EINVAL;
    if (key_type < 0 || key_type > 2) return ORACLE_EINVAL;
    for (size_t i = 0; i < n; i++)
        store_key(out, key_bits, i,
                  oracle_ordered_bits(load_key(keys, key_bits, i), key_bits, key_type,
                                      descending));
    return ORACLE_OK;
}

/*
 * Stable sort of keys of any type and direction: the plain sort of the
 * ordered bits (oracle_sort), carrying each key's input index as its value,
 * then a gather of the original keys and values by those indices. Bits
 * [begin_bit, end_bit) are those of the ordered key.
 */
int oracle_sort_typed(const void *keys_in, const uint32_t *vals_in, void *keys_out,
                      uint32_t *vals_out, int key_bits, size_t n, int begin_bit, int end_bit,
                      int d, int key_type, int descending)
{
    int rc = check_args(key_bits, begin_bit, end_bit, d);
    if (rc) return rc;
    if (key_type < 0 || key_type > 2 || n > 0xFFFFFFFFu) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    size_t kb = (size_t)key_bits / 8;
    void *t = malloc(kb * n), *t_out = malloc(kb * n);
    uint32_t *idx = (uint32_t *)malloc(4 * n), *idx_out = (uint32_t *)malloc(4 * n);
    if (!t || !t_out || !idx || !idx_out) {
        free(t); free(t_out); free(idx); free(idx_out);
        return ORACLE_ENOMEM;
    }
    oracle_ordered_keys(keys_in, key_bits, n, key_type, descending, t);
    for (size_t i = 0; i < n; i++) idx[i] = (uint32_t)i;
    rc = oracle_sort(t, idx, t_out, idx_out, key_bits, n, begin_bit, end_bit, d, NULL);
    if (rc == ORACLE_OK) {
        for (size_t i = 0; i < n; i++) {
            store_key(keys_out, key_bits, i, load_key(keys_in, key_bits, idx_out[i]));
            if (vals_in && vals_out) vals_out[i] = vals_in[idx_out[i]];
        }
    }
    free(t); free(t_out); free(idx); free(idx_out);
    return rc;
}

/*
 * Segmented sort: the same stable sort applied independently to every
 * segment [seg_off[s], seg_off[s+1]). Offsets must be non-decreasing, start at
 * 0 and end at n. This form is not in the paper; its definition is the
 * per-segment application of oracle_sort.
 */
int oracle_sort_segments(const void *keys_in, const uint32_t *vals_in, void *keys_out,
                         uint32_t *vals_out, int key_bits, size_t n,
                         const uint64_t *seg_off, size_t num_segments, int begin_bit,
                         int end_bit, int d)
{
    int rc = check_args(key_bits, begin_bit, end_bit, d);
    if (rc) return rc;
    size_t kb = (size_t)key_bits / 8;
    if (num_segments == 0) return n == 0 ? ORACLE_OK : ORACLE_EINVAL;
    if (seg_off[0] != 0 || seg_off[num_segments] != n) return ORACLE_EINVAL;
    for (size_t s = 0; s < num_segments; s++)
        if (seg_off[s + 1] < seg_off[s]) return ORACLE_EINVAL;
    for (size_t s = 0; s < num_segments; s++) {
        size_t a = (size_t)seg_off[s], len = (size_t)(seg_off[s + 1] - seg_off[s]);
        rc = oracle_sort((const char *)keys_in + a * kb, vals_in ? vals_in + a : NULL,
                         (char *)keys_out + a * kb, vals_out ? vals_out + a : NULL,
                         key_bits, len, begin_bit, end_bit, d, NULL);
        if (rc) return rc;
    }
    return ORACLE_OK;
}

/*
 * Segmented sort of keys of any type and direction: the typed stable sort
 * (oracle_sort_typed) applied independently to every segment
 * [seg_off[s], seg_off[s+1]), with the same offset rules as
 * oracle_sort_segments. Not in the paper; defined as that per-segment
 * application.
 */
int oracle_sort_segments_typed(const void *keys_in, const uint32_t *vals_in, void *keys_out,
                               uint32_t *vals_out, int key_bits, size_t n,
                               const uint64_t *seg_off, size_t num_segments, int begin_bit,
                               int end_bit, int d, int key_type, int descending)
{
    int rc = check_args(key_bits, begin_bit, end_bit, d);
    if (rc) return rc;
    size_t kb = (size_t)key_bits / 8;
    if (num_segments == 0) return n == 0 ? ORACLE_OK : ORACLE_EINVAL;
    if (seg_off[0] != 0 || seg_off[num_segments] != n) return ORACLE_EINVAL;
    for (size_t s = 0; s < num_segments; s++)
        if (seg_off[s + 1] < seg_off[s]) return ORACLE_EINVAL;
    for (size_t s = 0; s < num_segments; s++) {
        size_t a = (size_t)seg_off[s], len = (size_t)(seg_off[s + 1] - seg_off[s]);
        rc = oracle_sort_typed((const char *)keys_in + a * kb, vals_in ? vals_in + a : NULL,
                               (char *)keys_out + a * kb, vals_out ? vals_out + a : NULL,
                               key_bits, len, begin_bit, end_bit, d, key_type, descending);
        if (rc) return rc;
    }
    return ORACLE_OK;
}

/*
 * Final state of one chained-scan binning pass (Section 3, Figures 6 and 7f):
 * with the input cut into tiles of `tile` consecutive elements, every status
 * counter ends as status G holding the inclusive prefix, over this and all
 * earlier tiles, of the number of elements with that digit. The value is kept
 * modulo 2^30 as the 30-bit field stores it; callers keep n below 2^30.
 * status[t * 2^width + v] for tile t and digit v.
 */
int oracle_pass_status(const void *src_keys, int key_bits, size_t n, int lo, int width,
                       size_t tile, uint32_t *status)
{
    if (key_bits != 32 && key_bits != 64) return ORACLE_EINVAL;
    if (tile == 0 || width < 0 || width > 16) return ORACLE_EINVAL;
    size_t r = (size_t)1 << width;
    size_t g = (n + tile - 1) / tile;
    uint64_t *count = (uint64_t *)calloc(r, sizeof(uint64_t));
    uint64_t *col = (uint64_t *)malloc(sizeof(uint64_t) * (g ? g : 1));
    uint64_t *incl = (uint64_t *)malloc(sizeof(uint64_t) * (g ? g : 1));
    if (!count || !col || !incl) { free(count); free(col); free(incl); return ORACLE_ENOMEM; }
    for (size_t v = 0; v < r; v++) {
        for (size_t t = 0; t < g; t++) {
            size_t a = t * tile, b = a + tile < n ? a + tile : n;
            uint64_t c = 0;
            for (size_t i = a; i < b; i++)
                if (digit_at(load_key(src_keys, key_bits, i), lo, width) == v) c++;
            col[t] = c;
        }
        oracle_inclusive_scan(col, g, incl);
        for (size_t t = 0; t < g; t++)
            status[t * r + v] = (STATUS_G << 30) | (uint32_t)(incl[t] & 0x3FFFFFFFu);
    }
    free(count); free(col); free(incl);
    return ORACLE_OK;
}

/* Pack/unpack of the status word (Section 3, Figure 6). */
uint32_t oracle_status_pack(uint32_t status, uint32_t value)
{
    return (status << 30) | (value & 0x3FFFFFFFu);
}

void oracle_status_unpack(uint32_t word, uint32_t *status, uint32_t *value)
{
    *status = word >> 30;
    *value = word & 0x3FFFFFFFu;
}
