/*
 * onesweep.h: C ABI of an MI355X (gfx950) implementation of Onesweep, the
 * single-pass LSD radix sort of Adinets and Merrill (arXiv 2206.01784).
 *
 * The sort (Section 3) runs as three phases:
 *   1. one upfront pass that histograms every digit place at once,
 *   2. an exclusive sum of each place's histogram (global bin offsets),
 *   3. one chained-scan digit-binning kernel per digit place, which ranks the
 *      keys of a tile, obtains the tile's bin-relative offsets by decoupled
 *      look-back over per-tile status words and scatters keys (and values)
 *      stably, for about 2n global memory operations per place.
 *
 * Conventions shared by every entry point:
 *  - Device pointers (d_*) are caller-owned device memory; the library never
 *    allocates, frees or synchronises on the sort path and keeps no pointer
 *    once the enqueued work has completed.
 *  - Two-phase temporary storage: when d_temp is NULL the call only writes the
 *    required size to *temp_bytes and enqueues nothing (no GPU is touched).
 *    d_temp must be 256-byte aligned and at least that large.
 *  - All work is enqueued on `stream` (0 = the null stream) and is
 *    asynchronous; results are valid after the caller synchronises. The
 *    enqueued sequence uses kernels only (no memset or memcpy nodes), so a
 *    caller may capture it into a HIP graph.
 *  - Keys are 32- or 64-bit words ordered by the bit field
 *    [begin_bit, end_bit) (0 <= begin_bit <= end_bit <= key_bits) of their
 *    ordered bits: unsigned integers by default, signed or IEEE 754 keys and
 *    descending order through onesweep_config_t.key_type / descending; the
 *    whole key word is carried to the output. Values are opaque 32-bit
 *    payloads that travel with their keys.
 *  - Digit places are 8 bits wide (r = 256 bins); place j covers bits
 *    [begin_bit + 8j, min(begin_bit + 8j + 8, end_bit)), so
 *    p = ceil((end_bit - begin_bit) / 8) places (Section 1).
 *  - The output is always stable, because an LSD sort is stable by
 *    construction (Section 1); the `stable` argument is accepted for
 *    interface symmetry and ignored.
 *  - The chained-scan status words hold 30-bit values (Section 3, "Handling
 *    very large problems"): one chained scan covers fewer than 2^30 keys.
 *    Whole plain sorts (onesweep_sort_keys/pairs) bin large inputs in strips
 *    of at most 2^29 keys, each its own chained scan whose last tile hands
 *    the next strip its bin starts. From 2^31 elements on, and where the
 *    keys take more than 4 GiB (32-bit keys from 2^30 + 1, 64-bit keys from
 *    2^29 + 1: below that, positions are stored through buffer resources,
 *    whose offsets are 32-bit), they also keep 64-bit histogram counts (the
 *    upfront histogram runs over portions of at most 2^30 keys), 64-bit bin
 *    starts and 64-bit element positions, as that section describes, and
 *    accept n below 2^36; at those sizes only
 *    the default tile shape of each key width and value presence is built
 *    (other tile configurations return ONESWEEP_ERROR_UNSUPPORTED) and the
 *    reduce-then-scan baseline is not. The other entry points accept n
 *    below 2^30 (onesweep_binning_pass also at most 4 GiB of keys: 64-bit
 *    keys up to 2^29). Larger n returns ONESWEEP_ERROR_TOO_LARGE.
 *  - Errors are returned as status codes; nothing is enqueued when argument
 *    validation fails. onesweep_last_error() describes the last failure of
 *    the calling thread.
 */
#ifndef ONESWEEP_H
#define ONESWEEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *onesweep_stream_t; /* same type as hipStream_t */

typedef enum {
    ONESWEEP_SUCCESS = 0,
    ONESWEEP_ERROR_INVALID_VALUE = 1,     /* bad pointer, width, bit range, overlap */
    ONESWEEP_ERROR_TOO_LARGE = 2,         /* n beyond the entry point's limit (2^36 or 2^30) */
    ONESWEEP_ERROR_INSUFFICIENT_TEMP = 3, /* *temp_bytes below the required size */
    ONESWEEP_ERROR_HIP = 4,               /* a HIP runtime call failed */
    ONESWEEP_ERROR_UNSUPPORTED = 5        /* configuration not built into the library */
} onesweep_status_t;

/* Kinds of kernel launch reported through onesweep_trace_t. */
typedef enum {
    ONESWEEP_KERNEL_RESET = 0,     /* clears histograms, tile counters, status words */
    ONESWEEP_KERNEL_HISTOGRAM = 1, /* phase 1: all-place histogram */
    ONESWEEP_KERNEL_SCAN = 2,      /* phase 2: exclusive sums and pass plan */
    ONESWEEP_KERNEL_BINNING = 3,   /* phase 3: one chained-scan binning pass */
    ONESWEEP_KERNEL_COPY = 4,      /* final copy when no pass (or an odd count) ran */
    ONESWEEP_KERNEL_CLASSIFY = 5,  /* segmented sort: offsets -> classes and tiles */
    ONESWEEP_KERNEL_LDS_SORT = 6,  /* segmented sort: whole segments sorted in LDS */
    ONESWEEP_KERNEL_UPSWEEP = 7,   /* reduce-then-scan: per-tile digit counts */
    ONESWEEP_KERNEL_TILE_SCAN = 8, /* reduce-then-scan: prefix of counts over tiles */
    ONESWEEP_KERNEL_DOWNSWEEP = 9  /* reduce-then-scan: rank and scatter one place */
} onesweep_kernel_kind_t;

/* Values of onesweep_config_t.key_type: how the key bits are ordered. */
typedef enum {
    ONESWEEP_KEY_UNSIGNED = 0, /* unsigned integers */
    ONESWEEP_KEY_SIGNED = 1,   /* two's-complement integers */
    ONESWEEP_KEY_FLOAT = 2     /* IEEE 754 binary32 (32-bit keys) or binary64 (64-bit):
                                  -NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN, NaNs
                                  by payload bits */
} onesweep_key_type_t;

/* Values of onesweep_config_t.algorithm. */
typedef enum {
    ONESWEEP_ALGORITHM_ONESWEEP = 0,        /* Section 3: chained-scan digit binning */
    ONESWEEP_ALGORITHM_REDUCE_THEN_SCAN = 1 /* Section 2 baseline: upsweep, scan, downsweep */
} onesweep_algorithm_t;

#define ONESWEEP_TRACE_MAX 64

/*
 * Optional per-launch timing. The caller creates 2 * capacity HIP events with
 * timing enabled and passes their handles in `events`; the library records
 * events[2i] on the stream just before launch i and events[2i + 1] just after
 * it, sets kinds[i] and sets `count` to the number of launches recorded
 * (launches beyond capacity are not recorded). Elapsed times are read by the
 * caller with hipEventElapsedTime after synchronising.
 */
typedef struct {
    void **events;   /* hipEvent_t handles, 2 * capacity of them */
    int capacity;    /* launches that can be recorded */
    int count;       /* out: launches recorded by the last call */
    int kinds[ONESWEEP_TRACE_MAX]; /* out: onesweep_kernel_kind_t per launch */
} onesweep_trace_t;

/*
 * Kernel configuration. A NULL config, or 0 in a field, selects the default:
 * the autotuned plain configuration, a table of the fastest tile shape per
 * key width, value presence and input size measured on MI355X over sizes
 * 2^17..2^28 (smaller tiles below 2^18-2^19 keys). block_threads x
 * items_per_thread is the binning tile size T (Section 3 dispatches one
 * workgroup per tile). Only combinations compiled into the library are
 * accepted; others return ONESWEEP_ERROR_UNSUPPORTED.
 */
typedef struct {
    int digit_bits;          /* width d of a digit place: 0 (= 8) or 4..8; the sort
                                makes ceil((end_bit - begin_bit) / d) passes, at
                                most 8 (more returns ONESWEEP_ERROR_UNSUPPORTED).
                                8 is fastest on MI355X (Table 2's trade-off: a
                                binning pass costs about the same at any width) */
    int block_threads;       /* binning workgroup size: 256, 512 or 1024 */
    int items_per_thread;    /* binning items per thread */
    int hist_blocks_per_cu;  /* histogram grid = CUs x this (persistent, tile-cyclic) */
    int rank_algorithm;      /* wave-level digit match: 0 default, 1 one ballot per
                                digit bit, 2 LDS presence masks, 3 ballots with
                                one LDS atomic per digit group (same output) */
    int segment_limits[3];   /* segmented sort only: longest segment sorted whole in
                                LDS by the 64-, 256- and 1024-thread class; 0 =
                                the class's capacity (512, 2048, 8192 keys), -1 =
                                class unused. Longer segments are binned tile by
                                tile. */
    int segment_streams;     /* segmented sort only: 0 = two streams when a batch has
                                both LDS-sorted and tiled segments (see
                                onesweep_sort_segments), 1 = the caller's stream only */
    int algorithm;           /* onesweep_sort_keys/pairs only, onesweep_algorithm_t:
                                0 = Onesweep; 1 = the reduce-then-scan baseline
                                (Section 2, "Reduce-then-scan digit binning"): per
                                digit place an upsweep that counts every tile's
                                digits, a scan of those counts over tiles and a
                                downsweep that ranks and scatters, ~3n memory
                                operations per place instead of ~2n. Same output;
                                built for the default tile shapes with ballot
                                ranking (others: ONESWEEP_ERROR_UNSUPPORTED). The
                                segmented sort and onesweep_binning_pass accept 0
                                only (else ONESWEEP_ERROR_INVALID_VALUE). */
    int key_type;            /* onesweep_key_type_t. Signed and floating-point keys
                                are ordered through a bit transform that maps their
                                order onto unsigned order (Section 3 names such
                                transforms for signed and floating-point keys): the
                                sign bit is flipped, and negative floating-point keys
                                have every bit flipped. Keys are stored unchanged;
                                the transform only decides digits, so begin_bit and
                                end_bit select bits of the transformed key. Applies to
                                every entry point that takes a config. */
    int descending;          /* 1: descending order (digits of the complemented
                                transformed key), still stable: equal keys keep their
                                input order. 0: ascending. */
    int strip_log2;          /* onesweep_sort_keys/pairs only: each binning pass runs
                                as consecutive strips of at most 2^strip_log2 keys
                                (whole tiles, at least one), each strip its own
                                chained scan whose last tile hands the next strip its
                                bin starts (Section 3, handling very large problems).
                                0 = 29, the default; else 11..29. Smaller strips only
                                serve tests of inputs below 2^29. */
    int lookback_spin_limit; /* bound of the look-back wait (Section 3: a tile
                                walks back over its predecessors' status words,
                                waiting on N, until it meets an inclusive prefix):
                                after this many polls of its window of
                                predecessors without meeting one, the tile gives
                                up, records a look-back error in temporary storage
                                and carries on with a wrong sum, so a protocol fault
                                ends the kernel (with wrong output) instead of
                                hanging the GPU. 0 = 2^22 polls (seconds; a
                                legitimate look-back takes a few). Where the error
                                is recorded: onesweep_binning_pass documents it; for
                                the other entry points it is internal. Negative
                                values are invalid. */
    onesweep_trace_t *trace; /* optional launch timing, may be NULL */
} onesweep_config_t;

/*
 * Sort n keys (Section 3, all three phases).
 * d_keys_in may equal d_keys_out (in-place); partial overlap is invalid.
 * key_bits is 32 or 64. Null pointers are accepted when n == 0.
 */
onesweep_status_t onesweep_sort_keys(void *d_temp, size_t *temp_bytes, const void *d_keys_in,
                                     void *d_keys_out, size_t n, int key_bits, int begin_bit,
                                     int end_bit, int stable, const onesweep_config_t *cfg,
                                     onesweep_stream_t stream);

/*
 * Sort n (key, value) pairs: keys as in onesweep_sort_keys, values are
 * uint32 and follow their keys (Section 3: values are loaded after the keys
 * are ranked and scattered with the same destinations).
 */
onesweep_status_t onesweep_sort_pairs(void *d_temp, size_t *temp_bytes, const void *d_keys_in,
                                      void *d_keys_out, const uint32_t *d_vals_in,
                                      uint32_t *d_vals_out, size_t n, int key_bits,
                                      int begin_bit, int end_bit, int stable,
                                      const onesweep_config_t *cfg, onesweep_stream_t stream);

/*
 * Allocation-free keys-only sort, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops and harnesses
 * that forbid hipMalloc. Same arguments, semantics and output as
 * onesweep_sort_keys, without d_temp / temp_bytes: the temporary storage is
 * a library-owned device array of ONESWEEP_NOALLOC_SCRATCH_BYTES (64 MiB) on
 * each GPU the library runs on, held until the process ends. The call
 * allocates nothing; it enqueues kernels only (graph-capturable).
 *  - Size limit: the temporary storage onesweep_sort_keys would need (its
 *    size query, which depends on n, key_bits, the bit range and cfg) must
 *    fit the array; with the default configuration that is about 15.9
 *    million 32-bit or 7.7 million 64-bit keys. Larger inputs return
 *    ONESWEEP_ERROR_TOO_LARGE before anything is enqueued.
 *  - The first call on a device looks up the array's device address
 *    (hipGetSymbolAddress, which may load the library's code on that
 *    device); make that call outside graph capture.
 *  - Every call on one GPU uses the same array: calls that overlap on one
 *    GPU (concurrent streams, threads or processes sharing the library
 *    instance) race and give wrong results; serialise them. Each call clears
 *    what must start at zero, so the previous call's contents do not matter.
 * Other errors as in onesweep_sort_keys.
 */
#define ONESWEEP_NOALLOC_SCRATCH_BYTES (64u << 20)
onesweep_status_t onesweep_sort_keys_noalloc(const void *d_keys_in, void *d_keys_out, size_t n,
                                             int key_bits, int begin_bit, int end_bit,
                                             int stable, const onesweep_config_t *cfg,
                                             onesweep_stream_t stream);

/*
 * Phase 1 alone (Section 3, upfront histogram kernel): d_hist[j * 256 + v]
 * receives the number of keys whose digit at place j is v (digits of the
 * key bits as cfg's key_type and descending order them), for all
 * p = ceil((end_bit - begin_bit) / d) places of d = cfg's digit_bits (8 by
 * default) bits; entries v >= 2^d stay 0. d_hist must hold p * 256 uint32
 * words; it is cleared first. n < 2^30.
 */
onesweep_status_t onesweep_histogram(const void *d_keys, size_t n, int key_bits, int begin_bit,
                                     int end_bit, uint32_t *d_hist,
                                     const onesweep_config_t *cfg, onesweep_stream_t stream);

/*
 * Phase 3, one binning iteration (Section 3, chained scan digit-binning
 * kernel): stably scatter the n keys (and values, when d_src_vals is not
 * NULL) of src into dst by the digit (k >> shift) & (2^width - 1), where k
 * is the key's bits as cfg's key_type and descending order them, with
 * d_bin_offsets[v] (256 uint32, device) the global start of bin v, which is
 * the exclusive sum of the digit counts. 1 <= width <= 8,
 * shift + width <= key_bits. src and dst must not overlap.
 * Temp layout (documented so tests can read the chained-scan state): bytes
 * [0, 256) hold the tile counter (uint32 0) and the error word (uint32 1:
 * bit 0 set when a tile gave up waiting, see
 * onesweep_config_t.lookback_spin_limit; bit 1 set when a tile found the
 * destination run of one of its digits outside [0, n), from offsets that do
 * not match the keys' digit counts: that tile writes nothing), then
 * ceil(n / T) rows of 256 uint32
 * status words (row = tile, column = digit; Figure 6 layout: 2-bit status
 * above a 30-bit value). After a pass without look-back error every word
 * holds status G (2) and the tile's inclusive prefix count.
 */
onesweep_status_t onesweep_binning_pass(void *d_temp, size_t *temp_bytes,
                                        const void *d_src_keys, void *d_dst_keys,
                                        const uint32_t *d_src_vals, uint32_t *d_dst_vals,
                                        size_t n, int key_bits, int shift, int width,
                                        const uint32_t *d_bin_offsets,
                                        const onesweep_config_t *cfg,
                                        onesweep_stream_t stream);

/*
 * Batched segmented sort: for every s < num_segments, the keys (and values)
 * in [d_seg_offsets[s], d_seg_offsets[s + 1]) are sorted as in
 * onesweep_sort_pairs, independently of every other segment; no key leaves
 * its segment. This batching is not in the paper: each segment is sorted by
 * the paper's method (Section 3), or, when it fits one workgroup's LDS, by
 * the same digit passes run entirely in LDS (one read and one write of the
 * segment).
 *  - d_seg_offsets: num_segments + 1 uint32 in device memory, read only on the
 *    device (the host never synchronises): non-decreasing, first 0, last n.
 *    Empty segments are allowed. Offsets that break these rules are detected
 *    on the device: then nothing is written to the outputs and the first
 *    uint32 of d_temp reads 1 after the call completes (0 otherwise; it is
 *    not written when n == 0). With begin_bit == end_bit the offsets are not
 *    read and the output is a copy of the input.
 *  - d_vals_in / d_vals_out: both NULL for keys only.
 *  - In-place (in == out) is allowed for keys and for values; partial
 *    overlap is invalid. The offsets must not overlap an output or d_temp.
 *  - n and num_segments must be below 2^30; num_segments == 0 requires n == 0.
 *  - cfg->segment_limits picks the segment classes; block_threads and
 *    items_per_thread pick the binning tile of the longer segments (a
 *    subset of the shapes of onesweep_sort_pairs is built for it).
 * The enqueued sequence is a fixed list of kernels whatever the offsets, so
 * it can be captured once and replayed. When the batch can hold both
 * LDS-sorted and tiled segments (and no trace is requested), the LDS-sort
 * kernels run on a library-owned second stream, forked from and joined back
 * to `stream` with events, so they overlap the tiled segments' passes. That
 * stream and its two events are created once per device, on the first such
 * call made outside graph capture (calls inside a capture before then use
 * one stream), and live until the process ends. Concurrent calls on one
 * device share the second stream; while one call is being captured, no other
 * thread may issue a segmented sort on that device until the capture ends.
 */
onesweep_status_t onesweep_sort_segments(void *d_temp, size_t *temp_bytes,
                                         const void *d_keys_in, void *d_keys_out,
                                         const uint32_t *d_vals_in, uint32_t *d_vals_out,
                                         size_t n, const uint32_t *d_seg_offsets,
                                         size_t num_segments, int key_bits, int begin_bit,
                                         int end_bit, int stable, const onesweep_config_t *cfg,
                                         onesweep_stream_t stream);

/*
 * Autotuner of the segmented sort (not in the paper): times
 * onesweep_sort_segments on the caller's data for every built tile shape of
 * the segmented path (32-bit keys: 256x8, 256x16, 512x16, 1024x8, 1024x11,
 * 1024x16, 1024x19;
 * 64-bit keys: 256x8, 256x16, 512x8, 1024x8, 1024x9, 1024x14) crossed with seven
 * settings of the segment class limits and with 8- and 7-bit digits (7 only
 * where the bit range makes at most 8 places)
 * (`repetitions` timed runs each, after one warm-up), writes the fastest
 * configuration to *cfg_out and leaves the output sorted by it. Arguments as
 * in onesweep_sort_segments, except that input and output must not alias
 * (the input is sorted many times). Temp storage: the largest any candidate
 * needs (size query with d_temp == NULL). Unlike the sort, this call creates
 * two HIP events and synchronises on them; it is not graph-capturable.
 * On input, cfg_out->key_type and cfg_out->descending select the key order
 * (other fields are ignored); on return *cfg_out is the chosen configuration
 * with that order and a NULL trace. cfg_out may be NULL for the size query
 * (unsigned ascending).
 */
onesweep_status_t onesweep_tune_segments(void *d_temp, size_t *temp_bytes,
                                         const void *d_keys_in, void *d_keys_out,
                                         const uint32_t *d_vals_in, uint32_t *d_vals_out,
                                         size_t n, const uint32_t *d_seg_offsets,
                                         size_t num_segments, int key_bits, int begin_bit,
                                         int end_bit, int repetitions,
                                         onesweep_config_t *cfg_out, onesweep_stream_t stream);

/*
 * ---- Learned configuration selection (not in the paper; the paper's
 * kernels are tuned by hand, Table 2). A small MLP predicts, from features
 * of a key sample, each configuration's sort time relative to the fastest,
 * and the selector picks the smallest prediction. The choice never changes
 * the sort's output (every configuration produces the unique stable order);
 * it changes the binning tile shape and the ranking method.
 *
 * Features (ONESWEEP_FEATURES floats): for each of the 8 digit places
 * (Section 1's p places of 8 bits over [begin_bit, end_bit); places past p
 * are zero) a 256-bin histogram of min(n, 4096) keys sampled at indices
 * floor(i * n / m), as fractions of the sample; then log2(n) / 32,
 * key_bits / 64 and has_values.
 *
 * Network (float32, ONESWEEP_MODEL_PARAMS parameters in one flat array):
 * a place encoder shared by the 8 places (256 -> 16, ReLU), the 8 encodings
 * and 3 scalars concatenated (131) -> 64 ReLU -> 64 ReLU -> 12 outputs.
 * Layout: We[256][16], be[16], W1[131][64], b1[64], W2[64][64], b2[64],
 * W3[64][12], b3[12], row-major with the input index first.
 *
 * Training: masked mean squared error between the outputs and targets
 * log(time_c / fastest time) of the configurations c that apply (mask 1),
 * then Adam (Kingma and Ba, arXiv 1412.6980; beta1 0.9, beta2 0.999,
 * eps 1e-8). Training batches pass the histogram part (batch x 2048, row
 * b = features[0:2048] of input b) and the scalar part (batch x 3)
 * separately.
 *
 * Model objects own device memory (allocated by create/load on the current
 * device, freed by onesweep_model_free); these calls may allocate and
 * synchronise and are not for graph capture, except onesweep_features and
 * onesweep_model_infer, which enqueue one kernel each.
 */
#define ONESWEEP_FEATURES 2051
#define ONESWEEP_MODEL_CLASSES 12
#define ONESWEEP_MODEL_PARAMS 17500

typedef struct onesweep_model onesweep_model_t;

/* New model: zero parameters, the default class table (every tile shape of
 * the plain sort with both ranking methods). max_batch bounds the training
 * batch (1..65536). */
onesweep_status_t onesweep_model_create(int max_batch, onesweep_model_t **model);
/* Model from a file written by onesweep_model_save (parameters and class
 * table); Adam state starts at zero. */
onesweep_status_t onesweep_model_load(const char *path, int max_batch, onesweep_model_t **model);
onesweep_status_t onesweep_model_save(const onesweep_model_t *model, const char *path);
void onesweep_model_free(onesweep_model_t *model);
size_t onesweep_model_num_params(void);
/* Host <-> device copies of the flat parameters (count must equal
 * ONESWEEP_MODEL_PARAMS); set also resets the Adam state and step. */
onesweep_status_t onesweep_model_set_params(onesweep_model_t *model, const float *host_params,
                                            size_t count);
onesweep_status_t onesweep_model_get_params(const onesweep_model_t *model, float *host_params,
                                            size_t count);
/* Configuration of class `index` (0..11) and its key-width mask (bit 0:
 * 32-bit keys, bit 1: 64-bit keys). */
onesweep_status_t onesweep_model_class(const onesweep_model_t *model, int index,
                                       onesweep_config_t *cfg_out, int *key_bits_mask);

/* Features of n device keys into d_features (ONESWEEP_FEATURES floats,
 * device). One kernel. */
onesweep_status_t onesweep_features(const void *d_keys, size_t n, int key_bits, int begin_bit,
                                    int end_bit, int has_values, float *d_features,
                                    onesweep_stream_t stream);
/* One forward pass (one kernel): d_out[12] predictions, *d_choice = the
 * class with the smallest prediction among the set bits of class_mask
 * (-1 if none). */
onesweep_status_t onesweep_model_infer(const onesweep_model_t *model, const float *d_features,
                                       unsigned class_mask, float *d_out, int *d_choice,
                                       onesweep_stream_t stream);
/* Batched forward (the training path): d_out[batch][12]. */
onesweep_status_t onesweep_model_forward(onesweep_model_t *model, const float *d_hist,
                                         const float *d_scalars, int batch, float *d_out,
                                         onesweep_stream_t stream);
/* Loss (d_loss, 1 float, may be NULL) and its gradient with respect to
 * every parameter (d_grad, ONESWEEP_MODEL_PARAMS floats, parameter layout).
 * d_y and d_mask: batch x 12. */
onesweep_status_t onesweep_model_gradients(onesweep_model_t *model, const float *d_hist,
                                           const float *d_scalars, const float *d_y,
                                           const float *d_mask, int batch, float *d_grad,
                                           float *d_loss, onesweep_stream_t stream);
/* gradients, then one Adam step with learning rate lr. */
onesweep_status_t onesweep_model_train_step(onesweep_model_t *model, const float *d_hist,
                                            const float *d_scalars, const float *d_y,
                                            const float *d_mask, int batch, float lr,
                                            float *d_loss, onesweep_stream_t stream);
/* Configuration for sorting these keys: features and one forward pass in a
 * single kernel, the class predicted fastest among those that apply to
 * key_bits (the class holding the autotuned default tile shape stays the
 * choice unless another is predicted faster by more than about 2%), then a
 * synchronisation of `stream` to read the choice (written by the kernel to
 * pinned host memory). A NULL model (or n == 0) yields the library default
 * (fields 0). cfg_out->key_type and cfg_out->descending are read on input
 * and kept (the features see the raw key bits); cfg_out->trace is NULL.
 * Calls on one model must not overlap. */
onesweep_status_t onesweep_select_config(const onesweep_model_t *model, const void *d_keys,
                                         size_t n, int key_bits, int begin_bit, int end_bit,
                                         int has_values, onesweep_config_t *cfg_out,
                                         onesweep_stream_t stream);

/* Sort with a learned configuration: onesweep_sort_keys (d_vals_in and
 * d_vals_out NULL) or onesweep_sort_pairs, with the binning tile shape and
 * ranking method picked by the model for these keys. For 2^26 <= n <= 2^28
 * the model's selection kernel (features and forward pass, as in
 * onesweep_select_config) runs on a stream owned by the model, forked from
 * `stream` with an event, while the sort's clear, histogram and
 * exclusive-sum kernels run on `stream`; the host then waits for the
 * selection only (an event, not the stream) and enqueues the binning passes
 * with the chosen shape, so the selection overlaps the first phases. The
 * autotuned default (the class holding the default tile shape) stays the
 * choice unless another class is predicted faster by more than about 2%.
 * Outside that size range, with a NULL model, or with cfg->algorithm set to
 * reduce-then-scan, the call is the plain sort with the default table and no
 * selection. The output is the same whatever is chosen (the stable order is
 * unique). cfg: key_type, descending, strip_log2 and trace are used; the tile
 * fields are ignored. *cfg_used (may be NULL) receives the configuration
 * the passes ran with. Temp storage as in onesweep_sort_keys (size query
 * with d_temp == NULL covers every class). Synchronises on the selection
 * event, so not graph-capturable; calls on one model must not overlap. */
onesweep_status_t onesweep_sort_learned(const onesweep_model_t *model, void *d_temp,
                                        size_t *temp_bytes, const void *d_keys_in,
                                        void *d_keys_out, const uint32_t *d_vals_in,
                                        uint32_t *d_vals_out, size_t n, int key_bits,
                                        int begin_bit, int end_bit, const onesweep_config_t *cfg,
                                        onesweep_config_t *cfg_used, onesweep_stream_t stream);

/* Binning tile size T = block_threads x items_per_thread that `cfg` resolves
 * to for this key width, value presence and n; 0 if the config is
 * unsupported. Pure host computation. */
size_t onesweep_tile_items(int key_bits, int has_values, size_t n, const onesweep_config_t *cfg);

/* Message describing the calling thread's last failure ("" if none). */
const char *onesweep_last_error(void);

/* Library version string. */
const char *onesweep_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ONESWEEP_H */
