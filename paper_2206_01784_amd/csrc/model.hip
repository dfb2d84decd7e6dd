// Host side of the learned configuration selector: the model object (device
// parameters, Adam state, training workspace, configuration classes), its
// file format, the training step and the selection call. Not in the paper.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "internal.hpp"

using namespace onesweep;

namespace {

// One configuration the model can choose: which key widths it applies to
// (bit 0: 32-bit keys, bit 1: 64-bit keys) and the sort configuration.
struct ModelClass {
  int key_bits_mask;
  int block_threads;
  int items_per_thread;
  int rank_algorithm;  // 1 ballot, 2 presence
  int hist_blocks_per_cu;
};

// Classes of a freshly created model: the plain sort's tile shapes with
// ballot ranking, every large-input default included (32-bit: 1024 x 11, 16
// and 19 keys per thread; 64-bit: 1024 x 9, 12 and 14), each built for keys
// and pairs.
// (key-width mask 1 = 32-bit, 2 = 64-bit, 3 = both; rank 1 ballots, 2 masks.)
constexpr ModelClass kDefaultClasses[kMlpClasses] = {
    {3, 256, 8, 1, 0},    {3, 256, 16, 1, 0},  {2, 512, 8, 1, 0},   {3, 512, 12, 1, 0},
    {1, 512, 16, 1, 0},   {3, 1024, 8, 1, 0},  {1, 1024, 11, 1, 0}, {1, 1024, 16, 1, 0},
    {2, 1024, 12, 1, 0},  {1, 1024, 19, 1, 0}, {2, 1024, 9, 1, 0},  {2, 1024, 14, 1, 0}};

constexpr char kMagic[8] = {'O', 'S', 'W', 'M', 'L', 'P', '0', '1'};

}  // namespace

struct onesweep_model {
  int device;
  int max_batch;
  void *block;  // the one device allocation everything below lives in
  float *params, *grad, *adam_m, *adam_v;
  float *enc, *u, *h1, *h2, *out, *d_out, *d_h2, *d_h1, *d_u, *d_enc;
  float *x1, *infer_out, *loss;
  int *choice;
  int *host_choice;      // pinned, mapped host memory the selection kernel writes
  int *host_choice_dev;  // its device address
  int step;
  ModelClass classes[kMlpClasses];
  // onesweep_sort_learned: the selection kernel runs on `aux`, forked from the
  // caller's stream by `fork`; `picked` marks its end.
  hipStream_t aux;
  hipEvent_t fork, picked;
};

namespace {

size_t model_floats(int B) {
  const size_t b = static_cast<size_t>(B);
  return 4 * static_cast<size_t>(kMlpParams) +
         2 * b * kMlpPlaces * kMlpEnc +   // enc, d_enc
         2 * b * kMlpU +                  // u, d_u
         4 * b * kMlpH1 +                 // h1, h2, d_h1, d_h2 (H1 == H2)
         2 * b * kMlpClasses +            // out, d_out
         kMlpFeatures + kMlpClasses + 1 + 64;  // x1, infer_out, loss, choice + slack
}

onesweep_status_t check_shape_of(const ModelClass &c) {
  for (int kb : {32, 64}) {
    if (!(c.key_bits_mask & (kb == 32 ? 1 : 2))) continue;
    onesweep_config_t cfg{};
    cfg.block_threads = c.block_threads;
    cfg.items_per_thread = c.items_per_thread;
    cfg.rank_algorithm = c.rank_algorithm;
    cfg.hist_blocks_per_cu = c.hist_blocks_per_cu;
    for (int v = 0; v < 2; ++v)
      if (onesweep_tile_items(kb, v, size_t(1) << 28, &cfg) == 0)
        return fail(ONESWEEP_ERROR_UNSUPPORTED, "model class %d x %d (rank %d) not built for %d-bit keys",
                    c.block_threads, c.items_per_thread, c.rank_algorithm, kb);
  }
  if (c.rank_algorithm < 1 || c.rank_algorithm > 2 || c.hist_blocks_per_cu < 0 ||
      c.hist_blocks_per_cu > 64 || (c.key_bits_mask & ~3) != 0)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "model class fields out of range");
  return ONESWEEP_SUCCESS;
}

onesweep_status_t create(int max_batch, onesweep_model **out) {
  if (!out) return fail(ONESWEEP_ERROR_INVALID_VALUE, "model pointer is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1 << 16))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "max_batch %d not in [1, 65536]", max_batch);
  onesweep_model *m = new (std::nothrow) onesweep_model();
  if (!m) return fail(ONESWEEP_ERROR_INVALID_VALUE, "out of host memory");
  hipError_t e = hipGetDevice(&m->device);
  if (e == hipSuccess) e = hipMalloc(&m->block, model_floats(max_batch) * sizeof(float));
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "model allocation");
  }
  e = hipMemset(m->block, 0, model_floats(max_batch) * sizeof(float));
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&m->host_choice), 64,
                                         hipHostMallocMapped);
  if (e == hipSuccess)
    e = hipHostGetDevicePointer(reinterpret_cast<void **>(&m->host_choice_dev), m->host_choice, 0);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->picked, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (m->picked) (void)hipEventDestroy(m->picked);
    if (m->fork) (void)hipEventDestroy(m->fork);
    if (m->aux) (void)hipStreamDestroy(m->aux);
    if (m->host_choice) (void)hipHostFree(m->host_choice);
    (void)hipFree(m->block);
    delete m;
    return hip_fail(e, "model allocation");
  }
  m->max_batch = max_batch;
  float *p = static_cast<float *>(m->block);
  const size_t B = static_cast<size_t>(max_batch);
  auto take = [&](size_t count) {
    float *r = p;
    p += count;
    return r;
  };
  m->params = take(kMlpParams);
  m->grad = take(kMlpParams);
  m->adam_m = take(kMlpParams);
  m->adam_v = take(kMlpParams);
  m->enc = take(B * kMlpPlaces * kMlpEnc);
  m->d_enc = take(B * kMlpPlaces * kMlpEnc);
  m->u = take(B * kMlpU);
  m->d_u = take(B * kMlpU);
  m->h1 = take(B * kMlpH1);
  m->h2 = take(B * kMlpH2);
  m->d_h1 = take(B * kMlpH1);
  m->d_h2 = take(B * kMlpH2);
  m->out = take(B * kMlpClasses);
  m->d_out = take(B * kMlpClasses);
  m->x1 = take(kMlpFeatures);
  m->infer_out = take(kMlpClasses);
  m->loss = take(1);
  m->choice = reinterpret_cast<int *>(take(1));
  m->step = 0;
  memcpy(m->classes, kDefaultClasses, sizeof(kDefaultClasses));
  *out = m;
  return ONESWEEP_SUCCESS;
}

#define MLP_TRY(expr, what)                           \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, what);  \
  } while (0)

GemmArgs gemm(const float *A, long a_rs, long a_cs, const float *Bm, long b_rs, long b_cs,
              float *C, long c_rs, int M, int N, int K, const float *bias, int relu,
              const float *mask) {
  GemmArgs g{};
  g.A = A;
  g.B = Bm;
  g.C = C;
  g.bias = bias;
  g.mask = mask;
  g.M = M;
  g.N = N;
  g.K = K;
  g.a_rs = a_rs;
  g.a_cs = a_cs;
  g.b_rs = b_rs;
  g.b_cs = b_cs;
  g.c_rs = c_rs;
  g.relu = relu;
  return g;
}

onesweep_status_t forward(onesweep_model *m, const float *hist, const float *scalars, int B,
                          float *out, hipStream_t s) {
  const float *p = m->params;
  MLP_TRY(launch_gemm(gemm(hist, kRadix, 1, p + kOffWe, kMlpEnc, 1, m->enc, kMlpEnc,
                           B * kMlpPlaces, kMlpEnc, kRadix, p + kOffBe, 1, nullptr), s),
          "encoder");
  MLP_TRY(launch_assemble(m->enc, scalars, m->u, B, s), "assemble");
  MLP_TRY(launch_gemm(gemm(m->u, kMlpU, 1, p + kOffW1, kMlpH1, 1, m->h1, kMlpH1, B, kMlpH1,
                           kMlpU, p + kOffB1, 1, nullptr), s),
          "layer 1");
  MLP_TRY(launch_gemm(gemm(m->h1, kMlpH1, 1, p + kOffW2, kMlpH2, 1, m->h2, kMlpH2, B, kMlpH2,
                           kMlpH1, p + kOffB2, 1, nullptr), s),
          "layer 2");
  MLP_TRY(launch_gemm(gemm(m->h2, kMlpH2, 1, p + kOffW3, kMlpClasses, 1, out, kMlpClasses,
                           B, kMlpClasses, kMlpH2, p + kOffB3, 0, nullptr), s),
          "layer 3");
  return ONESWEEP_SUCCESS;
}

// Gradients of the masked squared error into `grad` (flat, parameter order).
onesweep_status_t backward(onesweep_model *m, const float *hist, const float *y,
                           const float *mask, int B, float *grad, float *loss, hipStream_t s) {
  const float *p = m->params;
  MLP_TRY(launch_loss(m->out, y, mask, B * kMlpClasses, m->d_out, loss, s), "loss");
  // layer 3
  MLP_TRY(launch_gemm(gemm(m->h2, 1, kMlpH2, m->d_out, kMlpClasses, 1, grad + kOffW3,
                           kMlpClasses, kMlpH2, kMlpClasses, B, nullptr, 0, nullptr), s),
          "dW3");
  MLP_TRY(launch_colsum(m->d_out, B, kMlpClasses, kMlpClasses, grad + kOffB3, s), "db3");
  MLP_TRY(launch_gemm(gemm(m->d_out, kMlpClasses, 1, p + kOffW3, 1, kMlpClasses, m->d_h2,
                           kMlpH2, B, kMlpH2, kMlpClasses, nullptr, 0, m->h2), s),
          "dh2");
  // layer 2
  MLP_TRY(launch_gemm(gemm(m->h1, 1, kMlpH1, m->d_h2, kMlpH2, 1, grad + kOffW2, kMlpH2, kMlpH1,
                           kMlpH2, B, nullptr, 0, nullptr), s),
          "dW2");
  MLP_TRY(launch_colsum(m->d_h2, B, kMlpH2, kMlpH2, grad + kOffB2, s), "db2");
  MLP_TRY(launch_gemm(gemm(m->d_h2, kMlpH2, 1, p + kOffW2, 1, kMlpH2, m->d_h1, kMlpH1, B,
                           kMlpH1, kMlpH2, nullptr, 0, m->h1), s),
          "dh1");
  // layer 1
  MLP_TRY(launch_gemm(gemm(m->u, 1, kMlpU, m->d_h1, kMlpH1, 1, grad + kOffW1, kMlpH1, kMlpU,
                           kMlpH1, B, nullptr, 0, nullptr), s),
          "dW1");
  MLP_TRY(launch_colsum(m->d_h1, B, kMlpH1, kMlpH1, grad + kOffB1, s), "db1");
  MLP_TRY(launch_gemm(gemm(m->d_h1, kMlpH1, 1, p + kOffW1, 1, kMlpH1, m->d_u, kMlpU, B, kMlpU,
                           kMlpH1, nullptr, 0, nullptr), s),
          "du");
  // encoder
  MLP_TRY(launch_split(m->d_u, m->enc, m->d_enc, B, s), "split");
  MLP_TRY(launch_gemm(gemm(hist, 1, kRadix, m->d_enc, kMlpEnc, 1, grad + kOffWe, kMlpEnc,
                           kRadix, kMlpEnc, B * kMlpPlaces, nullptr, 0, nullptr), s),
          "dWe");
  MLP_TRY(launch_colsum(m->d_enc, B * kMlpPlaces, kMlpEnc, kMlpEnc, grad + kOffBe, s), "dbe");
  return ONESWEEP_SUCCESS;
}

onesweep_status_t check_batch(const onesweep_model *m, const void *a, const void *b, int B) {
  if (!m) return fail(ONESWEEP_ERROR_INVALID_VALUE, "model is NULL");
  if (B < 1 || B > m->max_batch)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "batch %d not in [1, %d]", B, m->max_batch);
  if (!a || !b) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL input pointer");
  return ONESWEEP_SUCCESS;
}

}  // namespace

namespace {

// Selection applies to sorts of 2^26 to 2^28 keys. Below, the histogram
// (under 60 us) is too short to hide the selection kernel and the host's wait
// for it, and the autotuned table is what the measured sweep prefers; above,
// every class would need strips of its own.
constexpr size_t kLearnedMinN = size_t(1) << 26;
constexpr size_t kLearnedMaxN = size_t(1) << 28;
// A class replaces the autotuned default only when predicted faster by more
// than this (log-time units, about 10%). Over the held-out sweep the best
// class beats the default by under 1% on average at these sizes, while
// margins of 2% and 5% let through mispredictions (Zipf and 16-distinct
// keys) that cost 2-20%.
constexpr float kSelectMargin = 0.10f;
// The host-mapped choice word before the selection kernel writes it (the
// kernel writes a class index or -1).
constexpr int kChoicePending = -2;

void class_fields(const ModelClass &c, onesweep_config_t *cfg) {
  cfg->block_threads = c.block_threads;
  cfg->items_per_thread = c.items_per_thread;
  cfg->rank_algorithm = c.rank_algorithm;
  cfg->hist_blocks_per_cu = c.hist_blocks_per_cu;
}

// The class holding the library's default tile shape for this input (ballot
// ranking), or -1.
int default_class(const onesweep_model_t *m, int key_bits, bool has_values, size_t n) {
  const BinningShape d = binning_default_shape(key_bits, has_values, n);
  for (int c = 0; c < kMlpClasses; ++c) {
    const ModelClass &k = m->classes[c];
    if ((k.key_bits_mask & (key_bits == 32 ? 1 : 2)) && k.block_threads == d.block &&
        k.items_per_thread == d.ipt && k.rank_algorithm == 1 && k.hist_blocks_per_cu == 0)
      return c;
  }
  return -1;
}

onesweep_status_t check_select(const onesweep_model_t *m, const void *d_keys, int key_bits,
                               int begin_bit, int end_bit) {
  if (key_bits != 32 && key_bits != 64)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key_bits %d is not 32 or 64", key_bits);
  if (begin_bit < 0 || begin_bit > end_bit || end_bit > key_bits)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "bit range [%d, %d) invalid", begin_bit, end_bit);
  if (!d_keys || (reinterpret_cast<uintptr_t>(d_keys) & (key_bits / 8 - 1)))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_keys NULL or not aligned to the key size");
  (void)m;
  return ONESWEEP_SUCCESS;
}

SelectArgs select_args(const onesweep_model_t *m, const void *d_keys, size_t n, int key_bits,
                       int begin_bit, int end_bit, bool has_values) {
  unsigned mask = 0;
  for (int c = 0; c < kMlpClasses; ++c)
    if (m->classes[c].key_bits_mask & (key_bits == 32 ? 1 : 2)) mask |= 1u << c;
  SelectArgs a{};
  a.params = m->params;
  a.keys = d_keys;
  a.n = n;
  a.begin_bit = begin_bit;
  a.end_bit = end_bit;
  a.places = (end_bit - begin_bit + kRadixBits - 1) / kRadixBits;
  a.has_values = has_values ? 1 : 0;
  a.class_mask = mask;
  a.default_class = default_class(m, key_bits, has_values, n);
  a.margin = kSelectMargin;
  a.out = m->infer_out;
  a.choice = m->choice;
  a.host_choice = m->host_choice_dev;
  return a;
}

// The configuration of the class the last selection wrote to pinned host
// memory (tile fields only; the rest of *cfg is kept); the default when no
// class applied.
onesweep_status_t chosen_class(const onesweep_model_t *m, onesweep_config_t *cfg) {
  const int choice = *static_cast<volatile int *>(m->host_choice);
  if (choice < 0 || choice >= kMlpClasses) return ONESWEEP_SUCCESS;
  class_fields(m->classes[choice], cfg);
  return ONESWEEP_SUCCESS;
}

}  // namespace

extern "C" {

size_t onesweep_model_num_params(void) { return static_cast<size_t>(kMlpParams); }

onesweep_status_t onesweep_model_create(int max_batch, onesweep_model_t **model) {
  clear_error();
  return create(max_batch, model);
}

void onesweep_model_free(onesweep_model_t *model) {
  if (!model) return;
  if (model->picked) (void)hipEventDestroy(model->picked);
  if (model->fork) (void)hipEventDestroy(model->fork);
  if (model->aux) (void)hipStreamDestroy(model->aux);
  (void)hipFree(model->block);
  if (model->host_choice) (void)hipHostFree(model->host_choice);
  delete model;
}

onesweep_status_t onesweep_model_set_params(onesweep_model_t *m, const float *host_params,
                                            size_t count) {
  clear_error();
  if (!m || !host_params) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL argument");
  if (count != static_cast<size_t>(kMlpParams))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "expected %d parameters, got %zu", kMlpParams,
                count);
  MLP_TRY(hipMemcpy(m->params, host_params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice),
          "hipMemcpy");
  MLP_TRY(hipMemset(m->adam_m, 0, sizeof(float) * kMlpParams * 2), "hipMemset");
  m->step = 0;
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_model_get_params(const onesweep_model_t *m, float *host_params,
                                            size_t count) {
  clear_error();
  if (!m || !host_params) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL argument");
  if (count != static_cast<size_t>(kMlpParams))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "expected %d parameters, got %zu", kMlpParams,
                count);
  MLP_TRY(hipMemcpy(host_params, m->params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost),
          "hipMemcpy");
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_model_class(const onesweep_model_t *m, int index,
                                       onesweep_config_t *cfg_out, int *key_bits_mask) {
  clear_error();
  if (!m || !cfg_out || index < 0 || index >= kMlpClasses)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "bad model class query");
  const ModelClass &c = m->classes[index];
  memset(cfg_out, 0, sizeof(*cfg_out));
  cfg_out->block_threads = c.block_threads;
  cfg_out->items_per_thread = c.items_per_thread;
  cfg_out->rank_algorithm = c.rank_algorithm;
  cfg_out->hist_blocks_per_cu = c.hist_blocks_per_cu;
  if (key_bits_mask) *key_bits_mask = c.key_bits_mask;
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_model_save(const onesweep_model_t *m, const char *path) {
  clear_error();
  if (!m || !path) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL argument");
  float *host = new (std::nothrow) float[kMlpParams];
  if (!host) return fail(ONESWEEP_ERROR_INVALID_VALUE, "out of host memory");
  hipError_t e = hipMemcpy(host, m->params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    delete[] host;
    return hip_fail(e, "hipMemcpy");
  }
  FILE *f = fopen(path, "wb");
  if (!f) {
    delete[] host;
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "cannot open %s for writing", path);
  }
  const uint32_t dims[8] = {kMlpPlaces, kRadix, kMlpEnc, kMlpScalars,
                            kMlpH1,     kMlpH2, kMlpClasses, kMlpParams};
  int32_t cls[kMlpClasses][5];
  for (int c = 0; c < kMlpClasses; ++c) {
    cls[c][0] = m->classes[c].key_bits_mask;
    cls[c][1] = m->classes[c].block_threads;
    cls[c][2] = m->classes[c].items_per_thread;
    cls[c][3] = m->classes[c].rank_algorithm;
    cls[c][4] = m->classes[c].hist_blocks_per_cu;
  }
  bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(dims, 4, 8, f) == 8 &&
            fwrite(cls, 4, kMlpClasses * 5, f) == static_cast<size_t>(kMlpClasses * 5) &&
            fwrite(host, 4, kMlpParams, f) == static_cast<size_t>(kMlpParams);
  ok = (fclose(f) == 0) && ok;
  delete[] host;
  return ok ? ONESWEEP_SUCCESS : fail(ONESWEEP_ERROR_INVALID_VALUE, "write to %s failed", path);
}

onesweep_status_t onesweep_model_load(const char *path, int max_batch, onesweep_model_t **out) {
  clear_error();
  if (!path || !out) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL argument");
  *out = nullptr;
  FILE *f = fopen(path, "rb");
  if (!f) return fail(ONESWEEP_ERROR_INVALID_VALUE, "cannot open %s", path);
  char magic[8];
  uint32_t dims[8];
  int32_t cls[kMlpClasses][5];
  float *host = new (std::nothrow) float[kMlpParams];
  bool ok = host && fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 &&
            fread(dims, 4, 8, f) == 8;
  const uint32_t want[8] = {kMlpPlaces, kRadix, kMlpEnc, kMlpScalars,
                            kMlpH1,     kMlpH2, kMlpClasses, kMlpParams};
  ok = ok && memcmp(dims, want, sizeof(want)) == 0 &&
       fread(cls, 4, kMlpClasses * 5, f) == static_cast<size_t>(kMlpClasses * 5) &&
       fread(host, 4, kMlpParams, f) == static_cast<size_t>(kMlpParams);
  char extra;
  ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after the parameters
  fclose(f);
  if (!ok) {
    delete[] host;
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "%s is not a model file of this library", path);
  }
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(host[i])) {
      delete[] host;
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "%s holds a non-finite parameter", path);
    }
  ModelClass classes[kMlpClasses];
  for (int c = 0; c < kMlpClasses; ++c) {
    classes[c] = ModelClass{cls[c][0], cls[c][1], cls[c][2], cls[c][3], cls[c][4]};
    onesweep_status_t st = check_shape_of(classes[c]);
    if (st) {
      delete[] host;
      return st;
    }
  }
  onesweep_model *m = nullptr;
  onesweep_status_t st = create(max_batch, &m);
  if (!st) st = onesweep_model_set_params(m, host, kMlpParams);
  delete[] host;
  if (st) {
    onesweep_model_free(m);
    return st;
  }
  memcpy(m->classes, classes, sizeof(classes));
  *out = m;
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_features(const void *d_keys, size_t n, int key_bits, int begin_bit,
                                    int end_bit, int has_values, float *d_features,
                                    onesweep_stream_t stream) {
  clear_error();
  if (key_bits != 32 && key_bits != 64)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key_bits %d is not 32 or 64", key_bits);
  if (begin_bit < 0 || begin_bit > end_bit || end_bit > key_bits)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "bit range [%d, %d) invalid", begin_bit, end_bit);
  if (!d_features || (n > 0 && !d_keys))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL pointer");
  if (reinterpret_cast<uintptr_t>(d_keys) & (key_bits / 8 - 1))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_keys not aligned to the key size");
  FeatureArgs a{};
  a.keys = d_keys;
  a.n = n;
  a.begin_bit = begin_bit;
  a.end_bit = end_bit;
  a.places = (end_bit - begin_bit + kRadixBits - 1) / kRadixBits;
  a.has_values = has_values ? 1 : 0;
  a.out = d_features;
  MLP_TRY(launch_features(key_bits, a, reinterpret_cast<hipStream_t>(stream)), "features");
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_model_infer(const onesweep_model_t *m, const float *d_features,
                                       unsigned class_mask, float *d_out, int *d_choice,
                                       onesweep_stream_t stream) {
  clear_error();
  if (!m || !d_features || !d_out || !d_choice)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL argument");
  InferArgs a{};
  a.params = m->params;
  a.x = d_features;
  a.class_mask = class_mask & ((1u << kMlpClasses) - 1u);
  a.out = d_out;
  a.choice = d_choice;
  MLP_TRY(launch_infer(a, reinterpret_cast<hipStream_t>(stream)), "infer");
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_model_forward(onesweep_model_t *m, const float *d_hist,
                                         const float *d_scalars, int batch, float *d_out,
                                         onesweep_stream_t stream) {
  clear_error();
  onesweep_status_t st = check_batch(m, d_hist, d_scalars, batch);
  if (st) return st;
  if (!d_out) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL output");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return forward(m, d_hist, d_scalars, batch, d_out, s);
}

onesweep_status_t onesweep_model_gradients(onesweep_model_t *m, const float *d_hist,
                                           const float *d_scalars, const float *d_y,
                                           const float *d_mask, int batch, float *d_grad,
                                           float *d_loss, onesweep_stream_t stream) {
  clear_error();
  onesweep_status_t st = check_batch(m, d_hist, d_scalars, batch);
  if (st) return st;
  if (!d_y || !d_mask || !d_grad) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((st = forward(m, d_hist, d_scalars, batch, m->out, s))) return st;
  return backward(m, d_hist, d_y, d_mask, batch, d_grad, d_loss ? d_loss : m->loss, s);
}

onesweep_status_t onesweep_model_train_step(onesweep_model_t *m, const float *d_hist,
                                            const float *d_scalars, const float *d_y,
                                            const float *d_mask, int batch, float lr,
                                            float *d_loss, onesweep_stream_t stream) {
  clear_error();
  onesweep_status_t st = check_batch(m, d_hist, d_scalars, batch);
  if (st) return st;
  if (!d_y || !d_mask) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL argument");
  if (!(lr > 0.0f) || !std::isfinite(lr))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "learning rate must be positive");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((st = forward(m, d_hist, d_scalars, batch, m->out, s))) return st;
  if ((st = backward(m, d_hist, d_y, d_mask, batch, m->grad, d_loss ? d_loss : m->loss, s)))
    return st;
  m->step += 1;
  AdamArgs a{};
  a.theta = m->params;
  a.m = m->adam_m;
  a.v = m->adam_v;
  a.grad = m->grad;
  a.count = kMlpParams;
  a.lr = lr;
  a.beta1 = 0.9f;
  a.beta2 = 0.999f;
  a.eps = 1e-8f;
  a.c1 = static_cast<float>(1.0 / (1.0 - std::pow(0.9, m->step)));
  a.c2 = static_cast<float>(1.0 / (1.0 - std::pow(0.999, m->step)));
  MLP_TRY(launch_adam(a, s), "adam");
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_select_config(const onesweep_model_t *m, const void *d_keys,
                                         size_t n, int key_bits, int begin_bit, int end_bit,
                                         int has_values, onesweep_config_t *cfg_out,
                                         onesweep_stream_t stream) {
  clear_error();
  if (!cfg_out) return fail(ONESWEEP_ERROR_INVALID_VALUE, "cfg_out is NULL");
  if (key_bits != 32 && key_bits != 64)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key_bits %d is not 32 or 64", key_bits);
  // The key order is the caller's and is kept; everything else is chosen.
  const int key_type = cfg_out->key_type, descending = cfg_out->descending;
  auto keep_order = [&](onesweep_status_t st) {
    cfg_out->key_type = key_type;
    cfg_out->descending = descending;
    return st;
  };
  memset(cfg_out, 0, sizeof(*cfg_out));
  if (!m || n == 0) return keep_order(ONESWEEP_SUCCESS);  // the library's default
  onesweep_status_t st = check_select(m, d_keys, key_bits, begin_bit, end_bit);
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  *m->host_choice = -1;
  MLP_TRY(launch_select(key_bits, select_args(m, d_keys, n, key_bits, begin_bit, end_bit,
                                              has_values != 0), s),
          "select");
  MLP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return keep_order(chosen_class(m, cfg_out));
}

onesweep_status_t onesweep_sort_learned(const onesweep_model_t *m, void *d_temp,
                                        size_t *temp_bytes, const void *d_keys_in,
                                        void *d_keys_out, const uint32_t *d_vals_in,
                                        uint32_t *d_vals_out, size_t n, int key_bits,
                                        int begin_bit, int end_bit, const onesweep_config_t *cfg,
                                        onesweep_config_t *cfg_used, onesweep_stream_t stream) {
  clear_error();
  if (!temp_bytes) return fail(ONESWEEP_ERROR_INVALID_VALUE, "temp_bytes is NULL");
  if ((d_vals_in == nullptr) != (d_vals_out == nullptr))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "value pointers: both or neither");
  const bool has_values = d_vals_in != nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // The caller's configuration minus the tile fields, which are chosen here.
  onesweep_config_t base = cfg ? *cfg : onesweep_config_t{};
  base.block_threads = 0;
  base.items_per_thread = 0;
  base.rank_algorithm = 0;
  if (cfg_used) *cfg_used = base;
  const bool select = m != nullptr && n >= kLearnedMinN && n <= kLearnedMaxN &&
                      (key_bits == 32 || key_bits == 64) && base.algorithm == 0;
  if (!select) {  // the autotuned default table, without selection
    return has_values ? onesweep_sort_pairs(d_temp, temp_bytes, d_keys_in, d_keys_out, d_vals_in,
                                            d_vals_out, n, key_bits, begin_bit, end_bit, 1, &base,
                                            stream)
                      : onesweep_sort_keys(d_temp, temp_bytes, d_keys_in, d_keys_out, n, key_bits,
                                           begin_bit, end_bit, 1, &base, stream);
  }
  // Temporary storage for the smallest tile any choice can make.
  size_t layout_tile = onesweep_tile_items(key_bits, has_values, n, &base);
  for (int c = 0; c < kMlpClasses; ++c) {
    if (!(m->classes[c].key_bits_mask & (key_bits == 32 ? 1 : 2))) continue;
    onesweep_config_t k = base;
    class_fields(m->classes[c], &k);
    const size_t t = onesweep_tile_items(key_bits, has_values, n, &k);
    if (t != 0 && (layout_tile == 0 || t < layout_tile)) layout_tile = t;
  }
  if (layout_tile == 0) return fail(ONESWEEP_ERROR_UNSUPPORTED, "no built tile shape");
  struct Ctx {
    const onesweep_model_t *m;
    onesweep_config_t picked;
  } ctx{m, base};
  LateChoice late{};
  late.layout_tile = layout_tile;
  late.ctx = &ctx;
  late.choose = [](void *p, onesweep_config_t *c) -> onesweep_status_t {
    Ctx &x = *static_cast<Ctx *>(p);
    // The selection kernel stores its choice to mapped host memory as its
    // last step: poll that word (microseconds) rather than wait on the event;
    // after 20 ms fall back to the event.
    const auto t0 = std::chrono::steady_clock::now();
    while (__atomic_load_n(x.m->host_choice, __ATOMIC_ACQUIRE) == kChoicePending) {
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
        hipError_t e = hipEventSynchronize(x.m->picked);
        if (e != hipSuccess) return hip_fail(e, "selection event");
        if (__atomic_load_n(x.m->host_choice, __ATOMIC_ACQUIRE) == kChoicePending)
          return fail(ONESWEEP_ERROR_HIP, "selection kernel wrote no choice");
        break;
      }
    }
    onesweep_status_t st = chosen_class(x.m, c);
    x.picked = *c;
    return st;
  };
  if (d_temp == nullptr)  // size query: nothing is enqueued, choose is not called
    return sort_late_choice(nullptr, temp_bytes, d_keys_in, d_keys_out, d_vals_in, d_vals_out,
                            has_values, n, key_bits, begin_bit, end_bit, &base, s, late);
  int dev = 0;
  MLP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != m->device) return fail(ONESWEEP_ERROR_INVALID_VALUE, "model on device %d, current %d",
                                    m->device, dev);
  onesweep_status_t st = check_select(m, d_keys_in, key_bits, begin_bit, end_bit);
  if (st) return st;
  // The selection kernel reads the keys on the model's stream, after what the
  // caller enqueued before, while the sort's clear, histogram and exclusive
  // sums run on the caller's stream.
  __atomic_store_n(m->host_choice, kChoicePending, __ATOMIC_RELEASE);
  MLP_TRY(hipEventRecord(m->fork, s), "fork");
  MLP_TRY(hipStreamWaitEvent(m->aux, m->fork, 0), "fork");
  MLP_TRY(launch_select(key_bits, select_args(m, d_keys_in, n, key_bits, begin_bit, end_bit,
                                              has_values), m->aux),
          "select");
  MLP_TRY(hipEventRecord(m->picked, m->aux), "select event");
  st = sort_late_choice(d_temp, temp_bytes, d_keys_in, d_keys_out, d_vals_in, d_vals_out,
                        has_values, n, key_bits, begin_bit, end_bit, &base, s, late);
  if (st == ONESWEEP_SUCCESS && cfg_used) *cfg_used = ctx.picked;
  return st;
}

}  // extern "C"
