// Learned configuration selection (not in the paper, which tunes its
// kernels by hand, Table 2): sampled digit-histogram features of the input,
// a small MLP that predicts each configuration's time relative to the best,
// and the kernels that train it (forward, masked squared-error loss,
// backward, Adam). Whatever configuration is chosen, the sort's output is
// the same: the choice only changes tile shape and ranking method.
//
// Network (float32): a place encoder shared by the 8 digit places
// (256 -> 16, ReLU); the 8 encodings and 3 scalars concatenated (131)
// -> 64 ReLU -> 64 ReLU -> 12 outputs. Parameters are one flat array:
// We[256][16], be[16], W1[131][64], b1[64], W2[64][64], b2[64], W3[64][12],
// b3[12] (row-major, input index first).
//
// The MLP is tiny (17.5 K parameters): a training step is a chain of small
// launches bound by launch latency, and one selection is a single
// workgroup reading 70 KB of weights from L2, so plain FMA loops over LDS
// tiles are used rather than matrix cores.
#include "device_common.hpp"
#include "internal.hpp"

namespace onesweep {

// ---------------------------------------------------------------- features
// One workgroup samples min(n, 4096) keys at indices floor(i * n / m),
// counts each place's digits in LDS and writes the fractions, then
// log2(n) / 32, key_bits / 64 and has_values.
template <typename K>
__global__ void __launch_bounds__(1024) features_kernel(FeatureArgs a) {
  __shared__ uint32_t s_hist[kMlpPlaces * kRadix];
  const K *keys = static_cast<const K *>(a.keys);
  const int tid = threadIdx.x;
  for (int i = tid; i < kMlpPlaces * kRadix; i += 1024) s_hist[i] = 0u;
  __syncthreads();
  const uint64_t n = a.n;
  const uint32_t m = n < kMlpSamples ? static_cast<uint32_t>(n) : kMlpSamples;
  for (uint32_t i = tid; i < m; i += 1024) {
    const K k = keys[static_cast<uint64_t>(i) * n / m];
    for (int j = 0; j < a.places; ++j) {
      const int lo = a.begin_bit + j * kRadixBits;
      const int width = min(kRadixBits, a.end_bit - lo);
      atomicAdd(&s_hist[j * kRadix + (static_cast<uint32_t>(k >> lo) & ((1u << width) - 1u))],
                1u);
    }
  }
  __syncthreads();
  for (int i = tid; i < kMlpPlaces * kRadix; i += 1024)
    a.out[i] = m ? __fdiv_rn(static_cast<float>(s_hist[i]), static_cast<float>(m)) : 0.0f;
  if (tid == 0) {
    a.out[kMlpPlaces * kRadix + 0] = n ? log2f(static_cast<float>(n)) / 32.0f : 0.0f;
    a.out[kMlpPlaces * kRadix + 1] = static_cast<float>(sizeof(K) * 8) / 64.0f;
    a.out[kMlpPlaces * kRadix + 2] = a.has_values ? 1.0f : 0.0f;
  }
}

hipError_t launch_features(int key_bits, const FeatureArgs &a, hipStream_t stream) {
  if (key_bits == 32)
    hipLaunchKernelGGL(features_kernel<uint32_t>, dim3(1), dim3(1024), 0, stream, a);
  else
    hipLaunchKernelGGL(features_kernel<uint64_t>, dim3(1), dim3(1024), 0, stream, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- inference
// The whole forward pass for one feature vector in one workgroup, then the
// configuration with the smallest predicted relative time among those whose
// mask bit is set. Writes the 12 outputs and the chosen index.
__global__ void __launch_bounds__(256) infer_kernel(InferArgs a) {
  __shared__ float s_x[kMlpFeatures];
  __shared__ float s_part[2][kMlpPlaces * kMlpEnc];
  __shared__ float s_u[kMlpU];
  __shared__ float s_h1[kMlpH1];
  __shared__ float s_h2[kMlpH2];
  __shared__ float s_out[kMlpClasses];
  const int tid = threadIdx.x;
  const float *p = a.params;
  const float *We = p + kOffWe, *be = p + kOffBe, *W1 = p + kOffW1, *b1 = p + kOffB1;
  const float *W2 = p + kOffW2, *b2 = p + kOffB2, *W3 = p + kOffW3, *b3 = p + kOffB3;
  for (int i = tid; i < kMlpFeatures; i += 256) s_x[i] = a.x[i];
  __syncthreads();
  {
    // encoder: output o = (place j, unit k); two threads per output, one per
    // half of the bins
    const int o = tid & (kMlpPlaces * kMlpEnc - 1), half = tid / (kMlpPlaces * kMlpEnc);
    const int j = o / kMlpEnc, k = o % kMlpEnc;
    float acc = 0.0f;
    for (int v = half * (kRadix / 2); v < (half + 1) * (kRadix / 2); ++v)
      acc = fmaf(s_x[j * kRadix + v], We[v * kMlpEnc + k], acc);
    s_part[half][o] = acc;
  }
  __syncthreads();
  if (tid < kMlpPlaces * kMlpEnc)
    s_u[tid] = fmaxf(s_part[0][tid] + s_part[1][tid] + be[tid % kMlpEnc], 0.0f);
  else if (tid < kMlpU)
    s_u[tid] = s_x[kMlpPlaces * kRadix + tid - kMlpPlaces * kMlpEnc];
  __syncthreads();
  if (tid < kMlpH1) {
    float acc = b1[tid];
    for (int i = 0; i < kMlpU; ++i) acc = fmaf(s_u[i], W1[i * kMlpH1 + tid], acc);
    s_h1[tid] = fmaxf(acc, 0.0f);
  }
  __syncthreads();
  if (tid < kMlpH2) {
    float acc = b2[tid];
    for (int i = 0; i < kMlpH1; ++i) acc = fmaf(s_h1[i], W2[i * kMlpH2 + tid], acc);
    s_h2[tid] = fmaxf(acc, 0.0f);
  }
  __syncthreads();
  if (tid < kMlpClasses) {
    float acc = b3[tid];
    for (int i = 0; i < kMlpH2; ++i) acc = fmaf(s_h2[i], W3[i * kMlpClasses + tid], acc);
    s_out[tid] = acc;
    a.out[tid] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    int best = -1;
    for (int c = 0; c < kMlpClasses; ++c)
      if (((a.class_mask >> c) & 1u) && (best < 0 || s_out[c] < s_out[best])) best = c;
    *a.choice = best;
  }
}

hipError_t launch_infer(const InferArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(infer_kernel, dim3(1), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- selection
// Features and the forward pass of one input fused into one workgroup of
// 1024 threads: the sampled digit counts and each layer's activations in
// LDS, the parameters read from global memory (70 KB, cached; the learned
// sort runs this kernel beside the histogram, whose LDS atomics would slow
// a copy of the parameters in LDS several times over). Dot products are
// split over groups of threads whose lanes read consecutive weights; partial
// sums meet in LDS. The result (outputs and the chosen class) equals
// infer_kernel's up to float32 summation order.
template <typename K>
__global__ void __launch_bounds__(1024) select_kernel(SelectArgs a) {
  constexpr int kThreads = 1024;
  constexpr int kEncOut = kMlpPlaces * kMlpEnc;  // 128
  __shared__ uint32_t s_hist[kMlpPlaces * kRadix];
  __shared__ float s_part[kThreads];
  __shared__ float s_u[kMlpU];
  __shared__ float s_h1[kMlpH1];
  __shared__ float s_h2[kMlpH2];
  __shared__ float s_out[kMlpClasses];
  const int tid = threadIdx.x;
  const K *keys = static_cast<const K *>(a.keys);
  for (int i = tid; i < kMlpPlaces * kRadix; i += kThreads) s_hist[i] = 0u;
  const float *__restrict__ params = a.params;
  const uint64_t n = a.n;
  const uint32_t m = n < kMlpSamples ? static_cast<uint32_t>(n) : kMlpSamples;
  K k[kMlpSamples / kThreads];
#pragma unroll
  for (int r = 0; r < static_cast<int>(kMlpSamples / kThreads); ++r) {
    const uint32_t i = tid + r * kThreads;
    k[r] = i < m ? keys[static_cast<uint64_t>(i) * n / m] : K(0);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < static_cast<int>(kMlpSamples / kThreads); ++r) {
    if (static_cast<uint32_t>(tid + r * kThreads) >= m) continue;
    for (int j = 0; j < a.places; ++j) {
      const int lo = a.begin_bit + j * kRadixBits;
      const int width = min(kRadixBits, a.end_bit - lo);
      atomicAdd(&s_hist[j * kRadix + (static_cast<uint32_t>(k[r] >> lo) & ((1u << width) - 1u))],
                1u);
    }
  }
  __syncthreads();
  const float *We = params + kOffWe, *be = params + kOffBe, *W1 = params + kOffW1;
  const float *b1 = params + kOffB1, *W2 = params + kOffW2, *b2 = params + kOffB2;
  const float *W3 = params + kOffW3, *b3 = params + kOffB3;
  const float fm = static_cast<float>(m);
  {
    // encoder: output o = (place o / 16, unit o % 16), 8 parts of 32 bins
    const int o = tid % kEncOut, part = tid / kEncOut;
    const int j = o / kMlpEnc, u = o % kMlpEnc;
    float acc = 0.0f;
    for (int v = part * 32; v < part * 32 + 32; ++v) {
      const float x = m ? __fdiv_rn(static_cast<float>(s_hist[j * kRadix + v]), fm) : 0.0f;
      acc = fmaf(x, We[v * kMlpEnc + u], acc);
    }
    s_part[part * kEncOut + o] = acc;
  }
  __syncthreads();
  if (tid < kEncOut) {
    float acc = 0.0f;
    for (int part = 0; part < kThreads / kEncOut; ++part) acc += s_part[part * kEncOut + tid];
    s_u[tid] = fmaxf(acc + be[tid % kMlpEnc], 0.0f);
  } else if (tid == kEncOut) {
    s_u[kEncOut + 0] = n ? log2f(static_cast<float>(n)) / 32.0f : 0.0f;
    s_u[kEncOut + 1] = static_cast<float>(sizeof(K) * 8) / 64.0f;
    s_u[kEncOut + 2] = a.has_values ? 1.0f : 0.0f;
  }
  __syncthreads();
  {
    // layer 1: output o, 16 parts striding over the 131 inputs
    const int o = tid % kMlpH1, part = tid / kMlpH1;
    float acc = 0.0f;
    for (int i = part; i < kMlpU; i += kThreads / kMlpH1) acc = fmaf(s_u[i], W1[i * kMlpH1 + o], acc);
    s_part[part * kMlpH1 + o] = acc;
  }
  __syncthreads();
  if (tid < kMlpH1) {
    float acc = b1[tid];
    for (int part = 0; part < kThreads / kMlpH1; ++part) acc += s_part[part * kMlpH1 + tid];
    s_h1[tid] = fmaxf(acc, 0.0f);
  }
  __syncthreads();
  {
    const int o = tid % kMlpH2, part = tid / kMlpH2;
    float acc = 0.0f;
    for (int i = part; i < kMlpH1; i += kThreads / kMlpH2) acc = fmaf(s_h1[i], W2[i * kMlpH2 + o], acc);
    s_part[part * kMlpH2 + o] = acc;
  }
  __syncthreads();
  if (tid < kMlpH2) {
    float acc = b2[tid];
    for (int part = 0; part < kThreads / kMlpH2; ++part) acc += s_part[part * kMlpH2 + tid];
    s_h2[tid] = fmaxf(acc, 0.0f);
  }
  __syncthreads();
  if (tid < kMlpClasses * 16) {
    const int o = tid % kMlpClasses, part = tid / kMlpClasses;
    float acc = 0.0f;
    for (int i = part; i < kMlpH2; i += 16) acc = fmaf(s_h2[i], W3[i * kMlpClasses + o], acc);
    s_part[part * kMlpClasses + o] = acc;
  }
  __syncthreads();
  if (tid < kMlpClasses) {
    float acc = b3[tid];
    for (int part = 0; part < 16; ++part) acc += s_part[part * kMlpClasses + tid];
    s_out[tid] = acc;
    a.out[tid] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    int best = -1;
    for (int c = 0; c < kMlpClasses; ++c)
      if (((a.class_mask >> c) & 1u) && (best < 0 || s_out[c] < s_out[best])) best = c;
    const int d = a.default_class;
    if (d >= 0 && ((a.class_mask >> d) & 1u) && !(s_out[best] < s_out[d] - a.margin)) best = d;
    *a.choice = best;
    // The host may poll this word while the kernel is still running.
    if (a.host_choice)
      __hip_atomic_store(a.host_choice, best, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

hipError_t launch_select(int key_bits, const SelectArgs &a, hipStream_t stream) {
  if (key_bits == 32)
    hipLaunchKernelGGL(select_kernel<uint32_t>, dim3(1), dim3(1024), 0, stream, a);
  else
    hipLaunchKernelGGL(select_kernel<uint64_t>, dim3(1), dim3(1024), 0, stream, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- training
// C[i][j] = epilogue(sum_k A(i, k) B(k, j)) for i < M, j < N, with
// A(i, k) = A[i * a_rs + k * a_cs] and B(k, j) = B[k * b_rs + j * b_cs], so
// transposed operands are stride swaps. Epilogue: + bias[j], ReLU, and a
// mask that zeroes C[i][j] where mask[i * c_rs + j] <= 0 (the backward of a
// ReLU whose output is `mask`). 32 x 32 output tiles, 32-deep K slices in
// LDS, 2 x 2 outputs per thread.
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  constexpr int kT = 32;
  __shared__ float s_a[kT][kT + 1];
  __shared__ float s_b[kT][kT + 1];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int i0 = blockIdx.y * kT, j0 = blockIdx.x * kT;
  float acc[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
  for (int k0 = 0; k0 < g.K; k0 += kT) {
    for (int e = tid; e < kT * kT; e += 256) {
      const int r = e / kT, c = e % kT;
      const int i = i0 + r, k = k0 + c;
      s_a[r][c] = (i < g.M && k < g.K)
                      ? g.A[static_cast<size_t>(i) * g.a_rs + static_cast<size_t>(k) * g.a_cs]
                      : 0.0f;
      const int kk = k0 + r, j = j0 + c;
      s_b[r][c] = (kk < g.K && j < g.N)
                      ? g.B[static_cast<size_t>(kk) * g.b_rs + static_cast<size_t>(j) * g.b_cs]
                      : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < kT; ++k) {
      const float a0 = s_a[ty * 2][k], a1 = s_a[ty * 2 + 1][k];
      const float b0 = s_b[k][tx * 2], b1 = s_b[k][tx * 2 + 1];
      acc[0][0] = fmaf(a0, b0, acc[0][0]);
      acc[0][1] = fmaf(a0, b1, acc[0][1]);
      acc[1][0] = fmaf(a1, b0, acc[1][0]);
      acc[1][1] = fmaf(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int di = 0; di < 2; ++di)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj) {
      const int i = i0 + ty * 2 + di, j = j0 + tx * 2 + dj;
      if (i >= g.M || j >= g.N) continue;
      float v = acc[di][dj];
      if (g.bias) v += g.bias[j];
      if (g.relu) v = fmaxf(v, 0.0f);
      const size_t at = static_cast<size_t>(i) * g.c_rs + j;
      if (g.mask && !(g.mask[at] > 0.0f)) v = 0.0f;
      g.C[at] = v;
    }
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((g.N + 31) / 32, (g.M + 31) / 32);
  hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, stream, g);
  return hipGetLastError();
}

// db[j] = sum_i dz[i * rs + j]
__global__ void __launch_bounds__(256) colsum_kernel(const float *dz, int rows, int cols, int rs,
                                                     float *db) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  float acc = 0.0f;
  for (int i = 0; i < rows; ++i) acc += dz[static_cast<size_t>(i) * rs + j];
  db[j] = acc;
}

hipError_t launch_colsum(const float *dz, int rows, int cols, int rs, float *db,
                         hipStream_t stream) {
  hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256), dim3(256), 0, stream, dz, rows,
                     cols, rs, db);
  return hipGetLastError();
}

// u[b] = (enc[b * 8 + j][k] for j, k), scalars[b]   (forward)
// d_enc[b * 8 + j][k] = d_u[b][j * 16 + k] where enc > 0, else 0   (backward)
__global__ void __launch_bounds__(256) assemble_kernel(const float *enc, const float *scalars,
                                                       float *u, int batch) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= batch * kMlpU) return;
  const int b = e / kMlpU, c = e % kMlpU;
  u[e] = c < kMlpPlaces * kMlpEnc ? enc[b * kMlpPlaces * kMlpEnc + c]
                                  : scalars[b * kMlpScalars + (c - kMlpPlaces * kMlpEnc)];
}

__global__ void __launch_bounds__(256) split_kernel(const float *d_u, const float *enc,
                                                    float *d_enc, int batch) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= batch * kMlpPlaces * kMlpEnc) return;
  const int b = e / (kMlpPlaces * kMlpEnc), c = e % (kMlpPlaces * kMlpEnc);
  d_enc[e] = enc[e] > 0.0f ? d_u[b * kMlpU + c] : 0.0f;
}

hipError_t launch_assemble(const float *enc, const float *scalars, float *u, int batch,
                           hipStream_t stream) {
  hipLaunchKernelGGL(assemble_kernel, dim3((batch * kMlpU + 255) / 256), dim3(256), 0, stream,
                     enc, scalars, u, batch);
  return hipGetLastError();
}

hipError_t launch_split(const float *d_u, const float *enc, float *d_enc, int batch,
                        hipStream_t stream) {
  hipLaunchKernelGGL(split_kernel, dim3((batch * kMlpPlaces * kMlpEnc + 255) / 256), dim3(256),
                     0, stream, d_u, enc, d_enc, batch);
  return hipGetLastError();
}

// Masked mean squared error: loss = sum mask (out - y)^2 / max(1, sum mask)
// and d_out = 2 mask (out - y) / max(1, sum mask). One workgroup.
__global__ void __launch_bounds__(256) loss_kernel(const float *out, const float *y,
                                                   const float *mask, int count, float *d_out,
                                                   float *loss) {
  __shared__ float s_red[256];
  const int tid = threadIdx.x;
  float m = 0.0f;
  for (int i = tid; i < count; i += 256) m += mask[i];
  s_red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) s_red[tid] += s_red[tid + w];
    __syncthreads();
  }
  const float denom = fmaxf(1.0f, s_red[0]);
  __syncthreads();
  float l = 0.0f;
  for (int i = tid; i < count; i += 256) {
    const float diff = mask[i] * (out[i] - y[i]);
    l = fmaf(diff, out[i] - y[i], l);
    d_out[i] = __fdiv_rn(2.0f * diff, denom);
  }
  s_red[tid] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) s_red[tid] += s_red[tid + w];
    __syncthreads();
  }
  if (tid == 0 && loss) *loss = __fdiv_rn(s_red[0], denom);
}

hipError_t launch_loss(const float *out, const float *y, const float *mask, int count,
                       float *d_out, float *loss, hipStream_t stream) {
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, stream, out, y, mask, count, d_out,
                     loss);
  return hipGetLastError();
}

// Adam (Kingma and Ba, Algorithm 1): c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void __launch_bounds__(256) adam_kernel(AdamArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.count) return;
  const float g = a.grad[i];
  const float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * g;
  const float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  const float m_hat = m * a.c1, v_hat = v * a.c2;
  a.theta[i] -= __fdiv_rn(a.lr * m_hat, sqrtf(v_hat) + a.eps);
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(adam_kernel, dim3((a.count + 255) / 256), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace onesweep
