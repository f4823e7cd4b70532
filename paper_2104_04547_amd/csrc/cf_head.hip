// Global average pooling + dense head of the 3D-CNN, and the fusion head.
//
// Pooling and the CNN dense layer close the 3D-CNN (Sec. 3.3.1, Table III: dense
// nodes).  The fusion head turns the two latents into one pK (Eq. 1) in any of the
// paper's three forms: Coherent Fusion (concatenation + SELU fusion layers, Sec.
// 2.2, Table V), Mid-level Fusion (model-specific SELU layers whose outputs join
// the raw latents, residual fusion layers, Sec. 2.1, Table IV) and Late Fusion
// (the mean of the two branches' own predictions, Sec. 2.1).  The host compiles
// the model's head into a short list of dense layers that one kernel runs.
// Inference applies no dropout.  Reductions run in a fixed order, so a pose's
// result does not depend on the batch it is scored in.
#include "cf_internal.h"

namespace cf {

namespace {

constexpr float kSeluLambda = 1.0507009873554804934193349852946f;
constexpr float kSeluAlpha = 1.6732632423543772848170429916717f;

template <typename T>
__global__ __launch_bounds__(256) void k_pool_dense(const T *__restrict__ act, int vox, int cstride, int c,
                                                    const float *__restrict__ dw, const float *__restrict__ db,
                                                    int n_dense, const float *__restrict__ dw2,
                                                    const float *__restrict__ db2, int n_dense2,
                                                    float *__restrict__ latent) {
  // 16-byte loads: each thread owns KV consecutive channels (a channel group g) of
  // the voxels v = vr, vr + NV, ... (NV = 256 / groups); the per-thread sums run
  // over v in ascending order and the NV partial sums of a channel are added in
  // order of vr, so the mean does not depend on scheduling
  constexpr int KV = 16 / sizeof(T);
  __shared__ float part[256 * KV];
  __shared__ float mean[256];
  __shared__ float hid[256];
  const int pose = blockIdx.x;
  const T *a = act + (int64_t)pose * vox * cstride;
  const int groups = cstride / KV, NV = 256 / groups;  // threads past NV * groups sit out
  const int g = threadIdx.x % groups, vr = threadIdx.x / groups;
  float s[KV];
#pragma unroll
  for (int q = 0; q < KV; ++q) s[q] = 0.0f;
  for (int v = vr < NV ? vr : vox; v < vox; v += NV) {
    const uint4 raw = *reinterpret_cast<const uint4 *>(a + (int64_t)v * cstride + g * KV);
    const T *x = reinterpret_cast<const T *>(&raw);
#pragma unroll
    for (int q = 0; q < KV; ++q) s[q] += (float)x[q];
  }
  if (vr < NV)
#pragma unroll
    for (int q = 0; q < KV; ++q) part[vr * cstride + g * KV + q] = s[q];
  __syncthreads();
  const float inv = 1.0f / (float)vox;
  for (int ch = threadIdx.x; ch < c; ch += 256) {
    float m = 0.0f;
    for (int r = 0; r < NV; ++r) m += part[r * cstride + ch];
    mean[ch] = m * inv;
  }
  __syncthreads();
  if (n_dense == 0) {
    for (int ch = threadIdx.x; ch < c; ch += 256) latent[(int64_t)pose * c + ch] = mean[ch];
  } else if (n_dense2 == 0) {
    for (int o = threadIdx.x; o < n_dense; o += 256) {
      float acc = db[o];
      for (int k = 0; k < c; ++k) acc += dw[o * c + k] * mean[k];
      latent[(int64_t)pose * n_dense + o] = acc > 0.f ? acc : 0.f;
    }
  } else {
    for (int o = threadIdx.x; o < n_dense; o += 256) {
      float acc = db[o];
      for (int k = 0; k < c; ++k) acc += dw[o * c + k] * mean[k];
      hid[o] = acc > 0.f ? acc : 0.f;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < n_dense2; o += 256) {
      float acc = db2[o];
      for (int k = 0; k < n_dense; ++k) acc += dw2[o * n_dense + k] * hid[k];
      latent[(int64_t)pose * n_dense2 + o] = acc > 0.f ? acc : 0.f;
    }
  }
}

__device__ inline float selu(float x) { return x > 0.f ? kSeluLambda * x : kSeluLambda * kSeluAlpha * expm1f(x); }

// One wavefront per pose; the feature buffer lives in LDS.
__global__ __launch_bounds__(64) void k_head(const float *__restrict__ cnn, int lc, const float *__restrict__ sg,
                                             int H, const float *__restrict__ prm, HeadProgram hp,
                                             float *__restrict__ scores) {
  __shared__ float z[kHeadBuf];
  const int pose = blockIdx.x;
  const int lane = threadIdx.x;
  for (int k = lane; k < lc + H; k += 64)
    z[k] = k < lc ? cnn[(int64_t)pose * lc + k] : sg[(int64_t)pose * H + (k - lc)];
  __syncthreads();
  for (int i = 0; i < hp.n_ops; ++i) {
    const HeadOp op = hp.op[i];
    const float *W = prm + op.w;
    for (int o = lane; o < op.n_out; o += 64) {
      float acc = prm[op.b + o];
      const float *row = W + (int64_t)o * (op.n0 + op.n1);
      for (int k = 0; k < op.n0; ++k) acc += row[k] * z[op.src0 + k];
      for (int k = 0; k < op.n1; ++k) acc += row[op.n0 + k] * z[op.src1 + k];
      if (op.act == kActRelu) acc = acc > 0.f ? acc : 0.f;
      else if (op.act == kActSelu) acc = selu(acc);
      if (op.res >= 0) acc += z[op.res + o];
      z[op.dst + o] = acc;
    }
    __syncthreads();
  }
  if (lane == 0) {
    float s = z[hp.out_slot[0]];
    if (hp.n_out == 2) s += z[hp.out_slot[1]];
    scores[pose] = hp.out_scale * s;
  }
}

}  // namespace

hipError_t launch_pool_dense(const void *act, int bf16, int n_poses, int vox, int cstride, int c,
                             const float *dense_w, const float *dense_b, int n_dense, const float *dense2_w,
                             const float *dense2_b, int n_dense2, float *latent, hipStream_t s) {
  if (n_poses <= 0) return hipSuccess;
  if (c > 256 || n_dense > 256 || n_dense2 > 256 || (n_dense2 && !n_dense)) return hipErrorInvalidValue;
  // channel groups of 16 bytes must tile the row, at most one per thread
  if (c > cstride || cstride % (bf16 ? 8 : 4) || cstride / (bf16 ? 8 : 4) > 256) return hipErrorInvalidValue;
  if (bf16)
    hipLaunchKernelGGL(k_pool_dense<bf16_t>, dim3(n_poses), dim3(256), 0, s, reinterpret_cast<const bf16_t *>(act),
                       vox, cstride, c, dense_w, dense_b, n_dense, dense2_w, dense2_b, n_dense2, latent);
  else
    hipLaunchKernelGGL(k_pool_dense<float>, dim3(n_poses), dim3(256), 0, s, reinterpret_cast<const float *>(act),
                       vox, cstride, c, dense_w, dense_b, n_dense, dense2_w, dense2_b, n_dense2, latent);
  return hipGetLastError();
}

hipError_t launch_head(const float *cnn_lat, int lc, const float *sg_lat, int H, const float *params,
                       const HeadProgram &hp, int n_poses, float *scores, hipStream_t s) {
  if (n_poses <= 0) return hipSuccess;
  if (lc + H > kHeadBuf || hp.n_ops < 1 || hp.n_ops > kHeadMaxOps) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_head, dim3(n_poses), dim3(64), 0, s, cnn_lat, lc, sg_lat, H, params, hp, scores);
  return hipGetLastError();
}

}  // namespace cf
