// Selection after scoring: best pose per compound and top-k compounds.
//
// In the paper's screen each compound has up to 10 docked poses per binding site
// (40 over four sites) and is represented by its strongest prediction -- the
// maximum Coherent Fusion pK over its poses (Sec. 5.2); compounds are then ranked
// and the best few purchased for assays (the 100-of-1,000,000 example, Sec. 3.4).
//
// cf_compound_max: one thread per segment (segments are short), NaN scores are
// ignored, ties go to the lowest pose index.
// cf_top_k: exact radix select on 64-bit keys (order-preserving 32-bit image of
// the value, then the complemented index, so every key is distinct and the
// ranking is "value descending, index ascending"): 8 passes of an 8-bit digit
// histogram find the k-th key, one pass collects the keys at or above it, and a
// single workgroup sorts those k keys.  Results are deterministic.
#include <algorithm>
#include <cfloat>
#include <climits>
#include <mutex>

#include "cf_internal.h"

namespace cf {

namespace {

constexpr int kSelThreads = 256;

__device__ inline uint64_t topk_key(float v, int i) {
  uint32_t u = v == 0.0f ? 0u : __float_as_uint(v);  // -0 and +0 are the same value
  uint32_t k;
  if (v != v)
    k = 0u;  // NaN ranks last
  else
    k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)k << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
}

__global__ __launch_bounds__(kSelThreads) void k_segmax(const float *__restrict__ scores, int n_scores,
                                                        const int32_t *__restrict__ off, int n_seg,
                                                        float *__restrict__ best, int32_t *__restrict__ best_idx,
                                                        int64_t *status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_seg) return;
  int a = off[c], b = off[c + 1];
  if (a < 0 || b < a || b > n_scores) {
    dev_fail(status, kDevBadOffsets);
    a = b = 0;
  }
  float m = -FLT_MAX;
  int idx = -1;
  for (int p = a; p < b; ++p) {
    const float v = scores[p];
    if (v == v && (idx < 0 || v > m)) {
      m = v;
      idx = p;
    }
  }
  best[c] = idx < 0 ? -INFINITY : m;
  best_idx[c] = idx;
}

// state: [0] prefix (uint64), [1] mask of decided bits, [2] k remaining
__global__ void k_topk_init(uint32_t *hist, uint64_t *state, int k) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x == 0) {
    state[0] = 0;
    state[1] = 0;
    state[2] = (uint64_t)k;
    state[3] = 0;  // collected count
  }
}

__global__ __launch_bounds__(kSelThreads) void k_topk_hist(const float *__restrict__ v, int n, int shift,
                                                           uint32_t *hist, const uint64_t *state) {
  __shared__ uint32_t h[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint64_t prefix = state[0], mask = state[1];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t key = topk_key(v[i], i);
    if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 0xFF], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// one thread: choose the digit whose bucket holds the k-th largest key, then
// clear the histogram for the next pass
__global__ void k_topk_pick(uint32_t *hist, uint64_t *state, int shift) {
  if (threadIdx.x == 0) {
    uint64_t krem = state[2];
    int d = 255;
    for (; d > 0; --d) {
      if (hist[d] >= krem) break;
      krem -= hist[d];
    }
    state[0] |= (uint64_t)d << shift;
    state[1] |= (uint64_t)0xFF << shift;
    state[2] = krem;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
}

__global__ __launch_bounds__(kSelThreads) void k_topk_collect(const float *__restrict__ v, int n, uint64_t *state,
                                                              uint64_t *cand, int k) {
  const uint64_t thr = state[0];  // the k-th largest key (all keys are distinct)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t key = topk_key(v[i], i);
    if (key >= thr) {
      const unsigned long long slot = atomicAdd(reinterpret_cast<unsigned long long *>(&state[3]), 1ull);
      if (slot < (unsigned long long)k) cand[slot] = key;
    }
  }
}

// bitonic sort of k <= 1024 keys (padded to a power of two with zeros), descending
__global__ __launch_bounds__(1024) void k_topk_sort(const uint64_t *cand, int k, const float *__restrict__ v,
                                                    int32_t *idx_out, float *val_out) {
  __shared__ uint64_t s[1024];
  int m = 1;
  while (m < k) m <<= 1;
  for (int i = threadIdx.x; i < m; i += blockDim.x) s[i] = i < k ? cand[i] : 0ull;
  __syncthreads();
  for (int size = 2; size <= m; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const uint64_t a = s[i], b = s[j];
          if (desc ? (a < b) : (a > b)) {
            s[i] = b;
            s[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const int idx = (int)(0xFFFFFFFFu - (uint32_t)(s[i] & 0xFFFFFFFFu));
    idx_out[i] = idx;
    if (val_out) val_out[i] = v[idx];
  }
}

}  // namespace

hipError_t launch_segmax(const float *scores, int n_scores, const int32_t *off, int n_seg, float *best,
                         int32_t *best_idx, int64_t *status, hipStream_t s) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_segmax, dim3((n_seg + kSelThreads - 1) / kSelThreads), dim3(kSelThreads), 0, s, scores,
                     n_scores, off, n_seg, best, best_idx, status);
  return hipGetLastError();
}

// Scratch of the allocation-free top-k: the 256-bin histogram (1 KB), the select
// state (64 B) and the k <= 1024 collected keys (8 KB).  One copy per GPU, held
// until the process ends; every allocation-free call on a GPU shares it.
static __device__ __align__(256) unsigned char scratch[kTopkScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's copy of `scratch`, looked up once per
// device (the array's name in host code is a host-side stand-in, not a device
// address).  Later calls read the cached pointer.
hipError_t topk_static_scratch(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_topk(const float *v, int n, int k, int32_t *idx_out, float *val_out, void *scratch,
                       hipStream_t s) {
  uint32_t *hist = reinterpret_cast<uint32_t *>(scratch);
  uint64_t *state = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(scratch) + 1024);
  uint64_t *cand = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(scratch) + 1024 + 64);
  const int blocks = (int)std::min<int64_t>(1024, ((int64_t)n + kSelThreads - 1) / kSelThreads);
  hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, s, hist, state, k);
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_topk_hist, dim3(blocks), dim3(kSelThreads), 0, s, v, n, shift, hist, state);
    hipLaunchKernelGGL(k_topk_pick, dim3(1), dim3(256), 0, s, hist, state, shift);
  }
  hipLaunchKernelGGL(k_topk_collect, dim3(blocks), dim3(kSelThreads), 0, s, v, n, state, cand, k);
  hipLaunchKernelGGL(k_topk_sort, dim3(1), dim3(1024), 0, s, cand, k, v, idx_out, val_out);
  return hipGetLastError();
}

}  // namespace cf
