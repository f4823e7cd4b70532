// SG-CNN forward: embedding, gated graph propagation and gated ligand readout.
//
// The paper's SG-CNN is PotentialNet built on gated graph sequence networks
// (Sec. 3.3.1, Table II): node states are propagated first over covalent edges
// (K_c rounds) and then over non-covalent edges (K_n rounds); each round sums
// the neighbours' states, applies a per-round message matrix and updates every
// state with a gated recurrent unit shared by the rounds of a stage; a gated sum
// over the ligand atoms ("gather") gives the latent that enters the fusion head.
//
// Design: one workgroup per pose (a pose's states, <= 4096 x H floats, stay in
// L2 between rounds).  Atoms are processed in blocks of 32: the neighbour sums
// are segmented CSR reductions (consecutive lanes = consecutive features, so a
// neighbour row is one coalesced read), and the message and GRU products run out
// of LDS with the weights staged once per round / stage, each thread owning one
// output feature for several atoms (register blocking).  In the precision form
// the GEMM operands (neighbour sums, messages, states and the message / GRU
// weights) are rounded to bfloat16 and accumulated in float32; gates, state
// update and readout stay float32.
#include "cf_internal.h"

namespace cf {

namespace {

constexpr int kThreads = 256;
constexpr int kBlk = 32;  // atoms per block

template <bool BF>
__device__ inline float rb(float x) {
  if constexpr (BF)
    return (float)(bf16_t)x;
  else
    return x;
}

__device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

template <int H, bool BF>
struct SgShared {
  float Wt[H * H];
  float Wih[H * 3 * H];
  float Whh[H * 3 * H];
  float A[kBlk * H];
  float M[kBlk * H];
  float Hc[kBlk * H];
};

template <int H, bool BF>
__global__ __launch_bounds__(kThreads) void k_sgcnn(SgWeights W, const int32_t *__restrict__ atom_off, int n_atoms,
                                                    const float *__restrict__ feat,
                                                    const uint8_t *__restrict__ is_lig, int p0,
                                                    const int32_t *__restrict__ cov_row,
                                                    const int32_t *__restrict__ cov_col, int64_t cov_cap,
                                                    const int32_t *__restrict__ nc_row,
                                                    const int32_t *__restrict__ nc_col, int64_t nc_cap,
                                                    int csr_global, float *__restrict__ hbuf,
                                                    int64_t hcap, float *__restrict__ sg_latent,
                                                    int64_t *__restrict__ status) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  SgShared<H, BF> &S = *reinterpret_cast<SgShared<H, BF> *>(smem_raw);
  constexpr int G = kThreads / H;     // thread groups (one output feature per thread)
  constexpr int APT = kBlk / G;       // atoms per thread in a block
  const int t = threadIdx.x;
  const int o = t % H, g = t / H;
  const int pl = blockIdx.x;
  const int base = atom_off[p0];
  int a0, a1;
  const bool ok = pose_range(atom_off, p0 + pl, n_atoms, a0, a1);
  const int n = a1 - a0;
  const int64_t lb = (int64_t)a0 - base;
  if (!ok || n <= 0 || lb < 0 || lb + n > hcap) {
    if (t == 0 && (!ok || lb < 0 || lb + n > hcap)) dev_fail(status, kDevBadOffsets);
    if (t < H) sg_latent[(int64_t)pl * H + t] = 0.0f;
    return;
  }
  float *h0 = hbuf, *h1 = hbuf + hcap * H;

  // ---- embedding h = W_e x + b_e (float32) ----
  for (int e = t; e < n * H; e += kThreads) {
    const int i = e / H, oo = e % H;
    const float *x = feat + (int64_t)(a0 + i) * CF_NCH;
    float v = W.embed_b[oo];
    for (int c = 0; c < CF_NCH; ++c) v += W.embed_wT[c * H + oo] * x[c];
    h0[(lb + i) * H + oo] = v;
  }
  __threadfence();
  __syncthreads();

  float *cur = h0, *nxt = h1;
  const int rounds = W.K_c + W.K_n;
  for (int r = 0; r < rounds; ++r) {
    const int stage = r < W.K_c ? 0 : 1;
    const int32_t *rowp = stage ? nc_row : cov_row;
    const int32_t *colp = stage ? nc_col : cov_col;
    const int64_t cap = stage ? nc_cap : cov_cap;
    for (int e = t; e < H * H; e += kThreads) S.Wt[e] = rb<BF>(W.msgT[r][e]);
    if (r == 0 || r == W.K_c) {
      for (int e = t; e < 3 * H * H; e += kThreads) {
        S.Wih[e] = rb<BF>(W.w_ihT[stage][e]);
        S.Whh[e] = rb<BF>(W.w_hhT[stage][e]);
      }
    }
    const float *bih = W.b_ih[stage], *bhh = W.b_hh[stage];
    __syncthreads();
    for (int blk = 0; blk < n; blk += kBlk) {
      // phase A: neighbour sums and the block's current states
      for (int e = t; e < kBlk * H; e += kThreads) {
        const int a = e / H, oo = e % H;
        const int i = blk + a;
        float s = 0.0f, hc = 0.0f;
        if (i < n) {
          const int64_t ri = csr_global ? (int64_t)a0 + i : lb + i;
          int64_t e0 = rowp[ri], e1 = rowp[ri + 1];
          if (e1 > cap) e1 = cap;
          if (e0 < 0) {
            dev_fail(status, kDevBadGraph);
            e0 = e1;
          }
          for (int64_t q = e0; q < e1; ++q) {
            int64_t j = colp[q];
            if (csr_global) j -= base;
            if (j < lb || j >= lb + n) {
              dev_fail(status, kDevBadGraph);
              continue;
            }
            s += cur[j * H + oo];
          }
          hc = cur[(lb + i) * H + oo];
        }
        S.A[a * H + oo] = rb<BF>(s);
        S.Hc[a * H + oo] = hc;
      }
      __syncthreads();
      // phase B: messages m = W_t a
      {
        float acc[APT];
#pragma unroll
        for (int u = 0; u < APT; ++u) acc[u] = 0.0f;
        for (int k = 0; k < H; ++k) {
          const float w = S.Wt[k * H + o];
#pragma unroll
          for (int u = 0; u < APT; ++u) acc[u] += w * S.A[(g * APT + u) * H + k];
        }
#pragma unroll
        for (int u = 0; u < APT; ++u) S.M[(g * APT + u) * H + o] = rb<BF>(acc[u]);
      }
      __syncthreads();
      // phase C: GRU update
      {
        float ir[APT], iz[APT], in_[APT], hr[APT], hz[APT], hn[APT];
#pragma unroll
        for (int u = 0; u < APT; ++u) {
          ir[u] = bih[o];
          iz[u] = bih[H + o];
          in_[u] = bih[2 * H + o];
          hr[u] = bhh[o];
          hz[u] = bhh[H + o];
          hn[u] = bhh[2 * H + o];
        }
        for (int k = 0; k < H; ++k) {
          const float wir = S.Wih[k * 3 * H + o], wiz = S.Wih[k * 3 * H + H + o], win = S.Wih[k * 3 * H + 2 * H + o];
          const float whr = S.Whh[k * 3 * H + o], whz = S.Whh[k * 3 * H + H + o], whn = S.Whh[k * 3 * H + 2 * H + o];
#pragma unroll
          for (int u = 0; u < APT; ++u) {
            const float m = S.M[(g * APT + u) * H + k];
            const float hk = rb<BF>(S.Hc[(g * APT + u) * H + k]);
            ir[u] += wir * m;
            iz[u] += wiz * m;
            in_[u] += win * m;
            hr[u] += whr * hk;
            hz[u] += whz * hk;
            hn[u] += whn * hk;
          }
        }
#pragma unroll
        for (int u = 0; u < APT; ++u) {
          const int a = g * APT + u;
          const int i = blk + a;
          if (i < n) {
            const float rr = sigm(ir[u] + hr[u]);
            const float zz = sigm(iz[u] + hz[u]);
            const float nn = tanhf(in_[u] + rr * hn[u]);
            const float hold = S.Hc[a * H + o];
            nxt[(lb + i) * H + o] = (1.0f - zz) * nn + zz * hold;
          }
        }
      }
      __syncthreads();
    }
    __threadfence();
    __syncthreads();
    float *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }

  // ---- gated readout over ligand atoms (float32) ----
  for (int e = t; e < (H + CF_NCH) * H; e += kThreads) S.Wih[e] = W.gate_wT[e];
  for (int e = t; e < H * H; e += kThreads) S.Whh[e] = W.val_wT[e];
  __syncthreads();
  float acc = 0.0f;
  for (int i = g; i < n; i += G) {
    if (!is_lig[a0 + i]) continue;
    const float *hi = cur + (lb + i) * H;
    const float *xi = feat + (int64_t)(a0 + i) * CF_NCH;
    float gt = W.gate_b[o], vl = W.val_b[o];
    for (int k = 0; k < H; ++k) {
      const float hk = hi[k];
      gt += S.Wih[k * H + o] * hk;
      vl += S.Whh[k * H + o] * hk;
    }
    for (int c = 0; c < CF_NCH; ++c) gt += S.Wih[(H + c) * H + o] * xi[c];
    acc += sigm(gt) * vl;
  }
  S.A[g * H + o] = acc;
  __syncthreads();
  if (t < H) {
    float s = 0.0f;
    for (int q = 0; q < G; ++q) s += S.A[q * H + t];
    sg_latent[(int64_t)pl * H + t] = s;
  }
}

template <int H, bool BF>
hipError_t launch_h(const SgWeights &W, const int32_t *atom_off, int n_atoms, const float *feat, const uint8_t *is_lig,
                    int p0, int n_poses, const int32_t *cov_row, const int32_t *cov_col, int64_t cov_cap,
                    const int32_t *nc_row, const int32_t *nc_col, int64_t nc_cap, int csr_global, float *hbuf,
                    int64_t hcap, float *sg_latent, int64_t *status, hipStream_t s) {
  static_assert((H + CF_NCH) * H <= 3 * H * H, "readout weights must fit the staging area");
  const size_t lds = sizeof(SgShared<H, BF>);
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sgcnn<H, BF>), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL((k_sgcnn<H, BF>), dim3(n_poses), dim3(kThreads), lds, s, W, atom_off, n_atoms, feat, is_lig, p0,
                     cov_row, cov_col, cov_cap, nc_row, nc_col, nc_cap, csr_global, hbuf, hcap, sg_latent,
                     status);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sgcnn(const SgWeights &W, int bf16, const int32_t *atom_off, int n_atoms, const float *feat,
                        const uint8_t *is_lig, int p0, int n_poses, const int32_t *cov_row,
                        const int32_t *cov_col, int64_t cov_cap, const int32_t *nc_row,
                        const int32_t *nc_col, int64_t nc_cap, int csr_global, float *hbuf,
                        int64_t hcap_atoms, float *sg_latent, int64_t *status, hipStream_t s) {
  if (n_poses <= 0) return hipSuccess;
  // The precision form keeps float32 operands here until the split-bfloat16
  // matrix-core path lands: single bfloat16 operands move scores by ~0.1 pK.
  bf16 = 0;
#define CF_SG(HH)                                                                                            \
  if (W.H == HH)                                                                                             \
    return bf16 ? launch_h<HH, true>(W, atom_off, n_atoms, feat, is_lig, p0, n_poses, cov_row, cov_col, cov_cap,      \
                                     nc_row, nc_col, nc_cap, csr_global, hbuf, hcap_atoms, sg_latent,        \
                                     status, s)                                                              \
                : launch_h<HH, false>(W, atom_off, n_atoms, feat, is_lig, p0, n_poses, cov_row, cov_col, cov_cap,     \
                                      nc_row, nc_col, nc_cap, csr_global, hbuf, hcap_atoms, sg_latent,       \
                                      status, s);
  CF_SG(16)
  CF_SG(32)
  CF_SG(64)
#undef CF_SG
  return hipErrorInvalidValue;
}

}  // namespace cf
