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
// L2 between rounds).  Atoms are processed in blocks: the neighbour sums are
// segmented CSR reductions (consecutive lanes = consecutive features, so a
// neighbour row is one coalesced read) staged in LDS, then the message and GRU
// products run on the block.
//   * plain form: float32 FMAs, weights staged in LDS, each thread owning one
//     output feature for several atoms;
//   * precision form (H = 32 or 64): the products run on the matrix cores as
//     v_mfma_f32_32x32x16_bf16 with every float32 operand split into a bfloat16
//     pair (hi + lo) and three products per term (hi*hi + hi*lo + lo*hi), float32
//     accumulation.  Single bfloat16 operands move the scores of this model by
//     ~0.1 pK; the split keeps ~16 mantissa bits.  Each wave owns a 32-atom x
//     32-feature tile of all six GRU gate products, so the gates, the state
//     update and the store happen straight from the accumulators.
#include "cf_internal.h"

namespace cf {

namespace {

constexpr int kThreads = 256;
constexpr int kGather = 8;  // neighbour rows per batch of the neighbour sums

__device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

// ---- shared pieces ------------------------------------------------------------

// h = W_e x + b_e for the pose's atoms (float32)
template <int H>
__device__ inline void sg_embed(const SgWeights &W, const float *__restrict__ feat, int a0, int n, int64_t lb,
                                float *h0) {
  for (int e = threadIdx.x; e < n * H; e += kThreads) {
    const int i = e / H, oo = e % H;
    const float *x = feat + (int64_t)(a0 + i) * CF_NCH;
    float v = W.embed_b[oo];
    for (int c = 0; c < CF_NCH; ++c) v += W.embed_wT[c * H + oo] * x[c];
    h0[(lb + i) * H + oo] = v;
  }
}

// Neighbour sums of atoms [blk, blk+nblk) into A (row stride ld) and their current
// states into Hc; rows past the pose are zero.  Each thread owns four consecutive
// features of a row (one 16-byte load per neighbour row segment) and H / 4 threads
// share a row.  The block's CSR rows are consecutive, so their columns form one
// contiguous range: it is staged in LDS (idx, up to icap entries; columns beyond
// that are read from memory) with coalesced loads, and every thread then walks NU
// of the block's rows at once (nblk <= NU * kThreads / (H / 4)), kSlots neighbours
// per row per step, so that up to 4 NU row loads are in flight with no index load
// in front of them.  Every feature's sum runs over the row's neighbours in CSR order.
template <int H, int NU>
__device__ inline void sg_aggregate(const float *__restrict__ cur, const int32_t *__restrict__ rowp,
                                    const int32_t *__restrict__ colp, int64_t cap, int csr_global, int a0, int base,
                                    int64_t lb, int n, int blk, int nblk, int ld, float *A, float *Hc, int32_t *idx,
                                    int icap, int64_t *status) {
  constexpr int TPR = H / 4;              // threads per row
  constexpr int RPI = kThreads / TPR;     // rows per pass
  constexpr int kSlots = 4;               // neighbours per row per step
  static_assert(H % 4 == 0 && kThreads % TPR == 0, "row split");
  const int tr = threadIdx.x / TPR, c4 = (threadIdx.x % TPR) * 4;
  const int nrow = min(nblk, n - blk);  // rows of the pose in this block (>= 1)
  const int64_t rb = csr_global ? (int64_t)a0 + blk : lb + blk;
  // this thread's rows and their edge ranges (empty for rows past the block)
  int64_t e0[NU], e1[NU];
  int64_t E0 = rowp[rb], E1 = rowp[rb + nrow];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int a = tr + RPI * u;
    e0[u] = e1[u] = 0;
    if (a < nrow) {
      e0[u] = rowp[rb + a];
      e1[u] = rowp[rb + a + 1];
    }
  }
  E1 = E1 < cap ? E1 : cap;
  const int64_t nst = E0 < 0 || E1 <= E0 ? 0 : (E1 - E0 < icap ? E1 - E0 : icap);
  // staged in batches of kStage loads per thread, all in flight together
  constexpr int kStage = 4;
  for (int64_t e0 = 0; e0 < nst; e0 += kStage * kThreads) {
    int32_t cv[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int64_t e = e0 + u * kThreads + threadIdx.x;
      cv[u] = e < nst ? colp[E0 + e] : 0;
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int64_t e = e0 + u * kThreads + threadIdx.x;
      if (e < nst) idx[e] = cv[u];
    }
  }
  bool anybad = false;
  int64_t len = 0;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    if (e1[u] > cap) e1[u] = cap;
    if (e0[u] < 0) {
      anybad = true;
      e0[u] = e1[u];
    }
    len = e1[u] - e0[u] > len ? e1[u] - e0[u] : len;
  }
  __syncthreads();
  float4 s[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) s[u] = make_float4(0.f, 0.f, 0.f, 0.f);
  // whole steps with a branch-free body: slots past a row's end and columns outside
  // the pose read the row's own state (the pose's first row for rows past the
  // block) and add nothing; a bad column is reported once after the loop
  for (int64_t k = 0; k < len; k += kSlots) {
    float4 v[NU][kSlots];
    bool use[NU][kSlots];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int a = tr + RPI * u;
      const int64_t self = lb + (a < nrow ? blk + a : 0);
#pragma unroll
      for (int w = 0; w < kSlots; ++w) {
        const int64_t q = e0[u] + k + w;
        const bool live = q < e1[u];
        const int64_t qs = q - E0;
        int64_t c = 0;
        if (live) c = (qs >= 0 && qs < nst) ? (int64_t)idx[qs] : (int64_t)colp[q];
        const int64_t j = csr_global ? c - base : c;
        const bool bad = j < lb || j >= lb + n;
        anybad |= live && bad;
        use[u][w] = live && !bad;
        v[u][w] = *reinterpret_cast<const float4 *>(cur + (use[u][w] ? j : self) * H + c4);
      }
    }
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
      for (int w = 0; w < kSlots; ++w) {
        s[u].x += use[u][w] ? v[u][w].x : 0.0f;
        s[u].y += use[u][w] ? v[u][w].y : 0.0f;
        s[u].z += use[u][w] ? v[u][w].z : 0.0f;
        s[u].w += use[u][w] ? v[u][w].w : 0.0f;
      }
  }
  if (anybad) dev_fail(status, kDevBadGraph);
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int a = tr + RPI * u;
    if (a < nblk) {
      const float4 hc = a < nrow ? *reinterpret_cast<const float4 *>(cur + (lb + blk + a) * H + c4)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4 *>(A + a * ld + c4) = s[u];
      *reinterpret_cast<float4 *>(Hc + a * ld + c4) = hc;
    }
  }
}

// s = sum over ligand atoms of sigmoid(W_g [h; x] + b_g) * (W_v h + b_v), float32.
// Wg, Wv: LDS copies of the transposed readout weights; red: >= kThreads floats.
template <int H>
__device__ inline void sg_readout(const SgWeights &W, const float *__restrict__ cur, const float *__restrict__ feat,
                                  const uint8_t *__restrict__ is_lig, int a0, int n, int64_t lb, const float *Wg,
                                  const float *Wv, float *red, float *out) {
  constexpr int G = kThreads / H;
  const int o = threadIdx.x % H, g = threadIdx.x / H;
  float acc = 0.0f;
  for (int i = g; i < n; i += G) {
    if (!is_lig[a0 + i]) continue;
    const float *hi = cur + (lb + i) * H;
    const float *xi = feat + (int64_t)(a0 + i) * CF_NCH;
    float gt = W.gate_b[o], vl = W.val_b[o];
    for (int k = 0; k < H; ++k) {
      const float hk = hi[k];
      gt += Wg[k * H + o] * hk;
      vl += Wv[k * H + o] * hk;
    }
    for (int c = 0; c < CF_NCH; ++c) gt += Wg[(H + c) * H + o] * xi[c];
    acc += sigm(gt) * vl;
  }
  red[g * H + o] = acc;
  __syncthreads();
  if ((int)threadIdx.x < H) {
    float s = 0.0f;
    for (int q = 0; q < G; ++q) s += red[q * H + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ---- plain form: float32 on the vector ALUs ----------------------------------

constexpr int kBlk = 32;  // atoms per block (plain form)

template <int H>
struct SgShared {
  float Wt[H * H];
  float Wih[H * 3 * H];
  float Whh[H * 3 * H];
  float A[kBlk * H];
  float M[kBlk * H];
  float Hc[kBlk * H];
};

template <int H>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(H >= 32 ? 3 : 2))) void k_sgcnn_f32(SgWeights W, const int32_t *__restrict__ atom_off,
                                                        int n_atoms, const float *__restrict__ feat,
                                                        const uint8_t *__restrict__ is_lig, int p0,
                                                        const int32_t *__restrict__ cov_row,
                                                        const int32_t *__restrict__ cov_col, int64_t cov_cap,
                                                        const int32_t *__restrict__ nc_row,
                                                        const int32_t *__restrict__ nc_col, int64_t nc_cap,
                                                        int csr_global, float *__restrict__ hbuf, int64_t hcap,
                                                        float *__restrict__ sg_latent, int64_t *__restrict__ status) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  SgShared<H> &S = *reinterpret_cast<SgShared<H> *>(smem_raw);
  constexpr int G = kThreads / H;  // thread groups (one output feature per thread)
  constexpr int APT = kBlk / G;    // atoms per thread in a block
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
  sg_embed<H>(W, feat, a0, n, lb, h0);
  __threadfence();
  __syncthreads();

  float *cur = h0, *nxt = h1;
  const int rounds = W.K_c + W.K_n;
  for (int r = 0; r < rounds; ++r) {
    const int stage = r < W.K_c ? 0 : 1;
    const int32_t *rowp = stage ? nc_row : cov_row;
    const int32_t *colp = stage ? nc_col : cov_col;
    const int64_t cap = stage ? nc_cap : cov_cap;
    for (int e = t; e < H * H; e += kThreads) S.Wt[e] = W.msgT[r][e];
    if (r == 0 || r == W.K_c) {
      for (int e = t; e < 3 * H * H; e += kThreads) {
        S.Wih[e] = W.w_ihT[stage][e];
        S.Whh[e] = W.w_hhT[stage][e];
      }
    }
    const float *bih = W.b_ih[stage], *bhh = W.b_hh[stage];
    __syncthreads();
    for (int blk = 0; blk < n; blk += kBlk) {
      sg_aggregate<H, (kBlk + 4 * kThreads / H - 1) / (4 * kThreads / H)>(cur, rowp, colp, cap, csr_global, a0, base, lb, n, blk, kBlk, H, S.A, S.Hc,
                      reinterpret_cast<int32_t *>(S.M), kBlk * H, status);
      __syncthreads();
      // messages m = W_t a
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
        for (int u = 0; u < APT; ++u) S.M[(g * APT + u) * H + o] = acc[u];
      }
      __syncthreads();
      // GRU update
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
            const float hk = S.Hc[(g * APT + u) * H + k];
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
            nxt[(lb + i) * H + o] = (1.0f - zz) * nn + zz * S.Hc[a * H + o];
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
  // readout (weights staged in the GRU areas)
  for (int e = t; e < (H + CF_NCH) * H; e += kThreads) S.Wih[e] = W.gate_wT[e];
  for (int e = t; e < H * H; e += kThreads) S.Whh[e] = W.val_wT[e];
  __syncthreads();
  sg_readout<H>(W, cur, feat, is_lig, a0, n, lb, S.Wih, S.Whh, S.A, sg_latent + (int64_t)pl * H);
}

// ---- precision form: split-bfloat16 MFMA --------------------------------------

typedef float f32x16v __attribute__((ext_vector_type(16)));

// hi/lo bfloat16 split of 8 consecutive floats
__device__ inline void split8(const float *p, bf16x8 &hi, bf16x8 &lo) {
  const float4 a = *reinterpret_cast<const float4 *>(p);
  const float4 b = *reinterpret_cast<const float4 *>(p + 4);
  const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const bf16_t h = (bf16_t)v[q];
    hi[q] = h;
    lo[q] = (bf16_t)(v[q] - (float)h);
  }
}

__device__ inline f32x16v mfma3(const bf16x8 &ah, const bf16x8 &al, const bf16x8 &bh, const bf16x8 &bl, f32x16v c) {
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c, 0, 0, 0);
  return c;
}

// Tile of one stage at width H: each of the four waves owns a 32-atom x 32-feature
// tile of the block (FB feature blocks x MBK atom blocks); rows padded to LD.
template <int H>
struct SgTile {
  static constexpr int LD = H + 4;      // padded row stride (floats)
  static constexpr int FB = H / 32;     // 32-feature blocks
  static constexpr int MBK = 4 / FB;    // 32-atom blocks per workgroup block
  static constexpr int BLK = 32 * MBK;  // atoms per block
  static constexpr int FLOATS = 3 * BLK * LD;  // A | M | Hc
  static_assert(H % 32 == 0 && H <= 128, "matrix-core widths are 32, 64 or 128");
};

// acc += A[row][0..K) W^T for this lane's output column `col` of N, W given as
// split-bfloat16 MFMA B operands ([K/16][N][16], hi and lo) -- three products per
// term -- or, for the plain form, as float32 W^T [K][N] on the 32x32x2 float32
// matrix instruction.
template <int K, bool F32>
__device__ inline f32x16v mm_row(const float *arow, const bf16_t *bhi, const bf16_t *blo, const float *bT, int N,
                                 int col, int khalf, f32x16v acc) {
  if constexpr (F32) {
#pragma unroll 8
    for (int k = 0; k < K; k += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(arow[k + khalf], bT[(int64_t)(k + khalf) * N + col], acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int ks = 0; ks < K / 16; ++ks) {
      bf16x8 ah, al;
      split8(arow + ks * 16 + khalf * 8, ah, al);
      const int64_t wo = ((int64_t)ks * N + col) * 16 + khalf * 8;
      acc = mfma3(ah, al, *reinterpret_cast<const bf16x8 *>(bhi + wo), *reinterpret_cast<const bf16x8 *>(blo + wo),
                  acc);
    }
  }
  return acc;
}

// One round of one stage at width H for the atoms [blk, blk + BLK) of a pose:
// neighbour sums of the current states (cur), the round's message product, the
// stage's GRU, the new states of those atoms written to nxt (row stride H).
template <int H, bool F32>
__device__ void sg_block(const SgWeights &W, int stage, int r, const int32_t *__restrict__ rowp,
                         const int32_t *__restrict__ colp, int64_t cap, int csr_global, int a0, int base, int64_t lb,
                         int n, int blk, const float *cur, float *nxt, float *lds, int64_t *status) {
  using T = SgTile<H>;
  constexpr int LD = T::LD, BLK = T::BLK;
  static_assert(BLK % (4 * kThreads / H) == 0, "whole rows per thread in the neighbour sums");
  float *A = lds, *M = lds + BLK * LD, *Hc = lds + 2 * BLK * LD;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int mb = wave / T::FB, fb = wave % T::FB;  // this wave's 32-atom x 32-feature tile
  const int lrow = lane & 31, khalf = lane >> 5;
  const int ocol = fb * 32 + lrow;  // output feature of this lane's accumulator column
  const float *bih = W.b_ih[stage], *bhh = W.b_hh[stage];
  const float bir = bih[ocol], biz = bih[H + ocol], bin = bih[2 * H + ocol];
  const float bhr = bhh[ocol], bhz = bhh[H + ocol], bhn = bhh[2 * H + ocol];
    sg_aggregate<H, BLK / (4 * kThreads / H)>(cur, rowp, colp, cap, csr_global, a0, base, lb, n, blk, BLK, LD, A, Hc,
                  reinterpret_cast<int32_t *>(M), BLK * LD, status);
    __syncthreads();
    // messages: M[atoms, ocol] = sum_k A[atoms, k] W_t[ocol, k]
    {
      f32x16v acc = {};
      acc = mm_row<H, F32>(&A[(mb * 32 + lrow) * LD], W.msg_hi[r], W.msg_lo[r], W.msgT[r], H, ocol, khalf, acc);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = mb * 32 + 8 * (j >> 2) + 4 * khalf + (j & 3);
        M[row * LD + ocol] = acc[j];
      }
    }
    __syncthreads();
    // GRU gates for this wave's tile: the reset and update gates accumulate their
    // input and hidden products in one accumulator each; the candidate keeps them
    // apart (the reset gate scales only the hidden part)
    {
      f32x16v gr = {}, gz = {}, gin = {}, ghn = {};
      const float *mrow = &M[(mb * 32 + lrow) * LD], *hrow = &Hc[(mb * 32 + lrow) * LD];
      if constexpr (F32) {
        const float *wi = W.w_ihT[stage], *wh = W.w_hhT[stage];
        gr = mm_row<H, true>(mrow, nullptr, nullptr, wi, 3 * H, ocol, khalf, gr);
        gr = mm_row<H, true>(hrow, nullptr, nullptr, wh, 3 * H, ocol, khalf, gr);
        gz = mm_row<H, true>(mrow, nullptr, nullptr, wi, 3 * H, H + ocol, khalf, gz);
        gz = mm_row<H, true>(hrow, nullptr, nullptr, wh, 3 * H, H + ocol, khalf, gz);
        gin = mm_row<H, true>(mrow, nullptr, nullptr, wi, 3 * H, 2 * H + ocol, khalf, gin);
        ghn = mm_row<H, true>(hrow, nullptr, nullptr, wh, 3 * H, 2 * H + ocol, khalf, ghn);
      } else {
        const bf16_t *ih = W.ih_hi[stage], *il = W.ih_lo[stage], *hh = W.hh_hi[stage], *hl = W.hh_lo[stage];
        constexpr int kUnroll = H <= 64 ? H / 16 : 2;  // wider: bounded unroll keeps it in registers
#pragma unroll kUnroll
        for (int ks = 0; ks < H / 16; ++ks) {
          bf16x8 mhi, mlo, hhi, hlo;
          split8(mrow + ks * 16 + khalf * 8, mhi, mlo);
          split8(hrow + ks * 16 + khalf * 8, hhi, hlo);
          const int64_t w0 = ((int64_t)ks * 3 * H + ocol) * 16 + khalf * 8;
          const int64_t gs = (int64_t)H * 16;  // next gate's rows
          gr = mfma3(mhi, mlo, *reinterpret_cast<const bf16x8 *>(ih + w0), *reinterpret_cast<const bf16x8 *>(il + w0), gr);
          gr = mfma3(hhi, hlo, *reinterpret_cast<const bf16x8 *>(hh + w0), *reinterpret_cast<const bf16x8 *>(hl + w0), gr);
          gz = mfma3(mhi, mlo, *reinterpret_cast<const bf16x8 *>(ih + w0 + gs), *reinterpret_cast<const bf16x8 *>(il + w0 + gs), gz);
          gz = mfma3(hhi, hlo, *reinterpret_cast<const bf16x8 *>(hh + w0 + gs), *reinterpret_cast<const bf16x8 *>(hl + w0 + gs), gz);
          gin = mfma3(mhi, mlo, *reinterpret_cast<const bf16x8 *>(ih + w0 + 2 * gs), *reinterpret_cast<const bf16x8 *>(il + w0 + 2 * gs), gin);
          ghn = mfma3(hhi, hlo, *reinterpret_cast<const bf16x8 *>(hh + w0 + 2 * gs), *reinterpret_cast<const bf16x8 *>(hl + w0 + 2 * gs), ghn);
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = mb * 32 + 8 * (j >> 2) + 4 * khalf + (j & 3);
        const int i = blk + row;
        if (i < n) {
          const float rr = sigm(gr[j] + (bir + bhr));
          const float zz = sigm(gz[j] + (biz + bhz));
          const float nn = tanhf(gin[j] + bin + rr * (ghn[j] + bhn));
          nxt[(lb + i) * H + ocol] = (1.0f - zz) * nn + zz * Hc[row * LD + ocol];
        }
      }
    }
    __syncthreads();
}

// K rounds of one stage at width H (rounds r0 .. r0+K-1 of the weight lists, GRU
// of stage `stage`) over all the pose's atom blocks; states ping-pong between cur
// and nxt (row stride H).
template <int H, bool F32>
__device__ void sg_rounds(const SgWeights &W, int stage, int r0, int K, const int32_t *__restrict__ rowp,
                          const int32_t *__restrict__ colp, int64_t cap, int csr_global, int a0, int base,
                          int64_t lb, int n, float *&cur, float *&nxt, float *lds, int64_t *status) {
  for (int r = r0; r < r0 + K; ++r) {
    for (int blk = 0; blk < n; blk += SgTile<H>::BLK)
      sg_block<H, F32>(W, stage, r, rowp, colp, cap, csr_global, a0, base, lb, n, blk, cur, nxt, lds, status);
    __threadfence();
    __syncthreads();
    float *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

template <int H>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_sgcnn_mfma(
    SgWeights W, const int32_t *__restrict__ atom_off, int n_atoms, const float *__restrict__ feat,
    const uint8_t *__restrict__ is_lig, int p0, const int32_t *__restrict__ cov_row,
    const int32_t *__restrict__ cov_col, int64_t cov_cap, const int32_t *__restrict__ nc_row,
    const int32_t *__restrict__ nc_col, int64_t nc_cap, int csr_global, float *__restrict__ hbuf, int64_t hcap,
    float *__restrict__ sg_latent, int64_t *__restrict__ status) {
  // rounds: A | M | Hc; readout (after the rounds): Wg | Wv | red, in the same
  // space, so that several poses share a CU
  extern __shared__ __attribute__((aligned(16))) float lds[];
  static_assert((H + CF_NCH) * H + H * H + kThreads <= SgTile<H>::FLOATS, "readout staging must fit");
  const int t = threadIdx.x;
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
  float *cur = hbuf, *nxt = hbuf + hcap * H;
  sg_embed<H>(W, feat, a0, n, lb, cur);
  __threadfence();
  __syncthreads();
  sg_rounds<H, false>(W, 0, 0, W.K_c, cov_row, cov_col, cov_cap, csr_global, a0, base, lb, n, cur, nxt, lds, status);
  sg_rounds<H, false>(W, 1, W.K_c, W.K_n, nc_row, nc_col, nc_cap, csr_global, a0, base, lb, n, cur, nxt, lds,
                      status);
  float *Wg = lds, *Wv = lds + (H + CF_NCH) * H, *red = Wv + H * H;
  for (int e = t; e < (H + CF_NCH) * H; e += kThreads) Wg[e] = W.gate_wT[e];
  for (int e = t; e < H * H; e += kThreads) Wv[e] = W.val_wT[e];
  __syncthreads();
  sg_readout<H>(W, cur, feat, is_lig, a0, n, lb, Wg, Wv, red, sg_latent + (int64_t)pl * H);
}

// ---- PotentialNet staging: covalent stage at width HC, per-atom gather,
// linear embedding to width HN, non-covalent stage at HN, readout over ligand
// atoms whose gate reads [h; g].  The per-atom work outside the rounds is small
// (float32 FMAs with the weights read through the caches). ----

// g_i = sigmoid(W_g1 [h_i; x_i] + b) * (W_v1 h_i + b), width HC
template <int HC>
__device__ void sg_mid_gather(const SgWeights &W, const float *__restrict__ cur, const float *__restrict__ feat,
                              int a0, int n, int64_t lb, float *__restrict__ gb) {
  for (int e = threadIdx.x; e < n * HC; e += kThreads) {
    const int i = e / HC, o = e % HC;
    const float *hi = cur + (lb + i) * HC;
    const float *xi = feat + (int64_t)(a0 + i) * CF_NCH;
    float gt = W.mid_gate_b[o], vl = W.mid_val_b[o];
    for (int k = 0; k < HC; ++k) {
      const float hk = hi[k];
      gt += W.mid_gate_wT[k * HC + o] * hk;
      vl += W.mid_val_wT[k * HC + o] * hk;
    }
    for (int c = 0; c < CF_NCH; ++c) gt += W.mid_gate_wT[(HC + c) * HC + o] * xi[c];
    gb[(lb + i) * HC + o] = sigm(gt) * vl;
  }
}

// h_i = W_e2 g_i + b, width HN
template <int HC, int HN>
__device__ void sg_embed2(const SgWeights &W, const float *__restrict__ gb, int n, int64_t lb, float *__restrict__ h) {
  for (int e = threadIdx.x; e < n * HN; e += kThreads) {
    const int i = e / HN, o = e % HN;
    const float *gi = gb + (lb + i) * HC;
    float v = W.embed2_b[o];
    for (int k = 0; k < HC; ++k) v += W.embed2_wT[k * HN + o] * gi[k];
    h[(lb + i) * HN + o] = v;
  }
}

// s = sum over ligand atoms of sigmoid(W_g [h; g] + b_g) * (W_v h + b_v), width HN
template <int HC, int HN>
__device__ void sg_readout_staged(const SgWeights &W, const float *__restrict__ cur, const float *__restrict__ gb,
                                  const uint8_t *__restrict__ is_lig, int a0, int n, int64_t lb, float *red,
                                  float *out) {
  constexpr int G = kThreads / HN;
  const int o = threadIdx.x % HN, g = threadIdx.x / HN;
  float acc = 0.0f;
  for (int i = g; i < n; i += G) {
    if (!is_lig[a0 + i]) continue;
    const float *hi = cur + (lb + i) * HN;
    const float *gi = gb + (lb + i) * HC;
    float gt = W.gate_b[o], vl = W.val_b[o];
    for (int k = 0; k < HN; ++k) {
      const float hk = hi[k];
      gt += W.gate_wT[k * HN + o] * hk;
      vl += W.val_wT[k * HN + o] * hk;
    }
    for (int k = 0; k < HC; ++k) gt += W.gate_wT[(HN + k) * HN + o] * gi[k];
    acc += sigm(gt) * vl;
  }
  red[g * HN + o] = acc;
  __syncthreads();
  if ((int)threadIdx.x < HN) {
    float s = 0.0f;
    for (int q = 0; q < G; ++q) s += red[q * HN + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

template <int HC, int HN, bool F32>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_sgcnn_staged(
    SgWeights W, const int32_t *__restrict__ atom_off, int n_atoms, const float *__restrict__ feat,
    const uint8_t *__restrict__ is_lig, int p0, const int32_t *__restrict__ cov_row,
    const int32_t *__restrict__ cov_col, int64_t cov_cap, const int32_t *__restrict__ nc_row,
    const int32_t *__restrict__ nc_col, int64_t nc_cap, int csr_global, float *__restrict__ hbuf, int64_t hcap,
    float *__restrict__ sg_latent, int64_t *__restrict__ status) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  static_assert(kThreads % HN == 0 && HC <= HN, "stage widths");
  const int t = threadIdx.x;
  const int pl = blockIdx.x;
  const int base = atom_off[p0];
  int a0, a1;
  const bool ok = pose_range(atom_off, p0 + pl, n_atoms, a0, a1);
  const int n = a1 - a0;
  const int64_t lb = (int64_t)a0 - base;
  if (!ok || n <= 0 || lb < 0 || lb + n > hcap) {
    if (t == 0 && (!ok || lb < 0 || lb + n > hcap)) dev_fail(status, kDevBadOffsets);
    if (t < HN) sg_latent[(int64_t)pl * HN + t] = 0.0f;
    return;
  }
  // Each stage has its own pair of state buffers indexed at its own row stride:
  // the workgroups of a launch run different poses at different stages at the
  // same time, so one buffer indexed at two strides would let a pose's wide rows
  // overwrite another pose's narrow ones.  Layout (floats): covalent states
  // 2 x [hcap][HC], covalent gather [hcap][HC], non-covalent states 2 x [hcap][HN].
  float *cur = hbuf, *nxt = hbuf + hcap * HC, *gb = hbuf + 2 * hcap * HC;
  float *cur2 = gb + hcap * HC, *nxt2 = cur2 + hcap * HN;
  sg_embed<HC>(W, feat, a0, n, lb, cur);
  __threadfence();
  __syncthreads();
  sg_rounds<HC, F32>(W, 0, 0, W.K_c, cov_row, cov_col, cov_cap, csr_global, a0, base, lb, n, cur, nxt, lds, status);
  sg_mid_gather<HC>(W, cur, feat, a0, n, lb, gb);
  __threadfence();
  __syncthreads();
  sg_embed2<HC, HN>(W, gb, n, lb, cur2);
  __threadfence();
  __syncthreads();
  sg_rounds<HN, F32>(W, 1, W.K_c, W.K_n, nc_row, nc_col, nc_cap, csr_global, a0, base, lb, n, cur2, nxt2, lds,
                     status);
  sg_readout_staged<HC, HN>(W, cur2, gb, is_lig, a0, n, lb, lds, sg_latent + (int64_t)pl * HN);
}

template <typename K>
void set_lds_attr(K kernel, size_t lds) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
}

template <int H>
hipError_t launch_h(const SgWeights &W, int mfma, const int32_t *atom_off, int n_atoms, const float *feat,
                    const uint8_t *is_lig, int p0, int n_poses, const int32_t *cov_row, const int32_t *cov_col,
                    int64_t cov_cap, const int32_t *nc_row, const int32_t *nc_col, int64_t nc_cap, int csr_global,
                    float *hbuf, int64_t hcap, float *sg_latent, int64_t *status, hipStream_t s) {
  static_assert((H + CF_NCH) * H <= 3 * H * H, "readout weights must fit the staging area");
  if constexpr (H >= 32) {
    if (mfma) {
      const size_t lds = sizeof(float) * SgTile<H>::FLOATS;
      static bool attr = false;
      if (!attr) {
        set_lds_attr(&k_sgcnn_mfma<H>, lds);
        attr = true;
      }
      hipLaunchKernelGGL((k_sgcnn_mfma<H>), dim3(n_poses), dim3(kThreads), lds, s, W, atom_off, n_atoms, feat,
                         is_lig, p0, cov_row, cov_col, cov_cap, nc_row, nc_col, nc_cap, csr_global, hbuf, hcap,
                         sg_latent, status);
      return hipGetLastError();
    }
  }
  const size_t lds = sizeof(SgShared<H>);
  static bool attr = false;
  if (!attr) {
    set_lds_attr(&k_sgcnn_f32<H>, lds);
    attr = true;
  }
  hipLaunchKernelGGL((k_sgcnn_f32<H>), dim3(n_poses), dim3(kThreads), lds, s, W, atom_off, n_atoms, feat, is_lig,
                     p0, cov_row, cov_col, cov_cap, nc_row, nc_col, nc_cap, csr_global, hbuf, hcap, sg_latent,
                     status);
  return hipGetLastError();
}

template <int HC, int HN>
hipError_t launch_staged(const SgWeights &W, int bf16, const int32_t *atom_off, int n_atoms, const float *feat,
                         const uint8_t *is_lig, int p0, int n_poses, const int32_t *cov_row, const int32_t *cov_col,
                         int64_t cov_cap, const int32_t *nc_row, const int32_t *nc_col, int64_t nc_cap,
                         int csr_global, float *hbuf, int64_t hcap, float *sg_latent, int64_t *status,
                         hipStream_t s) {
  constexpr int fl = SgTile<HC>::FLOATS > SgTile<HN>::FLOATS ? SgTile<HC>::FLOATS : SgTile<HN>::FLOATS;
  const size_t lds = sizeof(float) * (fl > kThreads ? fl : kThreads);
  if (bf16) {
    static bool attr = false;
    if (!attr) {
      set_lds_attr(&k_sgcnn_staged<HC, HN, false>, lds);
      attr = true;
    }
    hipLaunchKernelGGL((k_sgcnn_staged<HC, HN, false>), dim3(n_poses), dim3(kThreads), lds, s, W, atom_off,
                       n_atoms, feat, is_lig, p0, cov_row, cov_col, cov_cap, nc_row, nc_col, nc_cap, csr_global,
                       hbuf, hcap, sg_latent, status);
  } else {
    static bool attr = false;
    if (!attr) {
      set_lds_attr(&k_sgcnn_staged<HC, HN, true>, lds);
      attr = true;
    }
    hipLaunchKernelGGL((k_sgcnn_staged<HC, HN, true>), dim3(n_poses), dim3(kThreads), lds, s, W, atom_off,
                       n_atoms, feat, is_lig, p0, cov_row, cov_col, cov_cap, nc_row, nc_col, nc_cap, csr_global,
                       hbuf, hcap, sg_latent, status);
  }
  return hipGetLastError();
}

}  // namespace

// widths the staged kernel is built for (covalent, non-covalent)
bool sgcnn_staged_supported(int hc, int hn) {
  return (hc == 32 && (hn == 64 || hn == 128)) || (hc == 64 && hn == 128);
}

hipError_t launch_sgcnn(const SgWeights &W, int bf16, const int32_t *atom_off, int n_atoms, const float *feat,
                        const uint8_t *is_lig, int p0, int n_poses, const int32_t *cov_row,
                        const int32_t *cov_col, int64_t cov_cap, const int32_t *nc_row,
                        const int32_t *nc_col, int64_t nc_cap, int csr_global, float *hbuf,
                        int64_t hcap_atoms, float *sg_latent, int64_t *status, hipStream_t s) {
  if (n_poses <= 0) return hipSuccess;
  if (W.staged) {
    // the precision form needs the split-bfloat16 weight copies
    const int split = bf16 && W.msg_hi[0] != nullptr;
    if (bf16 && !split) return hipErrorInvalidValue;
#define CF_ST(HC, HN)                                                                                             if (W.H == HC && W.H2 == HN)                                                                                      return launch_staged<HC, HN>(W, split, atom_off, n_atoms, feat, is_lig, p0, n_poses, cov_row, cov_col,                                       cov_cap, nc_row, nc_col, nc_cap, csr_global, hbuf, hcap_atoms, sg_latent, status, s);
    CF_ST(32, 64)
    CF_ST(32, 128)
    CF_ST(64, 128)
#undef CF_ST
    return hipErrorInvalidValue;
  }
  // the matrix-core path needs the split-bfloat16 weight copies (precision form, H >= 32)
  const int mfma = bf16 && W.msg_hi[0] != nullptr;
#define CF_SG(HH)                                                                                              \
  if (W.H == HH)                                                                                               \
    return launch_h<HH>(W, mfma, atom_off, n_atoms, feat, is_lig, p0, n_poses, cov_row, cov_col, cov_cap,      \
                        nc_row, nc_col, nc_cap, csr_global, hbuf, hcap_atoms, sg_latent, status, s);
  CF_SG(16)
  CF_SG(32)
  CF_SG(64)
#undef CF_SG
  return hipErrorInvalidValue;
}

}  // namespace cf
