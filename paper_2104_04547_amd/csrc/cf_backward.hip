// Backward pass of the Coherent Fusion score, for fine-tuning.
//
// Coherent Fusion trains the fusion layers and both branches together: the loss
// gradient reaches the 3D-CNN and the SG-CNN through the concatenated latents
// (Sec. 2.2; training hyper-parameters in Table V).  These kernels compute, for
// one upstream gradient per pose g_p = dL/ds_p, the vector-Jacobian product
// sum_p g_p ds_p/dtheta for every parameter theta, in float32.
//
// Design: plain kernels, one output element per thread, every reduction in a
// fixed order (row chunks, then partial sums in order), so gradients are
// reproducible bit for bit and independent of the launch shape.
//   * per-atom matrix products of the SG-CNN (H <= 64): one thread per output
//     entry over a row of the weight matrix;
//   * weight gradients sum_i U[i][a] V[i][b] over atoms / poses / voxels: row
//     chunks into partial sums, then one pass adding the partials in order;
//   * conv weight gradient: LDS-tiled (32 output channels x 64 (tap, channel)
//     columns) over 16-voxel steps of one pose, partial per pose;
//   * conv data gradient: LDS-tiled (64 voxels x 64 channels) over taps and
//     16-channel steps, the transposed conv as a gather (stride 2 reads only the
//     output voxels a tap reaches).
#include <algorithm>
#include <cmath>

#include "cf_internal.h"

namespace cf {

namespace {

constexpr int kT = 256;

inline dim3 grid1(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kT - 1) / kT, 1 << 20))); }

__global__ __launch_bounds__(kT) void k_fill(float *p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) p[i] = v;
}

__global__ __launch_bounds__(kT) void k_add(float *dst, const float *src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) dst[i] += src[i];
}

// Y[i][j] (+)= b[j] + sum_k W[j][k] X[i][k]
__global__ __launch_bounds__(kT) void k_rowmat(const float *__restrict__ X, int ldx, int n, int K,
                                               const float *__restrict__ W, int ldw, const float *__restrict__ b,
                                               int J, float *__restrict__ Y, int ldy, int accumulate) {
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < (int64_t)n * J; e += (int64_t)gridDim.x * kT) {
    const int i = (int)(e / J), j = (int)(e % J);
    const float *x = X + (int64_t)i * ldx, *w = W + (int64_t)j * ldw;
    float acc = b ? b[j] : 0.0f;
    for (int k = 0; k < K; ++k) acc = fmaf(w[k], x[k], acc);
    float *y = Y + (int64_t)i * ldy + j;
    *y = accumulate ? *y + acc : acc;
  }
}

// Y[i][k] (+)= sum_j W[j][k] X[i][j]   (the transposed product: dX = dY W)
__global__ __launch_bounds__(kT) void k_rowmat_t(const float *__restrict__ X, int ldx, int n, int J,
                                                 const float *__restrict__ W, int ldw, int K, float *__restrict__ Y,
                                                 int ldy, int accumulate) {
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < (int64_t)n * K; e += (int64_t)gridDim.x * kT) {
    const int i = (int)(e / K), k = (int)(e % K);
    const float *x = X + (int64_t)i * ldx;
    float acc = 0.0f;
    for (int j = 0; j < J; ++j) acc = fmaf(W[(int64_t)j * ldw + k], x[j], acc);
    float *y = Y + (int64_t)i * ldy + k;
    *y = accumulate ? *y + acc : acc;
  }
}

// A[i][f] (+)= sum over the CSR row of atom i of S[col][f]; atom ids are local to
// the chunk (0 .. n-1).  A column outside the chunk is reported and skipped.
__global__ __launch_bounds__(kT) void k_agg(const int32_t *__restrict__ rowp, const int32_t *__restrict__ col,
                                            int64_t cap, const float *__restrict__ S, int n, int F,
                                            float *__restrict__ A, int accumulate, int64_t *status) {
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < (int64_t)n * F; e += (int64_t)gridDim.x * kT) {
    const int i = (int)(e / F), f = (int)(e % F);
    int64_t e0 = rowp[i], e1 = rowp[i + 1];
    if (e1 > cap) e1 = cap;
    float acc = 0.0f;
    for (int64_t q = e0; q < e1; ++q) {
      const int j = col[q];
      if (j < 0 || j >= n) {
        if (f == 0) dev_fail(status, kDevBadGraph);
        continue;
      }
      acc += S[(int64_t)j * F + f];
    }
    A[e] = accumulate ? A[e] + acc : acc;
  }
}

__device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

// GRU update from the stacked gate inputs GI = W_ih m + b_ih, GH = W_hh h + b_hh
// (gate rows r, z, n): h' = (1 - z) n + z h
__global__ __launch_bounds__(kT) void k_gru_fwd(const float *__restrict__ GI, const float *__restrict__ GH,
                                                const float *__restrict__ Hin, int n, int H, float *__restrict__ Hout) {
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < (int64_t)n * H; e += (int64_t)gridDim.x * kT) {
    const int64_t i = e / H;
    const int j = (int)(e % H);
    const float *gi = GI + i * 3 * H, *gh = GH + i * 3 * H;
    const float r = sigm(gi[j] + gh[j]), z = sigm(gi[H + j] + gh[H + j]);
    const float nn = tanhf(gi[2 * H + j] + r * gh[2 * H + j]);
    Hout[e] = (1.0f - z) * nn + z * Hin[e];
  }
}

// GRU backward, elementwise: from dh' the gradients of the gate inputs dGI
// (dr_pre, dz_pre, dn_pre), dGH (dr_pre, dz_pre, r dn_pre) and the direct part
// z dh' of dh
__global__ __launch_bounds__(kT) void k_gru_bwd(const float *__restrict__ GI, const float *__restrict__ GH,
                                                const float *__restrict__ Hin, const float *__restrict__ dHout, int n,
                                                int H, float *__restrict__ dGI, float *__restrict__ dGH,
                                                float *__restrict__ dHd) {
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < (int64_t)n * H; e += (int64_t)gridDim.x * kT) {
    const int64_t i = e / H;
    const int j = (int)(e % H);
    const float *gi = GI + i * 3 * H, *gh = GH + i * 3 * H;
    const float r = sigm(gi[j] + gh[j]), z = sigm(gi[H + j] + gh[H + j]);
    const float hn = gh[2 * H + j];
    const float nn = tanhf(gi[2 * H + j] + r * hn);
    const float d = dHout[e], h = Hin[e];
    const float dn = d * (1.0f - z), dz = d * (h - nn);
    const float dpn = dn * (1.0f - nn * nn);
    const float dpr = dpn * hn * r * (1.0f - r), dpz = dz * z * (1.0f - z);
    float *a = dGI + i * 3 * H, *b = dGH + i * 3 * H;
    a[j] = dpr;
    a[H + j] = dpz;
    a[2 * H + j] = dpn;
    b[j] = dpr;
    b[H + j] = dpz;
    b[2 * H + j] = dpn * r;
    dHd[e] = d * z;
  }
}

// readout s[p][j] = sum over the ligand atoms i of pose p (in order) of
// sigma(Gpre[i][j]) * V[i][j]
__global__ __launch_bounds__(kT) void k_readout(const float *__restrict__ Gpre, const float *__restrict__ V,
                                                const uint8_t *__restrict__ is_lig, const int32_t *__restrict__ atom_off,
                                                int p0, int np, int H, float *__restrict__ S) {
  const int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x;
  if (e >= (int64_t)np * H) return;
  const int p = (int)(e / H), j = (int)(e % H);
  const int base = atom_off[p0];
  const int a0 = atom_off[p0 + p], a1 = atom_off[p0 + p + 1];
  float acc = 0.0f;
  for (int a = a0; a < a1; ++a)
    if (is_lig[a]) {
      const int64_t i = (int64_t)(a - base) * H + j;
      acc = fmaf(sigm(Gpre[i]), V[i], acc);
    }
  S[e] = acc;
}

__global__ __launch_bounds__(kT) void k_readout_bwd(const float *__restrict__ Gpre, const float *__restrict__ V,
                                                    const uint8_t *__restrict__ is_lig,
                                                    const int32_t *__restrict__ atom_off, int p0, int np, int H,
                                                    const float *__restrict__ dS, float *__restrict__ dGpre,
                                                    float *__restrict__ dV) {
  const int base = atom_off[p0], n = atom_off[p0 + np] - base;
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < (int64_t)n * H; e += (int64_t)gridDim.x * kT) {
    const int i = (int)(e / H), j = (int)(e % H);
    // pose of atom i: binary search over the chunk's offsets
    int lo = 0, hi = np;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (atom_off[p0 + mid] - base <= i) lo = mid; else hi = mid;
    }
    float dg = 0.0f, dv = 0.0f;
    if (is_lig[base + i]) {
      const float g = sigm(Gpre[e]), ds = dS[(int64_t)lo * H + j];
      dg = ds * V[e] * g * (1.0f - g);
      dv = ds * g;
    }
    dGpre[e] = dg;
    dV[e] = dv;
  }
}

// C[a][b] (+)= sum_{i < n} U[i][a] V[i][b] (V = null: the column sums of U).
// Pass 1: chunk s of kRowsPerChunk rows -> partial[s][a][b]; pass 2 adds the
// partials in chunk order.
constexpr int kRowsPerChunk = 128;

__global__ __launch_bounds__(kT) void k_outer_partial(const float *__restrict__ U, int ldu,
                                                      const float *__restrict__ V, int ldv, int n, int A, int B,
                                                      float *__restrict__ part) {
  const int64_t ab = (int64_t)A * B;
  const int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x;
  const int s = blockIdx.y;
  if (e >= ab) return;
  const int a = (int)(e / B), b = (int)(e % B);
  const int i0 = s * kRowsPerChunk, i1 = min(n, i0 + kRowsPerChunk);
  float acc = 0.0f;
  for (int i = i0; i < i1; ++i) acc = fmaf(U[(int64_t)i * ldu + a], V ? V[(int64_t)i * ldv + b] : 1.0f, acc);
  part[(int64_t)s * ab + e] = acc;
}

__global__ __launch_bounds__(kT) void k_outer_sum(const float *__restrict__ part, int nchunk, int A, int B,
                                                  float *__restrict__ C, int ldc, int accumulate) {
  const int64_t ab = (int64_t)A * B;
  const int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x;
  if (e >= ab) return;
  float acc = 0.0f;
  for (int s = 0; s < nchunk; ++s) acc += part[(int64_t)s * ab + e];
  float *c = C + (e / B) * ldc + (e % B);
  *c = accumulate ? *c + acc : acc;
}

// ---- 3D-CNN ----

// pool[p][c] = mean over the voxels of act[p][v][c] (voxels in order)
__global__ __launch_bounds__(kT) void k_pool_mean(const float *__restrict__ act, int np, int64_t vox, int cstride,
                                                  int C, float *__restrict__ pool) {
  const int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x;
  if (e >= (int64_t)np * C) return;
  const int p = (int)(e / C), c = (int)(e % C);
  const float *a = act + (int64_t)p * vox * cstride + c;
  float acc = 0.0f;
  for (int64_t v = 0; v < vox; ++v) acc += a[v * cstride];
  pool[e] = acc / (float)vox;
}

// dact[p][v][c] = dpool[p][c] / vox (channels past C zero)
__global__ __launch_bounds__(kT) void k_pool_seed(const float *__restrict__ dpool, int np, int64_t vox, int cstride,
                                                  int C, float *__restrict__ dact) {
  const int64_t n = (int64_t)np * vox * cstride;
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    const int c = (int)(e % cstride);
    const int64_t p = e / (vox * cstride);
    dact[e] = c < C ? dpool[p * C + c] / (float)vox : 0.0f;
  }
}

// d *= (y > 0): the ReLU's gradient from its output (y = max(u, 0))
__global__ __launch_bounds__(kT) void k_relu_mask(float *__restrict__ d, const float *__restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    d[i] = y[i] > 0.0f ? d[i] : 0.0f;
}

// d *= (y > 0) for rows of width J laid out with stride ld
__global__ __launch_bounds__(kT) void k_relu_rows(float *__restrict__ y, int n, int J, int ld) {
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < (int64_t)n * J; e += (int64_t)gridDim.x * kT) {
    float *p = y + (e / J) * ld + (e % J);
    *p = *p > 0.0f ? *p : 0.0f;
  }
}

__global__ __launch_bounds__(kT) void k_relu_grad_rows(float *__restrict__ d, const float *__restrict__ pre, int n,
                                                       int J) {
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < (int64_t)n * J; e += (int64_t)gridDim.x * kT)
    d[e] = pre[e] > 0.0f ? d[e] : 0.0f;
}

// Folded weights transposed for the data gradient: WT[t][co][ci] = W[co][ci][t] * a[co],
// a = gamma / sqrt(var + eps) with BatchNorm, else 1.
__global__ __launch_bounds__(kT) void k_fold_wt(const float *__restrict__ W, const float *__restrict__ gamma,
                                                const float *__restrict__ var, int cout, int cin, int taps,
                                                float *__restrict__ WT) {
  const int64_t n = (int64_t)cout * cin * taps;
  for (int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    const int t = (int)(e % taps), ci = (int)((e / taps) % cin), co = (int)(e / ((int64_t)taps * cin));
    const float a = gamma ? (float)((double)gamma[co] / sqrt((double)var[co] + 1e-5)) : 1.0f;
    WT[((int64_t)t * cout + co) * cin + ci] = W[e] * a;
  }
}

// Weight gradient of one conv layer w.r.t. its folded weights, per pose:
//   part[p][co][t * cin + ci] = sum_o dY[p][o][co] * X[p][s o + t - P][ci]
// Workgroup: 32 output channels x 64 (tap, channel) columns of pose p; 16 output
// voxels per step, both operands staged in LDS; 8 accumulators per thread.
__global__ __launch_bounds__(kT) void k_conv_wgrad(const float *__restrict__ X, int D, int xstride, int cin,
                                                   const float *__restrict__ dY, int Do, int ystride, int cout,
                                                   int KS, int S, float *__restrict__ part) {
  __shared__ float sa[16][33];
  __shared__ float sb[16][65];
  const int q0 = blockIdx.x * 64, c0 = blockIdx.y * 32, p = blockIdx.z;
  const int taps = KS * KS * KS, Q = taps * cin, P = (KS - 1) / 2;
  const int tid = threadIdx.x;
  const int tc = tid / 16, tq = tid % 16;  // thread: channels c0 + 2 tc + {0, 1}, columns q0 + tq + 16 {0..3}
  float acc[2][4] = {};
  const int64_t vo = (int64_t)Do * Do * Do;
  const float *xp = X + (int64_t)p * D * D * D * xstride;
  const float *yp = dY + (int64_t)p * vo * ystride;
  for (int64_t o0 = 0; o0 < vo; o0 += 16) {
    // A: dY[o0 + r][c0 + c], r < 16, c < 32
    for (int e = tid; e < 16 * 32; e += kT) {
      const int r = e / 32, c = e % 32;
      const int64_t o = o0 + r;
      sa[r][c] = (o < vo && c0 + c < cout) ? yp[o * ystride + c0 + c] : 0.0f;
    }
    // B: X at s o + t - P, r < 16, column q = t * cin + ci
    for (int e = tid; e < 16 * 64; e += kT) {
      const int r = e / 64, qq = e % 64, q = q0 + qq;
      const int64_t o = o0 + r;
      float v = 0.0f;
      if (o < vo && q < Q) {
        const int t = q / cin, ci = q % cin;
        const int tz = t / (KS * KS), ty = (t / KS) % KS, tx = t % KS;
        const int oz = (int)(o / (Do * Do)), oy = (int)((o / Do) % Do), ox = (int)(o % Do);
        const int z = S * oz + tz - P, y = S * oy + ty - P, x = S * ox + tx - P;
        if (z >= 0 && z < D && y >= 0 && y < D && x >= 0 && x < D)
          v = xp[(((int64_t)z * D + y) * D + x) * xstride + ci];
      }
      sb[r][qq] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float a0 = sa[r][2 * tc], a1 = sa[r][2 * tc + 1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float b = sb[r][tq + 16 * u];
        acc[0][u] = fmaf(a0, b, acc[0][u]);
        acc[1][u] = fmaf(a1, b, acc[1][u]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int co = c0 + 2 * tc + h, q = q0 + tq + 16 * u;
      if (co < cout && q < Q) part[((int64_t)p * cout + co) * Q + q] = acc[h][u];
    }
}

// Data gradient of one conv layer (the transposed conv as a gather):
//   dX[p][v][ci] += sum_{t, co} dY[p][o][co] * WT[t][co][ci],  s o = v + P - t
// for the output voxels o (per axis) a tap reaches.  Workgroup: 64 input voxels
// x 64 channels of pose p; per tap, 16-channel steps of co staged in LDS.
__global__ __launch_bounds__(kT) void k_conv_dgrad(const float *__restrict__ dY, int Do, int ystride, int cout,
                                                   const float *__restrict__ WT, int cin, int KS, int S, int D,
                                                   int xstride, float *__restrict__ dX) {
  __shared__ float sa[64][17];
  __shared__ float sb[16][65];
  const int v0 = blockIdx.x * 64, ci0 = blockIdx.y * 64, p = blockIdx.z;
  const int taps = KS * KS * KS, P = (KS - 1) / 2;
  const int tid = threadIdx.x;
  const int tv = tid / 16, tcc = tid % 16;  // voxels v0 + 4 tv + {0..3}, channels ci0 + tcc + 16 {0..3}
  const int64_t vin = (int64_t)D * D * D, vo = (int64_t)Do * Do * Do;
  const float *yp = dY + (int64_t)p * vo * ystride;
  float acc[4][4] = {};
  for (int t = 0; t < taps; ++t) {
    const int tz = t / (KS * KS), ty = (t / KS) % KS, tx = t % KS;
    for (int c0 = 0; c0 < cout; c0 += 16) {
      for (int e = tid; e < 64 * 16; e += kT) {
        const int r = e / 16, c = e % 16;
        const int64_t v = v0 + r;
        float val = 0.0f;
        if (v < vin && c0 + c < cout) {
          const int z = (int)(v / (D * D)), y = (int)((v / D) % D), x = (int)(v % D);
          const int nz = z + P - tz, ny = y + P - ty, nx = x + P - tx;
          if (nz >= 0 && ny >= 0 && nx >= 0 && nz % S == 0 && ny % S == 0 && nx % S == 0) {
            const int oz = nz / S, oy = ny / S, ox = nx / S;
            if (oz < Do && oy < Do && ox < Do) val = yp[(((int64_t)oz * Do + oy) * Do + ox) * ystride + c0 + c];
          }
        }
        sa[r][c] = val;
      }
      for (int e = tid; e < 16 * 64; e += kT) {
        const int c = e / 64, cc = e % 64;
        sb[c][cc] = (c0 + c < cout && ci0 + cc < cin) ? WT[((int64_t)t * cout + c0 + c) * cin + ci0 + cc] : 0.0f;
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        float b[4], a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) b[u] = sb[c][tcc + 16 * u];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = sa[4 * tv + r][c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[r][u] = fmaf(a[r], b[u], acc[r][u]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t v = v0 + 4 * tv + r;
      const int ci = ci0 + tcc + 16 * u;
      if (v < vin && ci < cin) dX[((int64_t)p * vin + v) * xstride + ci] += acc[r][u];
    }
}

// Folded-weight gradients -> gradients of the blob's parameters, one workgroup
// per output channel co.  Folding: W' = a W, b' = a (b - mu) + beta with
// a = gamma / sqrt(var + eps) (without BatchNorm: a = 1, b' = b).  So
//   dW = a dW', db = a db', dbeta = db', dmean = -a db',
//   dgamma = g_a / sqrt(var + eps), dvar = -g_a a / (2 (var + eps)),
// with g_a = sum dW' W + db' (b - mu).  dWf: [co][t][ci]; blob W: [co][ci][t].
__global__ __launch_bounds__(kT) void k_fold_grad(const float *__restrict__ dWf, const float *__restrict__ dbf,
                                                  const float *__restrict__ W, const float *__restrict__ b,
                                                  const float *__restrict__ gamma, const float *__restrict__ mean,
                                                  const float *__restrict__ var, int cin, int taps,
                                                  float *__restrict__ gW, float *__restrict__ gb,
                                                  float *__restrict__ ggamma, float *__restrict__ gbeta,
                                                  float *__restrict__ gmean, float *__restrict__ gvar) {
  __shared__ double red[kT];
  const int co = blockIdx.x, tid = threadIdx.x;
  const double a = gamma ? (double)gamma[co] / sqrt((double)var[co] + 1e-5) : 1.0;
  const int64_t n = (int64_t)cin * taps;
  double ga = 0.0;
  for (int64_t e = tid; e < n; e += kT) {
    const int ci = (int)(e / taps), t = (int)(e % taps);
    const float d = dWf[((int64_t)co * taps + t) * cin + ci];
    const int64_t wi = (int64_t)co * n + e;
    ga += (double)d * (double)W[wi];
    gW[wi] += (float)(a * (double)d);
  }
  red[tid] = ga;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    const double db = dbf[co];
    gb[co] += (float)(a * db);
    if (gamma) {
      const double ve = (double)var[co] + 1e-5;
      const double g_a = red[0] + db * ((double)b[co] - (double)mean[co]);
      ggamma[co] += (float)(g_a / sqrt(ve));
      gbeta[co] += (float)db;
      gmean[co] += (float)(-a * db);
      gvar[co] += (float)(-g_a * a / (2.0 * ve));
    }
  }
}

// ---- Coherent Fusion head ----

__device__ inline float selu_f(float x) {
  constexpr float kL = 1.0507009873554805f, kA = 1.6732632423543772f;
  return x > 0.0f ? kL * x : kL * kA * expm1f(x);
}
__device__ inline float selu_d(float x) {
  constexpr float kL = 1.0507009873554805f, kA = 1.6732632423543772f;
  return x > 0.0f ? kL : kL * kA * expf(x);
}

// One workgroup per pose: the fusion block's forward (z_0 = [cnn; sg], hidden SELU
// layers, optionally residual after the first, linear output) and its backward
// from dscore.  Per-pose parameter gradients go to part[p][...] in the blob order
// of the head; dcnn / dsg are the latents' gradients.  prm: the head's blob
// parameters.
constexpr int kHeadMaxW = 512;

__global__ __launch_bounds__(kT) void k_head_bwd(const float *__restrict__ cnn, int lc, const float *__restrict__ sg,
                                                 int sgw, const float *__restrict__ prm, int nhid, int fh,
                                                 int residual, const float *__restrict__ dscore,
                                                 float *__restrict__ scores, float *__restrict__ dcnn,
                                                 float *__restrict__ dsg, float *__restrict__ part, int64_t nprm) {
  __shared__ float z[9][kHeadMaxW];    // z_0 .. z_nhid
  __shared__ float pre[8][kHeadMaxW];  // hidden pre-activations
  __shared__ float dz[2][kHeadMaxW];
  __shared__ float red[kT];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int fin = lc + sgw;
  for (int k = tid; k < fin; k += kT) z[0][k] = k < lc ? cnn[(int64_t)p * lc + k] : sg[(int64_t)p * sgw + k - lc];
  __syncthreads();
  // forward
  int64_t off = 0;
  int w = fin;
  for (int l = 0; l < nhid; ++l) {
    const float *W = prm + off, *b = prm + off + (int64_t)fh * w;
    for (int j = tid; j < fh; j += kT) {
      float acc = b[j];
      for (int k = 0; k < w; ++k) acc = fmaf(W[(int64_t)j * w + k], z[l][k], acc);
      pre[l][j] = acc;
      const float y = selu_f(acc);
      z[l + 1][j] = (residual && l > 0) ? y + z[l][j] : y;
    }
    __syncthreads();
    off += (int64_t)fh * w + fh;
    w = fh;
  }
  const float *Wo = prm + off;
  float acc = 0.0f;
  for (int k = tid; k < w; k += kT) acc = fmaf(Wo[k], z[nhid][k], acc);
  red[tid] = acc;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const float g = dscore[p];
  float *pp = part + (int64_t)p * nprm;
  if (tid == 0) {
    if (scores) scores[p] = red[0] + Wo[w];
    pp[off + w] = g;  // d b_out
  }
  for (int k = tid; k < w; k += kT) {
    pp[off + k] = g * z[nhid][k];  // d W_out
    dz[nhid & 1][k] = g * Wo[k];
  }
  __syncthreads();
  // backward through the hidden layers
  for (int l = nhid - 1; l >= 0; --l) {
    const int wi = l == 0 ? fin : fh;
    off -= (int64_t)fh * wi + fh;
    const float *W = prm + off;
    const int cur = (l + 1) & 1, nxt = l & 1;
    for (int j = tid; j < fh; j += kT) {
      const float dp = dz[cur][j] * selu_d(pre[l][j]);
      pp[off + (int64_t)fh * wi + j] = dp;  // d b
      pre[l][j] = dp;                       // reuse: dpre
    }
    __syncthreads();
    for (int e = tid; e < fh * wi; e += kT) pp[off + e] = pre[l][e / wi] * z[l][e % wi];  // d W
    for (int k = tid; k < wi; k += kT) {
      float s = 0.0f;
      for (int j = 0; j < fh; ++j) s = fmaf(W[(int64_t)j * wi + k], pre[l][j], s);
      dz[nxt][k] = (residual && l > 0) ? s + dz[cur][k] : s;
    }
    __syncthreads();
  }
  for (int k = tid; k < fin; k += kT) {
    const float d = dz[0][k];
    if (k < lc) dcnn[(int64_t)p * lc + k] = d; else dsg[(int64_t)p * sgw + k - lc] = d;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t bw_fill(float *p, int64_t n, float v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill, grid1(n), dim3(kT), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t bw_add(float *dst, const float *src, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_add, grid1(n), dim3(kT), 0, s, dst, src, n);
  return hipGetLastError();
}
hipError_t bw_rowmat(const float *X, int ldx, int n, int K, const float *W, int ldw, const float *b, int J, float *Y,
                     int ldy, int accumulate, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_rowmat, grid1((int64_t)n * J), dim3(kT), 0, s, X, ldx, n, K, W, ldw, b, J, Y, ldy, accumulate);
  return hipGetLastError();
}
hipError_t bw_rowmat_t(const float *X, int ldx, int n, int J, const float *W, int ldw, int K, float *Y, int ldy,
                       int accumulate, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_rowmat_t, grid1((int64_t)n * K), dim3(kT), 0, s, X, ldx, n, J, W, ldw, K, Y, ldy, accumulate);
  return hipGetLastError();
}
hipError_t bw_agg(const int32_t *rowp, const int32_t *col, int64_t cap, const float *S, int n, int F, float *A,
                  int accumulate, int64_t *status, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_agg, grid1((int64_t)n * F), dim3(kT), 0, s, rowp, col, cap, S, n, F, A, accumulate, status);
  return hipGetLastError();
}
hipError_t bw_gru_fwd(const float *GI, const float *GH, const float *Hin, int n, int H, float *Hout, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gru_fwd, grid1((int64_t)n * H), dim3(kT), 0, s, GI, GH, Hin, n, H, Hout);
  return hipGetLastError();
}
hipError_t bw_gru_bwd(const float *GI, const float *GH, const float *Hin, const float *dHout, int n, int H, float *dGI,
                      float *dGH, float *dHd, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gru_bwd, grid1((int64_t)n * H), dim3(kT), 0, s, GI, GH, Hin, dHout, n, H, dGI, dGH, dHd);
  return hipGetLastError();
}
hipError_t bw_readout(const float *Gpre, const float *V, const uint8_t *is_lig, const int32_t *atom_off, int p0,
                      int np, int H, float *S, hipStream_t s) {
  hipLaunchKernelGGL(k_readout, grid1((int64_t)np * H), dim3(kT), 0, s, Gpre, V, is_lig, atom_off, p0, np, H, S);
  return hipGetLastError();
}
hipError_t bw_readout_bwd(const float *Gpre, const float *V, const uint8_t *is_lig, const int32_t *atom_off, int p0,
                          int np, int H, int n_atoms, const float *dS, float *dGpre, float *dV, hipStream_t s) {
  if (n_atoms > 0)
    hipLaunchKernelGGL(k_readout_bwd, grid1((int64_t)n_atoms * H), dim3(kT), 0, s, Gpre, V, is_lig, atom_off, p0, np, H,
                       dS, dGpre, dV);
  return hipGetLastError();
}
int64_t bw_outer_scratch(int n, int A, int B) {
  return (int64_t)std::max(1, (n + kRowsPerChunk - 1) / kRowsPerChunk) * A * B;
}
hipError_t bw_outer(const float *U, int ldu, const float *V, int ldv, int n, int A, int B, float *C, int ldc,
                    int accumulate, float *part, hipStream_t s) {
  const int nchunk = std::max(1, (n + kRowsPerChunk - 1) / kRowsPerChunk);
  const int64_t ab = (int64_t)A * B;
  if (n > 0)
    hipLaunchKernelGGL(k_outer_partial, dim3((unsigned)((ab + kT - 1) / kT), nchunk), dim3(kT), 0, s, U, ldu, V, ldv,
                       n, A, B, part);
  else
    hipLaunchKernelGGL(k_fill, grid1(ab), dim3(kT), 0, s, part, ab, 0.0f);
  hipLaunchKernelGGL(k_outer_sum, dim3((unsigned)((ab + kT - 1) / kT)), dim3(kT), 0, s, part, n > 0 ? nchunk : 1, A, B,
                     C, ldc, accumulate);
  return hipGetLastError();
}
hipError_t bw_pool_mean(const float *act, int np, int64_t vox, int cstride, int C, float *pool, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_mean, grid1((int64_t)np * C), dim3(kT), 0, s, act, np, vox, cstride, C, pool);
  return hipGetLastError();
}
hipError_t bw_pool_seed(const float *dpool, int np, int64_t vox, int cstride, int C, float *dact, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_seed, grid1((int64_t)np * vox * cstride), dim3(kT), 0, s, dpool, np, vox, cstride, C, dact);
  return hipGetLastError();
}
hipError_t bw_relu_mask(float *d, const float *y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_relu_mask, grid1(n), dim3(kT), 0, s, d, y, n);
  return hipGetLastError();
}
hipError_t bw_relu_rows(float *y, int n, int J, int ld, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_relu_rows, grid1((int64_t)n * J), dim3(kT), 0, s, y, n, J, ld);
  return hipGetLastError();
}
hipError_t bw_relu_grad_rows(float *d, const float *pre, int n, int J, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_relu_grad_rows, grid1((int64_t)n * J), dim3(kT), 0, s, d, pre, n, J);
  return hipGetLastError();
}
hipError_t bw_fold_wt(const float *W, const float *gamma, const float *var, int cout, int cin, int taps, float *WT,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_fold_wt, grid1((int64_t)cout * cin * taps), dim3(kT), 0, s, W, gamma, var, cout, cin, taps, WT);
  return hipGetLastError();
}
hipError_t bw_conv_wgrad(const float *X, int D, int xstride, int cin, const float *dY, int Do, int ystride, int cout,
                         int KS, int S, int np, float *part, hipStream_t s) {
  const int Q = KS * KS * KS * cin;
  hipLaunchKernelGGL(k_conv_wgrad, dim3((Q + 63) / 64, (cout + 31) / 32, np), dim3(kT), 0, s, X, D, xstride, cin, dY,
                     Do, ystride, cout, KS, S, part);
  return hipGetLastError();
}
hipError_t bw_conv_dgrad(const float *dY, int Do, int ystride, int cout, const float *WT, int cin, int KS, int S, int D,
                         int xstride, int np, float *dX, hipStream_t s) {
  const int64_t vin = (int64_t)D * D * D;
  hipLaunchKernelGGL(k_conv_dgrad, dim3((unsigned)((vin + 63) / 64), (cin + 63) / 64, np), dim3(kT), 0, s, dY, Do,
                     ystride, cout, WT, cin, KS, S, D, xstride, dX);
  return hipGetLastError();
}
hipError_t bw_fold_grad(const float *dWf, const float *dbf, const float *W, const float *b, const float *gamma,
                        const float *mean, const float *var, int cout, int cin, int taps, float *gW, float *gb,
                        float *ggamma, float *gbeta, float *gmean, float *gvar, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_grad, dim3(cout), dim3(kT), 0, s, dWf, dbf, W, b, gamma, mean, var, cin, taps, gW, gb,
                     ggamma, gbeta, gmean, gvar);
  return hipGetLastError();
}
bool bw_head_ok(int fin, int fh, int nhid) { return fin <= kHeadMaxW && fh <= kHeadMaxW && nhid <= 8; }
hipError_t bw_head(const float *cnn, int lc, const float *sg, int sgw, const float *prm, int nhid, int fh, int residual,
                   const float *dscore, int np, float *scores, float *dcnn, float *dsg, float *part, int64_t nprm,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_head_bwd, dim3(np), dim3(kT), 0, s, cnn, lc, sg, sgw, prm, nhid, fh, residual, dscore, scores,
                     dcnn, dsg, part, nprm);
  return hipGetLastError();
}

}  // namespace cf
