// Stride-1 conv3d in the frequency domain of the two in-plane axes.
//
// The 3D-CNN (Sec. 3.3.1, Table III) applies cross-correlations with k^3 kernels
// and zero "same" padding.  For a stride-1 layer on a D^3 grid with D + k - 1 <= 32
// the (y, x) part of the correlation is exact as a product of 32 x 32 DFTs (the
// zero padding of the DFT covers the conv padding, so no wrap-around reaches an
// output), which leaves a k-tap correlation along z per (ky, kx) frequency:
//
//   Y[ky,kx](z, co) = sum_{dz, ci} X[ky,kx](z + dz - p, ci) G[ky,kx](dz, ci, co)
//   G[ky,kx](dz, ci, co) = sum_{dy,dx} W(co, ci, dz, dy, dx) e^{+2 pi i ((dy-p) ky + (dx-p) kx) / 32}
//
// with X the forward DFT of the input plane z and y = inverse DFT of Y.  Real
// inputs give Hermitian spectra, so kx runs over 0..16 only (544 columns).  The
// z-correlation is a complex GEMM per column (rows = (pose, z), K = (dz, ci),
// N = (re, im) x co) and runs on the bf16 MFMAs; the FFTs are HBM-bound streams.
// Per layer and pose the work drops from 2 k^3 cin cout D^3 FLOP to
// 8 k cin cout D 544 + O(D^2 log) -- 12x fewer at k = 7, D = 24.
//
// Three kernels per layer:
//   k_fft_fwd2d  one (pose, z, 8-channel chunk) plane: 2-D real FFT -> spectrum rows
//   k_fft_zconv  one (column, block of poses): the z-correlation on MFMAs
//   k_fft_inv2d  one (pose, z, 8-channel chunk) plane: inverse FFT, bias, residual,
//                ReLU, bf16 store in the activations' channels-last layout
// and, between two such layers, k_fft_mid: one layer's inverse and the next one's
// forward transform of the same plane.  Overlap-save tiles of 32^3 activations
// (64^3 grids) have their own forward (k_fft_fwd2d_t, which reads the tile's window);
// k_fft_inv2d takes them as tiles of its plane.
//
// Spectrum layout (bf16): [col][pose][z][chunk][re | im][8 channels] -- 64 bytes
// per 8 channels, so a (column, pose block) of the z-correlation is one
// contiguous run of rows, and one MFMA K step (16 deep) is 8 channels x (re, im).
#include <type_traits>

#include "cf_internal.h"
#include "cf_fft32.h"

namespace cf {

namespace {

constexpr int kN = 32, kNX = kN / 2 + 1, kCols = kN * kNX;  // 544 (ky, kx) columns
constexpr int kDMax = 30;                                      // D + k - 1 <= 32, k >= 3
constexpr int kRowsZ = 192;                                    // (pose, z) rows per z-correlation block
constexpr int kPanelRows = 288;                                // LDS rows of one block incl. z halo

// ---------------------------------------------------------------- plane transforms

// Thread roles in the plane kernels (256 threads): each 32-point FFT is shared by
// two adjacent lanes (see the lane-pair section below); the column transforms along
// ky / y run on all 256 threads, a lane pair per (kxp, channel), and the row
// transforms along x on threads 0 .. 8 D - 1 (8 W for a tile's window), a pair per
// (y, two channels).
//
// Columns: kxp 1 .. 15 is the complex column kx = kxp; kxp 0 carries the DC and
// Nyquist columns (kx 0 and 16) together.  Along y both are real sequences (the
// row transform of real data is real at kx 0 and 16), so they travel as the real
// and imaginary parts of one complex column t0 + i t16, which the row kernels
// read and write in place of column 0 (column 16 of T stays unused).  Forward:
// Z = FFT(t0 + i t16), X0[k] = (Z[k] + conj Z[-k]) / 2, X16[k] = (Z[k] - conj
// Z[-k]) / 2i, split by all threads from Z staged in fp32 (Zp).  Inverse: all
// threads first form Zp = H(Y0) + i H(Y16) from the spectrum, H the Hermitian part
// (H(Y)[k] = (Y[k] + conj Y[-k]) / 2); its inverse is Re IFFT(Y0) + i Re IFFT(Y16),
// the real parts that the row transform takes.
//
// The plane kernels take the grid edge as a template argument DT (0: D_rt at run
// time): with D a constant, the bounds tests inside the unrolled transforms fold
// away instead of turning into register-copy blocks.
// LDS of the plane kernels: the plane region (the larger of the row spectra
// [17][D + 1][8] complex and the spectrum of a plane, bf16 or fp32), then Zp
// [32][8] complex
__host__ __device__ constexpr int plane_lds_bytes(int D, bool f32 = false) {
  return kNX * (D + 1) * 8 * 8 > kCols * 16 * (f32 ? 4 : 2) ? kNX * (D + 1) * 8 * 8 : kCols * 16 * (f32 ? 4 : 2);
}
constexpr int kZpBytes = 32 * 8 * 8;

typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
// two floats rounded to bf16 (nearest even) by one conversion, lo in the low half
__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  const float2v two = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(two, bf16x2v));
}

// One complex value of channel c from a spectrum row [col][re | im][8]: fp32
// directly; bf16 from the two 32-bit words that hold the re and the im of the
// channel pair (c & ~1, c | 1), channel c being the low (even c) or the high half
// of each: a byte permute moves that half to the top of a float (one instruction
// per value, no exchange with the other channel's lane).
template <bool F32>
__device__ inline void spec_get(const void *Y, int col, int c, float &r, float &i) {
  if constexpr (F32) {
    const float *Yf = reinterpret_cast<const float *>(Y);
    r = Yf[col * 16 + c];
    i = Yf[col * 16 + 8 + c];
    return;
  }
  const uint32_t *Yw = reinterpret_cast<const uint32_t *>(Y);
  const uint32_t wr = Yw[col * 8 + (c >> 1)], wi = Yw[col * 8 + 4 + (c >> 1)];
  const uint32_t sel = (c & 1) ? 0x03020c0cu : 0x01000c0cu;  // 0x0c: a zero byte
  r = __uint_as_float(__builtin_amdgcn_perm(wr, wr, sel));
  i = __uint_as_float(__builtin_amdgcn_perm(wi, wi, sel));
}

// The inverse of spec_get: fp32 directly; bf16 as the two 16-bit halves of one
// rounding of (r, i), stored into the re and the im word of the channel pair.
template <bool F32>
__device__ inline void spec_put(void *Ov, int col, int c, float r, float i) {
  if constexpr (F32) {
    float *Of = reinterpret_cast<float *>(Ov);
    Of[col * 16 + c] = r;
    Of[col * 16 + 8 + c] = i;
    return;
  }
  uint16_t *O = reinterpret_cast<uint16_t *>(Ov);
  const uint32_t two = pack_bf16x2(r, i);
  O[(col * 8 + (c >> 1)) * 2 + (c & 1)] = (uint16_t)two;
  O[(col * 8 + 4 + (c >> 1)) * 2 + (c & 1)] = (uint16_t)(two >> 16);
}

// inverse, all 256 threads (ky = tid >> 3, c = tid & 7): Zp[ky][c] = H(Y0)[ky] + i H(Y16)[ky]
template <bool F32>
__device__ inline void dc_nyquist_pack(const void *Y, float2 *Zp, int tid) {
  const int ky = tid >> 3, c = tid & 7, m = (32 - ky) & 31;
  float ar, ai, br, bi, cr, ci, dr, di;
  spec_get<F32>(Y, ky * kNX, c, ar, ai);               // Y0[ky]
  spec_get<F32>(Y, m * kNX, c, br, bi);                // Y0[-ky]
  spec_get<F32>(Y, ky * kNX + kNX - 1, c, cr, ci);     // Y16[ky]
  spec_get<F32>(Y, m * kNX + kNX - 1, c, dr, di);      // Y16[-ky]
  const float h0r = 0.5f * (ar + br), h0i = 0.5f * (ai - bi);
  const float h1r = 0.5f * (cr + dr), h1i = 0.5f * (ci - di);
  Zp[ky * 8 + c] = make_float2(h0r - h1i, h0i + h1r);
}

// forward, all 256 threads: X0 and X16 at ky from Zp (the transform of t0 + i t16)
template <bool F32>
__device__ inline void dc_nyquist_split(const float2 *Zp, void *O, int tid) {
  const int ky = tid >> 3, c = tid & 7, m = (32 - ky) & 31;
  const float2 a = Zp[ky * 8 + c], b = Zp[m * 8 + c];
  spec_put<F32>(O, ky * kNX, c, 0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
  spec_put<F32>(O, ky * kNX + kNX - 1, c, 0.5f * (a.y + b.y), -0.5f * (a.x - b.x));
}

// ---------------------------------------------------------------- lane-pair transforms
//
// Every 32-point FFT of the plane kernels is shared by two adjacent lanes
// (fft32_pair_dit / fft32_pair_dif): the column phases run on all 256 threads
// (128 (column, channel) pairs) and the row phase on 8 D threads, each lane
// holding 16 points instead of 32, so that all four waves work in every phase and
// the register file holds half the transform state (at 24^3: 118 VGPRs for the
// fused transform against 153 with one transform per lane, four waves per SIMD
// instead of three).  Lane h = tid & 1 of a pair, partner tid ^ 1 (a quad
// permutation, so the exchange is a DPP move).

__device__ inline float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // lanes 1,0,3,2
}

// inverse columns, decimation in time: lane h takes ky = 2n + h (columns 1 .. 15
// from the spectrum; the packed DC / Nyquist column from Zp)
template <bool F32>
__device__ inline void col_inv_load2(const void *Y, int kxp, int c, int h, float (&re)[16], float (&im)[16]) {
#pragma unroll
  for (int n = 0; n < 16; ++n) spec_get<F32>(Y, (2 * n + h) * kNX + kxp, c, re[n], im[n]);
}
__device__ inline void col_inv_load_dc2(const float2 *Zp, int c, int h, float (&re)[16], float (&im)[16]) {
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    const float2 v = Zp[(2 * n + h) * 8 + c];
    re[n] = v.x;
    im[n] = v.y;
  }
}
// after fft32_pair_dit<true>: lane h holds y = 16 h + k; rows y < D of T
__device__ inline void col_inv_store2(float2 *T, int kxp, int c, int h, int D, const float (&re)[16],
                                      const float (&im)[16]) {
  const int DP = D + 1;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (16 * h + k < D) T[(kxp * DP + 16 * h + k) * 8 + c] = make_float2(re[k], im[k]);
}
// rows, inverse: lane h takes Z[2n + h] of the complex sequence A + i B of the two
// channels' Hermitian halves (Z[0], Z[16] from the packed column)
__device__ inline void row_inv_load2(const float2 *T, int y, int c0, int h, int D, float (&re)[16], float (&im)[16]) {
  const int DP = D + 1;
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    const int k = 2 * n + h;
    if (k == 0 || k == 16) {
      const float4 dc = *reinterpret_cast<const float4 *>(T + y * 8 + c0);  // A0, A16, B0, B16
      re[n] = k ? dc.y : dc.x;
      im[n] = k ? dc.w : dc.z;
    } else if (k < 16) {
      const float4 ab = *reinterpret_cast<const float4 *>(T + (k * DP + y) * 8 + c0);
      re[n] = ab.x - ab.w;
      im[n] = ab.y + ab.z;
    } else {
      const float4 ab = *reinterpret_cast<const float4 *>(T + ((32 - k) * DP + y) * 8 + c0);
      re[n] = ab.x + ab.w;
      im[n] = ab.z - ab.y;
    }
  }
}
// rows, forward, after fft32_pair_dif<false> (lane h holds X[2m + h]): the row
// spectra of the two channels at the frequencies of this lane's parity
__device__ inline void row_fwd_store2(float2 *T, int y, int c0, int h, int D, const float (&re)[16],
                                      const float (&im)[16]) {
  const int DP = D + 1;
  if (!h) *reinterpret_cast<float4 *>(T + y * 8 + c0) = make_float4(re[0], re[8], im[0], im[8]);
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int k = 2 * m + h;  // 1 .. 15 (k = 0 is the packed column)
    if (k == 0) continue;
    const int j = 16 - m - h;  // index of X[32 - k] in this lane
    *reinterpret_cast<float4 *>(T + (k * DP + y) * 8 + c0) =
        make_float4(0.5f * (re[m] + re[j]), 0.5f * (im[m] - im[j]), 0.5f * (im[m] + im[j]), -0.5f * (re[m] - re[j]));
  }
}
// forward columns, decimation in frequency: lane h takes y = 16 h + n (zero past D)
__device__ inline void col_fwd_load2(const float2 *T, int kxp, int c, int h, int D, float (&re)[16], float (&im)[16]) {
  const int DP = D + 1;
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    const int y = 16 * h + n;
    const float2 v = y < D ? T[(kxp * DP + y) * 8 + c] : make_float2(0.0f, 0.0f);
    re[n] = v.x;
    im[n] = v.y;
  }
}
// after fft32_pair_dif<false>: lane h holds ky = 2m + h of column kxp (spectrum), or
// of the packed column (Zp)
template <bool F32>
__device__ inline void col_fwd_store2(void *O, float2 *Zp, int kxp, int c, int h, const float (&re)[16],
                                      const float (&im)[16]) {
  if (kxp) {
#pragma unroll
    for (int m = 0; m < 16; ++m) spec_put<F32>(O, (2 * m + h) * kNX + kxp, c, re[m], im[m]);
  } else {
#pragma unroll
    for (int m = 0; m < 16; ++m) Zp[(2 * m + h) * 8 + c] = make_float2(re[m], im[m]);
  }
}

// ---------------------------------------------------------------- forward


// Overlap-save forward transform for grids of edge 2 TS beyond the 32-point
// transforms' reach (D + k - 1 > 32): each plane is 2 x 2 tiles of TS x TS outputs.
// A tile's input window spans TS + 2P positions per axis, from its origin - P:
// window position w holds array position (w - P) mod 32 (the left halo wraps to
// 32 - P .. 31), so the circular correlation of the 32-point DFTs gives the tile's
// outputs at array positions 0 .. TS - 1 exactly (TS + 2P <= 32).  One workgroup
// per (z, pose and tile, chunk), grid (2 TS, 4 np, nch); spectrum rows are indexed
// by (pose, tile) planes, so the z-correlation runs on them unchanged.
template <int KS, bool F32, int TS>
__global__ __launch_bounds__(256) void k_fft_fwd2d_t(const void *__restrict__ in_v, void *__restrict__ xs_v, int np,
                                                     int cin_pad, int nch) {
  using act_t = typename std::conditional<F32, float, bf16_t>::type;
  constexpr int kEsz = sizeof(act_t), kQ = kEsz;
  constexpr int P = (KS - 1) / 2, W = TS + 2 * P, WP = W + 1, Dz = 2 * TS;
  static_assert(W <= 32 && TS + P < 32 - P + 1, "window exceeds the 32-point transform");
  const act_t *in = reinterpret_cast<const act_t *>(in_v);
  act_t *xs = reinterpret_cast<act_t *>(xs_v);
  int chunk, z, pv;
  xcd_order(z, pv, chunk);
  const int p = pv >> 2, y0 = ((pv >> 1) & 1) * TS - P, x0 = (pv & 1) * TS - P;
  extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
  act_t *plane = reinterpret_cast<act_t *>(dyn_lds);    // [wx][wy (pitch WP)][8]
  float2 *T = reinterpret_cast<float2 *>(dyn_lds);      // [kx][wy (pitch WP)][8]
  const int tid = threadIdx.x;
  const act_t *src = in + (((int64_t)p * Dz + z) * Dz * Dz) * cin_pad + chunk * 8;
  for (int v = tid; v < W * W; v += 256) {
    const int wy = v / W, wx = v - wy * W;
    const int y = y0 + wy, x = x0 + wx;
    const bool inside = y >= 0 && y < Dz && x >= 0 && x < Dz;
#pragma unroll
    for (int q = 0; q < kEsz / 2; ++q)
      reinterpret_cast<uint4 *>(plane + (wx * WP + wy) * 8)[q] =
          inside ? reinterpret_cast<const uint4 *>(src + ((int64_t)y * Dz + x) * cin_pad)[q] : make_uint4(0, 0, 0, 0);
  }
  __syncthreads();
  // rows along x (window rows wy) on 8 W threads, a lane pair per (wy, two channels),
  // lane h taking array positions a = 16 h + n <- window column w(a)
  const int h = tid & 1, q = tid >> 1;
  {
    const bool roww = tid < 8 * W;
    const int wy = q >> 2, c0 = (q & 3) * 2;
    float re[16], im[16];
#pragma unroll
    for (int n = 0; n < 16; ++n) {
      const int a = 16 * h + n;
      const int w = a < TS + P ? a + P : (a >= 32 - P ? a - 32 + P : -1);
      re[n] = 0.0f;
      im[n] = 0.0f;
      if (roww && w >= 0) {
        if constexpr (F32) {
          const float2 two = *reinterpret_cast<const float2 *>(plane + (w * WP + wy) * 8 + c0);
          re[n] = two.x;
          im[n] = two.y;
        } else {
          const uint32_t two = *reinterpret_cast<const uint32_t *>(plane + (w * WP + wy) * 8 + c0);
          re[n] = __uint_as_float(two << 16);
          im[n] = __uint_as_float(two & 0xffff0000u);
        }
      }
    }
    __syncthreads();  // the plane is in registers; its LDS becomes the row spectra
    if (roww) {
      fft32_pair_dif<false>(re, im, h, pair_swap);
      row_fwd_store2(T, wy, c0, h, W, re, im);
    }
  }
  __syncthreads();
  // columns along y on all 256 threads: array position a <- window row w(a)
  const int kxp = q >> 3, c = q & 7;
  float re[16], im[16];
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    const int a = 16 * h + n;
    const int w = a < TS + P ? a + P : (a >= 32 - P ? a - 32 + P : -1);
    const float2 v = w >= 0 ? T[(kxp * WP + w) * 8 + c] : make_float2(0.0f, 0.0f);
    re[n] = v.x;
    im[n] = v.y;
  }
  fft32_pair_dif<false>(re, im, h, pair_swap);
  __syncthreads();
  act_t *O = reinterpret_cast<act_t *>(T);  // [col][re | im][8]
  float2 *Zp = reinterpret_cast<float2 *>(dyn_lds + plane_lds_bytes(W, F32));
  col_fwd_store2<F32>(O, Zp, kxp, c, h, re, im);
  __syncthreads();
  dc_nyquist_split<F32>(Zp, O, tid);
  __syncthreads();
  const int64_t rowb = (int64_t)nch * 16;
  for (int e = tid; e < kCols * kQ; e += 256) {
    const int col = e / kQ, hh = e % kQ;
    *reinterpret_cast<uint4 *>(xs + (((int64_t)col * np + pv) * Dz + z) * rowb + chunk * 16 + hh * (16 / kEsz)) =
        *reinterpret_cast<const uint4 *>(O + col * 16 + hh * (16 / kEsz));
  }
}


// Between two frequency-domain layers: the inverse of layer i (bias, residual,
// ReLU, bf16 rounding exactly as k_fft_inv2d stores it) feeds the forward
// transform of layer i + 1 in registers, so the activation makes no round trip
// through memory; it is stored only when a later layer reads it (OUT).
// One workgroup per (z, pose, chunk), grid (D, np, nch) in XCD order; the chunking
// of layer i's output is the chunking of layer i + 1's input.  LDS: the spectrum /
// row spectra (fft_lds_bytes) and, with a residual or a stored output, the
// activation plane [y][x][8].  The residual (RES) and the stored output (OUT) are
// template arguments: as run-time tests they put a branch and a wait on each
// value's residual read inside the epilogue of the row transforms.
template <int DT, bool F32, bool RES, bool OUT>
__global__ __launch_bounds__(256) void k_fft_mid(const void *__restrict__ ys_v, const float *__restrict__ bias,
                                                  const void *__restrict__ res_v, void *__restrict__ out_v,
                                                  void *__restrict__ xs_v, int np, int D_rt, int nch, int cout_store,
                                                  int lds_spec) {
  using act_t = typename std::conditional<F32, float, bf16_t>::type;
  constexpr int kEsz = sizeof(act_t), kQ = kEsz;
  const act_t *ys = reinterpret_cast<const act_t *>(ys_v);
  const act_t *res = reinterpret_cast<const act_t *>(res_v);
  act_t *out = reinterpret_cast<act_t *>(out_v);
  act_t *xs = reinterpret_cast<act_t *>(xs_v);
  const int D = DT ? DT : D_rt;
  int chunk, z, p;
  xcd_order(z, p, chunk);
  extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
  act_t *Y = reinterpret_cast<act_t *>(dyn_lds);
  float2 *T = reinterpret_cast<float2 *>(dyn_lds);
  float2 *Zp = reinterpret_cast<float2 *>(dyn_lds + plane_lds_bytes(D, F32));
  act_t *R = reinterpret_cast<act_t *>(dyn_lds + lds_spec);
  const int tid = threadIdx.x, h = tid & 1, q = tid >> 1;
  const int64_t rowb = (int64_t)nch * 16;
  const int64_t base = (((int64_t)p * D + z) * D * D) * cout_store + chunk * 8;
  for (int e = tid; e < kCols * kQ; e += 256) {
    const int col = e / kQ, hh = e % kQ;
    *reinterpret_cast<uint4 *>(Y + col * 16 + hh * (16 / kEsz)) = *reinterpret_cast<const uint4 *>(
        ys + (((int64_t)col * np + p) * D + z) * rowb + chunk * 16 + hh * (16 / kEsz));
  }
  if constexpr (RES)
    for (int v = tid; v < D * D; v += 256)
#pragma unroll
      for (int qq = 0; qq < kEsz / 2; ++qq)
        reinterpret_cast<uint4 *>(R + v * 8)[qq] = reinterpret_cast<const uint4 *>(res + base + (int64_t)v * cout_store)[qq];
  __syncthreads();
  const int kxp = q >> 3, c = q & 7;  // column pair of the column phases
  // inverse columns along ky
  {
    float re[16], im[16];
    dc_nyquist_pack<F32>(Y, Zp, tid);
    if (kxp) col_inv_load2<F32>(Y, kxp, c, h, re, im);
    __syncthreads();
    if (!kxp) col_inv_load_dc2(Zp, c, h, re, im);
    fft32_pair_dit<true>(re, im, h, pair_swap);
    col_inv_store2(T, kxp, c, h, D, re, im);
  }
  __syncthreads();
  // rows along x: inverse of two channels, epilogue (bf16 rounding in the bf16
  // form), then their forward transform (the next layer's input rows)
  {
    const bool roww = tid < 8 * D;
    const int y = q >> 2, c0 = (q & 3) * 2;
    float re[16], im[16];
    if (roww) {
      row_inv_load2(T, y, c0, h, D, re, im);
      fft32_pair_dit<true>(re, im, h, pair_swap);
      constexpr float kScale = 1.0f / (kN * kN);
      const float b0 = bias[chunk * 8 + c0], b1 = bias[chunk * 8 + c0 + 1];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int x = 16 * h + j;
        if (x < D) {
          float v0 = re[j] * kScale + b0, v1 = im[j] * kScale + b1;
          if constexpr (F32) {
            if constexpr (RES) {
              const float2 two = *reinterpret_cast<const float2 *>(R + (y * D + x) * 8 + c0);
              v0 += two.x;
              v1 += two.y;
            }
            v0 = v0 > 0.0f ? v0 : 0.0f;
            v1 = v1 > 0.0f ? v1 : 0.0f;
            if constexpr (OUT) *reinterpret_cast<float2 *>(R + (y * D + x) * 8 + c0) = make_float2(v0, v1);
            re[j] = v0;
            im[j] = v1;
          } else {
            if constexpr (RES) {
              const uint32_t two = *reinterpret_cast<const uint32_t *>(R + (y * D + x) * 8 + c0);
              v0 += __uint_as_float(two << 16);
              v1 += __uint_as_float(two & 0xffff0000u);
            }
            const bf16_t h0 = (bf16_t)(v0 > 0.0f ? v0 : 0.0f), h1 = (bf16_t)(v1 > 0.0f ? v1 : 0.0f);
            if constexpr (OUT)
              *reinterpret_cast<uint32_t *>(R + (y * D + x) * 8 + c0) =
                  (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
            re[j] = (float)h0;
            im[j] = (float)h1;
          }
        } else {
          re[j] = 0.0f;
          im[j] = 0.0f;
        }
      }
      fft32_pair_dif<false>(re, im, h, pair_swap);
      // no barrier between reading and rewriting T: each lane reads the row spectra
      // at the frequencies of its own parity (the mirror 32 - k has the same parity)
      // and writes back exactly those slots; the partner's values came by DPP
      row_fwd_store2(T, y, c0, h, D, re, im);
    }
  }
  __syncthreads();
  if constexpr (OUT)
    for (int v = tid; v < D * D; v += 256)
#pragma unroll
      for (int qq = 0; qq < kEsz / 2; ++qq)
        reinterpret_cast<uint4 *>(out + base + (int64_t)v * cout_store)[qq] = reinterpret_cast<const uint4 *>(R + v * 8)[qq];
  // forward columns along y
  float re[16], im[16];
  col_fwd_load2(T, kxp, c, h, D, re, im);
  fft32_pair_dif<false>(re, im, h, pair_swap);
  __syncthreads();
  act_t *O = reinterpret_cast<act_t *>(T);
  col_fwd_store2<F32>(O, Zp, kxp, c, h, re, im);
  __syncthreads();
  dc_nyquist_split<F32>(Zp, O, tid);
  __syncthreads();
  for (int e = tid; e < kCols * kQ; e += 256) {
    const int col = e / kQ, hh = e % kQ;
    *reinterpret_cast<uint4 *>(xs + (((int64_t)col * np + p) * D + z) * rowb + chunk * 16 + hh * (16 / kEsz)) =
        *reinterpret_cast<const uint4 *>(O + col * 16 + hh * (16 / kEsz));
  }
}

// Forward transform of one (z, pose, chunk) plane, grid (D, np, nch) in XCD order:
// the chunks of one plane run under one L2, where their pieces of each spectrum row
// (and of each input voxel) meet.  in: [P][D][D][D][cin_pad] of bf16 (F32 = false)
// or float; spectrum rows of the same type.  LDS layouts are padded so that the
// lanes of one access hit distinct banks: the input plane is held transposed,
// [x][y (pitch D + 1)][8 channels], and the half spectrum of the rows is
// [kx][y (pitch D + 1)][8] complex, aliasing the plane once it is in registers.
template <int DT, bool F32>
__global__ __launch_bounds__(256) void k_fft_fwd2d(const void *__restrict__ in_v, void *__restrict__ xs_v, int np,
                                                    int D_rt, int cin_pad, int nch) {
  using act_t = typename std::conditional<F32, float, bf16_t>::type;
  constexpr int kEsz = sizeof(act_t), kQ = kEsz;
  const act_t *in = reinterpret_cast<const act_t *>(in_v);
  act_t *xs = reinterpret_cast<act_t *>(xs_v);
  const int D = DT ? DT : D_rt;
  int chunk, z, p;
  xcd_order(z, p, chunk);
  extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
  act_t *plane = reinterpret_cast<act_t *>(dyn_lds);  // [x][y][8]
  float2 *T = reinterpret_cast<float2 *>(dyn_lds);    // [kx][y][8]
  float2 *Zp = reinterpret_cast<float2 *>(dyn_lds + plane_lds_bytes(D, F32));
  const int tid = threadIdx.x, h = tid & 1, q = tid >> 1, DP = D + 1;
  const act_t *src = in + (((int64_t)p * D + z) * D * D) * cin_pad + chunk * 8;
  for (int v = tid; v < D * D; v += 256) {
    const int y = v / D, x = v - y * D;
#pragma unroll
    for (int qq = 0; qq < kEsz / 2; ++qq)
      reinterpret_cast<uint4 *>(plane + (x * DP + y) * 8)[qq] =
          reinterpret_cast<const uint4 *>(src + (int64_t)v * cin_pad)[qq];
  }
  __syncthreads();
  // rows along x, two channels per complex transform: lane h takes x = 16 h + n
  {
    const bool roww = tid < 8 * D;
    const int y = q >> 2, c0 = (q & 3) * 2;
    float re[16], im[16];
#pragma unroll
    for (int n = 0; n < 16; ++n) {
      const int x = 16 * h + n;
      if (roww && x < D) {
        if constexpr (F32) {
          const float2 two = *reinterpret_cast<const float2 *>(plane + (x * DP + y) * 8 + c0);
          re[n] = two.x;
          im[n] = two.y;
        } else {
          const uint32_t two = *reinterpret_cast<const uint32_t *>(plane + (x * DP + y) * 8 + c0);
          re[n] = __uint_as_float(two << 16);
          im[n] = __uint_as_float(two & 0xffff0000u);
        }
      } else {
        re[n] = 0.0f;
        im[n] = 0.0f;
      }
    }
    __syncthreads();  // the plane is in registers; its LDS becomes the row spectra
    if (roww) {
      fft32_pair_dif<false>(re, im, h, pair_swap);
      row_fwd_store2(T, y, c0, h, D, re, im);
    }
  }
  __syncthreads();
  // columns along y
  const int kxp = q >> 3, c = q & 7;
  float re[16], im[16];
  col_fwd_load2(T, kxp, c, h, D, re, im);
  fft32_pair_dif<false>(re, im, h, pair_swap);
  __syncthreads();
  act_t *O = reinterpret_cast<act_t *>(T);  // [col][re | im][8]
  col_fwd_store2<F32>(O, Zp, kxp, c, h, re, im);
  __syncthreads();
  dc_nyquist_split<F32>(Zp, O, tid);
  __syncthreads();
  const int64_t rowb = (int64_t)nch * 16;
  for (int e = tid; e < kCols * kQ; e += 256) {
    const int col = e / kQ, hh = e % kQ;
    *reinterpret_cast<uint4 *>(xs + (((int64_t)col * np + p) * D + z) * rowb + chunk * 16 + hh * (16 / kEsz)) =
        *reinterpret_cast<const uint4 *>(O + col * 16 + hh * (16 / kEsz));
  }
}

// Inverse transform of one (z, pose, output chunk) plane, grid (D, np, nco) in XCD
// order: bias, residual, ReLU and the store in the activations' channels-last
// layout [P][D][D][D][cout_store].  The spectrum's DC and Nyquist columns travel
// packed, as in the fused transform.  NTL > 1 (overlap-save tiles): the plane of
// edge NTL * D is NTL x NTL tiles of D x D outputs, each with its own spectrum;
// grid (NTL * D, np * NTL^2, nco), np counting (pose, tile) planes.
template <int DT, bool F32, int NTL = 1>
__global__ __launch_bounds__(256) void k_fft_inv2d(const void *__restrict__ ys_v, const float *__restrict__ bias,
                                                    const void *__restrict__ res_v, void *__restrict__ out_v, int np,
                                                    int D_rt, int nco, int cout_store) {
  using act_t = typename std::conditional<F32, float, bf16_t>::type;
  constexpr int kEsz = sizeof(act_t), kQ = kEsz;
  const act_t *ys = reinterpret_cast<const act_t *>(ys_v);
  const act_t *res = reinterpret_cast<const act_t *>(res_v);
  act_t *out = reinterpret_cast<act_t *>(out_v);
  const int D = DT ? DT : D_rt;  // in-plane extent of one tile
  const int Dz = D * NTL;        // grid edge
  int chunk, z, pv;
  xcd_order(z, pv, chunk);
  const int p = pv / (NTL * NTL), y0 = (pv % (NTL * NTL)) / NTL * D, x0 = (pv % NTL) * D;
  extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
  act_t *Y = reinterpret_cast<act_t *>(dyn_lds);
  float2 *T = reinterpret_cast<float2 *>(dyn_lds);
  float2 *Zp = reinterpret_cast<float2 *>(dyn_lds + plane_lds_bytes(D, F32));
  const int tid = threadIdx.x, h = tid & 1, q = tid >> 1, DP = D + 1;
  const int64_t rowb = (int64_t)nco * 16;
  for (int e = tid; e < kCols * kQ; e += 256) {
    const int col = e / kQ, hh = e % kQ;
    *reinterpret_cast<uint4 *>(Y + col * 16 + hh * (16 / kEsz)) = *reinterpret_cast<const uint4 *>(
        ys + (((int64_t)col * np + pv) * Dz + z) * rowb + chunk * 16 + hh * (16 / kEsz));
  }
  __syncthreads();
  const int kxp = q >> 3, c = q & 7;
  {
    float re[16], im[16];
    dc_nyquist_pack<F32>(Y, Zp, tid);
    if (kxp) col_inv_load2<F32>(Y, kxp, c, h, re, im);
    __syncthreads();
    if (!kxp) col_inv_load_dc2(Zp, c, h, re, im);
    fft32_pair_dit<true>(re, im, h, pair_swap);
    col_inv_store2(T, kxp, c, h, D, re, im);
  }
  __syncthreads();
  const bool roww = tid < 8 * D;
  const int y = q >> 2, c0 = (q & 3) * 2;
  float re[16], im[16];
  if (roww) {
    row_inv_load2(T, y, c0, h, D, re, im);
    fft32_pair_dit<true>(re, im, h, pair_swap);
  }
  __syncthreads();  // the row spectra are read; T becomes the output plane
  float *O = reinterpret_cast<float *>(T);  // [x][y (pitch D + 1)][8] conv result + bias
  if (roww) {
    constexpr float kScale = 1.0f / (kN * kN);
    const float b0 = bias[chunk * 8 + c0], b1 = bias[chunk * 8 + c0 + 1];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int x = 16 * h + j;
      if (x < D) *reinterpret_cast<float2 *>(O + (x * DP + y) * 8 + c0) = make_float2(re[j] * kScale + b0, im[j] * kScale + b1);
    }
  }
  __syncthreads();
  const int64_t base = (((int64_t)p * Dz + z) * Dz * Dz) * cout_store + chunk * 8;
  for (int v0 = tid; v0 < D * D; v0 += 256) {
    const int yy = v0 / D, xx = v0 - yy * D;
    const int64_t v = (int64_t)(y0 + yy) * Dz + x0 + xx;
    float f[8];
    const float4 f0 = *reinterpret_cast<const float4 *>(O + (xx * DP + yy) * 8);
    const float4 f1 = *reinterpret_cast<const float4 *>(O + (xx * DP + yy) * 8 + 4);
    f[0] = f0.x; f[1] = f0.y; f[2] = f0.z; f[3] = f0.w; f[4] = f1.x; f[5] = f1.y; f[6] = f1.z; f[7] = f1.w;
    if constexpr (F32) {
      if (res) {
        const float4 r0 = *reinterpret_cast<const float4 *>(res + base + v * cout_store);
        const float4 r1 = *reinterpret_cast<const float4 *>(res + base + v * cout_store + 4);
        f[0] += r0.x; f[1] += r0.y; f[2] += r0.z; f[3] += r0.w; f[4] += r1.x; f[5] += r1.y; f[6] += r1.z; f[7] += r1.w;
      }
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) f[qq] = f[qq] > 0.0f ? f[qq] : 0.0f;
      float4 *dst = reinterpret_cast<float4 *>(out + base + v * cout_store);
      dst[0] = make_float4(f[0], f[1], f[2], f[3]);
      dst[1] = make_float4(f[4], f[5], f[6], f[7]);
    } else {
      if (res) {
        const uint4 r = *reinterpret_cast<const uint4 *>(res + base + v * cout_store);
        const bf16_t *rb = reinterpret_cast<const bf16_t *>(&r);
#pragma unroll
        for (int qq = 0; qq < 8; ++qq) f[qq] += (float)rb[qq];
      }
      uint4 o;
      bf16_t *ob = reinterpret_cast<bf16_t *>(&o);
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) ob[qq] = (bf16_t)(f[qq] > 0.0f ? f[qq] : 0.0f);
      *reinterpret_cast<uint4 *>(out + base + v * cout_store) = o;
    }
  }
}

// ---------------------------------------------------------------- z-correlation

// One (column, block of ppb poses): rows r = (pose pl, z), pl = r / D; the panel in
// LDS holds, per pose, its D spectrum rows between KS - 1 zero rows (the z
// padding), each row nch x 32 bytes + 16 (bank offset between consecutive rows).
// Real output column n < NT: (re, im) part n / (NT / 2) of channel n % (NT / 2).
// Waves: NT = 128 -> 2 row groups x 2 column groups, else 2 row groups; each wave
// 96 rows (3 blocks of 32).
template <int KS, int NT>
__global__ __launch_bounds__(NT == 128 ? 256 : 128) __attribute__((amdgpu_waves_per_eu(2))) void k_fft_zconv(
    const bf16_t *__restrict__ xs, const bf16_t *__restrict__ gp, bf16_t *__restrict__ ys, int np, int D, int nch,
    int ppb, int gbytes) {
  constexpr int P = (KS - 1) / 2;
  constexpr int WN = NT == 128 ? 2 : 1, NW = 2 * WN, NB = NT / WN / 32, MB = 3;
  constexpr int NBT = NT / 32;
  __shared__ __attribute__((aligned(16))) char lds[kPanelRows * 272];
  int pblk, col, zero;
  xcd_order(pblk, col, zero);
  (void)zero;
  const int p0 = pblk * ppb;
  const int nvalid = min(ppb, np - p0);
  const int rowb = nch * 32, pitch = rowb + 16;  // bytes
  const int zrows = D + KS - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wave_m = wave / WN, wave_n = wave % WN;
  const int khalf = lane >> 5, lrow = lane & 31;

  // panel: LDS rows rr = (pl, zz), zz = z + P; the loads of a batch are all in
  // flight before any is stored
  {
    constexpr int NTH = NW * 64, kIt = (kPanelRows * 16 + NTH - 1) / NTH, kBatch = 18;
    const int q16 = rowb / 16;  // uint4 per row
    const int total = ppb * zrows * q16;
    const bf16_t *src = xs + ((int64_t)col * np + p0) * D * (rowb / 2);
#pragma unroll
    for (int i0 = 0; i0 < kIt; i0 += kBatch) {
      uint4 pv[kBatch];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        const int e = (i0 + i) * NTH + tid;
        pv[i] = make_uint4(0, 0, 0, 0);
        if (i0 + i < kIt && e < total) {
          const int q = e % q16, rr = e / q16, pl = rr / zrows, zr = rr % zrows - P;
          if (pl < nvalid && zr >= 0 && zr < D)
            pv[i] = *reinterpret_cast<const uint4 *>(src + ((int64_t)pl * D + zr) * (rowb / 2) + q * 8);
        }
      }
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        const int e = (i0 + i) * NTH + tid;
        if (i0 + i < kIt && e < total) *reinterpret_cast<uint4 *>(lds + (e / q16) * pitch + (e % q16) * 16) = pv[i];
      }
    }
  }
  // tile rows r = (z, pl), pose fastest: the 16 rows of a lane group then fall on
  // 16 different bank quads of the 272-byte-pitch panel at D = 24
  int rowoff[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int r = wave_m * 96 + mb * 32 + lrow;
    const int pl = r % ppb, zl = r / ppb;
    rowoff[mb] = (zl < D ? (pl * zrows + zl) * pitch : 0) + khalf * 16;
  }
  typedef float accv __attribute__((ext_vector_type(16)));
  accv acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;
  __syncthreads();

  // K steps s = chunk * KS + dz; weight fragments [col][chunk][dz][NBT][64 lanes][8],
  // prefetched kPF steps ahead (past the last step the last one is loaded again)
  const int steps = nch * KS;
  const int step_bytes = NBT * 1024;
  const __amdgpu_buffer_rsrc_t wrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t *>(gp), (short)0, gbytes, 0x00020000);
  const int wbase = col * steps * step_bytes + (wave_n * NB * 64 + lane) * 16;
  if (col + 1 < (int)gridDim.y) {
    // warm L2 with a slice of the next column's weights: the workgroups of one
    // column run together on one XCD, the next column's follow them there
    const int colb = steps * step_bytes, slice = (colb + gridDim.x - 1) / gridDim.x;
    const int off = (col + 1) * colb + pblk * slice + tid * 128;
    if (tid * 128 < slice && off + 4 <= gbytes) {
      const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(wrs, off, 0, 0);
      if (v == 0x7fc00001u && np < 0) ys[0] = (bf16_t)0.0f;  // keeps the load; never true
    }
  }
  constexpr int kPF = 4;
  uint4 bq[kPF][NB];
#pragma unroll
  for (int q = 0; q < kPF; ++q)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      bq[q][nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                wrs, wbase + nb * 1024, min(q, steps - 1) * step_bytes, 0));
  // the row fragments of step s + 1 are read while the MFMAs of step s issue
  uint4 a[2][MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) a[0][mb] = *reinterpret_cast<const uint4 *>(lds + rowoff[mb]);
  int nchunk = 0, ndz = 1;  // step s + 1
  auto step = [&](const int s, const int ph) {
    if (ndz == KS) {
      ndz = 0;
      ++nchunk;
    }
    const int noff = s + 1 < steps ? ndz * pitch + nchunk * 32 : 0;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) a[(ph + 1) & 1][mb] = *reinterpret_cast<const uint4 *>(lds + rowoff[mb] + noff);
    ++ndz;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[ph & 1][mb]),
                                                               __builtin_bit_cast(bf16x8, bq[ph][nb]), acc[mb][nb], 0,
                                                               0, 0);
    const int sn = s + kPF;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      bq[ph][nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                 wrs, wbase + nb * 1024, min(sn, steps - 1) * step_bytes, 0));
  };
  // whole groups of kPF steps with no test inside (a test per step makes the
  // compiler's wait analysis drain every outstanding weight load), then the rest
  const int full = steps / kPF * kPF;
  for (int s0 = 0; s0 < full; s0 += kPF) {
#pragma unroll
    for (int ph = 0; ph < kPF; ++ph) step(s0 + ph, ph);
  }
#pragma unroll
  for (int ph = 0; ph < kPF; ++ph)
    if (full + ph < steps) step(full + ph, ph);

  // epilogue through LDS: rows of NT bf16 in the spectrum layout, then contiguous stores
  __syncthreads();
  constexpr int HALF = NT / 2;
  constexpr int orow = HALF * 4;  // bytes per output row (HALF channels x re, im x 2 B)
  constexpr int opitch = orow + 16;
  bf16_t *ot = reinterpret_cast<bf16_t *>(lds);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wave_m * 96 + mb * 32 + 8 * (r >> 2) + 4 * khalf + (r & 3);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int n = (wave_n * NB + nb) * 32 + lrow;
        const int part = n / HALF, co = n % HALF;
        ot[(row * opitch + (co >> 3) * 32 + part * 16) / 2 + (co & 7)] = (bf16_t)acc[mb][nb][r];
      }
    }
  __syncthreads();
  constexpr int q16 = orow / 16;
  bf16_t *dst = ys + ((int64_t)col * np + p0) * D * (orow / 2);
  for (int e = tid; e < ppb * D * q16; e += NW * 64) {
    const int q = e % q16, row = e / q16, pl = row % ppb, zl = row / ppb;
    if (pl < nvalid)
      *reinterpret_cast<uint4 *>(dst + ((int64_t)pl * D + zl) * (orow / 2) + q * 8) =
          *reinterpret_cast<const uint4 *>(lds + row * opitch + q * 16);
  }
}

// The same z-correlation for 128 real columns with RG row groups of 96 rows and
// the K walk in two halves of at most four channel chunks: the panel holds one
// half at a time (rows of 128 bytes + 16).  Each row group is two waves of 96 rows
// x 64 columns; the row groups read the same weight fragments at the same step, so
// the second read is served next to the CU and the L2 weight stream per row
// shrinks by RG.  RG = 2 (192 rows, 8 poses at 24^3): 52 KB of LDS (the epilogue
// staging), three workgroups per CU whose panel loads hide behind each other's
// MFMAs; 3 % faster than RG = 1 (six two-wave workgroups), while RG = 3 (two per
// CU) is 35 % slower: fewer workgroups leave the panel loads exposed.
// Tile rows r = (pl, z), z fastest.
constexpr int kRowsZH = 96, kPanelRowsH = 144, kZhRG = 2;

template <int KS, int RG>
__global__ __launch_bounds__(128 * RG) __attribute__((amdgpu_waves_per_eu(3))) void k_fft_zconv_h(
    const bf16_t *__restrict__ xs, const bf16_t *__restrict__ gp, bf16_t *__restrict__ ys, int np, int D, int nch,
    int ppb, int gbytes) {
  constexpr int P = (KS - 1) / 2, NT = 128, NB = 2, MB = 3, NBT = 4, NTH = 128 * RG;
  constexpr int PH = 4 * 32 + 16;                // panel row pitch (bytes)
  constexpr int HALF = NT / 2, orow = HALF * 4, opitch = orow + 16;
  constexpr int kRows = kRowsZH * RG, kPanel = kPanelRowsH * RG;
  constexpr int kLds = kRows * opitch > kPanel * PH ? kRows * opitch : kPanel * PH;
  __shared__ __attribute__((aligned(16))) char lds[kLds];
  int pblk, col, zero;
  xcd_order(pblk, col, zero);
  (void)zero;
  const int p0 = pblk * ppb;
  const int nvalid = min(ppb, np - p0);
  const int rowh = nch * 16;  // bf16 elements per spectrum row
  const int zrows = D + KS - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave_n = (tid >> 6) & 1, wave_m = tid >> 7;
  const int khalf = lane >> 5, lrow = lane & 31;
  int rowoff[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int r = wave_m * kRowsZH + mb * 32 + lrow;
    const int pl = r / D, zl = r % D;
    rowoff[mb] = (pl < ppb ? (pl * zrows + zl) * PH : 0) + khalf * 16;
  }
  typedef float accv __attribute__((ext_vector_type(16)));
  accv acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;

  const int step_bytes = NBT * 1024, steps = nch * KS;
  const __amdgpu_buffer_rsrc_t wrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t *>(gp), (short)0, gbytes, 0x00020000);
  const int wbase = col * steps * step_bytes + (wave_n * NB * 64 + lane) * 16;
  if (col + 1 < (int)gridDim.y) {
    // warm L2 with a slice of the next column's weights (as in k_fft_zconv)
    const int colb = steps * step_bytes, slice = (colb + gridDim.x - 1) / gridDim.x;
    const int off = (col + 1) * colb + pblk * slice + tid * 128;
    if (tid * 128 < slice && off + 4 <= gbytes) {
      const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(wrs, off, 0, 0);
      if (v == 0x7fc00001u && np < 0) ys[0] = (bf16_t)0.0f;  // keeps the load; never true
    }
  }
  const bf16_t *src = xs + ((int64_t)col * np + p0) * D * rowh;
  for (int h0 = 0; h0 < nch; h0 += 4) {
    const int nh = min(4, nch - h0);  // chunks in this half
    if (h0) __syncthreads();           // the previous half's panel is read
    {
      constexpr int kIt = (kPanel * 8 + NTH - 1) / NTH;  // uint4 per thread, 8 per row
      uint4 pv[kIt];
      const int q8 = nh * 2, total = ppb * zrows * q8;
#pragma unroll
      for (int i = 0; i < kIt; ++i) {
        const int e = i * NTH + tid;
        pv[i] = make_uint4(0, 0, 0, 0);
        if (e < total) {
          const int q = e % q8, rr = e / q8, pl = rr / zrows, zr = rr % zrows - P;
          if (pl < nvalid && zr >= 0 && zr < D)
            pv[i] = *reinterpret_cast<const uint4 *>(src + ((int64_t)pl * D + zr) * rowh + h0 * 16 + q * 8);
        }
      }
#pragma unroll
      for (int i = 0; i < kIt; ++i) {
        const int e = i * NTH + tid;
        if (e < total) *reinterpret_cast<uint4 *>(lds + (e / q8) * PH + (e % q8) * 16) = pv[i];
      }
    }
    __syncthreads();
    const int hsteps = nh * KS, sbase = h0 * KS;
    constexpr int kPF = 4;
    uint4 bq[kPF][NB];
#pragma unroll
    for (int q = 0; q < kPF; ++q)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bq[q][nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                  wrs, wbase + nb * 1024, (sbase + min(q, hsteps - 1)) * step_bytes, 0));
    uint4 a[2][MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) a[0][mb] = *reinterpret_cast<const uint4 *>(lds + rowoff[mb]);
    int nchunk = 0, ndz = 1;  // step s + 1 within the half
    // one K step: the row fragments of step s + 1 are read while the MFMAs of step s
    // issue, and the weight fragments of step s + kPF replace those just used
    auto step = [&](const int s, const int ph) {
      if (ndz == KS) {
        ndz = 0;
        ++nchunk;
      }
      const int noff = s + 1 < hsteps ? ndz * PH + nchunk * 32 : 0;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a[(ph + 1) & 1][mb] = *reinterpret_cast<const uint4 *>(lds + rowoff[mb] + noff);
      ++ndz;
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[ph & 1][mb]),
                                                                 __builtin_bit_cast(bf16x8, bq[ph][nb]), acc[mb][nb],
                                                                 0, 0, 0);
      const int sn = s + kPF;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bq[ph][nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                   wrs, wbase + nb * 1024, (sbase + min(sn, hsteps - 1)) * step_bytes, 0));
    };
    // whole groups of kPF steps with no test inside (a test per step makes the
    // compiler's wait analysis drain every outstanding weight load), then the rest
    const int full = hsteps / kPF * kPF;
    for (int s0 = 0; s0 < full; s0 += kPF) {
#pragma unroll
      for (int ph = 0; ph < kPF; ++ph) step(s0 + ph, ph);
    }
#pragma unroll
    for (int ph = 0; ph < kPF; ++ph)
      if (full + ph < hsteps) step(full + ph, ph);
  }

  // epilogue through LDS: rows of NT bf16 in the spectrum layout, then contiguous
  // stores.  Lanes 2m and 2m + 1 hold columns n and n + 1 of one 8-channel group:
  // each lane packs its rows r and r + 1, the pair swaps halves by a DPP move, and
  // the even lane writes row r, the odd lane row r + 1, as 32-bit words
  __syncthreads();
  const int odd = lane & 1;
  const uint32_t sel = odd ? 0x03020706u : 0x05040100u;  // byte picks from {partner, own}
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int row = wave_m * kRowsZH + mb * 32 + 8 * (r >> 2) + 4 * khalf + (r & 3) + odd;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int n = (wave_n * NB + nb) * 32 + (lrow & ~1);
        const int part = n / HALF, co = n % HALF;
        const uint32_t own = pack_bf16x2(acc[mb][nb][r], acc[mb][nb][r + 1]);
        const uint32_t other = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)own, 0xB1, 0xF, 0xF, false);
        *reinterpret_cast<uint32_t *>(lds + row * opitch + (co >> 3) * 32 + part * 16 + (co & 7) * 2) =
            __builtin_amdgcn_perm(other, own, sel);
      }
    }
  __syncthreads();
  constexpr int q16 = orow / 16;
  bf16_t *dst = ys + ((int64_t)col * np + p0) * D * (orow / 2);
  for (int e = tid; e < nvalid * D * q16; e += NTH) {
    const int q = e % q16, row = e / q16;
    *reinterpret_cast<uint4 *>(dst + (int64_t)row * (orow / 2) + q * 8) =
        *reinterpret_cast<const uint4 *>(lds + row * opitch + q * 16);
  }
}

// The z-correlation with fp32 spectra on the fp32 matrix instruction (32x32x2):
// the same blocking as k_fft_zconv_h (96 rows of (pose, z), the K walk in halves
// of at most four channel chunks through an LDS panel), NT = 64 NB real columns
// over two waves.  One K step (chunk, dz) is 16 deep (8 channels x re, im) and
// takes eight MFMAs; MFMA j reads K indices j and 8 + j, so a lane's A fragment
// is 8 contiguous floats of its row (khalf 0: re of the 8 channels, khalf 1: im)
// and its B fragment the 8 matching weight values, both two 16-byte loads.
template <int KS, int NB>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) void k_fft_zconv_f32(
    const float *__restrict__ xs, const float *__restrict__ gp, float *__restrict__ ys, int np, int D, int nch,
    int ppb, int gbytes) {
  constexpr int P = (KS - 1) / 2, NT = 64 * NB, MB = 3, NBT = NT / 32, NTH = 128;
  constexpr int PH = 4 * 64 + 16;                // panel row pitch (bytes): 4 chunks x 16 floats
  constexpr int HALF = NT / 2, orow = HALF * 8, opitch = orow + 16;
  constexpr int kLds = kRowsZH * opitch > kPanelRowsH * PH ? kRowsZH * opitch : kPanelRowsH * PH;
  __shared__ __attribute__((aligned(16))) char lds[kLds];
  int pblk, col, zero;
  xcd_order(pblk, col, zero);
  (void)zero;
  const int p0 = pblk * ppb;
  const int nvalid = min(ppb, np - p0);
  const int rowf = nch * 16;  // floats per spectrum row
  const int zrows = D + KS - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave_n = tid >> 6;
  const int khalf = lane >> 5, lrow = lane & 31;
  int rowoff[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int r = mb * 32 + lrow;
    const int pl = r / D, zl = r % D;
    rowoff[mb] = (pl < ppb ? (pl * zrows + zl) * PH : 0) + khalf * 32;
  }
  f32x16 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;

  const int step_bytes = NBT * 2048, steps = nch * KS;
  const __amdgpu_buffer_rsrc_t wrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(gp), (short)0, gbytes, 0x00020000);
  const int wbase = col * steps * step_bytes + (wave_n * NB * 64 + lane) * 32;
  if (col + 1 < (int)gridDim.y) {
    // warm L2 with a slice of the next column's weights (as in k_fft_zconv)
    const int colb = steps * step_bytes, slice = (colb + gridDim.x - 1) / gridDim.x;
    const int off = (col + 1) * colb + pblk * slice + tid * 128;
    if (tid * 128 < slice && off + 4 <= gbytes) {
      const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(wrs, off, 0, 0);
      if (v == 0x7fc00001u && np < 0) ys[0] = 0.0f;  // keeps the load; never true
    }
  }
  const float *src = xs + ((int64_t)col * np + p0) * D * rowf;
  for (int h0 = 0; h0 < nch; h0 += 4) {
    const int nh = min(4, nch - h0);  // chunks in this half
    if (h0) __syncthreads();           // the previous half's panel is read
    {
      constexpr int kIt = (kPanelRowsH * 16 + NTH - 1) / NTH;  // uint4 per thread, 16 per row
      constexpr int kBatch = 9;
      const int q16 = nh * 4, total = ppb * zrows * q16;
#pragma unroll
      for (int i0 = 0; i0 < kIt; i0 += kBatch) {
        uint4 pv[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
          const int e = (i0 + i) * NTH + tid;
          pv[i] = make_uint4(0, 0, 0, 0);
          if (i0 + i < kIt && e < total) {
            const int q = e % q16, rr = e / q16, pl = rr / zrows, zr = rr % zrows - P;
            if (pl < nvalid && zr >= 0 && zr < D)
              pv[i] = *reinterpret_cast<const uint4 *>(src + ((int64_t)pl * D + zr) * rowf + h0 * 16 + q * 4);
          }
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
          const int e = (i0 + i) * NTH + tid;
          if (i0 + i < kIt && e < total) *reinterpret_cast<uint4 *>(lds + (e / q16) * PH + (e % q16) * 16) = pv[i];
        }
      }
    }
    __syncthreads();
    const int hsteps = nh * KS, sbase = h0 * KS;
    int nchunk = 0, ndz = 0;
    uint4 bq[NB][2];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        bq[nb][q] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                  wrs, wbase + nb * 2048 + q * 16, sbase * step_bytes, 0));
    for (int s = 0; s < hsteps; ++s) {
      const int aoff = ndz * PH + nchunk * 64;
      if (++ndz == KS) {
        ndz = 0;
        ++nchunk;
      }
      float a[MB][8];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const float4 a0 = *reinterpret_cast<const float4 *>(lds + rowoff[mb] + aoff);
        const float4 a1 = *reinterpret_cast<const float4 *>(lds + rowoff[mb] + aoff + 16);
        a[mb][0] = a0.x; a[mb][1] = a0.y; a[mb][2] = a0.z; a[mb][3] = a0.w;
        a[mb][4] = a1.x; a[mb][5] = a1.y; a[mb][6] = a1.z; a[mb][7] = a1.w;
      }
      float b[NB][8];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        __builtin_memcpy(&b[nb][0], &bq[nb][0], 16);
        __builtin_memcpy(&b[nb][4], &bq[nb][1], 16);
      }
      // the next step's weight fragments are in flight during this step's MFMAs
      const int sn = min(s + 1, hsteps - 1);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          bq[nb][q] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                    wrs, wbase + nb * 2048 + q * 16, (sbase + sn) * step_bytes, 0));
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb][j], b[nb][j], acc[mb][nb], 0, 0, 0);
    }
  }

  // epilogue through LDS: rows of NT floats in the spectrum layout, then contiguous stores
  __syncthreads();
  float *ot = reinterpret_cast<float *>(lds);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = mb * 32 + 8 * (r >> 2) + 4 * khalf + (r & 3);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int n = (wave_n * NB + nb) * 32 + lrow;
        const int part = n / HALF, co = n % HALF;
        ot[(row * opitch) / 4 + (co >> 3) * 16 + part * 8 + (co & 7)] = acc[mb][nb][r];
      }
    }
  __syncthreads();
  constexpr int q16 = orow / 16;
  float *dst = ys + ((int64_t)col * np + p0) * D * (orow / 4);
  for (int e = tid; e < nvalid * D * q16; e += NTH) {
    const int q = e % q16, row = e / q16;
    *reinterpret_cast<uint4 *>(dst + (int64_t)row * (orow / 4) + q * 4) =
        *reinterpret_cast<const uint4 *>(lds + row * opitch + q * 16);
  }
}

// ---------------------------------------------------------------- weights

// One thread per (col, chunk, dz, 32-column block, lane): the 8 values of one MFMA
// B fragment, bf16 or fp32 (element j is K index 8 * khalf + j, the order both
// z-correlations read).  w: folded fp32 weights [cout][cin][k][k][k].
template <typename T>
__global__ void k_fft_gspec(const float *__restrict__ w, T *__restrict__ gp, int cin, int cout, int nch, int KS,
                            int nbt) {
  const int64_t total = (int64_t)kCols * nch * KS * nbt * 64;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int lane = (int)(t % 64), nbk = (int)((t / 64) % nbt);
  const int dz = (int)((t / (64 * nbt)) % KS), chunk = (int)((t / (64 * nbt * KS)) % nch);
  const int col = (int)(t / ((int64_t)64 * nbt * KS * nch));
  const int ky = col / kNX, kx = col % kNX, P = (KS - 1) / 2;
  const int n = nbk * 32 + (lane & 31), half = nbt * 16;
  const int part = n / half, co = n % half;
  T v[8];
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * (lane >> 5) + j, ci = chunk * 8 + (k & 7), xim = k >> 3;
    float gr = 0.0f, gi = 0.0f;
    if (ci < cin && co < cout) {
      const float *wk = w + (((int64_t)co * cin + ci) * KS + dz) * KS * KS;
      for (int dy = 0; dy < KS; ++dy)
        for (int dx = 0; dx < KS; ++dx) {
          const int ph = (((dy - P) * ky + (dx - P) * kx) % 32 + 32) % 32;
          const float c = ph < 16 ? kFftCos32[ph] : -kFftCos32[ph - 16];
          const float s = ph < 16 ? kFftSin32[ph] : -kFftSin32[ph - 16];
          gr += wk[dy * KS + dx] * c;
          gi += wk[dy * KS + dx] * s;
        }
    }
    // Y = X G:  Yr = Xr Gr - Xi Gi,  Yi = Xr Gi + Xi Gr
    const float b = part == 0 ? (xim == 0 ? gr : -gi) : (xim == 0 ? gi : gr);
    v[j] = (T)b;
  }
#pragma unroll
  for (int q = 0; q < (int)sizeof(T) / 2; ++q) {
    uint4 o;
    __builtin_memcpy(&o, reinterpret_cast<const char *>(v) + 16 * q, 16);
    reinterpret_cast<uint4 *>(gp + t * 8)[q] = o;
  }
}

int nch_of(const ConvLayer &L) { return (L.cin + 7) / 8; }

// dynamic LDS of the plane transforms: the plane region (the input plane and the
// output staging fit in it) and the packed DC / Nyquist column
size_t fft_lds_bytes(int D, bool f32) { return (size_t)plane_lds_bytes(D, f32) + kZpBytes; }
int nbt_of(const ConvLayer &L) { return L.cout * 2 / 32; }
int esz_of(const ConvLayer &L) { return L.spec_f32 ? 4 : 2; }

// overlap-save tiling for the grids of edge 32 (2 x 2 tiles of 16 x 16 outputs per
// plane, each through a window of 16 + k - 1 <= 32 positions)
constexpr int kTileTS = 16;
bool fft_tiled(const ConvLayer &L, int D) { return D == 2 * kTileTS && L.k <= 7 && D + L.k - 1 > kN; }
int fft_planes(const ConvLayer &L, int D, int np) { return fft_tiled(L, D) ? 4 * np : np; }

}  // namespace

bool fft_conv_layer_ok(const ConvLayer &L) {
  if (L.spec_f32)  // the fp32 z-correlation covers 32 and 64 output channels
    return L.stride == 1 && (L.k == 3 || L.k == 5 || L.k == 7) && L.cin <= 64 && L.cin_pad % 8 == 0 &&
           (L.cout == 32 || L.cout == 64) && L.cout_store % 8 == 0;
  return L.stride == 1 && (L.k == 3 || L.k == 5 || L.k == 7) && L.cin <= 64 && L.cin_pad % 8 == 0 &&
         (L.cout == 16 || L.cout == 32 || L.cout == 64) && L.cout_store % 8 == 0;
}

bool fft_conv_ok(const ConvLayer &L, int D) {
  if (!L.gspec || !fft_conv_layer_ok(L)) return false;
  if (!fft_tiled(L, D) && (D < 1 || D + L.k - 1 > kN || D > kDMax)) return false;
  if (L.spec_f32) {
    const int ppb = kRowsZH / D;
    return ppb >= 1 && ppb * (D + L.k - 1) <= kPanelRowsH;
  }
  const int ppb = kRowsZ / D;
  return ppb >= 1 && ppb * (D + L.k - 1) <= kPanelRows;
}

int64_t fft_conv_gspec_bytes(const ConvLayer &L) {
  return (int64_t)kCols * nch_of(L) * L.k * nbt_of(L) * 512 * esz_of(L);
}

// work buffer: the input spectrum rows at offset 0 (room for 8 chunks, the most a
// layer takes), the output spectrum rows after them; fixed offsets, so that one
// layer's output spectrum is where the next layer's fused transform finds it
int64_t fft_spec_in_elems(int D, int np) { return (int64_t)kCols * np * D * 8 * 16; }

int64_t fft_conv_work_bytes(const ConvLayer &L, int D, int np) {
  const int npv = fft_planes(L, D, np);
  return (fft_spec_in_elems(D, npv) + (int64_t)kCols * npv * D * (L.cout / 8) * 16) * esz_of(L);
}

hipError_t fft_conv_prepare(ConvLayer &L, const float *w_folded_dev, hipStream_t s) {
  const int64_t total = (int64_t)kCols * nch_of(L) * L.k * nbt_of(L) * 64;
  const dim3 grd((unsigned)((total + 255) / 256));
  if (L.spec_f32)
    hipLaunchKernelGGL(k_fft_gspec<float>, grd, dim3(256), 0, s, w_folded_dev, reinterpret_cast<float *>(L.gspec),
                       L.cin, L.cout, nch_of(L), L.k, nbt_of(L));
  else
    hipLaunchKernelGGL(k_fft_gspec<bf16_t>, grd, dim3(256), 0, s, w_folded_dev, reinterpret_cast<bf16_t *>(L.gspec),
                       L.cin, L.cout, nch_of(L), L.k, nbt_of(L));
  return hipGetLastError();
}

void fft_conv_stage_cost(int stage, const ConvLayer &L, int D, int np, double *flop, double *bytes) {
  const double e = esz_of(L);
  const double npv = fft_planes(L, D, np);  // spectra per z: one per pose, or per (pose, tile)
  const double spec_in = (double)kCols * npv * D * nch_of(L) * 16 * e, spec_out = (double)kCols * npv * D * (L.cout / 8) * 16 * e;
  const double vox = (double)np * D * D * D;
  if (stage == 0) {  // 2-D real FFTs of planes zero-padded to 32 x 32: ~2.5 N^2 log2 N^2 FLOP each
    *flop = 2.5 * kN * kN * 10.0 * npv * D * L.cin;
    *bytes = vox * L.cin_pad * e + spec_in;
  } else if (stage == 1) {  // complex multiply-adds over (dz, ci) per column and output row
    *flop = 8.0 * L.cin * L.cout * L.k * D * kCols * npv;
    *bytes = spec_in + spec_out + (double)L.gspec_bytes;
  } else {
    *flop = 2.5 * kN * kN * 10.0 * npv * D * L.cout;
    *bytes = spec_out + vox * L.cout_store * e * (L.res_src >= 0 ? 2 : 1);
  }
}

bool fft_conv_fusable(const ConvLayer &L, const ConvLayer &Ln, int D) {
  // tiled layers are not fused: the next layer's windows need the neighbouring tiles
  return fft_conv_ok(L, D) && fft_conv_ok(Ln, D) && !fft_tiled(L, D) && L.cout == Ln.cin &&
         Ln.cin_pad == L.cout_store && L.spec_f32 == Ln.spec_f32;
}

hipError_t launch_fft_mid(const ConvLayer &L, const ConvLayer &Ln, const void *res, void *out, int np, int D,
                          void *work, hipStream_t s) {
  if (!fft_conv_fusable(L, Ln, D) || !work) return hipErrorInvalidValue;
  const int nch = L.cout / 8;
  const bool f32 = L.spec_f32;
  char *xs = reinterpret_cast<char *>(work);
  char *ys = xs + fft_spec_in_elems(D, np) * esz_of(L);
  const size_t spec = fft_lds_bytes(D, f32), lds = spec + ((res || out) ? (size_t)D * D * 8 * esz_of(L) : 0);
#define CF_MID3(DT, F, R, O)                                                                                  \
  hipLaunchKernelGGL((k_fft_mid<DT, F, R, O>), dim3(D, np, nch), dim3(256), lds, s, ys, L.bias, res, out, xs, np, D, \
                     nch, L.cout_store, (int)spec)
#define CF_MID2(DT, F)                                 \
  do {                                                 \
    if (res && out) CF_MID3(DT, F, true, true);        \
    else if (res) CF_MID3(DT, F, true, false);         \
    else if (out) CF_MID3(DT, F, false, true);         \
    else CF_MID3(DT, F, false, false);                 \
  } while (0)
  if (f32) {
    if (D == 24) CF_MID2(24, true); else if (D == 16) CF_MID2(16, true); else if (D == 12) CF_MID2(12, true); else CF_MID2(0, true);
  } else {
    if (D == 24) CF_MID2(24, false); else if (D == 16) CF_MID2(16, false); else if (D == 12) CF_MID2(12, false); else CF_MID2(0, false);
  }
#undef CF_MID2
#undef CF_MID3
  return hipGetLastError();
}

hipError_t launch_fft_conv(const ConvLayer &L, const void *in, const void *res, void *out, int np, int D, void *work,
                           hipStream_t s, int stage) {
  if (!fft_conv_ok(L, D) || !work) return hipErrorInvalidValue;
  const int nch = nch_of(L), nco = L.cout / 8;
  const bool f32 = L.spec_f32, tiled = fft_tiled(L, D);
  np = fft_planes(L, D, np);  // spectra per z: poses, or (pose, tile) planes
  char *xs = reinterpret_cast<char *>(work);
  char *ys = xs + fft_spec_in_elems(D, np) * esz_of(L);
  if ((stage < 0 || stage == 0) && tiled) {
#define CF_FWDT(KS, F)                                                                                      \
  hipLaunchKernelGGL((k_fft_fwd2d_t<KS, F, kTileTS>), dim3(D, np, nch), dim3(256),                            \
                     fft_lds_bytes(kTileTS + KS - 1, F), s, in, xs, np, L.cin_pad, nch)
    if (f32) {
      if (L.k == 7) CF_FWDT(7, true); else if (L.k == 5) CF_FWDT(5, true); else CF_FWDT(3, true);
    } else {
      if (L.k == 7) CF_FWDT(7, false); else if (L.k == 5) CF_FWDT(5, false); else CF_FWDT(3, false);
    }
#undef CF_FWDT
  } else if (stage < 0 || stage == 0) {
#define CF_FWD(DT, F)                                                                               \
  hipLaunchKernelGGL((k_fft_fwd2d<DT, F>), dim3(D, np, nch), dim3(256), fft_lds_bytes(D, F), s, in, xs, np, D, \
                     L.cin_pad, nch)
    if (f32) {
      if (D == 24) CF_FWD(24, true); else if (D == 16) CF_FWD(16, true); else if (D == 12) CF_FWD(12, true); else CF_FWD(0, true);
    } else {
      if (D == 24) CF_FWD(24, false); else if (D == 16) CF_FWD(16, false); else if (D == 12) CF_FWD(12, false); else CF_FWD(0, false);
    }
#undef CF_FWD
  }
  if ((stage < 0 || stage == 1) && f32) {
    const int ppb = kRowsZH / D;
    const dim3 zg((np + ppb - 1) / ppb, kCols, 1);
    const float *gp = reinterpret_cast<const float *>(L.gspec);
    const float *xf = reinterpret_cast<const float *>(xs);
    float *yf = reinterpret_cast<float *>(ys);
    const int gb = (int)L.gspec_bytes;
#define CF_ZF(KS, NB) hipLaunchKernelGGL((k_fft_zconv_f32<KS, NB>), zg, dim3(128), 0, s, xf, gp, yf, np, D, nch, ppb, gb)
    if (L.cout == 64) {
      if (L.k == 7) CF_ZF(7, 2); else if (L.k == 5) CF_ZF(5, 2); else CF_ZF(3, 2);
    } else {
      if (L.k == 7) CF_ZF(7, 1); else if (L.k == 5) CF_ZF(5, 1); else CF_ZF(3, 1);
    }
#undef CF_ZF
  } else if ((stage < 0 || stage == 1) && L.cout == 64 && (kZhRG * kRowsZH / D) * (D + L.k - 1) <= kZhRG * kPanelRowsH) {
    const int ppb = kZhRG * kRowsZH / D;
    const dim3 zg((np + ppb - 1) / ppb, kCols, 1);
    const bf16_t *gp = reinterpret_cast<const bf16_t *>(L.gspec);
    const bf16_t *xb = reinterpret_cast<const bf16_t *>(xs);
    bf16_t *yb = reinterpret_cast<bf16_t *>(ys);
    const int gb = (int)L.gspec_bytes;
    if (L.k == 7)
      hipLaunchKernelGGL((k_fft_zconv_h<7, kZhRG>), zg, dim3(128 * kZhRG), 0, s, xb, gp, yb, np, D, nch, ppb, gb);
    else if (L.k == 5)
      hipLaunchKernelGGL((k_fft_zconv_h<5, kZhRG>), zg, dim3(128 * kZhRG), 0, s, xb, gp, yb, np, D, nch, ppb, gb);
    else
      hipLaunchKernelGGL((k_fft_zconv_h<3, kZhRG>), zg, dim3(128 * kZhRG), 0, s, xb, gp, yb, np, D, nch, ppb, gb);
  } else if (stage < 0 || stage == 1) {
    const int ppb = kRowsZ / D;
    const dim3 zg((np + ppb - 1) / ppb, kCols, 1);
    const bf16_t *gp = reinterpret_cast<const bf16_t *>(L.gspec);
    const bf16_t *xb = reinterpret_cast<const bf16_t *>(xs);
    bf16_t *yb = reinterpret_cast<bf16_t *>(ys);
    const int gb = (int)L.gspec_bytes;
#define CF_ZCONV(KS, NT) \
  hipLaunchKernelGGL((k_fft_zconv<KS, NT>), zg, dim3(NT == 128 ? 256 : 128), 0, s, xb, gp, yb, np, D, nch, ppb, gb)
    const int nt = L.cout * 2;
    if (L.k == 7) {
      if (nt == 128) CF_ZCONV(7, 128); else if (nt == 64) CF_ZCONV(7, 64); else CF_ZCONV(7, 32);
    } else if (L.k == 5) {
      if (nt == 128) CF_ZCONV(5, 128); else if (nt == 64) CF_ZCONV(5, 64); else CF_ZCONV(5, 32);
    } else {
      if (nt == 128) CF_ZCONV(3, 128); else if (nt == 64) CF_ZCONV(3, 64); else CF_ZCONV(3, 32);
    }
#undef CF_ZCONV
  }
  if ((stage < 0 || stage == 2) && tiled) {
    if (f32)
      hipLaunchKernelGGL((k_fft_inv2d<kTileTS, true, 2>), dim3(D, np, nco), dim3(256), fft_lds_bytes(kTileTS, true), s,
                         ys, L.bias, res, out, np, kTileTS, nco, L.cout_store);
    else
      hipLaunchKernelGGL((k_fft_inv2d<kTileTS, false, 2>), dim3(D, np, nco), dim3(256), fft_lds_bytes(kTileTS, false),
                         s, ys, L.bias, res, out, np, kTileTS, nco, L.cout_store);
  } else if (stage < 0 || stage == 2) {
#define CF_INV(DT, F)                                                                                      \
  hipLaunchKernelGGL((k_fft_inv2d<DT, F>), dim3(D, np, nco), dim3(256), fft_lds_bytes(D, F), s, ys, L.bias, res, \
                     out, np, D, nco, L.cout_store)
    if (f32) {
      if (D == 24) CF_INV(24, true); else if (D == 16) CF_INV(16, true); else if (D == 12) CF_INV(12, true); else CF_INV(0, true);
    } else {
      if (D == 24) CF_INV(24, false); else if (D == 16) CF_INV(16, false); else if (D == 12) CF_INV(12, false); else CF_INV(0, false);
    }
#undef CF_INV
  }
  return hipGetLastError();
}

}  // namespace cf
