// conv3d as an implicit GEMM on the CDNA4 matrix cores (MFMA).
//
// The 3D-CNN head (Sec. 3.3.1, Table III) is a stack of 3-D convolutions with
// BatchNorm (folded into weights and bias at context creation), ReLU and
// residual adds; it holds >99 % of the scoring FLOPs, so it is the one place the
// path is a dense contraction: M = output voxels, N = output channels,
// K = input channels x k^3 taps.
//
// Design (per workgroup = one spatial output tile of one pose, all of N or an
// N-tile of 64/128 columns):
//   * activations are channels-last; K is walked as (channel chunk, tap).  For
//     each 16-channel chunk (bf16) or 8-channel chunk (fp32) the tile's input
//     halo is staged once in LDS (32 bytes per voxel), then all k^3 taps are read
//     from LDS as shifted windows: no im2col buffer, and each input byte is
//     fetched from L2 once per tile and chunk.
//   * LDS rows are padded by 16 bytes (so the 16 lanes of one ds_read_b128 phase
//     hit disjoint banks) and stride-2 layers store the halo parity-split per
//     axis, so consecutive output voxels stay 32 bytes apart for every tap.
//   * the weight (B) fragments are pre-packed so that one 16-byte load per lane
//     gives one MFMA operand; they stream from L2/L1 straight into VGPRs.
//   * bf16: v_mfma_f32_32x32x16_bf16, one per (32-row block, 32-column block)
//     per chunk-tap; fp32: four v_mfma_f32_32x32x2_f32 (channels stored
//     even/odd-interleaved within a chunk so a lane's four K values are
//     contiguous).  Accumulation is fp32 in both.
//   * epilogue: + folded bias, + residual tensor, ReLU, convert, store.
#include <algorithm>

#include "cf_internal.h"

namespace cf {

namespace {

template <typename T>
struct Frag;
template <>
struct Frag<bf16_t> {
  static constexpr int CC = 16;  // channels per chunk
};
template <>
struct Frag<float> {
  static constexpr int CC = 8;
};

__device__ inline int stored_index(int h, int n, int S) { return S == 1 ? h : (h & 1) * ((n + 1) >> 1) + (h >> 1); }

template <typename T, int KS, int S, int TZ, int TY, int TX, int NW, int NT>
struct ConvCfg {
  static constexpr int CC = Frag<T>::CC;
  static constexpr int PAD = (KS - 1) / 2;
  static constexpr int HZ = TZ * S + KS - S, HY = TY * S + KS - S, HX = TX * S + KS - S;
  static constexpr int ROW = HX * 32 + 16;  // bytes
  static constexpr int SLAB = HY * ROW;
  static constexpr int LDS = HZ * SLAB;
  static constexpr int MT = TZ * TY * TX;
  static constexpr int WM = MT / NW;
  static constexpr int MB = WM / 32, NB = NT / 32;
  static_assert(WM % 32 == 0, "rows per wave must be a multiple of 32");
  static_assert(LDS <= 163840, "halo exceeds LDS");
};

template <typename T, int KS, int S, int TZ, int TY, int TX, int NW, int NT>
__global__ __launch_bounds__(NW * 64) void k_conv(const T *__restrict__ in, const T *__restrict__ wpk,
                                                   const float *__restrict__ bias,
                                                   const T *__restrict__ res, T *__restrict__ out, int D,
                                                   int Do, int cin_pad, int cout_pad32, int cout,
                                                   int cout_store, int nty, int ntx, int wbytes) {
  using C = ConvCfg<T, KS, S, TZ, TY, TX, NW, NT>;
  constexpr int CC = C::CC;
  __shared__ __attribute__((aligned(16))) char lds[C::LDS];

  int tile, pose, nblk;
  xcd_order(tile, pose, nblk);
  const int n0 = nblk * NT;
  const int tz0 = (tile / (nty * ntx)) * TZ, ty0 = ((tile / ntx) % nty) * TY, tx0 = (tile % ntx) * TX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int khalf = lane >> 5, lrow = lane & 31;
  const int nchunks = cin_pad / CC;

  // per M-block LDS byte offset of this lane's output row (tap (0,0,0))
  int rowoff[C::MB];
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb) {
    const int m = wave * C::WM + mb * 32 + lrow;
    const int z = m / (TY * TX), y = (m / TX) % TY, x = m % TX;
    rowoff[mb] = z * C::SLAB + y * C::ROW + x * 32 + khalf * 16;
  }

  typedef float accv __attribute__((ext_vector_type(16)));
  accv acc[C::MB][C::NB];
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;

  const int oz = tz0 * S - C::PAD, oy = ty0 * S - C::PAD, ox = tx0 * S - C::PAD;
  const int64_t pose_in = (int64_t)pose * D * D * D;
  constexpr int HZ2 = S == 1 ? 0 : (C::HZ + 1) / 2;
  constexpr int HY2 = S == 1 ? 0 : (C::HY + 1) / 2;
  constexpr int HX2 = S == 1 ? 0 : (C::HX + 1) / 2;

  // ---- halo staging: 32 bytes per voxel; iteration `it` of a thread covers voxel
  // it * threads + tid.  All of a thread's loads are issued before the first LDS
  // store, so a chunk's staging costs about one memory latency, which the other
  // workgroup on the CU covers with its MFMAs. ----
  constexpr int NV = C::HZ * C::HY * C::HX;
  constexpr int NTH = NW * 64;
  constexpr int HITER = (NV + NTH - 1) / NTH;
  auto halo_load = [&](int it, int ch, uint4 &lo, uint4 &hi) {
    const int v = it * NTH + (int)threadIdx.x;
    lo = make_uint4(0, 0, 0, 0);
    hi = lo;
    if (v < NV) {
      const int hx = v % C::HX, hy = (v / C::HX) % C::HY, hz = v / (C::HX * C::HY);
      const int gz = oz + hz, gy = oy + hy, gx = ox + hx;
      if ((unsigned)gz < (unsigned)D && (unsigned)gy < (unsigned)D && (unsigned)gx < (unsigned)D) {
        const T *src = in + ((pose_in + ((int64_t)gz * D + gy) * D + gx) * cin_pad + ch * CC);
        lo = reinterpret_cast<const uint4 *>(src)[0];
        hi = reinterpret_cast<const uint4 *>(src)[1];
      }
    }
  };
  auto halo_store = [&](int it, uint4 lo, uint4 hi) {
    const int v = it * NTH + (int)threadIdx.x;
    if (v < NV) {
      const int hx = v % C::HX, hy = (v / C::HX) % C::HY, hz = v / (C::HX * C::HY);
      if (sizeof(T) == 4) {  // fp32: channels (0..7) -> (0,2,4,6 | 1,3,5,7)
        const uint4 a = lo, b = hi;
        lo = make_uint4(a.x, a.z, b.x, b.z);
        hi = make_uint4(a.y, a.w, b.y, b.w);
      }
      const int off = stored_index(hz, C::HZ, S) * C::SLAB + stored_index(hy, C::HY, S) * C::ROW +
                      stored_index(hx, C::HX, S) * 32;
      *reinterpret_cast<uint4 *>(lds + off) = lo;
      *reinterpret_cast<uint4 *>(lds + off + 16) = hi;
    }
  };
  const int tap_bytes = nchunks * cout_pad32 * CC * (int)sizeof(T);
  const __amdgpu_buffer_rsrc_t wrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(wpk), (short)0, wbytes, 0x00020000);
  for (int chunk = 0; chunk < nchunks; ++chunk) {
    if (chunk) __syncthreads();  // every wave is done reading the previous chunk's halo
    {
      uint4 hl[HITER], hh[HITER];
#pragma unroll
      for (int it = 0; it < HITER; ++it) halo_load(it, chunk, hl[it], hh[it]);
#pragma unroll
      for (int it = 0; it < HITER; ++it) halo_store(it, hl[it], hh[it]);
    }
    __syncthreads();
    // Taps are consecutive in the packed weights, so the B fragments of tap t+1 and
    // t+2 are in flight while tap t's MFMAs issue.  They are buffer loads with the
    // tap offset in a scalar register (no per-tap address arithmetic); reads past
    // the buffer return zero.
    int vb[C::NB];
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb)
      vb[nb] = (((chunk * cout_pad32 + n0 + nb * 32 + lrow) * CC) + khalf * (CC / 2)) * (int)sizeof(T);
    uint4 b1[C::NB], b2[C::NB];
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb) {
      b1[nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wrs, vb[nb], 0, 0));
      b2[nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wrs, vb[nb], tap_bytes, 0));
    }
    int soff = 2 * tap_bytes;
    for (int dz = 0; dz < KS; ++dz) {
      const int offz = (S == 1 ? dz : (dz & 1) * HZ2 + (dz >> 1)) * C::SLAB;
      for (int dy = 0; dy < KS; ++dy) {
        const int offzy = offz + (S == 1 ? dy : (dy & 1) * HY2 + (dy >> 1)) * C::ROW;
#pragma unroll
        for (int dx = 0; dx < KS; ++dx) {
          const int toff = offzy + (S == 1 ? dx : (dx & 1) * HX2 + (dx >> 1)) * 32;
          uint4 bfr[C::NB];
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) {
            bfr[nb] = b1[nb];
            b1[nb] = b2[nb];
            b2[nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wrs, vb[nb], soff, 0));
          }
          soff += tap_bytes;
          uint4 afr[C::MB];
#pragma unroll
          for (int mb = 0; mb < C::MB; ++mb) afr[mb] = *reinterpret_cast<const uint4 *>(lds + rowoff[mb] + toff);
#pragma unroll
          for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < C::NB; ++nb) {
              if constexpr (sizeof(T) == 2) {
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, afr[mb]), __builtin_bit_cast(bf16x8, bfr[nb]), acc[mb][nb], 0, 0, 0);
              } else {
                const float4 a = __builtin_bit_cast(float4, afr[mb]);
                const float4 b = __builtin_bit_cast(float4, bfr[nb]);
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc[mb][nb], 0, 0, 0);
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc[mb][nb], 0, 0, 0);
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc[mb][nb], 0, 0, 0);
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc[mb][nb], 0, 0, 0);
              }
            }
        }
      }
    }
  }

  // ---- epilogue: bias, residual, ReLU, store ----
  const int64_t pose_out = (int64_t)pose * Do * Do * Do;
  auto row_base = [&](int m, bool &valid) -> int64_t {
    const int z = tz0 + m / (TY * TX), y = ty0 + (m / TX) % TY, x = tx0 + m % TX;
    valid = z < Do && y < Do && x < Do;
    return (pose_out + ((int64_t)z * Do + y) * Do + x) * cout_store;
  };
  if constexpr (sizeof(T) == 2 && C::MT * NT * 2 <= C::LDS) {
    // bf16: the output tile goes through LDS so that residual reads and output
    // writes are 16-byte row segments instead of 2-byte scatters.
    bf16_t *ot = reinterpret_cast<bf16_t *>(lds);  // [MT][NT]
    constexpr int SEG = NT / 8;                       // 16-byte segments per row
    __syncthreads();                                  // halo no longer needed
    if (res) {
      for (int e = threadIdx.x; e < C::MT * SEG; e += NTH) {
        const int m = e / SEG, q = e % SEG;
        bool valid;
        const int64_t ob = row_base(m, valid);
        if (valid && n0 + q * 8 + 8 <= cout_store)
          *reinterpret_cast<uint4 *>(ot + m * NT + q * 8) = *reinterpret_cast<const uint4 *>(res + ob + n0 + q * 8);
      }
      __syncthreads();
    }
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = wave * C::WM + mb * 32 + 8 * (r >> 2) + 4 * khalf + (r & 3);
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          const int col = nb * 32 + lrow;
          float v = acc[mb][nb][r] + bias[n0 + col];
          if (res) v += (float)ot[m * NT + col];
          ot[m * NT + col] = (bf16_t)(v > 0.0f ? v : 0.0f);
        }
      }
    __syncthreads();
    for (int e = threadIdx.x; e < C::MT * SEG; e += NTH) {
      const int m = e / SEG, q = e % SEG;
      bool valid;
      const int64_t ob = row_base(m, valid);
      if (valid && n0 + q * 8 + 8 <= cout_store)
        *reinterpret_cast<uint4 *>(out + ob + n0 + q * 8) = *reinterpret_cast<const uint4 *>(ot + m * NT + q * 8);
    }
  } else {
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = wave * C::WM + mb * 32 + 8 * (r >> 2) + 4 * khalf + (r & 3);
        bool valid;
        const int64_t ob = row_base(m, valid);
        if (!valid) continue;
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          const int n = n0 + nb * 32 + lrow;
          if (n >= cout) continue;
          float v = acc[mb][nb][r] + bias[n];
          if (res) v += (float)res[ob + n];
          v = v > 0.0f ? v : 0.0f;
          out[ob + n] = (T)v;
        }
      }
    }
  }
}

// ---- bf16 with 8-channel chunks and tap pairs ---------------------------------
//
// Same implicit GEMM, but the K walk pairs two consecutive taps of one 8-channel
// chunk into each 16-deep MFMA step: lanes of the first K half read their row at
// tap 2p, lanes of the second half at tap 2p+1.  The halo then needs 16 bytes per
// voxel, so an 8x8x8 output tile (128 rows per wave, 8 MFMAs per step) fits twice
// per CU, halving the weight traffic per FLOP of the 64-row tiles; and a 19-channel
// input costs 3 chunks instead of the 2 x 16 = 32 padded channels.
//
// Two further knobs serve the 64 -> 128 stride-2 layer, whose 12^3 output tiles
// poorly and whose weights do not stay in L2: WN waves split the columns (each
// wave 64 x 64, half the weight loads per MFMA of a 32 x 128 wave), and PP poses
// share one workgroup (the same tile of consecutive poses, one halo each), so one
// pass over the weights serves PP times the rows.
template <int KS, int S, int TZ, int TY, int TX, int NW, int NT, int WN, int PP>
struct Conv8Cfg {
  static_assert(KS >= 3 && KS % 2 == 1, "odd kernel of at least 3 taps per axis");
  static constexpr int PAD = (KS - 1) / 2;
  static constexpr int HZ = TZ * S + KS - S, HY = TY * S + KS - S, HX = TX * S + KS - S;
  // Row pitch.  A 16-lane group of a 16-byte LDS read covers two 8-voxel output
  // rows; a pitch of 128 mod 256 bytes puts those rows on disjoint banks.  Taken
  // unless only a tighter pitch keeps two workgroups per CU (or fits at all):
  // then the tight pitch + 16 bytes, or without the 16 bytes as a last resort.
  static constexpr int ROW_CF = ((HX * 16 + 127) / 256) * 256 + 128, ROW_T = HX * 16 + 16;
  static constexpr int PLANES = PP * HZ * HY;
  static constexpr int ROW = (PLANES * ROW_CF <= 81920)   ? ROW_CF
                             : (PLANES * ROW_T <= 81920)  ? ROW_T
                             : (PLANES * ROW_CF <= 163840) ? ROW_CF
                             : (PLANES * ROW_T <= 163840)  ? ROW_T
                                                           : HX * 16;  // bytes
  static constexpr int SLAB = HY * ROW;
  // Rows of a 16-lane group: two runs of 8 voxels (TX = 8) YD rows apart, with YD
  // the smallest of 1, 2, 4 that puts them 128 mod 256 bytes apart (disjoint banks)
  // when the pitch itself cannot be (the tight pitch of one-workgroup halos).
  static constexpr int YD = (TX != 8 || ROW % 256 == 128)            ? 1
                            : ((2 * ROW) % 256 == 128 && TY % 4 == 0) ? 2
                            : ((4 * ROW) % 256 == 128 && TY % 8 == 0) ? 4
                                                                      : 1;
  // PP poses per workgroup (the same tile of consecutive poses): the halo of
  // pose pp sits at pp * HALO1, its rows are tile rows pp * MT1 .. + MT1.  Each
  // weight fragment then serves PP times the rows.
  static constexpr int HALO1 = HZ * SLAB, HALO = PP * HALO1;
  static constexpr int MT1 = TZ * TY * TX, MT = PP * MT1;
  // the NW waves form NWM row groups x WN column groups: wave w takes rows
  // (w / WN) * WM .. + WM and columns (w % WN) * NT / WN .. + NT / WN
  static constexpr int NWM = NW / WN;
  static constexpr int WM = MT / NWM;
  static constexpr int MB = WM / 32, NB = NT / WN / 32;
  static constexpr int TAPS = KS * KS * KS, PAIRS = (TAPS + 1) / 2;
  // epilogue: output rows go through LDS in groups of MBG 32-row blocks per row group
  static constexpr int MBG = (NWM * 32 * NT * 2 * MB <= HALO) ? MB : ((NWM * 32 * NT * 2 * 2 <= HALO && MB % 2 == 0) ? 2 : 1);
  static constexpr int EPI = NWM * 32 * MBG * NT * 2;
  static constexpr int LDS = HALO > EPI ? HALO : EPI;
  // Waves per SIMD the tile allows: a halo above half the LDS leaves one
  // workgroup per CU, so a four-wave workgroup owns its SIMDs' whole register file
  // (512 per lane); six-wave workgroups run two per CU (three waves per SIMD).
  static constexpr int WPE = (NW == 6 || NW == 12) ? 3 : ((LDS > 81920 && NW <= 4) ? 1 : 2);
  // Halo voxels each thread loads per chunk, and how many of those loads are in
  // flight at once (one batch per L2 round trip): all of them where the
  // registers allow, else batches of 6 beside 128 accumulator registers.
  static constexpr int NV1 = HZ * HY * HX, HITER = (PP * NV1 + NW * 64 - 1) / (NW * 64);
  static constexpr int HB_MAX = WPE == 1 ? 40 : (MB * NB <= 4 ? 16 : 6);
  static constexpr int HB = HITER < HB_MAX ? HITER : HB_MAX;
  static_assert(NW % WN == 0 && NT % (32 * WN) == 0, "waves split the columns in 32-column blocks");
  static_assert(WM % 32 == 0, "rows per wave must be a multiple of 32");
  static_assert(LDS <= 163840, "halo exceeds LDS");
};

// Output voxel (z, y, x) of tile row ml (one pose's tile): x fastest in runs of TX;
// with YD > 1 the y order pairs y with y + YD in consecutive runs.
template <int TY, int TX, int YD>
__device__ inline void tile_coord(int ml, int &z, int &y, int &x) {
  z = ml / (TY * TX);
  const int r = ml % (TY * TX), g = r / TX;
  x = r % TX;
  if (YD == 4)
    y = (g & ~7) + (g >> 1 & 3) + 4 * (g & 1);
  else if (YD == 2)
    y = (g & ~3) + (g >> 1 & 1) + 2 * (g & 1);
  else
    y = g;
}

template <int KS, int S, int TZ, int TY, int TX, int NW, int NT, int WN, int PP>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(Conv8Cfg<KS, S, TZ, TY, TX, NW, NT, WN, PP>::WPE))) void k_conv8(const bf16_t *__restrict__ in, const bf16_t *__restrict__ wpk,
                                                    const float *__restrict__ bias, const bf16_t *__restrict__ res,
                                                    bf16_t *__restrict__ out, int n_poses, int D, int Do, int cin_pad,
                                                    int nchunks, int cout_pad32, int cout, int cout_store, int nty,
                                                    int ntx, int wbytes) {
  using C = Conv8Cfg<KS, S, TZ, TY, TX, NW, NT, WN, PP>;
  __shared__ __attribute__((aligned(16))) char lds[C::LDS];
  int tile, pblk, nblk;
  xcd_order(tile, pblk, nblk);
  const int pose0 = pblk * PP;
  const int n0 = nblk * NT;
  const int tz0 = (tile / (nty * ntx)) * TZ, ty0 = ((tile / ntx) % nty) * TY, tx0 = (tile % ntx) * TX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wave_m = wave / WN, ncol0 = (wave % WN) * (NT / WN);
  const int khalf = lane >> 5, lrow = lane & 31;
  constexpr int NTH = NW * 64;

  int rowoff[C::MB];
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb) {
    const int m = wave_m * C::WM + mb * 32 + lrow;
    const int pp = m / C::MT1, ml = m % C::MT1;
    int z, y, x;
    tile_coord<TY, TX, C::YD>(ml, z, y, x);
    rowoff[mb] = pp * C::HALO1 + z * C::SLAB + y * C::ROW + x * 16;
  }
  typedef float accv __attribute__((ext_vector_type(16)));
  accv acc[C::MB][C::NB];
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;

  const int oz = tz0 * S - C::PAD, oy = ty0 * S - C::PAD, ox = tx0 * S - C::PAD;
  const int64_t pose_in = (int64_t)pose0 * D * D * D;
  constexpr int HZ2 = S == 1 ? 0 : (C::HZ + 1) / 2;
  constexpr int HY2 = S == 1 ? 0 : (C::HY + 1) / 2;
  constexpr int HX2 = S == 1 ? 0 : (C::HX + 1) / 2;
  constexpr int NV = PP * C::NV1;
  constexpr int HITER = C::HITER, HB = C::HB;
  auto tapoff = [&](int dz, int dy, int dx) {
    return (S == 1 ? dz : (dz & 1) * HZ2 + (dz >> 1)) * C::SLAB +
           (S == 1 ? dy : (dy & 1) * HY2 + (dy >> 1)) * C::ROW + (S == 1 ? dx : (dx & 1) * HX2 + (dx >> 1)) * 16;
  };

  // LDS offset of this lane's tap in pair p whose first tap is (z, y, x): lanes of
  // the first K half read tap 2p, the second half tap 2p + 1 (the first tap again
  // past the last tap, whose weights are zero)
  auto pair_toff = [&](int p, int z, int y, int x) {
    int ez = z, ey = y, ex = x + 1;
    if (ex == KS) {
      ex = 0;
      if (++ey == KS) {
        ey = 0;
        ++ez;
      }
    }
    const int t0 = tapoff(z, y, x);
    const int t1 = (2 * p + 1 < C::TAPS) ? tapoff(ez, ey, ex) : t0;
    return khalf ? t1 : t0;
  };
  // weight prefetch distance in pairs, even (the row fragments ping-pong inside
  // the unrolled pair loop); the packed weights carry kConvPadSteps zero pairs past
  // the end.  Several poses per workgroup means one workgroup per CU and weights
  // beyond L2 (the 64 -> 128 stride-2 layer): six pairs ahead there (5 % faster
  // than four; eight spill at 256 registers)
  constexpr int kPF = PP > 1 ? 6 : ((C::NB <= 2 && KS > 3) ? 4 : 2);
  static_assert(kPF <= kConvPadSteps, "prefetch past the weight padding");
  const int pair_bytes = nchunks * cout_pad32 * 16 * 2;
  const __amdgpu_buffer_rsrc_t wrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t *>(wpk), (short)0, wbytes, 0x00020000);
  for (int chunk = 0; chunk < nchunks; ++chunk) {
    if (chunk) __syncthreads();
    // the chunk's first channel of the workgroup's first pose (uniform); voxel
    // offsets from it fit 32 bits (PP * D^3 * cin_pad elements), which keeps the
    // per-voxel address arithmetic out of 64-bit multiplies
    const bf16_t *cin0 = in + pose_in * cin_pad + chunk * 8;
#pragma unroll
    for (int it0 = 0; it0 < HITER; it0 += HB) {
      uint4 hv[HB];
#pragma unroll
      for (int it = it0; it < it0 + HB && it < HITER; ++it) {
        const int v = it * NTH + (int)threadIdx.x;
        hv[it - it0] = make_uint4(0, 0, 0, 0);
        if (v < NV) {
          const int pp = PP == 1 ? 0 : v / C::NV1, vl = PP == 1 ? v : v % C::NV1;
          const int hx = vl % C::HX, hy = (vl / C::HX) % C::HY, hz = vl / (C::HX * C::HY);
          const int gz = oz + hz, gy = oy + hy, gx = ox + hx;
          if ((unsigned)gz < (unsigned)D && (unsigned)gy < (unsigned)D && (unsigned)gx < (unsigned)D &&
              (PP == 1 || pose0 + pp < n_poses))
            hv[it - it0] = *reinterpret_cast<const uint4 *>(cin0 + (((pp * D + gz) * D + gy) * D + gx) * cin_pad);
        }
      }
#pragma unroll
      for (int it = it0; it < it0 + HB && it < HITER; ++it) {
        const int v = it * NTH + (int)threadIdx.x;
        if (v < NV) {
          const int pp = PP == 1 ? 0 : v / C::NV1, vl = PP == 1 ? v : v % C::NV1;
          const int hx = vl % C::HX, hy = (vl / C::HX) % C::HY, hz = vl / (C::HX * C::HY);
          const int off = pp * C::HALO1 + stored_index(hz, C::HZ, S) * C::SLAB + stored_index(hy, C::HY, S) * C::ROW +
                          stored_index(hx, C::HX, S) * 16;
          *reinterpret_cast<uint4 *>(lds + off) = hv[it - it0];
        }
      }
    }
    __syncthreads();
    int vb[C::NB];
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb) vb[nb] = ((chunk * cout_pad32 + n0 + ncol0 + nb * 32 + lrow) * 16 + khalf * 8) * 2;
    // software pipeline: the weight fragments of pair p + kPF and the LDS row
    // fragments of pair p + 1 are in flight while the MFMAs of pair p issue.  The
    // pair loop is unrolled by kPF so that both rings are indexed at compile time
    // (no register moves, so no wait on the newest loads).
    uint4 bq[kPF][C::NB];
#pragma unroll
    for (int q = 0; q < kPF; ++q)
#pragma unroll
      for (int nb = 0; nb < C::NB; ++nb)
        bq[q][nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wrs, vb[nb], q * pair_bytes, 0));
    int soff = kPF * pair_bytes;
    uint4 ar[2][C::MB];
    {
      const int t0 = pair_toff(0, 0, 0, 0);
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb) ar[0][mb] = *reinterpret_cast<const uint4 *>(lds + rowoff[mb] + t0);
    }
    int dz = 0, dy = 0, dx = 2;  // first tap of pair 1
    auto pair = [&](const int p, const int ph) {
      // the last pair re-reads offset 0 of its rows (inside the halo) instead
      const int tn = (p + 1 < C::PAIRS) ? pair_toff(p + 1, dz, dy, dx) : 0;
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb) ar[(ph + 1) & 1][mb] = *reinterpret_cast<const uint4 *>(lds + rowoff[mb] + tn);
      __builtin_amdgcn_sched_barrier(0);  // keep those reads ahead of this pair's MFMAs
      dx += 2;
      if (dx >= KS) {
        dx -= KS;
        if (++dy == KS) {
          dy = 0;
          ++dz;
        }
      }
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ar[ph & 1][mb]),
                                                                 __builtin_bit_cast(bf16x8, bq[ph][nb]), acc[mb][nb],
                                                                 0, 0, 0);
#pragma unroll
      for (int nb = 0; nb < C::NB; ++nb)
        bq[ph][nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wrs, vb[nb], soff, 0));
      soff += pair_bytes;
    };
    // whole groups of kPF pairs with no test inside (so that the compiler's wait
    // analysis keeps every weight load of the ring in flight), then the rest
    constexpr int kFull = C::PAIRS / kPF * kPF;
    for (int p0 = 0; p0 < kFull; p0 += kPF) {
#pragma unroll
      for (int ph = 0; ph < kPF; ++ph) pair(p0 + ph, ph);
    }
#pragma unroll
    for (int ph = 0; ph < kPF; ++ph)
      if (kFull + ph < C::PAIRS) pair(kFull + ph, ph);
  }

  // ---- epilogue through LDS, MBG row blocks per wave at a time ----
  const int64_t pose_out = (int64_t)pose0 * Do * Do * Do;
  auto row_base = [&](int m, bool &valid) -> int64_t {
    const int pp = m / C::MT1, ml = m % C::MT1;
    int z, y, x;
    tile_coord<TY, TX, C::YD>(ml, z, y, x);
    z += tz0;
    y += ty0;
    x += tx0;
    valid = z < Do && y < Do && x < Do && (PP == 1 || pose0 + pp < n_poses);
    return (pose_out + (((int64_t)pp * Do + z) * Do + y) * Do + x) * cout_store;
  };
  bf16_t *ot = reinterpret_cast<bf16_t *>(lds);  // [NWM][MBG*32][NT]
  constexpr int SEG = NT / 8;
  constexpr int GR = C::MBG * 32;  // rows per row group per epilogue group
  // local row lr of group g -> tile row (lr / GR) * WM + (g + (lr % GR) / 32) * 32 + lr % 32
#pragma unroll
  for (int g = 0; g < C::MB; g += C::MBG) {
    __syncthreads();
    if (res) {
      for (int e = threadIdx.x; e < C::NWM * GR * SEG; e += NTH) {
        const int lr = e / SEG, q = e % SEG;
        const int m = (lr / GR) * C::WM + g * 32 + lr % GR;
        bool valid;
        const int64_t ob = row_base(m, valid);
        if (valid && n0 + q * 8 + 8 <= cout_store)
          *reinterpret_cast<uint4 *>(ot + lr * NT + q * 8) = *reinterpret_cast<const uint4 *>(res + ob + n0 + q * 8);
      }
      __syncthreads();
    }
#pragma unroll
    for (int mb = g; mb < g + C::MBG; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int lr = wave_m * GR + (mb - g) * 32 + 8 * (r >> 2) + 4 * khalf + (r & 3);
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          const int col = ncol0 + nb * 32 + lrow;
          float v = acc[mb][nb][r] + bias[n0 + col];
          if (res) v += (float)ot[lr * NT + col];
          ot[lr * NT + col] = (bf16_t)(v > 0.0f ? v : 0.0f);
        }
      }
    __syncthreads();
    for (int e = threadIdx.x; e < C::NWM * GR * SEG; e += NTH) {
      const int lr = e / SEG, q = e % SEG;
      const int m = (lr / GR) * C::WM + g * 32 + lr % GR;
      bool valid;
      const int64_t ob = row_base(m, valid);
      if (valid && n0 + q * 8 + 8 <= cout_store)
        *reinterpret_cast<uint4 *>(out + ob + n0 + q * 8) = *reinterpret_cast<const uint4 *>(ot + lr * NT + q * 8);
    }
  }
}

// ---- bf16 with 4-channel chunks and tap quads -----------------------------------
//
// For inputs whose channel count leaves much of an 8-channel chunk empty (the
// 19-channel grid: 24 padded channels, 21 % zeros) the K walk takes 4 channels x 4
// taps per 16-deep MFMA step: lanes of the first K half read taps 4q and 4q + 1,
// the second half 4q + 2 and 4q + 3, 8 bytes (4 channels) each.  19 channels cost
// 20, and the halo needs 8 bytes per voxel, so the 21^3 halo of an 8^3 stride-2
// tile fits twice per CU.  Tap offsets come from a table in LDS.
template <int KS, int S, int TZ, int TY, int TX, int NW, int NT>
struct Conv4Cfg {
  static_assert(KS >= 3 && KS % 2 == 1, "odd kernel of at least 3 taps per axis");
  static constexpr int PAD = (KS - 1) / 2;
  static constexpr int HZ = TZ * S + KS - S, HY = TY * S + KS - S, HX = TX * S + KS - S;
  static constexpr int ROW = HX * 8 + 8, SLAB = HY * ROW, HALO = HZ * SLAB;  // bytes
  static constexpr int TAPS = KS * KS * KS, QUADS = (TAPS + 3) / 4, TAB = QUADS * 4 * 4;
  static constexpr int MT = TZ * TY * TX, WM = MT / NW, MB = WM / 32, NB = NT / 32;
  static constexpr int MBG = (NW * 32 * NT * 2 * MB <= HALO) ? MB : ((NW * 32 * NT * 2 * 2 <= HALO && MB % 2 == 0) ? 2 : 1);
  static constexpr int EPI = NW * 32 * MBG * NT * 2;
  static constexpr int LDS = TAB + (HALO > EPI ? HALO : EPI);
  static constexpr int WPE = LDS > 81920 ? 1 : 2;
  static constexpr int HITER = (HZ * HY * HX + NW * 64 - 1) / (NW * 64);
  // halo loads in flight per batch (one round trip each): all of them up to 20
  // voxels per thread, else two batches (the 21^3 halo of the first layer: 37
  // voxels per thread in 19 + 18 instead of batches of 8, 4-5 % faster)
  static constexpr int HB = HITER <= 20 ? HITER : (HITER + 1) / 2;
  static_assert(WM % 32 == 0, "rows per wave must be a multiple of 32");
  static_assert(LDS <= 163840, "halo exceeds LDS");
};

template <int KS, int S, int TZ, int TY, int TX, int NW, int NT>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(Conv4Cfg<KS, S, TZ, TY, TX, NW, NT>::WPE))) void k_conv4(
    const bf16_t *__restrict__ in, const bf16_t *__restrict__ wpk, const float *__restrict__ bias,
    const bf16_t *__restrict__ res, bf16_t *__restrict__ out, int D, int Do, int cin_pad, int nchunks, int cout_pad32,
    int cout_store, int nty, int ntx, int wbytes, int chunk_major) {
  using C = Conv4Cfg<KS, S, TZ, TY, TX, NW, NT>;
  __shared__ __attribute__((aligned(16))) char lds[C::LDS];
  int *tab = reinterpret_cast<int *>(lds);  // [QUADS * 4] tap offsets into the halo
  char *halo = lds + C::TAB;
  int tile, pose, nblk;
  xcd_order(tile, pose, nblk);
  const int n0 = nblk * NT;
  const int tz0 = (tile / (nty * ntx)) * TZ, ty0 = ((tile / ntx) % nty) * TY, tx0 = (tile % ntx) * TX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int khalf = lane >> 5, lrow = lane & 31;
  constexpr int NTH = NW * 64;
  constexpr int HZ2 = (C::HZ + 1) / 2, HY2 = (C::HY + 1) / 2, HX2 = (C::HX + 1) / 2;
  for (int t = threadIdx.x; t < C::QUADS * 4; t += NTH) {
    int off = 0;  // taps past the last read offset 0 (their weights are zero)
    if (t < C::TAPS) {
      const int dz = t / (KS * KS), dy = (t / KS) % KS, dx = t % KS;
      off = (S == 1 ? dz : (dz & 1) * HZ2 + (dz >> 1)) * C::SLAB + (S == 1 ? dy : (dy & 1) * HY2 + (dy >> 1)) * C::ROW +
            (S == 1 ? dx : (dx & 1) * HX2 + (dx >> 1)) * 8;
    }
    tab[t] = off;
  }
  int rowoff[C::MB];
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb) {
    const int m = wave * C::WM + mb * 32 + lrow;
    const int z = m / (TY * TX), y = (m / TX) % TY, x = m % TX;
    rowoff[mb] = z * C::SLAB + y * C::ROW + x * 8;
  }
  typedef float accv __attribute__((ext_vector_type(16)));
  accv acc[C::MB][C::NB];
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;
  const int oz = tz0 * S - C::PAD, oy = ty0 * S - C::PAD, ox = tx0 * S - C::PAD;
  const int64_t pose_in = (int64_t)pose * D * D * D;
  constexpr int NV = C::HZ * C::HY * C::HX;
  constexpr int kPF = 4;  // weights stay in L2 here: six quads ahead measured 6 % slower
  static_assert(kPF <= kConvPadSteps, "prefetch past the weight padding");
  const int quad_bytes = nchunks * cout_pad32 * 16 * 2;
  const __amdgpu_buffer_rsrc_t wrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t *>(wpk), (short)0, wbytes, 0x00020000);
  for (int chunk = 0; chunk < nchunks; ++chunk) {
    __syncthreads();  // the table is written / the previous chunk's halo is read
    // the chunk's channels of this pose (uniform) and the elements per voxel: voxel
    // offsets from there fit 32 bits, which keeps the per-voxel address arithmetic
    // out of 64-bit multiplies
    const bf16_t *cin0 = chunk_major ? in + ((int64_t)pose * nchunks + chunk) * D * D * D * 4
                                     : in + pose_in * cin_pad + chunk * 4;
    const int vstride = chunk_major ? 4 : cin_pad;
    // batches of HB loads in flight; the batch loop is not unrolled, so the halo
    // addressing is recomputed per chunk rather than hoisted and held in registers
#pragma unroll 1
    for (int it0 = 0; it0 < C::HITER; it0 += C::HB) {
      uint2 hv[C::HB];  // static indices only, so the batch stays in registers
#pragma unroll
      for (int i = 0; i < C::HB; ++i) {
        const int v = (it0 + i) * NTH + (int)threadIdx.x;
        hv[i] = make_uint2(0, 0);
        if (it0 + i < C::HITER && v < NV) {
          const int hx = v % C::HX, hy = (v / C::HX) % C::HY, hz = v / (C::HX * C::HY);
          const int gz = oz + hz, gy = oy + hy, gx = ox + hx;
          if ((unsigned)gz < (unsigned)D && (unsigned)gy < (unsigned)D && (unsigned)gx < (unsigned)D)
            hv[i] = *reinterpret_cast<const uint2 *>(cin0 + ((gz * D + gy) * D + gx) * vstride);
        }
      }
#pragma unroll
      for (int i = 0; i < C::HB; ++i) {
        const int v = (it0 + i) * NTH + (int)threadIdx.x;
        if (it0 + i < C::HITER && v < NV) {
          const int hx = v % C::HX, hy = (v / C::HX) % C::HY, hz = v / (C::HX * C::HY);
          const int off = stored_index(hz, C::HZ, S) * C::SLAB + stored_index(hy, C::HY, S) * C::ROW +
                          stored_index(hx, C::HX, S) * 8;
          *reinterpret_cast<uint2 *>(halo + off) = hv[i];
        }
      }
    }
    __syncthreads();
    int vb[C::NB];
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb) vb[nb] = ((chunk * cout_pad32 + n0 + nb * 32 + lrow) * 16 + khalf * 8) * 2;
    uint4 bq[kPF][C::NB];
#pragma unroll
    for (int q = 0; q < kPF; ++q)
#pragma unroll
      for (int nb = 0; nb < C::NB; ++nb)
        bq[q][nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wrs, vb[nb], q * quad_bytes, 0));
    int soff = kPF * quad_bytes;
    // row fragments one quad ahead: two 8-byte reads per row block (taps t, t + 1)
    uint4 ar[2][C::MB];
    {
      const int t0 = tab[2 * khalf], t1 = tab[2 * khalf + 1];
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb) {
        const uint2 lo = *reinterpret_cast<const uint2 *>(halo + rowoff[mb] + t0);
        const uint2 hi = *reinterpret_cast<const uint2 *>(halo + rowoff[mb] + t1);
        ar[0][mb] = make_uint4(lo.x, lo.y, hi.x, hi.y);
      }
    }
    auto quad = [&](const int q, const int ph) {
      const int qn = q + 1 < C::QUADS ? q + 1 : q;
      const int t0 = tab[4 * qn + 2 * khalf], t1 = tab[4 * qn + 2 * khalf + 1];
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb) {
        const uint2 lo = *reinterpret_cast<const uint2 *>(halo + rowoff[mb] + t0);
        const uint2 hi = *reinterpret_cast<const uint2 *>(halo + rowoff[mb] + t1);
        ar[(ph + 1) & 1][mb] = make_uint4(lo.x, lo.y, hi.x, hi.y);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ar[ph & 1][mb]),
                                                                 __builtin_bit_cast(bf16x8, bq[ph][nb]), acc[mb][nb],
                                                                 0, 0, 0);
#pragma unroll
      for (int nb = 0; nb < C::NB; ++nb)
        bq[ph][nb] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wrs, vb[nb], soff, 0));
      soff += quad_bytes;
    };
    // whole groups of kPF quads with no test inside (so that the compiler's wait
    // analysis keeps every weight load of the ring in flight), then the rest
    constexpr int kFull = C::QUADS / kPF * kPF;
    for (int q0 = 0; q0 < kFull; q0 += kPF) {
#pragma unroll
      for (int ph = 0; ph < kPF; ++ph) quad(q0 + ph, ph);
    }
#pragma unroll
    for (int ph = 0; ph < kPF; ++ph)
      if (kFull + ph < C::QUADS) quad(kFull + ph, ph);
  }

  // ---- epilogue through LDS (as k_conv8) ----
  const int64_t pose_out = (int64_t)pose * Do * Do * Do;
  auto row_base = [&](int m, bool &valid) -> int64_t {
    const int z = tz0 + m / (TY * TX), y = ty0 + (m / TX) % TY, x = tx0 + m % TX;
    valid = z < Do && y < Do && x < Do;
    return (pose_out + ((int64_t)z * Do + y) * Do + x) * cout_store;
  };
  bf16_t *ot = reinterpret_cast<bf16_t *>(halo);  // [NW][MBG*32][NT]
  constexpr int SEG = NT / 8;
  constexpr int GR = C::MBG * 32;
#pragma unroll
  for (int g = 0; g < C::MB; g += C::MBG) {
    __syncthreads();
    if (res) {
      for (int e = threadIdx.x; e < NW * GR * SEG; e += NTH) {
        const int lr = e / SEG, qq = e % SEG;
        const int m = (lr / GR) * C::WM + g * 32 + lr % GR;
        bool valid;
        const int64_t ob = row_base(m, valid);
        if (valid && n0 + qq * 8 + 8 <= cout_store)
          *reinterpret_cast<uint4 *>(ot + lr * NT + qq * 8) = *reinterpret_cast<const uint4 *>(res + ob + n0 + qq * 8);
      }
      __syncthreads();
    }
#pragma unroll
    for (int mb = g; mb < g + C::MBG; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int lr = wave * GR + (mb - g) * 32 + 8 * (r >> 2) + 4 * khalf + (r & 3);
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          const int col = nb * 32 + lrow;
          float v = acc[mb][nb][r] + bias[n0 + col];
          if (res) v += (float)ot[lr * NT + col];
          ot[lr * NT + col] = (bf16_t)(v > 0.0f ? v : 0.0f);
        }
      }
    __syncthreads();
    for (int e = threadIdx.x; e < NW * GR * SEG; e += NTH) {
      const int lr = e / SEG, qq = e % SEG;
      const int m = (lr / GR) * C::WM + g * 32 + lr % GR;
      bool valid;
      const int64_t ob = row_base(m, valid);
      if (valid && n0 + qq * 8 + 8 <= cout_store)
        *reinterpret_cast<uint4 *>(out + ob + n0 + qq * 8) = *reinterpret_cast<const uint4 *>(ot + lr * NT + qq * 8);
    }
  }
}

template <int KS, int S, int TZ, int TY, int TX, int NW, int NT>
hipError_t launch_q(const ConvLayer &L, const void *in, const void *res, void *out, int n_poses, int D,
                    hipStream_t s) {
  const int Do = (D + 2 * ((KS - 1) / 2) - KS) / S + 1;
  const int ntz = (Do + TZ - 1) / TZ, nty = (Do + TY - 1) / TY, ntx = (Do + TX - 1) / TX;
  const dim3 grid(ntz * nty * ntx, n_poses, L.cout_pad32 / NT);
  hipLaunchKernelGGL((k_conv4<KS, S, TZ, TY, TX, NW, NT>), grid, dim3(NW * 64), 0, s,
                     reinterpret_cast<const bf16_t *>(in), reinterpret_cast<const bf16_t *>(L.wpk4), L.bias,
                     reinterpret_cast<const bf16_t *>(res), reinterpret_cast<bf16_t *>(out), D, Do, L.cin_pad,
                     (L.cin + 3) / 4, L.cout_pad32, L.cout_store, nty, ntx, (int)L.wbytes4, L.in_cm4);
  return hipGetLastError();
}

struct Variant {
  const char *name;
  int ks, s, tz, ty, tx, nw, nt;
  int pairs;  // 1: bf16 8-channel tap-pair kernel (k_conv8, weights in wpk8); 2: 4-channel tap quads (k_conv4, wpk4)
  hipError_t (*launch_bf16)(const ConvLayer &, const void *, const void *, void *, int, int, hipStream_t);
  hipError_t (*launch_f32)(const ConvLayer &, const void *, const void *, void *, int, int, hipStream_t);
};

template <int KS, int S, int TZ, int TY, int TX, int NW, int NT, int WN, int PP>
hipError_t launch_p(const ConvLayer &L, const void *in, const void *res, void *out, int n_poses, int D,
                    hipStream_t s) {
  const int Do = (D + 2 * ((KS - 1) / 2) - KS) / S + 1;
  const int ntz = (Do + TZ - 1) / TZ, nty = (Do + TY - 1) / TY, ntx = (Do + TX - 1) / TX;
  const dim3 grid(ntz * nty * ntx, (n_poses + PP - 1) / PP, L.cout_pad32 / NT);
  hipLaunchKernelGGL((k_conv8<KS, S, TZ, TY, TX, NW, NT, WN, PP>), grid, dim3(NW * 64), 0, s,
                     reinterpret_cast<const bf16_t *>(in), reinterpret_cast<const bf16_t *>(L.wpk8), L.bias,
                     reinterpret_cast<const bf16_t *>(res), reinterpret_cast<bf16_t *>(out), n_poses, D, Do, L.cin_pad,
                     (L.cin + 7) / 8, L.cout_pad32, L.cout, L.cout_store, nty, ntx, (int)L.wbytes8);
  return hipGetLastError();
}

template <typename T, int KS, int S, int TZ, int TY, int TX, int NW, int NT>
hipError_t launch_t(const ConvLayer &L, const void *in, const void *res, void *out, int n_poses, int D,
                    hipStream_t s) {
  const int Do = (D + 2 * ((KS - 1) / 2) - KS) / S + 1;
  const int ntz = (Do + TZ - 1) / TZ, nty = (Do + TY - 1) / TY, ntx = (Do + TX - 1) / TX;
  const dim3 grid(ntz * nty * ntx, n_poses, L.cout_pad32 / NT);
  hipLaunchKernelGGL((k_conv<T, KS, S, TZ, TY, TX, NW, NT>), grid, dim3(NW * 64), 0, s,
                     reinterpret_cast<const T *>(in), reinterpret_cast<const T *>(L.wpk), L.bias,
                     reinterpret_cast<const T *>(res), reinterpret_cast<T *>(out), D, Do, L.cin_pad,
                     L.cout_pad32, L.cout, L.cout_store, nty, ntx, (int)L.wbytes);
  return hipGetLastError();
}

#define CF_VARIANT(KS, S, TZ, TY, TX, NW, NT)                                                 \
  Variant {                                                                                   \
    "k" #KS "s" #S "_t" #TZ "x" #TY "x" #TX "_w" #NW "_n" #NT, KS, S, TZ, TY, TX, NW, NT, 0,   \
        &launch_t<bf16_t, KS, S, TZ, TY, TX, NW, NT>, &launch_t<float, KS, S, TZ, TY, TX, NW, NT> \
  }
#define CF_VARIANT8(KS, S, TZ, TY, TX, NW, NT)                                                   \
  Variant {                                                                                      \
    "p8k" #KS "s" #S "_t" #TZ "x" #TY "x" #TX "_w" #NW "_n" #NT, KS, S, TZ, TY, TX, NW, NT, 1,   \
        &launch_p<KS, S, TZ, TY, TX, NW, NT, 1, 1>, nullptr                                      \
  }
// WN waves across the columns (each wave: NT / WN columns of its row group)
#define CF_VARIANT8N(KS, S, TZ, TY, TX, NW, NT, WN)                                                      \
  Variant {                                                                                              \
    "p8k" #KS "s" #S "_t" #TZ "x" #TY "x" #TX "_w" #NW "c" #WN "_n" #NT, KS, S, TZ, TY, TX, NW, NT, 1,   \
        &launch_p<KS, S, TZ, TY, TX, NW, NT, WN, 1>, nullptr                                             \
  }
#define CF_VARIANT4(KS, S, TZ, TY, TX, NW, NT)                                                   \
  Variant {                                                                                      \
    "q4k" #KS "s" #S "_t" #TZ "x" #TY "x" #TX "_w" #NW "_n" #NT, KS, S, TZ, TY, TX, NW, NT, 2,   \
        &launch_q<KS, S, TZ, TY, TX, NW, NT>, nullptr                                            \
  }
// ... and PP poses per workgroup
#define CF_VARIANT8P(KS, S, TZ, TY, TX, NW, NT, WN, PP)                                                           \
  Variant {                                                                                                       \
    "p8k" #KS "s" #S "_t" #TZ "x" #TY "x" #TX "_w" #NW "c" #WN "_n" #NT "_p" #PP, KS, S, TZ, TY, TX, NW, NT, 1,   \
        &launch_p<KS, S, TZ, TY, TX, NW, NT, WN, PP>, nullptr                                                     \
  }

const Variant kVariants[] = {
    CF_VARIANT(7, 1, 8, 8, 8, 4, 64),   // 0: full-model residual layers
    CF_VARIANT(7, 1, 4, 8, 8, 4, 64),   // 1
    CF_VARIANT(7, 1, 8, 8, 8, 8, 64),   // 2
    CF_VARIANT(7, 2, 4, 4, 8, 4, 64),   // 3: stride-2 layers
    CF_VARIANT(7, 2, 4, 4, 8, 4, 128),  // 4
    CF_VARIANT(7, 2, 2, 8, 8, 4, 64),   // 5
    CF_VARIANT(5, 1, 8, 8, 8, 4, 32),   // 6: tiny model
    CF_VARIANT(5, 1, 4, 8, 8, 4, 32),   // 7
    CF_VARIANT(7, 1, 4, 8, 8, 2, 64),   // 8: 128 rows per wave, two workgroups per CU
    CF_VARIANT(7, 2, 4, 4, 8, 2, 64),   // 9
    CF_VARIANT(7, 2, 4, 4, 8, 2, 128),  // 10
    CF_VARIANT(7, 2, 2, 8, 8, 2, 64),   // 11
    CF_VARIANT8(7, 1, 8, 8, 8, 4, 64),  // 12: tap pairs, 128 rows per wave
    CF_VARIANT8(7, 1, 4, 8, 8, 4, 64),  // 13
    CF_VARIANT8(7, 1, 4, 8, 8, 2, 64),  // 14
    CF_VARIANT8(7, 2, 4, 4, 8, 4, 64),  // 15
    CF_VARIANT8(7, 2, 4, 8, 8, 4, 64),  // 16
    CF_VARIANT8(7, 2, 4, 4, 8, 4, 128), // 17
    CF_VARIANT8(7, 2, 4, 8, 8, 4, 128), // 18
    CF_VARIANT8(5, 1, 8, 8, 8, 4, 32),  // 19
    CF_VARIANT8(7, 2, 8, 8, 8, 4, 64),  // 20: stride-2 first layer, 512-row tile
    CF_VARIANT8(7, 1, 8, 8, 8, 8, 64),  // 21
    CF_VARIANT8(7, 2, 4, 4, 12, 6, 128), // 22: 12^3 outputs of a 24^3 input in 9 whole tiles
    // 5^3 and 3^3 kernels (the paper-shaped model: 32 filters of 5^3, 64 of 3^3)
    CF_VARIANT8(5, 2, 8, 8, 8, 4, 32),   // 23
    CF_VARIANT8(5, 2, 4, 8, 8, 4, 32),   // 24
    CF_VARIANT8(5, 1, 4, 8, 8, 2, 32),   // 25
    CF_VARIANT8(3, 1, 8, 8, 8, 4, 64),   // 26
    CF_VARIANT8(3, 1, 4, 8, 8, 4, 64),   // 27
    CF_VARIANT8(3, 2, 8, 8, 8, 4, 64),   // 28
    CF_VARIANT8(3, 2, 4, 8, 8, 4, 64),   // 29
    CF_VARIANT(5, 2, 4, 8, 8, 4, 32),    // 30
    CF_VARIANT(3, 1, 8, 8, 8, 4, 64),    // 31
    CF_VARIANT(3, 1, 4, 8, 8, 4, 64),    // 32
    CF_VARIANT(3, 2, 4, 8, 8, 4, 64),    // 33
    CF_VARIANT(3, 2, 4, 4, 8, 4, 64),    // 34
    // stride-2 tiles whose halo allows one workgroup per CU: eight waves hide more latency
    CF_VARIANT8(7, 2, 8, 8, 8, 8, 64),   // 35
    CF_VARIANT8(7, 2, 4, 8, 8, 8, 128),  // 36
    CF_VARIANT8(5, 2, 8, 8, 8, 8, 32),   // 37
    // 128-column stride-2 layers with the columns split over two waves (64 rows x
    // 64 columns per wave: half the weight-fragment loads per MFMA of 17/22)
    CF_VARIANT8N(7, 2, 4, 4, 12, 6, 128, 2),  // 38: 12^3 outputs in 9 whole tiles
    CF_VARIANT8N(7, 2, 4, 4, 8, 4, 128, 2),   // 39
    // two poses per workgroup: 384 rows share each weight fragment (the 5.6 MB of
    // weights of the 64 -> 128 layer exceed an XCD's L2, so weight traffic per row
    // sets its speed); 12^3 outputs in 9 whole tiles
    CF_VARIANT8P(7, 2, 4, 4, 12, 8, 128, 2, 2),   // 40
    // 4-channel tap quads for the 19-channel grid
    CF_VARIANT4(7, 2, 8, 8, 8, 4, 64),   // 41: 21^3 halo at 8 bytes per voxel, two workgroups per CU
    CF_VARIANT4(5, 2, 8, 8, 8, 4, 32),   // 42
    CF_VARIANT4(5, 1, 8, 8, 8, 4, 32),   // 43
    CF_VARIANT4(7, 1, 8, 8, 8, 4, 32),   // 44  (the bf16 grid is read by tap-quad kernels only: one per
    CF_VARIANT4(3, 1, 8, 8, 8, 4, 32),   // 45   first-layer shape)
    CF_VARIANT4(3, 2, 8, 8, 8, 4, 32)    // 46
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

// one more variant id past the direct kernels: the frequency-domain path
constexpr int kFftVariant = kNumVariants;

int conv_num_variants() { return kNumVariants + 1; }
const char *conv_variant_name(int v) {
  return (v >= 0 && v < kNumVariants) ? kVariants[v].name : (v == kFftVariant ? "fft32" : "?");
}

bool conv_variant_ok(int v, const ConvLayer &L, int bf16, int D_in) {
  if (v == kFftVariant) return (bf16 ? !L.spec_f32 : L.spec_f32) && fft_conv_ok(L, D_in);
  if (v < 0 || v >= kNumVariants) return false;
  const Variant &V = kVariants[v];
  if (V.pairs == 2) return bf16 && L.wpk4 && V.ks == L.k && V.s == L.stride && L.cout_pad32 % V.nt == 0 && L.cin_pad % 4 == 0;
  if (V.pairs) return bf16 && L.wpk8 && V.ks == L.k && V.s == L.stride && L.cout_pad32 % V.nt == 0 && L.cin_pad % 8 == 0;
  const int cc = bf16 ? 16 : 8;
  return V.ks == L.k && V.s == L.stride && L.cout_pad32 % V.nt == 0 && L.cin_pad % cc == 0;
}

int conv_default_variant(const ConvLayer &L, int D_in, int bf16) {
  // measured on MI355X at 48^3: 7^3 stride-1 layers in the frequency domain (bf16:
  // 3x the tap-pair kernel), tap quads for the 19-channel first layer, tap pairs
  // for the 128-column stride-2 layer (two poses per workgroup); fp32 has no tap
  // kernels
  if (L.k == 7 && conv_variant_ok(kFftVariant, L, bf16, D_in)) return kFftVariant;
  const int pref[] = {12, 40, 41, 17, 20, 19, 23, 26, 28, 4, 3, 6, 1, 0, 2, 5, 7, 8, 9, 10, 11, 13, 14, 15, 16, 18,
                      21, 22, 24, 25, 27, 29, 30, 31, 32, 33, 34, 35, 36, 37, 38, 39, 42, 43, 44, 45, 46};
  for (int v : pref)
    if (conv_variant_ok(v, L, bf16, D_in)) return v;
  return -1;
}

bool conv_variant_is_fft(int v) { return v == kFftVariant; }

int64_t conv_work_bytes(int v, const ConvLayer &L, int D_in, int n_poses) {
  return v == kFftVariant ? fft_conv_work_bytes(L, D_in, n_poses) : 0;
}

namespace {
// Seeded values uniform in [0, 0.5) (SplitMix64 finaliser of seed + index): the
// autotuner times kernels on data that toggles like real activations, since
// the chip sustains a higher clock on constant operands.
__global__ __launch_bounds__(256) void k_fill_random(void *p, int64_t n, int bf16, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const float v = (float)(z >> 40) * (0.5f / 16777216.0f);
    if (bf16)
      reinterpret_cast<bf16_t *>(p)[i] = (bf16_t)v;
    else
      reinterpret_cast<float *>(p)[i] = v;
  }
}
}  // namespace

hipError_t launch_fill_random(void *p, int64_t bytes, int bf16, uint64_t seed, hipStream_t s) {
  const int64_t n = bytes / (bf16 ? 2 : 4);
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_fill_random, dim3((unsigned)blocks), dim3(256), 0, s, p, n, bf16, seed);
  return hipGetLastError();
}

hipError_t launch_conv(int variant, const ConvLayer &L, int bf16, const void *in, const void *res,
                       void *out, int n_poses, int D_in, void *work, hipStream_t s) {
  if (!conv_variant_ok(variant, L, bf16, D_in)) return hipErrorInvalidValue;
  if (variant == kFftVariant) return launch_fft_conv(L, in, res, out, n_poses, D_in, work, s);
  const Variant &V = kVariants[variant];
  return bf16 ? V.launch_bf16(L, in, res, out, n_poses, D_in, s) : V.launch_f32(L, in, res, out, n_poses, D_in, s);
}

}  // namespace cf
