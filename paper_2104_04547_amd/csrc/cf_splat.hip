// Pose centres and Gaussian atom splatting into channels-last voxel grids.
//
// Voxelisation is the 3D-CNN's input representation (Sec. 1); its sizing and
// atom propagation are taken from the predecessor model (Sec. 3.3).  Here: 1 A
// voxels centred on the pose centre, Gaussian weights exp(-d^2 / 2 sigma^2) with
// sigma = 0.5 A truncated at 3 sigma, normalised per atom over its whole support.
//
// Design: a binning pass, then one workgroup per (pose, 2 x 4 x G tile).
//   * k_splat_bin (one workgroup per pose): each atom's support box (at most 4
//     voxels per axis) reaches at most 3 x 2 tiles; the atoms are counted per tile,
//     the counts scanned and the atoms listed per tile (the order inside a list
//     does not matter, see below), and each atom's normaliser -- the sum of its
//     weights over the whole (unclipped) support -- is computed once, by one wave
//     per atom, one candidate voxel per lane, as an exact integer reduction.
//   * k_splat: the tile's accumulators sit in LDS as 2^20 fixed-point int32, so
//     the atomics are exact and the result does not depend on the order in which
//     waves add contributions.  The list is dealt to the four waves in turn (one
//     atom per lane) and each wave sweeps its atoms one after another: an atom's candidate
//     voxels form at most a 4 x 4 x 4 box, one per lane, and the adds are
//     wavefront-wide LDS atomics.  The finished tile is streamed to HBM once.
// Results are bitwise independent of launch shape, list order and atom
// scheduling, so a 90 degree rotation of a pose permutes its grid exactly.
#include "cf_internal.h"

namespace cf {

namespace {

constexpr int kTA = 2, kTB = 4;   // tile extent along grid axes 0 and 1 (axis 2 whole)
constexpr int kRcut = 1536;       // 3 sigma in u
constexpr float kInv2s2 = 1.0f / 524288.0f;

__device__ inline int64_t floordiv(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

// value of lane b (wave-uniform b)
__device__ inline int rdlane(int v, int b) { return __builtin_amdgcn_readlane(v, b); }
__device__ inline int64_t rdlane64(int64_t v, int b) {
  const uint32_t lo = (uint32_t)rdlane((int)(uint32_t)v, b), hi = (uint32_t)rdlane((int)(uint32_t)(v >> 32), b);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(64) void k_centers(const int32_t *__restrict__ atom_off, int n_atoms,
                                                const int32_t *__restrict__ xyz,
                                                const uint8_t *__restrict__ is_lig, int p0,
                                                int32_t *__restrict__ center_out, int64_t *status) {
  const int p = p0 + blockIdx.x;
  int a0, a1;
  if (!pose_range(atom_off, p, n_atoms, a0, a1) && threadIdx.x == 0) dev_fail(status, kDevBadOffsets);
  int64_t s[3] = {0, 0, 0}, sa[3] = {0, 0, 0};
  int n = 0, na = 0;
  for (int a = a0 + threadIdx.x; a < a1; a += 64) {
    const int l = is_lig[a] != 0;
    for (int d = 0; d < 3; ++d) {
      const int64_t x = xyz[3 * a + d];
      sa[d] += x;
      if (l) s[d] += x;
    }
    n += l;
    na += 1;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    for (int d = 0; d < 3; ++d) {
      s[d] += __shfl_xor(s[d], o, 64);
      sa[d] += __shfl_xor(sa[d], o, 64);
    }
    n += __shfl_xor(n, o, 64);
    na += __shfl_xor(na, o, 64);
  }
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    const int64_t sd = d == 0 ? s[0] : (d == 1 ? s[1] : s[2]);
    const int64_t sad = d == 0 ? sa[0] : (d == 1 ? sa[1] : sa[2]);
    const int64_t S = n > 0 ? sd : sad;
    const int64_t N = n > 0 ? n : (na > 0 ? na : 1);
    center_out[3 * (p - p0) + d] = (int32_t)floordiv(2 * S + N, 2 * N);
  }
}

// Support box of an atom (voxel index ranges per axis, from 3 sigma) relative to
// the grid of edge G centred on (c0, c1, c2); X* receive the atom's offsets from
// the centre.
struct AtomBox {
  int64_t X0, X1, X2;
  int lo0, lo1, lo2, hi0, hi1, hi2;
};
__device__ inline AtomBox atom_box(const int32_t *xyz, int a, int64_t c0, int64_t c1, int64_t c2, int G) {
  const int64_t off = 512LL * (G - 1);
  AtomBox b;
  b.X0 = xyz[3 * a] - c0;
  b.X1 = xyz[3 * a + 1] - c1;
  b.X2 = xyz[3 * a + 2] - c2;
  b.lo0 = (int)floordiv(b.X0 + off - kRcut + 1023, 1024);
  b.lo1 = (int)floordiv(b.X1 + off - kRcut + 1023, 1024);
  b.lo2 = (int)floordiv(b.X2 + off - kRcut + 1023, 1024);
  b.hi0 = (int)floordiv(b.X0 + off + kRcut, 1024);
  b.hi1 = (int)floordiv(b.X1 + off + kRcut, 1024);
  b.hi2 = (int)floordiv(b.X2 + off + kRcut, 1024);
  return b;
}

// Weight of candidate voxel (v0, v1, v2) for an atom at offset X from the centre
// (0 outside the 3 sigma support).
__device__ inline float splat_weight(int64_t X0, int64_t X1, int64_t X2, int v0, int v1, int v2, int G, bool &in) {
  const int64_t d0 = X0 - 512LL * (2 * v0 - G + 1);
  const int64_t d1 = X1 - 512LL * (2 * v1 - G + 1);
  const int64_t d2 = X2 - 512LL * (2 * v2 - G + 1);
  const int64_t D = d0 * d0 + d1 * d1 + d2 * d2;
  in = D <= (int64_t)kRcut * kRcut;
  return in ? expf(-(float)D * kInv2s2) : 0.0f;
}

constexpr int kBinThreads = 256;
constexpr int kMaxTiles = (96 / kTA) * (96 / kTB);   // G <= 96
// an atom's support spans at most 4 voxels per axis, so at most (T + 2) / T + 1
// tiles of extent T
constexpr int tiles_spanned(int T) { return (T + 2) / T + 1; }
constexpr int kMaxTilesPerAtom = tiles_spanned(kTA) * tiles_spanned(kTB);

// One workgroup per pose.  Zs[a - base] = the atom's normaliser; bin_off[pl][t]
// (ntiles + 1 entries per pose) = where tile t's list starts in bin_atoms (local
// atom ids a - base), the pose's lists occupying bin_atoms[kMaxTilesPerAtom (a0 - base) ...].
__global__ __launch_bounds__(kBinThreads) void k_splat_bin(const int32_t *__restrict__ atom_off, int n_atoms,
                                                          const int32_t *__restrict__ xyz,
                                                          const int32_t *__restrict__ centers, int p0, int G,
                                                          int64_t atoms_cap, double *__restrict__ Zs,
                                                          int32_t *__restrict__ bin_off,
                                                          int32_t *__restrict__ bin_atoms) {
  __shared__ int cnt[kMaxTiles];
  __shared__ int part[kBinThreads];
  const int pl = blockIdx.x, p = p0 + pl, tid = threadIdx.x;
  const int ntb = G / kTB, ntiles = (G / kTA) * ntb;
  int a0, a1;
  pose_range(atom_off, p, n_atoms, a0, a1);  // malformed offsets: empty (k_splat reports them)
  const int base = min(max(atom_off[p0], 0), n_atoms);
  if (a0 < base || (int64_t)a1 - base > atoms_cap) a0 = a1 = base;  // outside the scratch: no atoms
  const int64_t c0 = centers[3 * pl], c1 = centers[3 * pl + 1], c2 = centers[3 * pl + 2];
  for (int t = tid; t < ntiles; t += kBinThreads) cnt[t] = 0;
  __syncthreads();
  // the tiles an atom reaches (its box overlaps the tile and the grid along axis 2)
  auto tiles_of = [&](const AtomBox &b, int &t0a, int &t0b, int &t1a, int &t1b) {
    const bool z_in = b.lo2 <= G - 1 && b.hi2 >= 0;
    t0a = max(0, b.lo0 < 0 ? 0 : b.lo0 / kTA);
    t0b = min(G / kTA - 1, b.hi0 < 0 ? -1 : b.hi0 / kTA);
    t1a = max(0, b.lo1 < 0 ? 0 : b.lo1 / kTB);
    t1b = min(ntb - 1, b.hi1 < 0 ? -1 : b.hi1 / kTB);
    if (!z_in || b.hi0 < 0 || b.hi1 < 0 || b.lo0 > G - 1 || b.lo1 > G - 1) t0b = t0a - 1;
  };
  for (int a = a0 + tid; a < a1; a += kBinThreads) {
    const AtomBox b = atom_box(xyz, a, c0, c1, c2, G);
    int t0a, t0b, t1a, t1b;
    tiles_of(b, t0a, t0b, t1a, t1b);
    for (int i = t0a; i <= t0b; ++i)
      for (int j = t1a; j <= t1b; ++j) atomicAdd(&cnt[i * ntb + j], 1);
  }
  __syncthreads();
  // exclusive scan of the counts: each thread sums a run of tiles, the runs' sums
  // are scanned, then each run is written with its offset
  const int per = (ntiles + kBinThreads - 1) / kBinThreads;
  int run = 0;
  for (int t = tid * per; t < min(ntiles, (tid + 1) * per); ++t) run += cnt[t];
  part[tid] = run;
  __syncthreads();
  for (int o = 1; o < kBinThreads; o <<= 1) {
    const int v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  const int list0 = kMaxTilesPerAtom * (a0 - base);
  int acc = list0 + part[tid] - run;
  int32_t *bo = bin_off + (int64_t)pl * (ntiles + 1);
  for (int t = tid * per; t < min(ntiles, (tid + 1) * per); ++t) {
    const int c = cnt[t];
    bo[t] = acc;
    cnt[t] = acc;  // becomes the tile's fill cursor
    acc += c;
  }
  if (tid == kBinThreads - 1) bo[ntiles] = list0 + part[kBinThreads - 1];
  __syncthreads();
  for (int a = a0 + tid; a < a1; a += kBinThreads) {
    const AtomBox b = atom_box(xyz, a, c0, c1, c2, G);
    int t0a, t0b, t1a, t1b;
    tiles_of(b, t0a, t0b, t1a, t1b);
    for (int i = t0a; i <= t0b; ++i)
      for (int j = t1a; j <= t1b; ++j) bin_atoms[atomicAdd(&cnt[i * ntb + j], 1)] = a - base;
  }
  // normalisers: one wave per atom, candidate voxel per lane.  Every w >=
  // exp(-4.5) > 2^-7 is an exact multiple of 2^-31, so w * 2^40 is an exact
  // integer and the integer wave sum is the exact sum of the float weights.
  const int lane = tid & 63, wave = tid >> 6;
  for (int a = a0 + wave; a < a1; a += kBinThreads / 64) {
    const AtomBox b = atom_box(xyz, a, c0, c1, c2, G);
    bool in;
    const float w = splat_weight(b.X0, b.X1, b.X2, b.lo0 + (lane >> 4), b.lo1 + ((lane >> 2) & 3), b.lo2 + (lane & 3), G, in);
    const int64_t wq = (int64_t)((double)w * 1099511627776.0);
    const double Z = (double)wave_sum_i64(wq) * (1.0 / 1099511627776.0);
    if (lane == 0) Zs[a - base] = Z;
  }
}

// MODE 0: float [19]; 1: bf16 [19]; 2: float [cpad]; 3: bf16 [cpad] (channels >= 19 zero);
// 4: bf16 in 4-channel chunks, chunk-major per pose: [P][cpad / 4][G^3][4]
template <int MODE>
__global__ __launch_bounds__(256) void k_splat(const int32_t *__restrict__ atom_off, int n_atoms,
                                               const int32_t *__restrict__ xyz,
                                               const float *__restrict__ feat,
                                               const int32_t *__restrict__ centers, int p0, int G,
                                               void *__restrict__ grid, int cpad,
                                               const double *__restrict__ Zs, const int32_t *__restrict__ bin_off,
                                               const int32_t *__restrict__ bin_atoms,
                                               int64_t *__restrict__ status) {
  // bin_atoms and Zs are indexed by atom - base, base = the launch's first atom
  extern __shared__ __attribute__((aligned(16))) int acc[];  // [kTA][kTB][G][19]
  __shared__ int budget;        // range budget used by the atoms reaching this tile
  const int pl = blockIdx.y;    // pose within this launch
  const int p = p0 + pl;
  const int ntb = G / kTB, ntiles = (G / kTA) * ntb;
  const int i0 = (blockIdx.x / ntb) * kTA, j0 = (blockIdx.x % ntb) * kTB;
  const int nacc = kTA * kTB * G * CF_NCH;  // a multiple of 4 (kTA * kTB is)
  static_assert((kTA * kTB) % 4 == 0, "accumulators cleared 16 bytes at a time");
  for (int e = threadIdx.x; e < nacc / 4; e += blockDim.x) reinterpret_cast<int4 *>(acc)[e] = make_int4(0, 0, 0, 0);
  if (threadIdx.x == 0) budget = 0;
  int a0, a1;
  if (!pose_range(atom_off, p, n_atoms, a0, a1) && blockIdx.x == 0 && threadIdx.x == 0)
    dev_fail(status, kDevBadOffsets);
  const int base = min(max(atom_off[p0], 0), n_atoms);
  const int64_t c0 = centers[3 * pl], c1 = centers[3 * pl + 1], c2 = centers[3 * pl + 2];
  const int l0 = bin_off[(int64_t)pl * (ntiles + 1) + blockIdx.x], l1 = bin_off[(int64_t)pl * (ntiles + 1) + blockIdx.x + 1];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the tile's list is dealt to the waves in turn (entry q0 + 4 k to lane k of wave
  // q0 - l0), so that a list of a few dozen atoms keeps all four waves sweeping
  for (int q0 = l0 + wave; q0 < l1; q0 += 256) {
    const int q = q0 + 4 * lane;
    bool ov = false;
    AtomBox bx{};
    double Za = 1.0;
    if (q < l1) {
      const int a = base + bin_atoms[q];
      bx = atom_box(xyz, a, c0, c1, c2, G);
      Za = Zs[a - base];
      ov = bx.lo0 <= i0 + kTA - 1 && bx.hi0 >= i0 && bx.lo1 <= j0 + kTB - 1 && bx.hi1 >= j0 && bx.lo2 <= G - 1 &&
           bx.hi2 >= 0;
    }
    // the lanes of the listed atoms hold their features; the sweep below reads
    // them (and the coordinates) from that lane instead of from memory
    float fr[CF_NCH];
#pragma unroll
    for (int ch = 0; ch < CF_NCH; ++ch) fr[ch] = 0.0f;
    int cost = 0;
    if (ov) {
      const int a = base + bin_atoms[q];
      float mf = 0.0f;
      bool bad = false;
#pragma unroll
      for (int ch = 0; ch < CF_NCH; ++ch) {
        fr[ch] = feat[(int64_t)CF_NCH * a + ch];
        bad |= !(fabsf(fr[ch]) <= kFeatMax);
        mf = fmaxf(mf, fabsf(fr[ch]));
      }
      cost = bad ? (int)kFeatMax + 1 : (int)ceilf(mf);  // NaN and |f| > 64 count 65
    }
    {
      int wc = cost;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) wc += __shfl_xor(wc, o, 64);
      if (lane == 0 && wc) atomicAdd(&budget, wc);
    }
    uint64_t m = __ballot(ov);
    while (m) {
      const int b = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int v0 = rdlane(bx.lo0, b) + (lane >> 4), v1 = rdlane(bx.lo1, b) + ((lane >> 2) & 3),
                v2 = rdlane(bx.lo2, b) + (lane & 3);
      bool in;
      const float w = splat_weight(rdlane64(bx.X0, b), rdlane64(bx.X1, b), rdlane64(bx.X2, b), v0, v1, v2, G, in);
      const double Z = __longlong_as_double(rdlane64(__double_as_longlong(Za), b));
      const float f = (float)((double)w / Z);
      const bool tile = in && v0 >= i0 && v0 < i0 + kTA && v1 >= j0 && v1 < j0 + kTB && v2 >= 0 && v2 < G;
      if (tile) {
        int *dst = acc + (((v0 - i0) * kTB + (v1 - j0)) * G + v2) * CF_NCH;
        // a feature out of range adds nothing and is reported once.  A zero feature
        // (most channels of an atom: one-hot element and flags) adds nothing either;
        // the feature is the same on every lane, so skipping its add is a uniform
        // branch and the sums are unchanged
        bool badf = false;
#pragma unroll
        for (int ch = 0; ch < CF_NCH; ++ch) {
          const float fv = __int_as_float(rdlane(__float_as_int(fr[ch]), b));
          if (fv != 0.0f) {
            const bool okf = fabsf(fv) <= kFeatMax;
            badf |= !okf;
            atomicAdd(dst + ch, okf ? (int)rintf(fv * f * kSplatScale) : 0);
          }
        }
        if (badf) dev_fail(status, kDevBadFeature);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && budget > kSplatBudget) dev_fail(status, kDevGridRange);
  // stream the tile out
  const int nvox = kTA * kTB * G;
  if (MODE == 0 || MODE == 1) {
    for (int e = threadIdx.x; e < nvox * CF_NCH; e += blockDim.x) {
      const int v = e / CF_NCH, ch = e - v * CF_NCH;
      const int k = v % G, jj = (v / G) % kTB, ii = v / (G * kTB);
      const int64_t gv = (((int64_t)pl * G + (i0 + ii)) * G + (j0 + jj)) * G + k;
      const float val = (float)acc[e] * kSplatInvScale;
      if (MODE == 0)
        reinterpret_cast<float *>(grid)[gv * CF_NCH + ch] = val;
      else
        reinterpret_cast<bf16_t *>(grid)[gv * CF_NCH + ch] = (bf16_t)val;
    }
  } else if (MODE == 4) {
    // chunk slowest, voxel fastest: consecutive threads write consecutive 8-byte voxels
    const int ng = cpad / 4;
    const int64_t g3 = (int64_t)G * G * G;
    for (int e = threadIdx.x; e < nvox * ng; e += blockDim.x) {
      const int g = e / nvox, v = e - g * nvox;
      const int k = v % G, jj = (v / G) % kTB, ii = v / (G * kTB);
      const int64_t vloc = ((int64_t)(i0 + ii) * G + (j0 + jj)) * G + k;
      float val[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ch = g * 4 + q;
        val[q] = ch < CF_NCH ? (float)acc[v * CF_NCH + ch] * kSplatInvScale : 0.0f;
      }
      const uint32_t lo = (uint32_t)__builtin_bit_cast(uint16_t, (bf16_t)val[0]) |
                          ((uint32_t)__builtin_bit_cast(uint16_t, (bf16_t)val[1]) << 16);
      const uint32_t hi = (uint32_t)__builtin_bit_cast(uint16_t, (bf16_t)val[2]) |
                          ((uint32_t)__builtin_bit_cast(uint16_t, (bf16_t)val[3]) << 16);
      *reinterpret_cast<uint2 *>(reinterpret_cast<bf16_t *>(grid) + (((int64_t)pl * ng + g) * g3 + vloc) * 4) =
          make_uint2(lo, hi);
    }
  } else {
    const int ng = cpad / 8;
    for (int e = threadIdx.x; e < nvox * ng; e += blockDim.x) {
      const int v = e / ng, g = e - v * ng;
      const int k = v % G, jj = (v / G) % kTB, ii = v / (G * kTB);
      const int64_t gv = (((int64_t)pl * G + (i0 + ii)) * G + (j0 + jj)) * G + k;
      float val[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int ch = g * 8 + q;
        val[q] = ch < CF_NCH ? (float)acc[v * CF_NCH + ch] * kSplatInvScale : 0.0f;
      }
      if (MODE == 2) {
        float4 *dst = reinterpret_cast<float4 *>(reinterpret_cast<float *>(grid) + gv * cpad + g * 8);
        dst[0] = make_float4(val[0], val[1], val[2], val[3]);
        dst[1] = make_float4(val[4], val[5], val[6], val[7]);
      } else {
        bf16x8 pk;
#pragma unroll
        for (int q = 0; q < 8; ++q) pk[q] = (bf16_t)val[q];
        *reinterpret_cast<bf16x8 *>(reinterpret_cast<bf16_t *>(grid) + gv * cpad + g * 8) = pk;
      }
    }
  }
}

// Public [19]-channel grid -> the internal layout (conversion between precisions
// allowed): padded [cpad] channels-last, or with chunk4 = voxels per pose the bf16
// 4-channel chunk-major layout [P][cpad / 4][G^3][4].
__global__ __launch_bounds__(256) void k_grid_repack4(const void *__restrict__ src, int src_bf16, int64_t n_vox,
                                                      bf16_t *__restrict__ dst, int cpad, int64_t vpp) {
  const int ng = cpad / 4;
  const int64_t total = n_vox * ng;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    // (pose, chunk, voxel) with the voxel fastest
    const int64_t pose = e / (vpp * ng), r = e - pose * vpp * ng;
    const int g = (int)(r / vpp);
    const int64_t v = pose * vpp + (r - (int64_t)g * vpp);
    bf16_t val[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = g * 4 + q;
      float f = 0.0f;
      if (ch < CF_NCH)
        f = src_bf16 ? (float)reinterpret_cast<const bf16_t *>(src)[v * CF_NCH + ch]
                     : reinterpret_cast<const float *>(src)[v * CF_NCH + ch];
      val[q] = (bf16_t)f;
    }
    uint2 o;
    __builtin_memcpy(&o, val, 8);
    *reinterpret_cast<uint2 *>(dst + e * 4) = o;
  }
}

__global__ __launch_bounds__(256) void k_grid_repack(const void *__restrict__ src, int src_bf16,
                                                     int64_t n_vox, void *__restrict__ dst,
                                                     int dst_bf16, int cpad) {
  const int ng = cpad / 8;
  const int64_t total = n_vox * ng;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = e / ng;
    const int g = (int)(e - v * ng);
    float val[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ch = g * 8 + q;
      if (ch < CF_NCH)
        val[q] = src_bf16 ? (float)reinterpret_cast<const bf16_t *>(src)[v * CF_NCH + ch]
                          : reinterpret_cast<const float *>(src)[v * CF_NCH + ch];
      else
        val[q] = 0.0f;
    }
    if (dst_bf16) {
      bf16x8 pk;
#pragma unroll
      for (int q = 0; q < 8; ++q) pk[q] = (bf16_t)val[q];
      *reinterpret_cast<bf16x8 *>(reinterpret_cast<bf16_t *>(dst) + v * cpad + g * 8) = pk;
    } else {
      float4 *d = reinterpret_cast<float4 *>(reinterpret_cast<float *>(dst) + v * cpad + g * 8);
      d[0] = make_float4(val[0], val[1], val[2], val[3]);
      d[1] = make_float4(val[4], val[5], val[6], val[7]);
    }
  }
}

}  // namespace

hipError_t launch_centers(const int32_t *atom_off, int n_atoms, const int32_t *xyz, const uint8_t *is_lig,
                          int p0, int n_poses, int32_t *center_out, int64_t *status, hipStream_t s) {
  if (n_poses <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_centers, dim3(n_poses), dim3(64), 0, s, atom_off, n_atoms, xyz, is_lig, p0, center_out,
                     status);
  return hipGetLastError();
}

int64_t splat_work_bytes(int n_poses, int64_t atoms, int G) {
  const int64_t ntiles = (int64_t)(G / kTA) * (G / kTB);
  return atoms * 8 + (int64_t)n_poses * (ntiles + 1) * 4 + atoms * kMaxTilesPerAtom * 4 + 256;
}

hipError_t launch_splat(const int32_t *atom_off, int n_atoms, const int32_t *xyz, const float *feat,
                        const int32_t *centers, int p0, int n_poses, int G, void *grid, int out_mode,
                        int cpad, void *work, int64_t atoms_cap, int64_t *status, hipStream_t s) {
  if (n_poses <= 0) return hipSuccess;
  if (!work || G > 96) return hipErrorInvalidValue;
  const int ntiles = (G / kTA) * (G / kTB);
  double *Zs = reinterpret_cast<double *>(work);
  int32_t *bin_off = reinterpret_cast<int32_t *>(Zs + atoms_cap);
  int32_t *bin_atoms = bin_off + (int64_t)n_poses * (ntiles + 1);
  hipLaunchKernelGGL(k_splat_bin, dim3(n_poses), dim3(kBinThreads), 0, s, atom_off, n_atoms, xyz, centers, p0, G,
                     atoms_cap, Zs, bin_off, bin_atoms);
  const dim3 grd(ntiles, n_poses);
  const size_t lds = sizeof(int) * kTA * kTB * G * CF_NCH;
#define CF_SPLAT(M)                                                                                          \
  hipLaunchKernelGGL(k_splat<M>, grd, dim3(256), lds, s, atom_off, n_atoms, xyz, feat, centers, p0, G, grid, cpad, \
                     Zs, bin_off, bin_atoms, status)
  switch (out_mode) {
    case 0: CF_SPLAT(0); break;
    case 1: CF_SPLAT(1); break;
    case 2: CF_SPLAT(2); break;
    case 3: CF_SPLAT(3); break;
    case 4: CF_SPLAT(4); break;
    default: return hipErrorInvalidValue;
  }
#undef CF_SPLAT
  return hipGetLastError();
}

hipError_t launch_grid_repack(const void *src, int src_bf16, int n_vox, void *dst, int dst_bf16,
                              int cpad, hipStream_t s, int64_t chunk4_vpp) {
  if (chunk4_vpp > 0) {
    const int64_t total = (int64_t)n_vox * (cpad / 4);
    const int blocks = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_grid_repack4, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, src, src_bf16,
                       (int64_t)n_vox, reinterpret_cast<bf16_t *>(dst), cpad, chunk4_vpp);
    return hipGetLastError();
  }
  const int64_t total = (int64_t)n_vox * (cpad / 8);
  const int blocks = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_grid_repack, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, src, src_bf16,
                     (int64_t)n_vox, dst, dst_bf16, cpad);
  return hipGetLastError();
}

}  // namespace cf
