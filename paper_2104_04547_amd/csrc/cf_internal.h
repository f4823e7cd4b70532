// Internal declarations shared by the HIP translation units of libcf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cf.h"

namespace cf {

typedef __bf16 bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Fixed-point scale of the splat accumulators: 2^20 units per feature unit.
constexpr float kSplatScale = 1048576.0f;
constexpr float kSplatInvScale = 1.0f / 1048576.0f;
constexpr float kFeatMax = 64.0f;
// Range budget of one splat tile: the sum over the atoms that reach the tile of
// ceil(max_channel |feature|).  One atom adds at most 0.4922 feature units (the
// weight of an atom on a voxel centre) times |feature| to a voxel, so a budget of
// 4096 keeps every partial sum of every voxel below 2016 * 2^20 + 4096 / 2 units,
// inside int32.  A tile over budget is reported instead of wrapping silently.
constexpr int kSplatBudget = 4096;

// Device status word layout (int64[4]): [0] first error code (0 = none),
// [1] covalent edges needed, [2] non-covalent edges needed, [3] detail.
enum DevErr : int64_t {
  kDevOk = 0,
  kDevBadOffsets = 1,
  kDevBadFeature = 2,
  kDevCoordRange = 3,
  kDevCapacity = 4,
  kDevPoseTooLarge = 5,
  kDevBadGraph = 6,
  kDevGridRange = 7,
};

__device__ inline void dev_fail(int64_t *status, int64_t code) {
  atomicCAS(reinterpret_cast<unsigned long long *>(status), 0ull, (unsigned long long)code);
}

// Atom range [a0, a1) of pose p, checked against the batch arrays (n_atoms rows).
// Malformed offsets give an empty range and false.
__device__ inline bool pose_range(const int32_t *atom_off, int p, int n_atoms, int &a0, int &a1) {
  a0 = atom_off[p];
  a1 = atom_off[p + 1];
  const bool ok = a0 >= 0 && a1 >= a0 && a1 <= n_atoms && a1 - a0 <= CF_MAX_POSE_ATOMS;
  if (!ok) a1 = a0 = 0;
  return ok;
}

// Work order that keeps neighbouring work on one XCD.  The dispatcher hands
// consecutive workgroups of a grid to the chip's 8 XCDs in turn, and each XCD has
// its own L2: renumber the linear workgroup id so that every XCD receives a
// contiguous range of the logical order (z fastest, then x, then y -- for the
// conv kernels: output-channel block, tile, pose), so that the tiles of a pose,
// which share halo voxels, run under one L2.
__device__ inline void xcd_order(int &x, int &y, int &z) {
  constexpr int kXcd = 8;
  const int gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const int n = gx * gy * gz;
  const int L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int q = n / kXcd, r = n % kXcd, xcd = L % kXcd, k = L / kXcd;
  const int l = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
  z = l % gz;
  x = (l / gz) % gx;
  y = l / (gz * gx);
}

// Zero K steps past the end of the packed tap-pair / tap-quad weights: the conv
// kernels prefetch weight fragments up to this many steps ahead.
constexpr int kConvPadSteps = 6;

// ---- per-layer conv launch description (host side) ----
struct ConvLayer {
  int cin, cout, k, stride, res_src;
  int cin_pad;     // input channel stride (multiple of the chunk width)
  int cout_pad32;  // output channels rounded up to 32 (packed weight rows)
  int cout_store;  // output channel stride (multiple of 16)
  void *wpk;       // packed weights (precision dtype)
  int64_t wbytes;  // size of the packed weights in bytes
  void *wpk8;      // bf16 only: weights packed for the tap-pair kernel
  int64_t wbytes8;
  void *wpk4;      // bf16, input channels not a multiple of 8: weights packed for the tap-quad kernel
  int64_t wbytes4;
  int in_cm4;      // the input is the bf16 grid in 4-channel chunk-major layout [P][cin_pad / 4][D^3][4]
  float *bias;     // folded bias [cout_pad32]
  void *gspec;     // stride-1 layers: in-plane spectra of the weights (frequency-domain path)
  int64_t gspec_bytes;
  int spec_f32;    // the frequency-domain path runs on fp32 spectra and activations (the plain form)
};

// Kernel launchers (defined in the .hip files).
hipError_t launch_centers(const int32_t *atom_off, int n_atoms, const int32_t *xyz, const uint8_t *is_lig,
                          int p0, int n_poses, int32_t *center_out, int64_t *status, hipStream_t s);
// out_mode: 0 = float [19], 1 = bf16 [19], 2 = float padded [cpad], 3 = bf16 padded [cpad],
// 4 = bf16 4-channel chunk-major [P][cpad / 4][G^3][4]
// work: splat_work_bytes(n_poses, atoms_cap, G) bytes of scratch (per-atom normalisers
// and the per-tile atom lists), atoms_cap >= the atoms of poses p0 .. p0 + n_poses - 1
hipError_t launch_splat(const int32_t *atom_off, int n_atoms, const int32_t *xyz, const float *feat,
                        const int32_t *centers, int p0, int n_poses, int G, void *grid, int out_mode,
                        int cpad, void *work, int64_t atoms_cap, int64_t *status, hipStream_t s);
int64_t splat_work_bytes(int n_poses, int64_t atoms, int G);
// chunk4_vpp > 0: bf16 4-channel chunk-major output with that many voxels per pose
hipError_t launch_grid_repack(const void *src, int src_bf16, int n_vox, void *dst, int dst_bf16,
                              int cpad, hipStream_t s, int64_t chunk4_vpp = 0);

hipError_t launch_graph(const int32_t *atom_off, int n_atoms, const int32_t *xyz, int p0, int n_poses, int r_cov,
                        int r_nc, int32_t *cov_row, int32_t *cov_col, int64_t cov_cap, int32_t *nc_row,
                        int32_t *nc_col, int64_t nc_cap, int32_t *deg_scratch, int64_t n_chunk_cap,
                        int64_t *pose_scratch, int64_t *status, hipStream_t s);

int conv_num_variants();
const char *conv_variant_name(int v);
bool conv_variant_ok(int v, const ConvLayer &L, int bf16, int D_in);
int conv_default_variant(const ConvLayer &L, int D_in, int bf16);
// device scratch a variant needs for n_poses (0 for the direct kernels)
int64_t conv_work_bytes(int v, const ConvLayer &L, int D_in, int n_poses);
hipError_t launch_conv(int variant, const ConvLayer &L, int bf16, const void *in, const void *res,
                       void *out, int n_poses, int D_in, void *work, hipStream_t s);
// seeded values uniform in [0, 0.5) over `bytes` of bf16 or fp32 elements
hipError_t launch_fill_random(void *p, int64_t bytes, int bf16, uint64_t seed, hipStream_t s);

// frequency-domain stride-1 conv (cf_fftconv.hip)
bool fft_conv_layer_ok(const ConvLayer &L);     // layer shape supported (spectra prepared at create)
bool fft_conv_ok(const ConvLayer &L, int D);    // ... and at input size D
int64_t fft_conv_gspec_bytes(const ConvLayer &L);
int64_t fft_conv_work_bytes(const ConvLayer &L, int D, int n_poses);
hipError_t fft_conv_prepare(ConvLayer &L, const float *w_folded_dev, hipStream_t s);
// stage -1: the whole layer; 0, 1, 2: forward plane FFTs, z-correlation, inverse
hipError_t launch_fft_conv(const ConvLayer &L, const void *in, const void *res, void *out, int n_poses, int D,
                           void *work, hipStream_t s, int stage = -1);
// two consecutive frequency-domain layers whose activation between them can stay
// in the transform kernels; launch_fft_mid runs layer L's inverse (its spectrum in
// the work buffer) and layer Ln's forward transform in one kernel, storing the
// activation only when out != null
bool fft_conv_fusable(const ConvLayer &L, const ConvLayer &Ln, int D);
hipError_t launch_fft_mid(const ConvLayer &L, const ConvLayer &Ln, const void *res, void *out, int n_poses, int D,
                          void *work, hipStream_t s);
// algorithmic FLOP and HBM bytes of one stage for n_poses
void fft_conv_stage_cost(int stage, const ConvLayer &L, int D, int n_poses, double *flop, double *bytes);
bool conv_variant_is_fft(int v);

hipError_t launch_pool_dense(const void *act, int bf16, int n_poses, int vox, int cstride, int c,
                             const float *dense_w, const float *dense_b, int n_dense, const float *dense2_w,
                             const float *dense2_b, int n_dense2, float *latent, hipStream_t s);

// SG-CNN weights on the device, transposed to [k][out] so that consecutive lanes
// (consecutive outputs) read consecutive words.
// Widths: H is the covalent stage's (padded with zero weights to a kernel width),
// H2 the non-covalent stage's (= H without staging).  "Stage s width" below is
// H for s = 0 and H2 for s = 1; the readout runs at H2.
struct SgWeights {
  int H, K_c, K_n;
  int H2;                           // non-covalent stage width
  int staged;                       // PotentialNet staging: per-atom gather between the stages
  const float *embed_wT, *embed_b;  // [19][H], [H]
  const float *msgT[16];            // per round [Hs][Hs] (covalent rounds first)
  const float *w_ihT[2], *w_hhT[2]; // per stage [Hs][3Hs] (gate columns r, z, n)
  const float *b_ih[2], *b_hh[2];   // per stage [3Hs]
  const float *gate_wT, *gate_b;    // [H2+U][H2], [H2]; U = 19 (raw features) or H (staged: the gather)
  const float *val_wT, *val_b;      // [H2][H2], [H2]
  const float *mid_gate_wT, *mid_gate_b;  // staged: [H+19][H], [H]
  const float *mid_val_wT, *mid_val_b;    // staged: [H][H], [H]
  const float *embed2_wT, *embed2_b;      // staged: [H][H2], [H2]
  // precision form (H >= 32): split-bfloat16 copies (hi = bf16(w), lo = bf16(w - hi))
  // packed as MFMA B operands, [K/16][N][16] with element [ks][n][e] = W[n][16 ks + e]
  const bf16_t *msg_hi[16], *msg_lo[16];  // N = Hs
  const bf16_t *ih_hi[2], *ih_lo[2];      // N = 3Hs
  const bf16_t *hh_hi[2], *hh_lo[2];      // N = 3Hs
};
// csr_global = 1: rows indexed by global atom id and columns are global ids (the
// public neighbour-list layout); 0: both are relative to the first atom of pose p0.
hipError_t launch_sgcnn(const SgWeights &W, int bf16, const int32_t *atom_off, int n_atoms, const float *feat,
                        const uint8_t *is_lig, int p0, int n_poses, const int32_t *cov_row,
                        const int32_t *cov_col, int64_t cov_cap, const int32_t *nc_row,
                        const int32_t *nc_col, int64_t nc_cap, int csr_global, float *hbuf,
                        int64_t hcap_atoms, float *sg_latent, int64_t *status, hipStream_t s);

// ---- backward pass (cf_backward.hip): float32, deterministic reductions ----
hipError_t bw_fill(float *p, int64_t n, float v, hipStream_t s);
hipError_t bw_add(float *dst, const float *src, int64_t n, hipStream_t s);
// Y[i][j] (+)= b[j] + sum_k W[j*ldw + k] X[i*ldx + k], i < n, j < J, k < K
hipError_t bw_rowmat(const float *X, int ldx, int n, int K, const float *W, int ldw, const float *b, int J, float *Y,
                     int ldy, int accumulate, hipStream_t s);
// Y[i][k] (+)= sum_j W[j*ldw + k] X[i*ldx + j], i < n, j < J, k < K
hipError_t bw_rowmat_t(const float *X, int ldx, int n, int J, const float *W, int ldw, int K, float *Y, int ldy,
                       int accumulate, hipStream_t s);
// A[i][f] (+)= sum over CSR row i (chunk-local ids) of S[col][f]
hipError_t bw_agg(const int32_t *rowp, const int32_t *col, int64_t cap, const float *S, int n, int F, float *A,
                  int accumulate, int64_t *status, hipStream_t s);
hipError_t bw_gru_fwd(const float *GI, const float *GH, const float *Hin, int n, int H, float *Hout, hipStream_t s);
hipError_t bw_gru_bwd(const float *GI, const float *GH, const float *Hin, const float *dHout, int n, int H, float *dGI,
                      float *dGH, float *dHd, hipStream_t s);
hipError_t bw_readout(const float *Gpre, const float *V, const uint8_t *is_lig, const int32_t *atom_off, int p0,
                      int np, int H, float *S, hipStream_t s);
hipError_t bw_readout_bwd(const float *Gpre, const float *V, const uint8_t *is_lig, const int32_t *atom_off, int p0,
                          int np, int H, int n_atoms, const float *dS, float *dGpre, float *dV, hipStream_t s);
// C[a*ldc + b] (+)= sum_{i < n} U[i*ldu + a] V[i*ldv + b] (V null: 1); part holds
// bw_outer_scratch(n, A, B) floats
int64_t bw_outer_scratch(int n, int A, int B);
hipError_t bw_outer(const float *U, int ldu, const float *V, int ldv, int n, int A, int B, float *C, int ldc,
                    int accumulate, float *part, hipStream_t s);
hipError_t bw_pool_mean(const float *act, int np, int64_t vox, int cstride, int C, float *pool, hipStream_t s);
hipError_t bw_pool_seed(const float *dpool, int np, int64_t vox, int cstride, int C, float *dact, hipStream_t s);
hipError_t bw_relu_mask(float *d, const float *y, int64_t n, hipStream_t s);
hipError_t bw_relu_rows(float *y, int n, int J, int ld, hipStream_t s);
hipError_t bw_relu_grad_rows(float *d, const float *pre, int n, int J, hipStream_t s);
hipError_t bw_fold_wt(const float *W, const float *gamma, const float *var, int cout, int cin, int taps, float *WT,
                      hipStream_t s);
hipError_t bw_conv_wgrad(const float *X, int D, int xstride, int cin, const float *dY, int Do, int ystride, int cout,
                         int KS, int S, int np, float *part, hipStream_t s);
hipError_t bw_conv_dgrad(const float *dY, int Do, int ystride, int cout, const float *WT, int cin, int KS, int S, int D,
                         int xstride, int np, float *dX, hipStream_t s);
hipError_t bw_fold_grad(const float *dWf, const float *dbf, const float *W, const float *b, const float *gamma,
                        const float *mean, const float *var, int cout, int cin, int taps, float *gW, float *gb,
                        float *ggamma, float *gbeta, float *gmean, float *gvar, hipStream_t s);
bool bw_head_ok(int fin, int fh, int nhid);
hipError_t bw_head(const float *cnn, int lc, const float *sg, int sgw, const float *prm, int nhid, int fh, int residual,
                   const float *dscore, int np, float *scores, float *dcnn, float *dsg, float *part, int64_t nprm,
                   hipStream_t s);

// covalent / non-covalent widths (after padding) the staged SG-CNN kernel supports
bool sgcnn_staged_supported(int hc, int hn);

hipError_t launch_segmax(const float *scores, int n_scores, const int32_t *off, int n_seg, float *best,
                         int32_t *best_idx, int64_t *status, hipStream_t s);
// scratch: 1088 + 8 k bytes
hipError_t launch_topk(const float *v, int n, int k, int32_t *idx_out, float *val_out, void *scratch, hipStream_t s);
// Top-k scratch: histogram (1024 B) + select state (64 B) + up to kTopkMaxK keys.
constexpr int kTopkMaxK = 1024;
constexpr size_t kTopkScratchBytes = 1024 + 64 + 8 * (size_t)kTopkMaxK;
constexpr int kMaxDevices = 64;
// Device address of the library's static top-k scratch on the current device.
hipError_t topk_static_scratch(void **out);

// A fusion head as a list of dense layers over a per-pose feature buffer that
// starts as [cnn latent (lc) | sg latent (H)]; each layer reads the concatenation
// of two slices, writes a new slice, applies its activation and optionally adds
// another slice (a skip connection).  The score is out_scale * the sum of the out
// slots (Late Fusion: the mean of the two branch predictions).
constexpr int kHeadMaxOps = 12;
constexpr int kHeadBuf = 1024;  // floats per pose
enum HeadAct : int { kActNone = 0, kActRelu = 1, kActSelu = 2 };
struct HeadOp {
  int src0, n0;    // input = [slice (src0, n0) ; slice (src1, n1)], n1 may be 0
  int src1, n1;
  int dst, n_out;  // output slice (disjoint from the inputs and res)
  int act;         // HeadAct
  int res;         // >= 0: add slice [res, res + n_out) after the activation
  int w, b;        // offsets (floats) of W [n_out][n0 + n1] and b [n_out] in the parameter array
};
struct HeadProgram {
  int n_ops;
  HeadOp op[kHeadMaxOps];
  int n_out;       // 1 or 2
  int out_slot[2];
  float out_scale;
};
// Counter that changes whenever the context (re)allocates a scratch buffer: work
// captured into a graph before a change refers to freed memory and must not be
// replayed.
int64_t scratch_generation(const cf_ctx *c);

hipError_t launch_head(const float *cnn_lat, int lc, const float *sg_lat, int H, const float *params,
                       const HeadProgram &hp, int n_poses, float *scores, hipStream_t s);

}  // namespace cf
