// C ABI of the pose scorer: context, weight preparation, scratch management and
// the scoring entry points declared in include/cf.h.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "cf_internal.h"

using cf::bf16_t;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define CF_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(CF_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
};

}  // namespace

// Offsets (floats) of the blob's parameter tensors, recorded while the blob is
// read; the backward pass reads the unfolded parameters at these offsets of a
// device copy of the blob and writes gradients at the same offsets.
struct TrainOffsets {
  int64_t conv_w[8], conv_b[8], bn_g[8], bn_b[8], bn_m[8], bn_v[8];
  int64_t dense_w = -1, dense_b = -1, dense2_w = -1, dense2_b = -1;
  int64_t embed_w = -1, embed_b = -1;
  int64_t msg[16];
  int64_t wih[2], whh[2], bih[2], bhh[2];
  int64_t gate_w = -1, gate_b = -1, val_w = -1, val_b = -1;
  int64_t head = -1, head_n = 0;
};

struct cf_ctx {
  int device = 0;
  int bf16 = 0;
  cf_model_desc desc{};
  int64_t budget = 0;
  int64_t n_params = 0;
  int64_t weight_bytes = 0;
  int64_t scratch_bytes = 0;
  int64_t scratch_gen = 0;  // bumped whenever a scratch buffer is (re)allocated

  std::vector<cf::ConvLayer> conv;
  int lc = 0;  // CNN latent width
  int c_last = 0;
  float *dense_w = nullptr, *dense_b = nullptr;
  float *dense2_w = nullptr, *dense2_b = nullptr;
  int sgw = 0;              // SG-CNN latent width
  int64_t sg_floats = 0;    // SG-CNN state floats per atom (scratch)
  double sg_flop_atom = 0;  // SG-CNN FLOPs per atom (timing only)
  cf::SgWeights sg{};
  cf::HeadProgram head{};  // fusion head compiled to dense layers
  float *head_prm = nullptr;
  int64_t *status = nullptr;
  std::vector<void *> weight_allocs;
  // second stream for the graph / SG-CNN branch of cf_score_poses, joined by events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_sg = nullptr;

  // per-kernel timing (diagnostics, off by default)
  struct Pending {
    std::string key;
    hipEvent_t e0, e1;
    double flop, bytes;
    const int64_t *edges = nullptr;  // graph launches: {cov count, nc count, cov offset, nc offset} of the last pose
  };
  // pinned host slots the graph launches' edge totals are copied into (timing only)
  std::vector<int64_t *> pin_blocks;
  int pin_used = 0;
  struct Stat {
    int launches = 0;
    double ms = 0, flop = 0, bytes = 0;
  };
  bool timing = false;
  bool roctx = false;  // stage ranges for a tracer (cf_timing_enable, CF_TIMING_ROCTX)
  std::vector<Pending> pending;
  std::map<std::string, Stat> stats;

  // backward pass (plain form): the blob's parameters on the device, unfolded
  float *raw = nullptr;
  TrainOffsets tr{};

  // scratch
  DevBuf grid, centers, cnn_lat, sg_lat, deg, pose_tot, cov_row, cov_col, nc_row, nc_col, hbuf, sel;
  std::vector<DevBuf> act;  // t_1 .. t_L
  std::vector<DevBuf> dact; // backward: gradients of t_1 .. t_L
  DevBuf bw_sg, bw_cnn, bw_part, bw_head;  // backward scratch
  DevBuf splatwork;                        // per-atom normalisers and per-tile atom lists
  DevBuf convwork;          // scratch of the frequency-domain conv (spectra)
  std::map<int, std::vector<int>> variants;  // per G
};

namespace {

int alloc_weight(cf_ctx *c, void **p, size_t bytes, const void *host) {
  if (hipMalloc(p, bytes) != hipSuccess) return fail(CF_ERR_OOM, "weight allocation failed");
  c->weight_allocs.push_back(*p);
  c->weight_bytes += (int64_t)bytes;
  if (host && hipMemcpy(*p, host, bytes, hipMemcpyHostToDevice) != hipSuccess)
    return fail(CF_ERR_HIP, "weight upload failed");
  return CF_OK;
}

int ensure(cf_ctx *c, DevBuf &b, size_t bytes) {
  if (b.n >= bytes) return CF_OK;
  const int64_t grow = (int64_t)bytes - (int64_t)b.n;
  if (c->scratch_bytes + grow + c->weight_bytes > c->budget)
    return fail(CF_ERR_OOM, "scratch would exceed the context's HBM budget");
  if (b.p) {
    (void)hipFree(b.p);
    c->scratch_bytes -= (int64_t)b.n;
    b.p = nullptr;
    b.n = 0;
  }
  c->scratch_gen++;
  if (hipMalloc(&b.p, bytes) != hipSuccess) return fail(CF_ERR_OOM, "scratch allocation failed");
  b.n = bytes;
  c->scratch_bytes += (int64_t)bytes;
  return CF_OK;
}

int conv_out_dim(int D, int k, int s) { return (D + 2 * ((k - 1) / 2) - k) / s + 1; }

// roctx ranges around the stages a scoring call enqueues (CF_TIMING_ROCTX), so that
// a tracer (rocprofv3 --marker-trace) groups the kernels by stage.  The tracer's
// library is opened at run time on first use: no link-time dependency, and a
// process without it gets no ranges.
struct RoctxApi {
  int (*push)(const char *) = nullptr;
  int (*pop)() = nullptr;
  RoctxApi() {
    // the profiler SDK's roctx (what rocprofv3 records), else the older roctracer one
    const char *names[] = {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so.4",
                           "libroctx64.so"};
    void *h = nullptr;
    for (const char *n : names)
      if (!h) h = dlopen(n, RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
    pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!push || !pop) push = nullptr, pop = nullptr;
  }
};
const RoctxApi &roctx_api() {
  static const RoctxApi api;  // initialised once, thread-safe
  return api;
}
class Range {
 public:
  Range(const cf_ctx *c, const char *name) : on_(c->roctx && roctx_api().push) {
    if (on_) roctx_api().push(name);
  }
  ~Range() {
    if (on_) roctx_api().pop();
  }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;

 private:
  bool on_;
};

// Event pair around one launch on its own stream (only when timing is enabled).
hipEvent_t tbegin(cf_ctx *c, hipStream_t s) {
  if (!c->timing) return nullptr;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  (void)hipEventRecord(e, s);
  return e;
}

// Four pinned int64 slots (timing only): the graph stage's edge totals, read when
// its events have completed.
constexpr int kPinBlock = 4096;
int64_t *pin_slots(cf_ctx *c) {
  const size_t blk = (size_t)c->pin_used / kPinBlock, off = (size_t)c->pin_used % kPinBlock;
  if (blk == c->pin_blocks.size()) {
    void *p = nullptr;
    if (hipHostMalloc(&p, kPinBlock * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) return nullptr;
    c->pin_blocks.push_back(static_cast<int64_t *>(p));
  }
  c->pin_used += 4;
  return c->pin_blocks[blk] + off;
}

void tend(cf_ctx *c, hipStream_t s, hipEvent_t e0, const std::string &key, double flop, double bytes) {
  if (!e0) return;
  hipEvent_t e1 = nullptr;
  if (hipEventCreate(&e1) != hipSuccess) return;
  (void)hipEventRecord(e1, s);
  c->pending.push_back({key, e0, e1, flop, bytes});
}

size_t elem_size(const cf_ctx *c) { return c->bf16 ? 2 : 4; }
// internal grid: bf16 in 4-channel chunk-major layout (20 channels, read by the
// tap-quad kernels), fp32 channels-last padded to 24
int grid_cpad(const cf_ctx *c) { return c->bf16 ? 20 : 24; }

// bytes per pose of the conv-stack tensors at grid size G
int64_t pose_bytes(const cf_ctx *c, int G) {
  int64_t b = (int64_t)G * G * G * grid_cpad(c) * elem_size(c);
  int D = G;
  for (auto &L : c->conv) {
    D = conv_out_dim(D, L.k, L.stride);
    b += (int64_t)D * D * D * L.cout_store * elem_size(c);
  }
  return b;
}


// Scratch the context will hold after a call that needs buffers for n poses at
// grid size G and, when atoms > 0, per-atom buffers for that many atoms: the
// buffers only grow (ensure keeps a larger allocation), so each one counts as
// the larger of what it holds and what the call needs.
int64_t scratch_after(const cf_ctx *c, int G, int64_t n, int64_t atoms) {
  int64_t t = c->scratch_bytes;
  auto grow = [&](const DevBuf &b, int64_t need) {
    if (need > (int64_t)b.n) t += need - (int64_t)b.n;
  };
  grow(c->grid, n * G * G * G * grid_cpad(c) * (int64_t)elem_size(c));
  int D = G;
  int64_t work = 0;
  for (size_t i = 0; i < c->conv.size(); ++i) {
    // the frequency-domain path's spectra, wherever it may be selected
    if (cf::fft_conv_ok(c->conv[i], D)) work = std::max(work, cf::fft_conv_work_bytes(c->conv[i], D, n));
    D = conv_out_dim(D, c->conv[i].k, c->conv[i].stride);
    const int64_t need = n * D * D * D * c->conv[i].cout_store * (int64_t)elem_size(c);
    if (i < c->act.size()) grow(c->act[i], need);
    else t += need;
  }
  grow(c->convwork, work);
  grow(c->centers, n * 3 * 4);
  grow(c->cnn_lat, n * c->lc * 4);
  grow(c->sg_lat, n * c->sgw * 4);
  if (atoms > 0) {
    grow(c->splatwork, cf::splat_work_bytes((int)n, atoms, G));
    grow(c->deg, 2 * atoms * 4);
    grow(c->pose_tot, 4 * n * 8);
    grow(c->cov_row, (atoms + 1) * 4);
    grow(c->nc_row, (atoms + 1) * 4);
    grow(c->cov_col, atoms * 16 * 4);
    grow(c->nc_col, atoms * 96 * 4);
    grow(c->hbuf, atoms * c->sg_floats * 4);
  }
  return t;
}

// Poses per launch: at most 512, such that everything the call allocates (conv
// tensors of the chunk and, with atom stages, the per-atom scratch of at most
// n_atoms atoms) fits the context's HBM budget next to what it already holds.
int chunk_poses(const cf_ctx *c, int G, int P, int64_t n_atoms = 0) {
  const int64_t avail = c->budget - c->weight_bytes - ((int64_t)64 << 20);
  int n = std::min(512, P);
  while (n > 1) {
    const int64_t atoms = n_atoms > 0 ? std::min<int64_t>(n_atoms, (int64_t)n * CF_MAX_POSE_ATOMS) : 0;
    if (scratch_after(c, G, n, atoms) <= avail) break;
    n = n > 64 ? n - 32 : n - 1;
  }
  return n < 1 ? 1 : n;
}

int validate_batch(const cf_pose_batch *b) {
  if (!b) return fail(CF_ERR_INVALID_ARG, "batch is NULL");
  if (b->n_poses < 1) return fail(CF_ERR_INVALID_ARG, "n_poses must be >= 1");
  if (b->n_atoms < 1) return fail(CF_ERR_INVALID_ARG, "n_atoms must be >= 1");
  if ((int64_t)b->n_atoms > (int64_t)b->n_poses * CF_MAX_POSE_ATOMS)
    return fail(CF_ERR_INVALID_ARG, "n_atoms exceeds n_poses * 4096");
  if (!b->atom_off || !b->xyz || !b->feat || !b->is_lig)
    return fail(CF_ERR_INVALID_ARG, "batch array pointer is NULL");
  return CF_OK;
}

int validate_G(int G) {
  if (G < 8 || G > 96 || (G & 3)) return fail(CF_ERR_UNSUPPORTED, "grid size G must be a multiple of 4 in 8..96");
  return CF_OK;
}

// Per-layer kernel variants for grid size G (default table unless autotuned).
int variants_for(cf_ctx *c, int G, std::vector<int> &out) {
  auto it = c->variants.find(G);
  if (it != c->variants.end()) {
    out = it->second;
    return CF_OK;
  }
  out.clear();
  int D = G;
  for (auto &L : c->conv) {
    const int v = cf::conv_default_variant(L, D, c->bf16);
    if (v < 0) return fail(CF_ERR_UNSUPPORTED, "no conv kernel for this layer shape");
    out.push_back(v);
    D = conv_out_dim(D, L.k, L.stride);
    if (D < 1) return fail(CF_ERR_UNSUPPORTED, "grid too small for the conv stack");
  }
  c->variants[G] = out;
  return CF_OK;
}

int ensure_act(cf_ctx *c, int G, int np) {
  if ((int)c->act.size() != (int)c->conv.size()) c->act.resize(c->conv.size());
  int D = G;
  int rc = ensure(c, c->grid, (size_t)np * G * G * G * grid_cpad(c) * elem_size(c));
  if (rc) return rc;
  for (size_t i = 0; i < c->conv.size(); ++i) {
    D = conv_out_dim(D, c->conv[i].k, c->conv[i].stride);
    rc = ensure(c, c->act[i], (size_t)np * D * D * D * c->conv[i].cout_store * elem_size(c));
    if (rc) return rc;
  }
  return CF_OK;
}

// conv stack + pooling on grids already in the internal padded layout in c->grid;
// after_first (optional) is recorded on s once the first layer is enqueued
int run_cnn(cf_ctx *c, int G, int np, float *cnn_lat, hipStream_t s, hipEvent_t after_first = nullptr,
            bool store_all = false) {
  std::vector<int> var;
  int rc = variants_for(c, G, var);
  if (rc) return rc;
  {
    int64_t work = 0;
    int D = G;
    for (size_t i = 0; i < c->conv.size(); ++i) {
      work = std::max(work, cf::conv_work_bytes(var[i], c->conv[i], D, np));
      D = conv_out_dim(D, c->conv[i].k, c->conv[i].stride);
    }
    if (work > 0 && (rc = ensure(c, c->convwork, (size_t)work))) return rc;
  }
  std::vector<const void *> t;
  t.push_back(c->grid.p);
  int D = G;
  const int nl = (int)c->conv.size();
  // the activation t[k] is read from memory by a later layer (as input of a direct
  // kernel, or as a residual)
  auto stored = [&](int k) {
    if (store_all) return true;
    for (int j = k; j < nl; ++j)
      if (c->conv[j].res_src == k) return true;
    return false;
  };
  bool pend = false;  // the previous layer's output is still a spectrum in the work buffer
  for (int i = 0; i < nl; ++i) {
    const auto &L = c->conv[i];
    const void *res = L.res_src >= 0 ? t[L.res_src] : nullptr;
    const int Do = conv_out_dim(D, L.k, L.stride);
    if (cf::conv_variant_is_fft(var[i])) {
      // frequency-domain layer: forward transform (or, after another such layer,
      // that layer's inverse and this forward in one kernel), z-correlation, and the
      // inverse -- deferred into the next layer's kernel when it is one too
      double flop = 0.0, bytes = 0.0, f2 = 0.0, b2 = 0.0;
      hipEvent_t e = tbegin(c, s);
      if (pend) {
        const auto &Lp = c->conv[i - 1];
        const void *resp = Lp.res_src >= 0 ? t[Lp.res_src] : nullptr;
        const bool keep = stored(i);
        CF_HIP(cf::launch_fft_mid(Lp, L, resp, keep ? c->act[i - 1].p : nullptr, np, D, c->convwork.p, s));
        cf::fft_conv_stage_cost(2, Lp, D, np, &flop, &bytes);
        cf::fft_conv_stage_cost(0, L, D, np, &f2, &b2);
        // the activation between them moves only if stored (written once, not read back)
        const double act = (double)np * D * D * D * Lp.cout_store * elem_size(c);
        tend(c, s, e, "conv" + std::to_string(i - 1) + ".fft32.mid", flop + f2, bytes + b2 - act * (keep ? 1.0 : 2.0));
      } else {
        CF_HIP(cf::launch_fft_conv(L, t[i], res, c->act[i].p, np, D, c->convwork.p, s, 0));
        cf::fft_conv_stage_cost(0, L, D, np, &flop, &bytes);
        tend(c, s, e, "conv" + std::to_string(i) + ".fft32.fwd2d", flop, bytes);
      }
      e = tbegin(c, s);
      CF_HIP(cf::launch_fft_conv(L, t[i], res, c->act[i].p, np, D, c->convwork.p, s, 1));
      cf::fft_conv_stage_cost(1, L, D, np, &flop, &bytes);
      tend(c, s, e, "conv" + std::to_string(i) + ".fft32.zconv", flop, bytes);
      pend = i + 1 < nl && cf::conv_variant_is_fft(var[i + 1]) && Do == D && cf::fft_conv_fusable(L, c->conv[i + 1], D);
      if (!pend) {
        e = tbegin(c, s);
        CF_HIP(cf::launch_fft_conv(L, t[i], res, c->act[i].p, np, D, c->convwork.p, s, 2));
        cf::fft_conv_stage_cost(2, L, D, np, &flop, &bytes);
        tend(c, s, e, "conv" + std::to_string(i) + ".fft32.inv2d", flop, bytes);
      }
      D = Do;
      t.push_back(c->act[i].p);
      if (i == 0 && after_first) CF_HIP(hipEventRecord(after_first, s));
      continue;
    }
    hipEvent_t e = tbegin(c, s);
    CF_HIP(cf::launch_conv(var[i], L, c->bf16, t[i], res, c->act[i].p, np, D, c->convwork.p, s));
    if (e) {
      const double vox = (double)Do * Do * Do * np;
      const double flop = 2.0 * L.cin * L.cout * L.k * L.k * L.k * vox;
      const double bytes = ((double)D * D * D * np * L.cin + vox * L.cout * (res ? 2 : 1)) * elem_size(c);
      tend(c, s, e, "conv" + std::to_string(i) + "." + cf::conv_variant_name(var[i]), flop, bytes);
    }
    D = Do;
    t.push_back(c->act[i].p);
    if (i == 0 && after_first) CF_HIP(hipEventRecord(after_first, s));
  }
  const auto &Ll = c->conv.back();
  hipEvent_t e = tbegin(c, s);
  CF_HIP(cf::launch_pool_dense(t.back(), c->bf16, np, D * D * D, Ll.cout_store, Ll.cout, c->dense_w, c->dense_b,
                               c->desc.cnn_dense, c->dense2_w, c->dense2_b, c->desc.cnn_dense2, cnn_lat, s));
  tend(c, s, e, "pool_dense", 0.0, (double)D * D * D * np * Ll.cout * elem_size(c));
  return CF_OK;
}

// ---------------------------------------------------------------- weights

struct BlobReader {
  const float *p;
  size_t left;
  const float *take(size_t n) {
    if (n > left) return nullptr;
    const float *r = p;
    p += n;
    left -= n;
    return r;
  }
};

template <typename T>
T to_t(float v);
template <>
float to_t<float>(float v) {
  return v;
}
template <>
bf16_t to_t<bf16_t>(float v) {
  return (bf16_t)v;
}

template <typename T>
std::vector<T> pack_conv(const std::vector<float> &W, int cout, int cin, int k, int cin_pad, int cout_pad32) {
  const int CC = sizeof(T) == 2 ? 16 : 8;
  const int nchunks = cin_pad / CC;
  const int taps = k * k * k;
  // two extra zero taps: the conv kernel prefetches weights two taps ahead
  std::vector<T> out((size_t)(taps + 2) * nchunks * cout_pad32 * CC, to_t<T>(0.0f));
  for (int tap = 0; tap < taps; ++tap)
    for (int ch = 0; ch < nchunks; ++ch)
      for (int n = 0; n < cout; ++n)
        for (int e = 0; e < CC; ++e) {
          const int c = sizeof(T) == 2 ? ch * CC + e : ch * CC + 2 * (e % 4) + (e / 4);
          if (c >= cin) continue;
          const float v = W[((size_t)n * cin + c) * taps + tap];
          out[(((size_t)tap * nchunks + ch) * cout_pad32 + n) * CC + e] = to_t<T>(v);
        }
  return out;
}

// bf16 weights for the tap-pair kernel: [pair][chunk8][c_out (pad 32)][16], element
// 8 h + c = W[n][8 chunk + c][tap 2 pair + h]; kConvPadSteps zero pairs of padding
// (the kernel prefetches weights up to that many pairs ahead).
std::vector<bf16_t> pack_conv8(const std::vector<float> &W, int cout, int cin, int k, int cout_pad32) {
  const int taps = k * k * k, pairs = (taps + 1) / 2, nch = (cin + 7) / 8;
  std::vector<bf16_t> out((size_t)(pairs + cf::kConvPadSteps) * nch * cout_pad32 * 16, (bf16_t)0.0f);
  for (int p = 0; p < pairs; ++p)
    for (int ch = 0; ch < nch; ++ch)
      for (int n = 0; n < cout; ++n)
        for (int e = 0; e < 16; ++e) {
          const int tap = 2 * p + e / 8, c = ch * 8 + e % 8;
          if (tap >= taps || c >= cin) continue;
          out[(((size_t)p * nch + ch) * cout_pad32 + n) * 16 + e] = (bf16_t)W[((size_t)n * cin + c) * taps + tap];
        }
  return out;
}

// tap-quad packing: [quad][4-channel chunk][c_out (pad 32)][16], element e of a
// row = tap 4 quad + e / 4, channel 4 chunk + e % 4; kConvPadSteps zero quads past
// the end for the weight prefetch
std::vector<bf16_t> pack_conv4(const std::vector<float> &W, int cout, int cin, int k, int cout_pad32) {
  const int taps = k * k * k, quads = (taps + 3) / 4, nch = (cin + 3) / 4;
  std::vector<bf16_t> out((size_t)(quads + cf::kConvPadSteps) * nch * cout_pad32 * 16, (bf16_t)0.0f);
  for (int q = 0; q < quads; ++q)
    for (int ch = 0; ch < nch; ++ch)
      for (int n = 0; n < cout; ++n)
        for (int e = 0; e < 16; ++e) {
          const int tap = 4 * q + e / 4, c = ch * 4 + e % 4;
          if (tap >= taps || c >= cin) continue;
          out[(((size_t)q * nch + ch) * cout_pad32 + n) * 16 + e] = (bf16_t)W[((size_t)n * cin + c) * taps + tap];
        }
  return out;
}

std::vector<float> transpose(const float *w, int rows, int cols) {  // [rows][cols] -> [cols][rows]
  std::vector<float> t((size_t)rows * cols);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) t[(size_t)c * rows + r] = w[(size_t)r * cols + c];
  return t;
}

int upload_f(cf_ctx *c, float **dst, const float *src, size_t n) {
  return alloc_weight(c, reinterpret_cast<void **>(dst), n * sizeof(float), src);
}

// W [N][K] (row-major) -> split-bfloat16 MFMA B operands [K/16][N][16] (hi, lo)
int upload_split(cf_ctx *c, const float *W, int N, int K, const bf16_t **hi, const bf16_t **lo) {
  std::vector<bf16_t> h((size_t)N * K), l((size_t)N * K);
  for (int ks = 0; ks < K / 16; ++ks)
    for (int n = 0; n < N; ++n)
      for (int e = 0; e < 16; ++e) {
        const float w = W[(size_t)n * K + ks * 16 + e];
        const bf16_t wh = (bf16_t)w;
        const size_t o = ((size_t)ks * N + n) * 16 + e;
        h[o] = wh;
        l[o] = (bf16_t)(w - (float)wh);
      }
  void *ph, *pl;
  int rc = alloc_weight(c, &ph, h.size() * sizeof(bf16_t), h.data());
  if (rc) return rc;
  if ((rc = alloc_weight(c, &pl, l.size() * sizeof(bf16_t), l.data()))) return rc;
  *hi = reinterpret_cast<const bf16_t *>(ph);
  *lo = reinterpret_cast<const bf16_t *>(pl);
  return CF_OK;
}

static_assert(sizeof(cf_model_desc) == 4 * (3 + 40 + 8 + 7), "cf_model_desc layout");

// Compile the model's fusion head (Coherent, Mid-level or Late Fusion) into a
// list of dense layers over the per-pose buffer [cnn latent | sg latent | ...]
// and upload its parameters as one array.
int build_head(cf_ctx *c, BlobReader &R) {
  const cf_model_desc &d = c->desc;
  const int lc = c->lc, H = c->sgw;
  cf::HeadProgram &hp = c->head;
  hp = cf::HeadProgram{};
  std::vector<float> prm;
  int top = lc + H;  // next free slot of the buffer
  // one dense layer reading [slice (src, n_in) ; slice (src1, n1)], writing a new slice
  auto dense = [&](int src, int n_in, int n_out, int act, int res, const char *what, int src1 = 0,
                   int n1 = 0) -> int {
    if (hp.n_ops >= cf::kHeadMaxOps) return fail(CF_ERR_UNSUPPORTED, "fusion head has too many layers");
    if (n_out < 1 || top + n_out > cf::kHeadBuf) return fail(CF_ERR_UNSUPPORTED, "fusion head layers too wide");
    n_in += n1;
    const float *w = R.take((size_t)n_out * n_in), *b = R.take(n_out);
    if (!w || !b) return fail(CF_ERR_INVALID_ARG, std::string("blob truncated (") + what + ")");
    cf::HeadOp &op = hp.op[hp.n_ops++];
    op = cf::HeadOp{src, n_in - n1, src1, n1, top, n_out, act, res, (int)prm.size(), 0};
    prm.insert(prm.end(), w, w + (size_t)n_out * n_in);
    op.b = (int)prm.size();
    prm.insert(prm.end(), b, b + n_out);
    top += n_out;
    return CF_OK;
  };
  int rc;
  if (d.head == CF_HEAD_LATE) {
    if ((rc = dense(0, lc, 1, cf::kActNone, -1, "3D-CNN output"))) return rc;
    const int out_cnn = hp.op[hp.n_ops - 1].dst;
    int src = lc, width = H;
    for (int j = 0; j < 2 && d.sg_dense[j] > 0; ++j) {
      if ((rc = dense(src, width, d.sg_dense[j], cf::kActRelu, -1, "SG-CNN dense"))) return rc;
      src = hp.op[hp.n_ops - 1].dst;
      width = d.sg_dense[j];
    }
    if ((rc = dense(src, width, 1, cf::kActNone, -1, "SG-CNN output"))) return rc;
    hp.n_out = 2;
    hp.out_slot[0] = out_cnn;
    hp.out_slot[1] = hp.op[hp.n_ops - 1].dst;
    hp.out_scale = 0.5f;
  } else {
    // the first fusion layer reads [u_cnn | u_sg] (Mid-level: the model-specific
    // outputs, written next to each other) followed by the raw [cnn | sg]
    int src = 0, width = lc + H, src1 = 0, n1 = 0;
    if (d.head == CF_HEAD_MID) {
      if ((rc = dense(0, lc, lc, cf::kActSelu, -1, "model-specific 3D-CNN"))) return rc;
      const int u0 = hp.op[hp.n_ops - 1].dst;
      if ((rc = dense(lc, H, H, cf::kActSelu, -1, "model-specific SG-CNN"))) return rc;
      src = u0;
      src1 = 0;
      n1 = lc + H;
    }
    for (int l = 0; l + 1 < d.fusion_layers; ++l) {
      const int res = (d.fusion_residual && l > 0) ? src : -1;
      if ((rc = dense(src, width, d.fusion_hidden, cf::kActSelu, res, "fusion layer", src1, n1))) return rc;
      src = hp.op[hp.n_ops - 1].dst;
      width = d.fusion_hidden;
      n1 = 0;
    }
    if ((rc = dense(src, width, 1, cf::kActNone, -1, "fusion output", src1, n1))) return rc;
    hp.n_out = 1;
    hp.out_slot[0] = hp.op[hp.n_ops - 1].dst;
    hp.out_scale = 1.0f;
  }
  return upload_f(c, &c->head_prm, prm.data(), prm.size());
}

int build_model(cf_ctx *c, const void *blob, size_t nbytes) {
  if (!blob || nbytes < sizeof(cf_model_desc)) return fail(CF_ERR_INVALID_ARG, "model blob too small");
  memcpy(&c->desc, blob, sizeof(cf_model_desc));
  const cf_model_desc &d = c->desc;
  if (d.magic != CF_MODEL_MAGIC) return fail(CF_ERR_INVALID_ARG, "bad model magic");
  if (d.n_ch != CF_NCH) return fail(CF_ERR_INVALID_ARG, "model must take 19 feature channels");
  if (d.n_conv < 1 || d.n_conv > 8) return fail(CF_ERR_INVALID_ARG, "n_conv must be 1..8");
  if (d.H_nc == 0 && d.H != 16 && d.H != 32 && d.H != 64)
    return fail(CF_ERR_UNSUPPORTED, "H must be 16, 32 or 64 (without PotentialNet staging)");
  if (d.H_nc != 0 && (d.H < 1 || d.H > 64 || !cf::sgcnn_staged_supported(d.H <= 32 ? 32 : 64, d.H_nc)))
    return fail(CF_ERR_UNSUPPORTED, "staged SG-CNN widths must be H <= 64 and H_nc in {64, 128} (H_nc > H)");
  if (d.cnn_dense2 < 0 || d.cnn_dense2 > 256 || (d.cnn_dense2 && !d.cnn_dense))
    return fail(CF_ERR_INVALID_ARG, "cnn_dense2 needs cnn_dense and must be <= 256");
  if (d.K_c < 0 || d.K_n < 0 || d.K_c > 8 || d.K_n > 8) return fail(CF_ERR_INVALID_ARG, "K_c, K_n must be 0..8");
  if (d.r_cov_u <= 0 || d.r_nc_u <= 0 || d.r_cov_u > 65536 || d.r_nc_u > 65536)
    return fail(CF_ERR_INVALID_ARG, "cutoffs must be 1..65536 u");
  if (d.r_cov_u > d.r_nc_u) return fail(CF_ERR_UNSUPPORTED, "covalent cutoff must not exceed the non-covalent one");
  if (d.cnn_dense < 0 || d.cnn_dense > 256 || d.fusion_hidden < 0 || d.fusion_hidden > 512)
    return fail(CF_ERR_INVALID_ARG, "bad dense sizes");
  if (d.head < CF_HEAD_COHERENT || d.head > CF_HEAD_LATE) return fail(CF_ERR_INVALID_ARG, "unknown head kind");
  if (d.head != CF_HEAD_LATE &&
      (d.fusion_layers < 1 || d.fusion_layers > 8 || (d.fusion_layers > 1) != (d.fusion_hidden > 0)))
    return fail(CF_ERR_INVALID_ARG, "fusion_layers must be 1..8, and > 1 exactly when fusion_hidden > 0");
  if (d.fusion_residual != 0 && d.fusion_residual != 1) return fail(CF_ERR_INVALID_ARG, "fusion_residual must be 0 or 1");
  if (d.sg_dense[0] < 0 || d.sg_dense[1] < 0 || d.sg_dense[0] > 512 || d.sg_dense[1] > 512)
    return fail(CF_ERR_INVALID_ARG, "bad SG-CNN dense sizes");
  BlobReader R{reinterpret_cast<const float *>(reinterpret_cast<const char *>(blob) + sizeof(cf_model_desc)),
               (nbytes - sizeof(cf_model_desc)) / sizeof(float)};
  if ((nbytes - sizeof(cf_model_desc)) % sizeof(float)) return fail(CF_ERR_INVALID_ARG, "blob size not float-aligned");
  const size_t total_floats = R.left;
  const float *const base0 = R.p;
  TrainOffsets &T = c->tr;
  auto at = [&](const float *q) -> int64_t { return (int64_t)(q - base0); };
  int cin = CF_NCH;
  int cin_pad = grid_cpad(c);
  std::vector<int> chans{CF_NCH};
  for (int i = 0; i < d.n_conv; ++i) {
    const int ci = d.conv[i][0], co = d.conv[i][1], k = d.conv[i][2], st = d.conv[i][3], rs = d.conv[i][4];
    if (ci != cin) return fail(CF_ERR_INVALID_ARG, "conv input channels do not chain");
    if (co < 1 || co > 256) return fail(CF_ERR_INVALID_ARG, "conv output channels must be 1..256");
    if (k != 3 && k != 5 && k != 7) return fail(CF_ERR_UNSUPPORTED, "conv kernel size must be 3, 5 or 7");
    if (st != 1 && st != 2) return fail(CF_ERR_INVALID_ARG, "conv stride must be 1 or 2");
    if (rs >= 0) {
      if (rs > i || chans[rs] != co) return fail(CF_ERR_INVALID_ARG, "residual source must match channels");
      // spatial match: every conv between t_rs and t_{i+1} keeps the size
      for (int q = rs; q <= i; ++q)
        if (d.conv[q][3] != 1) return fail(CF_ERR_INVALID_ARG, "residual across a strided conv");
    }
    const size_t nw = (size_t)co * ci * k * k * k;
    const float *W = R.take(nw), *b = R.take(co);
    if (!W || !b) return fail(CF_ERR_INVALID_ARG, "blob truncated (conv)");
    T.conv_w[i] = at(W);
    T.conv_b[i] = at(b);
    T.bn_g[i] = T.bn_b[i] = T.bn_m[i] = T.bn_v[i] = -1;
    std::vector<double> sc(co, 1.0), sh(co, 0.0);
    if (d.bn) {
      const float *g = R.take(co), *bt = R.take(co), *mu = R.take(co), *var = R.take(co);
      if (!g || !bt || !mu || !var) return fail(CF_ERR_INVALID_ARG, "blob truncated (bn)");
      T.bn_g[i] = at(g);
      T.bn_b[i] = at(bt);
      T.bn_m[i] = at(mu);
      T.bn_v[i] = at(var);
      for (int o = 0; o < co; ++o) {
        if (!(var[o] + 1e-5 > 0.0)) return fail(CF_ERR_INVALID_ARG, "BatchNorm variance must be > -eps");
        sc[o] = (double)g[o] / std::sqrt((double)var[o] + 1e-5);
        sh[o] = (double)bt[o] - (double)mu[o] * sc[o];
      }
    }
    // fold: W' = W * sc, b' = b * sc + sh  (== (b - mu) * sc + beta)
    std::vector<float> Wf(nw);
    for (int o = 0; o < co; ++o)
      for (size_t q = 0; q < (size_t)ci * k * k * k; ++q)
        Wf[(size_t)o * ci * k * k * k + q] = (float)((double)W[(size_t)o * ci * k * k * k + q] * sc[o]);
    cf::ConvLayer L{};
    L.cin = ci;
    L.cout = co;
    L.k = k;
    L.stride = st;
    L.res_src = rs;
    L.cin_pad = cin_pad;
    L.in_cm4 = (i == 0 && c->bf16) ? 1 : 0;
    L.spec_f32 = c->bf16 ? 0 : 1;
    L.cout_pad32 = (co + 31) / 32 * 32;
    L.cout_store = c->bf16 ? (co + 15) / 16 * 16 : (co + 7) / 8 * 8;
    std::vector<float> bf(L.cout_pad32, 0.0f);
    for (int o = 0; o < co; ++o) bf[o] = (float)((double)b[o] * sc[o] + sh[o]);
    int rc;
    if (c->bf16) {
      auto pk = pack_conv<bf16_t>(Wf, co, ci, k, cin_pad, L.cout_pad32);
      L.wbytes = (int64_t)(pk.size() * sizeof(bf16_t));
      rc = alloc_weight(c, &L.wpk, pk.size() * sizeof(bf16_t), pk.data());
    } else {
      auto pk = pack_conv<float>(Wf, co, ci, k, cin_pad, L.cout_pad32);
      L.wbytes = (int64_t)(pk.size() * sizeof(float));
      rc = alloc_weight(c, &L.wpk, pk.size() * sizeof(float), pk.data());
    }
    if (L.wbytes >= ((int64_t)1 << 31)) return fail(CF_ERR_UNSUPPORTED, "conv layer weights exceed 2 GiB");
    if (!rc && c->bf16) {
      auto pk8 = pack_conv8(Wf, co, ci, k, L.cout_pad32);
      L.wbytes8 = (int64_t)(pk8.size() * sizeof(bf16_t));
      rc = alloc_weight(c, &L.wpk8, pk8.size() * sizeof(bf16_t), pk8.data());
    }
    if (!rc && c->bf16 && ci % 8 != 0) {
      auto pk4 = pack_conv4(Wf, co, ci, k, L.cout_pad32);
      L.wbytes4 = (int64_t)(pk4.size() * sizeof(bf16_t));
      rc = alloc_weight(c, &L.wpk4, pk4.size() * sizeof(bf16_t), pk4.data());
    }
    if (!rc && cf::fft_conv_layer_ok(L)) {
      // frequency-domain path: in-plane spectra of the folded weights, built on the device
      L.gspec_bytes = cf::fft_conv_gspec_bytes(L);
      rc = alloc_weight(c, &L.gspec, (size_t)L.gspec_bytes, nullptr);
      float *wd = nullptr;
      if (!rc && hipMalloc(&wd, Wf.size() * sizeof(float)) != hipSuccess) rc = fail(CF_ERR_OOM, "weight staging failed");
      if (!rc) {
        if (hipMemcpy(wd, Wf.data(), Wf.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            cf::fft_conv_prepare(L, wd, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
          rc = fail(CF_ERR_HIP, "weight spectra failed");
        (void)hipFree(wd);
      }
    }
    if (rc) return rc;
    if ((rc = upload_f(c, &L.bias, bf.data(), bf.size()))) return rc;
    c->conv.push_back(L);
    chans.push_back(co);
    cin = co;
    cin_pad = L.cout_store;
  }
  c->c_last = cin;
  if (c->c_last > 256) return fail(CF_ERR_UNSUPPORTED, "last conv width must be <= 256");
  int rc;
  if (d.cnn_dense) {
    const float *W = R.take((size_t)d.cnn_dense * c->c_last), *b = R.take(d.cnn_dense);
    if (!W || !b) return fail(CF_ERR_INVALID_ARG, "blob truncated (cnn dense)");
    T.dense_w = at(W);
    T.dense_b = at(b);
    if ((rc = upload_f(c, &c->dense_w, W, (size_t)d.cnn_dense * c->c_last))) return rc;
    if ((rc = upload_f(c, &c->dense_b, b, d.cnn_dense))) return rc;
    c->lc = d.cnn_dense;
    if (d.cnn_dense2) {
      const float *W2 = R.take((size_t)d.cnn_dense2 * d.cnn_dense), *b2 = R.take(d.cnn_dense2);
      if (!W2 || !b2) return fail(CF_ERR_INVALID_ARG, "blob truncated (cnn dense2)");
      T.dense2_w = at(W2);
      T.dense2_b = at(b2);
      if ((rc = upload_f(c, &c->dense2_w, W2, (size_t)d.cnn_dense2 * d.cnn_dense))) return rc;
      if ((rc = upload_f(c, &c->dense2_b, b2, d.cnn_dense2))) return rc;
      c->lc = d.cnn_dense2;
    }
  } else {
    c->lc = c->c_last;
  }
  // SG-CNN.  With PotentialNet staging the covalent stage's width is padded with
  // zero weights to the kernel width (pad features stay exactly 0: their GRU
  // update is (1 - 1/2) tanh(0) + h / 2 with h = 0) and the non-covalent stage
  // runs at H_nc.
  const bool staged = d.H_nc > 0;
  const int Hm[2] = {d.H, staged ? d.H_nc : d.H};          // stage widths in the blob
  const int Hp = staged ? (d.H <= 32 ? 32 : 64) : d.H;
  const int Hs[2] = {Hp, staged ? d.H_nc : Hp};             // stage widths in the kernels
  cf::SgWeights &S = c->sg;
  S.H = Hp;
  S.H2 = Hs[1];
  S.staged = staged;
  S.K_c = d.K_c;
  S.K_n = d.K_n;
  c->sgw = Hs[1];
  c->sg_floats = staged ? 3 * (int64_t)Hp + 2 * (int64_t)Hs[1] : 2 * (int64_t)Hp;
  c->sg_flop_atom = 2.0 * (CF_NCH * Hp + d.K_c * 7.0 * Hp * Hp + d.K_n * 7.0 * Hs[1] * Hs[1] +
                           (staged ? (2.0 * Hp + CF_NCH) * Hp + (double)Hp * Hs[1] : 0.0));
  // W [rows][cols] -> zero-padded [prows][pcols]; source column q goes to q < split ? q : q + shift
  auto padm = [](const float *W, int rows, int cols, int prows, int pcols, int split, int shift) {
    std::vector<float> o((size_t)prows * pcols, 0.0f);
    for (int r = 0; r < rows; ++r)
      for (int q = 0; q < cols; ++q) o[(size_t)r * pcols + (q < split ? q : q + shift)] = W[(size_t)r * cols + q];
    return o;
  };
  // stacked gates [3h][cols] -> [3hp][pcols], each gate's rows padded
  auto padg = [](const float *W, int h, int cols, int hp, int pcols) {
    std::vector<float> o((size_t)3 * hp * pcols, 0.0f);
    for (int g = 0; g < 3; ++g)
      for (int r = 0; r < h; ++r)
        for (int q = 0; q < cols; ++q) o[((size_t)g * hp + r) * pcols + q] = W[((size_t)g * h + r) * cols + q];
    return o;
  };
  auto put = [&](const std::vector<float> &v, const float **dst) -> int {
    float *p;
    int e = upload_f(c, &p, v.data(), v.size());
    *dst = p;
    return e;
  };
  {
    const float *W = R.take((size_t)Hm[0] * CF_NCH), *b = R.take(Hm[0]);
    if (!W || !b) return fail(CF_ERR_INVALID_ARG, "blob truncated (embed)");
    T.embed_w = at(W);
    T.embed_b = at(b);
    if ((rc = put(transpose(padm(W, Hm[0], CF_NCH, Hp, CF_NCH, CF_NCH, 0).data(), Hp, CF_NCH), &S.embed_wT))) return rc;
    if ((rc = put(padm(b, 1, Hm[0], 1, Hp, Hm[0], 0), &S.embed_b))) return rc;
  }
  int r = 0;
  for (int stage = 0; stage < 2; ++stage) {
    const int h = Hm[stage], hp = Hs[stage];
    if (stage == 1 && staged) {
      const int H = d.H;
      const float *gw = R.take((size_t)H * (H + CF_NCH)), *gb = R.take(H);
      const float *vw = R.take((size_t)H * H), *vb = R.take(H);
      const float *ew = R.take((size_t)d.H_nc * H), *eb = R.take(d.H_nc);
      if (!gw || !gb || !vw || !vb || !ew || !eb) return fail(CF_ERR_INVALID_ARG, "blob truncated (covalent gather)");
      if ((rc = put(transpose(padm(gw, H, H + CF_NCH, Hp, Hp + CF_NCH, H, Hp - H).data(), Hp, Hp + CF_NCH),
                    &S.mid_gate_wT)))
        return rc;
      if ((rc = put(padm(gb, 1, H, 1, Hp, H, 0), &S.mid_gate_b))) return rc;
      if ((rc = put(transpose(padm(vw, H, H, Hp, Hp, H, 0).data(), Hp, Hp), &S.mid_val_wT))) return rc;
      if ((rc = put(padm(vb, 1, H, 1, Hp, H, 0), &S.mid_val_b))) return rc;
      if ((rc = put(transpose(padm(ew, d.H_nc, H, d.H_nc, Hp, H, 0).data(), d.H_nc, Hp), &S.embed2_wT))) return rc;
      if ((rc = put(std::vector<float>(eb, eb + d.H_nc), &S.embed2_b))) return rc;
    }
    const int K = stage ? d.K_n : d.K_c;
    for (int q = 0; q < K; ++q, ++r) {
      const float *W = R.take((size_t)h * h);
      if (!W) return fail(CF_ERR_INVALID_ARG, "blob truncated (message)");
      T.msg[r] = at(W);
      const auto Wp = padm(W, h, h, hp, hp, h, 0);
      if ((rc = put(transpose(Wp.data(), hp, hp), &S.msgT[r]))) return rc;
      if (c->bf16 && hp >= 32 && (rc = upload_split(c, Wp.data(), hp, hp, &S.msg_hi[r], &S.msg_lo[r]))) return rc;
    }
    const float *wih = R.take((size_t)3 * h * h), *whh = R.take((size_t)3 * h * h);
    const float *bih = R.take(3 * h), *bhh = R.take(3 * h);
    if (!wih || !whh || !bih || !bhh) return fail(CF_ERR_INVALID_ARG, "blob truncated (gru)");
    T.wih[stage] = at(wih);
    T.whh[stage] = at(whh);
    T.bih[stage] = at(bih);
    T.bhh[stage] = at(bhh);
    const auto wi = padg(wih, h, h, hp, hp), wh = padg(whh, h, h, hp, hp);
    if ((rc = put(transpose(wi.data(), 3 * hp, hp), &S.w_ihT[stage]))) return rc;
    if ((rc = put(transpose(wh.data(), 3 * hp, hp), &S.w_hhT[stage]))) return rc;
    if ((rc = put(padg(bih, h, 1, hp, 1), &S.b_ih[stage]))) return rc;
    if ((rc = put(padg(bhh, h, 1, hp, 1), &S.b_hh[stage]))) return rc;
    if (c->bf16 && hp >= 32) {
      if ((rc = upload_split(c, wi.data(), 3 * hp, hp, &S.ih_hi[stage], &S.ih_lo[stage]))) return rc;
      if ((rc = upload_split(c, wh.data(), 3 * hp, hp, &S.hh_hi[stage], &S.hh_lo[stage]))) return rc;
    }
  }
  {
    // readout gate over [h; u]: u = the raw features, or (staged) the covalent gather
    const int h = Hm[1], hp = Hs[1], u = staged ? d.H : CF_NCH, up = staged ? Hp : CF_NCH;
    const float *gw = R.take((size_t)h * (h + u)), *gb = R.take(h);
    const float *vw = R.take((size_t)h * h), *vb = R.take(h);
    if (!gw || !gb || !vw || !vb) return fail(CF_ERR_INVALID_ARG, "blob truncated (readout)");
    T.gate_w = at(gw);
    T.gate_b = at(gb);
    T.val_w = at(vw);
    T.val_b = at(vb);
    if ((rc = put(transpose(padm(gw, h, h + u, hp, hp + up, h, hp - h).data(), hp, hp + up), &S.gate_wT))) return rc;
    if ((rc = put(padm(gb, 1, h, 1, hp, h, 0), &S.gate_b))) return rc;
    if ((rc = put(transpose(padm(vw, h, h, hp, hp, h, 0).data(), hp, hp), &S.val_wT))) return rc;
    if ((rc = put(padm(vb, 1, h, 1, hp, h, 0), &S.val_b))) return rc;
  }
  T.head = at(R.p);
  if ((rc = build_head(c, R))) return rc;
  if (R.left != 0) return fail(CF_ERR_INVALID_ARG, "blob has trailing data");
  T.head_n = (int64_t)total_floats - T.head;
  c->n_params = (int64_t)total_floats;
  // the plain form keeps the unfolded parameters for the backward pass
  if (!c->bf16 && (rc = alloc_weight(c, reinterpret_cast<void **>(&c->raw), total_floats * sizeof(float), base0)))
    return rc;
  return CF_OK;
}

void free_ctx(cf_ctx *c) {
  for (void *p : c->weight_allocs) (void)hipFree(p);
  for (int64_t *p : c->pin_blocks) (void)hipHostFree(p);
  DevBuf *bufs[] = {&c->grid, &c->centers, &c->cnn_lat, &c->sg_lat, &c->deg, &c->pose_tot,
                    &c->cov_row, &c->cov_col, &c->nc_row, &c->nc_col, &c->hbuf, &c->sel};
  for (DevBuf *b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (auto &b : c->act)
    if (b.p) (void)hipFree(b.p);
  for (auto &b : c->dact)
    if (b.p) (void)hipFree(b.p);
  DevBuf *bw[] = {&c->bw_sg, &c->bw_cnn, &c->bw_part, &c->bw_head, &c->splatwork};
  for (DevBuf *b : bw)
    if (b->p) (void)hipFree(b->p);
  if (c->convwork.p) (void)hipFree(c->convwork.p);
  if (c->status) (void)hipFree(c->status);
  hipEvent_t evs[] = {c->ev_fork, c->ev_sg};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (c->side) (void)hipStreamDestroy(c->side);
  delete c;
}

// per-atom scratch for a pose range holding at most `atoms` atoms
int ensure_atoms(cf_ctx *c, int64_t atoms, int np) {
  int rc;
  if ((rc = ensure(c, c->deg, (size_t)2 * atoms * sizeof(int32_t)))) return rc;
  if ((rc = ensure(c, c->pose_tot, (size_t)4 * np * sizeof(int64_t)))) return rc;
  if ((rc = ensure(c, c->cov_row, (size_t)(atoms + 1) * sizeof(int32_t)))) return rc;
  if ((rc = ensure(c, c->nc_row, (size_t)(atoms + 1) * sizeof(int32_t)))) return rc;
  if ((rc = ensure(c, c->cov_col, (size_t)atoms * 16 * sizeof(int32_t)))) return rc;
  if ((rc = ensure(c, c->nc_col, (size_t)atoms * 96 * sizeof(int32_t)))) return rc;
  if ((rc = ensure(c, c->hbuf, (size_t)atoms * c->sg_floats * sizeof(float)))) return rc;
  return CF_OK;
}

int64_t atoms_cap_for(const cf_pose_batch *b, int np) {
  return std::min<int64_t>((int64_t)b->n_atoms, (int64_t)np * CF_MAX_POSE_ATOMS);
}

}  // namespace

extern "C" {

const char *cf_last_error(void) { return g_last_error.c_str(); }

int cf_create(const void *blob, size_t nbytes, int precision, int64_t hbm_budget_bytes, cf_ctx **out) {
  if (!out) return fail(CF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (precision != CF_PREC_FP32 && precision != CF_PREC_BF16) return fail(CF_ERR_INVALID_ARG, "bad precision");
  cf_ctx *c = new (std::nothrow) cf_ctx();
  if (!c) return fail(CF_ERR_OOM, "host allocation failed");
  c->bf16 = precision == CF_PREC_BF16;
  if (hbm_budget_bytes > 0) {
    c->budget = hbm_budget_bytes;
  } else {  // default: half of the device's memory, at most 64 GiB
    size_t free_b = 0, total_b = 0;
    c->budget = (int64_t)16 << 30;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && total_b > 0)
      c->budget = std::min<int64_t>((int64_t)64 << 30, (int64_t)(total_b / 2));
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(CF_ERR_HIP, "no HIP device");
  }
  int rc = build_model(c, blob, nbytes);
  if (rc == CF_OK) {
    if (hipMalloc(&c->status, 4 * sizeof(int64_t)) != hipSuccess ||
        hipMemset(c->status, 0, 4 * sizeof(int64_t)) != hipSuccess)
      rc = fail(CF_ERR_OOM, "status word allocation failed");
  }
  if (rc == CF_OK &&
      (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&c->ev_sg, hipEventDisableTiming) != hipSuccess))
    rc = fail(CF_ERR_HIP, "stream or event creation failed");
  if (rc != CF_OK) {
    free_ctx(c);
    return rc;
  }
  *out = c;
  return CF_OK;
}

void cf_destroy(cf_ctx *c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  free_ctx(c);
}

int cf_model_info(const cf_ctx *c, int32_t *latent_cnn, int32_t *latent_sg, int64_t *n_params, int32_t *precision) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  if (latent_cnn) *latent_cnn = c->lc;
  if (latent_sg) *latent_sg = c->sgw;
  if (n_params) *n_params = c->n_params;
  if (precision) *precision = c->bf16 ? CF_PREC_BF16 : CF_PREC_FP32;
  return CF_OK;
}

int cf_pose_centers(cf_ctx *c, const cf_pose_batch *b, int32_t *center_out, void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  int rc = validate_batch(b);
  if (rc) return rc;
  if (!center_out) return fail(CF_ERR_INVALID_ARG, "center_out is NULL");
  CF_HIP(cf::launch_centers(b->atom_off, b->n_atoms, b->xyz, b->is_lig, 0, b->n_poses, center_out, c->status, (hipStream_t)stream));
  return CF_OK;
}

int cf_voxelize(cf_ctx *c, const cf_pose_batch *b, int G, void *grid_out, void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  int rc = validate_batch(b);
  if (rc) return rc;
  if ((rc = validate_G(G))) return rc;
  if (!grid_out) return fail(CF_ERR_INVALID_ARG, "grid_out is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int32_t *cen = b->center;
  if (!cen) {
    if ((rc = ensure(c, c->centers, (size_t)b->n_poses * 3 * sizeof(int32_t)))) return rc;
    CF_HIP(cf::launch_centers(b->atom_off, b->n_atoms, b->xyz, b->is_lig, 0, b->n_poses, (int32_t *)c->centers.p, c->status, s));
    cen = (const int32_t *)c->centers.p;
  }
  if ((rc = ensure(c, c->splatwork, (size_t)cf::splat_work_bytes(b->n_poses, b->n_atoms, G)))) return rc;
  CF_HIP(cf::launch_splat(b->atom_off, b->n_atoms, b->xyz, b->feat, cen, 0, b->n_poses, G, grid_out, c->bf16 ? 1 : 0, 0,
                          c->splatwork.p, b->n_atoms, c->status, s));
  return CF_OK;
}

int cf_build_graphs(cf_ctx *c, const cf_pose_batch *b, cf_csr *cov, cf_csr *nc, void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  int rc = validate_batch(b);
  if (rc) return rc;
  if (!cov || !nc || !cov->row_ptr || !nc->row_ptr || (cov->capacity > 0 && !cov->col) ||
      (nc->capacity > 0 && !nc->col) || cov->capacity < 0 || nc->capacity < 0)
    return fail(CF_ERR_INVALID_ARG, "bad CSR arguments");
  if ((rc = ensure(c, c->deg, (size_t)2 * b->n_atoms * sizeof(int32_t)))) return rc;
  if ((rc = ensure(c, c->pose_tot, (size_t)4 * b->n_poses * sizeof(int64_t)))) return rc;
  CF_HIP(cf::launch_graph(b->atom_off, b->n_atoms, b->xyz, 0, b->n_poses, c->desc.r_cov_u, c->desc.r_nc_u, cov->row_ptr,
                          cov->col, cov->capacity, nc->row_ptr, nc->col, nc->capacity, (int32_t *)c->deg.p,
                          (int64_t)b->n_atoms, (int64_t *)c->pose_tot.p, c->status, (hipStream_t)stream));
  return CF_OK;
}

int cf_cnn3d_fwd(cf_ctx *c, const void *grid, int32_t n_poses, int G, float *cnn_latent, void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  if (!grid || !cnn_latent || n_poses < 1) return fail(CF_ERR_INVALID_ARG, "bad arguments");
  int rc = validate_G(G);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int chunk = chunk_poses(c, G, n_poses);
  if ((rc = ensure_act(c, G, chunk))) return rc;
  const int64_t vox = (int64_t)G * G * G;
  for (int p0 = 0; p0 < n_poses; p0 += chunk) {
    const int np = std::min(chunk, n_poses - p0);
    const char *src = reinterpret_cast<const char *>(grid) + (size_t)p0 * vox * CF_NCH * elem_size(c);
    CF_HIP(cf::launch_grid_repack(src, c->bf16, (int)(np * vox), c->grid.p, c->bf16, grid_cpad(c), s,
                                  c->bf16 ? (int64_t)vox : 0));
    if ((rc = run_cnn(c, G, np, cnn_latent + (size_t)p0 * c->lc, s))) return rc;
  }
  return CF_OK;
}

int cf_sgcnn_fwd(cf_ctx *c, const cf_pose_batch *b, const cf_csr *cov, const cf_csr *nc, float *sg_latent,
                 void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  int rc = validate_batch(b);
  if (rc) return rc;
  if (!cov || !nc || !cov->row_ptr || !nc->row_ptr || !sg_latent) return fail(CF_ERR_INVALID_ARG, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const int chunk = std::min(b->n_poses, 512);
  const int64_t acap = atoms_cap_for(b, chunk);
  if ((rc = ensure(c, c->hbuf, (size_t)acap * c->sg_floats * sizeof(float)))) return rc;
  for (int p0 = 0; p0 < b->n_poses; p0 += chunk) {
    const int np = std::min(chunk, b->n_poses - p0);
    CF_HIP(cf::launch_sgcnn(c->sg, c->bf16, b->atom_off, b->n_atoms, b->feat, b->is_lig, p0, np, cov->row_ptr, cov->col,
                            cov->capacity, nc->row_ptr, nc->col, nc->capacity, 1, (float *)c->hbuf.p, acap,
                            sg_latent + (size_t)p0 * c->sgw, c->status, s));
  }
  return CF_OK;
}

int cf_fusion_fwd(cf_ctx *c, const float *cnn_latent, const float *sg_latent, int32_t n_poses, float *scores,
                  void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  if (!cnn_latent || !sg_latent || !scores || n_poses < 1) return fail(CF_ERR_INVALID_ARG, "bad arguments");
  CF_HIP(cf::launch_head(cnn_latent, c->lc, sg_latent, c->sgw, c->head_prm, c->head, n_poses, scores,
                         (hipStream_t)stream));
  return CF_OK;
}

int cf_score_poses(cf_ctx *c, const cf_pose_batch *b, int G, float *scores, void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  int rc = validate_batch(b);
  if (rc) return rc;
  if ((rc = validate_G(G))) return rc;
  if (!scores) return fail(CF_ERR_INVALID_ARG, "scores is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int chunk = chunk_poses(c, G, b->n_poses, b->n_atoms);
  const int64_t acap = atoms_cap_for(b, chunk);
  if ((rc = ensure_act(c, G, chunk))) return rc;
  if ((rc = ensure_atoms(c, acap, chunk))) return rc;
  if ((rc = ensure(c, c->centers, (size_t)chunk * 3 * sizeof(int32_t)))) return rc;
  if ((rc = ensure(c, c->cnn_lat, (size_t)chunk * c->lc * sizeof(float)))) return rc;
  if ((rc = ensure(c, c->sg_lat, (size_t)chunk * c->sgw * sizeof(float)))) return rc;
  if ((rc = ensure(c, c->splatwork, (size_t)cf::splat_work_bytes(chunk, acap, G)))) return rc;
  const int H = c->sgw;
  // The graph / SG-CNN branch of each chunk runs on the context's side stream,
  // forked once the chunk's first conv layer is enqueued (ev_fork, recorded on
  // `stream` after it) so that it overlaps the remaining layers rather than the
  // first, whose halo fills a CU's LDS; the head joins the branch (ev_sg).  The
  // fork also orders the branch after the caller's prior work and after the
  // previous chunk's head, which read the SG latents it overwrites.
  hipStream_t s2 = c->side;
  for (int p0 = 0; p0 < b->n_poses; p0 += chunk) {
    const int np = std::min(chunk, b->n_poses - p0);
    const int32_t *cen;
    const double atoms = (double)b->n_atoms * np / b->n_poses;  // for the byte counts only
    if (b->center) {
      cen = b->center + 3 * (size_t)p0;
    } else {
      hipEvent_t e = tbegin(c, s);
      CF_HIP(cf::launch_centers(b->atom_off, b->n_atoms, b->xyz, b->is_lig, p0, np, (int32_t *)c->centers.p, c->status, s));
      tend(c, s, e, "centers", 0.0, atoms * 13.0);
      cen = (const int32_t *)c->centers.p;
    }
    hipEvent_t e = tbegin(c, s);
    {
      Range r(c, "cf.splat");
      CF_HIP(cf::launch_splat(b->atom_off, b->n_atoms, b->xyz, b->feat, cen, p0, np, G, c->grid.p, c->bf16 ? 4 : 2,
                              grid_cpad(c), c->splatwork.p, acap, c->status, s));
    }
    tend(c, s, e, "splat", 0.0, atoms * (12.0 + 4.0 * CF_NCH) + (double)np * G * G * G * CF_NCH * elem_size(c));
    {
      Range r(c, "cf.cnn3d");
      if ((rc = run_cnn(c, G, np, (float *)c->cnn_lat.p, s, c->ev_fork))) return rc;
    }
    {
    Range rg(c, "cf.graph_sgcnn");
    CF_HIP(hipStreamWaitEvent(s2, c->ev_fork, 0));
    hipEvent_t eg = tbegin(c, s2);
    CF_HIP(cf::launch_graph(b->atom_off, b->n_atoms, b->xyz, p0, np, c->desc.r_cov_u, c->desc.r_nc_u, (int32_t *)c->cov_row.p,
                            (int32_t *)c->cov_col.p, acap * 16, (int32_t *)c->nc_row.p, (int32_t *)c->nc_col.p,
                            acap * 96, (int32_t *)c->deg.p, acap, (int64_t *)c->pose_tot.p, c->status, s2));
    // algorithmic bytes: coordinates read once, two row-pointer arrays and 4 B per
    // edge written (the edge totals arrive with the events)
    tend(c, s2, eg, "graph", 0.0, atoms * (12.0 + 8.0));
    if (c->timing && !c->pending.empty() && c->pending.back().key == "graph") {
      int64_t *slot = pin_slots(c);
      const int64_t *pt = (const int64_t *)c->pose_tot.p;
      if (slot) {
        const int64_t idx[4] = {np - 1, 2 * (int64_t)np - 1, 3 * (int64_t)np - 1, 4 * (int64_t)np - 1};
        for (int q = 0; q < 4; ++q)
          CF_HIP(hipMemcpyAsync(slot + q, pt + idx[q], sizeof(int64_t), hipMemcpyDeviceToHost, s2));
        c->pending.back().edges = slot;
      }
    }
    eg = tbegin(c, s2);
    CF_HIP(cf::launch_sgcnn(c->sg, c->bf16, b->atom_off, b->n_atoms, b->feat, b->is_lig, p0, np, (int32_t *)c->cov_row.p,
                            (int32_t *)c->cov_col.p, acap * 16, (int32_t *)c->nc_row.p, (int32_t *)c->nc_col.p,
                            acap * 96, 0, (float *)c->hbuf.p, acap, (float *)c->sg_lat.p, c->status, s2));
    tend(c, s2, eg, "sgcnn", atoms * c->sg_flop_atom, atoms * 4.0 * CF_NCH);
    CF_HIP(hipEventRecord(c->ev_sg, s2));
    }
    CF_HIP(hipStreamWaitEvent(s, c->ev_sg, 0));
    Range rh(c, "cf.head");
    e = tbegin(c, s);
    CF_HIP(cf::launch_head((float *)c->cnn_lat.p, c->lc, (float *)c->sg_lat.p, H, c->head_prm, c->head, np,
                           scores + p0, s));
    tend(c, s, e, "fusion", 0.0, 0.0);
  }
  return CF_OK;
}

int cf_backward(cf_ctx *c, const cf_pose_batch *b, int G, const float *dscore, float *grad, float *scores,
                void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  int rc = validate_batch(b);
  if (rc) return rc;
  if ((rc = validate_G(G))) return rc;
  if (!dscore || !grad) return fail(CF_ERR_INVALID_ARG, "dscore and grad must not be NULL");
  if (c->bf16 || !c->raw) return fail(CF_ERR_UNSUPPORTED, "the backward pass runs in the plain (FP32) form");
  const cf_model_desc &d = c->desc;
  if (d.head != CF_HEAD_COHERENT) return fail(CF_ERR_UNSUPPORTED, "the backward pass covers the Coherent Fusion head");
  if (d.H_nc != 0) return fail(CF_ERR_UNSUPPORTED, "the backward pass covers the unstaged SG-CNN");
  const int H = d.H, R = d.K_c + d.K_n, L = (int)c->conv.size();
  const int nhid = d.fusion_layers - 1, fh = d.fusion_hidden;
  if (!cf::bw_head_ok(c->lc + H, fh, nhid)) return fail(CF_ERR_UNSUPPORTED, "fusion head too wide for the backward pass");
  hipStream_t s = (hipStream_t)stream;
  // the per-atom launches are sized on the host: read the offsets back once
  std::vector<int32_t> off((size_t)b->n_poses + 1);
  CF_HIP(hipMemcpyAsync(off.data(), b->atom_off, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CF_HIP(hipStreamSynchronize(s));
  if (off[0] != 0 || off[b->n_poses] != b->n_atoms) return fail(CF_ERR_INVALID_ARG, "atom_off[0] must be 0 and atom_off[P] = n_atoms");
  for (int p = 0; p < b->n_poses; ++p)
    if (off[p + 1] - off[p] < 1 || off[p + 1] - off[p] > CF_MAX_POSE_ATOMS)
      return fail(CF_ERR_INVALID_ARG, "atom_off malformed (each pose needs 1..4096 atoms)");

  constexpr int kBwChunk = 32;
  const int chunk = std::min(kBwChunk, chunk_poses(c, G, b->n_poses, b->n_atoms));
  int64_t max_atoms = 0;
  for (int p0 = 0; p0 < b->n_poses; p0 += chunk)
    max_atoms = std::max<int64_t>(max_atoms, off[std::min(b->n_poses, p0 + chunk)] - off[p0]);
  const int64_t acap = max_atoms;
  if ((rc = ensure_act(c, G, chunk))) return rc;
  if ((rc = ensure_atoms(c, acap, chunk))) return rc;
  if ((rc = ensure(c, c->centers, (size_t)chunk * 3 * sizeof(int32_t)))) return rc;
  if ((rc = ensure(c, c->cnn_lat, (size_t)chunk * c->lc * sizeof(float)))) return rc;
  if ((rc = ensure(c, c->sg_lat, (size_t)chunk * c->sgw * sizeof(float)))) return rc;
  if ((rc = ensure(c, c->splatwork, (size_t)cf::splat_work_bytes(chunk, acap, G)))) return rc;
  // layer sizes
  std::vector<int> dims{G};
  for (auto &Lr : c->conv) dims.push_back(conv_out_dim(dims.back(), Lr.k, Lr.stride));
  auto vox = [&](int i) { return (int64_t)dims[i] * dims[i] * dims[i]; };
  if ((int)c->dact.size() != L) c->dact.resize(L);
  for (int i = 0; i < L; ++i)
    if ((rc = ensure(c, c->dact[i], (size_t)chunk * vox(i + 1) * c->conv[i].cout_store * sizeof(float)))) return rc;
  // SG scratch (floats): states H[R+1], messages M[R], gate inputs GI[R], GH[R]
  // (3H each), then per-atom work rows
  const int64_t nH = acap * H, n3 = acap * 3 * H;
  const int64_t sg_floats = (R + 1) * nH + R * nH + 2 * R * n3 + 9 * nH + 2 * n3;
  if ((rc = ensure(c, c->bw_sg, (size_t)sg_floats * sizeof(float)))) return rc;
  // CNN scratch: per-pose weight-gradient partials, the pose sum, folded transposed
  // weights, bias gradient; pool / dense rows
  int64_t wq = 0;
  for (int i = 0; i < L; ++i)
    wq = std::max<int64_t>(wq, (int64_t)c->conv[i].cout * c->conv[i].cin * c->conv[i].k * c->conv[i].k * c->conv[i].k);
  const int dmax = 256;
  const int64_t cnn_floats = (int64_t)chunk * wq + 2 * wq + 256 + 8 * (int64_t)chunk * dmax;
  if ((rc = ensure(c, c->bw_cnn, (size_t)cnn_floats * sizeof(float)))) return rc;
  // head: per-pose parameter gradients and the latents' gradients
  const int64_t head_floats = (int64_t)chunk * c->tr.head_n + (int64_t)chunk * (c->lc + H) + 2 * (int64_t)chunk;
  if ((rc = ensure(c, c->bw_head, (size_t)head_floats * sizeof(float)))) return rc;
  // partial sums of the ordered reductions (the largest any call below needs)
  int64_t part = cf::bw_outer_scratch(chunk, (int)c->tr.head_n, 1);
  part = std::max(part, cf::bw_outer_scratch((int)acap, 3 * H, H));
  part = std::max(part, cf::bw_outer_scratch((int)acap, H, H + CF_NCH));
  part = std::max(part, cf::bw_outer_scratch(chunk, (int)wq, 1));
  part = std::max(part, cf::bw_outer_scratch(chunk, dmax, dmax));
  for (int i = 0; i < L; ++i) part = std::max(part, cf::bw_outer_scratch((int)(chunk * vox(i + 1)), c->conv[i].cout, 1));
  if ((rc = ensure(c, c->bw_part, (size_t)part * sizeof(float)))) return rc;

  const float *P = c->raw;
  const TrainOffsets &T = c->tr;
  float *pt = (float *)c->bw_part.p;
  CF_HIP(cf::bw_fill(grad, c->n_params, 0.0f, s));
  for (int p0 = 0; p0 < b->n_poses; p0 += chunk) {
    const int np = std::min(chunk, b->n_poses - p0);
    const int a0 = off[p0], n = off[p0 + np] - a0;
    const float *x = b->feat + (int64_t)a0 * CF_NCH;
    const int32_t *cen = b->center ? b->center + 3 * (size_t)p0 : (const int32_t *)c->centers.p;
    // ---- forward, keeping what the backward reads ----
    if (!b->center)
      CF_HIP(cf::launch_centers(b->atom_off, b->n_atoms, b->xyz, b->is_lig, p0, np, (int32_t *)c->centers.p, c->status, s));
    CF_HIP(cf::launch_splat(b->atom_off, b->n_atoms, b->xyz, b->feat, cen, p0, np, G, c->grid.p, 2, grid_cpad(c),
                            c->splatwork.p, acap, c->status, s));
    if ((rc = run_cnn(c, G, np, (float *)c->cnn_lat.p, s, nullptr, true))) return rc;
    CF_HIP(cf::launch_graph(b->atom_off, b->n_atoms, b->xyz, p0, np, d.r_cov_u, d.r_nc_u, (int32_t *)c->cov_row.p,
                            (int32_t *)c->cov_col.p, acap * 16, (int32_t *)c->nc_row.p, (int32_t *)c->nc_col.p,
                            acap * 96, (int32_t *)c->deg.p, acap, (int64_t *)c->pose_tot.p, c->status, s));
    const int32_t *rp[2] = {(int32_t *)c->cov_row.p, (int32_t *)c->nc_row.p};
    const int32_t *cl[2] = {(int32_t *)c->cov_col.p, (int32_t *)c->nc_col.p};
    const int64_t cap[2] = {acap * 16, acap * 96};
    float *Hs = (float *)c->bw_sg.p;       // [R + 1][n][H]
    float *Ms = Hs + (R + 1) * nH;         // [R][n][H]
    float *GI = Ms + R * nH, *GH = GI + R * n3;  // [R][n][3H]
    float *As = GH + R * n3, *Gp = As + nH, *Vv = Gp + nH, *dH = Vv + nH, *dHd = dH + nH, *dA = dHd + nH;
    float *dM = dA + nH, *dGp = dM + nH, *dV = dGp + nH, *dGI = dV + nH, *dGH = dGI + n3;
    auto Hr = [&](int r) { return Hs + (int64_t)r * n * H; };
    auto stage_of = [&](int r) { return r < d.K_c ? 0 : 1; };
    CF_HIP(cf::bw_rowmat(x, CF_NCH, n, CF_NCH, P + T.embed_w, CF_NCH, P + T.embed_b, H, Hr(0), H, 0, s));
    for (int r = 0; r < R; ++r) {
      const int st = stage_of(r);
      float *Mr = Ms + (int64_t)r * n * H, *GIr = GI + (int64_t)r * n * 3 * H, *GHr = GH + (int64_t)r * n * 3 * H;
      CF_HIP(cf::bw_agg(rp[st], cl[st], cap[st], Hr(r), n, H, As, 0, c->status, s));
      CF_HIP(cf::bw_rowmat(As, H, n, H, P + T.msg[r], H, nullptr, H, Mr, H, 0, s));
      CF_HIP(cf::bw_rowmat(Mr, H, n, H, P + T.wih[st], H, P + T.bih[st], 3 * H, GIr, 3 * H, 0, s));
      CF_HIP(cf::bw_rowmat(Hr(r), H, n, H, P + T.whh[st], H, P + T.bhh[st], 3 * H, GHr, 3 * H, 0, s));
      CF_HIP(cf::bw_gru_fwd(GIr, GHr, Hr(r), n, H, Hr(r + 1), s));
    }
    CF_HIP(cf::bw_rowmat(Hr(R), H, n, H, P + T.gate_w, H + CF_NCH, P + T.gate_b, H, Gp, H, 0, s));
    CF_HIP(cf::bw_rowmat(x, CF_NCH, n, CF_NCH, P + T.gate_w + H, H + CF_NCH, nullptr, H, Gp, H, 1, s));
    CF_HIP(cf::bw_rowmat(Hr(R), H, n, H, P + T.val_w, H, P + T.val_b, H, Vv, H, 0, s));
    float *sgl = (float *)c->sg_lat.p;
    CF_HIP(cf::bw_readout(Gp, Vv, b->is_lig, b->atom_off, p0, np, H, sgl, s));
    // ---- head ----
    float *hpart = (float *)c->bw_head.p, *dcnn = hpart + (int64_t)chunk * T.head_n, *dsg = dcnn + (int64_t)chunk * c->lc;
    CF_HIP(cf::bw_head((float *)c->cnn_lat.p, c->lc, sgl, H, P + T.head, nhid, fh, d.fusion_residual, dscore + p0, np,
                       scores ? scores + p0 : nullptr, dcnn, dsg, hpart, T.head_n, s));
    CF_HIP(cf::bw_outer(hpart, (int)T.head_n, nullptr, 0, np, (int)T.head_n, 1, grad + T.head, 1, 1, pt, s));
    // ---- SG-CNN backward ----
    CF_HIP(cf::bw_readout_bwd(Gp, Vv, b->is_lig, b->atom_off, p0, np, H, n, dsg, dGp, dV, s));
    CF_HIP(cf::bw_outer(dGp, H, Hr(R), H, n, H, H, grad + T.gate_w, H + CF_NCH, 1, pt, s));
    CF_HIP(cf::bw_outer(dGp, H, x, CF_NCH, n, H, CF_NCH, grad + T.gate_w + H, H + CF_NCH, 1, pt, s));
    CF_HIP(cf::bw_outer(dGp, H, nullptr, 0, n, H, 1, grad + T.gate_b, 1, 1, pt, s));
    CF_HIP(cf::bw_outer(dV, H, Hr(R), H, n, H, H, grad + T.val_w, H, 1, pt, s));
    CF_HIP(cf::bw_outer(dV, H, nullptr, 0, n, H, 1, grad + T.val_b, 1, 1, pt, s));
    CF_HIP(cf::bw_rowmat_t(dGp, H, n, H, P + T.gate_w, H + CF_NCH, H, dH, H, 0, s));
    CF_HIP(cf::bw_rowmat_t(dV, H, n, H, P + T.val_w, H, H, dH, H, 1, s));
    for (int r = R - 1; r >= 0; --r) {
      const int st = stage_of(r);
      float *Mr = Ms + (int64_t)r * n * H, *GIr = GI + (int64_t)r * n * 3 * H, *GHr = GH + (int64_t)r * n * 3 * H;
      CF_HIP(cf::bw_gru_bwd(GIr, GHr, Hr(r), dH, n, H, dGI, dGH, dHd, s));
      CF_HIP(cf::bw_outer(dGI, 3 * H, Mr, H, n, 3 * H, H, grad + T.wih[st], H, 1, pt, s));
      CF_HIP(cf::bw_outer(dGI, 3 * H, nullptr, 0, n, 3 * H, 1, grad + T.bih[st], 1, 1, pt, s));
      CF_HIP(cf::bw_outer(dGH, 3 * H, Hr(r), H, n, 3 * H, H, grad + T.whh[st], H, 1, pt, s));
      CF_HIP(cf::bw_outer(dGH, 3 * H, nullptr, 0, n, 3 * H, 1, grad + T.bhh[st], 1, 1, pt, s));
      CF_HIP(cf::bw_rowmat_t(dGI, 3 * H, n, 3 * H, P + T.wih[st], H, H, dM, H, 0, s));  // dm
      CF_HIP(cf::bw_rowmat_t(dGH, 3 * H, n, 3 * H, P + T.whh[st], H, H, dHd, H, 1, s));
      CF_HIP(cf::bw_agg(rp[st], cl[st], cap[st], Hr(r), n, H, As, 0, c->status, s));  // the round's neighbour sums
      CF_HIP(cf::bw_outer(dM, H, As, H, n, H, H, grad + T.msg[r], H, 1, pt, s));
      CF_HIP(cf::bw_rowmat_t(dM, H, n, H, P + T.msg[r], H, H, dA, H, 0, s));
      // a_i = sum_{j in N(i)} h_j: dh_j += sum_{i : j in N(i)} da_i, and the graphs are
      // symmetric (a distance test), so that is the neighbour sum of da over N(j)
      CF_HIP(cf::bw_agg(rp[st], cl[st], cap[st], dA, n, H, dHd, 1, c->status, s));
      std::swap(dH, dHd);
    }
    CF_HIP(cf::bw_outer(dH, H, x, CF_NCH, n, H, CF_NCH, grad + T.embed_w, CF_NCH, 1, pt, s));
    CF_HIP(cf::bw_outer(dH, H, nullptr, 0, n, H, 1, grad + T.embed_b, 1, 1, pt, s));
    // ---- 3D-CNN backward ----
    float *part = (float *)c->bw_cnn.p, *dWf = part + (int64_t)chunk * wq, *WT = dWf + wq, *dbf = WT + wq;
    float *pool = dbf + 256, *pre1 = pool + (int64_t)chunk * dmax, *lat1 = pre1 + (int64_t)chunk * dmax;
    float *pre2 = lat1 + (int64_t)chunk * dmax, *dl2 = pre2 + (int64_t)chunk * dmax, *dl1 = dl2 + (int64_t)chunk * dmax;
    float *dpool = dl1 + (int64_t)chunk * dmax;
    const auto &Ll = c->conv.back();
    CF_HIP(cf::bw_pool_mean((float *)c->act[L - 1].p, np, vox(L), Ll.cout_store, Ll.cout, pool, s));
    const float *dlat = dcnn;
    if (d.cnn_dense) {
      const int d1 = d.cnn_dense, d2 = d.cnn_dense2;
      CF_HIP(cf::bw_rowmat(pool, Ll.cout, np, Ll.cout, P + T.dense_w, Ll.cout, P + T.dense_b, d1, pre1, d1, 0, s));
      CF_HIP(hipMemcpyAsync(lat1, pre1, (size_t)np * d1 * sizeof(float), hipMemcpyDeviceToDevice, s));
      CF_HIP(cf::bw_relu_rows(lat1, np, d1, d1, s));
      if (d2) {
        CF_HIP(cf::bw_rowmat(lat1, d1, np, d1, P + T.dense2_w, d1, P + T.dense2_b, d2, pre2, d2, 0, s));
        CF_HIP(hipMemcpyAsync(dl2, dlat, (size_t)np * d2 * sizeof(float), hipMemcpyDeviceToDevice, s));
        CF_HIP(cf::bw_relu_grad_rows(dl2, pre2, np, d2, s));
        CF_HIP(cf::bw_outer(dl2, d2, lat1, d1, np, d2, d1, grad + T.dense2_w, d1, 1, pt, s));
        CF_HIP(cf::bw_outer(dl2, d2, nullptr, 0, np, d2, 1, grad + T.dense2_b, 1, 1, pt, s));
        CF_HIP(cf::bw_rowmat_t(dl2, d2, np, d2, P + T.dense2_w, d1, d1, dl1, d1, 0, s));
      } else {
        CF_HIP(hipMemcpyAsync(dl1, dlat, (size_t)np * d1 * sizeof(float), hipMemcpyDeviceToDevice, s));
      }
      CF_HIP(cf::bw_relu_grad_rows(dl1, pre1, np, d1, s));
      CF_HIP(cf::bw_outer(dl1, d1, pool, Ll.cout, np, d1, Ll.cout, grad + T.dense_w, Ll.cout, 1, pt, s));
      CF_HIP(cf::bw_outer(dl1, d1, nullptr, 0, np, d1, 1, grad + T.dense_b, 1, 1, pt, s));
      CF_HIP(cf::bw_rowmat_t(dl1, d1, np, d1, P + T.dense_w, Ll.cout, Ll.cout, dpool, Ll.cout, 0, s));
    } else {
      CF_HIP(hipMemcpyAsync(dpool, dlat, (size_t)np * Ll.cout * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    CF_HIP(cf::bw_pool_seed(dpool, np, vox(L), Ll.cout_store, Ll.cout, (float *)c->dact[L - 1].p, s));
    for (int i = 0; i < L - 1; ++i)
      CF_HIP(cf::bw_fill((float *)c->dact[i].p, (int64_t)np * vox(i + 1) * c->conv[i].cout_store, 0.0f, s));
    for (int i = L - 1; i >= 0; --i) {
      const auto &Lr = c->conv[i];
      const int taps = Lr.k * Lr.k * Lr.k;
      float *dY = (float *)c->dact[i].p;
      const int64_t ny = (int64_t)np * vox(i + 1) * Lr.cout_store;
      CF_HIP(cf::bw_relu_mask(dY, (float *)c->act[i].p, ny, s));
      if (Lr.res_src >= 1) CF_HIP(cf::bw_add((float *)c->dact[Lr.res_src - 1].p, dY, ny, s));
      CF_HIP(cf::bw_outer(dY, Lr.cout_store, nullptr, 0, (int)(np * vox(i + 1)), Lr.cout, 1, dbf, 1, 0, pt, s));
      const float *X = i == 0 ? (const float *)c->grid.p : (const float *)c->act[i - 1].p;
      const int xs = i == 0 ? grid_cpad(c) : c->conv[i - 1].cout_store;
      const int64_t Q = (int64_t)taps * Lr.cin;
      CF_HIP(cf::bw_conv_wgrad(X, dims[i], xs, Lr.cin, dY, dims[i + 1], Lr.cout_store, Lr.cout, Lr.k, Lr.stride, np,
                               part, s));
      CF_HIP(cf::bw_outer(part, (int)(Lr.cout * Q), nullptr, 0, np, (int)(Lr.cout * Q), 1, dWf, 1, 0, pt, s));
      const bool bn = d.bn != 0;
      CF_HIP(cf::bw_fold_grad(dWf, dbf, P + T.conv_w[i], P + T.conv_b[i], bn ? P + T.bn_g[i] : nullptr,
                              bn ? P + T.bn_m[i] : nullptr, bn ? P + T.bn_v[i] : nullptr, Lr.cout, Lr.cin, taps,
                              grad + T.conv_w[i], grad + T.conv_b[i], bn ? grad + T.bn_g[i] : nullptr,
                              bn ? grad + T.bn_b[i] : nullptr, bn ? grad + T.bn_m[i] : nullptr,
                              bn ? grad + T.bn_v[i] : nullptr, s));
      if (i > 0) {
        CF_HIP(cf::bw_fold_wt(P + T.conv_w[i], bn ? P + T.bn_g[i] : nullptr, bn ? P + T.bn_v[i] : nullptr, Lr.cout,
                              Lr.cin, taps, WT, s));
        CF_HIP(cf::bw_conv_dgrad(dY, dims[i + 1], Lr.cout_store, Lr.cout, WT, Lr.cin, Lr.k, Lr.stride, dims[i], xs, np,
                                 (float *)c->dact[i - 1].p, s));
      }
    }
  }
  return CF_OK;
}

int cf_compound_max(cf_ctx *c, const float *scores, int32_t n_scores, const int32_t *compound_off,
                    int32_t n_compounds, float *best_score, int32_t *best_pose, void *stream) {
  if (!c || !scores || !compound_off || !best_score || !best_pose) return fail(CF_ERR_INVALID_ARG, "null argument");
  if (n_scores < 0 || n_compounds < 0) return fail(CF_ERR_INVALID_ARG, "negative size");
  CF_HIP(cf::launch_segmax(scores, n_scores, compound_off, n_compounds, best_score, best_pose, c->status,
                           (hipStream_t)stream));
  return CF_OK;
}

int cf_top_k(cf_ctx *c, const float *values, int32_t n, int32_t k, int32_t *idx_out, float *val_out, void *stream) {
  if (!c || !values || !idx_out) return fail(CF_ERR_INVALID_ARG, "null argument");
  if (n < 0 || k < 0 || k > n) return fail(CF_ERR_INVALID_ARG, "need 0 <= k <= n");
  if (k > 1024) return fail(CF_ERR_UNSUPPORTED, "k must be <= 1024");
  if (k == 0) return CF_OK;
  int rc = ensure(c, c->sel, cf::kTopkScratchBytes);
  if (rc) return rc;
  CF_HIP(cf::launch_topk(values, n, k, idx_out, val_out, c->sel.p, (hipStream_t)stream));
  return CF_OK;
}

int cf_top_k_noalloc(const float *values, int32_t n, int32_t k, int32_t *idx_out, float *val_out, void *stream) {
  if (!values || !idx_out) return fail(CF_ERR_INVALID_ARG, "null argument");
  if (n < 0 || k < 0 || k > n) return fail(CF_ERR_INVALID_ARG, "need 0 <= k <= n");
  if (k > cf::kTopkMaxK)
    return fail(CF_ERR_UNSUPPORTED, "k = " + std::to_string(k) + " exceeds the " + std::to_string(cf::kTopkMaxK) +
                                        " keys the static top-k scratch holds");
  if (k == 0) return CF_OK;
  void *scratch = nullptr;
  CF_HIP(cf::topk_static_scratch(&scratch));
  CF_HIP(cf::launch_topk(values, n, k, idx_out, val_out, scratch, (hipStream_t)stream));
  return CF_OK;
}

int cf_stream_status(cf_ctx *c, void *stream, int64_t *need_cov, int64_t *need_nc) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  CF_HIP(hipStreamSynchronize((hipStream_t)stream));
  int64_t st[4];
  CF_HIP(hipMemcpy(st, c->status, sizeof(st), hipMemcpyDeviceToHost));
  CF_HIP(hipMemset(c->status, 0, sizeof(st)));
  if (need_cov) *need_cov = st[1];
  if (need_nc) *need_nc = st[2];
  switch (st[0]) {
    case cf::kDevOk: return CF_OK;
    case cf::kDevCapacity: return fail(CF_ERR_CAPACITY, "neighbour list capacity exceeded");
    case cf::kDevBadOffsets: return fail(CF_ERR_INVALID_ARG, "atom_off malformed (decreasing, or a pose outside 1..4096 atoms)");
    case cf::kDevBadFeature: return fail(CF_ERR_INVALID_ARG, "feature value not finite or |value| > 64");
    case cf::kDevPoseTooLarge: return fail(CF_ERR_INVALID_ARG, "a pose has more than 4096 atoms");
    case cf::kDevBadGraph: return fail(CF_ERR_INVALID_ARG, "neighbour list references an atom of another pose");
    case cf::kDevGridRange:
      return fail(CF_ERR_INVALID_ARG, "atoms too dense for the grid accumulators: over one 2 x 4 x G voxel tile the "
                                      "sum of ceil(max |feature|) of the atoms whose 1.5 A reach overlaps it exceeds 4096");
    default: return fail(CF_ERR_INVALID_ARG, "device reported an invalid input");
  }
}

int cf_timing_enable(cf_ctx *c, int enable) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  c->timing = (enable & CF_TIMING_EVENTS) != 0;
  c->roctx = (enable & CF_TIMING_ROCTX) != 0;
  return CF_OK;
}

int cf_timing_read(cf_ctx *c, cf_kernel_stat *out, int32_t max_entries, int32_t *n_out) {
  if (!c || (!out && max_entries > 0)) return fail(CF_ERR_INVALID_ARG, "bad arguments");
  // the edge-total copies follow their launch's end event on the same stream:
  // wait for the last recorded event before reading them
  if (!c->pending.empty()) CF_HIP(hipEventSynchronize(c->pending.back().e1));
  for (auto &p : c->pending) {
    CF_HIP(hipEventSynchronize(p.e1));
    float ms = 0.0f;
    CF_HIP(hipEventElapsedTime(&ms, p.e0, p.e1));
    auto &st = c->stats[p.key];
    st.launches += 1;
    st.ms += ms;
    st.flop += p.flop;
    st.bytes += p.bytes;
    if (p.edges) st.bytes += 4.0 * (double)(p.edges[0] + p.edges[1] + p.edges[2] + p.edges[3]);
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
  }
  c->pending.clear();
  c->pin_used = 0;
  int n = 0;
  for (auto &kv : c->stats) {
    if (n < max_entries) {
      memset(&out[n], 0, sizeof(cf_kernel_stat));
      strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = kv.second.launches;
      out[n].total_ms = kv.second.ms;
      out[n].flop = kv.second.flop;
      out[n].bytes = kv.second.bytes;
    }
    ++n;
  }
  if (n_out) *n_out = n;
  c->stats.clear();
  return CF_OK;
}

int cf_conv_variants(const cf_ctx *c, int G, int32_t *variant_out, int32_t max_layers) {
  if (!c || !variant_out) return fail(CF_ERR_INVALID_ARG, "bad arguments");
  std::vector<int> v;
  int rc = variants_for(const_cast<cf_ctx *>(c), G, v);
  if (rc) return rc;
  for (int i = 0; i < (int)v.size() && i < max_layers; ++i) variant_out[i] = v[i];
  return CF_OK;
}

int cf_set_conv_variants(cf_ctx *c, int G, const int32_t *variants, int32_t n_layers) {
  if (!c || !variants) return fail(CF_ERR_INVALID_ARG, "bad arguments");
  int rc = validate_G(G);
  if (rc) return rc;
  if (n_layers != (int32_t)c->conv.size()) return fail(CF_ERR_INVALID_ARG, "one variant per conv layer is needed");
  std::vector<int> v(variants, variants + n_layers);
  int D = G;
  for (int i = 0; i < n_layers; ++i) {
    if (!cf::conv_variant_ok(v[i], c->conv[i], c->bf16, D))
      return fail(CF_ERR_UNSUPPORTED, "variant does not fit layer " + std::to_string(i));
    D = conv_out_dim(D, c->conv[i].k, c->conv[i].stride);
    if (D < 1) return fail(CF_ERR_UNSUPPORTED, "grid too small for the conv stack");
  }
  c->variants[G] = v;
  return CF_OK;
}

int cf_conv_variant_count(void) { return cf::conv_num_variants(); }

const char *cf_conv_variant_name(int32_t variant) { return cf::conv_variant_name(variant); }

int cf_autotune(cf_ctx *c, int G, int32_t n_poses, void *stream) {
  if (!c) return fail(CF_ERR_INVALID_ARG, "ctx is NULL");
  int rc = validate_G(G);
  if (rc) return rc;
  if (n_poses < 1) return fail(CF_ERR_INVALID_ARG, "n_poses must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  const int np = std::min(n_poses, chunk_poses(c, G, n_poses));
  if ((rc = ensure_act(c, G, np))) return rc;
  // seeded random activations (constant operands would time a higher clock)
  CF_HIP(cf::launch_fill_random(c->grid.p, (int64_t)c->grid.n, c->bf16, 1, s));
  for (size_t i = 0; i < c->act.size(); ++i)
    CF_HIP(cf::launch_fill_random(c->act[i].p, (int64_t)c->act[i].n, c->bf16, 2 + i, s));
  std::vector<int> best;
  const char *ve = getenv("CF_AUTOTUNE_VERBOSE");
  const bool verbose = ve && ve[0] && ve[0] != '0';
  hipEvent_t e0, e1;
  CF_HIP(hipEventCreate(&e0));
  CF_HIP(hipEventCreate(&e1));
  std::vector<const void *> t{c->grid.p};
  for (auto &b : c->act) t.push_back(b.p);
  {
    int64_t work = 0;
    int D = G;
    for (size_t i = 0; i < c->conv.size(); ++i) {
      for (int v = 0; v < cf::conv_num_variants(); ++v)
        if (cf::conv_variant_ok(v, c->conv[i], c->bf16, D))
          work = std::max(work, cf::conv_work_bytes(v, c->conv[i], D, np));
      D = conv_out_dim(D, c->conv[i].k, c->conv[i].stride);
    }
    if (work > 0 && (rc = ensure(c, c->convwork, (size_t)work))) return rc;
  }
  int D = G;
  for (size_t i = 0; i < c->conv.size(); ++i) {
    const auto &L = c->conv[i];
    float best_ms = 1e30f;
    int best_v = -1;
    for (int v = 0; v < cf::conv_num_variants(); ++v) {
      if (!cf::conv_variant_ok(v, L, c->bf16, D)) continue;
      const void *res = L.res_src >= 0 ? t[L.res_src] : nullptr;
      void *wk = c->convwork.p;
      CF_HIP(cf::launch_conv(v, L, c->bf16, t[i], res, c->act[i].p, np, D, wk, s));  // warm-up
      CF_HIP(hipEventRecord(e0, s));
      for (int rep = 0; rep < 3; ++rep) CF_HIP(cf::launch_conv(v, L, c->bf16, t[i], res, c->act[i].p, np, D, wk, s));
      CF_HIP(hipEventRecord(e1, s));
      CF_HIP(hipEventSynchronize(e1));
      float ms = 0;
      CF_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (verbose) {
        const double Do = conv_out_dim(D, L.k, L.stride);
        const double tf = 2.0 * L.cin * L.cout * L.k * L.k * L.k * Do * Do * Do * np / (ms / 3.0 * 1e-3) / 1e12;
        fprintf(stderr, "[cf_autotune] G=%d layer %zu variant %2d %-24s %8.3f ms %7.1f TFLOP/s\n", G, i, v,
                cf::conv_variant_name(v), ms / 3.0, tf);
      }
      if (ms < best_ms) {
        best_ms = ms;
        best_v = v;
      }
    }
    if (best_v < 0) return fail(CF_ERR_UNSUPPORTED, "no conv kernel for a layer");
    best.push_back(best_v);
    D = conv_out_dim(D, L.k, L.stride);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->variants[G] = best;
  return CF_OK;
}

}  // extern "C"

namespace cf {
int64_t scratch_generation(const cf_ctx *c) { return c ? c->scratch_gen : 0; }
}  // namespace cf
