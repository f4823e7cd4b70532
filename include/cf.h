/*
 * cf.h -- C ABI of the Coherent Fusion pose scorer for AMD Instinct MI355X (gfx950).
 *
 * The library scores docked protein-ligand poses with a Coherent Fusion model
 * (Stevenson et al., "High-Throughput Virtual Screening of Small Molecule
 * Inhibitors for SARS-CoV-2 Protein Targets with Deep Fusion Models", SC 2021):
 * each pose is turned into a voxel grid read by a 3D-CNN and into a spatial graph
 * with covalent and non-covalent edges read by an SG-CNN; the two latents are
 * concatenated and fused into one predicted affinity pK = -log K (Sec. 1,
 * Sec. 2.1 Eq. 1, Sec. 2.2, Fig. 1, Sec. 3.3).  The paper's screening runs score
 * fixed-size batches of featurised poses per GPU and return one prediction per
 * pose (Sec. 4.2); this ABI takes such a batch, ragged and packed, and returns
 * one score per pose.
 *
 * Conventions (all entry points):
 *   - Array pointers inside cf_pose_batch / cf_csr and all grid / latent / score
 *     pointers are DEVICE pointers owned by the caller.  The library never frees
 *     them and never keeps them after the call returns.
 *   - Every compute call is asynchronous on `stream` (a hipStream_t; NULL is the
 *     default stream) and returns a cf_status.  Argument errors that the host can
 *     see (sizes, null pointers, unsupported shapes) are reported before anything
 *     is enqueued.  Errors only the device can see (malformed offsets, CSR
 *     capacity overflow, coordinates or features out of range) set a per-context
 *     device status word that cf_stream_status() reports.
 *   - A context is not re-entrant: use one context per host thread at a time.
 *     Several contexts may share a device.
 *   - No C++ exception crosses this boundary.  cf_last_error() returns a
 *     thread-local message for the last non-OK status.
 *
 * Units and layouts:
 *   - Coordinates are int32 in u = 2^-10 Angstrom.  All distance tests are exact
 *     integer tests (so neighbour lists are reproducible bit for bit).
 *   - 19 feature channels per atom, float32, |value| <= 64.
 *   - Voxel grids are channels-last: grid[pose][i][j][k][channel], where voxel
 *     (i, j, k) has centre center + (i - (G-1)/2, j - (G-1)/2, k - (G-1)/2) A
 *     (1 A spacing).
 */
#ifndef CF_H
#define CF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CF_OK = 0,
  CF_ERR_INVALID_ARG = -1, /* bad argument (host) or malformed batch data (device) */
  CF_ERR_CAPACITY = -2,    /* a caller-provided CSR is too small; see cf_stream_status */
  CF_ERR_OOM = -3,         /* device allocation failed or would exceed the HBM budget */
  CF_ERR_HIP = -4,         /* a HIP runtime call failed */
  CF_ERR_UNSUPPORTED = -5, /* valid request outside what the library implements */
  CF_ERR_CANCELLED = -6    /* serving request cancelled before it was scheduled */
} cf_status;

typedef enum {
  CF_PREC_FP32 = 0, /* plain form: every stage in float32 */
  CF_PREC_BF16 = 1  /* precision form: conv3d and graph-conv GEMMs take bfloat16
                       operands (round to nearest even) with float32 accumulation;
                       splatting, folded BatchNorm bias, gates and the fusion head
                       stay float32 */
} cf_precision;

#define CF_NCH 19            /* feature channels per atom */
#define CF_MAX_POSE_ATOMS 4096
#define CF_MODEL_MAGIC 0x314D4643u /* "CFM1" */

/* Fusion head forms (Sec. 2.1-2.2; Tables IV-V).  Coherent: SELU fusion layers
 * over the concatenated latents.  Mid-level: each latent first passes through its
 * own SELU dense layer, whose output joins the raw latents before the fusion
 * layers (optionally residual).  Late: each branch predicts a pK on its own and
 * the score is their unweighted mean.  Dropout is the identity at inference. */
typedef enum { CF_HEAD_COHERENT = 0, CF_HEAD_MID = 1, CF_HEAD_LATE = 2 } cf_head_kind;

typedef struct cf_ctx cf_ctx;

/* A ragged batch of poses, packed CSR-style: atoms of pose p are rows
 * atom_off[p] .. atom_off[p+1]-1 of xyz / feat / is_lig. */
typedef struct {
  int32_t n_poses;          /* P >= 1 */
  int32_t n_atoms;          /* N = atom_off[P] */
  const int32_t *atom_off;  /* [P+1], atom_off[0] = 0, each pose has 1..4096 atoms */
  const int32_t *xyz;       /* [N][3] coordinates, units 2^-10 A */
  const float *feat;        /* [N][19] atom features */
  const uint8_t *is_lig;    /* [N] 1 = ligand atom, 0 = pocket atom */
  const int32_t *center;    /* [P][3] grid centres (2^-10 A) or NULL: the library then
                               uses the rounded ligand centroid (cf_pose_centers) */
} cf_pose_batch;

/* Compressed sparse rows of a neighbour list.  row_ptr has n_atoms+1 entries,
 * col has `capacity` entries; columns are global atom ids, ascending in a row. */
typedef struct {
  int32_t *row_ptr;
  int32_t *col;
  int64_t capacity;
} cf_csr;

/* Model blob (host memory), little-endian:
 *   cf_model_desc header, then float32 parameters in this order --
 *   for each conv i: W [c_out][c_in][k][k][k], b [c_out], and if bn:
 *       gamma, beta, running_mean, running_var (each [c_out]);
 *   if cnn_dense: W [cnn_dense][c_out_last], b [cnn_dense];
 *   if cnn_dense2: W [cnn_dense2][cnn_dense], b [cnn_dense2];
 *   SG-CNN (S = the SG latent width: H_nc if H_nc > 0, else H):
 *       embed W [H][19], b [H];
 *       covalent stage: message W_t [H][H] for each of its K_c rounds, then GRU
 *       w_ih [3H][H], w_hh [3H][H], b_ih [3H], b_hh [3H] (gate rows stacked r, z, n);
 *       if H_nc > 0 (PotentialNet staging): covalent gather gate W [H][H+19], b [H],
 *       value W [H][H], b [H]; embedding W [H_nc][H], b [H_nc];
 *       non-covalent stage: as the covalent one at width S (K_n rounds);
 *       readout gate W [S][S+U], b [S] (U = 19, or H with staging: the gate reads
 *       [h; covalent gather]); readout value W [S][S], b [S];
 *   head CF_HEAD_LATE: 3D-CNN output W [1][latent_cnn], b [1]; for each
 *       sg_dense[j] > 0: W [sg_dense[j]][previous width], b [sg_dense[j]];
 *       SG-CNN output W [1][last width], b [1];
 *   head CF_HEAD_MID: model-specific W [latent_cnn][latent_cnn], b [latent_cnn],
 *       then W [S][S], b [S]; then the fusion block below, its input being
 *       [specific cnn; specific sg; cnn latent; sg latent] (2 (latent_cnn + S));
 *   head CF_HEAD_COHERENT: the fusion block over [cnn latent; sg latent];
 *   fusion block: fusion_layers - 1 hidden layers W [fusion_hidden][input width],
 *       b [fusion_hidden], then output W [1][fusion_hidden or input width], b [1].
 * Conv i reads tensor t_i and writes t_{i+1} (t_0 = voxel grid); res_src >= 0
 * adds t_{res_src} before the ReLU of conv i. */
typedef struct {
  uint32_t magic;        /* CF_MODEL_MAGIC */
  int32_t n_ch;          /* must be 19 */
  int32_t n_conv;        /* 1..8 */
  int32_t conv[8][5];    /* c_in, c_out, k (3, 5 or 7), stride (1|2), res_src */
  int32_t bn;            /* 1: inference BatchNorm after every conv */
  int32_t cnn_dense;     /* 0: CNN latent = pooled features; else dense + ReLU width */
  int32_t H;             /* SG-CNN width: 16, 32 or 64 (covalent stage: 1..64 with H_nc) */
  int32_t K_c, K_n;      /* covalent / non-covalent propagation rounds (<= 8 each) */
  int32_t r_cov_u;       /* covalent cutoff, 2^-10 A */
  int32_t r_nc_u;        /* non-covalent cutoff, 2^-10 A */
  int32_t fusion_hidden; /* width of the fusion block's hidden SELU layers */
  int32_t head;          /* cf_head_kind */
  int32_t fusion_layers; /* dense layers of the fusion block incl. the output, 1..8;
                            > 1 requires fusion_hidden > 0 (unused by CF_HEAD_LATE) */
  int32_t fusion_residual; /* 1: hidden layers after the first add their input */
  int32_t sg_dense[2];   /* CF_HEAD_LATE: SG-CNN dense (ReLU) widths before its
                            output, 0 = absent (a 0 ends the list) */
  int32_t cnn_dense2;    /* second 3D-CNN dense + ReLU width (needs cnn_dense), 0 = none */
  int32_t H_nc;          /* 0, or PotentialNet staging (Sec. 3.3.1, Table II gather
                            widths): the covalent stage (width H) ends in a per-atom
                            gated gather, embedded to the non-covalent stage's width
                            H_nc (64 or 128, > H) */
} cf_model_desc;

/* Create a scoring context on the current device.  Copies the weights (the blob
 * may be freed afterwards), folds BatchNorm into the conv weights and bias in
 * double precision (stored float32), and repacks weights for the kernels.
 * hbm_budget_bytes bounds the
 * scratch the context may allocate (0 = half of the
 * device memory, at most 64 GiB); batches larger than the budget
 * allows are scored in chunks.  Section refs: model structure Sec. 2.2, 3.3. */
int cf_create(const void *host_model_blob, size_t nbytes, int precision,
              int64_t hbm_budget_bytes, cf_ctx **out);
void cf_destroy(cf_ctx *ctx);

/* Grid centre of every pose: the ligand centroid rounded to the nearest unit
 * (halves up), floor((2*sum x + n) / (2*n)) per axis over ligand atoms; the
 * centroid of all atoms if a pose has none.  center_out: device [P][3] int32.
 * (Grid placement is deferred by the paper to its predecessor, Sec. 3.3.) */
int cf_pose_centers(cf_ctx *ctx, const cf_pose_batch *batch, int32_t *center_out, void *stream);

/* Voxelise every pose (3D representation, Sec. 1; grid sizing and atom
 * propagation, Sec. 3.3): each atom spreads its features over the voxels within
 * 1.5 A (3 sigma, sigma = 0.5 A) of it with weights exp(-d^2 / (2 sigma^2)),
 * normalised over that whole support; voxels outside the grid are dropped.
 * grid_out: device [P][G][G][G][19], float32 (ctx precision FP32) or bfloat16
 * (BF16).  G a multiple of 4, 8 <= G <= 96. */
int cf_voxelize(cf_ctx *ctx, const cf_pose_batch *batch, int G, void *grid_out, void *stream);

/* Covalent (d <= r_cov) and non-covalent (d <= r_nc) neighbour lists: all
 * ordered pairs i != j of the same pose (two edge types by distance threshold,
 * Sec. 1; thresholds Table II).  Rows by atom, columns ascending, global atom
 * ids.  If an edge count exceeds a capacity, nothing beyond the capacity is
 * written, row_ptr is still complete, and cf_stream_status returns
 * CF_ERR_CAPACITY with the required counts. */
int cf_build_graphs(cf_ctx *ctx, const cf_pose_batch *batch, cf_csr *cov, cf_csr *nc, void *stream);

/* 3D-CNN head (Sec. 3.3.1, Table III): conv stack with folded BatchNorm, ReLU
 * and residual adds, global average pooling, optional dense + ReLU.
 * grid: device [P][G][G][G][19] in the context's precision (as cf_voxelize
 * writes it).  cnn_latent: device [P][latent_cnn] float32. */
int cf_cnn3d_fwd(cf_ctx *ctx, const void *grid, int32_t n_poses, int G, float *cnn_latent, void *stream);

/* SG-CNN head (PotentialNet / gated graph sequence networks, Sec. 3.3.1,
 * Table II): linear embedding, K_c covalent then K_n non-covalent rounds of
 * neighbour sum -> message matrix -> GRU update, then a sigmoid-gated sum over
 * ligand atoms.  cov / nc as written by cf_build_graphs for the same batch.
 * sg_latent: device [P][H] float32. */
int cf_sgcnn_fwd(cf_ctx *ctx, const cf_pose_batch *batch, const cf_csr *cov, const cf_csr *nc,
                 float *sg_latent, void *stream);

/* Fusion head alone (Eq. 1; Sec. 2.1-2.2, Tables IV-V, per the model's
 * cf_head_kind): one pK per pose from its two latents.  cnn_latent: device
 * [P][latent_cnn] float32; sg_latent: device [P][H] float32; scores: device [P]
 * float32.  Computed in float32 in both precision forms. */
int cf_fusion_fwd(cf_ctx *ctx, const float *cnn_latent, const float *sg_latent, int32_t n_poses, float *scores,
                  void *stream);

/* Whole path: centres (unless given), voxelisation, 3D-CNN, neighbour lists,
 * SG-CNN and the model's fusion head (Coherent Fusion by default, Sec. 2.2,
 * 3.3.3, Table V; inference without dropout).  scores: device [P] float32 pK, in
 * batch order.  Uses context-owned scratch; poses are processed in chunks. */
int cf_score_poses(cf_ctx *ctx, const cf_pose_batch *batch, int G, float *scores, void *stream);

/* Synchronise `stream`, then report and clear the context's device status word:
 * CF_OK, or the first device-side error since the last call.  For
 * CF_ERR_CAPACITY, *need_cov / *need_nc (if non-NULL) receive the edge counts a
 * retry needs. */
int cf_stream_status(cf_ctx *ctx, void *stream, int64_t *need_cov, int64_t *need_nc);

/* Thread-local description of the last non-OK status returned on this thread. */
const char *cf_last_error(void);

/* Model summary: latent widths, parameter count, precision. */
int cf_model_info(const cf_ctx *ctx, int32_t *latent_cnn, int32_t *latent_sg, int64_t *n_params,
                  int32_t *precision);

/* Conv autotuning (batching form): time the candidate tile / wave layouts of
 * every conv layer at grid size G on a synthetic batch of n_poses poses and keep
 * the fastest per layer (cached in the context and reused for that G). */
int cf_autotune(cf_ctx *ctx, int G, int32_t n_poses, void *stream);

/* Chosen kernel variant per conv layer for grid size G (after cf_autotune or the
 * default table): variant_out[n_conv]. */
int cf_conv_variants(const cf_ctx *ctx, int G, int32_t *variant_out, int32_t max_layers);
/* Pin the conv kernel variant of every layer for grid size G (e.g. a cached
 * autotuning result).  CF_ERR_UNSUPPORTED if a variant does not fit its layer. */
int cf_set_conv_variants(cf_ctx *ctx, int G, const int32_t *variants, int32_t n_layers);
/* Number of conv kernel variants in the library and the name of one (tile shape,
 * waves, output-channel tile; "p8" = bf16 tap-pair kernel). */
int cf_conv_variant_count(void);
const char *cf_conv_variant_name(int32_t variant);

/* Per-kernel timing (diagnostics).  While enabled, every kernel launch made by
 * the scoring entry points is bracketed by a pair of HIP events recorded on the
 * launch's own stream.  cf_timing_read synchronises on them and returns, per
 * kernel kind (conv layers are keyed "conv<i>.<variant>"), the launch count,
 * summed device time and the algorithmic FLOPs and bytes those launches cover
 * (for a conv layer: 2 * c_in * c_out * k^3 * output voxels; padding channels
 * are not counted).  Reading clears the accumulated entries.  out may hold
 * max_entries entries; *n_out receives the number available. */
typedef struct {
  char name[64];
  int32_t launches;
  double total_ms;
  double flop;
  double bytes;
} cf_kernel_stat;
/* enable: a bit set of CF_TIMING_EVENTS (the event pairs above) and CF_TIMING_ROCTX
 * (roctx ranges "cf.splat", "cf.cnn3d", "cf.graph_sgcnn", "cf.head" around what
 * cf_score_poses enqueues for each chunk, for a tracer such as rocprofv3
 * --marker-trace; the roctx library is opened at run time and, when it is absent,
 * the ranges are skipped).  0 turns both off. */
#define CF_TIMING_EVENTS 1
#define CF_TIMING_ROCTX 2
int cf_timing_enable(cf_ctx *ctx, int enable);
int cf_timing_read(cf_ctx *ctx, cf_kernel_stat *out, int32_t max_entries, int32_t *n_out);

/* ---- Backward pass (fine-tuning) ----------------------------------------------
 * Coherent Fusion trains the fusion layers and both branches together, the loss
 * gradient reaching the 3D-CNN and the SG-CNN through the concatenated latents
 * (Sec. 2.2; training hyper-parameters in Table V).  cf_backward scores the batch
 * and returns, for one upstream gradient per pose dscore[p] = dL/ds_p (e.g. s_p -
 * y_p for a squared-error loss), grad[theta] = sum_p dscore[p] ds_p/dtheta for
 * every parameter theta of the model blob, in the blob's order and layout
 * (n_params floats, cf_model_info), BatchNorm running mean and variance included.
 * grad is overwritten.  scores (device [P]) or NULL receives the scores the
 * forward computed.  All pointers are device pointers owned by the caller.
 * Requirements: a CF_PREC_FP32 context (float32 throughout), the Coherent Fusion
 * head and the unstaged SG-CNN (H_nc = 0); otherwise CF_ERR_UNSUPPORTED.  Unlike
 * the scoring calls it reads batch->atom_off back to the host (one synchronous
 * copy on `stream`) to size its per-atom launches, and checks it there.  Poses
 * are processed in chunks of at most 32; every reduction runs in a fixed order,
 * so the result is reproducible bit for bit.  Device-detected input errors are
 * reported by cf_stream_status as for scoring. */
int cf_backward(cf_ctx *ctx, const cf_pose_batch *batch, int G, const float *dscore, float *grad, float *scores,
                void *stream);

/* ---- Selection after scoring --------------------------------------------------
 * Per-compound aggregation: the paper represents each compound by its strongest
 * prediction over all its docked poses (the maximum Coherent Fusion pK; up to 10
 * poses per site, Sec. 5.2).  Segment c covers scores[compound_off[c] ..
 * compound_off[c+1]); best_score[c] is its maximum and best_pose[c] the lowest
 * index attaining it.  NaN scores are ignored; an empty (or all-NaN) segment gives
 * -inf and -1.  Offsets outside [0, n_scores] are reported by cf_stream_status.
 * All pointers are device pointers. */
int cf_compound_max(cf_ctx *ctx, const float *scores, int32_t n_scores, const int32_t *compound_off,
                    int32_t n_compounds, float *best_score, int32_t *best_pose, void *stream);
/* Top-k selection (the paper's example: the best 100 of a million screened
 * compounds, Sec. 3.4): the k largest values in descending order, ties by lower
 * index, NaN last; idx_out [k], val_out [k] or NULL.  0 <= k <= min(n, 1024). */
int cf_top_k(cf_ctx *ctx, const float *values, int32_t n, int32_t k, int32_t *idx_out, float *val_out,
             void *stream);
/* cf_top_k without a context, for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, ordering and results as cf_top_k, but its scratch
 * (histogram, select state and up to 1024 keys, 9,280 bytes) is a static device
 * array of the library, one copy per GPU held until the process ends, whose
 * address is looked up once per device on the first call there.  Calls no
 * hipMalloc / hipFree and clears what must start at zero with a kernel.  k > 1024
 * returns CF_ERR_UNSUPPORTED.  Calls on one GPU share the array: two calls whose
 * work overlaps on that GPU (different streams, or different host threads without
 * ordering) race and may return wrong results; calls ordered on one stream are
 * safe. */
int cf_top_k_noalloc(const float *values, int32_t n, int32_t k, int32_t *idx_out, float *val_out, void *stream);

/* ---- Serving engine (continuous batching) ------------------------------------
 * The request-driven form of the paper's per-GPU scoring loop (Sec. 4.2): each
 * request carries one or more poses (host arrays, copied before submit returns)
 * and its own grid size.  A scheduler thread owns n_slots device slots (a stream,
 * a scoring context with resident weights and scratch, pinned staging); whenever
 * a slot is free it packs queued requests of one grid size, in arrival order,
 * into one batch of up to slot_poses poses / slot_atoms atoms, pads it with empty
 * poses to a power-of-two bucket and replays the hipGraph captured for that
 * (grid size, bucket) -- so requests that arrive while others run are admitted as
 * slots free up, and batches on different slots overlap on the device.  A pose's
 * score is bitwise the same whatever batch it lands in.  Each slot's context
 * gets an equal share of hbm_budget_bytes and splits a batch into chunks that
 * fit it; queued work waits for a free slot and is never rejected for lack of
 * memory. */
typedef struct cf_engine cf_engine;
typedef struct {
  int32_t n_slots;          /* 1..8 concurrent batches */
  int32_t slot_poses;       /* poses per batch, 1..512 */
  int64_t slot_atoms;       /* atoms per batch */
  int64_t hbm_budget_bytes; /* for all slots together; 0 = 32 GiB */
  int32_t use_graphs;       /* 1: capture and replay hipGraphs per (G, bucket) */
  int32_t reserved;
} cf_engine_config;
int cf_engine_create(const void *host_model_blob, size_t nbytes, int precision, const cf_engine_config *cfg,
                     cf_engine **out);
/* Host pointers: atom_off [n_poses+1] (atom_off[0] = 0), xyz [N][3], feat [N][19],
 * is_lig [N]; G a multiple of 4 in 8..96.  Returns a ticket for cf_engine_poll.
 * Offsets and features (finite, |value| <= 64) are checked here, so a malformed
 * request is rejected before it can share a batch.  Should the device still
 * report an error for a batch (e.g. neighbour lists overflowing the batch's edge
 * capacity), each of its requests is scored again alone and only the one at
 * fault returns the error; every request's scores are the ones it gets alone. */
int cf_engine_submit(cf_engine *e, int32_t n_poses, const int32_t *atom_off, const int32_t *xyz, const float *feat,
                     const uint8_t *is_lig, int32_t G, uint64_t *ticket);
/* *done = 1 once scored: scores_out (host [n_poses]) and *latency_ms (submit to
 * scores on the host) are filled, the ticket is released and the request's
 * status (device-side checks included) is returned. */
int cf_engine_poll(cf_engine *e, uint64_t ticket, float *scores_out, int32_t *done, double *latency_ms);
/* Cancel a request that is still queued: it leaves the queue and is never scored;
 * *cancelled = 1, and cf_engine_poll then reports it done with CF_ERR_CANCELLED
 * (releasing the ticket).  A request already packed into a batch on the device
 * runs to completion (*cancelled = 0).  The paper's screening jobs isolate
 * failures by rescheduling work (Sec. 4.3); a serving caller withdraws work this
 * way (a deadline passed, a client went away). */
int cf_engine_cancel(cf_engine *e, uint64_t ticket, int32_t *cancelled);
int cf_engine_wait_all(cf_engine *e);
int cf_engine_info(cf_engine *e, int64_t *poses_done, int64_t *batches, int64_t *graph_replays, int64_t *queued);
const char *cf_engine_last_error(cf_engine *e);
void cf_engine_destroy(cf_engine *e);

#ifdef __cplusplus
}
#endif

#endif /* CF_H */
