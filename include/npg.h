/*
 * npg.h -- C-ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of photon-driven neural path guiding (Zhu et al., "Photon-Driven
 * Neural Path Guiding", arXiv 2010.01775):
 *
 *   photons -> leaves of an adaptive spatial hierarchy   npg_build_hierarchy
 *   -> per-leaf 2D directional histograms                npg_splat_histograms
 *   -> raw sampling map (normalised energy)              npg_normalize_input
 *   -> CNN reconstruction of a sampling density          npg_reconstruct_density
 *   -> pdf + marginal/conditional CDF tables             npg_build_cdf
 *   -> guided direction sampling / pdf evaluation        npg_sample_dirs, npg_eval_pdf
 *
 * Conventions (all entry points):
 *  - Pointers whose names end in _dev are device pointers OWNED BY THE CALLER
 *    (for instance memory of torch tensors).  The library never frees or
 *    reallocates them.  It allocates only its own scratch space and model
 *    weights, charged against the context's HBM budget.
 *  - Every call takes the caller's stream (a hipStream_t passed as void*,
 *    NULL = the default stream), only enqueues work and returns without
 *    waiting, except where a call says it synchronises.  Calls on one context
 *    must be issued from one host thread at a time and, when they share the
 *    context's scratch space, in one stream order (use one context per
 *    concurrently used stream).
 *  - Return value: NPG_OK (0) or a negative code.  Argument errors (null
 *    pointers, sizes out of range) are detected on the host before anything
 *    is enqueued.  Data-dependent errors (a direction that is not finite, a
 *    position outside the unit box, a leaf id >= L, a uniform outside [0,1))
 *    are raised by the kernels into a device error word; the offending
 *    outputs are written as documented per call, and npg_sync_status reports
 *    and clears the word.  npg_last_error returns a message for the last
 *    failing call.
 *  - Map sizes H (rows, z) and W (columns, azimuth) are powers of two in
 *    [4, 1024].  Per-leaf maps are stored row-major [leaf][z row][phi column].
 */
#ifndef NPG_H
#define NPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NPG_OK 0
#define NPG_E_ARG -1      /* invalid argument (null pointer, bad size, bad model)   */
#define NPG_E_RANGE -2    /* data-dependent input out of range (see each call)      */
#define NPG_E_CAPACITY -3 /* more leaves than the caller's capacity                 */
#define NPG_E_BUDGET -4   /* scratch space would exceed the context's HBM budget    */
#define NPG_E_HIP -5      /* a HIP runtime call failed                              */

typedef struct npg_ctx npg_ctx;
typedef struct npg_model npg_model;

/* Arithmetic of the network's convolutions.  Inputs, normalisation, the
 * per-leaf totals and the CDF prefixes are FP64/FP32 in every mode. */
typedef enum {
  NPG_FP32 = 0, /* FP32 weights; FP64 activations and accumulation        */
  NPG_BF16 = 1, /* BF16 activations and weights, FP32 accumulation          */
  NPG_FP8 = 2   /* FP8 e4m3 (OCP) with static per-layer scales, FP32 accum.  */
} npg_precision;

/* Device pointers of a batch of per-leaf CDF tables (as written by
 * npg_build_cdf).  pdf [L][H][W] (1/sr), marg [L][H+1], cond [L][H][W+1],
 * total [L] (FP64 sum of the density, may be NULL for sampling). */
typedef struct {
  const float *pdf_dev;
  const float *marg_dev;
  const float *cond_dev;
  const double *total_dev;
  uint32_t L;
  int32_t H;
  int32_t W;
} npg_tables;

/* Octree parameters (Sec. 7.1 "Voxel subdivision": split a voxel while its
 * photon count exceeds a threshold, recursively, with a depth cap). */
typedef struct {
  uint32_t split_count; /* a cell splits iff its count > split_count ...      */
  int32_t max_depth;    /* ... and its depth < max_depth; 0 <= max_depth <= 8  */
} npg_hier_params;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`.  hbm_budget_bytes bounds the
 * scratch space and model weights the library itself allocates on that
 * device (0 = no bound).  *out is set on success. */
int npg_create(npg_ctx **out, int device, uint64_t hbm_budget_bytes);

/* Waits for nothing; frees the context's scratch space.  The caller must
 * have synchronised every stream it used with the context. */
void npg_destroy(npg_ctx *ctx);

/* Message of the last failing call on ctx ("" if none).  Valid until the
 * next call on ctx. */
const char *npg_last_error(const npg_ctx *ctx);

/* Synchronises `stream`, then returns NPG_E_RANGE if any kernel launched
 * with ctx flagged a data-dependent error since the previous check (and
 * clears the flag), NPG_E_HIP if the stream reports a fault, else NPG_OK. */
int npg_sync_status(npg_ctx *ctx, void *stream);

/* Bytes of device memory the library currently holds for ctx (scratch) and
 * the high-water mark. */
void npg_memory_usage(const npg_ctx *ctx, uint64_t *current, uint64_t *peak);

/* FLOPs of the network convolutions launched with ctx since the last reset,
 * as each layer was launched (2 per multiply-add; host-side count):
 * *matrix those issued on the matrix cores (a nearest-upsampled input taken
 * in the phase-merged form counts 4 taps per upsampled channel instead of
 * 9), *vector those of the first layers, 1x1 heads and direct convolutions
 * on the vector ALUs (a first layer recomputed inside the next layer's patch
 * staging counts every patch pixel).  reset != 0 zeroes the counts after
 * reading them.  Either pointer may be NULL. */
void npg_conv_flops(npg_ctx *ctx, double *matrix, double *vector, int reset);

/* Context tunables (value >= 0):
 *   "graphs"       1: npg_reconstruct_fused captures its launches into a HIP
 *                  graph on the second call with the same arguments on a
 *                  non-default stream and replays it afterwards (default 0)
 *   "chunk_leaves" leaves per network chunk (and at most per gather batch
 *                  of npg_reconstruct_experts); 0 = autotuned or 1024
 *   "force_direct" 1: direct convolutions only (testing; default 0)
 *   "fuse_first"   0: store the first layer's activations instead of
 *                  computing them inside the second layer's input staging
 *                  (default 1; the results are identical)
 *   "pool_outputs" 0: each U-Net encoder level pools the level above's
 *                  stored output while staging it, instead of reading the
 *                  2x2 means that level stored beside its output (default
 *                  1; the results are identical)
 *   "upsample_taps9" 1: FP32-mode decoder convolutions take all nine taps on
 *                  their nearest-upsampled channels instead of four
 *                  phase-merged taps per output phase (testing; default 0;
 *                  the results agree to rounding)
 *   "tile_cap"     largest matrix-core tile, in units of 64 output pixels:
 *                  1, 2, 4 or 8 (a value in between rounds down; default 4;
 *                  a tuned table caps each layer further; testing: every
 *                  tile shape gives identical results)
 * NPG_E_ARG for an unknown name or a negative value. */
int npg_set_option(npg_ctx *ctx, const char *name, int64_t value);

/* ------------------------------------------------------------------ model */

/* Loads a network from an NPGW v1 weight file held in host memory:
 *   'NPGW' | u32 version = 1 | u32 arch | u32 levels | u32 n_layers |
 *   per layer: u32 cout, u32 cin, u32 k, f32 w[cout][cin][k][k], f32 b[cout]
 * (little endian).  arch 1 = chain of 3x3 convolutions, ReLU between them,
 * softplus after the last, 1 input and 1 output channel.  arch 2 = U-Net
 * with `levels` resolution levels: encoder level d = two 3x3 conv + ReLU on
 * the 2x2-average-pooled output of level d-1; decoder level d = two 3x3
 * conv + ReLU on [nearest x2 upsample of level d+1, skip of level d];
 * head = 1x1 conv to one channel + softplus (the compact U-Net of Sec. 6.1,
 * whose published figure and weights are not available, so the file's
 * weights are stand-ins).  arch 3 = the paper-style U-Net of Sec. 6.1 on the
 * five input channels: ELU after every 3x3 conv; encoder level d: a =
 * ELU(conv(x)), o = ELU(conv(a)) + a (the first conv being the masked
 * five-channel layer); the deepest level: a = ELU(conv(x)), b =
 * ELU(conv_dilation2(a)) + a, o = ELU(conv_dilation4(b)) + b; decoder level
 * d: a = ELU(conv([up(o), skip_d])), o = ELU(conv(a)) + a; head as arch 2;
 * 4 * levels layers.  Zero padding.  The host buffer is not retained.
 * Weights are repacked on the device for FP32 and BF16; FP8 needs
 * npg_model_calibrate_fp8 first.  NPG_E_ARG for a malformed file. */
int npg_model_load(npg_ctx *ctx, const void *host_bytes, size_t n_bytes, npg_model **out);
void npg_model_free(npg_model *model);

/* Sets the static FP8 (OCP e4m3) scales of a model from a calibration batch
 * of L energy maps [L][H][W] (device): the network runs once in NPG_FP32 and
 * records the largest stored output of every ReLU layer; that layer's
 * activations are then stored as e4m3 in units of amax/448.  Each 3x3
 * weight tensor fed by stored activations gets its input channels' units
 * folded in and one scale per output channel (amax/448 of the folded
 * weights); the first layer and the 1x1 head keep float32 weights.  Values
 * above the calibrated range saturate at +-448 units.  Synchronises
 * `stream`; may be called again to recalibrate.  Scales stay fixed between
 * calibrations, so a leaf's FP8 result does not depend on the other leaves
 * of a batch.  NPG_E_ARG for an empty batch or a map size the model does
 * not fit. */
int npg_model_calibrate_fp8(npg_ctx *ctx, npg_model *model, const uint64_t *energy_dev,
                            uint32_t L, int H, int W, void *stream);

/* The paper's hierarchical grid (Sec. 7.1; Sec. 8, path-guiding details): a
 * regular grid of res^3 voxels over the box [lo, hi], each valid voxel split
 * into a local binary KD tree. */
typedef struct {
  int32_t res;         /* voxels per axis (the paper: 100), 1..1024            */
  float lo[3], hi[3];  /* scene box, hi > lo per axis                          */
  double split_count;  /* a node splits if its photon count > split_count ...  */
  double split_var;    /* ... or its normal variance > split_var (the paper:
                          500 * sqrt(2^t) at iteration t, and 0.5) ...         */
  int32_t max_depth;   /* ... while its depth < max_depth (the paper: 8), 0..16 */
} npg_kdgrid_params;

/* One node of the local KD trees.  info & 3 = split axis (0, 1, 2) with the
 * children at nodes (info >> 2) and (info >> 2) + 1, points with coordinate
 * < split going to the first; info & 3 == 3: a leaf, leaf id = info >> 2. */
typedef struct {
  float split;
  uint32_t info;
} npg_kd_node;

/* ------------------------------------------------------------- hot path */

/* Assigns photons to the leaves of an adaptive octree over the unit box
 * (Sec. 7.1 "Voxel subdivision"; Algorithm 1, subdivision step).  The root
 * [0,1)^3 has depth 0; a cell splits into its 8 midpoint octants iff its
 * photon count > split_count and its depth < max_depth.  Leaves are the
 * unsplit cells holding at least one photon, numbered in ascending Morton
 * order (x in the lowest bit of each bit triple).
 *   pos_dev        [n][3] float32 positions, each coordinate in [0, 1)
 *   perm_dev       [n] out: photon indices grouped by leaf; within a leaf in
 *                  input order (stable), so leaf l owns perm[off[l]..off[l+1])
 *   leaf_of_dev    [n] out: leaf id of each photon (input order); may be NULL
 *   leaf_off_dev   [max_leaves+1] out: CSR offsets into perm
 *   leaf_key_dev   [max_leaves] out: Morton code of the leaf cell's lowest
 *                  corner on the 2^21 lattice (63 bits); may be NULL
 *   leaf_depth_dev [max_leaves] out: depth of the leaf cell; may be NULL
 *   n_leaves_out   host out: number of leaves L
 * Synchronises `stream` (L is read back).  A position outside [0,1)^3 or
 * not finite returns NPG_E_RANGE (outputs unspecified).  L > max_leaves
 * returns NPG_E_CAPACITY with *n_leaves_out = L (nothing past max_leaves
 * is written).  n <= 2^32 - 1. */
int npg_build_hierarchy(npg_ctx *ctx, const float *pos_dev, uint64_t n, const npg_hier_params *params,
                        uint32_t *perm_dev, uint32_t *leaf_of_dev, uint32_t *leaf_off_dev,
                        uint64_t *leaf_key_dev, uint8_t *leaf_depth_dev, uint32_t max_leaves,
                        uint32_t *n_leaves_out, void *stream);

/* npg_build_hierarchy that also puts the photons' directions and weights
 * in leaf order (the photons of Eq. "photon" grouped by voxel, Sec. 7.1):
 * dir_sorted[i] = dir[perm[i]], w_sorted[i] = w[perm[i]], so that
 * npg_splat_histograms reads every leaf's photons as one contiguous run
 * (perm NULL, leaf_off as written here).  The directions and weights move
 * with the permutation through its sort, read and written in order, instead
 * of being gathered through perm afterwards.
 *   dir_dev [n][3] float32, w_dev [n] uint32: the photons in input order
 *   dir_sorted_dev [n][3], w_sorted_dev [n]: out, leaf order (must not alias
 *   the inputs)
 * Every other argument, output and error as in npg_build_hierarchy (no
 * leaf_of output). */
int npg_build_hierarchy_sorted(npg_ctx *ctx, const float *pos_dev, const float *dir_dev, const uint32_t *w_dev,
                               uint64_t n, const npg_hier_params *params, uint32_t *perm_dev, float *dir_sorted_dev,
                               uint32_t *w_sorted_dev, uint32_t *leaf_off_dev, uint64_t *leaf_key_dev,
                               uint8_t *leaf_depth_dev, uint32_t max_leaves, uint32_t *n_leaves_out, void *stream);

/* Valid voxels (Sec. 7.1, detecting valid voxels; Algorithm 1, path step):
 * a voxel is valid iff at least one bounce point of the camera paths lies in
 * it.  The voxel of a point p is floor((p - lo) * (res / (hi - lo))) per axis,
 * in FP64 and clamped to [0, res-1]; voxel id = ix + res * (iy + res * iz).
 *   pts_dev    [n][3] float32 bounce points
 *   valid_dev  [res^3] out: 1 for valid voxels, 0 otherwise (overwritten)
 * A non-finite point returns NPG_E_RANGE (it marks nothing). */
int npg_mark_valid(npg_ctx *ctx, const npg_kdgrid_params *params, const float *pts_dev, uint64_t n,
                   uint8_t *valid_dev, void *stream);

/* Builds the paper's hierarchical grid over one iteration's photons
 * (Sec. 7.1 "Voxel subdivision"; Algorithm 1, subdivision step; Sec. 8
 * parameters).  Photons in invalid voxels are dropped.  A node (a valid
 * voxel holding photons, depth 0, or a sub-voxel) with M photons splits iff
 * depth < max_depth, M >= 2 and (M > split_count or V > split_var), where V
 * = 1 - |mean normal|^2 over its photons, from integer sums of the normals
 * quantised as rint(clamp(n, -1, 1) * 2^20) and evaluated in FP64 as
 * 1 - ((Sx*Sx + Sy*Sy) + Sz*Sz) / ((M*M) * 2^40) (no normals: V = 0).  The
 * split axis is the longest of the node's box (ties: lower axis; a voxel's
 * box is [lo + i*step, lo + (i+1)*step], step = (hi - lo) / res in FP64, cut
 * at each split); the split coordinate s is the (M/2)-th smallest (0-based)
 * photon coordinate on that axis (-0 read as +0); photons with coordinate
 * < s go to the first child.  A node with no photon below s stays a leaf.
 * Leaves are numbered voxel by voxel in ascending voxel id, depth first
 * with the first child first.
 *   pos_dev       [n][3] float32 photon positions
 *   normal_dev    [n][3] float32 unit surface normals at the hit points, or
 *                 NULL (the variance criterion is then off)
 *   valid_dev     [res^3] voxel validity (npg_mark_valid), or NULL (all valid)
 *   perm_dev      [n] out: photon indices grouped by leaf, ascending within a
 *                 leaf; leaf l owns perm[off[l]..off[l+1]), off[L] = number of
 *                 photons in valid voxels (the rest of perm is unspecified)
 *   leaf_off_dev  [max_leaves+1] out: CSR offsets into perm
 *   cell_root_dev [res^3] out: root node of each voxel, -1 for voxels that
 *                 are invalid or hold no photon
 *   nodes_dev     [2*max_leaves] out: the trees (npg_kd_node), the voxels'
 *                 roots first in ascending voxel id, then level by level
 *   n_leaves_out, n_nodes_out  host out: L and the number of nodes
 * Synchronises `stream`.  A non-finite position, or a non-finite normal of a
 * photon in a valid voxel, returns NPG_E_RANGE; more than max_leaves leaves
 * NPG_E_CAPACITY (outputs
 * unspecified, *n_leaves_out = 0).  n <= 2^32 - 1, max_leaves < 2^29. */
int npg_build_kdgrid(npg_ctx *ctx, const npg_kdgrid_params *params, const float *pos_dev,
                     const float *normal_dev, uint64_t n, const uint8_t *valid_dev, uint32_t *perm_dev,
                     uint32_t *leaf_off_dev, int32_t *cell_root_dev, npg_kd_node *nodes_dev, uint32_t max_leaves,
                     uint32_t *n_leaves_out, uint32_t *n_nodes_out, void *stream);

/* Point location in the hierarchical grid (Sec. 8: the voxel in O(1), then
 * O(depth) down its local tree): the leaf containing each query point, or
 * 0xFFFFFFFF in voxels without a tree.  The voxel rule is that of
 * npg_mark_valid; a point with coordinate < split descends to the first
 * child (-0 read as +0).
 *   q_dev         [n][3] float32 query points
 *   cell_root_dev, nodes_dev, n_nodes: as written by npg_build_kdgrid
 *   leaf_dev      [n] out: leaf ids
 * A non-finite point, or a node index >= n_nodes met in the walk, gives
 * 0xFFFFFFFF and NPG_E_RANGE at the next npg_sync_status. */
int npg_locate(npg_ctx *ctx, const npg_kdgrid_params *params, const int32_t *cell_root_dev,
               const npg_kd_node *nodes_dev, uint32_t n_nodes, const float *q_dev, uint64_t n, uint32_t *leaf_dev,
               void *stream);

/* Bins photons into per-leaf energy and count maps (Eq. "photon": the
 * energy of bin k of voxel j is the sum of the energies of the voxel's
 * photons whose direction falls in bin k; plus the photon count per bin,
 * an input channel of Sec. 6).  Direction -> bin is the exact equal-area
 * rule: row iz = #{b in 1..H-1 : z >= -1 + 2b/H}; column = azimuth sector
 * bounded by the rays e_b = Rot90^q(RN32(cos t), RN32(sin t)),
 * t = 2 pi r / W, b = q W/4 + r, tested with exact FP64 cross products
 * (x = y = 0 -> column 0).  Directions need not be normalised.
 *   dir_dev      [N][3] float32 directions;  w_dev [N] uint32 photon energy
 *                in fixed point (units of 2^-16; any value)
 *   perm_dev     NULL: leaf l owns photons leaf_off[l]..leaf_off[l+1]-1;
 *                else it owns photons perm[leaf_off[l]..leaf_off[l+1]-1]
 *   leaf_off_dev [L+1] CSR offsets (non-decreasing)
 *   energy_dev   [L][H][W] uint64 out (exact integer sums)
 *   count_dev    [L][H][W] uint32 out, or NULL
 *   accumulate   0: overwrite the maps; 1: add to them (progressive
 *                accumulation over iterations, Sec. 5)
 * Integer sums make the result independent of photon order and chunking.
 * A non-finite direction flags NPG_E_RANGE and the photon is skipped. */
int npg_splat_histograms(npg_ctx *ctx, const float *dir_dev, const uint32_t *w_dev,
                         const uint32_t *perm_dev, const uint32_t *leaf_off_dev, uint32_t L,
                         int H, int W, uint64_t *energy_dev, uint32_t *count_dev, int accumulate,
                         void *stream);

/* Raw sampling map fed to the network (Sec. 7.2: the accumulated energy
 * map is normalised): x = H*W*E / sum(E) computed in FP64 and stored as
 * float32 (mean 1); an all-zero leaf gives a zero map.
 *   energy_dev [L][H][W] uint64;  x_dev [L][H][W] float32 out. */
int npg_normalize_input(npg_ctx *ctx, const uint64_t *energy_dev, uint32_t L, int H, int W,
                        float *x_dev, void *stream);

/* Reconstructs the sampling density of every leaf with the network
 * (Sec. 6: S_d = F(S_e); the raw map S_e is the normalised energy map of
 * npg_normalize_input, computed on the fly: kept in binary64 in NPG_FP32
 * mode, rounded to float32 as npg_normalize_input stores it otherwise).
 *   energy_dev  [L][H][W] uint64;  count_dev: reserved for the count input
 *               channels of the paper's five-channel network, may be NULL
 *   density_dev [L][H][W] float32 out, softplus output (>= 0)
 * A U-Net needs H and W divisible by 2^(levels-1).  Leaves are processed
 * in chunks that fit the context's budget; NPG_E_BUDGET if not even one
 * leaf fits.  NPG_E_ARG for NPG_FP8 on an uncalibrated model. */
int npg_reconstruct_density(npg_ctx *ctx, const npg_model *model, const uint64_t *energy_dev,
                            const uint32_t *count_dev, uint32_t L, int H, int W,
                            npg_precision precision, float *density_dev, void *stream);

/* npg_reconstruct_density without allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same network, arguments, outputs and
 * errors as npg_reconstruct_density (one-channel models), but its
 * activations and per-leaf totals live in a static device array of the
 * library (256 MiB, of which 255 MiB are used; each GPU the library runs on
 * holds its own copy until the process ends), and the call allocates
 * nothing.  The leaves run in chunks that fit the array (the tuned or
 * "chunk_leaves" chunk, made smaller where needed), so L is unbounded;
 * results equal npg_reconstruct_density's bit for bit.  A map size whose
 * single leaf does not fit the array returns NPG_E_BUDGET.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different contexts of that GPU) race and must
 * be serialised by the caller. */
int npg_reconstruct_density_noalloc(npg_ctx *ctx, const npg_model *model, const uint64_t *energy_dev,
                                    uint32_t L, int H, int W, npg_precision precision, float *density_dev,
                                    void *stream);

/* The network on the paper's five input channels (Sec. 6): the raw maps
 * of iterations t and t-1 (x = H*W*E/sum(E), 0 for an empty map), their
 * photon-count maps normalised the same way (each value rounded to
 * float32), and the mask B of bins holding photons at t; the first layer is
 * a masked (partial) convolution: only taps with B = 1 contribute, the sum
 * is rescaled by 9/S for the S valid in-map taps (0 where S = 0), then bias
 * and the activation; the rest is the U-Net of npg_reconstruct_density
 * (arch 2 with a 5-channel first layer, ReLU) or the paper-style U-Net
 * (arch 3, ELU).  Other entry points reject five-channel models and this
 * one rejects the others.
 *   energy_dev, energy_prev_dev [L][H][W] uint64;  count_dev, count_prev_dev
 *   [L][H][W] uint32 (as written by npg_splat_histograms for iterations t
 *   and t-1);  density_dev [L][H][W] float32 out
 * NPG_FP32 or NPG_BF16 (NPG_E_ARG for NPG_FP8). */
int npg_reconstruct_density5(npg_ctx *ctx, const npg_model *model, const uint64_t *energy_dev,
                             const uint32_t *count_dev, const uint64_t *energy_prev_dev,
                             const uint32_t *count_prev_dev, uint32_t L, int H, int W, npg_precision precision,
                             float *density_dev, void *stream);

/* Mixture of experts by leaf photon count (Sec. 8, Implementation, training: five
 * networks, each for one range of photons per voxel, [0,100), [100,500),
 * [500,1000), [1000,5000) and [5000,inf)).  Leaf l holds
 * n_l = leaf_off[l+1] - leaf_off[l] photons and goes to expert
 * e = #{k : bounds[k] <= n_l}; its density is that of
 * npg_reconstruct_density with models[e] (bit for bit: each expert's leaves
 * are gathered, in leaf order, into one batch run by the same kernels, and
 * the densities are scattered back).
 *   models       host array of n_experts model handles, 1 <= n_experts <= 8
 *                (the same precision must be usable with each: FP8 needs
 *                every model calibrated)
 *   bounds       host array of n_experts - 1 strictly increasing counts
 *   leaf_off_dev [L+1] uint32 leaf CSR offsets (as in npg_splat_histograms)
 *   energy_dev   [L][H][W] uint64;  density_dev [L][H][W] float32 out
 *   counts_out   host array of n_experts (leaves per expert) or NULL
 * Synchronises `stream` once (the leaves per expert size the launches) and
 * holds gather buffers for the call's duration (within the budget). */
int npg_reconstruct_experts(npg_ctx *ctx, const npg_model *const *models, int n_experts,
                            const uint32_t *bounds, const uint32_t *leaf_off_dev, const uint64_t *energy_dev,
                            uint32_t L, int H, int W, npg_precision precision, float *density_dev,
                            uint32_t *counts_out, void *stream);

/* The batched form of the path (Sec. 7.2, sampling map reconstruction: after
 * an iteration's photons are traced, every valid voxel that received new
 * photons gets its map reconstructed by the network, as one batch): splat ->
 * normalise -> network -> CDF for a
 * batch of leaves of uneven photon counts, processed in chunks whose energy
 * maps and densities live only in library scratch (the per-leaf maps of the
 * whole batch are never written).  Arguments as in npg_splat_histograms,
 * npg_reconstruct_density and npg_build_cdf; the results equal those of the
 * three calls in sequence (bit for bit: same kernels, same per-leaf order).
 * With the "graphs" option the launch sequence is captured once and
 * replayed on repeated calls with identical arguments. */
int npg_reconstruct_fused(npg_ctx *ctx, const npg_model *model, const float *dir_dev, const uint32_t *w_dev,
                          const uint32_t *perm_dev, const uint32_t *leaf_off_dev, uint32_t L, int H, int W,
                          npg_precision precision, float *pdf_dev, float *marg_dev, float *cond_dev,
                          double *total_dev, void *stream);

/* Autotuner: times each convolution of the network on `probe_leaves`
 * synthetic leaves of H x W under each pixel-tile size (64, 128, 256, 512 pixels
 * per workgroup) and then the leaf-chunk size, and keeps the fastest choices
 * in ctx for (model, precision, H, W); later reconstruct calls of that shape
 * use them (npg_reconstruct_density5 for a five-channel model, which tunes
 * in FP32 or BF16 only).  The choice never changes a result (every output
 * sums its terms in the same order).  Synchronises `stream`. */
int npg_autotune(npg_ctx *ctx, const npg_model *model, int H, int W, npg_precision precision,
                 uint32_t probe_leaves, void *stream);

/* The tuned table for (model, precision, H, W): out[0] = leaves per chunk,
 * out[1..] = tile cap (1, 2, 4 x 64 pixels) of each convolution call.
 * Returns the number of entries (0 if not tuned); writes at most capacity. */
int npg_tune_table(const npg_ctx *ctx, const npg_model *model, int H, int W, npg_precision precision,
                   int32_t *out, int capacity);

/* Sampling pdf and CDF tables of each leaf (Eq. "energy_target": the guide
 * pdf is proportional to the map value over the bin's solid angle; Sec. 7.3:
 * a CDF from a cumulative sum over pixels, sampled like an environment map).
 *   p_k = s_k / S, S = sum_k s_k in FP64;  pdf_k = p_k H W / (4 pi)  [1/sr]
 *   marg: M_0 = 0, M_i = sum_{i'<i} sum_j p_{i',j}, M_H = 1
 *   cond: C_{i,0} = 0, C_{i,j} = sum_{j'<j} p_{i,j'} / m_i, C_{i,W} = 1,
 *         a row with m_i = 0 gets C_{i,j} = j/W
 * Prefixes in FP64, stored as float32.
 *   density_dev [L][H][W] float32 (>= 0);  pdf_dev [L][H][W] out;
 *   marg_dev [L][H+1] out;  cond_dev [L][H][W+1] out;  total_dev [L] out
 *   (FP64 S; may be NULL)
 * A leaf whose density has a negative or non-finite value or sums to zero
 * flags NPG_E_RANGE; its tables are written as NaN and its total as 0. */
int npg_build_cdf(npg_ctx *ctx, const float *density_dev, uint32_t L, int H, int W, float *pdf_dev,
                  float *marg_dev, float *cond_dev, double *total_dev, void *stream);

/* Guided direction sampling (Algorithm 1, guided-sampling step): for query
 * q with leaf l and uniforms (u1, u2) in [0,1):
 *   row i = max{i in [0,H-1] : M_i <= u1}, column j = max{j : C_{i,j} <= u2},
 *   t1 = (u1 - M_i)/(M_{i+1} - M_i), t2 likewise (clamped to [0,1)),
 *   z = -1 + 2(i + t1)/H, phi = 2 pi (j + t2)/W,
 *   dir = (sqrt(1-z^2) cos phi, sqrt(1-z^2) sin phi, z), pdf = pdf[l][i][j].
 *   leaf_dev [n] uint32;  u_dev [n][2] float32
 *   dir_out_dev [n][3] float32 out;  pdf_out_dev [n] float32 out;
 *   bin_out_dev [n] uint32 out (i*W + j) or NULL
 * leaf >= L or a uniform outside [0,1) flags NPG_E_RANGE; that query's
 * direction and pdf are NaN and its bin 0xffffffff. */
int npg_sample_dirs(npg_ctx *ctx, const npg_tables *tables, const uint32_t *leaf_dev,
                    const float *u_dev, uint64_t n, float *dir_out_dev, float *pdf_out_dev,
                    uint32_t *bin_out_dev, void *stream);

/* pdf of directions under their leaf's map: pdf[l][bin(dir)], with the bin
 * rule of npg_splat_histograms (the guide term of the one-sample MIS pdf,
 * Eq. "mis_coef").
 *   leaf_dev [n];  dir_dev [n][3] float32;  pdf_out_dev [n] float32 out
 * leaf >= L or a non-finite direction flags NPG_E_RANGE; pdf 0 there. */
int npg_eval_pdf(npg_ctx *ctx, const npg_tables *tables, const uint32_t *leaf_dev,
                 const float *dir_dev, uint64_t n, float *pdf_out_dev, void *stream);

/* One-sample MIS of BSDF sampling and guiding (Sec. 7.3, Eq. "mis_alpha"
 * and Eq. "mis_coef").  Per leaf j, from the path statistics of its bounces:
 * nu_B, nu_G = summed contributions of bounces whose direction came from
 * BSDF / guided sampling, Q_B, Q_G = their numbers:
 *   alpha_j = (nu_B/Q_B) / (nu_B/Q_B + nu_G/Q_G) once Q_B >= 50 and
 *   Q_G >= 50 (0.5 before, and 0.5 if both averages are 0), clamped to
 *   [0.2, 0.8]; computed in FP64, stored as float32.
 *   nu_b_dev, nu_g_dev [L] float32 (>= 0);  q_b_dev, q_g_dev [L] uint32
 *   alpha_dev [L] float32 out
 * A negative or non-finite contribution flags NPG_E_RANGE and gives 0.5. */
int npg_mis_alpha(npg_ctx *ctx, const float *nu_b_dev, const float *nu_g_dev, const uint32_t *q_b_dev,
                  const uint32_t *q_g_dev, uint32_t L, float *alpha_dev, void *stream);

/* One-sample MIS sampling with a cosine-lobe BSDF about a per-query normal
 * (the stand-in BSDF, p_BSDF(w) = max(0, n.w)/pi):
 *   u = (u0, u1, u2) in [0,1)^3;  a = alpha[l]
 *   u0 < a: BSDF sample, r = sqrt(u1), phi = 2 pi u2,
 *           w = r cos(phi) t + r sin(phi) b + sqrt(1 - u1) n with the
 *           orthonormal frame (t, b, n) of Duff et al. 2017 (JCGT 6(1));
 *   else:   the guided sample of npg_sample_dirs from (u1, u2);
 *   pdf = a p_BSDF(w) + (1 - a) p_guide(w), p_guide = pdf[l][bin] with the
 *   sampled bin for guided samples and the bin rule of npg_splat_histograms
 *   for BSDF samples.
 *   alpha_dev [L];  leaf_dev [n];  normal_dev [n][3] (unit);  u_dev [n][3]
 *   dir_out_dev [n][3] out;  pdf_out_dev [n] out;  strategy_out_dev [n]
 *   uint8 out (1 = BSDF, 0 = guided) or NULL
 * leaf >= L, a uniform outside [0,1) or a non-finite normal flags
 * NPG_E_RANGE; that query's direction and pdf are NaN. */
int npg_sample_mis(npg_ctx *ctx, const npg_tables *tables, const float *alpha_dev, const uint32_t *leaf_dev,
                   const float *normal_dev, const float *u_dev, uint64_t n, float *dir_out_dev,
                   float *pdf_out_dev, uint8_t *strategy_out_dev, void *stream);

/* The one-sample MIS pdf of directions (Eq. "mis_coef" with the cosine-lobe
 * BSDF): a p_BSDF(w) + (1 - a) pdf[l][bin(w)], a = alpha[l].
 *   alpha_dev [L];  leaf_dev [n];  normal_dev [n][3];  dir_dev [n][3]
 *   pdf_out_dev [n] out
 * leaf >= L or a non-finite direction or normal flags NPG_E_RANGE; pdf 0
 * there. */
int npg_eval_pdf_mis(npg_ctx *ctx, const npg_tables *tables, const float *alpha_dev, const uint32_t *leaf_dev,
                     const float *normal_dev, const float *dir_dev, uint64_t n, float *pdf_out_dev,
                     void *stream);

/* ---------------------------------------------------------------- serving */

/* A server takes reconstruction and sampling requests as a render loop emits
 * them (Algorithm 1 and Sec. 7: each iteration traces photons, reconstructs
 * the maps of the voxels they reached, then guides the iteration's paths by
 * sampling those maps, Sec. 7.3) and runs them with continuous batching: a
 * scheduler thread owns
 * n_slots device streams; whenever one is free it launches the oldest
 * waiting request, merged with every later waiting reconstruction of the
 * same map size (up to max_batch_leaves leaves, as long as their tables fit
 * in the table arena) into one batch whose kernels process the leaves of
 * all its requests together.  Requests admitted while others run overlap on
 * the device.  Reconstruction tables stay resident in the arena until the
 * request is released.  A request's results do not depend on the batch it
 * ran in.  All pointers stay owned by the caller and must stay valid until
 * the request completes. */
typedef struct npg_server npg_server;

typedef struct {
  uint32_t n_slots;            /* concurrent batches (streams), 1..16                      */
  uint32_t max_batch_leaves;   /* leaves merged into one batch; 0 = one request per batch  */
  uint64_t table_bytes;        /* device arena for resident tables (charged to ctx)        */
  uint64_t slot_scratch_bytes; /* scratch budget of each slot (0 = unbounded)              */
  npg_precision precision;     /* network precision (FP8: model calibrated beforehand)     */
} npg_serve_params;

typedef struct {
  uint64_t submitted, completed, batches, leaves, merged_requests, max_concurrent, queued;
  uint64_t table_bytes_free;
} npg_serve_stats;

/* Creates a server on ctx's device for `model` (which must outlive it). */
int npg_serve_create(npg_ctx *ctx, const npg_model *model, const npg_serve_params *params, npg_server **out);

/* Waits for work in flight, then frees everything the server holds. */
void npg_serve_destroy(npg_server *server);

/* Reconstruction request for L leaves of an H x W map.  Leaf l owns photons
 * leaf_begin_host[l] .. + leaf_count_host[l] - 1 of dir_dev / w_dev (host
 * arrays are copied).  Tables (pdf, marg, cond, total as in npg_build_cdf)
 * are allocated in the arena at admission.  NPG_E_BUDGET if they can never
 * fit in the arena.  *ticket identifies the request. */
int npg_serve_submit_recon(npg_server *server, const float *dir_dev, const uint32_t *w_dev,
                           const uint32_t *leaf_begin_host, const uint32_t *leaf_count_host, uint32_t L, int H,
                           int W, uint64_t *ticket);

/* Sampling request (as npg_sample_dirs, without bins) against the resident
 * tables of a reconstruction ticket; it runs after that reconstruction. */
int npg_serve_submit_sample(npg_server *server, uint64_t recon_ticket, const uint32_t *leaf_dev,
                            const float *u_dev, uint64_t n, float *dir_out_dev, float *pdf_out_dev,
                            uint64_t *ticket);

/* 1 = done (latency from submit to completion in microseconds), 0 = pending,
 * negative = failed or unknown ticket.  npg_serve_wait blocks until done. */
int npg_serve_poll(npg_server *server, uint64_t ticket, double *latency_us);
int npg_serve_wait(npg_server *server, uint64_t ticket, double *latency_us);

/* Device tables of a completed reconstruction request. */
int npg_serve_tables(npg_server *server, uint64_t recon_ticket, npg_tables *out);

/* Copies the tables of a completed reconstruction request into caller
 * buffers (layouts as in npg_build_cdf; total may be NULL), on `stream`. */
int npg_serve_copy_tables(npg_server *server, uint64_t recon_ticket, float *pdf_dev, float *marg_dev,
                          float *cond_dev, double *total_dev, void *stream);

/* Forgets a request: its ticket is unknown afterwards (poll and wait return
 * NPG_E_ARG), so read its latency first.  A reconstruction's tables return
 * to the arena once it has finished and no sampling request submitted
 * against it is still unfinished. */
int npg_serve_release(npg_server *server, uint64_t ticket);

/* Message of the server's most recent failure (a failed request, an unknown
 * ticket); "" if none.  The pointer stays valid until the calling thread's
 * next call of this function. */
const char *npg_serve_last_error(npg_server *server);

void npg_serve_get_stats(npg_server *server, npg_serve_stats *out);

/* The float32 boundary rays of a W-column map, (x, y) pairs for b = 0..W-1,
 * as the kernels use them (host memory out, 2*W floats). */
int npg_bin_boundaries(int W, float *xy_out);

#ifdef __cplusplus
}
#endif
#endif /* NPG_H */
