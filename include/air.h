/*
 * air.h -- C ABI of the MI355X (gfx950) adaptive image ray-tracing library.
 *
 * Method: Parkin 2010, "Adaptive image ray-tracing for astrophysical
 * simulations" (MNRAS Letter).  Section 2 defines the scheme: a coarse base
 * image (step i), one ray per pixel integrating a quantity through the
 * simulation grid (step ii), a scan of the image with a truncation-error test
 * and a 2:1 level rule between adjacent pixels (step iii), refinement with
 * tree book-keeping (step iv), repeated until nothing refines or a resolution
 * cap (step v), then integration and output (step vi).  Section 3 gives the
 * error estimate (Eq. 2 in 1-D, Eq. 3 in 2-D), the refinement threshold
 * xi >= xi_crit, and the flux definition used in Table 1.
 *
 * Conventions shared by every call:
 *  - All array arguments marked "device" are HIP device pointers owned by the
 *    caller; the library never frees or retains them after the call returns.
 *    Host pointers are marked "host".
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL = the
 *    null stream).  Calls that return host results (counts, flux, stats)
 *    synchronise that stream before returning.
 *  - Field arrays are float32, x fastest: index x + nx*(y + ny*z) on a uniform
 *    grid; block-major (block b's bs^3 cells from b*bs^3, x fastest inside)
 *    on a block-AMR grid.
 *  - Image pixel (L, i, j) of a view: level L, i along e_u, j along e_v,
 *    e_u = normalise(up x dir), e_v = dir x e_u; the level-L raster has
 *    R_L = coarse_n * 2^L pixels a side, pixel size width / R_L, and the
 *    pixel's ray passes through its centre along +dir (front to back from
 *    the observer).  Rasters are row-major: index j*R + i.
 *  - A context is not thread-safe: use one per host thread.
 *  - Every call returns an air_status; on failure, air_last_error() holds a
 *    message and the outputs are undefined.  No exception crosses the ABI.
 */
#ifndef AIR_H
#define AIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t air_status;
#define AIR_OK 0
#define AIR_EINVAL (-1)    /* bad argument, detected on the host before any launch */
#define AIR_ENOMEM (-2)    /* device allocation failed */
#define AIR_EDEVICE (-3)   /* a HIP call failed; air_last_error() has its text */
#define AIR_ECAPACITY (-4) /* an output buffer is too small: tree->n_nodes holds the size needed */
#define AIR_ENOTSUP (-5)   /* combination the library does not support */

#define AIR_MAX_LEVELS 12 /* image levels 0..11 */
#define AIR_MAX_BANDS 8
#define AIR_MAX_VIEWS 4096

/* grid kinds */
#define AIR_GRID_UNIFORM 0
#define AIR_GRID_BLOCK_AMR 1
/* field kinds */
#define AIR_FIELD_RHO_J_KAPPA 0 /* rho, emissivity j, opacity kappa: one band */
#define AIR_FIELD_RHO_T 1       /* rho, T; band b: kappa = k0_b rho T^-s_b, j = rho^2 T^q_b */

/* node state bits (air_tree.state) */
#define AIR_NODE_EXIST 1u
#define AIR_NODE_TESTED 2u    /* base pixel or child of a flagged pixel: eligible for the test */
#define AIR_NODE_FLAGGED 4u   /* the test asked for refinement (xi >= xi_crit) */
#define AIR_NODE_BALANCE 8u   /* created only to keep the 2:1 level rule; never tested */
#define AIR_NODE_REFINED 16u  /* has four children */
#define AIR_NODE_EVALUATED 32u /* the test was evaluated at this node */

/* Simulation grid (section 3 uses a block-structured AMR grid; the
 * uniform grid is the one-level special case). */
typedef struct {
  int32_t kind;     /* AIR_GRID_* */
  int32_t n[3];     /* uniform: cells per axis.  AMR: base blocks per axis */
  double lo[3];     /* box corner; the box is [lo, hi) with half-open cells */
  double hi[3];
  int32_t bs;        /* AMR: cells per block edge (power of two, 2..32) */
  int32_t max_level; /* AMR: deepest block level (ratio-2 refinement), 0..20 */
  int32_t n_blocks;  /* AMR: number of blocks; base blocks first, x fastest */
  const int32_t* block_level; /* device [n_blocks] */
  const int32_t* block_coord; /* device [n_blocks][3]: block coordinate at its own level */
  const int32_t* block_child; /* device [n_blocks]: first of 8 children (offset cx+2cy+4cz) or -1 */
} air_grid;
/* A call that takes a block-AMR grid reads the three tables back on its
 * stream (a blocking copy of 20 bytes per block) and returns EINVAL unless
 * they describe one hierarchy (below).  air_field_pack always checks them and
 * remembers, on its context, the tables it packed with: later calls on that
 * context that pass the same tables (pointers and sizes) with that packed
 * field skip the read-back.  Tables changed in place after packing must be
 * packed again (the packed layout follows them anyway).  The hierarchy:
 * base block b at level 0 with
 * coordinate (b % n0, b / n0 % n1, b / (n0 n1)); every other block the child
 * of exactly one earlier block; children stored consecutively after their
 * parent, one level deeper, at coordinate 2 * parent + offset bits; no
 * children at max_level; finest cells per axis (n * bs << max_level) and
 * total cells (n_blocks * bs^3) below 2^30. */

/* Cell data (device, float32). */
typedef struct {
  int32_t kind;    /* AIR_FIELD_* */
  int32_t n_bands; /* 1 for AIR_FIELD_RHO_J_KAPPA; 1..AIR_MAX_BANDS for AIR_FIELD_RHO_T */
  const float* rho;   /* density: the column N integrates it */
  const float* emis;  /* emissivity (RHO_J_KAPPA) */
  const float* kappa; /* opacity (RHO_J_KAPPA) */
  const float* temp;  /* temperature (RHO_T) */
  double band[AIR_MAX_BANDS][3]; /* host values (k0, s, q) per band (RHO_T) */
  const void* packed; /* device, may be NULL: the march layout written by air_field_pack for these
                         arrays; when NULL every call packs into context memory first */
} air_field;

/* Orthographic view (section 3 uses a face-on view along an axis). */
typedef struct {
  double dir[3];    /* looking direction (need not be unit length) */
  double up[3];     /* up hint; must not be parallel to dir */
  double center[3]; /* image centre in grid coordinates */
  double width;     /* image side length in grid units */
} air_view;

/* air_params.flags: time every march and test launch with HIP events
 * (air_stats.ms_march / ms_test; otherwise they are 0).  The events sit
 * between the kernels on the stream and lengthen the call a little. */
#define AIR_FLAG_TIMING 1u
/* air_params.flags: the images hold the super-resolved raster (section 2
 * step vi: interpolation across neighbouring pixels of different levels)
 * instead of the painted leaves: each pixel of the finest raster, inside a
 * level-L leaf, is the bilinear interpolation at its centre of the level-L
 * samples around it (a level-L node's value, or where none exists the value
 * of the level-(L-1) node covering the position; edges clamped).  Trees and
 * fluxes (sums over leaves) are unchanged. */
#define AIR_FLAG_SUPERRES 2u

/* Refinement parameters (sections 2 and 3). */
typedef struct {
  int32_t coarse_n;  /* N0: base image is N0 x N0 (step i) */
  int32_t max_level; /* number of refinements allowed (step v cap) */
  float xi_crit_I;   /* refine iff xi(I) >= xi_crit_I; > 1 disables (xi <= 1) */
  float xi_crit_N;   /* same for the column density N; several variables are OR-ed */
  float band_weight[AIR_MAX_BANDS]; /* the tested intensity is sum_b w_b I_b */
  uint32_t flags;    /* AIR_FLAG_* bits; others must be 0 */
} air_params;

/* Pixel quadtree in canonical order: by level, then coarse pixel (row-major),
 * then Morton order inside the coarse pixel, so the four children of a node
 * are consecutive.  All arrays are device memory of `capacity` entries
 * supplied by the caller; a NULL array is skipped. */
typedef struct {
  int64_t capacity;                     /* in: entries in each array below */
  int64_t n_nodes;                      /* out: nodes = rays traced */
  int64_t n_per_level[AIR_MAX_LEVELS];  /* out */
  int64_t n_leaves;                     /* out */
  int8_t* level;       /* device */
  int32_t* ix;         /* device: pixel index along e_u at its level */
  int32_t* iy;         /* device: pixel index along e_v */
  int32_t* parent;     /* device: node index of the parent, -1 at level 0 */
  int32_t* first_child;/* device: node index of the first of 4 children, or -1 */
  uint8_t* state;      /* device: AIR_NODE_* bits */
  float* I;            /* device [n_bands][capacity]: intensity per band */
  float* N;            /* device: column density */
  float* xi_I;         /* device: xi of the tested intensity, NaN if not evaluated */
  float* xi_N;         /* device: xi of N, NaN if not evaluated */
  int32_t* visits;     /* device: cells crossed by the node's ray */
} air_tree;

/* Counters of one call (host). */
typedef struct {
  int64_t rays;                          /* rays traced (all tree nodes) */
  int64_t rays_per_level[AIR_MAX_LEVELS];
  int64_t hits;                          /* rays that crossed the grid */
  int64_t visits;                        /* (ray, cell) segments marched */
  int64_t leaves;
  int64_t tested;                        /* nodes where the test was evaluated */
  int64_t flagged;
  int64_t balance;                       /* nodes created by the 2:1 rule */
  int32_t depth;                         /* deepest level reached */
  int32_t march_launches;                /* march kernel launches in the call */
  double ms_total;  /* device time of the call, first kernel to last (HIP events on the stream) */
  double ms_march;  /* with AIR_FLAG_TIMING: device time of the march kernels, summed over launches */
  double ms_test;   /* with AIR_FLAG_TIMING: device time of the test / 2:1 closure / compaction kernels */
} air_stats;

typedef struct air_ctx air_ctx;

/* Bytes of the march layout of a field, or a negative air_status for
 * invalid arguments. */
int64_t air_field_packed_bytes(const air_grid* grid, const air_field* field);

/*
 * Write the march layout of `field` into `packed` (device, `bytes` >=
 * air_field_packed_bytes): the cells are grouped in 2x2x2 bricks (brick
 * index x fastest over ceil(n/2) bricks per axis; cell inside the brick
 * x&1 | (y&1)<<1 | (z&1)<<2; on a block-AMR grid the same inside each
 * block, blocks in table order) and each cell's values are adjacent, 16 B
 * (rho, j, kappa, 1/kappa) for RHO_J_KAPPA and for one-band RHO_T (its j,
 * kappa and 1/kappa evaluated here, once, in float32 exactly as the march
 * would), or 8 B
 * (rho, T) for RHO_T with 2..8 bands, so one brick of a one-band field is one
 * 128-byte cache line and a visit is one load.  A one-band RHO_T field on a
 * uniform grid is followed, at the next multiple of 256 bytes, by the same
 * bricks as 8-byte (rho, T) records: the marches of levels whose rays lie at
 * least half a cell apart read those (two bricks per line), evaluating the
 * same optics, so either copy gives the same bits.  A block-AMR field is
 * followed, at the next multiple of 256 bytes, by the leaf block of every
 * position of the finest block lattice ((n[0] n[1] n[2]) << 3 max_level
 * uint32 entries, x fastest, each leaf id << 4 | its level; none when that
 * lattice has more than 2^26 positions or max_level > 15), so the march
 * locates a block with one load instead of a descent of the child table.
 * Pass the buffer as field->packed to later calls; it holds a copy, so it
 * must be packed again after the arrays change.  Errors: EINVAL (sizes,
 * NULL pointers, block tables), ENOTSUP (either copy >= 4 GiB).
 */
air_status air_field_pack(air_ctx* ctx, const air_grid* grid, const air_field* field, void* packed,
                          int64_t bytes, void* stream);

/* Create a context on HIP device `device`.  The context owns device
 * workspace (per-level pixel maps, work queue, counters) that grows on demand
 * and is freed by air_destroy. */
air_status air_create(air_ctx** out, int32_t device);
void air_destroy(air_ctx* ctx);
/* Message for the last failure on this context ("" if none). */
const char* air_last_error(const air_ctx* ctx);

/* The launch shapes air_render_batch tuned on this context (one entry per
 * workload shape: grid, views, coarse size, levels, bands; results never
 * depend on them, only time does), kept across processes.
 * air_tune_save writes them to a text file at path: a header line naming the
 * device's architecture and compute-unit count, then one line per shape.
 * air_tune_load reads such a file into the context (entries of the same
 * shape are replaced) so that later batches skip their tuning runs; it
 * rejects the whole file, taking nothing, if the header names another
 * device type or any entry is malformed.  Host file I/O only.
 * Errors: EINVAL (NULL path, unreadable or unwritable file, bad contents,
 * other device type; the reason in air_last_error), EDEVICE. */
air_status air_tune_save(air_ctx* ctx, const char* path);
air_status air_tune_load(air_ctx* ctx, const char* path);

/* Library-owned tree buffers (the air_tree arrays, any render's output):
 * air_tree_alloc allocates every array of *tree on the context's device for
 * `capacity` nodes and n_bands bands (1..AIR_MAX_BANDS) and sets
 * tree->capacity; air_tree_free frees the arrays of a tree made by
 * air_tree_alloc (never caller-allocated arrays) and zeroes the struct.
 * The caller owns the result until it calls air_tree_free; destroying the
 * context does not free it.  Errors: EINVAL (NULL tree, capacity outside
 * 1..2^31-1, n_bands out of range), ENOMEM (nothing stays allocated),
 * EDEVICE. */
air_status air_tree_alloc(air_ctx* ctx, int32_t n_bands, int64_t capacity, air_tree* tree);
air_status air_tree_free(air_ctx* ctx, air_tree* tree);

/*
 * Plain AIR for n_views views of one grid (section 2 steps i-vi), the views
 * refined level by level in lockstep.  For each view:
 *  - every base pixel is traced and tested;
 *  - at level L < max_level every tested node's xi is computed from its 3x3
 *    level-L neighbourhood (a missing neighbour takes the value of the
 *    covering level-(L-1) node; a direction without both neighbours inside
 *    the image is dropped with the mixed terms);
 *  - flagged nodes get 4 tested children, and the 2:1 rule (edge and corner
 *    neighbours) is closed by refining coarser nodes, whose children are
 *    balance nodes;
 *  - all new nodes are traced before the next level.
 * Outputs (each may be NULL):
 *  trees   host array [n_views] of air_tree with caller device buffers;
 *  images  device [n_views][n_bands + 1][R][R], R = coarse_n * 2^max_level:
 *          the leaves painted over their squares, bands then N;
 *  flux    host [n_views][n_bands]: sum over leaves of pixel area x I_b,
 *          reduced in double precision in a fixed order;
 *  stats   host, summed over views.
 * Errors: EINVAL (checked before any launch), ECAPACITY (a tree's capacity
 * is below its node count; n_nodes holds the count), EDEVICE, ENOMEM.
 */
air_status air_render(air_ctx* ctx, const air_grid* grid, const air_field* field, const air_view* views,
                      int32_t n_views, const air_params* params, air_tree* trees, float* images,
                      double* flux, air_stats* stats, void* stream);

/*
 * air_render for many views and bands in one captured launch sequence: the
 * first call for a workload shape times the level loop under a few launch
 * shapes (march waves per CU, test blocks per CU; results do not depend on
 * them) and keeps the fastest; the whole device sequence of the call (level
 * loop, canonical tree, raster, flux) is captured once into a HIP graph and
 * replayed while every launch argument stays the same (same buffers and
 * sizes; the views' contents may change).  Arguments, outputs and errors as
 * air_render, bit for bit equal to it; AIR_FLAG_TIMING is ignored.
 */
air_status air_render_batch(air_ctx* ctx, const air_grid* grid, const air_field* field, const air_view* views,
                            int32_t n_views, const air_params* params, air_tree* trees, float* images,
                            double* flux, air_stats* stats, void* stream);

/*
 * Fixed-resolution baseline (section 3, Table 1 "Fixed"): every pixel of the
 * level-`level` raster of each view is traced.  images: device
 * [n_views][n_bands + 1][R][R] with R = coarse_n * 2^level (NULL skips the
 * write, the rays are still traced); flux: host [n_views][n_bands] or NULL.
 */
air_status air_render_fixed(air_ctx* ctx, const air_grid* grid, const air_field* field,
                            const air_view* views, int32_t n_views, int32_t coarse_n, int32_t level,
                            float* images, double* flux, air_stats* stats, void* stream);

/*
 * air_render_fixed for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same rays, kernels and results, with its workspace (counters, view
 * table, flux partial sums) in a static device array of
 * AIR_NOALLOC_SCRATCH_BYTES that the library holds on each GPU until the
 * process ends.  It calls no allocation, no memset and no synchronisation, so
 * it can be captured; it returns once the work is enqueued on `stream`.
 *  images: device [n_views][n_bands + 1][R][R], R = coarse_n * 2^level;
 *  flux:   DEVICE [n_views][n_bands] float64, may be NULL (needs images).
 * Limits (EINVAL beyond them): n_views <= AIR_NOALLOC_MAX_VIEWS; with flux,
 * n_views * n_bands * ceil(R^2 / 4096) * 8 bytes <= AIR_NOALLOC_SCRATCH_BYTES
 * - 4096 (e.g. 16 views x 8 bands at R = 2048); field->packed must be set
 * (air_field_pack), and a block-AMR grid's tables must have been checked by
 * air_field_pack on this context for that packed field (nothing is read back).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other contexts, other threads) race; order them on one
 * stream.  Errors: EINVAL, ENOTSUP, EDEVICE.
 */
#define AIR_NOALLOC_MAX_VIEWS 16
#define AIR_NOALLOC_SCRATCH_BYTES (2u << 20)
air_status air_render_fixed_noalloc(air_ctx* ctx, const air_grid* grid, const air_field* field,
                                    const air_view* views, int32_t n_views, int32_t coarse_n, int32_t level,
                                    float* images, double* flux, void* stream);

/*
 * Trace n individual pixels of one view (section 2 step ii), e.g. to sample
 * a large image.  level/ix/iy: device [n]; I: device [n_bands][n]; N, visits
 * (nullable): device [n].
 */
air_status air_trace_pixels(air_ctx* ctx, const air_grid* grid, const air_field* field,
                            const air_view* view, int32_t coarse_n, int64_t n, const int32_t* level,
                            const int32_t* ix, const int32_t* iy, float* I, float* N, int32_t* visits,
                            void* stream);

/* ------------------------------------------------------------------------
 * Per-pixel spectra (section 2 step vi: integrated quantities such as
 * broadband images; an integrated spectrum needs every pixel's spectrum until
 * the image is final).  A spectrum is n_bins energy bins of a (rho, T) field:
 *   kappa_b = k0_b rho T^-s_b,   j_b = e0_b rho^2 T^q_b exp(-E_b / T)
 * (T > 0), each integrated along the ray like a band.  The image is refined
 * on the broadband sum_b weight_b I_b.
 * ---------------------------------------------------------------------- */
#define AIR_MAX_BINS 1024
typedef struct {
  int32_t n_bins;       /* 1..AIR_MAX_BINS */
  const double* bins;   /* host [n_bins][5]: k0, s, e0, q, E */
  const float* weight;  /* host [n_bins]: broadband weights (>= 0) */
} air_spectrum;

/*
 * Plain AIR of n_views views on the broadband of `spectrum` (uniform grid,
 * field kind AIR_FIELD_RHO_T; its n_bands and band table are not used):
 * arguments and tree outputs as air_render, with the trees' I holding the one
 * band sum_b weight_b I_b (params.band_weight is not used) and:
 *  spectra  device [sum_k trees[k].capacity][n_bins] or NULL: every node's
 *           spectrum, view k's nodes from row sum_{k' < k} trees[k'].capacity,
 *           in the trees' canonical order;
 *  images   device [n_views][2][R][R]: broadband and column of the leaves;
 *  flux     host [n_views][n_bins] or NULL: the image's spectrum, sum over
 *           leaves of pixel area x I_b (float64, fixed order).
 * trees is required.  Errors as air_render; ENOTSUP for block-AMR grids or
 * AIR_FLAG_SUPERRES.
 */
air_status air_render_spectra(air_ctx* ctx, const air_grid* grid, const air_field* field, const air_view* views,
                              int32_t n_views, const air_params* params, const air_spectrum* spectrum,
                              air_tree* trees, float* spectra, float* images, double* flux, air_stats* stats,
                              void* stream);

/* ------------------------------------------------------------------------
 * Learned depth proposal.  A small network (four 3x3 convolutions,
 * 4 -> 32 -> 32 -> 32 -> 6 channels, zero padding, ReLU after the first
 * three) reads four maps of the coarse trace and predicts, per coarse pixel,
 * the deepest level of its final tree (classes 0..5).  air_render_learned
 * traces every node down to a depth chosen from that prediction in one
 * speculative march, then runs the level loop of air_render, which traces
 * only the nodes the speculation did not cover.  Its outputs are bit for bit
 * those of air_render; only the time differs.
 * ---------------------------------------------------------------------- */
#define AIR_CNN_FEATURES 4
#define AIR_CNN_CLASSES 6
#define AIR_CNN_PARAMS 21414 /* for each layer: weights [cout][3][3][cin], then bias [cout] */

typedef struct air_cnn air_cnn;

/* A network on the context's device, parameters zero, feature mean 0 and
 * scale 1.  Destroy it before its context. */
air_status air_cnn_create(air_ctx* ctx, air_cnn** out);
void air_cnn_destroy(air_cnn* net);
/* Host parameters [AIR_CNN_PARAMS] (float32 master copy) and the feature
 * standardisation (x - mean) / scale applied to the raw maps (scale > 0).
 * Resets the optimiser state. */
air_status air_cnn_set(air_ctx* ctx, air_cnn* net, const float* params, const float* feat_mean,
                       const float* feat_scale);
/* Copy the parameters and the standardisation back to the host (any may be
 * NULL); synchronises the context's device. */
air_status air_cnn_get(air_ctx* ctx, const air_cnn* net, float* params, float* feat_mean, float* feat_scale);
/* Checkpoint of a network for resuming its training: air_cnn_save writes the
 * parameters, the feature standardisation, the optimiser's moment estimates
 * and step count to the file at path (a binary header, then float32 arrays,
 * in the host's byte order); air_cnn_load reads such a file into net,
 * replacing all of these, so that the next air_cnn_adam continues exactly
 * where the saved network stopped.  Both synchronise the context's device.
 * air_cnn_load checks the header, the sizes and that every value is finite
 * (scales > 0, second moments >= 0) before it changes net.
 * Errors: EINVAL (NULL path, unreadable or unwritable file, a file that is
 * not such a checkpoint; the reason in air_last_error), EDEVICE. */
air_status air_cnn_save(air_ctx* ctx, const air_cnn* net, const char* path);
air_status air_cnn_load(air_ctx* ctx, air_cnn* net, const char* path);

/*
 * Raw input maps of the coarse trace, device [n_views][coarse_n][coarse_n][4]
 * in raster order (row j = pixel index along e_v): log10(I_w + 1e-30) with
 * I_w = sum_b band_weight[b] I_b (host [n_bands]), log10(N + 1e-30), the
 * finest grid level the ray crosses (-1 for a miss), and
 * log10(rho_max / rho_min) over the cells it crosses (0 for a miss or a zero
 * density).
 */
air_status air_features(air_ctx* ctx, const air_grid* grid, const air_field* field, const air_view* views,
                        int32_t n_views, int32_t coarse_n, const float* band_weight, float* features,
                        void* stream);

/*
 * Forward pass on n_maps raw maps (device [n_maps][h][w][4], standardised
 * with the network's mean and scale, then rounded to bfloat16) into logits
 * (device [n_maps][h][w][8] float32, classes 0..5 in the first six).
 * Weights and activations are bfloat16, accumulation float32.
 */
air_status air_cnn_forward(air_ctx* ctx, air_cnn* net, const float* features, int32_t n_maps, int32_t h,
                           int32_t w, float* logits, void* stream);

/*
 * Loss and gradient of one batch: class-weighted softmax cross-entropy,
 * sum_p cw[t_p] (-log softmax(z_p)[t_p]) / sum_p cw[t_p], with labels device
 * [n_maps][h][w] (values outside 0..5 are clamped) and class_weight host
 * [6].  loss: host, may be NULL (then the call does not wait).  The
 * gradient is kept in the network for air_cnn_adam and copied to grad
 * (device [AIR_CNN_PARAMS] float32) when grad is not NULL.
 */
air_status air_cnn_loss_grad(air_ctx* ctx, air_cnn* net, const float* features, const int32_t* labels,
                             int32_t n_maps, int32_t h, int32_t w, const float* class_weight, double* loss,
                             float* grad, void* stream);

/*
 * Intermediate tensors of the last air_cnn_forward or air_cnn_loss_grad call
 * on this context (an air_render_learned call in between discards them), for
 * inspection layer by layer.  P = n_maps * h * w pixels in the order of the
 * features; every tensor is pixel-major with its channels adjacent:
 *   AIR_CNN_T_X0  bfloat16 [P][8]: the standardised input maps (channels 0..3, 4..7 zero);
 *   AIR_CNN_T_A1..A3  bfloat16 [P][32]: the outputs of layers 0..2 after bias and ReLU
 *                  (the inputs of layers 1..3);
 *   AIR_CNN_T_Z   float32 [P][8]: the logits (classes 0..5);
 *   AIR_CNN_T_DZ  bfloat16 [P][8]: the loss gradient with respect to the logits
 *                  (air_cnn_loss_grad only);
 *   AIR_CNN_T_D3..D1  bfloat16 [P][32]: the loss gradient with respect to A3..A1,
 *                  masked where the activation is zero (air_cnn_loss_grad only).
 * Copies the tensor to out (device, at least the size above) on the stream.
 * Errors: EINVAL (no such call, unknown tensor, gradients asked of a forward
 * call, out too small).
 */
#define AIR_CNN_T_X0 0
#define AIR_CNN_T_A1 1
#define AIR_CNN_T_A2 2
#define AIR_CNN_T_A3 3
#define AIR_CNN_T_Z 4
#define AIR_CNN_T_DZ 5
#define AIR_CNN_T_D3 6
#define AIR_CNN_T_D2 7
#define AIR_CNN_T_D1 8
air_status air_cnn_tensor(air_ctx* ctx, int32_t which, void* out, int64_t bytes, void* stream);

/* One Adam step (bias-corrected) with the network's last gradient. */
air_status air_cnn_adam(air_ctx* ctx, air_cnn* net, float lr, float beta1, float beta2, float eps, void* stream);

/* Training labels: the deepest level of a finished tree (from air_render)
 * inside each coarse pixel, device int32 [coarse_n][coarse_n] raster order. */
air_status air_tree_depth(air_ctx* ctx, const air_tree* tree, int32_t coarse_n, int32_t* depth, void* stream);

/* Cost model of the depth choice: per coarse pixel, the depth d in
 * 0..min(max_depth, params.max_level) minimising
 * c_ray * (4 + 16 + ... + 4^d) + c_sweep * P(deeper than d). */
typedef struct {
  float c_ray;
  float c_sweep;
  int32_t max_depth;
  uint32_t flags; /* reserved, must be 0 */
} air_learn_params;

typedef struct {
  int64_t spec_rays;                    /* rays traced by the speculative march */
  int64_t wasted;                       /* speculative rays that are no tree node */
  int64_t missing;                      /* tree nodes below level 0 the level loop traced */
  int64_t depth_hist[AIR_MAX_LEVELS];   /* coarse pixels per chosen depth */
  double ms_features; /* with AIR_FLAG_TIMING: feature maps + network + depth choice + work list */
  double ms_spec;     /* with AIR_FLAG_TIMING: the speculative march */
} air_learn_stats;

/*
 * air_render with the learned proposal (arguments as air_render, plus the
 * network, its cost model and optional counters).  Trees, images and fluxes
 * equal air_render's bit for bit.
 */
air_status air_render_learned(air_ctx* ctx, const air_grid* grid, const air_field* field, const air_view* views,
                              int32_t n_views, const air_params* params, const air_cnn* net,
                              const air_learn_params* learn, air_tree* trees, float* images, double* flux,
                              air_stats* stats, air_learn_stats* learn_stats, void* stream);

/*
 * air_render with a given speculation depth per coarse pixel in place of the
 * network's choice: the baselines the learned proposal is measured against
 * (a constant depth, or the true depths of a finished tree from
 * air_tree_depth).  depth: device uint8 [n_views][coarse_n][coarse_n] in
 * raster order, each clamped to min(max_depth, params.max_level, 5); the
 * nodes of each coarse pixel's subtree down to that depth are traced in one
 * speculative march before the level loop.  Outputs equal air_render's bit
 * for bit; learn_stats (may be NULL) counts speculative, wasted and missing
 * rays.  Errors as air_render.
 */
air_status air_render_proposal(air_ctx* ctx, const air_grid* grid, const air_field* field, const air_view* views,
                               int32_t n_views, const air_params* params, const uint8_t* depth, int32_t max_depth,
                               air_tree* trees, float* images, double* flux, air_stats* stats,
                               air_learn_stats* learn_stats, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* AIR_H */
