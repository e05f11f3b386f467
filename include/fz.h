/*
 * fz.h - C ABI of the MI355X (gfx950) error-bounded compressor.
 *
 * The library implements the data-parallel path of the FZMod-Default pipeline
 * of FZModules (Sec. 3.3): value-range or absolute error bound (Sec. 3.2
 * preprocessing), dual-quantisation Lorenzo prediction with outliers
 * (Sec. 3.1), a histogram of the quantisation codes and a Huffman code built
 * from it (Sec. 3.2), chunked Huffman encoding, and the reverse path
 * (Huffman decoding, outlier scatter and inverse Lorenzo, Sec. 1 and
 * Sec. 3.3.1).  Every stage runs as a HIP kernel on the device; the
 * Huffman stages, which FZMod-Default runs on the CPU, run on the GPU here.
 *
 * Conventions
 *  - Pointers named d_* are device pointers; h_* are host pointers.
 *  - A field is float32, row-major, dims[0] the fastest axis; unused axes of
 *    dims are 1.  ndim is 1, 2 or 3.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    All work of a call is enqueued on it.
 *  - The caller owns every buffer and the stream; the library never frees
 *    them.  The context owns all scratch memory.
 *  - Functions return FZ_OK (0) or a negative FZ_ERR_* code; no exception or
 *    abort crosses the boundary.  On error, output contents are unspecified,
 *    *h_out_bytes is 0, and the context stays usable.
 *  - A context is used by one host thread at a time.  Calls on one context
 *    are serialised by that thread; two contexts may run concurrently.
 *
 * Container ("FZM1", little-endian): a 128-byte header, the code lengths
 * (4 bits per symbol, 1024 symbols), [the predictor map, 2 bits per block,
 * for the AUTO predictor modes], [the regression coefficients, int32[4] per
 * regression block in block order], one u16 bit count per block, the
 * bit-contiguous Huffman stream (u32 words, most significant bit first), the
 * outliers (u32 position[], i32 residual[]) and the lossless patches
 * (u32 position[], u32 float bits[]), each section 16-byte aligned.  When
 * that would not be smaller than the raw data the container holds the raw
 * floats instead ("verbatim", header flag bit 0).
 */
#ifndef FZ_H
#define FZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fz_ctx fz_ctx;

/* Error-bound modes (Sec. 3.2 preprocessing, Sec. 4.2 metrics).
 * FZ_EB_ABS: |x - x_hat| <= eb for every value.
 * FZ_EB_REL: |x - x_hat| <= eb * (max(x) - min(x)); a constant field uses eb. */
enum { FZ_EB_ABS = 0, FZ_EB_REL = 1 };

/* Predictors, per block of 8x8x8 (2D: 32x16, 1D: 512) values.  The paper's
 * pipeline uses the first-order Lorenzo predictor (Sec. 3.1); it names
 * higher-order Lorenzo and linear regression as the SZ-family predictors
 * (Sec. 2.1) and leaves choosing among them per block to future work
 * (Sec. 5).  Neighbours outside the block count as zero.
 *  FZ_PRED_LORENZO1   first-order Lorenzo for every block
 *  FZ_PRED_LORENZO2   second-order Lorenzo (weights 1, -2, 1 per axis)
 *  FZ_PRED_REGRESSION linear fit per block, 4 int32 coefficients with 8
 *                     fractional bits stored per block
 *  FZ_PRED_AUTO_MLP   per block, chosen by the learned selector network
 *                     (fz_selector_set / fz_selector_load first, else
 *                     FZ_ERR_UNSUPPORTED)
 *  FZ_PRED_AUTO_TRIAL per block, the predictor whose codes cost the fewest
 *                     bits under the Huffman code of the first-order
 *                     histogram (+64 bits per outlier, +128 for the
 *                     coefficients); ties go to the lower number.
 *  FZ_PRED_INTERP     the interpolation predictor of the quality-oriented
 *                     pipeline (Sec. 3.3, FZMod-Quality: G-Interp in place
 *                     of Lorenzo), over the whole field, not block-local:
 *                     anchors every 8 values per axis by first-order
 *                     Lorenzo on the anchor grid, then levels of stride 4,
 *                     2, 1 interpolated along one axis from the neighbours
 *                     at -/+s and -/+3s (cubic (-1, 9, 9, -1)/16, linear at
 *                     the upper edge, the lower neighbour past it).  The
 *                     paper gives no formula: this is the library's reading.
 *                     Huffman codec only; one residual field of 4 bytes per
 *                     value of extra device memory in both directions.
 *  FZ_PRED_GLOBAL     first-order Lorenzo over the whole field (Sec. 3.1's
 *                     predictor with neighbours in other blocks; zero only
 *                     outside the field): no residuals at block faces, so
 *                     smooth fields lose the per-block corner outliers.
 *                     Decoding adds prefix-sum passes over the whole field
 *                     and 4 bytes per value of residual scratch.  Huffman
 *                     codec only.
 * The AUTO modes store a 2-bit map of the choice in the container, so
 * decompression never repeats the choice. */
enum {
    FZ_PRED_LORENZO1 = 0,
    FZ_PRED_LORENZO2 = 1,
    FZ_PRED_REGRESSION = 2,
    FZ_PRED_AUTO_MLP = 3,
    FZ_PRED_AUTO_TRIAL = 4,
    FZ_PRED_INTERP = 5,
    FZ_PRED_GLOBAL = 6
};

enum {
    FZ_OK = 0,
    FZ_ERR_ARG = -1,         /* bad ndim/dims/pointer/size argument             */
    FZ_ERR_EB = -2,          /* eb not finite or <= 0, or resolved eb out of range */
    FZ_ERR_NONFINITE = -3,   /* the field holds a NaN or an infinity            */
    FZ_ERR_CAPACITY = -4,    /* output buffer smaller than required             */
    FZ_ERR_CORRUPT = -5,     /* container fails validation                      */
    FZ_ERR_HIP = -6,         /* a HIP runtime call failed                       */
    FZ_ERR_NOMEM = -7,       /* device or host allocation failed                */
    FZ_ERR_UNSUPPORTED = -8, /* valid but unsupported option (radius, predictor) */
    FZ_ERR_INTERNAL = -9,    /* a device-side consistency check failed          */
    FZ_ERR_SCRATCH = -10     /* fz_decompress_noalloc: more blocks than its scratch holds */
};

typedef struct {
    uint32_t ndim;     /* 1, 2 or 3                                   */
    uint64_t dims[3];  /* extents, dims[0] fastest; unused axes = 1  */
    uint32_t eb_mode;  /* FZ_EB_ABS or FZ_EB_REL                      */
    double eb;         /* > 0 and finite                              */
    uint32_t pred;     /* FZ_PRED_*                                   */
    uint32_t radius;   /* quantisation radius; 512 (1024 code bins)   */
} fz_params;

/* Create a context on HIP device `device`.  `max_elems` sizes the scratch
 * memory up front (0 = allocate on first use); larger fields later grow it.
 * Returns FZ_OK, FZ_ERR_ARG, FZ_ERR_HIP or FZ_ERR_NOMEM. */
int fz_ctx_create(fz_ctx **out, int device, uint64_t max_elems);

/* Release the context and its scratch memory (NULL is ignored). */
void fz_ctx_destroy(fz_ctx *ctx);

/* Bytes the output buffer of fz_compress must hold for these parameters:
 * the larger of the verbatim container (128 + 4 N) and the packed sections
 * written before the verbatim decision (about 656 + 3 N / 64 + 1.5 N),
 * rounded up to 16.  0 if the parameters are invalid. */
uint64_t fz_compress_bound(const fz_params *p);

/* Compress the field d_in (N floats, device) into d_out (device, out_cap
 * bytes, out_cap >= fz_compress_bound).  Synchronises `stream` once and
 * writes the container size to *h_out_bytes.  Sec. 3.1-3.3. */
int fz_compress(fz_ctx *ctx, const fz_params *p, const float *d_in, void *d_out, uint64_t out_cap,
                uint64_t *h_out_bytes, void *stream);

/* FZMod-Speed pipeline (Sec. 3.3; Sec. 3.2 names the FZ-GPU bit-shuffle and
 * dictionary encoder as the fast alternative to Huffman coding): the same
 * error bound, prequantisation, first-order Lorenzo prediction, outliers and
 * patches as fz_compress, then, in place of the histogram, Huffman code and
 * encoder, a bit-shuffle of the codes: each value's residual d folded to a
 * 10-bit symbol (zigzag: 0, -1, 1, -2 -> 0, 1, 2, 3; 1023 = outlier), each
 * block's 512 symbol slots cut into 16 groups of 32 whose 10 bit planes are
 * 32-bit words, and only the non-zero words kept, listed by a 160-bit mask
 * per block.  No histogram barrier: the encoder runs right after the
 * quantiser.  Container: header flag bit 1 set, predictor 0, then the masks
 * (5 u32 per block), the kept words, the outliers and the patches (16-byte
 * aligned sections); verbatim when not smaller than the raw floats.
 * fz_decompress and fz_decompress_batch read these containers too.  p->pred
 * must be FZ_PRED_LORENZO1 (else FZ_ERR_UNSUPPORTED); otherwise as
 * fz_compress. */
int fz_compress_speed(fz_ctx *ctx, const fz_params *p, const float *d_in, void *d_out, uint64_t out_cap,
                      uint64_t *h_out_bytes, void *stream);

/* Parse a container header held in host memory (at least 128 bytes): the
 * container the compressor writes, whose size defines the compression ratio
 * (Sec. 4.2).  Fills *p, *n_elems (values in the field) and *total_bytes
 * (container size).  Returns FZ_OK or FZ_ERR_CORRUPT. */
int fz_header_read(const void *h_hdr, uint64_t n, fz_params *p, uint64_t *n_elems, uint64_t *total_bytes);

/* Decompress the container d_in (device, in_bytes) into d_out (device,
 * out_elems >= N floats): the reverse path (Sec. 1, Sec. 3.3.1: Huffman or
 * bit-shuffle decoding, outlier scatter, inverse prediction, dequantisation,
 * then the lossless patches).  h_hdr is an optional host copy of the first 128
 * bytes of the container (NULL: the library copies it from the device).
 * Synchronises `stream` at the end to report validation errors.
 * Returns FZ_OK, FZ_ERR_CORRUPT, FZ_ERR_CAPACITY, ... */
int fz_decompress(fz_ctx *ctx, const void *d_in, uint64_t in_bytes, const void *h_hdr, float *d_out,
                  uint64_t out_elems, void *stream);

/* Graph mode (Sec. 3.3.1: the paper runs pipelines as CUDASTF tasks over
 * logical data; the runtime infers the data dependencies from the tasks'
 * access modes and runs independent stages concurrently).  With graph mode
 * on, each fz_compress, fz_compress_speed and fz_decompress call is built
 * as a list of stage tasks, each declaring the data it reads, writes or
 * reduces into; dependencies are inferred from those accesses, independent
 * stages are placed on separate streams (for example the outlier-count scan
 * beside the Huffman code and encoder, or the outlier index beside the
 * chunk-offset scan), and the call is captured once into a graph that later
 * calls with the same parameters, header and buffers replay.  Outputs are
 * identical to the eager calls.  `streams`: 0 = eager calls (the default);
 * 1 = graph mode with every stage on one stream (a captured chain);
 * 2..4 = at most that many streams (larger values mean 4).  Per-stage timing
 * is not recorded in graph mode (the whole-call timing filter "call" is).
 * Returns FZ_OK, or FZ_ERR_ARG for a negative count. */
int fz_set_graph_mode(fz_ctx *ctx, int streams);

/* Shape of the last captured graph of a kind (which: 0 = compression,
 * 1 = decompression): its tasks, the streams they were laid out on, the
 * most tasks at one depth of the dependency graph (1 = a chain) and its
 * dependency edges after transitive reduction.  FZ_ERR_ARG when no graph of
 * that kind was captured. */
int fz_graph_info(fz_ctx *ctx, int which, int *h_tasks, int *h_streams, int *h_width, int *h_edges);

/* Human-readable text for a status code (static storage). */
const char *fz_strerror(int status);

/* Per-stage timing.  When enabled, compress/decompress record HIP events
 * around each kernel on the call's stream; fz_stage_times then returns the
 * stage durations in milliseconds of the last call (count in *n).
 * Stage names are given by fz_stage_name. */
int fz_set_timing(fz_ctx *ctx, int enable);
int fz_stage_times(fz_ctx *ctx, float *h_ms, int max, int *n);
const char *fz_stage_name(fz_ctx *ctx, int i);

/* Restrict the timing to one stage: with `stage` set (a stage name as
 * fz_stage_name gives it, shorter than 32 bytes; the string is copied),
 * calls record one event just before that stage and one after it, and
 * fz_stage_times returns that stage alone (0 stages for a call without it);
 * every other stage runs without events in between.  The name "call"
 * times each whole call as one stage named "call": one event before its
 * first kernel and one after its last, none in between.  NULL restores
 * timing of every stage.  FZ_ERR_ARG for a name of 32 bytes or more. */
int fz_set_timing_stage(fz_ctx *ctx, const char *stage);

/* Stage dump for parity checks: the 1024-bin code histogram of the last
 * successful fz_compress call on this context (Sec. 3.2). */
int fz_last_histogram(fz_ctx *ctx, uint32_t *h_hist);

/* ------------------------------------------------------------------ batches
 * Many fields of any shapes, bounds and predictors in one call.  The
 * fields' kernel sequences run as a few concurrent chains (one stream and
 * one set of scratch per chain, fields assigned longest first), captured
 * once into a HIP graph and replayed while the batch's description
 * (parameters, pointers, launch knobs) stays the same; one synchronisation
 * per call.  The paper's CUDASTF pipeline runs branches of one field's
 * pipeline concurrently (Sec. 3.3.1); here whole fields run concurrently.
 * Containers are identical to those of fz_compress. */

/* Bytes the output of fz_compress_batch must hold: the sum of each field's
 * fz_compress_bound rounded up to 16.  0 if any parameter set is invalid. */
uint64_t fz_compress_batch_bound(uint32_t n, const fz_params *p);

/* Compress n fields: params p[n], d_in[n] (host array of device pointers).
 * The containers are written back to back into d_out (device, 16-byte
 * aligned, out_cap >= fz_compress_batch_bound), each starting on a 16-byte
 * boundary with zero bytes up to it; h_offsets (host, n + 1 entries)
 * receives container i's start, h_offsets[n] the end of the last.  The
 * containers go through device scratch owned by the context (the batch's
 * bound in bytes).  Synchronises `stream` once.  The first failing field's
 * status is returned. */
int fz_compress_batch(fz_ctx *ctx, uint32_t n, const fz_params *p, const float *const *d_in, void *d_out,
                      uint64_t out_cap, uint64_t *h_offsets, void *stream);

/* Decompress n containers packed as fz_compress_batch writes them: d_in
 * (device), h_offsets (host, n + 1), into d_out[n] (host array of device
 * pointers) of out_elems[n] floats each.  Synchronises `stream` twice
 * (headers, end). */
int fz_decompress_batch(fz_ctx *ctx, uint32_t n, const void *d_in, const uint64_t *h_offsets, float *const *d_out,
                        const uint64_t *out_elems, void *stream);

/* Autotuner: times this batch under each chain count (1, 2, 4, 8, 16, at
 * most n) and workgroups-per-CU setting of the quantiser and encoders (4,
 * 8, 16) and keeps the fastest for batches of the same class (log2 of the
 * field count and of the total value count) and for the fields' classes
 * (dimensionality, log2 of the value count, bound mode, predictor).  These
 * knobs never change a container.  Runs the batch (writing d_out) several
 * times.  fz_batch_tuning reports the setting a batch would use.
 * Currently switched off: returns FZ_ERR_UNSUPPORTED (a run over the twelve
 * launch configurations ended in a host crash whose cause is not found);
 * batches use the default knobs. */
int fz_batch_autotune(fz_ctx *ctx, uint32_t n, const fz_params *p, const float *const *d_in, void *d_out,
                      uint64_t out_cap, void *stream);
int fz_batch_tuning(fz_ctx *ctx, uint32_t n, const fz_params *p, uint32_t *h_chains, uint32_t *h_wg_per_cu);

/* ------------------------------------------------ per-block predictor choice
 * The paper leaves choosing a predictor per block automatically to future
 * work (Sec. 5); these calls expose the pieces of that choice.
 *
 * Block order: x fastest, then y, then z (block index = bx + nbx (by + nby
 * bz)); edge blocks are truncated. */
#define FZ_FEATURES 16          /* features per block                      */
#define FZ_SELECTOR_PARAMS 5475 /* floats in the selector's parameter set  */

/* Blocks of a field with these dims (0 if invalid). */
uint64_t fz_block_count(const fz_params *p);

/* The 16 features (version 2) of every block of d_in, computed from the
 * prequantised values at p's error bound over the block's sample, its first
 * 128 positions in block-local row-major order (the lower box: z < 2 of an
 * 8x8x8 block, y < 4 of a 32x16 block, x < 128 of a 512 block; an edge
 * block's sample is that box cut to the block), to d_feat (device,
 * row-major [nblocks][16] float32, feat_cap >= 16 nblocks floats):
 *  0 plog2(1 + variance), 1 plog2(1 + max - min),
 *  2-4 plog2(1 + mean |first difference|) along x, y, z,
 *  5-7 the same for second differences, 8-10 for mixed differences in xy,
 *  yz, xz (pairs inside the sample), 11 plog2(1 + mean |first-order
 *  residual|), 12 plog2(1 + max |first-order residual|), 13 outlier
 *  fraction of the first-order residuals, 14 plog2(1 + max |q|),
 *  15 plog2(1 + |mean q|); plog2(1 + v) is the piecewise-linear base-2
 *  logarithm read from the bits of the float 1 + v.  Bit-identical on any
 *  IEEE machine.  Synchronises `stream`. */
int fz_block_features(fz_ctx *ctx, const fz_params *p, const float *d_in, float *d_feat, uint64_t feat_cap,
                      void *stream);

/* Run the selector network on every block: d_choice[b] (device, nblocks
 * bytes) = predictor 0, 1 or 2; d_y (device, nullable, [nblocks][3]
 * float32) = the network's predicted log2(1 + bits) per predictor.
 * FZ_ERR_UNSUPPORTED without a selector.  Synchronises `stream`. */
int fz_block_select(fz_ctx *ctx, const fz_params *p, const float *d_in, uint8_t *d_choice, float *d_y,
                    void *stream);

/* Exhaustive trial (the FZ_PRED_AUTO_TRIAL choice): d_choice[b] and the
 * three costs in bits d_costs[3 b + p] (device, nullable).  Synchronises
 * `stream`. */
int fz_block_trial(fz_ctx *ctx, const fz_params *p, const float *d_in, uint8_t *d_choice, uint32_t *d_costs,
                   void *stream);

/* Selector parameters, host float32[FZ_SELECTOR_PARAMS] in this order:
 * mu[16], rs[16] (standardisation z = (f - mu) * rs), W1[64][16], b1[64],
 * W2[64][64], b2[64], W3[3][64], b3[3]; hidden layers use ReLU; every dot
 * product is a chain of fused multiply-adds (one rounding per term) in
 * index order from its bias, so that a given parameter set picks the same
 * predictors on any IEEE machine.  set copies them to the device (all
 * must be finite); get returns FZ_ERR_UNSUPPORTED if none is set. */
int fz_selector_set(fz_ctx *ctx, const float *h_params, uint64_t n);
int fz_selector_get(fz_ctx *ctx, float *h_params, uint64_t n);

/* Selector files: 8 bytes "FZSEL\0\0\0", u32 feature-set version (2),
 * u32 parameter count, then the parameters (little-endian float32).
 * load returns FZ_ERR_CORRUPT for a file of another format or version. */
int fz_selector_save(fz_ctx *ctx, const char *path);
int fz_selector_load(fz_ctx *ctx, const char *path);

/* Training of the selector (on the device, fp32). */
typedef struct {
    uint32_t epochs; /* passes over the samples (>= 1)                      */
    uint32_t batch;  /* minibatch size, 1 .. 2^20 (4096 is the default use) */
    float lr;        /* Adam step size (1e-3)                               */
    float beta1;     /* Adam moment decays (0.9, 0.999), in [0, 1)          */
    float beta2;
    float eps;       /* Adam epsilon (1e-8), > 0                            */
    uint64_t seed;   /* initial weights and minibatch order                 */
} fz_train_params;

/* Fit the selector to n samples (blocks): d_feat [n][16] float32 from
 * fz_block_features and d_costs [n][3] uint32 bits per predictor from
 * fz_block_trial, both device.  Targets are log2(1 + bits).  mu and rs
 * are set to the features' mean and inverse standard deviation (rs = 1
 * for a constant feature); each layer's weights and biases start uniform
 * in (-1/sqrt(fan-in), 1/sqrt(fan-in)) from the seed; each epoch visits the samples in a seeded shuffled order in
 * minibatches, one Adam step per minibatch on the mean squared error.
 * h_loss (host, nullable, epochs floats) receives each epoch's mean
 * minibatch loss.  On success the trained network becomes the context's
 * selector.  Allocates device memory for the duration of the call;
 * synchronises `stream`. */
int fz_selector_train(fz_ctx *ctx, const float *d_feat, const uint32_t *d_costs, uint64_t n,
                      const fz_train_params *tp, float *h_loss, void *stream);

/* Gradient of the mean squared error of the context's selector over n
 * samples (1 .. 2^20; d_feat [n][16], d_target [n][3] float32, device) to
 * h_grad (host, FZ_SELECTOR_PARAMS floats; 0 for mu and rs) and the loss
 * to *h_loss (nullable).  For gradient checks.  Synchronises `stream`. */
int fz_selector_grad(fz_ctx *ctx, const float *d_feat, const float *d_target, uint64_t n, float *h_grad,
                     float *h_loss, void *stream);

/* One Adam step (Kingma and Ba) of the training kernel on host arrays of
 * FZ_SELECTOR_PARAMS floats each, in place: for every learned parameter
 * (W1 onwards; mu and rs are left as they are)
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   w -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * step number t >= 1, fp32.  The same kernel fz_selector_train runs after
 * each minibatch; exposed for checks against a reference Adam.  Copies the
 * four arrays through device memory the context allocates for the call;
 * synchronises `stream`.  FZ_ERR_ARG for a null array, t < 1, lr <= 0,
 * eps <= 0 or a beta outside [0, 1). */
int fz_selector_adam_step(fz_ctx *ctx, float *h_w, float *h_m, float *h_v, const float *h_g, int t, float lr,
                          float beta1, float beta2, float eps, void *stream);

/* Allocation-free decompression, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as fz_decompress, without a
 * context: the scratch is one statically sized device array per GPU
 * (fz_noalloc_scratch_bytes bytes, held until the process ends), found on
 * the current device at the first call there.  Accepts first-order Lorenzo
 * containers (FZ_PRED_LORENZO1, Huffman or bit-shuffle coded) of at most
 * FZ_NOALLOC_MAX_BLOCKS blocks and verbatim containers of any size; other predictors give
 * FZ_ERR_UNSUPPORTED, more blocks FZ_ERR_SCRATCH, before any kernel runs.
 * Every call on one GPU shares that GPU's array (each call clears what it
 * needs first): calls that overlap on one GPU, on any streams or host
 * threads, race and must be serialised by the caller.  Calls no hipMalloc or
 * hipFree.  Synchronises `stream`. */
#define FZ_NOALLOC_MAX_BLOCKS 131072u /* 2^26 values in full 8x8x8 blocks */
int fz_decompress_noalloc(const void *d_in, uint64_t in_bytes, const void *h_hdr, float *d_out,
                          uint64_t out_elems, void *stream);

/* Size in bytes of the per-GPU scratch array of fz_decompress_noalloc. */
uint64_t fz_noalloc_scratch_bytes(void);

#ifdef __cplusplus
}
#endif
#endif /* FZ_H */
