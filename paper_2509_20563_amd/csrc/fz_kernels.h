// Host-side launchers of the libfz kernels (one declaration per kernel group).
#pragma once

#include "fz_common.h"

namespace fz {

// fz_quant.hip
void launch_reset(hipStream_t st, Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2,
                  uint32_t n2, uint64_t* d3, uint32_t n3, uint64_t off_chunks, uint64_t off_stream, uint64_t nreg);
void launch_fill32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v);
void launch_minmax(hipStream_t st, const float* x, uint64_t N, int vec, Misc* misc, int grid);
void launch_quant(hipStream_t st, int grid, const float* x, const Geom& g, uint32_t mode, double eb, int vec,
                  Misc* misc, uint32_t* hist, uint16_t* codes, uint32_t ntiles, uint32_t* tile_cnt, uint2* ostage,
                  uint2* pstage, int fixed_pred, const uint8_t* bpred,
                  int32_t* coef);
void launch_quant_shuffle(hipStream_t st, int grid, const float* x, const Geom& g, uint32_t mode, double eb, int vec,
                          Misc* misc, uint32_t* hist, uint32_t* slots, uint32_t ntiles, uint32_t* tile_cnt,
                          uint2* ostage, uint2* pstage);
void launch_trial(hipStream_t st, int grid, const float* x, const Geom& g, uint32_t mode, double eb, int vec,
                  Misc* misc, uint32_t ntiles, const uint32_t* cw_ref, uint8_t* choice, uint32_t* costs);

// fz_select.hip: the learned selector (features over each block's sample,
// then the network; feat [nblocks][16] float, choice one byte per block)
uint32_t feature_tiles(uint32_t nblocks);
void launch_features(hipStream_t st, int grid, const float* x, const Geom& g, uint32_t mode, double eb, int vec,
                     Misc* misc, float* feat);
void launch_mlp(hipStream_t st, int grid, const float* feat, uint32_t n, const float* sel, float* yout,
                uint8_t* choice);

// fz_scan.hip
void launch_scan(hipStream_t st, int kind, const void* in, uint32_t n, uint64_t* out, uint64_t* desc, uint32_t* ctr,
                 Misc* misc, uint64_t expect);
uint32_t scan_tiles(uint32_t n);

// fz_huffman.hip
void launch_codebook(hipStream_t st, uint32_t* hist, uint8_t* out_lens, uint32_t* cw, Misc* misc);
void launch_encode(hipStream_t st, int grid, const uint16_t* codes, const Geom& g, const uint32_t* cw, Misc* misc,
                   uint32_t ntiles, uint8_t* out, uint64_t* desc, uint64_t* tile_start, uint32_t* tfirst,
                   uint32_t* tlast);
uint32_t encode_groups(uint32_t ntiles);
void launch_finalize(hipStream_t st, const Geom& g, uint32_t mode, double eb, uint32_t pred, Misc* misc,
                     uint8_t* out, uint32_t ntiles, const uint64_t* tile_start, const uint32_t* tfirst,
                     const uint32_t* tlast, const uint32_t* tile_cnt, const uint64_t* tile_off, const uint2* ostage,
                     const uint2* pstage, const uint8_t* bpred, const uint64_t* reg_idx, const int32_t* coef,
                     const float* x, uint32_t codec = 0);

// fz_train.hip: selector training (device scratch of one minibatch)
struct TrainScratch {
    float *Z, *H1, *H2, *DY, *DH1, *DH2, *SE, *grad;
};
void launch_targets(hipStream_t st, const uint32_t* costs, uint64_t n, float* t);
void launch_feature_stats(hipStream_t st, const float* feat, uint64_t n, float* w);
void launch_train_batch(hipStream_t st, const float* w, const float* feat, const float* tgt, const uint32_t* idx,
                        uint32_t B, TrainScratch& s, float* loss_out);
void launch_adam(hipStream_t st, float* w, float* m, float* v, const float* g, int t, float lr, float b1, float b2,
                 float eps);


// fz_speed.hip: the bit-shuffle codec (staging slots of the quantiser +
// offsets -> masks + kept words in the container; masks + kept words ->
// field)
void launch_shuffle_copy(hipStream_t st, const Geom& g, const uint32_t* slots, const uint64_t* off, uint8_t* out,
                         uint64_t limit);
void launch_unshuffle(hipStream_t st, const Geom& g, const uint32_t* masks, const uint32_t* kept, uint64_t nkept,
                      const uint64_t* off, const uint32_t* opos, const int32_t* oval, const uint2* oidx,
                      uint64_t n_out, double e2, float* out, Misc* misc);

// fz_batch.hip
void launch_field_record(hipStream_t st, const Misc* misc, uint64_t slot, uint64_t* rec, int decode);
void launch_pack(hipStream_t st, const uint8_t* stage, const uint64_t* rec, uint64_t* offs, uint32_t n, uint8_t* out);
void launch_gather_headers(hipStream_t st, const uint8_t* in, const uint64_t* offs, uint32_t n, uint8_t* hdr);

// fz_decode.hip
void launch_copy(hipStream_t st, const uint8_t* src, float* dst, uint64_t n);
// the decompression's first launch: the per-call reset (as launch_reset) and
// the decode table built from the packed code lengths
void launch_reset_lut(hipStream_t st, Misc* misc, uint32_t* hist, uint64_t* d1, uint32_t n1, uint64_t* d2,
                      uint32_t n2, uint64_t* d3, uint32_t n3, uint64_t off_chunks, uint64_t off_stream,
                      uint64_t nreg, const uint8_t* lens_packed, uint16_t* lut);
void launch_outlier_index(hipStream_t st, const Geom& g, const uint32_t* opos, uint64_t n_out, uint2* oidx,
                          Misc* misc);
void launch_decode(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t stream_words,
                   const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                   const int32_t* oval, const uint2* oidx, uint64_t n_out, double e2, float* out,
                   int vec, Misc* misc);
void launch_map_unpack(hipStream_t st, const uint8_t* map, uint32_t nblocks, uint8_t* bpred, Misc* misc);
void launch_decode_pred(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t stream_words,
                        const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                        const int32_t* oval, const uint2* oidx, uint64_t n_out, int32_t* res,
                        int fixed_pred, const uint8_t* bpred, const uint64_t* reg_idx, const int32_t* coefs,
                        uint64_t nreg, double e2, float* out, int vec, Misc* misc);
// residuals only (row-major int32, N values), for the whole-field
// predictors (interpolation, global Lorenzo); vec: res 16-byte aligned and
// rows a multiple of 4 values
void launch_decode_residuals(hipStream_t st, const Geom& g, const uint32_t* stream, uint64_t stream_words,
                             const uint64_t* off, const uint16_t* chunks, const uint16_t* lut, const uint32_t* opos,
                             const int32_t* oval, const uint2* oidx, uint64_t n_out, int32_t* res, int vec,
                             Misc* misc);
// fz_interp.hip: residuals q (row-major) to grid values in place, then
// dequantised row-major floats
void launch_interp_inverse(hipStream_t st, const Geom& g, int32_t* q, double e2, float* out);
// fz_global.hip: residuals q (row-major, in place) of the global Lorenzo
// predictor to dequantised row-major floats; 1D uses desc (look-back
// descriptors, global_scan_tiles(N) of them) and misc->mtile_ctr
uint32_t global_scan_tiles(uint64_t N);
void launch_global_inverse(hipStream_t st, const Geom& g, int32_t* q, uint64_t* desc, Misc* misc, double e2,
                           float* out, int vec);
void launch_patch(hipStream_t st, const Geom& g, const uint32_t* ppos, const uint32_t* pbits, uint64_t n_pat,
                  float* out, Misc* misc);

// fz_api.hip: decompression of a first-order Lorenzo (or verbatim)
// container on scratch the caller provides, for up to max_blocks blocks
// (misc: one Misc; hist: kHistCopies * kBins; lut: kLut; desc_chunks:
// scan_tiles(max_blocks); off and oidx: max_blocks each)
struct DecodeScratch {
    Misc* misc;
    uint32_t* hist;
    uint16_t* lut;
    uint64_t* desc_chunks;
    uint64_t* off;
    uint2* oidx;
    uint32_t max_blocks;
};
int decompress_on_scratch(const DecodeScratch& s, const void* d_in, uint64_t in_bytes, const void* h_hdr,
                          float* d_out, uint64_t out_elems, hipStream_t st);

}  // namespace fz
