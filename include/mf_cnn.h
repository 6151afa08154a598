/*
 * mf_cnn.h -- kernels of the bracket-proposal network (not in the paper).
 *
 * A small CNN predicts, per 8x8-pixel cell, a value bracket [lo, hi] meant
 * to contain the medians of the cell's pixels; the exact filter then ranks
 * only the pixels inside a tile's bracket (median_filter_learned).  These
 * entry points expose the network's kernels for training and testing.
 * All pointers are DEVICE pointers; calls are asynchronous on `stream`;
 * argument errors return MF_ERR_INVALID_ARG before anything is queued.
 *
 * Layouts: activations bf16 [H][W][32] (32 channels per cell); weights bf16
 * [cout][9][32] with tap = 3 * (dy + 1) + (dx + 1); bias f32 [cout].
 * cout is 32 (hidden layers) or 16 (output layer: channel 0 = lo, 1 = hi).
 * Convolutions are 3x3, stride 1, zero padding, bf16 x bf16 products summed
 * in float32 on MFMA.
 */
#ifndef MF_CNN_H
#define MF_CNN_H

#include <stddef.h>

#include "median_filter.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One 16x32 by 32x16 bfloat16 matrix product on the MFMA unit (row-major
 * inputs and output, D f32), for checking the operand layout. */
int mf_mfma_probe(const void* a, const void* b, float* d, hipStream_t stream);

/* y = conv3x3(x, w) + bias with an epilogue:
 *   mode 0: bf16 [H][W][32] = relu(.)               (cout must be 32)
 *   mode 1: f32 [H][W][cout] = (.)                  (cout 16 or 32)
 *   mode 2: bf16 [H][W][32] = (.) * [mask > 0], mask a bf16 activation,
 *           bias may be NULL (backward data through a ReLU; cout 32).
 * cout == 16 always writes f32 (mode is ignored but must be 1). */
int mf_cnn_conv_forward(const void* x, int H, int W, const void* w, const float* bias, int cout,
                        int mode, const void* mask, void* y, hipStream_t stream);

/* Weights for backward data: wf[ci][t][co] = w[co][8 - t][ci] (co < cout,
 * else 0); wf is bf16 [32][9][32].  Then dX = mf_cnn_conv_forward(dY, wf). */
int mf_cnn_flip_weights(const void* w, int cout, void* wf, hipStream_t stream);

/* Weight and bias gradients: dw[co][t][ci] = sum_cells dy[cell][co] *
 * x[cell + offset(t)][ci], db[co] = sum_cells dy[cell][co] (f32).  x and dy
 * are bf16 [H][W][32] (dy channels >= cout ignored).  Split over blocks of
 * segs_per_block 32-cell row segments into `workspace` (floats; size from
 * mf_cnn_wgrad_workspace), then reduced in a fixed order (deterministic). */
long long mf_cnn_wgrad_workspace(int H, int W, int cout, int segs_per_block);
int mf_cnn_conv_wgrad(const void* x, const void* dy, int H, int W, int cout, int segs_per_block,
                      float* workspace, float* dw, float* db, hipStream_t stream);

/* Pinball loss of out[cell][0] (lo) and out[cell][1] (hi) (f32, out_ch
 * floats per cell) against tgt[cell][2]: writes d(sum of losses)/d(out) as
 * bf16 [ncell][32] (channels 2..31 zero) and per-256-cell partial sums of
 * the loss to part_loss[ceil(ncell / 256)]. */
int mf_cnn_pinball(const float* out, int out_ch, const float* tgt, int ncell, float tau_lo,
                   float tau_hi, void* dout, float* part_loss, hipStream_t stream);

/* Network input per 8x8 cell (bf16 [ceil(h/8)][ceil(w/8)][32]): channel 0 =
 * mean pixel value / 255 (u8) or / 65535 (u16), channel 1 = radius / 64. */
int mf_cnn_features(const void* img, int w, int h, size_t stride_bytes, int dtype, int radius,
                    void* feat, hipStream_t stream);

/* The whole network for inference in one launch: features (as
 * mf_cnn_features), three 32-channel ReLU layers and the 16-channel output
 * layer, writing out f32 [ceil(h/8)][ceil(w/8)][16].  w_bf16[l] and bias[l]
 * (l = 0..3) are layer l's weights (16-byte aligned) and bias in the
 * layouts above (cout 32, 32, 32, 16).  Equal bit for bit to mf_cnn_features followed by
 * mf_cnn_conv_forward in modes 0, 0, 0 and 1; nothing is allocated and no
 * intermediate activation is written to memory. */
int mf_cnn_net_forward(const void* img, int w, int h, size_t stride_bytes, int dtype, int radius,
                       const void* const* w_bf16, const float* const* bias, float* out,
                       hipStream_t stream);

/* Training targets per cell (f32 [cells][2]): min and max of the median
 * image over the cell, divided by 255 or 65535. */
int mf_cnn_targets(const void* med, int w, int h, size_t stride_bytes, int dtype, float* tgt,
                   hipStream_t stream);

/* Adam step (step >= 1) on n float32 parameters with their moments; also
 * writes the bf16 copy p_bf16 (may be NULL). */
int mf_cnn_adam(float* p, float* m, float* v, const float* grad, int n, float lr, float b1,
                float b2, float eps, int step, void* p_bf16, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The network object and the learned filter.
 *
 * mf_learned holds the parameters (float32 master copy + bf16 copy, layout
 * W1 b1 W2 b2 W3 b3 W4 b4 as above, mf_learned_param_count() floats), the
 * Adam state and device workspaces sized on first use.  Create: He-normal
 * weights from `seed`, output biases lo = 0, hi = 1 (an untrained network
 * brackets the full range).  Workspace growth synchronizes the device.  One
 * object must not be used from two streams at once.
 * ------------------------------------------------------------------------ */
typedef struct mf_learned mf_learned;

int mf_learned_create(unsigned long long seed, mf_learned** out);
void mf_learned_destroy(mf_learned* net);
int mf_learned_param_count(void);
/* Host float32 copies of all parameters (synchronous); set also resets the
 * Adam state. */
int mf_learned_get_params(const mf_learned* net, float* host);
int mf_learned_set_params(mf_learned* net, const float* host);
/* Host float32 copy of the parameter gradient of the last train step
 * (synchronous; same layout as the parameters; the loss is the pinball loss
 * summed over cells).  Zero before the first step. */
int mf_learned_get_grads(const mf_learned* net, float* host);
/* Bracket margin added on both sides, in units of the dtype's full range
 * (calibrated on held-out images by the caller). */
int mf_learned_set_margin(mf_learned* net, float margin);

/* Forward pass over the cells of an 8-bit or 16-bit image (one launch,
 * as mf_cnn_net_forward): out_cells is f32 [ceil(h/8)][ceil(w/8)][16]
 * (device), channel 0 = lo, 1 = hi. */
int mf_learned_forward(mf_learned* net, const void* img, int w, int h, size_t stride_bytes,
                       int dtype, int radius, float* out_cells, hipStream_t stream);

/* One Adam step (learning rate lr) on the pinball loss (tau 0.02 for lo,
 * 0.98 for hi) of the cell brackets against the min/max of `median` (the
 * exact median image, same size/stride/dtype as img) over each cell.  If
 * loss is not NULL it receives the mean loss (synchronous). */
int mf_learned_train_step(mf_learned* net, const void* img, const void* median, int w, int h,
                          size_t stride_bytes, int dtype, int radius, float lr, float* loss,
                          hipStream_t stream);

/* Tile grid the learned and bracketed filters use for this image: tile
 * counts, the output tile size (the tallest default shape; it may differ
 * from the plain filter's choice, mf_query_plan), and the most in-bracket
 * box pixels a tile can rank (a tile with more is recomputed whole by the
 * plain engine).  Any output pointer may be NULL. */
int mf_learned_tile_grid(int w, int h, int dtype, const mf_footprint* fp, int* tiles_x,
                         int* tiles_y, int* bracket_capacity, int* tile_w, int* tile_h);

/* Exact median filter of an 8/16-bit plane with caller-supplied per-tile
 * value brackets: tile_brackets (device) holds (lo, hi) pairs of unsigned
 * ints, tiles_x * tiles_y of them in row-major tile order (lo > hi: no
 * bracket, the tile is computed by the plain engine).  A tile ranks only
 * its box pixels inside the bracket.  Output pixels whose median lies
 * outside their tile's bracket are recomputed one by one (exact selection
 * over the window), and tiles with more in-bracket pixels than the
 * bracketed layout holds (mf_learned_tile_grid) are recomputed whole by the
 * plain engine, so the output always equals median_filter's.  8/16-bit
 * planes, any radius, w * h < 2^32.  fallback_px (host, may be NULL; if set
 * the call synchronizes) receives the number of output pixels recomputed
 * either way.  `net` supplies workspace only (grown on demand, which
 * synchronizes the device). */
int median_filter_bracketed(const void* img, int w, int h, size_t stride_bytes, int dtype,
                            const mf_footprint* fp, int boundary, const unsigned int* tile_brackets,
                            mf_learned* net, void* out, unsigned long long* fallback_px,
                            hipStream_t stream);

/* Learned filter: the network proposes the brackets (union of a tile's
 * cells, widened by the margin; a bracket wider than 0.3 of the value range
 * is dropped and the tile computed by the plain engine), then as
 * median_filter_bracketed. */
int median_filter_learned(const void* img, int w, int h, size_t stride_bytes, int dtype,
                          const mf_footprint* fp, int boundary, mf_learned* net, void* out,
                          unsigned long long* fallback_px, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MF_CNN_H */
