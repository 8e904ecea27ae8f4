/* surrogate.h -- C ABI of the learned surrogate's gfx950 kernels: a 3D
 * convolutional encoder-decoder trained on coarse solver snapshots
 * (phi, u, v, w, p) that advances them by a fixed number of solver steps.
 *
 * The paper has no learned part; the network, its loss (mean squared error)
 * and optimiser (Adam with bias correction) are this library's own
 * definitions.  The convolution is the padded 3 x 3 x 3 cross-correlation
 *     y[n, p, o] = b[o] + sum_{k, c} w[o, k, c] X[n, s p + k - 1, c]
 * with stride s in {1, 2} and X the input upsampled by u in {1, 2} by
 * nearest neighbour (X[q] = x[q / u]), zero outside; output extent
 * ceil(u n / s) per axis.
 *
 * Conventions (every function):
 *   - pointers are device pointers unless stated; the caller allocates and
 *     frees every buffer; nothing is allocated by these calls;
 *   - activations are bf16 (stored as uint16_t) in N, D, H, W, C order with C
 *     a multiple of 16 (at most 64); weights are bf16 [co][27][ci] (tap
 *     index k = (kz * 3 + ky) * 3 + kx) with the flipped copy
 *     wf[c][26 - k][o] = w[o][k][c] used by the data gradient; master
 *     weights, gradients and optimiser
 *     moments are float;
 *   - calls are asynchronous on `stream` (hipStream_t, NULL = default);
 *   - return 0 on success, SG_EINVAL for inconsistent sizes or a null
 *     required pointer (nothing is launched), SG_EDEVICE if a launch failed
 *     (text in sg_last_error()).
 */
#ifndef SURROGATE_H
#define SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SG_OK = 0, SG_EINVAL = -1, SG_EDEVICE = -3 };

const char* sg_last_error(void);

/* Forward convolution.  x [n, d, h, w, ci]; wgt [co][27][ci]; bias [co];
 * y [n, od, oh, ow, co] with od = ceil(up d / stride) etc.
 *   relu : y = max(z, 0) (else y = z), z the biased convolution;
 *   skip : nullable [n, od, oh, ow, co], added after the activation;
 *   yr   : nullable, receives max(z, 0) (or z) before the skip is added
 *          (the gradient needs the activation's own sign).
 * stride 2 with up 2 is rejected.  Stride-1 layers with ci == co <= 32,
 * and the 32 -> 16 and 64 -> 32 channel upsampling layers, stage each
 * block's input brick with its halo in LDS. */
int sg_conv3d_fwd(const uint16_t* x, int n, int d, int h, int w, int ci, const uint16_t* wgt,
                  const float* bias, int co, int stride, int up, int relu, const uint16_t* skip,
                  uint16_t* y, uint16_t* yr, void* stream);

/* Data gradient.  dz [n, od, oh, ow, co] (gradient of the layer's
 * pre-activation); wgt_f [ci][27][co], the flipped copy of the layer's
 * weights (sg_flip_weights); output at the layer input [n, d, h, w, ci]:
 *   g    = sum over the taps and output voxels that read each input voxel
 *          (+ add[...] if add is non-null: a gradient arriving by another path);
 *   da   : nullable, receives g;
 *   dzp  : receives g masked by mask > 0 (mask: the previous layer's
 *          activation before any skip; null: no mask).
 * Stride-1 layers with ci == co == 16 run as a convolution of dz with
 * wgt_f from an LDS halo tile. */
int sg_conv3d_bwd_data(const uint16_t* dz, int n, int d, int h, int w, int ci, const uint16_t* wgt_f,
                       int co, int stride, int up, const uint16_t* add, const uint16_t* mask,
                       uint16_t* da, uint16_t* dzp, void* stream);

/* Workspace (bytes) of sg_conv3d_bwd_weight for these sizes. */
size_t sg_conv3d_bwd_weight_workspace(int n, int d, int h, int w, int ci, int co, int stride, int up);

/* Weight and bias gradients: dw [co][27][ci] = sum over output voxels of
 * dz[v, o] X[n, s p + k - 1, c]; db [co] = sum of dz.  x [n, d, h, w, ci],
 * dz [n, od, oh, ow, co]; ws of at least the size above.  Summation order
 * is fixed (split over voxel chunks, partials added in a fixed order), so the
 * result is deterministic.  Overwrites dw and db. */
int sg_conv3d_bwd_weight(const uint16_t* x, int n, int d, int h, int w, int ci, const uint16_t* dz, int co,
                         int stride, int up, void* ws, size_t ws_bytes, float* dw, float* db, void* stream);

/* Flipped bf16 weight copy for the data gradient: wf[c][26 - k][o] = w[o][k][c]. */
int sg_flip_weights(const uint16_t* w, int co, int ci, uint16_t* wf, void* stream);

/* Folded bf16 weights of a x2 upsampling layer's data gradient, wu [ci][64][co]:
 * wu[c][a][o] = sum over taps k with k_d in F(a_d) on every axis d of
 * w[o][k][c], where a = (az * 4 + ay) * 4 + ax and F(a) = {2}, {1, 2}, {0, 1},
 * {0} for a = 0..3 (summed in FP32, rounded once to bf16).  Along an axis,
 * output p = 2 r - 1 + a of the layer reaches input voxel r through exactly
 * the taps of F(a), over both upsampled copies of r. */
int sg_fold_up_weights(const uint16_t* w, int co, int ci, uint16_t* wu, void* stream);

/* Data gradient of a stride-1, x2 upsampling layer from the folded weights
 * wu (sg_fold_up_weights): g[n, r, c] = sum over a in 4 x 4 x 4 and o of
 * wu[c][a][o] dz[n, 2 r - 1 + a, o] (zero outside), a 4 x 4 x 4 stride-2
 * gather with K = 64 co instead of 27 x 8 co.  Arguments and outputs (add,
 * mask, da, dzp) as sg_conv3d_bwd_data with stride 1 and up 2; equal to it
 * up to the rounding of the folded weights to bf16. */
int sg_conv3d_bwd_data_up2(const uint16_t* dz, int n, int d, int h, int w, int ci, const uint16_t* wu, int co,
                           const uint16_t* add, const uint16_t* mask, uint16_t* da, uint16_t* dzp,
                           void* stream);

/* Adam step with bias correction over a flat float buffer of `count`
 * parameters (master p, moments m and v, gradient g), step number t >= 1;
 * pb (nullable) receives the bf16 copy of the updated parameters. */
int sg_adam(float* p, float* m, float* v, const float* g, long long count, int t, float lr, float beta1,
            float beta2, float eps, uint16_t* pb, void* stream);

/* Per-channel normalisation of [n, c, vox] float: xn = (x - shift[c]) * scale[c]
 * (shift, scale: device arrays of c floats).  In place allowed. */
int sg_normalize(const float* x, int n, int c, long long vox, const float* shift, const float* scale,
                 float* xn, void* stream);

/* Pack normalised [n, c, vox] float into bf16 [n, vox, cpad] (channels
 * c..cpad-1 zero), cpad a multiple of 16 >= c. */
int sg_pack(const float* xn, int n, int c, long long vox, int cpad, uint16_t* xb, void* stream);

/* Residual loss: pred = xn + rs[c] r[..., c] (rs: device array of c
 * increment scales, null for ones), d = pred - tn,
 *   L = mean over n c vox of d^2 + mass_weight * mean_n (S_n / vox)^2,
 * S_n the sum of d over the voxels of channel 0 (the phase field) of sample
 * n: the second term asks the prediction to carry the phase-field content
 * of the target.  r [n, vox, cpad] bf16 (the last layer's output); writes
 * dr [n, vox, cpad] = dL/dr (zero in the padding channels) and, if loss is
 * non-null, L as a double.  ws (required): device workspace of 2048 doubles
 * (FP64 partial sums added in a fixed order, then the per-sample sums);
 * mass_weight >= 0, and n <= 1024 when it is positive. */
int sg_residual_loss(const float* xn, const float* tn, const uint16_t* r, const float* rs, int n, int c,
                     long long vox, int cpad, float mass_weight, uint16_t* dr, double* loss, void* ws,
                     void* stream);

/* Prediction in physical units:
 * out[n, c, vox] = (xn + rs[c] r[..., c]) / scale[c] + shift[c] (rs nullable). */
int sg_unpack(const float* xn, const uint16_t* r, const float* rs, int n, int c, long long vox, int cpad,
              const float* shift, const float* scale, float* out, void* stream);

/* Coarse window of solver fields: phi [nz, ny, nx], u [3][nz][ny][nx],
 * p [nz, ny, nx] (the layout of lbm_fields) averaged over
 * 2 x 2 x 2 blocks into out [5][dw][ny/2][nx/2] = (phi, ux, uy, uz, p) for
 * coarse planes z0c .. z0c + dw - 1; planes at or beyond nz/2 are zero.
 * nx and ny even. */
int sg_coarsen(const float* phi, const float* u, const float* p, int nx, int ny, int nz, int z0c, int dw,
               float* out, void* stream);

/* Phase-field budget of coarse states x [n, c, d, h, w] (phi in channel 0,
 * u_z in channel 3): per sample, in FP64, sums[3 i + 0] = sum phi,
 * sums[3 i + 1] = sum over the plane z = 0 of phi u_z, sums[3 i + 2] = the
 * same over z = d - 1.  sums is a device array of 3 n doubles. */
int sg_phi_budget(const float* x, int n, int c, int d, int h, int w, double* sums, void* stream);

/* Gather rows of a float store: out[j, :] = store[idx[j], :] for j < n,
 * rows of `len` elements; idx is a device array of n row indices, each in
 * [0, rows) (checked on the device: an index out of range yields a row of
 * NaN). */
int sg_gather(const float* store, long long rows, long long len, const long long* idx, int n, float* out,
              void* stream);

#ifdef __cplusplus
}
#endif
#endif
