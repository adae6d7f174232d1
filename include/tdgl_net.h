/*
 * tdgl_net.h — C ABI of the learned initial-state proposal in libtdgl.
 *
 * A small 3-D convolutional encoder-decoder proposes the polarisation a TDGL
 * relaxation starts from; the TDGL step (tdgl.h) then relaxes from it and
 * decides the final state.  The paper motivates this use of the
 * solver (section 5: relaxed states it generates serve as datasets for
 * data-driven methods); the network itself is this library's addition.
 * It is trained on the GPU by this library's own forward and backward
 * kernels: BF16 weights and activations on the matrix cores, FP32
 * accumulation, FP32 master weights and Adam.
 *
 * The network (width w, a power of two >= 8; grid nx x ny x nz, powers of
 * two with nz >= 4, cells z < thickness form the film, the rest vacuum):
 *   input, 5 channels, each times the film mask m: (T - 350 K) / 100 K, m,
 *     and 10 m^2/C times a low-resolution noise field (C/m^2) repeated over
 *     blocks of noise_div^3 cells;
 *   conv = 3x3x3 cross-correlation with zero padding and bias, tap
 *     t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) reading x[p + (dz, dy, dx)];
 *   act = leaky ReLU, slope 1/8; pool = 2x2x2 mean; up = 2x repetition;
 *   e0a = act(conv(x; 5->w)), e0 = act(conv(e0a; w->w)),
 *   e1a = act(conv(pool e0; w->2w)), e1 = act(conv(e1a; 2w->2w)),
 *   b1 = act(conv(pool e1; 2w->4w)), b2 = act(conv(b1; 4w->4w)),
 *   b3 = act(conv(b2; 4w->4w)), u1 = act(conv(up b3; 4w->2w)) + e1,
 *   u1b = act(conv(u1; 2w->2w)), u0 = act(conv(up u1b; 2w->w)) + e0,
 *   u0b = act(conv(u0; w->w)), P = m * conv(u0b; w->3) in C/m^2.
 *   Loss: sum over film cells and components of (P - P_target)^2 over
 *   3 x the film cells of the batch.
 * Parameters form one FP32 vector: per layer in the order above, W as
 * [cout][27][cin] (C order), then the bias [cout].  w = 32 gives 1,721,859.
 *
 * Storage: BF16 activations are channels-last [position][channel], the
 * channel count padded to a multiple of 16; P and targets are FP32
 * [sample][3][nz][ny][nx].  Conditions: T (K) and thickness (layers, an
 * integer value in a float) per dataset row, noise [row][3][nz/s][ny/s][nx/s]
 * with s = noise_div.  Device arrays are borrowed for the call only.
 *
 * Status codes are those of tdgl.h.  Work runs on the stream given at
 * creation; calls that return host values synchronise that stream.
 */
#ifndef TDGL_NET_H
#define TDGL_NET_H

#include <stddef.h>
#include "tdgl.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdgl_net tdgl_net;

typedef struct {
    int nx, ny, nz;     /* sample grid: powers of two, nx, ny >= 4, nz >= 4      */
    int width;          /* w: power of two in [8, 128]                           */
    int noise_div;      /* s: power of two dividing nx, ny and nz                */
    int max_batch;      /* samples per call, 1..4096                             */
} tdgl_net_cfg;

/* Create a network with all parameters zero and allocate its device
 * buffers (activations of max_batch samples).  Errors: TDGL_E_ARG (shape
 * rules above), TDGL_E_NOMEM, TDGL_E_HIP.  stream: hipStream_t or NULL. */
tdgl_status tdgl_net_create(const tdgl_net_cfg *cfg, void *hip_stream, tdgl_net **out);
void tdgl_net_destroy(tdgl_net *net);
const char *tdgl_net_last_error(const tdgl_net *net);
tdgl_status tdgl_net_num_params(const tdgl_net *net, long long *n);

/* Copy the FP32 parameter vector in from / out to host memory (n entries,
 * the layout above).  set_params also resets the Adam moments and step.
 * Synchronising. */
tdgl_status tdgl_net_set_params(tdgl_net *net, const float *host, long long n);
tdgl_status tdgl_net_get_params(tdgl_net *net, float *host, long long n);

/* Forward pass of nb samples (1..max_batch).  Sample i uses dataset row
 * idx[i] (device int array) or row i if idx is NULL; T, thick, noise are
 * device arrays over the dataset rows.  The library cannot see the length
 * of these device arrays: every idx entry (or, without idx, every row
 * below nb) must be a row they hold.  P_out (device, may be NULL to keep
 * the result internal) receives [nb][3][nz][ny][nx] FP32 in C/m^2, zero in
 * the vacuum layers.  Asynchronous. */
tdgl_status tdgl_net_forward(tdgl_net *net, int nb, const int *idx, const float *T,
                             const float *thick, const float *noise, float *P_out);

/* In-plane symmetry ops (training augmentation).  ops[i] (device int,
 * bits: 1 mirror x, 2 mirror y, 4 swap x and y -- ignored unless nx == ny)
 * replaces sample i's noise field and target by their images under the op:
 * F'(x, y) = D F(src(x, y)) with src = swap(mirror_x(mirror_y(x, y))),
 * F'_x = (-1)^mirror_x F_(swap ? y : x), F'_y = (-1)^mirror_y F_(swap ? x : y),
 * F'_z = F_z.  The open film is invariant under these ops, so the relaxed
 * state of the image of a start is the image of its relaxed state.  NULL:
 * no op. */

/* Forward and backward pass against target rows (device
 * [row][3][nz][ny][nx]), each sample under its symmetry op (ops may be
 * NULL).  Returns the loss and, if grad_host is not NULL, the gradient in
 * the parameter layout; the gradient stays on the device for
 * tdgl_net_adam.  Synchronising. */
tdgl_status tdgl_net_loss_grad(tdgl_net *net, int nb, const int *idx, const int *ops,
                               const float *T, const float *thick, const float *noise,
                               const float *target, double *loss, float *grad_host);

/* One Adam step (Kingma and Ba 2015, bias-corrected) with the gradient of
 * the last tdgl_net_loss_grad.  TDGL_E_STATE if there is none.  Async. */
tdgl_status tdgl_net_adam(tdgl_net *net, double lr, double beta1, double beta2, double eps);

/* nsteps training steps of nb samples each: step s uses rows
 * idx[s * nb .. s * nb + nb - 1] (device) under the symmetry ops
 * ops[s * nb ..] (device, or NULL), forward, backward, Adam with the given
 * rate.  losses_host (nsteps doubles, may be NULL) receives each step's
 * loss before its update.  Synchronising. */
tdgl_status tdgl_net_train(tdgl_net *net, int nsteps, int nb, const int *idx, const int *ops,
                           const float *T, const float *thick, const float *noise,
                           const float *target, double lr, double beta1, double beta2,
                           double eps, double *losses_host);

/* Time the parts of one training step of nb samples (rows 0..nb-1):
 * ms[0] forward, ms[1] loss + backward + gradient reduction, ms[2] Adam,
 * ms[3] the conv kernels of the forward pass, ms[4] the conv kernels of the
 * backward-data pass, ms[5] the weight-gradient kernels; means over reps
 * runs, HIP events on the network's stream.  Leaves parameters unchanged
 * (no Adam step is kept).  Synchronising. */
tdgl_status tdgl_net_profile(tdgl_net *net, int nb, const float *T, const float *thick,
                             const float *noise, const float *target, int reps, double *ms);

/* ---- single layers, for tests of the kernels (raw device pointers) ----
 * tdgl_nn_conv3: one 3x3x3 convolution of nb samples on a 2^lx x 2^ly x
 * 2^lz grid, BF16 channels-last.  in: cin_p channels (at half resolution
 * and read through 2x repetition when in_up2); w: [cout_p][27 cin_p]
 * (k = tap * cin_p + ci); epi selects the epilogue:
 *   0 out = act(acc + bias); 1 out = act(acc + bias), out2 = out + aux;
 *   2 P [nb][3][z][y][x] FP32 = m (acc + bias), m from thick[sample];
 *   3 out = acc; 4 out = acc * act'(aux); 5 out = acc, out2 = acc * act'(aux)
 * (act' = 1 where aux > 0, else 1/8).  cin_p, cout_p: powers of two >= 16
 * (cout_p = 16 for epi 2).  Asynchronous on stream (hipStream_t or NULL). */
tdgl_status tdgl_nn_conv3(int epi, const void *in, int in_up2, const void *w, const float *bias,
                          int nb, int lx, int ly, int lz, int cin_p, int cout_p, void *out,
                          void *out2, const void *aux, float *P, const float *thick,
                          void *hip_stream);

/* Workspace bytes of tdgl_nn_conv3_wgrad for these sizes. */
tdgl_status tdgl_nn_wgrad_workspace(int nb, int lx, int ly, int lz, int cin_p, int cout_p,
                                    size_t *bytes);

/* Weight and bias gradient of a conv: grad (device FP32, cout_p * 27 *
 * cin_p + cout_p) = sum over positions of g[n][co] * in[n + tap][ci], then
 * sum over positions of g[n][co].  g: [n][cout_p] BF16 at the conv's grid;
 * in as for tdgl_nn_conv3.  workspace: device memory of the size above.
 * Asynchronous. */
tdgl_status tdgl_nn_conv3_wgrad(const void *g, const void *in, int in_up2, int nb, int lx, int ly,
                                int lz, int cin_p, int cout_p, void *workspace, size_t ws_bytes,
                                float *grad, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* TDGL_NET_H */
