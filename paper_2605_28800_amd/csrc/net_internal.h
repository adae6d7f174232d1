// Kernels of the initial-state proposal network (3-D conv encoder-decoder)
// and their launchers, shared by net.hip and net_api.cpp.
//
// Tensors are BF16 (stored as uint16), channels-last: [position][channel],
// position = ((b * Z + z) * Y + y) * X + x, the channel count padded to a
// multiple of 16.  Grid sizes are powers of two (log2 in lx, ly, lz).
// Weights: forward [cout_p][27 * cin_p] (k = tap * cin_p + ci), the
// backward-data copy [cin_p][27 * cout_p] with the tap mirrored; tap
// t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace tdgl_nn {

typedef uint16_t bf16_t;

constexpr float SLOPE = 0.125f;     // leaky ReLU slope for negative arguments (exact in BF16)

// epilogues of the implicit-GEMM convolution
enum ConvEpi {
  EPI_ACT = 0,        // out = act(acc + bias)
  EPI_ACT_SKIP = 1,   // out = act(acc + bias), out2 = out + aux
  EPI_P = 2,          // P (FP32, [b][3][z][y][x]) = film mask * (acc + bias)
  EPI_RAW = 3,        // out = acc
  EPI_RAW_D = 4,      // out = acc * act'(aux)
  EPI_RAW_AND_D = 5,  // out = acc, out2 = acc * act'(aux)
};

struct ConvArgs {
  const bf16_t *in;   // input tensor, cin_p channels (half resolution if in_up2)
  const bf16_t *w;    // [cout_p][27 * cin_p]
  const float *bias;  // [cout_p] or null
  bf16_t *out, *out2; // [n][cout_p]
  const bf16_t *aux;  // [n][cout_p]: skip addend or activation
  float *P;           // EPI_P output
  const float *thick; // EPI_P: film thickness per dataset row
  const int *idx;     // EPI_P: dataset row of each sample (null: identity)
  int in_up2;         // input is the nearest-neighbour upsampling of a half grid
  int lx, ly, lz, nb; // output grid (log2) and samples
  int cin_p, cout_p;
};

struct WgradArgs {
  const bf16_t *g;    // [n][cout_p] gradient of the layer output (pre-activation)
  const bf16_t *in;   // layer input (half resolution if in_up2), cin_p channels
  float *part;        // [splits][cout_p][27 * cin_p]
  float *bpart;       // [splits][cout_p]
  int in_up2;
  int lx, ly, lz, nb;
  int cin_p, cout_p;
  int splits, chunk;  // positions per split (multiple of 32)
};

hipError_t launch_conv(int epi, const ConvArgs &a, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs &a, hipStream_t s);
void wgrad_split(long long npos, int kp, int *splits, int *chunk);

// elementwise parts
// ops: per-sample in-plane symmetry op (bits: 1 mirror x, 2 mirror y, 4 swap
// x and y on square grids), or null for none
hipError_t launch_input(const float *T, const float *thick, const float *noise, const int *idx,
                        const int *ops, int lx, int ly, int lz, int nb, int noise_div, bf16_t *x0,
                        hipStream_t s);
hipError_t launch_pool(const bf16_t *in, int lx, int ly, int lz, int nb, int c_p, bf16_t *out,
                       hipStream_t s);
hipError_t launch_pool_bwd(const bf16_t *g, const bf16_t *add, const bf16_t *a, int lx, int ly,
                           int lz, int nb, int c_p, bf16_t *out, hipStream_t s);
hipError_t launch_up_bwd(const bf16_t *g, const bf16_t *a, int lx, int ly, int lz, int nb,
                         int c_p, bf16_t *out, hipStream_t s);
hipError_t launch_loss(const float *P, const float *target, const float *thick, const int *idx,
                       const int *ops, int lx, int ly, int lz, int nb, bf16_t *gy,
                       double *partials, int *nblocks, hipStream_t s);
hipError_t launch_sum_partials(const double *partials, int n, double *out, hipStream_t s);
hipError_t launch_reduce_grad(const float *part, const float *bpart, int splits, int cin,
                              int cout, int cin_p, int cout_p, float *grad, hipStream_t s);
// Adam step number t (from 1)
hipError_t launch_adam(float *master, float *m, float *v, const float *grad, long long n,
                       double lr, double b1, double b2, double eps, long long t, hipStream_t s);
hipError_t launch_cast_weights(const float *master, int cin, int cout, int cin_p, int cout_p,
                               bf16_t *w, bf16_t *wt, float *bias, hipStream_t s);

}  // namespace tdgl_nn
