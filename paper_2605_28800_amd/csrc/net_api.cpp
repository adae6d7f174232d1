// Runtime of the initial-state proposal network: device buffers, the
// forward / backward / Adam sequence of kernel launches, and the C ABI of
// include/tdgl_net.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "net_internal.h"
#include "tdgl_net.h"

using namespace tdgl_nn;

namespace {

constexpr int NLAYER = 12;

int pad16(int c) {
  int p = 16;
  while (p < c) p <<= 1;
  return p;
}
bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

struct Layer {
  int cin, cout, cin_p, cout_p;
  int level;          // grid level of the conv's output (0 full, 1 half, 2 quarter)
  int up2;            // input read through 2x repetition
  long long off;      // offset of W in the parameter vector; bias at off + cout*27*cin
  bf16_t *w = nullptr, *wt = nullptr;
  float *bias = nullptr;
};

}  // namespace

struct tdgl_net {
  tdgl_net_cfg cfg{};
  hipStream_t s = nullptr;
  std::string err;
  int lx = 0, ly = 0, lz = 0;
  Layer L[NLAYER];
  long long nparam = 0;
  float *master = nullptr, *mom1 = nullptr, *mom2 = nullptr, *grad = nullptr;
  long long adam_t = 0;
  bool have_grad = false;
  // activations (BF16 channels-last) and gradients
  bf16_t *x0, *e0a, *e0, *p1, *e1a, *e1, *p2, *b1, *b2, *b3, *t8, *u1, *u1b, *t10, *u0, *u0b;
  bf16_t *gy, *g11, *gu0, *g10, *gq0, *g9, *gu1, *g8, *gq1, *g7, *g6, *g5, *gp2, *g4, *g3, *gp1,
      *g2, *g1;
  float *P = nullptr;
  float *part = nullptr, *bpart = nullptr;
  double *loss_part = nullptr, *loss_dev = nullptr;
  std::vector<void *> allocs;

  ~tdgl_net() {
    for (void *p : allocs) (void)hipFree(p);
  }
  int lvx(int l) const { return lx - l; }
  int lvy(int l) const { return ly - l; }
  int lvz(int l) const { return lz - l; }
  long long cells(int l) const { return 1LL << (lvx(l) + lvy(l) + lvz(l)); }
};

namespace {

tdgl_status fail(tdgl_net *n, tdgl_status st, const std::string &msg) {
  if (n) n->err = msg;
  return st;
}

tdgl_status hip_fail(tdgl_net *n, hipError_t e, const char *where) {
  return fail(n, TDGL_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

template <class T>
bool alloc(tdgl_net *n, T **p, size_t elems) {
  void *q = nullptr;
  if (hipMalloc(&q, elems * sizeof(T) > 0 ? elems * sizeof(T) : 16) != hipSuccess) return false;
  n->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return true;
}

#define CK(expr)                                          \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail(n, e_, #expr);  \
  } while (0)

// one conv launch of layer l
hipError_t conv_fwd(tdgl_net *n, int l, int nb, const bf16_t *in, int epi, bf16_t *out,
                    bf16_t *out2, const bf16_t *aux, const int *idx, const float *thick) {
  const Layer &Ly = n->L[l];
  ConvArgs a{};
  a.in = in;
  a.w = Ly.w;
  a.bias = Ly.bias;
  a.out = out;
  a.out2 = out2;
  a.aux = aux;
  a.P = n->P;
  a.thick = thick;
  a.idx = idx;
  a.in_up2 = Ly.up2;
  a.lx = n->lvx(Ly.level);
  a.ly = n->lvy(Ly.level);
  a.lz = n->lvz(Ly.level);
  a.nb = nb;
  a.cin_p = Ly.cin_p;
  a.cout_p = Ly.cout_p;
  return launch_conv(epi, a, n->s);
}

// backward-data launch of layer l: gradient g (cout_p channels) -> cin_p channels
hipError_t conv_bwd(tdgl_net *n, int l, int nb, const bf16_t *g, int epi, bf16_t *out,
                    bf16_t *out2, const bf16_t *aux) {
  const Layer &Ly = n->L[l];
  ConvArgs a{};
  a.in = g;
  a.w = Ly.wt;
  a.out = out;
  a.out2 = out2;
  a.aux = aux;
  a.lx = n->lvx(Ly.level);
  a.ly = n->lvy(Ly.level);
  a.lz = n->lvz(Ly.level);
  a.nb = nb;
  a.cin_p = Ly.cout_p;
  a.cout_p = Ly.cin_p;
  return launch_conv(epi, a, n->s);
}

hipError_t wgrad(tdgl_net *n, int l, int nb, const bf16_t *g, const bf16_t *in) {
  const Layer &Ly = n->L[l];
  WgradArgs a{};
  a.g = g;
  a.in = in;
  a.part = n->part;
  a.bpart = n->bpart;
  a.in_up2 = Ly.up2;
  a.lx = n->lvx(Ly.level);
  a.ly = n->lvy(Ly.level);
  a.lz = n->lvz(Ly.level);
  a.nb = nb;
  a.cin_p = Ly.cin_p;
  a.cout_p = Ly.cout_p;
  wgrad_split((long long)nb * n->cells(Ly.level), 27 * Ly.cin_p, &a.splits, &a.chunk);
  hipError_t e = launch_wgrad(a, n->s);
  if (e != hipSuccess) return e;
  return launch_reduce_grad(n->part, n->bpart, a.splits, Ly.cin, Ly.cout, Ly.cin_p, Ly.cout_p,
                            n->grad + Ly.off, n->s);
}

hipError_t cast_all(tdgl_net *n) {
  for (int l = 0; l < NLAYER; ++l) {
    const Layer &Ly = n->L[l];
    hipError_t e = launch_cast_weights(n->master + Ly.off, Ly.cin, Ly.cout, Ly.cin_p, Ly.cout_p,
                                       Ly.w, Ly.wt, Ly.bias, n->s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t forward(tdgl_net *n, int nb, const int *idx, const int *ops, const float *T,
                   const float *thick, const float *noise) {
  hipError_t e;
#define RUN(x) \
  if ((e = (x)) != hipSuccess) return e
  RUN(launch_input(T, thick, noise, idx, ops, n->lx, n->ly, n->lz, nb, n->cfg.noise_div, n->x0,
                   n->s));
  RUN(conv_fwd(n, 0, nb, n->x0, EPI_ACT, n->e0a, nullptr, nullptr, idx, thick));
  RUN(conv_fwd(n, 1, nb, n->e0a, EPI_ACT, n->e0, nullptr, nullptr, idx, thick));
  RUN(launch_pool(n->e0, n->lx, n->ly, n->lz, nb, n->L[1].cout_p, n->p1, n->s));
  RUN(conv_fwd(n, 2, nb, n->p1, EPI_ACT, n->e1a, nullptr, nullptr, idx, thick));
  RUN(conv_fwd(n, 3, nb, n->e1a, EPI_ACT, n->e1, nullptr, nullptr, idx, thick));
  RUN(launch_pool(n->e1, n->lx - 1, n->ly - 1, n->lz - 1, nb, n->L[3].cout_p, n->p2, n->s));
  RUN(conv_fwd(n, 4, nb, n->p2, EPI_ACT, n->b1, nullptr, nullptr, idx, thick));
  RUN(conv_fwd(n, 5, nb, n->b1, EPI_ACT, n->b2, nullptr, nullptr, idx, thick));
  RUN(conv_fwd(n, 6, nb, n->b2, EPI_ACT, n->b3, nullptr, nullptr, idx, thick));
  RUN(conv_fwd(n, 7, nb, n->b3, EPI_ACT_SKIP, n->t8, n->u1, n->e1, idx, thick));
  RUN(conv_fwd(n, 8, nb, n->u1, EPI_ACT, n->u1b, nullptr, nullptr, idx, thick));
  RUN(conv_fwd(n, 9, nb, n->u1b, EPI_ACT_SKIP, n->t10, n->u0, n->e0, idx, thick));
  RUN(conv_fwd(n, 10, nb, n->u0, EPI_ACT, n->u0b, nullptr, nullptr, idx, thick));
  RUN(conv_fwd(n, 11, nb, n->u0b, EPI_P, nullptr, nullptr, nullptr, idx, thick));
  return hipSuccess;
}

// loss into *loss_dev, gradient into n->grad
hipError_t backward(tdgl_net *n, int nb, const int *idx, const int *ops, const float *thick,
                    const float *target, double *loss_dev) {
  hipError_t e;
  int nblk = 0;
  RUN(launch_loss(n->P, target, thick, idx, ops, n->lx, n->ly, n->lz, nb, n->gy, n->loss_part,
                  &nblk, n->s));
  RUN(launch_sum_partials(n->loss_part, nblk, loss_dev, n->s));
  const int l0x = n->lx, l0y = n->ly, l0z = n->lz;
  RUN(wgrad(n, 11, nb, n->gy, n->u0b));
  RUN(conv_bwd(n, 11, nb, n->gy, EPI_RAW_D, n->g11, nullptr, n->u0b));
  RUN(wgrad(n, 10, nb, n->g11, n->u0));
  RUN(conv_bwd(n, 10, nb, n->g11, EPI_RAW_AND_D, n->gu0, n->g10, n->t10));
  RUN(wgrad(n, 9, nb, n->g10, n->u1b));
  RUN(conv_bwd(n, 9, nb, n->g10, EPI_RAW, n->gq0, nullptr, nullptr));
  RUN(launch_up_bwd(n->gq0, n->u1b, l0x, l0y, l0z, nb, n->L[9].cin_p, n->g9, n->s));
  RUN(wgrad(n, 8, nb, n->g9, n->u1));
  RUN(conv_bwd(n, 8, nb, n->g9, EPI_RAW_AND_D, n->gu1, n->g8, n->t8));
  RUN(wgrad(n, 7, nb, n->g8, n->b3));
  RUN(conv_bwd(n, 7, nb, n->g8, EPI_RAW, n->gq1, nullptr, nullptr));
  RUN(launch_up_bwd(n->gq1, n->b3, l0x - 1, l0y - 1, l0z - 1, nb, n->L[7].cin_p, n->g7, n->s));
  RUN(wgrad(n, 6, nb, n->g7, n->b2));
  RUN(conv_bwd(n, 6, nb, n->g7, EPI_RAW_D, n->g6, nullptr, n->b2));
  RUN(wgrad(n, 5, nb, n->g6, n->b1));
  RUN(conv_bwd(n, 5, nb, n->g6, EPI_RAW_D, n->g5, nullptr, n->b1));
  RUN(wgrad(n, 4, nb, n->g5, n->p2));
  RUN(conv_bwd(n, 4, nb, n->g5, EPI_RAW, n->gp2, nullptr, nullptr));
  RUN(launch_pool_bwd(n->gp2, n->gu1, n->e1, l0x - 1, l0y - 1, l0z - 1, nb, n->L[4].cin_p, n->g4,
                      n->s));
  RUN(wgrad(n, 3, nb, n->g4, n->e1a));
  RUN(conv_bwd(n, 3, nb, n->g4, EPI_RAW_D, n->g3, nullptr, n->e1a));
  RUN(wgrad(n, 2, nb, n->g3, n->p1));
  RUN(conv_bwd(n, 2, nb, n->g3, EPI_RAW, n->gp1, nullptr, nullptr));
  RUN(launch_pool_bwd(n->gp1, n->gu0, n->e0, l0x, l0y, l0z, nb, n->L[2].cin_p, n->g2, n->s));
  RUN(wgrad(n, 1, nb, n->g2, n->e0a));
  RUN(conv_bwd(n, 1, nb, n->g2, EPI_RAW_D, n->g1, nullptr, n->e0a));
  RUN(wgrad(n, 0, nb, n->g1, n->x0));
  return hipSuccess;
}

hipError_t adam_step(tdgl_net *n, double lr, double b1, double b2, double eps) {
  n->adam_t += 1;
  hipError_t e =
      launch_adam(n->master, n->mom1, n->mom2, n->grad, n->nparam, lr, b1, b2, eps, n->adam_t, n->s);
  if (e != hipSuccess) return e;
  return cast_all(n);
}
#undef RUN

tdgl_status check_batch(tdgl_net *n, int nb, const float *T, const float *thick,
                        const float *noise) {
  if (!n) return TDGL_E_ARG;
  if (nb < 1 || nb > n->cfg.max_batch)
    return fail(n, TDGL_E_ARG, "batch outside 1..max_batch");
  if (!T || !thick || !noise) return fail(n, TDGL_E_ARG, "null condition array");
  return TDGL_OK;
}

}  // namespace

extern "C" {

tdgl_status tdgl_net_create(const tdgl_net_cfg *cfg, void *hip_stream, tdgl_net **out) {
  if (!cfg || !out) return TDGL_E_ARG;
  *out = nullptr;
  const tdgl_net_cfg c = *cfg;
  if (!pow2(c.nx) || !pow2(c.ny) || !pow2(c.nz) || c.nx < 4 || c.ny < 4 || c.nz < 4 ||
      c.nx > 4096 || c.ny > 4096 || c.nz > 4096 || !pow2(c.width) || c.width < 8 ||
      c.width > 128 || !pow2(c.noise_div) || c.noise_div > c.nx || c.noise_div > c.ny ||
      c.noise_div > c.nz || c.max_batch < 1 || c.max_batch > 4096)
    return TDGL_E_ARG;
  if ((long long)c.max_batch * c.nx * c.ny * c.nz > (1LL << 31)) return TDGL_E_ARG;
  tdgl_net *n = new tdgl_net();
  n->cfg = c;
  n->s = static_cast<hipStream_t>(hip_stream);
  n->lx = ilog2(c.nx);
  n->ly = ilog2(c.ny);
  n->lz = ilog2(c.nz);
  const int w = c.width;
  const int shp[NLAYER][2] = {{5, w},         {w, w},         {w, 2 * w},     {2 * w, 2 * w},
                              {2 * w, 4 * w}, {4 * w, 4 * w}, {4 * w, 4 * w}, {4 * w, 2 * w},
                              {2 * w, 2 * w}, {2 * w, w},     {w, w},         {w, 3}};
  const int level[NLAYER] = {0, 0, 1, 1, 2, 2, 2, 1, 1, 0, 0, 0};
  long long off = 0;
  for (int l = 0; l < NLAYER; ++l) {
    Layer &Ly = n->L[l];
    Ly.cin = shp[l][0];
    Ly.cout = shp[l][1];
    Ly.cin_p = pad16(Ly.cin);
    Ly.cout_p = pad16(Ly.cout);
    Ly.level = level[l];
    Ly.up2 = (l == 7 || l == 9) ? 1 : 0;
    Ly.off = off;
    off += (long long)Ly.cout * 27 * Ly.cin + Ly.cout;
  }
  n->nparam = off;
  const size_t B = (size_t)c.max_batch;
  const size_t c0 = B * (size_t)n->cells(0), c1 = B * (size_t)n->cells(1),
               c2 = B * (size_t)n->cells(2);
  const int w0 = n->L[1].cout_p, w1 = n->L[3].cout_p, w2 = n->L[5].cout_p;
  bool ok = alloc(n, &n->master, n->nparam) && alloc(n, &n->mom1, n->nparam) &&
            alloc(n, &n->mom2, n->nparam) && alloc(n, &n->grad, n->nparam);
  for (int l = 0; ok && l < NLAYER; ++l) {
    Layer &Ly = n->L[l];
    const size_t nw = (size_t)Ly.cout_p * 27 * Ly.cin_p;
    ok = alloc(n, &Ly.w, nw) && alloc(n, &Ly.wt, nw) && alloc(n, &Ly.bias, (size_t)Ly.cout_p);
  }
  ok = ok && alloc(n, &n->x0, c0 * 16) && alloc(n, &n->e0a, c0 * w0) && alloc(n, &n->e0, c0 * w0) &&
       alloc(n, &n->p1, c1 * w0) && alloc(n, &n->e1a, c1 * w1) && alloc(n, &n->e1, c1 * w1) &&
       alloc(n, &n->p2, c2 * w1) && alloc(n, &n->b1, c2 * w2) && alloc(n, &n->b2, c2 * w2) &&
       alloc(n, &n->b3, c2 * w2) && alloc(n, &n->t8, c1 * w1) && alloc(n, &n->u1, c1 * w1) &&
       alloc(n, &n->u1b, c1 * w1) && alloc(n, &n->t10, c0 * w0) && alloc(n, &n->u0, c0 * w0) &&
       alloc(n, &n->u0b, c0 * w0) && alloc(n, &n->P, c0 * 3);
  ok = ok && alloc(n, &n->gy, c0 * 16) && alloc(n, &n->g11, c0 * w0) && alloc(n, &n->gu0, c0 * w0) &&
       alloc(n, &n->g10, c0 * w0) && alloc(n, &n->gq0, c0 * w1) && alloc(n, &n->g9, c1 * w1) &&
       alloc(n, &n->gu1, c1 * w1) && alloc(n, &n->g8, c1 * w1) && alloc(n, &n->gq1, c1 * w2) &&
       alloc(n, &n->g7, c2 * w2) && alloc(n, &n->g6, c2 * w2) && alloc(n, &n->g5, c2 * w2) &&
       alloc(n, &n->gp2, c2 * w1) && alloc(n, &n->g4, c1 * w1) && alloc(n, &n->g3, c1 * w1) &&
       alloc(n, &n->gp1, c1 * w0) && alloc(n, &n->g2, c0 * w0) && alloc(n, &n->g1, c0 * w0);
  // split-reduction buffers: the largest over the layers at max_batch
  size_t part = 0, bpart = 0;
  for (int l = 0; l < NLAYER; ++l) {
    const Layer &Ly = n->L[l];
    int sp, ch;
    wgrad_split((long long)B * n->cells(Ly.level), 27 * Ly.cin_p, &sp, &ch);
    part = std::max(part, (size_t)sp * Ly.cout_p * 27 * Ly.cin_p);
    bpart = std::max(bpart, (size_t)sp * Ly.cout_p);
  }
  const size_t lp = (c0 + 255) / 256;
  ok = ok && alloc(n, &n->part, part) && alloc(n, &n->bpart, bpart) &&
       alloc(n, &n->loss_part, lp) && alloc(n, &n->loss_dev, 4096 + 1);
  if (!ok) {
    delete n;
    return TDGL_E_NOMEM;
  }
  hipError_t e = hipMemsetAsync(n->master, 0, n->nparam * sizeof(float), n->s);
  if (e == hipSuccess) e = hipMemsetAsync(n->mom1, 0, n->nparam * sizeof(float), n->s);
  if (e == hipSuccess) e = hipMemsetAsync(n->mom2, 0, n->nparam * sizeof(float), n->s);
  if (e == hipSuccess) e = cast_all(n);
  if (e == hipSuccess) e = hipStreamSynchronize(n->s);
  if (e != hipSuccess) {
    delete n;
    return TDGL_E_HIP;
  }
  *out = n;
  return TDGL_OK;
}

void tdgl_net_destroy(tdgl_net *n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->s);
  delete n;
}

const char *tdgl_net_last_error(const tdgl_net *n) { return n ? n->err.c_str() : "null network"; }

tdgl_status tdgl_net_num_params(const tdgl_net *n, long long *np) {
  if (!n || !np) return TDGL_E_ARG;
  *np = n->nparam;
  return TDGL_OK;
}

tdgl_status tdgl_net_set_params(tdgl_net *n, const float *host, long long np) {
  if (!n || !host) return TDGL_E_ARG;
  if (np != n->nparam) return fail(n, TDGL_E_ARG, "parameter count mismatch");
  CK(hipMemcpyAsync(n->master, host, np * sizeof(float), hipMemcpyHostToDevice, n->s));
  CK(hipMemsetAsync(n->mom1, 0, np * sizeof(float), n->s));
  CK(hipMemsetAsync(n->mom2, 0, np * sizeof(float), n->s));
  CK(cast_all(n));
  CK(hipStreamSynchronize(n->s));
  n->adam_t = 0;
  n->have_grad = false;
  return TDGL_OK;
}

tdgl_status tdgl_net_get_params(tdgl_net *n, float *host, long long np) {
  if (!n || !host) return TDGL_E_ARG;
  if (np != n->nparam) return fail(n, TDGL_E_ARG, "parameter count mismatch");
  CK(hipMemcpyAsync(host, n->master, np * sizeof(float), hipMemcpyDeviceToHost, n->s));
  CK(hipStreamSynchronize(n->s));
  return TDGL_OK;
}

tdgl_status tdgl_net_forward(tdgl_net *n, int nb, const int *idx, const float *T,
                             const float *thick, const float *noise, float *P_out) {
  tdgl_status st = check_batch(n, nb, T, thick, noise);
  if (st != TDGL_OK) return st;
  CK(forward(n, nb, idx, nullptr, T, thick, noise));
  if (P_out)
    CK(hipMemcpyAsync(P_out, n->P, (size_t)nb * 3 * n->cells(0) * sizeof(float),
                      hipMemcpyDeviceToDevice, n->s));
  return TDGL_OK;
}

tdgl_status tdgl_net_loss_grad(tdgl_net *n, int nb, const int *idx, const int *ops, const float *T,
                               const float *thick, const float *noise, const float *target,
                               double *loss, float *grad_host) {
  tdgl_status st = check_batch(n, nb, T, thick, noise);
  if (st != TDGL_OK) return st;
  if (!target || !loss) return fail(n, TDGL_E_ARG, "null target or loss");
  CK(forward(n, nb, idx, ops, T, thick, noise));
  CK(backward(n, nb, idx, ops, thick, target, n->loss_dev));
  CK(hipMemcpyAsync(loss, n->loss_dev, sizeof(double), hipMemcpyDeviceToHost, n->s));
  if (grad_host)
    CK(hipMemcpyAsync(grad_host, n->grad, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->s));
  CK(hipStreamSynchronize(n->s));
  n->have_grad = true;
  if (!std::isfinite(*loss)) return fail(n, TDGL_E_NONFINITE, "non-finite loss");
  return TDGL_OK;
}

tdgl_status tdgl_net_adam(tdgl_net *n, double lr, double b1, double b2, double eps) {
  if (!n) return TDGL_E_ARG;
  if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(n, TDGL_E_ARG, "Adam hyper-parameters out of range");
  if (!n->have_grad) return fail(n, TDGL_E_STATE, "no gradient: call tdgl_net_loss_grad first");
  CK(adam_step(n, lr, b1, b2, eps));
  return TDGL_OK;
}

tdgl_status tdgl_net_train(tdgl_net *n, int nsteps, int nb, const int *idx, const int *ops,
                           const float *T, const float *thick, const float *noise,
                           const float *target, double lr, double b1, double b2, double eps,
                           double *losses_host) {
  tdgl_status st = check_batch(n, nb, T, thick, noise);
  if (st != TDGL_OK) return st;
  if (!idx || !target || nsteps < 1 || nsteps > 4096)
    return fail(n, TDGL_E_ARG, "training needs idx, target and 1..4096 steps");
  if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(n, TDGL_E_ARG, "Adam hyper-parameters out of range");
  for (int k = 0; k < nsteps; ++k) {
    const int *ik = idx + (size_t)k * nb;
    const int *ok = ops ? ops + (size_t)k * nb : nullptr;
    CK(forward(n, nb, ik, ok, T, thick, noise));
    CK(backward(n, nb, ik, ok, thick, target, n->loss_dev + k));
    CK(adam_step(n, lr, b1, b2, eps));
  }
  std::vector<double> l(nsteps);
  CK(hipMemcpyAsync(l.data(), n->loss_dev, nsteps * sizeof(double), hipMemcpyDeviceToHost, n->s));
  CK(hipStreamSynchronize(n->s));
  n->have_grad = true;
  if (losses_host) std::memcpy(losses_host, l.data(), nsteps * sizeof(double));
  for (double v : l)
    if (!std::isfinite(v)) return fail(n, TDGL_E_NONFINITE, "non-finite loss");
  return TDGL_OK;
}

tdgl_status tdgl_net_profile(tdgl_net *n, int nb, const float *T, const float *thick,
                             const float *noise, const float *target, int reps, double *ms) {
  tdgl_status st = check_batch(n, nb, T, thick, noise);
  if (st != TDGL_OK) return st;
  if (!target || !ms || reps < 1) return fail(n, TDGL_E_ARG, "profile arguments");
  // the Adam steps below work on the real buffers: save and restore them
  const size_t pb = n->nparam * sizeof(float);
  std::vector<float> keep(3 * (size_t)n->nparam);
  CK(hipMemcpyAsync(keep.data(), n->master, pb, hipMemcpyDeviceToHost, n->s));
  CK(hipMemcpyAsync(keep.data() + n->nparam, n->mom1, pb, hipMemcpyDeviceToHost, n->s));
  CK(hipMemcpyAsync(keep.data() + 2 * n->nparam, n->mom2, pb, hipMemcpyDeviceToHost, n->s));
  CK(hipStreamSynchronize(n->s));
  const long long keep_t = n->adam_t;
  hipEvent_t ev[4];
  for (auto &e : ev) CK(hipEventCreate(&e));
  double acc[3] = {0, 0, 0};
  // warm-up
  CK(forward(n, nb, nullptr, nullptr, T, thick, noise));
  CK(backward(n, nb, nullptr, nullptr, thick, target, n->loss_dev));
  for (int r = 0; r < reps; ++r) {
    CK(hipEventRecord(ev[0], n->s));
    CK(forward(n, nb, nullptr, nullptr, T, thick, noise));
    CK(hipEventRecord(ev[1], n->s));
    CK(backward(n, nb, nullptr, nullptr, thick, target, n->loss_dev));
    CK(hipEventRecord(ev[2], n->s));
    CK(adam_step(n, 1e-3, 0.9, 0.999, 1e-8));
    CK(hipEventRecord(ev[3], n->s));
    CK(hipEventSynchronize(ev[3]));
    float a, b, c;
    CK(hipEventElapsedTime(&a, ev[0], ev[1]));
    CK(hipEventElapsedTime(&b, ev[1], ev[2]));
    CK(hipEventElapsedTime(&c, ev[2], ev[3]));
    acc[0] += a;
    acc[1] += b;
    acc[2] += c;
  }
  // conv kernels alone: forward, backward-data and weight gradient of all layers
  double kc[3] = {0, 0, 0};
  for (int r = 0; r < reps; ++r) {
    CK(hipEventRecord(ev[0], n->s));
    const bf16_t *fin[NLAYER] = {n->x0, n->e0a, n->p1, n->e1a, n->p2, n->b1,
                                 n->b2, n->b3,  n->u1, n->u1b, n->u0, n->u0b};
    bf16_t *scratch_out[NLAYER] = {n->g1, n->g1, n->g3, n->g3, n->g5, n->g5,
                                   n->g5, n->g8, n->g8, n->g10, n->g10, nullptr};
    for (int l = 0; l < NLAYER - 1; ++l)
      CK(conv_fwd(n, l, nb, fin[l], EPI_ACT, scratch_out[l], nullptr, nullptr, nullptr, thick));
    CK(conv_fwd(n, 11, nb, n->u0b, EPI_P, nullptr, nullptr, nullptr, nullptr, thick));
    CK(hipEventRecord(ev[1], n->s));
    const bf16_t *gin[NLAYER] = {n->g1, n->g2, n->g3, n->g4, n->g5, n->g6,
                                 n->g7, n->g8, n->g9, n->g10, n->g11, n->gy};
    bf16_t *bout[NLAYER] = {nullptr, n->gu0, n->gp1, n->gu1, n->gp2, n->gu1,
                            n->gu1,  n->gq1, n->gu1, n->gq0, n->gu0, n->gu0};
    for (int l = 1; l < NLAYER; ++l)
      CK(conv_bwd(n, l, nb, gin[l], EPI_RAW, bout[l], nullptr, nullptr));
    CK(hipEventRecord(ev[2], n->s));
    for (int l = 0; l < NLAYER; ++l) {
      const Layer &Ly = n->L[l];
      WgradArgs a{};
      a.g = gin[l];
      a.in = fin[l];
      a.part = n->part;
      a.bpart = n->bpart;
      a.in_up2 = Ly.up2;
      a.lx = n->lvx(Ly.level);
      a.ly = n->lvy(Ly.level);
      a.lz = n->lvz(Ly.level);
      a.nb = nb;
      a.cin_p = Ly.cin_p;
      a.cout_p = Ly.cout_p;
      wgrad_split((long long)nb * n->cells(Ly.level), 27 * Ly.cin_p, &a.splits, &a.chunk);
      CK(launch_wgrad(a, n->s));
    }
    CK(hipEventRecord(ev[3], n->s));
    CK(hipEventSynchronize(ev[3]));
    float a, b, c;
    CK(hipEventElapsedTime(&a, ev[0], ev[1]));
    CK(hipEventElapsedTime(&b, ev[1], ev[2]));
    CK(hipEventElapsedTime(&c, ev[2], ev[3]));
    kc[0] += a;
    kc[1] += b;
    kc[2] += c;
  }
  for (auto &e : ev) CK(hipEventDestroy(e));
  CK(hipMemcpyAsync(n->master, keep.data(), pb, hipMemcpyHostToDevice, n->s));
  CK(hipMemcpyAsync(n->mom1, keep.data() + n->nparam, pb, hipMemcpyHostToDevice, n->s));
  CK(hipMemcpyAsync(n->mom2, keep.data() + 2 * n->nparam, pb, hipMemcpyHostToDevice, n->s));
  CK(cast_all(n));
  CK(hipStreamSynchronize(n->s));
  n->adam_t = keep_t;
  ms[0] = acc[0] / reps;
  ms[1] = acc[1] / reps;
  ms[2] = acc[2] / reps;
  ms[3] = kc[0] / reps;
  ms[4] = kc[1] / reps;
  ms[5] = kc[2] / reps;
  n->have_grad = false;
  return TDGL_OK;
}

tdgl_status tdgl_nn_conv3(int epi, const void *in, int in_up2, const void *w, const float *bias,
                          int nb, int lx, int ly, int lz, int cin_p, int cout_p, void *out,
                          void *out2, const void *aux, float *P, const float *thick,
                          void *hip_stream) {
  if (epi < EPI_ACT || epi > EPI_RAW_AND_D || lx < 0 || ly < 0 || lz < 0 || lx > 12 || ly > 12 ||
      lz > 12 || nb < 1 || ((long long)nb << (lx + ly + lz)) > (1LL << 31))
    return TDGL_E_ARG;
  ConvArgs a{};
  a.in = static_cast<const bf16_t *>(in);
  a.w = static_cast<const bf16_t *>(w);
  a.bias = bias;
  a.out = static_cast<bf16_t *>(out);
  a.out2 = static_cast<bf16_t *>(out2);
  a.aux = static_cast<const bf16_t *>(aux);
  a.P = P;
  a.thick = thick;
  a.in_up2 = in_up2 ? 1 : 0;
  a.lx = lx;
  a.ly = ly;
  a.lz = lz;
  a.nb = nb;
  a.cin_p = cin_p;
  a.cout_p = cout_p;
  hipError_t e = launch_conv(epi, a, static_cast<hipStream_t>(hip_stream));
  if (e == hipErrorInvalidValue) return TDGL_E_ARG;
  return e == hipSuccess ? TDGL_OK : TDGL_E_HIP;
}

tdgl_status tdgl_nn_wgrad_workspace(int nb, int lx, int ly, int lz, int cin_p, int cout_p,
                                    size_t *bytes) {
  if (!bytes || nb < 1 || lx < 0 || ly < 0 || lz < 0 || lx > 12 || ly > 12 || lz > 12 ||
      !pow2(cin_p) || cin_p < 16 || !pow2(cout_p) || cout_p < 16)
    return TDGL_E_ARG;
  int sp, ch;
  wgrad_split((long long)nb << (lx + ly + lz), 27 * cin_p, &sp, &ch);
  *bytes = ((size_t)sp * cout_p * 27 * cin_p + (size_t)sp * cout_p) * sizeof(float);
  return TDGL_OK;
}

tdgl_status tdgl_nn_conv3_wgrad(const void *g, const void *in, int in_up2, int nb, int lx, int ly,
                                int lz, int cin_p, int cout_p, void *workspace, size_t ws_bytes,
                                float *grad, void *hip_stream) {
  size_t need = 0;
  if (tdgl_nn_wgrad_workspace(nb, lx, ly, lz, cin_p, cout_p, &need) != TDGL_OK || !g || !in ||
      !workspace || !grad || ws_bytes < need)
    return TDGL_E_ARG;
  WgradArgs a{};
  a.g = static_cast<const bf16_t *>(g);
  a.in = static_cast<const bf16_t *>(in);
  a.in_up2 = in_up2 ? 1 : 0;
  a.lx = lx;
  a.ly = ly;
  a.lz = lz;
  a.nb = nb;
  a.cin_p = cin_p;
  a.cout_p = cout_p;
  wgrad_split((long long)nb << (lx + ly + lz), 27 * cin_p, &a.splits, &a.chunk);
  a.part = static_cast<float *>(workspace);
  a.bpart = a.part + (size_t)a.splits * cout_p * 27 * cin_p;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = launch_wgrad(a, s);
  if (e == hipSuccess)
    e = launch_reduce_grad(a.part, a.bpart, a.splits, cin_p, cout_p, cin_p, cout_p, grad, s);
  if (e == hipErrorInvalidValue) return TDGL_E_ARG;
  return e == hipSuccess ? TDGL_OK : TDGL_E_HIP;
}

}  // extern "C"
