// Kernels of the initial-state proposal network: implicit-GEMM 3x3x3
// convolutions on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), the weight gradient with an LDS transpose and split
// reduction, and the elementwise parts (input assembly, pooling, upsampling
// adjoint, loss, Adam).
//
// MFMA 16x16x32 operand layout (wave64): lane l holds A[m = l % 16][k = 8 (l / 16) + 0..7]
// and B[k = 8 (l / 16) + 0..7][n = l % 16]; the result D[m = 4 (l / 16) + i][n = l % 16],
// i = 0..3, sits in the lane's four accumulator registers.
#include "net_internal.h"

#include <cmath>

namespace tdgl_nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }
// round to nearest, ties to even (finite inputs)
__device__ inline bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ inline float act(float z) { return z > 0.f ? z : SLOPE * z; }
__device__ inline float act_slope(bf16_t y) { return bf2f(y) > 0.f ? 1.f : SLOPE; }

__device__ inline bf16x8 load8(const bf16_t *p) { return *reinterpret_cast<const bf16x8 *>(p); }
__device__ inline bf16x8 zero8() {
  bf16x8 z;
  for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.f;
  return z;
}

struct Pos {
  int b, z, y, x;
};
__device__ inline Pos decode(long long n, int lx, int ly, int lz) {
  Pos p;
  p.x = (int)(n & ((1 << lx) - 1));
  p.y = (int)((n >> lx) & ((1 << ly) - 1));
  p.z = (int)((n >> (lx + ly)) & ((1 << lz) - 1));
  p.b = (int)(n >> (lx + ly + lz));
  return p;
}

// element offset of the gathered input at (position p + tap d) of a conv
// whose output grid is (lx, ly, lz); -1 outside the grid
__device__ inline long long gather_index(const Pos &p, int dz, int dy, int dx, int lx, int ly,
                                         int lz, int up2) {
  const int z = p.z + dz, y = p.y + dy, x = p.x + dx;
  if ((unsigned)z >= (1u << lz) || (unsigned)y >= (1u << ly) || (unsigned)x >= (1u << lx))
    return -1;
  if (up2) {
    const int cx = lx - 1, cy = ly - 1, cz = lz - 1;
    return ((((long long)p.b << cz) + (z >> 1)) << (cy + cx)) + ((long long)(y >> 1) << cx) +
           (x >> 1);
  }
  return ((((long long)p.b << lz) + z) << (ly + lx)) + ((long long)y << lx) + x;
}

// ----------------------------------------------------------------- conv
// One work-group: 4 waves x 16 * NB output positions, 16 * MB output
// channels (blockIdx.y selects the channel block).  K = 27 * cin_p runs in
// steps of 32: each lane gathers 8 consecutive input channels of one tap
// for each of its NB position columns, and 8 consecutive weights per 16-row
// block; the operands of step k + 1 are loaded while step k's MFMAs run.
template <int MB, int NB>
__device__ __forceinline__ void conv_operands(const ConvArgs &a, const bf16_t *wrow, int kp,
                                              int lc, int k0, int kq, const Pos *p,
                                              const bool *inb, bf16x8 *av, bf16x8 *bv) {
  const int k = k0 + 8 * kq;
  const bool kv = k < kp;
  const int t = k >> lc, ci = k & (a.cin_p - 1);
  const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  for (int mb = 0; mb < MB; ++mb) av[mb] = kv ? load8(wrow + (size_t)mb * 16 * kp + k) : zero8();
  for (int j = 0; j < NB; ++j) {
    long long src = -1;
    if (kv && inb[j]) src = gather_index(p[j], dz, dy, dx, a.lx, a.ly, a.lz, a.in_up2);
    bv[j] = src >= 0 ? load8(a.in + src * a.cin_p + ci) : zero8();
  }
}

// epilogue of one lane: channels co0 .. co0 + 3 of output position n (p its
// coordinates; ls = log2 of the cells per sample)
template <int EPI>
__device__ __forceinline__ void conv_store(const ConvArgs &a, const Pos &p, long long n, int ls,
                                           int co0, const floatx4 v) {
  const size_t o = (size_t)n * a.cout_p + co0;
  if (EPI == EPI_P) {
    if (co0 != 0) return;
    const int row = a.idx ? a.idx[p.b] : p.b;
    const float m = (float)p.z < a.thick[row] ? 1.f : 0.f;
    const long long r = n & ((1LL << ls) - 1);
    for (int c = 0; c < 3; ++c) a.P[(((long long)p.b * 3 + c) << ls) + r] = m * (v[c] + a.bias[c]);
    return;
  }
  bf16_t r4[4], s4[4];
  if (EPI == EPI_ACT || EPI == EPI_ACT_SKIP) {
    for (int i = 0; i < 4; ++i) r4[i] = f2bf(act(v[i] + a.bias[co0 + i]));
  } else {
    for (int i = 0; i < 4; ++i) r4[i] = f2bf(v[i]);
  }
  if (EPI == EPI_ACT_SKIP || EPI == EPI_RAW_D || EPI == EPI_RAW_AND_D) {
    const uint2 ax = *reinterpret_cast<const uint2 *>(a.aux + o);
    const bf16_t xa[4] = {(bf16_t)(ax.x & 0xFFFF), (bf16_t)(ax.x >> 16), (bf16_t)(ax.y & 0xFFFF),
                          (bf16_t)(ax.y >> 16)};
    for (int i = 0; i < 4; ++i)
      s4[i] = EPI == EPI_ACT_SKIP ? f2bf(bf2f(r4[i]) + bf2f(xa[i])) : f2bf(v[i] * act_slope(xa[i]));
  }
  uint2 w0, w1;
  w0.x = r4[0] | ((uint32_t)r4[1] << 16);
  w0.y = r4[2] | ((uint32_t)r4[3] << 16);
  w1.x = s4[0] | ((uint32_t)s4[1] << 16);
  w1.y = s4[2] | ((uint32_t)s4[3] << 16);
  if (EPI == EPI_RAW_D) {
    *reinterpret_cast<uint2 *>(a.out + o) = w1;
    return;
  }
  *reinterpret_cast<uint2 *>(a.out + o) = w0;
  if (EPI == EPI_ACT_SKIP || EPI == EPI_RAW_AND_D) *reinterpret_cast<uint2 *>(a.out2 + o) = w1;
}

template <int MB, int NB, int EPI>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, col = lane & 15;
  const int ls = a.lx + a.ly + a.lz;
  const long long npos = (long long)a.nb << ls;
  const int kp = 27 * a.cin_p;
  const int lc = __builtin_ctz(a.cin_p);
  const int co_blk = blockIdx.y * MB * 16;
  const long long nbase = ((long long)blockIdx.x * 4 + wave) * (16 * NB);

  Pos p[NB];
  bool inb[NB];
  for (int j = 0; j < NB; ++j) {
    const long long n = nbase + 16 * j + col;
    inb[j] = n < npos;
    p[j] = decode(inb[j] ? n : 0, a.lx, a.ly, a.lz);
  }

  floatx4 acc[MB][NB];
  for (int mb = 0; mb < MB; ++mb)
    for (int j = 0; j < NB; ++j) acc[mb][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const bf16_t *wrow = a.w + (size_t)(co_blk + col) * kp;
  bf16x8 av[MB], bv[NB];
  conv_operands<MB, NB>(a, wrow, kp, lc, 0, kq, p, inb, av, bv);
  for (int k0 = 0; k0 < kp; k0 += 32) {
    bf16x8 an[MB], bn[NB];
    if (k0 + 32 < kp) conv_operands<MB, NB>(a, wrow, kp, lc, k0 + 32, kq, p, inb, an, bn);
    for (int mb = 0; mb < MB; ++mb)
      for (int j = 0; j < NB; ++j)
        acc[mb][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mb], bv[j], acc[mb][j], 0, 0, 0);
    for (int mb = 0; mb < MB; ++mb) av[mb] = an[mb];
    for (int j = 0; j < NB; ++j) bv[j] = bn[j];
  }

  // epilogue: this lane holds channels co0 .. co0 + 3 of position n
  for (int j = 0; j < NB; ++j) {
    if (!inb[j]) continue;
    const long long n = nbase + 16 * j + col;
    for (int mb = 0; mb < MB; ++mb)
      conv_store<EPI>(a, p[j], n, ls, co_blk + mb * 16 + 4 * kq, acc[mb][j]);
  }
}

// LDS-tiled variant for grids with X >= 16, Y >= NR and Z >= 4: a
// work-group owns a 4 x NR x 16 (z, y, x) block, wave w the NR rows of
// plane w; per chunk of CC input channels the 6 x (NR + 2) x 18 input halo
// of the block is staged in LDS once, and all 27 taps read their operand
// from there.  MB * NR = 16 accumulator tiles per wave (NR >= 2).
constexpr int HX = 18;

template <int MB, int NR, int CC, int EPI>
__global__ __launch_bounds__(256) void k_conv_tile(ConvArgs a) {
  constexpr int HY = NR + 2, HZ = 6, HPOS = HZ * HY * HX;
  constexpr int LD = CC + 8;                       // LDS row stride (elements)
  extern __shared__ bf16_t halo[];                 // [HPOS][LD]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = lane >> 4, col = lane & 15;
  const int X = 1 << a.lx, Y = 1 << a.ly, Z = 1 << a.lz;
  const int tx_n = X >> 4, ty_n = Y / NR, tz_n = Z >> 2;
  const int per_b = tx_n * ty_n * tz_n;
  const int b = blockIdx.x / per_b;
  int rem = blockIdx.x % per_b;
  const int z0 = (rem / (tx_n * ty_n)) * 4;
  rem %= tx_n * ty_n;
  const int y0 = (rem / tx_n) * NR, x0 = (rem % tx_n) * 16;
  const int kp = 27 * a.cin_p;
  const int co_blk = blockIdx.y * MB * 16;

  floatx4 acc[MB][NR];
  for (int mb = 0; mb < MB; ++mb)
    for (int j = 0; j < NR; ++j) acc[mb][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const bf16_t *wrow = a.w + (size_t)(co_blk + col) * kp;

  for (int ci0 = 0; ci0 < a.cin_p; ci0 += CC) {
    for (int h = tid; h < HPOS * (CC / 8); h += 256) {
      const int pos = h / (CC / 8), c8 = h % (CC / 8);
      Pos hp;
      hp.b = b;
      hp.z = z0 - 1 + pos / (HY * HX);
      hp.y = y0 - 1 + (pos / HX) % HY;
      hp.x = x0 - 1 + pos % HX;
      const long long src = gather_index(hp, 0, 0, 0, a.lx, a.ly, a.lz, a.in_up2);
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (src >= 0) v = *reinterpret_cast<const uint4 *>(a.in + src * a.cin_p + ci0 + 8 * c8);
      *reinterpret_cast<uint4 *>(halo + pos * LD + 8 * c8) = v;
    }
    __syncthreads();
    // K within the chunk: kk = tap * CC + c, steps of 32
    for (int kk0 = 0; kk0 < 27 * CC; kk0 += 32) {
      const int kk = kk0 + 8 * kq;
      const bool kv = kk < 27 * CC;
      const int t = kv ? kk / CC : 0, c = kk % CC;
      const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;   // 0..2: halo offsets
      bf16x8 av[MB];
      for (int mb = 0; mb < MB; ++mb)
        av[mb] = kv ? load8(wrow + (size_t)mb * 16 * kp + t * a.cin_p + ci0 + c) : zero8();
      const bf16_t *hb = halo + (((wave + dz) * HY + dy) * HX + col + dx) * LD + c;
      for (int j = 0; j < NR; ++j) {
        const bf16x8 bv = kv ? *reinterpret_cast<const bf16x8 *>(hb + j * HX * LD) : zero8();
        for (int mb = 0; mb < MB; ++mb)
          acc[mb][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mb], bv, acc[mb][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  const int ls = a.lx + a.ly + a.lz;
  for (int j = 0; j < NR; ++j) {
    Pos pj;
    pj.b = b;
    pj.z = z0 + wave;
    pj.y = y0 + j;
    pj.x = x0 + col;
    const long long n = ((((long long)b << a.lz) + pj.z) * Y + pj.y) * (long long)X + pj.x;
    for (int mb = 0; mb < MB; ++mb)
      conv_store<EPI>(a, pj, n, ls, co_blk + mb * 16 + 4 * kq, acc[mb][j]);
  }
}

template <int MB, int EPI>
static hipError_t conv_tile(const ConvArgs &a, dim3 grid, hipStream_t s) {
  // rows per wave NR = 16 / MB (2..8); channel chunk of 16 per halo load:
  // 6 x (NR + 2) x 18 positions x 24 elements x 2 B (<= 52 KB)
  constexpr int NR = MB >= 8 ? 2 : 16 / MB > 8 ? 8 : 16 / MB;
  const size_t shm = (size_t)6 * (NR + 2) * HX * 24 * 2;
  hipLaunchKernelGGL((k_conv_tile<MB, NR, 16, EPI>), grid, dim3(256), shm, s, a);
  return hipGetLastError();
}

// positions per wave: 16 * NB with MB * NB = 16 accumulator tiles (NB >= 2)
template <int EPI>
static hipError_t conv_mb(const ConvArgs &a, long long npos, hipStream_t s) {
  const int mb = a.cout_p / 16 >= 8 ? 8 : a.cout_p / 16;
  const int nr = mb >= 8 ? 2 : 16 / mb > 8 ? 8 : 16 / mb;
  if (a.lx >= 4 && (1 << a.ly) >= nr && a.lz >= 2) {
    const long long blocks = npos / (64LL * nr);
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks, a.cout_p / (16 * mb), 1);
    switch (mb) {
      case 1: return conv_tile<1, EPI>(a, grid, s);
      case 2: return conv_tile<2, EPI>(a, grid, s);
      case 4: return conv_tile<4, EPI>(a, grid, s);
      case 8: return conv_tile<8, EPI>(a, grid, s);
      default: return hipErrorInvalidValue;
    }
  }
  const int nbk = mb >= 8 ? 2 : 16 / mb > 8 ? 8 : 16 / mb;
  const long long blocks = (npos + 64 * nbk - 1) / (64 * nbk);
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  dim3 grid((unsigned)blocks, a.cout_p / (16 * mb), 1);
  switch (mb) {
    case 1: hipLaunchKernelGGL((k_conv<1, 8, EPI>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_conv<2, 8, EPI>), grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_conv<4, 4, EPI>), grid, dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_conv<8, 2, EPI>), grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

hipError_t launch_conv(int epi, const ConvArgs &a, hipStream_t s) {
  if (!pow2(a.cin_p) || a.cin_p < 16 || !pow2(a.cout_p) || a.cout_p < 16 || a.nb < 1 ||
      a.lx < 0 || a.ly < 0 || a.lz < 0 || (a.in_up2 && (a.lx < 1 || a.ly < 1 || a.lz < 1)) ||
      a.cout_p / 16 > 8 * 65535)
    return hipErrorInvalidValue;
  if (!a.in || !a.w || (epi != EPI_P && !a.out)) return hipErrorInvalidValue;
  if (epi == EPI_P && (a.cout_p != 16 || !a.P || !a.thick || !a.bias))
    return hipErrorInvalidValue;
  if ((epi == EPI_ACT || epi == EPI_ACT_SKIP) && !a.bias) return hipErrorInvalidValue;
  if ((epi == EPI_ACT_SKIP || epi == EPI_RAW_AND_D) && !a.out2) return hipErrorInvalidValue;
  if ((epi == EPI_ACT_SKIP || epi == EPI_RAW_D || epi == EPI_RAW_AND_D) && !a.aux)
    return hipErrorInvalidValue;
  const long long npos = (long long)a.nb << (a.lx + a.ly + a.lz);
  switch (epi) {
    case EPI_ACT: return conv_mb<EPI_ACT>(a, npos, s);
    case EPI_ACT_SKIP: return conv_mb<EPI_ACT_SKIP>(a, npos, s);
    case EPI_P: return conv_mb<EPI_P>(a, npos, s);
    case EPI_RAW: return conv_mb<EPI_RAW>(a, npos, s);
    case EPI_RAW_D: return conv_mb<EPI_RAW_D>(a, npos, s);
    case EPI_RAW_AND_D: return conv_mb<EPI_RAW_AND_D>(a, npos, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------- weight grad
// dW[co][k] = sum_n G[n][co] X[n][k] over one split's positions, k = tap * cin_p + ci.
// Work-group: 16 * MB output channels (blockIdx.z) x 64 k columns
// (blockIdx.x, 16 per wave), positions in slabs of 32 * WS.  Both tiles are
// transposed through LDS so that each lane reads 8 consecutive positions for
// the matrix core.  The blockIdx.x == 0 groups also sum G over the
// positions (bias gradient).
constexpr int WS = 4;                  // 32-position MFMA steps per LDS slab
constexpr int WG_LD = 32 * WS + 8;     // LDS row stride (elements)

template <int MB>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  __shared__ bf16_t gs[MB * 16][WG_LD];
  __shared__ bf16_t xs[64][WG_LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = lane >> 4, col = lane & 15;
  const int ls = a.lx + a.ly + a.lz;
  const long long npos = (long long)a.nb << ls;
  const int kp = 27 * a.cin_p;
  const int lc = __builtin_ctz(a.cin_p);
  const int kt0 = blockIdx.x * 64;
  const int co_blk = blockIdx.z * MB * 16;
  const long long p0 = (long long)blockIdx.y * a.chunk;
  const long long p1 = p0 + a.chunk < npos ? p0 + a.chunk : npos;
  const bool bias_thread = blockIdx.x == 0 && tid < MB * 16;

  floatx4 acc[MB];
  for (int mb = 0; mb < MB; ++mb) acc[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;

  for (long long pb = p0; pb < p1; pb += 32 * WS) {
    for (int c = tid; c < MB * 64 * WS; c += 256) {
      const int gl = c % (32 * WS), c8 = c / (32 * WS);
      const long long n = pb + gl;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (n < p1) v = *reinterpret_cast<const uint4 *>(a.g + n * a.cout_p + co_blk + 8 * c8);
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
      for (int i = 0; i < 4; ++i) {
        gs[8 * c8 + 2 * i][gl] = (bf16_t)(w4[i] & 0xFFFF);
        gs[8 * c8 + 2 * i + 1][gl] = (bf16_t)(w4[i] >> 16);
      }
    }
    for (int c = tid; c < 256 * WS; c += 256) {
      const int nl = c % (32 * WS), k8 = c / (32 * WS);
      const int kx = kt0 + 8 * k8;
      const long long n = pb + nl;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (kx < kp && n < p1) {
        const int t = kx >> lc, ci = kx & (a.cin_p - 1);
        const Pos p = decode(n, a.lx, a.ly, a.lz);
        const long long src =
            gather_index(p, t / 9 - 1, (t / 3) % 3 - 1, t % 3 - 1, a.lx, a.ly, a.lz, a.in_up2);
        if (src >= 0) v = *reinterpret_cast<const uint4 *>(a.in + src * a.cin_p + ci);
      }
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
      for (int i = 0; i < 4; ++i) {
        xs[8 * k8 + 2 * i][nl] = (bf16_t)(w4[i] & 0xFFFF);
        xs[8 * k8 + 2 * i + 1][nl] = (bf16_t)(w4[i] >> 16);
      }
    }
    __syncthreads();
    for (int st = 0; st < WS; ++st) {
      const int n8 = 32 * st + 8 * kq;
      const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&xs[wave * 16 + col][n8]);
      for (int mb = 0; mb < MB; ++mb) {
        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&gs[mb * 16 + col][n8]);
        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[mb], 0, 0, 0);
      }
    }
    if (bias_thread)
      for (int i = 0; i < 32 * WS; ++i) bsum += bf2f(gs[tid][i]);
    __syncthreads();
  }
  const int k = kt0 + wave * 16 + col;
  if (k < kp) {
    for (int mb = 0; mb < MB; ++mb)
      for (int i = 0; i < 4; ++i) {
        const int co = co_blk + mb * 16 + 4 * kq + i;
        a.part[((size_t)blockIdx.y * a.cout_p + co) * kp + k] = acc[mb][i];
      }
  }
  if (bias_thread) a.bpart[(size_t)blockIdx.y * a.cout_p + co_blk + tid] = bsum;
}

void wgrad_split(long long npos, int kp, int *splits, int *chunk) {
  const long long ktiles = (kp + 63) / 64;
  long long s = (1024 + ktiles - 1) / ktiles;           // aim at ~1024 work-groups
  const long long smax = (npos + 255) / 256;            // at least 256 positions each
  if (s > smax) s = smax;
  if (s < 1) s = 1;
  long long c = (npos + s - 1) / s;
  c = (c + 32 * WS - 1) / (32 * WS) * (32 * WS);   // whole LDS slabs
  s = (npos + c - 1) / c;
  *splits = (int)s;
  *chunk = (int)c;
}

hipError_t launch_wgrad(const WgradArgs &a, hipStream_t s) {
  if (!pow2(a.cin_p) || a.cin_p < 16 || !pow2(a.cout_p) || a.cout_p < 16 || a.nb < 1 ||
      a.splits < 1 || a.chunk < 32 || (a.chunk & 31) || a.splits > 65535 ||
      (a.in_up2 && (a.lx < 1 || a.ly < 1 || a.lz < 1)))
    return hipErrorInvalidValue;
  const int kp = 27 * a.cin_p;
  const int mb = a.cout_p / 16 >= 8 ? 8 : a.cout_p / 16;
  dim3 grid((kp + 63) / 64, a.splits, a.cout_p / (16 * mb));
  switch (mb) {
    case 1: hipLaunchKernelGGL(k_wgrad<1>, grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_wgrad<2>, grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_wgrad<4>, grid, dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_wgrad<8>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ elementwise
// In-plane symmetry op of a sample (bits: 1 mirror x, 2 mirror y, 4 swap x
// and y; swap only on square grids): the sample's vector fields F become
// F'(x, y) = D F(src(x, y)) with src = swap(mirror_x(mirror_y(x, y))) and
// F'_x = (-1)^mx F_(swap ? y : x), F'_y = (-1)^my F_(swap ? x : y), F'_z = F_z.
struct SymOp {
  int mx, my, sw;
  __device__ explicit SymOp(int op) : mx(op & 1), my((op >> 1) & 1), sw((op >> 2) & 1) {}
  // source (x, y) of destination (x, y) on an X x Y grid
  __device__ void src(int &x, int &y, int X, int Y) const {
    if (my) y = Y - 1 - y;
    if (mx) x = X - 1 - x;
    if (sw) {
      const int t = x;
      x = y;
      y = t;
    }
  }
  // source component and sign of destination component c
  __device__ int comp(int c) const { return (sw && c < 2) ? 1 - c : c; }
  __device__ float sign(int c) const { return (c == 0 && mx) || (c == 1 && my) ? -1.f : 1.f; }
};

__global__ void k_input(const float *T, const float *thick, const float *noise, const int *idx,
                        const int *ops, int lx, int ly, int lz, int nb, int ld, bf16_t *x0) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ls = lx + ly + lz;
  if (n >= ((long long)nb << ls)) return;
  const Pos p = decode(n, lx, ly, lz);
  const int row = idx ? idx[p.b] : p.b;
  const float m = (float)p.z < thick[row] ? 1.f : 0.f;
  const int cx = lx - ld, cy = ly - ld, cz = lz - ld;
  const SymOp g(ops ? ops[p.b] & (lx == ly ? 7 : 3) : 0);
  int qx = p.x >> ld, qy = p.y >> ld;
  g.src(qx, qy, 1 << cx, 1 << cy);
  const long long cell = (((long long)(p.z >> ld) << cy) + qy) * (1LL << cx) + qx;
  const long long nc = 1LL << (cx + cy + cz);
  float v[16];
  for (int c = 0; c < 16; ++c) v[c] = 0.f;
  v[0] = m * ((T[row] - 350.f) / 100.f);
  v[1] = m;
  for (int c = 0; c < 3; ++c)
    v[2 + c] = m * (g.sign(c) * noise[((long long)row * 3 + g.comp(c)) * nc + cell] * 10.f);
  uint32_t w[8];
  for (int i = 0; i < 8; ++i) w[i] = f2bf(v[2 * i]) | ((uint32_t)f2bf(v[2 * i + 1]) << 16);
  uint4 *o = reinterpret_cast<uint4 *>(x0 + n * 16);
  o[0] = make_uint4(w[0], w[1], w[2], w[3]);
  o[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

hipError_t launch_input(const float *T, const float *thick, const float *noise, const int *idx,
                        const int *ops, int lx, int ly, int lz, int nb, int noise_div, bf16_t *x0,
                        hipStream_t s) {
  if (!pow2(noise_div)) return hipErrorInvalidValue;
  const int ld = __builtin_ctz(noise_div);
  if (ld > lx || ld > ly || ld > lz) return hipErrorInvalidValue;
  const long long n = (long long)nb << (lx + ly + lz);
  hipLaunchKernelGGL(k_input, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, thick, noise,
                     idx, ops, lx, ly, lz, nb, ld, x0);
  return hipGetLastError();
}

__device__ inline void unpack8(const uint4 v, float *f) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  for (int i = 0; i < 4; ++i) {
    f[2 * i] = bf2f((bf16_t)(w[i] & 0xFFFF));
    f[2 * i + 1] = bf2f((bf16_t)(w[i] >> 16));
  }
}
__device__ inline uint4 pack8(const float *f) {
  uint32_t w[4];
  for (int i = 0; i < 4; ++i) w[i] = f2bf(f[2 * i]) | ((uint32_t)f2bf(f[2 * i + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}
__device__ inline void unpack8_raw(const uint4 v, bf16_t *h) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  for (int i = 0; i < 4; ++i) {
    h[2 * i] = (bf16_t)(w[i] & 0xFFFF);
    h[2 * i + 1] = (bf16_t)(w[i] >> 16);
  }
}

// fine position of child c (0..7) of coarse position q; (lx, ly, lz) fine grid
__device__ inline long long child(const Pos &q, int c, int lx, int ly, int lz) {
  const int z = 2 * q.z + (c >> 2), y = 2 * q.y + ((c >> 1) & 1), x = 2 * q.x + (c & 1);
  return ((((long long)q.b << lz) + z) << (ly + lx)) + ((long long)y << lx) + x;
}

// coarse average of 2x2x2 blocks; (lx, ly, lz) is the fine grid
__global__ void k_pool(const bf16_t *in, int lx, int ly, int lz, int nb, int c8, bf16_t *out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int cls = lx + ly + lz - 3;
  if (i >= ((long long)nb << cls) * c8) return;
  const long long q = i / c8;
  const int ch = (int)(i % c8) * 8;
  const Pos cp = decode(q, lx - 1, ly - 1, lz - 1);
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < 8; ++c) {
    float f[8];
    unpack8(*reinterpret_cast<const uint4 *>(in + child(cp, c, lx, ly, lz) * (8 * c8) + ch), f);
    for (int k = 0; k < 8; ++k) s[k] += f[k];
  }
  for (int k = 0; k < 8; ++k) s[k] *= 0.125f;
  *reinterpret_cast<uint4 *>(out + q * (8 * c8) + ch) = pack8(s);
}

// out[fine] = (g[coarse] / 8 + add[fine]) * act'(a[fine])
__global__ void k_pool_bwd(const bf16_t *g, const bf16_t *add, const bf16_t *a, int lx, int ly,
                           int lz, int nb, int c8, bf16_t *out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ls = lx + ly + lz;
  if (i >= ((long long)nb << ls) * c8) return;
  const long long n = i / c8;
  const int ch = (int)(i % c8) * 8;
  const Pos p = decode(n, lx, ly, lz);
  const long long q = ((((long long)p.b << (lz - 1)) + (p.z >> 1)) << (ly - 1 + lx - 1)) +
                      ((long long)(p.y >> 1) << (lx - 1)) + (p.x >> 1);
  const int C = 8 * c8;
  float gv[8], av[8];
  bf16_t ah[8];
  unpack8(*reinterpret_cast<const uint4 *>(g + q * C + ch), gv);
  if (add) unpack8(*reinterpret_cast<const uint4 *>(add + n * C + ch), av);
  unpack8_raw(*reinterpret_cast<const uint4 *>(a + n * C + ch), ah);
  float r[8];
  for (int k = 0; k < 8; ++k) r[k] = (gv[k] * 0.125f + (add ? av[k] : 0.f)) * act_slope(ah[k]);
  *reinterpret_cast<uint4 *>(out + n * C + ch) = pack8(r);
}

// out[coarse] = (sum of g over the 8 children) * act'(a[coarse]); (lx, ly, lz) fine grid
__global__ void k_up_bwd(const bf16_t *g, const bf16_t *a, int lx, int ly, int lz, int nb, int c8,
                         bf16_t *out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int cls = lx + ly + lz - 3;
  if (i >= ((long long)nb << cls) * c8) return;
  const long long q = i / c8;
  const int ch = (int)(i % c8) * 8;
  const int C = 8 * c8;
  const Pos cp = decode(q, lx - 1, ly - 1, lz - 1);
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < 8; ++c) {
    float f[8];
    unpack8(*reinterpret_cast<const uint4 *>(g + child(cp, c, lx, ly, lz) * C + ch), f);
    for (int k = 0; k < 8; ++k) s[k] += f[k];
  }
  bf16_t ah[8];
  unpack8_raw(*reinterpret_cast<const uint4 *>(a + q * C + ch), ah);
  for (int k = 0; k < 8; ++k) s[k] *= act_slope(ah[k]);
  *reinterpret_cast<uint4 *>(out + q * C + ch) = pack8(s);
}

static hipError_t ew_check(int lx, int ly, int lz, int nb, int c_p, bool coarse) {
  if (c_p < 8 || (c_p & 7) || nb < 1 || (coarse && (lx < 1 || ly < 1 || lz < 1)))
    return hipErrorInvalidValue;
  return hipSuccess;
}

hipError_t launch_pool(const bf16_t *in, int lx, int ly, int lz, int nb, int c_p, bf16_t *out,
                       hipStream_t s) {
  if (ew_check(lx, ly, lz, nb, c_p, true) != hipSuccess) return hipErrorInvalidValue;
  const long long n = ((long long)nb << (lx + ly + lz - 3)) * (c_p / 8);
  hipLaunchKernelGGL(k_pool, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, lx, ly, lz,
                     nb, c_p / 8, out);
  return hipGetLastError();
}

hipError_t launch_pool_bwd(const bf16_t *g, const bf16_t *add, const bf16_t *a, int lx, int ly,
                           int lz, int nb, int c_p, bf16_t *out, hipStream_t s) {
  if (ew_check(lx, ly, lz, nb, c_p, true) != hipSuccess) return hipErrorInvalidValue;
  const long long n = ((long long)nb << (lx + ly + lz)) * (c_p / 8);
  hipLaunchKernelGGL(k_pool_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, add, a,
                     lx, ly, lz, nb, c_p / 8, out);
  return hipGetLastError();
}

hipError_t launch_up_bwd(const bf16_t *g, const bf16_t *a, int lx, int ly, int lz, int nb,
                         int c_p, bf16_t *out, hipStream_t s) {
  if (ew_check(lx, ly, lz, nb, c_p, true) != hipSuccess) return hipErrorInvalidValue;
  const long long n = ((long long)nb << (lx + ly + lz - 3)) * (c_p / 8);
  hipLaunchKernelGGL(k_up_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, a, lx, ly,
                     lz, nb, c_p / 8, out);
  return hipGetLastError();
}

// squared error of P against the target rows over the film cells, divided by
// 3 x the film cells of the batch (FP64 partial per block), and the BF16
// gradient 2 m (P - target) / count in channels 0..2 of 16
__global__ __launch_bounds__(256) void k_loss(const float *P, const float *target,
                                              const float *thick, const int *idx, const int *ops,
                                              int lx, int ly, int lz, int nb, bf16_t *gy,
                                              double *partials) {
  __shared__ double red[4];
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  const int ls = lx + ly + lz;
  // 3 x the film cells of the batch
  double count = 0.0;
  for (int b = 0; b < nb; ++b) {
    const float th = thick[idx ? idx[b] : b];
    const float layers = ceilf(fminf(fmaxf(th, 0.f), (float)(1 << lz)));
    count += 3.0 * (double)layers * (double)(1LL << (lx + ly));
  }
  const double inv_count = count > 0.0 ? 1.0 / count : 0.0;
  double e = 0.0;
  if (n < ((long long)nb << ls)) {
    const Pos p = decode(n, lx, ly, lz);
    const int row = idx ? idx[p.b] : p.b;
    const float m = (float)p.z < thick[row] ? 1.f : 0.f;
    const long long r = n & ((1LL << ls) - 1);
    // the target is read through the sample's symmetry op
    const SymOp op(ops ? ops[p.b] & (lx == ly ? 7 : 3) : 0);
    int sx = p.x, sy = p.y;
    op.src(sx, sy, 1 << lx, 1 << ly);
    const long long rs = ((long long)p.z << (lx + ly)) + ((long long)sy << lx) + sx;
    float g[16];
    for (int c = 0; c < 16; ++c) g[c] = 0.f;
    for (int c = 0; c < 3; ++c) {
      const double d = (double)P[(((long long)p.b * 3 + c) << ls) + r] -
                       (double)op.sign(c) *
                           (double)target[(((long long)row * 3 + op.comp(c)) << ls) + rs];
      e += m * d * d;
      g[c] = (float)(m * 2.0 * d * inv_count);
    }
    uint32_t w[8];
    for (int i = 0; i < 8; ++i) w[i] = f2bf(g[2 * i]) | ((uint32_t)f2bf(g[2 * i + 1]) << 16);
    uint4 *o = reinterpret_cast<uint4 *>(gy + n * 16);
    o[0] = make_uint4(w[0], w[1], w[2], w[3]);
    o[1] = make_uint4(w[4], w[5], w[6], w[7]);
  }
  for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * inv_count;
}

hipError_t launch_loss(const float *P, const float *target, const float *thick, const int *idx,
                       const int *ops, int lx, int ly, int lz, int nb, bf16_t *gy,
                       double *partials, int *nblocks, hipStream_t s) {
  const long long n = (long long)nb << (lx + ly + lz);
  const long long nbk = (n + 255) / 256;
  if (nb < 1 || nbk > 0x7FFFFFFF) return hipErrorInvalidValue;
  *nblocks = (int)nbk;
  hipLaunchKernelGGL(k_loss, dim3((unsigned)nbk), dim3(256), 0, s, P, target, thick, idx, ops, lx,
                     ly, lz, nb, gy, partials);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sum_partials(const double *p, int n, double *out) {
  __shared__ double red[4];
  double e = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) e += p[i];
  for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_sum_partials(const double *partials, int n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, n, out);
  return hipGetLastError();
}

// flat gradient of one layer (public order: W [cout][27][cin], then b [cout])
__global__ void k_reduce_grad(const float *part, const float *bpart, int splits, int cin,
                              int cout, int cin_p, int cout_p, float *grad) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nw = (long long)cout * 27 * cin;
  if (i >= nw + cout) return;
  float s = 0.f;
  if (i < nw) {
    const int ci = (int)(i % cin);
    const int t = (int)((i / cin) % 27);
    const int co = (int)(i / (27LL * cin));
    const size_t kp = 27 * (size_t)cin_p;
    for (int sp = 0; sp < splits; ++sp)
      s += part[((size_t)sp * cout_p + co) * kp + (size_t)t * cin_p + ci];
  } else {
    const int co = (int)(i - nw);
    for (int sp = 0; sp < splits; ++sp) s += bpart[(size_t)sp * cout_p + co];
  }
  grad[i] = s;
}

hipError_t launch_reduce_grad(const float *part, const float *bpart, int splits, int cin,
                              int cout, int cin_p, int cout_p, float *grad, hipStream_t s) {
  const long long n = (long long)cout * 27 * cin + cout;
  hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part,
                     bpart, splits, cin, cout, cin_p, cout_p, grad);
  return hipGetLastError();
}

// omb1 = 1 - beta1, omb2 = 1 - beta2 and the bias corrections c1, c2 come
// from the host in FP64, so that the first step's m / c1 and v / c2 are g and
// g^2 to within a rounding
__global__ void k_adam(float *master, float *m, float *v, const float *grad, long long n,
                       float lr, float b1, float b2, float omb1, float omb2, float eps, float c1,
                       float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + omb1 * g;
  const float vi = b2 * v[i] + omb2 * g * g;
  m[i] = mi;
  v[i] = vi;
  master[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float *master, float *m, float *v, const float *grad, long long n,
                       double lr, double b1, double b2, double eps, long long t, hipStream_t s) {
  const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, master, m, v,
                     grad, n, (float)lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2),
                     (float)eps, (float)c1, (float)c2);
  return hipGetLastError();
}

// FP32 master (one layer, public order) -> BF16 forward [cout_p][27 cin_p],
// mirrored backward-data copy [cin_p][27 cout_p] and the padded FP32 bias
__global__ void k_cast_weights(const float *master, int cin, int cout, int cin_p, int cout_p,
                               bf16_t *w, bf16_t *wt, float *bias) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nw = (long long)cout_p * 27 * cin_p;
  if (i < nw) {
    const int ci = (int)(i % cin_p);
    const int t = (int)((i / cin_p) % 27);
    const int co = (int)(i / (27LL * cin_p));
    const float val = (co < cout && ci < cin) ? master[((long long)co * 27 + t) * cin + ci] : 0.f;
    const bf16_t h = f2bf(val);
    w[i] = h;
    wt[((size_t)ci * 27 + (26 - t)) * cout_p + co] = h;
  } else if (i < nw + cout_p) {
    const int co = (int)(i - nw);
    bias[co] = co < cout ? master[(long long)cout * 27 * cin + co] : 0.f;
  }
}

hipError_t launch_cast_weights(const float *master, int cin, int cout, int cin_p, int cout_p,
                               bf16_t *w, bf16_t *wt, float *bias, hipStream_t s) {
  const long long n = (long long)cout_p * 27 * cin_p + cout_p;
  hipLaunchKernelGGL(k_cast_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, master,
                     cin, cout, cin_p, cout_p, w, wt, bias);
  return hipGetLastError();
}

}  // namespace tdgl_nn
