// FFT pass kernels of the electrostatic convolution (paper section 3: the
// electrostatic field is evaluated with FFTs plus custom kernels for the
// intermediate operations; eq 6 as a zero-padded convolution with the
// cell-averaged dipolar tensor).
//
//   k_fx   : real rows -> half spectra along x (two rows per complex line).
//            Zero padding beyond n_in is implicit.
//   k_col  : complex FFT along a strided axis for a tile of adjacent columns
//            (y passes, tensor y/z passes).  Reads n_in points, writes n_out.
//   k_zmul : per (kx, ky) column: forward z FFT of the three components,
//            E^_i = sum_j N~_ij P^_j with the octant-stored real tensor
//            spectrum, inverse z FFT, cropped to the physical layers.
#include "fft_core.h"
#include "internal.h"

namespace tdgl {

// ---------------------------------------------------------------- x pass
template <typename T, int M>
__global__ void k_fx(const T *__restrict__ in, long long nrows, int n_in, long long in_stride,
                     cpx<T> *__restrict__ out, long long out_stride,
                     const cpx<T> *__restrict__ tw, int lpw)
{
    constexpr int TPL = M / 8;
    constexpr int LEN = LinePad<M>::len;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid - l * TPL;
    const long long ra = ((long long)blockIdx.x * lpw + l) * 2;
    const long long rb = ra + 1;
    const bool act = (l < lpw) && (ra < nrows);
    const bool hasb = act && (rb < nrows);
    TwReg<T, M> tr;
    twiddle_load(tr, tw, t);
    cpx<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int x = t + q * TPL;
        T av = T(0), bv = T(0);
        if (act && x < n_in) av = in[ra * in_stride + x];
        if (hasb && x < n_in) bv = in[rb * in_stride + x];
        v[q] = {av, bv};
    }
    cpx<T> *L = lds + l * LEN;
    const IdxPad pad{};
    fft_line<T, M, false>(v, L, pad, t, tr, act);
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < 8; ++q) L[pad(t + q * TPL)] = v[q];
    }
    __syncthreads();
    if (act) {
        for (int k = t; k <= M / 2; k += TPL) {
            const cpx<T> zk = L[pad(k)], zm = L[pad((M - k) & (M - 1))];
            // A = (Z[k] + conj Z[M-k]) / 2,  B = (Z[k] - conj Z[M-k]) / (2i)
            out[ra * out_stride + k] = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            if (hasb) out[rb * out_stride + k] = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
        }
    }
}

// ------------------------------------------------------------ column pass
// Element e of column col in batch b sits at  b*bstride + e*lstride + col.
// Columns of all batches are numbered j = b*C + col and tiled CT at a time,
// so no tile is left partly empty when C is not a multiple of CT.
// In-place use (in == out) is safe: every thread stores exactly the
// positions it loaded.
template <typename T, int M, bool INV>
__global__ void k_col(const cpx<T> *in, cpx<T> *out, long long C, long long ncols, int CT,
                      long long in_bstride, long long out_bstride, long long lstride, int n_in,
                      int n_out, const cpx<T> *__restrict__ tw)
{
    constexpr int TPL = M / 8;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int cc = tid % CT, t = tid / CT;
    const long long j = (long long)blockIdx.x * CT + cc;
    const bool act = j < ncols;
    const long long b = act ? j / C : 0;
    const long long col = act ? j - b * C : 0;
    const cpx<T> *src = in + b * in_bstride + col;
    TwReg<T, M> tr;
    twiddle_load(tr, tw, t);
    cpx<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = t + q * TPL;
        v[q] = (act && e < n_in) ? src[(long long)e * lstride] : cpx<T>{T(0), T(0)};
    }
    fft_line<T, M, INV>(v, lds + cc, IdxStride{CT}, t, tr, act);
    cpx<T> *dst = out + b * out_bstride + col;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = t + q * TPL;
        if (act && e < n_out) dst[(long long)e * lstride] = v[q];
    }
}

// ------------------------------------------------- z pass with multiply
// S: [3][nz][my][hx] complex (in place).  Nt: [6][MZ/2+1][my/2+1][hx] real,
// components xx yy zz xy xz yz; xy is odd in ky, xz odd in kz, yz odd in
// both, so entries outside the stored octant take the mirrored value with
// the corresponding sign.
// FP64 blocks stay at <= 512 threads so each wave may hold up to 256 VGPRs
template <typename T>
struct ZmulMaxThreads {
    static constexpr int v = sizeof(T) == 8 ? 512 : 1024;
};

template <typename T, int MZ>
__global__ void __launch_bounds__(ZmulMaxThreads<T>::v) k_zmul(cpx<T> *S, const T *__restrict__ Nt, int nz, int my, int hx, int CT,
                       const cpx<T> *__restrict__ tw)
{
    constexpr int TPL = MZ / 8;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int cc = tid % CT;
    const int t = (tid / CT) % TPL;
    const int c = tid / (CT * TPL);
    const long long plane = (long long)my * hx;
    // (ky, kx) columns are contiguous within a (component, z) plane
    const long long j = (long long)blockIdx.x * CT + cc;
    const bool act = j < plane;
    const int ky = act ? (int)(j / hx) : 0;
    const int kx = act ? (int)(j - (long long)ky * hx) : 0;
    cpx<T> *col = S + (long long)c * nz * plane + (act ? j : 0);
    TwReg<T, MZ> tr;
    twiddle_load(tr, tw, t);
    // tensor row c at this thread's (kx, ky, kz) points, fetched up front
    const int hy = my / 2;
    const int kyo = ky <= hy ? ky : my - ky;
    const T sy = ky > hy ? T(-1) : T(1);
    const long long s6 = (long long)(MZ / 2 + 1) * (hy + 1) * hx;
    const int i0 = c == 0 ? 0 : (c == 1 ? 3 : 4);   // (c,x) (c,y) (c,z)
    const int i1 = c == 0 ? 3 : (c == 1 ? 1 : 5);
    const int i2 = c == 0 ? 4 : (c == 1 ? 5 : 2);
    auto sgn = [&](int comp, T sz) -> T {
        return comp == 3 ? sy : (comp == 4 ? sz : (comp == 5 ? sy * sz : T(1)));
    };
    T nrow[8][3];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int kz = t + q * TPL;
        const int kzo = kz <= MZ / 2 ? kz : MZ - kz;
        const T sz = kz > MZ / 2 ? T(-1) : T(1);
        const T *nb = Nt + ((long long)kzo * (hy + 1) + kyo) * hx + kx;
        nrow[q][0] = act ? nb[i0 * s6] * sgn(i0, sz) : T(0);
        nrow[q][1] = act ? nb[i1 * s6] * sgn(i1, sz) : T(0);
        nrow[q][2] = act ? nb[i2 * s6] * sgn(i2, sz) : T(0);
    }
    cpx<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int z = t + q * TPL;
        v[q] = (act && z < nz) ? col[(long long)z * plane] : cpx<T>{T(0), T(0)};
    }
    cpx<T> *L = lds + c * MZ * CT + cc;
    fft_line<T, MZ, false>(v, L, IdxStride{CT}, t, tr, act);
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < 8; ++q) L[(t + q * TPL) * CT] = v[q];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kz = t + q * TPL;
            const cpx<T> p0 = lds[(0 * MZ + kz) * CT + cc];
            const cpx<T> p1 = lds[(1 * MZ + kz) * CT + cc];
            const cpx<T> p2 = lds[(2 * MZ + kz) * CT + cc];
            const T n0 = nrow[q][0], n1 = nrow[q][1], n2 = nrow[q][2];
            v[q] = {n0 * p0.x + n1 * p1.x + n2 * p2.x, n0 * p0.y + n1 * p1.y + n2 * p2.y};
        }
    }
    __syncthreads();
    fft_line<T, MZ, true>(v, L, IdxStride{CT}, t, tr, act);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int z = t + q * TPL;
        if (act && z < nz) col[(long long)z * plane] = v[q];
    }
}

// -------------------------------------------------------------- launchers
#define TDGL_LEN_SWITCH(M, CALL)                       \
    switch (M) {                                       \
    case 8: { constexpr int LEN_ = 8; CALL; }          \
    case 16: { constexpr int LEN_ = 16; CALL; }        \
    case 32: { constexpr int LEN_ = 32; CALL; }        \
    case 64: { constexpr int LEN_ = 64; CALL; }        \
    case 128: { constexpr int LEN_ = 128; CALL; }      \
    case 256: { constexpr int LEN_ = 256; CALL; }      \
    case 512: { constexpr int LEN_ = 512; CALL; }      \
    case 1024: { constexpr int LEN_ = 1024; CALL; }    \
    default: return hipErrorInvalidValue;              \
    }

template <typename T, int M>
static hipError_t fx_impl(const void *in, long long nrows, int n_in, long long in_stride,
                          void *out, long long out_stride, const void *tw, hipStream_t s)
{
    constexpr int TPL = M / 8;
    const int lpw = TPL >= 256 ? 1 : 256 / TPL;
    const long long nlines = (nrows + 1) / 2;
    const long long blocks = (nlines + lpw - 1) / lpw;
    if (blocks <= 0) return hipSuccess;
    const size_t shm = (size_t)lpw * LinePad<M>::len * sizeof(cpx<T>);
    hipLaunchKernelGGL((k_fx<T, M>), dim3((unsigned)blocks), dim3(lpw * TPL), shm, s,
                       (const T *)in, nrows, n_in, in_stride, (cpx<T> *)out, out_stride,
                       (const cpx<T> *)tw + M, lpw);
    return hipGetLastError();
}

hipError_t launch_fx(int prec, int M, const void *in, long long nrows, int n_in,
                     long long in_stride, void *out, long long out_stride, const void *tw,
                     hipStream_t s)
{
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH(M, return (fx_impl<float, LEN_>(in, nrows, n_in, in_stride, out,
                                                         out_stride, tw, s)))
    } else {
        TDGL_LEN_SWITCH(M, return (fx_impl<double, LEN_>(in, nrows, n_in, in_stride, out,
                                                          out_stride, tw, s)))
    }
}

// columns per work-group: 128-byte row segments where the length allows,
// at most 1024 threads and 64 KiB of LDS.
template <typename T, int M>
static int col_tile()
{
    constexpr int TPL = M / 8;
    int ct = 128 / (int)sizeof(cpx<T>);
    while (ct > 1 && (ct * TPL > 1024 || (size_t)ct * M * sizeof(cpx<T>) > 65536)) ct /= 2;
    return ct;
}

template <typename T, int M>
static hipError_t col_impl(bool inv, const void *in, void *out, long long C, long long nbatch,
                           long long in_bstride, long long out_bstride, long long lstride,
                           int n_in, int n_out, const void *tw, hipStream_t s)
{
    constexpr int TPL = M / 8;
    const int ct = col_tile<T, M>();
    const long long ncols = C * nbatch;
    const long long gx = (ncols + ct - 1) / ct;
    if (gx <= 0) return hipSuccess;
    if (gx > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t shm = (size_t)ct * M * sizeof(cpx<T>);
    dim3 grid((unsigned)gx);
    if (inv)
        hipLaunchKernelGGL((k_col<T, M, true>), grid, dim3(ct * TPL), shm, s,
                           (const cpx<T> *)in, (cpx<T> *)out, C, ncols, ct, in_bstride,
                           out_bstride, lstride, n_in, n_out, (const cpx<T> *)tw + M);
    else
        hipLaunchKernelGGL((k_col<T, M, false>), grid, dim3(ct * TPL), shm, s,
                           (const cpx<T> *)in, (cpx<T> *)out, C, ncols, ct, in_bstride,
                           out_bstride, lstride, n_in, n_out, (const cpx<T> *)tw + M);
    return hipGetLastError();
}

hipError_t launch_col(int prec, int M, bool inv, const void *in, void *out, long long C,
                      long long nbatch, long long in_bstride, long long out_bstride,
                      long long lstride, int n_in, int n_out, const void *tw, hipStream_t s)
{
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH(M, return (col_impl<float, LEN_>(inv, in, out, C, nbatch, in_bstride,
                                                          out_bstride, lstride, n_in, n_out,
                                                          tw, s)))
    } else {
        TDGL_LEN_SWITCH(M, return (col_impl<double, LEN_>(inv, in, out, C, nbatch, in_bstride,
                                                           out_bstride, lstride, n_in, n_out,
                                                           tw, s)))
    }
}

template <typename T, int MZ>
static hipError_t zmul_impl(const Geom &g, void *S, const void *Nt, const void *tw,
                            hipStream_t s)
{
    constexpr int TPL = MZ / 8;
    int ct = 128 / (int)sizeof(cpx<T>);
    while (ct > 1 && (3 * ct * TPL > ZmulMaxThreads<T>::v ||
                      (size_t)3 * ct * MZ * sizeof(cpx<T>) > 65536))
        ct /= 2;
    const long long ncols = (long long)g.my * g.hx;
    const long long gx = (ncols + ct - 1) / ct;
    const size_t shm = (size_t)3 * ct * MZ * sizeof(cpx<T>);
    hipLaunchKernelGGL((k_zmul<T, MZ>), dim3((unsigned)gx), dim3(3 * ct * TPL), shm, s,
                       (cpx<T> *)S, (const T *)Nt, g.nz, g.my, g.hx, ct,
                       (const cpx<T> *)tw + MZ);
    return hipGetLastError();
}

hipError_t launch_zmul(int prec, const Geom &g, void *S, const void *Nt, const void *tw,
                       hipStream_t s)
{
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH(g.mz, return (zmul_impl<float, LEN_>(g, S, Nt, tw, s)))
    } else {
        TDGL_LEN_SWITCH(g.mz, return (zmul_impl<double, LEN_>(g, S, Nt, tw, s)))
    }
}

}  // namespace tdgl
