// FFT pass kernels of the electrostatic convolution (paper section 3: the
// electrostatic field is evaluated with FFTs plus custom kernels for the
// intermediate operations; eq 6 as a zero-padded convolution with the
// cell-averaged dipolar tensor).
//
// The spectra of a context are stored in blocks of KB consecutive kx
// (internal.h): the x spectra S1 as element (kx, row) at
// ((kx/KB)*rows + row)*KB + kx%KB with row = (c*nz + z)*ny + y, the y spectra
// S2 likewise with rows of my points.  One block of KB kx planes of all
// components is contiguous; in it, column j = ky*KB + kx%KB of line
// (c, z) sits at (c*nz + z)*my*KB + j.
//
//   k_fx    : real rows -> half spectra along x (each row one complex line
//             of half length), zero padding beyond n_in implicit; output
//             written kx-major through an LDS transpose.
//   k_row   : complex FFT of contiguous lines (y passes; tensor y pass).
//   k_col   : complex FFT along a strided axis for tiles of adjacent columns
//             (tensor z pass).
//   k_zmul  : per (kx, ky) column: forward z FFT of the three components,
//             E^_i = sum_j N~_ij P^_j with the octant-stored real tensor
//             spectrum, inverse z FFT, cropped to the physical layers.
//   k_plane : the three passes above fused for one kx plane held in LDS.
#include <type_traits>

#include "fft_core.h"
#include "internal.h"

namespace tdgl {

// ---------------------------------------------------------------- x pass
// Rows r of n_in reals (stride in_stride) -> out[k * out_kstride + r],
// k = 0..M/2.  Each row is one complex line of M/2 points (real_split); a
// work-group transforms lpw consecutive rows and writes the spectra through
// an LDS staging area, so that stores along r are contiguous.  tw: base of
// the twiddle tables (table of length L at offset L).
// BLK: out is KB-blocked with out_kstride = nrows (internal.h).
template <typename T, int M, bool BLK>
__global__ void k_fx(const T *__restrict__ in, long long nrows, int n_in, long long in_stride,
                     cpx<T> *__restrict__ out, long long out_kstride,
                     const cpx<T> *__restrict__ tw, int lpw, Freeze fz)
{
    constexpr int M2 = M / 2;
    constexpr int PPT = HalfLine<M2>::PPT, TPL = HalfLine<M2>::TPL;
    constexpr int LEN = LinePad<M2>::len;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *stg = lds + lpw * LEN;                  // [M2 + 1][lpw] output staging
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int l = tid / TPL, t = tid - l * TPL;
    const long long r0 = (long long)blockIdx.x * lpw;
    const long long r = r0 + l;
    const bool act = (l < lpw) && (r < nrows) && !fz.skip(r);
    TwReg<T, M2> tr;
    twiddle_load(tr, tw + tw_off(M2), t);
    cpx<T> wk[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) wk[q] = tw[tw_off(M) + t + q * TPL];
    cpx<T> v[PPT];
    const T *row = in + (act ? r : 0) * in_stride;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int n = t + q * TPL;
        const T ev = (act && 2 * n < n_in) ? row[2 * n] : T(0);
        const T od = (act && 2 * n + 1 < n_in) ? row[2 * n + 1] : T(0);
        v[q] = {ev, od};
    }
    cpx<T> *L = lds + (l < lpw ? l : 0) * LEN;
    half_fft<T, M2, false>(v, L, t, tr, act);
    __syncthreads();                                // scratch becomes the exchange buffer
    cpx<T> *zx = lds + (l < lpw ? l : 0) * M2;
    if (act) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) zx[t + q * TPL] = v[q];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int k = t + q * TPL;
            cpx<T> xh;
            stg[k * lpw + l] = real_split(zx[k], zx[k == 0 ? 0 : M2 - k], wk[q], xh);
            if (k == 0) stg[M2 * lpw + l] = xh;
        }
    }
    __syncthreads();
    const int rows_here = (int)((nrows - r0) < lpw ? (nrows - r0) : lpw);
    if constexpr (BLK) {
        // e = (block of KB kx, row, kx in block): contiguous stores
        constexpr int NKB = (M2 + KB) / KB;            // blocks covering k = 0..M2
        for (int e = tid; e < NKB * KB * lpw; e += nthr) {
            const int sub = e & (KB - 1), rest = e >> KBS;
            const int kb = rest / lpw, rl = rest - kb * lpw, k = kb * KB + sub;
            if (k <= M2 && rl < rows_here && !fz.skip(r0 + rl))
                out[((long long)kb * out_kstride + r0 + rl) * KB + sub] = stg[k * lpw + rl];
        }
    } else {
        for (int e = tid; e < (M2 + 1) * lpw; e += nthr) {
            const int k = e / lpw, rl = e - k * lpw;
            if (rl < rows_here && !fz.skip(r0 + rl)) out[k * out_kstride + r0 + rl] = stg[e];
        }
    }
}

// ---------------------------------------------------------- row pass
// Line r: n_in points at in + r*in_stride, n_out points to out + r*out_stride.
// In-place use is safe (each thread stores exactly the positions it loaded).
// HALF: n_in == M/2 for a forward pass, n_out == M/2 for an inverse one (an
// open dimension padded to twice its length): the zero inputs or the
// discarded outputs are known at compile time and their arithmetic drops out.
template <typename T, int M, bool INV, bool HALF>
__global__ void k_row(const cpx<T> *in, cpx<T> *out, long long nlines, long long in_stride,
                      long long out_stride, int n_in, int n_out, const cpx<T> *__restrict__ tw,
                      int lpw, Freeze fz)
{
    constexpr int PPT = Plan<M>::PPT, TPL = Plan<M>::TPL;
    constexpr int LEN = LinePad<M>::len;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid - l * TPL;
    const long long line = (long long)blockIdx.x * lpw + l;
    const bool act = l < lpw && line < nlines && !fz.skip(line);
    TwReg<T, M> tr;
    twiddle_load(tr, tw, t);
    const cpx<T> *src = in + (act ? line : 0) * in_stride;
    cpx<T> v[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int e = t + q * TPL;
        const bool in_ok = (HALF && !INV) ? q < PPT / 2 : e < n_in;
        v[q] = (act && in_ok) ? src[e] : cpx<T>{T(0), T(0)};
    }
    fft_line<T, M, INV>(v, lds + (l < lpw ? l : 0) * LEN, IdxPad{}, t, tr, act);
    cpx<T> *dst = out + (act ? line : 0) * out_stride;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int e = t + q * TPL;
        const bool out_ok = (HALF && INV) ? q < PPT / 2 : e < n_out;
        if (act && out_ok) dst[e] = v[q];
    }
}

// ------------------------------------------------- row pass, kx blocks
// The y passes of a context: lines (kx, r), r < R, between the KB-blocked
// x spectra S1 (line of ny points at ((kx/KB)*R + r)*ny*KB + kx%KB, point
// stride KB) and the KB-blocked y spectra S2 (line of my points, same form).
// Forward: S1 -> S2; inverse: S2 -> S1.  The KB lines of one block sit in
// adjacent lanes, so that every load and store of a wave is contiguous.
// Lines of kx >= hx (the padding of the last block) are idle.
template <typename T, int M, bool INV, bool HALF>
__global__ void k_rowb(const cpx<T> *in, cpx<T> *out, int hx, unsigned R, unsigned mR, int ny,
                       int my, int n_in, int n_out, const cpx<T> *__restrict__ tw, int lpw,
                       Freeze fz, int nt)
{
    constexpr int PPT = Plan<M>::PPT, TPL = Plan<M>::TPL;
    constexpr int LEN = LinePad<M>::len;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int sub = tid & (KB - 1), tq = tid >> KBS;
    const int t = tq & (TPL - 1), lg = tq / TPL;
    const int l = lg * KB + sub;                         // LDS line slot
    const unsigned rb = blockIdx.x * (unsigned)(lpw / KB) + lg;   // (kx / KB) * R + r
    const unsigned kxb = udiv(rb, R, mR), r = rb - kxb * R;
    const int kx = (int)kxb * KB + sub;
    const bool act = l < lpw && kx < hx && !fz.skip((long long)kx * R + r);
    TwReg<T, M> tr;
    twiddle_load(tr, tw, t);
    const long long b1 = (long long)rb * ny * KB + sub;     // S1 line
    const long long b2 = (long long)rb * my * KB + sub;     // S2 line
    const cpx<T> *src = in + (act ? (INV ? b2 : b1) : 0);
    cpx<T> v[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int e = t + q * TPL;
        const bool in_ok = (HALF && !INV) ? q < PPT / 2 : e < n_in;
        v[q] = (act && in_ok) ? src[(long long)e * KB] : cpx<T>{T(0), T(0)};
    }
    // a line's lanes (KB * TPL of them) lie within one wave where 4 TPL <= 64:
    // its stages then need wave-level barriers only
    fft_line<T, M, INV, IdxPad, KB * TPL <= 64>(v, lds + (l < lpw ? l : 0) * LEN, IdxPad{}, t, tr,
                                                act);
    cpx<T> *dst = out + (act ? (INV ? b1 : b2) : 0);
    if (nt) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int e = t + q * TPL;
            const bool out_ok = (HALF && INV) ? q < PPT / 2 : e < n_out;
            if (act && out_ok) st_nt(&dst[(long long)e * KB], v[q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int e = t + q * TPL;
            const bool out_ok = (HALF && INV) ? q < PPT / 2 : e < n_out;
            if (act && out_ok) dst[(long long)e * KB] = v[q];
        }
    }
}

// ------------------------------------------------------------ column pass
// Element e of column col in batch b sits at  b*bstride + e*lstride + col.
// Columns of all batches are numbered j = b*C + col and tiled CT at a time.
// In-place use (in == out) is safe.
template <typename T, int M, bool INV>
__global__ void k_col(const cpx<T> *in, cpx<T> *out, long long C, long long ncols, int CT,
                      long long in_bstride, long long out_bstride, long long lstride, int n_in,
                      int n_out, const cpx<T> *__restrict__ tw)
{
    constexpr int TPL = M / 8;
    extern __shared__ __align__(16) unsigned char smem_raw[];
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
    fft_line<T, M, INV>(v, lds + cc, IdxStridePad{CT}, t, tr, act);
    cpx<T> *dst = out + b * out_bstride + col;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = t + q * TPL;
        if (act && e < n_out) dst[(long long)e * lstride] = v[q];
    }
}

// ---------------------------------------------------- tensor row fetch
// Row c of the interaction tensor at (kx, ky, kz) from the octant store
// Nt(kx, q, kz', ky') (q: xx yy zz xy xz yz; kz' <= mz/2, ky' <= my/2), in
// blocks of KB kx as the spectra.  xy is odd in ky, xz odd in kz, yz odd in
// both.
struct TensorRow {
    int i0, i1, i2;    // components (c,x) (c,y) (c,z) of row c
    __device__ explicit TensorRow(int c, int)
        : i0(c == 0 ? 0 : (c == 1 ? 3 : 4)), i1(c == 0 ? 3 : (c == 1 ? 1 : 5)),
          i2(c == 0 ? 4 : (c == 1 ? 5 : 2)) {}
};

template <typename T>
__device__ __forceinline__ T odd_sign(int comp, T sy, T sz)
{
    return comp == 3 ? sy : (comp == 4 ? sz : (comp == 5 ? sy * sz : T(1)));
}

template <typename T>
__device__ __forceinline__ void tensor_row(const T *__restrict__ Nt, int kx, int ky, int kz,
                                           int my, int mz, const TensorRow &r, T &n0, T &n1,
                                           T &n2)
{
    const int hy = my / 2 + 1, hz = mz / 2 + 1;
    const int kyo = ky <= my / 2 ? ky : my - ky;
    const int kzo = kz <= mz / 2 ? kz : mz - kz;
    const T sy = ky > my / 2 ? T(-1) : T(1);
    const T sz = kz > mz / 2 ? T(-1) : T(1);
    const long long qs = (long long)hz * hy * KB;
    const T *b = Nt + (long long)(kx >> KBS) * 6 * qs + ((long long)kzo * hy + kyo) * KB +
                 (kx & (KB - 1));
    n0 = b[r.i0 * qs] * odd_sign(r.i0, sy, sz);
    n1 = b[r.i1 * qs] * odd_sign(r.i1, sy, sz);
    n2 = b[r.i2 * qs] * odd_sign(r.i2, sy, sz);
}

// ------------------------------------------------- z pass with multiply
// S: the KB-blocked y spectra (in place); work-group = (block of KB kx,
// instance, tile of CT consecutive columns j = ky*KB + kx%KB) x 3
// components, so that each z row of the tile is CT contiguous values; the
// tensor is shared by the instances.  Columns per group: 64-byte rows where
// threads (<= 1024 FP32 / 512 FP64) and LDS (<= 64 KiB) allow.
template <typename T, int MZ, int RB>
struct ZmulCfg {
    static constexpr int TPL = MZ / 8;
    static constexpr int MAXT = sizeof(T) == 8 ? 512 : 1024;
    static constexpr int fit(int ct)
    {
        return (ct > 1 && (3 * ct * TPL > MAXT ||
                           (size_t)3 * ct * LinePad<MZ>::len * sizeof(cpx<T>) > 65536))
                   ? fit(ct / 2)
                   : ct;
    }
    static constexpr int CT = fit(RB / (int)sizeof(cpx<T>));    // rows of RB bytes
    static constexpr int NTHR = 3 * CT * TPL;
    // Register allocation, measured on the 128x128x32 film (64-point z
    // transforms), its FP64 version, the 256x256x64 bilayer (128 points) and
    // the batched boxes.  Up to 64 points: the tensor row is loaded after the
    // forward transform and FP32 groups leave room for 6 waves per SIMD
    // (<= 80 VGPRs); from 128 points on, the tensor loads overlap the
    // forward transform and the LDS lines take component-aligned values
    // (paired 4-byte accesses), which keeps the 768-thread groups at two per
    // CU (with 8-byte accesses the allocation grows past 80 VGPRs and the
    // bilayer's z pass slows from 172 to 250 us).
    static constexpr bool LATE = MZ <= 64;
    static constexpr int WEU = (sizeof(T) == 4 && MZ <= 64) ? 6 : 1;
    using LT = typename std::conditional<(MZ >= 128), cpx1<T>, cpx<T>>::type;
};

// HALF: nz == MZ/2 (an open dimension padded to twice its length): the upper
// half of the forward transform's inputs is zero and the upper half of the
// inverse transform's outputs is discarded, both known at compile time, so
// their arithmetic drops out.
template <typename T, int MZ, int RB, bool HALF>
__global__ void __launch_bounds__((ZmulCfg<T, MZ, RB>::NTHR))
    __attribute__((amdgpu_waves_per_eu(ZmulCfg<T, MZ, RB>::WEU)))
    k_zmul(cpx<T> *S, const T *__restrict__ Nt, int nz, int my, int hx, int nb,
           const cpx<T> *__restrict__ tw, const int *__restrict__ frozen, unsigned mgx,
           unsigned mnb, int nt)
{
    using C = ZmulCfg<T, MZ, RB>;
    using LT = typename C::LT;
    constexpr int TPL = C::TPL, CT = C::CT;
    constexpr int LZ = LinePad<MZ>::len;
    // From 128 points on the base is offset by a value the compiler cannot
    // prove zero (it is: grids hold fewer than 2^31 groups), so that it keeps
    // the element type's 4-byte alignment instead of merging the pairs into
    // 8-byte accesses (whose schedule needs 90 registers here).
    extern __shared__ unsigned char smem_raw[];
    LT *lds = reinterpret_cast<LT *>(smem_raw + (MZ >= 128 ? (blockIdx.x >> 31) * 4u : 0u));
    const int tid = threadIdx.x;
    const int cc = tid % CT;
    const int t = (tid / CT) % TPL;
    const int c = tid / (CT * TPL);
    const unsigned tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const unsigned kbb = udiv(tile, gridDim.x, mgx);           // (kx block, instance)
    const unsigned kblk = udiv(kbb, (unsigned)nb, mnb);
    if (frozen && frozen[kbb - kblk * nb]) return;  // the whole group: one instance
    const int myb = my * KB;                         // columns of a block plane
    const int j = (int)(tile - kbb * gridDim.x) * CT + cc;
    const int ky = j >> KBS, kx = (int)kblk * KB + (j & (KB - 1));
    const bool act = j < myb && kx < hx;
    const int kyc = act ? ky : 0, kxc = act ? kx : 0;
    // uniform base, unsigned 32-bit offsets within one block plane
    cpx<T> *plane = S + (long long)kbb * 3 * nz * myb;
    const int hy = my / 2 + 1, hz = MZ / 2 + 1;
    const unsigned qs = (unsigned)hz * hy * KB;      // one tensor component of a block
    // uniform base of the block's octant; byte offsets within it (an octant
    // block holds 6 KB (MZ/2+1)(my/2+1) values, far below 2^32 bytes)
    const T *tplane = Nt + (long long)kblk * 6 * qs;
    const unsigned col = (unsigned)(c * nz) * myb + (act ? j : 0);
    constexpr unsigned CSZ = sizeof(cpx<T>);         // byte offsets: 3 nz myb CSZ < 2^32
    // data first: the forward transform waits for these loads only, the
    // tensor loads behind them complete during the transform
    cpx<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int z = t + q * TPL;
        const bool in = HALF ? q < 4 : z < nz;
        v[q] = (act && in) ? ld_at(plane, (col + (unsigned)z * myb) * CSZ) : cpx<T>{T(0), T(0)};
    }
    // row c of the tensor: components (c,x) (c,y) (c,z) of the octant store
    // Nt(kx, comp, kz', ky') (comp: xx yy zz xy xz yz), KB-blocked in kx; xy
    // is odd in ky, xz odd in kz, yz odd in both
    const int i0 = c == 0 ? 0 : (c == 1 ? 3 : 4);
    const int i1 = c == 0 ? 3 : (c == 1 ? 1 : 5);
    const int i2 = c == 0 ? 4 : (c == 1 ? 5 : 2);
    const bool yneg = kyc > my / 2;
    const unsigned kyo = yneg ? my - kyc : kyc;
    auto ysign = [&](int i) { return (yneg && (i == 3 || i == 5)) ? T(-1) : T(1); };
    const T ys0 = ysign(i0), ys1 = ysign(i1), ys2 = ysign(i2);
    const bool zo0 = i0 == 4 || i0 == 5, zo1 = i1 == 4 || i1 == 5, zo2 = i2 == 4 || i2 == 5;
    constexpr unsigned SZ = sizeof(T);
    const unsigned kxs = (unsigned)(kxc & (KB - 1));
    const unsigned o0 = (i0 * qs + kyo * KB + kxs) * SZ, o1 = (i1 * qs + kyo * KB + kxs) * SZ,
                   o2 = (i2 * qs + kyo * KB + kxs) * SZ;
    T nrow[8][3];
    auto load_tensor = [&]() {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kz = t + q * TPL;
            const bool zneg = kz > MZ / 2;
            const unsigned kzo = (unsigned)(zneg ? MZ - kz : kz) * hy * (KB * SZ);
            nrow[q][0] = ld_at(tplane, o0 + kzo) * ((zneg && zo0) ? -ys0 : ys0);
            nrow[q][1] = ld_at(tplane, o1 + kzo) * ((zneg && zo1) ? -ys1 : ys1);
            nrow[q][2] = ld_at(tplane, o2 + kzo) * ((zneg && zo2) ? -ys2 : ys2);
        }
    };
    if constexpr (!C::LATE) load_tensor();
    TwReg<T, MZ> tr;
    twiddle_load(tr, tw, t);
    const IdxStridePad ip{CT};
    LT *L = lds + c * LZ * CT + cc;
    // a column's lanes lie within one wave where CT TPL <= 64
    constexpr bool WAVE = CT * TPL <= 64;
    fft_line<T, MZ, false, IdxStridePad, WAVE>(v, L, ip, t, tr, act);
    if constexpr (C::LATE) load_tensor();
    // element kz = t + q*TPL of a line sits at ip(t) + ip.shift(q*TPL) when
    // TPL is a multiple of 8 (a constant offset per q)
    auto ipq = [&](int q) {
        if constexpr (TPL % 8 == 0) return ip(t) + ip.shift(q * TPL);
        else return ip(t + q * TPL);
    };
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < 8; ++q) lds_put(&L[ipq(q)], v[q]);
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int o = ipq(q) + cc;
            const cpx<T> p0 = lds_get(&lds[0 * LZ * CT + o]);
            const cpx<T> p1 = lds_get(&lds[1 * LZ * CT + o]);
            const cpx<T> p2 = lds_get(&lds[2 * LZ * CT + o]);
            const T n0 = nrow[q][0], n1 = nrow[q][1], n2 = nrow[q][2];
            v[q] = {n0 * p0.x + n1 * p1.x + n2 * p2.x, n0 * p0.y + n1 * p1.y + n2 * p2.y};
        }
    }
    __syncthreads();
    fft_line<T, MZ, true, IdxStridePad, WAVE>(v, L, ip, t, tr, act);
    if (nt) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int z = t + q * TPL;
            const bool out = HALF ? q < 4 : z < nz;
            if (act && out) st_nt(at(plane, (col + (unsigned)z * myb) * CSZ), v[q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int z = t + q * TPL;
            const bool out = HALF ? q < 4 : z < nz;
            if (act && out) *at(plane, (col + (unsigned)z * myb) * CSZ) = v[q];
        }
    }
}

// ----------------------------------------------------- fused plane pass
// One work-group per kx.  The plane [3][nz][MY] (lines padded one slot per 8)
// sits in LDS: y transforms of all (c, z) lines, then the z pass with the
// tensor multiply in chunks of CK ky columns (scratch [3][MZ][CK]), then the
// inverse y transforms.  S1 (KB-blocked, read with a stride of KB) in/out,
// in place; one work-group per (kx, instance).
template <typename T, int MY, int MZ>
struct PlaneCfg {
    // FP64 groups use at most 384 threads, leaving 256 VGPRs per wave
    static constexpr int CAP = sizeof(T) == 8 ? 384 : 768;
    static constexpr int TPLY = MY / 8, TPLZ = MZ / 8;
    static constexpr int CK = (3 * MY * TPLZ <= CAP) ? MY : CAP / (3 * TPLZ);
    static constexpr int NTHR = 3 * CK * TPLZ;                 // threads per group
    static constexpr int YROUND = NTHR / TPLY;                 // y lines per round
    static constexpr int LINE = LinePad<MY>::len;
};

template <typename T, int MY, int MZ>
size_t plane_lds_bytes(int nz)
{
    using C = PlaneCfg<T, MY, MZ>;
    return (size_t)(3 * nz * C::LINE + 3 * LinePad<MZ>::len * C::CK) * sizeof(cpx<T>);
}

template <typename T, int MY, int MZ>
__global__ void __launch_bounds__((PlaneCfg<T, MY, MZ>::NTHR))
    k_plane(cpx<T> *S1, const T *__restrict__ Nt, int ny, int nz, int nb,
            const cpx<T> *__restrict__ twy, const cpx<T> *__restrict__ twz,
            const int *__restrict__ frozen)
{
    using C = PlaneCfg<T, MY, MZ>;
    constexpr int TPLY = C::TPLY, TPLZ = C::TPLZ, CK = C::CK, LINE = C::LINE;
    static_assert(C::YROUND >= 1 && C::NTHR <= 1024, "plane configuration");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T> *pl = reinterpret_cast<cpx<T> *>(smem_raw);        // [3*nz][LINE]
    cpx<T> *zs = pl + 3 * nz * LINE;                            // [3][MZ + MZ/8][CK]
    constexpr int LZ = LinePad<MZ>::len;
    const IdxStridePad ipz{CK};
    const int tid = threadIdx.x;
    const int kx = blockIdx.x / nb;          // work-group = plane (kx, instance)
    if (frozen && frozen[blockIdx.x % nb]) return;
    const IdxPad pad{};
    const int nlines = 3 * nz;
    // row (line, y) of this plane in the KB-blocked S1: stride KB
    const int bi = blockIdx.x - kx * nb;
    cpx<T> *gplane = S1 + ((long long)(kx >> KBS) * nb * nlines + (long long)bi * nlines) * ny * KB +
                     (kx & (KB - 1));

    // y-pass roles
    const int ly = tid / TPLY, ty = tid - ly * TPLY;
    TwReg<T, MY> twy_r;
    twiddle_load(twy_r, twy, ty);
    // z-pass roles
    const int cc = tid % CK, tz = (tid / CK) % TPLZ, cz = tid / (CK * TPLZ);
    TwReg<T, MZ> twz_r;
    twiddle_load(twz_r, twz, tz);

    // load the plane (rows y >= ny are zero padding)
    for (int e = tid; e < nlines * MY; e += C::NTHR) {
        const int line = e / MY, y = e - line * MY;
        pl[line * LINE + pad(y)] = y < ny ? gplane[((long long)line * ny + y) * KB] : cpx<T>{T(0), T(0)};
    }

    auto ypass = [&](auto inv_tag) {
        constexpr bool INV = decltype(inv_tag)::value;
        for (int r0 = 0; r0 < nlines; r0 += C::YROUND) {
            const int line = r0 + ly;
            const bool act = line < nlines;
            cpx<T> *L = pl + (act ? line : 0) * LINE;
            __syncthreads();
            cpx<T> v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = act ? L[pad(ty + q * TPLY)] : cpx<T>{T(0), T(0)};
            __syncthreads();
            fft_line<T, MY, INV>(v, L, pad, ty, twy_r, act);
            __syncthreads();
            if (act) {
#pragma unroll
                for (int q = 0; q < 8; ++q) L[pad(ty + q * TPLY)] = v[q];
            }
        }
    };
    ypass(std::false_type{});

    // z pass with the tensor multiply, CK ky columns at a time
    for (int ky0 = 0; ky0 < MY; ky0 += CK) {
        const int ky = ky0 + cc;
        const TensorRow trow(cz, 0);
        T nrow[8][3];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            tensor_row(Nt, kx, ky, tz + q * TPLZ, MY, MZ, trow, nrow[q][0], nrow[q][1], nrow[q][2]);
        __syncthreads();
        cpx<T> v[8];
        const cpx<T> *colp = pl + (cz * nz) * LINE + pad(ky);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int z = tz + q * TPLZ;
            v[q] = z < nz ? colp[z * LINE] : cpx<T>{T(0), T(0)};
        }
        cpx<T> *L = zs + cz * LZ * CK + cc;
        fft_line<T, MZ, false>(v, L, ipz, tz, twz_r, true);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) L[ipz(tz + q * TPLZ)] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kz = tz + q * TPLZ;
            const cpx<T> p0 = zs[0 * LZ * CK + ipz(kz) + cc];
            const cpx<T> p1 = zs[1 * LZ * CK + ipz(kz) + cc];
            const cpx<T> p2 = zs[2 * LZ * CK + ipz(kz) + cc];
            const T n0 = nrow[q][0], n1 = nrow[q][1], n2 = nrow[q][2];
            v[q] = {n0 * p0.x + n1 * p1.x + n2 * p2.x, n0 * p0.y + n1 * p1.y + n2 * p2.y};
        }
        __syncthreads();
        fft_line<T, MZ, true>(v, L, ipz, tz, twz_r, true);
        cpx<T> *colw = pl + (cz * nz) * LINE + pad(ky);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int z = tz + q * TPLZ;
            if (z < nz) colw[z * LINE] = v[q];
        }
    }

    ypass(std::true_type{});
    __syncthreads();
    for (int e = tid; e < nlines * ny; e += C::NTHR) {
        const int line = e / ny, y = e - line * ny;
        gplane[(long long)e * KB] = pl[line * LINE + pad(y)];
    }
}

// -------------------------------------------------------------- launchers
// lengths of the x and y transforms: powers of two and 3 * 2^a
#define TDGL_LEN_SWITCH_XY(M, CALL)                    \
    switch (M) {                                       \
    case 8: { constexpr int LEN_ = 8; CALL; }          \
    case 16: { constexpr int LEN_ = 16; CALL; }        \
    case 24: { constexpr int LEN_ = 24; CALL; }        \
    case 32: { constexpr int LEN_ = 32; CALL; }        \
    case 48: { constexpr int LEN_ = 48; CALL; }        \
    case 64: { constexpr int LEN_ = 64; CALL; }        \
    case 96: { constexpr int LEN_ = 96; CALL; }        \
    case 128: { constexpr int LEN_ = 128; CALL; }      \
    case 192: { constexpr int LEN_ = 192; CALL; }      \
    case 256: { constexpr int LEN_ = 256; CALL; }      \
    case 384: { constexpr int LEN_ = 384; CALL; }      \
    case 512: { constexpr int LEN_ = 512; CALL; }      \
    case 768: { constexpr int LEN_ = 768; CALL; }      \
    case 1024: { constexpr int LEN_ = 1024; CALL; }    \
    default: return hipErrorInvalidValue;              \
    }

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
                          void *out, long long out_kstride, const void *tw, hipStream_t s,
                          Freeze fz, bool blocked)
{
    constexpr int M2 = M / 2;
    constexpr int TPL = HalfLine<M2>::TPL;
    const int lpw = TPL >= 256 ? 1 : 256 / TPL;
    const long long blocks = (nrows + lpw - 1) / lpw;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t shm = ((size_t)lpw * LinePad<M2>::len + (size_t)(M2 + 1) * lpw) *
                       sizeof(cpx<T>);
    if (blocked && out_kstride != nrows) return hipErrorInvalidValue;
    if (blocked)
        hipLaunchKernelGGL((k_fx<T, M, true>), dim3((unsigned)blocks), dim3(lpw * TPL), shm, s,
                           (const T *)in, nrows, n_in, in_stride, (cpx<T> *)out, out_kstride,
                           (const cpx<T> *)tw, lpw, fz);
    else
        hipLaunchKernelGGL((k_fx<T, M, false>), dim3((unsigned)blocks), dim3(lpw * TPL), shm, s,
                           (const T *)in, nrows, n_in, in_stride, (cpx<T> *)out, out_kstride,
                           (const cpx<T> *)tw, lpw, fz);
    return hipGetLastError();
}

hipError_t launch_fx(int prec, int M, const void *in, long long nrows, int n_in,
                     long long in_stride, void *out, long long out_kstride, const void *tw,
                     hipStream_t s, Freeze fz, bool blocked)
{
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH_XY(M, return (fx_impl<float, LEN_>(in, nrows, n_in, in_stride, out,
                                                         out_kstride, tw, s, fz, blocked)))
    } else {
        TDGL_LEN_SWITCH_XY(M, return (fx_impl<double, LEN_>(in, nrows, n_in, in_stride, out,
                                                          out_kstride, tw, s, fz, blocked)))
    }
}

template <typename T, int M>
static hipError_t row_impl(bool inv, const void *in, void *out, long long nlines,
                           long long in_stride, long long out_stride, int n_in, int n_out,
                           const void *tw, hipStream_t s, Freeze fz)
{
    constexpr int TPL = Plan<M>::TPL;
    const int lpw = TPL >= 128 ? 1 : 128 / TPL;     // 128-thread groups (measured best)
    const long long blocks = (nlines + lpw - 1) / lpw;
    if (blocks <= 0) return hipSuccess;
    const size_t shm = (size_t)lpw * LinePad<M>::len * sizeof(cpx<T>);
    const dim3 grid((unsigned)blocks), blk(lpw * TPL);
    const cpx<T> *ci = (const cpx<T> *)in;
    cpx<T> *co = (cpx<T> *)out;
    const cpx<T> *twm = (const cpx<T> *)tw + tw_off(M);
    // (the HALF forms need at least two threads per line or M >= 16)
    const bool half = M >= 16 && (inv ? (n_out == M / 2 && n_in == M) : (n_in == M / 2));
    if (inv && half)
        hipLaunchKernelGGL((k_row<T, M, true, true>), grid, blk, shm, s, ci, co, nlines,
                           in_stride, out_stride, n_in, n_out, twm, lpw, fz);
    else if (inv)
        hipLaunchKernelGGL((k_row<T, M, true, false>), grid, blk, shm, s, ci, co, nlines,
                           in_stride, out_stride, n_in, n_out, twm, lpw, fz);
    else if (half)
        hipLaunchKernelGGL((k_row<T, M, false, true>), grid, blk, shm, s, ci, co, nlines,
                           in_stride, out_stride, n_in, n_out, twm, lpw, fz);
    else
        hipLaunchKernelGGL((k_row<T, M, false, false>), grid, blk, shm, s, ci, co, nlines,
                           in_stride, out_stride, n_in, n_out, twm, lpw, fz);
    return hipGetLastError();
}

hipError_t launch_row(int prec, int M, bool inv, const void *in, void *out, long long nlines,
                      long long in_stride, long long out_stride, int n_in, int n_out,
                      const void *tw, hipStream_t s, Freeze fz)
{
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH_XY(M, return (row_impl<float, LEN_>(inv, in, out, nlines, in_stride,
                                                          out_stride, n_in, n_out, tw, s, fz)))
    } else {
        TDGL_LEN_SWITCH_XY(M, return (row_impl<double, LEN_>(inv, in, out, nlines, in_stride,
                                                           out_stride, n_in, n_out, tw, s, fz)))
    }
}

// The x pass's LDS (fx_impl's shm) exceeds 64 KiB for FP64 lines of 1024
// points: raise the limit of both forms.
template <typename T, int M>
static hipError_t fx_prepare()
{
    constexpr int M2 = M / 2;
    constexpr int TPL = HalfLine<M2>::TPL;
    constexpr int lpw = TPL >= 256 ? 1 : 256 / TPL;
    constexpr size_t shm = ((size_t)lpw * LinePad<M2>::len + (size_t)(M2 + 1) * lpw) *
                           sizeof(cpx<T>);
    if (shm <= 65536) return hipSuccess;
    const void *f[2] = {(const void *)k_fx<T, M, false>, (const void *)k_fx<T, M, true>};
    for (const void *k : f) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)shm);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t prepare_fx(int prec, int M)
{
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH_XY(M, return (fx_prepare<float, LEN_>()))
    } else {
        TDGL_LEN_SWITCH_XY(M, return (fx_prepare<double, LEN_>()))
    }
}

template <typename T, int M>
static hipError_t rowb_prepare()
{
    constexpr int TPL = Plan<M>::TPL;
    constexpr int lpw = TPL >= 128 / KB ? KB : 128 / TPL;
    constexpr size_t shm = (size_t)lpw * LinePad<M>::len * sizeof(cpx<T>);
    if (shm <= 65536) return hipSuccess;
    const void *f[4] = {(const void *)k_rowb<T, M, false, false>,
                        (const void *)k_rowb<T, M, false, true>,
                        (const void *)k_rowb<T, M, true, false>,
                        (const void *)k_rowb<T, M, true, true>};
    for (const void *k : f) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)shm);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int M>
static hipError_t rowb_impl(bool inv, const void *S1, void *S2, int hx, long long R, int ny,
                            int my, int n_in, int n_out, const void *tw, hipStream_t s,
                            Freeze fz, int nt)
{
    constexpr int TPL = Plan<M>::TPL;
    // 128-thread groups as the plain row pass, but at least one block of KB lines
    // (above 64 KiB of LDS, i.e. 1024-point FP64 lines, rowb_prepare has
    // raised the kernels' limit)
    const int lpw = TPL >= 128 / KB ? KB : 128 / TPL;
    const long long rows = (long long)hx_blocked(hx) / KB * R;      // line blocks
    const long long blocks = (rows + lpw / KB - 1) / (lpw / KB);
    if (blocks <= 0) return hipSuccess;
    if (rows >= (1LL << 32) || blocks > 0x7fffffffLL || lpw * TPL > 1024)
        return hipErrorInvalidValue;
    const unsigned mR = div_magic((unsigned)R, (unsigned long long)blocks * (lpw / KB));
    const size_t shm = (size_t)lpw * LinePad<M>::len * sizeof(cpx<T>);
    const dim3 grid((unsigned)blocks), blk(lpw * TPL);
    const cpx<T> *twm = (const cpx<T> *)tw + tw_off(M);
    const bool half = M >= 16 && (inv ? (n_out == M / 2 && n_in == M) : (n_in == M / 2));
    const unsigned Ru = (unsigned)R;
    if (inv && half)
        hipLaunchKernelGGL((k_rowb<T, M, true, true>), grid, blk, shm, s, (const cpx<T> *)S2,
                           (cpx<T> *)S1, hx, Ru, mR, ny, my, n_in, n_out, twm, lpw, fz, nt);
    else if (inv)
        hipLaunchKernelGGL((k_rowb<T, M, true, false>), grid, blk, shm, s, (const cpx<T> *)S2,
                           (cpx<T> *)S1, hx, Ru, mR, ny, my, n_in, n_out, twm, lpw, fz, nt);
    else if (half)
        hipLaunchKernelGGL((k_rowb<T, M, false, true>), grid, blk, shm, s, (const cpx<T> *)S1,
                           (cpx<T> *)S2, hx, Ru, mR, ny, my, n_in, n_out, twm, lpw, fz, nt);
    else
        hipLaunchKernelGGL((k_rowb<T, M, false, false>), grid, blk, shm, s, (const cpx<T> *)S1,
                           (cpx<T> *)S2, hx, Ru, mR, ny, my, n_in, n_out, twm, lpw, fz, nt);
    return hipGetLastError();
}

hipError_t prepare_row_blocked(int prec, int M)
{
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH_XY(M, return (rowb_prepare<float, LEN_>()))
    } else {
        TDGL_LEN_SWITCH_XY(M, return (rowb_prepare<double, LEN_>()))
    }
}

hipError_t launch_row_blocked(int prec, int M, bool inv, const void *S1, void *S2, int hx,
                              long long R, int ny, int my, int n_in, int n_out, const void *tw,
                              hipStream_t s, Freeze fz, int nt)
{
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH_XY(M, return (rowb_impl<float, LEN_>(inv, S1, S2, hx, R, ny, my, n_in,
                                                           n_out, tw, s, fz, nt)))
    } else {
        TDGL_LEN_SWITCH_XY(M, return (rowb_impl<double, LEN_>(inv, S1, S2, hx, R, ny, my, n_in,
                                                            n_out, tw, s, fz, nt)))
    }
}

// columns per work-group: 128-byte row segments where the length allows,
// at most 1024 threads and 64 KiB of LDS.
template <typename T, int M>
static int col_tile()
{
    constexpr int TPL = M / 8;
    int ct = 128 / (int)sizeof(cpx<T>);
    while (ct > 1 && (ct * TPL > 1024 || (size_t)ct * LinePad<M>::len * sizeof(cpx<T>) > 65536))
        ct /= 2;
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
    const size_t shm = (size_t)ct * LinePad<M>::len * sizeof(cpx<T>);
    dim3 grid((unsigned)gx);
    if (inv)
        hipLaunchKernelGGL((k_col<T, M, true>), grid, dim3(ct * TPL), shm, s,
                           (const cpx<T> *)in, (cpx<T> *)out, C, ncols, ct, in_bstride,
                           out_bstride, lstride, n_in, n_out, (const cpx<T> *)tw + tw_off(M));
    else
        hipLaunchKernelGGL((k_col<T, M, false>), grid, dim3(ct * TPL), shm, s,
                           (const cpx<T> *)in, (cpx<T> *)out, C, ncols, ct, in_bstride,
                           out_bstride, lstride, n_in, n_out, (const cpx<T> *)tw + tw_off(M));
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

template <typename T, int MZ, int RB>
static hipError_t zmul_tile(const Geom &g, void *S, const void *Nt, const void *tw, hipStream_t s)
{
    using C = ZmulCfg<T, MZ, RB>;
    const int gx = (g.my * KB + C::CT - 1) / C::CT;          // column tiles of a block plane
    const int nkb = hx_blocked(g.hx) / KB;
    if ((long long)nkb * g.nb > 65535) return hipErrorInvalidValue;
    const size_t shm = (size_t)3 * C::CT * LinePad<MZ>::len * sizeof(cpx<T>);
    const unsigned long long ntile = (unsigned long long)gx * nkb * g.nb;
    const unsigned mgx = div_magic((unsigned)gx, ntile);
    const unsigned mnb = div_magic((unsigned)g.nb, (unsigned long long)nkb * g.nb);
    if (2 * g.nz == MZ)
        hipLaunchKernelGGL((k_zmul<T, MZ, RB, true>), dim3(gx, nkb * g.nb), dim3(C::NTHR), shm,
                           s, (cpx<T> *)S, (const T *)Nt, g.nz, g.my, g.hx, g.nb,
                           (const cpx<T> *)tw + tw_off(MZ), g.frozen, mgx, mnb, g.nt);
    else
        hipLaunchKernelGGL((k_zmul<T, MZ, RB, false>), dim3(gx, nkb * g.nb), dim3(C::NTHR), shm,
                           s, (cpx<T> *)S, (const T *)Nt, g.nz, g.my, g.hx, g.nb,
                           (const cpx<T> *)tw + tw_off(MZ), g.frozen, mgx, mnb, g.nt);
    return hipGetLastError();
}

// Column tiles of rb = 64, 128 or 256 bytes per z row; 0 picks 128 bytes, or
// 64 where 128 would leave fewer than 1024 work-groups (measured on the
// 128x128x32 film, the 256x256x64 bilayer and the batched boxes;
// tdgl_autotune tries all three).
int zmul_auto_tile(int prec, const Geom &g)
{
    const int esz = prec == PREC_F32 ? 8 : 16;
    const int ct = 128 / esz;
    const long long groups = (long long)((g.my * KB + ct - 1) / ct) * (hx_blocked(g.hx) / KB) * g.nb;
    return groups < 1024 ? 64 : 128;
}

template <typename T, int MZ>
static hipError_t zmul_impl(const Geom &g, void *S, const void *Nt, const void *tw, int rb,
                            hipStream_t s)
{
    switch (rb) {
    case 64: return zmul_tile<T, MZ, 64>(g, S, Nt, tw, s);
    case 128: return zmul_tile<T, MZ, 128>(g, S, Nt, tw, s);
    case 256: return zmul_tile<T, MZ, 256>(g, S, Nt, tw, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zmul(int prec, const Geom &g, void *S, const void *Nt, const void *tw,
                       int tile_bytes, hipStream_t s)
{
    const int rb = tile_bytes == 0 ? zmul_auto_tile(prec, g) : tile_bytes;
    if (prec == PREC_F32) {
        TDGL_LEN_SWITCH(g.mz, return (zmul_impl<float, LEN_>(g, S, Nt, tw, rb, s)))
    } else {
        TDGL_LEN_SWITCH(g.mz, return (zmul_impl<double, LEN_>(g, S, Nt, tw, rb, s)))
    }
}

// ---- plane path: instantiated for my in 8..256 and mz in 8..128
template <typename T, int MY, int MZ>
static hipError_t plane_impl(const Geom &g, void *S1, const void *Nt, const void *tw,
                             size_t lds_max, hipStream_t s, bool query)
{
    using C = PlaneCfg<T, MY, MZ>;
    const size_t shm = plane_lds_bytes<T, MY, MZ>(g.nz);
    if (shm > lds_max) return hipErrorInvalidConfiguration;
    if (query) {
        if (shm > 65536)
            return hipFuncSetAttribute((const void *)k_plane<T, MY, MZ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        return hipSuccess;
    }
    hipLaunchKernelGGL((k_plane<T, MY, MZ>), dim3(g.hx * g.nb), dim3(C::NTHR), shm, s,
                       (cpx<T> *)S1, (const T *)Nt, g.ny, g.nz, g.nb,
                       (const cpx<T> *)tw + tw_off(MY), (const cpx<T> *)tw + tw_off(MZ), g.frozen);
    return hipGetLastError();
}

#define TDGL_PLANE_MZ(T, MY)                                                              \
    switch (g.mz) {                                                                       \
    case 8: return plane_impl<T, MY, 8>(g, S1, Nt, tw, lds_max, s, query);                \
    case 16: return plane_impl<T, MY, 16>(g, S1, Nt, tw, lds_max, s, query);              \
    case 32: return plane_impl<T, MY, 32>(g, S1, Nt, tw, lds_max, s, query);              \
    case 64: return plane_impl<T, MY, 64>(g, S1, Nt, tw, lds_max, s, query);              \
    case 128: return plane_impl<T, MY, 128>(g, S1, Nt, tw, lds_max, s, query);            \
    default: return hipErrorInvalidValue;                                                 \
    }

#define TDGL_PLANE_MY(T)                        \
    switch (g.my) {                             \
    case 8: TDGL_PLANE_MZ(T, 8)                 \
    case 16: TDGL_PLANE_MZ(T, 16)               \
    case 32: TDGL_PLANE_MZ(T, 32)               \
    case 64: TDGL_PLANE_MZ(T, 64)               \
    case 128: TDGL_PLANE_MZ(T, 128)             \
    case 256: TDGL_PLANE_MZ(T, 256)             \
    default: return hipErrorInvalidValue;       \
    }

// query = true: check that the plane path fits the device's LDS and set the
// kernel's dynamic-LDS limit (call once, outside graph capture).
hipError_t launch_plane(int prec, const Geom &g, void *S1, const void *Nt, const void *tw,
                        size_t lds_max, hipStream_t s, bool query)
{
    if (prec == PREC_F32) {
        TDGL_PLANE_MY(float)
    } else {
        TDGL_PLANE_MY(double)
    }
}

}  // namespace tdgl
