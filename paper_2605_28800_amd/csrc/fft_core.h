// Mixed-radix Stockham FFT of one line per group of threads, for gfx950.
//
// A line of length M (a power of two, 8..1024, or 3 * 2^a, 12..768) is owned
// by M/PPT threads of PPT points each (8 for powers of two, 12 otherwise).
// Thread t of the line holds the elements x[t + q*M/PPT], q < PPT, in
// registers on entry and the outputs X[t + q*M/PPT] (natural order) on exit.
// Only the exchanges between radix stages go through LDS, so a pass kernel
// can load its inputs from and store its outputs to global memory directly,
// with consecutive threads touching consecutive addresses.
//
// Stage with radix R after stages of total length P (Stockham autosort):
// butterfly i in [0, M/R), k = i mod P, inputs x[i + r M/R] twiddled by
// W_{PR}^{rk}, R-point DFT, outputs to y[(i-k) R + k + r P].  The first stage
// (P = 1) needs no twiddles and reads the registers; the last stage
// (P R = M) writes y[i + r M/R], which is again the register layout.
// Radices: 8, 4, 2 for powers of two; 4, 2 and a last 3 otherwise.
//
// Forward transforms use W = exp(-2 pi i/M); inverse transforms the
// conjugate, unnormalised.
#pragma once

#include <hip/hip_runtime.h>

namespace tdgl {

// Aligned to its own size, so that a complex value moves as one 8-byte
// (FP32) or 16-byte (FP64) access; in LDS those take 16-bit byte offsets
// where pairs of separate accesses take 8-bit element offsets, which the
// strides of the transforms overflow.
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

// A complex value in LDS at the alignment of one component: it moves as two
// separate accesses.  The transforms take either element type for their
// LDS lines (measured per kernel: the long z transforms keep lower register
// counts with this one).
template <typename T>
struct cpx1 {
    T x, y;
};
template <typename T>
__device__ __forceinline__ cpx<T> lds_get(const cpx<T> *p) { return *p; }
template <typename T>
__device__ __forceinline__ cpx<T> lds_get(const cpx1<T> *p) { return {p->x, p->y}; }
template <typename T>
__device__ __forceinline__ void lds_put(cpx<T> *p, cpx<T> v) { *p = v; }
template <typename T>
__device__ __forceinline__ void lds_put(cpx1<T> *p, cpx<T> v)
{
    p->x = v.x;
    p->y = v.y;
}

// Non-temporal stores, for the spectra and states that a step kernel writes
// for the next kernel when the context asks for them (Geom::nt, uniform; the
// kernels branch once around their store loops): the lines then stream out
// instead of staying dirty in the writing XCD's L2, which otherwise writes
// them back when the kernel ends.  Measured: the 128x128x32 film's Heun step
// 76 -> 66 us and the 256x256x64 bilayer's 0.86 -> 0.82 ms with them, the
// batched boxes 10-13 % slower, so the context chooses.
template <typename T>
__device__ __forceinline__ void st_nt(cpx<T> *p, cpx<T> v)
{
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 x = {v.x, v.y};
    __builtin_nontemporal_store(x, reinterpret_cast<v2 *>(p));
}
template <typename T>
__device__ __forceinline__ void st_nt(T *p, T v) { __builtin_nontemporal_store(v, p); }

// A value at a uniform base plus a 32-bit byte offset.  Written this way
// (the offset zero-extended next to the access) the load takes the
// scalar-base form, one 32-bit offset register per access, instead of a
// 64-bit address per lane: callers keep the offsets below 2^32 bytes.
template <typename T>
__device__ __forceinline__ T ld_at(const T *base, unsigned boff)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff);
}
template <typename T>
__device__ __forceinline__ T *at(T *base, unsigned boff)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff);
}

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b)
{
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> rot90(cpx<T> a)
{
    return INV ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cpx<T> *v)
{
    cpx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cpx<T> *v)
{
    cpx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    cpx<T> t2 = cadd(v[1], v[3]), t3 = rot90<T, INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

// 8-point DFT as radix-2 (n, n+4) pairs, W_8^n twiddles, two 4-point DFTs.
template <typename T, bool INV>
__device__ __forceinline__ void dft8(cpx<T> *v)
{
    const T s = T(0.70710678118654752440084436210485);
    cpx<T> a[4], b[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        a[n] = cadd(v[n], v[n + 4]);
        b[n] = csub(v[n], v[n + 4]);
    }
    {
        cpx<T> u = b[1];
        b[1] = INV ? cpx<T>{s * (u.x - u.y), s * (u.x + u.y)}
                   : cpx<T>{s * (u.x + u.y), s * (u.y - u.x)};
        b[2] = rot90<T, INV>(b[2]);
        u = b[3];
        b[3] = INV ? cpx<T>{-s * (u.x + u.y), s * (u.x - u.y)}
                   : cpx<T>{s * (u.y - u.x), -s * (u.x + u.y)};
    }
    dft4<T, INV>(a);
    dft4<T, INV>(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = a[k];
        v[2 * k + 1] = b[k];
    }
}

// 3-point DFT: X0 = a + b + c, X1,2 = a - (b + c)/2 -/+ i (sqrt 3 / 2)(b - c)
// for the forward transform (signs of the imaginary part swapped for the
// inverse).
template <typename T, bool INV>
__device__ __forceinline__ void dft3(cpx<T> *v)
{
    const T h = T(0.86602540378443864676372317075294);     // sqrt(3) / 2
    const cpx<T> s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const cpx<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    const cpx<T> r = INV ? cpx<T>{-h * d.y, h * d.x} : cpx<T>{h * d.y, -h * d.x};   // -/+ i h d
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(cpx<T> *v)
{
    if constexpr (R == 8) dft8<T, INV>(v);
    else if constexpr (R == 4) dft4<T, INV>(v);
    else if constexpr (R == 3) dft3<T, INV>(v);
    else dft2<T, INV>(v);
}

// LDS index policies for one line's scratch.  Besides the index of element
// e, each gives the index difference idx(e + d) - idx(e) for a displacement
// d that is a multiple of 8 (shift) and for 0 <= d < 8 from an e that is a
// multiple of 8 (near): the stages form one base index per butterfly and
// reach its R elements by constant offsets, which fold into the LDS
// instructions' immediate offsets.
struct IdxStride {      // element e of the line at e * s (lines interleaved)
    int s;
    __device__ __forceinline__ int operator()(int e) const { return e * s; }
    __device__ __forceinline__ int shift(int d) const { return d * s; }
    __device__ __forceinline__ int near(int d) const { return d * s; }
};
struct IdxPad {         // contiguous line, one pad slot after every 8 elements
    __device__ __forceinline__ int operator()(int e) const { return e + (e >> 3); }
    __device__ __forceinline__ int shift(int d) const { return d + (d >> 3); }
    __device__ __forceinline__ int near(int d) const { return d; }
};
struct IdxStridePad {   // lines interleaved at stride s, one pad row after every 8
    int s;              // elements: 64 lanes of 8-byte accesses hit the minimum of
                        // two LDS bank cycles in every radix stage
    __device__ __forceinline__ int operator()(int e) const { return (e + (e >> 3)) * s; }
    __device__ __forceinline__ int shift(int d) const { return (d + (d >> 3)) * s; }
    __device__ __forceinline__ int near(int d) const { return d * s; }
};

template <int M>
struct LinePad {
    static constexpr int len = M + M / 8;   // LDS elements per line with IdxPad
};

// Stockham plan of a line of M points.  M = 2^a: eight points per thread,
// radix 8 while at least 8 points remain, then 4 or 2.  M = 3 * 2^a (a >= 2):
// twelve points per thread, radix 4 while a multiple of 12 remains, one
// radix 2 where 6 remain, and a last radix-3 stage, so that every stage
// before the last has a power-of-two span P.
template <int M>
struct Plan {
    static constexpr bool R3 = M % 3 == 0;
    static constexpr int PPT = R3 ? 12 : 8;    // points per thread
    static constexpr int TPL = M / PPT;        // threads per line
    static constexpr int radix(int P)
    {
        return !R3 ? (M / P >= 8 ? 8 : M / P)
                   : (M / P == 3 ? 3 : (M / P % 12 == 0 ? 4 : 2));
    }
};

// Stage s spans P points (the product of the earlier radices) with radix R;
// each thread does NB = PPT / R butterflies.  Each thread needs NB*(R-1)
// twiddles per stage s >= 1; they depend only on the thread's position, so
// a kernel loads them into registers at its start (TwReg), overlapping their
// latency with the data loads, and the stages read them from registers.
template <int M, int S>
struct Stage {
    using Prev = Stage<M, (S > 0 ? S - 1 : 0)>;
    static constexpr int P = S == 0 ? 1 : Prev::P * Prev::R;
    static constexpr int R = Plan<M>::radix(P);
    static constexpr int NB = Plan<M>::PPT / R;
    static constexpr int NTW = S == 0 ? 0 : NB * (R - 1);
    static constexpr int OFF = S == 0 ? 0 : Prev::OFF + Prev::NTW;
    static constexpr bool LAST = P * R == M;
};
template <int M>
struct Stage<M, 0> {
    static constexpr int P = 1, R = Plan<M>::radix(1), NB = Plan<M>::PPT / R, NTW = 0, OFF = 0;
    static constexpr bool LAST = (R == M);
};

template <int M, int S = 0>
constexpr int twiddle_count()
{
    if constexpr (Stage<M, S>::LAST) return Stage<M, S>::OFF + Stage<M, S>::NTW;
    else return twiddle_count<M, S + 1>();
}

template <typename T, int M>
struct TwReg {
    static constexpr int N = twiddle_count<M>();
    cpx<T> w[N > 0 ? N : 1];
};

template <typename T, int M, int S = 1>
__device__ __forceinline__ void twiddle_load(TwReg<T, M> &tr, const cpx<T> *__restrict__ tab,
                                             int t)
{
    if constexpr (!Stage<M, 0>::LAST) {
        using St = Stage<M, S>;
        constexpr int TPL = Plan<M>::TPL;
#pragma unroll
        for (int b = 0; b < St::NB; ++b) {
            const int i = t + b * TPL;
            const int k = i & (St::P - 1);
#pragma unroll
            for (int r = 1; r < St::R; ++r)
                tr.w[St::OFF + b * (St::R - 1) + r - 1] = tab[r * k * (M / (St::P * St::R))];
        }
        if constexpr (!St::LAST) twiddle_load<T, M, S + 1>(tr, tab, t);
    }
}

// Barrier between the stages of a line: the whole work-group, or (WAVE)
// only the wave, when every line of the caller lies within one wave (then
// the other waves of the group need not take part).
template <bool WAVE>
__device__ __forceinline__ void line_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    } else {
        __syncthreads();
    }
}

// Stages s >= 1.  Every thread of the work-group (WAVE: of the wave) must
// reach these barriers; threads with act == false only skip memory traffic.
template <typename T, int M, int S, bool INV, class Idx, bool WAVE = false, class LT>
__device__ __forceinline__ void fft_stages(cpx<T> (&v)[Plan<M>::PPT], LT *lds, Idx idx, int t,
                                           const TwReg<T, M> &tr, bool act)
{
    using St = Stage<M, S>;
    constexpr int R = St::R, NB = St::NB, P = St::P;
    constexpr int PPT = Plan<M>::PPT, TPL = Plan<M>::TPL;
    constexpr int MR = M / R;
    static_assert((P & (P - 1)) == 0, "the span of a stage is a power of two");
    // element i + d of a read, j + r P of a write: constant offsets from one
    // base index when the displacements are multiples of 8
    constexpr bool FAST_READ = TPL % 8 == 0 && MR % 8 == 0;
    constexpr bool FAST_WRITE = P % 8 == 0;
    line_sync<WAVE>();
    if (act) {
        if constexpr (FAST_READ) {
            const int f0 = idx(t);
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    v[b * R + r] = lds_get(&lds[f0 + idx.shift(b * TPL + r * MR)]);
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int i = t + b * TPL;
#pragma unroll
                for (int r = 0; r < R; ++r) v[b * R + r] = lds_get(&lds[idx(i + r * MR)]);
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cpx<T> w = tr.w[St::OFF + b * (R - 1) + r - 1];
                v[b * R + r] = INV ? cmulc(v[b * R + r], w) : cmul(v[b * R + r], w);
            }
            dftR<T, R, INV>(v + b * R);
        }
    }
    if constexpr (St::LAST) {
        if constexpr (NB > 1) {
            cpx<T> tmp[PPT];
#pragma unroll
            for (int q = 0; q < PPT; ++q) tmp[q] = v[q];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < R; ++r) v[b + r * NB] = tmp[b * R + r];
        }
    } else {
        line_sync<WAVE>();
        if (act) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int i = t + b * TPL;
                const int k = i & (P - 1);
                const int j = (i - k) * R + k;
                if constexpr (FAST_WRITE) {
                    const int fj = idx(j);
#pragma unroll
                    for (int r = 0; r < R; ++r) lds_put(&lds[fj + idx.shift(r * P)], v[b * R + r]);
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) lds_put(&lds[idx(j + r * P)], v[b * R + r]);
                }
            }
        }
        fft_stages<T, M, S + 1, INV, Idx, WAVE>(v, lds, idx, t, tr, act);
    }
}

// Full line transform: thread t holds elements t + q TPL (q < PPT) on entry
// and the transform at the same positions on exit.  The caller must make
// sure no thread still reads the line's LDS region from an earlier use
// (barrier) before calling, and must barrier again before reusing it
// afterwards.  tr: this thread's twiddles (twiddle_load with the forward
// table; the inverse conjugates them).
template <typename T, int M, bool INV, class Idx, bool WAVE = false, class LT>
__device__ __forceinline__ void fft_line(cpx<T> (&v)[Plan<M>::PPT], LT *lds, Idx idx, int t,
                                         const TwReg<T, M> &tr, bool act)
{
    static_assert(M >= 8 && M <= 1024 &&
                      ((M & (M - 1)) == 0 || (M % 3 == 0 && M >= 12 && ((M / 3) & (M / 3 - 1)) == 0)),
                  "length");
    using S0 = Stage<M, 0>;
    constexpr int R0 = S0::R, NB0 = S0::NB, TPL = Plan<M>::TPL;
    if constexpr (NB0 == 1) {
        // one radix-PPT butterfly over the thread's own elements
        if (act) dftR<T, R0, INV>(v);
        if constexpr (!S0::LAST) {
            if (act) {
                const int f8 = idx(R0 * t);
#pragma unroll
                for (int r = 0; r < R0; ++r) lds_put(&lds[f8 + idx.near(r)], v[r]);
            }
        }
    } else {
        // butterfly b of the first stage takes the thread's elements b + NB0 r
        // (points t + (b + NB0 r) TPL, i.e. i + r M/R0 with i = t + b TPL)
        if (act) {
#pragma unroll
            for (int b = 0; b < NB0; ++b) {
                cpx<T> u[R0];
#pragma unroll
                for (int r = 0; r < R0; ++r) u[r] = v[b + NB0 * r];
                dftR<T, R0, INV>(u);
#pragma unroll
                for (int r = 0; r < R0; ++r) lds_put(&lds[idx((t + b * TPL) * R0 + r)], u[r]);
            }
        }
    }
    if constexpr (!S0::LAST) fft_stages<T, M, 1, INV, Idx, WAVE>(v, lds, idx, t, tr, act);
}

// Quotient n / d of uniform operands through d's magic number m =
// ceil(2^32 / d) (div_magic on the host; 0 for d = 1): one scalar high
// multiply instead of the vector division sequence.  Exact while n * d < 2^32;
// the launchers check that bound and pass m = DIV_SLOW otherwise.
constexpr unsigned DIV_SLOW = 0xffffffffu;
__host__ __device__ __forceinline__ unsigned div_magic(unsigned d, unsigned long long nmax)
{
    if (d <= 1) return 0u;
    if (nmax * d >= (1ULL << 32)) return DIV_SLOW;
    return (unsigned)(((1ULL << 32) + d - 1) / d);
}
__device__ __forceinline__ unsigned udiv(unsigned n, unsigned d, unsigned m)
{
    if (m == 0u) return n;
    if (m == DIV_SLOW) return n / d;
    return __umulhi(n, m);
}

// Work-groups of a launch are dealt round-robin to the eight XCDs of the
// chip, each with its own L2.  xcd_tile maps the linear work-group index b
// (of n) to a tile index such that every XCD receives one contiguous range
// of tiles, so tiles that share cache lines (neighbouring rows, mirrored
// tensor columns) meet in the same L2.  A bijection of [0, n).
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned n)
{
    constexpr unsigned X = 8;
    const unsigned q = n / X, r = n % X;
    const unsigned x = b % X, i = b / X;
    return x * q + (x < r ? x : r) + i;
}

// Real lines through complex transforms of half length.  A real line x of M
// points is the complex line z[n] = x[2n] + i x[2n+1] of M/2 points; with
// Z = DFT_{M/2}(z), E[k] = (Z[k] + conj Z[M/2-k])/2 and
// O[k] = (Z[k] - conj Z[M/2-k])/(2i) are the DFTs of the even and odd samples,
// and X[k] = E[k] + W_M^k O[k], X[k + M/2] = E[k] - W_M^k O[k].
// real_split returns X[k] and sets xh = X[k + M/2] (needed at k = 0 only).
// Both helpers round every operation separately (no contraction into FMAs),
// so that a spectrum computed here does not depend on which of the results
// the calling kernel keeps: the x pass and the update kernel's forward
// transform must agree bit for bit.
template <typename T>
__device__ __forceinline__ cpx<T> real_split(cpx<T> zk, cpx<T> zm, cpx<T> wk, cpx<T> &xh)
{
#pragma clang fp contract(off)
    const cpx<T> ev = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    const cpx<T> od = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
    const cpx<T> wo = {od.x * wk.x - od.y * wk.y, od.x * wk.y + od.y * wk.x};
    xh = {ev.x - wo.x, ev.y - wo.y};
    return {ev.x + wo.x, ev.y + wo.y};
}

// The inverse: from the half spectrum X[0..M/2] of a real line (a = X[k],
// b = X[M/2-k]) the complex line Z'[k] = (a + conj b) + i W_M^-k (a - conj b)
// = 2 (E[k] + i O[k]), whose unnormalised inverse DFT of length M/2 is
// M (x[2n] + i x[2n+1]), the unnormalised inverse real DFT of length M.
template <typename T>
__device__ __forceinline__ cpx<T> real_merge(cpx<T> a, cpx<T> b, cpx<T> wk)
{
#pragma clang fp contract(off)
    const cpx<T> e = {a.x + b.x, a.y - b.y};
    const cpx<T> f = {a.x - b.x, a.y + b.y};
    const cpx<T> d = {f.x * wk.x + f.y * wk.y, f.y * wk.x - f.x * wk.y};   // f conj(wk)
    return {e.x - d.y, e.y + d.x};
}

// Complex transform of one line of M2 points: the plan's threads of PPT
// points each, or, for M2 = 4, one thread's registers.
template <int M2>
struct HalfLine {
    static constexpr int PPT = M2 >= 8 ? Plan<M2 >= 8 ? M2 : 8>::PPT : M2;   // points per thread
    static constexpr int TPL = M2 / PPT;                                   // threads per line
};

template <typename T, int M2, bool INV, bool WAVE = false>
__device__ __forceinline__ void half_fft(cpx<T> (&v)[HalfLine<M2>::PPT], cpx<T> *lds, int t,
                                         const TwReg<T, M2> &tr, bool act)
{
    if constexpr (M2 >= 8) fft_line<T, M2, INV, IdxPad, WAVE>(v, lds, IdxPad{}, t, tr, act);
    else if (act) dft4<T, INV>(v);
}

}  // namespace tdgl
