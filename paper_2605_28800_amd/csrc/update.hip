// Fused local-field and time-integration kernel.
//
// One work-group owns yt consecutive rows (all x) of one z layer, for all
// three components:
//   0. per cell (all waves): Landau field (minus the P-derivative of eq 3),
//      gradient field (eq 4, diagonal part, 7-point stencil; neighbours
//      across an open surface or in vacuum are dropped, periodic dimensions
//      wrap) and the cross terms' field;
//   1. (the waves that hold the x lines, beside step 0) inverse x transform
//      of the electrostatic field rows: each real row of padded length M is
//      one complex line of M/2 points (even samples real, odd samples
//      imaginary), built from the half spectrum on the fly;
//   2. after one barrier, per cell: the electrostatic field (eqs 5-6) and
//      the applied field (eq 7) are added, then
//        STEP  : an explicit stage of eq 1 (L = 1, reduced time):
//                stage 0  P_out = P_in + dtau E          (Euler / Heun predictor)
//                stage 1  P_out = (P_old + P_in)/2 + dtau/2 E   (Heun corrector)
//        FIELD : E written out in V/m
//        ENERGY: FP64 partial sums of the energy terms and of P;
//   3. STEP with fx_out: forward x transform of the new rows (again M/2
//      complex points per row, split into the half spectrum), written over
//      the spectra rows read in step 1, so the next field evaluation starts
//      at the y pass.
// The spectra are stored in blocks of KB consecutive kx (internal.h), so the
// yt rows of a group read and write yt*KB contiguous values per block.
#include <mutex>

#include "fft_core.h"
#include "internal.h"

namespace tdgl {

template <typename T>
__device__ __forceinline__ T landau_dfdp(const T p[3], const T sq[3], const T *cf, int i)
{
    const int j = i == 0 ? 1 : 0;
    const int k = i == 2 ? 1 : 2;
    const T sj = sq[j] + sq[k];
    const T s4 = sq[j] * sq[j] + sq[k] * sq[k];
    // d/dP_i of eq 3 (cf: a1x a1y a1z a11 a12 a111 a112 a123)
    return p[i] * (T(2) * cf[i] + T(4) * cf[3] * sq[i] + T(2) * cf[4] * sj +
                   T(6) * cf[5] * sq[i] * sq[i] + cf[6] * (T(4) * sq[i] * sj + T(2) * s4) +
                   T(2) * cf[7] * sq[j] * sq[k]);
}

template <typename T>
__device__ __forceinline__ T landau_f(const T sq[3], const T *cf)
{
    const T x = sq[0], y = sq[1], z = sq[2];
    return cf[0] * x + cf[1] * y + cf[2] * z + cf[3] * (x * x + y * y + z * z) +
           cf[4] * (x * y + y * z + z * x) + cf[5] * (x * x * x + y * y * y + z * z * z) +
           cf[6] * (x * x * (y + z) + y * y * (x + z) + z * z * (x + y)) + cf[7] * x * y * z;
}

// Dormand-Prince 5(4) tableau (Dormand & Prince 1980): row s of RK_A gives
// the weights of k_1..k_s for the stage point s + 1 (row 6 is the
// fifth-order solution); RK_E = fifth- minus fourth-order weights.
__constant__ double RK_A[6][6] = {
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
__constant__ double RK_E[7] = {35.0 / 384 - 5179.0 / 57600, 0, 500.0 / 1113 - 7571.0 / 16695,
                               125.0 / 192 - 393.0 / 640, -2187.0 / 6784 + 92097.0 / 339200,
                               11.0 / 84 - 187.0 / 2100, -1.0 / 40};

// Cross terms of the gradient energy (G12 P_i,i P_j,j and (G44 - G44')
// P_i,j P_j,i) for one cell, with cell-centred central differences in which
// a missing neighbour takes the cell's own value.  The field is minus the
// exact gradient of that discrete energy: with D_d the central difference
// and D_d^T its adjoint,
//   H_i -= g12 sum_{j != i} D_i^T(D_j P_j) + gm sum_{j != i} D_j^T(D_i P_j).
// ex[2d + s]: neighbour of the cell along d on side s (0: -, 1: +) exists;
// nb[2d + s]: its offset (the cell's own when missing); cn: the edge values
// (centre when missing); P: component bases.  Corner (a s, b t) exists iff
// both edges do (the layer map depends on z only).
template <typename T>
struct CrossArgs {
    const T *P[3];
    int off;
    int nb[6];
    bool ex[6];
    T ih[3];            // 1 / (2 h_d)
};

// F(q) = D_b Q at q = cell + s a (s = -1, 0, +1)
template <typename T>
__device__ __forceinline__ T cross_db(const CrossArgs<T> &x, const T (&cn)[6][3], T pc, int comp,
                                      int a, int s, int b)
{
    if (s == 0) return (cn[2 * b + 1][comp] - cn[2 * b][comp]) * x.ih[b];
    const int e = 2 * a + (s > 0 ? 1 : 0);
    if (!x.ex[e]) return T(0);                       // multiplied by 0 below
    const int qa = x.nb[e];
    const T qv = cn[e][comp];
    const T up = x.ex[2 * b + 1] ? x.P[comp][qa + (x.nb[2 * b + 1] - x.off)] : qv;
    const T dn = x.ex[2 * b] ? x.P[comp][qa + (x.nb[2 * b] - x.off)] : qv;
    (void)pc;
    return (up - dn) * x.ih[b];
}

// (D_a^T (D_b Q))(cell)
template <typename T>
__device__ __forceinline__ T cross_t(const CrossArgs<T> &x, const T (&cn)[6][3], T pc, int comp,
                                     int a, int b)
{
    const bool em = x.ex[2 * a], ep = x.ex[2 * a + 1];
    const T fm = cross_db(x, cn, pc, comp, a, -1, b);
    const T fp = cross_db(x, cn, pc, comp, a, +1, b);
    const T f0 = cross_db(x, cn, pc, comp, a, 0, b);
    T r = (em ? fm : T(0)) - (ep ? fp : T(0));
    r += f0 * (T(ep ? 0 : 1) - T(em ? 0 : 1));
    return r * x.ih[a];
}

template <typename T>
struct UpdMaxThreads {    // FP64 groups stay at 512 threads (room for 256 VGPRs)
    static constexpr int v = sizeof(T) == 8 ? 512 : 1024;
};

// NT: the new state and its spectrum go out as non-temporal stores (the
// context's store mode, instantiated for the stepping mode only)
template <typename T, int M, int MODE, bool NT>
__global__ void __launch_bounds__(UpdMaxThreads<T>::v)
    k_update(UpdArgs a, Geom g, const cpx<T> *__restrict__ tw)
{
    // The x transforms of real rows run as complex transforms of length M/2
    // (real_split / real_merge).  Line l = c*yt + yy (component c, row yy)
    // is owned by TPL consecutive lanes of one wave; the partner values
    // X[M/2-k] and Z[M/2-k] of the split and the merge come from the lane
    // TPL - t of the same line (lane permutes, no LDS round trip).
    constexpr int M2 = M / 2;
    constexpr int PPT = HalfLine<M2>::PPT;     // points per thread
    constexpr int TPL = HalfLine<M2>::TPL;     // threads per row
    constexpr int LEN = LinePad<M2>::len;
    constexpr int CPT = 2;                     // cells per thread, at most
    static_assert(64 % TPL == 0, "a line must not straddle waves");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int yt = a.yt;                       // a power of two
    const int ysh = __ffs(yt) - 1;
    const int nrows = 3 * yt;
    const int tid = threadIdx.x, nthr = blockDim.x;
    // tile = (instance b, layer z, row group), instance-major
    const unsigned tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const unsigned zb = udiv(tile, gridDim.x, a.mgx);
    const unsigned bq = udiv(zb, (unsigned)nz, a.mnz);
    const int z = (int)(zb - bq * nz), b = (int)bq, y0 = (int)(tile - zb * gridDim.x) * yt;
    if constexpr (MODE == UPD_STEP || MODE == UPD_ENERGY) {
        if (g.frozen && g.frozen[b]) {            // a retired instance (whole group)
            if constexpr (MODE == UPD_STEP) {     // its state is carried over unchanged
                const long long cm = (long long)nz * ny * nx;
                const int nrow = ny - y0 < yt ? ny - y0 : yt;
                const T *src = reinterpret_cast<const T *>(a.P_in) + 3LL * b * cm;
                T *dst = reinterpret_cast<T *>(a.P_out) + 3LL * b * cm;
                const long long base = ((long long)z * ny + y0) * nx;
                for (int e = threadIdx.x; e < 3 * nrow * nx; e += blockDim.x) {
                    const int c = e / (nrow * nx), r = e - c * nrow * nx;
                    dst[c * cm + base + r] = src[c * cm + base + r];
                }
            } else if (threadIdx.x < 8) {
                a.partials[(long long)tile * 8 + threadIdx.x] = 0.0;
            }
            return;
        }
    }
    // LDS: rows hs[(c*yt + yy)*HS + x] (HS = nx + 2 rounded down to even, so
    // that (even, odd) sample pairs are aligned as one complex value), then
    // the FFT scratch per line.
    const int HS = (nx + 2) & ~1;
    const size_t hbytes = ((size_t)nrows * HS * sizeof(T) + 15) / 16 * 16;
    T *hs = reinterpret_cast<T *>(smem_raw);
    cpx<T> *scr = reinterpret_cast<cpx<T> *>(smem_raw + hbytes);
    const int plane = ny * nx;                 // components hold < 2^31 cells
    const long long comp = (long long)nz * plane;
    const T *coef0 = reinterpret_cast<const T *>(a.coef) + (long long)b * nz * NCOEF;
    const T *coefz = coef0 + (long long)z * NCOEF;
    const KParams<T> *kp = reinterpret_cast<const KParams<T> *>(a.kp);
    const bool material = coefz[8] != T(0);
    const unsigned terms = a.terms;
    constexpr bool STEPPING = MODE == UPD_STEP || MODE == UPD_STEP_MS || MODE == UPD_STEP_RK;
    T rkerr = T(0);                            // STEP_RK stage 7: max scaled error
    const bool do_fx = STEPPING && a.fx_out;
    const int ny_here = ny - y0 < yt ? ny - y0 : yt;

    // line roles
    const int l = tid / TPL, t = tid - l * TPL;
    const bool lact = l < nrows;
    const int lc = lact ? l >> ysh : 0, lyy = lact ? l & (yt - 1) : 0;
    const bool has = lact && lyy < ny_here;
    const int lane = tid & 63;
    const int partner = (lane - t) + ((TPL - t) & (TPL - 1));
    cpx<T> *L = scr + (lact ? l : 0) * LEN;
    cpx<T> *S1 = reinterpret_cast<cpx<T> *>(a.S1);
    // S1 in blocks of KB kx: X[k] of this row at s1row[(k / KB) * kst + k % KB]
    const long long kst = 3LL * g.nb * nz * ny * KB;   // S1 stride between kx blocks
    cpx<T> *s1row = S1 + (((long long)(b * 3 + lc) * nz + z) * ny + y0 + (has ? lyy : 0)) * KB;
    auto s1k = [&](int k) -> long long { return (long long)(k >> KBS) * kst + (k & (KB - 1)); };
    // the waves that hold the x lines (every line lies within one wave, so
    // their transforms need wave-level barriers only, and the waves without
    // lines never wait for them before the field rows are complete)
    const int fft_waves = (nrows * TPL + 63) >> 6;
    const bool lwave = (tid >> 6) < fft_waves;          // uniform per wave
    const bool fftw = a.elec_in && lwave;

    // twiddles of the transforms (a small table, cached)
    TwReg<T, M2> tr;
    cpx<T> wk[PPT];                            // W_M^k, k = t + q*TPL
    auto load_twiddles = [&]() {
        twiddle_load(tr, tw + tw_off(M2), t);
#pragma unroll
        for (int q = 0; q < PPT; ++q) wk[q] = tw[tw_off(M) + t + q * TPL];
    };

    // ---- 1. (line waves) electrostatic field rows: the spectrum X[k],
    // k = t + q*TPL, of this thread's row (lane t = 0 also reads X[M/2]),
    // inverse x transform of half length, rows into LDS.  For rows of up to
    // 128 points (early: the line waves are few among the cell waves) the
    // line waves do this before loading their cells, while the other waves
    // work on their local terms; for longer rows, where most waves hold
    // lines, after the local terms (measured on the 128x128x32 film and the
    // 256x256x64 bilayer).
    constexpr bool early = M <= 128;
    cpx<T> xa[PPT], xn = {T(0), T(0)};
    auto load_spectra = [&]() {
#pragma unroll
        for (int q = 0; q < PPT; ++q)
            xa[q] = has ? s1row[s1k(t + q * TPL)] : cpx<T>{T(0), T(0)};
        if (has && t == 0) xn = s1row[s1k(M2)];
    };
    auto field_rows = [&]() {
        load_twiddles();
        cpx<T> v[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            // X[M2 - k]: lane TPL - t, point PPT-1-q; for t = 0 it is this
            // lane's point PPT - q (or X[M2] at q = 0)
            const int qs = PPT - 1 - q;
            cpx<T> b = {__shfl(xa[qs].x, partner, 64), __shfl(xa[qs].y, partner, 64)};
            if (t == 0) b = q == 0 ? xn : xa[(PPT - q) % PPT];
            cpx<T> A = xa[q];
            if (t == 0 && q == 0) {                    // X[0], X[M/2] are real
                A.y = T(0);
                b.y = T(0);
            }
            v[q] = real_merge(A, b, wk[q]);
        }
        half_fft<T, M2, true, true>(v, L, t, tr, lact);
        if (lact) {
            T *ha = hs + l * HS;
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int n = t + q * TPL;
                if (2 * n + 1 < nx) {
                    *reinterpret_cast<cpx<T> *>(ha + 2 * n) = v[q];
                } else if (2 * n < nx) {
                    ha[2 * n] = v[q].x;
                }
            }
        }
    };
    if constexpr (early) {
        if (fftw) {
            load_spectra();
            field_rows();
        }
    }

    // ---- prologue: issue the global loads up front, the cells first
    // cells: centre, neighbours (-x +x -y +y -z +z; a missing neighbour is
    // the centre itself, so its difference vanishes), old state.  Nothing
    // here waits for a loaded value: the z neighbours are the geometric ones
    // and a vacuum neighbour layer is dropped afterwards (hzm, hzp), so the
    // layer flags arrive while the cells do
    const int zm = z > 0 ? z - 1 : (g.pz ? nz - 1 : -1);
    const int zp = z < nz - 1 ? z + 1 : (g.pz ? 0 : -1);
    const bool need_nb = (terms & T_GRAD) != 0;
    const bool need_old = (MODE == UPD_STEP && a.stage == 1) || (MODE == UPD_STEP_MS && a.stage == 3);
    const T *Pin0 = reinterpret_cast<const T *>(a.P_in) + 3 * b * comp;
    const T *Pold0 = a.P_old ? reinterpret_cast<const T *>(a.P_old) + 3 * b * comp : nullptr;
    // uniform bases of the components in this layer and in the neighbour
    // layers (a missing neighbour layer: this one); a cell is its byte
    // offset within the layer (a layer holds at most 1024 x 1024 cells)
    const int zoff = z * plane;
    const int zmoff = zm >= 0 ? zm * plane : zoff;
    const int zpoff = zp >= 0 ? zp * plane : zoff;
    const T *Pz[3], *Pzm[3], *Pzp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Pz[c] = Pin0 + c * comp + zoff;
        Pzm[c] = Pin0 + c * comp + zmoff;
        Pzp[c] = Pin0 + c * comp + zpoff;
    }
    constexpr unsigned SZ = sizeof(T);
    const unsigned nx_div = 0xffffffffu / (unsigned)nx + 1u;   // e / nx for e < 2^16
    T cp[CPT][3], cn[CPT][6][3], co[CPT][3];
    bool cok[CPT];
    int cyy[CPT], cx[CPT], cip[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const unsigned e = tid + i * nthr;
        const int yy = nx == 1 ? (int)e : (int)__umulhi(e, nx_div);
        const int x = (int)e - yy * nx, y = y0 + yy;
        cok[i] = yy < ny_here;
        const int yc = cok[i] ? y : y0, xc = cok[i] ? x : 0;   // a valid cell for the tail
        cyy[i] = yy;
        cx[i] = x;
        const int ip = yc * nx + xc;                             // within the layer
        cip[i] = ip;
        const unsigned cb = (unsigned)ip * SZ;
#pragma unroll
        for (int c = 0; c < 3; ++c) cp[i][c] = ld_at(Pz[c], cb);
        if (need_nb) {
            const int xm = xc > 0 ? ip - 1 : (g.px ? ip + nx - 1 : ip);
            const int xp = xc < nx - 1 ? ip + 1 : (g.px ? ip - nx + 1 : ip);
            const int ym = yc > 0 ? ip - nx : (g.py ? ip + plane - nx : ip);
            const int yp = yc < ny - 1 ? ip + nx : (g.py ? ip - plane + nx : ip);
            const unsigned nb[4] = {(unsigned)xm * SZ, (unsigned)xp * SZ, (unsigned)ym * SZ,
                                    (unsigned)yp * SZ};
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int c = 0; c < 3; ++c) cn[i][d][c] = ld_at(Pz[c], nb[d]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cn[i][4][c] = ld_at(Pzm[c], cb);
                cn[i][5][c] = ld_at(Pzp[c], cb);
            }
        }
        if (need_old) {
#pragma unroll
            for (int c = 0; c < 3; ++c) co[i][c] = ld_at(Pold0 + c * comp + zoff, cb);
        }
    }


    if constexpr (!early) {
        if (fftw) load_spectra();                   // behind the cell loads
    }
    // z neighbours in vacuum layers are dropped (they read as the centre)
    const bool hzm = zm >= 0 && coef0[(long long)zm * NCOEF + 8] != T(0);
    const bool hzp = zp >= 0 && coef0[(long long)zp * NCOEF + 8] != T(0);
    if (need_nb) {
#pragma unroll
        for (int i = 0; i < CPT; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!hzm) cn[i][4][c] = cp[i][c];
                if (!hzp) cn[i][5][c] = cp[i][c];
            }
    }
    // ---- 0. local terms of every cell (Landau, gradient, cross terms); the
    // neighbours are dead afterwards
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    T Eloc[CPT][3];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        T *E = Eloc[i];
        E[0] = E[1] = E[2] = T(0);
        if (!cok[i]) continue;
        const unsigned cb = (unsigned)cip[i] * SZ;
        const T *p = cp[i];
        T sq[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) sq[c] = p[c] * p[c];
        T fg = T(0);
        if (material) {
            if (terms & T_LANDAU) {
#pragma unroll
                for (int c = 0; c < 3; ++c) E[c] -= landau_dfdp(p, sq, coefz, c);
            }
            if (terms & T_GRAD) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T pc = p[c];
                    const T lx = (cn[i][0][c] - pc) + (cn[i][1][c] - pc);
                    const T ly = (cn[i][2][c] - pc) + (cn[i][3][c] - pc);
                    const T lz = (cn[i][4][c] - pc) + (cn[i][5][c] - pc);
                    E[c] += kp->gh2[c][0] * lx + kp->gh2[c][1] * ly + kp->gh2[c][2] * lz;
                    if (MODE == UPD_ENERGY) {
                        // edges towards +x, +y, +z, each counted once
                        const T dx_ = cn[i][1][c] - pc, dy_ = cn[i][3][c] - pc, dz_ = cn[i][5][c] - pc;
                        fg += T(0.5) * (kp->gh2[c][0] * dx_ * dx_ + kp->gh2[c][1] * dy_ * dy_ +
                                        kp->gh2[c][2] * dz_ * dz_);
                    }
                }
                if (MODE == UPD_ENERGY && (kp->g12 != T(0) || kp->gm != T(0))) {
                    // cross terms of eq 4 at the cell (central differences,
                    // missing neighbours = the cell itself)
                    T D[3][3];                               // D[i][d] = D_d P_i
#pragma unroll
                    for (int ci = 0; ci < 3; ++ci)
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            D[ci][d] = (cn[i][2 * d + 1][ci] - cn[i][2 * d][ci]) * kp->inv2h[d];
                    fg += kp->g12 * (D[0][0] * D[1][1] + D[1][1] * D[2][2] + D[2][2] * D[0][0]) +
                          kp->gm * (D[0][1] * D[1][0] + D[1][2] * D[2][1] + D[2][0] * D[0][2]);
                }
                if (a.cross) {                               // their field, from k_cross
                    const T *hx = reinterpret_cast<const T *>(a.cross) + 3LL * b * comp + zoff;
#pragma unroll
                    for (int c = 0; c < 3; ++c) E[c] += ld_at(hx + c * comp, cb);
                }
            }
        }
        if constexpr (MODE == UPD_ENERGY) {
            if (material) {
                if (terms & T_LANDAU) acc[0] += (double)landau_f(sq, coefz);
                acc[1] += (double)fg;
                if (terms & T_EXT)
                    acc[3] += -((double)p[0] * kp->eext[0] + (double)p[1] * kp->eext[1] +
                                (double)p[2] * kp->eext[2]);
                acc[4] += (double)p[0];
                acc[5] += (double)p[1];
                acc[6] += (double)p[2];
            }
        }
        (void)fg;
    }

    if constexpr (!early) {
        if (fftw) field_rows();
    }
    if (do_fx && lwave && !fftw) load_twiddles();
    if (a.elec_in) __syncthreads();                // the field rows are in LDS

    // ---- 2. the electrostatic and applied fields, and the update
    const T dtau = kp->dtau;
    T *Pout = reinterpret_cast<T *>(a.P_out) + 3 * b * comp;
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        if (!cok[i]) continue;
        const int yy = cyy[i], x = cx[i];
        const int off = zoff + cip[i];           // the multistep and RK buffers
        const unsigned cb = (unsigned)cip[i] * SZ;
        const T *p = cp[i];
        (void)off;
        T *E = Eloc[i];
        T hel[3] = {T(0), T(0), T(0)};
        if (a.elec_in) {
#pragma unroll
            for (int c = 0; c < 3; ++c) hel[c] = hs[((c << ysh) + yy) * HS + x];
        }
        if (material) {
            if (a.elec_in) {
#pragma unroll
                for (int c = 0; c < 3; ++c) E[c] += hel[c];
            }
            if (terms & T_EXT) {
#pragma unroll
                for (int c = 0; c < 3; ++c) E[c] += kp->eext[c];
            }
        }
        if constexpr (STEPPING) {
            T o[3];
            if constexpr (MODE == UPD_STEP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (!material) o[c] = T(0);
                    else if (a.stage == 0) o[c] = p[c] + dtau * E[c];
                    else o[c] = T(0.5) * (co[i][c] + p[c]) + T(0.5) * dtau * E[c];
                }
            } else if constexpr (MODE == UPD_STEP_RK) {
                // k_s = E at this stage point; stages 1-6 form the next point
                // P_n + h sum_j A[s][j] k_j, stage 7 the error estimate
                const int st = a.stage;
                const long long ko = 3LL * g.nb * comp;          // one k buffer
                const long long ho = 3LL * b * comp + off;
                T *K = reinterpret_cast<T *>(a.rk_k);
                const T *Pn = reinterpret_cast<const T *>(a.rk_base);
                const T h = (T)a.rk_h;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T e = material ? E[c] : T(0);
                    K[(st - 1) * ko + c * comp + ho] = e;
                    const T pn = Pn[c * comp + ho];
                    if (st < 7) {
                        T acc = T(RK_A[st - 1][st - 1]) * e;
                        for (int j = 0; j < st - 1; ++j)
                            acc += T(RK_A[st - 1][j]) * K[j * ko + c * comp + ho];
                        o[c] = material ? pn + h * acc : T(0);
                    } else {
                        T acc = T(RK_E[6]) * e;
                        for (int j = 0; j < 6; ++j)
                            acc += T(RK_E[j]) * K[j * ko + c * comp + ho];
                        const T sc = T(a.rk_atol) +
                                     T(a.rk_rtol) * (fabs(pn) > fabs(p[c]) ? fabs(pn) : fabs(p[c]));
                        const T r = fabs(h * acc) / sc;
                        rkerr = r > rkerr ? r : rkerr;
                        o[c] = p[c];                             // P5 itself (for the spectrum)
                    }
                }
            } else {
                // multistep stages; the history holds E at the corrected states
                const long long ho = 3LL * b * comp + off;
                const T *ha = reinterpret_cast<const T *>(a.hist_a);
                const T *hb = reinterpret_cast<const T *>(a.hist_b);
                T *hw = reinterpret_cast<T *>(a.hist_w);
                const T k12 = dtau / T(12);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T e = material ? E[c] : T(0);
                    if (a.stage == 0) {
                        o[c] = p[c] + dtau * e;                          // Heun predictor
                    } else if (a.stage == 2) {                           // AB3 predictor
                        const T e1 = ha[c * comp + ho], e2 = hb[c * comp + ho];
                        o[c] = p[c] + k12 * (T(23) * e - T(16) * e1 + T(5) * e2);
                    } else {                                             // AM2 corrector
                        const T en = ha[c * comp + ho], e1 = hb[c * comp + ho];
                        o[c] = co[i][c] + k12 * (T(5) * e + T(8) * en - e1);
                    }
                    if (!material) o[c] = T(0);
                    if (a.stage != 3) hw[c * comp + ho] = e;
                }
            }
            bool bad = false;
            const bool store = !(MODE == UPD_STEP_RK && a.stage == 7);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (store) {
                    if constexpr (NT) st_nt(at(Pout + c * comp + zoff, cb), o[c]);
                    else *at(Pout + c * comp + zoff, cb) = o[c];
                }
                bad = bad || !isfinite(o[c]);
                if (do_fx) hs[((c << ysh) + yy) * HS + x] = o[c];
            }
            if (bad) atomicOr(a.flag, 1);
        } else if constexpr (MODE == UPD_FIELD) {
            const T sc = kp->out_scale;
#pragma unroll
            for (int c = 0; c < 3; ++c) *at(Pout + c * comp + zoff, cb) = material ? sc * E[c] : T(0);
        } else {
            if (material && a.elec_in)
                acc[2] += -0.5 * ((double)p[0] * hel[0] + (double)p[1] * hel[1] +
                                  (double)p[2] * hel[2]);
        }
    }

    // ---- 3. x spectrum of the new rows (half length), written back kx-major
    if (do_fx) __syncthreads();                    // the new rows are in LDS
    if (do_fx && lwave) {
        cpx<T> v[PPT];
        const T *ha = hs + (lact ? l : 0) * HS;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int n = t + q * TPL;
            if (has && 2 * n + 1 < nx) {
                v[q] = *reinterpret_cast<const cpx<T> *>(ha + 2 * n);
            } else {
                v[q] = {(has && 2 * n < nx) ? ha[2 * n] : T(0), T(0)};
            }
        }
        half_fft<T, M2, false, true>(v, L, t, tr, lact);
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            // Z[M2 - k]: as for the inverse; for t = 0 this lane's point
            // (PPT - q) mod PPT
            const int qs = PPT - 1 - q;
            cpx<T> zm_ = {__shfl(v[qs].x, partner, 64), __shfl(v[qs].y, partner, 64)};
            if (t == 0) zm_ = v[(PPT - q) % PPT];
            cpx<T> xh;
            const cpx<T> xk = real_split(v[q], zm_, wk[q], xh);
            if (has) {
                if constexpr (NT) {
                    st_nt(&s1row[s1k(t + q * TPL)], xk);
                    if (t == 0 && q == 0) st_nt(&s1row[s1k(M2)], xh);
                } else {
                    s1row[s1k(t + q * TPL)] = xk;
                    if (t == 0 && q == 0) s1row[s1k(M2)] = xh;
                }
            }
        }
    }

    if constexpr (MODE == UPD_STEP_RK) {
        if (a.stage == 7) {                      // block maximum of the scaled error
            double m = (double)rkerr;
            for (int o2 = 32; o2 > 0; o2 >>= 1) {
                const double v = __shfl_xor(m, o2, 64);
                m = v > m ? v : m;
            }
            __syncthreads();
            double *red = reinterpret_cast<double *>(smem_raw);
            if (lane == 0) red[tid >> 6] = m;
            __syncthreads();
            if (tid == 0) {
                double mm = 0.0;
                for (int w = 0; w < (nthr + 63) / 64; ++w) mm = red[w] > mm ? red[w] : mm;
                a.partials[(long long)tile * 8] = mm;
            }
        }
    }

    if constexpr (MODE == UPD_ENERGY) {
        __syncthreads();
        double *red = reinterpret_cast<double *>(smem_raw);
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            double sacc = acc[k];
            for (int off = 32; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off, 64);
            acc[k] = sacc;
        }
        const int wave = tid >> 6;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 7; ++k) red[wave * 8 + k] = acc[k];
        }
        __syncthreads();
        if (tid < 7) {
            double sacc = 0.0;
            const int nw = (nthr + 63) / 64;
            for (int w = 0; w < nw; ++w) sacc += red[w * 8 + tid];
            a.partials[(long long)tile * 8 + tid] = sacc;
        }
    }
}

// LDS bytes of the update kernel for rows-per-group yt: the rows
// [3 yt][HS] (HS = nx + 2 rounded down to even) and the half-length FFT
// scratch [3 yt][M/2 + M/16].
template <typename T, int M>
static size_t update_lds(const Geom &g, int yt)
{
    const size_t a = ((size_t)3 * yt * ((g.nx + 2) & ~1) * sizeof(T) + 15) / 16 * 16;
    const size_t b = (size_t)3 * yt * LinePad<M / 2>::len * sizeof(cpx<T>);
    size_t tot = a + b;
    if (tot < 16 * 8 * sizeof(double)) tot = 16 * 8 * sizeof(double);
    return tot;
}

// LDS one work-group may use on gfx950 (160 KiB per CU).  Tiles are kept at
// 64 KiB or less where the smallest (two rows) allows; FP64 rows of 512
// cells padded to 1024 points need 80 KiB, and update_prepare raises the
// kernels' limit for them.
constexpr size_t UPD_LDS_MAX = 160 * 1024;

template <typename T, int M>
static size_t update_lds_cap(const Geom &g)
{
    return update_lds<T, M>(g, 2) > 65536 ? UPD_LDS_MAX : 65536;
}

// tpl: threads per line of the half-length transform
static int update_threads(const Geom &g, int yt, int tpl)
{
    int nthr = 3 * yt * tpl;                // one row per line of M/2 points
    if (nthr < 256) nthr = 256;
    if (nthr < (yt * g.nx + 1) / 2) nthr = (yt * g.nx + 1) / 2;   // <= 2 cells per thread
    return (nthr + 63) / 64 * 64;
}

// Rows per work-group: a power of two, limited by threads (<= 2 cells per
// thread, <= 1024 FP32 / 512 FP64 threads) and 64 KiB of LDS.
template <typename T, int M>
static int rows_for(const Geom &g)
{
    const int maxthr = UpdMaxThreads<T>::v;
    const int ny_even = g.ny + (g.ny & 1);
    int best = 2;
    // at most 8 rows for FP32 and 4 for FP64, 2 for rows of 512 points or
    // more (measured best on the 128x128x32 film and the 256x256x64
    // bilayer; tdgl_autotune picks per grid)
    const int ymax = M >= 512 ? 2 : (sizeof(T) == 4 ? 8 : 4);
    for (int yt = 2; yt <= ymax && yt <= (ny_even > 2 ? ny_even : 2); yt *= 2) {
        if (update_threads(g, yt, HalfLine<M / 2>::TPL) > maxthr) break;
        if (yt > 2 && update_lds<T, M>(g, yt) > 65536) break;
        best = yt;
    }
    return best;
}

#define TDGL_ROWS_LEN(T)                                   \
    switch (g.mx) {                                        \
    case 8: return rows_for<T, 8>(g);                      \
    case 16: return rows_for<T, 16>(g);                    \
    case 24: return rows_for<T, 24>(g);                    \
    case 32: return rows_for<T, 32>(g);                    \
    case 48: return rows_for<T, 48>(g);                    \
    case 64: return rows_for<T, 64>(g);                    \
    case 96: return rows_for<T, 96>(g);                    \
    case 128: return rows_for<T, 128>(g);                  \
    case 192: return rows_for<T, 192>(g);                  \
    case 256: return rows_for<T, 256>(g);                  \
    case 384: return rows_for<T, 384>(g);                  \
    case 512: return rows_for<T, 512>(g);                  \
    case 768: return rows_for<T, 768>(g);                  \
    case 1024: return rows_for<T, 1024>(g);                \
    default: return 2;                                     \
    }

int update_rows_per_block(int prec, const Geom &g)
{
    if (prec == PREC_F32) {
        TDGL_ROWS_LEN(float)
    } else {
        TDGL_ROWS_LEN(double)
    }
}

template <typename T, int M, int MODE>
static hipError_t update_impl(const Geom &g, const UpdArgs &a, const void *tw, hipStream_t s,
                              int *nblocks_out)
{
    const int nthr = update_threads(g, a.yt, HalfLine<M / 2>::TPL);
    const size_t shm = update_lds<T, M>(g, a.yt);
    if (shm > update_lds_cap<T, M>(g) || nthr > UpdMaxThreads<T>::v)
        return hipErrorInvalidConfiguration;
    if ((long long)g.nz * g.nb > 65535) return hipErrorInvalidValue;
    dim3 grid((g.ny + a.yt - 1) / a.yt, g.nz * g.nb);
    if (nblocks_out) *nblocks_out = (int)(grid.x * grid.y);
    UpdArgs am = a;
    am.mgx = div_magic(grid.x, (unsigned long long)grid.x * grid.y);
    am.mnz = div_magic((unsigned)g.nz, (unsigned long long)g.nz * g.nb);
    bool launched = false;
    if constexpr (MODE == UPD_STEP) {
        if (g.nt) {
            hipLaunchKernelGGL((k_update<T, M, MODE, true>), grid, dim3(nthr), shm, s, am, g,
                               (const cpx<T> *)tw);
            launched = true;
        }
    }
    if (!launched)
        hipLaunchKernelGGL((k_update<T, M, MODE, false>), grid, dim3(nthr), shm, s, am, g,
                           (const cpx<T> *)tw);
    return hipGetLastError();
}

#define TDGL_MODE_SWITCH(T, LEN)                                                          \
    switch (mode) {                                                                       \
    case UPD_STEP: return update_impl<T, LEN, UPD_STEP>(g, a, tw, s, nblocks_out);        \
    case UPD_STEP_MS: return update_impl<T, LEN, UPD_STEP_MS>(g, a, tw, s, nblocks_out);  \
    case UPD_STEP_RK: return update_impl<T, LEN, UPD_STEP_RK>(g, a, tw, s, nblocks_out);  \
    case UPD_FIELD: return update_impl<T, LEN, UPD_FIELD>(g, a, tw, s, nblocks_out);      \
    default: return update_impl<T, LEN, UPD_ENERGY>(g, a, tw, s, nblocks_out);            \
    }

#define TDGL_UPD_LEN(T)                                        \
    switch (g.mx) {                                            \
    case 8: TDGL_MODE_SWITCH(T, 8)                             \
    case 16: TDGL_MODE_SWITCH(T, 16)                           \
    case 24: TDGL_MODE_SWITCH(T, 24)                           \
    case 32: TDGL_MODE_SWITCH(T, 32)                           \
    case 48: TDGL_MODE_SWITCH(T, 48)                           \
    case 64: TDGL_MODE_SWITCH(T, 64)                           \
    case 96: TDGL_MODE_SWITCH(T, 96)                           \
    case 128: TDGL_MODE_SWITCH(T, 128)                         \
    case 192: TDGL_MODE_SWITCH(T, 192)                         \
    case 256: TDGL_MODE_SWITCH(T, 256)                         \
    case 384: TDGL_MODE_SWITCH(T, 384)                         \
    case 512: TDGL_MODE_SWITCH(T, 512)                         \
    case 768: TDGL_MODE_SWITCH(T, 768)                         \
    case 1024: TDGL_MODE_SWITCH(T, 1024)                       \
    default: return hipErrorInvalidValue;                      \
    }

hipError_t launch_update(int prec, int mode, const Geom &g, const UpdArgs &a, const void *tw,
                         hipStream_t s, int *nblocks_out)
{
    if (prec == PREC_F32) {
        TDGL_UPD_LEN(float)
    } else {
        TDGL_UPD_LEN(double)
    }
}

// Raise the LDS limit of every update kernel of row length M above 64 KiB
// when even the two-row tile needs more (update_lds_cap).
template <typename T, int M>
static hipError_t update_prepare(const Geom &g)
{
    if (update_lds<T, M>(g, 2) <= 65536) return hipSuccess;
    const void *f[6] = {(const void *)k_update<T, M, UPD_STEP, true>,
                        (const void *)k_update<T, M, UPD_STEP, false>,
                        (const void *)k_update<T, M, UPD_FIELD, false>,
                        (const void *)k_update<T, M, UPD_ENERGY, false>,
                        (const void *)k_update<T, M, UPD_STEP_MS, false>,
                        (const void *)k_update<T, M, UPD_STEP_RK, false>};
    for (const void *k : f) {
        const hipError_t e =
            hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)UPD_LDS_MAX);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#define TDGL_PREP_LEN(T)                                   \
    switch (g.mx) {                                        \
    case 512: return update_prepare<T, 512>(g);            \
    case 768: return update_prepare<T, 768>(g);            \
    case 1024: return update_prepare<T, 1024>(g);          \
    default: return hipSuccess;                            \
    }

hipError_t prepare_update(int prec, const Geom &g)
{
    if (prec == PREC_F32) {
        TDGL_PREP_LEN(float)
    } else {
        TDGL_PREP_LEN(double)
    }
}

// ------------------------------------------------------- gradient cross terms
// Field of the cross terms of eq 4 for every cell of every instance
// (see cross_t); vacuum cells get 0.  H: [nb][3][nz][ny][nx].
template <typename T>
__global__ void k_cross(const T *__restrict__ P, T *__restrict__ H, Geom g,
                        const T *__restrict__ coef, const KParams<T> *__restrict__ kp)
{
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int plane = nx * ny;
    const long long comp = (long long)nz * plane;
    const long long ncell = comp * g.nb;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ncell;
         e += (long long)gridDim.x * blockDim.x) {
        const int b = (int)(e / comp);
        if (g.frozen && g.frozen[b]) continue;          // retired: its field is not used
        const int off = (int)(e - (long long)b * comp);
        const int z = off / plane, y = (off - z * plane) / nx, x = off - z * plane - y * nx;
        const T *cf = coef + (long long)b * nz * NCOEF;
        T *Hb = H + 3LL * b * comp;
        if (cf[(long long)z * NCOEF + 8] == T(0)) {
            for (int c = 0; c < 3; ++c) Hb[c * comp + off] = T(0);
            continue;
        }
        const int zm = z > 0 ? z - 1 : (g.pz ? nz - 1 : -1);
        const int zp = z < nz - 1 ? z + 1 : (g.pz ? 0 : -1);
        CrossArgs<T> xa;
        const T *Pb = P + 3LL * b * comp;
        xa.P[0] = Pb;
        xa.P[1] = Pb + comp;
        xa.P[2] = Pb + 2 * comp;
        xa.off = off;
        xa.ex[0] = x > 0 || g.px;
        xa.ex[1] = x < nx - 1 || g.px;
        xa.ex[2] = y > 0 || g.py;
        xa.ex[3] = y < ny - 1 || g.py;
        xa.ex[4] = zm >= 0 && cf[(long long)zm * NCOEF + 8] != T(0);
        xa.ex[5] = zp >= 0 && cf[(long long)zp * NCOEF + 8] != T(0);
        xa.nb[0] = x > 0 ? off - 1 : (g.px ? off + nx - 1 : off);
        xa.nb[1] = x < nx - 1 ? off + 1 : (g.px ? off - nx + 1 : off);
        xa.nb[2] = y > 0 ? off - nx : (g.py ? off + plane - nx : off);
        xa.nb[3] = y < ny - 1 ? off + nx : (g.py ? off - plane + nx : off);
        xa.nb[4] = xa.ex[4] ? off + (zm - z) * plane : off;
        xa.nb[5] = xa.ex[5] ? off + (zp - z) * plane : off;
        for (int d = 0; d < 3; ++d) xa.ih[d] = kp->inv2h[d];
        T cn[6][3];
        for (int d = 0; d < 6; ++d)
            for (int c = 0; c < 3; ++c) cn[d][c] = xa.P[c][xa.nb[d]];
        for (int ci = 0; ci < 3; ++ci) {
            T hm = T(0);
            for (int cj = 0; cj < 3; ++cj) {
                if (cj == ci) continue;
                hm += kp->g12 * cross_t(xa, cn, T(0), cj, ci, cj);
                hm += kp->gm * cross_t(xa, cn, T(0), cj, cj, ci);
            }
            Hb[ci * comp + off] = -hm;
        }
    }
}

hipError_t launch_cross(int prec, const Geom &g, const void *P, void *H, const void *coef,
                        const void *kp, hipStream_t s)
{
    const long long n = (long long)g.nx * g.ny * g.nz * g.nb;
    const unsigned blocks = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (prec == PREC_F32)
        hipLaunchKernelGGL((k_cross<float>), dim3(blocks), dim3(256), 0, s, (const float *)P,
                           (float *)H, g, (const float *)coef, (const KParams<float> *)kp);
    else
        hipLaunchKernelGGL((k_cross<double>), dim3(blocks), dim3(256), 0, s, (const double *)P,
                           (double *)H, g, (const double *)coef, (const KParams<double> *)kp);
    return hipGetLastError();
}

// ------------------------------------------------------------ small kernels
// instance b = blockIdx.x sums its n partials part[b*n .. b*n + n) into out[b*8 ..]
__global__ void k_reduce_partials(const double *__restrict__ part, int n, double *out)
{
    __shared__ double red[256];
    const int tid = threadIdx.x;
    part += (long long)blockIdx.x * n * 8;
    out += blockIdx.x * 8;
    for (int k = 0; k < 8; ++k) {
        double s = 0.0;
        for (int i = tid; i < n; i += 256) s += part[(long long)i * 8 + k];
        red[tid] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) out[k] = red[0];
        __syncthreads();
    }
}

hipError_t launch_reduce_partials(const double *partials, int n, int nb, double *out,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_partials, dim3(nb), dim3(256), 0, s, partials, n, out);
    return hipGetLastError();
}

// Energies in their final units on the device: instance b = blockIdx.x sums
// its n partials (as k_reduce_partials) and writes out[b*8 ..]: the four
// terms times joule (J per reduced unit), their total, and the three
// polarisation sums / ncell * P0.  The products and the sum are evaluated
// exactly as the host does it for tdgl_energies (no contraction), so both
// give the same bits.
__global__ void k_reduce_energies(const double *__restrict__ part, int n, double joule,
                                  double ncell, double P0, double *out)
{
#pragma clang fp contract(off)
    __shared__ double red[256];
    __shared__ double tot[8];
    const int tid = threadIdx.x;
    part += (long long)blockIdx.x * n * 8;
    out += blockIdx.x * 8;
    for (int k = 0; k < 8; ++k) {
        double s = 0.0;
        for (int i = tid; i < n; i += 256) s += part[(long long)i * 8 + k];
        red[tid] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) tot[k] = red[0];
        __syncthreads();
    }
    if (tid == 0) {
        double F[4];
        for (int k = 0; k < 4; ++k) F[k] = tot[k] * joule;
        for (int k = 0; k < 4; ++k) out[k] = F[k];
        out[4] = F[0] + F[1] + F[2] + F[3];
        for (int k = 0; k < 3; ++k) out[5 + k] = ncell > 0.0 ? tot[4 + k] / ncell * P0 : 0.0;
    }
}

hipError_t launch_reduce_energies(const double *partials, int n, int nb, double joule,
                                  double ncell, double P0, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_energies, dim3(nb), dim3(256), 0, s, partials, n, joule, ncell,
                       P0, out);
    return hipGetLastError();
}

// Relaxation test on the device (FP64).  E[b*8 + 4]: total energy of
// instance b (J, k_reduce_energies).  init: Fprev = F, step = -1, frozen = 0,
// counter = 0, stopped = -1.  Otherwise, until every instance has relaxed,
// the step counter advances by `check` and every instance b that has not
// relaxed yet is tested,
//   |F_b - Fprev_b| < rtol * max(|F_b|, floor),
// and on success gets step_b = counter (frozen_b = 1 if retire); Fprev_b = F_b.
// remaining = number of instances with step < 0; when it reaches 0, stopped =
// counter and every instance is frozen, so later launches change nothing.
__global__ void k_relax_test(const double *__restrict__ E, RelaxState r, int nb, int init,
                             long long check, double rtol, double floor, int retire)
{
    __shared__ int cnt[256];
    const int tid = threadIdx.x;
    if (!init && r.stopped[0] >= 0) return;
    const long long n = init ? 0 : r.counter[0] + check;
    int left = 0;
    for (int b = tid; b < nb; b += 256) {
        const double F = E[(long long)b * 8 + 4];
        if (init) {
            r.step[b] = -1;
            r.frozen[b] = 0;
            ++left;
        } else if (r.step[b] < 0) {
            const double dF = fabs(F - r.Fprev[b]);
            const double sc = fabs(F) > floor ? fabs(F) : floor;
            if (dF < rtol * sc) {
                r.step[b] = n;
                if (retire) r.frozen[b] = 1;
            } else {
                ++left;
            }
        }
        r.Fprev[b] = F;
    }
    cnt[tid] = left;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) cnt[tid] += cnt[tid + w];
        __syncthreads();
    }
    const int total = cnt[0];
    if (!init && total == 0)
        for (int b = tid; b < nb; b += 256) r.frozen[b] = 1;
    if (tid == 0) {
        r.remaining[0] = total;
        r.counter[0] = n;
        r.stopped[0] = (!init && total == 0) ? n : -1;
    }
}

hipError_t launch_relax_test(const double *E, const RelaxState &r, int nb, bool init,
                             long long check, double rtol, double floor, bool retire,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_relax_test, dim3(1), dim3(256), 0, s, E, r, nb, init ? 1 : 0, check,
                       rtol, floor, retire ? 1 : 0);
    return hipGetLastError();
}

// Fixed device scratch of the allocation-free energy entry point (energy
// partials of every work-group and instance).  Each device holds its own
// copy for the life of the process.  In host code the name below is not a
// device address: the address of this device's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mutex;
void *scratch_addr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t scratch_address(double **out)
{
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_addr[dev] = p;
    }
    *out = static_cast<double *>(scratch_addr[dev]);
    return hipSuccess;
}

// dst = scale * src, with a precision change if asked (multiply in double)
template <typename S, typename D>
__global__ void k_convert(const S *__restrict__ src, D *__restrict__ dst, size_t n, double scale)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = scale == 1.0 ? (D)src[i] : (D)(scale * (double)src[i]);
}

hipError_t launch_convert(int src_prec, const void *src, int dst_prec, void *dst, size_t n,
                          double scale, hipStream_t s)
{
    const unsigned blocks = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (n == 0) return hipSuccess;
    if (src_prec == PREC_F32 && dst_prec == PREC_F64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(blocks), dim3(256), 0, s,
                           (const float *)src, (double *)dst, n, scale);
    else if (src_prec == PREC_F64 && dst_prec == PREC_F32)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(blocks), dim3(256), 0, s,
                           (const double *)src, (float *)dst, n, scale);
    else if (src_prec == PREC_F32)
        hipLaunchKernelGGL((k_convert<float, float>), dim3(blocks), dim3(256), 0, s,
                           (const float *)src, (float *)dst, n, scale);
    else
        hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks), dim3(256), 0, s,
                           (const double *)src, (double *)dst, n, scale);
    return hipGetLastError();
}

template <typename T>
__global__ void k_zero_layers(T *P, const T *__restrict__ coef, int nz, long long plane)
{
    const int z = blockIdx.y;
    const int c = blockIdx.z % 3, b = blockIdx.z / 3;     // component, instance
    if (coef[((long long)b * nz + z) * NCOEF + 8] != T(0)) return;
    T *row = P + ((long long)(b * 3 + c) * nz + z) * plane;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < plane;
         i += (long long)gridDim.x * blockDim.x)
        row[i] = T(0);
}

hipError_t launch_zero_layers(int prec, void *P, const void *coef, const Geom &g, hipStream_t s)
{
    const long long plane = (long long)g.nx * g.ny;
    const unsigned bx = (unsigned)((plane + 255) / 256 < 1024 ? (plane + 255) / 256 : 1024);
    dim3 grid(bx, g.nz, 3 * g.nb);
    if (prec == PREC_F32)
        hipLaunchKernelGGL((k_zero_layers<float>), grid, dim3(256), 0, s, (float *)P,
                           (const float *)coef, g.nz, plane);
    else
        hipLaunchKernelGGL((k_zero_layers<double>), grid, dim3(256), 0, s, (double *)P,
                           (const double *)coef, g.nz, plane);
    return hipGetLastError();
}

}  // namespace tdgl
