// Declarations shared by the host API (tdgl_api.cpp) and the HIP kernel
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace tdgl {

constexpr int NCOEF = 12;      // per z layer: a1x a1y a1z a11 a12 a111 a112 a123, material, pad
constexpr int MAXLEN = 1024;   // largest FFT length
// twiddle tables of every length L (W_L^k, k < L): powers of two at offset L,
// lengths 3 * 2^a at 2 MAXLEN + L (tw_off in fft_core.h)
constexpr int TW_ENTRIES = 4 * MAXLEN;
__host__ __device__ constexpr int tw_off(int L)
{
    return (L & (L - 1)) == 0 ? L : 2 * MAXLEN + L;
}
constexpr int GL_MAXN = 24;    // Gauss-Legendre table rows/columns

enum { PREC_F32 = 0, PREC_F64 = 1 };

// The x spectra (S1) and y spectra (S2) of a context are stored in blocks of
// KB consecutive kx: element (kx, row) at ((kx / KB) * rows + row) * KB +
// kx % KB, where row = ((b*3 + c)*nz + z)*L + y runs over all rows of all
// instances (L = ny for S1, my for S2).  A work-group of the update kernel,
// which reads and writes yt consecutive rows for every kx, then touches
// whole 128-byte lines (yt * KB * 8 bytes per block), the y passes read and
// write KB lines side by side, and the z pass reads tiles of (ky, kx)
// columns.  The buffers hold hx rounded up to a multiple of KB.
constexpr int KB = 4;
constexpr int KBS = 2;                  // log2(KB)
__host__ __device__ constexpr int hx_blocked(int hx) { return (hx + KB - 1) / KB * KB; }
enum { T_LANDAU = 1, T_GRAD = 2, T_ELEC = 4, T_EXT = 8 };

// Device-resident scalars read by the update kernel (can change between
// graph launches without re-capturing).
template <typename T>
struct KParams {
    T dtau;          // reduced time step
    T eext[3];       // reduced applied field
    T gh2[3][3];     // g[i][d] / h_d^2: gradient coefficient of component i along d
    T out_scale;     // V/m per reduced field unit (field output)
    T g12, gm;       // cross terms of the gradient energy: G12, G44 - G44' (reduced)
    T inv2h[3];      // 1 / (2 h_d), reduced cell sizes
    T pad[3];
};

struct Geom {
    int nx, ny, nz;      // physical cells
    int mx, my, mz;      // padded FFT lengths
    int hx;              // mx/2 + 1
    int px, py, pz;      // periodic flags
    int nb = 1;          // instances of this grid advanced together (batch)
    // per-instance flags (device, nb ints) of instances that no longer
    // advance (relaxed and retired): the FFT passes skip their lines and the
    // update kernel copies their state unchanged; null = none
    const int *frozen = nullptr;
    // the step kernels' stores of spectra and states are non-temporal (a
    // per-context choice, see st_nt)
    int nt = 0;
};

// Frozen-instance test for kernels that see flat line or row indices:
// index i belongs to instance (i / per) % nb.
struct Freeze {
    const int *flag = nullptr;
    long long per = 1;
    int nb = 1;
    __device__ __forceinline__ bool skip(long long i) const
    {
        return flag && flag[(int)((i / per) % nb)];
    }
};

// Update kernel modes.  UPD_STEP_MS: stages of the multistep scheme
// (0: Heun predictor that also stores E; 2: Adams-Bashforth predictor that
// stores E; 3: Adams-Moulton corrector).
// UPD_STEP_RK: stage s = 1..7 of the RK45 step (stages 1-6 store k_s and
// form the next stage point; stage 7 stores k_7 and reduces the error).
enum { UPD_STEP = 0, UPD_FIELD = 1, UPD_ENERGY = 2, UPD_STEP_MS = 3, UPD_STEP_RK = 4 };

struct UpdArgs {
    const void *P_in;      // state the field is evaluated at
    const void *P_old;     // Heun corrector: state at the start of the step
    void *P_out;           // new state (STEP) or field (FIELD)
    void *S1;              // x spectra in kx blocks of KB (above): field in, new P spectrum out
    const void *coef;      // [nz][NCOEF]
    const void *kp;        // KParams<T>
    double *partials;      // ENERGY: [grid][8]
    int *flag;             // non-finite flag
    int stage;             // STEP: 0 = P_in + dtau E, 1 = (P_old + P_in)/2 + dtau/2 E
    unsigned terms;        // term mask for this evaluation
    int elec_in;           // read the electrostatic field rows from S1
    int fx_out;            // write the x-spectrum of P_out to S1
    int yt;                // rows per work-group (a power of two)
    void *hist_w;          // STEP_MS stages 0, 2: E of P_in is stored here
    const void *hist_a;    // STEP_MS stage 2: E_{n-1}; stage 3: E_n
    const void *hist_b;    // STEP_MS stage 2: E_{n-2}; stage 3: E_{n-1}
    const void *rk_base;   // STEP_RK: P_n
    void *rk_k;            // STEP_RK: k_1..k_7, each [nb][3][nz][ny][nx]
    double rk_h;           // STEP_RK: step size
    double rk_atol, rk_rtol;
    const void *cross;     // field of the gradient cross terms (k_cross), or null
    unsigned mgx, mnz;     // magic numbers of the launch's grid divisions (set by the launcher)
};

// field of the cross terms of the gradient energy (G12, G44 - G44') of P
hipError_t launch_cross(int prec, const Geom &g, const void *P, void *H, const void *coef,
                        const void *kp, hipStream_t s);

// x pass: output element k of row r at out[k*out_kstride + r] (kx-major), or,
// with blocked (out_kstride = number of rows), in the KB-blocked layout above
hipError_t launch_fx(int prec, int M, const void *in, long long nrows, int n_in,
                     long long in_stride, void *out, long long out_kstride,
                     const void *tw, hipStream_t s, Freeze fz = {}, bool blocked = false);
hipError_t launch_row(int prec, int M, bool inv, const void *in, void *out, long long nlines,
                      long long in_stride, long long out_stride, int n_in, int n_out,
                      const void *tw, hipStream_t s, Freeze fz = {});
// y pass between the KB-blocked x spectra S1 (lines of ny points, rows per
// kx: R = nb*3*nz) and the KB-blocked y spectra S2 (lines of my points):
// forward S1 -> S2, inverse S2 -> S1
hipError_t launch_row_blocked(int prec, int M, bool inv, const void *S1, void *S2, int hx,
                              long long R, int ny, int my, int n_in, int n_out, const void *tw,
                              hipStream_t s, Freeze fz, int nt);
// once per context, outside graph capture: lets the blocked y passes of
// length M use more than 64 KiB of LDS where they need it
hipError_t prepare_row_blocked(int prec, int M);
hipError_t launch_plane(int prec, const Geom &g, void *S1, const void *Nt, const void *tw,
                        size_t lds_max, hipStream_t s, bool query);
hipError_t launch_col(int prec, int M, bool inv, const void *in, void *out, long long C,
                      long long nbatch, long long in_bstride, long long out_bstride,
                      long long lstride, int n_in, int n_out, const void *tw, hipStream_t s);
// z pass with the tensor multiply; tile_bytes: bytes per z row of a column
// tile (64, 128, 256; 0 = zmul_auto_tile)
hipError_t launch_zmul(int prec, const Geom &g, void *S, const void *Nt, const void *tw,
                       int tile_bytes, hipStream_t s);
int zmul_auto_tile(int prec, const Geom &g);
hipError_t launch_update(int prec, int mode, const Geom &g, const UpdArgs &a,
                         const void *tw, hipStream_t s, int *nblocks_out);
int update_rows_per_block(int prec, const Geom &g);
// Raise the LDS limits of the update kernels and of the x pass above 64 KiB
// where their smallest tiles need it (FP64 at 1024 points); once per device
hipError_t prepare_update(int prec, const Geom &g);
hipError_t prepare_fx(int prec, int M);
hipError_t launch_reduce_partials(const double *partials, int n, int nb, double *out,
                                  hipStream_t s);
// final energies [nb][8] (J and C/m^2, as tdgl_energies_batch) from the partials
hipError_t launch_reduce_energies(const double *partials, int n, int nb, double joule,
                                  double ncell, double P0, double *out, hipStream_t s);
// relaxation bookkeeping on the device (tdgl_relax), nb entries each
struct RelaxState {
    double *Fprev;        // total energy at the previous check (J)
    long long *step;      // step at which the instance relaxed, -1 = not yet
    int *frozen;          // retired instances (Geom::frozen)
    long long *counter;   // steps done since the relaxation started
    long long *stopped;   // counter when the last instance relaxed, -1 before
    int *remaining;       // instances not relaxed yet
};
hipError_t launch_relax_test(const double *E, const RelaxState &r, int nb, bool init,
                             long long check, double rtol, double floor, bool retire,
                             hipStream_t s);
// fixed device scratch of the allocation-free entry point: SCRATCH_DOUBLES
// doubles per device; *out = this device's address (current device)
constexpr size_t SCRATCH_DOUBLES = 131072;        // 1 MiB
hipError_t scratch_address(double **out);
hipError_t launch_convert(int src_prec, const void *src, int dst_prec, void *dst, size_t n,
                          double scale, hipStream_t s);
hipError_t launch_zero_layers(int prec, void *P, const void *coef, const Geom &g, hipStream_t s);

// tensor construction (FP64)
hipError_t launch_tensor_real(const Geom &g, unsigned pmask, int mimg, double dx, double dy,
                              double dz, const double *gl_t, const double *gl_w, double *R,
                              hipStream_t s);
hipError_t launch_tensor_k0(const Geom &g, unsigned pmask, double *R, double *sums,
                            hipStream_t s);
hipError_t launch_tensor_octant(int prec, const Geom &g, const void *C, double scale, void *Nt,
                                hipStream_t s);

}  // namespace tdgl
