/*
 * tdgl.h — C ABI of libtdgl: one time-dependent Ginzburg-Landau (TDGL) time
 * step of the full three-component polarisation P on a 3-D finite-difference
 * grid, on an AMD Instinct MI355X (gfx950).
 *
 * The method (paper section 2): dP/dt = -L dF/dP (eq 1) with
 * F = F_Land + F_Grad + F_Elec + F_Ext (eq 2): sixth-order Landau energy
 * (eq 3), gradient energy (eq 4), electrostatic energy of the bound charges
 * (eqs 5-6, finite sample in vacuum, P = 0 outside), applied-field energy
 * (eq 7).  Section 3: P uniform in each cell, per-cell materials, time-
 * dependent excitation, several explicit integrators, per-term on/off flags,
 * Table 2 normalisation.  The electrostatic field is a zero-padded FFT
 * convolution with the cell-averaged dipolar tensor.
 *
 * Conventions shared by all entry points
 *  - Units at the boundary are SI: P in C/m^2, fields in V/m, T in K,
 *    lengths in m, energies in J.  Internally the library works in the
 *    reduced units of Table 2 with a fixed reference stiffness alpha_ref
 *    (tdgl_set_scales); the time step dtau is given in reduced time
 *    tau = alpha_ref * L * t with L = 1.
 *  - Arrays of P and of fields are structure-of-arrays [3][nz][ny][nx]
 *    (component slowest, x fastest), row-major, densely packed.
 *  - Every call returns a tdgl_status; nothing is thrown across the ABI.
 *    On an argument error the context is left unchanged.  The message of
 *    the last failure is available from tdgl_last_error.
 *  - Device work is enqueued on the HIP stream given to tdgl_create, in
 *    call order.  Calls documented as "synchronising" wait for that stream.
 *  - A context is not thread-safe.  Separate contexts are independent.
 *  - Pointers passed in are borrowed for the duration of the call only,
 *    except a workspace bound with tdgl_bind_workspace.
 */
#ifndef TDGL_H
#define TDGL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDGL_ABI_VERSION 1

typedef struct tdgl_ctx tdgl_ctx;

typedef enum {
    TDGL_OK = 0,
    TDGL_E_ARG = -1,          /* invalid argument; context unchanged          */
    TDGL_E_NOMEM = -2,        /* device allocation failed                     */
    TDGL_E_HIP = -3,          /* HIP runtime error (no device, launch failure)*/
    TDGL_E_NONFINITE = -4,    /* a non-finite P appeared during tdgl_step     */
    TDGL_E_STATE = -5,        /* call out of order (e.g. step before set_P)   */
    TDGL_E_UNSUPPORTED = -6   /* valid input this library does not handle     */
} tdgl_status;

enum { TDGL_FP32 = 0, TDGL_FP64 = 1 };            /* arithmetic of the step     */
enum { TDGL_EULER = 0, TDGL_HEUN = 1, TDGL_AB3M2 = 2, TDGL_RK45 = 3 };   /* integrators */
/* energy terms (section 3: each contribution can be switched on or off) */
enum { TDGL_LANDAU = 1, TDGL_GRAD = 2, TDGL_ELEC = 4, TDGL_EXT = 8, TDGL_ALL = 15 };

/* Grid (section 3, finite differences with P uniform per cell).
 * periodic_mask: bit0 x, bit1 y, bit2 z.  Supported: 0 (open box in vacuum,
 * the paper's setting), 3 (film periodic in x and y, open in z) and 7
 * (fully periodic).  Open dimensions are zero-padded to the smallest power
 * of two >= max(8, 2n-1), or in x and y to 3 * 2^a (>= 24) where that is
 * smaller (96 cells: 192); a periodic dimension needs n a power of two in
 * [8, 1024].  Padded lengths must not exceed 1024, and an FP64 context
 * takes rows of at most 512 cells (nx <= 512; the time-step kernel's
 * smallest tile must fit 512 threads); tdgl_create returns
 * TDGL_E_UNSUPPORTED otherwise.  tdgl_get_dims reports the padded lengths. */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;            /* cell edge lengths, m                      */
    unsigned periodic_mask;
} tdgl_grid;

/* Landau coefficients of one material (eq 3), forms of Table 1:
 *   a1_form 0: alpha1(T) = a1_slope * (T - a1_T0)
 *   a1_form 1: alpha1(T) = a1_A * (coth(a1_Ts/T) - coth(a1_Ts/a1_T0))
 *   alpha11(T)  = a11_slope  * (T - a11_Tref)  + a11_offset
 *   alpha111(T) = a111_slope * (T - a111_Tref) + a111_offset
 *   alpha12, alpha112, alpha123 constant.
 * rs scales the z part of the quadratic term (strain parameter of the
 * skyrmion study, section 4.4): alpha1 (Px^2 + Py^2) + rs alpha1 Pz^2.
 * SI units as in Table 1. */
typedef struct {
    int a1_form;
    double a1_slope, a1_T0, a1_A, a1_Ts;
    double a11_slope, a11_Tref, a11_offset;
    double a12;
    double a111_slope, a111_Tref, a111_offset;
    double a112, a123;
    double rs;
} tdgl_material;

#define TDGL_MAX_MATERIALS 16

/* ABI version of the loaded library (TDGL_ABI_VERSION at build time). */
int tdgl_abi_version(void);

/* Create a context for one simulation.  precision: TDGL_FP32 or TDGL_FP64
 * (arithmetic of the step; tensor construction and energy sums are always
 * FP64).  hip_stream: a hipStream_t (NULL = default stream).  No device
 * memory is touched until the first call that needs it.
 * Errors: TDGL_E_ARG (bad sizes or mask), TDGL_E_UNSUPPORTED (FFT length,
 * or 2^31 cells or more). */
tdgl_status tdgl_create(const tdgl_grid *grid, int precision, void *hip_stream,
                        tdgl_ctx **out);

/* A context holding nbatch independent simulations of the same grid and
 * model (materials, layer map, gradient, scales, tensor, E_ext, integrator)
 * that may differ in temperature and state: every kernel of a step covers
 * all instances in one launch.  The paper runs many simulations in
 * parallel to cut the total cost (section 3) and relaxes batches of
 * single-cell runs from random starts (section 4.2).  State arrays gain a
 * leading instance dimension: P is [nbatch][3][nz][ny][nx].  Instance
 * results are identical to those of nbatch separate contexts.
 * tdgl_create is tdgl_create_batch with nbatch = 1.  Errors as tdgl_create;
 * TDGL_E_ARG for nbatch outside 1..4096, TDGL_E_UNSUPPORTED when
 * nz * nbatch exceeds 65535. */
tdgl_status tdgl_create_batch(const tdgl_grid *grid, int nbatch, int precision,
                              void *hip_stream, tdgl_ctx **out);

/* Number of instances of the context. */
tdgl_status tdgl_get_batch(const tdgl_ctx *ctx, int *nbatch);

/* Release the context and all device memory it allocated.  NULL is a no-op. */
void tdgl_destroy(tdgl_ctx *ctx);

/* Message of the last failed call on ctx (empty if none).  Owned by ctx. */
const char *tdgl_last_error(const tdgl_ctx *ctx);

/* dims out[7]: nx, ny, nz, padded mx, my, mz, hx = mx/2+1. */
tdgl_status tdgl_get_dims(const tdgl_ctx *ctx, int out[7]);

/* Bytes of device workspace the context needs for its state, spectra,
 * tensor, relaxation bookkeeping, the field of the gradient cross terms and
 * the buffers of the integrator set at the time of the call (AB3M2: three
 * P-sized field histories; RK45: eight P-sized stage buffers), tensor
 * construction temporaries excluded.  Set the integrator first. */
tdgl_status tdgl_workspace_size(const tdgl_ctx *ctx, size_t *bytes);

/* Hand the context caller-owned device memory (e.g. a torch tensor) of at
 * least tdgl_workspace_size bytes, 256-byte aligned, instead of letting it
 * allocate: every buffer of every step then lives in it.  Must precede every
 * call that touches the device; the memory must outlive the context.  A
 * later switch to an integrator whose buffers do not fit makes tdgl_step
 * fail with TDGL_E_STATE.  Without a bound workspace the library allocates
 * its own, and the buffers of a later integrator switch separately.
 * Errors: TDGL_E_ARG (size, alignment), TDGL_E_STATE (device memory already
 * allocated). */
tdgl_status tdgl_bind_workspace(tdgl_ctx *ctx, void *dev_ptr, size_t bytes);

/* Normalisation of Table 2: P0 (C/m^2), alpha_ref (N m^2 C^-2, > 0, used in
 * place of |alpha1(T)| so reduced time is the same at every temperature),
 * G110 (N m^4 C^-2), eps_b (background permittivity, section 2). */
tdgl_status tdgl_set_scales(tdgl_ctx *ctx, double P0, double alpha_ref, double G110,
                            double eps_b);

/* Define material id (0 <= id < TDGL_MAX_MATERIALS). */
tdgl_status tdgl_set_material(tdgl_ctx *ctx, int id, const tdgl_material *mat);

/* Material of every z layer (section 3: spatially varying parameters),
 * ids[nz]; -1 marks a vacuum layer, where P is held at zero. */
tdgl_status tdgl_set_layer_materials(tdgl_ctx *ctx, const signed char *ids);

/* Gradient coefficients of eq 4 (N m^4 C^-2), the same for the whole
 * sample.  Discretised as an energy: squared derivatives on the cell
 * edges (G11 along the component, G44 + G44' across, the 7-point stencil)
 * plus, for the cross products G12 P_i,i P_j,j and (G44 - G44') P_i,j P_j,i,
 * cell-centred central differences in which a missing neighbour (open
 * surface, vacuum) takes the cell's own value; the field is minus the
 * exact gradient of that discrete energy, in the interior
 * G11 d_ii P_i + (G44 + G44') d_jj P_i + (G12 + G44 - G44') d_ij P_j. */
tdgl_status tdgl_set_gradient(tdgl_ctx *ctx, double G11, double G12, double G44,
                              double G44p);

/* Build the electrostatic interaction tensor on the device in FP64 (eq 6 for
 * cell-wise uniform P: cell-averaged dipolar tensor, closed form for touching
 * cells and Gauss-Legendre quadrature elsewhere; periodic dimensions sum
 * lattice images |offset| <= (mimg + 1/2) * n and fix the in-plane k = 0
 * mode to its infinite-lattice value), transform it and keep one octant of
 * the real spectrum with -kappa/(mx my mz) folded in.  Needs set_scales.
 * Synchronising.  Temporaries of about 24 * mx*my*mz bytes are allocated for
 * the duration of the call.  mimg in [0, 64]. */
tdgl_status tdgl_build_tensor(tdgl_ctx *ctx, int mimg);

/* Copy the tensor octant spectrum ([hx][6][mz/2+1][my/2+1], component order
 * xx yy zz xy xz yz, -kappa/(mx my mz) folded in, converted to double) to
 * host memory dst of count doubles.  Synchronising.  For tests and
 * inspection. */
tdgl_status tdgl_get_tensor_spectrum(tdgl_ctx *ctx, double *dst, size_t count);

/* Temperature (K) for the Table 1 coefficient forms, for every instance. */
tdgl_status tdgl_set_temperature(tdgl_ctx *ctx, double T_kelvin);

/* Temperature of each instance: T_kelvin[nbatch] (host memory).  The
 * reduced scales stay shared (one alpha_ref), so only the Landau
 * coefficients differ between instances. */
tdgl_status tdgl_set_temperatures(tdgl_ctx *ctx, const double *T_kelvin);

/* Uniform applied field E_ext (V/m), eq 7.  May change between tdgl_step
 * calls (time-dependent excitation, section 3). */
tdgl_status tdgl_set_eext(tdgl_ctx *ctx, double ex, double ey, double ez);

/* Energy terms in the effective field (TDGL_* bits). */
tdgl_status tdgl_set_terms(tdgl_ctx *ctx, unsigned mask);

/* Integrator and reduced time step dtau > 0 (section 3 lists the
 * schemes): TDGL_EULER; TDGL_HEUN (predictor P~ = P + dtau E(P), corrector
 * (P + P~)/2 + dtau/2 E(P~)); TDGL_AB3M2, the multistep scheme read as the
 * third-order Adams-Bashforth predictor with the two-step Adams-Moulton
 * corrector, two field evaluations per step, started by two Heun steps.
 * AB3M2 keeps the fields of the last two steps in three P-sized device
 * buffers (see tdgl_workspace_size), and tdgl_set_P, this call and
 * tdgl_autotune restart it (the next two steps are Heun steps).
 * TDGL_RK45: the adaptive Dormand-Prince 5(4) pair, seven field evaluations
 * per attempt; dtau is the first trial step, tdgl_step(n) makes n accepted
 * steps (see tdgl_set_rk_tolerances); RK45 steps are launched eagerly and
 * synchronise once per attempt.  This call resets the RK45 time and step. */
tdgl_status tdgl_set_integrator(tdgl_ctx *ctx, int scheme, double dtau);

/* RK45 error control: an attempt is accepted when, over every cell and
 * component of every instance, |h sum_j (b_j - b*_j) k_j| <= atol +
 * rtol max(|P_n|, |P_n+1|) (reduced units, P/P0); the next step is h times
 * min(5, max(0.2, 0.9 err^-1/5)) after acceptance, max(0.2, 0.9 err^-1/5)
 * after rejection (a batch shares one step size).  Defaults 1e-8, 1e-6.
 * Errors: TDGL_E_ARG for negative, non-finite or both-zero tolerances. */
tdgl_status tdgl_set_rk_tolerances(tdgl_ctx *ctx, double atol, double rtol);

/* RK45 progress since tdgl_set_integrator: reduced time of the accepted
 * steps, the current step size and the number of rejected attempts. */
tdgl_status tdgl_get_rk_state(const tdgl_ctx *ctx, double *tau, double *h, long long *rejected);

/* Number of steps captured per HIP graph by tdgl_step (default 64; 0 runs
 * plain stream launches).  tdgl_step(n) launches n / steps graphs of that
 * chunk and the remainder as one graph of its own length; instantiated
 * graphs are cached per length and launch configuration (the cache is
 * emptied when it holds 32 graphs and a new remainder length comes). */
tdgl_status tdgl_set_graph_chunk(tdgl_ctx *ctx, int steps);

/* FFT pass layout: path 0 (default) fuses the y pass, the z pass with the
 * tensor multiply and the inverse y pass into one kernel per kx plane when
 * that plane fits in one work-group's LDS, and uses three kernels
 * otherwise; path 1 always uses the three kernels.  Results agree to
 * rounding.  tdgl_get_fft_path reports whether the fused kernel is in use
 * (known after the first call that touches the device). */
tdgl_status tdgl_set_fft_path(tdgl_ctx *ctx, int path);
tdgl_status tdgl_get_fft_path(const tdgl_ctx *ctx, int *fused);

/* Rows of one z layer handled by one work-group of the update kernel (a
 * power of two, 2..64; 0 restores the built-in choice).  A tuning knob: results do not
 * depend on it.  Launches that would exceed the device's work-group limits
 * fail with TDGL_E_HIP at the next step. */
tdgl_status tdgl_set_update_rows(tdgl_ctx *ctx, int rows);

/* Column tile of the z pass: bytes of each z row a work-group loads (64,
 * 128 or 256; 0 restores the built-in choice: 128, or 64 where that leaves
 * fewer than 1024 work-groups).  A tuning knob: results do not depend on
 * it.  tdgl_get_z_tile reports the tile in use (the built-in choice
 * resolved). */
tdgl_status tdgl_set_z_tile(tdgl_ctx *ctx, int row_bytes);
tdgl_status tdgl_get_z_tile(const tdgl_ctx *ctx, int *row_bytes);

/* How the step kernels store the spectra and states that the next kernel
 * reads: 1 non-temporal (streamed past the L2), 2 plain, 0 the built-in
 * choice (non-temporal for a single instance, plain for a batch, as measured
 * on the 128x128x32 film, the 256x256x64 bilayer and batches of small boxes).
 * A tuning knob: results do not depend on it.  tdgl_get_store_mode reports
 * 1 or 2. */
tdgl_status tdgl_set_store_mode(tdgl_ctx *ctx, int mode);
tdgl_status tdgl_get_store_mode(const tdgl_ctx *ctx, int *mode);

/* Load P (C/m^2, [nbatch][3][nz][ny][nx]) from src: host memory if
 * src_on_device is 0, device memory otherwise; src_precision TDGL_FP32 or TDGL_FP64 (converted
 * to the context precision).  P is the state variable of eq 1, uniform in
 * each cell (section 3); it is kept as P/P0 (Table 2).  Vacuum layers are set to zero and the
 * non-finite flag is cleared.  Needs the model to be complete (scales,
 * every material named by the layer map, gradient coefficients when the
 * gradient term is on).  Host sources are copied before return. */
tdgl_status tdgl_set_P(tdgl_ctx *ctx, const void *src, int src_on_device, int src_precision);

/* Store the current P to dst (layout of tdgl_set_P; host or device, FP32 or
 * FP64), converted back from P/P0 (Table 2) to C/m^2.  Host
 * destinations are synchronising and report TDGL_E_NONFINITE like
 * tdgl_sync (the data is copied either way). */
tdgl_status tdgl_get_P(tdgl_ctx *ctx, void *dst, int dst_on_device, int dst_precision);

/* Advance nsteps time steps of eq 1 in reduced time (Table 2, L = 1) with the
 * integrator of tdgl_set_integrator (section 3: explicit schemes, Heun
 * named); each field evaluation is E_eff = -dF/dP of eq 2 with the terms
 * of eqs 3-7 that tdgl_set_terms switches on (one Euler step = 1 field
 * evaluation, one Heun step = 2).  Asynchronous: a non-finite P produced by a step is recorded on
 * the device and reported as TDGL_E_NONFINITE by the next tdgl_sync,
 * tdgl_energies or host tdgl_get_P; P then holds the bad state (restore a
 * copy taken with tdgl_get_P and retry with a smaller dtau).  Needs set_P,
 * and build_tensor when the electrostatic term is on. */
tdgl_status tdgl_step(tdgl_ctx *ctx, long long nsteps);

/* Effective field E_eff = -dF/dP (V/m) of the current P, eq 1 with eq 2:
 * the Landau (eq 3), gradient (eq 4), electrostatic (eqs 5-6) and applied
 * (eq 7) fields in mask (a subset of TDGL_ALL), written to device memory dst_dev
 * ([nbatch][3][nz][ny][nx], context precision).  Vacuum cells get 0. */
tdgl_status tdgl_eval_field(tdgl_ctx *ctx, unsigned mask, void *dst_dev);

/* Energies of the current P with the context's term mask, in J (eq 2 and
 * its terms, eqs 3-7, summed over the cells of volume dx dy dz; the
 * electrostatic term is -1/2 sum P.E_elec, eq 5):
 * F[0] Landau, F[1] gradient, F[2] electrostatic, F[3] external, F[4] total;
 * meanP[3]: mean P over material cells (C/m^2).  FP64 accumulation.
 * Synchronising.  For a batch: instance 0. */
tdgl_status tdgl_energies(tdgl_ctx *ctx, double F[5], double meanP[3]);

/* tdgl_energies for every instance: F[nbatch][5], meanP[nbatch][3] (host
 * memory). */
tdgl_status tdgl_energies_batch(tdgl_ctx *ctx, double *F, double *meanP);

/* Allocation-free variant of tdgl_energies_batch, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Enqueues the energy evaluation
 * of every instance on the context's stream and writes out_dev[nbatch][8]
 * in device memory (caller-owned, 8-byte aligned): F_Land, F_Grad, F_Elec,
 * F_Ext, F total (J), mean P x, y, z over material cells (C/m^2) -- the
 * same values, bit for bit, as tdgl_energies_batch.  Asynchronous: nothing
 * waits for the stream and the non-finite flag is not read.
 * Scratch: the per-work-group partial sums go to a fixed device array of
 * TDGL_NOALLOC_SCRATCH_BYTES per device, which the library holds from the
 * first call on that device until the process ends; the call needs
 * 64 * nbatch * nz * ceil(ny / rows) bytes of it (rows: the update tile,
 * tdgl_set_update_rows) and fails with TDGL_E_UNSUPPORTED, before enqueuing
 * anything, when that exceeds the limit.  Every call on a device shares that
 * device's array: calls that overlap on one device (different streams, or
 * concurrent threads) race and give wrong results; calls on one stream are
 * ordered and safe.  Nothing of a previous call is reused.
 * Needs P to be set (the context's own buffers exist then: this call never
 * allocates them).  Model changes since the last step are uploaded first,
 * which waits for the stream; under capture, make them before capturing. */
#define TDGL_NOALLOC_SCRATCH_BYTES (1u << 20)
tdgl_status tdgl_energies_noalloc(tdgl_ctx *ctx, double *out_dev);

/* Relax every instance to the energy criterion (the relaxed states of the
 * paper's parallel runs, sections 3 and 4.2; the paper gives no criterion,
 * this library's reading): the instances advance in calls of `check` steps
 * and after each the total energy F of every instance (eq 2, FP64, as
 * tdgl_energies_batch) is compared on the device with its value `check`
 * steps earlier; instance b has relaxed at step n when
 *   |F_b(n) - F_b(n - check)| < rtol * max(|F_b(n)|, floor),
 *   floor = floor_factor * alpha_ref * P0^2 * nx*ny*nz*dx*dy*dz  (J).
 * relax_step[nbatch] (host) receives n, or -1 if the instance did not relax
 * within max_steps (the last call may pass max_steps by less than check);
 * *steps_taken (may be NULL) the steps done, which stop at the first check
 * where every instance has relaxed.  retire = 1: an instance stops
 * advancing at the check where it relaxed (its P stays that state, and its
 * lines are skipped by every kernel); retire = 0: all advance until the last
 * one relaxes.  Euler and Heun run as captured graphs of up to 5000 steps
 * with the energies and the test inside, synchronising once per graph;
 * AB3M2 and RK45 advance through tdgl_step, synchronise once per check and
 * ignore retire.  Errors as tdgl_step; TDGL_E_ARG for check outside
 * 1..1e6, max_steps < 0, rtol <= 0, floor_factor < 0, retire not 0/1. */
tdgl_status tdgl_relax(tdgl_ctx *ctx, long long check, long long max_steps, double rtol,
                       double floor_factor, int retire, long long *relax_step,
                       long long *steps_taken);

/* tdgl_relax for nctx contexts at once, e.g. batches of different grid
 * shapes (the paper's many parallel simulations, section 3): every captured
 * graph holds each context's steps, energies and tests as parallel branches
 * (one graph per chunk of up to 5000 steps across all the shapes), launched
 * on the first context's stream after the other contexts' earlier work;
 * their later work waits for it.  Same arguments and criterion as
 * tdgl_relax; relax_step receives the instances of every context in order
 * (sum of their nbatch entries); *steps_taken is the largest of the
 * contexts'.  Every context must use Euler or Heun with graphs on
 * (TDGL_E_UNSUPPORTED otherwise) and live on one device.  Errors of a
 * context are reported by its tdgl_last_error. */
tdgl_status tdgl_relax_group(tdgl_ctx *const *ctxs, int nctx, long long check,
                             long long max_steps, double rtol, double floor_factor, int retire,
                             long long *relax_step, long long *steps_taken);

/* Quasi-static field sweep (the paper drives samples with a time-dependent
 * external field, section 3, and traces P against E in section 4.4): for
 * each of the nvalues applied fields e[i][3] (V/m, host memory) in turn,
 * set E_ext, advance steps_per_value steps and record the mean P of every
 * instance in meanP[nvalues][nbatch][3] (C/m^2) and, if F is not NULL, the
 * energies in F[nvalues][nbatch][5] (J).  A triangle wave in E_z gives the
 * hysteresis loop P_z(E_z).  Synchronising once per value; E_ext keeps the
 * last value.  Errors as tdgl_step and tdgl_energies. */
tdgl_status tdgl_sweep_eext(tdgl_ctx *ctx, const double *e, int nvalues,
                            long long steps_per_value, double *meanP, double *F);

/* Reduced per-layer Landau coefficients ([nz][8]: a1x a1y a1z a11 a12 a111
 * a112 a123, zero for vacuum; instance 0 of a batch) and scalars out[8]:
 * kappa, hx*, hy*, hz*, dV*, energy scale (J), field scale (V/m), l0 (m).
 * Host-side; for tests. */
tdgl_status tdgl_get_reduced(const tdgl_ctx *ctx, double *coef, double scal[8]);

/* Advance nsteps time steps with plain stream launches and time every kernel
 * with HIP events recorded on the context's stream around it.  ms_out[5]
 * receives the mean duration (ms) per launch of: y forward pass (or the
 * fused y-z-y plane kernel), z pass with tensor multiply, y inverse pass,
 * update (predictor / Euler stage), update (Heun corrector); 0 for kernels
 * that did not run.  Synchronising.
 * For benchmarks and profiling; the state advances like tdgl_step (AB3M2
 * contexts advance with Heun steps and restart their multistep history). */
tdgl_status tdgl_profile_step(tdgl_ctx *ctx, int nsteps, double ms_out[5]);

/* Time every kernel of one field evaluation on its own: for each kernel a
 * HIP graph of nrep launches of that kernel alone, on the context's live
 * buffers, is replayed once to warm up and once between two HIP events on
 * the context's stream; ms_out[5] receives the mean duration (ms) per launch
 * in the order of tdgl_profile_step (0 for kernels the configuration does
 * not use).  The kernels then run back to back as in a step, without
 * event markers between them.  P is saved before and restored after, the
 * non-finite flag is kept, and the next step rebuilds its spectra, so the
 * simulation state is unchanged; intermediate spectra are not.  Allocates
 * and frees one P-sized device buffer; synchronising.  1 <= nrep <= 100000. */
tdgl_status tdgl_profile_kernels(tdgl_ctx *ctx, int nrep, double ms_out[5]);

/* Pick the fastest launch configuration for this context by measurement:
 * each candidate (fused plane pass where it fits or the three passes,
 * times update tiles of 2, 4, 8, 16 rows; then, for the three passes, the
 * z-pass tiles of 64, 128 and 256 bytes with the rows found; last, the
 * other store mode) advances the current state by nsteps steps as one
 * graph, once to warm up and once timed with HIP events, always from the
 * same saved P.  The fastest stays set (as with tdgl_set_fft_path,
 * tdgl_set_update_rows, tdgl_set_z_tile and tdgl_set_store_mode);
 * choice[0] = 1 if it uses the fused pass, choice[1] = rows; *ms_per_step
 * (may be NULL) its time.  P, the
 * step parity and the non-finite flag are restored.  Allocates and frees
 * one P-sized device buffer; synchronising.  1 <= nsteps <= 100000. */
tdgl_status tdgl_autotune(tdgl_ctx *ctx, int nsteps, int choice[2], double *ms_per_step);

/* Wait for all work of the context; returns TDGL_E_NONFINITE if a step
 * produced a non-finite P. */
tdgl_status tdgl_sync(tdgl_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TDGL_H */
