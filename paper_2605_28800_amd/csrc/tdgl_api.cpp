// Host side of the libtdgl C ABI (include/tdgl.h).
//
// Holds the context (grid, FFT plan, materials, scales, state buffers),
// turns the SI inputs of the paper's Tables 1-2 into the reduced
// coefficients the kernels use, and enqueues one TDGL step as
//     Fy -> Fz*N*Iz -> Iy -> (Ix + local terms + update + Fx)
// per field evaluation (one for Euler, two for Heun), captured into HIP
// graphs of several steps.
#include "../../include/tdgl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace tdgl;

namespace {

constexpr double EPS0 = 8.8541878128e-12;   // F/m (CODATA 2018)

// A captured chunk of steps bakes in everything its launches take by value:
// the buffer parity, scheme, term mask and whether the cross-term kernel
// runs (device-side scalars such as dtau, E_ext and the coefficients are
// read at run time and need no new capture).
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    int cur = 0, scheme = 0, chunk = 0;
    unsigned terms = 0;
    bool cross = false;
    int hpos = 0;                 // multistep history phase at the chunk start
    // relaxation chunks (tdgl_relax): chunk = checks per graph
    bool relax = false, retire = false;
    long long check = 0, nmat = 0;
    double rtol = 0.0, floor = 0.0, joule = 0.0, P0 = 0.0;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// relaxation bookkeeping per instance: previous total energy (double), relax
// step (long long), frozen flag (int, padded); then three counters
constexpr size_t RLX_BYTES_PER_INSTANCE = 24;
// steps per captured relaxation graph (a whole number of checks)
constexpr long long RELAX_GRAPH_STEPS = 5000;

int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// FFT length for an open x or y dimension of n cells: the smallest power of
// two or 3 * 2^a (at least 24) that holds the 2n - 1 offsets, at least 8
int fft_len_xy(int n)
{
    const int p = next_pow2(2 * n - 1);
    int t = 24;
    while (t < 2 * n - 1) t <<= 1;
    const int m = t < p ? t : p;
    return m < 8 ? 8 : m;
}

}  // namespace

struct tdgl_ctx {
    Geom g{};
    double d[3]{};
    unsigned pmask = 0;
    int prec = 0;
    size_t esz = 4;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    // host-side model state
    bool scales_set = false;
    double P0 = 1.0, alpha_ref = 0.0, G110 = 0.0, eps_b = 1.0;
    tdgl_material mats[TDGL_MAX_MATERIALS]{};
    bool mat_set[TDGL_MAX_MATERIALS]{};
    std::vector<signed char> layer;
    bool grad_set = false;
    double G11 = 0, G12 = 0, G44 = 0, G44p = 0;
    int nb = 1;                           // instances of the grid (batch)
    std::vector<double> Tb;               // temperature per instance
    double eext[3] = {0, 0, 0};
    unsigned terms = TDGL_ALL;
    int scheme = TDGL_HEUN;
    double dtau = 1e-3;
    int graph_chunk = 64;
    // device
    bool dev_init = false;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    void *P[2]{};
    void *S1 = nullptr, *S2 = nullptr, *Nt = nullptr, *coef = nullptr, *kp = nullptr;
    void *twf = nullptr, *twd = nullptr;
    double *gl = nullptr, *partials = nullptr, *res = nullptr;
    void *rlx = nullptr;          // relaxation bookkeeping (tdgl_relax)
    int *flag = nullptr;
    int cur = 0;
    int yt = 2;
    // buffers only some models need: in a bound workspace after the core
    // regions (layout_of), otherwise allocated on first use (*_own)
    void *hist = nullptr;         // multistep: three E buffers
    void *rkbuf = nullptr;        // RK45: stage point Q and k_1..k_7
    void *xbuf = nullptr;         // field of the gradient cross terms
    bool hist_own = false, rk_own = false, x_own = false;
    double rk_h = 0.0, rk_tau = 0.0, rk_atol = 1e-8, rk_rtol = 1e-6;
    long long rk_rejected = 0;
    int hist_count = 0;           // valid history entries (0..2)
    int hist_pos = 0;             // buffer of the newest entry
    size_t lds_max = 65536;      // dynamic LDS one work-group may use on this device
    int fft_path = 0;            // 0: fused plane pass when it fits, 1: three passes
    int ztile = 0;               // z-pass column tile, bytes per z row (0: built-in choice)
    bool use_plane = false;
    int nblocks = 1;
    bool P_set = false, tensor_built = false, spec_valid = false, params_dirty = true;
    int mimg = -1;
    std::vector<GraphEntry> graphs;
    std::string err;
};

namespace {

tdgl_status fail(tdgl_ctx *c, tdgl_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

#define HIP_TRY(c, expr)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((c), TDGL_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// ---- layout of the device workspace
struct Layout {
    size_t P, S1, S2, Nt, coef, kp, twf, twd, gl, partials, flag, res, rlx;
    size_t xbuf, extra, total;     // cross-term field; history or RK45 buffers
};

bool cross_terms(const tdgl_ctx *c);

// Core regions, then the field of the gradient cross terms (always laid out:
// the gradient may change between steps), then the multistep history
// (scheme AB3M2) or the RK45 stage buffers (scheme RK45) of the scheme set
// when the layout is taken.
Layout layout_of(const tdgl_ctx *c, int scheme)
{
    const Geom &g = c->g;
    const size_t N = (size_t)g.nx * g.ny * g.nz * g.nb;   // cells of all instances
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.P = take(2 * 3 * N * c->esz);
    L.S1 = take((size_t)3 * g.nb * g.nz * g.ny * hx_blocked(g.hx) * 2 * c->esz);
    L.S2 = take((size_t)3 * g.nb * g.nz * g.my * hx_blocked(g.hx) * 2 * c->esz);
    L.Nt = take((size_t)6 * (g.mz / 2 + 1) * (g.my / 2 + 1) * hx_blocked(g.hx) * c->esz);
    L.coef = take((size_t)g.nb * g.nz * NCOEF * c->esz);
    L.kp = take(sizeof(KParams<double>));
    L.twf = take((size_t)TW_ENTRIES * 2 * sizeof(float));
    L.twd = take((size_t)TW_ENTRIES * 2 * sizeof(double));
    L.gl = take((size_t)2 * GL_MAXN * GL_MAXN * sizeof(double));
    L.partials = take((size_t)c->nblocks * g.nb * 8 * sizeof(double));
    L.flag = take(sizeof(int));
    L.res = take((size_t)8 * g.nb * sizeof(double));
    L.rlx = take(RLX_BYTES_PER_INSTANCE * g.nb + 32);
    const size_t pbytes = 3 * N * c->esz;
    L.xbuf = take(pbytes);
    L.extra = off;
    if (scheme == TDGL_AB3M2) take(3 * pbytes);
    if (scheme == TDGL_RK45) take(8 * pbytes);
    L.total = off;
    return L;
}

Layout layout_of(const tdgl_ctx *c) { return layout_of(c, c->scheme); }

// Gauss-Legendre nodes and weights on [0,1] (Newton on the Legendre
// recurrence in long double); row n of the tables holds n nodes.
void gauss_legendre_tables(double *t, double *w)
{
    for (int i = 0; i < GL_MAXN * GL_MAXN; ++i) t[i] = w[i] = 0.0;
    for (int n = 1; n < GL_MAXN; ++n) {
        for (int i = 0; i < n; ++i) {
            long double x = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
            long double dp = 1.0L;
            for (int it = 0; it < 100; ++it) {
                long double p0 = 1.0L, p1 = x;
                for (int k = 2; k <= n; ++k) {
                    long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                if (n == 1) { p0 = 1.0L; p1 = x; }
                dp = n * (x * p1 - p0) / (x * x - 1.0L);
                long double dx = p1 / dp;
                x -= dx;
                if (fabsl(dx) < 1e-19L) break;
            }
            {   // final derivative at the converged root
                long double p0 = 1.0L, p1 = x;
                for (int k = 2; k <= n; ++k) {
                    long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (x * p1 - p0) / (x * x - 1.0L);
            }
            const long double wt = 2.0L / ((1.0L - x * x) * dp * dp);
            t[n * GL_MAXN + i] = (double)(0.5L * (x + 1.0L));
            w[n * GL_MAXN + i] = (double)(0.5L * wt);
        }
    }
}

// twiddles W_M^k = exp(-2 pi i k / M) for every power-of-two M, table of M at offset M
template <typename T>
std::vector<T> twiddle_table()
{
    std::vector<T> tw(2 * TW_ENTRIES, T(0));
    auto fill = [&](int M) {
        const int o = tw_off(M);
        for (int k = 0; k < M; ++k) {
            const long double a = -2.0L * 3.14159265358979323846264338327950288L * k / M;
            tw[2 * (o + k)] = (T)cosl(a);
            tw[2 * (o + k) + 1] = (T)sinl(a);
        }
    };
    for (int M = 1; M <= MAXLEN; M <<= 1) fill(M);           // powers of two
    for (int M = 12; M <= MAXLEN; M <<= 1) fill(M);          // 3 * 2^a
    return tw;
}

void choose_path(tdgl_ctx *c);

tdgl_status ensure_device(tdgl_ctx *c)
{
    if (c->dev_init) return TDGL_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(c, TDGL_E_HIP, "no HIP device available");
    HIP_TRY(c, hipStreamCreate(&c->cap));
    Layout L = layout_of(c);
    if (!c->ws) {
        void *p = nullptr;
        if (hipMalloc(&p, L.total) != hipSuccess)
            return fail(c, TDGL_E_NOMEM, "hipMalloc(%zu) failed", L.total);
        c->ws = p;
        c->ws_bytes = L.total;
        c->ws_owned = true;
    }
    char *b = static_cast<char *>(c->ws);
    const size_t N = (size_t)c->g.nx * c->g.ny * c->g.nz * c->g.nb;
    c->P[0] = b + L.P;
    c->P[1] = b + L.P + 3 * N * c->esz;
    c->S1 = b + L.S1;
    c->S2 = b + L.S2;
    c->Nt = b + L.Nt;
    c->coef = b + L.coef;
    c->kp = b + L.kp;
    c->twf = b + L.twf;
    c->twd = b + L.twd;
    c->gl = reinterpret_cast<double *>(b + L.gl);
    c->partials = reinterpret_cast<double *>(b + L.partials);
    c->flag = reinterpret_cast<int *>(b + L.flag);
    c->res = reinterpret_cast<double *>(b + L.res);
    c->rlx = b + L.rlx;
    c->xbuf = b + L.xbuf;
    if (c->scheme == TDGL_AB3M2) c->hist = b + L.extra;
    if (c->scheme == TDGL_RK45) c->rkbuf = b + L.extra;
    auto twf = twiddle_table<float>();
    auto twd = twiddle_table<double>();
    std::vector<double> gl(2 * GL_MAXN * GL_MAXN);
    gauss_legendre_tables(gl.data(), gl.data() + GL_MAXN * GL_MAXN);
    HIP_TRY(c, hipMemcpy(c->twf, twf.data(), twf.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->twd, twd.data(), twd.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->gl, gl.data(), gl.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemset(c->flag, 0, sizeof(int)));
    int dev = 0, optin = 0;
    HIP_TRY(c, hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) ==
            hipSuccess && optin > 0)
        c->lds_max = (size_t)optin;
    c->dev_init = true;
    choose_path(c);
    if (prepare_row_blocked(c->prec, c->g.my) != hipSuccess)
        return fail(c, TDGL_E_HIP, "cannot raise the LDS limit of the y pass");
    // the x pass in the context's precision and in FP64 (the tensor build)
    if (prepare_fx(c->prec, c->g.mx) != hipSuccess || prepare_fx(PREC_F64, c->g.mx) != hipSuccess)
        return fail(c, TDGL_E_HIP, "cannot raise the LDS limit of the x pass");
    if (prepare_update(c->prec, c->g) != hipSuccess)
        return fail(c, TDGL_E_HIP, "cannot raise the LDS limit of the update kernel");
    return TDGL_OK;
}

const void *tw(const tdgl_ctx *c) { return c->prec == PREC_F32 ? c->twf : c->twd; }

// The fused plane pass is used when one kx plane of the three components
// (plus the z-pass scratch) fits in the LDS of one work-group.
void choose_path(tdgl_ctx *c)
{
    c->use_plane = c->fft_path == 0 &&
                   launch_plane(c->prec, c->g, nullptr, nullptr, nullptr, c->lds_max, nullptr,
                                true) == hipSuccess;
}

// ---- reduced parameters (Table 2 with alpha_ref in place of |alpha1|)
void landau_si(const tdgl_material &m, double T, double out[8])
{
    double a1;
    if (m.a1_form == 0) a1 = m.a1_slope * (T - m.a1_T0);
    else a1 = m.a1_A * (1.0 / std::tanh(m.a1_Ts / T) - 1.0 / std::tanh(m.a1_Ts / m.a1_T0));
    out[0] = a1;
    out[1] = a1;
    out[2] = m.rs * a1;
    out[3] = m.a11_slope * (T - m.a11_Tref) + m.a11_offset;
    out[4] = m.a12;
    out[5] = m.a111_slope * (T - m.a111_Tref) + m.a111_offset;
    out[6] = m.a112;
    out[7] = m.a123;
}

tdgl_status check_model(tdgl_ctx *c)
{
    if (!c->scales_set) return fail(c, TDGL_E_STATE, "tdgl_set_scales has not been called");
    for (int z = 0; z < c->g.nz; ++z) {
        const int id = c->layer[z];
        if (id >= 0 && !c->mat_set[id])
            return fail(c, TDGL_E_STATE, "layer %d uses material %d, which is not set", z, id);
    }
    if ((c->terms & TDGL_GRAD) && !c->grad_set)
        return fail(c, TDGL_E_STATE, "gradient term on but tdgl_set_gradient not called");
    return TDGL_OK;
}

void reduced(const tdgl_ctx *c, std::vector<double> &coef, double scal[8], double gh2[3][3])
{
    const double l0 = std::sqrt(c->G110 / c->alpha_ref);
    const double h[3] = {c->d[0] / l0, c->d[1] / l0, c->d[2] / l0};
    coef.assign((size_t)c->g.nb * c->g.nz * NCOEF, 0.0);
    for (int bz = 0; bz < c->g.nb * c->g.nz; ++bz) {
        const int z = bz % c->g.nz, b = bz / c->g.nz;
        const int id = c->layer[z];
        if (id < 0 || !c->mat_set[id]) continue;
        double si[8];
        landau_si(c->mats[id], c->Tb[b], si);
        const double a = c->alpha_ref, p2 = c->P0 * c->P0, p4 = p2 * p2;
        double *o = &coef[(size_t)bz * NCOEF];
        o[0] = si[0] / a;
        o[1] = si[1] / a;
        o[2] = si[2] / a;
        o[3] = si[3] * p2 / a;
        o[4] = si[4] * p2 / a;
        o[5] = si[5] * p4 / a;
        o[6] = si[6] * p4 / a;
        o[7] = si[7] * p4 / a;
        o[8] = 1.0;
    }
    scal[0] = 1.0 / (EPS0 * c->eps_b * c->alpha_ref);
    scal[1] = h[0];
    scal[2] = h[1];
    scal[3] = h[2];
    scal[4] = h[0] * h[1] * h[2];
    scal[5] = c->alpha_ref * c->P0 * c->P0 * l0 * l0 * l0;
    scal[6] = c->alpha_ref * c->P0;
    scal[7] = l0;
    for (int i = 0; i < 3; ++i)
        for (int dd = 0; dd < 3; ++dd) {
            const double gcoef = c->grad_set ? ((i == dd ? c->G11 : c->G44 + c->G44p) / c->G110) : 0.0;
            gh2[i][dd] = gcoef / (h[dd] * h[dd]);
        }
}

template <typename T>
tdgl_status upload_params_t(tdgl_ctx *c)
{
    std::vector<double> coef;
    double scal[8], gh2[3][3];
    reduced(c, coef, scal, gh2);
    std::vector<T> cf(coef.size());
    for (size_t i = 0; i < coef.size(); ++i) cf[i] = (T)coef[i];
    KParams<T> kp{};
    kp.dtau = (T)c->dtau;
    for (int k = 0; k < 3; ++k) kp.eext[k] = (T)(c->eext[k] / scal[6]);
    for (int i = 0; i < 3; ++i)
        for (int dd = 0; dd < 3; ++dd) kp.gh2[i][dd] = (T)gh2[i][dd];
    kp.out_scale = (T)scal[6];
    kp.g12 = c->grad_set ? (T)(c->G12 / c->G110) : T(0);
    kp.gm = c->grad_set ? (T)((c->G44 - c->G44p) / c->G110) : T(0);
    for (int k = 0; k < 3; ++k) kp.inv2h[k] = (T)(0.5 / scal[1 + k]);
    HIP_TRY(c, hipMemcpyAsync(c->coef, cf.data(), cf.size() * sizeof(T), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->kp, &kp, sizeof kp, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->params_dirty = false;
    return TDGL_OK;
}

bool cross_terms(const tdgl_ctx *c) { return c->grad_set && (c->G12 != 0.0 || c->G44 != c->G44p); }

tdgl_status upload_params(tdgl_ctx *c)
{
    if (!c->params_dirty) return TDGL_OK;
    tdgl_status st = check_model(c);
    if (st != TDGL_OK) return st;
    st = ensure_device(c);
    if (st != TDGL_OK) return st;
    if (cross_terms(c) && !c->xbuf) {
        const size_t pbytes = (size_t)3 * c->g.nx * c->g.ny * c->g.nz * c->g.nb * c->esz;
        if (hipMalloc(&c->xbuf, pbytes) != hipSuccess) {
            c->xbuf = nullptr;
            return fail(c, TDGL_E_NOMEM, "gradient cross-term buffer: hipMalloc failed");
        }
        c->x_own = true;
    }
    return c->prec == PREC_F32 ? upload_params_t<float>(c) : upload_params_t<double>(c);
}

void drop_graphs(tdgl_ctx *c)
{
    for (auto &e : c->graphs)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    c->graphs.clear();
}

bool elec_on(const tdgl_ctx *c) { return (c->terms & TDGL_ELEC) != 0; }

// ---- enqueue helpers
hipError_t enq_fx(tdgl_ctx *c, const void *P, hipStream_t s)
{
    const Geom &g = c->g;
    const long long rows = 3LL * g.nb * g.nz * g.ny;      // rows of all instances
    const Freeze fz{g.frozen, 3LL * g.nz * g.ny, g.nb};   // rows [nb][3][nz][ny]
    return launch_fx(c->prec, g.mx, P, rows, g.nx, g.nx, c->S1, rows, tw(c), s, fz, true);
}

// the y passes between S1 (x spectra) and S2 (y spectra), both in blocks of
// KB kx; lines (kx, r) with r < nb*3*nz
hipError_t enq_yfwd(tdgl_ctx *c, hipStream_t s, bool freeze = true)
{
    const Geom &g = c->g;
    const Freeze fz{freeze ? g.frozen : nullptr, 3LL * g.nz, g.nb};   // line kx*R + r
    return launch_row_blocked(c->prec, g.my, false, c->S1, c->S2, g.hx, 3LL * g.nb * g.nz, g.ny,
                              g.my, g.ny, g.my, tw(c), s, fz, g.nt);
}

hipError_t enq_yinv(tdgl_ctx *c, hipStream_t s, bool freeze = true)
{
    const Geom &g = c->g;
    const Freeze fz{freeze ? g.frozen : nullptr, 3LL * g.nz, g.nb};
    return launch_row_blocked(c->prec, g.my, true, c->S1, c->S2, g.hx, 3LL * g.nb * g.nz, g.ny,
                              g.my, g.my, g.ny, tw(c), s, fz, g.nt);
}

// y pass, z pass with the tensor, inverse y pass: S1 (x spectra) -> S1
// (field rows), fused into one kernel when possible.
hipError_t enq_yz(tdgl_ctx *c, hipStream_t s)
{
    const Geom &g = c->g;
    if (c->use_plane) return launch_plane(c->prec, g, c->S1, c->Nt, tw(c), c->lds_max, s, false);
    hipError_t e = enq_yfwd(c, s);
    if (e != hipSuccess) return e;
    e = launch_zmul(c->prec, g, c->S2, c->Nt, tw(c), c->ztile, s);
    if (e != hipSuccess) return e;
    return enq_yinv(c, s);
}

// field of the gradient cross terms at Pin into xbuf, when the model has them
hipError_t enq_cross(tdgl_ctx *c, const void *Pin, unsigned terms, UpdArgs &a, hipStream_t s)
{
    a.cross = nullptr;
    if (!(terms & TDGL_GRAD) || !cross_terms(c) || !c->xbuf) return hipSuccess;
    a.cross = c->xbuf;
    return launch_cross(c->prec, c->g, Pin, c->xbuf, c->coef, c->kp, s);
}

hipError_t enq_upd(tdgl_ctx *c, int mode, const void *Pin, const void *Pold, void *Pout,
                   int stage, unsigned terms, bool elec_in, bool fx_out, hipStream_t s,
                   double *partials = nullptr)
{
    UpdArgs a{};
    hipError_t ce = enq_cross(c, Pin, terms, a, s);
    if (ce != hipSuccess) return ce;
    a.P_in = Pin;
    a.P_old = Pold;
    a.P_out = Pout;
    a.S1 = c->S1;
    a.coef = c->coef;
    a.kp = c->kp;
    a.partials = partials ? partials : c->partials;
    a.flag = c->flag;
    a.stage = stage;
    a.terms = terms;
    a.elec_in = elec_in ? 1 : 0;
    a.fx_out = fx_out ? 1 : 0;
    a.yt = c->yt;
    return launch_update(c->prec, mode, c->g, a, tw(c), s, nullptr);
}

hipError_t enq_eval(tdgl_ctx *c, int mode, const void *Pin, const void *Pold, void *Pout,
                    int stage, unsigned terms, bool elec, bool fx_out, hipStream_t s,
                    double *partials = nullptr)
{
    if (elec) {
        hipError_t e = enq_yz(c, s);
        if (e != hipSuccess) return e;
    }
    return enq_upd(c, mode, Pin, Pold, Pout, stage, terms, elec, fx_out, s, partials);
}

// multistep history buffer k (0..2)
void *hist_buf(const tdgl_ctx *c, int k)
{
    const size_t pbytes = (size_t)3 * c->g.nx * c->g.ny * c->g.nz * c->g.nb * c->esz;
    return static_cast<char *>(c->hist) + (size_t)k * pbytes;
}

// one multistep step; *count, *pos: history entries and newest buffer
hipError_t enq_step_ms(tdgl_ctx *c, int cur, int *count, int *pos, hipStream_t s)
{
    const bool el = elec_on(c);
    const unsigned t = c->terms;
    void *A = c->P[cur], *B = c->P[1 - cur];
    const int nw = (*pos + 1) % 3;                      // buffer for E_n
    UpdArgs a{};
    a.S1 = c->S1;
    a.coef = c->coef;
    a.kp = c->kp;
    a.partials = c->partials;
    a.flag = c->flag;
    a.terms = t;
    a.elec_in = el ? 1 : 0;
    a.fx_out = el ? 1 : 0;
    a.yt = c->yt;
    a.hist_w = hist_buf(c, nw);
    hipError_t e = el ? enq_yz(c, s) : hipSuccess;
    if (e != hipSuccess) return e;
    a.P_in = A;
    a.P_out = B;
    if (*count < 2) {                                   // start-up: Heun, storing E_n
        a.stage = 0;
        e = enq_cross(c, A, t, a, s);
        if (e == hipSuccess) e = launch_update(c->prec, UPD_STEP_MS, c->g, a, tw(c), s, nullptr);
        if (e != hipSuccess) return e;
        e = enq_eval(c, UPD_STEP, B, A, A, 1, t, el, el, s);
    } else {
        a.stage = 2;                                    // AB3 predictor -> B
        a.hist_a = hist_buf(c, *pos);
        a.hist_b = hist_buf(c, (*pos + 2) % 3);
        e = enq_cross(c, A, t, a, s);
        if (e == hipSuccess) e = launch_update(c->prec, UPD_STEP_MS, c->g, a, tw(c), s, nullptr);
        if (e != hipSuccess) return e;
        if (el) e = enq_yz(c, s);                       // AM2 corrector -> A
        if (e != hipSuccess) return e;
        a.stage = 3;
        a.P_in = B;
        a.P_old = A;
        a.P_out = A;
        a.hist_w = nullptr;
        a.hist_a = hist_buf(c, nw);
        a.hist_b = hist_buf(c, *pos);
        e = enq_cross(c, B, t, a, s);
        if (e == hipSuccess) e = launch_update(c->prec, UPD_STEP_MS, c->g, a, tw(c), s, nullptr);
    }
    if (e != hipSuccess) return e;
    *pos = nw;
    if (*count < 2) ++*count;
    return hipSuccess;
}

// one time step starting from buffer *cur (updated for Euler)
hipError_t enq_step(tdgl_ctx *c, int *cur, hipStream_t s)
{
    const bool el = elec_on(c);
    const unsigned t = c->terms;
    void *A = c->P[*cur], *B = c->P[1 - *cur];
    if (c->scheme == TDGL_EULER) {
        hipError_t e = enq_eval(c, UPD_STEP, A, nullptr, B, 0, t, el, el, s);
        *cur = 1 - *cur;
        return e;
    }
    hipError_t e = enq_eval(c, UPD_STEP, A, nullptr, B, 0, t, el, el, s);
    if (e != hipSuccess) return e;
    return enq_eval(c, UPD_STEP, B, A, A, 1, t, el, el, s);
}

tdgl_status get_graph(tdgl_ctx *c, int chunk, hipGraphExec_t *out)
{
    const bool cross = cross_terms(c) && (c->terms & TDGL_GRAD) && c->xbuf;
    const int hpos = c->scheme == TDGL_AB3M2 ? c->hist_pos : 0;
    for (auto &e : c->graphs)
        if (!e.relax && e.cur == c->cur && e.scheme == c->scheme && e.chunk == chunk &&
            e.terms == c->terms && e.cross == cross && e.hpos == hpos) {
            *out = e.exec;
            return TDGL_OK;
        }
    hipGraph_t graph = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int cur = c->cur;
    int hcount = 2, hp = hpos;      // graphs are captured only with a full history
    hipError_t le = hipSuccess;
    for (int i = 0; i < chunk && le == hipSuccess; ++i)
        le = c->scheme == TDGL_AB3M2 ? enq_step_ms(c, cur, &hcount, &hp, c->cap)
                                     : enq_step(c, &cur, c->cap);
    hipError_t ee = hipStreamEndCapture(c->cap, &graph);
    if (le != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, TDGL_E_HIP, "graph capture failed: %s",
                    hipGetErrorString(le != hipSuccess ? le : ee));
    }
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess)
        return fail(c, TDGL_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    GraphEntry ge;
    ge.exec = exec;
    ge.cur = c->cur;
    ge.scheme = c->scheme;
    ge.chunk = chunk;
    ge.terms = c->terms;
    ge.cross = cross;
    ge.hpos = hpos;
    c->graphs.push_back(ge);
    *out = exec;
    return TDGL_OK;
}

// ---- relaxation (tdgl_relax)
RelaxState relax_state(const tdgl_ctx *c)
{
    const size_t nb = (size_t)c->g.nb;
    char *b = static_cast<char *>(c->rlx);
    RelaxState r;
    r.Fprev = reinterpret_cast<double *>(b);
    r.step = reinterpret_cast<long long *>(b + 8 * nb);
    r.frozen = reinterpret_cast<int *>(b + 16 * nb);
    r.counter = reinterpret_cast<long long *>(b + 24 * nb);
    r.stopped = reinterpret_cast<long long *>(b + 24 * nb + 8);
    r.remaining = reinterpret_cast<int *>(b + 24 * nb + 16);
    return r;
}

struct RelaxArgs {
    long long check;
    double rtol, floor;     // floor in J
    bool retire;
    double joule;           // J per reduced energy unit
    long long nmat;         // material cells per instance
};

// Energies of the current state of every instance (the spectra must be the
// current state's: S1 from the last update or from a fresh x pass), reduced
// on the device to J exactly as tdgl_energies_batch does, then the relaxation
// test.  Leaves S1 holding field rows.
hipError_t enq_relax_check(tdgl_ctx *c, const void *P, const RelaxArgs &ra, bool init,
                           hipStream_t s)
{
    const bool el = elec_on(c);
    hipError_t e = enq_eval(c, UPD_ENERGY, P, nullptr, nullptr, 0, c->terms, el, false, s);
    if (e != hipSuccess) return e;
    const int ngroups = ((c->g.ny + c->yt - 1) / c->yt) * c->g.nz;
    e = launch_reduce_energies(c->partials, ngroups, c->g.nb, ra.joule, (double)ra.nmat, c->P0,
                               c->res, s);
    if (e != hipSuccess) return e;
    return launch_relax_test(c->res, relax_state(c), c->g.nb, init, ra.check, ra.rtol, ra.floor,
                             ra.retire, s);
}

// nchecks relaxation checks into stream s (being captured): each `check`
// steps, the energies and the test, then the x pass of the state for the next
// step.  Every kernel skips (the update kernel: carries over) the instances
// the test froze.  *cur: buffer parity before and after.
hipError_t enq_relax_chunk(tdgl_ctx *c, int nchecks, const RelaxArgs &ra, hipStream_t s, int *cur)
{
    const bool el = elec_on(c);
    c->g.frozen = relax_state(c).frozen;
    hipError_t le = hipSuccess;
    for (int k = 0; k < nchecks && le == hipSuccess; ++k) {
        for (long long i = 0; i < ra.check && le == hipSuccess; ++i) le = enq_step(c, cur, s);
        if (le == hipSuccess) le = enq_relax_check(c, c->P[*cur], ra, false, s);
        if (le == hipSuccess && el) le = enq_fx(c, c->P[*cur], s);
    }
    c->g.frozen = nullptr;
    return le;
}

// A captured graph of enq_relax_chunk, cached per configuration.
tdgl_status get_relax_graph(tdgl_ctx *c, int nchecks, const RelaxArgs &ra, hipGraphExec_t *out,
                            int *cur_after)
{
    const bool cross = cross_terms(c) && (c->terms & TDGL_GRAD) && c->xbuf;
    for (auto &e : c->graphs)
        if (e.relax && e.cur == c->cur && e.scheme == c->scheme && e.chunk == nchecks &&
            e.terms == c->terms && e.cross == cross && e.check == ra.check &&
            e.retire == ra.retire && e.rtol == ra.rtol && e.floor == ra.floor &&
            e.joule == ra.joule && e.nmat == ra.nmat && e.P0 == c->P0) {
            *out = e.exec;
            *cur_after = e.hpos;
            return TDGL_OK;
        }
    hipGraph_t graph = nullptr;
    hipError_t le = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    int cur = c->cur;
    if (le == hipSuccess) {
        le = enq_relax_chunk(c, nchecks, ra, c->cap, &cur);
        hipError_t ee = hipStreamEndCapture(c->cap, &graph);
        if (le == hipSuccess) le = ee;
    }
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, TDGL_E_HIP, "relaxation graph capture failed: %s", hipGetErrorString(le));
    }
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess)
        return fail(c, TDGL_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    GraphEntry ge;
    ge.exec = exec;
    ge.cur = c->cur;
    ge.scheme = c->scheme;
    ge.chunk = nchecks;
    ge.terms = c->terms;
    ge.cross = cross;
    ge.hpos = cur;                 // buffer parity after the chunk
    ge.relax = true;
    ge.retire = ra.retire;
    ge.check = ra.check;
    ge.rtol = ra.rtol;
    ge.floor = ra.floor;
    ge.joule = ra.joule;
    ge.nmat = ra.nmat;
    ge.P0 = c->P0;
    c->graphs.push_back(ge);
    *out = exec;
    *cur_after = cur;
    return TDGL_OK;
}

tdgl_status read_flag(tdgl_ctx *c)
{
    int f = 0;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (f) return fail(c, TDGL_E_NONFINITE, "a time step produced a non-finite polarisation");
    return TDGL_OK;
}

}  // namespace

// =========================================================================
extern "C" {

int tdgl_abi_version(void) { return TDGL_ABI_VERSION; }

tdgl_status tdgl_create(const tdgl_grid *grid, int precision, void *hip_stream, tdgl_ctx **out)
{
    return tdgl_create_batch(grid, 1, precision, hip_stream, out);
}

tdgl_status tdgl_create_batch(const tdgl_grid *grid, int nbatch, int precision, void *hip_stream,
                              tdgl_ctx **out)
{
    if (!out) return TDGL_E_ARG;
    *out = nullptr;
    if (!grid) return TDGL_E_ARG;
    if (precision != TDGL_FP32 && precision != TDGL_FP64) return TDGL_E_ARG;
    if (nbatch < 1 || nbatch > 4096) return TDGL_E_ARG;
    const int n[3] = {grid->nx, grid->ny, grid->nz};
    const double d[3] = {grid->dx, grid->dy, grid->dz};
    for (int k = 0; k < 3; ++k) {
        if (n[k] < 1 || n[k] > 4096) return TDGL_E_ARG;
    }
    if ((long long)n[0] * n[1] * n[2] >= (1LL << 31)) return TDGL_E_UNSUPPORTED;
    // the update kernel's smallest tile (two rows, two cells per thread) fits
    // the 512 threads of an FP64 group for rows of at most 512 cells
    if (precision == TDGL_FP64 && n[0] > 512) return TDGL_E_UNSUPPORTED;
    if ((long long)n[2] * nbatch > 65535) return TDGL_E_UNSUPPORTED;     // launch grid rows
    for (int k = 0; k < 3; ++k) {
        if (!(d[k] > 0.0) || !std::isfinite(d[k])) return TDGL_E_ARG;
    }
    const unsigned pm = grid->periodic_mask;
    if (pm != 0u && pm != 3u && pm != 7u) return TDGL_E_UNSUPPORTED;
    int m[3];
    for (int k = 0; k < 3; ++k) {
        if (pm >> k & 1u) {
            if (n[k] < 8 || (n[k] & (n[k] - 1)) != 0) return TDGL_E_UNSUPPORTED;
            m[k] = n[k];
        } else if (k < 2) {
            m[k] = fft_len_xy(n[k]);
        } else {
            m[k] = next_pow2(2 * n[k] - 1);     // the z pass takes powers of two
            if (m[k] < 8) m[k] = 8;
        }
        if (m[k] > MAXLEN) return TDGL_E_UNSUPPORTED;
    }
    tdgl_ctx *c = new (std::nothrow) tdgl_ctx();
    if (!c) return TDGL_E_NOMEM;
    c->g = Geom{n[0], n[1], n[2], m[0], m[1], m[2], m[0] / 2 + 1,
                (int)(pm & 1u), (int)(pm >> 1 & 1u), (int)(pm >> 2 & 1u)};
    for (int k = 0; k < 3; ++k) c->d[k] = d[k];
    c->pmask = pm;
    c->prec = precision;
    c->esz = precision == TDGL_FP32 ? 4 : 8;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->g.nb = nbatch;
    c->g.nt = nbatch == 1 ? 1 : 0;       // the built-in store mode (tdgl_set_store_mode)
    c->Tb.assign(nbatch, 300.0);
    c->layer.assign(n[2], 0);
    c->yt = update_rows_per_block(c->prec, c->g);
    c->nblocks = ((c->g.ny + 1) / 2) * c->g.nz;   // partial sums for any row tile >= 2
    *out = c;
    return TDGL_OK;
}

void tdgl_destroy(tdgl_ctx *c)
{
    if (!c) return;
    if (c->dev_init) {
        (void)hipStreamSynchronize(c->stream);
        drop_graphs(c);
        if (c->ws_owned && c->ws) (void)hipFree(c->ws);
        if (c->hist && c->hist_own) (void)hipFree(c->hist);
        if (c->rkbuf && c->rk_own) (void)hipFree(c->rkbuf);
        if (c->xbuf && c->x_own) (void)hipFree(c->xbuf);
        if (c->cap) (void)hipStreamDestroy(c->cap);
    }
    delete c;
}

const char *tdgl_last_error(const tdgl_ctx *c) { return c ? c->err.c_str() : "null context"; }

tdgl_status tdgl_get_batch(const tdgl_ctx *c, int *nbatch)
{
    if (!c || !nbatch) return TDGL_E_ARG;
    *nbatch = c->g.nb;
    return TDGL_OK;
}

tdgl_status tdgl_get_dims(const tdgl_ctx *c, int out[7])
{
    if (!c || !out) return TDGL_E_ARG;
    const Geom &g = c->g;
    const int v[7] = {g.nx, g.ny, g.nz, g.mx, g.my, g.mz, g.hx};
    for (int k = 0; k < 7; ++k) out[k] = v[k];
    return TDGL_OK;
}

tdgl_status tdgl_workspace_size(const tdgl_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return TDGL_E_ARG;
    *bytes = layout_of(c).total;
    return TDGL_OK;
}

tdgl_status tdgl_bind_workspace(tdgl_ctx *c, void *dev_ptr, size_t bytes)
{
    if (!c) return TDGL_E_ARG;
    if (c->dev_init) return fail(c, TDGL_E_STATE, "device memory already in use");
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) != 0)
        return fail(c, TDGL_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < layout_of(c).total)
        return fail(c, TDGL_E_ARG, "workspace too small: %zu < %zu", bytes, layout_of(c).total);
    c->ws = dev_ptr;
    c->ws_bytes = bytes;
    c->ws_owned = false;
    return TDGL_OK;
}

tdgl_status tdgl_set_scales(tdgl_ctx *c, double P0, double alpha_ref, double G110, double eps_b)
{
    if (!c) return TDGL_E_ARG;
    if (!(P0 > 0) || !(alpha_ref > 0) || !(G110 > 0) || !(eps_b > 0) || !std::isfinite(P0) ||
        !std::isfinite(alpha_ref) || !std::isfinite(G110) || !std::isfinite(eps_b))
        return fail(c, TDGL_E_ARG, "scales must be positive and finite");
    const bool geom_change = !c->scales_set || alpha_ref != c->alpha_ref || G110 != c->G110 ||
                             eps_b != c->eps_b;
    c->P0 = P0;
    c->alpha_ref = alpha_ref;
    c->G110 = G110;
    c->eps_b = eps_b;
    c->scales_set = true;
    if (geom_change) c->tensor_built = false;
    c->params_dirty = true;
    return TDGL_OK;
}

tdgl_status tdgl_set_material(tdgl_ctx *c, int id, const tdgl_material *m)
{
    if (!c) return TDGL_E_ARG;
    if (!m || id < 0 || id >= TDGL_MAX_MATERIALS) return fail(c, TDGL_E_ARG, "bad material id");
    if (m->a1_form != 0 && m->a1_form != 1) return fail(c, TDGL_E_ARG, "a1_form must be 0 or 1");
    if (m->a1_form == 1 && (!(m->a1_Ts > 0) || !(m->a1_T0 > 0)))
        return fail(c, TDGL_E_ARG, "Barrett form needs a1_Ts > 0 and a1_T0 > 0");
    c->mats[id] = *m;
    c->mat_set[id] = true;
    c->params_dirty = true;
    return TDGL_OK;
}

tdgl_status tdgl_set_layer_materials(tdgl_ctx *c, const signed char *ids)
{
    if (!c) return TDGL_E_ARG;
    if (!ids) return fail(c, TDGL_E_ARG, "null layer map");
    for (int z = 0; z < c->g.nz; ++z)
        if (ids[z] < -1 || ids[z] >= TDGL_MAX_MATERIALS)
            return fail(c, TDGL_E_ARG, "layer %d: material id %d out of range", z, (int)ids[z]);
    c->layer.assign(ids, ids + c->g.nz);
    c->params_dirty = true;
    c->spec_valid = false;
    return TDGL_OK;
}

tdgl_status tdgl_set_gradient(tdgl_ctx *c, double G11, double G12, double G44, double G44p)
{
    if (!c) return TDGL_E_ARG;
    if (!std::isfinite(G11) || !std::isfinite(G12) || !std::isfinite(G44) || !std::isfinite(G44p))
        return fail(c, TDGL_E_ARG, "gradient coefficients must be finite");
    c->G11 = G11;
    c->G12 = G12;
    c->G44 = G44;
    c->G44p = G44p;
    c->grad_set = true;
    c->params_dirty = true;
    return TDGL_OK;
}

tdgl_status tdgl_build_tensor(tdgl_ctx *c, int mimg)
{
    if (!c) return TDGL_E_ARG;
    if (mimg < 0 || mimg > 64) return fail(c, TDGL_E_ARG, "mimg must be in [0, 64]");
    if (!c->scales_set) return fail(c, TDGL_E_STATE, "tdgl_set_scales has not been called");
    tdgl_status st = ensure_device(c);
    if (st != TDGL_OK) return st;
    const Geom &g = c->g;
    const size_t nreal = (size_t)g.mx * g.my * g.mz;
    const size_t ncplx = (size_t)g.mz * g.my * g.hx;
    double *R = nullptr;
    void *C = nullptr;
    if (hipMalloc(&R, 6 * nreal * sizeof(double)) != hipSuccess)
        return fail(c, TDGL_E_NOMEM, "tensor build: hipMalloc failed");
    if (hipMalloc(&C, 6 * ncplx * 2 * sizeof(double)) != hipSuccess) {
        (void)hipFree(R);
        return fail(c, TDGL_E_NOMEM, "tensor build: hipMalloc failed");
    }
    const double l0 = std::sqrt(c->G110 / c->alpha_ref);
    const double kappa = 1.0 / (EPS0 * c->eps_b * c->alpha_ref);
    hipError_t e = launch_tensor_real(g, c->pmask, mimg, c->d[0] / l0, c->d[1] / l0,
                                      c->d[2] / l0, c->gl, c->gl + GL_MAXN * GL_MAXN, R,
                                      c->stream);
    if (e == hipSuccess) e = launch_tensor_k0(g, c->pmask, R, nullptr, c->stream);
    // spectrum C[kx][q][mz][my]: x pass (kx-major), y rows, z columns
    const long long rows = 6LL * g.mz * g.my;
    if (e == hipSuccess)
        e = launch_fx(PREC_F64, g.mx, R, rows, g.mx, g.mx, C, rows, c->twd, c->stream);
    if (e == hipSuccess)
        e = launch_row(PREC_F64, g.my, false, C, C, (long long)g.hx * 6 * g.mz, g.my, g.my, g.my,
                       g.my, c->twd, c->stream);
    if (e == hipSuccess)
        e = launch_col(PREC_F64, g.mz, false, C, C, g.my, (long long)g.hx * 6,
                       (long long)g.mz * g.my, (long long)g.mz * g.my, g.my, g.mz, g.mz, c->twd,
                       c->stream);
    if (e == hipSuccess)
        e = launch_tensor_octant(c->prec, g, C, -kappa / (double)nreal, c->Nt, c->stream);
    hipError_t se = hipStreamSynchronize(c->stream);
    (void)hipFree(R);
    (void)hipFree(C);
    if (e != hipSuccess || se != hipSuccess)
        return fail(c, TDGL_E_HIP, "tensor build failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : se));
    c->tensor_built = true;
    c->mimg = mimg;
    return TDGL_OK;
}

tdgl_status tdgl_get_tensor_spectrum(tdgl_ctx *c, double *dst, size_t count)
{
    if (!c || !dst) return TDGL_E_ARG;
    if (!c->tensor_built) return fail(c, TDGL_E_STATE, "tensor not built");
    const Geom &g = c->g;
    const size_t qs = (size_t)(g.mz / 2 + 1) * (g.my / 2 + 1);
    const size_t n = 6 * qs * g.hx;
    if (count < n) return fail(c, TDGL_E_ARG, "need %zu doubles", n);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // the device copy is stored in blocks of KB kx: [hx/KB][6][kz][ky][KB]
    const size_t nblk = 6 * qs * hx_blocked(g.hx);
    std::vector<double> tmp(nblk);
    if (c->prec == PREC_F64) {
        HIP_TRY(c, hipMemcpy(tmp.data(), c->Nt, nblk * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tf(nblk);
        HIP_TRY(c, hipMemcpy(tf.data(), c->Nt, nblk * sizeof(float), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < nblk; ++i) tmp[i] = tf[i];
    }
    for (size_t kx = 0; kx < (size_t)g.hx; ++kx)
        for (size_t e = 0; e < 6 * qs; ++e)
            dst[kx * 6 * qs + e] = tmp[((kx / KB) * 6 * qs + e) * KB + kx % KB];
    return TDGL_OK;
}

tdgl_status tdgl_set_temperature(tdgl_ctx *c, double T)
{
    if (!c) return TDGL_E_ARG;
    if (!(T > 0) || !std::isfinite(T)) return fail(c, TDGL_E_ARG, "temperature must be > 0");
    c->Tb.assign(c->g.nb, T);
    c->params_dirty = true;
    return TDGL_OK;
}

tdgl_status tdgl_set_temperatures(tdgl_ctx *c, const double *T)
{
    if (!c) return TDGL_E_ARG;
    if (!T) return fail(c, TDGL_E_ARG, "null temperatures");
    for (int b = 0; b < c->g.nb; ++b)
        if (!(T[b] > 0) || !std::isfinite(T[b]))
            return fail(c, TDGL_E_ARG, "temperature of instance %d must be > 0", b);
    c->Tb.assign(T, T + c->g.nb);
    c->params_dirty = true;
    return TDGL_OK;
}

tdgl_status tdgl_set_eext(tdgl_ctx *c, double ex, double ey, double ez)
{
    if (!c) return TDGL_E_ARG;
    if (!std::isfinite(ex) || !std::isfinite(ey) || !std::isfinite(ez))
        return fail(c, TDGL_E_ARG, "E_ext must be finite");
    c->eext[0] = ex;
    c->eext[1] = ey;
    c->eext[2] = ez;
    c->params_dirty = true;
    return TDGL_OK;
}

tdgl_status tdgl_set_terms(tdgl_ctx *c, unsigned mask)
{
    if (!c) return TDGL_E_ARG;
    if (mask & ~(unsigned)TDGL_ALL) return fail(c, TDGL_E_ARG, "unknown term bits");
    if ((mask & TDGL_ELEC) != (c->terms & TDGL_ELEC)) c->spec_valid = false;
    c->terms = mask;
    c->params_dirty = true;
    return TDGL_OK;
}

tdgl_status tdgl_set_integrator(tdgl_ctx *c, int scheme, double dtau)
{
    if (!c) return TDGL_E_ARG;
    if (scheme != TDGL_EULER && scheme != TDGL_HEUN && scheme != TDGL_AB3M2 &&
        scheme != TDGL_RK45)
        return fail(c, TDGL_E_ARG, "unknown scheme");
    if (!(dtau > 0) || !std::isfinite(dtau)) return fail(c, TDGL_E_ARG, "dtau must be > 0");
    c->scheme = scheme;
    c->dtau = dtau;
    c->hist_count = 0;            // the multistep history assumes one dtau
    c->rk_h = dtau;               // RK45: first trial step
    c->rk_tau = 0.0;
    c->rk_rejected = 0;
    c->params_dirty = true;
    return TDGL_OK;
}

tdgl_status tdgl_set_graph_chunk(tdgl_ctx *c, int steps)
{
    if (!c) return TDGL_E_ARG;
    if (steps < 0 || steps > 100000) return fail(c, TDGL_E_ARG, "graph chunk out of range");
    c->graph_chunk = steps;
    return TDGL_OK;
}

tdgl_status tdgl_set_fft_path(tdgl_ctx *c, int path)
{
    if (!c) return TDGL_E_ARG;
    if (path != 0 && path != 1) return fail(c, TDGL_E_ARG, "path must be 0 or 1");
    c->fft_path = path;
    drop_graphs(c);
    if (c->dev_init) choose_path(c);
    return TDGL_OK;
}

tdgl_status tdgl_set_update_rows(tdgl_ctx *c, int rows)
{
    if (!c) return TDGL_E_ARG;
    if (rows < 0 || rows > 64 || rows == 1 || (rows & (rows - 1)))
        return fail(c, TDGL_E_ARG, "rows must be 0 or a power of two in 2..64");
    const int yt = rows == 0 ? update_rows_per_block(c->prec, c->g) : rows;
    // the launch checks threads and LDS; probe with a zero-size query here
    const int nb = ((c->g.ny + yt - 1) / yt) * c->g.nz;
    if (c->dev_init && nb > c->nblocks)
        return fail(c, TDGL_E_STATE, "more row groups than the workspace was sized for");
    c->yt = yt;
    if (!c->dev_init) c->nblocks = nb > c->nblocks ? nb : c->nblocks;
    drop_graphs(c);
    return TDGL_OK;
}

tdgl_status tdgl_set_store_mode(tdgl_ctx *c, int mode)
{
    if (!c) return TDGL_E_ARG;
    if (mode < 0 || mode > 2) return fail(c, TDGL_E_ARG, "store mode must be 0, 1 or 2");
    c->g.nt = mode == 0 ? (c->g.nb == 1 ? 1 : 0) : (mode == 1 ? 1 : 0);
    drop_graphs(c);
    return TDGL_OK;
}

tdgl_status tdgl_get_store_mode(const tdgl_ctx *c, int *mode)
{
    if (!c || !mode) return TDGL_E_ARG;
    *mode = c->g.nt ? 1 : 2;
    return TDGL_OK;
}

tdgl_status tdgl_set_z_tile(tdgl_ctx *c, int row_bytes)
{
    if (!c) return TDGL_E_ARG;
    if (row_bytes != 0 && row_bytes != 64 && row_bytes != 128 && row_bytes != 256)
        return fail(c, TDGL_E_ARG, "z tile must be 0, 64, 128 or 256 bytes");
    c->ztile = row_bytes;
    drop_graphs(c);
    return TDGL_OK;
}

tdgl_status tdgl_get_z_tile(const tdgl_ctx *c, int *row_bytes)
{
    if (!c || !row_bytes) return TDGL_E_ARG;
    *row_bytes = c->ztile == 0 ? zmul_auto_tile(c->prec, c->g) : c->ztile;
    return TDGL_OK;
}

tdgl_status tdgl_get_fft_path(const tdgl_ctx *c, int *fused)
{
    if (!c || !fused) return TDGL_E_ARG;
    *fused = c->use_plane ? 1 : 0;
    return TDGL_OK;
}

tdgl_status tdgl_set_P(tdgl_ctx *c, const void *src, int on_dev, int src_prec)
{
    if (!c) return TDGL_E_ARG;
    if (!src) return fail(c, TDGL_E_ARG, "null source");
    if (src_prec != TDGL_FP32 && src_prec != TDGL_FP64) return fail(c, TDGL_E_ARG, "bad precision");
    tdgl_status st = upload_params(c);
    if (st != TDGL_OK) return st;
    const Geom &g = c->g;
    const size_t n = (size_t)3 * g.nx * g.ny * g.nz * g.nb;
    void *dst = c->P[c->cur];
    // stored in units of P0 (Table 2)
    const double inv = 1.0 / c->P0;
    if (on_dev) {
        HIP_TRY(c, launch_convert(src_prec, src, c->prec, dst, n, inv, c->stream));
    } else {
        std::vector<unsigned char> tmp(n * c->esz);
        for (size_t i = 0; i < n; ++i) {
            const double v = (src_prec == TDGL_FP32 ? (double)static_cast<const float *>(src)[i]
                                                    : static_cast<const double *>(src)[i]) * inv;
            if (c->prec == PREC_F32) reinterpret_cast<float *>(tmp.data())[i] = (float)v;
            else reinterpret_cast<double *>(tmp.data())[i] = v;
        }
        HIP_TRY(c, hipMemcpyAsync(dst, tmp.data(), tmp.size(), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    HIP_TRY(c, launch_zero_layers(c->prec, dst, c->coef, g, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    c->P_set = true;
    c->spec_valid = false;
    c->hist_count = 0;
    return TDGL_OK;
}

tdgl_status tdgl_get_P(tdgl_ctx *c, void *dst, int on_dev, int dst_prec)
{
    if (!c) return TDGL_E_ARG;
    if (!dst) return fail(c, TDGL_E_ARG, "null destination");
    if (dst_prec != TDGL_FP32 && dst_prec != TDGL_FP64) return fail(c, TDGL_E_ARG, "bad precision");
    if (!c->P_set) return fail(c, TDGL_E_STATE, "P has not been set");
    const Geom &g = c->g;
    const size_t n = (size_t)3 * g.nx * g.ny * g.nz * g.nb;
    const void *src = c->P[c->cur];
    if (on_dev) {
        HIP_TRY(c, launch_convert(c->prec, src, dst_prec, dst, n, c->P0, c->stream));
        return TDGL_OK;
    }
    std::vector<unsigned char> tmp(n * c->esz);
    HIP_TRY(c, hipMemcpyAsync(tmp.data(), src, tmp.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < n; ++i) {
        const double v = (c->prec == PREC_F32 ? (double)reinterpret_cast<const float *>(tmp.data())[i]
                                              : reinterpret_cast<const double *>(tmp.data())[i]) * c->P0;
        if (dst_prec == TDGL_FP32) static_cast<float *>(dst)[i] = (float)v;
        else static_cast<double *>(dst)[i] = v;
    }
    return read_flag(c);
}

namespace {

// The history (AB3M2) or stage buffers (RK45) of scheme: in a bound
// workspace, the region after the cross-term field, which must be large
// enough (TDGL_E_STATE otherwise); without one, a device allocation of
// its own, made once.
tdgl_status extra_buffer(tdgl_ctx *c, int scheme, size_t bytes, void **out, bool *own)
{
    const Layout L = layout_of(c, scheme);
    if (L.total <= c->ws_bytes) {            // the workspace already has room
        *out = static_cast<char *>(c->ws) + L.extra;
        *own = false;
        return TDGL_OK;
    }
    if (c->ws_owned) {
        if (hipMalloc(out, bytes) != hipSuccess) {
            *out = nullptr;
            return fail(c, TDGL_E_NOMEM, "buffers of the integrator: hipMalloc(%zu) failed", bytes);
        }
        *own = true;
        return TDGL_OK;
    }
    return fail(c, TDGL_E_STATE,
                "the bound workspace (%zu bytes) lacks the %zu bytes of this integrator's "
                "buffers: set the integrator before tdgl_workspace_size and bind %zu bytes",
                c->ws_bytes, bytes, L.total);
}

// One accepted RK45 step (attempts repeat until one is accepted).
tdgl_status rk45_step(tdgl_ctx *c)
{
    const Geom &g = c->g;
    const size_t n3 = (size_t)3 * g.nx * g.ny * g.nz * g.nb;
    const size_t pbytes = n3 * c->esz;
    if (!c->rkbuf) {
        tdgl_status st = extra_buffer(c, TDGL_RK45, 8 * pbytes, &c->rkbuf, &c->rk_own);
        if (st != TDGL_OK) return st;
    }
    const bool el = elec_on(c);
    const int ngroups = ((g.ny + c->yt - 1) / c->yt) * g.nz * g.nb;
    std::vector<double> part((size_t)ngroups * 8);
    for (int attempt = 0; attempt < 64; ++attempt) {
        void *Pn = c->P[c->cur], *W0 = c->P[1 - c->cur];
        void *Q = c->rkbuf;
        void *K = static_cast<char *>(c->rkbuf) + pbytes;
        if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, Pn, c->stream));
        UpdArgs a{};
        a.S1 = c->S1;
        a.coef = c->coef;
        a.kp = c->kp;
        a.partials = c->partials;
        a.flag = c->flag;
        a.terms = c->terms;
        a.elec_in = el ? 1 : 0;
        a.fx_out = el ? 1 : 0;
        a.yt = c->yt;
        a.rk_base = Pn;
        a.rk_k = K;
        a.rk_h = c->rk_h;
        a.rk_atol = c->rk_atol;
        a.rk_rtol = c->rk_rtol;
        // stage s reads the point written by stage s - 1; the fifth-order
        // solution (stage 6 output) lands in W0 = P[1 - cur]
        const void *in = Pn;
        for (int st = 1; st <= 7; ++st) {
            if (el) HIP_TRY(c, enq_yz(c, c->stream));
            void *out = st == 7 ? const_cast<void *>(in) : ((st % 2 == 0) ? W0 : Q);
            a.stage = st;
            a.P_in = in;
            a.P_out = out;
            HIP_TRY(c, enq_cross(c, in, c->terms, a, c->stream));
            HIP_TRY(c, launch_update(c->prec, UPD_STEP_RK, g, a, tw(c), c->stream, nullptr));
            in = out;
        }
        HIP_TRY(c, hipMemcpyAsync(part.data(), c->partials, part.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        double err = 0.0;
        for (int i = 0; i < ngroups; ++i) err = part[(size_t)i * 8] > err ? part[(size_t)i * 8] : err;
        if (!std::isfinite(err)) return fail(c, TDGL_E_NONFINITE, "RK45 error estimate not finite");
        const double fac = err > 0.0 ? 0.9 * std::pow(err, -0.2) : 5.0;
        if (err <= 1.0) {                        // accept: P5 (and its spectrum) is current
            c->rk_tau += c->rk_h;
            c->rk_h *= std::min(5.0, std::max(0.2, fac));
            c->cur = 1 - c->cur;
            c->spec_valid = el;
            return TDGL_OK;
        }
        ++c->rk_rejected;                        // reject: retry from P_n
        c->rk_h *= std::max(0.2, fac);
        c->spec_valid = false;
    }
    return fail(c, TDGL_E_NONFINITE, "RK45: 64 rejected attempts in a row");
}

}  // namespace

tdgl_status tdgl_set_rk_tolerances(tdgl_ctx *c, double atol, double rtol)
{
    if (!c) return TDGL_E_ARG;
    if (!(atol >= 0) || !(rtol >= 0) || !(atol + rtol > 0) || !std::isfinite(atol) ||
        !std::isfinite(rtol))
        return fail(c, TDGL_E_ARG, "tolerances must be >= 0, finite, not both 0");
    c->rk_atol = atol;
    c->rk_rtol = rtol;
    return TDGL_OK;
}

tdgl_status tdgl_get_rk_state(const tdgl_ctx *c, double *tau, double *h, long long *rejected)
{
    if (!c || !tau || !h || !rejected) return TDGL_E_ARG;
    *tau = c->rk_tau;
    *h = c->rk_h;
    *rejected = c->rk_rejected;
    return TDGL_OK;
}

tdgl_status tdgl_step(tdgl_ctx *c, long long nsteps)
{
    if (!c) return TDGL_E_ARG;
    if (nsteps < 0) return fail(c, TDGL_E_ARG, "nsteps < 0");
    if (!c->P_set) return fail(c, TDGL_E_STATE, "P has not been set");
    if (elec_on(c) && !c->tensor_built)
        return fail(c, TDGL_E_STATE, "electrostatic term on but tensor not built");
    if (nsteps == 0) return TDGL_OK;
    tdgl_status st = upload_params(c);
    if (st != TDGL_OK) return st;
    const bool el = elec_on(c);
    if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
    if (c->scheme == TDGL_RK45) {
        for (long long i = 0; i < nsteps; ++i) {
            st = rk45_step(c);
            if (st != TDGL_OK) return st;
        }
        return TDGL_OK;
    }
    const bool ms = c->scheme == TDGL_AB3M2;
    long long left = nsteps;
    if (ms) {
        if (!c->hist) {
            const size_t pbytes = (size_t)3 * c->g.nx * c->g.ny * c->g.nz * c->g.nb * c->esz;
            st = extra_buffer(c, TDGL_AB3M2, 3 * pbytes, &c->hist, &c->hist_own);
            if (st != TDGL_OK) return st;
        }
        for (; left > 0 && c->hist_count < 2; --left)      // start-up steps, plain launches
            HIP_TRY(c, enq_step_ms(c, c->cur, &c->hist_count, &c->hist_pos, c->stream));
    }
    // whole chunks, then the remainder as one graph of its own length (graphs
    // are cached per length; an odd Euler graph flips the buffer parity)
    const int chunk = c->graph_chunk;
    while (chunk > 0 && left > 0) {
        const int len = left >= chunk ? chunk : (int)left;
        if (len != chunk && c->graphs.size() >= 32) drop_graphs(c);   // bound the cache
        hipGraphExec_t exec = nullptr;
        st = get_graph(c, len, &exec);
        if (st != TDGL_OK) return st;
        HIP_TRY(c, hipGraphLaunch(exec, c->stream));
        if (ms) c->hist_pos = (c->hist_pos + len) % 3;
        if (c->scheme == TDGL_EULER && (len & 1)) c->cur = 1 - c->cur;
        left -= len;
    }
    for (; left > 0; --left) {
        if (ms) {
            HIP_TRY(c, enq_step_ms(c, c->cur, &c->hist_count, &c->hist_pos, c->stream));
            continue;
        }
        int cur = c->cur;
        HIP_TRY(c, enq_step(c, &cur, c->stream));
        c->cur = cur;
    }
    c->spec_valid = el;
    return TDGL_OK;
}

tdgl_status tdgl_eval_field(tdgl_ctx *c, unsigned mask, void *dst)
{
    if (!c) return TDGL_E_ARG;
    if (!dst) return fail(c, TDGL_E_ARG, "null destination");
    if (mask & ~(unsigned)TDGL_ALL) return fail(c, TDGL_E_ARG, "unknown term bits");
    if (!c->P_set) return fail(c, TDGL_E_STATE, "P has not been set");
    const bool el = (mask & TDGL_ELEC) != 0;
    if (el && !c->tensor_built) return fail(c, TDGL_E_STATE, "tensor not built");
    if ((mask & TDGL_GRAD) && !c->grad_set)
        return fail(c, TDGL_E_STATE, "gradient coefficients not set");
    tdgl_status st = upload_params(c);
    if (st != TDGL_OK) return st;
    if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
    HIP_TRY(c, enq_eval(c, UPD_FIELD, c->P[c->cur], nullptr, dst, 0, mask, el, false, c->stream));
    if (el) c->spec_valid = false;
    return TDGL_OK;
}

namespace {

// energies of every instance: F[b*5 + 0..4] (J), meanP[b*3 + 0..2] (C/m^2)
tdgl_status energies_all(tdgl_ctx *c, double *F, double *meanP)
{
    if (!c->P_set) return fail(c, TDGL_E_STATE, "P has not been set");
    const bool el = elec_on(c);
    if (el && !c->tensor_built) return fail(c, TDGL_E_STATE, "tensor not built");
    tdgl_status st = upload_params(c);
    if (st != TDGL_OK) return st;
    if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
    HIP_TRY(c, enq_eval(c, UPD_ENERGY, c->P[c->cur], nullptr, nullptr, 0, c->terms, el, false,
                        c->stream));
    if (el) c->spec_valid = false;
    // one partial per work-group of the launch just made, instance-major
    const int ngroups = ((c->g.ny + c->yt - 1) / c->yt) * c->g.nz;
    HIP_TRY(c, launch_reduce_partials(c->partials, ngroups, c->g.nb, c->res, c->stream));
    std::vector<double> r((size_t)8 * c->g.nb);
    HIP_TRY(c, hipMemcpyAsync(r.data(), c->res, r.size() * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    st = read_flag(c);
    std::vector<double> coef;
    double scal[8], gh2[3][3];
    reduced(c, coef, scal, gh2);
    const double f = scal[4] * scal[5];
    long long nmat = 0;
    for (int z = 0; z < c->g.nz; ++z)
        if (c->layer[z] >= 0) nmat += (long long)c->g.nx * c->g.ny;
    for (int b = 0; b < c->g.nb; ++b) {
        const double *rb = &r[(size_t)8 * b];
        double *Fb = F + 5 * b;
        for (int k = 0; k < 4; ++k) Fb[k] = rb[k] * f;
        Fb[4] = Fb[0] + Fb[1] + Fb[2] + Fb[3];
        for (int k = 0; k < 3; ++k) meanP[3 * b + k] = nmat ? rb[4 + k] / (double)nmat * c->P0 : 0.0;
    }
    return st;
}

}  // namespace

tdgl_status tdgl_energies(tdgl_ctx *c, double F[5], double meanP[3])
{
    if (!c) return TDGL_E_ARG;
    if (!F || !meanP) return fail(c, TDGL_E_ARG, "null output");
    if (c->g.nb == 1) return energies_all(c, F, meanP);
    std::vector<double> Fa((size_t)5 * c->g.nb), Ma((size_t)3 * c->g.nb);
    tdgl_status st = energies_all(c, Fa.data(), Ma.data());
    for (int k = 0; k < 5; ++k) F[k] = Fa[k];
    for (int k = 0; k < 3; ++k) meanP[k] = Ma[k];
    return st;
}

tdgl_status tdgl_energies_batch(tdgl_ctx *c, double *F, double *meanP)
{
    if (!c) return TDGL_E_ARG;
    if (!F || !meanP) return fail(c, TDGL_E_ARG, "null output");
    return energies_all(c, F, meanP);
}

tdgl_status tdgl_energies_noalloc(tdgl_ctx *c, double *out_dev)
{
    if (!c) return TDGL_E_ARG;
    if (!out_dev) return fail(c, TDGL_E_ARG, "null output");
    // every buffer but the scratch must already exist: no call below allocates
    if (!c->P_set || !c->dev_init) return fail(c, TDGL_E_STATE, "P has not been set");
    const bool el = elec_on(c);
    if (el && !c->tensor_built) return fail(c, TDGL_E_STATE, "tensor not built");
    if (c->params_dirty) {
        tdgl_status st = check_model(c);
        if (st != TDGL_OK) return st;
    }
    const int ngroups = ((c->g.ny + c->yt - 1) / c->yt) * c->g.nz;
    const size_t need = (size_t)ngroups * c->g.nb * 8;
    if (need > SCRATCH_DOUBLES)
        return fail(c, TDGL_E_UNSUPPORTED,
                    "energy partials need %zu doubles; the fixed scratch holds %zu "
                    "(use tdgl_energies_batch)", need, (size_t)SCRATCH_DOUBLES);
    double *scr = nullptr;
    HIP_TRY(c, scratch_address(&scr));
    tdgl_status st = upload_params(c);      // no allocation: the workspace holds every buffer
    if (st != TDGL_OK) return st;
    if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
    HIP_TRY(c, enq_eval(c, UPD_ENERGY, c->P[c->cur], nullptr, nullptr, 0, c->terms, el, false,
                        c->stream, scr));
    if (el) c->spec_valid = false;
    std::vector<double> coef;
    double scal[8], gh2[3][3];
    reduced(c, coef, scal, gh2);
    long long nmat = 0;
    for (int z = 0; z < c->g.nz; ++z)
        if (c->layer[z] >= 0) nmat += (long long)c->g.nx * c->g.ny;
    HIP_TRY(c, launch_reduce_energies(scr, ngroups, c->g.nb, scal[4] * scal[5], (double)nmat,
                                      c->P0, out_dev, c->stream));
    return TDGL_OK;
}

namespace {

// Validation, model upload, the relaxation arguments and the initial energies
// (the test's reference) of one context.
tdgl_status relax_begin(tdgl_ctx *c, long long check, long long max_steps, double rtol,
                        double floor_factor, int retire, RelaxArgs *ra, bool *graphed)
{
    if (check < 1 || check > 1000000) return fail(c, TDGL_E_ARG, "check must be in 1..1e6");
    if (max_steps < 0) return fail(c, TDGL_E_ARG, "max_steps < 0");
    if (!(rtol > 0) || !std::isfinite(rtol)) return fail(c, TDGL_E_ARG, "rtol must be > 0");
    if (!(floor_factor >= 0) || !std::isfinite(floor_factor))
        return fail(c, TDGL_E_ARG, "floor_factor must be >= 0");
    if (retire != 0 && retire != 1) return fail(c, TDGL_E_ARG, "retire must be 0 or 1");
    if (!c->P_set) return fail(c, TDGL_E_STATE, "P has not been set");
    const bool el = elec_on(c);
    if (el && !c->tensor_built) return fail(c, TDGL_E_STATE, "tensor not built");
    tdgl_status st = upload_params(c);
    if (st != TDGL_OK) return st;
    // floor: alpha_ref P0^2 (J/m^3) * floor_factor * sample volume
    const double vol = (double)c->g.nx * c->g.ny * c->g.nz * c->d[0] * c->d[1] * c->d[2];
    // graphed chunks for the schemes whose steps are graphed; the multistep
    // scheme and RK45 step through tdgl_step and are never retired
    *graphed = (c->scheme == TDGL_EULER || c->scheme == TDGL_HEUN) && c->graph_chunk > 0;
    std::vector<double> coef;
    double scal[8], gh2[3][3];
    reduced(c, coef, scal, gh2);
    long long nmat = 0;
    for (int z = 0; z < c->g.nz; ++z)
        if (c->layer[z] >= 0) nmat += (long long)c->g.nx * c->g.ny;
    *ra = RelaxArgs{check, rtol, floor_factor * c->alpha_ref * c->P0 * c->P0 * vol,
                    *graphed && retire == 1, scal[4] * scal[5], nmat};
    if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
    HIP_TRY(c, enq_relax_check(c, c->P[c->cur], *ra, true, c->stream));
    c->spec_valid = false;
    return TDGL_OK;
}

// Relax steps and steps taken of one context (synchronising).
tdgl_status relax_finish(tdgl_ctx *c, long long *relax_step, long long *steps_taken)
{
    const RelaxState rs = relax_state(c);
    long long counters[2] = {0, -1};
    std::vector<long long> steps((size_t)c->g.nb);
    HIP_TRY(c, hipMemcpyAsync(steps.data(), rs.step, steps.size() * sizeof(long long),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(counters, rs.counter, 2 * sizeof(long long), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < c->g.nb; ++b) relax_step[b] = steps[(size_t)b];
    if (steps_taken) *steps_taken = counters[1] >= 0 ? counters[1] : counters[0];
    // frozen instances skipped the last x passes: the next step starts afresh
    c->spec_valid = false;
    return TDGL_OK;
}

}  // namespace

tdgl_status tdgl_relax(tdgl_ctx *c, long long check, long long max_steps, double rtol,
                       double floor_factor, int retire, long long *relax_step,
                       long long *steps_taken)
{
    if (!c) return TDGL_E_ARG;
    if (!relax_step) return fail(c, TDGL_E_ARG, "null relax_step");
    RelaxArgs ra{};
    bool graphed = false;
    tdgl_status st = relax_begin(c, check, max_steps, rtol, floor_factor, retire, &ra, &graphed);
    if (st != TDGL_OK) return st;
    const bool el = elec_on(c);
    const RelaxState rs = relax_state(c);
    long long done = 0;
    int remaining = c->g.nb;
    const long long per_graph = std::max(1LL, RELAX_GRAPH_STEPS / check);
    while (done < max_steps && remaining > 0) {
        const long long want = (max_steps - done + check - 1) / check;      // checks left
        if (graphed) {
            const int nchk = (int)std::min(per_graph, want);
            if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
            if (c->graphs.size() >= 32) drop_graphs(c);
            hipGraphExec_t exec = nullptr;
            int cur_after = c->cur;
            st = get_relax_graph(c, nchk, ra, &exec, &cur_after);
            if (st != TDGL_OK) return st;
            HIP_TRY(c, hipGraphLaunch(exec, c->stream));
            c->cur = cur_after;
            c->spec_valid = el;
            done += nchk * check;
        } else {
            st = tdgl_step(c, check);
            if (st != TDGL_OK) return st;
            if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
            HIP_TRY(c, enq_relax_check(c, c->P[c->cur], ra, false, c->stream));
            c->spec_valid = false;
            done += check;
        }
        HIP_TRY(c, hipMemcpyAsync(&remaining, rs.remaining, sizeof(int), hipMemcpyDeviceToHost,
                                  c->stream));
        st = read_flag(c);                   // synchronises
        if (st != TDGL_OK) return st;
    }
    return relax_finish(c, relax_step, steps_taken);
}

tdgl_status tdgl_relax_group(tdgl_ctx *const *ctxs, int nctx, long long check,
                             long long max_steps, double rtol, double floor_factor, int retire,
                             long long *relax_step, long long *steps_taken)
{
    if (!ctxs || nctx < 1 || nctx > 64 || !relax_step) return TDGL_E_ARG;
    for (int i = 0; i < nctx; ++i) {
        if (!ctxs[i]) return TDGL_E_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(ctxs[i], TDGL_E_ARG, "context listed twice");
    }
    tdgl_ctx *c0 = ctxs[0];
    std::vector<RelaxArgs> ra((size_t)nctx);
    for (int i = 0; i < nctx; ++i) {
        tdgl_ctx *c = ctxs[i];
        if (!(c->scheme == TDGL_EULER || c->scheme == TDGL_HEUN) || c->graph_chunk <= 0)
            return fail(c, TDGL_E_UNSUPPORTED,
                        "a relaxation group needs Euler or Heun contexts with graphs");
        bool graphed = false;
        tdgl_status st = relax_begin(c, check, max_steps, rtol, floor_factor, retire,
                                     &ra[(size_t)i], &graphed);
        if (st != TDGL_OK) return st;
    }
    // events: [0, nctx) join the contexts' streams to the first one around
    // each graph launch; [nctx, 2 nctx) fork and join the branches in capture
    std::vector<hipEvent_t> ev((size_t)2 * nctx, nullptr);
    struct Cleanup {
        std::vector<hipEvent_t> &ev;
        std::vector<std::pair<std::vector<int>, hipGraphExec_t>> graphs;
        ~Cleanup()
        {
            for (auto &e : ev)
                if (e) (void)hipEventDestroy(e);
            for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        }
    } cl{ev, {}};
    for (auto &e : ev) HIP_TRY(c0, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    long long done = 0;
    long long remaining = 1;
    const long long per_graph = std::max(1LL, RELAX_GRAPH_STEPS / check);
    std::vector<int> rem((size_t)nctx, 0);
    while (done < max_steps && remaining > 0) {
        const long long want = (max_steps - done + check - 1) / check;
        const int nchk = (int)std::min(per_graph, want);
        // key: checks per graph and every context's buffer parity
        std::vector<int> key{nchk};
        for (int i = 0; i < nctx; ++i) {
            tdgl_ctx *c = ctxs[i];
            if (elec_on(c) && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
            key.push_back(c->cur);
        }
        hipGraphExec_t exec = nullptr;
        for (auto &g : cl.graphs)
            if (g.first == key) exec = g.second;
        std::vector<int> cur_after((size_t)nctx);
        for (int i = 0; i < nctx; ++i) cur_after[(size_t)i] = ctxs[i]->cur;
        if (!exec) {
            hipGraph_t graph = nullptr;
            hipError_t le = hipStreamBeginCapture(c0->cap, hipStreamCaptureModeThreadLocal);
            if (le == hipSuccess) {
                le = hipEventRecord(ev[(size_t)nctx], c0->cap);        // fork
                for (int i = 1; i < nctx && le == hipSuccess; ++i)
                    le = hipStreamWaitEvent(ctxs[i]->cap, ev[(size_t)nctx], 0);
                // (the branches of the contexts run side by side in one graph)
                for (int i = 0; i < nctx && le == hipSuccess; ++i)
                    le = enq_relax_chunk(ctxs[i], nchk, ra[(size_t)i], ctxs[i]->cap,
                                         &cur_after[(size_t)i]);
                for (int i = 1; i < nctx && le == hipSuccess; ++i) {  // join
                    le = hipEventRecord(ev[(size_t)(nctx + i)], ctxs[i]->cap);
                    if (le == hipSuccess)
                        le = hipStreamWaitEvent(c0->cap, ev[(size_t)(nctx + i)], 0);
                }
                hipError_t ee = hipStreamEndCapture(c0->cap, &graph);
                if (le == hipSuccess) le = ee;
            }
            if (le != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(c0, TDGL_E_HIP, "relaxation group capture failed: %s",
                            hipGetErrorString(le));
            }
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess)
                return fail(c0, TDGL_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
            cl.graphs.emplace_back(key, exec);
        } else {
            int cur = 0;
            for (int i = 0; i < nctx; ++i) {       // parities after the chunk
                cur = ctxs[i]->cur;
                if (ctxs[i]->scheme == TDGL_EULER && ((long long)nchk * check) % 2) cur = 1 - cur;
                cur_after[(size_t)i] = cur;
            }
        }
        // the graph runs on the first context's stream after every context's
        // earlier work, and every context's later work waits for it
        for (int i = 1; i < nctx; ++i) {
            HIP_TRY(c0, hipEventRecord(ev[(size_t)i], ctxs[i]->stream));
            HIP_TRY(c0, hipStreamWaitEvent(c0->stream, ev[(size_t)i], 0));
        }
        HIP_TRY(c0, hipGraphLaunch(exec, c0->stream));
        HIP_TRY(c0, hipEventRecord(ev[0], c0->stream));
        for (int i = 0; i < nctx; ++i) {
            tdgl_ctx *c = ctxs[i];
            if (i > 0) HIP_TRY(c, hipStreamWaitEvent(c->stream, ev[0], 0));
            c->cur = cur_after[(size_t)i];
            c->spec_valid = elec_on(c);
            HIP_TRY(c, hipMemcpyAsync(&rem[(size_t)i], relax_state(c).remaining, sizeof(int),
                                      hipMemcpyDeviceToHost, c->stream));
        }
        done += nchk * check;
        remaining = 0;
        for (int i = 0; i < nctx; ++i) {
            tdgl_status st = read_flag(ctxs[i]);  // synchronises
            if (st != TDGL_OK) return st;
            remaining += rem[(size_t)i];
        }
    }
    long long off = 0, most = 0;
    for (int i = 0; i < nctx; ++i) {
        long long taken = 0;
        tdgl_status st = relax_finish(ctxs[i], relax_step + off, &taken);
        if (st != TDGL_OK) return st;
        off += ctxs[i]->g.nb;
        most = std::max(most, taken);
    }
    if (steps_taken) *steps_taken = most;
    return TDGL_OK;
}

tdgl_status tdgl_get_reduced(const tdgl_ctx *c, double *coef, double scal[8])
{
    if (!c || !coef || !scal) return TDGL_E_ARG;
    if (!c->scales_set) return TDGL_E_STATE;
    std::vector<double> cf;
    double gh2[3][3];
    reduced(c, cf, scal, gh2);
    for (int z = 0; z < c->g.nz; ++z)
        for (int k = 0; k < 8; ++k) coef[z * 8 + k] = cf[(size_t)z * NCOEF + k];
    return TDGL_OK;
}

tdgl_status tdgl_profile_step(tdgl_ctx *c, int nsteps, double ms_out[5])
{
    if (!c) return TDGL_E_ARG;
    if (!ms_out || nsteps < 1) return fail(c, TDGL_E_ARG, "need nsteps >= 1 and ms_out");
    if (!c->P_set) return fail(c, TDGL_E_STATE, "P has not been set");
    const bool el = elec_on(c);
    if (el && !c->tensor_built)
        return fail(c, TDGL_E_STATE, "electrostatic term on but tensor not built");
    tdgl_status st = upload_params(c);
    if (st != TDGL_OK) return st;
    if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
    const int nev = c->scheme == TDGL_EULER ? 1 : 2;    // AB3M2 is timed with Heun stages
    c->hist_count = 0;
    // events: per evaluation y_fwd, z, y_inv, update -> 5 markers
    std::vector<hipEvent_t> ev((size_t)nsteps * nev * 5);
    for (auto &e : ev) HIP_TRY(c, hipEventCreate(&e));
    double sum[5] = {0, 0, 0, 0, 0};
    int cnt[5] = {0, 0, 0, 0, 0};
    hipError_t le = hipSuccess;
    size_t k = 0;
    const Geom &g = c->g;
    for (int sidx = 0; sidx < nsteps && le == hipSuccess; ++sidx) {
        for (int e = 0; e < nev && le == hipSuccess; ++e) {
            void *A = c->P[c->cur], *B = c->P[1 - c->cur];
            const void *Pin = e == 0 ? A : B;
            const void *Pold = e == 0 ? nullptr : A;
            void *Pout = e == 0 ? B : A;
            hipEvent_t *E = &ev[k];
            k += 5;
            (void)hipEventRecord(E[0], c->stream);
            if (el && c->use_plane) {
                le = launch_plane(c->prec, g, c->S1, c->Nt, tw(c), c->lds_max, c->stream, false);
                (void)hipEventRecord(E[1], c->stream);
                (void)hipEventRecord(E[2], c->stream);
                (void)hipEventRecord(E[3], c->stream);
            } else if (el) {
                le = enq_yfwd(c, c->stream, false);
                (void)hipEventRecord(E[1], c->stream);
                if (le == hipSuccess) le = launch_zmul(c->prec, g, c->S2, c->Nt, tw(c), c->ztile, c->stream);
                (void)hipEventRecord(E[2], c->stream);
                if (le == hipSuccess) le = enq_yinv(c, c->stream, false);
                (void)hipEventRecord(E[3], c->stream);
            } else {
                (void)hipEventRecord(E[1], c->stream);
                (void)hipEventRecord(E[2], c->stream);
                (void)hipEventRecord(E[3], c->stream);
            }
            if (le == hipSuccess)
                le = enq_upd(c, UPD_STEP, Pin, Pold, Pout, e, c->terms, el, el, c->stream);
            (void)hipEventRecord(E[4], c->stream);
        }
        if (c->scheme == TDGL_EULER) c->cur = 1 - c->cur;
    }
    (void)le;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    k = 0;
    for (int sidx = 0; sidx < nsteps; ++sidx)
        for (int e = 0; e < nev; ++e) {
            hipEvent_t *E = &ev[k];
            k += 5;
            float ms;
            if (el) {
                for (int q = 0; q < (c->use_plane ? 1 : 3); ++q) {
                    (void)hipEventElapsedTime(&ms, E[q], E[q + 1]);
                    sum[q] += ms;
                    cnt[q]++;
                }
            }
            (void)hipEventElapsedTime(&ms, E[3], E[4]);
            sum[3 + e] += ms;
            cnt[3 + e]++;
        }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (le != hipSuccess) return fail(c, TDGL_E_HIP, "profile launch: %s", hipGetErrorString(le));
    for (int q = 0; q < 5; ++q) ms_out[q] = cnt[q] ? sum[q] / cnt[q] : 0.0;
    c->spec_valid = el;
    return TDGL_OK;
}

tdgl_status tdgl_profile_kernels(tdgl_ctx *c, int nrep, double ms_out[5])
{
    if (!c) return TDGL_E_ARG;
    if (!ms_out || nrep < 1 || nrep > 100000)
        return fail(c, TDGL_E_ARG, "need 1 <= nrep <= 100000 and ms_out");
    if (!c->P_set) return fail(c, TDGL_E_STATE, "P has not been set");
    const bool el = elec_on(c);
    if (el && !c->tensor_built)
        return fail(c, TDGL_E_STATE, "electrostatic term on but tensor not built");
    tdgl_status st = upload_params(c);
    if (st != TDGL_OK) return st;
    for (int q = 0; q < 5; ++q) ms_out[q] = 0.0;
    if (el && !c->spec_valid) HIP_TRY(c, enq_fx(c, c->P[c->cur], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int flag0 = 0;
    HIP_TRY(c, hipMemcpy(&flag0, c->flag, sizeof(int), hipMemcpyDeviceToHost));
    const size_t pbytes = (size_t)3 * c->g.nx * c->g.ny * c->g.nz * c->g.nb * c->esz;
    void *save = nullptr;
    HIP_TRY(c, hipMalloc(&save, pbytes));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipMemcpyAsync(save, c->P[c->cur], pbytes, hipMemcpyDeviceToDevice, c->stream);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    void *A = c->P[c->cur], *B = c->P[1 - c->cur];
    const Geom &g = c->g;
    const unsigned t = c->terms;
    // one kernel, nrep times, as one graph; returns ms per launch
    auto time_kernel = [&](int which, double *out) -> hipError_t {
        auto launch = [&](hipStream_t s) -> hipError_t {
            switch (which) {
            case 0:
                if (c->use_plane)
                    return launch_plane(c->prec, g, c->S1, c->Nt, tw(c), c->lds_max, s, false);
                return enq_yfwd(c, s, false);
            case 1: return launch_zmul(c->prec, g, c->S2, c->Nt, tw(c), c->ztile, s);
            case 2: return enq_yinv(c, s, false);
            case 3: return enq_upd(c, UPD_STEP, A, nullptr, B, 0, t, el, el, s);
            default: return enq_upd(c, UPD_STEP, B, A, A, 1, t, el, el, s);
            }
        };
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t r = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
        if (r != hipSuccess) return r;
        hipError_t le = hipSuccess;
        for (int i = 0; i < nrep && le == hipSuccess; ++i) le = launch(c->cap);
        r = hipStreamEndCapture(c->cap, &graph);
        if (le != hipSuccess) r = le;
        if (r == hipSuccess) r = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (r == hipSuccess) r = hipGraphLaunch(exec, c->stream);
        if (r == hipSuccess) r = hipEventRecord(e0, c->stream);
        if (r == hipSuccess) r = hipGraphLaunch(exec, c->stream);
        if (r == hipSuccess) r = hipEventRecord(e1, c->stream);
        if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
        float ms = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (r == hipSuccess) *out = (double)ms / nrep;
        return r;
    };
    // the update first (it reads the live spectra), the y passes next (each
    // launch recomputes the same output), the in-place z pass last
    if (he == hipSuccess) he = time_kernel(3, &ms_out[3]);
    if (he == hipSuccess && c->scheme != TDGL_EULER) he = time_kernel(4, &ms_out[4]);
    if (el) {
        if (he == hipSuccess) he = time_kernel(0, &ms_out[0]);
        if (he == hipSuccess && !c->use_plane) he = time_kernel(2, &ms_out[2]);
        if (he == hipSuccess && !c->use_plane) he = time_kernel(1, &ms_out[1]);
    }
    // restore P and the flag whatever happened above
    hipError_t re = hipMemcpyAsync(c->P[c->cur], save, pbytes, hipMemcpyDeviceToDevice, c->stream);
    if (re == hipSuccess)
        re = hipMemcpyAsync(c->flag, &flag0, sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (re == hipSuccess) re = hipStreamSynchronize(c->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(save);
    c->spec_valid = false;
    if (he != hipSuccess) return fail(c, TDGL_E_HIP, "kernel profile: %s", hipGetErrorString(he));
    if (re != hipSuccess) return fail(c, TDGL_E_HIP, "state restore: %s", hipGetErrorString(re));
    return TDGL_OK;
}

tdgl_status tdgl_sweep_eext(tdgl_ctx *c, const double *e, int nvalues, long long steps_per_value,
                            double *meanP, double *F)
{
    if (!c) return TDGL_E_ARG;
    if (!e || !meanP || nvalues < 1 || steps_per_value < 0)
        return fail(c, TDGL_E_ARG, "need field values, outputs, nvalues >= 1, steps >= 0");
    for (int i = 0; i < 3 * nvalues; ++i)
        if (!std::isfinite(e[i])) return fail(c, TDGL_E_ARG, "field value %d is not finite", i / 3);
    const int nb = c->g.nb;
    std::vector<double> Fb((size_t)5 * nb), Mb((size_t)3 * nb);
    for (int i = 0; i < nvalues; ++i) {
        tdgl_status st = tdgl_set_eext(c, e[3 * i], e[3 * i + 1], e[3 * i + 2]);
        if (st == TDGL_OK) st = tdgl_step(c, steps_per_value);
        if (st == TDGL_OK) st = energies_all(c, Fb.data(), Mb.data());
        if (st != TDGL_OK) return st;
        for (int b = 0; b < nb; ++b) {
            for (int k = 0; k < 3; ++k) meanP[((size_t)i * nb + b) * 3 + k] = Mb[(size_t)3 * b + k];
            if (F)
                for (int k = 0; k < 5; ++k) F[((size_t)i * nb + b) * 5 + k] = Fb[(size_t)5 * b + k];
        }
    }
    return TDGL_OK;
}

tdgl_status tdgl_autotune(tdgl_ctx *c, int nsteps, int choice[2], double *ms_per_step)
{
    if (!c) return TDGL_E_ARG;
    if (!choice || nsteps < 1 || nsteps > 100000)
        return fail(c, TDGL_E_ARG, "need 1 <= nsteps <= 100000 and choice");
    if (!c->P_set) return fail(c, TDGL_E_STATE, "P has not been set");
    if (elec_on(c) && !c->tensor_built)
        return fail(c, TDGL_E_STATE, "electrostatic term on but tensor not built");
    tdgl_status st = upload_params(c);
    if (st != TDGL_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int flag0 = 0;
    HIP_TRY(c, hipMemcpy(&flag0, c->flag, sizeof(int), hipMemcpyDeviceToHost));
    const size_t pbytes = (size_t)3 * c->g.nx * c->g.ny * c->g.nz * c->g.nb * c->esz;
    void *save = nullptr;
    HIP_TRY(c, hipMalloc(&save, pbytes));
    const int cur0 = c->cur;
    const int path0 = c->fft_path, yt0 = c->yt, chunk0 = c->graph_chunk;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipMemcpyAsync(save, c->P[cur0], pbytes, hipMemcpyDeviceToDevice, c->stream);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    const int nb_groups = c->nblocks;               // partials the workspace holds per instance
    const int zt0 = c->ztile, nt0 = c->g.nt;
    double best = 1e300;
    int best_path = path0, best_yt = yt0, best_zt = zt0, best_nt = nt0;
    tdgl_status rs = TDGL_OK;
    c->graph_chunk = nsteps;                        // one graph of nsteps steps per candidate
    // time the current configuration from the saved state; false if the
    // device rejects it (the candidate is skipped)
    auto trial = [&](double *ms_step) -> bool {
        drop_graphs(c);
        // every candidate starts from the saved state and runs the same steps
        he = hipMemcpyAsync(c->P[cur0], save, pbytes, hipMemcpyDeviceToDevice, c->stream);
        if (he != hipSuccess) return false;
        c->cur = cur0;
        c->spec_valid = false;
        rs = tdgl_step(c, nsteps);                  // warm-up: captures the graph
        if (rs != TDGL_OK) {                        // a tile the device rejects: skip it
            rs = TDGL_OK;
            (void)hipGetLastError();
            return false;
        }
        he = hipMemcpyAsync(c->P[cur0], save, pbytes, hipMemcpyDeviceToDevice, c->stream);
        c->cur = cur0;
        c->spec_valid = false;
        if (he == hipSuccess) he = hipEventRecord(e0, c->stream);
        if (he == hipSuccess) rs = tdgl_step(c, nsteps);
        if (he == hipSuccess && rs == TDGL_OK) he = hipEventRecord(e1, c->stream);
        if (he == hipSuccess && rs == TDGL_OK) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess && rs == TDGL_OK) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess || rs != TDGL_OK) return false;
        *ms_step = ms / nsteps;
        return true;
    };
    for (int path = 0; path <= 1 && he == hipSuccess && rs == TDGL_OK; ++path) {
        c->fft_path = path;
        choose_path(c);
        if (path == 0 && !c->use_plane) continue;   // the fused pass does not fit
        for (int yt = 2; yt <= 16 && he == hipSuccess && rs == TDGL_OK; yt *= 2) {
            if (((c->g.ny + yt - 1) / yt) * c->g.nz > nb_groups) continue;
            if (yt > 2 && yt > c->g.ny + (c->g.ny & 1)) break;
            c->yt = yt;
            c->ztile = 0;
            double ms = 0;
            if (trial(&ms) && ms < best) {
                best = ms;
                best_path = path;
                best_yt = yt;
                best_zt = 0;
            }
        }
    }
    // then the z-pass tile of the three-pass path, with the rows found
    if (best_path == 1 && best < 1e300) {
        c->fft_path = 1;
        choose_path(c);
        c->yt = best_yt;
        for (int zt = 64; zt <= 256 && he == hipSuccess && rs == TDGL_OK; zt *= 2) {
            c->ztile = zt;
            double ms = 0;
            if (trial(&ms) && ms < best) {
                best = ms;
                best_zt = zt;
            }
        }
        c->ztile = best_zt;
    }
    // last, the other store mode with everything else found
    if (best < 1e300 && he == hipSuccess && rs == TDGL_OK) {
        c->fft_path = best_path;
        choose_path(c);
        c->yt = best_yt;
        c->g.nt = 1 - nt0;
        double ms = 0;
        if (trial(&ms) && ms < best) {
            best = ms;
            best_nt = c->g.nt;
        }
    }
    // the winner stays set; the state goes back to what it was
    c->fft_path = best_path;
    c->yt = best_yt;
    c->ztile = best_zt;
    c->g.nt = best_nt;
    c->graph_chunk = chunk0;
    drop_graphs(c);
    if (c->dev_init) choose_path(c);
    hipError_t re = hipMemcpyAsync(c->P[cur0], save, pbytes, hipMemcpyDeviceToDevice, c->stream);
    if (re == hipSuccess)
        re = hipMemcpyAsync(c->flag, &flag0, sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (re == hipSuccess) re = hipStreamSynchronize(c->stream);
    c->cur = cur0;
    c->spec_valid = false;
    c->hist_count = 0;            // the trial runs overwrote the multistep history
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(save);
    if (rs != TDGL_OK) return rs;
    if (he != hipSuccess) return fail(c, TDGL_E_HIP, "autotune: %s", hipGetErrorString(he));
    if (re != hipSuccess) return fail(c, TDGL_E_HIP, "state restore: %s", hipGetErrorString(re));
    if (best == 1e300) return fail(c, TDGL_E_HIP, "autotune: no candidate ran");
    choice[0] = c->use_plane ? 1 : 0;
    choice[1] = best_yt;
    if (ms_per_step) *ms_per_step = best;
    return TDGL_OK;
}

tdgl_status tdgl_sync(tdgl_ctx *c)
{
    if (!c) return TDGL_E_ARG;
    if (!c->dev_init) return TDGL_OK;
    return read_flag(c);
}

}  // extern "C"
