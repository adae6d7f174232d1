/*
 * Dipolar interaction tensor of two uniformly polarised box cells — oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the CPU oracle that the
 * parity tests, the smoke check and the benchmark's CPU baseline use.  The
 * product library never links, loads or calls it, and it shares no code with
 * the GPU path.
 *
 * What it computes (paper §2, eq 6 and the remark that P is uniform inside
 * every finite-difference cell, §3): for piecewise-uniform P the bound charges
 * of eq 6 sit on cell faces, so the field is a sum of fields of uniformly
 * polarised boxes.  Averaging that field over a target cell gives
 *
 *     E_i(target) = -(1/(eps0 epsB)) * sum_src N_ij(r_t - r_s) P_j(src),
 *     N_ij(R)     = -(1/(4 pi V)) Int_tgt Int_src d_i d_j (1/|x - x'|),
 *
 * the cell-averaged (Newell-type) demagnetising tensor, V = dx dy dz.
 *
 * Two evaluations of the same definition are provided:
 *  - closed form (Newell, Williams & Dunlop 1993): N_xx is minus the triple
 *    second difference of a function f with d_y^2 d_z^2 f = 1/r, N_xy the
 *    same for g with d_x d_y d_z^2 g = 1/r.  Evaluated in long double,
 *    because the 27-term difference cancels heavily as |R| grows.
 *  - quadrature: the source/target double integral is a single integral of
 *    the kernel (delta_ij r^2 - 3 r_i r_j)/r^5 against the tent weight
 *    prod_k (d_k - |u_k|) on [-d,d]^3; each dimension is split at the kink
 *    and integrated with n-point Gauss-Legendre on each half.  n follows from
 *    the Bernstein-ellipse bound for the nearest complex singularity.
 *
 * The closed form is used for offsets with every |o_k| <= 1 (touching or
 * overlapping cells), the quadrature everywhere else.  Periodic dimensions add
 * lattice images in a symmetric window (see orc_offset_table).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

typedef long double ld;

#define ORC_MAXN 24

/* ---- closed form ------------------------------------------------------- */

/* f(x,y,z): even in every argument. */
static ld newell_f(ld x, ld y, ld z)
{
    x = fabsl(x); y = fabsl(y); z = fabsl(z);
    ld x2 = x * x, y2 = y * y, z2 = z * z;
    ld R = sqrtl(x2 + y2 + z2);
    if (R == 0.0L) return 0.0L;
    ld r = 0.0L;
    if (y > 0 && x2 + z2 > 0) r += 0.5L * y * (z2 - x2) * asinhl(y / sqrtl(x2 + z2));
    if (z > 0 && x2 + y2 > 0) r += 0.5L * z * (y2 - x2) * asinhl(z / sqrtl(x2 + y2));
    if (x > 0 && y > 0 && z > 0) r -= x * y * z * atanl(y * z / (x * R));
    r += (2.0L * x2 - y2 - z2) * R / 6.0L;
    return r;
}

/* g(x,y,z): odd in x, odd in y, even in z. */
static ld newell_g(ld x, ld y, ld z)
{
    ld s = 1.0L;
    if (x < 0) { s = -s; x = -x; }
    if (y < 0) { s = -s; y = -y; }
    z = fabsl(z);
    ld x2 = x * x, y2 = y * y, z2 = z * z;
    ld R = sqrtl(x2 + y2 + z2);
    if (R == 0.0L) return 0.0L;
    ld r = 0.0L;
    if (z > 0 && x2 + y2 > 0) r += x * y * z * asinhl(z / sqrtl(x2 + y2));
    if (x > 0 && y2 + z2 > 0) r += y / 6.0L * (3.0L * z2 - y2) * asinhl(x / sqrtl(y2 + z2));
    if (y > 0 && x2 + z2 > 0) r += x / 6.0L * (3.0L * z2 - x2) * asinhl(y / sqrtl(x2 + z2));
    if (z > 0) r -= z2 * z / 6.0L * atanl(x * y / (z * R));
    if (y > 0) r -= z * y2 / 2.0L * atanl(x * z / (y * R));
    if (x > 0) r -= z * x2 / 2.0L * atanl(y * z / (x * R));
    r -= x * y * R / 3.0L;
    return s * r;
}

/* -(1/(4 pi V)) * (triple second difference of fn) at (X,Y,Z), cell (a,b,c). */
static ld second_diff3(ld (*fn)(ld, ld, ld), ld X, ld Y, ld Z, ld a, ld b, ld c)
{
    static const ld wt[3] = {1.0L, -2.0L, 1.0L};
    ld s = 0.0L;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                s += wt[i] * wt[j] * wt[k] *
                     fn(X + (i - 1) * a, Y + (j - 1) * b, Z + (k - 1) * c);
    return -s / (4.0L * 3.14159265358979323846264338327950288L * a * b * c);
}

/* Component order everywhere: xx, yy, zz, xy, xz, yz. */
void orc_newell(const double R[3], const double d[3], double out[6])
{
    ld X = R[0], Y = R[1], Z = R[2], a = d[0], b = d[1], c = d[2];
    out[0] = (double)second_diff3(newell_f, X, Y, Z, a, b, c);
    out[1] = (double)second_diff3(newell_f, Y, X, Z, b, a, c);
    out[2] = (double)second_diff3(newell_f, Z, Y, X, c, b, a);
    out[3] = (double)second_diff3(newell_g, X, Y, Z, a, b, c);
    out[4] = (double)second_diff3(newell_g, X, Z, Y, a, c, b);
    out[5] = (double)second_diff3(newell_g, Y, Z, X, b, c, a);
}

/* Newell's f and g themselves, exported so tests can check their defining
 * differential identities. */
double orc_newell_f(double x, double y, double z) { return (double)newell_f(x, y, z); }
double orc_newell_g(double x, double y, double z) { return (double)newell_g(x, y, z); }

/* ---- quadrature -------------------------------------------------------- */

/* Gauss-Legendre nodes t and weights w on [0,1], row n (n nodes) of the
 * caller-provided tables gl_t[ORC_MAXN][ORC_MAXN], gl_w[...]. */
void orc_quad(const double R[3], const double d[3], int n,
              const double *t, const double *w, double out[6])
{
    /* per-dimension signed offsets and weights (both halves of the tent) */
    double ux[2 * ORC_MAXN], uy[2 * ORC_MAXN], uz[2 * ORC_MAXN], W[2 * ORC_MAXN];
    for (int q = 0; q < n; ++q) {
        double wq = w[q] * (1.0 - t[q]);
        W[q] = wq; W[n + q] = wq;
        ux[q] = d[0] * t[q]; ux[n + q] = -d[0] * t[q];
        uy[q] = d[1] * t[q]; uy[n + q] = -d[1] * t[q];
        uz[q] = d[2] * t[q]; uz[n + q] = -d[2] * t[q];
    }
    ld acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 2 * n; ++a) {
        double rx = R[0] + ux[a];
        for (int b = 0; b < 2 * n; ++b) {
            double ry = R[1] + uy[b];
            double wab = W[a] * W[b];
            for (int c = 0; c < 2 * n; ++c) {
                double rz = R[2] + uz[c];
                double r2 = rx * rx + ry * ry + rz * rz;
                double ir2 = 1.0 / r2;
                double ir5 = ir2 * ir2 / sqrt(r2);
                double ww = wab * W[c] * ir5;
                acc[0] += ww * (r2 - 3.0 * rx * rx);
                acc[1] += ww * (r2 - 3.0 * ry * ry);
                acc[2] += ww * (r2 - 3.0 * rz * rz);
                acc[3] += ww * (-3.0 * rx * ry);
                acc[4] += ww * (-3.0 * rx * rz);
                acc[5] += ww * (-3.0 * ry * rz);
            }
        }
    }
    const double pref = d[0] * d[1] * d[2] / (4.0 * 3.14159265358979323846);
    for (int k = 0; k < 6; ++k) out[k] = (double)(acc[k] * pref);
}

/* Order n for a singularity at normalised distance a from the integration
 * half-interval: Bernstein ellipse through z = 1 + i a, error ~ rho^(-2n),
 * target 1e-17. */
int orc_quad_order(double a)
{
    /* rho = |z + sqrt(z^2 - 1)|, z = 1 + i a, principal branch with |rho|>1 */
    double zr = 1.0, zi = a;
    double wr = zr * zr - zi * zi - 1.0, wi = 2.0 * zr * zi;   /* z^2 - 1 */
    double m = sqrt(sqrt(wr * wr + wi * wi));
    double ang = 0.5 * atan2(wi, wr);
    double sr = m * cos(ang), si = m * sin(ang);
    double r1 = hypot(zr + sr, zi + si), r2 = hypot(zr - sr, zi - si);
    double rho = r1 > r2 ? r1 : r2;
    int n = (int)ceil(39.14 / (2.0 * log(rho)));
    if (n < 2) n = 2;
    if (n > ORC_MAXN - 1) n = ORC_MAXN - 1;
    return n;
}

/* N(R) for integer cell offset o (R = o * d): closed form when all |o_k| <= 1,
 * quadrature otherwise.  gl_t/gl_w: [ORC_MAXN][ORC_MAXN] tables. */
void orc_cell_tensor(const double o[3], const double d[3],
                     const double *gl_t, const double *gl_w, double out[6])
{
    double R[3] = {o[0] * d[0], o[1] * d[1], o[2] * d[2]};
    if (fabs(o[0]) <= 1.0 && fabs(o[1]) <= 1.0 && fabs(o[2]) <= 1.0) {
        orc_newell(R, d, out);
        return;
    }
    double dmax = d[0], g2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        if (d[k] > dmax) dmax = d[k];
        double gk = fabs(o[k]) - 1.0;
        if (gk > 0) g2 += gk * d[k] * gk * d[k];
    }
    int n = orc_quad_order(2.0 * sqrt(g2) / dmax);
    orc_quad(R, d, n, gl_t + n * ORC_MAXN, gl_w + n * ORC_MAXN, out);
}

/* Interaction tensor for one table index of a grid (see orc_offset_table). */
static void offset_entry(const int N[3], unsigned pmask, int mimg, const double d[3],
                         const double *gl_t, const double *gl_w, const int idx[3],
                         double out6[6])
{
    /* image lists per dimension */
    double offs[3][2 * 64 + 4], wts[3][2 * 64 + 4];
    int cnt[3];
    for (int k = 0; k < 3; ++k) {
        cnt[k] = 0;
        if (!(pmask >> k & 1u)) {
            offs[k][0] = idx[k] - (N[k] - 1);
            wts[k][0] = 1.0;
            cnt[k] = 1;
        } else {
            double lim = (mimg + 0.5) * N[k];
            for (int m = -mimg - 1; m <= mimg + 1; ++m) {
                double o = idx[k] + (double)m * N[k];
                double ao = fabs(o);
                if (ao < lim) { offs[k][cnt[k]] = o; wts[k][cnt[k]] = 1.0; cnt[k]++; }
                else if (ao == lim) { offs[k][cnt[k]] = o; wts[k][cnt[k]] = 0.5; cnt[k]++; }
            }
        }
    }
    ld acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < cnt[0]; ++a)
        for (int b = 0; b < cnt[1]; ++b)
            for (int c = 0; c < cnt[2]; ++c) {
                double o[3] = {offs[0][a], offs[1][b], offs[2][c]};
                double t6[6];
                orc_cell_tensor(o, d, gl_t, gl_w, t6);
                double wgt = wts[0][a] * wts[1][b] * wts[2][c];
                for (int q = 0; q < 6; ++q) acc[q] += wgt * t6[q];
            }
    for (int q = 0; q < 6; ++q) out6[q] = (double)acc[q];
}

/* Dense table of the interaction tensor over all cell offsets of a grid.
 *
 *   N[3] = cells per dimension; pmask bit k set => dimension k periodic.
 *   Open dimension k:     K_k = 2 N_k - 1 entries, index i <-> offset i-(N_k-1).
 *   Periodic dimension k: K_k = N_k entries, index i <-> offset class i mod N_k,
 *     summed over lattice images o = i + m N_k with |o| <= (mimg + 1/2) N_k,
 *     weight 1/2 on the window boundary (keeps the table even/odd exactly).
 *   out: [6][Kz][Ky][Kx], x fastest.  No k=0 correction is applied here.
 */
void orc_offset_table(const int N[3], unsigned pmask, int mimg, const double d[3],
                      const double *gl_t, const double *gl_w, double *out)
{
    int K[3];
    for (int k = 0; k < 3; ++k) K[k] = (pmask >> k & 1u) ? N[k] : 2 * N[k] - 1;
    const size_t plane = (size_t)K[0] * K[1] * K[2];
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int iz = 0; iz < K[2]; ++iz)
        for (int iy = 0; iy < K[1]; ++iy)
            for (int ix = 0; ix < K[0]; ++ix) {
                int idx[3] = {ix, iy, iz};
                double t6[6];
                offset_entry(N, pmask, mimg, d, gl_t, gl_w, idx, t6);
                size_t lin = ((size_t)iz * K[1] + iy) * K[0] + ix;
                for (int q = 0; q < 6; ++q) out[q * plane + lin] = t6[q];
            }
}

/* One entry of the same table (index idx[3] as in orc_offset_table). */
void orc_offset_entry(const int N[3], unsigned pmask, int mimg, const double d[3],
                      const double *gl_t, const double *gl_w, const int idx[3],
                      double out6[6])
{
    offset_entry(N, pmask, mimg, d, gl_t, gl_w, idx, out6);
}
