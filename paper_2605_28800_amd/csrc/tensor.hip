// Electrostatic interaction tensor, built once per geometry in FP64.
//
// For P uniform inside each box cell (paper section 3), the bound charges of
// eq 6 sit on cell faces and the field averaged over a target cell is
//   E(target) = -1/(eps0 epsB) * sum_src N(r_t - r_s) P(src),
//   N_ij(R)   = -1/(4 pi V) Int_tgt Int_src d_i d_j |x - x'|^-1,
// the cell-averaged dipolar ("demagnetising") tensor of two boxes.
//
// Evaluation:
//  * touching or overlapping cells (every |o_k| <= 1): Newell's closed form,
//    N_xx = -(1/(4 pi V)) * (triple second difference of f), N_xy likewise
//    with g, where d_y^2 d_z^2 f = 1/r and d_x d_y d_z^2 g = 1/r;
//  * all other offsets: the double cell integral is one integral of
//    (delta_ij r^2 - 3 r_i r_j)/r^5 against the tent weight prod(d_k - |u_k|)
//    over [-d, d]^3, done with n-point Gauss-Legendre on each half of every
//    dimension, n from the Bernstein-ellipse bound of the nearest complex
//    singularity (error target 1e-17 relative to the entry).
// Placement (k_tensor_real): open dimensions use wrap-around order on the
// padded grid (offset o at o mod M, the gap N..M-N stays zero); periodic
// dimensions sum lattice images o + m N with |o + m N| <= (mimg + 1/2) N,
// weight 1/2 on the window edge.  k_tensor_k0 then sets the in-plane k = 0
// mode of an x-y periodic film to its infinite-lattice value (a uniformly
// polarised infinite sheet: zz sum 1 in its own layer, every other sum 0).
#include <cmath>

#include "fft_core.h"
#include "internal.h"

namespace tdgl {

__device__ static double newell_fd(double x, double y, double z)
{
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    if (R == 0.0) return 0.0;
    double r = (2.0 * x2 - y2 - z2) * R / 6.0;
    if (y > 0.0 && x2 + z2 > 0.0) r += 0.5 * y * (z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z > 0.0 && x2 + y2 > 0.0) r += 0.5 * z * (y2 - x2) * asinh(z / sqrt(x2 + y2));
    if (x > 0.0 && y > 0.0 && z > 0.0) r -= x * y * z * atan(y * z / (x * R));
    return r;
}

__device__ static double newell_gd(double x, double y, double z)
{
    double sgn = 1.0;
    if (x < 0.0) { sgn = -sgn; x = -x; }
    if (y < 0.0) { sgn = -sgn; y = -y; }
    z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    if (R == 0.0) return 0.0;
    double r = -x * y * R / 3.0;
    if (z > 0.0 && x2 + y2 > 0.0) r += x * y * z * asinh(z / sqrt(x2 + y2));
    if (x > 0.0 && y2 + z2 > 0.0) r += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
    if (y > 0.0 && x2 + z2 > 0.0) r += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z > 0.0) r -= z2 * z / 6.0 * atan(x * y / (z * R));
    if (y > 0.0) r -= z * y2 / 2.0 * atan(x * z / (y * R));
    if (x > 0.0) r -= z * x2 / 2.0 * atan(y * z / (x * R));
    return sgn * r;
}

// -(1/(4 pi a b c)) * sum_{i,j,k in -1..1} w_i w_j w_k fn(X+i a, Y+j b, Z+k c), w = (1,-2,1)
template <bool G>
__device__ static double newell_comb(double X, double Y, double Z, double a, double b, double c)
{
    double s = 0.0;
    for (int i = -1; i <= 1; ++i) {
        const double wi = i == 0 ? -2.0 : 1.0;
        for (int j = -1; j <= 1; ++j) {
            const double wj = j == 0 ? -2.0 : 1.0;
            double sk = 0.0;
            for (int k = -1; k <= 1; ++k) {
                const double wk = k == 0 ? -2.0 : 1.0;
                const double f = G ? newell_gd(X + i * a, Y + j * b, Z + k * c)
                                   : newell_fd(X + i * a, Y + j * b, Z + k * c);
                sk += wk * f;
            }
            s += wi * wj * sk;
        }
    }
    return -s / (4.0 * M_PI * a * b * c);
}

// components xx yy zz xy xz yz
__device__ static void newell6(double X, double Y, double Z, double a, double b, double c,
                               double *out)
{
    out[0] = newell_comb<false>(X, Y, Z, a, b, c);
    out[1] = newell_comb<false>(Y, X, Z, b, a, c);
    out[2] = newell_comb<false>(Z, Y, X, c, b, a);
    out[3] = newell_comb<true>(X, Y, Z, a, b, c);
    out[4] = newell_comb<true>(X, Z, Y, a, c, b);
    out[5] = newell_comb<true>(Y, Z, X, b, c, a);
}

// Gauss-Legendre order for a singularity at normalised distance a:
// rho = |z + sqrt(z^2 - 1)|, z = 1 + i a, error ~ rho^-2n <= 1e-17.
__device__ static int quad_order(double a)
{
    // z^2 - 1 = (1 + i a)^2 - 1 = -a^2 + 2 i a
    const double wr = -a * a, wi = 2.0 * a;
    const double mod = sqrt(sqrt(wr * wr + wi * wi));
    const double ang = 0.5 * atan2(wi, wr);
    const double sr = mod * cos(ang), si = mod * sin(ang);
    const double r1 = hypot(1.0 + sr, a + si), r2 = hypot(1.0 - sr, a - si);
    const double rho = r1 > r2 ? r1 : r2;
    int n = (int)ceil(39.14 / (2.0 * log(rho)));
    if (n < 2) n = 2;
    if (n > GL_MAXN - 1) n = GL_MAXN - 1;
    return n;
}

__device__ static void quad6(double X, double Y, double Z, double a, double b, double c, int n,
                             const double *__restrict__ t, const double *__restrict__ w,
                             double *out)
{
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int ia = 0; ia < 2 * n; ++ia) {
        const int qa = ia < n ? ia : ia - n;
        const double rx = X + (ia < n ? a : -a) * t[qa];
        const double wa = w[qa] * (1.0 - t[qa]);
        double accb[6] = {0, 0, 0, 0, 0, 0};
        for (int ib = 0; ib < 2 * n; ++ib) {
            const int qb = ib < n ? ib : ib - n;
            const double ry = Y + (ib < n ? b : -b) * t[qb];
            const double wb = w[qb] * (1.0 - t[qb]);
            double accc[6] = {0, 0, 0, 0, 0, 0};
            for (int ic = 0; ic < 2 * n; ++ic) {
                const int qc = ic < n ? ic : ic - n;
                const double rz = Z + (ic < n ? c : -c) * t[qc];
                const double wc = w[qc] * (1.0 - t[qc]);
                const double r2 = rx * rx + ry * ry + rz * rz;
                const double ir2 = 1.0 / r2;
                const double ww = wc * ir2 * ir2 / sqrt(r2);
                accc[0] += ww * (r2 - 3.0 * rx * rx);
                accc[1] += ww * (r2 - 3.0 * ry * ry);
                accc[2] += ww * (r2 - 3.0 * rz * rz);
                accc[3] -= ww * 3.0 * rx * ry;
                accc[4] -= ww * 3.0 * rx * rz;
                accc[5] -= ww * 3.0 * ry * rz;
            }
            for (int q = 0; q < 6; ++q) accb[q] += wb * accc[q];
        }
        for (int q = 0; q < 6; ++q) acc[q] += wa * accb[q];
    }
    const double pref = a * b * c / (4.0 * M_PI);
    for (int q = 0; q < 6; ++q) out[q] = acc[q] * pref;
}

// N for integer cell offset (ox, oy, oz)
__device__ static void cell_tensor(double ox, double oy, double oz, double a, double b,
                                   double c, const double *gl_t, const double *gl_w,
                                   double *out)
{
    if (fabs(ox) <= 1.0 && fabs(oy) <= 1.0 && fabs(oz) <= 1.0) {
        newell6(ox * a, oy * b, oz * c, a, b, c, out);
        return;
    }
    const double gx = fabs(ox) > 1.0 ? (fabs(ox) - 1.0) * a : 0.0;
    const double gy = fabs(oy) > 1.0 ? (fabs(oy) - 1.0) * b : 0.0;
    const double gz = fabs(oz) > 1.0 ? (fabs(oz) - 1.0) * c : 0.0;
    const double dmax = fmax(a, fmax(b, c));
    const int n = quad_order(2.0 * sqrt(gx * gx + gy * gy + gz * gz) / dmax);
    quad6(ox * a, oy * b, oz * c, a, b, c, n, gl_t + n * GL_MAXN, gl_w + n * GL_MAXN, out);
}

struct DimImages {
    int periodic, N, M, mimg;
};

// offset range for padded position p along one dimension:
// returns false if p lies in the zero gap of an open dimension.
__device__ static bool dim_range(const DimImages &d, int p, int &m0, int &m1)
{
    if (!d.periodic) {
        if (p < d.N || p > d.M - d.N) { m0 = m1 = 0; return true; }
        return false;
    }
    m0 = -d.mimg - 1;
    m1 = d.mimg + 1;
    return true;
}

__device__ static bool dim_offset(const DimImages &d, int p, int m, double &o, double &wgt)
{
    if (!d.periodic) {
        o = p < d.N ? (double)p : (double)(p - d.M);
        wgt = 1.0;
        return true;
    }
    o = (double)p + (double)m * d.N;
    const double lim = (d.mimg + 0.5) * d.N;
    const double ao = fabs(o);
    if (ao < lim) { wgt = 1.0; return true; }
    if (ao == lim) { wgt = 0.5; return true; }
    return false;
}

__global__ void k_tensor_real(Geom g, DimImages dx_, DimImages dy_, DimImages dz_, double a,
                              double b, double c, const double *__restrict__ gl_t,
                              const double *__restrict__ gl_w, double *__restrict__ R)
{
    const long long total = (long long)g.mx * g.my * g.mz;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int ix = (int)(idx % g.mx);
    const int iy = (int)((idx / g.mx) % g.my);
    const int iz = (int)(idx / ((long long)g.mx * g.my));
    int x0, x1, y0, y1, z0, z1;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (dim_range(dx_, ix, x0, x1) && dim_range(dy_, iy, y0, y1) && dim_range(dz_, iz, z0, z1)) {
        for (int mx = x0; mx <= x1; ++mx) {
            double ox, wx;
            if (!dim_offset(dx_, ix, mx, ox, wx)) continue;
            for (int my = y0; my <= y1; ++my) {
                double oy, wy;
                if (!dim_offset(dy_, iy, my, oy, wy)) continue;
                for (int mz = z0; mz <= z1; ++mz) {
                    double oz, wz;
                    if (!dim_offset(dz_, iz, mz, oz, wz)) continue;
                    double t6[6];
                    cell_tensor(ox, oy, oz, a, b, c, gl_t, gl_w, t6);
                    const double wgt = wx * wy * wz;
                    for (int q = 0; q < 6; ++q) acc[q] += wgt * t6[q];
                }
            }
        }
    }
    for (int q = 0; q < 6; ++q) R[q * total + idx] = acc[q];
}

hipError_t launch_tensor_real(const Geom &g, unsigned pmask, int mimg, double dx, double dy,
                              double dz, const double *gl_t, const double *gl_w, double *R,
                              hipStream_t s)
{
    DimImages ix{(int)(pmask & 1u), g.nx, g.mx, mimg};
    DimImages iy{(int)((pmask >> 1) & 1u), g.ny, g.my, mimg};
    DimImages iz{(int)((pmask >> 2) & 1u), g.nz, g.mz, mimg};
    const long long total = (long long)g.mx * g.my * g.mz;
    const long long blocks = (total + 127) / 128;
    hipLaunchKernelGGL(k_tensor_real, dim3((unsigned)blocks), dim3(128), 0, s, g, ix, iy, iz,
                       dx, dy, dz, gl_t, gl_w, R);
    return hipGetLastError();
}

// In-plane k = 0 correction.  Film (pmask 3): one block per (component, z
// position); fully periodic (pmask 7): one block per component.
__global__ void k_tensor_k0(Geom g, int full, double *R)
{
    __shared__ double red[256];
    const int q = blockIdx.y;
    const long long total = (long long)g.mx * g.my * g.mz;
    const int tid = threadIdx.x;
    long long start, count;
    double target;
    if (full) {
        start = 0;
        count = total;
        target = 0.0;
    } else {
        const int iz = blockIdx.x;
        // open z: positions in the zero gap hold no offset
        if (iz >= g.nz && iz <= g.mz - g.nz) return;
        const int dz = iz < g.nz ? iz : iz - g.mz;
        start = (long long)iz * g.mx * g.my;
        count = (long long)g.mx * g.my;
        target = (q == 2 && dz == 0) ? 1.0 : 0.0;
    }
    double *p = R + q * total + start;
    double s = 0.0;
    for (long long i = tid; i < count; i += 256) s += p[i];
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double corr = (target - red[0]) / (double)count;
    for (long long i = tid; i < count; i += 256) p[i] += corr;
}

hipError_t launch_tensor_k0(const Geom &g, unsigned pmask, double *R, double *sums,
                            hipStream_t s)
{
    (void)sums;
    if (pmask == 3u)
        hipLaunchKernelGGL(k_tensor_k0, dim3(g.mz, 6), dim3(256), 0, s, g, 0, R);
    else if (pmask == 7u)
        hipLaunchKernelGGL(k_tensor_k0, dim3(1, 6), dim3(256), 0, s, g, 1, R);
    else
        return hipSuccess;
    return hipGetLastError();
}

// Octant of the real spectrum, scaled:
//   Nt(kx, q, kz, ky) = scale * Re C[kx][q][kz][ky],  kz <= mz/2, ky <= my/2,
// from the full spectrum C[kx][q][mz][my], stored in blocks of KB kx:
// Nt(kx, q, kz, ky) at (((kx/KB)*6 + q)*(mz/2+1) + kz)*(my/2+1) + ky)*KB + kx%KB.
template <typename T>
__global__ void k_tensor_octant(Geom g, const cpx<double> *__restrict__ C, double scale,
                                T *__restrict__ Nt)
{
    const int hy = g.my / 2 + 1, hz = g.mz / 2 + 1;
    const long long total = (long long)g.hx * 6 * hz * hy;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int ky = (int)(idx % hy);
    const int kz = (int)((idx / hy) % hz);
    const long long kq = idx / ((long long)hy * hz);      // kx*6 + q
    const long long src = (kq * g.mz + kz) * g.my + ky;
    // stored in blocks of KB kx, as the spectra that it multiplies
    const long long kx = kq / 6, q = kq - kx * 6;
    const long long dst = ((((kx >> KBS) * 6 + q) * hz + kz) * hy + ky) * KB + (kx & (KB - 1));
    Nt[dst] = (T)(scale * C[src].x);
}

hipError_t launch_tensor_octant(int prec, const Geom &g, const void *C, double scale, void *Nt,
                                hipStream_t s)
{
    const long long total = (long long)g.hx * 6 * (g.mz / 2 + 1) * (g.my / 2 + 1);
    const long long blocks = (total + 255) / 256;
    if (prec == PREC_F32)
        hipLaunchKernelGGL((k_tensor_octant<float>), dim3((unsigned)blocks), dim3(256), 0, s, g,
                           (const cpx<double> *)C, scale, (float *)Nt);
    else
        hipLaunchKernelGGL((k_tensor_octant<double>), dim3((unsigned)blocks), dim3(256), 0, s,
                           g, (const cpx<double> *)C, scale, (double *)Nt);
    return hipGetLastError();
}

}  // namespace tdgl
