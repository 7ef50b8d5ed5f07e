// FP64 tensor setup (Sec. 2 of the paper: generalized Newell formulas for
// cuboids of unequal thickness; appendices A and B for the stencil form).
//
// For a target cell of layer i and a source cell of layer j at lateral offset
// (X, Y) = (p dx, q dy) and Z = z_i - z_j (bottom to bottom):
//   N_kl = -1/(4 pi dx dy t_i) sum_{a,b,c} s_a s_b s_c Phi_kl(X+a, Y+b, Z+c)
// with the x and y stencils {+d: 1, 0: -2, -d: 1} (equal lateral sizes) and the
// z stencil {t_i: 1, 0: -1, t_i - t_j: -1, -t_j: 1}; Phi_xx = f(x,y,z),
// Phi_yy = f(y,x,z), Phi_zz = f(z,x,y), Phi_xy = g(x,y,z), Phi_xz = g(x,z,y),
// Phi_yz = g(y,z,x).
//
// The 64-term sum cancels catastrophically as the separation grows (FP64
// keeps ~1e-9 relative at six cell sizes and nothing at a few hundred).
// Beyond rho = R_centres / max(dx, dy, t_i, t_j) >= 6 the same cell average is
// taken as Gauss-Legendre quadrature of the dipole kernel
//   N_kl = -1/(4 pi |tau|) int_tau int_tau' (3 r_k r_l - r^2 delta_kl) / r^5,
// written as a one-dimensional integral per axis over the difference
// coordinate with the overlap (triangle / trapezoid) weight, split at its
// kinks; n = 5, 4, 3 points per piece for rho < 12, < 32, beyond.
#pragma once
#include "hfd_device.hpp"

namespace hfd {

struct PairGeo {
    double ti, tj, Z, pad;  // target thickness, source thickness, bottom offset
};

// Newell's f and g (closed forms of the two four-fold face integrals).
// Evaluated on absolute values: f is even in every argument; g is odd in its
// first two arguments and even in the third.  Terms with a vanishing
// polynomial prefactor are their limit value 0.
__device__ inline double newell_f(double x, double y, double z)
{
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = (2.0 * x2 - y2 - z2) * R * (1.0 / 6.0);
    const double a = 0.5 * y * (z2 - x2);
    if (a != 0.0) r += a * asinh(y / sqrt(x2 + z2));
    const double b = 0.5 * z * (y2 - x2);
    if (b != 0.0) r += b * asinh(z / sqrt(x2 + y2));
    const double c = x * y * z;
    if (c != 0.0) r -= c * atan(y * z / (x * R));
    return r;
}

__device__ inline double newell_g(double x, double y, double z)
{
    const double s = (x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0)) * (y > 0 ? 1.0 : (y < 0 ? -1.0 : 0.0));
    if (s == 0.0) return 0.0;
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = -x * y * R * (1.0 / 3.0);
    if (z != 0.0) {
        r += x * y * z * asinh(z / sqrt(x2 + y2));
        r -= z2 * z * (1.0 / 6.0) * atan(x * y / (z * R));
        r -= 0.5 * z * y2 * atan(x * z / (y * R));
        r -= 0.5 * z * x2 * atan(y * z / (x * R));
    }
    const double py = y * (3.0 * z2 - y2) * (1.0 / 6.0);
    if (py != 0.0) r += py * asinh(x / sqrt(y2 + z2));
    const double px = x * (3.0 * z2 - x2) * (1.0 / 6.0);
    if (px != 0.0) r += px * asinh(y / sqrt(x2 + z2));
    return s * r;
}

// z-derivatives of the six Phi_kl (for the thickness gradient).
// df/dx and df/dz (f symmetric in its last two arguments), dg/dx (g
// symmetric in its first two) and dg/dz, obtained by differentiating the
// closed forms; all algebraic remainders reduce to the R terms.
__device__ inline double sgnd(double v) { return v > 0 ? 1.0 : (v < 0 ? -1.0 : 0.0); }

__device__ inline double dfdx_nn(double x, double y, double z)  // x, y, z >= 0
{
    const double x2 = x * x, y2 = y * y, z2 = z * z, R = sqrt(x2 + y2 + z2);
    double r = x * R;
    if (x * y != 0.0) r -= x * y * asinh(y / sqrt(x2 + z2));
    if (x * z != 0.0) r -= x * z * asinh(z / sqrt(x2 + y2));
    if (x * y * z != 0.0) r -= y * z * atan(y * z / (x * R));
    return r;
}
__device__ inline double dfdz_nn(double x, double y, double z)
{
    const double x2 = x * x, y2 = y * y, z2 = z * z, R = sqrt(x2 + y2 + z2);
    double r = -0.5 * z * R;
    if (y * z != 0.0) r += y * z * asinh(y / sqrt(x2 + z2));
    if (z != 0.0 && y2 != x2) r += 0.5 * (y2 - x2) * asinh(z / sqrt(x2 + y2));
    if (x * y * z != 0.0) r -= x * y * atan(y * z / (x * R));
    return r;
}
__device__ inline double dgdx_nn(double x, double y, double z)
{
    const double x2 = x * x, y2 = y * y, z2 = z * z, R = sqrt(x2 + y2 + z2);
    double r = -0.5 * y * R;
    if (y * z != 0.0) r += y * z * asinh(z / sqrt(x2 + y2));
    if (y != 0.0 && z2 != x2) r += 0.5 * (z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (x * y * z != 0.0) r -= x * z * atan(y * z / (x * R));
    return r;
}
__device__ inline double dgdz_nn(double x, double y, double z)
{
    const double x2 = x * x, y2 = y * y, z2 = z * z, R = sqrt(x2 + y2 + z2);
    double r = 0.0;
    if (z == 0.0) return 0.0;
    if (x * y != 0.0) {
        r += x * y * asinh(z / sqrt(x2 + y2));
        r -= 0.5 * z2 * atan(x * y / (z * R));
    }
    if (y != 0.0) {
        r += y * z * asinh(x / sqrt(y2 + z2));
        if (x != 0.0) r -= 0.5 * y2 * atan(x * z / (y * R));
    }
    if (x != 0.0) {
        r += x * z * asinh(y / sqrt(x2 + z2));
        if (y != 0.0) r -= 0.5 * x2 * atan(y * z / (x * R));
    }
    return r;
}
// d f(a0, a1, a2) / d a_k at signed arguments (f even -> derivative odd in a_k)
__device__ inline double df_arg(int k, double a0, double a1, double a2)
{
    const double x = fabs(a0), y = fabs(a1), z = fabs(a2);
    if (k == 0) return sgnd(a0) * dfdx_nn(x, y, z);
    if (k == 1) return sgnd(a1) * dfdz_nn(x, z, y);
    return sgnd(a2) * dfdz_nn(x, y, z);
}
// d g(a0, a1, a2) / d a_k (g odd in a0, a1; even in a2)
__device__ inline double dg_arg(int k, double a0, double a1, double a2)
{
    const double x = fabs(a0), y = fabs(a1), z = fabs(a2);
    if (k == 0) return sgnd(a1) * dgdx_nn(x, y, z);
    if (k == 1) return sgnd(a0) * dgdx_nn(y, x, z);
    return sgnd(a0) * sgnd(a1) * sgnd(a2) * dgdz_nn(x, y, z);
}

__device__ inline double phi_c(int c, double x, double y, double z)
{
    switch (c) {
    case 0: return newell_f(x, y, z);
    case 1: return newell_f(y, x, z);
    case 2: return newell_f(z, x, y);
    case 3: return newell_g(x, y, z);
    case 4: return newell_g(x, z, y);
    default: return newell_g(y, z, x);
    }
}
__device__ inline double dphi_dz_c(int c, double x, double y, double z)
{
    switch (c) {
    case 0: return df_arg(2, x, y, z);
    case 1: return df_arg(2, y, x, z);
    case 2: return df_arg(0, z, x, y);
    case 3: return dg_arg(2, x, y, z);
    case 4: return dg_arg(1, x, z, y);
    default: return dg_arg(1, y, z, x);
    }
}

__device__ inline void newell_entry(double X, double Y, double Z, double dx, double dy, double ti,
                                    double tj, double* out)
{
    const double ox[3] = {dx, 0.0, -dx}, oy[3] = {dy, 0.0, -dy}, w3[3] = {1.0, -2.0, 1.0};
    const double oz[4] = {ti, 0.0, ti - tj, -tj}, w4[4] = {1.0, -1.0, -1.0, 1.0};
    const double pref = -1.0 / (4.0 * M_PI * dx * dy * ti);
    for (int c = 0; c < 6; ++c) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += w4[k] * phi_c(c, X + ox[a], Y + oy[b], Z + oz[k]);
                acc += w3[a] * w3[b] * s;
            }
        out[c] = pref * acc;
    }
}

template <int N>
struct GLRule;
template <>
struct GLRule<3> {
    static constexpr double x[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
    static constexpr double w[3] = {0.55555555555555555556, 0.88888888888888888889,
                                    0.55555555555555555556};
};
template <>
struct GLRule<4> {
    static constexpr double x[4] = {-0.86113631159405257522, -0.3399810435848562648,
                                    0.3399810435848562648, 0.86113631159405257522};
    static constexpr double w[4] = {0.34785484513745385737, 0.65214515486254614263,
                                    0.65214515486254614263, 0.34785484513745385737};
};
template <>
struct GLRule<5> {
    static constexpr double x[5] = {-0.9061798459386639928, -0.53846931010568309104, 0.0,
                                    0.53846931010568309104, 0.9061798459386639928};
    static constexpr double w[5] = {0.23692688505618908751, 0.47862867049936646804,
                                    0.56888888888888888889, 0.47862867049936646804,
                                    0.23692688505618908751};
};

template <int N>
__device__ inline void gl_entry(double X, double Y, double Z, double dx, double dy, double ti,
                                double tj, double* out)
{
    using G = GLRule<N>;
    // lateral difference coordinate u in [-d, d], weight (d - |u|)
    double xs[2 * N], wx[2 * N], ys[2 * N], wy[2 * N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double ux = 0.5 * dx * (1.0 + G::x[k]), wxk = 0.5 * dx * G::w[k] * (dx - ux);
        xs[k] = X + ux; xs[N + k] = X - ux; wx[k] = wxk; wx[N + k] = wxk;
        const double uy = 0.5 * dy * (1.0 + G::x[k]), wyk = 0.5 * dy * G::w[k] * (dy - uy);
        ys[k] = Y + uy; ys[N + k] = Y - uy; wy[k] = wyk; wy[N + k] = wyk;
    }
    // z difference v = s - s' in [-tj, ti], weight |[0, ti] cap [v, v + tj]|,
    // linear on the pieces split at 0 and ti - tj
    double zs[3 * N], wz[3 * N];
    int nzn = 0;
    const double a = fmin(0.0, ti - tj), b = fmax(0.0, ti - tj);
    const double lo[3] = {-tj, a, b}, hi[3] = {a, b, ti};
#pragma unroll
    for (int piece = 0; piece < 3; ++piece) {
        const double L = hi[piece] - lo[piece];
        if (!(L > 0.0)) continue;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double v = lo[piece] + 0.5 * L * (1.0 + G::x[k]);
            zs[nzn] = Z + v;
            wz[nzn] = 0.5 * L * G::w[k] * (fmin(ti, v + tj) - fmax(0.0, v));
            ++nzn;
        }
    }
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int iz = 0; iz < nzn; ++iz) {
        const double z = zs[iz];
        double az[6] = {0, 0, 0, 0, 0, 0};
        for (int iy = 0; iy < 2 * N; ++iy) {
            const double y = ys[iy];
            double ay[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int ix = 0; ix < 2 * N; ++ix) {
                const double x = xs[ix];
                const double r2 = x * x + y * y + z * z;
                const double ir = 1.0 / sqrt(r2);
                const double ir2 = ir * ir;
                const double w5 = wx[ix] * ir2 * ir2 * ir;
                ay[0] += w5 * (3.0 * x * x - r2);
                ay[1] += w5 * (3.0 * y * y - r2);
                ay[2] += w5 * (3.0 * z * z - r2);
                ay[3] += w5 * (3.0 * x * y);
                ay[4] += w5 * (3.0 * x * z);
                ay[5] += w5 * (3.0 * y * z);
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) az[c] += wy[iy] * ay[c];
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += wz[iz] * az[c];
    }
    const double pref = -1.0 / (4.0 * M_PI * dx * dy * ti);
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = pref * acc[c];
}

__device__ inline void tensor_entry(double X, double Y, double Z, double dx, double dy, double ti,
                                    double tj, double* out)
{
    const double zc = Z + 0.5 * (ti - tj);
    const double dmax = fmax(fmax(dx, dy), fmax(ti, tj));
    const double rho = sqrt(X * X + Y * Y + zc * zc) / dmax;
    if (rho < 6.0) newell_entry(X, Y, Z, dx, dy, ti, tj, out);
    else if (rho < 12.0) gl_entry<5>(X, Y, Z, dx, dy, ti, tj, out);
    else if (rho < 32.0) gl_entry<4>(X, Y, Z, dx, dy, ti, tj, out);
    else gl_entry<3>(X, Y, Z, dx, dy, ti, tj, out);
}

// parity sign of component c under x -> -x (sx = -1) and y -> -y (sy = -1)
__device__ inline double parity_sign(int c, int sx, int sy)
{
    switch (c) {
    case 3: return (double)(sx * sy);  // xy odd, odd
    case 4: return (double)sx;         // xz odd in x
    case 5: return (double)sy;         // yz odd in y
    default: return 1.0;
    }
}

// Real-space tensor of `npairs` pairs on the quadrant p in [0, nx), q in [0, ny).
// mode 0: write the zero-padded periodic arrays W[pair][6][Ly][Lx] (all four
//         sign images); W must be zeroed beforehand.
// mode 1: write the offset table W[pair][6][2ny-1][2nx-1].
__global__ __launch_bounds__(128) void k_tensor_real(double* __restrict__ W,
                                                     const PairGeo* __restrict__ pg, int npairs,
                                                     int nx, int ny, int Lx, int Ly, double dx,
                                                     double dy, int mode)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)nx * ny;
    if (idx >= per * npairs) return;
    const int u = (int)(idx / per);
    const int q = (int)((idx / nx) % ny), p = (int)(idx % nx);
    const PairGeo G = pg[u];
    double N[6];
    tensor_entry(p * dx, q * dy, G.Z, dx, dy, G.ti, G.tj, N);
    if (p == 0) { N[3] = 0.0; N[4] = 0.0; }  // odd in x
    if (q == 0) { N[3] = 0.0; N[5] = 0.0; }  // odd in y
    if (mode == 0) {
        const long long plane = (long long)Lx * Ly;
        double* base = W + (long long)u * 6 * plane;
        for (int sy = 1; sy >= -1; sy -= 2) {
            if (sy < 0 && q == 0) continue;
            const int qq = sy > 0 ? q : Ly - q;
            for (int sx = 1; sx >= -1; sx -= 2) {
                if (sx < 0 && p == 0) continue;
                const int pp = sx > 0 ? p : Lx - p;
                for (int c = 0; c < 6; ++c)
                    base[c * plane + (long long)qq * Lx + pp] = parity_sign(c, sx, sy) * N[c];
            }
        }
    } else {
        const int Wo = 2 * nx - 1, Ho = 2 * ny - 1;
        const long long plane = (long long)Wo * Ho;
        double* base = W + (long long)u * 6 * plane;
        for (int sy = 1; sy >= -1; sy -= 2) {
            if (sy < 0 && q == 0) continue;
            for (int sx = 1; sx >= -1; sx -= 2) {
                if (sx < 0 && p == 0) continue;
                const int pi = sx * p + nx - 1, qi = sy * q + ny - 1;
                for (int c = 0; c < 6; ++c)
                    base[c * plane + (long long)qi * Wo + pi] = parity_sign(c, sx, sy) * N[c];
            }
        }
    }
}

// Lateral-stencilled z-derivative of Phi at height zeta (one per distinct
// interface difference):  d(p, q) = -1/(4 pi dx dy) sum_{a,b} s_a s_b
// dPhi_kl/dz(p dx + a, q dy + b, zeta), written like mode 0 above.
// The stencil points of neighbouring lattice entries are the lattice points
// themselves, so a block evaluates dPhi/dz once on its tile of 16 x 16
// entries plus a one-point halo (18 x 18 points, LDS) and applies the 3 x 3
// stencil from there: 1.3 evaluations per entry and component instead of 9.
constexpr int kDTile = 16;
__global__ __launch_bounds__(kDTile * kDTile) void k_dtensor_real(double* __restrict__ W,
                                                                  const double* __restrict__ zeta,
                                                                  int nx, int ny, int Lx, int Ly,
                                                                  double dx, double dy)
{
    constexpr int E = kDTile + 2;  // tile with halo
    __shared__ double F[6][E][E];
    const int u = blockIdx.z;
    const int p0 = blockIdx.x * kDTile, q0 = blockIdx.y * kDTile;
    const double zt = zeta[u];
    for (int k = threadIdx.x; k < E * E; k += blockDim.x) {
        const int ey = k / E, ex = k - ey * E;
        const double X = (double)(p0 + ex - 1) * dx, Y = (double)(q0 + ey - 1) * dy;
        for (int c = 0; c < 6; ++c) F[c][ey][ex] = dphi_dz_c(c, X, Y, zt);
    }
    __syncthreads();
    const int tx = threadIdx.x % kDTile, ty = threadIdx.x / kDTile;
    const int p = p0 + tx, q = q0 + ty;
    if (p >= nx || q >= ny) return;
    // offsets {+d, 0, -d} with weights {1, -2, 1}, as in newell_entry
    const int oi[3] = {1, 0, -1};
    const double w3[3] = {1.0, -2.0, 1.0};
    const double pref = -1.0 / (4.0 * M_PI * dx * dy);
    double N[6];
    for (int c = 0; c < 6; ++c) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) acc += w3[a] * w3[b] * F[c][ty + 1 + oi[b]][tx + 1 + oi[a]];
        N[c] = pref * acc;
    }
    if (p == 0) { N[3] = 0.0; N[4] = 0.0; }
    if (q == 0) { N[3] = 0.0; N[5] = 0.0; }
    const long long plane = (long long)Lx * Ly;
    double* base = W + (long long)u * 6 * plane;
    for (int sy = 1; sy >= -1; sy -= 2) {
        if (sy < 0 && q == 0) continue;
        const int qq = sy > 0 ? q : Ly - q;
        for (int sx = 1; sx >= -1; sx -= 2) {
            if (sx < 0 && p == 0) continue;
            const int pp = sx > 0 ? p : Lx - p;
            for (int c = 0; c < 6; ++c)
                base[c * plane + (long long)qq * Lx + pp] = parity_sign(c, sx, sy) * N[c];
        }
    }
}

// Pack the FP64 2D spectra F[nsig][M][Ly] (x pass packed, column 0 = kx 0 and
// Lx/2) of arrays with the lateral parity of the tensor into the quadrant
// kx in [0, M], ky in [0, Ly/2]: real part for the even-even and odd-odd
// components, imaginary part for the odd-even ones, times scale[pair].
// comps: number of stored components per pair (5: xx, yy, xy, xz, yz;
// 6: all); the source has 6 arrays per pair in the order xx yy zz xy xz yz.
// row_outer: output [kx][pair_total][comps][ky] with this call's pairs at
// pair0 (each kx row of a table contiguous); else [pair][comp][kx][ky].
template <typename R>
__global__ __launch_bounds__(256) void k_pack(const cpx<double>* __restrict__ F, R* __restrict__ Qout,
                                              const double* __restrict__ scale, int npairs, int comps,
                                              int M, int Ly, int QX, int QY, int pair0,
                                              int pair_total, int row_outer)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)comps * QX * QY;
    if (idx >= per * npairs) return;
    const int u = (int)(idx / per);
    const long long rem = idx % per;
    const int c = (int)(rem / ((long long)QX * QY));
    const int kx = (int)((rem / QY) % QX), ky = (int)(rem % QY);
    const int c6 = comps == 5 ? (c < 2 ? c : c + 1) : c;
    const cpx<double>* Fs = F + ((long long)u * 6 + c6) * M * Ly;
    cpx<double> val;
    if (kx == 0 || kx == M) {
        const cpx<double> z1 = Fs[ky], z2 = Fs[(Ly - ky) & (Ly - 1)];
        if (kx == 0) val = {0.5 * (z1.x + z2.x), 0.5 * (z1.y - z2.y)};
        else val = {0.5 * (z1.y + z2.y), 0.5 * (z2.x - z1.x)};
    } else {
        val = Fs[(long long)kx * Ly + ky];
    }
    const bool imag = (c6 == 4 || c6 == 5);
    const long long o = row_outer
        ? (((long long)kx * pair_total + pair0 + u) * comps + c) * QY + ky
        : idx;
    Qout[o] = (R)((imag ? val.y : val.x) * scale[u]);
}

}  // namespace hfd
