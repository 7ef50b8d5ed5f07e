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
// kinks; n = 5, 4, 3, 2 points per piece for rho < 12, < 32, < 100, beyond
// (the 2-point rule's error there is ~1e-9 of the entry and falls as rho^-4).
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

// Gauss-Legendre rules on [-1, 1] with n = 2 .. 5 points (row n - 2).
struct GLTable {
    double x[4][5], w[4][5];
};
constexpr GLTable kGL = {
    {{-0.57735026918962576451, 0.57735026918962576451},
     {-0.77459666924148337704, 0.0, 0.77459666924148337704},
     {-0.86113631159405257522, -0.3399810435848562648, 0.3399810435848562648, 0.86113631159405257522},
     {-0.9061798459386639928, -0.53846931010568309104, 0.0, 0.53846931010568309104,
      0.9061798459386639928}},
    {{1.0, 1.0},
     {0.55555555555555555556, 0.88888888888888888889, 0.55555555555555555556},
     {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263, 0.34785484513745385737},
     {0.23692688505618908751, 0.47862867049936646804, 0.56888888888888888889, 0.47862867049936646804,
      0.23692688505618908751}}};
// the same table in device memory, for loops over nodes that are not unrolled
__constant__ GLTable kGLDev = kGL;

// 1 / sqrt(r2) from the hardware estimate and one Newton step for
// f(y) = y^-2 - r2 (the estimate's relative error e becomes ~1.5 e^2)
__device__ inline double rsqrt_newton(double r2)
{
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-r2 * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// Cell average of the dipole kernel by n-point Gauss-Legendre quadrature.
// Lateral axes: the difference coordinate u in [-d, d] with weight d - |u|,
// written as the points X + u_k and X - u_k for the nodes u_k of [0, d] (the
// kink at u = 0 is an end point).  For one z point and one y point the x sums
//   A0 = sum w r^-5,  A1 = sum w x r^-5,  A2 = sum w x^2 r^-5
// give every component: with c = y^2 + z^2,
//   xx: 2 A2 - c A0,   yy: (2 y^2 - z^2) A0 - A2,   xy: 3 y A1,
//   xz: 3 z A1,        yz: 3 y z A0,                zz = -(xx + yy);
// the y sums of A0, y A0, y^2 A0, A1, y A1, A2 carry them to the z level.
// gl_znode adds the weighted contribution of one z point to S = (xx, yy, xy,
// xz, yz).
template <int N>
__device__ inline void gl_znode(const double* xp, const double* xm, const double* wx, double Y,
                                double dy, double z, double wz, double* S)
{
    constexpr int R = N - 2;
    const double z2 = z * z;
    double B0 = 0.0, By = 0.0, Byy = 0.0, B1 = 0.0, B1y = 0.0, B2 = 0.0;
#pragma unroll
    for (int ky = 0; ky < N; ++ky) {
        const double uy = 0.5 * dy * (1.0 + kGL.x[R][ky]);
        const double wy = 0.5 * dy * kGL.w[R][ky] * (dy - uy);
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            const double y = sy ? Y - uy : Y + uy;
            const double c = fma(y, y, z2);
            double A0 = 0.0, A1 = 0.0, A2 = 0.0;
#pragma unroll
            for (int kx = 0; kx < N; ++kx) {
#pragma unroll
                for (int sx = 0; sx < 2; ++sx) {
                    const double x = sx ? xm[kx] : xp[kx];
                    const double ir = rsqrt_newton(fma(x, x, c));
                    const double ir2 = ir * ir;
                    const double w5 = wx[kx] * (ir2 * ir2 * ir);
                    const double t = w5 * x;
                    A0 += w5;
                    A1 += t;
                    A2 = fma(t, x, A2);
                }
            }
            const double t0 = wy * A0, t1 = wy * A1, ty0 = t0 * y;
            B0 += t0;
            By += ty0;
            Byy = fma(ty0, y, Byy);
            B1 += t1;
            B1y = fma(t1, y, B1y);
            B2 = fma(wy, A2, B2);
        }
    }
    S[0] = fma(wz, 2.0 * B2 - Byy - z2 * B0, S[0]);
    S[1] = fma(wz, 2.0 * Byy - z2 * B0 - B2, S[1]);
    S[2] = fma(wz, 3.0 * B1y, S[2]);
    S[3] = fma(wz, 3.0 * z * B1, S[3]);
    S[4] = fma(wz, 3.0 * z * By, S[4]);
}

// z axis: for n >= 3 the difference coordinate v = s - s' in [-tj, ti] with
// weight |[0, ti] cap [v, v + tj]|, linear on the pieces split at 0 and
// ti - tj (3n points, 2n for equal thicknesses); for n = 2 the product of the
// two cells' own 2-point rules (4 points; the same error order, fewer points
// when the thicknesses differ).  z_node gives point k of the list (k < 4 for
// n = 2, k < 3n otherwise) and its weight; false for the points of an empty
// piece.
template <int N>
__device__ inline bool z_node(int k, double ti, double tj, double& v, double& wz)
{
    constexpr int R = N - 2;
    if (N == 2) {
        v = 0.5 * ti * (1.0 + kGLDev.x[0][k >> 1]) - 0.5 * tj * (1.0 + kGLDev.x[0][k & 1]);
        wz = 0.25 * ti * tj;
        return true;
    }
    const int piece = k / N, kz = k - piece * N;
    const double a = fmin(0.0, ti - tj), b = fmax(0.0, ti - tj);
    const double lo = piece == 0 ? -tj : (piece == 1 ? a : b);
    const double hi = piece == 0 ? a : (piece == 1 ? b : ti);
    const double L = hi - lo;
    if (!(L > 0.0)) return false;
    v = lo + 0.5 * L * (1.0 + kGLDev.x[R][kz]);
    wz = 0.5 * L * kGLDev.w[R][kz] * (fmin(ti, v + tj) - fmax(0.0, v));
    return true;
}
template <int N>
__device__ inline int z_count()
{
    return N == 2 ? 4 : 3 * N;
}

// lateral nodes of the x axis: X + u_k, X - u_k and their weight
template <int N>
__device__ inline void x_nodes(double X, double dx, double* xp, double* xm, double* wx)
{
    constexpr int R = N - 2;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double u = 0.5 * dx * (1.0 + kGL.x[R][k]);
        xp[k] = X + u;
        xm[k] = X - u;
        wx[k] = 0.5 * dx * kGL.w[R][k] * (dx - u);
    }
}

// the six components from the z-level sums S = (xx, yy, xy, xz, yz)
__device__ inline void gl_finish(const double* S, double dx, double dy, double ti, double* out)
{
    const double pref = -1.0 / (4.0 * M_PI * dx * dy * ti);
    out[0] = pref * S[0];
    out[1] = pref * S[1];
    out[2] = -(out[0] + out[1]);
    out[3] = pref * S[2];
    out[4] = pref * S[3];
    out[5] = pref * S[4];
}

template <int N>
__device__ inline void gl_entry(double X, double Y, double Z, double dx, double dy, double ti,
                                double tj, double* out)
{
    double xp[N], xm[N], wx[N];
    x_nodes<N>(X, dx, xp, xm, wx);
    double S[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < z_count<N>(); ++k) {
        double v, wz;
        if (z_node<N>(k, ti, tj, v, wz)) gl_znode<N>(xp, xm, wx, Y, dy, Z + v, wz, S);
    }
    gl_finish(S, dx, dy, ti, out);
}

// Centre distance of the entry in units of the largest cell size; decides
// between the 64-term form (rho < 6) and quadrature.  No contraction, so that
// the two kernels below, which split the entries by it, round it alike.
__device__ inline double entry_rho(double X, double Y, double Z, double dx, double dy, double ti,
                                   double tj)
{
#pragma clang fp contract(off)
    const double zc = Z + 0.5 * (ti - tj);
    const double dmax = fmax(fmax(dx, dy), fmax(ti, tj));
    return sqrt(X * X + Y * Y + zc * zc) / dmax;
}
constexpr double kNearRho = 6.0, kMidRho = 32.0;

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

// Write component c of the quadrant entry (p, q) of pair u.
// mode 1: the offset table W[pair][6][2ny-1][2nx-1], with the sign images;
// mode 2: the quadrant alone, W[pair][6][ny][nx] (the transforms supply the images).
__device__ inline void store_component(double* __restrict__ W, int mode, int u, int c, int p, int q,
                                       double v, int nx, int ny)
{
    if ((p == 0 && (c == 3 || c == 4)) || (q == 0 && (c == 3 || c == 5))) v = 0.0;  // odd axes
    if (mode == 2) {
        W[(((long long)u * 6 + c) * ny + q) * nx + p] = v;
        return;
    }
    const int Wo = 2 * nx - 1, Ho = 2 * ny - 1;
    double* base = W + ((long long)u * 6 + c) * Wo * Ho;
    for (int sy = 1; sy >= -1; sy -= 2) {
        if (sy < 0 && q == 0) continue;
        for (int sx = 1; sx >= -1; sx -= 2) {
            if (sx < 0 && p == 0) continue;
            base[(long long)(sy * q + ny - 1) * Wo + (sx * p + nx - 1)] = parity_sign(c, sx, sy) * v;
        }
    }
}

// Real-space tensor of `npairs` pairs on the quadrant p in [0, nx), q in [0, ny),
// in three launches that split the entries at rho = 6 and rho = 32 (see
// store_component for the output modes).
//
// Near entries (64-term form) on tiles of kNTile x kNTile entries of the box
// p < pn, q < qn that holds every entry with rho < 6.  The lateral stencil
// points of neighbouring entries are the lattice points themselves, so a
// block first evaluates Phi_c at the tile's lattice points plus a one-point
// halo, for the four z offsets of the z stencil (LDS), then each (entry,
// component) applies the 3 x 3 x 4 stencil from there: 2.25 evaluations per
// entry and term instead of 9, in the summation order of the direct sum.
// Items are ordered component-major so that a wave evaluates one Phi_c.
constexpr int kNTile = 4;
__global__ __launch_bounds__(256) void k_tensor_near(double* __restrict__ W,
                                                     const PairGeo* __restrict__ pg, int nx, int ny,
                                                     double dx, double dy, int mode,
                                                     int pn, int qn)
{
    constexpr int E = kNTile + 2, EE = E * E;
    __shared__ double F[6][4][EE];
    const int u = blockIdx.z;
    const int p0 = blockIdx.x * kNTile, q0 = blockIdx.y * kNTile;
    const PairGeo G = pg[u];
    const double oz[4] = {G.ti, 0.0, G.ti - G.tj, -G.tj};
    for (int i = threadIdx.x; i < 6 * 4 * EE; i += blockDim.x) {
        const int c = i / (4 * EE), k = (i / EE) % 4, e = i % EE;
        const int ey = e / E, ex = e - ey * E;
        F[c][k][e] = phi_c(c, (double)(p0 + ex - 1) * dx, (double)(q0 + ey - 1) * dy, G.Z + oz[k]);
    }
    __syncthreads();
    if (threadIdx.x >= 6 * kNTile * kNTile) return;
    const int c = threadIdx.x / (kNTile * kNTile), t = threadIdx.x % (kNTile * kNTile);
    const int tx = t % kNTile, ty = t / kNTile;
    const int p = p0 + tx, q = q0 + ty;
    if (p >= pn || q >= qn || p >= nx || q >= ny) return;
    if (!(entry_rho(p * dx, q * dy, G.Z, dx, dy, G.ti, G.tj) < kNearRho)) return;
    // offsets {+d, 0, -d} with weights {1, -2, 1}; z weights {1, -1, -1, 1}
    const int oi[3] = {1, 0, -1};
    const double w3[3] = {1.0, -2.0, 1.0}, w4[4] = {1.0, -1.0, -1.0, 1.0};
    double acc = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const int e = (ty + 1 + oi[b]) * E + (tx + 1 + oi[a]);
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += w4[k] * F[c][k][e];
            acc += w3[a] * w3[b] * s;
        }
    const double pref = -1.0 / (4.0 * M_PI * dx * dy * G.ti);
    store_component(W, mode, u, c, p, q, pref * acc, nx, ny);
}

// Entries with 6 <= rho < 32 (5 and 4 points per piece, up to 15 z points
// of 100 and 64 lateral points each) over the box p < pm, q < qm that holds
// them: 16 lanes per entry, one z point per lane, summed across the lanes, so
// that no lane runs the whole entry alone.
constexpr int kMidLanes = 16;
__global__ __launch_bounds__(256) void k_tensor_mid(double* __restrict__ W,
                                                    const PairGeo* __restrict__ pg, int nx, int ny,
                                                    double dx, double dy, int mode,
                                                    int pm, int qm)
{
    const int l = threadIdx.x % kMidLanes;
    const int e = blockIdx.x * (256 / kMidLanes) + threadIdx.x / kMidLanes;
    const int u = blockIdx.y;
    // every test below is the same for the 16 lanes of an entry
    if (e >= pm * qm) return;
    const int p = e % pm, q = e / pm;
    if (p >= nx || q >= ny) return;
    const PairGeo G = pg[u];
    const double X = p * dx, Y = q * dy;
    const double rho = entry_rho(X, Y, G.Z, dx, dy, G.ti, G.tj);
    if (rho < kNearRho || !(rho < kMidRho)) return;
    double S[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double v, wz;
    if (rho < 12.0) {
        double xp[5], xm[5], wx[5];
        x_nodes<5>(X, dx, xp, xm, wx);
        if (l < z_count<5>() && z_node<5>(l, G.ti, G.tj, v, wz))
            gl_znode<5>(xp, xm, wx, Y, dy, G.Z + v, wz, S);
    } else {
        double xp[4], xm[4], wx[4];
        x_nodes<4>(X, dx, xp, xm, wx);
        if (l < z_count<4>() && z_node<4>(l, G.ti, G.tj, v, wz))
            gl_znode<4>(xp, xm, wx, Y, dy, G.Z + v, wz, S);
    }
#pragma unroll
    for (int off = kMidLanes / 2; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < 5; ++i) S[i] += __shfl_xor(S[i], off, kMidLanes);
    double N[6];
    gl_finish(S, dx, dy, G.ti, N);
    if (l < 6) store_component(W, mode, u, l, p, q, N[l], nx, ny);
}

// Entries with rho >= 32 (3 points per piece below rho = 100, 2 beyond), one
// thread per entry: blocks of 16 x 16 entries, 8 x 8 per wave.  The block
// index runs over the pairs fastest and then over the tile rows from the
// origin outwards, so that the tiles with the most points start first.
__global__ __launch_bounds__(256) void k_tensor_far(double* __restrict__ W,
                                                    const PairGeo* __restrict__ pg, int npairs,
                                                    int nx, int ny, double dx, double dy,
                                                    int mode)
{
    const int u = (int)(blockIdx.x % (unsigned)npairs), t = (int)(blockIdx.x / (unsigned)npairs);
    const int ntx = (nx + 15) / 16;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = (t % ntx) * 16 + (w & 1) * 8 + (lane & 7);
    const int q = (t / ntx) * 16 + (w >> 1) * 8 + (lane >> 3);
    if (p >= nx || q >= ny) return;
    const PairGeo G = pg[u];
    const double X = p * dx, Y = q * dy;
    const double rho = entry_rho(X, Y, G.Z, dx, dy, G.ti, G.tj);
    if (rho < kMidRho) return;
    double N[6];
    if (rho < 100.0) gl_entry<3>(X, Y, G.Z, dx, dy, G.ti, G.tj, N);
    else gl_entry<2>(X, Y, G.Z, dx, dy, G.ti, G.tj, N);
#pragma unroll
    for (int c = 0; c < 6; ++c) store_component(W, mode, u, c, p, q, N[c], nx, ny);
}

// Lateral-stencilled z-derivative of Phi at height zeta (one per distinct
// interface difference):  d(p, q) = -1/(4 pi dx dy) sum_{a,b} s_a s_b
// dPhi_kl/dz(p dx + a, q dy + b, zeta), written as quadrants W[zeta][6][ny][nx].
// The stencil points of neighbouring lattice entries are the lattice points
// themselves, so a block evaluates dPhi/dz once on its tile of 16 x 16
// entries plus a one-point halo (18 x 18 points, LDS) and applies the 3 x 3
// stencil from there: 1.3 evaluations per entry and component instead of 9.
constexpr int kDTile = 16;
__global__ __launch_bounds__(kDTile * kDTile) void k_dtensor_real(double* __restrict__ W,
                                                                  const double* __restrict__ zeta,
                                                                  int nx, int ny, double dx,
                                                                  double dy)
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
    // offsets {+d, 0, -d} with weights {1, -2, 1}, as in k_tensor_near
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
    for (int c = 0; c < 6; ++c) W[(((long long)u * 6 + c) * ny + q) * nx + p] = N[c];
}

// y transforms of the tensor tables and their packing, in one kernel.
// Input: the x-pass spectra of the ny quadrant rows, F[pair][6][M + 1][ny]
// (FP64): for each component the non-zero part of its x transform, real for
// the x-even components (xx, yy, zz, yz) and imaginary for the x-odd ones
// (xy, xz).  A column is extended to length Ly by its y parity: v(y) for
// y < ny, sy v(Ly - y) for Ly - y < ny, zero between (sy = -1 for the y-odd
// xy and yz).  The y transform of a real y-even column is real, of a y-odd
// one imaginary, so two columns of the same y parity take one complex
// transform z = a + i b whose real and imaginary parts are the two results
// (y odd: Z = i (A' + i B'), A' = Im Z, B' = -Re Z): the pairs (xx, yy),
// (zz, xz) and (xy, yz), three transforms per column instead of six.
// Output per component, the quadrant kx in [0, M], ky in [0, Ly/2] of the 2D
// transform: its real part for xx, yy, zz, xy, its imaginary part for xz, yz
// (the non-zero one), times scale[pair].  With F = i f for an x-odd column:
// xy = Re(i i A') = -A', xz = Im(i A) = A; yz = Im(i A') = A'.
// comps: 5 (xx, yy, xy, xz, yz; zz follows from the trace) or 6 (all, in the
// order xx yy zz xy xz yz); row_outer: output [kx][pair_total][comps][ky] with
// this call's pairs at pair0, else [pair][comps][kx][ky].  src (optional): the
// spectra of output pair u are F[src[u]], none if src[u] < 0.
template <int LY>
struct TabShape {
    static constexpr int V = fft_vals(LY);
    static constexpr int GT = LY / V;
    static constexpr int NG0 = 256 / GT;
    static constexpr int NGL = (int)(65536 / (sizeof(cpx<double>) * fft_region(LY)));
    static constexpr int NG = NG0 < NGL ? NG0 : (NGL < 1 ? 1 : NGL);
    static constexpr int NT = NG * GT;
};

template <typename R, int LY>
__global__ __launch_bounds__((TabShape<LY>::NT)) void k_ytab(
    const double* __restrict__ F, R* __restrict__ Qout, const double* __restrict__ scale,
    int npairs, int comps, int M, int ny, int QX, int QY, int pair0, int pair_total, int row_outer,
    const int* __restrict__ src, const cpx<double>* __restrict__ twy)
{
    using S = TabShape<LY>;
    __shared__ cpx<double> sh[S::NG * fft_region(LY)];
    const int grp = threadIdx.x / S::GT, g = threadIdx.x % S::GT;
    const int ncol = M + 1;
    const long long task = (long long)blockIdx.x * S::NG + grp;
    if (task >= (long long)npairs * ncol * 3) return;
    const int k = (int)(task % 3);
    const int kx = (int)((task / 3) % ncol);
    const int u = (int)(task / (3LL * ncol));
    const int su = src ? src[u] : u;
    if (su < 0) return;
    const double sc = scale[u];
    // the pair of columns: (xx, yy), (zz, xz), (xy, yz); the third is y-odd
    const int c1 = k == 0 ? 0 : (k == 1 ? 2 : 3), c2 = k == 0 ? 1 : (k == 1 ? 4 : 5);
    const double sy = k == 2 ? -1.0 : 1.0;
    const double* a = F + (((long long)su * 6 + c1) * ncol + kx) * ny;
    const double* b = F + (((long long)su * 6 + c2) * ncol + kx) * ny;
    auto put = [&](int c6, int ky, double v) {
        const int oc = comps == 6 ? c6 : (c6 < 2 ? c6 : (c6 == 2 ? -1 : c6 - 1));
        if (oc < 0) return;
        const long long o = row_outer
            ? (((long long)tab_row(kx, M) * pair_total + pair0 + u) * comps + oc) * QY + ky
            : (((long long)u * comps + oc) * QX + kx) * QY + ky;
        Qout[o] = (R)(v * sc);
    };
    wave_fft<double, LY, false>(
        sh + grp * fft_region(LY), g, twy, 1,
        [&](int pos) -> cpx<double> {
            if (pos < ny) return {a[pos], b[pos]};
            const int m = LY - pos;
            if (m < ny) return {sy * a[m], sy * b[m]};
            return {0.0, 0.0};
        },
        [&](int pos, cpx<double> z) {
            if (pos > LY / 2) return;
            if (k < 2) {
                put(c1, pos, z.x);
                put(c2, pos, z.y);
            } else {
                put(3, pos, -z.y);
                put(5, pos, -z.x);
            }
        });
}

}  // namespace hfd
