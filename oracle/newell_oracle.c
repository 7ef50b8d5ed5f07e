/*
 * Reference oracle for the hybrid-FFT demagnetization field on non-equidistant
 * layers (Heistracher et al., arXiv:1910.07054).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow CPU implementation of
 * what the GPU library computes.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * HIP library and must never be called on the product path.
 *
 * Precision: every Newell kernel value and every stencil sum is carried in
 * x87 extended precision (`long double`, 64-bit mantissa).  The 64-term
 * difference that forms a tensor entry cancels catastrophically at large
 * separation (the paper calls the method exact and is silent on floating
 * point); extended precision keeps the cancellation error roughly 2000x below
 * that of an FP64 evaluation, which is still not enough beyond some fifty
 * cell sizes.  Layer-pair table entries whose cuboid centres are at least FAR_RHO
 * times the largest cell dimension apart are therefore taken from the
 * definition the closed forms integrate: the cell-averaged dipole kernel,
 * integrated over both cuboids by tensor-product Gauss-Legendre quadrature
 * (smooth there, so a few points per axis reach rounding level).  Field sums
 * are accumulated in FP64.
 *
 * Conventions (Sec. 2 of the paper, "Generalized Newell Equation"):
 *   - the tensor N relates a source cuboid at the origin with dimensions
 *     (dx', dy', dz') to a target cuboid of dimensions (dx, dy, dz) whose
 *     origin sits at the offset (X, Y, Z);
 *   - the averaged field in the target is  <h> = -N m_source;
 *   - component order everywhere: xx, yy, zz, xy, xz, yz.
 *
 * Parity of the kernels (even/odd in each argument) is used only to evaluate
 * f and g on absolute values, which is an identity of the closed forms.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long double LD;

#define PI_L 3.141592653589793238462643383279502884L

/* ------------------------------------------------------------------------ */
/* Newell kernels f and g (Sec. 2.1, closed form of F2's antiderivative, and */
/* Sec. 2.2, closed form of G2's antiderivative).                            */
/* A term whose polynomial prefactor vanishes is dropped: that is its limit  */
/* value, and it avoids the 0/0 inside the inverse functions.                */
/* ------------------------------------------------------------------------ */

static LD f_pos(LD x, LD y, LD z) /* x, y, z >= 0 */
{
    LD x2 = x * x, y2 = y * y, z2 = z * z;
    LD R = sqrtl(x2 + y2 + z2);
    LD r = 0.0L;
    LD p1 = 0.5L * y * (z2 - x2);
    if (p1 != 0.0L) r += p1 * asinhl(y / sqrtl(x2 + z2));
    LD p2 = 0.5L * z * (y2 - x2);
    if (p2 != 0.0L) r += p2 * asinhl(z / sqrtl(x2 + y2));
    LD p3 = x * y * z;
    if (p3 != 0.0L) r -= p3 * atanl(y * z / (x * R));
    r += (2.0L * x2 - y2 - z2) * R / 6.0L;
    return r;
}

static LD g_pos(LD x, LD y, LD z) /* x, y, z >= 0 */
{
    LD x2 = x * x, y2 = y * y, z2 = z * z;
    LD R = sqrtl(x2 + y2 + z2);
    LD r = 0.0L;
    LD p1 = x * y * z;
    if (p1 != 0.0L) r += p1 * asinhl(z / sqrtl(x2 + y2));
    LD p2 = y * (3.0L * z2 - y2) / 6.0L;
    if (p2 != 0.0L) r += p2 * asinhl(x / sqrtl(y2 + z2));
    LD p3 = x * (3.0L * z2 - x2) / 6.0L;
    if (p3 != 0.0L) r += p3 * asinhl(y / sqrtl(x2 + z2));
    LD p4 = z2 * z / 6.0L;
    if (p4 != 0.0L) r -= p4 * atanl(x * y / (z * R));
    LD p5 = 0.5L * z * y2;
    if (p5 != 0.0L) r -= p5 * atanl(x * z / (y * R));
    LD p6 = 0.5L * z * x2;
    if (p6 != 0.0L) r -= p6 * atanl(y * z / (x * R));
    r -= x * y * R / 3.0L;
    return r;
}

static LD sgn(LD v) { return v > 0 ? 1.0L : (v < 0 ? -1.0L : 0.0L); }

/* f is even in every argument. */
static LD f_ld(LD x, LD y, LD z) { return f_pos(fabsl(x), fabsl(y), fabsl(z)); }
/* g is odd in its first two arguments and even in the third. */
static LD g_ld(LD x, LD y, LD z)
{
    return sgn(x) * sgn(y) * g_pos(fabsl(x), fabsl(y), fabsl(z));
}

/* Partial derivatives of f and g (derived by differentiating the closed
 * forms above; the algebraic remainders collapse to the R terms).  They are
 * used only for the thickness gradient and are pinned against finite
 * differences of f and g by the tests. */
static LD dfdx_pos(LD x, LD y, LD z)
{
    LD x2 = x * x, y2 = y * y, z2 = z * z, R = sqrtl(x2 + y2 + z2), r = x * R;
    if (x * y != 0.0L) r -= x * y * asinhl(y / sqrtl(x2 + z2));
    if (x * z != 0.0L) r -= x * z * asinhl(z / sqrtl(x2 + y2));
    if (y * z != 0.0L && x != 0.0L) r -= y * z * atanl(y * z / (x * R));
    return r;
}
static LD dfdz_pos(LD x, LD y, LD z)
{
    LD x2 = x * x, y2 = y * y, z2 = z * z, R = sqrtl(x2 + y2 + z2), r = -0.5L * z * R;
    if (y * z != 0.0L) r += y * z * asinhl(y / sqrtl(x2 + z2));
    if ((y2 - x2) != 0.0L && z != 0.0L) r += 0.5L * (y2 - x2) * asinhl(z / sqrtl(x2 + y2));
    if (x * y != 0.0L && z != 0.0L) r -= x * y * atanl(y * z / (x * R));
    return r;
}
static LD dgdx_pos(LD x, LD y, LD z)
{
    LD x2 = x * x, y2 = y * y, z2 = z * z, R = sqrtl(x2 + y2 + z2), r = -0.5L * y * R;
    if (y * z != 0.0L) r += y * z * asinhl(z / sqrtl(x2 + y2));
    if ((z2 - x2) != 0.0L && y != 0.0L) r += 0.5L * (z2 - x2) * asinhl(y / sqrtl(x2 + z2));
    if (x * z != 0.0L && y != 0.0L) r -= x * z * atanl(y * z / (x * R));
    return r;
}
static LD dgdz_pos(LD x, LD y, LD z)
{
    LD x2 = x * x, y2 = y * y, z2 = z * z, R = sqrtl(x2 + y2 + z2), r = 0.0L;
    if (x * y != 0.0L && z != 0.0L) r += x * y * asinhl(z / sqrtl(x2 + y2));
    if (y * z != 0.0L && x != 0.0L) r += y * z * asinhl(x / sqrtl(y2 + z2));
    if (x * z != 0.0L && y != 0.0L) r += x * z * asinhl(y / sqrtl(x2 + z2));
    if (z != 0.0L) {
        if (x * y != 0.0L) r -= 0.5L * z2 * atanl(x * y / (z * R));
        if (y != 0.0L && x * z != 0.0L) r -= 0.5L * y2 * atanl(x * z / (y * R));
        if (x != 0.0L && y * z != 0.0L) r -= 0.5L * x2 * atanl(y * z / (x * R));
    }
    return r;
}
/* d f / d(arg a) with the parity of f (even): derivative is odd in arg a. */
static LD df_ld(int a, LD x, LD y, LD z)
{
    LD ax = fabsl(x), ay = fabsl(y), az = fabsl(z);
    switch (a) {
    case 0: return sgn(x) * dfdx_pos(ax, ay, az);
    case 1: return sgn(y) * dfdz_pos(ax, az, ay); /* f symmetric in (y, z) */
    default: return sgn(z) * dfdz_pos(ax, ay, az);
    }
}
/* d g / d(arg a); g odd in x and y, even in z. */
static LD dg_ld(int a, LD x, LD y, LD z)
{
    LD ax = fabsl(x), ay = fabsl(y), az = fabsl(z);
    switch (a) {
    case 0: return sgn(y) * dgdx_pos(ax, ay, az);
    case 1: return sgn(x) * dgdx_pos(ay, ax, az); /* g symmetric in (x, y) */
    default: return sgn(x) * sgn(y) * sgn(z) * dgdz_pos(ax, ay, az);
    }
}

/* Phi_kl(x, y, z) for the six components (the "permutation of variables"
 * rule of Sec. 2: stencil offsets stay on their physical axis, only the
 * argument order of f or g changes). */
static LD phi_ld(int comp, LD x, LD y, LD z)
{
    switch (comp) {
    case 0: return f_ld(x, y, z); /* xx */
    case 1: return f_ld(y, x, z); /* yy */
    case 2: return f_ld(z, x, y); /* zz */
    case 3: return g_ld(x, y, z); /* xy */
    case 4: return g_ld(x, z, y); /* xz */
    default: return g_ld(y, z, x); /* yz */
    }
}
/* d Phi_kl / dz (derivative with respect to the physical z offset). */
static LD dphi_dz_ld(int comp, LD x, LD y, LD z)
{
    switch (comp) {
    case 0: return df_ld(2, x, y, z);
    case 1: return df_ld(2, y, x, z);
    case 2: return df_ld(0, z, x, y);
    case 3: return dg_ld(2, x, y, z);
    case 4: return dg_ld(1, x, z, y);
    default: return dg_ld(1, y, z, x);
    }
}

double hfdo_f(double x, double y, double z) { return (double)f_ld(x, y, z); }
double hfdo_g(double x, double y, double z) { return (double)g_ld(x, y, z); }
double hfdo_df(int a, double x, double y, double z) { return (double)df_ld(a, x, y, z); }
double hfdo_dg(int a, double x, double y, double z) { return (double)dg_ld(a, x, y, z); }
double hfdo_phi(int comp, double x, double y, double z) { return (double)phi_ld(comp, x, y, z); }

/* ------------------------------------------------------------------------ */
/* Tensor of one cuboid pair (Sec. 2.1 / 2.2 with appendices A and B).       */
/* The four-point difference  S(d, d') = {+d: +1, 0: -1, d-d': -1, -d': +1}  */
/* is the grouping of the appendices (F1 over y, F over z, N over x); the     */
/* x-offsets of N_xx and of N_xy follow the same pattern once the printed     */
/* last term of N_xy is read as G(X - dx', Y + dy, Z).                        */
/*   N_kl = -1/(4 pi dx dy dz) sum_{a,b,c} s_a s_b s_c Phi_kl(X+a, Y+b, Z+c)  */
/* ------------------------------------------------------------------------ */
static void stencil4(LD d, LD ds, LD off[4], LD w[4])
{
    off[0] = d;       w[0] = 1.0L;
    off[1] = 0.0L;    w[1] = -1.0L;
    off[2] = d - ds;  w[2] = -1.0L;
    off[3] = -ds;     w[3] = 1.0L;
}

void hfdo_tensor_cuboids(double X, double Y, double Z, double dx, double dy, double dz,
                         double dxs, double dys, double dzs, double *out)
{
    LD ox[4], wx[4], oy[4], wy[4], oz[4], wz[4];
    stencil4(dx, dxs, ox, wx);
    stencil4(dy, dys, oy, wy);
    stencil4(dz, dzs, oz, wz);
    LD pref = -1.0L / (4.0L * PI_L * (LD)dx * (LD)dy * (LD)dz);
    for (int comp = 0; comp < 6; ++comp) {
        LD acc = 0.0L;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                for (int c = 0; c < 4; ++c)
                    acc += wx[a] * wy[b] * wz[c] *
                           phi_ld(comp, (LD)X + ox[a], (LD)Y + oy[b], (LD)Z + oz[c]);
        out[comp] = (double)(pref * acc);
    }
}

/* Same pair, derivative with respect to the z offset Z of the target. */
void hfdo_dtensor_dZ_cuboids(double X, double Y, double Z, double dx, double dy, double dz,
                             double dxs, double dys, double dzs, double *out)
{
    LD ox[4], wx[4], oy[4], wy[4], oz[4], wz[4];
    stencil4(dx, dxs, ox, wx);
    stencil4(dy, dys, oy, wy);
    stencil4(dz, dzs, oz, wz);
    LD pref = -1.0L / (4.0L * PI_L * (LD)dx * (LD)dy * (LD)dz);
    for (int comp = 0; comp < 6; ++comp) {
        LD acc = 0.0L;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                for (int c = 0; c < 4; ++c)
                    acc += wx[a] * wy[b] * wz[c] *
                           dphi_dz_ld(comp, (LD)X + ox[a], (LD)Y + oy[b], (LD)Z + oz[c]);
        out[comp] = (double)(pref * acc);
    }
}

/* ------------------------------------------------------------------------ */
/* Far field: N_kl = -1/(4 pi |tau|) int_tau int_tau' (3 r_k r_l - r^2 d_kl)  */
/* / r^5, r = x - x', for a target cuboid tau = [X, X+dx] x [Y, Y+dy] x       */
/* [Z, Z+dz] and a source cuboid tau' = [0, dxs] x [0, dys] x [0, dzs]:      */
/* FAR_N Gauss-Legendre points per axis on each of the six axes.             */
/* ------------------------------------------------------------------------ */
#define FAR_RHO 50.0L
#define FAR_N 3

/* nodes and weights of the n-point rule on [-1, 1]: Newton iteration on the
 * Legendre polynomial P_n from the Chebyshev estimate */
static void gauss_legendre(int n, LD *x, LD *w)
{
    for (int i = 0; i < n; ++i) {
        LD z = cosl(PI_L * (i + 0.75L) / (n + 0.5L)), dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            LD p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                LD p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0L; }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            LD dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

static void quad_far(LD X, LD Y, LD Z, LD dx, LD dy, LD dz, LD dxs, LD dys, LD dzs, LD out[6])
{
    LD gx[FAR_N], gw[FAR_N];
    gauss_legendre(FAR_N, gx, gw);
    LD acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < FAR_N; ++a)
    for (int b = 0; b < FAR_N; ++b)
    for (int c = 0; c < FAR_N; ++c) {
        const LD xt = X + 0.5L * dx * (1 + gx[a]), yt = Y + 0.5L * dy * (1 + gx[b]),
                 zt = Z + 0.5L * dz * (1 + gx[c]);
        const LD wt = gw[a] * gw[b] * gw[c];
        for (int d = 0; d < FAR_N; ++d)
        for (int e = 0; e < FAR_N; ++e)
        for (int f = 0; f < FAR_N; ++f) {
            const LD rx = xt - 0.5L * dxs * (1 + gx[d]), ry = yt - 0.5L * dys * (1 + gx[e]),
                     rz = zt - 0.5L * dzs * (1 + gx[f]);
            const LD r2 = rx * rx + ry * ry + rz * rz;
            const LD ir5 = 1.0L / (r2 * r2 * sqrtl(r2));
            const LD w = wt * gw[d] * gw[e] * gw[f] * ir5;
            acc[0] += w * (3 * rx * rx - r2);
            acc[1] += w * (3 * ry * ry - r2);
            acc[2] += w * (3 * rz * rz - r2);
            acc[3] += w * 3 * rx * ry;
            acc[4] += w * 3 * rx * rz;
            acc[5] += w * 3 * ry * rz;
        }
    }
    /* the rule integrates over [-1, 1]^6: Jacobian (dx dy dz dxs dys dzs) / 64 */
    const LD jac = dx * dy * dz * dxs * dys * dzs / 64.0L;
    for (int k = 0; k < 6; ++k) out[k] = -acc[k] * jac / (4.0L * PI_L * dx * dy * dz);
}

void hfdo_tensor_far(double X, double Y, double Z, double dx, double dy, double dz, double dxs,
                     double dys, double dzs, double *out)
{
    LD o[6];
    quad_far(X, Y, Z, dx, dy, dz, dxs, dys, dzs, o);
    for (int k = 0; k < 6; ++k) out[k] = (double)o[k];
}

/* Replace the entries of a pair table (layout below) whose centres are at
 * least FAR_RHO cell sizes apart by the quadrature values. */
static void far_entries(int nx, int ny, LD dx, LD dy, LD tb, LD tt, LD sb, LD st, double *table)
{
    const int Wo = 2 * nx - 1, Ho = 2 * ny - 1;
    const LD dz = tt - tb, dzs = st - sb;
    LD big = dx > dy ? dx : dy;
    if (dz > big) big = dz;
    if (dzs > big) big = dzs;
    const LD Z = tb - sb, zc = Z + 0.5L * dz - 0.5L * dzs;
#pragma omp parallel for schedule(dynamic, 8)
    for (int qi = 0; qi < Ho; ++qi) {
        const LD Y = (LD)(qi - (ny - 1)) * dy;
        for (int pi = 0; pi < Wo; ++pi) {
            const LD X = (LD)(pi - (nx - 1)) * dx;
            if (sqrtl(X * X + Y * Y + zc * zc) < FAR_RHO * big) continue;
            LD o[6];
            quad_far(X, Y, Z, dx, dy, dz, dx, dy, dzs, o);
            for (int k = 0; k < 6; ++k) table[(size_t)k * Wo * Ho + (size_t)qi * Wo + pi] = (double)o[k];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Layer-pair tables on the lateral lattice (Sec. 3, equal dx, dy for every  */
/* cell; each layer has its own thickness).  Translation invariance gives    */
/* N^{ij}(p, q) for lateral offsets p in [-(nx-1), nx-1], q in [-(ny-1),     */
/* ny-1] (target index minus source index).  The sum is taken in the order   */
/* of the appendices: Phi on the lattice, then the y group (F1), then the z  */
/* group (F), then the x group (N).                                          */
/* Output layout: table[comp][q + ny - 1][p + nx - 1], FP64.                 */
/* ------------------------------------------------------------------------ */

/* z offsets of the four z-stencil points for target [tb, tt], source [sb, st]:
 * Z + {dz, 0, dz - dz', -dz'} with Z = tb - sb. */
static void zpoints(LD tb, LD tt, LD sb, LD st, LD zc[4], LD wc[4])
{
    zc[0] = tt - sb; wc[0] = 1.0L;
    zc[1] = tb - sb; wc[1] = -1.0L;
    zc[2] = tt - st; wc[2] = -1.0L;
    zc[3] = tb - st; wc[3] = 1.0L;
}

/* Lateral grouping of one lattice of values lat[(2ny+1)][(2nx+1)] (lattice
 * point (P, Q) at [Q + ny][P + nx]) into acc[(2ny-1)][(2nx-1)] += w * (y then x
 * differences).  Stencils for equal lateral sizes: offsets {+1, 0, 0, -1} with
 * weights {+1, -1, -1, +1} (the four-point rule with d = d'). */
static void lateral_group(int nx, int ny, const LD *lat, LD *tmp, LD *acc, LD w)
{
    const int W = 2 * nx + 1, Wo = 2 * nx - 1, Ho = 2 * ny - 1;
    static const int off[4] = {1, 0, 0, -1};
    static const LD wt[4] = {1.0L, -1.0L, -1.0L, 1.0L};
    /* y group: tmp[q][P] for q in [-(ny-1), ny-1], P in [-nx, nx] */
#pragma omp parallel for schedule(static)
    for (int qi = 0; qi < Ho; ++qi) {
        int q = qi - (ny - 1);
        for (int P = 0; P < W; ++P) {
            LD s = 0.0L;
            for (int b = 0; b < 4; ++b) s += wt[b] * lat[(q + off[b] + ny) * W + P];
            tmp[qi * W + P] = s;
        }
    }
    /* x group */
#pragma omp parallel for schedule(static)
    for (int qi = 0; qi < Ho; ++qi) {
        for (int pi = 0; pi < Wo; ++pi) {
            int p = pi - (nx - 1);
            LD s = 0.0L;
            for (int a = 0; a < 4; ++a) s += wt[a] * tmp[qi * W + (p + off[a] + nx)];
            acc[qi * Wo + pi] += w * s;
        }
    }
}

static void fill_lattice(int nx, int ny, LD dx, LD dy, LD zc, int comp, int deriv, LD *lat)
{
    const int W = 2 * nx + 1, H = 2 * ny + 1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int Qi = 0; Qi < H; ++Qi) {
        LD Y = (LD)(Qi - ny) * dy;
        for (int Pi = 0; Pi < W; ++Pi) {
            LD X = (LD)(Pi - nx) * dx;
            lat[Qi * W + Pi] = deriv ? dphi_dz_ld(comp, X, Y, zc) : phi_ld(comp, X, Y, zc);
        }
    }
}

/* Table of N^{ij} for target layer [tb, tt] and source layer [sb, st]. */
int hfdo_pair_table(int nx, int ny, double dx, double dy, double tb, double tt, double sb,
                    double st, double *table)
{
    if (nx < 1 || ny < 1 || !(dx > 0) || !(dy > 0) || !(tt > tb) || !(st > sb)) return -1;
    const int W = 2 * nx + 1, H = 2 * ny + 1, Wo = 2 * nx - 1, Ho = 2 * ny - 1;
    LD *lat = (LD *)malloc(sizeof(LD) * (size_t)W * H);
    LD *tmp = (LD *)malloc(sizeof(LD) * (size_t)W * Ho);
    LD *acc = (LD *)malloc(sizeof(LD) * (size_t)Wo * Ho);
    if (!lat || !tmp || !acc) { free(lat); free(tmp); free(acc); return -2; }
    LD zc[4], wc[4];
    zpoints(tb, tt, sb, st, zc, wc);
    LD pref = -1.0L / (4.0L * PI_L * (LD)dx * (LD)dy * ((LD)tt - (LD)tb));
    for (int comp = 0; comp < 6; ++comp) {
        memset(acc, 0, sizeof(LD) * (size_t)Wo * Ho);
        for (int c = 0; c < 4; ++c) {
            fill_lattice(nx, ny, dx, dy, zc[c], comp, 0, lat);
            lateral_group(nx, ny, lat, tmp, acc, wc[c]);
        }
        double *o = table + (size_t)comp * Wo * Ho;
        for (size_t k = 0; k < (size_t)Wo * Ho; ++k) o[k] = (double)(pref * acc[k]);
    }
    free(lat); free(tmp); free(acc);
    far_entries(nx, ny, dx, dy, tb, tt, sb, st, table);
    return 0;
}

/* Derivative tables of N^{ij} with respect to the four interface positions
 * (target top, target bottom, source top, source bottom).
 * Writing N = pref * sum_c s_c Psi(zeta_c) with pref = -1/(4 pi dx dy t) and
 * t = top_t - bot_t, zeta = {top_t - bot_s, bot_t - bot_s, top_t - top_s,
 * bot_t - top_s}:
 *   dN/dtop_t = -N/t + pref [Psi'(z0) - Psi'(z2)]
 *   dN/dbot_t = +N/t + pref [Psi'(z3) - Psi'(z1)]
 *   dN/dtop_s = pref [Psi'(z2) - Psi'(z3)]
 *   dN/dbot_s = pref [Psi'(z1) - Psi'(z0)]
 * Output: dtab[4][6][2ny-1][2nx-1]. */
int hfdo_pair_dtable(int nx, int ny, double dx, double dy, double tb, double tt, double sb,
                     double st, double *dtab)
{
    if (nx < 1 || ny < 1 || !(dx > 0) || !(dy > 0) || !(tt > tb) || !(st > sb)) return -1;
    const int W = 2 * nx + 1, H = 2 * ny + 1, Wo = 2 * nx - 1, Ho = 2 * ny - 1;
    const size_t n2 = (size_t)Wo * Ho;
    LD *lat = (LD *)malloc(sizeof(LD) * (size_t)W * H);
    LD *tmp = (LD *)malloc(sizeof(LD) * (size_t)W * Ho);
    LD *psi = (LD *)malloc(sizeof(LD) * n2 * 5); /* Psi'(z0..z3) and N/pref */
    if (!lat || !tmp || !psi) { free(lat); free(tmp); free(psi); return -2; }
    LD zc[4], wc[4];
    zpoints(tb, tt, sb, st, zc, wc);
    LD t = (LD)tt - (LD)tb;
    LD pref = -1.0L / (4.0L * PI_L * (LD)dx * (LD)dy * t);
    for (int comp = 0; comp < 6; ++comp) {
        memset(psi, 0, sizeof(LD) * n2 * 5);
        for (int c = 0; c < 4; ++c) {
            fill_lattice(nx, ny, dx, dy, zc[c], comp, 1, lat);
            lateral_group(nx, ny, lat, tmp, psi + (size_t)c * n2, 1.0L);
            fill_lattice(nx, ny, dx, dy, zc[c], comp, 0, lat);
            lateral_group(nx, ny, lat, tmp, psi + 4 * n2, wc[c]);
        }
        for (size_t k = 0; k < n2; ++k) {
            LD N = pref * psi[4 * n2 + k];
            LD p0 = psi[k], p1 = psi[n2 + k], p2 = psi[2 * n2 + k], p3 = psi[3 * n2 + k];
            dtab[(0 * 6 + comp) * n2 + k] = (double)(-N / t + pref * (p0 - p2));
            dtab[(1 * 6 + comp) * n2 + k] = (double)(N / t + pref * (p3 - p1));
            dtab[(2 * 6 + comp) * n2 + k] = (double)(pref * (p2 - p3));
            dtab[(3 * 6 + comp) * n2 + k] = (double)(pref * (p1 - p0));
        }
    }
    free(lat); free(tmp); free(psi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Brute-force field (Sec. 3, discrete field over all cell pairs):           */
/*   h_i(p) = - sum_j sum_q N^{ij}(p - q) m_j(q)      (M_s = 1)               */
/* and its transpose (the adjoint with respect to m):                         */
/*   g_j(q) = - sum_i sum_p N^{ij}(p - q) g_i(p)                             */
/* m, g: [3][nz][ny][nx] FP64.  samp: nsamp triples (layer, iy, ix); with    */
/* nsamp <= 0 every cell is evaluated and out has layout [3][nz][ny][nx],    */
/* otherwise out is [nsamp][3].                                              */
/* ------------------------------------------------------------------------ */
static double sym(const double *t6, int r, int c)
{
    static const int idx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    return t6[idx[r][c]];
}

int hfdo_field(int nx, int ny, int nz, double dx, double dy, const double *zbot,
               const double *thick, const double *m, int nsamp, const int *samp, double *out,
               int transpose)
{
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    const int Wo = 2 * nx - 1, Ho = 2 * ny - 1;
    const size_t n2 = (size_t)Wo * Ho, cells = (size_t)nx * ny, lay = cells;
    const size_t comp_stride = (size_t)nz * cells;
    int all = (nsamp <= 0 || samp == NULL);
    int ns = all ? nz * nx * ny : nsamp;
    int *sl = (int *)malloc(sizeof(int) * 3 * (size_t)ns);
    double *acc = (double *)calloc((size_t)ns * 3, sizeof(double));
    double *tab = (double *)malloc(sizeof(double) * 6 * n2);
    if (!sl || !acc || !tab) { free(sl); free(acc); free(tab); return -2; }
    if (all) {
        int k = 0;
        for (int l = 0; l < nz; ++l)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) { sl[3 * k] = l; sl[3 * k + 1] = y; sl[3 * k + 2] = x; ++k; }
    } else {
        memcpy(sl, samp, sizeof(int) * 3 * (size_t)ns);
    }
    for (int a = 0; a < nz; ++a) {       /* layer of the evaluated cells   */
        int has = 0;
        for (int k = 0; k < ns; ++k) if (sl[3 * k] == a) { has = 1; break; }
        if (!has) continue;
        for (int b = 0; b < nz; ++b) {   /* layer of the summed cells      */
            /* forward: target a, source b: N^{ab}(p - q); transpose: target b, source a: N^{ba}(q - p) */
            int ti = transpose ? b : a, si = transpose ? a : b;
            int rc = hfdo_pair_table(nx, ny, dx, dy, zbot[ti], zbot[ti] + thick[ti], zbot[si],
                                     zbot[si] + thick[si], tab);
            if (rc) { free(sl); free(acc); free(tab); return rc; }
#pragma omp parallel for schedule(dynamic, 1)
            for (int k = 0; k < ns; ++k) {
                if (sl[3 * k] != a) continue;
                int py = sl[3 * k + 1], px = sl[3 * k + 2];
                double s0 = 0, s1 = 0, s2 = 0;
                for (int qy = 0; qy < ny; ++qy) {
                    for (int qx = 0; qx < nx; ++qx) {
                        int dpx = transpose ? qx - px : px - qx;
                        int dpy = transpose ? qy - py : py - qy;
                        size_t o = (size_t)(dpy + ny - 1) * Wo + (size_t)(dpx + nx - 1);
                        double t6[6];
                        for (int c = 0; c < 6; ++c) t6[c] = tab[c * n2 + o];
                        size_t cell = (size_t)b * lay + (size_t)qy * nx + qx;
                        double v0 = m[cell], v1 = m[comp_stride + cell], v2 = m[2 * comp_stride + cell];
                        s0 += sym(t6, 0, 0) * v0 + sym(t6, 0, 1) * v1 + sym(t6, 0, 2) * v2;
                        s1 += sym(t6, 1, 0) * v0 + sym(t6, 1, 1) * v1 + sym(t6, 1, 2) * v2;
                        s2 += sym(t6, 2, 0) * v0 + sym(t6, 2, 1) * v1 + sym(t6, 2, 2) * v2;
                    }
                }
                acc[3 * k] -= s0; acc[3 * k + 1] -= s1; acc[3 * k + 2] -= s2;
            }
        }
    }
    if (all) {
        for (int k = 0; k < ns; ++k) {
            size_t cell = (size_t)sl[3 * k] * lay + (size_t)sl[3 * k + 1] * nx + sl[3 * k + 2];
            out[cell] = acc[3 * k];
            out[comp_stride + cell] = acc[3 * k + 1];
            out[2 * comp_stride + cell] = acc[3 * k + 2];
        }
    } else {
        memcpy(out, acc, sizeof(double) * 3 * (size_t)ns);
    }
    free(sl); free(acc); free(tab);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Thickness gradient of  L = <g, h(m)>  (h as above).                        */
/*   dL/dt_k = - sum_{i,j} sum_{p,q} g_i(p) . dN^{ij}(p - q)/dt_k m_j(q)      */
/* The layers are stacked with fixed gaps: raising t_k moves every layer      */
/* above k up by the same amount, so d bot_l/dt_k = [k < l] and               */
/* d top_l/dt_k = [k <= l].                                                   */
/* mode 0: g is a full field [3][nz][ny][nx] and the pair sums are taken     */
/*         cell by cell (O((nx ny)^2) per pair);                             */
/* mode 1: g is uniform within each layer, given as gvec[nz][3]; the sum over */
/*         p of the derivative table is then a box sum over offsets.          */
/* Outputs: gt[nz], and if giface != NULL the interface gradients             */
/*          giface[2*l] = dL/dbot_l, giface[2*l+1] = dL/dtop_l.               */
/* ------------------------------------------------------------------------ */
int hfdo_thickness_grad(int nx, int ny, int nz, double dx, double dy, const double *zbot,
                        const double *thick, const double *m, const double *g, int mode,
                        double *gt, double *giface)
{
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    const int Wo = 2 * nx - 1, Ho = 2 * ny - 1;
    const size_t n2 = (size_t)Wo * Ho, cells = (size_t)nx * ny;
    const size_t cs = (size_t)nz * cells;
    double *dt = (double *)malloc(sizeof(double) * 24 * n2);
    double *gb = (double *)calloc((size_t)nz, sizeof(double));
    double *gtp = (double *)calloc((size_t)nz, sizeof(double));
    double *box = (mode == 1) ? (double *)malloc(sizeof(double) * (size_t)(Wo + 1) * (Ho + 1)) : NULL;
    if (!dt || !gb || !gtp || (mode == 1 && !box)) { free(dt); free(gb); free(gtp); free(box); return -2; }
    for (int i = 0; i < nz; ++i) {
        /* a target layer whose upstream gradient is zero contributes nothing */
        int gzero = 1;
        if (mode == 1) {
            for (int r = 0; r < 3; ++r) if (g[3 * (size_t)i + r] != 0.0) gzero = 0;
        } else {
            for (int r = 0; r < 3 && gzero; ++r)
                for (size_t c = 0; c < cells; ++c)
                    if (g[(size_t)r * cs + (size_t)i * cells + c] != 0.0) { gzero = 0; break; }
        }
        if (gzero) continue;
        for (int j = 0; j < nz; ++j) {
            int rc = hfdo_pair_dtable(nx, ny, dx, dy, zbot[i], zbot[i] + thick[i], zbot[j],
                                      zbot[j] + thick[j], dt);
            if (rc) { free(dt); free(gb); free(gtp); free(box); return rc; }
            double E[4] = {0, 0, 0, 0}; /* top_i, bot_i, top_j, bot_j */
            for (int w = 0; w < 4; ++w) {
                const double *D = dt + (size_t)w * 6 * n2;
                double s = 0.0;
                if (mode == 0) {
#pragma omp parallel for reduction(+ : s) schedule(dynamic, 1)
                    for (int py = 0; py < ny; ++py)
                        for (int px = 0; px < nx; ++px) {
                            size_t tc = (size_t)i * cells + (size_t)py * nx + px;
                            double g0 = g[tc], g1 = g[cs + tc], g2 = g[2 * cs + tc];
                            for (int qy = 0; qy < ny; ++qy)
                                for (int qx = 0; qx < nx; ++qx) {
                                    size_t o = (size_t)(py - qy + ny - 1) * Wo + (size_t)(px - qx + nx - 1);
                                    double t6[6];
                                    for (int c = 0; c < 6; ++c) t6[c] = D[c * n2 + o];
                                    size_t sc = (size_t)j * cells + (size_t)qy * nx + qx;
                                    double v0 = m[sc], v1 = m[cs + sc], v2 = m[2 * cs + sc];
                                    s += g0 * (sym(t6, 0, 0) * v0 + sym(t6, 0, 1) * v1 + sym(t6, 0, 2) * v2)
                                       + g1 * (sym(t6, 1, 0) * v0 + sym(t6, 1, 1) * v1 + sym(t6, 1, 2) * v2)
                                       + g2 * (sym(t6, 2, 0) * v0 + sym(t6, 2, 1) * v1 + sym(t6, 2, 2) * v2);
                                }
                        }
                } else {
                    const double *gv = g + 3 * (size_t)i;
                    for (int r = 0; r < 3; ++r) {
                        if (gv[r] == 0.0) continue;
                        for (int cc = 0; cc < 3; ++cc) {
                            static const int idx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
                            const double *Dc = D + (size_t)idx[r][cc] * n2;
                            /* 2D prefix sums over the offset table */
                            for (int a = 0; a <= Ho; ++a) box[(size_t)a * (Wo + 1)] = 0.0;
                            for (int b = 0; b <= Wo; ++b) box[b] = 0.0;
                            for (int a = 0; a < Ho; ++a)
                                for (int b = 0; b < Wo; ++b)
                                    box[(size_t)(a + 1) * (Wo + 1) + b + 1] =
                                        Dc[(size_t)a * Wo + b] + box[(size_t)a * (Wo + 1) + b + 1] +
                                        box[(size_t)(a + 1) * (Wo + 1) + b] - box[(size_t)a * (Wo + 1) + b];
                            double sub = 0.0;
                            for (int qy = 0; qy < ny; ++qy)
                                for (int qx = 0; qx < nx; ++qx) {
                                    /* offsets d = p - q, p over the grid: rows qy..., index d + n - 1 */
                                    int a0 = -qy + ny - 1, a1 = ny - 1 - qy + ny - 1; /* inclusive */
                                    int b0 = -qx + nx - 1, b1 = nx - 1 - qx + nx - 1;
                                    double bs = box[(size_t)(a1 + 1) * (Wo + 1) + b1 + 1] -
                                                box[(size_t)a0 * (Wo + 1) + b1 + 1] -
                                                box[(size_t)(a1 + 1) * (Wo + 1) + b0] +
                                                box[(size_t)a0 * (Wo + 1) + b0];
                                    size_t sc = (size_t)j * cells + (size_t)qy * nx + qx;
                                    sub += bs * m[(size_t)cc * cs + sc];
                                }
                            s += gv[r] * sub;
                        }
                    }
                }
                E[w] = -s;
            }
            gtp[i] += E[0]; gb[i] += E[1]; gtp[j] += E[2]; gb[j] += E[3];
        }
    }
    for (int k = 0; k < nz; ++k) {
        double s = 0.0;
        for (int l = 0; l < nz; ++l) {
            if (k < l) s += gb[l];
            if (k <= l) s += gtp[l];
        }
        gt[k] = s;
    }
    if (giface)
        for (int l = 0; l < nz; ++l) { giface[2 * l] = gb[l]; giface[2 * l + 1] = gtp[l]; }
    free(dt); free(gb); free(gtp); free(box);
    return 0;
}

int hfdo_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
