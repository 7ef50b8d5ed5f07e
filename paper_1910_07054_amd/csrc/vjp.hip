// Thickness gradient of L = <g, h(m)> (h = -N * m) for every state.
//
// With T^{ij} = -DFT2(N^{ij}) / (Lx Ly) the field is H_i = sum_j T^{ij} M_j and
//   L = sum_k sum_{ij} conj(G_i(k)) . T^{ij}(k) M_j(k)   (full Lx x Ly grid),
// G, M the 2D DFTs of the zero-padded g and m.  N^{ij} depends on the four
// interfaces bot_i, top_i (target) and bot_j, top_j (source) through
// N = -1/(4 pi dx dy t_i) sum_c s_c Psi(zeta_c), zeta = {top_i - bot_j,
// bot_i - bot_j, top_i - top_j, bot_i - top_j}, s = {+1, -1, -1, +1}, Psi the
// lateral-stencilled Phi.  With D(zeta) the normalized DFT of
// -1/(4 pi dx dy) dPsi/dz (zeta):
//   dT/dtop_i = -T/t_i + (D(z0) - D(z2))/t_i     dT/dbot_i = T/t_i + (D(z3) - D(z1))/t_i
//   dT/dtop_j = (D(z2) - D(z3))/t_i             dT/dbot_j = (D(z1) - D(z0))/t_i
// Each interface gradient is a sum over frequencies and ordered pairs of
// P[X] = Re sum_cc' X_cc' conj(G_i,c) M_j,c'.  The half spectrum holds
// kx in [1, M) once (weight 2, the mirror -kx is the complex conjugate) and
// the packed column 0 carries kx = 0 and kx = Lx/2 (weight 1 each).
// Stacks keep their gaps: d bot_l/dt_k = [k < l], d top_l/dt_k = [k <= l].
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

namespace {

// Re sum_cc' A_cc' X_cc' for a symmetric tensor block A given on the quadrant:
// real components (xx, yy, zz, xy), imaginary ones (xz, yz) given as q with
// A = i q.  X_cc' = conj(g_c) m_c'.
template <typename R>
struct Cross {
    // symmetric combinations of X: xx, yy, zz, (xy + yx), (xz + zx), (yz + zy)
    double re[6], im[6];
};

template <typename R>
__device__ inline Cross<R> cross_spectrum(const cpx<R> g[3], const cpx<R> m[3])
{
    Cross<R> X;
    auto cr = [&](int a, int b, double& re, double& im) {
        // conj(g_a) m_b
        re = (double)g[a].x * m[b].x + (double)g[a].y * m[b].y;
        im = (double)g[a].x * m[b].y - (double)g[a].y * m[b].x;
    };
    double r1, i1, r2, i2;
    cr(0, 0, X.re[0], X.im[0]);
    cr(1, 1, X.re[1], X.im[1]);
    cr(2, 2, X.re[2], X.im[2]);
    cr(0, 1, r1, i1); cr(1, 0, r2, i2); X.re[3] = r1 + r2; X.im[3] = i1 + i2;
    cr(0, 2, r1, i1); cr(2, 0, r2, i2); X.re[4] = r1 + r2; X.im[4] = i1 + i2;
    cr(1, 2, r1, i1); cr(2, 1, r2, i2); X.re[5] = r1 + r2; X.im[5] = i1 + i2;
    return X;
}

// contraction with real parts a[0..3] (xx, yy, zz, xy) and imaginary q[4..5]
template <typename R>
__device__ inline double contract(const Cross<R>& X, double xx, double yy, double zz, double xy,
                                  double xz, double yz)
{
    return xx * X.re[0] + yy * X.re[1] + zz * X.re[2] + xy * X.re[3] - xz * X.im[4] - yz * X.im[5];
}

template <typename T>
__device__ inline T block_sum(T v, T* red)
{
    // wave reduction then across waves (blockDim.x multiple of 64, <= 1024)
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    return s;  // valid in thread 0
}

}  // namespace

// One thread per (state b, spectrum point).  pass 0 accumulates the terms of the
// target layer's interfaces (outer index = target i), pass 1 those of the
// source layer's interfaces (outer index = source j).
// Output partial[b][blk][2 nz]: (d/dbot_l, d/dtop_l) per layer, per block.
template <typename R>
__global__ __launch_bounds__(256) void k_tgrad(const cpx<R>* __restrict__ Mh,
                                               const cpx<R>* __restrict__ Gh, int nz, int M, int LY,
                                               const R* __restrict__ Q, long long qgs,
                                               const R* __restrict__ D, long long dgs,
                                               const int* __restrict__ zidx, int g_first,
                                               const R* __restrict__ lp, int bpg, int QX, int QY,
                                               int b0, double* __restrict__ partial)
{
    __shared__ double red[16];
    const int b = b0 + blockIdx.y;
    const int geom = b / bpg;
    const long long npts = (long long)M * LY;
    const long long pt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = pt < npts;
    const int kx = active ? (int)(pt / LY) : 0, ky = active ? (int)(pt % LY) : 0;
    const int S = 3 * nz;
    const long long sst = (long long)M * LY;
    const cpx<R>* mb = Mh + ((long long)b * S * M + kx) * LY;
    const cpx<R>* gb = Gh + ((long long)b * S * M + kx) * LY;
    const R* Qg = Q + (long long)geom * qgs;
    const R* Dg = D + (long long)(geom - g_first) * dgs;
    const int* zg = zidx + (long long)geom * nz * nz * 4;
    const R* lpg = lp + (long long)geom * 2 * nz;
    const long long cs = (long long)QX * QY;
    const int half = LY / 2;
    const int kq = ky <= half ? ky : LY - ky;
    const double sgy = ky <= half ? 1.0 : -1.0;
    const int kyn = (LY - ky) & (LY - 1);
    const int npts_here = (kx == 0) ? 2 : 1;
    const double wgt = (kx == 0) ? 1.0 : 2.0;
    double* out = partial + ((long long)b * gridDim.x + blockIdx.x) * 2 * nz;

    // spectrum of signal (c, l) at this point; p selects A (kx = 0) or B (kx = Lx/2)
    auto spec = [&](const cpx<R>* base, int c, int l, int p) -> cpx<R> {
        const cpx<R> z1 = base[(c * nz + l) * sst + ky];
        if (kx != 0) return z1;
        const cpx<R> z2 = base[(c * nz + l) * sst + kyn];
        return p == 0 ? cpx<R>{R(0.5) * (z1.x + z2.x), R(0.5) * (z1.y - z2.y)}
                      : cpx<R>{R(0.5) * (z1.y + z2.y), R(0.5) * (z2.x - z1.x)};
    };

    for (int pass = 0; pass < 2; ++pass) {
        for (int o = 0; o < nz; ++o) {
            double acc_bot = 0.0, acc_top = 0.0;
            if (active) {
                for (int k = 0; k < nz; ++k) {
                    const int i = pass == 0 ? o : k, j = pass == 0 ? k : o;
                    const double ti = 1.0 / (double)lpg[i];
                    for (int p = 0; p < npts_here; ++p) {
                        const int row = (kx == 0) ? (p == 0 ? 0 : M) : kx;
                        cpx<R> g3[3], m3[3];
                        for (int c = 0; c < 3; ++c) {
                            g3[c] = spec(gb, c, i, p);
                            m3[c] = spec(mb, c, j, p);
                        }
                        const Cross<R> X = cross_spectrum<R>(g3, m3);
                        const int* zz4 = zg + (i * nz + j) * 4;
                        double PD[4];
                        for (int c = 0; c < 4; ++c) {
                            const int zi = zz4[c];
                            const R* d = Dg + (long long)zi * 6 * cs + (long long)row * QY + kq;
                            PD[c] = contract<R>(X, d[0], d[cs], d[2 * cs], sgy * (double)d[3 * cs],
                                                d[4 * cs], sgy * (double)d[5 * cs]);
                        }
                        double PT = 0.0;
                        if (pass == 0) {
                            const int a = i < j ? i : j, bq = i < j ? j : i;
                            const int u = a * nz - a * (a - 1) / 2 + (bq - a);
                            const R* q = Qg + ((long long)row * (nz * (nz + 1) / 2) + u) * 5 * QY + kq;
                            const double simag = i <= j ? 1.0 : -1.0;
                            const double xx = q[0], yy = q[QY], xy = sgy * (double)q[2 * QY];
                            const double xz = simag * (double)q[3 * QY];
                            const double yz = simag * sgy * (double)q[4 * QY];
                            const double zz = -(xx + yy) + (i == j ? (double)lpg[nz + i] : 0.0);
                            // stored blocks are t_i T^{ij}
                            PT = contract<R>(X, xx, yy, zz, xy, xz, yz) / ti;
                        }
                        if (pass == 0) {
                            acc_top += wgt * (-PT + PD[0] - PD[2]) / ti;
                            acc_bot += wgt * (PT + PD[3] - PD[1]) / ti;
                        } else {
                            acc_top += wgt * (PD[2] - PD[3]) / ti;
                            acc_bot += wgt * (PD[1] - PD[0]) / ti;
                        }
                    }
                }
            }
            const double sb = block_sum(acc_bot, red);
            if (threadIdx.x == 0) out[2 * o] = (pass == 0 ? 0.0 : out[2 * o]) + sb;
            const double st = block_sum(acc_top, red);
            if (threadIdx.x == 0) out[2 * o + 1] = (pass == 0 ? 0.0 : out[2 * o + 1]) + st;
        }
    }
}

// Sum the block partials (fixed order) and apply the stacking chain rule.
__global__ __launch_bounds__(64) void k_tgrad_finish(const double* __restrict__ partial, int nparts,
                                                     int nz, double* __restrict__ grad_t)
{
    const int b = blockIdx.x;
    extern __shared__ double gi[];  // [2 nz]
    for (int v = threadIdx.x; v < 2 * nz; v += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nparts; ++k) s += partial[((long long)b * nparts + k) * 2 * nz + v];
        gi[v] = s;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
        double s = 0.0;
        for (int l = 0; l < nz; ++l) {
            if (k < l) s += gi[2 * l];
            if (k <= l) s += gi[2 * l + 1];
        }
        grad_t[(long long)b * nz + k] = s;
    }
}

hipError_t launch_tgrad(bool fp64, const void* Mh, const void* Gh, int nz, int M, int LY, int b0,
                        int nb, const void* Q, long long qgs, const void* D, long long dgs,
                        const int* zidx, int g_first, const void* lp, int bpg, int QX, int QY,
                        double* partial, int nblk, hipStream_t s)
{
    dim3 grid(nblk, nb);
    if (fp64)
        hipLaunchKernelGGL(k_tgrad<double>, grid, dim3(256), 0, s, (const cpx<double>*)Mh,
                           (const cpx<double>*)Gh, nz, M, LY, (const double*)Q, qgs,
                           (const double*)D, dgs, zidx, g_first, (const double*)lp, bpg, QX, QY, b0,
                           partial);
    else
        hipLaunchKernelGGL(k_tgrad<float>, grid, dim3(256), 0, s, (const cpx<float>*)Mh,
                           (const cpx<float>*)Gh, nz, M, LY, (const float*)Q, qgs, (const float*)D,
                           dgs, zidx, g_first, (const float*)lp, bpg, QX, QY, b0, partial);
    return hipGetLastError();
}

hipError_t launch_tgrad_finish(const double* partial, int nparts, int B, int nz, double* grad_t,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_tgrad_finish, dim3(B), dim3(64), sizeof(double) * 2 * nz, s, partial,
                       nparts, nz, grad_t);
    return hipGetLastError();
}

}  // namespace hfd
