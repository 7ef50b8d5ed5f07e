// Instances of the FP64 tensor-setup kernels.
#include "launch.hpp"
#include <algorithm>
#include <cmath>
#include "tensor_kernels.hpp"

namespace hfd {

static_assert(sizeof(PairGeo) == sizeof(PairGeoH), "pair record layout");

hipError_t launch_tensor_real(double* W, const PairGeoH* pg, int npairs, int nx, int ny, int Lx,
                              int Ly, double dx, double dy, double tmax, int mode, hipStream_t s)
{
    (void)Lx;
    (void)Ly;
    if (npairs <= 0 || nx <= 0 || ny <= 0) return hipSuccess;
    if (mode != 1 && mode != 2) return hipErrorInvalidValue;
    // boxes of every entry with rho < 6 and rho < 32: p dx and q dy stay below
    // rho max(dx, dy, t)
    const double dmax = std::max(std::max(dx, dy), tmax);
    const int pn = (int)std::min<double>(nx, std::floor(kNearRho * dmax / dx) + 2.0);
    const int qn = (int)std::min<double>(ny, std::floor(kNearRho * dmax / dy) + 2.0);
    const int pm = (int)std::min<double>(nx, std::floor(kMidRho * dmax / dx) + 2.0);
    const int qm = (int)std::min<double>(ny, std::floor(kMidRho * dmax / dy) + 2.0);
    const long long tiles = (long long)((nx + 15) / 16) * ((ny + 15) / 16);
    const int epb = 256 / kMidLanes;
    if (tiles * npairs > 0x7fffffffLL || npairs > 65535) return hipErrorInvalidValue;
    const dim3 ngrid((unsigned)((pn + kNTile - 1) / kNTile), (unsigned)((qn + kNTile - 1) / kNTile),
                     (unsigned)npairs);
    hipLaunchKernelGGL(k_tensor_near, ngrid, dim3(256), 0, s, W, (const PairGeo*)pg, nx, ny, dx, dy,
                       mode, pn, qn);
    const dim3 mgrid((unsigned)((pm * qm + epb - 1) / epb), (unsigned)npairs);
    hipLaunchKernelGGL(k_tensor_mid, mgrid, dim3(256), 0, s, W, (const PairGeo*)pg, nx, ny, dx, dy,
                       mode, pm, qm);
    hipLaunchKernelGGL(k_tensor_far, dim3((unsigned)(tiles * npairs)), dim3(256), 0, s, W,
                       (const PairGeo*)pg, npairs, nx, ny, dx, dy, mode);
    return hipGetLastError();
}

hipError_t launch_dtensor_real(double* W, const double* zeta, int nzeta, int nx, int ny, double dx,
                               double dy, hipStream_t s)
{
    if (nzeta <= 0) return hipSuccess;
    if (nzeta > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((nx + kDTile - 1) / kDTile), (unsigned)((ny + kDTile - 1) / kDTile),
                    (unsigned)nzeta);
    hipLaunchKernelGGL(k_dtensor_real, grid, dim3(kDTile * kDTile), 0, s, W, zeta, nx, ny, dx, dy);
    return hipGetLastError();
}

template <typename R, int LY>
static hipError_t ytab_t(const void* F, void* Q, const double* scale, int npairs, int comps, int M,
                         int ny, int QX, int QY, int pair0, int pair_total, int row_outer,
                         const int* src, const void* twy, hipStream_t s)
{
    using S = TabShape<LY>;
    const long long tasks = (long long)npairs * (M + 1) * 3;
    const long long nb = (tasks + S::NG - 1) / S::NG;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ytab<R, LY>), dim3((unsigned)nb), dim3(S::NT), 0, s, (const double*)F,
                       (R*)Q, scale, npairs, comps, M, ny, QX, QY, pair0, pair_total, row_outer, src,
                       (const cpx<double>*)twy);
    return hipGetLastError();
}

template <typename R>
static hipError_t ytab_r(int Ly, const void* F, void* Q, const double* scale, int npairs, int comps,
                         int M, int ny, int QX, int QY, int pair0, int pair_total, int row_outer,
                         const int* src, const void* twy, hipStream_t s)
{
    switch (Ly) {
#define HFD_YTAB(L) \
    case L: return ytab_t<R, L>(F, Q, scale, npairs, comps, M, ny, QX, QY, pair0, pair_total, row_outer, src, twy, s);
    HFD_YTAB(8) HFD_YTAB(16) HFD_YTAB(32) HFD_YTAB(64) HFD_YTAB(128) HFD_YTAB(256) HFD_YTAB(512)
    HFD_YTAB(1024) HFD_YTAB(2048) HFD_YTAB(4096)
#undef HFD_YTAB
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ytab(bool out_fp64, const void* F, void* Q, const double* scale, int npairs,
                       int comps, int M, int ny, int Ly, int QX, int QY, int pair0, int pair_total,
                       int row_outer, const void* twy64, hipStream_t s, const int* src)
{
    if (npairs <= 0) return hipSuccess;
    if ((comps != 5 && comps != 6) || M < 1 || ny < 1 || 2 * ny > Ly + 1) return hipErrorInvalidValue;
    return out_fp64 ? ytab_r<double>(Ly, F, Q, scale, npairs, comps, M, ny, QX, QY, pair0, pair_total,
                                     row_outer, src, twy64, s)
                    : ytab_r<float>(Ly, F, Q, scale, npairs, comps, M, ny, QX, QY, pair0, pair_total,
                                    row_outer, src, twy64, s);
}


// Zero n doubles with a kernel (used instead of a memset node on paths that a
// caller may capture in a graph).
__global__ __launch_bounds__(256) void k_zero64(double* __restrict__ p, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

hipError_t launch_zero64(double* p, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero64, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace hfd
