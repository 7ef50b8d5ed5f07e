// Instances of the y-pass column kernels and of the five-pass z-mixing kernel.
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

// half: the column holds at most LY/2 values (the field path; the tensor
// transforms run on full columns)
template <typename R, int LY>
static hipError_t yfwd_t(const void* in, void* out, int n, long long ncols, const void* tw,
                         hipStream_t s)
{
    using S = YPassShape<R, LY>;
    const long long nb = (ncols + S::NG - 1) / S::NG;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    if (2 * n <= LY)
        hipLaunchKernelGGL((k_yfwd<R, LY, true>), dim3((unsigned)nb), dim3(S::NT), 0, s,
                           (const cpx<R>*)in, (cpx<R>*)out, n, ncols, (const cpx<R>*)tw);
    else
        hipLaunchKernelGGL((k_yfwd<R, LY, false>), dim3((unsigned)nb), dim3(S::NT), 0, s,
                           (const cpx<R>*)in, (cpx<R>*)out, n, ncols, (const cpx<R>*)tw);
    return hipGetLastError();
}

template <typename R, int LY>
static hipError_t yinv_t(const void* in, void* out, int n, long long ncols, const void* tw,
                         hipStream_t s)
{
    using S = YPassShape<R, LY>;
    const long long nb = (ncols + S::NG - 1) / S::NG;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    if (2 * n <= LY)
        hipLaunchKernelGGL((k_yinv<R, LY, true>), dim3((unsigned)nb), dim3(S::NT), 0, s,
                           (const cpx<R>*)in, (cpx<R>*)out, n, ncols, (const cpx<R>*)tw);
    else
        hipLaunchKernelGGL((k_yinv<R, LY, false>), dim3((unsigned)nb), dim3(S::NT), 0, s,
                           (const cpx<R>*)in, (cpx<R>*)out, n, ncols, (const cpx<R>*)tw);
    return hipGetLastError();
}

#define HFD_Y_CASES(F, R, ...)                         \
    switch (LY) {                                      \
    case 8: return F<R, 8>(__VA_ARGS__);               \
    case 16: return F<R, 16>(__VA_ARGS__);             \
    case 32: return F<R, 32>(__VA_ARGS__);             \
    case 64: return F<R, 64>(__VA_ARGS__);             \
    case 128: return F<R, 128>(__VA_ARGS__);           \
    case 256: return F<R, 256>(__VA_ARGS__);           \
    case 512: return F<R, 512>(__VA_ARGS__);           \
    case 1024: return F<R, 1024>(__VA_ARGS__);         \
    case 2048: return F<R, 2048>(__VA_ARGS__);         \
    case 4096: return F<R, 4096>(__VA_ARGS__);         \
    default: return hipErrorInvalidValue;              \
    }

hipError_t launch_yfwd(bool fp64, int LY, const void* in, void* out, int n_in, long long ncols,
                       const void* twy, hipStream_t s)
{
    if (fp64) { HFD_Y_CASES(yfwd_t, double, in, out, n_in, ncols, twy, s) }
    HFD_Y_CASES(yfwd_t, float, in, out, n_in, ncols, twy, s)
}

hipError_t launch_yinv(bool fp64, int LY, const void* in, void* out, int n_out, long long ncols,
                       const void* twy, hipStream_t s)
{
    if (fp64) { HFD_Y_CASES(yinv_t, double, in, out, n_out, ncols, twy, s) }
    HFD_Y_CASES(yinv_t, float, in, out, n_out, ncols, twy, s)
}

template <int IB>
static hipError_t mix_pairs_t(bool fp64, const void* Mh, void* Hh, int nz, int M, int LY, int B,
                              const void* Q, long long qcs, const int* qslot, int QY, const void* lp,
                              int bpg, int adjoint, int kx0, int nkx, hipStream_t s)
{
    const int ngrp = (nz + IB - 1) / IB;
    const long long tiles = (long long)((LY / 2 + 31) / 32) * nkx * B;
    const long long nblk = (tiles + 7) / 8 * 8 * ngrp;
    if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblk);
    if (fp64)
        hipLaunchKernelGGL((k_mix_pairs<double, IB>), grid, dim3(64), 0, s,
                           (const cpx<double>*)Mh, (cpx<double>*)Hh, nz, M, LY, (const double*)Q, qcs,
                           qslot, QY, (const double*)lp, bpg, adjoint, kx0, nkx, B);
    else
        hipLaunchKernelGGL((k_mix_pairs<float, IB>), grid, dim3(64), 0, s,
                           (const cpx<float>*)Mh, (cpx<float>*)Hh, nz, M, LY, (const float*)Q, qcs,
                           qslot, QY, (const float*)lp, bpg, adjoint, kx0, nkx, B);
    return hipGetLastError();
}

// 4 target layers per lane up to 15 layers, 2 from 16 on (measured at 32 layers:
// 0.396 ms against 0.421 ms for 4 and 0.541 ms for 8; at 4 layers 4 is
// slightly ahead)
hipError_t launch_mix_generic(bool fp64, const void* Mh, void* Hh, int nz, int M, int LY, int B,
                              const void* Q, long long qcs, const int* qslot, int QX, int QY,
                              const void* lp, int bpg, int adjoint, int kx0, int nkx, hipStream_t s)
{
    (void)QX;
    if (nkx <= 0) return hipSuccess;
    if (nz >= 16)
        return mix_pairs_t<2>(fp64, Mh, Hh, nz, M, LY, B, Q, qcs, qslot, QY, lp, bpg, adjoint, kx0, nkx, s);
    return mix_pairs_t<4>(fp64, Mh, Hh, nz, M, LY, B, Q, qcs, qslot, QY, lp, bpg, adjoint, kx0, nkx, s);
}

}  // namespace hfd
