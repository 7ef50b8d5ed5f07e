// Instances of the x-pass kernels for every padded length 8..4096.
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

template <typename R, int LX>
static hipError_t xfwd_t(const void* in, void* out, int nx, int ny, long long iss, int irs, int nsig,
                         const void* tw, hipStream_t s)
{
    using S = XPassShape<R, LX>;
    static bool attr_done = false;
    if (S::LDS > 65536 && !attr_done) {
        attr_done = true;
        hipError_t e = hipFuncSetAttribute((const void*)k_xfwd<R, LX>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::LDS);
        if (e != hipSuccess) return e;
    }
    dim3 grid((ny + S::TY - 1) / S::TY, nsig);
    hipLaunchKernelGGL((k_xfwd<R, LX>), grid, dim3(S::NT), S::LDS, s, (const R*)in, (cpx<R>*)out,
                       nx, ny, iss, irs, (const cpx<R>*)tw);
    return hipGetLastError();
}

template <typename R, int LX>
static hipError_t xinv_t(const void* in, void* out, int nx, int ny, long long oss, int ors, int nsig,
                         const void* tw, hipStream_t s)
{
    using S = XPassShape<R, LX>;
    static bool attr_done = false;
    if (S::LDS > 65536 && !attr_done) {
        attr_done = true;
        hipError_t e = hipFuncSetAttribute((const void*)k_xinv<R, LX>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::LDS);
        if (e != hipSuccess) return e;
    }
    dim3 grid((ny + S::TY - 1) / S::TY, nsig);
    hipLaunchKernelGGL((k_xinv<R, LX>), grid, dim3(S::NT), S::LDS, s, (const cpx<R>*)in, (R*)out,
                       nx, ny, oss, ors, (const cpx<R>*)tw);
    return hipGetLastError();
}

#define HFD_X_CASES(F, R, ...)                         \
    switch (LX) {                                      \
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

hipError_t launch_xfwd(bool fp64, int LX, const void* in, void* out, int nx, int ny,
                       long long in_sig_stride, int in_row_stride, int nsig, const void* twx,
                       hipStream_t s)
{
    if (fp64) { HFD_X_CASES(xfwd_t, double, in, out, nx, ny, in_sig_stride, in_row_stride, nsig, twx, s) }
    HFD_X_CASES(xfwd_t, float, in, out, nx, ny, in_sig_stride, in_row_stride, nsig, twx, s)
}

hipError_t launch_xinv(bool fp64, int LX, const void* in, void* out, int nx, int ny,
                       long long out_sig_stride, int out_row_stride, int nsig, const void* twx,
                       hipStream_t s)
{
    if (fp64) { HFD_X_CASES(xinv_t, double, in, out, nx, ny, out_sig_stride, out_row_stride, nsig, twx, s) }
    HFD_X_CASES(xinv_t, float, in, out, nx, ny, out_sig_stride, out_row_stride, nsig, twx, s)
}

}  // namespace hfd
