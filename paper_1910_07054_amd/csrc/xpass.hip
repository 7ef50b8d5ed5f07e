// Instances of the x-pass kernels for every padded length 8..4096, with the
// rows per block (TY) chosen at run time among the compiled tile sizes.  The
// field path (rows of nx <= LX/2 values) runs the HALF kernels, which skip
// the zero half in the first radix pass (forward) or the cropped half in the
// last (inverse); full rows (the tensor transforms) run the default tile
// without that pruning.
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

namespace {

// a tile size is compiled for a length when its block fits (<= 1024 threads,
// <= 160 KB of LDS) and it is not the default one
template <typename R, int LX, int TY>
constexpr bool x_tile_ok()
{
    using S = XPassShape<R, LX, TY>;
    return S::GT * TY <= 1024 && S::GT * TY >= 64 && S::LDS <= 163840;
}

template <typename R, int LX, int TY, bool HALF>
hipError_t xfwd_t(const void* in, void* out, int nx, int ny, long long iss, int irs, int nsig,
                  const void* tw, hipStream_t s)
{
    using S = XPassShape<R, LX, TY>;
    hipError_t e = ensure_lds_limit((const void*)k_xfwd<R, LX, TY, HALF>, (int)S::LDS);
    if (e != hipSuccess) return e;
    const long long rows = (long long)nsig * ny;
    if (rows > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)((rows + S::TY - 1) / S::TY));
    hipLaunchKernelGGL((k_xfwd<R, LX, TY, HALF>), grid, dim3(S::NT), S::LDS, s, (const R*)in,
                       (cpx<R>*)out, nx, ny, (int)rows, iss, irs, (const cpx<R>*)tw);
    return hipGetLastError();
}

template <typename R, int LX, int TY, bool HALF>
hipError_t xinv_t(const void* in, void* out, int nx, int ny, long long oss, int ors, int nsig,
                  const void* tw, hipStream_t s)
{
    using S = XPassShape<R, LX, TY>;
    hipError_t e = ensure_lds_limit((const void*)k_xinv<R, LX, TY, HALF>, (int)S::LDS);
    if (e != hipSuccess) return e;
    const long long rows = (long long)nsig * ny;
    if (rows > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)((rows + S::TY - 1) / S::TY));
    hipLaunchKernelGGL((k_xinv<R, LX, TY, HALF>), grid, dim3(S::NT), S::LDS, s, (const cpx<R>*)in,
                       (R*)out, nx, ny, (int)rows, oss, ors, (const cpx<R>*)tw);
    return hipGetLastError();
}

template <bool FWD, typename R, int LX, int TY>
hipError_t x_one(const void* in, void* out, int nx, int ny, long long ss, int rs, int nsig,
                 const void* tw, hipStream_t s)
{
    const bool half = 2 * nx <= LX;
    if constexpr (TY == 0 || x_tile_ok<R, LX, TY>()) {
        if (half) {
            if constexpr (FWD) return xfwd_t<R, LX, TY, true>(in, out, nx, ny, ss, rs, nsig, tw, s);
            else return xinv_t<R, LX, TY, true>(in, out, nx, ny, ss, rs, nsig, tw, s);
        }
        if constexpr (TY == 0) {
            if constexpr (FWD) return xfwd_t<R, LX, 0, false>(in, out, nx, ny, ss, rs, nsig, tw, s);
            else return xinv_t<R, LX, 0, false>(in, out, nx, ny, ss, rs, nsig, tw, s);
        }
    }
    return hipErrorInvalidValue;
}

template <bool FWD, typename R, int LX>
hipError_t x_ty(int ty, const void* in, void* out, int nx, int ny, long long ss, int rs, int nsig,
                const void* tw, hipStream_t s)
{
    switch (ty) {
    case 0: return x_one<FWD, R, LX, 0>(in, out, nx, ny, ss, rs, nsig, tw, s);
    case 4: return x_one<FWD, R, LX, 4>(in, out, nx, ny, ss, rs, nsig, tw, s);
    case 8: return x_one<FWD, R, LX, 8>(in, out, nx, ny, ss, rs, nsig, tw, s);
    case 12: return x_one<FWD, R, LX, 12>(in, out, nx, ny, ss, rs, nsig, tw, s);
    case 16: return x_one<FWD, R, LX, 16>(in, out, nx, ny, ss, rs, nsig, tw, s);
    case 24: return x_one<FWD, R, LX, 24>(in, out, nx, ny, ss, rs, nsig, tw, s);
    case 32: return x_one<FWD, R, LX, 32>(in, out, nx, ny, ss, rs, nsig, tw, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool FWD, typename R>
hipError_t x_lx(int LX, int ty, const void* in, void* out, int nx, int ny, long long ss, int rs,
                int nsig, const void* tw, hipStream_t s)
{
    switch (LX) {
    case 8: return x_ty<FWD, R, 8>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 16: return x_ty<FWD, R, 16>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 32: return x_ty<FWD, R, 32>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 64: return x_ty<FWD, R, 64>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 128: return x_ty<FWD, R, 128>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 256: return x_ty<FWD, R, 256>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 512: return x_ty<FWD, R, 512>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 1024: return x_ty<FWD, R, 1024>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 2048: return x_ty<FWD, R, 2048>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    case 4096: return x_ty<FWD, R, 4096>(ty, in, out, nx, ny, ss, rs, nsig, tw, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <int LX>
static hipError_t xtab_t(const double* in, void* out, int nx, int ny, long long nrows, const void* tw,
                         hipStream_t s)
{
    using S = XPassShape<double, LX, 0>;
    hipError_t e = ensure_lds_limit((const void*)k_xtab<LX, 0>, (int)S::LDS);
    if (e != hipSuccess) return e;
    if (nrows > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)((nrows + S::TY - 1) / S::TY));
    hipLaunchKernelGGL((k_xtab<LX, 0>), grid, dim3(S::NT), S::LDS, s, in, (double*)out, nx, ny,
                       (int)nrows, (const cpx<double>*)tw);
    return hipGetLastError();
}

hipError_t launch_xtab(int LX, const double* in, void* out, int nx, int ny, int nsig, const void* twx64,
                       hipStream_t s)
{
    if (nsig <= 0 || ny <= 0) return hipSuccess;
    if (nx < 1 || 2 * nx > LX + 1) return hipErrorInvalidValue;
    const long long rows = (long long)nsig * ny;
    switch (LX) {
    case 8: return xtab_t<8>(in, out, nx, ny, rows, twx64, s);
    case 16: return xtab_t<16>(in, out, nx, ny, rows, twx64, s);
    case 32: return xtab_t<32>(in, out, nx, ny, rows, twx64, s);
    case 64: return xtab_t<64>(in, out, nx, ny, rows, twx64, s);
    case 128: return xtab_t<128>(in, out, nx, ny, rows, twx64, s);
    case 256: return xtab_t<256>(in, out, nx, ny, rows, twx64, s);
    case 512: return xtab_t<512>(in, out, nx, ny, rows, twx64, s);
    case 1024: return xtab_t<1024>(in, out, nx, ny, rows, twx64, s);
    case 2048: return xtab_t<2048>(in, out, nx, ny, rows, twx64, s);
    case 4096: return xtab_t<4096>(in, out, nx, ny, rows, twx64, s);
    default: return hipErrorInvalidValue;
    }
}

bool x_tile_supported(bool fp64, int LX, int ty)
{
    if (ty == 0) return true;
    if (ty != 4 && ty != 8 && ty != 12 && ty != 16 && ty != 24 && ty != 32) return false;
    const int M = LX / 2;
    const int V = fft_vals(M), GT = M / V;
    const size_t lds = (fp64 ? 16 : 8) * (size_t)ty * (size_t)(fft_region(M) | 1);
    return GT * ty <= 1024 && GT * ty >= 64 && lds <= 163840;
}

hipError_t launch_xfwd(bool fp64, int LX, const void* in, void* out, int nx, int ny,
                       long long in_sig_stride, int in_row_stride, int nsig, const void* twx,
                       hipStream_t s, int ty)
{
    if (fp64) return x_lx<true, double>(LX, ty, in, out, nx, ny, in_sig_stride, in_row_stride, nsig, twx, s);
    return x_lx<true, float>(LX, ty, in, out, nx, ny, in_sig_stride, in_row_stride, nsig, twx, s);
}

hipError_t launch_xinv(bool fp64, int LX, const void* in, void* out, int nx, int ny,
                       long long out_sig_stride, int out_row_stride, int nsig, const void* twx,
                       hipStream_t s, int ty)
{
    if (fp64) return x_lx<false, double>(LX, ty, in, out, nx, ny, out_sig_stride, out_row_stride, nsig, twx, s);
    return x_lx<false, float>(LX, ty, in, out, nx, ny, out_sig_stride, out_row_stride, nsig, twx, s);
}

}  // namespace hfd
