// Instances of the fused y-pass (y-DFT, z-mixing, inverse y-DFT in LDS):
// the generic kernel (layer count up to NZMAX at run time); single-precision
// 256- and 512-point columns of up to 10 layers and 1024-point columns of up
// to 4 go to the exact-layer-count kernels (fused_exact_*.hip).
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

namespace {
constexpr size_t kMaxFusedLds = 163840;  // 160 KB of LDS per CU on gfx950

// register budget: 1024-point columns run 16 waves per block (128 VGPRs),
// which holds the accumulators of at most 4 layers
template <typename R>
int nzmax_for(int nz, int LY)
{
    if (sizeof(R) == 8 || LY >= 1024) return nz <= 4 ? 4 : 0;
    return nz <= 4 ? 4 : (nz <= 8 ? 8 : (nz <= 12 ? 12 : 0));
}



hipError_t set_lds(const void* kernel, size_t lds)
{
    // the limit is raised once to the largest possible size
    return lds > 65536 ? ensure_lds_limit(kernel, (int)kMaxFusedLds) : hipSuccess;
}

template <typename R, int LY, int NZMAX, bool ADJ>
hipError_t fused_a(int nz, void* X, int ny, int M, int bpg, int G, const void* Q, long long qcs, const int* qslot,
                   int QY, const void* lp, const void* tw, hipStream_t s)
{
    const size_t lds = sizeof(cpx<R>) * 3 * (size_t)nz * fft_region(LY);
    hipError_t e = set_lds((const void*)k_ymix_fused<R, LY, NZMAX, ADJ>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ymix_fused<R, LY, NZMAX, ADJ>), dim3(M, bpg, G), dim3(FusedShape<LY>::NT),
                       lds, s, (cpx<R>*)X, ny, nz, M, (const R*)Q, qcs, qslot, QY, (const R*)lp, bpg,
                       (const cpx<R>*)tw);
    return hipGetLastError();
}

template <typename R, int LY, int NZMAX>
hipError_t fused_t(int nz, void* X, int ny, int M, int bpg, int G, const void* Q, long long qcs, const int* qslot,
                   int QY, const void* lp, int adjoint, const void* tw, hipStream_t s)
{
    if (adjoint) return fused_a<R, LY, NZMAX, true>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    return fused_a<R, LY, NZMAX, false>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
}

template <typename R, int LY>
hipError_t fused_nz(int nz, void* X, int ny, int M, int bpg, int G, const void* Q, long long qcs, const int* qslot,
                    int QY, const void* lp, int adjoint, const void* tw, hipStream_t s)
{
    switch (nzmax_for<R>(nz, LY)) {
    case 4: return fused_t<R, LY, 4>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    case 8:
        if constexpr (sizeof(R) == 4 && LY < 1024)
            return fused_t<R, LY, 8>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
        return hipErrorInvalidValue;
    case 12:
        if constexpr (sizeof(R) == 4 && LY < 1024)
            return fused_t<R, LY, 12>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t fused_ly(int LY, int nz, void* X, int ny, int M, int bpg, int G, const void* Q,
                    long long qcs, const int* qslot, int QY, const void* lp, int adjoint, const void* tw,
                    hipStream_t s)
{
    switch (LY) {
    case 8: return fused_nz<R, 8>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    case 16: return fused_nz<R, 16>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    case 32: return fused_nz<R, 32>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    case 64: return fused_nz<R, 64>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    case 128: return fused_nz<R, 128>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    case 256: return fused_nz<R, 256>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    case 512: return fused_nz<R, 512>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    case 1024: return fused_nz<R, 1024>(nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, tw, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool fused_supported(bool fp64, int LY, int nz, size_t* lds_bytes)
{
    const size_t lds = (fp64 ? 16 : 8) * 3 * (size_t)nz * fft_region(LY);
    if (lds_bytes) *lds_bytes = lds;
    if (LY < 8 || LY > 1024) return false;
    if ((fp64 ? nzmax_for<double>(nz, LY) : nzmax_for<float>(nz, LY)) == 0) return false;
    return lds <= kMaxFusedLds;
}

hipError_t launch_fused(bool fp64, int LY, int nz, void* X, int ny, int M, int B, const void* Q,
                        long long qcs, const int* qslot, int QX, int QY, const void* lp, int bpg,
                        int adjoint, const void* twy, hipStream_t s, bool generic)
{
    (void)QX;
    if (!fused_supported(fp64, LY, nz, nullptr)) return hipErrorInvalidValue;
    if (bpg < 1 || B % bpg != 0) return hipErrorInvalidValue;
    const int G = B / bpg;
    if (!generic && fused_exact_supported(fp64, LY, nz))
        return launch_fused_exact(LY, nz, adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, twy, s);
    if (fp64)
        return fused_ly<double>(LY, nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, twy, s);
    return fused_ly<float>(LY, nz, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, adjoint, twy, s);
}

}  // namespace hfd
