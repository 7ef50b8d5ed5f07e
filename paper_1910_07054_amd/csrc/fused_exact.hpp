// Launch of the exact-layer-count fused y pass (k_ymix_fused_nz), included by
// the translation units that instantiate it for a range of layer counts (the
// instances are split over several files to compile in parallel).
#pragma once
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

template <int NZ, bool ADJ>
hipError_t fused_exact_a(void* X, int ny, int M, int bpg, int G, const void* Q, long long qgs,
                         int QY, const void* lp, const void* tw, hipStream_t s)
{
    constexpr int LY = 512;
    const size_t lds = sizeof(cpx<float>) * 3 * (size_t)NZ * LY;
    if (lds > 65536) {
        hipError_t e = ensure_lds_limit((const void*)k_ymix_fused_nz<float, LY, NZ, ADJ>, 163840);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_ymix_fused_nz<float, LY, NZ, ADJ>), dim3(M, bpg, G),
                       dim3(FusedShape<LY>::NT), lds, s, (cpx<float>*)X, ny, M, (const float*)Q,
                       qgs, QY, (const float*)lp, bpg, (const cpx<float>*)tw);
    return hipGetLastError();
}

template <int NZ>
hipError_t fused_exact_t(int adjoint, void* X, int ny, int M, int bpg, int G, const void* Q,
                         long long qgs, int QY, const void* lp, const void* tw, hipStream_t s)
{
    if (adjoint) return fused_exact_a<NZ, true>(X, ny, M, bpg, G, Q, qgs, QY, lp, tw, s);
    return fused_exact_a<NZ, false>(X, ny, M, bpg, G, Q, qgs, QY, lp, tw, s);
}

}  // namespace hfd
