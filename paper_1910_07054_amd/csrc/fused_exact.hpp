// Launch of the exact-layer-count fused y pass (k_ymix_fused_nz), included by
// the translation units that instantiate it for a range of layer counts (the
// instances are split over several files to compile in parallel).
#pragma once
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

template <int LY, int NZ, bool ADJ>
hipError_t fused_exact_a(void* X, int ny, int M, int bpg, int G, const void* Q, long long qcs, const int* qslot,
                         int QY, const void* lp, const void* tw, hipStream_t s)
{
    const size_t lds = sizeof(cpx<float>) * 3 * (size_t)NZ * fft_region(LY);
    constexpr bool own_col0 = LY <= ExactShape<LY>::NT;
    if (lds > 65536) {
        hipError_t e = ensure_lds_limit((const void*)k_ymix_fused_nz<float, LY, NZ, ADJ>, 163840);
        if (e != hipSuccess) return e;
        if constexpr (!own_col0) {
            e = ensure_lds_limit((const void*)k_ymix_fused<float, LY, 4, ADJ>, 163840);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL((k_ymix_fused_nz<float, LY, NZ, ADJ>), dim3(own_col0 ? M : M - 1, bpg, G),
                       dim3(ExactShape<LY>::NT), lds, s, (cpx<float>*)X, ny, M, (const float*)Q,
                       qcs, qslot, QY, (const float*)lp, bpg, (const cpx<float>*)tw);
    if constexpr (!own_col0) {
        // the packed column 0 (kx = 0 and Lx/2) by the generic kernel
        static_assert(NZ <= 4, "generic 1024-point column kernel holds up to 4 layers");
        hipLaunchKernelGGL((k_ymix_fused<float, LY, 4, ADJ>), dim3(1, bpg, G), dim3(FusedShape<LY>::NT),
                           lds, s, (cpx<float>*)X, ny, NZ, M, (const float*)Q, qcs, qslot, QY,
                           (const float*)lp, bpg, (const cpx<float>*)tw);
    }
    return hipGetLastError();
}

template <int LY, int NZ>
hipError_t fused_exact_t(int adjoint, void* X, int ny, int M, int bpg, int G, const void* Q,
                         long long qcs, const int* qslot, int QY, const void* lp, const void* tw, hipStream_t s)
{
    if (adjoint) return fused_exact_a<LY, NZ, true>(X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    return fused_exact_a<LY, NZ, false>(X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
}

}  // namespace hfd
