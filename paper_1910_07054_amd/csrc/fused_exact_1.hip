// Exact-layer-count fused y pass, 512-point columns, 1 to 4 layers.
#include "fused_exact.hpp"

namespace hfd {

hipError_t launch_fused_exact_1(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                   const void* Q, long long qcs, const int* qslot, int QY, const void* lp,
                                   const void* tw, hipStream_t s)
{
    switch (nz) {
    case 1: return fused_exact_t<512, 1>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    case 2: return fused_exact_t<512, 2>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    case 3: return fused_exact_t<512, 3>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    case 4: return fused_exact_t<512, 4>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hfd
