// Exact-layer-count fused y pass, 512-point columns, 8 to 10 layers.
#include "fused_exact.hpp"

namespace hfd {

hipError_t launch_fused_exact_3(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                   const void* Q, long long qcs, const int* qslot, int QY, const void* lp,
                                   const void* tw, hipStream_t s)
{
    switch (nz) {
    case 8: return fused_exact_t<512, 8>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    case 9: return fused_exact_t<512, 9>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    case 10: return fused_exact_t<512, 10>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hfd
