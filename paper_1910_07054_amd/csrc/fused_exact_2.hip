// Exact-layer-count fused y pass, 512-point columns, 5 to 7 layers.
#include "fused_exact.hpp"

namespace hfd {

hipError_t launch_fused_exact_2(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                   const void* Q, long long qcs, const int* qslot, int QY, const void* lp,
                                   const void* tw, hipStream_t s)
{
    switch (nz) {
    case 5: return fused_exact_t<512, 5>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    case 6: return fused_exact_t<512, 6>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    case 7: return fused_exact_t<512, 7>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hfd
