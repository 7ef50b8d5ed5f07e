// Exact-layer-count fused y pass, 256-point columns, 1 to 10 layers.
#include "fused_exact.hpp"

namespace hfd {

hipError_t launch_fused_exact_5(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                const void* Q, long long qcs, const int* qslot, int QY, const void* lp,
                                const void* tw, hipStream_t s)
{
#define HFD_EXACT_256(N) \
    case N: return fused_exact_t<256, N>(adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s)
    switch (nz) {
    HFD_EXACT_256(1);
    HFD_EXACT_256(2);
    HFD_EXACT_256(3);
    HFD_EXACT_256(4);
    HFD_EXACT_256(5);
    HFD_EXACT_256(6);
    HFD_EXACT_256(7);
    HFD_EXACT_256(8);
    HFD_EXACT_256(9);
    HFD_EXACT_256(10);
    default: return hipErrorInvalidValue;
    }
#undef HFD_EXACT_256
}

}  // namespace hfd
