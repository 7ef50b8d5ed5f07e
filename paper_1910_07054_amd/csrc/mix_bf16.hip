// Split-BF16 MFMA z-mixing (batched states).
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

long long split_tensor_bytes(int G, int nz, int QX, int QY)
{
    return (long long)G * nz * (nz + 1) / 2 * 5 * QX * QY * 3 * 2;
}

hipError_t launch_split_tensor(const float*, void*, int, int, int, int, const float*, int, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t launch_mix_bf16(const void*, void*, int, int, int, int, const void*, long long, int, int,
                           const void*, int, int, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace hfd
