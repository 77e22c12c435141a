// Fused z kernels, grouped form, float.
#include "zfused.hpp"

namespace dds {
DDS_Z_INSTANTIATE(float, true)
}  // namespace dds
