// Fused z kernels, serial form, float.
#include "zfused.hpp"

namespace dds {
DDS_Z_INSTANTIATE(float, false)
}  // namespace dds
