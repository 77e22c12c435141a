// Fused z kernels, grouped form, double.
#include "zfused.hpp"

namespace dds {
DDS_Z_INSTANTIATE(double, true)
}  // namespace dds
