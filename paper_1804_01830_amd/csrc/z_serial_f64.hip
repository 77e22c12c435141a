// Fused z kernels, serial form, double.
#include "zfused.hpp"

namespace dds {
DDS_Z_INSTANTIATE(double, false)
}  // namespace dds
