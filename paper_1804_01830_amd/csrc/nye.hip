// Density channels in the axis basis from per-cell line directions: for the
// three fixed line directions e_x, e_y, e_z, rho_{3l+gamma} = n t_l b_gamma
// (the Nye tensor), written or added (several dislocation families per cell
// in successive calls). Elementwise and HBM-bound: 7 values read, 9 written
// (9 more read when adding) per cell.
#include "ddstress_internal.hpp"

namespace dds {

namespace {

template <typename T, bool ADD>
__global__ void __launch_bounds__(256) k_nye(const T* __restrict__ n, const T* __restrict__ t, const T* __restrict__ b,
                                             T* __restrict__ rho, int64_t cells, int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t r = e / cells, c = e - r * cells;       // realisation, cell
    const T nv = n[e];
    const T* tr = t + r * 3 * cells + c;
    const T* br = b + r * 3 * cells + c;
    T* out = rho + r * 9 * cells + c;
    const T bv[3] = {br[0], br[cells], br[2 * cells]};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const T nt = nv * tr[l * cells];
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const T v = nt * bv[g];
            T* o = out + (3 * l + g) * cells;
            if constexpr (ADD) *o = *o + v;
            else *o = v;
        }
    }
}

template <typename T>
void launch(const void* n, const void* t, const void* b, void* rho, int64_t cells, int64_t total, bool add,
            hipStream_t st) {
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (add)
        hipLaunchKernelGGL((k_nye<T, true>), dim3(blocks), dim3(256), 0, st, static_cast<const T*>(n),
                           static_cast<const T*>(t), static_cast<const T*>(b), static_cast<T*>(rho), cells, total);
    else
        hipLaunchKernelGGL((k_nye<T, false>), dim3(blocks), dim3(256), 0, st, static_cast<const T*>(n),
                           static_cast<const T*>(t), static_cast<const T*>(b), static_cast<T*>(rho), cells, total);
    check_hip(hipGetLastError(), "axis-basis density launch");
}

}  // namespace
}  // namespace dds

using namespace dds;

extern "C" ddstress_status ddstress_nye_density(const void* n, const void* t, const void* b, int32_t precision,
                                                const int32_t grid[3], int32_t nbatch, int32_t accumulate, void* rho,
                                                void* stream) {
    return guarded([&] {
        if (!n || !t || !b || !rho || !grid) fail(DDSTRESS_E_INVALID, "NULL argument");
        if (precision != 32 && precision != 64) fail(DDSTRESS_E_INVALID, "precision must be 32 or 64");
        if (nbatch < 1) fail(DDSTRESS_E_INVALID, "nbatch must be >= 1");
        if (accumulate != 0 && accumulate != 1) fail(DDSTRESS_E_INVALID, "accumulate must be 0 or 1");
        for (int a = 0; a < 3; ++a)
            if (grid[a] < 1) fail(DDSTRESS_E_INVALID, "grid sizes must be >= 1");
        const int64_t cells = (int64_t)grid[0] * grid[1] * grid[2];
        const int64_t total = cells * nbatch;
        if ((total + 255) / 256 > 0x7fffffff) fail(DDSTRESS_E_UNSUPPORTED, "too many cells");
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (precision == 32) launch<float>(n, t, b, rho, cells, total, accumulate != 0, st);
        else launch<double>(n, t, b, rho, cells, total, accumulate != 0, st);
    });
}
