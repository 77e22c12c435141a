// In-plane mean square of each stress component at each height (Sec. 6,
// Eq. 20). Standalone: one block per (realisation, component, layer) plane, FP64
// accumulation in a fixed order (four independent partial sums per thread,
// then a tree over the block), so the result does not depend on anything
// but the input. Reads the stress once: an HBM-bound reduction. Fused with
// the stress call: the inverse x pass leaves one sum of squares per row and
// k_rowsq_finish adds the rows of each plane in a fixed order.
#include "ddstress_internal.hpp"

namespace dds {

namespace {

constexpr int kStatThreads = 512;

template <typename T>
__global__ void __launch_bounds__(kStatThreads)
    k_plane_ms(const T* __restrict__ sigma, int64_t plane, double inv_plane, double* __restrict__ out) {
    const T* p = sigma + (int64_t)blockIdx.x * plane;
    const int t = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t e = t;
    for (; e + 3 * kStatThreads < plane; e += 4 * kStatThreads) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = (double)p[e + q * kStatThreads];
            acc[q] += v * v;
        }
    }
    for (int q = 0; e < plane; e += kStatThreads, ++q) {
        const double v = (double)p[e];
        acc[q & 3] += v * v;
    }
    __shared__ double red[kStatThreads];
    red[t] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    for (int w = kStatThreads / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[blockIdx.x] = red[0] * inv_plane;
}

// One wave per plane (four per block): lane l adds rows l, l + 64, ... in
// order (consecutive lanes read consecutive rows), then the 64 partial sums
// are combined by a butterfly; the order is fixed, so every call gives the
// same bits.
__global__ void __launch_bounds__(256) k_rowsq_finish(const double* __restrict__ rowsq, int64_t nplanes, int ny,
                                                      double inv, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= nplanes) return;           // whole waves: the butterfly below has every lane
    const double* r = rowsq + p * ny;
    double s = 0.0;
    for (int y = lane; y < ny; y += 64) s += r[y];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) out[p] = s * inv;
}

}  // namespace

void launch_rowsq_finish(const double* rowsq, int64_t nplanes, int ny, double inv, double* out, hipStream_t s) {
    if (nplanes <= 0) return;
    if ((nplanes + 3) / 4 > 0x7fffffffLL) fail(DDSTRESS_E_UNSUPPORTED, "too many planes for one launch");
    hipLaunchKernelGGL(k_rowsq_finish, dim3((unsigned)((nplanes + 3) / 4)), dim3(256), 0, s, rowsq, nplanes, ny, inv,
                       out);
    check_hip(hipGetLastError(), "plane statistics finish launch");
}

}  // namespace dds

using namespace dds;

extern "C" ddstress_status ddstress_plane_mean_square(const void* sigma, int32_t precision, const int32_t n[3],
                                                      int32_t nbatch, double* out, void* stream) {
    return guarded([&] {
        if (!sigma || !out || !n) fail(DDSTRESS_E_INVALID, "NULL argument");
        if (precision != 32 && precision != 64) fail(DDSTRESS_E_INVALID, "precision must be 32 or 64");
        if (nbatch < 1) fail(DDSTRESS_E_INVALID, "nbatch must be >= 1");
        for (int a = 0; a < 3; ++a)
            if (n[a] < 1) fail(DDSTRESS_E_INVALID, "grid sizes must be >= 1");
        const int64_t planes = (int64_t)nbatch * 6 * n[2];
        if (planes > 0x7fffffff) fail(DDSTRESS_E_UNSUPPORTED, "too many planes");
        const int64_t plane = (int64_t)n[0] * n[1];
        hipStream_t st = static_cast<hipStream_t>(stream);
        const double inv = 1.0 / (double)plane;
        if (precision == 32)
            hipLaunchKernelGGL((k_plane_ms<float>), dim3((unsigned)planes), dim3(kStatThreads), 0, st,
                               static_cast<const float*>(sigma), plane, inv, out);
        else
            hipLaunchKernelGGL((k_plane_ms<double>), dim3((unsigned)planes), dim3(kStatThreads), 0, st,
                               static_cast<const double*>(sigma), plane, inv, out);
        check_hip(hipGetLastError(), "plane statistics launch");
    });
}
