// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <new>
#include <string>

#include "../../include/ddstress.h"
#include "fft_device.hpp"

namespace dds {

// Error plumbing: the C entry points catch these and turn them into statuses.
struct Error {
    ddstress_status status;
    std::string msg;
};
[[noreturn]] void fail(ddstress_status s, const std::string& msg);
void check_hip(hipError_t e, const char* what);
void set_last_error(const std::string& msg);

// Runs f and turns what it throws into a status (the message is kept for
// ddstress_last_error).
template <class F>
ddstress_status guarded(F&& f) {
    try {
        f();
        return DDSTRESS_OK;
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return DDSTRESS_E_NOMEM;
    } catch (...) {
        set_last_error("unexpected internal error");
        return DDSTRESS_E_DEVICE;
    }
}

// Device buffer that frees itself.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t n, const char* what) {
        release();
        if (n == 0) n = 256;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            fail(DDSTRESS_E_NOMEM, std::string("device allocation failed: ") + what + " (" +
                                       std::to_string(n) + " bytes)");
        }
        bytes = n;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}
inline int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Largest supported FFT length on any axis.
constexpr int kMaxLen = 1024;
// Twiddle table: entry L-1+k holds exp(-2 pi i k / L) for every power of two L <= kMaxLen.
constexpr int kTwiddleEntries = 2 * kMaxLen;

template <typename T>
void fill_twiddles(cplx<T>* host);   // kTwiddleEntries entries

// Periodic boundary conditions in the layer plane (axis 0: x, 1: y).
inline bool periodic_axis(const ddstress_desc* d, int axis) {
    return (d->flags & (axis == 0 ? DDSTRESS_FLAG_PERIODIC_X : DDSTRESS_FLAG_PERIODIC_Y)) != 0;
}
constexpr int kMaxPbcShells = 32;
constexpr int kDefaultPbcShells = 15;

// ---- pass launchers (passes.hip) -------------------------------------------
// Real-to-complex transform of length P = 2M along contiguous rows.
template <typename T>
void launch_x_r2c(int M, int ev, const T* in, cplx<T>* out, int64_t nrows, int n_in, int64_t in_stride,
                  int64_t out_stride, const cplx<T>* tw, int rows_per_block, hipStream_t s);
// Complex-to-real transform of length P = 2M along rows, keeping n_out reals.
// With rowsq, also the sum of squares of each row's outputs (FP64) at
// rowsq[row] (the plane statistics of Eq. 20, summed per plane afterwards).
template <typename T>
void launch_x_c2r(int M, int ev, const cplx<T>* in, T* out, int64_t nrows, int n_out, int64_t in_stride,
                  int64_t out_stride, const cplx<T>* tw, int rows_per_block, hipStream_t s,
                  double* rowsq = nullptr);

// Sum of squares of one row held by TC consecutive lanes of a wave (lane j
// owns pairs j + TC m, m < E; n_out reals are valid), in FP64, reduced in a
// fixed order; lane 0 writes it.
template <typename T, int E, int TC>
__device__ __forceinline__ void row_square_sum(const cplx<T>* reg, int j, int n_out, double* dst) {
    static_assert(TC >= 1 && (TC & (TC - 1)) == 0, "power-of-two lanes per row");
    if constexpr (TC > 64) {
        // rows of more than 64 lanes (half lengths above 512) are never planned
        if (j == 0) *dst = __builtin_nan("");
        return;
    }
    double sq = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i0 = 2 * (j + TC * m);
        if (i0 < n_out) sq += (double)reg[m].x * (double)reg[m].x;
        if (i0 + 1 < n_out) sq += (double)reg[m].y * (double)reg[m].y;
    }
#pragma unroll
    for (int o = TC / 2; o > 0; o >>= 1) sq += __shfl_xor(sq, o, TC);
    if (j == 0) *dst = sq;
}
// Plane statistics from row sums: out[p] = inv * sum_{y < ny} rowsq[p ny + y]
// (in a fixed order), for planes p < nplanes (stats.hip).
void launch_rowsq_finish(const double* rowsq, int64_t nplanes, int ny, double inv, double* out, hipStream_t s);
// Complex transform of length N along a strided axis, on tiles of consecutive columns.
struct ColGeom {
    int ncols;             // valid columns (consecutive in memory)
    int n_in, n_out;       // rows read (the rest are zero) and rows written
    int64_t nouter, nplanes;
    int64_t irs, ios, ips; // input row / outer / plane strides (elements)
    int64_t ors, oos, ops; // output strides
};
template <typename T>
void launch_col_fft(int N, int ev, bool forward, const cplx<T>* in, cplx<T>* out, const ColGeom& g,
                    const cplx<T>* tw, int tk, hipStream_t s);
// Fused forward z transform, contraction with the kernel spectrum and inverse z.
struct ZGeom {
    int nky_s, nkz_s;      // spectrum rows kept along ky and kz (Py or Py/2+1, Pz or Pz/2+1)
    uint64_t sgn_y, sgn_z; // bit c*6+v set: S_{v,c} is odd under ky -> -ky (resp. kz -> -kz)
    int ncols;             // valid kx columns
    int ntiles;            // kx tiles (ncols rounded up to tk)
    int nky;               // ky rows (blocks along y)
    int nz;                // rows read and written along z
    int C, B;              // channels and batch
    int64_t irs, iqs, ios; // input z / plane / ky strides
    int64_t ors, oqs, oos; // output strides (6B planes)
    int strip;             // the spectrum keeps the Nyquist strip where the tiles allow it
    int nyq;               // groups of the Nyquist strip (z_nyq_groups; set by launch_z_fused)
};
// Plans of at least this many realisations keep the Nyquist strip.
constexpr int kZStripBatch = 4;

// Nyquist strip of the fused z pass (plans of kZStripBatch or more
// realisations, ZGeom::strip). When the last kx tile would hold the
// column kx = M (= ncols - 1) alone, which happens whenever M is a multiple of
// the tile width tk, that tile's blocks hold the column at tk consecutive ky
// instead: group q covers ky = q tk .. q tk + tk - 1, and only ky <= Py/2 is
// evaluated (the column is Hermitian along y; the rest is written as the
// conjugate mirror); one block per group and realisation. The spectrum keeps
// the strip in the last tile's slot, group q at row q, lane c at column c.
// Returns the number of groups, or 0 when the last tile holds other columns
// too.
__host__ __device__ inline int z_nyq_groups(int ncols, int tk, int nky) {
    return (ncols > tk && (ncols - 1) % tk == 0) ? (nky / 2 + tk) / tk : 0;
}
template <typename T>
void launch_z_fused(int N, int ev, int groups, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& g,
                    const cplx<T>* tw, int tk, hipStream_t s);

// Launch geometry: threads per block, element classes and defaults.
int x_threads(int M, int rows, int ev);
struct XLayout {
    int ld, s;       // LDS row stride and pad shift of the x passes
};
XLayout x_lds_layout(int M, int E, int elem_bytes);
int x_lds_ld(int M, int E, int elem_bytes);
int col_threads(int N, int tk, int ev);
int z_threads(int N, int groups, int tk, int ev);
int default_ev_col(int N);
int default_ev_z(int N, int groups, int elem_bytes);
bool ev_col_ok(int ev);
bool ev_z_ok(int N, int ev, int elem_bytes);
int default_col_tk(int N, int elem_bytes);
int default_rows(int M, int elem_bytes);
int default_z_tk(int N, int C, int groups, int elem_bytes);
size_t z_lds_bytes(int N, int tk, int C, int groups, int elem_bytes);
int z_lds_ld(int tk, int elem_bytes);
bool z_groups_ok(int groups, int C);
int default_z_groups(int N, int C, int B, int elem_bytes);
int z_max_threads(int groups);
size_t z_stage_bytes(int tk, int C, int nkz, int elem_bytes);
bool z_stage_spec(int N, int tk, int C, int nkz, int B, int elem_bytes);
// The wave form of the fused z pass (FP32, z length 64, element class 8, one
// thread group): one wave per tile of kZWaveTile columns and realisation.
constexpr int kZWaveTile = 8;
bool z_wave_form(int N, int ev, int groups, int elem_bytes);
size_t z_wave_lds_bytes(int N, int C, int nkz, int B);

// Fused z launch for C = NC channels and one form (zfused.hpp; instantiated
// per form and precision in z_serial_f32.hip, z_grouped_f64.hip, ...).
template <typename T, int NC, bool GROUPED>
void z_dispatch(int N, int ev, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& g,
                const cplx<T>* tw, int tk, int64_t blocks, hipStream_t s);

// Fused forward x and y, and fused inverse y and x, for planes that fit one
// block's LDS (yx_fused.hip): FP32, Py = 256, M = 128. The spectrum planes
// (Py rows of wx complex values) are interleaved in groups of zp: plane p
// starts at (p / zp) zp Py wx + (p % zp) wx and its rows are zp wx apart
// (zp = 1: each plane contiguous).
bool yx_inv_fits(int Py, int M, int ny, int elem_bytes);
void launch_yx_inv(const cplx<float>* in, float* out, int64_t nplanes, int Py, int M, int ny, int nx, int64_t wx,
                   const cplx<float>* tw, hipStream_t s, double* rowsq = nullptr, int zp = 1);
void launch_xy_fwd(const float* in, cplx<float>* out, int64_t nplanes, int Py, int M, int ny, int nx, int64_t wx,
                   const cplx<float>* tw, hipStream_t s, int zp = 1);

// Every power-of-two transform length the passes support.
#define DDS_FOR_LENGTHS(X, EV) X(1, EV) X(2, EV) X(4, EV) X(8, EV) X(16, EV) X(32, EV) X(64, EV) \
    X(128, EV) X(256, EV) X(512, EV) X(1024, EV)

// ---- kernel build (kernel_build.hip) ---------------------------------------
struct KernelParams {
    int n[3];
    int P[3];
    double d[3];
    double s[3];       // subcell edges
    int m[3];          // subcells per axis
    double t[3];       // unit line direction
    double mu, nu;
    double h_cell, h_sub;
    double dV;
    double near_lim;   // S * max(d)
    int per[2];        // 1: x (y) periodic, P = N there, offsets summed over replica shells
    int shells;        // replica shells n_sh of the periodic axes
};
KernelParams make_kernel_params(const ddstress_desc& desc, int line, const int P[3]);
// 18 planes [gamma][v][Pz][Py][Px] of FP64 coefficients.
void launch_kernel_build(const KernelParams& p, double* out, hipStream_t s);
// Mirror parity statistics of the 18 planes (see k_mirror_stats): 90 values.
void launch_mirror_stats(const double* kr, const int P[3], unsigned long long* stats, hipStream_t s);
// Spectrum extraction: S[kyc][tile][c][v][kzc][tk] = Im(Khat) / P for channels 3*line..3*line+2,
// kyc < nky, kzc < nkz.
template <typename T>
void launch_extract(const cplx<double>* kh, T* spec, int line, int C, int ncols, int64_t wx, int Py, int Pz,
                    int nky, int nkz, int tk, int ntiles, bool strip, double inv_p, unsigned long long* maxbits,
                    hipStream_t s);

}  // namespace dds
