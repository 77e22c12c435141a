// The five passes of one stress evaluation (zero-padded convolution of
// Eq. (10) by the convolution theorem, Sec. 2.3):
//   x: real-to-complex along x      (rows contiguous)
//   y: complex along y              (strided, tiles of consecutive kx)
//   z: forward z, per-wavevector contraction with the kernel spectrum,
//      inverse z                    (strided, fused, accumulators in registers)
//   y: inverse, cropped to Ny
//   x: complex-to-real, cropped to Nx
// The same x and strided kernels, instantiated in FP64, transform the
// interaction coefficients when a plan is built.
#include "ddstress_internal.hpp"

namespace dds {

// ----------------------------------------------------------------------------
// x: real-to-complex of length P = 2M. Row r has n_in reals (the rest of the P
// inputs are zero). The reals are packed in pairs, z[m] = x[2m] + i x[2m+1],
// transformed with length M and split into the M+1 non-redundant outputs
//   X[k] = (Z[k] + conj Z[M-k]) / 2 - (i/2) exp(-2 pi i k / P) (Z[k] - conj Z[M-k]).
// ----------------------------------------------------------------------------
template <typename T, int M, int E>
__global__ void __launch_bounds__(512) k_x_r2c(const T* __restrict__ in, cplx<T>* __restrict__ out,
                                               int64_t nrows, int n_in, int64_t in_stride,
                                               int64_t out_stride, const cplx<T>* __restrict__ tw,
                                               int rows_per_block, int pairs) {
    constexpr int Tc = M / E;
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int j = threadIdx.x % Tc;
    const int rl = threadIdx.x / Tc;
    const int64_t row = (int64_t)blockIdx.x * rows_per_block + rl;
    const bool valid = row < nrows;
    const RowMajor lay{M + 1};
    const T* src = in + (valid ? row : 0) * in_stride;
    cplx<T> reg[E];
    if (pairs) {        // rows aligned to a pair of reals and n_in even: one access per pair
        const cplx<T>* src2 = reinterpret_cast<const cplx<T>*>(src);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int p = j + Tc * m;
            reg[m] = (valid && 2 * p < n_in) ? src2[p] : cplx<T>{T(0), T(0)};
        }
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i0 = 2 * (j + Tc * m);
            T a = T(0), b = T(0);
            if (valid && i0 < n_in) a = src[i0];
            if (valid && i0 + 1 < n_in) b = src[i0 + 1];
            reg[m] = {a, b};
        }
    }
    fft_regs<T, M, E, true>(reg, lds, lay, rl, j, tw + (M - 1));
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) lds[lay(j + Tc * m, rl)] = reg[m];
    __syncthreads();
    if (!valid) return;
    cplx<T>* dst = out + row * out_stride;
    const cplx<T>* tw2 = tw + (2 * M - 1);
    const T half = T(0.5);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = j + Tc * m;
        const cplx<T> zk = lds[lay(k, rl)];
        const cplx<T> zm = cconj(lds[lay((M - k) & (M - 1), rl)]);
        const cplx<T> e = cadd(zk, zm);
        const cplx<T> wd = cmul(tw2[k], csub(zk, zm));          // W_P^k (Z[k] - conj Z[M-k])
        dst[k] = {half * (e.x + wd.y), half * (e.y - wd.x)};   // e/2 - (i/2) wd
    }
    if (j == 0) {
        const cplx<T> z0 = lds[lay(0, rl)];
        dst[M] = {z0.x - z0.y, T(0)};
    }
}

// ----------------------------------------------------------------------------
// x: complex-to-real of length P = 2M (unnormalised inverse), from the M+1
// non-redundant inputs of each row, keeping the first n_out reals:
//   Z'[k] = (X[k] + conj X[M-k]) + i exp(+2 pi i k / P) (X[k] - conj X[M-k]),
//   z = inverse length-M transform of Z',  x[2m] = Re z[m], x[2m+1] = Im z[m].
// ----------------------------------------------------------------------------
template <typename T, int M, int E>
__global__ void __launch_bounds__(512) k_x_c2r(const cplx<T>* __restrict__ in, T* __restrict__ out,
                                               int64_t nrows, int n_out, int64_t in_stride,
                                               int64_t out_stride, const cplx<T>* __restrict__ tw,
                                               int rows_per_block, int pairs) {
    constexpr int Tc = M / E;
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int j = threadIdx.x % Tc;
    const int rl = threadIdx.x / Tc;
    const int64_t row = (int64_t)blockIdx.x * rows_per_block + rl;
    const bool valid = row < nrows;
    const RowMajor lay{M + 1};
    const cplx<T>* src = in + (valid ? row : 0) * in_stride;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = j + Tc * m;
        lds[lay(k, rl)] = valid ? src[k] : cplx<T>{T(0), T(0)};
    }
    if (j == 0) lds[lay(M, rl)] = valid ? src[M] : cplx<T>{T(0), T(0)};
    __syncthreads();
    const cplx<T>* tw2 = tw + (2 * M - 1);
    cplx<T> reg[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = j + Tc * m;
        const cplx<T> xk = lds[lay(k, rl)];
        const cplx<T> xm = cconj(lds[lay(M - k, rl)]);
        const cplx<T> e = cadd(xk, xm);
        const cplx<T> wd = twmul<false>(csub(xk, xm), tw2[k]);   // exp(+2 pi i k/P) (X[k] - conj X[M-k])
        reg[m] = {e.x - wd.y, e.y + wd.x};                       // e + i wd
    }
    fft_regs<T, M, E, false>(reg, lds, lay, rl, j, tw + (M - 1));
    if (!valid) return;
    T* dst = out + row * out_stride;
    if (pairs) {        // rows aligned to a pair of reals and n_out even
        cplx<T>* dst2 = reinterpret_cast<cplx<T>*>(dst);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int p = j + Tc * m;
            if (2 * p < n_out) dst2[p] = reg[m];
        }
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i0 = 2 * (j + Tc * m);
            if (i0 < n_out) dst[i0] = reg[m].x;
            if (i0 + 1 < n_out) dst[i0 + 1] = reg[m].y;
        }
    }
}

// ----------------------------------------------------------------------------
// Complex transform of length N along a strided axis. A block owns `tk`
// consecutive columns (contiguous in memory) of one (outer, plane) pair and
// all N rows of them; rows >= n_in are zero, rows >= n_out are not written.
// Every global load of a block precedes its first store, so in == out works.
// ----------------------------------------------------------------------------
template <typename T, int N, int E, bool FWD>
__global__ void __launch_bounds__(512) k_col_fft(const cplx<T>* in, cplx<T>* out, ColGeom g,
                                                 const cplx<T>* __restrict__ tw, int tk,
                                                 int64_t ntiles) {
    constexpr int Tc = N / E;
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int c = threadIdx.x % tk;
    const int j = threadIdx.x / tk;
    int64_t bid = blockIdx.x;
    const int64_t tile = bid % ntiles;
    bid /= ntiles;
    const int64_t outer = bid % g.nouter;
    const int64_t plane = bid / g.nouter;
    const int64_t col = tile * tk + c;
    const bool valid = col < g.ncols;
    const cplx<T>* src = in + plane * g.ips + outer * g.ios + (valid ? col : 0);
    const int irs = (int)g.irs, ors = (int)g.ors;   // in-block offsets fit in 32 bits (N * stride < 2^31)
    cplx<T> reg[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = j + Tc * m;
        reg[m] = (valid && i < g.n_in) ? src[i * irs] : cplx<T>{T(0), T(0)};
    }
    fft_regs<T, N, E, FWD>(reg, lds, ColMajor{tk}, c, j, tw + (N - 1));
    if (!valid) return;
    cplx<T>* dst = out + plane * g.ops + outer * g.oos + col;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = j + Tc * m;
        if (i < g.n_out) dst[i * ors] = reg[m];
    }
}

// ----------------------------------------------------------------------------
// Fused z pass. A block owns `tk` consecutive kx columns at one ky. For every
// realisation b it transforms the C density columns along z (length N, nz
// inputs), accumulates the six stress spectra
//     sigma^_v(k) = sum_c i S_{v,c}(k) rho^_c(k)        (K^ = i S, K odd)
// in registers with a fixed channel order, and transforms each back along z,
// writing the first nz rows. The spectrum tile of the block is stored
// contiguously as [c][v][kz][tk].
// The loads are software-pipelined: the density column and the spectrum
// values of the next channel (or of the next realisation's first channel) are
// requested before the current transform, whose barriers do not wait for
// global loads, so their latency overlaps the FFT work.
// ----------------------------------------------------------------------------
template <typename T, int N, int E, int NC>
__global__ void __launch_bounds__(512) k_z_fused(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                 const T* __restrict__ spec, ZGeom g,
                                                 const cplx<T>* __restrict__ tw, int tk) {
    constexpr int Tc = N / E;
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int c = threadIdx.x % tk;
    const int j = threadIdx.x / tk;
    const int tile = blockIdx.x % g.ntiles;
    const int ky = blockIdx.x / g.ntiles;
    const int col = tile * tk + c;
    const bool valid = col < g.ncols;
    const int colc = valid ? col : 0;
    const ColMajor lay{tk};
    const cplx<T>* twN = tw + (N - 1);
    const int ors = (int)g.ors;                      // in-block offsets fit in 32 bits
    // Spectrum tile of this block: [c][v][kzc][tk] at row kyc. With a y mirror
    // only ky <= Py/2 is stored and row Py - ky stands in for ky > Py/2; with a
    // z mirror only kz <= N/2 is stored and elements m >= E/2 (kz >= N/2) read
    // kz' = N - kz = (Tc - j) + Tc (E - 1 - m). Odd planes change sign.
    const bool flip_y = g.nky_s < g.nky && 2 * ky > g.nky;
    const int kyc = flip_y ? g.nky - ky : ky;
    const bool zc = g.nkz_s < N;
    const int nkz = g.nkz_s;
    const T* sp = spec + ((int64_t)kyc * g.ntiles + tile) * (int64_t)g.C * 6 * nkz * tk;
    const __amdgpu_buffer_rsrc_t srs = make_rsrc(sp, (uint32_t)((size_t)g.C * 6 * nkz * tk * sizeof(T)));
    const int s_lane = (j * tk + c) * (int)sizeof(T);
    const int s_lane_m = ((Tc - j) * tk + c) * (int)sizeof(T);
    // density planes: rows z < nz of the block's columns; rows >= nz lie beyond the resource (read as zero)
    const cplx<T>* in_b = in + (int64_t)ky * g.ios + (int64_t)tile * tk;
    const uint32_t plane_bytes = (uint32_t)((size_t)g.nz * g.irs * sizeof(cplx<T>));
    // lanes of padding columns (col >= ncols) read the tile's first column, which is valid
    const int r_lane = (j * (int)g.irs + (valid ? c : 0)) * (int)sizeof(cplx<T>);
    const int r_step = Tc * (int)g.irs * (int)sizeof(cplx<T>);
    cplx<T>* out_b = out + (int64_t)ky * g.oos + colc;

#define DDS_LOAD_RHO(DST, BB, CH)                                                          \
    {                                                                                      \
        const __amdgpu_buffer_rsrc_t rr_ = make_rsrc(in_b + (int64_t)((BB) * g.C + (CH)) * g.iqs, plane_bytes); \
        _Pragma("unroll") for (int m = 0; m < E; ++m) DST[m] = buf_cplx<T>(rr_, r_lane, m * r_step); \
    }
#define DDS_LOAD_SPEC(DST, CH)                                                             \
    {                                                                                      \
        _Pragma("unroll") for (int v = 0; v < 6; ++v) {                                    \
            const int base_ = ((CH) * 6 + v) * nkz;                                        \
            _Pragma("unroll") for (int m = 0; m < E; ++m) {                                \
                const bool mir_ = zc && (2 * m >= E);      /* uniform: selects, no branch */ \
                DST[v][m] = buf_real<T>(srs, mir_ ? s_lane_m : s_lane,                     \
                                        (base_ + (mir_ ? Tc * (E - 1 - m) : Tc * m)) * tk * (int)sizeof(T)); \
            }                                                                              \
        }                                                                                  \
    }

    cplx<T> cur[E], nxt[E];
    T sv[6][E];
    DDS_LOAD_RHO(cur, 0, 0)
    DDS_LOAD_SPEC(sv, 0)
    for (int b = 0; b < g.B; ++b) {
        cplx<T> acc[6][E];
#pragma unroll
        for (int v = 0; v < 6; ++v)
#pragma unroll
            for (int m = 0; m < E; ++m) acc[v][m] = {T(0), T(0)};
        // channels in groups of three (one line direction): unrolled inside a
        // group, a runtime loop over the groups
        for (int l = 0; l < NC / 3; ++l) {
#pragma unroll
            for (int gq = 0; gq < 3; ++gq) {
                const int ch = 3 * l + gq;
                const bool more = gq < 2 || l + 1 < NC / 3;
                if (more) DDS_LOAD_RHO(nxt, b, ch + 1)
                fft_regs<T, N, E, true>(cur, lds, lay, c, j, twN);
#pragma unroll
                for (int v = 0; v < 6; ++v) {
                    // signs of mirrored spectrum rows (wave-uniform)
                    const int bit = ch * 6 + v;
                    const T sy = (flip_y && ((g.sgn_y >> bit) & 1)) ? T(-1) : T(1);
                    const T sz = ((g.sgn_z >> bit) & 1) ? -sy : sy;
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const T sval = ((zc && 2 * m >= E) ? sz : sy) * sv[v][m];
                        acc[v][m].x -= sval * cur[m].y;
                        acc[v][m].y += sval * cur[m].x;
                    }
                }
                if (more) {
                    DDS_LOAD_SPEC(sv, ch + 1)
#pragma unroll
                    for (int m = 0; m < E; ++m) cur[m] = nxt[m];
                }
            }
        }
        if (b + 1 < g.B) {      // first channel of the next realisation
            DDS_LOAD_RHO(cur, b + 1, 0)
            DDS_LOAD_SPEC(sv, 0)
        }
#undef DDS_LOAD_RHO
#undef DDS_LOAD_SPEC
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            fft_regs<T, N, E, false>(acc[v], lds, lay, c, j, twN);
            if (valid) {
                cplx<T>* dst = out_b + (int64_t)(b * 6 + v) * g.oqs;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int z = j + Tc * m;
                    if (z < g.nz) dst[z * ors] = acc[v][m];
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Launch geometry and dispatch. A transform of length N runs with
// E = min(N, ev) elements per thread, where the element class ev is a tuning
// choice (it also bounds the radix, R <= E): 8 or 16 for the x and y passes;
// 4 (FP32) or 2 (FP64) for the fused z pass, which keeps six accumulators,
// the next channel's spectrum values and density column per element in
// registers (larger classes spill).
// ----------------------------------------------------------------------------
static int ecount(int N, int ev) { return N < ev ? N : ev; }
int x_threads(int M, int rows, int ev) { return rows * (M / ecount(M, ev)); }
int col_threads(int N, int tk, int ev) { return tk * (N / ecount(N, ev)); }
int z_threads(int N, int tk, int ev) { return tk * (N / ecount(N, ev)); }
int default_ev_col(int N) { return N <= 64 ? 8 : 16; }
int default_ev_z(int elem_bytes) { return elem_bytes <= 4 ? 4 : 2; }
bool ev_col_ok(int ev) { return ev == 8 || ev == 16; }
bool ev_z_ok(int ev, int elem_bytes) { return elem_bytes <= 4 ? ev == 4 : ev == 2; }

int default_col_tk(int N, int elem_bytes) {
    const int tc = N / ecount(N, default_ev_col(N));
    const int tk_min = elem_bytes <= 4 ? 16 : 8;
    int tk = 256 / tc;
    if (tk < tk_min) tk = tk_min;
    while (tk > 1 && tk * tc > 512) tk /= 2;
    while (tk > 1 && (int64_t)N * tk * 2 * elem_bytes > 64 * 1024) tk /= 2;
    return tk;
}

int default_rows(int M, int elem_bytes) {
    const int tc = M / ecount(M, default_ev_col(M));
    int rows = 256 / tc;
    if (rows < 1) rows = 1;
    while (rows > 1 && (int64_t)rows * (M + 1) * 2 * elem_bytes > 64 * 1024) rows /= 2;
    return rows;
}

int default_z_tk(int N, int elem_bytes) {
    const int tc = N / ecount(N, default_ev_z(elem_bytes));
    const int tk_min = elem_bytes <= 4 ? 16 : 8;
    int tk = 256 / tc;
    if (tk < tk_min) tk = tk_min;
    while (tk > 1 && tk * tc > 512) tk /= 2;
    while (tk > 1 && (int64_t)N * tk * 2 * elem_bytes > 64 * 1024) tk /= 2;
    return tk;
}

#define DDS_FOR_LENGTHS(X, EV) X(1, EV) X(2, EV) X(4, EV) X(8, EV) X(16, EV) X(32, EV) X(64, EV) \
    X(128, EV) X(256, EV) X(512, EV) X(1024, EV)

// Real rows can be accessed in pairs when every row starts on a pair boundary.
template <typename T>
static int pairs_ok(const T* base, int64_t stride, int n) {
    return ((reinterpret_cast<uintptr_t>(base) % (2 * sizeof(T))) == 0 && stride % 2 == 0 && n % 2 == 0) ? 1 : 0;
}

template <typename T, int EV>
static void x_r2c_ev(int M, const T* in, cplx<T>* out, int64_t nrows, int n_in, int64_t in_stride,
                     int64_t out_stride, const cplx<T>* tw, int rows, hipStream_t s) {
    const int64_t blocks = (nrows + rows - 1) / rows;
    const int pairs = pairs_ok(in, in_stride, n_in);
    const size_t lds = (size_t)rows * (M + 1) * sizeof(cplx<T>);
    switch (M) {
#define X_CASE(L, EVV)                                                                                     \
    case L: {                                                                                              \
        constexpr int E = L < EVV ? L : EVV;                                                               \
        hipLaunchKernelGGL((k_x_r2c<T, L, E>), dim3((unsigned)blocks), dim3(rows * (L / E)), lds, s, in, out, \
                           nrows, n_in, in_stride, out_stride, tw, rows, pairs);                           \
        break;                                                                                             \
    }
        DDS_FOR_LENGTHS(X_CASE, EV)
#undef X_CASE
        default: fail(DDSTRESS_E_UNSUPPORTED, "x transform length not supported");
    }
}

template <typename T, int EV>
static void x_c2r_ev(int M, const cplx<T>* in, T* out, int64_t nrows, int n_out, int64_t in_stride,
                     int64_t out_stride, const cplx<T>* tw, int rows, hipStream_t s) {
    const int64_t blocks = (nrows + rows - 1) / rows;
    const int pairs = pairs_ok(out, out_stride, n_out);
    const size_t lds = (size_t)rows * (M + 1) * sizeof(cplx<T>);
    switch (M) {
#define X_CASE(L, EVV)                                                                                     \
    case L: {                                                                                              \
        constexpr int E = L < EVV ? L : EVV;                                                               \
        hipLaunchKernelGGL((k_x_c2r<T, L, E>), dim3((unsigned)blocks), dim3(rows * (L / E)), lds, s, in, out, \
                           nrows, n_out, in_stride, out_stride, tw, rows, pairs);                          \
        break;                                                                                             \
    }
        DDS_FOR_LENGTHS(X_CASE, EV)
#undef X_CASE
        default: fail(DDSTRESS_E_UNSUPPORTED, "x transform length not supported");
    }
}

template <typename T, int EV, bool FWD>
static void col_ev(int N, const cplx<T>* in, cplx<T>* out, const ColGeom& g, const cplx<T>* tw, int tk,
                   int64_t ntiles, int64_t blocks, hipStream_t s) {
    const size_t lds = (size_t)N * tk * sizeof(cplx<T>);
    switch (N) {
#define C_CASE(L, EVV)                                                                                     \
    case L: {                                                                                              \
        constexpr int E = L < EVV ? L : EVV;                                                               \
        hipLaunchKernelGGL((k_col_fft<T, L, E, FWD>), dim3((unsigned)blocks), dim3(tk * (L / E)), lds, s, in, \
                           out, g, tw, tk, ntiles);                                                        \
        break;                                                                                             \
    }
        DDS_FOR_LENGTHS(C_CASE, EV)
#undef C_CASE
        default: fail(DDSTRESS_E_UNSUPPORTED, "column transform length not supported");
    }
}

template <typename T, int EV, int NC>
static void z_ev(int N, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& g, const cplx<T>* tw,
                 int tk, int64_t blocks, hipStream_t s) {
    const size_t lds = (size_t)N * tk * sizeof(cplx<T>);
    switch (N) {
#define Z_CASE(L, EVV)                                                                                     \
    case L: {                                                                                              \
        constexpr int E = L < EVV ? L : EVV;                                                               \
        hipLaunchKernelGGL((k_z_fused<T, L, E, NC>), dim3((unsigned)blocks), dim3(tk * (L / E)), lds, s, in, \
                           out, spec, g, tw, tk);                                                          \
        break;                                                                                             \
    }
        DDS_FOR_LENGTHS(Z_CASE, EV)
#undef Z_CASE
        default: fail(DDSTRESS_E_UNSUPPORTED, "z transform length not supported");
    }
}

template <typename T>
void launch_x_r2c(int M, int ev, const T* in, cplx<T>* out, int64_t nrows, int n_in, int64_t in_stride,
                  int64_t out_stride, const cplx<T>* tw, int rows, hipStream_t s) {
    if (nrows <= 0) return;
    if (ev == 8) x_r2c_ev<T, 8>(M, in, out, nrows, n_in, in_stride, out_stride, tw, rows, s);
    else if (ev == 16) x_r2c_ev<T, 16>(M, in, out, nrows, n_in, in_stride, out_stride, tw, rows, s);
    else fail(DDSTRESS_E_INVALID, "x element class must be 8 or 16");
    check_hip(hipGetLastError(), "x r2c launch");
}

template <typename T>
void launch_x_c2r(int M, int ev, const cplx<T>* in, T* out, int64_t nrows, int n_out, int64_t in_stride,
                  int64_t out_stride, const cplx<T>* tw, int rows, hipStream_t s) {
    if (nrows <= 0) return;
    if (ev == 8) x_c2r_ev<T, 8>(M, in, out, nrows, n_out, in_stride, out_stride, tw, rows, s);
    else if (ev == 16) x_c2r_ev<T, 16>(M, in, out, nrows, n_out, in_stride, out_stride, tw, rows, s);
    else fail(DDSTRESS_E_INVALID, "x element class must be 8 or 16");
    check_hip(hipGetLastError(), "x c2r launch");
}

template <typename T>
void launch_col_fft(int N, int ev, bool forward, const cplx<T>* in, cplx<T>* out, const ColGeom& g,
                    const cplx<T>* tw, int tk, hipStream_t s) {
    const int64_t ntiles = (g.ncols + tk - 1) / tk;
    const int64_t blocks = ntiles * g.nouter * g.nplanes;
    if (blocks <= 0) return;
    if (blocks > 0x7fffffffLL) fail(DDSTRESS_E_UNSUPPORTED, "grid too large for one launch");
    if (ev == 8 && forward) col_ev<T, 8, true>(N, in, out, g, tw, tk, ntiles, blocks, s);
    else if (ev == 8) col_ev<T, 8, false>(N, in, out, g, tw, tk, ntiles, blocks, s);
    else if (ev == 16 && forward) col_ev<T, 16, true>(N, in, out, g, tw, tk, ntiles, blocks, s);
    else if (ev == 16) col_ev<T, 16, false>(N, in, out, g, tw, tk, ntiles, blocks, s);
    else fail(DDSTRESS_E_INVALID, "column element class must be 8 or 16");
    check_hip(hipGetLastError(), "column fft launch");
}

template <typename T>
void launch_z_fused(int N, int ev, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& g,
                    const cplx<T>* tw, int tk, hipStream_t s) {
    const int64_t blocks = (int64_t)g.ntiles * g.nky;
    if (blocks <= 0) return;
    if (!ev_z_ok(ev, (int)sizeof(T))) fail(DDSTRESS_E_INVALID, "z element class not supported for this precision");
    constexpr int EV = sizeof(T) == 4 ? 4 : 2;
    switch (g.C) {     // the channel loop is unrolled: one instance per line count
        case 3: z_ev<T, EV, 3>(N, in, out, spec, g, tw, tk, blocks, s); break;
        case 6: z_ev<T, EV, 6>(N, in, out, spec, g, tw, tk, blocks, s); break;
        case 9: z_ev<T, EV, 9>(N, in, out, spec, g, tw, tk, blocks, s); break;
        default: fail(DDSTRESS_E_INVALID, "channel count must be 3, 6 or 9");
    }
    check_hip(hipGetLastError(), "fused z launch");
}

#define INSTANTIATE(T)                                                                                     \
    template void launch_x_r2c<T>(int, int, const T*, cplx<T>*, int64_t, int, int64_t, int64_t, const cplx<T>*, \
                                  int, hipStream_t);                                                       \
    template void launch_x_c2r<T>(int, int, const cplx<T>*, T*, int64_t, int, int64_t, int64_t, const cplx<T>*, \
                                  int, hipStream_t);                                                       \
    template void launch_col_fft<T>(int, int, bool, const cplx<T>*, cplx<T>*, const ColGeom&, const cplx<T>*, \
                                    int, hipStream_t);                                                     \
    template void launch_z_fused<T>(int, int, const cplx<T>*, cplx<T>*, const T*, const ZGeom&, const cplx<T>*, \
                                    int, hipStream_t);
INSTANTIATE(float)
INSTANTIATE(double)
#undef INSTANTIATE

}  // namespace dds
