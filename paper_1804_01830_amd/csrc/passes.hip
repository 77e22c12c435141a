// The x and y passes and the host-side launch rules of all passes; the fused
// z kernels are in zfused.hpp (compiled in separate units).
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

#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

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
                                               int rows_per_block, int pairs, int ld, int lsh) {
    constexpr int Tc = M / E;
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int j = threadIdx.x % Tc;
    const int rl = threadIdx.x / Tc;
    const int64_t row = (int64_t)blockIdx.x * rows_per_block + rl;
    const bool valid = row < nrows;
    const RowPad lay{ld, lsh};
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
    // a row's Tc threads (Tc <= 64 for every planned length) are consecutive
    // lanes of one wave and its LDS row is its own: the transform and the
    // split synchronise within the wave
    constexpr bool WV = Tc <= 64;
    fft_regs<T, M, E, true, false, WV>(reg, lds, lay, rl, j, tw + (M - 1));
    stage_sync<WV>();
#pragma unroll
    for (int m = 0; m < E; ++m) lds[lay(j + Tc * m, rl)] = reg[m];
    stage_sync<WV>();
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
                                               int rows_per_block, int pairs, int ld, int lsh,
                                               double* __restrict__ rowsq) {
    constexpr int Tc = M / E;
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int j = threadIdx.x % Tc;
    const int rl = threadIdx.x / Tc;
    const int64_t row = (int64_t)blockIdx.x * rows_per_block + rl;
    const bool valid = row < nrows;
    const RowPad lay{ld, lsh};
    const cplx<T>* src = in + (valid ? row : 0) * in_stride;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = j + Tc * m;
        lds[lay(k, rl)] = valid ? src[k] : cplx<T>{T(0), T(0)};
    }
    constexpr bool WV = Tc <= 64;          // the row is its wave's own (see k_x_r2c)
    if (j == 0) lds[lay(M, rl)] = valid ? src[M] : cplx<T>{T(0), T(0)};
    stage_sync<WV>();
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
    fft_regs<T, M, E, false, false, WV>(reg, lds, lay, rl, j, tw + (M - 1));
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
    if (rowsq) row_square_sum<T, E, Tc>(reg, j, n_out, rowsq + row);
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
// Launch geometry and dispatch. A transform of length N runs with
// E = min(N, ev) elements per thread, where the element class ev is a tuning
// choice (it also bounds the radix, R <= E): 8 or 16 for the x and y passes;
// 4 (FP32) or 2 (FP64) for the fused z pass, whose threads keep their
// spectrum values and accumulators per element in registers. Long z
// transforms (N >= 256) with many channels also take 2, 4 or 8 times that
// class, so that one column per group fits a block.
// ----------------------------------------------------------------------------
static int ecount(int N, int ev) { return N < ev ? N : ev; }
int x_threads(int M, int rows, int ev) { return rows * (M / ecount(M, ev)); }
int col_threads(int N, int tk, int ev) { return tk * (N / ecount(N, ev)); }
// Threads of a fused z block: `groups` groups (1, or one per density channel)
// of tk x N/E threads.
int z_threads(int N, int groups, int tk, int ev) { return groups * tk * (N / ecount(N, ev)); }
int z_max_threads(int groups) { return groups == 1 ? 512 : 768; }
bool z_groups_ok(int groups, int C) { return groups == 1 || groups == C; }
// Many realisations amortise the grouped form's larger blocks; it is the
// default from 16 realisations on, where one column per group fits a block
// (threads and LDS).
int default_z_groups(int N, int C, int B, int elem_bytes) {
    if (B < 16) return 1;
    const int ev = default_ev_z(N, C, elem_bytes);
    const int e = N < ev ? N : ev;
    const bool fits = z_threads(N, C, 1, e) <= z_max_threads(C) && z_lds_bytes(N, 1, C, C, elem_bytes) <= 64 * 1024;
    return fits ? C : 1;
}

// LDS column stride of the fused z kernels (one column block per tile).
int z_lds_ld(int tk, int elem_bytes) {
    (void)elem_bytes;
    return tk;
}

// LDS of a fused z block, in N x ld column blocks: the single-group form
// exchanges through one; the grouped form keeps one per channel or per stress
// component, whichever are more (the regions are reused).
size_t z_lds_bytes(int N, int tk, int C, int groups, int elem_bytes) {
    const int regions = groups == 1 ? 1 : (C > 6 ? C : 6);
    return (size_t)regions * N * z_lds_ld(tk, elem_bytes) * 2 * elem_bytes;
}

// The single-group form stages its spectrum tile (nkz rows of (6C + 1) tk
// values) in LDS for the compile-time widths tk = 4, 8, 16, when there are
// realisations to reuse it (B >= 2) and the tile and the exchange block fit
// 64 KiB together (z lengths up to 256; in FP64 with three channels only,
// more would spill registers).
size_t z_stage_bytes(int tk, int C, int nkz, int elem_bytes) {
    return (size_t)nkz * (6 * C + 1) * tk * elem_bytes;
}
bool z_stage_spec(int N, int tk, int C, int nkz, int B, int elem_bytes) {
    return B >= 2 && N <= 256 && (tk == 4 || tk == 8 || tk == 16) && (elem_bytes <= 4 || C == 3) &&
           z_lds_bytes(N, tk, C, 1, elem_bytes) + z_stage_bytes(tk, C, nkz, elem_bytes) <= 64 * 1024;
}
int default_ev_col(int N) { return N <= 64 ? 8 : 16; }
static int base_ev_z(int elem_bytes) { return elem_bytes <= 4 ? 4 : 2; }
constexpr int kLongZ = 256;              // shortest z length with the larger classes

bool ev_z_ok(int N, int ev, int elem_bytes) {
    const int b = base_ev_z(elem_bytes);
    if (ev == b) return true;
    if (elem_bytes == 4 && N == 64 && ev == 8) return true;          // the wave form
    return N >= kLongZ && ev <= 16 && (ev == 2 * b || ev == 4 * b || ev == 8 * b);
}

// The wave form: FP32, z length 64, element class 8, one thread group; its
// tile is kZWaveTile columns (8 lanes each: one wave).
bool z_wave_form(int N, int ev, int groups, int elem_bytes) {
    return elem_bytes == 4 && N == 64 && ev == 8 && groups == 1;
}
// Its LDS: the staged spectrum tile (16-byte aligned) and one 64 x 8 exchange
// region per wave (min(B, 4) waves).
size_t z_wave_lds_bytes(int N, int C, int nkz, int B) {
    const int wpb = B >= 4 ? 4 : (B >= 2 ? 2 : 1);
    return (z_stage_bytes(kZWaveTile, C, nkz, 4) + 15) / 16 * 16 + (size_t)wpb * N * kZWaveTile * 8;
}

// The base class, or the smallest larger one with which a block of one
// column per group fits.
int default_ev_z(int N, int groups, int elem_bytes) {
    int ev = base_ev_z(elem_bytes);
    while (z_threads(N, groups, 1, ev) > z_max_threads(groups) && ev_z_ok(N, 2 * ev, elem_bytes)) ev *= 2;
    return ev;
}
bool ev_col_ok(int ev) { return ev == 8 || ev == 16; }

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
    const int e = ecount(M, default_ev_col(M));
    const int tc = M / e;
    const int ld = x_lds_ld(M, e, elem_bytes);
    int rows = 256 / tc;
    if (rows < 1) rows = 1;
    while (rows > 1 && (int64_t)rows * ld * 2 * elem_bytes > 64 * 1024) rows /= 2;
    return rows;
}

int default_z_tk(int N, int C, int groups, int elem_bytes) {
    const int tc = N / ecount(N, default_ev_z(N, groups, elem_bytes));
    int tk;
    if (groups == 1) {
        const int tk_min = elem_bytes <= 4 ? 16 : 8;
        tk = 256 / tc;
        if (tk < tk_min) tk = tk_min;
    } else {
        tk = 128 / tc;
    }
    if (tk < 1) tk = 1;
    while (tk > 1 && (z_lds_bytes(N, tk, C, groups, elem_bytes) > 64 * 1024 ||
                      z_threads(N, groups, tk, ecount(N, default_ev_z(N, groups, elem_bytes))) > z_max_threads(groups)))
        tk /= 2;
    return tk;
}


// LDS layout of the x passes: element i of row r at r * ld + i + (i >> s),
// one pad element every 2^s. The layout is chosen per (M, E, precision) by
// evaluating an LDS bank model over a few candidates: 32 banks of 4 bytes, an
// access of w bytes per lane served 128 / w lanes at a time, each group taking
// as many cycles as the most distinct dwords on one bank. (The model
// reproduces the bank-conflict counters measured on the passes' kernels.) The
// accesses modelled are one block's Stockham exchanges (the same index
// formulas as fft_stage), the row split reads of k and M - k and of element M.
namespace {

int lds_group_cycles(const std::vector<int>& addr, int width) {
    const int per = std::max(1, 128 / width);
    int cycles = 0;
    for (size_t g0 = 0; g0 < addr.size(); g0 += per) {
        std::map<int, std::set<int>> banks;
        for (size_t l = g0; l < std::min(addr.size(), g0 + per); ++l)
            for (int d = 0; d < width / 4; ++d) {
                const int dw = addr[l] / 4 + d;
                banks[dw % 32].insert(dw);
            }
        size_t worst = 0;
        for (auto& kv : banks) worst = std::max(worst, kv.second.size());
        cycles += (int)worst;
    }
    return cycles;
}

double x_layout_cost(int M, int E, int elem, int ld, int s) {
    const int Tc = M / E, width = 2 * elem;
    const int nthr = std::min(256, std::max(64, Tc));
    auto lay = [&](int i, int r) { return (r * ld + i + (i >> s)) * width; };
    std::vector<std::function<int(int, int)>> acc;
    for (int Ns = 1; Ns < M;) {
        const int R = std::min(std::min(8, E), M / Ns), NB = E / R;
        const bool first = Ns == 1, last = Ns * R == M;
        for (int q = 0; q < NB; ++q)
            for (int r = 0; r < R; ++r) {
                if (!first) acc.push_back([=](int j, int row) { return lay(j + Tc * q + r * (M / R), row); });
                if (!last)
                    acc.push_back([=](int j, int row) {
                        const int b = j + Tc * q;
                        return lay((b / Ns) * Ns * R + (b % Ns) + r * Ns, row);
                    });
            }
        Ns *= R;
    }
    for (int m = 0; m < E; ++m) {
        acc.push_back([=](int j, int row) { return lay(j + Tc * m, row); });
        acc.push_back([=](int j, int row) { return lay((M - (j + Tc * m)) & (M - 1), row); });
    }
    long cycles = 0, ideal = 0;
    std::vector<int> addr;
    for (int w0 = 0; w0 < nthr; w0 += 64)
        for (auto& f : acc) {
            addr.clear();
            for (int t = w0; t < std::min(nthr, w0 + 64); ++t) addr.push_back(f(t % Tc, t / Tc));
            cycles += lds_group_cycles(addr, width);
            ideal += ((int)addr.size() * width + 127) / 128;
        }
    return (double)cycles / (double)std::max(1L, ideal);
}

}  // namespace

XLayout x_lds_layout(int M, int E, int elem_bytes) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, XLayout> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(M, E, elem_bytes);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    XLayout best{M + 1, 30};
    if (M >= 8) {
        double best_cost = x_layout_cost(M, E, elem_bytes, M + 1, 30);
        for (int s : {3, 4})
            for (int extra = 0; extra < 16; ++extra) {
                const int ld = M + (M >> s) + 1 + extra;
                const double c = x_layout_cost(M, E, elem_bytes, ld, s);
                if (c < best_cost - 1e-9) {
                    best_cost = c;
                    best = {ld, s};
                }
            }
    }
    cache[key] = best;
    return best;
}
int x_lds_ld(int M, int E, int elem_bytes) { return x_lds_layout(M, E, elem_bytes).ld; }

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
    switch (M) {
#define X_CASE(L, EVV)                                                                                     \
    case L: {                                                                                              \
        constexpr int E = L < EVV ? L : EVV;                                                               \
        const XLayout xl = x_lds_layout(L, E, (int)sizeof(T));                                            \
        const size_t lds = (size_t)rows * xl.ld * sizeof(cplx<T>);                                         \
        hipLaunchKernelGGL((k_x_r2c<T, L, E>), dim3((unsigned)blocks), dim3(rows * (L / E)), lds, s, in, out, \
                           nrows, n_in, in_stride, out_stride, tw, rows, pairs, xl.ld, xl.s);                           \
        break;                                                                                             \
    }
        DDS_FOR_LENGTHS(X_CASE, EV)
#undef X_CASE
        default: fail(DDSTRESS_E_UNSUPPORTED, "x transform length not supported");
    }
}

template <typename T, int EV>
static void x_c2r_ev(int M, const cplx<T>* in, T* out, int64_t nrows, int n_out, int64_t in_stride,
                     int64_t out_stride, const cplx<T>* tw, int rows, double* rowsq, hipStream_t s) {
    const int64_t blocks = (nrows + rows - 1) / rows;
    const int pairs = pairs_ok(out, out_stride, n_out);
    switch (M) {
#define X_CASE(L, EVV)                                                                                     \
    case L: {                                                                                              \
        constexpr int E = L < EVV ? L : EVV;                                                               \
        const XLayout xl = x_lds_layout(L, E, (int)sizeof(T));                                            \
        const size_t lds = (size_t)rows * xl.ld * sizeof(cplx<T>);                                         \
        hipLaunchKernelGGL((k_x_c2r<T, L, E>), dim3((unsigned)blocks), dim3(rows * (L / E)), lds, s, in, out, \
                           nrows, n_out, in_stride, out_stride, tw, rows, pairs, xl.ld, xl.s, rowsq);                   \
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
                  int64_t out_stride, const cplx<T>* tw, int rows, hipStream_t s, double* rowsq) {
    if (nrows <= 0) return;
    if (ev == 8) x_c2r_ev<T, 8>(M, in, out, nrows, n_out, in_stride, out_stride, tw, rows, rowsq, s);
    else if (ev == 16) x_c2r_ev<T, 16>(M, in, out, nrows, n_out, in_stride, out_stride, tw, rows, rowsq, s);
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
void launch_z_fused(int N, int ev, int groups, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& geom,
                    const cplx<T>* tw, int tk, hipStream_t s) {
    if (tk < 1 || geom.ntiles != (geom.ncols + tk - 1) / tk)
        fail(DDSTRESS_E_INVALID, "fused z tiles do not match the tile width");
    ZGeom g = geom;
    g.nyq = g.strip ? z_nyq_groups(g.ncols, tk, g.nky) : 0;
    // tiles x ky rows; in place of the Nyquist strip's tile, its groups x realisations
    const int64_t blocks = g.nyq > 0 ? (int64_t)(g.ntiles - 1) * g.nky + (int64_t)g.nyq * g.B
                                     : (int64_t)g.ntiles * g.nky;
    if (blocks <= 0) return;
    if (blocks > 0x7fffffffLL) fail(DDSTRESS_E_UNSUPPORTED, "grid too large for one launch");
    if (!ev_z_ok(N, ev, (int)sizeof(T))) fail(DDSTRESS_E_INVALID, "z element class not supported for this length");
    if (!z_groups_ok(groups, g.C)) fail(DDSTRESS_E_INVALID, "z thread groups must be 1 or the channel count");
    if (ev == 8 && N == 64 && sizeof(T) == 4) {
        if (!z_wave_form(N, ev, groups, 4) || tk != kZWaveTile || z_wave_lds_bytes(N, g.C, g.nkz_s, g.B) > 64 * 1024)
            fail(DDSTRESS_E_INVALID, "the wave form of the fused z pass takes one thread group, 8-column tiles "
                                     "and 64 KiB of LDS");
    } else if (tk < 1 || z_threads(N, groups, tk, ev) > z_max_threads(groups) ||
               z_lds_bytes(N, tk, g.C, groups, (int)sizeof(T)) > 64 * 1024) {
        fail(DDSTRESS_E_INVALID, "fused z block exceeds the thread or LDS limit");
    }
    // one instance per channel count: the channel loops are unrolled
    const bool grouped = groups != 1;
    switch (g.C) {
        case 3:
            grouped ? z_dispatch<T, 3, true>(N, ev, in, out, spec, g, tw, tk, blocks, s)
                    : z_dispatch<T, 3, false>(N, ev, in, out, spec, g, tw, tk, blocks, s);
            break;
        case 6:
            grouped ? z_dispatch<T, 6, true>(N, ev, in, out, spec, g, tw, tk, blocks, s)
                    : z_dispatch<T, 6, false>(N, ev, in, out, spec, g, tw, tk, blocks, s);
            break;
        case 9:
            grouped ? z_dispatch<T, 9, true>(N, ev, in, out, spec, g, tw, tk, blocks, s)
                    : z_dispatch<T, 9, false>(N, ev, in, out, spec, g, tw, tk, blocks, s);
            break;
        default: fail(DDSTRESS_E_INVALID, "channel count must be 3, 6 or 9");
    }
    check_hip(hipGetLastError(), "fused z launch");
}

#define INSTANTIATE(T)                                                                                     \
    template void launch_x_r2c<T>(int, int, const T*, cplx<T>*, int64_t, int, int64_t, int64_t, const cplx<T>*, \
                                  int, hipStream_t);                                                       \
    template void launch_x_c2r<T>(int, int, const cplx<T>*, T*, int64_t, int, int64_t, int64_t, const cplx<T>*, \
                                  int, hipStream_t, double*);                                              \
    template void launch_col_fft<T>(int, int, bool, const cplx<T>*, cplx<T>*, const ColGeom&, const cplx<T>*, \
                                    int, hipStream_t);                                                     \
    template void launch_z_fused<T>(int, int, int, const cplx<T>*, cplx<T>*, const T*, const ZGeom&,          \
                                    const cplx<T>*, int, hipStream_t);
INSTANTIATE(float)
INSTANTIATE(double)
#undef INSTANTIATE

}  // namespace dds
