// Fused x and y passes of planes that fit in one block's LDS: the inverse
// y and inverse x (complex-to-real) after the z pass, and the forward x
// (real-to-complex) and forward y before it.
//
// Inverse. After the fused z pass, every (realisation, stress component,
// z) plane holds Py rows of M+1 complex values (kx); the plain path transforms
// its kx columns back along y into Ny rows (written to memory) and then each
// row back along x into Nx reals (read again). Here one block of 1024 threads
// keeps the Ny x (M+1) intermediate plane in LDS, so it never travels to
// memory:
//   1. the kx columns are transformed along y (8 elements per thread) in
//      rounds of 16-column groups; each group exchanges through its own LDS
//      region placed after the plane columns already finished, so a round
//      takes up to two groups, as many as the remaining LDS holds (32, 32, 32,
//      32 and 1 columns at Py = 256, M = 128);
//      rows y < Ny go to the plane, stored as column c at c (Py/2) + (y ^ (c & 15))
//      (the XOR spreads a group's 16 columns over the banks);
//   2. each row is combined into Z'[k] = (X[k] + conj X[M-k]) + i exp(+2 pi i k / P)
//      (X[k] - conj X[M-k]) (the same split as k_x_c2r), transformed along x
//      with the plane's LDS reused for the exchanges, and written as Nx reals.
// The block walks over planes (one resident block per CU); the column loads
// of the next round, and of the next plane's first round, are requested
// before the current transforms so their latency overlaps them. The
// arithmetic is that of the two plain passes at element classes 8 (y) and 16
// (x), so results are identical.
//
// Forward. Every (realisation, channel, z) plane of the density holds Ny rows
// of Nx reals. One block transforms each row along x (real-to-complex, the
// split of k_x_r2c) and keeps the (M+1) x Ny spectrum plane in LDS, column c
// at (M - c) (Py/2) + (y ^ (c & 15)) (reversed, so the columns consumed first
// free a contiguous range at the end), then transforms the kx columns along y
// (rows >= Ny are the zero padding; 8 elements per thread) in rounds of
// 16-column groups whose exchange regions take the LDS freed so far (16, 32,
// 32, 32 and 17 columns at Py = 256, M = 128), writing the Py rows of each
// column. Same arithmetic as the separate passes at element classes 16 (x)
// and 8 (y).
#include "ddstress_internal.hpp"

namespace dds {

namespace {

constexpr int kYXThreads = 1024;
constexpr int kYXLds = 160 * 1024;       // LDS per block on gfx950
constexpr int kYXBlocks = 256;           // one resident block per compute unit

// Round r of the column transforms: first column, groups and columns.
template <int PY, int M, int GC, int GT>
__device__ __forceinline__ void yx_round(int c0, int& groups, int& ncols) {
    constexpr int PLD = PY / 2;
    constexpr int CAP = kYXLds / (int)sizeof(cplx<float>);
    groups = (CAP - c0 * PLD) / (PY * GC);
    if (groups > kYXThreads / GT) groups = kYXThreads / GT;
    ncols = groups * GC < M + 1 - c0 ? groups * GC : M + 1 - c0;
    groups = (ncols + GC - 1) / GC;
}

template <int PY, int M>
__global__ void __launch_bounds__(kYXThreads) k_yx_inv(const cplx<float>* __restrict__ in, float* __restrict__ out,
                                                       int64_t nplanes, int ny, int nx, int64_t wx,
                                                       const cplx<float>* __restrict__ tw, int xld, int xsh,
                                                       int pairs, double* __restrict__ rowsq) {
    using T = float;
    constexpr int M1 = M + 1;
    constexpr int PLD = PY / 2;                          // plane column stride: rows y < Py/2
    constexpr int GC = 16, EY = 8, TCY = PY / EY;        // y: 16 columns per group, Tc threads per column
    constexpr int GT = GC * TCY;                         // threads per group
    constexpr int EX = 16, TCX = M / EX;                 // x: Tc threads per row
    static_assert(kYXThreads % GT == 0 && kYXThreads / TCX >= PY / 2, "launch shape");
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int t = threadIdx.x;
    const int gi = t / GT, tl = t % GT, cl = tl % GC, jy0 = tl / GC;    // column-transform roles
    const int jx0 = t % TCX, y = t / TCX;                                // row-transform roles
    const bool row_ok = y < ny;
    const cplx<T>* tw2 = tw + (2 * M - 1);
    int jy = jy0;

    // The block walks over planes; the loads of the next round (or of the next
    // plane's first round) are requested before the current transform.
    cplx<T> nxt[EY];
    auto load_cols = [&](int64_t pl, int c0) {
        int groups, ncols;
        yx_round<PY, M, GC, GT>(c0, groups, ncols);
        const int c = c0 + gi * GC + cl;
        const bool valid = gi < groups && c < M1;
        const cplx<T>* src = in + pl * (int64_t)PY * wx;
#pragma unroll
        for (int m = 0; m < EY; ++m)
            nxt[m] = valid ? src[(int64_t)(jy + TCY * m) * wx + c] : cplx<T>{T(0), T(0)};
    };
    int64_t plane = blockIdx.x;
    if (plane < nplanes) load_cols(plane, 0);
    for (; plane < nplanes; plane += gridDim.x) {
        // Per-thread indices re-derived each plane: keeps the twiddles and
        // addresses of both steps from being held in registers across the loop.
        int jx = jx0;
        jy = jy0;
        asm volatile("" : "+v"(jx), "+v"(jy));
        // 1. inverse y of the kx columns, rounds of groups
        for (int c0 = 0; c0 < M1;) {
            int groups, ncols;
            yx_round<PY, M, GC, GT>(c0, groups, ncols);
            asm volatile("" : "+v"(jy));                  // per round, as above
            const bool act = gi < groups;                // whole waves
            const int c = c0 + gi * GC + cl;
            const bool valid = act && c < M1;
            cplx<T> reg[EY];
#pragma unroll
            for (int m = 0; m < EY; ++m) reg[m] = nxt[m];
            if (c0 + ncols < M1) load_cols(plane, c0 + ncols);
            cplx<T>* scratch = lds + c0 * PLD + (act ? gi : 0) * (PY * GC);
            fft_regs<T, PY, EY, false>(reg, scratch, ColMajor{GC}, cl, jy, tw + (PY - 1), act);
            __syncthreads();                             // the groups' last exchange reads are done
            if (valid) {
#pragma unroll
                for (int m = 0; m < (EY + 1) / 2; ++m) {    // rows y = j + Tc m < Py/2
                    const int yy = jy + TCY * m;
                    if (yy < ny) lds[c * PLD + (yy ^ (c & 15))] = reg[m];
                }
            }
            c0 += ncols;
        }
        if (plane + gridDim.x < nplanes) load_cols(plane + gridDim.x, 0);
        __syncthreads();

        // 2. per row: split into Z', inverse x, Nx reals
        cplx<T> reg[EX];
#pragma unroll
        for (int m = 0; m < EX; ++m) {
            const int k = jx + TCX * m;
            const int km = M - k;
            const int yr = row_ok ? y : 0;
            const cplx<T> xk = lds[k * PLD + (yr ^ (k & 15))];
            const cplx<T> xm = cconj(lds[km * PLD + (yr ^ (km & 15))]);
            const cplx<T> e = cadd(xk, xm);
            const cplx<T> wd = twmul<false>(csub(xk, xm), tw2[k]);   // exp(+2 pi i k/P) (X[k] - conj X[M-k])
            reg[m] = {e.x - wd.y, e.y + wd.x};                       // e + i wd
        }
        __syncthreads();                             // the plane is read: its LDS serves the x exchanges
        fft_regs<T, M, EX, false>(reg, lds, RowPad{xld, xsh}, y, jx, tw + (M - 1));
        if (row_ok) {
            T* dst = out + plane * (int64_t)ny * nx + (int64_t)y * nx;
            if (pairs) {
                cplx<T>* dst2 = reinterpret_cast<cplx<T>*>(dst);
#pragma unroll
                for (int m = 0; m < EX; ++m) {
                    const int q = jx + TCX * m;
                    if (2 * q < nx) dst2[q] = reg[m];
                }
            } else {
#pragma unroll
                for (int m = 0; m < EX; ++m) {
                    const int i0 = 2 * (jx + TCX * m);
                    if (i0 < nx) dst[i0] = reg[m].x;
                    if (i0 + 1 < nx) dst[i0 + 1] = reg[m].y;
                }
            }
            if (rowsq) row_square_sum<T, EX, TCX>(reg, jx, nx, rowsq + plane * (int64_t)ny + y);
        }
        __syncthreads();                             // the x exchanges are done before the next plane's columns
    }
}


template <int PY, int M>
__global__ void __launch_bounds__(kYXThreads) k_xy_fwd(const float* __restrict__ in, cplx<float>* __restrict__ out,
                                                       int ny, int nx, int64_t wx, const cplx<float>* __restrict__ tw,
                                                       int xld, int xsh, int pairs) {
    using T = float;
    constexpr int M1 = M + 1;
    constexpr int PLD = PY / 2;
    constexpr int GC = 16, EY = 8, TCY = PY / EY;
    constexpr int GT = GC * TCY;
    constexpr int CAP = kYXLds / (int)sizeof(cplx<T>);
    constexpr int EX = 16, TCX = M / EX;
    static_assert(kYXThreads % GT == 0 && kYXThreads / TCX >= PY / 2, "launch shape");
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int t = threadIdx.x;
    const int64_t plane = blockIdx.x;

    // 1. per row: reals in pairs, length-M transform, split into M+1 outputs
    {
        const int j = t % TCX, y = t / TCX;
        const bool row_ok = y < ny;
        const T* src = in + plane * (int64_t)ny * nx + (int64_t)(row_ok ? y : 0) * nx;
        cplx<T> reg[EX];
        if (pairs) {
            const cplx<T>* src2 = reinterpret_cast<const cplx<T>*>(src);
#pragma unroll
            for (int m = 0; m < EX; ++m) {
                const int q = j + TCX * m;
                reg[m] = (row_ok && 2 * q < nx) ? src2[q] : cplx<T>{T(0), T(0)};
            }
        } else {
#pragma unroll
            for (int m = 0; m < EX; ++m) {
                const int i0 = 2 * (j + TCX * m);
                T a = T(0), b = T(0);
                if (row_ok && i0 < nx) a = src[i0];
                if (row_ok && i0 + 1 < nx) b = src[i0 + 1];
                reg[m] = {a, b};
            }
        }
        const RowPad lay{xld, xsh};
        fft_regs<T, M, EX, true>(reg, lds, lay, y, j, tw + (M - 1));
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EX; ++m) lds[lay(j + TCX * m, y)] = reg[m];
        __syncthreads();
        const cplx<T>* tw2 = tw + (2 * M - 1);
        const T half = T(0.5);
        cplx<T> xs[EX];
#pragma unroll
        for (int m = 0; m < EX; ++m) {
            const int k = j + TCX * m;
            const cplx<T> zk = lds[lay(k, y)];
            const cplx<T> zm = cconj(lds[lay((M - k) & (M - 1), y)]);
            const cplx<T> e = cadd(zk, zm);
            const cplx<T> wd = cmul(tw2[k], csub(zk, zm));          // W_P^k (Z[k] - conj Z[M-k])
            xs[m] = {half * (e.x + wd.y), half * (e.y - wd.x)};     // e/2 - (i/2) wd
        }
        const cplx<T> z0 = lds[lay(0, y)];
        __syncthreads();                                 // the row spectra are read: the plane takes their LDS
        if (row_ok) {
#pragma unroll
            for (int m = 0; m < EX; ++m) {
                const int k = j + TCX * m;
                lds[(M - k) * PLD + (y ^ (k & 15))] = xs[m];
            }
            if (j == 0) lds[0 * PLD + (y ^ (M & 15))] = cplx<T>{z0.x - z0.y, T(0)};     // column M
        }
    }
    __syncthreads();

    // 2. forward y of the kx columns, rounds of groups growing into the freed LDS
    {
        cplx<T>* dst = out + plane * (int64_t)PY * wx;
        const int gi = t / GT, tl = t % GT, cl = tl % GC;
        int j = tl / GC;
        for (int c0 = 0; c0 < M1;) {
            asm volatile("" : "+v"(j));   // per round: keeps the twiddles from being held across rounds
            int groups = kYXThreads / GT, ncols = 0;
            for (; groups > 1; --groups) {
                ncols = groups * GC < M1 - c0 ? groups * GC : M1 - c0;
                const int g2 = (ncols + GC - 1) / GC;
                if (g2 * PY * GC <= CAP - (M1 - c0 - ncols) * PLD) break;
            }
            ncols = groups * GC < M1 - c0 ? groups * GC : M1 - c0;
            groups = (ncols + GC - 1) / GC;
            const bool act = gi < groups;
            const int c = c0 + gi * GC + cl;
            const bool valid = act && c < M1;
            cplx<T> reg[EY];
#pragma unroll
            for (int m = 0; m < EY; ++m) {
                const int y = j + TCY * m;
                reg[m] = (valid && 2 * m < EY && y < ny) ? lds[(M - c) * PLD + (y ^ (c & 15))]
                                                         : cplx<T>{T(0), T(0)};
            }
            cplx<T>* scratch = lds + (M1 - c0 - ncols) * PLD + (act ? gi : 0) * (PY * GC);
            fft_regs<T, PY, EY, true>(reg, scratch, ColMajor{GC}, cl, j, tw + (PY - 1), act);
            if (valid) {
#pragma unroll
                for (int m = 0; m < EY; ++m) dst[(int64_t)(j + TCY * m) * wx + c] = reg[m];
            }
            c0 += ncols;
        }
    }
}

}  // namespace

bool yx_inv_fits(int Py, int M, int ny, int elem_bytes) {
    if (elem_bytes != 4 || Py != 256 || M != 128 || ny < 1 || ny > Py / 2) return false;
    const XLayout xl = x_lds_layout(M, 16, elem_bytes);
    return (size_t)(Py / 2) * xl.ld * 2 * elem_bytes <= (size_t)kYXLds &&
           (size_t)(M + 1) * (Py / 2) * 2 * elem_bytes <= (size_t)kYXLds;
}

void launch_xy_fwd(const float* in, cplx<float>* out, int64_t nplanes, int Py, int M, int ny, int nx, int64_t wx,
                   const cplx<float>* tw, hipStream_t s) {
    if (nplanes <= 0) return;
    if (!yx_inv_fits(Py, M, ny, 4)) fail(DDSTRESS_E_INVALID, "plane does not fit the fused forward x-y kernel");
    if (nplanes > 0x7fffffffLL) fail(DDSTRESS_E_UNSUPPORTED, "grid too large for one launch");
    const XLayout xl = x_lds_layout(M, 16, 4);
    const int pairs = (reinterpret_cast<uintptr_t>(in) % 8 == 0 && nx % 2 == 0) ? 1 : 0;
    hipLaunchKernelGGL((k_xy_fwd<256, 128>), dim3((unsigned)nplanes), dim3(kYXThreads), kYXLds, s, in, out, ny, nx,
                       wx, tw, xl.ld, xl.s, pairs);
    check_hip(hipGetLastError(), "fused forward x-y launch");
}

void launch_yx_inv(const cplx<float>* in, float* out, int64_t nplanes, int Py, int M, int ny, int nx, int64_t wx,
                   const cplx<float>* tw, hipStream_t s, double* rowsq) {
    if (nplanes <= 0) return;
    if (!yx_inv_fits(Py, M, ny, 4)) fail(DDSTRESS_E_INVALID, "plane does not fit the fused inverse y-x kernel");
    if (nplanes > 0x7fffffffLL) fail(DDSTRESS_E_UNSUPPORTED, "grid too large for one launch");
    const XLayout xl = x_lds_layout(M, 16, 4);
    const int pairs = (reinterpret_cast<uintptr_t>(out) % 8 == 0 && nx % 2 == 0) ? 1 : 0;
    // one resident block per CU walks over the planes
    const int64_t grid = nplanes < kYXBlocks ? nplanes : kYXBlocks;
    hipLaunchKernelGGL((k_yx_inv<256, 128>), dim3((unsigned)grid), dim3(kYXThreads), kYXLds, s, in, out, nplanes, ny,
                       nx, wx, tw, xl.ld, xl.s, pairs, rowsq);
    check_hip(hipGetLastError(), "fused inverse y-x launch");
}

}  // namespace dds
