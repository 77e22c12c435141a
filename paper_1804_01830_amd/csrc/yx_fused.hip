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
//      takes up to two groups, as many as the remaining LDS holds (4 rounds of
//      32 columns at Py = 256, M = 128: columns 0 and M, whose transforms are
//      real, travel together as X[0] + i X[M]);
//      rows y < Ny go to the plane, stored as column c at c (Py/2) + (y ^ (c & 15))
//      (the XOR spreads a group's 16 columns over the banks);
//   2. each row is combined into Z'[k] = (X[k] + conj X[M-k]) + i exp(+2 pi i k / P)
//      (X[k] - conj X[M-k]) (the same split as k_x_c2r), transformed along x
//      with the plane's LDS reused for the exchanges, and written as Nx reals.
// The block walks over planes (one resident block per CU); the column loads
// of the next round, and of the next plane's first round, are requested
// before the current transforms so their latency overlaps them. The
// arithmetic is that of the two plain passes at element classes 8 (y) and 16
// (x), except for the packed columns 0 and M (so the results agree with the
// separate passes to rounding, not bit for bit).
//
// Twiddles. Vector-memory loads and stores complete in issue order, so a
// twiddle load issued after a column prefetch (or after a round's stores)
// would wait for it. The y twiddles are therefore loaded into registers once
// per plane, before the prefetches, and the x phase reads its two tables
// (exp(-2 pi i k / M) and exp(-2 pi i k / P), k < M) from the top 2M values of
// LDS, which the row exchanges leave free.
//
// Forward. Every (realisation, channel, z) plane of the density holds Ny rows
// of Nx reals. A block (one resident per CU, walking over planes, the next
// plane's rows requested before the current plane's column transforms)
// transforms each row along x (real-to-complex, the split of k_x_r2c; with an
// open x axis the upper half of every packed row is zero and the first stage
// skips it) and keeps the (M+1) x Ny spectrum plane in LDS, column c
// at (M - c) (Py/2) + (y ^ (c & 15)) (reversed, so the columns consumed first
// free a contiguous range at the end), then transforms the kx columns along y
// (rows >= Ny are the zero padding; 8 elements per thread) in rounds of
// 16-column groups whose exchange regions take the LDS freed so far (16, 32,
// 32, 32 and 17 columns at Py = 256, M = 128), writing the Py rows of each
// column. Same values as the separate passes at element classes 16 (x) and
// 8 (y): the first stages skip only inputs that are zero.
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
    ncols = groups * GC < M - c0 ? groups * GC : M - c0;
    groups = (ncols + GC - 1) / GC;
}

template <int PY, int M>
__global__ void __launch_bounds__(kYXThreads) k_yx_inv(const cplx<float>* __restrict__ in, float* __restrict__ out,
                                                       int64_t nplanes, int ny, int nx, int64_t wx,
                                                       const cplx<float>* __restrict__ tw, int xld, int xsh,
                                                       int pairs, double* __restrict__ rowsq, int zp) {
    using T = float;
    constexpr int PLD = PY / 2;                          // plane column stride: rows y < Py/2
    constexpr int GC = 16, EY = 8, TCY = PY / EY;        // y: 16 columns per group, Tc threads per column
    constexpr int GT = GC * TCY;                         // threads per group
    constexpr int EX = 16, TCX = M / EX;                 // x: Tc threads per row
    constexpr int TWY = tw_count(PY, EY);                // y twiddles per thread
    static_assert(kYXThreads % GT == 0 && kYXThreads / TCX >= PY / 2, "launch shape");
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* const twl = lds + kYXLds / (int)sizeof(cplx<T>) - 2 * M;   // x-phase twiddles (see below)
    const int t = threadIdx.x;
    const int gi = t / GT, tl = t % GT, cl = tl % GC, jy0 = tl / GC;    // column-transform roles
    const int jx0 = t % TCX, y = t / TCX;                                // row-transform roles
    const bool row_ok = y < ny;
    int jy = jy0;

    // The block walks over planes; the loads of the next round (or of the next
    // plane's first round) are requested before the current transform.
    cplx<T> nxt[EY];
    // Columns 0 and M (kx = 0 and the Nyquist column) are Hermitian along ky,
    // so their inverse transforms are real: they travel as the one column
    // X[0] + i X[M] and come out as Re = column 0, Im = column M (the z pass
    // writes column M exactly Hermitian; column 0's rounding-level imaginary
    // part is dropped). The rounds cover columns 0 .. M-1.
    auto load_cols = [&](int64_t pl, int c0) {
        int groups, ncols;
        yx_round<PY, M, GC, GT>(c0, groups, ncols);
        const int c = c0 + gi * GC + cl;
        const bool valid = gi < groups && c < M;
        const cplx<T>* src = in + (pl / zp) * zp * (int64_t)PY * wx + (pl % zp) * wx;   // interleaved planes
        const int64_t rs = (int64_t)zp * wx;
#pragma unroll
        for (int m = 0; m < EY; ++m) {
            const int64_t r = (int64_t)(jy + TCY * m) * rs;
            nxt[m] = valid ? src[r + c] : cplx<T>{T(0), T(0)};
            if (valid && c == 0) {
                const cplx<T> xm = src[r + M];
                nxt[m] = {nxt[m].x - xm.y, nxt[m].y + xm.x};
            }
        }
    };
    int64_t plane = blockIdx.x;
    if (plane < nplanes) load_cols(plane, 0);
    for (; plane < nplanes; plane += gridDim.x) {
        // Per-thread indices re-derived each plane: keeps the twiddles and
        // addresses of both steps from being held in registers across the loop.
        int jx = jx0;
        jy = jy0;
        asm volatile("" : "+v"(jx), "+v"(jy));
        // 1. inverse y of the kx columns, rounds of groups. The twiddles are
        //    loaded once per plane, before the next round's columns are
        //    requested: vector loads (and stores) complete in issue order, so
        //    a twiddle load issued after them would wait for them.
        cplx<T> twy[TWY];
        load_tw_stages<T, PY, EY, 1, 0>(twy, jy, tw + (PY - 1));
        // the x-phase tables, written to the top of LDS after the rounds (which
        // use all of it): exp(-2 pi i k / M) and exp(-2 pi i k / P), k < M
        const cplx<T> tv = t < 2 * M ? tw[t < M ? (M - 1) + t : (2 * M - 1) + (t - M)] : cplx<T>{T(0), T(0)};
        for (int c0 = 0; c0 < M;) {
            int groups, ncols;
            yx_round<PY, M, GC, GT>(c0, groups, ncols);
            asm volatile("" : "+v"(jy));                  // per round, as above
            const bool act = gi < groups;                // whole waves
            const int c = c0 + gi * GC + cl;
            const bool valid = act && c < M;
            cplx<T> reg[1][EY];
#pragma unroll
            for (int m = 0; m < EY; ++m) reg[0][m] = nxt[m];
            if (c0 + ncols < M) load_cols(plane, c0 + ncols);
            cplx<T>* scratch = lds + c0 * PLD + (act ? gi : 0) * (PY * GC);
            fft_regs_k<T, PY, EY, false, false, 1, TWY>(reg, twy, scratch, 0, ColMajor{GC}, cl, jy, act);
            __syncthreads();                             // the groups' last exchange reads are done
            if (valid) {
#pragma unroll
                for (int m = 0; m < (EY + 1) / 2; ++m) {    // rows y = j + Tc m < Py/2
                    const int yy = jy + TCY * m;
                    if (yy < ny) lds[c * PLD + (yy ^ (c & 15))] = reg[0][m];
                }
            }
            c0 += ncols;
        }
        if (plane + gridDim.x < nplanes) load_cols(plane + gridDim.x, 0);
        if (t < 2 * M) twl[t] = tv;                  // the rounds' exchange reads are done
        __syncthreads();

        // 2. per row: split into Z', inverse x, Nx reals (twiddles from LDS: they
        //    never wait behind the next plane's column loads)
        cplx<T> reg[EX];
#pragma unroll
        for (int m = 0; m < EX; ++m) {
            const int k = jx + TCX * m;
            const int km = M - k;
            const int yr = row_ok ? y : 0;
            cplx<T> xk = lds[k * PLD + (yr ^ (k & 15))];
            cplx<T> xm = cconj(lds[(km & (M - 1)) * PLD + (yr ^ (km & 15))]);
            if (m == 0 && k == 0) {                  // X[0] and X[M], both real, packed in column 0
                xm = {xk.y, T(0)};
                xk = {xk.x, T(0)};
            }
            const cplx<T> e = cadd(xk, xm);
            const cplx<T> wd = twmul<false>(csub(xk, xm), twl[M + k]);   // exp(+2 pi i k/P) (X[k] - conj X[M-k])
            reg[m] = {e.x - wd.y, e.y + wd.x};                       // e + i wd
        }
        __syncthreads();                             // the plane is read: its LDS serves the x exchanges
        // each row's TCX threads are consecutive lanes of one wave with an LDS
        // row of their own: its stages synchronise within the wave
        fft_regs<T, M, EX, false, false, true>(reg, lds, RowPad{xld, xsh}, y, jx, twl);
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
        // (no barrier here: the next plane's first LDS write follows the barrier
        // inside its first transform stage, which every thread reaches only
        // after this plane's reads)
    }
}


template <int PY, int M, bool HX>
__global__ void __launch_bounds__(kYXThreads) k_xy_fwd(const float* __restrict__ in, cplx<float>* __restrict__ out,
                                                       int64_t nplanes, int ny, int nx, int64_t wx,
                                                       const cplx<float>* __restrict__ tw, int xld, int xsh,
                                                       int pairs, int zp) {
    using T = float;
    constexpr int M1 = M + 1;
    constexpr int PLD = PY / 2;
    constexpr int GC = 16, EY = 8, TCY = PY / EY;
    constexpr int GT = GC * TCY;
    constexpr int CAP = kYXLds / (int)sizeof(cplx<T>);
    constexpr int EX = 16, TCX = M / EX;
    constexpr int EL = HX ? EX / 2 : EX;                 // row elements that can be non-zero
    constexpr int TWY = tw_count(PY, EY);                // y twiddles per thread
    static_assert(kYXThreads % GT == 0 && kYXThreads / TCX >= PY / 2, "launch shape");
    constexpr int CAPF = CAP - 2 * M;                    // the top 2M values hold the x-phase twiddles
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int t = threadIdx.x;
    // x-phase twiddle tables in LDS (read there, they never wait behind the
    // previous plane's stores): exp(-2 pi i k / M) and exp(-2 pi i k / P), k < M
    cplx<T>* const twl = lds + CAPF;
    for (int i = t; i < 2 * M; i += kYXThreads) twl[i] = i < M ? tw[(M - 1) + i] : tw[(2 * M - 1) + (i - M)];

    // The block walks over planes; the rows of the next plane are requested
    // before the current plane's column transforms. Per-thread indices are
    // re-derived at each use (here and per plane below): keeps addresses and
    // twiddles from being held in registers across the loop.
    cplx<T> nxt[EL];
    // Past the last plane (have == false) the registers are set to zero, so the
    // previous rows are dead once they are consumed.
    auto load_rows = [&](int64_t pl, bool have) {
        int tr = t;
        asm volatile("" : "+v"(tr));
        const int jx0 = tr % TCX, y = tr / TCX;
        const bool row_ok = have && y < ny;
        if (!have) pl = 0;
        const T* src = in + pl * (int64_t)ny * nx + (int64_t)(row_ok ? y : 0) * nx;
        if (pairs) {
            const cplx<T>* src2 = reinterpret_cast<const cplx<T>*>(src);
#pragma unroll
            for (int m = 0; m < EL; ++m) {
                const int q = jx0 + TCX * m;
                nxt[m] = (row_ok && 2 * q < nx) ? src2[q] : cplx<T>{T(0), T(0)};
            }
        } else {
#pragma unroll
            for (int m = 0; m < EL; ++m) {
                const int i0 = 2 * (jx0 + TCX * m);
                T a = T(0), b = T(0);
                if (row_ok && i0 < nx) a = src[i0];
                if (row_ok && i0 + 1 < nx) b = src[i0 + 1];
                nxt[m] = {a, b};
            }
        }
    };
    int64_t plane = blockIdx.x;
    load_rows(plane, plane < nplanes);
    for (; plane < nplanes; plane += gridDim.x) {
        int tt = t;
        asm volatile("" : "+v"(tt));
        const int j = tt % TCX, yr = tt / TCX;
        // 1. per row: reals in pairs, length-M transform, split into M+1 outputs
        cplx<T> reg[EX];
#pragma unroll
        for (int m = 0; m < EX; ++m) reg[m] = m < EL ? nxt[m] : cplx<T>{T(0), T(0)};
        const RowPad lay{xld, xsh};
        // the previous plane's column rounds are done with the LDS; from here
        // to the split, each row's TCX threads (consecutive lanes of one wave)
        // work on an LDS row of their own and synchronise within the wave
        __syncthreads();
        fft_regs<T, M, EX, true, HX, true>(reg, lds, lay, yr, j, twl);
        stage_sync<true>();
#pragma unroll
        for (int m = 0; m < EX; ++m) lds[lay(j + TCX * m, yr)] = reg[m];
        stage_sync<true>();
        {
            const T half = T(0.5);
            cplx<T> xs[EX];
#pragma unroll
            for (int m = 0; m < EX; ++m) {
                const int k = j + TCX * m;
                const cplx<T> zk = lds[lay(k, yr)];
                const cplx<T> zm = cconj(lds[lay((M - k) & (M - 1), yr)]);
                const cplx<T> e = cadd(zk, zm);
                const cplx<T> wd = cmul(twl[M + k], csub(zk, zm));      // W_P^k (Z[k] - conj Z[M-k])
                xs[m] = {half * (e.x + wd.y), half * (e.y - wd.x)};     // e/2 - (i/2) wd
            }
            const cplx<T> z0 = lds[lay(0, yr)];
            T zM = z0.x - z0.y;                          // column M
            // The split is finished before the barrier: only its outputs are held across it.
#pragma unroll
            for (int m = 0; m < EX; ++m) asm volatile("" : "+v"(xs[m].x), "+v"(xs[m].y));
            asm volatile("" : "+v"(zM));
            __syncthreads();                             // the row spectra are read: the plane takes their LDS
            if (yr < ny) {
#pragma unroll
                for (int m = 0; m < EX; ++m) {
                    const int k = j + TCX * m;
                    lds[(M - k) * PLD + (yr ^ (k & 15))] = xs[m];
                }
                if (j == 0) lds[0 * PLD + (yr ^ (M & 15))] = cplx<T>{zM, T(0)};
            }
        }
        __syncthreads();

        // 2. forward y of the kx columns (rows >= Ny are zero padding, Ny <= Py/2),
        //    rounds of groups growing into the freed LDS. The twiddles are loaded
        //    once per plane, before the next plane's rows are requested: vector
        //    loads (and stores) complete in issue order, so a twiddle load issued
        //    after the rows or a round's stores would wait for them.
        cplx<T>* dst = out + (plane / zp) * zp * (int64_t)PY * wx + (plane % zp) * wx;   // interleaved planes
        const int64_t rs = (int64_t)zp * wx;
        const int gi = tt / GT, cl = (tt % GT) % GC;
        int jy = (tt % GT) / GC;
        cplx<T> twy[TWY];
        load_tw_stages<T, PY, EY, 1, 0>(twy, jy, tw + (PY - 1));
        load_rows(plane + gridDim.x, plane + gridDim.x < nplanes);
        for (int c0 = 0; c0 < M1;) {
            asm volatile("" : "+v"(jy));  // per round: keeps the twiddles from being held across rounds
            int groups = kYXThreads / GT, ncols = 0;
            for (; groups > 1; --groups) {
                ncols = groups * GC < M1 - c0 ? groups * GC : M1 - c0;
                const int g2 = (ncols + GC - 1) / GC;
                if (g2 * PY * GC <= CAPF - (M1 - c0 - ncols) * PLD) break;
            }
            ncols = groups * GC < M1 - c0 ? groups * GC : M1 - c0;
            groups = (ncols + GC - 1) / GC;
            const bool act = gi < groups;
            const int c = c0 + gi * GC + cl;
            const bool valid = act && c < M1;
            cplx<T> col[1][EY];
#pragma unroll
            for (int m = 0; m < EY; ++m) {
                const int yy = jy + TCY * m;
                col[0][m] = (valid && 2 * m < EY && yy < ny) ? lds[(M - c) * PLD + (yy ^ (c & 15))]
                                                              : cplx<T>{T(0), T(0)};
            }
            cplx<T>* scratch = lds + (M1 - c0 - ncols) * PLD + (act ? gi : 0) * (PY * GC);
            fft_regs_k<T, PY, EY, true, true, 1, TWY>(col, twy, scratch, 0, ColMajor{GC}, cl, jy, act);
            if (valid) {
#pragma unroll
                for (int m = 0; m < EY; ++m) dst[(int64_t)(jy + TCY * m) * rs + c] = col[0][m];
            }
            c0 += ncols;
        }
        // (the next plane's row transforms start with a barrier)
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
                   const cplx<float>* tw, hipStream_t s, int zp) {
    if (nplanes <= 0) return;
    if (!yx_inv_fits(Py, M, ny, 4)) fail(DDSTRESS_E_INVALID, "plane does not fit the fused forward x-y kernel");
    if ((size_t)(Py / 2) * x_lds_layout(M, 16, 4).ld + 2 * (size_t)M > (size_t)kYXLds / sizeof(cplx<float>))
        fail(DDSTRESS_E_INVALID, "row exchanges and twiddle tables exceed the fused forward kernel's LDS");
    if (nplanes > 0x7fffffffLL) fail(DDSTRESS_E_UNSUPPORTED, "grid too large for one launch");
    if (zp < 1 || nplanes % zp != 0) fail(DDSTRESS_E_INVALID, "plane interleave must divide the plane count");
    const XLayout xl = x_lds_layout(M, 16, 4);
    const int pairs = (reinterpret_cast<uintptr_t>(in) % 8 == 0 && nx % 2 == 0) ? 1 : 0;
    // one resident block per CU walks over the planes; rows of nx <= M reals
    // (an open x axis) leave the upper half of the packed row zero
    const int64_t grid = nplanes < kYXBlocks ? nplanes : kYXBlocks;
    if (nx <= M)
        hipLaunchKernelGGL((k_xy_fwd<256, 128, true>), dim3((unsigned)grid), dim3(kYXThreads), kYXLds, s, in, out,
                           nplanes, ny, nx, wx, tw, xl.ld, xl.s, pairs, zp);
    else
        hipLaunchKernelGGL((k_xy_fwd<256, 128, false>), dim3((unsigned)grid), dim3(kYXThreads), kYXLds, s, in, out,
                           nplanes, ny, nx, wx, tw, xl.ld, xl.s, pairs, zp);
    check_hip(hipGetLastError(), "fused forward x-y launch");
}

void launch_yx_inv(const cplx<float>* in, float* out, int64_t nplanes, int Py, int M, int ny, int nx, int64_t wx,
                   const cplx<float>* tw, hipStream_t s, double* rowsq, int zp) {
    if (nplanes <= 0) return;
    if (!yx_inv_fits(Py, M, ny, 4)) fail(DDSTRESS_E_INVALID, "plane does not fit the fused inverse y-x kernel");
    if ((size_t)(Py / 2) * x_lds_layout(M, 16, 4).ld + 2 * (size_t)M > (size_t)kYXLds / sizeof(cplx<float>))
        fail(DDSTRESS_E_INVALID, "row exchanges and twiddle tables exceed the fused inverse kernel's LDS");
    if (nplanes > 0x7fffffffLL) fail(DDSTRESS_E_UNSUPPORTED, "grid too large for one launch");
    if (zp < 1 || nplanes % zp != 0) fail(DDSTRESS_E_INVALID, "plane interleave must divide the plane count");
    const XLayout xl = x_lds_layout(M, 16, 4);
    const int pairs = (reinterpret_cast<uintptr_t>(out) % 8 == 0 && nx % 2 == 0) ? 1 : 0;
    // one resident block per CU walks over the planes
    const int64_t grid = nplanes < kYXBlocks ? nplanes : kYXBlocks;
    hipLaunchKernelGGL((k_yx_inv<256, 128>), dim3((unsigned)grid), dim3(kYXThreads), kYXLds, s, in, out, nplanes, ny,
                       nx, wx, tw, xl.ld, xl.s, pairs, rowsq, zp);
    check_hip(hipGetLastError(), "fused inverse y-x launch");
}

}  // namespace dds
