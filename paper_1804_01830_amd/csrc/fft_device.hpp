// Device-side building blocks of the power-of-two FFTs used by every pass.
//
// One transform of length N is done by Tc = N / E threads. Thread j owns the
// E elements x[j + Tc*m], m = 0..E-1, in registers both before the first
// stage and after the last one (the Stockham autosort ordering keeps that
// distribution), so a forward transform can hand its output straight to an
// inverse transform in registers, and the first stage loads / last stage
// stores go to global memory with consecutive threads on consecutive rows.
// Between stages the data goes through LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace dds {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
// Fused multiply-add. Complex products are written with it explicitly, each
// component one rounded product and one fused multiply-add, so their rounding
// does not depend on which product the compiler would contract in a given
// context: every kernel that forms the same product gets the same bits.
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {fmad(a.x, b.x, -(a.y * b.y)), fmad(a.x, b.y, a.y * b.x)};
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }

// Multiply by the twiddle w (table holds forward values exp(-2 pi i k / N));
// the inverse transform uses its conjugate.
template <bool FWD, typename T>
__device__ __forceinline__ cplx<T> twmul(cplx<T> a, cplx<T> w) {
    if (FWD) return cmul(a, w);
    return {fmad(a.x, w.x, a.y * w.y), fmad(a.y, w.x, -(a.x * w.y))};
}

// Multiply by -i (forward) or +i (inverse).
template <bool FWD, typename T>
__device__ __forceinline__ cplx<T> rot90(cplx<T> a) {
    if (FWD) return {a.y, -a.x};
    return {-a.y, a.x};
}

template <bool FWD, typename T>
__device__ __forceinline__ void dft2(cplx<T>* v) {
    cplx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <bool FWD, typename T>
__device__ __forceinline__ void dft4(cplx<T>* v) {
    cplx<T> t0 = cadd(v[0], v[2]);
    cplx<T> t1 = csub(v[0], v[2]);
    cplx<T> t2 = cadd(v[1], v[3]);
    cplx<T> t3 = rot90<FWD>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, t3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, t3);
}

template <bool FWD, typename T>
__device__ __forceinline__ void dft8(cplx<T>* v) {
    // even/odd split: two length-4 transforms joined with the eighth roots
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<FWD>(e);
    dft4<FWD>(o);
    const T h = T(0.70710678118654752440084436210484904);
    // o1 * w8, o2 * w8^2 = -/+ i, o3 * w8^3, with w8 = (1 -/+ i)/sqrt 2
    cplx<T> o1, o3;
    if (FWD) {
        o1 = {(o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h};
        o3 = {(o[3].y - o[3].x) * h, -(o[3].x + o[3].y) * h};
    } else {
        o1 = {(o[1].x - o[1].y) * h, (o[1].x + o[1].y) * h};
        o3 = {-(o[3].x + o[3].y) * h, (o[3].x - o[3].y) * h};
    }
    cplx<T> o2 = rot90<FWD>(o[2]);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <int R, bool FWD, typename T>
__device__ __forceinline__ void dftR(cplx<T>* v) {
    if constexpr (R == 2) dft2<FWD>(v);
    else if constexpr (R == 4) dft4<FWD>(v);
    else if constexpr (R == 8) dft8<FWD>(v);
}

// Length-R DFTs whose upper inputs v[R/2 .. R-1] are zero (the first stage of
// a transform of zero-padded data); those inputs are never read. Same values
// as the full DFTs above with zeros there.
template <bool FWD, typename T>
__device__ __forceinline__ void dft4_hz(cplx<T>* v) {
    const cplx<T> a = v[0];
    const cplx<T> b = rot90<FWD>(v[1]);
    v[2] = csub(a, v[1]);
    v[0] = cadd(a, v[1]);
    v[1] = cadd(a, b);
    v[3] = csub(a, b);
}

template <bool FWD, typename T>
__device__ __forceinline__ void dft8_hz(cplx<T>* v) {
    cplx<T> e[4] = {v[0], v[2], v[0], v[0]};
    cplx<T> o[4] = {v[1], v[3], v[1], v[1]};
    dft4_hz<FWD>(e);
    dft4_hz<FWD>(o);
    const T h = T(0.70710678118654752440084436210484904);
    cplx<T> o1, o3;
    if (FWD) {
        o1 = {(o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h};
        o3 = {(o[3].y - o[3].x) * h, -(o[3].x + o[3].y) * h};
    } else {
        o1 = {(o[1].x - o[1].y) * h, (o[1].x + o[1].y) * h};
        o3 = {-(o[3].x + o[3].y) * h, (o[3].x - o[3].y) * h};
    }
    cplx<T> o2 = rot90<FWD>(o[2]);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <int R, bool FWD, typename T>
__device__ __forceinline__ void dftR_hz(cplx<T>* v) {
    if constexpr (R == 1) {
    } else if constexpr (R == 2) v[1] = v[0];
    else if constexpr (R == 4) dft4_hz<FWD>(v);
    else if constexpr (R == 8) dft8_hz<FWD>(v);
}

constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Raw buffer loads: a 128-bit resource (base, byte size) kept in scalar
// registers, a per-lane 32-bit byte offset and a wave-uniform byte offset.
// Reads at or beyond the resource's size return zero.
constexpr int kBufferFlags = 0x00020000;   // raw (untyped) dword access on gfx9-family targets

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferFlags);
}

template <typename T>
__device__ __forceinline__ T buf_real(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float buf_real<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_real<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return __hiloint2double((int)v[1], (int)v[0]);
}

template <typename T>
__device__ __forceinline__ cplx<T> buf_cplx(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ cplx<float> buf_cplx<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return {__uint_as_float(v[0]), __uint_as_float(v[1])};
}
template <>
__device__ __forceinline__ cplx<double> buf_cplx<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return {__hiloint2double((int)v[1], (int)v[0]), __hiloint2double((int)v[3], (int)v[2])};
}

// Raw buffer store of one complex value: dropped by the hardware when the
// byte offset lies at or beyond the resource's size.
template <typename T>
__device__ __forceinline__ void buf_store_cplx(__amdgpu_buffer_rsrc_t r, int voff, int soff, cplx<T> v);
template <>
__device__ __forceinline__ void buf_store_cplx<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff, cplx<float> v) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 d = {__float_as_uint(v.x), __float_as_uint(v.y)};
    __builtin_amdgcn_raw_buffer_store_b64(d, r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void buf_store_cplx<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff, cplx<double> v) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const unsigned long long a = (unsigned long long)__double_as_longlong(v.x);
    const unsigned long long b = (unsigned long long)__double_as_longlong(v.y);
    const u4 d = {(unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32)};
    __builtin_amdgcn_raw_buffer_store_b128(d, r, voff, soff, 0);
}

// The hardware hands consecutive workgroups of a launch to the eight XCDs in
// turn, and each XCD has its own L2. Logical block index of workgroup b of nb
// such that every XCD works through one contiguous range of logical blocks
// (neighbouring column tiles, which share cache lines, then meet in one L2).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int X = 8;
    const int q = nb / X, r = nb % X;
    const int x = b % X, i = b / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// LDS addressing of element i of transform (column / row) c.
struct ColMajor {      // element i of column c at i*ld + c (tiles of consecutive columns)
    int ld;
    __device__ __forceinline__ int operator()(int i, int c) const { return i * ld + c; }
};
struct RowPad {        // element i of row r at r*ld + i + (i >> s): one pad element every 2^s
    int ld, s;
    __device__ __forceinline__ int operator()(int i, int r) const { return r * ld + i + (i >> s); }
};

// Synchronisation between the stages of a transform. A transform whose
// threads (and LDS region) all belong to one wave needs no workgroup barrier:
// the LDS executes one wave's instructions in order, so its writes are seen by
// its later reads; only the compiler must keep them in order (WAVE). Other
// transforms take a workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void stage_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One radix-R Stockham stage. Butterfly b = j + Tc*q (q < E/R) reads
// x[b + r N/R], multiplies by exp(-/+ 2 pi i (b mod Ns) r / (Ns R)), applies
// the length-R DFT and writes (b / Ns) Ns R + (b mod Ns) + r Ns.
// HZ: elements N/2 .. N-1 of the input are zero (zero padding); the first
// stage then never reads them (same values).
template <typename T, int N, int E, bool FWD, int Ns, int R, bool HZ, bool WAVE, class Lay>
__device__ __forceinline__ void fft_stage(cplx<T> (&reg)[E], cplx<T>* lds, Lay lay, int c, int j,
                                          const cplx<T>* __restrict__ tw, bool act) {
    constexpr int Tc = N / E;
    constexpr int NB = E / R;
    constexpr bool first = (Ns == 1);
    constexpr bool last = (Ns * R == N);
    cplx<T> v[NB][R];
    if constexpr (first) {
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = reg[q + r * NB];
    } else {
        stage_sync<WAVE>();
        if (act) {
#pragma unroll
            for (int q = 0; q < NB; ++q)
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = lds[lay(j + Tc * q + r * (N / R), c)];
        }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if constexpr (!first) {
            const int k = (j + Tc * q) & (Ns - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) v[q][r] = twmul<FWD>(v[q][r], tw[k * r * (N / (Ns * R))]);
        }
        if constexpr (first && HZ)
            dftR_hz<R, FWD>(v[q]);
        else
            dftR<R, FWD>(v[q]);
    }
    if constexpr (last) {
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) reg[q + r * NB] = v[q][r];
    } else {
        stage_sync<WAVE>();   // every thread has read its inputs (or the buffer's previous user is done)
        if (act) {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int b = j + Tc * q;
                const int base = (b / Ns) * Ns * R + (b & (Ns - 1));
#pragma unroll
                for (int r = 0; r < R; ++r) lds[lay(base + r * Ns, c)] = v[q][r];
            }
        }
    }
}

template <typename T, int N, int E, bool FWD, int Ns, bool HZ, bool WAVE, class Lay>
__device__ __forceinline__ void fft_stages(cplx<T> (&reg)[E], cplx<T>* lds, Lay lay, int c, int j,
                                           const cplx<T>* __restrict__ tw, bool act) {
    if constexpr (Ns < N) {
        constexpr int R = cmin(cmin(8, E), N / Ns);
        fft_stage<T, N, E, FWD, Ns, R, HZ, WAVE>(reg, lds, lay, c, j, tw, act);
        fft_stages<T, N, E, FWD, Ns * R, HZ, WAVE>(reg, lds, lay, c, j, tw, act);
    }
}

// Twiddles of every stage after the first, for the butterflies one thread
// owns: their count and a load (once); fftk_stage takes them from registers.
// A kernel that runs many transforms of one length keeps them for all of
// them (the inverse uses their conjugates).
constexpr int tw_count(int N, int E, int Ns = 1) {
    return Ns >= N ? 0
                   : (Ns == 1 ? 0 : (E / cmin(cmin(8, E), N / Ns)) * (cmin(cmin(8, E), N / Ns) - 1)) +
                         tw_count(N, E, Ns * cmin(cmin(8, E), N / Ns));
}

template <typename T, int N, int E, int Ns, int K, int TWC>
__device__ __forceinline__ void load_tw_stages(cplx<T> (&w)[TWC], int j, const cplx<T>* __restrict__ tw) {
    if constexpr (Ns < N) {
        constexpr int R = cmin(cmin(8, E), N / Ns);
        constexpr int Tc = N / E;
        constexpr int NB = E / R;
        if constexpr (Ns > 1) {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int k = (j + Tc * q) & (Ns - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) w[K + q * (R - 1) + r - 1] = tw[k * r * (N / (Ns * R))];
            }
            load_tw_stages<T, N, E, Ns * R, K + NB * (R - 1)>(w, j, tw);
        } else {
            load_tw_stages<T, N, E, Ns * R, K>(w, j, tw);
        }
    }
}

// K transforms of length N taken through the stages together, with the
// twiddles in registers (see load_tw_stages): one barrier before the reads and
// one before the writes of each stage serve all K, whose exchanges use the LDS
// regions lds + k * region. HZ: inputs m >= E/2 of every transform are zero
// (zero-padded data) and are not read. Threads with act == false (whole
// waves) take part in the barriers without touching LDS or computing.
template <typename T, int N, int E, bool FWD, bool HZ, int Ns, int R, int KT, int K, int TWC, bool WAVE, class Lay>
__device__ __forceinline__ void fftk_stage(cplx<T> (&reg)[K][E], const cplx<T> (&w)[TWC], cplx<T>* lds, int region,
                                           Lay lay, int c, int j, bool act) {
    constexpr int Tc = N / E;
    constexpr int NB = E / R;
    constexpr bool first = (Ns == 1);
    constexpr bool last = (Ns * R == N);
    cplx<T> v[K][NB][R];
    if constexpr (first) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < NB; ++q)
#pragma unroll
                for (int r = 0; r < (HZ ? (R + 1) / 2 : R); ++r) v[k][q][r] = reg[k][q + r * NB];
    } else {
        stage_sync<WAVE>();
        if (act) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int q = 0; q < NB; ++q)
#pragma unroll
                    for (int r = 0; r < R; ++r) v[k][q][r] = lds[k * region + lay(j + Tc * q + r * (N / R), c)];
        }
    }
    if (act) {          // idle waves skip the arithmetic too
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if constexpr (!first) {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[k][q][r] = twmul<FWD>(v[k][q][r], w[KT + q * (R - 1) + r - 1]);
                }
                if constexpr (first && HZ) dftR_hz<R, FWD>(v[k][q]);
                else dftR<R, FWD>(v[k][q]);
            }
    }
    if constexpr (last) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < NB; ++q)
#pragma unroll
                for (int r = 0; r < R; ++r) reg[k][q + r * NB] = v[k][q][r];
    } else {
        stage_sync<WAVE>();
        if (act) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    const int b = j + Tc * q;
                    const int base = (b / Ns) * Ns * R + (b & (Ns - 1));
#pragma unroll
                    for (int r = 0; r < R; ++r) lds[k * region + lay(base + r * Ns, c)] = v[k][q][r];
                }
        }
    }
}

template <typename T, int N, int E, bool FWD, bool HZ, int Ns, int KT, int K, int TWC, bool WAVE, class Lay>
__device__ __forceinline__ void fftk_stages(cplx<T> (&reg)[K][E], const cplx<T> (&w)[TWC], cplx<T>* lds, int region,
                                            Lay lay, int c, int j, bool act) {
    if constexpr (Ns < N) {
        constexpr int R = cmin(cmin(8, E), N / Ns);
        fftk_stage<T, N, E, FWD, HZ, Ns, R, KT, K, TWC, WAVE>(reg, w, lds, region, lay, c, j, act);
        fftk_stages<T, N, E, FWD, HZ, Ns * R, (Ns == 1 ? KT : KT + (E / R) * (R - 1)), K, TWC, WAVE>(
            reg, w, lds, region, lay, c, j, act);
    }
}

// WAVE: as for fft_regs, the threads and LDS regions of these transforms
// belong to one wave, whose stages then synchronise within the wave.
template <typename T, int N, int E, bool FWD, bool HZ, int K, int TWC, bool WAVE = false, class Lay>
__device__ __forceinline__ void fft_regs_k(cplx<T> (&reg)[K][E], const cplx<T> (&w)[TWC], cplx<T>* lds, int region,
                                           Lay lay, int c, int j, bool act = true) {
    static_assert(N % E == 0, "E must divide N");
    fftk_stages<T, N, E, FWD, HZ, 1, 0, K, TWC, WAVE>(reg, w, lds, region, lay, c, j, act);
}

// Full transform of length N on the register distribution described above.
// `tw` points at the table of exp(-2 pi i k / N), k < N. Every thread of the
// block must call it (it contains barriers when N > E); threads with act ==
// false (whole waves) take part in the barriers without touching LDS. With
// HZ the upper half of the input is zero padding and its registers are not read.
// WAVE: the N/E threads of each transform are consecutive lanes of one wave
// and its LDS region is touched by no other wave, so the stages synchronise
// within the wave only (see stage_sync).
template <typename T, int N, int E, bool FWD, bool HZ = false, bool WAVE = false, class Lay>
__device__ __forceinline__ void fft_regs(cplx<T> (&reg)[E], cplx<T>* lds, Lay lay, int c, int j,
                                         const cplx<T>* __restrict__ tw, bool act = true) {
    static_assert(N % E == 0, "E must divide N");
    static_assert(!HZ || E >= 2, "a zero upper half needs two elements per thread");
    static_assert(!WAVE || (N / E <= 64 && 64 % (N / E) == 0), "a wave-local transform fits one wave");
    fft_stages<T, N, E, FWD, 1, HZ, WAVE>(reg, lds, lay, c, j, tw, act);
}

}  // namespace dds
