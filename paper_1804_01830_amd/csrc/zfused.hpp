// Fused z kernels (single-group and grouped forms) and their launch
// dispatch. Each form and precision is instantiated in a unit of its own
// (z_serial_f32.hip, ...), so the many template instances compile in parallel.
#pragma once

#include "ddstress_internal.hpp"

namespace dds {

// Logical block -> (kx tile, ky), P (even) rows of nt tiles: row 0, then for
// q = 1 .. P/2 - 1 the tiles of rows q and P - q interleaved (tile t of row q,
// tile t of row P - q, tile t + 1 of row q, ...), then row P/2. Rows ky and
// P - ky read the same stored spectrum tile when the y mirror applies; as
// neighbouring blocks (on one XCD, by xcd_block) the second read finds it in
// L2 instead of HBM. A bijection onto [0, nt) x [0, P).
__device__ __forceinline__ void z_block_coords(int blk, int nt, int P, int& tile, int& ky) {
    if (blk < nt || P < 4) {            // row 0 (P = 2: rows 0 and 1, no pairs)
        tile = blk % nt;
        ky = blk / nt;
        return;
    }
    const int b = blk - nt;
    const int paired = (P / 2 - 1) * 2 * nt;
    if (b < paired) {
        const int q = b / (2 * nt) + 1, w = b % (2 * nt);
        tile = w >> 1;
        ky = (w & 1) ? P - q : q;
    } else {
        tile = b - paired;
        ky = P / 2;
    }
}

// The last kx column, kx = M = Px/2 (the Nyquist column of the real-to-complex
// x spectra), is Hermitian along y because the stress is real: at every z its
// values at ky and Py - ky are complex conjugates. The block at 0 < ky < Py/2
// writes both; at ky > Py/2 that column is not written, and a block whose tile
// holds column M alone (tile * tk == M) does no work there.
struct NyquistRole {
    bool skip_block;    // the whole block has nothing to write
    bool own;           // this lane writes its column at ky
    bool mirror;        // this lane also writes the conjugate at Py - ky
};
__device__ __forceinline__ NyquistRole nyquist_role(int tile, int tk, int col, int ky, bool valid, const ZGeom& g) {
    const int m = g.ncols - 1;
    const bool nyq = valid && col == m;
    const bool upper = 2 * ky > g.nky;
    return {tile * tk == m && upper, valid && !(nyq && upper), nyq && ky > 0 && 2 * ky < g.nky};
}

// Roles of a block of the fused z pass and of its lane in column slot c of
// the tile: the spectrum tile and stored row it reads, the element offsets of
// its input and output columns, and its realisations [b0, b1). With a Nyquist
// strip (g.nyq groups, see z_nyq_groups) the last tile is the strip, whose
// blocks hold the column kx = M at ky = q tk + c for group q. A strip lane
// reads and writes its own row (one cache line per value, against one per
// tk values elsewhere), so each strip block takes one realisation: blocks
// q B + b come first, short, and never form the launch's tail. The following
// blocks take the other kx tiles by z_block_coords and every realisation.
//
// Logical block of this workgroup: the strip's blocks are the first
// workgroups, which the hardware deals to the eight XCDs in turn (so each
// XCD gets its share of them); the others go through xcd_block, which gives
// every XCD a contiguous range of the remaining tiles.
__device__ __forceinline__ int z_logical_block(const ZGeom& g) {
    const int b = (int)blockIdx.x, strip = g.nyq * g.B;
    return b < strip ? b : strip + xcd_block(b - strip, (int)gridDim.x - strip);
}
struct ZRoles {
    int tile, kyc;        // spectrum tile and stored row
    bool flip_y;          // row kyc is the y mirror of the block's ky (odd planes change sign)
    int64_t in0;          // offset of the block's first input column in a density plane
    int lane_in;          // offset of this lane's column from in0 (lanes without data: 0, a valid column)
    int64_t own, mir;     // offsets of this lane's output column at its ky and at Py - ky
    int64_t own0;         // the block's first own output column (own = own0 + lane_out)
    int lane_out;
    uint32_t in_bytes;    // bytes from in0, and from own0, to the end of a density / stress plane
    uint32_t out_bytes;
    int b0, b1;           // realisations of the block
    NyquistRole nq;
};
template <typename T>
__device__ __forceinline__ ZRoles z_roles(int blk, int tk, int c, const ZGeom& g) {
    ZRoles r;
    const int tiles = g.nyq > 0 ? g.ntiles - 1 : g.ntiles;
    const int strip_blocks = g.nyq * g.B;
    if (blk < strip_blocks) {                    // the Nyquist strip
        const int q = blk / g.B, m = g.ncols - 1;
        r.b0 = blk - q * g.B;
        r.b1 = r.b0 + 1;
        const int ky = q * tk + c;
        const bool valid = 2 * ky <= g.nky;
        const int kyv = valid ? ky : q * tk;
        r.tile = g.ntiles - 1;
        r.kyc = q;
        r.flip_y = false;
        r.in0 = (int64_t)q * tk * g.ios + m;
        r.lane_in = valid ? c * (int)g.ios : 0;
        r.own = (int64_t)kyv * g.oos + m;
        r.mir = (int64_t)(g.nky - kyv) * g.oos + m;
        r.own0 = (int64_t)q * tk * g.oos + m;
        r.lane_out = (kyv - q * tk) * (int)g.oos;
        r.in_bytes = (uint32_t)((g.iqs - r.in0) * (int64_t)sizeof(cplx<T>));
        r.out_bytes = (uint32_t)((g.oqs - r.own0) * (int64_t)sizeof(cplx<T>));
        r.nq = {false, valid, valid && ky > 0 && 2 * ky < g.nky};
        return r;
    }
    int tile, ky;
    z_block_coords(blk - strip_blocks, tiles, g.nky, tile, ky);
    const int col = tile * tk + c;
    const bool valid = col < g.ncols;
    const int colc = valid ? col : 0;
    r.b0 = 0;
    r.b1 = g.B;
    r.tile = tile;
    r.flip_y = g.nky_s < g.nky && 2 * ky > g.nky;
    r.kyc = r.flip_y ? g.nky - ky : ky;
    r.in0 = (int64_t)ky * g.ios + (int64_t)tile * tk;
    r.lane_in = valid ? c : 0;
    r.own = (int64_t)ky * g.oos + colc;
    r.mir = (int64_t)(g.nky - ky) * g.oos + colc;
    r.own0 = (int64_t)ky * g.oos + (int64_t)tile * tk;
    r.lane_out = valid ? c : 0;
    r.in_bytes = (uint32_t)((g.iqs - r.in0) * (int64_t)sizeof(cplx<T>));
    r.out_bytes = (uint32_t)((g.oqs - r.own0) * (int64_t)sizeof(cplx<T>));
    r.nq = nyquist_role(tile, tk, col, ky, valid, g);
    return r;
}

// Byte offsets of a lane's rows z = j + Tc m (m < EH) at row stride rs from
// its block's base, the lane's column at `lane` elements: rows z >= nz, and
// every row when `on` is false, take the resource's size `end` as offset, so
// their loads read zero and their stores are dropped (the row part Tc m rs
// is added as the wave-uniform offset, which keeps them beyond it).
template <typename T, int EH>
__device__ __forceinline__ void row_offsets(int (&off)[EH], bool on, int j, int Tc, int lane, int rs, int nz,
                                            uint32_t end) {
#pragma unroll
    for (int m = 0; m < EH; ++m)
        off[m] = (on && j + Tc * m < nz) ? (j * rs + lane) * (int)sizeof(cplx<T>) : (int)end;
}

// Sign flip of x when the (wave-uniform) mask holds the sign bit: one integer
// operation in place of a select and a product with -1 (the same bits).
__device__ __forceinline__ float flip_sign(float x, uint32_t msk) { return __uint_as_float(__float_as_uint(x) ^ msk); }
__device__ __forceinline__ double flip_sign(double x, uint32_t msk) {
    return __longlong_as_double(__double_as_longlong(x) ^ (long long)((uint64_t)msk << 32));
}
__device__ __forceinline__ uint32_t sign_mask(bool neg) { return neg ? 0x80000000u : 0u; }

// Copy a block's spectrum tile [c][v][kz][TK] (nkz rows kz, NC channels,
// six components) into LDS as rows kz of [c][v][TK] values with the row
// stride (6 NC + 1) TK, applying the y-mirror sign of the odd planes (bit
// c 6 + v of sgn_y) when flip_y. NT threads (tid < NT) copy 16-byte pieces,
// up to CH loads each in flight before their stores; a piece never straddles
// a source row (TK is a multiple of its width). The caller synchronises.
template <typename T, int NC, int TK, int NT, int CH = 16>
__device__ __forceinline__ void stage_spectrum_tile(T* s_l, __amdgpu_buffer_rsrc_t srs, int nkz, bool flip_y,
                                                    uint64_t sgn_y, int tid) {
    constexpr int KS = (6 * NC + 1) * TK;
    constexpr int VW = 16 / (int)sizeof(T);
    const int n_vals = NC * 6 * nkz * TK;
    const float rcp = 1.0f / (float)nkz;
    for (int k0 = 0; k0 * NT * VW < n_vals; k0 += CH) {
        uint4 piece[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k)
            piece[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(srs, (tid + (k0 + k) * NT) * 16,
                                                                                    0, 0));
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int i = (tid + (k0 + k) * NT) * VW;    // first value of the piece
            if (i < n_vals) {
                const int r = i / TK, cc = i % TK;
                int cv = (int)((float)r * rcp);
                if (cv * nkz > r) --cv;
                if ((cv + 1) * nkz <= r) ++cv;
                const int kz = r - cv * nkz;
                const bool neg = flip_y && ((sgn_y >> cv) & 1);      // cv = c 6 + v
                uint4 q = piece[k];
                if (neg) {                                              // flip the sign bits
                    if constexpr (sizeof(T) == 4) {
                        q.x ^= 0x80000000u; q.y ^= 0x80000000u; q.z ^= 0x80000000u; q.w ^= 0x80000000u;
                    } else {
                        q.y ^= 0x80000000u; q.w ^= 0x80000000u;
                    }
                }
                *reinterpret_cast<uint4*>(s_l + kz * KS + cv * TK + cc) = q;
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Fused z pass, single-group form. A block owns `tk` consecutive kx columns at
// one ky (in the Nyquist strip: the column kx = M at tk consecutive ky, see
// z_roles) and one group of Tc * tk threads. For every realisation b it
// transforms the C density columns along z one after the other (rows
// z >= N/2 are the zero padding and are not loaded), accumulates the six
// stress spectra
//     sigma^_v(k) = sum_c i S_{v,c}(k) rho^_c(k)      (K^ = i S, K odd)
// in registers, summing the channels in increasing order (the same arithmetic
// as the grouped form), and transforms each back along z, writing rows
// z < nz. The density column of the next channel (or of the next
// realisation's first channel) is requested before the current transform, so
// its latency overlaps the FFT work.
//
// TK > 0 fixes the tile width at compile time: the block then copies its
// spectrum tile once into LDS, as rows kz of [c][v][TK] values with a row
// stride of (6C + 1) TK (the odd multiple of TK puts the rows a wave reads on
// distinct banks), with the y-mirror sign applied, and every realisation reads
// it there; all LDS offsets are immediates. TK = 0 takes the width at run time
// and reads the spectrum from memory for each realisation. Fewer threads per
// column than the grouped form: better for few realisations.
// ----------------------------------------------------------------------------
template <typename T, int N, int E, int NC, int TK>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TK > 0 && NC == 3 ? 3 : 1))) k_z_serial(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                  const T* __restrict__ spec, ZGeom g,
                                                  const cplx<T>* __restrict__ tw, int tk_arg, int ld_arg) {
    constexpr int Tc = N / E;
    constexpr int EH = (E + 1) / 2;        // elements that can hold data rows (z < N/2)
    constexpr bool HZ = N > 1;             // the upper half of every input column is padding
    constexpr bool SL = TK > 0;            // spectrum staged in LDS
    constexpr int KS = (6 * NC + 1) * (TK > 0 ? TK : 1);   // staged row stride (values)
    const int tk = SL ? TK : tk_arg;
    const int ld = SL ? TK : ld_arg;
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int c = threadIdx.x % tk;
    const int j = threadIdx.x / tk;
    const int blk = z_logical_block(g);
    const ZRoles ro = z_roles<T>(blk, tk, c, g);
    const NyquistRole nq = ro.nq;
    if (nq.skip_block) return;                   // uniform over the block, before any barrier
    const ColMajor lay{ld};
    const int ors = (int)g.ors;
    // Spectrum tile of this block: [c][v][kzc][tk] at row kyc. With a y mirror
    // only ky <= Py/2 is stored and row Py - ky stands in for ky > Py/2; with
    // a z mirror only kz <= N/2 is stored and elements m >= E/2 read
    // kz' = N - kz = (Tc - j) + Tc (E - 1 - m). Odd planes change sign.
    const bool flip_y = ro.flip_y;
    const bool zc = g.nkz_s < N;
    const int nkz = g.nkz_s;
    const T* sp = spec + ((int64_t)ro.kyc * g.ntiles + ro.tile) * (int64_t)g.C * 6 * nkz * tk;
    const __amdgpu_buffer_rsrc_t srs = make_rsrc(sp, (uint32_t)((size_t)g.C * 6 * nkz * tk * sizeof(T)));
    const int s_lane = (j * tk + c) * (int)sizeof(T);
    const int s_lane_m = ((Tc - j) * tk + c) * (int)sizeof(T);
    // density rows z < nz of the block's columns (rows >= nz read zero; lanes
    // without data read a valid column)
    const cplx<T>* in_b = in + ro.in0;
    int r_off[EH];
    row_offsets<T, EH>(r_off, true, j, Tc, ro.lane_in, (int)g.irs, g.nz, ro.in_bytes);
    const int r_step = Tc * (int)g.irs * (int)sizeof(cplx<T>);
    cplx<T>* mir_b = out + ro.mir;
    // own stores: rows z < nz of the lane's output column (lanes without an
    // own column store nothing)
    const cplx<T>* out_b = out + ro.own0;
    int o_off[EH];
    row_offsets<T, EH>(o_off, nq.own, j, Tc, ro.lane_out, ors, g.nz, ro.out_bytes);
    const int o_step = Tc * ors * (int)sizeof(cplx<T>);

#define DDS_LOAD_RHO(DST, BB, CH)                                                          \
    {                                                                                      \
        const __amdgpu_buffer_rsrc_t rr_ = make_rsrc(in_b + (int64_t)((BB) * g.C + (CH)) * g.iqs, ro.in_bytes); \
        _Pragma("unroll") for (int m = 0; m < EH; ++m) DST[0][m] = buf_cplx<T>(rr_, r_off[m], m * r_step); \
    }
    cplx<T> cur[1][E], nxt[1][E];
    DDS_LOAD_RHO(cur, ro.b0, 0)
    constexpr int TWC = tw_count(N, E) > 0 ? tw_count(N, E) : 1;
    cplx<T> twr[TWC];
    load_tw_stages<T, N, E, 1, 0, TWC>(twr, j, tw + (N - 1));

    T* s_l = reinterpret_cast<T*>(smem_raw + (size_t)N * ld * sizeof(cplx<T>));
    // Staged row of each element: kz = j + Tc m, or with a z mirror, for the
    // upper half, its mirror row (Tc - j) + Tc (E - 1 - m). The mirror choice is
    // made once per element and hidden from the optimiser: left visible, it
    // became one selected address per element and read (about 70 registers held
    // across the realisations, which spilled) instead of an immediate offset.
    int s_row[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        s_row[m] = j * KS + c + Tc * m * KS;
        if (2 * m >= E) {
            s_row[m] = zc ? (Tc - j) * KS + c + Tc * (E - 1 - m) * KS : s_row[m];
            asm volatile("" : "+v"(s_row[m]));
        }
    }
    if constexpr (SL) {
        stage_spectrum_tile<T, NC, TK, TK * Tc>(s_l, srs, nkz, flip_y, g.sgn_y, (int)threadIdx.x);
        __syncthreads();
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
// Staged values: element m of this lane reads row offset s_row[m] (mirrored
// or not) plus an immediate per (channel, component).
#define DDS_LOAD_SPEC_SL(DST, CH)                                                          \
    {                                                                                      \
        _Pragma("unroll") for (int v = 0; v < 6; ++v)                                      \
            _Pragma("unroll") for (int m = 0; m < E; ++m)                                  \
                DST[v][m] = s_l[s_row[m] + ((CH) * 6 + v) * TK];                           \
    }

    T sv[6][E];
    if constexpr (!SL) DDS_LOAD_SPEC(sv, 0)
    for (int b = ro.b0; b < ro.b1; ++b) {
        cplx<T> acc[6][1][E];
#pragma unroll
        for (int v = 0; v < 6; ++v)
#pragma unroll
            for (int m = 0; m < E; ++m) acc[v][0][m] = {T(0), T(0)};
        // channels in groups of three (one line direction): unrolled inside a
        // group, a runtime loop over the groups
        for (int l = 0; l < NC / 3; ++l) {
#pragma unroll
            for (int gq = 0; gq < 3; ++gq) {
                const int ch = 3 * l + gq;
                const bool more = gq < 2 || l + 1 < NC / 3;
                if (more) DDS_LOAD_RHO(nxt, b, ch + 1)
                fft_regs_k<T, N, E, true, HZ, 1>(cur, twr, lds, 0, lay, c, j);
                // staged values are read from LDS here, after the transform (they
                // need no registers while it runs); values from memory were
                // requested before it
                if constexpr (SL) DDS_LOAD_SPEC_SL(sv, ch)
#pragma unroll
                for (int v = 0; v < 6; ++v) {
                    // signs of mirrored spectrum rows (wave-uniform); staged
                    // values already carry the y sign
                    const int bit = ch * 6 + v;
                    T sval[E];
                    if constexpr (SL) {
                        // staged values carry the y sign: the z sign of the upper elements
                        const uint32_t mz = sign_mask(zc && ((g.sgn_z >> bit) & 1));
#pragma unroll
                        for (int m = 0; m < E; ++m) sval[m] = 2 * m < E ? sv[v][m] : flip_sign(sv[v][m], mz);
                    } else {
                        const T sy = (flip_y && ((g.sgn_y >> bit) & 1)) ? T(-1) : T(1);
                        const T sz = ((g.sgn_z >> bit) & 1) ? -sy : sy;
#pragma unroll
                        for (int m = 0; m < E; ++m) sval[m] = ((zc && 2 * m >= E) ? sz : sy) * sv[v][m];
                    }
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        acc[v][0][m].x -= sval[m] * cur[0][m].y;
                        acc[v][0][m].y += sval[m] * cur[0][m].x;
                    }
                }
                if (more) {
                    if constexpr (!SL) DDS_LOAD_SPEC(sv, ch + 1)
#pragma unroll
                    for (int m = 0; m < EH; ++m) cur[0][m] = nxt[0][m];
                }
            }
        }
        if (b + 1 < ro.b1) {    // first channel of the next realisation
            DDS_LOAD_RHO(cur, b + 1, 0)
            if constexpr (!SL) DDS_LOAD_SPEC(sv, 0)
        }
#undef DDS_LOAD_RHO
#undef DDS_LOAD_SPEC
#undef DDS_LOAD_SPEC_SL
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            fft_regs_k<T, N, E, false, false, 1>(acc[v], twr, lds, 0, lay, c, j);
            if constexpr (SL) {
                const __amdgpu_buffer_rsrc_t orr = make_rsrc(out_b + (int64_t)(b * 6 + v) * g.oqs, ro.out_bytes);
#pragma unroll
                for (int m = 0; m < EH; ++m) buf_store_cplx<T>(orr, o_off[m], m * o_step, acc[v][0][m]);
            } else if (nq.own) {
                // (the unstaged form is short of scalar registers: plain stores)
                cplx<T>* dst = out + ro.own + (int64_t)(b * 6 + v) * g.oqs;
#pragma unroll
                for (int m = 0; m < EH; ++m) {
                    const int z = j + Tc * m;
                    if (z < g.nz) dst[z * ors] = acc[v][0][m];
                }
            }
            if (nq.mirror) {
                cplx<T>* dst = mir_b + (int64_t)(b * 6 + v) * g.oqs;
#pragma unroll
                for (int m = 0; m < EH; ++m) {
                    const int z = j + Tc * m;
                    if (z < g.nz) dst[z * ors] = cconj(acc[v][0][m]);
                }
            }
        }
    }
}


// ----------------------------------------------------------------------------
// Fused z pass, wave form (FP32, z length 64, 8 elements per thread). A block
// owns TK = 8 consecutive kx columns at one ky (or a group of the Nyquist
// strip, see z_roles), stages their spectrum tile in
// LDS once (as the single-group form does) and runs WPB waves; wave w
// evaluates realisations b = w, w + WPB, ... on its own. Its 64 lanes hold the
// 8 columns with 8 lanes each (lane = 8 j + c: rows j + 8 m of column c), so
// a wave load or store covers 8 rows of 64 contiguous bytes, and every
// transform's lanes are in the wave: the stages exchange through a
// wave-private LDS region and synchronise within the wave (no workgroup
// barrier after the staging). Per realisation the C density columns are
// transformed along z (rows z >= N/2 are padding and are not loaded) and kept
// in registers; then for each stress component
//     sigma^_v(k) = sum_c i S_{v,c}(k) rho^_c(k)      (K^ = i S, K odd),
// summed over c in increasing order, is transformed back along z and rows
// z < nz are written. The next realisation's density is requested before the
// inverse transforms. The radix sequence (8, 8) differs from the other forms'
// (4, 4, 4), so results agree with them to rounding, not bit for bit.
// ----------------------------------------------------------------------------
template <typename T, int N, int E, int NC, int WPB>
__global__ void __launch_bounds__(64 * WPB) k_z_wave(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                     const T* __restrict__ spec, ZGeom g,
                                                     const cplx<T>* __restrict__ tw) {
    constexpr int TK = kZWaveTile;
    constexpr int Tc = N / E;
    static_assert(Tc * TK == 64, "the tile's columns fill one wave");
    constexpr int EH = (E + 1) / 2;        // elements that can hold data rows (z < N/2)
    constexpr bool HZ = true;              // the upper half of every input column is padding
    constexpr int KS = (6 * NC + 1) * TK;  // staged row stride (values)
    extern __shared__ unsigned char smem_raw[];
    // the wave index is uniform over the wave: kept in a scalar register, the
    // realisations (and the buffer resources of their planes) are too
    const int lane = (int)threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int c = lane % TK, j = lane / TK;
    const int blk = z_logical_block(g);
    const ZRoles ro = z_roles<T>(blk, TK, c, g);
    const NyquistRole nq = ro.nq;
    if (nq.skip_block) return;                   // uniform over the block, before any barrier
    const int ors = (int)g.ors;
    // spectrum tile (see the single-group form): rows kyc, mirrored rows signed
    const bool flip_y = ro.flip_y;
    const bool zc = g.nkz_s < N;
    const int nkz = g.nkz_s;
    const T* sp = spec + ((int64_t)ro.kyc * g.ntiles + ro.tile) * (int64_t)g.C * 6 * nkz * TK;
    const __amdgpu_buffer_rsrc_t srs = make_rsrc(sp, (uint32_t)((size_t)g.C * 6 * nkz * TK * sizeof(T)));
    T* s_l = reinterpret_cast<T*>(smem_raw);
    const size_t stage_bytes = ((size_t)nkz * KS * sizeof(T) + 15) / 16 * 16;
    cplx<T>* xw = reinterpret_cast<cplx<T>*>(smem_raw + stage_bytes) + w * (N * TK);    // this wave's exchanges
    const ColMajor lay{TK};
    // density rows z < nz (rows >= nz read zero; lanes without data read a
    // valid column)
    const cplx<T>* in_b = in + ro.in0;
    int r_off[EH];
    row_offsets<T, EH>(r_off, true, j, Tc, ro.lane_in, (int)g.irs, g.nz, ro.in_bytes);
    const int r_step = Tc * (int)g.irs * (int)sizeof(cplx<T>);
    cplx<T>* out_b = out + ro.own;
    cplx<T>* mir_b = out + ro.mir;

    cplx<T> nxt[NC][EH];
    auto load_rho = [&](int b) {
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
            const __amdgpu_buffer_rsrc_t rr = make_rsrc(in_b + (int64_t)(b * g.C + ch) * g.iqs, ro.in_bytes);
#pragma unroll
            for (int m = 0; m < EH; ++m) nxt[ch][m] = buf_cplx<T>(rr, r_off[m], m * r_step);
        }
    };
    if (ro.b0 + w < ro.b1) load_rho(ro.b0 + w);
    constexpr int TWC = tw_count(N, E) > 0 ? tw_count(N, E) : 1;
    cplx<T> twr[TWC];
    load_tw_stages<T, N, E, 1, 0, TWC>(twr, j, tw + (N - 1));
    // staged row of each element (see the single-group form)
    int s_row[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        s_row[m] = j * KS + c + Tc * m * KS;
        if (2 * m >= E) {
            s_row[m] = zc ? (Tc - j) * KS + c + Tc * (E - 1 - m) * KS : s_row[m];
            asm volatile("" : "+v"(s_row[m]));
        }
    }
    stage_spectrum_tile<T, NC, TK, 64 * WPB>(s_l, srs, nkz, flip_y, g.sgn_y, (int)threadIdx.x);
    __syncthreads();

    for (int b = ro.b0 + w; b < ro.b1; b += WPB) {
        cplx<T> rho[NC][1][E];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
#pragma unroll
            for (int m = 0; m < EH; ++m) rho[ch][0][m] = nxt[ch][m];
            fft_regs_k<T, N, E, true, HZ, 1, TWC, true>(rho[ch], twr, xw, 0, lay, c, j);
        }
        if (b + WPB < ro.b1) load_rho(b + WPB);
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            cplx<T> acc[1][E];
#pragma unroll
            for (int m = 0; m < E; ++m) acc[0][m] = {T(0), T(0)};
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) {
                const uint32_t mz = sign_mask(zc && ((g.sgn_z >> (ch * 6 + v)) & 1));   // staged values carry the y sign
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const T sv = s_l[s_row[m] + (ch * 6 + v) * TK];
                    const T sval = 2 * m >= E ? flip_sign(sv, mz) : sv;
                    acc[0][m].x -= sval * rho[ch][0][m].y;
                    acc[0][m].y += sval * rho[ch][0][m].x;
                }
            }
            fft_regs_k<T, N, E, false, false, 1, TWC, true>(acc, twr, xw, 0, lay, c, j);
            if (nq.own) {
                cplx<T>* dst = out_b + (int64_t)(b * 6 + v) * g.oqs;
#pragma unroll
                for (int m = 0; m < EH; ++m) {
                    const int z = j + Tc * m;
                    if (z < g.nz) dst[z * ors] = acc[0][m];
                }
            }
            if (nq.mirror) {
                cplx<T>* dst = mir_b + (int64_t)(b * 6 + v) * g.oqs;
#pragma unroll
                for (int m = 0; m < EH; ++m) {
                    const int z = j + Tc * m;
                    if (z < g.nz) dst[z * ors] = cconj(acc[0][m]);
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Fused z pass, grouped form. A block owns `tk` consecutive kx columns at one
// ky (or a group of the Nyquist strip, see z_roles) and one group of Tc * tk threads per density channel (G = C groups). For
// every realisation b:
//   1. group g transforms channel g along z (length N; rows z >= N/2 are the
//      zero padding and are not loaded) and puts rho^_g(kz) in LDS;
//   2. group g forms the stress spectra of its components (v = 2g, 2g + 1
//      when C = 3, v = g otherwise),
//          sigma^_v(k) = sum_c i S_{v,c}(k) rho^_c(k)      (K^ = i S, K odd),
//      summing over c in increasing order, and transforms them back along z,
//      keeping rows z < nz. With C = 9 the groups g >= 6 have no component;
//      they transform zeros alongside, to keep the block's barriers, and
//      store nothing.
// A group's transforms share their barriers, and a thread's spectrum values
// (components x C x E numbers) stay in registers for all realisations. The
// spectrum tile of the block is stored contiguously as [c][v][kz][tk]. The
// density is requested before the spectrum values, so the first transform
// waits for it alone, and the next realisation's density before the inverse
// transforms, so its latency overlaps them.
// ----------------------------------------------------------------------------
// WV: each group is exactly one wave (tk Tc = 64) and owns its LDS region
// for both transforms (one stress component per group, NC > 3): the stages of
// its transforms synchronise within the wave, and the block meets only to
// publish the channel spectra and after the contraction has read them.
template <typename T, int N, int E, int NC, bool WV>
__global__ void __launch_bounds__(768) k_z_grouped(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                   const T* __restrict__ spec, ZGeom g,
                                                   const cplx<T>* __restrict__ tw, int tk, int ld) {
    static_assert(!WV || NC > 3, "wave-local groups need one stress component and one LDS region per group");
    constexpr int Tc = N / E;
    constexpr int OPG = NC == 3 ? 2 : 1;   // stress components per group
    constexpr int EH = (E + 1) / 2;        // elements that can hold data rows (z < N/2)
    constexpr bool HZ = N > 1;             // the upper half of every input column is padding
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    const int per = tk * Tc;
    const int grp = threadIdx.x / per;
    const int t = threadIdx.x - grp * per;
    const int c = t % tk;
    const int j = t / tk;
    const int blk = z_logical_block(g);
    const ZRoles ro = z_roles<T>(blk, tk, c, g);
    const bool has_v = OPG * grp < 6;      // wave-uniform
    const ColMajor lay{ld};
    const int region = N * ld;             // one transform column block in LDS

    // density rows z < nz of the block's columns (rows >= nz read zero; lanes
    // without data read a valid column). A wave can hold two groups (tk Tc <
    // 64), so the channel plane differs across its lanes: the loads take
    // per-lane addresses rather than one buffer resource per wave.
    const cplx<T>* in_l = in + ro.in0 + (int64_t)grp * g.iqs + ro.lane_in + (int64_t)j * g.irs;
    const int64_t in_real = (int64_t)g.C * g.iqs;
    const int64_t r_step = (int64_t)Tc * g.irs;
    cplx<T> fw[1][E];
    auto load_rows = [&](int b) {
#pragma unroll
        for (int m = 0; m < EH; ++m)
            fw[0][m] = j + Tc * m < g.nz ? in_l[b * in_real + m * r_step] : cplx<T>{T(0), T(0)};
    };
    const int ors = (int)g.ors;                      // in-block offsets fit in 32 bits
    cplx<T>* out_b = out + ro.own;
    const NyquistRole nq = ro.nq;
    if (nq.skip_block) return;                   // uniform over the block, before any barrier
    cplx<T>* mir_b = out + ro.mir;

    load_rows(ro.b0);
    constexpr int TWC = tw_count(N, E) > 0 ? tw_count(N, E) : 1;
    cplx<T> twr[TWC];
    load_tw_stages<T, N, E, 1, 0, TWC>(twr, j, tw + (N - 1));

    // Spectrum values of this thread: its components, all channels, elements
    // kz = j + Tc m. With a y mirror only ky <= Py/2 is stored and row Py - ky
    // stands in for ky > Py/2; with a z mirror only kz <= N/2 is stored and
    // elements m >= E/2 read kz' = N - kz = (Tc - j) + Tc (E - 1 - m). Odd
    // planes change sign; the signs are applied once, here.
    const bool flip_y = ro.flip_y;
    const bool zc = g.nkz_s < N;
    const int nkz = g.nkz_s;
    T sv[OPG][NC][E];
    {
        const T* sp = spec + ((int64_t)ro.kyc * g.ntiles + ro.tile) * (int64_t)g.C * 6 * nkz * tk;
        const __amdgpu_buffer_rsrc_t srs = make_rsrc(sp, (uint32_t)((size_t)g.C * 6 * nkz * tk * sizeof(T)));
        const int s_lane = (j * tk + c) * (int)sizeof(T);
        const int s_lane_m = ((Tc - j) * tk + c) * (int)sizeof(T);
#pragma unroll
        for (int k = 0; k < OPG; ++k)
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) {
                const int v = has_v ? OPG * grp + k : 0;
                const int bit = ch * 6 + v;
                const T sy = (flip_y && ((g.sgn_y >> bit) & 1)) ? T(-1) : T(1);
                const T sz = ((g.sgn_z >> bit) & 1) ? -sy : sy;
                const int base = (ch * 6 + v) * nkz;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const bool mir = zc && (2 * m >= E);
                    const T val = buf_real<T>(srs, mir ? s_lane_m : s_lane,
                                              (base + (mir ? Tc * (E - 1 - m) : Tc * m)) * tk * (int)sizeof(T));
                    sv[k][ch][m] = (mir ? sz : sy) * val;
                }
            }
    }

    for (int b = ro.b0; b < ro.b1; ++b) {
        // 1. forward transform of channel grp; its spectrum to LDS region grp
        fft_regs_k<T, N, E, true, HZ, 1, TWC, WV>(fw, twr, lds + grp * region, region, lay, c, j);
        __syncthreads();                             // the last stage's LDS reads are done
#pragma unroll
        for (int m = 0; m < E; ++m) lds[grp * region + lay(j + Tc * m, c)] = fw[0][m];
        __syncthreads();
        // 2. contraction for this group's components
        cplx<T> acc[OPG][E];
#pragma unroll
        for (int k = 0; k < OPG; ++k)
#pragma unroll
            for (int m = 0; m < E; ++m) acc[k][m] = {T(0), T(0)};
#pragma unroll
        for (int ch = 0; ch < NC; ++ch)
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const cplx<T> r = lds[ch * region + lay(j + Tc * m, c)];
#pragma unroll
                for (int k = 0; k < OPG; ++k) {
                    acc[k][m].x -= sv[k][ch][m] * r.y;
                    acc[k][m].y += sv[k][ch][m] * r.x;
                }
            }
        if (b + 1 < ro.b1) load_rows(b + 1);
        // inverse transforms (their first stage's barrier precedes any LDS write;
        // wave-local stages have none, so the block meets here first)
        if constexpr (WV) __syncthreads();
        fft_regs_k<T, N, E, false, false, OPG, TWC, WV>(acc, twr, lds + OPG * grp * region, region, lay, c, j);
        if (nq.own && has_v) {
#pragma unroll
            for (int k = 0; k < OPG; ++k) {
                cplx<T>* dst = out_b + (int64_t)(b * 6 + OPG * grp + k) * g.oqs;
#pragma unroll
                for (int m = 0; m < EH; ++m) {
                    const int z = j + Tc * m;
                    if (z < g.nz) dst[z * ors] = acc[k][m];
                }
            }
        }
        if (nq.mirror && has_v) {
#pragma unroll
            for (int k = 0; k < OPG; ++k) {
                cplx<T>* dst = mir_b + (int64_t)(b * 6 + OPG * grp + k) * g.oqs;
#pragma unroll
                for (int m = 0; m < EH; ++m) {
                    const int z = j + Tc * m;
                    if (z < g.nz) dst[z * ors] = cconj(acc[k][m]);
                }
            }
        }
    }
}


template <typename T, int L, int E, int NC, bool GROUPED>
static void z_launch(int64_t blocks, int tk, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& g,
                     const cplx<T>* tw, hipStream_t s) {
    const int groups = GROUPED ? NC : 1;
    size_t lds = z_lds_bytes(L, tk, NC, groups, (int)sizeof(T));
    const int ld = z_lds_ld(tk, (int)sizeof(T));
    const dim3 block(groups * tk * (L / E));
    if constexpr (!GROUPED && sizeof(T) == 4 && L == 64 && E == 8) {
        // the wave form (the only single-group form with 8 elements at length 64)
        const int wpb = g.B >= 4 ? 4 : (g.B >= 2 ? 2 : 1);
        const size_t stage = (z_stage_bytes(kZWaveTile, NC, g.nkz_s, 4) + 15) / 16 * 16;
        const size_t lw = stage + (size_t)wpb * L * kZWaveTile * sizeof(cplx<T>);
        const dim3 grid((unsigned)blocks);
        if (wpb == 4)
            hipLaunchKernelGGL((k_z_wave<T, L, E, NC, 4>), grid, dim3(256), lw, s, in, out, spec, g, tw);
        else if (wpb == 2)
            hipLaunchKernelGGL((k_z_wave<T, L, E, NC, 2>), grid, dim3(128), lw, s, in, out, spec, g, tw);
        else
            hipLaunchKernelGGL((k_z_wave<T, L, E, NC, 1>), grid, dim3(64), lw, s, in, out, spec, g, tw);
        (void)tk;
    } else if constexpr (GROUPED) {
        if constexpr (NC > 3 && L / E <= 64 && 64 % (L / E) == 0) {
            if (tk * (L / E) == 64) {
                hipLaunchKernelGGL((k_z_grouped<T, L, E, NC, true>), dim3((unsigned)blocks), block, lds, s, in, out,
                                   spec, g, tw, tk, ld);
                return;
            }
        }
        hipLaunchKernelGGL((k_z_grouped<T, L, E, NC, false>), dim3((unsigned)blocks), block, lds, s, in, out, spec, g,
                           tw, tk, ld);
    } else if constexpr (L >= 2 && L <= 256) {
        if (z_stage_spec(L, tk, NC, g.nkz_s, g.B, (int)sizeof(T))) {
            lds += z_stage_bytes(tk, NC, g.nkz_s, (int)sizeof(T));
            const dim3 grid((unsigned)blocks);
            if (tk == 4)
                hipLaunchKernelGGL((k_z_serial<T, L, E, NC, 4>), grid, block, lds, s, in, out, spec, g, tw, tk, ld);
            else if (tk == 8)
                hipLaunchKernelGGL((k_z_serial<T, L, E, NC, 8>), grid, block, lds, s, in, out, spec, g, tw, tk, ld);
            else
                hipLaunchKernelGGL((k_z_serial<T, L, E, NC, 16>), grid, block, lds, s, in, out, spec, g, tw, tk, ld);
        } else {
            hipLaunchKernelGGL((k_z_serial<T, L, E, NC, 0>), dim3((unsigned)blocks), block, lds, s, in, out, spec, g,
                               tw, tk, ld);
        }
    } else {
        hipLaunchKernelGGL((k_z_serial<T, L, E, NC, 0>), dim3((unsigned)blocks), block, lds, s, in, out, spec, g, tw,
                           tk, ld);
    }
}

template <typename T, int EV, int NC, bool GROUPED>
static void z_ev(int N, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& g, const cplx<T>* tw,
                 int tk, int64_t blocks, hipStream_t s) {
    switch (N) {
#define Z_CASE(L, EVV)                                                                                     \
    case L: z_launch<T, L, (L < EVV ? L : EVV), NC, GROUPED>(blocks, tk, in, out, spec, g, tw, s); break;
        DDS_FOR_LENGTHS(Z_CASE, EV)
#undef Z_CASE
        default: fail(DDSTRESS_E_UNSUPPORTED, "z transform length not supported");
    }
}

// Larger element classes, instantiated for the long z lengths only.
template <typename T, int EV, int NC, bool GROUPED>
static void z_ev_long(int N, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& g, const cplx<T>* tw,
                      int tk, int64_t blocks, hipStream_t s) {
    switch (N) {
        case 256: z_launch<T, 256, EV, NC, GROUPED>(blocks, tk, in, out, spec, g, tw, s); break;
        case 512: z_launch<T, 512, EV, NC, GROUPED>(blocks, tk, in, out, spec, g, tw, s); break;
        case 1024: z_launch<T, 1024, EV, NC, GROUPED>(blocks, tk, in, out, spec, g, tw, s); break;
        default: fail(DDSTRESS_E_UNSUPPORTED, "z transform length not supported");
    }
}

template <typename T, int NC, bool GROUPED>
void z_dispatch(int N, int ev, const cplx<T>* in, cplx<T>* out, const T* spec, const ZGeom& g,
                       const cplx<T>* tw, int tk, int64_t blocks, hipStream_t s) {
    constexpr int EV = sizeof(T) == 4 ? 4 : 2;
    if constexpr (sizeof(T) == 4 && !GROUPED) {
        if (N == 64 && ev == 8) {
            z_launch<T, 64, 8, NC, false>(blocks, tk, in, out, spec, g, tw, s);
            return;
        }
    }
    if (ev == EV) z_ev<T, EV, NC, GROUPED>(N, in, out, spec, g, tw, tk, blocks, s);
    else if (ev == 2 * EV) z_ev_long<T, 2 * EV, NC, GROUPED>(N, in, out, spec, g, tw, tk, blocks, s);
    else if (ev == 4 * EV) z_ev_long<T, 4 * EV, NC, GROUPED>(N, in, out, spec, g, tw, tk, blocks, s);
    else if constexpr (8 * EV <= 16) {
        if (ev == 8 * EV) z_ev_long<T, 8 * EV, NC, GROUPED>(N, in, out, spec, g, tw, tk, blocks, s);
        else fail(DDSTRESS_E_INVALID, "z element class not supported");
    } else {
        fail(DDSTRESS_E_INVALID, "z element class not supported");
    }
}


#define DDS_Z_INSTANTIATE(T, GROUPED)                                                                      \
    template void z_dispatch<T, 3, GROUPED>(int, int, const cplx<T>*, cplx<T>*, const T*, const ZGeom&,     \
                                            const cplx<T>*, int, int64_t, hipStream_t);                    \
    template void z_dispatch<T, 6, GROUPED>(int, int, const cplx<T>*, cplx<T>*, const T*, const ZGeom&,     \
                                            const cplx<T>*, int, int64_t, hipStream_t);                    \
    template void z_dispatch<T, 9, GROUPED>(int, int, const cplx<T>*, cplx<T>*, const T*, const ZGeom&,     \
                                            const cplx<T>*, int, int64_t, hipStream_t);

}  // namespace dds
