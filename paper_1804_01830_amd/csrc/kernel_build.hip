// Interaction coefficients on the device, in FP64 (Sec. 2.2 and 2.3), and
// their replica-shell sums for periodic boundaries in the plane (Sec. 4).
//
// For one line direction t and each unit Burgers vector e_gamma,
//   K_{v,gamma}(D) = dV / h * sigma^AB_v(p; e_gamma, t, h)
// is the stress per unit length of a segment (Eq. 9b) times the cell volume.
// Far cells: p = D o d (cell-centre offset) with h the cell's chord along t.
// Near cells (|D_a| d_a <= S max d on every axis): target and source cells are
// split into m_a subcells per axis; the coefficient is the mean over target
// subcells of the sum over source subcells, i.e. the sum over sub-offsets
// delta (|delta_a| < m_a) with weight prod_a (m_a - |delta_a|) / m_a^2 of the
// subcell coefficient at p = D o d + delta o s, h the subcell chord. The
// self-term is zero: with identical subdivision every sub-offset pair
// +delta / -delta cancels because a centred segment's field is odd.
//
// The segment stress is the coordinate-free Eq. (6)-(7), evaluated at each
// end point E with R = p - E, R_t = R + |R| t = rho + (|R| + L) t,
// L = R.t, rho = R - L t, and |R| + L computed as |rho|^2 / (|R| - L) when
// L < 0. Points behind the segment centre use the same segment described from
// B to A (t -> -t, b -> -b), which keeps them off the singular ray R_t = 0.
#include <atomic>
#include <cmath>

#include "ddstress_internal.hpp"

namespace dds {

namespace {

// Voigt pairs (xx, yy, zz, yz, xz, xy).
__device__ __constant__ int kVa[6] = {0, 1, 2, 1, 0, 0};
__device__ __constant__ int kVb[6] = {0, 1, 2, 2, 2, 1};

// acc[g*6+v] += coef * sigma_v at one end point for b = bsign * e_g.
__device__ void eq6_end(const double R[3], const double t[3], double bsign, double coef,
                        double mu, double nu, double* acc) {
    const double Rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    const double L = R[0] * t[0] + R[1] * t[1] + R[2] * t[2];
    double rho[3] = {R[0] - L * t[0], R[1] - L * t[1], R[2] - L * t[2]};
    const double rho2 = rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2];
    const double rpl = (L >= 0.0) ? (Rn + L) : rho2 / (Rn - L);
    const double Y[3] = {rho[0] + rpl * t[0], rho[1] + rpl * t[1], rho[2] + rpl * t[2]};
    const double Y2 = Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2];
    const double inv_y2 = 1.0 / Y2;
    const double lr = L / Rn;
    const double pref = coef * mu / (M_PI * Y2);
    const double k1 = 1.0 / (1.0 - nu);
    const double k2 = 0.5 / (1.0 - nu);
    // Y x t (its components are the triple products (e_g, Y, t))
    const double yxt[3] = {Y[1] * t[2] - Y[2] * t[1], Y[2] * t[0] - Y[0] * t[2], Y[0] * t[1] - Y[1] * t[0]};
    for (int g = 0; g < 3; ++g) {
        // b = bsign e_g: b x Y and b x t
        double bY[3], bt[3];
        const int g1 = (g + 1) % 3, g2 = (g + 2) % 3;
        bY[g] = 0.0;
        bY[g1] = -bsign * Y[g2];
        bY[g2] = bsign * Y[g1];
        bt[g] = 0.0;
        bt[g1] = -bsign * t[g2];
        bt[g2] = bsign * t[g1];
        const double trip = bsign * yxt[g];
        for (int v = 0; v < 6; ++v) {
            const int a = kVa[v], c = kVb[v];
            const double phi = 2.0 * inv_y2 * (rho[a] * Y[c] + Y[a] * rho[c] + lr * Y[a] * Y[c]);
            const double s1 = 0.5 * (bY[a] * t[c] + bY[c] * t[a]);
            const double s2 = 0.5 * (bt[a] * Y[c] + bt[c] * Y[a]);
            const double dl = (a == c) ? 1.0 : 0.0;
            acc[g * 6 + v] += pref * (s1 - k1 * s2 - k2 * trip * (dl + t[a] * t[c] + phi));
        }
    }
}

// acc += coef * sigma^AB(p) of the segment of length h along t centred at 0.
__device__ void segment(const double p[3], double h, const double t[3], double coef, double mu,
                        double nu, double* acc) {
    const double hh = 0.5 * h;
    const double pt = p[0] * t[0] + p[1] * t[1] + p[2] * t[2];
    const double RB[3] = {p[0] - hh * t[0], p[1] - hh * t[1], p[2] - hh * t[2]};
    const double RA[3] = {p[0] + hh * t[0], p[1] + hh * t[1], p[2] + hh * t[2]};
    if (pt >= 0.0) {
        eq6_end(RB, t, 1.0, coef, mu, nu, acc);
        eq6_end(RA, t, 1.0, -coef, mu, nu, acc);
    } else {
        const double tr[3] = {-t[0], -t[1], -t[2]};
        eq6_end(RA, tr, -1.0, coef, mu, nu, acc);
        eq6_end(RB, tr, -1.0, -coef, mu, nu, acc);
    }
}

__device__ __forceinline__ bool wrap_offset(int i, int n, int P, int& off) {
    if (i < n) { off = i; return true; }
    if (i > P - n) { off = i - P; return true; }
    return false;
}

// acc += w * K(D): one open-boundary coefficient (far: centre offset; near:
// weighted sum over sub-offsets; D = 0: the zero self-term).
__device__ void add_coefficient(const KernelParams& kp, const int D[3], double w, double* acc) {
    if (D[0] == 0 && D[1] == 0 && D[2] == 0) return;
    bool near = true;
    for (int a = 0; a < 3; ++a) near = near && (fabs((double)D[a]) * kp.d[a] <= kp.near_lim);
    if (!near) {
        const double p[3] = {D[0] * kp.d[0], D[1] * kp.d[1], D[2] * kp.d[2]};
        segment(p, kp.h_cell, kp.t, w * kp.dV / kp.h_cell, kp.mu, kp.nu, acc);
        return;
    }
    for (int dz = -(kp.m[2] - 1); dz < kp.m[2]; ++dz)
        for (int dy = -(kp.m[1] - 1); dy < kp.m[1]; ++dy)
            for (int dx = -(kp.m[0] - 1); dx < kp.m[0]; ++dx) {
                const double wx = (double)(kp.m[0] - abs(dx)) / (double)(kp.m[0] * kp.m[0]);
                const double wy = (double)(kp.m[1] - abs(dy)) / (double)(kp.m[1] * kp.m[1]);
                const double wz = (double)(kp.m[2] - abs(dz)) / (double)(kp.m[2] * kp.m[2]);
                const double ws = wx * wy * wz;
                const double p[3] = {D[0] * kp.d[0] + dx * kp.s[0], D[1] * kp.d[1] + dy * kp.s[1],
                                     D[2] * kp.d[2] + dz * kp.s[2]};
                segment(p, kp.h_sub, kp.t, w * ws * kp.dV / kp.h_sub, kp.mu, kp.nu, acc);
            }
}

// Offsets represented by grid index i on one axis: the wrap-order offset of a
// zero-padded axis (none in the padding gap), or on a periodic axis (P = N)
// the representative in [-N/2, N/2), with both -N/2 and +N/2 at half weight
// for the half period. Returns the number of representatives (0, 1 or 2).
__device__ __forceinline__ int axis_reps(int i, int n, int P, bool periodic, int rep[2], double wt[2]) {
    if (periodic) {
        const int h = n / 2;
        if (i == h && (n & 1) == 0) {
            rep[0] = -h;
            rep[1] = h;
            wt[0] = wt[1] = 0.5;
            return 2;
        }
        rep[0] = i <= h ? i : i - n;
        wt[0] = 1.0;
        return 1;
    }
    wt[0] = 1.0;
    return wrap_offset(i, n, P, rep[0]) ? 1 : 0;
}

// One thread per (x, y) point of one z plane of the FFT grid: blockIdx.y
// and blockIdx.z carry the y and z indices, so no 64-bit division is needed.
// On a periodic axis the coefficient is the sum over the replica shells
// |k|, |l| <= n_sh of the offset's representative (Eq. 13).
__global__ void __launch_bounds__(256) k_kernel_build(double* __restrict__ out, KernelParams kp, int64_t plane) {
    const int ix = blockIdx.x * blockDim.x + threadIdx.x;
    const int iy = blockIdx.y;
    const int iz = blockIdx.z;
    if (ix >= kp.P[0]) return;
    const int64_t idx = ((int64_t)iz * kp.P[1] + iy) * kp.P[0] + ix;
    double acc[18];
    for (int q = 0; q < 18; ++q) acc[q] = 0.0;
    int rx[2], ry[2], dzv;
    double wx[2], wy[2];
    const int nx = axis_reps(ix, kp.n[0], kp.P[0], kp.per[0] != 0, rx, wx);
    const int ny = axis_reps(iy, kp.n[1], kp.P[1], kp.per[1] != 0, ry, wy);
    const bool zin = wrap_offset(iz, kp.n[2], kp.P[2], dzv);
    const int sx = kp.per[0] ? kp.shells : 0;
    const int sy = kp.per[1] ? kp.shells : 0;
    if (zin) {
        for (int a = 0; a < nx; ++a)
            for (int b = 0; b < ny; ++b) {
                const double w = wx[a] * wy[b];
                for (int k = -sx; k <= sx; ++k)
                    for (int l = -sy; l <= sy; ++l) {
                        const int D[3] = {rx[a] + k * kp.n[0], ry[b] + l * kp.n[1], dzv};
                        add_coefficient(kp, D, w, acc);
                    }
            }
    }
    for (int q = 0; q < 18; ++q) out[q * plane + idx] = acc[q];
}

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* a, double v) {
    // non-negative doubles order like their bit patterns
    atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

// Mirror parity of the 18 coefficient planes: for each plane q and mirror
// axis a (0: y -> -y, 1: z -> -z), max |K - K'| and max |K + K'| with K' the
// value at the mirrored offset, and max |K|. stats[q*5 + {0,1,2,3,4}] =
// {even_y, odd_y, even_z, odd_z, max}. One thread per (x, y, z) point.
__global__ void __launch_bounds__(256) k_mirror_stats(const double* __restrict__ kr, int Px, int Py, int Pz,
                                                      int64_t plane, unsigned long long* __restrict__ stats) {
    const int ix = blockIdx.x * blockDim.x + threadIdx.x;
    const int iy = blockIdx.y;
    const int iz = blockIdx.z;
    const bool ok = ix < Px;
    const int my = (Py - iy) & (Py - 1);
    const int mz = (Pz - iz) & (Pz - 1);
    const int64_t i0 = ((int64_t)iz * Py + iy) * Px + (ok ? ix : 0);
    const int64_t iyv = ((int64_t)iz * Py + my) * Px + (ok ? ix : 0);
    const int64_t izv = ((int64_t)mz * Py + iy) * Px + (ok ? ix : 0);
    __shared__ double red[5][256];
    for (int q = 0; q < 18; ++q) {
        double v[5] = {0, 0, 0, 0, 0};
        if (ok) {
            const double k = kr[q * plane + i0];
            const double ky = kr[q * plane + iyv];
            const double kz = kr[q * plane + izv];
            v[0] = fabs(k - ky);
            v[1] = fabs(k + ky);
            v[2] = fabs(k - kz);
            v[3] = fabs(k + kz);
            v[4] = fabs(k);
        }
        for (int e = 0; e < 5; ++e) red[e][threadIdx.x] = v[e];
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                for (int e = 0; e < 5; ++e) red[e][threadIdx.x] = fmax(red[e][threadIdx.x], red[e][threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0)
            for (int e = 0; e < 5; ++e) atomic_max_nonneg(&stats[q * 5 + e], red[e][0]);
        __syncthreads();
    }
}

// Spectrum extraction: S = Im(K^) / P for the channels 3*line .. 3*line+2,
// stored as [kyc][tile][c][v][kzc][tk] for kyc < nky, kzc < nkz (the kept
// halves when a mirror symmetry lets the rest be reconstructed). With a
// Nyquist strip (strip_on and z_nyq_groups) the last tile's slot at row q holds instead
// the column kx = M at ky = q tk + col, for ky <= Py/2 (zeros elsewhere). One
// thread per (kx in the tiled range, kyc, kzc), looping over the 18 planes;
// also the maxima of |Re K^| and |Im K^| over the kept entries.
template <typename T>
__global__ void __launch_bounds__(256) k_extract(const cplx<double>* __restrict__ kh, T* __restrict__ spec,
                                                 int line, int C, int ncols, int64_t wx, int Py, int Pz, int nky,
                                                 int nkz, int tk, int ntiles, int strip_on, double inv_p,
                                                 unsigned long long* __restrict__ maxbits) {
    const int kx = blockIdx.x * blockDim.x + threadIdx.x;
    const int ky = blockIdx.y;
    const int kz = blockIdx.z;
    const int kxr = ntiles * tk;
    double re = 0.0, im = 0.0;
    if (kx < kxr) {
        const int tile = kx / tk, col = kx % tk;
        const bool strip = strip_on && tile == ntiles - 1 && z_nyq_groups(ncols, tk, Py) > 0;
        const int sx = strip ? ncols - 1 : kx;                  // source column and row
        const int sy = strip ? ky * tk + col : ky;
        const bool have = strip ? 2 * sy <= Py : kx < ncols;
        for (int gv = 0; gv < 18; ++gv) {
            const int g = gv / 6, v = gv % 6;
            const int ch = 3 * line + g;
            const int64_t o = (((((int64_t)ky * ntiles + tile) * C + ch) * 6 + v) * nkz + kz) * tk + col;
            if (have) {
                const cplx<double> val = kh[(((int64_t)gv * Pz + kz) * Py + sy) * wx + sx];
                re = fmax(re, fabs(val.x));
                im = fmax(im, fabs(val.y));
                spec[o] = (T)(val.y * inv_p);
            } else {
                spec[o] = T(0);
            }
        }
    }
    __shared__ double sre[256], sim[256];
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sre[threadIdx.x] = fmax(sre[threadIdx.x], sre[threadIdx.x + w]);
            sim[threadIdx.x] = fmax(sim[threadIdx.x], sim[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomic_max_nonneg(&maxbits[0], sre[0]);
        atomic_max_nonneg(&maxbits[1], sim[0]);
    }
}

double chord(const double box[3], const double t[3]) {
    double best = INFINITY;
    for (int a = 0; a < 3; ++a)
        if (t[a] != 0.0) best = std::fmin(best, box[a] / std::fabs(t[a]));
    return best;
}

}  // namespace

KernelParams make_kernel_params(const ddstress_desc& desc, int line, const int P[3]) {
    KernelParams kp{};
    double dmin = desc.d[0], dmax = desc.d[0];
    for (int a = 0; a < 3; ++a) {
        kp.n[a] = desc.n[a];
        kp.P[a] = P[a];
        kp.d[a] = desc.d[a];
        dmin = std::fmin(dmin, desc.d[a]);
        dmax = std::fmax(dmax, desc.d[a]);
    }
    for (int a = 0; a < 3; ++a) {
        kp.m[a] = std::max(1, (int)std::floor(desc.d[a] / dmin + 0.5));
        kp.s[a] = desc.d[a] / kp.m[a];
    }
    const double* tl = desc.t[line];
    const double tn = std::sqrt(tl[0] * tl[0] + tl[1] * tl[1] + tl[2] * tl[2]);
    for (int a = 0; a < 3; ++a) kp.t[a] = tl[a] / tn;
    kp.mu = desc.mu;
    kp.nu = desc.nu;
    kp.h_cell = chord(kp.d, kp.t);
    kp.h_sub = chord(kp.s, kp.t);
    kp.dV = desc.d[0] * desc.d[1] * desc.d[2];
    const int S = desc.near_shells == 0 ? 2 : desc.near_shells;
    kp.near_lim = S * dmax;
    kp.per[0] = periodic_axis(&desc, 0) ? 1 : 0;
    kp.per[1] = periodic_axis(&desc, 1) ? 1 : 0;
    kp.shells = desc.pbc_shells == 0 ? kDefaultPbcShells : desc.pbc_shells;
    return kp;
}

void launch_kernel_build(const KernelParams& kp, double* out, hipStream_t s) {
    const int64_t plane = (int64_t)kp.P[0] * kp.P[1] * kp.P[2];
    const dim3 grid((unsigned)((kp.P[0] + 255) / 256), (unsigned)kp.P[1], (unsigned)kp.P[2]);
    hipLaunchKernelGGL(k_kernel_build, grid, dim3(256), 0, s, out, kp, plane);
    check_hip(hipGetLastError(), "kernel build launch");
}

void launch_mirror_stats(const double* kr, const int P[3], unsigned long long* stats, hipStream_t s) {
    const int64_t plane = (int64_t)P[0] * P[1] * P[2];
    const dim3 grid((unsigned)((P[0] + 255) / 256), (unsigned)P[1], (unsigned)P[2]);
    hipLaunchKernelGGL(k_mirror_stats, grid, dim3(256), 0, s, kr, P[0], P[1], P[2], plane, stats);
    check_hip(hipGetLastError(), "mirror statistics launch");
}

template <typename T>
void launch_extract(const cplx<double>* kh, T* spec, int line, int C, int ncols, int64_t wx, int Py, int Pz,
                    int nky, int nkz, int tk, int ntiles, bool strip, double inv_p, unsigned long long* maxbits,
                    hipStream_t s) {
    const int kxr = ntiles * tk;
    const dim3 grid((unsigned)((kxr + 255) / 256), (unsigned)nky, (unsigned)nkz);
    hipLaunchKernelGGL((k_extract<T>), grid, dim3(256), 0, s, kh, spec, line, C, ncols, wx, Py, Pz, nky, nkz, tk,
                       ntiles, strip ? 1 : 0, inv_p, maxbits);
    check_hip(hipGetLastError(), "spectrum extraction launch");
}

template void launch_extract<float>(const cplx<double>*, float*, int, int, int, int64_t, int, int, int, int, int,
                                    int, bool, double, unsigned long long*, hipStream_t);
template void launch_extract<double>(const cplx<double>*, double*, int, int, int, int64_t, int, int, int, int, int,
                                     int, bool, double, unsigned long long*, hipStream_t);

template <typename T>
void fill_twiddles(cplx<T>* host) {
    // entry L-1+k = exp(-2 pi i k / L), evaluated in long double and rounded once
    host[0] = {T(1), T(0)};
    for (int L = 2; L <= kMaxLen; L <<= 1) {
        for (int k = 0; k < L; ++k) {
            const long double pi = 3.141592653589793238462643383279502884L;
            const long double a = 2.0L * pi * (long double)k / (long double)L;
            const long double c = cosl(a), sn = sinl(a);
            host[L - 1 + k] = {(T)c, (T)(-sn)};
        }
    }
    host[kTwiddleEntries - 1] = {T(1), T(0)};
}
template void fill_twiddles<float>(cplx<float>*);
template void fill_twiddles<double>(cplx<double>*);

}  // namespace dds
