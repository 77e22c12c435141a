// Relaxation of the dislocation stress under free top and bottom surfaces
// (Sec. 5, Eq. 14-18): explicit pseudo-time steps of the Navier-Cauchy
// equation driven by f = div sigma^dis, periodic in x and y, with ghost
// layers that carry the traction conditions Eq. (16c).
//
// Discretisation (nodes at cell centres, surfaces through the first and last
// node layers): second derivatives by central second differences, mixed
// derivatives as products of central first differences, f by central
// differences (second-order one-sided in z on the surface layers), the ghost
// layers rewritten from the real layers after each step (Eq. 18b and its
// analogues), the total stress by Hooke's law with central differences.
//
// Kernels, all HBM-bound stencils: k_relax_load (f, surface terms, u = 0),
// k_relax_march (one explicit step into the other state buffer, marching
// along z with LDS planes), k_relax_ghost (both ghost layers), k_relax_norm
// (max |update| / dt), k_relax_stress.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "ddstress_internal.hpp"

namespace dds {

namespace {

constexpr int kRelaxBX = 64, kRelaxBY = 4;
// Tile of the z-marching step and the number of blocks its z chunks aim at.
#ifndef DDS_RELAX_TX
#define DDS_RELAX_TX 64
#endif
#ifndef DDS_RELAX_TY
#define DDS_RELAX_TY 16
#endif
#ifndef DDS_RELAX_BLOCKS
#define DDS_RELAX_BLOCKS 512
#endif
constexpr int kRelaxBlocks = DDS_RELAX_BLOCKS;
constexpr int kRelaxMaxN = 4096;

template <typename T>
struct RelaxGeom {
    int nx, ny, nz;
    int64_t plane;        // nx * ny
    int64_t cstride;      // (nz + 2) * plane: one displacement component with its ghost layers
    int64_t fstride;      // nz * plane: one force component / stress component
    T hx, hy, hz;         // 1 / (2 d): central first differences
    T qx, qy, qz;         // 1 / d^2: second differences
    T A, B, dt;
    T twodz, nu, inv1mnu; // 2 dz, nu, 1 / (1 - nu)
    T lam;                // A - 2B
    T c_shear, c_normal;  // (1 + nu) / E and (1 + nu)(1 - 2 nu) / E (Eq. 16c)
};

__device__ __forceinline__ int nxt(int i, int n) { return i + 1 == n ? 0 : i + 1; }
__device__ __forceinline__ int prv(int i, int n) { return i == 0 ? n - 1 : i - 1; }

// Voigt index of the symmetric pair (a, b).
__device__ __forceinline__ int voigt(int a, int b) {
    if (a == b) return a;
    const int s = a + b;            // (1,2) -> 3, (0,2) -> 2, (0,1) -> 1
    return s == 3 ? 3 : (s == 2 ? 4 : 5);
}

// v = A grad div u - B rot rot u + f at node (i, j, k) (k = node layer),
// written as (A - B) grad div u + B laplacian u.
template <typename T>
__device__ __forceinline__ void navier_update(const T* __restrict__ u, const T* __restrict__ f, const RelaxGeom<T>& g,
                                             int i, int j, int k, T v[3], T u0[3]) {
    const int ip = nxt(i, g.nx), im = prv(i, g.nx), jp = nxt(j, g.ny), jm = prv(j, g.ny);
    const int64_t L = (int64_t)(k + 1) * g.plane;
    const int64_t r0 = (int64_t)j * g.nx, rp = (int64_t)jp * g.nx, rm = (int64_t)jm * g.nx;
    T dxx[3], dyy[3], dzz[3], dxy[3], dxz[3], dyz[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T* uc = u + c * g.cstride;
        const T* lz = uc + L;
        const T* lu = lz + g.plane;       // layer above
        const T* ld = lz - g.plane;       // layer below
        const T c0 = lz[r0 + i];
        u0[c] = c0;
        dxx[c] = (lz[r0 + ip] - T(2) * c0 + lz[r0 + im]) * g.qx;
        dyy[c] = (lz[rp + i] - T(2) * c0 + lz[rm + i]) * g.qy;
        dzz[c] = (lu[r0 + i] - T(2) * c0 + ld[r0 + i]) * g.qz;
        dxy[c] = ((lz[rp + ip] - lz[rp + im]) * g.hx - (lz[rm + ip] - lz[rm + im]) * g.hx) * g.hy;
        dxz[c] = ((lu[r0 + ip] - lu[r0 + im]) * g.hx - (ld[r0 + ip] - ld[r0 + im]) * g.hx) * g.hz;
        dyz[c] = ((lu[rp + i] - lu[rm + i]) * g.hy - (ld[rp + i] - ld[rm + i]) * g.hy) * g.hz;
    }
    const T gd[3] = {dxx[0] + dxy[1] + dxz[2], dxy[0] + dyy[1] + dyz[2], dxz[0] + dyz[1] + dzz[2]};
    const int64_t n = (int64_t)k * g.plane + r0 + i;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T lap = dxx[a] + dyy[a] + dzz[a];
        v[a] = (g.A - g.B) * gd[a] + g.B * lap + f[a * g.fstride + n];
    }
}

// max |v| over the nodes into *red (the bit pattern of a non-negative double
// orders like the value). One thread per node; the update norm only.
template <typename T>
__global__ void __launch_bounds__(kRelaxBX* kRelaxBY)
    k_relax_norm(const T* __restrict__ u, const T* __restrict__ f, RelaxGeom<T> g, unsigned long long* __restrict__ red) {
    const int i = blockIdx.x * kRelaxBX + threadIdx.x;
    const int j = blockIdx.y * kRelaxBY + threadIdx.y;
    const int k = blockIdx.z;
    const bool ok = i < g.nx && j < g.ny;
    T v[3] = {T(0), T(0), T(0)}, u0[3];
    if (ok) navier_update(u, f, g, i, j, k, v, u0);
    __shared__ double sm[kRelaxBX * kRelaxBY];
    const int t = threadIdx.y * kRelaxBX + threadIdx.x;
    sm[t] = fmax(fmax(fabs((double)v[0]), fabs((double)v[1])), fabs((double)v[2]));
    __syncthreads();
    for (int w = kRelaxBX * kRelaxBY / 2; w > 0; w >>= 1) {
        if (t < w) sm[t] = fmax(sm[t], sm[t + w]);
        __syncthreads();
    }
    if (t == 0) atomicMax(red, (unsigned long long)__double_as_longlong(sm[0]));
}

// Ghost values at column (i, j) of the bottom (top = 0) or top surface from
// the real layers of u (Eq. 16c solved for the ghost value, Eq. 18b).
template <typename T>
__device__ __forceinline__ void ghost_value(const T* __restrict__ u, const T* __restrict__ phi, const RelaxGeom<T>& g,
                                            int top, int i, int j, T out[3]) {
    const int s = top ? g.nz : 1, inner = top ? g.nz - 1 : 2;
    const int ip = nxt(i, g.nx), im = prv(i, g.nx), jp = nxt(j, g.ny), jm = prv(j, g.ny);
    const int64_t r0 = (int64_t)j * g.nx, rp = (int64_t)jp * g.nx, rm = (int64_t)jm * g.nx;
    const T* ux = u;
    const T* uy = u + g.cstride;
    const T* uz = u + 2 * g.cstride;
    const int64_t ls = (int64_t)s * g.plane, li = (int64_t)inner * g.plane;
    const T gx = (uz[ls + r0 + ip] - uz[ls + r0 + im]) * g.hx;      // d u_z / dx on the surface
    const T gy = (uz[ls + rp + i] - uz[ls + rm + i]) * g.hy;        // d u_z / dy
    const T dxy = (ux[ls + r0 + ip] - ux[ls + r0 + im]) * g.hx + (uy[ls + rp + i] - uy[ls + rm + i]) * g.hy;
    const int64_t q = (int64_t)top * 3 * g.plane + r0 + i;
    const T pxz = phi[q], pyz = phi[q + g.plane], pzz = phi[q + 2 * g.plane];
    if (!top) {
        out[0] = ux[li + r0 + i] + g.twodz * (gx - T(2) * pxz);
        out[1] = uy[li + r0 + i] + g.twodz * (gy - T(2) * pyz);
        out[2] = uz[li + r0 + i] - g.twodz * (pzz - g.nu * dxy) * g.inv1mnu;
    } else {
        out[0] = ux[li + r0 + i] + g.twodz * (T(2) * pxz - gx);
        out[1] = uy[li + r0 + i] + g.twodz * (T(2) * pyz - gy);
        out[2] = uz[li + r0 + i] + g.twodz * (pzz - g.nu * dxy) * g.inv1mnu;
    }
}

// One explicit step, marching along z: a block owns a TX x TY tile of
// columns and a chunk of node layers; the three displacement planes the
// stencil touches (layers k - 1, k, k + 1, three components, one halo cell
// on each side, periodic wrap) live in LDS in a rotating set of three slots,
// and the next plane is fetched into registers while the current layer is
// computed. Each displacement value is read from memory once per chunk
// (plus halos and the two planes that chunks share); the blocks of one tile
// take consecutive logical indices, which xcd_block keeps on one XCD. The
// ghost planes are read like the others (a ghost pass follows every step:
// evaluating them in the surface blocks instead puts their dependent loads
// on the critical path and was slower).
template <typename T, int TX, int TY>
__global__ void __launch_bounds__(TX* TY)
    k_relax_march(const T* __restrict__ u, T* __restrict__ un, const T* __restrict__ f, RelaxGeom<T> g, int tiles_x,
                  int nchunks, int kc) {
    constexpr int W = TX + 2, H = TY + 2, PL = W * H;           // plane tile with halo
    constexpr int NT = TX * TY, PER = (PL + NT - 1) / NT;       // loads per thread per component
    __shared__ T lds[3][3][PL];                                 // [slot][component][tile]
    const int nb = gridDim.x;
    const int lb = xcd_block(blockIdx.x, nb);
    const int chunk = lb % nchunks, tile = lb / nchunks;
    const int i0 = (tile % tiles_x) * TX, j0 = (tile / tiles_x) * TY;
    const int k0 = chunk * kc;
    const int k1 = min(g.nz, k0 + kc);
    if (k0 >= k1) return;                                       // uniform per block
    const int t = threadIdx.x, tx = t % TX, ty = t / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool ok = i < g.nx && j < g.ny;
    // global offsets (within one layer) of this thread's share of the halo tile
    int64_t off[PER];
    int slot_e[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = t + q * NT;
        slot_e[q] = e < PL ? e : -1;
        const int ex = e % W, ey = e / W;
        int gx = (i0 + ex - 1) % g.nx, gy = (j0 + ey - 1) % g.ny;
        if (gx < 0) gx += g.nx;
        if (gy < 0) gy += g.ny;
        off[q] = (int64_t)gy * g.nx + gx;
    }
    T pre[3][PER];
    auto fetch = [&](int layer) {
        const int64_t lo = (int64_t)layer * g.plane;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (slot_e[q] >= 0) pre[c][q] = u[c * g.cstride + lo + off[q]];
    };
    auto store = [&](int layer) {
        const int sl = layer % 3;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (slot_e[q] >= 0) lds[sl][c][slot_e[q]] = pre[c][q];
    };
    const int ctr = (ty + 1) * W + tx + 1;
    auto compute = [&](int k) {
        if (!ok) return;
        const int L = k + 1;
        const int sd = (L - 1) % 3, sc = L % 3, su = (L + 1) % 3;
        T dxx[3], dyy[3], dzz[3], dxy[3], dxz[3], dyz[3], u0[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T* lz = lds[sc][c];
            const T* lu = lds[su][c];
            const T* ld = lds[sd][c];
            const T c0 = lz[ctr];
            u0[c] = c0;
            dxx[c] = (lz[ctr + 1] - T(2) * c0 + lz[ctr - 1]) * g.qx;
            dyy[c] = (lz[ctr + W] - T(2) * c0 + lz[ctr - W]) * g.qy;
            dzz[c] = (lu[ctr] - T(2) * c0 + ld[ctr]) * g.qz;
            dxy[c] = ((lz[ctr + W + 1] - lz[ctr + W - 1]) * g.hx - (lz[ctr - W + 1] - lz[ctr - W - 1]) * g.hx) * g.hy;
            dxz[c] = ((lu[ctr + 1] - lu[ctr - 1]) * g.hx - (ld[ctr + 1] - ld[ctr - 1]) * g.hx) * g.hz;
            dyz[c] = ((lu[ctr + W] - lu[ctr - W]) * g.hy - (ld[ctr + W] - ld[ctr - W]) * g.hy) * g.hz;
        }
        const T gd[3] = {dxx[0] + dxy[1] + dxz[2], dxy[0] + dyy[1] + dyz[2], dxz[0] + dyz[1] + dzz[2]};
        const int64_t n = (int64_t)k * g.plane + (int64_t)j * g.nx + i;
        const int64_t o = n + g.plane;                          // the same node in the displacement layout
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T lap = dxx[a] + dyy[a] + dzz[a];
            const T v = (g.A - g.B) * gd[a] + g.B * lap + f[a * g.fstride + n];
            un[a * g.cstride + o] = u0[a] + g.dt * v;
        }
    };
    fetch(k0);
    store(k0);
    fetch(k0 + 1);
    store(k0 + 1);
    fetch(k0 + 2);
    for (int k = k0; k < k1; ++k) {
        const int L = k + 1;                                    // u layer of node layer k
        store(L + 1);
        __syncthreads();
        if (k + 1 < k1) fetch(L + 2);                           // overlaps the arithmetic below
        compute(k);
        __syncthreads();                                        // slot (L - 1) % 3 is refilled next
    }
}

// Ghost layers from the real layers (Eq. 16c on both surfaces). One thread
// per (i, j); blockIdx.z = 0 bottom, 1 top.
template <typename T>
__global__ void __launch_bounds__(kRelaxBX* kRelaxBY)
    k_relax_ghost(T* __restrict__ u, const T* __restrict__ phi, RelaxGeom<T> g) {
    const int i = blockIdx.x * kRelaxBX + threadIdx.x;
    const int j = blockIdx.y * kRelaxBY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int top = blockIdx.z;
    T v[3];
    ghost_value(u, phi, g, top, i, j, v);
    const int64_t o = (int64_t)(top ? g.nz + 1 : 0) * g.plane + (int64_t)j * g.nx + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c * g.cstride + o] = v[c];
}

// f = div sigma^dis on the nodes, the surface terms phi [2][3][Ny][Nx] and
// u = 0 on the node layers.
template <typename T>
__global__ void __launch_bounds__(kRelaxBX* kRelaxBY)
    k_relax_load(const T* __restrict__ s, T* __restrict__ f, T* __restrict__ phi, T* __restrict__ u,
                 RelaxGeom<T> g) {
    const int i = blockIdx.x * kRelaxBX + threadIdx.x;
    const int j = blockIdx.y * kRelaxBY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const int ip = nxt(i, g.nx), im = prv(i, g.nx), jp = nxt(j, g.ny), jm = prv(j, g.ny);
    const int64_t r0 = (int64_t)j * g.nx;
    const int64_t n = (int64_t)k * g.plane + r0 + i;
    const int64_t px = (int64_t)k * g.plane + r0, py = (int64_t)k * g.plane;
    for (int a = 0; a < 3; ++a) {
        const T* sx = s + voigt(a, 0) * g.fstride;
        const T* sy = s + voigt(a, 1) * g.fstride;
        const T* sz = s + voigt(a, 2) * g.fstride;
        const T ddx = (sx[px + ip] - sx[px + im]) * g.hx;
        const T ddy = (sy[py + (int64_t)jp * g.nx + i] - sy[py + (int64_t)jm * g.nx + i]) * g.hy;
        T ddz;
        const int64_t c = r0 + i;
        if (k == 0) {
            ddz = (T(-3) * sz[c] + T(4) * sz[g.plane + c] - sz[2 * g.plane + c]) * g.hz;
        } else if (k == g.nz - 1) {
            const int64_t b = (int64_t)k * g.plane + c;
            ddz = (T(3) * sz[b] - T(4) * sz[b - g.plane] + sz[b - 2 * g.plane]) * g.hz;
        } else {
            ddz = (sz[n + g.plane] - sz[n - g.plane]) * g.hz;
        }
        f[a * g.fstride + n] = ddx + ddy + ddz;
        u[a * g.cstride + (int64_t)(k + 1) * g.plane + r0 + i] = T(0);
    }
    if (k == 0 || k == g.nz - 1) {
        const int side = k == 0 ? 0 : 1;
        const int64_t q = (int64_t)side * 3 * g.plane + r0 + i;
        phi[q] = -g.c_shear * s[4 * g.fstride + n];
        phi[q + g.plane] = -g.c_shear * s[3 * g.fstride + n];
        phi[q + 2 * g.plane] = -g.c_normal * s[2 * g.fstride + n];
    }
}

// sigma_total = sigma_dis + sigma(u) (Hooke's law, central differences; the
// ghost layers supply the z differences on the surface layers).
template <typename T>
__global__ void __launch_bounds__(kRelaxBX* kRelaxBY)
    k_relax_stress(const T* __restrict__ u, const T* sd, T* out, RelaxGeom<T> g) {
    const int i = blockIdx.x * kRelaxBX + threadIdx.x;
    const int j = blockIdx.y * kRelaxBY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const int ip = nxt(i, g.nx), im = prv(i, g.nx), jp = nxt(j, g.ny), jm = prv(j, g.ny);
    const int64_t L = (int64_t)(k + 1) * g.plane;
    const int64_t r0 = (int64_t)j * g.nx, rp = (int64_t)jp * g.nx, rm = (int64_t)jm * g.nx;
    T G[3][3];      // G[c][a] = d u_c / d x_a
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T* lz = u + c * g.cstride + L;
        G[c][0] = (lz[r0 + ip] - lz[r0 + im]) * g.hx;
        G[c][1] = (lz[rp + i] - lz[rm + i]) * g.hy;
        G[c][2] = (lz[g.plane + r0 + i] - lz[r0 + i - g.plane]) * g.hz;
    }
    const T div = G[0][0] + G[1][1] + G[2][2];
    const int64_t n = (int64_t)k * g.plane + r0 + i;
    constexpr int pa[6] = {0, 1, 2, 1, 0, 0}, pb[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
    for (int v = 0; v < 6; ++v) {
        const T eps = T(0.5) * (G[pa[v]][pb[v]] + G[pb[v]][pa[v]]);
        T add = T(2) * g.B * eps;
        if (v < 3) add += g.lam * div;
        out[v * g.fstride + n] = sd[v * g.fstride + n] + add;
    }
}

template <typename T>
RelaxGeom<T> make_geom(const ddstress_relax_desc& d, double dt, double A, double B) {
    RelaxGeom<T> g{};
    g.nx = d.n[0];
    g.ny = d.n[1];
    g.nz = d.n[2];
    g.plane = (int64_t)g.nx * g.ny;
    g.cstride = (int64_t)(g.nz + 2) * g.plane;
    g.fstride = (int64_t)g.nz * g.plane;
    g.hx = T(1.0 / (2.0 * d.d[0]));
    g.hy = T(1.0 / (2.0 * d.d[1]));
    g.hz = T(1.0 / (2.0 * d.d[2]));
    g.qx = T(1.0 / (d.d[0] * d.d[0]));
    g.qy = T(1.0 / (d.d[1] * d.d[1]));
    g.qz = T(1.0 / (d.d[2] * d.d[2]));
    g.A = T(A);
    g.B = T(B);
    g.dt = T(dt);
    g.twodz = T(2.0 * d.d[2]);
    g.nu = T(d.nu);
    g.inv1mnu = T(1.0 / (1.0 - d.nu));
    g.lam = T(A - 2.0 * B);
    const double E = 2.0 * d.mu * (1.0 + d.nu);
    g.c_shear = T((1.0 + d.nu) / E);
    g.c_normal = T((1.0 + d.nu) * (1.0 - 2.0 * d.nu) / E);
    return g;
}

// Re-raise the status of a nested entry point (its message is already set).
void check_status(ddstress_status s) {
    if (s != DDSTRESS_OK) throw Error{s, ddstress_last_error()};
}

void validate_relax(const ddstress_relax_desc* d) {
    if (!d) fail(DDSTRESS_E_INVALID, "descriptor is NULL");
    if (d->n[0] < 1 || d->n[1] < 1) fail(DDSTRESS_E_INVALID, "Nx and Ny must be >= 1");
    if (d->n[2] < 3) fail(DDSTRESS_E_INVALID, "Nz must be >= 3 (two surface layers and an interior)");
    for (int a = 0; a < 3; ++a) {
        if (!(d->d[a] > 0.0) || !std::isfinite(d->d[a])) fail(DDSTRESS_E_INVALID, "spacings must be finite and > 0");
        if (d->n[a] > kRelaxMaxN) fail(DDSTRESS_E_UNSUPPORTED, "more than 4096 nodes along an axis");
    }
    if (!(d->mu > 0.0) || !std::isfinite(d->mu)) fail(DDSTRESS_E_INVALID, "mu must be finite and > 0");
    if (!(d->nu > -1.0 && d->nu < 0.5)) fail(DDSTRESS_E_INVALID, "nu must lie in (-1, 0.5)");
    if (d->precision != 32 && d->precision != 64) fail(DDSTRESS_E_INVALID, "precision must be 32 or 64");
    if (!(d->dt >= 0.0) || !std::isfinite(d->dt)) fail(DDSTRESS_E_INVALID, "dt must be finite and >= 0");
}

}  // namespace
}  // namespace dds

using namespace dds;

struct ddstress_relax_s {
    ddstress_relax_desc desc;
    double A = 0, B = 0, dt = 0;
    DevBuf u[2], f, phi, red;
    int cur = 0;
    bool loaded = false;
    int64_t steps = 0;

    int64_t nodes() const { return (int64_t)desc.n[0] * desc.n[1] * desc.n[2]; }
    int64_t plane() const { return (int64_t)desc.n[0] * desc.n[1]; }
    size_t elem() const { return desc.precision == 32 ? 4 : 8; }
    dim3 grid(int z) const {
        return dim3((unsigned)((desc.n[0] + kRelaxBX - 1) / kRelaxBX), (unsigned)((desc.n[1] + kRelaxBY - 1) / kRelaxBY),
                    (unsigned)z);
    }

    template <typename T>
    void load(const T* s, hipStream_t st) {
        const RelaxGeom<T> g = make_geom<T>(desc, dt, A, B);
        hipLaunchKernelGGL((k_relax_load<T>), grid(desc.n[2]), dim3(kRelaxBX, kRelaxBY), 0, st, s, f.as<T>(),
                           phi.as<T>(), u[0].as<T>(), g);
        check_hip(hipGetLastError(), "relaxation load launch");
        hipLaunchKernelGGL((k_relax_ghost<T>), grid(2), dim3(kRelaxBX, kRelaxBY), 0, st, u[0].as<T>(), phi.as<T>(), g);
        check_hip(hipGetLastError(), "relaxation ghost launch");
        cur = 0;
    }
    template <typename T>
    void iterate(int n, hipStream_t st) {
        const RelaxGeom<T> g = make_geom<T>(desc, dt, A, B);
        // z-marching tiles of TX x TY columns; z chunks so that about kRelaxBlocks blocks run
        constexpr int TX = DDS_RELAX_TX, TY = DDS_RELAX_TY;
        const int tiles_x = (desc.n[0] + TX - 1) / TX, tiles_y = (desc.n[1] + TY - 1) / TY;
        const int tiles = tiles_x * tiles_y;
        int nchunks = std::max(1, std::min(desc.n[2], (kRelaxBlocks + tiles - 1) / tiles));
        const int kc = (desc.n[2] + nchunks - 1) / nchunks;
        nchunks = (desc.n[2] + kc - 1) / kc;
        const unsigned blocks = (unsigned)(tiles * nchunks);
        for (int s = 0; s < n; ++s) {
            T* a = u[cur].as<T>();
            T* b = u[cur ^ 1].as<T>();
            hipLaunchKernelGGL((k_relax_march<T, TX, TY>), dim3(blocks), dim3(TX * TY), 0, st, a, b, f.as<T>(), g,
                               tiles_x, nchunks, kc);
            check_hip(hipGetLastError(), "relaxation step launch");
            hipLaunchKernelGGL((k_relax_ghost<T>), grid(2), dim3(kRelaxBX, kRelaxBY), 0, st, b, phi.as<T>(), g);
            check_hip(hipGetLastError(), "relaxation ghost launch");
            cur ^= 1;
        }
    }
    template <typename T>
    void norm(hipStream_t st) {
        const RelaxGeom<T> g = make_geom<T>(desc, dt, A, B);
        hipLaunchKernelGGL((k_relax_norm<T>), grid(desc.n[2]), dim3(kRelaxBX, kRelaxBY), 0, st, u[cur].as<T>(),
                           f.as<T>(), g, red.as<unsigned long long>());
        check_hip(hipGetLastError(), "relaxation norm launch");
    }
    template <typename T>
    void stress(const T* sd, T* out, hipStream_t st) {
        const RelaxGeom<T> g = make_geom<T>(desc, dt, A, B);
        hipLaunchKernelGGL((k_relax_stress<T>), grid(desc.n[2]), dim3(kRelaxBX, kRelaxBY), 0, st, u[cur].as<T>(), sd,
                           out, g);
        check_hip(hipGetLastError(), "relaxation stress launch");
    }
};

extern "C" {

ddstress_status ddstress_relax_create(const ddstress_relax_desc* desc, ddstress_relax* out) {
    return guarded([&] {
        if (!out) fail(DDSTRESS_E_INVALID, "output pointer is NULL");
        *out = nullptr;
        validate_relax(desc);
        std::unique_ptr<ddstress_relax_s> r(new ddstress_relax_s());
        r->desc = *desc;
        const double E = 2.0 * desc->mu * (1.0 + desc->nu);
        r->A = E * (1.0 - desc->nu) / ((1.0 + desc->nu) * (1.0 - 2.0 * desc->nu));
        r->B = E / (2.0 * (1.0 + desc->nu));
        const double dmin = std::fmin(desc->d[0], std::fmin(desc->d[1], desc->d[2]));
        r->dt = desc->dt > 0.0 ? desc->dt : dmin * dmin / (5.0 * r->A - 3.0 * r->B);
        if (!(r->dt > 0.0) || !std::isfinite(r->dt))
            fail(DDSTRESS_E_INVALID, "the default step min(d)^2 / (5A - 3B) is not positive for this nu; pass dt");
        const size_t e = r->elem();
        const size_t ub = (size_t)3 * (desc->n[2] + 2) * (size_t)r->plane() * e;
        r->u[0].alloc(ub, "relaxation displacement");
        r->u[1].alloc(ub, "relaxation displacement");
        r->f.alloc((size_t)3 * r->nodes() * e, "relaxation force");
        r->phi.alloc((size_t)6 * r->plane() * e, "relaxation surface terms");
        r->red.alloc(sizeof(unsigned long long), "relaxation norm");
        *out = r.release();
    });
}

ddstress_status ddstress_relax_set_load(ddstress_relax r, const void* sigma_dis, void* stream) {
    return guarded([&] {
        if (!r) fail(DDSTRESS_E_INVALID, "plan is NULL");
        if (!sigma_dis) fail(DDSTRESS_E_INVALID, "sigma_dis is NULL");
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (r->desc.precision == 32) r->load(static_cast<const float*>(sigma_dis), st);
        else r->load(static_cast<const double*>(sigma_dis), st);
        r->loaded = true;
        r->steps = 0;
    });
}

ddstress_status ddstress_relax_iterate(ddstress_relax r, int32_t n_steps, void* stream) {
    return guarded([&] {
        if (!r) fail(DDSTRESS_E_INVALID, "plan is NULL");
        if (n_steps < 0) fail(DDSTRESS_E_INVALID, "n_steps must be >= 0");
        if (!r->loaded) fail(DDSTRESS_E_STATE, "iterate before set_load");
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (r->desc.precision == 32) r->iterate<float>(n_steps, st);
        else r->iterate<double>(n_steps, st);
        r->steps += n_steps;
    });
}

ddstress_status ddstress_relax_update_norm(ddstress_relax r, double* out, void* stream) {
    return guarded([&] {
        if (!r || !out) fail(DDSTRESS_E_INVALID, "NULL argument");
        if (!r->loaded) fail(DDSTRESS_E_STATE, "update_norm before set_load");
        hipStream_t st = static_cast<hipStream_t>(stream);
        check_hip(hipMemsetAsync(r->red.p, 0, sizeof(unsigned long long), st), "clear norm");
        if (r->desc.precision == 32) r->norm<float>(st);
        else r->norm<double>(st);
        unsigned long long bits = 0;
        check_hip(hipMemcpyAsync(&bits, r->red.p, sizeof bits, hipMemcpyDeviceToHost, st), "norm readback");
        check_hip(hipStreamSynchronize(st), "norm");
        std::memcpy(out, &bits, sizeof(double));
    });
}

ddstress_status ddstress_relax_solve(ddstress_relax r, double rel_tol, int32_t max_steps, int32_t check_every,
                                     int32_t* steps_taken, double* final_norm, void* stream) {
    return guarded([&] {
        if (!r) fail(DDSTRESS_E_INVALID, "plan is NULL");
        if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) fail(DDSTRESS_E_INVALID, "rel_tol must be finite and >= 0");
        if (max_steps < 0 || check_every < 1) fail(DDSTRESS_E_INVALID, "max_steps >= 0 and check_every >= 1");
        if (!r->loaded) fail(DDSTRESS_E_STATE, "solve before set_load");
        hipStream_t st = static_cast<hipStream_t>(stream);
        double first = 0.0, now = 0.0;
        check_status(ddstress_relax_update_norm(r, &first, stream));
        now = first;
        int32_t taken = 0;
        while (taken < max_steps && now > rel_tol * first) {
            const int32_t n = std::min(check_every, max_steps - taken);
            if (r->desc.precision == 32) r->iterate<float>(n, st);
            else r->iterate<double>(n, st);
            r->steps += n;
            taken += n;
            check_status(ddstress_relax_update_norm(r, &now, stream));
        }
        if (steps_taken) *steps_taken = taken;
        if (final_norm) *final_norm = now;
    });
}

ddstress_status ddstress_relax_stress(ddstress_relax r, const void* sigma_dis, void* sigma_total, void* stream) {
    return guarded([&] {
        if (!r || !sigma_dis || !sigma_total) fail(DDSTRESS_E_INVALID, "NULL argument");
        if (!r->loaded) fail(DDSTRESS_E_STATE, "stress before set_load");
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (r->desc.precision == 32)
            r->stress(static_cast<const float*>(sigma_dis), static_cast<float*>(sigma_total), st);
        else
            r->stress(static_cast<const double*>(sigma_dis), static_cast<double*>(sigma_total), st);
    });
}

ddstress_status ddstress_relax_displacement(ddstress_relax r, void* u, void* stream) {
    return guarded([&] {
        if (!r || !u) fail(DDSTRESS_E_INVALID, "NULL argument");
        if (!r->loaded) fail(DDSTRESS_E_STATE, "displacement before set_load");
        const size_t bytes = (size_t)3 * (r->desc.n[2] + 2) * (size_t)r->plane() * r->elem();
        check_hip(hipMemcpyAsync(u, r->u[r->cur].p, bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
                  "displacement copy");
    });
}

ddstress_status ddstress_relax_get_info(ddstress_relax r, ddstress_relax_info* info) {
    return guarded([&] {
        if (!r || !info) fail(DDSTRESS_E_INVALID, "NULL argument");
        info->dt = r->dt;
        info->A = r->A;
        info->B = r->B;
        info->work_bytes = r->u[0].bytes + r->u[1].bytes + r->f.bytes + r->phi.bytes + r->red.bytes;
        info->steps = r->steps;
    });
}

ddstress_status ddstress_relax_destroy(ddstress_relax r) {
    return guarded([&] {
        if (!r) return;
        (void)hipDeviceSynchronize();
        delete r;
    });
}

}  // extern "C"
