// C entry points: plan construction, density hand-over and the stress call.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ddstress_internal.hpp"

namespace dds {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

[[noreturn]] void fail(ddstress_status s, const std::string& msg) { throw Error{s, msg}; }

void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? DDSTRESS_E_NOMEM : DDSTRESS_E_DEVICE,
             std::string(what) + ": " + hipGetErrorString(e));
    }
}

namespace {

// Shape facts derived from a descriptor.
struct Shape {
    int N[3];        // grid
    int P[3];        // padded FFT lengths
    int M, M1;       // x half length and non-redundant columns (M + 1)
    int64_t wx;      // row stride of x spectra (complex elements)
    int C, B, L;
    int elem;        // bytes per real
    int tkz, ntz;    // fused z tile and number of kx tiles
    int zg;          // fused z thread groups: 1, or one per channel (C)
    bool mir_y, mir_z;          // spectrum kept for ky <= Py/2 (kz <= Pz/2) only, by mirror parity
    int nkys, nkzs;             // spectrum rows kept along ky and kz
    uint64_t sgn_y, sgn_z;      // bit c*6+v: S_{v,c} odd under ky -> -ky (kz -> -kz)
    bool zstrip;                // the spectrum keeps the fused z pass's Nyquist strip (z_nyq_groups)
    int64_t cells() const { return (int64_t)N[0] * N[1] * N[2]; }
    int64_t padded() const { return (int64_t)P[0] * P[1] * P[2]; }
};

void validate(const ddstress_desc* d) {
    if (!d) fail(DDSTRESS_E_INVALID, "descriptor is NULL");
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1) fail(DDSTRESS_E_INVALID, "grid sizes must be >= 1");
        if (!(d->d[a] > 0.0) || !std::isfinite(d->d[a])) fail(DDSTRESS_E_INVALID, "cell sizes must be finite and > 0");
    }
    for (int a = 0; a < 3; ++a)
        if (d->n[a] > kMaxLen / 2) fail(DDSTRESS_E_UNSUPPORTED, "grid sizes above 512 per axis are not supported");
    if (!(d->mu > 0.0) || !std::isfinite(d->mu)) fail(DDSTRESS_E_INVALID, "mu must be finite and > 0");
    if (!(d->nu > -1.0 && d->nu < 0.5)) fail(DDSTRESS_E_INVALID, "nu must lie in (-1, 0.5)");
    if (d->n_lines < 1 || d->n_lines > 3) fail(DDSTRESS_E_INVALID, "n_lines must be 1, 2 or 3");
    for (int l = 0; l < d->n_lines; ++l) {
        const double n2 = d->t[l][0] * d->t[l][0] + d->t[l][1] * d->t[l][1] + d->t[l][2] * d->t[l][2];
        if (!(n2 > 0.0) || !std::isfinite(n2)) fail(DDSTRESS_E_INVALID, "line directions must be finite and nonzero");
    }
    if (d->precision != 32 && d->precision != 64) fail(DDSTRESS_E_INVALID, "precision must be 32 or 64");
    if (d->batch < 1) fail(DDSTRESS_E_INVALID, "batch must be >= 1");
    if (d->near_shells < 0) fail(DDSTRESS_E_INVALID, "near_shells must be >= 0");
    const uint32_t known = DDSTRESS_FLAG_PERIODIC_X | DDSTRESS_FLAG_PERIODIC_Y | DDSTRESS_FLAG_FULL_SPECTRUM;
    if ((d->flags & ~known) != 0) fail(DDSTRESS_E_UNSUPPORTED, "unknown flag bits");
    for (int a = 0; a < 2; ++a)
        if (periodic_axis(d, a) && (d->n[a] < 2 || (d->n[a] & (d->n[a] - 1)) != 0))
            fail(DDSTRESS_E_UNSUPPORTED, "a periodic axis needs a power-of-two size >= 2");
    if (d->flags & (DDSTRESS_FLAG_PERIODIC_X | DDSTRESS_FLAG_PERIODIC_Y)) {
        if (d->pbc_shells < 0) fail(DDSTRESS_E_INVALID, "pbc_shells must be >= 0");
        if (d->pbc_shells > kMaxPbcShells) fail(DDSTRESS_E_UNSUPPORTED, "pbc_shells above 32 are not supported");
    }
}

// A mirror a -> -a maps every line segment onto itself (possibly reversed)
// when each line direction has t_a = 0 or is parallel to e_a; then every
// coefficient plane is even or odd under that mirror (checked numerically
// when the plan is built).
bool predict_mirror(const ddstress_desc* d, int axis) {
    if (d->flags & DDSTRESS_FLAG_FULL_SPECTRUM) return false;
    for (int l = 0; l < d->n_lines; ++l) {
        const double* t = d->t[l];
        const bool perp = t[axis] == 0.0;
        const bool along = t[(axis + 1) % 3] == 0.0 && t[(axis + 2) % 3] == 0.0;
        if (!perp && !along) return false;
    }
    return true;
}

void set_mirrors(Shape& s, bool my, bool mz) {
    s.mir_y = my && s.P[1] >= 2;
    s.mir_z = mz && s.P[2] >= 2;
    s.nkys = s.mir_y ? s.P[1] / 2 + 1 : s.P[1];
    s.nkzs = s.mir_z ? s.P[2] / 2 + 1 : s.P[2];
}

Shape make_shape(const ddstress_desc* d) {
    Shape s{};
    for (int a = 0; a < 3; ++a) {
        s.N[a] = d->n[a];
        s.P[a] = (a < 2 && periodic_axis(d, a)) ? d->n[a] : std::max(2, next_pow2(2 * d->n[a] - 1));
    }
    s.M = s.P[0] / 2;
    s.M1 = s.M + 1;
    s.wx = round_up(s.M1, 16);
    s.L = d->n_lines;
    s.C = 3 * d->n_lines;
    s.B = d->batch;
    s.elem = d->precision == 32 ? 4 : 8;
    s.zg = default_z_groups(s.P[2], s.C, s.B, s.elem);
    // A strip block carries one realisation with one cache line per value;
    // with few realisations it would outlast the other blocks of the launch.
    s.zstrip = s.B >= kZStripBatch;
    s.tkz = default_z_tk(s.P[2], s.C, s.zg, s.elem);
    s.ntz = (s.M1 + s.tkz - 1) / s.tkz;
    set_mirrors(s, predict_mirror(d, 1), predict_mirror(d, 2));
    s.sgn_y = s.sgn_z = 0;
    // The fused z pass addresses a density (or stress) group of Nz Py Wx
    // complex values through buffer resources with 32-bit byte offsets: the
    // group, bounded here by Pz/2 >= Nz rows, must lie within a signed 32-bit
    // offset.
    const int64_t zrow_bytes = (int64_t)s.P[1] * s.wx * 2 * s.elem;
    if ((int64_t)(s.P[2] / 2) * zrow_bytes > (int64_t)INT32_MAX)
        fail(DDSTRESS_E_UNSUPPORTED, "grid too large for the z pass's 32-bit plane offsets: Pz/2 * Py * Wx complex "
                                     "values (" + std::to_string((s.P[2] / 2) * zrow_bytes) + " bytes) exceed 2^31 - 1");
    return s;
}

size_t spec_bytes(const Shape& s) {
    return (size_t)s.nkys * s.ntz * s.C * 6 * (size_t)s.nkzs * s.tkz * s.elem;
}
size_t twiddle_bytes(const Shape& s) { return (size_t)kTwiddleEntries * 2 * s.elem; }
// complex elements of the two ping-pong work buffers
int64_t work1_elems(const Shape& s) {
    const int64_t a = (int64_t)s.B * s.C * s.N[2] * s.N[1] * s.wx;
    const int64_t b = (int64_t)s.B * 6 * s.N[2] * s.P[1] * s.wx;
    return std::max(a, b);
}
int64_t work2_elems(const Shape& s) {
    const int64_t a = (int64_t)s.B * s.C * s.N[2] * s.P[1] * s.wx;
    const int64_t b = (int64_t)s.B * 6 * s.N[2] * s.N[1] * s.wx;
    return std::max(a, b);
}
size_t density_bytes(const Shape& s) { return (size_t)s.B * s.C * s.cells() * s.elem; }
size_t sigma_bytes(const Shape& s) { return (size_t)s.B * 6 * s.cells() * s.elem; }
size_t build_real_bytes(const Shape& s) { return (size_t)18 * s.padded() * sizeof(double); }
size_t build_cplx_bytes(const Shape& s) {
    return (size_t)18 * s.P[2] * s.P[1] * (size_t)s.wx * sizeof(cplx<double>);
}

}  // namespace
}  // namespace dds

using namespace dds;

struct ddstress_plan_s {
    ddstress_desc desc;
    Shape shape;
    std::shared_ptr<DevBuf> spec;   // kernel spectrum, plan precision (shared by plans of one geometry)
    std::shared_ptr<DevBuf> tw;     // twiddles, plan precision
    DevBuf work1, work2;
    DevBuf rho_own;     // density copy (HOST / DEVICE_COPY)
    DevBuf sigma_tmp;   // stress staging for HOST output
    const void* rho = nullptr;
    bool have_density = false;
    int rows_x = 1, tk_y = 1;      // x rows and y columns per block
    int ex = 16, ey = 16, ez = 8;  // element classes of the x, y and fused z passes
    bool yx = false;               // inverse y and x as one kernel
    bool xy = false;               // forward x and y as one kernel
    double* plane_stats = nullptr; // Eq. 20 output of every stress call (device), or none
    DevBuf rowsq;                  // per-row sums of squares behind it
    double re_max = 0.0, im_max = 0.0;
    // per-pass event timing: events are pooled and reused between folds; each
    // recorded call fills 6 slots with pool indices (a pass fused into the
    // previous one repeats its slot instead of recording another event, since
    // every event record takes stream time)
    bool profiling = false;
    std::vector<hipEvent_t> events;
    std::vector<size_t> slots;
    size_t ev_used = 0;
    double pass_ms[5] = {0, 0, 0, 0, 0};
    int64_t timed_calls = 0;
    // graph replay of the per-call launch sequence, keyed by buffers and batch
    struct GraphEntry {
        const void* rho;
        void* sigma;
        int nb;
        hipGraphExec_t exec;
    };
    bool use_graph = false;
    std::vector<GraphEntry> graphs;     // most recently used last
    hipStream_t cap_stream = nullptr;
    static constexpr size_t kMaxGraphs = 8;
    ~ddstress_plan_s() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        drop_graphs();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
    void drop_graphs() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    void mark(hipStream_t st) {
        if (!profiling) return;
        if (ev_used == events.size()) {
            hipEvent_t e;
            check_hip(hipEventCreate(&e), "event create");
            events.push_back(e);
        }
        check_hip(hipEventRecord(events[ev_used], st), "event record");
        slots.push_back(ev_used++);
    }
    void mark_fused() {     // the pass just enqueued ran inside the previous one: zero time
        if (!profiling) return;
        slots.push_back(slots.back());
    }
    void fold_events() {
        for (size_t i = 0; i + 5 < slots.size(); i += 6) {
            check_hip(hipEventSynchronize(events[slots[i + 5]]), "event sync");
            for (int k = 0; k < 5; ++k) {
                if (slots[i + k] == slots[i + k + 1]) continue;
                float ms = 0.f;
                check_hip(hipEventElapsedTime(&ms, events[slots[i + k]], events[slots[i + k + 1]]), "event time");
                pass_ms[k] += ms;
            }
            ++timed_calls;
        }
        ev_used = 0;
        slots.clear();
    }
};

namespace {

// Plan build, FP64 throughout: (1) when a mirror symmetry is predicted, the
// coefficients of every line are evaluated once and the parity of each of
// their planes under y -> -y and z -> -z is measured; the kept spectrum rows
// and the signs follow (a plane without a definite parity cancels the
// compression along that axis); (2) per line, the coefficients are evaluated,
// transformed (x real-to-complex, y, z) and the imaginary part of the kept
// rows is stored in the plan precision.
template <typename T>
void build_spectrum(ddstress_plan_s* p, hipStream_t st) {
    Shape& s = p->shape;
    DevBuf kr, kc, tw64, maxbits, stats;
    kr.alloc(build_real_bytes(s), "kernel coefficients");
    maxbits.alloc(2 * sizeof(unsigned long long), "spectrum check");
    if (s.mir_y || s.mir_z) {
        const size_t nstat = (size_t)s.L * 18 * 5;
        stats.alloc(nstat * sizeof(unsigned long long), "mirror statistics");
        check_hip(hipMemsetAsync(stats.p, 0, stats.bytes, st), "clear mirror statistics");
        for (int l = 0; l < s.L; ++l) {
            KernelParams kp = make_kernel_params(p->desc, l, s.P);
            launch_kernel_build(kp, kr.as<double>(), st);
            launch_mirror_stats(kr.as<double>(), s.P, stats.as<unsigned long long>() + (size_t)l * 90, st);
        }
        std::vector<unsigned long long> hs(nstat);
        check_hip(hipMemcpyAsync(hs.data(), stats.p, nstat * sizeof(unsigned long long), hipMemcpyDeviceToHost, st),
                  "mirror statistics readback");
        check_hip(hipStreamSynchronize(st), "mirror statistics");
        bool ok_y = s.mir_y, ok_z = s.mir_z;
        uint64_t sy = 0, sz = 0;
        for (int l = 0; l < s.L; ++l)
            for (int q = 0; q < 18; ++q) {          // q = gamma * 6 + v
                double v[5];
                for (int e = 0; e < 5; ++e) std::memcpy(&v[e], &hs[((size_t)l * 18 + q) * 5 + e], sizeof(double));
                const double tol = 1e-13 * v[4];
                const int bit = (3 * l + q / 6) * 6 + q % 6;
                if (v[0] <= tol) {
                } else if (v[1] <= tol) {
                    sy |= 1ull << bit;
                } else {
                    ok_y = false;
                }
                if (v[2] <= tol) {
                } else if (v[3] <= tol) {
                    sz |= 1ull << bit;
                } else {
                    ok_z = false;
                }
            }
        set_mirrors(s, ok_y, ok_z);
        s.sgn_y = ok_y ? sy : 0;
        s.sgn_z = ok_z ? sz : 0;
    }
    p->spec->alloc(spec_bytes(s), "kernel spectrum");
    kc.alloc(build_cplx_bytes(s), "kernel transform");
    tw64.alloc((size_t)kTwiddleEntries * sizeof(cplx<double>), "FP64 twiddles");
    std::vector<cplx<double>> host(kTwiddleEntries);
    fill_twiddles<double>(host.data());
    check_hip(hipMemcpyAsync(tw64.p, host.data(), host.size() * sizeof(cplx<double>), hipMemcpyHostToDevice, st),
              "twiddle upload");
    check_hip(hipMemsetAsync(maxbits.p, 0, 2 * sizeof(unsigned long long), st), "clear spectrum check");
    const cplx<double>* tw = tw64.as<cplx<double>>();
    const int64_t plane_r = s.padded();
    const int64_t plane_c = (int64_t)s.P[2] * s.P[1] * s.wx;
    const int rows = default_rows(s.M, 8);
    const int tky = default_col_tk(s.P[1], 8);
    const int tkz = default_col_tk(s.P[2], 8);
    const double inv_p = 1.0 / (double)plane_r;
    for (int l = 0; l < s.L; ++l) {
        KernelParams kp = make_kernel_params(p->desc, l, s.P);
        launch_kernel_build(kp, kr.as<double>(), st);
        // x: 18 * Pz * Py rows of Px reals (no padding: the coefficients fill the grid)
        launch_x_r2c<double>(s.M, default_ev_col(s.M), kr.as<double>(), kc.as<cplx<double>>(),
                             18LL * s.P[2] * s.P[1], s.P[0], s.P[0], s.wx, tw, rows, st);
        ColGeom gy{};
        gy.ncols = s.M1;
        gy.n_in = s.P[1];
        gy.n_out = s.P[1];
        gy.nouter = 1;
        gy.nplanes = 18LL * s.P[2];
        gy.irs = gy.ors = s.wx;
        gy.ios = gy.oos = 0;
        gy.ips = gy.ops = (int64_t)s.P[1] * s.wx;
        launch_col_fft<double>(s.P[1], default_ev_col(s.P[1]), true, kc.as<cplx<double>>(), kc.as<cplx<double>>(),
                               gy, tw, tky, st);
        ColGeom gz{};
        gz.ncols = s.M1;
        gz.n_in = s.P[2];
        gz.n_out = s.P[2];
        gz.nouter = s.P[1];
        gz.nplanes = 18;
        gz.irs = gz.ors = (int64_t)s.P[1] * s.wx;
        gz.ios = gz.oos = s.wx;
        gz.ips = gz.ops = plane_c;
        launch_col_fft<double>(s.P[2], default_ev_col(s.P[2]), true, kc.as<cplx<double>>(), kc.as<cplx<double>>(),
                               gz, tw, tkz, st);
        launch_extract<T>(kc.as<cplx<double>>(), p->spec->as<T>(), l, s.C, s.M1, s.wx, s.P[1], s.P[2], s.nkys, s.nkzs,
                          s.tkz, s.ntz, s.zstrip, inv_p, maxbits.as<unsigned long long>(), st);
    }
    unsigned long long bits[2] = {0, 0};
    check_hip(hipMemcpyAsync(bits, maxbits.p, sizeof(bits), hipMemcpyDeviceToHost, st), "spectrum check readback");
    check_hip(hipStreamSynchronize(st), "plan build");
    double re, im;
    std::memcpy(&re, &bits[0], sizeof(double));
    std::memcpy(&im, &bits[1], sizeof(double));
    p->re_max = re;
    p->im_max = im;
    // K is odd, so K^ is purely imaginary and only Im K^ is kept: a real part
    // above the rounding of the FP64 transforms would be dropped silently. The
    // scale is max |Im K^|, or, for a kernel that cancels to rounding (a
    // period of two cells on every in-plane axis and one layer), mu min(d),
    // the size of one near-cell coefficient up to a factor of order one.
    const double dmin = std::min(p->desc.d[0], std::min(p->desc.d[1], p->desc.d[2]));
    const double scale = std::max(im, p->desc.mu * dmin);
    if (!(re <= 1e-13 * scale)) {
        char msg[256];
        std::snprintf(msg, sizeof(msg),
                      "kernel spectrum is not purely imaginary (max |Re K^| = %.3e, max |Im K^| = %.3e): the plan "
                      "keeps Im K^ only, which needs an odd kernel",
                      re, im);
        fail(DDSTRESS_E_UNSUPPORTED, msg);
    }
}

template <typename T>
void upload_twiddles(ddstress_plan_s* p, hipStream_t st) {
    std::vector<cplx<T>> host(kTwiddleEntries);
    fill_twiddles<T>(host.data());
    check_hip(hipMemcpyAsync(p->tw->p, host.data(), host.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, st),
              "twiddle upload");
    check_hip(hipStreamSynchronize(st), "twiddle upload");
}

// Pass k (0..4: x forward, y forward, fused z, y inverse, x inverse) of one
// evaluation of the first nb densities. Where the plan fuses forward x and y
// (inverse y and x), pass 0 (3) runs both and pass 1 (4) enqueues nothing.
// Each pass reads only what the previous one wrote, so a pass enqueued
// several times in a row recomputes the same output.
// Plane statistics targets of one call: per-row sums of squares and the
// per-plane results (both NULL: no statistics).
// Layout of the spectrum buffers between the y passes and the fused z pass,
// per group (realisation and channel, or realisation and stress component).
// Plane-major, [group][z][ky][kx]: each (group, z) plane contiguous, Py rows
// of wx complex values. Ky-major, [group][ky][z][kx]: the Nz z-rows of each
// ky together, so a z column's rows lie wx values apart and the fused z pass
// reads and writes neighbouring 128-byte pieces rather than one piece per
// plane; a (group, z) plane then has its rows Nz wx apart. The fused x-y
// kernels, which walk the planes of a group one after the other, take the
// ky-major layout at no cost (interleave Nz); the separate column passes,
// whose blocks own one plane's columns, keep their rows together in the
// plane-major layout. Each buffer takes the layout of its y pass.
// Forward y (separate pass): x-pass output [group][z][y][kx] -> plane-major.
ColGeom fwd_y_geom(const Shape& s, int64_t groups) {
    const int Ny = s.N[1], Nz = s.N[2], Py = s.P[1];
    ColGeom g{};
    g.ncols = s.M1;
    g.n_in = Ny;
    g.n_out = Py;
    g.nouter = 1;
    g.nplanes = groups * Nz;
    g.irs = s.wx;
    g.ips = (int64_t)Ny * s.wx;
    g.ors = s.wx;
    g.ops = (int64_t)Py * s.wx;
    return g;
}
// Inverse y (separate pass): plane-major -> [group][z][y][kx] (Ny rows).
ColGeom inv_y_geom(const Shape& s, int64_t groups) {
    const int Ny = s.N[1], Nz = s.N[2], Py = s.P[1];
    ColGeom g{};
    g.ncols = s.M1;
    g.n_in = Py;
    g.n_out = Ny;
    g.nouter = 1;
    g.nplanes = groups * Nz;
    g.irs = s.wx;
    g.ips = (int64_t)Py * s.wx;
    g.ors = s.wx;
    g.ops = (int64_t)Ny * s.wx;
    return g;
}
// Fused z pass: the density buffer ky-major when kin, the stress buffer when kout.
ZGeom z_geom(const Shape& s, int tk, int nb, bool kin, bool kout) {
    const int Nz = s.N[2], Py = s.P[1];
    ZGeom g{};
    g.nky_s = s.nkys;
    g.nkz_s = s.nkzs;
    g.sgn_y = s.sgn_y;
    g.sgn_z = s.sgn_z;
    g.ncols = s.M1;
    g.ntiles = (s.M1 + tk - 1) / tk;
    g.nky = Py;
    g.nz = Nz;
    g.C = s.C;
    g.B = nb;
    g.irs = kin ? s.wx : (int64_t)Py * s.wx;             // z rows
    g.ios = kin ? (int64_t)Nz * s.wx : s.wx;             // ky rows
    g.iqs = (int64_t)Nz * Py * s.wx;
    g.ors = kout ? s.wx : (int64_t)Py * s.wx;
    g.oos = kout ? (int64_t)Nz * s.wx : s.wx;
    g.oqs = g.iqs;
    g.strip = s.zstrip ? 1 : 0;
    return g;
}

struct StatsTarget {
    double* rowsq;
    double* stats;
};
StatsTarget plan_stats(const ddstress_plan_s* p);

template <typename T>
void enqueue_pass(ddstress_plan_s* p, int k, const T* rho, T* sigma, int nb, hipStream_t st,
                  StatsTarget stt) {
    Shape s = p->shape;
    s.B = nb;       // realisations evaluated by this call (<= the plan's batch)
    cplx<T>* w1 = p->work1.as<cplx<T>>();
    cplx<T>* w2 = p->work2.as<cplx<T>>();
    const cplx<T>* tw = p->tw->as<cplx<T>>();
    const int64_t BC = (int64_t)s.B * s.C;
    const int64_t B6 = (int64_t)s.B * 6;
    const int Nx = s.N[0], Ny = s.N[1], Nz = s.N[2], Py = s.P[1];
    const bool xy = sizeof(T) == 4 && p->xy;
    const bool yx = sizeof(T) == 4 && p->yx;
    if (k == 0) {
        if constexpr (sizeof(T) == 4) {
            if (xy) {
                launch_xy_fwd(rho, w2, BC * Nz, Py, s.M, Ny, Nx, s.wx, tw, st, Nz);   // ky-major
                return;
            }
        }
        // x forward: rows (b, c, z, y) of Nx reals -> M+1 complex
        launch_x_r2c<T>(s.M, p->ex, rho, w1, BC * Nz * Ny, Nx, Nx, s.wx, tw, p->rows_x, st);
    } else if (k == 1) {
        if (xy) return;
        // y forward: Ny rows -> Py rows
        launch_col_fft<T>(Py, p->ey, true, w1, w2, fwd_y_geom(s, BC), tw, p->tk_y, st);
    } else if (k == 2) {
        // z forward + contraction + z inverse
        launch_z_fused<T>(s.P[2], p->ez, s.zg, w2, w1, p->spec->as<T>(), z_geom(s, s.tkz, s.B, xy, yx), tw, s.tkz,
                          st);
    } else if (k == 3 || k == 4) {
        // plane statistics (Eq. 20) from per-row sums of the inverse x pass
        double* rowsq = stt.stats ? stt.rowsq : nullptr;
        double* stats_out = stt.stats;
        const double inv_plane = 1.0 / ((double)Nx * (double)Ny);
        if (k == 3) {
            if constexpr (sizeof(T) == 4) {
                if (yx) {
                    launch_yx_inv(w1, sigma, B6 * Nz, Py, s.M, Ny, Nx, s.wx, tw, st, rowsq, Nz);   // ky-major
                    if (rowsq) launch_rowsq_finish(rowsq, B6 * Nz, Ny, inv_plane, stats_out, st);
                    return;
                }
            }
            // y inverse: Py rows -> Ny rows
            launch_col_fft<T>(Py, p->ey, false, w1, w2, inv_y_geom(s, B6), tw, p->tk_y, st);
        } else {
            if (yx) return;
            // x inverse: rows (b, v, z, y) -> Nx reals
            launch_x_c2r<T>(s.M, p->ex, w2, sigma, B6 * Nz * Ny, Nx, s.wx, Nx, tw, p->rows_x, st, rowsq);
            if (rowsq) launch_rowsq_finish(rowsq, B6 * Nz, Ny, inv_plane, stats_out, st);
        }
    }
}

StatsTarget plan_stats(const ddstress_plan_s* p) {
    return {p->plane_stats ? p->rowsq.as<double>() : nullptr, p->plane_stats};
}

// Whether pass k runs inside the previous pass's kernel (and enqueues nothing).
bool pass_fused_away(const ddstress_plan_s* p, int k) {
    if (p->shape.elem != 4) return false;
    return (k == 1 && p->xy) || (k == 4 && p->yx);
}

template <typename T>
void run_stress(ddstress_plan_s* p, const T* rho, T* sigma, int nb, hipStream_t st) {
    p->mark(st);
    for (int k = 0; k < 5; ++k) {
        enqueue_pass<T>(p, k, rho, sigma, nb, st, plan_stats(p));
        if (pass_fused_away(p, k)) p->mark_fused();     // no event: its time shows as zero
        else p->mark(st);
    }
}

// Row sums of squares for ddstress_stress_batch_stats_noalloc: a file-scope
// device array (each GPU the library runs on holds its own copy until the
// process ends), addressed from the host through the per-device address that
// hipGetSymbolAddress returns, never through the array's host-side name.
constexpr size_t kNoAllocRowsq = size_t(1) << 21;      // doubles (16 MiB)
static __device__ __align__(256) double scratch[kNoAllocRowsq];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array (looked up once per device).
double* device_scratch() {
    int dev = -1;
    check_hip(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxDevices) fail(DDSTRESS_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (!ptr) fail(DDSTRESS_E_DEVICE, "scratch symbol address is NULL");
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}

template <typename T>
void capture_stress(ddstress_plan_s* p, const T* rho, T* sigma, int nb, hipGraphExec_t* exec) {
    if (!p->cap_stream) check_hip(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "capture stream");
    check_hip(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipGraph_t g = nullptr;
    try {
        run_stress<T>(p, rho, sigma, nb, p->cap_stream);
    } catch (...) {
        (void)hipStreamEndCapture(p->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    check_hip(hipStreamEndCapture(p->cap_stream, &g), "end capture");
    hipError_t e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    check_hip(e, "graph instantiate");
}

// Enqueue one evaluation: a replayed graph when enabled (and not profiling), else direct launches.
template <typename T>
void enqueue_stress(ddstress_plan_s* p, const T* rho, T* sigma, int nb, hipStream_t st) {
    if (!p->use_graph || p->profiling) {
        run_stress<T>(p, rho, sigma, nb, st);
        return;
    }
    auto& gs = p->graphs;
    size_t i = 0;
    for (; i < gs.size(); ++i)
        if (gs[i].rho == rho && gs[i].sigma == sigma && gs[i].nb == nb) break;
    if (i == gs.size()) {
        if (gs.size() == ddstress_plan_s::kMaxGraphs) {
            (void)hipGraphExecDestroy(gs.front().exec);
            gs.erase(gs.begin());
        }
        ddstress_plan_s::GraphEntry ge{rho, sigma, nb, nullptr};
        capture_stress<T>(p, rho, sigma, nb, &ge.exec);
        gs.push_back(ge);
        i = gs.size() - 1;
    } else if (i + 1 != gs.size()) {
        std::rotate(gs.begin() + i, gs.begin() + i + 1, gs.end());
        i = gs.size() - 1;
    }
    check_hip(hipGraphLaunch(gs[i].exec, st), "graph launch");
}

// Launch-shape limits shared by the defaults, the autotuner and tuned plans.
constexpr int kMaxThreads = 512;
constexpr size_t kMaxLds = 64 * 1024;
bool rows_ok(const Shape& s, int r, int ev) {
    const int e = s.M < ev ? s.M : ev;
    return r >= 1 && ev_col_ok(ev) && x_threads(s.M, r, ev) <= kMaxThreads &&
           (size_t)r * x_lds_ld(s.M, e, s.elem) * 2 * s.elem <= kMaxLds;
}
bool col_ok(const Shape& s, int N, int tk, int ev) {
    return tk >= 1 && ev_col_ok(ev) && col_threads(N, tk, ev) <= kMaxThreads &&
           (size_t)N * tk * 2 * s.elem <= kMaxLds;
}
bool z_ok(const Shape& s, int tk, int ev, int groups) {
    if (s.elem == 4 && s.P[2] == 64 && ev == 8)         // the wave form: fixed tile, one group
        return z_wave_form(s.P[2], ev, groups, s.elem) && tk == kZWaveTile &&
               z_wave_lds_bytes(s.P[2], s.C, s.nkzs, s.B) <= kMaxLds;
    return tk >= 1 && z_groups_ok(groups, s.C) && ev_z_ok(s.P[2], ev, s.elem) &&
           z_threads(s.P[2], groups, tk, ev) <= z_max_threads(groups) &&
           z_lds_bytes(s.P[2], tk, s.C, groups, s.elem) <= kMaxLds;
}

struct LaunchChoice {
    int rows_x, ex, tk_y, ey, ez, zg;
    bool yx, xy;
};

bool yx_ok(const Shape& s) { return yx_inv_fits(s.P[1], s.M, s.N[1], s.elem); }

LaunchChoice default_launch(const Shape& s) {
    return {default_rows(s.M, s.elem), default_ev_col(s.M), default_col_tk(s.P[1], s.elem), default_ev_col(s.P[1]),
            default_ev_z(s.P[2], s.zg, s.elem), s.zg, yx_ok(s), yx_ok(s)};
}

// Apply a tuning (zero element classes select the defaults) after checking it.
LaunchChoice apply_tuning(Shape& s, const ddstress_tuning* t) {
    LaunchChoice c = default_launch(s);
    if (!t) return c;
    const int zg = t->z_groups ? t->z_groups : c.zg;
    const int ex = t->ex ? t->ex : c.ex, ey = t->ey ? t->ey : c.ey;
    const int ez = t->ez ? t->ez : default_ev_z(s.P[2], zg, s.elem);
    if (!rows_ok(s, t->rows_x, ex) || !col_ok(s, s.P[1], t->tk_y, ey) || !z_ok(s, t->tk_z, ez, zg))
        fail(DDSTRESS_E_INVALID, "tuning choice outside the launch limits of this shape");
    if (t->yx < 0 || t->yx > 2 || (t->yx == 2 && !yx_ok(s)) || t->xy < 0 || t->xy > 2 || (t->xy == 2 && !yx_ok(s)))
        fail(DDSTRESS_E_INVALID, "fused x-y passes do not apply to this shape");
    c = {t->rows_x, ex, t->tk_y, ey, ez, zg, t->yx == 0 ? yx_ok(s) : t->yx == 2, t->xy == 0 ? yx_ok(s) : t->xy == 2};
    s.zg = zg;
    s.tkz = t->tk_z;
    s.ntz = (s.M1 + s.tkz - 1) / s.tkz;
    return c;
}

void create_plan(const ddstress_desc* desc, const ddstress_tuning* tuning, hipStream_t st, ddstress_plan* out) {
    if (!out) fail(DDSTRESS_E_INVALID, "output plan pointer is NULL");
    *out = nullptr;
    validate(desc);
    auto* p = new ddstress_plan_s();
    try {
        p->desc = *desc;
        p->shape = make_shape(desc);
        const LaunchChoice lc = apply_tuning(p->shape, tuning);
        p->rows_x = lc.rows_x;
        p->ex = lc.ex;
        p->tk_y = lc.tk_y;
        p->ey = lc.ey;
        p->ez = lc.ez;
        p->yx = lc.yx;
        p->xy = lc.xy;
        const Shape& s = p->shape;
        p->spec = std::make_shared<DevBuf>();
        p->tw = std::make_shared<DevBuf>();
        p->tw->alloc(twiddle_bytes(s), "twiddles");
        p->work1.alloc((size_t)work1_elems(s) * 2 * s.elem, "work buffer 1");
        p->work2.alloc((size_t)work2_elems(s) * 2 * s.elem, "work buffer 2");
        if (s.elem == 4) {
            upload_twiddles<float>(p, st);
            build_spectrum<float>(p, st);
        } else {
            upload_twiddles<double>(p, st);
            build_spectrum<double>(p, st);
        }
    } catch (...) {
        delete p;
        throw;
    }
    *out = p;
}

// Median device time of `reps` runs of f on stream st (after two warm-up runs).
template <class F>
float time_median(hipStream_t st, int reps, F&& f) {
    hipEvent_t a, b;
    check_hip(hipEventCreate(&a), "event create");
    check_hip(hipEventCreate(&b), "event create");
    std::vector<float> t;
    try {
        for (int i = 0; i < 2; ++i) f();
        for (int i = 0; i < reps; ++i) {
            check_hip(hipEventRecord(a, st), "event record");
            f();
            check_hip(hipEventRecord(b, st), "event record");
            check_hip(hipEventSynchronize(b), "event sync");
            float ms = 0.f;
            check_hip(hipEventElapsedTime(&ms, a, b), "event time");
            t.push_back(ms);
        }
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

// Time every admissible tile choice of each pass on zero-filled buffers of the
// plan's shape and keep the fastest. Tile choices do not change the arithmetic.
template <typename T>
void autotune_impl(const ddstress_desc* desc, hipStream_t st, ddstress_tuning* out) {
    Shape s = make_shape(desc);
    const int64_t BC = (int64_t)s.B * s.C, B6 = (int64_t)s.B * 6;
    const int Nx = s.N[0], Ny = s.N[1], Nz = s.N[2], Py = s.P[1], Pz = s.P[2];
    std::vector<int> zev;
    for (int ev = 2; ev <= 16; ev *= 2)
        if (ev_z_ok(Pz, ev, s.elem)) zev.push_back(ev);
    struct ZChoice { int tk, ev, groups; };
    std::vector<ZChoice> zlist;
    for (int groups : {1, s.C})
        for (int ev : zev)
            for (int tk = 1; tk <= 256; tk *= 2)
                if (z_ok(s, tk, ev, groups) && z_threads(Pz, groups, tk, ev) >= 64) zlist.push_back({tk, ev, groups});
    if (zlist.empty()) zlist.push_back({s.tkz, default_ev_z(Pz, s.zg, s.elem), s.zg});
    size_t spec_max = 0;
    for (auto& z : zlist) {
        Shape t = s;
        t.tkz = z.tk;
        t.ntz = (s.M1 + z.tk - 1) / z.tk;
        spec_max = std::max(spec_max, spec_bytes(t));
    }
    DevBuf rho, sig, w1, w2, spec, tw;
    rho.alloc(density_bytes(s), "tuning density");
    sig.alloc(sigma_bytes(s), "tuning stress");
    w1.alloc((size_t)work1_elems(s) * 2 * s.elem, "tuning work 1");
    w2.alloc((size_t)work2_elems(s) * 2 * s.elem, "tuning work 2");
    spec.alloc(spec_max, "tuning spectrum");
    tw.alloc(twiddle_bytes(s), "tuning twiddles");
    check_hip(hipMemsetAsync(rho.p, 0, rho.bytes, st), "clear");
    check_hip(hipMemsetAsync(w1.p, 0, w1.bytes, st), "clear");
    check_hip(hipMemsetAsync(w2.p, 0, w2.bytes, st), "clear");
    check_hip(hipMemsetAsync(spec.p, 0, spec.bytes, st), "clear");
    std::vector<cplx<T>> host(kTwiddleEntries);
    fill_twiddles<T>(host.data());
    check_hip(hipMemcpyAsync(tw.p, host.data(), host.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, st), "upload");
    check_hip(hipStreamSynchronize(st), "tuning setup");
    const cplx<T>* twp = tw.as<cplx<T>>();
    const int reps = 5;
    const bool verbose = std::getenv("DDSTRESS_TUNE_VERBOSE") != nullptr;

    float best = 1e30f;
    for (int ev : {8, 16})
        for (int r = 1; r <= kMaxThreads; r *= 2) {
            if (!rows_ok(s, r, ev) || (ev == 16 && s.M <= 8)) continue;
            float ms = time_median(st, reps, [&] {
                launch_x_r2c<T>(s.M, ev, rho.as<T>(), w1.as<cplx<T>>(), BC * Nz * Ny, Nx, Nx, s.wx, twp, r, st);
                launch_x_c2r<T>(s.M, ev, w2.as<cplx<T>>(), sig.as<T>(), B6 * Nz * Ny, Nx, s.wx, Nx, twp, r, st);
            });
            if (verbose) std::fprintf(stderr, "[tune] x rows=%d ev=%d %.5f ms\n", r, ev, ms);
            if (ms < best) { best = ms; out->rows_x = r; out->ex = ev; out->ms[0] = ms; }
        }
    best = 1e30f;
    for (int ev : {8, 16})
        for (int tk = 1; tk <= 256; tk *= 2) {
            if (!col_ok(s, Py, tk, ev) || col_threads(Py, tk, ev) < 64 || (ev == 16 && Py <= 8)) continue;
            const ColGeom gy = fwd_y_geom(s, BC);
            const ColGeom gi = inv_y_geom(s, B6);
            float ms = time_median(st, reps, [&] {
                launch_col_fft<T>(Py, ev, true, w1.as<cplx<T>>(), w2.as<cplx<T>>(), gy, twp, tk, st);
                launch_col_fft<T>(Py, ev, false, w1.as<cplx<T>>(), w2.as<cplx<T>>(), gi, twp, tk, st);
            });
            if (verbose) std::fprintf(stderr, "[tune] y tk=%d ev=%d %.5f ms\n", tk, ev, ms);
            if (ms < best) { best = ms; out->tk_y = tk; out->ey = ev; out->ms[1] = ms; }
        }
    best = 1e30f;
    for (auto& z : zlist) {
        const int tk = z.tk, ev = z.ev, groups = z.groups;
        // the layouts of fused x-y passes where they apply (they are chosen below)
        ZGeom gz = z_geom(s, tk, s.B, sizeof(T) == 4 && yx_ok(s), sizeof(T) == 4 && yx_ok(s));
        gz.sgn_y = gz.sgn_z = 0;                 // (the tuning spectrum is zeros)
        float ms = time_median(st, reps, [&] {
            launch_z_fused<T>(Pz, ev, groups, w2.as<cplx<T>>(), w1.as<cplx<T>>(), spec.as<T>(), gz, twp, tk, st);
        });
        if (verbose) std::fprintf(stderr, "[tune] z tk=%d ev=%d groups=%d %.5f ms\n", tk, ev, groups, ms);
        if (ms < best) {
            best = ms;
            out->tk_z = tk;
            out->ez = ev;
            out->z_groups = groups;
            out->ms[2] = ms;
        }
    }
    // inverse y and x, forward x and y: the chosen separate passes against the fused kernels
    out->yx = 1;
    out->xy = 1;
    if constexpr (sizeof(T) == 4) {
        if (yx_ok(s)) {
            const ColGeom gi = inv_y_geom(s, B6);
            const float sep = time_median(st, reps, [&] {
                launch_col_fft<T>(Py, out->ey, false, w1.as<cplx<T>>(), w2.as<cplx<T>>(), gi, twp, out->tk_y, st);
                launch_x_c2r<T>(s.M, out->ex, w2.as<cplx<T>>(), sig.as<T>(), B6 * Nz * Ny, Nx, s.wx, Nx, twp,
                                out->rows_x, st);
            });
            const float fused = time_median(st, reps, [&] {
                launch_yx_inv(w1.as<cplx<float>>(), sig.as<float>(), B6 * Nz, Py, s.M, Ny, Nx, s.wx, twp, st,
                              nullptr, Nz);
            });
            if (verbose) std::fprintf(stderr, "[tune] inverse y+x separate %.5f ms fused %.5f ms\n", sep, fused);
            if (fused < sep) out->yx = 2;
            const ColGeom gy = fwd_y_geom(s, BC);
            const float sepf = time_median(st, reps, [&] {
                launch_x_r2c<T>(s.M, out->ex, rho.as<T>(), w1.as<cplx<T>>(), BC * Nz * Ny, Nx, Nx, s.wx, twp,
                                out->rows_x, st);
                launch_col_fft<T>(Py, out->ey, true, w1.as<cplx<T>>(), w2.as<cplx<T>>(), gy, twp, out->tk_y, st);
            });
            const float fusedf = time_median(st, reps, [&] {
                launch_xy_fwd(rho.as<float>(), w2.as<cplx<float>>(), BC * Nz, Py, s.M, Ny, Nx, s.wx, twp, st, Nz);
            });
            if (verbose) std::fprintf(stderr, "[tune] forward x+y separate %.5f ms fused %.5f ms\n", sepf, fusedf);
            out->xy = fusedf < sepf ? 2 : 1;
        }
    }
    check_hip(hipStreamSynchronize(st), "tuning");
}

}  // namespace

extern "C" {

ddstress_status ddstress_plan_footprint(const ddstress_desc* desc, size_t* cached_bytes, size_t* work_bytes,
                                        size_t* build_bytes) {
    return guarded([&] {
        validate(desc);
        const Shape s = make_shape(desc);
        if (cached_bytes) *cached_bytes = spec_bytes(s) + twiddle_bytes(s);
        if (work_bytes)
            *work_bytes = (size_t)(work1_elems(s) + work2_elems(s)) * 2 * s.elem + density_bytes(s);
        if (build_bytes) *build_bytes = build_real_bytes(s) + build_cplx_bytes(s);
    });
}

ddstress_status ddstress_plan_create(const ddstress_desc* desc, void* stream, ddstress_plan* out) {
    return guarded([&] { create_plan(desc, nullptr, static_cast<hipStream_t>(stream), out); });
}

ddstress_status ddstress_set_density(ddstress_plan plan, const void* rho, int32_t where, void* stream) {
    return guarded([&] {
        if (!plan) fail(DDSTRESS_E_INVALID, "plan is NULL");
        if (!rho) fail(DDSTRESS_E_INVALID, "density pointer is NULL");
        hipStream_t st = static_cast<hipStream_t>(stream);
        const size_t bytes = density_bytes(plan->shape);
        if (where == DDSTRESS_DEVICE_BORROW) {
            plan->rho = rho;
        } else if (where == DDSTRESS_HOST || where == DDSTRESS_DEVICE_COPY) {
            if (!plan->rho_own.p) plan->rho_own.alloc(bytes, "density buffer");
            check_hip(hipMemcpyAsync(plan->rho_own.p, rho, bytes,
                                     where == DDSTRESS_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st),
                      "density copy");
            plan->rho = plan->rho_own.p;
        } else {
            fail(DDSTRESS_E_INVALID, "unknown buffer location");
        }
        plan->have_density = true;
    });
}

ddstress_status ddstress_stress(ddstress_plan plan, void* sigma, int32_t where, void* stream) {
    return guarded([&] {
        if (!plan) fail(DDSTRESS_E_INVALID, "plan is NULL");
        if (!sigma) fail(DDSTRESS_E_INVALID, "stress pointer is NULL");
        if (!plan->have_density) fail(DDSTRESS_E_STATE, "no density set on this plan");
        if (where != DDSTRESS_HOST && where != DDSTRESS_DEVICE_COPY && where != DDSTRESS_DEVICE_BORROW)
            fail(DDSTRESS_E_INVALID, "unknown buffer location");
        hipStream_t st = static_cast<hipStream_t>(stream);
        void* dst = sigma;
        const size_t bytes = sigma_bytes(plan->shape);
        if (where == DDSTRESS_HOST) {
            if (!plan->sigma_tmp.p) plan->sigma_tmp.alloc(bytes, "stress staging buffer");
            dst = plan->sigma_tmp.p;
        }
        if (plan->shape.elem == 4)
            enqueue_stress<float>(plan, static_cast<const float*>(plan->rho), static_cast<float*>(dst), plan->shape.B,
                                  st);
        else
            enqueue_stress<double>(plan, static_cast<const double*>(plan->rho), static_cast<double*>(dst),
                                   plan->shape.B, st);
        if (where == DDSTRESS_HOST)
            check_hip(hipMemcpyAsync(sigma, dst, bytes, hipMemcpyDeviceToHost, st), "stress copy to host");
    });
}

ddstress_status ddstress_autotune(const ddstress_desc* desc, void* stream, ddstress_tuning* out) {
    return guarded([&] {
        validate(desc);
        if (!out) fail(DDSTRESS_E_INVALID, "output pointer is NULL");
        std::memset(out, 0, sizeof(*out));
        if (desc->precision == 32)
            autotune_impl<float>(desc, static_cast<hipStream_t>(stream), out);
        else
            autotune_impl<double>(desc, static_cast<hipStream_t>(stream), out);
    });
}

ddstress_status ddstress_plan_create_tuned(const ddstress_desc* desc, const ddstress_tuning* tuning, void* stream,
                                           ddstress_plan* out) {
    return guarded([&] {
        if (!tuning) fail(DDSTRESS_E_INVALID, "tuning is NULL");
        create_plan(desc, tuning, static_cast<hipStream_t>(stream), out);
    });
}

ddstress_status ddstress_plan_share(ddstress_plan src, int32_t batch, ddstress_plan* out) {
    return guarded([&] {
        if (!src || !out) fail(DDSTRESS_E_INVALID, "NULL argument");
        if (batch < 1) fail(DDSTRESS_E_INVALID, "batch must be >= 1");
        *out = nullptr;
        auto* p = new ddstress_plan_s();
        try {
            p->desc = src->desc;
            p->desc.batch = batch;
            p->shape = make_shape(&p->desc);
            p->shape.tkz = src->shape.tkz;      // the shared spectrum's layout
            p->shape.ntz = src->shape.ntz;
            p->shape.zg = src->shape.zg;
            p->shape.mir_y = src->shape.mir_y;
            p->shape.mir_z = src->shape.mir_z;
            p->shape.nkys = src->shape.nkys;
            p->shape.nkzs = src->shape.nkzs;
            p->shape.sgn_y = src->shape.sgn_y;
            p->shape.sgn_z = src->shape.sgn_z;
            p->shape.zstrip = src->shape.zstrip;
            p->spec = src->spec;
            p->tw = src->tw;
            p->rows_x = src->rows_x;
            p->tk_y = src->tk_y;
            p->ex = src->ex;
            p->ey = src->ey;
            p->ez = src->ez;
            p->yx = src->yx;
            p->xy = src->xy;
            p->re_max = src->re_max;
            p->im_max = src->im_max;
            const Shape& s = p->shape;
            p->work1.alloc((size_t)work1_elems(s) * 2 * s.elem, "work buffer 1");
            p->work2.alloc((size_t)work2_elems(s) * 2 * s.elem, "work buffer 2");
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
    });
}

ddstress_status ddstress_stress_batch(ddstress_plan plan, const void* rho, void* sigma, int32_t nbatch,
                                      void* stream) {
    return guarded([&] {
        if (!plan) fail(DDSTRESS_E_INVALID, "plan is NULL");
        if (!rho || !sigma) fail(DDSTRESS_E_INVALID, "NULL buffer");
        if (nbatch < 1 || nbatch > plan->shape.B) fail(DDSTRESS_E_INVALID, "nbatch must lie in [1, batch]");
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (plan->shape.elem == 4)
            enqueue_stress<float>(plan, static_cast<const float*>(rho), static_cast<float*>(sigma), nbatch, st);
        else
            enqueue_stress<double>(plan, static_cast<const double*>(rho), static_cast<double*>(sigma), nbatch, st);
    });
}

ddstress_status ddstress_stress_batch_stats_noalloc(ddstress_plan plan, const void* rho, void* sigma, int32_t nbatch,
                                                   double* stats, void* stream) {
    return guarded([&] {
        if (!plan) fail(DDSTRESS_E_INVALID, "plan is NULL");
        if (!rho || !sigma || !stats) fail(DDSTRESS_E_INVALID, "NULL buffer");
        if (nbatch < 1 || nbatch > plan->shape.B) fail(DDSTRESS_E_INVALID, "nbatch must lie in [1, batch]");
        const Shape& s = plan->shape;
        const size_t rows = (size_t)nbatch * 6 * s.N[2] * (size_t)s.N[1];
        if (rows > kNoAllocRowsq)
            fail(DDSTRESS_E_UNSUPPORTED, "nbatch * 6 * Nz * Ny = " + std::to_string(rows) +
                                             " row sums exceed the static scratch of " +
                                             std::to_string(kNoAllocRowsq) + " doubles");
        const StatsTarget stt{device_scratch(), stats};
        hipStream_t st = static_cast<hipStream_t>(stream);
        for (int k = 0; k < 5; ++k) {
            if (s.elem == 4)
                enqueue_pass<float>(plan, k, static_cast<const float*>(rho), static_cast<float*>(sigma), nbatch, st,
                                    stt);
            else
                enqueue_pass<double>(plan, k, static_cast<const double*>(rho), static_cast<double*>(sigma), nbatch,
                                     st, stt);
        }
    });
}

ddstress_status ddstress_plan_get_info(ddstress_plan plan, ddstress_info* info) {
    return guarded([&] {
        if (!plan || !info) fail(DDSTRESS_E_INVALID, "NULL argument");
        const Shape& s = plan->shape;
        std::memset(info, 0, sizeof(*info));
        KernelParams kp = make_kernel_params(plan->desc, 0, s.P);
        for (int a = 0; a < 3; ++a) {
            info->padded[a] = s.P[a];
            info->subdiv[a] = kp.m[a];
        }
        info->channels = s.C;
        info->batch = s.B;
        info->precision = plan->desc.precision;
        info->tile_z = s.tkz;
        info->tile_y = plan->tk_y;
        info->rows_x = plan->rows_x;
        info->mirror_y = s.mir_y ? 1 : 0;
        info->mirror_z = s.mir_z ? 1 : 0;
        info->ex = plan->ex;
        info->ey = plan->ey;
        info->ez = plan->ez;
        info->z_groups = s.zg;
        info->yx_fused = plan->yx ? 1 : 0;
        info->xy_fused = plan->xy ? 1 : 0;
        info->cached_bytes = plan->spec->bytes + plan->tw->bytes;
        info->work_bytes = plan->work1.bytes + plan->work2.bytes + plan->rho_own.bytes + plan->sigma_tmp.bytes;
        info->kernel_real_max = plan->re_max;
        info->kernel_imag_max = plan->im_max;
    });
}

ddstress_status ddstress_plan_set_profiling(ddstress_plan plan, int32_t enable) {
    return guarded([&] {
        if (!plan) fail(DDSTRESS_E_INVALID, "plan is NULL");
        plan->ev_used = 0;
        plan->slots.clear();
        plan->profiling = enable != 0;
        for (double& v : plan->pass_ms) v = 0.0;
        plan->timed_calls = 0;
    });
}

ddstress_status ddstress_plan_set_graph(ddstress_plan plan, int32_t enable) {
    return guarded([&] {
        if (!plan) fail(DDSTRESS_E_INVALID, "plan is NULL");
        plan->use_graph = enable != 0;
        if (!plan->use_graph) plan->drop_graphs();
    });
}

ddstress_status ddstress_plan_get_pass_times(ddstress_plan plan, double ms[5], int64_t* calls) {
    return guarded([&] {
        if (!plan || !ms) fail(DDSTRESS_E_INVALID, "NULL argument");
        plan->fold_events();
        for (int k = 0; k < 5; ++k) ms[k] = plan->pass_ms[k];
        if (calls) *calls = plan->timed_calls;
    });
}

ddstress_status ddstress_plan_time_passes(ddstress_plan plan, void* sigma, int32_t reps, double ms[5],
                                          void* stream) {
    return guarded([&] {
        if (!plan || !sigma || !ms) fail(DDSTRESS_E_INVALID, "NULL argument");
        if (reps < 1) fail(DDSTRESS_E_INVALID, "reps must be >= 1");
        if (!plan->have_density) fail(DDSTRESS_E_STATE, "no density set on this plan");
        hipStream_t st = static_cast<hipStream_t>(stream);
        hipEvent_t ev[10] = {};
        try {
            for (auto& e : ev) check_hip(hipEventCreate(&e), "event create");
            for (int k = 0; k < 5; ++k) {
                check_hip(hipEventRecord(ev[2 * k], st), "event record");
                if (!pass_fused_away(plan, k))
                    for (int r = 0; r < reps; ++r) {
                        if (plan->shape.elem == 4)
                            enqueue_pass<float>(plan, k, static_cast<const float*>(plan->rho),
                                                static_cast<float*>(sigma), plan->shape.B, st, plan_stats(plan));
                        else
                            enqueue_pass<double>(plan, k, static_cast<const double*>(plan->rho),
                                                 static_cast<double*>(sigma), plan->shape.B, st, plan_stats(plan));
                    }
                check_hip(hipEventRecord(ev[2 * k + 1], st), "event record");
            }
            check_hip(hipEventSynchronize(ev[9]), "event sync");
            for (int k = 0; k < 5; ++k) {
                float t = 0.f;
                check_hip(hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]), "event time");
                ms[k] = pass_fused_away(plan, k) ? 0.0 : (double)t / reps;
            }
        } catch (...) {
            for (auto& e : ev)
                if (e) (void)hipEventDestroy(e);
            throw;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
    });
}

ddstress_status ddstress_plan_destroy(ddstress_plan plan) {
    return guarded([&] {
        if (!plan) return;
        (void)hipDeviceSynchronize();
        delete plan;
    });
}

ddstress_status ddstress_plan_set_plane_stats(ddstress_plan plan, double* stats) {
    return guarded([&] {
        if (!plan) fail(DDSTRESS_E_INVALID, "plan is NULL");
        if (stats && !plan->rowsq.p)
            plan->rowsq.alloc((size_t)plan->shape.B * 6 * plan->shape.N[2] * (size_t)plan->shape.N[1] * sizeof(double),
                              "plane statistics row sums");
        if (stats != plan->plane_stats) plan->drop_graphs();      // captured launches carry the pointers
        plan->plane_stats = stats;
    });
}

ddstress_status ddstress_kernel_realspace(const ddstress_desc* desc, int32_t line, double* out, void* stream) {
    return guarded([&] {
        validate(desc);
        if (line < 0 || line >= desc->n_lines) fail(DDSTRESS_E_INVALID, "line index out of range");
        if (!out) fail(DDSTRESS_E_INVALID, "output pointer is NULL");
        const Shape s = make_shape(desc);
        KernelParams kp = make_kernel_params(*desc, line, s.P);
        launch_kernel_build(kp, out, static_cast<hipStream_t>(stream));
    });
}

const char* ddstress_last_error(void) { return g_last_error.c_str(); }

const char* ddstress_version(void) { return "ddstress 0.1.0 (gfx950)"; }

}  // extern "C"
