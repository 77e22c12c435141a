/*
 * ddstress: stress of a site-dependent dislocation density on a rectangular
 * grid of (possibly shape-anisotropic) cells, evaluated as the zero-padded FFT
 * convolution of the density with precomputed interaction coefficients.
 *
 * Method: Berkov & Gorn, arXiv:1804.01830.
 *   - Stress of a volume element and of the whole density: Sec. 2.1, Eq. (2),
 *     Eq. (3a), Eq. (3b).
 *   - Segment stress: Sec. 2.2, Eq. (6)-(7) (coordinate-free form).
 *   - Interaction function f = sigma^AB / (Delta l b): Sec. 2.2, Eq. (9b).
 *   - Discrete sum over cells and its FFT evaluation: Sec. 2.3, Eq. (10).
 *   - Near-cell subdivision without multipole moments, zero self-term:
 *     Sec. 2.3, Fig. 3.
 *
 * The computed quantity, for every cell r0 of the grid,
 *     sigma_v(r0) = sum_{cells i} sum_{c < C} K_{v,c}(r0 - r_i) rho_c(r_i),
 * is Eq. (10) summed over the dislocation types of Eq. (3b). Cell (i, j, k)
 * has its centre at (i dx, j dy, k dz). By default the sample sits in an
 * infinite medium: open boundaries, no periodic images. With
 * DDSTRESS_FLAG_PERIODIC_X and/or _Y the sample is continued periodically in
 * the layer plane (Sec. 4): K is replaced by its sum over replica shells,
 * Eq. (12)-(13), and the sum over cells runs over one period.
 *
 * Density channels. A plan has L line directions t_l (1 <= L <= 3) and
 * C = 3L density channels; channel c = 3 l + gamma holds the line density
 * (dislocations per unit area, unit length^-2) of direction t_l multiplied by
 * their Burgers component gamma (x, y, z), so rho_c has unit length^-1 and a
 * Burgers vector that varies from cell to cell is folded into the channels.
 *
 * Stress output. Six components per cell in Voigt order
 * (xx, yy, zz, yz, xz, xy), in the unit of mu.
 *
 * Array layouts (element type: float when precision == 32, double when 64):
 *   rho:   [B][C][Nz][Ny][Nx]   x fastest, contiguous
 *   sigma: [B][6][Nz][Ny][Nx]   x fastest, contiguous
 *
 * Streams are hipStream_t passed as void* (NULL = the null stream). Every
 * call that takes a stream only enqueues work on it and returns; completion
 * is observed through the stream. A plan is not thread-safe; distinct plans
 * may run concurrently on distinct streams.
 *
 * Errors: every call returns a status and never throws. Argument and state
 * errors are detected before anything is enqueued. A HIP error reported by
 * the runtime while enqueueing is returned as DDSTRESS_E_DEVICE. The message
 * of the last failing call on the calling thread is ddstress_last_error().
 */
#ifndef DDSTRESS_H
#define DDSTRESS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddstress_plan_s* ddstress_plan;

typedef enum {
    DDSTRESS_OK = 0,
    DDSTRESS_E_INVALID = 1,      /* bad argument or descriptor */
    DDSTRESS_E_NOMEM = 2,        /* device allocation failed */
    DDSTRESS_E_DEVICE = 3,       /* HIP runtime error */
    DDSTRESS_E_STATE = 4,        /* call out of order (e.g. stress before set_density) */
    DDSTRESS_E_UNSUPPORTED = 5   /* valid but not implemented (e.g. a size above the limits) */
} ddstress_status;

/* Where a buffer passed to set_density / stress lives. */
typedef enum {
    DDSTRESS_HOST = 0,           /* host memory: copied asynchronously on the stream */
    DDSTRESS_DEVICE_COPY = 1,    /* device memory: copied into a plan-owned buffer */
    DDSTRESS_DEVICE_BORROW = 2   /* device memory used in place by the next stress() calls;
                                    the caller keeps it alive and unchanged until they complete */
} ddstress_where;

/* Problem statement: grid, cell sizes, elastic constants, line directions.
 * Limits: 1 <= N_a <= 512 on every axis; 1 <= n_lines <= 3; batch >= 1; and
 * (Pz / 2) Py Wx complex values of the plan precision span at most 2^31 - 1
 * bytes, with Wx = (Px / 2 + 1) rounded up to a multiple of 16 (the z pass
 * addresses one density plane with 32-bit offsets): with Px = Py = 1024 this
 * holds up to Nz = 256 in FP32 and Nz = 128 in FP64; larger grids are
 * DDSTRESS_E_UNSUPPORTED. */
typedef struct {
    int32_t n[3];          /* Nx, Ny, Nz (x fastest in memory) */
    double  d[3];          /* dx, dy, dz > 0, same length unit as 1/rho */
    double  mu;            /* isotropic shear modulus > 0 */
    double  nu;            /* Poisson ratio, -1 < nu < 0.5 */
    int32_t n_lines;       /* L, 1..3; C = 3L channels */
    double  t[3][3];       /* line directions t_l (normalised by the library; |t| = 0 is invalid) */
    int32_t precision;     /* 32 or 64: arithmetic of the per-call FFTs and contraction.
                              The interaction coefficients and their transform are always FP64. */
    int32_t batch;         /* B >= 1 densities per stress() call sharing this plan */
    int32_t near_shells;   /* S: a cell offset D is subdivided when |D_a| d_a <= S max(d) on every
                              axis; 0 selects the default 2, negative is invalid */
    uint32_t flags;        /* OR of DDSTRESS_FLAG_*; other bits are DDSTRESS_E_UNSUPPORTED */
    int32_t pbc_shells;    /* n_sh: replica shells |k|, |l| <= n_sh of Eq. (13) along the periodic axes;
                              0 selects the default 15, 1..32 as given, negative is invalid, above 32
                              unsupported; ignored without a periodic flag */
} ddstress_desc;

/* Periodic boundary conditions along x (y) in the layer plane (Sec. 4). The
 * axis is transformed at its own length, so N_a must be a power of two
 * (2..512; DDSTRESS_E_UNSUPPORTED otherwise), and the coefficient of a cell
 * offset D is
 *     F(D) = sum_{|k|, |l| <= n_sh} K(D' + (k Nx, l Ny, 0))
 * (Eq. 13, k only along a periodic x, l only along a periodic y), where D' is
 * D reduced into [-N_a/2, N_a/2) on each periodic axis, and at the half period
 * D'_a = -N_a/2 the mean of the sums around -N_a/2 and +N_a/2 is taken (the
 * two representatives are equally central; the mean keeps F odd, as K is).
 * A replica term is subdivided when its own offset is near; only the central
 * term of D = 0 is the zero self-term. z is never periodic. Costs
 * (2 n_sh + 1)^2 times the coefficient evaluations of an open plan at build
 * time and nothing per call. */
#define DDSTRESS_FLAG_PERIODIC_X 1u
#define DDSTRESS_FLAG_PERIODIC_Y 2u

/* Store the kernel spectrum for every wavevector even where a mirror symmetry
 * would let half of it be reconstructed (see ddstress_info.mirror_y). */
#define DDSTRESS_FLAG_FULL_SPECTRUM 4u

/* Read-only facts about a plan. */
typedef struct {
    int32_t padded[3];     /* FFT lengths Px, Py, Pz: powers of two >= max(2, 2 N_a - 1); N_a on a
                              periodic axis */
    int32_t subdiv[3];     /* subcells per axis m_a = max(1, floor(d_a / min(d) + 1/2)) */
    int32_t channels;      /* C = 3 L */
    int32_t batch;         /* B */
    int32_t precision;     /* 32 or 64 */
    int32_t tile_z;        /* columns per block of the fused z kernel (fixes the spectrum layout) */
    int32_t tile_y;        /* columns per block of the y passes */
    int32_t rows_x;        /* rows per block of the x passes */
    int32_t ex, ey, ez;    /* element classes of the x, y and fused z passes (see ddstress_tuning) */
    int32_t z_groups;      /* thread groups per column tile of the fused z pass (see ddstress_tuning) */
    int32_t yx_fused;      /* 1: inverse y and inverse x run as one kernel (see ddstress_tuning) */
    int32_t xy_fused;      /* 1: forward x and forward y run as one kernel (see ddstress_tuning) */
    int32_t mirror_y;      /* 1: every coefficient plane is even or odd under y -> -y (each line direction
                              has t_y = 0 or is parallel to e_y), so the spectrum is kept for ky <= Py/2
                              only, with a sign per plane for the mirrored rows */
    int32_t mirror_z;      /* the same for z -> -z and kz <= Pz/2 */
    size_t  cached_bytes;  /* device bytes held for the plan's lifetime (kernel spectrum, tables) */
    size_t  work_bytes;    /* device bytes of per-call work buffers */
    double  kernel_real_max;  /* max |Re K^| over the spectrum: zero up to rounding (K is odd) */
    double  kernel_imag_max;  /* max |Im K^| */
} ddstress_info;

/* Launch shapes of the passes: a tuning choice. A transform of length N runs
 * with E = min(N, e) elements per thread and radices <= E, where the element
 * class e is 8 or 16 for the x and y passes and 4 (FP32) / 2 (FP64) for the
 * fused z pass (for Pz >= 256 also 2, 4 or 8 times that, at most 16); 0
 * selects the default. The fused z pass runs either one thread group per
 * column tile, which transforms every channel and stress component, or one
 * group per density channel (z_groups = C), which split the transforms; both
 * sum the channels in the same order. Tile sizes and group counts change which
 * threads do the work, not the arithmetic (bit-identical results); element
 * classes change the radix sequence and hence the rounding (within the
 * stated tolerances). */
typedef struct {
    int32_t rows_x;        /* rows per block of the x passes (forward and inverse) */
    int32_t tk_y;          /* consecutive kx columns per block of the y passes */
    int32_t tk_z;          /* consecutive kx columns per block of the fused z pass */
    int32_t ex, ey, ez;    /* element classes of the x, y and fused z passes (0: default) */
    int32_t z_groups;      /* fused z thread groups: 1 or C (0: default, C when batch >= 16) */
    int32_t yx;            /* inverse y and x: 1 two passes, 2 one fused kernel that keeps each
                              (realisation, component, z) plane in LDS (FP32 with Py = 256 and
                              Px = 256 only), 0 default (fused where it applies) */
    int32_t xy;            /* forward x and y: 1 two passes, 2 one fused kernel (same shapes), 0 default */
    float   ms[3];         /* autotune: median device ms of the chosen x pair, y pair and z pass */
} ddstress_tuning;

/* Device bytes a plan for `desc` will hold (with the mirror symmetries the
 * line directions predict; a plan whose coefficients fail the numerical parity
 * check keeps the full spectrum and holds more): `cached_bytes` for its lifetime,
 * `work_bytes` for its per-call buffers, `build_bytes` transiently during
 * ddstress_plan_create. Any output pointer may be NULL. Synchronous, no
 * device work. Returns DDSTRESS_E_INVALID for an invalid descriptor. */
ddstress_status ddstress_plan_footprint(const ddstress_desc* desc, size_t* cached_bytes,
                                        size_t* work_bytes, size_t* build_bytes);

/* Build a plan: validates the descriptor, evaluates the interaction
 * coefficients K_{v,c} on every cell offset in FP64 on the device (Eq. 6,
 * Eq. 9b times the cell volume, near-cell subdivision, K(0) = 0), transforms
 * them with an FP64 3D FFT and keeps the spectrum (purely imaginary because K
 * is odd) in the plan precision. Work runs on `stream`; the call returns after
 * the build has completed (it synchronises the stream). On success *out owns
 * device memory until ddstress_plan_destroy. A transform whose real part
 * exceeds 1e-13 of its imaginary part (max over the kept wavevectors; for a
 * kernel that cancels to rounding, 1e-13 mu min(d)) fails with
 * DDSTRESS_E_UNSUPPORTED: only Im K^ is kept. */
ddstress_status ddstress_plan_create(const ddstress_desc* desc, void* stream, ddstress_plan* out);

/* Autotuner: times every admissible tile size, element class and z group
 * count of each pass, and the fused against the separate x and y passes (threads per block <= 512, 768 for the grouped z pass;
 * LDS <= 64 KiB) on zero-filled buffers of the descriptor's
 * shape, precision and batch, with HIP events on `stream` (median of five runs
 * after two warm-up runs), and returns the fastest per pass. Synchronous;
 * allocates its buffers for the duration of the call. */
ddstress_status ddstress_autotune(const ddstress_desc* desc, void* stream, ddstress_tuning* out);

/* As ddstress_plan_create, with the launch shapes of `tuning` (for example
 * from ddstress_autotune). DDSTRESS_E_INVALID if a choice is outside the
 * limits for this shape. */
ddstress_status ddstress_plan_create_tuned(const ddstress_desc* desc, const ddstress_tuning* tuning, void* stream,
                                           ddstress_plan* out);

/* Hand the B densities [B][C][Nz][Ny][Nx] (plan precision) to the plan.
 * Defined by Sec. 2.1, Eq. (3b): the stress of the whole sample is the sum
 * over dislocation types of the density n times the Burgers vector b times
 * the interaction function, and f is linear in b, so the density of type
 * (t_l, b) enters as the three channels rho_{3l+gamma} = n b_gamma (unit
 * length^-1), cell (i, j, k) holding the value at its centre (i dx, j dy, k dz).
 * rho: B realisations, C = 3L channels each, x fastest, contiguous.
 * Ownership: HOST and DEVICE_COPY enqueue a copy on `stream` into a buffer the
 * plan owns (the caller may reuse rho once the stream has passed that point;
 * host memory should be pinned for the copy to be asynchronous);
 * DEVICE_BORROW records the pointer only, and the caller keeps the buffer
 * alive and unchanged until the stress calls that read it have completed.
 * Errors: DDSTRESS_E_INVALID for a NULL plan or rho or an unknown `where`;
 * DDSTRESS_E_NOMEM if the plan's density buffer cannot be allocated (first
 * copying call); DDSTRESS_E_DEVICE if the copy cannot be enqueued. */
ddstress_status ddstress_set_density(ddstress_plan plan, const void* rho, int32_t where, void* stream);

/* Enqueue the stress evaluation of the current densities on `stream`.
 * Defined by Sec. 2.3, Eq. (10): for every cell r0,
 *     sigma_v(r0) = sum_{cells i} sum_c K_{v,c}(r0 - r_i) rho_c(r_i),
 * a discrete linear convolution, evaluated by the convolution theorem on the
 * grid zero-padded to P_a >= 2 N_a - 1 per open axis (no wrap-around):
 * forward x (real-to-complex), y and z transforms of the density channels,
 * the per-wavevector contraction sigma^_v = sum_c K^_{v,c} rho^_c with the
 * plan's kernel spectrum (c in increasing order), inverse z, y and x
 * (complex-to-real) transforms cropped to the grid.
 * sigma: [B][6][Nz][Ny][Nx] in the plan precision, Voigt order (xx, yy, zz,
 * yz, xz, xy), unit of mu, x fastest, contiguous; owned by the caller.
 * `where` is DDSTRESS_HOST (written through a plan-owned device buffer and an
 * asynchronous copy: host memory should be pinned) or DDSTRESS_DEVICE_COPY /
 * DDSTRESS_DEVICE_BORROW (both: written in place on the device).
 * Errors: DDSTRESS_E_INVALID for a NULL plan or sigma or an unknown `where`;
 * DDSTRESS_E_STATE if no density was set; DDSTRESS_E_NOMEM if the staging
 * buffer of a HOST output cannot be allocated; DDSTRESS_E_DEVICE if a launch
 * or copy cannot be enqueued. */
ddstress_status ddstress_stress(ddstress_plan plan, void* sigma, int32_t where, void* stream);

/* A second plan of the same geometry (grid, cells, constants, lines,
 * precision, near shells) for `batch` realisations, with its own work buffers
 * and the kernel spectrum of `src` shared, not copied: the spectrum stays
 * alive until the last plan sharing it is destroyed. No device work; plans
 * sharing a spectrum may run concurrently on distinct streams. */
ddstress_status ddstress_plan_share(ddstress_plan src, int32_t batch, ddstress_plan* out);

/* One-shot evaluation of the first `nbatch` (1 <= nbatch <= batch) densities:
 * `rho` [nbatch][C][Nz][Ny][Nx] and `sigma` [nbatch][6][Nz][Ny][Nx] are device
 * buffers in the plan precision. Enqueued on `stream`; the plan's
 * set_density state is neither used nor changed. The result of a realisation
 * does not depend on nbatch or on its position in the batch (every
 * realisation goes through the same arithmetic in the same order). */
ddstress_status ddstress_stress_batch(ddstress_plan plan, const void* rho, void* sigma, int32_t nbatch,
                                      void* stream);

/* Facts about a plan (see ddstress_info). */
ddstress_status ddstress_plan_get_info(ddstress_plan plan, ddstress_info* info);

/* Per-pass timing with HIP events recorded on the stream of each stress()
 * call: enable != 0 switches it on (and clears the totals), 0 switches it off.
 * The five passes are, in order: x real-to-complex, y forward, fused z
 * (forward z + contraction + inverse z), y inverse, x complex-to-real. A pass
 * that runs inside the previous one's kernel (y forward with x forward, x
 * inverse with y inverse, where a plane fits one block's LDS) records no event
 * of its own and reports zero. Every event record takes some stream time. */
ddstress_status ddstress_plan_set_profiling(ddstress_plan plan, int32_t enable);

/* Graph replay: with enable != 0, stress() and stress_batch() record their
 * launch sequence once per (density buffer, stress buffer, nbatch) into a HIP
 * graph (captured on a private stream, at most 8 kept per plan, least recently
 * used dropped first) and replay it on the caller's stream; the arithmetic is
 * the same as with direct launches. 0 switches it off and frees the graphs.
 * While profiling is on, calls launch directly. */
ddstress_status ddstress_plan_set_graph(ddstress_plan plan, int32_t enable);

/* Accumulated device milliseconds of each pass over the stress() calls made
 * since profiling was enabled, and the number of those calls. Synchronises
 * the recorded events; call it after the stream work has been issued. */
ddstress_status ddstress_plan_get_pass_times(ddstress_plan plan, double ms[5], int64_t* calls);

/* Average device milliseconds per launch of each of the five passes (order
 * as for ddstress_plan_get_pass_times): every pass is enqueued `reps` >= 1
 * times back to back on `stream`, in path order, on the current densities,
 * between two HIP events per pass (two events per pass, not per launch, so
 * the per-launch event cost does not enter). A pass reads only what the one
 * before it wrote, so repeating it recomputes the same output and `sigma`
 * (device buffer [B][6][Nz][Ny][Nx], plan precision) ends with the stress of
 * one ordinary evaluation. A pass fused into the previous one reports zero.
 * Synchronises `stream`. DDSTRESS_E_STATE if no density was set. Measurement
 * only: the same kernels and launch shapes as ddstress_stress. */
ddstress_status ddstress_plan_time_passes(ddstress_plan plan, void* sigma, int32_t reps, double ms[5],
                                          void* stream);

/* Free a plan and its device memory (synchronises the device first). NULL is
 * accepted. */
ddstress_status ddstress_plan_destroy(ddstress_plan plan);

/* The interaction coefficients of one line direction as the plan builds them
 * (Sec. 2.3: Eq. 9b times the cell volume, near-cell subdivision, K(0) = 0),
 * written in FP64 to the device buffer `out` laid out [3][6][Pz][Py][Px]
 * (Burgers component gamma, Voigt component, then the padded grid in wrap
 * order: index i on axis a holds offset i for i < N_a, i - P_a for
 * i > P_a - N_a, and zero in between; on a periodic axis P_a = N_a and index i
 * holds the replica sum F of offset i modulo N_a). `out` must hold
 * 18 Px Py Pz doubles. Enqueued on `stream`. */
ddstress_status ddstress_kernel_realspace(const ddstress_desc* desc, int32_t line, double* out,
                                          void* stream);

/* Plane statistics with every stress call: with stats != NULL, each
 * ddstress_stress / ddstress_stress_batch call also writes, for the
 * realisations it evaluates, stats[b][v][k] = (1 / (Nx Ny)) sum_{i,j}
 * sigma[b][v][k][j][i]^2 (Eq. 20; as ddstress_plane_mean_square, summed in
 * another fixed order), computed in the inverse x pass from the values it
 * writes (no second read of sigma): one FP64 sum of squares per row, then
 * the rows of each plane in a fixed order. stats: device buffer of batch * 6 * Nz
 * doubles, kept by the caller while set. The first non-NULL call allocates
 * batch * 6 * Nz * Ny doubles of row sums for the plan's lifetime; NULL
 * switches the statistics off. Drops the plan's captured graphs. */
ddstress_status ddstress_plan_set_plane_stats(ddstress_plan plan, double* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ddstress_stress_batch with the plane statistics of
 * ddstress_plan_set_plane_stats, allocating nothing. Evaluates the first
 * `nbatch` densities `rho` [nbatch][C][Nz][Ny][Nx] into `sigma`
 * [nbatch][6][Nz][Ny][Nx] (device buffers, plan precision) and writes
 * stats[b][v][k] (device, nbatch * 6 * Nz doubles), with the same kernels,
 * arithmetic and bits as ddstress_stress_batch on a plan whose statistics
 * are set. The per-row sums behind the statistics go to a static device array
 * of 2^21 doubles (16 MiB) that each GPU the library runs on holds until the
 * process ends, instead of a plan-owned buffer: nbatch * 6 * Nz * Ny above
 * 2^21 is DDSTRESS_E_UNSUPPORTED. Every row sum is written before it is read,
 * so nothing needs clearing between calls; calls that overlap on one GPU
 * (concurrent streams, plans or threads) share that array and race. Launches
 * directly (no graph replay, no profiling events) and ignores the plan's own
 * statistics setting; calls no hipMalloc, hipFree or allocating routine.
 * Enqueued on `stream`. */
ddstress_status ddstress_stress_batch_stats_noalloc(ddstress_plan plan, const void* rho, void* sigma, int32_t nbatch,
                                                   double* stats, void* stream);

/* Density channels in the axis basis (the Nye tensor) for line directions
 * that vary from cell to cell. Sec. 2.1 takes the stress of a volume element
 * as linear in the line direction t; that is exact for infinitesimal
 * segments, so a density n of lines along t with Burgers vector b acts, up to
 * a near-field error that falls as (cell size / distance)^2, like the three
 * axis densities n t_l. For a plan whose three line directions are e_x, e_y,
 * e_z (C = 9), the channels are
 *     rho[b][3 l + gamma] = n t_l b_gamma.
 * n: [nbatch][Nz][Ny][Nx]; t, b: [nbatch][3][Nz][Ny][Nx] (t as given, its
 * length is the caller's convention); rho: [nbatch][9][Nz][Ny][Nx]; device
 * buffers of float (precision 32) or double (64). accumulate = 1 adds to rho
 * (one call per dislocation family), 0 overwrites it. Enqueued on `stream`. */
ddstress_status ddstress_nye_density(const void* n, const void* t, const void* b, int32_t precision,
                                     const int32_t grid[3], int32_t nbatch, int32_t accumulate, void* rho,
                                     void* stream);

/* In-plane statistics (Sec. 6, Eq. 20): for each realisation b, stress
 * component v and layer k,
 *     out[b][v][k] = (1 / (Nx Ny)) sum_{i,j} sigma[b][v][k][j][i]^2,
 * the mean square over the plane (as printed, without subtracting the plane
 * mean). sigma: device buffer [nbatch][6][Nz][Ny][Nx] of float
 * (precision 32) or double (64), e.g. the output of ddstress_stress; out:
 * device buffer of nbatch * 6 * Nz doubles. Accumulated in FP64 in a fixed
 * order (the same input gives the same bits). Enqueued on `stream`. */
ddstress_status ddstress_plane_mean_square(const void* sigma, int32_t precision, const int32_t n[3],
                                           int32_t nbatch, double* out, void* stream);

/* ---- Relaxation under free surfaces (Sec. 5, Eq. 14-18) --------------------
 *
 * A film of Nx x Ny x Nz nodes (cell centres), periodic in x and y (Eq. 16a),
 * with traction-free top and bottom surfaces through the first and the last
 * node layer (Eq. 16b). Given the dislocation stress sigma^dis on the nodes
 * (for example the output of ddstress_stress), the displacement u solves the
 * Navier-Cauchy equation Eq. (14),
 *     A grad div u - B rot rot u + f = 0,   f = div sigma^dis (Eq. 15),
 * A = lambda + 2 mu, B = mu, with the surface conditions Eq. (16c), and the
 * total stress is sigma^dis + sigma(u) (Hooke's law). u is found as the
 * stationary state of the explicit pseudo-time iteration Eq. (17):
 *     u <- u + dt (A grad div u - B rot rot u + f)
 * with central differences (second differences for the Laplacian, products
 * of central first differences for the mixed derivatives; f by central
 * differences, second-order one-sided on the two surface layers) and ghost
 * layers below and above the film rewritten after every step from Eq. (16c)
 * (Eq. 18b and its analogues). The caller chooses the number of steps (the
 * paper gives no stopping rule) and may watch ddstress_relax_update_norm.
 *
 * Layouts (float when precision == 32, double when 64), x fastest:
 *   sigma^dis, sigma_total: [6][Nz][Ny][Nx], Voigt order (xx, yy, zz, yz, xz, xy)
 *   u (with ghost layers):  [3][Nz + 2][Ny][Nx]; layer k + 1 holds node layer k
 * All pointers are device memory. */
typedef struct ddstress_relax_s* ddstress_relax;

typedef struct {
    int32_t n[3];          /* Nx, Ny >= 1, Nz >= 3 node layers; at most 4096 per axis */
    double  d[3];          /* node spacings dx, dy, dz > 0 */
    double  mu;            /* shear modulus > 0 (B of Eq. 14) */
    double  nu;            /* Poisson ratio, -1 < nu < 0.5 */
    int32_t precision;     /* 32 or 64 */
    double  dt;            /* pseudo-time step; 0 selects min(d)^2 / (5A - 3B) (Sec. 5), negative is
                              invalid. That step is stable for cubic cells when nu > 1/8 */
} ddstress_relax_desc;

typedef struct {
    double  dt;            /* the step in use */
    double  A, B;          /* moduli of Eq. (14) */
    size_t  work_bytes;    /* device bytes held (two displacement states, force, surface terms) */
    int64_t steps;         /* steps taken since the last ddstress_relax_set_load */
} ddstress_relax_info;

/* Allocate a relaxation plan. Synchronous; no load yet. */
ddstress_status ddstress_relax_create(const ddstress_relax_desc* desc, ddstress_relax* out);

/* Take the load: computes f (Eq. 15) and the surface terms of Eq. (16c)
 * from sigma_dis and resets u to zero (ghost layers from Eq. 16c). sigma_dis
 * is read during the call's kernels only. Enqueued on `stream`. */
ddstress_status ddstress_relax_set_load(ddstress_relax r, const void* sigma_dis, void* stream);

/* Enqueue n_steps >= 0 explicit steps of Eq. (17) on `stream`.
 * DDSTRESS_E_STATE before set_load. */
ddstress_status ddstress_relax_iterate(ddstress_relax r, int32_t n_steps, void* stream);

/* max over the nodes of |A grad div u - B rot rot u + f| for the current u:
 * the size of the next step's update divided by dt. Synchronises `stream`. */
ddstress_status ddstress_relax_update_norm(ddstress_relax r, double* out, void* stream);

/* Iterate until the update norm falls to rel_tol times its value at the
 * first check of this call, or until max_steps steps have been taken, checking
 * every check_every steps (>= 1). A stopping rule of the caller's choosing
 * (the paper gives none): steps_taken and final_norm (either may be NULL)
 * report the outcome; reaching max_steps is not an error. Synchronises
 * `stream` at every check. */
ddstress_status ddstress_relax_solve(ddstress_relax r, double rel_tol, int32_t max_steps, int32_t check_every,
                                     int32_t* steps_taken, double* final_norm, void* stream);

/* sigma_total = sigma_dis + sigma(u) on the nodes (sigma_total may be
 * sigma_dis itself). Enqueued on `stream`. */
ddstress_status ddstress_relax_stress(ddstress_relax r, const void* sigma_dis, void* sigma_total, void* stream);

/* Copy the current u with its ghost layers into `u`. Enqueued on `stream`. */
ddstress_status ddstress_relax_displacement(ddstress_relax r, void* u, void* stream);

ddstress_status ddstress_relax_get_info(ddstress_relax r, ddstress_relax_info* info);

/* Free the plan (synchronises the device first). NULL is accepted. */
ddstress_status ddstress_relax_destroy(ddstress_relax r);

/* Message of the last failing call on this thread ("" if none). */
const char* ddstress_last_error(void);

/* Library version string. */
const char* ddstress_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DDSTRESS_H */
