"""ctypes binding of ``libddstress.so`` (declared in ``include/ddstress.h``).

Argument marshalling only: every step of the stress evaluation runs in the HIP
library. Device memory and streams come from PyTorch (ROCm); the library
receives raw device pointers and a ``hipStream_t``. There is no CPU fallback:
if the library is missing or cannot be loaded, ``load()`` raises.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libddstress.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE, E_UNSUPPORTED = range(6)
FLAG_PERIODIC_X, FLAG_PERIODIC_Y, FLAG_FULL_SPECTRUM = 1, 2, 4
HOST, DEVICE_COPY, DEVICE_BORROW = 0, 1, 2
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_STATE", 5: "E_UNSUPPORTED"}

# names exported by the library, in header order
EXPORTS = ("ddstress_plan_footprint", "ddstress_autotune", "ddstress_plan_create", "ddstress_plan_create_tuned",
           "ddstress_set_density", "ddstress_stress",
           "ddstress_plan_share", "ddstress_stress_batch", "ddstress_plan_get_info", "ddstress_plan_set_profiling", "ddstress_plan_set_graph", "ddstress_plan_get_pass_times", "ddstress_plan_time_passes",
           "ddstress_plan_destroy", "ddstress_kernel_realspace", "ddstress_plan_set_plane_stats", "ddstress_stress_batch_stats_noalloc",
           "ddstress_nye_density",
           "ddstress_plane_mean_square",
           "ddstress_relax_create", "ddstress_relax_set_load", "ddstress_relax_iterate", "ddstress_relax_update_norm",
           "ddstress_relax_solve", "ddstress_relax_stress", "ddstress_relax_displacement", "ddstress_relax_get_info", "ddstress_relax_destroy",
           "ddstress_last_error", "ddstress_version")
PASS_NAMES = ("x_r2c", "y_fwd", "z_fused", "y_inv", "x_c2r")


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("d", ctypes.c_double * 3), ("mu", ctypes.c_double),
                ("nu", ctypes.c_double), ("n_lines", ctypes.c_int32), ("t", (ctypes.c_double * 3) * 3),
                ("precision", ctypes.c_int32), ("batch", ctypes.c_int32), ("near_shells", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("pbc_shells", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("rows_x", ctypes.c_int32), ("tk_y", ctypes.c_int32), ("tk_z", ctypes.c_int32),
                ("ex", ctypes.c_int32), ("ey", ctypes.c_int32), ("ez", ctypes.c_int32),
                ("z_groups", ctypes.c_int32), ("yx", ctypes.c_int32), ("xy", ctypes.c_int32),
                ("ms", ctypes.c_float * 3)]


class Info(ctypes.Structure):
    _fields_ = [("padded", ctypes.c_int32 * 3), ("subdiv", ctypes.c_int32 * 3), ("channels", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("precision", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("rows_x", ctypes.c_int32), ("ex", ctypes.c_int32),
                ("ey", ctypes.c_int32), ("ez", ctypes.c_int32), ("z_groups", ctypes.c_int32),
                ("yx_fused", ctypes.c_int32), ("xy_fused", ctypes.c_int32), ("mirror_y", ctypes.c_int32),
                ("mirror_z", ctypes.c_int32),
                ("cached_bytes", ctypes.c_size_t), ("work_bytes", ctypes.c_size_t),
                ("kernel_real_max", ctypes.c_double), ("kernel_imag_max", ctypes.c_double)]


class RelaxDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("d", ctypes.c_double * 3), ("mu", ctypes.c_double),
                ("nu", ctypes.c_double), ("precision", ctypes.c_int32), ("dt", ctypes.c_double)]


class RelaxInfo(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("A", ctypes.c_double), ("B", ctypes.c_double),
                ("work_bytes", ctypes.c_size_t), ("steps", ctypes.c_int64)]


class DDStressError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path=LIB_PATH):
    """Load the library once and declare the signatures. Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run python -m paper_1804_01830_amd.build)")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    S = ctypes.c_size_t
    lib.ddstress_plan_footprint.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(S), ctypes.POINTER(S),
                                            ctypes.POINTER(S)]
    lib.ddstress_plan_create.argtypes = [ctypes.POINTER(Desc), P, ctypes.POINTER(P)]
    lib.ddstress_autotune.argtypes = [ctypes.POINTER(Desc), P, ctypes.POINTER(Tuning)]
    lib.ddstress_plan_create_tuned.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Tuning), P, ctypes.POINTER(P)]
    lib.ddstress_set_density.argtypes = [P, P, ctypes.c_int32, P]
    lib.ddstress_stress.argtypes = [P, P, ctypes.c_int32, P]
    lib.ddstress_plan_get_info.argtypes = [P, ctypes.POINTER(Info)]
    lib.ddstress_plan_destroy.argtypes = [P]
    lib.ddstress_kernel_realspace.argtypes = [ctypes.POINTER(Desc), ctypes.c_int32, P, P]
    lib.ddstress_plan_set_profiling.argtypes = [P, ctypes.c_int32]
    lib.ddstress_plan_set_graph.argtypes = [P, ctypes.c_int32]
    lib.ddstress_plan_share.argtypes = [P, ctypes.c_int32, ctypes.POINTER(P)]
    lib.ddstress_stress_batch.argtypes = [P, P, P, ctypes.c_int32, P]
    lib.ddstress_plan_get_pass_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.ddstress_plan_time_passes.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), P]
    lib.ddstress_plan_set_plane_stats.argtypes = [P, P]
    lib.ddstress_plan_set_plane_stats.restype = ctypes.c_int
    lib.ddstress_stress_batch_stats_noalloc.argtypes = [P, P, P, ctypes.c_int32, P, P]
    lib.ddstress_stress_batch_stats_noalloc.restype = ctypes.c_int
    lib.ddstress_nye_density.argtypes = [P, P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                         ctypes.c_int32, P, P]
    lib.ddstress_nye_density.restype = ctypes.c_int
    lib.ddstress_plane_mean_square.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, P, P]
    lib.ddstress_plane_mean_square.restype = ctypes.c_int
    lib.ddstress_relax_create.argtypes = [ctypes.POINTER(RelaxDesc), ctypes.POINTER(P)]
    lib.ddstress_relax_set_load.argtypes = [P, P, P]
    lib.ddstress_relax_iterate.argtypes = [P, ctypes.c_int32, P]
    lib.ddstress_relax_update_norm.argtypes = [P, ctypes.POINTER(ctypes.c_double), P]
    lib.ddstress_relax_solve.argtypes = [P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), P]
    lib.ddstress_relax_stress.argtypes = [P, P, P, P]
    lib.ddstress_relax_displacement.argtypes = [P, P, P]
    lib.ddstress_relax_get_info.argtypes = [P, ctypes.POINTER(RelaxInfo)]
    lib.ddstress_relax_destroy.argtypes = [P]
    for name in EXPORTS:
        if name.startswith("ddstress_relax"):
            getattr(lib, name).restype = ctypes.c_int
    for name in ("ddstress_plan_footprint", "ddstress_autotune", "ddstress_plan_create", "ddstress_plan_create_tuned",
                 "ddstress_set_density", "ddstress_stress",
                 "ddstress_plan_share", "ddstress_stress_batch", "ddstress_plan_get_info", "ddstress_plan_set_graph", "ddstress_plan_set_profiling", "ddstress_plan_set_graph", "ddstress_plan_get_pass_times",
                 "ddstress_plan_time_passes", "ddstress_plan_destroy", "ddstress_kernel_realspace"):
        getattr(lib, name).restype = ctypes.c_int
    lib.ddstress_last_error.restype = ctypes.c_char_p
    lib.ddstress_last_error.argtypes = []
    lib.ddstress_version.restype = ctypes.c_char_p
    lib.ddstress_version.argtypes = []
    _lib = lib
    return lib


def check(status):
    if status != OK:
        raise DDStressError(status, load().ddstress_last_error().decode())


def make_desc(n, d, mu, nu, lines, precision=32, batch=1, near_shells=0, flags=0, periodic=(False, False),
              pbc_shells=0):
    """Descriptor of a plan. ``periodic`` = (x, y) sets the periodic-boundary
    flags; ``pbc_shells`` is the replica shell count (0: the default 15)."""
    desc = Desc()
    for a in range(3):
        desc.n[a] = int(n[a])
        desc.d[a] = float(d[a])
    desc.mu = float(mu)
    desc.nu = float(nu)
    lines = [list(map(float, t)) for t in lines]
    desc.n_lines = len(lines)
    for l, t in enumerate(lines[:3]):
        for a in range(3):
            desc.t[l][a] = t[a]
    desc.precision = int(precision)
    desc.batch = int(batch)
    desc.near_shells = int(near_shells)
    desc.flags = int(flags) | (FLAG_PERIODIC_X if periodic[0] else 0) | (FLAG_PERIODIC_Y if periodic[1] else 0)
    desc.pbc_shells = int(pbc_shells)
    return desc


def footprint(desc):
    c, w, b = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    check(load().ddstress_plan_footprint(ctypes.byref(desc), ctypes.byref(c), ctypes.byref(w), ctypes.byref(b)))
    return c.value, w.value, b.value


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


class Plan:
    """Owns one ``ddstress_plan``. Tensors are torch CUDA tensors of the plan
    precision; ``stream`` is a torch stream (default: the current stream)."""

    def __init__(self, desc, stream=None, tuning=None, _handle=None):
        self.desc = desc
        self._h = ctypes.c_void_p()
        if _handle is not None:
            self._h = _handle
        elif tuning is None:
            check(load().ddstress_plan_create(ctypes.byref(desc), _stream_handle(stream), ctypes.byref(self._h)))
        else:
            check(load().ddstress_plan_create_tuned(ctypes.byref(desc), ctypes.byref(tuning), _stream_handle(stream),
                                                    ctypes.byref(self._h)))
        self.n = tuple(desc.n)
        self.channels = 3 * desc.n_lines
        self.batch = desc.batch
        self.precision = desc.precision

    def info(self):
        info = Info()
        check(load().ddstress_plan_get_info(self._h, ctypes.byref(info)))
        return info

    @property
    def handle(self):
        return self._h

    def set_density(self, rho, where=DEVICE_BORROW, stream=None):
        """Hand the density to the plan: a CUDA tensor borrowed (DEVICE_BORROW)
        or copied (DEVICE_COPY), or a CPU tensor copied from host memory (HOST;
        pinned memory makes the copy asynchronous)."""
        self._check_tensor(rho, (self.batch, self.channels), host=(where == HOST))
        self._rho_ref = rho           # keeps a borrowed buffer alive
        check(load().ddstress_set_density(self._h, ctypes.c_void_p(rho.data_ptr()), where,
                                          _stream_handle(stream)))

    def stress(self, sigma, stream=None, where=DEVICE_BORROW):
        """Evaluate into ``sigma``: a CUDA tensor, or a CPU tensor with
        where=HOST (copied back on the stream; synchronise before reading)."""
        self._check_tensor(sigma, (self.batch, 6), host=(where == HOST))
        check(load().ddstress_stress(self._h, ctypes.c_void_p(sigma.data_ptr()), where,
                                     _stream_handle(stream)))
        return sigma

    def share(self, batch):
        """A plan of the same geometry with ``batch`` realisations and its own
        work buffers, sharing this plan's kernel spectrum."""
        h = ctypes.c_void_p()
        check(load().ddstress_plan_share(self._h, int(batch), ctypes.byref(h)))
        desc = Desc.from_buffer_copy(self.desc)
        desc.batch = int(batch)
        return Plan(desc, _handle=h)

    def stress_batch(self, rho, sigma, nbatch, stream=None):
        """Evaluate the first ``nbatch`` realisations of the device tensors
        ``rho`` (nbatch, C, Nz, Ny, Nx) and ``sigma`` (nbatch, 6, Nz, Ny, Nx)."""
        self._check_tensor(rho, (nbatch, self.channels))
        self._check_tensor(sigma, (nbatch, 6))
        check(load().ddstress_stress_batch(self._h, ctypes.c_void_p(rho.data_ptr()),
                                           ctypes.c_void_p(sigma.data_ptr()), int(nbatch),
                                           _stream_handle(stream)))
        return sigma

    def new_output(self):
        import torch
        dt = torch.float32 if self.precision == 32 else torch.float64
        nx, ny, nz = self.n
        return torch.empty((self.batch, 6, nz, ny, nx), dtype=dt, device="cuda")

    def _check_tensor(self, t, lead, host=False):
        import torch
        dt = torch.float32 if self.precision == 32 else torch.float64
        nx, ny, nz = self.n
        where = "CPU" if host else "CUDA"
        if (t.is_cuda == host or t.dtype != dt or not t.is_contiguous()
                or tuple(t.shape) != (*lead, nz, ny, nx)):
            raise ValueError(f"expected a contiguous {where} {dt} tensor of shape {(*lead, nz, ny, nx)}, "
                             f"got {tuple(t.shape)} {t.dtype} on {t.device}")

    def set_plane_stats(self, stats):
        """With a CUDA float64 tensor (batch, 6, Nz), every stress call also
        writes the Eq. (20) plane mean squares of its output there (computed in
        the inverse x pass); None switches it off."""
        import torch
        if stats is not None:
            nz = self.n[2]
            if not stats.is_cuda or stats.dtype != torch.float64 or not stats.is_contiguous() \
                    or tuple(stats.shape) != (self.batch, 6, nz):
                raise ValueError(f"expected a contiguous CUDA float64 tensor of shape {(self.batch, 6, nz)}")
        self._stats_ref = stats
        check(load().ddstress_plan_set_plane_stats(self._h, ctypes.c_void_p(stats.data_ptr() if stats is not None
                                                                            else None)))

    def set_profiling(self, enable=True):
        check(load().ddstress_plan_set_profiling(self._h, 1 if enable else 0))

    def set_graph(self, enable=True):
        check(load().ddstress_plan_set_graph(self._h, 1 if enable else 0))

    def pass_times(self):
        """(dict pass name -> total ms, number of timed stress calls)."""
        ms = (ctypes.c_double * 5)()
        calls = ctypes.c_int64()
        check(load().ddstress_plan_get_pass_times(self._h, ms, ctypes.byref(calls)))
        return dict(zip(PASS_NAMES, list(ms))), calls.value

    def stress_batch_stats_noalloc(self, rho, sigma, nbatch, stats, stream=None):
        """As stress_batch, also writing the Eq. (20) plane statistics of the
        result to ``stats`` (CUDA float64 (nbatch, 6, Nz)); the library
        allocates nothing for it (its row sums live in a static device array)."""
        import torch
        self._check_tensor(rho, (nbatch, self.channels))
        self._check_tensor(sigma, (nbatch, 6))
        if (not stats.is_cuda or stats.dtype != torch.float64 or not stats.is_contiguous()
                or tuple(stats.shape) != (nbatch, 6, self.n[2])):
            raise ValueError(f"expected a contiguous CUDA float64 tensor of shape {(nbatch, 6, self.n[2])}")
        check(load().ddstress_stress_batch_stats_noalloc(self._h, ctypes.c_void_p(rho.data_ptr()),
                                                         ctypes.c_void_p(sigma.data_ptr()), int(nbatch),
                                                         ctypes.c_void_p(stats.data_ptr()), _stream_handle(stream)))
        return sigma

    def time_passes(self, sigma, reps, stream=None):
        """Average device ms per launch of each pass (dict pass name -> ms),
        each pass enqueued `reps` times back to back between two events on
        the current densities; `sigma` (CUDA tensor of the output shape)
        receives the stress."""
        self._check_tensor(sigma, (self.batch, 6))
        ms = (ctypes.c_double * 5)()
        check(load().ddstress_plan_time_passes(self._h, ctypes.c_void_p(sigma.data_ptr()), int(reps), ms,
                                               _stream_handle(stream)))
        return dict(zip(PASS_NAMES, list(ms)))

    def close(self):
        if self._h:
            check(load().ddstress_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Relax:
    """Owns one ``ddstress_relax`` plan: relaxation of a dislocation stress
    field under free top and bottom surfaces, periodic in x and y. Tensors are
    torch CUDA tensors of the plan precision."""

    def __init__(self, n, d, mu, nu, precision=64, dt=0.0):
        self.desc = RelaxDesc()
        for a in range(3):
            self.desc.n[a] = int(n[a])
            self.desc.d[a] = float(d[a])
        self.desc.mu = float(mu)
        self.desc.nu = float(nu)
        self.desc.precision = int(precision)
        self.desc.dt = float(dt)
        self.n = tuple(int(v) for v in n)
        self.precision = int(precision)
        self._h = ctypes.c_void_p()
        check(load().ddstress_relax_create(ctypes.byref(self.desc), ctypes.byref(self._h)))

    def _check(self, t, shape):
        import torch
        dt = torch.float32 if self.precision == 32 else torch.float64
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"expected a contiguous CUDA {dt} tensor of shape {shape}, got {tuple(t.shape)} "
                             f"{t.dtype} on {t.device}")

    def _sigma_shape(self):
        nx, ny, nz = self.n
        return (6, nz, ny, nx)

    def set_load(self, sigma_dis, stream=None):
        self._check(sigma_dis, self._sigma_shape())
        check(load().ddstress_relax_set_load(self._h, ctypes.c_void_p(sigma_dis.data_ptr()), _stream_handle(stream)))

    def iterate(self, n_steps, stream=None):
        check(load().ddstress_relax_iterate(self._h, int(n_steps), _stream_handle(stream)))

    def update_norm(self, stream=None):
        out = ctypes.c_double()
        check(load().ddstress_relax_update_norm(self._h, ctypes.byref(out), _stream_handle(stream)))
        return out.value

    def solve(self, rel_tol, max_steps, check_every=500, stream=None):
        """Iterate until the update norm falls to rel_tol of its first value
        (or max_steps); returns (steps taken, final update norm)."""
        steps = ctypes.c_int32()
        norm = ctypes.c_double()
        check(load().ddstress_relax_solve(self._h, float(rel_tol), int(max_steps), int(check_every),
                                          ctypes.byref(steps), ctypes.byref(norm), _stream_handle(stream)))
        return steps.value, norm.value

    def stress(self, sigma_dis, out=None, stream=None):
        import torch
        self._check(sigma_dis, self._sigma_shape())
        if out is None:
            out = torch.empty_like(sigma_dis)
        self._check(out, self._sigma_shape())
        check(load().ddstress_relax_stress(self._h, ctypes.c_void_p(sigma_dis.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def displacement(self, stream=None):
        import torch
        nx, ny, nz = self.n
        dt = torch.float32 if self.precision == 32 else torch.float64
        u = torch.empty((3, nz + 2, ny, nx), dtype=dt, device="cuda")
        check(load().ddstress_relax_displacement(self._h, ctypes.c_void_p(u.data_ptr()), _stream_handle(stream)))
        return u

    def info(self):
        info = RelaxInfo()
        check(load().ddstress_relax_get_info(self._h, ctypes.byref(info)))
        return info

    def close(self):
        if self._h:
            check(load().ddstress_relax_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


AXIS_LINES = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))


def nye_density(n, t, b, rho=None, accumulate=False, stream=None):
    """Axis-basis channels rho[:, 3 l + g] = n t_l b_g for a plan with the
    line directions AXIS_LINES. n: (nb, Nz, Ny, Nx); t, b: (nb, 3, Nz, Ny, Nx);
    CUDA tensors of one float dtype. Returns rho (nb, 9, Nz, Ny, Nx)."""
    import torch
    for x in (n, t, b):
        if not x.is_cuda or not x.is_contiguous() or x.dtype != n.dtype or x.dtype not in (torch.float32,
                                                                                            torch.float64):
            raise ValueError("n, t, b must be contiguous CUDA tensors of one float dtype")
    nb, nz, ny, nx = n.shape
    if tuple(t.shape) != (nb, 3, nz, ny, nx) or tuple(b.shape) != (nb, 3, nz, ny, nx):
        raise ValueError(f"t and b must have shape {(nb, 3, nz, ny, nx)}")
    if rho is None:
        rho = torch.empty((nb, 9, nz, ny, nx), dtype=n.dtype, device=n.device)
    elif tuple(rho.shape) != (nb, 9, nz, ny, nx) or rho.dtype != n.dtype or not rho.is_contiguous():
        raise ValueError(f"rho must be a contiguous {n.dtype} tensor of shape {(nb, 9, nz, ny, nx)}")
    grid = (ctypes.c_int32 * 3)(nx, ny, nz)
    check(load().ddstress_nye_density(ctypes.c_void_p(n.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                      ctypes.c_void_p(b.data_ptr()), 32 if n.dtype == torch.float32 else 64, grid,
                                      int(nb), 1 if accumulate else 0, ctypes.c_void_p(rho.data_ptr()),
                                      _stream_handle(stream)))
    return rho


def plane_mean_square(sigma, out=None, stream=None):
    """Eq. (20): the mean square over each layer plane of a CUDA tensor
    (nb, 6, Nz, Ny, Nx) (float32 or float64); returns (nb, 6, Nz) float64."""
    import torch
    if not sigma.is_cuda or sigma.dim() != 5 or sigma.shape[1] != 6 or not sigma.is_contiguous() \
            or sigma.dtype not in (torch.float32, torch.float64):
        raise ValueError(f"expected a contiguous CUDA float tensor (nb, 6, Nz, Ny, Nx), got {tuple(sigma.shape)} "
                         f"{sigma.dtype} on {sigma.device}")
    nb, _, nz, ny, nx = sigma.shape
    if out is None:
        out = torch.empty((nb, 6, nz), dtype=torch.float64, device=sigma.device)
    n = (ctypes.c_int32 * 3)(nx, ny, nz)
    check(load().ddstress_plane_mean_square(ctypes.c_void_p(sigma.data_ptr()), 32 if sigma.dtype == torch.float32
                                            else 64, n, int(nb), ctypes.c_void_p(out.data_ptr()),
                                            _stream_handle(stream)))
    return out


def autotune(desc, stream=None):
    """Time the admissible launch shapes of each pass on the device; returns a Tuning."""
    t = Tuning()
    check(load().ddstress_autotune(ctypes.byref(desc), _stream_handle(stream), ctypes.byref(t)))
    return t


def kernel_realspace(desc, line, out, stream=None):
    """FP64 interaction coefficients of one line direction into the CUDA
    tensor ``out`` of shape (3, 6, Pz, Py, Px) (see the header)."""
    check(load().ddstress_kernel_realspace(ctypes.byref(desc), int(line), ctypes.c_void_p(out.data_ptr()),
                                           _stream_handle(stream)))
    return out


def padded_lengths(n, periodic=(False, False)):
    """FFT lengths of a plan: N on a periodic axis, else the power of two
    >= max(2, 2N - 1)."""
    out = []
    for a, v in enumerate(n):
        if a < 2 and periodic[a]:
            out.append(int(v))
            continue
        p = 1
        while p < 2 * v - 1:
            p *= 2
        out.append(max(2, p))
    return tuple(out)
