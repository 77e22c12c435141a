"""Helpers shared by the GPU tests: run the HIP path through the C ABI on a
workload dict and compare with oracle results."""
import numpy as np


def gpu_stress(w, precision=64, near_shells=0, where_rho=None, periodic=(False, False), pbc_shells=0):
    """sigma (B, 6, Nz, Ny, Nx) as float64 numpy, computed by the HIP library."""
    import torch
    from paper_1804_01830_amd import binding as B
    rho = np.asarray(w["rho"])
    desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=precision,
                       batch=rho.shape[0], near_shells=near_shells, periodic=periodic, pbc_shells=pbc_shells)
    plan = B.Plan(desc)
    dt = torch.float32 if precision == 32 else torch.float64
    r = torch.from_numpy(rho).to(device="cuda", dtype=dt).contiguous()
    plan.set_density(r, where=B.DEVICE_BORROW if where_rho is None else where_rho)
    out = plan.new_output()
    plan.stress(out)
    torch.cuda.synchronize()
    res = out.double().cpu().numpy()
    plan.close()
    return res


def rel_l2(got, ref):
    """Relative L2 error per Voigt component (axis -4 of (..., 6, Nz, Ny, Nx)
    or axis 0 of (6, T)) and over the whole tensor. A component whose reference
    norm is below 1e-3 of the whole norm is measured against the whole norm."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    whole = np.linalg.norm(ref)
    if whole == 0.0:
        # a reference that is exactly zero (e.g. a single cell: K(0) = 0) must be met exactly
        e = 0.0 if np.all(got == 0.0) else np.inf
        return np.full(6, e), e
    comp = []
    for v in range(6):
        g = np.take(got, v, axis=-4 if got.ndim >= 4 else 0)
        r = np.take(ref, v, axis=-4 if ref.ndim >= 4 else 0)
        comp.append(np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-3 * whole))
    return np.array(comp), np.linalg.norm(got - ref) / whole


def rel_l2_split(got, ref, floor=1e-3):
    """The per-component errors of rel_l2, split by how they are measured:
    `own` maps each component whose reference norm is at least `floor` of the
    whole-tensor norm to its error relative to its own norm; `small` maps the
    others (components that are zero or nearly so, where a relative error has
    no meaning) to their error norm relative to the whole-tensor norm."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    whole = np.linalg.norm(ref)
    own, small = {}, {}
    for v in range(6):
        g = np.take(got, v, axis=-4 if got.ndim >= 4 else 0)
        r = np.take(ref, v, axis=-4 if ref.ndim >= 4 else 0)
        rn, e = np.linalg.norm(r), np.linalg.norm(g - r)
        if whole > 0.0 and rn >= floor * whole:
            own[v] = e / rn
        else:
            small[v] = e / whole if whole > 0.0 else (0.0 if e == 0.0 else np.inf)
    return own, small

