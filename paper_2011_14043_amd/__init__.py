"""MI355X implicit FDTD: fundamental and conventional ADI / LOD1 / SS2 / LOD2.

Thin Python front end of libfdtd.so (C ABI in include/fdtd.h).  PyTorch is
used only for device memory and the current HIP stream; the computation runs
in the library's HIP kernels.

    plan = Plan(nx, ny, nz, dt, dx, dy, dz, scheme="adi", form="fundamental",
                dtype=torch.float32, eps_r=eps)       # eps: (nz, ny, nx) float32
    energies = plan.run(E, H, nsteps, source=Source(...), energy_every=1)

E = [Ex, Ey, Ez], H = [Hx, Hy, Hz]: contiguous device tensors of shape
(nz+1, ny+1, nx+1), updated in place.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _lib

__all__ = ["Plan", "BatchPlan", "Source", "FdtdError", "load_library", "ProbeEnergy", "probe_energy", "optimized_stencil"]

FdtdError = _lib.FdtdError


def load_library():
    return _lib.lib()


@dataclass(frozen=True)
class Source:
    """Ez point source in cell (i, j, k); see fdtd_source in include/fdtd.h."""
    i: int
    j: int
    k: int
    f0: float = 10e9
    tau: float = 0.1e-9
    t0: float = 0.4e-9
    amp: float = 1.0e10

    def _c(self):
        return _lib.FdtdSource(self.i, self.j, self.k, self.f0, self.tau, self.t0, self.amp)


def _dtype_code(dtype, solve, refine):
    """fdtd_dtype of (field type, solve type, refine): for float32 fields and
    solves, refine None lets the library choose (FDTD_F32), True forces
    refined solves (FDTD_F32_REFINE), False plain ones (FDTD_F32_PLAIN); other
    precisions take refine None or False."""
    import torch
    if dtype not in (torch.float32, torch.float64):
        raise ValueError("dtype must be float32 or float64")
    if dtype == torch.float64 and solve != torch.float64:
        raise ValueError("float64 fields need float64 solves")
    if refine and (dtype != torch.float32 or solve != torch.float32):
        raise ValueError("refine applies to float32 fields with float32 solves")
    if dtype == torch.float64:
        return _lib.DTYPES["f64"]
    if solve == torch.float64:
        return _lib.DTYPES["f32_f64solve"]
    if refine is None:
        return _lib.DTYPES["f32"]
    return _lib.DTYPES["f32_refine"] if refine else _lib.DTYPES["f32_plain"]


def _ptrs(ts, dtype, shape, device):
    import torch
    if len(ts) != 3:
        raise ValueError("need three components")
    for t in ts:
        if not isinstance(t, torch.Tensor) or t.dtype != dtype or tuple(t.shape) != shape \
                or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"field must be a contiguous {dtype} device tensor of shape {shape}")
        if device is not None and t.device != device:
            raise ValueError("fields must live on the plan's device")
    return (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ts])


class Plan:
    """One simulation plan (fdtd_plan).  Not thread-safe."""

    def __init__(self, nx, ny, nz, dt, dx, dy, dz, scheme="adi", form="fundamental",
                 dtype=None, eps_r=None, stream=None, device=None, solve_dtype=None, refine=None, mu_r=None):
        """dtype: field storage (float32/float64); solve_dtype: arithmetic of the
        line solves (defaults to dtype; float64 with float32 fields selects
        FDTD_F32_F64SOLVE); refine (float32 fields and solves): None lets the
        library choose (FDTD_F32: refined wherever refined passes are built),
        True always refines them once (FDTD_F32_REFINE, fundamental forms),
        False never (FDTD_F32_PLAIN).  `refined` tells what the plan does.
        eps_r, mu_r: relative permittivity and permeability per cell,
        (nz, ny, nx); None means 1."""
        import torch
        L = _lib.lib()
        self.dtype = dtype if dtype is not None else torch.float32
        solve = solve_dtype if solve_dtype is not None else self.dtype
        code = _dtype_code(self.dtype, solve, refine)
        self.shape = (nz + 1, ny + 1, nx + 1)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        keep = []

        def cell_map(m, name):
            if m is None:
                return None
            t = m if isinstance(m, torch.Tensor) else torch.as_tensor(m)
            t = t.to(dtype=torch.float32).contiguous()
            if tuple(t.shape) != (nz, ny, nx):
                raise ValueError(f"{name} must have shape (nz, ny, nx)")
            keep.append(t)
            return t.data_ptr()

        desc = _lib.FdtdDesc(nx, ny, nz, dt, dx, dy, dz, _lib.SCHEMES[scheme], _lib.FORMS[form],
                             code, cell_map(eps_r, "eps_r"), cell_map(mu_r, "mu_r"), 0)
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = s
            h = ctypes.c_void_p()
            _lib.check(L.fdtd_plan(ctypes.byref(desc), ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)),
                       "fdtd_plan")
        self._h = h
        del keep
        self.scheme, self.form = scheme, form
        self.order = 2
        self.refined = self._refined()

    def _refined(self) -> bool:
        r = ctypes.c_int()
        _lib.check(_lib.lib().fdtd_get_refined(self._h, ctypes.byref(r)), "fdtd_get_refined")
        return bool(r.value)

    def run(self, E, H, nsteps, source: Source | None = None, energy_every: int = 0):
        """Advance E, H in place by nsteps; returns the energy trace (list) if
        energy_every > 0, else None (asynchronous on the plan's stream)."""
        L = _lib.lib()
        pe = _ptrs(E, self.dtype, self.shape, self.device)
        ph = _ptrs(H, self.dtype, self.shape, self.device)
        src = ctypes.byref(source._c()) if source is not None else None
        if energy_every > 0:
            n = nsteps // energy_every + 1
            buf = (ctypes.c_double * n)()
            _lib.check(L.fdtd_run(self._h, pe, ph, int(nsteps), src, buf, int(energy_every)), "fdtd_run")
            return list(buf)
        _lib.check(L.fdtd_run(self._h, pe, ph, int(nsteps), src, None, 1), "fdtd_run")
        return None

    def step(self, E, H, source: Source | None = None):
        L = _lib.lib()
        src = ctypes.byref(source._c()) if source is not None else None
        _lib.check(L.fdtd_step(self._h, _ptrs(E, self.dtype, self.shape, self.device),
                               _ptrs(H, self.dtype, self.shape, self.device), src), "fdtd_step")

    def set_graph(self, steps: int):
        """Steps per captured HIP graph of fdtd_run (0: launch every step directly)."""
        _lib.check(_lib.lib().fdtd_set_graph(self._h, int(steps)), "fdtd_set_graph")

    def set_order(self, order: int):
        """Accuracy order of the staggered differences: 2 (Yee) or 4
        (fdtd_set_order; fundamental forms, unit permeability).  Order 4 has
        no refined solves: FP32 plans with the library's choice (refine None)
        solve in FP64 with FP32 fields, refine=False plans in FP32.  Refreshes
        `refined`."""
        _lib.check(_lib.lib().fdtd_set_order(self._h, int(order)), "fdtd_set_order")
        self.order = int(order)
        self.refined = self._refined()

    def set_stencil(self, outer: float):
        """Outer weight b of the order-4 plan's 4-point difference
        (fdtd_set_stencil; -1/24: fourth order)."""
        _lib.check(_lib.lib().fdtd_set_stencil(self._h, float(outer)), "fdtd_set_stencil")

    def set_step(self, n: int):
        _lib.check(_lib.lib().fdtd_set_step(self._h, int(n)), "fdtd_set_step")

    def set_timing(self, per_launch):
        """per_launch: False/0 off, True/1 every step, k >= 1 every k-th step
        (HIP events around each line pass of those steps)."""
        k = int(per_launch) if not isinstance(per_launch, bool) else (1 if per_launch else 0)
        _lib.check(_lib.lib().fdtd_set_timing(self._h, k), "fdtd_set_timing")

    def last_timing(self):
        """{'main_ms', 'yz_ms_avg', 'x_ms_avg', 'yz_launches', 'x_launches'}."""
        main = ctypes.c_double()
        avg = (ctypes.c_double * 2)()
        cnt = (ctypes.c_int * 2)()
        _lib.check(_lib.lib().fdtd_last_timing(self._h, ctypes.byref(main), avg, cnt), "fdtd_last_timing")
        return {"main_ms": main.value, "yz_ms_avg": avg[0], "x_ms_avg": avg[1],
                "yz_launches": cnt[0], "x_launches": cnt[1]}

    def diff_norm(self, Ea, Ha, Eb, Hb):
        """(sum eps|Ea-Eb|^2 + mu|Ha-Hb|^2, sum eps|Eb|^2 + mu|Hb|^2) in FP64 on the
        device; sqrt of their ratio is the energy-weighted relative L2 distance."""
        out = (ctypes.c_double * 2)()
        _lib.check(_lib.lib().fdtd_diff_norm(self._h, _ptrs(Ea, self.dtype, self.shape, self.device),
                                             _ptrs(Ha, self.dtype, self.shape, self.device),
                                             _ptrs(Eb, self.dtype, self.shape, self.device),
                                             _ptrs(Hb, self.dtype, self.shape, self.device), out),
                   "fdtd_diff_norm")
        return out[0], out[1]

    def diff_norm_noalloc(self, Ea, Ha, Eb, Hb):
        """diff_norm through fdtd_diff_norm_noalloc: no device allocation (its
        work area is the library's static per-GPU array; overlapping calls on
        one GPU race)."""
        out = (ctypes.c_double * 2)()
        _lib.check(_lib.lib().fdtd_diff_norm_noalloc(self._h, _ptrs(Ea, self.dtype, self.shape, self.device),
                                                     _ptrs(Ha, self.dtype, self.shape, self.device),
                                                     _ptrs(Eb, self.dtype, self.shape, self.device),
                                                     _ptrs(Hb, self.dtype, self.shape, self.device), out),
                   "fdtd_diff_norm_noalloc")
        return out[0], out[1]

    def set_cg(self, tol: float = 1e-12, maxit: int = 500):
        """Conjugate-gradient controls of a Crank-Nicolson plan."""
        _lib.check(_lib.lib().fdtd_set_cg(self._h, float(tol), int(maxit)), "fdtd_set_cg")

    def last_cg(self):
        """{'iterations': CG iterations of the last run, 'rel_residual': largest final |r|/|b|}."""
        it = ctypes.c_longlong()
        rel = ctypes.c_double()
        _lib.check(_lib.lib().fdtd_last_cg(self._h, ctypes.byref(it), ctypes.byref(rel)), "fdtd_last_cg")
        return {"iterations": it.value, "rel_residual": rel.value}

    def kernel_config(self, axis: int) -> dict:
        """Kernel configuration of the passes along axis 0 (x), 1 (y), 2 (z)."""
        c = _lib.FdtdKernelConfig()
        _lib.check(_lib.lib().fdtd_get_kernel_config(self._h, axis, ctypes.byref(c)), "fdtd_get_kernel_config")
        return {"chunk": c.chunk, "tile_x": c.tile_x, "block_threads": c.block_threads, "remap": c.remap}

    def set_kernel_config(self, axis: int, chunk: int, tile_x: int = 0, block_threads: int = 256, remap: int = 1):
        c = _lib.FdtdKernelConfig(chunk, tile_x, block_threads, remap)
        _lib.check(_lib.lib().fdtd_set_kernel_config(self._h, axis, ctypes.byref(c)), "fdtd_set_kernel_config")

    def autotune(self, reps: int = 3):
        """Time every valid kernel configuration per axis and keep the fastest;
        returns the best mean launch time per axis [ms]."""
        best = (ctypes.c_double * 3)()
        _lib.check(_lib.lib().fdtd_autotune(self._h, int(reps), best), "fdtd_autotune")
        return list(best)

    def grad_eps(self, E, H, nsteps, probe, source: Source | None = None, design_box=None,
                 ckpt_every: int = 50):
        """Probe objective J = dt * sum_n |E(u^n)|^2 at node `probe` = (i, j, k)
        over nsteps steps from the fields E, H (not modified), and, if
        design_box = (i0, i1, j0, j1, k0, k1) is given, dJ/d eps_r over those
        cells as a float64 device tensor of shape (k1-k0, j1-j0, i1-i0)
        (fdtd_grad_eps; fundamental ADI plans).  Returns (J, grad or None)."""
        import torch
        L = _lib.lib()
        pe = _ptrs(E, self.dtype, self.shape, self.device)
        ph = _ptrs(H, self.dtype, self.shape, self.device)
        src = ctypes.byref(source._c()) if source is not None else None
        J = ctypes.c_double()
        i, j, k = (int(v) for v in probe)
        if design_box is None:
            _lib.check(L.fdtd_grad_eps(self._h, pe, ph, int(nsteps), src, i, j, k, None, int(ckpt_every),
                                       ctypes.byref(J), None), "fdtd_grad_eps")
            return J.value, None
        b = [int(v) for v in design_box]
        if len(b) != 6:
            raise ValueError("design_box = (i0, i1, j0, j1, k0, k1)")
        shape = (max(b[5] - b[4], 0), max(b[3] - b[2], 0), max(b[1] - b[0], 0))
        # never hand over a NULL buffer (that selects J only): the library
        # itself rejects an empty or out-of-range box
        buf = torch.empty(max(shape[0] * shape[1] * shape[2], 1), dtype=torch.float64, device=self.device)
        box = (ctypes.c_int * 6)(*b)
        _lib.check(L.fdtd_grad_eps(self._h, pe, ph, int(nsteps), src, i, j, k, box, int(ckpt_every),
                                   ctypes.byref(J), ctypes.c_void_p(buf.data_ptr())), "fdtd_grad_eps")
        return J.value, buf.view(shape)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.lib().fdtd_destroy(self._h), "fdtd_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()



class BatchPlan(Plan):
    """Independent grids stepped together: by default one launch per sub-step
    (its three line passes) over all grids of a group, eight time steps per
    captured HIP graph (fdtd_plan_batch; fundamental forms).  grids: list of
    (nx, ny, nz, eps_r or None)."""

    def __init__(self, grids, dt, dx, dy, dz, scheme="adi", dtype=None, stream=None, device=None,
                 solve_dtype=None, refine=None):
        import torch
        L = _lib.lib()
        self.dtype = dtype if dtype is not None else torch.float32
        solve = solve_dtype if solve_dtype is not None else self.dtype
        code = _dtype_code(self.dtype, solve, refine)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.shapes = []
        keep = []
        descs = (_lib.FdtdDesc * len(grids))()
        for g, (nx, ny, nz, eps_r) in enumerate(grids):
            eps_ptr = None
            if eps_r is not None:
                e = eps_r if isinstance(eps_r, torch.Tensor) else torch.as_tensor(eps_r)
                e = e.to(dtype=torch.float32).contiguous()
                if tuple(e.shape) != (nz, ny, nx):
                    raise ValueError(f"eps_r of grid {g} must have shape {(nz, ny, nx)}")
                keep.append(e)
                eps_ptr = e.data_ptr()
            descs[g] = _lib.FdtdDesc(nx, ny, nz, dt, dx, dy, dz, _lib.SCHEMES[scheme], _lib.FORMS["fundamental"],
                                     code, eps_ptr, None, 0)
            self.shapes.append((nz + 1, ny + 1, nx + 1))
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = s
            h = ctypes.c_void_p()
            _lib.check(L.fdtd_plan_batch(descs, len(grids), ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)),
                       "fdtd_plan_batch")
        self._h = h
        self.scheme, self.form = scheme, "fundamental"
        self.refined = self._refined()

    def run(self, fields, nsteps):
        """fields: list of (E, H) per grid, updated in place (asynchronous)."""
        if len(fields) != len(self.shapes):
            raise ValueError(f"need fields for {len(self.shapes)} grids")
        pe = (ctypes.c_void_p * (3 * len(fields)))()
        ph = (ctypes.c_void_p * (3 * len(fields)))()
        for g, (E, H) in enumerate(fields):
            e = _ptrs(E, self.dtype, self.shapes[g], self.device)
            h = _ptrs(H, self.dtype, self.shapes[g], self.device)
            for c in range(3):
                pe[3 * g + c] = e[c]
                ph[3 * g + c] = h[c]
        _lib.check(_lib.lib().fdtd_run_batch(self._h, pe, ph, int(nsteps)), "fdtd_run_batch")

    def step(self, *a, **k):
        raise TypeError("BatchPlan has no step(); use run(fields, 1)")

    def grad_eps(self, *a, **k):
        raise TypeError("the adjoint gradient is defined for single-grid plans")


def optimized_stencil(theta_max: float) -> float:
    """Outer weight of the 4-point difference that minimizes the squared
    modified-wavenumber error over k dw in [0, theta_max]
    (fdtd_stencil_optimized)."""
    out = ctypes.c_double()
    _lib.check(_lib.lib().fdtd_stencil_optimized(float(theta_max), ctypes.byref(out)), "fdtd_stencil_optimized")
    return out.value


from .autograd import ProbeEnergy, probe_energy  # noqa: E402
