"""ctypes binding of libvmg.so (the gfx950 nonlinear multigrid library).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory (``Tensor.data_ptr()``) and the
current HIP stream.  The functions mirror the C ABI in ``include/vmg.h``:
``plan_create``, ``solve``, ``plan_destroy``, ``last_error``,
``solve_periodic``, ``residual``, ``fill_ghosts``, ``fill_interior``, ``ghost_count``,
``smooth``, ``plan_stats``, ``plan_config``, ``plan_level_count``, ``plan_set_schedule``,
``plan_schedule``, ``plan_get_cycle``, ``plan_set_cycle``, ``plan_tune_cycle``, ``plan_time_sweeps``,
``plan_sweep_time``, ``total_force``, ``mass_assign``, ``mass_assign_region``,
``solve_levels``; ``Plan`` and ``LevelsPlan`` wrap plan handles.

There is no fallback: if the library is missing or no GPU is present the
calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvmg.so")

VMG_OK, VMG_EINVAL, VMG_ENOMEM, VMG_EHIP, VMG_ENOCONV, VMG_ENONFINITE = range(6)
STATUS_NAMES = {0: "VMG_OK", 1: "VMG_EINVAL", 2: "VMG_ENOMEM", 3: "VMG_EHIP", 4: "VMG_ENOCONV",
                5: "VMG_ENONFINITE"}
FP64, MIXED = 0, 1
PERIODIC, DIRICHLET = 0, 1
GRAPH, AUTOTUNE = 1, 2


class VmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("bc", ctypes.c_int32), ("h", ctypes.c_double),
                ("offset", ctypes.c_int64), ("ghost_offset", ctypes.c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("kappa", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_cycles", ctypes.c_int32), ("prec", ctypes.c_int32), ("nu1", ctypes.c_int32),
                ("nu2", ctypes.c_int32), ("flags", ctypes.c_uint32), ("inner_cycles", ctypes.c_int32),
                ("tau_factor", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("rms0", ctypes.c_double), ("rms", ctypes.c_double), ("compat_c", ctypes.c_double),
                ("cycles", ctypes.c_int32), ("inner_cycles", ctypes.c_int32),
                ("n_guarded", ctypes.c_int64), ("tau_rms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Cycle(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("inner_cycles", ctypes.c_int32),
                ("coarse_sweeps", ctypes.c_int32), ("coarse_tail", ctypes.c_int32), ("batch_blocks", ctypes.c_int32),
                ("coarse_nu1", ctypes.c_int32), ("coarse_nu2", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class History(ctypes.Structure):
    _fields_ = [("rms", ctypes.c_double), ("cbar", ctypes.c_double), ("n_guarded", ctypes.c_double),
                ("tau_rms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Nest(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_int32), ("origin", ctypes.c_int32 * 3)]


# Every symbol declared in include/vmg.h (checked by the CPU test-suite).
EXPORTS = ["vmg_plan_create", "vmg_solve", "vmg_plan_destroy", "vmg_last_error",
           "vmg_solve_periodic", "vmg_residual", "vmg_fill_ghosts", "vmg_ghost_count",
           "vmg_smooth", "vmg_plan_stats", "vmg_plan_config", "vmg_fill_interior", "vmg_total_force",
           "vmg_mass_assign", "vmg_mass_assign_workspace", "vmg_solve_levels", "vmg_levels_create",
           "vmg_levels_solve", "vmg_levels_destroy", "vmg_mass_assign_region", "vmg_plan_level_count",
           "vmg_plan_set_schedule", "vmg_plan_schedule", "vmg_mass_assign_noalloc", "vmg_plan_get_cycle",
           "vmg_plan_set_cycle", "vmg_plan_tune_cycle", "vmg_plan_time_sweeps", "vmg_plan_sweep_time",
           "vmg_plan_time_levels", "vmg_plan_level_time", "vmg_plan_history"]

_lib = None


def load():
    """Load libvmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1303_0008_amd.build` "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, P = ctypes.c_void_p, ctypes.POINTER
    L.vmg_plan_create.argtypes = [P(vp), P(Grid), ctypes.c_int32, P(Params), vp]
    L.vmg_solve.argtypes = [vp, vp, vp, vp, vp, P(Result)]
    L.vmg_plan_destroy.argtypes = [vp]
    L.vmg_last_error.restype = ctypes.c_char_p
    L.vmg_solve_periodic.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int32, vp, P(ctypes.c_double),
                                     P(ctypes.c_int32), vp]
    L.vmg_residual.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, P(Result)]
    L.vmg_fill_ghosts.argtypes = [vp, P(ctypes.c_int32), ctypes.c_double, P(Grid), P(ctypes.c_int32),
                                  ctypes.c_int32, vp, vp]
    L.vmg_fill_interior.argtypes = [vp, P(ctypes.c_int32), ctypes.c_double, P(Grid), P(ctypes.c_int32),
                                    ctypes.c_int32, vp, vp]
    L.vmg_ghost_count.argtypes = [P(ctypes.c_int32)]
    L.vmg_ghost_count.restype = ctypes.c_int64
    L.vmg_smooth.argtypes = [vp, ctypes.c_int32]
    L.vmg_total_force.argtypes = [vp, vp, P(ctypes.c_int32), ctypes.c_double, vp, vp, vp]
    L.vmg_mass_assign.argtypes = [vp, ctypes.c_int64, P(ctypes.c_int32), ctypes.c_int32, vp, ctypes.c_int64, vp,
                                  vp]
    L.vmg_mass_assign_workspace.argtypes = [ctypes.c_int64, P(ctypes.c_int32)]
    L.vmg_mass_assign_noalloc.argtypes = [vp, ctypes.c_int64, P(ctypes.c_int32), ctypes.c_int32, vp, vp]
    L.vmg_mass_assign_region.argtypes = [vp, ctypes.c_int64, P(ctypes.c_int32), ctypes.c_double,
                                         P(ctypes.c_double), ctypes.c_double, ctypes.c_int32, vp, ctypes.c_int64,
                                         vp, vp]
    L.vmg_solve_levels.argtypes = [P(Grid), P(Nest), ctypes.c_int32, P(Params), vp, vp, vp, P(Result), vp]
    L.vmg_levels_create.argtypes = [P(vp), P(Grid), P(Nest), ctypes.c_int32, P(Params), vp]
    L.vmg_levels_solve.argtypes = [vp, vp, vp, vp, P(Result)]
    L.vmg_levels_destroy.argtypes = [vp]
    L.vmg_levels_destroy.restype = None
    L.vmg_mass_assign_workspace.restype = ctypes.c_int64
    L.vmg_plan_stats.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64)]
    i32p = P(ctypes.c_int32)
    L.vmg_plan_config.argtypes = [vp, i32p, i32p, i32p, i32p, i32p]
    L.vmg_plan_level_count.argtypes = [vp]
    L.vmg_plan_level_count.restype = ctypes.c_int32
    L.vmg_plan_set_schedule.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.vmg_plan_schedule.argtypes = [vp, ctypes.c_int32, i32p, i32p, i32p]
    L.vmg_plan_time_sweeps.argtypes = [vp, ctypes.c_int32]
    L.vmg_plan_sweep_time.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int64)]
    L.vmg_plan_time_levels.argtypes = [vp, ctypes.c_int32]
    L.vmg_plan_level_time.argtypes = [vp, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int64)]
    L.vmg_plan_history.argtypes = [vp, ctypes.c_int32, P(History), ctypes.c_int32, i32p]
    L.vmg_plan_get_cycle.argtypes = [vp, P(Cycle)]
    L.vmg_plan_set_cycle.argtypes = [vp, P(Cycle)]
    L.vmg_plan_tune_cycle.argtypes = [vp, vp, vp, vp, vp, P(Cycle), P(ctypes.c_double)]
    for name in EXPORTS:
        if name not in ("vmg_last_error", "vmg_ghost_count", "vmg_mass_assign_workspace", "vmg_levels_destroy",
                        "vmg_plan_level_count"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def last_error():
    return load().vmg_last_error().decode()


def _check(st, allow=()):
    if st != VMG_OK and st not in allow:
        raise VmgError(st, last_error())
    return st


def _ptr(t):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("arrays must be contiguous float64 tensors on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def ghost_count(n):
    n = (n,) * 3 if isinstance(n, int) else tuple(n)
    return int(load().vmg_ghost_count((ctypes.c_int32 * 3)(*n)))


def make_grid(n, h=None, bc=PERIODIC, offset=0, ghost_offset=0):
    n = (n,) * 3 if isinstance(n, int) else tuple(int(v) for v in n)
    g = Grid()
    g.n[:] = n
    g.bc = bc
    g.h = (1.0 / n[0]) if h is None else h
    g.offset = offset
    g.ghost_offset = ghost_offset
    return g


def make_params(alpha, kappa, tol, max_cycles=100, prec=FP64, nu1=0, nu2=0, flags=0, inner_cycles=0,
                tau_factor=0.0):
    p = Params()
    p.alpha, p.kappa, p.tol = alpha, kappa, tol
    p.max_cycles, p.prec, p.nu1, p.nu2, p.flags = max_cycles, prec, nu1, nu2, flags
    p.inner_cycles = inner_cycles
    p.tau_factor = tau_factor
    return p


def plan_create(grids, params, stream=None):
    """vmg_plan_create: returns an opaque handle (int)."""
    arr = (Grid * len(grids))(*grids)
    h = ctypes.c_void_p()
    _check(load().vmg_plan_create(ctypes.byref(h), arr, len(grids), ctypes.byref(params),
                                  _stream(stream)))
    return h.value


def plan_destroy(handle):
    _check(load().vmg_plan_destroy(ctypes.c_void_p(handle)))


def solve(handle, delta, phi, ghost=None, source=None, n_grids=1, allow_noconv=False):
    """vmg_solve: phi (in: guess, out: solution).  Returns a list of result dicts."""
    res = (Result * n_grids)()
    st = load().vmg_solve(ctypes.c_void_p(handle), _ptr(delta), _ptr(ghost), _ptr(source), _ptr(phi),
                          res)
    _check(st, allow=(VMG_ENOCONV,) if allow_noconv else ())
    out = [r.as_dict() for r in res]
    for r in out:
        r["status"] = st
    return out


def residual(handle, g, delta, phi, d=None, ghost=None, source=None):
    """vmg_residual: residual field (into d, optional) and its RMS for grid g."""
    r = Result()
    _check(load().vmg_residual(ctypes.c_void_p(handle), g, _ptr(delta), _ptr(ghost), _ptr(source),
                               _ptr(phi), _ptr(d), ctypes.byref(r)))
    return r.as_dict()


def solve_periodic(delta, alpha, kappa, tol, phi, precision=FP64, stream=None):
    """vmg_solve_periodic on an n^3 unit box; returns (rms, cycles)."""
    n = delta.shape[-1]
    rms = ctypes.c_double()
    cyc = ctypes.c_int32()
    _check(load().vmg_solve_periodic(_ptr(delta), n, alpha, kappa, tol, precision, _ptr(phi),
                                     ctypes.byref(rms), ctypes.byref(cyc), _stream(stream)))
    return rms.value, cyc.value


def fill_ghosts(parent, parent_h, grids, origins, ghost, stream=None):
    """vmg_fill_ghosts: trilinear refinement boundary values from a periodic parent."""
    n2, n1, n0 = parent.shape
    npar = (ctypes.c_int32 * 3)(n0, n1, n2)
    arr = (Grid * len(grids))(*grids)
    flat = [int(v) for o in origins for v in o]
    org = (ctypes.c_int32 * len(flat))(*flat)
    _check(load().vmg_fill_ghosts(_ptr(parent), npar, parent_h, arr, org, len(grids), _ptr(ghost),
                                  _stream(stream)))


def make_nest(parent, origin=(0, 0, 0)):
    n = Nest()
    n.parent = parent
    n.origin[:] = tuple(int(v) for v in origin)
    return n


def solve_levels(grids, nests, params, delta, ghost, phi, stream=None, allow_noconv=False):
    """vmg_solve_levels: the domain grid (grids[0]) and its nested refinements,
    level by level, each refinement from its parent's interpolated solution.
    delta/ghost/phi: device float64 tensors holding every grid at its offset.
    Returns a list of result dicts (one per grid)."""
    n = len(grids)
    garr = (Grid * n)(*grids)
    narr = (Nest * n)(*nests)
    res = (Result * n)()
    st = load().vmg_solve_levels(garr, narr, n, ctypes.byref(params), _ptr(delta), _ptr(ghost), _ptr(phi), res,
                                 _stream(stream))
    _check(st, allow=(VMG_ENOCONV,) if allow_noconv else ())
    out = [r.as_dict() for r in res]
    for r in out:
        r["status"] = st
    return out


class LevelsPlan:
    """Owning wrapper of a vmg_levels plan (create once, solve many times)."""

    def __init__(self, grids, nests, params, stream=None):
        self.n = len(grids)
        self.handle = ctypes.c_void_p()
        _check(load().vmg_levels_create(ctypes.byref(self.handle), (Grid * self.n)(*grids),
                                        (Nest * self.n)(*nests), self.n, ctypes.byref(params), _stream(stream)))

    def solve(self, delta, ghost, phi, allow_noconv=False):
        res = (Result * self.n)()
        st = load().vmg_levels_solve(self.handle, _ptr(delta), _ptr(ghost), _ptr(phi), res)
        _check(st, allow=(VMG_ENOCONV,) if allow_noconv else ())
        out = [r.as_dict() for r in res]
        for r in out:
            r["status"] = st
        return out

    def close(self):
        if self.handle:
            load().vmg_levels_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fill_interior(parent, parent_h, grids, origins, phi, stream=None):
    """vmg_fill_interior: trilinear initial guess on refinements from a periodic parent."""
    n2, n1, n0 = parent.shape
    npar = (ctypes.c_int32 * 3)(n0, n1, n2)
    arr = (Grid * len(grids))(*grids)
    flat = [int(v) for o in origins for v in o]
    org = (ctypes.c_int32 * len(flat))(*flat)
    _check(load().vmg_fill_interior(_ptr(parent), npar, parent_h, arr, org, len(grids), _ptr(phi),
                                    _stream(stream)))


def total_force(phi_newton, phi, h, psi=None, force=None, stream=None):
    """vmg_total_force: Psi = phi_N + phi/2 and the acceleration -grad Psi on a
    periodic grid (device float64 tensors shaped (n2, n1, n0)).  Returns
    (psi, force) with force shaped (3, n2, n1, n0); psi is None unless given."""
    n2, n1, n0 = phi.shape
    if force is None:
        import torch
        force = torch.empty((3,) + tuple(phi.shape), dtype=phi.dtype, device=phi.device)
    n = (ctypes.c_int32 * 3)(n0, n1, n2)
    _check(load().vmg_total_force(_ptr(phi_newton), _ptr(phi), n, float(h), _ptr(psi), _ptr(force),
                                  _stream(stream)))
    return psi, force


ASSIGN_CIC, ASSIGN_TSC = 1, 2


def mass_assign_workspace(n_particles, n):
    """vmg_mass_assign_workspace: device workspace bytes for mass_assign."""
    nn = (n,) * 3 if isinstance(n, int) else tuple(int(v) for v in n)
    return int(load().vmg_mass_assign_workspace(int(n_particles), (ctypes.c_int32 * 3)(*nn)))


def mass_assign(pos, n, scheme=ASSIGN_TSC, delta=None, workspace=None, stream=None):
    """vmg_mass_assign: density contrast of unit-mass particles (device float64
    tensor of shape (N, 3), columns x, y, z in box units) on a periodic grid of
    n cells (int or (n0, n1, n2)); returns delta shaped (n2, n1, n0).
    `workspace` (a device uint8 tensor of at least mass_assign_workspace bytes)
    is allocated when not given."""
    import torch
    nn = (n,) * 3 if isinstance(n, int) else tuple(int(v) for v in n)
    if delta is None:
        delta = torch.empty(nn[::-1], dtype=torch.float64, device=pos.device)
    npart = int(pos.shape[0]) if pos.dim() else 0
    if workspace is None:
        need = mass_assign_workspace(npart, nn)
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=pos.device)
    if not workspace.is_cuda or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 tensor on the GPU")
    c = (ctypes.c_int32 * 3)(*nn)
    _check(load().vmg_mass_assign(_ptr(pos), npart, c, int(scheme), ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel(), _ptr(delta), _stream(stream)))
    return delta


def mass_assign_noalloc(pos, n, delta, scheme=ASSIGN_TSC, stream=None):
    """vmg_mass_assign_noalloc: mass_assign with the library's static workspace
    (allocates nothing; ``delta`` (n2, n1, n0) float64 must be given)."""
    nn = (n,) * 3 if isinstance(n, int) else tuple(int(v) for v in n)
    npart = int(pos.shape[0]) if pos.dim() else 0
    _check(load().vmg_mass_assign_noalloc(_ptr(pos), npart, (ctypes.c_int32 * 3)(*nn), int(scheme), _ptr(delta),
                                          _stream(stream)))
    return delta


def mass_assign_region(pos, n, h, corner, mean_count, scheme=ASSIGN_TSC, delta=None, workspace=None, stream=None):
    """vmg_mass_assign_region: density contrast on a refinement region of n cells
    (int or (n0, n1, n2)) of size h, cell (0,0,0) corner at ``corner`` (box
    units); mean_count = the box's mean particles per cell of size h.  Returns
    delta shaped (n2, n1, n0)."""
    import torch
    nn = (n,) * 3 if isinstance(n, int) else tuple(int(v) for v in n)
    if delta is None:
        delta = torch.empty(nn[::-1], dtype=torch.float64, device=pos.device)
    npart = int(pos.shape[0]) if pos.dim() else 0
    if workspace is None:
        workspace = torch.empty(max(mass_assign_workspace(npart, nn), 1), dtype=torch.uint8, device=pos.device)
    if not workspace.is_cuda or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 tensor on the GPU")
    c = (ctypes.c_int32 * 3)(*nn)
    cr = (ctypes.c_double * 3)(*[float(v) for v in corner])
    _check(load().vmg_mass_assign_region(_ptr(pos), npart, c, float(h), cr, float(mean_count), int(scheme),
                                         ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _ptr(delta),
                                         _stream(stream)))
    return delta


def smooth(handle, sweeps):
    """vmg_smooth: finest-level smoother sweeps on the plan's state (measurement hook)."""
    _check(load().vmg_smooth(ctypes.c_void_p(handle), sweeps))


def plan_stats(handle):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().vmg_plan_stats(ctypes.c_void_p(handle), ctypes.byref(a), ctypes.byref(b),
                                 ctypes.byref(c)))
    return dict(cell_updates=a.value, finest_sweeps=b.value, finest_cells=c.value)


def plan_config(handle):
    """vmg_plan_config: the schedule the plan uses (tile height, z chunk, nu1, nu2, coarse sweeps)."""
    v = [ctypes.c_int32() for _ in range(5)]
    _check(load().vmg_plan_config(ctypes.c_void_p(handle), *[ctypes.byref(x) for x in v]))
    return dict(zip(("tile_y", "z_chunk", "nu1", "nu2", "coarse_sweeps"), (x.value for x in v)))


def plan_level_count(handle):
    """vmg_plan_level_count: levels of the plan that run the fused sweep."""
    return int(load().vmg_plan_level_count(ctypes.c_void_p(handle)))


def plan_set_schedule(handle, level, tile_y, z_chunk, pipe=1):
    """vmg_plan_set_schedule: install a sweep schedule on one level: tile height, z chunk and
    pipe 0/1 (the z march with three- or four-plane rings) or 2 (8^3 bricks: up to two sweeps
    per launch on coarser periodic levels, one on any level of a Dirichlet batch)."""
    _check(load().vmg_plan_set_schedule(ctypes.c_void_p(handle), int(level), int(tile_y), int(z_chunk), int(pipe)))


def plan_schedule(handle, level):
    """vmg_plan_schedule: (tile_y, z_chunk, pipe) the fused sweep of a level runs."""
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().vmg_plan_schedule(ctypes.c_void_p(handle), int(level), ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)))
    return a.value, b.value, c.value


def plan_time_sweeps(handle, enable=True):
    """vmg_plan_time_sweeps: time every finest-level sweep of later solves with HIP events."""
    _check(load().vmg_plan_time_sweeps(ctypes.c_void_p(handle), 1 if enable else 0))


def plan_sweep_time(handle):
    """vmg_plan_sweep_time: (summed microseconds, launches) of the timed finest sweeps."""
    us, n = ctypes.c_double(), ctypes.c_int64()
    _check(load().vmg_plan_sweep_time(ctypes.c_void_p(handle), ctypes.byref(us), ctypes.byref(n)))
    return us.value, n.value


def plan_time_levels(handle, enable=True):
    """vmg_plan_time_levels: time each level's share of later iterations with HIP events."""
    _check(load().vmg_plan_time_levels(ctypes.c_void_p(handle), 1 if enable else 0))


def plan_level_time(handle, level):
    """vmg_plan_level_time: (summed microseconds, iterations timed) of a level."""
    us, n = ctypes.c_double(), ctypes.c_int64()
    _check(load().vmg_plan_level_time(ctypes.c_void_p(handle), int(level), ctypes.byref(us), ctypes.byref(n)))
    return us.value, n.value


def plan_history(handle, grid=0):
    """vmg_plan_history: the norms of the last solve's initial guess and after each
    iteration, as a list of dicts (rms, cbar, n_guarded, tau_rms)."""
    n = ctypes.c_int32()
    _check(load().vmg_plan_history(ctypes.c_void_p(handle), int(grid), None, 0, ctypes.byref(n)))
    buf = (History * max(n.value, 1))()
    _check(load().vmg_plan_history(ctypes.c_void_p(handle), int(grid), buf, n.value, ctypes.byref(n)))
    return [buf[i].as_dict() for i in range(n.value)]


def write_history_jsonl(path, history, **meta):
    """Append one JSON line per iteration of a residual history (plan_history) to
    ``path``: {"iteration": k, "rms": ..., ...} plus the ``meta`` fields."""
    import json
    with open(path, "a") as fh:
        for k, h in enumerate(history):
            fh.write(json.dumps(dict(meta, iteration=k, **h)) + "\n")


def plan_get_cycle(handle):
    """vmg_plan_get_cycle: the plan's cycle schedule as a dict."""
    c = Cycle()
    _check(load().vmg_plan_get_cycle(ctypes.c_void_p(handle), ctypes.byref(c)))
    return c.as_dict()


def plan_set_cycle(handle, **fields):
    """vmg_plan_set_cycle: change fields of the plan's cycle schedule (others kept)."""
    c = Cycle()
    _check(load().vmg_plan_get_cycle(ctypes.c_void_p(handle), ctypes.byref(c)))
    for k, v in fields.items():
        setattr(c, k, int(v))
    _check(load().vmg_plan_set_cycle(ctypes.c_void_p(handle), ctypes.byref(c)))


def plan_tune_cycle(handle, delta, phi_work, ghost=None, source=None):
    """vmg_plan_tune_cycle: time solves of this input for candidate cycle
    schedules, install the fastest; returns (cycle dict, median ms)."""
    c = Cycle()
    ms = ctypes.c_double()
    _check(load().vmg_plan_tune_cycle(ctypes.c_void_p(handle), _ptr(delta), _ptr(ghost), _ptr(source),
                                      _ptr(phi_work), ctypes.byref(c), ctypes.byref(ms)))
    return c.as_dict(), ms.value


class Plan:
    """Owning wrapper of a plan handle."""

    def __init__(self, grids, params, stream=None):
        self.grids = list(grids)
        self.handle = plan_create(self.grids, params, stream)

    def solve(self, delta, phi, ghost=None, source=None, allow_noconv=False):
        return solve(self.handle, delta, phi, ghost, source, len(self.grids), allow_noconv)

    def residual(self, g, delta, phi, d=None, ghost=None, source=None):
        return residual(self.handle, g, delta, phi, d, ghost, source)

    def smooth(self, sweeps):
        smooth(self.handle, sweeps)

    def stats(self):
        return plan_stats(self.handle)

    def config(self):
        return plan_config(self.handle)

    def level_count(self):
        return plan_level_count(self.handle)

    def set_schedule(self, level, tile_y, z_chunk, pipe=1):
        plan_set_schedule(self.handle, level, tile_y, z_chunk, pipe)

    def schedule(self, level):
        return plan_schedule(self.handle, level)

    def time_sweeps(self, enable=True):
        plan_time_sweeps(self.handle, enable)

    def sweep_time(self):
        return plan_sweep_time(self.handle)

    def time_levels(self, enable=True):
        plan_time_levels(self.handle, enable)

    def level_time(self, level):
        return plan_level_time(self.handle, level)

    def history(self, grid=0):
        return plan_history(self.handle, grid)

    def cycle(self):
        return plan_get_cycle(self.handle)

    def set_cycle(self, **fields):
        plan_set_cycle(self.handle, **fields)

    def tune_cycle(self, delta, phi_work, ghost=None, source=None):
        return plan_tune_cycle(self.handle, delta, phi_work, ghost, source)

    def close(self):
        if self.handle:
            plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_field(delta, alpha, kappa, tol=1e-10, precision=FP64, max_cycles=100, phi0=None, flags=0,
                nu1=0, nu2=0):
    """Convenience: solve one periodic grid given a (n2, n1, n0) float64 CUDA tensor."""
    import torch
    n2, n1, n0 = delta.shape
    phi = torch.zeros_like(delta) if phi0 is None else phi0.clone()
    with Plan([make_grid((n0, n1, n2))], make_params(alpha, kappa, tol, max_cycles, precision, nu1, nu2,
                                                     flags)) as p:
        info = p.solve(delta.contiguous(), phi)[0]
    return phi, info
