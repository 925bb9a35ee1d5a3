"""ctypes wrapper of ``vmg_oracle.c`` -- TEST INFRASTRUCTURE ONLY.

Plain FP64 CPU implementation of the discrete Vainshtein equation of Li, Zhao &
Koyama (Sec. III.A-III.C): the paper's Sigma_ijk with splitting constant w,
the sign(alpha_p) root, lexicographic Newton-Gauss-Seidel and FAS V-cycles.
Conventions: ``alpha`` is the coefficient of the nonlinear term in
Lap(phi) + alpha[(Lap phi)^2 - (d_i d_j phi)^2] = kappa*delta, i.e. the
reciprocal of the paper's alpha (= 3 beta a^4 / R_c^2).

Fields are numpy float64 arrays of shape (n2, n1, n0) (x fastest).  Dirichlet
ghosts use the compact order documented in ``vmg_oracle.c`` (``ghosts_to_pad``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
W_PAPER = 1.0 / 3.0
_lib = None
# VMG_ORACLE_LIB names another build of vmg_oracle.c to load instead (the
# sanitizer build of the tests); it is used as it is, never rebuilt here
_LIB_ENV = "VMG_ORACLE_LIB"


def build(force=True):
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", _LIB, _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(cmd)
    return _LIB


def build_sanitized(path):
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal) into ``path``.  Load it by setting VMG_ORACLE_LIB=path
    in a process started with the ASan runtime preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", path, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return path


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get(_LIB_ENV)
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        ip = P(ctypes.c_int)
        L.or_residual.argtypes = [ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, dp, dp, dp, dp, dp, dp]
        L.or_solve.argtypes = [ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, dp]
        L.or_relax.argtypes = [ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, dp, dp, dp, dp, ctypes.c_int]
        L.or_cell_operator.argtypes = [ip, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, dp]
        L.or_fill_ghosts.argtypes = [ip, ctypes.c_double, dp, ip, ctypes.c_double, ip, dp]
        L.or_fill_interior.argtypes = [ip, ctypes.c_double, dp, ip, ctypes.c_double, ip, dp]
        L.or_total_force.argtypes = [ip, ctypes.c_double, dp, dp, dp, dp]
        L.or_mass_assign.argtypes = [dp, ctypes.c_long, ip, ctypes.c_int, dp]
        L.or_mass_assign_region.argtypes = [dp, ctypes.c_long, ip, ctypes.c_double, dp, ctypes.c_double,
                                             ctypes.c_int, dp]
        L.or_truncation_error.argtypes = [ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, dp, dp, dp, dp, dp]
        L.or_ghost_count.argtypes = [ip]
        L.or_ghost_count.restype = ctypes.c_long
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ivec(v):
    return (ctypes.c_int * 3)(*[int(x) for x in v])


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _dims(delta):
    n2, n1, n0 = delta.shape
    return (n0, n1, n2)


def ghost_count(n):
    return int(lib().or_ghost_count(_ivec(n)))


def residual(delta, phi, alpha, kappa, h=None, ghost=None, source=None, w=W_PAPER, want_field=True):
    """Residual d = L^h phi + cbar - f of a given phi.  Returns (d or None, info dict)."""
    delta, phi, ghost, source = _f64(delta), _f64(phi), _f64(ghost), _f64(source)
    n = _dims(delta)
    h = 1.0 / n[0] if h is None else h
    periodic = 1 if ghost is None else 0
    d = np.empty_like(delta) if want_field else None
    st = np.zeros(4)
    lib().or_residual(_ivec(n), periodic, h, alpha, kappa, w, _dp(delta), _dp(ghost), _dp(source),
                      _dp(phi), _dp(d), _dp(st))
    return d, dict(rms=st[0], cbar=st[1], mean_root=st[2], n_guarded=int(st[3]))


def solve(delta, alpha, kappa, h=None, ghost=None, source=None, phi0=None, tol=0.0, max_cycles=200,
          nu1=2, nu2=2, w=W_PAPER):
    """Solve the discrete equation (periodic if ``ghost`` is None, else Dirichlet).
    tol=0 iterates to the FP64 rounding floor (stagnation).  Returns (phi, info)."""
    delta, ghost, source = _f64(delta), _f64(ghost), _f64(source)
    n = _dims(delta)
    h = 1.0 / n[0] if h is None else h
    periodic = 1 if ghost is None else 0
    phi = np.zeros_like(delta) if phi0 is None else np.array(phi0, dtype=np.float64, order="C")
    info = np.zeros(4)
    lib().or_solve(_ivec(n), periodic, h, alpha, kappa, w, _dp(delta), _dp(ghost), _dp(source),
                   _dp(phi), tol, max_cycles, nu1, nu2, _dp(info))
    return phi, dict(rms=info[0], cycles=int(info[1]), cbar=info[2], n_guarded=int(info[3]))


def relax(delta, phi, alpha, kappa, sweeps, h=None, ghost=None, source=None, w=W_PAPER):
    """``sweeps`` lexicographic Newton-Gauss-Seidel sweeps, no multigrid."""
    delta, ghost, source = _f64(delta), _f64(ghost), _f64(source)
    n = _dims(delta)
    h = 1.0 / n[0] if h is None else h
    phi = np.array(phi, dtype=np.float64, order="C")
    lib().or_relax(_ivec(n), 1 if ghost is None else 0, h, alpha, kappa, w, _dp(delta), _dp(ghost),
                   _dp(source), _dp(phi), sweeps)
    return phi


def cell_operator(delta, phi, alpha, kappa, ijk, h=None, ghost=None, w=W_PAPER):
    """(L^h phi, dL/dphi, Sigma_ijk, root) at one cell (Sec. III.B)."""
    delta, phi, ghost = _f64(delta), _f64(phi), _f64(ghost)
    n = _dims(delta)
    h = 1.0 / n[0] if h is None else h
    out = np.zeros(4)
    lib().or_cell_operator(_ivec(n), 1 if ghost is None else 0, h, alpha, kappa, w, _dp(delta),
                           _dp(ghost), _dp(phi), int(ijk[0]), int(ijk[1]), int(ijk[2]), _dp(out))
    return tuple(out)


def fill_interior(parent, n, h, origin, H=None):
    """Initial guess on a patch (n cells of size h, cell (0,0,0) at origin*h from
    the parent's cell (0,0,0) corner): trilinear interpolation of the
    cell-centred ``parent`` (cells of size H, default: the unit box; periodic
    indexing) at every cell centre, shaped (n2, n1, n0)."""
    parent = _f64(parent)
    npar = _dims(parent)
    H = 1.0 / npar[0] if H is None else H
    nn = (n,) * 3 if np.isscalar(n) else tuple(n)
    out = np.zeros(nn[::-1])
    rc = lib().or_fill_interior(_ivec(npar), H, _dp(parent), _ivec(nn), h, _ivec(origin), _dp(out))
    assert rc == 0
    return out


def fill_ghosts(parent, n, h, origin, H=None):
    """Ghost shell of a patch (n cells of size h, cell (0,0,0) at origin*h from
    the parent's cell (0,0,0) corner) by trilinear interpolation of the
    cell-centred ``parent`` field (cells of size H, default: the unit box;
    periodic indexing)."""
    parent = _f64(parent)
    npar = _dims(parent)
    H = 1.0 / npar[0] if H is None else H
    nn = (n,) * 3 if np.isscalar(n) else tuple(n)
    g = np.zeros(ghost_count(nn))
    rc = lib().or_fill_ghosts(_ivec(npar), H, _dp(parent), _ivec(nn), h, _ivec(origin), _dp(g))
    assert rc == 0
    return g


def solve_levels(levels, alpha, kappa, tol=0.0, max_cycles=200):
    """Multilevel solve (Sec. III.C: the domain grid and every refinement are
    solved, a refinement taking its boundary values interpolated from the
    coarser level; Sec. IV.D: a refinement over the overdensity with boundary
    values from the domain grid).  ``levels``: list of dicts in parent-before-
    child order with keys delta (n2, n1, n0), h, parent (-1 for the root),
    origin (3 ints: cell (0,0,0) of the grid in its own cells from the
    parent's cell (0,0,0) corner) and, for a root, ghost (None: periodic).
    Each refinement starts from the trilinear interpolation of its parent's
    solution (ghost shell and interior) and is solved to ``tol``.  Returns
    (phis, infos)."""
    phis, infos = [], []
    for g in levels:
        if g["parent"] < 0:
            phi, info = solve(g["delta"], alpha, kappa, h=g["h"], ghost=g.get("ghost"), tol=tol,
                              max_cycles=max_cycles)
        else:
            par = levels[g["parent"]]
            n = _dims(g["delta"])
            P = phis[g["parent"]]
            ghost = fill_ghosts(P, n, g["h"], g["origin"], H=par["h"])
            phi0 = fill_interior(P, n, g["h"], g["origin"], H=par["h"])
            phi, info = solve(g["delta"], alpha, kappa, h=g["h"], ghost=ghost, phi0=phi0, tol=tol,
                              max_cycles=max_cycles)
            info["ghost"] = ghost
        phis.append(phi)
        infos.append(info)
    return phis, infos


def total_force(phi_n, phi, h):
    """Total potential Psi = phi_N + phi/2 (Sec. II.B) and the acceleration
    -grad Psi by periodic central differences (Sec. III.B) on a grid of cell
    size h.  Returns (psi, g) with g shaped (3, n2, n1, n0): gx, gy, gz."""
    phi_n, phi = _f64(phi_n), _f64(phi)
    n = _dims(phi)
    psi = np.zeros_like(phi)
    g = np.zeros((3,) + phi.shape)
    rc = lib().or_total_force(_ivec(n), float(h), _dp(phi_n), _dp(phi), _dp(psi), _dp(g))
    assert rc == 0
    return psi, g


def truncation_error(delta, phi, alpha, kappa, h=None, ghost=None, w=W_PAPER):
    """Truncation-error estimate tau^h = L^H(R phi) - R L^h(phi) of Sec. III.C on
    the next coarser level of a grid with even sides: periodic if ``ghost`` is
    None, else Dirichlet with those boundary values (the coarse level reads their
    restriction).  Returns (tau, rms): rms is the RMS of tau, with its mean
    removed on a periodic grid."""
    delta, phi, ghost = _f64(delta), _f64(phi), _f64(ghost)
    n = _dims(delta)
    h = 1.0 / n[0] if h is None else h
    tau = np.zeros(tuple(s // 2 for s in delta.shape))
    rms = ctypes.c_double()
    rc = lib().or_truncation_error(_ivec(n), 1 if ghost is None else 0, h, alpha, kappa, w, _dp(delta),
                                   _dp(ghost), _dp(phi), _dp(tau),
                                   ctypes.cast(ctypes.pointer(rms), ctypes.POINTER(ctypes.c_double)))
    assert rc == 0
    return tau, rms.value


def mass_assign(pos, n, scheme="tsc"):
    """Density contrast delta = rho/mean(rho) - 1 of unit-mass particles (pos:
    N x 3, box units in [0, 1), columns x, y, z) on a periodic unit box of n
    cells (int or (n0, n1, n2)) by cloud-in-cell ("cic") or triangular-shaped
    cloud ("tsc", the scheme of Sec. VI) assignment; shaped (n2, n1, n0)."""
    pos = _f64(pos)
    nn = (n,) * 3 if np.isscalar(n) else tuple(n)
    out = np.zeros(nn[::-1])
    rc = lib().or_mass_assign(_dp(pos), pos.shape[0], _ivec(nn), {"cic": 1, "tsc": 2}[scheme], _dp(out))
    assert rc == 0
    return out


def mass_assign_region(pos, n, h, corner, mean_count, scheme="tsc"):
    """Density contrast on a refinement region of n cells (int or (n0, n1, n2))
    of size h with cell (0,0,0) corner at ``corner`` (box units, not periodic):
    mass per cell / mean_count - 1, mean_count the box's mean particles per cell
    of this size; shaped (n2, n1, n0)."""
    pos = _f64(pos)
    nn = (n,) * 3 if np.isscalar(n) else tuple(n)
    out = np.zeros(nn[::-1])
    c = np.asarray(corner, dtype=np.float64)
    rc = lib().or_mass_assign_region(_dp(pos), pos.shape[0], _ivec(nn), float(h), _dp(c), float(mean_count),
                                     {"cic": 1, "tsc": 2}[scheme], _dp(out))
    assert rc == 0
    return out
