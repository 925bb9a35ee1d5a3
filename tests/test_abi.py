"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vmg_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("vmg_plan_create", "vmg_solve", "vmg_plan_destroy", "vmg_last_error",
                 "vmg_solve_periodic"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1303_0008_amd import vmg
    lib = vmg.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(vmg.EXPORTS) == declared_functions()


def test_ghost_count_matches_oracle(oracle_mod):
    from paper_1303_0008_amd import vmg
    for n in [(2, 2, 2), (16, 16, 16), (5, 7, 9)]:
        assert vmg.ghost_count(n) == oracle_mod.ghost_count(n)


def test_plan_create_rejects_bad_arguments():
    """Argument validation happens before any device call."""
    from paper_1303_0008_amd import vmg
    lib = vmg.load()
    h = ctypes.c_void_p()
    g = vmg.make_grid(32)
    p = vmg.make_params(0.1, 1.5, tol=-1.0)
    assert lib.vmg_plan_create(ctypes.byref(h), ctypes.byref(g), 1, ctypes.byref(p), None) == vmg.VMG_EINVAL
    assert "tol" in vmg.last_error()
    p = vmg.make_params(0.1, 1.5, tol=1e-8)
    g2 = vmg.make_grid(2)
    assert lib.vmg_plan_create(ctypes.byref(h), ctypes.byref(g2), 1, ctypes.byref(p), None) == vmg.VMG_EINVAL
    arr = (vmg.Grid * 2)(vmg.make_grid(32), vmg.make_grid(32))
    assert lib.vmg_plan_create(ctypes.byref(h), arr, 2, ctypes.byref(p), None) == vmg.VMG_EINVAL
    assert lib.vmg_solve(None, None, None, None, None, None) == vmg.VMG_EINVAL
    # the truncation-error rule needs a coarser level on every grid (an odd Dirichlet grid has none)
    pt = vmg.make_params(0.1, 1.5, tol=1e-8, tau_factor=0.3)
    gd = vmg.make_grid(5, 1 / 64, vmg.DIRICHLET)
    assert lib.vmg_plan_create(ctypes.byref(h), ctypes.byref(gd), 1, ctypes.byref(pt), None) == vmg.VMG_EINVAL
    assert "coarser level" in vmg.last_error()
    # inner cycles: only for the mixed path, never negative
    for prec, inner in ((vmg.FP64, 2), (vmg.MIXED, -1)):
        p = vmg.make_params(0.1, 1.5, tol=1e-8, prec=prec, inner_cycles=inner)
        assert lib.vmg_plan_create(ctypes.byref(h), ctypes.byref(g), 1, ctypes.byref(p), None) == vmg.VMG_EINVAL


def test_mass_assign_rejects_bad_arguments():
    """vmg_mass_assign validates before any device call (Sec. VI assignment)."""
    from paper_1303_0008_amd import vmg
    lib = vmg.load()
    n = (ctypes.c_int32 * 3)(8, 8, 8)
    fake = ctypes.c_void_p(256)         # never dereferenced: each call fails validation first
    need = lib.vmg_mass_assign_workspace(100, n)
    assert need >= 100 * 12
    assert lib.vmg_mass_assign_workspace(0, n) == -1
    args = (n, vmg.ASSIGN_TSC, fake, need, fake, None)
    assert lib.vmg_mass_assign(None, 100, *args) == vmg.VMG_EINVAL
    assert lib.vmg_mass_assign(fake, 0, *args) == vmg.VMG_EINVAL
    assert "n_particles" in vmg.last_error()
    assert lib.vmg_mass_assign(fake, 1 << 31, *args) == vmg.VMG_EINVAL
    assert lib.vmg_mass_assign(fake, 100, n, 3, fake, need, fake, None) == vmg.VMG_EINVAL
    assert "scheme" in vmg.last_error()
    for bad in ((8, 0, 8), (8, 8, 65536)):
        bad = (ctypes.c_int32 * 3)(*bad)
        assert lib.vmg_mass_assign(fake, 100, bad, vmg.ASSIGN_CIC, fake, need, fake, None) == vmg.VMG_EINVAL
    assert lib.vmg_mass_assign(fake, 100, n, vmg.ASSIGN_CIC, fake, need - 1, fake, None) == vmg.VMG_EINVAL
    assert "workspace" in vmg.last_error()
    assert lib.vmg_mass_assign(fake, 100, n, vmg.ASSIGN_CIC, ctypes.c_void_p(264), need, fake,
                               None) == vmg.VMG_EINVAL
    assert lib.vmg_mass_assign(fake, 100, n, vmg.ASSIGN_CIC, None, need, fake, None) == vmg.VMG_EINVAL


def test_solve_levels_rejects_bad_nesting():
    """vmg_solve_levels validates the tree before any device call (Sec. III.C
    refinements: half the parent's cell size, inside the parent)."""
    from paper_1303_0008_amd import vmg
    lib = vmg.load()
    fake = ctypes.c_void_p(256)
    p = vmg.make_params(0.1, 1.5, 1e-8)

    def call(grids, nests):
        n = len(grids)
        res = (vmg.Result * n)()
        return lib.vmg_solve_levels((vmg.Grid * n)(*grids), (vmg.Nest * n)(*nests), n, ctypes.byref(p), fake,
                                    fake, fake, res, None)

    dom = vmg.make_grid(32)
    ok = vmg.make_grid(8, 1 / 64, vmg.DIRICHLET, 32 ** 3, 0)
    # the domain grid must come first, periodic, parent -1
    assert call([ok], [vmg.make_nest(-1)]) == vmg.VMG_EINVAL
    assert call([dom, ok], [vmg.make_nest(0), vmg.make_nest(0)]) == vmg.VMG_EINVAL
    # parent must precede the child; cell size must halve
    assert call([dom, ok], [vmg.make_nest(-1), vmg.make_nest(1)]) == vmg.VMG_EINVAL
    bad_h = vmg.make_grid(8, 1 / 48, vmg.DIRICHLET, 32 ** 3, 0)
    assert call([dom, bad_h], [vmg.make_nest(-1), vmg.make_nest(0)]) == vmg.VMG_EINVAL
    assert "halves" in vmg.last_error()
    # origin outside a periodic parent
    assert call([dom, ok], [vmg.make_nest(-1), vmg.make_nest(0, (64, 0, 0))]) == vmg.VMG_EINVAL
    # under a refinement: one parent cell of margin on every side
    child = vmg.make_grid(4, 1 / 128, vmg.DIRICHLET, 32 ** 3 + 512, 400)
    for origin in ((1, 2, 2), (2, 2, 13)):      # 13 + 4 > 2 * 8 - 2
        assert call([dom, ok, child], [vmg.make_nest(-1), vmg.make_nest(0, (8, 8, 8)),
                                        vmg.make_nest(1, origin)]) == vmg.VMG_EINVAL
        assert "margin" in vmg.last_error()
    # refinements need a ghost array
    res = (vmg.Result * 2)()
    assert lib.vmg_solve_levels((vmg.Grid * 2)(dom, ok), (vmg.Nest * 2)(vmg.make_nest(-1), vmg.make_nest(0)), 2,
                                ctypes.byref(p), fake, None, fake, res, None) == vmg.VMG_EINVAL
