"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

A sanitizer build of ``oracle/vmg_oracle.c`` runs every oracle entry point on
small periodic and Dirichlet grids in a child process started with the ASan
runtime preloaded; any out-of-bounds access, use of freed memory or undefined
behaviour (signed overflow, bad shifts, misaligned access) ends it with a
report.  The values are not checked here (the pins do that), only that the
runs are clean.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import numpy as np
    from oracle import oracle as O
    from paper_1303_0008_amd import inputs as I
    rng = np.random.default_rng(5)
    # periodic 8^3 and 6x4x8 (odd coarse sizes stop the hierarchy early)
    for shape in ((8, 8, 8), (8, 4, 6)):
        d = rng.standard_normal(shape)
        d -= d.mean()
        phi, info = O.solve(d, 0.2, 1.5, tol=1e-9, max_cycles=20)
        O.residual(d, phi, 0.2, 1.5)
        O.relax(d, phi.copy(), 0.2, 1.5, 2)
        O.cell_operator(d, phi, 0.2, 1.5, (1, 2, 3))
        O.truncation_error(d, phi, 0.2, 1.5)
    # Dirichlet 8^3 with ghosts interpolated from a periodic 8^3 parent
    P = rng.standard_normal((8, 8, 8)) * 1e-3
    n = (8, 8, 8)
    gh = O.fill_ghosts(P, n, 1.0 / 16, (4, 4, 4), H=1.0 / 8)
    p0 = O.fill_interior(P, n, 1.0 / 16, (4, 4, 4), H=1.0 / 8)
    d = rng.standard_normal((8, 8, 8))
    phi, info = O.solve(d, 0.2, 1.5, h=1.0 / 16, ghost=gh, phi0=p0, tol=1e-9, max_cycles=20)
    O.residual(d, phi, 0.2, 1.5, h=1.0 / 16, ghost=gh)
    O.truncation_error(d, phi, 0.2, 1.5, h=1.0 / 16, ghost=gh)
    # multilevel tree: domain and one refinement
    root = dict(delta=P * 0 + rng.standard_normal((8, 8, 8)), h=1.0 / 8, parent=-1, origin=(0, 0, 0))
    root["delta"] -= root["delta"].mean()
    ref = dict(delta=rng.standard_normal((8, 8, 8)), h=1.0 / 16, parent=0, origin=(4, 4, 4))
    O.solve_levels([root, ref], 0.2, 1.5, tol=1e-8, max_cycles=20)
    O.total_force(phi, phi, 1.0 / 16)
    pos = rng.random((1000, 3))
    for scheme in ("cic", "tsc"):
        O.mass_assign(pos, 8, scheme)
        O.mass_assign_region(pos, 8, 1.0 / 16, (0.25, 0.25, 0.25), 1000 / 512.0, scheme)
    print("sanitized oracle runs clean")
""")


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle import oracle as O
    lib = O.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's ASan runtime is not installed")
    env = dict(os.environ)
    env.update(VMG_ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle runs clean" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
