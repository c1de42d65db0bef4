"""libhenry loads, exports every symbol the header declares, and its struct layout
matches the header as compiled by gcc (CPU only: no device calls)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "henry.h")


def _declared():
    txt = open(HEADER).read()
    return re.findall(r"HENRY_API\s+[\w\s\*]+?\b(\w+)\s*\(", txt)


def test_header_declares_the_abi():
    from paper_2403_17018_amd import _lib
    assert sorted(_declared()) == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2403_17018_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert exported == set(_declared())


def test_struct_layout_matches_header(tmp_path):
    """Size and every field offset of each ABI struct, gcc against the ctypes binding."""
    from paper_2403_17018_amd import _lib
    structs = {"henry_problem": _lib.henry_problem, "henry_grid": _lib.henry_grid,
               "henry_solver_opts": _lib.henry_solver_opts, "henry_batch": _lib.henry_batch}
    exprs, want = [], []
    for name, cls in structs.items():
        exprs.append(f"sizeof({name})")
        want.append(ctypes.sizeof(cls))
        for f in cls._fields_:
            exprs.append(f"offsetof({name}, {f[0]})")
            want.append(getattr(cls, f[0]).offset)
    body = "".join(f'printf("%zu\\n", (size_t)({x}));' for x in exprs)
    src = tmp_path / "sz.c"
    src.write_text('#include "henry.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(void){' + body + 'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert dict(zip(exprs, got)) == dict(zip(exprs, want))


def test_defaults_match_the_workload_constants():
    import paper_2403_17018_amd as P
    p = P.problem()
    assert (p.Lx, p.Ly, p.T, p.rho0, p.rho1, p.mu, p.g) == (2.0, 1.0, 36000.0, 1000.0, 1025.0, 1e-3, 9.81)
    assert (p.Dm, p.K_mean, p.q_in, p.corr_len) == (1.88571e-5, 1.020408e-9, 6.6e-5, 0.5)
    o = P.solver_opts()
    assert o.mg_precision == 64 and o.nu_pre == 1 and o.nu_post == 2 and o.coarse_nx == 16 and o.coarse_ny == 8
    assert o.newton_tol == 1e-9 and o.krylov_rtol == 3e-2 and o.newton_extrapolate == 1 and o.newton_predict == 1.0
    assert o.newton_jac_reuse == 1e-3


def test_optimal_samples_host_helper_matches_oracle():
    """mlmc_optimal_samples is host arithmetic (eq. M_ell); compared with the oracle's formula."""
    import paper_2403_17018_amd as P
    from oracle import mlmc as M
    V = [1.4e-5, 2e-6, 5e-7, 1e-7]
    s = [1.156, 4.113, 20.382, 139.0]
    for eps in (0.01, 0.003, 0.001):
        m, cost = P.optimal_samples(V, s, eps)
        o = M.optimal_samples(V, s, eps)
        assert m == list(o["m"]) and cost == pytest.approx(o["cost"], rel=1e-14)
    with pytest.raises(P.HenryError):
        P.optimal_samples([1.0], [0.0], 0.1)
