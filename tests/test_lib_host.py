"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/sem.h declares, validates arguments on the host, and builds the same
mesh (node coordinates, surface nodes) as the oracle.  No device calls."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "sem.h")).read()
    return sorted(set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    from paper_1512_02548_amd import lib
    names = header_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIBPATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def make(nx, nz, P, L, periodic, **kw):
    from paper_1512_02548_amd import lib
    ns = P * nx + (0 if periodic else 1)
    return lib.Mesh(nx, nz, P, L, periodic, np.ones(ns), np.zeros(ns), bind=False, **kw)


@pytest.mark.parametrize("nx,nz,P,periodic", [(8, 2, 4, True), (5, 3, 6, False), (4, 1, 2, True), (3, 2, 8, False)])
def test_mesh_matches_oracle(nx, nz, P, periodic):
    from oracle.mesh import Mesh as OMesh
    L = 2.5
    m = make(nx, nz, P, L, periodic)
    om = OMesh(nx, nz, P, L, periodic)
    assert m.n == om.n and m.ns == om.ns
    x, s = m.node_coords()
    # same node set (match by coordinates)
    a = np.lexsort((np.round(s, 10), np.round(x, 10)))
    b = np.lexsort((np.round(om.sigma, 10), np.round(om.x, 10)))
    assert np.max(np.abs(x[a] - om.x[b])) < 1e-13 and np.max(np.abs(s[a] - om.sigma[b])) < 1e-13
    # surface nodes in x order
    xs = m.surface_x()
    assert np.max(np.abs(xs - om.xs_surf)) < 1e-13
    assert m.info.n_elem == om.E and m.info.np == om.Np


def test_host_argument_checks():
    from paper_1512_02548_amd import lib
    with pytest.raises(lib.SemError):
        make(8, 2, 9, 1.0, True)          # order out of range
    with pytest.raises(lib.SemError):
        make(1, 2, 4, 1.0, True)          # periodic needs nx >= 2
    with pytest.raises(lib.SemError):
        make(8, 2, 4, 1.0, True, filter_ic=1, filter_sigma=0.9)   # would filter vertex modes
    with pytest.raises(lib.SemError):
        make(8, 2, 4, -1.0, True)
    m = make(8, 2, 4, 1.0, True)
    assert m.info.workspace_bytes > 0
    # device calls on an unbound mesh are rejected on the host
    import ctypes as C
    code = lib.sem_set_surface(m.handle, None, None, None)
    assert code == lib.SEM_E_INVAL


@pytest.mark.parametrize("periodic", [True, False])
def test_workspace_layout_complete(periodic):
    """sem_mesh_bind checks that every device array the kernels use has a
    place in the workspace before it uploads anything; on a host without a
    GPU the call must get past that check and fail only at the first upload."""
    import ctypes as C
    import torch
    from paper_1512_02548_amd import lib
    if torch.cuda.is_available():
        pytest.skip("checks the no-device path")
    m = make(8, 2, 4, 6.28, periodic)
    code = lib.sem_mesh_bind(m.handle, C.c_void_p(1 << 20), m.info.workspace_bytes, None)
    assert code == lib.SEM_E_DEVICE, lib.sem_last_error()


@pytest.mark.parametrize("P,Pf,ic,sf", [(1, 2, 2, 0.9), (4, 6, 3, 0.95), (6, 9, 5, 0.995), (8, 12, 8, 0.5)])
def test_reference_operators_match_oracle(P, Pf, ic, sf):
    """The host builder's Dr, Ds, M (matched by node coordinates), filter F,
    fine-grid interpolation I and fine mass M_f agree with the oracle's to
    rounding (relative 1e-13 of each matrix's largest entry)."""
    from oracle.refelem import Ref1D, RefTri, filter_matrix, fine_grid
    from paper_1512_02548_amd import lib
    h = lib.reference_operators(P, Pf, ic, sf)
    ref = RefTri(P)
    key = lambda r, s: [(round(a, 10), round(b, 10)) for a, b in zip(r, s)]
    pos = {k: i for i, k in enumerate(key(ref.r, ref.s))}
    perm = np.array([pos[k] for k in key(h["r"], h["s"])])     # host node i = oracle node perm[i]
    assert np.max(np.abs(h["r"] - ref.r[perm])) < 1e-14 and np.max(np.abs(h["s"] - ref.s[perm])) < 1e-14
    for name, A in (("Dr", ref.Dr), ("Ds", ref.Ds), ("M", ref.M)):
        B = A[np.ix_(perm, perm)]
        assert np.max(np.abs(h[name] - B)) < 1e-13 * np.max(np.abs(B)), name
    I, Mf = fine_grid(P, Pf)
    for name, B in (("F", filter_matrix(P, ic, sf)), ("I", I), ("Mf", Mf)):
        assert np.max(np.abs(h[name] - B)) < 1e-13 * np.max(np.abs(B)), name
    with pytest.raises(lib.SemError):
        lib.reference_operators(P, P - 1 if P > 1 else 0)
