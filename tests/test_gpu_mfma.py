"""Matrix-core checks: the lane layout the MFMA kernels assume, and the MFMA
stiffness apply against the reference vector-ALU kernel and the oracle."""
import numpy as np
import pytest

from helpers import Pair, cuda, host, oracle_fields, rel_err

pytestmark = pytest.mark.gpu


def test_mfma_lane_layout():
    from paper_1512_02548_amd import lib
    m = lib.Mesh(8, 2, 4, 2 * np.pi, True, np.ones(32), np.zeros(32))
    err, raw = m.selftest_mfma(raw=True)
    np.set_printoptions(linewidth=200)
    print("f64 lanes x v:\n", raw[:256].reshape(64, 4))
    print("f32 lanes x v:\n", raw[256:].reshape(64, 4))
    assert err == 0.0


@pytest.mark.parametrize("case", [(8, 2, 4, 2 * np.pi, True), (16, 4, 6, 2 * np.pi, True),
                                  (7, 3, 5, 3.0, False), (5, 1, 8, 2.0, False), (9, 8, 3, 4.0, True),
                                  (6, 2, 1, 1.0, False), (4, 2, 2, 1.0, True), (3, 5, 7, 2.0, False)])
def test_mfma_stiffness_matches_reference_and_oracle(case):
    nx, nz, P, L, periodic = case
    from oracle.mesh import Mesh as OMesh
    xs = OMesh(nx, 1, P, L, periodic).xs_surf
    k = 2 * np.pi / L
    eta = 0.1 * np.cos(k * xs) + 0.03 * np.sin(2 * k * xs)
    h = 1.0 - 0.2 * np.cos(k * xs) ** 2
    hx = 0.4 * k * np.cos(k * xs) * np.sin(k * xs)
    pm = Pair(nx, nz, P, L, periodic, h, hx, variant=0)           # MFMA
    from paper_1512_02548_amd import lib
    ref = lib.Mesh(nx, nz, P, L, periodic, h, hx, variant=1)      # reference kernel
    of = oracle_fields(pm, eta, np.sin(k * xs))
    ex = cuda(of["etax"])
    pm.m.set_surface(cuda(eta), ex)
    ref.set_surface(cuda(eta), ex)
    u_or = np.random.default_rng(3).standard_normal(pm.om.n)
    u = cuda(pm.to_lib(u_or))
    y1, y2 = cuda(np.zeros(pm.m.n)), cuda(np.zeros(pm.m.n))
    pm.m.apply(lib.SEM_OP_STIFFNESS, u, y1)
    ref.apply(lib.SEM_OP_STIFFNESS, u, y2)
    assert rel_err(host(y1), host(y2)) < 1e-13
    assert rel_err(pm.to_oracle(host(y1)), of["A"] @ u_or) < 1e-13
