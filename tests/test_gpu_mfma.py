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


# (the last two: deep tanks, 40 and 34 layers at fourth order, whose element
# and node-sum tables and input region exceed what a workgroup stages
# through registers, so the staging's remainder loops run; five tiles per
# block)
@pytest.mark.parametrize("case", [(8, 2, 4, 2 * np.pi, True), (16, 4, 6, 2 * np.pi, True),
                                  (7, 3, 5, 3.0, False), (5, 1, 8, 2.0, False), (9, 8, 3, 4.0, True),
                                  (6, 2, 1, 1.0, False), (4, 2, 2, 1.0, True), (3, 5, 7, 2.0, False),
                                  (4, 40, 4, 2.0, True), (3, 34, 4, 1.5, False)])
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


@pytest.mark.parametrize("case", [(40, 2, 4, 2 * np.pi, True), (37, 4, 6, 3.0, False), (26, 8, 6, 2 * np.pi, True),
                                  (19, 2, 8, 2.0, False), (33, 1, 7, 2 * np.pi, True), (21, 3, 5, 2.5, False)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_several_blocks_per_workgroup_bitwise(case, prec, monkeypatch):
    """The stiffness kernel that runs several blocks per workgroup (chosen for
    launches of thousands of blocks) gives the one-block kernel's result bit
    for bit: forced through SEM_STIFF_BLOCKS on small tanks whose last
    workgroup gets a ragged share of blocks."""
    import torch
    from paper_1512_02548_amd import lib
    nx, nz, P, L, periodic = case
    from oracle.mesh import Mesh as OMesh
    xs = OMesh(nx, 1, P, L, periodic).xs_surf
    k = 2 * np.pi / L
    h = 1.0 - 0.2 * np.cos(k * xs) ** 2
    hx = 0.4 * k * np.cos(k * xs) * np.sin(k * xs)
    m = lib.Mesh(nx, nz, P, L, periodic, h, hx, tiles_per_block=4 if nz > 1 else 2)
    eta = 0.1 * np.cos(k * xs) + 0.03 * np.sin(2 * k * xs)
    ex = 0.1 * k * (-np.sin(k * xs)) + 0.06 * k * np.cos(2 * k * xs)
    m.set_surface(cuda(eta), cuda(ex))
    dt = torch.float64 if prec == 0 else torch.float32
    u = torch.tensor(np.random.default_rng(11).standard_normal(m.n), dtype=dt, device="cuda")
    outs = {}
    for kb in (None, 2, 3):
        if kb is None:
            monkeypatch.delenv("SEM_STIFF_BLOCKS", raising=False)
        else:
            monkeypatch.setenv("SEM_STIFF_BLOCKS", str(kb))
        y = torch.full_like(u, np.nan)
        m.apply_timed(lib.SEM_OP_STIFFNESS, u, y, 1, prec)
        if prec == 0:
            y2 = torch.full_like(u, np.nan)
            m.apply(lib.SEM_OP_STIFFNESS, u, y2)
            outs[kb] = (host(y), host(y2))
        else:
            outs[kb] = (y.cpu().numpy(),)
    for kb in (2, 3):
        for a, b in zip(outs[None], outs[kb]):
            # (the single apply leaves a walled tank's wall line to the fix-up: NaN in both)
            assert np.array_equal(a, b, equal_nan=True), kb
            assert np.isfinite(a[: m.n - (0 if periodic else nz * P + 1)]).all()
