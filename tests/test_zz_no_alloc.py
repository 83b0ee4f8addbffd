"""sem_free_surface_rhs_noalloc (scratch in the library's static device array)
against sem_free_surface_rhs (scratch in the mesh workspace), through the
C ABI: bitwise the same right-hand sides on two calls in a row, the second
on a smaller tank, and a clear error for a tank too large for the array."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def tank_inputs(nx, nz, P, L, periodic, Pf, seed):
    import torch
    from paper_1512_02548_amd import lib
    ns = nx * P + (0 if periodic else 1)
    m = lib.Mesh(nx, nz, P, L, periodic, np.ones(ns), np.zeros(ns), overint=Pf)
    xs = m.surface_x()
    rng = np.random.default_rng(seed)
    k = 2 * np.pi / L
    eta = 0.1 * np.cos(k * xs) + 0.02 * rng.standard_normal() * np.sin(3 * k * xs)
    etax = -0.1 * k * np.sin(k * xs)
    phix = 0.5 * np.cos(k * xs + 0.3)
    w = 0.4 * np.sin(k * xs)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    return m, [t(eta), t(etax), t(phix), t(w)]


def both(m, ins):
    import torch
    ref = [torch.full_like(ins[0], np.nan) for _ in range(2)]
    out = [torch.full_like(ins[0], np.nan) for _ in range(2)]
    m.free_surface_rhs(*ins, *ref)
    m.free_surface_rhs_noalloc(*ins, *out)
    torch.cuda.synchronize()
    return [r.cpu().numpy() for r in ref], [o.cpu().numpy() for o in out]


def test_noalloc_matches_workspace_entry_point_twice_then_rejects_oversize():
    from paper_1512_02548_amd import lib
    # first call: 48 columns, P = 6, over-integrated at Pf = 9, periodic
    m1, in1 = tank_inputs(48, 2, 6, 2 * np.pi, True, 9, 1)
    ref, out = both(m1, in1)
    for r, o in zip(ref, out):
        assert np.all(np.isfinite(o)) and np.array_equal(r, o)
    # second call: a smaller walled tank, P = 4 (the array keeps the first
    # call's larger contents; nothing of them may leak into this result)
    m2, in2 = tank_inputs(9, 1, 4, 3.0, False, 4, 2)
    ref, out = both(m2, in2)
    for r, o in zip(ref, out):
        assert np.all(np.isfinite(o)) and np.array_equal(r, o)
    # too large for the array: 2 nx (P+1) + 2 ns doubles above 4 MiB
    nx = 90000
    big = lib.Mesh(nx, 1, 1, 1000.0, True, np.ones(nx), np.zeros(nx))
    import torch
    z = torch.zeros(nx, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.SemError) as e:
        big.free_surface_rhs_noalloc(z, z, z, z, z.clone(), z.clone())
    assert e.value.code == lib.SEM_E_INVAL
