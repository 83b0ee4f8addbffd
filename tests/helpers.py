"""Shared helpers for the GPU parity tests: build the same tank in the library
and in the oracle, and map between their node numberings by coordinates."""
import numpy as np

from oracle import laplace as olap
from oracle import surface as osrf
from oracle.mesh import Mesh as OMesh


def node_permutation(lib_mesh, omesh):
    """perm[i] = oracle index of library node i (matched by coordinates)."""
    x, s = lib_mesh.node_coords()
    L = omesh.L
    kx = lambda v: np.round(np.mod(v, L) if omesh.periodic else v, 9)
    kl = {(a, b): i for i, (a, b) in enumerate(zip(kx(omesh.x), np.round(omesh.sigma, 9)))}
    perm = np.array([kl[(a, b)] for a, b in zip(kx(x), np.round(s, 9))])
    assert len(set(perm)) == len(perm)
    return perm


class Pair:
    """Library mesh (bound on the GPU) + oracle mesh + numbering map."""

    def __init__(self, nx, nz, P, L, periodic, h, hx, filter_ic=None, filter_sigma=1.0, Pf=None, g=9.81,
                 restart=30, variant=0, sigma_levels=None):
        from paper_1512_02548_amd import lib
        self.lib = lib
        self.m = lib.Mesh(nx, nz, P, L, periodic, h, hx, g=g, filter_ic=filter_ic, filter_sigma=filter_sigma,
                          overint=Pf, restart=restart, variant=variant, sigma_levels=sigma_levels)
        self.om = OMesh(nx, nz, P, L, periodic, sigma_levels=sigma_levels)
        self.perm = node_permutation(self.m, self.om)
        self.h = np.asarray(h, float)
        self.hx = np.asarray(hx, float)
        assert np.max(np.abs(self.m.surface_x() - self.om.xs_surf)) < 1e-12

    def to_lib(self, v_oracle):
        return np.asarray(v_oracle)[self.perm]

    def to_oracle(self, v_lib):
        out = np.empty(self.om.n)
        out[self.perm] = v_lib
        return out


def cuda(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def oracle_fields(pair, eta, phis):
    """The oracle's per-stage quantities for a surface state."""
    om = pair.om
    s1 = osrf.Surface1D(om)
    etax = s1.recover_dx(eta)
    phix = s1.recover_dx(phis)
    G, d = olap.coefficients(om, eta, etax, pair.h, pair.hx)
    A = olap.stiffness(om, G)
    Phi = olap.solve_direct(om, A, phis)
    return dict(s1=s1, etax=etax, phix=phix, G=G, d=d, A=A, Phi=Phi)
