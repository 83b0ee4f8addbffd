"""Free-surface operators (oracle; test infrastructure).

Sec. 3.1.3 (gradient recovery): a C0 derivative is recovered by the global
L2 projection M u = S_x phi with S_x = int dN_j/dx N_i.  On the 1D surface
mesh this gives eta_x and phi~_x; per element M'^e = J_e M_1 and
S_x^e = J_e M_1 (2/dx) D_1 = M_1 D_1.

The vertical surface velocity comes from M w = S_z Phi (eqs. "velocpot",
"velocpot2") with S_z = int sigma_z dN_j/dsigma N_i, evaluated
quadrature-free (Sec. 3.2) with the nodal values of sigma_z = 1/d:
S_z^k = |J^k| M diag(1/d) D_sigma^k, D_sigma^k = r_sigma D_r + s_sigma D_s.
Both integrals are taken over the computational (x, sigma) domain, so the 2D
mass matrix sum_k |J^k| M is constant in time; w~ is w on S^FS.  The
horizontal velocity in the volume comes from the same projection of
d phi/dx = d_x Phi + sigma_x d_sigma Phi (eq. representationU with the
chain rule of the sigma-map).

Sec. 3.1.1 gives the weak free-surface equations (eq. "FSproblem"),

    int eta_t v   = int [-eta_x phi~_x + w~ (1 + eta_x^2)] v,
    int phi~_t v  = int [-g eta - 1/2 (phi~_x^2 - w~^2 (1 + eta_x^2))] v,

with the sign of the w~^2 term taken from the PDE (eq. "FSphi"); the
semi-discrete form printed in Sec. 3.1.1 carries the opposite sign, which
the energy pin in the tests rules out.  Sec. 3.3 over-integrates the right
sides: the nodal fields are interpolated to the GLL(Pf) nodes, the integrands
are formed pointwise there and projected with J_e I^T M_h.  Pf = P means no
over-integration.

Sec. 3.4: the filter F = V^ S V^{-1} acts element by element on eta and phi~.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .refelem import Ref1D, fine_grid, filter_matrix


class Surface1D:
    """Assembled 1D operators of the surface mesh (periodic or walls)."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.P = mesh.P
        self.ref1 = mesh.ref1
        self.idx = mesh.surface_elements()              # (Nx, P+1)
        self.Je = 0.5 * mesh.dx
        ns = mesh.ns
        rows = np.repeat(self.idx, self.P + 1, axis=1).ravel()
        cols = np.tile(self.idx, (1, self.P + 1)).ravel()
        Me = self.Je * self.ref1.M
        Se = self.ref1.M @ self.ref1.D
        nel = self.idx.shape[0]
        self.Mp = sp.csr_matrix((np.tile(Me.ravel(), nel), (rows, cols)), shape=(ns, ns))
        self.Sx = sp.csr_matrix((np.tile(Se.ravel(), nel), (rows, cols)), shape=(ns, ns))
        self._lu = spla.splu(self.Mp.tocsc())

    def solve_mass(self, rhs):
        return self._lu.solve(np.asarray(rhs, dtype=float))

    def recover_dx(self, f):
        """C0 derivative by the global L2 projection M' f_x = S_x f."""
        return self.solve_mass(self.Sx @ np.asarray(f, dtype=float))

    def assemble_vec(self, local):
        out = np.zeros(self.mesh.ns)
        np.add.at(out, self.idx, local)
        return out

    def fs_rhs(self, eta, etax, phix, w, g, Pf):
        """Over-integrated Galerkin right-hand sides, then M' solves:
        returns (eta_t, phi~_t)."""
        I, Mf = fine_grid(self.P, Pf)
        loc_eta, loc_phi = [], []
        for e in range(self.idx.shape[0]):
            ix = self.idx[e]
            et, ex, px, ww = (I @ np.asarray(v)[ix] for v in (eta, etax, phix, w))
            f_eta = -ex * px + ww * (1.0 + ex * ex)
            f_phi = -g * et - 0.5 * (px * px - ww * ww * (1.0 + ex * ex))
            loc_eta.append(self.Je * I.T @ Mf @ f_eta)
            loc_phi.append(self.Je * I.T @ Mf @ f_phi)
        return (self.solve_mass(self.assemble_vec(np.array(loc_eta))),
                self.solve_mass(self.assemble_vec(np.array(loc_phi))))

    def apply_filter(self, f, ic, sigma_f):
        """Per-element modal filter.  The filter leaves the element end values
        unchanged (vertex modes untouched), so shared nodes stay single-valued."""
        F = filter_matrix(self.P, ic, sigma_f)
        f = np.asarray(f, dtype=float)
        out = f.copy()
        for e in range(self.idx.shape[0]):
            out[self.idx[e]] = F @ f[self.idx[e]]
        return out


def mass2d(mesh):
    """Constant 2D mass matrix of the computational domain, sum_k |J^k| M."""
    from .laplace import assemble
    return assemble(mesh, [mesh.J[k] * mesh.ref.M for k in range(mesh.E)])


def sz_times(mesh, Phi, d):
    """S_z Phi assembled: sum_k R_k^T |J^k| M diag(1/d) D_sigma^k Phi_k."""
    ref = mesh.ref
    out = np.zeros(mesh.n)
    for k in range(mesh.E):
        Dsig = mesh.Lam[k, 0, 1] * ref.Dr + mesh.Lam[k, 1, 1] * ref.Ds
        loc = mesh.J[k] * ref.M @ ((Dsig @ Phi[mesh.EToN[k]]) / d[k])
        np.add.at(out, mesh.EToN[k], loc)
    return out


def su_times(mesh, Phi, sigx):
    """S_u Phi assembled: sum_k R_k^T |J^k| M (D_x^k + diag(sigma_x) D_sigma^k) Phi_k,
    the quadrature-free form of int (d_x Phi + sigma_x d_sigma Phi) N_i over
    the computational domain (chain rule of the sigma-map, Sec. 2; the
    horizontal velocity of eq. representationU)."""
    ref = mesh.ref
    out = np.zeros(mesh.n)
    for k in range(mesh.E):
        Dx = mesh.Lam[k, 0, 0] * ref.Dr + mesh.Lam[k, 1, 0] * ref.Ds
        Dsig = mesh.Lam[k, 0, 1] * ref.Dr + mesh.Lam[k, 1, 1] * ref.Ds
        Pk = Phi[mesh.EToN[k]]
        loc = mesh.J[k] * ref.M @ (Dx @ Pk + sigx[k] * (Dsig @ Pk))
        np.add.at(out, mesh.EToN[k], loc)
    return out


def recover_u(mesh, Phi, sigx, Mc=None):
    """Horizontal velocity u = d phi/dx on all nodes from the global L2
    projection M u = S_u Phi (Sec. 3.1.3, eq. representationU)."""
    Mc = mass2d(mesh) if Mc is None else Mc
    return spla.spsolve(Mc.tocsc(), su_times(mesh, Phi, sigx))


def recover_w(mesh, Phi, d, Mc=None):
    """Vertical velocity w on all nodes from M w = S_z Phi; w~ = w[surf]."""
    Mc = mass2d(mesh) if Mc is None else Mc
    w = spla.spsolve(Mc.tocsc(), sz_times(mesh, Phi, d))
    return w
