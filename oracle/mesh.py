"""Structured triangular mesh of the sigma-domain (oracle; test infrastructure).

The computational domain of Sec. 2 is the fixed box [0, L] x [0, 1] in (x, sigma).
It is split into Nx columns of uniform width and Nz layers (uniform in sigma
unless levels are given), and every quadrilateral is cut along its diagonal
from (x_c, s_j) to (x_{c+1}, s_{j+1}) into two order-P triangles carrying the
reference nodes of RefTri (Sec. 3.1.4).  Global C0 nodes are identified by their
coordinates, with x-periodicity when requested.  The free-surface index set
S^FS of Sec. 3.1.3 is the set of nodes with sigma = 1, ordered by x.
"""
import numpy as np

from .refelem import Ref1D, RefTri


class Mesh:
    def __init__(self, nx, nz, P, length, periodic=True, sigma_levels=None):
        self.nx, self.nz, self.P = int(nx), int(nz), int(P)
        self.L = float(length)
        self.periodic = bool(periodic)
        self.ref = RefTri(self.P)
        self.ref1 = Ref1D(self.P)
        self.dx = self.L / self.nx
        xs = np.linspace(0.0, self.L, self.nx + 1)
        if sigma_levels is None:
            ss = np.linspace(0.0, 1.0, self.nz + 1)
        else:
            ss = np.asarray(sigma_levels, dtype=float)
            assert ss.shape == (self.nz + 1,) and ss[0] == 0.0 and ss[-1] == 1.0
        self.xs, self.ss = xs, ss
        r, s = self.ref.r, self.ref.s

        ecol, elay, etyp, ex, esig, lam, jac = [], [], [], [], [], [], []
        for c in range(self.nx):
            for j in range(self.nz):
                for t in (0, 1):
                    if t == 0:   # lower triangle: A=(x_c,s_j) B=(x_c+1,s_j) C=(x_c+1,s_j+1)
                        A, B, C = (xs[c], ss[j]), (xs[c + 1], ss[j]), (xs[c + 1], ss[j + 1])
                    else:        # upper triangle: A=(x_c,s_j) B=(x_c+1,s_j+1) C=(x_c,s_j+1)
                        A, B, C = (xs[c], ss[j]), (xs[c + 1], ss[j + 1]), (xs[c], ss[j + 1])
                    A, B, C = np.array(A), np.array(B), np.array(C)
                    # affine map of Sec. 3.1.2: (x, sigma) = -(r+s)/2 A + (1+r)/2 B + (1+s)/2 C
                    X = -0.5 * (r + s) * A[0] + 0.5 * (1 + r) * B[0] + 0.5 * (1 + s) * C[0]
                    S = -0.5 * (r + s) * A[1] + 0.5 * (1 + r) * B[1] + 0.5 * (1 + s) * C[1]
                    dxdrs = np.column_stack([(B - A) / 2.0, (C - A) / 2.0])  # d(x,sig)/d(r,s)
                    ecol.append(c)
                    elay.append(j)
                    etyp.append(t)
                    ex.append(X)
                    esig.append(S)
                    lam.append(np.linalg.inv(dxdrs))          # Lambda = d(r,s)/d(x,sig)
                    jac.append(np.linalg.det(dxdrs))          # |J^k|
        self.ecol = np.array(ecol)
        self.elay = np.array(elay)
        self.etyp = np.array(etyp)
        self.ex = np.array(ex)            # (E, Np) unwrapped x of element nodes
        self.esig = np.array(esig)        # (E, Np)
        self.Lam = np.array(lam)          # (E, 2, 2)
        self.J = np.array(jac)            # (E,)
        self.E = len(ecol)
        self.Np = self.ref.Np
        self._number_nodes()

    def _number_nodes(self):
        """Identify coincident element nodes by coordinates (x wrapped when
        periodic) and number them in order of first appearance."""
        x = self.ex.ravel().copy()
        sg = self.esig.ravel().copy()
        if self.periodic:
            x = np.mod(x, self.L)
            x[np.abs(x - self.L) < 1e-12 * self.L] = 0.0
        h = 1e-7 * min(self.dx, np.min(np.diff(self.ss))) / self.P
        kx = np.floor(x / h + 0.5).astype(np.int64)
        ks = np.floor(sg / h + 0.5).astype(np.int64)
        keys = kx * (1 << 31) + ks
        _, first, inv = np.unique(keys, return_index=True, return_inverse=True)
        # renumber by first appearance
        order = np.argsort(first)
        rank = np.empty_like(order)
        rank[order] = np.arange(len(order))
        gid = rank[inv]
        n = len(first)
        cx = np.zeros(n)
        cs = np.zeros(n)
        cx[gid] = x
        cs[gid] = sg
        # every point merged into a node must sit on it, and distinct nodes
        # must be far apart (guards the rounding-based identification)
        if np.max(np.abs(cx[gid] - x)) > 1e-9 * self.L or np.max(np.abs(cs[gid] - sg)) > 1e-9:
            raise RuntimeError("node identification failed")
        ordr = np.lexsort((cs, cx))
        gap = np.hypot(np.diff(cx[ordr]), np.diff(cs[ordr]))
        if gap.size and gap.min() < 1e3 * h:
            raise RuntimeError("two distinct nodes are too close")
        self.n = n
        self.x, self.sigma = cx, cs
        self.EToN = gid.reshape(self.E, self.Np)
        surf = np.where(np.abs(cs - 1.0) < 1e-12)[0]
        self.surf = surf[np.argsort(cx[surf])]
        self.ns = len(self.surf)
        self.is_surf = np.zeros(n, dtype=bool)
        self.is_surf[self.surf] = True
        self.free = np.where(~self.is_surf)[0]
        self.mult = np.bincount(self.EToN.ravel(), minlength=n)
        # the surface nodes form the 1D mesh: element c holds nodes c*P + m
        self.xs_surf = cx[self.surf]
        expect = (self.xs[:-1, None] + 0.5 * self.dx * (1 + self.ref1.r[None, :])).ravel()
        expect = expect.reshape(self.nx, self.P + 1)[:, :self.P].ravel()
        if not self.periodic:
            expect = np.concatenate([expect, [self.L]])
        if self.ns != len(expect) or np.max(np.abs(self.xs_surf - expect)) > 1e-10 * self.L:
            raise RuntimeError("surface nodes are not the GLL points of the columns")

    # ------------------------------------------------------------ helpers
    def surface_elements(self):
        """(Nx, P+1) indices into the x-ordered surface arrays for each 1D
        surface element (column), periodic wrap included."""
        c = np.arange(self.nx)[:, None]
        m = np.arange(self.P + 1)[None, :]
        idx = c * self.P + m
        if self.periodic:
            idx = idx % self.ns
        return idx

    def column_interp(self, fs):
        """Value at every element node of the column's degree-P interpolant of
        x-ordered surface data fs (the nodal positions of Sec. 2's metric
        terms).  Returns (E, Np)."""
        idx = self.surface_elements()
        rloc = 2.0 * (self.ex - self.xs[self.ecol][:, None]) / self.dx - 1.0
        out = np.empty((self.E, self.Np))
        for k in range(self.E):
            I = self.ref1.interp_matrix(rloc[k])
            out[k] = I @ np.asarray(fs)[idx[self.ecol[k]]]
        return out

    def node_z(self, eta_nodes, h_nodes):
        """Physical z of element nodes: z = sigma d - h (inverse of eq. sigtrans)."""
        return self.esig * (eta_nodes + h_nodes) - h_nodes
