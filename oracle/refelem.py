"""Reference-element operators (oracle; test infrastructure only).

Follows Sec. 3.1.4 ("Nodal prismatic Lagrange finite elements in two space
dimensions"): orthonormal Jacobi bases, the modal-nodal duality through the
generalised Vandermonde matrix V (eq. "duality"), Lagrange derivatives through
V^{-T} and V_r (eq. "derivative"), the quadrature-free mass matrix
M = (V V^T)^{-1} (eq. "massmatrix") and D_r = V_r V^{-1}.  The triangle node set
is Warburton's warp-and-blend construction, which the paper cites for simplex
nodes.  Sec. 3.3 supplies the fine-grid interpolation and mass matrix used for
over-integration and Sec. 3.4 the modal filter with the modified 1D basis.

Library primitives used as steps: scipy.special.eval_jacobi (classical Jacobi
polynomials), scipy.special.roots_jacobi (Gauss-Jacobi nodes) and numpy's
dense inverse.
"""
from math import factorial, gamma, sqrt

import numpy as np
from scipy.special import eval_jacobi, roots_jacobi

# Optimised blending parameter alpha of Warburton's warp-and-blend nodes,
# indexed by the polynomial order P (published table, Warburton 2006).
# Above P = 15 the construction uses 5/3.
ALPHA_OPT = (0.0, 0.0, 0.0, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832,
             1.3648, 1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258)


# ---------------------------------------------------------------- 1D pieces
def jacobi_norm(n, a, b):
    """L2 norm of the classical Jacobi polynomial P_n^(a,b) under the weight
    (1-x)^a (1+x)^b on [-1, 1]."""
    val = (2.0 ** (a + b + 1) / (2 * n + a + b + 1)
           * gamma(n + a + 1) * gamma(n + b + 1)
           / (gamma(n + a + b + 1) * factorial(n)))
    return sqrt(val)


def orthojacobi(x, n, a, b):
    """Orthonormal Jacobi polynomial ~P_n^(a,b)(x) (Sec. 3.1.4, orthogonality
    property below eq. "eq_basis")."""
    return eval_jacobi(n, a, b, np.asarray(x, dtype=float)) / jacobi_norm(n, a, b)


def orthojacobi_deriv(x, n, a, b):
    """d/dx of ~P_n^(a,b): the classical identity
    d/dx P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1)."""
    x = np.asarray(x, dtype=float)
    if n == 0:
        return np.zeros_like(x)
    return (0.5 * (n + a + b + 1) * eval_jacobi(n - 1, a + 1, b + 1, x)
            / jacobi_norm(n, a, b))


def gll_nodes(P):
    """Gauss-Lobatto-Legendre nodes on [-1, 1]: the end points and the roots of
    P_{P-1}^(1,1) (the zeros of the derivative of the Legendre polynomial)."""
    if P < 1:
        raise ValueError("order must be >= 1")
    if P == 1:
        return np.array([-1.0, 1.0])
    inner = np.sort(roots_jacobi(P - 1, 1.0, 1.0)[0])
    return np.concatenate(([-1.0], inner, [1.0]))


def vandermonde1d(P, r):
    """V_ij = ~P_j(r_i), j = 0..P (orthonormal Legendre)."""
    r = np.asarray(r, dtype=float)
    return np.stack([orthojacobi(r, j, 0, 0) for j in range(P + 1)], axis=1)


def grad_vandermonde1d(P, r):
    r = np.asarray(r, dtype=float)
    return np.stack([orthojacobi_deriv(r, j, 0, 0) for j in range(P + 1)], axis=1)


class Ref1D:
    """1D GLL element of order P: nodes r, V, D = V_r V^{-1}, M = (V V^T)^{-1}."""

    def __init__(self, P):
        self.P = P
        self.r = gll_nodes(P)
        self.V = vandermonde1d(P, self.r)
        self.Vinv = np.linalg.inv(self.V)
        self.D = grad_vandermonde1d(P, self.r) @ self.Vinv
        self.M = np.linalg.inv(self.V @ self.V.T)

    def interp_matrix(self, rout):
        """Evaluate the degree-P nodal interpolant at points rout:
        I = V(rout) V^{-1} (modal-nodal duality)."""
        return vandermonde1d(self.P, rout) @ self.Vinv


def fine_grid(P, Pf):
    """Over-integration operators of Sec. 3.3: the interpolation I_H^h from the
    GLL(P) nodes to the GLL(Pf) nodes and the fine mass matrix M_h."""
    coarse, fine = Ref1D(P), Ref1D(Pf)
    return coarse.interp_matrix(fine.r), fine.M


def modified_basis(P, r):
    """The boundary/bubble basis of Sec. 3.4: phi_0 = (1-r)/2, phi_1 = (1+r)/2,
    phi_{n+1} = (1-r)(1+r)/4 * P_{n-1}^(1,1)(r), n = 1..P-1."""
    r = np.asarray(r, dtype=float)
    cols = [0.5 * (1 - r), 0.5 * (1 + r)]
    for n in range(1, P):
        cols.append(0.25 * (1 - r) * (1 + r) * eval_jacobi(n - 1, 1.0, 1.0, r))
    return np.stack(cols, axis=1)


def filter_matrix(P, ic, sigma_f):
    """F = V^ S V^{-1} (Sec. 3.4) with V^_ij = phi_j(r_i) at the GLL nodes and
    S = diag(sigma_i): sigma_i = 1 for modes i < ic and sigma_f for ic <= i <= P.

    Reading of the printed filter formula: with s = 0 every mode i >= ic is
    scaled by the same factor exp(-alpha); the library takes (ic, sigma_f)
    directly.  ic < 2 would touch the vertex modes and break C0 continuity,
    so it is rejected.
    """
    if ic < 2:
        raise ValueError("filter cut-off must leave the two vertex modes alone (ic >= 2)")
    r = gll_nodes(P)
    Vh = modified_basis(P, r)
    s = np.array([1.0 if i < ic else sigma_f for i in range(P + 1)])
    return Vh @ np.diag(s) @ np.linalg.inv(Vh)


# ---------------------------------------------------------------- triangle
def _equispaced_interp(P, values, t):
    """Evaluate at t the degree-P polynomial through (t_m, values_m) with
    t_m = -1 + 2m/P (plain Lagrange products)."""
    tm = np.linspace(-1.0, 1.0, P + 1)
    out = np.zeros_like(t)
    for m in range(P + 1):
        lm = np.ones_like(t)
        for q in range(P + 1):
            if q != m:
                lm *= (t - tm[q]) / (tm[m] - tm[q])
        out += values[m] * lm
    return out


def warp_blend_nodes(P, alpha=None):
    """Warburton's warp-and-blend nodes on the reference triangle
    {(-1,-1), (1,-1), (-1,1)} in (r, s) coordinates.

    Construction (from the mathematics): start from the equispaced barycentric
    lattice on an equilateral triangle; for every edge, displace points along
    the edge direction by the 1D warp w(t) = [degree-P interpolant through the
    equispaced nodes of (GLL - equispaced)](t) divided by (1 - t^2), where t is
    the difference of the two edge barycentric coordinates; blend it into the
    interior with 4*lam_a*lam_b (the two edge vertices) times
    (1 + (alpha*lam_c)^2) (the opposite vertex).  On an edge the blend equals
    1 - t^2, so edge nodes land exactly on the GLL points.

    Node order: rows of constant s from s = -1 upward, r increasing in a row.
    alpha: blending parameter; None takes the published optimum for P.
    """
    if P == 0:
        return np.array([-1.0 / 3.0]), np.array([-1.0 / 3.0])
    if alpha is None:
        alpha = ALPHA_OPT[P] if P < len(ALPHA_OPT) else 5.0 / 3.0
    lamA, lamB, lamC = [], [], []
    for j in range(P + 1):
        for i in range(P + 1 - j):
            lamB.append(i / P)
            lamC.append(j / P)
            lamA.append(1.0 - i / P - j / P)
    lamA, lamB, lamC = (np.array(v) for v in (lamA, lamB, lamC))
    # equilateral vertices
    A = np.array([-1.0, -1.0 / sqrt(3.0)])
    B = np.array([1.0, -1.0 / sqrt(3.0)])
    C = np.array([0.0, 2.0 / sqrt(3.0)])
    X = lamA * A[0] + lamB * B[0] + lamC * C[0]
    Y = lamA * A[1] + lamB * B[1] + lamC * C[1]
    disp = gll_nodes(P) - np.linspace(-1.0, 1.0, P + 1)
    lam = {"A": lamA, "B": lamB, "C": lamC}
    vert = {"A": A, "B": B, "C": C}
    for p0, p1, q in (("A", "B", "C"), ("B", "C", "A"), ("C", "A", "B")):
        t = lam[p1] - lam[p0]
        w = _equispaced_interp(P, disp, t)
        inner = np.abs(t) < 1.0 - 1e-10
        factor = np.where(inner, w / np.where(inner, 1.0 - t * t, 1.0), 0.0)
        mag = 4.0 * lam[p0] * lam[p1] * factor * (1.0 + (alpha * lam[q]) ** 2)
        e = (vert[p1] - vert[p0]) / np.linalg.norm(vert[p1] - vert[p0])
        X = X + mag * e[0]
        Y = Y + mag * e[1]
    # back to barycentric coordinates of the warped points, then to (r, s)
    lc = (sqrt(3.0) * Y + 1.0) / 3.0
    lb = (X + 1.0 - lc) / 2.0
    return 2.0 * lb - 1.0, 2.0 * lc - 1.0


def rs_to_ab(r, s):
    """Collapsed coordinates of the simplex: a = 2(1+r)/(1-s) - 1, b = s
    (a := -1 at the top vertex s = 1)."""
    r = np.asarray(r, dtype=float)
    s = np.asarray(s, dtype=float)
    top = np.isclose(s, 1.0, atol=1e-14)
    a = np.where(top, -1.0, 2.0 * (1.0 + r) / np.where(top, 1.0, 1.0 - s) - 1.0)
    return a, s


def simplex_modes(P):
    return [(i, j) for i in range(P + 1) for j in range(P + 1 - i)]


def simplex_basis(r, s, i, j):
    """Orthonormal basis on the reference triangle (area 2):
    psi_ij = sqrt(2) ~P_i(a) ~P_j^(2i+1,0)(b) (1-b)^i."""
    a, b = rs_to_ab(r, s)
    return sqrt(2.0) * orthojacobi(a, i, 0, 0) * orthojacobi(b, j, 2 * i + 1, 0) * (1 - b) ** i


def simplex_grad(r, s, i, j):
    """(d/dr, d/ds) of psi_ij by the chain rule through (a, b):
    da/dr = 2/(1-b), da/ds = (1+a)/(1-b), written so that every negative power
    of (1-b) cancels against the (1-b)^i factor."""
    a, b = rs_to_ab(r, s)
    f, df = orthojacobi(a, i, 0, 0), orthojacobi_deriv(a, i, 0, 0)
    g, dg = orthojacobi(b, j, 2 * i + 1, 0), orthojacobi_deriv(b, j, 2 * i + 1, 0)
    omb = 1.0 - b
    pim1 = omb ** (i - 1) if i >= 1 else np.zeros_like(b)
    dr = sqrt(2.0) * df * g * 2.0 * pim1
    ds = sqrt(2.0) * (df * (1 + a) * g * pim1 + f * dg * omb ** i - i * f * g * pim1)
    return dr, ds


class RefTri:
    """Order-P nodal triangle: nodes (r, s), V, V_r, V_s, D_r, D_s, M."""

    def __init__(self, P):
        self.P = P
        self.Np = (P + 1) * (P + 2) // 2
        self.r, self.s = warp_blend_nodes(P)
        modes = simplex_modes(P)
        self.V = np.stack([simplex_basis(self.r, self.s, i, j) for i, j in modes], axis=1)
        grads = [simplex_grad(self.r, self.s, i, j) for i, j in modes]
        self.Vr = np.stack([g[0] for g in grads], axis=1)
        self.Vs = np.stack([g[1] for g in grads], axis=1)
        self.Vinv = np.linalg.inv(self.V)
        self.Dr = self.Vr @ self.Vinv
        self.Ds = self.Vs @ self.Vinv
        self.M = np.linalg.inv(self.V @ self.V.T)
