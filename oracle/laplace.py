"""sigma-transformed Laplace problem (oracle; test infrastructure).

Sec. 2 (Governing equations): with d = eta + h the sigma-map has Jacobian
[[1, 0], [sigma_x, sigma_z]] with sigma_x = ((1-sigma) h_x - sigma eta_x)/d and
sigma_z = 1/d, and the transformed problem is div^c(K grad^c Phi) = 0 with
K = J J^T / det J.  Written out,

    K = [[d, q], [q, (1 + q^2)/d]],   q = (1 - sigma) h_x - sigma eta_x,

which reduces to the printed matrix when h_x = 0; det K = 1.

Sec. 3.1.2: L_ij = -sum_k int |J^k| (K grad N_j) . grad N_i over the reference
element.  Sec. 3.2 (eq. "localintegrals") evaluates every element integral
quadrature-free through the nodal mass matrix: the flux f = K grad Phi is
represented by its nodal interpolant and the test-function derivative is
integrated exactly against it, which gives

    A^k = sum_{a,b in {r,s}} D_a^T M diag(G_ab) D_b,   G = |J^k| Lam K Lam^T

at the element nodes (Lam = d(r,s)/d(x,sigma)).  A^k is symmetric whenever G
is constant on the element (still water over a flat bed), which is the case
the symmetry remark of Sec. 3.1.2 covers; with a moving surface it is not, and
the paper's own solver (sparse LU, Sec. 3.1.2) does not need symmetry.  The
symmetric part (A^k + A^k^T)/2 was tried as an alternative and rejected: it
interpolates G times the derivative of the discrete test function, which is
not smooth, and its error stops decreasing with P (the manufactured-solution
pin in the tests shows both behaviours); it is kept here as
``element_stiffness_sym`` only for that comparison.

The Dirichlet condition Phi = phi~ on S^FS (eq. "eq:FSeqs") is imposed by
moving the surface columns to the right-hand side:
A_FF Phi_F = -A_FS phi~.  The oracle solves with sparse LU (scipy splu), the
paper's solver class; a reference right-preconditioned GMRES with a plain
element-block-Jacobi preconditioner is provided for Krylov cross-checks.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class DomainError(ValueError):
    """The sigma-map is singular: some water column height d = eta + h <= 0."""


def coefficients(mesh, eta_s, etax_s, h_s, hx_s):
    """Geometric factors at every element node.

    Returns G (E, Np, 3) = (G_rr, G_rs, G_ss) and d (E, Np).  eta, eta_x, h
    and h_x at a node are the values of the column's degree-P surface
    interpolants at the node's x (the metric terms are evaluated from the
    known surface and bottom positions, Sec. 2)."""
    eta = mesh.column_interp(eta_s)
    etax = mesh.column_interp(etax_s)
    h = mesh.column_interp(h_s)
    hx = mesh.column_interp(hx_s)
    d = eta + h
    if np.any(d <= 0.0):
        raise DomainError("water column height d = eta + h must be positive")
    sig = mesh.esig
    q = (1.0 - sig) * hx - sig * etax
    K = np.empty(d.shape + (2, 2))
    K[..., 0, 0] = d
    K[..., 0, 1] = q
    K[..., 1, 0] = q
    K[..., 1, 1] = (1.0 + q * q) / d
    G = np.einsum("kac,kicd,kbd->kiab", mesh.Lam, K, mesh.Lam) * mesh.J[:, None, None, None]
    return np.stack([G[..., 0, 0], G[..., 0, 1], G[..., 1, 1]], axis=-1), d


def sigma_x(mesh, eta_s, etax_s, h_s, hx_s):
    """d(sigma)/dx of the sigma-map at every element node (Sec. 2, the
    Jacobian's off-diagonal entry): ((1 - sigma) h_x - sigma eta_x) / d, with
    the column interpolants of the surface data.  Returns (E, Np)."""
    eta = mesh.column_interp(eta_s)
    etax = mesh.column_interp(etax_s)
    h = mesh.column_interp(h_s)
    hx = mesh.column_interp(hx_s)
    sig = mesh.esig
    return ((1.0 - sig) * hx - sig * etax) / (eta + h)


def element_stiffness(ref, Gk):
    """A^k = sum_ab D_a^T M diag(G_ab) D_b (quadrature-free, Sec. 3.2)."""
    D = (ref.Dr, ref.Ds)
    Gab = ((Gk[:, 0], Gk[:, 1]), (Gk[:, 1], Gk[:, 2]))
    A = np.zeros((ref.Np, ref.Np))
    for a in range(2):
        for b in range(2):
            A += D[a].T @ ref.M @ np.diag(Gab[a][b]) @ D[b]
    return A


def element_stiffness_sym(ref, Gk):
    """Symmetric part of A^k (rejected alternative, see the module docstring)."""
    A = element_stiffness(ref, Gk)
    return 0.5 * (A + A.T)


def assemble(mesh, mats):
    """Global matrix sum_k R_k^T A^k R_k (domain decomposition, Sec. 3.1.2)."""
    rows = np.repeat(mesh.EToN, mesh.Np, axis=1).ravel()
    cols = np.tile(mesh.EToN, (1, mesh.Np)).ravel()
    return sp.csr_matrix((np.asarray(mats).ravel(), (rows, cols)), shape=(mesh.n, mesh.n))


def stiffness(mesh, G, sym=False):
    f = element_stiffness_sym if sym else element_stiffness
    return assemble(mesh, [f(mesh.ref, G[k]) for k in range(mesh.E)])


def dirichlet_split(mesh, A, phi_s):
    """A_FF and the lifted right-hand side b = -A_FS phi~."""
    F, S = mesh.free, mesh.surf
    A = A.tocsr()
    AFF = A[F][:, F].tocsc()
    b = -(A[F][:, S] @ np.asarray(phi_s))
    return AFF, b


def solve_direct(mesh, A, phi_s):
    """Phi on all nodes: the free part from A_FF Phi_F = -A_FS phi~ by sparse LU
    (dense Cholesky-free LU for tiny systems), the surface part = phi~."""
    AFF, b = dirichlet_split(mesh, A, phi_s)
    if AFF.shape[0] <= 1500:
        xF = np.linalg.solve(AFF.toarray(), b)
    else:
        xF = spla.splu(AFF).solve(b)
    Phi = np.empty(mesh.n)
    Phi[mesh.free] = xF
    Phi[mesh.surf] = phi_s
    return Phi


def laplace_solve(mesh, eta_s, etax_s, phi_s, h_s, hx_s):
    """The per-stage Laplace problem: returns Phi (n,), G and d at the nodes."""
    G, d = coefficients(mesh, eta_s, etax_s, h_s, hx_s)
    A = stiffness(mesh, G)
    return solve_direct(mesh, A, phi_s), G, d


# ------------------------------------------------------- reference Krylov
def still_water_G(mesh, h0):
    """Geometric factors of still water (eta = 0) over a flat bed of depth h0:
    K = diag(h0, 1/h0)."""
    K = np.array([[h0, 0.0], [0.0, 1.0 / h0]])
    G = np.einsum("kac,cd,kbd->kab", mesh.Lam, K, mesh.Lam) * mesh.J[:, None, None]
    Gn = np.stack([G[:, 0, 0], G[:, 0, 1], G[:, 1, 1]], axis=-1)
    return np.repeat(Gn[:, None, :], mesh.Np, axis=1)


def block_jacobi(mesh, A0, dirichlet=True):
    """Element-block Jacobi (additive Schwarz on element patches):
    B = sum_k R_k^T W_k C_k^{-1} W_k R_k, C_k = principal submatrix of the
    assembled A0 on element k's (free) nodes, W_k = diag(mult^{-1/2}).
    The paper leaves the preconditioner open; this is a plain reference
    choice for the Krylov cross-checks.
    Returns a function r -> z on full-length vectors (surface entries 0)."""
    A0 = A0.tocsr()
    w = 1.0 / np.sqrt(mesh.mult)
    blocks = []
    for k in range(mesh.E):
        nodes = mesh.EToN[k]
        keep = ~mesh.is_surf[nodes] if dirichlet else np.ones(mesh.Np, bool)
        idx = nodes[keep]
        C = A0[idx][:, idx].toarray()
        blocks.append((idx, np.linalg.inv(C), w[idx]))

    def apply(r):
        z = np.zeros(mesh.n)
        for idx, Ci, wk in blocks:
            z[idx] += wk * (Ci @ (wk * r[idx]))
        return z
    return apply


def pcg(apply_A, apply_B, b, x0, rtol, max_iter=100000):
    """Textbook preconditioned conjugate gradients; stops when the recursive
    residual satisfies ||r||_2 <= rtol ||b||_2.  Returns (x, iterations)."""
    x = x0.copy()
    r = b - apply_A(x)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), 0
    z = apply_B(r)
    p = z.copy()
    rz = r @ z
    for it in range(max_iter):
        if np.linalg.norm(r) <= rtol * nb:
            return x, it
        q = apply_A(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = apply_B(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter


def gmres(apply_A, apply_B, b, x0, rtol, restart=30, max_iter=100000):
    """Textbook restarted GMRES with right preconditioning (Arnoldi with
    modified Gram-Schmidt, Givens rotations).  Stops when the Arnoldi residual
    estimate satisfies ||r|| <= rtol ||b||.  Returns (x, iterations)."""
    x = x0.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), 0
    total = 0
    while total < max_iter:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * nb:
            return x, total
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j = 0
        while j < restart and total < max_iter:
            Z.append(apply_B(V[j]))
            w = apply_A(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] != 0.0 else w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j += 1
            total += 1
            if abs(g[j]) <= rtol * nb:
                break
        y = np.linalg.solve(np.triu(H[:j, :j]), g[:j])
        x = x + sum(y[i] * Z[i] for i in range(j))
        if abs(g[j]) <= rtol * nb:
            return x, total
    return x, total


def laplace_krylov(mesh, A, phi_s, h0, x0=None, rtol=1e-12, restart=30):
    """Reference GMRES on the Dirichlet-reduced system with the still-water
    element-block-Jacobi preconditioner; vectors are full length with zero
    surface entries.  Returns (Phi, iterations)."""
    A = A.tocsr()
    mask = (~mesh.is_surf).astype(float)
    lift = np.zeros(mesh.n)
    lift[mesh.surf] = phi_s
    b = -(A @ lift) * mask
    B = block_jacobi(mesh, stiffness(mesh, still_water_G(mesh, h0)))
    x0 = np.zeros(mesh.n) if x0 is None else np.asarray(x0, float) * mask
    x, it = gmres(lambda v: (A @ (v * mask)) * mask, B, b, x0, rtol, restart)
    return x * mask + lift, it
