"""Pins of the oracle's Laplace step, gradient recovery and free-surface
right-hand side (CPU): exact harmonic solutions, the linear dispersion
relation, invariants of K and of the assembled operator, brute-force checks."""
import numpy as np
import pytest

from oracle import exact
from oracle import laplace as lap
from oracle import surface as srf
from oracle.mesh import Mesh
from oracle.refelem import fine_grid, gll_nodes


def flat(m, h=1.0):
    return np.full(m.ns, h), np.zeros(m.ns)


def manufactured_error(P, amp, sym=False, nx=4, nz=2, k=1.0, h=1.0):
    """Max nodal error of Phi and w~ against the harmonic function
    cosh(k(z+h))/cosh(kh) sin(kx) on a deformed periodic surface."""
    L = 2 * np.pi / k
    m = Mesh(nx, nz, P, L, True)
    s1 = srf.Surface1D(m)
    xs = m.xs_surf
    eta = amp * np.cos(k * xs) + 0.3 * amp * np.sin(2 * k * xs)
    etax = s1.recover_dx(eta)
    phis = exact.harmonic_phi(xs, eta, k, h)
    G, d = lap.coefficients(m, eta, etax, *flat(m, h))
    Phi = lap.solve_direct(m, lap.stiffness(m, G, sym=sym), phis)
    en = m.column_interp(eta)
    z = m.node_z(en, np.full_like(en, h))
    ephi = np.max(np.abs(Phi[m.EToN] - exact.harmonic_phi(m.ex, z, k, h)))
    w = srf.recover_w(m, Phi, d)[m.surf]
    ew = np.max(np.abs(w - exact.harmonic_w(xs, eta, k, h)))
    return ephi, ew


def test_manufactured_solution_converges_exponentially():
    """Phi_h -> Phi_ex and w~ -> dPhi_ex/dz exponentially in P on a deformed
    surface (exercises the whole K tensor incl. q = -sigma eta_x)."""
    Ps = [2, 4, 6, 8]
    errs = [manufactured_error(P, 0.1) for P in Ps]
    ephi = [e[0] for e in errs]
    ew = [e[1] for e in errs]
    for a, b in zip(ephi, ephi[1:]):
        assert b < a / 8.0
    assert ephi[-1] < 2e-6 and ew[-1] < 1e-4
    assert ew[-1] < ew[1] / 50


def test_symmetrised_operator_stalls():
    """The symmetric part of the quadrature-free operator is inconsistent:
    its error stops improving with P, proportionally to the wave amplitude,
    while the paper-literal operator keeps converging."""
    lit = manufactured_error(8, 0.1)[0]
    sym8 = manufactured_error(8, 0.1, sym=True)[0]
    sym6 = manufactured_error(6, 0.1, sym=True)[0]
    assert sym8 > 100 * lit
    assert sym8 > 0.3 * sym6


@pytest.mark.parametrize("kh", [0.5, 1.0, 2.0])
def test_discrete_dtn_matches_dispersion(kh):
    """eta = 0, phi~ = sin kx: w~/phi~ -> k tanh(kh) (linear dispersion
    relation omega^2 = g k tanh kh of Sec. 4.2), exponentially in P."""
    k = 1.0
    errs = []
    for P in (2, 4, 6, 8):
        m = Mesh(4, 2, P, 2 * np.pi / k, True)
        xs = m.xs_surf
        eta = np.zeros(m.ns)
        phis = np.sin(k * xs)
        G, d = lap.coefficients(m, eta, eta, *flat(m, kh))
        Phi = lap.solve_direct(m, lap.stiffness(m, G), phis)
        w = srf.recover_w(m, Phi, d)[m.surf]
        mask = np.abs(phis) > 0.5
        ratio = w[mask] / phis[mask]
        errs.append(np.max(np.abs(ratio - k * np.tanh(k * kh))))
    assert errs[3] < errs[2] / 10 < errs[1] / 100 < errs[0] / 1000
    assert errs[3] < 1e-6


def test_K_invariants_and_operator_structure():
    m = Mesh(6, 3, 4, 5.0, False)
    rng = np.random.default_rng(1)
    xs = m.xs_surf
    eta = 0.2 * np.sin(2 * np.pi * xs / 5.0) + 0.05 * rng.standard_normal() * np.cos(xs)
    h = 1.0 - 0.3 * np.exp(-(xs - 2.5) ** 2)
    hx = 0.6 * (xs - 2.5) * np.exp(-(xs - 2.5) ** 2)
    s1 = srf.Surface1D(m)
    G, d = lap.coefficients(m, eta, s1.recover_dx(eta), h, hx)
    # det G = |J|^2 det(Lam)^2 det K = 1 at every node
    detG = G[..., 0] * G[..., 2] - G[..., 1] ** 2
    assert np.max(np.abs(detG - 1.0)) < 1e-12
    A = lap.stiffness(m, G)
    # constants are annihilated (row sums vanish before the Dirichlet split)
    assert np.max(np.abs(A @ np.ones(m.n))) < 1e-11 * abs(A).max()
    # still water over a flat bed: the operator is symmetric
    A0 = lap.stiffness(m, lap.still_water_G(m, 1.0))
    assert abs(A0 - A0.T).max() < 1e-13 * abs(A0).max()
    # the moving-surface operator is not, but its symmetric part on the free
    # nodes is positive definite
    AFF, _ = lap.dirichlet_split(m, A, np.zeros(m.ns))
    S = 0.5 * (AFF + AFF.T).toarray()
    assert np.linalg.eigvalsh(S).min() > 0


def test_krylov_matches_direct():
    """Reference GMRES with the element-block-Jacobi preconditioner reaches the
    sparse-LU solution (brute force on a tiny system)."""
    m = Mesh(8, 2, 4, 2 * np.pi, True)
    s1 = srf.Surface1D(m)
    xs = m.xs_surf
    eta = 0.15 * np.cos(xs)
    phis = exact.harmonic_phi(xs, eta, 1.0, 1.0)
    G, d = lap.coefficients(m, eta, s1.recover_dx(eta), *flat(m))
    A = lap.stiffness(m, G)
    Phi = lap.solve_direct(m, A, phis)
    Phi2, it = lap.laplace_krylov(m, A, phis, 1.0, rtol=1e-13)
    assert np.max(np.abs(Phi2 - Phi)) < 1e-11 * np.max(np.abs(Phi))
    assert 0 < it < 200
    # dense solve of the same system agrees with splu
    AFF, b = lap.dirichlet_split(m, A, phis)
    assert np.max(np.abs(np.linalg.solve(AFF.toarray(), b) - Phi[m.free])) < 1e-12
    # mass-matrix PCG of the w projection agrees with the direct solve
    Mc = srf.mass2d(m)
    rhs = srf.sz_times(m, Phi, d)
    Bm = lap.block_jacobi(m, Mc, dirichlet=False)
    wp, itm = lap.pcg(lambda v: Mc @ v, Bm, rhs, np.zeros(m.n), 1e-14)
    assert np.max(np.abs(wp - srf.recover_w(m, Phi, d, Mc))) < 1e-12
    assert itm < 60


def test_gradient_recovery():
    # walls: exact for global polynomials of degree <= P
    m = Mesh(5, 1, 4, 3.0, False)
    s1 = srf.Surface1D(m)
    x = m.xs_surf
    f = 0.3 * x ** 4 - x ** 3 + 2 * x - 1
    assert np.max(np.abs(s1.recover_dx(f) - (1.2 * x ** 3 - 3 * x ** 2 + 2))) < 1e-11
    # periodic: spectral for sin kx
    errs = []
    for P in (2, 4, 6, 8):
        m = Mesh(4, 1, P, 2 * np.pi, True)
        s1 = srf.Surface1D(m)
        errs.append(np.max(np.abs(s1.recover_dx(np.sin(m.xs_surf)) - np.cos(m.xs_surf))))
    assert errs[-1] < 1e-7 and errs[-1] < errs[0] / 1e4


def test_over_integration_exact_for_polynomial_products():
    """With Pf >= the degree of the integrands, the over-integrated projection
    J_e I^T M_h F equals Gauss quadrature of the exact integrand; with Pf = P
    (no over-integration) it does not (aliasing)."""
    P = 3
    m = Mesh(2, 1, P, 2.0, False)
    s1 = srf.Surface1D(m)
    x = m.xs_surf
    eta = 0.1 * x ** 2 - 0.05 * x
    etax, phix, w = 0.2 * x - 0.05, 0.3 * x ** 3 - x, 0.1 * x + 0.2
    g = 9.81
    # exact integrals of F v per element by 20-point Gauss-Legendre
    gx, gw = np.polynomial.legendre.leggauss(20)
    from oracle.refelem import Ref1D
    R = Ref1D(P)

    def exact_rhs():
        out_e, out_p = np.zeros(m.ns), np.zeros(m.ns)
        for e in range(m.nx):
            xq = m.xs[e] + 0.5 * m.dx * (1 + gx)
            ex = 0.2 * xq - 0.05
            px = 0.3 * xq ** 3 - xq
            ww = 0.1 * xq + 0.2
            et = 0.1 * xq ** 2 - 0.05 * xq
            fe = -ex * px + ww * (1 + ex ** 2)
            fp = -g * et - 0.5 * (px ** 2 - ww ** 2 * (1 + ex ** 2))
            Nq = R.interp_matrix(gx)          # nodal basis at Gauss points
            idx = s1.idx[e]
            out_e[idx] += 0.5 * m.dx * Nq.T @ (gw * fe)
            out_p[idx] += 0.5 * m.dx * Nq.T @ (gw * fp)
        return s1.solve_mass(out_e), s1.solve_mass(out_p)

    te, tp = exact_rhs()
    fe, fp = s1.fs_rhs(eta, etax, phix, w, g, Pf=3 * P)      # integrand degree <= 3P
    assert np.max(np.abs(fe - te)) < 1e-11 and np.max(np.abs(fp - tp)) < 1e-11
    ae, ap = s1.fs_rhs(eta, etax, phix, w, g, Pf=P)
    assert max(np.max(np.abs(ae - te)), np.max(np.abs(ap - tp))) > 1e-4
    I, Mf = fine_grid(P, 3 * P)
    assert I.shape == (3 * P + 1, P + 1) and np.allclose(gll_nodes(3 * P)[[0, -1]], [-1, 1])


def test_K_matches_sigma_map_jacobian_on_sloping_bed():
    """K = J J^T / det J with J = d(x, sigma)/d(x, z) of the sigma-map
    sigma(x, z) = (z + h(x)) / (eta(x) + h(x)) (Sec. 2, eqs. sigtrans and
    jacobian).  J is taken here by complex-step differentiation of the map
    itself at the physical position of every element node of a sloping-bed
    tank, independently of the closed form in coefficients().  eta and h are
    global polynomials of degree <= P so that the column interpolants are
    exact; G = |J^k| Lam K Lam^T is compared at every node."""
    P = 4
    m = Mesh(5, 3, P, 4.0, False)
    eta_f = lambda x: 0.12 - 0.03 * x + 0.01 * x ** 3 - 0.0015 * x ** 4
    h_f = lambda x: 1.0 - 0.09 * x + 0.02 * x ** 2
    etax_f = lambda x: -0.03 + 0.03 * x ** 2 - 0.006 * x ** 3
    hx_f = lambda x: -0.09 + 0.04 * x
    xs = m.xs_surf
    G, d = lap.coefficients(m, eta_f(xs), etax_f(xs), h_f(xs), hx_f(xs))

    def sigma(x, z):
        return (z + h_f(x)) / (eta_f(x) + h_f(x))

    x = m.ex
    z = m.esig * (eta_f(x) + h_f(x)) - h_f(x)
    step = 1e-30
    sx = np.imag(sigma(x + 1j * step, z)) / step
    sz = np.imag(sigma(x, z + 1j * step)) / step
    det = sz
    Kref = np.empty(x.shape + (2, 2))
    Kref[..., 0, 0] = 1.0 / det
    Kref[..., 0, 1] = sx / det
    Kref[..., 1, 0] = sx / det
    Kref[..., 1, 1] = (sx * sx + sz * sz) / det
    Gref = np.einsum("kac,kicd,kbd->kiab", m.Lam, Kref, m.Lam) * m.J[:, None, None, None]
    assert np.max(np.abs(d - 1.0 / sz)) < 1e-13
    assert np.max(np.abs(G[..., 0] - Gref[..., 0, 0])) < 1e-12
    assert np.max(np.abs(G[..., 1] - Gref[..., 0, 1])) < 1e-12
    assert np.max(np.abs(G[..., 2] - Gref[..., 1, 1])) < 1e-12
    # the bed slope really enters: a quarter of the nodes see |q| > 0.02
    assert np.mean(np.abs(sx / sz) > 0.02) > 0.25


def test_volume_kinematics_projection_sloping_bed():
    """The projections M u = S_u Phi and M w = S_z Phi of a smooth field
    phi(x, z) sampled at the nodes of a sloping-bed tank with a deformed
    surface recover d phi/dx and d phi/dz at every node, converging
    exponentially in P (exercises sigma_x with both its h_x and eta_x parts;
    the field need not be harmonic for this)."""
    L = 4.0
    phi_f = lambda x, z: np.sin(1.3 * x + 0.4) * np.exp(0.7 * z) + 0.2 * x * z * z
    phix_f = lambda x, z: 1.3 * np.cos(1.3 * x + 0.4) * np.exp(0.7 * z) + 0.2 * z * z
    phiz_f = lambda x, z: 0.7 * np.sin(1.3 * x + 0.4) * np.exp(0.7 * z) + 0.4 * x * z
    errs = []
    for P in (2, 4, 6, 8):
        m = Mesh(4, 2, P, L, False)
        xs = m.xs_surf
        eta = 0.1 * np.cos(1.1 * xs) + 0.05 * np.sin(0.4 * xs)
        etax = -0.11 * np.sin(1.1 * xs) + 0.02 * np.cos(0.4 * xs)
        h = 1.0 - 0.3 * np.exp(-(xs - 2.0) ** 2)
        hx = 0.6 * (xs - 2.0) * np.exp(-(xs - 2.0) ** 2)
        en, hn = m.column_interp(eta), m.column_interp(h)
        z = m.node_z(en, hn)
        Phi = np.zeros(m.n)
        Phi[m.EToN] = phi_f(m.ex, z)
        sx = lap.sigma_x(m, eta, etax, h, hx)
        _, d = lap.coefficients(m, eta, etax, h, hx)
        u = srf.recover_u(m, Phi, sx)
        w = srf.recover_w(m, Phi, d)
        ux = np.max(np.abs(u[m.EToN] - phix_f(m.ex, z)))
        wz = np.max(np.abs(w[m.EToN] - phiz_f(m.ex, z)))
        errs.append(max(ux, wz))
    # measured: 1.8e-1, 6.1e-3, 5.5e-4, 4.1e-5
    assert errs[1] < errs[0] / 8 and errs[2] < errs[1] / 8 and errs[3] < errs[2] / 8
    assert errs[3] < 1e-4


def test_volume_kinematics_manufactured_harmonic():
    """Laplace solve + projections on a deformed surface over a flat bed:
    u and w at every node converge to the gradient of the harmonic function
    cosh(k(z+h))/cosh(kh) sin(kx) (Sec. 4.3's kinematics, exact solution)."""
    k, h = 1.0, 1.0
    errs = []
    for P in (2, 4, 6):
        m = Mesh(4, 2, P, 2 * np.pi, True)
        s1 = srf.Surface1D(m)
        xs = m.xs_surf
        eta = 0.1 * np.cos(xs) + 0.03 * np.sin(2 * xs)
        etax = s1.recover_dx(eta)
        G, d = lap.coefficients(m, eta, etax, *flat(m, h))
        Phi = lap.solve_direct(m, lap.stiffness(m, G), exact.harmonic_phi(xs, eta, k, h))
        u = srf.recover_u(m, Phi, lap.sigma_x(m, eta, etax, *flat(m, h)))
        w = srf.recover_w(m, Phi, d)
        z = m.node_z(m.column_interp(eta), np.full((m.E, m.Np), h))
        ue = k * np.cosh(k * (z + h)) / np.cosh(k * h) * np.cos(k * m.ex)
        errs.append(max(np.max(np.abs(u[m.EToN] - ue)),
                        np.max(np.abs(w[m.EToN] - exact.harmonic_w(m.ex, z, k, h)))))
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10
    assert errs[2] < 2e-3
