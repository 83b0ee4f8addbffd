"""Pins of the oracle's reference-element operators (CPU).

Each check compares against something the mathematics fixes independently of
the oracle's own construction: closed-form GLL nodes, exact integrals of
monomials over the reference triangle, exact derivatives of polynomials, the
textbook linear-triangle stiffness, symmetry of the node set."""
from math import comb, factorial, sqrt

import numpy as np
import pytest

from oracle.refelem import (Ref1D, RefTri, filter_matrix, fine_grid, gll_nodes,
                            modified_basis)


def tri_monomial_integral(a, b):
    """int over {(-1,-1),(1,-1),(-1,1)} of r^a s^b, from r = 2u-1, s = 2v-1 and
    int_{u,v>=0,u+v<=1} u^p v^q = p! q! / (p+q+2)!  (area element 4 du dv)."""
    tot = 0.0
    for p in range(a + 1):
        for q in range(b + 1):
            coef = comb(a, p) * comb(b, q) * 2 ** p * 2 ** q * (-1) ** (a - p) * (-1) ** (b - q)
            tot += coef * factorial(p) * factorial(q) / factorial(p + q + 2)
    return 4.0 * tot


def test_gll_closed_forms():
    # textbook Gauss-Lobatto-Legendre nodes
    assert np.allclose(gll_nodes(1), [-1, 1], atol=0)
    assert np.allclose(gll_nodes(2), [-1, 0, 1], atol=1e-15)
    assert np.allclose(gll_nodes(3), [-1, -1 / sqrt(5), 1 / sqrt(5), 1], atol=1e-15)
    assert np.allclose(gll_nodes(4), [-1, -sqrt(3 / 7), 0, sqrt(3 / 7), 1], atol=1e-15)
    # P = 5: +-sqrt(1/3 -+ 2 sqrt(7)/21)
    inner = sorted([sqrt(1 / 3 - 2 * sqrt(7) / 21), sqrt(1 / 3 + 2 * sqrt(7) / 21)])
    g5 = gll_nodes(5)
    assert np.allclose(g5[3:5], inner, atol=1e-15) and np.allclose(g5[1:3], [-inner[1], -inner[0]], atol=1e-15)


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6, 7, 8])
def test_1d_operators_exact(P):
    R = Ref1D(P)
    r = R.r
    for a in range(P + 1):
        f = r ** a
        df = a * r ** (a - 1) if a else 0 * r
        assert np.max(np.abs(R.D @ f - df)) < 1e-12
        for b in range(P + 1):
            exact = (1 - (-1) ** (a + b + 1)) / (a + b + 1)
            assert abs(f @ R.M @ (r ** b) - exact) < 1e-13
    # interpolation to the fine grid reproduces polynomials of degree <= P
    I, Mf = fine_grid(P, 2 * P)
    rf = gll_nodes(2 * P)
    for a in range(P + 1):
        assert np.max(np.abs(I @ r ** a - rf ** a)) < 1e-13
    # fine mass integrates degree <= 4P exactly
    for a in range(0, 2 * P + 1):
        exact = (1 - (-1) ** (a + 1)) / (a + 1)
        assert abs(np.ones(2 * P + 1) @ Mf @ rf ** a - exact) < 1e-13


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6, 8])
def test_triangle_operators_exact(P):
    T = RefTri(P)
    r, s = T.r, T.s
    assert T.Np == (P + 1) * (P + 2) // 2 == len(r)
    one = np.ones(T.Np)
    assert abs(one @ T.M @ one - 2.0) < 1e-13                       # area
    assert np.max(np.abs(T.Dr @ one)) < 1e-12 and np.max(np.abs(T.Ds @ one)) < 1e-12
    assert np.all(np.linalg.eigvalsh(0.5 * (T.M + T.M.T)) > 0)
    mono = [(a, b) for a in range(P + 1) for b in range(P + 1 - a)]
    for a, b in mono:
        f = r ** a * s ** b
        fr = a * r ** max(a - 1, 0) * s ** b if a else 0 * r
        fs = b * r ** a * s ** max(b - 1, 0) if b else 0 * r
        assert np.max(np.abs(T.Dr @ f - fr)) < 1e-11
        assert np.max(np.abs(T.Ds @ f - fs)) < 1e-11
    # mass matrix integrates products of degree-P polynomials exactly
    for a, b in mono[:: max(1, len(mono) // 6)]:
        for c, d in mono[:: max(1, len(mono) // 5)]:
            lhs = (r ** a * s ** b) @ T.M @ (r ** c * s ** d)
            assert abs(lhs - tri_monomial_integral(a + c, b + d)) < 1e-12


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6, 8])
def test_warp_blend_node_set(P):
    T = RefTri(P)
    g = gll_nodes(P)
    # the three edges carry the GLL points
    assert np.allclose(np.sort(T.r[np.abs(T.s + 1) < 1e-13]), g, atol=1e-14)
    assert np.allclose(np.sort(T.s[np.abs(T.r + 1) < 1e-13]), g, atol=1e-14)
    hyp = np.abs(T.r + T.s) < 1e-13
    assert np.allclose(np.sort(T.r[hyp]), g, atol=1e-14)
    # invariant under the symmetries of the triangle: r <-> s and the vertex
    # rotation (r, s) -> (s, -1 - r - s)
    pts = np.round(np.column_stack([T.r, T.s]), 12)
    for img in (np.column_stack([T.s, T.r]), np.column_stack([T.s, -1 - T.r - T.s])):
        a = sorted(map(tuple, pts))
        b = sorted(map(tuple, np.round(img, 12)))
        assert np.allclose(np.array(a), np.array(b), atol=1e-11)
    if P == 3:   # the one interior node is the centroid
        inner = (np.abs(T.r + 1) > 1e-12) & (np.abs(T.s + 1) > 1e-12) & ~hyp
        assert np.allclose([T.r[inner][0], T.s[inner][0]], [-1 / 3, -1 / 3], atol=1e-14)
    assert np.linalg.cond(T.V) < 50


def test_p1_stiffness_is_textbook():
    """P = 1, K = I: the quadrature-free stiffness equals the linear-triangle
    stiffness (b_i b_j + c_i c_j)/(4 area) on a physical triangle."""
    from oracle.laplace import element_stiffness
    T = RefTri(1)
    X = np.array([[0.3, 0.1], [1.7, 0.4], [0.6, 1.3]])   # vertices A, B, C
    dxdrs = np.column_stack([(X[1] - X[0]) / 2, (X[2] - X[0]) / 2])
    Lam = np.linalg.inv(dxdrs)
    J = np.linalg.det(dxdrs)
    G = J * Lam @ Lam.T
    Gk = np.tile([G[0, 0], G[0, 1], G[1, 1]], (3, 1))
    A = element_stiffness(T, Gk)
    # nodes of RefTri(1) are the vertices in the order A, B, C
    assert np.allclose(np.column_stack([T.r, T.s]), [[-1, -1], [1, -1], [-1, 1]])
    e1, e2 = X[1] - X[0], X[2] - X[0]
    area = 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])
    b = np.array([X[1, 1] - X[2, 1], X[2, 1] - X[0, 1], X[0, 1] - X[1, 1]])
    c = np.array([X[2, 0] - X[1, 0], X[0, 0] - X[2, 0], X[1, 0] - X[0, 0]])
    ref = (np.outer(b, b) + np.outer(c, c)) / (4 * area)
    assert np.max(np.abs(A - ref)) < 1e-13


@pytest.mark.parametrize("P,ic,sf", [(6, 5, 0.995), (6, 6, 0.95), (4, 3, 0.9), (8, 2, 0.5)])
def test_filter_properties(P, ic, sf):
    F = filter_matrix(P, ic, sf)
    r = gll_nodes(P)
    # end values (vertex modes) untouched -> C0 continuity kept
    for _ in range(3):
        f = np.random.default_rng(P + ic).standard_normal(P + 1)
        g = F @ f
        assert abs(g[0] - f[0]) < 1e-13 and abs(g[-1] - f[-1]) < 1e-13
    # polynomials of degree < ic pass unchanged
    for a in range(ic):
        assert np.max(np.abs(F @ r ** a - r ** a)) < 1e-12
    ev = np.sort(np.abs(np.linalg.eigvals(F)))
    assert np.allclose(ev[: P + 1 - ic], sf, atol=1e-12) and np.allclose(ev[P + 1 - ic:], 1.0, atol=1e-12)
    # mean preserved when only modes >= 3 are touched (int phi_{n+1} = 0, n >= 2)
    M = Ref1D(P).M
    f = np.cos(2.0 * r) + r ** P
    if ic >= 3:
        assert abs(np.ones(P + 1) @ M @ (F @ f - f)) < 1e-13
    # the modified basis: bubble mode 2 integrates to 1/3 (so ic = 2 changes the mean)
    Vh = modified_basis(P, r)
    assert abs(np.ones(P + 1) @ M @ Vh[:, 2] - 1 / 3) < 1e-13


def test_filter_rejects_vertex_modes():
    with pytest.raises(ValueError):
        filter_matrix(6, 1, 0.9)


def lebesgue_constant(r, s, P, n=120):
    """max over a uniform sample of the reference triangle of sum_i |l_i|,
    with the Lagrange basis of the node set (r, s) evaluated through the
    orthonormal simplex basis."""
    from oracle.refelem import simplex_basis, simplex_modes
    modes = simplex_modes(P)
    V = np.stack([simplex_basis(r, s, i, j) for i, j in modes], axis=1)
    g = np.linspace(-1.0, 1.0, n + 1)
    R, S = np.meshgrid(g, g)
    inside = R + S <= 1e-12
    Vs = np.stack([simplex_basis(R[inside], S[inside], i, j) for i, j in modes], axis=1)
    return np.abs(Vs @ np.linalg.inv(V)).sum(axis=1).max()


@pytest.mark.parametrize("P", [6, 7, 8, 9])
def test_alpha_opt_minimises_lebesgue_constant(P):
    """Warburton's alpha_opt is defined as the blending parameter that
    minimises the Lebesgue constant of the warp-and-blend nodes.  The nodes
    the oracle builds for order P (through its table lookup) must therefore
    beat alpha = 0 and the table entries of the neighbouring orders, and lie
    within 0.5% of the best value on an alpha grid."""
    from oracle.refelem import ALPHA_OPT, warp_blend_nodes
    lam = lebesgue_constant(*warp_blend_nodes(P), P)
    others = [lebesgue_constant(*warp_blend_nodes(P, a), P) for a in (0.0, ALPHA_OPT[P - 1], ALPHA_OPT[P + 1])]
    assert lam < min(others) - 1e-3
    grid = [lebesgue_constant(*warp_blend_nodes(P, a), P) for a in np.linspace(0.5, 2.0, 16)]
    assert lam < 1.005 * min(grid)
