"""Pins of the FP64 oracle's single-node arithmetic against what the paper and
the mathematics fix (lattice symmetries, moment identities, exact stencils,
the equilibrium of the chemical potential, closed forms of the WMRT products).
Each test is chosen so that a plausible slip in the oracle (a wrong sign, a
dropped term, a transposed matrix, a wrong velocity order) fails it."""
import itertools

import numpy as np
import pytest

import oracle

LATTICES = (9, 19)


def _isotropic4(e, w):
    d = 3
    T = np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e)
    I = np.eye(d)
    ref = (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I)
           + np.einsum("il,jk->ijkl", I, I)) / 9.0
    return T, ref


@pytest.mark.parametrize("q", LATTICES)
def test_lattice_isotropy_and_opposites(q):
    e, w, opp, M, Mi, s = oracle.lattice(q)
    d = 2 if q == 9 else 3
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ e).max() < 1e-16
    second = np.einsum("a,ai,aj->ij", w, e, e)
    ref2 = np.zeros((3, 3))
    ref2[:d, :d] = np.eye(d) / 3.0
    assert np.abs(second - ref2).max() < 1e-15
    assert np.abs(np.einsum("a,ai,aj,ak->ijk", w, e, e, e)).max() < 1e-16
    T, ref = _isotropic4(e.astype(float), w)
    if d == 3:
        assert np.abs(T - ref).max() < 1e-15
    else:
        assert np.abs(T[:2, :2, :2, :2] - ref[:2, :2, :2, :2]).max() < 1e-15
    for a in range(q):
        assert (e[opp[a]] == -e[a]).all()


def test_d3q19_order_matches_appendix_a():
    """Rows 1-3 of the printed D3Q19 matrix are e_x, e_y, e_z, and the inlet
    unknowns of a face with inward normal +x are 1, 7, 9, 11, 13 (appendix B)."""
    e, w, opp, M, Mi, s = oracle.lattice(19)
    assert (M[1] == e[:, 0]).all() and (M[2] == e[:, 1]).all() and (M[3] == e[:, 2]).all()
    assert sorted(np.nonzero(e[:, 0] == 1)[0].tolist()) == [1, 7, 9, 11, 13]
    # stress rows (relaxed with s_nu) are xy, yz, xz, 2x^2-y^2-z^2, y^2-z^2
    ex, ey, ez = e.T
    assert (M[4] == ex * ey).all() and (M[5] == ey * ez).all() and (M[6] == ex * ez).all()
    assert (M[7] == 2 * ex**2 - ey**2 - ez**2).all() and (M[8] == ey**2 - ez**2).all()
    assert s.tolist() == [0, 0, 0, 0, 1, 1, 1, 1, 1] + [0] * 10


def test_d2q9_order_matches_appendix_a():
    """Rows 3 and 5 of the printed D2Q9 matrix are j_x and j_y; the inlet
    unknowns of a face with inward normal +x are 1, 5, 8 (appendix B)."""
    e, w, opp, M, Mi, s = oracle.lattice(9)
    assert (M[3] == e[:, 0]).all() and (M[5] == e[:, 1]).all()
    assert sorted(np.nonzero(e[:, 0] == 1)[0].tolist()) == [1, 5, 8]
    ex, ey = e[:, 0], e[:, 1]
    assert (M[7] == ex**2 - ey**2).all() and (M[8] == ex * ey).all()
    assert w[0] == 4 / 9 and np.allclose(w[1:5], 1 / 9) and np.allclose(w[5:], 1 / 36)


def test_moment_matrices():
    e, w, opp, M, Mi, s = oracle.lattice(19)
    D = M @ np.diag(w) @ M.T
    diag = np.array([1, 1 / 3, 1 / 3, 1 / 3, 1 / 9, 1 / 9, 1 / 9, 4 / 3, 4 / 9, 2 / 3, 2 / 3, 2 / 3,
                     2 / 3, 2 / 9, 2 / 9, 2 / 9, 2, 4 / 3, 4 / 9])
    assert np.abs(D - np.diag(diag)).max() < 1e-15
    assert np.abs(M @ Mi - np.eye(19)).max() < 1e-14
    e9, w9, _, M9, Mi9, _ = oracle.lattice(9)
    D9 = M9 @ M9.T
    assert np.abs(D9 - np.diag(np.diag(D9))).max() == 0.0
    assert np.abs(M9 @ Mi9 - np.eye(9)).max() < 1e-14


def _rand_u(rng, q, scale=0.05):
    u = rng.uniform(-scale, scale, 3)
    if q == 9:
        u[2] = 0.0
    return u


@pytest.mark.parametrize("q", LATTICES)
def test_equilibrium_moments(q):
    rng = np.random.default_rng(1)
    e, w, *_ = oracle.lattice(q)
    d = 2 if q == 9 else 3
    for _ in range(5):
        u = _rand_u(rng, q)
        ps = rng.uniform(-0.1, 0.1)
        f = oracle.feq(q, ps, u)
        assert abs(f.sum() - ps) < 1e-15
        assert np.abs(f @ e - u).max() < 1e-16
        Pi = np.einsum("a,ai,aj->ij", f, e, e)
        ref = np.outer(u, u)
        ref[:d, :d] += ps / 3.0 * np.eye(d)
        assert np.abs(Pi - ref).max() < 1e-15
        phi = rng.uniform(0, 1)
        h = oracle.heq(q, phi, u)
        assert abs(h.sum() - phi) < 1e-15
        assert np.abs(h @ e - phi * u).max() < 1e-16


@pytest.mark.parametrize("q", LATTICES)
def test_forcing_moments(q):
    """sum F^phi = 0, sum e F^phi = theta n / 3 with theta = (1 - 4(phi-1/2)^2)/xi."""
    rng = np.random.default_rng(2)
    e, w, *_ = oracle.lattice(q)
    for _ in range(5):
        gp = _rand_u(rng, q, 0.2)
        phi = rng.uniform(0, 1)
        xi = 4.0
        F = oracle.phase_forcing(q, phi, gp, xi)
        theta = (1 - 4 * (phi - 0.5) ** 2) / xi
        n = gp / np.linalg.norm(gp)
        assert abs(F.sum()) < 1e-16
        assert np.abs(F @ e - theta * n / 3.0).max() < 1e-16


@pytest.mark.parametrize("q", LATTICES)
def test_stencils_exact_on_polynomials(q):
    e, w, *_ = oracle.lattice(q)
    rng = np.random.default_rng(3)
    x0 = rng.uniform(-2, 2, 3)
    if q == 9:
        x0[2] = 0
    b = rng.uniform(-1, 1, 3)
    if q == 9:
        b[2] = 0
    lin = lambda x: 0.3 + x @ b
    grad, lap = oracle.grad_lap(q, np.array([lin(x0 + ea) for ea in e]))
    assert np.abs(grad - b).max() < 1e-14 and abs(lap) < 1e-14
    A = rng.uniform(-1, 1, (3, 3))
    A = A + A.T
    if q == 9:
        A[2, :] = A[:, 2] = 0
    quad = lambda x: x @ A @ x
    grad, lap = oracle.grad_lap(q, np.array([quad(x0 + ea) for ea in e]))
    assert np.abs(grad - 2 * A @ x0).max() < 1e-13
    assert abs(lap - 2 * np.trace(A)) < 1e-13


def test_stencil_second_order_on_sinusoid():
    """Gradient error of the isotropic stencil falls as dx^2 on a sinusoid."""
    e, w, *_ = oracle.lattice(19)
    errs = []
    for k in (0.2, 0.1, 0.05):
        x0 = np.array([0.37, 0.11, -0.23])
        f = lambda x: np.sin(k * (x[0] + 2 * x[1] - x[2]))
        grad, lap = oracle.grad_lap(19, np.array([f(x0 + ea) for ea in e]))
        exact = k * np.cos(k * (x0[0] + 2 * x0[1] - x0[2])) * np.array([1, 2, -1])
        errs.append(np.abs(grad - exact).max() / k)
    slope = np.log(errs[0] / errs[2]) / np.log(4.0)
    assert 1.9 < slope < 2.1


def test_chemical_potential_vanishes_on_equilibrium_profile():
    """The tanh kernel (Eq. kernel_function) is the equilibrium of mu_phi with
    beta = 12 sigma/xi, kappa = 3 sigma xi/2: with the bulk term
    4 beta phi (phi-1)(phi-1/2) the discrete residual is small and shrinks
    as xi grows; with the printed factor (1-phi) it does not."""
    e, w, *_ = oracle.lattice(9)
    sigma = 1e-3
    worst = []
    for xi in (4.0, 8.0):
        beta = 12 * sigma / xi
        prof = lambda x: 0.5 + 0.5 * np.tanh(2 * x / xi)
        res, res_printed = 0.0, 0.0
        for x in np.linspace(-2 * xi, 2 * xi, 41):
            phin = np.array([prof(x + ea[0]) for ea in e])
            _, lap = oracle.grad_lap(9, phin)
            mu = oracle.chem_potential(phin[0], lap, sigma, xi)
            res = max(res, abs(mu))
            kappa = 1.5 * sigma * xi
            printed = 4 * beta * phin[0] * (1 - phin[0]) * (phin[0] - 0.5) - kappa * lap
            res_printed = max(res_printed, abs(printed))
        worst.append(res / beta)
        assert res < 2e-2 * beta
        assert res_printed > 0.1 * beta
    assert worst[1] < worst[0] / 3.0


def _hermite_projection(q, y):
    """Closed-form projection of y onto the stress modes relaxed with s_nu.
    D3Q19 (weighted orthogonal): 4.5 w_a (e_a e_a : dev Pi_y).
    D2Q9 (plain orthogonal basis of the printed matrix):
    [(e_x^2 - e_y^2)(Pi_xx - Pi_yy) + e_x e_y Pi_xy] / 4."""
    e, w, *_ = oracle.lattice(q)
    e = e.astype(float)
    Pi = np.einsum("a,ai,aj->ij", y, e, e)
    if q == 19:
        dev = Pi - np.trace(Pi) / 3.0 * np.eye(3)
        return 4.5 * w * np.einsum("ai,aj,ij->a", e, e, dev)
    ex, ey = e[:, 0], e[:, 1]
    return ((ex**2 - ey**2) * (Pi[0, 0] - Pi[1, 1]) + ex * ey * Pi[0, 1]) / 4.0


@pytest.mark.parametrize("q", LATTICES)
def test_wmrt_collision_equals_closed_form(q):
    """g+ = g - M^-1 S M (g - fbar) + F_a equals fbar + (1 - s) P(g - fbar) + F_a,
    P the projection onto the stress modes, s = 1/(tau + 1/2)."""
    rng = np.random.default_rng(4)
    e, w, *_ = oracle.lattice(q)
    for tau in (0.003, 0.3, 1.7):
        s = 1.0 / (tau + 0.5)
        u = _rand_u(rng, q)
        ps = rng.uniform(-0.01, 0.01)
        feq = oracle.feq(q, ps, u)
        g = feq + 1e-3 * rng.standard_normal(q)
        F = _rand_u(rng, q, 1e-4)
        rho = rng.uniform(0.01, 1)
        gp = oracle.collide_g(q, g, feq, F, rho, tau)
        Fa = w * (e @ F) / (rho / 3.0)
        fbar = feq - 0.5 * Fa
        ref = fbar + (1 - s) * _hermite_projection(q, g - fbar) + Fa
        assert np.abs(gp - ref).max() < 1e-15


@pytest.mark.parametrize("q", LATTICES)
def test_wmrt_is_bgk_at_tau_half(q):
    """With s_nu = 1 every moment relaxes fully: WMRT = BGK (Eq. bgk_collision)."""
    rng = np.random.default_rng(5)
    e, w, *_ = oracle.lattice(q)
    u = _rand_u(rng, q)
    feq = oracle.feq(q, 0.01, u)
    g = feq + 1e-3 * rng.standard_normal(q)
    F = _rand_u(rng, q, 1e-4)
    gp = oracle.collide_g(q, g, feq, F, 0.5, 0.5)
    Fa = w * (e @ F) / (0.5 / 3.0)
    bgk = g - (g - (feq - 0.5 * Fa)) / (0.5 + 0.5) + Fa
    assert np.abs(gp - bgk).max() < 1e-15


@pytest.mark.parametrize("q", LATTICES)
def test_bgk_operator_reduces_to_wmrt_at_tau_half(q):
    """The selectable BGK operator (Eqs. bgk_collision, viscous_force_bgk)
    and WMRT coincide when s_nu = 1, and differ otherwise; with f^eq built
    from p* = sum g, BGK keeps sum g (sum F_a = 0)."""
    rng = np.random.default_rng(8)
    e, w, *_ = oracle.lattice(q)
    u = _rand_u(rng, q)
    g = oracle.feq(q, 0.01, u) + 1e-3 * rng.standard_normal(q)
    feq = oracle.feq(q, g.sum(), u)
    F = _rand_u(rng, q, 1e-4)
    gr = _rand_u(rng, q, 0.3)
    for tau, same in ((0.5, True), (0.05, False), (1.3, False)):
        a = oracle.collide_g(q, g, feq, F, 0.7, tau, op="bgk")
        b = oracle.collide_g(q, g, feq, F, 0.7, tau, op="wmrt")
        fa = oracle.viscous_force(q, g, feq, tau, gr, op="bgk")
        fb = oracle.viscous_force(q, g, feq, tau, gr, op="wmrt")
        if same:
            assert np.abs(a - b).max() < 1e-16 and np.abs(fa - fb).max() < 1e-17
        else:
            assert np.abs(a - b).max() > 1e-6 and np.abs(fa - fb).max() > 1e-6 * np.abs(fb).max()
        assert abs(a.sum() - g.sum()) < 1e-15


@pytest.mark.parametrize("q", LATTICES)
def test_viscous_force_closed_form(q):
    """F_mu = -tau [s dev(Pi) + tr(Pi)/d I] grad rho, Pi = sum e e (g - feq)."""
    rng = np.random.default_rng(6)
    e, w, *_ = oracle.lattice(q)
    d = 2 if q == 9 else 3
    for tau in (0.01, 0.3, 2.0):
        s = 1.0 / (tau + 0.5)
        u = _rand_u(rng, q)
        feq = oracle.feq(q, 0.02, u)
        g = feq + 1e-3 * rng.standard_normal(q)
        gr = _rand_u(rng, q, 0.3)
        fmu = oracle.viscous_force(q, g, feq, tau, gr)
        Pi = np.einsum("a,ai,aj->ij", g - feq, e, e)[:d, :d]
        tr = np.trace(Pi) / d
        T = s * (Pi - tr * np.eye(d)) + tr * np.eye(d)
        ref = np.zeros(3)
        ref[:d] = -tau * T @ gr[:d]
        assert np.abs(fmu - ref).max() < 1e-16 + 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("q", LATTICES)
def test_phase_collision_conserves_phi(q):
    rng = np.random.default_rng(7)
    for _ in range(5):
        phi = rng.uniform(-0.1, 1.1)
        u = _rand_u(rng, q)
        gp = _rand_u(rng, q, 0.3)
        h = oracle.heq(q, phi, u) + 1e-3 * rng.standard_normal(q)
        hp = oracle.collide_h(q, h, h.sum(), u, gp, 4.0, 0.02)
        assert abs(hp.sum() - h.sum()) < 2e-15


@pytest.mark.parametrize("q", LATTICES)
def test_node_update_at_rest_is_fixed(q):
    """Uniform phase, zero velocity and pressure: the node update returns its input."""
    cfg = dict(q=q, nx=4, ny=4, nz=1 if q == 9 else 4, rho_h=1.0, rho_l=1e-3, tau_h=0.3,
               tau_l=0.05, sigma=1e-3, xi=4.0, mobility=0.02)
    for phi in (0.0, 1.0):
        h = oracle.heq(q, phi, np.zeros(3))
        g = oracle.feq(q, 0.0, np.zeros(3))
        hp, gp, un = oracle.collide_node(cfg, h, g, np.zeros(3), np.full(q, phi))
        assert np.abs(hp - h).max() < 1e-16 and np.abs(gp - g).max() < 1e-16
        assert np.abs(un).max() == 0.0
