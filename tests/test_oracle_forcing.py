"""Pins for the second-order part of the oracle's forcing: Guo's bracket (Eq. 23, Sec. 3.2),
its image in moment space (Eq. 34, Sec. 4.4.2) and Li's shifted velocity (Eq. 31-32, Sec. 4.3).

Each expected value is a closed form derived from the moments of the lattice, not the oracle's
formula typed again: a wrong velocity in the bracket (u instead of v), a wrong c_s^4 factor, a
dropped symmetric term, or upsilon read as the kinematic viscosity c_s^2 (tau - 1/2) instead of
(tau - 1/2) each fails one of these tests."""
import numpy as np
import pytest

from paper_1412_5170_amd import inputs

# the D2Q9 set written out here for the moment sums (order: rest, axes, diagonals)
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


def _moments(B):
    """Zeroth, first and second moments of nine values."""
    return (B.sum(), np.array([(B * EX).sum(), (B * EY).sum()]),
            np.array([[(B * EX * EX).sum(), (B * EX * EY).sum()],
                      [(B * EY * EX).sum(), (B * EY * EY).sum()]]))


def test_guo_bracket_moments(oracle):
    """Guo's source must add exactly F to the momentum and F V + V F to the momentum flux, and
    nothing to the mass (the Chapman-Enskog requirements behind Eq. 23): sum B = 0,
    sum B e = F, sum B e_i e_j = F_i V_j + V_i F_j."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        Fx, Fy, Vx, Vy = rng.normal(size=4) * np.array([1e-3, 1e-3, 0.1, 0.1])
        B = oracle.guo_bracket(Fx, Fy, Vx, Vy)
        m0, m1, m2 = _moments(B)
        F, V = np.array([Fx, Fy]), np.array([Vx, Vy])
        scale = np.abs(F).max()
        assert abs(m0) < 1e-16 * scale * 10
        assert np.allclose(m1, F, rtol=1e-14, atol=1e-18)
        assert np.allclose(m2, np.outer(F, V) + np.outer(V, F), rtol=1e-13,
                           atol=1e-15 * scale * np.abs(V).max())


def test_guo_source_in_moment_space(oracle):
    """S = M B(V) for the oracle's moment matrix, against the closed form
    (0, 6 V.F, -6 V.F, F_x, -F_x, F_y, -F_y, 2 (V_x F_x - V_y F_y), V_x F_y + V_y F_x) that
    follows from the bracket's moments up to fourth order on D2Q9."""
    M, _ = oracle.mrt_matrix()
    rng = np.random.default_rng(12)
    for _ in range(20):
        Fx, Fy, Vx, Vy = rng.normal(size=4) * np.array([1e-3, 1e-3, 0.1, 0.1])
        S = M @ oracle.guo_bracket(Fx, Fy, Vx, Vy)
        vf = Vx * Fx + Vy * Fy
        want = np.array([0.0, 6 * vf, -6 * vf, Fx, -Fx, Fy, -Fy, 2 * (Vx * Fx - Vy * Fy),
                         Vx * Fy + Vy * Fx])
        assert np.allclose(S, want, rtol=1e-13, atol=1e-17), (S, want)


def _node_state(oracle, thermo, scheme, coll, tau, s=None, n=6, seed=3, sigma=0.11):
    O = oracle
    s = s or (1.0,) * 9
    p = O.Params(nx=n, ny=n, T=thermo.temperature(0.7), tau=tau, K=1.0, A=-0.3, sigma=sigma,
                 scheme=getattr(O, scheme), collision=getattr(O, coll), s=s)
    f = inputs.random_populations(seed, n, n, 0.05, 0.35, 0.05)
    return p, f, O.fields(p, f)


def _second_moment_field(f):
    """sum_a f_a e_ai e_aj per node: [2, 2, ny, nx]."""
    e = np.stack([EX, EY])
    return np.einsum("ia,ja,ayx->ijyx", e, e, f)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 1.7])
def test_guo_bgk_momentum_flux_closed_form(oracle, thermo, tau):
    """BGK with Guo's forcing (Eq. 1 + Eq. 23), node by node: the post-collision momentum flux
    is Pi* = Pi - (Pi - Pi_eq(rho, v)) / tau + (1 - 1/(2 tau)) (F v + v F), with
    Pi_eq(rho, v) = rho (I/3 + v v) the flux of Eq. 2 and v = u + F / (2 rho).  Using u for v in
    the equilibrium or the bracket, or a wrong c_s^4 in the bracket, breaks it."""
    p, f, fl = _node_state(oracle, thermo, "GUO", "BGK", tau)
    post = oracle.collide(p, f)
    rho, vx, vy, Fx, Fy = fl["rho"], fl["vx"], fl["vy"], fl["Fx"], fl["Fy"]
    Pi = _second_moment_field(f)
    v = np.stack([vx, vy])
    F = np.stack([Fx, Fy])
    eye = np.eye(2)[:, :, None, None]
    Pi_eq = rho * (eye / 3 + v[:, None] * v[None, :])
    want = Pi - (Pi - Pi_eq) / tau + (1 - 1 / (2 * tau)) * (F[:, None] * v[None, :] +
                                                             v[:, None] * F[None, :])
    got = _second_moment_field(post)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-17)
    # the same with u in place of v is measurably different on this state
    u = np.stack([fl["ux"], fl["uy"]])
    wrong = Pi - (Pi - rho * (eye / 3 + u[:, None] * u[None, :])) / tau + \
        (1 - 1 / (2 * tau)) * (F[:, None] * u[None, :] + u[:, None] * F[None, :])
    assert np.abs(wrong - got).max() > 1e3 * np.abs(got - want).max()


def test_guo_mrt_moments_closed_form(oracle, thermo):
    """MRT with Guo's source (Eq. 34-35): in moment space m* = m - Lambda (m - m_eq) +
    (I - Lambda/2) S with m_eq = rho (1, -2 + 3 v.v, 1 - 3 v.v, v_x, -v_x, v_y, -v_y,
    v_x^2 - v_y^2, v_x v_y) and S the closed form of the test above, at v = u + F / (2 rho)."""
    tau = 0.8
    s = (1.0, 1.1, 1.2, 1.0, 1.3, 1.0, 1.3, 1 / tau, 1 / tau)
    p, f, fl = _node_state(oracle, thermo, "GUO", "MRT", tau, s=s)
    M, _ = oracle.mrt_matrix()
    post = oracle.collide(p, f)
    m = np.einsum("ka,ayx->kyx", M, f)
    got = np.einsum("ka,ayx->kyx", M, post)
    rho, vx, vy, Fx, Fy = fl["rho"], fl["vx"], fl["vy"], fl["Fx"], fl["Fy"]
    v2 = vx * vx + vy * vy
    meq = rho * np.stack([np.ones_like(vx), -2 + 3 * v2, 1 - 3 * v2, vx, -vx, vy, -vy,
                          vx * vx - vy * vy, vx * vy])
    vf = vx * Fx + vy * Fy
    S = np.stack([0 * vf, 6 * vf, -6 * vf, Fx, -Fx, Fy, -Fy, 2 * (vx * Fx - vy * Fy),
                  vx * Fy + vy * Fx])
    sv = np.array(s)[:, None, None]
    want = m - sv * (m - meq) + (1 - sv / 2) * S
    assert np.allclose(got, want, rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 1.5])
def test_li_bgk_extra_flux(oracle, thermo, tau):
    """Li's term (Eq. 31 with upsilon = tau - 1/2) changes Guo's BGK collision only in the
    momentum flux, by (1 - 1/(2 tau)) (F dv + dv F) with dv = sigma F / ((tau - 1/2) psi^2),
    i.e. exactly (1/tau) 2 sigma F F / psi^2 -- the extra pressure whose Chapman-Enskog
    strength makes Eq. 32 hold.  Reading upsilon as c_s^2 (tau - 1/2) would triple it."""
    sigma = 0.11
    pl, f, fl = _node_state(oracle, thermo, "GUO_LI", "BGK", tau, sigma=sigma)
    pg, _, _ = _node_state(oracle, thermo, "GUO", "BGK", tau, sigma=sigma)
    d = oracle.collide(pl, f) - oracle.collide(pg, f)
    m0, m1 = d.sum(0), np.stack([(d * EX[:, None, None]).sum(0), (d * EY[:, None, None]).sum(0)])
    F = np.stack([fl["Fx"], fl["Fy"]])
    X = 2 * sigma * F[:, None] * F[None, :] / fl["psi"] ** 2
    got = _second_moment_field(d)
    scale = np.abs(X).max() / tau
    assert scale > 1e-8                          # the state has a real force
    assert np.abs(m0).max() < 1e-13 * scale and np.abs(m1).max() < 1e-13 * scale
    assert np.allclose(got, X / tau, rtol=1e-10, atol=1e-12 * scale)


def test_li_mrt_per_moment_source(oracle, thermo):
    """Li's term in the MRT collision (the per-moment reading of Eq. 31 for Eq. 34): with
    X = 2 sigma F F / psi^2, the difference Li - Guo of the post-collision moments is
    (0, 3 s_e tr X, -3 s_eps tr X, 0, 0, 0, 0, s_nu (X_xx - X_yy), s_nu X_xy) -- each moment's
    source (I - Lambda/2) X_k / (1/s_k - 1/2) collapses to s_k X_k -- and with every rate equal
    to 1/tau it is the BGK extra flux of the test above."""
    sigma, tau = 0.11, 0.8
    s = (1.0, 1.1, 1.2, 1.0, 1.3, 1.0, 1.3, 1 / tau, 1 / tau)
    pl, f, fl = _node_state(oracle, thermo, "GUO_LI", "MRT", tau, s=s, sigma=sigma)
    pg, _, _ = _node_state(oracle, thermo, "GUO", "MRT", tau, s=s, sigma=sigma)
    M, _ = oracle.mrt_matrix()
    dm = np.einsum("ka,ayx->kyx", M, oracle.collide(pl, f) - oracle.collide(pg, f))
    c = 2 * sigma / fl["psi"] ** 2
    Xxx, Xyy, Xxy = c * fl["Fx"] ** 2, c * fl["Fy"] ** 2, c * fl["Fx"] * fl["Fy"]
    tr = Xxx + Xyy
    z = np.zeros_like(tr)
    want = np.stack([z, 3 * s[1] * tr, -3 * s[2] * tr, z, z, z, z, s[7] * (Xxx - Xyy),
                     s[8] * Xxy])
    scale = np.abs(want).max()
    assert scale > 1e-8
    assert np.allclose(dm, want, rtol=1e-10, atol=1e-12 * scale)
    # equal rates: the BGK flux (1/tau) X
    s_eq = (1 / tau,) * 9
    pl, _, _ = _node_state(oracle, thermo, "GUO_LI", "MRT", tau, s=s_eq, sigma=sigma)
    pg, _, _ = _node_state(oracle, thermo, "GUO", "MRT", tau, s=s_eq, sigma=sigma)
    d = oracle.collide(pl, f) - oracle.collide(pg, f)
    X = np.stack([np.stack([Xxx, Xxy]), np.stack([Xxy, Xyy])])
    assert np.allclose(_second_moment_field(d), X / tau, rtol=1e-10, atol=1e-12 * scale)
