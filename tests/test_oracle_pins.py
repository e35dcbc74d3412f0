"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: values the paper prints (Table 2),
closed-form solutions, exact moment identities of the Hermite construction, invariants (mass,
affinity, lattice symmetry) and convergence orders.  Together they are chosen so that a dropped term,
a wrong sign or index, or a transposed operand anywhere in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _E(c=1.0):
    ex, ey, w = O.lattice()
    return c * ex.astype(float), c * ey.astype(float), w


# ---- P1: lattice (Sec. 2.2) --------------------------------------------------------------------

def test_lattice_velocity_set_and_weights():
    ex, ey, w = O.lattice()
    pairs = sorted(zip(ex.tolist(), ey.tolist()))
    assert pairs == sorted([(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)])
    for i in range(9):
        n2 = ex[i] ** 2 + ey[i] ** 2
        assert w[i] == {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}[n2]


def test_lattice_isotropy():
    c = 2.7
    ex, ey, w = _E(c)
    cs2 = c * c / 3
    e = [ex, ey]
    assert abs(w.sum() - 1) < 1e-15
    for a in range(2):
        assert abs((w * e[a]).sum()) < 1e-14
        for b in range(2):
            assert abs((w * e[a] * e[b]).sum() - cs2 * (a == b)) < 1e-13
            for g in range(2):
                assert abs((w * e[a] * e[b] * e[g]).sum()) < 1e-12
                for d in range(2):
                    want = cs2 * cs2 * ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g))
                    assert abs((w * e[a] * e[b] * e[g] * e[d]).sum() - want) < 1e-12


# ---- diagnostics: the error norms and mass written out (Sec. 3, Eq. (33)) ----------------------

def test_error_norms_closed_form():
    """Integer fields whose error norms are exact: the difference d = phi_num - phi_ref has
    ||d||_2 = 5 with its largest magnitude (4) on a negative entry, ||phi_ref||_2 = 13, and
    ||phi_num||_2^2 = 178, so a norm taken over phi_num, a dropped square root, a signed maximum or a
    wrong node count gives a different number."""
    ref = np.array([[3.0, 0.0, 4.0], [0.0, 12.0, 0.0]])
    d = np.array([[-4.0, 2.0, 1.0], [2.0, 0.0, 0.0]])
    num = ref + d
    assert O.l2_rel_error(num, ref) == 5.0 / 13.0
    assert O.max_abs_error(num, ref) == 4.0
    assert O.rms_error(num, ref) == math.sqrt(25.0 / 6.0)
    assert O.mass(num) == 20.0
    # the same pair swapped: the norm is taken over the second argument, the maximum is symmetric
    assert O.l2_rel_error(ref, num) == 5.0 / math.sqrt(178.0)
    assert O.max_abs_error(ref, num) == 4.0
    # a field equal to its reference has zero error; a zero field has relative error 1
    assert O.l2_rel_error(ref, ref) == 0.0 and O.max_abs_error(ref, ref) == 0.0
    assert O.l2_rel_error(np.zeros_like(ref), ref) == 1.0
    # correctly rounded sums: cancelling magnitudes that a naive float sum loses
    big = np.array([1e16, 1.0, -1e16, 1.0])
    assert O.mass(big) == 2.0
    assert O.l2_rel_error(np.array([1e8 + 3.0, 4.0]), np.array([1e8, 0.0])) == 5.0 / 1e8


# ---- P2: equilibrium moments (Sec. 2.2, Eq. (6)) ----------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 4.0)
    cs2 = c * c / 3
    phi = rng.uniform(0.1, 2.0)
    ux, uy = rng.uniform(-0.3, 0.3, 2) * c
    geq = O.equilibrium(phi, ux, uy, c)
    ex, ey, _ = _E(c)
    tol = 1e-12 * phi * c ** 4
    assert abs(geq.sum() - phi) < 1e-14
    assert abs((ex * geq).sum() - phi * ux) < tol
    assert abs((ey * geq).sum() - phi * uy) < tol
    assert abs((ex * ex * geq).sum() - (phi * ux * ux + cs2 * phi)) < tol
    assert abs((ey * ey * geq).sum() - (phi * uy * uy + cs2 * phi)) < tol
    assert abs((ex * ey * geq).sum() - phi * ux * uy) < tol
    # third order: the mixed moments are those of the continuous equilibrium (they need the
    # third-order Hermite term) ...
    assert abs((ex * ex * ey * geq).sum() - (cs2 * phi * uy + phi * ux * ux * uy)) < tol
    assert abs((ex * ey * ey * geq).sum() - (cs2 * phi * ux + phi * ux * uy * uy)) < tol
    # ... while e_x^3 = c^2 e_x on D2Q9 caps the diagonal one (the known lattice defect)
    assert abs((ex ** 3 * geq).sum() - 3 * cs2 * phi * ux) < tol


# ---- P3: TRT-R collision in moment space (Sec. 2.2, Eqs. (8), (12), (13)) ---------------------

def _moments9(f, ex, ey):
    return np.array([f.sum(), (ex * f).sum(), (ey * f).sum(), (ex * ex * f).sum(), (ey * ey * f).sum(),
                     (ex * ey * f).sum(), (ex * ex * ey * f).sum(), (ex * ey * ey * f).sum(),
                     (ex * ex * ey * ey * f).sum()])


def _expected_post_moments(phi, j, Pi, ux, uy, om1, om2, cs2, s_eff=0.0, V=(0.0, 0.0), om3=0.0, B3=(0.0, 0.0)):
    """All nine raw moments of the post-collision (plus source/aux) populations, from the
    orthogonality of the Hermite basis on D2Q9: the zeroth moment is conserved (plus the source),
    the first relaxes with 1 - 1/tau1, the second Hermite moment with 1 - 1/tau2, the third Hermite
    moments (xxy, xyy) with 1 - 1/tau3 (0 for TRT-R: B3 is the third-order non-equilibrium moment),
    and the fourth-order moment follows from the equilibrium and the projected parts."""
    u = np.array([ux, uy])
    B = j - phi * u
    N = Pi - cs2 * phi * np.eye(2) - phi * np.outer(u, u)
    m0 = phi + s_eff
    m1 = phi * u + om1 * B + np.asarray(V)
    H2 = phi * np.outer(u, u) + om2 * N
    m2 = H2 + cs2 * m0 * np.eye(2)
    mxxy = cs2 * phi * uy + phi * ux * ux * uy + om1 * cs2 * B[1] + cs2 * V[1] + om3 * B3[0]
    mxyy = cs2 * phi * ux + phi * ux * uy * uy + om1 * cs2 * B[0] + cs2 * V[0] + om3 * B3[1]
    mxxyy = phi * cs2 * (cs2 + ux * ux + uy * uy) + om2 * cs2 * (N[0, 0] + N[1, 1]) + cs2 * cs2 * s_eff
    return np.array([m0, m1[0], m1[1], m2[0, 0], m2[1, 1], m2[0, 1], mxxy, mxyy, mxxyy])


@pytest.mark.parametrize("seed", [3, 4, 5, 6])
def test_collision_moments(seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 4.0)
    cs2 = c * c / 3
    g = rng.uniform(0.0, 0.3, 9)
    ux, uy = rng.uniform(-0.3, 0.3, 2) * c
    tau1, tau2 = rng.uniform(0.51, 2.0, 2)
    C = O.collide(g, ux, uy, tau1, tau2, c)
    ex, ey, _ = _E(c)
    phi = g.sum()
    j = np.array([(ex * g).sum(), (ey * g).sum()])
    Pi = np.array([[(ex * ex * g).sum(), (ex * ey * g).sum()], [(ex * ey * g).sum(), (ey * ey * g).sum()]])
    want = _expected_post_moments(phi, j, Pi, ux, uy, 1 - 1 / tau1, 1 - 1 / tau2, cs2)
    got = _moments9(C, ex, ey)
    scale = np.array([1, c, c, c * c, c * c, c * c, c ** 3, c ** 3, c ** 4])
    np.testing.assert_allclose(got / scale, want / scale, rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_mrt_collision_moments(seed):
    """MRT-R (Eq. (11) to third order): the third Hermite moments relax with 1 - 1/tau3 from their
    equilibrium values phi u_x^2 u_y, phi u_x u_y^2, by B_xxy = sum (e_x^2 e_y - cs2 e_y) g - phi u_x^2 u_y
    (and likewise xyy); every other moment is that of TRT-R; tau3 = 1 is TRT-R exactly."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 4.0)
    cs2 = c * c / 3
    g = rng.uniform(0.0, 0.3, 9)
    ux, uy = rng.uniform(-0.3, 0.3, 2) * c
    tau1, tau2, tau3 = rng.uniform(0.51, 2.0, 3)
    C = O.collide_mrt(g, ux, uy, tau1, tau2, tau3, c)
    ex, ey, _ = _E(c)
    phi = g.sum()
    j = np.array([(ex * g).sum(), (ey * g).sum()])
    Pi = np.array([[(ex * ex * g).sum(), (ex * ey * g).sum()], [(ex * ey * g).sum(), (ey * ey * g).sum()]])
    B3 = ((ex * ex * ey * g).sum() - cs2 * j[1] - phi * ux * ux * uy,
          (ex * ey * ey * g).sum() - cs2 * j[0] - phi * ux * uy * uy)
    want = _expected_post_moments(phi, j, Pi, ux, uy, 1 - 1 / tau1, 1 - 1 / tau2, cs2, om3=1 - 1 / tau3, B3=B3)
    got = _moments9(C, ex, ey)
    scale = np.array([1, c, c, c * c, c * c, c * c, c ** 3, c ** 3, c ** 4])
    np.testing.assert_allclose(got / scale, want / scale, rtol=0, atol=1e-13)
    assert np.array_equal(O.collide_mrt(g, ux, uy, tau1, tau2, 1.0, c), O.collide(g, ux, uy, tau1, tau2, c))


def test_relaxation_pair():
    # kappa = (tau1 - 1/2) cs2 dt and Lambda = (tau1 - 1/2)(tau2 - 1/2) (Sec. 2.4)
    dx, dt, lam = 0.03, 0.002, 0.25
    cs2 = (dx / dt) ** 2 / 3
    for kappa in (1e-4, 1e-3, 0.05):
        t1, t2 = O.relaxation(kappa, dx, dt, lam)
        assert abs((t1 - 0.5) * cs2 * dt - kappa) < 1e-15 * max(1.0, kappa) * 10
        assert abs((t1 - 0.5) * (t2 - 0.5) - lam) < 1e-13


# ---- one step seen through its moments (Sec. 2.2, Eq. (14) with Eqs. (3), (16)) ----------------

@pytest.mark.parametrize("aux,boundary", [(O.AUX_LOCAL, O.BC_PERIODIC), (O.AUX_NONE, O.BC_PERIODIC),
                                          (O.AUX_LOCAL, O.BC_NEE), (O.AUX_LOCAL, O.BC_WALLS)])
def test_step_moments_with_source_and_aux(aux, boundary):
    """Un-stream one oracle step and check all nine moments of P_i at every node away from the
    periodic seam (periodic), at every node including the edges (Dirichlet edges, where the
    derivative across the edge is one-sided), or on every row (walls: a population that crossed a
    wall came back as -P_i + 2 g_eq^+(phi_w), which the test inverts with g_eq from the oracle's
    equilibrium).  With the solid-body rotation u = (-U0 y, U0 x) both differences are exact, so
    u_b d_b u_a is the closed form (-U0^2 x, -U0^2 y) (centripetal)."""
    n = 12
    U0 = 1.3
    X, Y, dx = W.mesh(n, n, -1.0, 1.0)
    dt = dx / 3.0
    c = dx / dt
    cs2 = c * c / 3
    lam = 0.3
    rng = np.random.default_rng(11)
    D = 1e-3 * (1 + 0.5 * rng.uniform(-1, 1, (n, n)))
    ux, uy = -U0 * Y, U0 * X
    g = rng.uniform(0.0, 0.2, (9, n, n))
    S = rng.uniform(-1, 1, (n, n))
    dS = rng.uniform(-1, 1, (n, n))
    p = O.Problem(n, n, dx, dt, lam, 0.0, aux, boundary)
    phi_w = rng.uniform(0.2, 0.8, (n, n))
    out = O.step(p, g, ux, uy, D, S, dS, phi_b=phi_w if boundary == O.BC_WALLS else None)
    ex, ey, _ = _E(1.0)
    P = np.empty_like(out)
    for i in range(9):  # P_i(x) = g_i^{n+1}(x + e_i dt)
        P[i] = np.roll(out[i], shift=(-int(ey[i]), -int(ex[i])), axis=(0, 1))
    if boundary == O.BC_WALLS:
        opp = [int(np.flatnonzero((ex == -ex[i]) & (ey == -ey[i]))[0]) for i in range(9)]
        for k in (0, n - 1):
            for jx in range(n):
                ge = O.equilibrium(phi_w[k, jx], ux[k, jx], uy[k, jx], c)
                for i in range(9):
                    if (k == 0 and ey[i] < 0) or (k == n - 1 and ey[i] > 0):
                        P[i, k, jx] = -out[opp[i], k, jx] + ge[i] + ge[opp[i]]
    Ec = _E(c)
    nodes = range(n) if boundary == O.BC_NEE else range(1, n - 1)
    rows = range(n) if boundary in (O.BC_NEE, O.BC_WALLS) else range(1, n - 1)
    for k in rows:
        for jx in nodes:
            gl = g[:, k, jx]
            phi = gl.sum()
            j = np.array([(Ec[0] * gl).sum(), (Ec[1] * gl).sum()])
            Pi = np.array([[(Ec[0] ** 2 * gl).sum(), (Ec[0] * Ec[1] * gl).sum()],
                           [(Ec[0] * Ec[1] * gl).sum(), (Ec[1] ** 2 * gl).sum()]])
            tau1 = 0.5 + D[k, jx] / (cs2 * dt)
            tau2 = 0.5 + lam / (tau1 - 0.5)
            beta = 1 - 1 / (2 * tau1)
            s_eff = dt * S[k, jx] + 0.5 * dt * dt * dS[k, jx]
            u = np.array([ux[k, jx], uy[k, jx]])
            acc = np.array([-U0 * U0 * X[k, jx], -U0 * U0 * Y[k, jx]]) if aux == O.AUX_LOCAL else np.zeros(2)
            V = dt * beta * phi * acc + beta * u * s_eff
            want = _expected_post_moments(phi, j, Pi, u[0], u[1], 1 - 1 / tau1, 1 - 1 / tau2, cs2, s_eff, V)
            got = _moments9(P[:, k, jx], *Ec[:2])
            scale = np.array([1, c, c, c * c, c * c, c * c, c ** 3, c ** 3, c ** 4])
            np.testing.assert_allclose(got / scale, want / scale, rtol=0, atol=2e-13)


def test_uniform_state_step_is_the_collision():
    """A spatially uniform state with constant u and D streams onto itself: one step equals the
    collision, with tau1 from kappa and tau2 from Lambda."""
    n, dx, dt, lam, kappa = 5, 0.1, 0.01, 0.2, 0.02
    c = dx / dt
    rng = np.random.default_rng(7)
    g0 = rng.uniform(0.01, 0.2, 9)
    ux, uy = 0.1 * c, -0.05 * c
    g = np.broadcast_to(g0[:, None, None], (9, n, n)).copy()
    p = O.Problem(n, n, dx, dt, lam, kappa, O.AUX_LOCAL)
    out = O.step(p, g, ux, uy)
    t1, t2 = O.relaxation(kappa, dx, dt, lam)
    C = O.collide(g0, ux, uy, t1, t2, c)
    np.testing.assert_allclose(out, np.broadcast_to(C[:, None, None], out.shape), rtol=0, atol=1e-15)


# ---- P4 / P5 / P6: invariants -----------------------------------------------------------------

@pytest.mark.parametrize("aux", [O.AUX_LOCAL, O.AUX_FLUX])
def test_mass_conservation(aux):
    cfg = W.PulseConfig(N=32, steps=100, D_variable=True)
    f = W.rotating_pulse(cfg)
    p = O.Problem(32, 32, f["dx"], f["dt"], f["lam"], cfg.D, aux)
    g = O.init(p, f["phi0"], f["ux"], f["uy"])
    m0 = O.mass(O.phi(p, g))
    g = O.run(p, g, cfg.steps, f["ux"], f["uy"], f["D"])
    assert abs(O.mass(O.phi(p, g)) - m0) < 1e-13 * abs(m0)


def test_step_is_affine():
    n = 8
    X, Y, dx = W.mesh(n, n, -1.0, 1.0)
    rng = np.random.default_rng(21)
    p = O.Problem(n, n, dx, dx / 2.0, 0.25, 3e-3, O.AUX_LOCAL)
    ux, uy = rng.uniform(-0.5, 0.5, (2, n, n))
    g, h = rng.uniform(0, 1, (2, 9, n, n))
    a = 0.37
    lhs = O.step(p, a * g + (1 - a) * h, ux, uy)
    rhs = a * O.step(p, g, ux, uy) + (1 - a) * O.step(p, h, ux, uy)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14)
    S = rng.uniform(-1, 1, (n, n))
    lhs = O.step(p, a * g + (1 - a) * h, ux, uy, None, S, S)
    rhs = a * O.step(p, g, ux, uy, None, S, S) + (1 - a) * O.step(p, h, ux, uy, None, S, S)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14)


# velocity index after a +90 degree rotation of the lattice, derived from the oracle's own order
def _rot_perm():
    ex, ey, _ = O.lattice()
    idx = {(int(ex[i]), int(ey[i])): i for i in range(9)}
    return [idx[(-int(ey[i]), int(ex[i]))] for i in range(9)]


def _rot_field(f):
    # node (j, k) -> (-k, j) on an n x n periodic lattice centred on index 0: new[k', j'] = f[k, j]
    n = f.shape[-1]
    out = np.empty_like(f)
    for k in range(n):
        for j in range(n):
            out[..., j % n, (-k) % n] = f[..., k, j]
    return out


@pytest.mark.parametrize("aux", [O.AUX_LOCAL, O.AUX_FLUX])
def test_rotation_and_shift_covariance(aux):
    """Rotating the lattice by 90 degrees (populations relabelled, u rotated as a vector, D and S
    moved as scalars) commutes with one step; so does a periodic shift."""
    n = 7
    rng = np.random.default_rng(5)
    p = O.Problem(n, n, 0.1, 0.02, 0.25, 0.0, aux)
    g = rng.uniform(0, 1, (9, n, n))
    ux, uy = rng.uniform(-1, 1, (2, n, n))
    D = rng.uniform(1e-3, 5e-3, (n, n))
    S = rng.uniform(-1, 1, (n, n))
    perm = _rot_perm()
    out = O.step(p, g, ux, uy, D, S, S)
    g_r = np.empty_like(g)
    out_r = np.empty_like(out)
    for i in range(9):
        g_r[perm[i]] = _rot_field(g[i])
        out_r[perm[i]] = _rot_field(out[i])
    ux_r, uy_r = _rot_field(-uy), _rot_field(ux)
    got = O.step(p, g_r, ux_r, uy_r, _rot_field(D), _rot_field(S), _rot_field(S))
    np.testing.assert_allclose(got, out_r, rtol=0, atol=1e-13)
    sh = (2, -3)
    got = O.step(p, np.roll(g, sh, (1, 2)), np.roll(ux, sh, (0, 1)), np.roll(uy, sh, (0, 1)),
                 np.roll(D, sh, (0, 1)), np.roll(S, sh, (0, 1)), np.roll(S, sh, (0, 1)))
    np.testing.assert_allclose(got, np.roll(out, sh, (1, 2)), rtol=0, atol=1e-13)


# ---- P7 / P8: closed forms and convergence ----------------------------------------------------

def test_nee_edge_moments():
    """apply_nee rebuilds each edge node from its inward neighbour x_f (diagonal at a corner): the
    new node carries phi = phi_b and j = phi_b u_b + (j_f - phi_f u_f), because g_eq carries the
    moments phi and phi u; interior nodes are untouched.  Checked with x_f found independently."""
    nx, ny = 7, 6
    X, Y, dx = W.mesh(nx, ny, -1.0, 1.0)
    dt = dx / 3.0
    c = dx / dt
    rng = np.random.default_rng(17)
    g = rng.uniform(0.0, 0.2, (9, ny, nx))
    ux = c * rng.uniform(-0.1, 0.1, (ny, nx))
    uy = c * rng.uniform(-0.1, 0.1, (ny, nx))
    phi_b = rng.uniform(0.5, 1.5, (ny, nx))
    p = O.Problem(nx, ny, dx, dt, 0.25, 1e-3, O.AUX_LOCAL, O.BC_NEE)
    out = O.apply_nee(p, g, ux, uy, phi_b)
    Ec = _E(c)
    for y in range(ny):
        for x in range(nx):
            if 0 < x < nx - 1 and 0 < y < ny - 1:
                assert np.array_equal(out[:, y, x], g[:, y, x])
                continue
            xf = 1 if x == 0 else (nx - 2 if x == nx - 1 else x)
            yf = 1 if y == 0 else (ny - 2 if y == ny - 1 else y)
            gf = g[:, yf, xf]
            phif = gf.sum()
            jf = np.array([(Ec[0] * gf).sum(), (Ec[1] * gf).sum()])
            got = out[:, y, x]
            assert abs(got.sum() - phi_b[y, x]) < 1e-14
            want_j = phi_b[y, x] * np.array([ux[y, x], uy[y, x]]) + jf - phif * np.array([ux[yf, xf], uy[yf, xf]])
            np.testing.assert_allclose([(Ec[0] * got).sum(), (Ec[1] * got).sum()], want_j, rtol=0, atol=1e-13 * c)


def test_nee_equilibrium_is_a_fixed_point():
    """A state at equilibrium everywhere, with phi_b equal to its own phi, is left unchanged."""
    n = 6
    X, Y, dx = W.mesh(n, n, -1.0, 1.0)
    dt = dx / 4.0
    rng = np.random.default_rng(19)
    phi = rng.uniform(0.5, 1.5, (n, n))
    ux, uy = -2.0 * Y, 1.5 * X
    p = O.Problem(n, n, dx, dt, 0.25, 1e-3, O.AUX_LOCAL, O.BC_NEE)
    g = O.init(p, phi, ux, uy)
    np.testing.assert_allclose(O.apply_nee(p, g, ux, uy, phi), g, rtol=0, atol=1e-14)


# ---- walls by halfway anti-bounce-back; the slip-free free parameter (Sec. 3.3) -----------------

def _channel_error(tau1, tau2, ny=12, nx=3, phi_bot=0.3, phi_top=0.7, S0=2e-3):
    """Steady diffusion across a channel with walls at y = -1/2 and y = ny - 1/2 (lattice units),
    wall values phi_bot / phi_top, uniform source S0, u = 0: the exact profile is
    phi = phi_bot + (phi_top - phi_bot) (y + 1/2) / ny + S0 / (2 kappa) (y + 1/2)(ny - 1/2 - y).
    Returns the relative RMS error of the converged oracle solution."""
    cs2 = 1.0 / 3.0
    kappa = (tau1 - 0.5) * cs2
    p = O.Problem(nx, ny, 1.0, 1.0, (tau1 - 0.5) * (tau2 - 0.5), kappa, O.AUX_LOCAL, O.BC_WALLS)
    z = np.zeros((ny, nx))
    pb = np.zeros((ny, nx))
    pb[0, :], pb[-1, :] = phi_bot, phi_top
    S = np.full((ny, nx), S0)
    g = O.init(p, np.full((ny, nx), 0.5), z, z)
    prev = None
    for _ in range(400):
        g = O.run(p, g, 2000, z, z, None, S, None, phi_b=pb)
        phi = O.phi(p, g)
        if prev is not None and np.abs(phi - prev).max() < 1e-15:
            break
        prev = phi
    y = np.arange(ny)[:, None] + 0.5
    exact = phi_bot + (phi_top - phi_bot) * y / ny + S0 / (2 * kappa) * y * (ny - y)
    return float(np.sqrt(np.mean((phi - exact) ** 2)) / np.abs(exact).max())


@pytest.mark.parametrize("tau1", [0.6, 0.8, 1.2])
def test_slip_free_relation_of_the_free_parameter(tau1):
    """The free relaxation time tau2 = 3(1 - 4 tau1) / (8(1 - 2 tau1)) of Sec. 3.3 (tau1 = 0.8 gives
    1.375) makes the halfway anti-bounce-back walls slip-free: the linear-plus-parabolic steady
    profile is reproduced to round-off, while tau2 off that value leaves an O(1e-4) wall error."""
    tau2 = 3 * (1 - 4 * tau1) / (8 * (1 - 2 * tau1))
    if tau1 == 0.8:
        assert abs(tau2 - 1.375) < 1e-15
    assert _channel_error(tau1, tau2) < 1e-12
    assert _channel_error(tau1, tau2 + 0.15) > 1e-5
    assert _channel_error(tau1, tau2 - 0.15) > 1e-5


# ---- P9 / P14: the paper's printed Table 2 ----------------------------------------------------

def test_table2_typo_reading():
    t = _table2()
    e20, e40, e60 = (_x1_error(N, 0.005, O.AUX_LOCAL) for N in (20, 40, 60))
    assert abs(e40 / t["printed_typo"]["E_r"] - 1) > 0.05
    assert abs(e40 / 3.741e-3 - 1) < 1e-3


def test_aux_term_matters():
    """Dropping G (or using the flux-difference reading) misses Table 2, by far more than its
    printed precision: the paper's claim that the space-derivative term improves accuracy."""
    t = _table2()
    want = t["E_r"]["0.05"][4]
    e_local = _x1_error(100, 0.05, O.AUX_LOCAL)
    e_none = _x1_error(100, 0.05, O.AUX_NONE)
    assert abs(e_local / want - 1) < 1e-3
    assert e_none > 1.05 * e_local


# ---- the flux-difference reading of the auxiliary term ----------------------------------------

def test_flux_reading_equals_local_for_uniform_phi():
    """For uniform phi and a divergence-free linear u, d_b(phi u_a u_b) - u_a d_b(phi u_b) equals
    phi u_b d_b u_a exactly with central differences, so both forms give the same step away from
    the periodic seam."""
    n = 10
    X, Y, dx = W.mesh(n, n, -1.0, 1.0)
    ux, uy = -2.0 * Y, 2.0 * X
    rng = np.random.default_rng(9)
    geq = O.equilibrium(0.7, 0.0, 0.0, 3.0)
    g = np.broadcast_to(geq[:, None, None], (9, n, n)).copy()
    p_l = O.Problem(n, n, dx, dx / 3.0, 0.25, 2e-3, O.AUX_LOCAL)
    p_f = O.Problem(n, n, dx, dx / 3.0, 0.25, 2e-3, O.AUX_FLUX)
    a = O.step(p_l, g, ux, uy)
    b = O.step(p_f, g, ux, uy)
    np.testing.assert_allclose(a[:, 2:-2, 2:-2], b[:, 2:-2, 2:-2], rtol=0, atol=1e-14)
    assert rng is not None


def test_flux_reading_converges_to_local():
    """The two forms differ at O(dx^2) on a smooth pulse."""
    diffs = []
    for N in (32, 64, 128):
        cfg = W.PulseConfig(N=N, steps=int(round(0.05 / ((2.0 / N) / 10.0))))
        f = W.rotating_pulse(cfg)
        out = []
        for aux in (O.AUX_LOCAL, O.AUX_FLUX):
            p = O.Problem(N, N, f["dx"], cfg.dt, cfg.lam, cfg.D, aux)
            g = O.run(p, O.init(p, f["phi0"], f["ux"], f["uy"]), cfg.steps, f["ux"], f["uy"])
            out.append(O.phi(p, g))
        diffs.append(O.rms_error(out[0], out[1]))
    orders = [math.log2(diffs[k] / diffs[k + 1]) for k in range(2)]
    assert all(o > 1.7 for o in orders), (diffs, orders)


# ---- the complex-step build ------------------------------------------------------------------

def test_complex_build_matches_real_and_fd():
    n = 6
    rng = np.random.default_rng(13)
    X, Y, dx = W.mesh(n, n, -1.0, 1.0)
    p = O.Problem(n, n, dx, dx / 4.0, 0.25, 0.0, O.AUX_LOCAL)
    ux, uy = -Y, X
    phi0 = np.exp(-(X ** 2 + Y ** 2) / 0.2)
    D = 2e-3 * (1 + 0.3 * rng.uniform(-1, 1, (n, n)))
    dD = rng.uniform(-1, 1, (n, n)) * 1e-3
    g0 = O.init(p, phi0, ux, uy)
    gr = O.run(p, g0, 5, ux, uy, D)
    gz = O.run(p, g0.astype(complex), 5, ux, uy, D.astype(complex))
    np.testing.assert_allclose(gz.real, gr, rtol=0, atol=1e-14)
    h = 1e-30
    gz = O.run(p, g0.astype(complex), 5, ux, uy, D + 1j * h * dD)
    deriv = gz.imag / h
    eps = 1e-4
    fd = (O.run(p, g0, 5, ux, uy, D + eps * dD) - O.run(p, g0, 5, ux, uy, D - eps * dD)) / (2 * eps)
    np.testing.assert_allclose(deriv, fd, rtol=0, atol=1e-8 * np.abs(deriv).max())


# ---- the slower convergence and Table 2 pins run last (the mutation check stops at the first failure)

def _x1_error(N, kappa, aux):
    f = W.x1_problem(N, kappa)
    p = O.Problem(N, N, f["dx"], f["dt"], f["lam"], kappa, aux)
    g = O.init(p, f["phi0"], f["ux"], f["uy"])
    for s in range(f["steps"]):
        S, dS = f["source"](s * f["dt"])
        g = O.step(p, g, f["ux"], f["uy"], None, S, dS)
    er = O.rms_error(O.phi(p, g), f["exact"](f["steps"] * f["dt"]))
    return er * N / (N + 1)  # E_r over the paper's (N+1)^2 nodes (fixture's normalisation note)


def _table2():
    with open(os.path.join(GOLDEN, "table2_present.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("kappa", ["0.005", "0.01", "0.05"])
def test_table2_present_column(kappa):
    """The oracle on a periodic proxy of the Sec. 3 benchmark reproduces every printed E_r of the
    'Present' column of Table 2 to its four printed digits, and the printed orders."""
    t = _table2()
    errs = [_x1_error(N, float(kappa), O.AUX_LOCAL) for N in t["N"]]
    for N, e, want in zip(t["N"], errs, t["E_r"][kappa]):
        assert abs(e / want - 1) < 1e-3, (N, e, want)
    for k in range(1, 5):
        order = math.log(errs[k - 1] / errs[k]) / math.log(t["N"][k] / t["N"][k - 1])
        assert abs(order - t["order"][kappa][k]) < 0.01, (k, order)


def _x1_error_dirichlet(N, kappa):
    """The benchmark on the paper's own grid: N + 1 nodes per axis, the closed form imposed on the
    four edges by non-equilibrium extrapolation before every step and before the final read-out."""
    f = W.x1_problem(N, kappa, dirichlet=True)
    n = f["nx"]
    p = O.Problem(n, n, f["dx"], f["dt"], f["lam"], kappa, O.AUX_LOCAL, O.BC_NEE)
    g = O.init(p, f["phi0"], f["ux"], f["uy"])
    for s in range(f["steps"]):
        t = s * f["dt"]
        g = O.apply_nee(p, g, f["ux"], f["uy"], f["exact"](t))
        S, dS = f["source"](t)
        g = O.step(p, g, f["ux"], f["uy"], None, S, dS)
    T = f["steps"] * f["dt"]
    g = O.apply_nee(p, g, f["ux"], f["uy"], f["exact"](T))
    return O.rms_error(O.phi(p, g), f["exact"](T))


@pytest.mark.parametrize("kappa", ["0.005", "0.01", "0.05"])
def test_table2_on_the_dirichlet_grid(kappa):
    """On the (N+1)^2 grid with Dirichlet edges the oracle reproduces the 'Present' column of
    Table 2 directly (no node-count factor) to its printed digits."""
    t = _table2()
    for N, want in zip(t["N"], t["E_r"][kappa]):
        e = _x1_error_dirichlet(N, float(kappa))
        assert abs(e / want - 1) < 1e-3, (N, e, want)


def _pulse_error(cfg):
    f = W.rotating_pulse(cfg)
    p = O.Problem(cfg.N, cfg.N, f["dx"], cfg.dt, cfg.lam, cfg.D, O.AUX_LOCAL)
    g = O.init(p, f["phi0"], f["ux"], f["uy"])
    g = O.run(p, g, cfg.steps, f["ux"], f["uy"], f["D"])
    return O.rms_error(O.phi(p, g), W.pulse_reference(cfg, f))


def test_heat_kernel_second_order():
    """u = 0: a Gaussian spreads as the heat kernel with kappa = (tau1 - 1/2) cs2 dt (Sec. 2.4).
    Diffusive scaling (tau1 fixed); the error must fall at second order."""
    errs = []
    for N in (32, 64, 128):
        dt = 0.00625 * (32 / N) ** 2
        cfg = W.PulseConfig(N=N, steps=int(round(0.1 / dt)), U0=0.0, D=1e-2, xc0=0.0, yc0=0.0,
                            dt_override=dt)
        errs.append(_pulse_error(cfg))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[0] < 3e-3
    assert all(1.8 < o < 2.2 for o in orders), (errs, orders)


def test_rotating_pulse_closed_form_second_order():
    """Solid-body rotation u = (-pi y, pi x), D = 1e-3, c = 10 (the 64^2 workload and two
    refinements), t = 0.125: converges to the closed form at second order."""
    errs = []
    for N in (64, 128, 256):
        dt = (2.0 / N) / 10.0
        cfg = W.PulseConfig(N=N, steps=int(round(0.125 / dt)))
        errs.append(_pulse_error(cfg))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[-1] < 4e-4
    assert all(1.7 < o < 2.2 for o in orders), (errs, orders)


# ---- Dirichlet edges by non-equilibrium extrapolation (the boundary scheme of Sec. 3) ----------


def test_threaded_oracle_is_bitwise_the_serial_one():
    """The OpenMP build (rows of a step over host threads), used for the all-cores CPU baseline and
    for stored expected values of large cases, gives exactly the single-threaded results."""
    cfg = W.PulseConfig(N=48, steps=12, D_variable=True)
    f = W.rotating_pulse(cfg)
    rng = np.random.default_rng(7)
    S = 0.1 * rng.uniform(-1, 1, (48, 48))
    for aux in (O.AUX_LOCAL, O.AUX_FLUX):
        p = O.Problem(48, 48, f["dx"], f["dt"], cfg.lam, cfg.D, aux)
        g0 = O.init(p, f["phi0"], f["ux"], f["uy"])
        a = O.run(p, g0, cfg.steps, f["ux"], f["uy"], D=f["D"], S=S, dSdt=-S)
        b, used = O.run_threads(p, g0, cfg.steps, f["ux"], f["uy"], D=f["D"], S=S, dSdt=-S, threads=4)
        assert used == 4
        assert np.array_equal(a, b)
