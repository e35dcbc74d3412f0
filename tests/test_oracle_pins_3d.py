"""Pins of the D3Q19 and D3Q27 FP64 oracles against what the mathematics fixes (CPU only): lattice
identities, Hermite moment identities of the equilibrium and of the TRT-R collision, one step seen
through its moments, mass conservation, invariance under a cyclic permutation of the axes (which
ties the velocity tables, the streaming and the auxiliary-term differences of all three axes
together), the closed-form decay and drift of a Fourier mode along z at second order, and, for
D3Q27 (the tensor product of D1Q3 with D2Q9), the reduction of a z-uniform state with u_z = 0 to
the two-dimensional oracle when the populations are summed over e_z."""
import math

import numpy as np
import pytest

import oracle as O

LATTICES = [19, 27]


def _E(q, c=1.0):
    ex, ey, ez, w = O.lattice3(q)
    return c * ex.astype(float), c * ey.astype(float), c * ez.astype(float), w


@pytest.mark.parametrize("q", LATTICES)
def test_lattice_identities(q):
    ex, ey, ez, w = _E(q)
    e = np.stack([ex, ey, ez])
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1) < 1e-15
    assert len({tuple(v) for v in e.T}) == q
    assert np.array_equal(e[:, 0], np.zeros(3))
    for i in range(1, q, 2):  # i and i + 1 (odd i) are opposite, the order the library's planes use
        assert np.array_equal(e[:, i + 1], -e[:, i])
        assert w[i] == w[i + 1]
    np.testing.assert_allclose(e @ w, 0, atol=1e-16)
    np.testing.assert_allclose((e * w) @ e.T, cs2 * np.eye(3), atol=1e-16)
    d = np.eye(3)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                assert abs((w * e[a] * e[b] * e[c]).sum()) < 1e-16
                for f in range(3):
                    m4 = (w * e[a] * e[b] * e[c] * e[f]).sum()
                    want = cs2 * cs2 * (d[a, b] * d[c, f] + d[a, c] * d[b, f] + d[a, f] * d[b, c])
                    assert abs(m4 - want) < 1e-16, (a, b, c, f)


def test_d3q27_is_the_tensor_product_of_d1q3():
    """Every moment factorises into one-dimensional D1Q3 moments (weights 2/3, 1/6, 1/6): m(0) = 1,
    m(odd) = 0, m(even > 0) = 1/3.  This fixes all 27 weights and velocities at once."""
    ex, ey, ez, w = _E(27)
    m = lambda p: 1.0 if p == 0 else (0.0 if p % 2 else 1.0 / 3.0)
    for a in range(5):
        for b in range(5):
            for c in range(5):
                got = (w * ex ** a * ey ** b * ez ** c).sum()
                assert abs(got - m(a) * m(b) * m(c)) < 4e-16, (a, b, c)


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_equilibrium_moments(q, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 3.0)
    cs2 = c * c / 3
    phi = rng.uniform(0.1, 2.0)
    u = rng.uniform(-0.3, 0.3, 3) * c
    geq = O.equilibrium3(phi, u, c, q)
    ex, ey, ez, _ = _E(q, c)
    e = np.stack([ex, ey, ez])
    tol = 1e-12 * phi * c ** 4
    assert abs(geq.sum() - phi) < 1e-14
    np.testing.assert_allclose(e @ geq, phi * u, atol=tol)
    np.testing.assert_allclose((e * geq) @ e.T, phi * np.outer(u, u) + cs2 * phi * np.eye(3), atol=tol)
    # e_x^3 = c^2 e_x on the lattice: the xxx moment is 3 c_s^2 phi u_x, missing phi u_x^3 (lattice defect)
    assert abs((ex ** 3 * geq).sum() - 3 * cs2 * phi * u[0]) < tol
    if q == 19:
        # no D3Q19 velocity has three non-zero components: the xyz moment is lost (lattice defect)
        assert abs((ex * ey * ez * geq).sum()) < tol
        # with u in the x-y plane the mixed third moments are those of the continuous equilibrium
        u2 = np.array([u[0], u[1], 0.0])
        g2 = O.equilibrium3(phi, u2, c, q)
        assert abs((ex * ex * ey * g2).sum() - (cs2 * phi * u2[1] + phi * u2[0] ** 2 * u2[1])) < tol
        assert abs((ex * ey * ey * g2).sum() - (cs2 * phi * u2[0] + phi * u2[0] * u2[1] ** 2)) < tol
    else:
        # D3Q27 carries every mixed third moment of the continuous equilibrium, for any u
        assert abs((ex * ey * ez * geq).sum() - phi * u[0] * u[1] * u[2]) < tol
        for a, b in ((0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)):
            got = (e[a] * e[a] * e[b] * geq).sum()
            assert abs(got - (cs2 * phi * u[b] + phi * u[a] ** 2 * u[b])) < tol, (a, b)


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("seed", [4, 5, 6])
def test_collision_moments(q, seed):
    """Moments 0-2 of the TRT-R collision: phi conserved, j relaxes with 1 - 1/tau1, the second
    Hermite moment with 1 - 1/tau2 (exact on both lattices by their fourth-order isotropy)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 3.0)
    cs2 = c * c / 3
    g = rng.uniform(0.0, 0.2, q)
    u = rng.uniform(-0.3, 0.3, 3) * c
    tau1, tau2 = rng.uniform(0.51, 2.0, 2)
    C = O.collide3(g, u, tau1, tau2, c)
    ex, ey, ez, _ = _E(q, c)
    e = np.stack([ex, ey, ez])
    phi, j, Pi = g.sum(), e @ g, (e * g) @ e.T
    N = Pi - cs2 * phi * np.eye(3) - phi * np.outer(u, u)
    tol = 1e-13
    assert abs(C.sum() - phi) < tol
    np.testing.assert_allclose((e @ C) / c, (phi * u + (1 - 1 / tau1) * (j - phi * u)) / c, atol=tol)
    want2 = phi * np.outer(u, u) + (1 - 1 / tau2) * N + cs2 * phi * np.eye(3)
    np.testing.assert_allclose(((e * C) @ e.T) / c ** 2, want2 / c ** 2, atol=tol)


def test_d3q27_collision_keeps_only_the_equilibrium_third_moments():
    """Regularisation drops all non-equilibrium content above second order, so the third-order
    Hermite moments (H_xyz, and H_xxy and the like) of the post-collision populations are those of
    g_eq(phi, u), phi u_a u_b u_c, whatever g carries."""
    rng = np.random.default_rng(17)
    c = 1.7
    cs2 = c * c / 3
    g = rng.uniform(0.0, 0.2, 27)
    u = rng.uniform(-0.3, 0.3, 3) * c
    C = O.collide3(g, u, 0.9, 1.3, c)
    phi = g.sum()
    ex, ey, ez, _ = _E(27, c)
    e = np.stack([ex, ey, ez])
    assert abs(ex * ey * ez @ C - phi * u[0] * u[1] * u[2]) < 1e-13 * c ** 3
    for a, b in ((0, 1), (1, 2), (2, 0), (1, 0)):
        H = e[a] * e[a] * e[b] - cs2 * e[b]
        assert abs(H @ C - phi * u[a] ** 2 * u[b]) < 1e-13 * c ** 3, (a, b)
    # the non-equilibrium part of g does reach the raw xxy moment through the relaxed first moment
    assert abs(ex * ex * ey @ C - (cs2 * (e @ C)[1] + phi * u[0] ** 2 * u[1])) < 1e-13 * c ** 3


def _mesh3(n, lo=-1.0, hi=1.0):
    dx = (hi - lo) / n
    x = lo + dx * np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z, dx


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("axis", ["z", "x"])
def test_step_moments_with_source_and_aux(q, axis):
    """Un-stream one step and check moments 0-2 of P_i at every node away from the periodic seam.
    Under a solid-body rotation about the z (or x) axis the central difference is exact, so
    u_b d_b u_a is the centripetal closed form."""
    n, U0 = 8 if q == 19 else 6, 1.1
    X, Y, Z, dx = _mesh3(n)
    dt = dx / 3.0
    c = dx / dt
    cs2 = c * c / 3
    lam = 0.3
    rng = np.random.default_rng(9)
    if axis == "z":
        u = np.stack([-U0 * Y, U0 * X, 0 * X])
        acc = np.stack([-U0 ** 2 * X, -U0 ** 2 * Y, 0 * X])
    else:
        u = np.stack([0 * X, -U0 * Z, U0 * Y])
        acc = np.stack([0 * X, -U0 ** 2 * Y, -U0 ** 2 * Z])
    D = 1e-3 * (1 + 0.5 * rng.uniform(-1, 1, X.shape))
    g = rng.uniform(0.0, 0.2, (q,) + X.shape)
    S = rng.uniform(-1, 1, X.shape)
    dS = rng.uniform(-1, 1, X.shape)
    p = O.Problem3(n, n, n, dx, dt, lam, 0.0, O.AUX_LOCAL, q)
    out = O.step3(p, g, u, D, S, dS)
    ex, ey, ez, _ = _E(q, 1.0)
    P = np.empty_like(out)
    for i in range(q):  # P_i(x) = g_i^{n+1}(x + e_i dt)
        P[i] = np.roll(out[i], shift=(-int(ez[i]), -int(ey[i]), -int(ex[i])), axis=(0, 1, 2))
    E = np.stack(_E(q, c)[:3])
    for l in range(1, n - 1):
        for k in range(1, n - 1):
            for jx in range(1, n - 1):
                gl = g[:, l, k, jx]
                phi, jv, Pi = gl.sum(), E @ gl, (E * gl) @ E.T
                tau1 = 0.5 + D[l, k, jx] / (cs2 * dt)
                tau2 = 0.5 + lam / (tau1 - 0.5)
                beta = 1 - 1 / (2 * tau1)
                s_eff = dt * S[l, k, jx] + 0.5 * dt * dt * dS[l, k, jx]
                un = u[:, l, k, jx]
                V = dt * beta * phi * acc[:, l, k, jx] + beta * un * s_eff
                N = Pi - cs2 * phi * np.eye(3) - phi * np.outer(un, un)
                Pl = P[:, l, k, jx]
                assert abs(Pl.sum() - (phi + s_eff)) < 2e-14
                np.testing.assert_allclose((E @ Pl) / c, (phi * un + (1 - 1 / tau1) * (jv - phi * un) + V) / c,
                                           atol=2e-14)
                want2 = phi * np.outer(un, un) + (1 - 1 / tau2) * N + cs2 * (phi + s_eff) * np.eye(3)
                np.testing.assert_allclose(((E * Pl) @ E.T) / c ** 2, want2 / c ** 2, atol=2e-14)


@pytest.mark.parametrize("q", LATTICES)
def test_mass_conservation(q):
    n = 6
    X, Y, Z, dx = _mesh3(n)
    rng = np.random.default_rng(3)
    u = 0.4 * rng.uniform(-1, 1, (3,) + X.shape)
    D = 2e-3 * (1 + 0.5 * rng.uniform(-1, 1, X.shape))
    p = O.Problem3(n, n, n, dx, dx / 2.0, 0.25, 0.0, O.AUX_LOCAL, q)
    g = O.init3(p, rng.uniform(0.5, 1.5, X.shape), u)
    m0 = math.fsum(O.phi3(p, g).ravel())
    g = O.run3(p, g, 10, u, D)
    assert abs(math.fsum(O.phi3(p, g).ravel()) - m0) < 1e-12 * m0


@pytest.mark.parametrize("q", LATTICES)
def test_cyclic_axis_permutation_covariance(q):
    """Relabel the axes (x, y, z) -> (z, x, y): arrays are transposed, velocity components and
    population indices permuted; one step must commute with the relabelling (random u, D, S)."""
    nx, ny, nz = 5, 6, 7
    rng = np.random.default_rng(12)
    sh = (nz, ny, nx)
    g = rng.uniform(0.0, 0.2, (q,) + sh)
    u = 0.3 * rng.uniform(-1, 1, (3,) + sh)
    D = 1e-3 * (1 + 0.5 * rng.uniform(-1, 1, sh))
    S = rng.uniform(-1, 1, sh)
    dx, dt, lam = 0.1, 0.05, 0.25
    p = O.Problem3(nx, ny, nz, dx, dt, lam, 0.0, O.AUX_LOCAL, q)
    out = O.step3(p, g, u, D, S)

    def T(f):  # new x = old y, new y = old z, new z = old x; array axes (z, y, x)
        return np.transpose(f, (2, 0, 1))

    ex, ey, ez, _ = O.lattice3(q)
    perm = [next(j for j in range(q) if (ex[j], ey[j], ez[j]) == (ey[i], ez[i], ex[i])) for i in range(q)]

    def Tpop(gg):
        r = np.empty((q,) + T(gg[0]).shape)
        for i in range(q):
            r[perm[i]] = T(gg[i])
        return r
    uT = np.stack([T(u[1]), T(u[2]), T(u[0])])
    pT = O.Problem3(ny, nz, nx, dx, dt, lam, 0.0, O.AUX_LOCAL, q)
    outT = O.step3(pT, Tpop(g), uT, T(D), T(S))
    np.testing.assert_allclose(outT, Tpop(out), rtol=0, atol=1e-15)


def test_d3q27_z_uniform_state_reduces_to_d2q9():
    """D3Q27 is D2Q9 x D1Q3.  For a state uniform in z with u_z = 0 (and z-independent u, D, S),
    summing the populations of one step over e_z gives exactly the two-dimensional oracle's step of
    the summed state: the third-order equilibrium, the regularised non-equilibrium, the auxiliary
    term, the source and the streaming all reduce.  The populations themselves are random, so each
    e_z layer is different."""
    nx, ny, nz = 7, 6, 3
    rng = np.random.default_rng(31)
    dx, dt, lam = 0.1, 0.05, 0.25
    g2 = rng.uniform(0.0, 0.2, (27, ny, nx))
    g = np.ascontiguousarray(np.broadcast_to(g2[:, None], (27, nz, ny, nx)))
    ux, uy = 0.3 * rng.uniform(-1, 1, (2, ny, nx))
    D = 1e-3 * (1 + 0.5 * rng.uniform(-1, 1, (ny, nx)))
    S = rng.uniform(-1, 1, (ny, nx))
    dS = rng.uniform(-1, 1, (ny, nx))
    u = np.stack([np.broadcast_to(ux, (nz, ny, nx)), np.broadcast_to(uy, (nz, ny, nx)), np.zeros((nz, ny, nx))])
    b = lambda f: np.broadcast_to(f, (nz, ny, nx))
    p3 = O.Problem3(nx, ny, nz, dx, dt, lam, 0.0, O.AUX_LOCAL, 27)
    out3 = O.step3(p3, g, u, b(D), b(S), b(dS))

    ex, ey, ez, _ = O.lattice3(27)
    ex2, ey2, _ = O.lattice()
    to2 = [next(k for k in range(9) if (ex2[k], ey2[k]) == (ex[i], ey[i])) for i in range(27)]

    def marg(gg):
        m = np.zeros((9,) + gg.shape[1:])
        for i in range(27):
            m[to2[i]] += gg[i]
        return m
    p2 = O.Problem(nx, ny, dx, dt, lam, 0.0, O.AUX_LOCAL)
    out2 = O.step(p2, marg(g2), ux, uy, D, S, dS)
    for z in range(nz):
        np.testing.assert_allclose(marg(out3[:, z]), out2, rtol=0, atol=1e-15)


def _mode_error(q, N, axis_u=0.0):
    """A Fourier mode along z on a 3 x 3 x N lattice, u = (0, 0, U): phi = 1 + a sin(k(z - U t))
    exp(-kappa k^2 t), exact for the advection-diffusion equation; diffusive scaling."""
    L, kappa, a = 1.0, 0.02, 0.5
    dx = L / N
    dt = 2.0 * dx * dx  # dx^2/dt fixed: tau1 = 1/2 + 3 kappa dt / dx^2 = 0.62 on every grid
    steps = int(round(0.05 / dt))
    k = 2 * math.pi / L
    z = dx * np.arange(N)
    sh = (N, 3, 3)
    Zg = np.broadcast_to(z[:, None, None], sh)
    u = np.zeros((3,) + sh)
    u[2] = axis_u
    p = O.Problem3(3, 3, N, dx, dt, 1.0 / 6.0, kappa, O.AUX_LOCAL, q)
    g = O.init3(p, 1 + a * np.sin(k * Zg), u)
    g = O.run3(p, g, steps, u)
    t = steps * dt
    exact = 1 + a * np.sin(k * (Zg - axis_u * t)) * math.exp(-kappa * k * k * t)
    return float(np.sqrt(np.mean((O.phi3(p, g) - exact) ** 2)))


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("U", [0.0, 0.4])
def test_fourier_mode_along_z_second_order(q, U):
    errs = [_mode_error(q, N, U) for N in (16, 32, 64)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 4e-4  # amplitude 0.5
    assert all(1.8 < o < 2.3 for o in orders), (errs, orders)


def test_problem_rejects_other_lattices():
    with pytest.raises(ValueError):
        O.Problem3(3, 3, 3, 0.1, 0.1, 0.25, q=15)
    p = O.Problem3(3, 3, 3, 0.1, 0.1, 0.25, 1e-3, q=27)
    with pytest.raises(ValueError):
        O.phi3(p, np.zeros((19, 3, 3, 3)))
