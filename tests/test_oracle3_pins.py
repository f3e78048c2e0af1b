"""Pins of the three-dimensional oracle (oracle/rd3_oracle.cpp) against what
the mathematics fixes: K(n) equals the Jacobian of the Euler flux along n
(complex step), K+ + K- = K with K+ K- = 0 and the right eigenvalues; the
tetrahedron residual equals the exact surface integral of the flux when Z is
linear (edge-midpoint quadrature, exact for the quadratic flux); the N and
LDA parts add up to the residual; a supersonic tetrahedron sends everything
to its one downstream corner; uniform states are steady; periodic boxes
conserve mass, momentum and energy; the CFL limit has its closed form on
the regular box; stored normals point inwards and a bounded box's residual
total is its boundary flux; RK2 with the N scheme is Heun's method (two
forward Euler steps averaged with the start)."""
import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I

G = 1.4


@pytest.fixture(scope="module")
def O():
    import oracle3
    oracle3.build(force=False)
    return oracle3


def flux_n(W, n, gamma=G):
    """Euler flux along n (not necessarily unit) of W [5] (complex allowed)."""
    rho, m = W[0], W[1:4]
    u = m / rho
    p = (gamma - 1.0) * (W[4] - 0.5 * rho * np.sum(u * u))
    un = np.sum(u * n)
    return np.concatenate([[rho * un], m * un + p * n, [(W[4] + p) * un]])


def w_from_z(Z, gamma=G):
    rho = Z[0] * Z[0]
    u = Z[1:4] / Z[0]
    h = Z[4] / Z[0]
    p = (gamma - 1.0) / gamma * (rho * h - 0.5 * rho * np.sum(u * u))
    return np.concatenate([[rho], rho * u, [rho * h - p]])


def z_from_w(W, gamma=G):
    rho = W[0]
    u = W[1:4] / rho
    p = (gamma - 1.0) * (W[4] - 0.5 * rho * np.sum(u * u))
    s = np.sqrt(rho)
    return np.concatenate([[s], s * u, [s * (W[4] + p) / rho]])


def random_state(rng, mach=0.5):
    rho = 0.5 + rng.random()
    p = 0.5 + rng.random()
    c = np.sqrt(G * p / rho)
    u = rng.normal(size=3)
    u *= mach * c / np.linalg.norm(u)
    return I.prim_to_cons3(np.array([rho]), u[0], u[1], u[2], p)[:, 0]


def random_tet(rng):
    while True:
        p = rng.random((4, 3))
        vol = np.dot(p[1] - p[0], np.cross(p[2] - p[0], p[3] - p[0])) / 6
        if abs(vol) > 0.02:
            if vol < 0:
                p[[1, 2]] = p[[2, 1]]
            return p


def test_k_is_the_flux_jacobian(O):
    rng = np.random.default_rng(1)
    for mach in (0.3, 0.9, 2.5):
        for _ in range(5):
            W = random_state(rng, mach)
            n = rng.normal(size=3)
            J = np.zeros((5, 5))
            for q in range(5):
                Wc = W.astype(complex)
                Wc[q] += 1e-30j
                J[:, q] = flux_n(Wc, n).imag / 1e-30
            K, Kp, Km = O.kmat(W, n, G)
            assert np.abs(K - J).max() <= 1e-12 * np.abs(J).max()
            assert np.abs(Kp + Km - K).max() <= 1e-12 * np.abs(J).max()
            assert np.abs(Kp @ Km).max() <= 1e-11 * np.abs(J).max() ** 2
            rho = W[0]
            u = W[1:4] / rho
            c = np.sqrt(G * (G - 1) * (W[4] / rho - 0.5 * u @ u))
            nn = np.linalg.norm(n)
            lam = np.sort(nn * (u @ n / nn + np.array([-c, 0, 0, 0, c])))
            assert np.allclose(np.sort(np.linalg.eigvals(K).real), lam, rtol=1e-9, atol=1e-9)
            assert np.allclose(np.sort(np.linalg.eigvals(Kp).real), np.maximum(lam, 0), atol=1e-9)


def test_residual_is_the_surface_integral(O):
    """phi^T = integral over the boundary of F(Z) . n_out dS with Z linear in
    the tetrahedron: F is quadratic in Z, so the three-edge-midpoint rule on
    each face is exact."""
    rng = np.random.default_rng(2)
    for _ in range(10):
        p = random_tet(rng)
        W4 = np.stack([random_state(rng, 0.7) for _ in range(4)])
        Z4 = np.stack([z_from_w(w) for w in W4])
        total = np.zeros(5)
        for i in range(4):
            j, k, l = [q for q in range(4) if q != i]
            n = 0.5 * np.cross(p[k] - p[j], p[l] - p[j])
            if np.dot(n, p[i] - p[j]) > 0:
                n = -n  # outward
            for a, b in ((j, k), (k, l), (l, j)):
                total += flux_n(w_from_z(0.5 * (Z4[a] + Z4[b])), n) / 3.0
        r = O.tet(W4, p, G, O.B)
        assert np.abs(r["phiT"] - total).max() <= 1e-12 * np.abs(total).max()
        # every scheme splits the same residual
        for s in (O.N, O.LDA, O.B, O.BMAX, O.BMIN):
            q = O.tet(W4, p, G, s)
            assert np.abs(q["phi"].sum(axis=0) - q["phiT"]).max() <= 1e-12 * np.abs(q["phiT"]).max()
        assert np.all((r["theta"] >= 0) & (r["theta"] <= 1))


def test_supersonic_tetrahedron_is_fully_upwind(O):
    """With the flow supersonic and pointing at one corner, every other
    corner sees only outgoing characteristics (K_i^+ = 0) and all parts
    go to the downstream corner, for every scheme."""
    p = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    centroid = p.mean(axis=0)
    rng = np.random.default_rng(3)
    for down in range(4):
        d = p[down] - centroid
        d /= np.linalg.norm(d)
        W4 = []
        for _ in range(4):
            rho, pr = 1 + 0.05 * rng.random(), 1 + 0.05 * rng.random()
            u = 8.0 * np.sqrt(G * pr / rho) * d
            W4.append(I.prim_to_cons3(np.array([rho]), u[0], u[1], u[2], pr)[:, 0])
        W4 = np.stack(W4)
        for s in (O.N, O.LDA, O.B):
            r = O.tet(W4, p, G, s)
            scale = np.abs(r["phiT"]).max()
            others = [i for i in range(4) if i != down]
            assert np.abs(r["phi"][others]).max() <= 1e-11 * scale
            assert np.abs(r["phi"][down] - r["phiT"]).max() <= 1e-11 * scale


def test_uniform_states_are_steady_and_boxes_conserve(O):
    m = I.cube_tets(5, jitter=0.25, seed=4)
    om = O.OracleMesh3(m)
    _, _, _, V = om.geometry()
    U = I.ic3_uniform(m, 1.3, 0.4, -0.3, 0.2, 0.8)
    for s in (O.N, O.LDA, O.B):
        assert np.abs(om.residual(U, s)).max() <= 1e-13
    W = I.ic3_random_smooth(m, seed=5)
    dt = om.max_dt(W, 0.4)
    for s in (O.N, O.LDA, O.B, O.BMAX, O.BMIN):
        for order in (1, 2):
            W1 = om.step(W, dt, s, order)
            assert np.abs((W1 - W) @ V).max() <= 1e-14 * 10
            assert np.abs(W1 - W).max() > 1e-4  # something happened


def test_geometry_and_cfl_closed_forms(O):
    """Regular periodic box of N^3 cells, h = 1/N: every tetrahedron has volume
    h^3 / 6, every vertex volume h^3, inward normals summing to zero; with a
    uniform state the CFL limit is h / (4 sqrt 2 (|u| + c)) per unit CFL number
    (24 tetrahedra per vertex, largest face area h^2 / sqrt 2)."""
    N = 4
    m = I.cube_tets(N)
    om = O.OracleMesh3(m)
    vol, nrm, smax, V = om.geometry()
    h = 1.0 / N
    assert np.allclose(vol, h ** 3 / 6, rtol=1e-14)
    assert np.allclose(V, h ** 3, rtol=1e-14)
    assert np.abs(nrm.sum(axis=1)).max() <= 1e-16
    assert np.allclose(smax, h * h / np.sqrt(2), rtol=1e-14)
    rho, u, p = 1.1, np.array([0.3, -0.4, 0.2]), 0.9
    U = I.ic3_uniform(m, rho, *u, p)
    lam = np.linalg.norm(u) + np.sqrt(G * p / rho)
    assert om.max_dt(U, 0.5) == pytest.approx(0.5 * h / (4 * np.sqrt(2) * lam), rel=1e-13)


def test_inward_normals_and_mesh_residual_total(O):
    """Each stored face normal points towards its own corner, and on a
    bounded box the sum of the vertex residuals (all interior faces cancel)
    equals the sum over tetrahedra of the exact surface integrals of the
    flux with Z linear (edge-midpoint quadrature)."""
    m = I.cube_tets(2, periodic=(False, False, False), jitter=0.2, seed=21)
    om = O.OracleMesh3(m)
    _, nrm, _, _ = om.geometry()
    P = np.stack([m["x"], m["y"], m["z"]], axis=1)
    for t, corners in enumerate(m["tet"]):
        for i in range(4):
            face = [corners[q] for q in range(4) if q != i]
            assert np.dot(nrm[t, i], P[corners[i]] - P[face].mean(axis=0)) > 0
    W = I.ic3_random_smooth(m, seed=22, amp=0.2)
    R = om.residual(W, O.N)
    Z = np.stack([z_from_w(W[:, v]) for v in range(m["nv"])])
    total = np.zeros(5)
    for corners in m["tet"]:
        p = P[corners]
        for i in range(4):
            j, k, l = [corners[q] for q in range(4) if q != i]
            n = 0.5 * np.cross(P[k] - P[j], P[l] - P[j])
            if np.dot(n, p[i] - P[j]) > 0:
                n = -n
            for a, b in ((j, k), (k, l), (l, j)):
                total += flux_n(w_from_z(0.5 * (Z[a] + Z[b])), n) / 3.0
    assert np.abs(R.sum(axis=1) - total).max() <= 1e-12 * np.abs(total).max()


def test_rk2_with_the_n_scheme_is_heun(O):
    """With the N scheme and global lumping the two-stage step is Heun's
    method on dW/dt = -R(W)/V: the stage-2 mass term |T|/4 (W* - W^n)/dt sums
    to V (W* - W^n)/dt at every vertex, so the RK2 step equals the mean of
    W^n and two forward Euler steps."""
    m = I.cube_tets(4, jitter=0.2, seed=23)
    om = O.OracleMesh3(m)
    W = I.ic3_random_smooth(m, seed=24)
    dt = om.max_dt(W, 0.3)
    heun = 0.5 * (W + om.step(om.step(W, dt, O.N, O.EULER1), dt, O.N, O.EULER1))
    rk2 = om.step(W, dt, O.N, O.RK2)
    assert np.abs(rk2 - heun).max() <= 1e-13 * np.abs(W).max()
    # and the other schemes are not (their stage-2 parts are not per-vertex linear)
    assert np.abs(om.step(W, dt, O.B, O.RK2) - rk2).max() > 1e-8
