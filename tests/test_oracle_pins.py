"""Pins for the CPU oracle: each test checks the oracle against something other
than itself (closed forms, theorems of the paper, dense brute force, invariants,
finite differences), chosen so that a dropped term, a wrong sign or index, a
swapped direction or a transposed operand fails at least one of them.

Paper passages: eq. stab_func_FIE and eq. stab_func_DR (stability functions),
section 3 (parareal, finite termination, convergence factor eq. conv_factor),
Theorem 1 and Theorem 2 (bounds on the convergence factor), section 2.1 (the
split operators and the partition of unity), eq. FIE_method, eq. DR_method.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.optimize

import oracle
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore")


# ---------------------------------------------------------------- helpers ---
def mode2d(nx, ny, k1, k2):
    x = np.arange(1, nx + 1) / (nx + 1)
    y = np.arange(1, ny + 1) / (ny + 1)
    return np.outer(np.sin(k2 * np.pi * y), np.sin(k1 * np.pi * x))


def lam1d(n, k, a=1.0):
    """Eigenvalue magnitude of -(a u_xx)_h on sin(k pi x): (4a/h^2) sin^2(k pi h / 2)."""
    h = 1.0 / (n + 1)
    return 4.0 * a / h ** 2 * math.sin(k * math.pi * h / 2) ** 2


def problem(w, **over):
    """Oracle problem from a workload (faces from theta when given)."""
    kw = dict(dim=w.dim, nx=w.nx, ny=w.ny, T=w.T, n_slices=w.n_slices, fine_steps=w.fine_steps,
              coarse_steps=w.coarse_steps, split=w.split, fine=w.fine, c=w.c)
    if w.theta is not None:
        ax, ay = oracle.faces_from_theta(w.nx, w.ny, w.theta, dim=w.dim)
    else:
        ax, ay = w.ax, w.ay
    kw.update(ax=ax, ay=ay, rho=w.rho)
    kw.update(over)
    return oracle.Problem(**kw)


def dense_dim2(nx, ny, ax, ay, c=0.0):
    """Dense A_x, A_y assembled edge by edge from the face arrays (test-side code)."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    N = nx * ny
    Ax = np.zeros((N, N))
    Ay = np.zeros((N, N))
    idx = lambda i, j: j * nx + i
    for j in range(ny):
        for f in range(nx + 1):
            a = ax[j, f] / hx ** 2
            p, q = f - 1, f
            if p >= 0:
                Ax[idx(p, j), idx(p, j)] -= a
            if q < nx:
                Ax[idx(q, j), idx(q, j)] -= a
            if p >= 0 and q < nx:
                Ax[idx(p, j), idx(q, j)] += a
                Ax[idx(q, j), idx(p, j)] += a
    for g in range(ny + 1):
        for i in range(nx):
            a = ay[g, i] / hy ** 2
            p, q = g - 1, g
            if p >= 0:
                Ay[idx(i, p), idx(i, p)] -= a
            if q < ny:
                Ay[idx(i, q), idx(i, q)] -= a
            if p >= 0 and q < ny:
                Ay[idx(i, p), idx(i, q)] += a
                Ay[idx(i, q), idx(i, p)] += a
    Ax -= np.eye(N) * c / 2
    Ay -= np.eye(N) * c / 2
    return Ax, Ay


def dense_1d(n, faces):
    h = 1.0 / (n + 1)
    A = np.zeros((n, n))
    for f in range(n + 1):
        a = faces[f] / h ** 2
        p, q = f - 1, f
        if p >= 0:
            A[p, p] -= a
        if q < n:
            A[q, q] -= a
        if p >= 0 and q < n:
            A[p, q] += a
            A[q, p] += a
    return A


def relerr(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


# ------------------------------------------- P1: closed-form amplification ---
@pytest.mark.parametrize("nx,ny,k1,k2,a,c,tau", [
    (32, 32, 1, 1, 1.0, 0.0, 0.0125), (17, 9, 3, 2, 2.5, 0.0, 0.01), (24, 31, 5, 7, 0.7, 3.0, 0.002),
    (40, 12, 40, 1, 1.0, 0.0, 1e-3)])
def test_fie_step_eigenmode_closed_form(nx, ny, k1, k2, a, c, tau):
    """eq. stab_func_FIE: one FIE step multiplies a sin-sin eigenmode by
    1/((1 - z_x)(1 - z_y)), z = -tau (lambda + c/2)."""
    P = oracle.Problem(dim=2, nx=nx, ny=ny, T=1, n_slices=1, fine_steps=1, c=c,
                       ax=np.full((ny, nx + 1), a), ay=np.full((ny + 1, nx), a))
    u = mode2d(nx, ny, k1, k2)
    zx = -tau * (lam1d(nx, k1, a) + c / 2)
    zy = -tau * (lam1d(ny, k2, a) + c / 2)
    R = 1.0 / ((1 - zx) * (1 - zy))
    assert relerr(P.fie_step(u, tau), R * u) < 1e-13


@pytest.mark.parametrize("nx,ny,k1,k2,tau", [(32, 32, 1, 1, 0.01), (15, 22, 4, 3, 0.003)])
def test_dr_step_eigenmode_closed_form(nx, ny, k1, k2, tau):
    """eq. stab_func_DR: R_DR = 1 + (prod 1/(1 - z_j)) sum z_j."""
    P = oracle.Problem(dim=2, nx=nx, ny=ny, T=1, n_slices=1, fine_steps=1,
                       ax=np.ones((ny, nx + 1)), ay=np.ones((ny + 1, nx)))
    u = mode2d(nx, ny, k1, k2)
    zx, zy = -tau * lam1d(nx, k1), -tau * lam1d(ny, k2)
    R = 1 + (zx + zy) / ((1 - zx) * (1 - zy))
    assert relerr(P.dr_step(u, tau), R * u) < 1e-13


def scalar_parareal(RG, RF, N, K):
    """Parareal on the scalar recursion (section 3) in mpmath: y[k][n], k = 0..K."""
    y0 = [mp.mpf(1)]
    for n in range(N):
        y0.append(RG * y0[-1])
    Y = [y0]
    for k in range(K):
        prev = Y[-1]
        new = [mp.mpf(1)]
        for n in range(N):
            new.append(RG * new[n] + RF * prev[n] - RG * prev[n])
        Y.append(new)
    return Y


def test_config1_parareal_matches_scalar_closed_form():
    """Config 1 (32x32, a=1, u0 = sin pi x sin pi y, T=0.1, N=8, s=16, K=8) is a single
    eigenmode, so every parareal iterate is y^k_n * u0 with y from the scalar recursion
    built from eq. stab_func_FIE. Checks every iterate k = 0..8 and every increment."""
    mp.mp.dps = 40
    w = W.config1()
    n, N, s = w.nx, w.n_slices, w.fine_steps
    h = mp.mpf(1) / (n + 1)
    lam = 4 / h ** 2 * mp.sin(mp.pi * h / 2) ** 2
    DT = mp.mpf("0.1") / N
    RG = 1 / (1 + DT * lam) ** 2
    RF = (1 / (1 + DT / s * lam) ** 2) ** s
    Y = scalar_parareal(RG, RF, N, 8)
    P = problem(w)
    umax = np.abs(w.u0).max()
    for k in range(0, 9):
        U, kd, hist = P.parareal(w.u0, k)
        assert kd == k
        for nn in range(N + 1):
            assert relerr(U[nn], float(Y[k][nn]) * w.u0) < 2e-13, (k, nn)
        if k > 0:
            inc = max(abs(Y[k][m] - Y[k - 1][m]) for m in range(1, N + 1)) * umax
            assert abs(hist[-1] - float(inc)) <= 1e-13 * umax + 1e-9 * float(inc)
    # finite termination: the 8th iterate equals the sequential fine solution
    seq = P.sequential_fine(w.u0)
    assert np.array_equal(P.parareal(w.u0, 8)[0], seq)
    # sequential fine amplitude at T against the closed form R_F^(N)
    assert relerr(seq[N], float(RF ** N) * w.u0) < 1e-13


def test_coarse_steps_and_reaction_closed_form():
    """Coarse propagator with 2 FIE steps and a reaction term: R_G = R(DT/2)^2."""
    nx, ny, c = 12, 9, 1.5
    P = oracle.Problem(dim=2, nx=nx, ny=ny, T=0.2, n_slices=4, fine_steps=5, coarse_steps=2, c=c,
                       ax=np.ones((ny, nx + 1)), ay=np.ones((ny + 1, nx)))
    u = mode2d(nx, ny, 2, 3)
    tau = 0.2 / 4 / 2
    zx, zy = -tau * (lam1d(nx, 2) + c / 2), -tau * (lam1d(ny, 3) + c / 2)
    assert relerr(P.coarse(u), u / ((1 - zx) * (1 - zy)) ** 2) < 1e-13
    tau = 0.2 / 4 / 5
    zx, zy = -tau * (lam1d(nx, 2) + c / 2), -tau * (lam1d(ny, 3) + c / 2)
    assert relerr(P.fine(u), u / ((1 - zx) * (1 - zy)) ** 5) < 1e-13


# ----------------------------- P3: convergence factor (eq. conv_factor) ---
def K_factor(z1, z2, s, fine="fie"):
    RG = 1 / ((1 - z1) * (1 - z2))
    if fine == "fie":
        RF = (1 / ((1 - z1 / s) * (1 - z2 / s))) ** s
    else:
        a, b = z1 / s, z2 / s
        RF = (1 + (a + b) / ((1 - a) * (1 - b))) ** s
    return abs(RF - RG) / (1 - abs(RG))


def test_theorem_constants():
    """Theorem 1: z*, z** are the two roots of 3 z e^z + 1 = 0 in [-3, 0]; H(0,0) = 4 is the
    minimum and H(-3,-3) = 16(1+3/e^6) the maximum of H = (1-z1)(1-z2)(3e^{z1+z2}+1) on
    [-3,0]^2. Theorem 2: 2 = H(0,0) < H <= 4(1+1/e^2) with H = (1-z1)(1-z2)(e^{z1+z2}+1)
    on [-1,0]^2."""
    f = lambda z: 3 * z * math.exp(z) + 1
    zs = scipy.optimize.brentq(f, -1, -0.3)
    zss = scipy.optimize.brentq(f, -3, -1)
    assert abs(zs + 0.6190612867) < 1e-8 and abs(zss + 1.5121345516) < 1e-8
    H = lambda a, b: (1 - a) * (1 - b) * (3 * math.exp(a + b) + 1)
    g = np.linspace(-3, 0, 301)
    vals = np.array([[H(a, b) for a in g] for b in g])
    assert abs(vals.min() - 4) < 1e-12 and abs(vals.max() - 16 * (1 + 3 * math.exp(-6))) < 1e-9
    H2 = lambda a, b: (1 - a) * (1 - b) * (math.exp(a + b) + 1)
    g = np.linspace(-1, 0, 201)
    vals = np.array([[H2(a, b) for a in g] for b in g])
    assert abs(vals.min() - 2) < 1e-12 and abs(vals.max() - 4 * (1 + math.exp(-2))) < 1e-9


def test_convergence_factor_bounds():
    """Theorem 1: K_FIE-FIE <= 1/3 on (-inf,0)^2, s >= 1; Theorem 2: K_FIE-DR < 1."""
    zs = -np.logspace(-4, 5, 60)
    for s in (1, 2, 16, 64, 1000):
        kmax = max(K_factor(a, b, s) for a in zs for b in zs)
        assert kmax <= 1 / 3 + 1e-12
        kdr = max(K_factor(a, b, s, "dr") for a in zs for b in zs)
        assert kdr < 1


def test_parareal_per_mode_contraction():
    """With a = 1 the sin-sin modes decouple (Remark after eq. conv_factor): each mode's
    amplitude follows the scalar parareal recursion, and the error against the fine
    solution contracts by at least K(lambda) per iteration."""
    nx, ny, N, s = 15, 11, 6, 4
    T = 0.3
    P = oracle.Problem(dim=2, nx=nx, ny=ny, T=T, n_slices=N, fine_steps=s,
                       ax=np.ones((ny, nx + 1)), ay=np.ones((ny + 1, nx)))
    modes = [(1, 1), (2, 5), (7, 3), (15, 11)]
    rng = np.random.default_rng(3)
    amps = rng.standard_normal(len(modes))
    u0 = sum(a * mode2d(nx, ny, *m) for a, m in zip(amps, modes))
    seq = P.sequential_fine(u0)
    DT = T / N
    for K in range(0, 4):
        U, _, _ = P.parareal(u0, K)
        for a0, (k1, k2) in zip(amps, modes):
            e = mode2d(nx, ny, k1, k2)
            proj = lambda v: (v * e).sum() / (e * e).sum()
            z1, z2 = -DT * lam1d(nx, k1), -DT * lam1d(ny, k2)
            RG = 1 / ((1 - z1) * (1 - z2))
            RF = (1 / ((1 - z1 / s) * (1 - z2 / s))) ** s
            Y = scalar_parareal(mp.mpf(RG), mp.mpf(RF), N, K)
            for n in range(N + 1):
                assert abs(proj(U[n]) - a0 * float(Y[K][n])) < 1e-13 * abs(a0) + 1e-15
            err_k = max(abs(proj(U[n]) - proj(seq[n])) for n in range(1, N + 1))
            err_0 = max(abs(a0 * float(Y[0][n]) - proj(seq[n])) for n in range(1, N + 1))
            assert err_k <= K_factor(z1, z2, s) ** K * err_0 + 1e-14


# ------------------------------------------------- P4: dense brute force ---
@pytest.mark.parametrize("nx,ny,c", [(4, 4, 0.0), (3, 5, 0.0), (5, 3, 2.0)])
def test_dim_split_dense_brute_force(nx, ny, c):
    """eq. FIE_method / eq. DR_method with the dense matrices I - tau A_x, I - tau A_y
    solved by LU: FIE step (x then y), DR step, fine, coarse, full parareal."""
    w = W.small_dim2(nx, ny, n_slices=3, fine_steps=4, seed=nx * 10 + ny, c=c)
    P = problem(w)
    Ax, Ay = dense_dim2(nx, ny, P.ax, P.ay, c)
    I = np.eye(nx * ny)
    u = w.u0.ravel()
    tau = 0.013
    fie = np.linalg.solve(I - tau * Ay, np.linalg.solve(I - tau * Ax, u))
    assert relerr(P.fie_step(w.u0, tau).ravel(), fie) < 1e-13
    dr = u + tau * (Ax + Ay) @ u
    dr = np.linalg.solve(I - tau * Ax, dr - tau * Ax @ u)
    dr = np.linalg.solve(I - tau * Ay, dr - tau * Ay @ u)
    assert relerr(P.dr_step(w.u0, tau).ravel(), dr) < 1e-13
    # propagators and parareal with dense maps
    DT, dt = w.T / w.n_slices, w.T / w.n_slices / w.fine_steps
    Sx, Sy = np.linalg.inv(I - DT * Ax), np.linalg.inv(I - DT * Ay)
    G = Sy @ Sx
    Fx, Fy = np.linalg.inv(I - dt * Ax), np.linalg.inv(I - dt * Ay)
    F = np.linalg.matrix_power(Fy @ Fx, w.fine_steps)
    assert relerr(P.coarse(w.u0).ravel(), G @ u) < 1e-13
    assert relerr(P.fine(w.u0).ravel(), F @ u) < 1e-12
    N = w.n_slices
    U = [u]
    for n in range(N):
        U.append(G @ U[-1])
    for k in range(2):
        Fk = [F @ U[n] for n in range(N)]
        new = [u]
        for n in range(N):
            new.append(G @ new[n] + Fk[n] - G @ U[n])
        U = new
    Uo, kd, _ = P.parareal(w.u0, 2)
    assert kd == 2
    assert relerr(Uo.reshape(N + 1, -1), np.array(U)) < 1e-12


@pytest.mark.parametrize("n,cores,colors,overlap", [(32, 4, 2, 4), (48, 4, 4, 6), (40, 2, 2, 8),
                                                    (36, 6, 3, 4)])
def test_dd_dense_brute_force(n, cores, colors, overlap):
    """Domain-decomposition FIE (section 2.1 sub-operators with rho_j a, eq. FIE_method):
    colours in order, each solved densely on the whole line."""
    w = W.small_dd1(n, cores, colors, overlap, n_slices=3, fine_steps=2, seed=n)
    P = problem(w)
    a = P.ax[0]
    tau = 3e-4
    u = w.u0.copy()
    for j in range(colors):
        Aj = dense_1d(n, w.rho[j] * a)
        u = np.linalg.solve(np.eye(n) - tau * Aj, u)
    assert relerr(P.fie_step(w.u0, tau), u) < 1e-13
    # and DR
    As = [dense_1d(n, w.rho[j] * a) for j in range(colors)]
    v = w.u0 + tau * sum(As) @ w.u0
    for j in range(colors):
        v = np.linalg.solve(np.eye(n) - tau * As[j], v - tau * As[j] @ w.u0)
    assert relerr(P.dr_step(w.u0, tau), v) < 1e-13


# --------------------------------------- P5: partition of unity invariants ---
def test_dd_partition_invariants():
    """Section 2.1: sum_j rho_j = 1 gives sum_j A_j = A; each A_j is symmetric; rows outside
    a colour's components are zero (identity rows of I - tau A_j); one colour with
    rho = 1 is plain backward Euler."""
    n = 64
    w = W.small_dd1(n, 4, 2, 8, n_slices=2, fine_steps=2, seed=5)
    assert np.all(np.abs(w.rho.sum(0) - 1) == 0)
    P = problem(w)
    Pplain = oracle.Problem(dim=1, nx=n, ny=1, T=w.T, n_slices=2, fine_steps=2, ax=P.ax)
    rng = np.random.default_rng(0)
    for _ in range(3):
        u = rng.standard_normal(n)
        s = P.apply_Aj(0, u) + P.apply_Aj(1, u)
        assert relerr(s, Pplain.apply_A(u)) < 1e-13
    for j in range(2):
        D = np.array([P.apply_Aj(j, e) for e in np.eye(n)]).T
        assert np.allclose(D, D.T, rtol=0, atol=1e-9 * np.abs(D).max())
        support = (w.rho[j][:-1] > 0) | (w.rho[j][1:] > 0)
        assert np.all(D[~support] == 0)
    one = oracle.Problem(dim=1, nx=n, ny=1, T=w.T, n_slices=2, fine_steps=2, split="dd",
                         ax=P.ax, rho=np.ones((1, n + 1)))
    A = dense_1d(n, P.ax[0])
    assert relerr(one.fie_step(w.u0, 1e-3), np.linalg.solve(np.eye(n) - 1e-3 * A, w.u0)) < 1e-13


def test_linear_pou_shape():
    """The linear partition of unity: overlap faces take (2m+1)/64 for overlap 32."""
    rho = W.linear_pou_1d(1024, 8, 32, 2)
    ramp = rho[1][128 - 16:128 + 16]
    assert np.array_equal(ramp * 64, np.arange(1, 64, 2))
    assert np.array_equal(rho.sum(0), np.ones(1025))


# -------------------------------------------- consistency of the operator ---
def test_operator_second_order_consistency():
    """Second-order FD (section 5): A applied to u = sin(pi x) sin(2 pi y) approximates
    div(a grad u) for a = 1 + 0.5 sin(2 pi x) cos(2 pi y) with O(h^2) error. A swapped
    face index or direction breaks the second order."""
    errs = []
    for n in (31, 63, 127):
        ax, ay = W.variable_faces_2d(n, n)
        P = oracle.Problem(dim=2, nx=n, ny=n, T=1, n_slices=1, fine_steps=1, ax=ax, ay=ay)
        x = np.arange(1, n + 1) / (n + 1)
        X, Y = np.meshgrid(x, x)  # [y, x]
        pi = np.pi
        u = np.sin(pi * X) * np.sin(2 * pi * Y)
        a = 1 + 0.5 * np.sin(2 * pi * X) * np.cos(2 * pi * Y)
        a_x = pi * np.cos(2 * pi * X) * np.cos(2 * pi * Y)
        a_y = -pi * np.sin(2 * pi * X) * np.sin(2 * pi * Y)
        u_x = pi * np.cos(pi * X) * np.sin(2 * pi * Y)
        u_y = 2 * pi * np.sin(pi * X) * np.cos(2 * pi * Y)
        Lu = a_x * u_x + a * (-pi ** 2 * u) + a_y * u_y + a * (-4 * pi ** 2 * u)
        errs.append(np.abs(P.apply_A(u) - Lu).max() / np.abs(Lu).max())
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4
    assert errs[-1] < 1e-3


# ------------------------------------------------- face rule from theta ---
def test_faces_from_theta_closed_form_2d():
    """Face coefficients from a nodal log coefficient (section 2.1, D = e^theta I, face
    value = mean of e^theta over the face's two nodes). With e^theta = 1 + x + 3y^2 the
    mean is a polynomial of the face's coordinates: x-face f of interior row j sits
    between nodes x = f h_x and (f+1) h_x at y = (j+1) h_y, y-face g of column i between
    y = g h_y and (g+1) h_y at x = (i+1) h_x. nx != ny and the different x and y
    dependence make a row/column swap or a one-node shift fail."""
    nx, ny = 7, 5
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    xe = np.arange(nx + 2) * hx
    ye = np.arange(ny + 2) * hy
    theta = np.log(1.0 + xe[None, :] + 3.0 * ye[:, None] ** 2)  # [y, x], boundary included
    ax, ay = oracle.faces_from_theta(nx, ny, theta)
    assert ax.shape == (ny, nx + 1) and ay.shape == (ny + 1, nx)
    for j in range(ny):
        y = (j + 1) * hy
        for f in range(nx + 1):
            want = 1.0 + (f + 0.5) * hx + 3.0 * y * y
            assert abs(ax[j, f] - want) <= 4e-16 * want, (j, f, ax[j, f], want)
    for g in range(ny + 1):
        y2 = 0.5 * ((g * hy) ** 2 + ((g + 1) * hy) ** 2)
        for i in range(nx):
            want = 1.0 + (i + 1) * hx + 3.0 * y2
            assert abs(ay[g, i] - want) <= 4e-16 * want, (g, i, ay[g, i], want)


def test_faces_from_theta_closed_form_1d():
    """1D face rule: face f joins extended nodes f and f+1 (x = f h, (f+1) h); with
    e^theta = 1 + x + 2x^2 the face value is 1 + (f + 1/2) h + (f^2 + (f+1)^2) h^2."""
    nx = 9
    h = 1.0 / (nx + 1)
    x = np.arange(nx + 2) * h
    ax, _ = oracle.faces_from_theta(nx, 1, np.log(1.0 + x + 2.0 * x * x), dim=1)
    for f in range(nx + 1):
        want = 1.0 + (f + 0.5) * h + (f * f + (f + 1) ** 2) * h * h
        assert abs(ax[0, f] - want) <= 4e-16 * want, (f, ax[0, f], want)


def test_faces_from_theta_operator_consistency():
    """The face rule feeds the operator of section 2.1 in the right direction: with
    D = e^theta I, e^theta = 1 + x + 3y^2, the discrete A applied to u = sin(pi x)
    sin(2 pi y) approximates div(D grad u) to second order in h (an x/y swap of the
    faces gives an O(1) error)."""
    errs = []
    pi = np.pi
    for n in (31, 63, 127):
        h = 1.0 / (n + 1)
        e = np.arange(n + 2) * h
        theta = np.log(1.0 + e[None, :] + 3.0 * e[:, None] ** 2)
        ax, ay = oracle.faces_from_theta(n, n, theta)
        P = oracle.Problem(dim=2, nx=n, ny=n, T=1, n_slices=1, fine_steps=1, ax=ax, ay=ay)
        x = e[1:-1]
        X, Y = np.meshgrid(x, x)  # [y, x]
        u = np.sin(pi * X) * np.sin(2 * pi * Y)
        a = 1.0 + X + 3.0 * Y ** 2
        Lu = (1.0 * pi * np.cos(pi * X) * np.sin(2 * pi * Y) - a * pi ** 2 * u
              + 6.0 * Y * 2 * pi * np.sin(pi * X) * np.cos(2 * pi * Y) - a * 4 * pi ** 2 * u)
        errs.append(np.abs(P.apply_A(u) - Lu).max() / np.abs(Lu).max())
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4
    assert errs[-1] < 1e-3


# ------------------------------------------------ P6: M-matrix invariants ---
@pytest.mark.parametrize("kind", ["dim", "dd"])
def test_maximum_principle_positivity_linearity(kind):
    w = (W.small_dim2(13, 10, 2, 3, seed=4) if kind == "dim"
         else W.small_dd1(96, 4, 2, 8, 2, 3, seed=4))
    P = problem(w)
    rng = np.random.default_rng(1)
    for tau in (1e-5, 1e-3, 1e-1):
        u = rng.standard_normal(w.u0.shape)
        v = P.fie_step(u, tau)
        assert np.abs(v).max() <= np.abs(u).max() * (1 + 1e-15)
        up = np.abs(u)
        assert np.all(P.fie_step(up, tau) >= 0)
        u2 = rng.standard_normal(w.u0.shape)
        lhs = P.fie_step(2.0 * u - 3.0 * u2, tau)
        assert relerr(lhs, 2.0 * v - 3.0 * P.fie_step(u2, tau)) < 1e-13


# ----------------------------------------------- P2: finite termination ---
@pytest.mark.parametrize("kind", ["dim", "dd", "dr"])
def test_finite_termination(kind):
    """Section 3: parareal reaches the sequential fine solution after at most N_c
    iterations; iterate k is exact on the first k coarse nodes (bitwise here, since the
    correction is evaluated as F + (G_new - G_old))."""
    if kind == "dd":
        w = W.small_dd1(64, 4, 2, 8, n_slices=5, fine_steps=3, seed=2, T=0.01)
    else:
        w = W.small_dim2(9, 7, n_slices=5, fine_steps=3, seed=2)
        if kind == "dr":
            w.fine = "dr"
    P = problem(w)
    seq = P.sequential_fine(w.u0)
    for k in range(0, w.n_slices + 1):
        U, kd, _ = P.parareal(w.u0, k)
        for n in range(k + 1):
            assert np.array_equal(U[n], seq[n]), (k, n)
        if k < w.n_slices:
            assert not np.array_equal(U[k + 1], seq[k + 1])


def test_tolerance_stop_and_increment():
    """The stopping rule: iterate until the increment max_n max |U^{k+1}_n - U^k_n| < tol."""
    w = W.small_dim2(11, 11, n_slices=8, fine_steps=4, seed=9)
    P = problem(w)
    U8, _, hist = P.parareal(w.u0, 8)
    assert np.all(np.diff(np.log(hist[:5])) < 0)
    tol = hist[2] * 1.0001
    U, kd, h2 = P.parareal(w.u0, 8, tol)
    assert kd == 3 and np.array_equal(h2, hist[:3])
    Uprev, _, _ = P.parareal(w.u0, 2)
    assert abs(np.abs(U - Uprev).max() - h2[-1]) <= 1e-15 * np.abs(U).max()


# ------------------------------------------------------------- P7: adjoint ---
def test_adjoint_dot_product_and_finite_differences():
    """Adjoint of the fine map: <S x, y> = <x, S^T y>; face and theta gradients of
    L = <lam, u(T)> against central differences (h = 1e-6)."""
    nx, ny = 5, 4
    w = W.small_dim2(nx, ny, n_slices=2, fine_steps=3, seed=11, T=0.02)
    P = problem(w)
    rng = np.random.default_rng(5)
    lam = rng.standard_normal((ny, nx))
    x = rng.standard_normal((ny, nx))
    g0, gax, gay = P.adjoint(x, lam)
    Sx = P.sequential_fine(x)[-1]
    assert abs((Sx * lam).sum() - (x * g0).sum()) < 1e-13 * abs((Sx * lam).sum())

    def loss(ax, ay):
        Q = oracle.Problem(dim=2, nx=nx, ny=ny, T=w.T, n_slices=2, fine_steps=3, ax=ax, ay=ay)
        return (Q.sequential_fine(x)[-1] * lam).sum()

    h = 1e-6
    for arr, g in ((P.ax, gax), (P.ay, gay)):
        for idx in [(0, 0), (1, 2), (ny - 1 if arr is P.ax else ny, nx - 1), (2, 3)]:
            ap, am = P.ax.copy(), P.ay.copy()
            tgt_p, tgt_m = (ap, None), (am, None)
            A1 = arr.copy()
            A1[idx] += h
            A2 = arr.copy()
            A2[idx] -= h
            if arr is P.ax:
                fd = (loss(A1, P.ay) - loss(A2, P.ay)) / (2 * h)
            else:
                fd = (loss(P.ax, A1) - loss(P.ax, A2)) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(abs(g[idx]), 1e-3), (idx, fd, g[idx])
    # theta chain rule
    gth = oracle.theta_grad(nx, ny, w.theta, gax, gay)

    def loss_t(th):
        ax, ay = oracle.faces_from_theta(nx, ny, th)
        return loss(ax, ay)

    for idx in [(0, 1), (2, 3), (3, 0), (ny + 1, nx), (0, 0)]:
        t1 = w.theta.copy()
        t1[idx] += h
        t2 = w.theta.copy()
        t2[idx] -= h
        fd = (loss_t(t1) - loss_t(t2)) / (2 * h)
        assert abs(fd - gth[idx]) <= 1e-6 * max(abs(gth[idx]), 1e-3), (idx, fd, gth[idx])
    assert gth[0, 0] == 0 and gth[-1, -1] == 0  # corner nodes touch no face


def test_increment_covers_first_slice():
    """The increment runs over every coarse node n >= 1, including n = 1: with a stiff
    high-frequency mode the largest change of the first correction sits at n = 1."""
    nx, ny = 9, 8
    P = oracle.Problem(dim=2, nx=nx, ny=ny, T=0.5, n_slices=4, fine_steps=3,
                       ax=np.ones((ny, nx + 1)), ay=np.ones((ny + 1, nx)))
    u0 = mode2d(nx, ny, nx, ny)
    U0, _, _ = P.parareal(u0, 0)
    U1, _, hist = P.parareal(u0, 1)
    d = np.abs(U1 - U0).reshape(P.n_slices + 1, -1).max(1)
    assert np.argmax(d) == 1 and d[0] == 0
    assert hist[0] == d.max()


# ---------------------------------------------------------- source terms ---
def _forced_problem(nx, ny, T, N, s, fine, forcing, theta_seed=2, c=0.0):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=theta_seed, T=T, c=c)
    w.fine = fine
    return problem(w, forcing=forcing)


def test_forcing_dr_preserves_forced_steady_state():
    """eq. DR_method with F = -A S (time independent): S solves U' = AU + F with
    U' = 0, and the DR step maps it to itself exactly (its first stage adds
    tau A S + tau F = 0 and every later stage returns S). FIE, with its first-
    order splitting error, moves it: a sign or scale error on tau F breaks the
    first property, a source added to the wrong stage the second."""
    nx, ny, N, s = 13, 11, 2, 3
    S = W.sine_modes_2d(nx, ny, seed=9)
    A = _forced_problem(nx, ny, 0.05, N, s, "fie", None, theta_seed=4, c=0.7)
    F = -A.apply_A(S)
    forcing = (F[None], np.ones((1, N * s)), np.ones((1, N)))
    dr = _forced_problem(nx, ny, 0.05, N, s, "dr", forcing, theta_seed=4, c=0.7)
    fie = _forced_problem(nx, ny, 0.05, N, s, "fie", forcing, theta_seed=4, c=0.7)
    assert np.abs(dr.fine(S, 1) - S).max() <= 1e-13 * np.abs(S).max()
    assert np.abs(fie.fine(S, 1) - S).max() > 1e-3 * np.abs(S).max()


@pytest.mark.parametrize("fine,steps", [("fie", (32, 64, 128)), ("dr", (16, 32, 64))])
def test_forcing_manufactured_first_order_in_time(fine, steps):
    """Manufactured semi-discrete solution U(t) = sin(2 pi t) S with the source
    F(t) = 2 pi cos(2 pi t) S - sin(2 pi t) A S (A the discrete operator, so
    the space error is zero): both splitting methods are first-order
    convergent (section 2.2), so halving dt halves the error at the slice
    ends, and the error is far below the solution's size."""
    nx, ny, T, N = 15, 13, 0.5, 2
    S = W.sine_modes_2d(nx, ny, seed=3)
    AS = _forced_problem(nx, ny, T, N, 1, fine, None).apply_A(S)
    g = lambda t: np.stack([2 * np.pi * np.cos(2 * np.pi * t), np.sin(2 * np.pi * t)])
    DT = T / N
    errs = []
    for s in steps:
        dt = DT / s
        tf = np.array([n * DT + (j + 1) * dt for n in range(N) for j in range(s)])
        tc = np.array([(n + 1) * DT for n in range(N)])
        P = _forced_problem(nx, ny, T, N, s, fine, (np.stack([S, -AS]), g(tf), g(tc)))
        U = P.sequential_fine(np.zeros_like(S))
        exact = np.stack([np.sin(2 * np.pi * n * DT) * S for n in range(N + 1)])
        errs.append(np.abs(U - exact).max())
    assert errs[-1] < 0.05 * np.abs(S).max()
    assert 1.75 < errs[-2] / errs[-1] < 2.25
    assert errs[0] > errs[1] > errs[2]


def test_forcing_superposition():
    """The forced propagators are affine: F(u) = F_unforced(u) + F(0)."""
    nx, ny, N, s = 9, 7, 3, 2
    rng = np.random.default_rng(11)
    forcing = (rng.standard_normal((2, ny, nx)), rng.standard_normal((2, N * s)),
               rng.standard_normal((2, N)))
    u = rng.standard_normal((ny, nx))
    for fine in ("fie", "dr"):
        Pf = _forced_problem(nx, ny, 0.1, N, s, fine, forcing)
        P0 = _forced_problem(nx, ny, 0.1, N, s, fine, None)
        for n in range(N):
            lhs = Pf.fine(u, n)
            rhs = P0.fine(u, n) + Pf.fine(np.zeros_like(u), n)
            assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()
        lhs = Pf.coarse(u, 1)
        assert np.abs(lhs - (P0.coarse(u, 1) + Pf.coarse(np.zeros_like(u), 1))).max() <= 1e-13


def test_manufactured_problem_converges():
    """The paper's test problem (section 5, u = sin 2pi t sin 2pi x sin 2pi y with
    its source): with dt proportional to h^2 the FIE fine solution's error
    (maximum over time of the discrete 2-norm, the paper's error measure)
    falls like h^2, i.e. by about 4 per halving of h (second-order finite
    differences, first-order FIE)."""
    errs = []
    for n, s in [(15, 4), (31, 16), (63, 64)]:
        w = W.manufactured2d(n, 8, s)
        P = problem(w, forcing=w.forcing)
        U = P.sequential_fine(w.u0)
        DT = w.T / w.n_slices
        exact = np.stack([np.sin(2 * np.pi * k * DT) * w.extra["exact_space"]
                          for k in range(w.n_slices + 1)])
        errs.append(np.sqrt(((U - exact) ** 2).sum(axis=(1, 2)) / (n + 1) ** 2).max())
    assert errs[0] > errs[1] > errs[2]
    assert 3.0 < errs[1] / errs[2] < 4.6
    assert errs[2] < 0.05


def test_threaded_parareal_composition_is_the_oracle_iteration():
    """The test harness that runs the oracle's slices on threads (used for the
    full-size batch comparisons) reproduces or_parareal bit for bit, with a
    source term so that the slice index reaches every fine call."""
    import workloads as W
    from gpu_helpers import oracle_problem, parareal_threaded
    w = W.manufactured2d(11, 5, 3)
    w.theta = 0.3 * W.smooth_field_2d(13, 13, ell=0.2, K=6, seed=9)
    O = oracle_problem(w)
    U1, k1, h1 = O.parareal(w.u0 + 0.1, 3)
    U2, h2 = parareal_threaded(O, w.u0 + 0.1, 3, workers=4)
    assert k1 == 3
    assert np.array_equal(U1, U2)
    assert np.array_equal(h1, np.asarray(h2))
