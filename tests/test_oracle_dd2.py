"""Pins of the oracle's 2D domain-decomposition split (section 2.1: subdomains
made of vertical strips, L_j u = div(rho_j D grad u) - rho_j c u; eq. FIE_method)
against facts that do not come from the oracle's own formulas:

- the split operators sum to the full operator (the dimensional-split operator
  of the same coefficients, a separate code path pinned by eigenmode closed forms);
- one colour with rho = 1 is implicit Euler on the full operator: closed-form
  amplification 1/(1 + tau (lambda_x + lambda_y + c)) on discrete sine modes;
- with a_y = 0 every grid row is the 1D domain-decomposition problem (the
  oracle's tridiagonal path);
- with D = I every strip system diagonalises under the sine transform in y;
  the substep computed mode by mode must agree;
- each substep map is symmetric (I - tau A_j is);
- FIE over the colours is first order in time against the exact flow exp(tA);
- parareal's finite termination (k = N reproduces the sequential fine solution).
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as W


def dd2_problem(w, **kw):
    ax, ay = oracle.faces_from_theta(w.nx, w.ny, w.theta)
    args = dict(dim=2, nx=w.nx, ny=w.ny, T=w.T, n_slices=w.n_slices, fine_steps=w.fine_steps,
                coarse_steps=w.coarse_steps, split="dd", c=w.c, ax=ax, ay=ay, rho=w.rho)
    args.update(kw)
    return oracle.Problem(**args)


def test_strip_pou_is_a_partition_of_unity():
    for n, q, beta, M in [(999, 2, 1 / 16, 2), (63, 3, 0.05, 2), (40, 1, 0.2, 3)]:
        r = W.strip_pou_2d(n, q, beta, M)
        assert r.shape == (M, 2 * n + 1)
        assert np.all(r >= 0) and np.all(r <= 1)
        assert np.abs(r.sum(axis=0) - 1.0).max() == 0.0
        # each colour's support is q strips
        for k in range(M):
            act = (r[k, 0:-1:2] > 0) | (r[k, 1::2] > 0) | (r[k, 2::2] > 0)
            runs = np.count_nonzero(np.diff(np.concatenate([[0], act.astype(int), [0]])) == 1)
            assert runs == q


@pytest.mark.parametrize("c", [0.0, 3.0])
def test_dd2_operators_sum_to_full_operator(c):
    w = W.small_dd2(23, 17, 2, 0.08, 2, 2, seed=3, c=c)
    P = dd2_problem(w)
    ax, ay = oracle.faces_from_theta(w.nx, w.ny, w.theta)
    Pdim = oracle.Problem(dim=2, nx=w.nx, ny=w.ny, T=w.T, n_slices=2, fine_steps=2, c=c, ax=ax,
                          ay=ay)
    u = np.random.default_rng(0).standard_normal((w.ny, w.nx))
    tot = P.apply_Aj(0, u) + P.apply_Aj(1, u)
    ref = Pdim.apply_A(u)
    assert np.abs(tot - ref).max() <= 1e-12 * np.abs(ref).max()


def test_dd2_single_colour_is_implicit_euler_on_sine_modes():
    nx, ny, tau, c = 15, 11, 3e-3, 2.0
    rho = np.ones((1, 2 * nx + 1))
    P = oracle.Problem(dim=2, nx=nx, ny=ny, T=1.0, n_slices=1, fine_steps=1, split="dd", c=c,
                       ax=np.ones((ny, nx + 1)), ay=np.ones((ny + 1, nx)), rho=rho)
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    x, y = np.arange(1, nx + 1) * hx, np.arange(1, ny + 1) * hy
    for p, q in [(1, 1), (3, 7), (nx, ny)]:
        u = np.outer(np.sin(q * np.pi * y), np.sin(p * np.pi * x))
        lam = 4 / hx ** 2 * np.sin(p * np.pi * hx / 2) ** 2 + 4 / hy ** 2 * np.sin(q * np.pi * hy / 2) ** 2
        got = P.fie_step(u, tau)
        assert np.abs(got - u / (1 + tau * (lam + c))).max() <= 1e-13


def test_dd2_without_y_coupling_is_rowwise_1d_dd():
    w = W.small_dd2(40, 6, 2, 0.1, 2, 2, seed=5)
    ax, _ = oracle.faces_from_theta(w.nx, w.ny, w.theta)
    P = oracle.Problem(dim=2, nx=w.nx, ny=w.ny, T=1.0, n_slices=1, fine_steps=1, split="dd", ax=ax,
                       ay=np.zeros((w.ny + 1, w.nx)), rho=w.rho)
    u = np.random.default_rng(1).standard_normal((w.ny, w.nx))
    tau = 2e-3
    got = P.fie_step(u, tau)
    rho_faces = w.rho[:, 0::2]
    for k in range(w.ny):
        P1 = oracle.Problem(dim=1, nx=w.nx, ny=1, T=1.0, n_slices=1, fine_steps=1, split="dd",
                            ax=ax[k], rho=rho_faces)
        ref = P1.fie_step(u[k], tau)
        assert np.abs(got[k] - ref).max() <= 1e-13 * np.abs(ref).max()


def _dst_substep(rho_k, tau, c, u, nx, ny):
    """(I - tau A_k) v = u for D = I by the orthonormal sine transform in y:
    every sine mode m of the column direction decouples into one tridiagonal
    system in x with the y eigenvalue mu_m scaled by rho at the node."""
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    k = np.arange(1, ny + 1)
    S = np.sqrt(2 / (ny + 1)) * np.sin(np.pi * np.outer(k, k) / (ny + 1))  # symmetric, S S = I
    mu = 4 / hy ** 2 * np.sin(k * np.pi * hy / 2) ** 2
    rf, rn = rho_k[0::2], rho_k[1::2]
    uh = S @ u
    vh = np.empty_like(uh)
    for m in range(ny):
        Mx = np.diag(1 + tau * ((rf[:-1] + rf[1:]) / hx ** 2 + rn * (mu[m] + c)))
        Mx -= np.diag(tau * rf[1:-1] / hx ** 2, 1) + np.diag(tau * rf[1:-1] / hx ** 2, -1)
        vh[m] = np.linalg.solve(Mx, uh[m])
    return S @ vh


@pytest.mark.parametrize("q,beta,c", [(2, 0.08, 0.0), (3, 0.05, 1.5)])
def test_dd2_constant_coefficient_matches_sine_transform(q, beta, c):
    nx, ny, tau = 48, 21, 4e-3
    rho = W.strip_pou_2d(nx, q, beta, 2)
    P = oracle.Problem(dim=2, nx=nx, ny=ny, T=1.0, n_slices=1, fine_steps=1, split="dd", c=c,
                       ax=np.ones((ny, nx + 1)), ay=np.ones((ny + 1, nx)), rho=rho)
    u = np.random.default_rng(2).standard_normal((ny, nx))
    ref = _dst_substep(rho[1], tau, c, _dst_substep(rho[0], tau, c, u, nx, ny), nx, ny)
    got = P.fie_step(u, tau)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_dd2_substep_map_is_symmetric():
    """Each S_j = (I - tau A_j)^{-1} is symmetric, so the FIE step S_1 S_0 has the
    transpose S_0 S_1, which is the FIE step with the colours swapped."""
    w = W.small_dd2(19, 13, 2, 0.1, 1, 1, seed=8, c=0.7)
    ax, ay = oracle.faces_from_theta(w.nx, w.ny, w.theta)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((2, w.ny, w.nx))
    mk = lambda r: oracle.Problem(dim=2, nx=w.nx, ny=w.ny, T=1.0, n_slices=1, fine_steps=1,
                                  split="dd", c=w.c, ax=ax, ay=ay, rho=r)
    P, Ps = mk(w.rho), mk(w.rho[::-1].copy())
    tau = 5e-3
    lhs = np.vdot(v, P.fie_step(u, tau))
    rhs = np.vdot(Ps.fie_step(v, tau), u)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_dd2_fie_is_first_order_in_time():
    nx = ny = 11
    w = W.small_dd2(nx, ny, 2, 0.12, 1, 1, seed=6, T=0.02)
    ax, ay = oracle.faces_from_theta(nx, ny, w.theta)
    Pd = oracle.Problem(dim=2, nx=nx, ny=ny, T=1.0, n_slices=1, fine_steps=1, ax=ax, ay=ay)
    n = nx * ny
    A = np.stack([Pd.apply_A(e.reshape(ny, nx)).ravel() for e in np.eye(n)], axis=1)
    exact = (scipy.linalg.expm(w.T * A) @ w.u0.ravel()).reshape(ny, nx)
    errs = []
    for s in (8, 16, 32):
        P = dd2_problem(w, n_slices=1, fine_steps=s)
        errs.append(np.abs(P.fine(w.u0) - exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2


def test_dd2_parareal_finite_termination():
    w = W.small_dd2(17, 12, 2, 0.1, 5, 3, seed=9)
    P = dd2_problem(w)
    U, k, _ = P.parareal(w.u0, w.n_slices)
    seq = P.sequential_fine(w.u0)
    assert k == w.n_slices
    assert np.abs(U - seq).max() <= 1e-13 * np.abs(seq).max()


def test_dd2_dr_keeps_the_forced_steady_state():
    """Douglas-Rachford (eq. DR_method) with a time-independent source F leaves
    U* = -A^{-1} F unchanged for any partition of unity: (I + tau A)U* + tau F = U*
    and every substep then solves (I - tau A_j)U* = U* - tau A_j U*."""
    nx, ny = 14, 11
    w = W.small_dd2(nx, ny, 2, 0.12, 1, 1, seed=12, c=0.5)
    ax, ay = oracle.faces_from_theta(nx, ny, w.theta)
    Pd = oracle.Problem(dim=2, nx=nx, ny=ny, T=1.0, n_slices=1, fine_steps=1, c=w.c, ax=ax, ay=ay)
    n = nx * ny
    A = np.stack([Pd.apply_A(e.reshape(ny, nx)).ravel() for e in np.eye(n)], axis=1)
    F = np.random.default_rng(5).standard_normal(n)
    ustar = np.linalg.solve(A, -F).reshape(ny, nx)
    for rho in (w.rho, W.strip_pou_2d(nx, 1, 0.2, 3)):
        P = oracle.Problem(dim=2, nx=nx, ny=ny, T=1.0, n_slices=1, fine_steps=1, split="dd",
                           fine="dr", c=w.c, ax=ax, ay=ay, rho=rho)
        got = P.dr_step(ustar, 7e-3, F=F.reshape(ny, nx))
        assert np.abs(got - ustar).max() <= 1e-11 * np.abs(ustar).max()
        # and FIE does not (the splitting error of a Lie step)
        assert np.abs(P.fie_step(ustar, 7e-3, F=F.reshape(ny, nx)) - ustar).max() > 1e-6 * np.abs(ustar).max()


def read_golden(name):
    import os
    vals = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = (t.strip() for t in line.split("="))
            vals[k] = float(v)
    return vals


def manufactured_error(n, N, s, q, beta, fine_map):
    """Maximum over the coarse time levels of the discrete 2-norm error of the
    fine solution of the paper's test problem (section 5)."""
    w = W.dd2_manufactured(n=n, n_slices=N, fine_steps=s, q=q, beta=beta)
    h = 1.0 / (n + 1)
    u = w.u0.copy()
    err = 0.0
    for k in range(N):
        u = fine_map(w, u, k)
        ex = np.sin(2 * np.pi * (k + 1) / N) * w.extra["exact_space"]
        err = max(err, np.sqrt(((u - ex) ** 2).sum()) * h)
    return err


def test_dd2_fine_error_matches_the_paper():
    """The paper prints the error of its fine approximation for the DD-split
    scalability runs; the oracle reproduces all printed digits."""
    g = read_golden("dd2_fine_error_h001.txt")
    n, N, s = int(g["n"]), int(g["n_slices"]), int(g["fine_steps"])
    cache = {}

    def fine(w, u, k):
        if "P" not in cache:
            cache["P"] = oracle.Problem(dim=2, nx=n, ny=n, T=1.0, n_slices=N, fine_steps=s,
                                        split="dd", ax=np.ones((n, n + 1)),
                                        ay=np.ones((n + 1, n)), rho=w.rho, forcing=w.forcing)
        return cache["P"].fine(u, k)

    err = manufactured_error(n, N, s, int(g["q"]), g["beta"], fine)
    # within half a unit of the last printed digit
    assert abs(err - g["error"]) <= 0.5e-7



def test_dd2_strip_solve_is_exact_to_rounding_on_an_ill_conditioned_strip():
    """A 560-column, 5-row strip at tau = 1/300 (condition number about 5000): the
    oracle's substep is the exact solve of its system up to a few units of
    roundoff. The reference does not use the oracle's solver: the same matrix
    entries (the FP64 values of the operator's definition) go to scipy's sparse
    LU, whose solution is refined once with a residual accumulated in long double
    (numpy)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    nx, ny, tau = 560, 5, 1.0 / 300
    w = W.small_dd2(nx, ny, 1, 0.1, 1, 1, seed=6, T=tau)
    w.rho = np.ones((1, 2 * nx + 1))
    ax, ay = oracle.faces_from_theta(nx, ny, w.theta)
    P = dd2_problem(w)
    u = W.sine_modes_2d(nx, ny, seed=3) + 0.01 * np.random.default_rng(4).standard_normal((ny, nx))
    x = P.fie_step(u, tau)
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    rows, cols, vals = [], [], []
    for k in range(ny):
        for i in range(nx):
            q = k * nx + i
            fw, fe = ax[k, i] / (hx * hx), ax[k, i + 1] / (hx * hx)
            fs, fn = ay[k, i] / (hy * hy), ay[k + 1, i] / (hy * hy)
            rows.append(q); cols.append(q); vals.append(1.0 + tau * (fw + fe + fs + fn))
            for ok, qq, f in ((i > 0, q - 1, fw), (i < nx - 1, q + 1, fe), (k > 0, q - nx, fs),
                              (k < ny - 1, q + nx, fn)):
                if ok:
                    rows.append(q); cols.append(qq); vals.append(-tau * f)
    rows, cols, vals = np.array(rows), np.array(cols), np.array(vals)
    B = sp.csc_matrix((vals, (rows, cols)), shape=(nx * ny, nx * ny))

    def residual(v):  # u - B v, every product and sum in long double
        L = np.longdouble
        acc = u.ravel().astype(L)
        np.add.at(acc, rows, -(vals.astype(L) * v.ravel().astype(L)[cols]))
        return acc

    lu = spla.splu(B)
    x0 = lu.solve(u.ravel())
    xref = x0.astype(np.longdouble) + lu.solve(np.asarray(residual(x0), np.float64))
    scale = float(np.abs(xref).max())
    err = float(np.abs(x.ravel().astype(np.longdouble) - xref).max()) / scale
    assert err <= 4e-15, err
    # the residual of the FP64-rounded solution is at the level of rounding x itself
    absBx = np.zeros(nx * ny)
    np.add.at(absBx, rows, np.abs(vals) * np.abs(x.ravel())[cols])
    assert float(np.abs(residual(x)).max()) <= 2 * 2.0 ** -53 * absBx.max()
    # the unrefined direct solve is not that accurate on this system
    assert float(np.abs(x0 - xref).max()) / scale > 2 * err
