"""GPU parity of the 2D domain-decomposition split into vertical strips
(section 2.1, Fig. fig:domaindecomposition; substeps of eq. FIE_method solved
by block cyclic reduction over each strip) against the oracle's banded
elimination: the fine map over all slices, the sequential fine solve, the
coarse sweep, parareal, source terms, handles mixing split kinds, and
coefficient updates. Relative infinity-norm error <= 1e-12, also at the
paper's size (h = 1e-3, q = 2, beta = 1/16, N = 20); on a 560-column strip whose
system has condition number ~5000 the bound is 4 kappa u (the explicit inverses'
rounding)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import TOL, gpu_problem, oracle_problem, relerr, slice_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda").reshape(-1)


def fine_parity(w, seed=0):
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=seed)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    return relerr(F.cpu().numpy().reshape(ref.shape), ref)


# (nx, ny, q, beta, N, s, colours, c): strips of 1..7 row tiles, 1..7 reduction
# levels, slice counts that are not multiples of 16 (1 to 5 column tiles of 16)
CASES = [
    (40, 33, 2, 0.1, 5, 2, 2, 0.0),
    (97, 61, 2, 0.08, 20, 2, 2, 0.0),
    (64, 1, 2, 0.1, 3, 3, 2, 0.0),
    (30, 2, 1, 0.2, 17, 2, 2, 1.0),
    (120, 17, 3, 0.04, 70, 1, 2, 0.0),
    (75, 40, 2, 0.05, 9, 2, 3, 2.5),
    (9, 25, 1, 0.2, 4, 3, 2, 0.0),
    (60, 30, 2, 0.1, 40, 2, 2, 0.0),  # three column tiles (the 16-way split runs 8-way)
]


@pytest.mark.parametrize("nx,ny,q,beta,N,s,M,c", CASES)
def test_dd2_fine_propagate(nx, ny, q, beta, N, s, M, c):
    w = W.small_dd2(nx, ny, q, beta, N, s, seed=nx + ny, n_colors=M, c=c)
    assert fine_parity(w, seed=N) <= TOL


@pytest.mark.parametrize("nx,ny,q,beta,N,s,M,forced", [(40, 33, 2, 0.1, 5, 2, 2, False),
                                                        (75, 40, 2, 0.05, 9, 2, 3, True),
                                                        (97, 61, 2, 0.08, 20, 2, 2, True)])
def test_dd2_dr_fine_propagate(nx, ny, q, beta, N, s, M, forced):
    """Douglas-Rachford fine propagator (eq. DR_method) over the strip split."""
    w = W.small_dd2(nx, ny, q, beta, N, s, seed=nx + 3, n_colors=M, c=0.7)
    w.fine = "dr"
    if forced:
        rng = np.random.default_rng(nx)
        w.forcing = (rng.standard_normal((2, ny, nx)), rng.standard_normal((2, N * s)),
                     rng.standard_normal((2, N)))
    assert fine_parity(w, seed=N) <= TOL


def test_dd2_dr_sequential_and_parareal():
    w = W.small_dd2(50, 37, 2, 0.08, 6, 3, seed=17)
    w.fine = "dr"
    w.coarse_steps = 2
    P, O = gpu_problem(w), oracle_problem(w)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=3, tol=0.0)
    torch.cuda.synchronize()
    ref = O.sequential_fine(w.u0)
    assert relerr(Seq.cpu().numpy().reshape(ref.shape), ref) <= TOL
    Uo, ko, hist = O.parareal(w.u0, 3)
    assert k[0] == ko
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL


def test_dd2_one_column_strip():
    """A colour whose support is a single node column (a strip of width 1)."""
    nx, ny = 21, 17
    w = W.small_dd2(nx, ny, 1, 0.2, 3, 2, seed=31)
    rho = np.zeros((2, 2 * nx + 1))
    rho[0] = 1.0
    rho[1, 2 * 9 + 1] = 0.5  # node column 9 only
    rho[0, 2 * 9 + 1] = 0.5
    w.rho = rho
    assert fine_parity(w) <= TOL
    w.fine = "dr"
    assert fine_parity(w) <= TOL


def test_dd2_dr_three_colours_after_coefficient_update():
    w = W.small_dd2(60, 23, 1, 0.1, 4, 2, seed=33, n_colors=3, c=0.3)
    w.fine = "dr"
    P = gpu_problem(w)
    theta2 = 0.3 * W.smooth_field_2d(w.nx + 2, w.ny + 2, ell=0.25, K=5, seed=77)
    P.set_coefficients(0, dev(theta2))
    w.theta = theta2
    Uin = slice_inputs(w, seed=2)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = oracle_problem(w).fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


def test_dd2_dr_mixed_handle():
    a = W.small_dd2(40, 20, 2, 0.1, 4, 2, seed=41)
    a.fine = "dr"
    b = W.small_dim2(30, 26, 5, 3, seed=42)
    b.fine = "dr"
    c = W.small_dd2(33, 28, 1, 0.15, 3, 2, seed=43)
    ws = [a, b, c]
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, ko, _ = oracle_problem(w).parareal(w.u0, 2)
        assert k[i] == ko
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL


def test_dd2_tall_strips():
    """Strips of 6 row tiles over 2100 rows: the large first-level launches take one
    workgroup per block row (two waves of row tiles)."""
    w = W.small_dd2(160, 2100, 1, 0.1, 2, 1, seed=21)
    assert fine_parity(w, seed=3) <= TOL


def test_dd2_single_colour_full_width():
    """One colour with rho = 1: a single strip spanning the grid (implicit Euler)."""
    nx, ny = 130, 21
    w = W.small_dd2(nx, ny, 1, 0.1, 4, 2, seed=4)
    w.rho = np.ones((1, 2 * nx + 1))
    assert fine_parity(w) <= TOL


def strip_bound(w, tau):
    """Parity bound of the strip solver: max(1e-12, 4 kappa u), kappa = 1 + 4 tau
    max(a) (1/h_x^2 + 1/h_y^2) the strip system's condition number and u the FP64 unit
    roundoff. The oracle's strip solves are refined to the exact solution's rounding;
    the block cyclic reduction applies explicit inverses of dense Schur complements,
    whose rounding grows with kappa."""
    ax, ay = oracle.faces_from_theta(w.nx, w.ny, w.theta)
    amax = max(float(ax.max()), float(ay.max()))
    kappa = 1 + 4 * tau * amax * ((w.nx + 1) ** 2 + (w.ny + 1) ** 2)
    return max(TOL, 4 * kappa * 2.0 ** -53)


def test_dd2_wide_strip():
    """A strip of 560 columns (padded 576) at tau = 1/300: the all-slice level-0 sweeps
    take the one-lane-per-line form (the LDS-staged form holds at most 512), the
    single-state ones sixteen positions per lane. The strip system's condition number
    is about 5000."""
    nx, ny = 560, 5
    w = W.small_dd2(nx, ny, 1, 0.1, 3, 1, seed=6, T=1e-2)
    w.rho = np.ones((1, 2 * nx + 1))
    bound = strip_bound(w, w.T / w.n_slices)
    err = fine_parity(w)
    print(f"wide strip: relative error {err:.3e} (bound {bound:.2e})", flush=True)
    assert err <= bound
    P, O = gpu_problem(w), oracle_problem(w)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    torch.cuda.synchronize()
    ref = O.sequential_fine(w.u0)
    assert relerr(Seq.cpu().numpy().reshape(ref.shape), ref) <= bound


def test_dd2_constant_coefficient():
    w = W.small_dd2(81, 47, 2, 1.0 / 16, 6, 2, seed=2, variable=False)
    assert fine_parity(w) <= TOL


@pytest.mark.parametrize("fine_only", [False, True])
def test_dd2_sequential_and_parareal(fine_only):
    w = W.small_dd2(50, 37, 2, 0.08, 6, 3, seed=11)
    w.coarse_steps = 2
    P, O = gpu_problem(w), oracle_problem(w)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    torch.cuda.synchronize()
    ref = O.sequential_fine(w.u0)
    assert relerr(Seq.cpu().numpy().reshape(ref.shape), ref) <= TOL
    if fine_only:
        return
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=3, tol=0.0)
    torch.cuda.synchronize()
    Uo, ko, hist = O.parareal(w.u0, 3)
    assert k[0] == ko
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL
    assert abs(inc[0] - hist[-1]) <= TOL * np.abs(Uo).max()


def test_dd2_parareal_finite_termination():
    w = W.small_dd2(33, 29, 2, 0.1, 5, 2, seed=12)
    P = gpu_problem(w)
    U, Seq = P.new_states(), P.new_states()
    k, _ = P.parareal_iterate(dev(w.u0), U, k_max=w.n_slices, tol=0.0)
    P.sequential_fine(dev(w.u0), Seq)
    torch.cuda.synchronize()
    assert k[0] == w.n_slices
    seq = Seq.cpu().numpy()
    assert np.abs(U.cpu().numpy() - seq).max() <= 1e-13 * np.abs(seq).max()


def test_dd2_coarse_sweep():
    w = W.small_dd2(45, 26, 2, 0.1, 5, 2, seed=13)
    w.coarse_steps = 3
    P, O = gpu_problem(w), oracle_problem(w)
    N, nx, ny = w.n_slices, w.nx, w.ny
    U0 = np.zeros((N + 1, ny, nx))
    U0[0] = w.u0
    G0 = np.zeros((N, ny, nx))
    O.coarse_sweep(None, G0, U0)
    U = dev(np.concatenate([w.u0[None], np.zeros((N, ny, nx))]))
    G = P.new_slices()
    P.coarse_sweep(None, G, U)
    torch.cuda.synchronize()
    assert relerr(U.cpu().numpy().reshape(U0.shape), U0) <= TOL
    assert relerr(G.cpu().numpy().reshape(G0.shape), G0) <= TOL


def test_dd2_with_source():
    w = W.small_dd2(60, 31, 2, 0.08, 7, 3, seed=14)
    w.coarse_steps = 2
    rng = np.random.default_rng(3)
    w.forcing = (rng.standard_normal((2, w.ny, w.nx)), rng.standard_normal((2, 7 * 3)),
                 rng.standard_normal((2, 7 * 2)))
    assert fine_parity(w) <= TOL
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    Uo, ko, _ = O.parareal(w.u0, 2)
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL


def test_dd2_manufactured_matches_oracle():
    w = W.dd2_manufactured(n=63, n_slices=8, fine_steps=8, q=2, beta=1.0 / 8)
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=3, tol=0.0)
    torch.cuda.synchronize()
    Uo, ko, _ = O.parareal(w.u0, 3)
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL


def test_dd2_mixed_handle():
    ws = [W.small_dd2(40, 20, 2, 0.1, 4, 2, seed=1), W.small_dim2(37, 29, 6, 3, seed=2),
          W.small_dd1(200, 4, 2, 8, 5, 3, seed=3), W.small_dd2(25, 50, 1, 0.15, 3, 3, seed=4)]
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, ko, _ = oracle_problem(w).parareal(w.u0, 2)
        assert k[i] == ko
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL


def test_dd2_set_coefficients():
    w = W.small_dd2(44, 30, 2, 0.1, 4, 2, seed=5)
    P = gpu_problem(w)
    theta2 = 0.4 * W.smooth_field_2d(w.nx + 2, w.ny + 2, ell=0.2, K=6, seed=99)
    P.set_coefficients(0, dev(theta2))
    w.theta = theta2
    O = oracle_problem(w)
    Uin = slice_inputs(w, seed=1)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


def test_dd2_rejects_bad_partition():
    import paper_2502_08370_amd as pr
    w = W.small_dd2(20, 10, 2, 0.1, 2, 2, seed=6)
    rho = w.rho.copy()
    rho[0, 5] += 0.25  # weights no longer sum to one at that sample
    d = dict(dim=2, nx=20, ny=10, T=0.01, n_slices=2, fine_steps=2, split="dd", theta=w.theta,
             rho=rho)
    with pytest.raises(pr.PrError):
        pr.Problem([d])


def test_dd2_paper_size_one_step_against_the_oracle():
    """h = 1e-3 (999^2), two subdomains of q = 2 vertical strips, beta = 1/16, N = 20
    slices, dt = 2.5e-3 (the paper's DD runs): one FIE step of every slice in the
    benchmark's launch configuration; slice 7 (seeded) compared element by element
    with the oracle (about 40 s of oracle time), the other slices (zero) must stay zero."""
    n, N = 999, 20
    w = W.dd2_manufactured(n=n, n_slices=N, fine_steps=1)
    w.T = N * 2.5e-3
    w.forcing = None
    P = gpu_problem(w)
    O = oracle_problem(w)
    rng = np.random.default_rng(7)
    Uin = np.zeros((N, n, n))
    Uin[7] = W.sine_modes_2d(n, n, seed=7) + 0.01 * rng.standard_normal((n, n))
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    Fo = F.cpu().numpy().reshape(N, n, n)
    print("999^2 strip step on the GPU done; oracle step (~40 s)", flush=True)
    ref = O.fie_step(Uin[7], w.T / N)
    err = relerr(Fo[7], ref)
    print(f"999^2 q=2 beta=1/16: relative error {err:.3e}", flush=True)
    assert err <= TOL
    assert np.abs(np.delete(Fo, 7, axis=0)).max() == 0.0


def test_dd2_fine_error_matches_the_paper_on_gpu():
    """The GPU sequential fine solve of the paper's DD-split scalability runs
    reproduces the fine-approximation error the paper prints (five digits)."""
    import os
    g = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "dd2_fine_error_h001.txt")):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = (t.strip() for t in line.split("="))
            g[k] = float(v)
    n, N, s = int(g["n"]), int(g["n_slices"]), int(g["fine_steps"])
    w = W.dd2_manufactured(n=n, n_slices=N, fine_steps=s, q=int(g["q"]), beta=g["beta"])
    P = gpu_problem(w)
    U = P.new_states()
    P.sequential_fine(dev(w.u0), U)
    torch.cuda.synchronize()
    U = U.cpu().numpy().reshape(N + 1, n, n)
    h = 1.0 / (n + 1)
    err = max(np.sqrt(((U[k] - np.sin(2 * np.pi * k / N) * w.extra["exact_space"]) ** 2).sum()) * h
              for k in range(1, N + 1))
    assert abs(err - g["error"]) <= 0.5e-7

