"""Lines longer than one segment of the one-wave-per-line solvers (1024
positions) and longer than the fine sweeps' LDS chunk store, under dimensional
splitting (section 2.2, eq. FIE_method: the substep line solves have no length
bound): every entry point against the oracle at 1e-12, for x lines and y lines,
one segment plus a ragged tail, exact multiples of the segment, and three
segments."""
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


LONG_SHAPES = [
    # nx, ny, N: x lines of one segment + 76, y lines of three segments (ragged),
    # exact two segments, one position past one segment
    (1100, 37, 64),
    (29, 2100, 3),
    (9, 2048, 64),
    (1025, 9, 5),
    # degenerate: one long line and lines of one point
    (3000, 1, 5),
    (1, 2049, 64),
]


@pytest.mark.parametrize("twisted,grouped,chunk", [(1, 1, 20), (1, 0, 32), (0, 0, 24)])
def test_fine_propagate_long_lines(twisted, grouped, chunk):
    for k, (nx, ny, N) in enumerate(LONG_SHAPES):
        w = W.small_dim2(nx, ny, n_slices=N, fine_steps=2, seed=70 + k)
        P, O = gpu_problem(w), oracle_problem(w)
        P.set_option("twisted", twisted)
        P.set_option("grouped", grouped)
        P.set_option("fine_chunk", chunk)
        Uin = slice_inputs(w, seed=k)
        F = P.new_slices()
        P.fine_propagate(dev(Uin), F)
        torch.cuda.synchronize()
        ref = O.fine_batch(Uin)
        assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL, (nx, ny, N)


@pytest.mark.parametrize("nx,ny,N,cs,T", [(1100, 40, 3, 2, 0.05), (40, 2100, 2, 1, 0.05),
                                           (1030, 1025, 2, 1, 0.05), (3000, 1, 2, 1, 1e-4),
                                           (1, 3000, 2, 2, 1e-4)])
def test_coarse_sweep_long_lines(nx, ny, N, cs, T):
    """Initial guess (mode 2) and correction with increment (mode 1) with the
    coarse y solve of the last coarse step fused, on segmented rows and columns.
    The one-point-wide grids take a moderate step (tau / h^2 about 225): at
    T = 0.05 the 3000-point lines' coarse step has tau / h^2 = 1.1e5, where two
    exact eliminations of one line agree only to about 2e-12."""
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=2, seed=nx + ny, T=T)
    w.coarse_steps = cs
    P, O = gpu_problem(w), oracle_problem(w)
    U0 = np.zeros((N + 1, ny, nx))
    U0[0] = w.u0
    G0 = np.zeros((N, ny, nx))
    O.coarse_sweep(None, G0, U0)
    U = dev(np.concatenate([w.u0[None], np.zeros((N, ny, nx))]))
    G = P.new_slices()
    inc = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    P.coarse_sweep(None, G, U, inc)
    torch.cuda.synchronize()
    assert relerr(U.cpu().numpy().reshape(U0.shape), U0) <= TOL
    assert relerr(G.cpu().numpy().reshape(G0.shape), G0) <= TOL
    rng = np.random.default_rng(5)
    Fh = U0[1:] + 0.01 * rng.standard_normal((N, ny, nx))
    U1, G1 = U0.copy(), G0.copy()
    inc_ref = O.coarse_sweep(Fh, G1, U1)
    U, G = dev(U0), dev(G0)
    P.coarse_sweep(dev(Fh), G, U, inc)
    torch.cuda.synchronize()
    assert relerr(U.cpu().numpy().reshape(U1.shape), U1) <= TOL
    assert relerr(G.cpu().numpy().reshape(G1.shape), G1) <= TOL
    assert abs(inc.item() - inc_ref) <= TOL * max(inc_ref, np.abs(U1).max())


@pytest.mark.parametrize("nx,ny,N,s,K", [(1300, 50, 6, 3, 3), (45, 3000, 4, 2, 2)])
def test_parareal_long_lines(nx, ny, N, s, K):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=N * s + 1)
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=K, tol=0.0)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    torch.cuda.synchronize()
    Uo, ko, hist = O.parareal(w.u0, K)
    assert k[0] == ko
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL
    assert abs(inc[0] - hist[-1]) <= TOL * np.abs(Uo).max()
    ref = O.sequential_fine(w.u0)
    assert relerr(Seq.cpu().numpy().reshape(ref.shape), ref) <= TOL


def test_douglas_rachford_long_lines():
    w = W.small_dim2(1100, 33, n_slices=4, fine_steps=3, seed=9)
    w.fine = "dr"
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=3)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("parallel,N", [(False, 3), (True, 3), (True, 64)])
def test_adjoint_long_lines(parallel, N):
    """Serial and parallel-in-time adjoints on 1100-point x lines; with 64 slices the
    parallel adjoint's recomputed forward steps take the grouped sweeps' long-line
    variant."""
    nx, ny = 1100, 21
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=2, seed=4)
    theta = w.theta
    P, O = gpu_problem(w), oracle_problem(w)
    lam = np.random.default_rng(4).standard_normal((ny, nx))
    g0 = torch.empty(nx * ny, dtype=torch.float64, device="cuda")
    gc = torch.empty((nx + 2) * (ny + 2), dtype=torch.float64, device="cuda")
    ck = P.new_states()
    if parallel:
        P.adjoint_parallel(dev(w.u0), dev(lam), g0, gc, ck)
    else:
        P.adjoint(dev(w.u0), dev(lam), g0, gc, ck)
    torch.cuda.synchronize()
    rg0, rgax, rgay = O.adjoint(w.u0, lam)
    assert relerr(g0.cpu().numpy().reshape(ny, nx), rg0) <= TOL
    rth = oracle.theta_grad(nx, ny, theta, rgax, rgay)
    assert relerr(gc.cpu().numpy().reshape(ny + 2, nx + 2), rth) <= TOL


def test_long_and_short_instances_in_one_handle():
    ws = [W.small_dim2(1100, 20, 5, 2, seed=1), W.small_dim2(30, 40, 8, 2, seed=2),
          W.small_dim2(17, 1500, 3, 2, seed=3)]
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, ko, _ = oracle_problem(w).parareal(w.u0, 2)
        assert k[i] == ko
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL


@pytest.mark.parametrize("fine,nx,ny,N", [("fie", 1100, 37, 64), ("fie", 29, 2100, 3),
                                          ("dr", 1100, 37, 4), ("dr", 33, 1500, 5)])
def test_source_term_long_lines(fine, nx, ny, N):
    """A source term (random spatial factor, the manufactured problem's time factors)
    on lines longer than one segment: the fine propagation of every slice and two
    parareal corrections against the oracle."""
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=2, seed=nx + ny + N)
    w.fine = fine
    src = W.manufactured2d(8, N, 2)
    S = np.random.default_rng(N).standard_normal((1, ny, nx))
    w.forcing = (S, src.forcing[1], src.forcing[2])
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=1)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL
    Uo, ko, _ = O.parareal(w.u0, 2)
    assert k[0] == ko
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL
