"""GPU parity of the source terms (F(t) = sum_m g_m(t) S_m on the first stage of
eq. FIE_method / eq. DR_method) against the oracle: the fine map over all
slices (FIE and DR, every lane width), the sequential fine solve, the coarse
sweep, parareal, forced and unforced instances in one handle, the DD
splitting, and the adjoint's forward recompute. Relative infinity-norm error
<= 1e-12. Also the paper's manufactured test problem (section 5): the GPU
solution's error against the exact solution matches the oracle's at a small
size and keeps falling with refinement at a large one."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import TOL, gpu_problem, oracle_problem, relerr, slice_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda").reshape(-1)


def random_forcing(ny, nx, N, s, cs, m, seed):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((m, ny, nx)) * 10.0
    return (S, rng.standard_normal((m, N * s)), rng.standard_normal((m, N * cs)))


def forced(nx, ny, N, s, m=2, fine="fie", seed=0, c=0.0, cs=1):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=seed, c=c)
    w.coarse_steps = cs
    w.fine = fine
    w.forcing = random_forcing(ny, nx, N, s, cs, m, seed + 100)
    return w


@pytest.mark.parametrize("nx,ny,N,s,m,fine", [(70, 45, 5, 3, 2, "fie"), (33, 97, 1, 4, 1, "fie"),
                                              (47, 31, 64, 3, 2, "dr"), (40, 20, 70, 2, 1, "dr"),
                                              (1, 1, 3, 2, 2, "fie")])
def test_forced_fine_propagate(nx, ny, N, s, m, fine):
    w = forced(nx, ny, N, s, m=m, fine=fine, seed=nx + N)
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=N)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("part", [2, 0])
@pytest.mark.parametrize("lanes,chunk", [(8, 16), (16, 32), (32, 16), (64, 32)])
def test_forced_layouts(lanes, chunk, part):
    w = forced(75, 66, 64, 2, fine="fie", seed=3, c=0.5)
    P, O = gpu_problem(w), oracle_problem(w)
    P.set_option("partitioned", part)
    P.set_option("lanes", lanes)
    P.set_option("fine_chunk", chunk)
    Uin = slice_inputs(w, seed=2)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("fine", ["fie", "dr"])
def test_forced_sequential_and_parareal(fine):
    w = forced(37, 29, 6, 4, fine=fine, seed=5, cs=2)
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
    assert abs(inc[0] - hist[-1]) <= TOL * np.abs(Uo).max()


def test_forced_coarse_sweep():
    w = forced(70, 45, 5, 2, seed=8, cs=3)
    P, O = gpu_problem(w), oracle_problem(w)
    N, nx, ny = 5, 70, 45
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


def test_forced_and_unforced_in_one_handle():
    ws = [forced(37, 29, 6, 3, seed=1), W.small_dim2(37, 29, 6, 3, seed=1),
          forced(64, 20, 16, 2, m=1, fine="dr", seed=2), W.small_dim2(20, 50, 3, 3, seed=3)]
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, ko, _ = oracle_problem(w).parareal(w.u0, 2)
        assert k[i] == ko
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL


@pytest.mark.parametrize("n,cores,colors,ov,N,s", [(200, 4, 2, 8, 5, 3), (640, 5, 5, 8, 3, 2)])
def test_forced_dd(n, cores, colors, ov, N, s):
    w = W.small_dd1(n, cores, colors, ov, n_slices=N, fine_steps=s, seed=n, T=1e-3)
    w.coarse_steps = 2
    w.forcing = random_forcing(1, n, N, s, 2, 2, n)
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=4)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL
    seq = O.sequential_fine(w.u0)
    assert relerr(Seq.cpu().numpy().reshape(seq.shape), seq) <= TOL
    Uo, ko, _ = O.parareal(w.u0, 2)
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL


def test_forced_adjoint_matches_oracle():
    import oracle
    nx, ny, N, s = 23, 17, 3, 4
    w = forced(nx, ny, N, s, seed=6)
    P, O = gpu_problem(w), oracle_problem(w)
    lam = np.random.default_rng(9).standard_normal((ny, nx))
    g0 = torch.empty(nx * ny, dtype=torch.float64, device="cuda")
    gc = torch.empty((nx + 2) * (ny + 2), dtype=torch.float64, device="cuda")
    ck = P.new_states()
    P.adjoint(dev(w.u0), dev(lam), g0, gc, ck)
    torch.cuda.synchronize()
    rg0, rgax, rgay = O.adjoint(w.u0, lam)
    assert relerr(g0.cpu().numpy().reshape(ny, nx), rg0) <= TOL
    rth = oracle.theta_grad(nx, ny, w.theta, rgax, rgay)
    assert relerr(gc.cpu().numpy().reshape(ny + 2, nx + 2), rth) <= TOL
    seq = O.sequential_fine(w.u0)
    assert relerr(ck.cpu().numpy().reshape(seq.shape), seq) <= TOL


def _manufactured_error(U, w):
    n = w.nx
    DT = w.T / w.n_slices
    exact = np.stack([np.sin(2 * np.pi * k * DT) * w.extra["exact_space"]
                      for k in range(w.n_slices + 1)])
    return np.sqrt(((U - exact) ** 2).sum(axis=(1, 2)) / (n + 1) ** 2).max()


def test_manufactured_problem_matches_oracle():
    """Section 5 test problem at a size the oracle runs quickly: the GPU
    sequential fine and converged parareal solutions equal the oracle's."""
    w = W.manufactured2d(63, 8, 16)
    P, O = gpu_problem(w), oracle_problem(w)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=8, tol=0.0)
    torch.cuda.synchronize()
    ref = O.sequential_fine(w.u0)
    seq = Seq.cpu().numpy().reshape(ref.shape)
    assert relerr(seq, ref) <= TOL
    assert relerr(U.cpu().numpy().reshape(ref.shape), ref) <= TOL
    assert abs(_manufactured_error(seq, w) - _manufactured_error(ref, w)) <= 1e-12


def test_manufactured_problem_converges_on_gpu():
    """With dt proportional to h^2 the error against the exact solution falls
    by about 4 per halving of h, up to 511^2 (section 5 error measure)."""
    errs = []
    for n, s in [(127, 4), (255, 16), (511, 64)]:
        w = W.manufactured2d(n, 8, s)
        P = gpu_problem(w)
        Seq = P.new_states()
        P.sequential_fine(dev(w.u0), Seq)
        torch.cuda.synchronize()
        errs.append(_manufactured_error(Seq.cpu().numpy().reshape(9, n, n), w))
    assert errs[0] > errs[1] > errs[2]
    assert 3.0 < errs[1] / errs[2] < 4.6
