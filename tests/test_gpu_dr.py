"""GPU parity of the Douglas-Rachford fine propagator (eq. DR_method) against the
oracle: the batched fine map over all slices, the sequential fine solve,
parareal with a DR fine and FIE coarse propagator (the FIE-DR pairing of
section 4), DR and FIE instances in one handle, and every lane width / chunk
length of the fine sweep. Relative infinity-norm error <= 1e-12.
"""
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


def dr(nx, ny, N, s, seed=0, c=0.0, variable=True, T=0.05):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=seed, variable=variable, c=c, T=T)
    w.fine = "dr"
    return w


@pytest.mark.parametrize("nx,ny,N,s,c", [
    (70, 45, 5, 3, 0.0),
    (33, 97, 1, 4, 1.5),
    (47, 31, 64, 3, 0.0),
    (40, 20, 70, 2, 3.0),
    (1, 1, 3, 2, 0.0),
    (2, 5, 2, 3, 0.5),
    (129, 3, 8, 2, 0.0),
    (3, 129, 8, 2, 0.0),
])
def test_dr_fine_propagate(nx, ny, N, s, c):
    w = dr(nx, ny, N, s, seed=nx + ny + N, c=c)
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=N)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


def test_dr_differs_from_fie():
    """The DR and FIE maps are different methods (same factors): guards against a
    DR flag that is silently ignored."""
    w = dr(37, 29, 4, 2, seed=5)
    f = W.small_dim2(37, 29, n_slices=4, fine_steps=2, seed=5)
    Uin = slice_inputs(w, seed=2)
    Pd, Pf = gpu_problem(w), gpu_problem(f)
    Fd, Ff = Pd.new_slices(), Pf.new_slices()
    Pd.fine_propagate(dev(Uin), Fd)
    Pf.fine_propagate(dev(Uin), Ff)
    torch.cuda.synchronize()
    assert relerr(Fd.cpu().numpy(), Ff.cpu().numpy()) > 1e-6


@pytest.mark.parametrize("lanes,chunk", [(8, 16), (16, 32), (32, 16), (64, 32)])
def test_dr_layouts(lanes, chunk):
    w = dr(75, 66, 64, 3, seed=9, c=1.0)
    P, O = gpu_problem(w), oracle_problem(w)
    P.set_option("lanes", lanes)
    P.set_option("fine_chunk", chunk)
    Uin = slice_inputs(w, seed=3)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


def test_dr_block_passes():
    """Slice blocks processed in passes (the stencil covers only the pass's blocks)."""
    w = dr(50, 40, 70, 3, seed=4)
    P, O = gpu_problem(w), oracle_problem(w)
    P.set_option("lanes", 8)
    P.set_option("blocks_per_pass", 3)
    Uin = slice_inputs(w, seed=6)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("nx,ny,N,s", [(37, 29, 4, 3), (65, 33, 2, 2)])
def test_dr_sequential_fine(nx, ny, N, s):
    w = dr(nx, ny, N, s, seed=11, c=0.7)
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    P.sequential_fine(dev(w.u0), U)
    torch.cuda.synchronize()
    ref = O.sequential_fine(w.u0)
    assert relerr(U.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("nx,ny,N,s,K", [(37, 29, 6, 5, 3), (64, 48, 8, 4, 8)])
def test_dr_parareal(nx, ny, N, s, K):
    w = dr(nx, ny, N, s, seed=N * s)
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=K, tol=0.0)
    torch.cuda.synchronize()
    Uo, ko, hist = O.parareal(w.u0, K)
    assert k[0] == ko
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL
    assert abs(inc[0] - hist[-1]) <= TOL * np.abs(Uo).max()


def test_dr_parareal_reaches_sequential_dr():
    """K = N iterations reproduce the sequential DR fine solution (section 3)."""
    w = dr(33, 33, 5, 4, seed=1, c=0.5)
    P = gpu_problem(w)
    U = P.new_states()
    P.parareal_iterate(dev(w.u0), U, k_max=5, tol=0.0)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    torch.cuda.synchronize()
    assert relerr(U.cpu().numpy(), Seq.cpu().numpy()) <= TOL


def test_dr_and_fie_in_one_handle():
    ws = [dr(37, 29, 6, 3, seed=1), W.small_dim2(37, 29, 6, 3, seed=1),
          dr(64, 20, 16, 2, seed=2, c=1.0), W.small_dim2(20, 50, 3, 3, seed=3)]
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, ko, _ = oracle_problem(w).parareal(w.u0, 2)
        assert k[i] == ko
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL


def test_dr_adjoint_rejected():
    import paper_2502_08370_amd as pr
    w = dr(16, 16, 2, 2, seed=0)
    P = gpu_problem(w)
    lam = torch.zeros(w.nx * w.ny, dtype=torch.float64, device="cuda")
    gu = torch.zeros_like(lam)
    gc = torch.zeros((w.nx + 2) * (w.ny + 2), dtype=torch.float64, device="cuda")
    with pytest.raises(pr.PrError) as e:
        P.adjoint(dev(w.u0), lam, gu, gc)
    assert "FIE" in str(e.value)
