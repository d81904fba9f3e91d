"""Oracle checks at the full workload sizes, in the launch configurations the
benchmark uses (section 3, the parareal iteration):

* the coarse sweep with the fused correction and increment (U_{n+1} = F_n +
  G(U_n) - G_old_n) on the 1023^2, N = 64 workload, every state compared: the
  coarse lines are 1023 long, 16 positions per lane;
* the batch workload's instance shapes (n = 511 with N = 64, n = 255 with
  N = 16, beside 63^2 and 127^2 instances) in one handle, two parareal
  corrections against the oracle iteration;
* one handle mixing fine-step counts (the grouped sweeps skip instances whose
  steps are done), a Douglas-Rachford instance, a source-term instance and a
  reaction term, against the oracle instance by instance.
"""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import TOL, gpu_problem, oracle_problem, parareal_threaded, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda").reshape(-1)


def test_varcoef2d_full_size_correction_sweep():
    w = W.config2()
    P, O = gpu_problem(w), oracle_problem(w)
    N, shape = w.n_slices, (w.ny, w.nx)
    u0 = np.asarray(w.u0, dtype=np.float64).reshape(shape)
    # the oracle's initial guess, then a seeded fine-propagator stand-in
    U0 = np.empty((N + 1,) + shape)
    U0[0] = u0
    G0 = np.empty((N,) + shape)
    O.coarse_sweep(None, G0, U0)
    rng = np.random.default_rng(11)
    Fh = U0[1:] * (1.0 + 0.02 * rng.standard_normal((N, 1, 1))) \
        + 1e-3 * rng.standard_normal((N,) + shape)
    U1, G1 = U0.copy(), G0.copy()
    inc_ref = O.coarse_sweep(Fh, G1, U1)
    U, G = dev(U0), dev(G0)
    inc = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    P.coarse_sweep(dev(Fh), G, U, inc)
    torch.cuda.synchronize()
    assert relerr(U.cpu().numpy().reshape(U1.shape), U1) <= TOL
    assert relerr(G.cpu().numpy().reshape(G1.shape), G1) <= TOL
    assert abs(inc.item() - inc_ref) <= TOL * np.abs(U1).max()
    assert inc_ref > 0


def test_batch_workload_shapes_two_corrections():
    shapes = [(511, 64), (63, 32), (255, 16), (127, 64), (63, 16)]
    ws = [W.batch_instance(i, n, N) for i, (n, N) in enumerate(shapes)]
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        print(f"instance {i}: {w.nx}^2, N={w.n_slices}", flush=True)
        Uo, hist = parareal_threaded(oracle_problem(w), w.u0, 2)
        assert k[i] == 2
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL
        assert abs(inc[i] - hist[-1]) <= TOL * np.abs(Uo).max()


def test_batch_mixed_steps_integrators_and_sources():
    ws = [W.small_dim2(70, 45, n_slices=6, fine_steps=3, seed=21),
          W.small_dim2(40, 66, n_slices=5, fine_steps=7, seed=22, c=1.5),
          W.small_dim2(33, 33, n_slices=8, fine_steps=1, seed=23)]
    dr = W.small_dim2(50, 41, n_slices=4, fine_steps=5, seed=24)
    dr.fine = "dr"
    src = W.manufactured2d(47, 6, 4)
    src.theta = 0.3 * W.smooth_field_2d(49, 49, ell=0.2, K=6, seed=25)
    ws += [dr, src]
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 + 0.05 for w in ws])
    for K in (1, 3):
        U = P.new_states()
        k, inc = P.parareal_iterate(u0, U, k_max=K, tol=0.0)
        torch.cuda.synchronize()
        for i, w in enumerate(ws):
            Uo, ko, hist = oracle_problem(w).parareal(w.u0 + 0.05, K)
            assert k[i] == ko == K
            assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL, (K, i)
            assert abs(inc[i] - hist[-1]) <= TOL * np.abs(Uo).max()
