"""GPU parity of the domain-decomposition splitting in 1D (section 2.1 partition
of unity, eq. FIE_method substeps in colour order) against the oracle.

Cases: 2 colours x q components (the alternating strips of the paper's
decomposition), M colours with one component each, ragged segment tails
(component lengths not multiples of 64), slice counts padded to the lane
width, and the full 2^20-node workload (every slice propagated on the GPU,
two sampled slices checked against the oracle)."""
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


DD_CASES = [
    # n, cores, colours, overlap, N, s, T
    (200, 4, 2, 8, 5, 3, 1e-3),
    (1000, 8, 2, 32, 32, 4, 1e-4),
    (640, 5, 5, 8, 3, 2, 1e-3),
    (640, 8, 8, 8, 1, 3, 1e-3),
    (130, 2, 2, 8, 9, 2, 1e-2),
    (4096, 8, 2, 32, 70, 2, 2.0 ** -12),
]


@pytest.mark.parametrize("n,cores,colors,ov,N,s,T", DD_CASES)
def test_dd_fine_propagate(n, cores, colors, ov, N, s, T):
    w = W.small_dd1(n, cores, colors, ov, n_slices=N, fine_steps=s, seed=n + N, T=T)
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=3)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("n,cores,colors,ov,N,s,T", DD_CASES[:4])
def test_dd_parareal_and_sequential(n, cores, colors, ov, N, s, T):
    w = W.small_dd1(n, cores, colors, ov, n_slices=N, fine_steps=s, seed=n, T=T)
    P, O = gpu_problem(w), oracle_problem(w)
    K = min(N, 3)
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


def test_dd_finite_termination():
    """Section 3: K = N iterations reproduce the sequential fine solution."""
    w = W.small_dd1(512, 4, 2, 16, n_slices=4, fine_steps=3, seed=8, T=1e-3)
    P = gpu_problem(w)
    U = P.new_states()
    P.parareal_iterate(dev(w.u0), U, k_max=4, tol=0.0)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    torch.cuda.synchronize()
    ref = oracle_problem(w).sequential_fine(w.u0)
    assert relerr(U.cpu().numpy().reshape(ref.shape), ref) <= TOL
    assert relerr(Seq.cpu().numpy().reshape(ref.shape), ref) <= TOL


def test_dd_full_size_sampled():
    """The 2^20-node, 8-component, 32-slice workload at its real shape: all
    slices propagated (s = 128) in the benchmark's launch configuration, slices
    0 and 31 compared with the oracle; the coarse propagator on slice 0 too."""
    w = W.config3()
    P, O = gpu_problem(w), oracle_problem(w)
    rng = np.random.default_rng(0)
    Uin = np.stack([w.u0 * (1 + 0.1 * k) for k in range(w.n_slices)])
    Uin[5] += 0.01 * rng.standard_normal(w.nx)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    got = F.cpu().numpy().reshape(Uin.shape)
    for k in (0, w.n_slices - 1):
        ref = O.fine(Uin[k])
        assert relerr(got[k], ref) <= TOL, k
    # coarse: the initial guess' first step
    U = P.new_states()
    G = P.new_slices()
    U[: w.nx].copy_(dev(w.u0))
    P.coarse_sweep(None, G, U)
    torch.cuda.synchronize()
    g1 = U.cpu().numpy()[w.nx: 2 * w.nx]
    assert relerr(g1, O.coarse(w.u0)) <= TOL


def random_pou(n, n_colors, seed, max_cover=3):
    """Random partition of unity: every face gets a random set of 1..max_cover
    colours with positive weights summing to 1. Components are short and
    fragmented, nodes are covered by up to max_cover + 1 colours, and colours
    meet in every order: the hard cases for the deferred-correction sources."""
    rng = np.random.default_rng(seed)
    rho = np.zeros((n_colors, n + 1))
    for f in range(n + 1):
        k = rng.integers(1, min(max_cover, n_colors) + 1)
        cols = rng.choice(n_colors, size=k, replace=False)
        wts = rng.random(k) + 0.05
        rho[cols, f] = wts / wts.sum()
    rho /= rho.sum(axis=0, keepdims=True)
    return rho


@pytest.mark.parametrize("n,colors,N,s,seed", [(300, 3, 3, 3, 1), (517, 4, 40, 2, 2),
                                               (129, 2, 9, 4, 3), (700, 5, 5, 2, 4)])
def test_dd_random_partition(n, colors, N, s, seed):
    w = W.small_dd1(n, 1, 1, 0, n_slices=N, fine_steps=s, seed=seed, T=1e-3)
    w.rho = random_pou(n, colors, seed)
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=5)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    Uo, ko, _ = O.parareal(w.u0, 2)
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL
