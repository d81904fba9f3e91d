"""GPU parity: every C-ABI entry point against the oracle on the same seeded
inputs (relative infinity-norm error <= 1e-12, the bound the method's FP64
arithmetic is held to).

Shapes span several fine-sweep chunks with ragged tails (nx, ny not multiples
of the chunk length 32), slice counts that exercise every lane width (1..64)
and padded slice blocks (N = 3, 37, 70), and the degenerate grids n = 1, 2.
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


FINE_CASES = [
    # nx, ny, N, s, variable
    (70, 45, 5, 3, True),
    (33, 97, 1, 4, True),
    (64, 64, 16, 2, True),
    (100, 37, 37, 2, True),
    (47, 31, 64, 3, True),
    (40, 20, 70, 2, True),
    (1, 1, 3, 2, True),
    (2, 5, 2, 3, False),
    (129, 3, 8, 2, True),
    (3, 129, 8, 2, True),
]


@pytest.mark.parametrize("part", [2, 0])
@pytest.mark.parametrize("nx,ny,N,s,var", FINE_CASES)
def test_fine_propagate(nx, ny, N, s, var, part):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=nx + 7 * ny + N, variable=var)
    P, O = gpu_problem(w), oracle_problem(w)
    P.set_option("partitioned", part)
    Uin = slice_inputs(w, seed=N)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


SWEEP_SHAPES = [
    # nx, ny, N: ragged groups of four lines (ny % 4 != 0), one- and two-chunk lines,
    # an odd number of chunks (uneven top and bottom parts), 64-slice and padded blocks
    (70, 45, 64),
    (19, 130, 64),
    (41, 23, 40),
    (100, 37, 3),
]


@pytest.mark.parametrize("twisted,grouped,chunk", [(1, 1, 20), (1, 1, 24), (1, 0, 16), (1, 0, 24),
                                                   (1, 0, 32), (0, 0, 20), (0, 0, 32)])
def test_fine_sweep_variants(twisted, grouped, chunk):
    """Every chunked fine-sweep form (one wave per line; two waves per line from the two ends;
    four lines per workgroup sharing their carry loads) and chunk length against the
    oracle, with and without a source term."""
    for k, (nx, ny, N) in enumerate(SWEEP_SHAPES):
        w = W.small_dim2(nx, ny, n_slices=N, fine_steps=3, seed=50 + k)
        if k == 1:
            src = W.manufactured2d(nx, N, 3)
            w.forcing = src.forcing
            S = np.random.default_rng(k).standard_normal((1, ny, nx))
            w.forcing = (S, src.forcing[1], src.forcing[2])
        P, O = gpu_problem(w), oracle_problem(w)
        P.set_option("partitioned", 0)
        P.set_option("twisted", twisted)
        P.set_option("grouped", grouped)
        P.set_option("fine_chunk", chunk)
        Uin = slice_inputs(w, seed=k)
        F = P.new_slices()
        P.fine_propagate(dev(Uin), F)
        torch.cuda.synchronize()
        ref = O.fine_batch(Uin)
        assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL, (nx, ny, N)


def test_varcoef2d_full_size_sampled():
    """The 1023^2, N = 64, s = 64 workload at its real shape, in the benchmark's
    launch configuration: all 64 slices propagated on the GPU, slices 0, 37 and 63
    compared with the oracle; the coarse propagator's first step of the initial
    guess too."""
    w = W.config2()
    P, O = gpu_problem(w), oracle_problem(w)
    rng = np.random.default_rng(0)
    u0 = np.asarray(w.u0, dtype=np.float64).reshape(w.ny, w.nx)
    Uin = np.stack([u0 * (1 + 0.01 * k) for k in range(w.n_slices)])
    Uin[37] += 0.01 * rng.standard_normal(u0.shape)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    got = F.cpu().numpy().reshape(Uin.shape)
    for k in (0, 37, w.n_slices - 1):
        ref = O.fine(Uin[k])
        assert relerr(got[k], ref.reshape(got[k].shape)) <= TOL, k
    U = P.new_states()
    G = P.new_slices()
    npts = w.nx * w.ny
    U[:npts].copy_(dev(u0))
    P.coarse_sweep(None, G, U)
    torch.cuda.synchronize()
    g1 = U.cpu().numpy()[npts: 2 * npts]
    assert relerr(g1, O.coarse(u0).reshape(-1)) <= TOL


def test_fine_propagate_reaction_and_stiff():
    """c > 0 (split equally over the two substeps) and a stiff fine step."""
    w = W.small_dim2(57, 41, n_slices=4, fine_steps=2, seed=3, c=2.5, T=2.0)
    P, O = gpu_problem(w), oracle_problem(w)
    Uin = slice_inputs(w, seed=1)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("nx,ny,N,cs", [(70, 45, 5, 1), (33, 97, 3, 2), (1, 1, 2, 1), (130, 66, 4, 3)])
def test_coarse_sweep(nx, ny, N, cs):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=2, seed=nx + ny)
    w.coarse_steps = cs
    P, O = gpu_problem(w), oracle_problem(w)
    npts = nx * ny
    rng = np.random.default_rng(5)
    # initial guess
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
    assert inc.item() == 0.0
    # correction sweep with some F
    Fh = U0[1:] + 0.01 * rng.standard_normal((N, ny, nx))
    U1, G1 = U0.copy(), G0.copy()
    inc_ref = O.coarse_sweep(Fh, G1, U1)
    U = dev(U0)
    G = dev(G0)
    P.coarse_sweep(dev(Fh), G, U, inc)
    torch.cuda.synchronize()
    assert relerr(U.cpu().numpy().reshape(U1.shape), U1) <= TOL
    assert relerr(G.cpu().numpy().reshape(G1.shape), G1) <= TOL
    assert abs(inc.item() - inc_ref) <= TOL * max(inc_ref, np.abs(U1).max())


@pytest.mark.parametrize("nx,ny,N,s,K", [(37, 29, 6, 5, 3), (64, 48, 8, 4, 8), (20, 70, 3, 2, 5)])
def test_parareal_iterate(nx, ny, N, s, K):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=N * s)
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=K, tol=0.0)
    torch.cuda.synchronize()
    Uo, ko, hist = O.parareal(w.u0, K)
    assert k[0] == ko
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL
    assert abs(inc[0] - hist[-1]) <= TOL * np.abs(Uo).max()


def test_parareal_tolerance_stop():
    w = W.small_dim2(45, 45, n_slices=10, fine_steps=4, seed=2)
    P, O = gpu_problem(w), oracle_problem(w)
    _, _, hist = O.parareal(w.u0, 10)
    tol = float(np.sqrt(hist[3] * hist[4]))  # between two increments: stop after 5
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=10, tol=tol)
    Uo, ko, h2 = O.parareal(w.u0, 10, tol)
    assert k[0] == ko == 5
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL


def test_config1_closed_form_and_finite_termination():
    """Config 1 end to end: K = N = 8 iterations reach the sequential fine solution
    (section 3), whose amplitude is the closed form R_F^(N s) of eq. stab_func_FIE."""
    w = W.config1()
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=8, tol=0.0)
    Seq = P.new_states()
    P.sequential_fine(dev(w.u0), Seq)
    torch.cuda.synchronize()
    Uo, _, _ = O.parareal(w.u0, 8)
    got = U.cpu().numpy().reshape(Uo.shape)
    assert relerr(got, Uo) <= TOL
    assert relerr(Seq.cpu().numpy().reshape(Uo.shape), Uo) <= TOL
    h = 1 / 33
    lam = 4 / h ** 2 * np.sin(np.pi * h / 2) ** 2
    amp = (1 / (1 + 0.1 / 8 / 16 * lam) ** 2) ** (8 * 16)
    assert relerr(got[-1], amp * w.u0) <= 1e-12


@pytest.mark.parametrize("nx,ny,N,s", [(37, 29, 4, 3), (65, 33, 2, 2)])
def test_sequential_fine(nx, ny, N, s):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=11)
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    P.sequential_fine(dev(w.u0), U)
    torch.cuda.synchronize()
    ref = O.sequential_fine(w.u0)
    assert relerr(U.cpu().numpy().reshape(ref.shape), ref) <= TOL


def test_batched_instances_match_single():
    """Several uneven instances in one handle give the same result as one handle each."""
    ws = [W.small_dim2(37, 29, 6, 3, seed=1), W.small_dim2(64, 64, 16, 3, seed=2),
          W.small_dim2(20, 50, 3, 3, seed=3), W.small_dim2(90, 15, 64, 3, seed=4)]
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, ko, _ = oracle_problem(w).parareal(w.u0, 2)
        got = P.view(U, i, "states").cpu().numpy()
        assert k[i] == ko
        assert relerr(got, Uo) <= TOL


def test_invalid_arguments_rejected():
    import paper_2502_08370_amd as pr
    w = W.small_dim2(8, 8, 2, 2, seed=0)
    d = dict(dim=2, nx=8, ny=8, T=-1.0, n_slices=2, fine_steps=2, theta=w.theta)
    with pytest.raises(pr.PrError) as e:
        pr.Problem([d])
    assert e.value.status == 1
    d["T"] = 0.1
    d["n_slices"] = 0
    with pytest.raises(pr.PrError):
        pr.Problem([d])


def test_profile_span_mode_counts():
    """Span-mode phase timers: one event pair per loop, the launch counts of the
    per-launch mode, and results unchanged by either mode."""
    w = W.small_dim2(40, 33, n_slices=6, fine_steps=3, seed=9)
    P = gpu_problem(w)
    Uin = dev(slice_inputs(w, seed=2))
    counts = {}
    outs = []
    for mode in (1, 3):
        P.profile(2)
        P.profile(mode)
        F = P.new_slices()
        P.fine_propagate(Uin, F)
        U = P.new_states()
        U[: w.nx * w.ny].copy_(dev(w.u0))
        G = P.new_slices()
        inc = torch.zeros(1, dtype=torch.float64, device="cuda")
        P.coarse_sweep(F, G, U, inc)
        torch.cuda.synchronize()
        P.profile(0)
        counts[mode] = {k: v[1] for k, v in P.profile_read().items()}
        outs.append((F.clone(), U.clone()))
    assert counts[1]["fine_sweep"] == counts[3]["fine_sweep"] == 2 * w.fine_steps
    assert counts[1]["coarse_x"] == counts[1]["coarse_y"] == w.n_slices
    assert counts[3]["coarse_sweep"] == 2 * w.n_slices and "coarse_x" not in counts[3]
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    import paper_2502_08370_amd as pr
    with pytest.raises(pr.PrError):
        P.profile(4)
