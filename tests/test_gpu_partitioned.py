"""Partitioned fine sweeps (few slices: a whole line of a slice block held by one
workgroup, cut into parts that are solved side by side and joined exactly;
section 2.2, eq. FIE_method: each substep is an exact solve of its line
systems) against the oracle at 1e-12: one, several and a ragged last slice block
(N = 1, 3, 20, 23, and with the form forced, 37 and 70), lines from 1 to 1024
positions in both directions, a
source term, the parareal iteration around them, a handle mixing instances that
take them with instances that do not, and the paper's 999^2, N = 20 size with
sampled slices (its 20-step run at a bound scaled by the line systems' condition
number, see test_partitioned_paper_size_sampled)."""
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


PART_SHAPES = [
    # nx, ny, N, s: one block of 20 slices (three parts per wave); 23 slices in blocks
    # of 12 and 11; 37 slices in blocks of 19 and 18, 70 in blocks of 24, 24 and 22
    # (more than 24 slices: the form forced); lines of 1, 2, 1000 and 1024 positions
    # (blocks of 10 slices for 20, 21 parts per wave for 3 slices)
    (120, 90, 20, 3),
    (700, 50, 23, 2),
    (300, 200, 37, 2),
    (200, 150, 70, 2),
    (1, 1, 3, 2),
    (2, 5, 2, 3),
    (1000, 7, 3, 2),
    (7, 1000, 20, 2),
    (1024, 33, 20, 2),
    (45, 1024, 1, 2),
]


@pytest.mark.parametrize("nx,ny,N,s", PART_SHAPES)
def test_partitioned_fine_propagate(nx, ny, N, s):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=nx + 3 * ny + N)
    P, O = gpu_problem(w), oracle_problem(w)
    if N > 24:
        P.set_option("partitioned", 2)
    assert P.get_option("partitioned_used") == 1
    Uin = slice_inputs(w, seed=N)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("nx,ny,N", [(120, 90, 20), (333, 40, 37), (64, 1000, 5)])
def test_partitioned_source_term(nx, ny, N):
    """The source enters the x sweep's right-hand side (the step's end time, each
    slice's own time factors)."""
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=3, seed=N)
    src = W.manufactured2d(8, N, 3)
    S = np.random.default_rng(N).standard_normal((2, ny, nx))
    g2 = np.stack([src.forcing[1][0], np.cos(np.arange(src.forcing[1].shape[1]))])
    gc = np.stack([src.forcing[2][0], np.ones(src.forcing[2].shape[1])])
    w.forcing = (S, g2, gc)
    P, O = gpu_problem(w), oracle_problem(w)
    P.set_option("partitioned", 2)
    assert P.get_option("partitioned_used") == 1
    Uin = slice_inputs(w, seed=2)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    ref = O.fine_batch(Uin)
    assert relerr(F.cpu().numpy().reshape(ref.shape), ref) <= TOL


@pytest.mark.parametrize("N,cs", [(20, 1), (7, 2)])
def test_partitioned_parareal(N, cs):
    w = W.small_dim2(150, 110, n_slices=N, fine_steps=4, seed=11)
    w.coarse_steps = cs
    P, O = gpu_problem(w), oracle_problem(w)
    U = P.new_states()
    k, inc = P.parareal_iterate(dev(w.u0), U, k_max=3, tol=0.0)
    torch.cuda.synchronize()
    Uo, ko, hist = O.parareal(w.u0, 3)
    assert k[0] == ko
    assert relerr(U.cpu().numpy().reshape(Uo.shape), Uo) <= TOL
    assert abs(inc[0] - hist[-1]) <= TOL * np.abs(Uo).max()


def test_partitioned_and_chunked_in_one_handle():
    """Instances that take the partitioned sweeps (20 and 3 slices), one that does
    not (1100-point lines) and a Douglas-Rachford one (chunked sweeps) advance
    together; the graph-captured correction replays both forms."""
    ws = [W.small_dim2(130, 70, 20, 3, seed=1), W.small_dim2(1100, 30, 64, 2, seed=2),
          W.small_dim2(60, 90, 3, 3, seed=3), W.small_dim2(50, 45, 20, 2, seed=4)]
    ws[3].fine = "dr"
    P = gpu_problem(ws)
    assert P.get_option("partitioned_used") == 2
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=3, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, ko, _ = oracle_problem(w).parareal(w.u0, 3)
        assert k[i] == ko
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL


def test_partitioned_default_rule():
    """By default the partitioned sweeps serve instances of at most 24 slices whose
    lines fit a workgroup; option 2 extends them to every instance whose lines fit,
    option 0 turns them off, and the usage count follows each setting."""
    ws = [W.small_dim2(300, 200, 24, 2, seed=1), W.small_dim2(300, 200, 32, 2, seed=2),
          W.small_dim2(1100, 20, 8, 2, seed=3)]
    P = gpu_problem(ws)
    assert P.get_option("partitioned") == 1 and P.get_option("partitioned_used") == 1
    P.set_option("partitioned", 2)
    assert P.get_option("partitioned_used") == 2
    P.set_option("partitioned", 0)
    assert P.get_option("partitioned_used") == 0
    with pytest.raises(Exception):
        P.set_option("partitioned", 3)


def test_partitioned_matches_chunked_form():
    """The two sweep forms solve the same systems: their fine maps agree to rounding
    (both are also held to the oracle above)."""
    w = W.small_dim2(257, 190, n_slices=20, fine_steps=5, seed=8)
    P = gpu_problem(w)
    Uin = dev(slice_inputs(w, seed=4))
    F1, F0 = P.new_slices(), P.new_slices()
    P.fine_propagate(Uin, F1)
    P.set_option("partitioned", 0)
    assert P.get_option("partitioned_used") == 0
    with pytest.raises(Exception):
        P.set_option("partitioned_used", 1)
    P.fine_propagate(Uin, F0)
    torch.cuda.synchronize()
    assert relerr(F1.cpu().numpy(), F0.cpu().numpy()) <= TOL


@pytest.mark.parametrize("case", ["paper_step", "paper_run", "variable"])
def test_partitioned_paper_size_sampled(case):
    """999^2, N = 20 (the paper's section 5 runs) in the benchmark's launch
    configuration: all slices propagated on the GPU, slices 0, 9 and 19 compared
    with the oracle. The slice inputs are smooth states of order one (slice 9 with
    added white noise of 1e-2).

    paper_step: one fine step at the paper's dt = 2.5e-3 (T = 0.05, s = 1), at
    1e-12. paper_run: the paper's s = 20 steps; each line system there has
    tau / h^2 = 2500 and condition number 1 + 4 tau / h^2 ~ 1e4, so two exact FP64
    eliminations of it (the oracle's and the GPU's, each with its own rounded
    factors) agree only to about that times the unit roundoff per solve, and the
    40 solves of a slice accumulate it: the bound is 40 * (1 + 4 tau / h^2) * eps.
    variable: a variable coefficient without source, s = 20 (tau / h^2 = 125), at
    1e-12."""
    if case == "variable":
        w = W.small_dim2(999, 999, n_slices=20, fine_steps=20, seed=20)
        base = w.u0
    else:
        w = W.manufactured2d(999, 20, 1, T=0.05) if case == "paper_step" else W.manufactured2d(999, 20, 20)
        base = w.extra["exact_space"]
    tol = TOL
    if case == "paper_run":
        k = (w.T / w.n_slices / w.fine_steps) * (w.nx + 1) ** 2
        tol = 2 * w.fine_steps * (1 + 4 * k) * np.finfo(np.float64).eps
    P, O = gpu_problem(w), oracle_problem(w)
    assert P.get_option("partitioned_used") == 1
    rng = np.random.default_rng(1)
    Uin = np.stack([base * (0.5 + 0.05 * k) for k in range(w.n_slices)])
    Uin[9] += 0.01 * rng.standard_normal(base.shape)
    F = P.new_slices()
    P.fine_propagate(dev(Uin), F)
    torch.cuda.synchronize()
    got = F.cpu().numpy().reshape(Uin.shape)
    for n in (0, 9, 19):
        ref = O.fine(Uin[n], n)
        assert relerr(got[n], ref) <= tol, n
