"""Batched instances (uneven grid sizes and slice counts in one handle): the
graph-captured parareal iteration against direct launches (bitwise, replay by
replay), per-instance convergence masking against the oracle run instance by
instance, and every tuning option / the autotuner against the oracle."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import TOL, gpu_problem, oracle_problem, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)


def small_batch(seed=0, count=10):
    rng = np.random.default_rng(seed)
    ws = []
    for i in range(count):
        n = int(rng.choice([15, 31, 63, 70]))
        N = int(rng.choice([4, 8, 16, 13]))
        ws.append(W.small_dim2(n, n + int(rng.integers(0, 9)), n_slices=N, fine_steps=3,
                               seed=100 + i, T=0.05))
    return ws


def test_graph_replays_match_direct_launches():
    ws = small_batch(1)
    Pg, Pe = gpu_problem(ws), gpu_problem(ws)
    Pe.set_option("graph", 0)
    assert Pg.get_option("graph") == 1 and Pe.get_option("graph") == 0
    u0 = Pg.pack_u0([w.u0 for w in ws])
    for K in (1, 2, 3, 5):
        Ug, Ue = Pg.new_states(), Pe.new_states()
        kg, ig = Pg.parareal_iterate(u0, Ug, k_max=K, tol=0.0)
        # eager work and a synchronisation between replays
        scratch = torch.randn(1 << 16, device="cuda", dtype=torch.float64).sum().item()
        ke, ie = Pe.parareal_iterate(u0, Ue, k_max=K, tol=0.0)
        torch.cuda.synchronize()
        assert kg == ke and ig == ie
        assert torch.equal(Ug, Ue), K
        assert np.isfinite(scratch)


def test_batch_tolerance_masking_matches_oracle():
    ws = small_batch(2)
    P = gpu_problem(ws)
    u0 = P.pack_u0([w.u0 for w in ws])
    # a tolerance that different instances reach after different iteration counts
    tol = 3e-7
    U = P.new_states()
    k, inc = P.parareal_iterate(u0, U, k_max=16, tol=tol)
    torch.cuda.synchronize()
    ks = set()
    for i, w in enumerate(ws):
        Uo, ko, hist = oracle_problem(w).parareal(w.u0, 16, tol)
        assert k[i] == ko, (i, k[i], ko)
        ks.add(ko)
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL
        assert abs(inc[i] - hist[-1]) <= TOL * np.abs(Uo).max()
    assert len(ks) > 1  # the masking was exercised


@pytest.mark.parametrize("part", [2, 0])
@pytest.mark.parametrize("lanes,chunk", [(8, 16), (16, 32), (32, 16), (0, 32)])
def test_layout_options(lanes, chunk, part):
    ws = [W.small_dim2(70, 45, 64, 3, seed=5), W.small_dim2(33, 50, 16, 3, seed=6)]
    P = gpu_problem(ws)
    P.set_option("partitioned", part)
    P.set_option("lanes", lanes)
    P.set_option("fine_chunk", chunk)
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, _, _ = oracle_problem(w).parareal(w.u0, 2)
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL


def test_autotune_keeps_results(tmp_path):
    ws = small_batch(3, count=4)
    P = gpu_problem(ws)
    res = P.autotune(cache=str(tmp_path / "tune.json"))
    assert res["lanes"] in (0, 8, 16, 32, 64) and res["fine_chunk"] in (16, 20, 24, 32)
    P2 = gpu_problem(ws)
    res2 = P2.autotune(cache=str(tmp_path / "tune.json"))
    assert res2["cached"] and res2["lanes"] == res["lanes"]
    u0 = P.pack_u0([w.u0 for w in ws])
    U = P.new_states()
    P.parareal_iterate(u0, U, k_max=2, tol=0.0)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        Uo, _, _ = oracle_problem(w).parareal(w.u0, 2)
        assert relerr(P.view(U, i, "states").cpu().numpy(), Uo) <= TOL


def test_graph_with_domain_decomposition_instances():
    """Handles holding 1D and 2D domain-decomposition instances beside a dimensional one
    are captured too: the graph bakes in which of them are still active and is captured
    again when one converges. Replays match direct launches bit for bit, and the run to
    a tolerance matches the oracle instance by instance."""
    ws = [W.small_dim2(37, 29, 6, 3, seed=1),
          W.small_dd1(300, 4, 2, 8, 6, 2, seed=2),
          W.small_dd2(40, 33, 2, 0.1, 6, 2, seed=3)]
    Pg, Pe = gpu_problem(ws), gpu_problem(ws)
    Pe.set_option("graph", 0)
    u0 = Pg.pack_u0([w.u0 for w in ws])
    hists = [oracle_problem(w).parareal(w.u0, 6)[2] for w in ws]
    # a tolerance between the third increments of the 1D DD and the dimensional
    # instance: the domain-decomposition instances stop first
    tol = float(np.sqrt(hists[1][2] * hists[0][2]))
    for K, t in ((1, 0.0), (4, 0.0), (6, tol)):
        Ug, Ue = Pg.new_states(), Pe.new_states()
        kg, ig = Pg.parareal_iterate(u0, Ug, k_max=K, tol=t)
        scratch = torch.randn(1 << 16, device="cuda", dtype=torch.float64).sum().item()
        ke, ie = Pe.parareal_iterate(u0, Ue, k_max=K, tol=t)
        torch.cuda.synchronize()
        assert kg == ke and ig == ie, (K, kg, ke)
        assert torch.equal(Ug, Ue), K
        assert np.isfinite(scratch)
        for i, w in enumerate(ws):
            Uo, ko, _ = oracle_problem(w).parareal(w.u0, K, t)
            assert kg[i] == ko, (K, i, kg[i], ko)
            assert relerr(Pg.view(Ug, i, "states").cpu().numpy(), Uo) <= TOL
    assert kg[1] < kg[0]  # a domain-decomposition instance converged first
