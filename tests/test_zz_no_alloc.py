"""pr_adjoint_noalloc (the adjoint with its workspace in the library's fixed
per-GPU scratch array) against pr_adjoint on the same handles, through the C
ABI: two calls in a row, the second on a smaller problem (the scratch keeps the
first call's contents), with and without caller checkpoints, both coefficient
modes; a problem larger than the scratch is refused before any launch."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import TOL, gpu_problem, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda").reshape(-1)


def _case(nx, ny, N, s, mode, seed):
    w = W.small_dim2(nx, ny, n_slices=N, fine_steps=s, seed=seed)
    if mode == "faces":
        w.ax, w.ay = oracle.faces_from_theta(nx, ny, w.theta)
        w.theta = None
    ncoef = (nx + 2) * (ny + 2) if mode == "theta" else ny * (nx + 1) + (ny + 1) * nx
    lam = np.random.default_rng(seed + 1).standard_normal((ny, nx))
    return w, ncoef, lam


def _run(P, w, ncoef, lam, noalloc, with_ckpt):
    g0 = torch.full((w.nx * w.ny,), np.nan, dtype=torch.float64, device="cuda")
    gc = torch.full((ncoef,), np.nan, dtype=torch.float64, device="cuda")
    ck = P.new_states() if with_ckpt else None
    fn = P.adjoint_noalloc if noalloc else P.adjoint
    fn(dev(w.u0), dev(lam), g0, gc, ck)
    torch.cuda.synchronize()
    return g0.cpu().numpy(), gc.cpu().numpy(), None if ck is None else ck.cpu().numpy()


@pytest.mark.parametrize("with_ckpt", [False, True])
def test_noalloc_adjoint_matches_pr_adjoint(with_ckpt):
    cases = [(96, 80, 4, 8, "theta", 3), (48, 37, 3, 5, "faces", 4)]  # second call smaller
    for nx, ny, N, s, mode, seed in cases:
        print(f"noalloc adjoint {nx}x{ny} N={N} s={s} {mode} ckpt={with_ckpt}", flush=True)
        w, ncoef, lam = _case(nx, ny, N, s, mode, seed)
        P = gpu_problem(w)
        ref = _run(P, w, ncoef, lam, noalloc=False, with_ckpt=with_ckpt)
        got = _run(P, w, ncoef, lam, noalloc=True, with_ckpt=with_ckpt)
        for a, b in zip(got, ref):
            if b is None:
                continue
            assert np.isfinite(a).all()
            assert relerr(a, b) <= TOL
            assert np.array_equal(a, b)  # same kernels in the same order: identical bits
        P.close()


def test_noalloc_adjoint_refuses_a_problem_above_the_scratch():
    import paper_2502_08370_amd as pr
    # (2 s + 2) states of 255^2 at s = 64 alone need 8.5e6 doubles > 8 Mi
    w, ncoef, lam = _case(255, 255, 2, 64, "theta", 5)
    P = gpu_problem(w)
    g0 = torch.zeros(w.nx * w.ny, dtype=torch.float64, device="cuda")
    gc = torch.zeros(ncoef, dtype=torch.float64, device="cuda")
    with pytest.raises(pr.PrError) as e:
        P.adjoint_noalloc(dev(w.u0), dev(lam), g0, gc)
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(g0.abs().max()) == 0.0 and float(gc.abs().max()) == 0.0
    P.close()
