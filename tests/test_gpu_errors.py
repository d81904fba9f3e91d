"""Error contract of the boundary on the GPU: a NaN in u0 makes the parareal
iteration stop with PR_ENUMERIC after its first correction (section 3: the
iteration stops on its increment, and a non-finite increment is an error);
the Python front end refuses tensors of the wrong dtype, device, layout or
size before anything is queued."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_helpers import gpu_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)


def test_nan_in_u0_stops_with_enumeric_after_one_correction():
    from paper_2502_08370_amd import _binding as B
    w = W.small_dim2(37, 29, n_slices=6, fine_steps=5, seed=1)
    P = gpu_problem(w)
    u0 = torch.as_tensor(w.u0, device="cuda").reshape(-1).contiguous()
    u0[100] = float("nan")
    U = P.new_states()
    k = (C.c_int * 1)()
    inc = (C.c_double * 1)()
    st = B.lib().pr_parareal_iterate(P._h, C.c_void_p(u0.data_ptr()), C.c_void_p(U.data_ptr()),
                                     5, 1e-8, k, inc, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == B.PR_ENUMERIC
    assert k[0] == 1
    assert not np.isfinite(inc[0])
    assert b"non-finite" in B.lib().pr_last_error()
    # the handle stays usable: a finite u0 converges as usual
    u0[100] = float(w.u0.reshape(-1)[100])
    kk, ii = P.parareal_iterate(u0, U, k_max=6, tol=0.0)
    assert kk == [6] and np.isfinite(ii[0])
    P.close()


def test_front_end_rejects_bad_tensors_before_any_launch():
    import paper_2502_08370_amd as pr
    w = W.small_dim2(20, 17, n_slices=3, fine_steps=2, seed=2)
    P = gpu_problem(w)
    n = P.totals["slices"]
    good_in = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    bad = {
        "float32": good_in.float(),
        "cpu": good_in.cpu(),
        "short": good_in[:-1],
        "strided": torch.ones(2 * n, dtype=torch.float64, device="cuda")[::2],
    }
    for name, t in bad.items():
        with pytest.raises(pr.PrError):
            P.fine_propagate(t, out)
    with pytest.raises(pr.PrError):
        P.coarse_sweep(None, out[:-1], P.new_states())
    with pytest.raises(pr.PrError):
        P.parareal_iterate(torch.zeros(w.nx * w.ny + 1, dtype=torch.float64, device="cuda"),
                           P.new_states(), k_max=1)
    with pytest.raises(pr.PrError):
        P.set_coefficients(0, np.zeros(5))
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0  # nothing ran
    P.close()
