"""MI355X-native parareal with splitting (arXiv 2502.08370): Python front end.

The numerical work runs in libpr.so (hand-written HIP for gfx950) behind the C
ABI of include/pr.h. This module marshals torch CUDA (HIP) tensors and the
current stream into those calls; torch provides device memory and streams
only.

    import paper_2502_08370_amd as pr
    prob = pr.Problem([dict(dim=2, nx=1023, ny=1023, T=0.05, n_slices=64, fine_steps=64,
                            ax=ax, ay=ay)])
    U = prob.new_states()
    k, inc = prob.parareal_iterate(u0, U, k_max=64, tol=1e-8)
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B
from ._binding import PrError

__all__ = ["Problem", "PrError", "lib"]

lib = B.lib


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(a, device):
    torch = _torch()
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.detach().to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


def _check_coef(dim, nx, ny, mode, cx, cy, device):
    """Coefficient arrays the library reads: nodal theta on the grid with its boundary
    nodes, or the x-faces and (2D) the y-faces."""
    if mode == B.PR_COEF_NODAL_LOG:
        _check(cx, device, (nx + 2) * (ny + 2) if dim == 2 else nx + 2, "theta")
    else:
        _check(cx, device, ny * (nx + 1), "ax")
        if dim == 2:
            _check(cy, device, (ny + 1) * nx, "ay")


_OPTS = {"graph": B.PR_OPT_GRAPH, "fine_chunk": B.PR_OPT_FINE_CHUNK, "lanes": B.PR_OPT_LANES,
         "blocks_per_pass": B.PR_OPT_BLOCKS_PER_PASS, "twisted": B.PR_OPT_TWISTED,
         "grouped": B.PR_OPT_GROUPED, "partitioned": B.PR_OPT_PARTITIONED,
         "partitioned_used": B.PR_OPT_PARTITIONED_USED}


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(t, device, count, name, optional=False):
    """The library reads and writes raw device pointers: refuse, before any launch,
    a tensor that is not a contiguous float64 tensor of exactly `count` elements
    on the handle's device."""
    torch = _torch()
    if t is None:
        if optional:
            return
        raise PrError(B.PR_EINVAL, f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise PrError(B.PR_EINVAL, f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise PrError(B.PR_EINVAL, f"{name} must be float64, got {t.dtype}")
    if t.device.type != device.type or (device.index is not None and t.device.index != device.index):
        raise PrError(B.PR_EINVAL, f"{name} is on {t.device}, the handle on {device}")
    if not t.is_contiguous():
        raise PrError(B.PR_EINVAL, f"{name} must be contiguous")
    if t.numel() != count:
        raise PrError(B.PR_EINVAL, f"{name} has {t.numel()} elements, expected {count}")


class Problem:
    """A handle over one or more independent problem instances (section 2.1 model,
    section 3 parareal).

    Each instance is a dict with keys: dim, nx, ny, T, n_slices, fine_steps,
    coarse_steps (1), split ('dim' | 'dd'), fine ('fie' | 'dr'), c (0.0), and
    either ax / ay (face coefficients) or theta (nodal log coefficient), plus rho
    (partition of unity, host array) for 'dd': (M, nx+1) face weights in 1D,
    (M, 2*nx+1) samples on the half grid of x in 2D (vertical strips), and optionally
    forcing = (S, g_fine, g_coarse): the source F(t) = sum_m g_m(t) S_m with S
    of shape (m, ny, nx), g_fine (m, n_slices*fine_steps) and g_coarse
    (m, n_slices*coarse_steps) at the step end times (m <= 2).
    """

    def __init__(self, instances, device="cuda", stream=None):
        torch = _torch()
        if isinstance(instances, dict):
            instances = [instances]
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        n = len(instances)
        descs = (B.PrProblemDesc * n)()
        keep = []
        self.instances = []
        for i, ins in enumerate(instances):
            d = descs[i]
            d.dim, d.nx = int(ins["dim"]), int(ins["nx"])
            d.ny = 1 if d.dim == 1 else int(ins["ny"])
            d.T = float(ins["T"])
            d.n_slices, d.fine_steps = int(ins["n_slices"]), int(ins["fine_steps"])
            d.coarse_steps = int(ins.get("coarse_steps", 1))
            d.fine = B.PR_DR if ins.get("fine", "fie") == "dr" else B.PR_FIE
            d.split = B.PR_SPLIT_DD if ins.get("split", "dim") == "dd" else B.PR_SPLIT_DIM
            d.c = float(ins.get("c", 0.0))
            if ins.get("theta") is not None:
                d.coef_mode = B.PR_COEF_NODAL_LOG
                cx, cy = _dev_f64(ins["theta"], self.device), None
            else:
                d.coef_mode = B.PR_COEF_FACES
                cx = _dev_f64(ins["ax"], self.device)
                cy = _dev_f64(ins.get("ay"), self.device)
            _check_coef(d.dim, d.nx, d.ny, d.coef_mode, cx, cy, self.device)
            keep += [cx, cy]
            d.coef_x, d.coef_y = _ptr(cx), _ptr(cy)
            rho = ins.get("rho")
            if rho is not None:
                rho = np.ascontiguousarray(rho, dtype=np.float64)
                keep.append(rho)
                d.n_colors = rho.shape[0]
                d.rho = C.c_void_p(rho.ctypes.data)
            forcing = ins.get("forcing")
            if forcing is not None:
                S, gf, gc = forcing
                m = int(np.asarray(S).shape[0])
                Sd = _dev_f64(np.asarray(S).reshape(m, -1), self.device)
                gf = np.ascontiguousarray(np.asarray(gf, dtype=np.float64).reshape(m, -1))
                gc = np.ascontiguousarray(np.asarray(gc, dtype=np.float64).reshape(m, -1))
                keep += [Sd, gf, gc]
                d.n_forcing = m
                d.forcing_space = _ptr(Sd)
                d.forcing_time_fine = C.c_void_p(gf.ctypes.data)
                d.forcing_time_coarse = C.c_void_p(gc.ctypes.data)
            self.instances.append(dict(dim=d.dim, nx=d.nx, ny=d.ny, n_slices=d.n_slices,
                                       fine_steps=d.fine_steps, coarse_steps=d.coarse_steps,
                                       fine=d.fine, split=d.split, n_forcing=d.n_forcing,
                                       n_colors=d.n_colors, coef_mode=d.coef_mode))
        h = C.c_void_p()
        B.check(B.lib().pr_create_problem(descs, n, _stream(stream), C.byref(h)))
        self._h = h
        lay = (B.PrInstanceLayout * n)()
        tot = (C.c_size_t * 3)()
        B.check(B.lib().pr_query_layout(h, lay, tot))
        self.layout = [dict(u0=l.u0_offset, slices=l.slices_offset, states=l.states_offset,
                            npts=l.npts, n_slices=l.n_slices) for l in lay]
        self.totals = dict(u0=tot[0], slices=tot[1], states=tot[2])
        del keep

    # ---------------------------------------------------------------- buffers
    def _new(self, kind):
        torch = _torch()
        return torch.zeros(self.totals[kind], dtype=torch.float64, device=self.device)

    def new_u0(self):
        return self._new("u0")

    def new_slices(self):
        return self._new("slices")

    def new_states(self):
        return self._new("states")

    def view(self, buf, i, kind):
        """Instance i's part of a packed buffer, shaped (count, ny, nx) or (ny, nx)."""
        l, ins = self.layout[i], self.instances[i]
        shape = (ins["ny"], ins["nx"]) if ins["dim"] == 2 else (ins["nx"],)
        off = l[kind]
        if kind == "u0":
            return buf[off:off + l["npts"]].view(shape)
        cnt = l["n_slices"] + (1 if kind == "states" else 0)
        return buf[off:off + cnt * l["npts"]].view((cnt,) + shape)

    def pack_u0(self, u0s):
        """Pack a list of per-instance initial states into one device buffer."""
        buf = self.new_u0()
        for i, u in enumerate(u0s):
            self.view(buf, i, "u0").copy_(_dev_f64(u, self.device).view(self.view(buf, i, "u0").shape))
        return buf

    # ------------------------------------------------------------ entry points
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            B.lib().pr_destroy_problem(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_coefficients(self, i, coef_x, coef_y=None, stream=None):
        cx, cy = _dev_f64(coef_x, self.device), _dev_f64(coef_y, self.device)
        ins = self.instances[i]
        _check_coef(ins["dim"], ins["nx"], ins["ny"], ins["coef_mode"], cx, cy, self.device)
        B.check(B.lib().pr_set_coefficients(self._h, int(i), _ptr(cx), _ptr(cy), _stream(stream)))
        _torch().cuda.current_stream().synchronize()

    def fine_propagate(self, U_in, F_out, stream=None):
        n = self.totals["slices"]
        _check(U_in, self.device, n, "U_in")
        _check(F_out, self.device, n, "F_out")
        B.check(B.lib().pr_fine_propagate(self._h, _ptr(U_in), _ptr(F_out), _stream(stream)))

    def coarse_sweep(self, F, G_old, U, inc=None, stream=None):
        _check(F, self.device, self.totals["slices"], "F", optional=True)
        _check(G_old, self.device, self.totals["slices"], "G_old")
        _check(U, self.device, self.totals["states"], "U")
        _check(inc, self.device, len(self.layout), "inc", optional=True)
        B.check(B.lib().pr_coarse_sweep(self._h, _ptr(F), _ptr(G_old), _ptr(U), _ptr(inc),
                                        _stream(stream)))

    def parareal_iterate(self, u0, U, k_max, tol=0.0, stream=None):
        _check(u0, self.device, self.totals["u0"], "u0")
        _check(U, self.device, self.totals["states"], "U")
        n = len(self.layout)
        k = (C.c_int * n)()
        inc = (C.c_double * n)()
        B.check(B.lib().pr_parareal_iterate(self._h, _ptr(u0), _ptr(U), int(k_max), float(tol), k,
                                            inc, _stream(stream)))
        return list(k), list(inc)

    def sequential_fine(self, u0, U, stream=None):
        _check(u0, self.device, self.totals["u0"], "u0")
        _check(U, self.device, self.totals["states"], "U")
        B.check(B.lib().pr_sequential_fine(self._h, _ptr(u0), _ptr(U), _stream(stream)))

    def set_option(self, name, value):
        """name: 'graph' (0/1), 'fine_chunk' (16/24/32), 'lanes' (0/8/16/32/64),
        'blocks_per_pass' (0 = all slice blocks per launch, k > 0 = k at a time),
        'twisted' (1: two waves per fine line, one from each end; 0: one wave),
        'grouped' (1: four lines per workgroup share their carry loads; 0: one line)."""
        B.check(B.lib().pr_set_option(self._h, _OPTS[name], int(value)))

    def get_option(self, name):
        v = C.c_int()
        B.check(B.lib().pr_get_option(self._h, _OPTS[name], C.byref(v)))
        return v.value

    def autotune(self, cache=None, stream=None):
        """Pick the fastest (lanes, fine_chunk) for this handle's shapes. With a cache
        path (JSON), reuse a previous choice for the same shapes."""
        import json
        import os
        # everything that selects the kernels and their work: shapes, steps, integrator,
        # split, colours and source terms
        key = json.dumps(sorted(tuple(ins[k] for k in ("dim", "nx", "ny", "n_slices", "fine_steps",
                                                         "coarse_steps", "fine", "split",
                                                         "n_colors", "n_forcing"))
                                for ins in self.instances))
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_option("lanes", table[key]["lanes"])
                self.set_option("fine_chunk", table[key]["fine_chunk"])
                self.set_option("twisted", table[key].get("twisted", 1))
                return dict(table[key], cached=True)
        lanes, chunk, ms = C.c_int(), C.c_int(), C.c_float()
        B.check(B.lib().pr_autotune(self._h, _stream(stream), C.byref(lanes), C.byref(chunk),
                                    C.byref(ms)))
        res = dict(lanes=lanes.value, fine_chunk=chunk.value, twisted=self.get_option("twisted"),
                   fine_ms=ms.value)
        if cache:
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            table[key] = res
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return dict(res, cached=False)

    def profile(self, mode):
        """1: start recording phase timers (one event pair per launch), 3: start them in
        span mode (one pair per loop of fine sweeps and per coarse sweep), 0: stop,
        2: clear."""
        B.check(B.lib().pr_profile_control(self._h, int(mode)))

    def profile_read(self):
        """{phase: (total ms, launches)} of the recorded phase timers."""
        out = B.PrProfile()
        B.check(B.lib().pr_profile_read(self._h, C.byref(out)))
        return {B.PHASE_NAMES[i]: (out.ms[i], out.count[i]) for i in range(B.PROFILE_PHASES)
                if out.count[i]}

    def _check_adjoint(self, u0, lambda_T, grad_u0, grad_coef, U_ckpt):
        n = self.totals["u0"]
        for t, name in ((u0, "u0"), (lambda_T, "lambda_T"), (grad_u0, "grad_u0")):
            _check(t, self.device, n, name)
        _check(grad_coef, self.device, self.coef_count(0), "grad_coef")
        _check(U_ckpt, self.device, self.totals["states"], "U_ckpt", optional=True)

    def coef_count(self, i):
        """Entries of instance i's coefficient (and coefficient gradient): nodal theta
        (nx+2)(ny+2) (nx+2 in 1D), or the x-faces followed by the y-faces."""
        ins = self.instances[i]
        nx, ny = ins["nx"], ins["ny"]
        if ins["coef_mode"] == B.PR_COEF_NODAL_LOG:
            return (nx + 2) * (ny + 2) if ins["dim"] == 2 else nx + 2
        return ny * (nx + 1) + ((ny + 1) * nx if ins["dim"] == 2 else 0)

    def adjoint(self, u0, lambda_T, grad_u0, grad_coef, U_ckpt=None, stream=None):
        self._check_adjoint(u0, lambda_T, grad_u0, grad_coef, U_ckpt)
        B.check(B.lib().pr_adjoint(self._h, _ptr(u0), _ptr(lambda_T), _ptr(grad_u0),
                                   _ptr(grad_coef), _ptr(U_ckpt), _stream(stream)))

    def adjoint_noalloc(self, u0, lambda_T, grad_u0, grad_coef, U_ckpt=None, stream=None):
        """pr_adjoint with its workspace in the library's fixed per-GPU scratch array
        (no device allocation; raises PrError when the problem does not fit it)."""
        self._check_adjoint(u0, lambda_T, grad_u0, grad_coef, U_ckpt)
        B.check(B.lib().pr_adjoint_noalloc(self._h, _ptr(u0), _ptr(lambda_T), _ptr(grad_u0),
                                           _ptr(grad_coef), _ptr(U_ckpt), _stream(stream)))

    def adjoint_parallel(self, u0, lambda_T, grad_u0, grad_coef, U_ckpt=None, k_max=0, tol=0.0,
                         stream=None):
        """Parallel-in-time adjoint (pr_adjoint_parallel): k_max = 0 computes the
        boundary adjoints exactly, k_max > 0 by parareal on the backward problem.
        Returns the number of backward parareal corrections done."""
        self._check_adjoint(u0, lambda_T, grad_u0, grad_coef, U_ckpt)
        k = C.c_int(0)
        B.check(B.lib().pr_adjoint_parallel(self._h, _ptr(u0), _ptr(lambda_T), _ptr(grad_u0),
                                            _ptr(grad_coef), _ptr(U_ckpt), int(k_max), float(tol),
                                            C.byref(k), _stream(stream)))
        return k.value
