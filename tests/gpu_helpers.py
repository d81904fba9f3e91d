"""Shared helpers for the GPU parity tests: build the HIP-path problem and the
oracle problem from the same seeded workload."""
import numpy as np

import oracle
import workloads as W

TOL = 1e-12  # relative infinity-norm parity bound


def relerr(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    den = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (den if den > 0 else 1.0))


def oracle_problem(w):
    if w.theta is not None:
        ax, ay = oracle.faces_from_theta(w.nx, w.ny, w.theta, dim=w.dim)
    else:
        ax, ay = w.ax, w.ay
    return oracle.Problem(dim=w.dim, nx=w.nx, ny=w.ny, T=w.T, n_slices=w.n_slices,
                          fine_steps=w.fine_steps, coarse_steps=w.coarse_steps, split=w.split,
                          fine=w.fine, c=w.c, ax=ax, ay=ay, rho=w.rho, forcing=w.forcing)


def instance_dict(w):
    d = dict(dim=w.dim, nx=w.nx, ny=w.ny, T=w.T, n_slices=w.n_slices, fine_steps=w.fine_steps,
             coarse_steps=w.coarse_steps, split=w.split, fine=w.fine, c=w.c)
    if w.theta is not None:
        d["theta"] = w.theta
    else:
        d["ax"], d["ay"] = w.ax, w.ay
    if w.rho is not None:
        d["rho"] = w.rho
    if w.forcing is not None:
        d["forcing"] = w.forcing
    return d


def gpu_problem(ws):
    import paper_2502_08370_amd as pr
    if not isinstance(ws, (list, tuple)):
        ws = [ws]
    return pr.Problem([instance_dict(w) for w in ws])


def slice_inputs(w, seed=0):
    """N seeded, smooth-plus-noise slice states (as parareal would feed F)."""
    rng = np.random.default_rng(seed)
    base = w.u0
    return np.stack([base * (0.5 + 0.5 * rng.random()) + 0.05 * rng.standard_normal(base.shape)
                     for _ in range(w.n_slices)])


def parareal_threaded(O, u0, k_max, workers=16):
    """The oracle's parareal iteration (or_parareal) composed from its own steps,
    with the fine propagations of the N slices run on a thread pool (each a call
    into the serial C oracle, which keeps no shared state): the initial coarse
    sweep, then per correction F_n = fine(U_n, n) for every n and the coarse
    sweep with the correction. Same operations in the same order per slice as
    or_parareal, so the results agree bitwise (checked on the CPU). Returns
    (U, increments)."""
    from concurrent.futures import ThreadPoolExecutor
    N = O.n_slices
    U = np.empty((N + 1,) + O.shape)
    U[0] = np.asarray(u0, dtype=np.float64).reshape(O.shape)
    G = np.empty((N,) + O.shape)
    O.coarse_sweep(None, G, U)
    hist = []
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for _ in range(k_max):
            F = np.stack(list(ex.map(lambda n: O.fine(U[n], n), range(N))))
            hist.append(O.coarse_sweep(F, G, U))
    return U, hist
