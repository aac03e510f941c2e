"""Build matching GPU lattices and oracle runs from one workload description.

Shared by the GPU tests, the smoke check and the benchmark's sampled checks;
it only forwards the same inputs to both sides.
"""
from __future__ import annotations

import numpy as np

from oracle import lbm_oracle as O

BCS = ("periodic", "fullway", "halfway")


def oracle_field(spec: dict, d: int):
    if spec is None:
        return None
    kind = spec["kind"]
    if kind == "tanh_bubble":
        return O.ExactField(kind, u=spec["u"], R=spec.get("R", 0.0), Rr=spec["Rr"],
                            W=spec["W"], center=spec.get("center"))
    return O.ExactField(kind, u=spec["u"], R=spec.get("R", 0.0), amps=spec["amps"],
                        kvecs=np.asarray(spec["kvecs"], float).reshape(len(spec["amps"]), d),
                        phases=spec.get("phases"))


def oracle_problem(d, dims, dx, spec=None, u=None, R=None, tau=0.5, bc=None, P=4, K=3,
                   origin=None, faces=None, shift=None, wall_data="jets"):
    u = spec["u"] if u is None else u
    R = spec.get("R", 0.0) if (R is None and spec is not None) else (R or 0.0)
    if faces is None:
        faces = [(b, b) if isinstance(b, str) else tuple(b) for b in (bc or ["periodic"] * d)]
    return O.Problem(d, dims, dx, u, R=R, tau=tau, origin=origin, bc=faces, P=P, K=K,
                     field=oracle_field(spec, d), shift=shift, wall_data=wall_data)


def gpu_lattice(d, dims, dx, spec=None, u=None, R=None, tau=0.5, bc=None, P=4, K=3,
                origin=None, precision="fp64", wall_data="jets"):
    from paper_2410_13165_amd import Lattice
    u = spec["u"] if u is None else u
    R = spec.get("R", 0.0) if (R is None and spec is not None) else (R or 0.0)
    return Lattice(d, dims, tau, dx=dx, u=u, R=R, origin=origin, bc=bc, P=P, K=K,
                   precision=precision, field=spec, wall_data=wall_data)


def to_oracle_order(arr: np.ndarray) -> np.ndarray:
    """(N_d, ..., N_1) C-order GPU layout -> oracle indexing (N_1, ..., N_d)."""
    return np.ascontiguousarray(arr.T)


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    den = float(np.linalg.norm(b.ravel()))
    return float(np.linalg.norm((a - b).ravel())) / (den if den > 0 else 1.0)


def gpu_populations(lat, info=None) -> np.ndarray:
    """Stored state of a GPU lattice as absolute populations in oracle order.

    fp64 / fp32: post-collision f*(t_n); fp32_split, fp32_hilo: pre-collision f(t_n).
    Returns shape (q, N_1, ..., N_d)."""
    import torch
    info = info or lat.info()
    q, nodes = info["q"], info["nodes"]
    blob = lat.get_state()
    torch.cuda.synchronize()
    pstride = info["pstride"]
    dims_rev = tuple(reversed(lat.dims))
    omega = info["omega"]
    if lat.precision == "fp64":
        f = blob[: q * pstride * 8].view(torch.float64).cpu().numpy().reshape(q, pstride)[:, :nodes]
    else:
        f = blob[: q * pstride * 4].view(torch.float32).cpu().numpy().reshape(q, pstride)[:, :nodes]
        f = f.astype(np.float64)
    if lat.precision == "fp32":
        t_next = (info["step"] + 1) * info["dt"]
        ref = info["phi_ref"] + lat_R(lat) * t_next
        f = f + omega[:, None] * ref
    if lat.precision == "fp32_split":
        phi = blob[q * pstride * 4:].view(torch.float64).cpu().numpy()[:nodes]
        f = f + omega[:, None] * phi[None, :]
    if lat.precision == "fp32_hilo":
        hl = blob[q * pstride * 4:].view(torch.float32).cpu().numpy()[:2 * nodes]
        phi = hl[0::2].astype(np.float64) + hl[1::2].astype(np.float64)
        f = f + omega[:, None] * phi[None, :]
    out = np.empty((q,) + tuple(lat.dims))
    for k in range(q):
        out[k] = to_oracle_order(f[k].reshape(dims_rev))
    return out


def lat_R(lat) -> float:
    return float(lat._params.R)


def local_oracle_phi(d, dims, dx, spec, bc, idx, r, P=4, K=3, tau=0.5, origin=None):
    """phi at global node `idx` after r steps, from an oracle run on the sub-box of
    radius r around it.  Sides that reach a Dirichlet wall keep it; the other
    sides are 'open' (wrapped), whose wrong values travel one node per step and
    reach the centre only after r + 1 steps."""
    origin = np.zeros(d) if origin is None else np.asarray(origin, float)
    for a in range(d):
        if bc[a] == "periodic":
            assert r <= idx[a] <= dims[a] - 1 - r, "sample too close to a periodic seam"
    lo = [max(0, idx[a] - r) for a in range(d)]
    hi = [min(dims[a] - 1, idx[a] + r) for a in range(d)]
    faces, sub_dims, shift, sub_origin = [], [], [], []
    for a in range(d):
        lf = bc[a] if (bc[a] != "periodic" and lo[a] == 0) else "open"
        hf = bc[a] if (bc[a] != "periodic" and hi[a] == dims[a] - 1) else "open"
        faces.append((lf, hf))
        sub_dims.append(hi[a] - lo[a] + 1)
        shift.append(0.5 if bc[a] == "halfway" else 0.0)
        sub_origin.append(origin[a] + lo[a] * dx)
    prob = oracle_problem(d, sub_dims, dx, spec, tau=tau, P=P, K=K, origin=sub_origin,
                          faces=faces, shift=shift)
    run = O.Run(prob).step(r)
    local = tuple(idx[a] - lo[a] for a in range(d))
    return float(run.phi()[local])
