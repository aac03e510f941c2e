"""Parameters of the long parity runs: the configurations at their own step
counts (D1Q3 plane wave, D3Q19 Dirichlet cubes, the D3Q19 Gaussian-field
gradient workload at a small grid, a stratified subset of the D2Q9 stability
sweep), and the node samples their results are compared on.

Shared by tests/golden/make_long_runs.py, which runs the FP64 oracle on them
and stores the sampled results in tests/golden/long_runs.npz, and by
tests/test_gpu_long_runs.py, which runs the HIP path on the same inputs.
Only parameters and index draws live here, nothing of the method.
"""
from __future__ import annotations

import numpy as np

from paper_2410_13165_amd import inputs

GOLDEN = "long_runs.npz"

# D3Q19 on [0,1]^3 with Dirichlet walls on all six faces and the benchmark's
# field (four random cosines, seed 3), at the configuration's 2000 steps on a
# 64^3 grid and at 200 steps on 128^3; the half-way variant at u = 1e-3 (1,1,1),
# where that scheme is stable.
CUBES = {
    "d3q19_fullway_64": {"n": 64, "bc": "fullway", "u": [0.05, 0.1, 0.08], "steps": 2000},
    "d3q19_fullway_128": {"n": 128, "bc": "fullway", "u": [0.05, 0.1, 0.08], "steps": 200},
    "d3q19_halfway_64": {"n": 64, "bc": "halfway", "u": [1e-3, 1e-3, 1e-3], "steps": 2000},
}

# The gradient workload's forward run (D3Q19 periodic, Gaussian random field of
# correlation length 0.1, seed 5, u = (0.05, 0.1, 0.08), tau = 1/2, K = 3 with
# fourth-order finite-difference gradients) at its 1000 steps on a 32^3 grid.
GRF = {"d3q19_grf_32": {"n": 32, "steps": 1000}}

# D2Q9 stability sweep: the first four instances of each grid size, in the
# order of inputs.sweep_specs(), over the sweep's 4000 steps.
SWEEP_PER_SIZE = 4


def cube_problem(name: str) -> dict:
    c = CUBES[name]
    n = c["n"]
    dx = 1.0 / (n - 1) if c["bc"] == "fullway" else 1.0 / n
    spec = inputs.random_cosines(3, c["u"], inputs.BENCH_D3Q19["R"], inputs.BENCH_D3Q19["seed"])
    return {"d": 3, "dims": (n, n, n), "dx": dx, "spec": spec, "bc": [c["bc"]] * 3,
            "steps": c["steps"]}


def grf_problem(name: str) -> dict:
    g = GRF[name]
    w = inputs.ADJOINT_D3Q19
    n = g["n"]
    phi0 = inputs.gaussian_random_field(n, 3, w["seed_init"], w["corr"])  # isotropic
    return {"d": 3, "dims": (n, n, n), "dx": 1.0 / n, "u": w["u"], "phi0": phi0,
            "steps": g["steps"]}


def sweep_subset():
    """(indices into sweep_specs(), specs, phi0 per instance in GPU node order)."""
    specs = inputs.sweep_specs()
    phi = inputs.sweep_phi0(specs)
    offs = np.concatenate([[0], np.cumsum([int(np.prod(sp["dims"])) for sp in specs])])
    pick = []
    for n in inputs.SWEEP_D2Q9["sizes"]:
        pick += [i for i, sp in enumerate(specs) if sp["dims"][0] == n][:SWEEP_PER_SIZE]
    return pick, [specs[i] for i in pick], [phi[offs[i]:offs[i + 1]].copy() for i in pick]


def sample_nodes(dims, seed: int, per_face: int = 256, per_edge: int = 8,
                 interior: int = 2048) -> np.ndarray:
    """Node indices (i_1, ..., i_d) to compare on: every corner, points on every
    edge (d >= 2) and face, and interior points, drawn from default_rng(seed).
    Returns an int64 array of shape (count, d), duplicates removed."""
    rng = np.random.default_rng(seed)
    d = len(dims)
    hi = np.array(dims) - 1
    pts = []
    for corner in np.ndindex(*([2] * d)):
        pts.append(np.array(corner) * hi)
    for a in range(d):
        for side in (0, hi[a]):
            q = np.stack([rng.integers(0, dims[b], per_face) for b in range(d)], axis=1)
            q[:, a] = side
            pts += list(q)
    if d >= 2:
        for a in range(d):  # edges along axis a
            others = [b for b in range(d) if b != a]
            for fixed in np.ndindex(*([2] * (d - 1))):
                q = np.stack([rng.integers(0, dims[b], per_edge) for b in range(d)], axis=1)
                for b, f in zip(others, fixed):
                    q[:, b] = f * hi[b]
                pts += list(q)
    q = np.stack([rng.integers(0, dims[b], interior) for b in range(d)], axis=1)
    pts += list(q)
    return np.unique(np.array(pts, dtype=np.int64), axis=0)
