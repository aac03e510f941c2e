"""GPU parity at the configurations' own run lengths.

* D1Q3 plane wave (N = 256, 1000 steps, tau = 1/2 and 0.8): against an oracle
  run in the test, and the RMSE against the exact solution.
* D3Q19 cubes with Dirichlet walls on all faces (full-way 64^3 x 2000 steps and
  128^3 x 200 steps; half-way 64^3 x 2000 steps at u = 1e-3 (1,1,1)), the
  Gaussian-field gradient workload's forward run at 32^3 x 1000 steps, and a
  stratified subset of the D2Q9 stability sweep over its 4000 steps: against
  the oracle's results stored by tests/golden/make_long_runs.py, on the sampled
  nodes (corners, edges, faces, interior) and on whole-lattice sums.
* D4Q33 with N_1 > 256, so the x_1 loop of the row kernels takes two strides.

Tolerances (relative L2 over the samples): float64 1e-12, split and hi/lo 2e-5.  Plain
float32 drifts by about 3.4e-8 relative per step (storage rounding), so past a
few hundred steps it is held to 1e-7 per step and its drift is printed.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import lbm_oracle as O
from paper_2410_13165_amd import inputs
from tests import long_runs as LR
from tests.pairs import gpu_lattice, oracle_problem, rel_l2, to_oracle_order

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", LR.GOLDEN)


def _tol(precision, steps):
    if precision == "fp64":
        return 1e-12
    if precision in ("fp32_split", "fp32_hilo"):
        return 2e-5
    return max(2e-5, 1e-7 * steps)


@pytest.fixture(scope="module")
def golden():
    with np.load(GOLDEN, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _compare(golden, name, phi_or, diag, precision, steps):
    idx = golden[f"{name}__idx"]
    want = golden[f"{name}__phi"]
    scal = golden[f"{name}__scal"]
    assert int(scal[4]) == steps
    got = phi_or[tuple(idx.T)]
    err = rel_l2(got, want)
    tol = _tol(precision, steps)
    print(f"[long] {name} {precision} steps={steps} samples={len(want)} rel L2 {err:.3e} "
          f"(tol {tol:.1e}); sum phi^2 {diag['sum_phi2']:.15g} vs {scal[1]:.15g}", flush=True)
    assert err <= tol, (name, precision, err)
    assert abs(diag["sum_phi2"] - scal[1]) <= 2 * tol * scal[1]
    assert abs(diag["sum_phi"] - scal[0]) <= tol * max(1.0, math.sqrt(scal[1] * len(phi_or.ravel())))
    assert abs(diag["entropy"] - scal[2]) <= 2 * tol * abs(scal[2])
    if np.isfinite(scal[3]):
        assert abs(diag["rmse"] - scal[3]) <= max(1e-3 * scal[3], tol * math.sqrt(scal[1] / phi_or.size))
    assert diag["nonfinite"] == 0


# ------------------------------------ D1Q3 plane wave, 256 nodes, 1000 steps ------

@pytest.mark.parametrize("tau", [0.5, 0.8])
def test_d1q3_plane_wave_1000_steps(tau):
    """D1Q3, periodic [0,1) with 256 nodes, u = 0.3, sin(2 pi x) with the K = 3
    initialisation, 1000 float64 steps (t = 3.90625)."""
    n, steps = 256, 1000
    spec = inputs.plane_sine(1, [0.3])
    run = O.Run(oracle_problem(1, (n,), 1.0 / n, spec, tau=tau)).step(steps)
    lat = gpu_lattice(1, (n,), 1.0 / n, spec, tau=tau)
    try:
        print(f"[long] D1Q3 tau={tau}", flush=True)
        lat.step(steps)
        phi = lat.phi().cpu().numpy()
        dg = lat.diagnostics()
    finally:
        lat.close()
    err = rel_l2(phi, run.phi())
    print(f"[long] D1Q3 tau={tau}: rel L2 vs oracle {err:.3e}, RMSE vs exact {dg['rmse']:.6e} "
          f"(oracle {run.rmse():.6e})", flush=True)
    assert err <= 1e-12
    # |RMSE_gpu - RMSE_oracle| is at most the RMS of the difference of the fields
    assert abs(dg["rmse"] - run.rmse()) <= np.sqrt(np.mean((phi - run.phi()) ** 2)) + 1e-16
    if tau == 0.5:
        assert dg["rmse"] < 1e-8  # fourth order at 256 nodes
    else:
        assert 1e-2 < dg["rmse"] < 1e-1  # tau != 1/2 is first order


# ------------------- D3Q19 Dirichlet cubes, 64^3 x 2000 and 128^3 x 200 steps ------

CUBE_CASES = [("d3q19_fullway_64", "fp64"), ("d3q19_fullway_64", "fp32_split"),
              ("d3q19_fullway_64", "fp32"), ("d3q19_fullway_128", "fp64"),
              ("d3q19_fullway_128", "fp32_split"), ("d3q19_fullway_128", "fp32"),
              ("d3q19_halfway_64", "fp64"), ("d3q19_halfway_64", "fp32_split"),
              ("d3q19_fullway_64", "fp32_hilo"), ("d3q19_halfway_64", "fp32_hilo")]


@pytest.mark.parametrize("name,precision", CUBE_CASES)
def test_dirichlet_cube_full_length(golden, name, precision):
    c = LR.cube_problem(name)
    print(f"[long] {name} {precision}", flush=True)
    lat = gpu_lattice(3, c["dims"], c["dx"], c["spec"], bc=c["bc"], precision=precision)
    try:
        lat.step(c["steps"])
        phi = to_oracle_order(lat.phi().cpu().numpy())
        dg = lat.diagnostics()
    finally:
        lat.close()
    _compare(golden, name, phi, dg, precision, c["steps"])


# ------------------ D3Q19 periodic Gaussian random field, 32^3 x 1000 steps ------

@pytest.mark.parametrize("precision", ["fp64", "fp32_split", "fp32_hilo", "fp32"])
def test_gaussian_field_forward_full_length(golden, precision):
    """The gradient workload's forward run (periodic, Gaussian random field,
    finite-difference initial gradient) at its 1000 steps on 32^3."""
    name = "d3q19_grf_32"
    g = LR.grf_problem(name)
    print(f"[long] {name} {precision}", flush=True)
    lat = gpu_lattice(3, g["dims"], g["dx"], None, u=g["u"], precision=precision)
    try:
        lat.set_initial(torch.from_numpy(np.ascontiguousarray(g["phi0"].T).ravel()))
        lat.step(g["steps"])
        phi = to_oracle_order(lat.phi().cpu().numpy())
        dg = lat.diagnostics()
    finally:
        lat.close()
    _compare(golden, name, phi, dg, precision, g["steps"])


# ------------------ D2Q9 stability-sweep subset, 64^2..512^2 x 4000 steps ------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sweep_subset_4000_steps(golden, precision):
    """Four instances of each grid size of the D2Q9 stability sweep (stable and
    unstable parameters), advanced together as one batch over the sweep's 4000
    steps (two-step passes), each against its own oracle run."""
    from paper_2410_13165_amd import Batch
    pick, specs, phis = LR.sweep_subset()
    print(f"[long] sweep subset {pick} {precision}", flush=True)
    b = Batch(2, specs, precision=precision)
    try:
        b.set_initial(torch.from_numpy(np.concatenate(phis)))
        b.step(4000)
        mom = b.moments()
        fields = [b.instance(i).phi().cpu().numpy() for i in range(len(specs))]
    finally:
        b.close()
    checked = 0
    for j, i in enumerate(pick):
        name = f"sweep_{i}"
        want = golden[f"{name}__phi"]
        if not np.all(np.isfinite(want)):
            print(f"[long] {name}: oracle overflowed, skipped", flush=True)
            continue
        phi = to_oracle_order(fields[j])
        dg = dict(zip(("sum_phi", "sum_phi2", "sum_err2", "entropy", "max_abs_phi", "nonfinite",
                       "rmse", "t"), mom[j]))
        _compare(golden, name, phi, dg, precision, 4000)
        checked += 1
    assert checked >= 12


def test_golden_metadata_matches_parameters(golden):
    meta = json.loads(str(golden["meta"]))
    assert meta["cubes"] == json.loads(json.dumps(LR.CUBES))
    assert meta["sweep"] == LR.sweep_subset()[0]


# ------------------------------------------------------------ D4Q33 ---------

@pytest.mark.parametrize("bc", ["periodic", "fullway", "halfway"])
def test_d4q33_long_first_axis(bc):
    """D4Q33 with 300 nodes along x_1: the row kernels' x_1 loop takes a
    second stride (and the wall rows too)."""
    dims = (300, 5, 4, 3)
    u = [0.05, -0.04, 0.03, 0.02] if bc != "halfway" else [1e-3] * 4
    spec = inputs.random_cosines(4, u, 0.5, seed=91, kmax=1.0)
    dx = 1.0 / (dims[0] - 1)
    prob = oracle_problem(4, dims, dx, spec, bc=[bc] * 4)
    run = O.Run(prob)
    lat = gpu_lattice(4, dims, dx, spec, bc=[bc] * 4)
    try:
        print(f"[long] D4Q33 {dims} {bc}", flush=True)
        for n in (1, 6):
            lat.step(n - lat.info()["step"])
            run.step(n - run.n)
            err = rel_l2(to_oracle_order(lat.phi().cpu().numpy()), run.phi())
            assert err <= 1e-12, (n, err)
    finally:
        lat.close()


# ------------------------------------------------------- precision contract --

def test_split_layouts_hold_the_discretisation_error_at_512():
    """The benchmark lattice (D3Q19 512^3 full-way, the benchmark field) over
    200 steps in every storage mode: the float32-split and hi/lo runs stay
    within a fifth of float64's own discretisation error (relative RMSE against
    the exact solution) of the float64 run; plain float32 does not, and its
    drift is printed beside them."""
    from paper_2410_13165_amd import Lattice
    w = inputs.BENCH_D3Q19
    n, steps = w["n"], 200
    spec = inputs.bench_field()
    phis, disc = {}, None
    for precision in ("fp64", "fp32_split", "fp32_hilo", "fp32"):
        print(f"[contract] {precision} 512^3 x {steps}", flush=True)
        lat = Lattice(3, (n, n, n), 0.5, dx=1.0 / (n - 1), u=spec["u"], R=spec["R"],
                      bc=["fullway"] * 3, precision=precision, field=spec)
        try:
            lat.step(steps)
            phis[precision] = lat.phi().clone()
            if precision == "fp64":
                dg = lat.diagnostics()
                disc = dg["rmse"] * math.sqrt(n ** 3) / float(phis["fp64"].norm())
        finally:
            lat.close()
            torch.cuda.empty_cache()
    ref = phis.pop("fp64")
    drift = {m: float((p - ref).norm()) / float(ref.norm()) for m, p in phis.items()}
    print(f"[contract] float64 relative discretisation error {disc:.3e}; drift {drift}", flush=True)
    assert drift["fp32_split"] < 0.2 * disc
    assert drift["fp32_hilo"] < 0.2 * disc
    assert drift["fp32"] > disc
