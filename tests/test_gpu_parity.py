"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: float64 storage 1e-12 relative (L2 of phi, and max-abs of the
populations relative to their scale); float32 storage 2e-5 relative on runs of
at most a few hundred steps; float32-split 2e-5 relative.  Sizes are ragged and
span several blocks along x_1 and several rows.
"""
import math

import numpy as np
import pytest

from oracle import lbm_oracle as O
from paper_2410_13165_amd import inputs
from tests.pairs import (gpu_lattice, gpu_populations, local_oracle_phi, oracle_problem,
                         rel_l2, to_oracle_order)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-12, "fp32": 2e-5, "fp32_split": 2e-5, "fp32_hilo": 2e-5}


def _phi(lat):
    return to_oracle_order(lat.phi().cpu().numpy())


def _check_pair(d, dims, dx, spec, steps, bc=None, P=4, K=3, tau=0.5, precision="fp64",
                origin=None, populations=True, wall_data="jets"):
    prob = oracle_problem(d, dims, dx, spec, tau=tau, bc=bc, P=P, K=K, origin=origin,
                          wall_data=wall_data)
    run = O.Run(prob)
    lat = gpu_lattice(d, dims, dx, spec, tau=tau, bc=bc, P=P, K=K, origin=origin,
                      precision=precision, wall_data=wall_data)
    try:
        print(f"[parity] d={d} dims={dims} bc={bc} P={P} K={K} tau={tau} {precision} "
              f"steps={steps} wall_data={wall_data}", flush=True)
        # step 0, then a few steps, then the rest
        for n in (0, 1, steps):
            lat.step(n - lat.info()["step"])
            run.step(n - run.n)
            err = rel_l2(_phi(lat), run.phi())
            assert err <= TOL[precision], (n, err)
            if populations and precision == "fp64":
                want = run.collide()
                got = gpu_populations(lat)
                scale = np.max(np.abs(want))
                assert np.max(np.abs(got - want)) <= 1e-12 * scale, n
        return lat, run
    finally:
        lat.close()


# ------------------------------------------------------------- periodic ----

@pytest.mark.parametrize("d,dims", [(1, (300,)), (2, (261, 37)), (3, (67, 29, 23)),
                                    (4, (13, 9, 7, 5))])
@pytest.mark.parametrize("tau", [0.5, 0.8])
def test_periodic_fp64(d, dims, tau):
    spec = inputs.random_cosines(d, [0.1, 0.2, 0.08, 0.05][:d], 0.7, seed=d)
    _check_pair(d, dims, 1.0 / dims[0], spec, 17, tau=tau)


@pytest.mark.parametrize("d,dims", [(2, (130, 67)), (3, (70, 33, 17))])
@pytest.mark.parametrize("precision", ["fp32", "fp32_split", "fp32_hilo"])
def test_periodic_reduced_precision(d, dims, precision):
    spec = inputs.random_cosines(d, [0.1, 0.2, 0.08][:d], 0.4, seed=10 + d)
    _check_pair(d, dims, 1.0 / dims[0], spec, 60, precision=precision)


# ------------------------------------------------------------- Dirichlet ---

@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
@pytest.mark.parametrize("d,dims", [(1, (97,)), (2, (77, 41)), (3, (35, 19, 23)),
                                    (4, (11, 8, 7, 6))])
def test_dirichlet_fp64(scheme, d, dims):
    u = [0.05, 0.1, 0.08, 0.03][:d]
    spec = inputs.random_cosines(d, u, 1.0, seed=20 + d, kmax=1.0)
    _check_pair(d, dims, 1.0 / (dims[0] - 1), spec, 15, bc=[scheme] * d)


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
@pytest.mark.parametrize("d,dims,precision", [(2, (45, 33), "fp64"), (2, (45, 33), "fp32"),
                                              (3, (35, 19, 23), "fp64"),
                                              (3, (35, 19, 23), "fp32_split"),
                                              (4, (11, 8, 7, 6), "fp64")])
def test_dirichlet_tau_not_one_half(scheme, d, dims, precision):
    """Walls with s = 1/tau != 2: the collision's (1 - s) f_k term, and with it the
    half-way schemes' -f*_kbar of the node, no longer vanish."""
    u = [0.05, 0.1, 0.08, 0.03][:d]
    spec = inputs.random_cosines(d, u, 1.0, seed=25 + d, kmax=1.0)
    _check_pair(d, dims, 1.0 / (dims[0] - 1), spec, 15, bc=[scheme] * d, tau=0.8,
                precision=precision)


@pytest.mark.parametrize("scheme,P", [("fullway", 1), ("fullway", 3), ("halfway", 1),
                                      ("halfway", 2), ("halfway", 3)])
def test_dirichlet_lower_orders(scheme, P):
    spec = inputs.example1([0.1, 0.1])
    n = 21 if scheme == "fullway" else 20
    _check_pair(2, (n, n), 1.0 / 20, spec, 30, bc=[scheme] * 2, P=P)


@pytest.mark.parametrize("scheme,P", [("fullway", 1), ("fullway", 3), ("halfway", 1),
                                      ("halfway", 2), ("halfway", 3)])
@pytest.mark.parametrize("d,dims,precision", [(3, (30, 17, 14), "fp64"),
                                              (3, (30, 17, 14), "fp32_split"),
                                              (4, (9, 8, 7, 6), "fp64")])
def test_dirichlet_lower_orders_d3_d4(scheme, P, d, dims, precision):
    """Wall orders below 4 (and K = 1 initialisation) in the wall-row kernels and
    the two-step passes of d = 3 and the wall rows of d = 4."""
    u = [0.05, 0.1, 0.08, 0.03][:d]
    spec = inputs.random_cosines(d, u, 1.0, seed=30 + d + P, kmax=1.0)
    _check_pair(d, dims, 1.0 / (dims[0] - 1), spec, 12, bc=[scheme] * d, P=P, K=1,
                precision=precision)


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
def test_mixed_periodic_and_dirichlet_axes(scheme):
    spec = inputs.random_cosines(3, [0.05, -0.1, 0.08], 0.5, seed=31, kmax=1.0)
    _check_pair(3, (40, 18, 21), 1.0 / 39, spec, 12, bc=["periodic", scheme, scheme])
    _check_pair(3, (40, 18, 21), 1.0 / 39, spec, 12, bc=[scheme, "periodic", scheme])
    # the same lattices with the faces given one by one (lbm_params.bc[a][side])
    _check_pair(3, (40, 18, 21), 1.0 / 39, spec, 12,
                bc=[(scheme, scheme), ("periodic", "periodic"), (scheme, scheme)])


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_dirichlet_rows_longer_than_a_block(scheme, precision):
    """300 nodes along x_1: the wall-row kernels of d >= 3 take one node per
    thread, in a full chunk of 256 and a ragged one of 44; the two-step passes
    span five x_1 tiles, the last ragged."""
    spec = inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0, seed=43, kmax=1.0)
    _check_pair(3, (300, 9, 8), 1.0 / 299, spec, 12, bc=[scheme] * 3, precision=precision)


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
@pytest.mark.parametrize("precision", ["fp32", "fp32_split", "fp32_hilo"])
def test_dirichlet_reduced_precision(scheme, precision):
    spec = inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0, seed=41, kmax=1.0)
    _check_pair(3, (45, 22, 19), 1.0 / 44, spec, 80, bc=[scheme] * 3, precision=precision)


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
@pytest.mark.parametrize("d,dims", [(2, (41, 30)), (3, (23, 17, 19)), (4, (9, 8, 7, 6))])
def test_tangential_wall_data(scheme, d, dims):
    """Remark 1: walls fed only by the data on the wall (time and tangential
    derivatives; normal ones from the equation).  GPU against the oracle's
    Remark-1 construction, and against the GPU's own jets path to rounding."""
    u = [0.05, -0.1, 0.08, 0.03][:d]
    spec = inputs.random_cosines(d, u, 0.6, seed=50 + d, kmax=1.0)
    dx = 1.0 / (dims[0] - 1)
    _check_pair(d, dims, dx, spec, 12, bc=[scheme] * d, wall_data="tangential")
    a = gpu_lattice(d, dims, dx, spec, bc=[scheme] * d, wall_data="tangential")
    b = gpu_lattice(d, dims, dx, spec, bc=[scheme] * d)
    try:
        a.step(30)
        b.step(30)
        assert rel_l2(_phi(a), _phi(b)) <= 1e-13
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp32_split", "fp32_hilo"])
def test_tangential_wall_data_reduced_precision_and_lower_order(precision):
    spec = inputs.example1([0.1, 0.1])
    _check_pair(2, (21, 21), 1.0 / 20, spec, 40, bc=["fullway"] * 2, P=3,
                wall_data="tangential")
    _check_pair(2, (20, 20), 1.0 / 20, spec, 40, bc=["halfway"] * 2, P=3,
                wall_data="tangential")
    _check_pair(3, (33, 19, 17), 1.0 / 32, inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0,
                                                                 seed=57, kmax=1.0),
                60, bc=["fullway"] * 3, precision=precision, wall_data="tangential")


def _node_state(lat):
    """Populations (split modes: g_k and the 8 bytes of phi) of the nodes, without the padding
    and x_1-face slots of the state blob."""
    info = lat.info()
    q, ps, nodes = info["q"], info["pstride"], info["nodes"]
    blob = lat.get_state()
    if lat.precision == "fp64":
        return blob.view(torch.float64).reshape(q, ps)[:, :nodes].clone()
    pop = blob[: q * ps * 4].view(torch.float32).reshape(q, ps)[:, :nodes]
    if lat.precision == "fp32":
        return pop.clone()
    phi = blob[q * ps * 4:].view(torch.float64)[:nodes]
    return torch.cat([pop.reshape(-1).view(torch.int32).to(torch.int64),
                      phi.view(torch.int64)])


@pytest.mark.parametrize("dims,bc,wall_data", [
    ((67, 29, 23), ["periodic"] * 3, "jets"),
    ((45, 30, 70), ["fullway"] * 3, "jets"),
    ((44, 27, 66), ["halfway"] * 3, "jets"),
    ((40, 18, 21), ["periodic", "fullway", "fullway"], "jets"),
    ((40, 18, 21), ["fullway", "periodic", "fullway"], "jets"),
    ((40, 18, 21), ["halfway", "halfway", "periodic"], "jets"),
    ((70, 15, 9), ["fullway"] * 3, "tangential"),
    ((3, 2, 5), ["fullway"] * 3, "jets"),
    ((5, 4, 3), ["periodic"] * 3, "jets"),
])
@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp32_split", "fp32_hilo"])
def test_two_step_passes_equal_single_steps_bitwise(dims, bc, wall_data, precision):
    """d = 3: steps taken two per bulk pass (intermediate state in LDS) give
    bitwise the populations of single steps, for periodic, full-way, half-way
    and mixed axes, ragged tiles and z-chunks, and odd step counts."""
    spec = inputs.random_cosines(3, [0.05, -0.1, 0.08], 0.7, seed=71, kmax=1.0)
    dx = 1.0 / max(dims[0] - 1, 1)
    a = gpu_lattice(3, dims, dx, spec, bc=bc, precision=precision, wall_data=wall_data)
    from paper_2410_13165_amd import Lattice
    b = Lattice(3, dims, 0.5, dx=dx, u=spec["u"], R=spec.get("R", 0.0), bc=bc, P=4, K=3,
                precision=precision, field=spec, wall_data=wall_data, steps_per_pass=1)
    try:
        assert a.info()["steps_per_pass"] == 2 and b.info()["steps_per_pass"] == 1
        print(f"[fused] dims={dims} bc={bc} {wall_data} {precision}", flush=True)
        for n in (2, 5, 14):
            a.step(n)
            b.step(n)
            assert a.info()["step"] == b.info()["step"]
            assert torch.equal(_node_state(a), _node_state(b)), n
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("dims,bc,wall_data", [
    ((261, 37), ["periodic"] * 2, "jets"),
    ((77, 41), ["fullway"] * 2, "jets"),
    ((76, 40), ["halfway"] * 2, "jets"),
    ((300, 19), ["periodic", "fullway"], "jets"),
    ((600, 21), ["fullway", "periodic"], "jets"),
    ((70, 30), ["halfway"] * 2, "tangential"),
    ((3, 2), ["fullway"] * 2, "jets"),
    ((520, 700), ["fullway"] * 2, "jets"),
])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_two_step_passes_d2_equal_single_steps_bitwise(dims, bc, wall_data, precision):
    """d = 2: the same check for the row-marching two-step pass (several tiles
    along x_1, ragged row chunks, walls on either axis)."""
    spec = inputs.random_cosines(2, [0.1, -0.15], 0.7, seed=73, kmax=1.0)
    dx = 1.0 / max(dims[0] - 1, 1)
    from paper_2410_13165_amd import Lattice
    a = gpu_lattice(2, dims, dx, spec, bc=bc, precision=precision, wall_data=wall_data)
    b = Lattice(2, dims, 0.5, dx=dx, u=spec["u"], R=spec.get("R", 0.0), bc=bc, P=4, K=3,
                precision=precision, field=spec, wall_data=wall_data, steps_per_pass=1)
    try:
        assert a.info()["steps_per_pass"] == 2 and b.info()["steps_per_pass"] == 1
        print(f"[fused2d] dims={dims} bc={bc} {wall_data} {precision}", flush=True)
        for n in (2, 5, 14):
            a.step(n)
            b.step(n)
            assert torch.equal(_node_state(a), _node_state(b)), n
    finally:
        a.close()
        b.close()


def test_two_step_profile_counts_passes():
    spec = inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0, seed=72, kmax=1.0)
    lat = gpu_lattice(3, (40, 30, 20), 1.0 / 39, spec, bc=["fullway"] * 3, precision="fp32")
    try:
        lat.profile_begin(10)
        lat.step(7)
        prof = lat.profile_end()
        assert prof["steps"] == 7 and prof["launches"] == 4
        assert prof["bulk_ms"] > 0 and prof["wall_ms"] > 0
    finally:
        lat.close()


def test_example1_source_term_fp32_reference():
    """R = 5 makes phi grow like R t; the float32 mode stores deviations from the
    uniform state omega (mean phi0 + R t) and must keep its accuracy."""
    spec = inputs.example1([0.1, 0.1])
    _check_pair(2, (41, 41), 1.0 / 40, spec, 200, bc=["fullway"] * 2, precision="fp32")
    _check_pair(2, (41, 41), 1.0 / 40, spec, 200, bc=["fullway"] * 2, precision="fp32_split")
    _check_pair(2, (41, 41), 1.0 / 40, spec, 200, bc=["fullway"] * 2, precision="fp32_hilo")


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
def test_exponential_field_d3(scheme):
    """An exponential exact solution in 3D: the d = 3 wall kernels of the
    exponential variants (full-way and half-way) against the oracle, float64
    at order 4 and the split mode at order 3."""
    spec = {"kind": "exp_sum", "amps": [0.7, -0.4], "kvecs": [[-1.0, 0.5, 0.8], [0.6, -0.9, 0.3]],
            "phases": [0.0, 0.0], "u": [0.06, -0.05, 0.08], "R": 0.5}
    _check_pair(3, (26, 19, 21), 1.0 / 25, spec, 20, bc=[scheme] * 3)
    _check_pair(3, (26, 19, 21), 1.0 / 25, spec, 20, bc=[scheme] * 3, P=3,
                precision="fp32_split")


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_split", "fp32_hilo"])
def test_dirichlet_fields_past_the_mode_cache(scheme, precision):
    """Six modes, more than the half-way wall kernels of d = 3 keep in registers:
    they then take one population at a time, with every mode past the first
    evaluated again per population (cosine and exponential fields, jets and
    tangential wall data).  Four modes take the register path elsewhere."""
    spec = inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0, seed=44, n_modes=6, kmax=1.0)
    _check_pair(3, (27, 14, 12), 1.0 / 26, spec, 12, bc=[scheme] * 3, precision=precision)
    _check_pair(3, (27, 14, 12), 1.0 / 26, spec, 12, bc=[scheme] * 3, precision=precision,
                wall_data="tangential")
    rng = np.random.default_rng(45)
    espec = {"kind": "exp_sum", "amps": rng.normal(size=6).tolist(),
             "kvecs": rng.uniform(-1.0, 1.0, size=(6, 3)).tolist(), "phases": [0.0] * 6,
             "u": [0.06, -0.05, 0.08], "R": 0.5}
    _check_pair(3, (27, 14, 12), 1.0 / 26, espec, 12, bc=[scheme] * 3, precision=precision)


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
@pytest.mark.parametrize("precision", ["fp32", "fp32_split", "fp32_hilo"])
def test_dirichlet_d4_reduced_precision(scheme, precision):
    """The D4Q33 wall-row kernels of the float32 storage modes against the oracle."""
    spec = inputs.random_cosines(4, [0.05, 0.1, 0.08, 0.03], 1.0, seed=24, kmax=1.0)
    _check_pair(4, (11, 8, 7, 6), 1.0 / 10, spec, 15, bc=[scheme] * 4, precision=precision)


def test_example3_d4q33_halfway_small_u():
    spec = inputs.diagonal_sine(4, [1e-3] * 4)
    _check_pair(4, (10, 10, 10, 10), 0.2, spec, 8, bc=["halfway"] * 4, origin=[-1.0] * 4)


# ----------------------------------------------- initial data from device ---

@pytest.mark.parametrize("K", [1, 3])
def test_set_initial_noise_and_fd_gradient(K):
    d, dims = 2, (64, 48)
    phi0 = inputs.noise((dims[1], dims[0]), seed=4)  # GPU layout (N_2, N_1)
    prob = oracle_problem(d, dims, 1.0 / 64, None, u=[0.3, -0.2], K=K)
    run = O.Run(prob, phi0=to_oracle_order(phi0))
    lat = gpu_lattice(d, dims, 1.0 / 64, None, u=[0.3, -0.2], K=K)
    try:
        lat.set_initial(torch.from_numpy(phi0.ravel()))
        for n in (0, 1, 25):
            lat.step(n - lat.info()["step"])
            run.step(n - run.n)
            assert rel_l2(_phi(lat), run.phi()) <= 1e-12
    finally:
        lat.close()


@pytest.mark.parametrize("d,dims", [(1, (50,)), (3, (20, 14, 9)), (4, (9, 7, 6, 5))])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_split", 2e-5)])
@pytest.mark.parametrize("K", [1, 3])
def test_set_initial_fd_gradient_all_dims(d, dims, precision, tol, K):
    """A device phi^0 with the fourth-order finite-difference gradient on every
    axis of d = 1, 3 and 4 (and K = 1), in float64 and the split storage."""
    u = [0.3, -0.2, 0.1, 0.15][:d]
    phi0 = inputs.noise(tuple(reversed(dims)), seed=5 + d)  # GPU layout (N_d, ..., N_1)
    prob = oracle_problem(d, dims, 1.0 / dims[0], None, u=u, K=K)
    run = O.Run(prob, phi0=to_oracle_order(phi0))
    lat = gpu_lattice(d, dims, 1.0 / dims[0], None, u=u, K=K, precision=precision)
    try:
        lat.set_initial(torch.from_numpy(phi0.ravel()))
        for n in (0, 1, 14):
            lat.step(n - lat.info()["step"])
            run.step(n - run.n)
            assert rel_l2(_phi(lat), run.phi()) <= tol, n
    finally:
        lat.close()


def test_set_initial_with_gradient():
    d, dims = 3, (20, 12, 9)
    rng = np.random.default_rng(9)
    phi0 = rng.normal(size=tuple(reversed(dims)))
    grad = rng.normal(size=(d,) + tuple(reversed(dims)))
    prob = oracle_problem(d, dims, 0.05, None, u=[0.1, 0.05, -0.1])
    g_or = np.stack([to_oracle_order(grad[a]) for a in range(d)], axis=-1)
    run = O.Run(prob, phi0=to_oracle_order(phi0), grad0=g_or)
    lat = gpu_lattice(d, dims, 0.05, None, u=[0.1, 0.05, -0.1])
    try:
        lat.set_initial(torch.from_numpy(phi0.ravel()), torch.from_numpy(grad.ravel()))
        lat.step(9)
        run.step(9)
        assert rel_l2(_phi(lat), run.phi()) <= 1e-12
    finally:
        lat.close()


# ----------------------------------------------------------- diagnostics ---

@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_split", "fp32_hilo"])
def test_diagnostics_match_oracle(precision):
    spec = inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0, seed=51, kmax=1.0)
    dims = (33, 17, 12)
    prob = oracle_problem(3, dims, 1.0 / 32, spec, bc=["fullway"] * 3)
    run = O.Run(prob).step(20)
    lat = gpu_lattice(3, dims, 1.0 / 32, spec, bc=["fullway"] * 3, precision=precision)
    try:
        lat.step(20)
        dg = lat.diagnostics()
        tol = 1e-12 if precision == "fp64" else 2e-5
        assert abs(dg["sum_phi"] - run.mass()) <= tol * np.sum(np.abs(run.phi()))
        assert abs(dg["entropy"] - run.entropy()) <= tol * abs(run.entropy())
        assert abs(dg["rmse"] - run.rmse()) <= max(tol * 10, 1e-3 * run.rmse())
        assert abs(dg["t"] - run.t) < 1e-15
        assert dg["nonfinite"] == 0
        assert abs(dg["max_abs_phi"] - np.max(np.abs(run.phi()))) <= tol * 10
    finally:
        lat.close()


def test_entropy_conserved_on_gpu_and_nan_at_tau_one():
    spec = inputs.random_cosines(2, [0.1, 0.2], 0.0, seed=61)
    lat = gpu_lattice(2, (256, 200), 1.0 / 256, spec)
    try:
        e0 = lat.diagnostics()["entropy"]
        lat.step(300)
        assert abs(lat.diagnostics()["entropy"] / e0 - 1) < 1e-12
    finally:
        lat.close()
    lat = gpu_lattice(2, (16, 16), 1.0 / 16, spec, tau=1.0)
    try:
        assert math.isnan(lat.diagnostics()["entropy"])
    finally:
        lat.close()


# -------------------------------------------------------- state and edges ---

@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_split", "fp32_hilo"])
def test_checkpoint_roundtrip_is_bitwise(precision):
    spec = inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0, seed=71, kmax=1.0)
    kw = dict(bc=["fullway"] * 3, precision=precision)
    a = gpu_lattice(3, (30, 20, 10), 1.0 / 29, spec, **kw)
    b = gpu_lattice(3, (30, 20, 10), 1.0 / 29, spec, **kw)
    try:
        a.step(7)
        snap = a.get_state().clone()
        a.step(5)
        b.set_state(snap, 7).step(5)
        assert torch.equal(a.phi(), b.phi())
        assert a.info()["step"] == b.info()["step"] == 12
    finally:
        a.close()
        b.close()


def test_runs_are_deterministic():
    spec = inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0, seed=72, kmax=1.0)
    res = []
    for _ in range(2):
        lat = gpu_lattice(3, (40, 30, 20), 1.0 / 39, spec, bc=["halfway"] * 3)
        try:
            lat.step(11)
            res.append((lat.phi().cpu().numpy(), lat.diagnostics()))
        finally:
            lat.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]


@pytest.mark.parametrize("dims,bc", [((1, 30), ["periodic", "periodic"]),
                                     ((2, 9), ["fullway", "fullway"]),
                                     ((2, 2), ["halfway", "halfway"]),
                                     ((5, 1, 7), ["periodic", "periodic", "periodic"])])
def test_degenerate_sizes(dims, bc):
    d = len(dims)
    spec = inputs.random_cosines(d, [0.1, -0.05, 0.02][:d], 0.3, seed=81, kmax=1.0)
    _check_pair(d, dims, 0.1, spec, 6, bc=bc)


@pytest.mark.parametrize("dims,scheme", [((2, 3, 2), "fullway"), ((3, 3, 3), "halfway"),
                                         ((70, 2, 3), "fullway"), ((65, 3, 2), "halfway"),
                                         ((3, 2, 3, 2), "fullway"), ((2, 3, 2, 3), "halfway")])
@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_degenerate_sizes_with_walls(dims, scheme, precision):
    """Lattices with two or three nodes on Dirichlet axes: every row, or every row
    but one, lies on or next to a wall, so the two-step passes of d = 3 update
    little or nothing themselves and the wall-row kernels carry the lattice."""
    d = len(dims)
    spec = inputs.random_cosines(d, [0.1, -0.05, 0.02, 0.04][:d], 0.3, seed=84, kmax=1.0)
    _check_pair(d, dims, 0.1, spec, 6, bc=[scheme] * d, precision=precision)


def test_zero_steps_and_error_reporting():
    from paper_2410_13165_amd import LbmError
    spec = inputs.random_cosines(2, [0.1, 0.1], 0.0, seed=82)
    lat = gpu_lattice(2, (16, 16), 1.0 / 16, spec)
    try:
        before = lat.phi().clone()
        lat.step(0)
        assert torch.equal(before, lat.phi())
        with pytest.raises(LbmError):
            lat.step(-1)
    finally:
        lat.close()
    # walls need a field; a lattice without field needs lbm_set_initial
    lat = gpu_lattice(2, (16, 16), 1.0 / 16, None, u=[0.1, 0.1])
    try:
        with pytest.raises(LbmError, match="initial"):
            lat.step(1)
    finally:
        lat.close()


# ------------------------------------------------------- full-size check ---

@pytest.mark.parametrize("precision,scheme", [("fp32", "fullway"), ("fp64", "fullway"),
                                              ("fp32_split", "fullway"), ("fp32_hilo", "fullway"),
                                              ("fp32", "halfway"), ("fp64", "halfway"),
                                              ("fp32_split", "halfway"), ("fp32_hilo", "halfway")])
def test_benchmark_configuration_sampled(precision, scheme):
    """D3Q19, 512^3 nodes, full-way (the benchmark) or half-way walls on all
    faces, in the benchmark's launch configuration (a two-step pass, then one
    single step): after r = 3 steps, phi at sampled nodes (interior, faces,
    edges, corners) against oracle runs on the sub-boxes of radius r around
    them."""
    w = inputs.BENCH_D3Q19
    n, r = w["n"], 3
    spec = inputs.bench_field()
    dx = 1.0 / (n - 1) if scheme == "fullway" else 1.0 / n
    bc = [scheme] * 3
    lat = gpu_lattice(3, (n, n, n), dx, spec, bc=bc, precision=precision)
    try:
        lat.step(r)
        phi = lat.phi()  # (z, y, x)
        rng = np.random.default_rng(5)
        samples = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, 200, 300), (511, 17, 1), (1, 1, 1),
                   (256, 0, 511), (2, 255, 510)]
        samples += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(6)]
        tol = TOL[precision]
        for idx in samples:
            want = local_oracle_phi(3, (n, n, n), dx, spec, bc, idx, r)
            got = float(phi[idx[2], idx[1], idx[0]])
            print(f"[sample] {precision} {scheme} {idx} got={got:.15g} want={want:.15g}",
                  flush=True)
            assert abs(got - want) <= tol * max(1.0, abs(want)), idx
    finally:
        lat.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_d2q9_2048_sampled(precision):
    """D2Q9 2048^2 periodic, the plane-wave workload of the grid-refinement
    study at its finest grid, in the benchmark's launch configuration (two
    steps per pass for d = 2, then one single step): after r = 5 steps, phi at
    sampled nodes against oracle runs on the sub-boxes of radius r."""
    n, r = 2048, 5
    spec = inputs.plane_sine(2, [0.1, 0.2])
    dx = 1.0 / n
    bc = ["periodic"] * 2
    lat = gpu_lattice(2, (n, n), dx, spec, bc=bc, precision=precision)
    try:
        assert lat.info()["steps_per_pass"] == 2
        lat.step(r)
        phi = lat.phi()  # (y, x)
        rng = np.random.default_rng(6)
        samples = [(r, r), (n - 1 - r, n - 1 - r), (1023, 1024), (255, 1790)]
        samples += [tuple(int(v) for v in rng.integers(r, n - r, 2)) for _ in range(8)]
        tol = TOL[precision]
        for idx in samples:
            want = local_oracle_phi(2, (n, n), dx, spec, bc, idx, r)
            got = float(phi[idx[1], idx[0]])
            print(f"[sample] d2q9 {precision} {idx} got={got:.15g} want={want:.15g}", flush=True)
            assert abs(got - want) <= tol * max(1.0, abs(want)), idx
    finally:
        lat.close()


def test_d2q9_fourth_order_convergence_fp64():
    """The plane-wave refinement study on the GPU (D2Q9, tau = 1/2, float64,
    64^2 .. 512^2, n steps to t = 1): the error ratio per halving of dx
    approaches 16, the fourth order of the method under acoustic scaling."""
    spec = inputs.plane_sine(2, [0.1, 0.2])
    errs = []
    for n in (64, 128, 256, 512):
        lat = gpu_lattice(2, (n, n), 1.0 / n, spec, precision="fp64")
        try:
            lat.step(n)
            errs.append(lat.diagnostics()["rmse"])
        finally:
            lat.close()
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(f"[convergence] rmse {errs} orders {orders}", flush=True)
    assert all(o > 3.7 for o in orders), orders
    assert abs(orders[-1] - 4.0) <= 0.15, orders


# --------------------------------------------------- Example 2 bubble ------

@pytest.mark.parametrize("d,n,K,precision", [(2, 100, 1, "fp64"), (2, 99, 3, "fp64"),
                                             (3, 39, 3, "fp64"), (2, 99, 3, "fp32_split"),
                                             (2, 95, 3, "fp32")])
def test_tanh_bubble_example2(d, n, K, precision):
    """Example 2: the periodic tanh bubble on [(d-4)/2, (4-d)/2]^d with
    Rr = 1/(5(d-1)), W = (5-d)/75, initialised in the kernel from the analytic
    value (K = 1) or value and gradient (K = 3), against the oracle; the RMSE
    of the device reduction (analytic bubble per node) against the oracle's.
    With K = 3 the node count is odd: the bubble's gradient is undefined at its
    centre (a conical kink), where a node coordinate rounding to 1e-17 instead
    of 0 picks an arbitrary direction of a non-zero slope."""
    u = [0.05, 0.1, 0.08][:d]
    spec = inputs.tanh_bubble(d, u)
    L = 4.0 - d
    dx = L / n
    origin = [(d - 4) / 2.0] * d
    steps = n // 4
    _check_pair(d, (n,) * d, dx, spec, steps, K=K, origin=origin, precision=precision)
    run = O.Run(oracle_problem(d, (n,) * d, dx, spec, K=K, origin=origin)).step(steps)
    lat = gpu_lattice(d, (n,) * d, dx, spec, K=K, origin=origin, precision=precision)
    try:
        lat.step(steps)
        dg = lat.diagnostics()
    finally:
        lat.close()
    print(f"[tanh] d={d} n={n} K={K} {precision}: rmse {dg['rmse']:.6e} oracle {run.rmse():.6e}",
          flush=True)
    # |RMSE_gpu - RMSE_oracle| <= RMS of the difference, and phi is O(1) here
    tol = max(1e-10, 1e-6 * run.rmse()) if precision == "fp64" else TOL[precision]
    assert abs(dg["rmse"] - run.rmse()) <= tol


# ------------------------------------------- moments mask, non-finite check --

def test_moments_what_mask():
    """lbm_moments computes only what its mask selects: the phi field alone,
    the sums without the per-node analytic field (RMSE NaN), each scalar group
    equal to the full request's."""
    from paper_2410_13165_amd import lbm as B
    spec = inputs.random_cosines(3, [0.05, 0.1, 0.08], 1.0, seed=83, kmax=1.0)
    lat = gpu_lattice(3, (33, 17, 12), 1.0 / 32, spec, bc=["fullway"] * 3)
    try:
        lat.step(9)
        full = lat.diagnostics()
        sums = lat.diagnostics(B.MOM_SUMS)
        err = lat.diagnostics(B.MOM_RMSE)
        ent = lat.diagnostics(B.MOM_ENTROPY)
        for k in ("sum_phi", "sum_phi2", "max_abs_phi", "nonfinite"):
            assert sums[k] == full[k] and math.isnan(err[k]) and math.isnan(ent[k])
        assert math.isnan(sums["rmse"]) and math.isnan(sums["entropy"])
        assert err["rmse"] == full["rmse"] and err["sum_err2"] == full["sum_err2"]
        assert ent["entropy"] == full["entropy"]
        assert sums["t"] == full["t"]
        phi = lat.phi()
        out = torch.empty_like(phi).reshape(-1)
        lib = lat.lib
        assert lib.lbm_moments(lat.handle, B.MOM_PHI, B.C.c_void_p(out.data_ptr()), None) == 0
        assert torch.equal(out.view_as(phi), phi)
        # a selected output without its pointer, or unknown bits, are refused
        assert lib.lbm_moments(lat.handle, B.MOM_PHI, None, None) == B.EINVAL
        assert lib.lbm_moments(lat.handle, B.MOM_SUMS, None, None) == B.EINVAL
        assert lib.lbm_moments(lat.handle, 64, None, None) == B.EINVAL
        assert lib.lbm_moments(lat.handle, 0, None, None) == 0
    finally:
        lat.close()


def _checked_lattice(precision, n, check_every, bc="halfway"):
    from paper_2410_13165_amd import Lattice
    spec = inputs.example1([0.4, 0.4])
    return Lattice(2, (n, n), 0.5, dx=1.0 / n, u=spec["u"], R=spec["R"], bc=[bc] * 2,
                   precision=precision, field=spec, check_every=check_every)


@pytest.mark.parametrize("precision,steps", [("fp32", 1000), ("fp64", 6000),
                                             ("fp32_split", 6000), ("fp32_hilo", 6000)])
def test_nonfinite_check_reports_blow_up(precision, steps):
    """Table 1's diverging row (half-way walls at u = (0.4, 0.4), Example 1,
    80 nodes per axis): the values overflow (float32 within 1000 steps, float64
    within 6000) and lbm_step returns LBM_ENONFINITE from its periodic check."""
    from paper_2410_13165_amd import LbmError
    from paper_2410_13165_amd import lbm as B
    lat = _checked_lattice(precision, 80, 50)
    try:
        print(f"[nonfinite] {precision} {steps}", flush=True)
        with pytest.raises(LbmError, match="non-finite") as ei:
            lat.step(steps)
        assert ei.value.code == B.ENONFINITE
        assert lat.diagnostics()["nonfinite"] > 0
    finally:
        lat.close()


def test_nonfinite_check_catches_nan_initial_field():
    from paper_2410_13165_amd import Lattice, LbmError
    from paper_2410_13165_amd import lbm as B
    phi0 = torch.from_numpy(inputs.noise((40, 48), seed=3))
    phi0[17, 5] = float("nan")
    for precision in ("fp64", "fp32", "fp32_split", "fp32_hilo"):
        lat = Lattice(2, (48, 40), 0.5, dx=1 / 48, u=[0.1, 0.2], precision=precision,
                      check_every=4)
        try:
            lat.set_initial(phi0.reshape(-1))
            lat.step(3)  # no check is due yet
            with pytest.raises(LbmError) as ei:
                lat.step(1)
            assert ei.value.code == B.ENONFINITE
        finally:
            lat.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_split", "fp32_hilo"])
def test_nonfinite_check_leaves_results_unchanged(precision):
    a = _checked_lattice(precision, 40, 3, bc="fullway")
    b = _checked_lattice(precision, 40, 0, bc="fullway")
    try:
        a.step(20)
        b.step(20)
        assert torch.equal(a.phi(), b.phi())
    finally:
        a.close()
        b.close()
