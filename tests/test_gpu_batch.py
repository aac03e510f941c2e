"""Batched lattices (one launch per step over all instances) against
per-instance oracle runs, and the stability sweep against the oracle's
brute-force spectral radius of the amplification matrix."""
import itertools

import numpy as np
import pytest

from oracle import lbm_oracle as O
from paper_2410_13165_amd import inputs
from tests.pairs import oracle_problem, rel_l2, to_oracle_order

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _specs(rng, count, sizes, tau_range, sig_range, d=2):
    specs = []
    for i in range(count):
        n = sizes[rng.integers(0, len(sizes))]
        dims = (n + int(rng.integers(0, 7)), n - int(rng.integers(0, 5)))[:d]
        specs.append({"dims": dims, "tau": float(rng.uniform(*tau_range)),
                      "u": rng.uniform(*sig_range, size=d).tolist(), "dx": 1.0 / dims[0]})
    return specs


def _concat_phi0(specs, seed):
    parts = [inputs.noise(tuple(reversed(sp["dims"])), seed + i, std=1e-3).ravel()
             for i, sp in enumerate(specs)]
    return parts, torch.from_numpy(np.concatenate(parts))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
@pytest.mark.parametrize("K", [1, 3])
def test_batch_matches_oracle_per_instance(precision, tol, K):
    from paper_2410_13165_amd import Batch
    rng = np.random.default_rng(40 + K)
    specs = _specs(rng, 7, [16, 24, 40], (0.5, 1.4), (-0.45, 0.45))
    for sp in specs:
        sp["K"] = K
    parts, phi0 = _concat_phi0(specs, 500)
    steps = 25
    with Batch(2, specs, precision=precision) as b:
        b.set_initial(phi0)
        b.step(steps)
        for i, sp in enumerate(specs):
            prob = oracle_problem(2, sp["dims"], sp["dx"], None, u=sp["u"], tau=sp["tau"], K=K)
            run = O.Run(prob, phi0=to_oracle_order(parts[i].reshape(tuple(reversed(sp["dims"])))))
            run.step(steps)
            got = to_oracle_order(b.instance(i).phi().cpu().numpy())
            assert rel_l2(got, run.phi()) <= tol, (i, sp)


@pytest.mark.parametrize("d", [1, 3, 4])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_batch_other_dimensions_match_oracle(d, precision, tol):
    """Batches of D1Q3, D3Q19 and D4Q33 lattices of uneven sizes, each with its own
    tau and u (the single-step batch kernel), against per-instance oracle runs."""
    from paper_2410_13165_amd import Batch
    rng = np.random.default_rng(60 + d)
    lo, hi = {1: (20, 70), 3: (5, 12), 4: (3, 7)}[d]
    specs = []
    for _ in range(5):
        dims = tuple(int(rng.integers(lo, hi)) for _ in range(d))
        specs.append({"dims": dims, "tau": float(rng.uniform(0.5, 1.2)),
                      "u": rng.uniform(-0.3, 0.3, size=d).tolist(), "dx": 1.0 / dims[0],
                      "K": 3})
    parts, phi0 = _concat_phi0(specs, 700 + d)
    steps = 12
    with Batch(d, specs, precision=precision) as b:
        b.set_initial(phi0)
        b.step(steps)
        for i, sp in enumerate(specs):
            prob = oracle_problem(d, sp["dims"], sp["dx"], None, u=sp["u"], tau=sp["tau"], K=3)
            run = O.Run(prob, phi0=to_oracle_order(parts[i].reshape(tuple(reversed(sp["dims"])))))
            run.step(steps)
            got = to_oracle_order(b.instance(i).phi().cpu().numpy())
            assert rel_l2(got, run.phi()) <= tol, (i, sp)


def test_tuner_restores_state_and_configs_agree():
    """Every block shape gives bitwise identical states; tuning leaves the
    state where it was."""
    from paper_2410_13165_amd import Batch
    rng = np.random.default_rng(44)
    specs = _specs(rng, 9, [32, 64, 100], (0.5, 1.2), (-0.4, 0.4))
    parts, phi0 = _concat_phi0(specs, 700)
    with Batch(2, specs, precision="fp32") as a, Batch(2, specs, precision="fp32") as b:
        a.set_initial(phi0)
        b.set_initial(phi0)
        a.step(3)
        b.step(3)
        before = [b.instance(i).phi().clone() for i in range(len(specs))]
        cfg = b.tune(5)
        print("[batch] tuned", cfg, flush=True)
        for i in range(len(specs)):
            assert torch.equal(before[i], b.instance(i).phi())
        assert b.instance(0).info()["step"] == 3
        a.step(40)
        b.step(40)
        for i in range(len(specs)):
            assert torch.equal(a.instance(i).phi(), b.instance(i).phi()), i


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_two_step_passes_equal_single_steps(precision):
    """d = 2 batches advance two steps per pass (one launch over a table of
    (instance, x_1 tile, row chunk)); the populations are bitwise those of the
    single-step batch, odd step counts included."""
    from paper_2410_13165_amd import Batch
    rng = np.random.default_rng(45)
    specs = _specs(rng, 11, [16, 64, 300, 520], (0.5, 1.6), (-0.4, 0.4))
    single = [dict(sp, steps_per_pass=1) for sp in specs]
    parts, phi0 = _concat_phi0(specs, 800)
    dt = torch.float64 if precision == "fp64" else torch.float32
    with Batch(2, specs, precision=precision) as a, Batch(2, single, precision=precision) as b:
        a.set_initial(phi0)
        b.set_initial(phi0)
        for n in (2, 7, 16):
            a.step(n)
            b.step(n)
            for i in range(len(specs)):
                ia, ib = a.instance(i).info(), b.instance(i).info()
                assert ia["steps_per_pass"] == 2 and ib["steps_per_pass"] == 1
                sa = a.instance(i).get_state().view(dt).reshape(ia["q"], ia["pstride"])
                sb = b.instance(i).get_state().view(dt).reshape(ib["q"], ib["pstride"])
                assert torch.equal(sa[:, : ia["nodes"]], sb[:, : ib["nodes"]]), (n, i)


def test_batch_rejects_stepping_an_instance():
    from paper_2410_13165_amd import Batch, LbmError
    specs = [{"dims": (16, 16), "tau": 0.5, "u": [0.1, 0.1], "dx": 1 / 16}]
    with Batch(2, specs, precision="fp64") as b:
        b.set_initial(torch.zeros(256, dtype=torch.float64))
        with pytest.raises(LbmError, match="batch"):
            b.instance(0).step(1)


def _rho(u, s, m=24):
    xs = np.linspace(0, 2 * np.pi, m, endpoint=False)
    return max(np.max(np.abs(np.linalg.eigvals(O.amplification_matrix(u, xi, s=s))))
               for xi in itertools.product(xs, repeat=len(u)))


def test_stability_sweep_matches_spectral_radius():
    """Instances with rho(G) > 1 (brute force over the wave numbers, any s) grow,
    the others do not; at s = 2 the region is the entropy region min omega > 0."""
    from paper_2410_13165_amd import Batch
    rng = np.random.default_rng(4)
    specs = _specs(rng, 24, [32], (0.5, 2.0), (-0.75, 0.75))
    # make a third of them s = 2 so that the entropy criterion applies
    for sp in specs[:8]:
        sp["tau"] = 0.5
    parts, phi0 = _concat_phi0(specs, 900)
    steps = 400
    with Batch(2, specs, precision="fp64") as b:
        b.set_initial(phi0)
        m0 = b.moments()
        b.step(steps)
        m1 = b.moments()
        infos = [b.instance(i).info() for i in range(len(specs))]
    growth = np.sqrt(m1[:, 1] / m0[:, 1])
    for i, sp in enumerate(specs):
        rho = _rho(sp["u"], 1.0 / sp["tau"])
        print(f"[sweep] u={np.round(sp['u'], 3)} tau={sp['tau']:.3f} rho={rho:.6f} "
              f"min_omega={infos[i]['min_omega']:.4f} growth={growth[i]:.3e}", flush=True)
        if rho > 1.02:
            assert growth[i] > 2.0, (i, rho, growth[i])
        elif rho < 1 + 1e-9:
            assert growth[i] < 1.2, (i, rho, growth[i])
        if sp["tau"] == 0.5 and abs(infos[i]["min_omega"]) > 1e-2:
            assert (infos[i]["min_omega"] > 0) == (rho < 1 + 1e-9), (i, rho)


def test_sweep_workload_full_size():
    """The stability-sweep workload at full size (512 D2Q9 instances of
    64^2..512^2, tau and u per instance, N(0, 1e-3) noise), in the benchmark's
    launch form (tuned block shape, two steps per pass, then one single step):
    after 5 steps one instance of each grid size against its own oracle run."""
    from paper_2410_13165_amd import Batch
    specs = inputs.sweep_specs()
    phi0 = inputs.sweep_phi0(specs)
    offs = np.concatenate([[0], np.cumsum([int(np.prod(sp["dims"])) for sp in specs])])
    picks = {}
    for i, sp in enumerate(specs):
        picks.setdefault(sp["dims"][0], i)
    steps = 5
    with Batch(2, specs, precision="fp32") as b:
        b.set_initial(torch.from_numpy(phi0))
        b.tune(2)
        b.step(steps)
        for n, i in sorted(picks.items()):
            sp = specs[i]
            print(f"[sweep] instance {i} dims={sp['dims']} tau={sp['tau']:.3f}", flush=True)
            prob = oracle_problem(2, sp["dims"], sp["dx"], None, u=sp["u"], tau=sp["tau"],
                                  K=sp["K"])
            part = phi0[offs[i]:offs[i + 1]].reshape(tuple(reversed(sp["dims"])))
            run = O.Run(prob, phi0=to_oracle_order(part)).step(steps)
            got = to_oracle_order(b.instance(i).phi().cpu().numpy())
            assert rel_l2(got, run.phi()) <= 2e-5, (i, sp)


@pytest.mark.skip(reason="the ordered-queue persistent form it drives stalled on MI355X twice "
                         "and is switched off (lbm_batch_set_launch no longer offers it)")
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("ychunk", [8, 64])
def test_persistent_launch_equals_per_pair_launches(precision, ychunk):
    """Every pair of steps of a call in one persistent launch (blocks claim
    (pair, tile) items from an ordered queue and wait on per-instance
    completion counters): bitwise the states of one launch per pair, odd
    step counts included, over instances of very different sizes."""
    from paper_2410_13165_amd import Batch
    rng = np.random.default_rng(46)
    specs = _specs(rng, 13, [16, 64, 300, 520], (0.5, 1.6), (-0.4, 0.4))
    parts, phi0 = _concat_phi0(specs, 850)
    with Batch(2, specs, precision=precision) as a, Batch(2, specs, precision=precision) as b:
        a.set_initial(phi0)
        b.set_initial(phi0)
        b.set_launch("persistent", ychunk)
        print(f"[persist] {precision} ychunk={ychunk}", flush=True)
        for n in (2, 7, 40):
            a.step(n)
            b.step(n)
            for i in range(len(specs)):
                assert torch.equal(a.instance(i).phi(), b.instance(i).phi()), (n, i)
            assert b.instance(0).info()["step"] == a.instance(0).info()["step"]


@pytest.mark.skip(reason="the ordered-queue persistent form it drives stalled on MI355X twice "
                         "and is switched off (lbm_batch_set_launch no longer offers it)")
def test_sweep_workload_persistent_full_size():
    """The full stability-sweep workload (512 instances, fp32) in one persistent
    launch per call: bitwise the per-pair launches after 10 steps, and one
    instance of each size against its oracle run."""
    from paper_2410_13165_amd import Batch
    specs = inputs.sweep_specs()
    phi0 = torch.from_numpy(inputs.sweep_phi0(specs))
    steps = 10
    picks = {}
    for i, sp in enumerate(specs):
        picks.setdefault(sp["dims"][0], i)
    with Batch(2, specs, precision="fp32") as a, Batch(2, specs, precision="fp32") as b:
        a.set_initial(phi0)
        b.set_initial(phi0)
        b.set_launch("persistent")
        a.step(steps)
        b.step(steps)
        for i in range(len(specs)):
            assert torch.equal(a.instance(i).phi(), b.instance(i).phi()), i
        offs = np.concatenate([[0], np.cumsum([int(np.prod(sp["dims"])) for sp in specs])])
        for n, i in sorted(picks.items()):
            sp = specs[i]
            prob = oracle_problem(2, sp["dims"], sp["dx"], None, u=sp["u"], tau=sp["tau"],
                                  K=sp["K"])
            part = phi0.numpy()[offs[i]:offs[i + 1]].reshape(tuple(reversed(sp["dims"])))
            run = O.Run(prob, phi0=to_oracle_order(part)).step(steps)
            got = to_oracle_order(b.instance(i).phi().cpu().numpy())
            assert rel_l2(got, run.phi()) <= 2e-5, (i, sp)


def test_tuner_covers_launch_forms_and_caches(tmp_path, monkeypatch):
    """The tuner times the launches the steps use (launch form and rows per
    tile of the two-step passes), reports the one it keeps, and serves the same
    batch shape from its cache afterwards (in memory, and appended to the file
    named by LBM_TUNE_CACHE)."""
    from paper_2410_13165_amd import Batch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LBM_TUNE_CACHE", str(cache))
    rng = np.random.default_rng(47)
    specs = _specs(rng, 6, [48, 96], (0.6, 1.2), (-0.3, 0.3))
    specs[0]["dims"] = (77, 51)  # a shape no other test tunes
    parts, phi0 = _concat_phi0(specs, 870)
    with Batch(2, specs, precision="fp32") as b:
        b.set_initial(phi0)
        cfg = b.tune(4)
        print("[batch] tuned", cfg, flush=True)
        assert cfg["form"] in ("per_pair", "resident") and 8 <= cfg["ychunk"] <= 64
        assert not cfg["cached"]
        again = b.tune(4)
        assert again["cached"] and again["form"] == cfg["form"] and again["ychunk"] == cfg["ychunk"]
    lines = cache.read_text().split()
    assert len(lines) == 6 and int(lines[2]) == cfg["ychunk"]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("ychunk", [8, 64])
def test_resident_launch_equals_per_pair_launches(precision, ychunk):
    """Every pair of steps of a call in one launch with one block per instance
    (the block walks its instance's tiles pair after pair; no block waits for
    another): bitwise the states of one launch per pair, odd step counts
    included, over instances of very different sizes."""
    from paper_2410_13165_amd import Batch
    rng = np.random.default_rng(48)
    specs = _specs(rng, 13, [16, 64, 300, 520], (0.5, 1.6), (-0.4, 0.4))
    parts, phi0 = _concat_phi0(specs, 880)
    with Batch(2, specs, precision=precision) as a, Batch(2, specs, precision=precision) as b:
        a.set_initial(phi0)
        b.set_initial(phi0)
        b.set_launch("resident", ychunk)
        print(f"[resident] {precision} ychunk={ychunk}", flush=True)
        for n in (2, 7, 40):
            a.step(n)
            b.step(n)
            for i in range(len(specs)):
                assert torch.equal(a.instance(i).phi(), b.instance(i).phi()), (n, i)
            assert b.instance(0).info()["step"] == a.instance(0).info()["step"]


def test_sweep_workload_resident_full_size():
    """The full stability-sweep workload (512 instances, fp32) advanced by one
    resident launch per call: bitwise the per-pair launches after 10 steps,
    and one instance of each size against its oracle run."""
    from paper_2410_13165_amd import Batch
    specs = inputs.sweep_specs()
    phi0 = torch.from_numpy(inputs.sweep_phi0(specs))
    steps = 10
    picks = {}
    for i, sp in enumerate(specs):
        picks.setdefault(sp["dims"][0], i)
    with Batch(2, specs, precision="fp32") as a, Batch(2, specs, precision="fp32") as b:
        a.set_initial(phi0)
        b.set_initial(phi0)
        b.set_launch("resident")
        a.step(steps)
        b.step(steps)
        for i in range(len(specs)):
            assert torch.equal(a.instance(i).phi(), b.instance(i).phi()), i
        offs = np.concatenate([[0], np.cumsum([int(np.prod(sp["dims"])) for sp in specs])])
        for n, i in sorted(picks.items()):
            sp = specs[i]
            prob = oracle_problem(2, sp["dims"], sp["dx"], None, u=sp["u"], tau=sp["tau"],
                                  K=sp["K"])
            part = phi0.numpy()[offs[i]:offs[i + 1]].reshape(tuple(reversed(sp["dims"])))
            run = O.Run(prob, phi0=to_oracle_order(part)).step(steps)
            got = to_oracle_order(b.instance(i).phi().cpu().numpy())
            assert rel_l2(got, run.phi()) <= 2e-5, (i, sp)


def test_tuner_times_launch_forms_restores_state_and_caches(tmp_path, monkeypatch):
    """lbm_batch_tune times the launches the steps use (per-pair or resident
    form, rows per tile, single-step block shape), leaves the states where they
    were, keeps a configuration that gives the same states as the default one,
    and serves the same batch shape from its cache afterwards (in memory, and
    appended to the file named by LBM_TUNE_CACHE)."""
    from paper_2410_13165_amd import Batch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LBM_TUNE_CACHE", str(cache))
    rng = np.random.default_rng(49)
    specs = _specs(rng, 7, [48, 96], (0.6, 1.2), (-0.3, 0.3))
    specs[0]["dims"] = (77, 51)  # a shape no other test tunes
    parts, phi0 = _concat_phi0(specs, 890)
    with Batch(2, specs, precision="fp32") as a, Batch(2, specs, precision="fp32") as b:
        a.set_initial(phi0)
        b.set_initial(phi0)
        a.step(3)
        b.step(3)
        before = [b.instance(i).phi().clone() for i in range(len(specs))]
        cfg = b.tune(4)
        print("[batch] tuned", cfg, flush=True)
        assert cfg["form"] in ("per_pair", "resident") and 8 <= cfg["ychunk"] <= 64
        assert not cfg["cached"]
        for i in range(len(specs)):
            assert torch.equal(before[i], b.instance(i).phi())
        assert b.instance(0).info()["step"] == 3
        a.step(41)
        b.step(41)
        for i in range(len(specs)):
            assert torch.equal(a.instance(i).phi(), b.instance(i).phi()), i
        again = b.tune(4)
        assert again["cached"] and again["form"] == cfg["form"] and again["ychunk"] == cfg["ychunk"]
    fields = cache.read_text().split()
    assert len(fields) == 6 and int(fields[2]) == cfg["ychunk"]


_TUNE_CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_2410_13165_amd import Batch, inputs
specs = [{"dims": (83, 45), "tau": 0.8, "u": [0.1, -0.2], "dx": 1.0 / 83},
         {"dims": (40, 61), "tau": 1.1, "u": [-0.3, 0.05], "dx": 1.0 / 40}]
phi0 = torch.from_numpy(np.concatenate(
    [inputs.noise(tuple(reversed(sp["dims"])), 900 + i, std=1e-3).ravel()
     for i, sp in enumerate(specs)]))
with Batch(2, specs, precision="fp32") as b:
    b.set_initial(phi0)
    cfg = b.tune(2)
    b.step(5)
    print(json.dumps(cfg), flush=True)
"""


def test_tuner_ignores_invalid_cache_entries(tmp_path):
    """An entry of the LBM_TUNE_CACHE file that names no launch the tuner could
    have chosen (zero rows per tile, an unknown launch form, a block shape the
    kernels were not built for) is not used: the batch is tuned again.  Each
    run is a child process, since the file is read once per process."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, LBM_TUNE_CACHE=str(cache))

    def child():
        print("[tune-cache] child run", flush=True)
        r = subprocess.run([sys.executable, "-c", _TUNE_CHILD, root], env=env,
                           capture_output=True, text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    first = child()
    assert not first["cached"]
    line = cache.read_text().split("\n")[0].split()
    assert len(line) == 6
    # same key hash, values no launch accepts
    cache.write_text(f"{line[0]} 7 0 64 0 0.5\nnot a line\n")
    second = child()
    assert not second["cached"]
    assert second["form"] in ("per_pair", "resident") and 8 <= second["ychunk"] <= 64
    # the re-tuned entry is appended and served to the next process
    third = child()
    assert third["cached"] and third["ychunk"] == second["ychunk"]
