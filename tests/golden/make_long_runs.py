"""Write tests/golden/long_runs.npz: the FP64 oracle's results of the long
parity runs of tests/long_runs.py, sampled on the nodes that
tests/long_runs.sample_nodes picks, plus whole-lattice sums.

Only the oracle computes anything here.  For each run NAME the archive holds
  NAME__idx   (count, d) int64 node indices (i_1, ..., i_d)
  NAME__phi   (count,) float64 phi at those nodes after the run's steps
  NAME__scal  [sum phi, sum phi^2, total entropy sum f^2/(2 omega), RMSE
               against the exact solution (NaN without one), steps]
The D2Q9 sweep instances are named sweep_<index into sweep_specs()>.

Run from the repository root:  python tests/golden/make_long_runs.py [-j N]
(about ten minutes on eight cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import lbm_oracle as O  # noqa: E402
from tests import long_runs as LR  # noqa: E402
from tests.pairs import oracle_problem  # noqa: E402


def _result(name, run, prob, with_rmse, seed):
    phi = run.phi()
    idx = LR.sample_nodes(prob.dims, seed)
    vals = phi[tuple(idx.T)]
    scal = [float(phi.sum()), float((phi * phi).sum()), run.entropy(),
            run.rmse() if with_rmse else float("nan"), float(run.n)]
    return name, idx, vals, np.array(scal)


def cube(name):
    c = LR.cube_problem(name)
    prob = oracle_problem(3, c["dims"], c["dx"], c["spec"], bc=c["bc"])
    t = time.time()
    run = O.Run(prob).step(c["steps"])
    print(f"{name}: {time.time() - t:.0f} s", flush=True)
    return _result(name, run, prob, True, 11)


def grf(name):
    g = LR.grf_problem(name)
    prob = oracle_problem(3, g["dims"], g["dx"], None, u=g["u"])
    t = time.time()
    run = O.Run(prob, phi0=g["phi0"]).step(g["steps"])  # isotropic: any axis order
    print(f"{name}: {time.time() - t:.0f} s", flush=True)
    return _result(name, run, prob, False, 12)


def sweep(args):
    i, sp, phi0 = args
    n1, n2 = sp["dims"]
    prob = oracle_problem(2, sp["dims"], sp["dx"], None, u=sp["u"], tau=sp["tau"], K=sp["K"])
    t = time.time()
    run = O.Run(prob, phi0=phi0.reshape(n2, n1).T).step(4000)
    print(f"sweep_{i} ({n1}^2): {time.time() - t:.0f} s", flush=True)
    return _result(f"sweep_{i}", run, prob, False, 13)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    out = {}
    pick, specs, phis = LR.sweep_subset()
    with ProcessPoolExecutor(args.j) as ex:
        futs = [ex.submit(cube, n) for n in LR.CUBES] + [ex.submit(grf, n) for n in LR.GRF]
        futs += [ex.submit(sweep, a) for a in zip(pick, specs, phis)]
        for f in futs:
            name, idx, vals, scal = f.result()
            out[f"{name}__idx"] = idx
            out[f"{name}__phi"] = vals
            out[f"{name}__scal"] = scal
    meta = {"cubes": LR.CUBES, "grf": LR.GRF, "sweep": pick}
    out["meta"] = np.array(json.dumps(meta))
    np.savez_compressed(os.path.join(HERE, LR.GOLDEN), **out)
    print("wrote", os.path.join(HERE, LR.GOLDEN))


if __name__ == "__main__":
    main()
