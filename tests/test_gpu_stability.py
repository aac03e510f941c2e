"""Stability maps on the GPU (lbm_stability_map) against the oracle's dense
eigenvalues of G(xi), and the paper's claim that the L2 and entropy stability
regions coincide away from omega_k = 0 (Sec. 4.2)."""
import itertools

import numpy as np
import pytest

from oracle import lbm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu_map(sigma, s, m, g=0.5):
    from paper_2410_13165_amd import stability_map
    out = stability_map(np.asarray(sigma, dtype=np.float64), s, m=m, g=g)
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("d,count,m", [(1, 40, 64), (2, 24, 12), (3, 8, 6), (4, 3, 4)])
def test_map_matches_oracle_eigenvalues(d, count, m):
    rng = np.random.default_rng(300 + d)
    sigma = rng.uniform(-0.65, 0.65, size=(count, d))
    sigma[: count // 4] *= 0.02  # near the origin (clustered eigenvalues)
    s = rng.choice([2.0, 1.0, 1.0 + 1e-9], size=count)
    s[::3] = rng.uniform(0.2, 2.0, size=len(s[::3]))
    print(f"[stability] d={d} count={count} m={m}", flush=True)
    got = _gpu_map(sigma, s, m)
    assert np.all(got["unconverged"] == 0)
    for i in range(count):
        want = O.spectral_radius_grid(sigma[i], float(s[i]), m)
        assert abs(got["rho"][i] - want) <= 1e-12 * max(1.0, want), (i, sigma[i], s[i])
        assert abs(got["min_omega"][i] - O.min_omega(sigma[i])) <= 1e-14


def test_map_g_weight_and_xi_zero():
    """m = 1 is xi = 0 only: rho = max(1, |1 - s|); the weight g of eq. (meq-4rd)
    changes m4 and with it omega and rho."""
    sig = np.array([[0.3, -0.2], [0.05, 0.1]])
    got = _gpu_map(sig, np.array([2.0, 0.4]), 1)
    np.testing.assert_allclose(got["rho"], [1.0, 1.0], atol=1e-14)
    for gw in (0.0, 0.25, 1.0):
        got = _gpu_map(sig, 2.0, 8, g=gw)
        for i in range(2):
            assert abs(got["min_omega"][i] - O.min_omega(sig[i], g=gw)) <= 1e-14
            want = O.spectral_radius_grid(sig[i], 2.0, 8, g=gw)
            assert abs(got["rho"][i] - want) <= 1e-12


@pytest.mark.parametrize("d,n,m", [(2, 61, 32), (3, 13, 16)])
def test_l2_region_equals_entropy_region(d, n, m):
    """At s = 2: every point with all omega_k > 0 has rho = 1 (Prop. 1 and
    Remark 6: the step preserves a weighted norm), and on this grid every point
    with some omega_k < -1e-3 has a growing mode (the numerical claim of
    Sec. 4.2)."""
    axis = np.linspace(-0.6, 0.6, n)
    sigma = np.array(list(itertools.product(axis, repeat=d)))
    print(f"[stability] region d={d} points={len(sigma)} m={m}", flush=True)
    got = _gpu_map(sigma, 2.0, m)
    assert np.all(got["unconverged"] == 0)
    mw, rho = got["min_omega"], got["rho"]
    inside = mw > 1e-9
    outside = mw < -1e-3
    assert inside.any() and outside.any()
    assert np.all(np.abs(rho[inside] - 1.0) <= 1e-12), np.max(np.abs(rho[inside] - 1))
    assert np.all(rho[outside] > 1.0 + 1e-9), sigma[outside][rho[outside] <= 1 + 1e-9]


def test_rejects_bad_arguments():
    from paper_2410_13165_amd import LbmError, stability_map
    with pytest.raises(LbmError, match="m must be"):
        stability_map(np.zeros((2, 2)), 2.0, m=0)
    with pytest.raises(LbmError, match="m\\^d"):
        stability_map(np.zeros((1, 4)), 2.0, m=1024)
    with pytest.raises(LbmError, match="d must be"):
        stability_map(np.zeros((1, 5)), 2.0, m=4)
