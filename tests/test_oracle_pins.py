"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them compares the oracle with
itself: they use printed values (tests/golden), closed forms printed elsewhere
in the paper, exact discrete solutions, brute force on tiny grids, invariants
and measured convergence orders.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import lbm_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- lattice ---

def _read_velocity_golden():
    cols = {}
    with open(os.path.join(GOLDEN, "velocity_sets.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            cols.setdefault(parts[0], {})[int(parts[1])] = [int(v) for v in parts[2:]]
    return cols


@pytest.mark.parametrize("name,d", [("D1Q3", 1), ("D2Q9", 2), ("D3Q19", 3)])
def test_velocity_set_matches_printed_columns(name, d):
    """Sec. 2.3, eqs. (d1q3), (d2q9), (d3q19): the printed velocity columns."""
    cols = _read_velocity_golden()[name]
    c = O.velocity_set(d)
    for axis in range(1, d + 1):
        assert list(c[:, axis - 1]) == cols[axis]


def _ddqq_columns(d):
    """Eq. (ddqq) assembled block by block from Q_p, J_1^p, J_2 and O_p."""
    J1 = [1, -1, -1, 1]
    J2 = [1, 1, -1, -1]

    def Q(p):
        v = [0] * (2 * d + 1)
        v[p] = 1
        v[d + p] = -1
        return v

    cols = []
    for k in range(1, d + 1):
        v = Q(k)
        # blocks for the pairs (l, m), l < m, lexicographic; axis k is J2 when it
        # is the higher index of the pair and J1 when it is the lower one
        for l in range(1, d + 1):
            for m in range(l + 1, d + 1):
                if k == l:
                    v += J1
                elif k == m:
                    v += J2
                else:
                    v += [0, 0, 0, 0]
        cols.append(v)
    eta = [2 * d * (d - 1) - 2 * i * (2 * d - 1 - i) for i in range(1, d + 1)]
    # eta_i counts the trailing zeros of column i (pairs with both indices > i)
    for i, col in enumerate(cols, start=1):
        tail = 0
        for val in reversed(col):
            if val != 0:
                break
            tail += 1
        if i < d:
            assert tail == eta[i - 1]
    return np.array(cols).T


@pytest.mark.parametrize("d", [4, 5])
def test_velocity_set_general_rule(d):
    """Eq. (ddqq): the block construction for d > 3, including eta_i."""
    assert np.array_equal(O.velocity_set(d), _ddqq_columns(d))


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_moment_matrix_invertible_and_opposites(d):
    c = O.velocity_set(d)
    M = O.moment_matrix(c)
    assert np.linalg.matrix_rank(M) == 2 * d * d + 1
    kb = O.opposite(c)
    assert np.array_equal(c[kb], -c)
    assert np.array_equal(kb[kb], np.arange(len(kb)))


# ------------------------------------------------------------------ omega ---

def _omega_closed_form(u, m4):
    """Eq. (omega_k-2), c = 1, with one m4 for every pair (Remark 5)."""
    u = np.asarray(u, float)
    d = len(u)
    c = O.velocity_set(d)
    w = np.empty(len(c))
    npairs = d * (d - 1) // 2
    w[0] = (3 - d - 2 * np.sum(u * u) + 3 * npairs * m4) / 3
    for i in range(d):
        w[1 + i] = ((4 - d) * u[i] + 1 + 2 * u[i] ** 2 - 3 * (d - 1) * m4) / 6
        w[1 + d + i] = (-(4 - d) * u[i] + 1 + 2 * u[i] ** 2 - 3 * (d - 1) * m4) / 6
    for k in range(2 * d + 1, len(c)):
        i, j = np.nonzero(c[k])[0]
        si, sj = c[k, i], c[k, j]
        w[k] = (3 * m4 + 2 * si * sj * u[i] * u[j] + si * u[i] + sj * u[j]) / 12
    return w


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_omega_solve_equals_printed_closed_form(d):
    """omega = M^{-1} eps (Sec. 2.3) against the closed form eq. (omega_k-2)."""
    rng = np.random.default_rng(10 + d)
    for _ in range(20):
        u = rng.uniform(-0.6, 0.6, d)
        m4 = rng.uniform(-0.2, 0.3)
        np.testing.assert_allclose(O.omega(u, m4=m4), _omega_closed_form(u, m4),
                                   rtol=0, atol=1e-14)


def test_omega_d1_printed():
    """Remark 4, d = 1: omega = ((2-2s^2)/3, s/2+(2s^2+1)/6, -s/2+(2s^2+1)/6)."""
    for s in np.linspace(-0.7, 0.7, 15):
        w = O.omega([s])
        ref = [(2 - 2 * s * s) / 3, s / 2 + (2 * s * s + 1) / 6, -s / 2 + (2 * s * s + 1) / 6]
        np.testing.assert_allclose(w, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_omega_reproduces_moment_conditions(d):
    """Eqs. (0-1-meq) and (third-condition-2): moments of omega summed directly
    over the velocities (no use of M or of the row order of eps)."""
    rng = np.random.default_rng(30 + d)
    c = O.velocity_set(d).astype(float)
    for _ in range(5):
        u = rng.uniform(-0.45, 0.45, d)
        w = O.omega(u)
        mom = lambda *powers: float(np.sum(w * np.prod(c ** np.array(powers), axis=1)))
        e = lambda i: tuple(1 if a == i else 0 for a in range(d))
        assert abs(np.sum(w) - 1) < 1e-14
        for i in range(d):
            p1 = np.array(e(i))
            assert abs(mom(*p1) - u[i]) < 1e-14                          # phi u_i
            assert abs(mom(*(2 * p1)) - (1 + 2 * u[i] ** 2) / 3) < 1e-14  # m2_ii
            assert abs(mom(*(3 * p1)) - u[i]) < 1e-14                     # m3_iii = c u_i
            for j in range(d):
                if j == i:
                    continue
                pj = np.array(e(j))
                assert abs(mom(*(p1 + pj)) - 2 * u[i] * u[j] / 3) < 1e-14  # m2_ij
                assert abs(mom(*(2 * p1 + pj)) - u[j] / 3) < 1e-14         # m3_iij
                for l in range(d):
                    if l in (i, j):
                        continue
                    pl = np.array(e(l))
                    assert abs(mom(*(p1 + pj + pl))) < 1e-14              # m3_ijl = 0
        if d >= 2:
            m4 = O.m4_interpolated(u)
            for i in range(d):
                for j in range(i + 1, d):
                    p = np.array(e(i)) * 2 + np.array(e(j)) * 2
                    assert abs(mom(*p) - m4) < 1e-14


def test_m4_two_dimensional_interval():
    """Remark 4 (d = 2): for |s_i| < 1/2 the printed interval for m4 is non-empty
    and eq. (meq-4rd) with g = 1/2 is its midpoint."""
    for s1, s2 in itertools.product(np.linspace(-0.45, 0.45, 7), repeat=2):
        lo = max((-1 + 2 * (s1 ** 2 + s2 ** 2)) / 3, (-2 * s1 * s2 + abs(s1 + s2)) / 3,
                 (2 * s1 * s2 + abs(s1 - s2)) / 3)
        hi = min((-abs(2 * s1) + 1 + 2 * s1 ** 2) / 3, (-abs(2 * s2) + 1 + 2 * s2 ** 2) / 3)
        assert lo < hi
        assert abs(O.m4_interpolated([s1, s2]) - 0.5 * (lo + hi)) < 1e-15


def test_entropy_region_one_and_two_dimensions():
    """Remark 4: omega > 0 iff |sigma_i| < 1/2 in 1D and 2D (g = 1/2)."""
    for s in np.linspace(-0.9, 0.9, 37):
        if abs(abs(s) - 0.5) < 1e-9:
            continue
        assert (O.min_omega([s]) > 0) == (abs(s) < 0.5)
    grid = np.linspace(-0.8, 0.8, 33)
    for s1, s2 in itertools.product(grid, repeat=2):
        if min(abs(abs(s1) - 0.5), abs(abs(s2) - 0.5)) < 1e-9:
            continue
        assert (O.min_omega([s1, s2]) > 0) == (abs(s1) < 0.5 and abs(s2) < 0.5)


@pytest.mark.parametrize("d", [3, 4, 5])
def test_entropy_region_higher_dimensions(d):
    """Remark 5, eq. (region-d>=3): with one m4 from eq. (meq-4rd), omega > 0
    exactly when max{...} < min{...}."""
    rng = np.random.default_rng(50 + d)
    for _ in range(300):
        s = rng.uniform(-0.6, 0.6, d)
        lower = [(-6 + 2 * d + 4 * np.sum(s * s)) / (3 * d * (d - 1))]
        for i in range(d):
            for j in range(i + 1, d):
                lower += [(abs(s[i] + s[j]) - 2 * s[i] * s[j]) / 3,
                          (abs(s[i] - s[j]) + 2 * s[i] * s[j]) / 3]
        upper = min((1 + 2 * s[i] ** 2 - abs((4 - d) * s[i])) / (3 * (d - 1)) for i in range(d))
        gap = upper - max(lower)
        if abs(gap) < 1e-9:
            continue
        assert (O.min_omega(s) > 0) == (gap > 0)


def test_example3_entropy_signs():
    """Example 3: entropy stability fails for u = 0.4*(1,1,1,1) and holds for 0.2,
    0.1, 0.05; also the other velocities used there."""
    assert O.min_omega([0.4] * 4) < 0
    for u in (0.2, 0.1, 0.05):
        assert O.min_omega([u] * 4) > 0
    assert O.min_omega([0.05, 0.2, 0.08, 0.1]) > 0
    assert O.min_omega([1e-3] * 4) > 0


# ------------------------------------------------------- collision, G(xi) ---

@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_collision_involution(d):
    """Eq. (G-3): at s = 2 and xi = 0, G^2 = I; in population space
    C = 2 omega 1^T - I squares to I and preserves sum_k f_k^2 / omega_k."""
    u = np.linspace(0.05, 0.3, d)
    G0 = O.amplification_matrix(u, np.zeros(d), s=2.0)
    np.testing.assert_allclose(G0 @ G0, np.eye(len(G0)), atol=1e-13)
    w = O.omega(u)
    C = 2 * np.outer(w, np.ones(len(w))) - np.eye(len(w))
    np.testing.assert_allclose(C @ C, np.eye(len(w)), atol=1e-14)
    W = np.diag(1 / w)
    np.testing.assert_allclose(C.T @ W @ C, W, rtol=1e-13, atol=1e-12)


def test_appendix_d_eigenvalues():
    """Appendix D: at sigma = -1/2 the eigenvalues of G(xi) are -e^{i xi},
    e^{-i xi/2}, -e^{-i xi/2} (imaginary unit restored; the conjugate set is the
    same statement for -xi)."""
    for xi in (0.3, 1.1, 2.5):
        ev = np.sort_complex(np.linalg.eigvals(O.amplification_matrix([-0.5], [xi])))
        want = np.sort_complex(np.array([-np.exp(1j * xi), np.exp(-0.5j * xi),
                                         -np.exp(-0.5j * xi)]))
        want_c = np.sort_complex(np.conj(want))
        ok = np.allclose(ev, want, atol=1e-12) or np.allclose(ev, want_c, atol=1e-12)
        assert ok, (ev, want)


def _population_G(u, xi, s):
    """Population-space version of eq. (G), obtained from the moment form."""
    d = len(u)
    M = O.moment_matrix(O.velocity_set(d))
    return np.linalg.inv(M) @ O.amplification_matrix(u, xi, s=s) @ M


@pytest.mark.parametrize("d,dims,s", [(1, (7,), 2.0), (2, (5, 4), 2.0), (2, (5, 4), 1.3),
                                      (3, (3, 4, 3), 2.0)])
def test_fourier_mode_is_exact(d, dims, s):
    """Eq. (G): a single Fourier mode evolves as G(xi)^n applied to its
    population vector, for any relaxation s."""
    rng = np.random.default_rng(7)
    u = rng.uniform(-0.3, 0.3, d)
    m = [rng.integers(0, n) for n in dims]
    xi = np.array([2 * np.pi * mj / n for mj, n in zip(m, dims)])
    prob = O.Problem(d, dims, 1.0, u, tau=1.0 / s)
    q = prob.q
    v = rng.normal(size=q) + 1j * rng.normal(size=q)
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in dims], indexing="ij"), -1)
    wave = np.exp(1j * (idx @ xi))
    f0 = v.reshape((q,) + (1,) * d) * wave
    run = O.Run(prob, f0=f0).step(6)
    Gp = _population_G(u, xi, s)
    want = np.linalg.matrix_power(Gp, 6) @ v
    np.testing.assert_allclose(run.f, want.reshape((q,) + (1,) * d) * wave, atol=1e-12)


@pytest.mark.parametrize("d,dims", [(1, (8,)), (2, (5, 5))])
def test_step_matrix_spectrum_brute_force(d, dims):
    """Sec. 4.2: the spectrum of the real-space step matrix on a periodic grid
    is the union over the grid wave numbers of the spectra of G(xi)."""
    u = [0.3] if d == 1 else [0.1, 0.35]
    prob = O.Problem(d, dims, 1.0, u)
    n = prob.q * int(np.prod(dims))
    A = np.empty((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        r = O.Run(prob, f0=e.reshape((prob.q,) + tuple(dims))).step(1)
        A[:, col] = r.f.ravel()
    ev = np.linalg.eigvals(A)
    ref = []
    for m in itertools.product(*[range(nn) for nn in dims]):
        xi = [2 * np.pi * mj / nn for mj, nn in zip(m, dims)]
        ref.extend(np.linalg.eigvals(O.amplification_matrix(u, xi)))
    ref = np.array(ref)
    # each eigenvalue of A has a partner in the union and vice versa
    for lam in ev:
        assert np.min(np.abs(ref - lam)) < 1e-8
    for lam in ref:
        assert np.min(np.abs(ev - lam)) < 1e-8
    # and the (weakly) stable case has spectral radius 1
    assert abs(np.max(np.abs(ev)) - 1) < 1e-9


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_fourth_order_consistency_of_amplification(d):
    """Eq. (fourth-me-2): the physical eigenvalue of G(h xi) matches the exact
    shift e^{-i sigma . h xi} up to O(h^5) per step (error slope 5)."""
    rng = np.random.default_rng(60 + d)
    u = rng.uniform(-0.2, 0.2, d)
    xhat = rng.normal(size=d)
    xhat /= np.linalg.norm(xhat)
    errs = []
    hs = [0.2, 0.1, 0.05]
    for h in hs:
        ev = np.linalg.eigvals(O.amplification_matrix(u, h * xhat))
        exact = np.exp(-1j * h * float(u @ xhat))
        errs.append(np.min(np.abs(ev - exact)))
    slopes = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(2)]
    assert all(4.8 < sl < 5.2 for sl in slopes), slopes


def test_unstable_parameters_have_growing_modes():
    """Sec. 4.2: the L2 and entropy regions coincide (omega_k != 0).  Points with
    a negative weight have rho(G) > 1; points inside have rho(G) = 1."""
    xis = np.linspace(0, 2 * np.pi, 41)
    def rho(u):
        return max(np.max(np.abs(np.linalg.eigvals(O.amplification_matrix(u, xi))))
                   for xi in itertools.product(xis, repeat=len(u)))
    assert abs(rho([0.45, 0.45]) - 1) < 1e-9
    assert rho([0.55, 0.1]) > 1.05
    assert abs(rho([0.49]) - 1) < 1e-9
    assert rho([0.55]) > 1.05


def test_spectral_radius_grid_pins():
    """The grid maximum of rho(G): xi = 0 alone gives the eigenvalues 1 and
    1 - s (eq. G-3 at s = 2); at s = 1 the collision is the rank-one projection
    omega 1^T, so rho(G(xi)) = |sum_k omega_k exp(-i c_k . xi)|; in 1D the
    region is |sigma| <= 1/2 (Sec. 4.2 and Appendix D)."""
    for s in (0.5, 1.0, 1.7, 2.0):
        assert abs(O.spectral_radius_grid([0.2, -0.1], s, 1) - max(1.0, abs(1 - s))) < 1e-12
    rng = np.random.default_rng(12)
    for d in (1, 2, 3):
        u = rng.uniform(-0.4, 0.4, d)
        c = O.velocity_set(d)
        w = O.omega(u)
        m = 6
        want = max(abs(np.sum(w * np.exp(-2j * np.pi * (c @ np.array(j)) / m)))
                   for j in itertools.product(range(m), repeat=d))
        assert abs(O.spectral_radius_grid(u, 1.0, m) - want) < 1e-12
    assert abs(O.spectral_radius_grid([0.5], 2.0, 64) - 1) < 1e-9
    assert abs(O.spectral_radius_grid([-0.3], 2.0, 64) - 1) < 1e-12
    assert O.spectral_radius_grid([0.52], 2.0, 64) > 1.01


# ------------------------------------------------------------------- jets ---

def _fd_derivative(fn, h, order):
    """Central finite differences of fn(eps) at eps = 0 (order 1..3, O(h^4))."""
    if order == 0:
        return fn(0.0)
    if order == 1:
        st, co = [-2, -1, 1, 2], [1 / 12, -8 / 12, 8 / 12, -1 / 12]
    elif order == 2:
        st, co = [-2, -1, 0, 1, 2], [-1 / 12, 16 / 12, -30 / 12, 16 / 12, -1 / 12]
    else:
        st, co = [-3, -2, -1, 1, 2, 3], [1 / 8, -1, 13 / 8, -13 / 8, 1, -1 / 8]
    return sum(cf * fn(s * h) for s, cf in zip(st, co)) / h ** order


@pytest.mark.parametrize("kind", ["cos_sum", "exp_sum"])
def test_jets_against_finite_differences(kind):
    """The directional/time jets used by the wall schemes against finite
    differences of the exact solution phi*(x - u t) + R t."""
    rng = np.random.default_rng(3)
    u = np.array([0.1, -0.2, 0.15])
    fld = O.ExactField(kind, u=u, R=0.7, amps=rng.normal(size=3),
                       kvecs=rng.uniform(-2, 2, (3, 3)), phases=rng.uniform(0, 6, 3))
    x = np.array([[0.3, -0.1, 0.2]])
    t = 0.4
    v = np.array([1.0, -1.0, 0.0])
    for a in range(4):
        for b in range(4 - a):
            got = fld.jet(x, t, a, b, v)[0]
            # mixed derivative: d_t^a of [(v.grad)^b phi*]
            inner = lambda tt: _fd_derivative(lambda e: fld.value(x + e * v, tt)[0], 1e-2, b)
            ref = _fd_derivative(lambda e: inner(t + e), 1e-2, a)
            assert abs(got - ref) < 2e-4 * max(1.0, abs(ref)), (a, b, got, ref)


# ------------------------------------------------- Remark-1 wall data ------

@pytest.mark.parametrize("kind", ["cos_sum", "exp_sum"])
@pytest.mark.parametrize("d", [2, 3])
def test_remark1_jets_equal_exact_jets(kind, d):
    """Remark 1 (with the 1/u_j restored): on a wall of axis j the time and
    tangential derivatives of the data alone reproduce every mixed jet
    d_t^a (c_k . grad)^b phi* with a + b <= 3, including the R term."""
    rng = np.random.default_rng(80 + d)
    u = rng.uniform(0.05, 0.3, d) * rng.choice([-1, 1], d)
    fld = O.ExactField(kind, u=u, R=0.9, amps=rng.normal(size=3),
                       kvecs=rng.uniform(-2, 2, (3, d)), phases=rng.uniform(0, 6, 3))
    prob = O.Problem(d, (4,) * d, 0.1, u, R=0.9, bc=[("fullway", "fullway")] * d,
                     field=fld, wall_data="tangential")
    run = O.Run(prob)
    t = 0.31
    for j in range(d):
        xb = rng.uniform(-1, 1, (5, d))
        xb[:, j] = 0.0
        axes = np.full(5, j)
        for k in range(prob.q):
            ck = prob.c[k].astype(float)
            for a in range(4):
                for b in range(4 - a):
                    got = run.wall_jet(xb, t, a, b, ck, axes)
                    ref = fld.jet(xb, t, a, b, ck)
                    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), \
                        (j, k, a, b)


@pytest.mark.parametrize("scheme", ["fullway", "halfway"])
def test_remark1_run_equals_jets_run(scheme):
    """Whole runs with the two kinds of wall data agree to rounding."""
    u = np.array([0.12, -0.07, 0.05])
    rng = np.random.default_rng(5)
    fld = O.ExactField("cos_sum", u=u, R=0.4, amps=rng.normal(size=2),
                       kvecs=rng.uniform(-3, 3, (2, 3)), phases=rng.uniform(0, 6, 2))
    out = []
    for wd in ("jets", "tangential"):
        prob = O.Problem(3, (6, 5, 5), 0.1, u, R=0.4, bc=[(scheme, scheme)] * 3, field=fld,
                         wall_data=wd)
        out.append(O.Run(prob).step(4).phi())
    assert np.max(np.abs(out[0] - out[1])) <= 1e-13 * np.max(np.abs(out[0]))


def test_remark1_needs_nonzero_normal_velocity():
    fld = O.ExactField("cos_sum", u=[0.1, 0.0], amps=[1.0], kvecs=[[1.0, 2.0]])
    prob = O.Problem(2, (5, 5), 0.1, [0.1, 0.0], bc=[("periodic", "periodic"),
                                                     ("fullway", "fullway")],
                     field=fld, wall_data="tangential")
    with pytest.raises(ValueError, match="u_j"):
        O.Run(prob).step(1)


# --------------------------------------------------------- wall schemes -----

def _exp_prob(u, scheme, P, R=0.3, dx=0.05):
    fld = O.ExactField("exp_sum", u=u, R=R, amps=[1.3], kvecs=[[0.7, -0.4]])
    return O.Problem(2, (6, 6), dx, u, R=R, bc=[(scheme, scheme)] * 2, P=P, field=fld)


@pytest.mark.parametrize("scheme,P,slope", [("fullway", 4, 5.0), ("halfway", 4, 4.0)])
def test_wall_schemes_match_exact_series(scheme, P, slope):
    """Full-way eq. (bun-1) is the third-order truncation of the bulk-consistent
    population (1 - tanh(D/2)) f^eq + dt R_k / 2 with D = dt (d_t + c_k . grad),
    the value that satisfies f(x + c dt, t + dt) = -f + 2 f^eq exactly for an
    exponential profile; half-way eq. (bun-2) is the third-order truncation of
    e^{a/2} [sech((a+b)/2) f^eq_k + sech((a-b)/2) f^eq_kbar] + dt (R_k + R_kbar)/2.
    The truncation error must fall as dt^4 (dt^5 for the full-way series, whose
    generating function 1 - tanh(D/2) has no D^4 term)."""
    u = np.array([0.15, -0.1])
    kappa = np.array([0.7, -0.4])
    errs = []
    for dx in (0.2, 0.1, 0.05):
        prob = _exp_prob(u, scheme, P, dx=dx)
        run = O.Run(prob)
        x = np.array([[0.2, 0.3]])
        t = 0.37
        k = 5  # diagonal (1, 1)
        ck = prob.c[k]
        kb = prob.kbar[k]
        F = 1.3 * np.exp(((x - u * t) @ kappa)[0])
        a = -prob.dt * float(kappa @ u)
        b = prob.dt * float(kappa @ ck)
        w, wb = prob.omega[k], prob.omega[kb]
        if scheme == "fullway":
            got = run.full_way(k, x, t)[0]
            # on the R t part the formula returns omega_k R t exactly
            exact = (1 - math.tanh((a + b) / 2)) * w * F + w * prob.R * t
        else:
            got = run.half_way(k, x, t)[0]
            sech = lambda z: 1 / math.cosh(z)
            exact = math.exp(a / 2) * (sech((a + b) / 2) * w + sech((a - b) / 2) * wb) * F
            exact += (w + wb) * (prob.R * t + prob.dt * prob.R)
        errs.append(abs(got - exact))
    slopes = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(2)]
    assert all(abs(sl - slope) < 0.3 for sl in slopes), (errs, slopes)


@pytest.mark.parametrize("scheme,P", [("fullway", 1), ("fullway", 3), ("fullway", 4),
                                      ("halfway", 1), ("halfway", 2), ("halfway", 3),
                                      ("halfway", 4)])
def test_uniform_state_is_exact_with_walls(scheme, P):
    """A uniform field phi = phi0 + R t is an exact solution of the scheme and
    of every wall formula (eqs. bun1, bun2).  The first-order half-way formula
    carries no source term, so for it only a constant (R = 0) is exact."""
    u = [0.2, -0.1]
    R = 0.0 if (scheme, P) == ("halfway", 1) else 0.8
    fld = O.ExactField("exp_sum", u=u, R=R, amps=[2.5], kvecs=[[0.0, 0.0]])
    n = 7 if scheme == "fullway" else 6
    prob = O.Problem(2, (n, n + 1), 0.1, u, R=R, bc=[(scheme, scheme)] * 2, P=P, field=fld)
    run = O.Run(prob).step(9)
    np.testing.assert_allclose(run.phi(), 2.5 + R * run.t, rtol=0, atol=1e-13)


# ------------------------------------------------------------- invariants ---

@pytest.mark.parametrize("d,dims,u", [(2, (12, 10), [0.1, 0.2]), (3, (6, 5, 7), [0.05, 0.1, 0.08]),
                                      (4, (4, 5, 4, 3), [0.2, 0.1, 0.1, 0.2])])
def test_total_entropy_conserved_periodic(d, dims, u):
    """Remark 6: with s = 2, R = 0 and periodic walls the total microscopic
    entropy sum_x sum_k f_k^2 / (2 omega_k) is conserved."""
    rng = np.random.default_rng(11)
    prob = O.Problem(d, dims, 0.1, u)
    run = O.Run(prob, phi0=rng.normal(size=dims))
    e0 = run.entropy()
    run.step(25)
    assert abs(run.entropy() / e0 - 1) < 1e-13


def test_entropy_not_conserved_for_other_relaxation():
    """Remark 6: s = 2 is necessary; with s != 2 the entropy decays."""
    rng = np.random.default_rng(12)
    prob = O.Problem(2, (10, 10), 0.1, [0.1, 0.2], tau=0.8)
    run = O.Run(prob, phi0=rng.normal(size=(10, 10)), grad0=np.zeros((10, 10, 2)))
    e0 = run.entropy()
    run.step(10)
    assert run.entropy() < e0 * (1 - 1e-3)


def test_mass_grows_by_source():
    """Eq. (0-1-meq): sum_k R_k = R, so with periodic walls sum_x phi grows by
    N dt R per step."""
    rng = np.random.default_rng(13)
    prob = O.Problem(2, (9, 8), 0.05, [0.1, -0.3], R=2.0, tau=0.7)
    run = O.Run(prob, phi0=rng.normal(size=(9, 8)), grad0=np.zeros((9, 8, 2)))
    m0 = run.mass()
    run.step(7)
    assert abs(run.mass() - (m0 + 72 * 7 * 0.05 * 2.0)) < 1e-11


# ----------------------------------------------------------- convergence ---

def _cr(errs, ratio=2.0):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ratio) for i in range(len(errs) - 1)]


def _periodic_sine(d, N, u, K=3, steps=None, fd=False):
    kv = np.full(d, 2 * np.pi)
    fld = O.ExactField("cos_sum", u=u, amps=[1.0], kvecs=[kv], phases=[-np.pi / 2])
    prob = O.Problem(d, (N,) * d, 1.0 / N, u, K=K, field=fld)
    if fd:
        X = prob.nodes()
        phi0 = fld.value(X, 0.0)
        run = O.Run(prob, phi0=phi0, grad0=O.fd4_gradient(phi0, prob.dx))
    else:
        run = O.Run(prob)
    run.step(steps if steps is not None else N)
    return run.rmse()


@pytest.mark.parametrize("d,Ns,u", [(1, (16, 32, 64, 128), [0.3]),
                                    (2, (16, 32, 64), [0.1, 0.2]),
                                    (3, (8, 16, 32), [0.05, 0.1, 0.08])])
def test_fourth_order_convergence_periodic(d, Ns, u):
    """Eq. (fourth-me-2) with the third-order initialisation (eq. ini-simp):
    the error falls by about 16 per halving of dx at acoustic scaling."""
    errs = [_periodic_sine(d, N, u) for N in Ns]
    cr = _cr(errs)
    assert 3.8 < cr[-1] < 4.3, (errs, cr)


def test_fourth_order_convergence_d4():
    """Example 3 (periodic, D4Q33, u = 0.1*(1,1,1,1)): fourth order."""
    errs = [_periodic_sine(4, N, [0.1] * 4, steps=N // 2) for N in (6, 12)]
    cr = _cr(errs)
    assert 3.6 < cr[0] < 4.6, (errs, cr)


def test_first_order_init_gives_second_order():
    """Eq. (cr-estimation), Example 2: f = f^eq (K = 1) limits the order to 2."""
    errs = [_periodic_sine(2, N, [0.1, 0.2], K=1) for N in (16, 32, 64)]
    cr = _cr(errs)
    assert 1.9 < cr[-1] < 2.1, cr


def test_fd_gradient_initialisation_keeps_fourth_order():
    """Eq. (ini-simp) with fourth-order central differences for grad phi0."""
    errs = [_periodic_sine(2, N, [0.1, 0.2], fd=True) for N in (16, 32, 64)]
    assert 3.8 < _cr(errs)[-1] < 4.3


def _example1(u, inv_dx, scheme, P=4, K=3, T=10.0):
    """Example 1 with the transported solution exp[-(x1-u1 t)-(x2-u2 t)] + R t."""
    fld = O.ExactField("exp_sum", u=u, R=5.0, amps=[1.0], kvecs=[[-1.0, -1.0]])
    N = inv_dx + (1 if scheme == "fullway" else 0)
    prob = O.Problem(2, (N, N), 1.0 / inv_dx, u, R=5.0, bc=[(scheme, scheme)] * 2,
                     P=P, K=K, field=fld)
    run = O.Run(prob).step(int(round(T * inv_dx)))
    return run.rmse()


def _golden_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(line.split())
    return rows


@pytest.mark.parametrize("row", range(5))
def test_table1_fullway_order(row):
    """Table 1, full-way rows: fourth-order convergence for all five u
    (printed CR 3.80-3.88).  Absolute magnitudes are not pinned: under this
    reading they come out 2-6x below the printed ones."""
    r = _golden_table("table1_fullway.txt")[row]
    u = (float(r[0]), float(r[1]))
    printed_cr = float(r[-1])
    errs = [_example1(u, n, "fullway") for n in (10, 20, 40)]
    cr = _cr(errs)
    assert all(np.isfinite(errs))
    assert abs(cr[-1] - printed_cr) < 0.45, (u, errs, cr)
    printed = [float(v) for v in r[2:5]]
    assert all(e < 1.5 * p for e, p in zip(errs, printed))


def test_table1_halfway_pattern():
    """Table 1, half-way rows: no convergence for |u| > 0.01 (the error grows
    under refinement, explosively at u = (0.2, 0.1)); convergence at order
    about 4 for u = (0.01, 0.01)."""
    rows = {(float(r[0]), float(r[1])): r for r in _golden_table("table1_halfway.txt")}
    e = [_example1((0.2, 0.1), n, "halfway") for n in (10, 20, 40)]
    printed = [float(v) for v in rows[(0.2, 0.1)][2:5]]
    assert e[0] < e[1] < e[2] and e[2] > 1e6
    # growth between the two finest levels within two decades of the printed one
    assert abs(math.log10(e[2] / e[1]) - math.log10(printed[2] / printed[1])) < 2
    e = [_example1((0.01, 0.01), n, "halfway") for n in (10, 20, 40)]
    assert 3.6 < _cr(e)[-1] < 4.4
    e = [_example1((0.1, 0.1), n, "halfway") for n in (10, 20, 40)]
    assert e[2] > e[1] > e[0]


@pytest.mark.parametrize("P,K,lo,hi", [(1, 3, 0.9, 1.1), (3, 3, 2.85, 3.15), (4, 1, 1.3, 2.3)])
def test_order_rule(P, K, lo, hi):
    """Eq. (cr-estimation): Z = min(K + 1, P) for the full-way scheme
    (u = (0.1, 0.1), Figs. 5-6).  K = 1 with P = 4 is pre-asymptotic toward 2."""
    errs = [_example1((0.1, 0.1), n, "fullway", P=P, K=K) for n in (10, 20, 40)]
    cr = _cr(errs)
    assert lo < cr[-1] < hi, cr


def test_halfway_third_order_reaches_fourth_at_small_u():
    """Sec. 5, Example 1: at u = (0.01, 0.01) the third-order half-way scheme
    behaves like the fourth-order one."""
    errs = [_example1((0.01, 0.01), n, "halfway", P=3) for n in (10, 20, 40)]
    assert 3.5 < _cr(errs)[-1] < 4.5


def test_fullway_fourth_order_in_three_dimensions():
    """The full-way scheme keeps fourth order in 3D at edges and corners."""
    u = [0.05, 0.1, 0.08]
    rng = np.random.default_rng(3)
    fld = O.ExactField("cos_sum", u=u, R=1.0, amps=rng.normal(size=2),
                       kvecs=2 * np.pi * rng.uniform(-1, 1, (2, 3)),
                       phases=rng.uniform(0, 2 * np.pi, 2))
    errs = []
    for inv in (8, 16, 32):
        prob = O.Problem(3, (inv + 1,) * 3, 1.0 / inv, u, R=1.0,
                         bc=[("fullway", "fullway")] * 3, field=fld)
        errs.append(O.Run(prob).step(inv // 2).rmse())
    assert 3.5 < _cr(errs)[-1] < 4.6, errs


# ------------------------------------------------ Example 2 tanh bubble ----

def _bubble(d, u, Rr=None, W=None, center=None):
    # Example 2: Rr = 1/(5(d-1)), W = (5-d)/75
    Rr = 1.0 / (5.0 * (d - 1)) if Rr is None else Rr
    W = (5.0 - d) / 75.0 if W is None else W
    return O.ExactField("tanh_bubble", u=u, Rr=Rr, W=W, center=center)


@pytest.mark.parametrize("d", [2, 3])
def test_tanh_bubble_value_is_a_logistic_profile(d):
    """Example 2: 1/2 - 1/2 tanh(z) is the logistic 1/(1 + e^{2z}); with
    z = (Rr - r)/(2W) the value is exactly 1/2 on the sphere r = Rr, tends to 0
    at the centre and to 1 far away, depends only on |x - c - u t| (radial,
    transported with u)."""
    rng = np.random.default_rng(20 + d)
    u = rng.uniform(-0.3, 0.3, d)
    c = rng.uniform(-0.2, 0.2, d)
    fld = _bubble(d, u, center=c)
    Rr, W = 1.0 / (5.0 * (d - 1)), (5.0 - d) / 75.0
    X = rng.uniform(-1, 1, (200, d))
    t = 0.37
    r = np.linalg.norm(X - u * t - c, axis=-1)
    np.testing.assert_allclose(fld.value(X, t), 1.0 / (1.0 + np.exp((Rr - r) / W)),
                               rtol=1e-13, atol=1e-15)
    # on the interface sphere, at the centre and far away
    dirs = rng.normal(size=(50, d))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    np.testing.assert_allclose(fld.value(c + u * t + Rr * dirs, t), 0.5, atol=1e-14)
    assert 0.0 < fld.value((c + u * t)[None], t)[0] < math.exp(-Rr / W)
    assert abs(fld.value((c + u * t + 50 * dirs[0])[None], t)[0] - 1.0) < 1e-15
    # radial: a rotation about the centre keeps the value
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    Y = (X - u * t - c) @ Q.T + u * t + c
    np.testing.assert_allclose(fld.value(Y, t), fld.value(X, t), rtol=1e-12, atol=1e-15)
    # transport: phi*(x, t) = phi*(x - u t, 0)
    np.testing.assert_allclose(fld.value(X, t), fld.value(X - u * t, 0.0), rtol=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_tanh_bubble_gradient_against_finite_differences(d):
    """grad phi*(x, 0) of the bubble (used by the K = 3 initialisation)
    against central differences of the value, away from the kink at the
    centre, where the gradient is taken as 0."""
    rng = np.random.default_rng(30 + d)
    c = rng.uniform(-0.1, 0.1, d)
    fld = _bubble(d, np.zeros(d), center=c)
    X = c + rng.uniform(-0.6, 0.6, (100, d))
    X = X[np.linalg.norm(X - c, axis=1) > 0.02]
    h = 1e-5
    g = fld.grad0(X)
    for a in range(d):
        e = np.zeros(d)
        e[a] = h
        fd = (fld.value(X + e, 0.0) - fld.value(X - e, 0.0)) / (2 * h)
        np.testing.assert_allclose(g[:, a], fd, rtol=1e-6, atol=1e-8)
    np.testing.assert_array_equal(fld.grad0(c[None]), np.zeros((1, d)))


@pytest.mark.parametrize("row", [3, 4])
def test_table2_first_order_rows(row):
    """Table 2, K = 1 rows at u = (0.05, 0.05) and (0.005, 0.005): D2Q9 periodic
    on [-1,1]^2 to T = 1 with 100 and 200 nodes across the domain.  The RMSE
    against the transported bubble matches the printed values within 10% and
    falls at second order (printed CR 2.04 and 2.02)."""
    r = _golden_table("table2_tanh_k1.txt")[row]
    u = (float(r[0]), float(r[1]))
    errs = []
    for n in (100, 200):
        dx = 2.0 / n
        prob = O.Problem(2, (n, n), dx, u, origin=[-1.0, -1.0], K=1, field=_bubble(2, u))
        errs.append(O.Run(prob).step(n // 2).rmse())
    printed = [float(v) for v in r[2:4]]
    for e, p in zip(errs, printed):
        assert abs(e / p - 1.0) < 0.10, (u, errs, printed)
    assert 1.8 < math.log2(errs[0] / errs[1]) < 2.3, errs
