"""Plain, slow FP64 CPU oracle for the unified fourth-order BGK lattice Boltzmann
model of the d-dimensional linear hyperbolic equation (Chen, Chai & Shi,
arXiv:2410.13165).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this module: only the test-suite, the package smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP implementation.

Everything is computed in float64 with NumPy, following the paper's order and
notation:

* lattice units c = 1, so dt = dx and sigma = u (Sec. 5 opening paragraph);
* velocity set DdQ(2d^2+1) (Sec. 2.3, eqs. d1q3, d2q9, d3q19, ddqq);
* natural-moment matrix M (same equations) and moment vector epsilon
  (eq. meq, built from eqs. 0-1-meq and third-condition-2);
* the fourth-order moment m4 from the interpolation formula eq. meq-4rd
  (Remark 5) with g = 1/2 by default (Sec. 5);
* EDF weights omega = M^{-1} epsilon (Sec. 2.3), so f^eq = omega*phi and
  R_k = omega_k*R;
* BGK evolution with relaxation s (eq. BGK-LB-Evolution; s = 2 gives
  eq. BGK-LB-Evolution-seq2);
* initialisation of order K = 1 (f = f^eq) or K = 3 (eq. ini-simp);
* Dirichlet walls: full-way schemes eq. bun1 (orders 1, 3, 4) and half-way
  anti-bounce-back schemes eq. bun2 (orders 1..4), used as
  f_k(x_f, t+dt) = -f*_kbar(x_f, t) + [right-hand side of bun2 at (x_b, t)];
* RMSE (eq. rmse), total microscopic entropy sum_x sum_k f_k^2/(2 omega_k)
  (eqs. entropy, skfk) and the amplification matrix G(xi) (eq. G).

Readings taken where the paper is silent or garbled (each listed in the
design notes):

* tau = 1/s is kept as a parameter; the K = 3 initialisation uses tau*dt in
  place of dt/2, which is what the first-order Taylor step of the general
  evolution gives and equals eq. ini-simp at s = 2.
* The half-way scheme subtracts the post-collision population f*_kbar at x_f
  (eq. collision), as the appendix derivation sums eqs. fi-2 and fi-star-2.
* The shift matrix carries the imaginary unit, T = diag(exp(-i c_k . xi)).
* Exact solutions are the transported profiles phi*(x,t) = F(x - u t) + R t,
  so every time derivative of a jet is -u.grad on F plus R on the R t term.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field as dc_field
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "velocity_set", "opposite", "moment_matrix", "m4_interpolated", "epsilon",
    "omega", "min_omega", "ExactField", "Problem", "Run", "amplification_matrix",
    "spectral_radius_grid", "fd4_gradient", "rmse",
]


# ---------------------------------------------------------------------------
# Lattice: Sec. 2.3, eqs. (d1q3), (d2q9), (d3q19), (ddqq)
# ---------------------------------------------------------------------------

def velocity_set(d: int) -> np.ndarray:
    """The DdQ(2d^2+1) velocities in the paper's order, shape (q, d), c = 1.

    Order: the rest velocity; +e_1..+e_d; -e_1..-e_d; then, for every pair
    i < j taken in lexicographic order, four diagonal velocities whose
    (c_i, c_j) components are J1 = (1,-1,-1,1) for the lower index and
    J2 = (1,1,-1,-1) for the higher index (eq. ddqq with Q_p, J_1, J_2, O_p).
    """
    if d < 1:
        raise ValueError("d must be >= 1")
    vel = [np.zeros(d, dtype=np.int64)]
    for sign in (1, -1):
        for i in range(d):
            e = np.zeros(d, dtype=np.int64)
            e[i] = sign
            vel.append(e)
    J1 = (1, -1, -1, 1)
    J2 = (1, 1, -1, -1)
    for i in range(d):
        for j in range(i + 1, d):
            for m in range(4):
                e = np.zeros(d, dtype=np.int64)
                e[i] = J1[m]
                e[j] = J2[m]
                vel.append(e)
    c = np.array(vel, dtype=np.int64)
    assert c.shape == (2 * d * d + 1, d)
    return c


def opposite(c: np.ndarray) -> np.ndarray:
    """kbar with c_kbar = -c_k (Sec. 3.2, half-way scheme)."""
    q = c.shape[0]
    kbar = np.empty(q, dtype=np.int64)
    for k in range(q):
        hits = [m for m in range(q) if np.array_equal(c[m], -c[k])]
        assert len(hits) == 1
        kbar[k] = hits[0]
    return kbar


def _pairs(d: int):
    return [(i, j) for i in range(d) for j in range(i + 1, d)]


def _ordered_pairs(d: int):
    # (i, j), i != j, ordered by i then j: the x_i^2 x_j rows of M
    return [(i, j) for i in range(d) for j in range(d) if j != i]


def moment_matrix(c: np.ndarray) -> np.ndarray:
    """Natural-moment matrix M (Sec. 2.3).

    Rows: 1; c_i; c_i^2; c_i c_j (i<j); c_i^2 c_j (i != j, by i then j);
    c_i^2 c_j^2 (i<j).  That is 1 + d + d + d(d-1)/2 + d(d-1) + d(d-1)/2
    = 2d^2 + 1 rows.
    """
    c = np.asarray(c, dtype=np.float64)
    q, d = c.shape
    rows = [np.ones(q)]
    rows += [c[:, i] for i in range(d)]
    rows += [c[:, i] ** 2 for i in range(d)]
    rows += [c[:, i] * c[:, j] for (i, j) in _pairs(d)]
    rows += [c[:, i] ** 2 * c[:, j] for (i, j) in _ordered_pairs(d)]
    rows += [c[:, i] ** 2 * c[:, j] ** 2 for (i, j) in _pairs(d)]
    M = np.array(rows)
    assert M.shape == (q, q)
    return M


# ---------------------------------------------------------------------------
# Moments of the equilibrium: eqs. (meq), (meq-4rd)
# ---------------------------------------------------------------------------

def m4_interpolated(u: Sequence[float], g: float = 0.5) -> float:
    """Common fourth-order moment m4 of all pairs, eq. (meq-4rd), c = 1.

    m4 = g * max{ (|s_i + s_j| - 2 s_i s_j)/3, (|s_i - s_j| + 2 s_i s_j)/3 over
                  pairs i<j;  (-6 + 2d + 4 sum s^2) / (3 d (d-1)) }
       + (1 - g) * min_i { (1 + 2 s_i^2 - |(4 - d) s_i|) / (3 (d-1)) }.
    Undefined for d = 1 (there is no fourth-order moment).
    """
    s = np.asarray(u, dtype=np.float64)
    d = s.size
    if d < 2:
        raise ValueError("m4 exists only for d >= 2")
    lower = [(-6.0 + 2 * d + 4.0 * float(np.sum(s * s))) / (3.0 * d * (d - 1))]
    for (i, j) in _pairs(d):
        lower.append((abs(s[i] + s[j]) - 2.0 * s[i] * s[j]) / 3.0)
        lower.append((abs(s[i] - s[j]) + 2.0 * s[i] * s[j]) / 3.0)
    upper = [(1.0 + 2.0 * s[i] ** 2 - abs((4 - d) * s[i])) / (3.0 * (d - 1))
             for i in range(d)]
    return g * max(lower) + (1.0 - g) * min(upper)


def epsilon(u: Sequence[float], m4: Optional[float]) -> np.ndarray:
    """Moment vector epsilon of eq. (meq), c = 1, row order of moment_matrix.

    [1; u_i; (1 + 2u_i^2)/3; 2 u_i u_j / 3 (i<j); u_j / 3 for x_i^2 x_j;
     m4 for x_i^2 x_j^2 (i<j)].
    """
    u = np.asarray(u, dtype=np.float64)
    d = u.size
    e = [1.0]
    e += [u[i] for i in range(d)]
    e += [(1.0 + 2.0 * u[i] ** 2) / 3.0 for i in range(d)]
    e += [2.0 * u[i] * u[j] / 3.0 for (i, j) in _pairs(d)]
    e += [u[j] / 3.0 for (i, j) in _ordered_pairs(d)]
    if d >= 2:
        e += [m4 for _ in _pairs(d)]
    return np.array(e, dtype=np.float64)


def omega(u: Sequence[float], g: float = 0.5, m4: Optional[float] = None) -> np.ndarray:
    """EDF weights omega = M^{-1} epsilon (Sec. 2.3), so f^eq_k = omega_k phi."""
    u = np.asarray(u, dtype=np.float64)
    d = u.size
    if d >= 2 and m4 is None:
        m4 = m4_interpolated(u, g)
    c = velocity_set(d)
    return np.linalg.solve(moment_matrix(c), epsilon(u, m4))


def min_omega(u: Sequence[float], g: float = 0.5, m4: Optional[float] = None) -> float:
    """Smallest EDF weight; entropy stability means all omega_k > 0 (Sec. 4.1)."""
    return float(np.min(omega(u, g, m4)))


# ---------------------------------------------------------------------------
# Exact solutions phi*(x,t) = F(x - u t) + R t and their jets
# ---------------------------------------------------------------------------

@dataclass
class ExactField:
    """Analytic solution family of eq. (HE) with constant u and R.

    kind = "cos_sum":  F(y) = sum_j a_j cos(kappa_j . y + theta_j)
    kind = "exp_sum":  F(y) = sum_j a_j exp(kappa_j . y)
    kind = "tanh_bubble": F(y) = 1/2 - 1/2 tanh((Rr - |y - center|)/(2W))
                          (Example 2; values and the initial gradient only)
    """
    kind: str
    u: np.ndarray
    R: float = 0.0
    amps: np.ndarray = dc_field(default_factory=lambda: np.zeros(0))
    kvecs: np.ndarray = dc_field(default_factory=lambda: np.zeros((0, 1)))
    phases: np.ndarray = dc_field(default_factory=lambda: np.zeros(0))
    Rr: float = 0.0
    W: float = 1.0
    center: Optional[np.ndarray] = None

    def __post_init__(self):
        self.u = np.asarray(self.u, dtype=np.float64)
        self.amps = np.asarray(self.amps, dtype=np.float64)
        self.kvecs = np.asarray(self.kvecs, dtype=np.float64).reshape(len(self.amps), -1) \
            if len(self.amps) else np.zeros((0, self.u.size))
        self.phases = np.asarray(self.phases, dtype=np.float64) if len(self.phases) \
            else np.zeros(len(self.amps))
        if self.center is None:
            self.center = np.zeros(self.u.size)
        self.center = np.asarray(self.center, dtype=np.float64)

    # value of phi* at points X (shape (..., d)) and time t
    def value(self, X: np.ndarray, t: float) -> np.ndarray:
        return self.jet(X, t, 0, 0, None)

    def jet(self, X: np.ndarray, t: float, a: int, b: int,
            v: Optional[np.ndarray]) -> np.ndarray:
        """d_t^a (v . grad)^b phi*(X, t).

        On F(x - u t) a time derivative is the directional derivative along
        -u; on the R t term only d_t^0 and d_t^1 survive (and only for b = 0).
        """
        X = np.asarray(X, dtype=np.float64)
        Y = X - self.u * t
        out = np.zeros(X.shape[:-1])
        if self.kind == "cos_sum":
            for aj, kj, thj in zip(self.amps, self.kvecs, self.phases):
                ph = Y @ kj + thj
                w = -float(kj @ self.u)
                p = float(kj @ v) if b else 1.0
                m = (a + b) % 4
                # derivatives of cos: cos, -sin, -cos, sin
                base = (np.cos(ph), -np.sin(ph), -np.cos(ph), np.sin(ph))[m]
                out = out + aj * (w ** a) * (p ** b) * base
        elif self.kind == "exp_sum":
            for aj, kj in zip(self.amps, self.kvecs):
                w = -float(kj @ self.u)
                p = float(kj @ v) if b else 1.0
                out = out + aj * (w ** a) * (p ** b) * np.exp(Y @ kj)
        elif self.kind == "tanh_bubble":
            if a or b:
                raise NotImplementedError("tanh bubble supplies values and grad0 only")
            r = np.sqrt(np.sum((Y - self.center) ** 2, axis=-1))
            out = 0.5 - 0.5 * np.tanh((self.Rr - r) / (2.0 * self.W))
        else:
            raise ValueError(self.kind)
        if a == 0 and b == 0:
            out = out + self.R * t
        elif a == 1 and b == 0:
            out = out + self.R
        return out

    def grad0(self, X: np.ndarray) -> np.ndarray:
        """grad phi*(X, 0), shape (..., d)."""
        X = np.asarray(X, dtype=np.float64)
        d = X.shape[-1]
        if self.kind == "tanh_bubble":
            Y = X - self.center
            r = np.sqrt(np.sum(Y * Y, axis=-1))
            z = (self.Rr - r) / (2.0 * self.W)
            dphi_dr = 0.5 / np.cosh(z) ** 2 / (2.0 * self.W)
            with np.errstate(invalid="ignore", divide="ignore"):
                unit = np.where(r[..., None] > 0, Y / r[..., None], 0.0)
            return dphi_dr[..., None] * unit
        g = np.zeros(X.shape)
        for i in range(d):
            e = np.zeros(d)
            e[i] = 1.0
            g[..., i] = self.jet(X, 0.0, 0, 1, e)
        return g


# ---------------------------------------------------------------------------
# Problem description and the time loop
# ---------------------------------------------------------------------------

PERIODIC, FULLWAY, HALFWAY, OPEN = "periodic", "fullway", "halfway", "open"


@dataclass
class Problem:
    """One lattice: dims (N_1..N_d), spacing dx, origin a, velocity u, source R.

    bc[j] is a pair (lower face, upper face) for axis j, each one of
    "periodic" (both faces), "fullway", "halfway" or "open".  An "open" face
    just wraps around and is only meant for sub-boxes whose edge values are
    discarded.  Node positions: x = a + i dx on periodic/full-way axes,
    x = a + (i + 1/2) dx on axes with a half-way face (eq. rmse, Fig. 1);
    `shift` overrides that offset (sub-boxes of a half-way lattice).
    """
    d: int
    dims: Sequence[int]
    dx: float
    u: Sequence[float]
    R: float = 0.0
    tau: float = 0.5
    origin: Optional[Sequence[float]] = None
    bc: Optional[Sequence[Sequence[str]]] = None
    P: int = 4          # boundary scheme order
    K: int = 3          # initialisation order
    g: float = 0.5
    m4: Optional[float] = None
    field: Optional[ExactField] = None
    shift: Optional[Sequence[float]] = None  # node offset per axis, in units of dx
    # "jets": the wall schemes take every derivative from the exact solution;
    # "tangential": only the Dirichlet data h on the wall are used (its time
    # and tangential derivatives), normal derivatives follow from the equation
    # (Remark 1, with the division by u_j the printed form omits)
    wall_data: str = "jets"

    def __post_init__(self):
        self.dims = tuple(int(n) for n in self.dims)
        assert len(self.dims) == self.d
        self.u = np.asarray(self.u, dtype=np.float64)
        if self.origin is None:
            self.origin = np.zeros(self.d)
        self.origin = np.asarray(self.origin, dtype=np.float64)
        if self.bc is None:
            self.bc = [(PERIODIC, PERIODIC)] * self.d
        self.bc = [tuple(b) for b in self.bc]
        self.c = velocity_set(self.d)
        self.q = self.c.shape[0]
        self.kbar = opposite(self.c)
        self.omega = omega(self.u, self.g, self.m4)
        self.s = 1.0 / self.tau
        self.dt = self.dx  # c = 1

    def axis_coords(self, j: int) -> np.ndarray:
        n = np.arange(self.dims[j], dtype=np.float64)
        if self.shift is not None:
            shift = float(self.shift[j])
        else:
            shift = 0.5 if HALFWAY in self.bc[j] else 0.0
        return self.origin[j] + (n + shift) * self.dx

    def nodes(self) -> np.ndarray:
        """Node coordinates, shape (N_1, ..., N_d, d)."""
        axes = [self.axis_coords(j) for j in range(self.d)]
        grids = np.meshgrid(*axes, indexing="ij")
        return np.stack(grids, axis=-1)


def fd4_gradient(phi: np.ndarray, dx: float) -> np.ndarray:
    """Fourth-order central differences on a periodic grid, shape (..., d)."""
    d = phi.ndim
    g = np.empty(phi.shape + (d,))
    for j in range(d):
        p1 = np.roll(phi, -1, axis=j)
        m1 = np.roll(phi, 1, axis=j)
        p2 = np.roll(phi, -2, axis=j)
        m2 = np.roll(phi, 2, axis=j)
        g[..., j] = (-p2 + 8.0 * p1 - 8.0 * m1 + m2) / (12.0 * dx)
    return g


def rmse(phi: np.ndarray, phi_exact: np.ndarray) -> float:
    """Eq. (rmse): root mean square over all lattice points."""
    return float(np.sqrt(np.mean((phi - phi_exact) ** 2)))


class Run:
    """Time loop of the model: f holds the pre-collision populations at t_n."""

    def __init__(self, prob: Problem, phi0: Optional[np.ndarray] = None,
                 grad0: Optional[np.ndarray] = None, f0: Optional[np.ndarray] = None):
        self.p = prob
        self.X = prob.nodes()
        self.n = 0
        if f0 is not None:
            self.f = np.array(f0, dtype=np.result_type(f0, np.float64))
        else:
            self.f = self._initial(phi0, grad0)
        self._masks = self._unknown_masks()
        self._axes = self._wall_axes()

    @property
    def t(self) -> float:
        return self.n * self.p.dt

    # -- initialisation, eq. (ini-simp) -------------------------------------
    def _initial(self, phi0, grad0) -> np.ndarray:
        p = self.p
        if phi0 is None:
            phi0 = p.field.value(self.X, 0.0)
        f = np.empty((p.q,) + p.dims)
        if p.K == 1:
            for k in range(p.q):
                f[k] = p.omega[k] * phi0
            return f
        if p.K != 3:
            raise ValueError("initialisation order K must be 1 or 3")
        if grad0 is None:
            if p.field is not None:
                grad0 = p.field.grad0(self.X)
            else:
                if any(b != (PERIODIC, PERIODIC) for b in p.bc):
                    raise ValueError("finite-difference gradient needs periodic axes")
                grad0 = fd4_gradient(phi0, p.dx)
        for k in range(p.q):
            v = p.u - p.c[k]
            # f_k = f_k^eq + tau dt (u - c_k) . grad f_k^eq   (tau = 1/2: eq. ini-simp)
            f[k] = p.omega[k] * (phi0 + p.tau * p.dt * (grad0 @ v))
        return f

    # -- which populations come from outside the domain ---------------------
    def _unknown_masks(self):
        p = self.p
        masks = []
        for k in range(p.q):
            m = np.zeros(p.dims, dtype=bool)
            for j in range(p.d):
                lo, hi = p.bc[j]
                idx = [slice(None)] * p.d
                if p.c[k, j] == 1 and lo in (FULLWAY, HALFWAY):
                    idx[j] = 0
                    m[tuple(idx)] = True
                if p.c[k, j] == -1 and hi in (FULLWAY, HALFWAY):
                    idx[j] = p.dims[j] - 1
                    m[tuple(idx)] = True
            masks.append(m)
        return masks

    def _wall_axes(self):
        """Per population, the lowest axis through which it enters from
        outside at each node (-1 where it is known): the wall whose data
        serve the Remark-1 construction."""
        p = self.p
        axes = []
        for k in range(p.q):
            ax = np.full(p.dims, -1, dtype=np.int64)
            for j in reversed(range(p.d)):
                lo, hi = p.bc[j]
                idx = [slice(None)] * p.d
                if p.c[k, j] == 1 and lo in (FULLWAY, HALFWAY):
                    idx[j] = 0
                    ax[tuple(idx)] = j
                if p.c[k, j] == -1 and hi in (FULLWAY, HALFWAY):
                    idx[j] = p.dims[j] - 1
                    ax[tuple(idx)] = j
            axes.append(ax)
        return axes

    # -- moments ------------------------------------------------------------
    def phi(self) -> np.ndarray:
        return self.f.sum(axis=0)

    def entropy(self) -> float:
        return float(np.sum(self.f ** 2 / (2.0 * self.p.omega.reshape((-1,) + (1,) * self.p.d))))

    def mass(self) -> float:
        return float(np.sum(self.phi()))

    def rmse(self) -> float:
        return rmse(self.phi(), self.p.field.value(self.X, self.t))

    # -- one time step ------------------------------------------------------
    def collide(self) -> np.ndarray:
        """Post-collision populations, eq. (BGK-LB-Evolution) right-hand side."""
        p = self.p
        phi = self.f.sum(axis=0)
        fstar = np.empty_like(self.f)
        for k in range(p.q):
            feq = p.omega[k] * phi
            Rk = p.omega[k] * p.R
            fstar[k] = self.f[k] - p.s * (self.f[k] - feq) + p.dt * Rk
        return fstar

    def step(self, nsteps: int = 1):
        for _ in range(nsteps):
            self._one_step()
        return self

    def _one_step(self):
        p = self.p
        t = self.t
        fstar = self.collide()
        fnew = np.empty_like(fstar)
        for k in range(p.q):
            # f_k(x + c_k dt, t + dt) = f*_k(x, t): roll by +c_k along each axis
            fnew[k] = np.roll(fstar[k], shift=tuple(int(v) for v in p.c[k]),
                              axis=tuple(range(p.d)))
        for k in range(p.q):
            m = self._masks[k]
            if not m.any():
                continue
            Xm = self.X[m]
            ax = self._axes[k][m]
            scheme = self._scheme_of(k)
            if scheme == FULLWAY:
                fnew[k][m] = self.full_way(k, Xm, t + p.dt, ax)
            else:
                xb = Xm - p.c[k] * (p.dx / 2.0)
                fnew[k][m] = -fstar[p.kbar[k]][m] + self.half_way(k, xb, t, ax)
        self.f = fnew
        self.n += 1

    def _scheme_of(self, k: int) -> str:
        kinds = set()
        p = self.p
        for j in range(p.d):
            lo, hi = p.bc[j]
            if p.c[k, j] == 1 and lo in (FULLWAY, HALFWAY):
                kinds.add(lo)
            if p.c[k, j] == -1 and hi in (FULLWAY, HALFWAY):
                kinds.add(hi)
        if len(kinds) != 1:
            raise ValueError("mixed full-way/half-way faces on one population")
        return kinds.pop()

    # -- boundary schemes ---------------------------------------------------
    def wall_jet(self, xb: np.ndarray, t: float, a: int, b: int, ck: np.ndarray,
                 axes: Optional[np.ndarray]) -> np.ndarray:
        """d_t^a (c_k . grad)^b phi* at wall points xb.

        wall_data = "jets": straight from the exact solution.  "tangential"
        (Remark 1): at a point on a wall of axis j only h = phi* restricted to
        the wall is used.  The equation d_t phi + u . grad phi = R gives
        d_j phi = (R - d_t phi - sum_{l != j} u_l d_l phi) / u_j, and on any
        derivative of phi the same relation without R.  Hence
        c_k . grad = A + (c_j / u_j) R [on phi itself] with
        A = alpha . grad_tan + beta d_t, alpha = c_k - (c_j / u_j) u (alpha_j = 0),
        beta = -c_j / u_j, and
        d_t^a (c_k . grad)^b phi = sum_i C(b, i) beta^i d_t^(a+i) (alpha . grad)^(b-i) phi
                                   - [a = 0, b = 1] beta R
        (the last term removes the R that d_t phi carries).  Every term on the
        right is a time or tangential derivative of the wall data.
        """
        p = self.p
        if p.wall_data == "jets" or b == 0:
            return p.field.jet(xb, t, a, b, ck)
        if p.wall_data != "tangential":
            raise ValueError(p.wall_data)
        out = np.zeros(xb.shape[:-1])
        for j in np.unique(axes):
            sel = axes == j
            if p.u[j] == 0.0:
                raise ValueError("Remark-1 wall data need u_j != 0")
            beta = -ck[j] / p.u[j]
            alpha = ck + beta * p.u
            alpha[j] = 0.0
            acc = np.zeros(int(sel.sum()))
            for i in range(b + 1):
                acc = acc + math.comb(b, i) * beta ** i * p.field.jet(xb[sel], t, a + i, b - i,
                                                                       alpha)
            if a == 0 and b == 1:
                acc = acc - beta * p.R
            out[sel] = acc
        return out

    def full_way(self, k: int, xb: np.ndarray, t: float,
                 axes: Optional[np.ndarray] = None) -> np.ndarray:
        """Eq. (bun1): unknown f_k(x_b, t) at a wall node, order P in {1, 3, 4}."""
        p = self.p
        ck = p.c[k].astype(np.float64)
        wk = p.omega[k]
        dt = p.dt
        Rk = wk * p.R

        def J(a, b):  # d_t^a (c_k . grad)^b f_k^eq at (x_b, t)
            return wk * self.wall_jet(xb, t, a, b, ck, axes)

        if p.P == 1:
            return J(0, 0)
        val = J(0, 0) - dt / 2 * J(0, 1) - dt / 2 * J(1, 0)
        if p.P == 3:
            return val + dt / 2 * Rk
        if p.P != 4:
            raise ValueError("full-way order must be 1, 3 or 4")
        val = (val + dt ** 3 / 8 * J(2, 1) + dt ** 3 / 8 * J(1, 2)
               + dt ** 3 / 24 * J(3, 0) + dt ** 3 / 24 * J(0, 3))
        return val + dt / 2 * Rk

    def half_way(self, k: int, xb: np.ndarray, t: float,
                 axes: Optional[np.ndarray] = None) -> np.ndarray:
        """Right-hand side of eq. (bun2) at (x_b, t), order P in {1, 2, 3, 4}.

        All directional derivatives are along c_k; f^eq_k + f^eq_kbar and
        f^eq_k - f^eq_kbar share the exact phi*, so they are (omega_k +/- omega_kbar)
        times the jets of phi*.
        """
        p = self.p
        ck = p.c[k].astype(np.float64)
        kb = p.kbar[k]
        wp = p.omega[k] + p.omega[kb]
        wm = p.omega[k] - p.omega[kb]
        dt = p.dt
        RR = wp * p.R  # R_k + R_kbar

        def S(a, b):
            return wp * self.wall_jet(xb, t, a, b, ck, axes)

        def Dm(a, b):
            return wm * self.wall_jet(xb, t, a, b, ck, axes)

        val = S(0, 0)
        if p.P == 1:
            return val
        val = val + dt / 2 * S(1, 0)
        if p.P == 2:
            return val + dt / 2 * RR
        val = val - dt ** 2 / 8 * S(0, 2) - dt ** 2 / 4 * Dm(1, 1)
        if p.P == 3:
            return val + dt / 2 * RR
        if p.P != 4:
            raise ValueError("half-way order must be 1, 2, 3 or 4")
        val = (val - dt ** 3 / 8 * Dm(2, 1) - dt ** 3 / 16 * S(1, 2)
               - dt ** 3 / 24 * S(3, 0))
        return val + dt / 2 * RR


# ---------------------------------------------------------------------------
# von Neumann analysis: eq. (G)
# ---------------------------------------------------------------------------

def amplification_matrix(u: Sequence[float], xi: Sequence[float], s: float = 2.0,
                         g: float = 0.5, m4: Optional[float] = None) -> np.ndarray:
    """Moment-space amplification matrix G(xi) = M T M^{-1} ((1-s) I + s eps e_1^T).

    At s = 2 this is eq. (G): M T M^{-1} (2 eps (x) e_1 - I), with
    T = diag(exp(-i c_k . xi)) for the pull direction of the streaming.
    """
    u = np.asarray(u, dtype=np.float64)
    d = u.size
    c = velocity_set(d)
    M = moment_matrix(c)
    if d >= 2 and m4 is None:
        m4 = m4_interpolated(u, g)
    eps = epsilon(u, m4)
    q = c.shape[0]
    e1 = np.zeros(q)
    e1[0] = 1.0
    T = np.diag(np.exp(-1j * (c @ np.asarray(xi, dtype=np.float64))))
    coll = (1.0 - s) * np.eye(q) + s * np.outer(eps, e1)
    return M @ T @ np.linalg.inv(M) @ coll


def spectral_radius_grid(u: Sequence[float], s: float, m: int, g: float = 0.5) -> float:
    """max over the grid xi = 2 pi j / m, j in {0..m-1}^d, of the spectral
    radius of G(xi) (Sec. 4.2), by dense eigenvalues of each matrix."""
    u = np.asarray(u, dtype=np.float64)
    best = 0.0
    for j in itertools.product(range(m), repeat=u.size):
        xi = 2.0 * np.pi * np.asarray(j, dtype=np.float64) / m
        G = amplification_matrix(u, xi, s=s, g=g)
        best = max(best, float(np.max(np.abs(np.linalg.eigvals(G)))))
    return best
