"""Pins for the oracle's interior point trajectory (Section 3.1).

GPU parity replays the oracle for the GPU's step count, so the oracle's
iterates after k steps (not only its converged solution) decide every parity
outcome.  These tests pin them:

* hand-derived fixtures (tests/golden/trajectory/*.json, each with its written
  derivation): the initial point, and for the one-variable box QP every
  quantity of the first Newton step (residuals, mu, the affine direction, its
  step to the boundary, mu_aff and sigma);
* an exact rational reference: the same method carried out in Fractions on the
  REDUCED Newton system (slacks and multipliers eliminated by hand, leaving
  [Qs + G^T D G, A^T; A, 0]), solved by exact Gaussian elimination.  It shares
  no formulation with the oracle, which factors the unreduced, unsymmetrised K
  of eq. cvxgen:affine by floating-point LU, and it has no rounding;
* the oracle replaying k = 0, 1, 2, 3 steps must match the exact reference to
  1e-12, and mutated readings of the method (sigma squared, 0.99 applied after
  the cap, no shift of the initial point, a single step length without the
  corrector) must miss it by far more, so the pin discriminates the readings
  it is meant to fix (R2-R4).
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle

HERE = os.path.join(os.path.dirname(__file__), "golden", "trajectory")


def _load(name):
    with open(os.path.join(HERE, name)) as f:
        return json.load(f)


def _frac(x):
    return Fr(x) if isinstance(x, str) else Fr(x).limit_denominator(10 ** 6)


def _exact_solve(M, rhs):
    """Exact Gaussian elimination (Fractions, first non-zero pivot)."""
    N = len(rhs)
    M = [row[:] + [r] for row, r in zip(M, rhs)]
    for k in range(N):
        piv = next(i for i in range(k, N) if M[i][k] != 0)
        M[k], M[piv] = M[piv], M[k]
        for i in range(k + 1, N):
            f = M[i][k] / M[k][k]
            if f:
                for j in range(k, N + 1):
                    M[i][j] -= f * M[k][j]
    x = [Fr(0)] * N
    for i in range(N - 1, -1, -1):
        x[i] = (M[i][N] - sum(M[i][j] * x[j] for j in range(i + 1, N))) / M[i][i]
    return x


class ExactIPM:
    """The method of Section 3.1 in exact arithmetic on the reduced system.

    Newton rows (unknowns dz, ds, dl, dnu), with r2 the complementarity row:
        Qs dz + G^T dl + A^T dnu = r_x,   lambda_i ds_i + s_i dl_i = r2_i,
        G dz + ds = r_s,                  A dz = r_y.
    Eliminating ds = r_s - G dz and dl = c + D G dz (D = lambda/s,
    c = (r2 - lambda o r_s)/s) leaves
        [Qs + G^T D G, A^T; A, 0] [dz; dnu] = [r_x - G^T c; r_y].
    `mut` names a deliberately wrong reading (for the discrimination test)."""

    def __init__(self, d, mut=None):
        self.mut = mut
        self.Q = [[_frac(v) for v in row] for row in d["Q"]]
        self.n = len(self.Q)
        self.q = [_frac(v) for v in d["q"]]
        self.G = [[_frac(v) for v in row] for row in d["G"]]
        self.h = [_frac(v) for v in d["h"]]
        self.A = [[_frac(v) for v in row] for row in d["A"]]
        self.b = [_frac(v) for v in d["b"]]
        self.m, self.p = len(self.G), len(self.A)
        n = self.n
        self.Qs = [[(self.Q[i][j] + self.Q[j][i]) / 2 for j in range(n)] for i in range(n)]

    def _kkt(self, D, rhs_z, rhs_y):
        n, p, G = self.n, self.p, self.G
        M = [[self.Qs[i][j] + sum(G[k][i] * D[k] * G[k][j] for k in range(self.m))
              for j in range(n)] + [self.A[k][i] for k in range(p)] for i in range(n)]
        M += [self.A[k][:] + [Fr(0)] * p for k in range(p)]
        x = _exact_solve(M, list(rhs_z) + list(rhs_y))
        return x[:n], x[n:]

    def _gz(self, z):
        return [sum(self.G[k][j] * z[j] for j in range(self.n)) for k in range(self.m)]

    def _gt(self, v):
        return [sum(self.G[k][i] * v[k] for k in range(self.m)) for i in range(self.n)]

    def init(self):
        """R4: the Newton matrix with (D(lambda), D(s)) replaced by (I, I)."""
        ones = [Fr(1)] * self.m
        gth = self._gt(self.h)
        z, nu = self._kkt(ones, [gth[i] - self.q[i] for i in range(self.n)], self.b)
        gz = self._gz(z)
        s = [self.h[k] - gz[k] for k in range(self.m)]
        lam = [-x for x in s]
        if self.mut != "no_shift":
            ms, ml = min(s), min(lam)
            if ms <= 0:
                s = [x + 1 - ms for x in s]
            if ml <= 0:
                lam = [x + 1 - ml for x in lam]
        return z, s, lam, nu

    def residuals(self, z, s, lam, nu):
        n, m, p = self.n, self.m, self.p
        gtl = self._gt(lam)
        atn = [sum(self.A[k][i] * nu[k] for k in range(p)) for i in range(n)]
        rx = [-(sum(self.Qs[i][j] * z[j] for j in range(n)) + self.q[i] + gtl[i] + atn[i])
              for i in range(n)]
        gz = self._gz(z)
        rs = [-(gz[k] + s[k] - self.h[k]) for k in range(m)]
        ry = [-(sum(self.A[k][j] * z[j] for j in range(n)) - self.b[k]) for k in range(p)]
        mu = sum(s[k] * lam[k] for k in range(m)) / m
        return rx, rs, ry, mu

    def direction(self, s, lam, rx, r2, rs, ry):
        m = self.m
        D = [lam[k] / s[k] for k in range(m)]
        c = [(r2[k] - lam[k] * rs[k]) / s[k] for k in range(m)]
        gtc = self._gt(c)
        dz, dnu = self._kkt(D, [rx[i] - gtc[i] for i in range(self.n)], ry)
        gdz = self._gz(dz)
        ds = [rs[k] - gdz[k] for k in range(m)]
        dl = [c[k] + D[k] * gdz[k] for k in range(m)]
        return dz, ds, dl, dnu

    @staticmethod
    def a_max(v, dv):
        r = [-x / d for x, d in zip(v, dv) if d < 0]
        return min(r) if r else None

    def step(self, z, s, lam, nu):
        """One Newton step; returns the new iterate and the step's quantities."""
        m = self.m
        rx, rs, ry, mu = self.residuals(z, s, lam, nu)
        dza, dsa, dla, dna = self.direction(s, lam, rx, [-s[k] * lam[k] for k in range(m)], rs, ry)
        am = [a for a in (self.a_max(s, dsa), self.a_max(lam, dla)) if a is not None]
        a_max_aff = min(am) if am else None
        a_aff = Fr(1) if a_max_aff is None else min(Fr(1), a_max_aff)
        mu_aff = sum((s[k] + a_aff * dsa[k]) * (lam[k] + a_aff * dla[k]) for k in range(m)) / m
        ratio = mu_aff / mu
        sigma = ratio ** 2 if self.mut == "sigma_squared" else ratio ** 3
        info = dict(r_x=rx, r_s=rs, mu=mu, dz_aff=dza, ds_aff=dsa, dlam_aff=dla,
                    a_max_aff=a_max_aff, alpha_aff=a_aff, mu_aff=mu_aff, sigma=sigma)
        if self.mut == "no_corrector":
            dz, ds, dl, dn = dza, dsa, dla, dna
        else:
            r2 = [sigma * mu - dsa[k] * dla[k] for k in range(m)]
            dzc, dsc, dlc, dnc = self.direction(s, lam, [Fr(0)] * self.n, r2, [Fr(0)] * m,
                                                [Fr(0)] * self.p)
            dz = [a + b for a, b in zip(dza, dzc)]
            ds = [a + b for a, b in zip(dsa, dsc)]
            dl = [a + b for a, b in zip(dla, dlc)]
            dn = [a + b for a, b in zip(dna, dnc)]
        am = [a for a in (self.a_max(s, ds), self.a_max(lam, dl)) if a is not None]
        amax = min(am) if am else None
        if amax is None:
            alpha = Fr(1)
        elif self.mut == "cap_then_099":
            alpha = Fr(99, 100) * min(Fr(1), amax)
        else:
            alpha = min(Fr(1), Fr(99, 100) * amax)
        info["alpha"] = alpha
        upd = lambda v, d: [x + alpha * y for x, y in zip(v, d)]
        return (upd(z, dz), upd(s, ds), upd(lam, dl), upd(nu, dn)), info

    def trajectory(self, steps):
        it = self.init()
        out, infos = [it], []
        for _ in range(steps):
            it, info = self.step(*it)
            out.append(it)
            infos.append(info)
        return out, infos


CASES = ["box_1d_steps.json", "simplex_2d_steps.json"]


def _arrays(d):
    n = len(d["q"])
    A = np.array(d["A"], float).reshape(-1, n) if d["A"] else None
    b = np.array(d["b"], float) if d["b"] else None
    return (np.array(d["Q"], float), np.array(d["q"], float), A, b,
            np.array(d["G"], float).reshape(-1, n), np.array(d["h"], float))


@pytest.mark.parametrize("name", CASES)
def test_hand_derived_initial_point(name):
    """The fixture's hand-derived initial point equals the exact reference's."""
    d = _load(name)
    z, s, lam, nu = ExactIPM(d).init()
    for key, v in (("z", z), ("s", s), ("lam", lam), ("nu", nu)):
        assert [Fr(x) for x in d["init"][key]] == v, key


def test_hand_derived_first_step_box_1d():
    """Every quantity of the hand-derived first Newton step of the one-variable
    box QP equals the exact reference's."""
    d = _load("box_1d_steps.json")
    ipm = ExactIPM(d)
    _, infos = ipm.trajectory(1)
    info = infos[0]
    for key, want in d["step0"].items():
        got = info[key]
        if isinstance(want, list):
            assert [Fr(x) for x in want] == got, key
        else:
            assert Fr(want) == got, key


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_oracle_replay_follows_exact_trajectory(name, k):
    """oracle.solve(replay=k) returns the iterate of the exact reference after k
    Newton steps, to 1e-12."""
    d = _load(name)
    traj, _ = ExactIPM(d).trajectory(k)
    z, s, lam, nu = (np.array([float(x) for x in v]) for v in traj[k])
    r = oracle.solve(*_arrays(d), replay=k)
    assert r["iters"] == k
    for key, want in (("z", z), ("s", s), ("lam", lam), ("nu", nu)):
        got = r[key]
        err = np.abs(got - want).max(initial=0.0) / (1.0 + np.abs(want).max(initial=0.0))
        assert err <= 1e-12, (name, k, key, got, want)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("mut", ["sigma_squared", "cap_then_099", "no_shift", "no_corrector"])
def test_pin_discriminates_misreadings(name, mut):
    """A wrong reading of sigma, of the step rule, of the initial shift or of the
    corrector changes the first iterates by far more than the 1e-12 above: at
    least one of the iterates after 0..3 steps moves by more than 1e-4 (or the
    misreading makes a Newton system singular)."""
    d = _load(name)
    good, _ = ExactIPM(d).trajectory(3)
    try:
        bad, _ = ExactIPM(d, mut=mut).trajectory(3)
    except (StopIteration, ZeroDivisionError):
        return  # the misreading breaks the method outright (a singular Newton system)
    worst = 0.0
    for a, b in zip(good, bad):
        for va, vb in zip(a, b):
            if va:
                worst = max(worst, max(abs(float(x - y)) for x, y in zip(va, vb)))
    assert worst > 1e-4, (name, mut, worst)
