"""Pins of the oracle's lattice, equilibrium and collision against exact
identities of the D3Q19 model (Sec. 2.1) and closed forms."""
from fractions import Fraction

import numpy as np
import pytest


def test_lattice_moments_exact(oracle_lib):
    """Weights and velocities: sum w = 1, sum w c = 0, sum w c c = I/3 and
    the fourth-order isotropy sum w c_i c_j c_k c_l = (d_ij d_kl + d_ik d_jl
    + d_il d_jk) / 9, in exact rationals (weights 1/3, 1/18, 1/36)."""
    c, w, opp = oracle_lib.lattice()
    fw = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12
    for a in range(19):
        assert w[a] == float(fw[a])
    assert sum(fw) == 1
    for i in range(3):
        assert sum(fw[a] * int(c[a, i]) for a in range(19)) == 0
        for j in range(3):
            s2 = sum(fw[a] * int(c[a, i]) * int(c[a, j]) for a in range(19))
            assert s2 == (Fraction(1, 3) if i == j else 0)
            for k in range(3):
                s3 = sum(fw[a] * int(c[a, i]) * int(c[a, j]) * int(c[a, k]) for a in range(19))
                assert s3 == 0
                for l in range(3):
                    s4 = sum(fw[a] * int(c[a, i] * c[a, j] * c[a, k] * c[a, l]) for a in range(19))
                    d = lambda p, q: 1 if p == q else 0
                    assert s4 == Fraction(d(i, j) * d(k, l) + d(i, k) * d(j, l) + d(i, l) * d(j, k), 9)


def test_lattice_velocity_set_and_opposites(oracle_lib):
    c, w, opp = oracle_lib.lattice()
    vecs = {tuple(int(v) for v in c[a]) for a in range(19)}
    want = {(0, 0, 0)} | {tuple(v) for v in np.eye(3, dtype=int)} | {tuple(-v) for v in np.eye(3, dtype=int)}
    for i in range(3):
        for j in range(i + 1, 3):
            for si in (1, -1):
                for sj in (1, -1):
                    v = [0, 0, 0]
                    v[i], v[j] = si, sj
                    want.add(tuple(v))
    assert vecs == want and len(vecs) == 19
    for a in range(19):
        assert opp[opp[a]] == a
        assert np.all(c[opp[a]] == -c[a])
    # ordering of the boundary: +x, -x, +y, -y, +z, -z, then edge pairs
    assert c[1].tolist() == [1, 0, 0] and c[2].tolist() == [-1, 0, 0]
    assert c[5].tolist() == [0, 0, 1] and c[7].tolist() == [1, 1, 0]
    assert c[17].tolist() == [0, 1, -1] and c[18].tolist() == [0, -1, 1]


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(oracle_lib, seed):
    """Sec. 2.1: the moments of f_eq are rho, rho u and, for the
    second-order equilibrium, rho (u u + I/3)."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.1, 0.1, 3)
    f = oracle_lib.feq(rho, u)
    c, w, _ = oracle_lib.lattice()
    assert abs(f.sum() - rho) <= 1e-15 * rho
    assert np.allclose(c.T @ f, rho * u, rtol=0, atol=1e-16)
    P = (c.T * f) @ c
    assert np.allclose(P, rho * (np.outer(u, u) + np.eye(3) / 3.0), rtol=0, atol=2e-16)
    assert np.allclose(oracle_lib.feq(rho, np.zeros(3)), rho * w, rtol=0, atol=1e-17)


def _params(**kw):
    d = dict(nx=1, ny=1, nz=1, periodic=(1, 1, 1), tau=0.6, sigma=0.0, g=(0.0, 0.0, 0.0),
             collision=0)
    d.update(kw)
    return d


@pytest.mark.parametrize("collision", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_collision_conserves_mass_and_momentum(oracle_lib, collision, seed):
    rng = np.random.default_rng(100 + seed)
    fin = oracle_lib.feq(1.0, rng.uniform(-0.05, 0.05, 3)) * rng.uniform(0.9, 1.1, 19)
    c, w, _ = oracle_lib.lattice()
    fout, rho, u = oracle_lib.collide(_params(collision=collision, tau=0.57), fin)
    assert abs(fout.sum() - fin.sum()) < 2e-15
    assert np.allclose(c.T @ fout, c.T @ fin, rtol=0, atol=2e-15)
    assert rho == pytest.approx(fin.sum(), rel=1e-15)
    # the fixed point: an equilibrium stays unchanged
    fe = oracle_lib.feq(1.03, np.array([0.02, -0.01, 0.03]))
    fo, _, _ = oracle_lib.collide(_params(collision=collision), fe)
    assert np.allclose(fo, fe, rtol=0, atol=2e-16)


def test_collision_relaxes_shear_stress(oracle_lib):
    """BGK relaxes the non-equilibrium second moment by (1 - omega); TRT
    relaxes even moments with omega+ = 1/tau, so it agrees on stress."""
    rng = np.random.default_rng(7)
    fin = oracle_lib.feq(1.0, np.array([0.03, 0.0, -0.02])) * rng.uniform(0.95, 1.05, 19)
    c, w, _ = oracle_lib.lattice()
    for coll in (0, 1):
        tau = 0.8
        fout, rho, u = oracle_lib.collide(_params(collision=coll, tau=tau), fin)
        fe = oracle_lib.feq(rho, u)
        Pin = (c.T * (fin - fe)) @ c
        Pout = (c.T * (fout - fe)) @ c
        assert np.allclose(Pout, (1 - 1 / tau) * Pin, rtol=0, atol=1e-15)


def test_trt_equals_bgk_when_rates_match(oracle_lib):
    """With Lambda = (tau - 1/2)^2 the odd rate equals the even rate and TRT
    is BGK."""
    rng = np.random.default_rng(9)
    fin = oracle_lib.feq(1.0, np.array([0.01, 0.02, 0.0])) * rng.uniform(0.9, 1.1, 19)
    tau = 0.7
    g = (1e-4, -2e-4, 3e-5)
    a, _, _ = oracle_lib.collide(_params(collision=0, tau=tau, g=g), fin)
    b, _, _ = oracle_lib.collide(_params(collision=1, tau=tau, g=g, trt_lambda=(tau - 0.5) ** 2), fin)
    assert np.allclose(a, b, rtol=0, atol=1e-15)


def test_guo_force_momentum(oracle_lib):
    """Guo forcing: the collision velocity is (sum c f + rho g/2) / rho and
    the post-collision momentum is rho u + rho g / 2 (half the force before,
    half after), so that u is recovered from post-collision PDFs as
    sum c f* / rho - g / 2."""
    rng = np.random.default_rng(11)
    fin = oracle_lib.feq(1.02, np.array([0.01, -0.03, 0.02])) * rng.uniform(0.97, 1.03, 19)
    c, w, _ = oracle_lib.lattice()
    g = np.array([2e-4, -1e-4, 5e-5])
    for coll in (0, 1):
        fout, rho, u = oracle_lib.collide(_params(collision=coll, tau=0.65, g=tuple(g)), fin)
        assert np.allclose(u, (c.T @ fin + 0.5 * rho * g) / rho, rtol=0, atol=1e-16)
        assert np.allclose(c.T @ fout, rho * u + 0.5 * rho * g, rtol=0, atol=2e-15)
        assert fout.sum() == pytest.approx(rho, rel=1e-15)


@pytest.mark.parametrize("collision", [0, 1])
@pytest.mark.parametrize("seed", range(3))
def test_boundary_velocity_is_the_collision_velocity(oracle_lib, collision, seed):
    """The gas-side equilibrium of an interface cell uses the velocity at
    the boundary (Sec. 2.2), read as the cell's own last collision
    velocity.  It is recovered from the post-collision PDFs, which under the
    Guo scheme carry rho u + rho g / 2 of momentum: the recovered velocity
    must equal the velocity the collision itself used, to round-off.  A
    recovery without the -g/2 shift is off by g/2 (here >= 5e-5)."""
    rng = np.random.default_rng(300 + seed)
    fin = oracle_lib.feq(rng.uniform(0.97, 1.03), rng.uniform(-0.05, 0.05, 3))
    fin = fin * rng.uniform(0.95, 1.05, 19)
    g = tuple(rng.uniform(-2e-3, 2e-3, 3) + np.sign(rng.uniform(-1, 1, 3)) * 1e-4)
    params = _params(collision=collision, tau=float(rng.uniform(0.55, 1.2)), g=g)
    fout, rho, u = oracle_lib.collide(params, fin)
    ub = oracle_lib.boundary_velocity(params, fout)
    assert np.max(np.abs(ub - u)) <= 1e-15
    # the shift matters at this size
    assert np.min(np.abs(np.asarray(g))) / 2 > 4e-5
