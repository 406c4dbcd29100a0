"""Pins of the interface normal weights, the gas inlet of the pore set-up
(Sec. 3.2: gas injected at a constant rate) and walls."""
import numpy as np
import pytest

import scenes
from scenes import GAS, IFACE, INLET, LIQ, WALL

P0 = scenes.P0


def test_youngs_weights_single_bump(oracle_lib):
    """Parker-Youngs gradient: central differences weighted 4 / 2 / 1 for
    face / edge / corner offsets.  With phi = 1 in one cell and 0 elsewhere,
    the normal of a cell at offset d from the bump is the weight of the
    remaining offset pair times the unit step along each axis where |d_i|=1."""
    n = 7
    N = n ** 3
    phi = np.zeros(N)
    c = 3 + n * (3 + n * 3)
    phi[c] = 1.0
    t = np.full(N, IFACE, np.uint8)
    sc = scenes.Scene("bump", n, n, n, (1, 1, 1), 0.6, 0.0, (0, 0, 0), 1e-2, 0.0, t, phi,
                      np.ones(N), np.zeros(3 * N), np.zeros(N, np.int32), [(0, 0, -1.0, P0)])
    o = oracle_lib.Oracle.from_scene(sc)
    _, nrm = o.geometry()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                i = (3 + dx) + n * ((3 + dy) + n * (3 + dz))
                d = (dx, dy, dz)
                want = []
                for k in range(3):
                    if d[k] == 0:
                        want.append(0.0)
                        continue
                    w = 1.0
                    for j in range(3):
                        if j != k:
                            w *= 2.0 if d[j] == 0 else 1.0
                    want.append(-d[k] * w)  # phi grows towards the bump
                assert nrm[:, i].tolist() == want, (d, nrm[:, i])


def _small_orifice(p_scale=1.0, Q=0.05, phi_above=None):
    sc = scenes.orifice(n=(16, 16, 20), r=3.0, g=1e-5, Q=Q)
    sc.bubbles = [(b[0], b[1], b[2], b[3] * p_scale) for b in sc.bubbles]
    if phi_above is not None:
        nx, ny = sc.nx, sc.ny
        z = np.arange(sc.n) // (nx * ny)
        inl = (sc.cell_type == INLET)
        above = np.roll(inl, nx * ny) & (z == 1)
        sc.phi = np.where(above, phi_above, sc.phi)
    return sc


def test_injection_adds_q_per_step(oracle_lib):
    """The bubble owning the inlet cells gains V* = Q per step, and nothing
    else changes V*."""
    sc = _small_orifice()
    o = oracle_lib.Oracle.from_scene(sc)
    b0 = o.bubbles()
    assert b0["flags"].tolist() == [1]
    steps = 25
    o.step(steps)
    b = o.bubbles()
    assert o.scalars()["n_topology"] == 0
    assert b["v_star"][0] == pytest.approx(b0["v_star"][0] + steps * 0.05, rel=1e-14)
    assert b["volume"][0] > b0["volume"][0]


def test_inlet_neighbours_never_fill(oracle_lib):
    """An under-pressured inlet bubble sucks liquid into the orifice; the
    interface cells next to inlet cells must stay interface so that no
    liquid cell ever touches an inlet cell.  Above 1 + eps such a cell is
    capped instead of filled: it keeps m = rho, passes the rest on as excess
    to interface neighbours that are not capped, and ends the step at fill
    level 1."""
    sc = _small_orifice(p_scale=0.8, Q=0.0, phi_above=0.999)
    o = oracle_lib.Oracle.from_scene(sc)
    nx, ny, nz = sc.nx, sc.ny, sc.nz
    m0 = o.scalars()["total_mass"]
    capped = 0
    for s in range(30):
        o.step(1)
        d = o.read()
        t3 = d["cell_type"].reshape(nz, ny, nx)
        ph3 = d["phi"].reshape(nz, ny, nx)
        # the cells right above the inlet
        above = t3[1][t3[0] == INLET]
        capped += int(np.sum(ph3[1][t3[0] == INLET] == 1.0))
        assert np.all(ph3[1][t3[0] == INLET] <= 1.0 + sc.eps)
        assert np.all(above == IFACE)
        inlet = t3 == INLET
        liq = t3 == LIQ
        for dz in (0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if not 1 <= abs(dx) + abs(dy) + abs(dz) <= 2:
                        continue
                    sh = np.zeros_like(inlet)
                    sh[dz:, :, :] = inlet[: nz - dz, :, :]
                    sh = np.roll(np.roll(sh, dy, 1), dx, 2)
                    assert not np.any(liq & sh)
    assert capped > 0  # the rule was exercised
    assert abs(o.scalars()["total_mass"] - m0) <= 1e-13 * m0


def test_walls_conserve_mass_with_interface(oracle_lib):
    sc = scenes.spheres(n=(18, 16, 14), centers=((9.0, 8.0, 7.0),), radii=(4.0,), walls=True,
                        periodic=(0, 0, 0), sigma=5e-3, rho_l=1.0, p_init=(1.1 * P0,), ss=8,
                        g=(0.0, 0.0, -1e-5))
    o = oracle_lib.Oracle.from_scene(sc)
    m0 = o.scalars()["total_mass"]
    o.step(40)
    assert abs(o.scalars()["total_mass"] - m0) < 1e-13 * m0
    d = o.read()
    assert np.all(d["cell_type"][sc.cell_type == WALL] == WALL)
