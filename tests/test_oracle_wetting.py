"""Pins of the two pieces of the pore case (Sec. 3.2) in the oracle: the
wetting rule at walls (a static contact angle entering the height-function
curvature through ghost columns) and the open top (an atmosphere bubble
held at p0 that absorbs the bubbles reaching it).

The wetting pin is geometric: a gas cap cut from a sphere of radius R by
the wall plane meets the wall at a known angle, so its curvature is -1/R
everywhere, also in the first fluid layer where the stencil reaches into
the wall.  With the cap's own angle the first layer is close to -1/R; the
mirror (90 degrees) and the supplementary angle (the sign of the
correction flipped) are far off."""
import numpy as np
import pytest

import scenes
from scenes import BUBBLE_ATMOSPHERE, BUBBLE_INLET, GAS, IFACE, INLET, LIQ, WALL

P0 = scenes.P0
R = 7.0


def _cap(theta, n=28, M=16):
    """Gas cap on the low z wall meeting it at theta (measured in the
    liquid): the sphere's centre lies R cos(theta) above the wall plane.
    The free box holds the whole sphere; layers above the plane become the
    fluid layers of the walled box."""
    h = R * np.cos(np.radians(theta))
    free = scenes.spheres(n=(n, n, 2 * M), centers=((n / 2.0, n / 2.0, M + h),), radii=(R,),
                          sigma=1e-3, rho_l=1.0)
    t3 = free.cell_type.reshape(2 * M, n, n)
    p3 = free.phi.reshape(2 * M, n, n)
    b3 = free.bubble_id.reshape(2 * M, n, n)
    nzw = M + 2
    tw = np.full((nzw, n, n), WALL, np.uint8)
    pw = np.zeros((nzw, n, n))
    bw = np.full((nzw, n, n), -1, np.int32)
    tw[1:M + 1], pw[1:M + 1], bw[1:M + 1] = t3[M:], p3[M:], b3[M:]
    N = tw.size
    params = dict(nx=n, ny=n, nz=nzw, periodic=(1, 1, 0), tau=0.6, sigma=1e-3,
                  g=(0.0, 0.0, 0.0), collision=0, eps_convert=1e-2)
    return params, tw.ravel(), pw.ravel(), np.ones(N), np.zeros(3 * N), bw.ravel(), [(0, 0, -1.0, P0)]


def _layer_kappa(oracle_lib, sc, angle):
    params = dict(sc[0], contact_angle=angle)
    o = oracle_lib.Oracle(params, *sc[1:])
    k, _ = o.geometry()
    shape = (params["nz"], params["ny"], params["nx"])
    t, ph, k3 = sc[1].reshape(shape), sc[2].reshape(shape), k.reshape(shape)
    out = []
    for layer in (1, 2, 3):
        sel = (t[layer] == IFACE) & (ph[layer] > 0.05) & (ph[layer] < 0.95)
        assert np.count_nonzero(sel) >= 16
        out.append((float(np.mean(k3[layer][sel]) * R), k3[layer]))
    return out


@pytest.mark.parametrize("theta", [50.0, 60.0, 70.0, 110.0, 120.0, 130.0])
def test_cap_curvature_at_its_contact_angle(oracle_lib, theta):
    sc = _cap(theta)
    own = _layer_kappa(oracle_lib, sc, theta)
    mirror = _layer_kappa(oracle_lib, sc, 90.0)
    flipped = _layer_kappa(oracle_lib, sc, 180.0 - theta)
    # first fluid layer: the cap's own angle gives the sphere's curvature
    assert own[0][0] == pytest.approx(-1.0, abs=0.25)
    assert abs(mirror[0][0] + 1.0) > 0.55
    assert abs(flipped[0][0] + 1.0) > abs(mirror[0][0] + 1.0)
    # deeper layers never reach into the wall: the angle changes nothing
    for layer in (1, 2):
        assert np.array_equal(own[layer][1], mirror[layer][1])


def test_neutral_angle_is_the_mirror(oracle_lib):
    sc = _cap(75.0)
    for a, b in ((0.0, 90.0),):
        ka = _layer_kappa(oracle_lib, sc, a)
        kb = _layer_kappa(oracle_lib, sc, b)
        assert np.array_equal(ka[0][1], kb[0][1])
    near = _layer_kappa(oracle_lib, sc, 89.0)
    assert not np.array_equal(near[0][1], _layer_kappa(oracle_lib, sc, 90.0)[0][1])


def _run(oracle_lib, sc, steps=1):
    o = oracle_lib.Oracle.from_scene(sc)
    b0 = o.bubbles()
    o.step(steps)
    return o, b0, o.bubbles()


def _flags(sc, flags):
    sc.bubbles = [(b, flags.get(b, f), v, p) for b, f, v, p in sc.bubbles]
    return sc


def test_atmosphere_holds_p0(oracle_lib):
    """An atmosphere bubble starts and stays at p0 while its volume
    changes (the other bubble of the box follows the ideal-gas law)."""
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, 0.5, 0)]
            + [(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 1)] + [(GAS, 0.0, 1)] * 3 + [(IFACE, 0.5, 1)]
            + [(LIQ, 1.0, -1)] * 2)
    sc = _flags(scenes.layers(spec, ny=4, nz=4, p_init={0: P0 * 1.2, 1: P0 * 1.2}),
                {0: BUBBLE_ATMOSPHERE})
    o = oracle_lib.Oracle.from_scene(sc)
    b = o.bubbles()
    assert b["pressure"][0] == P0 and b["pressure"][1] == pytest.approx(1.2 * P0, rel=1e-14)
    v0 = b["volume"].copy()
    o.step(30)
    b = o.bubbles()
    assert b["flags"].tolist() == [BUBBLE_ATMOSPHERE, 0]
    assert b["volume"][0] != v0[0]
    assert b["pressure"][0] == P0
    assert b["pressure"][1] == pytest.approx(P0 * b["v_star"][1] / b["volume"][1], rel=1e-14)


@pytest.mark.parametrize("first", [0, 1])
def test_bubble_joining_the_atmosphere(oracle_lib, first):
    """The merge of the film case with one of the two bubbles an
    atmosphere (either one): the joined bubble is an atmosphere at p0."""
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, -0.08, 0)]
            + [(LIQ, 1.0, -1)] + [(IFACE, 0.5, 1)] + [(GAS, 0.0, 1)] * 3 + [(IFACE, 0.5, 1)]
            + [(LIQ, 1.0, -1)] * 2)
    sc = _flags(scenes.layers(spec, ny=4, nz=4, p_init={0: P0 * 1.1, 1: P0 * 0.9}),
                {first: BUBBLE_ATMOSPHERE})
    o, b0, b1 = _run(oracle_lib, sc)
    assert b1["id"].tolist() == [2]
    assert b1["flags"].tolist() == [BUBBLE_ATMOSPHERE]
    assert b1["pressure"][0] == P0
    assert b1["v_star"][0] == pytest.approx(b0["v_star"].sum(), rel=1e-14)


def test_split_atmosphere_stays_atmosphere(oracle_lib):
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.5, 0)]
            + [(IFACE, 1.08, 0)] + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, 0.5, 0)]
            + [(LIQ, 1.0, -1)] * 3)
    sc = _flags(scenes.layers(spec, ny=4, nz=4, p_init={0: P0 * 1.05}), {0: BUBBLE_ATMOSPHERE})
    o, b0, b1 = _run(oracle_lib, sc)
    assert b1["id"].tolist() == [1, 2]
    assert b1["flags"].tolist() == [BUBBLE_ATMOSPHERE] * 2
    assert np.all(b1["pressure"] == P0)


def test_inlet_bubble_joining_the_atmosphere(oracle_lib):
    """An inlet-owning bubble that joins the atmosphere: both flags."""
    spec = ([(LIQ, 1.0, -1)] * 2 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] + [(INLET, 0.0, 0)]
            + [(GAS, 0.0, 0)] + [(IFACE, -0.08, 0)] + [(LIQ, 1.0, -1)] + [(IFACE, 0.5, 1)]
            + [(GAS, 0.0, 1)] * 3 + [(IFACE, 0.5, 1)] + [(LIQ, 1.0, -1)] * 2)
    sc = _flags(scenes.layers(spec, ny=4, nz=4), {0: BUBBLE_INLET, 1: BUBBLE_ATMOSPHERE})
    sc.inject_rate = 0.01
    o, b0, b1 = _run(oracle_lib, sc)
    assert b1["flags"].tolist() == [BUBBLE_INLET | BUBBLE_ATMOSPHERE]
    assert b1["pressure"][0] == P0
